"""Seeded synthetic events shaped like the paper's workload (section 2).

The paper runs on 100 simulated minimum-bias events of up to 5000 hits each, recorded by a
12-layer cylindrical silicon barrel around the interaction point, with track p_T > 500 MeV. That
dataset is not available, so this module draws stand-in events of the same shape: helices from
the origin in a solenoidal field, sampled on 12 barrel layers, smeared, plus uniform noise hits.

This module only produces inputs. It holds none of the Hough-transform arithmetic (no binning,
no votes), so the GPU path and the CPU oracle can both consume its events without sharing any of
the method's code. All draws use numpy's PCG64 with seed = 1000 * workload + event.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

#: Barrel layer radii in mm: 12 layers evenly spaced from 30 mm to 1000 mm.
LAYER_RADII_MM = np.array([30.0 + k * 970.0 / 11.0 for k in range(12)])
#: Solenoid field in tesla; a track of transverse momentum p_T [GeV] has radius p_T/(0.3 B) m.
B_FIELD_T = 2.0
#: Gaussian smearing of each coordinate, in mm (20 um).
SMEAR_MM = 0.020
#: Pseudorapidity acceptance.
ETA_MAX = 2.5


@dataclass(frozen=True)
class GridSpec:
    """Binning of the vote matrix: theta x phi x A x B, A and B in mm, threshold in votes."""
    n_theta: int
    n_phi: int
    n_a: int
    n_b: int
    a_min: float = -2000.0
    a_max: float = 2000.0
    b_min: float = -2000.0
    b_max: float = 2000.0
    threshold: int = 9
    phi_sectors: bool = False  # phi cells are independent sectors (paper section 4)

    @property
    def shape(self):
        return (self.n_theta, self.n_phi, self.n_a, self.n_b)

    @property
    def n_cells(self) -> int:
        return self.n_theta * self.n_phi * self.n_a * self.n_b

    def as_tuple(self):
        return (self.n_theta, self.n_phi, self.n_a, self.n_b, self.a_min, self.a_max,
                self.b_min, self.b_max, self.threshold, int(self.phi_sectors))


@dataclass(frozen=True)
class Workload:
    name: str
    grid: GridSpec
    description: str


#: The five workloads. The paper's own binning is 4 theta x 16 phi x 1024 A x 1024 B
#: (section 2) on events of up to 5000 hits.
WORKLOADS = {
    0: Workload("small-event-250hits-4x16x64x64", GridSpec(4, 16, 64, 64, threshold=8),
                "20 tracks x 12 layers + 10 noise hits; oracle-sized"),
    1: Workload("paper-event-5000hits-4x16x1024x1024", GridSpec(4, 16, 1024, 1024, threshold=9),
                "400 tracks x 12 layers + 200 noise hits = 5000 hits; the paper's binning"),
    2: Workload("batch-100x1000-8000hits-4x16x1024x1024", GridSpec(4, 16, 1024, 1024, threshold=9),
                "100 events per batch, hit counts uniform in [1000, 8000]"),
    3: Workload("stream-5k-40k-hits-4x16x1024x1024", GridSpec(4, 16, 1024, 1024, threshold=9),
                "Poisson arrivals, lognormal hit counts clipped to [5000, 40000]"),
    4: Workload("stress-105600hits-8x32x2048x2048", GridSpec(8, 32, 2048, 2048, threshold=9),
                "8000 tracks x 12 layers + 9600 noise hits, 16 events per batch"),
}


@dataclass
class Event:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    #: per-track truth: circle centre (A, B) in mm, radius R, charge, p_T, phi0, eta
    truth: dict = field(default_factory=dict)
    #: index of the generating track for each hit, -1 for noise
    track_of_hit: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.x.size)


def helix_hits(centre_a, centre_b, charge, cot_theta, radii=LAYER_RADII_MM):
    """Exact crossings of a helix from the origin with the barrel layers, in float64.

    The transverse projection is the circle through the origin with centre (A, B), radius
    R = |(A, B)|. At layer radius r the hit sits on that circle at azimuth
    psi_c + q*acos(r/(2R)), psi_c being the azimuth of the centre, and at z = s*cot(theta), with
    s = 2R*asin(r/(2R)) the transverse arc length from the origin. Layers the circle cannot reach
    (r > 2R) give no hit. Returns (x, y, z, layer_index) arrays.
    """
    A = np.atleast_1d(np.asarray(centre_a, np.float64))
    B = np.atleast_1d(np.asarray(centre_b, np.float64))
    q = np.atleast_1d(np.asarray(charge, np.float64))
    ct = np.atleast_1d(np.asarray(cot_theta, np.float64))
    R = np.hypot(A, B)
    psi_c = np.arctan2(B, A)
    r = np.asarray(radii, np.float64)[None, :]
    ratio = r / (2.0 * R[:, None])
    ok = ratio <= 1.0
    ratio = np.minimum(ratio, 1.0)
    phi = psi_c[:, None] + q[:, None] * np.arccos(ratio)
    s = 2.0 * R[:, None] * np.arcsin(ratio)
    x = r * np.cos(phi)
    y = r * np.sin(phi)
    z = s * ct[:, None]
    layer = np.broadcast_to(np.arange(r.shape[1])[None, :], x.shape)
    return x[ok], y[ok], z[ok], layer[ok], np.nonzero(ok)[0]


def _draw_tracks(rng: np.random.Generator, n_tracks: int):
    pt = rng.uniform(0.5, 5.0, n_tracks)
    q = np.where(rng.random(n_tracks) < 0.5, -1.0, 1.0)
    phi0 = rng.uniform(0.0, 2.0 * math.pi, n_tracks)
    eta = rng.uniform(-ETA_MAX, ETA_MAX, n_tracks)
    R = pt / (0.3 * B_FIELD_T) * 1000.0
    psi_c = phi0 - q * (math.pi / 2.0)
    A = R * np.cos(psi_c)
    B = R * np.sin(psi_c)
    return dict(pt=pt, q=q, phi0=phi0, eta=eta, R=R, A=A, B=B, cot_theta=np.sinh(eta))


def _noise(rng: np.random.Generator, n_noise: int):
    layer = rng.integers(0, LAYER_RADII_MM.size, n_noise)
    r = LAYER_RADII_MM[layer]
    phi = rng.uniform(0.0, 2.0 * math.pi, n_noise)
    zmax = r * math.sinh(ETA_MAX)
    z = rng.uniform(-zmax, zmax)
    return r * np.cos(phi), r * np.sin(phi), z


def make_hits(rng: np.random.Generator, n_tracks: int, n_noise: int) -> Event:
    """n_tracks helices on the 12 layers (smeared) plus n_noise uniform hits, shuffled, float32."""
    tr = _draw_tracks(rng, n_tracks)
    x, y, z, _layer, tid = helix_hits(tr["A"], tr["B"], tr["q"], tr["cot_theta"])
    x = x + rng.normal(0.0, SMEAR_MM, x.size)
    y = y + rng.normal(0.0, SMEAR_MM, y.size)
    z = z + rng.normal(0.0, SMEAR_MM, z.size)
    nx, ny, nz = _noise(rng, n_noise)
    X = np.concatenate([x, nx])
    Y = np.concatenate([y, ny])
    Z = np.concatenate([z, nz])
    owner = np.concatenate([tid, -np.ones(n_noise, np.int64)])
    perm = rng.permutation(X.size)
    return Event(X[perm].astype(np.float32), Y[perm].astype(np.float32),
                 Z[perm].astype(np.float32), tr, owner[perm])


def hits_split(n_hits: int):
    """Track/noise split used for events of a given size: 96% of hits on tracks."""
    n_tracks = int(math.floor(0.96 * n_hits / 12.0))
    return n_tracks, n_hits - 12 * n_tracks


def event_size(workload: int, event: int) -> int:
    rng = np.random.default_rng(1000 * workload + event)
    return _event_size(workload, rng)


def _event_size(workload: int, rng: np.random.Generator) -> int:
    if workload == 0:
        return 250
    if workload == 1:
        return 5000
    if workload == 2:
        return int(rng.integers(1000, 8001))
    if workload == 3:
        return int(np.clip(np.round(rng.lognormal(math.log(14142.0), 0.52)), 5000, 40000))
    if workload == 4:
        return 105600
    raise ValueError("unknown workload %r" % workload)


def make_event(workload: int, event: int) -> Event:
    """Event `event` of workload 0..4 (see WORKLOADS); deterministic in (workload, event)."""
    rng = np.random.default_rng(1000 * workload + event)
    if workload == 0:
        n_tracks, n_noise = 20, 10
    elif workload == 1:
        n_tracks, n_noise = 400, 200
    elif workload == 4:
        n_tracks, n_noise = 8000, 9600
    else:
        n_tracks, n_noise = hits_split(_event_size(workload, rng))
    ev = make_hits(rng, n_tracks, n_noise)
    return ev


def make_batch(workload: int, events) -> list:
    return [make_event(workload, e) for e in events]


def poisson_arrivals(rate_hz: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of n requests at the given mean rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))


def uniform_hits(rng: np.random.Generator, n: int, rmax: float = 1000.0, zmax: float = 2000.0):
    """Structureless hits (uniform in a box), float32; used for edge-case and stress inputs."""
    x = rng.uniform(-rmax, rmax, n).astype(np.float32)
    y = rng.uniform(-rmax, rmax, n).astype(np.float32)
    z = rng.uniform(-zmax, zmax, n).astype(np.float32)
    return x, y, z
