"""Pins of the CPU oracle against mathematics the paper fixes (no GPU involved).

Each test checks the oracle against something other than itself: exact rational arithmetic,
float64 angles, closed forms, a brute force over cells, a library routine (scipy's maximum
filter), hand-derived fixtures, invariants and noiseless single tracks. The tests tagged `pin`
are also run against deliberately broken builds of the oracle (test_oracle_mutants.py), where at
least one of them must fail.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import exactmath as em
from paper_1507_03074_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def og(oracle_mod, spec):
    return oracle_mod.OracleGrid(*spec.as_tuple())


CFG0 = synth.WORKLOADS[0].grid
CFG1 = synth.WORKLOADS[1].grid
CFG4 = synth.WORKLOADS[4].grid
RAGGED = synth.GridSpec(3, 5, 7, 9, a_min=-1500.0, a_max=1300.0, b_min=-1100.0, b_max=1700.0,
                        threshold=2)
TINY = synth.GridSpec(2, 4, 8, 8, threshold=2)


def random_hits(rng, n, rmin=30.0, rmax=1000.0, zmax=2500.0):
    r = rng.uniform(rmin, rmax, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    x = (r * np.cos(ph)).astype(np.float32)
    y = (r * np.sin(ph)).astype(np.float32)
    z = rng.uniform(-zmax, zmax, n).astype(np.float32)
    return x, y, z


# ---------------------------------------------------------------------------------------------
# O0: tables against their definition
# ---------------------------------------------------------------------------------------------
@pytest.mark.pin
@pytest.mark.parametrize("spec", [CFG0, CFG1, CFG4, RAGGED, TINY])
def test_tables_match_definitions(oracle_mod, spec):
    g = og(oracle_mod, spec)
    a2, inv, uphi, uth = oracle_mod.tables(g)
    for i in range(spec.n_a):
        exact = em.a_centre_x2(spec, i)
        # the table entry is the binary32 value nearest to twice the bin centre
        got = Fraction(float(a2[i]))
        ulp = Fraction(float(np.spacing(np.float32(abs(float(exact)) or 1.0))))
        assert abs(got - exact) <= ulp / 2, (i, float(got), float(exact))
    exact_inv = Fraction(spec.n_b) / (em.F(spec.b_max) - em.F(spec.b_min))
    assert abs(Fraction(float(inv)) - exact_inv) <= Fraction(float(np.spacing(inv))) / 2
    for m in range(2 * spec.n_phi):
        ang = m * math.pi / spec.n_phi
        assert abs(float(uphi[m, 0]) - math.cos(ang)) <= 6e-8
        assert abs(float(uphi[m, 1]) - math.sin(ang)) <= 6e-8
    for m in range(2 * spec.n_theta + 1):
        ang = m * math.pi / (2 * spec.n_theta)
        assert abs(float(uth[m, 0]) - math.cos(ang)) <= 6e-8
        assert abs(float(uth[m, 1]) - math.sin(ang)) <= 6e-8


@pytest.mark.parametrize("spec", [CFG0, CFG1, CFG4])
def test_paper_grids_have_exact_bin_centres(oracle_mod, spec):
    """On the +-2000 mm grids every twice-centre is a binary32 number, so A2 is exact and the
    A-mirror symmetry A2[n_a-1-i] == -A2[i] holds bit for bit."""
    a2, _, _, _ = oracle_mod.tables(og(oracle_mod, spec))
    for i in range(spec.n_a):
        assert Fraction(float(a2[i])) == em.a_centre_x2(spec, i)
    assert np.array_equal(a2[::-1], -a2)


# ---------------------------------------------------------------------------------------------
# O1-O3: per-hit values and (theta, phi) cells against float64 angles
# ---------------------------------------------------------------------------------------------
@pytest.mark.pin
@pytest.mark.parametrize("spec", [CFG0, CFG4, RAGGED])
def test_sectors_and_cells_match_atan2(oracle_mod, spec):
    rng = np.random.default_rng(11)
    x, y, z = random_hits(rng, 3000)
    info = oracle_mod.hit_info(og(oracle_mod, spec), x, y, z)
    checked = 0
    for h in range(x.size):
        assert info["valid"][h]
        th = em.theta_angle(x[h], y[h], z[h])
        ph = em.phi_angle(x[h], y[h])
        cells, dist = em.hit_cells_exact(spec, x[h], y[h], z[h])
        if dist < 1e-5:
            continue
        checked += 1
        assert info["s_phi"][h] == math.floor(ph / (math.pi / spec.n_phi))
        assert info["s_theta"][h] == math.floor(th / (math.pi / (2 * spec.n_theta)))
        got = sorted((int(t), int(p)) for t, p in info["cells"][h] if t >= 0)
        assert got == cells, (h, got, cells)
        assert info["n_cells"][h] == len(cells)
    assert checked > 0.99 * x.size


@pytest.mark.pin
def test_per_hit_values_are_correctly_rounded(oracle_mod):
    rng = np.random.default_rng(5)
    x, y, z = random_hits(rng, 2000)
    info = oracle_mod.hit_info(og(oracle_mod, CFG1), x, y, z)
    for h in range(x.size):
        X, Y = em.F(x[h]), em.F(y[h])
        r2 = float(np.float32(float(np.float32(X * X)) + float(np.float32(Y * Y))))
        assert info["r2"][h] == np.float32(r2)
        # sqrt and reciprocal: nearest binary32 to the exact value
        exact_r = math.sqrt(r2)
        assert abs(float(info["r"][h]) - exact_r) <= float(np.spacing(np.float32(exact_r))) / 2
        exact_k = Fraction(1) / (2 * Y)
        k = Fraction(float(info["k"][h]))
        assert abs(k - exact_k) <= Fraction(float(np.spacing(np.abs(info["k"][h])))) / 2


def test_degenerate_hits_vote_nothing(oracle_mod):
    g = og(oracle_mod, CFG0)
    inf, nan = np.inf, np.nan
    x = np.array([0, 0, 100, inf, 100, nan, 100, 100, 3e19, 1e-30], np.float32)
    y = np.array([0, 0, 0, 100, inf, 100, nan, 100, 3e19, 1e-30], np.float32)
    z = np.array([0, 50, 10, 0, 0, 0, 0, inf, 0, 0], np.float32)
    info = oracle_mod.hit_info(g, x, y, z)
    assert not info["valid"].any()
    M, votes = oracle_mod.fill(g, x, y, z)
    assert votes == 0 and not M.any()


def test_empty_event(oracle_mod):
    g = og(oracle_mod, CFG0)
    e = np.zeros(0, np.float32)
    M, votes = oracle_mod.fill(g, e, e, e)
    assert votes == 0 and M.shape == CFG0.shape and not M.any()
    cells, vv, n = oracle_mod.peaks(g, M)
    assert n == 0 and cells.size == 0


def test_invalid_grids_rejected(oracle_mod):
    bad = [
        synth.GridSpec(0, 16, 64, 64), synth.GridSpec(4, 2, 64, 64), synth.GridSpec(4, 16, 0, 64),
        synth.GridSpec(4, 16, 64, 64, a_min=1.0, a_max=1.0),
        synth.GridSpec(4, 16, 64, 64, b_min=float("nan")),
        synth.GridSpec(4, 16, 64, 64, threshold=0),
        synth.GridSpec(64, 64, 1 << 12, 1 << 12),  # 2^36 cells
        synth.GridSpec(1, 3, (1 << 24) + 1, 1),
    ]
    for b in bad:
        assert not oracle_mod.check_grid(og(oracle_mod, b)), b
    assert oracle_mod.check_grid(og(oracle_mod, CFG4))


# ---------------------------------------------------------------------------------------------
# O4-O5: bins against exact rational arithmetic (the exact result within the FP32 error bound)
# ---------------------------------------------------------------------------------------------
def single_hit_bins(oracle_mod, spec, x, y, z):
    """(i -> j or -1) of a one-hit event, read from the oracle's vote matrix, plus its cells."""
    M, _ = oracle_mod.fill(og(oracle_mod, spec), np.array([x]), np.array([y]), np.array([z]))
    nz = np.argwhere(M)
    cells = sorted({(int(t), int(p)) for t, p, _, _ in nz})
    j = -np.ones(spec.n_a, np.int64)
    if cells:
        t0, p0 = cells[0]
        for a, b in np.argwhere(M[t0, p0]):
            assert j[a] == -1, "two votes in one A row"
            j[a] = b
        for t, p in cells:
            assert np.array_equal(M[t, p], M[t0, p0]), "cells of one hit must hold one pattern"
    return j, cells, M


@pytest.mark.pin
@pytest.mark.parametrize("spec,n_hits", [(CFG0, 60), (RAGGED, 60), (CFG1, 6)])
def test_vote_bins_match_exact_arithmetic(oracle_mod, spec, n_hits):
    rng = np.random.default_rng(21)
    x, y, z = random_hits(rng, n_hits)
    # include near-axis hits (small |y|: steep lines, large k) and small radii
    x[:3] = np.float32([500.0, -700.0, 31.0])
    y[:3] = np.float32([0.75, -1.5, 29.0])
    ambiguous = total = 0
    for h in range(n_hits):
        j, cells, _ = single_hit_bins(oracle_mod, spec, x[h], y[h], z[h])
        for i in range(spec.n_a):
            f = em.exact_f(spec, x[h], y[h], i)
            bound = Fraction(em.f32_error_bound(spec, x[h], y[h], i))
            lo, hi = f - bound, f + bound
            if hi < 0 or lo >= spec.n_b:
                expect = -1                      # certainly outside the B range
            elif 0 <= lo and hi < spec.n_b and math.floor(lo) == math.floor(hi):
                expect = math.floor(f)           # certainly inside one bin
            else:
                if h >= 3:
                    ambiguous += 1
                continue
            if h >= 3:
                total += 1
            assert j[i] == expect, (h, i, float(f), int(j[i]))
    # binary32 leaves the bin undecided for a tiny fraction of the generic (h >= 3) votes
    assert ambiguous <= 0.002 * (total + ambiguous), (ambiguous, total)


# ---------------------------------------------------------------------------------------------
# Brute force over cells on tiny grids (different loop order, exact arithmetic)
# ---------------------------------------------------------------------------------------------
def safe_hits(spec, rng, n, margin_rad=1e-4, margin_bins=1e-3):
    xs, ys, zs = [], [], []
    while len(xs) < n:
        x, y, z = random_hits(rng, 1)
        _, dist = em.hit_cells_exact(spec, x[0], y[0], z[0])
        if dist < margin_rad:
            continue
        ok = True
        for i in range(spec.n_a):
            f = em.exact_f(spec, x[0], y[0], i)
            if abs(float(f - round(f))) < margin_bins:
                ok = False
                break
        if ok:
            xs.append(x[0]); ys.append(y[0]); zs.append(z[0])
    return (np.array(xs, np.float32), np.array(ys, np.float32), np.array(zs, np.float32))


@pytest.mark.pin
@pytest.mark.parametrize("spec", [TINY, RAGGED])
def test_fill_equals_brute_force_over_cells(oracle_mod, spec):
    rng = np.random.default_rng(3)
    x, y, z = safe_hits(spec, rng, 24)
    M, votes = oracle_mod.fill(og(oracle_mod, spec), x, y, z)
    ref = em.brute_force_matrix(spec, x, y, z)
    assert np.array_equal(M, ref)
    assert votes == int(ref.sum())


# ---------------------------------------------------------------------------------------------
# Closed-form vote totals per hit
# ---------------------------------------------------------------------------------------------
@pytest.mark.pin
@pytest.mark.parametrize("spec", [CFG0, RAGGED])
def test_vote_totals_closed_form(oracle_mod, spec):
    ev = synth.make_event(0, 7)
    x, y, z = ev.x[:120], ev.y[:120], ev.z[:120]
    g = og(oracle_mod, spec)
    compared = 0
    grand_expect = 0
    for h in range(x.size):
        n_a, edge_dist = em.n_a_closed_form(spec, x[h], y[h])
        cells, dist = em.hit_cells_exact(spec, x[h], y[h], z[h])
        if edge_dist < 1e-4 or dist < 1e-6:
            continue
        _, votes = oracle_mod.fill(g, x[h:h + 1], y[h:h + 1], z[h:h + 1])
        assert votes == len(cells) * n_a, (h, votes, len(cells), n_a)
        grand_expect += votes
        compared += 1
    assert compared >= 110
    # the per-hit totals add up to the event total (linearity of the counts)
    keep = [h for h in range(x.size)
            if em.n_a_closed_form(spec, x[h], y[h])[1] >= 1e-4
            and em.hit_cells_exact(spec, x[h], y[h], z[h])[1] >= 1e-6]
    M, votes = oracle_mod.fill(g, x[keep], y[keep], z[keep])
    assert votes == grand_expect == int(M.sum(dtype=np.int64))


# ---------------------------------------------------------------------------------------------
# Hand-derived worked examples
# ---------------------------------------------------------------------------------------------
@pytest.mark.pin
def test_hand_worked_examples(oracle_mod):
    with open(os.path.join(GOLDEN, "worked_examples.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        spec = synth.GridSpec(*case["grid"])
        g = og(oracle_mod, spec)
        hx = np.array([h[0] for h in case["hits"]], np.float32)
        hy = np.array([h[1] for h in case["hits"]], np.float32)
        hz = np.array([h[2] for h in case["hits"]], np.float32)
        M, votes = oracle_mod.fill(g, hx, hy, hz)
        expect = np.zeros(spec.shape, np.uint32)
        for t, p, a, b, v in case["votes"]:
            expect[t, p, a, b] = v
        assert np.array_equal(M, expect), case["name"]
        assert votes == case["total_votes"], case["name"]
        cells, vv, n = oracle_mod.peaks(g, M)
        assert [[int(c), int(v)] for c, v in zip(cells, vv)] == case["peaks"], case["name"]


# Exact bin edges. On a grid with A-bin centres A2/2 = 1, 3, 5, ... (A2 = 2, 6, 10, ...) and B in
# [0, 16) with 1 mm bins, the circle of hit (x, y) gives B = (x^2 + y^2 - A2 x) / (2 y) exactly:
# - (8, -4) and (8, 4): x^2 + y^2 = 80 = A2 x on A row 2, so B = 0 there, the lower edge of bin 0
#   (in binary32 the product (80 - 80) / (2 y) is -0 for y < 0, which is still >= 0);
# - (0, 32): B = 16 on every row, the upper edge of the range, which is open: no vote;
# - (0, 31.5): B = 15.75 on every row, bin 15;
# - (0, -2): B = -1 on every row, below the range: no vote.
EDGE_GRID = synth.GridSpec(1, 4, 8, 16, a_min=0.0, a_max=16.0, b_min=0.0, b_max=16.0, threshold=3)


@pytest.mark.pin
def test_bin_edges_exact(oracle_mod):
    g = og(oracle_mod, EDGE_GRID)
    for (x, y), rows in [((8.0, -4.0), {2: 0}), ((8.0, 4.0), {2: 0}), ((0.0, 32.0), {}),
                         ((0.0, 31.5), {a: 15 for a in range(8)}), ((0.0, -2.0), {})]:
        M, _ = oracle_mod.fill(g, np.array([x], np.float32), np.array([y], np.float32),
                               np.array([1.0], np.float32))
        for a, b in rows.items():
            # the hit lies in two phi cells (half-bin widening) and the one theta cell
            assert int(M[0, :, a, b].sum()) == 2, ((x, y), a, b)
        if not rows:
            assert not M.any(), (x, y)
        # the B bin on every other row follows from the exact circle
        for a in range(8):
            if a in rows:
                continue
            A2 = 4.0 * a + 2.0
            Bx = Fraction(int(x * 2), 2) ** 2 + Fraction(int(y * 2), 2) ** 2 - Fraction(int(A2)) * Fraction(int(x * 2), 2)
            Bx /= 2 * Fraction(int(y * 2), 2)
            expect = int(math.floor(Bx)) if 0 <= Bx < 16 else None
            got = np.argwhere(M[0, :, a, :].sum(axis=0))
            assert (expect is None and got.size == 0) or (got.size == 1 and int(got[0, 0]) == expect), \
                ((x, y), a, expect, got)


# ---------------------------------------------------------------------------------------------
# Invariants of the vote matrix
# ---------------------------------------------------------------------------------------------
@pytest.mark.pin
def test_hit_order_and_linearity(oracle_mod):
    g = og(oracle_mod, CFG0)
    ev = synth.make_event(0, 3)
    M, v = oracle_mod.fill(g, ev.x, ev.y, ev.z)
    perm = np.random.default_rng(0).permutation(ev.n)
    Mp, vp = oracle_mod.fill(g, ev.x[perm], ev.y[perm], ev.z[perm])
    assert np.array_equal(M, Mp) and v == vp
    h = ev.n // 3
    M1, v1 = oracle_mod.fill(g, ev.x[:h], ev.y[:h], ev.z[:h])
    M2, v2 = oracle_mod.fill(g, ev.x[h:], ev.y[h:], ev.z[h:])
    assert np.array_equal(M, M1 + M2) and v == v1 + v2


def _off_boundary(spec, x, y, z, margin=1e-5):
    keep = [h for h in range(x.size) if em.hit_cells_exact(spec, x[h], y[h], z[h])[1] > margin]
    return x[keep], y[keep], z[keep]


@pytest.mark.pin
@pytest.mark.parametrize("spec", [CFG0, synth.GridSpec(4, 16, 256, 128, threshold=9)])
def test_mirror_symmetries(oracle_mod, spec):
    """x -> -x maps A bin a to n_a-1-a and phi cell p to n_phi/2-1-p (mod n_phi), bit for bit,
    because A2 is antisymmetric and r2 - A2*x is unchanged; z -> -z maps theta cell t to
    n_theta-1-t and leaves (A, B) alone."""
    g = og(oracle_mod, spec)
    ev = synth.make_event(0, 12)
    x, y, z = _off_boundary(spec, ev.x, ev.y, ev.z)
    M, v = oracle_mod.fill(g, x, y, z)
    Mx, vx = oracle_mod.fill(g, -x, y, z)
    p = np.arange(spec.n_phi)
    pm = (spec.n_phi // 2 - 1 - p) % spec.n_phi
    assert vx == v
    assert np.array_equal(Mx[:, pm, ::-1, :], M)
    Mz, vz = oracle_mod.fill(g, x, y, -z)
    assert vz == v
    assert np.array_equal(Mz[::-1], M)


# ---------------------------------------------------------------------------------------------
# Noiseless single tracks: the generating cell is a peak with one vote per layer
# ---------------------------------------------------------------------------------------------
def single_track_case(spec, rng):
    dA = (spec.a_max - spec.a_min) / spec.n_a
    dB = (spec.b_max - spec.b_min) / spec.n_b
    while True:
        a0 = int(rng.integers(0, spec.n_a))
        b0 = int(rng.integers(0, spec.n_b))
        A0 = spec.a_min + (a0 + 0.5) * dA
        B0 = spec.b_min + (b0 + 0.5) * dB
        R = math.hypot(A0, B0)
        if not (900.0 <= R <= 1500.0):
            continue
        q = float(rng.choice([-1.0, 1.0]))
        cot = float(rng.uniform(-4.0, 4.0))
        x, y, z, layer, _ = synth.helix_hits([A0], [B0], [q], [cot])
        if x.size != 12:
            continue
        x, y, z = x.astype(np.float32), y.astype(np.float32), z.astype(np.float32)
        cellsets, ok = [], True
        for h in range(12):
            cells, dist = em.hit_cells_exact(spec, x[h], y[h], z[h])
            if dist < 1e-4:
                ok = False
            cellsets.append(set(cells))
        common = sorted(set.intersection(*cellsets))
        if not ok or not common:
            continue
        # the neighbouring A rows must not also collect all 12 votes in one B bin
        tie = False
        for da in (-1, 1):
            if not 0 <= a0 + da < spec.n_a:
                continue
            bins = {math.floor(em.exact_f(spec, x[h], y[h], a0 + da)) for h in range(12)}
            if len(bins) == 1:
                tie = True
        if tie:
            continue
        fs = [em.exact_f(spec, x[h], y[h], a0) for h in range(12)]
        if any(abs(float(f - (b0 + Fraction(1, 2)))) > 0.25 for f in fs):
            continue
        return x, y, z, (a0, b0), common


@pytest.mark.pin
@pytest.mark.parametrize("spec", [synth.GridSpec(4, 16, 64, 64, threshold=12),
                                  synth.GridSpec(4, 16, 1024, 1024, threshold=12)])
def test_single_track_peak(oracle_mod, spec):
    rng = np.random.default_rng(77 + spec.n_a)
    g = og(oracle_mod, spec)
    for _ in range(6 if spec.n_a == 64 else 2):
        x, y, z, (a0, b0), common = single_track_case(spec, rng)
        M, votes = oracle_mod.fill(g, x, y, z)
        t_star, p_star = common[0]
        for t, p in common:
            assert M[t, p, a0, b0] == 12
        assert M.max() == 12
        cells, vv, n = oracle_mod.peaks(g, M)
        expect = np.ravel_multi_index((t_star, p_star, a0, b0), spec.shape)
        assert n == 1 and int(cells[0]) == expect and int(vv[0]) == 12


# ---------------------------------------------------------------------------------------------
# O6: peaks against scipy's maximum filter and structural properties
# ---------------------------------------------------------------------------------------------
def tie_heavy_matrix(rng, shape):
    M = rng.integers(0, 4, size=shape).astype(np.uint32)
    spikes = rng.random(shape) < 0.02
    M[spikes] += rng.integers(3, 9, size=int(spikes.sum())).astype(np.uint32)
    return M


@pytest.mark.pin
@pytest.mark.parametrize("shape", [(2, 4, 8, 8), (3, 5, 7, 9), (4, 16, 64, 64), (1, 3, 5, 1)])
def test_peaks_match_maximum_filter(oracle_mod, shape):
    rng = np.random.default_rng(sum(shape))
    spec = synth.GridSpec(*shape, threshold=3)
    M = tie_heavy_matrix(rng, shape)
    cells, vv, n = oracle_mod.peaks(og(oracle_mod, spec), M)
    ref = em.peaks_by_max_filter(M, 3)
    assert n == ref.size
    assert np.array_equal(cells, ref)
    assert np.array_equal(vv, M.ravel()[ref])


@pytest.mark.pin
def test_peaks_of_events_match_maximum_filter(oracle_mod):
    g = og(oracle_mod, CFG0)
    nonempty = 0
    for e in range(30):
        ev = synth.make_event(0, e)
        M, _ = oracle_mod.fill(g, ev.x, ev.y, ev.z)
        cells, vv, n = oracle_mod.peaks(g, M)
        assert np.array_equal(cells, em.peaks_by_max_filter(M, CFG0.threshold))
        nonempty += n > 0
    assert nonempty >= 10


@pytest.mark.pin
def test_peak_list_structure(oracle_mod):
    rng = np.random.default_rng(8)
    shape = (3, 6, 20, 24)
    spec = synth.GridSpec(*shape, threshold=4)
    M = tie_heavy_matrix(rng, shape)
    cells, vv, n = oracle_mod.peaks(og(oracle_mod, spec), M)
    assert n == cells.size > 0
    assert np.all(np.diff(cells.astype(np.int64)) > 0)
    assert np.all(vv >= 4) and np.array_equal(vv, M.ravel()[cells])
    s = set(int(c) for c in cells)
    for c in cells:
        assert not (em.neighbours(shape, int(c)) & s)
    # the cell with the largest (votes, -index) is always a peak
    flat = M.ravel()
    best = int(np.flatnonzero(flat == flat.max())[0])
    assert best in s
    # capacity truncation keeps the first cells and still reports the total
    c2, v2, n2 = oracle_mod.peaks(og(oracle_mod, spec), M, capacity=3)
    assert n2 == n and np.array_equal(c2, cells[:3])


def test_threshold_above_max_gives_no_peaks(oracle_mod):
    spec = synth.GridSpec(4, 16, 64, 64, threshold=1000)
    ev = synth.make_event(0, 0)
    g = og(oracle_mod, spec)
    M, _ = oracle_mod.fill(g, ev.x, ev.y, ev.z)
    assert oracle_mod.peaks(g, M)[2] == 0


def test_regression_fixtures(oracle_mod):
    """Stored outputs of the oracle on workload-0 events (written by golden/make_golden.py);
    guards the oracle against unintended changes."""
    with open(os.path.join(GOLDEN, "cfg0_events.json")) as fh:
        data = json.load(fh)
    g = og(oracle_mod, CFG0)
    for rec in data["events"]:
        ev = synth.make_event(0, rec["event"])
        M, votes = oracle_mod.fill(g, ev.x, ev.y, ev.z)
        cells, vv, n = oracle_mod.peaks(g, M)
        assert votes == rec["votes"]
        assert [[int(c), int(v)] for c, v in zip(cells, vv)] == rec["peaks"]


@pytest.mark.pin
@pytest.mark.parametrize("spec", [CFG0, RAGGED, CFG4])
def test_readout_matches_definition(oracle_mod, spec):
    """rho = sqrt(A^2 + B^2) and phi = atan2(B, A) in [0, 2 pi) of the bin centres (section 2)."""
    rng = np.random.default_rng(4)
    cells = rng.integers(0, spec.n_cells, 500).astype(np.uint32)
    r = oracle_mod.readout(og(oracle_mod, spec), cells)
    t, p, a, b = np.unravel_index(cells.astype(np.int64), spec.shape)
    assert np.array_equal(r["t"], t) and np.array_equal(r["p"], p)
    assert np.array_equal(r["a"], a) and np.array_equal(r["b"], b)
    for i in range(0, 500, 7):
        A = em.F(spec.a_min) + (a[i] + Fraction(1, 2)) * (em.F(spec.a_max) - em.F(spec.a_min)) / spec.n_a
        Bc = em.F(spec.b_min) + (b[i] + Fraction(1, 2)) * (em.F(spec.b_max) - em.F(spec.b_min)) / spec.n_b
        assert abs(r["A"][i] - float(A)) <= 1e-9 * max(1.0, abs(float(A)))
        assert abs(r["B"][i] - float(Bc)) <= 1e-9 * max(1.0, abs(float(Bc)))
        assert r["rho"][i] == pytest.approx(math.hypot(float(A), float(Bc)), rel=1e-12)
        phi = math.atan2(float(Bc), float(A)) % (2 * math.pi)
        assert r["phi"][i] == pytest.approx(phi, abs=1e-12)
        assert 0.0 <= r["phi"][i] < 2 * math.pi
        assert r["theta"][i] == pytest.approx((t[i] + 0.5) * math.pi / spec.n_theta, rel=1e-14)


# ---------------------------------------------------------------------------------------------
# Sector variant (paper section 4): independent phi sectors, one M_H(A, B, theta) each
# ---------------------------------------------------------------------------------------------
def sectors(spec, n_phi=None):
    return synth.GridSpec(spec.n_theta, n_phi or spec.n_phi, spec.n_a, spec.n_b, spec.a_min,
                          spec.a_max, spec.b_min, spec.b_max, spec.threshold, phi_sectors=True)


@pytest.mark.pin
@pytest.mark.parametrize("spec", [sectors(CFG0), sectors(CFG0, 4), sectors(RAGGED, 1),
                                  sectors(RAGGED, 2)])
def test_sector_cells_match_atan2(oracle_mod, spec):
    rng = np.random.default_rng(21)
    x, y, z = random_hits(rng, 2000)
    info = oracle_mod.hit_info(og(oracle_mod, spec), x, y, z)
    checked = 0
    for h in range(x.size):
        cells, dist = em.hit_cells_exact(spec, x[h], y[h], z[h])
        if dist < 1e-5:
            continue
        checked += 1
        got = sorted((int(t), int(p)) for t, p in info["cells"][h] if t >= 0)
        assert got == cells, (h, got, cells)
        # one sector per hit; theta cells as in the 4-D transform
        assert len({p for _, p in got}) == 1
    assert checked > 0.99 * x.size


@pytest.mark.pin
@pytest.mark.parametrize("spec", [sectors(TINY), sectors(RAGGED, 2)])
def test_sector_fill_equals_brute_force(oracle_mod, spec):
    rng = np.random.default_rng(5)
    x, y, z = safe_hits(spec, rng, 24)
    M, votes = oracle_mod.fill(og(oracle_mod, spec), x, y, z)
    ref = em.brute_force_matrix(spec, x, y, z)
    assert np.array_equal(M, ref)
    assert votes == int(ref.sum())


@pytest.mark.pin
@pytest.mark.parametrize("spec", [CFG0, RAGGED])
def test_sector_votes_are_a_half_of_the_4d_votes(oracle_mod, spec):
    """Every valid hit votes in two phi cells of the 4-D transform and in one sector, with the
    same (A, B) line, so the totals differ by exactly a factor 2, and each sector's matrix is
    bounded cell by cell by the same slab of the 4-D matrix (its hits are a subset)."""
    g4, gs = og(oracle_mod, spec), og(oracle_mod, sectors(spec))
    for e in range(6):
        ev = synth.make_event(0, 40 + e)
        M4, v4 = oracle_mod.fill(g4, ev.x, ev.y, ev.z)
        Ms, vs = oracle_mod.fill(gs, ev.x, ev.y, ev.z)
        assert v4 == 2 * vs > 0
        assert int(M4.sum(dtype=np.int64)) == 2 * int(Ms.sum(dtype=np.int64))
        assert np.all(Ms <= M4)
        i4 = oracle_mod.hit_info(g4, ev.x, ev.y, ev.z)
        i_s = oracle_mod.hit_info(gs, ev.x, ev.y, ev.z)
        assert np.array_equal(i4["n_cells"], 2 * i_s["n_cells"])
        # the sector of a hit is the phi cell its own half-sector lies in
        own = i4["s_phi"] // 2
        for h in np.flatnonzero(i_s["valid"]):
            assert {int(p) for t, p in i_s["cells"][h] if t >= 0} == {int(own[h])}


@pytest.mark.pin
@pytest.mark.parametrize("shape", [(2, 4, 8, 8), (3, 5, 7, 9), (2, 1, 6, 5), (3, 2, 4, 1)])
def test_sector_peaks_match_maximum_filter(oracle_mod, shape):
    rng = np.random.default_rng(100 + sum(shape))
    spec = synth.GridSpec(*shape, threshold=3, phi_sectors=True)
    M = tie_heavy_matrix(rng, shape)
    cells, vv, n = oracle_mod.peaks(og(oracle_mod, spec), M)
    ref = em.peaks_by_max_filter(M, 3, phi_sectors=True)
    assert n == ref.size
    assert np.array_equal(cells, ref)
    assert np.array_equal(vv, M.ravel()[ref])
    # a sector peak list is the merge of the per-sector 3-D searches
    per = []
    for p in range(shape[1]):
        sub = np.ascontiguousarray(M[:, p:p + 1])
        c3, _, _ = oracle_mod.peaks(og(oracle_mod, synth.GridSpec(shape[0], 1, shape[2], shape[3],
                                                                  threshold=3, phi_sectors=True)), sub)
        tt, _, aa, bb = np.unravel_index(c3.astype(np.int64), (shape[0], 1, shape[2], shape[3]))
        per.extend(np.ravel_multi_index((tt, np.full_like(tt, p), aa, bb), shape).tolist())
    assert sorted(per) == cells.tolist()


@pytest.mark.pin
def test_sector_grid_limits(oracle_mod):
    base = dict(n_theta=2, n_a=4, n_b=4, a_min=-1.0, a_max=1.0, b_min=-1.0, b_max=1.0, threshold=1)
    assert oracle_mod.check_grid(oracle_mod.OracleGrid(n_phi=1, phi_sectors=1, **base))
    assert oracle_mod.check_grid(oracle_mod.OracleGrid(n_phi=2, phi_sectors=1, **base))
    assert not oracle_mod.check_grid(oracle_mod.OracleGrid(n_phi=2, phi_sectors=0, **base))
    assert not oracle_mod.check_grid(oracle_mod.OracleGrid(n_phi=4, phi_sectors=2, **base))


@pytest.mark.pin
def test_sector_single_track_peak(oracle_mod):
    """A noiseless track whose hits all lie in one sector: its generating cell holds one vote
    per layer and is the only peak."""
    spec = synth.GridSpec(4, 4, 64, 64, threshold=12, phi_sectors=True)
    g = og(oracle_mod, spec)
    rng = np.random.default_rng(8)
    for _ in range(5):
        x, y, z, (a0, b0), common = single_track_case(spec, rng)
        assert len({p for _, p in common}) == 1
        M, _ = oracle_mod.fill(g, x, y, z)
        for t, p in common:
            assert M[t, p, a0, b0] == 12
        cells, vv, n = oracle_mod.peaks(g, M)
        t_star, p_star = common[0]
        assert n == 1 and int(cells[0]) == np.ravel_multi_index((t_star, p_star, a0, b0), spec.shape)
