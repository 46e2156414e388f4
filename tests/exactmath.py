"""First-principles references used to pin the oracle.

Nothing here calls the oracle or the GPU library. Each function restates what the paper's
method means in plain mathematics (exact rationals or float64 angles), so that the oracle's
FP32 rule can be checked against it:

* the circle through the interaction point and a hit (x, y), x^2 + y^2 - 2Ax - 2By = 0, gives
  B(A) = (x^2 + y^2 - 2Ax) / (2y): a straight line in the (A, B) plane (paper section 2);
* a hit belongs to every (theta, phi) cell whose range, widened by half a bin on each side,
  contains its polar angle atan2(r, z) and its azimuth atan2(y, x);
* a peak is a cell at or above the threshold that beats every neighbour in its 3^4 box under the
  order (votes, -index) (sections 2 and 3).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

U32 = 2.0 ** -24  # unit roundoff of binary32


def F(v) -> Fraction:
    return Fraction(float(v))


def a_centre_x2(grid, i) -> Fraction:
    """Twice the exact centre of A bin i."""
    a_min, a_max = F(grid.a_min), F(grid.a_max)
    return 2 * a_min + (2 * i + 1) * (a_max - a_min) / grid.n_a


def exact_f(grid, x, y, i) -> Fraction:
    """Exact real B-bin coordinate of the vote of hit (x, y) in A bin i, from float32 inputs."""
    X, Y = F(x), F(y)
    B = (X * X + Y * Y - a_centre_x2(grid, i) * X) / (2 * Y)
    return (B - F(grid.b_min)) * grid.n_b / (F(grid.b_max) - F(grid.b_min))


def f32_error_bound(grid, x, y, i) -> float:
    """Bound on |f computed in binary32 - exact f| for the operation sequence
    r2 = x*x + y*y; num = r2 - A2*x; B = num*(1/(y+y)); f = (B - b_min)*invdB, each op rounded
    once (first-order error analysis, doubled for safety, plus the A2 table rounding)."""
    u = U32
    x, y = float(x), float(y)
    r2 = x * x + y * y
    a2 = float(a_centre_x2(grid, i))
    a2_err = abs(float(np.float32(a2)) - a2)
    num = r2 - a2 * x
    k = 1.0 / (2.0 * y)
    inv_db = grid.n_b / (float(grid.b_max) - float(grid.b_min))
    B = num * k
    d = B - float(grid.b_min)
    e_r2 = 2.01 * u * r2
    e_t = u * abs(a2 * x) + a2_err * abs(x) * 1.01
    e_num = e_r2 + e_t + u * (abs(num) + e_r2 + e_t)
    e_B = abs(k) * e_num * 1.01 + 2.01 * u * abs(num * k)
    e_d = e_B + u * (abs(d) + e_B)
    e_f = inv_db * e_d * 1.01 + 2.01 * u * abs(d) * inv_db
    return 2.0 * e_f + 1e-12


def phi_angle(x, y) -> float:
    a = math.atan2(float(y), float(x))
    return a + 2 * math.pi if a < 0 else a


def theta_angle(x, y, z) -> float:
    return math.atan2(math.hypot(float(x), float(y)), float(z))


def widened_cells(angle: float, n: int, span: float, periodic: bool):
    """Cells k whose range [k w, (k+1) w), w = span/n, widened by w/2 on both sides, holds angle."""
    w = span / n
    out = []
    for k in range(n):
        lo, hi = k * w - w / 2, (k + 1) * w + w / 2
        if periodic:
            # test angle, angle - span, angle + span against the unwrapped interval
            if any(lo <= a < hi for a in (angle, angle - span, angle + span)):
                out.append(k)
        elif lo <= angle < hi:
            out.append(k)
    return out


def boundary_distance(angle: float, n_half: int, span: float) -> float:
    """Distance from angle to the nearest half-bin boundary m*span/n_half."""
    w = span / n_half
    m = round(angle / w)
    return abs(angle - m * w)


def hit_cells_exact(grid, x, y, z):
    """(theta, phi) cells of a hit from float64 angles: list of (t, p), and the distance (rad)
    to the nearest half-bin boundary (small distances mean FP32 may legitimately differ)."""
    th = theta_angle(x, y, z)
    ph = phi_angle(x, y)
    tc = widened_cells(th, grid.n_theta, math.pi, periodic=False)
    if getattr(grid, "phi_sectors", False):
        # independent sectors: the one sector holding the azimuth, no widening
        pc = [min(int(ph // (2 * math.pi / grid.n_phi)), grid.n_phi - 1)]
    else:
        pc = widened_cells(ph, grid.n_phi, 2 * math.pi, periodic=True)
    dist = min(boundary_distance(th, 2 * grid.n_theta, math.pi),
               boundary_distance(ph, 2 * grid.n_phi, 2 * math.pi),
               ph, 2 * math.pi - ph)
    return sorted((t, p) for t in tc for p in pc), dist


def n_a_closed_form(grid, x, y):
    """Number of A-bin centres A_i with b_min <= B(A_i) < b_max, from the interval of A on which
    the line B(A) = r2/(2y) - A x/y stays inside the B range (closed form, no loop over bins).
    Returns (count, distance in A-bin units from the interval ends to the nearest centre)."""
    X, Y = F(x), F(y)
    r2 = X * X + Y * Y
    c = r2 / (2 * Y)
    s = X / Y
    a_min, a_max = F(grid.a_min), F(grid.a_max)
    dA = (a_max - a_min) / grid.n_a
    bmin, bmax = F(grid.b_min), F(grid.b_max)
    if s == 0:
        inside = bmin <= c < bmax
        return (grid.n_a if inside else 0), float("inf")
    # b_min <= c - A s < b_max  <=>  c - b_max < A s <= c - b_min
    lo_v, hi_v = (c - bmax) / s, (c - bmin) / s
    if s > 0:   # A in (lo_v, hi_v]
        lo, lo_open, hi, hi_open = lo_v, True, hi_v, False
    else:       # A in [hi_v, lo_v)
        lo, lo_open, hi, hi_open = hi_v, False, lo_v, True
    # centre index coordinate u(A) = (A - a_min)/dA - 1/2, centres at integer u
    ulo = (lo - a_min) / dA - Fraction(1, 2)
    uhi = (hi - a_min) / dA - Fraction(1, 2)
    i_min = math.floor(ulo) + 1 if lo_open else math.ceil(ulo)
    i_max = math.ceil(uhi) - 1 if hi_open else math.floor(uhi)
    i_min = max(i_min, 0)
    i_max = min(i_max, grid.n_a - 1)
    count = max(0, i_max - i_min + 1)

    def frac_dist(u):
        return float(abs(u - round(u)))
    return count, min(frac_dist(ulo), frac_dist(uhi))


def brute_force_matrix(grid, x, y, z):
    """Per-cell brute force over all (t, p, a, b) and all hits with exact arithmetic: a cell
    counts a hit when the hit lies in the widened (theta, phi) cell and the exact B of the hit's
    circle at the A-bin centre falls in B bin b."""
    nt, npf, na, nb = grid.n_theta, grid.n_phi, grid.n_a, grid.n_b
    M = np.zeros((nt, npf, na, nb), np.uint32)
    hits = []
    for h in range(len(x)):
        cells, _ = hit_cells_exact(grid, x[h], y[h], z[h])
        fa = [exact_f(grid, x[h], y[h], a) for a in range(na)]
        hits.append((set(cells), fa))
    for t in range(nt):
        for p in range(npf):
            for a in range(na):
                for b in range(nb):
                    cnt = 0
                    for cells, fa in hits:
                        if (t, p) not in cells:
                            continue
                        f = fa[a]
                        if 0 <= f < nb and math.floor(f) == b:
                            cnt += 1
                    M[t, p, a, b] = cnt
    return M


def peaks_by_max_filter(M: np.ndarray, threshold: int, phi_sectors: bool = False):
    """Peak cells from scipy's maximum filter on key = votes * 2^32 + (2^32 - 1 - index):
    absent theta/A/B neighbours are padded with -1, phi wraps around; with phi_sectors the
    window spans one phi cell (sectors have no phi neighbours)."""
    from scipy.ndimage import maximum_filter
    idx = np.arange(M.size, dtype=np.int64).reshape(M.shape)
    key = M.astype(np.int64) * (1 << 32) + ((1 << 32) - 1 - idx)
    size = (3, 1, 3, 3) if phi_sectors else 3
    mx = maximum_filter(key, size=size, mode=["constant", "wrap", "constant", "constant"], cval=-1)
    sel = (key == mx) & (M >= threshold)
    return np.flatnonzero(sel.ravel()).astype(np.uint32)


def neighbours(shape, c):
    """The up-to-80 neighbour indices of cell c in the 3^4 box (phi periodic)."""
    nt, npf, na, nb = shape
    t, p, a, b = np.unravel_index(c, shape)
    out = set()
    for dt in (-1, 0, 1):
        for dp in (-1, 0, 1):
            for da in (-1, 0, 1):
                for db in (-1, 0, 1):
                    if dt == dp == da == db == 0:
                        continue
                    tt, aa, bb = t + dt, a + da, b + db
                    if not (0 <= tt < nt and 0 <= aa < na and 0 <= bb < nb):
                        continue
                    pp = (p + dp) % npf
                    out.add(int(np.ravel_multi_index((tt, pp, aa, bb), shape)))
    out.discard(int(c))
    return out
