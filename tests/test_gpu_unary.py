"""The two correctly rounded operations of the per-hit values (bin rule O2: r = sqrt(r2) and
k = 1/(2y)), checked on the GPU for every one of the 2^32 binary32 inputs.

The check is the definition of correct rounding, evaluated exactly: a float result q of an
exact value t is correctly rounded (to nearest) iff t lies within half a unit in the last place
of q on each side; below a power of two the lower neighbour is only half a unit away. In double
precision, (q +- h)^2 (25-bit operands) and q * w (24-bit operands) are exact, so the tests
"(r - h_lo)^2 < v < (r + h_hi)^2" and "|1 - q w| <= h |w|" involve no rounding. Neither square
roots nor reciprocals of binary32 values can fall exactly half-way between two floats, so the
bounds are strict for the root. The checker uses only torch element-wise ops, each its own
launch, so nothing is contracted.
"""
import sys

import pytest

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import os
    import torch
    from paper_1507_03074_amd import binding as B
    from paper_1507_03074_amd import build as hbuild
    hbuild.ensure_built()  # a missing or stale library is rebuilt, never tested
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    B.lib()
    return B


def pow2(e):
    """2^e as float64 for an integer tensor e (from the bits, so exactly)."""
    import torch
    return ((e.to(torch.int64) + 1023) << 52).view(torch.float64)


def half_ulps(q):
    """Half the gap to the next float away from zero and half the gap towards zero, for finite
    nonzero float64 values holding binary32 numbers."""
    import torch
    a = q.abs()
    m, e = torch.frexp(a)  # a = m 2^e, m in [0.5, 1)
    ulp = torch.clamp(pow2(e - 24), min=2.0 ** -149)  # subnormals: a fixed spacing
    up = ulp / 2
    down = torch.where((m == 0.5) & (a > 2.0 ** -126), ulp / 4, ulp / 2)
    return up, down


def check_chunk(B, lo):
    import torch
    bits = (torch.arange(lo, lo + CHUNK, dtype=torch.int64, device="cuda") - (1 << 31)).to(torch.int32)
    v = bits.view(torch.float32)
    root = torch.empty_like(v)
    inv2 = torch.empty_like(v)
    B.ht_debug_unary(v, root, inv2)
    bad = {}

    # ---- root = sqrt(v)
    vn, rn = torch.isnan(v), torch.isnan(root)
    neg = (v < 0) & ~vn
    zero = v == 0
    pinf = torch.isinf(v) & (v > 0)
    ok = torch.zeros_like(vn)
    ok |= vn & rn
    ok |= neg & rn
    ok |= zero & (root.view(torch.int32) == v.view(torch.int32))  # sqrt(+-0) = +-0
    ok |= pinf & torch.isinf(root) & (root > 0)
    fin = ~(vn | neg | zero | pinf)
    vd, rd = v[fin].double(), root[fin].double()
    up, down = half_ulps(rd)
    good = (rd > 0) & torch.isfinite(rd) & ((rd - down) ** 2 < vd) & (vd < (rd + up) ** 2)
    ok[fin] = good
    bad["sqrt"] = (~ok).nonzero().flatten()

    # ---- inv2 = 1 / (v + v); v + v is exact (or overflows to inf, as in the kernel)
    w = v + v
    wn = torch.isnan(w)
    wz = w == 0
    winf = torch.isinf(w)
    ok = torch.zeros_like(wn)
    ok |= wn & torch.isnan(inv2)
    # 1/(+-0) = +-inf and 1/(+-inf) = +-0, with the sign of w
    ok |= wz & torch.isinf(inv2) & (torch.signbit(inv2) == torch.signbit(w))
    ok |= winf & (inv2 == 0) & (torch.signbit(inv2) == torch.signbit(w))
    fin = ~(wn | wz | winf)
    wd, qd = w[fin].double(), inv2[fin].double()
    aw = wd.abs()
    qinf = torch.isinf(qd)
    # overflow: |1/w| at or past FLT_MAX + half its ulp (2^128 - 2^103) rounds to inf
    good_inf = qinf & (torch.signbit(qd) == torch.signbit(wd)) & (aw * (2.0 ** 128 - 2.0 ** 103) <= 1.0)
    qf = torch.where(qinf, torch.ones_like(qd), qd)  # placeholder where q is inf
    up, down = half_ulps(qf)
    d = 1.0 - qf * wd  # exact: q w has at most 48 significant bits and lies near 1
    # d > 0: 1/w is farther from zero than q; d < 0: closer
    good_fin = (~qinf) & (qd != 0) & (torch.signbit(qd) == torch.signbit(wd)) & torch.where(
        d >= 0, d <= up * aw, -d <= down * aw)
    ok[fin] = good_inf | good_fin
    bad["inv2"] = (~ok).nonzero().flatten()

    out = {}
    for k, idx in bad.items():
        if idx.numel():
            i = idx[:5]
            out[k] = (int(idx.numel()), [hex(int(b) & 0xffffffff) for b in bits[i].tolist()],
                      root[i].tolist() if k == "sqrt" else inv2[i].tolist())
    return out


def test_unary_ops_correctly_rounded_for_every_input(B):
    import torch
    failures = {}
    for c in range((1 << 32) // CHUNK):
        lo = c * CHUNK
        say("unary ops: inputs 0x%08x .. 0x%08x" % (lo, lo + CHUNK - 1))
        r = check_chunk(B, lo)
        for k, v in r.items():
            failures.setdefault(k, []).append(v)
        torch.cuda.empty_cache()
    assert not failures, failures


def test_unary_ops_known_values(B):
    """Exact squares and reciprocals, signed zeros, infinities and the extremes, against the
    host's IEEE binary32 arithmetic (numpy float32 sqrt and division are correctly rounded)."""
    import numpy as np
    import torch
    vals = np.array([4.0, 2.25, 1.0, 0.25, 2.0, 0.5, 4.5, 3.0, -0.0, 0.0, np.inf, -np.inf, -1.0,
                     2.0 ** -149, 2.0 ** -126, 2.0 ** 127, 3.0e38, 1.0e-38, np.nan], np.float32)
    v = torch.from_numpy(vals).cuda()
    root = torch.empty_like(v)
    inv2 = torch.empty_like(v)
    B.ht_debug_unary(v, root, inv2)
    torch.cuda.synchronize()
    with np.errstate(all="ignore"):
        want_r = np.sqrt(vals)
        want_q = np.float32(1.0) / (vals + vals)
    for got, want in ((root.cpu().numpy(), want_r), (inv2.cpu().numpy(), want_q)):
        same = (got.view(np.uint32) == want.view(np.uint32)) | (np.isnan(got) & np.isnan(want))
        assert same.all(), [(float(vals[i]), float(got[i]), float(want[i])) for i in np.flatnonzero(~same)]
    assert root.cpu().numpy()[:4].tolist() == [2.0, 1.5, 1.0, 0.5]
