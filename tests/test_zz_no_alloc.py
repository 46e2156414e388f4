"""ht_fill_peaks_noalloc (all scratch in one fixed device array, no allocation) against
ht_fill_peaks, the entry point it is a variant of, through the C ABI: the vote matrix, the peak
list and the count must be identical, bit for bit, on two calls in a row (the second with a
smaller event, so it runs on what the first left in the shared array), on events that take the
direct slab lists and the counting sort, and when the grid (and so the table region) changes
between calls. The small events are also checked against the CPU oracle.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

from paper_1507_03074_amd import synth

pytestmark = pytest.mark.gpu

CFG0 = synth.WORKLOADS[0].grid
CFG1 = synth.WORKLOADS[1].grid
CFG4 = synth.WORKLOADS[4].grid


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1507_03074_amd import binding as B
    from paper_1507_03074_amd import build as hbuild
    hbuild.ensure_built()  # a missing or stale library is rebuilt, never tested
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    B.lib()
    for spec in (CFG0, CFG1):
        B.ht_set_tuning(spec)  # the default launch shapes, whatever ran before in this process
    return B


def run_both(B, spec, ev, capacity=1 << 18):
    """(matrix, cells, votes, n) from ht_fill_peaks_noalloc, then from ht_fill_peaks."""
    import torch
    x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
    res = []
    for fn in (B.ht_fill_peaks_noalloc, B.ht_fill_peaks):
        acc = B.new_acc(spec)
        acc.fill_(7)  # every cell must be overwritten
        out, nf = B.new_peaks(capacity)
        fn(spec, x, y, z, acc, out, capacity, nf)
        torch.cuda.synchronize()
        c, v, n = B.peaks_to_host(out, nf, capacity)
        res.append((B.as_u32(acc), c, v, n))
    return res


def assert_identical(a, b, tag):
    (ma, ca, va, na), (mb, cb, vb, nb) = a, b
    if not np.array_equal(ma, mb):
        bad = np.argwhere(ma != mb)
        raise AssertionError("%s: %d cells differ, first %s" % (tag, len(bad), bad[0]))
    assert na == nb, (tag, na, nb)
    assert np.array_equal(ca, cb) and np.array_equal(va, vb), tag


def oracle_check(spec, ev, got):
    from oracle import oracle
    g = oracle.OracleGrid(*spec.as_tuple())
    M, _ = oracle.fill(g, ev.x, ev.y, ev.z)
    oc, ov, on = oracle.peaks(g, M)
    m, c, v, n = got
    assert np.array_equal(m, M) and n == on and np.array_equal(c, oc) and np.array_equal(v, ov)


def test_noalloc_equals_fill_peaks_on_two_calls_the_second_smaller(gpu):
    B = gpu
    big = synth.make_event(1, 7)                   # 5000 hits, paper grid: direct lists
    small = synth.make_event(1, 8)
    keep = np.random.default_rng(3).random(small.n) < 0.3
    small = synth.Event(small.x[keep], small.y[keep], small.z[keep])
    for i, ev in enumerate((big, small)):
        say("noalloc call %d: %d hits on the paper grid" % (i + 1, ev.n))
        na, ref = run_both(B, CFG1, ev)
        assert_identical(na, ref, "call %d" % (i + 1))
        assert na[3] > 0


def test_noalloc_counting_sort_layout_and_grid_changes(gpu):
    B = gpu
    # the 40000-hit event of the served workload (its peaks come from the stencil over the
    # matrix), then 64000 hits (two events together), whose direct lists do not fit the fixed
    # array, so the call takes the counting sort; then small grids, so the table region is
    # rewritten
    big = synth.make_event(3, next(e for e in range(40) if synth.event_size(3, e) == 40000))
    assert big.n == 40000
    say("noalloc: %d hits on the paper grid" % big.n)
    na, ref = run_both(B, CFG1, big, capacity=1 << 19)
    assert_identical(na, ref, "40k-hit event")
    more = synth.make_event(3, next(e for e in range(40) if 20000 <= synth.event_size(3, e) <= 30000))
    ev = synth.Event(np.concatenate([big.x, more.x]), np.concatenate([big.y, more.y]),
                     np.concatenate([big.z, more.z]))
    say("noalloc: %d hits on the paper grid (counting sort)" % ev.n)
    na, ref = run_both(B, CFG1, ev, capacity=1 << 19)
    assert_identical(na, ref, "%d-hit event" % ev.n)
    for seed in (1, 2):
        e0 = synth.make_event(0, seed)
        say("noalloc: workload-0 event seed %d (%d hits)" % (seed, e0.n))
        na, ref = run_both(B, CFG0, e0)
        assert_identical(na, ref, "workload 0 seed %d" % seed)
        oracle_check(CFG0, e0, na)
        e1 = synth.make_event(1, 20 + seed)
        say("noalloc: back to the paper grid (%d hits)" % e1.n)
        na, ref = run_both(B, CFG1, e1)
        assert_identical(na, ref, "paper grid after workload 0, seed %d" % seed)


def test_noalloc_empty_event_and_refused_sizes(gpu):
    import torch
    B = gpu
    e = synth.Event(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    say("noalloc: empty event")
    na, ref = run_both(B, CFG0, e)
    assert_identical(na, ref, "empty event")
    assert na[3] == 0 and not na[0].any()
    # a stress event needs far more scratch than the array holds: refused on the host, before
    # any device work, with the bytes it needed in the message
    say("noalloc: a stress-grid event is refused")
    x = torch.zeros(105600, dtype=torch.float32, device="cuda")
    out, nf = B.new_peaks(16)
    acc = torch.empty(1, dtype=torch.int32, device="cuda")  # never written: the call is refused
    g = B.make_grid(CFG4)
    rc = B.lib().ht_fill_peaks_noalloc(ctypes.byref(g), B._ptr(x), B._ptr(x), B._ptr(x), x.numel(),
                                       B._ptr(acc), B._ptr(out), 16, B._ptr(nf), B._stream(None))
    assert rc == B.HT_EINVAL
    assert "bytes of scratch" in B.last_error()


def test_noalloc_failed_launch_leaves_the_array_usable(gpu):
    """A call whose launches stop part way (forced from the host: HT_TEST_FAIL_STAGE) must leave
    the shared counters consistent for the next call."""
    import torch
    B = gpu
    try:
        for i, stage in enumerate(("prep", "fill", "peaks")):
            ev = synth.make_event(0, 90 + i)
            say("noalloc: %s launch fails, then a normal call" % stage)
            os.environ["HT_TEST_FAIL_STAGE"] = stage
            x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
            acc = B.new_acc(CFG0)
            out, nf = B.new_peaks(1024)
            with pytest.raises(B.HTError) as ex:
                B.ht_fill_peaks_noalloc(CFG0, x, y, z, acc, out, 1024, nf)
            assert ex.value.code == B.HT_EDEVICE
            torch.cuda.synchronize()
            os.environ.pop("HT_TEST_FAIL_STAGE")
            nxt = synth.make_event(0, 95 + i)
            na, ref = run_both(B, CFG0, nxt)
            assert_identical(na, ref, "after a failed %s launch" % stage)
            oracle_check(CFG0, nxt, na)
    finally:
        os.environ.pop("HT_TEST_FAIL_STAGE", None)
