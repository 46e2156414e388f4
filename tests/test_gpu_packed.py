"""GPU parity of the counting-sort slab lists (k_prep, k_bucket, then k_fill reading packed lists
through their offsets) against the CPU oracle, bit for bit.

Direct per-slab lists are used while an event's lists stay within 512 MiB and a batch's scratch
within 8 GiB; past that every event of the call takes the counting sort. The 16-event batch of
105600-hit events on the 8x32x2048x2048 grid is such a batch. HT_PACKED_LISTS=1 forces the
counting sort on any call, so the same kernels are checked here on small grids, every launch
shape and every fill variant (two or eight records per thread, consecutive tiles with the
records held in registers), and then on the stress batch itself as the benchmark runs it.
"""
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
    return B


@pytest.fixture()
def packed():
    """Every call inside the test takes the counting-sort lists."""
    saved = os.environ.get("HT_PACKED_LISTS")
    os.environ["HT_PACKED_LISTS"] = "1"
    yield
    if saved is None:
        os.environ.pop("HT_PACKED_LISTS", None)
    else:
        os.environ["HT_PACKED_LISTS"] = saved


def oracle_run(spec, x, y, z):
    from oracle import oracle
    g = oracle.OracleGrid(*spec.as_tuple())
    M, votes = oracle.fill(g, x, y, z)
    cells, vv, n = oracle.peaks(g, M)
    return M, votes, cells, vv, n


def gpu_fused(B, spec, x, y, z, capacity=1 << 16):
    import torch
    xd, yd, zd = B.hits_to_device(x, y, z)
    acc, cells, votes, n = B.fill_peaks(spec, xd, yd, zd, capacity=capacity)
    torch.cuda.synchronize()
    return B.as_u32(acc), cells, votes, n


def assert_same(gM, gc, gv, gn, M, oc, ov, on, tag=""):
    assert gM.shape == M.shape
    if not np.array_equal(gM, M):
        bad = np.argwhere(gM != M)
        raise AssertionError("%s: %d cells differ, first %s gpu=%d oracle=%d" % (
            tag, len(bad), bad[0], gM[tuple(bad[0])], M[tuple(bad[0])]))
    assert gn == on, (tag, gn, on)
    assert np.array_equal(gc, oc) and np.array_equal(gv, ov), tag


def random_hits(seed, n, spread=1000.0):
    rng = np.random.default_rng(seed)
    return synth.uniform_hits(rng, n, spread, 2.5 * spread)


def test_switch_selects_packed_lists(gpu, packed):
    """The plan the batch call makes on the host: packed under the switch, direct without it."""
    B = gpu
    assert B.ht_debug_batch_plan(CFG0, [250, 0, 17])[0] is False
    os.environ.pop("HT_PACKED_LISTS")
    assert B.ht_debug_batch_plan(CFG0, [250, 0, 17])[0] is True
    os.environ["HT_PACKED_LISTS"] = "1"


def test_packed_small_events_bit_exact(gpu, packed):
    """Workload-0 events: the fused call, the separate fill, the atomic fill and ht_peaks."""
    import torch
    B = gpu
    nonempty = 0
    for e in range(40):
        ev = synth.make_event(0, e)
        if e % 10 == 0:
            say("packed lists: workload 0 event", e)
        gM, gc, gv, gn = gpu_fused(B, CFG0, ev.x, ev.y, ev.z)
        M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
        assert_same(gM, gc, gv, gn, M, oc, ov, on, "event %d" % e)
        nonempty += on > 0
        if e < 5:
            xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
            a1 = B.fill(CFG0, xd, yd, zd)
            a2 = B.fill(CFG0, xd, yd, zd, atomic=True)
            torch.cuda.synchronize()
            assert np.array_equal(B.as_u32(a1), M) and np.array_equal(B.as_u32(a2), M)
            c, v, n = B.peaks(CFG0, a1)
            assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)
    assert nonempty >= 15


RAGGED = [
    synth.GridSpec(3, 5, 7, 9, a_min=-1500.0, a_max=1300.0, b_min=-1100.0, b_max=1700.0, threshold=2),
    synth.GridSpec(2, 7, 100, 37, a_min=-999.0, a_max=1234.5, b_min=-1500.0, b_max=2000.0, threshold=3),
    synth.GridSpec(4, 16, 130, 66, threshold=4),
    synth.GridSpec(1, 3, 1, 1, threshold=1),
    synth.GridSpec(5, 3, 257, 1000, threshold=3),
]


@pytest.mark.parametrize("spec", RAGGED, ids=lambda s: "x".join(map(str, s.shape)))
def test_packed_ragged_grids_bit_exact(gpu, packed, spec):
    B = gpu
    for seed in range(3):
        say("packed lists: ragged grid", spec.shape, "seed", seed)
        x, y, z = random_hits(seed, 300)
        gM, gc, gv, gn = gpu_fused(B, spec, x, y, z)
        M, votes, oc, ov, on = oracle_run(spec, x, y, z)
        assert_same(gM, gc, gv, gn, M, oc, ov, on, "seed %d" % seed)


@pytest.mark.parametrize("rows", [1, 2, 4, 8, 16, 32, 64])
def test_packed_every_tile_shape_bit_exact(gpu, packed, rows):
    """Every A-row count, with tiles per workgroup 1, 4 and 16 (tiles in one slab, across slabs,
    past the last tile) and every store kind."""
    B = gpu
    for spec, ev in ((CFG0, synth.make_event(0, 3)),
                     (synth.GridSpec(4, 16, 100, 40, threshold=4), synth.make_event(0, 4))):
        M, votes, oc, ov, on = oracle_run(spec, ev.x, ev.y, ev.z)
        for gt, nt, tpb in ((16, 0, 1), (64, 1, 4), (32, 2, 16)):
            say("packed lists: rows", rows, "group tiles", gt, "store", nt, "tiles/block", tpb,
                "grid", spec.shape)
            B.ht_set_tuning(spec, rows=rows, group_tiles=gt, nt_store=nt, tiles_per_block=tpb)
            try:
                gM, gc, gv, gn = gpu_fused(B, spec, ev.x, ev.y, ev.z)
            finally:
                B.ht_set_tuning(spec)
            assert_same(gM, gc, gv, gn, M, oc, ov, on, "rows %d tpb %d" % (rows, tpb))


@pytest.mark.parametrize("rows,tpb,nt", [(1, 1, 0), (2, 4, 1), (4, 1, 2), (4, 8, 1), (8, 4, 0),
                                         (8, 16, 1), (16, 1, 1), (64, 1, 0)])
def test_packed_long_lists_bit_exact(gpu, packed, rows, tpb, nt):
    """About 1000 records per slab: eight records per thread per round trip (rows <= 8) and, with
    several tiles per workgroup, consecutive tiles of one slab with the records kept in
    registers."""
    B = gpu
    x, y, z = random_hits(77, 22000)
    M, votes, oc, ov, on = oracle_run(CFG0, x, y, z)
    say("packed lists: long lists, rows", rows, "tiles/block", tpb, "store", nt)
    B.ht_set_tuning(CFG0, rows=rows, tiles_per_block=tpb, nt_store=nt)
    try:
        gM, gc, gv, gn = gpu_fused(B, CFG0, x, y, z)
    finally:
        B.ht_set_tuning(CFG0)
    assert_same(gM, gc, gv, gn, M, oc, ov, on, "rows %d tpb %d" % (rows, tpb))


def test_packed_paper_grid_bit_exact(gpu, packed):
    """A paper-shaped event (5000 hits, 4x16x1024x1024) over the fill shapes the batch tuner
    picks from."""
    B = gpu
    ev = synth.make_event(1, 7)
    M, votes, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
    for rows, nt, tpb in ((4, 0, 1), (8, 1, 2), (4, 1, 8), (2, 2, 16)):
        say("packed lists: workload 1, rows", rows, "store", nt, "tiles/block", tpb)
        B.ht_set_tuning(CFG1, rows=rows, nt_store=nt, tiles_per_block=tpb)
        try:
            gM, gc, gv, gn = gpu_fused(B, CFG1, ev.x, ev.y, ev.z)
        finally:
            B.ht_set_tuning(CFG1)
        assert_same(gM, gc, gv, gn, M, oc, ov, on, "rows %d store %d tpb %d" % (rows, nt, tpb))


def test_packed_sector_grids_bit_exact(gpu, packed):
    B = gpu
    for spec in (synth.GridSpec(4, 4, 64, 64, threshold=8, phi_sectors=True),
                 synth.GridSpec(3, 2, 7, 9, a_min=-1500.0, a_max=1300.0, b_min=-1100.0, b_max=1700.0,
                                threshold=2, phi_sectors=True)):
        for e in range(4):
            ev = synth.make_event(0, 800 + e)
            say("packed lists: sector grid", spec.shape, "event", e)
            gM, gc, gv, gn = gpu_fused(B, spec, ev.x, ev.y, ev.z)
            M, votes, oc, ov, on = oracle_run(spec, ev.x, ev.y, ev.z)
            assert_same(gM, gc, gv, gn, M, oc, ov, on, "event %d" % e)


def test_packed_batch_and_graph_replays_bit_exact(gpu, packed):
    """Batches of uneven events (empty ones included) through the captured graph and through
    direct launches, replayed with host work in between."""
    import torch
    B = gpu
    for rep in range(3):
        hits = []
        for e in range(16):
            ev = synth.make_event(0, 1100 + 16 * rep + e)
            k = [ev.n, 0, 1, 17, ev.n - 40][e % 5]
            hits.append((ev.x[:k], ev.y[:k], ev.z[:k]))
        assert B.ht_debug_batch_plan(CFG0, [len(h[0]) for h in hits])[0] is False
        say("packed lists: batch replay", rep)
        os.environ["HT_BATCH_GRAPH"] = "1"
        try:
            g_res = B.fill_peaks_batch(CFG0, hits, capacity=64)
            os.environ["HT_BATCH_GRAPH"] = "0"
            e_res = B.fill_peaks_batch(CFG0, hits, capacity=64)
        finally:
            os.environ.pop("HT_BATCH_GRAPH", None)
        torch.cuda.synchronize()
        ga, ea = B.as_u32(g_res.acc), B.as_u32(e_res.acc)
        for i, (x, y, z) in enumerate(hits):
            M, votes, oc, ov, on = oracle_run(CFG0, x, y, z)
            assert np.array_equal(ga[i], M) and np.array_equal(ea[i], M), i
            for res in (g_res, e_res):
                c, v, n = res.peaks[i]
                assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), i


def test_packed_batch_of_paper_sized_events(gpu, packed):
    """Uneven workload-2 events (1000-8000 hits) on the paper grid, batched on packed lists."""
    B = gpu
    evs = [synth.make_event(2, 20 + e) for e in range(4)]
    say("packed lists: batch of 4 workload-2 events, sizes", [e.n for e in evs])
    res = B.fill_peaks_batch(CFG1, [(e.x, e.y, e.z) for e in evs], capacity=1 << 14)
    accs = B.as_u32(res.acc)
    for i, ev in enumerate(evs):
        M, votes, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
        assert np.array_equal(accs[i], M), i
        c, v, n = res.peaks[i]
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), i
    del res, accs


def test_packed_request_loop(gpu, packed):
    """The request loop with counting-sort lists in its slots."""
    import ctypes
    import time
    B = gpu
    evs = [synth.make_event(0, 1200 + e) for e in range(10)]
    lib = B.lib()
    g = B.make_grid(CFG0)
    opts = B.ServeOpts(1 << 30, 256, 2000, 4, 2, 64, 0)
    srv = ctypes.c_void_p()
    B.check(lib.ht_serve_create(ctypes.byref(g), ctypes.byref(opts), ctypes.byref(srv)))
    say("packed lists: request loop, 10 workload-0 events")
    try:
        fp = ctypes.POINTER(ctypes.c_float)
        tickets = []
        for ev in evs:
            t = ctypes.c_uint64()
            B.check(lib.ht_serve_submit(srv, ev.x.ctypes.data_as(fp), ev.y.ctypes.data_as(fp),
                                        ev.z.ctypes.data_as(fp), ev.n, ctypes.byref(t)))
            tickets.append(t.value)
        deadline = time.time() + 60
        for ev, t in zip(evs, tickets):
            out = (B.Peak * 256)()
            nf = ctypes.c_int64()
            while True:
                rc = lib.ht_serve_poll(srv, t, out, 256, ctypes.byref(nf), None)
                if rc != B.HT_EAGAIN:
                    break
                assert time.time() < deadline, "server did not finish"
                time.sleep(1e-4)
            B.check(rc)
            arr = np.frombuffer(out, dtype=np.uint32).reshape(-1, 2)[:nf.value]
            M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
            assert nf.value == on and np.array_equal(arr[:, 0], oc) and np.array_equal(arr[:, 1], ov)
    finally:
        lib.ht_serve_destroy(srv)


# ---------------------------------------------------------------------------------------------
# The stress batch as the benchmark runs it: 16 events of 105600 hits on 8x32x2048x2048 (4 GiB of
# counts each, 64 GiB in all), which takes the counting sort without any switch.
# ---------------------------------------------------------------------------------------------
STRESS_SHAPES = [None, (4, 0, 0, 1, 8)]  # default shape; the batch tuner's pick on this workload


@pytest.mark.timeout(1500)
@pytest.mark.parametrize("shape", STRESS_SHAPES, ids=["default", "rows4-nt-tpb8"])
def test_stress_batch_of_16_events_bit_exact(gpu, shape):
    """All 16 events' matrices and peak lists equal those of the per-event call (direct lists,
    checked against the oracle in full by test_stress_event_full_size); the first and the last
    event of the batch equal the oracle's in full."""
    import torch
    B = gpu
    assert os.environ.get("HT_PACKED_LISTS") is None
    n_ev, cap = 16, 1 << 20
    evs = [synth.make_event(4, e) for e in range(n_ev)]
    res = None
    if shape:
        B.ht_set_tuning(CFG4, B.Tuning(*shape))
    try:
        direct, scratch = B.ht_debug_batch_plan(CFG4, [e.n for e in evs])
        assert direct is False, "the stress batch must take the counting sort"
        say("stress batch: 16 x 105600 hits, shape", B.ht_get_tuning(CFG4).as_dict(),
            "scratch %.1f GB" % (scratch / 1e9))
        res = B.fill_peaks_batch(CFG4, [(e.x, e.y, e.z) for e in evs], capacity=cap)
        torch.cuda.synchronize()
        single = B.new_acc(CFG4)
        out, nf = B.new_peaks(cap)
        for i, ev in enumerate(evs):
            xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
            B.ht_fill_peaks(CFG4, xd, yd, zd, single, out, cap, nf)
            torch.cuda.synchronize()
            c, v, n = B.peaks_to_host(out, nf, cap)
            bc, bv, bn = res.peaks[i]
            assert bn == n and np.array_equal(bc, c) and np.array_equal(bv, v), i
            assert torch.equal(res.acc[i], single), i
            say("stress batch: event", i, "equals the per-event call,", n, "peaks")
        del single, out, nf
        for i in (0, n_ev - 1):
            say("stress batch: event", i, "against the oracle")
            gM = B.as_u32(res.acc[i])
            M, votes, oc, ov, on = oracle_run(CFG4, evs[i].x, evs[i].y, evs[i].z)
            assert int(gM.sum(dtype=np.int64)) == votes
            assert np.array_equal(gM, M), i
            del gM, M
            c, v, n = res.peaks[i]
            assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), i
    finally:
        if shape:
            B.ht_set_tuning(CFG4)
        del res
        torch.cuda.empty_cache()
