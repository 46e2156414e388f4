"""GPU parity of the stencil peak search (crowded events: k_peak_stencil over the written matrix,
then k_peak_write_dense from its peak words) against the CPU oracle, bit for bit.

The fused fill + peak search takes the stencil for events with at least `dense_hits` hits (by
default n_slabs n_b / 4: the 40000-hit served event does) on grids of at most 4 theta and 16 phi
cells. HT_DENSE_HITS moves that threshold, so the same kernels are checked here on small and
ragged grids, every row segment length (HT_DENSE_ROWS), ragged B chunks, one to four theta
cells, three to sixteen phi cells (the wrap), phi sectors, both paths of the ordered writer
(HT_DENSE_STAGE), truncated outputs, pinned-host outputs, batches that mix both searches (graph
and eager) and the request loop.
"""
import os
import sys

import numpy as np
import pytest

from paper_1507_03074_amd import synth

pytestmark = pytest.mark.gpu

CFG0 = synth.WORKLOADS[0].grid
CFG1 = synth.WORKLOADS[1].grid


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
        B.ht_set_tuning(spec)
    return B


@pytest.fixture()
def env():
    keys = ("HT_DENSE_HITS", "HT_DENSE_ROWS", "HT_BATCH_GRAPH", "HT_DENSE_STAGE")
    saved = {k: os.environ.get(k) for k in keys}
    yield os.environ
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def oracle_run(spec, x, y, z):
    from oracle import oracle
    g = oracle.OracleGrid(*spec.as_tuple())
    M, _ = oracle.fill(g, x, y, z)
    cells, vv, n = oracle.peaks(g, M)
    return M, cells, vv, n


def check(B, spec, x, y, z, tag, capacity=1 << 18):
    import torch
    xd, yd, zd = B.hits_to_device(x, y, z)
    acc = B.new_acc(spec)
    acc.fill_(5)
    acc, c, v, n = B.fill_peaks(spec, xd, yd, zd, acc=acc, capacity=capacity,
                                allow_truncation=True)
    torch.cuda.synchronize()
    M, oc, ov, on = oracle_run(spec, x, y, z)
    gM = B.as_u32(acc)
    if not np.array_equal(gM, M):
        bad = np.argwhere(gM != M)
        raise AssertionError("%s: %d cells differ, first %s" % (tag, len(bad), bad[0]))
    k = min(on, capacity)
    assert n == on, (tag, n, on)
    assert np.array_equal(c, oc[:k]) and np.array_equal(v, ov[:k]), tag
    return on


def random_hits(seed, n, spread=1000.0):
    rng = np.random.default_rng(seed)
    return synth.uniform_hits(rng, n, spread, 2.5 * spread)


def test_dense_threshold_reported(gpu):
    B = gpu
    t = B.ht_get_tuning(CFG1)
    assert t.dense_hits == 4 * 16 * 1024 // 4
    assert B.ht_get_tuning(synth.GridSpec(4, 16, 64, 60)).dense_hits > 0
    # a wave per phi cell holds every theta cell: at most 16 phi and 4 theta cells
    assert B.ht_get_tuning(synth.WORKLOADS[4].grid).dense_hits == -1
    assert B.ht_get_tuning(synth.GridSpec(5, 3, 64, 64)).dense_hits == -1
    assert B.ht_get_tuning(synth.GridSpec(2, 17, 64, 64)).dense_hits == -1
    assert B.ht_get_tuning(synth.GridSpec(4, 16, 64, 64)).dense_hits > 0


def test_dense_workload0_events(gpu, env):
    B = gpu
    env["HT_DENSE_HITS"] = "1"
    total = 0
    for seed in range(30):
        ev = synth.make_event(0, seed)
        total += check(B, CFG0, ev.x, ev.y, ev.z, "workload 0 seed %d" % seed)
    say("dense workload 0: %d peaks over 30 events" % total)
    assert total > 30


GRIDS = [
    synth.GridSpec(4, 16, 64, 64, threshold=4),
    synth.GridSpec(3, 5, 7, 16, a_min=-1500.0, a_max=1300.0, b_min=-1100.0, b_max=1700.0, threshold=2),
    synth.GridSpec(2, 7, 100, 40, a_min=-999.0, a_max=1234.5, b_min=-1500.0, b_max=2000.0, threshold=3),
    synth.GridSpec(4, 16, 130, 72, threshold=4),        # W = 64: a ragged second chunk of 8
    synth.GridSpec(4, 3, 257, 1000, threshold=3),       # three phi cells: the wrap is both ways
    synth.GridSpec(2, 16, 67, 192, threshold=3),        # sixteen phi cells, full 64-column chunks
    synth.GridSpec(1, 4, 33, 24, threshold=2),          # one theta cell
    synth.GridSpec(2, 5, 30, 62, threshold=2),          # one full chunk of 62 columns
    synth.GridSpec(3, 4, 25, 125, threshold=2),         # two full chunks and one column
    synth.GridSpec(2, 4, 33, 60, threshold=2),          # a row length that is no multiple of 8
    synth.GridSpec(2, 4, 40, 48, threshold=2, phi_sectors=True),
    synth.GridSpec(4, 2, 50, 130, threshold=2, phi_sectors=True),
    synth.GridSpec(3, 1, 20, 64, threshold=2, phi_sectors=True),
]


@pytest.mark.parametrize("spec", GRIDS, ids=lambda s: "x".join(map(str, s.shape)) + ("s" if s.phi_sectors else ""))
def test_dense_ragged_grids(gpu, env, spec):
    B = gpu
    env["HT_DENSE_HITS"] = "1"
    for seed in range(3):
        x, y, z = random_hits(seed, 300)
        check(B, spec, x, y, z, "%s seed %d" % (spec.shape, seed))


@pytest.mark.parametrize("rows", [1, 12, 13, 64, 4096])
def test_dense_row_segments(gpu, env, rows):
    B = gpu
    env["HT_DENSE_HITS"] = "1"
    env["HT_DENSE_ROWS"] = str(rows)
    spec = synth.GridSpec(4, 16, 130, 72, threshold=4)
    x, y, z = random_hits(rows, 400)
    check(B, spec, x, y, z, "rows %d" % rows)
    ev = synth.make_event(0, 3)
    check(B, CFG0, ev.x, ev.y, ev.z, "workload 0, rows %d" % rows)


@pytest.mark.parametrize("rows,gt", [(1, 16), (2, 64), (4, 32), (64, 16)])
def test_dense_peak_counts_per_group_of_tiles(gpu, env, rows, gt):
    """The stencil counts each row's peaks into its group of tiles (the ordered writer's output
    offsets): at every tile height and group size, including groups that end inside a segment
    of rows and groups that span two slabs."""
    B = gpu
    env["HT_DENSE_HITS"] = "1"
    for spec in (synth.GridSpec(4, 16, 130, 72, threshold=4), synth.GridSpec(3, 3, 37, 200, threshold=3)):
        try:
            B.ht_set_tuning(spec, rows=rows, group_tiles=gt)
            for seed in range(2):
                x, y, z = random_hits(100 + seed, 500)
                check(B, spec, x, y, z, "%s rows %d groups of %d" % (spec.shape, rows, gt))
        finally:
            B.ht_set_tuning(spec)


@pytest.mark.parametrize("stage", [None, "0", "17"], ids=["staged", "unstaged", "mixed"])
def test_dense_writer_paths(gpu, env, stage):
    """The ordered writer's paths: a group's peaks staged in LDS (at most HT_DENSE_STAGE of
    them, else each thread emits its own), and groups of more peak words than a thread holds in
    registers (groups of 64 tiles of 8 rows: 512 rows of 17 words on the paper grid)."""
    B = gpu
    env["HT_DENSE_HITS"] = "1"
    if stage is not None:
        env["HT_DENSE_STAGE"] = stage
    ev = synth.make_event(1, 90)
    for rows, gt in ((8, 16), (8, 64)):
        try:
            B.ht_set_tuning(CFG1, rows=rows, group_tiles=gt)
            check(B, CFG1, ev.x, ev.y, ev.z, "writer rows %d groups of %d stage %s" % (rows, gt, stage))
            check(B, CFG1, ev.x, ev.y, ev.z, "truncated", capacity=333)
        finally:
            B.ht_set_tuning(CFG1)
    spec = synth.GridSpec(4, 16, 130, 72, threshold=4)
    try:
        B.ht_set_tuning(spec, rows=64, group_tiles=64)
        x, y, z = random_hits(5, 2000)
        check(B, spec, x, y, z, "small grid, groups of 64 tiles of 64 rows, stage %s" % stage)
    finally:
        B.ht_set_tuning(spec)


def test_dense_paper_events_and_truncation(gpu, env):
    B = gpu
    env["HT_DENSE_HITS"] = "1"
    for e in range(3):
        ev = synth.make_event(1, 50 + e)
        say("dense paper event %d (%d hits)" % (e, ev.n))
        check(B, CFG1, ev.x, ev.y, ev.z, "paper event %d" % e)
    ev = synth.make_event(1, 60)
    check(B, CFG1, ev.x, ev.y, ev.z, "truncated", capacity=100)


def test_dense_largest_served_event_by_default(gpu):
    """The 40000-hit served event takes the stencil at the library's default threshold."""
    B = gpu
    ev = synth.make_event(3, next(e for e in range(40) if synth.event_size(3, e) == 40000))
    assert ev.n >= B.ht_get_tuning(CFG1).dense_hits
    say("largest served event, default threshold: %d hits" % ev.n)
    n = check(B, CFG1, ev.x, ev.y, ev.z, "40k-hit event", capacity=1 << 19)
    assert n > 100000


def test_dense_peaks_to_pinned_host(gpu, env):
    import torch
    B = gpu
    env["HT_DENSE_HITS"] = "1"
    ev = synth.make_event(1, 70)
    M, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
    x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
    acc = B.new_acc(CFG1)
    cap = 4096
    for off in (0, 1):   # 8-byte and 4-byte aligned outputs
        buf = torch.zeros((cap + 1) * 2, dtype=torch.int32, pin_memory=True)
        out = buf[off:off + 2 * cap].view(cap, 2)
        nf = torch.zeros(1, dtype=torch.int64, pin_memory=True)
        B.ht_fill_peaks(CFG1, x, y, z, acc, out, cap, nf)
        torch.cuda.synchronize()
        n = int(nf.item())
        got = out.numpy().view(np.uint32)[:n]
        assert n == on and np.array_equal(got[:, 0], oc) and np.array_equal(got[:, 1], ov)


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
def test_dense_and_pool_events_in_one_batch(gpu, env, graph):
    B = gpu
    env["HT_BATCH_GRAPH"] = "1" if graph else "0"
    evs = [synth.make_event(0, 200 + i) for i in range(8)]
    # events of 250 hits: threshold 200 makes all dense, 10**6 none; a mixed batch by trimming
    trimmed = []
    for i, e in enumerate(evs):
        k = 150 if i % 2 else e.n
        trimmed.append(synth.Event(e.x[:k], e.y[:k], e.z[:k]))
    env["HT_DENSE_HITS"] = "200"
    res = B.fill_peaks_batch(CFG0, [(e.x, e.y, e.z) for e in trimmed], capacity=1 << 12)
    acc = B.as_u32(res.acc)
    for i, e in enumerate(trimmed):
        M, oc, ov, on = oracle_run(CFG0, e.x, e.y, e.z)
        c, v, n = res.peaks[i]
        assert np.array_equal(acc[i], M), i
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), i


def test_dense_request_loop(gpu, env):
    B = gpu
    env["HT_DENSE_HITS"] = "2000"
    evs = [synth.make_event(1, 80 + i) for i in range(3)]
    small = [synth.make_event(0, 300 + i) for i in range(3)]
    mix = [evs[0], small[0], evs[1], small[1], evs[2], small[2]]
    with B.Server(CFG1, 4 << 30, peak_capacity=1 << 14, max_hits=6000, max_batch=4, n_streams=2,
                  queue_depth=16) as srv:
        tickets = [srv.submit(e.x, e.y, e.z) for e in mix]
        assert all(t is not None for t in tickets)
        import time
        got = {}
        deadline = time.time() + 60
        while len(got) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in got:
                    r = srv.poll(t)
                    if r is not None:
                        got[t] = r
            time.sleep(1e-4)
        assert len(got) == len(tickets)
    for t, e in zip(tickets, mix):
        M, oc, ov, on = oracle_run(CFG1, e.x, e.y, e.z)
        c, v, n, _ = got[t]
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)
