"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Vote counts are integers and the bin rule is fixed binary32 arithmetic on both sides, so every
comparison here is exact: vote matrices element by element, peak lists entry by entry.
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
    return B


@pytest.fixture()
def env_tiling():
    keys = ("HT_FILL_ROWS", "HT_CAND_CAP", "HT_FILL_LDS_BYTES", "HT_BATCH_GRAPH", "HT_POOL_BOUND",
            "HT_BATCH_PIECES", "HT_DENSE_HITS")
    saved = {k: os.environ.get(k) for k in keys}
    yield
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


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


def assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, tag=""):
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


# ---------------------------------------------------------------------------------------------
def test_hit_values_match_oracle(gpu):
    """r2, sqrt(r2), 1/(2y), half-sectors and cells of the device prep equal the oracle's bits."""
    import torch
    from oracle import oracle
    B = gpu
    rng = np.random.default_rng(1)
    n = 1 << 20
    mag = 10.0 ** rng.uniform(-3, 4, (3, n))
    sign = np.where(rng.random((3, n)) < 0.5, -1.0, 1.0)
    x, y, z = (mag * sign).astype(np.float32)
    # exact half-sector boundaries and degenerate values
    ang = np.arange(64) * np.pi / 16
    x[:64] = (500 * np.cos(ang)).astype(np.float32)
    y[:64] = (500 * np.sin(ang)).astype(np.float32)
    x[64:80] = [0, 0, 1, np.inf, np.nan, 1e30, -1e30, 3e19, 1e-30, 5, -5, 0, 7, 1e-20, 2e-23, 1e38]
    y[64:80] = [0, 1, 0, 1, 1, 1e30, 1e-30, 3e19, 1e-30, -0.0, 0.0, -3, np.inf, 1e-20, 2e-23, 1e38]
    for spec in (CFG0, CFG4, synth.GridSpec(3, 5, 7, 9, threshold=2)):
        say("hit values: grid", spec.shape)
        xd, yd, zd = B.hits_to_device(x, y, z)
        info, vals, slabs = B.ht_debug_hit_values(spec, xd, yd, zd)
        torch.cuda.synchronize()
        info, vals, slabs = info.cpu().numpy(), vals.cpu().numpy(), slabs.cpu().numpy()
        o = oracle.hit_info(oracle.OracleGrid(*spec.as_tuple()), x, y, z)
        assert np.array_equal(info[:, 0].astype(bool), o["valid"])
        v = o["valid"]
        assert np.array_equal(info[v, 1], o["s_theta"][v])
        assert np.array_equal(info[v, 2], o["s_phi"][v])
        assert np.array_equal(info[:, 3], o["n_cells"])
        for col, key in ((0, "r2"), (1, "r"), (2, "k")):
            assert vals[v, col].tobytes() == o[key][v].tobytes(), key
        oslab = np.where(o["cells"][:, :, 0] >= 0, o["cells"][:, :, 0] * spec.n_phi + o["cells"][:, :, 1], -1)
        assert np.array_equal(slabs, oslab)


def test_cfg0_events_bit_exact(gpu):
    B = gpu
    nonempty = 0
    for e in range(100):
        ev = synth.make_event(0, e)
        if e % 25 == 0:
            say("workload 0 event", e)
        gM, gc, gv, gn = gpu_fused(B, CFG0, ev.x, ev.y, ev.z)
        M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
        assert_same(CFG0, gM, gc, gv, gn, M, oc, ov, on, "event %d" % e)
        assert int(gM.sum(dtype=np.int64)) == votes
        nonempty += on > 0
    assert nonempty >= 40


def test_fill_paths_agree(gpu):
    """ht_fill (LDS tiles), ht_fill_atomic (global atomics) and the fused call give one matrix;
    ht_peaks on it gives the oracle's peaks."""
    import torch
    B = gpu
    for e in range(5):
        ev = synth.make_event(0, 200 + e)
        say("fill paths: workload 0 event", 200 + e)
        xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
        a1 = B.fill(CFG0, xd, yd, zd)
        a2 = B.fill(CFG0, xd, yd, zd, atomic=True)
        a3, _, _, _ = B.fill_peaks(CFG0, xd, yd, zd)
        torch.cuda.synchronize()
        M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
        for a in (a1, a2, a3):
            assert np.array_equal(B.as_u32(a), M)
        c, v, n = B.peaks(CFG0, a1)
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)


@pytest.mark.parametrize("shape,T", [((2, 4, 8, 8), 3), ((3, 5, 7, 9), 3), ((4, 16, 64, 64), 4),
                                     ((1, 3, 5, 1), 2), ((2, 3, 40, 130), 5), ((3, 4, 33, 64), 6)])
def test_peaks_on_arbitrary_matrices(gpu, shape, T):
    import torch
    from oracle import oracle
    B = gpu
    say("peaks on a random matrix", shape)
    rng = np.random.default_rng(sum(shape) + T)
    M = rng.integers(0, 4, size=shape).astype(np.uint32)
    spikes = rng.random(shape) < 0.03
    M[spikes] += rng.integers(3, 12, size=int(spikes.sum())).astype(np.uint32)
    spec = synth.GridSpec(*shape, threshold=T)
    acc = torch.from_numpy(M.view(np.int32).copy()).cuda()
    c, v, n = B.peaks(spec, acc)
    oc, ov, on = oracle.peaks(oracle.OracleGrid(*spec.as_tuple()), M)
    assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)


RAGGED = [
    synth.GridSpec(3, 5, 7, 9, a_min=-1500.0, a_max=1300.0, b_min=-1100.0, b_max=1700.0, threshold=2),
    synth.GridSpec(2, 7, 100, 37, a_min=-999.0, a_max=1234.5, b_min=-1500.0, b_max=2000.0, threshold=3),
    synth.GridSpec(4, 16, 130, 66, threshold=4),
    synth.GridSpec(1, 3, 1, 1, threshold=1),
    synth.GridSpec(5, 3, 257, 1000, threshold=3),
    synth.GridSpec(2, 4, 3, 20000, threshold=2),   # rows too wide for an LDS tile: atomic fill
]


@pytest.mark.parametrize("spec", RAGGED, ids=lambda s: "x".join(map(str, s.shape)))
def test_ragged_grids_bit_exact(gpu, spec):
    B = gpu
    for seed in range(3):
        say("ragged grid", spec.shape, "seed", seed)
        x, y, z = random_hits(seed, 300 if spec.n_b < 10000 else 60)
        gM, gc, gv, gn = gpu_fused(B, spec, x, y, z)
        M, votes, oc, ov, on = oracle_run(spec, x, y, z)
        assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "seed %d" % seed)


# The peak test gives each workgroup one contiguous run of the candidate pool once there are more
# than four candidates per wave of its grid (max(16, min(1024, ceil(n_tiles / 16))) workgroups),
# and numbers the runs per XCD when that grid is a multiple of 8. These grids have 495 tiles (31
# workgroups: plain numbering), 384 (24: XCD numbering, not a power of two) and 192 (16), each with
# thousands of candidates, so the runs end in ragged tails.
MANY_CANDIDATES = [((5, 3, 257, 1000), 495), ((3, 4, 256, 1000), 384), ((4, 16, 130, 66), 192)]


@pytest.mark.parametrize("shape,n_tiles", MANY_CANDIDATES, ids=lambda v: "x".join(map(str, v))
                         if isinstance(v, tuple) else str(v))
def test_many_candidates_every_run_layout_bit_exact(gpu, shape, n_tiles):
    B = gpu
    spec = synth.GridSpec(*shape, threshold=2)
    assert B.ht_tiling(spec)["n_tiles"] == n_tiles
    for seed in range(2):
        say("many candidates", shape, "seed", seed)
        x, y, z = random_hits(seed, 300)
        gM, gc, gv, gn = gpu_fused(B, spec, x, y, z)
        M, votes, oc, ov, on = oracle_run(spec, x, y, z)
        assert int((M >= spec.threshold).sum()) > 16 * max(16, (n_tiles + 15) // 16)
        assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "seed %d" % seed)


@pytest.mark.parametrize("rows", [1, 2, 4, 8, 16, 32, 64])
def test_every_tile_shape_bit_exact(gpu, rows):
    """Every launch shape the tuner can pick gives the same bits."""
    B = gpu
    for spec, ev in ((CFG0, synth.make_event(0, 3)), (synth.GridSpec(4, 16, 100, 40, threshold=4),
                                                       synth.make_event(0, 4))):
        M, votes, oc, ov, on = oracle_run(spec, ev.x, ev.y, ev.z)
        # tiles per workgroup 3 is not allowed; 1, 4 and 16 cover workgroups whose tiles
        # stay in one slab, span slabs, and run past the last tile
        for gt, nt, tpb in ((16, 0, 1), (64, 1, 4), (32, 2, 16)):
            say("tile rows", rows, "group tiles", gt, "store", nt, "tiles/block", tpb, "grid", spec.shape)
            B.ht_set_tuning(spec, rows=rows, group_tiles=gt, nt_store=nt, tiles_per_block=tpb)
            try:
                gM, gc, gv, gn = gpu_fused(B, spec, ev.x, ev.y, ev.z)
            finally:
                B.ht_set_tuning(spec)
            assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "rows %d" % rows)


def test_paper_grid_tile_shapes_bit_exact(gpu):
    B = gpu
    ev = synth.make_event(1, 7)
    M, votes, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
    for rows in (1, 2, 4, 8):
        for nt, tpb in ((0, 1), (1, 8), (2, 16), (0, 64)):
            say("workload 1, rows", rows, "store", nt, "tiles/block", tpb)
            B.ht_set_tuning(CFG1, rows=rows, nt_store=nt, group_tiles=32, tiles_per_block=tpb)
            try:
                gM, gc, gv, gn = gpu_fused(B, CFG1, ev.x, ev.y, ev.z)
            finally:
                B.ht_set_tuning(CFG1)
            assert_same(CFG1, gM, gc, gv, gn, M, oc, ov, on, "rows %d store %d tpb %d" % (rows, nt, tpb))


def test_candidate_overflow_uses_dense_path(gpu, env_tiling):
    """With 2 candidate slots per tile (and the pool not sized by the event's vote bound),
    crowded tiles overflow and are searched densely; the results must not change."""
    import torch
    B = gpu
    os.environ["HT_POOL_BOUND"] = "0"
    B.ht_set_tuning(CFG0, cand_cap=2)
    try:
        for e in (0, 1, 2):
            say("candidate overflow, workload 0 event", e)
            ev = synth.make_event(0, e)
            gM, gc, gv, gn = gpu_fused(B, CFG0, ev.x, ev.y, ev.z)
            M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
            assert_same(CFG0, gM, gc, gv, gn, M, oc, ov, on)
            acc = torch.from_numpy(M.view(np.int32).copy()).cuda()
            c, v, n = B.peaks(CFG0, acc)
            assert n == on and np.array_equal(c, oc)
    finally:
        B.ht_set_tuning(CFG0)


# the launch shape bench.py pins for its main line (rows 4, groups of 16 tiles, the default pool
# entries per tile, non-temporal stores, one tile per workgroup)
BENCH_SHAPE = dict(rows=4, group_tiles=16, cand_cap=0, nt_store=1, tiles_per_block=1)


@pytest.mark.parametrize("shape", ["default", "bench"])
def test_paper_sized_events_bit_exact(gpu, shape):
    """The 4x16x1024x1024 workload (5000 hits) at the library's default shape and at the shape
    the benchmark times."""
    B = gpu
    if shape == "bench":
        B.ht_set_tuning(CFG1, **BENCH_SHAPE)
    try:
        for e in (0, 1, 2):
            say("workload 1 event", e, shape)
            ev = synth.make_event(1, e)
            gM, gc, gv, gn = gpu_fused(B, CFG1, ev.x, ev.y, ev.z)
            M, votes, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
            assert_same(CFG1, gM, gc, gv, gn, M, oc, ov, on, "event %d %s" % (e, shape))
            assert on > 100
    finally:
        B.ht_set_tuning(CFG1)


def test_empty_and_degenerate_events(gpu):
    import torch
    B = gpu
    say("empty and degenerate events")
    # no hits: the matrix is all zero (it is overwritten, not accumulated) and there are no peaks
    acc = B.new_acc(CFG0)
    acc.fill_(7)
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    out, nf = B.new_peaks(16)
    B.ht_fill_peaks(CFG0, e, e, e, acc, out, 16, nf)
    torch.cuda.synchronize()
    assert not acc.any() and int(nf.item()) == 0
    # hits that vote nothing
    x = np.array([0, 0, np.nan, np.inf, 4, 1e30], np.float32)
    y = np.array([0, 0, 1, 1, 0, 1e30], np.float32)
    z = np.array([0, 1, 1, 1, 1, 1], np.float32)
    gM, gc, gv, gn = gpu_fused(B, CFG0, x, y, z)
    assert not gM.any() and gn == 0
    # capacity 0 and truncated capacity still report the total
    ev = synth.make_event(0, 1)
    M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
    assert on >= 3
    xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
    acc = B.new_acc(CFG0)
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    B.ht_fill_peaks(CFG0, xd, yd, zd, acc, None, 0, nf)
    torch.cuda.synchronize()
    assert int(nf.item()) == on
    out, nf = B.new_peaks(2)
    B.ht_fill_peaks(CFG0, xd, yd, zd, acc, out, 2, nf)
    torch.cuda.synchronize()
    c, v, n = B.peaks_to_host(out, nf, 2, allow_truncation=True)
    assert n == on and np.array_equal(c, oc[:2]) and np.array_equal(v, ov[:2])
    # the wrapper refuses a truncated list unless asked for one
    with pytest.raises(B.HTError) as err:
        B.peaks_to_host(out, nf, 2)
    assert err.value.code == B.HT_EOVERFLOW
    # threshold above every count
    spec = synth.GridSpec(4, 16, 64, 64, threshold=10 ** 6)
    gM, gc, gv, gn = gpu_fused(B, spec, ev.x, ev.y, ev.z)
    assert gn == 0 and np.array_equal(gM, M)


@pytest.mark.parametrize("n_hits", [40, 900])
@pytest.mark.parametrize("rows", [0, 4, 8])
def test_bin_edges_bit_exact(gpu, n_hits, rows):
    """Votes exactly on the B range's edges: B = 0 (as -0 for y < 0: still in bin 0) and B = b_max
    (outside the half-open range), with A-bin centres on integers, through the short-list fill
    (40 hits) and the branch-free long-list fill (900 hits: more than two records per thread and
    slab), with a short last tile (10 A rows in tiles of 4 or 8)."""
    B = gpu
    spec = synth.GridSpec(1, 4, 10, 16, a_min=0.0, a_max=20.0, b_min=0.0, b_max=16.0, threshold=3)
    say("bin edges", n_hits, rows)
    rng = np.random.default_rng(7 + n_hits + rows)
    edge = np.array([(8.0, -4.0), (8.0, 4.0), (0.0, 32.0), (0.0, 31.5), (0.0, -2.0)], np.float32)
    pick = rng.integers(0, len(edge), n_hits // 2)
    x = np.concatenate([edge[pick, 0], rng.uniform(-20.0, 20.0, n_hits - pick.size)]).astype(np.float32)
    y = np.concatenate([edge[pick, 1], rng.uniform(-20.0, 20.0, n_hits - pick.size)]).astype(np.float32)
    z = rng.uniform(-5.0, 5.0, n_hits).astype(np.float32)
    if rows:
        B.ht_set_tuning(spec, rows=rows)
    try:
        gM, gc, gv, gn = gpu_fused(B, spec, x, y, z)
    finally:
        B.ht_set_tuning(spec)
    M, votes, oc, ov, on = oracle_run(spec, x, y, z)
    assert int(M[0, :, 2, 0].sum()) >= 2  # the B = 0 votes are there
    assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "edges %d %d" % (n_hits, rows))


def boundary_hits(n_theta, n_phi, seed):
    """Hits on and next to the sector boundaries: azimuths m pi / n_phi and polar angles
    m pi / (2 n_theta) (the edges of the half-widened cells), each direction also one float32 step
    either side in x, y and z, at several radii."""
    rng = np.random.default_rng(seed)
    xs, ys, zs = [], [], []
    for m in range(2 * n_phi):
        ph = m * np.pi / n_phi
        for mt in range(1, 2 * n_theta):
            th = mt * np.pi / (2 * n_theta)
            for r in rng.uniform(30.0, 1000.0, 2):
                x, y = np.float32(r * np.cos(ph)), np.float32(r * np.sin(ph))
                z = np.float32(r / np.tan(th)) if abs(np.tan(th)) > 1e-12 else np.float32(0.0)
                for dx, dy, dz in ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    xs.append(np.nextafter(x, np.float32(np.inf * dx)) if dx else x)
                    ys.append(np.nextafter(y, np.float32(np.inf * dy)) if dy else y)
                    zs.append(np.nextafter(z, np.float32(np.inf * dz)) if dz else z)
    return (np.array(xs, np.float32), np.array(ys, np.float32), np.array(zs, np.float32))


@pytest.mark.parametrize("spec", [CFG0, synth.GridSpec(3, 5, 64, 64, threshold=3),
                                  synth.GridSpec(2, 4, 48, 40, threshold=2, phi_sectors=True)])
def test_sector_boundaries_bit_exact(gpu, spec):
    """Hits exactly on, and one float32 step off, every theta and phi boundary direction: the
    half-plane tests of the preparation against the oracle's, through the whole fused call."""
    B = gpu
    x, y, z = boundary_hits(spec.n_theta, spec.n_phi, 11)
    say("sector boundaries", spec.shape, x.size)
    gM, gc, gv, gn = gpu_fused(B, spec, x, y, z)
    M, votes, oc, ov, on = oracle_run(spec, x, y, z)
    assert votes > 0
    assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "boundaries %s" % (spec.shape,))


def test_batch_matches_single_events(gpu):
    B = gpu
    hits, specs = [], CFG0
    for e in range(24):
        ev = synth.make_event(0, 300 + e)
        k = [ev.n, 0, 1, 17][e % 4]  # uneven sizes, including empty events
        hits.append((ev.x[:k], ev.y[:k], ev.z[:k]))
    say("batch of", len(hits), "workload-0 events")
    res = B.fill_peaks_batch(specs, hits, capacity=64)
    accs = B.as_u32(res.acc)
    for i, (x, y, z) in enumerate(hits):
        M, votes, oc, ov, on = oracle_run(specs, x, y, z)
        assert np.array_equal(accs[i], M), i
        c, v, n = res.peaks[i]
        assert n == on and np.array_equal(c, oc[:64]) and np.array_equal(v, ov[:64]), i


def test_batch_graph_replays_match_eager(gpu, env_tiling):
    """The batch runs as a captured HIP graph. Replay it on several batches of one shape, with
    host work and synchronisation in between, and compare each replay with the direct launches
    of the same batch and with the oracle."""
    import torch
    B = gpu
    for rep in range(4):
        hits = []
        for e in range(12):
            ev = synth.make_event(0, 500 + 12 * rep + e)
            k = ev.n - (e % 3) * 40
            hits.append((ev.x[:k], ev.y[:k], ev.z[:k]))
        say("graph replay", rep)
        os.environ["HT_BATCH_GRAPH"] = "1"
        g_res = B.fill_peaks_batch(CFG0, hits, capacity=64)
        os.environ["HT_BATCH_GRAPH"] = "0"
        e_res = B.fill_peaks_batch(CFG0, hits, capacity=64)
        os.environ.pop("HT_BATCH_GRAPH")
        torch.cuda.synchronize()
        assert np.array_equal(B.as_u32(g_res.acc), B.as_u32(e_res.acc))
        for i, (x, y, z) in enumerate(hits):
            M, votes, oc, ov, on = oracle_run(CFG0, x, y, z)
            assert np.array_equal(B.as_u32(g_res.acc)[i], M)
            for res in (g_res, e_res):
                c, v, n = res.peaks[i]
                assert n == on and np.array_equal(c, oc[:64]) and np.array_equal(v, ov[:64])


@pytest.mark.parametrize("pieces,graph", [(2, True), (3, False), (8, True)])
def test_batch_split_into_overlapping_runs(gpu, env_tiling, pieces, graph):
    """HT_BATCH_PIECES: the batch's fills in runs, each run's peak search on a side stream beside
    the next run's fill (candidate pool and stencil events mixed), against the oracle."""
    B = gpu
    os.environ["HT_BATCH_PIECES"] = str(pieces)
    os.environ["HT_BATCH_GRAPH"] = "1" if graph else "0"
    os.environ["HT_DENSE_HITS"] = "200"  # the 250-hit events take the stencil, trimmed ones the pool
    hits = []
    for e in range(11):
        ev = synth.make_event(0, 700 + e)
        k = [ev.n, 150, 0, ev.n - 20][e % 4]
        hits.append((ev.x[:k], ev.y[:k], ev.z[:k]))
    say("batch in %d runs (%s)" % (pieces, "graph" if graph else "eager"))
    res = B.fill_peaks_batch(CFG0, hits, capacity=256)
    accs = B.as_u32(res.acc)
    for i, (x, y, z) in enumerate(hits):
        M, votes, oc, ov, on = oracle_run(CFG0, x, y, z)
        assert np.array_equal(accs[i], M), i
        c, v, n = res.peaks[i]
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), i


def test_batch_of_uneven_paper_sized_events(gpu):
    """Workload-2 events (1000-8000 hits) on the 4x16x1024x1024 grid, batched, vs the oracle."""
    B = gpu
    evs = [synth.make_event(2, e) for e in range(6)]
    say("batch of 6 workload-2 events, sizes", [e.n for e in evs])
    res = B.fill_peaks_batch(CFG1, [(e.x, e.y, e.z) for e in evs], capacity=1 << 14)
    accs = B.as_u32(res.acc)
    for i, ev in enumerate(evs):
        M, votes, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
        assert np.array_equal(accs[i], M), i
        c, v, n = res.peaks[i]
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), i
    del res, accs


def serve_all(B, spec, events, opts):
    import time
    lib = B.lib()
    g = B.make_grid(spec)
    srv = ctypes.c_void_p()
    B.check(lib.ht_serve_create(ctypes.byref(g), ctypes.byref(opts), ctypes.byref(srv)))
    try:
        tickets = []
        for ev in events:
            t = ctypes.c_uint64()
            fp = ctypes.POINTER(ctypes.c_float)
            while True:
                rc = lib.ht_serve_submit(srv, ev.x.ctypes.data_as(fp), ev.y.ctypes.data_as(fp),
                                         ev.z.ctypes.data_as(fp), ev.n, ctypes.byref(t))
                if rc != B.HT_EAGAIN:
                    break
                time.sleep(1e-4)
            B.check(rc)
            tickets.append(t.value)
        results = {}
        cap = opts.peak_capacity
        deadline = time.time() + 60
        while len(results) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t in results:
                    continue
                out = (B.Peak * cap)()
                nf = ctypes.c_int64()
                tm = B.Timing()
                rc = lib.ht_serve_poll(srv, t, out, cap, ctypes.byref(nf), ctypes.byref(tm))
                if rc == B.HT_EAGAIN:
                    continue
                B.check(rc)
                k = min(nf.value, cap)
                arr = np.frombuffer(out, dtype=np.uint32).reshape(-1, 2)[:k]
                results[t] = (arr[:, 0].copy(), arr[:, 1].copy(), nf.value, tm)
            time.sleep(1e-4)
        assert len(results) == len(tickets), "server did not finish"
        # a released ticket is unknown
        nf = ctypes.c_int64()
        assert lib.ht_serve_poll(srv, tickets[0], None, 0, ctypes.byref(nf), None) == B.HT_EINVAL
        return [results[t] for t in tickets]
    finally:
        lib.ht_serve_destroy(srv)


def test_serve_results_equal_alone_and_in_the_mix(gpu):
    B = gpu
    evs = [synth.make_event(0, 400 + e) for e in range(30)]
    one_slot = (4 * CFG0.n_cells + (8 << 20))
    opts = B.ServeOpts(3 * one_slot, 256, 2000, 4, 2, 64, 0)   # three slots: admission limits
    say("serve: 30 workload-0 events, 3 slots, 2 streams")
    mixed = serve_all(B, CFG0, evs, opts)
    for ev, (c, v, n, tm) in zip(evs, mixed):
        M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)
        assert tm.t_submit <= tm.t_admit <= tm.t_launch <= tm.t_done
    say("serve: the same events one at a time")
    for ev, (c, v, n, tm) in zip(evs[:5], mixed[:5]):
        (c1, v1, n1, _), = serve_all(B, CFG0, [ev], opts)
        assert n1 == n and np.array_equal(c1, c) and np.array_equal(v1, v)


def test_serve_paper_grid(gpu):
    B = gpu
    evs = [synth.make_event(3, e) for e in range(4)]
    say("serve: 4 workload-3 events, sizes", [e.n for e in evs])
    opts = B.ServeOpts(4 << 30, 1 << 17, 40000, 2, 2, 8, 0)
    res = serve_all(B, CFG1, evs, opts)
    for ev, (c, v, n, tm) in zip(evs, res):
        M, votes, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)


def test_largest_served_event_bit_exact(gpu):
    """The largest event of the served workload (40000 hits, about 2.6M cells at or above the
    threshold on the paper grid): more candidates than cand_cap per tile of the default shape,
    so its pool is sized by the vote bound. Plain call (default shape) and request loop against
    the oracle."""
    import torch
    B = gpu
    ev = max((synth.make_event(3, e) for e in range(40)), key=lambda e: e.n)
    assert ev.n == 40000
    say("largest served event: %d hits, plain path" % ev.n)
    M, votes, oc, ov, on = oracle_run(CFG1, ev.x, ev.y, ev.z)
    assert on > 1 << 15
    gM, gc, gv, gn = gpu_fused(B, CFG1, ev.x, ev.y, ev.z, capacity=1 << 19)
    assert_same(CFG1, gM, gc, gv, gn, M, oc, ov, on, "plain")
    del gM
    say("largest served event: request loop")
    opts = B.ServeOpts(4 << 30, 1 << 19, 40000, 2, 2, 8, 0)
    (c, v, n, tm), = serve_all(B, CFG1, [ev], opts)
    assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)
    torch.cuda.empty_cache()


def test_stress_event_full_size(gpu):
    """One 105600-hit event on the 8x32x2048x2048 grid (4 GiB of counts), bit-exact."""
    import torch
    B = gpu
    ev = synth.make_event(4, 0)
    say("stress event: workload 4, 105600 hits, 1G cells")
    xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
    acc, gc, gv, gn = B.fill_peaks(CFG4, xd, yd, zd, capacity=1 << 22)
    torch.cuda.synchronize()
    M, votes, oc, ov, on = oracle_run(CFG4, ev.x, ev.y, ev.z)
    say("stress event: oracle done, comparing")
    gM = B.as_u32(acc)
    del acc
    torch.cuda.empty_cache()
    assert np.array_equal(gM, M)
    assert gn == on and np.array_equal(gc, oc) and np.array_equal(gv, ov)


def test_autotuner_keeps_results_and_caches(gpu, tmp_path):
    from paper_1507_03074_amd import tune
    B = gpu
    evs = [synth.make_event(0, 600 + e) for e in range(2)]
    say("autotune workload-0 grid")
    rep = tune.autotune(CFG0, [(e.x, e.y, e.z) for e in evs], reps=3)
    assert rep["best"] is not None and rep["best"]["bit_exact"]
    assert all(c["bit_exact"] for c in rep["candidates"])
    try:
        applied = B.ht_get_tuning(CFG0).as_dict()
        assert applied == rep["best"]["tuning"]
        path = str(tmp_path / "cache.json")
        tune.save(rep, path)
        B.ht_set_tuning(CFG0)
        assert tune.load(CFG0, path)
        assert B.ht_get_tuning(CFG0).as_dict() == rep["best"]["tuning"]
        ev = synth.make_event(0, 610)
        gM, gc, gv, gn = gpu_fused(B, CFG0, ev.x, ev.y, ev.z)
        M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
        assert_same(CFG0, gM, gc, gv, gn, M, oc, ov, on)
    finally:
        B.ht_set_tuning(CFG0)


def test_readout_matches_oracle(gpu):
    """ht_readout (device, double rounded to float) against the oracle's readout in double:
    indices and votes exact, A and B exact (bin centres), rho/phi/theta within 1 ulp of float."""
    import torch
    from oracle import oracle
    B = gpu
    for spec, wl, e in ((CFG0, 0, 1), (CFG1, 1, 2), (synth.GridSpec(3, 5, 7, 9, threshold=2), 0, 3)):
        say("readout", spec.shape)
        ev = synth.make_event(wl, e)
        xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
        cap = 1 << 15
        acc = B.new_acc(spec)
        out, nf = B.new_peaks(cap)
        B.ht_fill_peaks(spec, xd, yd, zd, acc, out, cap, nf)
        tr = B.tracks_to_host(B.ht_readout(spec, out, nf, cap), nf, cap)
        torch.cuda.synchronize()
        cells, votes, n = B.peaks_to_host(out, nf, cap)
        assert n > 0 and len(tr) == n
        r = oracle.readout(oracle.OracleGrid(*spec.as_tuple()), cells)
        assert np.array_equal(tr["cell"], cells) and np.array_equal(tr["votes"], votes)
        for k in ("t", "p", "a", "b"):
            assert np.array_equal(tr[k], r[k]), k
        for k in ("A", "B", "rho", "phi", "theta"):
            ref = r[k].astype(np.float32)
            diff = np.abs(tr[k].astype(np.float64) - ref.astype(np.float64))
            assert np.all(diff <= np.spacing(np.abs(ref)).astype(np.float64)), k


def test_physics_single_track_found(gpu):
    """A noiseless single track: the peak's readout gives the generating (A, B) bin centre."""
    import torch
    from paper_1507_03074_amd import physics
    B = gpu
    spec = synth.GridSpec(4, 16, 1024, 1024, threshold=12)
    A0 = -2000.0 + (700 + 0.5) * 4000.0 / 1024
    B0 = -2000.0 + (300 + 0.5) * 4000.0 / 1024
    x, y, z, _, _ = synth.helix_hits([A0], [B0], [1.0], [0.3])
    x, y, z = (v.astype(np.float32) for v in (x, y, z))
    xd, yd, zd = B.hits_to_device(x, y, z)
    acc = B.new_acc(spec)
    out, nf = B.new_peaks(64)
    B.ht_fill_peaks(spec, xd, yd, zd, acc, out, 64, nf)
    tr = B.tracks_to_host(B.ht_readout(spec, out, nf, 64), nf, 64)
    torch.cuda.synchronize()
    assert len(tr) == 1 and tr["votes"][0] == 12
    assert (tr["a"][0], tr["b"][0]) == (700, 300)
    assert tr["A"][0] == np.float32(A0) and tr["B"][0] == np.float32(B0)
    fa, fb = physics.lsq_circle_through_origin(x, y)
    assert abs(fa - A0) < 1e-2 and abs(fb - B0) < 1e-2


def test_peaks_written_to_pinned_host_memory(gpu):
    """The peak kernels write straight into pinned host memory (no copy); results equal the
    oracle's on consecutive events, so no stale data survives between calls."""
    import torch
    B = gpu
    cap = 4096
    h_out = torch.zeros((cap, 2), dtype=torch.int32, pin_memory=True)
    h_nf = torch.zeros(1, dtype=torch.int64, pin_memory=True)
    acc = B.new_acc(CFG0)
    for e in range(8):
        ev = synth.make_event(0, 700 + e)
        say("pinned output, event", 700 + e)
        xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
        B.ht_fill_peaks(CFG0, xd, yd, zd, acc, h_out, cap, h_nf)
        torch.cuda.synchronize()
        M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
        assert int(h_nf[0]) == on
        got = h_out.numpy().view(np.uint32)[:on]
        assert np.array_equal(got[:, 0], oc) and np.array_equal(got[:, 1], ov)


def test_peaks_into_4_byte_aligned_output(gpu):
    """Peak lists that start 4 bytes past an 8-byte boundary (in device memory and in pinned host
    memory) take the two-store path and equal the oracle's; the 8-byte aligned ones take one
    8-byte store per peak."""
    import torch
    B = gpu
    cap = 4096
    acc = B.new_acc(CFG0)
    for where in ("cuda", "pinned"):
        if where == "cuda":
            base = torch.zeros(2 * cap + 1, dtype=torch.int32, device="cuda")
            nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        else:
            base = torch.zeros(2 * cap + 1, dtype=torch.int32, pin_memory=True)
            nf = torch.zeros(1, dtype=torch.int64, pin_memory=True)
        out = base[1:].view(cap, 2)
        assert out.data_ptr() % 8 == 4
        for e in range(4):
            ev = synth.make_event(0, 720 + e)
            say("4-byte aligned output,", where, "event", 720 + e)
            xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
            B.ht_fill_peaks(CFG0, xd, yd, zd, acc, out, cap, nf)
            torch.cuda.synchronize()
            M, votes, oc, ov, on = oracle_run(CFG0, ev.x, ev.y, ev.z)
            assert int(nf.cpu()[0]) == on
            got = out.cpu().numpy().view(np.uint32)[:on]
            assert np.array_equal(got[:, 0], oc) and np.array_equal(got[:, 1], ov)
            assert int(base.cpu()[0]) == 0  # nothing written before the array


def test_output_pointer_classification(gpu):
    """The host-side check that guards the peak outputs: device memory and mapped pinned host
    memory are accepted, unregistered host memory is refused. Only the classification is
    queried here (host only); no kernel is ever given a refused pointer."""
    import torch
    B = gpu
    dev = torch.zeros(16, dtype=torch.int32, device="cuda")
    pinned = torch.zeros(16, dtype=torch.int32, pin_memory=True)
    plain = torch.zeros(16, dtype=torch.int32)
    arr = np.zeros(16, np.int32)
    assert B.ht_debug_pointer_kind(dev.data_ptr()) == 1
    assert B.ht_debug_pointer_kind(pinned.data_ptr()) == 2
    assert B.ht_debug_pointer_kind(pinned.data_ptr() + 8) == 2
    assert B.ht_debug_pointer_kind(plain.data_ptr()) == 0
    assert B.ht_debug_pointer_kind(arr.ctypes.data) == 0


def test_alternating_grid_sizes_keep_counters_clean(gpu):
    """Calls alternate between grids with many and few (theta, phi) cells on one stream; the
    per-slab counters carried between calls must not leak counts from one grid to the next."""
    B = gpu
    big = synth.GridSpec(4, 16, 130, 66, threshold=4)
    small = synth.GridSpec(3, 5, 7, 9, threshold=2)
    wide = synth.GridSpec(8, 32, 16, 16, threshold=3)
    for k, spec in enumerate([big, small, big, wide, small, big, wide, big]):
        say("alternating grids, call", k, spec.shape)
        x, y, z = random_hits(100 + k, 300)
        gM, gc, gv, gn = gpu_fused(B, spec, x, y, z)
        M, votes, oc, ov, on = oracle_run(spec, x, y, z)
        assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "call %d" % k)


# ---------------------------------------------------------------------------------------------
# Sector variant (paper section 4): phi cells are independent sectors
# ---------------------------------------------------------------------------------------------
def sector_grid(spec, n_phi):
    return synth.GridSpec(spec.n_theta, n_phi, spec.n_a, spec.n_b, spec.a_min, spec.a_max,
                          spec.b_min, spec.b_max, spec.threshold, phi_sectors=True)


SECTOR_GRIDS = [sector_grid(CFG0, 4), sector_grid(CFG0, 16), sector_grid(CFG0, 1),
                synth.GridSpec(3, 2, 7, 9, a_min=-1500.0, a_max=1300.0, b_min=-1100.0, b_max=1700.0,
                               threshold=2, phi_sectors=True),
                synth.GridSpec(2, 4, 3, 20000, threshold=2, phi_sectors=True)]  # atomic fill


@pytest.mark.parametrize("spec", SECTOR_GRIDS, ids=lambda s: "x".join(map(str, s.shape)))
def test_sector_events_bit_exact(gpu, spec):
    """Fused fill + peaks, the separate fills and ht_peaks, in sector mode."""
    import torch
    B = gpu
    for e in range(6):
        ev = synth.make_event(0, 700 + e)
        x, y, z = (ev.x, ev.y, ev.z) if spec.n_b < 10000 else (ev.x[:60], ev.y[:60], ev.z[:60])
        say("sector grid", spec.shape, "event", e)
        gM, gc, gv, gn = gpu_fused(B, spec, x, y, z)
        M, votes, oc, ov, on = oracle_run(spec, x, y, z)
        assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "event %d" % e)
        xd, yd, zd = B.hits_to_device(x, y, z)
        a1 = B.fill(spec, xd, yd, zd)
        a2 = B.fill(spec, xd, yd, zd, atomic=True)
        torch.cuda.synchronize()
        assert np.array_equal(B.as_u32(a1), M) and np.array_equal(B.as_u32(a2), M)
        c, v, n = B.peaks(spec, a1)
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)


def test_sector_hit_values_match_oracle(gpu):
    import torch
    from oracle import oracle
    B = gpu
    rng = np.random.default_rng(12)
    x, y, z = synth.uniform_hits(rng, 50000, 1000.0, 2500.0)
    for spec in (sector_grid(CFG0, 4), sector_grid(CFG0, 1), sector_grid(CFG4, 2)):
        say("sector hit values: grid", spec.shape)
        xd, yd, zd = B.hits_to_device(x, y, z)
        info, vals, slabs = B.ht_debug_hit_values(spec, xd, yd, zd)
        torch.cuda.synchronize()
        info, slabs = info.cpu().numpy(), slabs.cpu().numpy()
        o = oracle.hit_info(oracle.OracleGrid(*spec.as_tuple()), x, y, z)
        assert np.array_equal(info[:, 3], o["n_cells"])
        oslab = np.where(o["cells"][:, :, 0] >= 0, o["cells"][:, :, 0] * spec.n_phi + o["cells"][:, :, 1], -1)
        assert np.array_equal(slabs, oslab)


@pytest.mark.parametrize("shape,T", [((2, 4, 8, 8), 3), ((3, 1, 7, 9), 3), ((4, 4, 64, 64), 4),
                                     ((2, 2, 40, 130), 5)])
def test_sector_peaks_on_arbitrary_matrices(gpu, shape, T):
    import torch
    from oracle import oracle
    B = gpu
    say("sector peaks on a random matrix", shape)
    rng = np.random.default_rng(sum(shape) + 7 * T)
    M = rng.integers(0, 4, size=shape).astype(np.uint32)
    spikes = rng.random(shape) < 0.03
    M[spikes] += rng.integers(3, 12, size=int(spikes.sum())).astype(np.uint32)
    spec = synth.GridSpec(*shape, threshold=T, phi_sectors=True)
    acc = torch.from_numpy(M.view(np.int32).copy()).cuda()
    c, v, n = B.peaks(spec, acc)
    oc, ov, on = oracle.peaks(oracle.OracleGrid(*spec.as_tuple()), M)
    assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)


def test_sector_paper_grid_and_batch(gpu):
    """The paper's four sectors on the paper-shaped workload: single events and one batch."""
    B = gpu
    spec = sector_grid(CFG1, 4)
    hits = []
    for e in range(3):
        ev = synth.make_event(1, 30 + e)
        say("sector paper grid, event", e)
        gM, gc, gv, gn = gpu_fused(B, spec, ev.x, ev.y, ev.z)
        M, votes, oc, ov, on = oracle_run(spec, ev.x, ev.y, ev.z)
        assert_same(spec, gM, gc, gv, gn, M, oc, ov, on, "event %d" % e)
        hits.append((ev.x, ev.y, ev.z))
    say("sector paper grid, batch of 3")
    res = B.fill_peaks_batch(spec, hits, capacity=1 << 14)
    accs = B.as_u32(res.acc)
    for i, (x, y, z) in enumerate(hits):
        M, votes, oc, ov, on = oracle_run(spec, x, y, z)
        assert np.array_equal(accs[i], M), i
        c, v, n = res.peaks[i]
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), i


def test_batch_autotuner_keeps_results(gpu):
    from paper_1507_03074_amd import tune
    B = gpu
    evs = [synth.make_event(0, 900 + e) for e in range(12)]
    say("autotune a workload-0 batch")
    before = B.ht_get_tuning(CFG0).as_dict()
    rep = tune.autotune_batch(CFG0, [(e.x, e.y, e.z) for e in evs], reps=2, capacity=256)
    try:
        assert rep["best"] is not None and all(c["bit_exact"] for c in rep["candidates"])
        assert B.ht_get_tuning(CFG0).as_dict() == rep["best"]["tuning"]
        res = B.fill_peaks_batch(CFG0, [(e.x, e.y, e.z) for e in evs], capacity=256)
        accs = B.as_u32(res.acc)
        for i, e in enumerate(evs):
            M, votes, oc, ov, on = oracle_run(CFG0, e.x, e.y, e.z)
            assert np.array_equal(accs[i], M)
            c, v, n = res.peaks[i]
            assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)
    finally:
        B.ht_set_tuning(CFG0)
    assert B.ht_get_tuning(CFG0).as_dict() == before


def test_largest_grid_2pow32_cells(gpu):
    """The largest grid the layout allows: 8 x 32 x 4096 x 4096 = 2^32 cells (16 GiB of counts),
    whose last cell index is 2^32 - 1. Fill and peaks bit-exact against the oracle."""
    import torch
    B = gpu
    spec = synth.GridSpec(8, 32, 4096, 4096, threshold=6)
    assert spec.n_cells == 1 << 32
    rng = np.random.default_rng(2024)
    n_tracks = 150
    ev = synth.make_hits(rng, n_tracks, 200)
    say("2^32-cell grid:", ev.n, "hits")
    xd, yd, zd = B.hits_to_device(ev.x, ev.y, ev.z)
    acc, gc, gv, gn = B.fill_peaks(spec, xd, yd, zd, capacity=1 << 20)
    torch.cuda.synchronize()
    say("2^32-cell grid: copying the matrix to the host")
    gM = B.as_u32(acc)
    del acc
    torch.cuda.empty_cache()
    say("2^32-cell grid: oracle")
    M, votes, oc, ov, on = oracle_run(spec, ev.x, ev.y, ev.z)
    say("2^32-cell grid: comparing")
    assert int(gM.sum(dtype=np.int64)) == votes
    assert np.array_equal(gM, M)
    assert gn == on and np.array_equal(gc, oc) and np.array_equal(gv, ov)
    assert on > 0


def test_serve_sector_grid(gpu):
    """The request loop on the four-sector grid: each result equals the oracle's."""
    B = gpu
    spec = sector_grid(CFG0, 4)
    evs = [synth.make_event(0, 950 + e) for e in range(12)]
    opts = B.ServeOpts(1 << 30, 256, 2000, 4, 2, 64, 0)
    say("serve: 12 workload-0 events on four sectors")
    res = serve_all(B, spec, evs, opts)
    for ev, (c, v, n, tm) in zip(evs, res):
        M, votes, oc, ov, on = oracle_run(spec, ev.x, ev.y, ev.z)
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)


@pytest.mark.parametrize("rows,tpb,nt", [(1, 1, 0), (2, 4, 1), (4, 1, 2), (8, 4, 0), (16, 1, 1), (64, 1, 0)])
def test_long_slab_lists_bit_exact(gpu, rows, tpb, nt):
    """Events with about 1000 records per slab: the fill loads its records in chunks of eight
    per thread (the long-list variant, rows <= 8) or two (wider tiles)."""
    B = gpu
    x, y, z = random_hits(77, 22000)
    M, votes, oc, ov, on = oracle_run(CFG0, x, y, z)
    say("long lists: rows", rows, "tiles/block", tpb, "store", nt)
    B.ht_set_tuning(CFG0, rows=rows, tiles_per_block=tpb, nt_store=nt)
    try:
        gM, gc, gv, gn = gpu_fused(B, CFG0, x, y, z)
    finally:
        B.ht_set_tuning(CFG0)
    assert_same(CFG0, gM, gc, gv, gn, M, oc, ov, on, "rows %d" % rows)
