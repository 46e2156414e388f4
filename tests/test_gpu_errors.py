"""Error paths and limits on the GPU, through the C ABI: launches that fail part way (forced from
the host with HT_TEST_FAIL_STAGE, so every kernel that does run exits normally) must leave the
library's counters usable, the request loop's refusals and overflow reports, and grids whose B
rows are too wide for an LDS tile. Every result that follows a failure is checked against the
CPU oracle, bit for bit.
"""
import ctypes
import os
import sys
import time

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
    return B


@pytest.fixture()
def env_keys():
    keys = ("HT_TEST_FAIL_STAGE", "HT_BATCH_GRAPH", "HT_PACKED_LISTS")
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
    M, _ = oracle.fill(g, x, y, z)
    cells, vv, n = oracle.peaks(g, M)
    return M, cells, vv, n


def check_event(B, spec, ev, tag):
    import torch
    x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
    acc, c, v, n = B.fill_peaks(spec, x, y, z, capacity=1 << 16)
    torch.cuda.synchronize()
    M, oc, ov, on = oracle_run(spec, ev.x, ev.y, ev.z)
    assert np.array_equal(B.as_u32(acc), M), tag
    assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), tag


def check_batch(B, spec, evs, tag):
    res = B.fill_peaks_batch(spec, [(e.x, e.y, e.z) for e in evs], capacity=1 << 14)
    acc = B.as_u32(res.acc)
    for i, e in enumerate(evs):
        M, oc, ov, on = oracle_run(spec, e.x, e.y, e.z)
        c, v, n = res.peaks[i]
        assert np.array_equal(acc[i], M), (tag, i)
        assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov), (tag, i)


@pytest.mark.parametrize("packed", [False, True], ids=["direct", "packed"])
def test_failed_single_event_launch_leaves_counters_usable(gpu, env_keys, packed):
    import torch
    B = gpu
    if packed:
        os.environ["HT_PACKED_LISTS"] = "1"
    seed = 40
    for stage in ("prep", "fill", "peaks", "prep"):
        ev = synth.make_event(0, seed)
        say("single event: %s launch fails (%s lists)" % (stage, "packed" if packed else "direct"))
        os.environ["HT_TEST_FAIL_STAGE"] = stage
        x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
        acc = B.new_acc(CFG0)
        out, nf = B.new_peaks(1024)
        with pytest.raises(B.HTError) as ex:
            B.ht_fill_peaks(CFG0, x, y, z, acc, out, 1024, nf)
        assert ex.value.code == B.HT_EDEVICE and "injected" in str(ex.value)
        torch.cuda.synchronize()
        os.environ.pop("HT_TEST_FAIL_STAGE")
        check_event(B, CFG0, synth.make_event(0, seed + 1), "after a failed %s launch" % stage)
        seed += 2


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
def test_failed_batch_launch_leaves_counters_usable(gpu, env_keys, graph):
    import torch
    B = gpu
    os.environ["HT_BATCH_GRAPH"] = "1" if graph else "0"
    for k, stage in enumerate(("prep", "fill", "peaks")):
        # a batch size not seen before: its graph is captured afresh (a cached graph is replayed
        # without going through the launches, so no failure could be injected into it)
        evs = [synth.make_event(0, 60 + i) for i in range(5 + k)]
        say("batch (%s): %s launch fails" % ("graph" if graph else "eager", stage))
        os.environ["HT_TEST_FAIL_STAGE"] = stage
        with pytest.raises(B.HTError) as ex:
            B.fill_peaks_batch(CFG0, [(e.x, e.y, e.z) for e in evs], capacity=1 << 14)
        assert ex.value.code == B.HT_EDEVICE
        torch.cuda.synchronize()
        os.environ.pop("HT_TEST_FAIL_STAGE")
        check_batch(B, CFG0, evs, "batch after a failed %s launch" % stage)


def test_wide_rows_candidate_scan_and_fill(gpu):
    """B rows of 65536 cells (256 KiB, more than an LDS tile or a workgroup's LDS): the fill takes
    global atomics and the candidate scan reads the rows from the matrix."""
    import torch
    from oracle import oracle
    B = gpu
    spec = synth.GridSpec(1, 3, 8, 65536, threshold=2)
    assert B.ht_tiling(spec)["lds_fill"] == 0
    say("wide rows: peaks of a random 1x3x8x65536 matrix")
    rng = np.random.default_rng(5)
    M = rng.integers(0, 3, size=spec.shape).astype(np.uint32)
    spikes = rng.random(spec.shape) < 0.01
    M[spikes] += rng.integers(2, 9, size=int(spikes.sum())).astype(np.uint32)
    acc = torch.from_numpy(M.view(np.int32).copy()).cuda()
    c, v, n = B.peaks(spec, acc, capacity=1 << 17)
    oc, ov, on = oracle.peaks(oracle.OracleGrid(*spec.as_tuple()), M)
    assert n == on and n > 1000 and np.array_equal(c, oc) and np.array_equal(v, ov)
    for seed in range(2):
        say("wide rows: fill and peaks, seed", seed)
        x, y, z = synth.uniform_hits(np.random.default_rng(seed), 200, 1000.0, 2500.0)
        ev = synth.Event(x, y, z)
        check_event(B, spec, ev, "wide rows seed %d" % seed)


# ---------------------------------------------------------------------------------------------
# Request loop
# ---------------------------------------------------------------------------------------------
def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _create(B, spec, opts):
    srv = ctypes.c_void_p()
    g = B.make_grid(spec)
    B.check(B.lib().ht_serve_create(ctypes.byref(g), ctypes.byref(opts), ctypes.byref(srv)))
    return srv


def _submit(B, srv, ev):
    t = ctypes.c_uint64()
    rc = B.lib().ht_serve_submit(srv, _fp(ev.x), _fp(ev.y), _fp(ev.z), ev.n, ctypes.byref(t))
    return rc, t.value


def _wait(B, srv, ticket, cap, timeout=60.0):
    out = (B.Peak * max(cap, 1))()
    nf = ctypes.c_int64()
    deadline = time.time() + timeout
    while time.time() < deadline:
        rc = B.lib().ht_serve_poll(srv, ticket, out, cap, ctypes.byref(nf), None)
        if rc != B.HT_EAGAIN:
            k = min(nf.value, cap)
            arr = np.frombuffer(out, dtype=np.uint32).reshape(-1, 2)[:k]
            return rc, arr[:, 0].copy(), arr[:, 1].copy(), nf.value
        time.sleep(1e-4)
    raise AssertionError("ticket %d did not finish" % ticket)


def test_serve_submit_flood_returns_eagain_then_drains(gpu):
    B = gpu
    evs = [synth.make_event(3, e) for e in range(4)]
    depth = 3
    opts = B.ServeOpts(2 << 30, 1 << 17, 40000, 1, 1, depth, 0)
    srv = _create(B, CFG1, opts)
    try:
        say("serve flood: queue_depth %d, events of %s hits" % (depth, [e.n for e in evs]))
        accepted, refused = [], 0
        for i in range(400):
            rc, t = _submit(B, srv, evs[i % len(evs)])
            if rc == B.HT_EAGAIN:
                refused += 1
                break
            B.check(rc)
            accepted.append((t, i % len(evs)))
        assert refused == 1, "the queue never filled"
        assert len(accepted) >= depth
        say("serve flood: %d accepted before HT_EAGAIN; draining" % len(accepted))
        expect = {}
        for t, k in accepted:
            rc, c, v, n = _wait(B, srv, t, 1 << 17)
            assert rc == B.HT_OK
            if k not in expect:
                e = evs[k]
                expect[k] = oracle_run(CFG1, e.x, e.y, e.z)[1:]
            oc, ov, on = expect[k]
            assert n == on and np.array_equal(c, oc) and np.array_equal(v, ov)
        # drained: submissions are accepted again
        rc, t = _submit(B, srv, evs[0])
        assert rc == B.HT_OK
        rc, c, v, n = _wait(B, srv, t, 1 << 17)
        assert rc == B.HT_OK and n == expect[0][2]
    finally:
        assert B.lib().ht_serve_destroy(srv) == B.HT_OK


def test_serve_destroy_with_requests_in_flight(gpu):
    B = gpu
    evs = [synth.make_event(3, e) for e in range(6)]
    opts = B.ServeOpts(2 << 30, 1 << 17, 40000, 2, 2, 16, 0)
    say("serve: destroy with %d requests submitted and none polled" % len(evs))
    srv = _create(B, CFG1, opts)
    for e in evs:
        rc, _ = _submit(B, srv, e)
        assert rc == B.HT_OK
    assert B.lib().ht_serve_destroy(srv) == B.HT_OK
    assert B.lib().ht_serve_destroy(None) == B.HT_OK
    # the library and the device are still fine: a new server serves an event exactly
    srv = _create(B, CFG0, B.ServeOpts(64 << 20, 256, 2000, 4, 1, 8, 0))
    try:
        e = synth.make_event(0, 77)
        rc, t = _submit(B, srv, e)
        assert rc == B.HT_OK
        rc, c, v, n = _wait(B, srv, t, 256)
        _, oc, ov, on = oracle_run(CFG0, e.x, e.y, e.z)
        assert rc == B.HT_OK and n == on and np.array_equal(c, oc) and np.array_equal(v, ov)
    finally:
        B.lib().ht_serve_destroy(srv)


def test_serve_poll_reports_overflow_with_the_first_peaks(gpu):
    B = gpu
    e = synth.make_event(1, 3)
    _, oc, ov, on = oracle_run(CFG1, e.x, e.y, e.z)
    assert on > 64
    # the server's own capacity is too small: HT_EOVERFLOW, the total and its first 8 peaks
    say("serve overflow: server capacity 8, %d peaks" % on)
    srv = _create(B, CFG1, B.ServeOpts(1 << 30, 8, 5000, 1, 1, 4, 0))
    try:
        rc, t = _submit(B, srv, e)
        assert rc == B.HT_OK
        rc, c, v, n = _wait(B, srv, t, 8)
        assert rc == B.HT_EOVERFLOW and n == on
        assert np.array_equal(c, oc[:8]) and np.array_equal(v, ov[:8])
        # the ticket is released even so
        nf = ctypes.c_int64()
        assert B.lib().ht_serve_poll(srv, t, None, 0, ctypes.byref(nf), None) == B.HT_EINVAL
    finally:
        B.lib().ht_serve_destroy(srv)
    # the caller's capacity is the smaller one
    say("serve overflow: caller capacity 5")
    srv = _create(B, CFG1, B.ServeOpts(1 << 30, 4096, 5000, 1, 1, 4, 0))
    try:
        rc, t = _submit(B, srv, e)
        assert rc == B.HT_OK
        rc, c, v, n = _wait(B, srv, t, 5)
        assert rc == B.HT_EOVERFLOW and n == on
        assert np.array_equal(c, oc[:5]) and np.array_equal(v, ov[:5])
    finally:
        B.lib().ht_serve_destroy(srv)
