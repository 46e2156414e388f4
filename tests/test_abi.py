"""C-ABI contract checks that need no GPU: the library loads, exports every declared symbol,
computes the bin-rule tables bit-identically to the oracle, and rejects bad arguments on the host
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1507_03074_amd import binding as B
from paper_1507_03074_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1507_03074_amd import build as hbuild
    hbuild.ensure_built()  # a missing or stale library is rebuilt, never tested
    return B.lib()


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(ht_\w+)\s*\(", text, re.M))
    return names


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"ht_fill", "ht_peaks", "ht_fill_peaks_batch", "ht_serve_submit", "ht_serve_poll"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(B.EXPORTS) == names


GRIDS = [synth.WORKLOADS[0].grid, synth.WORKLOADS[1].grid, synth.WORKLOADS[4].grid,
         synth.GridSpec(3, 5, 7, 9, a_min=-1500.0, a_max=1300.0, b_min=-1100.0, b_max=1700.0,
                        threshold=2),
         synth.GridSpec(2, 7, 100, 37, a_min=-999.0, a_max=1234.5, b_min=-3.0, b_max=7.25)]


@pytest.mark.parametrize("spec", GRIDS)
def test_tables_bit_identical_to_oracle(lib, spec):
    from oracle import oracle
    a2, inv, phi, th = B.ht_tables(spec)
    oa2, oinv, ophi, oth = oracle.tables(oracle.OracleGrid(*spec.as_tuple()))
    assert a2.tobytes() == oa2.tobytes()
    assert np.float32(inv).tobytes() == np.float32(oinv).tobytes()
    assert phi.tobytes() == ophi.tobytes()
    assert th.tobytes() == oth.tobytes()


def test_invalid_grid_rejected_on_host(lib):
    bad = synth.GridSpec(4, 2, 64, 64)
    g = B.make_grid(bad)
    dummy = ctypes.c_void_p(256)   # never dereferenced: validation fails first
    rc = lib.ht_fill(ctypes.byref(g), None, None, None, 0, dummy, None)
    assert rc == B.HT_EINVAL and "n_phi" in B.last_error()
    rc = lib.ht_peaks(ctypes.byref(g), dummy, None, 0, dummy, None)
    assert rc == B.HT_EINVAL and "n_phi" in B.last_error()
    for spec in [synth.GridSpec(64, 64, 4096, 4096), synth.GridSpec(4, 16, 64, 64, threshold=0),
                 synth.GridSpec(4, 16, 64, 64, a_min=5.0, a_max=5.0),
                 synth.GridSpec(200, 100, 8, 8)]:
        g = B.make_grid(spec)
        assert lib.ht_fill(ctypes.byref(g), None, None, None, 0, dummy, None) == B.HT_EINVAL
        assert "grid" in B.last_error() or "cells" in B.last_error() or "threshold" in B.last_error() \
            or "n_theta" in B.last_error()


def test_bad_arguments_rejected_on_host(lib):
    g = B.make_grid(synth.WORKLOADS[0].grid)
    # negative hit count, missing matrix, missing hit arrays
    assert lib.ht_fill(ctypes.byref(g), None, None, None, -1, ctypes.c_void_p(16), None) == B.HT_EINVAL
    assert lib.ht_fill(ctypes.byref(g), None, None, None, 0, None, None) == B.HT_EINVAL
    assert lib.ht_fill(ctypes.byref(g), None, None, None, 5, ctypes.c_void_p(16), None) == B.HT_EINVAL
    # peaks: capacity > 0 without an output array, or no n_found
    assert lib.ht_peaks(ctypes.byref(g), ctypes.c_void_p(16), None, 4, ctypes.c_void_p(16), None) == B.HT_EINVAL
    assert lib.ht_peaks(ctypes.byref(g), ctypes.c_void_p(16), None, 0, None, None) == B.HT_EINVAL
    ev = (B.Event * 1)(B.Event(0, -3, 0, 0))
    assert lib.ht_fill_peaks_batch(ctypes.byref(g), ev, 1, None, None, None, ctypes.c_void_p(16),
                                   None, ctypes.c_void_p(16), None) == B.HT_EINVAL
    assert lib.ht_fill_peaks_batch(ctypes.byref(g), ev, -1, None, None, None, None, None, None,
                                   None) == B.HT_EINVAL


def test_serve_options_validated_on_host(lib):
    g = B.make_grid(synth.WORKLOADS[0].grid)
    srv = ctypes.c_void_p()
    for opts in [B.ServeOpts(0, 16, 100, 4, 2, 8, 0), B.ServeOpts(1 << 30, 0, 100, 4, 2, 8, 0),
                 B.ServeOpts(1 << 30, 16, 100, 0, 2, 8, 0), B.ServeOpts(1 << 30, 16, 100, 4, 0, 8, 0),
                 B.ServeOpts(1 << 30, 16, 100, 4, 2, 0, 0)]:
        assert lib.ht_serve_create(ctypes.byref(g), ctypes.byref(opts), ctypes.byref(srv)) == B.HT_EINVAL
        assert not srv.value
    assert lib.ht_serve_destroy(None) == B.HT_OK
    t = ctypes.c_uint64()
    assert lib.ht_serve_submit(None, None, None, None, 0, ctypes.byref(t)) == B.HT_EINVAL


def test_tiling_covers_the_matrix(lib):
    for spec in GRIDS:
        t = B.ht_tiling(spec)
        rows = t["rows"]
        assert rows >= 1 and rows & (rows - 1) == 0 and rows <= 64
        tiles_per_slab = -(-spec.n_a // rows)
        assert t["n_tiles"] == spec.n_theta * spec.n_phi * tiles_per_slab
        assert t["cand_cap"] & (t["cand_cap"] - 1) == 0
        if t["lds_fill"]:
            assert rows * spec.n_b * 4 <= 65536


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libht.so")
    with pytest.raises(B.HTError):
        B.lib()


def test_tuning_validated_and_applied_on_host(lib):
    spec = synth.GridSpec(4, 16, 1024, 1024, threshold=9)
    default = B.ht_get_tuning(spec).as_dict()
    assert default["rows"] == B.ht_tiling(spec)["rows"]
    for bad in [dict(rows=3), dict(rows=128), dict(rows=32),  # 32 x 1024 x 4 B exceeds the LDS tile
                dict(group_tiles=8), dict(cand_cap=3), dict(cand_cap=8192), dict(nt_store=3),
                dict(tiles_per_block=3), dict(tiles_per_block=128), dict(tiles_per_block=-1),
                dict(dense_hits=-2)]:
        with pytest.raises(B.HTError):
            B.ht_set_tuning(spec, **bad)
        assert B.ht_get_tuning(spec).as_dict() == default
    assert default["tiles_per_block"] >= 1 and default["nt_store"] in (0, 1, 2)
    assert default["dense_hits"] == 4 * 16 * 1024 // 4
    B.ht_set_tuning(spec, rows=4, group_tiles=32, cand_cap=128, nt_store=2, tiles_per_block=16,
                    dense_hits=20000)
    try:
        got = B.ht_get_tuning(spec).as_dict()
        assert got == {"rows": 4, "group_tiles": 32, "cand_cap": 128, "nt_store": 2,
                       "tiles_per_block": 16, "dense_hits": 20000}
        # the threshold is not part of the key
        other = synth.GridSpec(4, 16, 1024, 1024, threshold=3)
        assert B.ht_get_tuning(other).as_dict() == got
        assert B.ht_tiling(spec)["n_tiles"] == 64 * 256
        # unspecified fields keep their defaults
        B.ht_set_tuning(spec, rows=2)
        got = B.ht_get_tuning(spec).as_dict()
        assert got["rows"] == 2 and got["group_tiles"] == default["group_tiles"]
        assert got["dense_hits"] == default["dense_hits"]
        B.ht_set_tuning(spec, dense_hits=-1)
        assert B.ht_get_tuning(spec).dense_hits == -1
    finally:
        B.ht_set_tuning(spec)
    assert B.ht_get_tuning(spec).as_dict() == default


def test_profile_modes_validated_on_host(lib):
    for mode in (1, 2, 0):
        assert lib.ht_profile_enable(mode) == 0
    for mode in (-1, 3):
        assert lib.ht_profile_enable(mode) == B.HT_EINVAL
    assert lib.ht_profile_enable(0) == 0


def test_debug_unary_validated_on_host(lib):
    """Checked before any device work: a negative size or a NULL array is HT_EINVAL; an empty
    call does nothing."""
    dummy = ctypes.c_void_p(256)
    assert lib.ht_debug_unary(dummy, dummy, dummy, -1, None) == B.HT_EINVAL
    assert lib.ht_debug_unary(None, None, None, 0, None) == 0
    assert lib.ht_debug_unary(None, dummy, dummy, 4, None) == B.HT_EINVAL
    assert lib.ht_debug_unary(dummy, dummy, None, 4, None) == B.HT_EINVAL


def test_sector_grids_validated_on_host(lib):
    """phi_sectors is 0 or 1; with sectors n_phi may be 1 or 2; the tables do not depend on it."""
    from oracle import oracle
    dummy = ctypes.c_void_p(256)
    g = B.make_grid(synth.GridSpec(4, 4, 64, 64, phi_sectors=True))
    g.phi_sectors = 2
    assert lib.ht_fill(ctypes.byref(g), None, None, None, 0, dummy, None) == B.HT_EINVAL
    assert "phi_sectors" in B.last_error()
    for n_phi in (1, 2, 4):
        spec = synth.GridSpec(3, n_phi, 16, 8, threshold=2, phi_sectors=True)
        a2, inv, uphi, uth = B.ht_tables(spec)
        oa2, oinv, ouphi, outh = oracle.tables(oracle.OracleGrid(*spec.as_tuple()))
        assert a2.tobytes() == oa2.tobytes() and uphi.tobytes() == ouphi.tobytes()
        assert B.ht_tiling(spec)["n_tiles"] >= 3 * n_phi


def test_batch_plan_on_host(lib, monkeypatch):
    """The slab-list layout of a batch, decided on the host before any device work: direct lists
    for the 100-event batch of up to 8000 hits on the paper grid, the counting sort for the
    16-event batch of 105600-hit events on the 8x32x2048x2048 grid (direct lists would need about
    0.73 GB per event, past 8 GiB in all), and the counting sort everywhere under
    HT_PACKED_LISTS=1."""
    cfg1, cfg4 = synth.WORKLOADS[1].grid, synth.WORKLOADS[4].grid
    direct, scratch = B.ht_debug_batch_plan(cfg1, [1000 + 70 * i for i in range(100)])
    assert direct and scratch > 0
    direct, scratch = B.ht_debug_batch_plan(cfg4, [105600] * 16)
    assert not direct
    one_direct, one_bytes = B.ht_debug_batch_plan(cfg4, [105600])
    assert one_direct and 16 * one_bytes > 8 << 30
    monkeypatch.setenv("HT_PACKED_LISTS", "1")
    assert B.ht_debug_batch_plan(cfg1, [5000])[0] is False
    monkeypatch.delenv("HT_PACKED_LISTS")
    assert B.ht_debug_batch_plan(cfg1, [5000])[0] is True
    # validation
    g = B.make_grid(cfg1)
    d, b = ctypes.c_int32(), ctypes.c_int64()
    ev = (B.Event * 1)(B.Event(0, -1, 0, 0))
    assert lib.ht_debug_batch_plan(ctypes.byref(g), ev, 1, ctypes.byref(d), ctypes.byref(b)) == B.HT_EINVAL
    assert lib.ht_debug_batch_plan(ctypes.byref(g), ev, 0, ctypes.byref(d), ctypes.byref(b)) == B.HT_EINVAL
