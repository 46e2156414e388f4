"""CPU oracle for the Hough-transform fill and peak search (ctypes wrapper over ht_oracle.c).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The GPU library never does, and this module imports nothing
from it. The arithmetic lives in ``ht_oracle.c`` (paper section 2: the vote along the circles
through the interaction point, then the local-maxima search above a threshold); this file only
compiles it with ``gcc -O2 -ffp-contract=off`` and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ht_oracle.c")
_LIB = os.path.join(_HERE, "libht_oracle.so")

# Strict IEEE binary32 evaluation: SSE2 floats on x86-64 (no x87 excess precision), no FMA
# contraction, no fast-math reassociation.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-fno-builtin"]


def build(force: bool = False) -> str:
    """Compile ht_oracle.c into libht_oracle.so next to it; returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("n_a", ctypes.c_int32), ("n_b", ctypes.c_int32),
                ("a_min", ctypes.c_float), ("a_max", ctypes.c_float),
                ("b_min", ctypes.c_float), ("b_max", ctypes.c_float),
                ("threshold", ctypes.c_uint32), ("phi_sectors", ctypes.c_int32)]


@dataclass(frozen=True)
class OracleGrid:
    n_theta: int
    n_phi: int
    n_a: int
    n_b: int
    a_min: float
    a_max: float
    b_min: float
    b_max: float
    threshold: int
    phi_sectors: int = 0  # 1: independent phi sectors (paper section 4)

    @property
    def shape(self):
        return (self.n_theta, self.n_phi, self.n_a, self.n_b)

    @property
    def n_cells(self) -> int:
        return self.n_theta * self.n_phi * self.n_a * self.n_b

    def _c(self) -> _Grid:
        return _Grid(self.n_theta, self.n_phi, self.n_a, self.n_b, self.a_min, self.a_max,
                     self.b_min, self.b_max, self.threshold, int(self.phi_sectors))


_lib = None


def _load(path: str | None = None):
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(path or build())
        P = ctypes.POINTER
        f32p, u32p, i32p = P(ctypes.c_float), P(ctypes.c_uint32), P(ctypes.c_int32)
        gp = P(_Grid)
        lib.oracle_check_grid.argtypes = [gp]
        lib.oracle_check_grid.restype = ctypes.c_int
        lib.oracle_tables.argtypes = [gp, f32p, f32p, f32p, f32p]
        lib.oracle_tables.restype = ctypes.c_int
        lib.oracle_hit_info.argtypes = [gp, f32p, f32p, f32p, ctypes.c_int64, i32p, f32p, i32p]
        lib.oracle_hit_info.restype = ctypes.c_int
        lib.oracle_fill.argtypes = [gp, f32p, f32p, f32p, ctypes.c_int64, u32p]
        lib.oracle_fill.restype = ctypes.c_int64
        lib.oracle_peaks.argtypes = [gp, u32p, u32p, u32p, ctypes.c_int64]
        lib.oracle_peaks.restype = ctypes.c_int64
        lib.oracle_readout.argtypes = [gp, u32p, ctypes.c_int64, P(ctypes.c_double)]
        lib.oracle_readout.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def check_grid(g: OracleGrid) -> bool:
    c = g._c()
    return _load().oracle_check_grid(ctypes.byref(c)) == 0


def tables(g: OracleGrid):
    """O0: (A2[n_a], invdB, Uphi[2 n_phi, 2], Utheta[2 n_theta + 1, 2]) as float32."""
    c = g._c()
    a2 = np.zeros(g.n_a, np.float32)
    inv = np.zeros(1, np.float32)
    uphi = np.zeros((2 * g.n_phi, 2), np.float32)
    uth = np.zeros((2 * g.n_theta + 1, 2), np.float32)
    rc = _load().oracle_tables(ctypes.byref(c), _ptr(a2, ctypes.c_float), _ptr(inv, ctypes.c_float),
                               _ptr(uphi, ctypes.c_float), _ptr(uth, ctypes.c_float))
    if rc != 0:
        raise ValueError("invalid grid")
    return a2, inv[0], uphi, uth


def hit_info(g: OracleGrid, x, y, z):
    """O1-O3 per hit: dict of valid, s_theta, s_phi, n_cells, r2, r, k, cells[n, 4, 2]."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.size
    info = np.zeros((n, 4), np.int32)
    vals = np.zeros((n, 3), np.float32)
    cells = np.zeros((n, 4, 2), np.int32)
    c = g._c()
    rc = _load().oracle_hit_info(ctypes.byref(c), _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                                 _ptr(z, ctypes.c_float), n, _ptr(info, ctypes.c_int32),
                                 _ptr(vals, ctypes.c_float), _ptr(cells, ctypes.c_int32))
    if rc != 0:
        raise ValueError("invalid grid")
    return dict(valid=info[:, 0].astype(bool), s_theta=info[:, 1], s_phi=info[:, 2],
                n_cells=info[:, 3], r2=vals[:, 0], r=vals[:, 1], k=vals[:, 2], cells=cells)


def fill(g: OracleGrid, x, y, z, out: np.ndarray | None = None):
    """O1-O5: returns (M as uint32 [n_theta, n_phi, n_a, n_b], number of votes)."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    if not (x.size == y.size == z.size):
        raise ValueError("x, y, z must have the same length")
    if out is None:
        out = np.empty(g.shape, np.uint32)
    assert out.dtype == np.uint32 and out.flags.c_contiguous and out.size == g.n_cells
    c = g._c()
    votes = _load().oracle_fill(ctypes.byref(c), _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                                _ptr(z, ctypes.c_float), x.size, _ptr(out, ctypes.c_uint32))
    if votes < 0:
        raise ValueError("invalid grid")
    return out.reshape(g.shape), int(votes)


def peaks(g: OracleGrid, M: np.ndarray, capacity: int | None = None):
    """O6: returns (cells uint32[k], votes uint32[k], total found); k = min(found, capacity)."""
    M = np.ascontiguousarray(M, dtype=np.uint32)
    assert M.size == g.n_cells
    c = g._c()
    lib = _load()
    if capacity is None:
        n = lib.oracle_peaks(ctypes.byref(c), _ptr(M, ctypes.c_uint32), None, None, 0)
        if n < 0:
            raise ValueError("invalid grid")
        capacity = int(n)
    cells = np.zeros(max(capacity, 1), np.uint32)
    votes = np.zeros(max(capacity, 1), np.uint32)
    n = lib.oracle_peaks(ctypes.byref(c), _ptr(M, ctypes.c_uint32), _ptr(cells, ctypes.c_uint32),
                         _ptr(votes, ctypes.c_uint32), capacity)
    if n < 0:
        raise ValueError("invalid grid")
    k = min(int(n), capacity)
    return cells[:k].copy(), votes[:k].copy(), int(n)


def readout(g: OracleGrid, cells):
    """Track parameters of peak cells: dict of t, p, a, b (int64) and A, B, rho, phi, theta."""
    cells = np.ascontiguousarray(cells, dtype=np.uint32)
    out = np.zeros((cells.size, 9), np.float64)
    c = g._c()
    rc = _load().oracle_readout(ctypes.byref(c), _ptr(cells, ctypes.c_uint32), cells.size,
                                _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("invalid grid")
    keys = ("t", "p", "a", "b", "A", "B", "rho", "phi", "theta")
    d = {k: out[:, i] for i, k in enumerate(keys)}
    for k in ("t", "p", "a", "b"):
        d[k] = d[k].astype(np.int64)
    return d
