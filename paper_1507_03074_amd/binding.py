"""ctypes binding of libht.so (include/ht.h, include/ht_debug.h).

Argument marshalling only: every step of the fill and the peak search runs in the library's HIP
kernels. PyTorch supplies device memory (tensors) and the current HIP stream. There is no CPU
fallback: if libht.so is missing, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libht.so")

HT_OK, HT_EINVAL, HT_ENOMEM, HT_EOVERFLOW, HT_EAGAIN, HT_EDEVICE = 0, -1, -2, -3, -4, -5
_NAMES = {0: "HT_OK", -1: "HT_EINVAL", -2: "HT_ENOMEM", -3: "HT_EOVERFLOW", -4: "HT_EAGAIN",
          -5: "HT_EDEVICE"}


class HTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("n_a", ctypes.c_int32), ("n_b", ctypes.c_int32),
                ("a_min", ctypes.c_float), ("a_max", ctypes.c_float),
                ("b_min", ctypes.c_float), ("b_max", ctypes.c_float),
                ("threshold", ctypes.c_uint32), ("phi_sectors", ctypes.c_int32)]

    @property
    def shape(self):
        return (self.n_theta, self.n_phi, self.n_a, self.n_b)

    @property
    def n_cells(self) -> int:
        return self.n_theta * self.n_phi * self.n_a * self.n_b


class Peak(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_uint32), ("votes", ctypes.c_uint32)]


class Track(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_uint32), ("votes", ctypes.c_uint32), ("t", ctypes.c_int32),
                ("p", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("A", ctypes.c_float), ("B", ctypes.c_float), ("rho", ctypes.c_float),
                ("phi", ctypes.c_float), ("theta", ctypes.c_float)]


TRACK_DTYPE = np.dtype([("cell", "<u4"), ("votes", "<u4"), ("t", "<i4"), ("p", "<i4"),
                        ("a", "<i4"), ("b", "<i4"), ("A", "<f4"), ("B", "<f4"), ("rho", "<f4"),
                        ("phi", "<f4"), ("theta", "<f4")])


class Event(ctypes.Structure):
    _fields_ = [("hit_offset", ctypes.c_int64), ("n_hits", ctypes.c_int64),
                ("peak_offset", ctypes.c_int64), ("peak_capacity", ctypes.c_int64)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("peak_capacity", ctypes.c_int64),
                ("max_hits", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("queue_depth", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("group_tiles", ctypes.c_int32),
                ("cand_cap", ctypes.c_int32), ("nt_store", ctypes.c_int32),
                ("tiles_per_block", ctypes.c_int32), ("dense_hits", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


#: every symbol the public headers declare
EXPORTS = ["ht_set_tuning", "ht_get_tuning", "ht_tables", "ht_fill", "ht_peaks", "ht_fill_peaks", "ht_fill_peaks_batch",
           "ht_fill_peaks_noalloc",
           "ht_serve_create", "ht_serve_submit", "ht_serve_poll", "ht_serve_destroy",
           "ht_last_error", "ht_debug_hit_values", "ht_debug_unary", "ht_fill_atomic", "ht_tiling",
           "ht_profile_enable", "ht_profile_read", "ht_bench_hbm_write", "ht_bench_hbm_read",
           "ht_bench_copy", "ht_bench_atomic_rand", "ht_bench_lds_atomic", "ht_readout",
           "ht_debug_pointer_kind", "ht_debug_batch_plan"]

_lib = None


def lib():
    """Load libht.so (raises HTError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HTError(HT_EDEVICE, "libht.so is not built (run __graft_entry__.build() or "
                                  "python -m paper_1507_03074_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    gp = ctypes.POINTER(Grid)
    f32p = ctypes.POINTER(ctypes.c_float)
    sig = {
        "ht_tables": ([gp, f32p, f32p, f32p, f32p], ctypes.c_int),
        "ht_set_tuning": ([gp, ctypes.POINTER(Tuning)], ctypes.c_int),
        "ht_get_tuning": ([gp, ctypes.POINTER(Tuning)], ctypes.c_int),
        "ht_tiling": ([gp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                       ctypes.POINTER(i32)], ctypes.c_int),
        "ht_fill": ([gp, vp, vp, vp, i64, vp, vp], ctypes.c_int),
        "ht_fill_atomic": ([gp, vp, vp, vp, i64, vp, vp], ctypes.c_int),
        "ht_peaks": ([gp, vp, vp, i64, vp, vp], ctypes.c_int),
        "ht_fill_peaks": ([gp, vp, vp, vp, i64, vp, vp, i64, vp, vp], ctypes.c_int),
        "ht_fill_peaks_noalloc": ([gp, vp, vp, vp, i64, vp, vp, i64, vp, vp], ctypes.c_int),
        "ht_fill_peaks_batch": ([gp, ctypes.POINTER(Event), i32, vp, vp, vp, vp, vp, vp, vp],
                                ctypes.c_int),
        "ht_debug_hit_values": ([gp, vp, vp, vp, i64, vp, vp, vp, vp], ctypes.c_int),
        "ht_debug_unary": ([vp, vp, vp, i64, vp], ctypes.c_int),
        "ht_readout": ([gp, vp, vp, i64, vp, vp], ctypes.c_int),
        "ht_debug_pointer_kind": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "ht_debug_batch_plan": ([gp, ctypes.POINTER(Event), i32, ctypes.POINTER(i32),
                                 ctypes.POINTER(i64)], ctypes.c_int),
        "ht_serve_create": ([gp, ctypes.POINTER(ServeOpts), ctypes.POINTER(vp)], ctypes.c_int),
        "ht_serve_submit": ([vp, f32p, f32p, f32p, i64, ctypes.POINTER(ctypes.c_uint64)],
                            ctypes.c_int),
        "ht_serve_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(Peak), i64,
                           ctypes.POINTER(i64), ctypes.POINTER(Timing)], ctypes.c_int),
        "ht_serve_destroy": ([vp], ctypes.c_int),
        "ht_last_error": ([], ctypes.c_char_p),
        "ht_profile_enable": ([ctypes.c_int], ctypes.c_int),
        "ht_profile_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                             ctypes.c_int], ctypes.c_int),
        "ht_bench_hbm_write": ([vp, i64, i32, vp], ctypes.c_int),
        "ht_bench_hbm_read": ([vp, i64, vp, vp], ctypes.c_int),
        "ht_bench_copy": ([vp, vp, i64, vp], ctypes.c_int),
        "ht_bench_atomic_rand": ([vp, i64, i64, vp], ctypes.c_int),
        "ht_bench_lds_atomic": ([i32, i32, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def last_error() -> str:
    return lib().ht_last_error().decode()


def check(rc: int):
    if rc != HT_OK:
        raise HTError(rc, last_error())
    return rc


def make_grid(spec) -> Grid:
    """Grid from a synth.GridSpec, a (n_theta, n_phi, n_a, n_b, a_min, a_max, b_min, b_max,
    threshold[, phi_sectors]) tuple, or a Grid."""
    if isinstance(spec, Grid):
        return spec
    t = spec.as_tuple() if hasattr(spec, "as_tuple") else tuple(spec)
    return Grid(*t)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise HTError(HT_EINVAL, "tensor arguments must live on the GPU")
        if t is not None and not t.is_contiguous():
            raise HTError(HT_EINVAL, "tensor arguments must be contiguous")


def _need_out(*ts):
    """Peak outputs: GPU tensors, or pinned host tensors (written directly by the kernels)."""
    for t in ts:
        if t is not None and not (t.is_cuda or t.is_pinned()):
            raise HTError(HT_EINVAL, "output tensors must live on the GPU or in pinned host memory")
        if t is not None and not t.is_contiguous():
            raise HTError(HT_EINVAL, "tensor arguments must be contiguous")


# ---------------------------------------------------------------------------------------------
# Entry points (same names as the C ABI), tensors in, status out
# ---------------------------------------------------------------------------------------------
def ht_tables(spec):
    g = make_grid(spec)
    a2 = np.zeros(g.n_a, np.float32)
    inv = np.zeros(1, np.float32)
    phi = np.zeros((2 * g.n_phi, 2), np.float32)
    th = np.zeros((2 * g.n_theta + 1, 2), np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    check(lib().ht_tables(ctypes.byref(g), a2.ctypes.data_as(fp), inv.ctypes.data_as(fp),
                          phi.ctypes.data_as(fp), th.ctypes.data_as(fp)))
    return a2, inv[0], phi, th


def ht_set_tuning(spec, tuning=None, **fields):
    """Set the launch shape for a grid (a Tuning, or fields rows/group_tiles/cand_cap/nt_store/
    tiles_per_block/dense_hits; unspecified fields keep the default). ht_set_tuning(spec)
    restores the defaults."""
    g = make_grid(spec)
    if tuning is None and not fields:
        return check(lib().ht_set_tuning(ctypes.byref(g), None))
    if tuning is None:
        unknown = set(fields) - {"rows", "group_tiles", "cand_cap", "nt_store", "tiles_per_block",
                                 "dense_hits"}
        if unknown:
            raise TypeError("unknown tuning fields: %s" % sorted(unknown))
        tuning = Tuning(fields.get("rows", 0), fields.get("group_tiles", 0),
                        fields.get("cand_cap", 0), fields.get("nt_store", -1),
                        fields.get("tiles_per_block", 0), fields.get("dense_hits", 0))
    return check(lib().ht_set_tuning(ctypes.byref(g), ctypes.byref(tuning)))


def ht_get_tuning(spec) -> Tuning:
    g = make_grid(spec)
    t = Tuning()
    check(lib().ht_get_tuning(ctypes.byref(g), ctypes.byref(t)))
    return t


def ht_tiling(spec):
    g = make_grid(spec)
    vals = [ctypes.c_int32() for _ in range(4)]
    check(lib().ht_tiling(ctypes.byref(g), *[ctypes.byref(v) for v in vals]))
    return dict(rows=vals[0].value, n_tiles=vals[1].value, cand_cap=vals[2].value,
                lds_fill=vals[3].value)


def ht_fill(spec, x, y, z, acc, stream=None, atomic=False):
    g = make_grid(spec)
    _need_cuda(x, y, z, acc)
    fn = lib().ht_fill_atomic if atomic else lib().ht_fill
    return check(fn(ctypes.byref(g), _ptr(x), _ptr(y), _ptr(z), x.numel(), _ptr(acc),
                    _stream(stream)))


def ht_peaks(spec, acc, out, capacity, n_found, stream=None):
    g = make_grid(spec)
    _need_cuda(acc)
    _need_out(out, n_found)
    return check(lib().ht_peaks(ctypes.byref(g), _ptr(acc), _ptr(out), capacity, _ptr(n_found),
                                _stream(stream)))


def ht_fill_peaks(spec, x, y, z, acc, out, capacity, n_found, stream=None):
    g = make_grid(spec)
    _need_cuda(x, y, z, acc)
    _need_out(out, n_found)
    return check(lib().ht_fill_peaks(ctypes.byref(g), _ptr(x), _ptr(y), _ptr(z), x.numel(),
                                     _ptr(acc), _ptr(out), capacity, _ptr(n_found),
                                     _stream(stream)))


def ht_fill_peaks_noalloc(spec, x, y, z, acc, out, capacity, n_found, stream=None):
    g = make_grid(spec)
    _need_cuda(x, y, z, acc)
    _need_out(out, n_found)
    return check(lib().ht_fill_peaks_noalloc(ctypes.byref(g), _ptr(x), _ptr(y), _ptr(z), x.numel(),
                                             _ptr(acc), _ptr(out), capacity, _ptr(n_found),
                                             _stream(stream)))


def ht_fill_peaks_batch(spec, events, x, y, z, acc, out, n_found, stream=None):
    g = make_grid(spec)
    _need_cuda(x, y, z, acc)
    _need_out(out, n_found)
    arr = (Event * len(events))(*events)
    return check(lib().ht_fill_peaks_batch(ctypes.byref(g), arr, len(events), _ptr(x), _ptr(y),
                                           _ptr(z), _ptr(acc), _ptr(out), _ptr(n_found),
                                           _stream(stream)))


def ht_readout(spec, out, n_found, capacity, stream=None):
    """Track parameters of a device peak list; returns a device uint8 tensor holding
    ht_track[capacity] records (view with TRACK_DTYPE after copying to the host)."""
    import torch
    g = make_grid(spec)
    _need_out(out, n_found)
    tracks = torch.empty((max(capacity, 1) * TRACK_DTYPE.itemsize,), dtype=torch.uint8,
                         device=out.device)
    check(lib().ht_readout(ctypes.byref(g), _ptr(out), _ptr(n_found), capacity, _ptr(tracks),
                           _stream(stream)))
    return tracks


def tracks_to_host(tracks, n_found, capacity):
    k = min(int(n_found.item()), capacity)
    return tracks.cpu().numpy().view(TRACK_DTYPE)[:k].copy()


def ht_debug_pointer_kind(ptr: int) -> int:
    """0 refused, 1 device memory, 2 mapped pinned host memory, 3 managed (host-only query)."""
    k = ctypes.c_int32()
    check(lib().ht_debug_pointer_kind(ctypes.c_void_p(ptr), ctypes.byref(k)))
    return k.value


def ht_debug_batch_plan(spec, n_hits):
    """(direct, scratch_bytes) that ht_fill_peaks_batch would use for events of these sizes at
    the grid's current launch shape (host only)."""
    g = make_grid(spec)
    arr = (Event * len(n_hits))(*[Event(0, int(n), 0, 0) for n in n_hits])
    d = ctypes.c_int32()
    b = ctypes.c_int64()
    check(lib().ht_debug_batch_plan(ctypes.byref(g), arr, len(n_hits), ctypes.byref(d),
                                    ctypes.byref(b)))
    return bool(d.value), b.value


def ht_debug_hit_values(spec, x, y, z, stream=None):
    import torch
    g = make_grid(spec)
    _need_cuda(x, y, z)
    n = x.numel()
    info = torch.zeros((n, 4), dtype=torch.int32, device=x.device)
    vals = torch.zeros((n, 3), dtype=torch.float32, device=x.device)
    slabs = torch.zeros((n, 4), dtype=torch.int32, device=x.device)
    check(lib().ht_debug_hit_values(ctypes.byref(g), _ptr(x), _ptr(y), _ptr(z), n, _ptr(info),
                                    _ptr(vals), _ptr(slabs), _stream(stream)))
    return info, vals, slabs


def ht_debug_unary(v, root, inv2, stream=None):
    """root = sqrt(v) and inv2 = 1 / (v + v) on the device (float32 tensors of one size)."""
    _need_cuda(v, root, inv2)
    n = v.numel()
    if root.numel() != n or inv2.numel() != n:
        raise ValueError("v, root and inv2 must have the same size")
    check(lib().ht_debug_unary(_ptr(v), _ptr(root), _ptr(inv2), n, _stream(stream)))


def ht_profile_enable(mode):
    """0 / False: off; 1 / True: every stage; 2: the fill stages only."""
    return check(lib().ht_profile_enable(int(mode)))


def ht_profile_read(name: str, reset: bool = False):
    """(summed milliseconds, number of launches) of one stage since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(lib().ht_profile_read(name.encode(), ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


# ---------------------------------------------------------------------------------------------
# Convenience wrappers
# ---------------------------------------------------------------------------------------------
def new_acc(spec, n_events: int = 1, device="cuda"):
    """A vote-matrix buffer (int32 storage holding the uint32 counts)."""
    import torch
    g = make_grid(spec)
    shape = g.shape if n_events == 1 else (n_events, *g.shape)
    return torch.empty(shape, dtype=torch.int32, device=device)


def new_peaks(capacity: int, device="cuda"):
    import torch
    return (torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=device),
            torch.zeros(1, dtype=torch.int64, device=device))


def as_u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def hits_to_device(x, y, z, device="cuda"):
    import torch
    return tuple(torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device) for a in (x, y, z))


def peaks_to_host(out, n_found, capacity, allow_truncation=False):
    """(cells, votes, n_found) of a peak list on the device. The count is the total found; when
    it exceeds the capacity the list holds only the first `capacity` peaks, and this raises
    HTError(HT_EOVERFLOW) unless allow_truncation is set."""
    n = int(n_found.item())
    if n > capacity and not allow_truncation:
        raise HTError(HT_EOVERFLOW, "%d peaks found, the output holds %d" % (n, capacity))
    k = min(n, capacity)
    arr = as_u32(out[:k]) if k else np.zeros((0, 2), np.uint32)
    return arr[:, 0].copy(), arr[:, 1].copy(), n


def fill(spec, x, y, z, acc=None, stream=None, atomic=False):
    if acc is None:
        acc = new_acc(spec, device=x.device)
    ht_fill(spec, x, y, z, acc, stream, atomic=atomic)
    return acc


def peaks(spec, acc, capacity=1 << 20, stream=None, allow_truncation=False):
    out, nf = new_peaks(capacity, acc.device)
    ht_peaks(spec, acc, out, capacity, nf, stream)
    return peaks_to_host(out, nf, capacity, allow_truncation)


def fill_peaks(spec, x, y, z, capacity=1 << 20, acc=None, stream=None, allow_truncation=False):
    if acc is None:
        acc = new_acc(spec, device=x.device)
    out, nf = new_peaks(capacity, x.device)
    ht_fill_peaks(spec, x, y, z, acc, out, capacity, nf, stream)
    cells, votes, n = peaks_to_host(out, nf, capacity, allow_truncation)
    return acc, cells, votes, n


@dataclass
class BatchResult:
    acc: object
    peaks: list       # per event (cells, votes, n_found)


def fill_peaks_batch(spec, hits, capacity=1 << 16, acc=None, stream=None, device="cuda",
                     allow_truncation=False):
    """hits: list of (x, y, z) host arrays. Returns per-event peak lists and the accumulators.
    Raises HTError(HT_EOVERFLOW) when an event has more peaks than `capacity`, unless
    allow_truncation is set (its list then holds the first `capacity` peaks)."""
    import torch
    xs = np.concatenate([np.asarray(h[0], np.float32) for h in hits]) if hits else np.zeros(0, np.float32)
    ys = np.concatenate([np.asarray(h[1], np.float32) for h in hits]) if hits else np.zeros(0, np.float32)
    zs = np.concatenate([np.asarray(h[2], np.float32) for h in hits]) if hits else np.zeros(0, np.float32)
    x, y, z = hits_to_device(xs, ys, zs, device)
    evs, off = [], 0
    for i, h in enumerate(hits):
        n = len(h[0])
        evs.append(Event(off, n, i * capacity, capacity))
        off += n
    if acc is None:
        acc = new_acc(spec, len(hits), device)
    out = torch.empty((max(len(hits) * capacity, 1), 2), dtype=torch.int32, device=device)
    nf = torch.zeros(max(len(hits), 1), dtype=torch.int64, device=device)
    ht_fill_peaks_batch(spec, evs, x, y, z, acc, out, nf, stream)
    torch.cuda.synchronize()
    res = []
    nfh = nf.cpu().numpy()
    outh = as_u32(out)
    for i in range(len(hits)):
        if int(nfh[i]) > capacity and not allow_truncation:
            raise HTError(HT_EOVERFLOW, "event %d: %d peaks found, the output holds %d"
                          % (i, int(nfh[i]), capacity))
        k = min(int(nfh[i]), capacity)
        seg = outh[i * capacity: i * capacity + k]
        res.append((seg[:, 0].copy(), seg[:, 1].copy(), int(nfh[i])))
    return BatchResult(acc, res)


class Server:
    """The library's request loop (ht_serve_*) over host numpy hits."""

    def __init__(self, spec, hbm_budget_bytes, peak_capacity=1 << 16, max_hits=40000,
                 max_batch=16, n_streams=2, queue_depth=256, device=0):
        self.grid = make_grid(spec)
        self.opts = ServeOpts(hbm_budget_bytes, peak_capacity, max_hits, max_batch, n_streams,
                              queue_depth, device)
        self.cap = peak_capacity
        self._h = ctypes.c_void_p()
        check(lib().ht_serve_create(ctypes.byref(self.grid), ctypes.byref(self.opts),
                                    ctypes.byref(self._h)))
        self._out = (Peak * peak_capacity)()

    def submit(self, x, y, z):
        """Returns a ticket, or None when the queue is full (HT_EAGAIN)."""
        fp = ctypes.POINTER(ctypes.c_float)
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        z = np.ascontiguousarray(z, np.float32)
        t = ctypes.c_uint64()
        rc = lib().ht_serve_submit(self._h, x.ctypes.data_as(fp), y.ctypes.data_as(fp),
                                   z.ctypes.data_as(fp), x.size, ctypes.byref(t))
        if rc == HT_EAGAIN:
            return None
        check(rc)
        return t.value

    def poll(self, ticket):
        """None while in flight; else (cells, votes, n_found, Timing)."""
        nf = ctypes.c_int64()
        tm = Timing()
        rc = lib().ht_serve_poll(self._h, ticket, self._out, self.cap, ctypes.byref(nf),
                                 ctypes.byref(tm))
        if rc == HT_EAGAIN:
            return None
        if rc not in (HT_OK, HT_EOVERFLOW):
            check(rc)
        k = min(nf.value, self.cap)
        arr = np.frombuffer(self._out, dtype=np.uint32).reshape(-1, 2)[:k]
        return arr[:, 0].copy(), arr[:, 1].copy(), nf.value, tm

    def close(self):
        if self._h:
            lib().ht_serve_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
