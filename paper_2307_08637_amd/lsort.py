"""ctypes binding of liblsort (C ABI in include/lsort.h).

Argument marshalling only: every step of the sort runs in the library's HIP
kernels.  Tensors must be torch CUDA (ROCm) tensors on the current device;
work is enqueued on torch's current stream.  If the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsort.so")

LS_F64, LS_U64, LS_I64, LS_F32 = 0, 1, 2, 3
MODEL = {"auto": 0, "rmi": 1, "mlp": 2, "splitter": 3}
FLAG_NO_FALLBACK, FLAG_SYNC_LEVELS, FLAG_FIXED_LEVELS, FLAG_COLLECT_STATS, FLAG_TUNED, FLAG_REFIT = 1, 2, 4, 8, 16, 32
FLAG_MODEL_BASE = 64
MAX_STAT_LEVELS = 32


class Options(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("model", C.c_uint32), ("buckets", C.c_uint32), ("leaves", C.c_uint32),
        ("tree_buckets", C.c_uint32), ("cutoff", C.c_uint32), ("max_levels", C.c_uint32), ("flags", C.c_uint32),
        ("sample_frac", C.c_double), ("fallback_ratio", C.c_double), ("seed", C.c_uint64),
        ("mlp_steps", C.c_uint32), ("mlp_sample", C.c_uint32), ("mlp_lr", C.c_float), ("tile", C.c_uint32),
        ("balance_pct", C.c_uint32), ("reserved", C.c_uint32 * 3),
    ]


class LevelStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "segments", "keys", "buckets", "max_bucket", "max_bucket_x1000_over_mean", "empty", "equality", "base",
        "recurse", "fallback", "learned", "tree", "radix")]


class Stats(C.Structure):
    _fields_ = [("levels", C.c_uint32), ("first_model", C.c_uint32), ("base_items", C.c_uint64),
                ("copy_items", C.c_uint64), ("mlp_loss_first", C.c_double), ("mlp_loss_last", C.c_double),
                ("overflow", C.c_uint32), ("merged_items", C.c_uint32), ("level", LevelStats * MAX_STAT_LEVELS)]


class KernelTiming(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint64), ("ms", C.c_double), ("keys", C.c_double)]


class LsortError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32, i32, dbl = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int, C.c_double
        sig = {
            "ls_sort": [vp, u64, i32, vp, vp, vp],
            "ls_sort_noalloc": [vp, u64, i32, vp, vp, vp],
            "ls_sort_payload64": [vp, u64, i32, vp, vp, vp],
            "ls_sort_segmented": [vp, vp, u64, u64, i32, vp, vp, vp],
            "ls_workspace_bytes": [u64, u64, i32, i32, vp, vp],
            "ls_set_workspace": [vp, C.c_size_t, vp],
            "ls_get_stats": [vp],
            "ls_sample": [vp, u64, i32, u64, u64, vp, vp],
            "ls_rmi_fit": [vp, u64, i32, u32, dbl, vp, vp],
            "ls_rmi_fit_block": [vp, u64, i32, u32, dbl, vp, vp],
            "ls_rmi_buckets": [vp, u64, i32, vp, u32, dbl, vp, vp],
            "ls_splitters": [vp, u64, i32, u32, vp, vp, vp, vp],
            "ls_splitter_buckets": [vp, u64, i32, vp, vp, u32, vp, vp],
            "ls_partition_rmi": [vp, vp, u64, i32, vp, u32, dbl, u32, vp, vp, vp, vp],
            "ls_partition_splitters": [vp, vp, u64, i32, vp, vp, u32, vp, vp, vp, vp],
            "ls_mlp_loss_grad": [vp, vp, vp, u64, vp, vp, vp],
            "ls_mlp_loss_grad_regions": [vp, vp, vp, u64, vp, vp, vp],
            "ls_mlp_train": [vp, u64, i32, vp, u32, C.c_float, vp, vp, vp, vp],
            "ls_mlp_buckets": [vp, u64, i32, vp, vp, u32, vp, vp],
            "ls_mlp_rmi_fit": [vp, u64, i32, vp, vp, u32, dbl, vp, vp],
            "ls_autotune": [C.c_char_p],
            "ls_load_tuning": [C.c_char_p],
            "ls_tuned_options": [u64, u64, vp],
            "ls_mlp_rmi_buckets": [vp, u64, i32, vp, vp, vp, u32, dbl, vp, vp],
            "ls_timing": [i32],
            "ls_timing_read": [vp, u32, vp],
            "ls_timing_records": [vp, u32, vp],
            "ls_stream_copy": [vp, vp, u64, vp],
            "ls_stream_read": [vp, u64, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.ls_last_error.restype = C.c_char_p
        L.ls_last_error.argtypes = []
        L.ls_version.restype = C.c_char_p
        L.ls_version.argtypes = []
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise LsortError(f"liblsort status {rc}: {lib().ls_last_error().decode()}")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype(t) -> int:
    """Key-type code of a tensor (or of a torch dtype)."""
    d = t if isinstance(t, torch.dtype) else t.dtype
    codes = {torch.float64: LS_F64, torch.uint64: LS_U64, torch.int64: LS_I64, torch.float32: LS_F32}
    if d not in codes:
        raise TypeError(f"keys must be float64, uint64, int64 or float32, got {d}")
    return codes[d]


def _dtype_engine(t: torch.Tensor) -> int:
    """Code for the single-step entry points (float64 / uint64 only)."""
    c = _dtype(t)
    if c not in (LS_F64, LS_U64):
        raise TypeError(f"this step takes float64 or uint64 keys, got {t.dtype}")
    return c


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def make_options(model="auto", buckets=0, leaves=0, tree_buckets=0, cutoff=0, max_levels=0, flags=0,
                 sample_frac=0.0, fallback_ratio=0.0, seed=0, mlp_steps=0, mlp_sample=0, mlp_lr=0.0, tile=0,
                 balance_pct=0,
                 stats=True, fixed_levels=False, no_fallback=False, tuned=False, refit=False,
                 model_base=False) -> Options:
    o = Options()
    o.struct_size = C.sizeof(Options)
    o.model = MODEL[model] if isinstance(model, str) else int(model)
    o.buckets, o.leaves, o.tree_buckets, o.cutoff, o.max_levels = buckets, leaves, tree_buckets, cutoff, max_levels
    f = flags | (FLAG_COLLECT_STATS if stats else 0)
    f |= FLAG_FIXED_LEVELS if fixed_levels else FLAG_SYNC_LEVELS
    f |= FLAG_NO_FALLBACK if no_fallback else 0
    f |= FLAG_TUNED if tuned else 0
    f |= FLAG_REFIT if refit else 0
    f |= FLAG_MODEL_BASE if model_base else 0
    o.flags = f
    o.sample_frac, o.fallback_ratio, o.seed = sample_frac, fallback_ratio, seed
    o.mlp_steps, o.mlp_sample, o.mlp_lr = mlp_steps, mlp_sample, mlp_lr
    o.tile = tile
    o.balance_pct = balance_pct
    return o


PAYLOAD64 = (torch.uint64, torch.int64, torch.float64)


def sort(keys: torch.Tensor, payload: torch.Tensor | None = None, **opts) -> None:
    """Sort keys (float64 / float32 by totalOrder, uint64 / int64 numerically)
    in place; payload (uint32, or any 8-byte type) follows stably."""
    _dev(keys, "keys")
    o = make_options(**opts)
    if payload is not None:
        _dev(payload, "payload")
        if payload.numel() != keys.numel():
            raise ValueError("payload must have one entry per key")
        if payload.dtype in PAYLOAD64:
            _check(lib().ls_sort_payload64(_ptr(keys), keys.numel(), _dtype(keys), _ptr(payload), C.byref(o),
                                           _stream()))
            return
        if payload.dtype != torch.uint32:
            raise ValueError("payload must be uint32 or an 8-byte type")
    _check(lib().ls_sort(_ptr(keys), keys.numel(), _dtype(keys), _ptr(payload), C.byref(o), _stream()))


def sort_noalloc(keys: torch.Tensor, payload: torch.Tensor | None = None, **opts) -> None:
    """sort() through the allocation-free entry point (fixed scratch array in
    the library; fixed level count; calls on one device must not overlap)."""
    _dev(keys, "keys")
    if payload is not None:
        _dev(payload, "payload")
        if payload.dtype != torch.uint32 or payload.numel() != keys.numel():
            raise ValueError("payload must be uint32 with one entry per key")
    o = make_options(**opts)
    _check(lib().ls_sort_noalloc(_ptr(keys), keys.numel(), _dtype(keys), _ptr(payload), C.byref(o), _stream()))


def sort_segmented(keys: torch.Tensor, offsets: torch.Tensor, payload: torch.Tensor | None = None,
                   total: int | None = None, **opts) -> None:
    """Sort each [offsets[i], offsets[i+1]) independently in one batched pass."""
    _dev(keys, "keys")
    _dev(offsets, "offsets")
    if offsets.dtype != torch.uint64:
        raise ValueError("offsets must be uint64")
    if payload is not None:
        _dev(payload, "payload")
        if payload.dtype != torch.uint32 or payload.numel() != keys.numel():
            raise ValueError("payload must be uint32 with one entry per key")
    m = offsets.numel() - 1
    tot = keys.numel() if total is None else int(total)
    o = make_options(**opts)
    _check(lib().ls_sort_segmented(_ptr(keys), _ptr(offsets), m, tot, _dtype(keys), _ptr(payload), C.byref(o),
                                   _stream()))


def stats() -> dict:
    s = Stats()
    _check(lib().ls_get_stats(C.byref(s)))
    levels = []
    for i in range(s.levels):
        lv = s.level[i]
        levels.append({f: getattr(lv, f) for f, _ in LevelStats._fields_})
    return {"levels": levels, "first_model": s.first_model, "base_items": s.base_items,
            "copy_items": s.copy_items, "mlp_loss_first": s.mlp_loss_first, "mlp_loss_last": s.mlp_loss_last,
            "overflow": s.overflow, "merged_items": s.merged_items}


def workspace_bytes(n: int, m: int = 1, dtype=torch.float64, payload=False, **opts) -> int:
    """payload: False / True (uint32) / 64 (64-bit payload)."""
    out = C.c_size_t()
    o = make_options(**opts)
    has = 2 if payload == 64 else int(bool(payload))
    _check(lib().ls_workspace_bytes(n, m, _dtype(dtype), has, C.byref(o), C.byref(out)))
    return out.value


def set_workspace(buf: torch.Tensor | None) -> None:
    if buf is None:
        _check(lib().ls_set_workspace(None, 0, _stream()))
    else:
        _dev(buf, "workspace")
        _check(lib().ls_set_workspace(_ptr(buf), buf.numel() * buf.element_size(), _stream()))


# -- single steps -------------------------------------------------------------------

def sample(keys: torch.Tensor, seed: int, S: int) -> torch.Tensor:
    _dev(keys, "keys")
    out = torch.empty(S, dtype=keys.dtype, device=keys.device)
    _check(lib().ls_sample(_ptr(keys), keys.numel(), _dtype_engine(keys), seed, S, _ptr(out), _stream()))
    return out


def rmi_fit(sorted_sample: torch.Tensor, L: int, R: float) -> torch.Tensor:
    _dev(sorted_sample, "sorted_sample")
    out = torch.empty(2 + 4 * L, dtype=torch.float64, device=sorted_sample.device)
    _check(lib().ls_rmi_fit(_ptr(sorted_sample), sorted_sample.numel(), _dtype_engine(sorted_sample), L, float(R), _ptr(out),
                            _stream()))
    return out


def rmi_fit_block(sorted_sample: torch.Tensor, L: int, R: int) -> torch.Tensor:
    _dev(sorted_sample, "sorted_sample")
    out = torch.empty(2 + 4 * L, dtype=torch.float64, device=sorted_sample.device)
    _check(lib().ls_rmi_fit_block(_ptr(sorted_sample), sorted_sample.numel(), _dtype_engine(sorted_sample), L, float(R),
                                  _ptr(out), _stream()))
    return out


def rmi_buckets(keys: torch.Tensor, params: torch.Tensor, L: int, R: float) -> torch.Tensor:
    _dev(keys, "keys")
    _dev(params, "params")
    out = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
    _check(lib().ls_rmi_buckets(_ptr(keys), keys.numel(), _dtype_engine(keys), _ptr(params), L, float(R), _ptr(out),
                                _stream()))
    return out


def splitters(sorted_sample: torch.Tensor, B: int):
    _dev(sorted_sample, "sorted_sample")
    u = torch.empty(max(B - 1, 1), dtype=torch.uint64, device=sorted_sample.device)
    eq = torch.zeros(max(B - 1, 1), dtype=torch.uint8, device=sorted_sample.device)
    m = torch.zeros(1, dtype=torch.uint32, device=sorted_sample.device)
    _check(lib().ls_splitters(_ptr(sorted_sample), sorted_sample.numel(), _dtype_engine(sorted_sample), B, _ptr(u), _ptr(eq),
                              _ptr(m), _stream()))
    k = int(m.cpu().item())
    return u[:k], eq[:k]


def splitter_buckets(keys: torch.Tensor, u: torch.Tensor, eq: torch.Tensor) -> torch.Tensor:
    _dev(keys, "keys")
    u = u.contiguous()
    eq = eq.contiguous()
    out = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
    _check(lib().ls_splitter_buckets(_ptr(keys), keys.numel(), _dtype_engine(keys), _ptr(u), _ptr(eq), u.numel(), _ptr(out),
                                     _stream()))
    return out


def partition_rmi(keys, params, L, R, nb, payload=None):
    _dev(keys, "keys")
    ok = torch.empty_like(keys)
    op = None if payload is None else torch.empty_like(payload)
    counts = torch.zeros(nb, dtype=torch.uint64, device=keys.device)
    _check(lib().ls_partition_rmi(_ptr(keys), _ptr(payload), keys.numel(), _dtype_engine(keys), _ptr(params), L, float(R), nb,
                                  _ptr(ok), _ptr(op), _ptr(counts), _stream()))
    return ok, op, counts


def partition_splitters(keys, u, eq, payload=None):
    _dev(keys, "keys")
    ok = torch.empty_like(keys)
    op = None if payload is None else torch.empty_like(payload)
    nb = u.numel() + 1 + int(eq.to(torch.int64).sum().item())
    counts = torch.zeros(nb, dtype=torch.uint64, device=keys.device)
    _check(lib().ls_partition_splitters(_ptr(keys), _ptr(payload), keys.numel(), _dtype_engine(keys), _ptr(u), _ptr(eq),
                                        u.numel(), _ptr(ok), _ptr(op), _ptr(counts), _stream()))
    return ok, op, counts


# -- MLP CDF ---------------------------------------------------------------------------

MLP_NP = 321


def mlp_loss_grad(params: torch.Tensor, t: torch.Tensor, y: torch.Tensor, regions: bool = False):
    """(loss, grad) of the mean squared error at params (float32[321]) over
    inputs t and targets y (float32, device); regions: by activation regions
    (t non-decreasing), as the training computes it."""
    for a, nm in ((params, "params"), (t, "t"), (y, "y")):
        _dev(a, nm)
        if a.dtype != torch.float32:
            raise ValueError(f"{nm} must be float32")
    grad = torch.empty(MLP_NP, dtype=torch.float32, device=t.device)
    loss = torch.empty(1, dtype=torch.float32, device=t.device)
    fn = lib().ls_mlp_loss_grad_regions if regions else lib().ls_mlp_loss_grad
    _check(fn(_ptr(params), _ptr(t), _ptr(y), t.numel(), _ptr(grad), _ptr(loss), _stream()))
    return loss, grad


def mlp_train(sorted_sample: torch.Tensor, steps: int, lr: float, params_init: torch.Tensor | None = None):
    """Train on a sorted sample: returns (params float32[321], lo_inv float64[2],
    losses float32[steps])."""
    _dev(sorted_sample, "sorted_sample")
    dev = sorted_sample.device
    params = torch.empty(MLP_NP, dtype=torch.float32, device=dev)
    lo_inv = torch.empty(2, dtype=torch.float64, device=dev)
    losses = torch.empty(max(steps, 1), dtype=torch.float32, device=dev)
    _check(lib().ls_mlp_train(_ptr(sorted_sample), sorted_sample.numel(), _dtype_engine(sorted_sample), _ptr(params_init),
                              steps, float(lr), _ptr(params), _ptr(lo_inv), _ptr(losses), _stream()))
    return params, lo_inv, losses[:steps]


def mlp_buckets(keys: torch.Tensor, params: torch.Tensor, lo_inv: torch.Tensor, R: int) -> torch.Tensor:
    _dev(keys, "keys")
    out = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
    _check(lib().ls_mlp_buckets(_ptr(keys), keys.numel(), _dtype_engine(keys), _ptr(params), _ptr(lo_inv), R, _ptr(out),
                                _stream()))
    return out


def mlp_rmi_fit(sorted_sample: torch.Tensor, params: torch.Tensor, lo_inv: torch.Tensor, L: int,
                R: float) -> torch.Tensor:
    _dev(sorted_sample, "sorted_sample")
    leaves = torch.empty(4 * L, dtype=torch.float64, device=sorted_sample.device)
    _check(lib().ls_mlp_rmi_fit(_ptr(sorted_sample), sorted_sample.numel(), _dtype_engine(sorted_sample), _ptr(params),
                                _ptr(lo_inv), L, float(R), _ptr(leaves), _stream()))
    return leaves


def mlp_rmi_buckets(keys: torch.Tensor, params: torch.Tensor, lo_inv: torch.Tensor, leaves: torch.Tensor, L: int,
                    R: float) -> torch.Tensor:
    _dev(keys, "keys")
    out = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
    _check(lib().ls_mlp_rmi_buckets(_ptr(keys), keys.numel(), _dtype_engine(keys), _ptr(params), _ptr(lo_inv), _ptr(leaves),
                                    L, float(R), _ptr(out), _stream()))
    return out

# -- tuning ---------------------------------------------------------------------------

def autotune(table_path: str) -> None:
    """Time the candidate options per size class on this device, write the
    JSON table and load it (about a minute)."""
    _check(lib().ls_autotune(os.fsencode(table_path)))


def load_tuning(table_path: str | None) -> None:
    """Load a table written by autotune (None: unload).  Calls made with
    tuned=True then take buckets / cutoff / tree_buckets from it."""
    _check(lib().ls_load_tuning(None if table_path is None else os.fsencode(table_path)))


def tuned_options(n: int, m: int = 1) -> dict:
    o = Options()
    _check(lib().ls_tuned_options(n, m, C.byref(o)))
    return {"buckets": o.buckets, "cutoff": o.cutoff, "tree_buckets": o.tree_buckets, "leaves": o.leaves,
            "tile": o.tile}

def timing(enable: bool) -> None:
    """Start (clearing earlier records) or stop per-kernel event timing."""
    _check(lib().ls_timing(int(enable)))


def timing_read() -> dict:
    """{kernel name: {"launches", "ms", "keys"}} summed over the recorded calls."""
    buf = (KernelTiming * 32)()
    cnt = C.c_uint32()
    _check(lib().ls_timing_read(buf, 32, C.byref(cnt)))
    return {buf[i].name.decode(): {"launches": buf[i].launches, "ms": buf[i].ms, "keys": buf[i].keys}
            for i in range(cnt.value)}


def timing_records(cap: int = 4096) -> list:
    """The recorded launches in order: [(kernel name, ms, level keys)]."""
    buf = (KernelTiming * cap)()
    cnt = C.c_uint32()
    _check(lib().ls_timing_records(buf, cap, C.byref(cnt)))
    return [(buf[i].name.decode(), buf[i].ms, buf[i].keys) for i in range(cnt.value)]


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """Reference copy of src's 8-byte words into dst (same size, 8-byte aligned)."""
    _dev(src, "src")
    _dev(dst, "dst")
    if src.numel() * src.element_size() != dst.numel() * dst.element_size() or src.element_size() != 8:
        raise ValueError("stream_copy needs two tensors of the same number of 8-byte elements")
    _check(lib().ls_stream_copy(_ptr(src), _ptr(dst), src.numel(), _stream()))


def stream_read(src: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Reference read of src's 8-byte words; returns a one-element uint64
    device tensor holding their sum mod 2^64."""
    _dev(src, "src")
    if src.element_size() != 8:
        raise ValueError("stream_read needs 8-byte elements")
    if out is None:
        out = torch.empty(2, dtype=torch.uint64, device=src.device)
    _check(lib().ls_stream_read(_ptr(src), src.numel(), _ptr(out), _stream()))
    return out[:1]


def version() -> str:
    return lib().ls_version().decode()
