"""CPU oracle for the learned sample sort -- TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded implementation of what the GPU path computes,
written from the paper ("LearnedSort as a learning-augmented SampleSort",
Carvalho & Lawrence, SSDBM 2023).  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product path
(the HIP library and its binding) never does.

The arithmetic lives in ``lsort_oracle.c`` (built with gcc into
``liblsort_oracle.so`` next to this file); this module only marshals numpy
arrays through ctypes.  See the C file for the passage each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lsort_oracle.c")
LIB = os.path.join(HERE, "liblsort_oracle.so")

F64, U64, I64, F32 = 0, 1, 2, 3
MLP_NP = 321


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        u64, u32, i32, dbl, vp = C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_void_p
        sig = {
            "orc_ord": (u64, [u64, i32]),
            "orc_unord": (u64, [u64, i32]),
            "orc_sort": (i32, [vp, vp, i32, vp, u64, i32]),
            "orc_sort_segmented": (i32, [vp, vp, i32, vp, u64, i32]),
            "orc_splitmix64_at": (u64, [u64, u64]),
            "orc_sample_index": (u64, [u64, u64, u64]),
            "orc_sample": (None, [vp, u64, u64, u64, vp]),
            "orc_dup_fraction": (dbl, [vp, u64, i32]),
            "orc_policy_learned": (i32, [u64, vp, u64, i32, dbl, dbl]),
            "orc_rmi_leaf": (u32, [dbl, dbl, u32, dbl]),
            "orc_rmi_fit": (None, [vp, u64, u32, dbl, vp, vp, vp, vp]),
            "orc_rmi_bucket": (u32, [vp, u32, dbl, u64, i32]),
            "orc_rmi_buckets": (None, [vp, u32, dbl, vp, u64, i32, vp]),
            "orc_splitters": (u32, [vp, u64, u32, i32, vp, vp]),
            "orc_splitter_bucket": (u32, [vp, vp, u32, u64, i32]),
            "orc_radix_shift": (u32, [u64, u64, u32]),
            "orc_radix_bucket": (u32, [u64, u32, u64, i32]),
            "orc_partition": (None, [vp, vp, vp, u64, u32, vp, vp, vp, vp]),
            "orc_mlp_forward": (dbl, [vp, dbl, vp, vp, vp, vp]),
            "orc_mlp_loss_grad": (dbl, [vp, vp, vp, u64, vp]),
            "orc_adam_step": (None, [vp, vp, vp, vp, u64, u64, dbl, dbl, dbl, dbl]),
            "orc_mlp_input": (C.c_float, [dbl, dbl, dbl]),
            "orc_mlp_eval_f32": (C.c_float, [vp, C.c_float]),
            "orc_mlp_bucket": (u32, [vp, dbl, dbl, u32, u64, i32]),
            "orc_implicit_pivots": (None, [vp, vp, u64, u32, i32, vp, vp]),
            "orc_pivot_quality": (dbl, [vp, u64, vp, u32]),
            "orc_ord_array": (None, [vp, u64, i32, vp]),
            "orc_splitter_buckets": (None, [vp, vp, u32, vp, u64, i32, vp]),
            "orc_radix_buckets": (None, [vp, u32, vp, u64, i32, vp]),
            "orc_mlp_buckets": (None, [vp, dbl, dbl, u32, vp, u64, i32, vp]),
            "orc_mlp_init": (None, [vp, u64, dbl, vp]),
            "orc_mlp_step_scale": (None, [vp, vp]),
            "orc_mlp_effective": (None, [vp, vp]),
            "orc_mlp_lo_inv": (None, [vp, u64, i32, vp]),
            "orc_model_x_array": (None, [vp, u64, i32, vp]),
            "orc_mlp_train": (None, [vp, vp, u64, vp, u32, dbl, i32, vp, vp]),
            "orc_mlp_inputs": (None, [vp, u64, i32, dbl, dbl, vp]),
            "orc_mlp_leaf": (u32, [vp, dbl, dbl, u32, dbl]),
            "orc_mlp_rmi_fit": (None, [vp, u64, vp, dbl, dbl, u32, dbl, vp, vp, vp]),
            "orc_mlp_rmi_bucket": (u32, [vp, dbl, dbl, vp, u32, dbl, u64, i32]),
            "orc_mlp_rmi_buckets": (None, [vp, dbl, dbl, vp, u32, dbl, vp, u64, i32, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float64:
        return F64
    if a.dtype == np.uint64:
        return U64
    if a.dtype == np.int64:
        return I64
    if a.dtype == np.float32:
        return F32
    raise TypeError(f"keys must be float64, uint64, int64 or float32, got {a.dtype}")


def raw_bits(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype == np.float32:
        return a.view(np.uint32).astype(np.uint64)
    return a.view(np.uint64)


# -- 1. key order ------------------------------------------------------------

def ord_keys(a: np.ndarray) -> np.ndarray:
    """Ordered-u64 image of keys (IEEE totalOrder for float64)."""
    r = raw_bits(a)
    out = np.empty(r.size, dtype=np.uint64)
    lib().orc_ord_array(_p(r), r.size, dtype_code(a), _p(out))
    return out


# -- 2. the sort ---------------------------------------------------------------

def _payload(payload):
    """(copy, width): uint32 payloads stay 4-byte, 64-bit ones are 8-byte."""
    if payload is None:
        return None, 4
    p = np.ascontiguousarray(payload)
    if p.dtype.itemsize == 8:
        return p.copy(), 8
    return np.ascontiguousarray(payload, dtype=np.uint32).copy(), 4


def sort(keys: np.ndarray, payload: np.ndarray | None = None, want_perm: bool = False):
    """Stable sort of keys (float64 / float32 by totalOrder, uint64 / int64
    numerically); payload uint32 or 64-bit.
    Returns (sorted keys, permuted payload or None[, perm])."""
    dt = dtype_code(keys)
    k = np.ascontiguousarray(keys).copy()
    p, pw = _payload(payload)
    perm = np.empty(k.size, dtype=np.uint64) if want_perm else None
    rc = lib().orc_sort(_p(k), _p(p), pw, _p(perm), k.size, dt)
    if rc:
        raise MemoryError("oracle sort: out of memory")
    return (k, p, perm) if want_perm else (k, p)


def sort_segmented(keys: np.ndarray, offsets: np.ndarray, payload: np.ndarray | None = None):
    dt = dtype_code(keys)
    k = np.ascontiguousarray(keys).copy()
    p, pw = _payload(payload)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    rc = lib().orc_sort_segmented(_p(k), _p(p), pw, _p(off), off.size - 1, dt)
    if rc:
        raise MemoryError("oracle sort: out of memory")
    return k, p


# -- 3. sampling -----------------------------------------------------------------

def splitmix64_at(seed: int, k: int) -> int:
    return lib().orc_splitmix64_at(seed, k)


def sample_index(seed: int, k: int, n: int) -> int:
    return lib().orc_sample_index(seed, k, n)


def sample(keys: np.ndarray, seed: int, S: int) -> np.ndarray:
    r = raw_bits(keys)
    out = np.empty(S, dtype=np.uint64)
    lib().orc_sample(_p(r), r.size, seed, S, _p(out))
    return out.view(keys.dtype)


# -- 4. duplicates and policy ------------------------------------------------------

def dup_fraction(sorted_sample: np.ndarray) -> float:
    r = raw_bits(sorted_sample)
    return lib().orc_dup_fraction(_p(r), r.size, dtype_code(sorted_sample))


def policy_learned(n: int, sorted_sample: np.ndarray, large_n: float = 1e5, dup_limit: float = 0.10) -> bool:
    r = raw_bits(sorted_sample)
    return bool(lib().orc_policy_learned(n, _p(r), r.size, dtype_code(sorted_sample), large_n, dup_limit))


# -- 5. RMI ------------------------------------------------------------------------

def model_x(keys: np.ndarray) -> np.ndarray:
    """Model input of every key (orc_model_x; NaN for a non-finite key)."""
    r = raw_bits(keys)
    out = np.empty(r.size)
    lib().orc_model_x_array(_p(r), r.size, dtype_code(keys), _p(out))
    return out


def rmi_fit(sorted_x: np.ndarray, L: int, R: float, root=None):
    """Fit the monotone two-level RMI on a sorted sample of model inputs.
    Returns (raw[2+4L], scaled[2+4L], counts[L])."""
    x = np.ascontiguousarray(sorted_x, dtype=np.float64)
    raw = np.empty(2 + 4 * L)
    scaled = np.empty(2 + 4 * L)
    counts = np.empty(L, dtype=np.uint64)
    r = None if root is None else np.ascontiguousarray(root, dtype=np.float64)
    lib().orc_rmi_fit(_p(x), x.size, L, float(R), _p(r), _p(raw), _p(scaled), _p(counts))
    return raw, scaled, counts


def rmi_leaf(alpha_r: float, beta_r: float, L: int, x: float) -> int:
    return lib().orc_rmi_leaf(alpha_r, beta_r, L, x)


def rmi_buckets(scaled: np.ndarray, L: int, R: float, keys: np.ndarray) -> np.ndarray:
    r = raw_bits(keys)
    out = np.empty(r.size, dtype=np.uint32)
    sc = np.ascontiguousarray(scaled, dtype=np.float64)
    lib().orc_rmi_buckets(_p(sc), L, float(R), _p(r), r.size, dtype_code(keys), _p(out))
    return out


# -- 6. splitter tree -----------------------------------------------------------------

def splitters(sorted_sample: np.ndarray, B: int):
    """Returns (unique splitters as ordered u64, equality flags)."""
    r = raw_bits(sorted_sample)
    u = np.empty(max(B - 1, 1), dtype=np.uint64)
    eq = np.zeros(max(B - 1, 1), dtype=np.uint8)
    m = lib().orc_splitters(_p(r), r.size, B, dtype_code(sorted_sample), _p(u), _p(eq))
    return u[:m].copy(), eq[:m].copy()


def splitter_buckets(u: np.ndarray, eq: np.ndarray, keys: np.ndarray) -> np.ndarray:
    r = raw_bits(keys)
    dt = dtype_code(keys)
    uu = np.ascontiguousarray(u, dtype=np.uint64)
    ee = np.ascontiguousarray(eq, dtype=np.uint8)
    out = np.empty(r.size, dtype=np.uint32)
    lib().orc_splitter_buckets(_p(uu), _p(ee), uu.size, _p(r), r.size, dt, _p(out))
    return out


# -- 7. range radix -------------------------------------------------------------------

def radix_shift(lo: int, hi: int, log2B: int) -> int:
    return lib().orc_radix_shift(lo, hi, log2B)


def radix_buckets(lo: int, shift: int, keys: np.ndarray) -> np.ndarray:
    r = raw_bits(keys)
    dt = dtype_code(keys)
    out = np.empty(r.size, dtype=np.uint32)
    lib().orc_radix_buckets(lo, shift, _p(r), r.size, dt, _p(out))
    return out


# -- 8. one partition level ---------------------------------------------------------------

def partition(keys: np.ndarray, bucket: np.ndarray, B: int, payload: np.ndarray | None = None):
    """Stable counting sort by bucket id. Returns (keys, payload, counts, starts)."""
    r = raw_bits(keys)
    b = np.ascontiguousarray(bucket, dtype=np.uint32)
    ok = np.empty_like(r)
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32)
    op = None if p is None else np.empty_like(p)
    counts = np.empty(B, dtype=np.uint64)
    starts = np.empty(B, dtype=np.uint64)
    lib().orc_partition(_p(r), _p(p), _p(b), r.size, B, _p(ok), _p(op), _p(counts), _p(starts))
    return ok.view(keys.dtype), op, counts, starts


# -- 9. MLP ---------------------------------------------------------------------------------

def mlp_forward(params: np.ndarray, t: float) -> float:
    p = np.ascontiguousarray(params, dtype=np.float64)
    return lib().orc_mlp_forward(_p(p), float(t), None, None, None, None)


def mlp_loss_grad(params: np.ndarray, t: np.ndarray, y: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float64)
    tt = np.ascontiguousarray(t, dtype=np.float64)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    g = np.empty(MLP_NP)
    loss = lib().orc_mlp_loss_grad(_p(p), _p(tt), _p(yy), tt.size, _p(g))
    return loss, g


def adam_step(p, m, v, g, step, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    p = np.array(p, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_adam_step(_p(p), _p(m), _p(v), _p(gg), p.size, step, lr, b1, b2, eps)
    return p, m, v


def mlp_input(x: float, lo: float, inv: float) -> float:
    return lib().orc_mlp_input(x, lo, inv)


def mlp_eval_f32(w: np.ndarray, t: float) -> float:
    ww = np.ascontiguousarray(w, dtype=np.float32)
    return lib().orc_mlp_eval_f32(_p(ww), float(t))


def mlp_buckets(w: np.ndarray, lo: float, inv: float, R: int, keys: np.ndarray) -> np.ndarray:
    ww = np.ascontiguousarray(w, dtype=np.float32)
    r = raw_bits(keys)
    dt = dtype_code(keys)
    out = np.empty(r.size, dtype=np.uint32)
    lib().orc_mlp_buckets(_p(ww), lo, inv, R, _p(r), r.size, dt, _p(out))
    return out



def mlp_init(t_sorted: np.ndarray, eps: float = 1e-3) -> np.ndarray:
    """Data-dependent start point (piecewise-linear interpolant of the sample
    CDF through its octiles, plus eps-sized trainable weights)."""
    t = np.ascontiguousarray(t_sorted, dtype=np.float64)
    p = np.empty(MLP_NP)
    lib().orc_mlp_init(_p(t), t.size, float(eps), _p(p))
    return p


def mlp_inputs(keys: np.ndarray, lo: float, inv: float) -> np.ndarray:
    r = raw_bits(keys)
    out = np.empty(r.size, dtype=np.float32)
    lib().orc_mlp_inputs(_p(r), r.size, dtype_code(keys), lo, inv, _p(out))
    return out


def mlp_lo_inv(sorted_keys: np.ndarray):
    """(lo, inv) of the model input from a sorted sample (orc_mlp_lo_inv)."""
    r = raw_bits(sorted_keys)
    out = np.empty(2)
    lib().orc_mlp_lo_inv(_p(r), r.size, dtype_code(sorted_keys), _p(out))
    return float(out[0]), float(out[1])


def effective(params: np.ndarray) -> np.ndarray:
    """fp32 effective weights (orc_mlp_effective)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    w = np.empty(MLP_NP, dtype=np.float32)
    lib().orc_mlp_effective(_p(p), _p(w))
    return w


def mlp_step_scale(p0: np.ndarray) -> np.ndarray:
    """Optimiser step scale of each parameter at the start point p0 (see
    orc_mlp_step_scale)."""
    p = np.ascontiguousarray(p0, dtype=np.float64)
    s = np.empty(MLP_NP)
    lib().orc_mlp_step_scale(_p(p), _p(s))
    return s


def mlp_train(t: np.ndarray, y: np.ndarray, p0: np.ndarray, steps: int, lr: float, final: bool = False):
    """Full-batch fp64 training (see orc_mlp_train).  Returns the parameters
    with the lowest loss seen (or, with final=True, those after the last
    step) and the losses of every step."""
    tt = np.ascontiguousarray(t, dtype=np.float64)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    p = np.ascontiguousarray(p0, dtype=np.float64)
    out = np.empty(MLP_NP)
    losses = np.empty(steps)
    lib().orc_mlp_train(_p(tt), _p(yy), tt.size, _p(p), steps, float(lr), 1 if final else 0, _p(out), _p(losses))
    return out, losses


def mlp_forward_full(params: np.ndarray, t: float):
    """(output, z1, h1, z2, h2) of the fp64 forward pass."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    z1, h1, z2, h2 = (np.empty(16) for _ in range(4))
    out = lib().orc_mlp_forward(_p(p), float(t), _p(z1), _p(h1), _p(z2), _p(h2))
    return out, z1, h1, z2, h2


def mlp_leaf(w: np.ndarray, lo: float, inv: float, L: int, x: float) -> int:
    ww = np.ascontiguousarray(w, dtype=np.float32)
    return lib().orc_mlp_leaf(_p(ww), lo, inv, L, float(x))


def mlp_rmi_fit(sorted_x: np.ndarray, w: np.ndarray, lo: float, inv: float, L: int, R: float):
    """Leaves of the two-level model whose root is the MLP: (raw[4L],
    scaled[4L], counts[L])."""
    x = np.ascontiguousarray(sorted_x, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float32)
    raw = np.empty(4 * L)
    scaled = np.empty(4 * L)
    counts = np.empty(L, dtype=np.uint64)
    lib().orc_mlp_rmi_fit(_p(x), x.size, _p(ww), lo, inv, L, float(R), _p(raw), _p(scaled), _p(counts))
    return raw, scaled, counts


def mlp_rmi_buckets(w: np.ndarray, lo: float, inv: float, scaled: np.ndarray, L: int, R: float,
                    keys: np.ndarray) -> np.ndarray:
    ww = np.ascontiguousarray(w, dtype=np.float32)
    q = np.ascontiguousarray(scaled, dtype=np.float64)
    r = raw_bits(keys)
    out = np.empty(r.size, dtype=np.uint32)
    lib().orc_mlp_rmi_buckets(_p(ww), lo, inv, _p(q), L, float(R), _p(r), r.size, dtype_code(keys), _p(out))
    return out

# -- 10. pivots ------------------------------------------------------------------------------

def implicit_pivots(keys: np.ndarray, bucket: np.ndarray, B: int):
    r = raw_bits(keys)
    b = np.ascontiguousarray(bucket, dtype=np.uint32)
    piv = np.zeros(B, dtype=np.uint64)
    has = np.zeros(B, dtype=np.uint8)
    lib().orc_implicit_pivots(_p(r), _p(b), r.size, B, dtype_code(keys), _p(piv), _p(has))
    return piv, has.astype(bool)


def pivot_quality(sorted_ord: np.ndarray, pivot_ord: np.ndarray, B: int) -> float:
    s = np.ascontiguousarray(sorted_ord, dtype=np.uint64)
    p = np.ascontiguousarray(pivot_ord, dtype=np.uint64)
    assert p.size >= B - 1
    return lib().orc_pivot_quality(_p(s), s.size, _p(p), B)
