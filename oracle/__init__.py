"""CPU oracle for the MoMA hot path: TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links, loads or
calls it, and it shares no code with the GPU library.

The arithmetic lives in ``moma_oracle.c`` (plain C: schoolbook big integers,
Knuth Algorithm D division, the NTT by its definition and a textbook radix-2
transform).  This module only marshals numpy arrays through ctypes.  Vectors
are element-major ``(n, L)`` uint32 arrays, limb 0 least significant.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "moma_oracle.c")
# MOMA_ORACLE_LIB names another build of the same source (the test suite runs
# the pins once more against a build with memory and undefined-behaviour checks)
_LIB = os.environ.get("MOMA_ORACLE_LIB") or os.path.join(_HERE, "libmoma_oracle.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True, out: str | None = None, flags: list[str] | None = None) -> str:
    """Compile the oracle with gcc and OpenMP (in place, next to its source, or
    to `out`; `flags` replaces the default -O2)."""
    path = out or _LIB
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        opt = list(flags) if flags else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        L = _lib
        for name in ("oracle_vadd", "oracle_vsub", "oracle_vmul"):
            getattr(L, name).argtypes = [_u32p, ctypes.c_int, ctypes.c_int64, _u32p, _u32p, _u32p]
        L.oracle_axpy.argtypes = [_u32p, ctypes.c_int, ctypes.c_int64, _u32p, _u32p, _u32p, _u32p]
        for name in ("oracle_ntt_direct", "oracle_intt_direct"):
            getattr(L, name).argtypes = [_u32p, ctypes.c_int, ctypes.c_int64, _u32p, _u32p, _i64p, ctypes.c_int64, _u32p]
        for name in ("oracle_ntt_radix2", "oracle_intt_radix2", "oracle_cyclic_conv"):
            getattr(L, name).argtypes = [_u32p, ctypes.c_int, ctypes.c_int64, _u32p, _u32p, _u32p]
        L.oracle_big_mul.argtypes = [_u32p, _u32p, ctypes.c_int, _u32p, ctypes.c_int]
        L.oracle_big_rem.argtypes = [_u32p, _u32p, ctypes.c_int, _u32p, ctypes.c_int]
        L.oracle_big_add.argtypes = [_u32p, _u32p, _u32p, ctypes.c_int]
        L.oracle_big_sub.argtypes = [_u32p, _u32p, _u32p, ctypes.c_int]
        L.oracle_mod_pow.argtypes = [_u32p, _u32p, _u32p, ctypes.c_int, _u32p, ctypes.c_int]
        L.oracle_mod_inv.argtypes = [_u32p, _u32p, _u32p, ctypes.c_int]
        L.oracle_addback_count.restype = ctypes.c_int64
        _dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_mlp_forward.argtypes = [_dp, _dp, ctypes.c_int64, _dp]
        L.oracle_mlp_grad.argtypes = [_dp, _dp, _dp, ctypes.c_int64, _dp, _dp]
        L.oracle_mlp_adam.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double]
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(_u32p)


def _limbs(v: int, L: int) -> np.ndarray:
    if v < 0 or v >> (32 * L):
        raise ValueError("value does not fit in L limbs")
    return np.array([(v >> (32 * j)) & 0xFFFFFFFF for j in range(L)], dtype=np.uint32)


def _int(a) -> int:
    v = 0
    for w in reversed([int(x) for x in a]):
        v = (v << 32) | w
    return v


def _vec(x, L):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    if x.ndim != 2 or x.shape[1] != L:
        raise ValueError(f"expected (n, {L}) uint32, got {x.shape}")
    return x


def addback_count() -> int:
    """Times the add-back branch of the division has run in this process."""
    return int(lib().oracle_addback_count())


def threads() -> int:
    return int(lib().oracle_threads())


# ----------------------------------------------------------------- words

def big_mul(a: int, b: int, la: int, lb: int) -> int:
    r = np.zeros(la + lb, dtype=np.uint32)
    assert lib().oracle_big_mul(_p(r), _p(_limbs(a, la)), la, _p(_limbs(b, lb)), lb) == 0
    return _int(r)


def big_rem(u: int, v: int, lu: int, lv: int) -> int:
    r = np.zeros(lv, dtype=np.uint32)
    rc = lib().oracle_big_rem(_p(r), _p(_limbs(u, lu)), lu, _p(_limbs(v, lv)), lv)
    if rc:
        raise ValueError(f"oracle_big_rem rc={rc}")
    return _int(r)


def big_add(a: int, b: int, n: int) -> tuple[int, int]:
    r = np.zeros(n, dtype=np.uint32)
    c = lib().oracle_big_add(_p(r), _p(_limbs(a, n)), _p(_limbs(b, n)), n)
    return _int(r), int(c)


def big_sub(a: int, b: int, n: int) -> tuple[int, int]:
    r = np.zeros(n, dtype=np.uint32)
    c = lib().oracle_big_sub(_p(r), _p(_limbs(a, n)), _p(_limbs(b, n)), n)
    return _int(r), int(c)


def mod_pow(a: int, e: int, q: int, L: int) -> int:
    ne = max(1, (e.bit_length() + 31) // 32)
    r = np.zeros(L, dtype=np.uint32)
    assert lib().oracle_mod_pow(_p(r), _p(_limbs(a, L)), _p(_limbs(e, ne)), ne, _p(_limbs(q, L)), L) == 0
    return _int(r)


def mod_inv(a: int, q: int, L: int) -> int:
    r = np.zeros(L, dtype=np.uint32)
    assert lib().oracle_mod_inv(_p(r), _p(_limbs(a, L)), _p(_limbs(q, L)), L) == 0
    return _int(r)


# ----------------------------------------------------------------- BLAS

def _binop(name, q, L, a, b):
    a, b = _vec(a, L), _vec(b, L)
    assert a.shape == b.shape
    out = np.zeros_like(a)
    rc = getattr(lib(), name)(_p(_limbs(q, L)), L, a.shape[0], _p(a), _p(b), _p(out))
    if rc:
        raise ValueError(f"{name} rc={rc}")
    return out


def vadd(q: int, L: int, a, b) -> np.ndarray:
    return _binop("oracle_vadd", q, L, a, b)


def vsub(q: int, L: int, a, b) -> np.ndarray:
    return _binop("oracle_vsub", q, L, a, b)


def vmul(q: int, L: int, a, b) -> np.ndarray:
    return _binop("oracle_vmul", q, L, a, b)


def axpy(q: int, L: int, alpha: int, x, y) -> np.ndarray:
    x, y = _vec(x, L), _vec(y, L)
    out = np.zeros_like(x)
    rc = lib().oracle_axpy(_p(_limbs(q, L)), L, x.shape[0], _p(_limbs(alpha, L)), _p(x), _p(y), _p(out))
    if rc:
        raise ValueError(f"oracle_axpy rc={rc}")
    return out


# ----------------------------------------------------------------- NTT

def _sel(ks, n):
    if ks is None:
        return None, n
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    return ks, ks.size


def ntt_direct(q: int, L: int, omega: int, x, ks=None) -> np.ndarray:
    """y_k = sum_j x_j omega^{jk} mod q for k in ks (all k if None), by the definition."""
    x = _vec(x, L)
    n = x.shape[0]
    ks, nk = _sel(ks, n)
    out = np.zeros((nk, L), dtype=np.uint32)
    kp = ks.ctypes.data_as(_i64p) if ks is not None else None
    rc = lib().oracle_ntt_direct(_p(_limbs(q, L)), L, n, _p(_limbs(omega, L)), _p(x), kp, nk, _p(out))
    if rc:
        raise ValueError(f"oracle_ntt_direct rc={rc}")
    return out


def intt_direct(q: int, L: int, omega: int, y, js=None) -> np.ndarray:
    """x_j = n^{-1} sum_k y_k omega^{-jk} mod q for j in js (all j if None); omega is the forward root."""
    y = _vec(y, L)
    n = y.shape[0]
    js, nj = _sel(js, n)
    out = np.zeros((nj, L), dtype=np.uint32)
    jp = js.ctypes.data_as(_i64p) if js is not None else None
    rc = lib().oracle_intt_direct(_p(_limbs(q, L)), L, n, _p(_limbs(omega, L)), _p(y), jp, nj, _p(out))
    if rc:
        raise ValueError(f"oracle_intt_direct rc={rc}")
    return out


def ntt_radix2(q: int, L: int, omega: int, x) -> np.ndarray:
    x = _vec(x, L)
    out = np.zeros_like(x)
    rc = lib().oracle_ntt_radix2(_p(_limbs(q, L)), L, x.shape[0], _p(_limbs(omega, L)), _p(x), _p(out))
    if rc:
        raise ValueError(f"oracle_ntt_radix2 rc={rc}")
    return out


def intt_radix2(q: int, L: int, omega: int, y) -> np.ndarray:
    y = _vec(y, L)
    out = np.zeros_like(y)
    rc = lib().oracle_intt_radix2(_p(_limbs(q, L)), L, y.shape[0], _p(_limbs(omega, L)), _p(y), _p(out))
    if rc:
        raise ValueError(f"oracle_intt_radix2 rc={rc}")
    return out


def cyclic_conv(q: int, L: int, a, b) -> np.ndarray:
    return _binop("oracle_cyclic_conv", q, L, a, b)


# ----------------------------------------------------------------- MLP (FP64)

MLP_IN, MLP_H = 7, 64


def mlp_nparams() -> int:
    return int(lib().oracle_mlp_nparams())


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def mlp_forward(params, x) -> np.ndarray:
    """Network output for each row of x (rows x MLP_IN)."""
    p, pp = _d(params)
    xx, xp = _d(x)
    y = np.zeros(xx.shape[0])
    _, yp = _d(y)
    assert lib().oracle_mlp_forward(pp, xp, xx.shape[0], yp) == 0
    return y


def mlp_grad(params, x, t) -> tuple[np.ndarray, float]:
    """Gradient of the mean squared error with respect to every parameter, and the loss."""
    p, pp = _d(params)
    xx, xp = _d(x)
    tt, tp = _d(t)
    g = np.zeros(mlp_nparams())
    loss = np.zeros(1)
    _, gp = _d(g)
    _, lp = _d(loss)
    assert lib().oracle_mlp_grad(pp, xp, tp, xx.shape[0], gp, lp) == 0
    return g, float(loss[0])


def mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on params, m, v (float64 arrays)."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g, gp = _d(grad)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib().oracle_mlp_adam(params.ctypes.data_as(dp), gp, m.ctypes.data_as(dp), v.ctypes.data_as(dp), step,
                                 lr, beta1, beta2, eps) == 0
