"""Python binding of the MoMA library for MI355X (gfx950).

Argument marshalling only: every step runs in the HIP kernels of libmoma.so
through the C ABI declared in include/moma.h.  PyTorch supplies device memory
and streams.  Importing this package fails loudly when libmoma.so is missing;
there is no CPU fallback.

Vectors are torch tensors on the GPU of shape (limbs, n) holding 32-bit words
(dtype torch.int32 or torch.uint32), limb-planar: row j is limb j (least
significant first) of every element.  Scalars q, omega and alpha are Python
ints.  All functions enqueue on the current torch stream unless `stream` is
given, and return the output tensor.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmoma.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_2501_07535_amd.build, or __graft_entry__.build())")

# torch ships its own HIP runtime with the same soname (libamdhip64.so.7).
# Loading torch first makes libmoma.so bind to that copy, so tensors, streams
# and our kernels share one runtime; a second runtime instance in the process
# would see no device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes():
    try:
        maps = open("/proc/self/maps").read().splitlines()
    except OSError:
        return []
    return sorted({ln.split()[-1] for ln in maps if "libamdhip64" in ln})


if len(_hip_runtimes()) > 1:
    raise ImportError(f"two HIP runtimes are loaded ({_hip_runtimes()}); import torch before loading libmoma.so")
_u32p = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p

for _name in ("moma_vadd", "moma_vsub", "moma_vmul"):
    getattr(_lib, _name).argtypes = [_u32p, ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, _vp, _vp]
    getattr(_lib, _name).restype = ctypes.c_int
_lib.moma_axpy.argtypes = [_u32p, ctypes.c_uint32, ctypes.c_uint64, _u32p, _vp, _vp, _vp, _vp]
_lib.moma_axpy.restype = ctypes.c_int
for _name in ("moma_ntt_fwd", "moma_ntt_inv"):
    getattr(_lib, _name).argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32, _vp, _vp, _vp]
    getattr(_lib, _name).restype = ctypes.c_int
_lib.moma_vmul_set_variant.argtypes = [_u32p, ctypes.c_uint32, ctypes.c_uint32]
_lib.moma_vmul_get_variant.argtypes = [_u32p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
_lib.moma_vmul_tune.argtypes = [_u32p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_uint32)]
for _name in ("moma_ntt_cyclic_mul", "moma_ntt_cyclic_mul_noalloc"):
    getattr(_lib, _name).argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32, _vp, _vp, _vp, _vp]
    getattr(_lib, _name).restype = ctypes.c_int
_lib.moma_ntt_prepare.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32]
_lib.moma_ntt_prepare.restype = ctypes.c_int
_lib.moma_ntt_describe.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32, _u32p, _u32p, ctypes.c_uint32,
                                   _u32p]
_lib.moma_ntt_describe.restype = ctypes.c_int
_lib.moma_check_canonical.argtypes = [_u32p, ctypes.c_uint32, ctypes.c_uint64, _vp, ctypes.POINTER(ctypes.c_uint64),
                                      _vp]
_lib.moma_check_canonical.restype = ctypes.c_int
_lib.moma_set_input_check.argtypes = [ctypes.c_int]
_lib.moma_set_input_check.restype = ctypes.c_int
for _name in ("moma_pack_planar", "moma_unpack_planar"):
    getattr(_lib, _name).argtypes = [ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, _vp]
    getattr(_lib, _name).restype = ctypes.c_int


class Schedule(ctypes.Structure):
    """Launch shape of a transform plan (see moma_ntt_schedule_t): as a tuple
    (tile_log, col_log, threads, radix_log, mul_variant); a 4-tuple means the
    schoolbook multiply (mul_variant 0)."""
    _fields_ = [("tile_log", ctypes.c_uint32), ("col_log", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("radix_log", ctypes.c_uint32), ("mul_variant", ctypes.c_uint32)]

    def as_tuple(self):
        return (self.tile_log, self.col_log, self.threads, self.radix_log, self.mul_variant)


NTT_MUL_SCHOOLBOOK, NTT_MUL_KARATSUBA = 0, 1
COSTMODEL_FEATURES = 7


_lib.moma_ntt_set_schedule.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(Schedule)]
_lib.moma_ntt_set_schedule.restype = ctypes.c_int
_lib.moma_ntt_get_schedule.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(Schedule)]
_lib.moma_ntt_get_schedule.restype = ctypes.c_int
_lib.moma_ntt_default_schedule.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(Schedule)]


class _Job(ctypes.Structure):
    _fields_ = [("q", _u32p), ("omega", _u32p), ("n", ctypes.c_uint64), ("limbs", ctypes.c_uint32),
                ("kind", ctypes.c_uint32), ("d_in", _vp), ("d_out", _vp), ("d_in2", _vp), ("alpha", _u32p)]


JOB_FORWARD, JOB_INVERSE, JOB_CYCLIC_MUL, JOB_VADD, JOB_VSUB, JOB_VMUL, JOB_AXPY = range(7)


_lib.moma_batch_create.argtypes = [ctypes.POINTER(_Job), ctypes.c_uint32, ctypes.POINTER(_vp)]
_lib.moma_batch_create.restype = ctypes.c_int
_lib.moma_batch_run.argtypes = [_vp, _vp]
_lib.moma_batch_run.restype = ctypes.c_int
_lib.moma_batch_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)]
_lib.moma_batch_info.restype = ctypes.c_int
_lib.moma_batch_destroy.argtypes = [_vp]
_lib.moma_batch_destroy.restype = ctypes.c_int


class _TuneOpts(ctypes.Structure):
    _fields_ = [("reps", ctypes.c_uint32), ("warmup", ctypes.c_uint32), ("top_k", ctypes.c_uint32),
                ("max_candidates", ctypes.c_uint32)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("best", Schedule), ("best_us", ctypes.c_float), ("timed", ctypes.c_uint32),
                ("feasible", ctypes.c_uint32)]


class _TuneRow(ctypes.Structure):
    _fields_ = [("limbs", ctypes.c_uint32), ("log2_n", ctypes.c_uint32), ("sched", Schedule), ("us", ctypes.c_float),
                ("reps", ctypes.c_uint32)]


class _TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


_fp = ctypes.POINTER(ctypes.c_float)
_lib.moma_ntt_tune.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_TuneOpts),
                               ctypes.POINTER(_TuneResult)]
_lib.moma_ntt_candidates.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(Schedule), ctypes.c_uint32,
                                     ctypes.POINTER(ctypes.c_uint32)]
_lib.moma_tune_db_count.restype = ctypes.c_uint32
_lib.moma_tune_db_get.argtypes = [ctypes.c_uint32, ctypes.POINTER(_TuneRow)]
_lib.moma_tune_db_clear.restype = None
_lib.moma_tune_db_save.argtypes = [ctypes.c_char_p]
_lib.moma_tune_db_load.argtypes = [ctypes.c_char_p]
_lib.moma_costmodel_features.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(Schedule), _fp]
_lib.moma_costmodel_train.argtypes = [_fp, _fp, ctypes.c_uint32, ctypes.POINTER(_TrainOpts), _fp]
_lib.moma_costmodel_predict.argtypes = [_fp, ctypes.c_uint32, _fp]
_lib.moma_costmodel_save.argtypes = [ctypes.c_char_p]
_lib.moma_costmodel_load.argtypes = [ctypes.c_char_p]
_lib.moma_costmodel_clear.restype = None
_lib.moma_mlp_nparams.restype = ctypes.c_uint32
_lib.moma_mlp_forward.argtypes = [_vp, _vp, ctypes.c_uint32, _vp, _vp]
_lib.moma_mlp_grad.argtypes = [_vp, _vp, _vp, ctypes.c_uint32, _vp, _vp, _vp]
_lib.moma_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_uint32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, _vp]
_lib.moma_strerror.argtypes = [ctypes.c_int]
_lib.moma_strerror.restype = ctypes.c_char_p
_lib.moma_last_error_detail.restype = ctypes.c_char_p
_lib.moma_version.restype = ctypes.c_char_p
_lib.moma_shutdown.restype = None

class _PeakRates(ctypes.Structure):
    _fields_ = [("add_u32", ctypes.c_double), ("add_co_addc_u32", ctypes.c_double), ("mad_u64_u32", ctypes.c_double),
                ("mad_addc_u32", ctypes.c_double), ("mul_lo_u32", ctypes.c_double), ("mul_hi_u32", ctypes.c_double),
                ("hbm_copy", ctypes.c_double), ("hbm_triad", ctypes.c_double), ("compute_units", ctypes.c_uint32)]


_lib.moma_measure_peaks.argtypes = [ctypes.POINTER(_PeakRates), ctypes.c_uint64, _vp]
_lib.moma_measure_peaks.restype = ctypes.c_int

MOMA_OK, MOMA_E_ARG, MOMA_E_MODULUS, MOMA_E_ROOT, MOMA_E_NOMEM, MOMA_E_HIP, MOMA_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6

EXPORTED = ("moma_strerror", "moma_last_error_detail", "moma_version", "moma_vadd", "moma_vsub", "moma_vmul",
            "moma_axpy", "moma_vmul_set_variant", "moma_vmul_get_variant", "moma_vmul_tune", "moma_ntt_fwd", "moma_ntt_inv", "moma_ntt_cyclic_mul", "moma_ntt_cyclic_mul_noalloc", "moma_ntt_prepare", "moma_ntt_describe",
            "moma_ntt_set_schedule", "moma_ntt_get_schedule", "moma_ntt_default_schedule", "moma_batch_create", "moma_batch_run",
            "moma_batch_info", "moma_batch_destroy", "moma_ntt_tune", "moma_ntt_candidates", "moma_tune_db_count",
            "moma_tune_db_get", "moma_tune_db_clear", "moma_tune_db_save", "moma_tune_db_load",
            "moma_costmodel_features", "moma_costmodel_train", "moma_costmodel_predict", "moma_costmodel_save",
            "moma_costmodel_load", "moma_costmodel_clear", "moma_mlp_nparams", "moma_mlp_forward", "moma_mlp_grad",
            "moma_mlp_adam", "moma_check_canonical", "moma_set_input_check", "moma_pack_planar",
            "moma_unpack_planar", "moma_measure_peaks", "moma_shutdown")


class MomaError(RuntimeError):
    def __init__(self, code: int):
        self.code = code
        super().__init__(f"{_lib.moma_strerror(code).decode()}: {_lib.moma_last_error_detail().decode()}")


def _check(rc: int):
    if rc != MOMA_OK:
        raise MomaError(rc)


def library():
    """The loaded ctypes library (for callers that want the raw C ABI)."""
    return _lib


def version() -> str:
    return _lib.moma_version().decode()


def _words(v: int, limbs: int):
    if v < 0 or v >> (32 * limbs):
        raise ValueError(f"value does not fit in {limbs} limbs")
    arr = (ctypes.c_uint32 * limbs)(*[(v >> (32 * j)) & 0xFFFFFFFF for j in range(limbs)])
    return arr


def _dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"{name} must hold 32-bit words (int32 or uint32)")
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous (limbs, n) tensor")
    return t


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _out(like, out):
    import torch
    if out is None:
        return torch.empty_like(like)
    _dev(out, "out")
    if out.shape != like.shape:
        raise ValueError("out has the wrong shape")
    return out


def _binop(fn, a, b, q, out, stream):
    _dev(a, "a"); _dev(b, "b")
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    limbs, n = a.shape
    out = _out(a, out)
    _check(fn(_words(q, limbs), limbs, n, a.data_ptr(), b.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


def vadd(a, b, q: int, out=None, stream=None):
    """out = (a + b) mod q elementwise."""
    return _binop(_lib.moma_vadd, a, b, q, out, stream)


def vsub(a, b, q: int, out=None, stream=None):
    """out = (a - b) mod q elementwise."""
    return _binop(_lib.moma_vsub, a, b, q, out, stream)


def vmul(a, b, q: int, out=None, stream=None):
    """out = (a * b) mod q elementwise."""
    return _binop(_lib.moma_vmul, a, b, q, out, stream)


def axpy(alpha: int, x, y, q: int, out=None, stream=None):
    """out = (alpha * x + y) mod q elementwise."""
    _dev(x, "x"); _dev(y, "y")
    if x.shape != y.shape:
        raise ValueError("x and y must have the same shape")
    limbs, n = x.shape
    out = _out(x, out)
    _check(_lib.moma_axpy(_words(q, limbs), limbs, n, _words(alpha, limbs), x.data_ptr(), y.data_ptr(),
                          out.data_ptr(), _stream(stream)))
    return out


VMUL_SCHOOLBOOK, VMUL_KARATSUBA = 0, 1


def check_canonical(x, q: int, stream=None) -> int:
    """Number of elements of x (a (limbs, n) limb-planar tensor) that are >= q;
    waits for the stream."""
    _dev(x, "x")
    limbs, n = x.shape
    bad = ctypes.c_uint64(0)
    _check(_lib.moma_check_canonical(_words(q, limbs), limbs, n, x.data_ptr(), ctypes.byref(bad), _stream(stream)))
    return int(bad.value)


def set_input_check(on: bool):
    """Debugging mode: every call first counts its non-canonical inputs and fails
    with MOMA_E_ARG if there are any (each such call waits for its stream)."""
    _check(_lib.moma_set_input_check(1 if on else 0))


def pack(x, out=None, stream=None):
    """Element-major (n, limbs) words -> the library's limb-planar (limbs, n)."""
    _dev(x, "x")
    n, limbs = x.shape
    if out is None:
        import torch
        out = torch.empty((limbs, n), dtype=x.dtype, device=x.device)
    _dev(out, "out")
    if tuple(out.shape) != (limbs, n):
        raise ValueError("out must have shape (limbs, n)")
    _check(_lib.moma_pack_planar(limbs, n, x.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


def unpack(x, out=None, stream=None):
    """Limb-planar (limbs, n) -> element-major (n, limbs) words."""
    _dev(x, "x")
    limbs, n = x.shape
    if out is None:
        import torch
        out = torch.empty((n, limbs), dtype=x.dtype, device=x.device)
    _dev(out, "out")
    if tuple(out.shape) != (n, limbs):
        raise ValueError("out must have shape (n, limbs)")
    _check(_lib.moma_unpack_planar(limbs, n, x.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


def vmul_set_variant(q: int, limbs: int, variant: int):
    """Word-product variant of vmul for moduli with q's compute limb count."""
    _check(_lib.moma_vmul_set_variant(_words(q, limbs), limbs, variant))


def vmul_get_variant(q: int, limbs: int) -> int:
    v = ctypes.c_uint32(0)
    _check(_lib.moma_vmul_get_variant(_words(q, limbs), limbs, ctypes.byref(v)))
    return int(v.value)


def vmul_tune(q: int, limbs: int, n: int, reps: int = 5) -> dict:
    """Time schoolbook and Karatsuba vmul on n elements and install the faster."""
    us = (ctypes.c_float * 2)()
    ch = ctypes.c_uint32(0)
    _check(_lib.moma_vmul_tune(_words(q, limbs), limbs, n, reps, us, ctypes.byref(ch)))
    return {"schoolbook_us": float(us[0]), "karatsuba_us": float(us[1]) or None, "chosen": int(ch.value)}


def ntt_fwd(x, q: int, omega: int, out=None, stream=None):
    """Forward NTT y_k = sum_j x_j omega^{jk} mod q, natural order in and out."""
    _dev(x, "x")
    limbs, n = x.shape
    out = _out(x, out)
    _check(_lib.moma_ntt_fwd(_words(q, limbs), _words(omega, limbs), n, limbs, x.data_ptr(), out.data_ptr(),
                             _stream(stream)))
    return out


def ntt_inv(y, q: int, omega: int, out=None, stream=None):
    """Inverse NTT x_j = n^-1 sum_k y_k omega^{-jk} mod q; omega is the forward root."""
    _dev(y, "y")
    limbs, n = y.shape
    out = _out(y, out)
    _check(_lib.moma_ntt_inv(_words(q, limbs), _words(omega, limbs), n, limbs, y.data_ptr(), out.data_ptr(),
                             _stream(stream)))
    return out


def ntt_cyclic_mul(a, b, q: int, omega: int, out=None, stream=None):
    """Cyclic product out = a * b mod (x^n - 1, q): inv(fwd(a) . fwd(b)), the pointwise
    product fused into the inverse transform's first pass."""
    _dev(a, "a"); _dev(b, "b")
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    limbs, n = a.shape
    out = _out(a, out)
    _check(_lib.moma_ntt_cyclic_mul(_words(q, limbs), _words(omega, limbs), n, limbs, a.data_ptr(), b.data_ptr(),
                                    out.data_ptr(), _stream(stream)))
    return out


def ntt_cyclic_mul_noalloc(a, b, q: int, omega: int, out, stream=None):
    """The cyclic product through the entry point that allocates no device
    memory: the plan must exist (ntt_prepare) and `out` is required; the
    spectra live in the library's fixed scratch array (NOALLOC_SCRATCH_WORDS)."""
    _dev(a, "a"); _dev(b, "b"); _dev(out, "out")
    if a.shape != b.shape or out.shape != a.shape:
        raise ValueError("a, b and out must have the same shape")
    limbs, n = a.shape
    _check(_lib.moma_ntt_cyclic_mul_noalloc(_words(q, limbs), _words(omega, limbs), n, limbs, a.data_ptr(),
                                            b.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


NOALLOC_SCRATCH_WORDS = 1 << 24  # MOMA_NOALLOC_SCRATCH_WORDS


def ntt_prepare(q: int, omega: int, n: int, limbs: int):
    """Build the plan (twiddle tables) for (q, omega, n, limbs) ahead of timed calls."""
    _check(_lib.moma_ntt_prepare(_words(q, limbs), _words(omega, limbs), n, limbs))


def ntt_describe(q: int, omega: int, n: int, limbs: int) -> dict:
    """Schedule of the plan: passes (kernel launches) per transform and stages per pass."""
    npasses, climbs = ctypes.c_uint32(0), ctypes.c_uint32(0)
    stages = (ctypes.c_uint32 * 16)()
    _check(_lib.moma_ntt_describe(_words(q, limbs), _words(omega, limbs), n, limbs, ctypes.byref(npasses), stages,
                                  16, ctypes.byref(climbs)))
    return {"passes": int(npasses.value), "stages": [int(stages[i]) for i in range(npasses.value)],
            "compute_limbs": int(climbs.value)}


def ntt_set_schedule(q: int, omega: int, n: int, limbs: int, sched=None):
    """Set the plan's launch shape: a (tile_log, col_log, threads, radix_log[, mul_variant]) tuple, or None
    for the plan's initial choice."""
    ptr = None
    if sched is not None:
        ptr = ctypes.byref(Schedule(*[int(v) for v in sched]))
    _check(_lib.moma_ntt_set_schedule(_words(q, limbs), _words(omega, limbs), n, limbs, ptr))


def _default_schedule_for(limbs_compute: int, log2_n: int) -> tuple:
    s = Schedule()
    _check(_lib.moma_ntt_default_schedule(limbs_compute, log2_n, ctypes.byref(s)))
    return s.as_tuple()


def ntt_default_schedule(limbs_compute: int, log2_n: int) -> tuple:
    """The fixed rule a fresh plan falls back to without timings or a loaded cost model."""
    return _default_schedule_for(limbs_compute, log2_n)


def ntt_get_schedule(q: int, omega: int, n: int, limbs: int) -> tuple:
    s = Schedule()
    _check(_lib.moma_ntt_get_schedule(_words(q, limbs), _words(omega, limbs), n, limbs, ctypes.byref(s)))
    return s.as_tuple()


class Batch:
    """Many transforms and BLAS calls run as one graph launch.

    jobs: iterable of (x, out, q, omega, kind) with x / out limb-planar device
    tensors of shape (limbs, n) (out may be x).  kind is JOB_FORWARD (or False),
    JOB_INVERSE (or True), JOB_CYCLIC_MUL or a BLAS kind (JOB_VADD, JOB_VSUB,
    JOB_VMUL, JOB_AXPY).  For a cyclic product and the BLAS kinds x is the
    pair (a, b) (axpy: (x, y)); for axpy the fourth entry is alpha, for the
    other BLAS kinds it is ignored.  The batch keeps references to the tensors;
    run() recomputes every job from its current inputs.
    """

    def __init__(self, jobs):
        self._keep = []
        recs = []
        for x, out, q, omega, kind in jobs:
            kind = int(kind)
            if kind not in range(7):
                raise ValueError(f"unknown job kind {kind}")
            pair = kind == JOB_CYCLIC_MUL or kind >= JOB_VADD
            x2 = None
            if pair:
                x, x2 = x
                _dev(x2, "b")
                if x2.shape != x.shape:
                    raise ValueError("the two inputs must have the same shape")
                self._keep.append(x2)
            _dev(x, "x")
            _dev(out, "out")
            limbs, n = x.shape
            qw = _words(q, limbs)
            ww = _words(omega if (kind < JOB_VADD and omega is not None) else 0, limbs)
            aw = _words(omega, limbs) if kind == JOB_AXPY else None
            self._keep += [x, out, qw, ww, aw]
            recs.append(_Job(ctypes.cast(qw, _u32p), ctypes.cast(ww, _u32p), n, limbs, kind, x.data_ptr(),
                             out.data_ptr(), x2.data_ptr() if pair else None,
                             ctypes.cast(aw, _u32p) if aw is not None else None))
        arr = (_Job * len(recs))(*recs)
        h = _vp()
        _check(_lib.moma_batch_create(arr, len(recs), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(_lib.moma_batch_run(self._h, _stream(stream)))

    def info(self) -> dict:
        nl, ni = ctypes.c_uint32(0), ctypes.c_uint64(0)
        _check(_lib.moma_batch_info(self._h, ctypes.byref(nl), ctypes.byref(ni)))
        return {"launches": int(nl.value), "items": int(ni.value)}

    def close(self):
        if getattr(self, "_h", None):
            _lib.moma_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


# ----------------------------------------------------------------- autotuner

def ntt_tune(q: int, omega: int, n: int, limbs: int, reps: int = 5, warmup: int = 2, top_k: int = 0,
             max_candidates: int = 0) -> dict:
    """Time the plan's launch shapes (all, or the cost model's top_k), install the fastest."""
    o = _TuneOpts(reps, warmup, top_k, max_candidates)
    r = _TuneResult()
    _check(_lib.moma_ntt_tune(_words(q, limbs), _words(omega, limbs), n, limbs, ctypes.byref(o), ctypes.byref(r)))
    return {"best": r.best.as_tuple(), "best_us": float(r.best_us), "timed": int(r.timed),
            "feasible": int(r.feasible)}


def ntt_candidates(limbs_compute: int, log2_n: int) -> list:
    cnt = ctypes.c_uint32(0)
    _check(_lib.moma_ntt_candidates(limbs_compute, log2_n, None, 0, ctypes.byref(cnt)))
    arr = (Schedule * max(1, cnt.value))()
    _check(_lib.moma_ntt_candidates(limbs_compute, log2_n, arr, cnt.value, ctypes.byref(cnt)))
    return [arr[i].as_tuple() for i in range(cnt.value)]


def tune_db_rows() -> list:
    out = []
    row = _TuneRow()
    for i in range(_lib.moma_tune_db_count()):
        _check(_lib.moma_tune_db_get(i, ctypes.byref(row)))
        out.append({"limbs": int(row.limbs), "log2_n": int(row.log2_n), "sched": row.sched.as_tuple(),
                    "us": float(row.us), "reps": int(row.reps)})
    return out


def tune_db_clear():
    _lib.moma_tune_db_clear()


def tune_db_save(path: str):
    _check(_lib.moma_tune_db_save(path.encode()))


def tune_db_load(path: str):
    _check(_lib.moma_tune_db_load(path.encode()))


# ----------------------------------------------------------------- cost model

def costmodel_features(limbs_compute: int, log2_n: int, sched) -> list:
    out = (ctypes.c_float * COSTMODEL_FEATURES)()
    _check(_lib.moma_costmodel_features(limbs_compute, log2_n, ctypes.byref(Schedule(*sched)), out))
    return list(out)


def _f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_fp)


def costmodel_train(features, log_us, epochs: int = 200, batch: int = 256, lr: float = 3e-3, seed: int = 1) -> float:
    """Train the model on the GPU from features (rows, 7) and log-microsecond targets; returns the final MSE."""
    f, fp = _f32(features)
    t, tp = _f32(log_us)
    mse = ctypes.c_float(0)
    _check(_lib.moma_costmodel_train(fp, tp, t.shape[0], ctypes.byref(_TrainOpts(epochs, batch, lr, seed)),
                                     ctypes.byref(mse)))
    return float(mse.value)


def costmodel_predict(features):
    import numpy as np
    f, fp = _f32(features)
    out = np.zeros(f.shape[0], dtype=np.float32)
    _check(_lib.moma_costmodel_predict(fp, f.shape[0], out.ctypes.data_as(_fp)))
    return out


def costmodel_save(path: str):
    _check(_lib.moma_costmodel_save(path.encode()))


def costmodel_load(path: str):
    _check(_lib.moma_costmodel_load(path.encode()))


def costmodel_clear():
    _lib.moma_costmodel_clear()


def mlp_nparams() -> int:
    return int(_lib.moma_mlp_nparams())


def mlp_forward(params, x, y, stream=None):
    """y[r] = network(x[r]) on device float32 tensors (params flat, x (rows, 6))."""
    _check(_lib.moma_mlp_forward(params.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr(), _stream(stream)))
    return y


def mlp_grad(params, x, t, grad, loss, stream=None):
    _check(_lib.moma_mlp_grad(params.data_ptr(), x.data_ptr(), t.data_ptr(), x.shape[0], grad.data_ptr(),
                              loss.data_ptr(), _stream(stream)))


def mlp_adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib.moma_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), step, lr, beta1,
                              beta2, eps, _stream(stream)))


def measure_peaks(hbm_bytes: int = 0, stream=None) -> dict:
    """Measured issue rates (lane operations per second) and HBM bandwidths
    (bytes per second); synchronises the stream."""
    r = _PeakRates()
    _check(_lib.moma_measure_peaks(ctypes.byref(r), hbm_bytes, _stream(stream)))
    return {name: getattr(r, name) for name, _ in _PeakRates._fields_}


def shutdown():
    _lib.moma_shutdown()


# The cost model trained on this device class's timing database (written by
# `python -m paper_2501_07535_amd.tuning train --model ...`): loaded at
# import so that new plans without timings start from its top-ranked
# schedule.  MOMA_NO_COSTMODEL=1 keeps the fixed default rule instead.
COSTMODEL_PATH = os.path.join(_HERE, "costmodel_gfx950.txt")


def load_packaged_costmodel() -> bool:
    if os.path.exists(COSTMODEL_PATH) and not os.environ.get("MOMA_NO_COSTMODEL"):
        costmodel_load(COSTMODEL_PATH)
        return True
    return False


load_packaged_costmodel()
