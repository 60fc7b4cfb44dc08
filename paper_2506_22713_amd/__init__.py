"""Python binding of the MI355X EOD-ABE library (argument marshalling only).

Every step of the method runs in the HIP kernels of ``libeodabe.so``; this
module only turns torch tensors into pointers and sizes, allocates the
caller-owned workspace and outputs with torch, and maps status codes to
exceptions.  Importing it fails loudly if the shared library has not been
built (``python -m paper_2506_22713_amd.build``).  Function names follow the
C ABI in ``include/eodabe.h``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeodabe.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"EOD-ABE HIP library not built: {LIB_PATH} is missing "
        "(run `python -m paper_2506_22713_amd.build`)")

_lib = ctypes.CDLL(LIB_PATH)

EODABE_OK = 0
EODABE_EINVAL = -1
EODABE_EWORKSPACE = -2
EODABE_ECAPACITY = -3
EODABE_ENONFINITE = -4
EODABE_EHIP = -5
EODABE_ENODEVICE = -6
EODABE_ESCRATCH = -7
EODABE_ESYNC = -8
NOALLOC_SCRATCH_BYTES = 64 << 20
EODABE_WTOL_FLOOR = 1
F32, F64 = 0, 1
SKETCH_NATIVE, SKETCH_F16, SKETCH_BF16 = 0, 1, 2

EXPORTED = [
    "eodabe_default_opts", "eodabe_create", "eodabe_create_host", "eodabe_destroy", "eodabe_workspace_size",
    "eodabe_factor", "eodabe_strerror", "eodabe_last_hip_error", "eodabe_philox",
    "eodabe_omega", "eodabe_sketch_workspace_size", "eodabe_sketch", "eodabe_basis",
    "eodabe_batched_workspace_size", "eodabe_factor_batched", "eodabe_tune_batched",
    "eodabe_profile", "eodabe_profile_read",
    "eodabe_mlp_param_count", "eodabe_mlp_workspace_size", "eodabe_mlp_forward", "eodabe_mlp_grad",
    "eodabe_mlp_adam", "eodabe_mlp_features", "eodabe_set_predictor", "eodabe_last_prediction",
    "eodabe_factor_noalloc", "eodabe_image_workspace_size", "eodabe_compress_image", "eodabe_features",
    "eodabe_knn_workspace_size", "eodabe_knn_cv", "eodabe_complex_workspace_size", "eodabe_factor_complex",
]
PROF_SKETCH, PROF_PROJECT, PROF_TILES = 0, 1, 2


class Opts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("power_iters", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("a_dtype", ctypes.c_int),
                ("sketch_dtype", ctypes.c_int), ("blocks_per_sync", ctypes.c_int),
                ("stream", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("blocks", ctypes.c_int),
                ("status_flags", ctypes.c_int), ("norm_a", ctypes.c_double),
                ("eps", ctypes.c_double), ("relres_est", ctypes.c_double)]


_vp, _i64, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
_lib.eodabe_default_opts.argtypes = [ctypes.POINTER(Opts)]
_lib.eodabe_default_opts.restype = None
_lib.eodabe_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(Opts)]
_lib.eodabe_create.restype = ctypes.c_int
_lib.eodabe_create_host.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(Opts)]
_lib.eodabe_create_host.restype = ctypes.c_int
_lib.eodabe_destroy.argtypes = [_vp]
_lib.eodabe_destroy.restype = None
_lib.eodabe_workspace_size.argtypes = [_vp, _i64, _i64, _i64]
_lib.eodabe_workspace_size.restype = _sz
_lib.eodabe_factor.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_double, _vp, _sz,
                               _vp, _vp, _vp, _i64, ctypes.POINTER(Info)]
_lib.eodabe_factor.restype = ctypes.c_int
# eodabe_factor through a CPython entry that converts its arguments in C
# (the same C-ABI call; ctypes' conversion costs microseconds per call)
try:
    from . import _fastcall
    _fastcall.bind(ctypes.cast(_lib.eodabe_factor, ctypes.c_void_p).value)
except ImportError:
    _fastcall = None
class ImageInfo(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64 * 4), ("channels", ctypes.c_int), ("relerr", ctypes.c_double),
                ("psnr", ctypes.c_double), ("ssim", ctypes.c_double), ("stored", ctypes.c_double),
                ("full", ctypes.c_double), ("reduction", ctypes.c_double), ("rank_bound", ctypes.c_double)]


_lib.eodabe_image_workspace_size.argtypes = [_vp, ctypes.c_int, _i64, _i64]
_lib.eodabe_image_workspace_size.restype = _sz
_lib.eodabe_compress_image.argtypes = [_vp, _vp, ctypes.c_int, _i64, _i64, ctypes.c_double, _vp, _sz, _vp, _i64,
                                       _vp, ctypes.POINTER(ImageInfo)]
_lib.eodabe_compress_image.restype = ctypes.c_int
_lib.eodabe_features.argtypes = [_vp, _vp, _vp, _i64, _i64, _i64, _vp, _i64]
_lib.eodabe_features.restype = ctypes.c_int
_lib.eodabe_knn_workspace_size.argtypes = [ctypes.c_int]
_lib.eodabe_knn_workspace_size.restype = _sz
_lib.eodabe_knn_cv.argtypes = [_vp, _vp, _i64, ctypes.c_int, _i64, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp,
                               _sz, _vp, ctypes.POINTER(ctypes.c_double)]
_lib.eodabe_knn_cv.restype = ctypes.c_int
_lib.eodabe_complex_workspace_size.argtypes = [_vp, _i64, _i64, _i64]
_lib.eodabe_complex_workspace_size.restype = _sz
_lib.eodabe_factor_complex.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_double, _vp, _sz,
                                       _vp, _vp, _vp, _i64, ctypes.POINTER(Info)]
_lib.eodabe_factor_complex.restype = ctypes.c_int
_lib.eodabe_factor_noalloc.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_double,
                                       _vp, _vp, _vp, _i64, ctypes.POINTER(Info)]
_lib.eodabe_factor_noalloc.restype = ctypes.c_int
_lib.eodabe_basis.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_double, _vp, _sz, _vp, _i64,
                              ctypes.POINTER(ctypes.c_double), _i64, ctypes.POINTER(Info)]
_lib.eodabe_basis.restype = ctypes.c_int
_lib.eodabe_strerror.argtypes = [ctypes.c_int]
_lib.eodabe_strerror.restype = ctypes.c_char_p
_lib.eodabe_last_hip_error.argtypes = [_vp]
_lib.eodabe_last_hip_error.restype = ctypes.c_int
_lib.eodabe_philox.argtypes = [_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint32, _i64, _vp]
_lib.eodabe_philox.restype = ctypes.c_int
_lib.eodabe_omega.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i64, _i64, _vp]
_lib.eodabe_omega.restype = ctypes.c_int
_lib.eodabe_sketch_workspace_size.argtypes = [_vp, _i64, _i64, _i64]
_lib.eodabe_sketch_workspace_size.restype = _sz
_lib.eodabe_sketch.argtypes = [_vp, _vp, _i64, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _sz]
_lib.eodabe_sketch.restype = ctypes.c_int
_lib.eodabe_batched_workspace_size.argtypes = [_vp, ctypes.c_int]
_lib.eodabe_batched_workspace_size.restype = _sz
_batched_args = [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _sz, _vp, ctypes.c_int64, _vp, _vp]
_lib.eodabe_factor_batched.argtypes = _batched_args + [_vp, _vp, _vp]
_lib.eodabe_factor_batched.restype = ctypes.c_int
_lib.eodabe_tune_batched.argtypes = _batched_args + [_vp]
_lib.eodabe_tune_batched.restype = ctypes.c_int
_lib.eodabe_mlp_param_count.argtypes = []
_lib.eodabe_mlp_param_count.restype = ctypes.c_int64
_lib.eodabe_mlp_workspace_size.argtypes = [ctypes.c_int]
_lib.eodabe_mlp_workspace_size.restype = _sz
_lib.eodabe_mlp_forward.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp, _vp, _sz]
_lib.eodabe_mlp_forward.restype = ctypes.c_int
_lib.eodabe_mlp_grad.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _sz, ctypes.POINTER(ctypes.c_double)]
_lib.eodabe_mlp_grad.restype = ctypes.c_int
_lib.eodabe_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_int]
_lib.eodabe_mlp_adam.restype = ctypes.c_int
_lib.eodabe_mlp_features.argtypes = [_vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _vp]
_lib.eodabe_mlp_features.restype = ctypes.c_int
_lib.eodabe_set_predictor.argtypes = [_vp, _vp, ctypes.c_double]
_lib.eodabe_set_predictor.restype = ctypes.c_int
_lib.eodabe_last_prediction.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
_lib.eodabe_last_prediction.restype = ctypes.c_int
_lib.eodabe_profile.argtypes = [_vp, ctypes.c_int]
_lib.eodabe_profile.restype = ctypes.c_int
_lib.eodabe_profile_read.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
_lib.eodabe_profile_read.restype = ctypes.c_int


class EodAbeError(RuntimeError):
    def __init__(self, status: int, where: str, hip: int = 0):
        msg = _lib.eodabe_strerror(status).decode()
        super().__init__(f"{where}: {msg} (status {status}" + (f", hip error {hip})" if hip else ")"))
        self.status = status


def strerror(status: int) -> str:
    return _lib.eodabe_strerror(status).decode()


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float32:
        return F32
    if t == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t} (float32 or float64)")


class Context:
    """One eodabe_ctx (bound to a stream and a set of options)."""

    def __init__(self, block: int = 32, power_iters: int = 0, seed: int = 0,
                 dtype: torch.dtype = torch.float32, sketch: int = SKETCH_NATIVE,
                 blocks_per_sync: int = 0, stream: torch.cuda.Stream | None = None,
                 host_only: bool = False):
        o = Opts()
        _lib.eodabe_default_opts(ctypes.byref(o))
        o.block, o.power_iters, o.seed = block, power_iters, seed & (2 ** 64 - 1)
        o.a_dtype, o.sketch_dtype, o.blocks_per_sync = _dtype_code(dtype), sketch, blocks_per_sync
        s = None if host_only else (stream if stream is not None else torch.cuda.current_stream())
        o.stream = s.cuda_stream if s is not None else None
        self.opts, self.dtype, self.stream = o, dtype, s
        h = _vp()
        create = _lib.eodabe_create_host if host_only else _lib.eodabe_create
        st = create(ctypes.byref(h), ctypes.byref(o))
        if st != EODABE_OK:
            raise EodAbeError(st, "eodabe_create_host" if host_only else "eodabe_create")
        self.h = h

    def set_predictor(self, params: torch.Tensor | None, margin: float = 0.1):
        """eodabe_set_predictor: attach (or detach with None) the learned warm
        start; the tensor is kept alive by the context.  Size workspaces
        afterwards (they depend on it)."""
        if params is not None:
            if params.dtype != torch.float32 or not params.is_cuda or not params.is_contiguous() \
                    or params.numel() != _lib.eodabe_mlp_param_count():
                raise EodAbeError(EODABE_EINVAL, "set_predictor: contiguous FP32 device parameters expected")
        self._check(_lib.eodabe_set_predictor(self.h, params.data_ptr() if params is not None else None,
                                              float(margin)), "eodabe_set_predictor")
        self._pred = params

    def last_prediction(self):
        """eodabe_last_prediction -> (d0, log(1+rank) head, 0.9-quantile head, used)."""
        d0, y0, y1, used = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        self._check(_lib.eodabe_last_prediction(self.h, ctypes.byref(d0), ctypes.byref(y0), ctypes.byref(y1),
                                                ctypes.byref(used)), "eodabe_last_prediction")
        return int(d0.value), float(y0.value), float(y1.value), int(used.value)

    def close(self):
        if getattr(self, "h", None):
            _lib.eodabe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, where: str):
        if st < 0:
            raise EodAbeError(st, where, _lib.eodabe_last_hip_error(self.h))
        return st

    def profile(self, enable: bool = True):
        """eodabe_profile: start (or stop) live HIP-event timing; resets totals."""
        self._check(_lib.eodabe_profile(self.h, int(enable)), "eodabe_profile")

    def profile_read(self, kind: int):
        """eodabe_profile_read -> (total_ms, launches, algorithmic_bytes)."""
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self._check(_lib.eodabe_profile_read(self.h, kind, ctypes.byref(ms), ctypes.byref(n),
                                             ctypes.byref(by)), "eodabe_profile_read")
        return ms.value, n.value, by.value

    def workspace_size(self, m: int, n: int, r_cap: int = 0) -> int:
        return int(_lib.eodabe_workspace_size(self.h, m, n, r_cap))

    def workspace(self, m: int, n: int, r_cap: int = 0) -> torch.Tensor:
        nb = self.workspace_size(m, n, r_cap)
        if nb == 0:
            raise EodAbeError(EODABE_EINVAL, "eodabe_workspace_size")
        return torch.empty(nb, dtype=torch.uint8, device="cuda")


class Factorization:
    """Result of factor(): A ~= U D Vt with U m x r (columns orthonormal), D
    r x r upper triangular and Vt r x n, views into the output buffers
    (Ut r_cap x m, core, Vt r_cap x n).  The views are made on first access:
    each costs the host microseconds, and back-to-back calls that only read
    the rank would otherwise keep the GPU waiting for them."""
    __slots__ = ("_bufs", "_views", "rank", "blocks", "eps", "norm_a", "status", "flags", "relres_est")

    def __init__(self, bufs, rank: int, blocks: int, eps: float, norm_a: float, status: int, flags: int,
                 relres_est: float = 0.0):
        self._bufs = bufs                  # (Ut, core, Vt) output buffers
        self._views = None
        self.rank = rank
        self.blocks = blocks
        self.eps = eps
        self.norm_a = norm_a
        self.status = status
        self.flags = flags
        self.relres_est = relres_est       # |T(l,l)| / ||A||_F at the stopping column (0: no stop)

    def _view(self, k: int) -> torch.Tensor:
        if self._views is None:
            Ut, core, Vt = self._bufs
            r = self.rank
            self._views = (Ut[:r].T, core[:r, :r], Vt[:r])
        return self._views[k]

    @property
    def U(self) -> torch.Tensor:
        return self._view(0)

    @property
    def D(self) -> torch.Tensor:
        return self._view(1)

    @property
    def Vt(self) -> torch.Tensor:
        return self._view(2)

    def __repr__(self) -> str:
        return (f"Factorization(rank={self.rank}, blocks={self.blocks}, eps={self.eps:g}, "
                f"norm_a={self.norm_a:g}, status={self.status}, flags={self.flags})")


def _check_matrix(A: torch.Tensor, dtype: torch.dtype):
    if not A.is_cuda or A.dim() != 2:
        raise ValueError("A must be a 2-D CUDA (HIP) tensor")
    if A.dtype != dtype:
        raise TypeError(f"A has dtype {A.dtype}, context expects {dtype}")
    if A.stride(1) != 1:
        raise ValueError("A must be row-major (stride(1) == 1)")


def alloc_outputs(A: torch.Tensor, r_cap: int = 0):
    """Caller-owned output buffers (Ut, core, Vt) for eodabe_factor."""
    m, n = A.shape
    rc = r_cap or min(m, n)
    return (torch.empty((max(rc, 1), m), dtype=A.dtype, device=A.device),
            torch.zeros((max(rc, 1), max(rc, 1)), dtype=A.dtype, device=A.device),
            torch.empty((max(rc, 1), n), dtype=A.dtype, device=A.device))


def factor(A: torch.Tensor, tol: float, ctx: Context | None = None, r_cap: int = 0,
           ws: torch.Tensor | None = None, out=None, **ctx_kw) -> Factorization:
    """eodabe_factor: A ~= U D V^T with the adaptive rank (Alg. 2 around Alg. 1)."""
    ctx = ctx or Context(**{"dtype": A.dtype, **ctx_kw})
    _check_matrix(A, ctx.dtype)
    m, n = A.shape
    rc = r_cap or min(m, n)
    if ws is None:
        ws = ctx.workspace(m, n, rc)
    Ut, core, Vt = out if out is not None else alloc_outputs(A, rc)
    lda = A.stride(0) if m > 1 else max(n, 1)
    if _fastcall is not None:
        st, r, blocks, flags, norm_a, eps, relres = _fastcall.factor(
            ctx.h.value if ctx.h is not None else 0, A.data_ptr(), m, n, lda, float(tol), ws.data_ptr(),
            ws.numel(), Ut.data_ptr(), core.data_ptr(), Vt.data_ptr(), rc)
        ctx._check(st, "eodabe_factor")
        return Factorization((Ut, core, Vt), r, blocks, eps, norm_a, st, flags, relres)
    info = Info()
    st = _lib.eodabe_factor(ctx.h, A.data_ptr(), m, n, lda, float(tol), ws.data_ptr(), ws.numel(),
                            Ut.data_ptr(), core.data_ptr(), Vt.data_ptr(), rc, ctypes.byref(info))
    ctx._check(st, "eodabe_factor")
    r = int(info.rank)
    return Factorization((Ut, core, Vt), r, int(info.blocks), float(info.eps), float(info.norm_a), st,
                         int(info.status_flags), float(info.relres_est))


def factor_complex(A: torch.Tensor, tol: float, ctx: Context | None = None, r_cap: int = 0,
                   **ctx_kw) -> Factorization:
    """eodabe_factor_complex: A ~= U D V^H for complex64 / complex128 A.
    Returns U (m x r), D (r x r) and Vt = V^H (r x n) views."""
    if A.dtype not in (torch.complex64, torch.complex128) or A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D complex64 or complex128 CUDA tensor")
    real = torch.float32 if A.dtype == torch.complex64 else torch.float64
    ctx = ctx or Context(**{"dtype": real, **ctx_kw})
    if ctx.dtype != real:
        raise ValueError("context dtype must be the real type of A")
    if A.stride(1) != 1:
        A = A.contiguous()
    m, n = A.shape
    rc = r_cap or min(m, n)
    wsz = _lib.eodabe_complex_workspace_size(ctx.h, m, n, rc)
    if wsz == 0:
        raise EodAbeError(EODABE_EINVAL, "eodabe_complex_workspace_size", 0)
    ws = torch.empty(wsz, dtype=torch.uint8, device=A.device)
    Ut = torch.empty((max(rc, 1), m), dtype=A.dtype, device=A.device)
    core = torch.zeros((max(rc, 1), max(rc, 1)), dtype=A.dtype, device=A.device)
    Vt = torch.empty((max(rc, 1), n), dtype=A.dtype, device=A.device)
    info = Info()
    lda = A.stride(0) if m > 1 else max(n, 1)
    st = _lib.eodabe_factor_complex(ctx.h, A.data_ptr(), m, n, lda, float(tol), ws.data_ptr(), wsz,
                                    Ut.data_ptr(), core.data_ptr(), Vt.data_ptr(), rc, ctypes.byref(info))
    ctx._check(st, "eodabe_factor_complex")
    r = int(info.rank)
    return Factorization((Ut, core, Vt), r, int(info.blocks), float(info.eps), float(info.norm_a), st,
                         int(info.status_flags), float(info.relres_est))


def factor_noalloc(A: torch.Tensor, tol: float, ctx: Context, out, r_cap: int = 0) -> Factorization:
    """eodabe_factor_noalloc: eodabe_factor with the library's static device
    scratch as workspace.  The caller passes the outputs (Ut, core, Vt as
    alloc_outputs returns them); nothing is allocated on the device here."""
    _check_matrix(A, ctx.dtype)
    m, n = A.shape
    rc = r_cap or min(m, n)
    Ut, core, Vt = out
    info = Info()
    lda = A.stride(0) if m > 1 else max(n, 1)
    st = _lib.eodabe_factor_noalloc(ctx.h, A.data_ptr(), m, n, lda, float(tol), Ut.data_ptr(),
                                    core.data_ptr(), Vt.data_ptr(), rc, ctypes.byref(info))
    ctx._check(st, "eodabe_factor_noalloc")
    r = int(info.rank)
    return Factorization((Ut, core, Vt), r, int(info.blocks), float(info.eps), float(info.norm_a), st,
                         int(info.status_flags), float(info.relres_est))


@dataclass
class CompressedImage:
    info: ImageInfo
    factors: list          # per channel (U m x r, D r x r, Vt r x n) views into the pool
    recon: torch.Tensor    # channels x h x w reconstruction U D V^T
    pool: torch.Tensor


def compress_image(img: torch.Tensor, tol: float, ctx: Context | None = None, **ctx_kw) -> CompressedImage:
    """eodabe_compress_image: factor every channel of a channels x h x w
    FP32 image, reconstruct it and report PSNR, SSIM, RelErr and storage."""
    ctx = ctx or Context(**{"dtype": torch.float32, **ctx_kw})
    if img.dim() != 3 or img.dtype != torch.float32 or not img.is_cuda:
        raise ValueError("img must be a channels x h x w float32 CUDA tensor")
    img = img.contiguous()
    c, h, w = img.shape
    rc = min(h, w)
    per = rc * (h + rc + w)
    pool = torch.empty(c * per, dtype=torch.float32, device=img.device)
    recon = torch.empty_like(img)
    wsz = _lib.eodabe_image_workspace_size(ctx.h, c, h, w)
    if wsz == 0:
        raise EodAbeError(EODABE_EINVAL, "eodabe_image_workspace_size", 0)
    ws = torch.empty(wsz, dtype=torch.uint8, device=img.device)
    info = ImageInfo()
    st = _lib.eodabe_compress_image(ctx.h, img.data_ptr(), c, h, w, float(tol), ws.data_ptr(), wsz,
                                    pool.data_ptr(), pool.numel(), recon.data_ptr(), ctypes.byref(info))
    ctx._check(st, "eodabe_compress_image")
    facs = []
    for ch in range(c):
        base = pool[ch * per:(ch + 1) * per]
        r = int(info.rank[ch])
        Ut = base[:rc * h].view(rc, h)
        core = base[rc * h:rc * (h + rc)].view(rc, rc)
        Vt = base[rc * (h + rc):].view(rc, w)
        facs.append((Ut[:r].T, core[:r, :r], Vt[:r]))
    return CompressedImage(info, facs, recon, pool)


def features(f: Factorization, ctx: Context | None = None) -> torch.Tensor:
    """eodabe_features: rows of U_hat D_hat (m x r FP32) from a factorization
    returned by factor()."""
    ctx = ctx or Context(dtype=torch.float32)
    m, r = f.U.shape
    F = torch.empty((m, max(r, 1)), dtype=torch.float32, device=f.U.device)
    Ut = f.U.T                      # rows of the Ut output buffer (stride m)
    st = _lib.eodabe_features(ctx.h, Ut.data_ptr(), f.D.data_ptr(), m, r, f.D.stride(0) if r else 0,
                              F.data_ptr(), F.stride(0))
    ctx._check(st, "eodabe_features")
    return F[:, :r]


def knn_cv(F: torch.Tensor, labels: torch.Tensor, fold: torch.Tensor, k: int, nclass: int,
           ctx: Context | None = None):
    """eodabe_knn_cv: KNN classification of every point by the points of the
    other folds.  Returns (pred (device int32), confusion (numpy), OA)."""
    import numpy as np
    ctx = ctx or Context(dtype=torch.float32)
    if F.dtype != torch.float32 or F.stride(1) != 1:
        raise ValueError("F must be float32 with unit column stride")
    m, d = F.shape
    pred = torch.empty(m, dtype=torch.int32, device=F.device)
    wsz = _lib.eodabe_knn_workspace_size(nclass)
    ws = torch.empty(max(wsz, 1), dtype=torch.uint8, device=F.device)
    conf = np.zeros((nclass, nclass), dtype=np.int64)
    oa = ctypes.c_double()
    st = _lib.eodabe_knn_cv(ctx.h, F.data_ptr(), m, d, F.stride(0), labels.data_ptr(), fold.data_ptr(), k, nclass,
                            pred.data_ptr(), ws.data_ptr(), wsz, conf.ctypes.data, ctypes.byref(oa))
    ctx._check(st, "eodabe_knn_cv")
    return pred, conf, float(oa.value)


def basis(A: torch.Tensor, tol: float, ctx: Context | None = None, r_cap: int = 0,
          ws: torch.Tensor | None = None, **ctx_kw):
    """eodabe_basis: Alg. 1 only.  Returns (Q (m x r), diagT (numpy), info)."""
    import numpy as np
    ctx = ctx or Context(**{"dtype": A.dtype, **ctx_kw})
    _check_matrix(A, ctx.dtype)
    m, n = A.shape
    rc = r_cap or min(m, n)
    if ws is None:
        ws = ctx.workspace(m, n, rc)
    Qt = torch.empty((max(rc, 1), m), dtype=A.dtype, device=A.device)
    diag = np.zeros(max(n, 1), dtype=np.float64)
    info = Info()
    lda = A.stride(0) if m > 1 else max(n, 1)
    st = _lib.eodabe_basis(ctx.h, A.data_ptr(), m, n, lda, float(tol), ws.data_ptr(), ws.numel(),
                           Qt.data_ptr(), rc, diag.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           diag.size, ctypes.byref(info))
    ctx._check(st, "eodabe_basis")
    r = int(info.rank)
    return Qt[:r].T, diag[: min(r + 1, n)], info


def philox(ctx: Context, seed: int, ctr0: int, ctr1: int, ctr2: int, count: int) -> torch.Tensor:
    """eodabe_philox: raw Philox4x32-10 words, shape (count, 4), int32 view of uint32."""
    out = torch.empty((max(count, 1), 4), dtype=torch.int32, device="cuda")
    ctx._check(_lib.eodabe_philox(ctx.h, seed & (2 ** 64 - 1), ctr0, ctr1, ctr2, count,
                                  out.data_ptr()), "eodabe_philox")
    return out[:count]


def omega(ctx: Context, n: int, col0: int, ncols: int, dtype: torch.dtype = torch.float32,
          ldo: int | None = None) -> torch.Tensor:
    """eodabe_omega: columns col0.. of the Gaussian test matrix, returned as (n, ncols)."""
    ldo = ldo or n
    out = torch.empty((max(ncols, 1), max(ldo, 1)), dtype=dtype, device="cuda")
    ctx._check(_lib.eodabe_omega(ctx.h, _dtype_code(dtype), n, col0, ncols, ldo, out.data_ptr()),
               "eodabe_omega")
    return out[:ncols, :n].T


def sketch(ctx: Context, A: torch.Tensor, col0: int, ncols: int) -> torch.Tensor:
    """eodabe_sketch: Y = A Omega(:, col0:col0+ncols), returned as (m, ncols)."""
    _check_matrix(A, ctx.dtype)
    m, n = A.shape
    nb = int(_lib.eodabe_sketch_workspace_size(ctx.h, m, n, ncols))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    Yt = torch.empty((max(ncols, 1), max(m, 1)), dtype=A.dtype, device="cuda")
    lda = A.stride(0) if m > 1 else max(n, 1)
    ctx._check(_lib.eodabe_sketch(ctx.h, A.data_ptr(), m, n, lda, col0, ncols, Yt.data_ptr(),
                                  max(m, 1), ws.data_ptr(), ws.numel()), "eodabe_sketch")
    return Yt[:ncols, :m].T


# ---------------------------------------------------------------- batched tiles
TILE_STATUS = {0: "ok", 1: "rank above the in-kernel cap (finished by the single-matrix path)",
               2: "non-finite", 3: "rank above r_cap"}


class Batch:
    """Argument arrays, output pool and workspace of eodabe_factor_batched
    for a fixed list of FP32 tiles (kept alive between calls)."""

    def __init__(self, ctx: Context, tiles, r_caps=None):
        import numpy as np
        self.ctx, self.tiles = ctx, list(tiles)
        nt = len(self.tiles)
        for T in self.tiles:
            _check_matrix(T, torch.float32)
        self.m = np.array([T.shape[0] for T in self.tiles], dtype=np.int64)
        self.n = np.array([T.shape[1] for T in self.tiles], dtype=np.int64)
        self.lda = np.array([T.stride(0) if T.shape[0] > 1 else max(T.shape[1], 1) for T in self.tiles],
                            dtype=np.int64)
        self.ptrs = (ctypes.c_void_p * max(nt, 1))(*[T.data_ptr() for T in self.tiles])
        rc = np.minimum(self.m, self.n) if r_caps is None else np.asarray(r_caps, dtype=np.int64)
        self.r_caps = rc.astype(np.int64)
        sizes = self.r_caps * self.m + self.r_caps * self.r_caps + self.r_caps * self.n
        self.offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if nt else np.zeros(0, np.int64)
        dev = self.tiles[0].device if nt else torch.device("cuda")
        self.pool = torch.zeros(int(sizes.sum()) if nt else 1, dtype=torch.float32, device=dev)
        nb = int(_lib.eodabe_batched_workspace_size(ctx.h, nt))
        self.ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        self.ranks = np.zeros(nt, dtype=np.int64)
        self.status = np.zeros(nt, dtype=np.int32)
        self.blocks = np.zeros(nt, dtype=np.int32)

    def _args(self, tol):
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        return [self.ctx.h, len(self.tiles), ctypes.cast(self.ptrs, ctypes.c_void_p), p(self.m), p(self.n),
                p(self.lda), float(tol), self.ws.data_ptr(), self.ws.numel(), self.pool.data_ptr(),
                self.pool.numel(), p(self.offsets), p(self.r_caps)]

    def run(self, tol: float):
        """eodabe_factor_batched; ranks, status and block widths land in
        self.ranks, self.status, self.blocks."""
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        st = _lib.eodabe_factor_batched(*self._args(tol), p(self.ranks), p(self.status), p(self.blocks))
        self.ctx._check(st, "eodabe_factor_batched")
        return self

    def tune(self, tol: float):
        """eodabe_tune_batched: block width per tile-size bucket (kept in ctx)."""
        import numpy as np
        chosen = np.zeros(4, dtype=np.int32)
        st = _lib.eodabe_tune_batched(*self._args(tol), chosen.ctypes.data_as(ctypes.c_void_p))
        self.ctx._check(st, "eodabe_tune_batched")
        return chosen

    def result(self, t: int):
        """(U (m x r), D (r x r), Vt (r x n), rank, status) of tile t."""
        m, n, rc, off = int(self.m[t]), int(self.n[t]), int(self.r_caps[t]), int(self.offsets[t])
        r = int(self.ranks[t])
        Ut = self.pool[off: off + rc * m].view(rc, m)
        core = self.pool[off + rc * m: off + rc * m + rc * rc].view(rc, rc)
        Vt = self.pool[off + rc * m + rc * rc: off + rc * m + rc * rc + rc * n].view(rc, n)
        return Ut[:r].T, core[:r, :r], Vt[:r], r, int(self.status[t])
