"""ctypes binding of librklt (include/rklt.h): argument marshalling only.

Every step of the codec runs in the HIP library; this module converts
Python values and torch tensors (device memory and streams) into the C
structures and pointers the ABI takes, and raises RkltError on a non-zero
status.  It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RKLT_LIBRARY may name another build of the same library (tuning experiments);
# by default the in-tree build is loaded.
LIB_PATH = os.environ.get("RKLT_LIBRARY") or os.path.join(_HERE, "librklt.so")

MAX_N = 32
ORTHOGONAL = 1
ADDS_ONLY = 2

OK, E_INVAL, E_SINGULAR, E_RANGE, E_NOMEM, E_HIP, E_STATE = range(7)
_STATUS = {0: "OK", 1: "E_INVAL", 2: "E_SINGULAR", 3: "E_RANGE", 4: "E_NOMEM", 5: "E_HIP",
           6: "E_STATE"}


class RkltError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Transform(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("flags", C.c_int32), ("rho", C.c_double), ("alpha", C.c_double),
        ("K", C.c_double * (MAX_N * MAX_N)), ("T", C.c_int32 * (MAX_N * MAX_N)),
        ("d", C.c_int64 * MAX_N), ("s", C.c_double * MAX_N),
        ("G", C.c_double * (MAX_N * MAX_N)),
        ("max_abs", C.c_int32), ("max_row_l1", C.c_int32),
    ]


class Image(C.Structure):
    _fields_ = [
        ("src", C.c_void_p), ("dst", C.c_void_p), ("coef_out", C.c_void_p),
        ("scaled_out", C.c_void_p),
        ("H", C.c_int32), ("W", C.c_int32), ("pitch_src", C.c_int32), ("pitch_dst", C.c_int32),
        ("transform_id", C.c_int32), ("r", C.c_int32), ("level_shift", C.c_int32),
        ("reserved", C.c_int32),
    ]


class Result(C.Structure):
    _fields_ = [("sse", C.c_uint64), ("mse", C.c_float), ("psnr_db", C.c_float),
                ("acc", C.c_uint64), ("tiles", C.c_uint32), ("reserved", C.c_uint32)]


RESULT_BYTES = C.sizeof(Result)  # 32


class Measures(C.Structure):
    _fields_ = [("coding_gain_db", C.c_double), ("coding_gain_tt_db", C.c_double),
                ("efficiency_pct", C.c_double), ("mse", C.c_double), ("error_energy", C.c_double)]


class DesignEntry(C.Structure):
    _fields_ = [("rho_first", C.c_double), ("rho_last", C.c_double), ("T", C.c_int32 * (MAX_N * MAX_N))]


class Tuning(C.Structure):
    _fields_ = [("wg_threads", C.c_int32), ("blocks_per_thread", C.c_int32),
                ("grid_wgs", C.c_int32), ("schedule", C.c_int32)]


def _load():
    # torch brings its own HIP runtime (same soname as /opt/rocm's).  Loading
    # torch first makes this library bind to that runtime, so that torch's
    # device pointers and stream handles are valid in both.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_2111_14239_amd.build_lib)")
    lib = C.CDLL(LIB_PATH)
    st = C.c_int
    vp = C.c_void_p
    sig = {
        "rklt_last_error": (C.c_char_p, []),
        "rklt_build_transform": (st, [C.c_int32, C.c_double, C.c_double, C.POINTER(Transform)]),
        "rklt_zigzag": (st, [C.c_int32, C.POINTER(C.c_int32)]),
        "rklt_ctx_create": (st, [C.c_int32, C.POINTER(vp)]),
        "rklt_ctx_destroy": (st, [vp]),
        "rklt_ctx_add_transform": (st, [vp, C.POINTER(Transform), C.POINTER(C.c_int32)]),
        "rklt_codec": (st, [vp, C.POINTER(Image), vp, C.POINTER(Tuning), vp]),
        "rklt_plan_create": (st, [vp, C.POINTER(Image), C.c_int32, C.POINTER(Tuning), C.POINTER(vp)]),
        "rklt_plan_run": (st, [vp, vp, vp]),
        "rklt_plan_destroy": (st, [vp]),
        "rklt_plan_info": (st, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
        "rklt_copy_bytes": (st, [vp, vp, C.c_size_t, vp]),
        "rklt_plan_launches": (st, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32 * 7)]),
        "rklt_plan_update": (st, [vp, C.POINTER(Image), C.c_int32, vp]),
        "rklt_ctx_transform_exact": (st, [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
        "rklt_ctx_mfma_form": (st, [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
        "rklt_plan_autotune": (st, [vp, vp, C.c_int32, vp, C.POINTER(Tuning)]),
        "rklt_plan_mssim": (st, [vp, vp, vp]),
        "rklt_klt_matrix": (st, [C.c_int32, C.c_double, C.POINTER(C.c_double)]),
        "rklt_dct_matrix": (st, [C.c_int32, C.POINTER(C.c_double)]),
        "rklt_ctx_add_float_transform": (st, [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "rklt_ctx_add_quantizer": (st, [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "rklt_transform_measures": (st, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                         C.POINTER(Measures)]),
        "rklt_algorithm1": (st, [C.c_int32, C.c_double, C.c_double, C.POINTER(DesignEntry), C.c_int32,
                                 C.POINTER(C.c_int32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("rklt_last_error", "rklt_build_transform", "rklt_zigzag", "rklt_ctx_create",
            "rklt_ctx_destroy", "rklt_ctx_add_transform", "rklt_codec", "rklt_plan_create",
            "rklt_plan_run", "rklt_plan_destroy", "rklt_plan_info", "rklt_copy_bytes",
            "rklt_plan_launches", "rklt_ctx_transform_exact", "rklt_plan_update", "rklt_ctx_mfma_form",
            "rklt_plan_autotune", "rklt_plan_mssim", "rklt_klt_matrix", "rklt_dct_matrix",
            "rklt_ctx_add_float_transform", "rklt_ctx_add_quantizer", "rklt_transform_measures",
            "rklt_algorithm1")


def lib():
    return _lib


def _check(status: int):
    if status != OK:
        raise RkltError(status, _lib.rklt_last_error().decode())


# --------------------------------------------------------------------------
# host-side transform design
# --------------------------------------------------------------------------

@dataclass
class TransformInfo:
    """A transform built by the library (host FP64), as numpy arrays."""
    N: int
    rho: float
    alpha: float
    K: np.ndarray
    T: np.ndarray
    d: np.ndarray
    s: np.ndarray
    G: np.ndarray
    flags: int
    max_abs: int
    max_row_l1: int
    raw: Transform

    @property
    def orthogonal(self) -> bool:
        return bool(self.flags & ORTHOGONAL)

    @property
    def adds_only(self) -> bool:
        return bool(self.flags & ADDS_ONLY)


def build_transform(N: int, rho: float, alpha: float) -> TransformInfo:
    """rklt_build_transform: T = round(alpha K_rho) and its derived tables."""
    t = Transform()
    _check(_lib.rklt_build_transform(int(N), float(rho), float(alpha), C.byref(t)))
    n2 = N * N
    return TransformInfo(
        N=N, rho=t.rho, alpha=t.alpha,
        K=np.ctypeslib.as_array(t.K)[:n2].reshape(N, N).copy(),
        T=np.ctypeslib.as_array(t.T)[:n2].reshape(N, N).astype(np.int64),
        d=np.ctypeslib.as_array(t.d)[:N].copy(),
        s=np.ctypeslib.as_array(t.s)[:N].copy(),
        G=np.ctypeslib.as_array(t.G)[:n2].reshape(N, N).copy(),
        flags=t.flags, max_abs=t.max_abs, max_row_l1=t.max_row_l1, raw=t)


def klt_matrix(N: int, rho: float) -> np.ndarray:
    """rklt_klt_matrix: the exact KLT K_rho (rows the basis vectors), FP64."""
    buf = (C.c_double * (N * N))()
    _check(_lib.rklt_klt_matrix(int(N), float(rho), buf))
    return np.ctypeslib.as_array(buf).reshape(N, N).copy()


def dct_matrix(N: int) -> np.ndarray:
    """rklt_dct_matrix: the orthonormal DCT-II (rows the basis vectors), FP64."""
    buf = (C.c_double * (N * N))()
    _check(_lib.rklt_dct_matrix(int(N), buf))
    return np.ctypeslib.as_array(buf).reshape(N, N).copy()


def transform_measures(That, ref, rho: float) -> dict:
    """rklt_transform_measures: Cg (two readings), eta, MSE and epsilon of
    T_hat against `ref` for the Markov-1 model of correlation rho (§3.1)."""
    That = np.ascontiguousarray(That, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    if That.shape != ref.shape or That.ndim != 2 or That.shape[0] != That.shape[1]:
        raise ValueError("transform_measures: two square matrices of one shape")
    m = Measures()
    P = C.POINTER(C.c_double)
    _check(_lib.rklt_transform_measures(int(That.shape[0]), That.ctypes.data_as(P), ref.ctypes.data_as(P),
                                        float(rho), C.byref(m)))
    return {f: float(getattr(m, f)) for f, _ in Measures._fields_}


def algorithm1(N: int, alpha: float, step: float) -> list[tuple[float, float, np.ndarray]]:
    """rklt_algorithm1: the distinct round(alpha K_rho) over the rho grid
    step, 2 step, ...: (first rho, last rho, T) per matrix."""
    n = C.c_int32()
    _check(_lib.rklt_algorithm1(int(N), float(alpha), float(step), None, 0, C.byref(n)))
    arr = (DesignEntry * max(n.value, 1))()
    _check(_lib.rklt_algorithm1(int(N), float(alpha), float(step), arr, n.value, C.byref(n)))
    return [(e.rho_first, e.rho_last, np.ctypeslib.as_array(e.T)[:N * N].reshape(N, N).astype(np.int64))
            for e in arr[:n.value]]


def zigzag(N: int) -> np.ndarray:
    """rklt_zigzag: natural index i*N + j of each zig-zag position."""
    buf = (C.c_int32 * (N * N))()
    _check(_lib.rklt_zigzag(int(N), buf))
    return np.ctypeslib.as_array(buf).copy()


# --------------------------------------------------------------------------
# device side (torch tensors supply memory and streams)
# --------------------------------------------------------------------------

def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    h = int(stream.cuda_stream)
    return h or None


def make_tuning(wg_threads=0, blocks_per_thread=0, grid_wgs=0, schedule=0):
    return Tuning(int(wg_threads), int(blocks_per_thread), int(grid_wgs), int(schedule))


ROW_ALIGN = 128


def empty_pitched(H: int, W: int, device="cuda"):
    """An uninitialised H x W uint8 device image whose rows start on 128-byte
    boundaries (pitch = W rounded up to 128): the layout the kernels read and
    write fastest, since no cache line of a row is shared with the next.
    Any pitch that is a multiple of 8 is accepted by the library."""
    import torch
    P = (int(W) + ROW_ALIGN - 1) // ROW_ALIGN * ROW_ALIGN
    return torch.empty((int(H), P), dtype=torch.uint8, device=device)[:, :int(W)]


def to_pitched(img, device="cuda"):
    """Copy a 2D uint8 array (numpy or torch) into a new pitched device image."""
    import torch
    t = torch.as_tensor(img)
    out = empty_pitched(t.shape[0], t.shape[1], device)
    out.copy_(t, non_blocking=False)
    return out


def new_results(n: int, device="cuda"):
    """A zero-filled device array of n rklt_result (uint8 tensor of n*32 bytes)."""
    import torch
    return torch.zeros(n * RESULT_BYTES, dtype=torch.uint8, device=device)


def read_results(res_tensor) -> list[dict]:
    """Copy a results array to the host and decode it."""
    raw = res_tensor.detach().cpu().numpy().tobytes()
    n = len(raw) // RESULT_BYTES
    arr = (Result * n).from_buffer_copy(raw)
    return [dict(sse=int(r.sse), mse=float(r.mse), psnr_db=float(r.psnr_db), tiles=int(r.tiles),
                 acc=int(r.acc)) for r in arr]


def image_desc(src, transform_id: int, r: int, dst=None, level_shift: int = 128,
               coef_out=None, scaled_out=None, H=None, W=None, pitch_src=None, pitch_dst=None) -> Image:
    """Describe one device image (a 2D uint8 tensor, or a flat one with H/W/pitches)."""
    if H is None:
        H, W = int(src.shape[0]), int(src.shape[1])
        pitch_src = int(src.stride(0))
        if dst is not None:
            pitch_dst = int(dst.stride(0))
    return Image(_ptr(src), _ptr(dst), _ptr(coef_out), _ptr(scaled_out), int(H), int(W),
                 int(pitch_src), int(pitch_dst or 0), int(transform_id), int(r), int(level_shift), 0)


class Context:
    """rklt_ctx: a device transform table on one GPU."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(_lib.rklt_ctx_create(int(device), C.byref(h)))
        self._h = h
        self.device = device
        self._ids: dict[tuple, int] = {}

    def close(self):
        if self._h:
            _lib.rklt_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def add_transform(self, t: TransformInfo) -> int:
        i = C.c_int32()
        _check(_lib.rklt_ctx_add_transform(self._h, C.byref(t.raw), C.byref(i)))
        return int(i.value)

    def transform_id(self, N: int, rho: float, alpha: float) -> int:
        """Build (host) and upload the transform for (N, rho, alpha); cached."""
        key = (int(N), float(rho), float(alpha))
        if key not in self._ids:
            self._ids[key] = self.add_transform(build_transform(N, rho, alpha))
        return self._ids[key]

    def add_float_transform(self, M) -> int:
        """rklt_ctx_add_float_transform: upload an N x N float transform
        (rows the basis vectors); returns its id."""
        M = np.ascontiguousarray(M, dtype=np.float64)
        if M.ndim != 2 or M.shape[0] != M.shape[1]:
            raise ValueError("add_float_transform: M must be square")
        i = C.c_int32()
        _check(_lib.rklt_ctx_add_float_transform(self._h, int(M.shape[0]),
                                                 M.ctypes.data_as(C.POINTER(C.c_double)), C.byref(i)))
        return int(i.value)

    def add_quantizer(self, tid: int, Q) -> int:
        """rklt_ctx_add_quantizer: id of rounded transform `tid` with the
        N x N quantisation matrix Q (Appendix A)."""
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        i = C.c_int32()
        _check(_lib.rklt_ctx_add_quantizer(self._h, int(tid), Q.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.byref(i)))
        return int(i.value)

    def float_transform_id(self, kind: str, N: int = 8, rho: float | None = None) -> int:
        """Id of a comparison transform, uploaded on first use: kind "dct"
        (orthonormal DCT-II) or "klt" (exact KLT of correlation rho)."""
        key = (kind, int(N), None if rho is None else float(rho))
        if key not in self._ids:
            if kind == "dct":
                M = dct_matrix(N)
            elif kind == "klt":
                if rho is None:
                    raise ValueError("float_transform_id: kind 'klt' needs rho")
                M = klt_matrix(N, rho)
            else:
                raise ValueError(f"float_transform_id: unknown kind {kind!r}")
            self._ids[key] = self.add_float_transform(M)
        return self._ids[key]

    def transform_exact(self, tid: int) -> tuple[bool, int]:
        """(exact, den): whether the N = 8 register kernel reconstructs exactly."""
        e, d = C.c_int32(), C.c_int64()
        _check(_lib.rklt_ctx_transform_exact(self._h, int(tid), C.byref(e), C.byref(d)))
        return bool(e.value), int(d.value)

    def mfma_form(self, tid: int, r: int) -> int:
        """Inverse form of the N = 8 matrix-core kernel for (transform, r):
        1 or 3 exact, 2 FP32, 0 not on that kernel."""
        f = C.c_int32()
        _check(_lib.rklt_ctx_mfma_form(self._h, int(tid), int(r), C.byref(f)))
        return int(f.value)

    def codec(self, img: Image, res_ptr: int, tuning: Tuning | None = None, stream=None):
        """rklt_codec: one image, one launch (plain path)."""
        _check(_lib.rklt_codec(self._h, C.byref(img), C.c_void_p(res_ptr),
                               C.byref(tuning) if tuning is not None else None,
                               C.c_void_p(_stream_handle(stream))))

    def plan(self, imgs: list[Image], tuning: Tuning | None = None) -> "Plan":
        return Plan(self, imgs, tuning)


class Plan:
    """rklt_plan: the device work list of a batch, run in one persistent launch."""

    def __init__(self, ctx: Context, imgs: list[Image], tuning: Tuning | None = None):
        arr = (Image * len(imgs))(*imgs)
        h = C.c_void_p()
        _check(_lib.rklt_plan_create(ctx.handle, arr, len(imgs),
                                     C.byref(tuning) if tuning is not None else None, C.byref(h)))
        self._h = h
        self.ctx = ctx
        self._refresh(len(imgs))

    def _refresh(self, n: int):
        h = self._h
        self.n = n
        tiles, grid, pixels = C.c_int64(), C.c_int32(), C.c_int64()
        _check(_lib.rklt_plan_info(h, C.byref(tiles), C.byref(grid), C.byref(pixels)))
        self.tiles, self.grid, self.pixels = int(tiles.value), int(grid.value), int(pixels.value)
        nl, per = C.c_int32(), (C.c_int32 * 7)()
        _check(_lib.rklt_plan_launches(h, C.byref(nl), per))
        self.launches = int(nl.value)
        # [panel, register N=8, matrix-core N=8, panel with a float transform,
        #  region matrix-core, region matrix-core with the quantiser,
        #  region matrix-core with a float transform]
        self.images_per_class = [int(v) for v in per]
        self.block8_images = self.images_per_class[1] + self.images_per_class[2]

    def run(self, res_ptr: int, stream=None):
        _check(_lib.rklt_plan_run(self._h, C.c_void_p(res_ptr), C.c_void_p(_stream_handle(stream))))

    def update(self, imgs: list[Image], stream=None):
        """rklt_plan_update: new images, asynchronous upload on `stream`."""
        arr = (Image * len(imgs))(*imgs)
        _check(_lib.rklt_plan_update(self._h, arr, len(imgs), C.c_void_p(_stream_handle(stream))))
        self._refresh(len(imgs))

    def autotune(self, res_ptr: int, reps: int = 10, stream=None) -> Tuning:
        """rklt_plan_autotune: time the candidate tile shapes on this plan's
        images and keep the fastest; returns the tuning kept."""
        t = Tuning()
        _check(_lib.rklt_plan_autotune(self._h, C.c_void_p(res_ptr), int(reps),
                                       C.c_void_p(_stream_handle(stream)), C.byref(t)))
        self._refresh(self.n)
        return t

    def mssim(self, out_ptr: int, stream=None):
        """rklt_plan_mssim: MSSIM of every image's reconstruction (n device
        doubles at out_ptr), after run() on the same stream."""
        _check(_lib.rklt_plan_mssim(self._h, C.c_void_p(out_ptr), C.c_void_p(_stream_handle(stream))))

    def close(self):
        if self._h:
            _lib.rklt_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_bytes(src, dst, nbytes: int, stream=None):
    """rklt_copy_bytes: the plain streaming copy used as bandwidth reference."""
    _check(_lib.rklt_copy_bytes(C.c_void_p(_ptr(src)), C.c_void_p(_ptr(dst)), int(nbytes),
                                C.c_void_p(_stream_handle(stream))))


def codec_image(ctx: Context, img, rho: float, alpha: float, r: int, level_shift: int = 128,
                N: int = 8, with_recon: bool = True, dump: bool = False, tuning=None, stream=None):
    """Convenience: code one device uint8 image (2D tensor) with the plain path.
    Returns (recon or None, results tensor, coef or None, scaled or None)."""
    import torch
    tid = ctx.transform_id(N, rho, alpha)
    dst = torch.empty_like(img) if with_recon else None
    coef = torch.empty(img.numel(), dtype=torch.int32, device=img.device) if dump else None
    scaled = torch.empty(img.numel(), dtype=torch.float32, device=img.device) if dump else None
    res = new_results(1, img.device)
    desc = image_desc(img, tid, r, dst=dst, level_shift=level_shift, coef_out=coef, scaled_out=scaled)
    ctx.codec(desc, _ptr(res), tuning, stream)
    return dst, res, coef, scaled


_default_ctx: dict = {}


def _ctx_for(device) -> Context:
    import torch
    dev = torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx not in _default_ctx:
        _default_ctx[idx] = Context(idx)
    return _default_ctx[idx]


def codec(img, rho: float, alpha: float, r: int, level_shift: int = 128, N: int = 8, ctx: Context | None = None):
    """Code one device uint8 image (2D tensor) on the plain path and wait:
    returns (reconstruction tensor, SSE, PSNR in dB)."""
    import torch
    ctx = ctx or _ctx_for(img.device)
    dst, res, _, _ = codec_image(ctx, img, rho, alpha, r, level_shift=level_shift, N=N)
    torch.cuda.current_stream(img.device).synchronize()
    out = read_results(res)[0]
    return dst, out["sse"], out["psnr_db"]


def codec_batch(images, params, ctx: Context | None = None, tuning: Tuning | None = None):
    """Code a list of device uint8 images in one batched launch per kernel
    class and wait.  params[i] = (rho, alpha, r) or (rho, alpha, r,
    level_shift, N).  Returns (reconstructions, list of result dicts)."""
    import torch
    if not images:
        return [], []
    ctx = ctx or _ctx_for(images[0].device)
    dsts, descs = [], []
    for img, p in zip(images, params):
        rho, alpha, r = p[0], p[1], p[2]
        ell = p[3] if len(p) > 3 else 128
        N = p[4] if len(p) > 4 else 8
        d = torch.empty_like(img)
        dsts.append(d)
        descs.append(image_desc(img, ctx.transform_id(N, rho, alpha), r, dst=d, level_shift=ell))
    res = new_results(len(images), images[0].device)
    plan = ctx.plan(descs, tuning)
    plan.run(_ptr(res))
    torch.cuda.current_stream(images[0].device).synchronize()
    plan.close()
    return dsts, read_results(res)
