"""Python binding of libemri.so: the MI355X (gfx950) semi-coherent EMRI track search.

Argument marshalling only.  Every step of the path runs in the library's HIP
kernels (or, for build_basis, its host C++); PyTorch supplies device memory and
the current HIP stream.  The functions mirror the C ABI in include/emri.h:

    build_sfts(x, dt, n_sft, psd)            -> Spectrogram
    build_basis(tracks, K)                   -> (f0, U, sv, box_lo, box_hi)
    score_tracks(spec, f0, U, coeffs, top_k) -> dict(stat, topk_val, topk_idx, ...)

There is no fallback: if the shared library is missing, or a call fails, an
exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemri.so")

F32, F16, C32 = 0, 1, 2
PLAIN, MIXED = 0, 1
_PRECISIONS = {"plain": PLAIN, "mixed": MIXED}
_DTYPES = {"f32": F32, "f16": F16, "c32": C32}
MAX_K = 32
MAX_TOPK = 4096

_lib = None


class EmriError(RuntimeError):
    def __init__(self, func: str, status: int, detail: str):
        super().__init__(f"{func} failed with status {status}: {detail}")
        self.status = status


class _Power(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n_seg", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("row_pitch", ctypes.c_int32), ("dtype", ctypes.c_int32), ("t_sft", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4), ("rescore_top", ctypes.c_int32)]


_vp, _i32, _i64, _dbl, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t


class _Problem(ctypes.Structure):
    _fields_ = [("power", _Power), ("f0", _vp), ("U", _vp), ("coeffs", _vp), ("n_tmpl", _i64),
                ("top_k", _i32), ("k_min", _i32), ("k_max", _i32), ("reserved", _i32),
                ("stat", _vp), ("topk_val", _vp), ("topk_idx", _vp)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("rows_per_step", _i32), ("templates_per_lane", _i32), ("precision", _i32), ("reserved", _i32 * 5)]


class _Plan(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_int64 * 24)]

class _Chain(ctypes.Structure):
    _fields_ = [("power", _Power), ("f0", _vp), ("U", _vp), ("box_lo", _vp), ("box_hi", _vp), ("coeffs", _vp),
                ("stat", _vp), ("n_walkers", _i32), ("k_min", _i32), ("k_max", _i32), ("reserved", _i32)]


class _ChirpOpts(ctypes.Structure):
    _fields_ = [("p_half", _i32), ("pad", _i32), ("f_min", ctypes.c_double), ("fdot_min", ctypes.c_double),
                ("reserved", _i32 * 4)]


class _SearchPlan(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_int64 * 40)]


SIGNATURES = {
    "build_sfts": (ctypes.c_int, [_vp, _i64, _dbl, _i32, _vp, ctypes.POINTER(_Power), _vp]),
    "build_basis": (ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "score_tracks_workspace_size": (ctypes.c_int, [ctypes.POINTER(_Power), _i32, _i64, _i32, _i32,
                                                   ctypes.POINTER(_sz)]),
    "score_tracks": (ctypes.c_int, [ctypes.POINTER(_Power), _vp, _vp, _i32, _vp, _i64, _i32, _vp, _vp, _vp,
                                    _vp, _vp, ctypes.POINTER(_Opts), _vp, _sz, _vp]),
    "score_tracks_noalloc": (ctypes.c_int, [ctypes.POINTER(_Power), _vp, _vp, _i32, _vp, _i64, _i32, _vp, _vp, _vp,
                                            _vp, _vp, ctypes.POINTER(_Opts), _vp]),
    "score_tracks_noalloc_limit": (_sz, []),
    "score_tracks_harmonics": (ctypes.c_int, [ctypes.POINTER(_Power), _vp, _vp, _i32, _vp, _i64, _i32,
                                              ctypes.POINTER(ctypes.c_double), _i32, _vp, _vp, _vp,
                                              ctypes.POINTER(_Opts), _vp, _sz, _vp]),
    "score_tracks_chirp_workspace_size": (ctypes.c_int, [ctypes.POINTER(_Power), _i32, _i64, _i32, _i32,
                                                         ctypes.POINTER(_sz)]),
    "score_tracks_chirp": (ctypes.c_int, [ctypes.POINTER(_Power), _vp, _vp, _vp, _i32, _vp, _i64, _i32, _vp, _vp,
                                          _vp, ctypes.POINTER(_ChirpOpts), _vp, _sz, _vp]),
    "score_batched_workspace_size": (ctypes.c_int, [ctypes.POINTER(_Problem), _i32, _i32, ctypes.POINTER(_sz)]),
    "score_batched_tile_options": (ctypes.c_int, [_i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "score_batched_plan": (ctypes.c_int, [ctypes.POINTER(_Problem), _i32, _i32, ctypes.POINTER(_BatchOpts), _vp,
                                          _sz, ctypes.POINTER(_Plan), _vp]),
    "score_batched_run": (ctypes.c_int, [ctypes.POINTER(_Plan), _vp]),
    "search_seed_workspace_size": (ctypes.c_int, [ctypes.POINTER(_Chain), _i32, _i32, _i32, ctypes.POINTER(_sz)]),
    "search_seed": (ctypes.c_int, [ctypes.POINTER(_Chain), _i32, _i32, _vp, _vp, _i32, ctypes.POINTER(_BatchOpts),
                                   _vp, _sz, _vp]),
    "search_workspace_size": (ctypes.c_int, [ctypes.POINTER(_Chain), _i32, _i32, ctypes.POINTER(_sz)]),
    "search_plan": (ctypes.c_int, [ctypes.POINTER(_Chain), _i32, _i32, ctypes.POINTER(_BatchOpts), _vp, _sz,
                                   ctypes.POINTER(_SearchPlan), _vp]),
    "search_generation": (ctypes.c_int, [ctypes.POINTER(_SearchPlan), _vp, _vp, _vp, _vp, _vp]),
    "search_generations": (ctypes.c_int, [ctypes.POINTER(_SearchPlan), _i32, _vp, _vp, _vp, _vp]),
    "search_best": (ctypes.c_int, [ctypes.POINTER(_SearchPlan), _vp, _vp, _vp, _vp, _vp, _vp]),
    "search_noise_moments": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "emri_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "emri_last_error": (ctypes.c_char_p, []),
}


def load():
    """Load libemri.so (built in place by paper_2510_20891_amd.build).

    PyTorch is imported first so that the library binds to the HIP runtime that
    PyTorch already uses (both carry the soname libamdhip64.so.7): one process,
    one runtime, shared streams and allocations.
    """
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the process's HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2510_20891_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(func: str, status: int) -> None:
    if status != 0:
        lib = load()
        raise EmriError(func, status, lib.emri_last_error().decode())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _require_cuda(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class Spectrogram:
    """Normalised power P[alpha, b] in device memory: ``data`` is (n_seg, row_pitch)."""
    data: "object"          # torch.Tensor, float32 or float16
    n_bins: int
    t_sft: float

    @property
    def n_seg(self) -> int:
        return int(self.data.shape[0])

    @property
    def row_pitch(self) -> int:
        return int(self.data.shape[1])

    @property
    def dtype_code(self) -> int:
        import torch
        return {torch.float16: F16, torch.complex64: C32}.get(self.data.dtype, F32)

    def power(self):
        """The (n_seg, n_bins) view of the power without row padding."""
        return self.data[:, : self.n_bins]

    def _struct(self) -> _Power:
        return _Power(self.data.data_ptr() if self.data.numel() else 0, self.n_seg, self.n_bins,
                      self.row_pitch, self.dtype_code, float(self.t_sft))


def default_row_pitch(n_bins: int) -> int:
    """Smallest multiple of 8 above n_bins: the padding element lets scoring stage several rows per step."""
    return (n_bins + 8) // 8 * 8


def spectrogram_from_power(power, t_sft: float, dtype: str = "f32"):
    """Wrap an (n_seg, n_bins) host or device array as a padded device Spectrogram."""
    import torch
    p = torch.as_tensor(power)
    n_seg, n_bins = p.shape
    tdtype = torch.float32 if dtype == "f32" else torch.float16
    data = torch.zeros((n_seg, default_row_pitch(n_bins)), dtype=tdtype, device="cuda")
    data[:, :n_bins] = p.to(device="cuda", dtype=tdtype)
    return Spectrogram(data, n_bins, float(t_sft))


def build_sfts(x, dt: float, n_sft: int, psd, dtype: str = "f32", row_pitch: int | None = None,
               stream=None) -> Spectrogram:
    """Normalised SFT power of a device FP64 time series (see include/emri.h)."""
    import torch
    _require_cuda(x, torch.float64, "x")
    _require_cuda(psd, torch.float64, "psd")
    n_bins = n_sft // 2 + 1
    n_seg = x.numel() // n_sft if n_sft > 0 else 0
    pitch = row_pitch or default_row_pitch(n_bins)
    tdtype = {"f32": torch.float32, "f16": torch.float16, "c32": torch.complex64}[dtype]
    data = torch.empty((n_seg, pitch), dtype=tdtype, device=x.device)
    pw = _Power(data.data_ptr() if data.numel() else 0, 0, 0, pitch, _DTYPES[dtype], 0.0)
    _check("build_sfts", load().build_sfts(_ptr(x), x.numel(), float(dt), int(n_sft), _ptr(psd),
                                           ctypes.byref(pw), _stream(stream)))
    assert pw.n_seg == n_seg and pw.n_bins == n_bins
    return Spectrogram(data, n_bins, pw.t_sft)


def build_basis(tracks, K: int):
    """Centred SVD basis of training tracks (host, FP64): (f0, U, sv, box_lo, box_hi)."""
    F = np.ascontiguousarray(tracks, dtype=np.float64)
    n_train, n_seg = F.shape
    f0 = np.empty(n_seg)
    U = np.empty((n_seg, K))
    sv, lo, hi = np.empty(K), np.empty(K), np.empty(K)
    p = lambda a: a.ctypes.data if a.size else None
    _check("build_basis", load().build_basis(F.ctypes.data, n_train, n_seg, int(K), f0.ctypes.data, p(U),
                                             p(sv), p(lo), p(hi)))
    return f0, U, sv, lo, hi


def score_tracks_workspace_size(spec: Spectrogram, K: int, n_tmpl: int, top_k: int,
                                stat_in_workspace: bool) -> int:
    out = ctypes.c_size_t(0)
    pw = spec._struct()
    _check("score_tracks_workspace_size",
           load().score_tracks_workspace_size(ctypes.byref(pw), int(K), int(n_tmpl), int(top_k),
                                              int(bool(stat_in_workspace)), ctypes.byref(out)))
    return int(out.value)


class Workspace:
    """A reusable device workspace that grows on demand.

    Use one workspace per stream: two calls in flight at once must not share
    one.  The buffer is allocated on the stream that uses it, so the caching
    allocator never hands it (or a replaced, smaller one) to work on another
    stream before that stream's queued kernels are done with it.
    """

    def __init__(self):
        self.buf = None
        self.stream = None

    def get(self, nbytes: int, device, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(device)
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            with torch.cuda.stream(s):
                self.buf = torch.empty(max(nbytes, 256) + 256, dtype=torch.uint8, device=device)
            self.stream = s
        elif self.stream is not None and s.cuda_stream != self.stream.cuda_stream:
            # reused on another stream: keep it alive until that stream's work is done
            self.buf.record_stream(s)
        base = self.buf.data_ptr()
        off = (-base) % 256
        return base + off, self.buf.numel() - off


_default_ws: dict = {}


def default_workspace(device, stream=None) -> Workspace:
    """The binding's own workspace for calls on `stream` (one per device and stream)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return _default_ws.setdefault((str(device), int(s.cuda_stream)), Workspace())


def score_tracks(spec: Spectrogram, f0, U, coeffs, top_k: int, *, want_stat: bool = True,
                 want_bins: bool = False, want_near_tie: bool = False, k_min: int = 0, k_max: int = -1,
                 precision: str = "plain", rescore_top: bool = False, out: dict | None = None,
                 workspace: Workspace | None = None, stream=None) -> dict:
    """Nearest-bin statistic and top-k of a coefficient batch (device tensors).

    f0: (n_seg,) float64;  U: (n_seg, K) float64;  coeffs: (n_tmpl, K) float32.
    precision: "plain" (FP64 contraction) or "mixed" (BF16-split matrix cores, FP64 rounding).
    rescore_top (mixed, top_k > 0): re-score the leading candidates with FP64
    positions before the top-k (their stat entries become the plain statistic).
    Returns tensors: ``stat`` (n_tmpl,) float32 if want_stat, ``topk_val`` (top_k,),
    ``topk_idx`` (top_k,) int64, and ``bins`` / ``n_near_tie`` if requested.
    ``out`` may hold preallocated tensors under the same keys.
    """
    import torch
    _require_cuda(f0, torch.float64, "f0")
    _require_cuda(U, torch.float64, "U")
    _require_cuda(coeffs, torch.float32, "coeffs")
    K = int(U.shape[1]) if U.dim() == 2 else 0
    n_tmpl = int(coeffs.shape[0])
    if coeffs.dim() != 2 or coeffs.shape[1] != K:
        raise ValueError("coeffs must be (n_tmpl, K)")
    dev = coeffs.device
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    out = {} if out is None else out
    res = {}
    with torch.cuda.stream(s):       # outputs belong to the stream that writes them
        if want_stat:
            res["stat"] = out.get("stat") if out.get("stat") is not None else torch.empty(n_tmpl, dtype=torch.float32, device=dev)
        res["topk_val"] = out.get("topk_val") if out.get("topk_val") is not None else torch.empty(top_k, dtype=torch.float32, device=dev)
        res["topk_idx"] = out.get("topk_idx") if out.get("topk_idx") is not None else torch.empty(top_k, dtype=torch.int64, device=dev)
        if want_bins:
            res["bins"] = torch.empty((n_tmpl, spec.n_seg), dtype=torch.int32, device=dev)
        if want_near_tie:
            res["n_near_tie"] = torch.empty(1, dtype=torch.int64, device=dev)
    nbytes = score_tracks_workspace_size(spec, K, n_tmpl, top_k, not want_stat)
    ws = workspace if workspace is not None else default_workspace(dev, s)
    ws_ptr, ws_len = ws.get(nbytes, dev, s)
    opts = _Opts(int(k_min), int(k_max), _PRECISIONS[precision])
    opts.rescore_top = int(bool(rescore_top))
    pw = spec._struct()
    _check("score_tracks", load().score_tracks(
        ctypes.byref(pw), _ptr(f0), _ptr(U) if K else None, K, _ptr(coeffs) if K else None, n_tmpl, int(top_k),
        _ptr(res.get("stat")), _ptr(res["topk_val"]) if top_k else None,
        _ptr(res["topk_idx"]) if top_k else None, _ptr(res.get("bins")),
        _ptr(res.get("n_near_tie")), ctypes.byref(opts), ws_ptr, ws_len, int(s.cuda_stream)))
    return res


def score_tracks_noalloc(spec: Spectrogram, f0, U, coeffs, top_k: int, stat, topk_val, topk_idx, *,
                         k_min: int = 0, k_max: int = -1, precision: str = "plain", stream=None) -> None:
    """score_tracks into caller-owned outputs with the library's static scratch (no allocation).

    ``stat`` (n_tmpl,) float32 or None, ``topk_val`` (top_k,) float32 and
    ``topk_idx`` (top_k,) int64 are device tensors the caller owns.  Calls that
    overlap on one GPU race on the shared scratch.
    """
    import torch
    _require_cuda(f0, torch.float64, "f0")
    _require_cuda(U, torch.float64, "U")
    _require_cuda(coeffs, torch.float32, "coeffs")
    K = int(U.shape[1]) if U.dim() == 2 else 0
    n_tmpl = int(coeffs.shape[0])
    if coeffs.dim() != 2 or coeffs.shape[1] != K:
        raise ValueError("coeffs must be (n_tmpl, K)")
    opts = _Opts(int(k_min), int(k_max), _PRECISIONS[precision])
    pw = spec._struct()
    _check("score_tracks_noalloc", load().score_tracks_noalloc(
        ctypes.byref(pw), _ptr(f0), _ptr(U) if K else None, K, _ptr(coeffs) if K else None, n_tmpl, int(top_k),
        _ptr(stat), _ptr(topk_val) if top_k else None, _ptr(topk_idx) if top_k else None, None, None,
        ctypes.byref(opts), _stream(stream)))


def score_tracks_harmonics(spec: Spectrogram, f0, U, coeffs, ratios, top_k: int, *, k_min: int = 0,
                           k_max: int = -1, want_stat: bool = True, out: dict | None = None,
                           workspace: Workspace | None = None, stream=None) -> dict:
    """Multi-harmonic statistic: harmonic h follows the track scaled by ratios[h]
    (1 to 4 harmonics, K from 1 to 16); returns ``stat``, ``topk_val``, ``topk_idx``."""
    import torch
    _require_cuda(f0, torch.float64, "f0")
    _require_cuda(U, torch.float64, "U")
    _require_cuda(coeffs, torch.float32, "coeffs")
    K = int(U.shape[1]) if U.dim() == 2 else 0
    n_tmpl = int(coeffs.shape[0])
    if coeffs.dim() != 2 or coeffs.shape[1] != K:
        raise ValueError("coeffs must be (n_tmpl, K)")
    r = [float(v) for v in ratios]
    rr = (ctypes.c_double * max(1, len(r)))(*r)
    dev = coeffs.device
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    out = {} if out is None else out
    res = {}
    with torch.cuda.stream(s):
        if want_stat:
            res["stat"] = out.get("stat") if out.get("stat") is not None else torch.empty(n_tmpl, dtype=torch.float32, device=dev)
        res["topk_val"] = out.get("topk_val") if out.get("topk_val") is not None else torch.empty(top_k, dtype=torch.float32, device=dev)
        res["topk_idx"] = out.get("topk_idx") if out.get("topk_idx") is not None else torch.empty(top_k, dtype=torch.int64, device=dev)
    nbytes = score_tracks_workspace_size(spec, K, n_tmpl, top_k, not want_stat)
    ws = workspace if workspace is not None else default_workspace(dev, s)
    ws_ptr, ws_len = ws.get(nbytes, dev, s)
    opts = _Opts(int(k_min), int(k_max), PLAIN)
    pw = spec._struct()
    _check("score_tracks_harmonics", load().score_tracks_harmonics(
        ctypes.byref(pw), _ptr(f0), _ptr(U) if K else None, K, _ptr(coeffs) if K else None, n_tmpl, len(r), rr,
        int(top_k), _ptr(res.get("stat")), _ptr(res["topk_val"]) if top_k else None,
        _ptr(res["topk_idx"]) if top_k else None, ctypes.byref(opts), ws_ptr, ws_len, int(s.cuda_stream)))
    return res


CHIRP_F_MIN = 10.0 ** -3.5
CHIRP_FDOT_MIN = 1e-13


def score_tracks_chirp(sfts: Spectrogram, psd, f0, U, coeffs, top_k: int, *, p_half: int = 100,
                       f_min: float = CHIRP_F_MIN, fdot_min: float = CHIRP_FDOT_MIN, want_stat: bool = True,
                       out: dict | None = None, workspace: Workspace | None = None, stream=None) -> dict:
    """The linear-chirp statistic over 2 p_half + 1 bins (complex SFTs from
    build_sfts(..., dtype="c32"), the FP64 PSD on the bins); see include/emri.h."""
    import torch
    _require_cuda(psd, torch.float64, "psd")
    _require_cuda(f0, torch.float64, "f0")
    _require_cuda(U, torch.float64, "U")
    _require_cuda(coeffs, torch.float32, "coeffs")
    if sfts.dtype_code != C32:
        raise TypeError("score_tracks_chirp needs complex SFTs (dtype c32)")
    K = int(U.shape[1]) if U.dim() == 2 else 0
    n_tmpl = int(coeffs.shape[0])
    if coeffs.dim() != 2 or coeffs.shape[1] != K:
        raise ValueError("coeffs must be (n_tmpl, K)")
    dev = coeffs.device
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    out = {} if out is None else out
    res = {}
    with torch.cuda.stream(s):
        if want_stat:
            res["stat"] = out.get("stat") if out.get("stat") is not None else torch.empty(n_tmpl, dtype=torch.float32, device=dev)
        res["topk_val"] = out.get("topk_val") if out.get("topk_val") is not None else torch.empty(top_k, dtype=torch.float32, device=dev)
        res["topk_idx"] = out.get("topk_idx") if out.get("topk_idx") is not None else torch.empty(top_k, dtype=torch.int64, device=dev)
    pw = sfts._struct()
    lib = load()
    nb = ctypes.c_size_t(0)
    _check("score_tracks_chirp_workspace_size", lib.score_tracks_chirp_workspace_size(
        ctypes.byref(pw), K, n_tmpl, int(top_k), int(not want_stat), ctypes.byref(nb)))
    ws = workspace if workspace is not None else default_workspace(dev, s)
    ws_ptr, ws_len = ws.get(int(nb.value), dev, s)
    opts = _ChirpOpts(int(p_half), 0, float(f_min), float(fdot_min))
    _check("score_tracks_chirp", lib.score_tracks_chirp(
        ctypes.byref(pw), _ptr(psd), _ptr(f0), _ptr(U) if K else None, K, _ptr(coeffs) if K else None, n_tmpl,
        int(top_k), _ptr(res.get("stat")), _ptr(res["topk_val"]) if top_k else None,
        _ptr(res["topk_idx"]) if top_k else None, ctypes.byref(opts), ws_ptr, ws_len, int(s.cuda_stream)))
    return res


def score_tracks_noalloc_limit() -> int:
    return int(load().score_tracks_noalloc_limit())


@dataclass
class Problem:
    """One scoring problem of a batched launch (device tensors; outputs allocated if None)."""
    spec: Spectrogram
    f0: "object"
    U: "object"
    coeffs: "object"
    top_k: int = 0
    k_min: int = 0
    k_max: int = -1
    stat: "object" = None
    topk_val: "object" = None
    topk_idx: "object" = None


def batched_tile_options(K: int) -> list[int]:
    out = (ctypes.c_int32 * 4)()
    n = ctypes.c_int32(0)
    _check("score_batched_tile_options", load().score_batched_tile_options(int(K), out, ctypes.byref(n)))
    return [int(out[i]) for i in range(n.value)]


class BatchPlan:
    """A planned batched launch over many problems (the batched form of score_tracks).

    ``run()`` only launches kernels, so it can be captured in a HIP graph
    (``torch.cuda.CUDAGraph``) and replayed; a replay re-reads the problems'
    current device inputs.  Keep the plan (and its tensors) alive while it is used.
    """

    def __init__(self, problems: list, K: int, rows_per_step: int = 0, templates_per_lane: int = 0,
                 precision: str = "plain", workspace=None, stream=None):
        import torch
        self.problems = list(problems)
        self.K = int(K)
        arr = (_Problem * max(1, len(self.problems)))()
        for i, pb in enumerate(self.problems):
            _require_cuda(pb.f0, torch.float64, "f0")
            _require_cuda(pb.U, torch.float64, "U")
            _require_cuda(pb.coeffs, torch.float32, "coeffs")
            dev = pb.coeffs.device
            n = int(pb.coeffs.shape[0])
            if pb.stat is None:
                pb.stat = torch.empty(n, dtype=torch.float32, device=dev)
            if pb.topk_val is None:
                pb.topk_val = torch.empty(pb.top_k, dtype=torch.float32, device=dev)
            if pb.topk_idx is None:
                pb.topk_idx = torch.empty(pb.top_k, dtype=torch.int64, device=dev)
            a = arr[i]
            a.power = pb.spec._struct()
            a.f0 = _ptr(pb.f0)
            a.U = _ptr(pb.U) if self.K else None
            a.coeffs = _ptr(pb.coeffs) if self.K and n else None
            a.n_tmpl = n
            a.top_k = int(pb.top_k)
            a.k_min = int(pb.k_min)
            a.k_max = int(pb.k_max)
            a.stat = _ptr(pb.stat) if n else None
            a.topk_val = _ptr(pb.topk_val) if pb.top_k else None
            a.topk_idx = _ptr(pb.topk_idx) if pb.top_k else None
        self._arr = arr
        lib = load()
        nbytes = ctypes.c_size_t(0)
        _check("score_batched_workspace_size",
               lib.score_batched_workspace_size(arr, len(self.problems), self.K, ctypes.byref(nbytes)))
        dev = self.problems[0].coeffs.device if self.problems else torch.device("cuda")
        self._ws = workspace or Workspace()
        ws_ptr, ws_len = self._ws.get(int(nbytes.value), dev, stream)
        self.opts = _BatchOpts(int(rows_per_step), int(templates_per_lane), _PRECISIONS[precision])
        self._plan = _Plan()
        _check("score_batched_plan", lib.score_batched_plan(arr, len(self.problems), self.K, ctypes.byref(self.opts),
                                                            ws_ptr, ws_len, ctypes.byref(self._plan),
                                                            _stream(stream)))

    def run(self, stream=None) -> None:
        _check("score_batched_run", load().score_batched_run(ctypes.byref(self._plan), _stream(stream)))


class RawBatchPlan:
    """A batched launch planned from a filled ``_Problem`` array (raw device
    pointers, e.g. sub-buffers of a caller's preallocated tensors): the fast
    path for a serving loop that plans a batch per launch.  The caller keeps
    every buffer the array points to alive while the plan is used."""

    def __init__(self, arr, n: int, K: int, precision: str = "plain", workspace=None, device=None, stream=None):
        lib = load()
        self.K = int(K)
        self._arr = arr
        nbytes = ctypes.c_size_t(0)
        _check("score_batched_workspace_size", lib.score_batched_workspace_size(arr, int(n), self.K,
                                                                                ctypes.byref(nbytes)))
        self._ws = workspace or Workspace()
        ws_ptr, ws_len = self._ws.get(int(nbytes.value), device, stream)
        self.opts = _BatchOpts(0, 0, _PRECISIONS[precision])
        self._plan = _Plan()
        _check("score_batched_plan", lib.score_batched_plan(arr, int(n), self.K, ctypes.byref(self.opts), ws_ptr,
                                                            ws_len, ctypes.byref(self._plan), _stream(stream)))

    def run(self, stream=None) -> None:
        _check("score_batched_run", load().score_batched_run(ctypes.byref(self._plan), _stream(stream)))


@dataclass
class Chain:
    """One search population (device tensors): ``coeffs`` (n_walkers, K) float32 and
    ``stat`` (n_walkers,) float32 are updated in place; f0 / U may be views of a
    longer basis (the basis shifted by whole segments)."""
    spec: Spectrogram
    f0: "object"
    U: "object"
    box_lo: "object"
    box_hi: "object"
    coeffs: "object"
    stat: "object"
    k_min: int = 0
    k_max: int = -1

    @property
    def n_walkers(self) -> int:
        return int(self.coeffs.shape[0])


def _chains_array(chains, K: int):
    import torch
    arr = (_Chain * max(1, len(chains)))()
    for i, c in enumerate(chains):
        for name, dt in (("f0", torch.float64), ("U", torch.float64), ("box_lo", torch.float64),
                         ("box_hi", torch.float64), ("coeffs", torch.float32), ("stat", torch.float32)):
            _require_cuda(getattr(c, name), dt, name)
        if tuple(c.coeffs.shape) != (c.n_walkers, K) or tuple(c.U.shape) != (c.spec.n_seg, K):
            raise ValueError("chain shapes do not match K and the spectrogram")
        a = arr[i]
        a.power = c.spec._struct()
        a.f0, a.U, a.box_lo, a.box_hi = _ptr(c.f0), _ptr(c.U), _ptr(c.box_lo), _ptr(c.box_hi)
        a.coeffs, a.stat = _ptr(c.coeffs), _ptr(c.stat)
        a.n_walkers, a.k_min, a.k_max = c.n_walkers, int(c.k_min), int(c.k_max)
    return arr


def search_seed(chains: list, K: int, draws, f_init, precision: str = "plain", workspace=None, stream=None) -> None:
    """Seed every chain's walkers from draws (n_chains * n_draw, K) float32 and
    f_init (n_chains * n_draw,) float64 device tensors (see include/emri.h)."""
    import torch
    _require_cuda(draws, torch.float32, "draws")
    _require_cuda(f_init, torch.float64, "f_init")
    n_draw = int(f_init.shape[0]) // max(1, len(chains))
    if draws.shape[0] != n_draw * len(chains) or f_init.shape[0] != n_draw * len(chains):
        raise ValueError("draws and f_init must hold n_draw rows per chain")
    arr = _chains_array(chains, K)
    lib = load()
    nb = ctypes.c_size_t(0)
    _check("search_seed_workspace_size", lib.search_seed_workspace_size(arr, len(chains), int(K), n_draw,
                                                                        ctypes.byref(nb)))
    dev = draws.device
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    ws = workspace or Workspace()
    ws_ptr, ws_len = ws.get(int(nb.value), dev, s)
    opts = _BatchOpts(0, 0, _PRECISIONS[precision])
    _check("search_seed", lib.search_seed(arr, len(chains), int(K), _ptr(draws), _ptr(f_init), n_draw,
                                          ctypes.byref(opts), ws_ptr, ws_len, int(s.cuda_stream)))


class SearchPlan:
    """A planned population search over many chains (Eq. (11)).

    ``generation(r1, r2, F)`` runs one differential-evolution generation on
    every chain; it only launches kernels, so it can be captured into a HIP
    graph.  r1, r2: int32 and F: float64 device tensors with one entry per
    walker, chains concatenated in order.  Keep the plan, its chains and its
    workspace alive while it is used."""

    def __init__(self, chains: list, K: int, precision: str = "plain", rows_per_step: int = 0,
                 templates_per_lane: int = 0, workspace=None, stream=None):
        import torch
        self.chains = list(chains)
        self.K = int(K)
        self._arr = _chains_array(self.chains, self.K)
        self.n_walkers = sum(c.n_walkers for c in self.chains)
        lib = load()
        nb = ctypes.c_size_t(0)
        _check("search_workspace_size", lib.search_workspace_size(self._arr, len(self.chains), self.K,
                                                                  ctypes.byref(nb)))
        dev = self.chains[0].coeffs.device
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        self._ws = workspace or Workspace()
        ws_ptr, ws_len = self._ws.get(int(nb.value), dev, s)
        self.opts = _BatchOpts(int(rows_per_step), int(templates_per_lane), _PRECISIONS[precision])
        self._plan = _SearchPlan()
        _check("search_plan", lib.search_plan(self._arr, len(self.chains), self.K, ctypes.byref(self.opts), ws_ptr,
                                              ws_len, ctypes.byref(self._plan), int(s.cuda_stream)))

    def generation(self, r1, r2, F, accepted=None, stream=None) -> None:
        import torch
        _require_cuda(r1, torch.int32, "r1")
        _require_cuda(r2, torch.int32, "r2")
        _require_cuda(F, torch.float64, "F")
        for t in (r1, r2, F):
            if t.numel() < self.n_walkers:
                raise ValueError("r1, r2 and F need one entry per walker")
        if accepted is not None:
            _require_cuda(accepted, torch.int32, "accepted")
            if accepted.numel() < self.n_walkers:
                raise ValueError("accepted needs one entry per walker")
        _check("search_generation", load().search_generation(ctypes.byref(self._plan), _ptr(r1), _ptr(r2), _ptr(F),
                                                             _ptr(accepted), _stream(stream)))

    def generations(self, r1, r2, F, stream=None) -> None:
        """len(r1) generations (r1, r2: int32 and F: float64 device tensors of
        shape (n_gen, walkers)), two at a time in one launch each; the result
        is that of as many generation() calls, bit for bit."""
        import torch
        _require_cuda(r1, torch.int32, "r1")
        _require_cuda(r2, torch.int32, "r2")
        _require_cuda(F, torch.float64, "F")
        n_gen = int(r1.shape[0]) if r1.dim() == 2 else 0
        for t in (r1, r2, F):
            if t.dim() != 2 or int(t.shape[0]) != n_gen or int(t.shape[1]) != self.n_walkers or not t.is_contiguous():
                raise ValueError("r1, r2 and F must be contiguous (n_gen, walkers) tensors")
        _check("search_generations", load().search_generations(ctypes.byref(self._plan), n_gen, _ptr(r1), _ptr(r2),
                                                               _ptr(F), _stream(stream)))

    def best(self, noise_mean=None, noise_std=None, stream=None) -> dict:
        """Per chain: best statistic and walker index, and the normalised statistic if noise moments are given."""
        import torch
        dev = self.chains[0].coeffs.device
        n = len(self.chains)
        out = {"stat": torch.empty(n, dtype=torch.float32, device=dev),
               "idx": torch.empty(n, dtype=torch.int32, device=dev)}
        if noise_mean is not None:
            _require_cuda(noise_mean, torch.float64, "noise_mean")
            _require_cuda(noise_std, torch.float64, "noise_std")
            out["norm"] = torch.empty(n, dtype=torch.float64, device=dev)
        _check("search_best", load().search_best(ctypes.byref(self._plan), _ptr(noise_mean), _ptr(noise_std),
                                                 _ptr(out["stat"]), _ptr(out["idx"]), _ptr(out.get("norm")),
                                                 _stream(stream)))
        return out


def search_noise_moments(best, stream=None):
    """Per-chain mean and sample standard deviation over noise-only searches:
    best is a (n_real, n_chains) float32 device tensor; returns two float64
    (n_chains,) device tensors."""
    import torch
    _require_cuda(best, torch.float32, "best")
    n_real, n_chains = int(best.shape[0]), int(best.shape[1])
    mean = torch.empty(n_chains, dtype=torch.float64, device=best.device)
    sd = torch.empty(n_chains, dtype=torch.float64, device=best.device)
    _check("search_noise_moments", load().search_noise_moments(_ptr(best), n_real, n_chains, _ptr(mean), _ptr(sd),
                                                               _stream(stream)))
    return mean, sd


__all__ = ["score_tracks_chirp", "score_tracks_harmonics", "Chain", "SearchPlan", "search_seed", "search_noise_moments", "Problem", "BatchPlan", "score_tracks_noalloc", "score_tracks_noalloc_limit", "batched_tile_options", "load", "build_sfts", "build_basis", "score_tracks", "score_tracks_workspace_size",
           "Spectrogram", "spectrogram_from_power", "Workspace", "default_workspace", "EmriError", "F32", "F16", "LIB_PATH"]
