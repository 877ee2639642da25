"""Python binding of libttm (ctypes).  Argument marshalling only: every step of
the matching path runs in the HIP kernels of libttm.so; PyTorch provides device
memory and the stream.  There is no fallback: if the library is missing or the
tensors are not on a GPU, the calls raise.

Functions mirror the C ABI in include/ttm.h:

* ``build_tensor_template(tmpl, mask, order, quats, weights, image_shape)``
* ``correlate(image, bank, mask, order, opt)``
* ``recover_pose(score, image, components, mask, order, opt)``
* ``rotation_map(image, bank, mask, order, seeds, opt)``
* ``correlate_tiled(image, bank, mask, order, tile, opt)``, ``autotune_tiles``,
  ``choose_tile``, ``batch_match(jobs, order, opt)``, ``BatchGraph``
* ``tm_classical(image, tmpl, mask, quats, opt)``
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libttm.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "ttm.h")

TTM_OK = 0
STATUS = {0: "TTM_OK", -1: "TTM_E_ARG", -2: "TTM_E_SIZE", -3: "TTM_E_WORKSPACE",
          -4: "TTM_E_HIP", -5: "TTM_E_NONFINITE"}
POSE_NOT_CONVERGED = 1
POSE_ZERO_NORM = 2
PEAKS_TRUNCATED = 4


class TTMError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


class Dims(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int32), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("eps_v", ctypes.c_float), ("threshold", ctypes.c_float),
                ("min_dist", ctypes.c_float), ("max_peaks", ctypes.c_int32),
                ("n_seeds", ctypes.c_int32), ("hopm_max_iter", ctypes.c_int32),
                ("hopm_tol", ctypes.c_double), ("refine", ctypes.c_int32),
                ("check_finite", ctypes.c_int32)]


class BatchJob(ctypes.Structure):
    """``ttm_batch_job``: one tomogram against one template (see include/ttm.h)."""
    _fields_ = [("image", ctypes.c_void_p), ("N", Dims), ("bank", ctypes.c_void_p), ("tile", ctypes.c_int32),
                ("components", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("tmpl", ctypes.c_void_p),
                ("L", Dims), ("out_score", ctypes.c_void_p), ("out_w", ctypes.c_void_p),
                ("out_pos", ctypes.c_void_p), ("out_quat", ctypes.c_void_p), ("out_lambda", ctypes.c_void_p),
                ("out_peak_score", ctypes.c_void_p), ("out_flags", ctypes.c_void_p),
                ("out_count", ctypes.c_void_p)]


_lib = None
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t
_I32 = ctypes.c_int32
_DIMS = Dims
_OPTP = ctypes.POINTER(Options)

_SIGS = {
    "ttm_default_options": (None, [_OPTP]),
    "ttm_num_components": (_I32, [_I32]),
    "ttm_supported_length": (_I32, [_I32]),
    "ttm_status_string": (ctypes.c_char_p, [_I32]),
    "ttm_bank_bytes": (_SZ, [_DIMS, _DIMS, _I32]),
    "ttm_build_workspace_bytes": (_SZ, [_DIMS, _I32, _I32, _DIMS]),
    "ttm_build_tensor_template": (_I32, [_P, _P, _DIMS, _I32, _P, _P, _I32, _P, _DIMS, _P, _P, _SZ, _P]),
    "ttm_correlate_workspace_bytes": (_SZ, [_DIMS, _DIMS, _I32]),
    "ttm_correlate": (_I32, [_P, _DIMS, _P, _DIMS, _I32, _P, _OPTP, _P, _P, _P, _SZ, _P]),
    "ttm_pose_workspace_bytes": (_SZ, [_DIMS, _DIMS, _I32, _OPTP]),
    "ttm_recover_pose": (_I32, [_P, _P, _P, _P, _P, _DIMS, _DIMS, _I32, _OPTP, _P, _P, _P, _P, _P, _P, _P,
                                _P, _SZ, _P]),
    "ttm_pose_at": (_I32, [_P, _P, _P, _P, _DIMS, _DIMS, _I32, _OPTP, _P, _I32, _P, _P, _P, _P, _P, _P, _SZ,
                           _P]),
    "ttm_pose_at_noalloc": (_I32, [_P, _P, _P, _P, _DIMS, _DIMS, _I32, _OPTP, _P, _I32, _P, _P, _P, _P, _P, _P]),
    "ttm_match_workspace_bytes": (_SZ, [_DIMS, _DIMS, _I32, _OPTP]),
    "ttm_match": (_I32, [_P, _DIMS, _P, _DIMS, _I32, _P, _P, _OPTP, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                         _SZ, _P]),
    "tm_classical_workspace_bytes": (_SZ, [_DIMS, _DIMS, _I32]),
    "tm_classical": (_I32, [_P, _DIMS, _P, _P, _DIMS, _P, _I32, _OPTP, _P, _P, _P, _SZ, _P]),
    "ttm_score_backward_workspace_bytes": (_SZ, [_DIMS, _I32, _I32, _I32]),
    "ttm_score_backward": (_I32, [_P, _DIMS, _P, _P, _DIMS, _I32, _P, _P, _I32, _P, _P, _I32, _P, _OPTP, _P, _P,
                                  _P, _SZ, _P]),
    "ttm_rotation_map_workspace_bytes": (_SZ, [_DIMS, _DIMS, _I32, _I32]),
    "ttm_rotation_map": (_I32, [_P, _DIMS, _P, _DIMS, _I32, _P, _OPTP, _P, _I32, _P, _P, _P, _P, _P, _P, _SZ,
                                _P]),
    "ttm_bank_bytes_2d": (_SZ, [_I32, _I32, _I32, _I32, _I32, _I32]),
    "ttm_build_workspace_bytes_2d": (_SZ, [_I32, _I32, _I32, _I32]),
    "ttm_build_tensor_template_2d": (_I32, [_P, _P, _I32, _I32, _I32, _P, _P, _I32, _P, _I32, _I32, _I32, _P, _P,
                                            _SZ, _P]),
    "ttm_match_2d_workspace_bytes": (_SZ, [_I32, _I32, _I32, _I32, _I32, _I32, _OPTP]),
    "ttm_match_2d": (_I32, [_P, _I32, _I32, _I32, _P, _P, _P, _P, _I32, _I32, _I32, _OPTP, _P, _P, _P, _P, _P, _P,
                            _P, _P, _P, _SZ, _P]),
    "ttm_snorm_workspace_bytes": (_SZ, [_DIMS, _I32, _I32]),
    "ttm_snorm": (_I32, [_P, _DIMS, _P, _P, _DIMS, _I32, _P, _P, _I32, _P, _P, _P, _I32, _P, _P, _P, _P, _SZ, _P]),
    "ttm_tile_count": (_I32, [_DIMS, _DIMS, _I32]),
    "ttm_choose_tile": (_I32, [_DIMS, _DIMS, _P, _P, _I32]),
    "ttm_correlate_tiled_workspace_bytes": (_SZ, [_DIMS, _I32, _I32]),
    "ttm_correlate_tiled": (_I32, [_P, _DIMS, _P, _DIMS, _I32, _I32, _P, _OPTP, _P, _P, _P, _SZ, _P]),
    "ttm_autotune_workspace_bytes": (_SZ, [_DIMS, _I32, _P, _I32]),
    "ttm_autotune_tiles": (_I32, [_P, _P, _I32, _DIMS, _I32, _P, _OPTP, _I32, _P, _P, _SZ, _P]),
    "ttm_batch_workspace_bytes": (_SZ, [_P, _I32, _I32, _OPTP, _I32]),
    "ttm_batch_match": (_I32, [_P, _I32, _I32, _OPTP, _I32, _P, _SZ, _P]),
    "ttm_batch_graph_create": (_I32, [_P, _I32, _I32, _OPTP, _I32, _P, _SZ, _P, _P]),
    "ttm_graph_launch": (_I32, [_P, _P]),
    "ttm_graph_destroy": (None, [_P]),
    "ttm_lowpass_workspace_bytes": (_SZ, [_DIMS]),
    "ttm_lowpass": (_I32, [_P, _DIMS, ctypes.c_float, _I32, _P, _P, _SZ, _P]),
    "ttm_profile_enable": (None, [_I32]),
    "ttm_profile_read": (_I32, [_P, _P, _I32]),
    "ttm_profile_class_name": (ctypes.c_char_p, [_I32]),
}

PROFILE_CLASSES = 13


def profile_enable(on: bool = True):
    """Record HIP event pairs around every kernel group (instrumentation)."""
    lib().ttm_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """Summed milliseconds and launch counts per kernel class since the last
    read (waits for the recorded events)."""
    ms = (ctypes.c_double * PROFILE_CLASSES)()
    cnt = (ctypes.c_int64 * PROFILE_CLASSES)()
    st = lib().ttm_profile_read(ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(cnt, ctypes.c_void_p),
                                PROFILE_CLASSES)
    if st < 0:
        raise TTMError(st, "ttm_profile_read")
    return {lib().ttm_profile_class_name(i).decode(): (ms[i], cnt[i]) for i in range(PROFILE_CLASSES)}


def declared_functions() -> list[str]:
    """Names of the functions declared in include/ttm.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"\b((?:ttm|tm)_[a-z_0-9]+)\s*\(", text)


def lib(path: str | None = None) -> ctypes.CDLL:
    """Load libttm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libttm.so not found at {p}: build it with "
                           "`python -m paper_2311_07561_amd.build_lib`")
    L = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = L
    return L


def _check(status: int, what: str):
    if status != TTM_OK:
        raise TTMError(status, what)


def _dims(shape) -> Dims:
    s = tuple(int(v) for v in shape)
    if len(s) != 3:
        raise ValueError("expected a 3-D shape")
    return Dims(*s)


def _dev(t: torch.Tensor, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor")
    return t.data_ptr()


def _i32_dev(t, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous int32 CUDA (HIP) tensor")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def default_options(**kw) -> Options:
    o = Options()
    lib().ttm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def num_components(order: int) -> int:
    k = lib().ttm_num_components(order)
    if k < 0:
        raise TTMError(k, "num_components")
    return k


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def build_tensor_template(tmpl: torch.Tensor, mask: torch.Tensor, order: int, quats, weights,
                          image_shape=None):
    """Tensor template components (K, L0, L1, L2) and, if ``image_shape`` is
    given, the correlation bank for images of that shape."""
    dev = tmpl.device
    K = num_components(order)
    L = _dims(tmpl.shape)
    q = torch.as_tensor(quats, dtype=torch.float32).contiguous().cpu()
    w = torch.as_tensor(weights, dtype=torch.float64).contiguous().cpu()
    nrot = q.shape[0]
    if q.shape != (nrot, 4) or w.shape != (nrot,):
        raise ValueError("quats must be (J, 4) and weights (J,)")
    comps = torch.empty((K,) + tuple(tmpl.shape), dtype=torch.float32, device=dev)
    N = _dims(image_shape) if image_shape is not None else Dims(0, 0, 0)
    bank = None
    if image_shape is not None:
        nb = lib().ttm_bank_bytes(N, L, K)
        bank = torch.empty(nb, dtype=torch.uint8, device=dev)
    nws = lib().ttm_build_workspace_bytes(L, order, nrot, N)
    ws = _workspace(nws, dev)
    st = lib().ttm_build_tensor_template(
        _dev(tmpl, "tmpl"), _dev(mask, "mask"), L, order, q.data_ptr(), w.data_ptr(), nrot,
        comps.data_ptr(), N, bank.data_ptr() if bank is not None else None, ws.data_ptr(), nws,
        _stream(dev))
    _check(st, "ttm_build_tensor_template")
    return comps, bank


def correlate(image: torch.Tensor, bank: torch.Tensor, mask: torch.Tensor, order: int,
              opt: Options | None = None, want_w: bool = True, workspace: torch.Tensor | None = None,
              out=None):
    """Frobenius score map F(x) and local normaliser w(x).  ``out`` may give
    preallocated (score, w) tensors (w may be None)."""
    dev = image.device
    K = num_components(order)
    N = _dims(image.shape)
    L = _dims(mask.shape)
    opt = opt or default_options()
    if out is not None:
        score, w = out
        _dev(score, "score")
        if w is not None:
            _dev(w, "w")
    else:
        score = torch.empty_like(image)
        w = torch.empty_like(image) if want_w else None
    nws = lib().ttm_correlate_workspace_bytes(N, L, K)
    ws = workspace if workspace is not None and workspace.numel() >= nws else _workspace(nws, dev)
    st = lib().ttm_correlate(_dev(image, "image"), N, bank.data_ptr(), L, order, _dev(mask, "mask"),
                             ctypes.byref(opt), score.data_ptr(),
                             w.data_ptr() if w is not None else None, ws.data_ptr(), ws.numel(),
                             _stream(dev))
    _check(st, "ttm_correlate")
    return score, w


def correlate_workspace(image_shape, L, order, device) -> torch.Tensor:
    K = num_components(order)
    return _workspace(lib().ttm_correlate_workspace_bytes(_dims(image_shape), _dims(L), K), device)


def _opt_dev(t, name):
    return None if t is None else _dev(t, name)


def recover_pose(score: torch.Tensor, image: torch.Tensor, components: torch.Tensor,
                 mask: torch.Tensor, order: int, opt: Options | None = None, want_C: bool = True,
                 tmpl: torch.Tensor | None = None):
    """Peaks of F and the dominant Z-eigenpair of C_n at each.  Returns a dict
    of device tensors trimmed to the number of peaks found (one sync).  The raw
    template ``tmpl`` is needed with ``opt.refine >= 2``."""
    dev = score.device
    K = num_components(order)
    N = _dims(score.shape)
    L = _dims(mask.shape)
    opt = opt or default_options()
    P = int(opt.max_peaks)
    pos = torch.zeros((P, 3), dtype=torch.int32, device=dev)
    quat = torch.zeros((P, 4), dtype=torch.float32, device=dev)
    lam = torch.zeros((P,), dtype=torch.float64, device=dev)
    pscore = torch.zeros((P,), dtype=torch.float32, device=dev)
    flags = torch.zeros((P,), dtype=torch.int32, device=dev)
    C = torch.zeros((P, K), dtype=torch.float64, device=dev) if want_C else None
    count = torch.zeros((2,), dtype=torch.int32, device=dev)
    nws = lib().ttm_pose_workspace_bytes(N, L, order, ctypes.byref(opt))
    ws = _workspace(nws, dev)
    st = lib().ttm_recover_pose(_dev(score, "score"), _dev(image, "image"), _dev(components, "components"),
                                _dev(mask, "mask"), _opt_dev(tmpl, "tmpl"), N, L, order, ctypes.byref(opt),
                                pos.data_ptr(),
                                quat.data_ptr(), lam.data_ptr(), pscore.data_ptr(), flags.data_ptr(),
                                C.data_ptr() if C is not None else None, count.data_ptr(), ws.data_ptr(),
                                nws, _stream(dev))
    _check(st, "ttm_recover_pose")
    cnt = count.cpu()
    n = int(cnt[0])
    out = dict(pos=pos[:n], quat=quat[:n], lam=lam[:n], score=pscore[:n], flags=flags[:n],
               truncated=bool(int(cnt[1]) & PEAKS_TRUNCATED), count=n)
    if C is not None:
        out["C"] = C[:n]
    return out


def pose_at(image: torch.Tensor, components: torch.Tensor, mask: torch.Tensor, order: int, positions,
            opt: Options | None = None, want_C: bool = True, tmpl: torch.Tensor | None = None) -> dict:
    """Dominant Z-eigenpair of C_n at caller-given positions (P, 3)."""
    dev = image.device
    K = num_components(order)
    N = _dims(image.shape)
    L = _dims(mask.shape)
    pos = torch.as_tensor(positions, dtype=torch.int32).reshape(-1, 3).contiguous().to(dev)
    P = pos.shape[0]
    opt = opt or default_options()
    if P > opt.max_peaks:
        opt = Options.from_buffer_copy(opt)
        opt.max_peaks = P
    out_pos = torch.zeros((P, 3), dtype=torch.int32, device=dev)
    quat = torch.zeros((P, 4), dtype=torch.float32, device=dev)
    lam = torch.zeros((P,), dtype=torch.float64, device=dev)
    flags = torch.zeros((P,), dtype=torch.int32, device=dev)
    C = torch.zeros((P, K), dtype=torch.float64, device=dev) if want_C else None
    nws = lib().ttm_pose_workspace_bytes(N, L, order, ctypes.byref(opt))
    ws = _workspace(nws, dev)
    st = lib().ttm_pose_at(_dev(image, "image"), _dev(components, "components"), _dev(mask, "mask"),
                           _opt_dev(tmpl, "tmpl"), N, L, order, ctypes.byref(opt), pos.data_ptr(), P, out_pos.data_ptr(), quat.data_ptr(),
                           lam.data_ptr(), flags.data_ptr(), C.data_ptr() if C is not None else None,
                           ws.data_ptr(), nws, _stream(dev))
    _check(st, "ttm_pose_at")
    out = dict(pos=out_pos, quat=quat, lam=lam, flags=flags)
    if C is not None:
        out["C"] = C
    return out


def pose_at_noalloc(image: torch.Tensor, components: torch.Tensor, mask: torch.Tensor, order: int,
                    positions: torch.Tensor, opt: Options, out: dict, tmpl: torch.Tensor | None = None):
    """ttm_pose_at_noalloc: ``pose_at`` with the library's static device
    scratch instead of a workspace; nothing is allocated here either.
    ``positions`` is an (P, 3) int32 CUDA tensor, ``out`` holds preallocated
    ``pos`` (P, 3) int32, ``quat`` (P, 4) float32, ``lam`` (P,) float64,
    ``flags`` (P,) int32 and optionally ``C`` (P, K) float64, all written on
    the current stream."""
    dev = image.device
    P = positions.shape[0]
    if positions.shape != (P, 3):
        raise ValueError("positions must be (P, 3)")
    C = out.get("C")
    st = lib().ttm_pose_at_noalloc(_dev(image, "image"), _dev(components, "components"), _dev(mask, "mask"),
                                   _opt_dev(tmpl, "tmpl"), _dims(image.shape), _dims(mask.shape), order,
                                   ctypes.byref(opt), _i32_dev(positions, "positions"), P,
                                   _i32_dev(out["pos"], "pos"), out["quat"].data_ptr(), out["lam"].data_ptr(),
                                   _i32_dev(out["flags"], "flags"), C.data_ptr() if C is not None else None,
                                   _stream(dev))
    _check(st, "ttm_pose_at_noalloc")


class PoseBuffers:
    """Preallocated outputs and workspace of ``recover_pose_async``."""

    def __init__(self, opt: Options, K: int, device):
        P = int(opt.max_peaks)
        self.pos = torch.zeros((P, 3), dtype=torch.int32, device=device)
        self.quat = torch.zeros((P, 4), dtype=torch.float32, device=device)
        self.lam = torch.zeros((P,), dtype=torch.float64, device=device)
        self.score = torch.zeros((P,), dtype=torch.float32, device=device)
        self.flags = torch.zeros((P,), dtype=torch.int32, device=device)
        self.C = torch.zeros((P, K), dtype=torch.float64, device=device)
        self.count = torch.zeros((2,), dtype=torch.int32, device=device)
        self.ws = _workspace(1 << 20, device)

    def result(self) -> dict:
        cnt = self.count.cpu()
        n = int(cnt[0])
        return dict(pos=self.pos[:n], quat=self.quat[:n], lam=self.lam[:n], score=self.score[:n],
                    flags=self.flags[:n], C=self.C[:n], count=n,
                    truncated=bool(int(cnt[1]) & PEAKS_TRUNCATED))


def recover_pose_async(score: torch.Tensor, image: torch.Tensor, components: torch.Tensor,
                       mask: torch.Tensor, order: int, opt: Options, bufs: PoseBuffers,
                       tmpl: torch.Tensor | None = None):
    """``recover_pose`` into preallocated buffers, without synchronising."""
    dev = score.device
    N = _dims(score.shape)
    L = _dims(mask.shape)
    nws = lib().ttm_pose_workspace_bytes(N, L, order, ctypes.byref(opt))
    if bufs.ws.numel() < nws:
        bufs.ws = _workspace(nws, dev)
    st = lib().ttm_recover_pose(_dev(score, "score"), _dev(image, "image"), _dev(components, "components"),
                                _dev(mask, "mask"), _opt_dev(tmpl, "tmpl"), N, L, order, ctypes.byref(opt),
                                bufs.pos.data_ptr(),
                                bufs.quat.data_ptr(), bufs.lam.data_ptr(), bufs.score.data_ptr(),
                                bufs.flags.data_ptr(), bufs.C.data_ptr(), bufs.count.data_ptr(),
                                bufs.ws.data_ptr(), bufs.ws.numel(), _stream(dev))
    _check(st, "ttm_recover_pose")


class MatchBuffers(PoseBuffers):
    """Preallocated outputs and workspace of ``match``."""

    def __init__(self, image_shape, L, order: int, opt: Options, device):
        K = num_components(order)
        super().__init__(opt, K, device)
        self.score = torch.empty(tuple(image_shape), dtype=torch.float32, device=device)
        self.w = torch.empty(tuple(image_shape), dtype=torch.float32, device=device)
        self.peak_score = torch.zeros((int(opt.max_peaks),), dtype=torch.float32, device=device)
        nws = lib().ttm_match_workspace_bytes(_dims(image_shape), _dims(L), order, ctypes.byref(opt))
        self.ws = _workspace(nws, device)

    def result(self) -> dict:
        cnt = self.count.cpu()
        n = int(cnt[0])
        return dict(pos=self.pos[:n], quat=self.quat[:n], lam=self.lam[:n], score=self.peak_score[:n],
                    flags=self.flags[:n], C=self.C[:n], count=n,
                    truncated=bool(int(cnt[1]) & PEAKS_TRUNCATED))


def match(image: torch.Tensor, bank: torch.Tensor, mask: torch.Tensor, order: int, opt: Options,
          bufs: MatchBuffers, tmpl: torch.Tensor | None = None):
    """Correlation, peaks and poses in one asynchronous call (ttm_match);
    results land in ``bufs`` (score map in bufs.score, w in bufs.w).  The raw
    template ``tmpl`` is needed with ``opt.refine >= 2``."""
    dev = image.device
    N = _dims(image.shape)
    L = _dims(mask.shape)
    st = lib().ttm_match(_dev(image, "image"), N, bank.data_ptr(), L, order, _dev(mask, "mask"),
                         _opt_dev(tmpl, "tmpl"), ctypes.byref(opt), bufs.score.data_ptr(), bufs.w.data_ptr(), bufs.pos.data_ptr(),
                         bufs.quat.data_ptr(), bufs.lam.data_ptr(), bufs.peak_score.data_ptr(),
                         bufs.flags.data_ptr(), bufs.C.data_ptr(), bufs.count.data_ptr(), bufs.ws.data_ptr(),
                         bufs.ws.numel(), _stream(dev))
    _check(st, "ttm_match")


def build_tensor_template_2d(tmpl: torch.Tensor, mask: torch.Tensor, order: int, zs, weights,
                             stack_shape=None):
    """Planar tensor template (ttm_build_tensor_template_2d): components
    (n + 1, L1, L2) and, if ``stack_shape`` = (B, n1, n2) is given, the bank
    for stacks of that shape.  ``zs`` are unit complex numbers (J, 2) of half
    the rotation angles."""
    dev = tmpl.device
    L1, L2 = (int(v) for v in tmpl.shape)
    z = torch.as_tensor(zs, dtype=torch.float32).contiguous().cpu()
    w = torch.as_tensor(weights, dtype=torch.float64).contiguous().cpu()
    nrot = z.shape[0]
    if z.shape != (nrot, 2) or w.shape != (nrot,):
        raise ValueError("zs must be (J, 2) and weights (J,)")
    comps = torch.empty((order + 1, L1, L2), dtype=torch.float32, device=dev)
    B = n1 = n2 = 0
    bank = None
    if stack_shape is not None:
        B, n1, n2 = (int(v) for v in stack_shape)
        nb = lib().ttm_bank_bytes_2d(B, n1, n2, L1, L2, order)
        if nb == 0:
            raise TTMError(-2, "ttm_bank_bytes_2d")
        bank = torch.empty(nb, dtype=torch.uint8, device=dev)
    nws = lib().ttm_build_workspace_bytes_2d(L1, L2, order, nrot)
    ws = _workspace(nws, dev)
    st = lib().ttm_build_tensor_template_2d(
        _dev(tmpl, "tmpl"), _dev(mask, "mask"), L1, L2, order, z.data_ptr(), w.data_ptr(), nrot,
        comps.data_ptr(), B, n1, n2, bank.data_ptr() if bank is not None else None, ws.data_ptr(), nws,
        _stream(dev))
    _check(st, "ttm_build_tensor_template_2d")
    return comps, bank


class Match2DBuffers:
    """Preallocated outputs and workspace of ``match_2d`` for stacks of shape
    (B, n1, n2) and an (L1, L2) template."""

    def __init__(self, stack_shape, L, order: int, opt: Options, device, want_w: bool = True):
        B, n1, n2 = (int(v) for v in stack_shape)
        P = int(opt.max_peaks)
        self.shape = (B, n1, n2)
        self.score = torch.empty((B, n1, n2), dtype=torch.float32, device=device)
        self.w = torch.empty((B, n1, n2), dtype=torch.float32, device=device) if want_w else None
        self.pos = torch.zeros((B, P, 2), dtype=torch.int32, device=device)
        self.z = torch.zeros((B, P, 2), dtype=torch.float32, device=device)
        self.lam = torch.zeros((B, P), dtype=torch.float64, device=device)
        self.peak_score = torch.zeros((B, P), dtype=torch.float32, device=device)
        self.flags = torch.zeros((B, P), dtype=torch.int32, device=device)
        self.count = torch.zeros((B, 2), dtype=torch.int32, device=device)
        nws = lib().ttm_match_2d_workspace_bytes(B, n1, n2, int(L[0]), int(L[1]), order, ctypes.byref(opt))
        if nws == 0:
            raise TTMError(-2, "ttm_match_2d_workspace_bytes")
        self.ws = _workspace(nws, device)

    def result(self, b: int) -> dict:
        """Plane b's peaks, trimmed to its count (one sync)."""
        n = int(self.count[b, 0])
        return dict(pos=self.pos[b, :n], z=self.z[b, :n], lam=self.lam[b, :n], score=self.peak_score[b, :n],
                    flags=self.flags[b, :n], count=n)


def match_2d(images: torch.Tensor, bank: torch.Tensor, comps: torch.Tensor, mask: torch.Tensor, order: int,
             opt: Options, bufs: Match2DBuffers, tmpl: torch.Tensor | None = None):
    """Planar TTM on a stack (ttm_match_2d): score maps, peaks and rotations
    of every plane into ``bufs``, asynchronously."""
    dev = images.device
    B, n1, n2 = (int(v) for v in images.shape)
    L1, L2 = (int(v) for v in mask.shape)
    st = lib().ttm_match_2d(
        _dev(images, "images"), B, n1, n2, bank.data_ptr(), _dev(comps, "comps"), _opt_dev(tmpl, "tmpl"),
        _dev(mask, "mask"), L1, L2, order, ctypes.byref(opt), bufs.score.data_ptr(),
        bufs.w.data_ptr() if bufs.w is not None else None, bufs.pos.data_ptr(), bufs.z.data_ptr(),
        bufs.lam.data_ptr(), bufs.peak_score.data_ptr(), bufs.flags.data_ptr(), bufs.count.data_ptr(),
        bufs.ws.data_ptr(), bufs.ws.numel(), _stream(dev))
    _check(st, "ttm_match_2d")


SNORM_FLAT, SNORM_NONPOS, SNORM_OUTSIDE, SNORM_TEMPLATE = 1, 2, 4, 8


def snorm(image: torch.Tensor, tmpl: torch.Tensor, mask: torch.Tensor, order: int, quats, weights,
          pos: torch.Tensor, lam: torch.Tensor, count: torch.Tensor | None = None,
          workspace: torch.Tensor | None = None):
    """S'-consistent normalisation (ttm_snorm): ``rho' = lambda / sqrt(D(window)
    D(template))`` at the positions ``pos`` (P, 3) int32 with their
    eigenvalues ``lam`` (P,) float64, using the tensor template's quadrature
    ``(quats, weights)``.  ``count`` (device int32, one element) limits the
    positions used.  Returns (rho (P,) float32, D (P + 1,) float64 with the
    template's last, flags (P,) int32); entries past ``count`` are zero."""
    dev = image.device
    N = _dims(image.shape)
    L = _dims(tmpl.shape)
    q = torch.as_tensor(quats, dtype=torch.float32).contiguous().cpu()
    w = torch.as_tensor(weights, dtype=torch.float64).contiguous().cpu()
    nrot = q.shape[0]
    if q.shape != (nrot, 4) or w.shape != (nrot,):
        raise ValueError("quats must be (J, 4) and weights (J,)")
    P = int(pos.shape[0])
    if tuple(pos.shape) != (P, 3) or tuple(lam.shape) != (P,):
        raise ValueError("pos must be (P, 3) and lam (P,)")
    _i32_dev(pos, "pos")
    _i32_dev(count, "count")
    if not lam.is_cuda or lam.dtype != torch.float64 or not lam.is_contiguous():
        raise ValueError("lam must be a contiguous float64 CUDA (HIP) tensor")
    rho = torch.zeros(P, dtype=torch.float32, device=dev)
    D = torch.zeros(P + 1, dtype=torch.float64, device=dev)
    flags = torch.zeros(P, dtype=torch.int32, device=dev)
    nws = lib().ttm_snorm_workspace_bytes(L, nrot, P)
    if nws == 0:
        raise TTMError(-2, "ttm_snorm_workspace_bytes")
    ws = workspace if workspace is not None and workspace.numel() >= nws else _workspace(nws, dev)
    st = lib().ttm_snorm(_dev(image, "image"), N, _dev(tmpl, "tmpl"), _dev(mask, "mask"), L, order,
                         q.data_ptr(), w.data_ptr(), nrot, pos.data_ptr(), lam.data_ptr(),
                         count.data_ptr() if count is not None else None, P, rho.data_ptr(), D.data_ptr(),
                         flags.data_ptr(), ws.data_ptr(), nws, _stream(dev))
    _check(st, "ttm_snorm")
    return rho, D, flags


def rotation_map_workspace(image_shape, L, order, n_seeds, device) -> torch.Tensor:
    n = lib().ttm_rotation_map_workspace_bytes(_dims(image_shape), _dims(L), order, int(n_seeds))
    if n == 0:
        raise TTMError(-1, "ttm_rotation_map_workspace_bytes")
    return _workspace(n, device)


def rotation_map(image: torch.Tensor, bank: torch.Tensor, mask: torch.Tensor, order: int, seeds,
                 opt: Options | None = None, want_w: bool = False, workspace: torch.Tensor | None = None,
                 out: dict | None = None) -> dict:
    """Dominant rotation and Z-eigenvalue of C_n(x) at every valid voxel.
    ``seeds`` (n_seeds x 4 quaternions, n_seeds a multiple of 32) is a device
    tensor or array-like.  Returns (or fills ``out``, a dict of preallocated
    tensors with the same keys) score [N], w [N] or None, quat [N + (4,)],
    lam [N] and unconverged (one int32), all device tensors; nothing is
    synchronised."""
    dev = image.device
    N = _dims(image.shape)
    L = _dims(mask.shape)
    opt = opt or default_options()
    if not torch.is_tensor(seeds):
        seeds = torch.as_tensor(seeds, dtype=torch.float32, device=dev)
    sd = seeds.to(device=dev, dtype=torch.float32).contiguous()
    if sd.dim() != 2 or sd.shape[1] != 4:
        raise ValueError("seeds must be an (n_seeds, 4) array of quaternions")
    J = int(sd.shape[0])
    if out is None:
        shape = tuple(image.shape)
        out = dict(score=torch.empty(shape, dtype=torch.float32, device=dev),
                   w=torch.empty(shape, dtype=torch.float32, device=dev) if want_w else None,
                   quat=torch.empty(shape + (4,), dtype=torch.float32, device=dev),
                   lam=torch.empty(shape, dtype=torch.float32, device=dev),
                   unconverged=torch.zeros((1,), dtype=torch.int32, device=dev))
    ws = workspace if workspace is not None else rotation_map_workspace(image.shape, mask.shape, order, J, dev)
    w = out.get("w")
    st = lib().ttm_rotation_map(_dev(image, "image"), N, bank.data_ptr(), L, order, _dev(mask, "mask"),
                                ctypes.byref(opt), _dev(sd, "seeds"), J, _dev(out["score"], "score"),
                                _opt_dev(w, "w"), _dev(out["quat"], "quat"), _dev(out["lam"], "lam"),
                                _i32_dev(out.get("unconverged"), "unconverged"), ws.data_ptr(), ws.numel(),
                                _stream(dev))
    _check(st, "ttm_rotation_map")
    return out


def tile_count(N, L, tile: int) -> int:
    n = lib().ttm_tile_count(_dims(N), _dims(L), int(tile))
    if n < 0:
        raise TTMError(n, "ttm_tile_count")
    return n


def correlate_tiled(image: torch.Tensor, bank: torch.Tensor, mask: torch.Tensor, order: int, tile: int,
                    opt: Options | None = None, want_w: bool = True, workspace: torch.Tensor | None = None,
                    out=None):
    """Score F and w of an image of any extent, correlated on tile^3 FFT tiles
    (``bank`` built with image_shape = (tile, tile, tile))."""
    dev = image.device
    N = _dims(image.shape)
    L = _dims(mask.shape)
    opt = opt or default_options()
    if out is not None:
        score, w = out
    else:
        score = torch.empty_like(image)
        w = torch.empty_like(image) if want_w else None
    nws = lib().ttm_correlate_tiled_workspace_bytes(L, order, int(tile))
    if nws == 0:
        raise TTMError(-2, "ttm_correlate_tiled_workspace_bytes")
    ws = workspace if workspace is not None and workspace.numel() >= nws else _workspace(nws, dev)
    st = lib().ttm_correlate_tiled(_dev(image, "image"), N, bank.data_ptr(), L, order, int(tile),
                                   _dev(mask, "mask"), ctypes.byref(opt), _dev(score, "score"), _opt_dev(w, "w"),
                                   ws.data_ptr(), ws.numel(), _stream(dev))
    _check(st, "ttm_correlate_tiled")
    return score, w


def autotune_tiles(banks: dict, L, mask: torch.Tensor, order: int, opt: Options | None = None,
                   repeats: int = 3) -> dict:
    """Median milliseconds of one tile correlation per candidate tile edge
    (``banks``: {edge: the template's bank built at (edge, edge, edge)});
    synchronises the current stream."""
    dev = mask.device
    opt = opt or default_options()
    edges = sorted(int(t) for t in banks)
    tiles = (ctypes.c_int32 * len(edges))(*edges)
    bptr = (ctypes.c_void_p * len(edges))(*[banks[t].data_ptr() for t in edges])
    ms = (ctypes.c_float * len(edges))()
    nws = lib().ttm_autotune_workspace_bytes(_dims(L), order, ctypes.cast(tiles, _P), len(edges))
    if nws == 0:
        raise TTMError(-2, "ttm_autotune_workspace_bytes")
    ws = _workspace(nws, dev)
    st = lib().ttm_autotune_tiles(ctypes.cast(bptr, _P), ctypes.cast(tiles, _P), len(edges), _dims(L), order,
                                  _dev(mask, "mask"), ctypes.byref(opt), int(repeats), ctypes.cast(ms, _P),
                                  ws.data_ptr(), ws.numel(), _stream(dev))
    _check(st, "ttm_autotune_tiles")
    return {t: float(ms[i]) for i, t in enumerate(edges)}


def choose_tile(N, L, table: dict) -> int:
    """The tile edge of ``table`` ({edge: ms per tile}) minimising tiles x ms."""
    edges = sorted(int(t) for t in table)
    tiles = (ctypes.c_int32 * len(edges))(*edges)
    ms = (ctypes.c_float * len(edges))(*[table[t] for t in edges])
    t = lib().ttm_choose_tile(_dims(N), _dims(L), ctypes.cast(tiles, _P), ctypes.cast(ms, _P), len(edges))
    if t < 0:
        raise TTMError(t, "ttm_choose_tile")
    return t


class BatchOutputs:
    """Device outputs of one batch job: score and w maps, pose rows."""

    def __init__(self, image_shape, max_peaks: int, device, want_w: bool = False):
        self.score = torch.empty(tuple(image_shape), dtype=torch.float32, device=device)
        self.w = torch.empty(tuple(image_shape), dtype=torch.float32, device=device) if want_w else None
        P = int(max_peaks)
        self.pos = torch.zeros((P, 3), dtype=torch.int32, device=device)
        self.quat = torch.zeros((P, 4), dtype=torch.float32, device=device)
        self.lam = torch.zeros((P,), dtype=torch.float64, device=device)
        self.peak_score = torch.zeros((P,), dtype=torch.float32, device=device)
        self.flags = torch.zeros((P,), dtype=torch.int32, device=device)
        self.count = torch.zeros((2,), dtype=torch.int32, device=device)

    def result(self) -> dict:
        cnt = self.count.cpu()
        n = int(cnt[0])
        return dict(pos=self.pos[:n], quat=self.quat[:n], lam=self.lam[:n], score=self.peak_score[:n],
                    flags=self.flags[:n], truncated=bool(int(cnt[1]) & PEAKS_TRUNCATED), count=n)


def batch_job(image: torch.Tensor, bank: torch.Tensor, tile: int, components: torch.Tensor, mask: torch.Tensor,
              out: BatchOutputs, tmpl: torch.Tensor | None = None) -> BatchJob:
    """The C descriptor of one job (the tensors must outlive every use of it)."""
    j = BatchJob()
    j.image = _dev(image, "image")
    j.N = _dims(image.shape)
    j.bank = bank.data_ptr()
    j.tile = int(tile)
    j.components = _dev(components, "components")
    j.mask = _dev(mask, "mask")
    j.tmpl = _opt_dev(tmpl, "tmpl")
    j.L = _dims(mask.shape)
    j.out_score = _dev(out.score, "score")
    j.out_w = _opt_dev(out.w, "w")
    j.out_pos = out.pos.data_ptr()
    j.out_quat = out.quat.data_ptr()
    j.out_lambda = out.lam.data_ptr()
    j.out_peak_score = out.peak_score.data_ptr()
    j.out_flags = out.flags.data_ptr()
    j.out_count = out.count.data_ptr()
    return j


def _jobs_array(jobs):
    arr = (BatchJob * len(jobs))(*jobs)
    return arr, ctypes.cast(arr, _P)


def batch_workspace(jobs, order: int, opt: Options, device, n_streams: int = 1) -> torch.Tensor:
    arr, ptr = _jobs_array(jobs)
    n = lib().ttm_batch_workspace_bytes(ptr, len(jobs), order, ctypes.byref(opt), int(n_streams))
    if n == 0:
        raise TTMError(-1, "ttm_batch_workspace_bytes")
    return _workspace(n, device)


def batch_match(jobs, order: int, opt: Options, workspace: torch.Tensor, device=None, n_streams: int = 1):
    """Run the jobs eagerly on the current stream (split over ``n_streams``
    concurrent branches forked from it and joined back to it when > 1; the
    workspace from ``batch_workspace(..., n_streams)``)."""
    arr, ptr = _jobs_array(jobs)
    st = lib().ttm_batch_match(ptr, len(jobs), order, ctypes.byref(opt), int(n_streams), workspace.data_ptr(),
                               workspace.numel(), _stream(device or workspace.device))
    _check(st, "ttm_batch_match")


class BatchGraph:
    """The jobs recorded into one hipGraph (captured on a side stream, split
    over ``n_streams`` concurrent branches, the workspace from
    ``batch_workspace(..., n_streams)``); ``launch()`` replays all of them as
    one launch on the current stream.  The job tensors and the workspace must
    stay alive and unchanged."""

    def __init__(self, jobs, order: int, opt: Options, workspace: torch.Tensor, n_streams: int = 1):
        self._keep = (list(jobs), workspace, opt)
        arr, ptr = _jobs_array(jobs)
        self._handle = ctypes.c_void_p()
        dev = workspace.device
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        st = lib().ttm_batch_graph_create(ptr, len(jobs), order, ctypes.byref(opt), int(n_streams),
                                          workspace.data_ptr(), workspace.numel(), side.cuda_stream,
                                          ctypes.byref(self._handle))
        _check(st, "ttm_batch_graph_create")
        self.device = dev

    def launch(self):
        st = lib().ttm_graph_launch(self._handle, _stream(self.device))
        _check(st, "ttm_graph_launch")

    def close(self):
        if self._handle:
            lib().ttm_graph_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lowpass(x: torch.Tensor, sigma: float, periodic: bool = True, out: torch.Tensor | None = None):
    """``x * h`` for the isotropic low-pass filter (ttm_lowpass): periodic for
    images, zero-extended for template boxes."""
    dev = x.device
    N = _dims(x.shape)
    out = torch.empty_like(x) if out is None else out
    nws = lib().ttm_lowpass_workspace_bytes(N)
    ws = _workspace(nws, dev)
    st = lib().ttm_lowpass(_dev(x, "x"), N, float(sigma), 1 if periodic else 0, _dev(out, "out"), ws.data_ptr(),
                           nws, _stream(dev))
    _check(st, "ttm_lowpass")
    return out


def score_backward(image: torch.Tensor, tmpl: torch.Tensor, mask: torch.Tensor, order: int, quats, weights,
                   components: torch.Tensor, positions, grad_score: torch.Tensor, opt: Options | None = None,
                   want_tmpl: bool = True, want_image: bool = True):
    """Gradient of ``sum_p grad_score[p] F(x_p)`` with respect to the raw
    template and the image (ttm_score_backward).  Returns (grad_tmpl,
    grad_image); either is None when not requested."""
    dev = image.device
    N = _dims(image.shape)
    L = _dims(tmpl.shape)
    q = torch.as_tensor(quats, dtype=torch.float32).contiguous().cpu()
    w = torch.as_tensor(weights, dtype=torch.float64).contiguous().cpu()
    nrot = q.shape[0]
    pos = torch.as_tensor(positions, dtype=torch.int32).reshape(-1, 3).contiguous().to(dev)
    P = pos.shape[0]
    gs = grad_score.to(device=dev, dtype=torch.float32).contiguous()
    if gs.numel() != P:
        raise ValueError("grad_score needs one value per position")
    opt = opt or default_options()
    gt = torch.empty_like(tmpl) if want_tmpl else None
    gi = torch.empty_like(image) if want_image else None
    nws = lib().ttm_score_backward_workspace_bytes(L, order, nrot, P)
    ws = _workspace(nws, dev)
    st = lib().ttm_score_backward(_dev(image, "image"), N, _dev(tmpl, "tmpl"), _dev(mask, "mask"), L, order,
                                  q.data_ptr(), w.data_ptr(), nrot, _dev(components, "components"),
                                  pos.data_ptr(), P, gs.data_ptr(), ctypes.byref(opt),
                                  gt.data_ptr() if gt is not None else None,
                                  gi.data_ptr() if gi is not None else None, ws.data_ptr(), nws, _stream(dev))
    _check(st, "ttm_score_backward")
    return gt, gi


class TTMScore(torch.autograd.Function):
    """F(x_p) at fixed positions as a differentiable function of the raw
    template and the image.  Forward: the tensor template and its spectra are
    rebuilt from the template (ttm_build_tensor_template) and the image is
    correlated (ttm_correlate); F is read at the positions.  Backward:
    ttm_score_backward.  Use ``TTMScore.apply(tmpl, image, mask, order,
    quats, weights, positions, opt)``."""

    @staticmethod
    def forward(ctx, tmpl, image, mask, order, quats, weights, positions, opt=None):
        comps, bank = build_tensor_template(tmpl, mask, order, quats, weights, image_shape=image.shape)
        score, _ = correlate(image, bank, mask, order, opt, want_w=False)
        pos = torch.as_tensor(positions, dtype=torch.long).reshape(-1, 3).to(image.device)
        F = score[pos[:, 0], pos[:, 1], pos[:, 2]]
        ctx.save_for_backward(tmpl, image, mask, comps)
        ctx.args = (order, quats, weights, pos.to(torch.int32), opt)
        return F

    @staticmethod
    def backward(ctx, grad_F):
        tmpl, image, mask, comps = ctx.saved_tensors
        order, quats, weights, pos, opt = ctx.args
        gt, gi = score_backward(image, tmpl, mask, order, quats, weights, comps, pos, grad_F, opt,
                                want_tmpl=ctx.needs_input_grad[0], want_image=ctx.needs_input_grad[1])
        return gt, gi, None, None, None, None, None, None


def tm_classical(image: torch.Tensor, tmpl: torch.Tensor, mask: torch.Tensor, quats,
                 opt: Options | None = None):
    """Best NCC over the rotation list and its index, per voxel."""
    dev = image.device
    N = _dims(image.shape)
    L = _dims(tmpl.shape)
    q = torch.as_tensor(quats, dtype=torch.float32).contiguous().cpu()
    nrot = q.shape[0]
    opt = opt or default_options()
    best = torch.empty_like(image)
    idx = torch.empty(image.shape, dtype=torch.int32, device=dev)
    nws = lib().tm_classical_workspace_bytes(N, L, nrot)
    ws = _workspace(nws, dev)
    st = lib().tm_classical(_dev(image, "image"), N, _dev(tmpl, "tmpl"), _dev(mask, "mask"), L,
                            q.data_ptr(), nrot, ctypes.byref(opt), best.data_ptr(), idx.data_ptr(),
                            ws.data_ptr(), nws, _stream(dev))
    _check(st, "tm_classical")
    return best, idx
