"""Python binding of libhtsvd (MI355X Haar-tSVD denoising).

Argument marshalling only: every step of the method runs in the HIP kernels of
libhtsvd.so.  PyTorch supplies device memory and the current stream.  The
functions named htsvd_* mirror the C ABI of include/htsvd.h one to one; the
Denoiser class is a small convenience layer over them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhtsvd.so")
DATA_DIR = os.path.join(_HERE, "data")

HTSVD_OK, HTSVD_EINVAL, HTSVD_ESHAPE, HTSVD_ENOMEM, HTSVD_EDEVICE, HTSVD_ENOTSUP, HTSVD_ESTATE = 0, -1, -2, -3, -4, -5, -6
HTSVD_NOALLOC_SCRATCH_BYTES = 64 << 20
HTSVD_SIGMA_AUTO = -1.0
HTSVD_K_AUTO = -1
_STATUS = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ENOMEM", -4: "EDEVICE", -5: "ENOTSUP", -6: "ESTATE"}


class htsvd_params(ctypes.Structure):
    _fields_ = [
        ("ps", ctypes.c_int32), ("stride", ctypes.c_int32), ("window", ctypes.c_int32), ("K", ctypes.c_int32),
        ("tau_mult", ctypes.c_double), ("adaptive", ctypes.c_int32), ("beta", ctypes.c_double),
        ("gamma_rank", ctypes.c_int32), ("gcp_num", ctypes.c_int32), ("gcp_den", ctypes.c_int32),
        ("estimator", ctypes.c_int32), ("subimage", ctypes.c_int32), ("n_vote", ctypes.c_int32),
        ("vote_seed", ctypes.c_uint64), ("ra", ctypes.c_int32), ("ra_sigma", ctypes.c_double),
    ]

    def replace(self, **kw) -> "htsvd_params":
        p = htsvd_params()
        ctypes.pointer(p)[0] = self
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class htsvd_image(ctypes.Structure):
    _fields_ = [
        ("d_in", ctypes.c_void_p), ("h", ctypes.c_int32), ("w", ctypes.c_int32), ("c", ctypes.c_int32),
        ("in_stride", ctypes.c_int64), ("sigma", ctypes.c_float), ("K", ctypes.c_int32),
        ("d_out", ctypes.c_void_p), ("out_stride", ctypes.c_int64),
    ]


class htsvd_sweep_item(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_float), ("K", ctypes.c_int32), ("d_out", ctypes.c_void_p),
                ("out_stride", ctypes.c_int64)]


class htsvd_batch_opts(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("k_sigma_cutoff", ctypes.c_float), ("tile_side", ctypes.c_int32)]


class HtsvdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS.get(status, "?"), status, msg))
        self.status = status


_lib = None

# C signatures: name -> (restype, argtypes)
_i32, _i64, _f32, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p
_PP = ctypes.POINTER(htsvd_params)
_SIGS = {
    "htsvd_create": (_i32, [ctypes.POINTER(_vp), ctypes.c_int]),
    "htsvd_destroy": (None, [_vp]),
    "htsvd_default_params": (_i32, [_i32, _PP]),
    "htsvd_set_basis": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "htsvd_ref_count": (_i32, [_i32, _i32, _i32]),
    "htsvd_basis_gram": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _i32, _i32, _vp, _vp]),
    "htsvd_learn_basis": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _i32, _i32, _vp, _vp, _vp]),
    "htsvd_block_match": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _PP, _vp, _vp, _vp]),
    "htsvd_denoise": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _f32, _PP, _vp, _i64, _vp]),
    "htsvd_denoise_tau": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _vp, _PP, _vp, _i64, _vp]),
    "htsvd_denoise_noalloc": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _f32, _PP, _vp, _i64, _vp]),
    "htsvd_denoise_sweep": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _i32, ctypes.POINTER(htsvd_sweep_item), _PP,
                                   _vp]),
    "htsvd_denoise_batch": (_i32, [_vp, _i32, ctypes.POINTER(htsvd_image), _PP, ctypes.POINTER(htsvd_batch_opts), _vp]),
    "htsvd_estimate_sigma": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _f32, _PP, _vp, _vp, _vp, _vp, _vp]),
    "htsvd_batch_inspect": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "htsvd_sync": (_i32, [_vp, _vp]),
    "htsvd_last_error": (ctypes.c_char_p, []),
    "htsvd_last_guard_count": (_i32, [_vp, _vp]),
    "htsvd_cnn_param_count": (_i32, [_i32]),
    "htsvd_cnn_init": (_i32, [_vp, _i32, ctypes.c_uint64]),
    "htsvd_cnn_set_weights": (_i32, [_vp, _i32, _vp, _i64]),
    "htsvd_cnn_get_weights": (_i32, [_vp, _vp, _i64]),
    "htsvd_cnn_forward": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _vp, _vp]),
    "htsvd_cnn_gradients": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "htsvd_cnn_train_step": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _f32, _vp, _vp]),
    "htsvd_cnn_save": (_i32, [_vp, ctypes.c_char_p]),
    "htsvd_cnn_load": (_i32, [_vp, ctypes.c_char_p]),
    "htsvd_band_guide": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _vp, _vp]),
    "htsvd_denoise_bands": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _f32, _PP, _vp, _i64, _vp]),
    "htsvd_set_band_memory": (_i32, [_vp, _i64]),
    "htsvd_band_sigma": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _vp, _vp]),
    "htsvd_block_match_video": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _i64, _i32, _PP, _vp, _vp, _vp]),
    "htsvd_denoise_video": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _i64, _i32, _f32, _PP, _vp, _i64, _vp]),
    "htsvd_ra_param_count": (_i32, [_i32]),
    "htsvd_ra_set_weights": (_i32, [_vp, _i32, _vp, _i64]),
    "htsvd_ra_get_weights": (_i32, [_vp, _i32, _vp, _i64]),
    "htsvd_ra_means": (_i32, [_vp, _vp, _i32, _i32, _i32, _i64, _vp, _i32, _i64, _vp, _vp]),
    "htsvd_ra_forward": (_i32, [_vp, _i32, _vp, _i64, _vp, _vp]),
    "htsvd_ra_gradients": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp]),
    "htsvd_ra_train_step": (_i32, [_vp, _i32, _vp, _vp, _i32, _f32, _vp, _vp]),
    "htsvd_set_timing": (_i32, [_vp, _i32]),
    "htsvd_stage_times": (_i32, [_vp, _vp, _vp]),
}
STAGES = ["bm", "clear", "filter", "normalize", "sigma"]


def lib():
    """Loads libhtsvd.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhtsvd.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2512_23569_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS.keys())


def _check(status: int):
    if status != HTSVD_OK:
        raise HtsvdError(status, lib().htsvd_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, dtype=None, name="tensor"):
    """Device pointer of a contiguous CUDA (HIP) tensor, or None."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _img_dims(t):
    if t.dim() == 2:
        h, w = t.shape
        c = 1
    elif t.dim() == 3:
        h, w, c = t.shape
    else:
        raise ValueError("image must be (h, w) or (h, w, c)")
    if t.stride(-1) != 1 and c > 1:
        raise ValueError("channels must be contiguous")
    if c > 1 and t.stride(1) != c:
        raise ValueError("pixels of a row must be contiguous")
    in_stride = t.stride(0)
    return int(h), int(w), int(c), int(in_stride)


# ---- one-to-one mirrors of the C ABI -------------------------------------------

def htsvd_create(device: int = 0):
    h = ctypes.c_void_p()
    _check(lib().htsvd_create(ctypes.byref(h), device))
    return h


def htsvd_destroy(ctx):
    lib().htsvd_destroy(ctx)


def htsvd_default_params(c: int) -> htsvd_params:
    p = htsvd_params()
    _check(lib().htsvd_default_params(c, ctypes.byref(p)))
    return p


def htsvd_set_basis(ctx, ps: int, c: int, U_slices: np.ndarray, V_slices: np.ndarray):
    u = np.ascontiguousarray(U_slices, dtype=np.float64).reshape(-1)
    v = np.ascontiguousarray(V_slices, dtype=np.float64).reshape(-1)
    _check(lib().htsvd_set_basis(ctx, ps, c, u.ctypes.data_as(_vp), v.ctypes.data_as(_vp)))


def htsvd_ref_count(n: int, ps: int, stride: int) -> int:
    return int(lib().htsvd_ref_count(n, ps, stride))


def htsvd_basis_gram(ctx, d_in, h, w, c, in_stride, ps, stride, d_gram, stream=None):
    import torch
    _check(lib().htsvd_basis_gram(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride, ps, stride,
                                  _dptr(d_gram, torch.int64, "d_gram"), _stream(stream)))


def htsvd_learn_basis(ctx, d_in, h, w, c, in_stride, ps, stride, stream=None):
    """Returns the learned pair as slice-major (c, ps, ps) FP64 arrays (also installed in ctx)."""
    import torch
    U = np.zeros((c, ps, ps), dtype=np.float64)
    V = np.zeros((c, ps, ps), dtype=np.float64)
    _check(lib().htsvd_learn_basis(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride, ps, stride,
                                   U.ctypes.data_as(_vp), V.ctypes.data_as(_vp), _stream(stream)))
    return U, V


def htsvd_block_match(ctx, d_in, h, w, c, in_stride, params, d_idx, d_dist=None, stream=None):
    import torch
    _check(lib().htsvd_block_match(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride, ctypes.byref(params),
                                   _dptr(d_idx, torch.int32, "d_idx"), _dptr(d_dist, torch.int32, "d_dist"),
                                   _stream(stream)))


def htsvd_denoise(ctx, d_in, h, w, c, in_stride, sigma, params, d_out, out_stride, stream=None):
    import torch
    _check(lib().htsvd_denoise(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride, float(sigma),
                               ctypes.byref(params), _dptr(d_out, torch.float32, "d_out"), out_stride,
                               _stream(stream)))


def htsvd_denoise_noalloc(ctx, d_in, h, w, c, in_stride, sigma, params, d_out, out_stride, stream=None):
    """htsvd_denoise with its scratch in the library's fixed per-GPU array (no allocation)."""
    import torch
    _check(lib().htsvd_denoise_noalloc(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride, float(sigma),
                                       ctypes.byref(params), _dptr(d_out, torch.float32, "d_out"), out_stride,
                                       _stream(stream)))


def htsvd_denoise_tau(ctx, d_in, h, w, c, in_stride, d_tau_ref, params, d_out, out_stride, stream=None):
    import torch
    _check(lib().htsvd_denoise_tau(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride,
                                   _dptr(d_tau_ref, torch.float64, "d_tau_ref"), ctypes.byref(params),
                                   _dptr(d_out, torch.float32, "d_out"), out_stride, _stream(stream)))


def htsvd_denoise_batch(ctx, images, params, use_graph=1, blocks_per_cu=1, k_sigma_cutoff=0.0, tile_side=0,
                        stream=None):
    """images: a sequence of htsvd_image (device pointers filled in by the caller)."""
    arr = (htsvd_image * len(images))(*images)
    opts = htsvd_batch_opts(int(use_graph), int(blocks_per_cu), float(k_sigma_cutoff), int(tile_side))
    _check(lib().htsvd_denoise_batch(ctx, len(images), arr, ctypes.byref(params), ctypes.byref(opts),
                                     _stream(stream)))


def htsvd_denoise_sweep(ctx, d_in, h, w, c, in_stride, items, params, stream=None):
    """items: a sequence of htsvd_sweep_item (device output pointers filled in by the caller)."""
    import torch
    arr = (htsvd_sweep_item * len(items))(*items)
    _check(lib().htsvd_denoise_sweep(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride, len(items), arr,
                                     ctypes.byref(params), _stream(stream)))


def htsvd_estimate_sigma(ctx, d_in, h, w, c, in_stride, sigma, params, d_sigma_est=None, d_sigma_hat=None,
                         d_votes=None, d_sigma_map=None, stream=None):
    import torch
    _check(lib().htsvd_estimate_sigma(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride, float(sigma),
                                      ctypes.byref(params), _dptr(d_sigma_est, torch.float64, "d_sigma_est"),
                                      _dptr(d_sigma_hat, torch.float64, "d_sigma_hat"),
                                      _dptr(d_votes, torch.int32, "d_votes"),
                                      _dptr(d_sigma_map, torch.float64, "d_sigma_map"), _stream(stream)))


def htsvd_batch_inspect(ctx, image, d_tau_ref=None, stream=None) -> int:
    """Group size of image `image` of the last batch (after the device's K choice); fills
    d_tau_ref with the thresholds its filter applied when given."""
    import torch
    k = ctypes.c_int32(0)
    _check(lib().htsvd_batch_inspect(ctx, int(image), ctypes.byref(k), _dptr(d_tau_ref, torch.float64, "d_tau_ref"),
                                     _stream(stream)))
    return int(k.value)


def htsvd_sync(ctx, stream=None):
    _check(lib().htsvd_sync(ctx, _stream(stream)))


def htsvd_last_error() -> str:
    return lib().htsvd_last_error().decode()


def htsvd_last_guard_count(ctx):
    out = (ctypes.c_int64 * 2)()
    _check(lib().htsvd_last_guard_count(ctx, ctypes.cast(out, _vp)))
    return int(out[0]), int(out[1])


def htsvd_set_timing(ctx, enable: bool):
    _check(lib().htsvd_set_timing(ctx, 1 if enable else 0))


def htsvd_stage_times(ctx):
    """{stage: (total ms, timed calls)} since timing was enabled."""
    ms = (ctypes.c_double * len(STAGES))()
    calls = (ctypes.c_int64 * len(STAGES))()
    _check(lib().htsvd_stage_times(ctx, ctypes.cast(ms, _vp), ctypes.cast(calls, _vp)))
    return {s: (float(ms[i]), int(calls[i])) for i, s in enumerate(STAGES)}


def htsvd_cnn_param_count(c: int) -> int:
    return int(lib().htsvd_cnn_param_count(c))


def htsvd_cnn_init(ctx, c: int, seed: int = 0):
    _check(lib().htsvd_cnn_init(ctx, c, seed))


def htsvd_cnn_set_weights(ctx, c: int, params: np.ndarray):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().htsvd_cnn_set_weights(ctx, c, a.ctypes.data_as(_vp), a.size))


def htsvd_cnn_get_weights(ctx, c: int) -> np.ndarray:
    a = np.zeros(htsvd_cnn_param_count(c), dtype=np.float32)
    _check(lib().htsvd_cnn_get_weights(ctx, a.ctypes.data_as(_vp), a.size))
    return a


def htsvd_cnn_forward(ctx, d_in, h, w, c, in_stride, d_log_sigma, stream=None):
    import torch
    _check(lib().htsvd_cnn_forward(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride,
                                   _dptr(d_log_sigma, torch.float32, "d_log_sigma"), _stream(stream)))


def htsvd_cnn_gradients(ctx, d_crops, n, h, w, c, d_target_log, d_grad, stream=None) -> float:
    import torch
    loss = ctypes.c_double(0.0)
    _check(lib().htsvd_cnn_gradients(ctx, _dptr(d_crops, torch.uint8, "d_crops"), n, h, w, c,
                                     _dptr(d_target_log, torch.float32, "d_target_log"),
                                     _dptr(d_grad, torch.float32, "d_grad"), ctypes.byref(loss), _stream(stream)))
    return float(loss.value)


def htsvd_cnn_train_step(ctx, d_crops, n, h, w, c, d_target_log, lr, want_loss=True, stream=None):
    import torch
    loss = ctypes.c_double(0.0)
    _check(lib().htsvd_cnn_train_step(ctx, _dptr(d_crops, torch.uint8, "d_crops"), n, h, w, c,
                                      _dptr(d_target_log, torch.float32, "d_target_log"), float(lr),
                                      ctypes.byref(loss) if want_loss else None, _stream(stream)))
    return float(loss.value) if want_loss else None


def htsvd_cnn_save(ctx, path: str):
    _check(lib().htsvd_cnn_save(ctx, path.encode()))


def htsvd_cnn_load(ctx, path: str):
    _check(lib().htsvd_cnn_load(ctx, path.encode()))


def htsvd_band_guide(ctx, d_in, h, w, bands, in_stride, d_guide, stream=None):
    import torch
    _check(lib().htsvd_band_guide(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, bands, in_stride,
                                  _dptr(d_guide, torch.uint8, "d_guide"), _stream(stream)))


def htsvd_band_sigma(ctx, d_in, h, w, bands, in_stride, stream=None) -> np.ndarray:
    """Band-wise noise levels (bands,) FP64 on the host."""
    import torch
    out = np.zeros(bands, dtype=np.float64)
    _check(lib().htsvd_band_sigma(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, bands, in_stride,
                                  out.ctypes.data_as(_vp), _stream(stream)))
    return out


def htsvd_set_band_memory(ctx, nbytes: int):
    _check(lib().htsvd_set_band_memory(ctx, int(nbytes)))


def htsvd_denoise_bands(ctx, d_in, h, w, bands, in_stride, sigma, params, d_out, out_stride, stream=None):
    import torch
    _check(lib().htsvd_denoise_bands(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, bands, in_stride, float(sigma),
                                     ctypes.byref(params), _dptr(d_out, torch.float32, "d_out"), out_stride,
                                     _stream(stream)))


def htsvd_block_match_video(ctx, d_in, T, h, w, c, in_stride, radius, params, d_idx, d_dist=None, stream=None):
    import torch
    _check(lib().htsvd_block_match_video(ctx, _dptr(d_in, torch.uint8, "d_in"), T, h, w, c, in_stride, radius,
                                         ctypes.byref(params), _dptr(d_idx, torch.int32, "d_idx"),
                                         _dptr(d_dist, torch.int32, "d_dist"),
                                         _stream(stream)))


def htsvd_denoise_video(ctx, d_in, T, h, w, c, in_stride, radius, sigma, params, d_out, out_stride, stream=None):
    import torch
    _check(lib().htsvd_denoise_video(ctx, _dptr(d_in, torch.uint8, "d_in"), T, h, w, c, in_stride, radius,
                                     float(sigma), ctypes.byref(params), _dptr(d_out, torch.float32, "d_out"),
                                     out_stride, _stream(stream)))


def htsvd_ra_param_count(c: int) -> int:
    return int(lib().htsvd_ra_param_count(c))


def htsvd_ra_set_weights(ctx, c: int, params: np.ndarray):
    a = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    _check(lib().htsvd_ra_set_weights(ctx, c, a.ctypes.data_as(_vp), a.size))


def htsvd_ra_get_weights(ctx, c: int) -> np.ndarray:
    a = np.zeros(htsvd_ra_param_count(c), dtype=np.float32)
    _check(lib().htsvd_ra_get_weights(ctx, c, a.ctypes.data_as(_vp), a.size))
    return a


def htsvd_ra_means(ctx, d_in, h, w, c, in_stride, d_idx, K, n_ref, d_means, stream=None):
    import torch
    _check(lib().htsvd_ra_means(ctx, _dptr(d_in, torch.uint8, "d_in"), h, w, c, in_stride,
                                _dptr(d_idx, torch.int32, "d_idx"), K, n_ref, _dptr(d_means, torch.float32, "d_means"),
                                _stream(stream)))


def htsvd_ra_forward(ctx, c, d_means, n, d_r, stream=None):
    import torch
    _check(lib().htsvd_ra_forward(ctx, c, _dptr(d_means, torch.float32, "d_means"), n,
                                  _dptr(d_r, torch.float32, "d_r"), _stream(stream)))


def htsvd_ra_gradients(ctx, c, d_noisy, d_clean, n, d_grad, stream=None) -> float:
    import torch
    loss = ctypes.c_double(0.0)
    _check(lib().htsvd_ra_gradients(ctx, c, _dptr(d_noisy, torch.float32, "d_noisy"),
                                    _dptr(d_clean, torch.float32, "d_clean"), n, _dptr(d_grad, torch.float32, "d_grad"),
                                    ctypes.byref(loss), _stream(stream)))
    return loss.value


def htsvd_ra_train_step(ctx, c, d_noisy, d_clean, n, lr, want_loss=True, stream=None):
    import torch
    loss = ctypes.c_double(0.0)
    _check(lib().htsvd_ra_train_step(ctx, c, _dptr(d_noisy, torch.float32, "d_noisy"),
                                     _dptr(d_clean, torch.float32, "d_clean"), n, float(lr),
                                     ctypes.byref(loss) if want_loss else None, _stream(stream)))
    return loss.value if want_loss else None


# ---- convenience layer ------------------------------------------------------------

def load_basis_slices(c: int, ps: int = 8):
    """The shipped basis pair for c channels as slice-major (c, ps, ps) FP64 arrays."""
    raw = np.fromfile(os.path.join(DATA_DIR, "basis_ps8_c%d.f64" % c), dtype="<f8")
    n = ps * ps * c
    return raw[:n].reshape(c, ps, ps), raw[n:].reshape(c, ps, ps)


class Denoiser:
    """Owns one library context on one device, with the shipped bases loaded."""

    def __init__(self, device: int = 0, load_network: bool = True):
        self.device = device
        self.ctx = htsvd_create(device)
        for c in (1, 3):
            U, V = load_basis_slices(c)
            htsvd_set_basis(self.ctx, 8, c, U, V)
        net = os.path.join(DATA_DIR, "sigma_cnn_c3.ckpt")
        if load_network and os.path.exists(net):
            htsvd_cnn_load(self.ctx, net)
        for c in (1, 3):
            ra = os.path.join(DATA_DIR, "ra_fcn_c%d.f32" % c)
            if load_network and os.path.exists(ra):
                htsvd_ra_set_weights(self.ctx, c, np.fromfile(ra, dtype="<f4"))

    def close(self):
        if self.ctx is not None:
            htsvd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def params(c: int, **kw) -> htsvd_params:
        return htsvd_default_params(c).replace(**kw)

    def block_match(self, img, params, with_dist=True, stream=None):
        import torch
        h, w, c, st = _img_dims(img)
        n_ref = htsvd_ref_count(h, 8, params.stride) * htsvd_ref_count(w, 8, params.stride)
        idx = torch.empty((n_ref, params.K), dtype=torch.int32, device=img.device)
        dist = torch.empty((n_ref, params.K), dtype=torch.int32, device=img.device) if with_dist else None
        htsvd_block_match(self.ctx, img, h, w, c, st, params, idx, dist, stream)
        return idx, dist

    def basis_gram(self, img, stride=4, stream=None):
        """Channel Gram sums (2, c, c, 8, 8) int64 of the image's reference patches."""
        import torch
        h, w, c, st = _img_dims(img)
        out = torch.empty((2, c, c, 8, 8), dtype=torch.int64, device=img.device)
        htsvd_basis_gram(self.ctx, img, h, w, c, st, 8, stride, out, stream)
        return out

    def learn_basis(self, img, stride=4, stream=None):
        """Learns the basis pair from this image and makes it the one used for its channel
        count; returns (U, V) slice-major (c, 8, 8) FP64."""
        h, w, c, st = _img_dims(img)
        return htsvd_learn_basis(self.ctx, img, h, w, c, st, 8, stride, stream)

    def denoise(self, img, sigma, params, out=None, stream=None):
        import torch
        h, w, c, st = _img_dims(img)
        if out is None:
            out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
        htsvd_denoise(self.ctx, img, h, w, c, st, sigma, params, out, out.stride(0), stream)
        return out

    def denoise_tau(self, img, tau_ref, params, out=None, stream=None):
        import torch
        h, w, c, st = _img_dims(img)
        if out is None:
            out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
        htsvd_denoise_tau(self.ctx, img, h, w, c, st, tau_ref, params, out, out.stride(0), stream)
        return out

    def denoise_batch(self, imgs, sigmas, params, Ks=None, outs=None, use_graph=True, blocks_per_cu=1,
                      k_sigma_cutoff=0.0, tile_side=0, stream=None):
        """Denoises a list of uint8 device images in one batched call; sigma HTSVD_SIGMA_AUTO
        (-1) estimates the level, K HTSVD_K_AUTO (-1) picks 16 or 32 on the device.  Returns the
        list of float32 outputs."""
        import torch
        if outs is None:
            outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in imgs]
        descs = []
        for i, x in enumerate(imgs):
            h, w, c, st = _img_dims(x)
            _dptr(x, torch.uint8, "image")
            _dptr(outs[i], torch.float32, "output")
            descs.append(htsvd_image(x.data_ptr(), h, w, c, st, float(sigmas[i]), int(Ks[i]) if Ks else 0,
                                     outs[i].data_ptr(), outs[i].stride(0)))
        htsvd_denoise_batch(self.ctx, descs, params, use_graph, blocks_per_cu, k_sigma_cutoff, tile_side, stream)
        return outs

    def denoise_sweep(self, img, settings, params, outs=None, stream=None):
        """Denoises one device image under several (sigma, K) settings with one grouping pass
        (params.K members, the largest K of the settings or more).  Returns the outputs."""
        import torch
        h, w, c, st = _img_dims(img)
        if outs is None:
            outs = [torch.empty(img.shape, dtype=torch.float32, device=img.device) for _ in settings]
        items = []
        for (sigma, K), o in zip(settings, outs):
            _dptr(o, torch.float32, "output")
            items.append(htsvd_sweep_item(float(sigma), int(K), o.data_ptr(), o.stride(0)))
        htsvd_denoise_sweep(self.ctx, img, h, w, c, st, items, params, stream)
        return outs

    def ra_means(self, img, idx, K, stream=None):
        """Mean patches (n_ref, 64c) FP32 of the groups idx (n_ref, K) over the device image."""
        import torch
        h, w, c, st = _img_dims(img)
        n_ref = idx.shape[0]
        out = torch.empty((n_ref, 64 * c), dtype=torch.float32, device=img.device)
        htsvd_ra_means(self.ctx, img, h, w, c, st, idx.contiguous(), K, n_ref, out, stream)
        return out

    def ra_forward(self, means, c, stream=None):
        """Network output r (n, 64c) for mean patches (n, 64c)."""
        import torch
        out = torch.empty_like(means)
        htsvd_ra_forward(self.ctx, c, means.contiguous(), means.shape[0], out, stream)
        return out

    def band_guide(self, cube, stream=None):
        """Gray grouping guide (h, w) uint8 of a device cube (h, w, bands)."""
        import torch
        h, w, b = cube.shape
        out = torch.empty((h, w), dtype=torch.uint8, device=cube.device)
        htsvd_band_guide(self.ctx, cube, h, w, b, cube.stride(0), out, stream)
        return out

    def band_sigma(self, cube, stream=None):
        """Band-wise noise levels of a device cube (h, w, bands) uint8: (bands,) FP64."""
        h, w, b = cube.shape
        return htsvd_band_sigma(self.ctx, cube, h, w, b, cube.stride(0), stream)

    def denoise_bands(self, cube, sigma, params, out=None, stream=None):
        """Hyperspectral denoising of a device cube (h, w, bands) uint8 with a known sigma, or
        HTSVD_SIGMA_AUTO for the band-wise noise rule; the basis for this band count comes from
        htsvd_set_basis or learn_basis."""
        import torch
        h, w, b = cube.shape
        if cube.stride(2) != 1 or cube.stride(1) != b:
            raise ValueError("bands of a pixel must be contiguous")
        if out is None:
            out = torch.empty(cube.shape, dtype=torch.float32, device=cube.device)
        htsvd_denoise_bands(self.ctx, cube, h, w, b, cube.stride(0), sigma, params, out, out.stride(0), stream)
        return out

    @staticmethod
    def _video_dims(frames):
        if frames.dim() == 3:
            T, h, w = frames.shape
            c = 1
        elif frames.dim() == 4:
            T, h, w, c = frames.shape
        else:
            raise ValueError("frames must be (T, h, w) or (T, h, w, c)")
        if not frames.is_contiguous():
            raise ValueError("frames must be contiguous")
        return T, h, w, c

    def block_match_video(self, frames, params, radius, with_dist=True, stream=None):
        """Spatio-temporal groups of device frames (T, h, w[, c]) uint8: idx (T*ny*nx, K) of
        (f*h + y)*w + x in the frames stacked vertically, and the distances."""
        import torch
        T, h, w, c = self._video_dims(frames)
        n_ref = T * htsvd_ref_count(h, 8, params.stride) * htsvd_ref_count(w, 8, params.stride)
        idx = torch.empty((n_ref, params.K), dtype=torch.int32, device=frames.device)
        dist = torch.empty((n_ref, params.K), dtype=torch.int32, device=frames.device) if with_dist else None
        htsvd_block_match_video(self.ctx, frames, T, h, w, c, w * c, radius, params, idx, dist, stream)
        return idx, dist

    def denoise_video(self, frames, sigma, params, radius, out=None, stream=None):
        """Video denoising with a known sigma: float32 frames of the input's shape."""
        import torch
        T, h, w, c = self._video_dims(frames)
        if out is None:
            out = torch.empty(frames.shape, dtype=torch.float32, device=frames.device)
        elif not out.is_contiguous() or out.shape != frames.shape:
            raise ValueError("out must be contiguous and of the frames' shape")
        htsvd_denoise_video(self.ctx, frames, T, h, w, c, w * c, radius, sigma, params, out, w * c, stream)
        return out

    def guard_count(self):
        return htsvd_last_guard_count(self.ctx)

    def sigma_map(self, img, stream=None):
        """Learned log(sigma) per 8x8 block, shape (ceil(h/8), ceil(w/8))."""
        import torch
        h, w, c, st = _img_dims(img)
        out = torch.empty(((h + 7) // 8, (w + 7) // 8), dtype=torch.float32, device=img.device)
        htsvd_cnn_forward(self.ctx, img, h, w, c, st, out, stream)
        return out
