"""Python binding of libmelt, the MI355X (gfx950) MelT frontend library.

The functions below carry the names of the C ABI in ``include/melt.h`` and only marshal
arguments: every step of the computation runs in the library's HIP kernels.  PyTorch is
used for device memory and streams; tensors are passed by ``data_ptr()`` and the current
HIP stream.  If the library is not built, importing works but every call raises
``MeltLibraryMissing``: there is no CPU fallback.

High-level helpers: :class:`MeltPlan` (owns a plan), :func:`melt_logmel` and
:class:`MeltFunction` (``torch.autograd.Function`` over ``melt_forward_proj`` /
``melt_backward``).
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "_lib" / "libmelt.so"

# enums of melt.h
MELT_OK, MELT_E_INVALID_ARG, MELT_E_UNSUPPORTED, MELT_E_NO_MEMORY, MELT_E_HIP, MELT_E_SHAPE = range(6)
MELT_WIN_HANN_SYMMETRIC, MELT_WIN_HANN_PERIODIC, MELT_WIN_RECT = range(3)
MELT_MEL_HTK, MELT_MEL_SLANEY = range(2)
MELT_PLACE_FILTER_CENTRES, MELT_PLACE_LINSPACE = range(2)
MELT_FB_NORM_NONE, MELT_FB_NORM_SLANEY = range(2)
MELT_OUT_LOG_POWER, MELT_OUT_LOG_MAGNITUDE, MELT_OUT_POWER, MELT_OUT_MAGNITUDE, MELT_OUT_MFCC = range(5)
(MELT_PREC_FP32, MELT_PREC_BF16, MELT_PREC_FP16, MELT_PREC_FP8_E4M3, MELT_PREC_BF16X3, MELT_PREC_FP16X3,
 MELT_PREC_FP8_E4M3_BLOCK32) = range(7)
# "fp8b": E4M3 with power-of-two scales per 32-sample block of the waveform
PRECISIONS = {"fp32": MELT_PREC_FP32, "bf16": MELT_PREC_BF16, "fp16": MELT_PREC_FP16,
              "fp8": MELT_PREC_FP8_E4M3, "bf16x3": MELT_PREC_BF16X3, "fp16x3": MELT_PREC_FP16X3,
              "fp8b": MELT_PREC_FP8_E4M3_BLOCK32}


class MeltLibraryMissing(RuntimeError):
    pass


class MeltError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {melt_status_string(status)}: {melt_last_error()}")


class melt_config(ctypes.Structure):
    _fields_ = [("sample_rate", ctypes.c_double), ("n_fft", ctypes.c_int32), ("hop", ctypes.c_int32),
                ("window", ctypes.c_int32), ("n_mels", ctypes.c_int32), ("fmin", ctypes.c_double),
                ("fmax", ctypes.c_double), ("mel_formula", ctypes.c_int32), ("placement", ctypes.c_int32),
                ("output", ctypes.c_int32), ("log_eps", ctypes.c_double), ("precision", ctypes.c_int32),
                ("fb_norm", ctypes.c_int32), ("n_mfcc", ctypes.c_int32)]


_lib = None
_SYMBOLS = {
    # name: (restype, argtypes)
    "melt_config_default": (ctypes.c_int, [ctypes.POINTER(melt_config)]),
    "melt_num_frames": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "melt_plan_create": (ctypes.c_int, [ctypes.POINTER(melt_config), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "melt_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "melt_plan_get_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(melt_config)]),
    "melt_plan_get_frequencies": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "melt_plan_get_basis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "melt_plan_set_basis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "melt_frame_offsets": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "melt_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "melt_forward_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "melt_forward_proj": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "stft_mel_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "melt_batch_prepare": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_void_p]),
    "melt_forward_prepared": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "stft_mel_forward_prepared": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "melt_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "melt_stream_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "melt_stream_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "melt_stream_reset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "melt_stream_max_frames": (ctypes.c_int32, [ctypes.c_void_p]),
    "melt_stream_push": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "melt_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_char_p, ctypes.c_int32]),
    "melt_variant_count": (ctypes.c_int32, [ctypes.c_void_p]),
    "melt_variant_name": (ctypes.c_char_p, [ctypes.c_void_p, ctypes.c_int32]),
    "melt_set_variant": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "melt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "melt_last_error": (ctypes.c_char_p, []),
}


def library_path() -> Path:
    return LIB_PATH


def load_library() -> ctypes.CDLL:
    """Loads libmelt.so (built by ``paper_2606_01009_amd.build``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise MeltLibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                                     f"python -m paper_2606_01009_amd.build")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in _SYMBOLS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SYMBOLS)


def _check(status, where):
    if status != MELT_OK:
        raise MeltError(status, where)


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ C-ABI mirrors

def melt_status_string(status: int) -> str:
    return load_library().melt_status_string(status).decode()


def melt_last_error() -> str:
    return load_library().melt_last_error().decode()


def melt_config_default() -> melt_config:
    c = melt_config()
    _check(load_library().melt_config_default(ctypes.byref(c)), "melt_config_default")
    return c


def melt_num_frames(n_samples: int, n_fft: int, hop: int) -> int:
    return int(load_library().melt_num_frames(int(n_samples), n_fft, hop))


def melt_plan_create(cfg: melt_config, device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load_library().melt_plan_create(ctypes.byref(cfg), device, ctypes.byref(h)), "melt_plan_create")
    return h


def melt_plan_destroy(plan) -> None:
    _check(load_library().melt_plan_destroy(plan), "melt_plan_destroy")


def melt_plan_get_frequencies(plan, n_mels: int) -> np.ndarray:
    out = np.empty(n_mels, np.float64)
    _check(load_library().melt_plan_get_frequencies(plan, out.ctypes.data_as(ctypes.c_void_p)),
           "melt_plan_get_frequencies")
    return out


def melt_plan_get_basis(plan, n_mels: int, n_fft: int) -> np.ndarray:
    out = np.empty((2 * n_mels, n_fft), np.float32)
    _check(load_library().melt_plan_get_basis(plan, out.ctypes.data_as(ctypes.c_void_p)), "melt_plan_get_basis")
    return out


def melt_plan_set_basis(plan, d_basis, stream=None) -> None:
    _check(load_library().melt_plan_set_basis(plan, _ptr(d_basis), _stream_handle(stream)), "melt_plan_set_basis")


def melt_frame_offsets(plan, d_clip_offsets, d_frame_offsets, stream=None) -> None:
    n = d_clip_offsets.numel() - 1
    _check(load_library().melt_frame_offsets(plan, _ptr(d_clip_offsets), n, _ptr(d_frame_offsets),
                                             _stream_handle(stream)), "melt_frame_offsets")


def melt_forward(plan, d_wave, d_clip_offsets, n_frames, d_out, stream=None) -> None:
    _check(load_library().melt_forward(plan, _ptr(d_wave), _ptr(d_clip_offsets), d_clip_offsets.numel() - 1,
                                       int(n_frames), _ptr(d_out), _stream_handle(stream)), "melt_forward")


def melt_forward_noalloc(plan, d_wave, d_clip_offsets, n_frames, d_out, stream=None) -> None:
    _check(load_library().melt_forward_noalloc(plan, _ptr(d_wave), _ptr(d_clip_offsets),
                                               d_clip_offsets.numel() - 1, int(n_frames), _ptr(d_out),
                                               _stream_handle(stream)), "melt_forward_noalloc")


def melt_forward_proj(plan, d_wave, d_clip_offsets, n_frames, d_out, d_proj, stream=None) -> None:
    _check(load_library().melt_forward_proj(plan, _ptr(d_wave), _ptr(d_clip_offsets), d_clip_offsets.numel() - 1,
                                            int(n_frames), _ptr(d_out), _ptr(d_proj), _stream_handle(stream)),
           "melt_forward_proj")


def stft_mel_forward(plan, d_wave, d_clip_offsets, n_frames, d_out, stream=None) -> None:
    _check(load_library().stft_mel_forward(plan, _ptr(d_wave), _ptr(d_clip_offsets), d_clip_offsets.numel() - 1,
                                           int(n_frames), _ptr(d_out), _stream_handle(stream)), "stft_mel_forward")


def melt_batch_prepare(plan, d_clip_offsets, n_frames, stream=None) -> None:
    _check(load_library().melt_batch_prepare(plan, _ptr(d_clip_offsets), d_clip_offsets.numel() - 1, int(n_frames),
                                             _stream_handle(stream)), "melt_batch_prepare")


def melt_forward_prepared(plan, d_wave, d_out, d_proj=None, stream=None) -> None:
    _check(load_library().melt_forward_prepared(plan, _ptr(d_wave), _ptr(d_out), _ptr(d_proj), _stream_handle(stream)),
           "melt_forward_prepared")


def stft_mel_forward_prepared(plan, d_wave, d_out, stream=None) -> None:
    _check(load_library().stft_mel_forward_prepared(plan, _ptr(d_wave), _ptr(d_out), _stream_handle(stream)),
           "stft_mel_forward_prepared")


def melt_backward(plan, d_wave, d_clip_offsets, n_frames, d_grad_out, d_proj, d_grad_wave, d_grad_basis,
                  stream=None) -> None:
    _check(load_library().melt_backward(plan, _ptr(d_wave), _ptr(d_clip_offsets), d_clip_offsets.numel() - 1,
                                        int(n_frames), _ptr(d_grad_out), _ptr(d_proj), _ptr(d_grad_wave),
                                        _ptr(d_grad_basis), _stream_handle(stream)), "melt_backward")


def melt_stream_create(plan, n_streams: int, max_chunk_len: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load_library().melt_stream_create(plan, n_streams, max_chunk_len, ctypes.byref(h)), "melt_stream_create")
    return h


def melt_stream_destroy(st) -> None:
    _check(load_library().melt_stream_destroy(st), "melt_stream_destroy")


def melt_stream_reset(st, stream=None) -> None:
    _check(load_library().melt_stream_reset(st, _stream_handle(stream)), "melt_stream_reset")


def melt_stream_max_frames(st) -> int:
    return int(load_library().melt_stream_max_frames(st))


def melt_stream_push(st, d_chunk, d_out, d_frames_emitted, stream=None) -> None:
    """d_chunk: [n_streams, chunk_len] float32 CUDA tensor; chunk_len is its second dimension."""
    _check(load_library().melt_stream_push(st, _ptr(d_chunk), int(d_chunk.shape[-1]), _ptr(d_out),
                                           _ptr(d_frames_emitted), _stream_handle(stream)), "melt_stream_push")


def melt_autotune(plan, total_frames: int) -> str:
    buf = ctypes.create_string_buffer(256)
    _check(load_library().melt_autotune(plan, int(total_frames), buf, 256), "melt_autotune")
    return buf.value.decode()


def melt_variant_count(plan) -> int:
    return int(load_library().melt_variant_count(plan))


def melt_variant_name(plan, v: int) -> str:
    return load_library().melt_variant_name(plan, int(v)).decode()


def melt_set_variant(plan, v: int, grid_per_cu: int = 0) -> None:
    _check(load_library().melt_set_variant(plan, int(v), int(grid_per_cu)), "melt_set_variant")


# ------------------------------------------------------------------ convenience layer

def make_config(sample_rate=16000.0, n_fft=400, hop=160, n_mels=80, fmin=0.0, fmax=None, *,
                precision="fp32", output=MELT_OUT_LOG_POWER, log_eps=1e-10, window=MELT_WIN_HANN_SYMMETRIC,
                mel_formula=MELT_MEL_HTK, placement=MELT_PLACE_FILTER_CENTRES, fb_norm=MELT_FB_NORM_NONE,
                n_mfcc=40):
    c = melt_config_default()
    c.sample_rate = float(sample_rate)
    c.n_fft = int(n_fft)
    c.hop = int(hop)
    c.n_mels = int(n_mels)
    c.fmin = float(fmin)
    c.fmax = float(sample_rate / 2 if fmax is None else fmax)
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.output = int(output)
    c.log_eps = float(log_eps)
    c.window = int(window)
    c.mel_formula = int(mel_formula)
    c.placement = int(placement)
    c.fb_norm = int(fb_norm)
    c.n_mfcc = int(n_mfcc)
    return c


def total_frames(clip_offsets, n_fft: int, hop: int) -> int:
    off = np.asarray(clip_offsets, np.int64)
    return int(sum(melt_num_frames(int(b - a), n_fft, hop) for a, b in zip(off[:-1], off[1:])))


class MeltStream:
    """Owns a streaming state over a MeltPlan; push() takes a [n_streams, chunk_len] tensor and
    returns (frames [n_streams, max_frames, out_cols], counts [n_streams]) device tensors (reused
    between pushes)."""

    def __init__(self, plan: "MeltPlan", n_streams: int, max_chunk_len: int):
        import torch
        self.plan = plan
        self.n_streams = n_streams
        self.handle = melt_stream_create(plan.handle, n_streams, max_chunk_len)
        self.max_frames = melt_stream_max_frames(self.handle)
        dev = f"cuda:{plan.device}"
        self.out = torch.zeros((n_streams, self.max_frames, plan.out_cols), dtype=torch.float32, device=dev)
        self.count = torch.zeros(n_streams, dtype=torch.int32, device=dev)

    def push(self, chunk):
        melt_stream_push(self.handle, chunk, self.out, self.count)
        return self.out, self.count

    def reset(self):
        melt_stream_reset(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            melt_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MeltPlan:
    """Owns a plan; forward/stft/backward take torch CUDA tensors."""

    def __init__(self, device: int = 0, **kw):
        self.cfg = make_config(**kw)
        self.device = device
        self.handle = melt_plan_create(self.cfg, device)
        self.n_mels, self.n_fft, self.hop = self.cfg.n_mels, self.cfg.n_fft, self.cfg.hop
        # width of an output row: n_mfcc cepstral coefficients under MELT_OUT_MFCC, else n_mels
        self.out_cols = self.cfg.n_mfcc if self.cfg.output == MELT_OUT_MFCC else self.n_mels
        # counts set_basis calls, so a backward can tell whether the basis it must
        # differentiate through is still the plan's
        self.basis_generation = 0

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            melt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def frequencies(self) -> np.ndarray:
        return melt_plan_get_frequencies(self.handle, self.n_mels)

    def basis(self) -> np.ndarray:
        return melt_plan_get_basis(self.handle, self.n_mels, self.n_fft)

    def set_basis(self, d_basis):
        melt_plan_set_basis(self.handle, d_basis.contiguous())
        self.basis_generation += 1

    def _out(self, n_frames, cols=None):
        import torch
        return torch.empty((n_frames, cols or self.out_cols), dtype=torch.float32, device=f"cuda:{self.device}")

    def forward(self, d_wave, d_offsets, n_frames, out=None, proj=None):
        out = self._out(n_frames) if out is None else out
        if proj is None:
            melt_forward(self.handle, d_wave, d_offsets, n_frames, out)
        else:
            melt_forward_proj(self.handle, d_wave, d_offsets, n_frames, out, proj)
        return out

    def stft_mel(self, d_wave, d_offsets, n_frames, out=None):
        out = self._out(n_frames) if out is None else out
        stft_mel_forward(self.handle, d_wave, d_offsets, n_frames, out)
        return out

    def backward(self, d_wave, d_offsets, n_frames, grad_out, proj=None, want_wave=True, want_basis=True):
        import torch
        gw = torch.empty_like(d_wave) if want_wave else None
        gb = torch.empty((2 * self.n_mels, self.n_fft), dtype=torch.float32, device=d_wave.device) \
            if want_basis else None
        melt_backward(self.handle, d_wave, d_offsets, n_frames, grad_out.contiguous(), proj, gw, gb)
        return gw, gb


def _make_function():
    import torch

    class MeltFunction(torch.autograd.Function):
        """out = MelT(wave) with gradients w.r.t. the waveform (and, via ``basis_param``, the
        learnable basis).  ``plan`` is a MeltPlan; offsets a CUDA int64 tensor."""

        @staticmethod
        def forward(ctx, wave, basis_param, plan, offsets, n_frames):
            if basis_param is not None:
                plan.set_basis(basis_param.detach())
            proj = torch.empty((n_frames, 2 * plan.n_mels), dtype=torch.float32, device=wave.device)
            out = plan.forward(wave.contiguous(), offsets, n_frames, proj=proj)
            # the basis this forward ran with is saved too (autograd's version check then
            # covers in-place changes to it), with the plan's basis generation
            ctx.save_for_backward(wave, proj, basis_param)
            ctx.plan, ctx.offsets, ctx.n_frames = plan, offsets, n_frames
            ctx.has_basis = basis_param is not None
            ctx.generation = plan.basis_generation
            return out

        @staticmethod
        def backward(ctx, g):
            wave, proj, basis_param = ctx.saved_tensors
            plan = ctx.plan
            if plan.basis_generation != ctx.generation:
                # another forward changed the plan's basis since this one ran
                if basis_param is None:
                    raise RuntimeError("melt_apply: the plan's basis was replaced (set_basis) between this "
                                       "forward and its backward; pass the basis as basis_param to differentiate "
                                       "through it")
                plan.set_basis(basis_param.detach())
                ctx.generation = plan.basis_generation
            gw, gb = plan.backward(wave, ctx.offsets, ctx.n_frames, g, proj=proj,
                                   want_wave=ctx.needs_input_grad[0], want_basis=ctx.has_basis)
            return gw, gb, None, None, None

    return MeltFunction


_MeltFunction = None


def melt_apply(wave, plan: MeltPlan, offsets, n_frames, basis_param=None):
    """Differentiable MelT forward (autograd through the library's backward kernels)."""
    global _MeltFunction
    if _MeltFunction is None:
        _MeltFunction = _make_function()
    return _MeltFunction.apply(wave, basis_param, plan, offsets, n_frames)


def melt_logmel(wave, offsets=None, plan: MeltPlan | None = None, **cfg):
    """One-shot MelT forward of a float32 CUDA waveform (all clips back to back)."""
    import torch
    if offsets is None:
        offsets = np.array([0, wave.numel()], np.int64)
    off_np = np.asarray(offsets.cpu() if hasattr(offsets, "cpu") else offsets, np.int64)
    own = plan is None
    plan = MeltPlan(**cfg) if own else plan
    T = total_frames(off_np, plan.n_fft, plan.hop)
    d_off = torch.from_numpy(off_np).to(wave.device)
    out = plan.forward(wave, d_off, T)
    return out
