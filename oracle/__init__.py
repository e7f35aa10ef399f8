"""FP64 CPU oracle for MelT and for the STFT + Mel-filterbank comparator.

TEST INFRASTRUCTURE ONLY.  This package is the correctness reference the GPU library is
checked against.  It shares no code with the GPU library and is loaded only by the tests,
the smoke check and the CPU-baseline leg of the benchmark; the product path never imports
it.

The arithmetic lives in ``melt_oracle.c`` (plain C, double precision, OpenMP over frames);
each C function cites the equation of the paper it writes out.  This module only compiles
that file with ``gcc`` and marshals numpy arrays through ``ctypes``.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py`` against
closed forms, library routines or invariants; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "melt_oracle.c"
_BUILD = _HERE / "_build"
_LIB_PATH = _BUILD / "libmelt_oracle.so"

# enum values shared with the C file (the oracle's own numbering)
OUT_LOG_POWER, OUT_LOG_MAGNITUDE, OUT_POWER, OUT_MAGNITUDE = 0, 1, 2, 3
WIN_HANN_SYMMETRIC, WIN_HANN_PERIODIC, WIN_RECT = 0, 1, 2
MEL_HTK, MEL_SLANEY = 0, 1
PLACE_FILTER_CENTRES, PLACE_LINSPACE = 0, 1
NORM_NONE, NORM_SLANEY = 0, 1
PREC_FP32, PREC_BF16, PREC_FP16, PREC_FP8_E4M3, PREC_BF16X3, PREC_FP16X3, PREC_FP8_E4M3_BLOCK32 = 0, 1, 2, 3, 4, 5, 6


def build(force: bool = False) -> Path:
    """Compile the oracle into ``oracle/_build/libmelt_oracle.so`` (gcc, -O2, OpenMP).

    No fast-math and no FMA contraction, so the FP32 steps of the operand models round
    exactly as IEEE single precision."""
    _BUILD.mkdir(exist_ok=True)
    if force or not _LIB_PATH.exists() or _LIB_PATH.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB_PATH.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = _LIB_PATH if _LIB_PATH.exists() else build()
        L = ctypes.CDLL(str(path))
        d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
        p = ctypes.c_void_p
        L.oracle_hz_to_mel.restype = d
        L.oracle_hz_to_mel.argtypes = [d, i]
        L.oracle_mel_to_hz.restype = d
        L.oracle_mel_to_hz.argtypes = [d, i]
        L.oracle_mel_grid_hz.argtypes = [i, d, d, i, p]
        L.oracle_melt_frequencies.argtypes = [i, d, d, i, i, p]
        L.oracle_window.argtypes = [i, i, p]
        L.oracle_num_frames.restype = i64
        L.oracle_num_frames.argtypes = [i64, i, i]
        L.oracle_total_frames.restype = i64
        L.oracle_total_frames.argtypes = [p, i, i, i]
        L.oracle_melt_forward.restype = i64
        L.oracle_melt_forward.argtypes = [p, p, i, d, i, i, i, p, i, i, d, p, p, p]
        L.oracle_melt_basis.argtypes = [d, i, i, p, i, p, p]
        L.oracle_melt_forward_basis.restype = i64
        L.oracle_melt_forward_basis.argtypes = [p, p, i, i, i, p, p, i, i, d, p, p, p]
        L.oracle_melt_backward.restype = i64
        L.oracle_melt_backward.argtypes = [p, i64, p, i, i, i, p, p, i, i, d, p, p, p, p]
        L.oracle_melt_chain.restype = None
        L.oracle_melt_chain.argtypes = [i64, i, p, p, p, i, d, p, p]
        L.oracle_melt_backward_linear.restype = i64
        L.oracle_melt_backward_linear.argtypes = [p, i64, p, i, i, i, p, p, i, p, p, p, p, p]
        L.oracle_power_spectrum.restype = i64
        L.oracle_power_spectrum.argtypes = [p, p, i, i, i, i, p]
        L.oracle_mel_filterbank.argtypes = [i, d, i, d, d, i, i, p]
        L.oracle_stft_mel_forward.restype = i64
        L.oracle_stft_mel_forward.argtypes = [p, p, i, d, i, i, i, i, d, d, i, i, i, d, p]
        L.oracle_dct2_ortho.argtypes = [i, i, p]
        for name in ("oracle_round_bf16", "oracle_round_fp16", "oracle_round_e4m3"):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [ctypes.c_float]
        L.oracle_block_exponent.restype = i
        L.oracle_block_exponent.argtypes = [ctypes.c_float]
        L.oracle_melt_forward_quant.restype = i64
        L.oracle_melt_forward_quant.argtypes = [p, p, i, i, i, p, p, i, i, i, d, p, p, p]
        L.oracle_num_threads.restype = i
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _wave(x) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.float32)
    if a.dtype != np.float32:
        raise TypeError("waveform must be float32")
    return a


def _offsets(clip_offsets, n_samples: int) -> np.ndarray:
    if clip_offsets is None:
        clip_offsets = [0, n_samples]
    return np.ascontiguousarray(clip_offsets, dtype=np.int64)


# ---------------------------------------------------------------- scalar helpers

def hz_to_mel(f: float, formula: int = MEL_HTK) -> float:
    return lib().oracle_hz_to_mel(float(f), formula)


def mel_to_hz(mu: float, formula: int = MEL_HTK) -> float:
    return lib().oracle_mel_to_hz(float(mu), formula)


def mel_grid_hz(n_mels: int, fmin: float, fmax: float, formula: int = MEL_HTK) -> np.ndarray:
    out = np.empty(n_mels + 2, np.float64)
    lib().oracle_mel_grid_hz(n_mels, fmin, fmax, formula, _ptr(out))
    return out


def melt_frequencies(n_mels, fmin, fmax, formula=MEL_HTK, placement=PLACE_FILTER_CENTRES):
    out = np.empty(n_mels, np.float64)
    lib().oracle_melt_frequencies(n_mels, fmin, fmax, formula, placement, _ptr(out))
    return out


def window(n: int, kind: int = WIN_HANN_SYMMETRIC) -> np.ndarray:
    out = np.empty(n, np.float64)
    lib().oracle_window(n, kind, _ptr(out))
    return out


def num_frames(n_samples: int, n_fft: int, hop: int) -> int:
    return int(lib().oracle_num_frames(int(n_samples), n_fft, hop))


def total_frames(clip_offsets, n_fft: int, hop: int) -> int:
    off = np.ascontiguousarray(clip_offsets, dtype=np.int64)
    return int(lib().oracle_total_frames(_ptr(off), len(off) - 1, n_fft, hop))


def round_bf16(x) -> np.ndarray:
    f = lib().oracle_round_bf16
    return np.array([f(float(v)) for v in np.asarray(x, np.float32).ravel()]).reshape(np.shape(x))


def round_fp16(x) -> np.ndarray:
    f = lib().oracle_round_fp16
    return np.array([f(float(v)) for v in np.asarray(x, np.float32).ravel()]).reshape(np.shape(x))


def round_e4m3(x) -> np.ndarray:
    f = lib().oracle_round_e4m3
    return np.array([f(float(v)) for v in np.asarray(x, np.float32).ravel()]).reshape(np.shape(x))


def block_exponent(m) -> np.ndarray:
    """Largest integer e with 2^e |m| <= 448, within [-127, 127]; 0 for m = 0."""
    f = lib().oracle_block_exponent
    return np.array([f(float(v)) for v in np.asarray(m, np.float32).ravel()], np.int64).reshape(np.shape(m))


# ---------------------------------------------------------------- MelT

def melt_forward(wave, clip_offsets=None, *, sr, n_fft, hop, freqs, window_kind=WIN_HANN_SYMMETRIC,
                 out_kind=OUT_LOG_POWER, eps=1e-10, return_ri=False):
    """Direct NDFT summation (Eqs. dmp_components, dmp_energy, meltf).  [T, M] float64."""
    x = _wave(wave)
    off = _offsets(clip_offsets, x.size)
    f = np.ascontiguousarray(freqs, np.float64)
    T = total_frames(off, n_fft, hop)
    M = f.size
    out = np.empty((T, M), np.float64)
    R = np.empty((T, M), np.float64) if return_ri else None
    I = np.empty((T, M), np.float64) if return_ri else None
    lib().oracle_melt_forward(_ptr(x), _ptr(off), len(off) - 1, float(sr), n_fft, hop, window_kind,
                              _ptr(f), M, out_kind, float(eps), _ptr(out), _ptr(R), _ptr(I))
    return (out, R, I) if return_ri else out


def melt_basis(*, sr, n_fft, freqs, window_kind=WIN_HANN_SYMMETRIC):
    """Window-folded basis (Eq. dmp_weights): (Wr, Wi), each [M, N] float64."""
    f = np.ascontiguousarray(freqs, np.float64)
    Wr = np.empty((f.size, n_fft), np.float64)
    Wi = np.empty((f.size, n_fft), np.float64)
    lib().oracle_melt_basis(float(sr), n_fft, window_kind, _ptr(f), f.size, _ptr(Wr), _ptr(Wi))
    return Wr, Wi


def melt_forward_basis(wave, clip_offsets=None, *, n_fft, hop, Wr, Wi, out_kind=OUT_LOG_POWER,
                       eps=1e-10, return_ri=False):
    """Projection with an explicit basis (Eq. dmp_projection).  [T, M] float64."""
    x = _wave(wave)
    off = _offsets(clip_offsets, x.size)
    Wr = np.ascontiguousarray(Wr, np.float64)
    Wi = np.ascontiguousarray(Wi, np.float64)
    M = Wr.shape[0]
    T = total_frames(off, n_fft, hop)
    out = np.empty((T, M), np.float64)
    R = np.empty((T, M), np.float64) if return_ri else None
    I = np.empty((T, M), np.float64) if return_ri else None
    lib().oracle_melt_forward_basis(_ptr(x), _ptr(off), len(off) - 1, n_fft, hop, _ptr(Wr), _ptr(Wi),
                                    M, out_kind, float(eps), _ptr(out), _ptr(R), _ptr(I))
    return (out, R, I) if return_ri else out


def melt_forward_quant(wave, clip_offsets=None, *, n_fft, hop, Wr, Wi, prec, out_kind=OUT_LOG_POWER,
                       eps=1e-10, return_ri=False):
    """Operand-rounding model of a reduced-precision projection (see the C file)."""
    x = _wave(wave)
    off = _offsets(clip_offsets, x.size)
    Wr = np.ascontiguousarray(Wr, np.float64)
    Wi = np.ascontiguousarray(Wi, np.float64)
    M = Wr.shape[0]
    T = total_frames(off, n_fft, hop)
    out = np.empty((T, M), np.float64)
    R = np.empty((T, M), np.float64) if return_ri else None
    I = np.empty((T, M), np.float64) if return_ri else None
    lib().oracle_melt_forward_quant(_ptr(x), _ptr(off), len(off) - 1, n_fft, hop, _ptr(Wr), _ptr(Wi),
                                    M, prec, out_kind, float(eps), _ptr(out), _ptr(R), _ptr(I))
    return (out, R, I) if return_ri else out


def melt_backward(wave, clip_offsets=None, *, n_fft, hop, Wr, Wi, grad_out, out_kind=OUT_LOG_POWER,
                  eps=1e-10):
    """Chain-rule gradient of the projection: (grad_wave, dWr, dWi)."""
    x = _wave(wave)
    off = _offsets(clip_offsets, x.size)
    Wr = np.ascontiguousarray(Wr, np.float64)
    Wi = np.ascontiguousarray(Wi, np.float64)
    g = np.ascontiguousarray(grad_out, np.float64)
    M = Wr.shape[0]
    gx = np.empty(x.size, np.float64)
    dWr = np.empty_like(Wr)
    dWi = np.empty_like(Wi)
    lib().oracle_melt_backward(_ptr(x), x.size, _ptr(off), len(off) - 1, n_fft, hop, _ptr(Wr), _ptr(Wi),
                               M, out_kind, float(eps), _ptr(g), _ptr(gx), _ptr(dWr), _ptr(dWi))
    return gx, dWr, dWi


def melt_chain(R, I, grad_out, *, out_kind=OUT_LOG_POWER, eps=1e-10):
    """Chain rule through the energy and output map (Eqs. meltf, dmp_energy): the gradients
    (Gr, Gi) of R and I for upstream grad_out, from any projections R, I [T, M]."""
    R = np.ascontiguousarray(R, np.float64)
    I = np.ascontiguousarray(I, np.float64)
    g = np.ascontiguousarray(grad_out, np.float64)
    if not (R.shape == I.shape == g.shape and R.ndim == 2):
        raise ValueError("R, I and grad_out must share one [T, M] shape")
    Gr = np.empty_like(R)
    Gi = np.empty_like(R)
    lib().oracle_melt_chain(R.shape[0], R.shape[1], _ptr(R), _ptr(I), _ptr(g), out_kind, float(eps), _ptr(Gr),
                            _ptr(Gi))
    return Gr, Gi


def melt_backward_linear(wave, clip_offsets=None, *, n_fft, hop, Wr, Wi, Gr, Gi, want_wave=True):
    """Transpose of the projection (Eq. dmp_projection) applied to the gradients (Gr, Gi) of
    R and I: (grad_wave, dWr, dWi), grad_wave overlap-added over the frames (None when
    want_wave is False)."""
    x = _wave(wave)
    off = _offsets(clip_offsets, x.size)
    Wr = np.ascontiguousarray(Wr, np.float64)
    Wi = np.ascontiguousarray(Wi, np.float64)
    Gr = np.ascontiguousarray(Gr, np.float64)
    Gi = np.ascontiguousarray(Gi, np.float64)
    M = Wr.shape[0]
    T = total_frames(off, n_fft, hop)
    if Gr.shape != (T, M) or Gi.shape != (T, M):
        raise ValueError("Gr and Gi must be [T, M]")
    gx = np.empty(x.size, np.float64) if want_wave else None
    dWr = np.empty_like(Wr)
    dWi = np.empty_like(Wi)
    lib().oracle_melt_backward_linear(_ptr(x), x.size, _ptr(off), len(off) - 1, n_fft, hop, _ptr(Wr), _ptr(Wi), M,
                                      _ptr(Gr), _ptr(Gi), _ptr(gx), _ptr(dWr), _ptr(dWi))
    return gx, dWr, dWi


# ---------------------------------------------------------------- STFT + filterbank

def power_spectrum(wave, clip_offsets=None, *, n_fft, hop, window_kind=WIN_HANN_SYMMETRIC):
    x = _wave(wave)
    off = _offsets(clip_offsets, x.size)
    T = total_frames(off, n_fft, hop)
    P = np.empty((T, n_fft // 2 + 1), np.float64)
    lib().oracle_power_spectrum(_ptr(x), _ptr(off), len(off) - 1, n_fft, hop, window_kind, _ptr(P))
    return P


def mel_filterbank(*, n_fft, sr, n_mels, fmin, fmax, formula=MEL_HTK, norm=NORM_NONE):
    F = np.empty((n_mels, n_fft // 2 + 1), np.float64)
    lib().oracle_mel_filterbank(n_fft, float(sr), n_mels, float(fmin), float(fmax), formula, norm, _ptr(F))
    return F


def stft_mel_forward(wave, clip_offsets=None, *, sr, n_fft, hop, n_mels, fmin, fmax,
                     window_kind=WIN_HANN_SYMMETRIC, formula=MEL_HTK, norm=NORM_NONE,
                     out_kind=OUT_LOG_POWER, eps=1e-10):
    x = _wave(wave)
    off = _offsets(clip_offsets, x.size)
    T = total_frames(off, n_fft, hop)
    out = np.empty((T, n_mels), np.float64)
    lib().oracle_stft_mel_forward(_ptr(x), _ptr(off), len(off) - 1, float(sr), n_fft, hop, window_kind,
                                  n_mels, float(fmin), float(fmax), formula, norm, out_kind, float(eps),
                                  _ptr(out))
    return out


def dct2_ortho(K: int, M: int) -> np.ndarray:
    D = np.empty((K, M), np.float64)
    lib().oracle_dct2_ortho(K, M, _ptr(D))
    return D


def cepstrum(L: np.ndarray, K: int) -> np.ndarray:
    """Eq. mfcct_matrix: C = L D^T for log-Mel rows L [T, M] and D the first K rows of the
    orthonormal DCT-II over M (MFCCT when L is the MelT log power, conventional MFCC when L
    is the filterbank log power)."""
    L = np.asarray(L, np.float64)
    return L @ dct2_ortho(K, L.shape[1]).T


def num_threads() -> int:
    return int(lib().oracle_num_threads())
