"""Seeded synthetic audio for the MelT workloads.

This module only draws inputs.  It holds none of the frontend's arithmetic (no window, no
basis, no projection, no filterbank) and is the one piece of code that both the oracle
tests and the GPU path use, so that both see the same float32 samples.

All signals are generated in float64 with ``numpy.random.default_rng(seed)`` and cast to
float32 once; the float32 array is the exact input of every consumer.  The paper measures
LibriSpeech speech; no dataset is available here, so these generators stand in for it with
the shapes of the paper's workloads (16 kHz, 25 ms frames, 10 ms hop, clips of seconds to
minutes).  No dataset item is reproduced.

Each config returns a dict: ``wave`` (float32, all clips concatenated), ``offsets`` (int64
clip boundaries, n_clips+1 entries) and the frontend parameters.
"""
from __future__ import annotations

import numpy as np


def _tones(rng, n, sr, n_tones=3, fband=(100.0, 7000.0), amp=1.0 / 3.0):
    t = np.arange(n, dtype=np.float64) / sr
    x = np.zeros(n, np.float64)
    for _ in range(n_tones):
        f = rng.uniform(*fband)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        x += amp * np.cos(2.0 * np.pi * f * t + ph)
    return x


def _pink(rng, n, rms=0.1):
    """White Gaussian noise shaped by 1/sqrt(f) in the frequency domain, scaled to `rms`."""
    w = rng.standard_normal(n)
    spec = np.fft.rfft(w)
    f = np.arange(spec.size, dtype=np.float64)
    f[0] = 1.0
    spec /= np.sqrt(f)
    spec[0] = 0.0
    x = np.fft.irfft(spec, n)
    return x * (rms / max(np.sqrt(np.mean(x * x)), 1e-30))


def _am_tones(rng, n, sr, n_tones=3, amp=0.1):
    t = np.arange(n, dtype=np.float64) / sr
    x = np.zeros(n, np.float64)
    for _ in range(n_tones):
        fc = rng.uniform(100.0, 7000.0)
        fa = rng.uniform(0.5, 8.0)
        depth = rng.uniform(0.0, 1.0)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=2)
        x += amp * (1.0 + depth * np.cos(2.0 * np.pi * fa * t + ph[0])) / (1.0 + depth) * \
            np.cos(2.0 * np.pi * fc * t + ph[1])
    return x


def _pack(clips):
    lens = np.array([c.size for c in clips], np.int64)
    off = np.zeros(len(clips) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    wave = np.concatenate(clips).astype(np.float32) if clips else np.zeros(0, np.float32)
    return wave, off


def spectral_params(sr=16000.0, n_fft=400, hop=160, n_mels=80, fmin=0.0, fmax=8000.0):
    return dict(sr=float(sr), n_fft=int(n_fft), hop=int(hop), n_mels=int(n_mels),
                fmin=float(fmin), fmax=float(fmax))


def config1(seed: int = 0):
    """One 1.0 s clip at 16 kHz: three tones at seeded frequencies in [100, 7000] Hz, each
    of amplitude 1/3, plus Gaussian noise of standard deviation 0.01; N=400, H=160, 80 HTK
    Mel bins over 0-8 kHz (98 frames)."""
    rng = np.random.default_rng(seed)
    n = 16000
    x = _tones(rng, n, 16000.0) + rng.normal(0.0, 0.01, n)
    wave, off = _pack([x])
    return dict(wave=wave, offsets=off, **spectral_params())


def config2(n_mels: int = 80, n_clips: int = 64, seconds: float = 30.0, seed_base: int = 1000,
            sr: float = 16000.0, n_fft: int = 400, hop: int = 160):
    """Batch of equal clips: pink noise (RMS 0.1) plus three amplitude-modulated tones
    (carrier 100-7000 Hz, modulation 0.5-8 Hz, depth 0-1, amplitude 0.1); seed 1000+c."""
    n = int(round(seconds * sr))
    clips = []
    for c in range(n_clips):
        rng = np.random.default_rng(seed_base + c)
        clips.append(_pink(rng, n) + _am_tones(rng, n, sr))
    wave, off = _pack(clips)
    return dict(wave=wave, offsets=off, **spectral_params(sr, n_fft, hop, n_mels, 0.0, sr / 2))


def config3(n_mels: int = 80, n_clips: int = 64, seconds: float = 30.0, seed_base: int = 2000):
    """Config-2 clips with amplitudes log-uniform over 60 dB: a per-clip gain and a gain per
    1 s segment, each 10^(U(-60, 0)/20)."""
    sr = 16000.0
    n = int(round(seconds * sr))
    clips = []
    for c in range(n_clips):
        rng = np.random.default_rng(seed_base + c)
        x = _pink(rng, n) + _am_tones(rng, n, sr)
        g = 10.0 ** (rng.uniform(-60.0, 0.0) / 20.0)
        seg = int(sr)
        n_seg = (n + seg - 1) // seg
        sg = 10.0 ** (rng.uniform(-60.0, 0.0, size=n_seg) / 20.0)
        x = x * g * np.repeat(sg, seg)[:n]
        clips.append(x)
    wave, off = _pack(clips)
    return dict(wave=wave, offsets=off, **spectral_params(sr, 400, 160, n_mels, 0.0, sr / 2))


def _chirps(rng, n, sr, n_chirps=4):
    t = np.arange(n, dtype=np.float64) / sr
    L = n / sr
    x = np.zeros(n, np.float64)
    for _ in range(n_chirps):
        tc = rng.uniform(0.0, L)
        sig = rng.uniform(0.05, 1.0)
        f0 = rng.uniform(100.0, 0.4 * sr)
        rate = rng.uniform(-2000.0, 2000.0)
        lo = max(0, int((tc - 5 * sig) * sr))
        hi = min(n, int((tc + 5 * sig) * sr) + 1)
        if hi <= lo:
            continue
        tt = t[lo:hi] - tc
        env = np.exp(-0.5 * (tt / sig) ** 2)
        x[lo:hi] += 0.25 * env * np.cos(2.0 * np.pi * (f0 * tt + 0.5 * rate * tt * tt))
    return x


def config4(variant: str = "16k", n_clips: int = 512, seed_base: int = 3000, max_seconds=30.0):
    """Ragged batch: clip lengths uniform in [0.5, max_seconds] s, each a sum of four
    Gaussian-modulated linear chirps.  variant '16k': sr 16 kHz, N=512, H=128, 128 Mel bins;
    variant '22k': sr 22.05 kHz, N=1024, H=256, 128 Mel bins."""
    sr, n_fft, hop = (16000.0, 512, 128) if variant == "16k" else (22050.0, 1024, 256)
    clips = []
    for c in range(n_clips):
        rng = np.random.default_rng(seed_base + c)
        n = int(round(rng.uniform(0.5, max_seconds) * sr))
        clips.append(_chirps(rng, n, sr))
    wave, off = _pack(clips)
    return dict(wave=wave, offsets=off, **spectral_params(sr, n_fft, hop, 128, 0.0, sr / 2))


def config5(n_clips: int = 32, seconds: float = 10.0, seed_base: int = 4000):
    """Differentiation workload: config-2 signals at 22.05 kHz, N=1024, H=256, 128 Mel bins,
    with a standard-normal upstream gradient drawn by `upstream_grad`."""
    sr = 22050.0
    n = int(round(seconds * sr))
    clips = []
    for c in range(n_clips):
        rng = np.random.default_rng(seed_base + c)
        clips.append(_pink(rng, n) + _am_tones(rng, n, sr))
    wave, off = _pack(clips)
    return dict(wave=wave, offsets=off, **spectral_params(sr, 1024, 256, 128, 0.0, sr / 2))


def upstream_grad(n_frames: int, n_mels: int, seed: int = 4999) -> np.ndarray:
    """Standard-normal upstream gradient [T, M] (float32)."""
    return np.random.default_rng(seed).standard_normal((n_frames, n_mels)).astype(np.float32)


def random_clips(lengths, seed: int = 0, scale: float = 0.5):
    """Gaussian noise clips of the given lengths (for edge cases: empty, sub-frame, ragged)."""
    rng = np.random.default_rng(seed)
    return _pack([scale * rng.standard_normal(int(n)) for n in lengths])
