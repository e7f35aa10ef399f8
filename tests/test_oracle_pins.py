"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, an independent library routine
(numpy.fft, scipy, transformers' audio utilities, torch dtype casts, mpmath), an invariant
of the mathematics, or a value the paper prints.  Together they are chosen so that a
dropped term, a wrong sign or index, or a transposed operand in the oracle fails one of
them.  None of them needs a GPU.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Mel scale (Eq. mel_scale)

def test_mel_scale_closed_forms(orc):
    # mu(700) = 2595 log10(2): the HTK formula at f = 700 Hz
    assert orc.hz_to_mel(700.0) == pytest.approx(2595.0 * math.log10(2.0), rel=1e-15)
    assert orc.hz_to_mel(0.0) == 0.0
    # Slaney scale: linear 3 Mel per 200 Hz below 1 kHz, so 1 kHz -> 15 Mel
    assert orc.hz_to_mel(1000.0, orc.MEL_SLANEY) == pytest.approx(15.0, rel=1e-15)
    for f in [0.0, 80.0, 440.0, 1000.0, 3999.0, 7600.0, 8000.0, 11025.0]:
        for form in (orc.MEL_HTK, orc.MEL_SLANEY):
            assert orc.mel_to_hz(orc.hz_to_mel(f, form), form) == pytest.approx(f, rel=1e-13, abs=1e-10)


def test_slaney_scale_pins(orc):
    """The Slaney scale (a Mel-formula option of both paths): 3 Mel per 200 Hz below 1 kHz,
    then 27 Mel per factor 6.4 of frequency.  Closed forms at the break, one and two log
    steps above it, the constant Mel width of an octave above 1 kHz, and the library routine
    (transformers.audio_utils.hertz_to_mel / mel_to_hertz, mel_scale="slaney") over 0-11 kHz.
    A wrong slope, break or log step fails one of them."""
    from transformers.audio_utils import hertz_to_mel, mel_to_hertz
    S = orc.MEL_SLANEY
    assert orc.hz_to_mel(500.0, S) == pytest.approx(7.5, rel=1e-15)
    assert orc.hz_to_mel(1000.0, S) == pytest.approx(15.0, rel=1e-15)
    assert orc.hz_to_mel(6400.0, S) == pytest.approx(42.0, rel=1e-15)            # 15 + 27
    assert orc.hz_to_mel(6400.0 * 6.4, S) == pytest.approx(69.0, rel=1e-15)      # 15 + 2 * 27
    octave = 27.0 * math.log(2.0) / math.log(6.4)
    for f in (1000.0, 1500.0, 3000.0, 5512.5):
        assert orc.hz_to_mel(2 * f, S) - orc.hz_to_mel(f, S) == pytest.approx(octave, rel=1e-13)
    f = np.linspace(0.0, 11025.0, 301)
    mu = np.array([orc.hz_to_mel(v, S) for v in f])
    assert np.allclose(mu, hertz_to_mel(f, mel_scale="slaney"), rtol=1e-14, atol=1e-13)
    m = np.linspace(0.0, 48.0, 97)
    assert np.allclose([orc.mel_to_hz(v, S) for v in m], mel_to_hertz(m, mel_scale="slaney"), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("M,fmin,fmax,sr", [(40, 0.0, 8000.0, 16000.0), (80, 80.0, 7600.0, 16000.0),
                                             (128, 0.0, 11025.0, 22050.0)])
def test_slaney_grid_and_filterbank(orc, M, fmin, fmax, sr):
    """Slaney-scale filter centres and triangles against transformers' routines: the
    (M+2)-point grid is mel_to_hertz of a uniform Mel grid, the analysis frequencies are its
    interior points (or the M-point grid for the linspace placement), and the triangular
    filterbank equals mel_filter_bank(mel_scale="slaney") with and without area norm."""
    from transformers.audio_utils import hertz_to_mel, mel_filter_bank, mel_to_hertz
    a, b = hertz_to_mel(fmin, mel_scale="slaney"), hertz_to_mel(fmax, mel_scale="slaney")
    grid = mel_to_hertz(np.linspace(a, b, M + 2), mel_scale="slaney")
    assert np.allclose(orc.mel_grid_hz(M, fmin, fmax, orc.MEL_SLANEY), grid, rtol=1e-13, atol=1e-9)
    assert np.allclose(orc.melt_frequencies(M, fmin, fmax, orc.MEL_SLANEY), grid[1:-1], rtol=1e-13)
    lin = mel_to_hertz(np.linspace(a, b, M), mel_scale="slaney")
    assert np.allclose(orc.melt_frequencies(M, fmin, fmax, orc.MEL_SLANEY, orc.PLACE_LINSPACE), lin,
                       rtol=1e-13, atol=1e-9)
    N = 512 if sr == 16000.0 else 1024
    for norm, lib_norm in ((orc.NORM_NONE, None), (orc.NORM_SLANEY, "slaney")):
        F = orc.mel_filterbank(n_fft=N, sr=sr, n_mels=M, fmin=fmin, fmax=fmax, formula=orc.MEL_SLANEY, norm=norm)
        ref = mel_filter_bank(N // 2 + 1, M, fmin, fmax, sr, norm=lib_norm, mel_scale="slaney").T
        assert np.allclose(F, ref, rtol=1e-10, atol=1e-12)


def test_mel_grid_and_centres(orc):
    g = orc.mel_grid_hz(80, 0.0, 8000.0)
    assert g[0] == pytest.approx(0.0, abs=1e-9) and g[-1] == pytest.approx(8000.0, rel=1e-14)
    mu = np.array([orc.hz_to_mel(f) for f in g])
    assert np.allclose(np.diff(mu), mu[-1] / 81.0, rtol=1e-12)   # uniform in Mel
    f = orc.melt_frequencies(80, 0.0, 8000.0)
    assert np.array_equal(f, g[1:-1])                              # filter centres
    # numerical value of the first centre: 700 (10^(mu_1/2595) - 1), mu_1 = mu(8000)/81
    mu1 = 2595.0 * math.log10(1.0 + 8000.0 / 700.0) / 81.0
    assert f[0] == pytest.approx(700.0 * (10.0 ** (mu1 / 2595.0) - 1.0), rel=1e-13)
    lin = orc.melt_frequencies(80, 0.0, 8000.0, placement=orc.PLACE_LINSPACE)
    assert lin[0] == pytest.approx(0.0, abs=1e-9) and lin[-1] == pytest.approx(8000.0, rel=1e-13)


# ------------------------------------------------------------------ window, frames

def test_window_matches_scipy(orc):
    from scipy.signal import windows
    for n in (2, 5, 16, 400, 512, 1024):
        assert np.allclose(orc.window(n, orc.WIN_HANN_SYMMETRIC), windows.hann(n, sym=True), atol=1e-15)
        assert np.allclose(orc.window(n, orc.WIN_HANN_PERIODIC), windows.hann(n, sym=False), atol=1e-15)
    assert np.all(orc.window(7, orc.WIN_RECT) == 1.0)


def test_frame_counts(orc):
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        gold = json.load(fh)
    c = gold["frames_1s_16k"]
    assert orc.num_frames(c["samples"], c["n_fft"], c["hop"]) == c["frames"]
    assert orc.num_frames(399, 400, 160) == 0
    assert orc.num_frames(400, 400, 160) == 1
    assert orc.num_frames(559, 400, 160) == 1
    assert orc.num_frames(560, 400, 160) == 2
    assert orc.num_frames(0, 400, 160) == 0


# ------------------------------------------------------------------ MelT projection

def _frame(n, seed=0):
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)


def test_ndft_on_bins_equals_rfft(orc):
    """P1: at f_m = k sr / N the Mel-spaced projection is the DFT at bin k: its energy equals
    |rfft(w x)|^2 from numpy's FFT and the oracle's own naive DFT."""
    N, H, sr = 400, 160, 16000.0
    x = _frame(N * 3)
    ks = np.array([0, 1, 2, 7, 50, 123, 199, 200])
    freqs = ks * sr / N
    S = orc.melt_forward(x, sr=sr, n_fft=N, hop=H, freqs=freqs, out_kind=orc.OUT_POWER)
    w = orc.window(N)
    T = S.shape[0]
    ref = np.stack([np.abs(np.fft.rfft(w * x[t * H:t * H + N].astype(np.float64))) ** 2 for t in range(T)])
    assert np.allclose(S, ref[:, ks], rtol=1e-11, atol=1e-9)
    P = orc.power_spectrum(x, n_fft=N, hop=H)
    assert np.allclose(P, ref, rtol=1e-11, atol=1e-9)
    # R = Re X_k and I = -Im X_k (the sign of the sin term)
    _, R, I = orc.melt_forward(x, sr=sr, n_fft=N, hop=H, freqs=freqs, out_kind=orc.OUT_POWER, return_ri=True)
    X0 = np.fft.rfft(w * x[:N].astype(np.float64))
    assert np.allclose(R[0], X0.real[ks], atol=1e-10)
    assert np.allclose(I[0], -X0.imag[ks], atol=1e-10)


def _hann_dtft(omega, N):
    """sum_n w[n] e^{i omega n} for the symmetric Hann window, in closed form:
    w[n] = 1/2 - (e^{i a n} + e^{-i a n})/4, a = 2 pi/(N-1), and each term is a geometric
    series G(v) = sum_{n<N} e^{i v n} = (e^{i v N} - 1)/(e^{i v} - 1)."""
    a = 2.0 * np.pi / (N - 1)

    def G(v):
        z = np.exp(1j * v)
        if abs(z - 1.0) < 1e-12:
            return complex(N)
        return (np.exp(1j * v * N) - 1.0) / (z - 1.0)

    return 0.5 * G(omega) - 0.25 * G(omega + a) - 0.25 * G(omega - a)


@pytest.mark.parametrize("N,sr,f_tone,f_an", [(400, 16000.0, 1234.5, 1234.5),
                                               (400, 16000.0, 1000.0, 1107.3),
                                               (512, 22050.0, 300.0, 4100.0),
                                               (1024, 22050.0, 9876.5, 9876.5)])
def test_hann_tone_closed_form(orc, N, sr, f_tone, f_an):
    """P2: for x[n] = A cos(th_x n + phi), R - iI = sum_n w x e^{-i th n}
    = A/2 [e^{i phi} Hw(th_x - th) + e^{-i phi} Hw(-th_x - th)] with Hw the Hann DTFT."""
    A, phi = 0.75, 0.4
    n = np.arange(N)
    th_x = 2 * np.pi * f_tone / sr
    th = 2 * np.pi * f_an / sr
    x = (A * np.cos(th_x * n + phi)).astype(np.float32)
    # use the float32 samples exactly: decompose the residual of the rounding separately
    resid = x.astype(np.float64) - A * np.cos(th_x * n + phi)
    w = orc.window(N)
    Z = A / 2 * (np.exp(1j * phi) * _hann_dtft(th_x - th, N) + np.exp(-1j * phi) * _hann_dtft(-th_x - th, N))
    Z += np.sum(w * resid * np.exp(-1j * th * n))     # exact contribution of the float32 rounding
    _, R, I = orc.melt_forward(x, sr=sr, n_fft=N, hop=N, freqs=[f_an], out_kind=orc.OUT_POWER, return_ri=True)
    assert R[0, 0] == pytest.approx(Z.real, rel=1e-10, abs=1e-10 * N)
    assert I[0, 0] == pytest.approx(-Z.imag, rel=1e-10, abs=1e-10 * N)
    if f_tone == f_an:
        # on-frequency: |R - iI| ~ A/2 sum w = A (N-1)/4 (plus the small image term)
        assert abs(Z) == pytest.approx(A * (N - 1) / 4.0, rel=0.02)


def test_projection_linearity(orc):
    """P3: (R, I) are linear in the frame; S scales by a^2, so the log shifts by 2 ln|a|."""
    N, H, sr = 400, 160, 16000.0
    f = orc.melt_frequencies(80, 0.0, 8000.0)
    # dyadic grid (multiples of 2^-12, |v| < 4) so that a x + b y is exact in float32
    x = (np.round(_frame(2000, 1) * 1024) / 4096).astype(np.float32)
    y = (np.round(_frame(2000, 2) * 1024) / 4096).astype(np.float32)
    a, b = np.float32(0.5), np.float32(-2.0)
    z = (a * x + b * y).astype(np.float32)
    _, Rx, Ix = orc.melt_forward(x, sr=sr, n_fft=N, hop=H, freqs=f, return_ri=True)
    _, Ry, Iy = orc.melt_forward(y, sr=sr, n_fft=N, hop=H, freqs=f, return_ri=True)
    Lz, Rz, Iz = orc.melt_forward(z, sr=sr, n_fft=N, hop=H, freqs=f, return_ri=True, eps=0.0)
    assert np.allclose(Rz, a * Rx + b * Ry, rtol=1e-12, atol=1e-12)
    assert np.allclose(Iz, a * Ix + b * Iy, rtol=1e-12, atol=1e-12)
    L1 = orc.melt_forward(x, sr=sr, n_fft=N, hop=H, freqs=f, eps=0.0)
    L2 = orc.melt_forward((4 * x).astype(np.float32), sr=sr, n_fft=N, hop=H, freqs=f, eps=0.0)
    assert np.allclose(L2 - L1, 2 * math.log(4.0), atol=1e-9)


def test_explicit_basis_matches_direct(orc):
    """Eq. dmp_weights/dmp_projection: folding the window into the basis gives the same R, I
    as windowing the frame (Eq. dmp_components)."""
    N, H, sr = 512, 128, 22050.0
    f = orc.melt_frequencies(32, 0.0, sr / 2)
    x = _frame(3000, 3)
    Wr, Wi = orc.melt_basis(sr=sr, n_fft=N, freqs=f)
    # the basis itself: row m is w[n] cos / sin (2 pi f_m n / sr), checked at 50 digits
    import mpmath
    mpmath.mp.dps = 50
    w = orc.window(N)
    for (m, n) in [(0, 1), (5, 511), (31, 300), (17, 256)]:
        arg = 2 * mpmath.pi * mpmath.mpf(f[m]) * n / mpmath.mpf(sr)
        # an FP64 argument of size |arg| carries ~|arg| ulp of phase error
        tol = 1e-15 * (1.0 + float(arg))
        assert Wr[m, n] == pytest.approx(float(mpmath.cos(arg)) * w[n], abs=tol)
        assert Wi[m, n] == pytest.approx(float(mpmath.sin(arg)) * w[n], abs=tol)
    L1, R1, I1 = orc.melt_forward(x, sr=sr, n_fft=N, hop=H, freqs=f, return_ri=True)
    L2, R2, I2 = orc.melt_forward_basis(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, return_ri=True)
    assert np.allclose(R1, R2, rtol=1e-12, atol=1e-12) and np.allclose(I1, I2, rtol=1e-12, atol=1e-12)
    assert np.allclose(L1, L2, atol=1e-10)


def test_silence_maps_to_log_floor(orc):
    """P4: x = 0 gives S = 0, so out = ln(eps) exactly, in both pipelines."""
    x = np.zeros(4000, np.float32)
    for eps in (1e-10, 1e-6):
        L = orc.melt_forward(x, sr=16000.0, n_fft=400, hop=160, freqs=orc.melt_frequencies(80, 0, 8000), eps=eps)
        assert np.all(L == math.log(eps))
        L2 = orc.stft_mel_forward(x, sr=16000.0, n_fft=400, hop=160, n_mels=80, fmin=0, fmax=8000, eps=eps)
        assert np.all(L2 == math.log(eps))


def test_output_kinds(orc):
    x = _frame(1000, 4)
    f = orc.melt_frequencies(16, 0, 8000)
    kw = dict(sr=16000.0, n_fft=400, hop=160, freqs=f, eps=1e-10)
    S = orc.melt_forward(x, out_kind=orc.OUT_POWER, **kw)
    assert np.allclose(orc.melt_forward(x, out_kind=orc.OUT_MAGNITUDE, **kw), np.sqrt(S), rtol=1e-14)
    assert np.allclose(orc.melt_forward(x, out_kind=orc.OUT_LOG_POWER, **kw), np.log(S + 1e-10), rtol=1e-14)
    assert np.allclose(orc.melt_forward(x, out_kind=orc.OUT_LOG_MAGNITUDE, **kw), np.log(np.sqrt(S) + 1e-10),
                       rtol=1e-14)


def test_ragged_clips_equal_separate_calls(orc):
    """Frames never straddle clips: a batched call equals per-clip calls concatenated;
    empty and shorter-than-N clips contribute no frames."""
    lengths = [0, 399, 400, 1234, 5, 2000, 560]
    wave, off = workloads.random_clips(lengths, seed=7)
    f = orc.melt_frequencies(20, 0, 8000)
    kw = dict(sr=16000.0, n_fft=400, hop=160, freqs=f)
    L = orc.melt_forward(wave, off, **kw)
    parts = [orc.melt_forward(wave[off[c]:off[c + 1]], **kw) for c in range(len(lengths))]
    assert L.shape[0] == sum(p.shape[0] for p in parts) == sum(orc.num_frames(n, 400, 160) for n in lengths)
    assert np.array_equal(L, np.concatenate(parts))


# ------------------------------------------------------------------ STFT + filterbank

def test_parseval(orc):
    """P5: sum over all N bins of |X_k|^2 = N sum_n (w x)^2; the one-sided spectrum counts
    bins 1..N/2-1 twice."""
    for N in (400, 512, 1024, 15):
        x = _frame(3 * N, 5)
        P = orc.power_spectrum(x, n_fft=N, hop=N)
        w = orc.window(N)
        for t in range(P.shape[0]):
            xt = w * x[t * N:(t + 1) * N].astype(np.float64)
            full = P[t, 0] + 2 * P[t, 1:(N + 1) // 2].sum() + (P[t, N // 2] if N % 2 == 0 else 0.0)
            assert full == pytest.approx(N * np.sum(xt * xt), rel=1e-12)


@pytest.mark.parametrize("N,sr,M,fmin,fmax", [(400, 16000, 80, 0.0, 8000.0), (400, 16000, 80, 80.0, 7600.0),
                                               (512, 16000, 128, 0.0, 8000.0), (1024, 22050, 128, 0.0, 11025.0),
                                               (400, 16000, 128, 0.0, 8000.0)])
def test_filterbank_matches_library(orc, N, sr, M, fmin, fmax):
    """The HTK triangular filterbank equals transformers.audio_utils.mel_filter_bank
    (a torchaudio/librosa-derived routine) with and without area normalisation."""
    from transformers.audio_utils import mel_filter_bank
    for norm, lib_norm in ((orc.NORM_NONE, None), (orc.NORM_SLANEY, "slaney")):
        F = orc.mel_filterbank(n_fft=N, sr=sr, n_mels=M, fmin=fmin, fmax=fmax, norm=norm)
        ref = mel_filter_bank(N // 2 + 1, M, fmin, fmax, sr, norm=lib_norm, mel_scale="htk").T
        assert np.allclose(F, ref, rtol=1e-10, atol=1e-12)


def test_filterbank_partition_of_unity(orc):
    """P6: unnormalised triangles sum to 1 at every bin between the first and last centre,
    and a triangle peaks at 1 on its centre."""
    N, sr, M = 1024, 16000.0, 40
    F = orc.mel_filterbank(n_fft=N, sr=sr, n_mels=M, fmin=0.0, fmax=8000.0)
    g = orc.mel_grid_hz(M, 0.0, 8000.0)
    fk = np.arange(N // 2 + 1) * sr / N
    inner = (fk >= g[1]) & (fk <= g[M])
    assert np.allclose(F.sum(axis=0)[inner], 1.0, atol=1e-12)
    assert np.all(F >= 0.0)
    # nnz bound of Eq. complexity_conv: nnz(F) <= M (N/2 + 1)
    assert np.count_nonzero(F) <= M * (N // 2 + 1)


def test_empty_filters_at_128_mels(orc):
    """At 16 kHz, N=400 and 128 HTK bins over 0-8 kHz the lowest triangles are narrower than
    the 40 Hz bin spacing; the ones that contain no bin are all-zero rows, so the comparator
    outputs ln(eps) there."""
    F = orc.mel_filterbank(n_fft=400, sr=16000.0, n_mels=128, fmin=0.0, fmax=8000.0)
    empty = np.where(F.sum(axis=1) == 0.0)[0]
    assert len(empty) >= 1 and np.all(empty < 16)


def test_stft_mel_matches_library_pipeline(orc):
    """The whole comparator (frame, symmetric Hann, DFT power, HTK filterbank, ln) equals
    transformers.audio_utils.spectrogram with numpy's FFT (single-precision spectrum, so
    the tolerance is float32-level)."""
    from transformers.audio_utils import mel_filter_bank, spectrogram, window_function
    cfg = workloads.config1(seed=3)
    x = cfg["wave"]
    N, H, sr, M = 400, 160, 16000, 80
    fb = mel_filter_bank(N // 2 + 1, M, 0.0, 8000.0, sr, norm=None, mel_scale="htk")
    ref = spectrogram(x, window_function(N, "hann", periodic=False), N, H, power=2.0, center=False,
                      mel_filters=fb, mel_floor=0.0, dtype=np.float64).T
    out = orc.stft_mel_forward(x, sr=sr, n_fft=N, hop=H, n_mels=M, fmin=0.0, fmax=8000.0,
                               out_kind=orc.OUT_POWER)
    assert out.shape == ref.shape == (98, 80)
    assert np.allclose(out, ref, rtol=2e-6, atol=1e-9 * ref.max())
    L = orc.stft_mel_forward(x, sr=sr, n_fft=N, hop=H, n_mels=M, fmin=0.0, fmax=8000.0, eps=1e-10)
    assert np.allclose(L, np.log(out + 1e-10), rtol=1e-14)
    mag = orc.stft_mel_forward(x, sr=sr, n_fft=N, hop=H, n_mels=M, fmin=0.0, fmax=8000.0,
                               out_kind=orc.OUT_MAGNITUDE)
    ref1 = spectrogram(x, window_function(N, "hann", periodic=False), N, H, power=1.0, center=False,
                       mel_filters=fb, mel_floor=0.0, dtype=np.float64).T
    assert np.allclose(mag, ref1, rtol=2e-6, atol=1e-9 * ref1.max())


# ------------------------------------------------------------------ gradient

def _tiny():
    # N=16, H=4, 4 analysis frequencies, 64 samples on a dyadic grid so that x +- h is
    # exact in float32
    rng = np.random.default_rng(11)
    x = (np.round(rng.uniform(-1, 1, 64) * 256) / 256).astype(np.float32)
    return x, 16, 4


def test_gradient_wave_central_difference(orc):
    """P10: for the power output S is quadratic in x, so the central difference with a
    float32-exact step is exact; for the log output it agrees to O(h^2)."""
    x, N, H = _tiny()
    f = np.array([1000.0, 2345.6, 4000.0, 7000.0])
    Wr, Wi = orc.melt_basis(sr=16000.0, n_fft=N, freqs=f)
    T = orc.num_frames(x.size, N, H)
    g = np.random.default_rng(12).standard_normal((T, 4))
    for kind, h, tol in ((orc.OUT_POWER, 2.0 ** -8, 1e-11), (orc.OUT_LOG_POWER, 2.0 ** -14, 2e-6)):
        gx, _, _ = orc.melt_backward(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, grad_out=g, out_kind=kind, eps=1e-3)
        fd = np.empty(x.size)
        for s in range(x.size):
            xp = x.copy(); xp[s] += np.float32(h)
            xm = x.copy(); xm[s] -= np.float32(h)
            op = orc.melt_forward_basis(xp, n_fft=N, hop=H, Wr=Wr, Wi=Wi, out_kind=kind, eps=1e-3)
            om = orc.melt_forward_basis(xm, n_fft=N, hop=H, Wr=Wr, Wi=Wi, out_kind=kind, eps=1e-3)
            fd[s] = np.sum(g * (op - om)) / (2 * h)
        assert np.allclose(gx, fd, rtol=tol, atol=tol * np.abs(fd).max())
    # samples after the last frame get zero gradient
    x2 = np.concatenate([x, np.ones(3, np.float32)])
    gx2, _, _ = orc.melt_backward(x2, n_fft=N, hop=H, Wr=Wr, Wi=Wi, grad_out=g, out_kind=orc.OUT_POWER)
    assert np.all(gx2[-3:] == 0.0)


def test_gradient_basis_central_difference(orc):
    """P10: dWr, dWi against central differences of the basis entries (FP64)."""
    x, N, H = _tiny()
    f = np.array([500.0, 3000.0, 6500.0])
    Wr, Wi = orc.melt_basis(sr=16000.0, n_fft=N, freqs=f)
    T = orc.num_frames(x.size, N, H)
    g = np.random.default_rng(13).standard_normal((T, 3))
    _, dWr, dWi = orc.melt_backward(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, grad_out=g, eps=1e-3)
    h = 1e-6
    for (which, dW) in ((0, dWr), (1, dWi)):
        for (m, n) in [(0, 0), (1, 7), (2, 15), (0, 9)]:
            Wp = [Wr.copy(), Wi.copy()]; Wp[which][m, n] += h
            Wm = [Wr.copy(), Wi.copy()]; Wm[which][m, n] -= h
            op = orc.melt_forward_basis(x, n_fft=N, hop=H, Wr=Wp[0], Wi=Wp[1], eps=1e-3)
            om = orc.melt_forward_basis(x, n_fft=N, hop=H, Wr=Wm[0], Wi=Wm[1], eps=1e-3)
            fd = np.sum(g * (op - om)) / (2 * h)
            assert dW[m, n] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_backward_linear_adjoint(orc):
    """P10 adjoint test: the transposed projection is the adjoint of the projection
    R = X Wr^T, I = X Wi^T, both in the waveform, <Gr, R(v)> + <Gi, I(v)> = <dx(G), v>, and
    in the basis, <Gr, X Vr^T> + <Gi, X Vi^T> = <dWr, Vr> + <dWi, Vi>, for random G, v, V on
    ragged clips (a clip tail that no frame covers gets zero)."""
    rng = np.random.default_rng(21)
    lengths = [37, 0, 100, 64, 15]
    x = rng.standard_normal(sum(lengths)).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    N, H, M = 16, 5, 3
    Wr, Wi = rng.standard_normal((M, N)), rng.standard_normal((M, N))
    T = orc.total_frames(off, N, H)
    Gr, Gi = rng.standard_normal((T, M)), rng.standard_normal((T, M))
    gx, dWr, dWi = orc.melt_backward_linear(x, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, Gr=Gr, Gi=Gi)
    v = rng.standard_normal(x.size).astype(np.float32)
    _, Rv, Iv = orc.melt_forward_basis(v, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, out_kind=orc.OUT_POWER,
                                       return_ri=True)
    lhs = np.sum(Gr * Rv) + np.sum(Gi * Iv)
    assert lhs == pytest.approx(float(np.dot(gx, v.astype(np.float64))), rel=1e-12)
    Vr, Vi = rng.standard_normal((M, N)), rng.standard_normal((M, N))
    _, RV, IV = orc.melt_forward_basis(x, off, n_fft=N, hop=H, Wr=Vr, Wi=Vi, out_kind=orc.OUT_POWER,
                                       return_ri=True)
    assert np.sum(Gr * RV) + np.sum(Gi * IV) == pytest.approx(np.sum(dWr * Vr) + np.sum(dWi * Vi), rel=1e-12)
    # samples after the last frame of a clip, and clips shorter than a frame, get zero
    T0 = orc.num_frames(lengths[0], N, H)
    tail = off[0] + (T0 - 1) * H + N
    assert tail < off[1] and np.all(gx[tail:off[1]] == 0.0) and np.all(gx[off[4]:off[5]] == 0.0)
    assert np.all(gx[:tail] != 0.0)


def test_chain_then_linear_is_the_gradient(orc):
    """The gradient splits into the chain rule through the output map (oracle_melt_chain)
    and the transposed projection: the composition equals oracle_melt_backward (itself
    pinned by central differences above) for every output kind."""
    x, N, H = _tiny()
    f = np.array([700.0, 2000.0, 5100.0])
    Wr, Wi = orc.melt_basis(sr=16000.0, n_fft=N, freqs=f)
    T = orc.num_frames(x.size, N, H)
    g = np.random.default_rng(14).standard_normal((T, 3))
    _, R, I = orc.melt_forward_basis(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, return_ri=True)
    for kind in (orc.OUT_LOG_POWER, orc.OUT_LOG_MAGNITUDE, orc.OUT_POWER, orc.OUT_MAGNITUDE):
        Gr, Gi = orc.melt_chain(R, I, g, out_kind=kind, eps=1e-3)
        a = orc.melt_backward_linear(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, Gr=Gr, Gi=Gi)
        b = orc.melt_backward(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, grad_out=g, out_kind=kind, eps=1e-3)
        for u, w in zip(a, b):
            assert np.allclose(u, w, rtol=1e-13, atol=1e-15)


# ------------------------------------------------------------------ MFCCT (Eq. mfcct_matrix)

def test_dct_matches_scipy(orc):
    from scipy.fft import dct
    M, K = 80, 40
    D = orc.dct2_ortho(K, M)
    eye = np.eye(M)
    ref = dct(eye, type=2, norm="ortho", axis=0)[:K]      # columns: DCT of unit vectors
    assert np.allclose(D, ref, atol=1e-14)
    assert np.allclose(orc.dct2_ortho(M, M) @ orc.dct2_ortho(M, M).T, eye, atol=1e-13)


# ------------------------------------------------------------------ operand rounding models

def test_rounding_models_match_torch_casts(orc):
    import torch
    rng = np.random.default_rng(21)
    v = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.uniform(-12, 3, 3000),
                        [0.0, -0.0, 1.0, -1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 2.0 ** -130, 6.1e-5, 65504.0],
                        # bf16 / fp16 / e4m3 halfway points (ties to even)
                        [1 + 2 ** -8 + 2 ** -9, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 1.0625, 1.1875, 2.0 ** -10,
                         3 * 2.0 ** -10, 440.0, 447.0]]).astype(np.float32)
    t = torch.from_numpy(v)
    assert np.array_equal(orc.round_bf16(v), t.to(torch.bfloat16).to(torch.float64).numpy())
    assert np.array_equal(orc.round_fp16(v), t.to(torch.float16).to(torch.float64).numpy())
    inr = np.abs(v) < 448.0
    assert np.array_equal(orc.round_e4m3(v[inr]), t[torch.from_numpy(inr)].to(torch.float8_e4m3fn)
                          .to(torch.float64).numpy())
    # saturation beyond the largest finite E4M3 value
    assert np.array_equal(orc.round_e4m3(np.array([448.0, 460.0, 464.0, 1e6, -1e6], np.float32)),
                          [448.0, 448.0, 448.0, 448.0, -448.0])


def test_quant_models_are_consistent(orc):
    """With operands already representable in the format, the operand model reduces to the
    plain FP64 projection; BF16x3 recovers about 16 bits of every product."""
    N, H, sr = 400, 160, 16000.0
    f = orc.melt_frequencies(16, 0, 8000)
    Wr, Wi = orc.melt_basis(sr=sr, n_fft=N, freqs=f)
    x = _frame(2000, 8)
    xb = orc.round_bf16(x).astype(np.float32)
    Wrb, Wib = orc.round_bf16(Wr.astype(np.float32)), orc.round_bf16(Wi.astype(np.float32))
    ref = orc.melt_forward_basis(xb, n_fft=N, hop=H, Wr=Wrb, Wi=Wib, out_kind=orc.OUT_POWER)
    q = orc.melt_forward_quant(xb, n_fft=N, hop=H, Wr=Wrb, Wi=Wib, prec=orc.PREC_BF16, out_kind=orc.OUT_POWER)
    assert np.allclose(q, ref, rtol=1e-13)
    exact = orc.melt_forward_basis(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, out_kind=orc.OUT_POWER)
    q3 = orc.melt_forward_quant(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=orc.PREC_BF16X3, out_kind=orc.OUT_POWER)
    q1 = orc.melt_forward_quant(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=orc.PREC_BF16, out_kind=orc.OUT_POWER)
    act = exact > 1e-6 * exact.max()
    e3 = np.abs(q3[act] / exact[act] - 1).max()
    e1 = np.abs(q1[act] / exact[act] - 1).max()
    assert e3 < 1e-3 and e3 < e1 / 30
    q8 = orc.melt_forward_quant(x, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=orc.PREC_FP8_E4M3, out_kind=orc.OUT_POWER)
    loud = exact > 1e-2 * exact.max()
    assert np.median(np.abs(q8[loud] / exact[loud] - 1)) < 0.1


def test_split_fp16_model_against_numpy_float16(orc):
    """The split-binary16 operand model (waveform pre-scaled by 2^10, hi + lo parts of the
    waveform and of the FP32 basis, xh Wh + xh Wl + xl Wh, unscaled) equals the same steps
    written with numpy's IEEE binary16 casts; its error against the exact projection stays
    within 3 2^-21 of sum |x W| (about 22 significant bits, FP32-level), at least 16 times
    below split bfloat16's where the samples are above 1e-4; a sample beyond binary16's range after the pre-scale makes its frames
    non-finite."""
    N, H, sr = 400, 160, 16000.0
    f = orc.melt_frequencies(16, 0, 8000)
    Wr, Wi = orc.melt_basis(sr=sr, n_fft=N, freqs=f)
    # amplitudes over 100 dB, so that low parts of quiet samples are exercised
    x = (_frame(2400, 31) * np.repeat(10.0 ** np.linspace(-5, 0, 6), 400)).astype(np.float32)
    off = np.array([0, x.size], np.int64)
    _, R, I = orc.melt_forward_quant(x, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=orc.PREC_FP16X3, return_ri=True)

    def split(v):
        hi = v.astype(np.float16)
        lo = (v - hi.astype(np.float32)).astype(np.float16)
        return hi.astype(np.float64), lo.astype(np.float64)

    xs = x * np.float32(1024.0)
    T = 1 + (x.size - N) // H
    for W, P in ((Wr, R), (Wi, I)):
        Wh, Wl = split(W.astype(np.float32))
        for t in range(T):
            xh, xl = split(xs[t * H:t * H + N])
            terms = xh * Wh + xh * Wl + xl * Wh
            ref = terms.sum(axis=1) / 1024.0
            scale = np.abs(terms).sum(axis=1) / 1024.0
            assert np.all(np.abs(P[t] - ref) <= 1e-12 * scale)
    exact = orc.melt_forward_basis(x, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, return_ri=True)[1]
    _, Rb, _ = orc.melt_forward_quant(x, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=orc.PREC_BF16X3, return_ri=True)
    sumabs = np.stack([np.abs(x[t * H:t * H + N].astype(np.float64)) @ np.abs(Wr).T for t in range(T)])
    e16 = np.abs(R - exact) / sumabs
    eb16 = np.abs(Rb - exact) / sumabs
    assert e16.max() <= 3 * 2.0 ** -21
    # frames from the third on hold samples of at least 1e-4 (the first straddle 1e-5, where the
    # binary16 low parts fall below the normal range and the error nears split bfloat16's)
    print(f"max error / sum|xW| from frame 3: split binary16 {e16[3:].max():.3g}, split bfloat16 {eb16[3:].max():.3g}")
    assert e16[3:].max() < eb16[3:].max() / 16
    # overflow: a sample of 64 is beyond binary16's range after the 2^10 pre-scale
    xo = x.copy()
    xo[500] = 64.0
    qo = orc.melt_forward_quant(xo, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=orc.PREC_FP16X3, out_kind=orc.OUT_POWER)
    assert not np.all(np.isfinite(qo[:3])) and np.all(np.isfinite(qo[4:]))


def test_block_exponent_is_the_largest_fitting_power_of_two(orc):
    """The block exponent is the largest integer e with 2^e m <= 448 (so 2^(e+1) m > 448),
    within the E8M0-undoable range [-127, 127], and 0 for a silent block."""
    rng = np.random.default_rng(5)
    m = np.concatenate([10.0 ** rng.uniform(-30, 30, 4000),
                        [448.0, 449.0, 224.0, 1.0, 1.75, 1.76, 3.5, 2.0 ** -100, 1e-37, 3e38]]).astype(np.float32)
    e = orc.block_exponent(m)
    m64 = m.astype(np.float64)
    assert np.all(np.ldexp(m64, e) <= 448.0)
    free = (e > -127) & (e < 127)
    assert np.all(np.ldexp(m64[free], e[free] + 1) > 448.0)
    assert orc.block_exponent(np.float32(0.0)) == 0
    assert list(orc.block_exponent(np.array([448, 449, 1.0, 1.76], np.float32))) == [0, -1, 8, 7]


def test_block_scaled_fp8_model_against_torch_float8(orc):
    """The FP8 block-scaled operand model (32-sample blocks from each clip's first sample,
    samples scaled by 2^e_b and cast to E4M3, basis rows scaled by 448 / max|row| and cast)
    equals the same steps written with torch's float8_e4m3fn casts and numpy block maxima, on
    two clips of uneven length and 80 dB of dynamics; scaling the waveform by a power of two
    scales R and I by exactly that power; on loud bins its error against the exact projection
    is that of 3-bit significands."""
    import torch
    N, H, sr = 400, 160, 16000.0
    f = orc.melt_frequencies(16, 0, 8000)
    Wr, Wi = orc.melt_basis(sr=sr, n_fft=N, freqs=f)
    lens = [2000, 1333]
    gains = np.concatenate([np.repeat(10.0 ** np.linspace(-4, 0, 5), 400), np.full(1333, 0.3)])
    x = (_frame(sum(lens), 17) * gains).astype(np.float32)
    off = np.array([0, lens[0], sum(lens)], np.int64)
    _, R, I = orc.melt_forward_quant(x, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=orc.PREC_FP8_E4M3_BLOCK32,
                                     return_ri=True)

    def e4m3(v):
        return torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()

    def block_exp(mx):
        # largest e with 2^e mx <= 448, by brute force over the whole range
        es = np.arange(-127, 128)
        ok = np.ldexp(mx[:, None], es[None, :]) <= 448.0
        return np.where(mx > 0, es[np.where(ok, es[None, :], -999).argmax(axis=1)], 0)

    xq = np.zeros(x.size)
    for c in range(2):
        seg = x[off[c]:off[c + 1]]
        nb = (seg.size + 31) // 32
        pad = np.zeros(nb * 32, np.float32)
        pad[:seg.size] = seg
        e = block_exp(np.abs(pad.reshape(nb, 32)).max(axis=1).astype(np.float64))
        ee = np.repeat(e, 32)[:seg.size]
        scaled = (seg.astype(np.float64) * np.ldexp(1.0, ee)).astype(np.float32)    # exact
        xq[off[c]:off[c + 1]] = np.ldexp(e4m3(scaled), -ee)
    row = 0
    for c in range(2):
        T = 1 + (lens[c] - N) // H
        for W, P in ((Wr, R), (Wi, I)):
            W32 = W.astype(np.float32)
            rs = np.float32(448.0) / np.abs(W32).max(axis=1)
            Wq = e4m3(W32 * rs[:, None]) / rs[:, None].astype(np.float64)
            for t in range(T):
                terms = Wq * xq[off[c] + t * H:off[c] + t * H + N]
                ref = terms.sum(axis=1)
                assert np.all(np.abs(P[row + t] - ref) <= 1e-12 * np.abs(terms).sum(axis=1) + 1e-300)
        row += T
    # power-of-two equivariance: every block exponent shifts, the E4M3 codes stay the same
    for k in (-7, 5):
        _, R2, I2 = orc.melt_forward_quant(np.ldexp(x, k).astype(np.float32), off, n_fft=N, hop=H, Wr=Wr, Wi=Wi,
                                           prec=orc.PREC_FP8_E4M3_BLOCK32, return_ri=True)
        assert np.array_equal(R2, np.ldexp(R, k)) and np.array_equal(I2, np.ldexp(I, k))
    exact = orc.melt_forward_basis(x, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, out_kind=orc.OUT_POWER)
    q = R ** 2 + I ** 2
    loud = exact > 1e-2 * exact.max(axis=1, keepdims=True)
    assert np.median(np.abs(q[loud] / exact[loud] - 1)) < 0.1


# ------------------------------------------------------------------ values the paper prints

def test_paper_log_convention(orc):
    """The paper's equivalence margin is printed both in nats and in dB (0.244 nat = 1.06 dB),
    which fixes the natural log in Eq. meltf and 10 log10 on power when converting to dB."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        gold = json.load(fh)
    d = gold["equivalence_margin"]
    assert round(d["nat"] * 10.0 / math.log(10.0), 2) == d["dB"]
    # the other candidate conventions do not reproduce the printed pair
    assert round(d["nat"] * 20.0 / math.log(10.0), 2) != d["dB"]
    assert round(d["nat"] * 10.0, 2) != d["dB"]


def test_cepstrum_closed_forms(orc):
    """Eq. mfcct_matrix: a constant log-Mel row c has only the DC coefficient c sqrt(M); with
    K = M the orthonormal DCT-II inverts exactly (C D = L); a single cosine row
    cos(pi k0 (m + 1/2) / M) has only coefficient k0, of size sqrt(M / 2)."""
    M = 80
    L = np.full((2, M), -3.25)
    C = orc.cepstrum(L, 40)
    assert np.allclose(C[:, 0], -3.25 * np.sqrt(M), rtol=1e-14) and np.allclose(C[:, 1:], 0.0, atol=1e-12)
    rng = np.random.default_rng(4)
    L = rng.standard_normal((5, M))
    C = orc.cepstrum(L, M)
    assert np.allclose(C @ orc.dct2_ortho(M, M), L, atol=1e-12)
    k0 = 7
    row = np.cos(np.pi * k0 * (np.arange(M) + 0.5) / M)[None, :]
    C = orc.cepstrum(row, 40)
    assert abs(C[0, k0] - np.sqrt(M / 2)) < 1e-12
    assert np.allclose(np.delete(C[0], k0), 0.0, atol=1e-12)
