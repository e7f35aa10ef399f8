"""GPU parity of the comparator (hand-written FFT + sparse Mel filterbank) against the FP64
STFT oracle (naive DFT + dense triangular filterbank), with the FFT error bound of
tests/parity.py as the pass condition."""
import numpy as np
import pytest

import workloads
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def melt():
    import paper_2606_01009_amd as m
    m.load_library()
    return m


def _run(torch, melt, plan, wave, off):
    T = melt.total_frames(off, plan.n_fft, plan.hop)
    d_wave = torch.from_numpy(np.ascontiguousarray(wave)).cuda()
    d_off = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    out = torch.full((T, plan.n_mels), float("nan"), dtype=torch.float32, device="cuda")
    plan.stft_mel(d_wave, d_off, T, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(orc, plan, L, wave, off, sr, fmin, fmax, norm=0, label=""):
    N, H, M = plan.n_fft, plan.hop, plan.n_mels
    P = orc.power_spectrum(wave, off, n_fft=N, hop=H)
    F = orc.mel_filterbank(n_fft=N, sr=sr, n_mels=M, fmin=fmin, fmax=fmax, norm=norm)
    pn = parity.fft_pair_norms(wave, off, N, H, orc.window(N))
    st = parity.check_stft_log(L, P, F, pn, N, 1e-10, label=label)
    print(f"{label}: dB error vs FP64 oracle on active bins: max {st['max_db']:.3g} rms {st['rms_db']:.3g}")
    return st


def test_config1(torch, melt, orc):
    cfg = workloads.config1()
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, fmin=0, fmax=8000)
    L = _run(torch, melt, plan, cfg["wave"], cfg["offsets"])
    assert L.shape == (98, 80)
    st = _check(orc, plan, L, cfg["wave"], cfg["offsets"], 16000.0, 0.0, 8000.0, label="stft config1")
    assert st["max_db"] < 0.02


@pytest.mark.parametrize("n_mels", [80, 128])
def test_config2_reduced(torch, melt, orc, n_mels):
    cfg = workloads.config2(n_mels=n_mels, n_clips=4, seconds=2.5)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=n_mels, fmin=0, fmax=8000)
    L = _run(torch, melt, plan, cfg["wave"], cfg["offsets"])
    _check(orc, plan, L, cfg["wave"], cfg["offsets"], 16000.0, 0.0, 8000.0, label=f"stft config2-reduced M={n_mels}")
    if n_mels == 128:
        # filters that contain no FFT bin give exactly the log floor (ln eps in FP32)
        F = orc.mel_filterbank(n_fft=400, sr=16000.0, n_mels=128, fmin=0.0, fmax=8000.0)
        empty = np.where(F.sum(axis=1) == 0)[0]
        assert len(empty) > 0
        assert np.all(L[:, empty] == L[0, empty[0]]) and abs(L[0, empty[0]] - np.log(1e-10)) < 4e-6


@pytest.mark.parametrize("geom", [(16000, 512, 128, 128, 0.0, 8000.0), (22050, 1024, 256, 128, 0.0, 11025.0),
                                  (16000, 400, 160, 80, 80.0, 7600.0), (16000, 256, 100, 40, 0.0, 8000.0),
                                  (16000, 1200, 160, 128, 0.0, 8000.0)])
def test_geometries_ragged(torch, melt, orc, geom):
    sr, N, H, M, fmin, fmax = geom
    lengths = [0, N - 1, N, N + H, 7 * N + 3, 40 * H + N + 5, 3]
    wave, off = workloads.random_clips(lengths, seed=13)
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, fmin=fmin, fmax=fmax)
    L = _run(torch, melt, plan, wave, off)
    assert L.shape[0] == sum(melt.melt_num_frames(n, N, H) for n in lengths)
    _check(orc, plan, L, wave, off, float(sr), fmin, fmax, label=f"stft {geom}")


def test_slaney_norm_and_magnitude(torch, melt, orc):
    cfg = workloads.config1(seed=2)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, fb_norm=melt.MELT_FB_NORM_SLANEY)
    L = _run(torch, melt, plan, cfg["wave"], cfg["offsets"])
    _check(orc, plan, L, cfg["wave"], cfg["offsets"], 16000.0, 0.0, 8000.0, norm=1, label="stft slaney")
    plan2 = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, output=melt.MELT_OUT_MAGNITUDE)
    Mg = _run(torch, melt, plan2, cfg["wave"], cfg["offsets"])
    ref = orc.stft_mel_forward(cfg["wave"], sr=16000.0, n_fft=400, hop=160, n_mels=80, fmin=0.0, fmax=8000.0,
                               out_kind=orc.OUT_MAGNITUDE)
    loud = ref > 1e-3 * ref.max()
    assert np.allclose(Mg[loud], ref[loud], rtol=1e-4)


def test_silence(torch, melt):
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    L = _run(torch, melt, plan, np.zeros(8000, np.float32), np.array([0, 8000]))
    assert np.all(L == L[0, 0]) and abs(L[0, 0] - np.log(1e-10)) < 4e-6


def test_full_size_sampled(torch, melt, orc):
    """The benchmark's batch and launch (64 x 30 s, 191 872 frames), sampled frames vs oracle."""
    cfg = workloads.config2(n_mels=80)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    L = _run(torch, melt, plan, cfg["wave"], cfg["offsets"])
    assert L.shape == (191872, 80) and np.all(np.isfinite(L))
    rng = np.random.default_rng(3)
    # sample pairs (even frame and its partner) so the FFT-packing bound is exact
    ev = 2 * rng.integers(0, 191872 // 2, 96)
    ids = np.unique(np.concatenate([ev, ev + 1]))
    sub, off = parity.frames_as_clips(cfg["wave"], cfg["offsets"], 400, 160, ids)
    # every clip has an even frame count (2998), so global frame f shares its FFT with f ^ 1;
    # both are in the sample, and the pair norm comes from the two sampled frames
    P = orc.power_spectrum(sub, off, n_fft=400, hop=160)
    F = orc.mel_filterbank(n_fft=400, sr=16000.0, n_mels=80, fmin=0.0, fmax=8000.0)
    w = orc.window(400)
    e = np.array([np.sum((w * sub[i * 400:(i + 1) * 400].astype(np.float64)) ** 2) for i in range(len(ids))])
    pos = {f: i for i, f in enumerate(ids)}
    pn = np.array([e[i] + (e[pos[f ^ 1]] if (f ^ 1) in pos else e.max()) for i, f in enumerate(ids)])
    parity.check_stft_log(L[ids], P, F, pn, 400, 1e-10, label="stft full sampled")


_CONFIG4 = {}


@pytest.mark.parametrize("variant", ["16k", "22k"])
def test_config4_full_size_sampled(torch, melt, orc, variant):
    """The ragged systems batch at full size (512 clips of U[0.5, 30] s; 16 kHz / N 512 / H 128
    or 22.05 kHz / N 1024 / H 256; 128 Mel bins up to the Nyquist frequency), as the systems
    benchmark launches the comparator.  The first and last frame of every clip and 128 random
    frames are checked against the oracle on those frames; the FFT bound takes each frame's
    own energy plus that of the frame sharing its complex FFT (clip-local index l ^ 1, none past
    the clip's last frame)."""
    if variant not in _CONFIG4:
        _CONFIG4.clear()
        _CONFIG4[variant] = workloads.config4(variant)
    cfg = _CONFIG4[variant]
    N, H, sr = cfg["n_fft"], cfg["hop"], cfg["sr"]
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=128, fmin=0.0, fmax=sr / 2)
    wave = cfg["wave"]
    off = np.asarray(cfg["offsets"], np.int64)
    L = _run(torch, melt, plan, wave, off)
    lens = off[1:] - off[:-1]
    T_c = np.where(lens >= N, 1 + (lens - N) // H, 0)
    fo = np.concatenate([[0], np.cumsum(T_c)])
    assert L.shape == (fo[-1], 128) and np.all(np.isfinite(L))
    has = T_c > 0
    rng = np.random.default_rng(4041)
    ids = np.unique(np.concatenate([fo[:-1][has], fo[1:][has] - 1, rng.integers(0, fo[-1], 128)]))
    clip = np.searchsorted(fo, ids, side="right") - 1
    loc = ids - fo[clip]
    w = orc.window(N)

    def energy(c, l):
        s0 = off[c] + l * H
        return float(np.sum((w * wave[s0:s0 + N].astype(np.float64)) ** 2))

    pn = np.array([energy(c, l) + (energy(c, l ^ 1) if (l ^ 1) < T_c[c] else 0.0) for c, l in zip(clip, loc)])
    sub, soff = parity.frames_as_clips(wave, off, N, H, ids)
    P = orc.power_spectrum(sub, soff, n_fft=N, hop=H)
    F = orc.mel_filterbank(n_fft=N, sr=sr, n_mels=128, fmin=0.0, fmax=sr / 2)
    st = parity.check_stft_log(L[ids], P, F, pn, N, 1e-10, label=f"stft config4 {variant} full sampled")
    print(f"stft config4 {variant}: dB error vs FP64 oracle on active bins: max {st['max_db']:.3g} "
          f"rms {st['rms_db']:.3g}")


def _many_lengths(n, N, H, seed):
    """n clip lengths from 0 to N + 12 H samples (empty, sub-frame and short clips), so the
    chunk schedule runs over several blocks of 1024 clips."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, N + 12 * H, n)


def test_many_clips_schedule(torch, melt, orc):
    """2600 clips: the schedule's prefix sums carry across blocks of 1024 clips, and the
    chunk table of a short batch uses one-sub-task chunks."""
    lengths = _many_lengths(2600, 400, 160, seed=21)
    wave, off = workloads.random_clips(lengths, seed=22)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    L = _run(torch, melt, plan, wave, off)
    assert L.shape[0] == sum(melt.melt_num_frames(int(n), 400, 160) for n in lengths)
    _check(orc, plan, L, wave, off, 16000.0, 0.0, 8000.0, label="stft 2600 clips")


def test_long_single_clip(torch, melt, orc):
    """One 160 s clip (15 998 frames): many chunks of one clip, written in parallel."""
    wave, off = workloads.random_clips([160 * 16000], seed=23)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    L = _run(torch, melt, plan, wave, off)
    assert L.shape == (15998, 80)
    _check(orc, plan, L, wave, off, 16000.0, 0.0, 8000.0, label="stft one 160 s clip")
