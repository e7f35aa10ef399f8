"""GPU parity of the cepstral outputs (MELT_OUT_MFCC): MFCCT = ln(S + eps) D^T (Eq.
mfcct_matrix) on the MelT path and the conventional MFCC on the FFT + filterbank path,
against the oracle's composition (log-Mel oracle, then its pinned orthonormal DCT-II).  The
pass condition carries each path's per-bin log-Mel bound through D (tests/parity.py
check_cepstrum).  Also: the paper's cepstral configuration (16 kHz, N = 1200, H = 160,
M = 128, K = 40), streaming equals batch, and the gradient through the cepstrum."""
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


def _gpu(torch, melt, plan, wave, off, comparator=False):
    T = melt.total_frames(off, plan.n_fft, plan.hop)
    d_wave = torch.from_numpy(np.ascontiguousarray(wave)).cuda()
    d_off = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    out = torch.full((T, plan.out_cols), float("nan"), dtype=torch.float32, device="cuda")
    (plan.stft_mel if comparator else plan.forward)(d_wave, d_off, T, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _melt_case(torch, melt, orc, wave, off, sr, N, H, M, K, prec, fmin=0.0, fmax=None):
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, fmin=fmin, fmax=fmax, precision=prec,
                         output=melt.MELT_OUT_MFCC, n_mfcc=K)
    assert plan.out_cols == K
    C = _gpu(torch, melt, plan, wave, off)
    _check_mfcct(orc, plan, C, wave, off, prec)
    return C


def _check_mfcct(orc, plan, C, wave, off, prec, label=""):
    N, H, M, K = plan.n_fft, plan.hop, plan.n_mels, plan.out_cols
    _, Wr, Wi = parity.oracle_basis(orc, plan.cfg)     # the oracle's own centres and basis
    eps = 1e-10
    if prec == "fp32":
        _, R, I = orc.melt_forward_basis(wave, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, eps=eps, return_ri=True)
        _, Ar, Ai = orc.melt_forward_basis(np.abs(wave), off, n_fft=N, hop=H, Wr=np.abs(Wr), Wi=np.abs(Wi), eps=eps,
                                           return_ri=True)
        bL, L = parity.log_error_radius(R, I, Ar, Ai, N, eps, extra_rel=1.0)
    else:
        code = {"bf16": orc.PREC_BF16, "fp16": orc.PREC_FP16, "fp8": orc.PREC_FP8_E4M3,
                "fp8b": orc.PREC_FP8_E4M3_BLOCK32}[prec]
        _, R, I = orc.melt_forward_quant(wave, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=code, eps=eps, return_ri=True)
        _, Ar, Ai = orc.melt_forward_quant(np.abs(wave), off, n_fft=N, hop=H, Wr=np.abs(Wr), Wi=np.abs(Wi), prec=code,
                                           eps=eps, return_ri=True)
        # FP8: the epilogue's unscaling adds up to four FP32 roundings
        bL, L = parity.log_error_radius(R, I, Ar, Ai, N, eps, extra_rel=4.0 if prec in ("fp8", "fp8b") else 0.0)
    D = orc.dct2_ortho(K, M)
    # after a 16-bit or FP8 projection the cepstrum runs as a split binary16 product
    label = label or f"MFCCT {prec} N={N} M={M} K={K}"
    st = parity.check_cepstrum(C, L, bL, D, label=label, split=prec != "fp32")
    print(f"{label}: max |dC| {st['max_abs']:.3g} (bound up to {st['max_bound']:.3g})")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mfcct_cepstral_full_size_sampled(torch, melt, orc, prec):
    """The cepstral workload at full size, as the workload sweep launches it: 64 clips x 30 s,
    N = 1200, H = 160, M = 128, K = 40 (191 552 frames; the K-split projection, then the
    cepstrum).  The first and last frame of every clip and 128 random frames are checked
    against the oracle evaluated on exactly those frames."""
    cfg = workloads.config2(n_mels=128)
    N, H = 1200, 160
    plan = melt.MeltPlan(sample_rate=16000.0, n_fft=N, hop=H, n_mels=128, fmin=0.0, fmax=8000.0, precision=prec,
                         output=melt.MELT_OUT_MFCC, n_mfcc=40)
    C = _gpu(torch, melt, plan, cfg["wave"], cfg["offsets"])
    off = np.asarray(cfg["offsets"], np.int64)
    lens = off[1:] - off[:-1]
    T_c = np.where(lens >= N, 1 + (lens - N) // H, 0)
    fo = np.concatenate([[0], np.cumsum(T_c)])
    assert C.shape == (fo[-1], 40) and fo[-1] == 191552 and np.all(np.isfinite(C))
    rng = np.random.default_rng(1200)
    ids = np.unique(np.concatenate([fo[:-1], fo[1:] - 1, rng.integers(0, fo[-1], 128)]))
    sub, soff = parity.frames_as_clips(cfg["wave"], off, N, H, ids)
    _check_mfcct(orc, plan, C[ids], sub, soff, prec, label=f"MFCCT {prec} cepstral full sampled")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp8", "fp8b"])
def test_mfcct_config1(torch, melt, orc, prec):
    cfg = workloads.config1()
    _melt_case(torch, melt, orc, cfg["wave"], cfg["offsets"], 16000.0, 400, 160, 80, 40, prec, fmax=8000.0)


@pytest.mark.parametrize("K", [1, 13, 31, 33, 40, 64, 80])
def test_mfcct_split_cepstrum_shapes(torch, melt, orc, K):
    """The split binary16 cepstrum over its coefficient tiles (one or two of 32, ragged) and
    Mel widths (80: five groups of 16; 128: eight), on a ragged batch whose row count is not
    a multiple of the 32-row tile.  K = 80 is past two tiles: the FP32 product takes it."""
    lengths = [400, 400 + 160 * 37 + 3, 16000 + 77]
    wave, off = workloads.random_clips(lengths, seed=40 + K)
    M = 128 if K == 64 else 80
    _melt_case(torch, melt, orc, wave, off, 16000.0, 400, 160, M, min(K, M), "bf16", fmax=8000.0)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mfcct_cepstral_configuration_16bit(torch, melt, orc, prec):
    """The cepstral configuration (N = 1200, M = 128, K = 40) at 16 bits: the K-split
    projection kernel (two row groups), then the split binary16 cepstrum."""
    lengths = [1199, 1200, 16000, 5 * 160 + 1200 + 7, 32000]
    wave, off = workloads.random_clips(lengths, seed=13)
    _melt_case(torch, melt, orc, wave, off, 16000.0, 1200, 160, 128, 40, prec, fmax=8000.0)


@pytest.mark.parametrize("M,K", [(16, 13), (64, 40), (64, 64), (80, 13), (128, 33), (128, 64), (112, 1)])
def test_mfcct_k_split_shapes(torch, melt, orc, M, K):
    """MFCCT at N = 1200 (the K-split projection kernel) over one row group (M <= 64) and
    two, one or two coefficient tiles of the split cepstrum, ragged clips whose chunks end in
    a partial frame tile."""
    lengths = [1200 + 160 * 70 + 5, 1200 + 160 * 33, 4000]
    wave, off = workloads.random_clips(lengths, seed=60 + M + K)
    plan = melt.MeltPlan(sample_rate=16000.0, n_fft=1200, hop=160, n_mels=M, fmax=8000.0, precision="bf16",
                         output=melt.MELT_OUT_MFCC, n_mfcc=K)
    assert "k-split" in melt.melt_variant_name(plan.handle, 0)
    _melt_case(torch, melt, orc, wave, off, 16000.0, 1200, 160, M, K, "bf16", fmax=8000.0)


def test_mfcct_is_deterministic_and_keeps_projections(torch, melt):
    """Two MFCCT calls are bit-identical, and the projections an MFCC plan stores for the
    backward equal those of the log-power plan."""
    wave, off = workloads.random_clips([16000, 23456, 1200], seed=71)
    kw = dict(sample_rate=16000.0, n_fft=1200, hop=160, n_mels=128, fmax=8000.0, precision="bf16")
    mf = melt.MeltPlan(output=melt.MELT_OUT_MFCC, n_mfcc=40, **kw)
    lp = melt.MeltPlan(**kw)
    T = melt.total_frames(off, 1200, 160)
    d_wave = torch.from_numpy(np.ascontiguousarray(wave)).cuda()
    d_off = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    outs, projs = [], []
    for plan, cols in ((mf, 40), (mf, 40), (lp, 128)):
        out = torch.full((T, cols), float("nan"), dtype=torch.float32, device="cuda")
        P = torch.full((T, 256), float("nan"), dtype=torch.float32, device="cuda")
        plan.forward(d_wave, d_off, T, out=out, proj=P)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        projs.append(P.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    assert np.all(np.isfinite(outs[0]))
    assert np.array_equal(projs[0], projs[2]) and np.array_equal(projs[1], projs[2])


def test_mfcct_cepstral_configuration(torch, melt, orc):
    """The paper's cepstral configuration: 16 kHz, N = 1200, H = 160, M = 128, K = 40,
    0-8 kHz, on ragged clips."""
    lengths = [1199, 1200, 16000, 5 * 160 + 1200 + 7, 32000]
    wave, off = workloads.random_clips(lengths, seed=12)
    _melt_case(torch, melt, orc, wave, off, 16000.0, 1200, 160, 128, 40, "fp32", fmax=8000.0)


def test_mfcc_comparator(torch, melt, orc):
    """Conventional MFCC: the comparator's log-Mel rows through the same DCT-II."""
    cfg = workloads.config1(seed=3)
    wave, off = cfg["wave"], cfg["offsets"]
    N, H, M, K, eps = 400, 160, 80, 40, 1e-10
    plan = melt.MeltPlan(sample_rate=16000, n_fft=N, hop=H, n_mels=M, fmax=8000.0, output=melt.MELT_OUT_MFCC,
                         n_mfcc=K)
    C = _gpu(torch, melt, plan, wave, off, comparator=True)
    P = orc.power_spectrum(wave, off, n_fft=N, hop=H)
    F = orc.mel_filterbank(sr=16000.0, n_fft=N, n_mels=M, fmin=0.0, fmax=8000.0)
    pn = parity.fft_pair_norms(wave, off, N, H, orc.window(N))
    bound, vac, mel, dmel = parity.stft_log_bound(P, F, pn, N, eps)
    L = np.log(mel + eps)
    width = np.maximum(np.log(mel + dmel + eps) - L, L - np.log(eps * (1 - 2 * parity.U32))) + 1e-6
    bL = np.where(vac, width, bound)
    st = parity.check_cepstrum(C, L, bL, orc.dct2_ortho(K, M), label="MFCC comparator")
    print(f"MFCC comparator: max |dC| {st['max_abs']:.3g}")


def test_mfcct_stream_equals_batch(torch, melt):
    cfg = workloads.config2(n_clips=2, seconds=1.0)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, output=melt.MELT_OUT_MFCC, n_mfcc=13)
    wave, off = cfg["wave"], cfg["offsets"]
    L0 = off[1] - off[0]
    eager = [_gpu(torch, melt, plan, wave[off[k]:off[k + 1]], np.array([0, L0])) for k in range(2)]
    st = melt.MeltStream(plan, 2, 160)
    got = [[], []]
    x = torch.from_numpy(np.stack([wave[off[k]:off[k + 1]] for k in range(2)])).cuda()
    for c0 in range(0, L0, 160):
        out, cnt = st.push(x[:, c0:c0 + 160].contiguous())
        torch.cuda.synchronize()
        o, n = out.cpu().numpy(), cnt.cpu().numpy()
        for k in range(2):
            got[k].append(o[k, :n[k]])
    for k in range(2):
        assert np.array_equal(np.concatenate(got[k]), eager[k])


def test_mfcct_backward(torch, melt, orc):
    """dL = dC D, then the log-power gradient; against the oracle gradient of the same chain."""
    cfg = workloads.config1(seed=6)
    wave, off = cfg["wave"], cfg["offsets"]
    N, H, M, K = 400, 160, 80, 40
    plan = melt.MeltPlan(sample_rate=16000, n_fft=N, hop=H, n_mels=M, output=melt.MELT_OUT_MFCC, n_mfcc=K)
    T = melt.total_frames(off, N, H)
    basis = plan.basis().astype(np.float64)
    Wr, Wi = basis[:M], basis[M:]
    rng = np.random.default_rng(2)
    gC = rng.standard_normal((T, K)).astype(np.float32)
    gL = gC.astype(np.float64) @ orc.dct2_ortho(K, M)
    gx_ref, dWr, dWi = orc.melt_backward(wave, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, grad_out=gL, out_kind=orc.OUT_LOG_POWER,
                                         eps=1e-10)
    d_wave = torch.from_numpy(wave).cuda()
    d_off = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    gw, gb = plan.backward(d_wave, d_off, T, torch.from_numpy(gC).cuda())
    torch.cuda.synchronize()
    rel = lambda a, b: float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))
    ex, eb = rel(gw.cpu().numpy(), gx_ref), rel(gb.cpu().numpy(), np.concatenate([dWr, dWi]))
    print(f"MFCCT backward: rel L2 d/dwave {ex:.2e}, d/dbasis {eb:.2e}")
    # the log power's 1/(S + eps) amplifies forward rounding on quiet bins (no 60 dB
    # restriction here: every bin feeds every coefficient), hence 1e-3
    assert ex < 1e-3 and eb < 1e-3
