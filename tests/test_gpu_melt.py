"""GPU parity of the MelT forward (melt_forward / melt_forward_proj) against the FP64 oracle.

FP32: against the plain FP64 oracle (direct NDFT summation).  BF16 / FP16 / split-BF16x3 /
split-FP16x3 / FP8 (per-frame and 32-sample block scales): against the oracle's operand model
of the same precision (operands rounded exactly as the
format defines, products and sums exact), so the only difference left is FP32
accumulation.  The pass condition is the per-bin bound of tests/parity.py; the dB error
against the plain FP64 oracle is reported for every precision.
"""
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


def _gpu_forward(torch, melt, plan, wave, off, proj=False):
    T = melt.total_frames(off, plan.n_fft, plan.hop)
    d_wave = torch.from_numpy(np.ascontiguousarray(wave)).cuda()
    d_off = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    out = torch.full((T, plan.n_mels), float("nan"), dtype=torch.float32, device="cuda")
    P = torch.full((T, 2 * plan.n_mels), float("nan"), dtype=torch.float32, device="cuda") if proj else None
    plan.forward(d_wave, d_off, T, out=out, proj=P)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (P.cpu().numpy() if proj else None)


def _oracle_fp32(orc, plan, wave, off, eps):
    # centres and basis from the oracle's own Mel scale and placement, not from the plan
    _, Wr, Wi = parity.oracle_basis(orc, plan.cfg)
    _, R, I = orc.melt_forward_basis(wave, off, n_fft=plan.n_fft, hop=plan.hop, Wr=Wr, Wi=Wi, eps=eps,
                                     return_ri=True)
    _, Ar, Ai = orc.melt_forward_basis(np.abs(wave), off, n_fft=plan.n_fft, hop=plan.hop, Wr=np.abs(Wr),
                                       Wi=np.abs(Wi), eps=eps, return_ri=True)
    return R, I, Ar, Ai, Wr, Wi


def _check(orc, melt, plan, L, wave, off, prec, eps=1e-10, label=""):
    R, I, Ar, Ai, Wr, Wi = _oracle_fp32(orc, plan, wave, off, eps)
    N = plan.n_fft
    if prec == "fp32":
        st = parity.check_log_power(L, R, I, Ar, Ai, N, eps, extra_rel=1.0, label=label)
    else:
        code = {"bf16": orc.PREC_BF16, "fp16": orc.PREC_FP16, "bf16x3": orc.PREC_BF16X3,
                "fp16x3": orc.PREC_FP16X3, "fp8": orc.PREC_FP8_E4M3, "fp8b": orc.PREC_FP8_E4M3_BLOCK32}[prec]
        _, Rq, Iq = orc.melt_forward_quant(wave, off, n_fft=N, hop=plan.hop, Wr=Wr, Wi=Wi, prec=code, eps=eps,
                                           return_ri=True)
        if prec in ("bf16x3", "fp16x3"):
            Aq_r, Aq_i, nt = Ar * 1.01, Ai * 1.01, 3 * N
        else:
            _, Aq_r, Aq_i = orc.melt_forward_quant(np.abs(wave), off, n_fft=N, hop=plan.hop, Wr=np.abs(Wr),
                                                   Wi=np.abs(Wi), prec=code, eps=eps, return_ri=True)
            nt = N
        # FP8: the FP32 epilogue multiplies by 1/s_t and 1/r_j (three more roundings); block-scaled
        # FP8 by 1/r_j
        parity.check_log_power(L, Rq, Iq, Aq_r, Aq_i, nt, eps, extra_rel=4.0 if prec in ("fp8", "fp8b") else 0.0,
                               label=label)
        st = parity.db_stats(L, np.log(R * R + I * I + eps), R * R + I * I)
    print(f"{label}: dB error vs FP64 oracle on active bins: max {st['max_db']:.3g} rms {st['rms_db']:.3g}")
    return st


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3", "fp16x3", "fp8", "fp8b"])
def test_config1_tiny(torch, melt, orc, prec):
    """One 1 s clip at 16 kHz, N=400, H=160, 80 HTK bins, 0-8 kHz: 98 frames."""
    cfg = workloads.config1()
    plan = melt.MeltPlan(sample_rate=cfg["sr"], n_fft=400, hop=160, n_mels=80, fmin=0, fmax=8000, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
    assert L.shape == (98, 80)
    st = _check(orc, melt, plan, L, cfg["wave"], cfg["offsets"], prec, label=f"config1 {prec}")
    if prec in ("fp32", "fp16x3"):
        # the FP32 bar; split binary16 keeps about 22 significant bits per product term
        assert st["max_db"] < 0.02 and st["rms_db"] < 2e-3
    if prec == "bf16x3":
        # reported, not a pass condition: the split product keeps ~16 significant bits per
        # term, so quiet bins carry about 2^8 times the FP32 error
        assert st["max_db"] < 0.5


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3", "fp16x3", "fp8", "fp8b"])
@pytest.mark.parametrize("n_mels", [80, 128])
def test_config2_reduced(torch, melt, orc, prec, n_mels):
    """Config-2 signals at reduced size (4 clips x 2.5 s = 4 x 248 frames: two full 128-frame
    chunks and a ragged tail per clip)."""
    cfg = workloads.config2(n_mels=n_mels, n_clips=4, seconds=2.5)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=n_mels, fmin=0, fmax=8000, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
    _check(orc, melt, plan, L, cfg["wave"], cfg["offsets"], prec, label=f"config2-reduced M={n_mels} {prec}")


@pytest.mark.parametrize("n_clips", [1, 63, 64, 65, 300])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_schedule_clip_counts(torch, melt, orc, prec, n_clips):
    """Chunk schedules of up to 64 clips (one wave's lanes, no barrier) and of more (the
    block-scan kernel): ragged clips with empty ones, clips shorter than a frame and clips of
    several chunks, against the oracle frame by frame (the output starts as NaN, so a frame
    no chunk covers fails)."""
    rng = np.random.default_rng(80 + n_clips)
    lengths = rng.integers(0, 400 + 300 * 160, n_clips)
    lengths[5::7] = 0
    lengths[3::11] = 399
    wave, off = workloads.random_clips(lengths, seed=81 + n_clips)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, wave, off)
    assert L.shape[0] == sum(melt.melt_num_frames(int(n), 400, 160) for n in lengths)
    _check(orc, melt, plan, L, wave, off, prec, label=f"{n_clips} clips {prec}")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp8", "fp8b"])
def test_ragged_edge_cases(torch, melt, orc, prec):
    """Empty clips, clips shorter than a frame, exactly one frame, one sample more, and
    lengths that end chunks at every residue."""
    lengths = [0, 399, 400, 401, 559, 560, 0, 3, 20479, 20480, 20641, 7777, 400]
    wave, off = workloads.random_clips(lengths, seed=5)
    off = off + 0   # offsets start at 0 here; a non-zero base is covered below
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, wave, off)
    assert L.shape[0] == sum(melt.melt_num_frames(n, 400, 160) for n in lengths)
    _check(orc, melt, plan, L, wave, off, prec, label=f"ragged {prec}")
    # a batch that starts part-way into the buffer: only clips 2.. of the same buffer
    L2, _ = _gpu_forward(torch, melt, plan, wave, off[2:])
    assert np.array_equal(L2, L[-L2.shape[0]:])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_many_clips_schedule(torch, melt, orc, prec):
    """2600 clips of 0 to N + 12 H samples (empty, sub-frame and short clips): the chunk
    schedule's prefix sums carry across blocks of 1024 clips."""
    lengths = np.random.default_rng(31).integers(0, 400 + 12 * 160, 2600)
    wave, off = workloads.random_clips(lengths, seed=32)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, wave, off)
    assert L.shape[0] == sum(melt.melt_num_frames(int(n), 400, 160) for n in lengths)
    _check(orc, melt, plan, L, wave, off, prec, label=f"2600 clips {prec}")


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16x3", "fp16x3", "fp8", "fp8b"])
def test_chunk_ring_refill(torch, melt, orc, prec):
    """20 000 clips of one to four frames, one chunk each: a persistent workgroup of the
    direct-to-LDS and producer/consumer kernels walks 39 or more chunks, so it reads chunk
    descriptors through at least one refill of its 32-entry LDS ring.  The default variant
    is checked against the oracle; every other variant with the ring must give the same
    bits (they share the per-frame arithmetic)."""
    rng = np.random.default_rng(41)
    nfr = rng.integers(1, 5, 20000)
    lengths = 400 + (nfr - 1) * 160 + rng.integers(0, 160, 20000)
    wave, off = workloads.random_clips(lengths, seed=42)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
    L0, _ = _gpu_forward(torch, melt, plan, wave, off)
    assert L0.shape[0] == int(nfr.sum())
    _check(orc, melt, plan, L0, wave, off, prec, label=f"20000 clips {prec}")
    for v in range(1, melt.melt_variant_count(plan.handle)):
        name = melt.melt_variant_name(plan.handle, v)
        if "lds-dma" not in name and "producer-consumer" not in name:
            continue
        melt.melt_set_variant(plan.handle, v, 0)
        L, _ = _gpu_forward(torch, melt, plan, wave, off)
        assert np.array_equal(L, L0), f"{prec} {name} differs from the default variant"


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_chunk_ring_refill_ksplit(torch, melt, orc, prec):
    """The same for the K-split kernel (22.05 kHz, N 1024, H 256, 128 Mel bins: two row
    groups of four tiles): 20 000 one- to four-frame clips, over 100 chunks per workgroup."""
    rng = np.random.default_rng(43)
    nfr = rng.integers(1, 5, 20000)
    lengths = 1024 + (nfr - 1) * 256 + rng.integers(0, 256, 20000)
    wave, off = workloads.random_clips(lengths, seed=44)
    plan = melt.MeltPlan(sample_rate=22050, n_fft=1024, hop=256, n_mels=128, precision=prec)
    assert "k-split" in melt.melt_variant_name(plan.handle, 0)
    L, _ = _gpu_forward(torch, melt, plan, wave, off)
    assert L.shape[0] == int(nfr.sum())
    _check(orc, melt, plan, L, wave, off, prec, label=f"20000 clips K-split {prec}")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3", "fp16x3", "fp8", "fp8b"])
def test_every_kernel_variant(torch, melt, orc, prec):
    """Every kernel variant of the precision (staging scheme x frames per chunk), pinned with
    melt_set_variant, on clips that end chunks of 64, 96 and 128 frames exactly, one frame
    past them and mid-way.  Geometries: the 16 kHz front end (hop a multiple of 4: vector
    span conversion), hop 50 (two-byte aligned rows: element-wise conversion) and N=480,
    hop 161 (32 k-groups, odd hop); 16, 24 and 96 Mel bins (1, 2 and 6 row tiles: the
    16-bit kernel's waves that share a row tile by frame tiles); 144 and 256 Mel bins (row
    groups of 5 + 4 and 8 + 8 tiles in the 16-bit kernel)."""
    geoms = [(16000, 400, 160, 80), (16000, 400, 50, 40), (16000, 480, 161, 64),
             (16000, 400, 160, 16), (16000, 400, 160, 24), (16000, 512, 128, 96),
             (16000, 400, 160, 144), (16000, 400, 160, 256)]
    if prec == "fp8":
        geoms = geoms[:1]
    elif prec == "fp8b":
        # hops that are whole 32-sample blocks; 9 and 16 row tiles are row groups of 5 + 4 and
        # 8 + 8; N 1024 (16 k-groups of 64) and N 256 (4)
        geoms = [g for g in geoms if g[2] % 32 == 0] + [(22050, 1024, 256, 128), (16000, 256, 128, 80)]
    elif prec == "fp32":
        geoms = geoms[:3]
    elif prec in ("bf16", "fp16"):
        # N 1024: 64 k-groups, the K-split kernel (two waves per row tile); 128 and 80 Mel bins
        # (row groups of 4 + 4 and 3 + 2 tiles).  N 1200 at hop 160 (the cepstral front end):
        # 75 k-groups, split unevenly into 40 + 35 at the fifth hop segment
        geoms = geoms + [(22050, 1024, 256, 128), (16000, 1024, 256, 80), (16000, 1200, 160, 128),
                         # 16 and 20 k-groups with 80, 128 and 64 Mel bins: the row-pair kernel (two
                         # basis tiles per wave; 5, 8 and 4 row tiles)
                         (16000, 256, 128, 80), (16000, 320, 160, 128), (16000, 256, 128, 64)]
    for sr, N, H, M in geoms:
        lengths = [0, N - 1, N, N + 1] + [(f - 1) * H + N + d for f in (64, 65, 96, 97, 128, 129, 200) for d in (0, 3)]
        wave, off = workloads.random_clips(lengths, seed=N + H)
        plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, precision=prec)
        n = melt.melt_variant_count(plan.handle)
        assert n >= 1
        for v in range(n):
            melt.melt_set_variant(plan.handle, v, 0)
            name = melt.melt_variant_name(plan.handle, v)
            L, _ = _gpu_forward(torch, melt, plan, wave, off)
            _check(orc, melt, plan, L, wave, off, prec, label=f"N={N} H={H} {prec} {name}")
        with pytest.raises(melt.MeltError):
            melt.melt_set_variant(plan.handle, n, 0)


@pytest.mark.parametrize("geom", [(16000, 256, 128, 80), (16000, 400, 160, 144), (16000, 512, 128, 96),
                                  (16000, 400, 160, 256)])
def test_fp8_producer_consumer(torch, melt, orc, geom):
    """The per-frame FP8 producer/consumer kernel pinned by name: 4, 7 and 8 k-groups of 64
    (n_fft 256, 400, 512), one row group and row groups of 5 + 4 and 8 + 8 tiles, on ragged
    clips that end its 64-frame chunks exactly, one frame past them and mid-way (the span and
    image buffers alternate per chunk)."""
    sr, N, H, M = geom
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, precision="fp8")
    names = [melt.melt_variant_name(plan.handle, v) for v in range(melt.melt_variant_count(plan.handle))]
    pc = [v for v, n in enumerate(names) if "producer-consumer" in n]
    assert len(pc) == 1
    melt.melt_set_variant(plan.handle, pc[0], 0)
    lengths = [0, N - 1, N] + [(f - 1) * H + N + d for f in (63, 64, 65, 128, 129, 200, 257) for d in (0, 3)]
    wave, off = workloads.random_clips(lengths, seed=N + M + 7)
    L, _ = _gpu_forward(torch, melt, plan, wave, off)
    _check(orc, melt, plan, L, wave, off, "fp8", label=f"fp8 producer/consumer {geom}")


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("geom", [(22050, 1024, 256, 128), (16000, 1200, 160, 128), (16000, 1024, 256, 40)])
def test_split_precisions_long_frames(torch, melt, orc, prec, geom):
    """The split precisions at frame lengths whose hi and lo basis tiles do not fit in a
    wave's registers (N 1024: 64 k-groups, N 1200 at hop 160: 75): the frame-split kernel
    with the basis streamed from L2, on ragged clips that end 128-frame chunks exactly, one
    frame past them and mid-way; one to eight row tiles."""
    sr, N, H, M = geom
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, precision=prec)
    assert "frame-split" in melt.melt_variant_name(plan.handle, 0)
    lengths = [N - 1, N, (127 * H + N), (128 * H + N), (200 * H + N + 5), 3 * N + 17]
    wave, off = workloads.random_clips(lengths, seed=N + M)
    L, _ = _gpu_forward(torch, melt, plan, wave, off)
    _check(orc, melt, plan, L, wave, off, prec, label=f"long frames {geom} {prec}")


@pytest.mark.parametrize("geom", [(16000, 512, 128, 128), (22050, 1024, 256, 128), (16000, 400, 100, 40),
                                  (8000, 256, 80, 24)])
def test_other_geometries(torch, melt, orc, geom):
    sr, N, H, M = geom
    lengths = [N - 1, N, 5 * N + 7, 31 * H + N, 2 * 128 * H + N + 3]
    wave, off = workloads.random_clips(lengths, seed=9)
    # FP8 too: every geometry here has an FP8 register tile (N 256, 400, 512, 1024), and 128
    # Mel bins put a row tile on every wave of the FP8 kernel; block-scaled FP8 where the hop
    # is whole 32-sample blocks
    for prec in ("fp32", "bf16", "fp8") + (("fp8b",) if H % 32 == 0 else ()):
        plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, precision=prec)
        L, _ = _gpu_forward(torch, melt, plan, wave, off)
        _check(orc, melt, plan, L, wave, off, prec, label=f"geometry {geom} {prec}")


def test_config3_precision_sweep(torch, melt, orc):
    """Precision sweep on config-3 signals (amplitudes log-uniform over 60 dB), reduced to
    4 clips x 2 s: every precision against its operand model (pass condition) and the dB
    error against the FP64 oracle per 10 dB band below each frame's peak (reported)."""
    cfg = workloads.config3(n_clips=4, seconds=2.0)
    for prec in ("fp32", "fp16x3", "bf16x3", "fp16", "bf16", "fp8", "fp8b"):
        plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
        L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
        st = _check(orc, melt, plan, L, cfg["wave"], cfg["offsets"], prec, label=f"config3 {prec}")
        if prec in ("fp32", "fp16x3"):
            assert st["max_db"] < 0.02 and st["rms_db"] < 2e-3, (prec, st)
        R, I, _, _, _, _ = _oracle_fp32(orc, plan, cfg["wave"], cfg["offsets"], 1e-10)
        S = R * R + I * I
        e = np.abs(parity.DB_PER_NAT * (L - np.log(S + 1e-10)))
        below = 10 * np.log10(S.max(axis=1, keepdims=True) / np.maximum(S, 1e-300))
        bands = []
        for lo in range(0, 80, 10):
            sel = (below >= lo) & (below < lo + 10)
            if np.any(sel):
                bands.append(f"{lo}-{lo + 10}dB: max {e[sel].max():.3g} rms {np.sqrt(np.mean(e[sel] ** 2)):.3g}")
        print(f"config3 {prec} per band below frame peak: " + "; ".join(bands))


def test_silence_is_log_eps(torch, melt):
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    wave = np.zeros(16000, np.float32)
    L, P = _gpu_forward(torch, melt, plan, wave, np.array([0, 16000]), proj=True)
    # every bin is the device's logf((float)eps), bit for bit, within 2 ulp of ln(1e-10)
    assert np.all(L == L[0, 0])
    assert abs(float(L[0, 0]) - np.log(1e-10)) <= 2 * np.spacing(np.float32(23.0))
    assert np.all(P == 0.0)


def test_projection_output(torch, melt, orc):
    """melt_forward_proj writes (R, I) per Mel bin, interleaved."""
    cfg = workloads.config1(seed=4)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    L, P = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"], proj=True)
    R, I, Ar, Ai, _, _ = _oracle_fp32(orc, plan, cfg["wave"], cfg["offsets"], 1e-10)
    tol = (400 + 1) * parity.U32 * 1.01
    assert np.all(np.abs(P[:, 0::2] - R) <= tol * Ar + 1e-30)
    assert np.all(np.abs(P[:, 1::2] - I) <= tol * Ai + 1e-30)
    L2, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
    assert np.array_equal(L, L2)


def test_output_kinds(torch, melt, orc):
    cfg = workloads.config1(seed=6)
    P_plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, output=melt.MELT_OUT_POWER)
    S, _ = _gpu_forward(torch, melt, P_plan, cfg["wave"], cfg["offsets"])
    R, I, Ar, Ai, _, _ = _oracle_fp32(orc, P_plan, cfg["wave"], cfg["offsets"], 1e-10)
    S_ref = R * R + I * I
    g = 402 * parity.U32
    dS = 2 * np.abs(R) * g * Ar + 2 * np.abs(I) * g * Ai + (g * Ar) ** 2 + (g * Ai) ** 2 + 3 * parity.U32 * S_ref
    assert np.all(np.abs(S - S_ref) <= dS * 1.01 + 1e-30)
    for kind, fn in ((melt.MELT_OUT_MAGNITUDE, np.sqrt), (melt.MELT_OUT_LOG_MAGNITUDE, lambda s: np.log(np.sqrt(s) + 1e-10))):
        plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, output=kind)
        out, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
        loud = S_ref > 1e-4 * S_ref.max()      # within 40 dB of the peak
        if kind == melt.MELT_OUT_MAGNITUDE:
            assert np.allclose(out[loud], fn(S_ref[loud]), rtol=1e-4, atol=0)
        else:                                     # log domain: absolute error in nats
            assert np.allclose(out[loud], fn(S_ref[loud]), rtol=0, atol=1e-4)
        if kind == melt.MELT_OUT_MAGNITUDE:       # everywhere: out^2 obeys the power bound
            assert np.all(np.abs(out.astype(np.float64) ** 2 - S_ref) <= dS * 1.02 + 8 * parity.U32 * S_ref + 1e-30)


def test_empty_calls(torch, melt):
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    d_off = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_wave = torch.zeros(10, dtype=torch.float32, device="cuda")
    out = torch.zeros((0, 80), dtype=torch.float32, device="cuda")
    plan.forward(d_wave, d_off, 0, out=out)            # n_clips = 0
    d_off2 = torch.tensor([0, 10], dtype=torch.int64, device="cuda")
    plan.forward(d_wave, d_off2, 0, out=out)           # one clip shorter than a frame
    torch.cuda.synchronize()
    with pytest.raises(melt.MeltError):
        melt.melt_forward(plan.handle, None, d_off2, 5, out)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3", "fp16x3", "fp8", "fp8b"])
def test_config2_full_size_sampled(torch, melt, orc, prec):
    """The benchmark's workload and launch: 64 clips x 30 s (191 872 frames, M=80), at every
    precision the benchmark times (each plan's default kernel, as the benchmark runs it).
    256 frames sampled across the batch (first/last of every clip included) are checked
    against the oracle evaluated on exactly those frames (with the rest of the last 32-sample
    block for block-scaled FP8)."""
    cfg = workloads.config2(n_mels=80)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
    assert L.shape == (191872, 80)
    assert np.all(np.isfinite(L))
    rng = np.random.default_rng(77)
    ids = np.unique(np.concatenate([rng.integers(0, L.shape[0], 128), np.arange(0, 191872, 2998),
                                    np.arange(2997, 191872, 2998)]))
    tail = (-400) % 32 if prec == "fp8b" else 0
    sub, off = parity.frames_as_clips(cfg["wave"], cfg["offsets"], 400, 160, ids, tail=tail)
    _check(orc, melt, plan, L[ids], sub, off, prec, label=f"config2 full sampled {prec}")


_CONFIG4 = {}


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3", "fp16x3", "fp8", "fp8b"])
@pytest.mark.parametrize("variant", ["16k", "22k"])
def test_config4_full_size_sampled(torch, melt, orc, variant, prec):
    """The ragged systems batch at full size, as the systems benchmark launches it: 512 clips of
    U[0.5, 30] s (16 kHz, N 512, H 128, or 22.05 kHz, N 1024, H 256; 128 Mel bins up to the
    Nyquist frequency).  The first and last frame of every clip and 128 random frames are
    checked against the oracle evaluated on exactly those frames."""
    if variant not in _CONFIG4:
        _CONFIG4.clear()                                  # one batch in host memory at a time
        _CONFIG4[variant] = workloads.config4(variant)
    cfg = _CONFIG4[variant]
    N, H, sr = cfg["n_fft"], cfg["hop"], cfg["sr"]
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=128, fmin=0.0, fmax=sr / 2, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
    off = np.asarray(cfg["offsets"], np.int64)
    lens = off[1:] - off[:-1]
    T_c = np.where(lens >= N, 1 + (lens - N) // H, 0)
    fo = np.concatenate([[0], np.cumsum(T_c)])
    assert L.shape == (fo[-1], 128)
    assert np.all(np.isfinite(L))
    has = T_c > 0
    rng = np.random.default_rng(4040)
    ids = np.unique(np.concatenate([fo[:-1][has], fo[1:][has] - 1, rng.integers(0, fo[-1], 128)]))
    sub, soff = parity.frames_as_clips(cfg["wave"], off, N, H, ids)
    _check(orc, melt, plan, L[ids], sub, soff, prec, label=f"config4 {variant} full sampled {prec}")


# ------------------------------------------------------------------ centres, basis and options
# Eq. mel_scale, Eq. inverse_mel and the filter-centre placement are checked against the
# oracle's own computation, never against values read back from the plan.

@pytest.mark.parametrize("formula", ["htk", "slaney"])
@pytest.mark.parametrize("placement", ["centres", "linspace"])
def test_plan_centres_and_basis_match_oracle(torch, melt, orc, formula, placement):
    """The plan's analysis frequencies equal the oracle's (its own Mel scale, inverse and
    placement) to 1e-13 relative, and the plan's FP32 basis is the oracle's FP64 basis of
    Eq. dmp_weights rounded once: |b - ref| <= 2^-24 |ref| + 2e-12, the second term covering
    the oracle's FP64 cos/sin of the unreduced argument (at most ~1.3e3 rad here, a few ulp
    of it).  Over the paper's two bands, 40 to 512 Mel bins and the three windows."""
    fcode = {"htk": melt.MELT_MEL_HTK, "slaney": melt.MELT_MEL_SLANEY}[formula]
    pcode = {"centres": melt.MELT_PLACE_FILTER_CENTRES, "linspace": melt.MELT_PLACE_LINSPACE}[placement]
    cases = [(fmin, fmax, M, melt.MELT_WIN_HANN_SYMMETRIC) for fmin, fmax in ((0.0, 8000.0), (80.0, 7600.0))
             for M in (40, 80, 128, 512)]
    cases += [(0.0, 8000.0, 80, melt.MELT_WIN_HANN_PERIODIC), (80.0, 7600.0, 80, melt.MELT_WIN_RECT)]
    for fmin, fmax, M, win in cases:
        plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=M, fmin=fmin, fmax=fmax,
                             mel_formula=fcode, placement=pcode, window=win)
        f_ref, Wr, Wi = parity.oracle_basis(orc, plan.cfg)
        f = plan.frequencies()
        assert np.allclose(f, f_ref, rtol=1e-13, atol=1e-9), (formula, placement, fmin, fmax, M)
        assert np.all(np.diff(f) > 0)
        ref = np.vstack([Wr, Wi])
        B = plan.basis().astype(np.float64)
        err = np.abs(B - ref) - (2.0 ** -24 * np.abs(ref) + 2e-12)
        assert np.all(err <= 0), (formula, placement, fmin, fmax, M, win, float(err.max()))
        plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "fp8b"])
def test_window_formula_placement_forward(torch, melt, orc, prec):
    """The periodic and rectangular windows, the Slaney scale and the M-point placement
    through the forward kernels on a 1 s clip, against the oracle's own basis."""
    cfg = workloads.config1(seed=8)
    opts = [dict(window=melt.MELT_WIN_HANN_PERIODIC), dict(window=melt.MELT_WIN_RECT),
            dict(mel_formula=melt.MELT_MEL_SLANEY), dict(placement=melt.MELT_PLACE_LINSPACE, fmin=80.0, fmax=7600.0)]
    for o in opts:
        kw = dict(sample_rate=16000, n_fft=400, hop=160, n_mels=80, fmin=0.0, fmax=8000.0, precision=prec)
        kw.update(o)
        plan = melt.MeltPlan(**kw)
        L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
        _check(orc, melt, plan, L, cfg["wave"], cfg["offsets"], prec, label=f"options {o} {prec}")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3", "fp8", "fp8b"])
def test_spectral_band_80_7600(torch, melt, orc, prec):
    """The paper's spectral front end (16 kHz, N 400, H 160, 80 Mel bins over 80-7600 Hz;
    Table "Audio frontend configuration") on config-2 signals, 4 clips x 2.5 s."""
    cfg = workloads.config2(n_mels=80, n_clips=4, seconds=2.5)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, fmin=80.0, fmax=7600.0, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
    _check(orc, melt, plan, L, cfg["wave"], cfg["offsets"], prec, label=f"80-7600 Hz {prec}")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3", "fp8", "fp8b"])
def test_512_mel_bins(torch, melt, orc, prec):
    """The top of the Mel-bin sweep (M = 512, the paper's break-even point; Fig. m_sweep) over
    80-7600 Hz: 32 row tiles, so four 16-bit (and FP8) row groups and, for FP32, several
    row-tile blocks per chunk.  2 clips x 2 s (two full chunks and a ragged tail each)."""
    cfg = workloads.config2(n_mels=512, n_clips=2, seconds=2.0)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=512, fmin=80.0, fmax=7600.0, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, cfg["wave"], cfg["offsets"])
    _check(orc, melt, plan, L, cfg["wave"], cfg["offsets"], prec, label=f"M=512 {prec}")


def test_512_mel_bins_fp8_all_wave_unsupported(torch, melt):
    """The all-wave per-frame FP8 kernels hold at most 8 row tiles (128 Mel bins): pinned at
    512 Mel bins they report the error and run nothing (the producer/consumer kernel, the
    default, takes row groups)."""
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=512, precision="fp8")
    wave = torch.zeros(16000, dtype=torch.float32, device="cuda")
    off = torch.tensor([0, 16000], dtype=torch.int64, device="cuda")
    names = [melt.melt_variant_name(plan.handle, v) for v in range(melt.melt_variant_count(plan.handle))]
    assert "producer-consumer" in names[0]
    others = [v for v, n in enumerate(names) if "producer-consumer" not in n]
    assert others
    for v in others:
        melt.melt_set_variant(plan.handle, v)
        with pytest.raises(melt.MeltError) as ei:
            plan.forward(wave, off, 98)
        assert ei.value.status == melt.MELT_E_UNSUPPORTED


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "fp8b"])
def test_hop_equals_n_fft(torch, melt, orc, prec):
    """Adjacent frames with no overlap (hop = n_fft = 256): one hop segment per frame."""
    lengths = [0, 255, 256, 257, 511, 512, 256 * 130 + 7, 256 * 300]
    wave, off = workloads.random_clips(lengths, seed=256)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=256, hop=256, n_mels=40, precision=prec)
    L, _ = _gpu_forward(torch, melt, plan, wave, off)
    assert L.shape[0] == sum(melt.melt_num_frames(n, 256, 256) for n in lengths)
    _check(orc, melt, plan, L, wave, off, prec, label=f"hop = n_fft {prec}")


def test_block_scaled_fp8_extreme_blocks(torch, melt, orc):
    """Block-scaled FP8 over the whole exponent range: a clip at 1e-37 (blocks whose exponent is
    the largest allowed, 127: the kernel's plain-conversion path), one at 3e3 (negative
    exponents), one of normal level with silent stretches (exponent 0), checked through the
    raw projections, clip by clip, against the operand model within the FP32 accumulation bound
    (the projections of the quiet clip are far below the log floor)."""
    rng = np.random.default_rng(61)
    lens = [4000, 4000, 4000]
    x = rng.standard_normal(sum(lens)).astype(np.float32)
    # the quiet clip stays in FP32's normal range (|x| >= 3e-38)
    x[:4000] = np.where(np.abs(x[:4000]) < 0.3, np.copysign(0.3, x[:4000]), x[:4000]) * np.float32(1e-37)
    x[4000:8000] *= np.float32(3e3)
    x[8000 + 1000:8000 + 2000] = 0.0
    off = np.array([0, 4000, 8000, 12000], np.int64)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision="fp8b")
    _, P = _gpu_forward(torch, melt, plan, x, off, proj=True)
    _, Wr, Wi = parity.oracle_basis(orc, plan.cfg)
    _, Rq, Iq = orc.melt_forward_quant(x, off, n_fft=400, hop=160, Wr=Wr, Wi=Wi, prec=orc.PREC_FP8_E4M3_BLOCK32,
                                       return_ri=True)
    _, Ar, Ai = orc.melt_forward_quant(np.abs(x), off, n_fft=400, hop=160, Wr=np.abs(Wr), Wi=np.abs(Wi),
                                       prec=orc.PREC_FP8_E4M3_BLOCK32, return_ri=True)
    g = 405 * parity.U32
    assert np.all(np.abs(P[:, 0::2] - Rq) <= g * Ar + 1e-45)
    assert np.all(np.abs(P[:, 1::2] - Iq) <= g * Ai + 1e-45)
    assert np.abs(Rq[:20]).max() > 0 and np.abs(P[:20, 0::2]).max() < 1e-30


def test_block_scaled_fp8_needs_whole_block_hops(torch, melt):
    """Block-scaled FP8 needs a hop of whole 32-sample blocks (reported at plan creation); the
    frame length needs an FP8 register tile (reported at the call)."""
    with pytest.raises(melt.MeltError) as ei:
        melt.MeltPlan(sample_rate=16000, n_fft=400, hop=100, n_mels=80, precision="fp8b")
    assert ei.value.status == melt.MELT_E_UNSUPPORTED
    plan = melt.MeltPlan(sample_rate=16000, n_fft=1200, hop=160, n_mels=80, precision="fp8b")
    wave = torch.zeros(16000, dtype=torch.float32, device="cuda")
    off = torch.tensor([0, 16000], dtype=torch.int64, device="cuda")
    with pytest.raises(melt.MeltError) as ei:
        plan.forward(wave, off, melt.melt_num_frames(16000, 1200, 160))
    assert ei.value.status == melt.MELT_E_UNSUPPORTED


def test_frame_offsets(torch, melt, orc):
    """melt_frame_offsets: the device prefix sums of the per-clip frame counts, against the
    oracle's frame count per clip, over 2600 ragged clips (prefix sums carried across blocks
    of 1024 clips), a batch starting part-way into the buffer, and an empty batch."""
    lengths = np.random.default_rng(51).integers(0, 400 + 30 * 160, 2600)
    _, off = workloads.random_clips(lengths, seed=52)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    for o in (off, off[5:] + 0, off[:1]):
        d_off = torch.from_numpy(np.ascontiguousarray(o, np.int64)).cuda()
        d_fo = torch.full((len(o),), -7, dtype=torch.int64, device="cuda")
        melt.melt_frame_offsets(plan.handle, d_off, d_fo)
        torch.cuda.synchronize()
        T_c = [orc.num_frames(int(b - a), 400, 160) for a, b in zip(o[:-1], o[1:])]
        ref = np.concatenate([[0], np.cumsum(T_c, dtype=np.int64)])
        assert np.array_equal(d_fo.cpu().numpy(), ref)
