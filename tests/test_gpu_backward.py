"""GPU parity of melt_backward (d/dwaveform by owner-computes overlap-add, d/dbasis by split-K
G^T X) against the FP64 oracle gradient, element by element.

The oracle's gradient is split into the chain rule through the output map
(oracle.melt_chain, from given projections) and the transposed projection
(oracle.melt_backward_linear); both are pinned on the CPU (central differences, adjoint
identities).  The reference takes the projections of the operands the GPU multiplied: the
exact FP64 projections after an FP32 forward, the oracle's BF16 operand model after a BF16
forward.  Every element of d/dwaveform and d/dbasis must then lie within a bound derived
from the arithmetic (tests/parity.py):
  - projections: |R_gpu - R| <= (gamma_N + u) sum|x W| (FP32; the extra u is the FP32
    rounding of the FP64 basis) or gamma_N sum|x_q W_q| (BF16 operands, FP32 accumulation);
  - G = 2 (R, I) g map'(S): parity.grad_proj_error propagates that through S and map';
  - dx = overlap-add of G W over 2M J + J FP32 terms, with the FP32 basis: per sample
    (1 + u) sum|dG||W| + u sum|G||W| + gamma_{2MJ+J} (1 + u) sum (|G| + |dG|)|W|;
  - dW = G^T X over T frames, split over frames and summed in a fixed order (at most
    T + 64 roundings deep): sum|dG||X| + gamma_{T+64} sum (|G| + |dG|)|X|.
The upstream gradient is standard normal on every bin whose energy the forward resolves to
better than a factor 2 (parity.grad_proj_error's `checkable`) and zero elsewhere: below
that, the forward value is rounding noise, and so is any gradient through it."""
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


def _reference_projections(orc, wave, off, N, H, Wr, Wi, prec):
    """(R, I, eR, eI): the projections of the operands the GPU multiplies and the bound on
    the GPU's FP32 accumulation of them."""
    aw = np.abs(wave)
    if prec == "fp32":
        _, R, I = orc.melt_forward_basis(wave, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, out_kind=orc.OUT_POWER,
                                         return_ri=True)
        _, Ar, Ai = orc.melt_forward_basis(aw, off, n_fft=N, hop=H, Wr=np.abs(Wr), Wi=np.abs(Wi),
                                           out_kind=orc.OUT_POWER, return_ri=True)
        gf = parity.gamma(N) + parity.U32
    else:
        code = {"bf16": orc.PREC_BF16, "fp16": orc.PREC_FP16}[prec]
        _, R, I = orc.melt_forward_quant(wave, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, prec=code, out_kind=orc.OUT_POWER,
                                         return_ri=True)
        _, Ar, Ai = orc.melt_forward_quant(aw, off, n_fft=N, hop=H, Wr=np.abs(Wr), Wi=np.abs(Wi), prec=code,
                                           out_kind=orc.OUT_POWER, return_ri=True)
        gf = parity.gamma(N)
    return R, I, gf * Ar, gf * Ai


def _upstream(R, I, eR, eI, kind, eps, seed, sharp=False):
    """Standard-normal upstream gradient on the checkable bins (optionally only on bins
    resolved to 1e-3 of their energy), zero elsewhere; and the G error bounds."""
    g = np.random.default_rng(seed).standard_normal(R.shape)
    _, _, ok = parity.grad_proj_error(R, I, eR, eI, g, kind, eps)
    if sharp:
        S = R * R + I * I
        ok &= 2 * (np.abs(R) * eR + np.abs(I) * eI) < 1e-3 * S
    g = np.where(ok, g, 0.0).astype(np.float32)
    dGr, dGi, _ = parity.grad_proj_error(R, I, eR, eI, g.astype(np.float64), kind, eps)
    dGr = np.where(g != 0, dGr, 0.0)
    dGi = np.where(g != 0, dGi, 0.0)
    return g, dGr, dGi, float(ok.mean()) if ok.size else 0.0


def _gpu_backward(torch, melt, plan, wave, off, T, g, M):
    d_wave = torch.from_numpy(wave).cuda()
    d_off = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    d_g = torch.from_numpy(g).cuda()
    proj = torch.empty((T, 2 * M), dtype=torch.float32, device="cuda")
    plan.forward(d_wave, d_off, T, proj=proj)
    gw, gb = plan.backward(d_wave, d_off, T, d_g, proj=proj)
    gw2, gb2 = plan.backward(d_wave, d_off, T, d_g, proj=None)      # projections recomputed
    torch.cuda.synchronize()
    return gw.cpu().numpy(), gb.cpu().numpy(), gw2.cpu().numpy(), gb2.cpu().numpy()


def _case(torch, melt, orc, wave, off, sr, N, H, M, prec="fp32", kind=0, eps=1e-10, seed=1, label=""):
    """Whole-batch element-wise check of d/dwave and d/dbasis, for two upstream gradients:
    on every checkable bin (complete; the bounds are as loose as the least resolved of those
    bins makes them), then only on bins whose energy the forward resolves to 1e-3 (sharp:
    bounds of ~1e-3 relative).  Returns the GPU results of the first."""
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, precision=prec, output=kind, log_eps=eps)
    T = melt.total_frames(off, N, H)
    _, Wr, Wi = parity.oracle_basis(orc, plan.cfg)
    R, I, eR, eI = _reference_projections(orc, wave, off, N, H, Wr, Wi, prec)
    J = -(-N // H)
    gk, gt, u = parity.gamma(2 * M * J + J), parity.gamma(T + 64), parity.U32
    aw, aWr, aWi = np.abs(wave), np.abs(Wr), np.abs(Wi)
    first = None
    for sharp in (False, True):
        g, dGr, dGi, frac = _upstream(R, I, eR, eI, kind, eps, seed + 100 * sharp, sharp)
        Gr, Gi = orc.melt_chain(R, I, g.astype(np.float64), out_kind=kind, eps=eps)
        gx_ref, dWr_ref, dWi_ref = orc.melt_backward_linear(wave, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, Gr=Gr, Gi=Gi)
        # d/dwave bound: one transposed projection of the combined per-element G weights
        cx_r = (1 + u) * (1 + gk) * dGr + (u + gk * (1 + u)) * np.abs(Gr)
        cx_i = (1 + u) * (1 + gk) * dGi + (u + gk * (1 + u)) * np.abs(Gi)
        bx, _, _ = orc.melt_backward_linear(aw, off, n_fft=N, hop=H, Wr=aWr, Wi=aWi, Gr=cx_r, Gi=cx_i)
        # d/dbasis bound
        _, bWr, bWi = orc.melt_backward_linear(aw, off, n_fft=N, hop=H, Wr=aWr, Wi=aWi,
                                               Gr=(1 + gt) * dGr + gt * np.abs(Gr), Gi=(1 + gt) * dGi + gt * np.abs(Gi),
                                               want_wave=False)
        gw, gb, gw2, gb2 = _gpu_backward(torch, melt, plan, wave, off, T, g, M)
        tag = f"{label} ({'well-resolved bins' if sharp else 'all checkable bins'})"
        sx = parity.check_within(gw, gx_ref, bx, f"{tag} d/dwave")
        sb = parity.check_within(gb, np.concatenate([dWr_ref, dWi_ref]), np.concatenate([bWr, bWi]), f"{tag} d/dbasis")
        print(f"{tag}: upstream on {frac:.3f} of the bins; d/dwave {sx}; d/dbasis {sb}")
        # recomputing the projections gives the same result bit for bit
        assert np.array_equal(gw, gw2) and np.array_equal(gb, gb2)
        if first is None:
            first = (gw, gb, gx_ref)
    return first


def test_config1_fp32(torch, melt, orc):
    cfg = workloads.config1()
    _case(torch, melt, orc, cfg["wave"], cfg["offsets"], 16000.0, 400, 160, 80, label="config1 fp32")


def test_ragged_and_short_clips(torch, melt, orc):
    lengths = [0, 399, 400, 1234, 5, 3000, 561, 20641]
    wave, off = workloads.random_clips(lengths, seed=3)
    gw, _, gx_ref = _case(torch, melt, orc, wave, off, 16000.0, 400, 160, 80, seed=2, label="ragged fp32")
    # samples that no frame covers (short clips, clip tails) have exactly zero gradient
    assert np.all(gw[gx_ref == 0.0] == 0.0)
    # clips of 399 and 5 samples have no frame at all
    assert np.all(gw[off[1]:off[2]] == 0.0) and np.all(gw[off[4]:off[5]] == 0.0)
    assert off[2] - off[1] == 399 and off[5] - off[4] == 5


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_other_output_kinds(torch, melt, orc, kind):
    cfg = workloads.config1(seed=8)
    _case(torch, melt, orc, cfg["wave"], cfg["offsets"], 16000.0, 400, 160, 80, kind=kind, seed=3,
          label=f"output kind {kind}")


def test_config5_geometry(torch, melt, orc):
    """22.05 kHz, N=1024, H=256, 128 Mel bins (the differentiation workload's frontend) on
    2 clips x 1 s."""
    cfg = workloads.config5(n_clips=2, seconds=1.0)
    _case(torch, melt, orc, cfg["wave"], cfg["offsets"], 22050.0, 1024, 256, 128, seed=4, label="config5-geometry fp32")


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_reduced_precision_forward(torch, melt, orc, prec):
    """The backward after a BF16 / FP16 forward: the saved projections are those of the
    rounded operands, so the reference is the oracle's operand model of that format."""
    cfg = workloads.config5(n_clips=2, seconds=1.0)
    _case(torch, melt, orc, cfg["wave"], cfg["offsets"], 22050.0, 1024, 256, 128, prec=prec, seed=5,
          label=f"config5-geometry {prec} forward")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_config5_full_size_sampled(torch, melt, orc, prec):
    """The differentiation workload at full size (32 x 10 s at 22.05 kHz, N 1024, H 256, 128 Mel
    bins, 27 456 frames) in the launch configuration the benchmark times: every element of
    d/dbasis (a sum over all frames), and d/dwave on 24 sampled segments of 1500 samples
    (clip starts, clip ends and interiors), each against the oracle evaluated on just the
    frames that overlap it.  Upstream on the well-resolved bins (sharp bounds)."""
    cfg = workloads.config5()
    wave, off = cfg["wave"], cfg["offsets"]
    sr, N, H, M = 22050.0, 1024, 256, 128
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, precision=prec)
    T = melt.total_frames(off, N, H)
    assert T == 27456
    _, Wr, Wi = parity.oracle_basis(orc, plan.cfg)
    R, I, eR, eI = _reference_projections(orc, wave, off, N, H, Wr, Wi, prec)
    g, dGr, dGi, frac = _upstream(R, I, eR, eI, 0, 1e-10, seed=6, sharp=True)
    Gr, Gi = orc.melt_chain(R, I, g.astype(np.float64))
    gw, gb, _, _ = _gpu_backward(torch, melt, plan, wave, off, T, g, M)
    J = -(-N // H)
    gk, gt, u = parity.gamma(2 * M * J + J), parity.gamma(T + 64), parity.U32
    # d/dbasis, every element
    _, dWr, dWi = orc.melt_backward_linear(wave, off, n_fft=N, hop=H, Wr=Wr, Wi=Wi, Gr=Gr, Gi=Gi, want_wave=False)
    _, bWr, bWi = orc.melt_backward_linear(np.abs(wave), off, n_fft=N, hop=H, Wr=np.abs(Wr), Wi=np.abs(Wi),
                                           Gr=(1 + gt) * dGr + gt * np.abs(Gr), Gi=(1 + gt) * dGi + gt * np.abs(Gi),
                                           want_wave=False)
    sb = parity.check_within(gb, np.concatenate([dWr, dWi]), np.concatenate([bWr, bWi]), f"config5 {prec} d/dbasis")
    # d/dwave on sampled segments: the frames t0..t1 of clip c that overlap [s0, s1) as one clip
    T_c = np.array([orc.num_frames(int(b - a), N, H) for a, b in zip(off[:-1], off[1:])])
    fo = np.concatenate([[0], np.cumsum(T_c)])
    rng = np.random.default_rng(61)
    L_seg = 1500
    for k in range(24):
        c = int(rng.integers(0, len(T_c)))
        clip_len = int(off[c + 1] - off[c])
        s0 = [0, clip_len - L_seg][k % 2] if k < 8 else int(rng.integers(0, clip_len - L_seg))
        s1 = s0 + L_seg
        t0 = max(0, -(-(s0 - N + 1) // H))
        t1 = min(int(T_c[c]) - 1, (s1 - 1) // H)
        sub = wave[off[c] + t0 * H: off[c] + t1 * H + N]
        so = np.array([0, sub.size], np.int64)
        rows = slice(fo[c] + t0, fo[c] + t1 + 1)
        gx, _, _ = orc.melt_backward_linear(sub, so, n_fft=N, hop=H, Wr=Wr, Wi=Wi, Gr=Gr[rows], Gi=Gi[rows])
        cx_r = (1 + u) * (1 + gk) * dGr[rows] + (u + gk * (1 + u)) * np.abs(Gr[rows])
        cx_i = (1 + u) * (1 + gk) * dGi[rows] + (u + gk * (1 + u)) * np.abs(Gi[rows])
        bx, _, _ = orc.melt_backward_linear(np.abs(sub), so, n_fft=N, hop=H, Wr=np.abs(Wr), Wi=np.abs(Wi), Gr=cx_r,
                                            Gi=cx_i)
        a = s0 - t0 * H          # the segment within the sub-clip
        hi = min(s1, (int(T_c[c]) - 1) * H + N)      # samples past the last frame get zero
        sx = parity.check_within(gw[off[c] + s0: off[c] + hi], gx[a: a + hi - s0], bx[a: a + hi - s0],
                                 f"config5 {prec} d/dwave clip {c} [{s0}, {s1})")
        assert np.all(gw[off[c] + hi: off[c] + s1] == 0.0)
    print(f"config5 full {prec}: upstream on {frac:.3f} of the bins; d/dbasis {sb}; last d/dwave segment {sx}")


def test_deterministic(torch, melt):
    cfg = workloads.config2(n_clips=3, seconds=2.0)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    T = melt.total_frames(cfg["offsets"], 400, 160)
    d_wave = torch.from_numpy(cfg["wave"]).cuda()
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    g = torch.randn((T, 80), device="cuda")
    a = plan.backward(d_wave, d_off, T, g)
    b = plan.backward(d_wave, d_off, T, g)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_autograd_function(torch, melt, orc):
    """torch.autograd through melt_apply: gradients w.r.t. the waveform and a learnable basis
    equal the direct backward call."""
    cfg = workloads.config1(seed=9)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    wave = torch.from_numpy(cfg["wave"]).cuda().requires_grad_(True)
    basis = torch.from_numpy(plan.basis()).cuda().requires_grad_(True)
    out = melt.melt_apply(wave, plan, d_off, 98, basis_param=basis)
    w = torch.randn_like(out)
    (out * w).sum().backward()
    gw, gb = plan.backward(wave.detach(), d_off, 98, w)
    torch.cuda.synchronize()
    assert torch.allclose(wave.grad, gw) and torch.allclose(basis.grad, gb)
    # a changed basis changes the forward: set_basis re-packs the plan's layouts
    basis2 = (basis.detach() * 2.0).contiguous()
    out2 = melt.melt_apply(wave.detach(), plan, d_off, 98, basis_param=basis2)
    assert torch.allclose(out2, out.detach() + 2 * np.log(2.0), atol=1e-3)


def test_empty_batch_and_graph_replay(torch, melt):
    """An empty batch writes d/dbasis = 0 with a fill kernel (no memset node, so the call can
    be captured).  The backward captured in a HIP graph and replayed gives the eager result
    bit for bit on every replay, with eager work and synchronisations between the replays."""
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    gb0 = torch.full((160, 400), float("nan"), dtype=torch.float32, device="cuda")
    none_off = torch.zeros(1, dtype=torch.int64, device="cuda")
    melt.melt_backward(plan.handle, torch.zeros(8, device="cuda"), none_off, 0,
                       torch.zeros((1, 80), device="cuda"), None, None, gb0)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(gb0)) == 0
    cfg = workloads.config1(seed=17)
    d_wave = torch.from_numpy(cfg["wave"]).cuda()
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    out = torch.empty((98, 80), device="cuda")
    proj = torch.empty((98, 160), device="cuda")
    plan.forward(d_wave, d_off, 98, out=out, proj=proj)
    gout = torch.randn((98, 80), device="cuda")
    gw = torch.empty_like(d_wave)
    gb = torch.empty((160, 400), device="cuda")
    melt.melt_backward(plan.handle, d_wave, d_off, 98, gout, proj, gw, gb)   # sizes the workspaces
    torch.cuda.synchronize()
    ref_w, ref_b = gw.clone(), gb.clone()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            melt.melt_backward(plan.handle, d_wave, d_off, 98, gout, proj, gw, gb)
    torch.cuda.synchronize()
    for k in range(4):
        gw.fill_(float("nan"))
        gb.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(gw, ref_w) and torch.equal(gb, ref_b), f"replay {k}"
        _ = (gout * 2.0).sum().item()      # eager work between replays
