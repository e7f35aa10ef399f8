"""The learnable basis (melt_plan_set_basis): re-packing for every precision, graph capture,
and autograd through several forwards that use different bases."""
import numpy as np
import pytest

import workloads

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


def _proj(torch, plan, d_wave, d_off, T):
    out = torch.empty((T, plan.n_mels), dtype=torch.float32, device="cuda")
    P = torch.empty((T, 2 * plan.n_mels), dtype=torch.float32, device="cuda")
    plan.forward(d_wave, d_off, T, out=out, proj=P)
    return out, P


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16x3", "fp16x3", "fp8", "fp8b"])
def test_set_basis_repacks_the_plan_precision(torch, melt, prec):
    """A basis scaled by 2 is exact in FP32, BF16, split BF16 and scaled FP8 (whose row
    scales halve exactly), so after set_basis the projections are exactly twice the original
    ones (FP16 rounds its subnormal entries, the window's edges, differently after scaling,
    so there it is only close); and setting the original basis back restores the original
    output bit for bit."""
    cfg = workloads.config1(seed=12)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
    d_wave = torch.from_numpy(cfg["wave"]).cuda()
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    out0, P0 = _proj(torch, plan, d_wave, d_off, 98)
    b = torch.from_numpy(plan.basis()).cuda()
    plan.set_basis(2.0 * b)
    _, P1 = _proj(torch, plan, d_wave, d_off, 98)
    plan.set_basis(b)
    out2, P2 = _proj(torch, plan, d_wave, d_off, 98)
    torch.cuda.synchronize()
    if prec in ("fp16", "fp16x3"):
        assert torch.allclose(P1, 2.0 * P0, rtol=1e-3, atol=1e-4 * float(P0.abs().max()))
    else:
        assert torch.equal(P1, 2.0 * P0)
    assert torch.equal(P2, P0) and torch.equal(out2, out0)


def test_set_basis_in_a_captured_graph(torch, melt):
    """set_basis + forward captured in one HIP graph and replayed with new basis contents:
    every replay equals the eager calls on the same basis, with eager work and
    synchronisations between the replays."""
    cfg = workloads.config1(seed=13)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision="bf16")
    d_wave = torch.from_numpy(cfg["wave"]).cuda()
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    b0 = torch.from_numpy(plan.basis()).cuda()
    src = b0.clone()
    out = torch.empty((98, 80), dtype=torch.float32, device="cuda")
    plan.forward(d_wave, d_off, 98, out=out)          # first call outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.set_basis(src)
            plan.forward(d_wave, d_off, 98, out=out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for k in range(4):
        scale = torch.from_numpy(rng.uniform(0.5, 2.0, (160, 1)).astype(np.float32)).cuda()
        src.copy_(b0 * scale)
        g.replay()
        torch.cuda.synchronize()
        got = out.clone()
        ref = torch.empty_like(out)
        plan.set_basis(b0 * scale)
        plan.forward(d_wave, d_off, 98, out=ref)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), k
        _ = (ref * 2).sum().item()                     # unrelated eager work between replays


def test_interleaved_forwards_keep_their_basis(torch, melt):
    """Two differentiable forwards with different bases before one backward: each term's
    gradient is taken through the basis its forward used (the plan re-sets it), equal to
    the direct backward calls with that basis; a forward without basis_param after the
    basis was replaced cannot be differentiated and says so."""
    cfg = workloads.config1(seed=14)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    w0 = torch.from_numpy(cfg["wave"]).cuda()
    b1 = torch.from_numpy(plan.basis()).cuda()
    b2 = (b1 * torch.linspace(0.5, 1.5, 400, device="cuda")).contiguous()
    x1 = w0.clone().requires_grad_(True)
    x2 = w0.clone().requires_grad_(True)
    p1 = b1.clone().requires_grad_(True)
    p2 = b2.clone().requires_grad_(True)
    out1 = melt.melt_apply(x1, plan, d_off, 98, basis_param=p1)
    out2 = melt.melt_apply(x2, plan, d_off, 98, basis_param=p2)
    u1, u2 = torch.randn_like(out1), torch.randn_like(out2)
    ((out1 * u1).sum() + (out2 * u2).sum()).backward()
    plan.set_basis(b1)
    gx1, gb1 = plan.backward(w0, d_off, 98, u1)
    plan.set_basis(b2)
    gx2, gb2 = plan.backward(w0, d_off, 98, u2)
    torch.cuda.synchronize()
    assert torch.equal(x1.grad, gx1) and torch.equal(p1.grad, gb1)
    assert torch.equal(x2.grad, gx2) and torch.equal(p2.grad, gb2)
    assert not torch.allclose(gx1, gx2)
    # the plan's basis changes after a forward that took none: its backward must refuse
    x3 = w0.clone().requires_grad_(True)
    out3 = melt.melt_apply(x3, plan, d_off, 98)
    plan.set_basis(b1)
    with pytest.raises(RuntimeError, match="basis was replaced"):
        out3.sum().backward()
