"""The allocation-free forward (melt_forward_noalloc) against melt_forward.

Both run the same schedule kernel and the same MelT kernel variant over the same batch, the
one with its chunk table in the plan's workspace and the other in the library's fixed
per-device scratch, so their outputs must be bit-identical.  Two calls in a row on one plan,
the second with a smaller batch, check that the scratch keeps nothing of the first call that
the second reads.  Sizes beyond the scratch and MFCC plans are rejected on the host, before
anything is enqueued.
"""
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


def _both(torch, melt, plan, wave, off):
    T = melt.total_frames(off, plan.n_fft, plan.hop)
    d_wave = torch.from_numpy(np.ascontiguousarray(wave)).cuda()
    d_off = torch.from_numpy(np.asarray(off, np.int64)).cuda()
    ref = torch.full((T, plan.n_mels), float("nan"), dtype=torch.float32, device="cuda")
    got = torch.full((T, plan.n_mels), float("nan"), dtype=torch.float32, device="cuda")
    melt.melt_forward(plan.handle, d_wave, d_off, T, ref)
    melt.melt_forward_noalloc(plan.handle, d_wave, d_off, T, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("prec,geom", [("fp32", (16000, 400, 160, 80)), ("bf16", (16000, 400, 160, 80)),
                                       ("fp16", (16000, 512, 128, 128)), ("fp8", (16000, 400, 160, 80)),
                                       ("fp8b", (16000, 400, 160, 80)),
                                       ("bf16x3", (16000, 400, 160, 80)), ("fp16x3", (16000, 400, 160, 80)),
                                       ("bf16", (22050, 1024, 256, 128))])
def test_noalloc_equals_forward(torch, melt, prec, geom):
    sr, N, H, M = geom
    plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, precision=prec)
    print(f"\nno-alloc forward: {prec} sr {sr} N {N} H {H} M {M}", flush=True)
    # first call: a ragged batch (a clip shorter than one frame, one a frame long, uneven
    # lengths past several chunks); second call: fewer, shorter clips
    for lengths in ([int(4.3 * sr), N - 1, N, int(0.71 * sr), int(2.05 * sr), 3 * H + N + 7],
                    [int(0.5 * sr) + 3, N + 2 * H]):
        wave, off = workloads.random_clips(lengths, seed=len(lengths))
        ref, got = _both(torch, melt, plan, wave, off)
        assert ref.shape[0] == melt.total_frames(off, N, H) > 0
        assert not np.isnan(ref).any()
        np.testing.assert_array_equal(got, ref)
    plan.close()


def test_noalloc_limits(torch, melt):
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    d_wave = torch.zeros(16000, dtype=torch.float32, device="cuda")
    d_off = torch.tensor([0, 16000], dtype=torch.int64, device="cuda")
    out = torch.zeros((98, 80), dtype=torch.float32, device="cuda")
    # a batch that would need more chunk entries than the scratch holds: refused on the host
    with pytest.raises(melt.MeltError) as e:
        melt.melt_forward_noalloc(plan.handle, d_wave, d_off, 128 * 32760, out)
    assert e.value.status == melt.MELT_E_SHAPE
    # empty batches enqueue nothing
    melt.melt_forward_noalloc(plan.handle, d_wave, d_off[:1], 0, out)
    plan.close()
    mf = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, output=melt.MELT_OUT_MFCC, n_mfcc=13)
    out13 = torch.zeros((98, 13), dtype=torch.float32, device="cuda")
    with pytest.raises(melt.MeltError) as e:
        melt.melt_forward_noalloc(mf.handle, d_wave, d_off, 98, out13)
    assert e.value.status == melt.MELT_E_UNSUPPORTED
    mf.close()
