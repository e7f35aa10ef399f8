"""Streaming MelT (melt_stream_*), its hipGraph capture, and the autotuner.

Frames of a stream are computed by the same kernel and the same k-ordered MFMA sequence as
the batch forward, so streaming output must equal melt_forward over the concatenated
stream bit for bit; a captured push replayed with new chunk contents must equal eager
pushes bit for bit."""
import json
import os

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


def _streams(n_streams, n_samples, seed=0):
    rng = np.random.default_rng(seed)
    return (0.3 * rng.standard_normal((n_streams, n_samples))).astype(np.float32)


def _batch_reference(torch, melt, plan, X):
    n_streams, L = X.shape
    off = np.arange(n_streams + 1, dtype=np.int64) * L
    T = melt.total_frames(off, plan.n_fft, plan.hop)
    out = plan.forward(torch.from_numpy(X.reshape(-1)).cuda(), torch.from_numpy(off).cuda(), T)
    torch.cuda.synchronize()
    per = T // n_streams
    return out.cpu().numpy().reshape(n_streams, per, plan.n_mels)


def _run_eager(torch, melt, plan, X, lengths, n_max):
    st = melt.MeltStream(plan, X.shape[0], n_max)
    got = [[] for _ in range(X.shape[0])]
    pos = 0
    for cl in lengths:
        chunk = torch.from_numpy(np.ascontiguousarray(X[:, pos:pos + cl])).cuda()
        out, cnt = st.push(chunk)
        torch.cuda.synchronize()
        o, c = out.cpu().numpy(), cnt.cpu().numpy()
        for s in range(X.shape[0]):
            got[s].append(o[s, :c[s]])
        pos += cl
    return [np.concatenate(g) for g in got], st


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_stream_equals_batch_16k(torch, melt, prec):
    """8 streams, 2 s each, pushed in 10 ms chunks (160 samples at 16 kHz)."""
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision=prec)
    X = _streams(8, 32000, seed=1)
    ref = _batch_reference(torch, melt, plan, X)
    got, _ = _run_eager(torch, melt, plan, X, [160] * 200, 160)
    for s in range(8):
        assert got[s].shape == ref[s].shape
        assert np.array_equal(got[s], ref[s])


def test_stream_systems_configuration(torch, melt):
    """The streaming systems row at its size: 512 streams at 16 kHz, 10 ms chunks (160 samples),
    N 512, H 128, 128 Mel bins; 40 pushes equal the batch forward of the same streams bit for
    bit."""
    plan = melt.MeltPlan(sample_rate=16000.0, n_fft=512, hop=128, n_mels=128, fmin=0.0, fmax=8000.0)
    X = _streams(512, 160 * 40, seed=5)
    ref = _batch_reference(torch, melt, plan, X)
    got, _ = _run_eager(torch, melt, plan, X, [160] * 40, 160)
    for s in range(512):
        assert got[s].shape == ref[s].shape
        assert np.array_equal(got[s], ref[s])


def test_stream_22k_alternating_chunks(torch, melt):
    """22.05 kHz, N=1024, H=256: 10 ms is 220.5 samples, so chunks alternate 220 and 221."""
    plan = melt.MeltPlan(sample_rate=22050, n_fft=1024, hop=256, n_mels=128)
    n_chunks = 100
    lengths = [220 + (i % 2) for i in range(n_chunks)]
    X = _streams(4, sum(lengths), seed=2)
    ref = _batch_reference(torch, melt, plan, X)
    got, _ = _run_eager(torch, melt, plan, X, lengths, 221)
    for s in range(4):
        assert np.array_equal(got[s], ref[s])


def test_stream_long_chunks_and_reset(torch, melt):
    """Chunks longer than one chunk of the kernel (several hundred frames per push)."""
    plan = melt.MeltPlan(sample_rate=16000, n_fft=512, hop=128, n_mels=128)
    X = _streams(3, 3 * 40000, seed=3)
    ref = _batch_reference(torch, melt, plan, X)
    got, st = _run_eager(torch, melt, plan, X, [40000, 40000, 40000], 40000)
    for s in range(3):
        assert np.array_equal(got[s], ref[s])
    st.reset()
    got2 = [[] for _ in range(3)]
    out, cnt = st.push(torch.from_numpy(np.ascontiguousarray(X[:, :40000])).cuda())
    torch.cuda.synchronize()
    for s in range(3):
        assert np.array_equal(out.cpu().numpy()[s, :cnt[s].item()], ref[s][:cnt[s].item()])


def test_stream_graph_replay(torch, melt):
    """One push captured in a graph, replayed over 60 chunks with eager work and
    synchronisation between replays; every replay equals the eager push."""
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80)
    n_streams, cl = 16, 160
    X = _streams(n_streams, 60 * cl, seed=4)
    eager, _ = _run_eager(torch, melt, plan, X, [cl] * 60, cl)
    st = melt.MeltStream(plan, n_streams, cl)
    static_in = torch.zeros((n_streams, cl), dtype=torch.float32, device="cuda")
    st.push(static_in)                           # warm-up outside capture (no allocation inside)
    torch.cuda.synchronize()
    st.reset()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            st.push(static_in)
    torch.cuda.synchronize()
    st.reset()
    torch.cuda.synchronize()
    got = [[] for _ in range(n_streams)]
    for i in range(60):
        static_in.copy_(torch.from_numpy(np.ascontiguousarray(X[:, i * cl:(i + 1) * cl])).cuda())
        g.replay()
        junk = torch.randn(1000, device="cuda").sum()    # unrelated eager work between replays
        torch.cuda.synchronize()
        o, c = st.out.cpu().numpy(), st.count.cpu().numpy()
        for k in range(n_streams):
            got[k].append(o[k, :c[k]])
        del junk
    for k in range(n_streams):
        assert np.array_equal(np.concatenate(got[k]), eager[k])


def test_autotune_and_cache(torch, melt, tmp_path, monkeypatch):
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MELT_AUTOTUNE_CACHE", str(cache))
    cfg = workloads.config2(n_clips=4, seconds=3.0)
    plan = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision="bf16")
    T = melt.total_frames(cfg["offsets"], 400, 160)
    d_wave = torch.from_numpy(cfg["wave"]).cuda()
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    before = plan.forward(d_wave, d_off, T).cpu().numpy()
    desc = melt.melt_autotune(plan.handle, 20000)
    print("autotune:", desc)
    assert "us" in desc
    after = plan.forward(d_wave, d_off, T).cpu().numpy()
    # both kernel variants compute the same products; results agree to FP32 accumulation
    assert np.allclose(after, before, atol=1e-3)
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    assert len(lines) == 1 and "n_fft=400" in lines[0]["key"]
    plan2 = melt.MeltPlan(sample_rate=16000, n_fft=400, hop=160, n_mels=80, precision="bf16")   # applies the cache
    again = plan2.forward(d_wave, d_off, T).cpu().numpy()
    assert np.array_equal(again, after)
