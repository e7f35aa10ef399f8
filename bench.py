#!/usr/bin/env python
"""Mel frames/s of the MelT GEMM path vs the FFT + filterbank path on one MI355X.

Workload: 64 clips x 30 s at 16 kHz (float32 pink noise + amplitude-modulated tones), N=400,
H=160, 80 HTK Mel bins over 0-8 kHz: T = 191 872 frames, GEMM 191 872 x 400 x 160.  Inputs
are resident in HBM before the timed region.  One step = one MelT forward over the batch
(chunk schedule + the persistent MFMA kernel); the comparator (hand-written FFT + sparse
filterbank) and the other precisions are timed the same way on the same batch and reported
beside it, each with its log-Mel error against the FP64 oracle on sampled frames.

Prints one JSON line.  `roofline` is for the dominant kernel (the MelT FP32 projection),
timed alone with HIP events over the same number of launches; `cpu_baseline` times the FP64
oracle on the host over the whole batch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3e12, "bf16": 2.5e15, "f16": 2.5e15, "fp8": 5.0e15, "hbm": 8.0e12}
# the sources of the dominant kernel (the FP32 MelT projection): a change to either makes the
# committed traffic counters stale
KERNEL_SRCS = [os.path.join(ROOT, "paper_2606_01009_amd", "csrc", f) for f in ("melt_f32.hip", "fwd_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "melt_f32_ws_config2_m80_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_id():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


_RAMP = {}


def device_ramp(torch, ms=300.0):
    """Keeps the GPU busy for about `ms` with an unrelated FP32 matrix product before a timed
    block, so that its clocks are in the state FP32 matrix work holds them in (measured: the
    first timed block of a process otherwise runs ~7 % slower, and a BF16 product does not
    bring the clocks there).  Not a step of any timed path."""
    if "a" not in _RAMP:
        _RAMP["a"] = torch.randn(4096, 4096, device="cuda", dtype=torch.float32)
        _RAMP["b"] = torch.randn(4096, 4096, device="cuda", dtype=torch.float32)
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(10):
            torch.mm(_RAMP["a"], _RAMP["b"])
        torch.cuda.synchronize()


def time_launches(torch, fn, steps, warmup, ramp=True):
    if ramp:
        device_ramp(torch)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps          # ms per launch


def bootstrap_ci(values, level=0.90, resamples=2000, seed=0):
    """Percentile bootstrap interval of the median of `values` (resampled with replacement)."""
    v = np.asarray(values, np.float64)
    rng = np.random.default_rng(seed)
    meds = np.median(v[rng.integers(0, v.size, size=(resamples, v.size))], axis=1)
    a = (1.0 - level) / 2.0
    return [float(np.quantile(meds, a)), float(np.quantile(meds, 1.0 - a))]


def trial_stats(torch, fn, calls, trials=20):
    """The timing protocol of the paper's experiments on this GPU: `trials` trials of `calls`
    back-to-back calls after a warm-up, each trial timed with HIP events around its calls (an
    event pair around every call would add its own gaps to sub-100 us kernels, so a trial
    gives the mean of its calls).  Median over the trials and its bootstrap 90 % interval,
    in ms per call."""
    device_ramp(torch)
    for _ in range(max(5, calls // 4)):
        fn()
    per = [time_launches(torch, fn, calls, 1 if t == 0 else 0, ramp=False) for t in range(trials)]
    return {"median_ms": float(np.median(per)), "ci90_ms": bootstrap_ci(per), "min_ms": float(np.min(per)),
            "max_ms": float(np.max(per)), "trials": trials, "calls_per_trial": calls}


class EnergyMeter:
    """Board energy from the amdsmi energy accumulator of the GPU torch uses (matched by PCI
    address).  On MI355X the accumulator (15.3 uJ per count) is republished about once per
    second with the time it was sampled, so a window runs over whole republication intervals:
    the first and last snapshots that fall inside a stretch of uninterrupted work (or of
    idling) bound it, and power = energy delta / sampled-time delta."""

    def __init__(self, torch):
        import amdsmi
        self.smi = amdsmi
        amdsmi.amdsmi_init()
        props = torch.cuda.get_device_properties(torch.cuda.current_device())
        want = (getattr(props, "pci_domain_id", 0), getattr(props, "pci_bus_id", -1), getattr(props, "pci_device_id", 0))
        self.handle = None
        for h in amdsmi.amdsmi_get_processor_handles():
            bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)          # "dddd:bb:dd.f"
            dom, bus, rest = bdf.split(":")
            if (int(dom, 16), int(bus, 16), int(rest.split(".")[0], 16)) == want:
                self.handle = h
        if self.handle is None:
            raise RuntimeError(f"no amdsmi GPU at PCI {want}")
        self.res_uj = amdsmi.amdsmi_get_energy_count(self.handle)["counter_resolution"]

    def _read(self):
        e = self.smi.amdsmi_get_energy_count(self.handle)
        return time.perf_counter(), e["energy_accumulator"], e["timestamp"]

    def _window(self, step, intervals, lead_s):
        """Calls step() until `intervals` republications have been seen after lead_s seconds;
        returns (joules, seconds, counter quanta) between the first and last of them."""
        t_start = time.perf_counter()
        last = self._read()
        snaps = []
        while len(snaps) < intervals + 1:
            step()
            r = self._read()
            if (r[1], r[2]) != (last[1], last[2]):
                if r[0] - t_start >= lead_s:
                    snaps.append(r)
                last = r
            if time.perf_counter() - t_start > lead_s + 3.0 * (intervals + 2):
                raise RuntimeError("energy counter not republished")
        (h0, a0, s0), (h1, a1, s1) = snaps[0], snaps[-1]
        dt_host = h1 - h0
        dt = (s1 - s0) * 1e-9
        if not (0.8 * dt_host < dt < 1.2 * dt_host):     # a sample time out of sequence: use the host's
            dt = dt_host
        return (a1 - a0) * self.res_uj * 1e-6, dt, int(a1 - a0)

    def idle_watts(self, torch, intervals=2):
        torch.cuda.synchronize()
        j, dt, q = self._window(lambda: time.sleep(0.0005), intervals, 0.2)
        return j / dt, dt, q

    def busy_watts(self, torch, fn, call_ms, intervals=3, lead_s=0.5):
        """Keeps the GPU busy with back-to-back calls of fn (batches of ~20 ms, at most three
        in flight) and returns the board power over whole republication intervals."""
        k = max(1, int(round(20.0 / max(call_ms, 1e-3))))
        inflight = []

        def step():
            for _ in range(k):
                fn()
            ev = torch.cuda.Event()
            ev.record()
            inflight.append(ev)
            if len(inflight) >= 3:
                inflight.pop(0).synchronize()

        j, dt, q = self._window(step, intervals, lead_s)
        torch.cuda.synchronize()
        return j / dt, dt, q

    def close(self):
        try:
            self.smi.amdsmi_shut_down()
        except Exception:
            pass


def energy_per_call(meter, torch, fn, call_ms, idle_w, frames):
    """Board and active (board minus idle) energy of one call, from the board power while
    the call runs back to back and its time per call (the paper's method: a counter delta
    over a window, less the idle baseline)."""
    w, dt, q = meter.busy_watts(torch, fn, call_ms)
    board_mj = w * call_ms
    active_mj = (w - idle_w) * call_ms
    return {"board_w": w, "idle_w": idle_w, "window_s": dt, "counter_quanta": q,
            "board_mj_per_call": board_mj, "active_mj_per_call": active_mj,
            "active_j_per_mframes": active_mj / frames * 1e3, "board_j_per_mframes": board_mj / frames * 1e3}


def sampled_error_db(out, wave, offsets, kind, freqs, n_fft=400, hop=160, n_mels=80, n_sample=256, seed=5):
    """dB error against the FP64 oracle on sampled frames (max / rms over bins within 80 dB
    of the sample's peak)."""
    import oracle
    from tests.parity import frames_as_clips
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(out.shape[0], n_sample, replace=False))
    sub, off = frames_as_clips(wave, offsets, n_fft, hop, ids)
    if kind == "melt":
        ref = oracle.melt_forward(sub, off, sr=16000.0, n_fft=n_fft, hop=hop, freqs=freqs)
    else:
        ref = oracle.stft_mel_forward(sub, off, sr=16000.0, n_fft=n_fft, hop=hop, n_mels=n_mels, fmin=0.0,
                                      fmax=8000.0)
    S = np.exp(ref)
    act = S >= S.max() * 1e-8
    e = (10.0 / np.log(10.0)) * (out[ids].astype(np.float64) - ref)
    return {"max_db": float(np.abs(e[act]).max()), "rms_db": float(np.sqrt(np.mean(e[act] ** 2))),
            "frames_sampled": int(n_sample)}


def oracle_freqs(n_mels, fmin=0.0, fmax=8000.0):
    """The oracle's own HTK Mel centres (Eq. mel_scale, Eq. inverse_mel) for the error check
    and the CPU baseline: nothing is taken from the plan being measured."""
    import oracle
    return oracle.melt_frequencies(n_mels, fmin, fmax, oracle.MEL_HTK, oracle.PLACE_FILTER_CENTRES)


def cpu_baseline(wave, offsets, freqs, T, min_seconds=10.0):
    """The FP64 oracle (direct NDFT summation, C + OpenMP) over the whole batch, repeated until
    at least min_seconds of wall time have passed."""
    import oracle
    oracle.build()
    passes, t0 = 0, time.perf_counter()
    while True:
        oracle.melt_forward(wave, offsets, sr=16000.0, n_fft=400, hop=160, freqs=freqs)
        passes += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    return {"value": passes * T / dt, "unit": "Mel frames/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"the whole batch (64 clips x 30 s, {T} frames) {passes} times, direct FP64 NDFT summation "
                      f"(C, OpenMP), {dt:.1f} s wall"}


def load_traffic(path, source_id):
    """HBM traffic of the dominant kernel from committed rocprofv3 --pmc summaries, or None if
    absent or taken on another version of the kernel source."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_id") != source_id:
        return None
    return t.get("hbm_bytes_per_launch")


def run_systems(torch, melt, workloads, path):
    """The systems rows on synthetic stand-ins: the ragged batch (512 clips of U[0.5, 30] s;
    16 kHz / N 512 / H 128 and 22.05 kHz / N 1024 / H 256, 128 Mel bins), streaming of 10 ms
    chunks over 512 streams (per push, eager and replayed from a captured graph), and the
    backward of the differentiation workload (32 x 10 s at 22.05 kHz, N 1024, H 256, 128 Mel
    bins): forward with saved projections, then d/dwaveform and d/dbasis."""
    rows = []

    def emit(r):
        rows.append(r)
        log("system " + ", ".join(f"{k} {v:.4g}" if isinstance(v, float) else f"{k} {v}" for k, v in r.items()))

    for variant in ("16k", "22k"):
        cfg = workloads.config4(variant)
        N, H, M, sr = cfg["n_fft"], cfg["hop"], cfg["n_mels"], cfg["sr"]
        T = melt.total_frames(cfg["offsets"], N, H)
        d_wave = torch.from_numpy(cfg["wave"]).cuda()
        d_off = torch.from_numpy(cfg["offsets"]).cuda()
        out = torch.empty((T, M), device="cuda")
        r = {"workload": f"ragged 512 clips U[0.5,30] s, {variant}: sr {sr:g}, N {N}, H {H}, M {M}", "frames": T}
        for prec in ("fp32", "bf16", "bf16x3"):
            plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, fmin=0.0, fmax=sr / 2, precision=prec)
            try:
                ms = time_launches(torch, lambda: plan.forward(d_wave, d_off, T, out=out), 20, 5)
            except melt.MeltError as e:
                r[f"melt_{prec}_error"] = str(e)
                continue
            r[f"melt_{prec}_ms"] = ms
            r[f"melt_{prec}_mframes_s"] = T / (ms * 1e-3) / 1e6
            if prec == "fp32":
                r["melt_fp32_tflops"] = T * 4 * N * M / (ms * 1e-3) / 1e12
        plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, fmin=0.0, fmax=sr / 2)
        ms = time_launches(torch, lambda: plan.stft_mel(d_wave, d_off, T, out=out), 20, 5)
        r["fft_ms"] = ms
        r["fft_mframes_s"] = T / (ms * 1e-3) / 1e6
        emit(r)
        del d_wave, out

    # streaming: 512 streams, 10 ms chunks (160 samples at 16 kHz), N 512, H 128, 128 Mel bins
    plan = melt.MeltPlan(sample_rate=16000.0, n_fft=512, hop=128, n_mels=128, fmin=0.0, fmax=8000.0)
    n_streams, cl, pushes = 512, 160, 200
    st = melt.MeltStream(plan, n_streams, cl)
    x = torch.randn((n_streams, cl), device="cuda") * 0.1
    st.push(x)
    torch.cuda.synchronize()
    eager = time_launches(torch, lambda: st.push(x), pushes, 20)
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            st.push(x)
    torch.cuda.synchronize()
    replay = time_launches(torch, g.replay, pushes, 20)
    emitted = int(st.count.sum().item())
    emit({"workload": "streaming 512 streams x 10 ms chunks (16 kHz, N 512, H 128, M 128)",
          "push_eager_us": eager * 1e3, "push_graph_us": replay * 1e3, "frames_per_push": emitted,
          "frames_per_s_graph": emitted / (replay * 1e-3)})
    st.close()

    # backward of the differentiation workload
    cfg = workloads.config5()
    N, H, M, sr = cfg["n_fft"], cfg["hop"], cfg["n_mels"], cfg["sr"]
    T = melt.total_frames(cfg["offsets"], N, H)
    d_wave = torch.from_numpy(cfg["wave"]).cuda()
    d_off = torch.from_numpy(cfg["offsets"]).cuda()
    gout = torch.from_numpy(workloads.upstream_grad(T, M)).cuda()
    for prec in ("fp32", "bf16"):
        plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, fmin=0.0, fmax=sr / 2, precision=prec)
        out = torch.empty((T, M), device="cuda")
        proj = torch.empty((T, 2 * M), device="cuda")
        fwd = time_launches(torch, lambda: plan.forward(d_wave, d_off, T, out=out, proj=proj), 20, 5)
        gw = torch.empty_like(d_wave)
        gb = torch.empty((2 * M, N), device="cuda")
        bwd = time_launches(torch, lambda: melt.melt_backward(plan.handle, d_wave, d_off, T, gout, proj, gw, gb),
                            20, 5)
        flop = 8.0 * N * M * T          # dX = G W and dW = G^T X, 4 N M each per frame
        emit({"workload": f"backward 32 x 10 s, sr {sr:g}, N {N}, H {H}, M {M}, {prec} forward", "frames": T,
              "forward_ms": fwd, "backward_ms": bwd, "backward_tflops": flop / (bwd * 1e-3) / 1e12,
              "backward_frac_fp32_mfma": flop / (bwd * 1e-3) / PEAK["f32"]})
    with open(path, "w") as fh:
        for r in rows:
            fh.write(json.dumps(r) + "\n")


def _pmc_average(csv_path, name_part, counter):
    """Mean per dispatch of `counter` over the dispatches of kernels whose name contains
    name_part, from a rocprofv3 --pmc counter_collection.csv."""
    import csv
    tot, ids = 0.0, set()
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter:
                tot += float(r["Counter_Value"])
                ids.add(r["Dispatch_Id"])
    if not ids:
        raise SystemExit(f"no {counter} for {name_part} in {csv_path}")
    return tot / len(ids), len(ids)


def write_traffic(pmc_dir, T, bytes_algo, wave_bytes):
    """Writes TRAFFIC_FILE from four rocprofv3 --pmc runs under pmc_dir (fp32_f, fp32_w:
    FETCH_SIZE / WRITE_SIZE of `--only fp32`; copy_f, copy_w: the same of `--only copy`).
    Each counter is scaled by what it reads for the copy kernel, which reads and writes
    wave_bytes once per launch."""
    find = lambda sub: os.path.join(pmc_dir, sub, "run_counter_collection.csv")
    fetch, nf = _pmc_average(find("fp32_f"), "k_melt_f32_ws", "FETCH_SIZE")
    write, nw = _pmc_average(find("fp32_w"), "k_melt_f32_ws", "WRITE_SIZE")
    cf, _ = _pmc_average(find("copy_f"), "vectorized_elementwise_kernel", "FETCH_SIZE")
    cw, _ = _pmc_average(find("copy_w"), "vectorized_elementwise_kernel", "WRITE_SIZE")
    kib = wave_bytes / 1024.0
    fs, ws = kib / cf, kib / cw
    hbm = fetch * 1024 * fs + write * 1024 * ws
    t = {"kernel": "k_melt_f32_ws (MelT FP32, 64 clips x 30 s, n_fft 400, hop 160, 80 Mel bins)",
         "kernel_source_id": kernel_source_id(),
         "fetch_kib_per_dispatch": round(fetch, 1), "write_kib_per_dispatch": round(write, 1),
         "dispatches_averaged": [nf, nw], "fetch_scale": round(fs, 5), "write_scale": round(ws, 5),
         "hbm_bytes_per_launch": int(hbm), "algorithmic_bytes_per_launch": int(bytes_algo), "frames": T,
         "commands": [f"rocprofv3 --pmc {c} -d <dir>/{w}_{x} -o run --output-format csv -- python3 bench.py "
                      f"--only {w} --steps 3 --warmup 1 --no-check"
                      for w in ("fp32", "copy") for c, x in (("FETCH_SIZE", "f"), ("WRITE_SIZE", "w"))]}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    log(f"bench: wrote {TRAFFIC_FILE}: {hbm / 1e6:.1f} MB per launch against {bytes_algo / 1e6:.1f} MB algorithmic")


def call_ms(torch, fn, calls=20, warmup=5, busy_ms=30.0, trials=20):
    """Median over `trials` trials of the mean time of `calls` back-to-back calls (HIP events)
    and its bootstrap 90 % interval, after about busy_ms of back-to-back calls so that the
    clocks have ramped up."""
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < busy_ms:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
    per = [time_launches(torch, fn, calls, warmup if t == 0 else 1, ramp=False) for t in range(trials)]
    return float(np.median(per)), bootstrap_ci(per)


def run_workloads(torch, melt, workloads, path):
    """The paper's efficiency workloads (Experiments) on synthetic stand-ins: per call,
    MelT FP32 / BF16 / BF16x3 against the FFT + filterbank path, each call a whole
    forward (chunk schedule + kernel).  Spectral configuration 16 kHz, N=400, H=160, fmin 80,
    fmax 7600; cepstral configuration N=1200, M=128, K=40, 0-8 kHz (Table "Audio frontend
    configuration")."""
    rows = []

    def measure(tag, wave, offsets, sr, N, H, M, fmin, fmax, output=0, K=40, precs=("fp32", "bf16", "bf16x3")):
        T = melt.total_frames(offsets, N, H)
        d_wave = torch.from_numpy(wave).cuda()
        d_off = torch.from_numpy(offsets).cuda()
        cols = K if output == melt.MELT_OUT_MFCC else M
        out = torch.empty((T, cols), dtype=torch.float32, device="cuda")
        rec = {"workload": tag, "frames": T, "clips": len(offsets) - 1, "n_fft": N, "hop": H, "n_mels": M,
               "output": "mfcc" if output == melt.MELT_OUT_MFCC else "log_power"}
        for prec in precs:
            try:
                plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, fmin=fmin, fmax=fmax, precision=prec,
                                     output=output, n_mfcc=K)
                rec[f"melt_{prec}_ms"], rec[f"melt_{prec}_ci90_ms"] = call_ms(
                    torch, lambda: plan.forward(d_wave, d_off, T, out=out))
            except melt.MeltError as e:
                rec[f"melt_{prec}_error"] = str(e)
        plan = melt.MeltPlan(sample_rate=sr, n_fft=N, hop=H, n_mels=M, fmin=fmin, fmax=fmax, output=output, n_mfcc=K)
        rec["fft_ms"], rec["fft_ci90_ms"] = call_ms(torch, lambda: plan.stft_mel(d_wave, d_off, T, out=out))
        for prec in precs:
            if f"melt_{prec}_ms" in rec:
                rec[f"speedup_{prec}_vs_fft"] = rec["fft_ms"] / rec[f"melt_{prec}_ms"]
        log(f"workload {tag}: " + ", ".join(f"{k} {v:.4g}" for k, v in rec.items() if isinstance(v, float)))
        rows.append(rec)

    # cepstral configuration: MFCCT vs MFCC on the 64 x 30 s batch
    cfg = workloads.config2(n_fft=1200, hop=160)
    measure("cepstral 64x30s N=1200 M=128 K=40 (MFCCT vs MFCC)", cfg["wave"], cfg["offsets"], 16000.0, 1200, 160,
            128, 0.0, 8000.0, output=melt.MELT_OUT_MFCC, precs=("fp32", "bf16"))
    # duration sweep: one clip of 1..160 s
    for sec in (1, 4, 10, 40, 160):
        cfg = workloads.config2(n_clips=1, seconds=float(sec))
        measure(f"duration {sec} s", cfg["wave"], cfg["offsets"], 16000.0, 400, 160, 80, 80.0, 7600.0)
    # Mel-bin sweep on 16 clips of 4 s
    for M in (40, 80, 128, 256, 512):
        cfg = workloads.config2(n_mels=M, n_clips=16, seconds=4.0)
        measure(f"n_mels {M} (16 x 4 s)", cfg["wave"], cfg["offsets"], 16000.0, 400, 160, M, 80.0, 7600.0)
    # batch sweep of 4 s clips
    for B in (1, 16, 64, 256):
        cfg = workloads.config2(n_clips=B, seconds=4.0)
        measure(f"batch {B} x 4 s", cfg["wave"], cfg["offsets"], 16000.0, 400, 160, 80, 80.0, 7600.0)
    with open(path, "w") as fh:
        for r in rows:
            fh.write(json.dumps(r) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n-mels", type=int, default=80)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time only the FP32 MelT path and the comparator")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled error check")
    ap.add_argument("--no-energy", action="store_true", help="skip the board-energy windows (amdsmi)")
    ap.add_argument("--trials", type=int, default=20, help="timing trials per path (median + bootstrap 90%% CI)")
    ap.add_argument("--only", default=None,
                    help="time one path only: fp32|bf16|fp16|bf16x3|fp16x3|fp8|fp8b|stft|copy (profiling)")
    ap.add_argument("--sweep", action="store_true", help="time every kernel variant of every precision and exit")
    ap.add_argument("--write-traffic", default=None, metavar="PMC_DIR",
                    help="write the committed traffic summary of the FP32 kernel from rocprofv3 --pmc runs "
                         "(subfolders fp32_f, fp32_w, copy_f, copy_w) and exit; runs on the CPU")
    ap.add_argument("--systems", default=None, metavar="PATH",
                    help="time the ragged batch, streaming (eager and graph) and backward workloads; write JSON "
                         "lines to PATH and exit")
    ap.add_argument("--workloads", default=None,
                    help="write the paper's efficiency workloads on synthetic stand-ins (cepstral configuration, "
                         "duration, Mel-bin and batch sweeps) as JSON lines to this file and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported (the frames of a batch "
              f"are independent, so N GPUs would each take 1/N of the clips with no communication)",
              file=sys.stderr)
        return 2

    if args.write_traffic:
        # the same workload's sizes, from its generator (no GPU needed)
        import workloads
        cfg = workloads.config2(n_mels=args.n_mels)
        T = int(sum(1 + (int(b - a) - 400) // 160 for a, b in zip(cfg["offsets"][:-1], cfg["offsets"][1:])))
        wave_bytes = cfg["wave"].nbytes
        write_traffic(args.write_traffic, T, wave_bytes + T * args.n_mels * 4 + 2 * args.n_mels * 400 * 4, wave_bytes)
        return 0

    import torch
    import paper_2606_01009_amd as melt
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    melt.load_library()
    M = args.n_mels
    full_line = not (args.only or args.sweep or args.workloads or args.systems)
    meter, idle = None, None
    if full_line and not args.no_energy:
        try:
            meter = EnergyMeter(torch)
            log("bench: idle board power (before any GPU work of the bench)")
            idle = meter.idle_watts(torch)
        except Exception as e:          # no counter on this machine: the line says so
            meter, idle = None, {"error": f"{type(e).__name__}: {e}"}
    log(f"bench: generating 64 x 30 s synthetic clips (n_mels={M})")
    cfg = workloads.config2(n_mels=M)
    wave, offsets = cfg["wave"], cfg["offsets"]
    T = melt.total_frames(offsets, 400, 160)
    d_wave = torch.from_numpy(wave).cuda()
    d_off = torch.from_numpy(offsets).cuda()
    out = torch.empty((T, M), dtype=torch.float32, device="cuda")
    flop_per_frame = 4 * 400 * M                       # 2 FLOP x N x 2M per frame
    bytes_per_launch = wave.nbytes + T * M * 4 + 2 * M * 400 * 4   # wave once + output once + basis

    def run_melt(prec):
        plan = melt.MeltPlan(sample_rate=16000.0, n_fft=400, hop=160, n_mels=M, fmin=0.0, fmax=8000.0, precision=prec)
        step_ms = time_launches(torch, lambda: plan.forward(d_wave, d_off, T, out=out), args.steps, args.warmup)
        melt.melt_batch_prepare(plan.handle, d_off, T)
        kern_ms = time_launches(torch, lambda: melt.melt_forward_prepared(plan.handle, d_wave, out),
                                args.steps, args.warmup)
        res = {"frames_per_s": T / (step_ms * 1e-3), "ms_per_step": step_ms, "kernel_ms": kern_ms,
               "tflops": T * flop_per_frame / (kern_ms * 1e-3) / 1e12,
               "hbm_gbps": bytes_per_launch / (kern_ms * 1e-3) / 1e9}
        if full_line:
            step = lambda: plan.forward(d_wave, d_off, T, out=out)
            res["trials"] = trial_stats(torch, step, args.steps, args.trials)
            if meter is not None:
                res["energy"] = energy_per_call(meter, torch, step, res["trials"]["median_ms"], idle[0], T)
        # the bound of each precision: FP32 and the split 16-bit products (three products per
        # term) are MFMA-bound, the others HBM-bound (the waveform read once and the output
        # written once)
        if prec in ("fp32", "bf16x3", "fp16x3"):
            work = T * flop_per_frame * (1 if prec == "fp32" else 3)
            peak = PEAK["f32"] if prec == "fp32" else PEAK["bf16"]
            res["roofline"] = {"bound": "mfma", "frac": work / (kern_ms * 1e-3) / peak}
        else:
            res["roofline"] = {"bound": "hbm", "frac": bytes_per_launch / (kern_ms * 1e-3) / PEAK["hbm"]}
        if not args.no_check:
            res["error_vs_fp64_oracle"] = sampled_error_db(out.cpu().numpy(), wave, offsets, "melt", oracle_freqs(M),
                                                           n_mels=M)
        log(f"bench: MelT {prec}: {res['frames_per_s'] / 1e6:.1f} M frames/s, kernel {kern_ms * 1e3:.1f} us")
        return res, plan

    def run_stft():
        plan = melt.MeltPlan(sample_rate=16000.0, n_fft=400, hop=160, n_mels=M, fmin=0.0, fmax=8000.0)
        step_ms = time_launches(torch, lambda: plan.stft_mel(d_wave, d_off, T, out=out), args.steps, args.warmup)
        melt.melt_batch_prepare(plan.handle, d_off, T)
        kern_ms = time_launches(torch, lambda: melt.stft_mel_forward_prepared(plan.handle, d_wave, out),
                                args.steps, args.warmup)
        res = {"frames_per_s": T / (step_ms * 1e-3), "ms_per_step": step_ms, "kernel_ms": kern_ms,
               "hbm_gbps": bytes_per_launch / (kern_ms * 1e-3) / 1e9,
               "roofline": {"bound": "hbm", "frac": bytes_per_launch / (kern_ms * 1e-3) / PEAK["hbm"]}}
        if full_line:
            step = lambda: plan.stft_mel(d_wave, d_off, T, out=out)
            res["trials"] = trial_stats(torch, step, args.steps, args.trials)
            if meter is not None:
                res["energy"] = energy_per_call(meter, torch, step, res["trials"]["median_ms"], idle[0], T)
        if not args.no_check:
            res["error_vs_fp64_oracle"] = sampled_error_db(out.cpu().numpy(), wave, offsets, "stft", None, n_mels=M)
        log(f"bench: FFT+filterbank: {res['frames_per_s'] / 1e6:.1f} M frames/s, kernel {kern_ms * 1e3:.1f} us")
        return res

    if args.workloads:
        run_workloads(torch, melt, workloads, args.workloads)
        return 0
    if args.systems:
        run_systems(torch, melt, workloads, args.systems)
        return 0

    if args.sweep:
        for prec in ("fp32", "bf16", "fp16", "bf16x3", "fp16x3", "fp8", "fp8b"):
            plan = melt.MeltPlan(sample_rate=16000.0, n_fft=400, hop=160, n_mels=M, precision=prec)
            desc = melt.melt_autotune(plan.handle, T)
            log(f"bench: autotune {prec}: {desc}")
        return 0

    if args.only:
        if args.only == "stft":
            run_stft()
        elif args.only == "copy":
            # a plain elementwise copy of the waveform buffer (read + write of 122.9 MB per
            # launch): the known-size kernel against which HBM traffic counters are scaled
            dst = torch.empty_like(d_wave)
            copy_ms = time_launches(torch, lambda: torch.mul(d_wave, 1.0, out=dst), args.steps, args.warmup)
            log(f"bench: copy kernel {wave.nbytes / 1e6:.1f} MB read + written: {copy_ms * 1e3:.1f} us, "
                f"{2 * wave.nbytes / (copy_ms * 1e-3) / 1e9:.0f} GB/s")
        else:
            run_melt(args.only)
        return 0

    fp32, plan32 = run_melt("fp32")
    plan32_variant = 0          # the plan's default kernel variant, the one timed
    comparator = run_stft()
    variants = {}
    if not args.no_variants:
        for prec in ("fp16x3", "bf16x3", "bf16", "fp16", "fp8", "fp8b"):
            try:
                variants[prec] = run_melt(prec)[0]
            except melt.MeltError as e:
                variants[prec] = {"error": str(e)}

    source_id = kernel_source_id()
    traffic = load_traffic(TRAFFIC_FILE, source_id)
    achieved = T * flop_per_frame / (fp32["kernel_ms"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK["f32"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / (PEAK["f32"] / 1e12), "traffic": traffic,
                "kernel": f"{melt.melt_variant_name(plan32.handle, plan32_variant)} (MelT FP32 projection + energy + log)",
                "flop_per_launch": T * flop_per_frame, "kernel_ms": fp32["kernel_ms"],
                "kernel_source_id": source_id}

    line = {
        "metric": "Mel frames/s: MelT GEMM vs FFT+filterbank on 1 MI355X at stated dB error",
        "value": fp32["frames_per_s"],
        "unit": "Mel frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 clips x 30 s at 16 kHz (pink noise + AM tones), n_fft=400, hop=160, "
                               f"n_mels={M} HTK 0-8 kHz, T={T} frames; MelT FP32 (v_mfma_f32_32x32x2f32)",
                   "frames": T, "n_fft": 400, "hop": 160, "n_mels": M, "clips": 64, "seconds_per_clip": 30},
        "error_vs_fp64_oracle": fp32.get("error_vs_fp64_oracle"),
        "comparator_fft_filterbank": comparator,
        "melt_fp32_vs_fft": fp32["frames_per_s"] / comparator["frames_per_s"],
        "variants": variants,
        "roofline": roofline,
        "trials": fp32.get("trials"),
        "energy": fp32.get("energy") if meter is not None else idle,
    }
    if meter is not None:
        line["energy_idle"] = {"board_w": idle[0], "window_s": idle[1], "counter_quanta": idle[2]}
        line["energy_vs_fft_active"] = comparator["energy"]["active_mj_per_call"] / fp32["energy"]["active_mj_per_call"]
        meter.close()
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        line["cpu_baseline"] = cpu_baseline(wave, offsets, oracle_freqs(M), T)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
