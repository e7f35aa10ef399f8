"""Parity bounds for the GPU path against the FP64 oracle (test infrastructure).

The GPU projection sums K products in FP32 (MFMA accumulation).  With u = 2^-24, the sum
of K terms computed in any order satisfies the classical bound
    |R_gpu - R| <= gamma_K * A,   gamma_K = K u / (1 - K u),   A = sum |terms|,
where the terms are the exact products of the operands the GPU actually multiplies (the
oracle's operand model gives those exactly).  One more u*A covers the FP32 rounding of the
basis in the FP32 path.  From the bounds on R and I:
    |S_gpu - S| <= 2|R| dR + dR^2 + 2|I| dI + dI^2 + 3 u (S + bound)       (R^2 + I^2 in FP32)
and for L = ln(S + eps):
    |L_gpu - L| <= |dS| / (S + eps - |dS|) + 4 ulp(L) + u          (logf and the eps rounding)
A bin whose bound is vacuous (|dS| >= S + eps) is only checked to lie in
[ln(eps (1 - 2u)), ln(S + |dS| + eps)].  These bounds are the pass condition; the dB error
statistics below are reported alongside.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
DB_PER_NAT = 10.0 / np.log(10.0)


def log_power_bound(R, I, A_r, A_i, n_terms, eps, extra_rel=1.0):
    """Per-bin bound on |L_gpu - L| for L = ln(R^2 + I^2 + eps).  Returns (bound, vacuous)."""
    g = n_terms * U32 / (1 - n_terms * U32) + extra_rel * U32
    dR = g * A_r
    dI = g * A_i
    S = R * R + I * I
    dS = 2 * np.abs(R) * dR + dR * dR + 2 * np.abs(I) * dI + dI * dI
    dS += 3 * U32 * (S + dS)
    den = S + eps - dS
    vac = den <= 0
    L = np.log(S + eps)
    bound = np.where(vac, np.inf, dS / np.where(vac, 1.0, den)) + 4 * np.spacing(np.abs(L).astype(np.float32)) + U32
    return bound, vac, S, dS


def check_log_power(L_gpu, R, I, A_r, A_i, n_terms, eps, extra_rel=1.0, label=""):
    """Asserts the per-bin bound; returns a dict of statistics (dB errors on active bins)."""
    L_gpu = np.asarray(L_gpu, np.float64)
    bound, vac, S, dS = log_power_bound(R, I, A_r, A_i, n_terms, eps, extra_rel)
    L = np.log(S + eps)
    err = np.abs(L_gpu - L)
    ok = ~vac
    bad = ok & (err > bound)
    if np.any(bad):
        idx = np.argwhere(bad)[:8]
        lines = [f"t={t} m={m} gpu={L_gpu[t, m]:.9g} oracle={L[t, m]:.9g} err={err[t, m]:.3g} bound={bound[t, m]:.3g}"
                 for t, m in idx]
        raise AssertionError(f"{label}: {int(bad.sum())} of {bad.size} bins beyond the FP32 bound\n" + "\n".join(lines))
    if np.any(vac):
        lo = np.log(eps * (1 - 2 * U32)) - 1e-6
        hi = np.log(S + dS + eps) + 1e-6
        inside = (L_gpu[vac] >= lo) & (L_gpu[vac] <= hi[vac])
        assert np.all(inside), f"{label}: noise-floor bins outside [ln eps, ln(S+dS+eps)]"
    return db_stats(L_gpu, L, S)


def db_stats(L_gpu, L_ref, S_ref, active_db=80.0):
    """dB error statistics over the bins within `active_db` of each clip's peak (all frames
    treated as one clip) and over all bins."""
    e = DB_PER_NAT * (np.asarray(L_gpu, np.float64) - L_ref)
    act = S_ref >= S_ref.max() * 10.0 ** (-active_db / 10.0) if S_ref.size else np.zeros(0, bool)
    ea = np.abs(e[act]) if np.any(act) else np.zeros(1)
    return dict(max_db=float(ea.max()), rms_db=float(np.sqrt(np.mean(ea ** 2))),
                p99_db=float(np.percentile(ea, 99)), max_db_all=float(np.abs(e).max()) if e.size else 0.0,
                active_frac=float(act.mean()) if act.size else 0.0)


def frames_as_clips(wave, offsets, n_fft, hop, frame_ids):
    """Re-expresses selected global frames as one-frame clips (start offsets), so the oracle
    can evaluate just those frames of a large batch."""
    offsets = np.asarray(offsets, np.int64)
    starts = []
    T_c = np.array([max(0, 1 + (b - a - n_fft) // hop) if b - a >= n_fft else 0
                    for a, b in zip(offsets[:-1], offsets[1:])], np.int64)
    fo = np.concatenate([[0], np.cumsum(T_c)])
    for f in frame_ids:
        c = int(np.searchsorted(fo, f, side="right") - 1)
        starts.append(offsets[c] + (f - fo[c]) * hop)
    segs = [wave[s:s + n_fft] for s in starts]
    sub = np.concatenate(segs).astype(np.float32)
    off = np.arange(len(segs) + 1, dtype=np.int64) * n_fft
    return sub, off
