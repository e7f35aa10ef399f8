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


def oracle_basis(orc, cfg):
    """The oracle's own analysis frequencies and window-folded basis for a plan
    configuration (a melt_config): Mel centres from the oracle's Mel scale (Eq. mel_scale,
    Eq. inverse_mel) with the configuration's formula and placement, and the basis of
    Eq. dmp_weights with its window.  Nothing here is taken from the plan under test, so
    the placement of the centres is checked too.  Returns (freqs, Wr, Wi)."""
    formula = {0: orc.MEL_HTK, 1: orc.MEL_SLANEY}[int(cfg.mel_formula)]
    placement = {0: orc.PLACE_FILTER_CENTRES, 1: orc.PLACE_LINSPACE}[int(cfg.placement)]
    window = {0: orc.WIN_HANN_SYMMETRIC, 1: orc.WIN_HANN_PERIODIC, 2: orc.WIN_RECT}[int(cfg.window)]
    f = orc.melt_frequencies(int(cfg.n_mels), float(cfg.fmin), float(cfg.fmax), formula, placement)
    Wr, Wi = orc.melt_basis(sr=float(cfg.sample_rate), n_fft=int(cfg.n_fft), freqs=f, window_kind=window)
    return f, Wr, Wi


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
        # the log is evaluated and stored in FP32: the same 4 ulps of |L| as the active-bin bound
        lo0 = np.log(eps * (1 - 2 * U32))
        lo = lo0 - 4 * np.spacing(np.float32(abs(lo0))) - 1e-6
        hi = np.log(S + dS + eps)
        hi = hi + 4 * np.spacing(np.abs(hi).astype(np.float32)) + 1e-6
        inside = (L_gpu[vac] >= lo) & (L_gpu[vac] <= hi[vac])
        if not np.all(inside):
            out = np.argwhere(vac)[~inside][:8]
            lines = [f"t={t} m={m} gpu={L_gpu[t, m]:.9g} S={S[t, m]:.3g} dS={dS[t, m]:.3g} lo={lo:.9g} "
                     f"hi={hi[t, m]:.9g}" for t, m in out]
            raise AssertionError(f"{label}: {int((~inside).sum())} noise-floor bins outside "
                                 f"[ln eps, ln(S+dS+eps)]\n" + "\n".join(lines))
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


def frames_as_clips(wave, offsets, n_fft, hop, frame_ids, tail=0):
    """Re-expresses selected global frames as one-frame clips (start offsets), so the oracle
    can evaluate just those frames of a large batch.  tail (< hop) keeps up to that many
    samples past each frame, within its clip: the rest of the frame's last 32-sample block, on
    which the block-scaled FP8 scale of that block depends."""
    assert 0 <= tail < hop
    offsets = np.asarray(offsets, np.int64)
    segs = []
    T_c = np.array([max(0, 1 + (b - a - n_fft) // hop) if b - a >= n_fft else 0
                    for a, b in zip(offsets[:-1], offsets[1:])], np.int64)
    fo = np.concatenate([[0], np.cumsum(T_c)])
    for f in frame_ids:
        c = int(np.searchsorted(fo, f, side="right") - 1)
        s = offsets[c] + (f - fo[c]) * hop
        segs.append(wave[s:min(s + n_fft + tail, offsets[c + 1])])
    sub = np.concatenate(segs).astype(np.float32)
    off = np.concatenate([[0], np.cumsum([len(g) for g in segs])]).astype(np.int64)
    return sub, off


def fft_pair_norms(wave, offsets, n_fft, hop, window):
    """For every frame, ||w x_f||^2 + ||w x_g||^2 where g is the frame that shares its complex
    FFT (frames 2p and 2p+1 of a clip are packed into one FFT as z = a + i b)."""
    offsets = np.asarray(offsets, np.int64)
    out = []
    for a, b in zip(offsets[:-1], offsets[1:]):
        L = b - a
        Tc = 1 + (L - n_fft) // hop if L >= n_fft else 0
        e = np.array([np.sum((window * wave[a + t * hop:a + t * hop + n_fft].astype(np.float64)) ** 2)
                      for t in range(Tc)])
        partner = np.zeros(Tc)
        for t in range(Tc):
            g = t ^ 1
            partner[t] = e[g] if g < Tc else 0.0
        out.append(e + partner)
    return np.concatenate(out) if out else np.zeros(0)


def log_error_radius(R, I, A_r, A_i, n_terms, eps, extra_rel=1.0):
    """A finite per-bin bound on |L_gpu - L| for the cepstrum: the log_power_bound, and on
    vacuous bins the width of the interval the GPU value is confined to."""
    bound, vac, S, dS = log_power_bound(R, I, A_r, A_i, n_terms, eps, extra_rel)
    L = np.log(S + eps)
    width = np.maximum(np.log(S + dS + eps) - L, L - np.log(eps * (1 - 2 * U32))) + 1e-6
    return np.where(vac, width, bound), L


def check_cepstrum(C_gpu, L, bL, D, label="", split=False):
    """C = L D^T (Eq. mfcct_matrix) from log-Mel rows L with per-bin error radius bL: the
    FP32 product adds gamma_M sum |D||L| plus the FP32 rounding of D (u sum |D||L|), so
        |C_gpu - C| <= |D| bL + (gamma_M + u) |D| |L| + u |C|.
    split: the product runs as Lh Dh + Lh Dl + Ll Dh on binary16 operands (hi + lo of the
    FP32 values scaled by 2^9 and 2^10).  Each lo rounds to 11 bits (|x - xh - xl| <= 2^-22 |x|
    on either side), the dropped Ll Dl is at most 2^-22 |L||D|, and 3M exact products are
    summed in FP32: (gamma_3M + u + 4 * 2^-22) |D| |L|, plus M times half a binary16 subnormal
    step per operand (2^-25 in the scaled units) for the lo parts that fall below the normal
    range."""
    C_gpu = np.asarray(C_gpu, np.float64)
    M = D.shape[1]
    C = L @ D.T
    if split:
        g = 3 * M * U32 / (1 - 3 * M * U32) + U32 + 4 * 2.0 ** -22
        tiny = M * (2.0 ** -25 / 2 ** 10 * np.abs(L).max(initial=0.0) + 2.0 ** -25 / 2 ** 9 + 2.0 ** -44)
    else:
        g = M * U32 / (1 - M * U32) + U32
        tiny = 0.0
    bound = bL @ np.abs(D).T + g * (np.abs(L) @ np.abs(D).T) + U32 * np.abs(C) + tiny + 1e-30
    err = np.abs(C_gpu - C)
    bad = err > bound
    if np.any(bad):
        idx = np.argwhere(bad)[:8]
        lines = [f"t={t} k={k} gpu={C_gpu[t, k]:.9g} oracle={C[t, k]:.9g} err={err[t, k]:.3g} bound={bound[t, k]:.3g}"
                 for t, k in idx]
        raise AssertionError(f"{label}: {int(bad.sum())} of {bad.size} coefficients beyond the bound\n" + "\n".join(lines))
    return {"max_abs": float(err.max()) if err.size else 0.0, "max_bound": float(bound.max()) if bound.size else 0.0}


def stft_log_bound(P, F, pair_norm2, n_fft, eps, c_fft=4.0):
    """Per-bin bound of the FFT + filterbank log-Mel output (see check_stft_log); returns
    (bound, vacuous, mel, dmel)."""
    levels = np.log2(n_fft)
    delta = c_fft * U32 * levels * np.sqrt(n_fft * pair_norm2)
    absX = np.sqrt(P)
    dP = 2 * absX * delta[:, None] + delta[:, None] ** 2
    mel = P @ F.T
    nnz = np.count_nonzero(F, axis=1)
    dmel = dP @ F.T + (nnz[None, :] + 3) * U32 * mel
    den = mel + eps - dmel
    vac = den <= 0
    L = np.log(mel + eps)
    bound = np.where(vac, np.inf, dmel / np.where(vac, 1.0, den)) + 4 * np.spacing(np.abs(L).astype(np.float32)) + U32
    return bound, vac, mel, dmel


def check_stft_log(L_gpu, P, F, pair_norm2, n_fft, eps, c_fft=4.0, label=""):
    """Bound for the FFT + filterbank path.  A floating-point FFT of size N has a norm-wise
    error ||dZ||_2 <= levels * eta * ||Z||_2 with eta a few u per butterfly level; Z here
    carries the two packed frames, ||Z||_2^2 = N (||w a||^2 + ||w b||^2).  Every bin therefore
    has |dX_k| <= delta = c_fft * u * log2(N) * sqrt(N * pair_norm2).  Then
    |dP_k| <= 2 |X_k| delta + delta^2, the non-negative filters give
    |dmel_m| <= sum_k F[m,k] |dP_k| + (nnz_m + 3) u mel_m, and the log adds its rounding."""
    L_gpu = np.asarray(L_gpu, np.float64)
    levels = np.log2(n_fft)
    delta = c_fft * U32 * levels * np.sqrt(n_fft * pair_norm2)          # [T]
    absX = np.sqrt(P)                                                     # [T, NB]
    dP = 2 * absX * delta[:, None] + delta[:, None] ** 2
    mel = P @ F.T
    nnz = np.count_nonzero(F, axis=1)
    dmel = dP @ F.T + (nnz[None, :] + 3) * U32 * mel
    den = mel + eps - dmel
    vac = den <= 0
    L = np.log(mel + eps)
    bound = np.where(vac, np.inf, dmel / np.where(vac, 1.0, den)) + 4 * np.spacing(np.abs(L).astype(np.float32)) + U32
    err = np.abs(L_gpu - L)
    bad = (~vac) & (err > bound)
    if np.any(bad):
        idx = np.argwhere(bad)[:8]
        lines = [f"t={t} m={m} gpu={L_gpu[t, m]:.9g} oracle={L[t, m]:.9g} err={err[t, m]:.3g} bound={bound[t, m]:.3g}"
                 for t, m in idx]
        raise AssertionError(f"{label}: {int(bad.sum())} of {bad.size} bins beyond the FFT bound\n" + "\n".join(lines))
    if np.any(vac):
        # the log is evaluated and stored in FP32: the same 4 ulps of |L| as the active-bin bound
        lo0 = np.log(eps * (1 - 2 * U32))
        lo = lo0 - 4 * np.spacing(np.float32(abs(lo0))) - 1e-6
        hi = np.log(mel + dmel + eps)
        hi = hi + 4 * np.spacing(np.abs(hi).astype(np.float32)) + 1e-6
        assert np.all(L_gpu[vac] <= hi[vac]) and np.all(L_gpu[vac] >= lo), label
    return db_stats(L_gpu, L, mel)


# ------------------------------------------------------------------ backward

def _map_dS(S, kind, eps):
    """d out / dS of the output maps (the same subgradient convention as the oracle)."""
    S = np.asarray(S, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        if kind == 0:
            return 1.0 / (S + eps)
        if kind == 1:
            r = np.sqrt(S)
            return np.where(S > 0, 1.0 / (2.0 * r * (r + eps)), np.inf)
        if kind == 2:
            return np.ones_like(S)
        return np.where(S > 0, 0.5 / np.sqrt(S), np.inf)


def grad_proj_error(R, I, eR, eI, g, kind, eps, c_round=8.0):
    """Per-element bound on the GPU's gradients of the projections, G = 2 (R, I) g map'(S)
    (chain rule through Eqs. meltf, dmp_energy), computed in FP32 from projections that
    differ from the reference R, I by at most eR, eI per bin.

    With S = R^2 + I^2 and |S_gpu - S| <= dS (products, sum and their FP32 roundings),
    map' is positive and non-increasing on [S - dS, S + dS], so it stays within
    phi_hi = map'(S - dS) and moves by at most dphi = max(map'(S - dS) - map'(S),
    map'(S) - map'(S + dS)).  Then
        |G_gpu - G| <= 2|g| (e phi_hi + |R| dphi) + c u 2|g| (|R| + e) phi_hi
    with c = 8 covering the FP32 evaluation of map' (square root, reciprocal), the products
    by g and by 2 R, and the rounding of S + eps.  Returns (dGr, dGi, checkable): a bin is
    checkable where dS < S / 2 (its energy is resolved to better than a factor 2; below
    that, the forward value is rounding noise and so is any gradient through it)."""
    R = np.asarray(R, np.float64)
    I = np.asarray(I, np.float64)
    S = R * R + I * I
    dS = (2 * np.abs(R) * eR + eR * eR + 2 * np.abs(I) * eI + eI * eI) * (1 + 2 * U32) + 2 * U32 * S
    checkable = dS < 0.5 * S
    if kind == 0:
        checkable |= (dS < 0.5 * (S + eps)) & (S + eps > 0)
    S_lo = np.maximum(S - dS, 0.0)
    S_hi = S + dS
    phi = _map_dS(S, kind, eps)
    phi_hi = _map_dS(S_lo, kind, eps)
    phi_lo = _map_dS(S_hi, kind, eps)
    with np.errstate(invalid="ignore"):
        dphi = np.maximum(phi_hi - phi, phi - phi_lo)
    ag = 2.0 * np.abs(np.asarray(g, np.float64))
    # phi_hi is infinite only where S - dS <= 0 (magnitude kinds), which is never checkable
    with np.errstate(invalid="ignore"):
        dGr = ag * (eR * phi_hi + np.abs(R) * dphi) + c_round * U32 * ag * (np.abs(R) + eR) * phi_hi
        dGi = ag * (eI * phi_hi + np.abs(I) * dphi) + c_round * U32 * ag * (np.abs(I) + eI) * phi_hi
    dGr = np.where(checkable, dGr, np.inf)
    dGi = np.where(checkable, dGi, np.inf)
    return dGr, dGi, checkable


def gamma(n):
    """gamma_n = n u / (1 - n u): the relative bound of an n-term FP32 sum of products in any
    order."""
    return n * U32 / (1 - n * U32)


def check_within(gpu, ref, bound, label, rel_slack=1e-6):
    """Element-wise |gpu - ref| <= bound (1 + rel_slack); returns statistics."""
    gpu = np.asarray(gpu, np.float64)
    err = np.abs(gpu - ref)
    bad = ~(err <= bound * (1 + rel_slack) + 1e-300)
    if np.any(bad):
        idx = np.flatnonzero(bad)[:8]
        lines = [f"i={i} gpu={gpu.flat[i]:.9g} ref={ref.flat[i]:.9g} err={err.flat[i]:.3g} bound={bound.flat[i]:.3g}"
                 for i in idx]
        raise AssertionError(f"{label}: {int(bad.sum())} of {bad.size} elements beyond the bound\n" + "\n".join(lines))
    scale = np.abs(ref)
    nz = scale > 0
    return {"max_err_over_bound": float(np.max(err / np.maximum(bound, 1e-300))) if err.size else 0.0,
            "median_rel_err": float(np.median(err[nz] / scale[nz])) if np.any(nz) else 0.0,
            "median_rel_bound": float(np.median(bound[nz] / scale[nz])) if np.any(nz) else 0.0}
