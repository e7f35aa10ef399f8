/*
 * FP64 CPU oracle for the MelT frontend (Direct Mel Projection + log) and for the
 * conventional STFT + triangular Mel filterbank pipeline it is compared with.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the GPU
 * library is checked against; it shares no code, header, table or constant with the
 * GPU library, and the product path never loads it.  Only tests, the smoke check and
 * the CPU-baseline leg of the benchmark use it.
 *
 * Everything is plain definition, evaluated in double precision, with no blocking,
 * no fast transform and no reordering beyond what the definitions state:
 *   - Mel scale and its inverse ............ Methodology, Eq. (mel_scale), Eq. (inverse_mel)
 *   - analysis frequencies ................. Methodology: the centres of the triangular
 *                                            Mel filterbank, uniformly spaced in Mel
 *   - symmetric Hann window ................ Methodology (x~_t[n] = w[n] x_t[n])
 *   - R, I by direct summation ............. Eq. (dmp_components)
 *   - S = R^2 + I^2, log(S + eps) .......... Eq. (dmp_energy), Eq. (meltf)
 *   - window folded into the basis ......... Eq. (dmp_weights), Eq. (dmp_projection)
 *   - STFT power + triangular filterbank ... Methodology (conventional Mel filtering on
 *                                            uniform FFT bins), Eq. (complexity_conv)
 *   - orthonormal DCT-II for MFCCT ......... Eq. (mfcct_matrix)
 * The gradient of the projection and the reduced-precision operand models are not in
 * the paper; they follow from the chain rule and from the published definitions of the
 * bfloat16, IEEE binary16 and OCP FP8 E4M3 formats.
 *
 * Conventions (readings where the paper is silent): frames start at t*hop with no
 * centring or padding; a clip shorter than n_fft has no frames; the additive eps is a
 * parameter; "log" is the natural logarithm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------ Mel scales */

/* Eq. (mel_scale): mu(f) = 2595 log10(1 + f/700) (formula 0, HTK).
 * formula 1 is the Slaney/Auditory-Toolbox scale (linear below 1 kHz, log above),
 * kept only as an option of the comparator's filterbank. */
double oracle_hz_to_mel(double f, int formula)
{
    if (formula == 0) return 2595.0 * log10(1.0 + f / 700.0);
    {
        const double f_sp = 200.0 / 3.0, min_log_hz = 1000.0;
        const double min_log_mel = min_log_hz / f_sp, logstep = log(6.4) / 27.0;
        if (f < min_log_hz) return f / f_sp;
        return min_log_mel + log(f / min_log_hz) / logstep;
    }
}

/* Eq. (inverse_mel): f = 700 (10^(mu/2595) - 1), and the Slaney inverse. */
double oracle_mel_to_hz(double mu, int formula)
{
    if (formula == 0) return 700.0 * (pow(10.0, mu / 2595.0) - 1.0);
    {
        const double f_sp = 200.0 / 3.0, min_log_hz = 1000.0;
        const double min_log_mel = min_log_hz / f_sp, logstep = log(6.4) / 27.0;
        if (mu < min_log_mel) return f_sp * mu;
        return min_log_hz * exp(logstep * (mu - min_log_mel));
    }
}

/* The M+2 points of the triangular filterbank, uniformly spaced in Mel between fmin and
 * fmax, mapped back to Hz.  Point 0 = fmin, point M+1 = fmax. */
void oracle_mel_grid_hz(int n_mels, double fmin, double fmax, int formula, double *out)
{
    double lo = oracle_hz_to_mel(fmin, formula), hi = oracle_hz_to_mel(fmax, formula);
    for (int i = 0; i < n_mels + 2; ++i)
        out[i] = oracle_mel_to_hz(lo + (hi - lo) * (double)i / (double)(n_mels + 1), formula);
}

/* MelT analysis frequencies f_m, m = 0..M-1.
 * placement 0: the centres of the M triangular filters, i.e. grid points 1..M of the
 *              M+2-point grid (the filterbank the Methodology names);
 * placement 1: M points uniformly spaced in Mel from fmin to fmax inclusive. */
void oracle_melt_frequencies(int n_mels, double fmin, double fmax, int formula, int placement,
                             double *f_out)
{
    if (placement == 0) {
        double *g = (double *)malloc(sizeof(double) * (size_t)(n_mels + 2));
        oracle_mel_grid_hz(n_mels, fmin, fmax, formula, g);
        for (int m = 0; m < n_mels; ++m) f_out[m] = g[m + 1];
        free(g);
    } else {
        double lo = oracle_hz_to_mel(fmin, formula), hi = oracle_hz_to_mel(fmax, formula);
        for (int m = 0; m < n_mels; ++m) {
            double mu = (n_mels == 1) ? lo : lo + (hi - lo) * (double)m / (double)(n_mels - 1);
            f_out[m] = oracle_mel_to_hz(mu, formula);
        }
    }
}

/* ------------------------------------------------------------------ window, frames */

/* kind 0: symmetric Hann, w[n] = 0.5 - 0.5 cos(2 pi n / (N-1));
 * kind 1: periodic Hann (denominator N); kind 2: rectangular. */
void oracle_window(int n, int kind, double *w)
{
    for (int i = 0; i < n; ++i) {
        if (kind == 2) { w[i] = 1.0; continue; }
        double den = (kind == 0) ? (double)(n - 1) : (double)n;
        w[i] = (n == 1) ? 1.0 : 0.5 - 0.5 * cos(2.0 * OR_PI * (double)i / den);
    }
}

/* Frames of a clip of L samples: 1 + floor((L - N) / H), none if L < N. */
int64_t oracle_num_frames(int64_t L, int n_fft, int hop)
{
    if (L < n_fft) return 0;
    return 1 + (L - n_fft) / hop;
}

/* Frame table: for every frame of every clip, its first sample.  Returns T. */
static int64_t frame_starts(const int64_t *clip_off, int n_clips, int n_fft, int hop,
                            int64_t **starts_out)
{
    int64_t T = 0;
    for (int c = 0; c < n_clips; ++c)
        T += oracle_num_frames(clip_off[c + 1] - clip_off[c], n_fft, hop);
    int64_t *st = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T > 0 ? T : 1));
    int64_t t = 0;
    for (int c = 0; c < n_clips; ++c) {
        int64_t Tc = oracle_num_frames(clip_off[c + 1] - clip_off[c], n_fft, hop);
        for (int64_t j = 0; j < Tc; ++j) st[t++] = clip_off[c] + j * hop;
    }
    *starts_out = st;
    return T;
}

int64_t oracle_total_frames(const int64_t *clip_off, int n_clips, int n_fft, int hop)
{
    int64_t T = 0;
    for (int c = 0; c < n_clips; ++c)
        T += oracle_num_frames(clip_off[c + 1] - clip_off[c], n_fft, hop);
    return T;
}

/* ------------------------------------------------------------------ output maps */

/* kind 0: ln(S + eps)          (Eq. meltf, power)
 * kind 1: ln(sqrt(S) + eps)    (magnitude option)
 * kind 2: S                    (power, no log)
 * kind 3: sqrt(S)              (magnitude, no log) */
static double output_map(double S, int kind, double eps)
{
    switch (kind) {
    case 0: return log(S + eps);
    case 1: return log(sqrt(S) + eps);
    case 2: return S;
    default: return sqrt(S);
    }
}

/* d output / dS (subgradient 0 for the magnitude forms at S = 0). */
static double output_map_dS(double S, int kind, double eps)
{
    switch (kind) {
    case 0: return 1.0 / (S + eps);
    case 1: return S > 0.0 ? 1.0 / (2.0 * sqrt(S) * (sqrt(S) + eps)) : 0.0;
    case 2: return 1.0;
    default: return S > 0.0 ? 1.0 / (2.0 * sqrt(S)) : 0.0;
    }
}

/* ------------------------------------------------------------------ MelT (NDFT) */

/* Eq. (dmp_components), (dmp_energy), (meltf) by direct summation:
 *   R[t,m] = sum_n w[n] x_t[n] cos(2 pi f_m n / sr)
 *   I[t,m] = sum_n w[n] x_t[n] sin(2 pi f_m n / sr)
 *   out[t,m] = map(R^2 + I^2)
 * The cos/sin of every (m, n) is evaluated from the plain argument in FP64.
 * out, R, I are [T, n_freq] frame-major; R and I may be NULL.  Returns T. */
int64_t oracle_melt_forward(const float *wave, const int64_t *clip_off, int n_clips, double sr,
                            int n_fft, int hop, int window, const double *freqs, int n_freq,
                            int out_kind, double eps, double *out, double *R_out, double *I_out)
{
    int64_t *st;
    int64_t T = frame_starts(clip_off, n_clips, n_fft, hop, &st);
    double *w = (double *)malloc(sizeof(double) * (size_t)n_fft);
    double *C = (double *)malloc(sizeof(double) * (size_t)n_fft * (size_t)n_freq);
    double *Sn = (double *)malloc(sizeof(double) * (size_t)n_fft * (size_t)n_freq);
    oracle_window(n_fft, window, w);
    for (int m = 0; m < n_freq; ++m)
        for (int n = 0; n < n_fft; ++n) {
            double arg = 2.0 * OR_PI * freqs[m] * (double)n / sr;
            C[(size_t)m * n_fft + n] = cos(arg);
            Sn[(size_t)m * n_fft + n] = sin(arg);
        }
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < T; ++t) {
        const float *x = wave + st[t];
        for (int m = 0; m < n_freq; ++m) {
            double r = 0.0, i = 0.0;
            for (int n = 0; n < n_fft; ++n) {
                double xt = w[n] * (double)x[n];
                r += xt * C[(size_t)m * n_fft + n];
                i += xt * Sn[(size_t)m * n_fft + n];
            }
            out[t * n_freq + m] = output_map(r * r + i * i, out_kind, eps);
            if (R_out) R_out[t * n_freq + m] = r;
            if (I_out) I_out[t * n_freq + m] = i;
        }
    }
    free(st); free(w); free(C); free(Sn);
    return T;
}

/* Eq. (dmp_weights): the window folded into the cos/sin basis,
 *   Wr[m,n] = w[n] cos(2 pi f_m n / sr),  Wi[m,n] = w[n] sin(2 pi f_m n / sr),
 * each [n_freq, n_fft] row-major. */
void oracle_melt_basis(double sr, int n_fft, int window, const double *freqs, int n_freq,
                       double *Wr, double *Wi)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n_fft);
    oracle_window(n_fft, window, w);
    for (int m = 0; m < n_freq; ++m)
        for (int n = 0; n < n_fft; ++n) {
            double arg = 2.0 * OR_PI * freqs[m] * (double)n / sr;
            Wr[(size_t)m * n_fft + n] = w[n] * cos(arg);
            Wi[(size_t)m * n_fft + n] = w[n] * sin(arg);
        }
    free(w);
}

/* Eq. (dmp_projection) with an explicit (possibly learned) basis, on frames
 * X[t, n] = x[start_t + n]:  R = X Wr^T, I = X Wi^T, out = map(R^2 + I^2). */
int64_t oracle_melt_forward_basis(const float *wave, const int64_t *clip_off, int n_clips,
                                  int n_fft, int hop, const double *Wr, const double *Wi,
                                  int n_freq, int out_kind, double eps, double *out,
                                  double *R_out, double *I_out)
{
    int64_t *st;
    int64_t T = frame_starts(clip_off, n_clips, n_fft, hop, &st);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < T; ++t) {
        const float *x = wave + st[t];
        for (int m = 0; m < n_freq; ++m) {
            double r = 0.0, i = 0.0;
            for (int n = 0; n < n_fft; ++n) {
                r += (double)x[n] * Wr[(size_t)m * n_fft + n];
                i += (double)x[n] * Wi[(size_t)m * n_fft + n];
            }
            out[t * n_freq + m] = output_map(r * r + i * i, out_kind, eps);
            if (R_out) R_out[t * n_freq + m] = r;
            if (I_out) I_out[t * n_freq + m] = i;
        }
    }
    free(st);
    return T;
}

/* Chain rule through out = map(S), S = R^2 + I^2 (Eqs. meltf, dmp_energy), for given
 * projections R, I and upstream gradient g, all [T, n_freq]:
 *   Gr = dL/dR = 2 R g map'(S),  Gi = dL/dI = 2 I g map'(S).
 * R and I may be the exact projections or those of a reduced-precision forward. */
void oracle_melt_chain(int64_t T, int n_freq, const double *R, const double *I, const double *g,
                       int out_kind, double eps, double *Gr, double *Gi)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < T * (int64_t)n_freq; ++e) {
        double k = g[e] * output_map_dS(R[e] * R[e] + I[e] * I[e], out_kind, eps);
        Gr[e] = 2.0 * R[e] * k;
        Gi[e] = 2.0 * I[e] * k;
    }
}

/* Transpose of the projection R = X Wr^T, I = X Wi^T (Eq. dmp_projection) applied to
 * gradients Gr, Gi [T, n_freq] of R and I:
 *   dX = Gr Wr + Gi Wi, overlap-added over the frames: dx[start_t + n] += dX[t, n]
 *   dWr = Gr^T X,  dWi = Gi^T X.
 * grad_wave has the length of the whole waveform buffer (samples in no frame get 0).
 * Any of grad_wave, dWr, dWi may be NULL.  Returns T. */
int64_t oracle_melt_backward_linear(const float *wave, int64_t n_samples, const int64_t *clip_off,
                                    int n_clips, int n_fft, int hop, const double *Wr,
                                    const double *Wi, int n_freq, const double *Gr,
                                    const double *Gi, double *grad_wave, double *dWr, double *dWi)
{
    int64_t *st;
    int64_t T = frame_starts(clip_off, n_clips, n_fft, hop, &st);
    if (grad_wave) {
        for (int64_t s = 0; s < n_samples; ++s) grad_wave[s] = 0.0;
        for (int64_t t = 0; t < T; ++t)            /* serial overlap-add: no races */
            for (int n = 0; n < n_fft; ++n) {
                double acc = 0.0;
                for (int m = 0; m < n_freq; ++m)
                    acc += Gr[t * n_freq + m] * Wr[(size_t)m * n_fft + n] +
                           Gi[t * n_freq + m] * Wi[(size_t)m * n_fft + n];
                grad_wave[st[t] + n] += acc;
            }
    }
    if (dWr || dWi) {
#pragma omp parallel for schedule(static)
        for (int m = 0; m < n_freq; ++m)
            for (int n = 0; n < n_fft; ++n) {
                double ar = 0.0, ai = 0.0;
                for (int64_t t = 0; t < T; ++t) {
                    double xv = (double)wave[st[t] + n];
                    ar += Gr[t * n_freq + m] * xv;
                    ai += Gi[t * n_freq + m] * xv;
                }
                if (dWr) dWr[(size_t)m * n_fft + n] = ar;
                if (dWi) dWi[(size_t)m * n_fft + n] = ai;
            }
    }
    free(st);
    return T;
}

/* Gradient of out = map(R^2 + I^2), R = X Wr^T, I = X Wi^T, given the upstream
 * gradient g [T, n_freq] (chain rule; not in the paper): the projections by
 * oracle_melt_forward_basis, then oracle_melt_chain, then oracle_melt_backward_linear.
 * grad_wave has the length of the whole waveform buffer (samples in no frame get 0).
 * Any of grad_wave, dWr, dWi may be NULL.  Returns T. */
int64_t oracle_melt_backward(const float *wave, int64_t n_samples, const int64_t *clip_off,
                             int n_clips, int n_fft, int hop, const double *Wr, const double *Wi,
                             int n_freq, int out_kind, double eps, const double *grad_out,
                             double *grad_wave, double *dWr, double *dWi)
{
    int64_t T = oracle_total_frames(clip_off, n_clips, n_fft, hop);
    size_t n = (size_t)(T > 0 ? T : 1) * (size_t)n_freq;
    double *R = (double *)malloc(sizeof(double) * n), *I = (double *)malloc(sizeof(double) * n);
    double *L = (double *)malloc(sizeof(double) * n);
    double *Gr = (double *)malloc(sizeof(double) * n), *Gi = (double *)malloc(sizeof(double) * n);
    oracle_melt_forward_basis(wave, clip_off, n_clips, n_fft, hop, Wr, Wi, n_freq, 2, eps, L, R, I);
    oracle_melt_chain(T, n_freq, R, I, grad_out, out_kind, eps, Gr, Gi);
    oracle_melt_backward_linear(wave, n_samples, clip_off, n_clips, n_fft, hop, Wr, Wi, n_freq, Gr, Gi,
                                grad_wave, dWr, dWi);
    free(R); free(I); free(L); free(Gr); free(Gi);
    return T;
}

/* ------------------------------------------------------------------ STFT + filterbank */

/* Power spectrum of every frame by the naive DFT (no FFT):
 *   X_k = sum_n w[n] x_t[n] exp(-2 pi i k n / N),  P[t,k] = |X_k|^2,  k = 0..N/2.
 * The twiddle index k*n is reduced mod N exactly in integers.  P is [T, N/2+1]. */
int64_t oracle_power_spectrum(const float *wave, const int64_t *clip_off, int n_clips, int n_fft,
                              int hop, int window, double *P)
{
    int64_t *st;
    int64_t T = frame_starts(clip_off, n_clips, n_fft, hop, &st);
    int nb = n_fft / 2 + 1;
    double *w = (double *)malloc(sizeof(double) * (size_t)n_fft);
    double *c = (double *)malloc(sizeof(double) * (size_t)n_fft);
    double *s = (double *)malloc(sizeof(double) * (size_t)n_fft);
    oracle_window(n_fft, window, w);
    for (int j = 0; j < n_fft; ++j) {
        c[j] = cos(2.0 * OR_PI * (double)j / (double)n_fft);
        s[j] = sin(2.0 * OR_PI * (double)j / (double)n_fft);
    }
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < T; ++t) {
        const float *x = wave + st[t];
        for (int k = 0; k < nb; ++k) {
            double re = 0.0, im = 0.0;
            for (int n = 0; n < n_fft; ++n) {
                int64_t j = ((int64_t)k * n) % n_fft;
                double xt = w[n] * (double)x[n];
                re += xt * c[j];
                im -= xt * s[j];
            }
            P[t * nb + k] = re * re + im * im;
        }
    }
    free(st); free(w); free(c); free(s);
    return T;
}

/* Triangular Mel filterbank on the uniform DFT bins f_k = k sr / N, k = 0..N/2:
 *   F[m,k] = max(0, min((f_k - g_m)/(g_{m+1} - g_m), (g_{m+2} - f_k)/(g_{m+2} - g_{m+1})))
 * with g the M+2-point grid; norm 1 scales each triangle by 2/(g_{m+2} - g_m) (unit area).
 * F is [n_mels, N/2+1] row-major, dense. */
void oracle_mel_filterbank(int n_fft, double sr, int n_mels, double fmin, double fmax,
                           int formula, int norm, double *F)
{
    int nb = n_fft / 2 + 1;
    double *g = (double *)malloc(sizeof(double) * (size_t)(n_mels + 2));
    oracle_mel_grid_hz(n_mels, fmin, fmax, formula, g);
    for (int m = 0; m < n_mels; ++m) {
        double scale = (norm == 1) ? 2.0 / (g[m + 2] - g[m]) : 1.0;
        for (int k = 0; k < nb; ++k) {
            double fk = (double)k * sr / (double)n_fft;
            double lower = (fk - g[m]) / (g[m + 1] - g[m]);
            double upper = (g[m + 2] - fk) / (g[m + 2] - g[m + 1]);
            double v = lower < upper ? lower : upper;
            F[(size_t)m * nb + k] = (v > 0.0 ? v : 0.0) * scale;
        }
    }
    free(g);
}

/* Conventional pipeline: mel[t,m] = sum_k F[m,k] |X_k|^p (p = 2 for the power kinds,
 * p = 1 for the magnitude kinds), then ln(mel + eps) for the log kinds. */
int64_t oracle_stft_mel_forward(const float *wave, const int64_t *clip_off, int n_clips, double sr,
                                int n_fft, int hop, int window, int n_mels, double fmin,
                                double fmax, int formula, int norm, int out_kind, double eps,
                                double *out)
{
    int nb = n_fft / 2 + 1;
    int64_t T = oracle_total_frames(clip_off, n_clips, n_fft, hop);
    double *P = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * (size_t)nb);
    double *F = (double *)malloc(sizeof(double) * (size_t)n_mels * (size_t)nb);
    oracle_power_spectrum(wave, clip_off, n_clips, n_fft, hop, window, P);
    oracle_mel_filterbank(n_fft, sr, n_mels, fmin, fmax, formula, norm, F);
    int magnitude = (out_kind == 1 || out_kind == 3);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < T; ++t)
        for (int m = 0; m < n_mels; ++m) {
            double acc = 0.0;
            for (int k = 0; k < nb; ++k) {
                double p = P[t * nb + k];
                acc += F[(size_t)m * nb + k] * (magnitude ? sqrt(p) : p);
            }
            out[t * n_mels + m] = (out_kind <= 1) ? log(acc + eps) : acc;
        }
    free(P); free(F);
    return T;
}

/* ------------------------------------------------------------------ MFCCT */

/* Orthonormal DCT-II matrix D [K, M]:
 *   D[k,m] = sqrt(c_k / M) cos(pi k (2m + 1) / (2M)),  c_0 = 1, c_k = 2 otherwise.
 * Eq. (mfcct_matrix): C = log(S + eps) D^T. */
void oracle_dct2_ortho(int K, int M, double *D)
{
    for (int k = 0; k < K; ++k)
        for (int m = 0; m < M; ++m)
            D[(size_t)k * M + m] = sqrt((k == 0 ? 1.0 : 2.0) / (double)M) *
                                   cos(OR_PI * (double)k * (2.0 * m + 1.0) / (2.0 * M));
}

/* ------------------------------------------------------------------ operand rounding */
/* Models of the storage formats a reduced-precision product rounds its operands to.
 * Round-to-nearest-even throughout, from the format definitions:
 *   bfloat16  : 1 sign, 8 exponent (bias 127), 7 fraction bits
 *   binary16  : 1 sign, 5 exponent (bias 15), 10 fraction bits, subnormals
 *   E4M3 (OCP): 1 sign, 4 exponent (bias 7), 3 fraction bits, subnormals, no infinity,
 *               largest finite 448; values beyond saturate to +-448.
 * Each takes an FP32 value and returns the rounded value exactly as a double. */

/* Round |v| (finite, >= 0) to a binary format with p significant bits whose normal range
 * starts at 2^emin, with subnormal spacing 2^(emin - p + 1).  Exact in double for the
 * magnitudes used here. */
static double round_to_format(double a, int p, int emin)
{
    if (a == 0.0) return 0.0;
    int e;
    frexp(a, &e);                 /* a = f * 2^e, f in [0.5, 1) -> exponent of a is e-1 */
    int ea = e - 1;
    if (ea < emin) ea = emin;     /* subnormal range: fixed spacing */
    double q = ldexp(1.0, ea - (p - 1));   /* spacing of representable values near a */
    double n = a / q;             /* exact: power-of-two scaling */
    double fl = floor(n);
    double r = n - fl;
    double k;
    if (r > 0.5) k = fl + 1.0;
    else if (r < 0.5) k = fl;
    else k = (fmod(fl, 2.0) == 0.0) ? fl : fl + 1.0;
    return k * q;
}

double oracle_round_bf16(float x)
{
    double a = fabs((double)x);
    double r = round_to_format(a, 8, -126);
    return x < 0 ? -r : r;
}

double oracle_round_fp16(float x)
{
    double a = fabs((double)x);
    double r = round_to_format(a, 11, -14);
    if (r > 65504.0) r = INFINITY;
    return x < 0 ? -r : r;
}

double oracle_round_e4m3(float x)
{
    double a = fabs((double)x);
    double r = round_to_format(a, 4, -6);
    if (r > 448.0) r = 448.0;
    return x < 0 ? -r : r;
}

/* Operand model of a reduced-precision MelT projection.
 *   prec 1 (BF16) / 2 (FP16): every frame sample and every basis entry (first rounded
 *       FP64 -> FP32) is rounded to the format; products and sums are exact.
 *   prec 3 (FP8 E4M3 with per-frame and per-row scaling): frame t is scaled by
 *       s_t = 448 / max_n |x_t[n]| and basis row j by r_j = 448 / max_n |W[j,n]|, both
 *       computed in FP32 (so that the rounding decision matches an FP32 computation),
 *       the scaled FP32 values are rounded to E4M3, and the exact product sum is divided
 *       by s_t r_j.  A silent frame (max 0) uses s_t = 1.
 *   prec 4 (BF16x3): x = xh + xl, W = Wh + Wl with xh = bf16(x), xl = bf16(x - xh) (FP32
 *       difference, exact) and the same for W; the product is xh Wh + xh Wl + xl Wh.
 *   prec 5 (FP16x3): as prec 4 with binary16 parts, the frame samples first multiplied by
 *       2^10 in FP32 (exact) and the product sum divided by 2^10; a sample whose scaled
 *       value exceeds binary16's range becomes infinite.
 *   prec 6 (FP8 E4M3 with 32-sample block scales): each clip is cut into blocks of 32
 *       samples from its first sample (samples past the clip end count as 0); block b gets
 *       the exponent e_b of block_exponent(max |x| over the block), every sample of the
 *       block is multiplied by 2^e_b in FP32 and rounded to E4M3, and a frame uses the
 *       values q 2^-e_b of its samples' blocks.  The basis is rounded as for prec 3 and the
 *       exact product sum divided by r_j.
 * Wr, Wi are the FP64 basis; out / R / I as in oracle_melt_forward_basis.  Returns T. */
/* The largest integer e with 2^e m <= 448 (the largest finite E4M3 value), m > 0, limited
 * to [-127, 127] (the exponents an E8M0 scale can undo); 0 for m = 0.  Found by stepping e
 * from 0, each comparison exact in double. */
static int block_exponent(double m)
{
    if (m == 0.0) return 0;
    int e = 0;
    while (e > -127 && ldexp(m, e) > 448.0) --e;
    while (e < 127 && ldexp(m, e + 1) <= 448.0) ++e;
    return e;
}

int oracle_block_exponent(float m) { return block_exponent(fabs((double)m)); }

int64_t oracle_melt_forward_quant(const float *wave, const int64_t *clip_off, int n_clips,
                                  int n_fft, int hop, const double *Wr, const double *Wi,
                                  int n_freq, int prec, int out_kind, double eps, double *out,
                                  double *R_out, double *I_out)
{
    int64_t *st;
    int64_t T = frame_starts(clip_off, n_clips, n_fft, hop, &st);
    size_t nb = (size_t)n_freq * (size_t)n_fft;
    /* basis as FP32 first, then per-format hi/lo (lo used only by BF16x3) and row scales */
    double *Bh = (double *)malloc(sizeof(double) * 2 * nb);
    double *Bl = (double *)malloc(sizeof(double) * 2 * nb);
    float *rs = (float *)malloc(sizeof(float) * 2 * (size_t)n_freq);
    for (int j = 0; j < 2 * n_freq; ++j) {
        const double *src = (j < n_freq) ? Wr + (size_t)j * n_fft : Wi + (size_t)(j - n_freq) * n_fft;
        float mx = 0.0f;
        for (int n = 0; n < n_fft; ++n) {
            float v = (float)src[n];
            if (fabsf(v) > mx) mx = fabsf(v);
        }
        volatile float sc = (mx > 0.0f) ? 448.0f / mx : 1.0f;
        rs[j] = sc;
        for (int n = 0; n < n_fft; ++n) {
            float v = (float)src[n];
            double h = 0.0, l = 0.0;
            if (prec == 1) h = oracle_round_bf16(v);
            else if (prec == 2) h = oracle_round_fp16(v);
            else if (prec == 3 || prec == 6) { volatile float vs = v * rs[j]; h = oracle_round_e4m3(vs); }
            else if (prec == 5) { h = oracle_round_fp16(v); l = oracle_round_fp16((float)(v - (float)h)); }
            else { h = oracle_round_bf16(v); l = oracle_round_bf16((float)(v - (float)h)); }
            Bh[(size_t)j * n_fft + n] = h;
            Bl[(size_t)j * n_fft + n] = l;
        }
    }
    /* prec 6: the block exponent of every sample of every clip */
    int *bexp = NULL;
    if (prec == 6) {
        int64_t total = n_clips > 0 ? clip_off[n_clips] : 0;
        bexp = (int *)malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
        for (int c = 0; c < n_clips; ++c)
            for (int64_t b0 = clip_off[c]; b0 < clip_off[c + 1]; b0 += 32) {
                int64_t b1 = b0 + 32 < clip_off[c + 1] ? b0 + 32 : clip_off[c + 1];
                double mx = 0.0;
                for (int64_t i = b0; i < b1; ++i) if (fabs((double)wave[i]) > mx) mx = fabs((double)wave[i]);
                int e = block_exponent(mx);
                for (int64_t i = b0; i < b1; ++i) bexp[i] = e;
            }
    }
#pragma omp parallel
    {
        double *xh = (double *)malloc(sizeof(double) * (size_t)n_fft);
        double *xl = (double *)malloc(sizeof(double) * (size_t)n_fft);
#pragma omp for schedule(static)
        for (int64_t t = 0; t < T; ++t) {
            const float *x = wave + st[t];
            float s_t = 1.0f;
            if (prec == 3) {
                float mx = 0.0f;
                for (int n = 0; n < n_fft; ++n) if (fabsf(x[n]) > mx) mx = fabsf(x[n]);
                volatile float sc = (mx > 0.0f) ? 448.0f / mx : 1.0f;
                s_t = sc;
            }
            for (int n = 0; n < n_fft; ++n) {
                float v = x[n];
                if (prec == 1) { xh[n] = oracle_round_bf16(v); xl[n] = 0.0; }
                else if (prec == 2) { xh[n] = oracle_round_fp16(v); xl[n] = 0.0; }
                else if (prec == 3) { volatile float vs = v * s_t; xh[n] = oracle_round_e4m3(vs); xl[n] = 0.0; }
                else if (prec == 6) {
                    int e = bexp[st[t] + n];
                    volatile float vs = ldexpf(v, e);
                    xh[n] = ldexp(oracle_round_e4m3(vs), -e);
                    xl[n] = 0.0;
                }
                else if (prec == 5) {
                    volatile float vs = v * 1024.0f;
                    xh[n] = oracle_round_fp16(vs);
                    xl[n] = isfinite(xh[n]) ? oracle_round_fp16((float)(vs - (float)xh[n])) : 0.0;
                }
                else { xh[n] = oracle_round_bf16(v); xl[n] = oracle_round_bf16((float)(v - (float)xh[n])); }
            }
            for (int m = 0; m < n_freq; ++m) {
                double acc[2];
                for (int h = 0; h < 2; ++h) {
                    int j = h * n_freq + m;
                    const double *bh = Bh + (size_t)j * n_fft, *bl = Bl + (size_t)j * n_fft;
                    double a = 0.0;
                    for (int n = 0; n < n_fft; ++n) {
                        a += xh[n] * bh[n];
                        if (prec == 4 || prec == 5) a += xh[n] * bl[n] + xl[n] * bh[n];
                    }
                    if (prec == 3) a /= (double)s_t * (double)rs[j];
                    if (prec == 6) a /= (double)rs[j];
                    if (prec == 5) a /= 1024.0;
                    acc[h] = a;
                }
                out[t * n_freq + m] = output_map(acc[0] * acc[0] + acc[1] * acc[1], out_kind, eps);
                if (R_out) R_out[t * n_freq + m] = acc[0];
                if (I_out) I_out[t * n_freq + m] = acc[1];
            }
        }
        free(xh); free(xl);
    }
    free(st); free(Bh); free(Bl); free(rs); free(bexp);
    return T;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
