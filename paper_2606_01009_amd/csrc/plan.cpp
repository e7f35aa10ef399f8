// Host-side plan construction: Mel analysis frequencies, the window-folded cos/sin basis in
// FP64, the hop-block geometry of the GEMM and the comparator's sparse filterbank.
//
// Methodology, Eq. (mel_scale) and Eq. (inverse_mel): the M analysis frequencies are the
// centres of the triangular Mel filterbank, uniformly spaced in Mel between fmin and fmax.
// Eq. (dmp_weights): W^(r)[m,n] = w[n] cos(2 pi f_m n / sr), W^(i)[m,n] = w[n] sin(...).
#include <cmath>
#include <cstring>

#include "melt_internal.h"

namespace melt {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// HTK: 2595 log10(1 + f/700); Slaney: 3 Mel per 200 Hz below 1 kHz, then logarithmic
// with 27 Mel per factor 6.4.
double to_mel(double hz, int formula) {
    if (formula == MELT_MEL_HTK) return 2595.0 * std::log10(1.0 + hz / 700.0);
    const double lin = 200.0 / 3.0, brk = 1000.0, step = std::log(6.4) / 27.0;
    return hz < brk ? hz / lin : brk / lin + std::log(hz / brk) / step;
}

double to_hz(double mel, int formula) {
    if (formula == MELT_MEL_HTK) return 700.0 * (std::pow(10.0, mel / 2595.0) - 1.0);
    const double lin = 200.0 / 3.0, brk = 1000.0, step = std::log(6.4) / 27.0;
    const double brk_mel = brk / lin;
    return mel < brk_mel ? mel * lin : brk * std::exp(step * (mel - brk_mel));
}

// (M+2)-point grid uniform in Mel, in Hz
std::vector<double> mel_grid(const melt_config &c) {
    const double a = to_mel(c.fmin, c.mel_formula), b = to_mel(c.fmax, c.mel_formula);
    std::vector<double> g(c.n_mels + 2);
    for (int i = 0; i <= c.n_mels + 1; ++i)
        g[i] = to_hz(a + (b - a) * double(i) / double(c.n_mels + 1), c.mel_formula);
    return g;
}

double window_at(int n, int N, int kind) {
    if (kind == MELT_WIN_RECT || N == 1) return 1.0;
    const double den = (kind == MELT_WIN_HANN_SYMMETRIC) ? double(N - 1) : double(N);
    return 0.5 - 0.5 * std::cos(kTwoPi * double(n) / den);
}

// Phase of f * n / sr in cycles, reduced to [0, 1) without losing bits: the product f*n is
// split exactly into p + e (Dekker/FMA two-product), p is reduced modulo sr exactly by
// fmod, and e is added back before dividing by sr.
double phase_cycles(double f, int n, double sr) {
    const double p = f * double(n);
    const double e = std::fma(f, double(n), -p);
    double r = std::fmod(p, sr) + e;
    if (r < 0.0) r += sr;
    if (r >= sr) r -= sr;
    return r / sr;
}

}  // namespace

void mel_frequencies(const melt_config &c, std::vector<double> &f) {
    f.assign(c.n_mels, 0.0);
    if (c.placement == MELT_PLACE_FILTER_CENTRES) {
        std::vector<double> g = mel_grid(c);
        for (int m = 0; m < c.n_mels; ++m) f[m] = g[m + 1];
    } else {
        const double a = to_mel(c.fmin, c.mel_formula), b = to_mel(c.fmax, c.mel_formula);
        for (int m = 0; m < c.n_mels; ++m)
            f[m] = to_hz(c.n_mels == 1 ? a : a + (b - a) * double(m) / double(c.n_mels - 1),
                         c.mel_formula);
    }
}

Geometry make_geometry(int N, int H, int group) {
    Geometry g;
    g.N = N;
    g.H = H;
    g.J = (N + H - 1) / H;
    g.group = group;
    g.Hp = ((std::min(N, H) + group - 1) / group) * group;
    g.n_groups = 0;
    for (int j = 0; j < g.J; ++j) {
        const int Lj = std::min(H, N - j * H);
        const int gj = (Lj + group - 1) / group;
        for (int q = 0; q < gj; ++q) {
            g.seg_of_group.push_back(j);
            g.col_of_group.push_back(q * group);
        }
        g.n_groups += gj;
    }
    return g;
}

// FP64 basis in the paper's stacked order: rows 0..M-1 cosines, rows M..2M-1 sines.
melt_status plan_build_host(Plan &p) {
    const melt_config &c = p.cfg;
    p.M = c.n_mels;
    p.N = c.n_fft;
    p.H = c.hop;
    p.row_tiles = (p.M + 15) / 16;
    mel_frequencies(c, p.freqs);
    p.basis64.assign(size_t(2) * p.M * p.N, 0.0);
    for (int m = 0; m < p.M; ++m)
        for (int n = 0; n < p.N; ++n) {
            const double w = window_at(n, p.N, c.window);
            const double ph = kTwoPi * phase_cycles(p.freqs[m], n, c.sample_rate);
            p.basis64[size_t(m) * p.N + n] = w * std::cos(ph);
            p.basis64[size_t(p.M + m) * p.N + n] = w * std::sin(ph);
        }
    p.geo32 = make_geometry(p.N, p.H, 8);
    p.geo16 = make_geometry(p.N, p.H, 16);
    p.geo8 = make_geometry(p.N, p.H, 64);
    // The staging helpers write every column c < H of a hop-block row at r * S + c, and the
    // LDS row stride S is at least the padded row length Hp: each row must cover the hop.
    for (const Geometry *g : {&p.geo32, &p.geo16, &p.geo8})
        if (g->Hp < p.H) return set_error(MELT_E_UNSUPPORTED, "hop-block row shorter than the hop (hop > n_fft)");
    return MELT_OK;
}

// Sparse triangular filterbank of the comparator on bins f_k = k sr / N, k = 0..N/2: the
// nonzero run of each filter, as (first bin, weights).  Peak-1 triangles, or unit area.
void build_filterbank(const melt_config &c, std::vector<int> &start, std::vector<int> &off,
                      std::vector<float> &w) {
    const std::vector<double> g = mel_grid(c);
    const int nb = c.n_fft / 2 + 1;
    start.assign(c.n_mels, 0);
    off.assign(c.n_mels + 1, 0);
    w.clear();
    for (int m = 0; m < c.n_mels; ++m) {
        const double lo = g[m], ce = g[m + 1], hi = g[m + 2];
        const double scale = (c.fb_norm == MELT_FB_NORM_SLANEY) ? 2.0 / (hi - lo) : 1.0;
        int first = -1;
        std::vector<float> run;
        for (int k = 0; k < nb; ++k) {
            const double fk = double(k) * c.sample_rate / double(c.n_fft);
            const double up = (fk - lo) / (ce - lo), down = (hi - fk) / (hi - ce);
            const double v = std::max(0.0, std::min(up, down)) * scale;
            if (v > 0.0) {
                if (first < 0) first = k;
                // the support of a triangle is one contiguous run of bins
                while (first + int(run.size()) < k) run.push_back(0.0f);
                run.push_back(float(v));
            }
        }
        start[m] = first < 0 ? 0 : first;
        off[m] = int(w.size());
        w.insert(w.end(), run.begin(), run.end());
    }
    off[c.n_mels] = int(w.size());
}

}  // namespace melt
