// Conventional STFT + triangular Mel filterbank on gfx950 (the comparator MelT replaces):
// per frame, window, N-point real DFT by a hand-written mixed-radix FFT, power on the
// uniform bins k = 0..N/2, sparse triangular Mel filters, log (Methodology: power values on
// uniformly spaced FFT bins aggregated through non-negative triangular weights; cost
// O(N log N + nnz(F_Mel)), Eq. complexity_conv).  Everything after the waveform read stays
// on chip; only the [T, M] output goes back to HBM.
//
// Two real frames a, b share one complex FFT of z = a + i b; the spectra separate as
// A[k] = (Z[k] + conj Z[N-k]) / 2 and B[k] = (Z[k] - conj Z[N-k]) / (2i).  The complex
// FFT uses the four-step split N = N1 N2 (n = N2 n1 + n2, k = k1 + N1 k2):
//   1. for each n2: N1-point DFT over n1, in registers of one thread
//   2. multiply by exp(-2 pi i n2 k1 / N)
//   3. for each k1: N2-point DFT over n2, in registers of one thread (after an LDS transpose)
// The small DFTs are fully unrolled Cooley-Tukey recursions with radix 2, 3, 4, 5
// butterflies whose twiddles are compile-time constants.
#include <cmath>

#include "melt_internal.h"

namespace melt {

typedef float sm_f32x4 __attribute__((ext_vector_type(4)));

void build_filterbank(const melt_config &c, std::vector<int> &start, std::vector<int> &off, std::vector<float> &w);

// ------------------------------------------------------------------ compile-time cos/sin

// cos and sin of 2 pi a / b for integers, in double precision, as constant expressions:
// quadrant reduction in integers, then Taylor series on an angle of at most pi/4.
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double ct_sin_small(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 14; ++i) {
        term *= -x2 / double((2 * i) * (2 * i + 1));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos_small(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 14; ++i) {
        term *= -x2 / double((2 * i - 1) * (2 * i));
        sum += term;
    }
    return sum;
}
struct CtCis {
    double c, s;
};
constexpr CtCis ct_cis(long a, long b) {
    a %= b;
    if (a < 0) a += b;
    const long q = (4 * a) / b;          // quadrant
    const long r = 4 * a - q * b;        // angle within the quadrant = (pi/2) r / b
    double c = 0, s = 0;
    if (2 * r <= b) {
        const double t = 0.5 * kPiD * double(r) / double(b);
        c = ct_cos_small(t);
        s = ct_sin_small(t);
    } else {
        const double t = 0.5 * kPiD * double(b - r) / double(b);
        c = ct_sin_small(t);
        s = ct_cos_small(t);
    }
    switch (q) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
    }
}

// ------------------------------------------------------------------ complex helpers

// 8-byte aligned, so that moving one value to or from LDS is one 64-bit access with an
// immediate offset
struct alignas(8) cf {
    float x, y;
};
__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cf mul_mi(cf a) { return {a.y, -a.x}; }   // -i a
__device__ __forceinline__ cf mul_pi(cf a) { return {-a.y, a.x}; }   // +i a
__device__ __forceinline__ cf cscale(cf a, float s) { return {a.x * s, a.y * s}; }

// multiply by exp(-2 pi i num / den) with the constant folded; quarter turns are exact
template <long NUM, long DEN>
__device__ __forceinline__ cf twiddle_const(cf a) {
    constexpr long n = ((NUM % DEN) + DEN) % DEN;
    if constexpr (n == 0) return a;
    else if constexpr (4 * n == DEN) return mul_mi(a);
    else if constexpr (2 * n == DEN) return {-a.x, -a.y};
    else if constexpr (4 * n == 3 * DEN) return mul_pi(a);
    else {
        constexpr CtCis w = ct_cis(n, DEN);
        constexpr float c = (float)w.c, s = (float)(-w.s);
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

// ------------------------------------------------------------------ small DFTs in registers
// Forward DFT X[k] = sum_n x[n] exp(-2 pi i n k / L), in place, natural order.  Sizes with
// two coprime factors use the prime-factor (Good-Thomas) mapping, which needs no twiddle
// multiplications between its two stages; prime powers use Cooley-Tukey.  Every index map
// is a compile-time register renaming.

constexpr int ct_part(int L, int p) {   // largest power of p dividing L
    int a = 1;
    while (L % p == 0) {
        L /= p;
        a *= p;
    }
    return a;
}
// first factor A of a coprime split L = A B (the power of 2, else of 3, in L), 0 if none
constexpr int pfa_factor(int L) {
    return (ct_part(L, 2) > 1 && ct_part(L, 2) < L) ? ct_part(L, 2)
           : (ct_part(L, 3) > 1 && ct_part(L, 3) < L) ? ct_part(L, 3) : 0;
}
constexpr int ct_inverse(int a, int m) {   // a^-1 mod m (gcd(a, m) = 1)
    for (int i = 1; i < m; ++i)
        if ((a * i) % m == 1) return i;
    return 1;
}

template <int L>
struct Radix {
    static constexpr int value = (L % 4 == 0 && L != 4) ? 4 : (L % 2 == 0 && L != 2) ? 2
                                 : (L % 3 == 0 && L != 3) ? 3 : (L % 5 == 0 && L != 5) ? 5 : L;
};

template <int L, int A = pfa_factor(L)>
struct DFT;

template <>
struct DFT<1, 0> {
    __device__ __forceinline__ static void run(cf *) {}
};
template <>
struct DFT<2, 0> {
    __device__ __forceinline__ static void run(cf *x) {
        const cf a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};
template <>
struct DFT<3, 0> {
    __device__ __forceinline__ static void run(cf *x) {
        const float s = 0.86602540378443864676f;   // sin(2 pi / 3)
        const cf a = cadd(x[1], x[2]), b = csub(x[1], x[2]);
        const cf t = {x[0].x - 0.5f * a.x, x[0].y - 0.5f * a.y};
        x[0] = cadd(x[0], a);
        const cf u = mul_mi(cscale(b, s));
        x[1] = cadd(t, u);
        x[2] = csub(t, u);
    }
};
template <>
struct DFT<4, 0> {
    __device__ __forceinline__ static void run(cf *x) {
        const cf a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const cf c = cadd(x[1], x[3]), d = mul_mi(csub(x[1], x[3]));
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, d);
        x[3] = csub(b, d);
    }
};
template <>
struct DFT<5, 0> {
    __device__ __forceinline__ static void run(cf *x) {
        constexpr CtCis w1 = ct_cis(1, 5), w2 = ct_cis(2, 5);
        const float c1 = (float)w1.c, s1 = (float)w1.s, c2 = (float)w2.c, s2 = (float)w2.s;
        const cf a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
        const cf a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
        const cf x0 = x[0];
        const cf t1 = {x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
        const cf t2 = {x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
        const cf u1 = mul_mi(cf{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
        const cf u2 = mul_mi(cf{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
        x[0] = cadd(x0, cadd(a1, a2));
        x[1] = cadd(t1, u1);
        x[4] = csub(t1, u1);
        x[2] = cadd(t2, u2);
        x[3] = csub(t2, u2);
    }
};

// Good-Thomas, L = A B with gcd(A, B) = 1: input n = (B a + A b) mod L, then B-point DFTs over
// b for each a, then A-point DFTs over a for each output index kb; output k is the residue
// pair (ka, kb) by the Chinese remainder theorem, k = (ka eA + kb eB) mod L.
template <int L, int A>
struct DFT {
    static constexpr int B = L / A;
    static constexpr int eA = B * ct_inverse(B % A, A);   // = 1 mod A, 0 mod B
    static constexpr int eB = A * ct_inverse(A % B, B);   // = 0 mod A, 1 mod B
    static_assert(A * B == L && A > 1 && B > 1, "coprime split");
    __device__ __forceinline__ static void run(cf *x) {
        cf t[A][B];
#pragma unroll
        for (int a = 0; a < A; ++a)
#pragma unroll
            for (int b = 0; b < B; ++b) t[a][b] = x[(B * a + A * b) % L];
#pragma unroll
        for (int a = 0; a < A; ++a) DFT<B>::run(t[a]);
#pragma unroll
        for (int kb = 0; kb < B; ++kb) {
            cf u[A];
#pragma unroll
            for (int a = 0; a < A; ++a) u[a] = t[a][kb];
            DFT<A>::run(u);
#pragma unroll
            for (int ka = 0; ka < A; ++ka) x[(ka * eA + kb * eB) % L] = u[ka];
        }
    }
};

// Cooley-Tukey for prime powers: L = R m, decimation in time
template <int L>
struct DFT<L, 0> {
    static constexpr int R = Radix<L>::value;
    static constexpr int Msub = L / R;
    static_assert(R * Msub == L && R <= 5, "DFT size must factor into 2, 3, 4, 5");

    template <int K>
    __device__ __forceinline__ static void combine(cf (&sub)[R][Msub], cf *x) {
        if constexpr (K < Msub) {
            cf t[R];
            apply<K, 0>(sub, t);
            DFT<R>::run(t);
#pragma unroll
            for (int q = 0; q < R; ++q) x[K + Msub * q] = t[q];
            combine<K + 1>(sub, x);
        }
    }
    template <int K, int J>
    __device__ __forceinline__ static void apply(cf (&sub)[R][Msub], cf (&t)[R]) {
        if constexpr (J < R) {
            t[J] = twiddle_const<(long)J * K, L>(sub[J][K]);
            apply<K, J + 1>(sub, t);
        }
    }
    __device__ __forceinline__ static void run(cf *x) {
        cf sub[R][Msub];
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int i = 0; i < Msub; ++i) sub[j][i] = x[R * i + j];
#pragma unroll
        for (int j = 0; j < R; ++j) DFT<Msub>::run(sub[j]);
        combine<0>(sub, x);
    }
};

// ------------------------------------------------------------------ kernel

struct StftArgs {
    const float *wave;
    const Chunk *chunks;
    const int *n_chunks;
    float *out;
    int64_t n_frames;
    const float *window;      // [N]
    const float2 *twiddle;    // [N], exp(-2 pi i j / N)
    const float *fb_w;        // concatenated filter weights
    const int *fb_start;      // [M] first bin
    const int *fb_off;        // [M+1] offsets into fb_w
    int fb_nnz;
    int M, H;
    float eps;
};

// output map of kind KIND (a melt_output); ln from the hardware base-2 logarithm, whose
// argument v + eps >= eps is a normal FP32 number
template <int KIND>
__device__ __forceinline__ float stft_out_map(float v, float eps) {
    if constexpr (KIND <= MELT_OUT_LOG_MAGNITUDE) return __builtin_amdgcn_logf(v + eps) * 0.693147180559945309f;
    else return v;
}

// Orders this wave's LDS traffic: everything before is complete and visible to every lane
// of the wave before anything after it.  Only lanes of one wave share a buffer, so no
// workgroup barrier is needed.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave owns FPW = 64 / TPF complex FFTs (2 FPW frames) per sub-task and runs the whole
// pipeline for them with wave-local LDS only; a chunk is up to SUB sub-tasks; the workgroup's
// waves take chunks independently (persistent loop over the chunk table).  The wave index,
// chunk and sub-task are wave-uniform (scalar registers), so the waveform is read through a
// buffer descriptor held in scalar registers whose bound zero-fills reads past the clip.
// The samples of the next sub-task are loaded during the current one's power and filter
// passes when PREFETCH (their registers fit beside those passes).
template <int N1, int N2, int WAVES, int SUB, int WPE, int KIND>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(WPE))) void k_stft_mel(StftArgs a) {
    constexpr int N = N1 * N2;
    constexpr int NB = N / 2 + 1;
    constexpr int TPF = N1 > N2 ? N1 : N2;        // lanes per FFT
    constexpr int FPW = 64 / TPF;                 // FFTs per wave per sub-task
    constexpr int LDB = N2 + 1;                   // padded row of the [k1][n2] layout
    constexpr int BUF = (N1 * LDB > N ? N1 * LDB : N);
    constexpr int JT = (NB + 63) / 64;            // bins per lane in the power pass
    constexpr bool MAG = (KIND == MELT_OUT_LOG_MAGNITUDE || KIND == MELT_OUT_MAGNITUDE);
    constexpr bool PREFETCH = N1 * N2 < 1200 && N1 != 20;
    // power spectra interleaved by bin: bin k holds the FPW spectra of half 0, then those of
    // half 1, each half padded to FP4 floats, so a step-5 lane reads its FPW values of one bin
    // in one access (16 bytes for FPW 3 and 4)
    constexpr int FP4 = FPW == 3 ? 4 : FPW;
    constexpr int PST = 2 * FP4;                  // floats per bin
    static_assert(NB * PST <= 2 * FPW * BUF, "power spectra must fit in the FFT rows");
    // LDS: the twiddles [k1][n2] in an array of their own, so that the compiler knows the
    // stores into the FFT rows cannot change them (in one array with the rows, every twiddle
    // read of step 1 waited for the store before it); then, dynamic, every wave's FFT rows,
    // the window, the filter weights (pre-scaled, see below), first bins and offsets
    __shared__ cf tw[N];
    extern __shared__ float smem[];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    cf *buf = reinterpret_cast<cf *>(smem) + wid * FPW * BUF;
    float *wl = reinterpret_cast<float *>(reinterpret_cast<cf *>(smem) + WAVES * FPW * BUF);
    float *fbw = wl + N;
    int *fbs = reinterpret_cast<int *>(fbw + a.fb_nnz);
    int *fbo = fbs + a.M;
    // the wave's 2 FPW power spectra [NB][2][FP4] are written over its FFT rows once read
    float *pw = reinterpret_cast<float *>(buf);
    for (int i = threadIdx.x; i < N; i += 64 * WAVES) {
        const int k1 = i / N2, n2 = i - k1 * N2;
        const float2 t = a.twiddle[(n2 * k1) % N];
        tw[i] = cf{t.x, t.y};
        wl[i] = a.window[i];
    }
    // The spectra below are 4 |X_k|^2 (2 |X_k| for the magnitude kinds): the halving of the
    // two-for-one separation moves into the weights, exactly (a power of two).
    for (int i = threadIdx.x; i < a.fb_nnz; i += 64 * WAVES) fbw[i] = a.fb_w[i] * (MAG ? 0.5f : 0.25f);
    for (int i = threadIdx.x; i < a.M; i += 64 * WAVES) fbs[i] = a.fb_start[i];
    for (int i = threadIdx.x; i <= a.M; i += 64 * WAVES) fbo[i] = a.fb_off[i];
    __syncthreads();

    const int p1 = lane / TPF, n2 = lane - p1 * TPF;                  // step-1 role
    const bool act1 = p1 < FPW && n2 < N2;
    const int p3 = lane / TPF, k1 = lane - p3 * TPF;                  // step-3 role
    const bool act3 = p3 < FPW && k1 < N1;

    const int nch = *a.n_chunks;
    const int nw = gridDim.x * WAVES;
    int c = blockIdx.x * WAVES + wid;
    if (c >= nch) return;
    // samples of one sub-task for this lane: frames 2 p1 and 2 p1 + 1 at points N2 n1 + n2
    float xa[N1], xb[N1];
    auto load = [&](const Chunk &ch, int sub) {
        const int64_t lim = ch.sample_end - ch.sample_start;
        const int records = (int)(lim < (int64_t(1) << 29) ? lim * 4 : (int64_t(1) << 31) - 4);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(a.wave + ch.sample_start), (short)0, records, 0x00020000);
        const int fa = 2 * FPW * sub + 2 * p1;
        const int va = (fa * a.H + n2) * 4, vb = va + a.H * 4;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            xa[n1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, va, N2 * n1 * 4, 0));
            xb[n1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vb, N2 * n1 * 4, 0));
        }
    };
    Chunk ch = a.chunks[c];
    int sub = 0;
    if (PREFETCH) load(ch, 0);
    for (;;) {
        const Chunk cur = ch;
        const int cur_sub = sub;
        if (!PREFETCH) load(cur, cur_sub);
        // advance to the next sub-task (this chunk or the wave's next chunk)
        ++sub;
        bool more = true;
        if (2 * FPW * sub >= cur.n_frames || sub >= SUB) {
            sub = 0;
            c += nw;
            more = c < nch;
            if (more) ch = a.chunks[c];
        }
        // step 1: window, N1-point DFTs over n1, four-step twiddle, store as [k1][n2]
        cf z[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            const float wv = act1 ? wl[N2 * n1 + n2] : 0.0f;
            z[n1] = cf{xa[n1] * wv, xb[n1] * wv};
        }
        DFT<N1>::run(z);
        if (act1) {
            cf *row1 = buf + p1 * BUF + n2;
#pragma unroll
            for (int q = 0; q < N1; ++q) row1[q * LDB] = cmul(z[q], tw[q * N2 + n2]);
        }
        wave_sync();
        // step 3: N2-point DFTs over n2, natural order k = k1 + N1 k2
        {
            cf y[N2];
            cf *row3 = buf + p3 * BUF;
            if (act3) {
#pragma unroll
                for (int q = 0; q < N2; ++q) y[q] = row3[k1 * LDB + q];
            }
            wave_sync();
            if (act3) {
                DFT<N2>::run(y);
#pragma unroll
                for (int q = 0; q < N2; ++q) row3[k1 + N1 * q] = y[q];
            }
        }
        wave_sync();
        // the next sub-task's samples load during the power and filter passes
        if (PREFETCH && more) load(ch, sub);
        // step 4: separate the two real spectra of each FFT and form 4 |X_k|^2 (2 |X_k|) on
        // bins k = lane + 64 j <= N/2: A = (Z[k] + conj Z[N-k]) / 2, B = (Z[k] - conj Z[N-k]) / (2i).
        // Every value is read before the wave writes the spectra over the FFT rows.
        {
            float pa[FPW][JT], pb[FPW][JT];
#pragma unroll
            for (int j = 0; j < JT; ++j) {
                const int k = lane + 64 * j;
                const int kn = (k == 0) ? 0 : N - k;
#pragma unroll
                for (int p = 0; p < FPW; ++p) {
                    pa[p][j] = pb[p][j] = 0.0f;
                    if (64 * j + 64 <= NB || k < NB) {
                        const cf zk = buf[p * BUF + k], zn = buf[p * BUF + kn];
                        const float s1 = zk.x + zn.x, s2 = zk.y - zn.y;
                        const float s3 = zk.y + zn.y, s4 = zk.x - zn.x;
                        pa[p][j] = s1 * s1 + s2 * s2;
                        pb[p][j] = s3 * s3 + s4 * s4;
                        if constexpr (MAG) {
                            pa[p][j] = __builtin_sqrtf(pa[p][j]);
                            pb[p][j] = __builtin_sqrtf(pb[p][j]);
                        }
                    }
                }
            }
            wave_sync();
#pragma unroll
            for (int j = 0; j < JT; ++j) {
                const int k = lane + 64 * j;
                if (64 * j + 64 <= NB || k < NB) {
                    // spectrum q = 2 p (A of FFT p) or 2 p + 1 (B); half h holds q = h FPW + f
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int f = 0; f < FPW; ++f) {
                            const int q = h * FPW + f;
                            v[f] = (q & 1) ? pb[q >> 1][j] : pa[q >> 1][j];
                        }
                        float *d = pw + k * PST + h * FP4;
                        if constexpr (FP4 == 4) {
                            *reinterpret_cast<sm_f32x4 *>(d) = sm_f32x4{v[0], v[1], v[2], v[3]};
                        } else {
#pragma unroll
                            for (int f = 0; f < FPW; ++f) d[f] = v[f];
                        }
                    }
                }
            }
        }
        wave_sync();
        // step 5: one lane per (Mel filter m, half h of the 2 FPW spectra), m = t / 2, so the
        // filters of one pass over the lanes have neighbouring widths; each weight read serves
        // FPW spectra; sums in increasing k; output map; store
        {
            const int f0 = 2 * FPW * cur_sub;
            for (int t = lane; t < 2 * a.M; t += 64) {
                const int m = t >> 1, h = t & 1;
                const float *ps = pw + fbs[m] * PST + h * FP4;
                const int j0 = fbo[m], nj = fbo[m + 1] - j0;
                const float *wj = fbw + j0;
                float acc[FPW];
#pragma unroll
                for (int f = 0; f < FPW; ++f) acc[f] = 0.0f;
                // the FPW values of bin fbs[m] + j
                auto bin = [&](int j, float (&x)[FPW]) {
                    if constexpr (FP4 == 4) {
                        const sm_f32x4 v = *reinterpret_cast<const sm_f32x4 *>(ps + j * PST);
#pragma unroll
                        for (int f = 0; f < FPW; ++f) x[f] = v[f];
                    } else {
#pragma unroll
                        for (int f = 0; f < FPW; ++f) x[f] = ps[j * PST + f];
                    }
                };
                int j = 0;
                for (; j + 1 < nj; j += 2) {
                    const float w0 = wj[j], w1 = wj[j + 1];
                    float x0[FPW], x1[FPW];
                    bin(j, x0);
                    bin(j + 1, x1);
#pragma unroll
                    for (int f = 0; f < FPW; ++f) {
                        acc[f] += w0 * x0[f];
                        acc[f] += w1 * x1[f];
                    }
                }
                if (j < nj) {
                    const float w0 = wj[j];
                    float x0[FPW];
                    bin(j, x0);
#pragma unroll
                    for (int f = 0; f < FPW; ++f) acc[f] += w0 * x0[f];
                }
#pragma unroll
                for (int f = 0; f < FPW; ++f) {
                    const int fa = f0 + h * FPW + f;
                    const int64_t row = cur.out_row + fa;
                    if (fa < cur.n_frames && row < a.n_frames)
                        a.out[row * a.M + m] = stft_out_map<KIND>(acc[f], a.eps);
                }
            }
        }
        wave_sync();
        if (!more) break;
    }
}

// ------------------------------------------------------------------ host side

namespace {

struct StftShape {
    int N1, N2, FPW, SUB;
};

bool stft_shape(int N, StftShape &s) {
    switch (N) {
    case 400: s = {20, 20, 3, 8}; return true;
    case 512: s = {16, 32, 2, 8}; return true;
    case 1024: s = {32, 32, 2, 8}; return true;
    case 256: s = {16, 16, 4, 8}; return true;
    case 1200: s = {30, 40, 1, 16}; return true;
    default: return false;
    }
}

constexpr int kStftWaves = 4;

size_t stft_lds_bytes(const StftShape &s, int M, int nnz) {
    const int N = s.N1 * s.N2;
    const int BUF = std::max(s.N1 * (s.N2 + 1), N);
    // twiddles (static) and FFT rows (the power spectra reuse the rows), window, weights,
    // starts, offsets
    return (size_t)N * 8 + (size_t)kStftWaves * s.FPW * BUF * 8 + (size_t)N * 4 + (size_t)nnz * 4 +
           (size_t)(2 * M + 1) * 4;
}

// waves per SIMD the kernel's registers are sized for: 3 (LDS allows three workgroups per CU),
// 1 for the 1200-point shape (its 40-point register DFTs need the whole register file)
template <int N1, int N2, int SUB, int KIND>
melt_status launch_kind(const StftArgs &a, size_t lds, int grid, hipStream_t s) {
    constexpr int WPE = (N1 * N2 >= 1200) ? 1 : 3;
    constexpr size_t kStatic = (size_t)N1 * N2 * sizeof(cf);   // the twiddle array
    (void)hipFuncSetAttribute((const void *)k_stft_mel<N1, N2, kStftWaves, SUB, WPE, KIND>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - kStatic));
    k_stft_mel<N1, N2, kStftWaves, SUB, WPE, KIND><<<grid, 64 * kStftWaves, lds - kStatic, s>>>(a);
    return hip_check(hipGetLastError(), "stft_mel launch");
}

template <int N1, int N2, int SUB>
melt_status launch_shape(const StftArgs &a, int kind, size_t lds, int grid, hipStream_t s) {
    switch (kind) {
    case MELT_OUT_LOG_POWER: return launch_kind<N1, N2, SUB, MELT_OUT_LOG_POWER>(a, lds, grid, s);
    case MELT_OUT_LOG_MAGNITUDE: return launch_kind<N1, N2, SUB, MELT_OUT_LOG_MAGNITUDE>(a, lds, grid, s);
    case MELT_OUT_POWER: return launch_kind<N1, N2, SUB, MELT_OUT_POWER>(a, lds, grid, s);
    case MELT_OUT_MAGNITUDE: return launch_kind<N1, N2, SUB, MELT_OUT_MAGNITUDE>(a, lds, grid, s);
    default: return set_error(MELT_E_UNSUPPORTED, "comparator output kind");
    }
}

}  // namespace

melt_status stft_plan_build(Plan &p) {
    StftShape sh;
    if (!stft_shape(p.N, sh)) return MELT_OK;   // comparator unsupported for this N: reported at call time
    std::vector<int> start, off;
    std::vector<float> w;
    build_filterbank(p.cfg, start, off, w);
    p.fb_nnz = (int)w.size();
    std::vector<float> win(p.N);
    std::vector<float2> tw(p.N);
    for (int n = 0; n < p.N; ++n) {
        double wv = 1.0;
        if (p.cfg.window != MELT_WIN_RECT) {
            const double den = (p.cfg.window == MELT_WIN_HANN_SYMMETRIC) ? double(p.N - 1) : double(p.N);
            wv = 0.5 - 0.5 * std::cos(2.0 * kPiD * double(n) / den);
        }
        win[n] = float(wv);
        const double ang = 2.0 * kPiD * double(n) / double(p.N);   // index already reduced: n < N
        tw[n] = make_float2(float(std::cos(ang)), float(-std::sin(ang)));
    }
    auto up = [](const void *src, size_t bytes, void **dst) -> melt_status {
        if (hipMalloc(dst, bytes ? bytes : 4) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "hipMalloc");
        if (bytes == 0) return MELT_OK;
        return hip_check(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy");
    };
    melt_status st = up(w.data(), w.size() * 4, (void **)&p.d_fb_w);
    if (st == MELT_OK) st = up(start.data(), start.size() * 4, (void **)&p.d_fb_start);
    if (st == MELT_OK) st = up(off.data(), off.size() * 4, (void **)&p.d_fb_off);
    if (st == MELT_OK) st = up(tw.data(), tw.size() * sizeof(float2), (void **)&p.d_twiddle);
    if (st == MELT_OK) st = up(win.data(), win.size() * 4, (void **)&p.d_window);
    return st;
}

int stft_chunk_frames(const Plan &p) {
    StftShape sh;
    return stft_shape(p.N, sh) ? 2 * sh.FPW * sh.SUB : 32;
}

// Chunk size for a batch of n_frames, in whole sub-tasks (1 to SUB).  Waves take chunks from
// a queue, so a batch runs in ceil(chunks / resident waves) rounds, each as long as one chunk.
// A short batch (at most four one-sub-task rounds) takes one sub-task per chunk, which
// spreads it widest.  Otherwise the size minimises rounds x (per-chunk cost), with a chunk
// of s sub-tasks costing about 3 + 10 s (measured at N = 400 on 64 x 30 s: one sub-task
// ~10 us per wave at full occupancy, ~3 us of per-chunk fetch and set-up); a partly filled
// last round is what that avoids.
int stft_batch_chunk_frames(const Plan &p, int64_t n_frames) {
    StftShape sh;
    if (!stft_shape(p.N, sh)) return 32;
    const int sub = 2 * sh.FPW;
    const size_t lds = stft_lds_bytes(sh, p.M, p.fb_nnz);
    const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / std::max<size_t>(lds, 1))));
    const int64_t waves = (int64_t)p.cu_count * per_cu * kStftWaves;
    const int64_t tasks = (n_frames + sub - 1) / sub;
    if (tasks <= 4 * waves) return sub;
    int best_s = 1;
    int64_t best_cost = -1;
    for (int s = 1; s <= sh.SUB; ++s) {
        const int64_t chunks = (tasks + s - 1) / s;
        const int64_t cost = (chunks + waves - 1) / waves * (3 + 10 * (int64_t)s);
        if (best_cost < 0 || cost <= best_cost) {
            best_cost = cost;
            best_s = s;
        }
    }
    return best_s * sub;
}

melt_status launch_stft_main(Plan &p, const float *d_wave, float *d_out, hipStream_t s) {
    StftShape sh;
    if (!stft_shape(p.N, sh) || !p.d_twiddle)
        return set_error(MELT_E_UNSUPPORTED, "comparator FFT supports n_fft in {256, 400, 512, 1024, 1200}");
    const int64_t n_frames = p.prepared_frames[1];
    if (n_frames < 0) return set_error(MELT_E_INVALID_ARG, "no batch prepared");
    if (n_frames == 0) return MELT_OK;
    const size_t lds = stft_lds_bytes(sh, p.M, p.fb_nnz);
    if (lds > 160 * 1024) return set_error(MELT_E_UNSUPPORTED, "comparator LDS too large");
    const int bf = p.prepared_bf[1];
    // MFCC: the log-Mel rows go to the plan workspace, then the DCT-II product to d_out
    float *mel_out = d_out;
    if (p.K > 0) {
        const melt_status st = ensure_lmel(p, n_frames);
        if (st != MELT_OK) return st;
        mel_out = p.d_lmel;
    }
    StftArgs a;
    a.wave = d_wave;
    a.chunks = p.d_chunks[1];
    a.n_chunks = p.d_nchunks + 1;
    a.out = mel_out;
    a.n_frames = n_frames;
    a.window = p.d_window;
    a.twiddle = p.d_twiddle;
    a.fb_w = p.d_fb_w;
    a.fb_start = p.d_fb_start;
    a.fb_off = p.d_fb_off;
    a.fb_nnz = p.fb_nnz;
    a.M = p.M;
    a.H = p.H;
    a.eps = (float)p.cfg.log_eps;
    const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / lds)));
    const int64_t est = (n_frames / bf + p.prepared_clips[1] + kStftWaves - 1) / kStftWaves;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(est, (int64_t)p.cu_count * per_cu));
    melt_status st;
    switch (p.N) {
    case 400: st = launch_shape<20, 20, 8>(a, p.kern_out, lds, grid, s); break;
    case 512: st = launch_shape<16, 32, 8>(a, p.kern_out, lds, grid, s); break;
    case 1024: st = launch_shape<32, 32, 8>(a, p.kern_out, lds, grid, s); break;
    case 256: st = launch_shape<16, 16, 8>(a, p.kern_out, lds, grid, s); break;
    case 1200: st = launch_shape<30, 40, 16>(a, p.kern_out, lds, grid, s); break;
    default: return set_error(MELT_E_UNSUPPORTED, "n_fft");
    }
    if (st != MELT_OK || p.K == 0) return st;
    return launch_row_matmul(p.d_lmel, n_frames, p.M, p.K, p.d_dct, p.M, 1, d_out, s);
}

}  // namespace melt
