// MFCCT (Eq. mfcct_matrix): C = ln(S + eps) D^T with D the K x M orthonormal DCT-II, and the
// same cepstrum on the comparator's log-Mel output.  A small dense product over rows: after a
// 16-bit or FP8 projection a split binary16 product on the 32x32x16 matrix cores, else on the
// FP32 matrix cores where its operands fit the LDS staging, else on the vector ALUs,
// out[r][j] = sum_i in[r][i] A[j][i], used for the forward (A = D, i = Mel bin) and for the
// backward of the cepstrum (A = D^T, i = cepstral index: dL = dC D).
#include <algorithm>
#include <cmath>

#include "melt_internal.h"

namespace melt {

constexpr int kDctRows = 64;     // rows per workgroup (one per lane)
constexpr int kDctJ = 8;         // outputs per lane per pass (each input read serves eight)

typedef float rm_f32x4 __attribute__((ext_vector_type(4)));

// Workgroup: 4 waves over 64 rows.  The rows' inputs are staged in LDS (row stride I + 1,
// conflict-free for the 64 lanes reading one column), and so is the matrix, transposed to
// At[i][j] (j padded to a multiple of 8), whose eight entries per step are one wave-uniform
// pair of 16-byte LDS reads.  Waves take the blocks of eight outputs round-robin; every lane
// computes its row's block, with the sums running in increasing i.  vec: the input and output
// are 16-byte aligned and I, J multiples of 4 (16-byte row loads and output stores).  (A
// persistent form, staging the matrix once per workgroup, ran slower: with two workgroups per
// CU the staging and the sums of a tile no longer overlap.)
__global__ __launch_bounds__(256) void k_row_matmul(const float *__restrict__ in, int64_t rows, int I, int J,
                                                    const float *__restrict__ A, int sj, int si,
                                                    float *__restrict__ out, int vec) {
    extern __shared__ float sm[];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ld = I + 1;
    const int Jp = (J + kDctJ - 1) / kDctJ * kDctJ;
    float *tile = sm;                              // [64][I + 1]
    float *At = sm + kDctRows * ld;                // [I][Jp], 16-byte aligned (64 (I + 1) floats in)
    for (int e = threadIdx.x; e < I * Jp; e += blockDim.x) {
        const int i = e / Jp, j = e - i * Jp;
        At[e] = j < J ? A[(size_t)j * sj + (size_t)i * si] : 0.0f;
    }
    const int64_t r0 = (int64_t)blockIdx.x * kDctRows;
    const int nr = (int)(rows - r0 < kDctRows ? rows - r0 : kDctRows);
    const float *src = in + r0 * I;                // the workgroup's rows are contiguous
    const int n = nr * I;
    if (vec) {
        for (int e = 4 * (int)threadIdx.x; e < n; e += 4 * (int)blockDim.x) {
            const rm_f32x4 v = *(const rm_f32x4 *)(src + e);
            const int r = e / I, i = e - r * I;    // four consecutive inputs of one row
            float *d = tile + r * ld + i;
            d[0] = v[0];
            d[1] = v[1];
            d[2] = v[2];
            d[3] = v[3];
        }
    } else {
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int r = e / I, i = e - r * I;
            tile[r * ld + i] = src[e];
        }
    }
    __syncthreads();
    if (lane >= nr) return;
    const float *x = tile + lane * ld;
    float *o = out + (r0 + lane) * J;
    for (int jb = kDctJ * wid; jb < J; jb += kDctJ * 4) {
        float acc[kDctJ] = {};
        const float *a = At + jb;
        for (int i = 0; i < I; ++i) {
            const float v = x[i];
            const rm_f32x4 a0 = *(const rm_f32x4 *)(a + i * Jp), a1 = *(const rm_f32x4 *)(a + i * Jp + 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc[q] += v * a0[q];
                acc[4 + q] += v * a1[q];
            }
        }
        if (vec && jb + kDctJ <= J) {
            *(rm_f32x4 *)(o + jb) = rm_f32x4{acc[0], acc[1], acc[2], acc[3]};
            *(rm_f32x4 *)(o + jb + 4) = rm_f32x4{acc[4], acc[5], acc[6], acc[7]};
        } else {
#pragma unroll
            for (int q = 0; q < kDctJ; ++q)
                if (jb + q < J) o[jb + q] = acc[q];
        }
    }
}

// The same product on the FP32 matrix cores (v_mfma_f32_16x16x4f32, FP32 products summed in
// FP32).  Persistent workgroups of 4 waves stage the matrix once as B-operand fragments,
//   Bf[((q 4 + e) TJ + t) 64 + lane] = A[j = 16 (jt0 + t) + (lane & 15)][i = 16 q + 4 (lane >> 4) + e],
// zero outside J x I, then walk blocks of 64 rows: a block is staged in LDS (zero-padded to
// QI = ceil(I / 16) groups of 16 inputs) and each wave multiplies 16 of its rows while the
// next block's rows load into registers.  Lane (g = lane >> 4, c = lane & 15) holds inputs
// 16 q + 4 g .. + 3 of row c, so the four lane groups of one MFMA cover inputs 16 q + e, + 4,
// + 8, + 12 (the summation order within a group of 16 is permuted, the same for every row).
// Each wave accumulates TJ output tiles of 16 columns; blockIdx.y selects which TJ tiles.
// A row's outputs depend on that row only, wherever it sits in the batch.  PRE: the rows are
// read as 16-byte vectors, at most 8 per thread per block (I <= 128), through registers.
template <int TJ, bool PRE>
__global__ __launch_bounds__(256) void k_row_mfma(const float *__restrict__ in, int64_t rows, int I, int J,
                                                  const float *__restrict__ A, int sj, int si,
                                                  float *__restrict__ out) {
    extern __shared__ float sm[];
    const int QI = (I + 15) >> 4;
    const int ld = 16 * QI + 4;                    // row stride: 16-byte aligned rows
    float *tile = sm;                              // [64][ld]
    float *Bf = sm + 64 * ld;                      // [QI][4][TJ][64]
    const int jt0 = blockIdx.y * TJ;
    for (int idx = threadIdx.x; idx < QI * 4 * TJ * 64; idx += blockDim.x) {
        const int l = idx & 63, t = (idx >> 6) % TJ, qe = (idx >> 6) / TJ;
        const int j = 16 * (jt0 + t) + (l & 15), i = 16 * (qe >> 2) + 4 * (l >> 4) + (qe & 3);
        Bf[idx] = (j < J && i < I) ? A[(size_t)j * sj + (size_t)i * si] : 0.0f;
    }
    // zero padding inputs of every row (their matrix entries are 0, but LDS may hold
    // non-finite values); the staging below never writes them
    const int pad = 16 * QI - I;
    for (int e = threadIdx.x; e < 64 * pad; e += blockDim.x) {
        const int r = e / pad;
        tile[r * ld + I + (e - r * pad)] = 0.0f;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const int64_t nblk = (rows + 63) / 64;
    int64_t blk = blockIdx.x;
    rm_f32x4 pre[PRE ? 8 : 1];
    auto fetch = [&](int64_t b) {              // rows of block b into registers
        const int64_t r0 = b * 64;
        const int n = (int)(rows - r0 < 64 ? rows - r0 : 64) * I;
        const float *src = in + r0 * I;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = 4 * (int)threadIdx.x + 1024 * u;
            if (e < n) pre[u] = *(const rm_f32x4 *)(src + e);
        }
    };
    if (PRE && blk < nblk) fetch(blk);
    for (; blk < nblk; blk += gridDim.x) {
        const int64_t r0 = blk * 64;
        const int nr = (int)(rows - r0 < 64 ? rows - r0 : 64);
        __syncthreads();                           // the previous block's rows are consumed
        if constexpr (PRE) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = 4 * (int)threadIdx.x + 1024 * u;
                if (e < nr * I) {
                    const int r = e / I, i = e - r * I;
                    *(rm_f32x4 *)(tile + r * ld + i) = pre[u];
                }
            }
            if (blk + gridDim.x < nblk) fetch(blk + gridDim.x);
        } else {
            const float *src = in + r0 * I;
            for (int e = threadIdx.x; e < nr * I; e += blockDim.x) {
                const int r = e / I, i = e - r * I;
                tile[r * ld + i] = src[e];
            }
        }
        __syncthreads();
        if (16 * wid >= nr) continue;
        const float *arow = tile + (16 * wid + c) * ld + 4 * g;
        rm_f32x4 acc[TJ];
#pragma unroll
        for (int t = 0; t < TJ; ++t) acc[t] = rm_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int q = 0; q < QI; ++q) {
            const rm_f32x4 a = *(const rm_f32x4 *)(arow + 16 * q);
            const float *bq = Bf + q * 4 * TJ * 64 + lane;
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int t = 0; t < TJ; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], bq[(e * TJ + t) * 64], acc[t], 0, 0, 0);
        }
        // lane holds rows 4 g + v of its wave's 16, column c of each tile
#pragma unroll
        for (int t = 0; t < TJ; ++t) {
            const int j = 16 * (jt0 + t) + c;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = r0 + 16 * wid + 4 * g + v;
                if (row < rows && j < J) out[row * J + j] = acc[t][v];
            }
        }
    }
}

// The cepstrum after a 16-bit or FP8 MelT projection, on the binary16 matrix cores as the
// split product Lh Dh + Lh Dl + Ll Dh (two 11-bit significands per operand; products exact in
// FP32, each term about 22 significant bits, far below the projection's own error).  The
// log-Mel values are pre-scaled by 2^9 (with eps at least the smallest normal, |L| <= 89, so
// 2^9 L stays below binary16's 65504) and the DCT by 2^10 (|D| <= 1), both exact, so that the
// low parts of small values stay normal; the FP32 sums are divided by 2^19.
// v_mfma_f32_32x32x16_f16 with the DCT as A and 32 log-Mel rows as B: lane (c = lane % 32,
// h = lane / 32) loads inputs 8 u + 4 h .. + 3 of row c for u < 2 NI (16-byte loads, the two
// halves of a wave reading adjacent 16 bytes of a row, all issued before the multiplies), so
// k-slot (h, e) of group g is input 16 g + 8 (e / 4) + 4 h + e % 4 on both operands.  The DCT
// fragments (TJ tiles of 32 coefficients by NI groups, hi and lo) are packed once per plan
// (k_pack_dct_x3) and held in registers for the wave's life.  Lane (c, h) ends with
// coefficients 32 t + 8 q + 4 h .. + 3 of row c.  Waves walk 32-row tiles.  The host
// guarantees I % 8 == 0, I <= 16 NI, J <= 32 TJ and 16-byte aligned input rows; vec: output
// rows 16-byte aligned too (J % 4 == 0).
typedef _Float16 cx_h16x8 __attribute__((ext_vector_type(8)));
typedef float cx_f32x16 __attribute__((ext_vector_type(16)));

// F[((t NI + g) 2 + part) 64 + lane][e] = part 0: hi, 1: lo of 2^10 D[32 t + lane % 32][i],
// i = 16 g + 8 (e / 4) + 4 (lane / 32) + e % 4, zero outside K x M
__global__ void k_pack_dct_x3(const float *__restrict__ D, int K, int M, int NI, int TJ, cx_h16x8 *__restrict__ F) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= TJ * NI * 2 * 64) return;
    const int lane = idx & 63, part = (idx >> 6) & 1, tg = idx >> 7, g = tg % NI, t = tg / NI;
    cx_h16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int j = 32 * t + (lane & 31), i = 16 * g + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const float d = (j < K && i < M) ? D[(size_t)j * M + i] * 1024.0f : 0.0f;
        const _Float16 dh = (_Float16)d;
        v[e] = part ? (_Float16)(d - (float)dh) : dh;
    }
    F[idx] = v;
}

template <int NI, int TJ>
__global__ __launch_bounds__(256) void k_cepstrum_x3(const float *__restrict__ in, int64_t rows, int I, int J,
                                                     const cx_h16x8 *__restrict__ F, float *__restrict__ out,
                                                     int vec) {
    const int lane = threadIdx.x & 63, c = lane & 31, h = lane >> 5;
    cx_h16x8 Dh[TJ][NI], Dl[TJ][NI];
#pragma unroll
    for (int t = 0; t < TJ; ++t)
#pragma unroll
        for (int g = 0; g < NI; ++g) {
            Dh[t][g] = F[((t * NI + g) * 2) * 64 + lane];
            Dl[t][g] = F[((t * NI + g) * 2 + 1) * 64 + lane];
        }
    const int64_t ntile = (rows + 31) >> 5;
    const int64_t wstep = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntile; tile += wstep) {
        const int64_t r = tile * 32 + c;
        const bool live = r < rows;
        const float *src = in + r * I + 4 * h;
        rm_f32x4 x[2 * NI];
#pragma unroll
        for (int u = 0; u < 2 * NI; ++u)
            x[u] = (live && 8 * u < I) ? *(const rm_f32x4 *)(src + 8 * u) : rm_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        cx_f32x16 acc[TJ];
#pragma unroll
        for (int t = 0; t < TJ; ++t) acc[t] = cx_f32x16{};
#pragma unroll
        for (int g = 0; g < NI; ++g) {
            cx_h16x8 lh, ll;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float v = x[2 * g + (e >> 2)][e & 3] * 512.0f;
                const _Float16 vh = (_Float16)v;
                lh[e] = vh;
                ll[e] = (_Float16)(v - (float)vh);
            }
#pragma unroll
            for (int t = 0; t < TJ; ++t) {
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dh[t][g], lh, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dl[t][g], lh, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dh[t][g], ll, acc[t], 0, 0, 0);
            }
        }
        if (!live) continue;
        float *o = out + r * J;
#pragma unroll
        for (int t = 0; t < TJ; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j0 = 32 * t + 8 * q + 4 * h;
                const rm_f32x4 v = rm_f32x4{acc[t][4 * q], acc[t][4 * q + 1], acc[t][4 * q + 2], acc[t][4 * q + 3]} *
                                   (1.0f / 524288.0f);
                if (vec && j0 + 4 <= J) {
                    *(rm_f32x4 *)(o + j0) = v;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (j0 + e < J) o[j0 + e] = v[e];
                }
            }
    }
}

namespace {

template <int TJ>
melt_status launch_mfma(const float *in, int64_t rows, int I, int J, const float *A, int sj, int si, float *out,
                        bool pre, size_t lds, hipStream_t s) {
    const void *k = pre ? (const void *)k_row_mfma<TJ, true> : (const void *)k_row_mfma<TJ, false>;
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t nblk = (rows + 63) / 64;
    const int gy = ((J + 15) / 16 + TJ - 1) / TJ;
    // two workgroups per CU over all launch columns
    const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(nblk, (2 * (int64_t)cus + gy - 1) / gy));
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (pre) k_row_mfma<TJ, true><<<grid, 256, lds, s>>>(in, rows, I, J, A, sj, si, out);
    else k_row_mfma<TJ, false><<<grid, 256, lds, s>>>(in, rows, I, J, A, sj, si, out);
    return hip_check(hipGetLastError(), "cepstrum launch");
}

}  // namespace

// the split binary16 cepstrum takes K <= 64 (one or two tiles of 32) and M <= 128, M % 8 == 0
static bool x3_fits(int K, int M) { return K >= 1 && K <= 64 && M % 8 == 0 && M >= 8 && M <= 128; }

melt_status pack_dct_x3(Plan &p) {
    if (!x3_fits(p.K, p.M)) return MELT_OK;
    const int ni = (p.M + 15) / 16, tj = (p.K + 31) / 32;
    const size_t n = (size_t)tj * ni * 2 * 64;
    if (hipMalloc(&p.d_dct_x3, n * 16) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "DCT fragments");
    k_pack_dct_x3<<<(unsigned)((n + 255) / 256), 256>>>(p.d_dct, p.K, p.M, ni, tj, (cx_h16x8 *)p.d_dct_x3);
    melt_status st = hip_check(hipGetLastError(), "pack DCT fragments");
    if (st == MELT_OK) st = hip_check(hipStreamSynchronize(nullptr), "pack DCT fragments");
    return st;
}

template <int NI, int TJ>
static melt_status launch_x3(const Plan &p, const float *in, int64_t rows, float *out, hipStream_t s) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t ntile = (rows + 31) / 32;
    const int vec = p.K % 4 == 0 && (uintptr_t)out % 16 == 0;
    // two workgroups of four waves per CU: the fragments and the rows in flight take ~250 VGPRs
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((ntile + 3) / 4, 2 * (int64_t)cus));
    k_cepstrum_x3<NI, TJ><<<(unsigned)grid, 256, 0, s>>>(in, rows, p.M, p.K, (const cx_h16x8 *)p.d_dct_x3, out, vec);
    return hip_check(hipGetLastError(), "cepstrum (split binary16) launch");
}

template <int TJ>
static melt_status launch_x3_tj(const Plan &p, const float *in, int64_t rows, float *out, hipStream_t s) {
    switch ((p.M + 15) / 16) {
    case 1: return launch_x3<1, TJ>(p, in, rows, out, s);
    case 2: return launch_x3<2, TJ>(p, in, rows, out, s);
    case 3: return launch_x3<3, TJ>(p, in, rows, out, s);
    case 4: return launch_x3<4, TJ>(p, in, rows, out, s);
    case 5: return launch_x3<5, TJ>(p, in, rows, out, s);
    case 6: return launch_x3<6, TJ>(p, in, rows, out, s);
    case 7: return launch_x3<7, TJ>(p, in, rows, out, s);
    default: return launch_x3<8, TJ>(p, in, rows, out, s);
    }
}

// the cepstrum of the plan's MelT forward: split binary16 matrix cores after a 16-bit or FP8
// projection (when the fragments were packed), FP32 matrix cores otherwise
melt_status launch_cepstrum(const Plan &p, const float *lmel, int64_t rows, float *out, hipStream_t s) {
    const int prec = p.cfg.precision;
    const bool low = prec == MELT_PREC_BF16 || prec == MELT_PREC_FP16 || prec == MELT_PREC_FP8_E4M3 ||
                     prec == MELT_PREC_FP8_E4M3_BLOCK32;
    if (rows <= 0) return MELT_OK;
    if (low && p.d_dct_x3 && (uintptr_t)lmel % 16 == 0) {
        return p.K <= 32 ? launch_x3_tj<1>(p, lmel, rows, out, s) : launch_x3_tj<2>(p, lmel, rows, out, s);
    }
    return launch_row_matmul(lmel, rows, p.M, p.K, p.d_dct, p.M, 1, out, s);
}

melt_status launch_row_matmul(const float *in, int64_t rows, int I, int J, const float *A, int sj, int si, float *out,
                              hipStream_t s) {
    if (rows <= 0) return MELT_OK;
    const int vec = (I % 4 == 0) && (J % 4 == 0) && ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
    // matrix cores when the staged rows and at least one output tile's fragments fit 80 KB
    // (two workgroups per CU)
    const int QI = (I + 15) / 16, JT = (J + 15) / 16;
    const size_t tile_bytes = (size_t)64 * (16 * QI + 4) * sizeof(float);
    const size_t frag_bytes = (size_t)QI * 4 * 64 * sizeof(float);        // per output tile
    const size_t budget = 80 * 1024;
    if (tile_bytes + frag_bytes <= budget) {
        const int tj = (int)std::min<size_t>(std::min(JT, 8), (budget - tile_bytes) / frag_bytes);
        const size_t lds = tile_bytes + (size_t)tj * frag_bytes;
        const bool pre = vec && I <= 128;
        switch (tj) {
        case 1: return launch_mfma<1>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        case 2: return launch_mfma<2>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        case 3: return launch_mfma<3>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        case 4: return launch_mfma<4>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        case 5: return launch_mfma<5>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        case 6: return launch_mfma<6>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        case 7: return launch_mfma<7>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        default: return launch_mfma<8>(in, rows, I, J, A, sj, si, out, pre, lds, s);
        }
    }
    const int Jp = (J + kDctJ - 1) / kDctJ * kDctJ;
    const size_t lds = ((size_t)kDctRows * (I + 1) + (size_t)I * Jp) * sizeof(float);
    if (lds > 160 * 1024) return set_error(MELT_E_UNSUPPORTED, "cepstrum input too wide");
    (void)hipFuncSetAttribute((const void *)k_row_matmul, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    const int64_t blocks = (rows + kDctRows - 1) / kDctRows;
    k_row_matmul<<<(unsigned)blocks, 256, lds, s>>>(in, rows, I, J, A, sj, si, out, vec);
    return hip_check(hipGetLastError(), "cepstrum launch");
}

// D[k][m] = sqrt((k == 0 ? 1 : 2) / M) cos(pi k (m + 1/2) / M), k < K: the first K rows of the
// orthonormal DCT-II, computed in FP64 (the argument reduced exactly: k (2m + 1) mod 4M).
void dct_matrix(int K, int M, std::vector<float> &D) {
    D.assign((size_t)K * M, 0.0f);
    const double pi = 3.14159265358979323846264338327950288;
    for (int k = 0; k < K; ++k)
        for (int m = 0; m < M; ++m) {
            const long long q = ((long long)k * (2 * m + 1)) % (4LL * M);
            const double v = std::sqrt((k == 0 ? 1.0 : 2.0) / M) * std::cos(pi * (double)q / (2.0 * M));
            D[(size_t)k * M + m] = (float)v;
        }
}

melt_status ensure_lmel(Plan &p, int64_t rows) {
    const size_t need = (size_t)(rows > 0 ? rows : 1) * p.M * sizeof(float);
    if (need <= p.lmel_cap) return MELT_OK;
    void *d = nullptr;
    if (hipMalloc(&d, need) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "log-Mel workspace");
    if (p.d_lmel) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p.d_lmel);
    }
    p.d_lmel = (float *)d;
    p.lmel_cap = need;
    return MELT_OK;
}

}  // namespace melt
