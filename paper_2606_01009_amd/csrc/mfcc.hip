// MFCCT (Eq. mfcct_matrix): C = ln(S + eps) D^T with D the K x M orthonormal DCT-II, and the
// same cepstrum on the comparator's log-Mel output.  A small dense product over rows,
// out[r][j] = sum_i in[r][i] A[j][i], used for the forward (A = D, i = Mel bin) and for the
// backward of the cepstrum (A = D^T, i = cepstral index: dL = dC D).
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

melt_status launch_row_matmul(const float *in, int64_t rows, int I, int J, const float *A, int sj, int si, float *out,
                              hipStream_t s) {
    if (rows <= 0) return MELT_OK;
    const int Jp = (J + kDctJ - 1) / kDctJ * kDctJ;
    const size_t lds = ((size_t)kDctRows * (I + 1) + (size_t)I * Jp) * sizeof(float);
    if (lds > 160 * 1024) return set_error(MELT_E_UNSUPPORTED, "cepstrum input too wide");
    (void)hipFuncSetAttribute((const void *)k_row_matmul, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    const int vec = (I % 4 == 0) && (J % 4 == 0) && ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
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
