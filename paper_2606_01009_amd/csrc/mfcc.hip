// MFCCT (Eq. mfcct_matrix): C = ln(S + eps) D^T with D the K x M orthonormal DCT-II, and the
// same cepstrum on the comparator's log-Mel output.  A small dense product over rows,
// out[r][j] = sum_i in[r][i] A[j][i], used for the forward (A = D, i = Mel bin) and for the
// backward of the cepstrum (A = D^T, i = cepstral index: dL = dC D).
#include <cmath>

#include "melt_internal.h"

namespace melt {

constexpr int kDctRows = 64;     // rows per workgroup (one per lane)
constexpr int kDctJ = 4;         // outputs per lane per pass (each input read serves four)

// Workgroup: 4 waves over 64 rows.  The rows' inputs are staged in LDS (row stride I + 1,
// conflict-free for the 64 lanes reading one column); wave w computes outputs
// j = 4 (w + 4 p) + 0..3 for its lane's row, with the matrix entries wave-uniform (scalar
// loads).  Sums run in increasing i.
__global__ __launch_bounds__(256) void k_row_matmul(const float *__restrict__ in, int64_t rows, int I, int J,
                                                    const float *__restrict__ A, int sj, int si,
                                                    float *__restrict__ out) {
    extern __shared__ float tile[];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t r0 = (int64_t)blockIdx.x * kDctRows;
    const int nr = (int)(rows - r0 < kDctRows ? rows - r0 : kDctRows);
    const int ld = I + 1;
    for (int e = threadIdx.x; e < nr * I; e += blockDim.x) {
        const int r = e / I, i = e - r * I;
        tile[r * ld + i] = in[(r0 + r) * I + i];
    }
    __syncthreads();
    if (lane >= nr) return;
    const float *x = tile + lane * ld;
    for (int jb = kDctJ * wid; jb < J; jb += kDctJ * 4) {
        float acc[kDctJ] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int i = 0; i < I; ++i) {
            const float v = x[i];
#pragma unroll
            for (int q = 0; q < kDctJ; ++q)
                if (jb + q < J) acc[q] += v * A[(size_t)(jb + q) * sj + (size_t)i * si];
        }
#pragma unroll
        for (int q = 0; q < kDctJ; ++q)
            if (jb + q < J) out[(r0 + lane) * J + jb + q] = acc[q];
    }
}

melt_status launch_row_matmul(const float *in, int64_t rows, int I, int J, const float *A, int sj, int si, float *out,
                              hipStream_t s) {
    if (rows <= 0) return MELT_OK;
    const size_t lds = (size_t)kDctRows * (I + 1) * sizeof(float);
    if (lds > 160 * 1024) return set_error(MELT_E_UNSUPPORTED, "cepstrum input too wide");
    (void)hipFuncSetAttribute((const void *)k_row_matmul, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    const int64_t blocks = (rows + kDctRows - 1) / kDctRows;
    k_row_matmul<<<(unsigned)blocks, 256, lds, s>>>(in, rows, I, J, A, sj, si, out);
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
