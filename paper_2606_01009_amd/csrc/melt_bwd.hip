// Gradient of the MelT forward on gfx950 (chain rule through Eqs. meltf, dmp_matrix_energy
// and dmp_projection; the paper has no backward pass).  For out = map(S), S = R^2 + I^2,
// R = X Wr^T, I = X Wi^T and upstream g:
//   G[t, 2m] = 2 R[t,m] g[t,m] map'(S),  G[t, 2m+1] = 2 I[t,m] g[t,m] map'(S)
//   dx[s]    = sum over (t, n) with start_t + n = s of (G W)[t, n]       (overlap-add)
//   dW       = G^T X                                                    (learnable basis)
// Everything is FP32 with MFMA, deterministic (no floating-point atomics):
//   k_bwd_grad   G over every frame (a flat pass over the [T, M] gradient)
//   k_bwd_fstart the start sample of every frame
//   k_bwd_dx     owner-computes overlap-add: hop-block row b of dx is sum_j G[b - j] W_j,
//                W_j = basis columns [jH, jH + H); each sample is written once
//   k_bwd_dw_tiled  split-K GEMM G^T X over frames into per-split partials (LDS-tiled)
//   k_bwd_reduce fixed-order sum of the partials into the stacked [2M, N] gradient
#include <algorithm>

#include "melt_internal.h"

namespace melt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRowsDx = 128;       // hop-block rows per dx chunk (4 waves x 32)
constexpr int kMaxCT = 8;          // column tiles of 32 samples per hop-block row (H <= 256)

// A backward row chunk: up to kRowsDx hop-block rows of one clip.
struct RowChunk {
    int64_t sample_start;   // first sample of row 0 of the chunk
    int64_t sample_end;     // clip end (exclusive)
    int64_t g_row0;         // G row of clip frame b0 (= frame offset of the clip + b0)
    int32_t n_rows;         // rows in this chunk
    int32_t t_lo;           // -b0: chunk-local row index of the clip's frame 0
    int32_t t_hi;           // T_c - b0: chunk-local index one past the clip's last frame
    int32_t pad;
};
static_assert(sizeof(RowChunk) == 40, "RowChunk layout");

// ------------------------------------------------------------------ schedule of row chunks

__global__ __launch_bounds__(1024) void k_schedule_rows(const int64_t *__restrict__ off, int n_clips, int N, int H,
                                                        RowChunk *__restrict__ tab, int64_t cap, int *__restrict__ n_out) {
    __shared__ int64_t sf[1024], sc[1024];
    __shared__ int64_t carry_f, carry_c;
    const int tid = threadIdx.x;
    if (tid == 0) carry_f = carry_c = 0;
    __syncthreads();
    for (int base = 0; base < n_clips; base += 1024) {
        const int c = base + tid;
        int64_t st = 0, L = 0;
        if (c < n_clips) {
            st = off[c];
            L = off[c + 1] - st;
        }
        if (L < 0) L = 0;
        const int64_t T = (L >= N) ? 1 + (L - N) / H : 0;
        const int64_t R = (L + H - 1) / H;                      // rows covering the whole clip
        const int64_t K = (R + kRowsDx - 1) / kRowsDx;
        sf[tid] = T;
        sc[tid] = K;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int64_t vf = tid >= d ? sf[tid - d] : 0;
            const int64_t vc = tid >= d ? sc[tid - d] : 0;
            __syncthreads();
            sf[tid] += vf;
            sc[tid] += vc;
            __syncthreads();
        }
        const int64_t fb = carry_f + sf[tid] - T;
        const int64_t cb = carry_c + sc[tid] - K;
        for (int64_t k = 0; k < K; ++k) {
            const int64_t idx = cb + k;
            if (idx >= cap) break;
            const int64_t b0 = k * kRowsDx;
            RowChunk e;
            e.sample_start = st + b0 * H;
            e.sample_end = st + L;
            e.g_row0 = fb + b0;
            e.n_rows = (int)((R - b0) < kRowsDx ? (R - b0) : kRowsDx);
            e.t_lo = (int)(-b0);
            e.t_hi = (int)(T - b0);
            e.pad = 0;
            tab[idx] = e;
        }
        __syncthreads();
        if (tid == 1023) {
            carry_f += sf[1023];
            carry_c += sc[1023];
        }
        __syncthreads();
    }
    if (tid == 0) *n_out = (int)(carry_c < cap ? carry_c : cap);
}

// ------------------------------------------------------------------ G and frame starts

__device__ __forceinline__ float map_dS(float S, int kind, float eps) {
    switch (kind) {
    case MELT_OUT_LOG_POWER: return 1.0f / (S + eps);
    case MELT_OUT_LOG_MAGNITUDE: {
        const float r = sqrtf(S);
        return S > 0.0f ? 1.0f / (2.0f * r * (r + eps)) : 0.0f;
    }
    case MELT_OUT_POWER: return 1.0f;
    default: return S > 0.0f ? 0.5f / sqrtf(S) : 0.0f;
    }
}

__global__ void k_fill_i64(int64_t *__restrict__ p, int64_t n, int64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f32(float *__restrict__ p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// G over every frame.  Element e = t M + m of the [T, M] upstream gradient pairs with
// projections proj[2e], proj[2e + 1] (R, I of Mel bin m) and G entries G[2e], G[2e + 1], so
// the pass is flat: two elements per thread step with 16-byte projection and G accesses and
// an 8-byte gradient load when vec (pointers aligned for them), one element otherwise.
__global__ __launch_bounds__(256) void k_bwd_grad(const float *__restrict__ gout, const float *__restrict__ proj,
                                                  int64_t n_elems, int kind, float eps, float *__restrict__ G,
                                                  int vec) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t e0 = 0;
    if (vec) {
        const int64_t npairs = n_elems / 2;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npairs; i += stride) {
            const f32x4 y = ((const f32x4 *)proj)[i];
            const float2 g = ((const float2 *)gout)[i];
            const float k0 = g.x * map_dS(y[0] * y[0] + y[1] * y[1], kind, eps);
            const float k1 = g.y * map_dS(y[2] * y[2] + y[3] * y[3], kind, eps);
            ((f32x4 *)G)[i] = f32x4{2.0f * y[0] * k0, 2.0f * y[1] * k0, 2.0f * y[2] * k1, 2.0f * y[3] * k1};
        }
        e0 = 2 * npairs;
    }
    for (int64_t e = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_elems; e += stride) {
        const float r = proj[2 * e], im = proj[2 * e + 1];
        const float k = gout[e] * map_dS(r * r + im * im, kind, eps);
        G[2 * e] = 2.0f * r * k;
        G[2 * e + 1] = 2.0f * im * k;
    }
}

// one workgroup per forward chunk: the start sample of each of its frames
__global__ __launch_bounds__(256) void k_bwd_fstart(const Chunk *__restrict__ chunks, const int *__restrict__ n_chunks,
                                                    int64_t n_frames, int H, int64_t *__restrict__ fstart) {
    const int nch = *n_chunks;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = chunks[c];
        for (int f = threadIdx.x; f < ch.n_frames; f += blockDim.x)
            if (ch.out_row + f < n_frames) fstart[ch.out_row + f] = ch.sample_start + (int64_t)f * H;
    }
}

// ------------------------------------------------------------------ dx: owner-computes overlap-add

// Basis for dx, fragment order [ct][j][q-group of 8][lane][4]: B[k = q][col = c] =
// W_q[jH + 32 ct + c] with q the interleaved row (2m cosine, 2m+1 sine) and lane half h
// holding q = 8 qg + 4 h + i for MFMA step i.
__global__ void k_pack_dx(const float *__restrict__ b32, int M, int N, int H, int J, int CT, float *__restrict__ out) {
    const int QG = (2 * M + 7) / 8;
    const int64_t total = (int64_t)CT * J * QG * 64 * 4;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = i & 3;
        const int lane = (i >> 2) & 63;
        int64_t r = i >> 8;
        const int qg = (int)(r % QG);
        r /= QG;
        const int j = (int)(r % J);
        const int ct = (int)(r / J);
        const int q = qg * 8 + 4 * (lane >> 5) + e;
        const int c = ct * 32 + (lane & 31);
        const int n = j * H + c;
        float v = 0.0f;
        if (q < 2 * M && c < H && n < N) v = b32[(size_t)((q & 1) * M + (q >> 1)) * N + n];
        out[i] = v;
    }
}

// 4 waves x 32 hop-block rows; each wave computes its rows x all CT column tiles.  G rows
// [b0 - J + 1, b0 + 128) of the clip are staged in LDS (zero outside the clip's frames).
template <int CT>
__global__ __launch_bounds__(256) void k_bwd_dx(const RowChunk *__restrict__ rc, const int *__restrict__ n_rc,
                                                const float *__restrict__ G, const f32x4 *__restrict__ bpack,
                                                int M, int H, int J, int S, int64_t n_frames, float *__restrict__ dx) {
    extern __shared__ float lds[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int Q = 2 * M, QG = (Q + 7) / 8;
    const int nch = *n_rc;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const RowChunk ch = rc[c];
        __syncthreads();
        // LDS row r holds G of chunk-local frame r - (J - 1)
        const int rows = ch.n_rows + J - 1;
        for (int i = tid; i < rows * QG * 8; i += 256) {
            const int r = i / (QG * 8), q = i - r * (QG * 8);
            const int tl = r - (J - 1);
            float v = 0.0f;
            if (q < Q && tl >= ch.t_lo && tl < ch.t_hi && ch.g_row0 + tl < n_frames) v = G[(ch.g_row0 + tl) * Q + q];
            lds[r * S + q] = v;
        }
        __syncthreads();
        const int rbase = wid * 32;
        if (rbase >= ch.n_rows) continue;
        f32x16 acc[CT];
#pragma unroll
        for (int t = 0; t < CT; ++t) acc[t] = f32x16{};
        for (int j = 0; j < J; ++j) {
            // output row i uses G of frame (i - j): LDS row i - j + J - 1
            const float *lp = lds + (rbase + (lane & 31) + J - 1 - j) * S + 4 * (lane >> 5);
            const f32x4 *bp = bpack + ((size_t)j * QG) * 64 + lane;
            for (int qg = 0; qg < QG; ++qg) {
                const f32x4 a = *(const f32x4 *)(lp + qg * 8);
                f32x4 b[CT];
#pragma unroll
                for (int t = 0; t < CT; ++t) b[t] = bp[((size_t)t * J * QG + qg) * 64];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int t = 0; t < CT; ++t)
                        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[t][i], acc[t], 0, 0, 0);
            }
        }
        // acc[t]: lane holds sample column 32 t + lane % 32 of rows 8(r/4) + 4h + r%4
        const int h = lane >> 5, col = lane & 31;
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int cc = t * 32 + col;
            if (cc >= H) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = rbase + 8 * (r >> 2) + 4 * h + (r & 3);
                if (row >= ch.n_rows) continue;
                const int64_t s = ch.sample_start + (int64_t)row * H + cc;
                if (s < ch.sample_end) dx[s] = acc[t][r];
            }
        }
    }
}

// ------------------------------------------------------------------ dW: split-K G^T X

// dW = G^T X, split over frames into per-split partials (q interleaved: q = 2m + {0: cos, 1:
// sin}).  A[i = q][k = t] = G[t][q], B[k = t][col = n] = x[start_t + n].  A workgroup owns a
// 128 (q) x 128 (n) block of dW over frames [t0, t1) of its split; each wave a 64 x 64 quarter (2 x 2 MFMA tiles).
// Per step, 16 frames of G (rows of q) and of the implicitly framed waveform (x[start_t + n])
// are staged in LDS (the next step's loads in flight during the MFMAs), then each wave runs
// 8 k-steps of 2 frames over its 4 tiles.  Rows are padded to 160 floats, so the two half-
// waves (frames 2s and 2s + 1) read different banks.
constexpr int kDwKB = 16, kDwRow = 160;
__global__ __launch_bounds__(256) void k_bwd_dw_tiled(const float *__restrict__ G, const int64_t *__restrict__ fstart,
                                                      const float *__restrict__ wave, int64_t T, int M, int N,
                                                      int splits, float *__restrict__ part) {
    __shared__ float Gs[kDwKB * kDwRow], Xs[kDwKB * kDwRow];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int Q = 2 * M;
    const int QB = (Q + 127) / 128, NB = (N + 127) / 128, blocks = QB * NB;
    const int split = blockIdx.x / blocks, bb = blockIdx.x - split * blocks;
    const int qb = bb / NB, nb = bb - qb * NB;
    const int q0 = qb * 128, n0 = nb * 128;
    const int64_t per = (T + splits - 1) / splits;
    const int64_t t0 = (int64_t)split * per, t1 = t0 + per < T ? t0 + per : T;
    const int wq = (wid & 1) * 64, wn = (wid >> 1) * 64;
    const int h = lane >> 5, l32 = lane & 31;
    // staging role: frame row sr of the step, 8 consecutive q and 8 consecutive n at sc
    const int sr = tid >> 4, sc = (tid & 15) * 8;
    f32x16 acc00 = f32x16{}, acc01 = f32x16{}, acc10 = f32x16{}, acc11 = f32x16{};
    float gr[8], xr[8];
    auto load = [&](int64_t tb) {
        const int64_t tf = tb + sr;
        const int64_t st = tf < t1 ? fstart[tf] : -1;      // -1: no frame (zero row)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int q = q0 + sc + e, n = n0 + sc + e;
            gr[e] = (st >= 0 && q < Q) ? G[tf * Q + q] : 0.0f;
            xr[e] = (st >= 0 && n < N) ? wave[st + n] : 0.0f;
        }
    };
    if (t0 < t1) load(t0);
    for (int64_t tb = t0; tb < t1; tb += kDwKB) {
        __syncthreads();                               // the previous step's LDS reads are done
        *(f32x4 *)(Gs + sr * kDwRow + sc) = f32x4{gr[0], gr[1], gr[2], gr[3]};
        *(f32x4 *)(Gs + sr * kDwRow + sc + 4) = f32x4{gr[4], gr[5], gr[6], gr[7]};
        *(f32x4 *)(Xs + sr * kDwRow + sc) = f32x4{xr[0], xr[1], xr[2], xr[3]};
        *(f32x4 *)(Xs + sr * kDwRow + sc + 4) = f32x4{xr[4], xr[5], xr[6], xr[7]};
        __syncthreads();
        if (tb + kDwKB < t1) load(tb + kDwKB);
#pragma unroll
        for (int k = 0; k < kDwKB / 2; ++k) {
            const int row = (2 * k + h) * kDwRow;
            const float a0 = Gs[row + wq + l32], a1 = Gs[row + wq + 32 + l32];
            const float b0 = Xs[row + wn + l32], b1 = Xs[row + wn + 32 + l32];
            acc00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc11, 0, 0, 0);
        }
    }
    // lane holds column n, rows q = tile base + 8(r/4) + 4h + r%4 (interleaved q)
    float *p = part + (size_t)split * Q * N;
    auto put = [&](const f32x16 &acc, int qbase, int nbase) {
        const int n = nbase + l32;
        if (n >= N) return;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int qq = qbase + 8 * (r >> 2) + 4 * h + (r & 3);
            if (qq < Q) p[(size_t)qq * N + n] = acc[r];
        }
    };
    put(acc00, q0 + wq, n0 + wn);
    put(acc01, q0 + wq, n0 + wn + 32);
    put(acc10, q0 + wq + 32, n0 + wn);
    put(acc11, q0 + wq + 32, n0 + wn + 32);
}

// Sums the splits' partials in split order (so the result does not depend on the launch),
// four consecutive n per thread with 16-byte loads when N is a multiple of 4, eight splits'
// loads in flight at a time.
__global__ void k_bwd_reduce(const float *__restrict__ part, int splits, int M, int N, float *__restrict__ dW) {
    const int64_t total = (int64_t)2 * M * N;
    if ((N & 3) == 0) {
        const int64_t total4 = total / 4;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total4;
             i += (int64_t)gridDim.x * blockDim.x) {
            f32x4 s = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            int k = 0;
            for (; k + 8 <= splits; k += 8) {
                f32x4 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = *(const f32x4 *)(part + (size_t)(k + u) * total + 4 * i);
#pragma unroll
                for (int u = 0; u < 8; ++u) s += v[u];
            }
            for (; k < splits; ++k) s += *(const f32x4 *)(part + (size_t)k * total + 4 * i);
            const int q = (int)((4 * i) / N), n = (int)(4 * i - (int64_t)q * N);
            *(f32x4 *)(dW + (size_t)((q & 1) * M + (q >> 1)) * N + n) = s;   // interleaved q -> stacked rows
        }
        return;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int k = 0; k < splits; ++k) s += part[(size_t)k * total + i];
        const int q = (int)(i / N), n = (int)(i - (int64_t)q * N);
        dW[(size_t)((q & 1) * M + (q >> 1)) * N + n] = s;    // interleaved q -> stacked rows
    }
}

// ------------------------------------------------------------------ host side

namespace {

melt_status grow(void **p, size_t *cap, size_t need) {
    if (need <= *cap) return MELT_OK;
    void *d = nullptr;
    if (hipMalloc(&d, need) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "backward workspace");
    if (*p) {
        (void)hipDeviceSynchronize();
        (void)hipFree(*p);
    }
    *p = d;
    *cap = need;
    return MELT_OK;
}

template <int CT>
melt_status launch_dx(Plan &p, const float *G, float *dx, int S, size_t lds, int grid, hipStream_t s) {
    (void)hipFuncSetAttribute((const void *)k_bwd_dx<CT>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    k_bwd_dx<CT><<<grid, 256, lds, s>>>((const RowChunk *)p.d_bwd_rows, p.d_nchunks + 1, G, (const f32x4 *)p.d_pack_dx,
                                        p.M, p.H, p.geo32.J, S, p.prepared_frames[0], dx);
    return hip_check(hipGetLastError(), "bwd dx launch");
}

}  // namespace

melt_status pack_basis_dx(Plan &p, hipStream_t s) {
    const int CT = (p.H + 31) / 32;
    if (CT > kMaxCT) return MELT_OK;     // dx unsupported for this hop; reported at call time
    const int J = p.geo32.J, QG = (2 * p.M + 7) / 8;
    const size_t need = (size_t)CT * J * QG * 64 * 4 * sizeof(float);
    melt_status st = grow(&p.d_pack_dx, &p.pack_dx_cap, need);
    if (st != MELT_OK) return st;
    k_pack_dx<<<256, 256, 0, s>>>(p.d_basis32, p.M, p.N, p.H, J, CT, (float *)p.d_pack_dx);
    return hip_check(hipGetLastError(), "pack dx");
}

melt_status launch_melt_backward(Plan &p, const float *d_wave, const int64_t *d_off, int n_clips, int64_t n_frames,
                                 const float *d_gout, const float *d_proj, float *d_gwave, float *d_gbasis,
                                 hipStream_t s) {
    if (n_clips == 0 || n_frames == 0) {
        // a fill kernel rather than a memset, so that the call can be captured in a HIP graph
        if (d_gbasis) {
            k_fill_f32<<<64, 256, 0, s>>>(d_gbasis, (int64_t)2 * p.M * p.N, 0.0f);
            return hip_check(hipGetLastError(), "bwd fill");
        }
        return MELT_OK;
    }
    const int M = p.M, N = p.N, H = p.H, J = p.geo32.J, Q = 2 * M;
    const int CT = (H + 31) / 32;
    if (d_gwave && CT > kMaxCT) return set_error(MELT_E_UNSUPPORTED, "backward d/dwave supports hop <= 256");
    // workspace: proj (if recomputed) | G | frame starts | dW partials
    // dW: 128 x 128 blocks, split over frames so that about two workgroups per CU run
    const int dw_blocks = ((Q + 127) / 128) * ((N + 127) / 128);
    const int splits = (int)std::max<int64_t>(
        1, std::min<int64_t>({64, (2 * (int64_t)p.cu_count + dw_blocks - 1) / dw_blocks, n_frames / 64}));
    const size_t proj_b = d_proj ? 0 : sizeof(float) * n_frames * Q;
    const size_t g_b = sizeof(float) * n_frames * Q;
    const size_t fs_b = sizeof(int64_t) * n_frames;
    const size_t part_b = d_gbasis ? sizeof(float) * splits * Q * N : 0;
    const size_t gl_b = p.K > 0 ? sizeof(float) * n_frames * M : 0;   // dL = dC D under MFCC
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    melt_status st = grow(&p.d_bwd_ws, &p.bwd_ws_cap, al(proj_b) + al(g_b) + al(fs_b) + al(part_b) + al(gl_b) + 256);
    if (st != MELT_OK) return st;
    char *w = (char *)p.d_bwd_ws;
    float *proj_ws = (float *)w;
    float *G = (float *)(w + al(proj_b));
    int64_t *fstart = (int64_t *)(w + al(proj_b) + al(g_b));
    float *part = (float *)(w + al(proj_b) + al(g_b) + al(fs_b));
    if (p.K > 0) {
        // the cepstrum is linear: upstream over the log-Mel rows is dC D
        float *gl = (float *)(w + al(proj_b) + al(g_b) + al(fs_b) + al(part_b));
        st = launch_row_matmul(d_gout, n_frames, p.K, M, p.d_dct, 1, M, gl, s);
        if (st != MELT_OK) return st;
        d_gout = gl;
    }
    // forward chunk table (table 0); projections recomputed when not supplied
    st = launch_schedule(p, 0, d_off, n_clips, melt_chunk_frames(p), n_frames, s);
    if (st != MELT_OK) return st;
    const float *proj = d_proj;
    if (!proj) {
        float *tmp_out = G;   // G's space holds the (unused) log output of the recomputation first
        st = launch_melt_main(p, d_wave, tmp_out, proj_ws, s);
        if (st != MELT_OK) return st;
        proj = proj_ws;
    }
    k_fill_i64<<<256, 256, 0, s>>>(fstart, n_frames, -1);
    st = hip_check(hipGetLastError(), "bwd fill");
    if (st != MELT_OK) return st;
    const int64_t nchunk_est = n_frames / melt_chunk_frames(p) + n_clips + 1;
    const int grid_prep = (int)std::min<int64_t>(nchunk_est, (int64_t)p.cu_count * 4);
    k_bwd_fstart<<<grid_prep, 256, 0, s>>>(p.d_chunks[0], p.d_nchunks, n_frames, H, fstart);
    st = hip_check(hipGetLastError(), "bwd frame starts");
    if (st != MELT_OK) return st;
    {
        const int64_t n_elems = n_frames * M;
        const int vec = ((uintptr_t)proj % 16 == 0) && ((uintptr_t)d_gout % 8 == 0) && ((uintptr_t)G % 16 == 0);
        const int grid_g = (int)std::max<int64_t>(1, std::min<int64_t>((n_elems / 2 + 255) / 256, (int64_t)p.cu_count * 8));
        k_bwd_grad<<<grid_g, 256, 0, s>>>(d_gout, proj, n_elems, p.kern_out, (float)p.cfg.log_eps, G, vec);
    }
    st = hip_check(hipGetLastError(), "bwd gradient of the projections");
    if (st != MELT_OK) return st;
    if (d_gwave) {
        // rows cover every sample of every clip (samples no frame covers get 0: their G
        // rows are zero)
        const int64_t rows_cap = n_frames / kRowsDx + 2 * (int64_t)n_clips + 2 + (int64_t)n_clips * (J + 1);
        st = grow(&p.d_bwd_rows, &p.bwd_rows_cap, sizeof(RowChunk) * rows_cap);
        if (st != MELT_OK) return st;
        k_schedule_rows<<<1, 1024, 0, s>>>(d_off, n_clips, N, H, (RowChunk *)p.d_bwd_rows,
                                           (int64_t)(p.bwd_rows_cap / sizeof(RowChunk)), p.d_nchunks + 1);
        st = hip_check(hipGetLastError(), "bwd row schedule");
        if (st != MELT_OK) return st;
        p.prepared_frames[1] = -1;   // table 1's count now describes row chunks
        const int S = ((Q + 7) / 8) * 8 + 4;
        const size_t lds = (size_t)(kRowsDx + J - 1) * S * sizeof(float);
        if (lds > 160 * 1024) return set_error(MELT_E_UNSUPPORTED, "backward LDS too large (n_mels * hop)");
        const int grid = (int)std::min<int64_t>(n_frames / kRowsDx + n_clips + 1, p.cu_count);
        switch (CT) {
        case 1: st = launch_dx<1>(p, G, d_gwave, S, lds, grid, s); break;
        case 2: st = launch_dx<2>(p, G, d_gwave, S, lds, grid, s); break;
        case 3: st = launch_dx<3>(p, G, d_gwave, S, lds, grid, s); break;
        case 4: st = launch_dx<4>(p, G, d_gwave, S, lds, grid, s); break;
        case 5: st = launch_dx<5>(p, G, d_gwave, S, lds, grid, s); break;
        case 6: st = launch_dx<6>(p, G, d_gwave, S, lds, grid, s); break;
        case 7: st = launch_dx<7>(p, G, d_gwave, S, lds, grid, s); break;
        default: st = launch_dx<8>(p, G, d_gwave, S, lds, grid, s); break;
        }
        if (st != MELT_OK) return st;
    }
    if (d_gbasis) {
        k_bwd_dw_tiled<<<dw_blocks * splits, 256, 0, s>>>(G, fstart, d_wave, n_frames, M, N, splits, part);
        st = hip_check(hipGetLastError(), "bwd dW");
        if (st != MELT_OK) return st;
        k_bwd_reduce<<<512, 256, 0, s>>>(part, splits, M, N, d_gbasis);
        st = hip_check(hipGetLastError(), "bwd reduce");
    }
    return st;
}

}  // namespace melt
