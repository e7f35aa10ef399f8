// MelT forward, FP8-E4M3 operands with per-frame and per-row scaling:
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales, FP32 accumulation and an FP32
// unscaling epilogue (Eq. dmp_projection, Eq. dmp_matrix_energy, Eq. meltf).
#include "fwd_common.h"

namespace melt {

// ------------------------------------------------------------------ FP8 E4M3 row-split kernel
//
// Per-frame scaling needs one quantised copy of every frame (a sample belongs to ~N/H
// frames with different scales), so the chunk's FP32 span is staged as hop-block rows, the
// maximum |x| of every frame is formed from per-row maxima, and each frame is quantised
// with s_t = 448 / max|x_t| into a frame-major E4M3 image in LDS (K = n padded to 64).
// One wave per 32-row basis tile keeps its E4M3 rows (pre-scaled by r_j = 448 / max|W_j|)
// in registers; v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales multiplies; the
// epilogue divides by s_t r_j in FP32 before R^2 + I^2.

template <int NG>
__global__ __launch_bounds__(512) void k_melt_f8_rs(FwdArgs a, const i32x8 *__restrict__ bq, const float *__restrict__ rinv_g,
                                                    int N, int bf) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6, nthreads = blockDim.x, nw = nthreads >> 6;
    constexpr int KP = NG * 64;             // padded frame length in the E4M3 image
    constexpr int SQ = KP + 16;             // row stride (bytes): 4 x odd dwords -> conflict-free 16-byte reads
    const int rows_max = bf + a.J - 1;
    float *xs = lds;                                                 // FP32 hop-block rows
    unsigned char *xq = reinterpret_cast<unsigned char *>(lds + rows_max * a.S);   // [bf][SQ] E4M3
    float *sinv = reinterpret_cast<float *>(xq + bf * SQ);           // [bf] 1 / s_t
    float *mfull = sinv + bf;                                        // [rows] max over the row
    float *mpre = mfull + rows_max;                                  // [rows] max over the last segment's prefix
    const int Llast = N - (a.J - 1) * a.H;                           // length of the last segment
    i32x8 A[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) A[g] = bq[((size_t)rt * NG + g) * 64 + lane];
    float rinv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rinv[r] = rinv_g[rt * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)];
    zero_pad_columns<ConvF32>(a, rows_max, xs, nthreads, 0);
    const int nch = *a.n_chunks;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = read_chunk(a.chunks, c);
        __syncthreads();
        stage_span<ConvF32, 8>(a, ch, xs, nthreads, 0);
        __syncthreads();
        // per-row maxima (whole row, and the prefix the last segment uses)
        const int rows = ch.n_frames + a.J - 1;
        for (int r = rt; r < rows; r += nw) {
            float mf = 0.0f, mp = 0.0f;
            for (int col = lane; col < a.H; col += 64) {
                const float v = fabsf(xs[r * a.S + col]);
                mf = fmaxf(mf, v);
                if (col < Llast) mp = fmaxf(mp, v);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                mf = fmaxf(mf, __shfl_xor(mf, o));
                mp = fmaxf(mp, __shfl_xor(mp, o));
            }
            if (lane == 0) {
                mfull[r] = mf;
                mpre[r] = mp;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < ch.n_frames; t += nthreads) {
            float mx = mpre[t + a.J - 1];
            for (int j = 0; j + 1 < a.J; ++j) mx = fmaxf(mx, mfull[t + j]);
            const float s = mx > 0.0f ? __fdiv_rn(448.0f, mx) : 1.0f;
            sinv[t] = s;                       // scale itself; inverted in the epilogue
        }
        __syncthreads();
        // quantise: frame t, samples n = 4u..4u+3 -> one 32-bit LDS word
        for (int i = threadIdx.x; i < ch.n_frames * (KP / 4); i += nthreads) {
            const int t = i / (KP / 4), u = i - t * (KP / 4);
            const float s = sinv[t];
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int n = 4 * u + e;
                float x = 0.0f;
                if (n < N) {
                    const int j = n / a.H, col = n - j * a.H;
                    x = xs[(t + j) * a.S + col];
                }
                v[e] = __fmul_rn(x, s);
            }
            *reinterpret_cast<unsigned *>(xq + t * SQ + 4 * u) = fp8x4(v[0], v[1], v[2], v[3]);
        }
        __syncthreads();
        const int nft = (ch.n_frames + 31) >> 5;
        for (int ft = 0; ft < nft; ft += 2) {
            const bool two = ft + 1 < nft;
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            const unsigned char *q0 = xq + (ft * 32 + (lane & 31)) * SQ + 32 * (lane >> 5);
            const unsigned char *q1 = q0 + 32 * SQ;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const uint4 b0l = *(const uint4 *)(q0 + 64 * g), b0h = *(const uint4 *)(q0 + 64 * g + 16);
                i32x8 B0 = {(int)b0l.x, (int)b0l.y, (int)b0l.z, (int)b0l.w, (int)b0h.x, (int)b0h.y, (int)b0h.z, (int)b0h.w};
                acc0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], B0, acc0, 0, 0, 0, 127, 0, 127);
                if (two) {
                    const uint4 b1l = *(const uint4 *)(q1 + 64 * g), b1h = *(const uint4 *)(q1 + 64 * g + 16);
                    i32x8 B1 = {(int)b1l.x, (int)b1l.y, (int)b1l.z, (int)b1l.w, (int)b1h.x, (int)b1h.y, (int)b1h.z, (int)b1h.w};
                    acc1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], B1, acc1, 0, 0, 0, 127, 0, 127);
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 1 && !two) break;
                f32x16 &acc = u ? acc1 : acc0;
                const int f = (ft + u) * 32 + (lane & 31);
                const float is = f < ch.n_frames ? 1.0f / sinv[f] : 0.0f;
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] = acc[r] * (is * rinv[r]);
                store_tile(a, ch, rt, f, lane, acc);
            }
        }
    }
}

// ------------------------------------------------------------------ FP8 kernel, direct-to-LDS staging
//
// As k_melt_f8_rs, with the chunk's sample span copied HBM -> LDS by direct-to-LDS loads
// (async_span) while the previous chunk multiplies.  Frame t of the chunk is span samples
// [tH, tH + N): its maximum comes from 16-sample block maxima when hop and frame are whole
// blocks, else from per-row maxima (no reduction per frame either way), and its E4M3
// image from one flat pass over every (frame, 4-sample word) of the chunk, 16-byte reads
// straight from the contiguous span.  Positions at or past the valid span (clip end) count
// as 0.  Outputs are stored straight from the
// accumulators.  Waves map to row tiles and frame tiles as in the 16-bit kernel
// (wave_layout: one or two leftover row tiles are shared by four waves, by frame tiles).
template <int NG>
__global__ __launch_bounds__(512) void k_melt_f8_as(FwdArgs a, const i32x8 *__restrict__ bq,
                                                    const float *__restrict__ rinv_g, int N, int bf, int scr_off,
                                                    int full, int psplit) {
    extern __shared__ float lds_f8[];
    const int lane = threadIdx.x & 63, nthreads = blockDim.x;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = nthreads >> 6;
    int rt = wid, part = 0, P = 1;
    if (wid >= full) {
        rt = full + (wid - full) / psplit;
        part = (wid - full) % psplit;
        P = psplit;
    }
    constexpr int KP = NG * 64;             // padded frame length in the E4M3 image
    constexpr int SQ = KP + 16;             // row stride (bytes): 4 x odd dwords -> conflict-free 16-byte reads
    unsigned char *xq = reinterpret_cast<unsigned char *>(lds_f8);              // [bf][SQ] E4M3
    float *sinv = reinterpret_cast<float *>(xq + bf * SQ);                       // [bf] s_t
    float *mfull = sinv + bf;                                                    // [bf + J - 1] row maxima
    float *mpre = mfull + bf + a.J - 1;                                          // [bf + J - 1] prefix maxima
    float *bmax = sinv + bf;                   // or [(bf + J - 1) H / 16] block maxima (same area)
    float *scratch = lds_f8 + scr_off;                                           // FP32 span
    i32x8 A[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) A[g] = bq[((size_t)rt * NG + g) * 64 + lane];
    float rinv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rinv[r] = rinv_g[rt * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)];
    const int nch = *a.n_chunks;
    // the next chunk's span is copied by the waves with the least multiply work (those
    // sharing a row tile; the upper half of the waves when every wave owns one): only they
    // wait for it, so the other waves never wait on their own output stores
    const int dma0 = full < nw ? full : nw / 2;
    const bool dma_wave = wid >= dma0;
    int c = blockIdx.x;
    if (c < nch) async_span(a, read_chunk(a.chunks, c), scratch);
    async_wait();
    __shared__ ChunkRing ring;
    for (int it = 0; c < nch; c += gridDim.x, ++it) {
        const int ri = it % kRing;
        if (ri == 0) ring_fill(ring, a.chunks, c, gridDim.x, nch);
        __syncthreads();                           // span of chunk c is in scratch; the image is free
        const Chunk ch = ring_get(ring, ri);
        const Chunk chn = ring_get(ring, ri + 1);
        const int valid = span_valid(a, ch);
        if ((a.H & 15) == 0 && (N & 15) == 0) {
            // Frame maxima from 16-sample block maxima (frames start and end on block
            // boundaries).  A wave reads 1024 contiguous samples as four 1 KB rows of 16-byte
            // reads (consecutive lanes, consecutive addresses); two quad permutations combine
            // the four lanes that hold one block.
            const int span_len = (ch.n_frames + a.J - 1) * a.H;
            const int nblk = span_len >> 4;
            for (int base = 1024 * wid; base < span_len; base += 1024 * nw) {
                float bmx[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int o = base + 256 * k + 4 * lane;
                    f32x4 v;
                    if (o + 4 <= valid) {
                        v = *(const f32x4 *)(scratch + o);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = o + e < valid ? scratch[o + e] : 0.0f;
                    }
                    float m = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
                    m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, m), 0xB1, 0xF, 0xF, false)));
                    m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, m), 0x4E, 0xF, 0xF, false)));
                    bmx[k] = m;
                }
                if ((lane & 3) == 0) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int blk = (base >> 4) + 16 * k + (lane >> 2);
                        if (blk < nblk) bmax[blk] = bmx[k];
                    }
                }
            }
            __syncthreads();
            // four consecutive lanes per frame, each over every fourth of its blocks
            const int bpf = N >> 4, bph = a.H >> 4;           // blocks per frame, per hop
            for (int i = threadIdx.x; i < 4 * ch.n_frames; i += nthreads) {
                const int t = i >> 2, q = i & 3;
                float mx = 0.0f;
                for (int j = q; j < bpf; j += 4) mx = fmaxf(mx, bmax[t * bph + j]);
                mx = fmaxf(mx, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, mx), 0xB1, 0xF, 0xF, false)));
                mx = fmaxf(mx, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, mx), 0x4E, 0xF, 0xF, false)));
                if (q == 0) sinv[t] = mx > 0.0f ? __fdiv_rn(448.0f, mx) : 1.0f;   // the scale; inverted in the epilogue
            }
            __syncthreads();
        } else {
            // Per-frame scales from per-row maxima: row r (span samples [rH, rH + H), 0 at or
            // past the clip end) gets the maximum of |x| over the whole row and over the prefix
            // of Llast samples that the last segment of a frame uses, four lanes per row.  Frame
            // t's maximum is then that of rows t .. t + J - 2 and the prefix of row t + J - 1.
            const int rows = ch.n_frames + a.J - 1;
            const int Llast = N - (a.J - 1) * a.H;
            for (int idx = threadIdx.x; idx < 4 * rows; idx += nthreads) {
                const int r = idx >> 2, q = idx & 3;
                const int c0 = (q * a.H) >> 2, c1 = ((q + 1) * a.H) >> 2;
                const int o0 = r * a.H;
                float mf = 0.0f, mp = 0.0f;
                if ((a.H & 15) == 0 && o0 + c1 <= valid) {
                    // quarter rows of a multiple of 4 samples, 16-byte aligned, all present
                    for (int col = c0; col < c1; col += 4) {
                        const f32x4 v = *(const f32x4 *)(scratch + o0 + col);
                        const float m4 = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
                        mf = fmaxf(mf, m4);
                        if (col + 4 <= Llast) mp = fmaxf(mp, m4);
                        else if (col < Llast)
                            for (int e = 0; e < Llast - col; ++e) mp = fmaxf(mp, fabsf(v[e]));
                    }
                } else {
                    for (int col = c0; col < c1; ++col) {
                        const float v = o0 + col < valid ? fabsf(scratch[o0 + col]) : 0.0f;
                        mf = fmaxf(mf, v);
                        if (col < Llast) mp = fmaxf(mp, v);
                    }
                }
                // the four lanes of a row are consecutive and active together
                mf = fmaxf(mf, __shfl_xor(mf, 1));
                mp = fmaxf(mp, __shfl_xor(mp, 1));
                mf = fmaxf(mf, __shfl_xor(mf, 2));
                mp = fmaxf(mp, __shfl_xor(mp, 2));
                if (q == 0) {
                    mfull[r] = mf;
                    mpre[r] = mp;
                }
            }
            __syncthreads();
            for (int t = threadIdx.x; t < ch.n_frames; t += nthreads) {
                float mx = mpre[t + a.J - 1];
                for (int j = 0; j + 1 < a.J; ++j) mx = fmaxf(mx, mfull[t + j]);
                sinv[t] = mx > 0.0f ? __fdiv_rn(448.0f, mx) : 1.0f;   // the scale; inverted in the epilogue
            }
            __syncthreads();
        }
        // E4M3 image: one wave per frame, lane words u = lane + 64 k (samples 4u .. 4u + 3 of the
        // frame scaled by s_t -> one 32-bit word, 0 past N and past the clip end), the loads of
        // four frames of the wave in flight together
        {
            constexpr int WPF = KP / 4;               // words per frame
            constexpr int KW = (WPF + 63) / 64;       // words per lane
            constexpr int FT = 4;                     // frames in flight per wave
            const bool vec = (a.H & 3) == 0 && (N & 3) == 0;
            for (int t0 = wid; t0 < ch.n_frames; t0 += FT * nw) {
                f32x4 x[FT][KW];
                float sc[FT];
#pragma unroll
                for (int h = 0; h < FT; ++h) {
                    const int t = t0 + h * nw;
                    sc[h] = 0.0f;
#pragma unroll
                    for (int k = 0; k < KW; ++k) x[h][k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                    if (t >= ch.n_frames) continue;
                    sc[h] = sinv[t];
                    const int base = t * a.H;
                    const bool whole = vec && base + N <= valid;    // every sample of the frame present
#pragma unroll
                    for (int k = 0; k < KW; ++k) {
                        const int n0 = 4 * (lane + 64 * k), o = base + n0;
                        if (whole) {
                            if (n0 < N) x[h][k] = *(const f32x4 *)(scratch + o);
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) x[h][k][e] = (n0 + e < N && o + e < valid) ? scratch[o + e] : 0.0f;
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < FT; ++h) {
                    const int t = t0 + h * nw;
                    if (t >= ch.n_frames) break;
                    unsigned *dst = reinterpret_cast<unsigned *>(xq + t * SQ);
#pragma unroll
                    for (int k = 0; k < KW; ++k) {
                        const int u = lane + 64 * k;
                        if (u < WPF)
                            dst[u] = fp8x4(__fmul_rn(x[h][k][0], sc[h]), __fmul_rn(x[h][k][1], sc[h]),
                                           __fmul_rn(x[h][k][2], sc[h]), __fmul_rn(x[h][k][3], sc[h]));
                    }
                }
            }
        }
        __syncthreads();                           // image ready; scratch is free
        if (dma_wave && c + (int)gridDim.x < nch) async_span_waves(a, chn, scratch, wid - dma0, nw - dma0);
        const int nft = (ch.n_frames + 31) >> 5;
        // The next chunk's copy must land before the barrier that starts the next iteration:
        // each wave waits ahead of its last tiles' stores (leaving those in flight), or after
        // the loop if it had no tile.
        bool waited = !dma_wave;
        const int step = P == 1 ? 2 : P;
        for (int ft = part; ft < nft; ft += step) {
            const bool two = step == 2 && ft + 1 < nft;
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            const unsigned char *q0 = xq + (ft * 32 + (lane & 31)) * SQ + 32 * (lane >> 5);
            if (step == 2) {
                // a lone last tile multiplies its own frames twice rather than branching
                const unsigned char *q1 = two ? q0 + 32 * SQ : q0;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const uint4 b0l = *(const uint4 *)(q0 + 64 * g), b0h = *(const uint4 *)(q0 + 64 * g + 16);
                    const uint4 b1l = *(const uint4 *)(q1 + 64 * g), b1h = *(const uint4 *)(q1 + 64 * g + 16);
                    const i32x8 B0 = {(int)b0l.x, (int)b0l.y, (int)b0l.z, (int)b0l.w, (int)b0h.x, (int)b0h.y, (int)b0h.z, (int)b0h.w};
                    const i32x8 B1 = {(int)b1l.x, (int)b1l.y, (int)b1l.z, (int)b1l.w, (int)b1h.x, (int)b1h.y, (int)b1h.z, (int)b1h.w};
                    acc0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], B0, acc0, 0, 0, 0, 127, 0, 127);
                    acc1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], B1, acc1, 0, 0, 0, 127, 0, 127);
                }
            } else {
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const uint4 b0l = *(const uint4 *)(q0 + 64 * g), b0h = *(const uint4 *)(q0 + 64 * g + 16);
                    const i32x8 B0 = {(int)b0l.x, (int)b0l.y, (int)b0l.z, (int)b0l.w, (int)b0h.x, (int)b0h.y, (int)b0h.z, (int)b0h.w};
                    acc0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], B0, acc0, 0, 0, 0, 127, 0, 127);
                }
            }
            if (!waited && ft + step >= nft) {
                async_wait();
                waited = true;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 1 && !two) break;
                f32x16 &acc = u ? acc1 : acc0;
                const int f = (ft + u) * 32 + (lane & 31);
                const float is = f < ch.n_frames ? 1.0f / sinv[f] : 0.0f;
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] = acc[r] * (is * rinv[r]);
                store_tile(a, ch, rt, (ft + u) * 32 + (lane & 31), lane, acc);
            }
        }
        if (!waited) async_wait();                 // no tile for this wave (or a frameless chunk)
    }
}

// ------------------------------------------------------------------ launch

template <int NG>
static melt_status launch_f8(Plan &p, const FwdArgs &a, size_t lds, int grid, int bf, hipStream_t s) {
    allow_lds(k_melt_f8_rs<NG>);
    k_melt_f8_rs<NG><<<grid, 64 * p.row_tiles, lds, s>>>(a, (const i32x8 *)p.d_pack_f8, p.d_rowscale, p.N, bf);
    return hip_check(hipGetLastError(), "melt f8 launch");
}

// LDS of the direct-to-LDS FP8 kernel at bf frames per chunk: the E4M3 image, the scales,
// the row and prefix maxima, the FP32 span (16-byte aligned), then the epilogue areas
size_t f8_as_scratch_offset(const Plan &p, int bf) {
    const int ng8 = (p.N + 63) / 64;
    const size_t rows = (size_t)(bf + p.geo32.J - 1);
    const size_t maxima = std::max(2 * rows, (rows * p.H + 15) / 16);    // row or block maxima
    const size_t img = (size_t)bf * (ng8 * 64 + 16) + (size_t)bf * 4 + maxima * 4;
    return (img + 15) & ~size_t(15);
}
size_t f8_as_lds_bytes(const Plan &p, int bf) {
    return (f8_as_scratch_offset(p, bf) + (size_t)(bf + p.geo32.J - 1) * p.H * 4 + 15) & ~size_t(15);
}

template <int NG>
static melt_status launch_f8_as(Plan &p, const FwdArgs &a, size_t lds, int grid, int bf, hipStream_t s) {
    allow_lds(k_melt_f8_as<NG>, kRingBytes);
    const WaveLayout w = wave_layout(p);
    k_melt_f8_as<NG><<<grid, 64 * w.waves, lds, s>>>(a, (const i32x8 *)p.d_pack_f8, p.d_rowscale, p.N, bf,
                                                     (int)(f8_as_scratch_offset(p, bf) / 4), w.full, w.psplit);
    return hip_check(hipGetLastError(), "melt f8 lds-dma launch");
}

melt_status launch_melt_f8(Plan &p, const FwdTask &t, bool lds_dma, int bf) {
    const Geometry &g = p.geo32;
    const int S = lds_stride(g.Hp, 4);
    const int ng8 = (p.N + 63) / 64;
    if (p.row_tiles > 8) return set_error(MELT_E_UNSUPPORTED, "too many Mel bins for the FP8 kernel");
    const FwdArgs a = make_args(p, g, S, t);
    const hipStream_t s = t.stream;
    if (lds_dma) {
        const size_t lds = f8_as_lds_bytes(p, bf);
        if (lds + kRingBytes > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS for the FP8 kernel");
        // as many workgroups per CU as LDS holds, at most two
        const int grid = persistent_grid(p, t.est_chunks, std::min(2, (int)(kMaxLds / (lds + kRingBytes))));
        switch (ng8) {
        case 4: return launch_f8_as<4>(p, a, lds, grid, bf, s);
        case 7: return launch_f8_as<7>(p, a, lds, grid, bf, s);
        case 8: return launch_f8_as<8>(p, a, lds, grid, bf, s);
        case 16: return launch_f8_as<16>(p, a, lds, grid, bf, s);
        default: return set_error(MELT_E_UNSUPPORTED, "FP8 kernel supports n_fft in (192, 256], (384, 512], (960, 1024]");
        }
    }
    const int grid = persistent_grid(p, t.est_chunks, 1);
    const int rows_max = bf + g.J - 1;
    const size_t lds = (size_t)rows_max * S * 4 + (size_t)bf * (ng8 * 64 + 16) + (size_t)bf * 4 + 2 * (size_t)rows_max * 4;
    if (lds > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS for the FP8 kernel");
    switch (ng8) {
    case 4: return launch_f8<4>(p, a, lds, grid, bf, s);
    case 7: return launch_f8<7>(p, a, lds, grid, bf, s);
    case 8: return launch_f8<8>(p, a, lds, grid, bf, s);
    case 16: return launch_f8<16>(p, a, lds, grid, bf, s);
    default: return set_error(MELT_E_UNSUPPORTED, "FP8 kernel supports n_fft in (192, 256], (384, 512], (960, 1024]");
    }
}

}  // namespace melt
