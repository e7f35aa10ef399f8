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

// ------------------------------------------------------------------ FP8 kernel, 32-sample block scales
//
// MELT_PREC_FP8_E4M3_BLOCK32.  The waveform is quantised once.  With the hop a multiple of 32,
// a chunk's span is whole 32-sample blocks of its clip, and so is every 32-sample k-block of a
// frame.  Block b gets the power-of-two scale 2^e_b (e_b the largest integer with
// 2^e_b max|x_b| <= 448; 0 for a silent block) and its samples are rounded to E4M3 into
// hop-block rows in LDS, one byte per sample, beside one E8M0 code 127 - e_b per block.  A
// frame's 64-sample k-group is two blocks, and v_mfma_scale_f32_32x32x64_f8f6f4 scales each:
// for column j of B the code of lane j covers k 0..31 and that of lane j + 32 covers k
// 32..63, while a lane's 32 operand bytes are k 16 h .. 16 h + 15 (bytes 0-15) and k 32 + 16 h
// .. (bytes 16-31), h = lane / 32.  So lane half h reads samples 16 h .. 16 h + 15 of block
// 2g and of block 2g + 1 (two 16-byte reads) and passes the code of block 2g + h; the basis
// is packed in the same order (k_pack_f8 with blocks = 1).  The product sums 2^-e_b q W_q
// over every block with no per-frame copy of the samples.  Basis rows keep the FP8_E4M3 row
// scales (unit scale in the MFMA, 1 / r_j in the epilogue).  Row groups, wave layout, chunk
// ring and span copies are those of k_melt_h16_as.

// byte offset, in the hop-block rows, of block i of a frame (samples 32 i .. 32 i + 31):
// row 32 i / H, column 32 i % H; blocks past the frame (32 i >= N, zero basis) read block 0
struct F8BlockTable {
    int off[32];
};
typedef short s16x2 __attribute__((ext_vector_type(2)));

// largest e with 2^e m <= 448 (m > 0 finite), clamped to [-127, 127]; 0 for m = 0.
// m = f 2^E with f in [0.5, 1): 2^e m <= 448 = 0.875 2^9 holds for e = 9 - E when f <= 0.875,
// else for e = 8 - E.
__device__ __forceinline__ int block_exp(float m) {
    if (!(m > 0.0f)) return 0;
    const int E = __builtin_amdgcn_frexp_expf(m);
    const float f = __builtin_amdgcn_frexp_mantf(m);
    const int e = (f <= 0.875f ? 9 : 8) - E;
    return e < -127 ? -127 : (e > 127 ? 127 : e);
}

// One lane's 32-sample block fb of a chunk's span, all in that lane: the block maximum, its
// exponent and the 32 E4M3 bytes.  The lane's eight 16-byte reads start at slot
// rot = (lane / 2) mod 8 of its 128-byte block and wrap, so that the 16 lanes of an LDS pass
// (blocks 128 bytes apart, or 4 KB apart in pairs of eight) touch 16 distinct 4-bank groups;
// each 4-sample group is written to its own 4-byte slot of the block's row bytes at `dst`.
// `whole` (wave-uniform): every active lane's block lies before `valid`; otherwise samples at
// or past `valid` (clip end) read as 0.  TWO_PASS reads the block twice (maximum, then
// conversion) to keep eight fewer vectors live, for kernels that hold more registers.
template <bool TWO_PASS>
__device__ __forceinline__ void convert_lane_block(const float *span, int valid, bool whole, int fb,
                                                   unsigned char *dst, int *codes) {
    const int rot = (threadIdx.x >> 1) & 7;
    const float *s1 = span + 32 * fb + 4 * rot, *s2 = s1 - 32;
    auto load = [&](int k) -> f32x4 {
        if (whole) return *(const f32x4 *)((k < 8 - rot ? s1 : s2) + 4 * k);
        f32x4 v;
        const int o = 32 * fb + 4 * ((k + rot) & 7);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = o + e < valid ? span[o + e] : 0.0f;
        return v;
    };
    auto amax = [](f32x4 v) { return fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))); };
    f32x4 v[TWO_PASS ? 1 : 8];
    float m = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if constexpr (TWO_PASS) {
            m = fmaxf(m, amax(load(k)));
        } else {
            v[k] = load(k);
            m = fmaxf(m, amax(v[k]));
        }
    }
    const int e = block_exp(m);
    unsigned char *d1 = dst + 4 * rot, *d2 = d1 - 32;
    auto store = [&](int k, unsigned w) { *(unsigned *)((k < 8 - rot ? d1 : d2) + 4 * k) = w; };
    // v_cvt_scalef32_pk_fp8_f32 rounds x / 2^floor(log2 s) to E4M3 in one step, so s = 2^-e
    // gives the E4M3 value of 2^e x.  2^-127 (e = 127, a block below 448 2^-127 but not
    // silent) is not a normal FP32 scale: a wave holding such a block takes ldexp and the
    // plain conversion.
    if (__builtin_amdgcn_ballot_w64(e >= 127) == 0) {
        const float sc = __builtin_bit_cast(float, (127 - e) << 23);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const f32x4 x = TWO_PASS ? load(k) : v[TWO_PASS ? 0 : k];
            const s16x2 lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(s16x2{0, 0}, x[0], x[1], sc, false);
            store(k, __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(lo, x[2], x[3], sc, true)));
        }
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const f32x4 x = TWO_PASS ? load(k) : v[TWO_PASS ? 0 : k];
            store(k, fp8x4(__builtin_ldexpf(x[0], e), __builtin_ldexpf(x[1], e), __builtin_ldexpf(x[2], e),
                           __builtin_ldexpf(x[3], e)));
        }
    }
    codes[fb] = 127 - e;
}

// byte offset of E4M3 block fb in the hop-block rows: row r = fb / bph (from the FP32 product
// (fb + 1/2) (1 / bph), exact while fb < 2^16: its error stays far below the 1 / (2 bph)
// margin), at 32 fb + r (S8 - H)
__device__ __forceinline__ int block_row_byte(int fb, float inv_bph, int pad) {
    return 32 * fb + (int)(((float)fb + 0.5f) * inv_bph) * pad;
}

// The chunk's FP32 span -> E4M3 hop-block rows (stride S8 bytes) and block codes, one block per
// lane, consecutive blocks over the lanes and waves.
__device__ __forceinline__ void convert_blocks(const FwdArgs &a, const Chunk &ch, const float *span,
                                               unsigned char *rows8, int S8, int *codes, float inv_bph) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
    const int nblk = ((ch.n_frames + a.J - 1) * a.H) >> 5;
    const int valid = span_valid(a, ch);
    const int pad = S8 - a.H;
    for (int f0 = 64 * wid; f0 < nblk; f0 += 64 * nw) {
        const int fb = f0 + lane;
        if (fb < nblk)
            convert_lane_block<true>(span, valid, 32 * (f0 + 64) <= valid, fb, rows8 + block_row_byte(fb, inv_bph, pad),
                                     codes);
    }
}

// One or two 32-frame tiles (q0, q1: the tiles' frame rows of this lane, plus 16 h; s0, s1:
// their block codes at the lane's half) against a wave's E4M3 basis tile: per k-group two
// 16-byte reads (blocks 2g and 2g + 1) and one code per tile, read D groups ahead.
template <int NG, bool TWO, int D = 2>
__device__ __forceinline__ void f8b_sweep(const i32x8 (&A)[NG], const F8BlockTable &bt, const unsigned char *q0,
                                          const unsigned char *q1, const int *s0, const int *s1, f32x16 &acc0,
                                          f32x16 &acc1) {
    i32x8 b0[D], b1[D];
    int c0[D], c1[D];
    auto fetch = [&](int g, int slot) {
        const int o0 = bt.off[2 * g], o1 = bt.off[2 * g + 1];
        const uint4 l0 = *(const uint4 *)(q0 + o0), h0 = *(const uint4 *)(q0 + o1);
        b0[slot] = i32x8{(int)l0.x, (int)l0.y, (int)l0.z, (int)l0.w, (int)h0.x, (int)h0.y, (int)h0.z, (int)h0.w};
        c0[slot] = s0[2 * g];
        if constexpr (TWO) {
            const uint4 l1 = *(const uint4 *)(q1 + o0), h1 = *(const uint4 *)(q1 + o1);
            b1[slot] = i32x8{(int)l1.x, (int)l1.y, (int)l1.z, (int)l1.w, (int)h1.x, (int)h1.y, (int)h1.z, (int)h1.w};
            c1[slot] = s1[2 * g];
        }
    };
#pragma unroll
    for (int g = 0; g < D && g < NG; ++g) fetch(g, g);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int slot = g % D;
        __builtin_amdgcn_sched_barrier(0);
        acc0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], b0[slot], acc0, 0, 0, 0, 127, 0, c0[slot]);
        if constexpr (TWO)
            acc1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], b1[slot], acc1, 0, 0, 0, 127, 0, c1[slot]);
        if (g + D < NG) fetch(g + D, slot);
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <int NG>
__global__ __launch_bounds__(512) void k_melt_f8b_as(
    FwdArgs a, const i32x8 *__restrict__ bq, const float *__restrict__ rinv_g, F8BlockTable bt, int S8, int code_off,
    int n_codes, int scr_off, int rgroups) {
    extern __shared__ float lds_f8b[];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
    const int grp = blockIdx.x % rgroups, gt_n = (a.row_tiles + rgroups - 1) / rgroups;
    const int r0 = grp * gt_n, cnt = min(a.row_tiles - r0, gt_n);
    const WaveLayout L = layout_for(cnt);
    const bool idle = wid >= L.waves;
    int rt = wid, part = 0, P = 1;
    if (wid >= L.full) {
        rt = L.full + (wid - L.full) / L.psplit;
        part = (wid - L.full) % L.psplit;
        P = L.psplit;
    }
    rt = idle ? r0 : r0 + rt;
    unsigned char *rows8 = reinterpret_cast<unsigned char *>(lds_f8b);
    int *codes = reinterpret_cast<int *>(lds_f8b) + code_off;
    float *span = lds_f8b + scr_off;
    const int bph = a.H >> 5;
    const float inv_bph = 1.0f / (float)bph;
    // codes past the chunk's blocks (read for blocks past a frame, or frames past the chunk)
    // are finite from the start
    for (int i = threadIdx.x; i < n_codes; i += blockDim.x) codes[i] = 127;
    i32x8 A[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) A[g] = bq[((size_t)rt * NG + g) * 64 + lane];
    float rinv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rinv[r] = rinv_g[rt * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)];
    const int dma0 = L.full < nw ? L.full : nw / 2;    // first copying wave
    const bool dma_wave = wid >= dma0;
    const int nch = *a.n_chunks;
    const int cstep = gridDim.x / rgroups;
    int c = blockIdx.x / rgroups;
    if (c < nch) async_span(a, read_chunk(a.chunks, c), span);
    async_wait();
    __shared__ ChunkRing ring;
    for (int it = 0; c < nch; c += cstep, ++it) {
        const int ri = it % kRing;
        if (ri == 0) ring_fill(ring, a.chunks, c, cstep, nch);
        __syncthreads();                           // span of chunk c has landed; rows are free
        const Chunk ch = ring_get(ring, ri);
        const Chunk chn = ring_get(ring, ri + 1);
        convert_blocks(a, ch, span, rows8, S8, codes, inv_bph);
        __syncthreads();                           // rows and codes ready; the span is free
        if (dma_wave && c + cstep < nch) async_span_waves(a, chn, span, wid - dma0, nw - dma0);
        const int nft = idle ? 0 : (ch.n_frames + 31) >> 5;
        bool waited = !dma_wave;
        const int step = P == 1 ? 2 : P;
        for (int ft = part; ft < nft; ft += step) {
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            const int f0 = ft * 32 + (lane & 31);
            const unsigned char *q0 = rows8 + f0 * S8 + 16 * (lane >> 5);
            const int *s0 = codes + f0 * bph + (lane >> 5);
            const bool two = step == 2 && ft + 1 < nft;
            if (two) {
                f8b_sweep<NG, true>(A, bt, q0, q0 + 32 * S8, s0, s0 + 32 * bph, acc0, acc1);
            } else {
                f8b_sweep<NG, false>(A, bt, q0, q0, s0, s0, acc0, acc1);
            }
            if (!waited && ft + step >= nft) {
                async_wait();
                waited = true;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 1 && !two) break;
                f32x16 &acc = u ? acc1 : acc0;
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] *= rinv[r];
                store_tile(a, ch, rt, (ft + u) * 32 + (lane & 31), lane, acc);
            }
        }
        if (!waited) async_wait();                 // no tile for this wave (or a frameless chunk)
    }
}

// ------------------------------------------------------------------ FP8 block-scaled, producer/consumer
//
// The arithmetic of k_melt_f8b_as, with a chunk's conversion and its multiplies on different
// waves so that they overlap (the conversion is vector-ALU and LDS work, the multiplies
// matrix-core and LDS work).  A workgroup of 12 waves: the first NC = (row tiles of the group)
// are consumers, one basis tile each, the other NP = 12 - NC producers.  Producer w owns the
// 256-sample blocks b = w, w + NP, ... of every chunk's span: it copies its blocks HBM -> LDS
// (direct-to-LDS) and converts exactly those into E4M3 rows and block codes, so no producer
// waits for another.  Two row/code buffers alternate: in iteration k the consumers multiply
// chunk k from one while the producers convert chunk k + 1 into the other and start the copy
// of chunk k + 2, with one barrier per chunk.  Three waves per SIMD: a consumer holds one
// basis tile (8 NG registers) and sweeps one frame tile at a time.  Chunk descriptors pass
// through a four-slot LDS ring: the first producer loads descriptor k + 3 in iteration k and
// stores it before the barrier (slot (k + 3) mod 4 was last read in iteration k - 1).

// the copies of one 256-sample block b of the chunk's valid span into the span: one 16-byte
// copy if the block is whole, else 4-byte copies of its valid samples
__device__ __forceinline__ void copy_block(const float *src, unsigned base, int valid, int b) {
    const int lane = threadIdx.x & 63;
    if (256 * (b + 1) <= valid) {
        lds_dma_x4(src + b * 256 + 4 * lane, base + b * 1024);
    } else {
        for (int q = 4 * b; q * 64 < valid; ++q) {
            const int o = q * 64 + lane;
            if (o < valid) lds_dma_x1(src + o, base + q * 256);
        }
    }
}

// A producer's conversion of its 256-sample blocks b = pw, pw + 4, ... of a chunk's span: per
// wave step eight of them, one E4M3 block per lane (convert_lane_block).  With NEXT, each
// step's blocks are then copied for the next chunk (`nx`) into the span, and after the loop
// those of this producer's blocks past this chunk's span.
template <bool NEXT>
__device__ __forceinline__ void convert_owned8(const FwdArgs &a, const Chunk &ch, float *span,
                                               unsigned char *rows8, int S8, int *codes, float inv_bph, int pw,
                                               int np, const Chunk &nx) {
    const int lane = threadIdx.x & 63;
    const int span_len = (ch.n_frames + a.J - 1) * a.H;
    const int nblk = span_len >> 5, n256 = (span_len + 255) >> 8;
    const int valid = span_valid(a, ch);
    const int pad = S8 - a.H;
    const float *nsrc = a.wave + nx.sample_start;
    const int nvalid = NEXT ? span_valid(a, nx) : 0;
    const unsigned base = __builtin_amdgcn_readfirstlane(lds_addr(span));
    int b0 = pw;
    for (; b0 < n256; b0 += 8 * np) {
        const int fb = 8 * (b0 + np * (lane >> 3)) + (lane & 7);
        // every lane's block before the clip end: the last lane's block is 8 (b0 + 7 np) + 7
        const bool whole = 256 * (b0 + 7 * np + 1) <= valid;
        if (fb < nblk) convert_lane_block<false>(span, valid, whole, fb, rows8 + block_row_byte(fb, inv_bph, pad), codes);
        if constexpr (NEXT) {
            // the blocks just read may be overwritten by the next chunk's copies
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (256 * (b0 + np * u) < nvalid) copy_block(nsrc, base, nvalid, b0 + np * u);
        }
    }
    if constexpr (NEXT) {
        for (; 256 * b0 < nvalid; b0 += np) copy_block(nsrc, base, nvalid, b0);
    }
}

// a producer's copies of its blocks of a chunk's valid span (no conversion pending)
__device__ __forceinline__ void copy_owned8(const FwdArgs &a, const Chunk &ch, float *span, int pw, int np) {
    const int valid = span_valid(a, ch);
    const float *src = a.wave + ch.sample_start;
    const unsigned base = __builtin_amdgcn_readfirstlane(lds_addr(span));
    for (int b = pw; 256 * b < valid; b += np) copy_block(src, base, valid, b);
}

__device__ __forceinline__ Chunk slot_get(const Chunk *slots, int i) {
    Chunk e = slots[i];
    e.sample_start = uniform64(e.sample_start);
    e.sample_end = uniform64(e.sample_end);
    e.out_row = uniform64(e.out_row);
    e.n_frames = __builtin_amdgcn_readfirstlane(e.n_frames);
    e.clip = __builtin_amdgcn_readfirstlane(e.clip);
    return e;
}

template <int NG>
__global__ __launch_bounds__(768) void k_melt_f8b_pc(FwdArgs a, const i32x8 *__restrict__ bq,
                                                    const float *__restrict__ rinv_g, F8BlockTable bt, int S8,
                                                    int buf_bytes, int code_off, int n_codes, int scr_off,
                                                    int rgroups) {
    extern __shared__ float lds_pc[];
    __shared__ __align__(16) Chunk dslot[4];
    __shared__ float rinv_s[8 * 32];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
    const int grp = blockIdx.x % rgroups, gt_n = (a.row_tiles + rgroups - 1) / rgroups;
    const int r0 = grp * gt_n, cnt = min(a.row_tiles - r0, gt_n);
    for (int i = threadIdx.x; i < 32 * cnt; i += blockDim.x) rinv_s[i] = rinv_g[32 * r0 + i];
    const int nc = cnt, np = nw - cnt;             // consumers (one row tile each), producers
    const bool producer = wid >= nc;
    const int pw = wid - nc;
    unsigned char *buf0 = reinterpret_cast<unsigned char *>(lds_pc);
    float *span = lds_pc + scr_off;
    const int bph = a.H >> 5;
    const float inv_bph = 1.0f / (float)bph;
    const int nch = *a.n_chunks;
    const int cstep = gridDim.x / rgroups;
    const int c0 = blockIdx.x / rgroups;
    // codes past a chunk's blocks (read for blocks past a frame, or frames past the chunk) are
    // finite from the start, in both buffers
    for (int i = threadIdx.x; i < n_codes; i += blockDim.x) {
        reinterpret_cast<int *>(buf0 + code_off)[i] = 127;
        reinterpret_cast<int *>(buf0 + buf_bytes + code_off)[i] = 127;
    }
    // prologue: descriptors 0..2 in their slots; the producers copy and convert chunk 0 into
    // buffer 0 and start the copy of chunk 1.  Producers and consumers then run loops of their
    // own (so that neither role's registers are live in the other's), with one barrier per
    // chunk in both.
    if (wid == nc && lane < 3 && c0 + lane * cstep < nch) dslot[lane] = a.chunks[c0 + lane * cstep];
    // the first chunk is copied and converted by every wave (blocks w, w + 12, ...); after a
    // barrier the producers start the copy of the second
    if (c0 < nch) {
        const Chunk ch = read_chunk(a.chunks, c0);
        copy_owned8(a, ch, span, wid, nw);
        async_wait();
        convert_owned8<false>(a, ch, span, buf0, S8, reinterpret_cast<int *>(buf0 + code_off), inv_bph, wid, nw, ch);
    }
    __syncthreads();
    if (producer) {
        if (c0 + cstep < nch) copy_owned8(a, read_chunk(a.chunks, c0 + cstep), span, pw, np);
        for (int it = 0; c0 + it * cstep < nch; ++it) {
            __syncthreads();                       // chunk it converted; buffer (it + 1) & 1 free
            const int c = c0 + it * cstep;
            if (c + cstep >= nch) continue;
            // the next descriptor as two 16-byte values in registers (a Chunk variable
            // assigned under this condition was placed in scratch memory: per-iteration stores
            // that reached HBM and a wait for every outstanding memory operation), loaded
            // through the scalar cache so that storing it waits for no copy
            uint4 nd0 = {}, nd1 = {};
            const bool load_desc = wid == nc && c + 3 * cstep < nch;
            async_wait();                          // this producer's copies of chunk it + 1
            if (load_desc) load_chunk_scalar(a.chunks, c + 3 * cstep, nd0, nd1);
            const Chunk ch1 = slot_get(dslot, (it + 1) & 3);
            unsigned char *rows = buf0 + ((it + 1) & 1) * buf_bytes;
            int *codes = reinterpret_cast<int *>(rows + code_off);
            if (c + 2 * cstep < nch)
                convert_owned8<true>(a, ch1, span, rows, S8, codes, inv_bph, pw, np, slot_get(dslot, (it + 2) & 3));
            else
                convert_owned8<false>(a, ch1, span, rows, S8, codes, inv_bph, pw, np, ch1);
            if (load_desc && lane == 0) {
                uint4 *dst = reinterpret_cast<uint4 *>(dslot + ((it + 3) & 3));
                dst[0] = nd0;
                dst[1] = nd1;
            }
        }
        return;
    }
    const int rt = r0 + wid;
    i32x8 A[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) A[g] = bq[((size_t)rt * NG + g) * 64 + lane];
    // the tile's row unscaling factors in LDS (read in the epilogue, not held in registers):
    // lane half h uses rows 8 q + 4 h .. + 3 of the tile, four consecutive floats per q
    const float *ri = rinv_s + 32 * wid + 4 * (lane >> 5);
    for (int it = 0; c0 + it * cstep < nch; ++it) {
        __syncthreads();                           // chunk it converted; buffer (it + 1) & 1 free
        const Chunk ch = slot_get(dslot, it & 3);
        const unsigned char *rows = buf0 + (it & 1) * buf_bytes;
        const int *codes = reinterpret_cast<const int *>(rows + code_off);
        const int nft = (ch.n_frames + 31) >> 5;
        for (int ft = 0; ft < nft; ++ft) {
            const int f0 = ft * 32 + (lane & 31);
            int off = f0 * S8 + 16 * (lane >> 5);
            asm volatile("" : "+v"(off));
            const unsigned char *q0 = rows + off;
            const int *s0 = codes + f0 * bph + (lane >> 5);
            f32x16 acc = f32x16{}, unused = f32x16{};
            f8b_sweep<NG, false>(A, bt, q0, q0, s0, s0, acc, unused);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 r4 = *(const f32x4 *)(ri + 8 * q);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[4 * q + e] *= r4[e];
            }
            store_tile(a, ch, rt, f0, lane, acc);
        }
    }
}

// ------------------------------------------------------------------ FP8 per-frame scales, producer/consumer
//
// The per-frame FP8 kernel on 12 waves (three per SIMD), arranged as k_melt_f8b_pc: the first
// NC waves (NC = row tiles of the group) are consumers holding one E4M3 basis tile each, the
// other 12 - NC are producers that quantise the next chunk while the consumers multiply this
// one.  A producer takes whole frames (frames p, p + NP, ..., four in flight): frame t of the
// chunk is span samples [tH, tH + N), samples past the clip end 0; a lane holds samples
// 4 u .. 4 u + 3 for its words u = lane + 64 k, the wave reduces max|x| over them, forms
// s_t = 448 / max (1 for a silent frame) and writes the frame's E4M3 image row (zeros past N).
// The FP32 span and the image are double buffered (chunk k in buffer k % 2): the copies of
// chunk it + 2 (256-sample blocks p, p + NP, ...) are issued at the start of iteration it into
// the buffer of chunk it, which every producer finished before the barrier that started the
// iteration, and each producer waits for its own at the end of the iteration (a producer
// reads samples other producers copied, so the wait precedes the next barrier).  One barrier
// per chunk; descriptors through a four-slot LDS ring.  The scales and the unscaling epilogue
// are those of k_melt_f8_as.  Per chunk the quantisation of whole frames (a wave-wide maximum
// per frame) costs the producers more than the all-wave kernel's block-maxima passes: at
// 80 Mel bins and n_fft 400 this kernel is slower than k_melt_f8_as, so it is the variant for
// row groups (more than 128 Mel bins), which k_melt_f8_as does not take.  Needs hop and frame
// multiples of 4 samples.
template <int NG>
__global__ __launch_bounds__(768) void k_melt_f8_pc(FwdArgs a, const i32x8 *__restrict__ bq,
                                                   const float *__restrict__ rinv_g, int N, int bf, int img_bytes,
                                                   int span_off, int span_bytes, int rgroups) {
    extern __shared__ float lds_fpc[];
    __shared__ __align__(16) Chunk dslot[4];
    __shared__ __align__(16) float rinv_s[8 * 32];
    constexpr int KP = NG * 64;             // padded frame length in the E4M3 image
    constexpr int SQ = KP + 16;             // row stride (bytes): conflict-free 16-byte reads
    constexpr int WPF = KP / 4;             // image words per frame
    constexpr int KW = (WPF + 63) / 64;     // words per lane
    constexpr int FT = 4;                   // frames in flight per producer wave
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
    const int grp = blockIdx.x % rgroups, gt_n = (a.row_tiles + rgroups - 1) / rgroups;
    const int r0 = grp * gt_n, cnt = min(a.row_tiles - r0, gt_n);
    const int nc = cnt, np = nw - cnt;             // consumers (one row tile each), producers
    const bool producer = wid >= nc;
    const int pw = wid - nc;
    for (int i = threadIdx.x; i < 32 * cnt; i += blockDim.x) rinv_s[i] = rinv_g[32 * r0 + i];
    unsigned char *img0 = reinterpret_cast<unsigned char *>(lds_fpc);
    float *span0 = reinterpret_cast<float *>(img0 + span_off);
    const bool vec = (a.H & 3) == 0 && (N & 3) == 0;
    const int nch = *a.n_chunks;
    const int cstep = gridDim.x / rgroups;
    const int c0 = blockIdx.x / rgroups;
    // image rows of chunk frames [w0, ...) step ws, of buffer `img` (scales after the rows)
    auto quantise = [&](const Chunk &ch, const float *span, unsigned char *img, int w0, int ws) {
        const int valid = span_valid(a, ch);
        float *sinv = reinterpret_cast<float *>(img + bf * SQ);
        for (int t0 = w0; t0 < ch.n_frames; t0 += FT * ws) {
            f32x4 x[FT][KW];
#pragma unroll
            for (int h = 0; h < FT; ++h) {
                const int t = t0 + h * ws;
#pragma unroll
                for (int k = 0; k < KW; ++k) x[h][k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                if (t >= ch.n_frames) continue;
                const int base = t * a.H;
                const bool whole = vec && base + N <= valid;
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    const int n0 = 4 * (lane + 64 * k), o = base + n0;
                    if (whole) {
                        if (n0 < N) x[h][k] = *(const f32x4 *)(span + o);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) x[h][k][e] = (n0 + e < N && o + e < valid) ? span[o + e] : 0.0f;
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < FT; ++h) {
                const int t = t0 + h * ws;              // wave-uniform
                if (t >= ch.n_frames) break;
                float m = 0.0f;
#pragma unroll
                for (int k = 0; k < KW; ++k)
                    m = fmaxf(m, fmaxf(fmaxf(fabsf(x[h][k][0]), fabsf(x[h][k][1])),
                                       fmaxf(fabsf(x[h][k][2]), fabsf(x[h][k][3]))));
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
                const float sc = m > 0.0f ? __fdiv_rn(448.0f, m) : 1.0f;   // inverted in the epilogue
                if (lane == 0) sinv[t] = sc;
                unsigned *dst = reinterpret_cast<unsigned *>(img + t * SQ);
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    const int u = lane + 64 * k;
                    if (u < WPF)
                        dst[u] = fp8x4(__fmul_rn(x[h][k][0], sc), __fmul_rn(x[h][k][1], sc),
                                       __fmul_rn(x[h][k][2], sc), __fmul_rn(x[h][k][3], sc));
                }
            }
        }
    };
    // prologue: descriptors 0..2 in their slots; every wave copies chunk 0 (blocks w, w + 12,
    // ...) into span 0, the producers also chunk 1 into span 1; after a barrier every wave
    // quantises frames of chunk 0 into image 0
    if (wid == nc && lane < 3 && c0 + lane * cstep < nch) dslot[lane] = a.chunks[c0 + lane * cstep];
    if (c0 < nch) copy_owned8(a, read_chunk(a.chunks, c0), span0, wid, nw);
    if (producer && c0 + cstep < nch)
        copy_owned8(a, read_chunk(a.chunks, c0 + cstep), reinterpret_cast<float *>(img0 + span_off + span_bytes), pw,
                    np);
    async_wait();
    __syncthreads();
    if (c0 < nch) quantise(read_chunk(a.chunks, c0), span0, img0, wid, nw);
    if (producer) {
        for (int it = 0; c0 + it * cstep < nch; ++it) {
            __syncthreads();                       // chunk it quantised; image (it + 1) & 1 free
            const int c = c0 + it * cstep;
            if (c + cstep >= nch) continue;
            float *span_nx = reinterpret_cast<float *>(img0 + span_off + (it & 1) * span_bytes);
            const float *span_cur = reinterpret_cast<const float *>(img0 + span_off + ((it + 1) & 1) * span_bytes);
            // chunk it + 2 into the span chunk it used
            if (c + 2 * cstep < nch) copy_owned8(a, slot_get(dslot, (it + 2) & 3), span_nx, pw, np);
            uint4 nd0 = {}, nd1 = {};              // the next descriptor (scalar loads), in registers
            const bool load_desc = wid == nc && c + 3 * cstep < nch;
            if (load_desc) load_chunk_scalar(a.chunks, c + 3 * cstep, nd0, nd1);
            quantise(slot_get(dslot, (it + 1) & 3), span_cur, img0 + ((it + 1) & 1) * img_bytes, pw, np);
            if (load_desc && lane == 0) {
                uint4 *dst = reinterpret_cast<uint4 *>(dslot + ((it + 3) & 3));
                dst[0] = nd0;
                dst[1] = nd1;
            }
            async_wait();                          // this producer's copies of chunk it + 2
        }
        return;
    }
    const int rt = r0 + wid;
    i32x8 A[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) A[g] = bq[((size_t)rt * NG + g) * 64 + lane];
    // the tile's row unscaling factors in LDS (read in the epilogue, not held in registers):
    // lane half h uses rows 8 q + 4 h .. + 3 of the tile, four consecutive floats per q
    const float *ri = rinv_s + 32 * wid + 4 * (lane >> 5);
    for (int it = 0; c0 + it * cstep < nch; ++it) {
        __syncthreads();                           // chunk it quantised; image (it + 1) & 1 free
        const Chunk ch = slot_get(dslot, it & 3);
        const unsigned char *xq = img0 + (it & 1) * img_bytes;
        const float *sinv = reinterpret_cast<const float *>(xq + bf * SQ);
        const int nft = (ch.n_frames + 31) >> 5;
        for (int ft = 0; ft < nft; ++ft) {
            const int f = ft * 32 + (lane & 31);
            int off = f * SQ + 32 * (lane >> 5);
            asm volatile("" : "+v"(off));
            const unsigned char *q0 = xq + off;
            f32x16 acc = f32x16{};
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const uint4 bl = *(const uint4 *)(q0 + 64 * g), bh = *(const uint4 *)(q0 + 64 * g + 16);
                const i32x8 B = {(int)bl.x, (int)bl.y, (int)bl.z, (int)bl.w, (int)bh.x, (int)bh.y, (int)bh.z, (int)bh.w};
                acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[g], B, acc, 0, 0, 0, 127, 0, 127);
            }
            const float is = f < ch.n_frames ? 1.0f / sinv[f] : 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 r4 = *(const f32x4 *)(ri + 8 * q);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[4 * q + e] = acc[4 * q + e] * (is * r4[e]);
            }
            store_tile(a, ch, rt, f, lane, acc);
        }
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

// LDS of the per-frame producer/consumer kernel: two images (rows then the frame scales) and
// two FP32 spans, each 16-byte aligned
static size_t f8_pc_img_bytes(const Plan &p, int bf) {
    const int ng8 = (p.N + 63) / 64;
    return ((size_t)bf * (ng8 * 64 + 16) + (size_t)bf * 4 + 15) & ~size_t(15);
}
static size_t f8_pc_span_bytes(const Plan &p, int bf) {
    return ((size_t)(bf + p.geo32.J - 1) * p.H * 4 + 15) & ~size_t(15);
}
size_t f8_pc_lds_bytes(const Plan &p, int bf) { return 2 * f8_pc_img_bytes(p, bf) + 2 * f8_pc_span_bytes(p, bf); }

template <int NG>
static melt_status launch_f8_pc_ng(Plan &p, const FwdArgs &a, size_t lds, int grid, int bf, int rg, hipStream_t s) {
    allow_lds(k_melt_f8_pc<NG>, 4 * sizeof(Chunk) + 8 * 32 * 4);
    const size_t img = f8_pc_img_bytes(p, bf);
    k_melt_f8_pc<NG><<<grid, 768, lds, s>>>(a, (const i32x8 *)p.d_pack_f8, p.d_rowscale, p.N, bf, (int)img,
                                            (int)(2 * img), (int)f8_pc_span_bytes(p, bf), rg);
    return hip_check(hipGetLastError(), "melt f8 producer/consumer launch");
}

template <int NG>
static melt_status launch_f8_as(Plan &p, const FwdArgs &a, size_t lds, int grid, int bf, hipStream_t s) {
    allow_lds(k_melt_f8_as<NG>, kRingBytes);
    const WaveLayout w = wave_layout(p);
    k_melt_f8_as<NG><<<grid, 64 * w.waves, lds, s>>>(a, (const i32x8 *)p.d_pack_f8, p.d_rowscale, p.N, bf,
                                                     (int)(f8_as_scratch_offset(p, bf) / 4), w.full, w.psplit);
    return hip_check(hipGetLastError(), "melt f8 lds-dma launch");
}

// LDS of the block-scaled FP8 kernel at bf frames per chunk: E4M3 hop-block rows (stride
// f8b_stride bytes), block codes, then the FP32 span (16-byte aligned)
int f8b_stride(const Plan &p) { return lds_stride(p.H, 1); }
static size_t f8b_codes(const Plan &p, int bf) {
    const int bph = p.H / 32, ng8 = (p.N + 63) / 64;
    // the chunk's blocks, and the codes read for blocks past the last frame of a tile
    return (size_t)std::max((bf + p.geo32.J - 1) * bph, (bf - 1) * bph + 2 * ng8);
}
static size_t f8b_codes_offset(const Plan &p, int bf) {
    return ((size_t)(bf + p.geo32.J - 1) * f8b_stride(p) + 15) & ~size_t(15);
}
static size_t f8b_span_offset(const Plan &p, int bf) {
    return (f8b_codes_offset(p, bf) + f8b_codes(p, bf) * 4 + 15) & ~size_t(15);
}
size_t f8b_lds_bytes(const Plan &p, int bf) {
    return f8b_span_offset(p, bf) + (size_t)(bf + p.geo32.J - 1) * p.H * 4;
}

template <int NG>
static melt_status launch_f8b_ng(Plan &p, const FwdArgs &a, const F8BlockTable &bt, size_t lds, int grid, int bf,
                                 int rg, hipStream_t s) {
    allow_lds(k_melt_f8b_as<NG>, kRingBytes);
    const WaveLayout w = wave_layout(p);
    k_melt_f8b_as<NG><<<grid, 64 * w.waves, lds, s>>>(
        a, (const i32x8 *)p.d_pack_f8, p.d_rowscale, bt, f8b_stride(p), (int)(f8b_codes_offset(p, bf) / 4),
        (int)f8b_codes(p, bf), (int)(f8b_span_offset(p, bf) / 4), rg);
    return hip_check(hipGetLastError(), "melt f8 block-scaled launch");
}

// LDS of the producer/consumer form: two row/code buffers, then the FP32 span
static size_t f8b_buf_bytes(const Plan &p, int bf) {
    return f8b_codes_offset(p, bf) + ((f8b_codes(p, bf) * 4 + 15) & ~size_t(15));
}
size_t f8b_pc_lds_bytes(const Plan &p, int bf) {
    return 2 * f8b_buf_bytes(p, bf) + (size_t)(bf + p.geo32.J - 1) * p.H * 4;
}
// its static LDS: the descriptor slots and the row unscaling factors of a row group
size_t f8b_pc_static_bytes() { return 4 * sizeof(Chunk) + 8 * 32 * sizeof(float); }

template <int NG>
static melt_status launch_f8b_pc_ng(Plan &p, const FwdArgs &a, const F8BlockTable &bt, size_t lds, int grid, int bf,
                                    int rg, hipStream_t s) {
    allow_lds(k_melt_f8b_pc<NG>, (int)f8b_pc_static_bytes());
    k_melt_f8b_pc<NG><<<grid, 768, lds, s>>>(a, (const i32x8 *)p.d_pack_f8, p.d_rowscale, bt, f8b_stride(p),
                                             (int)f8b_buf_bytes(p, bf), (int)f8b_codes_offset(p, bf),
                                             (int)f8b_codes(p, bf), (int)(2 * f8b_buf_bytes(p, bf) / 4), rg);
    return hip_check(hipGetLastError(), "melt f8 block-scaled producer/consumer launch");
}

melt_status launch_melt_f8b(Plan &p, const FwdTask &t, int bf, bool pc) {
    if (p.H % 32 != 0) return set_error(MELT_E_UNSUPPORTED, "FP8 with 32-sample block scales needs hop % 32 == 0");
    const int ng8 = (p.N + 63) / 64;
    if (ng8 != 4 && ng8 != 7 && ng8 != 8 && ng8 != 16)
        return set_error(MELT_E_UNSUPPORTED, "FP8 kernel supports n_fft in (192, 256], (384, 512], (960, 1024]");
    const Geometry &g = p.geo32;
    const FwdArgs a = make_args(p, g, lds_stride(g.Hp, 4), t);
    const size_t lds = pc ? f8b_pc_lds_bytes(p, bf) : f8b_lds_bytes(p, bf);
    if (lds + (pc ? f8b_pc_static_bytes() : (size_t)kRingBytes) > (size_t)kMaxLds)
        return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS for the FP8 kernel");
    F8BlockTable bt{};
    const int S8 = f8b_stride(p);
    for (int i = 0; i < 2 * ng8; ++i) {
        const int n = 32 * i;
        bt.off[i] = n < p.N ? (n / p.H) * S8 + n % p.H : 0;
    }
    // one persistent set of workgroups per row group, one workgroup per CU (its eight waves
    // take two waves' registers per SIMD)
    const int rg = row_groups(p);
    const int per_group =
        (int)std::max<int64_t>(1, std::min<int64_t>(t.est_chunks, ((int64_t)p.cu_count + rg - 1) / rg));
    const int grid = per_group * rg;
    if (pc) {
        switch (ng8) {
        case 4: return launch_f8b_pc_ng<4>(p, a, bt, lds, grid, bf, rg, t.stream);
        case 7: return launch_f8b_pc_ng<7>(p, a, bt, lds, grid, bf, rg, t.stream);
        case 8: return launch_f8b_pc_ng<8>(p, a, bt, lds, grid, bf, rg, t.stream);
        default: return set_error(MELT_E_UNSUPPORTED, "producer/consumer FP8 kernel: n_fft above 512");
        }
    }
    switch (ng8) {
    case 4: return launch_f8b_ng<4>(p, a, bt, lds, grid, bf, rg, t.stream);
    case 7: return launch_f8b_ng<7>(p, a, bt, lds, grid, bf, rg, t.stream);
    case 8: return launch_f8b_ng<8>(p, a, bt, lds, grid, bf, rg, t.stream);
    default: return launch_f8b_ng<16>(p, a, bt, lds, grid, bf, rg, t.stream);
    }
}

melt_status launch_melt_f8_pc(Plan &p, const FwdTask &t, int bf) {
    const int ng8 = (p.N + 63) / 64;
    if (p.H % 4 != 0 || p.N % 4 != 0)
        return set_error(MELT_E_UNSUPPORTED, "producer/consumer FP8 kernel: hop and n_fft must be multiples of 4");
    const int rg = row_groups(p), gt_n = (p.row_tiles + rg - 1) / rg;
    if (gt_n > 8) return set_error(MELT_E_UNSUPPORTED, "producer/consumer FP8 kernel: row group too large");
    const size_t lds = f8_pc_lds_bytes(p, bf);
    if (lds + 4 * sizeof(Chunk) + 8 * 32 * 4 > (size_t)kMaxLds)
        return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS for the FP8 kernel");
    const Geometry &g = p.geo32;
    const FwdArgs a = make_args(p, g, lds_stride(g.Hp, 4), t);
    // one persistent set of workgroups per row group, one workgroup per CU
    const int per_group =
        (int)std::max<int64_t>(1, std::min<int64_t>(t.est_chunks, ((int64_t)p.cu_count + rg - 1) / rg));
    const int grid = per_group * rg;
    switch (ng8) {
    case 4: return launch_f8_pc_ng<4>(p, a, lds, grid, bf, rg, t.stream);
    case 7: return launch_f8_pc_ng<7>(p, a, lds, grid, bf, rg, t.stream);
    case 8: return launch_f8_pc_ng<8>(p, a, lds, grid, bf, rg, t.stream);
    default: return set_error(MELT_E_UNSUPPORTED, "producer/consumer FP8 kernel: n_fft in (192, 256] or (384, 512]");
    }
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
