// MelT forward on gfx950: implicit framing in LDS + basis GEMM on MFMA + fused energy/log.
//
// Eq. (dmp_projection): R = X W^(r)T, I = X W^(i)T; Eq. (dmp_matrix_energy): S = R.R + I.I;
// Eq. (meltf): out = log(S + eps).  The GEMM is computed transposed, Y^T = W X^T, so that
// MFMA A operand = basis rows and B operand = frames, and the accumulator of one lane holds
// one frame's values for 16 basis rows.  The basis rows of a 32-row tile are permuted so
// that those 16 rows are the cos/sin pairs of 8 consecutive Mel bins: R^2 + I^2 is formed
// in-lane and each lane writes 8 consecutive outputs (two 16-byte stores).
//
// Frames are never materialised.  A chunk of up to BF consecutive frames of one clip needs
// the contiguous sample span [start, start + (BF - 1) H + N); it is staged once into LDS
// as "hop-block" rows (row r = samples [rH, rH + H), padded), and frame t is the
// concatenation of the first L_j samples of rows t + j, j = 0..J-1.  Reading the B operand
// of k-group (j, c) for the 32 frames of a tile is then 32 rows at one column: the padded
// row stride makes those reads bank-conflict free even though frames overlap.
#include "melt_internal.h"

namespace melt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

struct GroupTableBig {
    int n;
    int lds_off[512];
};

constexpr int kChunkF32 = 128;   // frames per chunk of the frame-split kernels (4 waves x 32)

// ------------------------------------------------------------------ schedule

// One workgroup: prefix sums over the clips of frame counts and chunk counts, then the
// chunk table.  n_chunks receives min(total, cap).
__global__ __launch_bounds__(1024) void k_schedule(const int64_t *__restrict__ off, int n_clips, int N,
                                                   int H, int bf, Chunk *__restrict__ tab, int64_t cap,
                                                   int *__restrict__ n_out) {
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
        const int64_t T = (L >= N) ? 1 + (L - N) / H : 0;
        const int64_t K = (T + bf - 1) / bf;
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
            Chunk e;
            e.sample_start = st + k * bf * (int64_t)H;
            e.sample_end = st + L;
            e.out_row = fb + k * bf;
            e.n_frames = (int)((T - k * bf) < bf ? (T - k * bf) : bf);
            e.clip = c;
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

__global__ __launch_bounds__(1024) void k_frame_offsets(const int64_t *__restrict__ off, int n_clips, int N,
                                                        int H, int64_t *__restrict__ fo) {
    __shared__ int64_t sf[1024];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n_clips; base += 1024) {
        const int c = base + tid;
        int64_t L = 0;
        if (c < n_clips) L = off[c + 1] - off[c];
        const int64_t T = (L >= N) ? 1 + (L - N) / H : 0;
        sf[tid] = T;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int64_t v = tid >= d ? sf[tid - d] : 0;
            __syncthreads();
            sf[tid] += v;
            __syncthreads();
        }
        if (c < n_clips) fo[c] = carry + sf[tid] - T;
        __syncthreads();
        if (tid == 1023) carry += sf[1023];
        __syncthreads();
    }
    if (tid == 0) fo[n_clips] = carry;
}

// ------------------------------------------------------------------ basis packing

// Row permutation of a 32-row tile.  The 32x32 MFMA accumulator puts row
// i = 8 g + 4 h + q (g = 0..3, h = lane / 32, q = 0..3) in register 4 g + q of lane half h.
// Row i carries Mel bin 8 h + 2 g + q / 2 of the tile, cosine for even q, sine for odd q,
// so register pairs (4g, 4g+1) and (4g+2, 4g+3) are (R, I) of consecutive Mel bins.
__device__ inline void tile_row_to_mel(int i, int &mel_local, int &part) {
    const int g = i >> 3, h = (i >> 2) & 1, q = i & 3;
    mel_local = 8 * h + 2 * g + (q >> 1);
    part = q & 1;
}

// Value of packed element (rt, group, lane, e): basis row (part, mel) at column
// k = j H + c + (group_size / 2) * (lane / 32) + e, zero outside the segment / N / M.
__device__ inline float packed_value(const float *__restrict__ b32, int M, int N, int H, int rt, int j, int c,
                                     int half_group, int lane, int e) {
    int mel_local, part;
    tile_row_to_mel(lane & 31, mel_local, part);
    const int mel = rt * 16 + mel_local;
    const int col = c + half_group * (lane >> 5) + e;
    const int Lj = min(H, N - j * H);
    if (mel >= M || col >= Lj) return 0.0f;
    return b32[(size_t)(part * M + mel) * N + j * H + col];
}

__device__ inline unsigned short f32_to_bf16_bits(float x) {
    __bf16 b = (__bf16)x;
    return __builtin_bit_cast(unsigned short, b);
}
__device__ inline unsigned short f32_to_f16_bits(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(unsigned short, h);
}
__device__ inline float bf16_bits_to_f32(unsigned short u) {
    return __builtin_bit_cast(float, (unsigned)u << 16);
}

// FP32 pack: [rt][group][lane][4]
__global__ void k_pack_f32(const float *__restrict__ b32, int M, int N, int H, const int *__restrict__ seg,
                           const int *__restrict__ col, int NG, int RT, float *__restrict__ out) {
    const int64_t total = (int64_t)RT * NG * 64 * 4;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = i & 3;
        const int lane = (i >> 2) & 63;
        const int64_t tg = i >> 8;
        const int g = (int)(tg % NG), rt = (int)(tg / NG);
        out[i] = packed_value(b32, M, N, H, rt, seg[g], col[g], 4, lane, e);
    }
}

// 16-bit pack: [rt][group][lane][8]; kind 0 = bf16, 1 = fp16, 2 = bf16 low part of the split
__global__ void k_pack_h16(const float *__restrict__ b32, int M, int N, int H, const int *__restrict__ seg,
                           const int *__restrict__ col, int NG, int RT, int kind, unsigned short *__restrict__ out) {
    const int64_t total = (int64_t)RT * NG * 64 * 8;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = i & 7;
        const int lane = (i >> 3) & 63;
        const int64_t tg = i >> 9;
        const int g = (int)(tg % NG), rt = (int)(tg / NG);
        const float v = packed_value(b32, M, N, H, rt, seg[g], col[g], 8, lane, e);
        unsigned short r;
        if (kind == 0) {
            r = f32_to_bf16_bits(v);
        } else if (kind == 1) {
            r = f32_to_f16_bits(v);
        } else {
            const float hi = bf16_bits_to_f32(f32_to_bf16_bits(v));
            r = f32_to_bf16_bits(v - hi);
        }
        out[i] = r;
    }
}

// ------------------------------------------------------------------ shared device pieces

// A chunk-table entry read into scalar registers (every lane of a workgroup uses the same
// chunk, so buffer descriptors built from it need no waterfall loop).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ Chunk read_chunk(const Chunk *tab, int c) {
    Chunk e = tab[c];
    e.sample_start = uniform64(e.sample_start);
    e.sample_end = uniform64(e.sample_end);
    e.out_row = uniform64(e.out_row);
    e.n_frames = __builtin_amdgcn_readfirstlane(e.n_frames);
    e.clip = __builtin_amdgcn_readfirstlane(e.clip);
    return e;
}

struct FwdArgs {
    const float *wave;
    const Chunk *chunks;
    const int *n_chunks;
    float *out;
    float *proj;
    int64_t n_frames;
    int M, J, H, Hp, S;    // S = LDS row stride in elements
    int row_tiles;
    int out_kind;
    float eps;
    float invH;            // 1 / H rounded to FP32 (row index of a span position)
};

__device__ inline float out_map(float S, int kind, float eps) {
    switch (kind) {
    case MELT_OUT_LOG_POWER: return logf(S + eps);
    case MELT_OUT_LOG_MAGNITUDE: return logf(sqrtf(S) + eps);
    case MELT_OUT_POWER: return S;
    default: return sqrtf(S);
    }
}

// Writes one 32-frame x 16-Mel tile from the accumulator of lane `lane` (frame
// `f_local` of the chunk).  Register pairs (4g, 4g+1), (4g+2, 4g+3) are (R, I) of Mel bins
// 8h + 2g and 8h + 2g + 1 of the tile.
__device__ inline void store_tile(const FwdArgs &a, const Chunk &ch, int rt, int f_local, int lane,
                                  const f32x16 &acc) {
    if (f_local >= ch.n_frames) return;
    const int64_t row = ch.out_row + f_local;
    if (row >= a.n_frames) return;
    const int h = lane >> 5;
    const int mel0 = rt * 16 + 8 * h;
    if (mel0 >= a.M) return;
    float v[8];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        v[2 * g] = out_map(acc[4 * g] * acc[4 * g] + acc[4 * g + 1] * acc[4 * g + 1], a.out_kind, a.eps);
        v[2 * g + 1] = out_map(acc[4 * g + 2] * acc[4 * g + 2] + acc[4 * g + 3] * acc[4 * g + 3], a.out_kind, a.eps);
    }
    float *o = a.out + row * a.M + mel0;
    if (mel0 + 8 <= a.M && (a.M & 3) == 0) {
        *(f32x4 *)o = f32x4{v[0], v[1], v[2], v[3]};
        *(f32x4 *)(o + 4) = f32x4{v[4], v[5], v[6], v[7]};
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (mel0 + e < a.M) o[e] = v[e];
    }
    if (a.proj) {
        float *p = a.proj + row * (2 * a.M) + 2 * mel0;
        if (mel0 + 8 <= a.M && (a.M & 1) == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) *(f32x4 *)(p + 4 * q) = f32x4{acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                if (mel0 + e / 2 < a.M) p[e] = acc[e];
        }
    }
}

// Operand formats of the staged frames.  store writes one element; store4 writes four
// consecutive ones (i a multiple of 4).
__device__ __forceinline__ unsigned pack2(unsigned short lo, unsigned short hi) { return lo | ((unsigned)hi << 16); }

struct ConvF32 {
    typedef float elem_t;
    __device__ static void store(float *l, int i, float v, int) { l[i] = v; }
    __device__ static void store4(float *l, int i, f32x4 v, int) { *(f32x4 *)(l + i) = v; }
};
struct ConvBF16 {
    typedef unsigned short elem_t;
    __device__ static void store(unsigned short *l, int i, float v, int) { l[i] = f32_to_bf16_bits(v); }
    __device__ static void store4(unsigned short *l, int i, f32x4 v, int) {
        *(uint2 *)(l + i) = uint2{pack2(f32_to_bf16_bits(v[0]), f32_to_bf16_bits(v[1])),
                                  pack2(f32_to_bf16_bits(v[2]), f32_to_bf16_bits(v[3]))};
    }
};
struct ConvF16 {
    typedef unsigned short elem_t;
    __device__ static void store(unsigned short *l, int i, float v, int) { l[i] = f32_to_f16_bits(v); }
    __device__ static void store4(unsigned short *l, int i, f32x4 v, int) {
        *(uint2 *)(l + i) = uint2{pack2(f32_to_f16_bits(v[0]), f32_to_f16_bits(v[1])),
                                  pack2(f32_to_f16_bits(v[2]), f32_to_f16_bits(v[3]))};
    }
};
// split-bf16: the high part at [i], the low part at [i + lo_off]
struct ConvBF16X3 {
    typedef unsigned short elem_t;
    __device__ static void store(unsigned short *l, int i, float v, int lo_off) {
        const unsigned short hb = f32_to_bf16_bits(v);
        l[i] = hb;
        l[i + lo_off] = f32_to_bf16_bits(v - bf16_bits_to_f32(hb));
    }
    __device__ static void store4(unsigned short *l, int i, f32x4 v, int lo_off) {
        unsigned short h[4], r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            h[e] = f32_to_bf16_bits(v[e]);
            r[e] = f32_to_bf16_bits(v[e] - bf16_bits_to_f32(h[e]));
        }
        *(uint2 *)(l + i) = uint2{pack2(h[0], h[1]), pack2(h[2], h[3])};
        *(uint2 *)(l + i + lo_off) = uint2{pack2(r[0], r[1]), pack2(r[2], r[3])};
    }
};

// Register staging of a chunk's contiguous sample span [start, start + (n_frames + J - 1) H):
// element u of a thread is span position o = tid + u * NT, so every load instruction of a
// wave reads 64 consecutive samples.  span_load issues all PRE loads at once (one memory
// round trip); span_store scatters them into the padded hop-block rows (row o / H, column
// o % H).  Samples at or past the clip end read as 0.
template <int PRE, int NT>
__device__ __forceinline__ void span_load(const FwdArgs &a, const Chunk &ch, float (&pf)[PRE]) {
    // buffer descriptor over [start, min(start + span, clip end)): loads past it return 0,
    // so the clip end needs no branch; one VGPR offset serves all PRE loads
    const int64_t start = ch.sample_start;
    const int64_t span = (int64_t)(ch.n_frames + a.J - 1) * a.H;
    const int64_t lim = ch.sample_end - start < span ? ch.sample_end - start : span;
    const int records = (int)(lim > 0 ? lim * 4 : 0);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(a.wave + start), (short)0, records, 0x00020000);
    const int voff = (int)threadIdx.x * 4;
#pragma unroll
    for (int u = 0; u < PRE; ++u)
        pf[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, u * NT * 4, 0));
}

__device__ __forceinline__ int span_row(const FwdArgs &a, int o) {
    int r = (int)(((float)o + 0.5f) * a.invH);
    const int c = o - r * a.H;
    r += (c >= a.H) - (c < 0);
    return r;
}

template <class Conv, int PRE, int NT>
__device__ __forceinline__ void span_store(const FwdArgs &a, const Chunk &ch, const float (&pf)[PRE],
                                           typename Conv::elem_t *lds, int lo_off) {
    const int span = (ch.n_frames + a.J - 1) * a.H;
    if (span >= PRE * NT) {         // whole register tile valid: no per-element branch
#pragma unroll
        for (int u = 0; u < PRE; ++u) {
            const int o = (int)threadIdx.x + u * NT;
            const int r = span_row(a, o);
            Conv::store(lds, r * a.S + (o - r * a.H), pf[u], lo_off);
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
        const int o = (int)threadIdx.x + u * NT;
        if (o < span) {
            const int r = span_row(a, o);
            Conv::store(lds, r * a.S + (o - r * a.H), pf[u], lo_off);
        }
    }
}

// Zero the pad columns [H, Hp) of `rows` LDS rows (never written by span_store).
template <class Conv>
__device__ __forceinline__ void zero_pad_columns(const FwdArgs &a, int rows, typename Conv::elem_t *lds, int nthreads,
                                                 int lo_off) {
    const int w = a.Hp - a.H;
    if (w <= 0) return;
    for (int i = threadIdx.x; i < rows * w; i += nthreads) {
        const int r = i / w, c = a.H + (i - r * w);
        Conv::store(lds, r * a.S + c, 0.0f, lo_off);
    }
}

// Staging without the register pipeline (the 16-bit kernels): batches of U loads per thread.
template <class Conv, int U>
__device__ __forceinline__ void stage_span(const FwdArgs &a, const Chunk &ch, typename Conv::elem_t *lds,
                                           int nthreads, int lo_off) {
    const int span = (ch.n_frames + a.J - 1) * a.H;
    for (int base = threadIdx.x; base < span; base += U * nthreads) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int o = base + u * nthreads;
            const int64_t s = ch.sample_start + o;
            v[u] = (o < span && s < ch.sample_end) ? a.wave[s] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int o = base + u * nthreads;
            if (o < span) {
                const int r = span_row(a, o);
                Conv::store(lds, r * a.S + (o - r * a.H), v[u], lo_off);
            }
        }
    }
}

// ------------------------------------------------------------------ direct-to-LDS staging
// The chunk's contiguous sample span is copied HBM -> LDS by global_load_lds_dword: each
// wave instruction moves 64 consecutive samples straight into LDS with no registers, so
// the copy of chunk c+1 runs while the MFMAs of chunk c execute.  Positions at or past
// `valid` (the span clipped to the clip end) are not loaded; consumers read them as 0.
__device__ __forceinline__ int span_valid(const FwdArgs &a, const Chunk &ch) {
    const int span = (ch.n_frames + a.J - 1) * a.H;
    int64_t lim = ch.sample_end - ch.sample_start;
    lim = lim < 0 ? 0 : lim;
    return (int)(lim < span ? lim : span);
}

// The copies are issued with inline assembly: the compiler does not track them, so it adds no
// wait for them before the LDS reads of the MFMA loop (which never touch the scratch area);
// async_wait and a barrier order them before the scratch is read.  M0 holds the wave's LDS
// destination; one wait state separates its write from the copy.
__device__ __forceinline__ unsigned lds_addr(const void *p) {
    return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

__device__ __forceinline__ void lds_dma_x4(const float *g, unsigned lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds) : "memory", "m0");
}

__device__ __forceinline__ void lds_dma_x1(const float *g, unsigned lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off" ::"v"(g), "s"(lds) : "memory", "m0");
}

// 16-byte copies (256 samples per wave instruction) over the whole blocks of the valid span,
// then 4-byte copies over its last partial block, so no lane reads past the clip end.
__device__ __forceinline__ void async_span(const FwdArgs &a, const Chunk &ch, float *scratch) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
    const int valid = span_valid(a, ch);
    const float *src = a.wave + ch.sample_start;
    const unsigned base = __builtin_amdgcn_readfirstlane(lds_addr(scratch));
    const int nfull = valid >> 8;
    for (int b = wid; b < nfull; b += nw) lds_dma_x4(src + b * 256 + 4 * lane, base + b * 1024);
    for (int b = 4 * nfull + wid; b * 64 < valid; b += nw) {
        const int o = b * 64 + lane;
        if (o < valid) lds_dma_x1(src + o, base + b * 256);
    }
}

__device__ __forceinline__ void async_wait() {
    __builtin_amdgcn_s_waitcnt(0);     // this wave's direct-to-LDS copies have landed
}

// scratch (contiguous span) -> padded hop-block rows in the kernel's operand format.  With
// H a multiple of 4, four consecutive samples never straddle a row: one 16-byte LDS read and
// one vector write per thread and step.
template <class Conv>
__device__ __forceinline__ void convert_span(const FwdArgs &a, const Chunk &ch, const float *scratch,
                                             typename Conv::elem_t *rows, int lo_off) {
    const int span = (ch.n_frames + a.J - 1) * a.H;
    const int valid = span_valid(a, ch);
    if ((a.H & 3) == 0) {
        for (int o = 4 * (int)threadIdx.x; o < span; o += 4 * (int)blockDim.x) {
            f32x4 v = *(const f32x4 *)(scratch + o);
            if (o + 4 > valid) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (o + e >= valid) v[e] = 0.0f;
            }
            const int r = span_row(a, o);
            Conv::store4(rows, r * a.S + (o - r * a.H), v, lo_off);
        }
        return;
    }
    for (int o = threadIdx.x; o < span; o += blockDim.x) {
        const float v = o < valid ? scratch[o] : 0.0f;
        const int r = span_row(a, o);
        Conv::store(rows, r * a.S + (o - r * a.H), v, lo_off);
    }
}

// ------------------------------------------------------------------ FP32 frame-split kernel
//
// 4 waves, one per SIMD; each wave owns 32 frames of the 128-frame chunk and computes all
// Mel bins for them, in blocks of RTB row tiles (RTB accumulators of 16 registers).  The
// basis is streamed from L2 in fragment order (one 16-byte load per row tile per 8-wide
// k-group, shared by the 4 waves through L1) and prefetched one group ahead.  While the
// MFMA loop of chunk c runs, the sample span of the workgroup's next chunk is already in
// flight into registers (PRE per thread); it is written to LDS after the loop.
template <int RTB, int PRE>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
void k_melt_f32_fs(FwdArgs a, const f32x4 *__restrict__ bpack, int NG) {
    extern __shared__ float lds[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nch = *a.n_chunks;
    const int GH = a.Hp / 8;     // k-groups per full hop segment
    zero_pad_columns<ConvF32>(a, kChunkF32 + a.J - 1, lds, 256, 0);
    // basis as a buffer: one VGPR offset per row tile, the k-group as a scalar offset
    const __amdgpu_buffer_rsrc_t brs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)bpack, (short)0, a.row_tiles * NG * 64 * 16, 0x00020000);
    float pf[PRE];
    int c = blockIdx.x;
    Chunk nxt;
    if (c < nch) {
        nxt = read_chunk(a.chunks, c);
        span_load<PRE, 256>(a, nxt, pf);
    }
    for (; c < nch; c += gridDim.x) {
        const Chunk ch = nxt;
        __syncthreads();
        span_store<ConvF32, PRE, 256>(a, ch, pf, lds, 0);
        __syncthreads();
        const bool more = c + (int)gridDim.x < nch;
        if (more) nxt = read_chunk(a.chunks, c + gridDim.x);
        const int fbase = wid * 32;
        if (fbase >= ch.n_frames) {
            if (more) span_load<PRE, 256>(a, nxt, pf);
            continue;
        }
        const float *lp = lds + (fbase + (lane & 31)) * a.S + 4 * (lane >> 5);
        for (int rb = 0; rb < a.row_tiles; rb += RTB) {
            f32x16 acc[RTB];
#pragma unroll
            for (int r = 0; r < RTB; ++r) acc[r] = f32x16{};
            int voff[RTB];
#pragma unroll
            for (int r = 0; r < RTB; ++r) voff[r] = ((min(rb + r, a.row_tiles - 1) * NG) * 64 + lane) * 16;
            // operands of k-group g: basis fragments of the RTB row tiles, and the frame
            // fragment at LDS offset (g / GH) S + 8 (g % GH)
            auto load = [&](f32x4 (&A)[RTB], f32x4 &B, int g) {
                const int j = g / GH;
#pragma unroll
                for (int r = 0; r < RTB; ++r)
                    A[r] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(brs, voff[r], g * 1024, 0));
                B = *(const f32x4 *)(lp + j * a.S + 8 * (g - j * GH));
            };
            auto mma = [&](const f32x4 (&A)[RTB], const f32x4 &B) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int r = 0; r < RTB; ++r)
                        acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[r][i], B[i], acc[r], 0, 0, 0);
            };
            f32x4 A0[RTB], A1[RTB], B0, B1;
            load(A0, B0, 0);
            for (int g = 0; g < NG; g += 2) {
                // ping-pong: the next group's loads are in flight while this group multiplies;
                // indices past the end are clamped so every load is unconditional.  The
                // scheduling barriers keep each load block above the MFMAs it overlaps.
                load(A1, B1, min(g + 1, NG - 1));
                __builtin_amdgcn_sched_barrier(0);
                mma(A0, B0);
                __builtin_amdgcn_sched_barrier(0);
                load(A0, B0, min(g + 2, NG - 1));
                __builtin_amdgcn_sched_barrier(0);
                // past the last group the B fragment is zeroed instead of branching, so the
                // loads above cannot be sunk into a conditional block
                const float keep = (g + 1 < NG) ? 1.0f : 0.0f;
                B1 *= keep;
                mma(A1, B1);
                __builtin_amdgcn_sched_barrier(0);
            }
            // the next chunk's span is requested only after the last basis wait of the
            // last row block: vmcnt drains in order, so loads issued earlier would hold up
            // every basis wait; here their latency overlaps the epilogue instead
            if (more && rb + RTB >= a.row_tiles) span_load<PRE, 256>(a, nxt, pf);
#pragma unroll
            for (int r = 0; r < RTB; ++r)
                if (rb + r < a.row_tiles) store_tile(a, ch, rb + r, fbase + (lane & 31), lane, acc[r]);
        }
    }
}

// ------------------------------------------------------------------ 16-bit register-tile MFMA sweep
//
// Two 32-frame tiles (LDS rows at l0 and l1) against a wave's basis tile held in registers:
// NS k-groups of 16, one v_mfma_f32_32x32x16 per tile and group.  The frame fragments are
// read D groups ahead into a ring of registers, and scheduling barriers keep each group's
// reads above the multiplies they overlap, so LDS latency hides behind D groups of MFMAs.
// X3 adds hi*lo + lo*hi products from the low parts (basis in Al, frames at lo_off).
template <int NS, bool X3, bool IS_F16>
__device__ __forceinline__ void mfma_sweep(const uint4 (&A)[NS], const uint4 (&Al)[X3 ? NS : 1],
                                           const unsigned short *l0, const unsigned short *l1,
                                           const GroupTableBig &gt, int lo_off, f32x16 &acc0, f32x16 &acc1) {
    constexpr int D = X3 ? 1 : 4;
    uint4 b0[D], b1[D], c0[X3 ? D : 1], c1[X3 ? D : 1];
    auto fetch = [&](int s, int slot) {
        const int o = gt.lds_off[s];
        b0[slot] = *(const uint4 *)(l0 + o);
        b1[slot] = *(const uint4 *)(l1 + o);
        if constexpr (X3) {
            c0[slot] = *(const uint4 *)(l0 + lo_off + o);
            c1[slot] = *(const uint4 *)(l1 + lo_off + o);
        }
    };
#pragma unroll
    for (int s = 0; s < D && s < NS; ++s) fetch(s, s);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int slot = s % D;
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (IS_F16) {
            const f16x8 av = __builtin_bit_cast(f16x8, A[s]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, __builtin_bit_cast(f16x8, b0[slot]), acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, __builtin_bit_cast(f16x8, b1[slot]), acc1, 0, 0, 0);
        } else {
            const bf16x8 av = __builtin_bit_cast(bf16x8, A[s]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, b0[slot]), acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, b1[slot]), acc1, 0, 0, 0);
            if constexpr (X3) {
                const bf16x8 al = __builtin_bit_cast(bf16x8, Al[s]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, __builtin_bit_cast(bf16x8, b0[slot]), acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, __builtin_bit_cast(bf16x8, b1[slot]), acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, c0[slot]), acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, c1[slot]), acc1, 0, 0, 0);
            }
        }
        if (s + D < NS) fetch(s + D, slot);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// ------------------------------------------------------------------ 16-bit row-split kernel
//
// One wave per 32-row basis tile (16 Mel bins); the wave keeps its whole basis tile in
// registers for the life of the persistent kernel (NS k-groups of 16 x 16-bit values per
// lane = 4 VGPRs each) and sweeps every frame tile of every chunk, two tiles at a time.
// Frames are staged in LDS already rounded to the 16-bit format.  X3 adds the low parts
// (split-bf16: hi*hi + hi*lo + lo*hi).
template <class Conv, int NS, bool X3, bool IS_F16>
__global__ __launch_bounds__(512) void k_melt_h16_rs(FwdArgs a, const uint4 *__restrict__ bhi,
                                                     const uint4 *__restrict__ blo, GroupTableBig gt, int bf) {
    extern __shared__ unsigned short lds16[];
    const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
    const int nthreads = blockDim.x;
    uint4 A[NS];
    uint4 Al[X3 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) A[s] = bhi[((size_t)rt * NS + s) * 64 + lane];
    if constexpr (X3) {
#pragma unroll
        for (int s = 0; s < NS; ++s) Al[s] = blo[((size_t)rt * NS + s) * 64 + lane];
    }
    const int lo_off = a.S * (bf + a.J - 1);
    zero_pad_columns<Conv>(a, bf + a.J - 1, lds16, nthreads, lo_off);
    const int nch = *a.n_chunks;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = read_chunk(a.chunks, c);
        __syncthreads();
        stage_span<Conv, 8>(a, ch, lds16, nthreads, lo_off);
        __syncthreads();
        const int nft = (ch.n_frames + 31) >> 5;
        for (int ft = 0; ft < nft; ft += 2) {
            const bool two = ft + 1 < nft;
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            const unsigned short *l0 = lds16 + (ft * 32 + (lane & 31)) * a.S + 8 * (lane >> 5);
            // a lone last tile multiplies its own rows twice rather than branching
            const unsigned short *l1 = two ? l0 + 32 * a.S : l0;
            mfma_sweep<NS, X3, IS_F16>(A, Al, l0, l1, gt, lo_off, acc0, acc1);
            store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc0);
            if (two) store_tile(a, ch, rt, (ft + 1) * 32 + (lane & 31), lane, acc1);
        }
    }
}

// ------------------------------------------------------------------ FP8 E4M3 row-split kernel
//
// Per-frame scaling needs one quantised copy of every frame (a sample belongs to ~N/H
// frames with different scales), so the chunk's FP32 span is staged as hop-block rows, the
// maximum |x| of every frame is formed from per-row maxima, and each frame is quantised
// with s_t = 448 / max|x_t| into a frame-major E4M3 image in LDS (K = n padded to 64).
// One wave per 32-row basis tile keeps its E4M3 rows (pre-scaled by r_j = 448 / max|W_j|)
// in registers; v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales multiplies; the
// epilogue divides by s_t r_j in FP32 before R^2 + I^2.

typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned fp8x4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (unsigned)w;
}

// E4M3 pack of the basis: [rt][group of 64][lane][32 bytes]; lane half h holds k = 64 g + 32 h + byte.
// Row scales r_j = 448 / max_n |W_j| (FP32); rinv[rt][i] = 1 / r_j of tile row i.
__global__ void k_pack_f8(const float *__restrict__ b32, int M, int N, int NG, int RT, unsigned *__restrict__ out,
                          float *__restrict__ rinv) {
    __shared__ float rmax[32];
    const int rt = blockIdx.x;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 32) {
        int ml, part;
        tile_row_to_mel(threadIdx.x, ml, part);
        const int mel = rt * 16 + ml;
        float mx = 0.0f;
        if (mel < M)
            for (int n = 0; n < N; ++n) mx = fmaxf(mx, fabsf(b32[(size_t)(part * M + mel) * N + n]));
        rmax[threadIdx.x] = mx;
        rinv[rt * 32 + threadIdx.x] = mx > 0.0f ? 1.0f / __fdiv_rn(448.0f, mx) : 1.0f;
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    int ml, part;
    tile_row_to_mel(lane & 31, ml, part);
    const int mel = rt * 16 + ml;
    const float mx = rmax[lane & 31];
    const float sc = mx > 0.0f ? __fdiv_rn(448.0f, mx) : 1.0f;
    for (int g = 0; g < NG; ++g)
        for (int w = 0; w < 8; ++w) {
            float v[4];
            for (int e = 0; e < 4; ++e) {
                const int k = g * 64 + 32 * (lane >> 5) + 4 * w + e;
                v[e] = (mel < M && k < N) ? __fmul_rn(b32[(size_t)(part * M + mel) * N + k], sc) : 0.0f;
            }
            out[(((size_t)rt * NG + g) * 64 + lane) * 8 + w] = fp8x4(v[0], v[1], v[2], v[3]);
        }
}

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

// Row-split 16-bit kernel with direct-to-LDS staging (default for BF16/FP16/BF16X3): as
// k_melt_h16_rs, but chunk c+1's span is copied into an FP32 scratch area while chunk c is
// multiplied; after a barrier all threads convert it into the operand rows.
template <class Conv, int NS, bool X3, bool IS_F16>
__global__ __launch_bounds__(512) void k_melt_h16_as(FwdArgs a, const uint4 *__restrict__ bhi,
                                                     const uint4 *__restrict__ blo, GroupTableBig gt, int bf,
                                                     int scr_off) {
    extern __shared__ float lds_as[];
    const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
    const int lo_off = a.S * (bf + a.J - 1);
    unsigned short *rows = reinterpret_cast<unsigned short *>(lds_as);
    float *scratch = lds_as + scr_off;             // FP32 span, after the operand rows
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows, blockDim.x, lo_off);
    uint4 A[NS];
    uint4 Al[X3 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) A[s] = bhi[((size_t)rt * NS + s) * 64 + lane];
    if constexpr (X3) {
#pragma unroll
        for (int s = 0; s < NS; ++s) Al[s] = blo[((size_t)rt * NS + s) * 64 + lane];
    }
    const int nch = *a.n_chunks;
    int c = blockIdx.x;
    if (c < nch) async_span(a, read_chunk(a.chunks, c), scratch);
    for (; c < nch; c += gridDim.x) {
        const Chunk ch = read_chunk(a.chunks, c);
        async_wait();
        __syncthreads();                           // span of chunk c is in scratch; rows are free
        convert_span<Conv>(a, ch, scratch, rows, lo_off);
        __syncthreads();                           // rows ready; scratch is free
        if (c + (int)gridDim.x < nch) async_span(a, read_chunk(a.chunks, c + gridDim.x), scratch);
        const int nft = (ch.n_frames + 31) >> 5;
        for (int ft = 0; ft < nft; ft += 2) {
            const bool two = ft + 1 < nft;
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            const unsigned short *l0 = rows + (ft * 32 + (lane & 31)) * a.S + 8 * (lane >> 5);
            // a lone last tile multiplies its own rows twice rather than branching
            const unsigned short *l1 = two ? l0 + 32 * a.S : l0;
            mfma_sweep<NS, X3, IS_F16>(A, Al, l0, l1, gt, lo_off, acc0, acc1);
            store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc0);
            if (two) store_tile(a, ch, rt, (ft + 1) * 32 + (lane & 31), lane, acc1);
        }
    }
}

// ------------------------------------------------------------------ 16-bit frame-split kernel
// Fallback for frame lengths whose basis tile does not fit in registers: as the FP32
// frame-split kernel, one 32x32x16 MFMA per k-group.
template <class Conv, int RTB, bool IS_F16>
__global__ __launch_bounds__(256, 1) void k_melt_h16_fs(FwdArgs a, const uint4 *__restrict__ bpack,
                                                        GroupTableBig gt) {
    extern __shared__ unsigned short lds16[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nch = *a.n_chunks;
    const int NG = gt.n;
    zero_pad_columns<Conv>(a, kChunkF32 + a.J - 1, lds16, 256, 0);
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = read_chunk(a.chunks, c);
        __syncthreads();
        stage_span<Conv, 8>(a, ch, lds16, 256, 0);
        __syncthreads();
        const int fbase = wid * 32;
        if (fbase >= ch.n_frames) continue;
        const unsigned short *lp = lds16 + (fbase + (lane & 31)) * a.S + 8 * (lane >> 5);
        for (int rb = 0; rb < a.row_tiles; rb += RTB) {
            f32x16 acc[RTB];
#pragma unroll
            for (int r = 0; r < RTB; ++r) acc[r] = f32x16{};
            const uint4 *bp = bpack + (size_t)rb * NG * 64 + lane;
            for (int g = 0; g < NG; ++g) {
                const uint4 b = *(const uint4 *)(lp + gt.lds_off[g]);
#pragma unroll
                for (int r = 0; r < RTB; ++r) {
                    if (rb + r >= a.row_tiles) continue;
                    const uint4 av = bp[((size_t)r * NG + g) * 64];
                    if constexpr (IS_F16)
                        acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av),
                                                                        __builtin_bit_cast(f16x8, b), acc[r], 0, 0, 0);
                    else
                        acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                                         __builtin_bit_cast(bf16x8, b), acc[r], 0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < RTB; ++r)
                if (rb + r < a.row_tiles) store_tile(a, ch, rb + r, fbase + (lane & 31), lane, acc[r]);
        }
    }
}

// ------------------------------------------------------------------ host side

namespace {

int lds_stride(int Hp, int esize) {
    // row stride (elements) whose dword count is an odd multiple of 4, so that the 16-byte
    // reads of 8 consecutive rows at one column fall in 8 distinct 4-bank groups
    const int per_dword = 4 / esize;
    int dw = (Hp + per_dword - 1) / per_dword;
    dw = ((dw + 3) / 4) * 4;
    if ((dw / 4) % 2 == 0) dw += 4;
    return dw * per_dword;
}

GroupTableBig make_table(const Geometry &g, int S) {
    GroupTableBig t{};
    t.n = g.n_groups;
    for (int i = 0; i < g.n_groups && i < 512; ++i) t.lds_off[i] = g.seg_of_group[i] * S + g.col_of_group[i];
    return t;
}

FwdArgs make_args(Plan &p, const Geometry &g, int S, const float *wave, float *out, float *proj,
                  int64_t n_frames, const Chunk *tab, const int *n_tab) {
    FwdArgs a;
    a.wave = wave;
    a.chunks = tab;
    a.n_chunks = n_tab;
    a.out = out;
    a.proj = proj;
    a.n_frames = n_frames;
    a.M = p.M;
    a.J = g.J;
    a.H = p.H;
    a.Hp = g.Hp;
    a.S = S;
    a.row_tiles = p.row_tiles;
    a.out_kind = p.cfg.output;
    a.eps = (float)p.cfg.log_eps;
    a.invH = (float)(1.0 / p.H);
    return a;
}

melt_status upload_ints(const std::vector<int> &v, int **d) {
    if (hipMalloc(d, sizeof(int) * (v.size() + 1)) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "hipMalloc");
    return hip_check(hipMemcpy(*d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice), "hipMemcpy");
}

constexpr int kBF32 = kChunkF32;
constexpr int kMaxLds = 160 * 1024;

template <class K>
void allow_lds(K kern) {
    (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
}

// workgroups per CU of a persistent launch: the tuned value, else the default
int grid_mult(const Plan &p, int dflt) { return p.tune_grid > 0 ? p.tune_grid : dflt; }

// row-split variants: number of k-groups with a compiled register tile
bool rs_supported(int NS) { return NS == 25 || NS == 32 || NS == 20 || NS == 16 || NS == 10; }

}  // namespace

melt_status pack_basis(Plan &p, hipStream_t s) {
    melt_status st;
    // per-group segment/column tables for the pack kernels (temporary device copies)
    auto pack_one = [&](const Geometry &g, auto launch) -> melt_status {
        int *dseg = nullptr, *dcol = nullptr;
        melt_status r = upload_ints(g.seg_of_group, &dseg);
        if (r == MELT_OK) r = upload_ints(g.col_of_group, &dcol);
        if (r == MELT_OK) {
            launch(dseg, dcol);
            r = hip_check(hipGetLastError(), "pack kernel");
        }
        if (r == MELT_OK) r = hip_check(hipStreamSynchronize(s), "pack sync");
        (void)hipFree(dseg);
        (void)hipFree(dcol);
        return r;
    };
    const int RT = p.row_tiles;
    st = pack_one(p.geo32, [&](int *seg, int *col) {
        k_pack_f32<<<256, 256, 0, s>>>(p.d_basis32, p.M, p.N, p.H, seg, col, p.geo32.n_groups, RT,
                                       (float *)p.d_pack_f32);
    });
    if (st != MELT_OK) return st;
    const int kind_hi = (p.cfg.precision == MELT_PREC_FP16) ? 1 : 0;
    st = pack_one(p.geo16, [&](int *seg, int *col) {
        k_pack_h16<<<256, 256, 0, s>>>(p.d_basis32, p.M, p.N, p.H, seg, col, p.geo16.n_groups, RT, kind_hi,
                                       (unsigned short *)p.d_pack_h16);
        k_pack_h16<<<256, 256, 0, s>>>(p.d_basis32, p.M, p.N, p.H, seg, col, p.geo16.n_groups, RT, 2,
                                       (unsigned short *)p.d_pack_lo);
    });
    if (st != MELT_OK) return st;
    const int ng8 = (p.N + 63) / 64;
    k_pack_f8<<<RT, 64, 0, s>>>(p.d_basis32, p.M, p.N, ng8, RT, (unsigned *)p.d_pack_f8, p.d_rowscale);
    st = hip_check(hipGetLastError(), "pack f8");
    if (st != MELT_OK) return st;
    return pack_basis_dx(p, s);
}

melt_status ensure_chunks(Plan &p, int which, int64_t needed) {
    if (needed <= p.chunk_cap[which]) return MELT_OK;
    int64_t cap = std::max<int64_t>(needed, 2 * p.chunk_cap[which]);
    Chunk *d = nullptr;
    if (hipMalloc(&d, sizeof(Chunk) * cap) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "chunk table");
    if (p.d_chunks[which]) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p.d_chunks[which]);
    }
    p.d_chunks[which] = d;
    p.chunk_cap[which] = cap;
    return MELT_OK;
}

melt_status launch_schedule(Plan &p, int which, const int64_t *d_off, int n_clips, int bf, int64_t n_frames,
                            hipStream_t s) {
    const int64_t need = n_frames / bf + n_clips + 1;
    melt_status st = ensure_chunks(p, which, need);
    if (st != MELT_OK) return st;
    k_schedule<<<1, 1024, 0, s>>>(d_off, n_clips, p.N, p.H, bf, p.d_chunks[which], p.chunk_cap[which],
                                  p.d_nchunks + which);
    st = hip_check(hipGetLastError(), "schedule launch");
    if (st == MELT_OK) {
        p.prepared_frames[which] = n_frames;
        if (which == 0) p.prepared_variant = p.tune_variant;
    }
    return st;
}

melt_status launch_frame_offsets(const int64_t *d_off, int n_clips, int N, int H, int64_t *d_fo, hipStream_t s) {
    k_frame_offsets<<<1, 1024, 0, s>>>(d_off, n_clips, N, H, d_fo);
    return hip_check(hipGetLastError(), "frame offsets launch");
}

// Kernel variants of a plan, in the order the autotuner times them (p.tune_variant selects;
// the first one is the default):
//   FP32       frame-split with register prefetch
//   BF16/FP16  row-split with direct-to-LDS staging (128- then 64-frame chunks), row-split
//              with register staging, frame-split (the only one when the frame is too long
//              for a register tile)
//   BF16X3     row-split with direct-to-LDS staging (96- then 64-frame chunks), row-split
//              with register staging
//   FP8        row-split
enum VariantKind { V_F32_FS, V_H16_AS, V_H16_RS, V_H16_FS, V_F8_RS };
struct Variant {
    VariantKind kind;
    int bf;          // frames per chunk
};

static bool rs_fits(const Plan &p) { return rs_supported(p.geo16.n_groups) && p.row_tiles <= 8; }

// LDS of the direct-to-LDS 16-bit kernel: operand rows, then the FP32 span scratch (16-byte aligned)
static size_t as_rows_bytes(const Plan &p, int bf) {
    const bool x3 = p.cfg.precision == MELT_PREC_BF16X3;
    return (size_t)(bf + p.geo16.J - 1) * lds_stride(p.geo16.Hp, 2) * 2 * (x3 ? 2 : 1);
}
static size_t as_lds_bytes(const Plan &p, int bf) {
    return ((as_rows_bytes(p, bf) + 15) & ~size_t(15)) + (size_t)(bf + p.geo16.J - 1) * p.H * 4;
}

static std::vector<Variant> variant_list(const Plan &p) {
    std::vector<Variant> v;
    switch (p.cfg.precision) {
    case MELT_PREC_FP32: v.push_back({V_F32_FS, kBF32}); break;
    case MELT_PREC_FP8_E4M3: v.push_back({V_F8_RS, kBF32}); break;
    default: {
        const bool x3 = p.cfg.precision == MELT_PREC_BF16X3;
        if (rs_fits(p)) {
            for (int bf : {128, 96, 64}) {
                if (bf == (x3 ? 128 : 96)) continue;
                if (as_lds_bytes(p, bf) <= (size_t)kMaxLds) v.push_back({V_H16_AS, bf});
            }
            v.push_back({V_H16_RS, 128});
        }
        if (!x3) v.push_back({V_H16_FS, kBF32});
    }
    }
    return v;
}

static Variant variant_at(const Plan &p, int i) {
    const std::vector<Variant> v = variant_list(p);
    if (v.empty()) return {V_H16_FS, kBF32};      // unsupported geometry: the launch reports it
    return v[i >= 0 && (size_t)i < v.size() ? i : 0];
}

int forward_variants(const Plan &p) { return (int)variant_list(p).size(); }

const char *forward_variant_name(const Plan &p, int i) {
    static thread_local char buf[64];
    const std::vector<Variant> v = variant_list(p);
    if (i < 0 || (size_t)i >= v.size()) return "none";
    const char *k = v[i].kind == V_F32_FS   ? "f32-frame-split"
                    : v[i].kind == V_H16_AS ? "h16-row-split-lds-dma"
                    : v[i].kind == V_H16_RS ? "h16-row-split"
                    : v[i].kind == V_H16_FS ? "h16-frame-split"
                                            : "f8-row-split";
    std::snprintf(buf, sizeof(buf), "%s-bf%d", k, v[i].bf);
    return buf;
}

int melt_chunk_frames(const Plan &p, int variant) { return variant_at(p, variant).bf; }
int melt_chunk_frames(const Plan &p) { return melt_chunk_frames(p, p.tune_variant); }

template <int RTB, int PRE>
static melt_status launch_f32_pre(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid,
                                  hipStream_t s) {
    allow_lds(k_melt_f32_fs<RTB, PRE>);
    k_melt_f32_fs<RTB, PRE><<<grid, 256, lds, s>>>(a, (const f32x4 *)p.d_pack_f32, gt.n);
    return hip_check(hipGetLastError(), "melt f32 launch");
}

// register prefetch depth: span of a full chunk, (128 + J - 1) H samples over 256 threads
template <int RTB>
static melt_status launch_f32_rtb(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid,
                                  hipStream_t s) {
    const int need = ((kBF32 + a.J - 1) * a.H + 255) / 256;
    if (need <= 48) return launch_f32_pre<RTB, 48>(p, a, gt, lds, grid, s);
    if (need <= 88) return launch_f32_pre<RTB, 88>(p, a, gt, lds, grid, s);
    if (need <= 136) return launch_f32_pre<RTB, 136>(p, a, gt, lds, grid, s);
    return set_error(MELT_E_UNSUPPORTED, "hop too large for the FP32 register pipeline");
}

template <class Conv, bool F16, int RTB>
static melt_status launch_h16fs_rtb(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid,
                                    hipStream_t s) {
    allow_lds(k_melt_h16_fs<Conv, RTB, F16>);
    k_melt_h16_fs<Conv, RTB, F16><<<grid, 256, lds, s>>>(a, (const uint4 *)p.d_pack_h16, gt);
    return hip_check(hipGetLastError(), "melt h16 fs launch");
}

template <class Conv, int NS, bool X3, bool F16>
static melt_status launch_rs_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                hipStream_t s) {
    allow_lds(k_melt_h16_rs<Conv, NS, X3, F16>);
    k_melt_h16_rs<Conv, NS, X3, F16><<<grid, 64 * p.row_tiles, lds, s>>>(
        a, (const uint4 *)p.d_pack_h16, (const uint4 *)p.d_pack_lo, gt, bf);
    return hip_check(hipGetLastError(), "melt h16 rs launch");
}

template <int NG>
static melt_status launch_f8(Plan &p, const FwdArgs &a, size_t lds, int grid, int bf, hipStream_t s) {
    allow_lds(k_melt_f8_rs<NG>);
    k_melt_f8_rs<NG><<<grid, 64 * p.row_tiles, lds, s>>>(a, (const i32x8 *)p.d_pack_f8, p.d_rowscale, p.N, bf);
    return hip_check(hipGetLastError(), "melt f8 launch");
}

template <class Conv, int NS, bool X3, bool F16>
static melt_status launch_as_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                int scr_off, hipStream_t s) {
    allow_lds(k_melt_h16_as<Conv, NS, X3, F16>);
    k_melt_h16_as<Conv, NS, X3, F16><<<grid, 64 * p.row_tiles, lds, s>>>(
        a, (const uint4 *)p.d_pack_h16, (const uint4 *)p.d_pack_lo, gt, bf, scr_off);
    return hip_check(hipGetLastError(), "melt h16 lds-dma launch");
}

template <class Conv, bool X3, bool F16>
static melt_status launch_as(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                             int scr_off, hipStream_t s) {
    switch (p.geo16.n_groups) {
    case 10: return launch_as_ns<Conv, 10, X3, F16>(p, a, gt, lds, grid, bf, scr_off, s);
    case 16: return launch_as_ns<Conv, 16, X3, F16>(p, a, gt, lds, grid, bf, scr_off, s);
    case 20: return launch_as_ns<Conv, 20, X3, F16>(p, a, gt, lds, grid, bf, scr_off, s);
    case 25: return launch_as_ns<Conv, 25, X3, F16>(p, a, gt, lds, grid, bf, scr_off, s);
    case 32: return launch_as_ns<Conv, 32, X3, F16>(p, a, gt, lds, grid, bf, scr_off, s);
    default: return set_error(MELT_E_UNSUPPORTED, "no register tile for this frame length");
    }
}

template <class Conv, bool X3, bool F16>
static melt_status launch_rs(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                             hipStream_t s) {
    switch (p.geo16.n_groups) {
    case 10: return launch_rs_ns<Conv, 10, X3, F16>(p, a, gt, lds, grid, bf, s);
    case 16: return launch_rs_ns<Conv, 16, X3, F16>(p, a, gt, lds, grid, bf, s);
    case 20: return launch_rs_ns<Conv, 20, X3, F16>(p, a, gt, lds, grid, bf, s);
    case 25: return launch_rs_ns<Conv, 25, X3, F16>(p, a, gt, lds, grid, bf, s);
    case 32: return launch_rs_ns<Conv, 32, X3, F16>(p, a, gt, lds, grid, bf, s);
    default: return set_error(MELT_E_UNSUPPORTED, "no register tile for this frame length");
    }
}

melt_status launch_melt_main(Plan &p, const float *d_wave, float *d_out, float *d_proj, hipStream_t s) {
    const int64_t n_frames = p.prepared_frames[0];
    if (n_frames < 0) return set_error(MELT_E_INVALID_ARG, "no batch prepared");
    if (n_frames == 0) return MELT_OK;
    const int v = p.prepared_variant;
    return launch_melt_table(p, v, p.d_chunks[0], p.d_nchunks, n_frames / melt_chunk_frames(p, v) + 1, n_frames,
                             d_wave, d_out, d_proj, s);
}

melt_status launch_melt_table(Plan &p, int variant, const Chunk *tab, const int *n_tab, int64_t est_chunks,
                              int64_t n_frames, const float *d_wave, float *d_out, float *d_proj, hipStream_t s) {
    const int prec = p.cfg.precision;
    if (prec == MELT_PREC_FP32) {
        const Geometry &g = p.geo32;
        const int S = lds_stride(g.Hp, 4);
        const size_t lds = (size_t)(kBF32 + g.J - 1) * S * 4;
        if (lds > (size_t)kMaxLds || g.n_groups > 512)
            return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS for FP32 kernel");
        const FwdArgs a = make_args(p, g, S, d_wave, d_out, d_proj, n_frames, tab, n_tab);
        const GroupTableBig gt = make_table(g, S);
        const int64_t est = est_chunks;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(est, (int64_t)p.cu_count * grid_mult(p, 1)));
        // register-prefetch variant: row tiles per block at most 5 (2 for the deepest
        // prefetch) so accumulators, basis prefetch and sample prefetch fit 512 registers
        const int need = ((kBF32 + g.J - 1) * p.H + 255) / 256;
        const int cap = need <= 88 ? 5 : 2;
        const int blocks = (p.row_tiles + cap - 1) / cap;
        switch ((p.row_tiles + blocks - 1) / blocks) {
        case 1: return launch_f32_rtb<1>(p, a, gt, lds, grid, s);
        case 2: return launch_f32_rtb<2>(p, a, gt, lds, grid, s);
        case 3: return launch_f32_rtb<3>(p, a, gt, lds, grid, s);
        case 4: return launch_f32_rtb<4>(p, a, gt, lds, grid, s);
        default: return launch_f32_rtb<5>(p, a, gt, lds, grid, s);
        }
    }
    if (prec == MELT_PREC_BF16 || prec == MELT_PREC_FP16 || prec == MELT_PREC_BF16X3) {
        const Geometry &g = p.geo16;
        const int S = lds_stride(g.Hp, 2);
        const bool f16 = prec == MELT_PREC_FP16;
        const bool x3 = prec == MELT_PREC_BF16X3;
        if (g.n_groups > 512) return set_error(MELT_E_UNSUPPORTED, "frame too long");
        const FwdArgs a = make_args(p, g, S, d_wave, d_out, d_proj, n_frames, tab, n_tab);
        const GroupTableBig gt = make_table(g, S);
        const Variant var = variant_at(p, variant);
        if (var.kind == V_H16_AS) {
            const int bf = var.bf;
            const size_t lds = as_lds_bytes(p, bf);
            if (lds > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
            const int scr_off = (int)(((as_rows_bytes(p, bf) + 15) & ~size_t(15)) / 4);
            const int per_cu = std::max(1, (int)(kMaxLds / lds));
            const int grid = (int)std::max<int64_t>(
                1, std::min<int64_t>(est_chunks, (int64_t)p.cu_count * grid_mult(p, std::min(per_cu, 2))));
            if (x3) return launch_as<ConvBF16X3, true, false>(p, a, gt, lds, grid, bf, scr_off, s);
            if (f16) return launch_as<ConvF16, false, true>(p, a, gt, lds, grid, bf, scr_off, s);
            return launch_as<ConvBF16, false, false>(p, a, gt, lds, grid, bf, scr_off, s);
        }
        if (var.kind == V_H16_RS) {
            const int bf = var.bf;
            const size_t lds = (size_t)(bf + g.J - 1) * S * 2 * (x3 ? 2 : 1);
            if (lds > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
            const int per_cu = std::max(1, (int)(kMaxLds / lds));
            const int grid = (int)std::max<int64_t>(
                1, std::min<int64_t>(est_chunks, (int64_t)p.cu_count * grid_mult(p, std::min(per_cu, 2))));
            if (x3) return launch_rs<ConvBF16X3, true, false>(p, a, gt, lds, grid, bf, s);
            if (f16) return launch_rs<ConvF16, false, true>(p, a, gt, lds, grid, bf, s);
            return launch_rs<ConvBF16, false, false>(p, a, gt, lds, grid, bf, s);
        }
        if (x3) return set_error(MELT_E_UNSUPPORTED, "BF16X3 needs the register-tile kernel (frame too long)");
        const size_t lds = (size_t)(kBF32 + g.J - 1) * S * 2;
        if (lds > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
        const int64_t est = est_chunks;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(est, (int64_t)p.cu_count * grid_mult(p, 2)));
        switch (std::min(p.row_tiles, 8)) {
        case 1: return f16 ? launch_h16fs_rtb<ConvF16, true, 1>(p, a, gt, lds, grid, s) : launch_h16fs_rtb<ConvBF16, false, 1>(p, a, gt, lds, grid, s);
        case 2: return f16 ? launch_h16fs_rtb<ConvF16, true, 2>(p, a, gt, lds, grid, s) : launch_h16fs_rtb<ConvBF16, false, 2>(p, a, gt, lds, grid, s);
        case 4: return f16 ? launch_h16fs_rtb<ConvF16, true, 4>(p, a, gt, lds, grid, s) : launch_h16fs_rtb<ConvBF16, false, 4>(p, a, gt, lds, grid, s);
        case 3:
        case 5:
        case 6: return f16 ? launch_h16fs_rtb<ConvF16, true, 6>(p, a, gt, lds, grid, s) : launch_h16fs_rtb<ConvBF16, false, 6>(p, a, gt, lds, grid, s);
        default: return f16 ? launch_h16fs_rtb<ConvF16, true, 8>(p, a, gt, lds, grid, s) : launch_h16fs_rtb<ConvBF16, false, 8>(p, a, gt, lds, grid, s);
        }
    }
    if (prec == MELT_PREC_FP8_E4M3) {
        const Geometry &g = p.geo32;
        const int S = lds_stride(g.Hp, 4);
        const int ng8 = (p.N + 63) / 64;
        const int bf = kBF32;
        const int rows_max = bf + g.J - 1;
        const size_t lds = (size_t)rows_max * S * 4 + (size_t)bf * (ng8 * 64 + 16) + (size_t)bf * 4 + 2 * (size_t)rows_max * 4;
        if (lds > (size_t)kMaxLds || p.row_tiles > 8)
            return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS for the FP8 kernel");
        const FwdArgs a = make_args(p, g, S, d_wave, d_out, d_proj, n_frames, tab, n_tab);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(est_chunks, (int64_t)p.cu_count * grid_mult(p, 1)));
        switch (ng8) {
        case 4: return launch_f8<4>(p, a, lds, grid, bf, s);
        case 7: return launch_f8<7>(p, a, lds, grid, bf, s);
        case 8: return launch_f8<8>(p, a, lds, grid, bf, s);
        case 16: return launch_f8<16>(p, a, lds, grid, bf, s);
        default: return set_error(MELT_E_UNSUPPORTED, "FP8 kernel supports n_fft in (192, 256], (384, 512], (960, 1024]");
        }
    }
    return set_error(MELT_E_UNSUPPORTED, "precision not implemented");
}

}  // namespace melt
