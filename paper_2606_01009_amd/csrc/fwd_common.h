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
//
// This header holds what the forward kernels share: the chunk-table access, the argument
// block, the fused energy/log epilogue, the operand formats, the span staging helpers and
// the host-side geometry helpers.  The kernels live in melt_f32.hip, melt_h16.hip and
// melt_f8.hip; melt_fwd.hip holds the schedule, the basis packing and the variant table.
#pragma once
#include <vector>
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

typedef int i32x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ basis row order and formats

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
__device__ inline float f16_bits_to_f32(unsigned short u) { return (float)__builtin_bit_cast(_Float16, u); }

// four FP32 values -> four E4M3 bytes (round to nearest even, saturating)
__device__ __forceinline__ unsigned fp8x4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (unsigned)w;
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
    float acc_scale;       // multiplies the accumulated projections (exact power of two; 1 unless FP16X3)
};

// Chunk descriptors of a persistent workgroup's iterations, staged in LDS.  Reading each
// descriptor from the table when it is needed puts a memory load, and a wait for it, at the
// top of every iteration; since a wave's vector memory operations complete in issue order,
// that wait also drains the wave's earlier output stores.  Instead the entries of iterations
// [w0, w0 + kRing + 2) are read once per kRing iterations (w0 a multiple of kRing), so an
// iteration can also see the chunks one and two iterations ahead.  The fill must follow a
// barrier that ends every read of the previous window and precede one before the reads.
constexpr int kRing = 32;
struct ChunkRing {
    Chunk e[kRing + 2];
};
constexpr int kRingBytes = (int)sizeof(ChunkRing);
__device__ __forceinline__ void ring_fill(ChunkRing &r, const Chunk *tab, int c_w0, int cstep, int nch) {
    const int t = threadIdx.x;
    if (t < kRing + 2) {
        const int c = c_w0 + t * cstep;
        if (c < nch) r.e[t] = tab[c];
    }
}
// entry i of the window (iteration w0 + i); only meaningful for a chunk index below n_chunks
__device__ __forceinline__ Chunk ring_get(const ChunkRing &r, int i) {
    Chunk e = r.e[i];
    e.sample_start = uniform64(e.sample_start);
    e.sample_end = uniform64(e.sample_end);
    e.out_row = uniform64(e.out_row);
    e.n_frames = __builtin_amdgcn_readfirstlane(e.n_frames);
    e.clip = __builtin_amdgcn_readfirstlane(e.clip);
    return e;
}

// Natural log from the hardware base-2 logarithm (v_log_f32, about 1 ulp on normal
// inputs) times ln 2.  Arguments are S + eps or sqrt(S) + eps with S >= 0 and eps >= the
// smallest normal FP32 (the plan rejects smaller eps), so they are always normal.
__device__ __forceinline__ float ln_normal(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }

template <int KIND>
__device__ __forceinline__ float out_map_k(float S, float eps) {
    if constexpr (KIND == MELT_OUT_LOG_POWER) return ln_normal(S + eps);
    else if constexpr (KIND == MELT_OUT_LOG_MAGNITUDE) return ln_normal(sqrtf(S) + eps);
    else if constexpr (KIND == MELT_OUT_POWER) return S;
    else return sqrtf(S);
}

// Energies S = R^2 + I^2 of the 8 Mel bins a lane holds in one 32x32 accumulator (register
// pairs (4g, 4g+1) and (4g+2, 4g+3) are (R, I) of bins 2g and 2g+1), mapped to the output
// kind.  The kind is uniform, so it is switched on once per tile rather than per element.
template <int KIND>
__device__ __forceinline__ void map8_k(const f32x16 &acc, float eps, float (&v)[8]) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        v[2 * g] = out_map_k<KIND>(acc[4 * g] * acc[4 * g] + acc[4 * g + 1] * acc[4 * g + 1], eps);
        v[2 * g + 1] = out_map_k<KIND>(acc[4 * g + 2] * acc[4 * g + 2] + acc[4 * g + 3] * acc[4 * g + 3], eps);
    }
}
__device__ __forceinline__ void map8(const f32x16 &acc, int kind, float eps, float (&v)[8]) {
    switch (kind) {
    case MELT_OUT_LOG_POWER: map8_k<MELT_OUT_LOG_POWER>(acc, eps, v); break;
    case MELT_OUT_LOG_MAGNITUDE: map8_k<MELT_OUT_LOG_MAGNITUDE>(acc, eps, v); break;
    case MELT_OUT_POWER: map8_k<MELT_OUT_POWER>(acc, eps, v); break;
    default: map8_k<MELT_OUT_MAGNITUDE>(acc, eps, v); break;
    }
}

// Writes one 32-frame x 16-Mel tile from the accumulator of lane `lane` (frame
// `f_local` of the chunk).  Register pairs (4g, 4g+1), (4g+2, 4g+3) are (R, I) of Mel bins
// 8h + 2g and 8h + 2g + 1 of the tile.
__device__ inline void store_tile(const FwdArgs &a, const Chunk &ch, int rt, int f_local, int lane,
                                  const f32x16 &acc_in) {
    if (f_local >= ch.n_frames) return;
    f32x16 acc = acc_in;
    if (a.acc_scale != 1.0f) {          // FP16X3: undo the waveform's pre-scale (exact)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] *= a.acc_scale;
    }
    const int64_t row = ch.out_row + f_local;
    if (row >= a.n_frames) return;
    const int h = lane >> 5;
    const int mel0 = rt * 16 + 8 * h;
    if (mel0 >= a.M) return;
    float v[8];
    map8(acc, a.out_kind, a.eps, v);
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
struct ConvF32 {
    typedef float elem_t;
    __device__ static void store(float *l, int i, float v, int) { l[i] = v; }
    __device__ static void store4(float *l, int i, f32x4 v, int) { *(f32x4 *)(l + i) = v; }
};
// two FP32 values -> two 16-bit values in one dword (the two-source v_cvt_pk_{bf16,f16}_f32,
// round to nearest even, as the scalar conversions)
typedef float cv_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 cv_bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 cv_f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(cv_f32x2{a, b}, cv_bf16x2));
}
__device__ __forceinline__ unsigned pk_f16(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(cv_f32x2{a, b}, cv_f16x2));
}

struct ConvBF16 {
    typedef unsigned short elem_t;
    __device__ static void store(unsigned short *l, int i, float v, int) { l[i] = f32_to_bf16_bits(v); }
    __device__ static void store4(unsigned short *l, int i, f32x4 v, int) {
        *(uint2 *)(l + i) = uint2{pk_bf16(v[0], v[1]), pk_bf16(v[2], v[3])};
    }
};
struct ConvF16 {
    typedef unsigned short elem_t;
    __device__ static void store(unsigned short *l, int i, float v, int) { l[i] = f32_to_f16_bits(v); }
    __device__ static void store4(unsigned short *l, int i, f32x4 v, int) {
        *(uint2 *)(l + i) = uint2{pk_f16(v[0], v[1]), pk_f16(v[2], v[3])};
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
        const unsigned h01 = pk_bf16(v[0], v[1]), h23 = pk_bf16(v[2], v[3]);
        // the high parts back in FP32: the low half of a dword shifted up, the high half masked
        const float r0 = v[0] - __builtin_bit_cast(float, h01 << 16), r1 = v[1] - __builtin_bit_cast(float, h01 & 0xffff0000u);
        const float r2 = v[2] - __builtin_bit_cast(float, h23 << 16), r3 = v[3] - __builtin_bit_cast(float, h23 & 0xffff0000u);
        *(uint2 *)(l + i) = uint2{h01, h23};
        *(uint2 *)(l + i + lo_off) = uint2{pk_bf16(r0, r1), pk_bf16(r2, r3)};
    }
};

// split-binary16 of the waveform pre-scaled by 2^10 (exact): the high part at [i], the low part
// (the FP32 residual, exact, rounded to binary16) at [i + lo_off]
struct ConvF16X3 {
    typedef unsigned short elem_t;
    __device__ static void store(unsigned short *l, int i, float v, int lo_off) {
        const float u = v * kF16x3Scale;
        const unsigned short hb = f32_to_f16_bits(u);
        l[i] = hb;
        l[i + lo_off] = f32_to_f16_bits(u - f16_bits_to_f32(hb));
    }
    __device__ static void store4(unsigned short *l, int i, f32x4 v, int lo_off) {
        const f32x4 u = v * kF16x3Scale;
        const unsigned h01 = pk_f16(u[0], u[1]), h23 = pk_f16(u[2], u[3]);
        const cv_f32x2 b01 = __builtin_convertvector(__builtin_bit_cast(cv_f16x2, h01), cv_f32x2);
        const cv_f32x2 b23 = __builtin_convertvector(__builtin_bit_cast(cv_f16x2, h23), cv_f32x2);
        *(uint2 *)(l + i) = uint2{h01, h23};
        *(uint2 *)(l + i + lo_off) = uint2{pk_f16(u[0] - b01[0], u[1] - b01[1]), pk_f16(u[2] - b23[0], u[3] - b23[1])};
    }
};

// Register staging of a chunk's contiguous sample span [start, start + (n_frames + J - 1) H)
// by NT threads: element u of thread t is span position o = t + u * NT, so every load instruction of a
// wave reads 64 consecutive samples.  span_load issues all PRE loads at once (one memory
// round trip); span_store scatters them into the padded hop-block rows (row o / H, column
// o % H).  Samples at or past the clip end read as 0.
template <int PRE, int NT>
__device__ __forceinline__ void span_load(const FwdArgs &a, const Chunk &ch, float (&pf)[PRE], int t) {
    // buffer descriptor over [start, min(start + span, clip end)): loads past it return 0,
    // so the clip end needs no branch; one VGPR offset serves all PRE loads
    const int64_t start = ch.sample_start;
    const int64_t span = (int64_t)(ch.n_frames + a.J - 1) * a.H;
    const int64_t lim = ch.sample_end - start < span ? ch.sample_end - start : span;
    const int records = (int)(lim > 0 ? lim * 4 : 0);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(a.wave + start), (short)0, records, 0x00020000);
    const int voff = t * 4;
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
                                           typename Conv::elem_t *lds, int lo_off, int t) {
    // element u of the thread is span position tid + u NT; its row and column advance by
    // (dr, dc) per element, so no division per element
    const int span = (ch.n_frames + a.J - 1) * a.H;
    const int dr = NT / a.H, dc = NT - dr * a.H;
    const int dad = dr * a.S + dc, wrap = a.S - a.H;
    int c = t;
    const int r0 = span_row(a, c);
    c -= r0 * a.H;
    int ad = r0 * a.S + c;
    const bool full = span >= PRE * NT;           // whole register tile valid: no per-element branch
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
        if (full || t + u * NT < span) Conv::store(lds, ad, pf[u], lo_off);
        c += dc;
        ad += dad;
        if (c >= a.H) {
            c -= a.H;
            ad += wrap;
        }
        asm volatile("" : "+v"(ad), "+v"(c));      // no address computed ahead (registers)
    }
}

// Vector form for H a multiple of 4 (four consecutive samples never straddle a row): vector
// v of thread t holds span samples [4(t + v NT), +4).  Each vector's row and column are
// computed on their own (no chain through the previous element), and it is written with
// one 16-byte LDS store.  A vector that crosses the clip end is loaded element by element
// (the buffer descriptor returns 0 past it).
template <int PV, int NT>
__device__ __forceinline__ void span_load4(const FwdArgs &a, const Chunk &ch, f32x4 (&pv)[PV], int t) {
    const int64_t start = ch.sample_start;
    const int64_t span = (int64_t)(ch.n_frames + a.J - 1) * a.H;
    const int64_t lim = ch.sample_end - start < span ? ch.sample_end - start : span;
    const int records = (int)(lim > 0 ? lim * 4 : 0);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(a.wave + start), (short)0, records, 0x00020000);
#pragma unroll
    for (int v = 0; v < PV; ++v) {
        const int o = 4 * (t + v * NT);
        if (o + 4 <= records / 4) {
            pv[v] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, o * 4, 0, 0));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                pv[v][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (o + e) * 4, 0, 0));
        }
    }
}

template <int PV, int NT>
__device__ __forceinline__ void span_store4(const FwdArgs &a, const Chunk &ch, const f32x4 (&pv)[PV], float *lds,
                                            int t) {
    const int span = (ch.n_frames + a.J - 1) * a.H;
#pragma unroll
    for (int v = 0; v < PV; ++v) {
        const int o = 4 * (t + v * NT);
        if (o < span) {
            const int r = span_row(a, o);
            *(f32x4 *)(lds + r * a.S + (o - r * a.H)) = pv[v];
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
// then 4-byte copies over its last partial block, so no lane reads past the clip end.  Waves
// w of nw (wave-uniform) share the blocks; returns the number of copy instructions this wave
// issued (each has at least one active lane).
__device__ __forceinline__ int async_span_waves(const FwdArgs &a, const Chunk &ch, float *scratch, int w, int nw) {
    const int lane = threadIdx.x & 63;
    const int valid = span_valid(a, ch);
    const float *src = a.wave + ch.sample_start;
    const unsigned base = __builtin_amdgcn_readfirstlane(lds_addr(scratch));
    const int nfull = valid >> 8;
    int n = 0;
    for (int b = w; b < nfull; b += nw, ++n) lds_dma_x4(src + b * 256 + 4 * lane, base + b * 1024);
    for (int b = 4 * nfull + w; b * 64 < valid; b += nw, ++n) {
        const int o = b * 64 + lane;
        if (o < valid) lds_dma_x1(src + o, base + b * 256);
    }
    return n;
}

__device__ __forceinline__ int async_span(const FwdArgs &a, const Chunk &ch, float *scratch) {
    return async_span_waves(a, ch, scratch, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), blockDim.x >> 6);
}

// Chunk descriptor i of the table (i wave-uniform) through the scalar data cache (the table is
// read-only in the forward kernels): the wait for it is on the scalar-memory counter, so it
// never includes the wave's direct-to-LDS copies, which the compiler does not track (the
// wait it places for a vector load issued before such copies is a full vmcnt(0)).
__device__ __forceinline__ void load_chunk_scalar(const Chunk *tab, int i, uint4 &lo, uint4 &hi) {
    typedef unsigned cu32x8 __attribute__((ext_vector_type(8)));
    typedef const __attribute__((address_space(4))) cu32x8 *cptr;
    const cu32x8 v = *(cptr)(tab + i);
    lo = make_uint4(v[0], v[1], v[2], v[3]);
    hi = make_uint4(v[4], v[5], v[6], v[7]);
}

__device__ __forceinline__ void async_wait() {
    __builtin_amdgcn_s_waitcnt(0);     // this wave's direct-to-LDS copies have landed
}

// s_waitcnt vmcnt(N) alone (expcnt and lgkmcnt fields at their no-wait maxima).
template <int N>
__device__ __forceinline__ void waitcnt_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt is six bits");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Waits until this wave's memory loads issued before its last n vector-memory instructions
// have completed.  Loads (direct-to-LDS copies included) complete in issue order, so while
// one of those older loads is outstanding, so are the n younger ones and the count exceeds
// n; younger stores only make the wait stricter.  n is rounded down to an immediate, which
// waits a little more than needed and never less.  n must be wave-uniform.
__device__ __forceinline__ void wait_vm_younger(int n) {
    n = __builtin_amdgcn_readfirstlane(n);
    if (n >= 63) waitcnt_vm<63>();
    else if (n >= 48) waitcnt_vm<48>();
    else if (n >= 32) waitcnt_vm<32>();
    else if (n >= 24) waitcnt_vm<24>();
    else if (n >= 16) waitcnt_vm<16>();
    else if (n >= 12) waitcnt_vm<12>();
    else if (n >= 8) waitcnt_vm<8>();
    else if (n >= 4) waitcnt_vm<4>();
    else waitcnt_vm<0>();
}

// scratch (contiguous span) -> padded hop-block rows in the kernel's operand format.  With
// H a multiple of 4, four consecutive samples never straddle a row: one 16-byte LDS read and
// one vector write per thread and step.
template <class Conv>
__device__ __forceinline__ void convert_span(const FwdArgs &a, const Chunk &ch, const float *scratch,
                                             typename Conv::elem_t *rows, int lo_off) {
    const int span = (ch.n_frames + a.J - 1) * a.H;
    const int valid = span_valid(a, ch);
    // the thread index made opaque, so that the addresses derived from it are formed here on
    // every call: hoisted out of a kernel's chunk loop they stay live across its multiply
    // phase, where register-heavy kernels spill them, and the reload's wait for the wave's
    // memory counter then also waits for its output stores in flight
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    if ((a.H & 3) == 0) {
        // Vectors of 4 samples, thread-strided by step = 4 nt; four per thread and pass, so
        // their LDS reads are in flight together.  The row and column advance by (dr, dc)
        // per vector, so no division per element.
        const int nt = blockDim.x, step = 4 * nt;
        const int dr = step / a.H, dc = step - dr * a.H;
        const int dad = dr * a.S + dc, wrap = a.S - a.H;
        int c = 4 * tid;
        const int r0 = span_row(a, c);
        c -= r0 * a.H;
        int ad = r0 * a.S + c;
        for (int o0 = 4 * tid; o0 < span; o0 += 4 * step) {
            f32x4 v[4];
            int at[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int o = o0 + u * step;
                v[u] = o < span ? *(const f32x4 *)(scratch + o) : f32x4{};
                at[u] = ad;
                c += dc;
                ad += dad;
                if (c >= a.H) {
                    c -= a.H;
                    ad += wrap;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int o = o0 + u * step;
                if (o < span) {
                    if (o + 4 > valid) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (o + e >= valid) v[u][e] = 0.0f;
                    }
                    Conv::store4(rows, at[u], v[u], lo_off);
                }
            }
        }
        return;
    }
    for (int o = tid; o < span; o += blockDim.x) {
        const float v = o < valid ? scratch[o] : 0.0f;
        const int r = span_row(a, o);
        Conv::store(rows, r * a.S + (o - r * a.H), v, lo_off);
    }
}

// ------------------------------------------------------------------ host-side geometry

constexpr int kBF32 = kChunkF32;
constexpr int kMaxLds = 160 * 1024;

inline int lds_stride(int Hp, int esize) {
    // row stride (elements) whose dword count is an odd multiple of 4, so that the 16-byte
    // reads of 8 consecutive rows at one column fall in 8 distinct 4-bank groups
    const int per_dword = 4 / esize;
    int dw = (Hp + per_dword - 1) / per_dword;
    dw = ((dw + 3) / 4) * 4;
    if ((dw / 4) % 2 == 0) dw += 4;
    return dw * per_dword;
}

inline GroupTableBig make_table(const Geometry &g, int S) {
    GroupTableBig t{};
    t.n = g.n_groups;
    for (int i = 0; i < g.n_groups && i < 512; ++i) t.lds_off[i] = g.seg_of_group[i] * S + g.col_of_group[i];
    return t;
}

// One forward launch: the chunk table, the batch and the destination.
struct FwdTask {
    const Chunk *tab;
    const int *n_tab;
    int64_t est_chunks;    // upper bound on the table's entries (sizes the grid)
    int64_t n_frames;
    const float *wave;
    float *out;
    float *proj;
    hipStream_t stream;
};

inline FwdArgs make_args(const Plan &p, const Geometry &g, int S, const FwdTask &t) {
    FwdArgs a;
    a.wave = t.wave;
    a.chunks = t.tab;
    a.n_chunks = t.n_tab;
    a.out = t.out;
    a.proj = t.proj;
    a.n_frames = t.n_frames;
    a.M = p.M;
    a.J = g.J;
    a.H = p.H;
    a.Hp = g.Hp;
    a.S = S;
    a.row_tiles = p.row_tiles;
    a.out_kind = p.kern_out;
    a.eps = (float)p.cfg.log_eps;
    a.invH = (float)(1.0 / p.H);
    a.acc_scale = p.cfg.precision == MELT_PREC_FP16X3 ? 1.0f / kF16x3Scale : 1.0f;
    return a;
}

template <class K>
inline void allow_lds(K kern, int static_bytes = 0) {
    // the limit covers dynamic LDS only: the kernel's static LDS comes off the 160 KB
    (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds - static_bytes);
}

// persistent grid: min(chunks, CUs x workgroups per CU (tuned value, else dflt))
inline int persistent_grid(const Plan &p, int64_t est_chunks, int dflt) {
    const int per_cu = p.tune_grid > 0 ? p.tune_grid : dflt;
    return (int)std::max<int64_t>(1, std::min<int64_t>(est_chunks, (int64_t)p.cu_count * per_cu));
}

// 16-bit row-split kernels: k-group counts with a compiled register tile
inline bool rs_supported(int NS) { return NS == 25 || NS == 32 || NS == 20 || NS == 16 || NS == 10; }
inline bool rs_fits(const Plan &p) { return rs_supported(p.geo16.n_groups) && p.row_tiles <= 8; }
// the direct-to-LDS kernel: any Mel count (row groups of at most 8 tiles)
inline bool as_fits(const Plan &p) { return rs_supported(p.geo16.n_groups); }
// the row-pair kernel: two basis tiles per wave (16 or 20 k-groups), 4, 5 or 8 row tiles
inline bool ap_fits(const Plan &p) {
    const int ng = p.geo16.n_groups;
    return (ng == 16 || ng == 20) && (p.row_tiles == 4 || p.row_tiles == 5 || p.row_tiles == 8);
}

// LDS of the direct-to-LDS 16-bit kernel: operand rows, then the FP32 span scratch (16-byte aligned)
inline size_t as_rows_bytes(const Plan &p, int bf) {
    const bool x3 = prec_split(p);
    return (size_t)(bf + p.geo16.J - 1) * lds_stride(p.geo16.Hp, 2) * 2 * (x3 ? 2 : 1);
}
// ... then nbuf FP32 spans the chunks' copies land in (each 16-byte aligned)
inline size_t as_scratch_offset(const Plan &p, int bf) { return (as_rows_bytes(p, bf) + 15) & ~size_t(15); }
inline size_t as_span_bytes(const Plan &p, int bf) { return ((size_t)(bf + p.geo16.J - 1) * p.H * 4 + 15) & ~size_t(15); }
inline size_t as_lds_bytes(const Plan &p, int bf, int nbuf = 1) {
    return as_scratch_offset(p, bf) + (size_t)nbuf * as_span_bytes(p, bf);
}
// Waves of the direct-to-LDS row-split kernels for a group of `rt` row tiles: `full` waves own
// one row tile each; when one or two row tiles remain beyond a multiple of four, four more
// waves share them (psplit waves per tile), so the work spreads evenly over the CU's four
// SIMDs.  More than 8 row tiles are cut into row groups of at most 8, one group per
// workgroup, so that a wave's basis tile stays register-resident.
struct WaveLayout {
    int full, psplit, waves;
};
__host__ __device__ inline WaveLayout layout_for(int rt) {
    const int rem = rt % 4;
    if ((rem == 1 || rem == 2) && rt - rem + 4 <= 8) return {rt - rem, 4 / rem, rt - rem + 4};
    return {rt, 1, rt};
}
inline int row_groups(const Plan &p) { return (p.row_tiles + 7) / 8; }
// the workgroup's waves: enough for the layout of every row group (the last may be smaller)
inline WaveLayout wave_layout(const Plan &p) {
    const int rg = row_groups(p), gt_n = (p.row_tiles + rg - 1) / rg;
    WaveLayout w = layout_for(gt_n);
    w.waves = std::max(w.waves, layout_for(p.row_tiles - (rg - 1) * gt_n).waves);
    return w;
}

// Producer/consumer 16-bit kernel: two operand-row buffers and nscr FP32 spans; needs
// producer waves (beyond the full-tile ones) in every row group.
inline size_t pp_rows_bytes(const Plan &p, int bf) { return (as_rows_bytes(p, bf) + 15) & ~size_t(15); }
inline size_t pp_lds_bytes(const Plan &p, int bf, int nscr) {
    return 2 * pp_rows_bytes(p, bf) + (size_t)nscr * as_span_bytes(p, bf);
}
inline bool pp_fits(const Plan &p) {
    if (!as_fits(p)) return false;
    const int rg = row_groups(p), gt_n = (p.row_tiles + rg - 1) / rg, nw = wave_layout(p).waves;
    for (int g = 0; g < rg; ++g)
        if (layout_for(std::min(p.row_tiles - g * gt_n, gt_n)).full >= nw) return false;
    return true;
}

// 12-wave producer/consumer 16-bit kernel: two operand-row buffers (16-byte aligned each), then
// the FP32 span; consumers hold one basis tile of at most 25 k-groups (three waves per SIMD)
inline size_t pc_rows_bytes(const Plan &p, int bf) {
    return ((size_t)(bf + p.geo16.J - 1) * lds_stride(p.geo16.Hp, 2) * 2 + 15) & ~size_t(15);
}
inline size_t pc_lds_bytes(const Plan &p, int bf) {
    return 2 * pc_rows_bytes(p, bf) + (size_t)(bf + p.geo16.J - 1) * p.H * 4;
}
inline bool pc_fits(const Plan &p) {
    const int ng = p.geo16.n_groups;
    return ng == 10 || ng == 16 || ng == 20 || ng == 25;
}

// K-split 16-bit kernel (frames too long for one wave's basis tile): two waves per row tile,
// the first holding the k-groups of the first J0 hop segments (ns0 groups), the second the
// rest (ns1 <= ns0 groups).  The split must leave the second half's groups at the first
// half's columns, J0 rows further down, so the second wave reads the same offsets shifted by
// delta = J0 S elements.  The halves need a compiled register tile (ks_supported).
struct KSplit {
    int ns0, ns1, delta;    // delta < 0: no valid split
};
inline bool ks_supported(int ns0, int ns1) {
    return (ns0 == ns1 && (ns0 == 16 || ns0 == 20 || ns0 == 25 || ns0 == 32)) || (ns0 == 40 && ns1 == 35);
}
inline KSplit ks_split(const Plan &p, int S) {
    const Geometry &g = p.geo16;
    const int G = g.n_groups;
    for (int j0 = 1; j0 < g.J; ++j0) {
        int h0 = 0;
        while (h0 < G && g.seg_of_group[h0] < j0) ++h0;
        const int h1 = G - h0;
        if (h1 <= 0 || h1 > h0 || !ks_supported(h0, h1)) continue;
        bool ok = true;
        for (int i = 0; i < h1 && ok; ++i)
            ok = g.seg_of_group[h0 + i] == g.seg_of_group[i] + j0 && g.col_of_group[h0 + i] == g.col_of_group[i];
        if (ok) return {h0, h1, j0 * S};
    }
    return {0, 0, -1};
}
inline bool ks_fits(const Plan &p) { return ks_split(p, lds_stride(p.geo16.Hp, 2)).delta > 0; }
inline int ks_row_groups(const Plan &p) { return (p.row_tiles + 3) / 4; }
inline size_t ks_scratch_offset(const Plan &p, int bf) {
    return ((size_t)(bf + p.geo16.J - 1) * lds_stride(p.geo16.Hp, 2) * 2 + 15) & ~size_t(15);
}
inline size_t ks_red_offset(const Plan &p, int bf) {
    return (ks_scratch_offset(p, bf) + (size_t)(bf + p.geo16.J - 1) * p.H * 4 + 15) & ~size_t(15);
}
inline size_t ks_lds_bytes(const Plan &p, int bf) {
    const int rg = ks_row_groups(p);
    return ks_red_offset(p, bf) + (size_t)((p.row_tiles + rg - 1) / rg) * 2048 * 4;
}

// per-family launchers (melt_f32.hip, melt_h16.hip, melt_f8.hip)
melt_status launch_melt_f32(Plan &p, const FwdTask &t, bool warp_specialised);
enum H16Kind { H16_LDS_DMA = 0, H16_REGISTER_STAGED = 1, H16_FRAME_SPLIT = 2, H16_K_SPLIT = 3, H16_PIPELINED = 4,
               H16_ROW_PAIR = 5, H16_PC12 = 6 };
melt_status launch_melt_h16(Plan &p, const FwdTask &t, H16Kind kind, int bf, int nbuf = 1);
melt_status launch_melt_f8(Plan &p, const FwdTask &t, bool lds_dma, int bf);
melt_status launch_melt_f8_pc(Plan &p, const FwdTask &t, int bf);
size_t f8_pc_lds_bytes(const Plan &p, int bf);
size_t f8_as_lds_bytes(const Plan &p, int bf);   // LDS of the direct-to-LDS FP8 kernel
melt_status launch_melt_f8b(Plan &p, const FwdTask &t, int bf, bool pc);   // FP8 with 32-sample block scales
size_t f8b_lds_bytes(const Plan &p, int bf);
size_t f8b_pc_lds_bytes(const Plan &p, int bf);   // its producer/consumer form (dynamic LDS)
size_t f8b_pc_static_bytes();

}  // namespace melt
