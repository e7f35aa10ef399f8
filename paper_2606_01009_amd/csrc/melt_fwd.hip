// MelT forward: chunk schedule of a ragged batch, basis packing for every operand format,
// the table of kernel variants and the dispatch to them.
#include <cstdio>
#include <mutex>
#include "fwd_common.h"

namespace melt {

// ------------------------------------------------------------------ schedule

// inclusive prefix sum over the 64 lanes of a wave (shuffles, no barrier)
__device__ __forceinline__ int64_t wave_scan(int64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// a / b for 0 <= a, 0 < b < 2^31: 32-bit division when a fits (the 64-bit one is a long
// software sequence)
__device__ __forceinline__ int64_t udiv_nonneg(int64_t a, int b) {
    return a <= 0x7fffffff ? (int64_t)((uint32_t)a / (uint32_t)b) : a / b;
}

// Chunk table for at most 64 clips, with no barrier: every wave holds the clips in its lanes
// (lane = clip) and scans their frame and chunk counts in registers; entry q (taken by lane
// q % 64 of wave (q / 64) % 16) finds its clip by a binary search over the lanes' chunk
// prefix sums (shuffles, every lane active).  n_chunks receives min(total, cap).
__global__ __launch_bounds__(1024) void k_schedule64(const int64_t *__restrict__ off, int n_clips, int N, int H,
                                                     int bf, Chunk *__restrict__ tab, int64_t cap,
                                                     int *__restrict__ n_out) {
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t st = 0, L = 0;
    if (lane < n_clips) {
        st = off[lane];
        L = off[lane + 1] - st;
    }
    const int64_t T = (L >= N) ? 1 + udiv_nonneg(L - N, H) : 0;
    const int64_t K = udiv_nonneg(T + bf - 1, bf);
    const int64_t pf = wave_scan(T, lane), pc = wave_scan(K, lane);
    const int64_t total = __shfl(pc, 63, 64);
    const int64_t nv = total < cap ? total : cap;
    // the same on every lane; made scalar so the loop below keeps every lane active
    const int64_t n = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(nv >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)nv));
    for (int64_t q0 = 64 * w; q0 < n; q0 += 1024) {      // wave-uniform trip count
        const int64_t q = q0 + lane;
        int t = 0;                                       // clips whose chunks all precede q
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1)
            if (__shfl(pc, t + d - 1, 64) <= q) t += d;
        // every shuffle runs on all lanes: a lane left out of one (a shuffle under a
        // condition) would read as zero to the lanes that source from it
        const int tp = t > 0 ? t - 1 : 0;
        const int64_t pc_p = __shfl(pc, tp, 64), pf_p = __shfl(pf, tp, 64);
        const int64_t pf_t = __shfl(pf, t & 63, 64);
        const int64_t st_t = __shfl(st, t & 63, 64), L_t = __shfl(L, t & 63, 64);
        const int64_t kc0 = t > 0 ? pc_p : 0;
        const int64_t fb = t > 0 ? pf_p : 0;
        const int64_t Tt = pf_t - fb;
        if (q < n) {
            const int64_t k = q - kc0;
            Chunk e;
            e.sample_start = st_t + k * bf * (int64_t)H;
            e.sample_end = st_t + L_t;
            e.out_row = fb + k * bf;
            e.n_frames = (int)((Tt - k * bf) < bf ? (Tt - k * bf) : bf);
            e.clip = t;
            tab[q] = e;
        }
    }
    if (threadIdx.x == 0) *n_out = (int)n;
}

// One workgroup: prefix sums over the clips of frame counts and chunk counts, then the
// chunk table.  n_chunks receives min(total, cap).
__global__ __launch_bounds__(1024) void k_schedule(const int64_t *__restrict__ off, int n_clips, int N,
                                                   int H, int bf, Chunk *__restrict__ tab, int64_t cap,
                                                   int *__restrict__ n_out) {
    __shared__ int64_t sf[1024], sc[1024], s_start[1024], s_len[1024];
    __shared__ int64_t wf[16], wc[16];
    __shared__ int64_t carry_f, carry_c;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry_f = carry_c = 0;
    for (int base = 0; base < n_clips; base += 1024) {
        const int c = base + tid;
        int64_t st = 0, L = 0;
        if (c < n_clips) {
            st = off[c];
            L = off[c + 1] - st;
        }
        const int64_t T = (L >= N) ? 1 + udiv_nonneg(L - N, H) : 0;
        const int64_t K = udiv_nonneg(T + bf - 1, bf);
        // inclusive prefix sums of T and K over the block: within each wave, then across the
        // 16 wave totals
        const int64_t pf = wave_scan(T, lane), pc = wave_scan(K, lane);
        if (lane == 63) {
            wf[w] = pf;
            wc[w] = pc;
        }
        __syncthreads();
        int64_t of = 0, oc = 0;
        for (int k = 0; k < w; ++k) {
            of += wf[k];
            oc += wc[k];
        }
        sf[tid] = pf + of;
        sc[tid] = pc + oc;
        s_start[tid] = st;
        s_len[tid] = L;
        __syncthreads();
        // entries of this block of clips, written by all threads: entry q belongs to the
        // first clip t whose inclusive chunk prefix exceeds q (binary search)
        const int64_t total = sc[1023];
        for (int64_t q = tid; q < total; q += 1024) {
            int lo = 0, hi = 1023;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sc[mid] > q) hi = mid;
                else lo = mid + 1;
            }
            const int t = lo;
            const int64_t kc0 = t > 0 ? sc[t - 1] : 0;         // clip t's first entry in the block
            const int64_t k = q - kc0;                          // chunk index within the clip
            const int64_t Tt = sf[t] - (t > 0 ? sf[t - 1] : 0);
            const int64_t fb = carry_f + (t > 0 ? sf[t - 1] : 0);
            const int64_t idx = carry_c + q;
            if (idx >= cap) break;
            Chunk e;
            e.sample_start = s_start[t] + k * bf * (int64_t)H;
            e.sample_end = s_start[t] + s_len[t];
            e.out_row = fb + k * bf;
            e.n_frames = (int)((Tt - k * bf) < bf ? (Tt - k * bf) : bf);
            e.clip = base + t;
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

// 16-bit pack: [rt][group][lane][8]; kind 0 = bf16, 1 = fp16, 2 = bf16 low part of the split,
// 3 = fp16 low part of the split
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
        } else if (kind == 3) {
            const float hi = f16_bits_to_f32(f32_to_f16_bits(v));
            r = f32_to_f16_bits(v - hi);
        } else {
            const float hi = bf16_bits_to_f32(f32_to_bf16_bits(v));
            r = f32_to_bf16_bits(v - hi);
        }
        out[i] = r;
    }
}

// E4M3 pack of the basis: [rt][group of 64][lane][32 bytes].  blocks = 0: lane half h holds
// k = 64 g + 32 h + byte (any k order serves a product with unit block scales, as long as the
// frames use the same).  blocks = 1: the order in which the 32x32x64 MFMA's two 32-k scale
// blocks are whole: bytes 0-15 of half h are k = 64 g + 16 h + byte (block 0), bytes 16-31
// are k = 64 g + 32 + 16 h + byte - 16 (block 1).  Row scales r_j = 448 / max_n |W_j| (FP32);
// rinv[rt][i] = 1 / r_j of tile row i.  One workgroup of 256 threads per row tile: eight
// threads per tile row share its maximum, then every thread packs whole 4-byte words.
__global__ __launch_bounds__(256) void k_pack_f8(const float *__restrict__ b32, int M, int N, int NG, int blocks,
                                                 unsigned *__restrict__ out, float *__restrict__ rinv) {
    __shared__ float rmax[32];
    const int rt = blockIdx.x, t = threadIdx.x;
    {
        const int i = t >> 3, sub = t & 7;
        int ml, part;
        tile_row_to_mel(i, ml, part);
        const int mel = rt * 16 + ml;
        float mx = 0.0f;
        if (mel < M)
            for (int n = sub; n < N; n += 8) mx = fmaxf(mx, fabsf(b32[(size_t)(part * M + mel) * N + n]));
        // the eight threads of a row are consecutive lanes of one wave
        mx = fmaxf(mx, __shfl_xor(mx, 1, 64));
        mx = fmaxf(mx, __shfl_xor(mx, 2, 64));
        mx = fmaxf(mx, __shfl_xor(mx, 4, 64));
        if (sub == 0) {
            rmax[i] = mx;
            rinv[rt * 32 + i] = mx > 0.0f ? 1.0f / __fdiv_rn(448.0f, mx) : 1.0f;
        }
    }
    __syncthreads();
    for (int idx = t; idx < NG * 512; idx += 256) {
        const int w = idx & 7, lane = (idx >> 3) & 63, g = idx >> 9;
        int ml, part;
        tile_row_to_mel(lane & 31, ml, part);
        const int mel = rt * 16 + ml;
        const float mx = rmax[lane & 31];
        const float sc = mx > 0.0f ? __fdiv_rn(448.0f, mx) : 1.0f;
        float v[4];
        for (int e = 0; e < 4; ++e) {
            const int bb = 4 * w + e, h = lane >> 5;
            const int k = blocks ? g * 64 + 32 * (bb >> 4) + 16 * h + (bb & 15) : g * 64 + 32 * h + bb;
            v[e] = (mel < M && k < N) ? __fmul_rn(b32[(size_t)(part * M + mel) * N + k], sc) : 0.0f;
        }
        out[(((size_t)rt * NG + g) * 64 + lane) * 8 + w] = fp8x4(v[0], v[1], v[2], v[3]);
    }
}

// ------------------------------------------------------------------ host side

namespace {

melt_status upload_ints(const std::vector<int> &v, int **d) {
    if (hipMalloc(d, sizeof(int) * (v.size() + 1)) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "hipMalloc");
    return hip_check(hipMemcpy(*d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice), "hipMemcpy");
}

}  // namespace

melt_status pack_tables_upload(Plan &p) {
    melt_status st = upload_ints(p.geo32.seg_of_group, &p.d_seg32);
    if (st == MELT_OK) st = upload_ints(p.geo32.col_of_group, &p.d_col32);
    if (st == MELT_OK) st = upload_ints(p.geo16.seg_of_group, &p.d_seg16);
    if (st == MELT_OK) st = upload_ints(p.geo16.col_of_group, &p.d_col16);
    return st;
}

// Re-packs the FP32 basis d_basis32 into the layout of the plan's precision (the only one
// its kernels read) and the backward's dx layout, enqueued on `s`: no allocation and no
// host synchronisation (the k-group tables were uploaded at plan creation).
melt_status pack_basis(Plan &p, hipStream_t s) {
    const int RT = p.row_tiles;
    switch (p.cfg.precision) {
    case MELT_PREC_FP32:
        k_pack_f32<<<256, 256, 0, s>>>(p.d_basis32, p.M, p.N, p.H, p.d_seg32, p.d_col32, p.geo32.n_groups, RT,
                                       (float *)p.d_pack_f32);
        break;
    case MELT_PREC_FP8_E4M3:
    case MELT_PREC_FP8_E4M3_BLOCK32:
        k_pack_f8<<<RT, 256, 0, s>>>(p.d_basis32, p.M, p.N, (p.N + 63) / 64,
                                     p.cfg.precision == MELT_PREC_FP8_E4M3_BLOCK32 ? 1 : 0, (unsigned *)p.d_pack_f8,
                                     p.d_rowscale);
        break;
    default: {
        const int kind_hi = prec_f16(p) ? 1 : 0;
        k_pack_h16<<<256, 256, 0, s>>>(p.d_basis32, p.M, p.N, p.H, p.d_seg16, p.d_col16, p.geo16.n_groups, RT, kind_hi,
                                       (unsigned short *)p.d_pack_h16);
        if (prec_split(p))
            k_pack_h16<<<256, 256, 0, s>>>(p.d_basis32, p.M, p.N, p.H, p.d_seg16, p.d_col16, p.geo16.n_groups, RT,
                                           kind_hi == 1 ? 3 : 2, (unsigned short *)p.d_pack_lo);
    }
    }
    const melt_status st = hip_check(hipGetLastError(), "pack basis");
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

melt_status launch_schedule(Plan &p, int which, const int64_t *d_off, int n_clips, int bf_max, int64_t n_frames,
                            hipStream_t s) {
    // Chunks of at most bf_max frames (the kernel's LDS image).  The comparator sizes its
    // chunks to the batch (whole sub-tasks, a few chunks per resident wave); measured, the
    // same for the MelT kernels costs more in per-chunk overhead than it gains, so their
    // chunks keep the full size.
    int bf = bf_max;
    if (which == 1 && n_frames > 0) bf = std::min(bf_max, stft_batch_chunk_frames(p, n_frames));
    const int64_t need = n_frames / bf + n_clips + 1;
    melt_status st = ensure_chunks(p, which, need);
    if (st != MELT_OK) return st;
    if (n_clips <= 64)
        k_schedule64<<<1, 1024, 0, s>>>(d_off, n_clips, p.N, p.H, bf, p.d_chunks[which], p.chunk_cap[which],
                                        p.d_nchunks + which);
    else
        k_schedule<<<1, 1024, 0, s>>>(d_off, n_clips, p.N, p.H, bf, p.d_chunks[which], p.chunk_cap[which],
                                      p.d_nchunks + which);
    st = hip_check(hipGetLastError(), "schedule launch");
    if (st == MELT_OK) {
        p.prepared_frames[which] = n_frames;
        p.prepared_bf[which] = bf;
        p.prepared_clips[which] = n_clips;
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
//   FP32       frame-split with staging waves, frame-split with register prefetch
//   BF16/FP16  the 12-wave producer/consumer kernel (96- or 64-frame chunks) where its
//              register tiles and LDS fit; row pairs (two basis tiles per wave) where they fit;
//              row-split with direct-to-LDS staging (one span buffer: 128- then 64-frame
//              chunks; then two span buffers), producer/consumer row-split (one span, then
//              two; only with producer waves), row-split with register staging, K-split (frames
//              too long for one wave's tile), frame-split (the fallback; for the split
//              precisions only where no register-tile kernel applies)
//   BF16X3 / FP16X3  the 8-wave producer/consumer kernel (hi and lo tiles, 64-frame chunks)
//              where it fits, then as above without row pairs and K-split, with one-span
//              chunks of 96 then 64 frames
//   FP8        row-split with direct-to-LDS staging (the largest chunk that fits LDS; 64-frame
//              chunks at two workgroups per CU), row-split with register staging, then the
//              producer/consumer kernel (first beyond 8 row tiles, which the others do not take)
//   FP8 with 32-sample block scales  producer/consumer block-scaled kernel, then the
//              one-buffer block-scaled kernel with 160- and 128-frame chunks
enum VariantKind { V_F32_WS, V_F32_FS, V_H16_PP, V_H16_AS, V_H16_AP, V_H16_RS, V_H16_KS, V_H16_FS, V_F8_AS, V_F8_RS,
                   V_F8B_AS, V_F8B_PC, V_H16_PC, V_F8_PC };
struct Variant {
    VariantKind kind;
    int bf;          // frames per chunk
    int nbuf = 1;    // FP32 span buffers of the direct-to-LDS 16-bit kernel
};

static std::vector<Variant> variant_list(const Plan &p) {
    std::vector<Variant> v;
    switch (p.cfg.precision) {
    case MELT_PREC_FP32:
        v.push_back({V_F32_WS, kBF32});
        v.push_back({V_F32_FS, kBF32});
        break;
    case MELT_PREC_FP8_E4M3: {
        // up to 8 row tiles: the largest all-wave chunk that fits LDS (one workgroup per CU),
        // then 64-frame chunks with two workgroups per CU; the producer/consumer kernel (two
        // images and two spans of 64-frame chunks) first beyond 8 row tiles, last otherwise
        const int ng8 = (p.N + 63) / 64;
        const bool pc = (ng8 == 4 || ng8 == 7 || ng8 == 8) && p.H % 4 == 0 && p.N % 4 == 0 &&
                        f8_pc_lds_bytes(p, 64) + 4 * sizeof(Chunk) + 8 * 32 * 4 <= (size_t)kMaxLds;
        if (pc && p.row_tiles > 8) v.push_back({V_F8_PC, 64});
        for (int bf : {128, 96, 64, 32})
            if (f8_as_lds_bytes(p, bf) + kRingBytes <= (size_t)kMaxLds) {
                v.push_back({V_F8_AS, bf});
                break;
            }
        if (!v.empty() && v.back().bf > 64 && 2 * (f8_as_lds_bytes(p, 64) + kRingBytes) <= (size_t)kMaxLds)
            v.push_back({V_F8_AS, 64});
        v.push_back({V_F8_RS, kBF32});
        if (pc && p.row_tiles <= 8) v.push_back({V_F8_PC, 64});
        break;
    }
    case MELT_PREC_FP8_E4M3_BLOCK32:
        // producer/consumer (the largest chunk whose two row buffers fit; three waves per SIMD,
        // so a basis tile of at most 8 k-groups of 64), then the one-buffer kernel at 160- and
        // 128-frame chunks
        for (int bf : {128, 96, 64})
            if ((p.N + 63) / 64 <= 8 && f8b_pc_lds_bytes(p, bf) + f8b_pc_static_bytes() <= (size_t)kMaxLds) {
                v.push_back({V_F8B_PC, bf});
                break;
            }
        for (int bf : {160, 128})
            if (f8b_lds_bytes(p, bf) + kRingBytes <= (size_t)kMaxLds) v.push_back({V_F8B_AS, bf});
        if (v.empty()) v.push_back({V_F8B_AS, 32});    // unsupported geometry: the launch reports it
        break;
    default: {
        const bool x3 = prec_split(p);
        // 12-wave producer/consumer first where it fits (96 then 64 frames per chunk), then row
        // pairs (two basis tiles per wave, 128 frames per chunk)
        if (!x3 && pc_fits(p))
            for (int bf : {96, 64})
                if (pc_lds_bytes(p, bf) + 4 * sizeof(Chunk) <= (size_t)kMaxLds) {
                    v.push_back({V_H16_PC, bf});
                    break;
                }
        // the split precisions' producer/consumer form (8 waves, hi and lo rows; 64-frame
        // chunks, row groups of at most 5 tiles): their default where it fits with at most 4
        // row groups (each group converts every chunk again: at 32 row tiles, 7 groups, the
        // row-split kernel is faster), the last variant otherwise
        const bool pc_x3 = x3 && pc_fits(p) && pc_x3_lds_bytes(p, 64) + 4 * sizeof(Chunk) <= (size_t)kMaxLds;
        const bool pc_x3_first = pc_x3 && (p.row_tiles + 4) / 5 <= 4;
        if (pc_x3_first) v.push_back({V_H16_PC, 64});
        if (!x3 && ap_fits(p) && as_lds_bytes(p, 128) + kRingBytes <= (size_t)kMaxLds) v.push_back({V_H16_AP, 128});
        if (as_fits(p)) {
            // one span buffer (128 then 64 frames per chunk; 96 then 64 for BF16X3), then two
            for (int bf : {128, 96, 64}) {
                if (bf == (x3 ? 128 : 96)) continue;
                if (as_lds_bytes(p, bf) + kRingBytes <= (size_t)kMaxLds) v.push_back({V_H16_AS, bf, 1});
            }
            for (int bf : {96, 64})
                if (as_lds_bytes(p, bf, 2) + kRingBytes <= (size_t)kMaxLds) {
                    v.push_back({V_H16_AS, bf, 2});
                    break;
                }
        }
        // row pairs (two basis tiles per wave, 128 frames per chunk)
        if (pp_fits(p)) {
            // producer/consumer: one span (96 or 64 frames per chunk), then two spans
            for (int bf : {96, 64})
                if (pp_lds_bytes(p, bf, 1) + kRingBytes <= (size_t)kMaxLds) {
                    v.push_back({V_H16_PP, bf, 1});
                    break;
                }
            for (int bf : {96, 64})
                if (pp_lds_bytes(p, bf, 2) + kRingBytes <= (size_t)kMaxLds) {
                    v.push_back({V_H16_PP, bf, 2});
                    break;
                }
        }
        if (rs_fits(p)) v.push_back({V_H16_RS, 128});
        if (!x3 && !as_fits(p) && ks_fits(p))
            for (int bf : {64, 32})
                if (ks_lds_bytes(p, bf) + kRingBytes <= (size_t)kMaxLds) {
                    v.push_back({V_H16_KS, bf});
                    break;
                }
        if (pc_x3 && !pc_x3_first) v.push_back({V_H16_PC, 64});
        // frame-split: the fallback for every 16-bit precision (the split ones only where no
        // register-tile kernel applies)
        if (!x3 || v.empty()) v.push_back({V_H16_FS, kBF32});
    }
    }
    return v;
}

void init_variants(Plan &p) {
    const std::vector<Variant> v = variant_list(p);
    p.n_variants = (int)std::min<size_t>(v.size(), Plan::kMaxVariants);
    for (int i = 0; i < p.n_variants; ++i) {
        p.var_kind[i] = v[i].kind;
        p.var_bf[i] = v[i].bf;
        p.var_nbuf[i] = v[i].nbuf;
    }
}

static Variant variant_at(const Plan &p, int i) {
    if (p.n_variants == 0) return {V_H16_FS, kBF32};    // unsupported geometry: the launch reports it
    const int k = i >= 0 && i < p.n_variants ? i : 0;
    return {(VariantKind)p.var_kind[k], p.var_bf[k], p.var_nbuf[k]};
}

int forward_variants(const Plan &p) { return p.n_variants; }

const char *forward_variant_name(const Plan &p, int i) {
    static thread_local char buf[64];
    if (i < 0 || i >= p.n_variants) return "none";
    const Variant v = variant_at(p, i);
    const char *k = v.kind == V_H16_PP   ? (v.nbuf == 2 ? "h16-producer-consumer-2span" : "h16-producer-consumer")
                    : v.kind == V_F32_WS ? "f32-frame-split-warp-specialised"
                    : v.kind == V_F32_FS ? "f32-frame-split"
                    : v.kind == V_H16_AS ? (v.nbuf == 2 ? "h16-row-split-lds-dma2" : "h16-row-split-lds-dma")
                    : v.kind == V_H16_AP ? "h16-row-pair-lds-dma"
                    : v.kind == V_H16_PC ? (p.cfg.precision == MELT_PREC_BF16X3 || p.cfg.precision == MELT_PREC_FP16X3
                                                ? "h16-producer-consumer-8w-lds-dma"
                                                : "h16-producer-consumer-12w-lds-dma")
                    : v.kind == V_H16_RS ? "h16-row-split"
                    : v.kind == V_H16_KS ? "h16-k-split-lds-dma"
                    : v.kind == V_H16_FS ? "h16-frame-split"
                    : v.kind == V_F8_AS  ? "f8-row-split-lds-dma"
                    : v.kind == V_F8_PC  ? "f8-producer-consumer-lds-dma"
                    : v.kind == V_F8B_AS ? "f8-block-scaled-lds-dma"
                    : v.kind == V_F8B_PC ? "f8-block-scaled-producer-consumer-lds-dma"
                                            : "f8-row-split";
    std::snprintf(buf, sizeof(buf), "%s-bf%d", k, v.bf);
    return buf;
}

int melt_chunk_frames(const Plan &p, int variant) { return variant_at(p, variant).bf; }
int melt_chunk_frames(const Plan &p) { return melt_chunk_frames(p, p.tune_variant); }

melt_status launch_melt_main(Plan &p, const float *d_wave, float *d_out, float *d_proj, hipStream_t s) {
    const int64_t n_frames = p.prepared_frames[0];
    if (n_frames < 0) return set_error(MELT_E_INVALID_ARG, "no batch prepared");
    if (n_frames == 0) return MELT_OK;
    const int v = p.prepared_variant;
    // chunk count bound: every clip ends in at most one partial chunk
    const int64_t est = n_frames / p.prepared_bf[0] + p.prepared_clips[0];
    if (p.K == 0)
        return launch_melt_table(p, v, p.d_chunks[0], p.d_nchunks, est, n_frames, d_wave, d_out, d_proj, s);
    // MFCCT (Eq. mfcct_matrix): log-Mel rows into the plan workspace, then C = L D^T
    melt_status st = ensure_lmel(p, n_frames);
    if (st == MELT_OK)
        st = launch_melt_table(p, v, p.d_chunks[0], p.d_nchunks, est, n_frames, d_wave, p.d_lmel, d_proj, s);
    if (st != MELT_OK) return st;
    return launch_cepstrum(p, p.d_lmel, n_frames, d_out, s);
}

melt_status launch_melt_table(Plan &p, int variant, const Chunk *tab, const int *n_tab, int64_t est_chunks,
                              int64_t n_frames, const float *d_wave, float *d_out, float *d_proj, hipStream_t s) {
    const FwdTask t{tab, n_tab, est_chunks, n_frames, d_wave, d_out, d_proj, s};
    const Variant v = variant_at(p, variant);
    switch (v.kind) {
    case V_F32_WS: return launch_melt_f32(p, t, true);
    case V_F32_FS: return launch_melt_f32(p, t, false);
    case V_H16_PP: return launch_melt_h16(p, t, H16_PIPELINED, v.bf, v.nbuf);
    case V_H16_AS: return launch_melt_h16(p, t, H16_LDS_DMA, v.bf, v.nbuf);
    case V_H16_AP: return launch_melt_h16(p, t, H16_ROW_PAIR, v.bf);
    case V_H16_PC: return launch_melt_h16(p, t, H16_PC12, v.bf);
    case V_H16_RS: return launch_melt_h16(p, t, H16_REGISTER_STAGED, v.bf);
    case V_H16_KS: return launch_melt_h16(p, t, H16_K_SPLIT, v.bf);
    case V_H16_FS: return launch_melt_h16(p, t, H16_FRAME_SPLIT, v.bf);
    case V_F8_AS: return launch_melt_f8(p, t, true, v.bf);
    case V_F8_PC: return launch_melt_f8_pc(p, t, v.bf);
    case V_F8_RS: return launch_melt_f8(p, t, false, v.bf);
    case V_F8B_AS: return launch_melt_f8b(p, t, v.bf, false);
    case V_F8B_PC: return launch_melt_f8b(p, t, v.bf, true);
    }
    return set_error(MELT_E_UNSUPPORTED, "precision not implemented");
}

// ------------------------------------------------------------------ allocation-free forward
// melt_forward_noalloc keeps its chunk count and chunk table in a fixed device array instead
// of the plan's (growable) workspace, for callers that cannot allocate.  Every GPU the
// library runs on holds its own copy until the process ends; the host side reaches it only
// through the address hipGetSymbolAddress returns for that device (the array's name in host
// code is not a device address).  All calls on one GPU share it: calls that overlap in time
// on one GPU race.
constexpr size_t kScratchBytes = size_t(1) << 20;    // 1 MiB per device
constexpr size_t kScratchTable = 256;                // byte offset of the table (count at 0)
constexpr int64_t kScratchChunks = int64_t((kScratchBytes - kScratchTable) / sizeof(Chunk));
constexpr int kScratchDevices = 64;
static_assert(kScratchChunks == 32760, "chunk capacity stated in melt.h");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kScratchDevices] = {};

// Called once per device at plan creation, with `device` current.
melt_status scratch_init(int device) {
    if (device < 0 || device >= kScratchDevices) return set_error(MELT_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return MELT_OK;
    void *ptr = nullptr;
    const melt_status st = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st != MELT_OK) return st;
    g_scratch_ptr[device] = ptr;
    return MELT_OK;
}

melt_status forward_noalloc(Plan &p, const float *d_wave, const int64_t *d_off, int n_clips, int64_t n_frames,
                            float *d_out, hipStream_t s) {
    if (p.K > 0) return set_error(MELT_E_UNSUPPORTED, "melt_forward_noalloc: MELT_OUT_MFCC needs a log-Mel workspace");
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_ptr[p.device];
    }
    if (!base) return set_error(MELT_E_HIP, "melt_forward_noalloc: no scratch address for this device");
    const int v = p.tune_variant;
    const int bf = melt_chunk_frames(p, v);
    // every clip ends in at most one partial chunk
    const int64_t need = n_frames / bf + n_clips + 1;
    if (need > kScratchChunks)
        return set_error(MELT_E_SHAPE, "melt_forward_noalloc: n_frames / " + std::to_string(bf) + " + n_clips + 1 = " +
                                           std::to_string(need) + " chunk entries exceed the 32760 of the scratch");
    int *n_tab = static_cast<int *>(base);
    Chunk *tab = reinterpret_cast<Chunk *>(static_cast<unsigned char *>(base) + kScratchTable);
    // the schedule kernels write the count unconditionally, so nothing in the scratch needs clearing
    if (n_clips <= 64) k_schedule64<<<1, 1024, 0, s>>>(d_off, n_clips, p.N, p.H, bf, tab, kScratchChunks, n_tab);
    else k_schedule<<<1, 1024, 0, s>>>(d_off, n_clips, p.N, p.H, bf, tab, kScratchChunks, n_tab);
    const melt_status st = hip_check(hipGetLastError(), "schedule launch");
    if (st != MELT_OK) return st;
    return launch_melt_table(p, v, tab, n_tab, need - 1, n_frames, d_wave, d_out, nullptr, s);
}

}  // namespace melt
