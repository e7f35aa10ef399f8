// MelT forward, 16-bit operands (BF16, FP16, split-BF16x3): v_mfma_f32_32x32x16_{bf16,f16}
// with FP32 accumulation (Eq. dmp_projection, Eq. dmp_matrix_energy, Eq. meltf).
#include "fwd_common.h"

namespace melt {

// ------------------------------------------------------------------ 16-bit register-tile MFMA sweep
//
// Two 32-frame tiles (LDS rows at l0 and l1) against a wave's basis tile held in registers:
// NS k-groups of 16, one v_mfma_f32_32x32x16 per tile and group.  The frame fragments are
// read D groups ahead into a ring of registers, and scheduling barriers keep each group's
// reads above the multiplies they overlap, so LDS latency hides behind D groups of MFMAs.
// X3 adds hi*lo + lo*hi products from the low parts (basis in Al, frames at lo_off), in
// bfloat16 or binary16 as the operands.  D is
// the depth of the fragment ring (a shallower ring frees registers for a longer basis tile).
template <int NS, bool X3, bool IS_F16, int D = (X3 ? 1 : 4)>
__device__ __forceinline__ void mfma_sweep(const uint4 (&A)[NS], const uint4 (&Al)[X3 ? NS : 1],
                                           const unsigned short *l0, const unsigned short *l1,
                                           const GroupTableBig &gt, int lo_off, f32x16 &acc0, f32x16 &acc1) {
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
            if constexpr (X3) {
                const f16x8 al = __builtin_bit_cast(f16x8, Al[s]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, __builtin_bit_cast(f16x8, b0[slot]), acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, __builtin_bit_cast(f16x8, b1[slot]), acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, __builtin_bit_cast(f16x8, c0[slot]), acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, __builtin_bit_cast(f16x8, c1[slot]), acc1, 0, 0, 0);
            }
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

// Sweep over one 32-frame tile into one accumulator (back-to-back MFMAs on the same
// accumulator forward their result).  X3 (split bfloat16 or binary16): hi*hi, lo*hi and hi*lo per k-group, which keeps
// the hi and lo basis tiles (8 NS VGPRs) beside a single tile's 16 accumulators.
template <int NS, bool X3, bool IS_F16>
__device__ __forceinline__ void mfma_sweep1(const uint4 (&A)[NS], const uint4 (&Al)[X3 ? NS : 1],
                                            const unsigned short *l0, const GroupTableBig &gt, int lo_off,
                                            f32x16 &acc) {
    constexpr int D = X3 ? 1 : 4;
    uint4 b[D], c[X3 ? D : 1];
    auto fetch = [&](int s, int slot) {
        const int o = gt.lds_off[s];
        b[slot] = *(const uint4 *)(l0 + o);
        if constexpr (X3) c[slot] = *(const uint4 *)(l0 + lo_off + o);
    };
#pragma unroll
    for (int s = 0; s < D && s < NS; ++s) fetch(s, s);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int slot = s % D;
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (IS_F16) {
            const f16x8 ah = __builtin_bit_cast(f16x8, A[s]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, __builtin_bit_cast(f16x8, b[slot]), acc, 0, 0, 0);
            if constexpr (X3) {
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, Al[s]),
                                                             __builtin_bit_cast(f16x8, b[slot]), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, __builtin_bit_cast(f16x8, c[slot]), acc, 0, 0, 0);
            }
        } else {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, A[s]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, __builtin_bit_cast(bf16x8, b[slot]), acc, 0, 0, 0);
            if constexpr (X3) {
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, Al[s]),
                                                              __builtin_bit_cast(bf16x8, b[slot]), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, __builtin_bit_cast(bf16x8, c[slot]), acc, 0, 0, 0);
            }
        }
        if (s + D < NS) fetch(s + D, slot);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// a chunk descriptor from an LDS slot, its fields made wave-uniform
__device__ __forceinline__ Chunk ring_slot(const Chunk *slots, int i) {
    Chunk e = slots[i];
    e.sample_start = uniform64(e.sample_start);
    e.sample_end = uniform64(e.sample_end);
    e.out_row = uniform64(e.out_row);
    e.n_frames = __builtin_amdgcn_readfirstlane(e.n_frames);
    e.clip = __builtin_amdgcn_readfirstlane(e.clip);
    return e;
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

// ------------------------------------------------------------------ 16-bit row-split kernel, direct-to-LDS staging
//
// Row-split 16-bit kernel with direct-to-LDS staging (default for BF16/FP16/BF16X3): as
// k_melt_h16_rs, but the chunks' spans are copied into FP32 scratch spans while earlier
// chunks are multiplied; after a barrier all threads convert the current span into the
// operand rows.  Outputs are stored straight from the accumulators (8 consecutive Mel bins
// per lane).
//
// Span buffers: with nbuf = 1 the copy of chunk c+1 is issued after chunk c's conversion and
// lands during its multiplies.  With nbuf = 2 the copy of chunk c+2 goes into the span just
// converted, so a copy is in flight across a whole iteration, conversion included, and the
// wait at the end of the iteration is for the copy issued one iteration earlier.
//
// The copies are issued by the waves with the least multiply work (those sharing a row tile,
// or idle ones; the upper half of the waves when every wave owns a tile).  Only those waves
// wait for them, so the other waves never wait on their own output stores.
//
// Wave layout (balanced over the CU's four SIMDs): waves 0..full-1 each own one row tile and
// sweep every frame tile of the chunk, two at a time; the remaining row tiles (one or two)
// are shared by four waves, psplit per tile, each taking every psplit-th frame tile.  With
// 80 Mel bins (5 row tiles) that is 8 waves, 4 for tile 4, so every SIMD carries 1.25 row
// tiles of work instead of one SIMD carrying two.
template <class Conv, int NS, bool X3, bool IS_F16>
__global__ __launch_bounds__(512) void k_melt_h16_as(FwdArgs a, const uint4 *__restrict__ bhi,
                                                     const uint4 *__restrict__ blo, GroupTableBig gt, int bf,
                                                     int scr_off, int scr_len, int nbuf, int rgroups) {
    extern __shared__ float lds_as[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // row group of this workgroup (fixed for its life, so the basis stays in registers):
    // tiles [grp * gt_n, min(RT, (grp + 1) * gt_n)); waves beyond the group's layout idle
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
    const int lo_off = a.S * (bf + a.J - 1);
    unsigned short *rows = reinterpret_cast<unsigned short *>(lds_as);
    float *span0 = lds_as + scr_off;               // FP32 spans, after the operand rows
    float *span1 = span0 + (nbuf == 2 ? scr_len : 0);
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows, blockDim.x, lo_off);
    uint4 A[NS];
    uint4 Al[X3 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) A[s] = bhi[((size_t)rt * NS + s) * 64 + lane];
    if constexpr (X3) {
#pragma unroll
        for (int s = 0; s < NS; ++s) Al[s] = blo[((size_t)rt * NS + s) * 64 + lane];
    }
    const int nw = blockDim.x >> 6;
    const int wu = __builtin_amdgcn_readfirstlane(wid);
    const int dma0 = L.full < nw ? L.full : nw / 2;    // first copying wave
    const bool dma_wave = wu >= dma0;
    const int nch = *a.n_chunks;
    const int cstep = gridDim.x / rgroups;         // the grid is a multiple of rgroups
    int c = blockIdx.x / rgroups;
    // prologue: every wave copies the first span; the copying waves also start the second
    if (c < nch) async_span(a, read_chunk(a.chunks, c), span0);
    int ahead = 0;
    if (nbuf == 2 && dma_wave && c + cstep < nch)
        ahead = async_span_waves(a, read_chunk(a.chunks, c + cstep), span1, wu - dma0, nw - dma0);
    wait_vm_younger(ahead);
    __shared__ ChunkRing ring;
    for (int it = 0; c < nch; c += cstep, ++it) {
        const int ri = it % kRing;
        if (ri == 0) ring_fill(ring, a.chunks, c, cstep, nch);
        float *cur = (it & 1) ? span1 : span0;
        __syncthreads();                           // span of chunk c has landed; rows are free
        const Chunk ch = ring_get(ring, ri);
        // the copy into `cur`: chunk c + nbuf * cstep.  The iteration ends with the copy of
        // chunk c + cstep landed: with nbuf = 2 the `younger` copies just issued may still fly.
        const int cn = c + nbuf * cstep;
        const Chunk chn = ring_get(ring, ri + nbuf);
        convert_span<Conv>(a, ch, cur, rows, lo_off);
        __syncthreads();                           // rows ready; span `cur` is free
        int younger = 0;
        if (dma_wave && cn < nch) {
            const int n = async_span_waves(a, chn, cur, wu - dma0, nw - dma0);
            younger = nbuf == 2 ? n : 0;
        }
        const int nft = idle ? 0 : (ch.n_frames + 31) >> 5;
        // A copying wave waits ahead of its last tile's stores (so those stores stay in flight
        // across the barrier), or after the loop if it had no tile.
        bool waited = !dma_wave;
        const int step = (P == 1 && !X3) ? 2 : P;
        for (int ft = part; ft < nft; ft += step) {
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            // opaque to the optimiser, so that it does not keep (lane offset + group offset)
            // of every k-group live in registers across the loop
            int off = (ft * 32 + (lane & 31)) * a.S + 8 * (lane >> 5);
            asm volatile("" : "+v"(off));
            const unsigned short *l0 = rows + off;
            if constexpr (!X3) {
                if (step == 2) {
                    const bool two = ft + 1 < nft;
                    // a lone last tile multiplies its own rows twice rather than branching
                    const unsigned short *l1 = two ? l0 + 32 * a.S : l0;
                    mfma_sweep<NS, false, IS_F16>(A, Al, l0, l1, gt, lo_off, acc0, acc1);
                    if (!waited && ft + 2 >= nft) {
                        wait_vm_younger(younger);
                        waited = true;
                    }
                    store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc0);
                    if (two) store_tile(a, ch, rt, (ft + 1) * 32 + (lane & 31), lane, acc1);
                    continue;
                }
            }
            mfma_sweep1<NS, X3, IS_F16>(A, Al, l0, gt, lo_off, acc0);
            if (!waited && ft + step >= nft) {
                wait_vm_younger(younger);
                waited = true;
            }
            store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc0);
        }
        if (!waited) wait_vm_younger(younger);     // no tile for this wave (or a frameless chunk)
    }
}

// ------------------------------------------------------------------ 16-bit row-pair kernel, direct-to-LDS staging
//
// As k_melt_h16_as (one span buffer), with waves that hold the basis tiles of two row tiles in
// registers, so each frame fragment read from LDS feeds two MFMAs: the multiply phase reads
// half as many fragments.  With 2 NS uint4 of basis per lane and eight waves (two per SIMD,
// 256 registers each) it fits up to NS = 20 k-groups (at 25 the two tiles spill).  A variant
// with four waves holding two or three tiles each (one per SIMD) was slower at every shape
// measured: the second wave per SIMD hides more than the halved fragment reads save.  Roles
// for a group of cnt row tiles (pair_role):
//   cnt 8: wave w takes the pair (2 (w/2), 2 (w/2) + 1) on frame tiles of parity w % 2;
//   cnt 5: waves 0-3 take the pairs (0, 1) and (2, 3) on alternate frame tiles, waves 4-7
//          the single tile 4 on every fourth frame tile (each SIMD: 4 + 1 tile products);
//   cnt 4: wave w takes the pair (2 (w/4), 2 (w/4) + 1) on every fourth frame tile.
// Waves 4-7 copy the next chunk's span (the single-tile ones when cnt = 5).
struct PairRole {
    int ta, tb, part, P;    // first tile, second tile (-1: none), first frame tile, frame-tile stride
};
__host__ __device__ inline bool pair_layout_ok(int cnt) { return cnt == 4 || cnt == 5 || cnt == 8; }
__device__ __forceinline__ PairRole pair_role(int cnt, int w) {
    if (cnt == 8) return {2 * (w >> 1), 2 * (w >> 1) + 1, w & 1, 2};
    if (cnt == 4) return {2 * (w >> 2), 2 * (w >> 2) + 1, w & 3, 4};
    if (w < 4) return {2 * (w >> 1), 2 * (w >> 1) + 1, w & 1, 2};
    return {4, -1, w - 4, 4};
}

// one 32-frame tile against two basis tiles: per k-group one fragment read, two MFMAs
template <int NS, bool IS_F16, int D = 2>
__device__ __forceinline__ void mfma_sweep_pair(const uint4 (&A0)[NS], const uint4 (&A1)[NS], const unsigned short *l0,
                                                const GroupTableBig &gt, f32x16 &acc0, f32x16 &acc1) {
    uint4 b[D];
#pragma unroll
    for (int s = 0; s < D && s < NS; ++s) b[s] = *(const uint4 *)(l0 + gt.lds_off[s]);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int slot = s % D;
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (IS_F16) {
            const f16x8 bv = __builtin_bit_cast(f16x8, b[slot]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, A0[s]), bv, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, A1[s]), bv, acc1, 0, 0, 0);
        } else {
            const bf16x8 bv = __builtin_bit_cast(bf16x8, b[slot]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A0[s]), bv, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, A1[s]), bv, acc1, 0, 0, 0);
        }
        if (s + D < NS) b[slot] = *(const uint4 *)(l0 + gt.lds_off[s + D]);
    }
    __builtin_amdgcn_sched_barrier(0);
}

template <class Conv, int NS, bool IS_F16>
__global__ __launch_bounds__(512, 1) void k_melt_h16_ap(FwdArgs a, const uint4 *__restrict__ bhi, GroupTableBig gt,
                                                        int bf, int scr_off) {
    extern __shared__ float lds_ap[];
    const int lane = threadIdx.x & 63;
    const int wu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const PairRole R = pair_role(a.row_tiles, wu);
    unsigned short *rows = reinterpret_cast<unsigned short *>(lds_ap);
    float *span = lds_ap + scr_off;
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows, blockDim.x, 0);
    uint4 A0[NS], A1[NS];
    const uint4 Al[1] = {};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        A0[s] = bhi[((size_t)R.ta * NS + s) * 64 + lane];
        A1[s] = R.tb >= 0 ? bhi[((size_t)R.tb * NS + s) * 64 + lane] : uint4{};
    }
    const bool dma_wave = wu >= 4;
    const int nch = *a.n_chunks;
    int c = blockIdx.x;
    if (c < nch) async_span(a, read_chunk(a.chunks, c), span);
    async_wait();
    __shared__ ChunkRing ring;
    for (int it = 0; c < nch; c += gridDim.x, ++it) {
        const int ri = it % kRing;
        if (ri == 0) ring_fill(ring, a.chunks, c, gridDim.x, nch);
        __syncthreads();                           // span of chunk c has landed; rows are free
        const Chunk ch = ring_get(ring, ri);
        const Chunk chn = ring_get(ring, ri + 1);
        convert_span<Conv>(a, ch, span, rows, 0);
        __syncthreads();                           // rows ready; the span is free
        if (dma_wave && c + (int)gridDim.x < nch) async_span_waves(a, chn, span, wu - 4, 4);
        const int nft = (ch.n_frames + 31) >> 5;
        // a copying wave waits ahead of its last tile's stores, or after the loop
        bool waited = !dma_wave;
        for (int ft = R.part; ft < nft; ft += R.P) {
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            int off = (ft * 32 + (lane & 31)) * a.S + 8 * (lane >> 5);
            asm volatile("" : "+v"(off));
            const unsigned short *l0 = rows + off;
            if (R.tb >= 0) mfma_sweep_pair<NS, IS_F16>(A0, A1, l0, gt, acc0, acc1);
            else mfma_sweep1<NS, false, IS_F16>(A0, Al, l0, gt, 0, acc0);
            if (!waited && ft + R.P >= nft) {
                async_wait();
                waited = true;
            }
            store_tile(a, ch, R.ta, ft * 32 + (lane & 31), lane, acc0);
            if (R.tb >= 0) store_tile(a, ch, R.tb, ft * 32 + (lane & 31), lane, acc1);
        }
        if (!waited) async_wait();                 // no tile for this wave (or a frameless chunk)
    }
}

// ------------------------------------------------------------------ 16-bit row-split kernel, producer/consumer
//
// The same wave layout and multiplies as k_melt_h16_as, with the staging taken off the
// multiply waves' path.  The waves from L.full on (those sharing a row tile, or idle ones)
// are producers: each owns the 256-sample blocks b = pw, pw + np, ... of every chunk's span,
// copies them HBM -> LDS (direct-to-LDS, FP32) and converts exactly those blocks into the
// operand rows, so no producer ever waits for another's copy.  Two operand-row buffers
// alternate: while all waves multiply chunk c from one, the producers fill the other with
// chunk c + 1.  One barrier per chunk.
//
// nscr = 2 span buffers: the copy of chunk c + 2 is issued first thing in the iteration of
// chunk c (into the span converted an iteration earlier) and waited for an iteration later;
// nscr = 1: it is issued after chunk c + 1's conversion.  Needs L.full < waves in every row
// group (checked by the host).
template <class Conv>
__device__ __forceinline__ void convert_owned(const FwdArgs &a, const Chunk &ch, const float *span,
                                              typename Conv::elem_t *rows, int lo_off, int pw, int np) {
    const int lane = threadIdx.x & 63;
    const int sp = (ch.n_frames + a.J - 1) * a.H;
    const int valid = span_valid(a, ch);
    if ((a.H & 3) == 0) {
        // four owned blocks per pass, their LDS reads in flight together; a vector never
        // straddles a row and the span length is a multiple of 4
        for (int b0 = pw; b0 * 256 < sp; b0 += 4 * np) {
            f32x4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int o = (b0 + u * np) * 256 + 4 * lane;
                v[u] = o < valid ? *(const f32x4 *)(span + o) : f32x4{};
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int o = (b0 + u * np) * 256 + 4 * lane;
                if (o < sp) {
                    if (o + 4 > valid) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (o + e >= valid) v[u][e] = 0.0f;
                    }
                    const int r = span_row(a, o);
                    Conv::store4(rows, r * a.S + (o - r * a.H), v[u], lo_off);
                }
            }
        }
        return;
    }
    for (int b = pw; b * 256 < sp; b += np) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int o = b * 256 + 4 * lane + e;
            if (o < sp) {
                const float v = o < valid ? span[o] : 0.0f;
                const int r = span_row(a, o);
                Conv::store(rows, r * a.S + (o - r * a.H), v, lo_off);
            }
        }
    }
}

// Direct-to-LDS copies of the valid span's blocks owned by producer pw of np: 16-byte copies
// over whole blocks, 4-byte copies over the owned last partial block (no lane reads past the
// clip end).  Returns the copy instructions issued (each has an active lane).
__device__ __forceinline__ int copy_owned(const FwdArgs &a, const Chunk &ch, float *span, int pw, int np) {
    const int lane = threadIdx.x & 63;
    const int valid = span_valid(a, ch);
    const float *src = a.wave + ch.sample_start;
    const unsigned base = __builtin_amdgcn_readfirstlane(lds_addr(span));
    const int nfull = valid >> 8;
    int n = 0;
    for (int b = pw; b < nfull; b += np, ++n) lds_dma_x4(src + b * 256 + 4 * lane, base + b * 1024);
    if ((valid & 255) != 0 && nfull % np == pw) {
        for (int q = 4 * nfull; q * 64 < valid; ++q, ++n) {
            const int o = q * 64 + lane;
            if (o < valid) lds_dma_x1(src + o, base + q * 256);
        }
    }
    return n;
}

template <class Conv, int NS, bool X3, bool IS_F16>
__global__ __launch_bounds__(512) void k_melt_h16_pp(FwdArgs a, const uint4 *__restrict__ bhi,
                                                     const uint4 *__restrict__ blo, GroupTableBig gt, int bf,
                                                     int rows_len, int scr_off, int scr_len, int nscr,
                                                     int rgroups) {
    extern __shared__ float lds_pp[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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
    const int lo_off = a.S * (bf + a.J - 1);
    unsigned short *rows0 = reinterpret_cast<unsigned short *>(lds_pp);
    unsigned short *rows1 = rows0 + rows_len;
    float *span0 = lds_pp + scr_off;
    float *span1 = span0 + (nscr == 2 ? scr_len : 0);
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows0, blockDim.x, lo_off);
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows1, blockDim.x, lo_off);
    uint4 A[NS];
    uint4 Al[X3 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) A[s] = bhi[((size_t)rt * NS + s) * 64 + lane];
    if constexpr (X3) {
#pragma unroll
        for (int s = 0; s < NS; ++s) Al[s] = blo[((size_t)rt * NS + s) * 64 + lane];
    }
    const int nw = blockDim.x >> 6;
    const int wu = __builtin_amdgcn_readfirstlane(wid);
    const bool producer = wu >= L.full;
    const int np = nw - L.full, pw = wu - L.full;
    const int nch = *a.n_chunks;
    const int cstep = gridDim.x / rgroups;
    int c = blockIdx.x / rgroups;
    if (producer && c < nch) {
        const Chunk c0 = read_chunk(a.chunks, c);
        copy_owned(a, c0, span0, pw, np);
        wait_vm_younger(0);
        convert_owned<Conv>(a, c0, span0, rows0, lo_off, pw, np);
        if (c + cstep < nch) copy_owned(a, read_chunk(a.chunks, c + cstep), span1, pw, np);
    }
    __syncthreads();
    __shared__ ChunkRing ring;
    for (int it = 0; c < nch; c += cstep, ++it) {
        const int ri = it % kRing;
        if (ri == 0) {
            ring_fill(ring, a.chunks, c, cstep, nch);
            __syncthreads();
        }
        const Chunk ch = ring_get(ring, ri);
        const unsigned short *cur = (it & 1) ? rows1 : rows0;
        unsigned short *nxt = (it & 1) ? rows0 : rows1;
        if (producer && c + cstep < nch) {
            // chunk c + cstep's span: span1 after even iterations; with one span buffer span0
            const float *sn = ((it & 1) == 0) ? span1 : span0;
            const Chunk cn = ring_get(ring, ri + 1);
            const bool more = c + 2 * cstep < nch;
            if (nscr == 2) {
                float *sf = ((it & 1) == 0) ? span0 : span1;       // chunk c's span, converted
                const int n = more ? copy_owned(a, ring_get(ring, ri + 2), sf, pw, np) : 0;
                wait_vm_younger(n);
                convert_owned<Conv>(a, cn, sn, nxt, lo_off, pw, np);
            } else {
                wait_vm_younger(0);
                convert_owned<Conv>(a, cn, sn, nxt, lo_off, pw, np);
                if (more) copy_owned(a, ring_get(ring, ri + 2), span0, pw, np);
            }
        }
        const int nft = idle ? 0 : (ch.n_frames + 31) >> 5;
        const int step = (P == 1 && !X3) ? 2 : P;
        for (int ft = part; ft < nft; ft += step) {
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            int off = (ft * 32 + (lane & 31)) * a.S + 8 * (lane >> 5);
            asm volatile("" : "+v"(off));
            const unsigned short *l0 = cur + off;
            if constexpr (!X3) {
                if (step == 2) {
                    const bool two = ft + 1 < nft;
                    const unsigned short *l1 = two ? l0 + 32 * a.S : l0;
                    mfma_sweep<NS, false, IS_F16>(A, Al, l0, l1, gt, lo_off, acc0, acc1);
                    store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc0);
                    if (two) store_tile(a, ch, rt, (ft + 1) * 32 + (lane & 31), lane, acc1);
                    continue;
                }
            }
            mfma_sweep1<NS, X3, IS_F16>(A, Al, l0, gt, lo_off, acc0);
            store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc0);
        }
        __syncthreads();       // rows `nxt` hold chunk c + cstep; rows `cur` are free
    }
}

// ------------------------------------------------------------------ 16-bit producer/consumer kernel, 12 waves
//
// The arrangement of the block-scaled FP8 producer/consumer kernel (melt_f8.hip) for BF16 and
// FP16: a chunk's conversion and its multiplies on different waves, so that they overlap.  A
// workgroup of 12 waves (three per SIMD): the first NC = (row tiles of the group) are
// consumers, each holding one basis tile in registers (NS k-groups of 16) and sweeping one
// frame tile at a time; the other NP = 12 - NC are producers.  Producer w owns the 256-sample
// blocks w, w + NP, ... of every chunk's span: it copies them HBM -> LDS (direct-to-LDS),
// waits for its own copies only and converts exactly those into the 16-bit hop-block rows of
// the other row buffer, then issues its copies of the chunk after next.  In iteration k the
// consumers multiply chunk k from one buffer while the producers fill the other with chunk
// k + 1; one barrier per chunk.  Chunk descriptors pass through a four-slot LDS ring: the first
// producer loads descriptor k + 3 in iteration k and stores it before the barrier (slot
// (k + 3) mod 4 was last read in iteration k - 1).  The first chunk is copied and converted by
// all twelve waves.
template <class Conv, int NS, bool X3, bool IS_F16>
__global__ __launch_bounds__(X3 ? 512 : 768) void k_melt_h16_pc(FwdArgs a, const uint4 *__restrict__ bhi,
                                                               const uint4 *__restrict__ blo, GroupTableBig gt,
                                                               int bf, int rows_len, int lo_off, int scr_off,
                                                               int rgroups) {
    extern __shared__ float lds_hpc[];
    __shared__ __align__(16) Chunk dslot[4];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
    const int grp = blockIdx.x % rgroups, gt_n = (a.row_tiles + rgroups - 1) / rgroups;
    const int r0 = grp * gt_n, cnt = min(a.row_tiles - r0, gt_n);
    const int nc = cnt, np = nw - cnt;             // consumers (one row tile each), producers
    const bool producer = wid >= nc;
    const int pw = wid - nc;
    unsigned short *rows0 = reinterpret_cast<unsigned short *>(lds_hpc);
    unsigned short *rows1 = rows0 + rows_len;
    float *span = lds_hpc + scr_off;
    const int nch = *a.n_chunks;
    const int cstep = gridDim.x / rgroups;
    const int c0 = blockIdx.x / rgroups;
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows0, blockDim.x, lo_off);
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows1, blockDim.x, lo_off);
    if (wid == nc && lane < 3 && c0 + lane * cstep < nch) dslot[lane] = a.chunks[c0 + lane * cstep];
    // the first chunk is copied and converted by every wave (blocks w, w + nw, ...); after a
    // barrier the producers start the copy of the second
    if (c0 < nch) {
        const Chunk ch = read_chunk(a.chunks, c0);
        copy_owned(a, ch, span, wid, nw);
        async_wait();
        convert_owned<Conv>(a, ch, span, rows0, lo_off, wid, nw);
    }
    __syncthreads();
    if (producer) {
        if (c0 + cstep < nch) copy_owned(a, read_chunk(a.chunks, c0 + cstep), span, pw, np);
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
            const Chunk ch1 = ring_slot(dslot, (it + 1) & 3);
            convert_owned<Conv>(a, ch1, span, ((it + 1) & 1) ? rows1 : rows0, lo_off, pw, np);
            if (load_desc && lane == 0) {
                uint4 *dst = reinterpret_cast<uint4 *>(dslot + ((it + 3) & 3));
                dst[0] = nd0;
                dst[1] = nd1;
            }
            if (c + 2 * cstep < nch) copy_owned(a, ring_slot(dslot, (it + 2) & 3), span, pw, np);
        }
        return;
    }
    const int rt = r0 + wid;
    uint4 A[NS], Al[X3 ? NS : 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) A[s] = bhi[((size_t)rt * NS + s) * 64 + lane];
    if constexpr (X3) {
#pragma unroll
        for (int s = 0; s < NS; ++s) Al[s] = blo[((size_t)rt * NS + s) * 64 + lane];
    } else {
        Al[0] = uint4{};
    }
    for (int it = 0; c0 + it * cstep < nch; ++it) {
        __syncthreads();                           // chunk it converted; buffer (it + 1) & 1 free
        const Chunk ch = ring_slot(dslot, it & 3);
        const unsigned short *rows = (it & 1) ? rows1 : rows0;
        const int nft = (ch.n_frames + 31) >> 5;
        for (int ft = 0; ft < nft; ++ft) {
            int off = (ft * 32 + (lane & 31)) * a.S + 8 * (lane >> 5);
            asm volatile("" : "+v"(off));
            f32x16 acc = f32x16{};
            mfma_sweep1<NS, X3, IS_F16>(A, Al, rows + off, gt, lo_off, acc);
            store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc);
        }
    }
}

// ------------------------------------------------------------------ 16-bit K-split kernel
//
// For frames whose basis tile is too long for one wave's registers (N = 1024: 64 k-groups;
// N = 1200 at hop 160: 75): two waves share each row tile.  The first holds the k-groups of
// the first hop segments (NS0 groups), the second the rest (NS1 <= NS0), whose columns are
// the first half's, `delta` elements (whole hop rows) further down.  Per pair of frame tiles
// the second wave hands its partial sums to the first through LDS, which adds them and
// stores.  A workgroup owns a row group of at most 4 tiles (8 waves); spans are staged as in
// k_melt_h16_as: the second-half waves, which store nothing, issue the span copies and wait
// for them, and chunk descriptors come from the LDS ring.
template <class Conv, int NS0, int NS1, bool IS_F16>
__global__ __launch_bounds__(512) void k_melt_h16_ks(FwdArgs a, const uint4 *__restrict__ bhi, GroupTableBig gt,
                                                     int bf, int scr_off, int red_off, int rgroups, int delta) {
    static_assert(NS1 <= NS0, "the first half is the longer one");
    constexpr int G = NS0 + NS1;
    constexpr int D = NS0 > 32 ? 2 : 4;           // fragment ring depth: registers for NS0 = 40
    extern __shared__ float lds_ks[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int grp = blockIdx.x % rgroups, gt_n = (a.row_tiles + rgroups - 1) / rgroups;
    const int r0 = grp * gt_n, cnt = min(a.row_tiles - r0, gt_n);
    const int kh = wid / gt_n, rl = wid - kh * gt_n;
    const bool idle = rl >= cnt;                   // a smaller last group leaves waves idle
    const int rt = r0 + (idle ? 0 : rl);
    unsigned short *rows = reinterpret_cast<unsigned short *>(lds_ks);
    float *scratch = lds_ks + scr_off;
    float *red = lds_ks + red_off + rl * 2048;     // [2 tiles][16 registers][64 lanes]
    zero_pad_columns<Conv>(a, bf + a.J - 1, rows, blockDim.x, 0);
    uint4 A[NS0];
    const uint4 Al[1] = {};
#pragma unroll
    for (int s = 0; s < NS0; ++s)
        A[s] = (kh == 0 || s < NS1) ? bhi[((size_t)rt * G + kh * NS0 + s) * 64 + lane] : uint4{};
    const int nch = *a.n_chunks;
    const int cstep = gridDim.x / rgroups;
    const int wu = __builtin_amdgcn_readfirstlane(wid);
    const bool copier = wu >= gt_n;                // second-half waves: no output stores
    int c = blockIdx.x / rgroups;
    if (c < nch) async_span(a, read_chunk(a.chunks, c), scratch);
    async_wait();
    __shared__ ChunkRing ring;
    for (int it = 0; c < nch; c += cstep, ++it) {
        const int ri = it % kRing;
        if (ri == 0) ring_fill(ring, a.chunks, c, cstep, nch);
        __syncthreads();                           // span of chunk c is in scratch; rows are free
        const Chunk ch = ring_get(ring, ri);
        const Chunk chn = ring_get(ring, ri + 1);
        convert_span<Conv>(a, ch, scratch, rows, 0);
        __syncthreads();                           // rows ready; scratch is free
        if (copier && c + cstep < nch) async_span_waves(a, chn, scratch, wu - gt_n, gt_n);
        const int nft = (ch.n_frames + 31) >> 5;
        for (int ft = 0; ft < nft; ft += 2) {      // the same trip count in every wave
            const bool two = ft + 1 < nft;
            f32x16 acc0 = f32x16{}, acc1 = f32x16{};
            if (!idle) {
                int off = (ft * 32 + (lane & 31)) * a.S + 8 * (lane >> 5) + kh * delta;
                asm volatile("" : "+v"(off));
                const unsigned short *l0 = rows + off;
                const unsigned short *l1 = two ? l0 + 32 * a.S : l0;
                if constexpr (NS0 == NS1) {
                    mfma_sweep<NS0, false, IS_F16, D>(A, Al, l0, l1, gt, 0, acc0, acc1);
                } else if (kh == 0) {
                    mfma_sweep<NS0, false, IS_F16, D>(A, Al, l0, l1, gt, 0, acc0, acc1);
                } else {
                    mfma_sweep<NS1, false, IS_F16, D>(reinterpret_cast<const uint4(&)[NS1]>(A), Al, l0, l1, gt, 0,
                                                      acc0, acc1);
                }
                if (kh == 1) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        red[r * 64 + lane] = acc0[r];
                        red[1024 + r * 64 + lane] = acc1[r];
                    }
                }
            }
            __syncthreads();                       // partial sums of the second halves in LDS
            if (!idle && kh == 0) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc0[r] += red[r * 64 + lane];
                    acc1[r] += red[1024 + r * 64 + lane];
                }
                store_tile(a, ch, rt, ft * 32 + (lane & 31), lane, acc0);
                if (two) store_tile(a, ch, rt, (ft + 1) * 32 + (lane & 31), lane, acc1);
            }
            __syncthreads();                       // the partial-sum area is free again
        }
        if (copier) async_wait();                  // the next chunk's copy has landed
    }
}

// ------------------------------------------------------------------ 16-bit frame-split kernel
// Fallback for frame lengths whose basis tile does not fit in registers: as the FP32
// frame-split kernel, one 32x32x16 MFMA per k-group, the basis fragments read from L2.
// X3 (split precisions): the frames' low parts are staged at lo_off and the basis low parts
// streamed beside the high ones, hi*hi + lo*hi + hi*lo per k-group.
template <class Conv, int RTB, bool IS_F16, bool X3>
__global__ __launch_bounds__(256, 1) void k_melt_h16_fs(FwdArgs a, const uint4 *__restrict__ bpack,
                                                        const uint4 *__restrict__ blo, GroupTableBig gt) {
    extern __shared__ unsigned short lds16[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nch = *a.n_chunks;
    const int NG = gt.n;
    const int lo_off = X3 ? a.S * (kChunkF32 + a.J - 1) : 0;
    zero_pad_columns<Conv>(a, kChunkF32 + a.J - 1, lds16, 256, lo_off);
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const Chunk ch = read_chunk(a.chunks, c);
        __syncthreads();
        stage_span<Conv, 8>(a, ch, lds16, 256, lo_off);
        __syncthreads();
        const int fbase = wid * 32;
        if (fbase >= ch.n_frames) continue;
        const unsigned short *lp = lds16 + (fbase + (lane & 31)) * a.S + 8 * (lane >> 5);
        for (int rb = 0; rb < a.row_tiles; rb += RTB) {
            f32x16 acc[RTB];
#pragma unroll
            for (int r = 0; r < RTB; ++r) acc[r] = f32x16{};
            const uint4 *bp = bpack + (size_t)rb * NG * 64 + lane;
            const uint4 *bl = blo + (size_t)rb * NG * 64 + lane;
            for (int g = 0; g < NG; ++g) {
                const uint4 b = *(const uint4 *)(lp + gt.lds_off[g]);
                uint4 bx = {};
                if constexpr (X3) bx = *(const uint4 *)(lp + lo_off + gt.lds_off[g]);
#pragma unroll
                for (int r = 0; r < RTB; ++r) {
                    if (rb + r >= a.row_tiles) continue;
                    const uint4 av = bp[((size_t)r * NG + g) * 64];
                    uint4 ax = {};
                    if constexpr (X3) ax = bl[((size_t)r * NG + g) * 64];
                    if constexpr (IS_F16) {
                        const f16x8 ah = __builtin_bit_cast(f16x8, av);
                        acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, __builtin_bit_cast(f16x8, b), acc[r], 0, 0, 0);
                        if constexpr (X3) {
                            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, ax),
                                                                            __builtin_bit_cast(f16x8, b), acc[r], 0, 0, 0);
                            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, __builtin_bit_cast(f16x8, bx), acc[r], 0, 0, 0);
                        }
                    } else {
                        const bf16x8 ah = __builtin_bit_cast(bf16x8, av);
                        acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, __builtin_bit_cast(bf16x8, b), acc[r], 0, 0, 0);
                        if constexpr (X3) {
                            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ax),
                                                                             __builtin_bit_cast(bf16x8, b), acc[r], 0, 0, 0);
                            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, __builtin_bit_cast(bf16x8, bx), acc[r], 0, 0, 0);
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < RTB; ++r)
                if (rb + r < a.row_tiles) store_tile(a, ch, rb + r, fbase + (lane & 31), lane, acc[r]);
        }
    }
}

// ------------------------------------------------------------------ launch

template <class Conv, bool F16, int RTB, bool X3 = false>
static melt_status launch_h16fs_rtb(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid,
                                    hipStream_t s) {
    allow_lds(k_melt_h16_fs<Conv, RTB, F16, X3>);
    k_melt_h16_fs<Conv, RTB, F16, X3><<<grid, 256, lds, s>>>(a, (const uint4 *)p.d_pack_h16,
                                                             (const uint4 *)p.d_pack_lo, gt);
    return hip_check(hipGetLastError(), "melt h16 fs launch");
}

// the split precisions on the frame-split kernel: four row tiles per sweep (the low-part
// loads double the basis traffic)
template <class Conv, bool F16>
static melt_status launch_h16fs_x3(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid,
                                   hipStream_t s) {
    switch (std::min(p.row_tiles, 4)) {
    case 1: return launch_h16fs_rtb<Conv, F16, 1, true>(p, a, gt, lds, grid, s);
    case 2: return launch_h16fs_rtb<Conv, F16, 2, true>(p, a, gt, lds, grid, s);
    default: return launch_h16fs_rtb<Conv, F16, 4, true>(p, a, gt, lds, grid, s);
    }
}

template <class Conv, int NS, bool X3, bool F16>
static melt_status launch_rs_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                hipStream_t s) {
    allow_lds(k_melt_h16_rs<Conv, NS, X3, F16>);
    k_melt_h16_rs<Conv, NS, X3, F16><<<grid, 64 * p.row_tiles, lds, s>>>(
        a, (const uint4 *)p.d_pack_h16, (const uint4 *)p.d_pack_lo, gt, bf);
    return hip_check(hipGetLastError(), "melt h16 rs launch");
}

struct SpanBufs {
    int off, len, n;    // first span (floats into LDS), floats per span, span count (1 or 2)
};

template <class Conv, int NS, bool X3, bool F16>
static melt_status launch_as_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                SpanBufs sb, hipStream_t s) {
    allow_lds(k_melt_h16_as<Conv, NS, X3, F16>, kRingBytes);
    const WaveLayout w = wave_layout(p);
    const int rg = row_groups(p);
    k_melt_h16_as<Conv, NS, X3, F16><<<grid, 64 * w.waves, lds, s>>>(
        a, (const uint4 *)p.d_pack_h16, (const uint4 *)p.d_pack_lo, gt, bf, sb.off, sb.len, sb.n, rg);
    return hip_check(hipGetLastError(), "melt h16 lds-dma launch");
}

template <class Conv, bool X3, bool F16>
static melt_status launch_as(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                             SpanBufs sb, hipStream_t s) {
    switch (p.geo16.n_groups) {
    case 10: return launch_as_ns<Conv, 10, X3, F16>(p, a, gt, lds, grid, bf, sb, s);
    case 16: return launch_as_ns<Conv, 16, X3, F16>(p, a, gt, lds, grid, bf, sb, s);
    case 20: return launch_as_ns<Conv, 20, X3, F16>(p, a, gt, lds, grid, bf, sb, s);
    case 25: return launch_as_ns<Conv, 25, X3, F16>(p, a, gt, lds, grid, bf, sb, s);
    case 32: return launch_as_ns<Conv, 32, X3, F16>(p, a, gt, lds, grid, bf, sb, s);
    default: return set_error(MELT_E_UNSUPPORTED, "no register tile for this frame length");
    }
}

template <class Conv, int NS, bool F16>
static melt_status launch_ap_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                hipStream_t s) {
    allow_lds(k_melt_h16_ap<Conv, NS, F16>, kRingBytes);
    k_melt_h16_ap<Conv, NS, F16><<<grid, 512, lds, s>>>(a, (const uint4 *)p.d_pack_h16, gt, bf,
                                                          (int)(as_scratch_offset(p, bf) / 4));
    return hip_check(hipGetLastError(), "melt h16 row-pair launch");
}

template <class Conv, bool F16>
static melt_status launch_ap(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                             hipStream_t s) {
    switch (p.geo16.n_groups) {
    case 16: return launch_ap_ns<Conv, 16, F16>(p, a, gt, lds, grid, bf, s);
    case 20: return launch_ap_ns<Conv, 20, F16>(p, a, gt, lds, grid, bf, s);
    default: return set_error(MELT_E_UNSUPPORTED, "row-pair kernel: no register tile for this frame length");
    }
}

template <class Conv, int NS, bool X3, bool F16>
static melt_status launch_pp_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                int nscr, hipStream_t s) {
    allow_lds(k_melt_h16_pp<Conv, NS, X3, F16>, kRingBytes);
    const WaveLayout w = wave_layout(p);
    const int rg = row_groups(p);
    const size_t rb = pp_rows_bytes(p, bf);
    k_melt_h16_pp<Conv, NS, X3, F16><<<grid, 64 * w.waves, lds, s>>>(
        a, (const uint4 *)p.d_pack_h16, (const uint4 *)p.d_pack_lo, gt, bf, (int)(rb / 2), (int)(2 * rb / 4),
        (int)(as_span_bytes(p, bf) / 4), nscr, rg);
    return hip_check(hipGetLastError(), "melt h16 producer/consumer launch");
}

template <class Conv, bool X3, bool F16>
static melt_status launch_pp(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                             int nscr, hipStream_t s) {
    switch (p.geo16.n_groups) {
    case 10: return launch_pp_ns<Conv, 10, X3, F16>(p, a, gt, lds, grid, bf, nscr, s);
    case 16: return launch_pp_ns<Conv, 16, X3, F16>(p, a, gt, lds, grid, bf, nscr, s);
    case 20: return launch_pp_ns<Conv, 20, X3, F16>(p, a, gt, lds, grid, bf, nscr, s);
    case 25: return launch_pp_ns<Conv, 25, X3, F16>(p, a, gt, lds, grid, bf, nscr, s);
    case 32: return launch_pp_ns<Conv, 32, X3, F16>(p, a, gt, lds, grid, bf, nscr, s);
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

// The split precisions on the producer/consumer kernel: a consumer holds the hi and lo basis
// tiles (2 NS fragments), so the workgroup has 8 waves (two per SIMD, 256 registers each) and
// row groups of at most 5 tiles (at least 3 producers); each row buffer holds the hi rows then
// the lo rows.
static int pc_x3_row_groups(const Plan &p) { return (p.row_tiles + 4) / 5; }
size_t pc_x3_lds_bytes(const Plan &p, int bf) {
    return 4 * pc_rows_bytes(p, bf) + (size_t)(bf + p.geo16.J - 1) * p.H * 4;
}

template <class Conv, int NS, bool X3, bool F16>
static melt_status launch_pc_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                int rg, hipStream_t s) {
    allow_lds(k_melt_h16_pc<Conv, NS, X3, F16>, (int)(4 * sizeof(Chunk)));
    const int part = (int)(pc_rows_bytes(p, bf) / 2);            // elements of one row image
    const int rows_len = X3 ? 2 * part : part;
    k_melt_h16_pc<Conv, NS, X3, F16><<<grid, X3 ? 512 : 768, lds, s>>>(
        a, (const uint4 *)p.d_pack_h16, (const uint4 *)p.d_pack_lo, gt, bf, rows_len, X3 ? part : 0,
        (int)(2 * rows_len * 2 / 4), rg);
    return hip_check(hipGetLastError(), "melt h16 producer/consumer launch");
}

template <class Conv, bool X3, bool F16>
static melt_status launch_pc(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf, int rg,
                             hipStream_t s) {
    switch (p.geo16.n_groups) {
    case 10: return launch_pc_ns<Conv, 10, X3, F16>(p, a, gt, lds, grid, bf, rg, s);
    case 16: return launch_pc_ns<Conv, 16, X3, F16>(p, a, gt, lds, grid, bf, rg, s);
    case 20: return launch_pc_ns<Conv, 20, X3, F16>(p, a, gt, lds, grid, bf, rg, s);
    case 25: return launch_pc_ns<Conv, 25, X3, F16>(p, a, gt, lds, grid, bf, rg, s);
    default: return set_error(MELT_E_UNSUPPORTED, "producer/consumer kernel: no register tile for this frame length");
    }
}

template <class Conv, int NS0, int NS1, bool F16>
static melt_status launch_ks_ns(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf,
                                int rg, int delta, hipStream_t s) {
    allow_lds(k_melt_h16_ks<Conv, NS0, NS1, F16>, kRingBytes);
    const int gt_n = (p.row_tiles + rg - 1) / rg;
    k_melt_h16_ks<Conv, NS0, NS1, F16><<<grid, 128 * gt_n, lds, s>>>(a, (const uint4 *)p.d_pack_h16, gt, bf,
                                                                     (int)(ks_scratch_offset(p, bf) / 4),
                                                                     (int)(ks_red_offset(p, bf) / 4), rg, delta);
    return hip_check(hipGetLastError(), "melt h16 k-split launch");
}

template <class Conv, bool F16>
static melt_status launch_ks(Plan &p, const FwdArgs &a, const GroupTableBig &gt, size_t lds, int grid, int bf, int rg,
                             const KSplit &k, hipStream_t s) {
    if (k.ns0 == 16 && k.ns1 == 16) return launch_ks_ns<Conv, 16, 16, F16>(p, a, gt, lds, grid, bf, rg, k.delta, s);
    if (k.ns0 == 20 && k.ns1 == 20) return launch_ks_ns<Conv, 20, 20, F16>(p, a, gt, lds, grid, bf, rg, k.delta, s);
    if (k.ns0 == 25 && k.ns1 == 25) return launch_ks_ns<Conv, 25, 25, F16>(p, a, gt, lds, grid, bf, rg, k.delta, s);
    if (k.ns0 == 32 && k.ns1 == 32) return launch_ks_ns<Conv, 32, 32, F16>(p, a, gt, lds, grid, bf, rg, k.delta, s);
    if (k.ns0 == 40 && k.ns1 == 35) return launch_ks_ns<Conv, 40, 35, F16>(p, a, gt, lds, grid, bf, rg, k.delta, s);
    return set_error(MELT_E_UNSUPPORTED, "no K-split register tile for this frame length");
}

melt_status launch_melt_h16(Plan &p, const FwdTask &t, H16Kind kind, int bf, int nbuf) {
    const int prec = p.cfg.precision;
    const Geometry &g = p.geo16;
    const int S = lds_stride(g.Hp, 2);
    const bool f16 = prec_f16(p);
    const bool x3 = prec_split(p);
    if (g.n_groups > 512) return set_error(MELT_E_UNSUPPORTED, "frame too long");
    const FwdArgs a = make_args(p, g, S, t);
    const GroupTableBig gt = make_table(g, S);
    const hipStream_t s = t.stream;
    if (kind == H16_LDS_DMA) {
        if (nbuf != 1 && nbuf != 2) return set_error(MELT_E_INVALID_ARG, "span buffer count must be 1 or 2");
        const size_t lds = as_lds_bytes(p, bf, nbuf);
        if (lds + kRingBytes > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
        const SpanBufs sb{(int)(as_scratch_offset(p, bf) / 4), (int)(as_span_bytes(p, bf) / 4), nbuf};
        // one persistent set of workgroups per row group, each walking all chunks
        const int rg = row_groups(p);
        const int per_cu = std::min(std::max(1, (int)(kMaxLds / (lds + kRingBytes))), 2);
        const int per_group = (int)std::max<int64_t>(1, std::min<int64_t>(t.est_chunks, ((int64_t)p.cu_count * per_cu + rg - 1) / rg));
        const int grid = per_group * rg;
        if (x3 && f16) return launch_as<ConvF16X3, true, true>(p, a, gt, lds, grid, bf, sb, s);
        if (x3) return launch_as<ConvBF16X3, true, false>(p, a, gt, lds, grid, bf, sb, s);
        if (f16) return launch_as<ConvF16, false, true>(p, a, gt, lds, grid, bf, sb, s);
        return launch_as<ConvBF16, false, false>(p, a, gt, lds, grid, bf, sb, s);
    }
    if (kind == H16_ROW_PAIR) {
        if (x3 || !ap_fits(p)) return set_error(MELT_E_UNSUPPORTED, "row-pair kernel: unsupported geometry");
        const size_t lds = as_lds_bytes(p, bf, 1);
        if (lds + kRingBytes > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(t.est_chunks, (int64_t)p.cu_count));
        if (f16) return launch_ap<ConvF16, true>(p, a, gt, lds, grid, bf, s);
        return launch_ap<ConvBF16, false>(p, a, gt, lds, grid, bf, s);
    }
    if (kind == H16_PC12) {
        if (!pc_fits(p)) return set_error(MELT_E_UNSUPPORTED, "producer/consumer kernel: unsupported geometry");
        const size_t lds = x3 ? pc_x3_lds_bytes(p, bf) : pc_lds_bytes(p, bf);
        if (lds + 4 * sizeof(Chunk) > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
        const int rg = x3 ? pc_x3_row_groups(p) : row_groups(p);
        const int per_group = (int)std::max<int64_t>(1, std::min<int64_t>(t.est_chunks, ((int64_t)p.cu_count + rg - 1) / rg));
        const int grid = per_group * rg;
        if (x3 && f16) return launch_pc<ConvF16X3, true, true>(p, a, gt, lds, grid, bf, rg, s);
        if (x3) return launch_pc<ConvBF16X3, true, false>(p, a, gt, lds, grid, bf, rg, s);
        if (f16) return launch_pc<ConvF16, false, true>(p, a, gt, lds, grid, bf, rg, s);
        return launch_pc<ConvBF16, false, false>(p, a, gt, lds, grid, bf, rg, s);
    }
    if (kind == H16_PIPELINED) {
        if (!pp_fits(p)) return set_error(MELT_E_UNSUPPORTED, "producer/consumer kernel: no producer waves");
        if (nbuf != 1 && nbuf != 2) return set_error(MELT_E_INVALID_ARG, "span buffer count must be 1 or 2");
        const size_t lds = pp_lds_bytes(p, bf, nbuf);
        if (lds + kRingBytes > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
        const int rg = row_groups(p);
        const int per_group = (int)std::max<int64_t>(1, std::min<int64_t>(t.est_chunks, ((int64_t)p.cu_count + rg - 1) / rg));
        const int grid = per_group * rg;
        if (x3 && f16) return launch_pp<ConvF16X3, true, true>(p, a, gt, lds, grid, bf, nbuf, s);
        if (x3) return launch_pp<ConvBF16X3, true, false>(p, a, gt, lds, grid, bf, nbuf, s);
        if (f16) return launch_pp<ConvF16, false, true>(p, a, gt, lds, grid, bf, nbuf, s);
        return launch_pp<ConvBF16, false, false>(p, a, gt, lds, grid, bf, nbuf, s);
    }
    if (kind == H16_K_SPLIT) {
        if (x3 || !ks_fits(p)) return set_error(MELT_E_UNSUPPORTED, "K-split kernel: unsupported geometry");
        const size_t lds = ks_lds_bytes(p, bf);
        if (lds + kRingBytes > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
        const int rg = ks_row_groups(p);
        const int per_group = (int)std::max<int64_t>(1, std::min<int64_t>(t.est_chunks, ((int64_t)p.cu_count + rg - 1) / rg));
        const int grid = per_group * rg;
        const KSplit k = ks_split(p, S);
        if (f16) return launch_ks<ConvF16, true>(p, a, gt, lds, grid, bf, rg, k, s);
        return launch_ks<ConvBF16, false>(p, a, gt, lds, grid, bf, rg, k, s);
    }
    if (kind == H16_REGISTER_STAGED) {
        const size_t lds = (size_t)(bf + g.J - 1) * S * 2 * (x3 ? 2 : 1);
        if (lds > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
        const int grid = persistent_grid(p, t.est_chunks, std::min(std::max(1, (int)(kMaxLds / lds)), 2));
        if (x3 && f16) return launch_rs<ConvF16X3, true, true>(p, a, gt, lds, grid, bf, s);
        if (x3) return launch_rs<ConvBF16X3, true, false>(p, a, gt, lds, grid, bf, s);
        if (f16) return launch_rs<ConvF16, false, true>(p, a, gt, lds, grid, bf, s);
        return launch_rs<ConvBF16, false, false>(p, a, gt, lds, grid, bf, s);
    }
    const size_t lds = (size_t)(kBF32 + g.J - 1) * S * 2 * (x3 ? 2 : 1);
    if (lds > (size_t)kMaxLds) return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS");
    const int grid = persistent_grid(p, t.est_chunks, 2);
    if (x3) return f16 ? launch_h16fs_x3<ConvF16X3, true>(p, a, gt, lds, grid, s)
                       : launch_h16fs_x3<ConvBF16X3, false>(p, a, gt, lds, grid, s);
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

}  // namespace melt
