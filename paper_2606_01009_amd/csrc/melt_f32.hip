// MelT forward, FP32 operands: v_mfma_f32_32x32x2f32 over a frame-split chunk with the basis
// streamed from L2 (Eq. dmp_projection, Eq. dmp_matrix_energy, Eq. meltf).
#include "fwd_common.h"

namespace melt {

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
        span_load<PRE, 256>(a, nxt, pf, tid);
    }
    for (; c < nch; c += gridDim.x) {
        const Chunk ch = nxt;
        __syncthreads();
        span_store<ConvF32, PRE, 256>(a, ch, pf, lds, 0, tid);
        __syncthreads();
        const bool more = c + (int)gridDim.x < nch;
        if (more) nxt = read_chunk(a.chunks, c + gridDim.x);
        const int fbase = wid * 32;
        if (fbase >= ch.n_frames) {
            if (more) span_load<PRE, 256>(a, nxt, pf, tid);
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
            if (more && rb + RTB >= a.row_tiles) span_load<PRE, 256>(a, nxt, pf, tid);
#pragma unroll
            for (int r = 0; r < RTB; ++r)
                if (rb + r < a.row_tiles) store_tile(a, ch, rb + r, fbase + (lane & 31), lane, acc[r]);
        }
    }
}

// ------------------------------------------------------------------ FP32 warp-specialised kernel
//
// 8 waves, 2 per SIMD: waves 0-3 multiply exactly as k_melt_f32_fs (32 frames each, basis
// streamed from L2), waves 4-7 only stage.  The stagers hold the next chunk's span in
// their own registers, loaded a whole chunk ahead, so the multiply waves' waits for basis
// fragments never include sample loads (the wait counter drains in order).  Per chunk:
// barrier A after the MFMA loop (the rows are free), then the stagers write the next rows
// while the multiply waves empty their accumulators, then barrier B.  The two roles run
// separate loops with the same barriers, so their registers are allocated independently.
//
// HANDOFF: the multiply waves only write the energies R^2 + I^2 of the last row-tile block
// into an LDS buffer (frame-major, row stride hs floats) between A and B; after B the
// stagers map them to the output kind and store whole output rows, coalesced, while the
// multiply waves already run the next chunk's MFMAs.  The stagers finish reading before
// the next barrier A, after which the buffer is written again.  Without it (LDS too small)
// the multiply waves store their tiles themselves.
// Mel bins [m0, m1) of the chunk's frames (m0: first bin of the last row-tile block, a
// multiple of 16; the earlier blocks were stored by the multiply waves themselves).
template <int KIND>
__device__ __forceinline__ void handoff_rows(const FwdArgs &a, const Chunk &ch, const float *hb, int hs, int m0,
                                             int m1, int lt) {
    // thread lt takes 4-Mel groups lt, lt + 256, ...: frame f = idx / Q, group q = idx % Q,
    // advanced incrementally
    const int Q = (m1 - m0 + 3) >> 2, total = ch.n_frames * Q;
    const int df = 256 / Q, dq = 256 - df * Q;
    int f = lt / Q, q = lt - f * Q;
    for (int idx = lt; idx < total; idx += 256) {
        const int m = m0 + 4 * q;
        const f32x4 e = *(const f32x4 *)(hb + f * hs + m);
        const int64_t row = ch.out_row + f;
        if (row < a.n_frames) {
            float *o = a.out + row * a.M + m;
            const f32x4 v{out_map_k<KIND>(e[0], a.eps), out_map_k<KIND>(e[1], a.eps), out_map_k<KIND>(e[2], a.eps),
                          out_map_k<KIND>(e[3], a.eps)};
            if ((a.M & 3) == 0 && m + 4 <= m1) {
                *(f32x4 *)o = v;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (m + k < m1) o[k] = v[k];
            }
        }
        f += df;
        q += dq;
        if (q >= Q) {
            q -= Q;
            ++f;
        }
    }
}

// energies of one 32x32 accumulator tile into the handoff buffer (8 Mel bins per lane)
__device__ __forceinline__ void handoff_tile(float *hb, int hs, int f_local, int rt, int lane, const f32x16 &acc) {
    const int mel0 = rt * 16 + 8 * (lane >> 5);
    f32x4 e0, e1;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        e0[2 * g] = acc[4 * g] * acc[4 * g] + acc[4 * g + 1] * acc[4 * g + 1];
        e0[2 * g + 1] = acc[4 * g + 2] * acc[4 * g + 2] + acc[4 * g + 3] * acc[4 * g + 3];
        e1[2 * g] = acc[8 + 4 * g] * acc[8 + 4 * g] + acc[9 + 4 * g] * acc[9 + 4 * g];
        e1[2 * g + 1] = acc[10 + 4 * g] * acc[10 + 4 * g] + acc[11 + 4 * g] * acc[11 + 4 * g];
    }
    *(f32x4 *)(hb + f_local * hs + mel0) = e0;
    *(f32x4 *)(hb + f_local * hs + mel0 + 4) = e1;
}

// the raw (R, I) projection of one tile, when requested
__device__ __forceinline__ void store_proj(const FwdArgs &a, const Chunk &ch, int rt, int f_local, int lane,
                                           const f32x16 &acc) {
    if (!a.proj || f_local >= ch.n_frames) return;
    const int64_t row = ch.out_row + f_local;
    const int mel0 = rt * 16 + 8 * (lane >> 5);
    if (row >= a.n_frames || mel0 >= a.M) return;
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

// Work items: the persistent grid walks items w = chunk * rsplit + part; part p of a chunk
// covers row tiles [p rps, min((p + 1) rps, row_tiles)).  rsplit > 1 spreads a batch with
// fewer chunks than compute units over more workgroups (each stages its chunk itself).
struct WorkItem {
    int c, r_lo, r_hi;
};
__device__ __forceinline__ WorkItem work_item(const FwdArgs &a, int w, int rsplit, int rps) {
    const int c = w / rsplit, part = w - c * rsplit;
    const int r_lo = part * rps;
    return {c, r_lo, min(r_lo + rps, a.row_tiles)};
}

// stager waves' epilogue for one work item (HANDOFF): Mel bins of its last row-tile block
template <int RTB>
__device__ __forceinline__ void stager_epilogue(const FwdArgs &a, const WorkItem &it, const float *hb, int hs,
                                                int lt) {
    const Chunk ch = read_chunk(a.chunks, it.c);
    const int m0 = (it.r_lo + ((it.r_hi - it.r_lo - 1) / RTB) * RTB) * 16;
    const int m1 = min(it.r_hi * 16, a.M);
    switch (a.out_kind) {
    case MELT_OUT_LOG_POWER: handoff_rows<MELT_OUT_LOG_POWER>(a, ch, hb, hs, m0, m1, lt); break;
    case MELT_OUT_LOG_MAGNITUDE: handoff_rows<MELT_OUT_LOG_MAGNITUDE>(a, ch, hb, hs, m0, m1, lt); break;
    case MELT_OUT_POWER: handoff_rows<MELT_OUT_POWER>(a, ch, hb, hs, m0, m1, lt); break;
    default: handoff_rows<MELT_OUT_MAGNITUDE>(a, ch, hb, hs, m0, m1, lt); break;
    }
}

// The stager role with 16-byte vectors (H a multiple of 4); same barriers as the scalar
// loop in k_melt_f32_ws.
template <int RTB, int PV, bool HANDOFF>
__device__ __forceinline__ void stage_rows_vec(const FwdArgs &a, const float *hb, int hs, float *lds, int lt, int w,
                                               int nwork, int rsplit, int rps) {
    f32x4 pv[PV];
    const int G = gridDim.x;
    if (w < nwork) {
        const Chunk ch = read_chunk(a.chunks, w / rsplit);
        span_load4<PV, 256>(a, ch, pv, lt);
        span_store4<PV, 256>(a, ch, pv, lds, lt);
    }
    __syncthreads();                               // rows of the first item ready
    if (w + G < nwork) span_load4<PV, 256>(a, read_chunk(a.chunks, (w + G) / rsplit), pv, lt);
    for (; w < nwork; w += G) {
        __syncthreads();                           // A: the multiply waves are done with the rows
        const int wn = w + G;
        if (wn < nwork) span_store4<PV, 256>(a, read_chunk(a.chunks, wn / rsplit), pv, lds, lt);
        __syncthreads();                           // B: rows of the next item ready; energies of item w in hb
        if constexpr (HANDOFF) stager_epilogue<RTB>(a, work_item(a, w, rsplit, rps), hb, hs, lt);
        if (wn + G < nwork) span_load4<PV, 256>(a, read_chunk(a.chunks, (wn + G) / rsplit), pv, lt);
    }
}

template <int RTB, int PRE, bool HANDOFF>
__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
void k_melt_f32_ws(FwdArgs a, const f32x4 *__restrict__ bpack, int NG, int hb_off, int hs, int rsplit) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwork = *a.n_chunks * rsplit;
    const int rps = (a.row_tiles + rsplit - 1) / rsplit;     // row tiles per work item
    float *hb = lds + hb_off;                      // handoff buffer (HANDOFF only)
    zero_pad_columns<ConvF32>(a, kChunkF32 + a.J - 1, lds, 512, 0);
    int w = blockIdx.x;
    const int G = gridDim.x;
    if (wid >= 4) {
        const int lt = (int)threadIdx.x - 256;
        if ((a.H & 3) == 0) {
            stage_rows_vec<RTB, PRE / 4, HANDOFF>(a, hb, hs, lds, lt, w, nwork, rsplit, rps);
            return;
        }
        float pf[PRE];
        if (w < nwork) {
            const Chunk ch = read_chunk(a.chunks, w / rsplit);
            span_load<PRE, 256>(a, ch, pf, lt);
            span_store<ConvF32, PRE, 256>(a, ch, pf, lds, 0, lt);
        }
        __syncthreads();                           // rows of the first item ready
        if (w + G < nwork) span_load<PRE, 256>(a, read_chunk(a.chunks, (w + G) / rsplit), pf, lt);
        for (; w < nwork; w += G) {
            __syncthreads();                       // A: the multiply waves are done with the rows
            const int wn = w + G;
            if (wn < nwork) span_store<ConvF32, PRE, 256>(a, read_chunk(a.chunks, wn / rsplit), pf, lds, 0, lt);
            __syncthreads();                       // B: rows of the next item ready; energies of item w in hb
            if constexpr (HANDOFF) stager_epilogue<RTB>(a, work_item(a, w, rsplit, rps), hb, hs, lt);
            if (wn + G < nwork) span_load<PRE, 256>(a, read_chunk(a.chunks, (wn + G) / rsplit), pf, lt);
        }
        return;
    }
    const int GH = a.Hp / 8;     // k-groups per full hop segment
    const __amdgpu_buffer_rsrc_t brs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)bpack, (short)0, a.row_tiles * NG * 64 * 16, 0x00020000);
    __syncthreads();
    for (; w < nwork; w += G) {
        const WorkItem it = work_item(a, w, rsplit, rps);
        const Chunk ch = read_chunk(a.chunks, it.c);
        const int fbase = wid * 32;
        const bool active = fbase < ch.n_frames;
        const float *lp = lds + (fbase + (lane & 31)) * a.S + 4 * (lane >> 5);
        for (int rb = it.r_lo; rb < it.r_hi; rb += RTB) {
            const bool last = rb + RTB >= it.r_hi;
            f32x16 acc[RTB];
#pragma unroll
            for (int r = 0; r < RTB; ++r) acc[r] = f32x16{};
            if (active) {
                int voff[RTB];
#pragma unroll
                for (int r = 0; r < RTB; ++r) voff[r] = ((min(rb + r, it.r_hi - 1) * NG) * 64 + lane) * 16;
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
                // ping-pong as in k_melt_f32_fs
                f32x4 A0[RTB], A1[RTB], B0, B1;
                load(A0, B0, 0);
                for (int g = 0; g < NG; g += 2) {
                    load(A1, B1, min(g + 1, NG - 1));
                    __builtin_amdgcn_sched_barrier(0);
                    mma(A0, B0);
                    __builtin_amdgcn_sched_barrier(0);
                    load(A0, B0, min(g + 2, NG - 1));
                    __builtin_amdgcn_sched_barrier(0);
                    const float keep = (g + 1 < NG) ? 1.0f : 0.0f;
                    B1 *= keep;
                    mma(A1, B1);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (last) __syncthreads();             // A: every row read; the stagers may overwrite
            if (active) {
#pragma unroll
                for (int r = 0; r < RTB; ++r) {
                    if (rb + r >= it.r_hi) continue;
                    if (HANDOFF && last) {
                        handoff_tile(hb, hs, fbase + (lane & 31), rb + r, lane, acc[r]);
                        store_proj(a, ch, rb + r, fbase + (lane & 31), lane, acc[r]);
                    } else {
                        store_tile(a, ch, rb + r, fbase + (lane & 31), lane, acc[r]);
                    }
                }
            }
        }
        __syncthreads();                           // B: rows of the next item ready
    }
}

// ------------------------------------------------------------------ launch

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

template <int RTB, int PRE>
static melt_status launch_f32_ws_pre(const FwdArgs &a, const f32x4 *bp, int NG, size_t lds, int grid, int rsplit,
                                     hipStream_t s) {
    // handoff buffer after the rows: 128 frames x hs floats, hs = 16 row tiles + 4 (an odd
    // number of 16-byte groups, so the 32 frames a wave writes spread over the banks)
    const int hs = a.row_tiles * 16 + 4;
    const size_t hb_off = (lds + 15) & ~size_t(15);
    const size_t with = hb_off + (size_t)kBF32 * hs * 4;
    if (with <= (size_t)kMaxLds) {
        allow_lds(k_melt_f32_ws<RTB, PRE, true>);
        k_melt_f32_ws<RTB, PRE, true><<<grid, 512, with, s>>>(a, bp, NG, (int)(hb_off / 4), hs, rsplit);
    } else {
        allow_lds(k_melt_f32_ws<RTB, PRE, false>);
        k_melt_f32_ws<RTB, PRE, false><<<grid, 512, lds, s>>>(a, bp, NG, 0, 0, rsplit);
    }
    return hip_check(hipGetLastError(), "melt f32 ws launch");
}

template <int RTB>
static melt_status launch_f32_ws_rtb(Plan &p, const FwdArgs &a, int NG, size_t lds, int grid, int rsplit,
                                     hipStream_t s) {
    const f32x4 *bp = (const f32x4 *)p.d_pack_f32;
    const int need = ((kBF32 + a.J - 1) * a.H + 255) / 256;
    if (need <= 48) return launch_f32_ws_pre<RTB, 48>(a, bp, NG, lds, grid, rsplit, s);
    if (need <= 88) return launch_f32_ws_pre<RTB, 88>(a, bp, NG, lds, grid, rsplit, s);
    if (need <= 136) return launch_f32_ws_pre<RTB, 136>(a, bp, NG, lds, grid, rsplit, s);
    return set_error(MELT_E_UNSUPPORTED, "hop too large for the FP32 staging waves");
}

melt_status launch_melt_f32(Plan &p, const FwdTask &t, bool warp_specialised) {
    const Geometry &g = p.geo32;
    const int S = lds_stride(g.Hp, 4);
    const size_t lds = (size_t)(kBF32 + g.J - 1) * S * 4;
    if (lds > (size_t)kMaxLds || g.n_groups > 512)
        return set_error(MELT_E_UNSUPPORTED, "frame geometry exceeds LDS for FP32 kernel");
    const FwdArgs a = make_args(p, g, S, t);
    const GroupTableBig gt = make_table(g, S);
    const int grid = persistent_grid(p, t.est_chunks, 1);
    const hipStream_t s = t.stream;
    if (warp_specialised) {
        // A batch with fewer chunks than compute units splits each chunk's row tiles over
        // rsplit workgroups (work items), so a short call still spreads over the machine;
        // otherwise one workgroup takes a whole chunk.
        int rsplit = 1;
        if (t.est_chunks < p.cu_count && p.row_tiles > 1) {
            rsplit = (int)std::min<int64_t>(p.row_tiles, (p.cu_count + t.est_chunks - 1) / std::max<int64_t>(t.est_chunks, 1));
            rsplit = (p.row_tiles + (p.row_tiles + rsplit - 1) / rsplit - 1) / ((p.row_tiles + rsplit - 1) / rsplit);
        }
        const int rps = (p.row_tiles + rsplit - 1) / rsplit;
        const int g2 = persistent_grid(p, t.est_chunks * rsplit, 1);
        // row tiles per block at most 5: accumulators and the basis ping-pong within the
        // 256 registers of two waves per SIMD
        const int blocks = (rps + 4) / 5;
        switch ((rps + blocks - 1) / blocks) {
        case 1: return launch_f32_ws_rtb<1>(p, a, gt.n, lds, g2, rsplit, s);
        case 2: return launch_f32_ws_rtb<2>(p, a, gt.n, lds, g2, rsplit, s);
        case 3: return launch_f32_ws_rtb<3>(p, a, gt.n, lds, g2, rsplit, s);
        case 4: return launch_f32_ws_rtb<4>(p, a, gt.n, lds, g2, rsplit, s);
        default: return launch_f32_ws_rtb<5>(p, a, gt.n, lds, g2, rsplit, s);
        }
    }
    // row tiles per block at most 5 (2 for the deepest prefetch) so accumulators, basis
    // prefetch and sample prefetch fit 512 registers
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

}  // namespace melt
