// Streaming MelT (many live audio streams, fixed-size pushes) and the autotuner.
//
// A stream holds the samples that no complete frame has used yet (fewer than n_fft).  A
// push of chunk_len samples per stream (len = carry + chunk_len samples, k = floor((len -
// N) / H) + 1 complete frames):
//   1. k_stream_pack (one workgroup): k per stream, the packed row offset of each stream
//      (prefix sums of k + J - 1 over streams with k > 0, J = ceil(N / H)) and the chunk
//      table of the packed clip
//   2. k_stream_copy: per stream, the k + J - 1 hop rows its frames read, taken from
//      [carry | chunk] (samples past the stream's end zeroed), into the packed buffer; and
//      the unconsumed tail [k H, len) into a staging slot.  Viewed as one clip, the packed
//      buffer's frame poff_s + t is stream s's frame t (the J - 1 frames that straddle two
//      streams are computed and discarded), so the streams' frames share MFMA tiles
//   3. the MelT main kernel over that clip (same kernels as melt_forward), into a
//      frame-major scratch
//   4. k_stream_finish: per stream, its k frames to its output slot, and the tail becomes
//      the new carry
// Frames are therefore identical to melt_forward over the concatenated stream.  No host
// synchronisation or allocation happens in a push, so it can be captured in a hipGraph.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>

#include "melt_internal.h"

struct melt_stream_s {
    melt::Plan *plan;
    int n_streams, max_chunk, max_frames, bf, variant;
    int64_t max_pack;           // frames of the packed clip at most: n_streams (max_frames + J - 1)
    int max_tab;                // chunks of the packed clip at most
    float *d_carry;             // [n_streams][N]
    int *d_carry_len;           // [n_streams]
    float *d_tail;              // [n_streams][N] unconsumed tail of the push (next carry)
    float *d_pack;              // [(max_pack + J - 1) H + pad] packed hop rows
    float *d_tmp;               // [max_pack][n_mels] outputs of the packed clip
    int64_t *d_poff;            // [n_streams] first packed frame of each stream
    melt::Chunk *d_tab;         // [max_tab]
    int *d_ntab;
    float *d_lmel;              // [n_streams * max_frames][n_mels] log-Mel rows (MELT_OUT_MFCC only)
};

namespace melt {

// one workgroup: frames per stream, packed row offsets (prefix sums of k + J - 1 over the
// streams with k > 0) and the chunk table of the packed clip
__global__ __launch_bounds__(1024) void k_stream_pack(const int *__restrict__ carry_len, int chunk_len, int n_streams,
                                                      int N, int J, int H, int bf, int *__restrict__ emitted,
                                                      int64_t *__restrict__ poff, Chunk *__restrict__ tab, int max_tab,
                                                      int *__restrict__ ntab) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0;
    for (int base = 0; base < n_streams; base += 1024) {
        const int st = base + tid;
        int k = 0;
        if (st < n_streams) {
            const int total = carry_len[st] + chunk_len;
            k = total >= N ? 1 + (total - N) / H : 0;
            emitted[st] = k;
        }
        int64_t v = k > 0 ? k + J - 1 : 0, incl = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t u = __shfl_up(incl, d, 64);
            if (lane >= d) incl += u;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int64_t before = carry;
        for (int q = 0; q < w; ++q) before += wsum[q];
        if (st < n_streams) poff[st] = before + incl - v;
        __syncthreads();
        if (tid == 1023) carry = before + incl;
        __syncthreads();
    }
    const int64_t rows = carry;
    const int64_t P = rows >= J ? rows - J + 1 : 0;      // frames of the packed clip
    const int nt = (int)min<int64_t>((P + bf - 1) / bf, (int64_t)max_tab);
    for (int j = tid; j < nt; j += 1024) {
        Chunk e;
        e.sample_start = (int64_t)j * bf * H;
        e.sample_end = rows * H;
        e.out_row = (int64_t)j * bf;
        e.n_frames = (int)min<int64_t>(bf, P - (int64_t)j * bf);
        e.clip = 0;
        tab[j] = e;
    }
    if (tid == 0) *ntab = nt;
}

// per stream: the hop rows of its frames from [carry | chunk] into the packed buffer (past
// the stream's end: zero, since those samples meet only zero basis weights or discarded
// frames and must be finite), and the tail [k H, len) into its staging slot
__global__ __launch_bounds__(256) void k_stream_copy(const float *__restrict__ chunk, int chunk_len,
                                                     const float *__restrict__ carry, const int *__restrict__ carry_len,
                                                     const int *__restrict__ emitted, const int64_t *__restrict__ poff,
                                                     int N, int J, int H, float *__restrict__ pack,
                                                     float *__restrict__ tail) {
    const int s = blockIdx.x;
    const int k = emitted[s];
    const int len0 = carry_len[s], total = len0 + chunk_len;
    const float *cs = carry + (size_t)s * N;
    const float *xs = chunk + (size_t)s * chunk_len;
    auto sample = [&](int i) { return i < len0 ? cs[i] : xs[i - len0]; };
    if (k > 0) {
        const int n = (k + J - 1) * H;
        float *dst = pack + poff[s] * H;
        for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = i < total ? sample(i) : 0.0f;
    }
    const int from = k * H;
    for (int i = threadIdx.x; i < total - from; i += blockDim.x) tail[(size_t)s * N + i] = sample(from + i);
}

// per stream: its k frames of the packed clip's outputs (width W) to its output slot, and
// the staged tail becomes the carry
__global__ __launch_bounds__(256) void k_stream_finish(const float *__restrict__ tmp, const int *__restrict__ emitted,
                                                       const int64_t *__restrict__ poff, int W, int max_frames,
                                                       float *__restrict__ out, int chunk_len, int N, int H,
                                                       const float *__restrict__ tail, float *__restrict__ carry,
                                                       int *__restrict__ carry_len) {
    const int s = blockIdx.x;
    const int k = emitted[s];
    const float *src = tmp + poff[s] * W;
    float *dst = out + (size_t)s * max_frames * W;
    for (int i = threadIdx.x; i < k * W; i += blockDim.x) dst[i] = src[i];
    const int rem = carry_len[s] + chunk_len - k * H;
    for (int i = threadIdx.x; i < rem; i += blockDim.x) carry[(size_t)s * N + i] = tail[(size_t)s * N + i];
    __syncthreads();   // every thread has read carry_len before it is replaced
    if (threadIdx.x == 0) carry_len[s] = rem;
}

__global__ void k_fill_int(int *__restrict__ p, int n, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------------ autotune cache

namespace {

std::string tune_key(const Plan &p) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p.device) == hipSuccess) arch = prop.gcnArchName;
    std::ostringstream k;
    k << "prec=" << p.cfg.precision << ",n_fft=" << p.N << ",hop=" << p.H << ",n_mels=" << p.M << ",arch=" << arch;
    return k.str();
}

// one entry per line: {"key": "...", "variant": v, "grid": g, "us": t}
bool cache_lookup(const std::string &path, const std::string &key, int &variant, int &grid) {
    std::ifstream f(path);
    std::string line;
    const std::string needle = "\"key\": \"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(needle) == std::string::npos) continue;
        const size_t v = line.find("\"variant\": "), g = line.find("\"grid\": ");
        if (v == std::string::npos || g == std::string::npos) continue;
        variant = std::atoi(line.c_str() + v + 11);
        grid = std::atoi(line.c_str() + g + 8);
        return true;
    }
    return false;
}

void cache_store(const std::string &path, const std::string &key, int variant, int grid, double us) {
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        const std::string needle = "\"key\": \"" + key + "\"";
        while (std::getline(f, line))
            if (!line.empty() && line.find(needle) == std::string::npos) keep.push_back(line);
    }
    std::ostringstream e;
    e << "{\"key\": \"" << key << "\", \"variant\": " << variant << ", \"grid\": " << grid << ", \"us\": " << us << "}";
    keep.push_back(e.str());
    std::ofstream o(path, std::ios::trunc);
    for (const auto &l : keep) o << l << "\n";
}

}  // namespace

void apply_tune_cache(Plan &p) {
    const char *path = std::getenv("MELT_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    int v = 0, g = 0;
    if (cache_lookup(path, tune_key(p), v, g)) {
        if (v >= 0 && v < forward_variants(p)) {
            p.tune_variant = v;
        }
        if (g >= 0 && g <= 4) p.tune_grid = g;
    }
}

}  // namespace melt

using namespace melt;

extern "C" {

melt_status melt_stream_create(melt_plan plan, int32_t n_streams, int32_t max_chunk_len, melt_stream_state *out) {
    if (!plan || !out || n_streams < 1 || max_chunk_len < 1 || max_chunk_len > (1 << 20))
        return set_error(MELT_E_INVALID_ARG, "bad streaming arguments");
    *out = nullptr;
    Plan *p = reinterpret_cast<Plan *>(plan);
    melt_status st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    melt_stream_s *S = new (std::nothrow) melt_stream_s();
    if (!S) return set_error(MELT_E_NO_MEMORY, "stream state");
    S->plan = p;
    S->n_streams = n_streams;
    S->max_chunk = max_chunk_len;
    S->max_frames = (max_chunk_len - 1) / p->H + 1;
    S->variant = p->tune_variant;     // kept for the life of the state
    S->bf = melt_chunk_frames(*p, S->variant);
    const int J = (p->N + p->H - 1) / p->H;
    S->max_pack = (int64_t)n_streams * (S->max_frames + J - 1);
    S->max_tab = (int)((S->max_pack + S->bf - 1) / S->bf);
    // packed buffer: the rows of every stream, plus the span a chunk's staging may read past
    // the last frame (J - 1 rows) and a vector of slack
    const size_t pack_len = (size_t)(S->max_pack + J) * p->H + 64;
    bool ok = hipMalloc(&S->d_carry, sizeof(float) * (size_t)n_streams * p->N) == hipSuccess;
    ok = ok && hipMalloc(&S->d_carry_len, sizeof(int) * n_streams) == hipSuccess;
    ok = ok && hipMalloc(&S->d_tail, sizeof(float) * (size_t)n_streams * p->N) == hipSuccess;
    ok = ok && hipMalloc(&S->d_pack, sizeof(float) * pack_len) == hipSuccess;
    ok = ok && hipMalloc(&S->d_tmp, sizeof(float) * (size_t)S->max_pack * p->M) == hipSuccess;
    ok = ok && hipMalloc(&S->d_poff, sizeof(int64_t) * n_streams) == hipSuccess;
    ok = ok && hipMalloc(&S->d_tab, sizeof(Chunk) * (size_t)S->max_tab) == hipSuccess;
    ok = ok && hipMalloc(&S->d_ntab, sizeof(int)) == hipSuccess;
    if (ok) ok = hipMemset(S->d_pack, 0, sizeof(float) * pack_len) == hipSuccess;
    S->d_lmel = nullptr;
    if (ok && p->K > 0) {
        const size_t bytes = sizeof(float) * (size_t)n_streams * S->max_frames * p->M;
        ok = hipMalloc(&S->d_lmel, bytes) == hipSuccess && hipMemset(S->d_lmel, 0, bytes) == hipSuccess;
    }
    if (!ok) {
        melt_stream_destroy(S);
        return set_error(MELT_E_NO_MEMORY, "stream buffers");
    }
    k_fill_int<<<(n_streams + 255) / 256, 256>>>(S->d_carry_len, n_streams, 0);
    st = hip_check(hipDeviceSynchronize(), "stream init");
    if (st != MELT_OK) {
        melt_stream_destroy(S);
        return st;
    }
    *out = S;
    return MELT_OK;
}

melt_status melt_stream_destroy(melt_stream_state S) {
    if (!S) return MELT_OK;
    (void)hipSetDevice(S->plan->device);
    (void)hipDeviceSynchronize();
    void *b[] = {S->d_carry, S->d_carry_len, S->d_tail, S->d_pack, S->d_tmp, S->d_poff, S->d_tab, S->d_ntab, S->d_lmel};
    for (void *x : b)
        if (x) (void)hipFree(x);
    delete S;
    return MELT_OK;
}

melt_status melt_stream_reset(melt_stream_state S, void *stream) {
    if (!S) return set_error(MELT_E_INVALID_ARG, "state is NULL");
    k_fill_int<<<(S->n_streams + 255) / 256, 256, 0, (hipStream_t)stream>>>(S->d_carry_len, S->n_streams, 0);
    return hip_check(hipGetLastError(), "stream reset");
}

int32_t melt_stream_max_frames(melt_stream_state S) { return S ? S->max_frames : 0; }

melt_status melt_stream_push(melt_stream_state S, const float *d_chunk, int32_t chunk_len, float *d_out,
                             int32_t *d_frames_emitted, void *stream) {
    if (!S || !d_chunk || !d_out || !d_frames_emitted) return set_error(MELT_E_INVALID_ARG, "NULL argument");
    if (chunk_len < 1 || chunk_len > S->max_chunk) return set_error(MELT_E_INVALID_ARG, "chunk_len out of range");
    Plan &p = *S->plan;
    hipStream_t s = (hipStream_t)stream;
    melt_status st = hip_check(hipSetDevice(p.device), "hipSetDevice");
    if (st != MELT_OK) return st;
    const int J = (p.N + p.H - 1) / p.H;
    k_stream_pack<<<1, 1024, 0, s>>>(S->d_carry_len, chunk_len, S->n_streams, p.N, J, p.H, S->bf, d_frames_emitted,
                                     S->d_poff, S->d_tab, S->max_tab, S->d_ntab);
    k_stream_copy<<<S->n_streams, 256, 0, s>>>(d_chunk, chunk_len, S->d_carry, S->d_carry_len, d_frames_emitted,
                                               S->d_poff, p.N, J, p.H, S->d_pack, S->d_tail);
    st = hip_check(hipGetLastError(), "stream pack");
    if (st != MELT_OK) return st;
    st = launch_melt_table(p, S->variant, S->d_tab, S->d_ntab, S->max_tab, S->max_pack, S->d_pack, S->d_tmp, nullptr, s);
    if (st != MELT_OK) return st;
    k_stream_finish<<<S->n_streams, 256, 0, s>>>(S->d_tmp, d_frames_emitted, S->d_poff, p.M, S->max_frames,
                                                 p.K > 0 ? S->d_lmel : d_out, chunk_len, p.N, p.H, S->d_tail,
                                                 S->d_carry, S->d_carry_len);
    st = hip_check(hipGetLastError(), "stream finish");
    if (st != MELT_OK) return st;
    if (p.K > 0) {
        // MFCCT over the whole slot block (rows past a stream's emitted count carry no meaning)
        const int64_t rows = (int64_t)S->n_streams * S->max_frames;
        st = launch_cepstrum(p, S->d_lmel, rows, d_out, s);
    }
    return st;
}

int32_t melt_variant_count(melt_plan plan) {
    const Plan *p = reinterpret_cast<const Plan *>(plan);
    return p ? forward_variants(*p) : 0;
}

const char *melt_variant_name(melt_plan plan, int32_t v) {
    const Plan *p = reinterpret_cast<const Plan *>(plan);
    return p ? forward_variant_name(*p, v) : "none";
}

melt_status melt_set_variant(melt_plan plan, int32_t v, int32_t grid_per_cu) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p) return set_error(MELT_E_INVALID_ARG, "plan is NULL");
    if (v < 0 || v >= forward_variants(*p)) return set_error(MELT_E_INVALID_ARG, "variant out of range");
    if (grid_per_cu < 0 || grid_per_cu > 4) return set_error(MELT_E_INVALID_ARG, "grid_per_cu must be in [0, 4]");
    p->tune_variant = v;
    p->tune_grid = grid_per_cu;
    return MELT_OK;
}

melt_status melt_autotune(melt_plan plan, int64_t total_frames, char *desc, int32_t desc_len) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || total_frames < 1) return set_error(MELT_E_INVALID_ARG, "bad autotune arguments");
    melt_status st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    // synthetic batch: clips of 2998 frames (30 s at 16 kHz with N=400, H=160 geometry)
    const int64_t per_clip = 2998;
    const int n_clips = (int)std::max<int64_t>(1, (total_frames + per_clip - 1) / per_clip);
    const int64_t clip_len = (per_clip - 1) * p->H + p->N;
    std::vector<int64_t> off(n_clips + 1);
    for (int c = 0; c <= n_clips; ++c) off[c] = c * clip_len;
    const int64_t T = (int64_t)n_clips * per_clip;
    float *d_wave = nullptr, *d_out = nullptr;
    int64_t *d_off = nullptr;
    bool ok = hipMalloc(&d_wave, sizeof(float) * off[n_clips]) == hipSuccess;
    ok = ok && hipMalloc(&d_out, sizeof(float) * T * p->M) == hipSuccess;
    ok = ok && hipMalloc(&d_off, sizeof(int64_t) * (n_clips + 1)) == hipSuccess;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (ok) ok = hipMemset(d_wave, 0, sizeof(float) * off[n_clips]) == hipSuccess &&
                 hipMemcpy(d_off, off.data(), sizeof(int64_t) * (n_clips + 1), hipMemcpyHostToDevice) == hipSuccess;
    const int save_v = p->tune_variant, save_g = p->tune_grid;
    int best_v = save_v, best_g = save_g;
    double best_us = 1e300;
    std::string best_name;
    if (ok) {
        for (int v = 0; v < forward_variants(*p) && st == MELT_OK; ++v) {
            for (int g = 1; g <= 3 && st == MELT_OK; ++g) {
                p->tune_variant = v;
                p->tune_grid = g;
                st = launch_schedule(*p, 0, d_off, n_clips, melt_chunk_frames(*p), T, nullptr);
                for (int w = 0; w < 2 && st == MELT_OK; ++w) st = launch_melt_main(*p, d_wave, d_out, nullptr, nullptr);
                if (st != MELT_OK) break;
                (void)hipEventRecord(e0, nullptr);
                for (int r = 0; r < 5 && st == MELT_OK; ++r) st = launch_melt_main(*p, d_wave, d_out, nullptr, nullptr);
                (void)hipEventRecord(e1, nullptr);
                if (st != MELT_OK || hipEventSynchronize(e1) != hipSuccess) break;
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double us = ms * 1000.0 / 5;
                if (std::getenv("MELT_AUTOTUNE_VERBOSE"))
                    std::fprintf(stderr, "melt_autotune: %s grid=%d: %.1f us\n", forward_variant_name(*p, v), g, us);
                if (us < best_us) {
                    best_us = us;
                    best_v = v;
                    best_g = g;
                    best_name = forward_variant_name(*p, v);
                }
            }
        }
    }
    p->tune_variant = best_v;
    p->tune_grid = best_g;
    p->prepared_frames[0] = -1;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d_wave);
    (void)hipFree(d_out);
    (void)hipFree(d_off);
    if (!ok) return set_error(MELT_E_NO_MEMORY, "autotune buffers");
    if (st != MELT_OK) {
        p->tune_variant = save_v;
        p->tune_grid = save_g;
        return st;
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s grid=%dx%d CUs %.1f us for %lld frames", best_name.c_str(), best_g,
                  p->cu_count, best_us, (long long)T);
    p->last_tune = buf;
    if (desc && desc_len > 0) {
        std::strncpy(desc, buf, desc_len - 1);
        desc[desc_len - 1] = 0;
    }
    const char *path = std::getenv("MELT_AUTOTUNE_CACHE");
    if (path && *path) cache_store(path, tune_key(*p), best_v, best_g, best_us);
    return MELT_OK;
}

}  // extern "C"
