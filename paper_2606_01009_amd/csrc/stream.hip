// Streaming MelT (many live audio streams, fixed-size pushes) and the autotuner.
//
// A stream holds the samples that no complete frame has used yet (fewer than n_fft).  A
// push of chunk_len samples per stream:
//   1. k_stream_assemble: per stream, [carry | chunk] into an assembly buffer; the number
//      of complete frames k = floor((len - N) / H) + 1; chunk-table entries that point the
//      MelT kernel at the assembly buffer with output rows in the stream's fixed slot
//   2. the MelT main kernel over that table (same kernels as melt_forward)
//   3. k_stream_keep: the unconsumed tail [k H, len) becomes the new carry
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
    int n_streams, max_chunk, max_frames, cps, bf, variant;
    int asm_stride;             // samples per stream in the assembly buffer
    float *d_carry;             // [n_streams][N]
    int *d_carry_len;           // [n_streams]
    float *d_asm;               // [n_streams][asm_stride]
    melt::Chunk *d_tab;         // [n_streams * cps]
    int *d_ntab;
    float *d_lmel;              // [n_streams * max_frames][n_mels] log-Mel rows (MELT_OUT_MFCC only)
};

namespace melt {

__global__ __launch_bounds__(256) void k_stream_assemble(const float *__restrict__ chunk, int chunk_len,
                                                         const float *__restrict__ carry, const int *__restrict__ carry_len,
                                                         int N, int H, float *__restrict__ asmb, int asm_stride,
                                                         int max_frames, int cps, int bf, Chunk *__restrict__ tab,
                                                         int *__restrict__ ntab, int *__restrict__ emitted,
                                                         int n_streams) {
    const int s = blockIdx.x;
    const int len0 = carry_len[s];
    const int total = len0 + chunk_len;
    float *dst = asmb + (size_t)s * asm_stride;
    for (int i = threadIdx.x; i < len0; i += blockDim.x) dst[i] = carry[(size_t)s * N + i];
    for (int i = threadIdx.x; i < chunk_len; i += blockDim.x) dst[len0 + i] = chunk[(size_t)s * chunk_len + i];
    const int k = total >= N ? 1 + (total - N) / H : 0;
    if (threadIdx.x == 0) emitted[s] = k;
    for (int j = threadIdx.x; j < cps; j += blockDim.x) {
        Chunk e;
        e.sample_start = (int64_t)s * asm_stride + (int64_t)j * bf * H;
        e.sample_end = (int64_t)s * asm_stride + total;
        e.out_row = (int64_t)s * max_frames + (int64_t)j * bf;
        const int nf = k - j * bf;
        e.n_frames = nf < 0 ? 0 : (nf > bf ? bf : nf);
        e.clip = s;
        tab[(size_t)s * cps + j] = e;
    }
    if (s == 0 && threadIdx.x == 0) *ntab = n_streams * cps;
}

__global__ __launch_bounds__(256) void k_stream_keep(int chunk_len, float *__restrict__ carry, int *__restrict__ carry_len,
                                                     int N, int H, const float *__restrict__ asmb, int asm_stride) {
    const int s = blockIdx.x;
    const int len0 = carry_len[s];
    const int total = len0 + chunk_len;
    const int k = total >= N ? 1 + (total - N) / H : 0;
    const int from = k * H;
    const int rem = total - from;
    const float *src = asmb + (size_t)s * asm_stride + from;
    for (int i = threadIdx.x; i < rem; i += blockDim.x) carry[(size_t)s * N + i] = src[i];
    __syncthreads();   // every thread has read len0 before it is replaced
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
    S->cps = (S->max_frames + S->bf - 1) / S->bf;
    // assembly stride: carry (< N) + chunk + the J - 1 hop rows a chunk's span may reach past
    // its last frame; multiple of 4 samples
    S->asm_stride = ((p->N + max_chunk_len + 4 * p->H + 3) / 4) * 4;
    bool ok = hipMalloc(&S->d_carry, sizeof(float) * (size_t)n_streams * p->N) == hipSuccess;
    ok = ok && hipMalloc(&S->d_carry_len, sizeof(int) * n_streams) == hipSuccess;
    ok = ok && hipMalloc(&S->d_asm, sizeof(float) * (size_t)n_streams * S->asm_stride) == hipSuccess;
    ok = ok && hipMalloc(&S->d_tab, sizeof(Chunk) * (size_t)n_streams * S->cps) == hipSuccess;
    ok = ok && hipMalloc(&S->d_ntab, sizeof(int)) == hipSuccess;
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
    void *b[] = {S->d_carry, S->d_carry_len, S->d_asm, S->d_tab, S->d_ntab, S->d_lmel};
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
    k_stream_assemble<<<S->n_streams, 256, 0, s>>>(d_chunk, chunk_len, S->d_carry, S->d_carry_len, p.N, p.H, S->d_asm,
                                                   S->asm_stride, S->max_frames, S->cps, S->bf, S->d_tab, S->d_ntab,
                                                   d_frames_emitted, S->n_streams);
    st = hip_check(hipGetLastError(), "stream assemble");
    if (st != MELT_OK) return st;
    const int64_t rows = (int64_t)S->n_streams * S->max_frames;
    st = launch_melt_table(p, S->variant, S->d_tab, S->d_ntab, (int64_t)S->n_streams * S->cps, rows, S->d_asm,
                           p.K > 0 ? S->d_lmel : d_out, nullptr, s);
    if (st != MELT_OK) return st;
    if (p.K > 0) {
        // MFCCT over the whole slot block (rows past a stream's emitted count carry no meaning)
        st = launch_row_matmul(S->d_lmel, rows, p.M, p.K, p.d_dct, p.M, 1, d_out, s);
        if (st != MELT_OK) return st;
    }
    k_stream_keep<<<S->n_streams, 256, 0, s>>>(chunk_len, S->d_carry, S->d_carry_len, p.N, p.H, S->d_asm,
                                               S->asm_stride);
    return hip_check(hipGetLastError(), "stream keep");
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
