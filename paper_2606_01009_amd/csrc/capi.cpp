// extern "C" entry points of libmelt (include/melt.h): argument validation, plan
// lifecycle and dispatch to the kernels.  No call aborts or throws across the ABI.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "melt_internal.h"

namespace melt {

static thread_local std::string g_last_error;

melt_status set_error(melt_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

melt_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return MELT_OK;
    return set_error(MELT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static melt_status validate(const melt_config &c) {
    if (!(c.sample_rate > 0.0) || !std::isfinite(c.sample_rate)) return set_error(MELT_E_INVALID_ARG, "sample_rate must be > 0");
    if (c.n_fft < 2 || c.n_fft > 4096) return set_error(MELT_E_INVALID_ARG, "n_fft must be in [2, 4096]");
    if (c.hop < 1 || c.hop > 65536) return set_error(MELT_E_INVALID_ARG, "hop must be in [1, 65536]");
    if (c.n_mels < 1 || c.n_mels > 512) return set_error(MELT_E_INVALID_ARG, "n_mels must be in [1, 512]");
    if (!(c.fmin >= 0.0) || !(c.fmax > c.fmin) || c.fmax > c.sample_rate / 2 * (1 + 1e-12))
        return set_error(MELT_E_INVALID_ARG, "need 0 <= fmin < fmax <= sample_rate / 2");
    if (c.window < 0 || c.window > 2) return set_error(MELT_E_INVALID_ARG, "bad window");
    if (c.mel_formula < 0 || c.mel_formula > 1) return set_error(MELT_E_INVALID_ARG, "bad mel_formula");
    if (c.placement < 0 || c.placement > 1) return set_error(MELT_E_INVALID_ARG, "bad placement");
    if (c.output < 0 || c.output > 4) return set_error(MELT_E_INVALID_ARG, "bad output");
    if (c.output == MELT_OUT_MFCC && (c.n_mfcc < 1 || c.n_mfcc > c.n_mels))
        return set_error(MELT_E_INVALID_ARG, "n_mfcc must be in [1, n_mels]");
    // the log epilogues take the hardware logarithm of S + eps, which needs a normal FP32 argument
    if (!(c.log_eps >= 1.1754943508222875e-38) || !std::isfinite(c.log_eps))
        return set_error(MELT_E_INVALID_ARG, "log_eps must be >= 1.18e-38 (the smallest normal FP32)");
    if (c.precision < 0 || c.precision > 6) return set_error(MELT_E_INVALID_ARG, "bad precision");
    // block-scaled FP8: a frame's 32-sample blocks must be blocks of the clip (hop a multiple of 32)
    if (c.precision == MELT_PREC_FP8_E4M3_BLOCK32 && c.hop % 32 != 0)
        return set_error(MELT_E_UNSUPPORTED, "FP8 with 32-sample block scales needs hop % 32 == 0");
    if (c.fb_norm < 0 || c.fb_norm > 1) return set_error(MELT_E_INVALID_ARG, "bad fb_norm");
    // Frames that skip samples (hop > n_fft) are not implemented: the kernels stage a chunk as
    // hop-block rows whose LDS stride covers min(n_fft, hop) columns, and the streaming carry
    // keeps n_fft - hop samples.  Rejected here, before any device work.
    if (c.hop > c.n_fft) return set_error(MELT_E_UNSUPPORTED, "hop > n_fft (frames that skip samples) is not supported");
    return MELT_OK;
}

static void free_plan(Plan *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    void *bufs[] = {p->d_basis32, p->d_pack_f32, p->d_pack_h16, p->d_pack_lo, p->d_pack_f8, p->d_rowscale,
                    p->d_fb_w, p->d_fb_start, p->d_fb_off, p->d_twiddle, p->d_window, p->d_chunks[0],
                    p->d_chunks[1], p->d_nchunks, p->d_pack_dx, p->d_bwd_ws, p->d_bwd_rows, p->d_dct,
                    p->d_dct_x3, p->d_lmel, p->d_seg32, p->d_col32, p->d_seg16, p->d_col16};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

static melt_status alloc(void **d, size_t bytes) {
    if (hipMalloc(d, bytes ? bytes : 4) != hipSuccess) return set_error(MELT_E_NO_MEMORY, "hipMalloc failed");
    return MELT_OK;
}

static melt_status check_batch(Plan *p, const void *wave, const int64_t *off, int32_t n_clips, int64_t n_frames,
                               const void *out) {
    if (!p) return set_error(MELT_E_INVALID_ARG, "plan is NULL");
    if (n_clips < 0 || n_frames < 0) return set_error(MELT_E_INVALID_ARG, "negative n_clips or n_frames");
    if (n_clips > 0 && !off) return set_error(MELT_E_INVALID_ARG, "clip_offsets is NULL");
    if (n_frames > 0 && (!wave || !out)) return set_error(MELT_E_INVALID_ARG, "wave or out is NULL");
    if (n_frames > (int64_t(1) << 40)) return set_error(MELT_E_SHAPE, "n_frames too large");
    return MELT_OK;
}

}  // namespace melt

using namespace melt;

extern "C" {

melt_status melt_config_default(melt_config *cfg) {
    if (!cfg) return set_error(MELT_E_INVALID_ARG, "cfg is NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->sample_rate = 16000.0;
    cfg->n_fft = 400;
    cfg->hop = 160;
    cfg->window = MELT_WIN_HANN_SYMMETRIC;
    cfg->n_mels = 80;
    cfg->fmin = 0.0;
    cfg->fmax = 8000.0;
    cfg->mel_formula = MELT_MEL_HTK;
    cfg->placement = MELT_PLACE_FILTER_CENTRES;
    cfg->output = MELT_OUT_LOG_POWER;
    cfg->log_eps = 1e-10;
    cfg->precision = MELT_PREC_FP32;
    cfg->fb_norm = MELT_FB_NORM_NONE;
    cfg->n_mfcc = 40;
    return MELT_OK;
}

int64_t melt_num_frames(int64_t n_samples, int32_t n_fft, int32_t hop) {
    if (n_fft < 1 || hop < 1) return -1;
    if (n_samples < n_fft) return 0;
    return 1 + (n_samples - n_fft) / hop;
}

melt_status melt_plan_create(const melt_config *cfg, int device, melt_plan *out) {
    if (!cfg || !out) return set_error(MELT_E_INVALID_ARG, "cfg or out is NULL");
    *out = nullptr;
    melt_status st = validate(*cfg);
    if (st != MELT_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return set_error(MELT_E_HIP, "no HIP device");
    if (device < 0 || device >= ndev) return set_error(MELT_E_INVALID_ARG, "bad device index");
    st = hip_check(hipSetDevice(device), "hipSetDevice");
    if (st != MELT_OK) return st;
    Plan *p = new (std::nothrow) Plan();
    if (!p) return set_error(MELT_E_NO_MEMORY, "plan");
    p->cfg = *cfg;
    p->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        p->cu_count = cus;
    st = plan_build_host(*p);
    const size_t nb = size_t(2) * p->M * p->N;
    const size_t RT = p->row_tiles;
    if (st == MELT_OK) st = alloc((void **)&p->d_basis32, nb * sizeof(float));
    if (st == MELT_OK) st = alloc(&p->d_pack_f32, RT * p->geo32.n_groups * 64 * 4 * sizeof(float));
    if (st == MELT_OK) st = alloc(&p->d_pack_h16, RT * p->geo16.n_groups * 64 * 8 * 2);
    if (st == MELT_OK) st = alloc(&p->d_pack_lo, RT * p->geo16.n_groups * 64 * 8 * 2);
    if (st == MELT_OK) st = alloc(&p->d_pack_f8, RT * ((p->N + 63) / 64) * 64 * 32);
    if (st == MELT_OK) st = alloc((void **)&p->d_rowscale, RT * 32 * sizeof(float));
    if (st == MELT_OK) st = alloc((void **)&p->d_nchunks, 2 * sizeof(int));
    if (st == MELT_OK) {
        std::vector<float> b32(nb);
        for (size_t i = 0; i < nb; ++i) b32[i] = float(p->basis64[i]);
        st = hip_check(hipMemcpy(p->d_basis32, b32.data(), nb * sizeof(float), hipMemcpyHostToDevice), "upload basis");
    }
    p->K = cfg->output == MELT_OUT_MFCC ? cfg->n_mfcc : 0;
    p->kern_out = cfg->output == MELT_OUT_MFCC ? MELT_OUT_LOG_POWER : cfg->output;
    if (st == MELT_OK && p->K > 0) {
        std::vector<float> D;
        dct_matrix(p->K, p->M, D);
        st = alloc((void **)&p->d_dct, D.size() * sizeof(float));
        if (st == MELT_OK)
            st = hip_check(hipMemcpy(p->d_dct, D.data(), D.size() * sizeof(float), hipMemcpyHostToDevice), "upload DCT");
        const int prec = cfg->precision;
        if (st == MELT_OK && (prec == MELT_PREC_BF16 || prec == MELT_PREC_FP16 || prec == MELT_PREC_FP8_E4M3 ||
                              prec == MELT_PREC_FP8_E4M3_BLOCK32))
            st = pack_dct_x3(*p);
    }
    if (st == MELT_OK) init_variants(*p);
    if (st == MELT_OK) st = pack_tables_upload(*p);
    if (st == MELT_OK) st = pack_basis(*p, nullptr);
    if (st == MELT_OK) st = hip_check(hipStreamSynchronize(nullptr), "pack basis");
    if (st == MELT_OK) st = stft_plan_build(*p);
    if (st == MELT_OK) st = ensure_chunks(*p, 0, 4096);
    if (st == MELT_OK) st = ensure_chunks(*p, 1, 4096);
    if (st == MELT_OK) st = scratch_init(device);
    if (st == MELT_OK) apply_tune_cache(*p);
    if (st != MELT_OK) {
        free_plan(p);
        return st;
    }
    *out = reinterpret_cast<melt_plan>(p);
    return MELT_OK;
}

melt_status melt_plan_destroy(melt_plan plan) {
    free_plan(reinterpret_cast<Plan *>(plan));
    return MELT_OK;
}

melt_status melt_plan_get_config(melt_plan plan, melt_config *cfg) {
    if (!plan || !cfg) return set_error(MELT_E_INVALID_ARG, "NULL argument");
    *cfg = reinterpret_cast<Plan *>(plan)->cfg;
    return MELT_OK;
}

melt_status melt_plan_get_frequencies(melt_plan plan, double *freqs_hz) {
    if (!plan || !freqs_hz) return set_error(MELT_E_INVALID_ARG, "NULL argument");
    Plan *p = reinterpret_cast<Plan *>(plan);
    std::memcpy(freqs_hz, p->freqs.data(), sizeof(double) * p->M);
    return MELT_OK;
}

melt_status melt_plan_get_basis(melt_plan plan, float *h_basis) {
    if (!plan || !h_basis) return set_error(MELT_E_INVALID_ARG, "NULL argument");
    Plan *p = reinterpret_cast<Plan *>(plan);
    melt_status st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    st = hip_check(hipDeviceSynchronize(), "sync");
    if (st != MELT_OK) return st;
    return hip_check(hipMemcpy(h_basis, p->d_basis32, sizeof(float) * 2 * p->M * p->N, hipMemcpyDeviceToHost),
                     "download basis");
}

melt_status melt_plan_set_basis(melt_plan plan, const float *d_basis, void *stream) {
    if (!plan || !d_basis) return set_error(MELT_E_INVALID_ARG, "NULL argument");
    Plan *p = reinterpret_cast<Plan *>(plan);
    hipStream_t s = (hipStream_t)stream;
    melt_status st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    st = hip_check(hipMemcpyAsync(p->d_basis32, d_basis, sizeof(float) * 2 * p->M * p->N, hipMemcpyDeviceToDevice, s),
                   "copy basis");
    if (st != MELT_OK) return st;
    return pack_basis(*p, s);
}

melt_status melt_frame_offsets(melt_plan plan, const int64_t *d_clip_offsets, int32_t n_clips,
                               int64_t *d_frame_offsets, void *stream) {
    if (!plan || !d_frame_offsets || (n_clips > 0 && !d_clip_offsets) || n_clips < 0)
        return set_error(MELT_E_INVALID_ARG, "bad argument");
    Plan *p = reinterpret_cast<Plan *>(plan);
    return launch_frame_offsets(d_clip_offsets, n_clips, p->N, p->H, d_frame_offsets, (hipStream_t)stream);
}

melt_status melt_forward(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets, int32_t n_clips,
                         int64_t n_frames, float *d_out, void *stream) {
    return melt_forward_proj(plan, d_wave, d_clip_offsets, n_clips, n_frames, d_out, nullptr, stream);
}

melt_status melt_forward_proj(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets, int32_t n_clips,
                              int64_t n_frames, float *d_out, float *d_proj, void *stream) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    melt_status st = check_batch(p, d_wave, d_clip_offsets, n_clips, n_frames, d_out);
    if (st != MELT_OK) return st;
    if (n_clips == 0 || n_frames == 0) return MELT_OK;
    st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = launch_schedule(*p, 0, d_clip_offsets, n_clips, melt_chunk_frames(*p), n_frames, s);
    if (st != MELT_OK) return st;
    return launch_melt_main(*p, d_wave, d_out, d_proj, s);
}

melt_status melt_forward_noalloc(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets,
                                 int32_t n_clips, int64_t n_frames, float *d_out, void *stream) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    melt_status st = check_batch(p, d_wave, d_clip_offsets, n_clips, n_frames, d_out);
    if (st != MELT_OK) return st;
    if (n_clips == 0 || n_frames == 0) return MELT_OK;
    st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    return forward_noalloc(*p, d_wave, d_clip_offsets, n_clips, n_frames, d_out, (hipStream_t)stream);
}

melt_status stft_mel_forward(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets, int32_t n_clips,
                             int64_t n_frames, float *d_out, void *stream) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    melt_status st = check_batch(p, d_wave, d_clip_offsets, n_clips, n_frames, d_out);
    if (st != MELT_OK) return st;
    if (n_clips == 0 || n_frames == 0) return MELT_OK;
    st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = launch_schedule(*p, 1, d_clip_offsets, n_clips, stft_chunk_frames(*p), n_frames, s);
    if (st != MELT_OK) return st;
    return launch_stft_main(*p, d_wave, d_out, s);
}

melt_status melt_batch_prepare(melt_plan plan, const int64_t *d_clip_offsets, int32_t n_clips, int64_t n_frames,
                               void *stream) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || n_clips < 0 || n_frames < 0 || (n_clips > 0 && !d_clip_offsets))
        return set_error(MELT_E_INVALID_ARG, "bad argument");
    melt_status st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (n_clips == 0) {
        p->prepared_frames[0] = p->prepared_frames[1] = 0;
        return MELT_OK;
    }
    st = launch_schedule(*p, 0, d_clip_offsets, n_clips, melt_chunk_frames(*p), n_frames, s);
    if (st != MELT_OK) return st;
    return launch_schedule(*p, 1, d_clip_offsets, n_clips, stft_chunk_frames(*p), n_frames, s);
}

melt_status melt_forward_prepared(melt_plan plan, const float *d_wave, float *d_out, float *d_proj, void *stream) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p) return set_error(MELT_E_INVALID_ARG, "plan is NULL");
    if (p->prepared_frames[0] > 0 && (!d_wave || !d_out)) return set_error(MELT_E_INVALID_ARG, "NULL buffer");
    melt_status st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    return launch_melt_main(*p, d_wave, d_out, d_proj, (hipStream_t)stream);
}

melt_status stft_mel_forward_prepared(melt_plan plan, const float *d_wave, float *d_out, void *stream) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p) return set_error(MELT_E_INVALID_ARG, "plan is NULL");
    if (p->prepared_frames[1] > 0 && (!d_wave || !d_out)) return set_error(MELT_E_INVALID_ARG, "NULL buffer");
    melt_status st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    return launch_stft_main(*p, d_wave, d_out, (hipStream_t)stream);
}

melt_status melt_backward(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets, int32_t n_clips,
                          int64_t n_frames, const float *d_grad_out, const float *d_proj, float *d_grad_wave,
                          float *d_grad_basis, void *stream) {
    Plan *p = reinterpret_cast<Plan *>(plan);
    melt_status st = check_batch(p, d_wave, d_clip_offsets, n_clips, n_frames, d_grad_out);
    if (st != MELT_OK) return st;
    st = hip_check(hipSetDevice(p->device), "hipSetDevice");
    if (st != MELT_OK) return st;
    return launch_melt_backward(*p, d_wave, d_clip_offsets, n_clips, n_frames, d_grad_out, d_proj, d_grad_wave,
                                d_grad_basis, (hipStream_t)stream);
}

const char *melt_status_string(melt_status s) {
    switch (s) {
    case MELT_OK: return "MELT_OK";
    case MELT_E_INVALID_ARG: return "MELT_E_INVALID_ARG";
    case MELT_E_UNSUPPORTED: return "MELT_E_UNSUPPORTED";
    case MELT_E_NO_MEMORY: return "MELT_E_NO_MEMORY";
    case MELT_E_HIP: return "MELT_E_HIP";
    case MELT_E_SHAPE: return "MELT_E_SHAPE";
    default: return "MELT_E_UNKNOWN";
    }
}

const char *melt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
