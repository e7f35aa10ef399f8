/*
 * melt.h - C ABI of the MI355X (gfx950) MelT frontend library (libmelt.so).
 *
 * MelT (arXiv 2606.01009, Methodology "Matmul-Native Mel Frontends") computes, for every
 * frame x_t of a waveform, the projections of the windowed frame onto cosines and sines at
 * Mel-spaced frequencies f_m (Eq. dmp_components), the energy S = R^2 + I^2
 * (Eq. dmp_energy) and log(S + eps) (Eq. meltf).  The window is folded into a fixed basis
 * (Eq. dmp_weights) so that all frames are projected by one GEMM against the stacked
 * cos/sin basis (Eq. dmp_projection).  The library also provides the conventional
 * pipeline the paper compares against (STFT power on uniform bins aggregated by
 * triangular Mel filters, then log; Methodology, Eq. complexity_conv), the gradient of
 * the projection for learnable frontends, and a streaming interface.
 *
 * Conventions shared by every entry point
 *   - All functions return melt_status (MELT_OK = 0).  Nothing aborts or throws across the
 *     ABI; melt_last_error() gives a thread-local message for the last failure.
 *   - Pointers documented "device" must point to memory on the plan's device that the
 *     caller allocated and owns; pointers documented "host" are ordinary host memory.
 *     The library never frees caller memory and keeps no pointer to it after a call
 *     returns (except a stream state's own buffers, which it owns).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is enqueued
 *     asynchronously on it; the call returns before the GPU finishes.
 *   - A batch of clips is one float32 buffer with all clips back to back, described by
 *     `clip_offsets` (int64, n_clips + 1 entries, non-decreasing, offsets[0] may be > 0):
 *     clip c is samples [offsets[c], offsets[c+1]).  A clip of L samples has
 *     T_c = 1 + floor((L - n_fft) / hop) frames if L >= n_fft and none otherwise (frames
 *     start at t*hop with no centring or padding).  Outputs are frame-major [T, n_mels]
 *     float32 with the frames of clip 0 first, T = sum_c T_c.
 *   - Calls that share a plan use the plan's workspace and must be issued on one stream
 *     (or otherwise serialised); use one plan per concurrent stream.
 */
#ifndef MELT_H
#define MELT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MELT_OK = 0,
    MELT_E_INVALID_ARG = 1,  /* a NULL pointer, a bad enum, or a parameter out of range */
    MELT_E_UNSUPPORTED = 2,  /* valid but not implemented for this configuration */
    MELT_E_NO_MEMORY = 3,    /* a host or device allocation failed */
    MELT_E_HIP = 4,          /* a HIP runtime call failed (detail in melt_last_error) */
    MELT_E_SHAPE = 5         /* sizes inconsistent with the plan (e.g. too many frames) */
} melt_status;

/* Analysis window, folded into the basis.  The paper uses the symmetric Hann window
 * w[n] = 0.5 - 0.5 cos(2 pi n / (N - 1)) (Methodology). */
typedef enum { MELT_WIN_HANN_SYMMETRIC = 0, MELT_WIN_HANN_PERIODIC = 1, MELT_WIN_RECT = 2 } melt_window;

/* Mel scale: HTK mu(f) = 2595 log10(1 + f/700) (Eq. mel_scale) or the Slaney scale. */
typedef enum { MELT_MEL_HTK = 0, MELT_MEL_SLANEY = 1 } melt_mel_formula;

/* Placement of the M analysis frequencies: the centres of the M triangular filters of the
 * conventional filterbank (interior points of an (M+2)-point grid uniform in Mel between
 * fmin and fmax; the reading used throughout), or M points uniform in Mel from fmin to
 * fmax inclusive. */
typedef enum { MELT_PLACE_FILTER_CENTRES = 0, MELT_PLACE_LINSPACE = 1 } melt_freq_placement;

/* Normalisation of the comparator's triangular filters: peak 1, or unit area (Slaney). */
typedef enum { MELT_FB_NORM_NONE = 0, MELT_FB_NORM_SLANEY = 1 } melt_fb_norm;

/* Output map applied to S = R^2 + I^2 (MelT) or to the filterbank sum (comparator):
 * ln(S + eps) (Eq. meltf), ln(sqrt(S) + eps), S, sqrt(S).  For the comparator the
 * magnitude kinds aggregate |X_k| instead of |X_k|^2.  MELT_OUT_MFCC is the cepstrum of
 * the log power, C = ln(S + eps) D^T with D the first n_mfcc rows of the orthonormal
 * DCT-II over the M Mel bins (Eq. mfcct_matrix: MFCCT for MelT; conventional MFCC for the
 * comparator); its rows are n_mfcc wide instead of n_mels. */
typedef enum {
    MELT_OUT_LOG_POWER = 0, MELT_OUT_LOG_MAGNITUDE = 1, MELT_OUT_POWER = 2, MELT_OUT_MAGNITUDE = 3,
    MELT_OUT_MFCC = 4
} melt_output;

/* Arithmetic of the projection GEMM (all accumulate in FP32; the basis is computed in
 * FP64 and rounded once):
 *   FP32     - FP32 operands (v_mfma_f32_32x32x2_f32)
 *   BF16     - bfloat16 operands
 *   FP16     - binary16 operands
 *   FP8_E4M3 - OCP E4M3 operands; each frame scaled by 448 / max|x_t| and each basis row by
 *              448 / max|row| before rounding, undone in FP32 after the product
 *   BF16X3   - split-bfloat16 compensated product xh*Wh + xh*Wl + xl*Wh: two 8-bit
 *              significands per operand, about 17 significant bits per product term
 *   FP16X3   - split-binary16 compensated product xh*Wh + xh*Wl + xl*Wh, products exact in
 *              FP32: two 11-bit significands per operand, about 22 significant bits per term
 *              (FP32-level).  The waveform is pre-scaled by 2^10 (exact) so that the low parts
 *              of quiet samples stay normal; the scale is undone on the FP32 projections.
 *              Samples must satisfy |x| < 63.9 (2^10 |x| within binary16's range); a
 *              larger sample overflows and the frames that contain it come out non-finite.
 *   FP8_E4M3_BLOCK32 - OCP E4M3 operands with power-of-two block scales instead of frame
 *              scales: the waveform of each clip is cut into 32-sample blocks from its first
 *              sample, block b is scaled by 2^e_b with e_b the largest integer such that
 *              2^e_b max|x_b| <= 448 (e_b = 0 for a silent block, clamped to [-127, 127])
 *              and rounded to E4M3 once; every frame reads its samples from that one image,
 *              and the matrix cores undo 2^-e_b per 32-sample block of the product (E8M0
 *              block scales of v_mfma_scale_f32_32x32x64_f8f6f4).  Basis rows are scaled as
 *              for FP8_E4M3.  This is block scaling, not per-frame scaling: a sample gets the
 *              scale of its own block whatever frame reads it.  Needs hop % 32 == 0
 *              (else MELT_E_UNSUPPORTED at plan creation) and, as FP8_E4M3, n_fft in
 *              (192, 256], (384, 512] or (960, 1024] (else MELT_E_UNSUPPORTED at the call). */
typedef enum {
    MELT_PREC_FP32 = 0, MELT_PREC_BF16 = 1, MELT_PREC_FP16 = 2, MELT_PREC_FP8_E4M3 = 3, MELT_PREC_BF16X3 = 4,
    MELT_PREC_FP16X3 = 5, MELT_PREC_FP8_E4M3_BLOCK32 = 6
} melt_precision;

/* Frontend parameters (Experiments, Table "Audio frontend configuration": 16 kHz,
 * N = 400, H = 160, M = 80).  Enumerations are stored as int32_t for a fixed layout. */
typedef struct {
    double  sample_rate;   /* Hz, > 0 */
    int32_t n_fft;         /* frame length N (window length), 2 .. 4096 */
    int32_t hop;           /* hop H, 1 .. min(n_fft, 65536); hop > n_fft gives MELT_E_UNSUPPORTED */
    int32_t window;        /* melt_window */
    int32_t n_mels;        /* M, 1 .. 512 */
    double  fmin, fmax;    /* 0 <= fmin < fmax <= sample_rate / 2 */
    int32_t mel_formula;   /* melt_mel_formula */
    int32_t placement;     /* melt_freq_placement */
    int32_t output;        /* melt_output */
    double  log_eps;       /* eps of the log kinds, >= 1.18e-38 (the smallest normal FP32; default 1e-10) */
    int32_t precision;     /* melt_precision of melt_forward */
    int32_t fb_norm;       /* melt_fb_norm of stft_mel_forward */
    int32_t n_mfcc;        /* K, cepstral coefficients of MELT_OUT_MFCC, 1 .. n_mels (default 40) */
} melt_config;

typedef struct melt_plan_s *melt_plan;
typedef struct melt_stream_s *melt_stream_state;

/* Fills `cfg` with the paper's spectral configuration at 16 kHz: N = 400, H = 160,
 * M = 80, symmetric Hann, HTK, filter-centre placement, fmin 0, fmax 8000, log power,
 * eps 1e-10, FP32, peak-1 filters, 40 cepstral coefficients.  cfg: host, caller-owned. */
melt_status melt_config_default(melt_config *cfg);

/* Number of frames of a clip of n_samples samples (see the conventions above); 0 if
 * n_samples < n_fft; -1 if n_fft < 1 or hop < 1. */
int64_t melt_num_frames(int64_t n_samples, int32_t n_fft, int32_t hop);

/* Builds a plan on HIP device `device`: the Mel analysis frequencies (Eq. mel_scale,
 * Eq. inverse_mel), the window-folded cos/sin basis (Eq. dmp_weights) in FP64 with exact
 * phase reduction, rounded and packed for every precision, the comparator's triangular
 * filterbank and FFT tables, and a small device workspace.  cfg: host, read only;
 * *out receives the plan (owned by the caller, freed by melt_plan_destroy).  Errors:
 * MELT_E_INVALID_ARG for out-of-range parameters, MELT_E_UNSUPPORTED for sizes the
 * kernels do not handle (among them hop > n_fft: frames that skip samples), MELT_E_HIP /
 * MELT_E_NO_MEMORY on runtime failures.  Parameters are validated before any device call. */
melt_status melt_plan_create(const melt_config *cfg, int device, melt_plan *out);

/* Frees the plan and its device memory (synchronises the plan's device first).  NULL ok. */
melt_status melt_plan_destroy(melt_plan plan);

/* Copies the plan's configuration into *cfg (host). */
melt_status melt_plan_get_config(melt_plan plan, melt_config *cfg);

/* The M analysis frequencies f_m in Hz (Eq. inverse_mel), FP64, into host array
 * freqs_hz[n_mels]. */
melt_status melt_plan_get_frequencies(melt_plan plan, double *freqs_hz);

/* The plan's current FP32 basis, in the paper's stacked order [W^(r); W^(i)]
 * (Eq. dmp_projection): rows 0..M-1 are w[n] cos(2 pi f_m n / sr), rows M..2M-1 the sines,
 * each n_fft long.  h_basis: host, float32 [2*n_mels, n_fft]. */
melt_status melt_plan_get_basis(melt_plan plan, float *h_basis);

/* Replaces the plan's basis (learnable frontends).  d_basis: device, float32
 * [2*n_mels, n_fft] in the stacked order above; it is read on `stream` and re-packed into
 * every precision's layout before later calls on that stream.  The comparator is not
 * affected. */
melt_status melt_plan_set_basis(melt_plan plan, const float *d_basis, void *stream);

/* Device prefix sums of the frame counts: d_frame_offsets[c] = sum_{c' < c} T_c' for
 * c = 0..n_clips.  d_clip_offsets: device int64 [n_clips + 1]; d_frame_offsets: device
 * int64 [n_clips + 1]. */
melt_status melt_frame_offsets(melt_plan plan, const int64_t *d_clip_offsets, int32_t n_clips,
                               int64_t *d_frame_offsets, void *stream);

/* MelT forward (Eqs. dmp_projection, dmp_matrix_energy, meltf): out[t, m] =
 * map(R[t,m]^2 + I[t,m]^2) for all frames of all clips, in the plan's precision.
 * One persistent launch covers the ragged batch; frames are read straight from the
 * waveform (no frame matrix is formed).
 *   d_wave         device float32, all clips back to back (read only)
 *   d_clip_offsets device int64 [n_clips + 1] (read only)
 *   n_clips        >= 0 (0 enqueues nothing)
 *   n_frames       T, the number of rows of d_out, which the caller computes as the sum of
 *                  the clips' frame counts (melt_num_frames per clip).  The library does not
 *                  read d_clip_offsets on the host, so it cannot check this: if the offsets
 *                  describe fewer frames, rows past their total are left untouched; if
 *                  more, frames from row n_frames on are not written.  Either way no
 *                  memory outside d_out's n_frames rows is written.
 *   d_out          device float32 [n_frames, n_mels] (written); [n_frames, n_mfcc] for
 *                  MELT_OUT_MFCC, which runs the Mel kernel into a plan workspace and then
 *                  the DCT-II product
 * Errors: MELT_E_INVALID_ARG (NULL pointers with n_frames > 0, negative counts). */
melt_status melt_forward(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets,
                         int32_t n_clips, int64_t n_frames, float *d_out, void *stream);

/* As melt_forward, for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the chunk count and chunk
 * table live in a fixed 1 MiB device array of the library (one per GPU, held until the
 * process ends) instead of the plan's growable workspace, and the call makes no hipMalloc,
 * hipFree or other allocating call.  The scratch holds at most 32 760 chunk-table entries:
 * the call needs n_frames / F + n_clips + 1 of them, F being the frames per chunk of the
 * plan's kernel variant (the "-bfF" suffix of melt_variant_name; 128 for the default FP32,
 * BF16 and FP16 kernels), so e.g. up to about 4 million frames in few clips.  Every call on
 * one GPU shares that GPU's scratch (from every plan): calls that overlap in time on one
 * GPU (on different streams, or from several host threads) race and must be serialised by
 * the caller.  Prepared batches of the plan are left untouched.  Arguments as in
 * melt_forward.
 * Errors: as melt_forward; MELT_E_SHAPE if the batch needs more chunk entries than the
 * scratch holds (checked on the host, nothing is enqueued); MELT_E_UNSUPPORTED for
 * MELT_OUT_MFCC plans (their cepstrum reads a log-Mel workspace the size of the batch). */
melt_status melt_forward_noalloc(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets,
                                 int32_t n_clips, int64_t n_frames, float *d_out, void *stream);

/* As melt_forward, also writing the raw projections for the backward pass:
 * d_proj device float32 [n_frames, 2 * n_mels], row t = (R[t,0], I[t,0], R[t,1], I[t,1], ...). */
melt_status melt_forward_proj(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets,
                              int32_t n_clips, int64_t n_frames, float *d_out, float *d_proj,
                              void *stream);

/* Conventional comparator: per frame, the symmetric-window N-point real DFT by a
 * hand-written mixed-radix FFT, the power |X_k|^2 (or |X_k| for the magnitude kinds) on
 * bins k = 0..N/2, the sparse triangular Mel filterbank (Methodology; nnz bound of
 * Eq. complexity_conv) and the output map, fused in one kernel in FP32.  Arguments as in
 * melt_forward.  MELT_E_UNSUPPORTED if n_fft has a prime factor other than 2, 3 or 5. */
melt_status stft_mel_forward(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets,
                             int32_t n_clips, int64_t n_frames, float *d_out, void *stream);

/* Prepared batches, for callers that run the same batch layout many times (serving loops,
 * benchmarks): melt_batch_prepare builds, on `stream`, the plan's chunk tables for the
 * clips in d_clip_offsets (as in melt_forward); melt_forward_prepared and
 * stft_mel_forward_prepared then launch only the main kernel over that batch.  The
 * tables stay valid until the next melt_forward / melt_forward_proj / stft_mel_forward /
 * melt_batch_prepare / melt_backward call on the plan (the backward builds its own batch's
 * tables in the same plan workspace).  Buffers as in melt_forward_proj / stft_mel_forward
 * (d_proj may be NULL). */
melt_status melt_batch_prepare(melt_plan plan, const int64_t *d_clip_offsets, int32_t n_clips,
                               int64_t n_frames, void *stream);
melt_status melt_forward_prepared(melt_plan plan, const float *d_wave, float *d_out, float *d_proj,
                                  void *stream);
melt_status stft_mel_forward_prepared(melt_plan plan, const float *d_wave, float *d_out, void *stream);

/* Gradient of the MelT forward (not in the paper; chain rule through Eqs. meltf,
 * dmp_matrix_energy, dmp_projection), in FP32:
 *   G[t, 2m]   = g[t,m] map'(S) 2 R[t,m],  G[t, 2m+1] = g[t,m] map'(S) 2 I[t,m]
 *   d_grad_wave[s] = sum over frames t and n with start_t + n = s of (G W)[t, n]
 *   d_grad_basis   = G^T X in the stacked order of melt_plan_get_basis
 *   d_grad_out   device float32 [n_frames, n_mels] (read only); [n_frames, n_mfcc] for
 *                MELT_OUT_MFCC (the cepstrum is linear: dL = dC D, then as log power)
 *   d_proj       device float32 [n_frames, 2 n_mels] from melt_forward_proj, or NULL to
 *                recompute the projections
 *   d_grad_wave  device float32, same length as d_wave's samples up to
 *                d_clip_offsets[n_clips] (written: samples in no frame get 0), or NULL
 *   d_grad_basis device float32 [2 n_mels, n_fft] (written, not accumulated), or NULL
 * Deterministic: no floating-point atomics. */
melt_status melt_backward(melt_plan plan, const float *d_wave, const int64_t *d_clip_offsets,
                          int32_t n_clips, int64_t n_frames, const float *d_grad_out,
                          const float *d_proj, float *d_grad_wave, float *d_grad_basis,
                          void *stream);

/* Streaming: n_streams independent audio streams over the plan (same frontend, same
 * precision).  Each stream keeps in device memory owned by the state the samples that
 * no complete frame has consumed yet (fewer than n_fft), so frames come out exactly as
 * melt_forward would produce them for the concatenated stream.
 *   melt_stream_create   n_streams >= 1, 1 <= max_chunk_len <= 1 << 20; allocates the
 *                        state (carry buffers, assembly buffers, a private chunk table)
 *   melt_stream_reset    empties every stream (enqueued on `stream`)
 *   melt_stream_max_frames  frames one push can emit per stream:
 *                        floor((max_chunk_len + n_fft - 1 - n_fft) / hop) + 1
 *   melt_stream_push     appends chunk_len (1..max_chunk_len) samples to every stream:
 *                        d_chunk device float32 [n_streams, chunk_len] (row-major);
 *                        writes stream s's new frames to d_out (device float32
 *                        [n_streams, max_frames, n_mels], or n_mfcc wide for
 *                        MELT_OUT_MFCC) rows [s * max_frames, + k) and k to
 *                        d_frames_emitted[s] (device int32 [n_streams]); under
 *                        MELT_OUT_MFCC the rows past k are written too, with no meaning.
 * A push is three kernel launches (four under MELT_OUT_MFCC: assemble, project, cepstrum,
 * keep the tail) with no host
 * synchronisation and no allocation: it can be captured in a hipGraph and replayed with
 * new chunk contents (one graph per chunk length).  Pushes on one state must be ordered
 * (one stream). */
melt_status melt_stream_create(melt_plan plan, int32_t n_streams, int32_t max_chunk_len,
                               melt_stream_state *out);
melt_status melt_stream_destroy(melt_stream_state st);
melt_status melt_stream_reset(melt_stream_state st, void *stream);
int32_t     melt_stream_max_frames(melt_stream_state st);
melt_status melt_stream_push(melt_stream_state st, const float *d_chunk, int32_t chunk_len, float *d_out,
                             int32_t *d_frames_emitted, void *stream);

/* Autotuning: times every kernel variant and launch size of melt_forward that applies to
 * this plan on a synthetic batch of total_frames frames (allocated and freed inside the
 * call; synchronises the device), keeps the fastest for later calls on the plan, and
 * records it in the JSON cache file named by the environment variable
 * MELT_AUTOTUNE_CACHE if set (entries keyed by precision, n_fft, hop, n_mels and device
 * name; melt_plan_create applies a matching entry).  Writes a one-line description of
 * the winner to `desc` (host, desc_len bytes, may be NULL). */
melt_status melt_autotune(melt_plan plan, int64_t total_frames, char *desc, int32_t desc_len);

/* Kernel variants of melt_forward for this plan's precision and geometry (the kernels that
 * can run it: staging scheme, frames per chunk).  melt_variant_count returns how many
 * there are (at least 1); melt_variant_name names variant v ("none" if v is out of
 * range; thread-local text, valid until the thread's next call); melt_set_variant pins variant v with grid_per_cu
 * workgroups per compute unit (0 = the kernel's default) for later forward, backward and
 * prepare calls on the plan.  Variant 0 with the default grid is chosen at plan creation;
 * melt_autotune overrides it.  A batch prepared before the change keeps the variant it was
 * prepared with, and so does a streaming state.  Error: MELT_E_INVALID_ARG for a v or
 * grid_per_cu out of range. */
int32_t     melt_variant_count(melt_plan plan);
const char *melt_variant_name(melt_plan plan, int32_t v);
melt_status melt_set_variant(melt_plan plan, int32_t v, int32_t grid_per_cu);

/* Human-readable name of a status; thread-local text of the last error. */
const char *melt_status_string(melt_status s);
const char *melt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MELT_H */
