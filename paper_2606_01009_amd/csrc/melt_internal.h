// Internal declarations of libmelt: the plan object, the chunk schedule and the
// kernel launchers.  Nothing here is part of the C ABI (include/melt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/melt.h"

namespace melt {

// ---------------------------------------------------------------- chunk schedule
// A chunk is up to `bf` consecutive frames of one clip; the persistent kernels walk a
// table of chunks so that a ragged batch is one launch.
struct Chunk {
    int64_t sample_start;  // first sample of the chunk's first frame
    int64_t sample_end;    // end of its clip (exclusive): samples at or past it read as 0
    int64_t out_row;       // output row of the chunk's first frame
    int32_t n_frames;      // frames in this chunk (1..bf)
    int32_t clip;          // clip index
};
static_assert(sizeof(Chunk) == 32, "Chunk layout");

// Hop-block geometry: a frame of N samples starting at t*H is the concatenation of
// segments j = 0..J-1 of length L_j = min(H, N - jH), segment j being the first L_j
// samples of hop-block row t + j (row r = samples [rH, rH + H)).  Each segment is padded
// to a multiple of the k-group of the GEMM (8 for FP32, 16 for 16-bit, 64 for FP8) with
// zero basis columns, so a k-group never straddles two rows.
struct Geometry {
    int N, H, J;         // frame length, hop, hop-block segments per frame
    int group;           // k-group size
    int Hp;              // padded row length used in LDS (multiple of `group`)
    int n_groups;        // total k-groups over all segments
    std::vector<int> seg_of_group, col_of_group;  // segment and first column of each group
};
Geometry make_geometry(int N, int H, int group);

// per-launch descriptor of the k-groups, passed by value (kernel argument)
constexpr int kMaxGroups = 160;
struct GroupTable {
    int n;                   // number of groups
    int lds_off[kMaxGroups]; // element offset in LDS of group g relative to a frame's row
};

// ---------------------------------------------------------------- plan
struct Plan {
    melt_config cfg{};
    int device = 0;
    int M = 0, N = 0, H = 0;
    int row_tiles = 0;                 // ceil(M / 16): 16 Mel bins (32 basis rows) per tile
    std::vector<double> freqs;         // f_m, Hz
    std::vector<double> basis64;       // stacked [2M][N]: cos rows then sin rows (FP64)
    // device memory (owned)
    float *d_basis32 = nullptr;        // stacked [2M][N] FP32 (the learnable parameter)
    void *d_pack_f32 = nullptr;        // FP32 fragment-packed basis (frame-split kernel)
    void *d_pack_h16 = nullptr;        // 16-bit packed basis (BF16 or FP16)
    void *d_pack_lo = nullptr;         // BF16x3 low part
    void *d_pack_f8 = nullptr;         // FP8 E4M3 packed basis
    float *d_rowscale = nullptr;       // FP8 per-row scales (packed row order)
    Geometry geo32, geo16, geo8;
    int *d_seg32 = nullptr, *d_col32 = nullptr;   // segment / first column of each k-group (device)
    int *d_seg16 = nullptr, *d_col16 = nullptr;
    // comparator (FFT + CSR filterbank)
    float *d_fb_w = nullptr;           // filter weights, concatenated per Mel bin
    int *d_fb_start = nullptr;         // first bin of each filter
    int *d_fb_off = nullptr;           // offset of each filter's weights [M+1]
    int fb_nnz = 0;
    float2 *d_twiddle = nullptr;       // exp(-2 pi i j / N), j < N
    float *d_window = nullptr;         // analysis window [N]
    // workspace: chunk tables of the MelT kernels (0) and of the comparator (1)
    Chunk *d_chunks[2] = {nullptr, nullptr};
    int *d_nchunks = nullptr;          // [2]
    int64_t chunk_cap[2] = {0, 0};
    int64_t prepared_frames[2] = {-1, -1};   // n_frames of the batch each table describes
    int prepared_variant = 0;                // kernel variant table 0 was built for
    int prepared_bf[2] = {128, 32};          // frames per chunk of each table
    int prepared_clips[2] = {0, 0};          // clips of the batch each table describes
    // backward: dx basis layout and workspaces (grown on demand)
    void *d_pack_dx = nullptr;
    size_t pack_dx_cap = 0;
    void *d_bwd_ws = nullptr;
    size_t bwd_ws_cap = 0;
    void *d_bwd_rows = nullptr;
    size_t bwd_rows_cap = 0;
    // MFCCT: the K x M DCT-II (device) and the log-Mel workspace it reads (grown on demand)
    int K = 0;                         // cepstral coefficients (MELT_OUT_MFCC), else 0
    int kern_out = 0;                  // output map of the Mel kernels (log power under MFCC)
    float *d_dct = nullptr;
    void *d_dct_x3 = nullptr;          // its split binary16 fragments (16-bit / FP8 plans, K <= 64)
    float *d_lmel = nullptr;
    size_t lmel_cap = 0;
    // kernel variants of the forward for this plan, fixed at plan creation (init_variants):
    // kind, frames per chunk, span buffers; read without allocating by every forward call
    static constexpr int kMaxVariants = 16;
    int n_variants = 0;
    int var_kind[kMaxVariants] = {}, var_bf[kMaxVariants] = {}, var_nbuf[kMaxVariants] = {};
    // tuning
    int cu_count = 256;
    int tune_variant = 0;                          // index of the chosen kernel variant
    int tune_grid = 0;                             // workgroups per CU (0 = kernel default)
    std::string last_tune;
};

// compensated (split) 16-bit precisions: a high and a low part per operand, three products
inline bool prec_split(const Plan &p) {
    return p.cfg.precision == MELT_PREC_BF16X3 || p.cfg.precision == MELT_PREC_FP16X3;
}
// 16-bit precisions whose operands are binary16
inline bool prec_f16(const Plan &p) {
    return p.cfg.precision == MELT_PREC_FP16 || p.cfg.precision == MELT_PREC_FP16X3;
}
// exact power-of-two pre-scale of the waveform under FP16X3 (keeps the low parts normal)
constexpr float kF16x3Scale = 1024.0f;

// status plumbing (capi.cpp)
melt_status set_error(melt_status s, const std::string &msg);
melt_status hip_check(hipError_t e, const char *what);

// plan construction (plan.cpp)
melt_status plan_build_host(Plan &p);
void mel_frequencies(const melt_config &cfg, std::vector<double> &f);

// kernels (melt_fwd.hip, stft_mel.hip, melt_bwd.hip)
melt_status pack_tables_upload(Plan &p);         // k-group tables of the pack kernels (plan creation)
melt_status pack_basis(Plan &p, hipStream_t s);   // enqueue only: no allocation, no synchronisation
melt_status pack_basis_dx(Plan &p, hipStream_t s);
melt_status ensure_chunks(Plan &p, int which, int64_t needed);
melt_status launch_schedule(Plan &p, int which, const int64_t *d_off, int n_clips, int bf, int64_t n_frames,
                            hipStream_t s);
melt_status launch_frame_offsets(const int64_t *d_off, int n_clips, int N, int H, int64_t *d_fo,
                                 hipStream_t s);
// chunk size (frames) of MelT kernel variant v / of the plan's chosen variant / of the comparator
int melt_chunk_frames(const Plan &p, int variant);
int melt_chunk_frames(const Plan &p);
int stft_chunk_frames(const Plan &p);
int stft_batch_chunk_frames(const Plan &p, int64_t n_frames);   // comparator chunk size for a batch
// main kernels over the batch prepared in table 0 / table 1
melt_status launch_melt_main(Plan &p, const float *d_wave, float *d_out, float *d_proj, hipStream_t s);
melt_status launch_stft_main(Plan &p, const float *d_wave, float *d_out, hipStream_t s);
// main MelT kernel (variant v) over an explicit chunk table built with that variant's chunk
// size (streaming); est_chunks sizes the grid
melt_status launch_melt_table(Plan &p, int variant, const Chunk *tab, const int *n_tab, int64_t est_chunks,
                              int64_t n_frames, const float *d_wave, float *d_out, float *d_proj, hipStream_t s);
void init_variants(Plan &p);             // melt_fwd.hip: fills the plan's variant table
size_t pc_x3_lds_bytes(const Plan &p, int bf);   // melt_h16.hip: split-precision producer/consumer LDS
int forward_variants(const Plan &p);
void apply_tune_cache(Plan &p);          // stream.hip: apply a MELT_AUTOTUNE_CACHE entry
const char *forward_variant_name(const Plan &p, int variant);
melt_status stft_plan_build(Plan &p);
// MFCCT (mfcc.hip): out[r][j] = sum_i in[r][i] A[j sj + i si]; the DCT-II; the workspace
melt_status launch_cepstrum(const Plan &p, const float *lmel, int64_t rows, float *out, hipStream_t s);
melt_status pack_dct_x3(Plan &p);        // plan creation, after the DCT upload
melt_status launch_row_matmul(const float *in, int64_t rows, int I, int J, const float *A, int sj, int si, float *out,
                              hipStream_t s);
void dct_matrix(int K, int M, std::vector<float> &D);
melt_status ensure_lmel(Plan &p, int64_t rows);
// allocation-free forward (melt_fwd.hip): per-device scratch address, and the forward over it
melt_status scratch_init(int device);
melt_status forward_noalloc(Plan &p, const float *d_wave, const int64_t *d_off, int n_clips, int64_t n_frames,
                            float *d_out, hipStream_t s);
melt_status launch_melt_backward(Plan &p, const float *d_wave, const int64_t *d_off, int n_clips,
                                 int64_t n_frames, const float *d_gout, const float *d_proj,
                                 float *d_gwave, float *d_gbasis, hipStream_t s);

}  // namespace melt
