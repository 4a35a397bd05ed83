// Host-side launchers of the device passes (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace litho {

using cf2 = float2;

// Geometry of one launch sequence (one focus plane of one chunk of clips).
struct PassGeo {
  int N = 0;      // grid side
  int Q = 0;      // side of the per-kernel transform grid (Q >= 4b + 1, or Q == N)
  int b = 0, B = 0, Bp = 0, nt = 0;   // field band |f| <= b, side, padded side, tiles
  int D = 0, Dp = 0, ntD = 0;         // intensity band |f| <= 2b: side 4b + 1, padded, tiles
  int K = 0;      // kernels used per plane
  int Kbank = 0;  // kernels stored per plane
  int P = 1, p = 0;
  int KC = 1, kper = 1;  // k-chunks of the adjoint column pass
  double dose = 1.0, slope = 0.0, thr = 0.0;
  double pw = 1.0;       // weight of the current plane's loss
  int loss_l1 = 0;       // 1: |Z - T| loss, 0: (Z - T)^2
};

// Outputs of the image epilogue.
struct EpiPtrs {
  float *image = nullptr;         // [clip][P][N][N] or nullptr
  const float *target = nullptr;  // [clip][N][N]; nullptr: no resist / loss / residual
  float *G = nullptr;             // [clip][N][N] residual dL/dI
  double *loss_part = nullptr;    // [clip][P][blocks]
};

constexpr int kTileCols = 4;

// Kernel-launch tracing (HIP events around each launch while enabled).
void prof_begin(const char *name, hipStream_t s);
void prof_end(const char *name, hipStream_t s);

// Threads per transform of length L (0 if L has no FFT plan).
int pass_threads(int L);
// Per-pass twiddle table of the length-L plan (see fft.hpp).
int twiddle_table(int L, std::vector<float2> &out);

int run_rows_fwd_real(const char *name, int L, const float *in, size_t in_clip, cf2 *out, int h, int Wp,
                      const cf2 *tw, float scale, int nclips, hipStream_t s);
int run_rows_inv_real(const char *name, int L, const cf2 *in, int h, int Wp, float *out, const EpiPtrs &ep,
                      const PassGeo &g, const cf2 *tw, float scale, int nclips, hipStream_t s);
// The ILT step's row pass on the N grid with the residual kept on chip: image
// band rows (h, Wp) -> image / resist / loss epilogue (ep.target required) ->
// the residual's forward row DFT, its band |gx| <= h stored in place of the
// image band rows.  Loss partials per block as run_rows_inv_real's MODE 1.
int run_rows_image_residual(const char *name, int L, cf2 *band, int h, int Wp, const EpiPtrs &ep,
                            const PassGeo &g, const cf2 *tw, float scale, int nclips, hipStream_t s);
// Same as run_rows_inv_real without epilogue, written as 1 where scale Re v >= thr, else 0.
int run_rows_inv_thresh(const char *name, int L, const cf2 *in, int h, int Wp, float *out, double thr,
                        const cf2 *tw, float scale, int nclips, hipStream_t s);
int run_col_fft(const char *name, int L, int dir, const cf2 *in, cf2 *out, int nt, int in_h, int out_h,
                const cf2 *tw, float scale, int nclips, hipStream_t s);
// Both column transforms of a band resampling between the inner grid Q and
// the clip grid N in one pass (up: Q rows -> band |f| <= h -> N rows; down:
// N rows -> band -> Q rows), with the resist Gaussian on the band when
// blur_sigma_px > 0.  Only for the pairs col_resample_ok accepts.
bool col_resample_ok(int Q, int N);
int run_col_resample(const char *name, int Q, int N, bool up, const cf2 *in, cf2 *out, int nt, int h,
                     const cf2 *twQ, const cf2 *twN, float scale, double blur_sigma_px, int nclips, hipStream_t s);
int run_pass_y_fwd(const cf2 *bank, const cf2 *Mh, cf2 *Y, const PassGeo &g, const cf2 *twQ, int nclips,
                   hipStream_t s);
int run_pass_x_fwd(const cf2 *Y, const EpiPtrs &ep, cf2 *Ib, const PassGeo &g, const cf2 *twQ, int nclips,
                   hipStream_t s);
int run_pass_x_adj(cf2 *Y, const float *G, size_t g_clip_stride, const cf2 *Gband, const PassGeo &g,
                   const cf2 *twQ, int nclips, hipStream_t s);
int run_pass_y_adj(const cf2 *V, const cf2 *bank, double2 *part, const PassGeo &g, const cf2 *twQ, int nclips,
                   hipStream_t s);
int run_grad_cols(const double2 *part, int nparts, cf2 *tmp, const PassGeo &g, const cf2 *twN, int nclips,
                  hipStream_t s);
int run_loss_reduce(const double *part, int n_per_clip, double *loss, int nclips, hipStream_t s);

// Split-precision band DFT-GEMM form of the forward column pass (matrix cores).
// Forward row pass of the resampled route as two dense DFT stages on the
// matrix cores (split-precision modes; inner grids Q = 32 P, P <= 32, Q < N):
// I_Q rows accumulated from Y_k and their row DFT to the 2b band, as
// run_pass_x_fwd's band output.  tab / twl from fill_row_mfma_table.
bool row_mfma_ok(int Q, int N);
void fill_row_mfma_table(int Q, bool bf16, std::vector<uint16_t> &tab, std::vector<float2> &twl);
int run_pass_x_fwd_mfma(const cf2 *Y, cf2 *Ib, const PassGeo &g, const void *tab, const cf2 *twl, const cf2 *twQ,
                        int prec, int nclips, hipStream_t s);
int run_pass_y_fwd_mfma(const cf2 *bank, const cf2 *Mh, cf2 *Y, const PassGeo &g, const void *tab, int prec,
                        int nclips, hipStream_t s);
// B-operand table of that GEMM for inner grid Q and band half-width b (FP16 or BF16 bits).
void fill_band_table(int Q, int b, bool bf16, std::vector<uint16_t> &out);
// Split-precision GEMM form of the adjoint column pass (g.KC / g.kper chunk the
// kernels as for run_pass_y_adj), and the B-operand table of its GEMM.
int run_pass_y_adj_mfma(const cf2 *V, const cf2 *bank, double2 *part, const PassGeo &g, const void *tab, int prec,
                        int nclips, hipStream_t s);
void fill_adj_table(int Q, int b, bool bf16, std::vector<uint16_t> &out);
// Workgroups of that GEMM per clip and kernel chunk.
int adj_gemm_blocks(int Bp, int B);

}  // namespace litho
