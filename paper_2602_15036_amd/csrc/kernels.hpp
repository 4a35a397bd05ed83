// Host-side launchers of the device passes (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "common.hpp"

namespace litho {

using cf2 = float2;

// Geometry of one launch sequence (one focus plane of one chunk of clips).
struct PassGeo {
  int N = 0;      // grid side
  int Q = 0;      // side of the per-kernel transform grid
  int b = 0, B = 0, Bp = 0, nt = 0;
  int K = 0;      // kernels used per plane
  int Kbank = 0;  // kernels stored per plane
  int P = 1, p = 0;
  int KC = 1, kper = 1;  // k-chunks of the adjoint column pass
  double dose = 1.0, slope = 0.0, thr = 0.0;
};

constexpr int kTileCols = 4;

// Kernel-launch tracing (HIP events around each launch while enabled).
void prof_begin(const char *name, hipStream_t s);
void prof_end(const char *name, hipStream_t s);

int pass_threads(int L);
int run_mask_spectrum(const float *mask, cf2 *S1, cf2 *Mh, const PassGeo &g, const cf2 *twN, int nclips,
                      hipStream_t s);
int run_pass_y_fwd(const cf2 *bank, const cf2 *Mh, cf2 *Y, const PassGeo &g, const cf2 *twQ, int nclips,
                   hipStream_t s);
int run_pass_x_fwd(const cf2 *Y, float *image, const float *target, float *G, double *loss_part,
                   const PassGeo &g, const cf2 *twQ, int nclips, hipStream_t s);
int run_pass_x_adj(cf2 *Y, const float *G, size_t g_clip_stride, const PassGeo &g, const cf2 *twQ, int nclips,
                   hipStream_t s);
int run_pass_y_adj(const cf2 *V, const cf2 *bank, double2 *part, const PassGeo &g, const cf2 *twQ, int nclips,
                   hipStream_t s);
int run_grad_finish(const double2 *part, int nparts, cf2 *tmp, float *grad, const PassGeo &g, const cf2 *twN,
                    int nclips, hipStream_t s);
int run_loss_reduce(const double *part, int n_per_clip, double *loss, int nclips, hipStream_t s);

}  // namespace litho
