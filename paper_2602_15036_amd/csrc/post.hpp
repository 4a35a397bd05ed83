// Host-side launchers of the post-image kernels (implemented in post.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "kernels.hpp"

namespace litho {

// Eq. 8's through-focus rule and Eq. 6's iso-level.
struct EpeRule {
  float t_eff = 0.f;     // E_tgt on the target edge
  float tol_neg = 0.f;   // lower tolerance (<= 0)
  float tol_pos = 0.f;   // upper tolerance (>= 0)
  int f0 = 0;            // index of the on-focus plane
};

// Per-channel affine map to [0, 1] of the Eq. 9 channels.
struct ChanNorm {
  int on = 0;
  float lo[3] = {0.f, 0.f, 0.f};
  float inv[3] = {1.f, 1.f, 1.f};
};

// Halo tiling of an H x W layout into n x n windows (core c = n - 2 halo,
// ty x tx tiles); t0 is the first tile of the current chunk.
struct TileGeo {
  int H = 0, W = 0, n = 0, halo = 0, c = 0, ty = 0, tx = 0, t0 = 0;
};

// Resist and loss of the tiled gradient.
struct TileLoss {
  float slope = 0.f, thr = 0.f;
  int l1 = 0;
  float w[8] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};  // plane weights
};

int run_tile_gather(const float *layout, const TileGeo &g, int cnt, float *out, hipStream_t s);
int run_tile_cores(const float *timg, int P, const TileGeo &g, int cnt, float *img, hipStream_t s);
int tile_residual_blocks(int n);
int run_tile_residual(const float *timg, const float *target, int P, const TileGeo &g, const TileLoss &lo, int cnt,
                      float *G, double *part, hipStream_t s);
int run_tile_grad_add(const float *tg, const TileGeo &g, int cnt, float *grad, hipStream_t s);
int run_fill(float *a, size_t n, float v, hipStream_t s);

// Chunks of 64 columns per row in the compaction passes (contours, EPE sites).
int compaction_chunks(int n);

// Largest image side of the allocation-free contour entry point, and this
// device's address (and size in ints) of the static scratch it uses.
int noalloc_max_n();
int noalloc_scratch(int **out, size_t *ints);

// Marching squares of one n x n image at `level`.  cnt: [n * chunks] scratch,
// off: [n * chunks + 1] scratch, total: device int receiving the segment count.
// Segments with index >= cap are not written.
int run_contours(const float *img, int n, float level, int *cnt, int *off, int *total, int cap, int *cell,
                 int *code, float *u, int *next, hipStream_t s);

// Edge placement error at the target's edge sites for P latent images E [P][n][n].
int run_epe(const float *target, const float *E, int n, int P, const EpeRule &rule, int *cnt, int *off,
            int *total, int cap, int *site, int *dir, float *epe, hipStream_t s);

// Gaussian transfer function of std sigma_px on an N-grid band of half-width h
// ([nt][2h+1][4] complex per clip, clips clip_stride complex values apart).
int run_band_gauss(float2 *band, int h, int nt, double N, double sigma_px, size_t clip_stride, int nclips,
                   hipStream_t s);

// part = psi * Mh per clip (per = complex values of one band).
int run_band_mul_psi(const double2 *psi, const float2 *mh, size_t per, double2 *part, int nclips, hipStream_t s);

// Channel-last Eq. 9 tensor from the layout, its image and dI/dM.
int run_channels(const float *zt, const float *img, size_t img_clip, const float *sens, int n, const ChanNorm &nm,
                 float *out, int nclips, hipStream_t s);

}  // namespace litho
