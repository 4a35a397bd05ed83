// C ABI of the steps after the image: Gaussian low-pass / resist blur,
// contours, edge placement error through focus and the Eq. 9 input channels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "litho_internal.hpp"
#include "post.hpp"

namespace litho {
namespace {

// Count and offset arrays of the compaction passes, per (device, stream),
// grown on demand and kept for the life of the process.
struct Scratch {
  int *base = nullptr;
  size_t ints = 0;
};
std::mutex g_scr_mu;
std::map<std::pair<int, hipStream_t>, Scratch> g_scr;

int acquire_scratch(hipStream_t s, size_t ints, int **out) {
  int dev = 0;
  LITHO_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scr_mu);
  Scratch &sc = g_scr[{dev, s}];
  if (sc.ints < ints) {
    if (sc.base) {
      LITHO_HIP_TRY(hipStreamSynchronize(s));
      LITHO_HIP_TRY(hipFree(sc.base));
      sc.base = nullptr;
      sc.ints = 0;
    }
    if (hipMalloc(&sc.base, ints * sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("litho: cannot allocate %zu bytes of compaction scratch", ints * sizeof(int));
      return LITHO_E_NOMEM;
    }
    sc.ints = ints;
  }
  *out = sc.base;
  return LITHO_OK;
}

// Band half-width of the Gaussian low-pass: the transfer function
// exp(-2 pi^2 s^2 f^2 / n^2) is below 1e-12 beyond it (1.1832 is
// sqrt(ln(1e12) / (2 pi^2)) rounded up in the fourth decimal), capped below
// the Nyquist frequency.
int lowpass_band(int n, double sigma_px) {
  const double h = std::ceil(1.1832 * double(n) / sigma_px);
  return int(std::min<double>(n / 2 - 1, h));
}

// N^2 * sum_k conj(c_k) sqrt(lambda_k) Phi_k(f), c_k = dose * sqrt(lambda_k) phi_k(0) with
// phi_k(0) = N^-2 sum_f Phi_k(f): the combined kernel whose field gives
// dI(r)/dm(r) = 2 Re[IDFT(Psi * DFT(m))](r), in the tiled band layout (FP64).
int sensitivity_kernel(litho_bank *bk, int plane, int K_use, const double2 **out) {
  std::lock_guard<std::mutex> lk(bk->mu);
  double2 *&d = bk->psi[{plane, K_use}];
  if (!d) {
    const HostBank &h = bk->host;
    const size_t BB = size_t(h.B) * h.B;
    const double NN = double(h.n) * double(h.n);
    std::vector<cd> psi(BB, cd(0.0, 0.0));
    for (int k = 0; k < K_use; ++k) {
      const cd *ph = &h.phi[(size_t(plane) * h.K + k) * BB];
      const double sl = std::sqrt(h.lambda[size_t(plane) * h.K + k]);
      cd sum(0.0, 0.0);
      for (size_t i = 0; i < BB; ++i) sum += ph[i];
      const cd c = h.dose * sl * sum / NN;
      const cd w = std::conj(c) * sl * NN;
      for (size_t i = 0; i < BB; ++i) psi[i] += w * ph[i];
    }
    std::vector<double2> tiles(size_t(bk->nt) * h.B * kTileCols, make_double2(0.0, 0.0));
    for (int r = 0; r < h.B; ++r)
      for (int j = 0; j < h.B; ++j) {
        const cd v = psi[size_t(r) * h.B + j];
        tiles[(size_t(j / kTileCols) * h.B + r) * kTileCols + (j % kTileCols)] = make_double2(v.real(), v.imag());
      }
    double2 *p = nullptr;
    if (hipMalloc(&p, tiles.size() * sizeof(double2)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("litho_ai_channels: cannot allocate the sensitivity kernel");
      return LITHO_E_NOMEM;
    }
    if (hipMemcpy(p, tiles.data(), tiles.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(p);
      set_error("litho_ai_channels: cannot upload the sensitivity kernel");
      return LITHO_E_HIP;
    }
    d = p;
  }
  *out = d;
  return LITHO_OK;
}

}  // namespace
}  // namespace litho

using namespace litho;

extern "C" int litho_lowpass(const litho_bank_t *bank, const float *d_in, int count, double sigma_px,
                             double threshold, float *d_out, void *hip_stream) {
  clear_error();
  if (!bank || count < 0 || (count > 0 && (!d_in || !d_out))) {
    set_error("litho_lowpass: NULL bank, image or output, or negative count");
    return LITHO_E_INVALID;
  }
  if (!(sigma_px > 0.0) || !std::isfinite(sigma_px)) {
    set_error("litho_lowpass: sigma_px must be positive and finite");
    return LITHO_E_INVALID;
  }
  if (count == 0) return LITHO_OK;
  litho_bank *bk = const_cast<litho_bank *>(bank);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int N = bk->host.n, h = lowpass_band(N, sigma_px), H = 2 * h + 1;
  const int Hp = (H + kTileCols - 1) / kTileCols * kTileCols, nt = Hp / kTileCols;
  const size_t NN = size_t(N) * N;
  const size_t per = (size_t(nt) * N * kTileCols + size_t(nt) * H * kTileCols) * sizeof(float2);
  const int chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(count), workspace_limit_bytes() / per)));
  char *ws = nullptr;
  LITHO_TRY(acquire_aux(bk, s, per * size_t(chunk), &ws));
  float2 *X1 = reinterpret_cast<float2 *>(ws);
  float2 *X2 = X1 + size_t(chunk) * nt * N * kTileCols;
  for (int c0 = 0; c0 < count; c0 += chunk) {
    const int c = std::min(chunk, count - c0);
    LITHO_TRY(run_rows_fwd_real("lowpass_rows", N, d_in + c0 * NN, NN, X1, h, Hp, bk->d_twN,
                                float(1.0 / (double(N) * double(N))), c, s));
    LITHO_TRY(run_col_fft("lowpass_cols_fwd", N, -1, X1, X2, nt, -1, h, bk->d_twN, 1.0f, c, s));
    LITHO_TRY(run_band_gauss(X2, h, nt, double(N), sigma_px, size_t(nt) * H * kTileCols, c, s));
    LITHO_TRY(run_col_fft("lowpass_cols_inv", N, +1, X2, X1, nt, h, -1, bk->d_twN, 1.0f, c, s));
    if (std::isnan(threshold)) {
      LITHO_TRY(run_rows_inv_real("lowpass_rows_inv", N, X1, h, Hp, d_out + c0 * NN, EpiPtrs{}, PassGeo{},
                                  bk->d_twN, 1.0f, c, s));
    } else {
      LITHO_TRY(run_rows_inv_thresh("lowpass_rows_thr", N, X1, h, Hp, d_out + c0 * NN, threshold, bk->d_twN, 1.0f,
                                    c, s));
    }
  }
  return LITHO_OK;
}

extern "C" int litho_contours(int n, const float *d_image, double level, int capacity, int *d_cell, int *d_code,
                              float *d_u, int *d_next, int *d_count, void *hip_stream) {
  clear_error();
  if (n < 2 || n > 4096) {
    set_error("litho_contours: n=%d outside 2..4096", n);
    return LITHO_E_UNSUPPORTED;
  }
  if (!d_image || !d_count || capacity < 0 || (capacity > 0 && (!d_cell || !d_code || !d_u || !d_next))) {
    set_error("litho_contours: NULL image or count, negative capacity, or NULL outputs with capacity > 0");
    return LITHO_E_INVALID;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t m = size_t(n) * compaction_chunks(n);
  int *scr = nullptr;
  LITHO_TRY(acquire_scratch(s, 2 * m + 1, &scr));
  return run_contours(d_image, n, float(level), scr, scr + m, d_count, capacity, d_cell, d_code, d_u, d_next, s);
}

extern "C" int litho_contours_noalloc(int n, const float *d_image, double level, int capacity, int *d_cell,
                                      int *d_code, float *d_u, int *d_next, int *d_count, void *hip_stream) {
  clear_error();
  if (n < 2 || n > noalloc_max_n()) {
    set_error("litho_contours_noalloc: n=%d outside 2..%d (the static scratch is sized for %d)", n, noalloc_max_n(),
              noalloc_max_n());
    return LITHO_E_UNSUPPORTED;
  }
  if (!d_image || !d_count || capacity < 0 || (capacity > 0 && (!d_cell || !d_code || !d_u || !d_next))) {
    set_error("litho_contours_noalloc: NULL image or count, negative capacity, or NULL outputs with capacity > 0");
    return LITHO_E_INVALID;
  }
  int *scr = nullptr;
  size_t ints = 0;
  LITHO_TRY(noalloc_scratch(&scr, &ints));
  const size_t m = size_t(n) * compaction_chunks(n);
  if (2 * m + 1 > ints) {
    set_error("litho_contours_noalloc: %zu scratch ints needed, %zu available", 2 * m + 1, ints);
    return LITHO_E_UNSUPPORTED;
  }
  // every count and offset the passes read is written by them first: nothing to clear
  return run_contours(d_image, n, float(level), scr, scr + m, d_count, capacity, d_cell, d_code, d_u, d_next,
                      static_cast<hipStream_t>(hip_stream));
}

extern "C" int litho_epe(int n, const float *d_target, const float *d_latent, int n_planes,
                         const litho_epe_rule_t *rule, int capacity, int *d_site, int *d_dir, float *d_epe,
                         int *d_count, void *hip_stream) {
  clear_error();
  if (n < 2 || n > 4096) {
    set_error("litho_epe: n=%d outside 2..4096", n);
    return LITHO_E_UNSUPPORTED;
  }
  if (!d_target || !d_latent || !rule || !d_count || n_planes < 1 || n_planes > 8 || capacity < 0 ||
      (capacity > 0 && (!d_site || !d_dir || !d_epe))) {
    set_error("litho_epe: NULL argument, n_planes outside 1..8, or NULL outputs with capacity > 0");
    return LITHO_E_INVALID;
  }
  if (rule->f0 < 0 || rule->f0 >= n_planes || !(rule->tol_neg <= 0.0) || !(rule->tol_pos >= 0.0)) {
    set_error("litho_epe: f0 outside the planes or tolerances of the wrong sign");
    return LITHO_E_INVALID;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  EpeRule r;
  r.t_eff = float(rule->t_eff);
  r.tol_neg = float(rule->tol_neg);
  r.tol_pos = float(rule->tol_pos);
  r.f0 = rule->f0;
  const size_t m = size_t(n) * compaction_chunks(n);
  int *scr = nullptr;
  LITHO_TRY(acquire_scratch(s, 2 * m + 1, &scr));
  return run_epe(d_target, d_latent, n, n_planes, r, scr, scr + m, d_count, capacity, d_site, d_dir, d_epe, s);
}

extern "C" int litho_ai_channels(const litho_bank_t *bank, const float *d_layout, int batch, int K_use, int plane,
                                 const double *h_norm, float *d_out, void *hip_stream) {
  clear_error();
  if (!bank || batch < 0 || (batch > 0 && (!d_layout || !d_out))) {
    set_error("litho_ai_channels: NULL bank, layout or output, or negative batch");
    return LITHO_E_INVALID;
  }
  litho_bank *bk = const_cast<litho_bank *>(bank);
  const HostBank &hb = bk->host;
  if (K_use < 1 || K_use > hb.K || plane < 0 || plane >= hb.n_focus) {
    set_error("litho_ai_channels: K_use=%d or plane=%d out of range", K_use, plane);
    return LITHO_E_INVALID;
  }
  ChanNorm nm;
  if (h_norm) {
    nm.on = 1;
    for (int c = 0; c < 3; ++c) {
      const double lo = h_norm[2 * c], hi = h_norm[2 * c + 1];
      if (!(hi > lo)) {
        set_error("litho_ai_channels: normalisation range %d has hi <= lo", c);
        return LITHO_E_INVALID;
      }
      nm.lo[c] = float(lo);
      nm.inv[c] = float(1.0 / (hi - lo));
    }
  }
  if (batch == 0) return LITHO_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const double2 *psi = nullptr;
  LITHO_TRY(sensitivity_kernel(bk, plane, K_use, &psi));
  const CallLayout L = plan_call(bk, 1, K_use, false, false, LITHO_PREC_FP32);
  const PassGeo &g = L.g;
  const int N = g.N, P = g.P;
  const size_t NN = size_t(N) * N;
  const size_t band = size_t(g.nt) * g.B * kTileCols;      // complex values of one B x B band
  const size_t rowsb = size_t(g.nt) * N * kTileCols;       // complex values of N band rows
  const size_t per = size_t(P) * NN * sizeof(float) + NN * sizeof(float) + band * sizeof(double2) +
                     rowsb * sizeof(float2) + band * sizeof(float2);
  const int chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(batch), workspace_limit_bytes() / per)));
  char *ws = nullptr;
  LITHO_TRY(acquire_aux(bk, s, per * size_t(chunk), &ws));
  float *img = reinterpret_cast<float *>(ws);
  float *sens = img + size_t(chunk) * P * NN;
  double2 *part = reinterpret_cast<double2 *>(sens + size_t(chunk) * NN);
  float2 *rows = reinterpret_cast<float2 *>(part + size_t(chunk) * band);
  float2 *mh = rows + size_t(chunk) * rowsb;
  for (int c0 = 0; c0 < batch; c0 += chunk) {
    const int c = std::min(chunk, batch - c0);
    const float *zt = d_layout + size_t(c0) * NN;
    // I0: the image of the layout at the chosen focus plane (Eq. 4)
    LITHO_TRY(image_grad_impl(bk, zt, c, K_use, nullptr, nullptr, nullptr, img, nullptr, nullptr, false,
                              LITHO_PREC_FP32, s, plane, plane + 1));
    // dI/dM: 2 Re IDFT(Psi * DFT(Z_t)) on the pupil band
    LITHO_TRY(run_rows_fwd_real("mask_rows", N, zt, NN, rows, g.b, g.Bp, bk->d_twN,
                                float(1.0 / (double(N) * double(N))), c, s));
    LITHO_TRY(run_col_fft("mask_cols", N, -1, rows, mh, g.nt, -1, g.b, bk->d_twN, 1.0f, c, s));
    LITHO_TRY(run_band_mul_psi(psi, mh, band, part, c, s));
    LITHO_TRY(run_grad_cols(part, 1, rows, g, bk->d_twN, c, s));
    LITHO_TRY(run_rows_inv_real("sens_rows", N, rows, g.b, g.Bp, sens, EpiPtrs{}, g, bk->d_twN, 2.0f, c, s));
    LITHO_TRY(run_channels(zt, img + size_t(plane) * NN, size_t(P) * NN, sens, N, nm, d_out + size_t(c0) * NN * 3,
                           c, s));
  }
  return LITHO_OK;
}

// ---------------------------------------------------------------- layouts beyond one clip
namespace litho {
namespace {

int tile_plan(const litho_bank *bk, int H, int W, int halo, TileGeo &g, const char *who) {
  const int n = bk->host.n;
  if (H < 1 || W < 1 || halo < 0 || n - 2 * halo < 1) {
    set_error("%s: need H, W >= 1 and 0 <= halo with a core n - 2 halo >= 1 (n=%d, halo=%d)", who, n, halo);
    return LITHO_E_INVALID;
  }
  g.H = H;
  g.W = W;
  g.n = n;
  g.halo = halo;
  g.c = n - 2 * halo;
  g.ty = (H + g.c - 1) / g.c;
  g.tx = (W + g.c - 1) / g.c;
  if (size_t(g.ty) * g.tx > size_t(1) << 24) {
    set_error("%s: %d x %d tiles exceed the supported 2^24", who, g.ty, g.tx);
    return LITHO_E_UNSUPPORTED;
  }
  return LITHO_OK;
}

}  // namespace
}  // namespace litho

extern "C" int litho_image_tiled(const litho_bank_t *bank, const float *d_layout, int H, int W, int halo, int K_use,
                                 float *d_image, int prec, void *hip_stream) {
  clear_error();
  if (!bank || !d_layout || !d_image) {
    set_error("litho_image_tiled: NULL bank, layout or image");
    return LITHO_E_INVALID;
  }
  litho_bank *bk = const_cast<litho_bank *>(bank);
  if (K_use < 1 || K_use > bk->host.K) {
    set_error("litho_image_tiled: K_use=%d outside 1..%d", K_use, bk->host.K);
    return LITHO_E_INVALID;
  }
  LITHO_TRY(check_prec(prec, "litho_image_tiled"));
  TileGeo g;
  LITHO_TRY(tile_plan(bk, H, W, halo, g, "litho_image_tiled"));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int P = bk->host.n_focus, T = g.ty * g.tx;
  const size_t nn = size_t(g.n) * g.n;
  const size_t per = (nn + size_t(P) * nn) * sizeof(float);
  const int chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(T), workspace_limit_bytes() / per)));
  char *ws = nullptr;
  LITHO_TRY(acquire_aux(bk, s, per * size_t(chunk), &ws));
  float *masks = reinterpret_cast<float *>(ws), *timg = masks + size_t(chunk) * nn;
  for (int t0 = 0; t0 < T; t0 += chunk) {
    const int cnt = std::min(chunk, T - t0);
    g.t0 = t0;
    LITHO_TRY(run_tile_gather(d_layout, g, cnt, masks, s));
    LITHO_TRY(image_grad_impl(bk, masks, cnt, K_use, nullptr, nullptr, nullptr, timg, nullptr, nullptr, false, prec,
                              s));
    LITHO_TRY(run_tile_cores(timg, P, g, cnt, d_image, s));
  }
  return LITHO_OK;
}

extern "C" int litho_image_grad_tiled(const litho_bank_t *bank, const float *d_layout, int H, int W, int halo,
                                      int K_use, const float *d_target, const litho_resist_t *resist,
                                      float *d_image, double *d_loss, float *d_grad, int prec, void *hip_stream) {
  clear_error();
  if (!bank || !d_layout || !d_target || !resist || !d_grad) {
    set_error("litho_image_grad_tiled: NULL bank, layout, target, resist or gradient");
    return LITHO_E_INVALID;
  }
  litho_bank *bk = const_cast<litho_bank *>(bank);
  if (K_use < 1 || K_use > bk->host.K) {
    set_error("litho_image_grad_tiled: K_use=%d outside 1..%d", K_use, bk->host.K);
    return LITHO_E_INVALID;
  }
  if (resist->blur_sigma_px != 0.0 || (resist->loss != LITHO_LOSS_L2 && resist->loss != LITHO_LOSS_L1)) {
    set_error("litho_image_grad_tiled: a resist blur is not supported on tiled layouts; loss must be L2 or L1");
    return LITHO_E_UNSUPPORTED;
  }
  LITHO_TRY(check_prec(prec, "litho_image_grad_tiled"));
  TileGeo g;
  LITHO_TRY(tile_plan(bk, H, W, halo, g, "litho_image_grad_tiled"));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int P = bk->host.n_focus, T = g.ty * g.tx, nblk = tile_residual_blocks(g.n);
  if (size_t(T) * P * nblk >= (size_t(1) << 31)) {
    set_error("litho_image_grad_tiled: %d tiles x %d planes of loss partials exceed 2^31", T, P);
    return LITHO_E_UNSUPPORTED;
  }
  TileLoss lo;
  lo.slope = float(resist->slope);
  lo.thr = float(resist->threshold);
  lo.l1 = resist->loss == LITHO_LOSS_L1 ? 1 : 0;
  for (int p = 0; p < P; ++p) lo.w[p] = resist->plane_weight ? float(resist->plane_weight[p]) : 1.f;
  const size_t nn = size_t(g.n) * g.n;
  // per tile: window mask, images and residuals of every plane, window gradient
  const size_t per = (2 * nn + 2 * size_t(P) * nn) * sizeof(float);
  const size_t parts = (size_t(T) * P * nblk * sizeof(double) + 255) & ~size_t(255);
  const size_t lim = workspace_limit_bytes();
  const int chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(T), (lim > parts ? lim - parts : 0) / per)));
  char *ws = nullptr;
  LITHO_TRY(acquire_aux(bk, s, parts + per * size_t(chunk), &ws));
  double *part = reinterpret_cast<double *>(ws);
  float *masks = reinterpret_cast<float *>(ws + parts);
  float *timg = masks + size_t(chunk) * nn;
  float *G = timg + size_t(chunk) * P * nn;
  float *tgrad = G + size_t(chunk) * P * nn;
  LITHO_TRY(run_fill(d_grad, size_t(H) * W, 0.f, s));
  for (int t0 = 0; t0 < T; t0 += chunk) {
    const int cnt = std::min(chunk, T - t0);
    g.t0 = t0;
    LITHO_TRY(run_tile_gather(d_layout, g, cnt, masks, s));
    LITHO_TRY(image_grad_impl(bk, masks, cnt, K_use, nullptr, nullptr, nullptr, timg, nullptr, nullptr, false, prec,
                              s));
    if (d_image) LITHO_TRY(run_tile_cores(timg, P, g, cnt, d_image, s));
    LITHO_TRY(run_tile_residual(timg, d_target, P, g, lo, cnt, G, part + size_t(t0) * P * nblk, s));
    LITHO_TRY(image_grad_impl(bk, masks, cnt, K_use, nullptr, nullptr, G, nullptr, nullptr, tgrad, true, prec, s));
    LITHO_TRY(run_tile_grad_add(tgrad, g, cnt, d_grad, s));
  }
  if (d_loss) LITHO_TRY(run_loss_reduce(part, T * P * nblk, d_loss, 1, s));
  return LITHO_OK;
}
