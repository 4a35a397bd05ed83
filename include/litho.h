/*
 * litho.h -- C ABI of the MI355X (gfx950) SOCS aerial-image library.
 *
 * The calls follow the paper's statement of the imaging problem (Sec. III-A):
 * a mask m, a normalised source S and a pupil P (NA cut-off plus a defocus
 * aberration per focus plane F) go in; the partially coherent aerial image
 * I(r; F) comes out.  The image is computed in the sum-of-coherent-systems
 * form of Eqs. 3-4,
 *
 *     I(r) = D * sum_k lambda_k |E_k(r)|^2,   E_k = IDFT( Phi_k * DFT(m) ),
 *
 * where {lambda_k, Phi_k} are the leading eigenpairs of the TCC of Eq. 2.
 * The resist is the sigmoid relaxation Z = 1 / (1 + exp(-a (I - t))) of the
 * threshold model of Eqs. 5 and 17 (resist kernel = delta), and the ILT loss is
 * L = sum_planes sum_r (Z - T)^2 against a target layout T.  The adjoint
 * returns dL/dm for the pixel mask (the mask-gradient channel of Eq. 9).
 *
 * Conventions shared by every call:
 *   - Return codes only (LITHO_OK or a negative LITHO_E_*); nothing throws or
 *     aborts across the ABI.  litho_last_error() gives the reason as text
 *     (thread-local, valid until the next call on the same thread).
 *   - Pointers named d_* are caller-owned DEVICE memory (HIP), pointers named
 *     h_* are caller-owned HOST memory.  The library never frees them.
 *   - Arrays are dense, row-major, float32 unless stated: a mask is
 *     [batch][n][n], an image [batch][n_focus][n][n].
 *   - Device calls are asynchronous on the caller's HIP stream (hipStream_t
 *     passed as void*, NULL = the null stream).  Inputs must stay valid, and
 *     outputs untouched, until that stream reaches the end of the call.
 *   - A bank owns device memory (kernels, FFT tables, workspaces) until
 *     litho_kernels_free().  Calls on different streams get separate
 *     workspaces; calls on one stream are ordered by the stream.
 *   - Grid sides n must be 2^j, 3*2^j or 5*2^j with 64 <= n <= 4096
 *     (LITHO_E_UNSUPPORTED otherwise).
 */
#ifndef LITHO_H
#define LITHO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LITHO_OK = 0,
  LITHO_PENDING = 1,         /* serve: result not ready yet */
  LITHO_E_INVALID = -1,      /* bad argument (NULL, size mismatch, out of range) */
  LITHO_E_UNSUPPORTED = -2,  /* valid but not supported (grid side, precision) */
  LITHO_E_NOMEM = -3,        /* device or host allocation failed / over budget */
  LITHO_E_HIP = -4,          /* a HIP runtime call failed */
  LITHO_E_BUSY = -5,         /* serve: queue full */
  LITHO_E_NOTFOUND = -6      /* serve: unknown or already collected ticket */
};

/* Source shapes (Eq. 2's S).  Lattice sources are sampled on a G x G lattice
 * over [-1, 1]^2 in units of NA with integer coordinates (i, j),
 * sigma = (i, j) / ((G - 1) / 2).  A point is kept when
 * sigma_in^2 h^2 <= i^2 + j^2 <= sigma_out^2 h^2 with h = (G - 1) / 2; the
 * x-dipole also requires |j| <= |i|, the y-dipole |i| <= |j|.  Kept points
 * weigh the same and the weights sum to one.  LITHO_SRC_POINTS takes the
 * caller's samples (optics.src_points); their weights are normalised to sum
 * one. */
enum { LITHO_SRC_ANNULAR = 0, LITHO_SRC_DIPOLE_X = 1, LITHO_SRC_DIPOLE_Y = 2, LITHO_SRC_POINTS = 3 };

/* Arithmetic of the DFT stages that run on the matrix cores (every other
 * pass stays FP32, and loss and gradient reductions stay FP64).
 *   FP32:        FFT passes in FP32.
 *   F16X3/BF16X3: dense DFT stages on the matrix cores, FP16 / BF16 operands
 *                split into hi + lo halves, products hi*hi + hi*lo + lo*hi,
 *                FP32 accumulation.  On inner grids 32 P <= 1024 of the
 *                resampled route the band-limited inverse row transform of
 *                the forward pass runs as two such stages (a 16 -> 32 DFT
 *                and a P-point DFT around an FP32 twiddle) and the column
 *                passes stay FP32; on the other inner grids the column
 *                transforms between the pupil band and the inner grid run as
 *                band DFT-GEMMs.  Near-FP32 (F16X3) or ~1e-5 relative
 *                (BF16X3) accuracy.
 *   F16/BF16:    the same stages with one FP16 / BF16 term (hi*hi only);
 *                ~1e-3 relative accuracy. */
enum { LITHO_PREC_FP32 = 0, LITHO_PREC_F16X3 = 1, LITHO_PREC_BF16X3 = 2, LITHO_PREC_F16 = 3, LITHO_PREC_BF16 = 4 };

/* Optical settings of one bank (Sec. III-A, Eqs. 1-2).  All lengths in nm.
 * The clip of n x n pixels is one period of the transforms.  The pupil is
 * P(f) = 1[|f| <= NA/lambda] exp(i 2 pi / lambda * F NA^2 / 4 * (2 rho^2 - 1)),
 * rho = lambda |f| / NA (the defocus Zernike term, paraxial), one bank plane
 * per focus value F in focus_nm. */
typedef struct litho_optics {
  int n;                    /* grid side in pixels */
  double pixel_nm;          /* pixel size */
  double wavelength_nm;     /* lambda */
  double na;                /* numerical aperture */
  int source_kind;          /* LITHO_SRC_* */
  int source_grid;          /* G, odd, >= 3 */
  double sigma_in;          /* inner radius, units of NA */
  double sigma_out;         /* outer radius, units of NA, <= 1 */
  int n_focus;              /* number of focus planes, 1..8 */
  const double *focus_nm;   /* h_[n_focus] focus offsets F (copied) */
  int K;                    /* SOCS kernels kept per plane (Eq. 3), 1..n_source */
  double dose;              /* D of Eq. 1 (scales I); 0 is taken as 1 */
  /* LITHO_SRC_POINTS only (else ignored): h_[n_src_points][3] samples
   * (sigma_x, sigma_y, weight >= 0), sigma in units of NA with |sigma| <= 1,
   * copied.  sigma_in, sigma_out and source_grid are then ignored; the band is
   * set by the largest |sigma|. */
  const double *src_points;
  int n_src_points;
} litho_optics_t;

typedef struct litho_bank litho_bank_t;

/* Geometry and spectrum of a bank. */
typedef struct litho_bank_info {
  int n;                    /* grid side */
  int b;                    /* band half-width: |kx|, |ky| <= b, b = floor((1 + sigma_max) R) */
  int B;                    /* band side 2b + 1 */
  int K;                    /* kernels per plane */
  int n_focus;              /* planes */
  int n_source;             /* sampled source points (TCC rank bound) */
  int inner_grid;           /* side of the grid the per-kernel transforms run on */
  double pupil_radius;      /* R = NA n p / lambda in frequency-index units */
  size_t device_bytes;      /* device memory held by the bank (without workspaces) */
  double clear_field;       /* D sum_k lambda_k |Phi_k(0)|^2 of the first plane: the image of a clear mask */
  double degeneracy_gap;    /* min over planes of (lambda_K - lambda_{K+1}) / lambda_1; 1 when K is the
                             * source rank, 0 for a loaded bank (unknown).  A cut inside a degenerate
                             * pair (gap ~ 0) makes the truncated image depend on the eigenbasis. */
} litho_bank_info_t;

/* Build the SOCS kernel bank of Eqs. 2-3 on the host in FP64 and upload it.
 *   optics: read only during the call.  out: receives the new bank.
 * The TCC = A A^H with A[f, s] = sqrt(S_s) P(f + sigma_s; F) is decomposed
 * through the Hermitian source-space Gram matrix A^H A (own Jacobi solver),
 * Phi_k = A nu_k / sqrt(lambda_k) with ||Phi_k||_2 = 1 over the band samples,
 * eigenvalues in descending order.  Errors: LITHO_E_INVALID (bad optics),
 * LITHO_E_UNSUPPORTED (n), LITHO_E_NOMEM / LITHO_E_HIP (upload). */
int litho_kernels_build(const litho_optics_t *optics, litho_bank_t **out);

/* Load a bank from caller-provided eigenpairs instead of building it.
 *   h_lambda: [n_focus][K] eigenvalues (>= 0).
 *   h_phi:    [n_focus][K][B][B][2] interleaved (re, im) float64, indexed
 *             [ky + b][kx + b] (centred band order).
 * Everything is copied.  The band side B must be odd and B <= n. */
int litho_kernels_load(int n, int B, int K, int n_focus, const double *h_lambda,
                       const double *h_phi, litho_bank_t **out);

int litho_kernels_info(const litho_bank_t *bank, litho_bank_info_t *info);

/* Choose the grid the per-kernel transforms run on.  Each field E_k is
 * band-limited to |f| <= b, so |E_k|^2 is band-limited to |f| <= 2b and
 * sampling the per-kernel work on a q x q grid with q >= 4b + 1 is exact; the
 * image is then carried to the n x n grid by one zero-padded transform per
 * clip and plane (and the residual back by one low-pass transform).
 *   q = 0: automatic (the default after build/load): the smallest supported
 *          side >= 4b + 1 below n, else n.
 *   q = n: transforms on the full grid.
 *   other: 2^j, 3*2^j or 5*2^j with 4b + 1 <= q <= n (LITHO_E_INVALID otherwise).
 * Must not be called while work on this bank is in flight. */
int litho_kernels_set_inner_grid(litho_bank_t *bank, int q);

/* Copy the eigenvalues, h_lambda_out: [n_focus][K]. */
int litho_kernels_eigenvalues(const litho_bank_t *bank, double *h_lambda_out);

/* Copy kernel Phi_k of plane p (FP64, unit norm), h_phi_out: [B][B][2]. */
int litho_kernels_phi(const litho_bank_t *bank, int plane, int k, double *h_phi_out);

/* Host-only FP64 eigenpairs of one focus plane (the first half of
 * litho_kernels_build, no device needed): the K_max largest eigenvalues of the
 * TCC of Eq. 2 (descending) into h_lambda_out[K_max] and, if h_phi_out is not
 * NULL, the unit-norm kernels Phi_k into h_phi_out[K_max][B][B][2] (centred
 * band order, B = 2b + 1 as reported in *B_out).  optics->K is ignored;
 * K_max must not exceed the number of source points (*n_source_out). */
int litho_socs_host(const litho_optics_t *optics, int plane, int K_max, double *h_lambda_out,
                    double *h_phi_out, int *B_out, int *n_source_out);

/* Release the bank and every workspace it holds.  Waits for the device. NULL is ignored. */
void litho_kernels_free(litho_bank_t *bank);

/* Forward SOCS image, Eq. 4, for each focus plane of the bank.
 *   d_mask:  [batch][n][n] mask values (the thin-mask transmission, 1 = clear).
 *   K_use:   kernels used per plane, 1..K (the K_use largest).
 *   d_image: [batch][n_focus][n][n] output.
 *   prec:    LITHO_PREC_*.
 * batch may be 0 (no work).  Asynchronous on hip_stream. */
int litho_image(const litho_bank_t *bank, const float *d_mask, int batch, int K_use,
                float *d_image, int prec, void *hip_stream);

/* Loss of the fused mode: the squared or the absolute resist mismatch. */
enum { LITHO_LOSS_L2 = 0, LITHO_LOSS_L1 = 1 };

typedef struct litho_resist {
  double slope;       /* a of the sigmoid resist (e.g. 50) */
  double threshold;   /* t, relative to the open-frame intensity (e.g. 0.3) */
  const double *plane_weight;  /* h_[n_focus] weights w_p of the planes' losses, or NULL (all 1) */
  /* Resist kernel K_resist of Eq. 5: a Gaussian of this standard deviation in
   * pixels (0 = delta, no blur).  The resist then sees R = I (x) K_resist
   * (periodic convolution; exact through the band |f| <= 2b that carries I)
   * and the residual is blurred back, dL/dI = K_resist (x) dL/dR. */
  double blur_sigma_px;
  /* LITHO_LOSS_L2: L = sum w_p (Z - T)^2.  LITHO_LOSS_L1: L = sum w_p |Z - T|,
   * the sigmoid relaxation of the lithography-consistency loss of Eqs. 15 and
   * 17 (T = Z_round of Eq. 16, t = tau_print), dL/dZ = w_p sign(Z - T). */
  int loss;
} litho_resist_t;

/* Forward image plus the ILT adjoint (mask gradient).
 * Two modes:
 *   fused loss  (d_target != NULL): Z = sigmoid(a (R - t)) with R = I, or
 *                R = I (x) K_resist when resist->blur_sigma_px > 0,
 *                L = sum_planes w_p sum_r (Z - T)^2 per clip (|Z - T| for LITHO_LOSS_L1),
 *                G = dL/dI = K_resist (x) [2 w_p (Z - T) a Z (1 - Z)] (L1: w_p sign(Z - T) a Z (1 - Z));
 *                resist must be non-NULL.  With blur, d_image receives R.
 *   VJP         (d_target == NULL): G = d_grad_image, [batch][n_focus][n][n].
 * For each plane and kernel the coherent field E_k is recomputed (never
 * stored) and correlated with G through the conjugate kernel:
 *   dL/dm = sum_p sum_k 2 lambda_k Re IDFT( conj(Phi_k) DFT(G_p E_k) ).
 *   d_image:    [batch][n_focus][n][n] or NULL (then not written).
 *   d_loss:     device double [batch] or NULL (fused mode only).
 *   d_grad_mask:[batch][n][n] output.
 * Asynchronous on hip_stream. */
int litho_image_grad(const litho_bank_t *bank, const float *d_mask, int batch, int K_use,
                     const float *d_target, const litho_resist_t *resist,
                     const float *d_grad_image, float *d_image, double *d_loss,
                     float *d_grad_mask, int prec, void *hip_stream);

/* ---------------------------------------------------------------- after the image
 * The steps that follow the aerial image in the paper's flow: the resist
 * kernel and the target low-pass (Gaussian filters, Eqs. 5 and 16), the
 * printed contour (the level set of Eq. 5, extracted by marching squares as
 * in Sec. II-D), the edge placement error through focus (Eqs. 6-8) and the
 * physics channels of the AI initialiser's input (Eq. 9). */

/* Periodic Gaussian low-pass of count real images [count][n][n] (n = the
 * bank's grid side; the bank supplies the transform tables and workspace):
 *   out = Re IDFT( DFT(in) * exp(-2 pi^2 s^2 (fx^2 + fy^2) / n^2) ),
 * the transfer function truncated where it falls below 1e-12, at
 * |fx|, |fy| <= h = min(n/2 - 1, ceil(1.1832 n / s)).  This is Eq. 5's resist
 * kernel K_resist applied to an image (exact to that truncation for an aerial
 * image, which is band-limited to |f| <= 2b) and Eq. 16's G_sigma.
 * threshold: NaN for the filtered values; otherwise out = 1 where the
 * filtered value is >= threshold, else 0 (Eq. 16's Z_round with
 * tau_round = threshold).  d_in and d_out may be the same array.
 * Errors: LITHO_E_INVALID (NULL pointers, sigma_px <= 0).  Asynchronous. */
int litho_lowpass(const litho_bank_t *bank, const float *d_in, int count, double sigma_px,
                  double threshold, float *d_out, void *hip_stream);

/* Marching-squares contours of one periodic image at `level` (Sec. II-D; the
 * contour C of Eq. 5 when the image is the resist image and level = T_eff).
 * Cell (y, x), 0 <= y, x < n, has corners v(y,x), v(y,x+1), v(y+1,x+1),
 * v(y+1,x) (indices mod n); a corner is inside when v >= level (float32).
 * Edges: 0 top, 1 right, 2 bottom, 3 left.  A cell with one or three inside
 * corners, or two adjacent ones, holds one segment; two diagonal inside
 * corners (a saddle) hold two, joined as the cell mean 0.25 ((c0 + c1) +
 * (c2 + c3)) >= level decides (centre inside or not).  Segments run with the
 * inside on their left (x to the right, y down) and are listed in raster
 * order of cells, then by start edge.  Per segment j < capacity:
 *   d_cell[j]  = y * n + x;
 *   d_code[j]  = start_edge * 4 + end_edge;
 *   d_u[2j], d_u[2j+1] = crossing parameters on the start and end edge,
 *                (level - a) / (b - a) from the edge's first corner a (left
 *                end of a horizontal edge, top end of a vertical one);
 *   d_next[j]  = index of the segment that starts where segment j ends (the
 *                segments form closed loops; indices may reach past capacity).
 * d_count (device int) receives the total number of segments; when it
 * exceeds capacity only the first capacity segments were written and the
 * call can be repeated with a larger capacity.  capacity 0 counts only (the
 * output pointers may then be NULL).  The library keeps count/offset scratch
 * of 2 n ceil(n/64) + 1 ints per device and stream.  2 <= n <= 4096
 * (LITHO_E_UNSUPPORTED otherwise).  Asynchronous. */
int litho_contours(int n, const float *d_image, double level, int capacity, int *d_cell, int *d_code,
                   float *d_u, int *d_next, int *d_count, void *hip_stream);

/* litho_contours for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results and errors, but its count and offset scratch
 * is a static device array of 2 * 4096 * 64 + 1 ints (about 2 MiB) that each
 * GPU the library runs on holds until the process ends; nothing is allocated
 * (no hipMalloc, hipFree or allocating library call).  n above 4096 (the
 * array's limit) gives LITHO_E_UNSUPPORTED.  Every call on one GPU uses that
 * GPU's single array: calls that overlap on one GPU (different streams, not
 * ordered) race and must not be issued; calls ordered on one stream are safe.
 * Every scratch value a call reads it first writes, so nothing is cleared. */
int litho_contours_noalloc(int n, const float *d_image, double level, int capacity, int *d_cell, int *d_code,
                           float *d_u, int *d_next, int *d_count, void *hip_stream);

/* Eq. 6's target level and Eq. 8's through-focus rule. */
typedef struct litho_epe_rule {
  double t_eff;     /* E_tgt on the target edge (the printing threshold) */
  double tol_neg;   /* tol_neg <= 0 */
  double tol_pos;   /* tol_pos >= 0 */
  int f0;           /* index of the on-focus plane among the latent images */
} litho_epe_rule_t;

/* Edge placement error at the edges of a binary target through focus
 * (Eqs. 6-8).  Sites are the 4-neighbour pixel pairs whose targets
 * (T >= 0.5) differ, listed per pixel (y, x) in raster order: first the pair
 * with (y, x+1), then with (y+1, x) (periodic).  At a site, for each latent
 * image E_p (d_latent [n_planes][n][n], e.g. the resist image of each focus
 * plane) the iso-level E = t_eff is located by Eq. 6 at the pair's midpoint:
 *   EPE_p = -(E_mid - t_eff) / |grad E|,  E_mid = (E_a + E_b) / 2,
 * with the normal derivative E_b - E_a and the tangential derivative a
 * quarter of the difference of the neighbouring pairs' sums on either side
 * (pixels; +-inf where the gradient vanishes, 0 if E_mid = t_eff too).  Per
 * site j < capacity: d_site[j] = y * n + x, d_dir[j] = 0 (pair along x) or
 * 1 (along y), d_epe[j][0 .. n_planes-1] = EPE_p, d_epe[j][n_planes] =
 * EPE_avg (Eq. 7), d_epe[j][n_planes+1] = EPE_eff (Eq. 8: EPE_f0 - tol_pos
 * above tol_pos, EPE_f0 - tol_neg below tol_neg, EPE_avg between, bounds
 * included).  Arithmetic in float32.  d_count and capacity as for
 * litho_contours; 1 <= n_planes <= 8.  Asynchronous. */
int litho_epe(int n, const float *d_target, const float *d_latent, int n_planes, const litho_epe_rule_t *rule,
              int capacity, int *d_site, int *d_dir, float *d_epe, int *d_count, void *hip_stream);

/* The three input channels of Eq. 9 for a batch of target layouts Z_t
 * (d_layout [batch][n][n]), channel last: d_out[batch][n][n][3] =
 *   (M0 = Z_t,  I0 = the SOCS image of Z_t at focus plane `plane` with K_use
 *    kernels (Eq. 4),  dI/dM = dI(r)/dm(r), the image's derivative with
 *    respect to the mask pixel at the same position,
 *    2 D sum_k lambda_k Re[ conj(E_k(r)) phi_k(0) ], phi_k(0) = IDFT(Phi_k)(0)).
 * h_norm: NULL (raw values) or [6] = (lo, hi) per channel; each channel is
 * then mapped to clip((v - lo) / (hi - lo), 0, 1) (the global normalisation
 * of Eq. 9).  Asynchronous. */
int litho_ai_channels(const litho_bank_t *bank, const float *d_layout, int batch, int K_use, int plane,
                      const double *h_norm, float *d_out, void *hip_stream);

/* ---------------------------------------------------------------- layouts beyond one clip
 * A layout larger than a clip (the paper's flow images full layouts; it does
 * not describe its tiling) is imaged through halo tiling with the bank's clip
 * side n: the H x W layout (row-major, opaque outside: m = 0) is cut into
 * n x n windows with a halo of `halo` pixels around a core of
 * c = n - 2 halo pixels; core (i, j) starts at (i c, j c) and its window at
 * (i c - halo, j c - halo), ceil(H / c) x ceil(W / c) tiles in raster order.
 * Each window is imaged as one periodic clip (Eq. 4, every focus plane of the
 * bank) and the image of its core is kept, so the halo must cover the
 * optical ambit for the seams to vanish.  Windows are processed in chunks
 * that fit the workspace limit.  Errors: LITHO_E_INVALID (NULL pointers, no
 * core left: n - 2 halo < 1, H or W < 1).  Asynchronous. */

/* d_layout [H][W]; d_image [n_focus][H][W]. */
int litho_image_tiled(const litho_bank_t *bank, const float *d_layout, int H, int W, int halo, int K_use,
                      float *d_image, int prec, void *hip_stream);

/* Tiled ILT loss and gradient: L = sum_p w_p sum over layout pixels of
 * (Z - T)^2 (|Z - T| for LITHO_LOSS_L1) with Z the sigmoid resist of the
 * tiled image (each layout pixel counted once, in its core), and dL/dm, the
 * exact derivative of that tiled loss: per window, the adjoint of
 * litho_image_grad with the residual restricted to the core, summed into
 * the layout gradient over the whole window in tile order (deterministic).
 * d_target [H][W]; resist: slope, threshold, plane weights and loss as for
 * litho_image_grad (blur_sigma_px must be 0: LITHO_E_UNSUPPORTED otherwise);
 * d_image [n_focus][H][W] or NULL; d_loss: device double [1] or NULL;
 * d_grad [H][W]. */
int litho_image_grad_tiled(const litho_bank_t *bank, const float *d_layout, int H, int W, int halo, int K_use,
                           const float *d_target, const litho_resist_t *resist, float *d_image, double *d_loss,
                           float *d_grad, int prec, void *hip_stream);

/* Per-kernel device timing (tracing).  While enabled, every kernel launch is
 * bracketed by HIP events on its own stream; litho_profile_read() waits for
 * those events and returns, per kernel name, the launch count and the summed
 * duration in milliseconds, then clears them.  Names are written as
 * "name=count:total_ms;" into buf (truncated to cap bytes, NUL-terminated). */
int litho_profile_enable(int on);
int litho_profile_read(char *buf, size_t cap);

/* ---------------------------------------------------------------- serving
 * Image formation and forward/adjoint modelling served as a stream of
 * batched work that keeps the device busy (Sec. V, inspection pipelines),
 * with data kept on the device and unavoidable host transfers staged in
 * pinned memory (Sec. II-D).
 * A persistent request loop (continuous batching): requests of mixed clip
 * size arrive at any time, are admitted while their device footprint fits in
 * hbm_budget bytes and a slot is free, run on that slot's own stream
 * concurrently with other slots, and complete independently.  Banks stay
 * resident for the life of the server (the caller keeps them alive). */
typedef struct litho_server litho_server_t;

typedef struct litho_serve_cfg {
  size_t hbm_budget;   /* bytes of device memory the server may hold: each slot keeps one arena
                        * (imaging workspace and request I/O buffers) sized for the largest
                        * request it ran; the sum of arenas and running requests never exceeds
                        * this, idle arenas are released when a request would not fit */
  int max_slots;       /* concurrent requests on the device (streams), 1..64 */
  int max_queue;       /* pending requests before submit returns LITHO_E_BUSY */
} litho_serve_cfg_t;

typedef struct litho_request {
  int bank;            /* index into the server's banks */
  int K_use;           /* kernels per plane, 1..K of that bank */
  int mode;            /* 0 = image only, 1 = image + loss + gradient */
  const float *h_mask;    /* [n][n] host, copied at submit */
  const float *h_target;  /* [n][n] host (mode 1), copied at submit */
  double slope, threshold; /* resist (mode 1) */
  int prec;            /* LITHO_PREC_* of the request */
  /* Device-resident I/O (optional).  When d_mask is not NULL the request reads
   * d_mask [n][n] (and d_target [n][n] in mode 1) from device memory and
   * writes d_image [n_focus][n][n] (and d_grad [n][n], plus d_loss [1] if not
   * NULL, in mode 1) there: h_mask and h_target are ignored, nothing is copied
   * to or from the host, and litho_serve_poll ignores h_image and h_grad
   * (info->loss is NaN; the loss is in d_loss).  The inputs must be complete
   * when litho_serve_submit is called (synchronise the stream that produced
   * them first); the caller keeps all five buffers alive, and the inputs
   * unmodified, until litho_serve_poll has returned the request. */
  const float *d_mask;
  const float *d_target;
  float *d_image;
  float *d_grad;
  double *d_loss;
} litho_request_t;

typedef struct litho_result_info {
  int status;          /* LITHO_OK or the error of the request */
  int n, n_focus;
  double loss;         /* mode 1 */
  double t_submit_us;  /* library clock (monotonic, microseconds) */
  double t_start_us;   /* admitted to a slot */
  double t_done_us;    /* device work finished */
} litho_result_info_t;

/* Create a server over n_banks resident banks (the pointers are copied; the
 * banks must outlive the server). */
int litho_serve_create(litho_bank_t *const *banks, int n_banks, const litho_serve_cfg_t *cfg,
                       litho_server_t **out);

/* Queue a request; *ticket receives its id.  Host masks/targets are copied
 * on the calling thread (into pinned staging from a server-wide pool capped by
 * LITHO_SERVE_PINNED_MB, default 4096, else into pageable memory), so the
 * caller may reuse them at once (device-resident requests: see
 * litho_request_t).  LITHO_E_NOMEM if the request can never fit hbm_budget,
 * LITHO_E_BUSY if the queue is full, LITHO_E_INVALID for a malformed request. */
int litho_serve_submit(litho_server_t *srv, const litho_request_t *req, uint64_t *ticket);

/* Wait up to timeout_us (0 = do not wait, < 0 = forever) for a ticket.
 * Returns LITHO_PENDING while running; on completion copies the image
 * ([n_focus][n][n]) and, for mode 1, the gradient ([n][n]) into the host
 * buffers on the calling thread (either may be NULL; both are ignored for device-resident requests,
 * whose results are already in their device buffers), fills *info and releases
 * the ticket. */
int litho_serve_poll(litho_server_t *srv, uint64_t ticket, float *h_image, float *h_grad,
                     litho_result_info_t *info, int64_t timeout_us);

/* Stop the loop, wait for in-flight work and free everything. NULL is ignored. */
void litho_serve_destroy(litho_server_t *srv);

/* Text of the last error on this thread ("" if none). */
const char *litho_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LITHO_H */
