// C ABI of the SOCS imaging library: banks, imaging, adjoint and tracing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bank.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "litho_internal.hpp"
#include "post.hpp"

// ============================================================ errors
namespace litho {
namespace {
thread_local std::string t_err;
}
void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
}
void clear_error() { t_err.clear(); }
const char *last_error() { return t_err.c_str(); }

// ============================================================ tracing
namespace {
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};
std::atomic<bool> g_prof{false};
std::mutex g_prof_mu;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_event_pool;
thread_local hipEvent_t t_pending = nullptr;

hipEvent_t take_event() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

void prof_begin(const char *name, hipStream_t s) {
  (void)name;
  t_pending = nullptr;
  if (!g_prof.load(std::memory_order_relaxed)) return;
  hipEvent_t e = take_event();
  if (e && hipEventRecord(e, s) == hipSuccess) t_pending = e;
}

void prof_end(const char *name, hipStream_t s) {
  if (!t_pending) return;
  hipEvent_t e = take_event();
  if (!e || hipEventRecord(e, s) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_recs.push_back({name, t_pending, e});
  t_pending = nullptr;
}

// ============================================================ geometry helpers
// Clip sides with an FFT plan: 2^j {1, 3, 5}, 64 <= n <= 4096.
bool supported_side(int n) { return pass_threads(n) != 0; }

// Smallest supported side >= 4b + 1 below n (exact for |E_k|^2, which is
// band-limited to |f| <= 2b), else n itself.
int auto_inner_grid(int n, int b) {
  static const int sizes[] = {64, 96, 128, 160, 192, 256, 320, 384, 512, 640, 768, 1024, 1280, 1536, 2048, 2560, 3072};
  for (int q : sizes)
    if (q >= 4 * b + 1 && q < n) return q;
  return n;
}

}  // namespace litho

using namespace litho;

// ============================================================ bank
namespace litho {
int make_twiddles(int L, float2 **out);
int set_inner_grid(litho_bank *bk, int q);
int auto_inner_grid(int n, int b);
}  // namespace litho

static int upload_bank(litho_bank *bk) {
  HostBank &h = bk->host;
  bk->Bp = (h.B + kTileCols - 1) / kTileCols * kTileCols;
  bk->nt = bk->Bp / kTileCols;
  LITHO_HIP_TRY(hipGetDevice(&bk->device));
  const size_t per = size_t(bk->nt) * h.B * kTileCols;
  std::vector<float2> tiles(size_t(h.n_focus) * h.K * per, make_float2(0.f, 0.f));
  for (int p = 0; p < h.n_focus; ++p)
    for (int k = 0; k < h.K; ++k) {
      const double sl = std::sqrt(h.lambda[size_t(p) * h.K + k]);
      const cd *ph = &h.phi[(size_t(p) * h.K + k) * h.B * h.B];
      float2 *dst = &tiles[(size_t(p) * h.K + k) * per];
      for (int r = 0; r < h.B; ++r)
        for (int j = 0; j < h.B; ++j) {
          const cd v = ph[size_t(r) * h.B + j] * sl;
          dst[(size_t(j / kTileCols) * h.B + r) * kTileCols + (j % kTileCols)] =
              make_float2(float(v.real()), float(v.imag()));
        }
    }
  bk->phi_bytes = tiles.size() * sizeof(float2);
  if (hipMalloc(&bk->d_phi, bk->phi_bytes) != hipSuccess) {
    set_error("litho: cannot allocate %zu bytes for the kernel bank", bk->phi_bytes);
    return LITHO_E_NOMEM;
  }
  LITHO_HIP_TRY(hipMemcpy(bk->d_phi, tiles.data(), bk->phi_bytes, hipMemcpyHostToDevice));
  LITHO_TRY(make_twiddles(h.n, &bk->d_twN));
  return set_inner_grid(bk, 0);
}

namespace litho {

// Per-pass twiddle table of the length-L FFT plan, uploaded once per bank.
int make_twiddles(int L, float2 **out) {
  std::vector<float2> tw;
  LITHO_TRY(twiddle_table(L, tw));
  if (hipMalloc(out, tw.size() * sizeof(float2)) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    set_error("litho: cannot allocate the twiddle table");
    return LITHO_E_NOMEM;
  }
  LITHO_HIP_TRY(hipMemcpy(*out, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
  return LITHO_OK;
}

int set_inner_grid(litho_bank *bk, int q) {
  const HostBank &h = bk->host;
  if (q == 0) q = auto_inner_grid(h.n, h.b);
  if (q != h.n && (pass_threads(q) == 0 || q < 4 * h.b + 1 || q > h.n)) {
    set_error("inner grid %d is not supported for n=%d, b=%d (needs 4b+1 <= q <= n from the FFT plan list)", q,
              h.n, h.b);
    return LITHO_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(bk->mu);
  bool tables = bk->d_rowtw != nullptr;
  for (void *t : bk->d_gemm) tables = tables || t;
  for (void *t : bk->d_rowmma) tables = tables || t;
  if ((bk->d_twQ && bk->d_twQ != bk->d_twN) || tables) LITHO_HIP_TRY(hipDeviceSynchronize());
  if (bk->d_twQ && bk->d_twQ != bk->d_twN) (void)hipFree(bk->d_twQ);
  for (void *&t : bk->d_gemm) {
    if (t) (void)hipFree(t);
    t = nullptr;
  }
  for (void *&t : bk->d_rowmma) {
    if (t) (void)hipFree(t);
    t = nullptr;
  }
  if (bk->d_rowtw) (void)hipFree(bk->d_rowtw);
  bk->d_rowtw = nullptr;
  bk->d_twQ = nullptr;
  bk->Q = q;
  if (q == h.n) {
    bk->d_twQ = bk->d_twN;
    return LITHO_OK;
  }
  return make_twiddles(q, &bk->d_twQ);
}

// Band DFT-GEMM table of the bank's inner grid (forward or adjoint column
// pass), uploaded on first use.
static int gemm_table(litho_bank *bk, bool adj, bool bf16, const void **out) {
  std::lock_guard<std::mutex> lk(bk->mu);
  void *&t = bk->d_gemm[(adj ? 2 : 0) + (bf16 ? 1 : 0)];
  if (!t) {
    std::vector<uint16_t> tab;
    if (adj)
      fill_adj_table(bk->Q, bk->host.b, bf16, tab);
    else
      fill_band_table(bk->Q, bk->host.b, bf16, tab);
    if (hipMalloc(&t, tab.size() * sizeof(uint16_t)) != hipSuccess) {
      (void)hipGetLastError();
      t = nullptr;
      set_error("litho: cannot allocate the band DFT-GEMM table");
      return LITHO_E_NOMEM;
    }
    LITHO_HIP_TRY(hipMemcpy(t, tab.data(), tab.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  *out = t;
  return LITHO_OK;
}

// Operand fragments and twiddles of the two-stage row transform for the
// bank's inner grid, uploaded on first use.
static int row_mfma_table(litho_bank *bk, bool bf16, const void **tab, const float2 **twl) {
  std::lock_guard<std::mutex> lk(bk->mu);
  void *&t = bk->d_rowmma[bf16 ? 1 : 0];
  if (!t || !bk->d_rowtw) {
    std::vector<uint16_t> frag;
    std::vector<float2> tw;
    fill_row_mfma_table(bk->Q, bf16, frag, tw);
    if (!t) {
      if (hipMalloc(&t, frag.size() * sizeof(uint16_t)) != hipSuccess) {
        (void)hipGetLastError();
        t = nullptr;
        set_error("litho: cannot allocate the row-transform operand table");
        return LITHO_E_NOMEM;
      }
      LITHO_HIP_TRY(hipMemcpy(t, frag.data(), frag.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    }
    if (!bk->d_rowtw) {
      if (hipMalloc(&bk->d_rowtw, tw.size() * sizeof(float2)) != hipSuccess) {
        (void)hipGetLastError();
        bk->d_rowtw = nullptr;
        set_error("litho: cannot allocate the row-transform twiddles");
        return LITHO_E_NOMEM;
      }
      LITHO_HIP_TRY(hipMemcpy(bk->d_rowtw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
    }
  }
  *tab = t;
  *twl = bk->d_rowtw;
  return LITHO_OK;
}

int check_prec(int prec, const char *who) {
  if (prec < LITHO_PREC_FP32 || prec > LITHO_PREC_BF16) {
    set_error("%s: unknown precision mode %d", who, prec);
    return LITHO_E_INVALID;
  }
  return LITHO_OK;
}

}  // namespace litho

extern "C" int litho_kernels_build(const litho_optics_t *optics, litho_bank_t **out) {
  clear_error();
  if (!optics || !out) {
    set_error("litho_kernels_build: NULL argument");
    return LITHO_E_INVALID;
  }
  *out = nullptr;
  if (!supported_side(optics->n)) {
    set_error("litho_kernels_build: grid side %d is not 2^j times 1, 3 or 5 in [64, 4096]", optics->n);
    return LITHO_E_UNSUPPORTED;
  }
  auto *bk = new litho_bank();
  int rc = build_host_bank(*optics, bk->host);
  if (rc == LITHO_OK) rc = upload_bank(bk);
  if (rc != LITHO_OK) {
    litho_kernels_free(bk);
    return rc;
  }
  *out = bk;
  return LITHO_OK;
}

extern "C" int litho_kernels_load(int n, int B, int K, int n_focus, const double *h_lambda, const double *h_phi,
                                  litho_bank_t **out) {
  clear_error();
  if (!out || !h_lambda || !h_phi) {
    set_error("litho_kernels_load: NULL argument");
    return LITHO_E_INVALID;
  }
  *out = nullptr;
  if (!supported_side(n)) {
    set_error("litho_kernels_load: grid side %d is not 2^j times 1, 3 or 5 in [64, 4096]", n);
    return LITHO_E_UNSUPPORTED;
  }
  if (B < 1 || (B % 2) == 0 || B > n || K < 1 || n_focus < 1 || n_focus > 8) {
    set_error("litho_kernels_load: invalid sizes (B=%d K=%d n_focus=%d)", B, K, n_focus);
    return LITHO_E_INVALID;
  }
  for (int i = 0; i < K * n_focus; ++i)
    if (!(h_lambda[i] >= 0.0) || !std::isfinite(h_lambda[i])) {
      set_error("litho_kernels_load: eigenvalue %d is negative or not finite", i);
      return LITHO_E_INVALID;
    }
  auto *bk = new litho_bank();
  HostBank &h = bk->host;
  h.n = n; h.B = B; h.b = (B - 1) / 2; h.K = K; h.n_focus = n_focus; h.n_source = 0; h.R = 0.0;
  h.lambda.assign(h_lambda, h_lambda + size_t(K) * n_focus);
  h.phi.resize(size_t(n_focus) * K * B * B);
  for (size_t i = 0; i < h.phi.size(); ++i) h.phi[i] = cd(h_phi[2 * i], h_phi[2 * i + 1]);
  h.gap.assign(n_focus, 0.0);
  int rc = upload_bank(bk);
  if (rc != LITHO_OK) {
    litho_kernels_free(bk);
    return rc;
  }
  *out = bk;
  return LITHO_OK;
}

extern "C" int litho_socs_host(const litho_optics_t *optics, int plane, int K_max, double *h_lambda_out,
                               double *h_phi_out, int *B_out, int *n_source_out) {
  clear_error();
  if (!optics || !h_lambda_out || K_max < 1) {
    set_error("litho_socs_host: invalid argument");
    return LITHO_E_INVALID;
  }
  if (plane < 0 || plane >= optics->n_focus || !optics->focus_nm) {
    set_error("litho_socs_host: plane %d outside the %d focus planes", plane, optics->n_focus);
    return LITHO_E_INVALID;
  }
  litho_optics_t one = *optics;
  one.n_focus = 1;
  one.focus_nm = optics->focus_nm + plane;
  one.K = K_max;
  HostBank hb;
  LITHO_TRY(build_host_bank(one, hb));
  std::memcpy(h_lambda_out, hb.lambda.data(), size_t(K_max) * sizeof(double));
  if (h_phi_out)
    for (size_t i = 0; i < hb.phi.size(); ++i) {
      h_phi_out[2 * i] = hb.phi[i].real();
      h_phi_out[2 * i + 1] = hb.phi[i].imag();
    }
  if (B_out) *B_out = hb.B;
  if (n_source_out) *n_source_out = hb.n_source;
  return LITHO_OK;
}

extern "C" int litho_kernels_info(const litho_bank_t *bk, litho_bank_info_t *info) {
  clear_error();
  if (!bk || !info) {
    set_error("litho_kernels_info: NULL argument");
    return LITHO_E_INVALID;
  }
  info->n = bk->host.n;
  info->b = bk->host.b;
  info->B = bk->host.B;
  info->K = bk->host.K;
  info->n_focus = bk->host.n_focus;
  info->n_source = bk->host.n_source;
  info->inner_grid = bk->Q;
  info->pupil_radius = bk->host.R;
  info->device_bytes = bk->phi_bytes + size_t(bk->host.n) * sizeof(float2);
  const HostBank &h = bk->host;
  double cf = 0.0;
  for (int k = 0; k < h.K; ++k)
    cf += h.lambda[size_t(k)] * std::norm(h.phi[(size_t(k) * h.B + h.b) * h.B + h.b]);
  info->clear_field = h.dose * cf;
  info->degeneracy_gap = h.gap.empty() ? 0.0 : *std::min_element(h.gap.begin(), h.gap.end());
  return LITHO_OK;
}

extern "C" int litho_kernels_set_inner_grid(litho_bank_t *bk, int q) {
  clear_error();
  if (!bk || q < 0) {
    set_error("litho_kernels_set_inner_grid: invalid argument");
    return LITHO_E_INVALID;
  }
  return set_inner_grid(bk, q);
}

extern "C" int litho_kernels_eigenvalues(const litho_bank_t *bk, double *h_lambda_out) {
  clear_error();
  if (!bk || !h_lambda_out) {
    set_error("litho_kernels_eigenvalues: NULL argument");
    return LITHO_E_INVALID;
  }
  std::memcpy(h_lambda_out, bk->host.lambda.data(), bk->host.lambda.size() * sizeof(double));
  return LITHO_OK;
}

extern "C" int litho_kernels_phi(const litho_bank_t *bk, int plane, int k, double *h_phi_out) {
  clear_error();
  if (!bk || !h_phi_out || plane < 0 || plane >= bk->host.n_focus || k < 0 || k >= bk->host.K) {
    set_error("litho_kernels_phi: invalid argument");
    return LITHO_E_INVALID;
  }
  const size_t BB = size_t(bk->host.B) * bk->host.B;
  const cd *src = &bk->host.phi[(size_t(plane) * bk->host.K + k) * BB];
  for (size_t i = 0; i < BB; ++i) {
    h_phi_out[2 * i] = src[i].real();
    h_phi_out[2 * i + 1] = src[i].imag();
  }
  return LITHO_OK;
}

extern "C" void litho_kernels_free(litho_bank_t *bk) {
  if (!bk) return;
  (void)hipDeviceSynchronize();
  for (auto &kv : bk->ws) {
    if (kv.second.base) (void)hipFree(kv.second.base);
    for (hipStream_t t : kv.second.side) (void)hipStreamDestroy(t);
    for (hipEvent_t e : kv.second.ev) (void)hipEventDestroy(e);
  }
  for (auto &kv : bk->aux)
    if (kv.second.base) (void)hipFree(kv.second.base);
  for (auto &kv : bk->psi)
    if (kv.second) (void)hipFree(kv.second);
  if (bk->d_twQ && bk->d_twQ != bk->d_twN) (void)hipFree(bk->d_twQ);
  for (void *t : bk->d_gemm)
    if (t) (void)hipFree(t);
  for (void *t : bk->d_rowmma)
    if (t) (void)hipFree(t);
  if (bk->d_rowtw) (void)hipFree(bk->d_rowtw);
  if (bk->d_twN) (void)hipFree(bk->d_twN);
  if (bk->d_phi) (void)hipFree(bk->d_phi);
  delete bk;
}

// ============================================================ workspace
namespace litho {

size_t workspace_limit_bytes() {
  const char *e = std::getenv("LITHO_WORKSPACE_MB");
  size_t mb = 8192;
  if (e && *e) mb = size_t(std::strtoull(e, nullptr, 10));
  return std::max<size_t>(mb, 1) << 20;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

CallLayout plan_call(const litho_bank *bk, int batch, int K_use, bool grad, bool fused, int prec, bool blur) {
  CallLayout L;
  const HostBank &h = bk->host;
  PassGeo &g = L.g;
  g.N = h.n; g.Q = bk->Q; g.b = h.b; g.B = h.B; g.Bp = bk->Bp; g.nt = bk->nt;
  g.D = 4 * h.b + 1;
  g.Dp = (g.D + kTileCols - 1) / kTileCols * kTileCols;
  g.ntD = g.Dp / kTileCols;
  g.K = K_use; g.Kbank = h.K; g.P = h.n_focus; g.dose = h.dose;
  // a resist blur acts on the intensity band, so it takes the resampling route
  // even when the per-kernel transforms run on the full grid
  const bool resample = g.Q != g.N || (blur && fused && grad);
  L.resample = resample;
  // split modes on inner grids 32 P (P <= 32) of the resampled route: the
  // forward row pass as two MFMA stages, every column pass in FP32; other
  // inner grids: the band DFT-GEMM column passes
  L.row_mfma = prec != LITHO_PREC_FP32 && g.Q != g.N && row_mfma_ok(g.Q, g.N);
  // k-chunks of the adjoint column pass: enough blocks to fill the device
  // (~2048: eight per CU; more chunks only add FP64 partials for the gradient
  // columns to read), each chunk summing kper kernels in FP32 before the FP64
  // reduction.  The GEMM form has one workgroup per 32-column block of the
  // band (~1024).
  {
    const bool gemm = prec != LITHO_PREC_FP32 && !L.row_mfma;
    const size_t units = gemm ? size_t(adj_gemm_blocks(g.Bp, g.B)) * batch : size_t(g.nt) * batch;
    const size_t target = gemm ? 1024 : 2048;
    const int want = int((target + units - 1) / units);
    const int kc = std::max(1, std::min(K_use, want));
    g.kper = (K_use + kc - 1) / kc;
    g.KC = (K_use + g.kper - 1) / g.kper;
  }
  // loss partials come from the row pass that applies the resist (N grid):
  // one per block; with resampling that pass takes two rows per transform
  L.nblk = resample ? (g.N / (256 / pass_threads(g.N)) + 1) / 2 : g.N / (256 / pass_threads(g.N));
  const size_t N = g.N, Q = g.Q;
  L.b_S1 = align256(size_t(g.nt) * N * kTileCols * sizeof(float2));
  L.b_Mh = align256(size_t(g.nt) * g.B * kTileCols * sizeof(float2));
  L.b_Y = align256(size_t(K_use) * g.nt * Q * kTileCols * sizeof(float2));
  // the residual G on the N grid is only stored where the adjoint row pass reads it
  // (no resampling); the resampled step keeps it on chip
  L.b_G = (grad && fused && !resample) ? align256(N * N * sizeof(float)) : 0;
  L.b_part = grad ? align256(size_t(g.P) * g.KC * g.nt * g.B * kTileCols * sizeof(double2)) : 0;
  L.b_loss = (grad && fused) ? align256(size_t(g.P) * L.nblk * sizeof(double)) : 0;
  L.b_X = resample ? align256(std::max(N, Q) * g.Dp * sizeof(float2)) : 0;
  // Few clips and several focus planes: the per-kernel passes of one plane
  // launch too few workgroups to fill the device, so the planes run
  // concurrently on side streams, each with its own Y, G and band buffers.
  // Row passes launch about Q / (256 / T) workgroups per clip.
  {
    const size_t row_blocks = size_t(Q) / (256 / pass_threads(g.Q)) * size_t(batch);
    L.pp = (g.P > 1 && row_blocks < 2048) ? g.P : 1;
  }
  const size_t per = L.b_S1 + L.b_Mh + L.b_part + L.b_loss + size_t(L.pp) * (L.b_Y + L.b_G + 2 * L.b_X);
  L.per_clip = per;
  const size_t lim = workspace_limit_bytes();
  L.chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(batch), lim / per)));
  return L;
}

static int grow_workspace(litho_bank *bk, std::map<hipStream_t, Workspace> &m, hipStream_t s, size_t bytes,
                          char **out) {
  std::lock_guard<std::mutex> lk(bk->mu);
  Workspace &w = m[s];
  if (w.bytes < bytes) {
    if (w.base) {
      LITHO_HIP_TRY(hipStreamSynchronize(s));
      LITHO_HIP_TRY(hipFree(w.base));
      w.base = nullptr;
      w.bytes = 0;
    }
    if (hipMalloc(&w.base, bytes) != hipSuccess) {
      (void)hipGetLastError();
      w.base = nullptr;
      set_error("litho: cannot allocate a %zu byte workspace", bytes);
      return LITHO_E_NOMEM;
    }
    w.bytes = bytes;
  }
  *out = static_cast<char *>(w.base);
  return LITHO_OK;
}

int acquire_workspace(litho_bank *bk, hipStream_t s, size_t bytes, char **out) {
  return grow_workspace(bk, bk->ws, s, bytes, out);
}

int acquire_aux(litho_bank *bk, hipStream_t s, size_t bytes, char **out) {
  return grow_workspace(bk, bk->aux, s, bytes, out);
}

// count side streams of the workspace of stream s, and count + 1 events.
int plane_streams(litho_bank *bk, hipStream_t s, int count, hipStream_t *side, hipEvent_t *ev) {
  std::lock_guard<std::mutex> lk(bk->mu);
  Workspace &w = bk->ws[s];
  while (int(w.side.size()) < count) {
    hipStream_t t = nullptr;
    LITHO_HIP_TRY(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
    w.side.push_back(t);
  }
  while (int(w.ev.size()) < count + 1) {
    hipEvent_t e = nullptr;
    LITHO_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    w.ev.push_back(e);
  }
  for (int i = 0; i < count; ++i) side[i] = w.side[i];
  for (int i = 0; i <= count; ++i) ev[i] = w.ev[i];
  return LITHO_OK;
}

// Forward (and optionally adjoint) over one chunk of clips.
int run_chunk(litho_bank *bk, const CallLayout &L, char *ws, const float *mask, int n, const float *target,
              const float *grad_image, float *image, double *loss, float *grad_mask, bool grad, hipStream_t s,
              const CallOpts &o, int prec, const void *gemm_fwd, const void *gemm_adj, const void *row_tab,
              const float2 *row_tw) {
  PassGeo g = L.g;
  g.slope = o.slope;
  g.thr = o.thr;
  g.loss_l1 = o.loss_l1;
  const double *plane_w = o.plane_w;
  char *p = ws;
  auto *S1 = reinterpret_cast<float2 *>(p); p += L.b_S1 * n;
  auto *Mh = reinterpret_cast<float2 *>(p); p += L.b_Mh * n;
  auto *part = reinterpret_cast<double2 *>(p); p += L.b_part * n;
  auto *lossp = reinterpret_cast<double *>(p); p += L.b_loss * n;
  // per concurrent plane: Y, G, X1, X2
  char *const plane_base = p;
  const size_t plane_bytes = (L.b_Y + L.b_G + 2 * L.b_X) * n;
  hipStream_t side[8] = {};
  hipEvent_t ev[9] = {};
  if (L.pp > 1) LITHO_TRY(plane_streams(bk, s, L.pp - 1, side, ev));
  const bool fused = target != nullptr;
  const bool resample = L.resample;
  const double blur = fused && grad ? o.blur_sigma : 0.0;
  const size_t NN = size_t(g.N) * g.N;
  const size_t band_clip = size_t(g.ntD) * g.D * kTileCols;  // complex values of one D x D band
  const int h2 = 2 * g.b;
  const float2 *twN = bk->d_twN, *twQ = bk->d_twQ;
  // mask spectrum (once per clip, shared by every plane)
  LITHO_TRY(run_rows_fwd_real("mask_rows", g.N, mask, NN, S1, g.b, g.Bp, twN,
                              float(1.0 / (double(g.N) * double(g.N))), n, s));
  LITHO_TRY(run_col_fft("mask_cols", g.N, -1, S1, Mh, g.nt, -1, g.b, twN, 1.0f, n, s));
  const int p_end = o.p1 < 0 ? g.P : std::min(g.P, o.p1);
  if (L.pp > 1) {
    // fork: the side streams start after the mask spectrum
    LITHO_HIP_TRY(hipEventRecord(ev[0], s));
    for (int i = 0; i < L.pp - 1; ++i) LITHO_HIP_TRY(hipStreamWaitEvent(side[i], ev[0], 0));
  }
  const hipStream_t s_main = s;
  for (int pl = o.p0; pl < p_end; ++pl) {
    const int slot = L.pp > 1 ? pl % L.pp : 0;
    char *q = plane_base + size_t(slot) * plane_bytes;
    auto *Y = reinterpret_cast<float2 *>(q); q += L.b_Y * n;
    auto *G = reinterpret_cast<float *>(q); q += L.b_G * n;
    auto *X1 = reinterpret_cast<float2 *>(q); q += L.b_X * n;
    auto *X2 = reinterpret_cast<float2 *>(q);
    // the N-row band of the image and of the residual: X2 when one pass does
    // both resampling column transforms (its input and output cannot share a
    // buffer), X1 otherwise
    const bool fuse_cols = resample && col_resample_ok(g.Q, g.N);
    float2 *const XN = fuse_cols ? X2 : X1;
    const hipStream_t s = slot == 0 ? s_main : side[slot - 1];
    EpiPtrs ep;
    ep.image = image;
    ep.target = grad && fused ? target : nullptr;
    ep.G = G;
    ep.loss_part = lossp;
    g.p = pl;
    g.pw = plane_w ? plane_w[pl] : 1.0;
    if (prec == LITHO_PREC_FP32 || L.row_mfma)
      LITHO_TRY(run_pass_y_fwd(bk->d_phi, Mh, Y, g, twQ, n, s));
    else
      LITHO_TRY(run_pass_y_fwd_mfma(bk->d_phi, Mh, Y, g, gemm_fwd, prec, n, s));
    if (!resample) {
      LITHO_TRY(run_pass_x_fwd(Y, ep, nullptr, g, twQ, n, s));
    } else {
      if (L.row_mfma)
        LITHO_TRY(run_pass_x_fwd_mfma(Y, X1, g, row_tab, row_tw, twQ, prec, n, s));
      else
        LITHO_TRY(run_pass_x_fwd(Y, EpiPtrs{}, X1, g, twQ, n, s));
      // resist kernel of Eq. 5 on the intensity band: R = I (x) K_resist
      if (fuse_cols) {
        LITHO_TRY(run_col_resample("up_cols", g.Q, g.N, true, X1, XN, g.ntD, h2, twQ, twN, 1.0f, blur, n, s));
      } else {
        LITHO_TRY(run_col_fft("up_cols_q", g.Q, -1, X1, X2, g.ntD, -1, h2, twQ, 1.0f, n, s));
        LITHO_TRY(run_band_gauss(X2, h2, g.ntD, double(g.N), blur, band_clip, n, s));
        LITHO_TRY(run_col_fft("up_cols_n", g.N, +1, X2, XN, g.ntD, h2, -1, twN, 1.0f, n, s));
      }
      if (grad && fused)  // image, loss and the residual's row DFT to the band, in place
        LITHO_TRY(run_rows_image_residual("image_residual_rows", g.N, XN, h2, g.Dp, ep, g, twN, 1.0f, n, s));
      else if (ep.image || ep.target)
        LITHO_TRY(run_rows_inv_real("up_rows", g.N, XN, h2, g.Dp, nullptr, ep, g, twN, 1.0f, n, s));
    }
    if (!grad) continue;
    const float *Gp = fused ? G : grad_image + size_t(pl) * NN;
    const size_t gstride = fused ? NN : size_t(g.P) * NN;
    if (!resample) {
      LITHO_TRY(run_pass_x_adj(Y, Gp, gstride, nullptr, g, twQ, n, s));
    } else {
      // G low-passed to |f| <= 2b and sampled on the Q grid (scaled by 1/Q^2);
      // the fused step's row DFT of G was done by the image row pass
      if (!fused) LITHO_TRY(run_rows_fwd_real("down_rows", g.N, Gp, gstride, XN, h2, g.Dp, twN, 1.0f, n, s));
      // dL/dI = K_resist (x) dL/dR (the Gaussian is symmetric)
      const float qscale = float(1.0 / (double(g.Q) * double(g.Q)));
      if (fuse_cols) {
        LITHO_TRY(run_col_resample("down_cols", g.Q, g.N, false, XN, X1, g.ntD, h2, twQ, twN, qscale, blur, n, s));
      } else {
        LITHO_TRY(run_col_fft("down_cols_n", g.N, -1, XN, X2, g.ntD, -1, h2, twN, 1.0f, n, s));
        LITHO_TRY(run_band_gauss(X2, h2, g.ntD, double(g.N), blur, band_clip, n, s));
        LITHO_TRY(run_col_fft("down_cols_q", g.Q, +1, X2, X1, g.ntD, h2, -1, twQ, qscale, n, s));
      }
      LITHO_TRY(run_pass_x_adj(Y, nullptr, 0, X1, g, twQ, n, s));
    }
    if (prec == LITHO_PREC_FP32 || L.row_mfma)
      LITHO_TRY(run_pass_y_adj(Y, bk->d_phi, part, g, twQ, n, s));
    else
      LITHO_TRY(run_pass_y_adj_mfma(Y, bk->d_phi, part, g, gemm_adj, prec, n, s));
  }
  if (L.pp > 1) {
    // join: the call's stream waits for every side stream
    for (int i = 0; i < L.pp - 1; ++i) {
      LITHO_HIP_TRY(hipEventRecord(ev[1 + i], side[i]));
      LITHO_HIP_TRY(hipStreamWaitEvent(s_main, ev[1 + i], 0));
    }
  }
  if (grad) {
    LITHO_TRY(run_grad_cols(part, g.P * g.KC, S1, g, twN, n, s));
    LITHO_TRY(run_rows_inv_real("grad_rows", g.N, S1, g.b, g.Bp, grad_mask, EpiPtrs{}, g, twN, 2.0f, n, s));
    if (fused && loss) LITHO_TRY(run_loss_reduce(lossp, g.P * L.nblk, loss, n, s));
  }
  return LITHO_OK;
}

}  // namespace litho

static int check_call(const litho_bank *bk, const float *d_mask, int batch, int K_use, int prec,
                      const char *who) {
  if (!bk) {
    set_error("%s: NULL bank", who);
    return LITHO_E_INVALID;
  }
  if (batch < 0) {
    set_error("%s: negative batch", who);
    return LITHO_E_INVALID;
  }
  if (batch > 0 && !d_mask) {
    set_error("%s: NULL mask", who);
    return LITHO_E_INVALID;
  }
  if (K_use < 1 || K_use > bk->host.K) {
    set_error("%s: K_use=%d outside 1..%d", who, K_use, bk->host.K);
    return LITHO_E_INVALID;
  }
  return litho::check_prec(prec, who);
}

namespace litho {

// Per-clip strides of the workspace sections are laid out [section][clip],
// so the kernels see dense per-clip arrays.  run_chunk() expects exactly that.
int image_grad_impl(litho_bank *bk, const float *d_mask, int batch, int K_use, const float *d_target,
                    const litho_resist_t *resist, const float *d_grad_image, float *d_image, double *d_loss,
                    float *d_grad_mask, bool grad, int prec, hipStream_t s, int p0, int p1, char *ext_ws,
                    size_t ext_bytes) {
  if (batch == 0) return LITHO_OK;
  const bool fused = d_target != nullptr;
  CallOpts o;
  if (resist) {
    o.slope = resist->slope;
    o.thr = resist->threshold;
    o.plane_w = resist->plane_weight;
    o.blur_sigma = resist->blur_sigma_px;
    o.loss_l1 = resist->loss == LITHO_LOSS_L1 ? 1 : 0;
  }
  o.p0 = p0;
  o.p1 = p1;
  CallLayout L = plan_call(bk, batch, K_use, grad, fused, prec, o.blur_sigma > 0.0);
  const void *gemm_fwd = nullptr, *gemm_adj = nullptr, *row_tab = nullptr;
  const float2 *row_tw = nullptr;
  if (prec != LITHO_PREC_FP32) {
    const bool bf = prec == LITHO_PREC_BF16X3 || prec == LITHO_PREC_BF16;
    if (L.row_mfma) {
      LITHO_TRY(row_mfma_table(bk, bf, &row_tab, &row_tw));
    } else {
      LITHO_TRY(gemm_table(bk, false, bf, &gemm_fwd));
      if (grad) LITHO_TRY(gemm_table(bk, true, bf, &gemm_adj));
    }
  }
  char *ws = nullptr;
  if (ext_ws) {
    // the caller's buffer (a serve slot's arena): one clip at a time if needed
    L.chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(L.chunk), ext_bytes / L.per_clip)));
    if (ext_bytes < L.per_clip) {
      set_error("litho: a %zu byte workspace is short of the %zu bytes one clip needs", ext_bytes, L.per_clip);
      return LITHO_E_INVALID;
    }
    ws = ext_ws;
  } else {
    LITHO_TRY(acquire_workspace(bk, s, L.per_clip * size_t(L.chunk), &ws));
  }
  const size_t NN = size_t(bk->host.n) * bk->host.n;
  const int P = bk->host.n_focus;
  for (int c0 = 0; c0 < batch; c0 += L.chunk) {
    const int n = std::min(L.chunk, batch - c0);
    LITHO_TRY(run_chunk(bk, L, ws, d_mask + size_t(c0) * NN, n, fused ? d_target + size_t(c0) * NN : nullptr,
                        d_grad_image ? d_grad_image + size_t(c0) * P * NN : nullptr,
                        d_image ? d_image + size_t(c0) * P * NN : nullptr, d_loss ? d_loss + c0 : nullptr,
                        d_grad_mask ? d_grad_mask + size_t(c0) * NN : nullptr, grad, s, o, prec, gemm_fwd,
                        gemm_adj, row_tab, row_tw));
  }
  return LITHO_OK;
}

}  // namespace litho

extern "C" int litho_image(const litho_bank_t *bank, const float *d_mask, int batch, int K_use, float *d_image,
                           int prec, void *hip_stream) {
  clear_error();
  LITHO_TRY(check_call(bank, d_mask, batch, K_use, prec, "litho_image"));
  if (batch > 0 && !d_image) {
    set_error("litho_image: NULL image");
    return LITHO_E_INVALID;
  }
  return image_grad_impl(const_cast<litho_bank *>(bank), d_mask, batch, K_use, nullptr, nullptr, nullptr,
                         d_image, nullptr, nullptr, false, prec, static_cast<hipStream_t>(hip_stream));
}

extern "C" int litho_image_grad(const litho_bank_t *bank, const float *d_mask, int batch, int K_use,
                                const float *d_target, const litho_resist_t *resist, const float *d_grad_image,
                                float *d_image, double *d_loss, float *d_grad_mask, int prec, void *hip_stream) {
  clear_error();
  LITHO_TRY(check_call(bank, d_mask, batch, K_use, prec, "litho_image_grad"));
  if (batch > 0 && !d_grad_mask) {
    set_error("litho_image_grad: NULL gradient output");
    return LITHO_E_INVALID;
  }
  if (d_target && !resist) {
    set_error("litho_image_grad: a target needs resist parameters");
    return LITHO_E_INVALID;
  }
  if (!d_target && !d_grad_image && batch > 0) {
    set_error("litho_image_grad: give either a target (fused loss) or dL/dI (VJP)");
    return LITHO_E_INVALID;
  }
  if (d_target && d_grad_image) {
    set_error("litho_image_grad: target and dL/dI are exclusive");
    return LITHO_E_INVALID;
  }
  if (d_loss && !d_target) {
    set_error("litho_image_grad: the loss exists only in fused mode");
    return LITHO_E_INVALID;
  }
  return image_grad_impl(const_cast<litho_bank *>(bank), d_mask, batch, K_use, d_target, resist, d_grad_image,
                         d_image, d_loss, d_grad_mask, true, prec, static_cast<hipStream_t>(hip_stream));
}

// ============================================================ tracing ABI
extern "C" int litho_profile_enable(int on) {
  clear_error();
  g_prof.store(on != 0);
  return LITHO_OK;
}

extern "C" int litho_profile_read(char *buf, size_t cap) {
  clear_error();
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_recs);
  }
  std::map<std::string, std::pair<long, double>> agg;
  int rc = LITHO_OK;
  for (auto &r : recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      set_error("litho_profile_read: event query failed");
      rc = LITHO_E_HIP;
    }
    auto &a = agg[r.name];
    a.first += 1;
    a.second += ms;
  }
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : recs) {
      g_event_pool.push_back(r.a);
      g_event_pool.push_back(r.b);
    }
  }
  std::string s;
  char tmp[160];
  for (auto &kv : agg) {
    snprintf(tmp, sizeof tmp, "%s=%ld:%.6f;", kv.first.c_str(), kv.second.first, kv.second.second);
    s += tmp;
  }
  if (buf && cap) {
    const size_t n = std::min(cap - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = '\0';
  }
  return rc;
}

extern "C" const char *litho_last_error(void) { return last_error(); }
