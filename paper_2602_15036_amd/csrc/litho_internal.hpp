// Library-internal state shared by the ABI implementation and the serve loop.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "bank.hpp"
#include "kernels.hpp"

namespace litho {

struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;
  // side streams (default priority) and fork/join events for focus planes
  // run concurrently with the call's own stream, created on first use
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
};

// Sizes of one call: geometry plus per-clip workspace sections.
struct CallLayout {
  PassGeo g;
  int nblk = 0;    // row-pass blocks per clip and plane (loss partials)
  bool resample = false;  // image carried through the 4b+1 intensity band (Q < N, or a resist blur)
  bool row_mfma = false;  // split modes: two-stage MFMA forward row pass, FP32 column passes
  int pp = 1;      // focus planes run concurrently (each with its own Y, G and band buffers)
  size_t b_S1 = 0, b_Mh = 0, b_Y = 0, b_G = 0, b_part = 0, b_loss = 0, b_X = 0;
  size_t per_clip = 0;
  int chunk = 1;   // clips per launch sequence
};

// Options of one imaging / adjoint call beyond the batch.
struct CallOpts {
  double slope = 0.0, thr = 0.0;    // sigmoid resist (fused loss)
  const double *plane_w = nullptr;  // per-plane loss weights or nullptr
  double blur_sigma = 0.0;          // Gaussian resist kernel (pixels), fused loss only
  int loss_l1 = 0;                  // fused loss: 1 = |Z - T|, 0 = (Z - T)^2
  int p0 = 0, p1 = -1;              // focus planes [p0, p1) to image (p1 < 0: all)
};

size_t workspace_limit_bytes();
bool supported_side(int n);

}  // namespace litho

struct litho_bank {
  litho::HostBank host;
  int Bp = 0, nt = 0, Q = 0;
  int device = 0;
  float2 *d_phi = nullptr;   // [P][K][nt][B][4], sqrt(lambda) folded in
  size_t phi_bytes = 0;
  float2 *d_twN = nullptr;   // exp(-2 pi i e / N)
  float2 *d_twQ = nullptr;   // exp(-2 pi i e / Q)
  // band DFT-GEMM tables for Q, built on first use: [forward FP16, forward BF16, adjoint FP16, adjoint BF16]
  void *d_gemm[4] = {nullptr, nullptr, nullptr, nullptr};
  // two-stage row transform operands for Q, built on first use: [FP16, BF16], and its twiddles
  void *d_rowmma[2] = {nullptr, nullptr};
  float2 *d_rowtw = nullptr;
  std::mutex mu;
  std::map<hipStream_t, litho::Workspace> ws;
  // second per-stream workspace for calls that hold buffers across an imaging call
  std::map<hipStream_t, litho::Workspace> aux;
  // combined kernels of the Eq. 9 sensitivity per (plane, K_use), built on first use
  std::map<std::pair<int, int>, double2 *> psi;
};

namespace litho {
CallLayout plan_call(const litho_bank *bk, int batch, int K_use, bool grad, bool fused, int prec,
                     bool blur = false);
int acquire_workspace(litho_bank *bk, hipStream_t s, size_t bytes, char **out);
int image_grad_impl(litho_bank *bk, const float *d_mask, int batch, int K_use, const float *d_target,
                    const litho_resist_t *resist, const float *d_grad_image, float *d_image, double *d_loss,
                    float *d_grad_mask, bool grad, int prec, hipStream_t s, int p0 = 0, int p1 = -1,
                    char *ext_ws = nullptr, size_t ext_bytes = 0);
int check_prec(int prec, const char *who);
int acquire_aux(litho_bank *bk, hipStream_t s, size_t bytes, char **out);
int plane_streams(litho_bank *bk, hipStream_t s, int count, hipStream_t *side, hipEvent_t *ev);
}  // namespace litho
