// Library-internal state shared by the ABI implementation and the serve loop.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "bank.hpp"
#include "kernels.hpp"

namespace litho {

struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;
};

// Sizes of one call: geometry plus per-clip workspace sections.
struct CallLayout {
  PassGeo g;
  int nblk = 0;    // row-pass blocks per clip and plane (loss partials)
  size_t b_S1 = 0, b_Mh = 0, b_Y = 0, b_G = 0, b_part = 0, b_loss = 0, b_X = 0;
  size_t per_clip = 0;
  int chunk = 1;   // clips per launch sequence
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
  std::mutex mu;
  std::map<hipStream_t, litho::Workspace> ws;
};

namespace litho {
CallLayout plan_call(const litho_bank *bk, int batch, int K_use, bool grad, bool fused, int prec);
int acquire_workspace(litho_bank *bk, hipStream_t s, size_t bytes, char **out);
int image_grad_impl(litho_bank *bk, const float *d_mask, int batch, int K_use, const float *d_target,
                    const litho_resist_t *resist, const float *d_grad_image, float *d_image, double *d_loss,
                    float *d_grad_mask, bool grad, int prec, hipStream_t s);
int check_prec(int prec, const char *who);
}  // namespace litho
