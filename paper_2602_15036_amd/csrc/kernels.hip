// SOCS aerial image and ILT adjoint on gfx950.
//
// Data layout.  Every band-limited intermediate is "tile-major": columns are
// grouped in tiles of kC = 4 adjacent frequency columns, and a tile stores all
// its rows contiguously, [tile][row][kC].  A column pass then reads and writes
// one contiguous block per tile, and a row pass handling kRowsPerChunk rows
// moves kC * rows * 8 bytes contiguous per tile.
//
// Forward per clip (Eq. 4, thin mask):
//   mask_rows   : real rows -> row DFT, keep |kx| <= b, scale 1/N^2   -> S1 [N x Bp]
//   col_fft     : column DFT of S1, keep |ky| <= b                   -> Mh [B x Bp]
// per focus plane and kernel k:
//   pass_y_fwd  : X = Phi'_k * Mh, inverse column DFT (B -> Q rows)  -> Y_k [Q x Bp]
//   pass_x_fwd  : per row, loop k: inverse row DFT of Y_k, |.|^2 accumulate;
//                 epilogue: image, sigmoid resist, loss partial, residual G.
// Adjoint per focus plane:
//   pass_x_adj  : per row, loop k: E_k = inverse row DFT of Y_k (recomputed),
//                 U = G * E_k, forward row DFT, keep |kx| <= b  -> V_k (in place)
//   pass_y_adj  : per column tile, loop k: forward column DFT of V_k, keep
//                 |ky| <= b, acc += conj(Phi'_k) * (.) in FP64     -> partials
// Finish per clip:
//   grad_cols   : sum partials (FP64, fixed order), inverse column DFT -> [N x Bp]
//   row_inv_real: inverse row DFT, 2 Re(.) -> dL/dm
//
// Phi'_k = sqrt(lambda_k) Phi_k, so I = sum_k |E'_k|^2 and the adjoint
// accumulator sum_k conj(Phi'_k) DFT(G E'_k) equals sum_k lambda_k conj(Phi_k) DFT(G E_k).
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "kernels.hpp"

namespace litho {
namespace dev {

constexpr int kC = 4;  // columns per tile

struct Geo {
  int N;      // grid side
  int Q;      // side of the grid the per-kernel transforms run on (== N here)
  int b, B;   // band half-width and side
  int Bp;     // B rounded up to kC
  int nt;     // Bp / kC tiles
  int K;      // kernels used per plane
  int Kbank;  // kernels stored per plane in the bank
  int P;      // planes
  int p;      // current plane
  int KC;     // k-chunks of the adjoint column pass
  int kper;   // kernels per k-chunk
  float dose;
  float slope, thr;
};

__device__ __forceinline__ int band_row_of(int pos, int L, int h) {
  // frequency position pos in [0, L) -> centred band row, or -1 if |f| > h
  if (pos <= h) return pos + h;
  if (pos >= L - h) return pos - L + h;
  return -1;
}

// ------------------------------------------------------------ mask rows
// S1[clip][jt][y][c] = scale * sum_x m[y][x] exp(-2 pi i kx x / N), kx = jt*kC + c - b.
template <int N>
__global__ __launch_bounds__(256) void k_mask_rows(const float *__restrict__ mask, cf *__restrict__ S1,
                                                   Geo g, const cf *__restrict__ tw, float scale) {
  constexpr int T = FftPlan<N>::T, E = N / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  cf *stage = smem;                              // [RPB][Bp]
  cf *xch = smem + RPB * g.Bp;                   // [RPB][lds_len<N>]
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int y0 = blockIdx.x * RPB, y = y0 + row, clip = blockIdx.y;
  const float *src = mask + (size_t(clip) * N + y) * N;
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = cmake(src[t + T * i], 0.0f);
  fft<N, -1>(v, xch + row * lds_len<N>(), t, tw);
  cf *st = stage + row * g.Bp;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int j = band_row_of(t + T * i, N, g.b);
    if (j >= 0) st[j] = cscale(v[i], scale);
  }
  for (int j = g.B + t; j < g.Bp; j += T) st[j] = cmake(0.f, 0.f);
  __syncthreads();
  cf *dst = S1 + size_t(clip) * g.nt * N * kC;
  const int chunk = RPB * kC;
  for (int e = threadIdx.x; e < RPB * g.Bp; e += blockDim.x) {
    const int jt = e / chunk, r = e % chunk, rr = r / kC, c = r % kC;
    dst[(size_t(jt) * N + y0 + rr) * kC + c] = stage[rr * g.Bp + jt * kC + c];
  }
}

// ------------------------------------------------------------ generic column pass
// For each tile column: a length-L DFT along the rows.  Input rows are either
// all L positions (in_h < 0) or a centred band of 2*in_h+1 rows placed at
// frequency positions (row - in_h) mod L; outputs are either all L rows
// (out_h < 0) or the centred band |f| <= out_h.  Values are scaled by `scale`.
template <int L, int DIR>
__global__ __launch_bounds__(512) void k_col_fft(const cf *__restrict__ in, cf *__restrict__ out, int nt,
                                                 int in_h, int out_h, size_t in_clip, size_t out_clip,
                                                 const cf *__restrict__ tw, float scale) {
  constexpr int T = FftPlan<L>::T, E = L / T;
  extern __shared__ cf smem[];
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int jt = blockIdx.x, clip = blockIdx.y;
  cf *buf = smem + c * lds_len<L>();
  const int rin = in_h < 0 ? L : 2 * in_h + 1;
  const int rout = out_h < 0 ? L : 2 * out_h + 1;
  const cf *src = in + clip * in_clip + size_t(jt) * rin * kC;
  cf *dst = out + clip * out_clip + size_t(jt) * rout * kC;
  if (in_h >= 0) {
    for (int e = threadIdx.x; e < kC * L; e += blockDim.x)
      smem[(e / L) * lds_len<L>() + lpad(e % L)] = cmake(0.f, 0.f);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < rin * kC; e += blockDim.x) {
    const int r = e / kC, cc = e % kC;
    int pos = r;
    if (in_h >= 0) pos = r - in_h < 0 ? r - in_h + L : r - in_h;
    smem[cc * lds_len<L>() + lpad(pos)] = src[e];
  }
  __syncthreads();
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = buf[lpad(t + T * i)];
  __syncthreads();
  fft<L, DIR>(v, buf, t, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int pos = t + T * i;
    const int r = out_h < 0 ? pos : band_row_of(pos, L, out_h);
    if (r >= 0) buf[lpad(r)] = cscale(v[i], scale);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rout * kC; e += blockDim.x) {
    const int r = e / kC, cc = e % kC;
    dst[e] = smem[cc * lds_len<L>() + lpad(r)];
  }
}

// ------------------------------------------------------------ forward column pass
// Y_k[jt][y][c] = sum_ky Phi'_k(ky, j) Mh(ky, j) exp(+2 pi i ky y / Q).
template <int Q>
__global__ __launch_bounds__(512) void k_pass_y_fwd(const cf *__restrict__ bank, const cf *__restrict__ Mh,
                                                    cf *__restrict__ Y, Geo g, const cf *__restrict__ tw) {
  constexpr int T = FftPlan<Q>::T, E = Q / T;
  extern __shared__ cf smem[];
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int jt = blockIdx.x, k = blockIdx.y, clip = blockIdx.z;
  cf *buf = smem + c * lds_len<Q>();
  for (int e = threadIdx.x; e < kC * Q; e += blockDim.x)
    smem[(e / Q) * lds_len<Q>() + lpad(e % Q)] = cmake(0.f, 0.f);
  __syncthreads();
  const cf *ph = bank + ((size_t(g.p) * g.Kbank + k) * g.nt + jt) * g.B * kC;
  const cf *mh = Mh + (size_t(clip) * g.nt + jt) * g.B * kC;
  for (int e = threadIdx.x; e < g.B * kC; e += blockDim.x) {
    const int r = e / kC, cc = e % kC;
    const int pos = r - g.b < 0 ? r - g.b + Q : r - g.b;
    smem[cc * lds_len<Q>() + lpad(pos)] = cmul(ph[e], mh[e]);
  }
  __syncthreads();
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = buf[lpad(t + T * i)];
  __syncthreads();
  fft<Q, +1>(v, buf, t, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) buf[lpad(t + T * i)] = v[i];
  __syncthreads();
  cf *dst = Y + ((size_t(clip) * g.K + k) * g.nt + jt) * size_t(Q) * kC;
  for (int e = threadIdx.x; e < Q * kC; e += blockDim.x)
    dst[e] = smem[(e % kC) * lds_len<Q>() + lpad(e / kC)];
}

// Loads rows y0..y0+RPB of one kernel's intermediate (all tiles) into `stage`.
template <int Q, int RPB>
__device__ __forceinline__ void load_band_rows(const cf *__restrict__ src, cf *stage, int y0, const Geo &g) {
  const int chunk = RPB * kC;
  for (int e = threadIdx.x; e < RPB * g.Bp; e += blockDim.x) {
    const int jt = e / chunk, r = e % chunk, rr = r / kC, c = r % kC;
    stage[rr * g.Bp + jt * kC + c] = src[(size_t(jt) * Q + y0 + rr) * kC + c];
  }
}

template <int Q, int RPB>
__device__ __forceinline__ void store_band_rows(cf *__restrict__ dst, const cf *stage, int y0, const Geo &g) {
  const int chunk = RPB * kC;
  for (int e = threadIdx.x; e < RPB * g.Bp; e += blockDim.x) {
    const int jt = e / chunk, r = e % chunk, rr = r / kC, c = r % kC;
    dst[(size_t(jt) * Q + y0 + rr) * kC + c] = stage[rr * g.Bp + jt * kC + c];
  }
}

// ------------------------------------------------------------ forward row pass
// I(y, x) = dose * sum_k |sum_kx Y_k(y, kx) exp(+2 pi i kx x / Q)|^2 and the
// resist epilogue.  Outputs: image (optional), residual G and loss partials
// (when target != nullptr).
template <int Q>
__global__ __launch_bounds__(256) void k_pass_x_fwd(const cf *__restrict__ Y, float *__restrict__ image,
                                                    const float *__restrict__ target, float *__restrict__ G,
                                                    double *__restrict__ loss_part, Geo g,
                                                    const cf *__restrict__ tw) {
  constexpr int T = FftPlan<Q>::T, E = Q / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  cf *stage = smem;
  cf *xch = smem + RPB * g.Bp;
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int y0 = blockIdx.x * RPB, y = y0 + row, clip = blockIdx.y;
  float acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = 0.f;
  const cf *st = stage + row * g.Bp;
  for (int k = 0; k < g.K; ++k) {
    load_band_rows<Q, RPB>(Y + (size_t(clip) * g.K + k) * g.nt * size_t(Q) * kC, stage, y0, g);
    __syncthreads();
    cf v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int j = band_row_of(t + T * i, Q, g.b);
      v[i] = j >= 0 ? st[j] : cmake(0.f, 0.f);
    }
    __syncthreads();
    fft<Q, +1>(v, xch + row * lds_len<Q>(), t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] += cabs2(v[i]);
  }
  const size_t pix = (size_t(clip) * g.P + g.p) * size_t(Q) * Q + size_t(y) * Q;
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int x = t + T * i;
    const float I = acc[i] * g.dose;
    if (image) image[pix + x] = I;
    if (target) {
      const float z = 1.0f / (1.0f + expf(-g.slope * (I - g.thr)));
      const float d = z - target[(size_t(clip) * Q + y) * Q + x];
      G[(size_t(clip) * Q + y) * Q + x] = 2.0f * d * g.slope * z * (1.0f - z);
      lsum += double(d) * double(d);
    }
  }
  if (target) {
    // block reduction in FP64, fixed order
    double *red = reinterpret_cast<double *>(smem);
    __syncthreads();
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[(size_t(clip) * g.P + g.p) * gridDim.x + blockIdx.x] = red[0];
  }
}

// ------------------------------------------------------------ adjoint row pass
// V_k(y, kx) = sum_x G(y, x) E'_k(y, x) exp(-2 pi i kx x / Q), |kx| <= b,
// E'_k recomputed from Y_k; V_k overwrites Y_k.
template <int Q>
__global__ __launch_bounds__(256) void k_pass_x_adj(cf *__restrict__ Y, const float *__restrict__ Gin,
                                                    size_t g_clip_stride, Geo g, const cf *__restrict__ tw) {
  constexpr int T = FftPlan<Q>::T, E = Q / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  cf *stage = smem;
  cf *xch = smem + RPB * g.Bp;
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int y0 = blockIdx.x * RPB, y = y0 + row, clip = blockIdx.y;
  float gr[E];
  const float *gsrc = Gin + clip * g_clip_stride + size_t(y) * Q;
#pragma unroll
  for (int i = 0; i < E; ++i) gr[i] = gsrc[t + T * i] * g.dose;
  cf *st = stage + row * g.Bp;
  for (int k = 0; k < g.K; ++k) {
    cf *yk = Y + (size_t(clip) * g.K + k) * g.nt * size_t(Q) * kC;
    load_band_rows<Q, RPB>(yk, stage, y0, g);
    __syncthreads();
    cf v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int j = band_row_of(t + T * i, Q, g.b);
      v[i] = j >= 0 ? st[j] : cmake(0.f, 0.f);
    }
    __syncthreads();
    fft<Q, +1>(v, xch + row * lds_len<Q>(), t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = cscale(v[i], gr[i]);
    fft<Q, -1>(v, xch + row * lds_len<Q>(), t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int j = band_row_of(t + T * i, Q, g.b);
      if (j >= 0) st[j] = v[i];
    }
    for (int j = g.B + t; j < g.Bp; j += T) st[j] = cmake(0.f, 0.f);
    __syncthreads();
    store_band_rows<Q, RPB>(yk, stage, y0, g);
    __syncthreads();
  }
}

// ------------------------------------------------------------ adjoint column pass
// part[clip][p*KC + kc][jt][ky][c] = sum_{k in chunk} conj(Phi'_k) * sum_y V_k(y, j) exp(-2 pi i ky y / Q)
template <int Q, int U>
__global__ __launch_bounds__(512) void k_pass_y_adj(const cf *__restrict__ V, const cf *__restrict__ bank,
                                                    double2 *__restrict__ part, Geo g,
                                                    const cf *__restrict__ tw) {
  constexpr int T = FftPlan<Q>::T, E = Q / T;
  extern __shared__ cf smem[];
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int jt = blockIdx.x, kc = blockIdx.y, clip = blockIdx.z;
  cf *buf = smem + c * lds_len<Q>();
  const int nE = g.B * kC;
  double2 acc[U];  // band entries e = threadIdx.x + blockDim.x * u, u < U
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = make_double2(0.0, 0.0);
  const int k0 = kc * g.kper, k1 = min(g.K, k0 + g.kper);
  for (int k = k0; k < k1; ++k) {
    const cf *src = V + ((size_t(clip) * g.K + k) * g.nt + jt) * size_t(Q) * kC;
    for (int e = threadIdx.x; e < Q * kC; e += blockDim.x)
      smem[(e % kC) * lds_len<Q>() + lpad(e / kC)] = src[e];
    __syncthreads();
    cf v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = buf[lpad(t + T * i)];
    __syncthreads();
    fft<Q, -1>(v, buf, t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int r = band_row_of(t + T * i, Q, g.b);
      if (r >= 0) buf[lpad(r)] = v[i];
    }
    __syncthreads();
    const cf *ph = bank + ((size_t(g.p) * g.Kbank + k) * g.nt + jt) * g.B * kC;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + blockDim.x * u;
      if (e < nE) {
        const cf val = smem[(e % kC) * lds_len<Q>() + lpad(e / kC)];
        const cf phv = ph[e];
        // conj(phi) * val
        acc[u].x += double(phv.x) * double(val.x) + double(phv.y) * double(val.y);
        acc[u].y += double(phv.x) * double(val.y) - double(phv.y) * double(val.x);
      }
    }
    __syncthreads();
  }
  double2 *dst = part + ((size_t(clip) * g.P * g.KC + size_t(g.p) * g.KC + kc) * g.nt + jt) * size_t(nE);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = threadIdx.x + blockDim.x * u;
    if (e < nE) dst[e] = acc[u];
  }
}

// ------------------------------------------------------------ gradient finish, columns
// Acc = sum over (plane, k-chunk) partials in FP64 (fixed order), scaled by 1/N^2,
// then the inverse column DFT (band rows -> N rows).
template <int N>
__global__ __launch_bounds__(512) void k_grad_cols(const double2 *__restrict__ part, int nparts,
                                                   cf *__restrict__ out, Geo g, const cf *__restrict__ tw) {
  constexpr int T = FftPlan<N>::T, E = N / T;
  extern __shared__ cf smem[];
  const int c = threadIdx.x / T, t = threadIdx.x % T;
  const int jt = blockIdx.x, clip = blockIdx.y;
  cf *buf = smem + c * lds_len<N>();
  for (int e = threadIdx.x; e < kC * N; e += blockDim.x)
    smem[(e / N) * lds_len<N>() + lpad(e % N)] = cmake(0.f, 0.f);
  __syncthreads();
  const int nE = g.B * kC;
  const double inv = 1.0 / (double(N) * double(N));
  for (int e = threadIdx.x; e < nE; e += blockDim.x) {
    double sx = 0.0, sy = 0.0;
    for (int s = 0; s < nparts; ++s) {
      const double2 a = part[((size_t(clip) * nparts + s) * g.nt + jt) * size_t(nE) + e];
      sx += a.x;
      sy += a.y;
    }
    const int r = e / kC, cc = e % kC;
    const int pos = r - g.b < 0 ? r - g.b + N : r - g.b;
    smem[cc * lds_len<N>() + lpad(pos)] = cmake(float(sx * inv), float(sy * inv));
  }
  __syncthreads();
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = buf[lpad(t + T * i)];
  __syncthreads();
  fft<N, +1>(v, buf, t, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) buf[lpad(t + T * i)] = v[i];
  __syncthreads();
  cf *dst = out + (size_t(clip) * g.nt + jt) * size_t(N) * kC;
  for (int e = threadIdx.x; e < N * kC; e += blockDim.x)
    dst[e] = smem[(e % kC) * lds_len<N>() + lpad(e / kC)];
}

// ------------------------------------------------------------ band rows -> real rows
// out[clip][y][x] = scale * Re sum_kx in(y, kx) exp(+2 pi i kx x / N)
template <int N>
__global__ __launch_bounds__(256) void k_rows_inv_real(const cf *__restrict__ in, float *__restrict__ out,
                                                       Geo g, const cf *__restrict__ tw, float scale) {
  constexpr int T = FftPlan<N>::T, E = N / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  cf *stage = smem;
  cf *xch = smem + RPB * g.Bp;
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int y0 = blockIdx.x * RPB, y = y0 + row, clip = blockIdx.y;
  load_band_rows<N, RPB>(in + size_t(clip) * g.nt * N * kC, stage, y0, g);
  __syncthreads();
  const cf *st = stage + row * g.Bp;
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int j = band_row_of(t + T * i, N, g.b);
    v[i] = j >= 0 ? st[j] : cmake(0.f, 0.f);
  }
  __syncthreads();
  fft<N, +1>(v, xch + row * lds_len<N>(), t, tw);
  float *dst = out + (size_t(clip) * N + y) * N;
#pragma unroll
  for (int i = 0; i < E; ++i) dst[t + T * i] = scale * v[i].x;
}

// ------------------------------------------------------------ loss reduction
__global__ __launch_bounds__(256) void k_loss_reduce(const double *__restrict__ part, int n_per_clip,
                                                     double *__restrict__ loss) {
  __shared__ double red[256];
  const int clip = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n_per_clip; i += blockDim.x) s += part[size_t(clip) * n_per_clip + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[clip] = red[0];
}

}  // namespace dev

// ======================================================================== host launchers

namespace {

using dev::cf;
using dev::FftPlan;
using dev::Geo;
using dev::kC;
using dev::lds_len;

dev::Geo to_geo(const PassGeo &pg) {
  Geo g;
  g.N = pg.N; g.Q = pg.Q; g.b = pg.b; g.B = pg.B; g.Bp = pg.Bp; g.nt = pg.nt;
  g.K = pg.K; g.Kbank = pg.Kbank; g.P = pg.P; g.p = pg.p; g.KC = pg.KC; g.kper = pg.kper;
  g.dose = float(pg.dose); g.slope = float(pg.slope); g.thr = float(pg.thr);
  return g;
}

template <typename F>
int launch(const char *name, const void *kernel, dim3 grid, size_t shmem, hipStream_t s, F &&go) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return LITHO_OK;
  if (shmem > 160 * 1024) {
    set_error("%s: %zu bytes of LDS exceed the 160 KiB per workgroup", name, shmem);
    return LITHO_E_UNSUPPORTED;
  }
  if (shmem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(shmem));
    if (e != hipSuccess) {
      set_error("%s: cannot raise the dynamic LDS limit to %zu bytes: %s", name, shmem, hipGetErrorString(e));
      return LITHO_E_HIP;
    }
  }
  prof_begin(name, s);
  go();
  prof_end(name, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s launch failed: %s", name, hipGetErrorString(e));
    return LITHO_E_HIP;
  }
  return LITHO_OK;
}

template <int N>
int mask_spectrum_n(const float *mask, cf *S1, cf *Mh, const PassGeo &pg, const cf *twN, int nclips,
                    hipStream_t s) {
  constexpr int T = FftPlan<N>::T, RPB = 256 / T;
  Geo g = to_geo(pg);
  size_t sh = (size_t(RPB) * g.Bp + size_t(RPB) * lds_len<N>()) * sizeof(cf);
  LITHO_TRY(launch("mask_rows", reinterpret_cast<const void *>(&dev::k_mask_rows<N>), dim3(N / RPB, nclips), sh, s, [&] {
    hipLaunchKernelGGL(dev::k_mask_rows<N>, dim3(N / RPB, nclips), dim3(256), sh, s, mask, S1, g, twN,
                       float(1.0 / (double(N) * double(N))));
  }));
  size_t shc = size_t(kC) * lds_len<N>() * sizeof(cf);
  LITHO_TRY(launch("mask_cols", reinterpret_cast<const void *>(&dev::k_col_fft<N, -1>), dim3(g.nt, nclips), shc, s, [&] {
    hipLaunchKernelGGL((dev::k_col_fft<N, -1>), dim3(g.nt, nclips), dim3(kC * T), shc, s, S1, Mh, g.nt, -1,
                       g.b, size_t(g.nt) * N * kC, size_t(g.nt) * g.B * kC, twN, 1.0f);
  }));
  return LITHO_OK;
}

template <int Q>
int pass_y_fwd_q(const cf *bank, const cf *Mh, cf *Y, const PassGeo &pg, const cf *twQ, int nclips,
                 hipStream_t s) {
  constexpr int T = FftPlan<Q>::T;
  Geo g = to_geo(pg);
  size_t sh = size_t(kC) * lds_len<Q>() * sizeof(cf);
  return launch("pass_y_fwd", reinterpret_cast<const void *>(&dev::k_pass_y_fwd<Q>), dim3(g.nt, g.K, nclips), sh, s, [&] {
    hipLaunchKernelGGL(dev::k_pass_y_fwd<Q>, dim3(g.nt, g.K, nclips), dim3(kC * T), sh, s, bank, Mh, Y, g,
                       twQ);
  });
}

template <int Q>
int pass_x_fwd_q(const cf *Y, float *image, const float *target, float *G, double *loss_part,
                 const PassGeo &pg, const cf *twQ, int nclips, hipStream_t s) {
  constexpr int T = FftPlan<Q>::T, RPB = 256 / T;
  Geo g = to_geo(pg);
  size_t sh = (size_t(RPB) * g.Bp + size_t(RPB) * lds_len<Q>()) * sizeof(cf);
  sh = std::max(sh, size_t(256) * sizeof(double));
  return launch("pass_x_fwd", reinterpret_cast<const void *>(&dev::k_pass_x_fwd<Q>), dim3(Q / RPB, nclips), sh, s, [&] {
    hipLaunchKernelGGL(dev::k_pass_x_fwd<Q>, dim3(Q / RPB, nclips), dim3(256), sh, s, Y, image, target, G,
                       loss_part, g, twQ);
  });
}

template <int Q>
int pass_x_adj_q(cf *Y, const float *G, size_t g_clip_stride, const PassGeo &pg, const cf *twQ, int nclips,
                 hipStream_t s) {
  constexpr int T = FftPlan<Q>::T, RPB = 256 / T;
  Geo g = to_geo(pg);
  size_t sh = (size_t(RPB) * g.Bp + size_t(RPB) * lds_len<Q>()) * sizeof(cf);
  return launch("pass_x_adj", reinterpret_cast<const void *>(&dev::k_pass_x_adj<Q>), dim3(Q / RPB, nclips), sh, s, [&] {
    hipLaunchKernelGGL(dev::k_pass_x_adj<Q>, dim3(Q / RPB, nclips), dim3(256), sh, s, Y, G, g_clip_stride, g,
                       twQ);
  });
}

template <int Q, int U>
int pass_y_adj_qu(const cf *V, const cf *bank, double2 *part, const PassGeo &pg, const cf *twQ, int nclips,
                  hipStream_t s) {
  constexpr int T = FftPlan<Q>::T;
  Geo g = to_geo(pg);
  size_t sh = size_t(kC) * lds_len<Q>() * sizeof(cf);
  return launch("pass_y_adj", reinterpret_cast<const void *>(&dev::k_pass_y_adj<Q, U>), dim3(g.nt, g.KC, nclips), sh, s, [&] {
    hipLaunchKernelGGL((dev::k_pass_y_adj<Q, U>), dim3(g.nt, g.KC, nclips), dim3(kC * T), sh, s, V, bank, part,
                       g, twQ);
  });
}

// The accumulator holds ceil(B / T) band entries per thread; pick the
// smallest register array that covers them.
template <int Q>
int pass_y_adj_q(const cf *V, const cf *bank, double2 *part, const PassGeo &pg, const cf *twQ, int nclips,
                 hipStream_t s) {
  constexpr int T = FftPlan<Q>::T;
  const int need = (pg.B + T - 1) / T;
  if (need <= 2) return pass_y_adj_qu<Q, 2>(V, bank, part, pg, twQ, nclips, s);
  if (need <= 4) return pass_y_adj_qu<Q, 4>(V, bank, part, pg, twQ, nclips, s);
  if (need <= 8) return pass_y_adj_qu<Q, 8>(V, bank, part, pg, twQ, nclips, s);
  if (need <= 16) return pass_y_adj_qu<Q, 16>(V, bank, part, pg, twQ, nclips, s);
  set_error("pass_y_adj: band side %d too large for %d threads per column", pg.B, T);
  return LITHO_E_UNSUPPORTED;
}

template <int N>
int grad_finish_n(const double2 *part, int nparts, cf *tmp, float *grad, const PassGeo &pg, const cf *twN,
                  int nclips, hipStream_t s) {
  constexpr int T = FftPlan<N>::T, RPB = 256 / T;
  Geo g = to_geo(pg);
  size_t shc = size_t(kC) * lds_len<N>() * sizeof(cf);
  LITHO_TRY(launch("grad_cols", reinterpret_cast<const void *>(&dev::k_grad_cols<N>), dim3(g.nt, nclips), shc, s, [&] {
    hipLaunchKernelGGL(dev::k_grad_cols<N>, dim3(g.nt, nclips), dim3(kC * T), shc, s, part, nparts, tmp, g,
                       twN);
  }));
  size_t sh = (size_t(RPB) * g.Bp + size_t(RPB) * lds_len<N>()) * sizeof(cf);
  return launch("grad_rows", reinterpret_cast<const void *>(&dev::k_rows_inv_real<N>), dim3(N / RPB, nclips), sh, s, [&] {
    hipLaunchKernelGGL(dev::k_rows_inv_real<N>, dim3(N / RPB, nclips), dim3(256), sh, s, tmp, grad, g, twN,
                       2.0f);
  });
}

}  // namespace

#define LITHO_DISPATCH_N(n, CALL)                 \
  switch (n) {                                    \
    case 64: { constexpr int NN = 64; return CALL; }     \
    case 128: { constexpr int NN = 128; return CALL; }   \
    case 256: { constexpr int NN = 256; return CALL; }   \
    case 512: { constexpr int NN = 512; return CALL; }   \
    case 1024: { constexpr int NN = 1024; return CALL; } \
    case 2048: { constexpr int NN = 2048; return CALL; } \
    case 4096: { constexpr int NN = 4096; return CALL; } \
    default:                                      \
      set_error("unsupported transform length %d", n); \
      return LITHO_E_UNSUPPORTED;                 \
  }

int run_mask_spectrum(const float *mask, cf2 *S1, cf2 *Mh, const PassGeo &pg, const cf2 *twN, int nclips,
                      hipStream_t s) {
  LITHO_DISPATCH_N(pg.N, (mask_spectrum_n<NN>(mask, (cf *)S1, (cf *)Mh, pg, (const cf *)twN, nclips, s)));
}
int run_pass_y_fwd(const cf2 *bank, const cf2 *Mh, cf2 *Y, const PassGeo &pg, const cf2 *twQ, int nclips,
                   hipStream_t s) {
  LITHO_DISPATCH_N(pg.Q, (pass_y_fwd_q<NN>((const cf *)bank, (const cf *)Mh, (cf *)Y, pg, (const cf *)twQ,
                                           nclips, s)));
}
int run_pass_x_fwd(const cf2 *Y, float *image, const float *target, float *G, double *loss_part,
                   const PassGeo &pg, const cf2 *twQ, int nclips, hipStream_t s) {
  LITHO_DISPATCH_N(pg.Q, (pass_x_fwd_q<NN>((const cf *)Y, image, target, G, loss_part, pg, (const cf *)twQ,
                                           nclips, s)));
}
int run_pass_x_adj(cf2 *Y, const float *G, size_t g_clip_stride, const PassGeo &pg, const cf2 *twQ, int nclips,
                   hipStream_t s) {
  LITHO_DISPATCH_N(pg.Q, (pass_x_adj_q<NN>((cf *)Y, G, g_clip_stride, pg, (const cf *)twQ, nclips, s)));
}
int run_pass_y_adj(const cf2 *V, const cf2 *bank, double2 *part, const PassGeo &pg, const cf2 *twQ, int nclips,
                   hipStream_t s) {
  LITHO_DISPATCH_N(pg.Q, (pass_y_adj_q<NN>((const cf *)V, (const cf *)bank, part, pg, (const cf *)twQ, nclips,
                                           s)));
}
int run_grad_finish(const double2 *part, int nparts, cf2 *tmp, float *grad, const PassGeo &pg, const cf2 *twN,
                    int nclips, hipStream_t s) {
  LITHO_DISPATCH_N(pg.N, (grad_finish_n<NN>(part, nparts, (cf *)tmp, grad, pg, (const cf *)twN, nclips, s)));
}
int run_loss_reduce(const double *part, int n_per_clip, double *loss, int nclips, hipStream_t s) {
  return launch("loss_reduce", reinterpret_cast<const void *>(&dev::k_loss_reduce), dim3(nclips), 0, s, [&] {
    hipLaunchKernelGGL(dev::k_loss_reduce, dim3(nclips), dim3(256), 0, s, part, n_per_clip, loss);
  });
}

int pass_threads(int L) {
  switch (L) {
    case 64: return FftPlan<64>::T;
    case 128: return FftPlan<128>::T;
    case 256: return FftPlan<256>::T;
    case 512: return FftPlan<512>::T;
    case 1024: return FftPlan<1024>::T;
    case 2048: return FftPlan<2048>::T;
    case 4096: return FftPlan<4096>::T;
    default: return 0;
  }
}

}  // namespace litho
