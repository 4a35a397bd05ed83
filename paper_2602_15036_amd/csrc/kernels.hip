// SOCS aerial image and ILT adjoint on gfx950.
//
// Data layout.  Every band-limited intermediate is "tile-major": columns are
// grouped in tiles of kC = 4 adjacent frequency columns, and a tile stores all
// its rows contiguously, [tile][row][kC].  A column pass then reads and writes
// one contiguous block per tile, and a row pass handling RPB rows moves
// RPB * kC * 8 bytes contiguous per tile.
//
// Grids.  The mask and the outputs live on the N x N grid.  The coherent
// fields E_k are band-limited to |f| <= b, so |E_k|^2 is band-limited to
// |f| <= 2b: sampling the per-kernel work on a Q x Q grid with Q >= 4b + 1 is
// exact, and the image is carried to the N grid by one zero-padded transform
// per clip.  Q == N skips that step.
//
// Forward per clip (Eq. 4, thin mask):
//   rows_fwd_real : real rows -> row DFT, keep |kx| <= b, scale 1/N^2    -> S1 [N x Bp]
//   col_fft       : column DFT of S1, keep |ky| <= b                     -> Mh [B x Bp]
// per focus plane:
//   pass_y_fwd    : per kernel k: X = Phi'_k * Mh, inverse column DFT (B -> Q rows) -> Y_k
//   pass_x_fwd    : per row, loop k: inverse row DFT of Y_k, |.|^2 accumulate; then
//                   Q == N: image + sigmoid resist + loss partial + residual G;
//                   Q <  N: forward row DFT of the Q-grid image, keep |gx| <= 2b
//   (Q < N)  col_fft<Q, -1> keep |gy| <= 2b, col_fft<N, +1> -> rows_inv_real<N>
//            with the image / resist epilogue
// Adjoint per focus plane:
//   (Q < N)  rows_fwd_real<N> of G keep |gx| <= 2b, col_fft<N, -1> keep |gy| <= 2b,
//            col_fft<Q, +1> -> G on the Q grid as a band
//   pass_x_adj    : per row: G row; loop k: E_k = inverse row DFT of Y_k
//                   (recomputed), U = G E_k, forward row DFT, keep |kx| <= b -> V_k
//   pass_y_adj    : per column tile, loop k: forward column DFT of V_k, keep |ky| <= b,
//                   acc += conj(Phi'_k) (.) in FP64 -> partials
// Finish per clip:
//   grad_cols     : sum partials (FP64, fixed order), inverse column DFT -> [N x Bp]
//   rows_inv_real : inverse row DFT, 2 Re(.) -> dL/dm
//
// Phi'_k = sqrt(lambda_k) Phi_k, so I = sum_k |E'_k|^2 and the adjoint
// accumulator sum_k conj(Phi'_k) DFT(G E'_k) equals sum_k lambda_k conj(Phi_k) DFT(G E_k).
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

namespace litho {
namespace dev {

constexpr int kC = 4;  // columns per tile

struct Geo {
  int N;      // grid side
  int Q;      // per-kernel grid side
  int b, B;   // band half-width and side
  int Bp;     // B rounded up to kC
  int nt;     // Bp / kC tiles
  int D, Dp, ntD;  // intensity band 4b + 1, padded, tiles
  int K;      // kernels used per plane
  int Kbank;  // kernels stored per plane in the bank
  int P;      // planes
  int p;      // current plane
  int KC;     // k-chunks of the adjoint column pass
  int kper;   // kernels per k-chunk
  float dose;
  float slope, thr;
  float pw;   // weight of the current plane's loss
  int loss_l1;  // 1: |Z - T| loss, 0: (Z - T)^2
};

// Outputs of the image epilogue (image, resist, loss, residual).
struct Epi {
  float *image;            // [clip][P][N][N] or nullptr
  const float *target;     // [clip][N][N] or nullptr (no resist)
  float *G;                // [clip][N][N] residual dL/dI (when target)
  double *loss_part;       // [clip][P][nblk]
};

// Band row of FFT position p in [0, L) for the band |f| <= h (2h < L):
// p + h for p <= h, p - L + h for p >= L - h.  As the unsigned minimum of
// p + h and p + h - L it is below 2h + 1 exactly for band positions.
__device__ __forceinline__ unsigned band_row_u(int p, int L, int h) {
  const unsigned q = unsigned(p + h);
  return min(q, q - unsigned(L));
}

// frequency position pos in [0, L) -> centred band row, or -1 if |f| > h (2h < L)
__device__ __forceinline__ int band_row_of(int pos, int L, int h) {
  const unsigned j = band_row_u(pos, L, h);
  return j < unsigned(2 * h + 1) ? int(j) : -1;
}

__device__ __forceinline__ int pos_of_band_row(int r, int h, int L) {
  return r - h < 0 ? r - h + L : r - h;
}

// Pruning.  Register element i of a length-L transform holds positions
// t + T*i, t < T.  When the band half-width h is at most (L - 1) / 4 (always
// on an inner grid Q >= 4b + 1), elements lying strictly between the two band
// edges for every lane are zero on input and unused on output.  Kernels built
// with PR = true state this at compile time, so the first FFT pass folds the
// zeros and the last pass drops the outputs nobody reads.
template <int L>
__host__ __device__ constexpr bool never_in_band(int i) {
  constexpr int T = FftPlan<L>::T, H = (L - 1) / 4;
  return T * i > H && T * i + T - 1 < L - H;
}
template <int L>
inline bool prunable(int h) { return h <= (L - 1) / 4; }

// Band row |f| <= h of row y of a tiled array [tiles][L][kC], read straight
// into the FFT register layout (thread t holds positions t + T*i).
template <int L, int T, bool PR = false>
__device__ __forceinline__ void load_band_row(cf (&v)[L / T], const cf *__restrict__ src, int y, int t, int h) {
  t = opaque_lane(t);
  const cf *row = src + size_t(y) * kC;
  const unsigned W = unsigned(2 * h + 1);
#pragma unroll
  for (int i = 0; i < L / T; ++i) {
    if (PR && never_in_band<L>(i)) {
      v[i] = cmake(0.f, 0.f);
      continue;
    }
    const unsigned j = band_row_u(t + T * i, L, h);
    v[i] = j < W ? row[(j >> 2) * unsigned(L * kC) + (j & 3)] : cmake(0.f, 0.f);
  }
}

// Writes the band |f| <= h of a row held in the FFT register layout (scaled)
// into row y of a tiled array, and zeros in its Wp - (2h+1) pad columns.
template <int L, int T, bool PR = false>
__device__ __forceinline__ void store_band_row(const cf (&v)[L / T], cf *__restrict__ dst, int y, int t, int h,
                                               int Wp, float scale) {
  t = opaque_lane(t);
  cf *row = dst + size_t(y) * kC;
  const unsigned W = unsigned(2 * h + 1);
#pragma unroll
  for (int i = 0; i < L / T; ++i) {
    if (PR && never_in_band<L>(i)) continue;
    const unsigned j = band_row_u(t + T * i, L, h);
    if (j < W) row[(j >> 2) * unsigned(L * kC) + (j & 3)] = cscale(v[i], scale);
  }
  for (unsigned j = W + t; j < unsigned(Wp); j += T) row[(j >> 2) * unsigned(L * kC) + (j & 3)] = cmake(0.f, 0.f);
}

// Raw buffer view of the uniform byte range [base, base + bytes).  Buffer
// range checking makes a load at an offset at or beyond `bytes` return zero
// and drops a store there, so positions off the band need neither a branch
// nor an address of their own.
constexpr unsigned kOffBand = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_view(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, int(bytes), 0x00020000);
}
// (whole-vector bit casts: a cast of one element of the loaded vector reads
// element 0 with this compiler)
using f2v = float __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cf buf_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const f2v f = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(r, int(off), 0, 0));
  return cmake(f.x, f.y);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, cf v) {
  using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  f2v f;
  f.x = v.x;
  f.y = v.y;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, f), r, int(off), 0, 0);
}

using d2v = double __attribute__((ext_vector_type(2)));
__device__ __forceinline__ d2v buf_load_d2(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, int(off), 0, 0));
}

// Byte offsets of the band row |f| <= h of row y of a tiled array
// [tiles][L][kC] in the FFT register layout (thread t holds positions
// t + T*i); kOffBand off the band.  Elements that the pruned variant never
// touches get no offset.
template <int L, int T, bool PR>
__device__ __forceinline__ void band_row_offsets(unsigned (&off)[L / T], int y, int t, int h) {
  t = opaque_lane(t);
  const unsigned W = unsigned(2 * h + 1), row = unsigned(y) * kC;
#pragma unroll
  for (int i = 0; i < L / T; ++i) {
    off[i] = kOffBand;
    if (PR && never_in_band<L>(i)) continue;
    const unsigned j = band_row_u(t + T * i, L, h);
    if (j < W) off[i] = ((j >> 2) * unsigned(L * kC) + (j & 3) + row) * unsigned(sizeof(cf));
  }
}

template <int L, int T, bool PR>
__device__ __forceinline__ void load_band_row_buf(cf (&v)[L / T], __amdgpu_buffer_rsrc_t r,
                                                  const unsigned (&off)[L / T]) {
#pragma unroll
  for (int i = 0; i < L / T; ++i) v[i] = PR && never_in_band<L>(i) ? cmake(0.f, 0.f) : buf_load(r, off[i]);
}

// Stores the band of a row (scaled); the Wp - (2h+1) pad columns are written
// with zeros by the threads t < Wp - (2h+1).
template <int L, int T, bool PR>
__device__ __forceinline__ void store_band_row_buf(const cf (&v)[L / T], __amdgpu_buffer_rsrc_t r,
                                                   const unsigned (&off)[L / T], int y, int t, int h, int Wp,
                                                   float scale) {
#pragma unroll
  for (int i = 0; i < L / T; ++i)
    if (!(PR && never_in_band<L>(i))) buf_store(r, off[i], cscale(v[i], scale));
  for (unsigned j = unsigned(2 * h + 1 + t); j < unsigned(Wp); j += T)
    buf_store(r, ((j >> 2) * unsigned(L * kC) + (j & 3) + unsigned(y) * kC) * unsigned(sizeof(cf)), cmake(0.f, 0.f));
}

// One band row of a tiled array [tiles][L][kC] of `bytes` bytes at a uniform
// base, through buffer loads/stores (offsets formed here, once per row).
template <int L, int T, bool PR = false>
__device__ __forceinline__ void load_band_row_v(cf (&v)[L / T], const cf *base, unsigned bytes, int y, int t,
                                                int h) {
  unsigned off[L / T];
  band_row_offsets<L, T, PR>(off, y, t, h);
  load_band_row_buf<L, T, PR>(v, buf_view(base, bytes), off);
}
template <int L, int T, bool PR = false>
__device__ __forceinline__ void store_band_row_v(const cf (&v)[L / T], cf *base, unsigned bytes, int y, int t,
                                                 int h, int Wp, float scale) {
  unsigned off[L / T];
  band_row_offsets<L, T, PR>(off, y, t, h);
  store_band_row_buf<L, T, PR>(v, buf_view(base, bytes), off, y, t, h, Wp, scale);
}

// Band-row I/O of the k-loop row passes over a tiled array [tiles][Q][kC]
// per kernel (kernel k at base + k * kstride).  The buffer form keeps the
// loop-invariant byte offsets of this thread's band positions in registers
// (pruned variants: half the positions); the plain form recomputes addresses
// per access and is kept where the offsets would not fit: unpruned variants
// and the long transforms of mixed radix.
template <int Q, bool PR>
struct BufRows {
  static constexpr bool value = PR && (FftPlan<Q>::T <= 32 || (Q & (Q - 1)) == 0);
};
template <int Q, int T, bool PR, bool BUF = BufRows<Q, PR>::value>
struct RowIO {
  unsigned off[Q / T];
  unsigned kbytes;
  int y, t, h;
  __device__ __forceinline__ RowIO(size_t kstride, int y_, int t_, int h_)
      : kbytes(unsigned(kstride * sizeof(cf))), y(y_), t(t_), h(h_) {
    band_row_offsets<Q, T, PR>(off, y, t, h);
  }
  __device__ __forceinline__ void load(cf (&v)[Q / T], const cf *base) const {
    load_band_row_buf<Q, T, PR>(v, buf_view(base, kbytes), off);
  }
  __device__ __forceinline__ void store(const cf (&v)[Q / T], cf *base, int Wp, float scale) const {
    store_band_row_buf<Q, T, PR>(v, buf_view(base, kbytes), off, y, t, h, Wp, scale);
  }
};
template <int Q, int T, bool PR>
struct RowIO<Q, T, PR, false> {
  int y, t, h;
  __device__ __forceinline__ RowIO(size_t, int y_, int t_, int h_) : y(y_), t(t_), h(h_) {}
  __device__ __forceinline__ void load(cf (&v)[Q / T], const cf *base) const {
    load_band_row<Q, T, PR>(v, base, y, t, h);
  }
  __device__ __forceinline__ void store(const cf (&v)[Q / T], cf *base, int Wp, float scale) const {
    store_band_row<Q, T, PR>(v, base, y, t, h, Wp, scale);
  }
};

// Block-wide FP64 sum in fixed order; `red` holds blockDim.x doubles.
__device__ __forceinline__ double block_sum(double v, double *red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// Image epilogue over row y of the N grid, held in the FFT register layout
// (thread t holds x = t + T*i): image write, sigmoid resist Z, residual
// G = 2 w (Z - T) a Z (1 - Z); returns the row's w (Z - T)^2 (0 without
// target), w the plane's loss weight.  Row pointers are formed once, so every
// access is the row base plus an immediate offset; the target row is read
// beforehand (load_target_row) so that its latency overlaps the transform.
template <int E, int T>
__device__ __forceinline__ void load_target_row(const Epi &ep, const Geo &g, int clip, int y, int t,
                                                float (&tg)[E]) {
#pragma unroll
  for (int i = 0; i < E; ++i) tg[i] = 0.f;
  if (!ep.target) return;
  const float *src = ep.target + (size_t(clip) * g.N + y) * g.N + t;
#pragma unroll
  for (int i = 0; i < E; ++i) tg[i] = src[T * i];
}
// The epilogue's values, with the residual row left in registers (gr; zero
// without target).
template <int E, int T>
__device__ __forceinline__ double image_epilogue_regs(const Epi &ep, const Geo &g, int clip, int y, int t,
                                                      const float (&I)[E], const float (&tg)[E], float (&gr)[E]) {
  const size_t NN = size_t(g.N) * g.N, ro = size_t(y) * g.N + t;
  if (ep.image) {
    float *img = ep.image + (size_t(clip) * g.P + g.p) * NN + ro;
#pragma unroll
    for (int i = 0; i < E; ++i) img[T * i] = I[i];
  }
#pragma unroll
  for (int i = 0; i < E; ++i) gr[i] = 0.f;
  if (!ep.target) return 0.0;
  double l = 0.0;
  if (g.loss_l1) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const float z = 1.0f / (1.0f + expf(-g.slope * (I[i] - g.thr)));
      const float d = z - tg[i];
      const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      gr[i] = g.pw * sg * g.slope * z * (1.0f - z);
      l += double(g.pw) * double(fabsf(d));
    }
    return l;
  }
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const float z = 1.0f / (1.0f + expf(-g.slope * (I[i] - g.thr)));
    const float d = z - tg[i];
    gr[i] = 2.0f * g.pw * d * g.slope * z * (1.0f - z);
    l += double(g.pw) * double(d) * double(d);
  }
  return l;
}
template <int E, int T>
__device__ __forceinline__ double image_epilogue_row(const Epi &ep, const Geo &g, int clip, int y, int t,
                                                     const float (&I)[E], const float (&tg)[E]) {
  float gr[E];
  const double l = image_epilogue_regs<E, T>(ep, g, clip, y, t, I, tg, gr);
  if (ep.target) {
    float *G = ep.G + size_t(clip) * g.N * g.N + size_t(y) * g.N + t;
#pragma unroll
    for (int i = 0; i < E; ++i) G[T * i] = gr[i];
  }
  return l;
}

// ------------------------------------------------------------ real rows -> band
// Row passes are wavefront-autonomous: each wavefront owns 64 / T rows, reads
// and writes them straight from global memory and exchanges only through its
// own LDS rows, so these kernels need no block barriers (T <= 64).
//
// out[clip][jt][y][c] = scale * sum_x in[y][x] exp(-2 pi i kx x / L), |kx| <= h,
// kx = jt*kC + c - h; the Wp - (2h+1) pad columns are written as zeros.
// Two real rows share one complex transform: Z = DFT(r0 + i r1) gives
// DFT(r0)[k] = (Z[k] + conj Z[-k]) / 2 and DFT(r1)[k] = (Z[k] - conj Z[-k]) / 2i,
// with Z[-k] read back through the transform's LDS region.
template <int L, bool PR>
__global__ __launch_bounds__(256) void k_rows_fwd_real(const float *__restrict__ in, size_t in_clip,
                                                       cf *__restrict__ out, int h, int Wp,
                                                       const cf *__restrict__ tw, float scale) {
  constexpr int T = FftPlan<L>::T, E = L / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  // rows y0, y0 + 1; a block past the last pair (L / RPB odd) recomputes the
  // last pair and stores nothing
  const int yp = 2 * (blockIdx.x * RPB + row), clip = blockIdx.y;
  const bool store = yp < L;
  const int y0 = store ? yp : L - 2;
  const float *src = in + clip * in_clip + size_t(y0) * L;
  cf *buf = smem + row * lds_len<L>();
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = cmake(src[t + T * i], src[L + t + T * i]);
  fft<L, -1>(v, buf, t, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) buf[t + T * i] = v[i];
  xsync<T>();
  cf w[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int p = t + T * i;
    const cf a = v[i], b = buf[p == 0 ? 0 : L - p];
    v[i] = cmake(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    w[i] = cmake(0.5f * (a.y + b.y), 0.5f * (b.x - a.x));
  }
  if (!store) return;
  cf *dst = out + size_t(clip) * (Wp / kC) * L * kC;
  const unsigned bytes = unsigned(size_t(Wp) * L * sizeof(cf));
  store_band_row_v<L, T, PR>(v, dst, bytes, y0, t, h, Wp, scale);
  store_band_row_v<L, T, PR>(w, dst, bytes, y0 + 1, t, h, Wp, scale);
}

// ------------------------------------------------------------ band rows -> real rows
// v = sum_kx in(y, kx) exp(+2 pi i kx x / L); MODE 0: out[y][x] = scale Re v;
// MODE 2: out[y][x] = 1 where scale Re v >= g.thr, else 0;
// MODE 1: I = scale Re v through the image / resist epilogue (L == N).  The
// image rows are real, so their band rows are Hermitian and MODE 1 sends two
// rows through one complex transform: X_y0 + i X_y1 yields row y0 in the real
// part and row y1 in the imaginary part (rows 2 (block RPB + row) and + 1).
template <int L, int MODE, bool PR>
__global__ __launch_bounds__(256) void k_rows_inv_real(const cf *__restrict__ in, int h, int Wp,
                                                       float *__restrict__ out, Epi ep, Geo g,
                                                       const cf *__restrict__ tw, float scale) {
  constexpr int T = FftPlan<L>::T, E = L / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int clip = blockIdx.y;
  const cf *src = in + size_t(clip) * (Wp / kC) * L * kC;
  cf v[E];
  if constexpr (MODE != 1) {
    const int y = blockIdx.x * RPB + row;
    load_band_row_v<L, T, PR>(v, src, unsigned(size_t(Wp) * L * sizeof(cf)), y, t, h);
    fft<L, +1>(v, smem + row * lds_len<L>(), t, tw);
    float *dst = out + (size_t(clip) * L + y) * L;
    if constexpr (MODE == 0) {
#pragma unroll
      for (int i = 0; i < E; ++i) dst[t + T * i] = scale * v[i].x;
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) dst[t + T * i] = scale * v[i].x >= g.thr ? 1.0f : 0.0f;
    }
  } else {
    // a block past the last pair (L / RPB odd) recomputes it and stores nothing
    const int yp = 2 * (blockIdx.x * RPB + row);
    const bool store = yp < L;
    const int y0 = store ? yp : L - 2;
    cf b[E];
    const unsigned bytes = unsigned(size_t(Wp) * L * sizeof(cf));
    load_band_row_v<L, T, PR>(v, src, bytes, y0, t, h);
    load_band_row_v<L, T, PR>(b, src, bytes, y0 + 1, t, h);
    float tg0[E], tg1[E];
    load_target_row<E, T>(ep, g, clip, y0, t, tg0);
    load_target_row<E, T>(ep, g, clip, y0 + 1, t, tg1);
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = cmake(v[i].x - b[i].y, v[i].y + b[i].x);
    fft<L, +1>(v, smem + row * lds_len<L>(), t, tw);
    double lsum = 0.0;
    if (store) {
      float I0[E], I1[E];
#pragma unroll
      for (int i = 0; i < E; ++i) {
        I0[i] = scale * v[i].x;
        I1[i] = scale * v[i].y;
      }
      lsum = image_epilogue_row<E, T>(ep, g, clip, y0, t, I0, tg0) +
             image_epilogue_row<E, T>(ep, g, clip, y0 + 1, t, I1, tg1);
    }
    if (ep.target) {
      const double s = block_sum(lsum, reinterpret_cast<double *>(smem));
      if (threadIdx.x == 0) ep.loss_part[(size_t(clip) * g.P + g.p) * gridDim.x + blockIdx.x] = s;
    }
  }
}

// ------------------------------------------------------------ image rows -> residual band rows
// The resampled ILT step's row pass on the N grid: rows y0, y0 + 1 of the
// image band (two Hermitian rows through one complex transform, as MODE 1
// above), the image / resist / loss epilogue, then the residual rows G_y0,
// G_y0+1 through one forward complex transform, split as in k_rows_fwd_real,
// and their band |gx| <= h stored over the image band rows they came from
// (each wavefront reads its two rows completely before writing them; a
// wavefront past the last pair reads nothing).  The residual never goes to
// HBM.
template <int L, bool PR>
__global__ __launch_bounds__(256) void k_rows_image_residual(cf *band, int h, int Wp, Epi ep, Geo g,
                                                             const cf *__restrict__ tw, float scale) {
  constexpr int T = FftPlan<L>::T, E = L / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int clip = blockIdx.y;
  cf *rows = band + size_t(clip) * (Wp / kC) * L * kC;
  const unsigned bytes = unsigned(size_t(Wp) * L * sizeof(cf));
  // a block past the last pair (L / RPB odd) recomputes it and stores nothing
  const int yp = 2 * (blockIdx.x * RPB + row);
  const bool store = yp < L;
  const int y0 = store ? yp : L - 2;
  cf *buf = smem + row * lds_len<L>();
  cf v[E], b[E];
  if (store) {
    load_band_row_v<L, T, PR>(v, rows, bytes, y0, t, h);
    load_band_row_v<L, T, PR>(b, rows, bytes, y0 + 1, t, h);
  } else {
    // the pair's owner may already have overwritten it: transform zeros
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = b[i] = cmake(0.f, 0.f);
  }
  float tg0[E], tg1[E];
  load_target_row<E, T>(ep, g, clip, y0, t, tg0);
  load_target_row<E, T>(ep, g, clip, y0 + 1, t, tg1);
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = cmake(v[i].x - b[i].y, v[i].y + b[i].x);
  fft<L, +1>(v, buf, t, tw);
  double lsum = 0.0;
  float g0[E], g1[E];
  {
    float I0[E], I1[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      I0[i] = scale * v[i].x;
      I1[i] = scale * v[i].y;
    }
    Epi e = ep;
    if (!store) e.image = nullptr;
    lsum = image_epilogue_regs<E, T>(e, g, clip, y0, t, I0, tg0, g0) +
           image_epilogue_regs<E, T>(e, g, clip, y0 + 1, t, I1, tg1, g1);
    if (!store) lsum = 0.0;
  }
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = cmake(g0[i], g1[i]);
  fft<L, -1>(v, buf, t, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) buf[t + T * i] = v[i];
  xsync<T>();
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int p = t + T * i;
    const cf a = v[i], m = buf[p == 0 ? 0 : L - p];
    v[i] = cmake(0.5f * (a.x + m.x), 0.5f * (a.y - m.y));
    b[i] = cmake(0.5f * (a.y + m.y), 0.5f * (m.x - a.x));
  }
  if (store) {
    store_band_row_v<L, T, PR>(v, rows, bytes, y0, t, h, Wp, 1.0f);
    store_band_row_v<L, T, PR>(b, rows, bytes, y0 + 1, t, h, Wp, 1.0f);
  }
  const double s = block_sum(lsum, reinterpret_cast<double *>(smem));
  if (threadIdx.x == 0) ep.loss_part[(size_t(clip) * g.P + g.p) * gridDim.x + blockIdx.x] = s;
}

// Exchange region of one transform, in four-byte slots: the half-width
// exchange (real parts, then imaginary parts: half the LDS per transform,
// twice the LDS instructions) or complex slots.  A column pass lays its
// columns out like the rows of a row pass (T threads and one region each, two
// regions per wavefront at T = 32), so one bank model holds for both.
template <int Q, bool HALF>
struct Xch {
  static_assert(!HALF || HalfPlan<Q>::ok, "no half-width exchange plan for this length");
  static constexpr int floats = HALF ? lds_len_half<Q>() : 2 * lds_len<Q>();
};
template <int Q, bool HALF, int DIR>
__device__ __forceinline__ void xch_fft(cf (&v)[Q / FftPlan<Q>::T], float *xch, int t, const cf *tw) {
  if constexpr (HALF)
    fft_half<Q, DIR>(v, xch, t, tw);
  else
    fft<Q, DIR>(v, reinterpret_cast<cf *>(xch), t, tw);
}
// The plain column transforms (mask spectrum, resampling, low-pass) take the
// half-width exchange at the lengths where the row passes do: up to 768 (the
// 640-point resampling columns 8% faster) and from 2560, where four complex
// regions held them to one workgroup per CU; at 1024 it cost 6%.
template <int L>
struct ColFftHalf {
  static constexpr bool value = HalfPlan<L>::ok && (L <= 768 || L >= 2560);
};

// ------------------------------------------------------------ column passes
// A column pass runs one length-L transform per tile column.  A block holds
// ColBlock<L>::tiles tiles (4 columns each, T threads per column); every
// thread reads and writes its own column entries straight from global memory
// (positions t + T*i), and exchanges only through its column's LDS region.
template <int L>
struct ColBlock {
  static constexpr int T = FftPlan<L>::T;
  static constexpr int threads = 4 * T > 256 ? 4 * T : 256;
  static constexpr int tiles = threads / (4 * T);
};

// Column (tile, c) handled by this thread of column block bx, and whether the
// tile exists.
template <int L>
__device__ __forceinline__ void col_coords(int bx, int nt, int &jt, int &c, int &t, bool &valid) {
  constexpr int T = FftPlan<L>::T;
  const int col = threadIdx.x / T;
  t = threadIdx.x % T;
  c = col % kC;
  jt = bx * ColBlock<L>::tiles + col / kC;
  valid = jt < nt;
  if (!valid) jt = nt - 1;  // keep addresses in range; results are not stored
}
template <int L>
__device__ __forceinline__ void col_coords(int nt, int &jt, int &c, int &t, bool &valid) {
  col_coords<L>(blockIdx.x, nt, jt, c, t, valid);
}

// Workgroup coordinates of a column pass whose grid z encodes (i, clip) as
// z = i + inner * clip, permuted so that consecutive workgroups of one XCD
// take the same (x, y, i) for consecutive clips.  Workgroups are handed to the
// 8 XCDs in turn (linear id, x fastest), and these ones read the same bank
// tiles, which then come from that XCD's L2 instead of once per clip from HBM.
// Used by the adjoint column pass (3% faster at 16 x 1024^2); the forward
// column pass, whose output stream dominates, ran 6% slower with it, and the
// split GEMM passes (bank tiles read through LDS staging) gained nothing, so
// they keep the plain order.  The map is a permutation of the grid: results
// do not depend on it.
struct BlockXYZ {
  int x, y, z;
};
__device__ __forceinline__ BlockXYZ clip_major_on_xcds(int inner) {
  constexpr int kXcds = 8;
  const int nx = gridDim.x, ny = gridDim.y, nz = gridDim.z, clips = nz / inner;
  const int n = nx * ny * nz;
  int lin = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int full = n - n % kXcds;
  if (lin < full) lin = (lin % kXcds) * (full / kXcds) + lin / kXcds;
  const int clip = lin % clips;
  int r = lin / clips;
  const int x = r % nx;
  r /= nx;
  return BlockXYZ{x, r % ny, r / ny + inner * clip};
}

// For each tile column: a length-L DFT along the rows.  Input rows are either
// all L positions (in_h < 0) or a centred band of 2*in_h+1 rows placed at
// frequency positions (row - in_h) mod L; outputs are either all L rows
// (out_h < 0) or the centred band |f| <= out_h.  Values are scaled by `scale`.
template <int L, int DIR>
__global__ __launch_bounds__(ColBlock<L>::threads) void k_col_fft(const cf *__restrict__ in, cf *__restrict__ out,
                                                                 int nt, int in_h, int out_h, size_t in_clip,
                                                                 size_t out_clip, const cf *__restrict__ tw,
                                                                 float scale) {
  constexpr int T = FftPlan<L>::T, E = L / T;
  extern __shared__ cf smem[];
  int jt, c, t;
  bool valid;
  col_coords<L>(nt, jt, c, t, valid);
  const int clip = blockIdx.y;
  float *xch = reinterpret_cast<float *>(smem) + (threadIdx.x / T) * Xch<L, ColFftHalf<L>::value>::floats;
  const int rin = in_h < 0 ? L : 2 * in_h + 1;
  const int rout = out_h < 0 ? L : 2 * out_h + 1;
  // buffer views of this clip's arrays; positions off the band read as zero
  // and are not written (buffer range checking)
  const auto src = buf_view(in + clip * in_clip, unsigned(size_t(nt) * rin * kC * sizeof(cf)));
  const auto dst = buf_view(out + clip * out_clip, unsigned(size_t(nt) * rout * kC * sizeof(cf)));
  const unsigned in0 = unsigned(jt * rin * kC + c), out0 = unsigned(jt * rout * kC + c);
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int pos = t + T * i;
    const int r = in_h < 0 ? pos : band_row_of(pos, L, in_h);
    v[i] = buf_load(src, r >= 0 ? (in0 + unsigned(r) * kC) * unsigned(sizeof(cf)) : kOffBand);
  }
  xch_fft<L, ColFftHalf<L>::value, DIR>(v, xch, t, tw);
  if (!valid) return;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int pos = t + T * i;
    const int r = out_h < 0 ? pos : band_row_of(pos, L, out_h);
    buf_store(dst, r >= 0 ? (out0 + unsigned(r) * kC) * unsigned(sizeof(cf)) : kOffBand, cscale(v[i], scale));
  }
}

// ------------------------------------------------------------ resampling column pass
// Both column transforms of a band resampling in one pass: for each tile
// column, a length-LA DFT (DIRA) of all LA rows, the band |f| <= h kept (and,
// with gc > 0, scaled by the Gaussian exp(-gc (kx^2 + ky^2)) of the resist
// blur), then a length-LB DFT (DIRB) of that band zero-padded to LB rows, all
// LB rows stored and scaled.  One tile per workgroup; the band crosses between
// the transforms in LDS, so the D x D band never goes to HBM.  Used both ways
// between the inner grid Q and the clip grid N (intensity up, residual down).
template <int LA, int LB>
struct Resample {
  static constexpr int TA = FftPlan<LA>::T, TB = FftPlan<LB>::T;
  static constexpr int threads = 4 * (TA > TB ? TA : TB);
  // half-width exchanges: the band staging then sets the workgroup's LDS
  static constexpr bool HA = HalfPlan<LA>::ok, HB = HalfPlan<LB>::ok;
  // band rows of one column in LDS (at most min(LA, LB)), plus two pad slots
  static constexpr int stage = (LA < LB ? LA : LB) + 2;
  static constexpr size_t bytes_a = size_t(4) * Xch<LA, HA>::floats * sizeof(float);
  static constexpr size_t bytes_b = size_t(4) * Xch<LB, HB>::floats * sizeof(float);
  static constexpr size_t bytes_s = size_t(4) * stage * sizeof(cf);
  static constexpr size_t bytes_o = size_t(LB) * kC * sizeof(cf);
  static constexpr size_t m1 = bytes_a > bytes_b ? bytes_a : bytes_b, m2 = bytes_s > bytes_o ? bytes_s : bytes_o;
  static constexpr size_t bytes = m1 > m2 ? m1 : m2;
  // each transform's threads fill whole wavefronts, and its exchanges
  // synchronise only its own wavefront (transforms wider than a wavefront
  // would need the workgroup barrier inside the per-column branches)
  static_assert((4 * TA) % 64 == 0 && (4 * TB) % 64 == 0, "transforms must fill whole wavefronts");
  static_assert(TA <= 64 && TB <= 64, "one wavefront per transform at most");
};
template <int LA, int DIRA, int LB, int DIRB>
__global__ __launch_bounds__((Resample<LA, LB>::threads)) void k_col_resample(const cf *__restrict__ in,
                                                                            cf *__restrict__ out, int h,
                                                                            size_t in_clip, size_t out_clip,
                                                                            const cf *__restrict__ twA,
                                                                            const cf *__restrict__ twB, float scale,
                                                                            float gc) {
  using RS = Resample<LA, LB>;
  constexpr int TA = RS::TA, TB = RS::TB, EA = LA / TA, EB = LB / TB;
  extern __shared__ cf smem[];
  float *const lds = reinterpret_cast<float *>(smem);
  cf *const stage = smem;  // [4][RS::stage], aliases the exchange regions
  const int jt = blockIdx.x, clip = blockIdx.y, nt = gridDim.x;
  // first transform: all LA rows in, the band kept in registers
  {
    const int col = threadIdx.x / TA, t = threadIdx.x % TA;
    cf v[EA];
    if (col < 4) {
      const auto src = buf_view(in + clip * in_clip, unsigned(size_t(nt) * LA * kC * sizeof(cf)));
      const unsigned in0 = unsigned((jt * LA + t) * kC + col) * unsigned(sizeof(cf));
#pragma unroll
      for (int i = 0; i < EA; ++i) v[i] = buf_load(src, in0 + unsigned(TA * i * kC * sizeof(cf)));
      xch_fft<LA, RS::HA, DIRA>(v, lds + col * Xch<LA, RS::HA>::floats, t, twA);
    }
    __syncthreads();
    if (col < 4) {
      const int kx = jt * kC + col - h;
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int r = band_row_of(t + TA * i, LA, h);
        if (r < 0) continue;
        cf x = v[i];
        if (gc > 0.f) x = kx <= h ? cscale(x, expf(-gc * float(kx * kx + (r - h) * (r - h)))) : cmake(0.f, 0.f);
        stage[col * RS::stage + r] = x;
      }
    }
  }
  __syncthreads();
  // second transform: the band zero-padded to LB rows, all LB rows out
  const int col = threadIdx.x / TB, t = threadIdx.x % TB;
  cf v[EB];
  if (col < 4) {
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int r = band_row_of(t + TB * i, LB, h);
      v[i] = r >= 0 ? stage[col * RS::stage + r] : cmake(0.f, 0.f);
    }
  }
  __syncthreads();
  if (col < 4) xch_fft<LB, RS::HB, DIRB>(v, lds + col * Xch<LB, RS::HB>::floats, t, twB);
  // the tile's LB rows of 4 columns cross the LDS once more, so that every
  // wavefront stores whole 32-byte rows (512 contiguous bytes per store);
  // column c of row r sits in slot c ^ ((r >> 3) & 3) of the row, which keeps
  // both the column-wise writes and the row-wise reads free of bank conflicts
  __syncthreads();
  if (col < 4) {
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int r = t + TB * i;
      smem[r * kC + (col ^ ((r >> 3) & 3))] = v[i];
    }
  }
  __syncthreads();
  cf *const dst = out + clip * out_clip + size_t(jt) * LB * kC;
#pragma unroll 4
  for (int e = threadIdx.x; e < LB * kC; e += RS::threads) {
    const int r = e >> 2;
    dst[e] = cscale(smem[(e & ~3) + ((e & 3) ^ ((r >> 3) & 3))], scale);
  }
}

// Twiddles of the k-loop passes are staged in LDS when the table is small
// next to the exchange buffers: table reads then wait on the LDS counter only,
// not behind the prefetched band loads in flight on the vector-memory counter
// (which retires in order).
template <int Q>
struct TwLds {
  static constexpr int entries = twiddle_table_size<Q>();
  static constexpr bool value = entries > 0 && entries * sizeof(cf) <= 16384;
  static constexpr size_t bytes = value ? entries * sizeof(cf) : 0;
};
template <int Q>
__device__ __forceinline__ const cf *stage_twiddles(const cf *__restrict__ tw, cf *lds) {
  if constexpr (!TwLds<Q>::value) {
    return tw;
  } else {
    for (int i = threadIdx.x; i < TwLds<Q>::entries; i += blockDim.x) lds[i] = tw[i];
    __syncthreads();
    return lds;
  }
}

// Which k-loop passes take the half-width exchange, as measured on the
// workloads of each length.  Row passes: at lengths up to 768 (the complex
// exchange held them at two workgroups per CU) and from 2560 (one); at
// 1024..2048 the extra LDS round trip cost more than the occupancy gained
// (the 1280-point row passes ran 20-35% slower with it).  Adjoint column
// pass: wherever a plan exists (3-16% faster).  Forward column pass: never
// (the 640-point pass, whose occupancy is then set by its registers, ran
// 29% slower with it).
template <int Q>
struct RowHalf {
  static constexpr bool value = HalfPlan<Q>::ok && (Q <= 768 || Q >= 2560);
};
template <int Q>
struct ColAdjHalf {
  static constexpr bool value = HalfPlan<Q>::ok;
};
template <int Q>
using RowXch = Xch<Q, RowHalf<Q>::value>;
template <int Q, int DIR>
__device__ __forceinline__ void row_fft(cf (&v)[Q / FftPlan<Q>::T], float *xch, int t, const cf *tw) {
  xch_fft<Q, RowHalf<Q>::value, DIR>(v, xch, t, tw);
}
// Exchange regions of a k-loop column block, then its staged twiddles (kept
// eight-byte aligned).
template <int Q, bool HALF>
struct ColXch {
  static constexpr int regions = ColBlock<Q>::threads / FftPlan<Q>::T;
  static_assert((regions * Xch<Q, HALF>::floats) % 2 == 0, "twiddles must start on a complex slot");
  static constexpr size_t bytes = size_t(regions) * Xch<Q, HALF>::floats * sizeof(float);
};

// ------------------------------------------------------------ forward column pass
// Y_k[jt][y][c] = sum_ky Phi'_k(ky, j) Mh(ky, j) exp(+2 pi i ky y / Q), for the
// kernels k0 .. k0 + kpb - 1 of this block: the mask-spectrum column stays in
// registers and the next kernel's column is loaded while one is transformed.
template <int Q, bool PR>
__global__ __launch_bounds__(ColBlock<Q>::threads) void k_pass_y_fwd(const cf *__restrict__ bank,
                                                                    const cf *__restrict__ Mh, cf *__restrict__ Y,
                                                                    Geo g, const cf *__restrict__ tw_table, int kpb) {
  constexpr int T = FftPlan<Q>::T, E = Q / T;
  extern __shared__ cf smem[];
  int jt, c, t;
  bool valid;
  col_coords<Q>(g.nt, jt, c, t, valid);
  const int k0 = blockIdx.y * kpb, k1 = min(g.K, k0 + kpb), clip = blockIdx.z;
  using X = Xch<Q, false>;
  float *const xbase = reinterpret_cast<float *>(smem);
  float *xch = xbase + (threadIdx.x / T) * X::floats;
  const cf *tw = stage_twiddles<Q>(tw_table, reinterpret_cast<cf *>(xbase + ColXch<Q, false>::regions * X::floats));
  const size_t kb = size_t(g.nt) * g.B * kC;
  const cf *ph = bank + (size_t(g.p) * g.Kbank * g.nt + jt) * g.B * kC + c;
  const cf *mh = Mh + (size_t(clip) * g.nt + jt) * g.B * kC + c;
  auto load_band = [&](cf (&dst)[E], const cf *col) {
    const int tt = opaque_lane(t);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      if (PR && never_in_band<Q>(i)) {
        dst[i] = cmake(0.f, 0.f);
        continue;
      }
      const int r = band_row_of(tt + T * i, Q, g.b);
      dst[i] = r >= 0 ? col[r * kC] : cmake(0.f, 0.f);
    }
  };
  cf m[E], nxt[E];
  load_band(m, mh);
  load_band(nxt, ph + k0 * kb);
  for (int k = k0; k < k1; ++k) {
    cf v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = cmul(nxt[i], m[i]);
    if (k + 1 < k1) load_band(nxt, ph + (k + 1) * kb);
    xch_fft<Q, false, +1>(v, xch, t, tw);
    if (valid) {
      cf *dst = Y + ((size_t(clip) * g.K + k) * g.nt + jt) * size_t(Q) * kC + c;
      const int tt = opaque_lane(t);
#pragma unroll
      for (int i = 0; i < E; ++i) dst[(tt + T * i) * kC] = v[i];
    }
  }
}

// Occupancy target of the k-loop row passes: four wavefronts per SIMD (128
// VGPRs) while a thread holds at most 20 values, two beyond.  The pruned
// adjoint pass of one-row-per-wavefront transforms keeps three.
template <int Q>
struct RowWaves {
  static constexpr int value = Q / FftPlan<Q>::T <= 20 ? 4 : 2;
};
template <int Q, bool PR>
struct AdjRowWaves {
  static constexpr int value = (PR && FftPlan<Q>::T > 32 && RowWaves<Q>::value > 3) ? 3 : RowWaves<Q>::value;
};
// The pruned row passes load the next kernel's band row while one is
// transformed; transforms of more than 20 values per thread skip it, since
// the second register copy would push them into AGPR spills at one wavefront
// per SIMD (occupancy hides their latency instead).
template <int Q, bool PR>
struct RowPrefetch {
  static constexpr bool value = PR && Q / FftPlan<Q>::T <= 20;
};

// Waves per SIMD that the LDS of a 256-thread row-pass block (exchange rows
// and staged twiddles) allows on a 160 KB CU; a register target above it buys
// nothing and only constrains the schedule.
template <int Q>
struct RowLdsWaves {
  static constexpr size_t bytes = size_t(256 / FftPlan<Q>::T) * RowXch<Q>::floats * sizeof(float) + TwLds<Q>::bytes;
  static constexpr int value = int(163840 / bytes) < 1 ? 1 : int(163840 / bytes);
};
template <int W, int Q>
struct CapWaves {
  static constexpr int value = W < RowLdsWaves<Q>::value ? W : RowLdsWaves<Q>::value;
};

// ------------------------------------------------------------ forward row pass
// I_Q(y, x) = dose * sum_k |sum_kx Y_k(y, kx) exp(+2 pi i kx x / Q)|^2.
// OUT 0 (Q == N): image / resist epilogue.  OUT 1 (Q < N): forward row DFT of
// the I_Q row, keep |gx| <= 2b, scale dose/Q^2, store tiled [ntD][Q][kC] in Ib.
// The 640-point forward row pass (the 1024^2 workloads' inner grid) runs at
// five wavefronts per SIMD without the band-row prefetch: its 1280
// workgroups per 16 clips then fit the device at once, and it ran 5% faster
// than at four with the prefetch.
template <int Q>
struct FwdRowWaves {
  static constexpr int value = Q == 640 ? 5 : RowWaves<Q>::value;
};
template <int Q, bool PR>
struct FwdPrefetch {
  static constexpr bool value = Q != 640 && RowPrefetch<Q, PR>::value;
};

template <int Q, int OUT, bool PR>
__global__ __launch_bounds__(256, (CapWaves<FwdRowWaves<Q>::value, Q>::value)) void k_pass_x_fwd(const cf *__restrict__ Y, Epi ep, cf *__restrict__ Ib, Geo g,
                                                    const cf *__restrict__ tw_table) {
  constexpr int T = FftPlan<Q>::T, E = Q / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int y = blockIdx.x * RPB + row, clip = blockIdx.y;
  float *const xbase = reinterpret_cast<float *>(smem);
  float *xch = xbase + row * RowXch<Q>::floats;
  const cf *tw = stage_twiddles<Q>(tw_table, reinterpret_cast<cf *>(xbase + RPB * RowXch<Q>::floats));
  float acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = 0.f;
  const size_t kstride = size_t(g.nt) * Q * kC;
  const cf *yc = Y + size_t(clip) * g.K * kstride;
  const RowIO<Q, T, PR> io(kstride, y, t, g.b);
  // pruned variant: the band row of kernel k + 1 (half the elements) is
  // loaded while kernel k is transformed
  cf nxt[E];
  if (FwdPrefetch<Q, PR>::value) io.load(nxt, yc);
  for (int k = 0; k < g.K; ++k) {
    cf v[E];
    if (FwdPrefetch<Q, PR>::value) {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = nxt[i];
      if (k + 1 < g.K) io.load(nxt, yc + (k + 1) * kstride);
    } else {
      io.load(v, yc + k * kstride);
    }
    row_fft<Q, +1>(v, xch, t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] += cabs2(v[i]);
  }
  if constexpr (OUT == 0) {
    float tg[E], I[E];
    load_target_row<E, T>(ep, g, clip, y, t, tg);
#pragma unroll
    for (int i = 0; i < E; ++i) I[i] = acc[i] * g.dose;
    const double lsum = image_epilogue_row<E, T>(ep, g, clip, y, t, I, tg);
    if (ep.target) {
      const double s = block_sum(lsum, reinterpret_cast<double *>(smem));
      if (threadIdx.x == 0) ep.loss_part[(size_t(clip) * g.P + g.p) * gridDim.x + blockIdx.x] = s;
    }
  } else {
    cf v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = cmake(acc[i], 0.f);
    row_fft<Q, -1>(v, xch, t, tw);
    store_band_row_v<Q, T>(v, Ib + size_t(clip) * g.ntD * size_t(Q) * kC, unsigned(size_t(g.Dp) * Q * sizeof(cf)),
                           y, t, 2 * g.b, g.Dp, g.dose / (float(Q) * float(Q)));
  }
}

// ------------------------------------------------------------ adjoint row pass
// V_k(y, kx) = sum_x G(y, x) E'_k(y, x) exp(-2 pi i kx x / Q), |kx| <= b,
// E'_k recomputed from Y_k; V_k overwrites Y_k (each row is owned by one
// wavefront, which reads it completely before writing it).
// GIN 0: G is a real [Q][Q] array per clip (Q == N), rows strided by Q.
// GIN 1: G is a band [ntD][Q][kC] (|gx| <= 2b) per clip; its row is synthesised.
template <int Q, int GIN, bool PR>
__global__ __launch_bounds__(256, (CapWaves<AdjRowWaves<Q, PR>::value, Q>::value)) void k_pass_x_adj(cf *__restrict__ Y, const float *__restrict__ Greal,
                                                    size_t g_clip_stride, const cf *__restrict__ Gband, Geo g,
                                                    const cf *__restrict__ tw_table) {
  constexpr int T = FftPlan<Q>::T, E = Q / T, RPB = 256 / T;
  extern __shared__ cf smem[];
  const int row = threadIdx.x / T, t = threadIdx.x % T;
  const int y = blockIdx.x * RPB + row, clip = blockIdx.y;
  float *const xbase = reinterpret_cast<float *>(smem);
  float *xch = xbase + row * RowXch<Q>::floats;
  const cf *tw = stage_twiddles<Q>(tw_table, reinterpret_cast<cf *>(xbase + RPB * RowXch<Q>::floats));
  float gr[E];
  if constexpr (GIN == 0) {
    const float *gsrc = Greal + clip * g_clip_stride + size_t(y) * Q;
#pragma unroll
    for (int i = 0; i < E; ++i) gr[i] = gsrc[t + T * i] * g.dose;
  } else {
    cf v[E];
    load_band_row_v<Q, T>(v, Gband + size_t(clip) * g.ntD * size_t(Q) * kC, unsigned(size_t(g.Dp) * Q * sizeof(cf)),
                          y, t, 2 * g.b);
    row_fft<Q, +1>(v, xch, t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) gr[i] = v[i].x * g.dose;
  }
  const size_t kstride = size_t(g.nt) * Q * kC;
  cf *yc = Y + size_t(clip) * g.K * kstride;
  const RowIO<Q, T, PR> io(kstride, y, t, g.b);
  // pruned variant: the band row of kernel k + 1 (half the elements) is
  // loaded while kernel k is transformed (each row is read completely before
  // this wavefront overwrites it)
  cf nxt[E];
  if (RowPrefetch<Q, PR>::value) io.load(nxt, yc);
  for (int k = 0; k < g.K; ++k) {
    cf v[E];
    if (RowPrefetch<Q, PR>::value) {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = nxt[i];
      if (k + 1 < g.K) io.load(nxt, yc + (k + 1) * kstride);
    } else {
      io.load(v, yc + k * kstride);
    }
    row_fft<Q, +1>(v, xch, t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = cscale(v[i], gr[i]);
    row_fft<Q, -1>(v, xch, t, tw);
    io.store(v, yc + k * kstride, g.Bp, 1.0f);
  }
}

// ------------------------------------------------------------ adjoint column pass
// part[clip][p*KC + kc][jt][ky][c] = sum_{k in chunk} conj(Phi'_k) * sum_y V_k(y, j) exp(-2 pi i ky y / Q)
// The chunk sum is accumulated in FP32 in the FFT register layout (band rows
// only) and stored in FP64; chunks and planes are summed in FP64 later.
template <int Q, bool PR>
__global__ __launch_bounds__(ColBlock<Q>::threads) void k_pass_y_adj(const cf *__restrict__ V,
                                                                    const cf *__restrict__ bank,
                                                                    double2 *__restrict__ part, Geo g,
                                                                    const cf *__restrict__ tw_table) {
  constexpr int T = FftPlan<Q>::T, E = Q / T;
  extern __shared__ cf smem[];
  int jt, c, t;
  bool valid;
  const BlockXYZ bid = clip_major_on_xcds(1);
  col_coords<Q>(bid.x, g.nt, jt, c, t, valid);
  const int kc = bid.y, clip = bid.z;
  constexpr bool H = ColAdjHalf<Q>::value;
  using X = Xch<Q, H>;
  float *const xbase = reinterpret_cast<float *>(smem);
  float *xch = xbase + (threadIdx.x / T) * X::floats;
  const cf *tw = stage_twiddles<Q>(tw_table, reinterpret_cast<cf *>(xbase + ColXch<Q, H>::regions * X::floats));
  cf acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = cmake(0.f, 0.f);
  const int k0 = kc * g.kper, k1 = min(g.K, k0 + g.kper);
  const cf *vcol = V + ((size_t(clip) * g.K + k0) * g.nt + jt) * size_t(Q) * kC + c;
  const size_t kstride = size_t(g.nt) * Q * kC;
  // small transforms (pruned, at most 20 values per thread): the column of
  // kernel k + 1 is loaded while kernel k is transformed
  constexpr bool PF = PR && E <= 20 && T <= 32;
  auto load_col = [&](cf (&dst)[E], int k) {
    const cf *src = vcol + (k - k0) * kstride;
    const int tt = opaque_lane(t);
#pragma unroll
    for (int i = 0; i < E; ++i) dst[i] = src[(tt + T * i) * kC];
  };
  cf nxt[E];
  if (PF) load_col(nxt, k0);
  for (int k = k0; k < k1; ++k) {
    cf v[E];
    if (PF) {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = nxt[i];
      if (k + 1 < k1) load_col(nxt, k + 1);
    } else {
      load_col(v, k);
    }
    // conj(Phi'_k) at this thread's band rows, loaded before the transform
    // so that it hides their latency (zero off the band)
    cf w[E];
    {
      const cf *ph = bank + ((size_t(g.p) * g.Kbank + k) * g.nt + jt) * g.B * kC + c;
      const int t2 = opaque_lane(t);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        w[i] = cmake(0.f, 0.f);
        if (PR && never_in_band<Q>(i)) continue;
        const int r = band_row_of(t2 + T * i, Q, g.b);
        if (r >= 0) w[i] = ph[r * kC];
      }
    }
    xch_fft<Q, H, -1>(v, xch, t, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      if (PR && never_in_band<Q>(i)) continue;
      acc[i] = make_float2(acc[i].x + w[i].x * v[i].x + w[i].y * v[i].y, acc[i].y + w[i].x * v[i].y - w[i].y * v[i].x);
    }
  }
  if (!valid) return;
  double2 *dst = part + ((size_t(clip) * g.P * g.KC + size_t(g.p) * g.KC + kc) * g.nt + jt) * size_t(g.B) * kC + c;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    if (PR && never_in_band<Q>(i)) continue;
    const int r = band_row_of(t + T * i, Q, g.b);
    if (r >= 0) dst[r * kC] = make_double2(acc[i].x, acc[i].y);
  }
}

// ------------------------------------------------------------ gradient finish, columns
// Acc = sum over (plane, k-chunk) partials in FP64 (fixed order), scaled by 1/N^2,
// then the inverse column DFT (band rows -> N rows).
template <int N, bool PR>
__global__ __launch_bounds__(ColBlock<N>::threads) void k_grad_cols(const double2 *__restrict__ part, int nparts,
                                                                   cf *__restrict__ out, Geo g,
                                                                   const cf *__restrict__ tw) {
  constexpr int T = FftPlan<N>::T, E = N / T;
  extern __shared__ cf smem[];
  int jt, c, t;
  bool valid;
  col_coords<N>(g.nt, jt, c, t, valid);
  const int clip = blockIdx.y;
  cf *buf = smem + (threadIdx.x / T) * lds_len<N>();
  const size_t nE = size_t(g.B) * kC;
  const double2 *src = part + size_t(clip) * nparts * g.nt * nE;
  const unsigned pbytes = unsigned(g.nt * nE * sizeof(double2));
  const double inv = 1.0 / (double(N) * double(N));
  // byte offsets of this thread's band rows in one partial (off the band:
  // out of range, read as zero)
  unsigned off[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int r = band_row_of(t + T * i, N, g.b);
    off[i] = r >= 0 ? unsigned(jt * nE + r * kC + c) * unsigned(sizeof(double2)) : kOffBand;
  }
  double sx[E], sy[E];
#pragma unroll
  for (int i = 0; i < E; ++i) sx[i] = sy[i] = 0.0;
  for (int s = 0; s < nparts; ++s) {
    const auto view = buf_view(src + size_t(s) * g.nt * nE, pbytes);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      if (PR && never_in_band<N>(i)) continue;
      const d2v a = buf_load_d2(view, off[i]);
      sx[i] += a.x;
      sy[i] += a.y;
    }
  }
  cf v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = cmake(float(sx[i] * inv), float(sy[i] * inv));
  fft<N, +1>(v, buf, t, tw);
  if (!valid) return;
  cf *dst = out + (size_t(clip) * g.nt + jt) * size_t(N) * kC + c;
#pragma unroll
  for (int i = 0; i < E; ++i) dst[(t + T * i) * kC] = v[i];
}


// ------------------------------------------------------------ split-precision band DFT-GEMM (MFMA)
// The forward column pass as a dense complex GEMM on the matrix cores:
//   Y_k^T[kx][y] = sum_ky X_k^T[kx][ky] W[ky][y],  X_k = Phi'_k * Mh,  W[ky][y] = exp(+2 pi i (ky - b) y / Q)
// with v_mfma_f32_32x32x16_{f16,bf16} and FP32 accumulation.  SPLIT operands are
// x = hi + lo (hi = round(x), lo = round(x - hi)) and the product keeps
// hi*hi + hi*lo + lo*hi.  A workgroup of four waves computes a 32 (kx) x 256 (y)
// tile, each wave 32 x 64.
// Operand layout of the 32x32x16 instruction: lane l holds A[l % 32][8 (l / 32) + j]
// and B[8 (l / 32) + j][l % 32], j = 0..7; accumulator register i of lane l holds
// D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename E>
struct Mfma;
template <>
struct Mfma<_Float16> {
  using V = h8v;
  __device__ __forceinline__ static f16v run(V a, V b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<__bf16> {
  using V = b8v;
  __device__ __forceinline__ static f16v run(V a, V b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// N-tiles (32 wide) per wave of the forward GEMM kernel (the adjoint one uses
// one); the waves per workgroup (NW) are a template parameter: 4 for the
// forward GEMM, 4 or 10 for the adjoint one.
constexpr int kGemmNtw = 2;

// A-operand fragments of one K-step (32 x 16) in LDS, in the instruction's
// lane order: component c, lane l, value j.  Components: re hi, im hi,
// -im hi and, when split, re lo, im lo, -im lo.  Each component row has 16
// spare fragments (128 values) that absorb the stores of threads without an
// element, so that no store needs a branch.
constexpr int kStageRow = 80;  // fragments per component row (64 used)
template <typename E, int NC>
struct AStage {
  typename Mfma<E>::V v[2][NC][kStageRow];
};

// Element e < 512 of the 32 x 16 A block (kx local m, K index kk) -> LDS
// slot; e in [512, 640) -> a spare slot.
__device__ __forceinline__ int a_slot(int e, int m, int kk) {
  return e < 512 ? (m + 32 * (kk >> 3)) * 8 + (kk & 7) : e;
}

template <typename E, bool SPLIT>
__device__ __forceinline__ void a_store(E *base, int slot, float xr, float xi) {
  // base points at component 0 of the stage buffer
  constexpr int R = 8 * kStageRow;
  const E hr = E(xr), hi = E(xi);
  base[slot] = hr;
  base[R + slot] = hi;
  base[2 * R + slot] = E(-xi);
  if constexpr (SPLIT) {
    const float lr = xr - float(hr), li = xi - float(hi);
    base[3 * R + slot] = E(lr);
    base[4 * R + slot] = E(li);
    base[5 * R + slot] = E(-li);
  }
}

// One K-step of the complex product on the matrix cores:
//   Dr += Ar Br - Ai Bi,  Di += Ar Bi + Ai Br
// with A from the LDS stage and B (re hi, im hi[, re lo, im lo]) in registers.
template <typename E, bool SPLIT, int NTW, int NB>
__device__ __forceinline__ void mfma_step(const typename Mfma<E>::V (&a)[SPLIT ? 6 : 3][kStageRow], int l,
                                          const typename Mfma<E>::V (&b)[NTW][NB], f16v (&acc_r)[NTW],
                                          f16v (&acc_i)[NTW]) {
  using V = typename Mfma<E>::V;
  const V arh = a[0][l], ari = a[1][l], nari = a[2][l];
#pragma unroll
  for (int n = 0; n < NTW; ++n) {
    acc_r[n] = Mfma<E>::run(arh, b[n][0], acc_r[n]);
    acc_r[n] = Mfma<E>::run(nari, b[n][1], acc_r[n]);
    acc_i[n] = Mfma<E>::run(arh, b[n][1], acc_i[n]);
    acc_i[n] = Mfma<E>::run(ari, b[n][0], acc_i[n]);
  }
  if constexpr (SPLIT) {
    const V arl = a[3][l], ail = a[4][l], nail = a[5][l];
#pragma unroll
    for (int n = 0; n < NTW; ++n) {
      acc_r[n] = Mfma<E>::run(arh, b[n][2], acc_r[n]);
      acc_r[n] = Mfma<E>::run(arl, b[n][0], acc_r[n]);
      acc_r[n] = Mfma<E>::run(nari, b[n][3], acc_r[n]);
      acc_r[n] = Mfma<E>::run(nail, b[n][1], acc_r[n]);
      acc_i[n] = Mfma<E>::run(arh, b[n][3], acc_i[n]);
      acc_i[n] = Mfma<E>::run(arl, b[n][1], acc_i[n]);
      acc_i[n] = Mfma<E>::run(ari, b[n][2], acc_i[n]);
      acc_i[n] = Mfma<E>::run(ail, b[n][0], acc_i[n]);
    }
  }
}

// The K loop shared by both GEMM kernels.  Software pipeline without register
// copies (a copy would wait for the load in flight): the loop is unrolled by
// two, LDS stage P = ks & 1 feeds K-step ks, raw A operands of K-step ks + 1
// were loaded two K-steps earlier into raw[(ks + 1) & 1], and the B fragments
// of ks + 1 are loaded into b[(ks + 1) & 1] while ks multiplies.
//   a_load(ks, R &)             raw A operands of K-step ks (any ks; clamped addresses, no
//                               arithmetic on the loaded values, which would wait for them)
//   a_put(stage, const R &, ks) zeroes what lies outside the operand and converts into LDS
//   b_load(ks, b)          B fragments of K-step ks (any ks; clamped)
// The stage written after the last K-step is never read.
template <typename E, bool SPLIT, int NTW, int NB, typename R, typename ALoad, typename APut, typename BLoad>
__device__ __forceinline__ void gemm_kloop(int ksteps, bool active,
                                           typename Mfma<E>::V (&st)[2][SPLIT ? 6 : 3][kStageRow],
                                           int l, ALoad &&a_load, APut &&a_put, BLoad &&b_load,
                                           f16v (&acc_r)[NTW], f16v (&acc_i)[NTW]) {
  using V = typename Mfma<E>::V;
  R raw[2];
  V b[2][NTW][NB];
  a_load(0, raw[0]);
  a_put(0, raw[0], 0);
  a_load(1, raw[1]);
  a_load(2, raw[0]);
  b_load(0, b[0]);
  __syncthreads();
  auto step = [&](auto pc, int ks) {
    constexpr int P = decltype(pc)::value;
    b_load(ks + 1, b[1 - P]);
    if (active) mfma_step<E, SPLIT, NTW, NB>(st[P], l, b[P], acc_r, acc_i);
    a_put(1 - P, raw[1 - P], ks + 1);
    a_load(ks + 3, raw[1 - P]);
    __syncthreads();
  };
  for (int ks = 0; ks < ksteps; ks += 2) {
    step(std::integral_constant<int, 0>{}, ks);
    if (ks + 1 < ksteps) step(std::integral_constant<int, 1>{}, ks + 1);
  }
}

// Table of the B operand: one block of 64 lanes x 8 values per (K-step,
// N-tile, component), components re hi, re lo, im hi, im lo.
//
// Workgroup: NW waves share one 32-column A block per K-step (built
// once in LDS from Phi'_k * M^, FP32 -> hi/lo); each wave multiplies it with
// kGemmNtw N-tiles of the DFT table, prefetched one K-step ahead.
template <typename E, bool SPLIT, int NW>
__global__ __launch_bounds__(64 * NW) void k_pass_y_fwd_mfma(const cf *__restrict__ bank,
                                                                   const cf *__restrict__ Mh, cf *__restrict__ Y,
                                                                   Geo g, const typename Mfma<E>::V *__restrict__ tab,
                                                                   float sin, float sout) {
  using V = typename Mfma<E>::V;
  constexpr int NC = SPLIT ? 6 : 3, NB = SPLIT ? 4 : 2, EPT = (512 + 64 * NW - 1) / (64 * NW);
  __shared__ AStage<E, NC> st;
  const int tid = threadIdx.x, l = tid & 63, m = l & 31, kg = l >> 5;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, scalar
  const int mt = blockIdx.x, k = blockIdx.z % g.K, clip = blockIdx.z / g.K;
  const int Q = g.Q, nQt = Q / 32, ksteps = (g.B + 15) / 16;
  const int nt0 = (blockIdx.y * NW + w) * kGemmNtw;
  const bool active = nt0 < nQt;
  // this thread's A elements: e = tid + 64 NW i -> tile 8 mt + e / 64, row (e / 4) % 16, column e % 4;
  // per element a fixed column pointer and row index, so that a K-step costs one add per load
  const cf *pa[EPT], *pm[EPT];
  int kyl[EPT], slot[EPT];
  bool col_ok[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + 64 * NW * i, jt = 8 * mt + (e >> 6);
    const size_t col = size_t(min(jt, g.nt - 1)) * g.B * kC + (e & 3);
    pa[i] = bank + (size_t(g.p) * g.Kbank + k) * g.nt * size_t(g.B) * kC + col;
    pm[i] = Mh + size_t(clip) * g.nt * size_t(g.B) * kC + col;
    kyl[i] = (e >> 2) & 15;
    slot[i] = a_slot(e, 4 * ((e >> 6) & 7) + (e & 3), kyl[i]);
    col_ok[i] = e < 512 && jt < g.nt;
  }
  struct Raw {
    cf v[2 * EPT];
  };
  // Loads in the K loop are unconditional (clamped addresses, zeroed when
  // stored), so that the compiler can count loads in flight.
  auto a_load = [&](int ks, Raw &x) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int r = min(16 * ks + kyl[i], g.B - 1) * kC;
      x.v[2 * i] = pa[i][r];
      x.v[2 * i + 1] = pm[i][r];
    }
  };
  auto a_put = [&](int buf, const Raw &x, int ks) {
    E *base = reinterpret_cast<E *>(&st.v[buf][0][0]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const float s = col_ok[i] && 16 * ks + kyl[i] < g.B ? sin : 0.0f;
      const cf v = cmul(x.v[2 * i], x.v[2 * i + 1]);
      a_store<E, SPLIT>(base, slot[i], v.x * s, v.y * s);
    }
  };
  const V *tab_l = tab + l;
  auto b_load = [&](int ks, V (&b)[kGemmNtw][NB]) {
#pragma unroll
    for (int n = 0; n < kGemmNtw; ++n) {
      const int nt = min(nt0 + n, nQt - 1);
      const V *tb = tab_l + (min(ks, ksteps - 1) * nQt + nt) * 4 * 64;
      b[n][0] = tb[0];
      b[n][1] = tb[128];
      if constexpr (SPLIT) {
        b[n][2] = tb[64];
        b[n][3] = tb[192];
      }
    }
  };
  f16v acc_r[kGemmNtw], acc_i[kGemmNtw];
#pragma unroll
  for (int n = 0; n < kGemmNtw; ++n) {
    acc_r[n] = f16v{};
    acc_i[n] = f16v{};
  }
  gemm_kloop<E, SPLIT, kGemmNtw, NB, Raw>(ksteps, active, st.v, l, a_load, a_put, b_load, acc_r, acc_i);
  // accumulator register i of lane l: D row 8 (i / 4) + 4 kg + i % 4 = four consecutive kx of tile 8 mt + 2 (i / 4) + kg
  cf *yk = Y + (size_t(clip) * g.K + k) * g.nt * size_t(Q) * kC;
#pragma unroll
  for (int n = 0; n < kGemmNtw; ++n) {
    if (nt0 + n >= nQt) break;
    const int y = 32 * (nt0 + n) + m;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jt = 8 * mt + 2 * q + kg;
      if (jt < g.nt) {
        // streaming stores: Y is read back by the next pass, not by this one, and
        // should not evict the DFT table from L2
        f4v *dst = reinterpret_cast<f4v *>(yk + (size_t(jt) * Q + y) * kC);
        const f4v lo = {acc_r[n][4 * q] * sout, acc_i[n][4 * q] * sout, acc_r[n][4 * q + 1] * sout,
                        acc_i[n][4 * q + 1] * sout};
        const f4v hi = {acc_r[n][4 * q + 2] * sout, acc_i[n][4 * q + 2] * sout, acc_r[n][4 * q + 3] * sout,
                        acc_i[n][4 * q + 3] * sout};
        __builtin_nontemporal_store(lo, dst);
        __builtin_nontemporal_store(hi, dst + 1);
      }
    }
  }
}

// Adjoint column pass as a GEMM: per kernel k,
//   U_k^T[kx][ky] = sum_y V_k^T[kx][y] W[y][ky],  W[y][ky] = exp(-2 pi i (ky - b) y / Q),
// then acc[kx][ky] += conj(Phi'_k[ky][kx]) U_k[ky][kx] over the kernels of the
// chunk (FP32), stored as the chunk's FP64 partial.  A workgroup owns 32 kx
// columns and NW 32-row tiles of ky, one per wave, so that with NW = 10 a
// 317-row band is covered by one workgroup and V_k is read once.  FP16 operands of V_k are
// scaled per workgroup and kernel by the power of two that puts the block's
// largest component in [2^13, 2^14).
template <typename E, bool SPLIT, int NW>
__global__ __launch_bounds__(64 * NW) void k_pass_y_adj_mfma(const cf *__restrict__ V,
                                                                   const cf *__restrict__ bank,
                                                                   double2 *__restrict__ part, Geo g,
                                                                   const typename Mfma<E>::V *__restrict__ tab) {
  using Vt = typename Mfma<E>::V;
  constexpr int NC = SPLIT ? 6 : 3, NB = SPLIT ? 4 : 2, EPT = (512 + 64 * NW - 1) / (64 * NW), NTW = 1;
  constexpr bool kHalf = __is_same(E, _Float16);
  __shared__ AStage<E, NC> st;
  __shared__ float wmax[NW];
  const int tid = threadIdx.x, l = tid & 63, m = l & 31, kg = l >> 5;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, scalar
  const int mt = blockIdx.x;
  const int kc = blockIdx.z % g.KC, clip = blockIdx.z / g.KC;
  const int Q = g.Q, ksteps = Q / 16, nBt = (g.B + 31) / 32;
  const int nt0 = (blockIdx.y * NW + w) * NTW;
  const bool active = nt0 < nBt;
  const size_t kstride = size_t(g.nt) * Q * kC;
  const cf *vc = V + size_t(clip) * g.K * kstride;
  // per element: column offset, row in the K-step, LDS slot and whether it lies in the band
  int colo[EPT], kyl[EPT], slot[EPT];
  bool col_ok[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + 64 * NW * i, jt = 8 * mt + (e >> 6);
    colo[i] = min(jt, g.nt - 1) * Q * kC + (e & 3);
    kyl[i] = (e >> 2) & 15;
    slot[i] = a_slot(e, 4 * ((e >> 6) & 7) + (e & 3), kyl[i]);
    col_ok[i] = e < 512 && jt < g.nt;
  }
  f16v tot_r[NTW], tot_i[NTW];
#pragma unroll
  for (int n = 0; n < NTW; ++n) {
    tot_r[n] = f16v{};
    tot_i[n] = f16v{};
  }
  const int k0 = kc * g.kper, k1 = min(g.K, k0 + g.kper);
  for (int k = k0; k < k1; ++k) {
    const cf *src = vc + k * kstride;
    struct Raw {
      cf v[EPT];
    };
    // unconditional loads (clamped addresses, zeroed after), as in the forward GEMM
    auto a_load = [&](int ks, Raw &x) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) x.v[i] = src[colo[i] + (16 * min(ks, ksteps - 1) + kyl[i]) * kC];
    };
    float sc = 1.0f;
    if constexpr (kHalf) {
      float mx = 0.f;
#pragma unroll 4
      for (int ks = 0; ks < ksteps; ++ks) {
        Raw x;
        a_load(ks, x);
#pragma unroll
        for (int i = 0; i < EPT; ++i)
          if (col_ok[i]) mx = fmaxf(mx, fmaxf(fabsf(x.v[i].x), fabsf(x.v[i].y)));
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
      if (l == 0) wmax[w] = mx;
      __syncthreads();
      mx = wmax[0];
#pragma unroll
      for (int i = 1; i < NW; ++i) mx = fmaxf(mx, wmax[i]);
      int ex = 0;
      (void)frexpf(mx, &ex);  // mx < 2^ex
      sc = mx > 0.f ? ldexpf(1.0f, 14 - ex) : 1.0f;
    }
    auto a_put = [&](int buf, const Raw &x, int) {
      E *base = reinterpret_cast<E *>(&st.v[buf][0][0]);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const float s = col_ok[i] ? sc : 0.0f;
        a_store<E, SPLIT>(base, slot[i], x.v[i].x * s, x.v[i].y * s);
      }
    };
    auto b_load = [&](int ks, Vt (&b)[NTW][NB]) {
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        const int nt = min(nt0 + n, nBt - 1);
        const Vt *tb = tab + l + (min(ks, ksteps - 1) * nBt + nt) * 4 * 64;
        b[n][0] = tb[0];
        b[n][1] = tb[128];
        if constexpr (SPLIT) {
          b[n][2] = tb[64];
          b[n][3] = tb[192];
        }
      }
    };
    f16v acc_r[NTW], acc_i[NTW];
#pragma unroll
    for (int n = 0; n < NTW; ++n) {
      acc_r[n] = f16v{};
      acc_i[n] = f16v{};
    }
    gemm_kloop<E, SPLIT, NTW, NB, Raw>(ksteps, active, st.v, l, a_load, a_put, b_load, acc_r, acc_i);
    // acc += conj(Phi'_k) U; register i of lane l is (kx = 32 mt + 8 (i / 4) + 4 kg + i % 4, ky)
    const float inv = 1.0f / sc;
    const cf *ph = bank + (size_t(g.p) * g.Kbank + k) * g.nt * size_t(g.B) * kC;
#pragma unroll
    for (int n = 0; n < NTW; ++n) {
      const int ky = 32 * (nt0 + n) + m;
      if (ky >= g.B) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int jt = 8 * mt + 2 * q + kg;
        if (jt >= g.nt) continue;
        const float4 *w4 = reinterpret_cast<const float4 *>(ph + (size_t(jt) * g.B + ky) * kC);
        const float4 wa = w4[0], wb = w4[1];
        const float wr[4] = {wa.x, wa.z, wb.x, wb.z}, wi[4] = {wa.y, wa.w, wb.y, wb.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int i = 4 * q + c;
          const float ur = acc_r[n][i] * inv, ui = acc_i[n][i] * inv;
          tot_r[n][i] += wr[c] * ur + wi[c] * ui;
          tot_i[n][i] += wr[c] * ui - wi[c] * ur;
        }
      }
    }
  }
  double2 *dst = part + ((size_t(clip) * g.P + g.p) * g.KC + kc) * g.nt * size_t(g.B) * kC;
#pragma unroll
  for (int n = 0; n < NTW; ++n) {
    const int ky = 32 * (nt0 + n) + m;
    if (ky >= g.B) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jt = 8 * mt + 2 * q + kg;
      if (jt >= g.nt) continue;
      double2 *d = dst + (size_t(jt) * g.B + ky) * kC;
#pragma unroll
      for (int c = 0; c < 4; ++c) d[c] = make_double2(tot_r[n][4 * q + c], tot_i[n][4 * q + c]);
    }
  }
}

// ------------------------------------------------------------ forward row pass, two MFMA stages
// The band-limited inverse row transform of the forward pass as two dense DFT
// stages on the matrix cores, for inner grids Q = 32 P with P <= 32.  With
// f = f0 + P f1' (0 <= f0 < P, -8 <= f1' < 8; every |f| <= b < Q/4 is one of
// these) and q = r + 32 s (0 <= r < 32, 0 <= s < P), w = exp(2 pi i / Q):
//   E_k(y, r + 32 s) = sum_f0 w^(f0 r) exp(2 pi i f0 s / P) sum_f1' exp(2 pi i f1' r / 32) Y_k(y, f)
// Stage 1 is one 32x32x16 K-step per real product (D1[f0][r], f1 = f1' + 8 as
// K), then the twiddle w^(f0 r) in FP32, then stage 2 contracts f0 (one or two
// K-steps, D2[r][s]).  Stage 1's accumulator registers are stage 2's A operand
// as they stand: register i of lane l holds f0 = 8 (i / 4) + 4 (l / 32) + i % 4
// and r = l % 32, so K-step t takes registers 8 t .. 8 t + 7 and the constant
// B operand lists f0 in that order.  Complex products take four real MFMAs
// (re*re + im*(-im), re*im + im*re); SPLIT keeps hi*hi + hi*lo + lo*hi.
// One wavefront per image row: |E_k|^2 is accumulated over the kernels in
// stage 2's register layout, then the I_Q row is moved to the FFT layout
// through LDS for the forward row DFT to the 2b band (the FP32 epilogue).
// tab: [3][6][64] operand fragments (stage 1, then stage 2's two K-steps;
// components re, im, -im, then their low halves); twl: [16][64] twiddles.
template <typename E, bool SPLIT, int P>
__global__ __launch_bounds__(256, 2) void k_pass_x_fwd_mfma(const cf *__restrict__ Y, cf *__restrict__ Ib, Geo g,
                                                        const typename Mfma<E>::V *__restrict__ tab,
                                                        const cf *__restrict__ twl, const cf *__restrict__ tw_table,
                                                        float sin, float sout) {
  constexpr int Q = 32 * P, T = FftPlan<Q>::T, EQ = Q / T, KS2 = P <= 16 ? 1 : 2, NC = SPLIT ? 6 : 3;
  using V = typename Mfma<E>::V;
  extern __shared__ cf smem[];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, m = l & 31, hl = l >> 5;
  const int y = blockIdx.x * 4 + w, clip = blockIdx.y;
  // LDS: stage 2's operand fragments and the twiddles (shared by the four
  // rows of the block, read per use to keep registers for occupancy), then
  // one exchange region per row
  V *const lb2 = reinterpret_cast<V *>(smem);
  cf *const ltw = reinterpret_cast<cf *>(lb2 + KS2 * NC * 64);
  float *const xch = reinterpret_cast<float *>(ltw + 16 * 64) + w * RowXch<Q>::floats;
  for (int e = threadIdx.x; e < KS2 * NC * 64; e += 256) {
    const int t = e / (NC * 64), c = (e / 64) % NC, ll = e % 64;
    lb2[e] = tab[((1 + t) * 6 + c) * 64 + ll];
  }
  for (int e = threadIdx.x; e < 16 * 64; e += 256) ltw[e] = twl[e];
  __syncthreads();
  // stage 1's constant operand stays in registers
  V b1[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) b1[c] = tab[c * 64 + l];
  // this lane's stage-1 A elements: f0 = m, f1 = 8 hl + j -> f = f0 + P (f1 - 8)
  const size_t kstride = size_t(g.nt) * Q * kC;
  const cf *yc = Y + size_t(clip) * g.K * kstride;
  // f = m + P (8 hl + j - 8) at column f + b: tile (f + b) / 4, slot (f + b) % 4
  const int f00 = m + P * (8 * hl - 8) + g.b;
  auto load = [&](cf (&x)[8], int k) {
    const cf *src = yc + size_t(k) * kstride + size_t(y) * kC;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int col = f00 + P * j;
      const bool ok = m < P && col >= 0 && col <= 2 * g.b;
      x[j] = ok ? src[(col >> 2) * (Q * kC) + (col & 3)] : cmake(0.f, 0.f);
    }
  };
  auto to_v = [&](const float (&x)[8], V &hi, V &lo) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const E h = E(x[j]);
      hi[j] = h;
      if constexpr (SPLIT) lo[j] = E(x[j] - float(h));
    }
  };
  // (ar + i ai)(br + i bi) accumulated into (dr, di): components 0 re, 1 im, 2 -im (+3 for the low halves)
  // the real and imaginary chains alternate, so that consecutive MFMAs do
  // not wait on each other's accumulator
  auto cmac = [&](const V &arh, const V &arl, const V &aih, const V &ail, const V (&b)[NC], f16v &dr, f16v &di) {
    dr = Mfma<E>::run(arh, b[0], dr);
    di = Mfma<E>::run(arh, b[1], di);
    dr = Mfma<E>::run(aih, b[2], dr);
    di = Mfma<E>::run(aih, b[0], di);
    if constexpr (SPLIT) {
      dr = Mfma<E>::run(arh, b[3], dr);
      di = Mfma<E>::run(arh, b[4], di);
      dr = Mfma<E>::run(arl, b[0], dr);
      di = Mfma<E>::run(arl, b[1], di);
      dr = Mfma<E>::run(aih, b[5], dr);
      di = Mfma<E>::run(aih, b[3], di);
      dr = Mfma<E>::run(ail, b[2], dr);
      di = Mfma<E>::run(ail, b[0], di);
    }
  };
  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k = 0; k < g.K; ++k) {
    cf raw[8];
    load(raw, k);
    float xr[8], xi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      xr[j] = raw[j].x * sin;
      xi[j] = raw[j].y * sin;
    }
    V arh, arl, aih, ail;
    to_v(xr, arh, arl);
    to_v(xi, aih, ail);
    f16v d1r = f16v{}, d1i = f16v{};
    cmac(arh, arl, aih, ail, b1, d1r, d1i);
    // twiddle w^(f0 r), FP32
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const cf tw = ltw[i * 64 + l];
      const float re = d1r[i] * tw.x - d1i[i] * tw.y;
      const float im = d1r[i] * tw.y + d1i[i] * tw.x;
      d1r[i] = re;
      d1i[i] = im;
    }
    f16v d2r = f16v{}, d2i = f16v{};
#pragma unroll
    for (int t = 0; t < KS2; ++t) {
      float pr[8], pi[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        pr[j] = d1r[8 * t + j];
        pi[j] = d1i[8 * t + j];
      }
      V prh, prl, pih, pil;
      to_v(pr, prh, prl);
      to_v(pi, pih, pil);
      V b2[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) b2[c] = lb2[(t * NC + c) * 64 + l];
      cmac(prh, prl, pih, pil, b2, d2r, d2i);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] += d2r[i] * d2r[i] + d2i[i] * d2i[i];
  }
  // I_Q row to the FFT layout: register i of lane l is position q = r + 32 s,
  // r = 8 (i / 4) + 4 hl + i % 4, s = m (s < P)
  if (m < P) {
#pragma unroll
    for (int i = 0; i < 16; ++i) xch[8 * (i >> 2) + 4 * hl + (i & 3) + 32 * m] = acc[i] * sout;
  }
  xsync<64>();
  // every lane of the wavefront takes part in the row transform; lanes with
  // the same t hold the same values
  const int t = l % T;
  cf v[EQ];
#pragma unroll
  for (int i = 0; i < EQ; ++i) v[i] = cmake(xch[t + T * i], 0.f);
  xsync<64>();
  row_fft<Q, -1>(v, xch, t, tw_table);
  if (l < T)
    store_band_row_v<Q, T>(v, Ib + size_t(clip) * g.ntD * size_t(Q) * kC, unsigned(size_t(g.Dp) * Q * sizeof(cf)),
                           y, t, 2 * g.b, g.Dp, g.dose / (float(Q) * float(Q)));
}


// ------------------------------------------------------------ loss reduction
__global__ __launch_bounds__(256) void k_loss_reduce(const double *__restrict__ part, int n_per_clip,
                                                     double *__restrict__ loss) {
  __shared__ double red[256];
  const int clip = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n_per_clip; i += blockDim.x) s += part[size_t(clip) * n_per_clip + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) loss[clip] = s;
}

}  // namespace dev

// ======================================================================== host launchers

namespace {

using dev::cf;
using dev::Epi;
using dev::FftPlan;
using dev::Geo;
using dev::kC;
using dev::lds_len;

Geo to_geo(const PassGeo &pg) {
  Geo g;
  g.N = pg.N; g.Q = pg.Q; g.b = pg.b; g.B = pg.B; g.Bp = pg.Bp; g.nt = pg.nt;
  g.D = pg.D; g.Dp = pg.Dp; g.ntD = pg.ntD;
  g.K = pg.K; g.Kbank = pg.Kbank; g.P = pg.P; g.p = pg.p; g.KC = pg.KC; g.kper = pg.kper;
  g.dose = float(pg.dose); g.slope = float(pg.slope); g.thr = float(pg.thr); g.pw = float(pg.pw);
  g.loss_l1 = pg.loss_l1;
  return g;
}

Epi to_epi(const EpiPtrs &e) {
  Epi o;
  o.image = e.image;
  o.target = e.target;
  o.G = e.G;
  o.loss_part = e.loss_part;
  return o;
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

#define KPTR(...) reinterpret_cast<const void *>(&__VA_ARGS__)

template <int L>
int rows_fwd_real_l(const char *name, const float *in, size_t in_clip, cf *out, int h, int Wp, const cf *tw,
                    float scale, int nclips, hipStream_t s) {
  constexpr int T = FftPlan<L>::T, RPB = 256 / T;
  size_t sh = size_t(RPB) * lds_len<L>() * sizeof(cf);
  const dim3 grid((L / RPB + 1) / 2, nclips);  // two rows per transform
  if (dev::prunable<L>(h))
    return launch(name, KPTR(dev::k_rows_fwd_real<L, true>), grid, sh, s, [&] {
      hipLaunchKernelGGL((dev::k_rows_fwd_real<L, true>), grid, dim3(256), sh, s, in, in_clip, out, h, Wp, tw, scale);
    });
  return launch(name, KPTR(dev::k_rows_fwd_real<L, false>), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_rows_fwd_real<L, false>), grid, dim3(256), sh, s, in, in_clip, out, h, Wp, tw, scale);
  });
}

template <int L, int MODE>
int rows_inv_real_l(const char *name, const cf *in, int h, int Wp, float *out, const EpiPtrs &ep,
                    const PassGeo &pg, const cf *tw, float scale, int nclips, hipStream_t s) {
  constexpr int T = FftPlan<L>::T, RPB = 256 / T;
  size_t sh = size_t(RPB) * lds_len<L>() * sizeof(cf);
  sh = std::max(sh, size_t(256) * sizeof(double));
  Geo g = to_geo(pg);
  Epi e = to_epi(ep);
  const dim3 grid(MODE == 1 ? (L / RPB + 1) / 2 : L / RPB, nclips);  // MODE 1: two rows per transform
  if (dev::prunable<L>(h))
    return launch(name, KPTR((dev::k_rows_inv_real<L, MODE, true>)), grid, sh, s, [&] {
      hipLaunchKernelGGL((dev::k_rows_inv_real<L, MODE, true>), grid, dim3(256), sh, s, in, h, Wp, out, e, g, tw,
                         scale);
    });
  return launch(name, KPTR((dev::k_rows_inv_real<L, MODE, false>)), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_rows_inv_real<L, MODE, false>), grid, dim3(256), sh, s, in, h, Wp, out, e, g, tw,
                       scale);
  });
}

template <int L>
int rows_image_residual_l(const char *name, cf *band, int h, int Wp, const EpiPtrs &ep, const PassGeo &pg,
                          const cf *tw, float scale, int nclips, hipStream_t s) {
  constexpr int T = FftPlan<L>::T, RPB = 256 / T;
  size_t sh = size_t(RPB) * lds_len<L>() * sizeof(cf);
  sh = std::max(sh, size_t(256) * sizeof(double));
  Geo g = to_geo(pg);
  Epi e = to_epi(ep);
  const dim3 grid((L / RPB + 1) / 2, nclips);  // the same blocks as rows_inv_real_l<L, 1>
  if (dev::prunable<L>(h))
    return launch(name, KPTR((dev::k_rows_image_residual<L, true>)), grid, sh, s, [&] {
      hipLaunchKernelGGL((dev::k_rows_image_residual<L, true>), grid, dim3(256), sh, s, band, h, Wp, e, g, tw,
                         scale);
    });
  return launch(name, KPTR((dev::k_rows_image_residual<L, false>)), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_rows_image_residual<L, false>), grid, dim3(256), sh, s, band, h, Wp, e, g, tw,
                       scale);
  });
}

template <int L>
constexpr size_t col_lds() {
  return size_t(dev::ColBlock<L>::threads / FftPlan<L>::T) * lds_len<L>() * sizeof(cf);
}
template <int L>
unsigned col_blocks(int nt) {
  return unsigned((nt + dev::ColBlock<L>::tiles - 1) / dev::ColBlock<L>::tiles);
}

template <int L, int DIR>
int col_fft_l(const char *name, const cf *in, cf *out, int nt, int in_h, int out_h, const cf *tw, float scale,
              int nclips, hipStream_t s) {
  const size_t rin = in_h < 0 ? L : 2 * in_h + 1, rout = out_h < 0 ? L : 2 * out_h + 1;
  constexpr size_t sh = size_t(dev::ColBlock<L>::threads / FftPlan<L>::T) *
                        dev::Xch<L, dev::ColFftHalf<L>::value>::floats * sizeof(float);
  const dim3 grid(col_blocks<L>(nt), nclips);
  return launch(name, KPTR(dev::k_col_fft<L, DIR>), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_col_fft<L, DIR>), grid, dim3(dev::ColBlock<L>::threads), sh, s, in, out, nt, in_h,
                       out_h, size_t(nt) * rin * kC, size_t(nt) * rout * kC, tw, scale);
  });
}

template <int LA, int DIRA, int LB, int DIRB>
int col_resample_l(const char *name, const cf *in, cf *out, int nt, int h, const cf *twA, const cf *twB,
                   float scale, float gc, int nclips, hipStream_t s) {
  using RS = dev::Resample<LA, LB>;
  const dim3 grid(nt, nclips);
  return launch(name, KPTR(dev::k_col_resample<LA, DIRA, LB, DIRB>), grid, RS::bytes, s, [&] {
    hipLaunchKernelGGL((dev::k_col_resample<LA, DIRA, LB, DIRB>), grid, dim3(RS::threads), RS::bytes, s, in, out, h,
                       size_t(nt) * LA * kC, size_t(nt) * LB * kC, twA, twB, scale, gc);
  });
}

template <int Q>
int pass_y_fwd_q(const cf *bank, const cf *Mh, cf *Y, const PassGeo &pg, const cf *twQ, int nclips,
                 hipStream_t s) {
  Geo g = to_geo(pg);
  constexpr size_t sh = dev::ColXch<Q, false>::bytes + dev::TwLds<Q>::bytes;
  // kernels per block: enough blocks to fill the device (~2560), the rest
  // looped inside a block
  const int per_k = col_blocks<Q>(g.nt) * nclips;
  const int groups = std::max(1, std::min(g.K, (2560 + per_k - 1) / per_k));
  const int kpb = (g.K + groups - 1) / groups;
  const dim3 grid(col_blocks<Q>(g.nt), (g.K + kpb - 1) / kpb, nclips);
  if (dev::prunable<Q>(g.b))
    return launch("pass_y_fwd", KPTR(dev::k_pass_y_fwd<Q, true>), grid, sh, s, [&] {
      hipLaunchKernelGGL((dev::k_pass_y_fwd<Q, true>), grid, dim3(dev::ColBlock<Q>::threads), sh, s, bank, Mh, Y, g,
                         twQ, kpb);
    });
  return launch("pass_y_fwd", KPTR(dev::k_pass_y_fwd<Q, false>), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_pass_y_fwd<Q, false>), grid, dim3(dev::ColBlock<Q>::threads), sh, s, bank, Mh, Y, g,
                       twQ, kpb);
  });
}

template <int Q>
int pass_x_fwd_q(const cf *Y, const EpiPtrs &ep, cf *Ib, const PassGeo &pg, const cf *twQ, int nclips,
                 hipStream_t s) {
  constexpr int T = FftPlan<Q>::T, RPB = 256 / T;
  Geo g = to_geo(pg);
  Epi e = to_epi(ep);
  const bool band = Ib != nullptr;
  size_t sh = size_t(RPB) * dev::RowXch<Q>::floats * sizeof(float);
  sh = std::max(sh, size_t(256) * sizeof(double)) + dev::TwLds<Q>::bytes;
  const bool pr = dev::prunable<Q>(g.b);
  const dim3 grid(Q / RPB, nclips);
#define LITHO_PX_FWD(OUT, PR)                                                                              \
  return launch("pass_x_fwd", KPTR(dev::k_pass_x_fwd<Q, OUT, PR>), grid, sh, s, [&] {                       \
    hipLaunchKernelGGL((dev::k_pass_x_fwd<Q, OUT, PR>), grid, dim3(256), sh, s, Y, e, Ib, g, twQ);          \
  })
  if (!band) {
    if (pr) LITHO_PX_FWD(0, true);
    LITHO_PX_FWD(0, false);
  }
  if (pr) LITHO_PX_FWD(1, true);
  LITHO_PX_FWD(1, false);
#undef LITHO_PX_FWD
}

template <typename E, bool SPLIT, int P>
int pass_x_fwd_mfma_p(const cf *Y, cf *Ib, const PassGeo &pg, const void *tab, const cf *twl, const cf *twQ,
                      float sin, int nclips, hipStream_t s) {
  constexpr int Q = 32 * P;
  Geo g = to_geo(pg);
  using Vt = typename dev::Mfma<E>::V;
  constexpr int KS2 = P <= 16 ? 1 : 2, NC = SPLIT ? 6 : 3;
  const size_t sh = size_t(KS2) * NC * 64 * sizeof(Vt) + 16 * 64 * sizeof(cf) +
                    size_t(4) * dev::RowXch<Q>::floats * sizeof(float);
  const dim3 grid(Q / 4, nclips);
  const float sout = 1.0f / (sin * sin);
  return launch("pass_x_fwd_mfma", KPTR(dev::k_pass_x_fwd_mfma<E, SPLIT, P>), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_pass_x_fwd_mfma<E, SPLIT, P>), grid, dim3(256), sh, s, Y, Ib, g,
                       static_cast<const Vt *>(tab), twl, twQ, sin, sout);
  });
}
template <typename E, bool SPLIT>
int pass_x_fwd_mfma_e(const cf *Y, cf *Ib, const PassGeo &pg, const void *tab, const cf *twl, const cf *twQ,
                      float sin, int nclips, hipStream_t s) {
  switch (pg.Q / 32) {
#define LITHO_XM(P) \
  case P:           \
    return pass_x_fwd_mfma_p<E, SPLIT, P>(Y, Ib, pg, tab, twl, twQ, sin, nclips, s);
    LITHO_XM(2) LITHO_XM(3) LITHO_XM(4) LITHO_XM(5) LITHO_XM(6) LITHO_XM(8) LITHO_XM(10) LITHO_XM(12)
    LITHO_XM(16) LITHO_XM(20) LITHO_XM(24) LITHO_XM(32)
#undef LITHO_XM
    default:
      set_error("no two-stage row transform for inner grid %d", pg.Q);
      return LITHO_E_UNSUPPORTED;
  }
}

template <int Q>
int pass_x_adj_q(cf *Y, const float *G, size_t g_clip_stride, const cf *Gband, const PassGeo &pg, const cf *twQ,
                 int nclips, hipStream_t s) {
  constexpr int T = FftPlan<Q>::T, RPB = 256 / T;
  Geo g = to_geo(pg);
  const bool band = Gband != nullptr;
  const size_t sh = size_t(RPB) * dev::RowXch<Q>::floats * sizeof(float) + dev::TwLds<Q>::bytes;
  const bool pr = dev::prunable<Q>(g.b);
  const dim3 grid(Q / RPB, nclips);
#define LITHO_PX_ADJ(GIN, PR)                                                                              \
  return launch("pass_x_adj", KPTR(dev::k_pass_x_adj<Q, GIN, PR>), grid, sh, s, [&] {                      \
    hipLaunchKernelGGL((dev::k_pass_x_adj<Q, GIN, PR>), grid, dim3(256), sh, s, Y, G, g_clip_stride, Gband, g, \
                       twQ);                                                                               \
  })
  if (!band) {
    if (pr) LITHO_PX_ADJ(0, true);
    LITHO_PX_ADJ(0, false);
  }
  if (pr) LITHO_PX_ADJ(1, true);
  LITHO_PX_ADJ(1, false);
#undef LITHO_PX_ADJ
}

template <int Q>
int pass_y_adj_q(const cf *V, const cf *bank, double2 *part, const PassGeo &pg, const cf *twQ, int nclips,
                 hipStream_t s) {
  Geo g = to_geo(pg);
  constexpr size_t sh = dev::ColXch<Q, dev::ColAdjHalf<Q>::value>::bytes + dev::TwLds<Q>::bytes;
  const dim3 grid(col_blocks<Q>(g.nt), g.KC, nclips);
  if (dev::prunable<Q>(g.b))
    return launch("pass_y_adj", KPTR(dev::k_pass_y_adj<Q, true>), grid, sh, s, [&] {
      hipLaunchKernelGGL((dev::k_pass_y_adj<Q, true>), grid, dim3(dev::ColBlock<Q>::threads), sh, s, V, bank, part,
                         g, twQ);
    });
  return launch("pass_y_adj", KPTR(dev::k_pass_y_adj<Q, false>), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_pass_y_adj<Q, false>), grid, dim3(dev::ColBlock<Q>::threads), sh, s, V, bank, part, g,
                       twQ);
  });
}

template <int N>
int grad_cols_n(const double2 *part, int nparts, cf *tmp, const PassGeo &pg, const cf *twN, int nclips,
                hipStream_t s) {
  Geo g = to_geo(pg);
  constexpr size_t sh = col_lds<N>();
  const dim3 grid(col_blocks<N>(g.nt), nclips);
  if (dev::prunable<N>(g.b))
    return launch("grad_cols", KPTR(dev::k_grad_cols<N, true>), grid, sh, s, [&] {
      hipLaunchKernelGGL((dev::k_grad_cols<N, true>), grid, dim3(dev::ColBlock<N>::threads), sh, s, part, nparts,
                         tmp, g, twN);
    });
  return launch("grad_cols", KPTR(dev::k_grad_cols<N, false>), grid, sh, s, [&] {
    hipLaunchKernelGGL((dev::k_grad_cols<N, false>), grid, dim3(dev::ColBlock<N>::threads), sh, s, part, nparts,
                       tmp, g, twN);
  });
}


// ---------------------------------------------------------------- split-precision band GEMM

template <typename E, bool SPLIT, int NW>
int pass_y_fwd_mfma_nw(const cf *bank, const cf *Mh, cf *Y, const Geo &g, const void *tab, float sin, int nclips,
                       hipStream_t s) {
  using V = typename dev::Mfma<E>::V;
  constexpr int per_group = 32 * NW * dev::kGemmNtw;
  const dim3 grid((g.Bp + 31) / 32, (g.Q + per_group - 1) / per_group, unsigned(g.K) * nclips);
  const float sout = 1.0f / sin;
  return launch("pass_y_fwd_mfma", KPTR(dev::k_pass_y_fwd_mfma<E, SPLIT, NW>), grid, 0, s, [&] {
    hipLaunchKernelGGL((dev::k_pass_y_fwd_mfma<E, SPLIT, NW>), grid, dim3(64 * NW), 0, s, bank, Mh, Y, g,
                       static_cast<const V *>(tab), sin, sout);
  });
}

// Waves of the adjoint GEMM workgroup: ten when the 32-row ky tiles come in
// groups of ten, else four.
inline int adj_gemm_waves(int B) { return (B + 31) / 32 % 10 == 0 ? 10 : 4; }

template <typename E>
int pass_y_fwd_mfma_e(const cf *bank, const cf *Mh, cf *Y, const PassGeo &pg, const void *tab, bool split,
                      float sin, int nclips, hipStream_t s) {
  Geo g = to_geo(pg);
  if (g.Q % 32 != 0) {
    set_error("pass_y_fwd_mfma: inner grid %d is not a multiple of 32", g.Q);
    return LITHO_E_UNSUPPORTED;
  }
  // four waves per workgroup: two workgroups fit a CU at these register counts
  if (split) return pass_y_fwd_mfma_nw<E, true, 4>(bank, Mh, Y, g, tab, sin, nclips, s);
  return pass_y_fwd_mfma_nw<E, false, 4>(bank, Mh, Y, g, tab, sin, nclips, s);
}

template <typename E>
void fill_band_table_e(int Q, int b, std::vector<uint16_t> &out) {
  const int B = 2 * b + 1, ksteps = (B + 15) / 16, nQt = Q / 32;
  out.assign(size_t(ksteps) * nQt * 4 * 64 * 8, 0);
  for (int ks = 0; ks < ksteps; ++ks)
    for (int nt = 0; nt < nQt; ++nt)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const int ky = 16 * ks + 8 * (l >> 5) + j, y = 32 * nt + (l & 31);
          double re = 0, im = 0;
          if (ky < B) {
            const long long e = ((long long)(ky - b) * y) % Q;
            const double a = 2.0 * M_PI * double(e) / double(Q);
            re = std::cos(a);
            im = std::sin(a);
          }
          const E rh = E(float(re)), ih = E(float(im));
          const E rl = E(float(re - double(float(rh)))), il = E(float(im - double(float(ih))));
          const E vals[4] = {rh, rl, ih, il};
          for (int c = 0; c < 4; ++c) {
            uint16_t bits;
            std::memcpy(&bits, &vals[c], 2);
            out[((((size_t(ks) * nQt + nt) * 4 + c) * 64) + l) * 8 + j] = bits;
          }
        }
}


template <typename E, bool SPLIT, int NW>
int pass_y_adj_mfma_nw(const cf *V, const cf *bank, double2 *part, const Geo &g, const void *tab, int nclips,
                       hipStream_t s) {
  using Vt = typename dev::Mfma<E>::V;
  constexpr int per_group = 32 * NW;
  const dim3 grid((g.Bp + 31) / 32, (g.B + per_group - 1) / per_group, unsigned(g.KC) * nclips);
  return launch("pass_y_adj_mfma", KPTR(dev::k_pass_y_adj_mfma<E, SPLIT, NW>), grid, 0, s, [&] {
    hipLaunchKernelGGL((dev::k_pass_y_adj_mfma<E, SPLIT, NW>), grid, dim3(64 * NW), 0, s, V, bank, part, g,
                       static_cast<const Vt *>(tab));
  });
}

template <typename E>
int pass_y_adj_mfma_e(const cf *V, const cf *bank, double2 *part, const PassGeo &pg, const void *tab, bool split,
                      int nclips, hipStream_t s) {
  Geo g = to_geo(pg);
  if (g.Q % 16 != 0) {
    set_error("pass_y_adj_mfma: inner grid %d is not a multiple of 16", g.Q);
    return LITHO_E_UNSUPPORTED;
  }
  const bool ten = adj_gemm_waves(g.B) == 10;
  if (split)
    return ten ? pass_y_adj_mfma_nw<E, true, 10>(V, bank, part, g, tab, nclips, s)
               : pass_y_adj_mfma_nw<E, true, 4>(V, bank, part, g, tab, nclips, s);
  return ten ? pass_y_adj_mfma_nw<E, false, 10>(V, bank, part, g, tab, nclips, s)
             : pass_y_adj_mfma_nw<E, false, 4>(V, bank, part, g, tab, nclips, s);
}

template <typename E>
void fill_adj_table_e(int Q, int b, std::vector<uint16_t> &out) {
  const int B = 2 * b + 1, ksteps = Q / 16, nBt = (B + 31) / 32;
  out.assign(size_t(ksteps) * nBt * 4 * 64 * 8, 0);
  for (int ks = 0; ks < ksteps; ++ks)
    for (int nt = 0; nt < nBt; ++nt)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const int y = 16 * ks + 8 * (l >> 5) + j, ky = 32 * nt + (l & 31);
          double re = 0, im = 0;
          if (ky < B) {
            const long long e = ((long long)(ky - b) * y) % Q;
            const double a = -2.0 * M_PI * double(e) / double(Q);
            re = std::cos(a);
            im = std::sin(a);
          }
          const E rh = E(float(re)), ih = E(float(im));
          const E rl = E(float(re - double(float(rh)))), il = E(float(im - double(float(ih))));
          const E vals[4] = {rh, rl, ih, il};
          for (int c = 0; c < 4; ++c) {
            uint16_t bits;
            std::memcpy(&bits, &vals[c], 2);
            out[((((size_t(ks) * nBt + nt) * 4 + c) * 64) + l) * 8 + j] = bits;
          }
        }
}

}  // namespace

// Every transform length with an FFT plan (2^j, 3 * 2^j, 5 * 2^j): clip sides
// and inner grids alike.  All length switches below expand this one list.
#define LITHO_FFT_SIZES(X, A)                                                                       \
  X(64, A) X(96, A) X(128, A) X(160, A) X(192, A) X(256, A) X(320, A) X(384, A) X(512, A) X(640, A) \
  X(768, A) X(1024, A) X(1280, A) X(1536, A) X(2048, A) X(2560, A) X(3072, A) X(4096, A)

#define LITHO_CASE(L, CALL) \
  case L: {                 \
    constexpr int NN = L;   \
    return CALL;            \
  }

#define LITHO_DISPATCH_N(n, CALL)                   \
  switch (n) {                                      \
    LITHO_FFT_SIZES(LITHO_CASE, CALL)               \
    default:                                        \
      set_error("unsupported grid side %d", n);     \
      return LITHO_E_UNSUPPORTED;                   \
  }

#define LITHO_DISPATCH_Q(q, CALL)                   \
  switch (q) {                                      \
    LITHO_FFT_SIZES(LITHO_CASE, CALL)               \
    default:                                        \
      set_error("unsupported inner grid side %d", q); \
      return LITHO_E_UNSUPPORTED;                   \
  }

int run_rows_fwd_real(const char *name, int L, const float *in, size_t in_clip, cf2 *out, int h, int Wp,
                      const cf2 *tw, float scale, int nclips, hipStream_t s) {
  LITHO_DISPATCH_N(L, (rows_fwd_real_l<NN>(name, in, in_clip, (cf *)out, h, Wp, (const cf *)tw, scale, nclips,
                                           s)));
}
int run_rows_inv_real(const char *name, int L, const cf2 *in, int h, int Wp, float *out, const EpiPtrs &ep,
                      const PassGeo &g, const cf2 *tw, float scale, int nclips, hipStream_t s) {
  if (ep.image || ep.target) {
    LITHO_DISPATCH_N(L, (rows_inv_real_l<NN, 1>(name, (const cf *)in, h, Wp, out, ep, g, (const cf *)tw, scale,
                                                 nclips, s)));
  }
  LITHO_DISPATCH_N(L, (rows_inv_real_l<NN, 0>(name, (const cf *)in, h, Wp, out, ep, g, (const cf *)tw, scale,
                                               nclips, s)));
}
int run_rows_image_residual(const char *name, int L, cf2 *band, int h, int Wp, const EpiPtrs &ep,
                            const PassGeo &g, const cf2 *tw, float scale, int nclips, hipStream_t s) {
  if (!ep.target || !ep.loss_part) {
    set_error("%s: needs a target and loss partials", name);
    return LITHO_E_INVALID;
  }
  LITHO_DISPATCH_N(L, (rows_image_residual_l<NN>(name, (cf *)band, h, Wp, ep, g, (const cf *)tw, scale, nclips,
                                                 s)));
}
int run_rows_inv_thresh(const char *name, int L, const cf2 *in, int h, int Wp, float *out, double thr,
                        const cf2 *tw, float scale, int nclips, hipStream_t s) {
  PassGeo g;
  g.thr = thr;
  LITHO_DISPATCH_N(L, (rows_inv_real_l<NN, 2>(name, (const cf *)in, h, Wp, out, EpiPtrs{}, g, (const cf *)tw,
                                               scale, nclips, s)));
}
int run_col_fft(const char *name, int L, int dir, const cf2 *in, cf2 *out, int nt, int in_h, int out_h,
                const cf2 *tw, float scale, int nclips, hipStream_t s) {
  if (dir < 0) {
    LITHO_DISPATCH_Q(L, (col_fft_l<NN, -1>(name, (const cf *)in, (cf *)out, nt, in_h, out_h, (const cf *)tw,
                                            scale, nclips, s)));
  }
  LITHO_DISPATCH_Q(L, (col_fft_l<NN, +1>(name, (const cf *)in, (cf *)out, nt, in_h, out_h, (const cf *)tw, scale,
                                          nclips, s)));
}
// The resampling pairs with a fused column pass: the inner grids of the
// 1024^2 and 2048^2 clips.  Other pairs take the two column transforms.
bool col_resample_ok(int Q, int N) { return (Q == 640 && N == 1024) || (Q == 1280 && N == 2048); }
int run_col_resample(const char *name, int Q, int N, bool up, const cf2 *in, cf2 *out, int nt, int h,
                     const cf2 *twQ, const cf2 *twN, float scale, double blur_sigma_px, int nclips, hipStream_t s) {
  const float gc = blur_sigma_px > 0.0
                       ? float(2.0 * 3.14159265358979323846 * 3.14159265358979323846 * blur_sigma_px * blur_sigma_px /
                               (double(N) * double(N)))
                       : 0.f;
  const cf *i = (const cf *)in, *tq = (const cf *)twQ, *tn = (const cf *)twN;
  cf *o = (cf *)out;
  if (Q == 640 && N == 1024) {
    if (up) return col_resample_l<640, -1, 1024, +1>(name, i, o, nt, h, tq, tn, scale, gc, nclips, s);
    return col_resample_l<1024, -1, 640, +1>(name, i, o, nt, h, tn, tq, scale, gc, nclips, s);
  }
  if (Q == 1280 && N == 2048) {
    if (up) return col_resample_l<1280, -1, 2048, +1>(name, i, o, nt, h, tq, tn, scale, gc, nclips, s);
    return col_resample_l<2048, -1, 1280, +1>(name, i, o, nt, h, tn, tq, scale, gc, nclips, s);
  }
  set_error("%s: no fused resampling pass between %d and %d", name, Q, N);
  return LITHO_E_UNSUPPORTED;
}
int run_pass_y_fwd(const cf2 *bank, const cf2 *Mh, cf2 *Y, const PassGeo &pg, const cf2 *twQ, int nclips,
                   hipStream_t s) {
  LITHO_DISPATCH_Q(pg.Q, (pass_y_fwd_q<NN>((const cf *)bank, (const cf *)Mh, (cf *)Y, pg, (const cf *)twQ,
                                           nclips, s)));
}
int run_pass_x_fwd(const cf2 *Y, const EpiPtrs &ep, cf2 *Ib, const PassGeo &pg, const cf2 *twQ, int nclips,
                   hipStream_t s) {
  LITHO_DISPATCH_Q(pg.Q, (pass_x_fwd_q<NN>((const cf *)Y, ep, (cf *)Ib, pg, (const cf *)twQ, nclips, s)));
}
int run_pass_x_fwd_mfma(const cf2 *Y, cf2 *Ib, const PassGeo &g, const void *tab, const cf2 *twl, const cf2 *twQ,
                        int prec, int nclips, hipStream_t s) {
  if (!row_mfma_ok(g.Q, g.N)) {
    set_error("no two-stage row transform for inner grid %d of a %d grid", g.Q, g.N);
    return LITHO_E_UNSUPPORTED;
  }
  const bool split = prec == LITHO_PREC_F16X3 || prec == LITHO_PREC_BF16X3;
  const bool bf = prec == LITHO_PREC_BF16X3 || prec == LITHO_PREC_BF16;
  // the band rows are at most ~0.05 in magnitude: FP16 operands are scaled by
  // 2^12 so that the low halves stay normal; the image is scaled back by 2^-24
  const cf *y = (const cf *)Y, *tl = (const cf *)twl, *tq = (const cf *)twQ;
  cf *ib = (cf *)Ib;
  if (bf) {
    if (split) return pass_x_fwd_mfma_e<__bf16, true>(y, ib, g, tab, tl, tq, 1.0f, nclips, s);
    return pass_x_fwd_mfma_e<__bf16, false>(y, ib, g, tab, tl, tq, 1.0f, nclips, s);
  }
  if (split) return pass_x_fwd_mfma_e<_Float16, true>(y, ib, g, tab, tl, tq, 4096.0f, nclips, s);
  return pass_x_fwd_mfma_e<_Float16, false>(y, ib, g, tab, tl, tq, 4096.0f, nclips, s);
}
int run_pass_x_adj(cf2 *Y, const float *G, size_t g_clip_stride, const cf2 *Gband, const PassGeo &pg,
                   const cf2 *twQ, int nclips, hipStream_t s) {
  LITHO_DISPATCH_Q(pg.Q, (pass_x_adj_q<NN>((cf *)Y, G, g_clip_stride, (const cf *)Gband, pg, (const cf *)twQ,
                                           nclips, s)));
}
int run_pass_y_adj(const cf2 *V, const cf2 *bank, double2 *part, const PassGeo &pg, const cf2 *twQ, int nclips,
                   hipStream_t s) {
  LITHO_DISPATCH_Q(pg.Q, (pass_y_adj_q<NN>((const cf *)V, (const cf *)bank, part, pg, (const cf *)twQ, nclips,
                                           s)));
}
int run_grad_cols(const double2 *part, int nparts, cf2 *tmp, const PassGeo &pg, const cf2 *twN, int nclips,
                  hipStream_t s) {
  LITHO_DISPATCH_N(pg.N, (grad_cols_n<NN>(part, nparts, (cf *)tmp, pg, (const cf *)twN, nclips, s)));
}
int run_loss_reduce(const double *part, int n_per_clip, double *loss, int nclips, hipStream_t s) {
  return launch("loss_reduce", KPTR(dev::k_loss_reduce), dim3(nclips), 0, s, [&] {
    hipLaunchKernelGGL(dev::k_loss_reduce, dim3(nclips), dim3(256), 0, s, part, n_per_clip, loss);
  });
}

int run_pass_y_fwd_mfma(const cf2 *bank, const cf2 *Mh, cf2 *Y, const PassGeo &g, const void *tab, int prec,
                        int nclips, hipStream_t s) {
  const bool split = prec == LITHO_PREC_F16X3 || prec == LITHO_PREC_BF16X3;
  const bool bf = prec == LITHO_PREC_BF16X3 || prec == LITHO_PREC_BF16;
  // |Phi'_k M^| <= 1 (the bank's diagonal sum is the source weight sum, the
  // mask spectrum is scaled 1/N^2), so FP16 operands are scaled by 2^12: still
  // far from the FP16 maximum, and the low halves stay normal down to 2^-14.
  if (bf) return pass_y_fwd_mfma_e<__bf16>((const cf *)bank, (const cf *)Mh, (cf *)Y, g, tab, split, 1.0f, nclips, s);
  return pass_y_fwd_mfma_e<_Float16>((const cf *)bank, (const cf *)Mh, (cf *)Y, g, tab, split, 4096.0f, nclips, s);
}

int run_pass_y_adj_mfma(const cf2 *V, const cf2 *bank, double2 *part, const PassGeo &g, const void *tab, int prec,
                        int nclips, hipStream_t s) {
  const bool split = prec == LITHO_PREC_F16X3 || prec == LITHO_PREC_BF16X3;
  if (prec == LITHO_PREC_BF16X3 || prec == LITHO_PREC_BF16)
    return pass_y_adj_mfma_e<__bf16>((const cf *)V, (const cf *)bank, part, g, tab, split, nclips, s);
  return pass_y_adj_mfma_e<_Float16>((const cf *)V, (const cf *)bank, part, g, tab, split, nclips, s);
}

int adj_gemm_blocks(int Bp, int B) {
  const int per = 32 * adj_gemm_waves(B);
  return (Bp + 31) / 32 * ((B + per - 1) / per);
}

void fill_adj_table(int Q, int b, bool bf16, std::vector<uint16_t> &out) {
  if (bf16)
    fill_adj_table_e<__bf16>(Q, b, out);
  else
    fill_adj_table_e<_Float16>(Q, b, out);
}

template <typename E>
void fill_row_mfma_table_e(int Q, std::vector<uint16_t> &tab, std::vector<float2> &twl) {
  const int P = Q / 32;
  auto put = [&](int part, int c, int l, int j, double v) {
    const E h = E(float(v));
    const E lo = E(float(v - double(float(h))));
    uint16_t bits;
    std::memcpy(&bits, &h, 2);
    tab[((size_t(part) * 6 + c) * 64 + l) * 8 + j] = bits;
    std::memcpy(&bits, &lo, 2);
    tab[((size_t(part) * 6 + c + 3) * 64 + l) * 8 + j] = bits;
  };
  auto put_c = [&](int part, int l, int j, double re, double im) {
    put(part, 0, l, j, re);
    put(part, 1, l, j, im);
    put(part, 2, l, j, -im);
  };
  tab.assign(size_t(3) * 6 * 64 * 8, 0);
  for (int l = 0; l < 64; ++l)
    for (int j = 0; j < 8; ++j) {
      const int hl = l >> 5, m = l & 31;
      // stage 1: B[f1 = 8 hl + j][r = m] = exp(2 pi i (f1 - 8) r / 32)
      {
        const double a = 2.0 * M_PI * double(((8 * hl + j - 8) * m) % 32) / 32.0;
        put_c(0, l, j, std::cos(a), std::sin(a));
      }
      // stage 2, K-step t: B[k = 8 hl + j][s = m] = exp(2 pi i f0 s / P) with f0 the
      // row of stage 1's accumulator register 8 t + j in a lane of this half
      for (int t = 0; t < 2; ++t) {
        const int f0 = 16 * t + 8 * (j >> 2) + 4 * hl + (j & 3), sidx = m;
        double re = 0, im = 0;
        if (f0 < P && sidx < P) {
          const double a = 2.0 * M_PI * double((f0 * sidx) % P) / double(P);
          re = std::cos(a);
          im = std::sin(a);
        }
        put_c(1 + t, l, j, re, im);
      }
    }
  // twiddles w^(f0 r), w = exp(2 pi i / Q), for register i of lane l
  twl.assign(size_t(16) * 64, make_float2(0.f, 0.f));
  for (int i = 0; i < 16; ++i)
    for (int l = 0; l < 64; ++l) {
      const int f0 = 8 * (i >> 2) + 4 * (l >> 5) + (i & 3), r = l & 31;
      if (f0 >= P) continue;
      const double a = 2.0 * M_PI * double((f0 * r) % Q) / double(Q);
      twl[size_t(i) * 64 + l] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
}

void fill_band_table(int Q, int b, bool bf16, std::vector<uint16_t> &out) {
  if (bf16)
    fill_band_table_e<__bf16>(Q, b, out);
  else
    fill_band_table_e<_Float16>(Q, b, out);
}

bool row_mfma_ok(int Q, int N) {
  // the inner grids 32 P (P <= 32) of the resampled route
  return Q < N && Q % 32 == 0 && Q / 32 <= 32 && pass_threads(Q) > 0;
}

void fill_row_mfma_table(int Q, bool bf16, std::vector<uint16_t> &tab, std::vector<float2> &twl) {
  if (bf16)
    fill_row_mfma_table_e<__bf16>(Q, tab, twl);
  else
    fill_row_mfma_table_e<_Float16>(Q, tab, twl);
}

int twiddle_table(int L, std::vector<float2> &out) {
  switch (L) {
#define LITHO_TW(X, _)                                                            \
  case X:                                                                         \
    out.assign(std::max(1, dev::twiddle_table_size<X>()), make_float2(0.f, 0.f)); \
    dev::fill_twiddles<X>(out.data());                                            \
    return LITHO_OK;
    LITHO_FFT_SIZES(LITHO_TW, 0)
#undef LITHO_TW
    default:
      set_error("no FFT plan for length %d", L);
      return LITHO_E_UNSUPPORTED;
  }
}

int pass_threads(int L) {
  switch (L) {
#define LITHO_T(X, _) \
  case X:             \
    return FftPlan<X>::T;
    LITHO_FFT_SIZES(LITHO_T, 0)
#undef LITHO_T
    default: return 0;
  }
}

}  // namespace litho
