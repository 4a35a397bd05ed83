// Kernels of the steps after the image: Gaussian band filter (resist blur of
// Eq. 5 and the low-pass of Eq. 16), marching-squares contours of a level set
// (Sec. II-D, the contour of Eq. 5), edge placement error through focus
// (Eqs. 6-8), and the pieces of the Eq. 9 input channels.
//
// The contour and EPE extractions are stream compactions over the image:
// one wavefront per (row, 64-column chunk) classifies its cells or pixels,
// counts their items with two ballots (each cell or pixel yields 0, 1 or 2
// items), a one-block scan turns the per-chunk counts into offsets, and a
// second pass writes every item at its raster-order position.  Both passes
// read the image once from HBM (neighbouring rows come from L2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "common.hpp"
#include "post.hpp"

namespace litho {
namespace dev {

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ int lane_id() { return int(threadIdx.x & 63); }

// Exclusive prefix over the wavefront of per-lane counts in {0, 1, 2}, and the
// wavefront total (two ballots: the low and the high bit of the count).
__device__ __forceinline__ int wave_excl_012(int c, int &total) {
  const unsigned long long b0 = __ballot(c & 1), b1 = __ballot(c >> 1);
  const unsigned long long lt = (1ull << lane_id()) - 1ull;
  total = __popcll(b0) + 2 * __popcll(b1);
  return __popcll(b0 & lt) + 2 * __popcll(b1 & lt);
}

// ---------------------------------------------------------------- marching squares
// Cell (y, x) has corners c0 = v(y, x), c1 = v(y, x+1), c2 = v(y+1, x+1),
// c3 = v(y+1, x) (periodic); edge 0 joins c0-c1 (top), 1 joins c1-c2 (right),
// 2 joins c3-c2 (bottom), 3 joins c0-c3 (left).  A corner is inside when its
// value is at least the level.  A cell with one or three inside corners has one
// segment, a cell with two adjacent inside corners one, two diagonal inside
// corners (a saddle) two: the cell mean decides whether the centre is inside,
// and each corner whose state differs from the centre is cut off by its own
// segment.  A segment runs from its start edge to its end edge with the inside
// on its left in (x right, y down) coordinates, i.e. where
// cross(end - start, p - start) > 0, decided on the segment between the two
// edge midpoints (doubled integer coordinates below).
//
// Encoded case: bits 0-1 segment count, then (start, end) of the first and the
// second segment, two bits each, segments in increasing start edge.

__device__ __forceinline__ int seg_orient(int ea, int eb, int rx, int ry) {
  // edge midpoints in doubled coordinates: (1,0) (2,1) (1,2) (0,1)
  const int ax = (ea == 0 || ea == 2) ? 1 : (ea == 1 ? 2 : 0);
  const int ay = (ea == 1 || ea == 3) ? 1 : (ea == 2 ? 2 : 0);
  const int bx = (eb == 0 || eb == 2) ? 1 : (eb == 1 ? 2 : 0);
  const int by = (eb == 1 || eb == 3) ? 1 : (eb == 2 ? 2 : 0);
  const int cr = (bx - ax) * (ry - ay) - (by - ay) * (rx - ax);
  return cr > 0 ? (ea | (eb << 2)) : (eb | (ea << 2));  // start | end << 2
}

__device__ __forceinline__ int cell_case(float c0, float c1, float c2, float c3, float lv) {
  const bool i0 = c0 >= lv, i1 = c1 >= lv, i2 = c2 >= lv, i3 = c3 >= lv;
  const int s = int(i0) + int(i1) + int(i2) + int(i3);
  if (s == 0 || s == 4) return 0;
  const bool x0 = i0 != i1, x1 = i1 != i2, x2 = i3 != i2, x3 = i0 != i3;
  if (!(x0 && x1 && x2 && x3)) {
    // one segment between the two crossed edges; reference: first inside corner
    const int ea = x0 ? 0 : (x1 ? 1 : 2);
    const int eb = x3 ? 3 : (x2 ? 2 : 1);
    const int ci = i0 ? 0 : (i1 ? 1 : (i2 ? 2 : 3));
    const int rx = (ci == 1 || ci == 2) ? 2 : 0, ry = (ci >= 2) ? 2 : 0;
    return 1 | (seg_orient(ea, eb, rx, ry) << 2);
  }
  // saddle
  const float mean = 0.25f * ((c0 + c1) + (c2 + c3));
  const bool ctr = mean >= lv;
  const bool ins[4] = {i0, i1, i2, i3};
  int segs[2], k = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (ins[i] == ctr) continue;
    // the two edges meeting at corner i, in increasing order
    const int ea = (i == 0) ? 0 : (i == 1 ? 0 : (i == 2 ? 1 : 2));
    const int eb = (i == 0) ? 3 : (i == 1 ? 1 : (i == 2 ? 2 : 3));
    const int rx = ins[i] ? ((i == 1 || i == 2) ? 2 : 0) : 1;
    const int ry = ins[i] ? ((i >= 2) ? 2 : 0) : 1;
    segs[k++ & 1] = seg_orient(ea, eb, rx, ry);
  }
  int a = segs[0], b = segs[1];
  if ((b & 3) < (a & 3)) {
    const int t = a;
    a = b;
    b = t;
  }
  return 2 | (a << 2) | (b << 6);
}

__device__ __forceinline__ int case_count(int cs) { return cs & 3; }
__device__ __forceinline__ int case_start(int cs, int j) { return (cs >> (2 + 4 * j)) & 3; }
__device__ __forceinline__ int case_end(int cs, int j) { return (cs >> (4 + 4 * j)) & 3; }

// Crossing parameter on edge e of a cell, measured from the edge's first corner.
__device__ __forceinline__ float edge_u(int e, float c0, float c1, float c2, float c3, float lv) {
  const float a = (e == 0 || e == 3) ? c0 : (e == 1 ? c1 : c3);
  const float b = (e == 0) ? c1 : (e == 3 ? c3 : c2);
  return (lv - a) / (b - a);
}

struct Img {
  const float *v;
  int n;
  __device__ __forceinline__ float at(int y, int x) const { return v[size_t(y) * n + x]; }
};

// Work item of a wavefront: row y, chunk cx of 64 columns (nch chunks per row).
__device__ __forceinline__ bool wave_item(int items, int &item) {
  item = int(blockIdx.x) * int(blockDim.x / 64) + int(threadIdx.x / 64);
  return item < items;
}

__global__ __launch_bounds__(256) void k_contour_count(Img im, float lv, int nch, int *__restrict__ cnt) {
  int item;
  if (!wave_item(im.n * nch, item)) return;
  const int n = im.n, y = item / nch, x = (item % nch) * 64 + lane_id();
  int c = 0;
  if (x < n) {
    const int xp = x + 1 == n ? 0 : x + 1, yp = y + 1 == n ? 0 : y + 1;
    c = case_count(cell_case(im.at(y, x), im.at(y, xp), im.at(yp, xp), im.at(yp, x), lv));
  }
  int total;
  wave_excl_012(c, total);
  if (lane_id() == 0) cnt[item] = total;
}

// Exclusive scan of cnt[0..m) into off[0..m], off[m] = total, *total_out =
// total; one block of 1024 threads, each owning a contiguous range.
__global__ __launch_bounds__(1024) void k_scan_counts(const int *__restrict__ cnt, int m, int *__restrict__ off,
                                                      int *__restrict__ total_out) {
  __shared__ int part[1024];
  const int t = threadIdx.x, per = (m + 1023) / 1024;
  const int s0 = min(m, t * per), s1 = min(m, s0 + per);
  int sum = 0;
  for (int i = s0; i < s1; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int add = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int i = s0; i < s1; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) {
    off[m] = part[1023];
    *total_out = part[1023];
  }
}

__global__ __launch_bounds__(256) void k_contour_emit(Img im, float lv, int nch, const int *__restrict__ off,
                                                      int cap, int *__restrict__ cell, int *__restrict__ code,
                                                      float *__restrict__ u, int *__restrict__ next) {
  int item;
  if (!wave_item(im.n * nch, item)) return;
  const int n = im.n, y = item / nch, cx = item % nch, x = cx * 64 + lane_id();
  const bool valid = x < n;
  const int xs = valid ? x : n - 1;  // in-range column for inactive lanes
  const int xm = xs == 0 ? n - 1 : xs - 1, xp = xs + 1 == n ? 0 : xs + 1, xpp = xp + 1 == n ? 0 : xp + 1;
  const int ym = y == 0 ? n - 1 : y - 1, yp = y + 1 == n ? 0 : y + 1, ypp = yp + 1 == n ? 0 : yp + 1;
  const float a00 = im.at(ym, xs), a01 = im.at(ym, xp);
  const float b_m = im.at(y, xm), b00 = im.at(y, xs), b01 = im.at(y, xp), b02 = im.at(y, xpp);
  const float c_m = im.at(yp, xm), c00 = im.at(yp, xs), c01 = im.at(yp, xp), c02 = im.at(yp, xpp);
  const float d00 = im.at(ypp, xs), d01 = im.at(ypp, xp);
  const int cs_up = valid ? cell_case(a00, a01, b01, b00, lv) : 0;  // cell (y-1, x)
  const int cs_me = valid ? cell_case(b00, b01, c01, c00, lv) : 0;  // cell (y, x)
  const int cs_dn = valid ? cell_case(c00, c01, d01, d00, lv) : 0;  // cell (y+1, x)
  const int cs_lf = cell_case(b_m, b00, c00, c_m, lv);              // cell (y, x-1)
  const int cs_rt = cell_case(b01, b02, c02, c01, lv);              // cell (y, x+1)
  int tot;
  const int p_up = wave_excl_012(case_count(cs_up), tot);
  const int p_me = wave_excl_012(case_count(cs_me), tot);
  const int p_dn = wave_excl_012(case_count(cs_dn), tot);
  if (!valid) return;
  const int nme = case_count(cs_me);
  if (nme == 0) return;
  const int i_me = off[y * nch + cx] + p_me;
  const int i_up = off[ym * nch + cx] + p_up;
  const int i_dn = off[yp * nch + cx] + p_dn;
  const int i_lf = x == 0 ? off[(y + 1) * nch] - case_count(cs_lf) : i_me - case_count(cs_lf);
  const int i_rt = x == n - 1 ? off[y * nch] : i_me + nme;
  for (int j = 0; j < nme; ++j) {
    const int g = i_me + j;
    if (g >= cap) break;
    const int st = case_start(cs_me, j), en = case_end(cs_me, j);
    const int nb = en == 0 ? cs_up : (en == 1 ? cs_rt : (en == 2 ? cs_dn : cs_lf));
    const int ib = en == 0 ? i_up : (en == 1 ? i_rt : (en == 2 ? i_dn : i_lf));
    const int want = en ^ 2;  // the shared edge, seen from the neighbour
    const int k = (case_count(nb) == 2 && case_start(nb, 0) != want) ? 1 : 0;
    cell[g] = y * n + x;
    code[g] = st * 4 + en;
    u[2 * size_t(g)] = edge_u(st, b00, b01, c01, c00, lv);
    u[2 * size_t(g) + 1] = edge_u(en, b00, b01, c01, c00, lv);
    next[g] = ib + k;
  }
}

// ---------------------------------------------------------------- EPE sites (Eqs. 6-8)
// Sites are the 4-neighbour pixel pairs whose binary targets (T >= 0.5)
// differ: per pixel (y, x) in raster order first the pair with (y, x+1), then
// with (y+1, x), periodic.

__device__ __forceinline__ int site_bits(const Img &t, int y, int x) {
  const int n = t.n, xp = x + 1 == n ? 0 : x + 1, yp = y + 1 == n ? 0 : y + 1;
  const bool b = t.at(y, x) >= 0.5f;
  return int(b != (t.at(y, xp) >= 0.5f)) | (int(b != (t.at(yp, x) >= 0.5f)) << 1);
}

__global__ __launch_bounds__(256) void k_site_count(Img tg, int nch, int *__restrict__ cnt) {
  int item;
  if (!wave_item(tg.n * nch, item)) return;
  const int n = tg.n, y = item / nch, x = (item % nch) * 64 + lane_id();
  int c = 0;
  if (x < n) {
    const int s = site_bits(tg, y, x);
    c = (s & 1) + (s >> 1);
  }
  int total;
  wave_excl_012(c, total);
  if (lane_id() == 0) cnt[item] = total;
}

// Eq. 6 at one site of one latent image: EPE = -(E_eff - t_eff) / |grad E_eff|
// with E_eff and its gradient at the midpoint of the pair: mean of the two
// pixels, normal derivative their difference, tangential derivative a quarter
// of the difference between the sums of the neighbouring pairs on either side.
__device__ __forceinline__ float site_epe(const Img &e, int y, int x, int dir, float t_eff) {
  const int n = e.n, xp = x + 1 == n ? 0 : x + 1, yp = y + 1 == n ? 0 : y + 1;
  const int xm = x == 0 ? n - 1 : x - 1, ym = y == 0 ? n - 1 : y - 1;
  const float p = e.at(y, x);
  float q, gt;
  if (dir == 0) {
    q = e.at(y, xp);
    gt = 0.25f * ((e.at(yp, x) + e.at(yp, xp)) - (e.at(ym, x) + e.at(ym, xp)));
  } else {
    q = e.at(yp, x);
    gt = 0.25f * ((e.at(y, xp) + e.at(yp, xp)) - (e.at(y, xm) + e.at(yp, xm)));
  }
  const float ev = 0.5f * (p + q) - t_eff;
  const float g = hypotf(q - p, gt);
  if (g > 0.f) return -ev / g;
  return ev == 0.f ? 0.f : (ev > 0.f ? -INFINITY : INFINITY);
}

__global__ __launch_bounds__(256) void k_site_emit(Img tg, const float *__restrict__ E, int P, int nch,
                                                   const int *__restrict__ off, int cap, EpeRule rule,
                                                   int *__restrict__ site, int *__restrict__ dir,
                                                   float *__restrict__ epe) {
  int item;
  if (!wave_item(tg.n * nch, item)) return;
  const int n = tg.n, y = item / nch, x = (item % nch) * 64 + lane_id();
  const int s = x < n ? site_bits(tg, y, x) : 0;
  int tot;
  const int pre = wave_excl_012((s & 1) + (s >> 1), tot);
  if (s == 0) return;
  int g = off[item] + pre;
  for (int d = 0; d < 2; ++d) {
    if (!((s >> d) & 1)) continue;
    if (g >= cap) return;
    site[g] = y * n + x;
    dir[g] = d;
    float *row = epe + size_t(g) * (P + 2);
    float sum = 0.f, e0 = 0.f;
    for (int p = 0; p < P; ++p) {
      const float v = site_epe(Img{E + size_t(p) * n * n, n}, y, x, d, rule.t_eff);
      row[p] = v;
      sum += v;
      if (p == rule.f0) e0 = v;
    }
    const float avg = sum / float(P);
    row[P] = avg;
    row[P + 1] = e0 > rule.tol_pos ? e0 - rule.tol_pos : (e0 < rule.tol_neg ? e0 - rule.tol_neg : avg);
    ++g;
  }
}

// ---------------------------------------------------------------- band filters

// Multiplies a centred band [tiles][rows][4] (|kx|, |ky| <= h, rows = 2h+1;
// columns beyond the band are padding) by the Gaussian transfer function
// exp(-c (kx^2 + ky^2)), c = 2 pi^2 s^2 / N^2, of every one of nclips bands.
__global__ __launch_bounds__(256) void k_band_gauss(float2 *__restrict__ band, int h, int nt, float c,
                                                    size_t clip_stride) {
  const int rows = 2 * h + 1;
  const size_t per = size_t(nt) * rows * 4;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= per) return;
  const int col = int(i % 4), r = int((i / 4) % rows), jt = int(i / (4 * size_t(rows)));
  const int kx = jt * 4 + col - h, ky = r - h;
  float2 *p = band + size_t(blockIdx.y) * clip_stride + i;
  const float g = kx <= h ? expf(-c * float(kx * kx + ky * ky)) : 0.f;
  float2 v = *p;
  v.x *= g;
  v.y *= g;
  *p = v;
}

// part[clip][tile][ky][c] = psi[tile][ky][c] * Mh[clip][tile][ky][c] (complex,
// FP64 result): the band of the mask filtered by one combined kernel.
__global__ __launch_bounds__(256) void k_band_mul_psi(const double2 *__restrict__ psi,
                                                      const float2 *__restrict__ mh, size_t per,
                                                      double2 *__restrict__ part) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= per) return;
  const size_t o = size_t(blockIdx.y) * per + i;
  const double2 a = psi[i];
  const float2 m = mh[o];
  part[o] = make_double2(a.x * double(m.x) - a.y * double(m.y), a.x * double(m.y) + a.y * double(m.x));
}

// Eq. 9 channels, channel last: out[clip][y][x][c] = clip((v_c - lo_c) / (hi_c - lo_c), 0, 1)
// for v_0 = the layout, v_1 = its image, v_2 = dI/dM; no mapping when norm is off.
__global__ __launch_bounds__(256) void k_channels(const float *__restrict__ zt, const float *__restrict__ img,
                                                  size_t img_clip, const float *__restrict__ sens, size_t nn,
                                                  ChanNorm nm, float *__restrict__ out) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const size_t clip = blockIdx.y;
  const float v[3] = {zt[clip * nn + i], img[clip * img_clip + i], sens[clip * nn + i]};
  float *o = out + (clip * nn + i) * 3;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float w = v[c];
    if (nm.on) w = fminf(1.f, fmaxf(0.f, (w - nm.lo[c]) * nm.inv[c]));
    o[c] = w;
  }
}

// ---------------------------------------------------------------- halo tiling
// Tile t (raster order, tx tiles per row) has its core at (ti c, tj c) and its
// n x n window at (ti c - halo, tj c - halo); the layout is H x W, opaque
// (0) outside.

__device__ __forceinline__ void tile_origin(const TileGeo &g, int tile, int &y0, int &x0) {
  y0 = (tile / g.tx) * g.c - g.halo;
  x0 = (tile % g.tx) * g.c - g.halo;
}

// out[t][y][x] = layout(y0 + y, x0 + x), 0 outside the layout.
__global__ __launch_bounds__(256) void k_tile_gather(const float *__restrict__ a, TileGeo g,
                                                     float *__restrict__ out) {
  const size_t nn = size_t(g.n) * g.n, i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  int y0, x0;
  tile_origin(g, g.t0 + int(blockIdx.y), y0, x0);
  const int Y = y0 + int(i / g.n), X = x0 + int(i % g.n);
  const bool in = Y >= 0 && Y < g.H && X >= 0 && X < g.W;
  out[blockIdx.y * nn + i] = in ? a[size_t(Y) * g.W + X] : 0.f;
}

// img[p][Y][X] = tile image [t][p][halo + yy][halo + xx] on the core pixels inside the layout.
__global__ __launch_bounds__(256) void k_tile_cores(const float *__restrict__ timg, int P, TileGeo g,
                                                    float *__restrict__ img) {
  const size_t cc = size_t(g.c) * g.c, i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= cc) return;
  const int t = blockIdx.y, p = blockIdx.z;
  int y0, x0;
  tile_origin(g, g.t0 + t, y0, x0);
  const int yy = int(i / g.c), xx = int(i % g.c);
  const int Y = y0 + g.halo + yy, X = x0 + g.halo + xx;
  if (Y >= g.H || X >= g.W) return;
  img[(size_t(p) * g.H + Y) * g.W + X] =
      timg[((size_t(t) * P + p) * g.n + g.halo + yy) * g.n + g.halo + xx];
}

// Resist, loss and residual of a tile, restricted to its core: Z = sigmoid(a (I - thr)),
// d = Z - T, G = w_p 2 d a Z (1 - Z) (L1: w_p sign(d) a Z (1 - Z)) on core pixels inside
// the layout and 0 elsewhere; part[(t P + p) blocks + block] = sum of w_p d^2 (|d|).
__global__ __launch_bounds__(256) void k_tile_residual(const float *__restrict__ timg,
                                                       const float *__restrict__ target, int P, TileGeo g,
                                                       TileLoss lo, float *__restrict__ G,
                                                       double *__restrict__ part) {
  __shared__ double red[256];
  const size_t nn = size_t(g.n) * g.n, i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int t = blockIdx.y, p = blockIdx.z;
  double l = 0.0;
  if (i < nn) {
    int y0, x0;
    tile_origin(g, g.t0 + t, y0, x0);
    const int y = int(i / g.n), x = int(i % g.n), Y = y0 + y, X = x0 + x;
    const bool core = y >= g.halo && y < g.halo + g.c && x >= g.halo && x < g.halo + g.c && Y < g.H && X < g.W;
    const size_t o = (size_t(t) * P + p) * nn + i;
    float gv = 0.f;
    if (core) {
      const float w = lo.w[p];
      const float z = 1.0f / (1.0f + expf(-lo.slope * (timg[o] - lo.thr)));
      const float d = z - target[size_t(Y) * g.W + X];
      if (lo.l1) {
        gv = w * (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) * lo.slope * z * (1.0f - z);
        l = double(w) * double(fabsf(d));
      } else {
        gv = 2.0f * w * d * lo.slope * z * (1.0f - z);
        l = double(w) * double(d) * double(d);
      }
    }
    G[o] = gv;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t(t) * P + p) * gridDim.x + blockIdx.x] = red[0];
}

// grad(Y, X) += sum over the tiles t0 .. t0 + cnt - 1 whose window holds (Y, X),
// in tile order, of their gradient at the window position.
__global__ __launch_bounds__(256) void k_tile_grad_add(const float *__restrict__ tg, TileGeo g, int cnt,
                                                       float *__restrict__ grad) {
  const size_t HW = size_t(g.H) * g.W, i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= HW) return;
  const int Y = int(i / g.W), X = int(i % g.W);
  const int ay = Y + g.halo - g.n + 1, ax = X + g.halo - g.n + 1;
  const int i0 = ay <= 0 ? 0 : (ay + g.c - 1) / g.c, i1 = min(g.ty - 1, (Y + g.halo) / g.c);
  const int j0 = ax <= 0 ? 0 : (ax + g.c - 1) / g.c, j1 = min(g.tx - 1, (X + g.halo) / g.c);
  const size_t nn = size_t(g.n) * g.n;
  float s = 0.f;
  for (int ti = i0; ti <= i1; ++ti)
    for (int tj = j0; tj <= j1; ++tj) {
      const int tile = ti * g.tx + tj;
      if (tile < g.t0 || tile >= g.t0 + cnt) continue;
      const int y = Y - (ti * g.c - g.halo), x = X - (tj * g.c - g.halo);
      s += tg[size_t(tile - g.t0) * nn + size_t(y) * g.n + x];
    }
  grad[i] += s;
}

__global__ __launch_bounds__(256) void k_fill(float *__restrict__ a, size_t n, float v) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

}  // namespace dev

// ---------------------------------------------------------------- allocation-free scratch
// Counts and offsets of the compaction passes for the largest supported
// image (n = 4096: 4096 rows x 64 chunks, twice, plus the total), for the
// allocation-free contour entry point.  Every device that runs it holds one
// copy for the life of the process.
constexpr int kNoAllocMaxN = 4096;
constexpr size_t kNoAllocInts = 2 * size_t(kNoAllocMaxN) * ((kNoAllocMaxN + 63) / 64) + 1;
static __device__ __align__(256) int scratch[kNoAllocInts];

// ======================================================================== host launchers

namespace {
int check_launch(const char *name) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s launch failed: %s", name, hipGetErrorString(e));
    return LITHO_E_HIP;
  }
  return LITHO_OK;
}
unsigned wave_blocks(int items) { return unsigned((items + 3) / 4); }
}  // namespace

int compaction_chunks(int n) { return (n + 63) / 64; }

int noalloc_max_n() { return kNoAllocMaxN; }

// Device address of this device's copy of the static scratch array, looked up
// once per device (the array's name in host code is only a stand-in).
int noalloc_scratch(int **out, size_t *ints) {
  static std::mutex mu;
  static int *addr[64] = {};
  int d = 0;
  LITHO_HIP_TRY(hipGetDevice(&d));
  if (d < 0 || d >= 64) {
    set_error("litho: device %d beyond the 64 the allocation-free scratch table covers", d);
    return LITHO_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[d]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("litho: hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
      return LITHO_E_HIP;
    }
    addr[d] = static_cast<int *>(p);
  }
  *out = addr[d];
  *ints = kNoAllocInts;
  return LITHO_OK;
}

int run_contours(const float *img, int n, float level, int *cnt, int *off, int *total, int cap, int *cell,
                 int *code, float *u, int *next, hipStream_t s) {
  const int nch = compaction_chunks(n), items = n * nch;
  dev::Img im{img, n};
  prof_begin("contour_count", s);
  hipLaunchKernelGGL(dev::k_contour_count, dim3(wave_blocks(items)), dim3(256), 0, s, im, level, nch, cnt);
  prof_end("contour_count", s);
  LITHO_TRY(check_launch("contour_count"));
  prof_begin("scan_counts", s);
  hipLaunchKernelGGL(dev::k_scan_counts, dim3(1), dim3(1024), 0, s, cnt, items, off, total);
  prof_end("scan_counts", s);
  LITHO_TRY(check_launch("scan_counts"));
  prof_begin("contour_emit", s);
  hipLaunchKernelGGL(dev::k_contour_emit, dim3(wave_blocks(items)), dim3(256), 0, s, im, level, nch, off, cap, cell,
                     code, u, next);
  prof_end("contour_emit", s);
  return check_launch("contour_emit");
}

int run_epe(const float *target, const float *E, int n, int P, const EpeRule &rule, int *cnt, int *off,
            int *total, int cap, int *site, int *dir, float *epe, hipStream_t s) {
  const int nch = compaction_chunks(n), items = n * nch;
  dev::Img tg{target, n};
  prof_begin("site_count", s);
  hipLaunchKernelGGL(dev::k_site_count, dim3(wave_blocks(items)), dim3(256), 0, s, tg, nch, cnt);
  prof_end("site_count", s);
  LITHO_TRY(check_launch("site_count"));
  prof_begin("scan_counts", s);
  hipLaunchKernelGGL(dev::k_scan_counts, dim3(1), dim3(1024), 0, s, cnt, items, off, total);
  prof_end("scan_counts", s);
  LITHO_TRY(check_launch("scan_counts"));
  prof_begin("site_emit", s);
  hipLaunchKernelGGL(dev::k_site_emit, dim3(wave_blocks(items)), dim3(256), 0, s, tg, E, P, nch, off, cap, rule,
                     site, dir, epe);
  prof_end("site_emit", s);
  return check_launch("site_emit");
}

int run_tile_gather(const float *layout, const TileGeo &g, int cnt, float *out, hipStream_t s) {
  const size_t nn = size_t(g.n) * g.n;
  prof_begin("tile_gather", s);
  hipLaunchKernelGGL(dev::k_tile_gather, dim3(unsigned((nn + 255) / 256), unsigned(cnt)), dim3(256), 0, s, layout,
                     g, out);
  prof_end("tile_gather", s);
  return check_launch("tile_gather");
}

int run_tile_cores(const float *timg, int P, const TileGeo &g, int cnt, float *img, hipStream_t s) {
  const size_t cc = size_t(g.c) * g.c;
  prof_begin("tile_cores", s);
  hipLaunchKernelGGL(dev::k_tile_cores, dim3(unsigned((cc + 255) / 256), unsigned(cnt), unsigned(P)), dim3(256), 0,
                     s, timg, P, g, img);
  prof_end("tile_cores", s);
  return check_launch("tile_cores");
}

int tile_residual_blocks(int n) { return int((size_t(n) * n + 255) / 256); }

int run_tile_residual(const float *timg, const float *target, int P, const TileGeo &g, const TileLoss &lo, int cnt,
                      float *G, double *part, hipStream_t s) {
  prof_begin("tile_residual", s);
  hipLaunchKernelGGL(dev::k_tile_residual, dim3(unsigned(tile_residual_blocks(g.n)), unsigned(cnt), unsigned(P)),
                     dim3(256), 0, s, timg, target, P, g, lo, G, part);
  prof_end("tile_residual", s);
  return check_launch("tile_residual");
}

int run_tile_grad_add(const float *tg, const TileGeo &g, int cnt, float *grad, hipStream_t s) {
  const size_t HW = size_t(g.H) * g.W;
  prof_begin("tile_grad_add", s);
  hipLaunchKernelGGL(dev::k_tile_grad_add, dim3(unsigned((HW + 255) / 256)), dim3(256), 0, s, tg, g, cnt, grad);
  prof_end("tile_grad_add", s);
  return check_launch("tile_grad_add");
}

int run_fill(float *a, size_t n, float v, hipStream_t s) {
  if (n == 0) return LITHO_OK;
  hipLaunchKernelGGL(dev::k_fill, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a, n, v);
  return check_launch("fill");
}

int run_band_gauss(float2 *band, int h, int nt, double N, double sigma_px, size_t clip_stride, int nclips,
                   hipStream_t s) {
  if (nclips <= 0 || sigma_px <= 0.0) return LITHO_OK;
  const size_t per = size_t(nt) * (2 * h + 1) * 4;
  const float c = float(2.0 * 3.14159265358979323846 * 3.14159265358979323846 * sigma_px * sigma_px / (N * N));
  prof_begin("band_gauss", s);
  hipLaunchKernelGGL(dev::k_band_gauss, dim3(unsigned((per + 255) / 256), unsigned(nclips)), dim3(256), 0, s, band,
                     h, nt, c, clip_stride);
  prof_end("band_gauss", s);
  return check_launch("band_gauss");
}

int run_band_mul_psi(const double2 *psi, const float2 *mh, size_t per, double2 *part, int nclips, hipStream_t s) {
  if (nclips <= 0) return LITHO_OK;
  prof_begin("band_mul_psi", s);
  hipLaunchKernelGGL(dev::k_band_mul_psi, dim3(unsigned((per + 255) / 256), unsigned(nclips)), dim3(256), 0, s, psi,
                     mh, per, part);
  prof_end("band_mul_psi", s);
  return check_launch("band_mul_psi");
}

int run_channels(const float *zt, const float *img, size_t img_clip, const float *sens, int n, const ChanNorm &nm,
                 float *out, int nclips, hipStream_t s) {
  if (nclips <= 0) return LITHO_OK;
  const size_t nn = size_t(n) * n;
  prof_begin("channels", s);
  hipLaunchKernelGGL(dev::k_channels, dim3(unsigned((nn + 255) / 256), unsigned(nclips)), dim3(256), 0, s, zt, img,
                     img_clip, sens, nn, nm, out);
  prof_end("channels", s);
  return check_launch("channels");
}

}  // namespace litho
