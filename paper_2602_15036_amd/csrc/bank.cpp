// Host FP64 construction of the SOCS kernel bank.
//
// Eq. 2 (Sec. III-A) writes the TCC as a source integral of pupil products.
// With a sampled source it factors as TCC = A A^H, A[f, s] = sqrt(S_s) P(f + sigma_s),
// so the nonzero eigenpairs of Eq. 3 follow from the small n_source x n_source
// Gram matrix A^H A: if A^H A nu = lambda nu then Phi = A nu / sqrt(lambda) is a
// unit eigenvector of the TCC with the same eigenvalue.  Only the Gram matrix is
// decomposed (own cyclic Jacobi, FP64), so the band-sized TCC is never formed.
#include "bank.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

#include "common.hpp"

namespace litho {

std::vector<SourcePoint> sample_source(const litho_optics_t &o) {
  std::vector<SourcePoint> pts;
  if (o.source_kind == LITHO_SRC_POINTS) {
    double sum = 0.0;
    for (int s = 0; s < o.n_src_points; ++s) sum += o.src_points[3 * s + 2];
    for (int s = 0; s < o.n_src_points; ++s)
      pts.push_back({o.src_points[3 * s], o.src_points[3 * s + 1], o.src_points[3 * s + 2] / sum});
    return pts;
  }
  const int h = (o.source_grid - 1) / 2;
  const double lo = o.sigma_in * o.sigma_in * h * h;
  const double hi = o.sigma_out * o.sigma_out * h * h;
  for (int j = -h; j <= h; ++j) {
    for (int i = -h; i <= h; ++i) {
      const double r2 = double(i * i + j * j);
      bool keep = (lo - 1e-9) <= r2 && r2 <= (hi + 1e-9);
      if (o.source_kind == LITHO_SRC_DIPOLE_X) keep = keep && std::abs(j) <= std::abs(i);
      if (o.source_kind == LITHO_SRC_DIPOLE_Y) keep = keep && std::abs(i) <= std::abs(j);
      if (keep) pts.push_back({double(i) / h, double(j) / h, 0.0});
    }
  }
  for (auto &p : pts) p.w = 1.0 / double(pts.size());
  return pts;
}

// Pupil of Eq. 2 at index-unit frequency (u, v): NA cut-off and the defocus
// Zernike term W = (F NA^2 / 4)(2 rho^2 - 1), phase 2 pi W / lambda.
static inline cd pupil(double u, double v, double R, double wl, double na, double focus) {
  const double d2 = u * u + v * v;
  if (!(d2 <= R * R)) return cd(0.0, 0.0);
  const double rho2 = d2 / (R * R);
  const double coeff = focus * na * na / 4.0;
  const double ph = (2.0 * M_PI / wl) * coeff * (2.0 * rho2 - 1.0);
  return cd(std::cos(ph), std::sin(ph));
}

void hermitian_jacobi(int n, std::vector<cd> &a, std::vector<double> &w, std::vector<cd> &v) {
  v.assign(size_t(n) * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) v[size_t(i) * n + i] = 1.0;
  auto A = [&](int r, int c) -> cd & { return a[size_t(r) * n + c]; };
  auto V = [&](int r, int c) -> cd & { return v[size_t(r) * n + c]; };
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale += std::abs(A(i, i).real());
  scale = std::max(scale, 1e-300);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(A(p, q));
    if (std::sqrt(off) <= 1e-17 * scale) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double mag = std::abs(A(p, q));
        if (mag <= 1e-300) continue;
        // Phase step: scale row/column q so that a_pq becomes real positive.
        const cd ph = A(p, q) / mag;       // e^{i phi}
        const cd phc = std::conj(ph);
        for (int k = 0; k < n; ++k) {
          A(k, q) *= phc;                  // column q times e^{-i phi}
          V(k, q) *= phc;
        }
        for (int k = 0; k < n; ++k) A(q, k) *= ph;   // row q times e^{+i phi}
        // Real Jacobi rotation on the now real symmetric (p, q) block.
        const double app = A(p, p).real(), aqq = A(q, q).real();
        const double bpq = A(p, q).real();
        const double theta = (aqq - app) / (2.0 * bpq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::abs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0);
        const double s = t * c;
        for (int k = 0; k < n; ++k) {      // A <- A P
          const cd akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
          const cd vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * vkq;
          V(k, q) = s * vkp + c * vkq;
        }
        for (int k = 0; k < n; ++k) {      // A <- P^T A
          const cd apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        A(p, q) = 0.0;
        A(q, p) = 0.0;
      }
    }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A(i, i).real();
}

int build_host_bank(const litho_optics_t &o, HostBank &hb) {
  const bool points = o.source_kind == LITHO_SRC_POINTS;
  if (o.n <= 0 || !(o.pixel_nm > 0) || !(o.wavelength_nm > 0) || !(o.na > 0) || o.n_focus < 1 ||
      o.n_focus > 8 || !o.focus_nm || o.K < 1 ||
      (!points && (o.source_grid < 3 || (o.source_grid % 2) == 0 || o.sigma_in < 0 || o.sigma_out < o.sigma_in ||
                   o.sigma_out > 1.0))) {
    set_error("litho_kernels_build: invalid optics");
    return LITHO_E_INVALID;
  }
  if (o.source_kind < LITHO_SRC_ANNULAR || o.source_kind > LITHO_SRC_POINTS) {
    set_error("litho_kernels_build: unknown source kind %d", o.source_kind);
    return LITHO_E_INVALID;
  }
  double sigma_max = o.sigma_out;
  if (points) {
    if (!o.src_points || o.n_src_points < 1) {
      set_error("litho_kernels_build: a point source needs src_points");
      return LITHO_E_INVALID;
    }
    double wsum = 0.0;
    sigma_max = 0.0;
    for (int s = 0; s < o.n_src_points; ++s) {
      const double sx = o.src_points[3 * s], sy = o.src_points[3 * s + 1], w = o.src_points[3 * s + 2];
      const double r = std::hypot(sx, sy);
      if (!(w >= 0.0) || !(r <= 1.0)) {
        set_error("litho_kernels_build: source point %d has |sigma| > 1 or a negative weight", s);
        return LITHO_E_INVALID;
      }
      sigma_max = std::max(sigma_max, r);
      wsum += w;
    }
    if (!(wsum > 0.0)) {
      set_error("litho_kernels_build: the source weights sum to zero");
      return LITHO_E_INVALID;
    }
  }
  const std::vector<SourcePoint> src = sample_source(o);
  const int ns = int(src.size());
  if (ns == 0) {
    set_error("litho_kernels_build: the source has no sample points");
    return LITHO_E_INVALID;
  }
  if (o.K > ns) {
    set_error("litho_kernels_build: K=%d exceeds the TCC rank bound (%d source points)", o.K, ns);
    return LITHO_E_INVALID;
  }
  const double R = o.na * o.n * o.pixel_nm / o.wavelength_nm;
  const int b = int(std::floor((1.0 + sigma_max) * R));
  const int B = 2 * b + 1;
  if (B > o.n) {
    set_error("litho_kernels_build: band side %d exceeds the grid side %d (undersampled clip)", B, o.n);
    return LITHO_E_INVALID;
  }
  hb.n = o.n; hb.b = b; hb.B = B; hb.K = o.K; hb.n_focus = o.n_focus; hb.n_source = ns; hb.R = R;
  hb.dose = o.dose > 0 ? o.dose : 1.0;
  hb.lambda.assign(size_t(o.n_focus) * o.K, 0.0);
  hb.phi.assign(size_t(o.n_focus) * o.K * B * B, cd(0.0, 0.0));
  hb.gap.assign(o.n_focus, 1.0);

  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  for (int p = 0; p < o.n_focus; ++p) {
    const double F = o.focus_nm[p];
    // Gram matrix A^H A, accumulated over band rows in parallel (each thread
    // owns a private partial sum; the partials are added in thread order).
    std::vector<std::vector<cd>> part(nthreads, std::vector<cd>(size_t(ns) * ns, cd(0.0, 0.0)));
    auto work = [&](unsigned tid) {
      std::vector<cd> a(ns);
      std::vector<int> nz;
      nz.reserve(ns);
      std::vector<cd> &g = part[tid];
      for (int ky = -b + int(tid); ky <= b; ky += int(nthreads)) {
        for (int kx = -b; kx <= b; ++kx) {
          nz.clear();
          for (int s = 0; s < ns; ++s) {
            const cd pv = pupil(kx + src[s].sx * R, ky + src[s].sy * R, R, o.wavelength_nm, o.na, F);
            if (pv != cd(0.0, 0.0)) {
              a[s] = std::sqrt(src[s].w) * pv;
              nz.push_back(s);
            }
          }
          for (int s : nz)
            for (int t : nz) g[size_t(s) * ns + t] += std::conj(a[s]) * a[t];
        }
      }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nthreads; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &t : th) t.join();
    std::vector<cd> gram(size_t(ns) * ns, cd(0.0, 0.0));
    for (unsigned t = 0; t < nthreads; ++t)
      for (size_t i = 0; i < gram.size(); ++i) gram[i] += part[t][i];
    // Hermitian by construction; symmetrise the rounding.
    for (int s = 0; s < ns; ++s)
      for (int t = s; t < ns; ++t) {
        const cd m = 0.5 * (gram[size_t(s) * ns + t] + std::conj(gram[size_t(t) * ns + s]));
        gram[size_t(s) * ns + t] = m;
        gram[size_t(t) * ns + s] = std::conj(m);
      }
    std::vector<double> w;
    std::vector<cd> nu;
    hermitian_jacobi(ns, gram, w, nu);
    std::vector<int> order(ns);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return w[x] > w[y]; });
    for (int k = 0; k < o.K; ++k) {
      if (!(w[order[k]] > 0.0)) {
        set_error("litho_kernels_build: K=%d exceeds the numerical TCC rank", o.K);
        return LITHO_E_INVALID;
      }
      hb.lambda[size_t(p) * o.K + k] = w[order[k]];
    }
    if (o.K < ns) hb.gap[p] = (w[order[o.K - 1]] - w[order[o.K]]) / w[order[0]];
    // Phi_k = A nu_k / sqrt(lambda_k) on the band, in centred raster order.
    auto phi_work = [&](unsigned tid) {
      std::vector<cd> a(ns);
      for (int ky = -b + int(tid); ky <= b; ky += int(nthreads)) {
        for (int kx = -b; kx <= b; ++kx) {
          bool any = false;
          for (int s = 0; s < ns; ++s) {
            const cd pv = pupil(kx + src[s].sx * R, ky + src[s].sy * R, R, o.wavelength_nm, o.na, F);
            a[s] = std::sqrt(src[s].w) * pv;
            any = any || pv != cd(0.0, 0.0);
          }
          if (!any) continue;
          for (int k = 0; k < o.K; ++k) {
            const int col = order[k];
            cd acc(0.0, 0.0);
            for (int s = 0; s < ns; ++s) acc += a[s] * nu[size_t(s) * ns + col];
            hb.phi[((size_t(p) * o.K + k) * B + (ky + b)) * B + (kx + b)] =
                acc / std::sqrt(hb.lambda[size_t(p) * o.K + k]);
          }
        }
      }
    };
    th.clear();
    for (unsigned t = 1; t < nthreads; ++t) th.emplace_back(phi_work, t);
    phi_work(0);
    for (auto &t : th) t.join();
    // Cosmetic phase: the largest-magnitude sample (first in raster order
    // within a relative 1e-9) is made real and positive.
    for (int k = 0; k < o.K; ++k) {
      cd *ph = &hb.phi[(size_t(p) * o.K + k) * B * B];
      double mx = 0.0;
      for (int i = 0; i < B * B; ++i) mx = std::max(mx, std::abs(ph[i]));
      int idx = 0;
      for (int i = 0; i < B * B; ++i)
        if (std::abs(ph[i]) >= mx * (1.0 - 1e-9)) { idx = i; break; }
      const cd rot = std::conj(ph[idx]) / std::abs(ph[idx]);
      for (int i = 0; i < B * B; ++i) ph[i] *= rot;
    }
  }
  return LITHO_OK;
}

}  // namespace litho
