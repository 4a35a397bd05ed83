// Host FP64 construction of the SOCS kernel bank (Eqs. 2-3).
#pragma once

#include <complex>
#include <vector>

#include "litho.h"

namespace litho {

using cd = std::complex<double>;

struct SourcePoint {
  double sx, sy;  // sigma, units of NA
  double w;       // normalised weight
};

// Eigenpairs of one or more focus planes on the centred (2b+1)^2 band.
struct HostBank {
  int n = 0, b = 0, B = 0, K = 0, n_focus = 0, n_source = 0;
  double R = 0.0;                 // pupil radius in frequency-index units
  double dose = 1.0;
  std::vector<double> lambda;     // [n_focus][K], descending per plane
  std::vector<cd> phi;            // [n_focus][K][B][B], unit 2-norm, [ky + b][kx + b]
  std::vector<double> gap;        // [n_focus] (lambda_K - lambda_{K+1}) / lambda_1, or 1 if K = rank
};

std::vector<SourcePoint> sample_source(const litho_optics_t &o);

// Hermitian eigensolver (cyclic complex Jacobi).  a: n x n row-major, destroyed.
// On return w holds the eigenvalues (ascending order not guaranteed) and v the
// eigenvectors as columns (row-major n x n).
void hermitian_jacobi(int n, std::vector<cd> &a, std::vector<double> &w, std::vector<cd> &v);

int build_host_bank(const litho_optics_t &o, HostBank &out);

}  // namespace litho
