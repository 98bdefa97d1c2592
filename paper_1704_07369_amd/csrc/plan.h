// Host-side (FP64) precomputation of the spectral multipliers of one plan.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace efm {

struct HostTables {
  int N = 0, d = 0, M = 0, kind = 0;
  double L = 0, R = 0, gamma_exp = 0;
  int n0 = 0, n1 = 0, n2 = 0;   // cell dims: (N,N,N) in 3D, (1,N,N) in 2D
  int64_t n = 0;                // points per cell
  int n_radial = 1;             // radial nodes (non-separable kernels), else 1
  bool unfiltered = false;      // sigma = 1 (Fourier collocation, no entropic filter)
  int truncation = 0;           // EC_TRUNC_BOX or EC_TRUNC_BALL
  std::vector<double> bcos;     // angular factor b(x) = sum_i bcos[i] x^i (empty: 1)
  int terms = 0;                // M' products in the gain (M n_radial)
  int J = 0;                    // transforms after the forward one: M' + 1
  // gamma[(j * n + idx) * 2 + {0,1}], idx = (k0 * n2 + k2) * n1 + k1
  std::vector<double> gamma;
};

// Inputs of the per-mode table formulas (table_math.h), host arrays.
struct TableSpec {
  int N = 0, d = 0, M = 0, nrad = 1;
  bool radial = false;
  int64_t n = 0;
  int J = 0;
  double R = 0, kf = 0, scale = 0, qmax = 0;
  std::vector<double> ex, ey, ez, px, py, wt;   // directions, 2D partners, weights (M)
  std::vector<double> rho, om;                  // radial nodes (nrad)
  std::vector<double> cheb;                     // Chebyshev coefficients of Phi_j
  std::vector<int> cheb_off;                    // nrad + 1 offsets into cheb
  std::vector<double> sig1;                     // 1D filter (N)
};

// Validates the arguments, fills the metadata of T (not T.gamma) and the
// inputs S of the per-mode formulas.  Returns 0 or an EC_ERR_* code with a
// message in err.
int build_spec(int N, int d, double L, int kind, double gamma_exp, double R, int n_radial,
               int unfiltered, int truncation, int n_bcos, const double* bcos, int M,
               HostTables& T, TableSpec& S, std::string& err);

// build_spec, then every mode of T.gamma on the host threads.
int build_tables(int N, int d, double L, int kind, double gamma_exp, double R,
                 int n_radial, int unfiltered, int truncation, int n_bcos, const double* bcos,
                 int M, HostTables& out, std::string& err);

// build_spec, then the J entries of the listed modes only (flat indices in the
// table layout, idx = (k0 n2 + k2) n1 + k1): out[(j n_modes + i) * 2 + {0,1}].
int build_table_modes(int N, int d, double L, int kind, double gamma_exp, double R,
                      int n_radial, int unfiltered, int truncation, int n_bcos,
                      const double* bcos, int M, int64_t n_modes, const int64_t* idx,
                      HostTables& T, std::vector<double>& out, std::string& err);

// Modified Jackson filter (section 3.2.2, eq. JacksonFilter2) for the mode
// value k of an N-point axis.
double jackson(int N, int k);

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

bool supported_size(int N, int d);

// exp(2 pi i j / N), j < N, as interleaved (cos, sin) FP64 pairs
std::vector<double> twiddle_table(int N);

}  // namespace efm
