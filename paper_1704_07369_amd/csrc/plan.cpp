// Host FP64 precomputation of the spectral multipliers (closed forms).
//
// Gain (section 3.3: Q+ = sum_{l,m} B^s(l,m) Fh_l Fh_m E_{l+m}) with the
// low-rank kernel B_fast(l,m) = sum_t w_t psi_t(l) phi_t(m) (section 4.1,
// eq. fastAlg) becomes sum_t w_t a_t(r) b_t(r) with
//   a_t = sum_k sigma_k psi_t(k) Fh_k E_k,   b_t = sum_k sigma_k phi_t(k) Fh_k E_k.
// The loss is F_r l_r with l = sum_k sigma_k^2 B_fast(k,k) Fh_k E_k (the loss
// identity of section 3.1.2 with the filtered kernel).  The kernels compute
// c_t = IDFT[(alpha_t + i beta_t) DFT F] with unnormalised transforms, so
// Re c_t Im c_t = w_t a_t b_t when
//   alpha_t = N^-d w_t sigma psi_t,  beta_t = N^-d sigma phi_t,
// and the last entry D = N^-d sigma^2 sum_t w_t psi_t phi_t gives l = Re c.
//
// Kernel-mode factors (polar form of eq. def_hatB, section 4.1, with
// s = pi k.e / L and, in 3D, q = pi |k_perp| / L the part of the wave vector
// orthogonal to e):
//   2D, Bt = 1/pi:  psi(s) = int_{-R}^{R} cos(rho s) d rho = 2 sin(R s)/s,
//                   B_fast = (1/pi) sum_{2M nodes} (pi/2M) psi(e_t) psi(e_t+pi/2)
//                   = (1/M) sum_{t<M} [psi(e_t) psi(e_t^perp) + (swap)] / 2;
//   3D, Bt = 1/pi:  psi_3(s) = int_{-R}^{R} |rho| cos(rho s) d rho
//                            = 2 R^2 [sinc(Rs) - sinc^2(Rs/2)/2],
//                   Phi(q) = 2 int_{disk radius R, normal e} cos(k.x) dx
//                          = 4 pi R J_1(R q)/q,
//                   B_fast = (Bt/2) sum_t w_t psi_3 Phi over a hemisphere rule.
#include "plan.h"

#include <cmath>

#include "../../include/ec.h"

namespace efm {

static const double PI = 3.14159265358979323846;

double jackson(int N, int k) {
  // n of eq. JacksonFilter2: (N-1)/2 for odd N; N/2 for even N (the reading
  // that reproduces the paper's Table 2; it gives sigma(-N/2) = 0).
  const int n = (N % 2) ? (N - 1) / 2 : N / 2;
  const int b = k < 0 ? -k : k;
  if (b >= n) return 0.0;
  const double a = PI / (n + 1);
  return ((n + 1 - b) * std::cos(a * b) + std::sin(a * b) / std::tan(a)) / (n + 1);
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

bool supported_size(int N, int d) {
  if (N == 8 || N == 12 || N == 16 || N == 24 || N == 32) return true;
  return d == 2 && (N == 64 || N == 128 || N == 256 || N == 512);   // LDS line transforms
}

std::vector<double> twiddle_table(int N) {
  // exp(2 pi i j / N) as (cos, sin) pairs: the quarter turns are exact and the
  // remainder r < N/4 is evaluated in long double, then rotated
  static const long double PIL = 3.141592653589793238462643383279502884L;
  std::vector<double> t(2 * (size_t)N);
  for (int j = 0; j < N; ++j) {
    const int q = (4 * j) / N;
    const int rr = 4 * j - q * N;                     // angle 2 pi rr / (4N), rr < N
    const long double a = 2.0L * PIL * (long double)rr / (4.0L * N);
    const double c = rr == 0 ? 1.0 : (double)cosl(a), sn = rr == 0 ? 0.0 : (double)sinl(a);
    double x = c, y = sn;
    for (int k = 0; k < q; ++k) { const double u = x; x = -y; y = u; }   // times i
    t[2 * j] = x;
    t[2 * j + 1] = y;
  }
  return t;
}

static double sinc(double x) {
  if (std::fabs(x) < 1e-4) {
    const double x2 = x * x;
    return 1.0 - x2 / 6.0 + x2 * x2 / 120.0;
  }
  return std::sin(x) / x;
}

static double psi2(double s, double R) { return 2.0 * R * sinc(R * s); }

static double psi3(double s, double R) {
  const double x = R * s;
  const double h = sinc(0.5 * x);
  return 2.0 * R * R * (sinc(x) - 0.5 * h * h);
}

static double phi3(double q, double R) {
  const double x = R * q;
  double j1x;  // J_1(x)/x
  if (x < 1e-4) j1x = 0.5 - x * x / 16.0;
  else j1x = std::cyl_bessel_j(1.0, x) / x;
  return 4.0 * PI * R * R * j1x;
}

static void hemisphere_split(int M, int& mm, int& mp) {
  mm = 1;
  for (int a = 1; a <= M; ++a)
    if (M % a == 0 && 2.0 * a * a <= M) mm = a;
  mp = M / mm;
}

int build_tables(int N, int d, double L, int kind, double gamma_exp, double R,
                 int M, HostTables& T, std::string& err) {
  if (d != 2 && d != 3) { err = "d must be 2 or 3"; return EC_ERR_ARG; }
  if (N < 4 || M < 1 || !(L > 0.0)) { err = "need N >= 4, M >= 1, L > 0"; return EC_ERR_ARG; }
  if (!supported_size(N, d)) {
    err = "unsupported N (supported: 8, 12, 16, 24, 32; in 2D also 64, 128, 256, 512)";
    return EC_ERR_UNSUPPORTED;
  }
  if (R <= 0.0) R = 4.0 * L / (3.0 * std::sqrt(2.0) + 1.0);
  const bool separable = (d == 2 && kind == EC_KERNEL_MAXWELL) || (d == 3 && kind == EC_KERNEL_HARD_SPHERE);
  if (!separable) { err = "only 2D Maxwell and 3D hard-sphere kernels are implemented"; return EC_ERR_UNSUPPORTED; }

  T.N = N; T.d = d; T.M = M; T.kind = kind; T.L = L; T.R = R; T.gamma_exp = gamma_exp;
  T.n0 = (d == 3) ? N : 1;
  T.n1 = N;
  T.n2 = N;
  T.n = (int64_t)T.n0 * T.n1 * T.n2;
  T.terms = M;
  T.J = M + 1;

  // directions: e[t], partner (2D) and weights w[t] (Bt folded in)
  std::vector<double> ex(M), ey(M), ez(M, 0.0), px(M, 0.0), py(M, 0.0), wt(M);
  if (d == 2) {
    for (int t = 0; t < M; ++t) {
      const double th = t * PI / (2.0 * M);
      ex[t] = std::cos(th); ey[t] = std::sin(th);
      px[t] = -ey[t]; py[t] = ex[t];
      wt[t] = 1.0 / M;     // 2 * Bt * pi/(2M) with Bt = 1/pi
    }
  } else {
    int mm, mp;
    hemisphere_split(M, mm, mp);
    std::vector<double> gx, gw;
    gauss_legendre(2 * mm, gx, gw);
    int t = 0;
    for (int i = 0; i < 2 * mm; ++i) {
      if (!(gx[i] > 0.0)) continue;
      const double mu = gx[i], st = std::sqrt(std::max(0.0, 1.0 - mu * mu));
      for (int j = 0; j < mp; ++j) {
        const double ph = 2.0 * PI * j / mp;
        ex[t] = st * std::cos(ph); ey[t] = st * std::sin(ph); ez[t] = mu;
        // (Bt/2) * w_GL * 2 pi / M_phi with Bt = 1/pi
        wt[t] = gw[i] / mp;
        ++t;
      }
    }
  }

  const double scale = 1.0 / (double)T.n;   // N^-d
  const double kf = PI / L;
  T.gamma.assign((size_t)2 * T.J * T.n, 0.0);
  std::vector<double> sig1(N);
  for (int i = 0; i < N; ++i) sig1[i] = jackson(N, i < (N + 1) / 2 ? i : i - N);
  auto mode = [N](int i) { return i < (N + 1) / 2 ? i : i - N; };

  for (int i0 = 0; i0 < T.n0; ++i0)
    for (int i2 = 0; i2 < T.n2; ++i2)
      for (int i1 = 0; i1 < T.n1; ++i1) {
        const int64_t idx = ((int64_t)i0 * T.n2 + i2) * T.n1 + i1;
        double kx, ky, kz, sig;
        if (d == 3) {
          kx = mode(i0); ky = mode(i1); kz = mode(i2);
          sig = sig1[i0] * sig1[i1] * sig1[i2];
        } else {
          kx = mode(i1); ky = mode(i2); kz = 0.0;
          sig = sig1[i1] * sig1[i2];
        }
        const double k2 = kx * kx + ky * ky + kz * kz;
        double diag = 0.0;
        for (int t = 0; t < M; ++t) {
          const double kd = kx * ex[t] + ky * ey[t] + kz * ez[t];
          double ps, ph;
          if (d == 2) {
            ps = psi2(kf * kd, R);
            ph = psi2(kf * (kx * px[t] + ky * py[t]), R);
          } else {
            ps = psi3(kf * kd, R);
            ph = phi3(kf * std::sqrt(std::max(0.0, k2 - kd * kd)), R);
          }
          T.gamma[((size_t)t * T.n + idx) * 2 + 0] = scale * wt[t] * sig * ps;
          T.gamma[((size_t)t * T.n + idx) * 2 + 1] = scale * sig * ph;
          diag += wt[t] * ps * ph;
        }
        T.gamma[((size_t)M * T.n + idx) * 2 + 0] = scale * sig * sig * diag;
        T.gamma[((size_t)M * T.n + idx) * 2 + 1] = 0.0;
      }
  return EC_OK;
}

}  // namespace efm
