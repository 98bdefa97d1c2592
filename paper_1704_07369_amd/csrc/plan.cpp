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
#include "table_math.h"

#include <algorithm>
#include <cmath>
#include <thread>

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
  if (d == 3 && (N == 64 || N == 128)) return true;   // two-pass / lines schedule
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

// The separable kernels' closed forms psi_2, psi_3 and Phi (above) are
// evaluated per mode by tm_psi2, tm_psi3 and tm_phi3 (table_math.h).

// ---- non-separable kernels (variable hard spheres, 3D Maxwell) ----------------
// Bt(y, z) = (1/pi) (|y|^2 + |z|^2)^a, a = (gamma - 1)/2, does not factor in
// (|y|, |z|).  With Gauss-Legendre radii (rho_j, omega_j) on [0, R] for y the
// polar form separates into M n_radial products
//   psi_{t,j}(k) = 2 omega_j rho_j cos(rho_j s),                 s = pi k.e_t / L,
//   phi_{t,j}(k) = Phi_j(q) = 4 pi int_0^R (rho_j^2 + r^2)^a J_0(q r) r dr,
//                                                                q = pi |k_perp| / L,
// with the hard-sphere weights w_t (reduces to psi_3 Phi as n_radial grows
// when gamma = 1).  Phi_j is an entire function of q; it is sampled at the
// Chebyshev points of [0, q_max] (each sample by Gauss-Legendre panels in r,
// graded at r ~ rho_j where the weight changes) and evaluated by Clenshaw.
//
// Truncation.  The box |y| <= R, |z| <= R is the Carleman truncation of
// section 1.2.  The classical form (eq. classical_hatB) integrates over
// |g| <= R; with y = (g + |g| w)/2 and z = (g - |g| w)/2, which are orthogonal
// with |y|^2 + |z|^2 = |g|^2, that is the ball |y|^2 + |z|^2 <= R^2 of the
// same Carleman integrand: the disk of phi_{t,j} shrinks to radius
// sqrt(R^2 - rho_j^2).  The radii are then rho = R sin(theta) with
// Gauss-Legendre in theta on [0, pi/2] (omega = R cos(theta) w_theta), which
// removes the square-root endpoint of the disk radius at rho = R.
struct ChebFn {
  double qmax = 0.0;
  std::vector<double> c;   // Chebyshev coefficients on [0, qmax] (summed by tm_cheb)
};

// b(x) = sum_i bcos[i] x^i (Horner); b = 1 when nb == 0
static double bcos_eval(const double* bcos, int nb, double x) {
  if (nb <= 0) return 1.0;
  double acc = 0.0;
  for (int i = nb - 1; i >= 0; --i) acc = acc * x + bcos[i];
  return acc;
}

// With an angular factor b(cos theta) in B(g, w), cos theta = g.w / |g|
// = (|y|^2 - |z|^2) / (|y|^2 + |z|^2) in the Carleman variables
// (y = (g + |g| w)/2, z = (g - |g| w)/2, orthogonal): for |y| = rho_j and
// |z| = r it joins the radial weight of Phi_j.
static ChebFn hankel_cheb(double rho, double a, double R, double qmax, const double* bcos,
                          int nb) {
  const double PI_ = 3.14159265358979323846;
  // r panels [0, 2 rho], [2 rho, 8 rho], [8 rho, R] (clipped to R)
  std::vector<double> edges = {0.0};
  for (double e : {2.0 * rho, 8.0 * rho})
    if (e < R) edges.push_back(e);
  edges.push_back(R);
  std::vector<double> rr, ww;
  for (size_t p = 0; p + 1 < edges.size(); ++p) {
    const double lo = edges[p], hi = edges[p + 1];
    const int n = (int)std::ceil(0.6 * qmax * (hi - lo)) + 40;
    std::vector<double> x, w;
    gauss_legendre(n, x, w);
    for (int i = 0; i < n; ++i) {
      const double r = 0.5 * (hi - lo) * (x[i] + 1.0) + lo;
      rr.push_back(r);
      ww.push_back(0.5 * (hi - lo) * w[i] * 4.0 * PI_ * r * std::pow(rho * rho + r * r, a) *
                   bcos_eval(bcos, nb, (rho * rho - r * r) / (rho * rho + r * r)));
    }
  }
  const int D = (int)std::ceil(0.75 * qmax * R) + 64;
  std::vector<double> fv(D);
  for (int m = 0; m < D; ++m) {
    const double q = 0.5 * qmax * (1.0 + std::cos(PI_ * (m + 0.5) / D));
    double acc = 0.0;
    for (size_t i = 0; i < rr.size(); ++i) acc += ww[i] * std::cyl_bessel_j(0.0, q * rr[i]);
    fv[m] = acc;
  }
  ChebFn f;
  f.qmax = qmax;
  f.c.assign(D, 0.0);
  for (int k = 0; k < D; ++k) {
    double acc = 0.0;
    for (int m = 0; m < D; ++m) acc += fv[m] * std::cos(PI_ * k * (m + 0.5) / D);
    f.c[k] = (k == 0 ? 1.0 : 2.0) * acc / D;
  }
  return f;
}

static void hemisphere_split(int M, int& mm, int& mp) {
  mm = 1;
  for (int a = 1; a <= M; ++a)
    if (M % a == 0 && 2.0 * a * a <= M) mm = a;
  mp = M / mm;
}

int build_spec(int N, int d, double L, int kind, double gamma_exp, double R, int n_radial,
               int unfiltered, int truncation, int n_bcos, const double* bcos, int M,
               HostTables& T, TableSpec& S, std::string& err) {
  if (d != 2 && d != 3) { err = "d must be 2 or 3"; return EC_ERR_ARG; }
  if (N < 4 || M < 1 || !(L > 0.0)) { err = "need N >= 4, M >= 1, L > 0"; return EC_ERR_ARG; }
  if (!supported_size(N, d)) {
    err = "unsupported N (supported: 8, 12, 16, 24, 32, 3D also 64, 128; 2D also 64 .. 512)";
    return EC_ERR_UNSUPPORTED;
  }
  if (truncation != EC_TRUNC_BOX && truncation != EC_TRUNC_BALL) {
    err = "truncation must be EC_TRUNC_BOX or EC_TRUNC_BALL";
    return EC_ERR_ARG;
  }
  const bool ball = truncation == EC_TRUNC_BALL;
  // largest R of the box bound: T >= (3 sqrt 2 + 1) R / 4 (Carleman),
  // T >= (3 + sqrt 2) R / 4 (classical form)
  if (R <= 0.0) R = 4.0 * L / (ball ? 3.0 + std::sqrt(2.0) : 3.0 * std::sqrt(2.0) + 1.0);
  const bool separable = (d == 2 && kind == EC_KERNEL_MAXWELL) || (d == 3 && kind == EC_KERNEL_HARD_SPHERE);
  const bool radial = d == 3 && (kind == EC_KERNEL_MAXWELL || kind == EC_KERNEL_VHS);
  if (!separable && !radial) {
    err = "kernels: 2D Maxwell; 3D hard spheres, Maxwell and variable hard spheres";
    return EC_ERR_UNSUPPORTED;
  }
  if (ball && !radial) {
    err = "the ball truncation needs a 3D radial kernel (EC_KERNEL_MAXWELL or EC_KERNEL_VHS)";
    return EC_ERR_UNSUPPORTED;
  }
  if (n_bcos < 0 || n_bcos > EC_MAX_BCOS || (n_bcos > 0 && !bcos)) {
    err = "n_bcos must be 0 .. EC_MAX_BCOS";
    return EC_ERR_ARG;
  }
  if (n_bcos > 0 && !radial) {
    err = "an angular factor b(cos theta) needs a 3D radial kernel (EC_KERNEL_MAXWELL or EC_KERNEL_VHS)";
    return EC_ERR_UNSUPPORTED;
  }
  const double gexp = kind == EC_KERNEL_MAXWELL ? 0.0 : (kind == EC_KERNEL_HARD_SPHERE ? 1.0 : gamma_exp);
  if (radial && !(gexp > -1.0 && gexp <= 1.0)) { err = "VHS needs -1 < gamma <= 1"; return EC_ERR_ARG; }
  const int nrad = radial ? (n_radial > 0 ? n_radial : 8) : 1;

  T.N = N; T.d = d; T.M = M; T.kind = kind; T.L = L; T.R = R; T.gamma_exp = gamma_exp;
  T.n_radial = nrad;
  T.unfiltered = unfiltered != 0;
  T.truncation = truncation;
  T.bcos.assign(bcos, bcos + std::max(0, n_bcos));
  T.n0 = (d == 3) ? N : 1;
  T.n1 = N;
  T.n2 = N;
  T.n = (int64_t)T.n0 * T.n1 * T.n2;
  T.terms = M * nrad;
  T.J = T.terms + 1;
  T.gamma_exp = gexp;

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
  std::vector<double> sig1(N);
  // sigma = 1 gives the unfiltered Fourier collocation method (eq. FCM), the
  // comparison of the positivity study (section 4.2, Fig. 2); for even N the
  // modes with a component -N/2 stay zero (even N reduces to odd N - 1,
  // section 4.1), as in the filtered case
  for (int i = 0; i < N; ++i) {
    const int k = i < (N + 1) / 2 ? i : i - N;
    sig1[i] = unfiltered ? ((N % 2 == 0 && k == -N / 2) ? 0.0 : 1.0) : jackson(N, k);
  }
  auto mode = [N](int i) { return i < (N + 1) / 2 ? i : i - N; };

  // radial factors of the non-separable kernels
  std::vector<double> rho, om, rdisk;
  std::vector<ChebFn> hank;
  if (radial) {
    std::vector<double> x, w;
    gauss_legendre(nrad, x, w);
    rho.resize(nrad);
    om.resize(nrad);
    rdisk.resize(nrad);
    for (int j = 0; j < nrad; ++j) {
      if (ball) {
        const double th = 0.25 * PI * (x[j] + 1.0), wth = 0.25 * PI * w[j];
        rho[j] = R * std::sin(th);
        om[j] = R * std::cos(th) * wth;
        rdisk[j] = R * std::cos(th);
      } else {
        rho[j] = 0.5 * R * (x[j] + 1.0);
        om[j] = 0.5 * R * w[j];
        rdisk[j] = R;
      }
    }
    double kmax2 = 0.0;   // largest |k|^2 over the modes bounds |k_perp|
    for (int i = 0; i < N; ++i) kmax2 = std::max(kmax2, (double)mode(i) * mode(i));
    const double qmax = kf * std::sqrt(3.0 * kmax2) * 1.0001;
    for (int j = 0; j < nrad; ++j)
      hank.push_back(hankel_cheb(rho[j], 0.5 * (gexp - 1.0), rdisk[j], qmax, T.bcos.data(),
                                 (int)T.bcos.size()));
  }

  S.N = N; S.d = d; S.M = M; S.nrad = nrad; S.radial = radial;
  S.n = T.n; S.J = T.J;
  S.R = R; S.kf = kf; S.scale = scale; S.qmax = 0.0;
  S.ex = ex; S.ey = ey; S.ez = ez; S.px = px; S.py = py; S.wt = wt;
  S.rho = rho; S.om = om; S.sig1 = sig1;
  S.cheb.clear();
  S.cheb_off.assign(1, 0);
  for (auto& h : hank) {
    S.qmax = h.qmax;
    S.cheb.insert(S.cheb.end(), h.c.begin(), h.c.end());
    S.cheb_off.push_back((int)S.cheb.size());
  }
  return EC_OK;
}

namespace {
TableView make_view(const TableSpec& S) {
  TableView V;
  V.N = S.N; V.d = S.d; V.M = S.M; V.nrad = S.nrad; V.radial = S.radial ? 1 : 0;
  V.n = S.n; V.J = S.J; V.R = S.R; V.kf = S.kf; V.scale = S.scale; V.qmax = S.qmax;
  V.ex = S.ex.data(); V.ey = S.ey.data(); V.ez = S.ez.data();
  V.px = S.px.data(); V.py = S.py.data(); V.wt = S.wt.data();
  V.rho = S.rho.data(); V.om = S.om.data();
  V.cheb = S.cheb.data(); V.cheb_off = S.cheb_off.data(); V.sig1 = S.sig1.data();
  return V;
}
}  // namespace

int build_table_modes(int N, int d, double L, int kind, double gamma_exp, double R,
                      int n_radial, int unfiltered, int truncation, int n_bcos,
                      const double* bcos, int M, int64_t n_modes, const int64_t* idx,
                      HostTables& T, std::vector<double>& out, std::string& err) {
  TableSpec S;
  const int rc = build_spec(N, d, L, kind, gamma_exp, R, n_radial, unfiltered, truncation,
                            n_bcos, bcos, M, T, S, err);
  if (rc) return rc;
  for (int64_t i = 0; i < n_modes; ++i)
    if (idx[i] < 0 || idx[i] >= T.n) {
      err = "mode index out of range";
      return EC_ERR_ARG;
    }
  const TableView V = make_view(S);
  out.assign((size_t)2 * T.J * n_modes, 0.0);
  for (int64_t i = 0; i < n_modes; ++i) fill_mode_at(V, idx[i], n_modes, i, out.data(), nullptr);
  return EC_OK;
}

int build_tables(int N, int d, double L, int kind, double gamma_exp, double R,
                 int n_radial, int unfiltered, int truncation, int n_bcos, const double* bcos,
                 int M, HostTables& T, std::string& err) {
  TableSpec S;
  const int rc = build_spec(N, d, L, kind, gamma_exp, R, n_radial, unfiltered, truncation,
                            n_bcos, bcos, M, T, S, err);
  if (rc) return rc;
  const TableView V = make_view(S);
  T.gamma.assign((size_t)2 * T.J * T.n, 0.0);
  double* g = T.gamma.data();
  // modes in parallel on the host threads (each writes its own entries)
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int64_t n = T.n;
  if (n * (int64_t)T.J < 4000000 || nth == 1) {
    for (int64_t idx = 0; idx < n; ++idx) fill_mode(V, idx, g, nullptr);
  } else {
    std::vector<std::thread> pool;
    for (int w = 0; w < nth; ++w)
      pool.emplace_back([&, w]() {
        for (int64_t idx = w; idx < n; idx += nth) fill_mode(V, idx, g, nullptr);
      });
    for (auto& th : pool) th.join();
  }
  return EC_OK;
}

}  // namespace efm
