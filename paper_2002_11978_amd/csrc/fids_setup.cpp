// Host-side set-up of the fast implicit difference scheme; see fids_setup.h.
#include "fids_setup.h"

#include <algorithm>
#include <cmath>
#include <array>
#include <limits>
#include <map>
#include <mutex>
#include <thread>

namespace fids {

static const long double kPiL = 3.141592653589793238462643383279502884L;

double mu_effective(const fids_params& p) {
  if (p.mu > 0) return p.mu;
  return p.dims == 2 ? ifl2d_mu(p.alpha) : 1.0 + p.alpha / 2;
}

int64_t row_stride(const fids_params& p) {
  if (p.dims != 2) return 0;
  int64_t S = 1;
  while (S < 2 * p.n - 1) S <<= 1;
  return S;
}

int64_t toeplitz_len(const fids_params& p) {
  return p.dims == 2 ? row_stride(p) * (p.n - 1) + p.n : p.n;
}

int64_t natural_len(const fids_params& p) { return p.dims == 2 ? p.n * p.n : p.n; }

int validate(const fids_params& p) {
  if (!(p.alpha > 0 && p.alpha < 2)) return FIDS_EINVAL;
  if (p.dims != 1 && p.dims != 2) return FIDS_EINVAL;
  if (p.dims == 2 && (p.n < 1 || p.n > (int64_t(1) << 11))) return FIDS_EINVAL;
  // 2-D: psi has no limit at xi = 0 for mu = 2 (it depends on the direction)
  if (p.dims == 2 && p.mu != 0 && !(p.mu > p.alpha && p.mu < 2)) return FIDS_EINVAL;
  const double mu = mu_effective(p);
  if (!(p.gamma > 0 && p.gamma < 1)) return FIDS_EINVAL;
  if (!(mu > p.alpha && mu <= 2)) return FIDS_EINVAL;
  if (!(p.r >= 1) || p.n < 1 || p.M < 1) return FIDS_EINVAL;
  if (!(p.l > 0) || !(p.T > 0)) return FIDS_EINVAL;
  if (!(p.soe_tol > 0 && p.soe_tol < 1) || !(p.krylov_tol > 0 && p.krylov_tol < 1)) return FIDS_EINVAL;
  if (p.krylov_maxit < 1 || p.restart < 1 || p.restart > 32) return FIDS_EINVAL;
  if (p.solver != FIDS_BICGSTAB && p.solver != FIDS_FGMRES && p.solver != FIDS_PCG) return FIDS_EINVAL;
  if (p.precision != FIDS_FP64 && p.precision != FIDS_MIXED) return FIDS_EINVAL;
  if (p.precision == FIDS_MIXED && p.solver != FIDS_FGMRES) return FIDS_EINVAL;
  if (p.precond != FIDS_STRANG && p.precond != FIDS_NONE && p.precond != FIDS_STRANG_K) return FIDS_EINVAL;
  if (p.x0_mode < 0 || p.x0_mode > 3) return FIDS_EINVAL;
  if (p.wg_count < 0 || p.wg_count > 4096) return FIDS_EINVAL;
  if (p.soe_helpers < -1 || p.soe_helpers > 4096) return FIDS_EINVAL;
  if (p.checkpoint_every < 0) return FIDS_EINVAL;
  if (p.history != FIDS_HISTORY_SOE && p.history != FIDS_HISTORY_DIRECT) return FIDS_EINVAL;
  // the direct history keeps a triangular table of M (M + 1) / 2 weights
  if (p.history == FIDS_HISTORY_DIRECT && p.M > (int64_t(1) << 16)) return FIDS_EINVAL;
  if (toeplitz_len(p) > (int64_t(1) << 21) || p.M > (int64_t(1) << 24)) return FIDS_EINVAL;
  return FIDS_OK;
}

int64_t embed_length(int64_t n) {
  int64_t L = 4;
  while (L < 2 * n) L <<= 1;
  return L;
}


// ---------------------------------------------------------------- 2-D operator
// The 2-D form of eq. (3.16x) on the square (-l, l)^2 (dims = 2): the
// splitting of (2.11) with psi(xi) = (2u(x) - u(x+xi) - u(x-xi)) / |xi|^mu and
// omega = |xi|^{mu-2-alpha}; on every unit cell C of the lattice (xi = h eta)
// inside |eta|_inf <= N_p, psi is taken as the mean of its corner values and
// omega is integrated exactly (node m gets W_m = 1/4 sum of int_C omega over
// its cells), and beyond that square both neighbours lie outside the domain
// and the integral of 2 u(x) |xi|^{-2-alpha} is exact.

// Gauss-Legendre rule on [-1, 1]: Newton's method on P_k from the Chebyshev
// guesses, P_k and P_k' by the three-term recurrence.
static void gauss_legendre(int k, std::vector<double>& x, std::vector<double>& w) {
  x.assign(k, 0.0);
  w.assign(k, 0.0);
  for (int i = 0; i < k; ++i) {
    long double z = std::cos((long double)kPiL * (i + 0.75L) / (k + 0.5L));
    long double dp = 1;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int j = 2; j <= k; ++j) {
        const long double p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = k * (z * p1 - p0) / (z * z - 1);
      const long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    x[i] = double(z);
    w[i] = double(2 / ((1 - z * z) * dp * dp));
  }
}

namespace {
struct GL {
  std::vector<double> x8, w8, x12, w12, x40, w40;
  GL() {
    gauss_legendre(8, x8, w8);
    gauss_legendre(12, x12, w12);
    gauss_legendre(40, x40, w40);
  }
};
const GL& gl() {
  static const GL g;
  return g;
}
}  // namespace

// int over [a, b] x [c, d] (first quadrant, 0 <= a < b, 0 <= c < d) of
// (x^2 + y^2)^{beta/2}, -2 < beta < 0.  A cell with a corner at the origin is
// integrated in polar coordinates (radial part exact, angular part by
// 40-point Gauss-Legendre on each of the two triangles); cells within 4 of
// the origin are split into 8 x 8 sub-cells with 12 x 12 points, the others
// take 8 x 8 points (the singularity is then at least 4 cell widths away).
static double cell_integral(double a, double b, double c, double d, double beta) {
  const GL& g = gl();
  if (a == 0.0 && c == 0.0) {
    const double nu = beta + 2.0;
    const double th = std::atan2(d, b);
    long double s1 = 0, s2 = 0;
    for (int i = 0; i < 40; ++i) {
      const double t1 = 0.5 * th * (g.x40[i] + 1.0);
      s1 += g.w40[i] * std::pow(b / std::cos(t1), nu);
      const double t2 = th + 0.5 * (0.5 * kPiL - th) * (g.x40[i] + 1.0);
      s2 += g.w40[i] * std::pow(d / std::sin(t2), nu);
    }
    return double((0.5L * th * s1 + 0.5L * (0.5L * kPiL - th) * s2) / nu);
  }
  const bool near = std::max(a, c) < 4.0;
  const int sub = near ? 8 : 1;
  const std::vector<double>& x = near ? g.x12 : g.x8;
  const std::vector<double>& w = near ? g.w12 : g.w8;
  const int k = int(x.size());
  long double tot = 0;
  const double hx = (b - a) / sub, hy = (d - c) / sub;
  for (int i = 0; i < sub; ++i)
    for (int j = 0; j < sub; ++j) {
      const double x0 = a + hx * (i + 0.5), y0 = c + hy * (j + 0.5);
      long double acc = 0;
      for (int p = 0; p < k; ++p) {
        const double xx = x0 + 0.5 * hx * x[p];
        for (int q = 0; q < k; ++q) {
          const double yy = y0 + 0.5 * hy * x[q];
          acc += w[p] * w[q] * std::pow(xx * xx + yy * yy, 0.5 * beta);
        }
      }
      tot += acc * 0.25L * hx * hy;
    }
  return double(tot);
}

// First-quadrant cell integrals I[k1 * K + k2] over [k1, k1+1] x [k2, k2+1], k < K.
static std::vector<double> quadrant_cells(int64_t K, double beta) {
  std::vector<double> I(size_t(K * K));
  const int nth = int(std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency())));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back([&, t] {
      for (int64_t k1 = t; k1 < K; k1 += nth)
        for (int64_t k2 = 0; k2 < K; ++k2)
          I[size_t(k1 * K + k2)] = cell_integral(double(k1), double(k1 + 1), double(k2), double(k2 + 1), beta);
    });
  for (auto& th : pool) th.join();
  return I;
}

// Error of the rule over [-K, K]^2 for psi = |eta|^{2-mu} (psi(0) = 0):
// sum over cells of (mean of psi at the corners) int_C omega - int_C |eta|^{-alpha},
// for K = 32, 64, 128 (partial sums of one pass over [0, 128)^2, times 4).
static std::array<double, 3> lattice_partials(double mu, double alpha) {
  constexpr int64_t K = 128;
  const std::vector<double> Ib = quadrant_cells(K, mu - 2.0 - alpha);
  const std::vector<double> Ia = quadrant_cells(K, -alpha);
  auto psi = [&](int64_t i, int64_t j) {
    return (i == 0 && j == 0) ? 0.0 : std::pow(double(i * i + j * j), 0.5 * (2.0 - mu));
  };
  std::array<long double, 3> S{0, 0, 0};
  for (int64_t k1 = 0; k1 < K; ++k1)
    for (int64_t k2 = 0; k2 < K; ++k2) {
      const double avg = 0.25 * (psi(k1, k2) + psi(k1 + 1, k2) + psi(k1, k2 + 1) + psi(k1 + 1, k2 + 1));
      const long double e = (long double)avg * Ib[size_t(k1 * K + k2)] - Ia[size_t(k1 * K + k2)];
      const int64_t r = std::max(k1, k2);
      if (r < 32) S[0] += e;
      if (r < 64) S[1] += e;
      S[2] += e;
    }
  return {double(4 * S[0]), double(4 * S[1]), double(4 * S[2])};
}

// The summed error extrapolated in K (its tail is K^{-alpha} (a + b K^{-2}):
// per-cell errors fall like |eta|^{-2-alpha}).
static double lattice_error(double mu, double alpha) {
  const std::array<double, 3> S = lattice_partials(mu, alpha);
  const double q1 = std::pow(2.0, -alpha), q2 = std::pow(2.0, -alpha - 2.0);
  const double R0 = (S[1] - q1 * S[0]) / (1.0 - q1), R1 = (S[2] - q1 * S[1]) / (1.0 - q1);
  return (R1 - q2 * R0) / (1.0 - q2);
}

double ifl2d_mu(double alpha) {
  static std::mutex mu_lock;
  static std::map<double, double> cache;
  {
    std::lock_guard<std::mutex> g(mu_lock);
    auto it = cache.find(alpha);
    if (it != cache.end()) return it->second;
  }
  // the error decreases in mu from +inf (mu -> alpha) to a negative value at
  // mu = 2: Illinois (modified regula falsi) on [alpha + 1e-6, 2]
  double a = alpha + 1e-6, b = 2.0;
  double fa = lattice_error(a, alpha), fb = lattice_error(b, alpha);
  int side = 0;
  double m = 0.5 * (a + b);
  for (int it = 0; it < 100; ++it) {
    m = (a * fb - b * fa) / (fb - fa);
    if (!(m > a && m < b)) m = 0.5 * (a + b);
    const double fm = lattice_error(m, alpha);
    if ((fm > 0) == (fa > 0)) {
      a = m;
      fa = fm;
      if (side == -1) fb *= 0.5;
      side = -1;
    } else {
      b = m;
      fb = fm;
      if (side == 1) fa *= 0.5;
      side = 1;
    }
    if (b - a <= 4e-16 * b || fm == 0.0) break;
  }
  std::lock_guard<std::mutex> g(mu_lock);
  cache[alpha] = m;
  return m;
}

std::vector<double> ifl2d_coefficients(int64_t n, double alpha, double l, double mu) {
  const int64_t Np = n + 1;
  const double h = 2.0 * l / double(Np);
  const std::vector<double> Iq = quadrant_cells(Np, mu - 2.0 - alpha);
  // cell with lower-left corner k (in [-Np, Np)) mirrored into the first quadrant
  auto cell = [&](int64_t k1, int64_t k2) -> double {
    if (k1 < -Np || k1 >= Np || k2 < -Np || k2 >= Np) return 0.0;
    const int64_t s1 = k1 >= 0 ? k1 : -k1 - 1, s2 = k2 >= 0 ? k2 : -k2 - 1;
    return Iq[size_t(s1 * Np + s2)];
  };
  auto W = [&](int64_t m1, int64_t m2) {
    return 0.25 * (cell(m1, m2) + cell(m1 - 1, m2) + cell(m1, m2 - 1) + cell(m1 - 1, m2 - 1));
  };
  // D: every node of the square (by symmetry: the first quadrant with axis
  // nodes counted twice and the corner node once per mirror image)
  long double D = 0;
  for (int64_t m1 = 0; m1 <= Np; ++m1)
    for (int64_t m2 = 0; m2 <= Np; ++m2) {
      if (m1 == 0 && m2 == 0) continue;
      const double w = W(m1, m2) / std::pow(double(m1 * m1 + m2 * m2), 0.5 * mu);
      const int mult = (m1 == 0 || m2 == 0) ? 2 : 4;
      D += (long double)mult * w;
    }
  {
    const GL& g = gl();
    long double e = 0;
    for (int i = 0; i < 40; ++i) e += g.w40[i] * std::pow(std::cos(kPiL / 8 * (g.x40[i] + 1.0)), alpha);
    D += 8.0L / alpha * std::pow(double(Np), -alpha) * (kPiL / 8) * e;
  }
  const double a2 = alpha * std::pow(2.0, alpha - 1.0) * std::tgamma(1.0 + alpha / 2) /
                    (double(kPiL) * std::tgamma(1.0 - alpha / 2));
  const double scale = a2 / std::pow(h, alpha);
  std::vector<double> a(size_t(n * n));
  for (int64_t q = 0; q < n; ++q)
    for (int64_t p = 0; p < n; ++p)
      a[size_t(p + n * q)] =
          (p == 0 && q == 0) ? scale * double(D) : -scale * W(p, q) / std::pow(double(p * p + q * q), 0.5 * mu);
  return a;
}

std::vector<double> ifl2d_padded_column(int64_t n, double alpha, double l, double mu, int64_t S) {
  const std::vector<double> a = ifl2d_coefficients(n, alpha, l, mu);
  std::vector<double> col(size_t(S * (n - 1) + n), 0.0);
  // node (i, j) sits at i + S j; the entry coupling offsets (p, q) is col[p + S q]
  // (S >= 2n - 1 keeps the offsets of different q apart)
  for (int64_t q = 0; q < n; ++q)
    for (int64_t p = -(n - 1); p < n; ++p) {
      const int64_t d = p + S * q;
      if (d >= 0) col[size_t(d)] = a[size_t((p < 0 ? -p : p) + n * q)];
    }
  return col;
}

// ---------------------------------------------------------------- time mesh
// tau_m = t_m - t_{m-1} = T (m/M)^r (1 - (1 - 1/m)^r), written with
// expm1/log1p so that no digits cancel for large m (Sec. 2.1 graded mesh).
std::vector<double> step_sizes(double T, int64_t M, double r) {
  std::vector<double> tau(M + 1, 0.0);
  for (int64_t m = 1; m <= M; ++m) {
    const double tm = T * std::pow(double(m) / double(M), r);
    tau[m] = (m == 1) ? tm : -tm * std::expm1(r * std::log1p(-1.0 / double(m)));
  }
  return tau;
}

// ---------------------------------------------------------------- direct history
// Graded-L1 weights a_k^{(m)} = (1/tau_k) int_{t_{k-1}}^{t_k} (t_m - s)^{-gamma} ds
// = [D_{k-1}^{1-gamma} - D_k^{1-gamma}] / ((1 - gamma) tau_k), D_j = t_m - t_j, k = 1..m
// (Sec. 2.1).  D_j = t_m (1 - (j/m)^r) is formed with expm1/log1p, the
// difference of powers as -D_{k-1}^nu expm1(nu log1p(-tau_k / D_{k-1})), and the
// last interval exactly (D_m = 0: a_m = tau_m^{-gamma} / (1 - gamma)); there
// tau_m / D_{m-1} = 1 up to rounding, and the residue's small power (nu = 1 -
// gamma) would not be small.
static std::vector<double> l1_row(double T, int64_t M, double r, double gamma, int64_t m,
                                  const std::vector<double>& tau) {
  std::vector<double> a(size_t(m) + 1, 0.0);
  const double tm = T * std::pow(double(m) / double(M), r);
  const double nu = 1.0 - gamma;
  auto dist = [&](int64_t j) {           // t_m - t_j, 0 <= j < m
    return j == 0 ? tm : -tm * std::expm1(r * std::log1p(double(j - m) / double(m)));
  };
  for (int64_t k = 1; k < m; ++k) {
    // D_k / D_{k-1} = 1 - tau_k / D_{k-1}: the step itself, not a difference of distances
    const double d0 = dist(k - 1);
    a[size_t(k)] = -std::pow(d0, nu) * std::expm1(nu * std::log1p(-tau[k] / d0)) / (nu * tau[k]);
  }
  a[size_t(m)] = std::pow(tau[m], -gamma) / nu;
  return a;
}

std::vector<double> direct_history_weights(double T, int64_t M, double r, double gamma) {
  const std::vector<double> tau = step_sizes(T, M, r);
  const double g = 1.0 / std::tgamma(1.0 - gamma);
  std::vector<double> w(size_t(M) * size_t(M + 1) / 2, 0.0);
  // rows are independent: interleaved over host threads (row m costs O(m))
  const int nt = int(std::max<int64_t>(1, std::min<int64_t>(
      {int64_t(std::max(1u, std::thread::hardware_concurrency())), 16, M / 512 + 1})));
  auto rows = [&](int t) {
    for (int64_t m = M - t; m >= 1; m -= nt) {
      const std::vector<double> a = l1_row(T, M, r, gamma, m, tau);
      double* row = w.data() + size_t(m - 1) * size_t(m) / 2;
      // b^m = g [a_1 u^0 + sum_{k=1}^{m-1} (a_{k+1} - a_k) u^k] + f^m  (eq. 4.1)
      row[0] = g * a[1];
      for (int64_t k = 1; k <= m - 1; ++k) row[k] = g * (a[size_t(k + 1)] - a[size_t(k)]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(rows, t);
  rows(0);
  for (auto& th : pool) th.join();
  return w;
}

// ---------------------------------------------------------------- IFL column
// (d+1)^nu - (d-1)^nu = d^nu [expm1(nu log1p(1/d)) - expm1(nu log1p(-1/d))].
static long double diff_pow(double d, double nu) {
  const long double dn = std::pow((long double)d, (long double)nu);
  return dn * (std::expm1l(nu * std::log1pl(1.0L / d)) - std::expm1l(nu * std::log1pl(-1.0L / d)));
}

std::vector<double> ifl_column(int64_t n, double alpha, double l, double mu) {
  if (!(mu > 0)) mu = 1.0 + alpha / 2;
  const double nu = mu - alpha;
  const double kmu = (mu == 2.0) ? 2.0 : 1.0;
  const int64_t Np = n + 1;
  const double h = 2.0 * l / double(Np);
  const double c1 = std::pow(2.0, alpha - 1) * alpha * std::tgamma((alpha + 1) / 2) /
                    (std::sqrt(double(kPiL)) * std::tgamma(1 - alpha / 2));
  const long double Ch = (long double)c1 / ((long double)nu * std::pow((long double)h, (long double)alpha));
  // diagonal of (3.16x): summed from the smallest terms up
  long double sum = 0;
  for (int64_t ell = Np - 1; ell >= 2; --ell)
    sum += diff_pow(double(ell), nu) / std::pow((long double)ell, (long double)mu);
  const long double tail = std::pow((long double)Np, (long double)nu) *
                           (-std::expm1l(nu * std::log1pl(-1.0L / Np))) /
                           std::pow((long double)Np, (long double)mu);
  const long double c2 = std::pow(2.0L, (long double)nu) + kmu - 1;
  const long double diag = sum + tail + c2 + 2.0L * nu / (alpha * std::pow((long double)Np, (long double)alpha));
  std::vector<double> col(n);
  col[0] = double(Ch * diag);
  if (n > 1) col[1] = double(-Ch * c2 / 2);
  for (int64_t d = 2; d < n; ++d)
    col[d] = double(-Ch * diff_pow(double(d), nu) / (2.0L * std::pow((long double)d, (long double)mu)));
  return col;
}

// ---------------------------------------------------------------- host FFT
void host_fft(std::vector<cplx>& a, int sign) {
  const size_t N = a.size();
  for (size_t i = 1, j = 0; i < N; ++i) {
    size_t bit = N >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= N; len <<= 1) {
    const size_t half = len / 2;
    std::vector<cplx> w(half);
    for (size_t k = 0; k < half; ++k) {
      const long double ang = sign * 2.0L * kPiL * (long double)k / (long double)len;
      w[k] = cplx(double(std::cos(ang)), double(std::sin(ang)));
    }
    for (size_t i = 0; i < N; i += len)
      for (size_t k = 0; k < half; ++k) {
        const cplx u = a[i + k], v = a[i + k + half] * w[k];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

// e^{i pi (k^2 mod 2n) / n}, the Bluestein chirp (k^2 reduced exactly).
static std::vector<cplx> make_chirp(int64_t n) {
  std::vector<cplx> c(n);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t ph = int64_t((unsigned __int128)(k) * (unsigned __int128)(k) % (unsigned __int128)(2 * n));
    const long double ang = kPiL * (long double)ph / (long double)n;
    c[k] = cplx(double(std::cos(ang)), double(std::sin(ang)));
  }
  return c;
}

static std::vector<cplx> embed_conj_chirp_hat(const std::vector<cplx>& chirp, int64_t L) {
  const int64_t n = int64_t(chirp.size());
  std::vector<cplx> b(L, cplx(0, 0));
  for (int64_t k = 0; k < n; ++k) b[k] = std::conj(chirp[k]);
  for (int64_t k = 1; k < n; ++k) b[L - k] = std::conj(chirp[k]);
  host_fft(b, -1);
  return b;
}

// lam_k = sum_j c_S[j] e^{2 pi i jk/n} for the Strang column c_S[j] = col[min(j, n-j)]
// (eq. 4.3).  Bluestein: jk = (j^2 + k^2 - (j-k)^2)/2.
std::vector<double> strang_eigs(const std::vector<double>& col) {
  const int64_t n = int64_t(col.size());
  std::vector<double> lam(n);
  if (n == 1) { lam[0] = col[0]; return lam; }
  const int64_t L = embed_length(n);
  const auto chirp = make_chirp(n);
  const auto bh = embed_conj_chirp_hat(chirp, L);
  std::vector<cplx> a(L, cplx(0, 0));
  for (int64_t j = 0; j < n; ++j) a[j] = col[std::min(j, n - j)] * chirp[j];
  host_fft(a, -1);
  for (int64_t k = 0; k < L; ++k) a[k] *= bh[k];
  host_fft(a, +1);
  for (int64_t k = 0; k < n; ++k) lam[k] = (chirp[k] * a[k] / double(L)).real();
  return lam;
}

// ---------------------------------------------------------------- SOE
// Jacobi eigen-solver for a small dense symmetric matrix (row-major, p x p).
static void sym_eig(std::vector<double>& A, int p, std::vector<double>& evals, std::vector<double>& V) {
  V.assign(size_t(p) * p, 0.0);
  for (int i = 0; i < p; ++i) V[i * p + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        tot += A[i * p + j] * A[i * p + j];
        if (i != j) off += A[i * p + j] * A[i * p + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int a = 0; a < p; ++a)
      for (int b = a + 1; b < p; ++b) {
        const double apq = A[a * p + b];
        if (apq == 0.0) continue;
        const double theta = (A[b * p + b] - A[a * p + a]) / (2 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        const double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < p; ++k) {  // columns a, b
          const double ka = A[k * p + a], kb = A[k * p + b];
          A[k * p + a] = c * ka - s * kb;
          A[k * p + b] = s * ka + c * kb;
        }
        for (int k = 0; k < p; ++k) {  // rows a, b
          const double ak = A[a * p + k], bk = A[b * p + k];
          A[a * p + k] = c * ak - s * bk;
          A[b * p + k] = s * ak + c * bk;
        }
        for (int k = 0; k < p; ++k) {
          const double ka = V[k * p + a], kb = V[k * p + b];
          V[k * p + a] = c * ka - s * kb;
          V[k * p + b] = s * ka + c * kb;
        }
      }
  }
  evals.resize(p);
  for (int i = 0; i < p; ++i) evals[i] = A[i * p + i];
}

// p-point Gauss rule of the discrete measure sum_i w_i delta(x - x_i):
// Lanczos on diag(x) from sqrt(w) (full re-orthogonalisation) gives the Jacobi
// matrix; its eigenvalues are the nodes and mu0 * (first eigenvector entry)^2
// the weights (Golub-Welsch).
static void gauss_of_discrete(const std::vector<double>& x, const std::vector<double>& w, int p,
                              std::vector<double>& nodes, std::vector<double>& weights) {
  const int K = int(x.size());
  long double mu0 = 0;
  for (double v : w) mu0 += v;
  std::vector<std::vector<double>> Q;
  std::vector<double> q(K), alpha, beta;
  for (int i = 0; i < K; ++i) q[i] = std::sqrt(w[i] / double(mu0));
  Q.push_back(q);
  for (int k = 0; k < p; ++k) {
    const auto& v = Q.back();
    std::vector<double> z(K);
    for (int i = 0; i < K; ++i) z[i] = x[i] * v[i];
    long double a = 0;
    for (int i = 0; i < K; ++i) a += (long double)v[i] * z[i];
    alpha.push_back(double(a));
    if (k == p - 1) break;
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& u : Q) {
        long double d = 0;
        for (int i = 0; i < K; ++i) d += (long double)u[i] * z[i];
        for (int i = 0; i < K; ++i) z[i] -= double(d) * u[i];
      }
    long double nb = 0;
    for (int i = 0; i < K; ++i) nb += (long double)z[i] * z[i];
    const double b = double(std::sqrt(nb));
    if (!(b > 0)) { p = k + 1; break; }
    beta.push_back(b);
    for (int i = 0; i < K; ++i) z[i] /= b;
    Q.push_back(z);
  }
  p = int(alpha.size());
  std::vector<double> J(size_t(p) * p, 0.0), ev, V;
  for (int i = 0; i < p; ++i) {
    J[i * p + i] = alpha[i];
    if (i + 1 < p) J[i * p + i + 1] = J[(i + 1) * p + i] = beta[i];
  }
  sym_eig(J, p, ev, V);
  nodes.resize(p);
  weights.resize(p);
  for (int i = 0; i < p; ++i) {
    nodes[i] = std::fabs(ev[i]);
    weights[i] = double(mu0) * V[0 * p + i] * V[0 * p + i];
  }
}

double soe_max_rel_error(const SoeNodes& q, double gamma, double delta, double T, int npts) {
  double worst = 0;
  const double a = std::log(delta), b = std::log(T);
  for (int i = 0; i < npts; ++i) {
    const double t = (npts == 1) ? T : std::exp(a + (b - a) * double(i) / double(npts - 1));
    long double sum = 0;
    for (size_t j = 0; j < q.s.size(); ++j) sum += (long double)q.w[j] * std::exp(-(long double)q.s[j] * t);
    const double e = double(std::fabs(sum * std::pow((long double)t, (long double)gamma) - 1.0L));
    worst = std::max(worst, e);
  }
  return worst;
}

// Sum-of-exponentials for t^{-gamma} on [delta, T] with relative error <= tol
// (Lemma 2.2 gives existence only; this construction is ours):
//   t^{-gamma} = (1/Gamma(gamma)) int_R exp(gamma y - t e^y) dy,
// trapezoid rule in y (the integrand is analytic in |Im y| < pi/2, so the
// error decays like exp(-2 pi d / h)), truncated where the tails fall below
// tol/10; the slow modes s_j < 1/T are then merged into a short Gauss rule of
// their discrete measure (e^{-s t} is nearly a low-degree polynomial in s
// there).  The result is checked on a dense logarithmic grid and the step is
// refined until it passes.
static int soe_build_uncached(double gamma, double delta, double T, double tol, SoeNodes& out) {
  if (!(delta > 0) || !(T >= delta) || !(tol > 0) || !(gamma > 0 && gamma < 1)) return FIDS_EINVAL;
  const double eta = 0.1, d = 0.5 * double(kPiL) - eta;
  double h = 2 * double(kPiL) * d / std::log(8.0 * std::pow(std::sin(eta), -gamma) / tol);
  const double gg = std::tgamma(gamma);
  const double ymax = std::log((std::log(10.0 / tol) + 4.0) / delta);
  const double ymin = std::log(tol * std::tgamma(1 + gamma) / 10.0) / gamma - std::log(T);
  int p_need = 1;
  {
    long double f = 1;  // 1/(2p)!
    for (p_need = 1; p_need < 14; ++p_need) {
      f /= (long double)(2 * p_need - 1) * (2 * p_need);
      if (f <= tol / 100) break;
    }
  }
  for (int attempt = 0; attempt < 12; ++attempt, h *= 0.85) {
    SoeNodes q;
    std::vector<double> xs, ws;
    for (int j = 0;; ++j) {
      const double y = ymax - j * h;
      if (y < ymin) break;
      const double s = std::exp(y), w = h * std::exp(gamma * y) / gg;
      if (s * T < 1.0) { xs.push_back(s); ws.push_back(w); }
      else { q.s.push_back(s); q.w.push_back(w); }
    }
    if (int(xs.size()) > p_need) {
      std::vector<double> gn, gw;
      gauss_of_discrete(xs, ws, p_need, gn, gw);
      for (size_t i = 0; i < gn.size(); ++i) { q.s.push_back(gn[i]); q.w.push_back(gw[i]); }
    } else {
      for (size_t i = 0; i < xs.size(); ++i) { q.s.push_back(xs[i]); q.w.push_back(ws[i]); }
    }
    if (soe_max_rel_error(q, gamma, delta, T, 3000) <= tol) { out = q; return FIDS_OK; }
  }
  return FIDS_EINVAL;
}

// ---------------------------------------------------------------- all tables
int build_tables(const fids_params& p, HostTables& t) {
  if (validate(p) != FIDS_OK) return FIDS_EINVAL;
  const double mu = mu_effective(p);
  const int64_t nt = toeplitz_len(p);
  t.n = nt;
  t.M = p.M;
  t.L = embed_length(nt);
  t.Nc = t.L / 2;
  t.g = 1.0 / std::tgamma(1.0 - p.gamma);
  t.tau = step_sizes(p.T, p.M, p.r);
  // The solution of (1.1) starts as u^0 + c t^gamma + ... (the weak
  // singularity the graded mesh resolves), which is linear in t^gamma: the
  // extrapolated initial guess is a polynomial in this coordinate.
  t.xv.assign(size_t(p.M) + 1, 0.0);
  for (int64_t m = 1; m <= p.M; ++m) t.xv[size_t(m)] = std::pow(double(m) / double(p.M), p.r * p.gamma);
  t.beta.assign(p.M + 1, 0.0);
  const double g2 = std::tgamma(2.0 - p.gamma);
  for (int64_t m = 1; m <= p.M; ++m) t.beta[m] = std::pow(t.tau[m], -p.gamma) / g2;
  // SOE on [tau_1, T]: the kernel argument t_m - s over every interval k < m
  // lies in [tau_m, t_m] with tau_m >= tau_1 (r >= 1).
  if (soe_build(p.gamma, t.tau[1], p.T, p.soe_tol, t.soe) != FIDS_OK) return FIDS_EINVAL;
  t.nexp = int(t.soe.s.size());
  t.gw.resize(t.nexp);
  for (int j = 0; j < t.nexp; ++j) t.gw[j] = t.g * t.soe.w[j];
  // F_j^{(m)} = sum_{k<m} c_{jk}^{(m)} (u^k - u^{k-1}),
  // c_{jk}^{(m)} = (1/tau_k) int_{t_{k-1}}^{t_k} e^{-s_j (t_m - s)} ds, obeys
  // F^{(m)} = e^{-s tau_m} F^{(m-1)} + theta_m (u^{m-1} - u^{m-2}) with
  // theta_{m,j} = e^{-s_j tau_m} (1 - e^{-s_j tau_{m-1}}) / (s_j tau_{m-1}).
  t.theta.assign(size_t(p.M + 1) * t.nexp, 0.0);
  t.decay.assign(size_t(p.M + 1) * t.nexp, 0.0);
  for (int64_t m = 1; m <= p.M; ++m)
    for (int j = 0; j < t.nexp; ++j) {
      const double s = t.soe.s[j];
      const double e = std::exp(-s * t.tau[m]);
      t.decay[size_t(m) * t.nexp + j] = e;
      if (m >= 2) {
        const double x = s * t.tau[m - 1];
        t.theta[size_t(m) * t.nexp + j] = e * (x > 0 ? -std::expm1(-x) / x : 1.0);
      }
    }
  t.soec.assign(p.M + 1, 0.0);
  for (int64_t m = 2; m <= p.M; ++m) {
    long double c = 0;
    for (int j = 0; j < t.nexp; ++j) c += (long double)t.gw[j] * t.theta[size_t(m) * t.nexp + j];
    t.soec[m] = double(c);
  }
  t.col = p.dims == 2 ? ifl2d_padded_column(p.n, p.alpha, p.l, mu, row_stride(p)) : ifl_column(p.n, p.alpha, p.l, mu);
  // symbol of the L-circulant whose leading n x n block is A
  {
    std::vector<cplx> e(t.L, cplx(0, 0));
    for (int64_t j = 0; j < nt; ++j) e[j] = t.col[j];
    for (int64_t j = 1; j < nt; ++j) e[t.L - j] = t.col[j];
    host_fft(e, -1);
    t.ahat.resize(t.Nc + 1);
    for (int64_t k = 0; k <= t.Nc; ++k) t.ahat[k] = e[k].real();
  }
  t.lam = strang_eigs(t.col);
  t.chirp = make_chirp(nt);
  t.chirp_hat = embed_conj_chirp_hat(t.chirp, t.L);
  return FIDS_OK;
}

// The node construction (quadrature, Lanczos, verification on a dense grid)
// takes tens of milliseconds; batches and repeated set-ups ask for the same
// (gamma, delta, T, tol) several times, so results are memoised.
int soe_build(double gamma, double delta, double T, double tol, SoeNodes& out) {
  static std::mutex mu;
  static std::map<std::array<double, 4>, SoeNodes> memo;
  const std::array<double, 4> key{gamma, delta, T, tol};
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = memo.find(key);
    if (it != memo.end()) {
      out = it->second;
      return FIDS_OK;
    }
  }
  const int st = soe_build_uncached(gamma, delta, T, tol, out);
  if (st == FIDS_OK) {
    std::lock_guard<std::mutex> g(mu);
    if (memo.size() > 4096) memo.clear();
    memo[key] = out;
  }
  return st;
}

}  // namespace fids
