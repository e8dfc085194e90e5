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

double mu_effective(const fids_params& p) { return p.mu > 0 ? p.mu : 1.0 + p.alpha / 2; }

int validate(const fids_params& p) {
  const double mu = mu_effective(p);
  if (!(p.alpha > 0 && p.alpha < 2)) return FIDS_EINVAL;
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
  if (p.n > (int64_t(1) << 21) || p.M > (int64_t(1) << 24)) return FIDS_EINVAL;
  return FIDS_OK;
}

int64_t embed_length(int64_t n) {
  int64_t L = 4;
  while (L < 2 * n) L <<= 1;
  return L;
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
  t.n = p.n;
  t.M = p.M;
  t.L = embed_length(p.n);
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
  t.col = ifl_column(p.n, p.alpha, p.l, mu);
  // symbol of the L-circulant whose leading n x n block is A
  {
    std::vector<cplx> e(t.L, cplx(0, 0));
    for (int64_t j = 0; j < p.n; ++j) e[j] = t.col[j];
    for (int64_t j = 1; j < p.n; ++j) e[t.L - j] = t.col[j];
    host_fft(e, -1);
    t.ahat.resize(t.Nc + 1);
    for (int64_t k = 0; k <= t.Nc; ++k) t.ahat[k] = e[k].real();
  }
  t.lam = strang_eigs(t.col);
  t.chirp = make_chirp(p.n);
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
