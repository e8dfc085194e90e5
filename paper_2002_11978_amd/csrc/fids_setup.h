// Host-side set-up of the fast implicit difference scheme (FP64 C++).
//
// Everything here runs once per problem, before any time level: the graded
// mesh and level coefficients (Sec. 2.1), the sum-of-exponentials nodes and
// their recurrence factors (Lemma 2.2, eq. 2.9), the first column of the IFL
// matrix A (eq. 3.16x) and its circulant-embedding symbol, the eigenvalues of
// Strang's circulant s(A) (eq. 4.3) and the Bluestein chirp used on the device
// to invert the per-level circulant.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

#include "fids.h"

namespace fids {

using cplx = std::complex<double>;

struct SoeNodes {
  std::vector<double> s, w;
};

struct HostTables {
  int64_t n = 0, M = 0;
  int64_t L = 0;        // embedding length: smallest power of two >= 2n (>= 4)
  int64_t Nc = 0;       // L / 2, length of the packed complex FFT
  int nexp = 0;         // SOE node count
  double g = 0;         // 1 / Gamma(1 - gamma)
  std::vector<double> tau;     // [M+1], tau[m] = t_m - t_{m-1}, tau[0] = 0
  std::vector<double> xv;      // [M+1], (t_m / T)^gamma: the coordinate of the extrapolated initial guess
  std::vector<double> beta;    // [M+1], beta[m] = g a_m^{(m)} = tau_m^{-gamma}/Gamma(2-gamma)
  std::vector<double> theta;   // [(M+1) * nexp], recurrence input factor (m >= 2)
  std::vector<double> decay;   // [(M+1) * nexp], e^{-s_j tau_m}
  std::vector<double> gw;      // [nexp], g w_j
  std::vector<double> soec;    // [M+1], c_m = sum_j g w_j theta_{m,j}
  SoeNodes soe;
  std::vector<double> col;     // [n], first column of A
  std::vector<double> ahat;    // [Nc+1], real symbol of A's L-circulant embedding
  std::vector<double> lam;     // [n], eigenvalues of s(A)
  std::vector<cplx> chirp;     // [n], e^{i pi k^2 / n}
  std::vector<cplx> chirp_hat; // [L], FFT_L of the embedded conj(chirp)
};

// Parameter checks of fids_init_problem; returns FIDS_OK or FIDS_EINVAL.
int validate(const fids_params& p);

// Effective mu (0 selects 1 + alpha/2, or mu*(alpha) for dims = 2).
double mu_effective(const fids_params& p);

// Layout of the unknowns: dims = 1, n of them; dims = 2, node (i, j) of the
// n x n grid at i + S j with the row stride S (the smallest power of two
// >= 2n - 1), so that the block-Toeplitz matrix acts as one symmetric
// Toeplitz matrix of order S (n - 1) + n on the padded vector.
int64_t row_stride(const fids_params& p);    // S (0 for dims = 1)
int64_t toeplitz_len(const fids_params& p);  // order of that Toeplitz matrix
int64_t natural_len(const fids_params& p);   // n or n^2: length of the caller's arrays

int64_t embed_length(int64_t n);

// 2-D operator (dims = 2): the splitting exponent mu*(alpha), the
// coefficients a[p + n q] of the block-Toeplitz matrix, and the first column
// of the padded Toeplitz matrix with row stride S.
double ifl2d_mu(double alpha);
std::vector<double> ifl2d_coefficients(int64_t n, double alpha, double l, double mu);
std::vector<double> ifl2d_padded_column(int64_t n, double alpha, double l, double mu, int64_t S);

// The pieces, exposed for the introspection entry points.
std::vector<double> ifl_column(int64_t n, double alpha, double l, double mu);
std::vector<double> strang_eigs(const std::vector<double>& col);
int soe_build(double gamma, double delta, double T, double tol, SoeNodes& out);
double soe_max_rel_error(const SoeNodes& q, double gamma, double delta, double T, int npts);
std::vector<double> step_sizes(double T, int64_t M, double r);

// Direct-history weights of eq. (4.1): row m (offset (m-1) m / 2) holds the
// coefficients of u^0..u^{m-1} in b^m (g included).
std::vector<double> direct_history_weights(double T, int64_t M, double r, double gamma);

// Full set-up; returns FIDS_OK / FIDS_EINVAL.
int build_tables(const fids_params& p, HostTables& t);

// In-place radix-2 complex FFT (sign = -1 forward, +1 inverse, unnormalised).
void host_fft(std::vector<cplx>& a, int sign);

}  // namespace fids
