// Device-side descriptors shared by the HIP kernels and the host launcher.
//
// Layout of every internal n-vector ("tile-major"): the real index i of the
// length-L zero-padded vector is packed in pairs z[k] = (x[2k], x[2k+1]),
// k = N2*n1 + n2 (four-step FFT split Nc = L/2 = N1*N2), and stored at
//     tile*(2*CT*N1) + 2*(n1*CT + c) + e,   n2 = tile*CT + c,  i = 2k + e,
// so that each column tile of the first FFT pass owns one contiguous block.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "fids.h"

namespace fids {

constexpr int kThreads = 512;     // threads per workgroup in every kernel
constexpr int kMaxFFT = 4096;     // longest per-workgroup FFT (complex points)
constexpr int kMaxRestart = 32;
constexpr int kRing = 4;          // states kept: u^m lives in u[m % kRing] (and A u^m in AU)
constexpr int kSoeBatch = 8;      // SOE nodes whose history values are loaded together
constexpr int kLoadBatch = 4;     // column-pass loads per thread issued together
constexpr int kPcgChecks = 3;     // true-residual checks of a PCG level
constexpr double kPcgSlack = 4.0; // PCG accepts a true residual up to this many tolerances
constexpr int kVecBatch = 2;      // solver element items per thread whose loads are issued together
constexpr int kMaxHelpers = 1024; // helper workgroups (one release-flag line each)
constexpr int kDirectChunks = 128; // direct history: most state chunks per element block
constexpr int kBarSlotWords = 32;  // group barrier: one 128-byte arrival slot per workgroup
constexpr int kMaxGroup = 256;     // workgroups of one problem (one co-resident workgroup per CU)
constexpr size_t kBarBytes = size_t(kMaxGroup) * kBarSlotWords * sizeof(unsigned);

// Direct history with helpers: state chunks for nh helpers over problems of n
// unknowns (element blocks of kThreads value pairs).
inline int direct_chunks(int64_t n, int nh) {
  const int64_t blocks = ((n + 1) / 2 + kThreads - 1) / kThreads;
  const int64_t c = nh / blocks;
  return int(c < 1 ? 1 : (c > kDirectChunks ? kDirectChunks : c));
}

// Partial-sum slots (one value per column tile each).
enum Slot {
  SL_BB = 0, SL_RV, SL_SS, SL_RS, SL_TS, SL_TT, SL_RT, SL_RR, SL_KB,
  SL_XX = 9,                      // ||x||^2 of the iterate whose true residual is formed
  SL_GM = 10,                     // FGMRES: kMaxRestart + 2 consecutive slots
  SL_COUNT = SL_GM + kMaxRestart + 2
};

// Two-pass FFT plan for Nc = N1 * N2 complex points.
struct Plan {
  int Nc, N1, N2, log1, log2, CT;
  int ntiles;        // N2 / CT column tiles
  int nunits;        // N1 / 2 row-pair units
  int RU;            // row-pair units per row group
  int nrg;           // nunits / RU row groups
  int rootmul;       // W_Nc = W_root^rootmul (2 for the real-packed plan, 1 complex)
  int twshift;       // split of the root table: j = (jh << twshift) + jl
  int twmask;
  int twres;         // twiddle tables copied to LDS: 0 all, 1 W_N1 and W_N2 only (the root
                     // tables stay in global memory), 2 none (long transforms whose tables
                     // and tiles do not fit the LDS together)
  int twn;           // twiddle values that copy holds (set with twres)
  const double2* tw1;  const float2* tw1f;   // W_{N1}^j, j < N1 (e^{-2 pi i j/N1})
  const double2* tw2;  const float2* tw2f;   // W_{N2}^j
  const double2* twlo; const float2* twlof;  // W_root^{jl}
  const double2* twhi; const float2* twhif;  // W_root^{jh << twshift}
};

// Twiddle values a launch copies to LDS (see Plan::twres).
inline int lds_twiddles(const Plan& pl, int L) {
  if (pl.twres >= 2) return 0;
  if (pl.twres == 1) return pl.N1 + pl.N2;
  return pl.N1 + pl.N2 + (pl.twmask + 1) + (L >> pl.twshift);
}

// Per-problem descriptor, in device memory.
struct Prob {
  int n, M, nexp;               // n: order of the Toeplitz matrix the solver applies (padded length in 2-D)
  int nn;                       // length of the caller's arrays per level: n (1-D) or nx^2 (2-D)
  int nx, sx, lsx;              // 2-D: nodes per axis, row stride S = 2^lsx (node (i, j) at i + S j); 1-D: 0
  int vmask, vlim;              // element i is an unknown iff i < n and (i & vmask) < vlim (1-D: 0, 1)
  int solver, precision, precond, kappa_td, x0_mode, maxit, restart, store_states;
  double tol;
  int g0, ng;                   // workgroups [g0, g0 + ng) cooperate on this problem
  int slot_first;               // first descriptor of the slot of problems these workgroups run in turn
  int L, vlen;                  // embedding length and tile-major vector length (= L)
  Plan pl;                      // real-packed plan, Nc = L/2
  // set-up tables
  const double* beta;           // [M+1]
  const double* tau;            // [M+1] tau_m = t_m - t_{m-1}
  const double* xv;             // [M+1] (t_m / T)^gamma, the initial guess's extrapolation coordinate
  const double* theta;          // [(M+1) * nexp]
  const double* decay;          // [(M+1) * nexp]
  const double* gw;             // [nexp]
  const double* ahat;           // [Nc+1]
  const double* qhat;           // [(M+1) * (Nc+1)] per-level P^{-1} symbols (FP64 path)
  const float* qhatf;           // same in FP32 (mixed path)
  // caller's arrays (natural layout)
  const double* kappa;
  const double* f;
  const double* phi;
  // state (tile-major, vlen doubles each)
  double* u[kRing];             // u^m lives in u[m % kRing]
  double* F;                    // [ntiles][nexp][2*CT*N1]
  double* kap;                  // kappa^m, tile-major
  double* dsc;                  // kbar_m / kappa^m, tile-major (kappa-scaled preconditioner)
  const double* kbar;           // [M+1] mean of kappa^m
  const double* kmax;           // [M+1] largest kappa^m_i (rounding level of a residual)
  double anorm;                 // ||A||_inf = a_0 + 2 sum_{d>=1} |a_d| (first column of A)
  double floor_scale;           // factor on the residual's rounding level (1; 0 accepts only kPcgSlack tol)
  double* vec[10];              // Krylov vectors (solver specific)
  float* zf;                    // FGMRES: Z basis in FP32 (mixed), [restart][vlen]
  double* zd;                   // FGMRES: Z basis in FP64, [restart][vlen]
  double* V;                    // FGMRES: V basis, [restart+1][vlen]
  double* uhist;                // [(M+1)][vlen] when store_states
  double2* T;                   // FFT intermediate, Nc complex
  const unsigned* symflag;      // highest level whose symbol, kbar and kmax are built (raised by the
                                //   symbol stream while the levels run), or null: all are built
  float2* Tf;                   // FP32 FFT intermediate, Nc complex
  double* part;                 // [SL_COUNT][ntiles]
  fids_step_info* info;         // [M]
  int* status;                  // [4]: status, last completed level, stop flag
  unsigned* bar;                // group barrier: generation of workgroup r at bar[r * kBarSlotWords]
  // SOE helpers: nh workgroups stream the history one level ahead
  int nh;                       // helper workgroups (0: the solver group streams F itself)
  const double* soec;           // [M+1] c_m = sum_j g w_j theta_{m,j}
  double* H1;                   // [2][vlen] sum_j g w_j e^{-s_j tau_m} F_j^{(m-1)}, slot m & 1
  double* AU;                   // [kRing][vlen] A u^k of the last levels, slot k % kRing
  unsigned* sync2;              // [0]: helper step completions, [64]: last completed level
  unsigned* hflag;              // [nh][64]: per-helper release flags (one 256-byte line each)
  // direct history (the scheme (4.1)): b^m = sum_{k<m} dhw[(m-1) m / 2 + k] u^k + f^m
  int history;                  // FIDS_HISTORY_SOE | FIDS_HISTORY_DIRECT
  const double* dhw;            // [M (M + 1) / 2] weights (g included), or null
  // with helpers (nh > 0) helper step k forms level k+1's sum without u^k in
  // djc chunks of the states (partials dpart[(k+1) & 1][chunk][vlen]) over dec
  // element blocks of kThreads active items (dact active rows of each tile)
  double* dpart;
  int dec, djc, dact;
  // forward snapshots for the adjoint's segment recomputation
  int ckpt_every;               // C (0: none)
  double* ckpt;                 // [(M-1)/C][nexp + 2 kRing][vlen]: u^{m-1..m-kRing}, A u^{m-1..m-kRing},
                                //   F^{(m-1)}
  // adjoint descriptor only (adjoint = 1): u[] holds the transposed solutions
  // y^m (lambda^m = y^m / kappa^m), F the adjoint history, uhist the forward
  // states u^m read back
  int adjoint;
  double* ubar[3];              // ubar^m lives in ubar[m % 3]
  double* lam;                  // lambda of the last finished level, tile-major
  double* gk;                   // dJ/dkappa accumulated over levels (time-independent kappa), tile-major
  double* g_kappa;              // caller's [M][nn] dJ/dkappa (time-dependent kappa) or null
  double* g_f;                  // caller's [M][nn] dJ/df or null
};

// Bluestein / symbol-precompute descriptor (batched over levels).
struct SymJob {
  int n, L, Nc, M;
  Plan plc;                     // complex plan of length L
  Plan plr;                     // real-packed plan of length L (Nc = L/2)
  const double* beta;           // [M+1]
  const double* kbar;           // [M+1] mean of kappa^m
  const double* lam;            // [n]
  const double2* chirp;         // [n]
  const double2* chirp_hat;     // [L]
  double2* Tb;                  // [chunk][L]
  double* q;                    // [chunk][n]
  double2* Tq;                  // [chunk][Nc]
  double* qhat;                 // [(M+1)][Nc+1] (may be null)
  float* qhatf;                 // [(M+1)][Nc+1] (may be null)
  int identity;                 // precond NONE: symbols are all ones
};

}  // namespace fids
