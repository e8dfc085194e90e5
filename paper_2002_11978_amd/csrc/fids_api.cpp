// C ABI of the library (include/fids.h): parameter checks, workspace layout,
// upload of the host set-up tables, and the launches of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "fids.h"
#include "fids_device.h"
#include "fids_launch.h"
#include "fids_setup.h"

using fids::cplx;
using fids::HostTables;
using fids::Plan;
using fids::Prob;
using fids::SymJob;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int ilog2i(int64_t v) { int r = 0; while ((int64_t(1) << r) < v) ++r; return r; }

// Shapes of a two-pass plan for Nc complex points: Nc = N1 * N2, column tiles
// of CT columns and row groups of RU row-pair units, each at most kTileCap
// points so that a workgroup's ping-pong buffers fit in LDS.
struct PlanShape {
  int Nc, N1, N2, log1, log2, CT, ntiles, nunits, RU, nrg;
};

constexpr int kTileCap = 2048;

PlanShape plan_shape(int64_t Nc, int target_tiles, int target_groups, int skew = 0, int cap = kTileCap) {
  PlanShape s{};
  const int p = ilog2i(Nc);
  s.Nc = int(Nc);
  // skew > 0 moves factors of two from the column length N1 to the row length
  // N2: more columns per tile for the same tile count, i.e. longer contiguous
  // runs (CT complex values) in the column passes' strided accesses
  s.log1 = std::max(1, (p + 1) / 2 - std::max(skew, 0));
  s.log2 = p - s.log1;
  s.N1 = 1 << s.log1;
  s.N2 = 1 << s.log2;
  int nt = 1;
  while (nt * 2 <= std::min(target_tiles, s.N2)) nt *= 2;   // powers of two only
  int ct = s.N2 / nt;
  while (ct > 1 && ct * s.N1 > cap) ct >>= 1;
  s.CT = ct;
  s.ntiles = s.N2 / s.CT;
  s.nunits = s.N1 / 2;
  int ng = 1;
  while (ng * 2 <= std::min(target_groups, s.nunits)) ng *= 2;
  int ru = s.nunits / ng;
  while (ru > 1 && 2 * ru * s.N2 > cap) ru >>= 1;
  s.RU = ru;
  s.nrg = s.nunits / s.RU;
  return s;
}

// Workgroups per problem: about one per 1024 packed points (a pass moves
// about 16 KiB per workgroup), at most 64.  The group barrier costs about
// 1.5 us + 70 ns per workgroup on MI355X, but the work inside a pass (LDS
// FFT stages, dependent global rounds) dominates, so wider groups win up to
// this size.
int default_group(int64_t Nc) {
  int64_t g = Nc / 1024;
  return int(std::max<int64_t>(1, std::min<int64_t>(64, g)));
}

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Workspace layout of one problem.  Offsets are bytes from ws_d.
struct Layout {
  size_t prob, job, abort_, symflag, status, bar, info, part;
  size_t beta, theta, decay, gw, ahat, lam, chirp, chirp_hat, kbar, kmax, xv;
  size_t tw1r, tw1rf, tw2r, tw2rf, tw1c, tw1cf, tw2c, tw2cf, twlo, twlof, twhi, twhif;
  size_t qhat, qhatf;
  size_t Tb, q, Tq;
  size_t u[fids::kRing], F, kap, dsc, vec[10], uhist, T, Tf, tau, V, Z, Zf, soec, H1, AU, sync2, hflag;
  // adjoint: segment snapshots and the adjoint descriptor's state
  size_t dhw, dpart;
  int djc_cap;      // direct history: state chunks dpart holds per slot
  size_t ckpt, aprob, ainfo, astatus, ubar[3], yr[fids::kRing], Fbar, alam, gk, AUa;
  int nck;          // snapshots held (levels kC + 1, k = 1..nck)
  int hist_cap;     // states uhist holds
  size_t total;
  int chunk;
  int twshift;
};

// Batch workspace: descriptors, status words and level reports of all
// members, then one single-problem workspace per member.
struct BatchLayout {
  size_t probs, status, info, abort_, head, total;
  std::vector<size_t> member, member_bytes;
};

struct Shapes {
  int64_t n, M, L, Nc;
  int nexp;
  int grp;                // workgroups the problem's group may use
  PlanShape pr, pc, ps;   // level plan, Bluestein (complex L) plan, symbol (real) plan
};

// Device memory the per-level symbol construction may use for its batches of
// levels (the caller's workspace; the allocation-free entry point uses less).
constexpr size_t kSymBudget = size_t(64) << 20;

Layout make_layout(const fids_params& p, const Shapes& sh, size_t sym_budget = kSymBudget) {
  Layout lo{};
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
  const size_t n = size_t(sh.n), M = size_t(sh.M), L = size_t(sh.L), Nc = size_t(sh.Nc), ne = size_t(sh.nexp);
  lo.prob = take(sizeof(Prob));
  lo.job = take(sizeof(SymJob));
  lo.abort_ = take(sizeof(int));
  lo.symflag = take(sizeof(unsigned));
  lo.status = take(4 * sizeof(int));
  lo.bar = take(fids::kBarBytes);
  lo.info = take(M * sizeof(fids_step_info));
  // partial sums: one slot per column tile; sized for the finest split (CT = 1)
  // so that the layout does not depend on the group size a batch assigns
  lo.part = take(size_t(fids::SL_COUNT) * size_t(sh.pr.N2) * sizeof(double));
  lo.beta = take((M + 1) * 8);
  lo.tau = take((M + 1) * 8);
  lo.soec = take((M + 1) * 8);
  lo.xv = take((M + 1) * 8);
  // synchronisation words on separate 4 KiB pages (separate memory channels)
  off = (off + 4095) / 4096 * 4096;
  lo.sync2 = take(4096);
  lo.hflag = take(4096 * 64);
  lo.theta = take((M + 1) * ne * 8);
  lo.decay = take((M + 1) * ne * 8);
  lo.gw = take(ne * 8);
  lo.ahat = take((Nc + 1) * 8);
  lo.lam = take(n * 8);
  lo.chirp = take(n * 16);
  lo.chirp_hat = take(L * 16);
  lo.kbar = take((M + 1) * 8);
  lo.kmax = take((M + 1) * 8);
  lo.tw1r = take(size_t(sh.pr.N1) * 16); lo.tw1rf = take(size_t(sh.pr.N1) * 8);
  lo.tw2r = take(size_t(sh.pr.N2) * 16); lo.tw2rf = take(size_t(sh.pr.N2) * 8);
  lo.tw1c = take(size_t(sh.pc.N1) * 16); lo.tw1cf = take(size_t(sh.pc.N1) * 8);
  lo.tw2c = take(size_t(sh.pc.N2) * 16); lo.tw2cf = take(size_t(sh.pc.N2) * 8);
  const int q = ilog2i(sh.L);
  lo.twshift = (q + 1) / 2;
  const size_t nlo = size_t(1) << lo.twshift, nhi = L >> lo.twshift;
  lo.twlo = take(nlo * 16); lo.twlof = take(nlo * 8);
  lo.twhi = take(nhi * 16); lo.twhif = take(nhi * 8);
  const bool mixed = p.precision == FIDS_MIXED;
  // FP64 symbols always (the mixed form falls back to them), FP32 copies for the mixed form
  lo.qhat = take((M + 1) * (Nc + 1) * 8);
  lo.qhatf = mixed ? take((M + 1) * (Nc + 1) * 4) : 0;
  // symbol scratch: levels built together, about sym_budget bytes
  const size_t per = L * 16 + n * 8 + Nc * 16;
  lo.chunk = int(std::max<size_t>(1, std::min<size_t>(M, sym_budget / per)));
  lo.Tb = take(size_t(lo.chunk) * L * 16);
  lo.q = take(size_t(lo.chunk) * n * 8);
  lo.Tq = take(size_t(lo.chunk) * Nc * 16);
  for (int i = 0; i < fids::kRing; ++i) lo.u[i] = take(L * 8);
  lo.F = take(ne * L * 8);
  lo.kap = take(L * 8);
  lo.dsc = take(L * 8);
  lo.H1 = take(2 * L * 8);
  lo.AU = take(size_t(fids::kRing) * L * 8);
  for (int i = 0; i < 10; ++i) lo.vec[i] = take(L * 8);
  const size_t C = size_t(std::max(p.checkpoint_every, 0));
  const bool direct = p.history == FIDS_HISTORY_DIRECT;
  lo.dhw = direct ? take(M * (M + 1) / 2 * 8) : 0;
  lo.djc_cap = direct ? fids::direct_chunks(n, fids::kMaxHelpers) : 0;
  lo.dpart = direct ? take(size_t(2) * size_t(lo.djc_cap) * L * 8) : 0;
  // the direct history reads every earlier state
  lo.hist_cap = (p.store_states || direct) ? int(M + 1) : (C > 0 ? int(std::min(C, M) + 1) : 0);
  lo.uhist = lo.hist_cap ? take(size_t(lo.hist_cap) * L * 8) : 0;
  lo.nck = (!p.store_states && !direct && C > 0) ? int((M - 1) / C) : 0;
  lo.ckpt = lo.nck ? take(size_t(lo.nck) * (ne + 2 * fids::kRing) * L * 8) : 0;
  if (!direct && (p.store_states || C > 0)) {
    lo.aprob = take(sizeof(Prob));
    lo.ainfo = take(M * sizeof(fids_step_info));
    lo.astatus = take(4 * sizeof(int));
    for (int i = 0; i < 3; ++i) lo.ubar[i] = take(L * 8);
    for (int i = 0; i < fids::kRing; ++i) lo.yr[i] = take(L * 8);
    lo.Fbar = take(ne * L * 8);
    lo.alam = take(L * 8);
    lo.gk = take(L * 8);
    lo.AUa = take(size_t(fids::kRing) * L * 8);
  }
  const bool gm = p.solver == FIDS_FGMRES;
  lo.V = gm ? take(size_t(p.restart + 1) * L * 8) : 0;
  lo.Z = gm ? take(size_t(p.restart) * L * 8) : 0;
  lo.Zf = (gm && mixed) ? take(size_t(p.restart) * L * 4) : 0;
  lo.T = take(Nc * 16);
  lo.Tf = take(Nc * 8);
  lo.total = off;
  return lo;
}

int shapes_of(const fids_params& p, Shapes& sh, fids::SoeNodes* soe_out) {
  if (fids::validate(p) != FIDS_OK) return FIDS_EINVAL;
  sh.n = fids::toeplitz_len(p);
  sh.M = p.M;
  sh.L = fids::embed_length(sh.n);
  sh.Nc = sh.L / 2;
  fids::SoeNodes soe;
  const double tau1 = p.T * std::pow(1.0 / double(p.M), p.r);
  if (fids::soe_build(p.gamma, tau1, p.T, p.soe_tol, soe) != FIDS_OK) return FIDS_EINVAL;
  sh.nexp = int(soe.s.size());
  const int grp = p.wg_count > 0 ? p.wg_count : env_int("FIDS_WG", default_group(sh.Nc));
  sh.grp = std::max(1, grp);
  // column tiles default to one per workgroup; FIDS_TILES overrides (tuning)
  const int skew = env_int("FIDS_SKEW", 0);
  sh.pr = plan_shape(sh.Nc, env_int("FIDS_TILES", grp), grp, skew);
  sh.pc = plan_shape(sh.L, std::max(1, int((sh.L >> ((ilog2i(sh.L) + 1) / 2)) / 8)), 1 << 30);
  sh.pc.RU = 1;
  sh.pc.nrg = sh.pc.nunits;
  // the symbol plan shares the level plan's N1 / N2 twiddle tables: same split
  sh.ps = plan_shape(sh.Nc, std::max(1, int((sh.Nc >> ((ilog2i(sh.Nc) + 1) / 2)) / 8)), 1 << 30, skew);
  sh.ps.RU = 1;
  sh.ps.nrg = sh.ps.nunits;
  if (soe_out) *soe_out = soe;
  return FIDS_OK;
}

std::vector<double2> twiddles(int64_t P) {
  std::vector<double2> t(P);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int64_t j = 0; j < P; ++j) {
    const long double a = -2.0L * pi * (long double)j / (long double)P;
    t[j] = make_double2(double(std::cos(a)), double(std::sin(a)));
  }
  return t;
}

std::vector<double2> root_table(int64_t L, int64_t count, int64_t step) {
  std::vector<double2> t(count);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int64_t j = 0; j < count; ++j) {
    const long double a = -2.0L * pi * (long double)(j * step) / (long double)L;
    t[j] = make_double2(double(std::cos(a)), double(std::sin(a)));
  }
  return t;
}

std::vector<float2> to_f(const std::vector<double2>& v) {
  std::vector<float2> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = make_float2(float(v[i].x), float(v[i].y));
  return o;
}

}  // namespace

struct fids_problem {
  fids_params prm{};
  HostTables tab;
  Shapes sh{};
  Layout lo{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Prob hp{};
  Prob* dp = nullptr;
  Prob ha{};                 // adjoint descriptor (when the layout has one)
  Prob* dpa = nullptr;
  SymJob hj{};
  SymJob* dj = nullptr;
  int* dabort = nullptr;
  int* dstatus = nullptr;
  int64_t level = 0;
  int64_t sym_hi = 0;        // per-level symbols (and kbar, kmax) valid for levels 1..sym_hi
  bool poisoned = false;     // a level failed: the state is only valid after fids_reset
  size_t lds = 0;
  unsigned long long timeout_ticks = 0;
  // symbols built on a stream of their own while the level kernel runs
  // (null: built on `stream` before the launch)
  hipStream_t sstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  unsigned* symflag = nullptr;
  // host copies kept alive for asynchronous uploads
  std::vector<std::vector<double2>> keep2;
  std::vector<std::vector<float2>> keepf;
  std::vector<double> keepd;     // direct-history weights
  ~fids_problem() {
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (sstream) (void)hipStreamDestroy(sstream);
  }
};

struct fids_batch {
  BatchLayout bl;
  int32_t count = 0;
  int64_t M = 0;
  int64_t level = 0;
  bool poisoned = false;
  bool graph_mode = false;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Prob* dprobs = nullptr;
  int* dstatus = nullptr;
  fids_step_info* dinfo = nullptr;
  size_t lds = 0;
  int total_wg = 0;              // workgroups of one launch (sum of the slots' groups)
  bool cooperative = false;      // some member has a group of more than one workgroup
  int* dabort = nullptr;
  unsigned long long timeout_ticks = 0;
  std::vector<Prob> hprobs;      // descriptors in launch order (slots)
  std::vector<fids_problem*> members;
  std::vector<int> groups;       // workgroups of each member's group
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;   // capture needs a stream other than the legacy default
  // members' symbols are built on kBatchSymStreams streams at once (each
  // member's small symbol kernels leave most of the device idle)
  static constexpr int kBatchSymStreams = 4;
  hipStream_t sstreams[kBatchSymStreams] = {};
  hipEvent_t sev[kBatchSymStreams + 1] = {};
  ~fids_batch() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : sev)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t t : sstreams)
      if (t) (void)hipStreamDestroy(t);
    for (fids_problem* h : members) delete h;
  }
};

namespace {

// Records the call site and message of a failed HIP call (fids_last_error).
thread_local char g_last_error[256] = "";
bool hip_bad(hipError_t e, int line) {
  if (e == hipSuccess) return false;
  std::snprintf(g_last_error, sizeof(g_last_error), "fids_api.cpp:%d: %s (%d)", line, hipGetErrorString(e),
                int(e));
  return true;
}

#define HIPCHK(x)                                    \
  do {                                               \
    if (hip_bad((x), __LINE__)) return FIDS_EDEVICE; \
  } while (0)

template <typename T>
T* at(char* ws, size_t off) { return reinterpret_cast<T*>(ws + off); }

int upload(fids_problem* h, size_t off, const void* src, size_t bytes) {
  if (bytes == 0) return FIDS_OK;
  HIPCHK(hipMemcpyAsync(h->ws + off, src, bytes, hipMemcpyHostToDevice, h->stream));
  return FIDS_OK;
}

void fill_plan(Plan& pl, const PlanShape& s, int rootmul, char* ws, const Layout& lo, bool complex_plan) {
  pl.twres = 0;
  pl.Nc = s.Nc; pl.N1 = s.N1; pl.N2 = s.N2; pl.log1 = s.log1; pl.log2 = s.log2; pl.CT = s.CT;
  pl.ntiles = s.ntiles; pl.nunits = s.nunits; pl.RU = s.RU; pl.nrg = s.nrg; pl.rootmul = rootmul;
  pl.twshift = lo.twshift; pl.twmask = (1 << lo.twshift) - 1;
  pl.twn = fids::lds_twiddles(pl, s.Nc * rootmul);
  pl.tw1 = at<double2>(ws, complex_plan ? lo.tw1c : lo.tw1r);
  pl.tw1f = at<float2>(ws, complex_plan ? lo.tw1cf : lo.tw1rf);
  pl.tw2 = at<double2>(ws, complex_plan ? lo.tw2c : lo.tw2r);
  pl.tw2f = at<float2>(ws, complex_plan ? lo.tw2cf : lo.tw2rf);
  pl.twlo = at<double2>(ws, lo.twlo); pl.twlof = at<float2>(ws, lo.twlof);
  pl.twhi = at<double2>(ws, lo.twhi); pl.twhif = at<float2>(ws, lo.twhif);
}

// The first twiddle residency (all tables in LDS, then the root tables out,
// then all out) whose level-kernel LDS fits `cap`.
int fit_lds(Prob& hp, size_t cap) {
  for (int r = 0; r <= 2; ++r) {
    hp.pl.twres = r;
    hp.pl.twn = fids::lds_twiddles(hp.pl, hp.L);
    if (fids::level_lds_bytes(hp) <= cap) return FIDS_OK;
  }
  return FIDS_EDEVICE;
}

// Builds kbar_m, kmax_m and the per-level preconditioner symbols of levels
// sym_hi+1..m_hi (those of earlier levels are current) on stream s, raising
// the problem's symbol flag after each chunk of levels when it has one.
int build_symbols(fids_problem* h, int64_t m_hi, hipStream_t s) {
  const int a = int(h->sym_hi + 1), cnt = int(m_hi - h->sym_hi);
  HIPCHK(fids::launch_kbar(h->hp.kappa, int(fids::natural_len(h->prm)), a, cnt, h->prm.kappa_time_dependent,
                           at<double>(h->ws, h->lo.kbar), at<double>(h->ws, h->lo.kmax), s));
  for (int m0 = a; m0 <= int(m_hi); m0 += h->lo.chunk) {
    const int c = std::min(h->lo.chunk, int(m_hi) - m0 + 1);
    HIPCHK(fids::launch_symbols(h->hj, h->dj, m0, c, s));
    if (h->symflag) HIPCHK(fids::launch_flag(h->symflag, unsigned(m0 + c - 1), s));
  }
  h->sym_hi = m_hi;
  return FIDS_OK;
}

int ensure_symbols(fids_problem* h, int64_t m_hi) {
  m_hi = std::min<int64_t>(m_hi, h->sh.M);
  if (h->sym_hi >= m_hi) return FIDS_OK;
  return build_symbols(h, m_hi, h->stream);
}
int ensure_symbols(fids_problem* h) { return ensure_symbols(h, h->sh.M); }

// One cooperative launch of the level kernel for descriptor `d` and a wait
// for its status words {status, last completed level}; `after` (may be null)
// is an event of other work the stream then waits for as well.
int launch_wait(fids_problem* h, const Prob& hd, Prob* d, int m_begin, int m_end, int hist_lo, int ckpt_on,
                int stat[2], hipEvent_t after = nullptr) {
  const hipError_t ez = hipMemsetAsync(h->dabort, 0, sizeof(int), h->stream);
  const hipError_t el = ez != hipSuccess ? ez
                        : fids::launch_levels(hd, d, 1, hd.ng + hd.nh, h->lds, m_begin, m_end, hist_lo, ckpt_on,
                                              h->timeout_ticks, h->dabort, h->stream);
  // the stream waits for the other work even when the launch failed, so that
  // nothing enqueued on it later overlaps that work
  if (after) HIPCHK(hipStreamWaitEvent(h->stream, after, 0));
  if (hip_bad(el, __LINE__)) return FIDS_EDEVICE;
  HIPCHK(hipMemcpyAsync(stat, hd.status, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (stat[0] == FIDS_EDEVICE) {
    // a group barrier timed out: clear the barrier words for the next launch
    HIPCHK(hipMemsetAsync(hd.bar, 0, fids::kBarBytes, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return FIDS_OK;
}

int hist_lo_of(const fids_problem* h) { return h->prm.store_states ? 0 : -1; }

// Levels level+1..m_end in one launch (symbols of exactly those levels built
// first); infos_host (may be NULL) receives the reports of the levels run,
// entry k for level level+1+k.
int run_levels(fids_problem* h, int64_t m_end, fids_step_info* infos_host) {
  if (h->level >= h->sh.M || h->poisoned) return FIDS_ESTATE;
  int st = FIDS_OK;
  hipEvent_t after = nullptr;
  if (h->sstream && h->sym_hi < m_end && env_int("FIDS_SYM_OVERLAP", 1) != 0) {
    // the symbols of these levels are built on the symbol stream, a chunk of
    // levels at a time, on the CUs the solver group leaves free; each level
    // waits for its own (the first chunk is ready after about 0.2 ms)
    HIPCHK(hipEventRecord(h->ev_in, h->stream));
    HIPCHK(hipStreamWaitEvent(h->sstream, h->ev_in, 0));
    st = build_symbols(h, m_end, h->sstream);
    HIPCHK(hipEventRecord(h->ev_out, h->sstream));
    if (st != FIDS_OK) {
      HIPCHK(hipStreamWaitEvent(h->stream, h->ev_out, 0));
      return st;
    }
    after = h->ev_out;
  } else {
    st = ensure_symbols(h, m_end);
    if (st != FIDS_OK) return st;
  }
  const int m_begin = int(h->level + 1);
  int stat[2] = {0, 0};
  st = launch_wait(h, h->hp, h->dp, m_begin, int(m_end), hist_lo_of(h), h->lo.nck > 0, stat, after);
  if (st != FIDS_OK) return st;
  const int64_t last = stat[1];
  const int64_t first = m_begin;
  const int64_t upto = std::min<int64_t>(m_end, std::max<int64_t>(last + (stat[0] != FIDS_OK ? 1 : 0), first - 1));
  if (infos_host && upto >= first) {
    HIPCHK(hipMemcpy(infos_host, at<fids_step_info>(h->ws, h->lo.info) + (first - 1),
                     size_t(upto - first + 1) * sizeof(fids_step_info), hipMemcpyDeviceToHost));
  }
  if (last >= first) h->level = last;
  if (stat[0] != FIDS_OK) h->poisoned = true;
  return stat[0];
}

// Forward state entering level a = kC + 1 from its snapshot (a = 1: the
// initial state u^0 = u^{-1} = phi, empty history).
int restore_segment(fids_problem* h, int a) {
  const Prob& hp = h->hp;
  const size_t vb = size_t(hp.vlen) * 8;
  if (a == 1) {
    HIPCHK(hipMemsetAsync(hp.F, 0, size_t(hp.nexp) * vb, h->stream));
    HIPCHK(hipMemsetAsync(hp.AU, 0, size_t(fids::kRing) * vb, h->stream));
    HIPCHK(fids::launch_init_state(hp, h->dp, h->stream));
    return FIDS_OK;
  }
  const int C = hp.ckpt_every;
  constexpr int R = fids::kRing;
  const double* ck = hp.ckpt + size_t((a - 1) / C - 1) * size_t(hp.nexp + 2 * R) * hp.vlen;
  const size_t v = size_t(hp.vlen);
  for (int k = 0; k < R; ++k) {
    const int slot = (a - 1 - k + 2 * R) % R;    // u^{a-1-k}, A u^{a-1-k}
    HIPCHK(hipMemcpyAsync(hp.u[slot], ck + size_t(k) * v, vb, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(hp.AU + size_t(slot) * v, ck + size_t(R + k) * v, vb, hipMemcpyDeviceToDevice,
                          h->stream));
  }
  HIPCHK(hipMemcpyAsync(hp.F, ck + size_t(2 * R) * v, size_t(hp.nexp) * vb, hipMemcpyDeviceToDevice, h->stream));
  return FIDS_OK;
}

// Parameter overrides of a batch member.
void batch_params(fids_params& p, int group = 1) {
  p.wg_count = group;
  p.soe_helpers = 0;
  p.checkpoint_every = 0;
  p.store_states = 0;
}

// Set-up of one problem.  A batch member (batch = true) runs on a single
// workgroup (ng = 1, no helpers, no snapshots); the batch sets the LDS limit
// and synchronises once for all of its members.
int init_impl(const fids_params* pin, const double* kappa_d, const double* f_d, const double* phi_d,
              void* ws_d, size_t ws_bytes, void* hip_stream, int batch_group, fids_problem** out,
              size_t sym_budget = kSymBudget, bool overlap = true) {
  const bool batch = batch_group > 0;
  fids_params pb = *pin;
  if (batch) batch_params(pb, batch_group);
  const fids_params* p = &pb;
  if (pb.history == FIDS_HISTORY_DIRECT) {
    pb.store_states = 1;      // every earlier state is read by the direct history
    pb.checkpoint_every = 0;
  }
  fids_problem* h = new (std::nothrow) fids_problem();
  if (!h) return FIDS_EINVAL;
  h->prm = *p;
  if (shapes_of(*p, h->sh, nullptr) != FIDS_OK || fids::build_tables(*p, h->tab) != FIDS_OK) {
    delete h;
    return FIDS_EINVAL;
  }
  h->sh.nexp = h->tab.nexp;
  h->lo = make_layout(*p, h->sh, sym_budget);
  if (ws_bytes < h->lo.total) { delete h; return FIDS_EINVAL; }
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(ws_d);
  char* ws = h->ws;
  const Layout& lo = h->lo;
  const HostTables& t = h->tab;
  int st = FIDS_OK;
  auto fail = [&](int code) { delete h; return code; };
  if (hip_bad(hipMemsetAsync(ws, 0, lo.total, h->stream), __LINE__)) return fail(FIDS_EDEVICE);
  // tables
  st |= upload(h, lo.beta, t.beta.data(), t.beta.size() * 8);
  st |= upload(h, lo.tau, t.tau.data(), t.tau.size() * 8);
  st |= upload(h, lo.soec, t.soec.data(), t.soec.size() * 8);
  st |= upload(h, lo.xv, t.xv.data(), t.xv.size() * 8);
  st |= upload(h, lo.theta, t.theta.data(), t.theta.size() * 8);
  st |= upload(h, lo.decay, t.decay.data(), t.decay.size() * 8);
  st |= upload(h, lo.gw, t.gw.data(), t.gw.size() * 8);
  st |= upload(h, lo.ahat, t.ahat.data(), t.ahat.size() * 8);
  st |= upload(h, lo.lam, t.lam.data(), t.lam.size() * 8);
  st |= upload(h, lo.chirp, t.chirp.data(), t.chirp.size() * 16);
  st |= upload(h, lo.chirp_hat, t.chirp_hat.data(), t.chirp_hat.size() * 16);
  auto put2 = [&](size_t o, size_t of, std::vector<double2> v) {
    h->keepf.push_back(to_f(v));
    h->keep2.push_back(std::move(v));
    st |= upload(h, o, h->keep2.back().data(), h->keep2.back().size() * 16);
    st |= upload(h, of, h->keepf.back().data(), h->keepf.back().size() * 8);
  };
  if (lo.dhw) {
    h->keepd = fids::direct_history_weights(p->T, p->M, p->r, p->gamma);
    st |= upload(h, lo.dhw, h->keepd.data(), h->keepd.size() * 8);
  }
  put2(lo.tw1r, lo.tw1rf, twiddles(h->sh.pr.N1));
  put2(lo.tw2r, lo.tw2rf, twiddles(h->sh.pr.N2));
  put2(lo.tw1c, lo.tw1cf, twiddles(h->sh.pc.N1));
  put2(lo.tw2c, lo.tw2cf, twiddles(h->sh.pc.N2));
  put2(lo.twlo, lo.twlof, root_table(h->sh.L, int64_t(1) << lo.twshift, 1));
  put2(lo.twhi, lo.twhif, root_table(h->sh.L, h->sh.L >> lo.twshift, int64_t(1) << lo.twshift));
  if (st != FIDS_OK) return fail(FIDS_EDEVICE);
  // problem descriptor
  Prob& hp = h->hp;
  hp.n = int(h->sh.n); hp.M = int(p->M); hp.nexp = t.nexp;
  hp.nn = int(fids::natural_len(*p));
  hp.nx = p->dims == 2 ? int(p->n) : 0;
  hp.sx = int(fids::row_stride(*p));
  hp.lsx = hp.sx > 0 ? ilog2i(hp.sx) : 0;
  hp.vmask = hp.sx > 0 ? hp.sx - 1 : 0;
  hp.vlim = hp.sx > 0 ? hp.nx : 1;
  hp.solver = p->solver; hp.precision = p->precision; hp.precond = p->precond;
  hp.kappa_td = p->kappa_time_dependent; hp.x0_mode = p->x0_mode; hp.maxit = p->krylov_maxit;
  hp.restart = p->restart; hp.store_states = p->store_states; hp.tol = p->krylov_tol;
  hp.L = int(h->sh.L); hp.vlen = int(h->sh.L);
  fill_plan(hp.pl, h->sh.pr, 2, ws, lo, false);
  hp.g0 = 0;
  hp.slot_first = 0;
  // one workgroup per column tile or row group, up to the group size (a
  // workgroup runs several tiles in turn where the LDS tile cap forces more
  // tiles than that; sums stay per tile, so the result does not depend on ng);
  // at most kMaxGroup, the arrival slots of the group barrier
  hp.ng = std::max(1, std::min({std::max(hp.pl.ntiles, hp.pl.nrg), h->sh.grp, fids::kMaxGroup}));
  hp.soec = at<double>(ws, lo.soec);
  hp.H1 = at<double>(ws, lo.H1);
  hp.AU = at<double>(ws, lo.AU);
  hp.sync2 = at<unsigned>(ws, lo.sync2);
  hp.hflag = at<unsigned>(ws, lo.hflag);
  hp.xv = at<double>(ws, lo.xv);
  hp.beta = at<double>(ws, lo.beta); hp.tau = at<double>(ws, lo.tau); hp.theta = at<double>(ws, lo.theta); hp.decay = at<double>(ws, lo.decay);
  hp.gw = at<double>(ws, lo.gw); hp.ahat = at<double>(ws, lo.ahat);
  hp.qhat = lo.qhat ? at<double>(ws, lo.qhat) : nullptr;
  hp.qhatf = lo.qhatf ? at<float>(ws, lo.qhatf) : nullptr;
  hp.kappa = kappa_d; hp.f = f_d; hp.phi = phi_d;
  for (int i = 0; i < fids::kRing; ++i) hp.u[i] = at<double>(ws, lo.u[i]);
  hp.F = at<double>(ws, lo.F); hp.kap = at<double>(ws, lo.kap); hp.dsc = at<double>(ws, lo.dsc);
  hp.kbar = at<double>(ws, lo.kbar);
  hp.kmax = at<double>(ws, lo.kmax);
  {
    // ||A||_inf of the symmetric Toeplitz A: its first row's absolute sum, at most a_0 + 2 sum_{d>=1} |a_d|
    long double a = std::fabs((long double)t.col[0]);
    for (size_t d = 1; d < t.col.size(); ++d) a += 2.0L * std::fabs((long double)t.col[d]);
    hp.anorm = double(a);
  }
  {
    const char* fs = std::getenv("FIDS_FLOOR_SCALE");
    hp.floor_scale = fs ? std::max(0.0, std::atof(fs)) : 1.0;
  }
  for (int i = 0; i < 10; ++i) hp.vec[i] = at<double>(ws, lo.vec[i]);
  hp.V = lo.V ? at<double>(ws, lo.V) : nullptr;
  hp.zd = lo.Z ? at<double>(ws, lo.Z) : nullptr;
  hp.zf = lo.Zf ? at<float>(ws, lo.Zf) : nullptr;
  hp.uhist = lo.uhist ? at<double>(ws, lo.uhist) : nullptr;
  hp.T = at<double2>(ws, lo.T); hp.Tf = at<float2>(ws, lo.Tf);
  hp.history = p->history;
  hp.dhw = lo.dhw ? at<double>(ws, lo.dhw) : nullptr;
  hp.dpart = lo.dpart ? at<double>(ws, lo.dpart) : nullptr;
  hp.dec = hp.djc = hp.dact = 0;
  hp.ckpt_every = std::max(p->checkpoint_every, 0);
  hp.ckpt = lo.ckpt ? at<double>(ws, lo.ckpt) : nullptr;
  hp.adjoint = 0;
  hp.part = at<double>(ws, lo.part);
  hp.info = at<fids_step_info>(ws, lo.info);
  hp.status = at<int>(ws, lo.status);
  hp.bar = at<unsigned>(ws, lo.bar);
  h->dp = at<Prob>(ws, lo.prob);
  h->dabort = at<int>(ws, lo.abort_);
  h->dstatus = hp.status;
  // symbol job
  SymJob& j = h->hj;
  j.n = int(h->sh.n); j.L = int(h->sh.L); j.Nc = int(h->sh.Nc); j.M = int(p->M);
  fill_plan(j.plc, h->sh.pc, 1, ws, lo, true);
  fill_plan(j.plr, h->sh.ps, 2, ws, lo, false);
  j.beta = hp.beta; j.kbar = at<double>(ws, lo.kbar); j.lam = at<double>(ws, lo.lam);
  j.chirp = at<double2>(ws, lo.chirp); j.chirp_hat = at<double2>(ws, lo.chirp_hat);
  j.Tb = at<double2>(ws, lo.Tb); j.q = at<double>(ws, lo.q); j.Tq = at<double2>(ws, lo.Tq);
  j.qhat = const_cast<double*>(hp.qhat); j.qhatf = const_cast<float*>(hp.qhatf);
  j.identity = p->precond == FIDS_NONE;
  h->dj = at<SymJob>(ws, lo.job);
  {
    // long transforms: leave twiddle tables in global memory until the
    // tiles and tables fit the LDS (Plan::twres)
    size_t cap = 0;
    if (hip_bad(fids::level_lds_cap(hp, &cap), __LINE__)) return fail(FIDS_EDEVICE);
    if (fit_lds(hp, cap) != FIDS_OK) {
      std::snprintf(g_last_error, sizeof(g_last_error), "fids_api.cpp:%d: level kernel needs %zu bytes of LDS (%zu available)",
                    __LINE__, fids::level_lds_bytes(hp), cap);
      return fail(FIDS_EDEVICE);
    }
  }
  h->lds = fids::level_lds_bytes(hp);
  if (batch) {
    hp.ng = batch_group;
    hp.nh = 0;
  } else {
    if (h->lds > 65536 && hip_bad(fids::set_level_lds_limit(hp, h->lds), __LINE__)) return fail(FIDS_EDEVICE);
    // SOE helpers use the CUs the solver group leaves free (the launch must
    // stay co-resident)
    int dev = 0, cus = 0, per_cu = 0;
    if (hip_bad(hipGetDevice(&dev), __LINE__) ||
        hip_bad(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), __LINE__) ||
        hip_bad(fids::level_max_blocks(hp, h->lds, &per_cu), __LINE__))
      return fail(FIDS_EDEVICE);
    const int resident = cus * std::max(per_cu, 0);
    if (resident < hp.ng) {
      std::snprintf(g_last_error, sizeof(g_last_error),
                    "fids_api.cpp:%d: %d workgroups cannot be co-resident (%d fit)", __LINE__, hp.ng, resident);
      return fail(FIDS_EDEVICE);
    }
    // SOE history, auto = one helper per solver workgroup: the helpers take
    // the history stream (2 nexp n values per level) out of the solver's
    // right-hand-side phase.  Measured on MI355X, PCG form: n = 65535 with
    // 64 + 64 workgroups 738 -> 720 ms per 2048 levels (32: 731, 96: 728,
    // 128: 736); n = 16383, 16 + 16: 345 -> 329 ms per 1024 levels; n = 4095,
    // 4 + 4: 174 -> 166 ms per 512 levels.  The direct history's sum over
    // every earlier state is a stream of m n values per level: auto = every
    // free workgroup.
    const bool direct = p->history == FIDS_HISTORY_DIRECT;
    int nh = p->soe_helpers >= 0 ? p->soe_helpers
                                 : (direct ? fids::kMaxHelpers : env_int("FIDS_HELPERS", hp.ng));
    nh = std::max(0, std::min({nh, resident - hp.ng, fids::kMaxHelpers}));
    // snapshots are taken where the solver group streams the history itself
    if (p->checkpoint_every > 0) nh = 0;
    hp.nh = nh;
    // a problem of its own (not a batch member, not the static entry point)
    // whose launch leaves at least half of the CUs free builds its symbols
    // on a second stream while its levels run (the levels wait for them, so
    // the symbol kernels must find free CUs: helpers that fill the device
    // rule it out)
    if (overlap && 2 * (hp.ng + hp.nh) <= cus) {
      h->symflag = at<unsigned>(ws, lo.symflag);
      if (hip_bad(hipStreamCreateWithFlags(&h->sstream, hipStreamNonBlocking), __LINE__) ||
          hip_bad(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming), __LINE__) ||
          hip_bad(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming), __LINE__))
        return fail(FIDS_EDEVICE);
    }
    hp.symflag = h->symflag;
    if (direct && nh > 0) {
      // active rows of a tile hold the natural value pairs below ceil(n / 2)
      hp.dact = int(((h->sh.n + 1) / 2 + hp.pl.N2 - 1) / hp.pl.N2);
      const int nact = hp.pl.ntiles * hp.dact * hp.pl.CT;
      hp.dec = (nact + fids::kThreads - 1) / fids::kThreads;
      hp.djc = std::max(1, std::min(nh / hp.dec, lo.djc_cap));
    }
  }
  if (lo.aprob) {
    Prob& ha = h->ha;
    ha = hp;
    ha.adjoint = 1;
    ha.nh = 0;
    ha.f = nullptr;
    ha.ckpt = nullptr;
    for (int i = 0; i < fids::kRing; ++i) ha.u[i] = at<double>(ws, lo.yr[i]);
    for (int i = 0; i < 3; ++i) ha.ubar[i] = at<double>(ws, lo.ubar[i]);
    ha.F = at<double>(ws, lo.Fbar);
    ha.lam = at<double>(ws, lo.alam);
    ha.gk = at<double>(ws, lo.gk);
    ha.AU = at<double>(ws, lo.AUa);
    ha.info = at<fids_step_info>(ws, lo.ainfo);
    ha.status = at<int>(ws, lo.astatus);
    ha.g_kappa = nullptr;
    ha.g_f = nullptr;
    h->dpa = at<Prob>(ws, lo.aprob);
  }
  if (upload(h, lo.prob, &h->hp, sizeof(Prob)) != FIDS_OK) return fail(FIDS_EDEVICE);
  if (upload(h, lo.job, &h->hj, sizeof(SymJob)) != FIDS_OK) return fail(FIDS_EDEVICE);
  if (hip_bad(fids::launch_init_state(hp, h->dp, h->stream), __LINE__)) return fail(FIDS_EDEVICE);
  int dev = 0, rate_khz = 0;
  if (hip_bad(hipGetDevice(&dev), __LINE__)) return fail(FIDS_EDEVICE);
  if (hip_bad(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev), __LINE__)) return fail(FIDS_EDEVICE);
  h->timeout_ticks = (unsigned long long)(std::max(rate_khz, 1000)) * 1000ull * 4ull;  // 4 s
  if (!batch && hip_bad(hipStreamSynchronize(h->stream), __LINE__)) return fail(FIDS_EDEVICE);
  *out = h;
  return FIDS_OK;
}

// ---------------------------------------------------------------- batch helpers
// Work of one level of a member, in units of the embedding length L (the
// passes stream O(L) data each), and the extra cost of a group of k > 1
// workgroups (about 50 group barriers per level at 1.5 us + 70 ns per
// workgroup, which is worth about 260 + 12 k units at 0.29 us per unit on
// one workgroup).
double group_cost(double c, int k) { return c / k + (k > 1 ? 260.0 + 12.0 * k : 0.0); }

// Schedule of a batch on R co-resident workgroups: members whose cost
// exceeds the makespan target T get a group of k > 1 workgroups (powers of
// two up to kmax); the others are packed first-fit-decreasing into
// one-workgroup slots of capacity T.  The smallest feasible T is found by
// bisection.  Returns the slots (group size, members in run order).
struct Slot {
  int ng;
  std::vector<int> members;
};

bool schedule_at(double T, const std::vector<double>& c, const std::vector<int>& kmax, int R,
                 std::vector<Slot>* out) {
  std::vector<Slot> slots;
  std::vector<int> small;
  int total = 0;
  for (size_t i = 0; i < c.size(); ++i) {
    if (c[i] <= T) { small.push_back(int(i)); continue; }
    int k = 2;
    while (k <= kmax[i] && group_cost(c[i], k) > T) k *= 2;
    if (k > kmax[i]) return false;
    slots.push_back({k, {int(i)}});
    total += k;
    if (total > R) return false;
  }
  std::sort(small.begin(), small.end(), [&](int a, int b) { return c[size_t(a)] > c[size_t(b)]; });
  std::vector<double> load;
  std::vector<Slot> bins;
  for (int i : small) {
    size_t j = 0;
    while (j < bins.size() && load[j] + c[size_t(i)] > T) ++j;
    if (j == bins.size()) {
      bins.push_back({1, {}});
      load.push_back(0.0);
      if (total + int(bins.size()) > R) return false;
    }
    bins[j].members.push_back(i);
    load[j] += c[size_t(i)];
  }
  if (out) {
    *out = slots;
    out->insert(out->end(), bins.begin(), bins.end());
  }
  return true;
}

// Workgroups the schedule leaves free go to the members that already have a
// group of several workgroups, heaviest first (prio: the SOE history's size
// n N_exp, which the length-L cost leaves out): each doubling that fits.
// A group of k > 1 costs more than the model's c / k + overhead (on MI355X a
// two-workgroup member with L = 32768 took 1.56x the level time of a
// one-workgroup member with L = 16384), so these members set the makespan
// and the free workgroups shorten it.
void upgrade_groups(std::vector<Slot>& out, const std::vector<int>& kmax, const std::vector<double>& prio, int R) {
  int used = 0;
  for (const Slot& sl : out) used += sl.ng;
  std::vector<size_t> cand;
  for (size_t k = 0; k < out.size(); ++k)
    if (out[k].ng > 1 && out[k].members.size() == 1) cand.push_back(k);
  std::stable_sort(cand.begin(), cand.end(), [&](size_t a, size_t b) {
    return prio[size_t(out[a].members[0])] > prio[size_t(out[b].members[0])];
  });
  for (bool changed = true; changed;) {
    changed = false;
    for (size_t k : cand) {
      Slot& sl = out[k];
      if (2 * sl.ng <= kmax[size_t(sl.members[0])] && used + sl.ng <= R) {
        used += sl.ng;
        sl.ng *= 2;
        changed = true;
      }
    }
  }
}

std::vector<Slot> schedule_batch(const std::vector<double>& c, const std::vector<int>& kmax, int R,
                                 const std::vector<double>* prio = nullptr) {
  double lo = 0.0, hi = 0.0;
  for (size_t i = 0; i < c.size(); ++i) {
    double best = c[i];
    for (int k = 2; k <= kmax[i]; k *= 2) best = std::min(best, group_cost(c[i], k));
    lo = std::max(lo, best);
    hi += c[i];
  }
  std::vector<Slot> out;
  if (!schedule_at(hi, c, kmax, R, &out)) {
    // fewer workgroups than needed even with everything packed: one slot
    out.assign(1, {1, {}});
    for (size_t i = 0; i < c.size(); ++i) out[0].members.push_back(int(i));
    return out;
  }
  if (!schedule_at(lo, c, kmax, R, &out)) {
    for (int it = 0; it < 60; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (schedule_at(mid, c, kmax, R, nullptr)) hi = mid;
      else lo = mid;
    }
    schedule_at(hi, c, kmax, R, &out);
  }
  if (prio) upgrade_groups(out, kmax, *prio, R);
  return out;
}

// Per-member cost (embedding length L), largest useful group (powers of two,
// at least 1024 packed points per workgroup, at most 64) and, optionally, a
// bound on the level kernel's LDS (one-workgroup plans have the largest tiles)
// with a descriptor for the occupancy query.
int batch_costs(const fids_params* p, int32_t count, std::vector<double>& cost, std::vector<int>& kmax,
                size_t* lds_bound, Prob* probe, std::vector<double>* prio = nullptr) {
  cost.assign(size_t(count), 0.0);
  kmax.assign(size_t(count), 1);
  if (prio) prio->assign(size_t(count), 0.0);
  for (int32_t i = 0; i < count; ++i) {
    fids_params q = p[i];
    batch_params(q, 1);
    Shapes sh;
    if (shapes_of(q, sh, nullptr) != FIDS_OK) return FIDS_EINVAL;
    cost[size_t(i)] = double(sh.L);
    if (prio) (*prio)[size_t(i)] = double(sh.n) * double(sh.nexp);
    int k = 1;
    while (k * 2 <= std::min(64, sh.pr.N2) && int64_t(k) * 2 * 1024 <= sh.Nc) k *= 2;
    kmax[size_t(i)] = k;
    if (lds_bound && probe) {
      probe->nexp = sh.nexp; probe->L = int(sh.L); probe->precision = q.precision; probe->solver = q.solver;
      probe->pl.CT = sh.pr.CT; probe->pl.N1 = sh.pr.N1; probe->pl.N2 = sh.pr.N2; probe->pl.RU = sh.pr.RU;
      const int tws = (ilog2i(sh.L) + 1) / 2;
      probe->pl.twshift = tws; probe->pl.twmask = (1 << tws) - 1;
      size_t cap = 0;
      if (fids::level_lds_cap(*probe, &cap) != hipSuccess) return FIDS_EDEVICE;
      if (fit_lds(*probe, cap) != FIDS_OK) return FIDS_EDEVICE;
      *lds_bound = std::max(*lds_bound, fids::level_lds_bytes(*probe));
    }
  }
  return FIDS_OK;
}

int batch_layout(const fids_params* p, int32_t count, BatchLayout& bl) {
  const int64_t M = p[0].M;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
  bl.probs = take(size_t(count) * sizeof(Prob));
  bl.status = take(size_t(count) * 4 * sizeof(int));
  bl.info = take(size_t(count) * size_t(std::max<int64_t>(M, 1)) * sizeof(fids_step_info));
  bl.abort_ = take(sizeof(int));
  bl.head = off;
  bl.member.resize(size_t(count));
  bl.member_bytes.resize(size_t(count));
  for (int32_t i = 0; i < count; ++i) {
    // one kernel instance serves the batch: members share M and the solver variant
    if (p[i].M != M || p[i].solver != p[0].solver || p[i].precision != p[0].precision) return FIDS_EINVAL;
    if (p[i].history != FIDS_HISTORY_SOE) return FIDS_EINVAL;
    fids_params q = p[i];
    batch_params(q);
    Shapes sh;
    if (shapes_of(q, sh, nullptr) != FIDS_OK) return FIDS_EINVAL;
    const size_t bytes = make_layout(q, sh).total;
    bl.member[size_t(i)] = take(bytes);
    bl.member_bytes[size_t(i)] = bytes;
  }
  bl.total = off;
  return FIDS_OK;
}

hipError_t batch_launch(fids_batch* b, int m0, int m1, hipStream_t s) {
  if (!b->cooperative)
    return fids::launch_levels_plain(b->hprobs[0], b->dprobs, b->count, b->total_wg, b->lds, m0, m1, s);
  hipError_t e = hipMemsetAsync(b->dabort, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  return fids::launch_levels(b->hprobs[0], b->dprobs, b->count, b->total_wg, b->lds, m0, m1, -1, 0,
                             b->timeout_ticks, b->dabort, s);
}

// Members' symbols not yet built, spread over the batch's symbol streams
// (after the work already on the batch stream, which then waits for them).
int batch_symbols(fids_batch* b) {
  constexpr int K = fids_batch::kBatchSymStreams;
  bool need = false;
  for (fids_problem* h : b->members) need |= h->sym_hi < h->sh.M;
  if (!need) return FIDS_OK;
  if (!b->sstreams[0]) {
    for (int k = 0; k < K; ++k) HIPCHK(hipStreamCreateWithFlags(&b->sstreams[k], hipStreamNonBlocking));
    for (hipEvent_t& e : b->sev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(b->sev[K], b->stream));
  for (int k = 0; k < K; ++k) HIPCHK(hipStreamWaitEvent(b->sstreams[k], b->sev[K], 0));
  int k = 0, st = FIDS_OK;
  for (fids_problem* h : b->members) {
    if (h->sym_hi >= h->sh.M) continue;
    st = build_symbols(h, h->sh.M, b->sstreams[k]);
    if (st != FIDS_OK) break;
    k = (k + 1) % K;
  }
  // the batch stream waits for whatever was enqueued, also after a failure
  for (int j = 0; j < K; ++j) {
    HIPCHK(hipEventRecord(b->sev[j], b->sstreams[j]));
    HIPCHK(hipStreamWaitEvent(b->stream, b->sev[j], 0));
  }
  return st;
}

// Waits for a batch launch over levels [m0, m1] and folds the members' status
// words: the first failing member's status is returned; the batch level
// advances to m1 only if every member completed it.
int batch_finish(fids_batch* b, int m0, int m1) {
  std::vector<int> w(size_t(b->count) * 4);
  HIPCHK(hipMemcpyAsync(w.data(), b->dstatus, w.size() * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  int st = FIDS_OK;
  for (int32_t i = 0; i < b->count; ++i) {
    const int si = w[size_t(i) * 4], last = w[size_t(i) * 4 + 1];
    if (st == FIDS_OK && si != FIDS_OK) st = si;
    if (st == FIDS_OK && last != m1) st = FIDS_EDEVICE;
  }
  (void)m0;
  if (st == FIDS_OK) b->level = m1;
  else b->poisoned = true;
  return st;
}

// ------------------------------------------------ allocation-free entry point
// Workspace of fids_solve_static: a fixed device array in the library's code
// object, so the call allocates no device memory.  Each device the library
// runs on holds its own copy (kScratchBytes) from module load to process end.
// In host code `scratch` only names the symbol: its device address comes
// from hipGetSymbolAddress, once per device with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchSymBudget = size_t(4) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu[kMaxDevices];
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device; the caller holds g_scratch_mu[dev]).
int scratch_address(int dev, void** out) {
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign) return FIDS_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FIDS_OK;
}

}  // namespace

extern "C" {

int fids_solve_static(const fids_params* p, const double* kappa_d, const double* f_d, const double* phi_d,
                      double* uT_d, fids_step_info* per_step, void* hip_stream) {
  if (!p || !kappa_d || !f_d || !phi_d) return FIDS_EINVAL;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return FIDS_EINVAL;
  // one call at a time per device in this process: the array is shared
  std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
  void* ws = nullptr;
  int st = scratch_address(dev, &ws);
  if (st != FIDS_OK) return st;
  {
    Shapes sh;
    if (shapes_of(*p, sh, nullptr) != FIDS_OK) return FIDS_EINVAL;
    fids_params q = *p;
    if (q.history == FIDS_HISTORY_DIRECT) q.store_states = 1;
    const size_t need = make_layout(q, sh, kScratchSymBudget).total;
    if (need > kScratchBytes) {
      std::snprintf(g_last_error, sizeof(g_last_error),
                    "fids_solve_static: the problem needs %zu bytes of device memory, the static array holds %zu",
                    need, kScratchBytes);
      return FIDS_EINVAL;
    }
  }
  fids_problem* h = nullptr;
  // init clears the part of the array the problem uses (the last call's
  // contents are still there)
  st = init_impl(p, kappa_d, f_d, phi_d, ws, kScratchBytes, hip_stream, 0, &h, kScratchSymBudget, false);
  if (st != FIDS_OK) return st;
  st = run_levels(h, h->sh.M, per_step);
  if (st == FIDS_OK && uT_d) {
    if (hip_bad(fids::launch_to_natural(h->hp, h->dp, h->hp.u[h->sh.M % fids::kRing], uT_d, h->stream), __LINE__))
      st = FIDS_EDEVICE;
  }
  if (hip_bad(hipStreamSynchronize(h->stream), __LINE__) && st == FIDS_OK) st = FIDS_EDEVICE;
  delete h;
  return st;
}

int fids_params_default(fids_params* p) {
  if (!p) return FIDS_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->alpha = 1.5; p->gamma = 0.5; p->l = 1.0; p->T = 1.0;
  p->n = 255; p->M = 64; p->r = 3.0; p->mu = 0.0;
  p->soe_tol = 1e-10; p->krylov_tol = 1e-12; p->krylov_maxit = 200; p->restart = 20;
  p->solver = FIDS_BICGSTAB; p->precision = FIDS_FP64; p->precond = FIDS_STRANG;
  p->kappa_time_dependent = 1; p->x0_mode = 0; p->store_states = 0; p->wg_count = 0;
  p->soe_helpers = -1; p->checkpoint_every = 0; p->dims = 1;
  return FIDS_OK;
}

const char* fids_last_error(void) { return g_last_error; }

const char* fids_strerror(int s) {
  switch (s) {
    case FIDS_OK: return "ok";
    case FIDS_EINVAL: return "invalid argument";
    case FIDS_EDEVICE: return "HIP device error";
    case FIDS_ENOCONV: return "Krylov solver did not converge";
    case FIDS_ENUMERIC: return "non-finite value on the device";
    case FIDS_ESTATE: return "call not valid in the current state";
    default: return "unknown status";
  }
}

int fids_workspace_size(const fids_params* p, size_t* bytes) {
  if (!p || !bytes) return FIDS_EINVAL;
  Shapes sh;
  if (shapes_of(*p, sh, nullptr) != FIDS_OK) return FIDS_EINVAL;
  *bytes = make_layout(*p, sh).total;
  return FIDS_OK;
}

int fids_init_problem(const fids_params* p, const double* kappa_d, const double* f_d, const double* phi_d,
                      void* ws_d, size_t ws_bytes, void* hip_stream, fids_problem** out) {
  if (!p || !kappa_d || !f_d || !phi_d || !ws_d || !out) return FIDS_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws_d) % kAlign) return FIDS_EINVAL;
  *out = nullptr;
  return init_impl(p, kappa_d, f_d, phi_d, ws_d, ws_bytes, hip_stream, 0, out);
}

int fids_reset(fids_problem* h) {
  if (!h) return FIDS_EINVAL;
  HIPCHK(fids::launch_init_state(h->hp, h->dp, h->stream));
  HIPCHK(hipMemsetAsync(h->hp.F, 0, size_t(h->hp.nexp) * h->hp.vlen * 8, h->stream));
  HIPCHK(hipMemsetAsync(h->hp.H1, 0, size_t(2) * h->hp.vlen * 8, h->stream));
  HIPCHK(hipMemsetAsync(h->hp.sync2, 0, 4096, h->stream));
  HIPCHK(hipMemsetAsync(h->hp.hflag, 0, 4096 * 64, h->stream));
  HIPCHK(hipMemsetAsync(h->hp.status, 0, 4 * sizeof(int), h->stream));
  HIPCHK(hipMemsetAsync(h->hp.bar, 0, fids::kBarBytes, h->stream));
  if (h->symflag) HIPCHK(hipMemsetAsync(h->symflag, 0, sizeof(unsigned), h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->level = 0;
  h->poisoned = false;
  h->sym_hi = 0;  // every pass from level 0 rebuilds the per-level symbols it runs through
  return FIDS_OK;
}

int fids_prepare(fids_problem* h) {
  if (!h) return FIDS_EINVAL;
  const int st = ensure_symbols(h);
  if (st != FIDS_OK) return st;
  HIPCHK(hipStreamSynchronize(h->stream));
  return FIDS_OK;
}

int fids_destroy(fids_problem* h) {
  delete h;
  return FIDS_OK;
}

int fids_solve_levels(fids_problem* h, int64_t count, double* u_out_d, fids_step_info* per_step) {
  if (!h) return FIDS_EINVAL;
  if (h->level >= h->sh.M) return FIDS_ESTATE;
  if (count < 1 || count > h->sh.M - h->level) return FIDS_EINVAL;
  const int64_t m = h->level + count;
  const int st = run_levels(h, m, per_step);
  if (st != FIDS_OK) return st;
  if (u_out_d) {
    HIPCHK(fids::launch_to_natural(h->hp, h->dp, h->hp.u[m % fids::kRing], u_out_d, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return FIDS_OK;
}

int fids_step(fids_problem* h, double* u_out_d, fids_step_info* info) {
  if (!h) return FIDS_EINVAL;
  if (h->level >= h->sh.M) return FIDS_ESTATE;
  return fids_solve_levels(h, 1, u_out_d, info);
}

int fids_solve_all(fids_problem* h, double* uT_d, double* u_all_d, fids_step_info* per_step) {
  if (!h) return FIDS_EINVAL;
  if (u_all_d && !h->prm.store_states) return FIDS_EINVAL;
  if (h->level >= h->sh.M) return FIDS_ESTATE;
  const int64_t first = h->level + 1;
  const int st = run_levels(h, h->sh.M, per_step ? per_step + (first - 1) : nullptr);
  if (st != FIDS_OK) return st;
  if (uT_d) HIPCHK(fids::launch_to_natural(h->hp, h->dp, h->hp.u[h->sh.M % fids::kRing], uT_d, h->stream));
  if (u_all_d) HIPCHK(fids::launch_to_natural(h->hp, h->dp, h->hp.uhist, u_all_d, h->stream, h->sh.M + 1));
  HIPCHK(hipStreamSynchronize(h->stream));
  return FIDS_OK;
}

int fids_adjoint(fids_problem* h, const double* dJ_duT_d, double* g_kappa_d, double* g_f_d, double* g_phi_d) {
  if (!h || !dJ_duT_d) return FIDS_EINVAL;
  if (!h->dpa || h->poisoned || h->level != h->sh.M) return FIDS_ESTATE;
  int st = ensure_symbols(h);
  if (st != FIDS_OK) return st;
  const int M = int(h->sh.M);
  Prob& ha = h->ha;
  const size_t vb = size_t(ha.vlen) * 8;
  ha.g_kappa = (ha.kappa_td && g_kappa_d) ? g_kappa_d : nullptr;
  ha.g_f = g_f_d;
  HIPCHK(hipMemcpyAsync(h->dpa, &ha, sizeof(Prob), hipMemcpyHostToDevice, h->stream));
  for (int i = 0; i < 3; ++i) HIPCHK(hipMemsetAsync(ha.ubar[i], 0, vb, h->stream));
  for (int i = 0; i < fids::kRing; ++i) HIPCHK(hipMemsetAsync(ha.u[i], 0, vb, h->stream));
  HIPCHK(hipMemsetAsync(ha.F, 0, size_t(ha.nexp) * vb, h->stream));
  HIPCHK(hipMemsetAsync(ha.gk, 0, vb, h->stream));
  HIPCHK(hipMemsetAsync(ha.lam, 0, vb, h->stream));
  HIPCHK(hipMemsetAsync(ha.status, 0, 4 * sizeof(int), h->stream));
  HIPCHK(fids::launch_from_natural(ha, h->dpa, dJ_duT_d, ha.ubar[M % 3], h->stream));
  int stat[2] = {0, 0};
  if (h->prm.store_states) {
    st = launch_wait(h, ha, h->dpa, M, 1, 0, 0, stat);
    if (st != FIDS_OK) return st;
    if (stat[0] != FIDS_OK) return stat[0];
    if (stat[1] != 1) return FIDS_EDEVICE;
  } else {
    const int C = h->hp.ckpt_every;
    const int nseg = (M + C - 1) / C;
    for (int k = nseg - 1; k >= 0; --k) {
      const int a = k * C + 1, b = std::min((k + 1) * C, M);
      st = restore_segment(h, a);
      if (st != FIDS_OK) return st;
      int fst[2] = {0, 0};
      HIPCHK(hipMemsetAsync(h->hp.status, 0, 2 * sizeof(int), h->stream));
      st = launch_wait(h, h->hp, h->dp, a, b, a - 1, 0, fst);
      if (st != FIDS_OK) return st;
      h->level = fst[1];
      if (fst[0] != FIDS_OK || fst[1] != b) {
        h->poisoned = true;
        return fst[0] != FIDS_OK ? fst[0] : FIDS_EDEVICE;
      }
      st = launch_wait(h, ha, h->dpa, b, a, a - 1, 0, stat);
      if (st != FIDS_OK) return st;
      if (stat[0] != FIDS_OK) return stat[0];
      if (stat[1] != a) return FIDS_EDEVICE;
    }
  }
  if (g_phi_d) HIPCHK(fids::launch_to_natural(ha, h->dpa, ha.ubar[0], g_phi_d, h->stream));
  if (g_kappa_d && !ha.kappa_td) HIPCHK(fids::launch_to_natural(ha, h->dpa, ha.gk, g_kappa_d, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return FIDS_OK;
}

int fids_precond_symbol(fids_problem* h, int64_t m, double* q, double* qhat) {
  if (!h || m < 1 || m > h->sh.M) return FIDS_EINVAL;
  const int n = int(h->sh.n), Nc = int(h->sh.Nc);
  // level m's kbar and symbol alone, with the kernels the solves use (the
  // values are the same whichever batch of levels builds them)
  HIPCHK(fids::launch_kbar(h->hp.kappa, n, int(m), 1, h->prm.kappa_time_dependent, at<double>(h->ws, h->lo.kbar),
                           at<double>(h->ws, h->lo.kmax), h->stream));
  HIPCHK(fids::launch_symbols(h->hj, h->dj, int(m), 1, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (q) {
    if (h->hj.identity) {
      for (int i = 0; i < n; ++i) q[i] = i == 0 ? 1.0 : 0.0;
    } else {
      HIPCHK(hipMemcpy(q, h->hj.q, size_t(n) * sizeof(double), hipMemcpyDeviceToHost));
    }
  }
  if (qhat)
    HIPCHK(hipMemcpy(qhat, h->hp.qhat + size_t(m) * size_t(Nc + 1), size_t(Nc + 1) * sizeof(double),
                     hipMemcpyDeviceToHost));
  return FIDS_OK;
}

int fids_adjoint_report(const fids_problem* h, fids_step_info* per_step) {
  if (!h || !per_step) return FIDS_EINVAL;
  if (!h->dpa) return FIDS_ESTATE;
  HIPCHK(hipMemcpy(per_step, h->ha.info, size_t(h->sh.M) * sizeof(fids_step_info), hipMemcpyDeviceToHost));
  return FIDS_OK;
}

// ---------------------------------------------------------------- batched
int fids_batch_workspace_size(const fids_params* p, int32_t count, size_t* bytes) {
  if (!p || !bytes || count < 1) return FIDS_EINVAL;
  BatchLayout bl;
  const int st = batch_layout(p, count, bl);
  if (st != FIDS_OK) return st;
  *bytes = bl.total;
  return FIDS_OK;
}

int fids_batch_init(const fids_params* p, int32_t count, const double* const* kappa_d, const double* const* f_d,
                    const double* const* phi_d, void* ws_d, size_t ws_bytes, void* hip_stream, fids_batch** out) {
  if (!p || count < 1 || !kappa_d || !f_d || !phi_d || !ws_d || !out) return FIDS_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws_d) % kAlign) return FIDS_EINVAL;
  *out = nullptr;
  for (int32_t i = 0; i < count; ++i)
    if (!kappa_d[i] || !f_d[i] || !phi_d[i]) return FIDS_EINVAL;
  BatchLayout bl;
  if (batch_layout(p, count, bl) != FIDS_OK) return FIDS_EINVAL;
  if (ws_bytes < bl.total) return FIDS_EINVAL;
  fids_batch* b = new (std::nothrow) fids_batch();
  if (!b) return FIDS_EINVAL;
  b->bl = bl;
  b->count = count;
  b->M = p[0].M;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->ws = static_cast<char*>(ws_d);
  auto fail = [&](int code) { delete b; return code; };
  if (hip_bad(hipMemsetAsync(b->ws, 0, bl.head, b->stream), __LINE__)) return fail(FIDS_EDEVICE);
  b->dprobs = at<Prob>(b->ws, bl.probs);
  b->dstatus = at<int>(b->ws, bl.status);
  b->dinfo = at<fids_step_info>(b->ws, bl.info);
  b->dabort = at<int>(b->ws, bl.abort_);
  // costs, largest groups and an LDS bound (one-workgroup plans have the largest tiles)
  std::vector<double> cost;
  std::vector<int> kmax;
  size_t lds_bound = 0;
  Prob probe{};
  std::vector<double> prio;
  if (batch_costs(p, count, cost, kmax, &lds_bound, &probe, &prio) != FIDS_OK) return fail(FIDS_EINVAL);
  // graph mode: one workgroup per member, so that every level is an ordinary
  // launch a HIP graph can hold (a group of several workgroups needs a
  // cooperative launch)
  const char* mode = std::getenv("FIDS_BATCH_MODE");
  const bool want_graph = mode && std::strcmp(mode, "graph") == 0;
  if (want_graph) kmax.assign(size_t(count), 1);
  int resident = count;
  {
    int dev = 0, cus = 0, per_cu = 0;
    probe.adjoint = 0;
    if (lds_bound > 65536 && hip_bad(fids::set_level_lds_limit(probe, lds_bound), __LINE__)) return fail(FIDS_EDEVICE);
    if (hip_bad(hipGetDevice(&dev), __LINE__) ||
        hip_bad(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), __LINE__) ||
        hip_bad(fids::level_max_blocks(probe, lds_bound, &per_cu), __LINE__))
      return fail(FIDS_EDEVICE);
    resident = std::max(1, cus * per_cu);
  }
  const std::vector<Slot> slots = schedule_batch(cost, kmax, resident, &prio);
  b->hprobs.resize(size_t(count));
  b->members.assign(size_t(count), nullptr);
  b->groups.assign(size_t(count), 1);
  int g0 = 0, desc = 0;
  for (const Slot& sl : slots) {
    const int first = desc;
    for (int i : sl.members) {
      fids_problem* h = nullptr;
      const int st = init_impl(&p[i], kappa_d[i], f_d[i], phi_d[i], b->ws + bl.member[size_t(i)],
                               bl.member_bytes[size_t(i)], hip_stream, sl.ng, &h);
      if (st != FIDS_OK) return fail(st);
      b->members[size_t(i)] = h;
      b->groups[size_t(i)] = sl.ng;
      // status words and level reports of every member sit together in the batch header
      h->hp.status = b->dstatus + 4 * size_t(i);
      h->hp.info = b->dinfo + size_t(i) * size_t(b->M);
      h->dstatus = h->hp.status;
      h->hp.g0 = g0;
      h->hp.slot_first = first;
      b->hprobs[size_t(desc)] = h->hp;
      b->lds = std::max(b->lds, h->lds);
      if (upload(h, h->lo.prob, &h->hp, sizeof(Prob)) != FIDS_OK) return fail(FIDS_EDEVICE);
      ++desc;
    }
    g0 += sl.ng;
    if (sl.ng > 1) b->cooperative = true;
  }
  b->total_wg = g0;
  if (b->lds > 65536 && hip_bad(fids::set_level_lds_limit(b->hprobs[0], b->lds), __LINE__)) return fail(FIDS_EDEVICE);
  if (b->cooperative) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hip_bad(hipGetDevice(&dev), __LINE__) ||
        hip_bad(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), __LINE__) ||
        hip_bad(fids::level_max_blocks(b->hprobs[0], b->lds, &per_cu), __LINE__))
      return fail(FIDS_EDEVICE);
    if (cus * per_cu < b->total_wg) {
      std::snprintf(g_last_error, sizeof(g_last_error), "fids_api.cpp:%d: batch needs %d co-resident workgroups (%d fit)",
                    __LINE__, b->total_wg, cus * per_cu);
      return fail(FIDS_EDEVICE);
    }
    int rate_khz = 0;
    if (hip_bad(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev), __LINE__)) return fail(FIDS_EDEVICE);
    b->timeout_ticks = (unsigned long long)(std::max(rate_khz, 1000)) * 1000ull * 4ull;  // 4 s
  }
  if (hipMemcpyAsync(b->dprobs, b->hprobs.data(), size_t(count) * sizeof(Prob), hipMemcpyHostToDevice,
                     b->stream) != hipSuccess) {
    hip_bad(hipGetLastError(), __LINE__);
    return fail(FIDS_EDEVICE);
  }
  if (hip_bad(hipStreamSynchronize(b->stream), __LINE__)) return fail(FIDS_EDEVICE);
  b->graph_mode = want_graph && !b->cooperative;
  *out = b;
  return FIDS_OK;
}

int fids_batch_step(fids_batch* b, fids_step_info* info) {
  if (!b) return FIDS_EINVAL;
  if (b->level >= b->M || b->poisoned) return FIDS_ESTATE;
  int st = batch_symbols(b);
  if (st != FIDS_OK) return st;
  const int m = int(b->level + 1);
  HIPCHK(batch_launch(b, m, m, b->stream));
  st = batch_finish(b, m, m);
  if (info) {
    std::vector<fids_step_info> all(size_t(b->count) * size_t(b->M));
    HIPCHK(hipMemcpy(all.data(), b->dinfo, all.size() * sizeof(fids_step_info), hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < b->count; ++i) info[i] = all[size_t(i) * size_t(b->M) + size_t(m - 1)];
  }
  return st;
}

int fids_batch_solve_all(fids_batch* b, double* const* uT_d, fids_step_info* info) {
  if (!b) return FIDS_EINVAL;
  if (b->level >= b->M || b->poisoned) return FIDS_ESTATE;
  int st = batch_symbols(b);
  if (st != FIDS_OK) return st;
  const int m0 = int(b->level + 1), M = int(b->M);
  if (b->graph_mode) {
    // one graph node per level, captured once for a solve from level 1
    if (m0 == 1) {
      if (!b->graph_exec) {
        if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        for (int m = 1; m <= M; ++m)
          if (hip_bad(batch_launch(b, m, m, b->cap_stream), __LINE__)) {
            (void)hipStreamEndCapture(b->cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return FIDS_EDEVICE;
          }
        HIPCHK(hipStreamEndCapture(b->cap_stream, &g));
        const hipError_t e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (hip_bad(e, __LINE__)) { b->graph_exec = nullptr; return FIDS_EDEVICE; }
      }
      HIPCHK(hipGraphLaunch(b->graph_exec, b->stream));
    } else {
      for (int m = m0; m <= M; ++m)
        HIPCHK(batch_launch(b, m, m, b->stream));
    }
  } else {
    HIPCHK(batch_launch(b, m0, M, b->stream));
  }
  st = batch_finish(b, m0, M);
  if (info) HIPCHK(hipMemcpy(info, b->dinfo, size_t(b->count) * size_t(M) * sizeof(fids_step_info),
                             hipMemcpyDeviceToHost));
  if (st != FIDS_OK) return st;
  if (uT_d) {
    for (int32_t i = 0; i < b->count; ++i) {
      if (!uT_d[i]) continue;
      const fids_problem* h = b->members[size_t(i)];
      HIPCHK(fids::launch_to_natural(h->hp, h->dp, h->hp.u[M % fids::kRing], uT_d[i], b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
  }
  return FIDS_OK;
}

int fids_batch_solve_levels(fids_batch* b, int64_t count, double* const* u_d, fids_step_info* info) {
  if (!b) return FIDS_EINVAL;
  if (b->level >= b->M || b->poisoned) return FIDS_ESTATE;
  if (count < 1 || count > b->M - b->level) return FIDS_EINVAL;
  int st = batch_symbols(b);
  if (st != FIDS_OK) return st;
  const int m0 = int(b->level + 1), m1 = int(b->level + count);
  HIPCHK(batch_launch(b, m0, m1, b->stream));
  st = batch_finish(b, m0, m1);
  if (info) HIPCHK(hipMemcpy(info, b->dinfo, size_t(b->count) * size_t(b->M) * sizeof(fids_step_info),
                             hipMemcpyDeviceToHost));
  if (st != FIDS_OK) return st;
  if (u_d) {
    for (int32_t i = 0; i < b->count; ++i) {
      if (!u_d[i]) continue;
      const fids_problem* h = b->members[size_t(i)];
      HIPCHK(fids::launch_to_natural(h->hp, h->dp, h->hp.u[m1 % fids::kRing], u_d[i], b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
  }
  return FIDS_OK;
}

int fids_batch_prepare(fids_batch* b) {
  if (!b) return FIDS_EINVAL;
  const int st = batch_symbols(b);
  if (st != FIDS_OK) return st;
  HIPCHK(hipStreamSynchronize(b->stream));
  return FIDS_OK;
}

int fids_batch_status(const fids_batch* b, int32_t* status, int64_t* last_level) {
  if (!b || !status) return FIDS_EINVAL;
  std::vector<int> w(size_t(b->count) * 4);
  HIPCHK(hipMemcpy(w.data(), b->dstatus, w.size() * sizeof(int), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < b->count; ++i) {
    status[i] = w[size_t(i) * 4];
    if (last_level) last_level[i] = w[size_t(i) * 4 + 1];
  }
  return FIDS_OK;
}

int fids_batch_groups(const fids_batch* b, int32_t* ng) {
  if (!b || !ng) return FIDS_EINVAL;
  for (int32_t i = 0; i < b->count; ++i) ng[i] = b->groups[size_t(i)];
  return FIDS_OK;
}

int fids_batch_plan(const fids_params* p, int32_t count, int32_t resident, int32_t* ng, int32_t* slot,
                    double* makespan) {
  if (!p || count < 1 || resident < 1 || !ng || !slot) return FIDS_EINVAL;
  std::vector<double> cost;
  std::vector<int> kmax;
  std::vector<double> prio;
  if (batch_costs(p, count, cost, kmax, nullptr, nullptr, &prio) != FIDS_OK) return FIDS_EINVAL;
  const std::vector<Slot> slots = schedule_batch(cost, kmax, resident, &prio);
  double worst = 0.0;
  for (size_t k = 0; k < slots.size(); ++k) {
    double load = 0.0;
    for (int i : slots[k].members) {
      ng[i] = slots[k].ng;
      slot[i] = int32_t(k);
      load += group_cost(cost[size_t(i)], slots[k].ng);
    }
    worst = std::max(worst, load);
  }
  if (makespan) *makespan = worst;
  return FIDS_OK;
}

int fids_batch_tune(fids_batch* b, int32_t levels, int32_t* tile_ct) {
  if (!b || levels < 1) return FIDS_EINVAL;
  if (b->level != 0 || b->poisoned) return FIDS_ESTATE;
  const int lv = int(std::min<int64_t>(levels, b->M));
  int dev = 0, max_lds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
  {
    const int sst = batch_symbols(b);
    if (sst != FIDS_OK) return sst;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // classes of members with equal embedding length and group size
  std::map<std::pair<int, int>, std::vector<int>> classes;
  for (int32_t i = 0; i < b->count; ++i) classes[{b->members[size_t(i)]->hp.L, b->groups[size_t(i)]}].push_back(i);
  int st = FIDS_OK;
  for (auto& kv : classes) {
    const int ng = kv.first.second;
    fids_problem* rep_h = b->members[size_t(kv.second.front())];
    const Prob keep = rep_h->hp;
    const PlanShape base = rep_h->sh.pr;
    struct Cand { PlanShape ps; size_t lds; float ms; };
    std::vector<Cand> cands;
    for (int cap : {kTileCap, 2 * kTileCap})
      for (int mul : {1, 2, 4}) {
        PlanShape ps = plan_shape(base.Nc, ng * mul, ng, 0, cap);
        if (ps.N1 != base.N1 || ps.N2 != base.N2) continue;
        // the LDS need grows with each member's SOE node count: it must fit for all of the class
        size_t lds = 0;
        for (int i : kv.second) {
          Prob t = b->members[size_t(i)]->hp;
          t.pl.CT = ps.CT; t.pl.ntiles = ps.ntiles; t.pl.RU = ps.RU; t.pl.nrg = ps.nrg;
          lds = std::max(lds, fids::level_lds_bytes(t));
        }
        if (lds + 4096 > size_t(max_lds)) continue;   // room for the kernel's static LDS
        bool dup = false;
        for (const Cand& c : cands) dup |= (c.ps.CT == ps.CT && c.ps.RU == ps.RU);
        if (!dup) cands.push_back({ps, lds, 0.f});
      }
    for (Cand& c : cands) {
      // the representative alone, from level 0, on its group
      Prob trial = keep;
      trial.pl.CT = c.ps.CT; trial.pl.ntiles = c.ps.ntiles; trial.pl.RU = c.ps.RU; trial.pl.nrg = c.ps.nrg;
      trial.g0 = 0;
      trial.slot_first = 0;
      trial.status = keep.status;
      HIPCHK(hipMemcpy(rep_h->dp, &trial, sizeof(Prob), hipMemcpyHostToDevice));
      HIPCHK(fids::launch_init_state(trial, rep_h->dp, b->stream));
      HIPCHK(hipMemsetAsync(trial.F, 0, size_t(trial.nexp) * trial.vlen * 8, b->stream));
      HIPCHK(hipMemsetAsync(trial.AU, 0, size_t(fids::kRing) * trial.vlen * 8, b->stream));
      HIPCHK(hipMemsetAsync(trial.bar, 0, fids::kBarBytes, b->stream));
      if (c.lds > 65536) HIPCHK(fids::set_level_lds_limit(trial, c.lds));
      HIPCHK(hipEventRecord(e0, b->stream));
      if (ng > 1) {
        HIPCHK(hipMemsetAsync(b->dabort, 0, sizeof(int), b->stream));
        HIPCHK(fids::launch_levels(trial, rep_h->dp, 1, ng, c.lds, 1, lv, -1, 0, b->timeout_ticks, b->dabort,
                                   b->stream));
      } else {
        HIPCHK(fids::launch_levels_plain(trial, rep_h->dp, 1, 1, c.lds, 1, lv, b->stream));
      }
      HIPCHK(hipEventRecord(e1, b->stream));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipEventElapsedTime(&c.ms, e0, e1));
      int w[2] = {0, 0};
      HIPCHK(hipMemcpy(w, keep.status, sizeof(w), hipMemcpyDeviceToHost));
      if (w[0] != FIDS_OK) { st = w[0]; c.ms = 1e30f; }
    }
    size_t best = 0;
    for (size_t k = 1; k < cands.size(); ++k)
      if (cands[k].ms < cands[best].ms) best = k;
    for (int i : kv.second) {
      fids_problem* h = b->members[size_t(i)];
      h->hp.pl.CT = cands[best].ps.CT; h->hp.pl.ntiles = cands[best].ps.ntiles;
      h->hp.pl.RU = cands[best].ps.RU; h->hp.pl.nrg = cands[best].ps.nrg;
      h->lds = fids::level_lds_bytes(h->hp);
      if (tile_ct) tile_ct[i] = cands[best].ps.CT;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // descriptors in launch order, member copies, LDS limit
  b->lds = 0;
  for (size_t d = 0; d < b->hprobs.size(); ++d) {
    for (fids_problem* h : b->members) {
      if (h->hp.status == b->hprobs[d].status) {
        b->hprobs[d].pl = h->hp.pl;
        break;
      }
    }
  }
  for (fids_problem* h : b->members) {
    b->lds = std::max(b->lds, h->lds);
    HIPCHK(hipMemcpyAsync(h->dp, &h->hp, sizeof(Prob), hipMemcpyHostToDevice, b->stream));
  }
  if (b->lds > 65536) HIPCHK(fids::set_level_lds_limit(b->hprobs[0], b->lds));
  HIPCHK(hipMemcpyAsync(b->dprobs, b->hprobs.data(), b->hprobs.size() * sizeof(Prob), hipMemcpyHostToDevice,
                        b->stream));
  // a captured level graph holds the old tiling's launch shape and LDS size:
  // drop it so that the next solve captures the tuned one
  if (b->graph_exec) {
    HIPCHK(hipStreamSynchronize(b->stream));
    (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
  }
  const int rs = fids_batch_reset(b);
  return st != FIDS_OK ? st : rs;
}

int fids_batch_reset(fids_batch* b) {
  if (!b) return FIDS_EINVAL;
  for (fids_problem* h : b->members) {
    HIPCHK(fids::launch_init_state(h->hp, h->dp, b->stream));
    HIPCHK(hipMemsetAsync(h->hp.F, 0, size_t(h->hp.nexp) * h->hp.vlen * 8, b->stream));
    HIPCHK(hipMemsetAsync(h->hp.AU, 0, size_t(fids::kRing) * h->hp.vlen * 8, b->stream));
    HIPCHK(hipMemsetAsync(h->hp.bar, 0, fids::kBarBytes, b->stream));
    h->sym_hi = 0;
  }
  HIPCHK(hipMemsetAsync(b->dstatus, 0, size_t(b->count) * 4 * sizeof(int), b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  b->level = 0;
  b->poisoned = false;
  return FIDS_OK;
}

int fids_batch_destroy(fids_batch* b) {
  delete b;
  return FIDS_OK;
}

// ---------------------------------------------------------------- introspection
int fids_soe_nodes(double gamma, double delta, double T, double tol, int32_t cap, double* s, double* w,
                   int32_t* count) {
  if (!s || !w || !count) return FIDS_EINVAL;
  fids::SoeNodes q;
  if (fids::soe_build(gamma, delta, T, tol, q) != FIDS_OK) return FIDS_EINVAL;
  *count = int32_t(q.s.size());
  if (*count > cap) return FIDS_EINVAL;
  std::copy(q.s.begin(), q.s.end(), s);
  std::copy(q.w.begin(), q.w.end(), w);
  return FIDS_OK;
}

int fids_ifl_column(int64_t n, double alpha, double l, double mu, double* col) {
  if (!col || n < 1 || !(alpha > 0 && alpha < 2) || !(l > 0)) return FIDS_EINVAL;
  const double me = mu > 0 ? mu : 1 + alpha / 2;
  if (!(me > alpha && me <= 2)) return FIDS_EINVAL;
  const auto c = fids::ifl_column(n, alpha, l, me);
  std::copy(c.begin(), c.end(), col);
  return FIDS_OK;
}

int fids_ifl2d_mu(double alpha, double* mu) {
  if (!mu || !(alpha > 0 && alpha < 2)) return FIDS_EINVAL;
  *mu = fids::ifl2d_mu(alpha);
  return FIDS_OK;
}

int fids_ifl2d_coefficients(int64_t n, double alpha, double l, double mu, double* a) {
  if (!a || n < 1 || n > (int64_t(1) << 11) || !(alpha > 0 && alpha < 2) || !(l > 0)) return FIDS_EINVAL;
  if (mu != 0 && !(mu > alpha && mu < 2)) return FIDS_EINVAL;
  const double me = mu > 0 ? mu : fids::ifl2d_mu(alpha);
  const auto c = fids::ifl2d_coefficients(n, alpha, l, me);
  std::copy(c.begin(), c.end(), a);
  return FIDS_OK;
}

int fids_strang_eigs(int64_t n, double alpha, double l, double mu, double* lam) {
  if (!lam || n < 1 || !(alpha > 0 && alpha < 2) || !(l > 0)) return FIDS_EINVAL;
  const double me = mu > 0 ? mu : 1 + alpha / 2;
  if (!(me > alpha && me <= 2)) return FIDS_EINVAL;
  const auto e = fids::strang_eigs(fids::ifl_column(n, alpha, l, me));
  std::copy(e.begin(), e.end(), lam);
  return FIDS_OK;
}

int fids_direct_weights(double gamma, double T, int64_t M, double r, int64_t m, double* w) {
  if (!w || M < 1 || m < 1 || m > M || M > (int64_t(1) << 16) || !(gamma > 0 && gamma < 1) || !(T > 0) || !(r >= 1))
    return FIDS_EINVAL;
  const std::vector<double> all = fids::direct_history_weights(T, M, r, gamma);
  const double* row = all.data() + size_t(m - 1) * size_t(m) / 2;
  std::copy(row, row + m, w);
  return FIDS_OK;
}

int fids_level_coefficients(double gamma, double T, int64_t M, double r, double* beta) {
  if (!beta || M < 1 || !(gamma > 0 && gamma < 1) || !(T > 0) || !(r >= 1)) return FIDS_EINVAL;
  const auto tau = fids::step_sizes(T, M, r);
  const double g2 = std::tgamma(2.0 - gamma);
  for (int64_t m = 1; m <= M; ++m) beta[m - 1] = std::pow(tau[m], -gamma) / g2;
  return FIDS_OK;
}

}  // extern "C"
