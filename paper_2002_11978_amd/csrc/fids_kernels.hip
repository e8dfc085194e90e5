// gfx950 kernels of the fast implicit difference scheme.
//
// Per time level m (eq. 3.15 / matrix form 3.16gu) the device does:
//   1. the SOE history update F_j <- e^{-s_j tau_m} F_j + theta_{m,j} (u^{m-1} - u^{m-2})
//      and the right-hand side b = b_m' u^{m-1} - sum_j g w_j F_j + f^m
//      (b_m' = g a_m^{(m)}), one stream over F;
//   2. a Krylov solve of (b_m' I + K_m A) x = b, right-preconditioned by
//      Strang's circulant P_m = b_m' I + kbar_m s(A) (eq. 4.3), where A v and
//      P_m^{-1} v are products with symmetric Toeplitz matrices evaluated
//      through a length-L circulant embedding and real-packed FFTs.
// Every FFT is a two-pass (four-step) transform Nc = N1 * N2 with LDS-resident
// Stockham stages; the passes over columns (A: forward, C: inverse) carry the
// element-wise vector work of the solver, the pass over row pairs (B) applies
// the real symbol.  One persistent cooperative launch runs all levels; the
// workgroups of a problem meet at a group barrier between passes.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fids_device.h"
#include "fids_launch.h"

namespace fids {

// ------------------------------------------------------------- complex helpers
template <typename R> struct CxT;
template <> struct CxT<double> { using type = double2; };
template <> struct CxT<float> { using type = float2; };
template <typename R> using Cx = typename CxT<R>::type;

template <typename R> __device__ __forceinline__ Cx<R> mk(R x, R y) { Cx<R> c; c.x = x; c.y = y; return c; }
template <typename R> __device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R> __device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R> __device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename R> __device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {
  return mk<R>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename R> __device__ __forceinline__ Cx<R> cconj(Cx<R> a) { return mk<R>(a.x, -a.y); }
template <typename R> __device__ __forceinline__ Cx<R> cscale(Cx<R> a, R s) { return mk<R>(a.x * s, a.y * s); }

template <typename R> __device__ __forceinline__ const Cx<R>* tw_n1(const Plan& p);
template <> __device__ __forceinline__ const double2* tw_n1<double>(const Plan& p) { return p.tw1; }
template <> __device__ __forceinline__ const float2* tw_n1<float>(const Plan& p) { return p.tw1f; }
template <typename R> __device__ __forceinline__ const Cx<R>* tw_n2(const Plan& p);
template <> __device__ __forceinline__ const double2* tw_n2<double>(const Plan& p) { return p.tw2; }
template <> __device__ __forceinline__ const float2* tw_n2<float>(const Plan& p) { return p.tw2f; }

// W_root^j = e^{-2 pi i j / root} from the split table.
template <typename R> __device__ __forceinline__ Cx<R> tw_root(const Plan& p, unsigned j);
template <> __device__ __forceinline__ double2 tw_root<double>(const Plan& p, unsigned j) {
  return cmul<double>(p.twhi[j >> p.twshift], p.twlo[j & p.twmask]);
}
template <> __device__ __forceinline__ float2 tw_root<float>(const Plan& p, unsigned j) {
  return cmul<float>(p.twhif[j >> p.twshift], p.twlof[j & p.twmask]);
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// ------------------------------------------------------------- LDS FFT
// Self-sorting Stockham FFT of `count` sequences of length P stored back to
// back in LDS, ping-ponging between `src` and `dst` (radix-4 stages, then one
// radix-2 stage when log2 P is odd).  sign = -1: forward e^{-2 pi i jk/P};
// +1: inverse, unnormalised.  The caller synchronises before the call; the
// result pointer (src or dst) is returned after a final barrier.
template <typename R>
__device__ __forceinline__ Cx<R>* lds_fft(Cx<R>* src, Cx<R>* dst, int P, int logP, int count, int sign,
                                          const Cx<R>* tw) {
  int Ns = 1, logNs = 0;
  int rem = logP;
  while (rem > 0) {
    const int lr = rem >= 2 ? 2 : 1;
    const int lognb = logP - lr, nb = 1 << lognb;
    const int total = count << lognb;
    const int tstep = P >> (logNs + lr);
    if (lr == 2) {
      for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        const int c = idx >> lognb, j = idx & (nb - 1), k = j & (Ns - 1);
        const Cx<R>* s = src + c * P;
        Cx<R> a0 = s[j], a1 = s[j + nb], a2 = s[j + 2 * nb], a3 = s[j + 3 * nb];
        if (Ns > 1) {
          const int t = k * tstep;
          Cx<R> w1 = tw[t], w2 = tw[2 * t], w3 = tw[3 * t];
          if (sign > 0) { w1 = cconj<R>(w1); w2 = cconj<R>(w2); w3 = cconj<R>(w3); }
          a1 = cmul<R>(a1, w1); a2 = cmul<R>(a2, w2); a3 = cmul<R>(a3, w3);
        }
        const Cx<R> t0 = cadd<R>(a0, a2), t1 = csub<R>(a0, a2);
        const Cx<R> t2 = cadd<R>(a1, a3), t3 = csub<R>(a1, a3);
        const Cx<R> it3 = (sign < 0) ? mk<R>(t3.y, -t3.x) : mk<R>(-t3.y, t3.x);
        Cx<R>* d = dst + c * P + ((j - k) << 2) + k;
        d[0] = cadd<R>(t0, t2);
        d[Ns] = cadd<R>(t1, it3);
        d[2 * Ns] = csub<R>(t0, t2);
        d[3 * Ns] = csub<R>(t1, it3);
      }
    } else {
      for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        const int c = idx >> lognb, j = idx & (nb - 1), k = j & (Ns - 1);
        const Cx<R>* s = src + c * P;
        Cx<R> a0 = s[j], a1 = s[j + nb];
        if (Ns > 1) {
          Cx<R> w1 = tw[k * tstep];
          if (sign > 0) w1 = cconj<R>(w1);
          a1 = cmul<R>(a1, w1);
        }
        Cx<R>* d = dst + c * P + ((j - k) << 1) + k;
        d[0] = cadd<R>(a0, a1);
        d[Ns] = csub<R>(a0, a1);
      }
    }
    __syncthreads();
    Cx<R>* tmp = src; src = dst; dst = tmp;
    Ns <<= lr; logNs += lr; rem -= lr;
  }
  return src;
}

// ------------------------------------------------------------- passes
// Column pass A: buf holds CT columns (buf[c*N1 + n1] = z[N2*n1 + c0 + c]);
// forward N1-point FFTs, twiddle W_Nc^{n2 k1}, store T[k1*N2 + n2].
// buf has room for 2 * CT * N1 points (ping-pong).
template <typename R>
__device__ __forceinline__ void tileA_fft_store(const Plan& pl, int tile, Cx<R>* buf, Cx<R>* T) {
  __syncthreads();
  const Cx<R>* res = lds_fft<R>(buf, buf + pl.CT * pl.N1, pl.N1, pl.log1, pl.CT, -1, tw_n1<R>(pl));
  const int c0 = tile * pl.CT, logCT = ilog2(pl.CT);
  const int total = pl.CT * pl.N1;
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int c = idx & (pl.CT - 1), k1 = idx >> logCT;
    Cx<R> v = res[c * pl.N1 + k1];
    const unsigned e = unsigned((c0 + c) * k1) * unsigned(pl.rootmul);
    if (e) v = cmul<R>(v, tw_root<R>(pl, e));
    T[k1 * pl.N2 + c0 + c] = v;
  }
}

// Column pass C: load T[k1*N2 + n2] for the tile, inverse N1-point FFTs;
// afterwards buf[c*N1 + n1] = Nc * z'[N2*n1 + c0 + c] (the result is copied
// back into the first half of buf when the stage count is odd).
template <typename R>
__device__ __forceinline__ void tileC_load_ifft(const Plan& pl, int tile, const Cx<R>* T, Cx<R>* buf) {
  const int c0 = tile * pl.CT, logCT = ilog2(pl.CT);
  const int total = pl.CT * pl.N1;
  __syncthreads();
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int c = idx & (pl.CT - 1), k1 = idx >> logCT;
    buf[c * pl.N1 + k1] = T[k1 * pl.N2 + c0 + c];
  }
  __syncthreads();
  const Cx<R>* res = lds_fft<R>(buf, buf + total, pl.N1, pl.log1, pl.CT, +1, tw_n1<R>(pl));
  if (res != buf) {
    for (int idx = threadIdx.x; idx < total; idx += kThreads) buf[idx] = res[idx];
    __syncthreads();
  }
}

// Row pass B of a real-packed transform, one unit = rows (u, N1-u), or rows
// (0, N1/2) for u = 0.  Forward N2-point FFTs give Z[k1 + N1 k2]; each Z[k]
// is paired with Z[Nc-k] to split the spectrum X of the real length-L input,
//   X[k] = E + W_L^k O,  X[k+Nc] = E - W_L^k O,
//   E = (Z[k] + Z*[Nc-k])/2,  O = -i (Z[k] - Z*[Nc-k])/2.
// mode 0: multiply by the real even symbol S (S[k], S[Nc-k]), repack for the
// inverse, inverse N2-point FFTs, twiddle W_Nc^{-n2 k1}, store T.
// mode 1: write Re X[k] (k < Nc) and Re X[Nc] to spec / specf.
template <typename R, typename RS>
__device__ __forceinline__ void rowB_real(const Plan& pl, int unit, const Cx<R>* Tin, Cx<R>* Tout, const RS* S,
                          Cx<R>* buf, int mode, double* spec, float* specf) {
  const int N1 = pl.N1, N2 = pl.N2, Nc = pl.Nc;
  const int ka = unit, kb = (unit == 0) ? (N1 >> 1) : (N1 - unit);
  Cx<R>* b0 = buf;
  Cx<R>* b1 = buf + 2 * N2;
  __syncthreads();
  for (int idx = threadIdx.x; idx < 2 * N2; idx += kThreads) {
    const int r = idx >> pl.log2, n2 = idx & (N2 - 1);
    b0[idx] = Tin[(r ? kb : ka) * N2 + n2];
  }
  __syncthreads();
  {
    Cx<R>* res = lds_fft<R>(b0, b1, N2, pl.log2, 2, -1, tw_n2<R>(pl));
    if (res != b0) { b1 = b0; b0 = res; }   // b0: spectrum rows, b1: free
  }
  for (int idx = threadIdx.x; idx < 2 * N2; idx += kThreads) {
    const int r = idx >> pl.log2, k2 = idx & (N2 - 1);
    const int k1 = r ? kb : ka;
    const int k = k1 + N1 * k2;
    const int pr = (unit == 0) ? r : 1 - r;
    const int pk2 = (k1 == 0) ? ((N2 - k2) & (N2 - 1)) : (N2 - 1 - k2);
    const Cx<R> Zk = b0[idx];
    const Cx<R> Zt = cconj<R>(b0[pr * N2 + pk2]);
    const Cx<R> E = cscale<R>(cadd<R>(Zk, Zt), R(0.5));
    const Cx<R> D = csub<R>(Zk, Zt);
    const Cx<R> O = mk<R>(R(0.5) * D.y, R(-0.5) * D.x);
    const Cx<R> W = tw_root<R>(pl, unsigned(k));
    const Cx<R> WO = cmul<R>(W, O);
    const Cx<R> X0 = cadd<R>(E, WO), X1 = csub<R>(E, WO);
    if (mode == 0) {
      const R s0 = R(S[k]), s1 = R(S[Nc - k]);
      const Cx<R> Y0 = cscale<R>(X0, s0), Y1 = cscale<R>(X1, s1);
      const Cx<R> Ep = cscale<R>(cadd<R>(Y0, Y1), R(0.5));
      const Cx<R> Op = cscale<R>(cmulc<R>(csub<R>(Y0, Y1), W), R(0.5));
      b1[idx] = mk<R>(Ep.x - Op.y, Ep.y + Op.x);
    } else {
      if (spec) spec[k] = double(X0.x);
      if (specf) specf[k] = float(X0.x);
      if (k == 0) {
        if (spec) spec[Nc] = double(X1.x);
        if (specf) specf[Nc] = float(X1.x);
      }
    }
  }
  if (mode != 0) return;
  __syncthreads();
  const Cx<R>* res = lds_fft<R>(b1, b0, N2, pl.log2, 2, +1, tw_n2<R>(pl));
  for (int idx = threadIdx.x; idx < 2 * N2; idx += kThreads) {
    const int r = idx >> pl.log2, n2 = idx & (N2 - 1);
    const int k1 = r ? kb : ka;
    Cx<R> v = res[idx];
    const unsigned e = unsigned(n2 * k1) * unsigned(pl.rootmul);
    if (e) v = cmulc<R>(v, tw_root<R>(pl, e));
    Tout[k1 * N2 + n2] = v;
  }
}

// Row pass B of a complex transform: forward N2-point FFTs, multiply by the
// complex symbol Sc[k1 + N1 k2], inverse, twiddle, store.
__device__ __forceinline__ void rowB_complex(const Plan& pl, int unit, double2* T, const double2* Sc, double2* buf) {
  const int N1 = pl.N1, N2 = pl.N2;
  const int ka = unit, kb = (unit == 0) ? (N1 >> 1) : (N1 - unit);
  __syncthreads();
  for (int idx = threadIdx.x; idx < 2 * N2; idx += kThreads) {
    const int r = idx >> pl.log2, n2 = idx & (N2 - 1);
    buf[idx] = T[(r ? kb : ka) * N2 + n2];
  }
  __syncthreads();
  double2* res = lds_fft<double>(buf, buf + 2 * N2, N2, pl.log2, 2, -1, pl.tw2);
  double2* oth = (res == buf) ? buf + 2 * N2 : buf;
  for (int idx = threadIdx.x; idx < 2 * N2; idx += kThreads) {
    const int r = idx >> pl.log2, k2 = idx & (N2 - 1);
    const int k1 = r ? kb : ka;
    res[idx] = cmul<double>(res[idx], Sc[k1 + N1 * k2]);
  }
  __syncthreads();
  res = lds_fft<double>(res, oth, N2, pl.log2, 2, +1, pl.tw2);
  for (int idx = threadIdx.x; idx < 2 * N2; idx += kThreads) {
    const int r = idx >> pl.log2, n2 = idx & (N2 - 1);
    const int k1 = r ? kb : ka;
    double2 v = res[idx];
    const unsigned e = unsigned(n2 * k1) * unsigned(pl.rootmul);
    if (e) v = cmulc<double>(v, tw_root<double>(pl, e));
    T[k1 * N2 + n2] = v;
  }
}

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup of NV values per thread, same result in every
// thread; the summation order is fixed (deterministic).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[kThreads / 64][NV > 0 ? NV : 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wv][i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += red[w][i];
    v[i] = s;
  }
  __syncthreads();
}

// Reduce NV partial-sum slots (ntiles entries each) of a problem.
template <int NV>
__device__ __forceinline__ void reduce_slots(const Prob& p, const int (&slot)[NV], double (&out)[NV]) {
  const int nt = p.pl.ntiles;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0;
    for (int t = threadIdx.x; t < nt; t += kThreads) s += p.part[slot[i] * nt + t];
    out[i] = s;
  }
  block_sum<NV>(out);
}

template <int NV>
__device__ __forceinline__ void write_partials(const Prob& p, int tile, const int (&slot)[NV], double (&v)[NV]) {
  block_sum<NV>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) p.part[slot[i] * p.pl.ntiles + tile] = v[i];
}

// ------------------------------------------------------------- group barrier
// All workgroups of one problem meet here.  Thread 0 publishes the
// workgroup's writes (agent-scope release), arrives on a counter and waits for
// the generation to advance (agent-scope acquire).  A wall-clock timeout or an
// abort raised by another workgroup makes every waiter return false, so the
// launch always drains.
__device__ __forceinline__ bool group_barrier(const Prob& p, unsigned& gen, unsigned long long timeout,
                              int* abort_flag) {
  __shared__ int s_ok;
  __syncthreads();
  if (p.ng == 1) return true;
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    const unsigned g = gen;
    const unsigned prev = __hip_atomic_fetch_add(&p.bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == unsigned(p.ng - 1)) {
      __hip_atomic_store(&p.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&p.bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(&p.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
        if (wall_clock64() - t0 > timeout) {
          __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    gen = g + 1u;
    __threadfence();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// ------------------------------------------------------------- element helpers
struct TileIdx {
  int tile, c0, logCT, toff, total;
};
__device__ __forceinline__ TileIdx tile_idx(const Plan& pl, int tile) {
  TileIdx t;
  t.tile = tile;
  t.c0 = tile * pl.CT;
  t.logCT = ilog2(pl.CT);
  t.total = pl.CT * pl.N1;
  t.toff = tile * 2 * t.total;
  return t;
}

// item idx of a tile -> real index i0 = 2k (k = N2*n1 + c0 + c), LDS slot.
__device__ __forceinline__ void item(const Plan& pl, const TileIdx& t, int idx, int& i0, int& slot) {
  const int c = idx & (pl.CT - 1), n1 = idx >> t.logCT;
  i0 = 2 * (pl.N2 * n1 + t.c0 + c);
  slot = c * pl.N1 + n1;
}

__device__ __forceinline__ double2 ld2(const double* a, int off) { return *reinterpret_cast<const double2*>(a + off); }
__device__ __forceinline__ void st2(double* a, int off, double2 v) { *reinterpret_cast<double2*>(a + off) = v; }
__device__ __forceinline__ double2 nat2(const double* a, int i0, int n) {
  return make_double2(i0 < n ? a[i0] : 0.0, i0 + 1 < n ? a[i0 + 1] : 0.0);
}
__device__ __forceinline__ double2 mask2(double2 v, int i0, int n) {
  return make_double2(i0 < n ? v.x : 0.0, i0 + 1 < n ? v.y : 0.0);
}

// ------------------------------------------------------------- BiCGSTAB level
// Vector roles in Prob::vec for BiCGSTAB.
enum { VR = 0, VRH, VP, VV, VS, VT, VPH, VSH };

struct Ctl {
  unsigned gen;
  unsigned long long timeout;
  int* abort_flag;
};

#define BARRIER()                                                     \
  do {                                                                \
    if (!group_barrier(p, ctl.gen, ctl.timeout, ctl.abort_flag)) {    \
      return FIDS_EDEVICE;                                            \
    }                                                                 \
  } while (0)

__device__ __forceinline__ void write_info(const Prob& p, int rank, int m, int iters, int matvecs, double relres, int status) {
  if (rank == 0 && threadIdx.x == 0) {
    fids_step_info in;
    in.m = m;
    in.iters = iters;
    in.matvecs = matvecs;
    in.relres = relres;
    p.info[m - 1] = in;
    p.status[0] = status;
    if (status == FIDS_OK) p.status[1] = m;
  }
}

// SOE history update + right-hand side for level m, fused with the first
// column pass of P_m^{-1} applied to b (x0 = 0 so r = r^ = p = b).
__device__ __forceinline__ void phase_soe(const Prob& p, int m, int rank, double* lds_tab, double2* buf) {
  const Plan& pl = p.pl;
  const int nexp = p.nexp;
  // per-level SOE factors into LDS (shared by all tiles of this workgroup)
  double* th = lds_tab;
  double* de = lds_tab + nexp;
  double* gw = lds_tab + 2 * nexp;
  __syncthreads();
  for (int j = threadIdx.x; j < nexp; j += kThreads) {
    th[j] = p.theta[size_t(m) * nexp + j];
    de[j] = p.decay[size_t(m) * nexp + j];
    gw[j] = p.gw[j];
  }
  __syncthreads();
  const double bm = p.beta[m];
  const double* um1 = p.u[(m - 1) % 3];
  const double* um2 = p.u[(m + 1) % 3];  // (m-2) mod 3
  double* x = p.u[m % 3];
  const double* fm = p.f + size_t(m - 1) * p.n;
  const double* km = p.kappa + (p.kappa_td ? size_t(m - 1) * p.n : 0);
  const int blk = 2 * pl.CT * pl.N1;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    double acc[1] = {0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 b = make_double2(0.0, 0.0);
      if (i0 < p.n) {
        const double2 a1 = ld2(um1, off);
        double2 h = make_double2(0.0, 0.0);
        if (m >= 2) {
          const double2 a2 = ld2(um2, off);
          const double2 d = make_double2(a1.x - a2.x, a1.y - a2.y);
          double* Fp = p.F + size_t(tile) * nexp * blk + 2 * idx;
          for (int j = 0; j < nexp; ++j) {
            double2 fj = ld2(Fp, j * blk);
            fj.x = de[j] * fj.x + th[j] * d.x;
            fj.y = de[j] * fj.y + th[j] * d.y;
            st2(Fp, j * blk, fj);
            h.x += gw[j] * fj.x;
            h.y += gw[j] * fj.y;
          }
        }
        const double2 fv = nat2(fm, i0, p.n);
        b = mask2(make_double2(bm * a1.x - h.x + fv.x, bm * a1.y - h.y + fv.y), i0, p.n);
        st2(p.kap, off, nat2(km, i0, p.n));
        if (p.store_states) st2(p.uhist + size_t(m - 1) * p.vlen, off, a1);
      }
      st2(p.vec[VR], off, b);
      st2(p.vec[VRH], off, b);
      st2(p.vec[VP], off, b);
      st2(x, off, make_double2(0.0, 0.0));
      acc[0] += b.x * b.x + b.y * b.y;
      buf[sl] = b;
    }
    const int sl_bb[1] = {SL_BB};
    write_partials<1>(p, tile, sl_bb, acc);
    tileA_fft_store<double>(pl, tile, buf, p.T);
  }
}

// B pass with symbol S over all units of the problem.
template <typename RS>
__device__ __forceinline__ void phase_rows(const Prob& p, int rank, const RS* S, double2* buf) {
  for (int u = rank; u < p.pl.nunits; u += p.ng) rowB_real<double, RS>(p.pl, u, p.T, p.T, S, buf, 0, nullptr, nullptr);
}

// C pass of P^{-1}: z = crop(IFFT), store z into vec[dst], then A pass of A on z.
__device__ __forceinline__ void phase_C_then_A(const Prob& p, int rank, int dst, double2* buf) {
  const Plan& pl = p.pl;
  const double inv = 1.0 / double(pl.Nc);
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, buf);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const double2 z = mask2(cscale<double>(buf[sl], inv), i0, p.n);
      st2(p.vec[dst], t.toff + 2 * idx, z);
      buf[sl] = z;
    }
    tileA_fft_store<double>(pl, tile, buf, p.T);
  }
}

// C pass of A: y = A z;  out = b_m' z + kappa .* y;  partials of dots.
// which = 0: v = M p^, partial (r^, v).   which = 1: t = M s^, partials (t,s), (t,t), (r^,t).
__device__ __forceinline__ void phase_C_matvec(const Prob& p, int m, int rank, int which, double2* buf) {
  const Plan& pl = p.pl;
  const double inv = 1.0 / double(pl.Nc);
  const double bm = p.beta[m];
  const double* z = p.vec[which == 0 ? VPH : VSH];
  double* out = p.vec[which == 0 ? VV : VT];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, buf);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      if (i0 >= p.n) continue;
      const int off = t.toff + 2 * idx;
      const double2 y = cscale<double>(buf[sl], inv);
      const double2 zz = ld2(z, off), kk = ld2(p.kap, off);
      const double2 o = mask2(make_double2(bm * zz.x + kk.x * y.x, bm * zz.y + kk.y * y.y), i0, p.n);
      st2(out, off, o);
      const double2 rh = ld2(p.vec[VRH], off);
      if (which == 0) {
        acc[0] += rh.x * o.x + rh.y * o.y;
      } else {
        const double2 s = ld2(p.vec[VS], off);
        acc[0] += o.x * s.x + o.y * s.y;
        acc[1] += o.x * o.x + o.y * o.y;
        acc[2] += rh.x * o.x + rh.y * o.y;
      }
    }
    if (which == 0) {
      double a1[1] = {acc[0]};
      const int sl[1] = {SL_RV};
      write_partials<1>(p, tile, sl, a1);
    } else {
      const int sl[3] = {SL_TS, SL_TT, SL_RT};
      write_partials<3>(p, tile, sl, acc);
    }
  }
}

// s = r - alpha v; partials (s,s), (r^,s); A pass of P^{-1} on s.
__device__ __forceinline__ void phase_s(const Prob& p, int rank, double alpha, double2* buf) {
  const Plan& pl = p.pl;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    double acc[2] = {0.0, 0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 s = make_double2(0.0, 0.0);
      if (i0 < p.n) {
        const double2 r = ld2(p.vec[VR], off), v = ld2(p.vec[VV], off), rh = ld2(p.vec[VRH], off);
        s = mask2(make_double2(r.x - alpha * v.x, r.y - alpha * v.y), i0, p.n);
        st2(p.vec[VS], off, s);
        acc[0] += s.x * s.x + s.y * s.y;
        acc[1] += rh.x * s.x + rh.y * s.y;
      }
      buf[sl] = s;
    }
    const int sl[2] = {SL_SS, SL_RS};
    write_partials<2>(p, tile, sl, acc);
    tileA_fft_store<double>(pl, tile, buf, p.T);
  }
}

// x += alpha p^ + omega s^; r = s - omega t; p = r + beta (p - omega v);
// partial (r,r); A pass of P^{-1} on p.
__device__ __forceinline__ void phase_update(const Prob& p, int m, int rank, double alpha, double omega, double beta,
                             double2* buf) {
  const Plan& pl = p.pl;
  double* x = p.u[m % 3];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    double acc[1] = {0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 pn = make_double2(0.0, 0.0);
      if (i0 < p.n) {
        const double2 ph = ld2(p.vec[VPH], off), sh = ld2(p.vec[VSH], off);
        const double2 s = ld2(p.vec[VS], off), tt = ld2(p.vec[VT], off);
        const double2 po = ld2(p.vec[VP], off), v = ld2(p.vec[VV], off);
        double2 xx = ld2(x, off);
        xx.x += alpha * ph.x + omega * sh.x;
        xx.y += alpha * ph.y + omega * sh.y;
        st2(x, off, mask2(xx, i0, p.n));
        const double2 r = mask2(make_double2(s.x - omega * tt.x, s.y - omega * tt.y), i0, p.n);
        st2(p.vec[VR], off, r);
        pn = mask2(make_double2(r.x + beta * (po.x - omega * v.x), r.y + beta * (po.y - omega * v.y)), i0, p.n);
        st2(p.vec[VP], off, pn);
        acc[0] += r.x * r.x + r.y * r.y;
      }
      buf[sl] = pn;
    }
    const int sl[1] = {SL_RR};
    write_partials<1>(p, tile, sl, acc);
    tileA_fft_store<double>(pl, tile, buf, p.T);
  }
}

// x += alpha p^ (half-iteration exit).
__device__ __forceinline__ void phase_half(const Prob& p, int m, int rank, double alpha) {
  const Plan& pl = p.pl;
  double* x = p.u[m % 3];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      if (i0 >= p.n) continue;
      const int off = t.toff + 2 * idx;
      const double2 ph = ld2(p.vec[VPH], off);
      double2 xx = ld2(x, off);
      xx.x += alpha * ph.x;
      xx.y += alpha * ph.y;
      st2(x, off, mask2(xx, i0, p.n));
    }
  }
}

__device__ __forceinline__ bool bad(double v) { return !isfinite(v); }

// One level of FIDS with right-preconditioned BiCGSTAB (x0 = 0).
__device__ __forceinline__ int level_bicgstab(const Prob& p, int m, int rank, Ctl& ctl, double* lds_tab, double2* buf) {
  const size_t nsym = size_t(p.pl.Nc) + 1;
  const double* Q = p.qhat + size_t(m) * nsym;
  const double tol = p.tol;
  phase_soe(p, m, rank, lds_tab, buf);
  BARRIER();
  double red1[1];
  {
    const int sl[1] = {SL_BB};
    reduce_slots<1>(p, sl, red1);
  }
  const double bb = red1[0];
  if (bad(bb)) { write_info(p, rank, m, 0, 0, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
  const double bnorm = sqrt(bb);
  if (bb == 0.0) { write_info(p, rank, m, 0, 0, 0.0, FIDS_OK); return FIDS_OK; }
  double rho = bb, alpha = 0, omega = 0;
  int it = 0, mv = 0;
  for (;;) {
    phase_rows<double>(p, rank, Q, buf);                 // P^{-1} p
    BARRIER();
    phase_C_then_A(p, rank, VPH, buf);                   // p^ ; A p^ (column pass)
    BARRIER();
    phase_rows<double>(p, rank, p.ahat, buf);
    BARRIER();
    phase_C_matvec(p, m, rank, 0, buf);                  // v = M p^
    BARRIER();
    ++mv;
    {
      const int sl[1] = {SL_RV};
      reduce_slots<1>(p, sl, red1);
    }
    const double rv = red1[0];
    if (bad(rv)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
    if (rv == 0.0) { write_info(p, rank, m, it, mv, 1.0, FIDS_ENOCONV); return FIDS_ENOCONV; }
    alpha = rho / rv;
    phase_s(p, rank, alpha, buf);                        // s = r - alpha v ; P^{-1} s (column pass)
    BARRIER();
    double red2[2];
    {
      const int sl[2] = {SL_SS, SL_RS};
      reduce_slots<2>(p, sl, red2);
    }
    const double ss = red2[0], rs = red2[1];
    if (bad(ss)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
    if (sqrt(ss) <= tol * bnorm) {
      phase_half(p, m, rank, alpha);
      BARRIER();
      write_info(p, rank, m, it + 1, mv, sqrt(ss) / bnorm, FIDS_OK);
      return FIDS_OK;
    }
    phase_rows<double>(p, rank, Q, buf);
    BARRIER();
    phase_C_then_A(p, rank, VSH, buf);
    BARRIER();
    phase_rows<double>(p, rank, p.ahat, buf);
    BARRIER();
    phase_C_matvec(p, m, rank, 1, buf);                  // t = M s^
    BARRIER();
    ++mv;
    ++it;
    double red3[3];
    {
      const int sl[3] = {SL_TS, SL_TT, SL_RT};
      reduce_slots<3>(p, sl, red3);
    }
    const double ts = red3[0], tt = red3[1], rt = red3[2];
    if (bad(ts) || bad(tt)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
    if (tt == 0.0) { write_info(p, rank, m, it, mv, sqrt(ss) / bnorm, FIDS_ENOCONV); return FIDS_ENOCONV; }
    omega = ts / tt;
    const double rho_new = rs - omega * rt;
    if (omega == 0.0) { write_info(p, rank, m, it, mv, sqrt(ss) / bnorm, FIDS_ENOCONV); return FIDS_ENOCONV; }
    const double beta = (rho_new / rho) * (alpha / omega);
    phase_update(p, m, rank, alpha, omega, beta, buf);   // x, r, p ; P^{-1} p (column pass)
    BARRIER();
    {
      const int sl[1] = {SL_RR};
      reduce_slots<1>(p, sl, red1);
    }
    const double rr = red1[0];
    if (bad(rr)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
    if (sqrt(rr) <= tol * bnorm) { write_info(p, rank, m, it, mv, sqrt(rr) / bnorm, FIDS_OK); return FIDS_OK; }
    if (it >= p.maxit || rho_new == 0.0) {
      write_info(p, rank, m, it, mv, sqrt(rr) / bnorm, FIDS_ENOCONV);
      return FIDS_ENOCONV;
    }
    rho = rho_new;
  }
}

// ------------------------------------------------------------- level kernel
__global__ void __launch_bounds__(kThreads) k_levels(const Prob* probs, int nprob, int m_begin, int m_end,
                                                     unsigned long long timeout, int* abort_flag) {
  extern __shared__ double2 dyn[];
  // find this workgroup's problem
  int pid = 0;
  for (int q = 0; q < nprob; ++q)
    if (int(blockIdx.x) >= probs[q].g0) pid = q;
  const Prob& p = probs[pid];
  const int rank = int(blockIdx.x) - p.g0;
  if (rank < 0 || rank >= p.ng) return;
  double* lds_tab = reinterpret_cast<double*>(dyn);
  const int tab_c = (3 * p.nexp + 1) / 2;  // in double2 units
  double2* buf = dyn + tab_c;
  Ctl ctl;
  ctl.gen = 0;
  ctl.timeout = timeout;
  ctl.abort_flag = abort_flag;
  if (threadIdx.x == 0) ctl.gen = __hip_atomic_load(&p.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int m = m_begin; m <= m_end; ++m) {
    const int st = level_bicgstab(p, m, rank, ctl, lds_tab, buf);
    if (st != FIDS_OK) {
      if (rank == 0 && threadIdx.x == 0 && st == FIDS_EDEVICE) p.status[0] = FIDS_EDEVICE;
      return;
    }
  }
  // keep u^M with the stored states (tile-local copy, no barrier needed)
  if (p.store_states && m_end == p.M) {
    const double* uM = p.u[p.M % 3];
    for (int tile = rank; tile < p.pl.ntiles; tile += p.ng) {
      const TileIdx t = tile_idx(p.pl, tile);
      for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
        const int off = t.toff + 2 * idx;
        st2(p.uhist + size_t(p.M) * p.vlen, off, ld2(uM, off));
      }
    }
  }
}

// ------------------------------------------------------------- small kernels
__global__ void __launch_bounds__(kThreads) k_init_state(const Prob* pp) {
  const Prob& p = *pp;
  const Plan& pl = p.pl;
  const int tile = blockIdx.x;
  const TileIdx t = tile_idx(pl, tile);
  for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
    int i0, sl;
    item(pl, t, idx, i0, sl);
    const int off = t.toff + 2 * idx;
    const double2 v = nat2(p.phi, i0, p.n);
    st2(p.u[0], off, v);
    if (p.store_states) st2(p.uhist, off, v);
  }
}

__global__ void __launch_bounds__(kThreads) k_to_natural(const Prob* pp, const double* src, double* dst) {
  const Prob& p = *pp;
  const Plan& pl = p.pl;
  const int tile = blockIdx.x;
  const TileIdx t = tile_idx(pl, tile);
  for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
    int i0, sl;
    item(pl, t, idx, i0, sl);
    const double2 v = ld2(src, t.toff + 2 * idx);
    if (i0 < p.n) dst[i0] = v.x;
    if (i0 + 1 < p.n) dst[i0 + 1] = v.y;
  }
}

__global__ void __launch_bounds__(kThreads) k_kbar(const double* kappa, int n, int td, double* kbar) {
  const int m = blockIdx.x + 1;
  const double* row = kappa + (td ? size_t(m - 1) * n : 0);
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += kThreads) acc[0] += row[i];
  block_sum<1>(acc);
  if (threadIdx.x == 0) kbar[m] = acc[0] / double(n);
}

// Symbols, step 1: complex column pass of a_k = chirp_k / (b_m' + kbar_m lam_k).
__global__ void __launch_bounds__(kThreads) k_sym_a(const SymJob* jj, int m0) {
  extern __shared__ double2 dyn[];
  const SymJob& j = *jj;
  const Plan& pl = j.plc;
  const int m = m0 + blockIdx.y;
  const int tile = blockIdx.x;
  const double bm = j.beta[m], kb = j.kbar[m];
  double2* T = j.Tb + size_t(blockIdx.y) * j.L;
  const TileIdx t = tile_idx(pl, tile);
  for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
    const int c = idx & (pl.CT - 1), n1 = idx >> t.logCT;
    const int k = pl.N2 * n1 + t.c0 + c;
    double2 a = make_double2(0.0, 0.0);
    if (k < j.n) a = cscale<double>(j.chirp[k], 1.0 / (bm + kb * j.lam[k]));
    dyn[c * pl.N1 + n1] = a;
  }
  tileA_fft_store<double>(pl, tile, dyn, T);
}

// Symbols, step 2: multiply by the chirp spectrum (row pass).
__global__ void __launch_bounds__(kThreads) k_sym_b(const SymJob* jj) {
  extern __shared__ double2 dyn[];
  const SymJob& j = *jj;
  rowB_complex(j.plc, blockIdx.x, j.Tb + size_t(blockIdx.y) * j.L, j.chirp_hat, dyn);
}

// Symbols, step 3: inverse column pass, q_j = Re(chirp_j c_j) / (n L).
__global__ void __launch_bounds__(kThreads) k_sym_c(const SymJob* jj) {
  extern __shared__ double2 dyn[];
  const SymJob& j = *jj;
  const Plan& pl = j.plc;
  const int tile = blockIdx.x;
  const TileIdx t = tile_idx(pl, tile);
  tileC_load_ifft<double>(pl, tile, j.Tb + size_t(blockIdx.y) * j.L, dyn);
  double* q = j.q + size_t(blockIdx.y) * j.n;
  const double sc = 1.0 / (double(j.n) * double(j.L));
  for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
    const int c = idx & (pl.CT - 1), n1 = idx >> t.logCT;
    const int k = pl.N2 * n1 + t.c0 + c;
    if (k < j.n) q[k] = cmul<double>(j.chirp[k], dyn[c * pl.N1 + n1]).x * sc;
  }
}

// Symbols, step 4: real-packed column pass of the L-embedding of q.
__global__ void __launch_bounds__(kThreads) k_sym_d(const SymJob* jj) {
  extern __shared__ double2 dyn[];
  const SymJob& j = *jj;
  const Plan& pl = j.plr;
  const int tile = blockIdx.x;
  const TileIdx t = tile_idx(pl, tile);
  const double* q = j.q + size_t(blockIdx.y) * j.n;
  for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
    int i0, sl;
    item(pl, t, idx, i0, sl);
    double v[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = i0 + e;
      v[e] = (i < j.n) ? q[i] : ((i > j.L - j.n) ? q[j.L - i] : 0.0);
    }
    dyn[sl] = make_double2(v[0], v[1]);
  }
  tileA_fft_store<double>(pl, tile, dyn, j.Tq + size_t(blockIdx.y) * j.Nc);
}

// Symbols, step 5: row pass in spectrum mode -> qhat[m][0..Nc].
__global__ void __launch_bounds__(kThreads) k_sym_e(const SymJob* jj, int m0) {
  extern __shared__ double2 dyn[];
  const SymJob& j = *jj;
  const int m = m0 + blockIdx.y;
  const size_t ns = size_t(j.Nc) + 1;
  double2* T = j.Tq + size_t(blockIdx.y) * j.Nc;
  rowB_real<double, double>(j.plr, blockIdx.x, T, T, (const double*)nullptr, dyn, 1,
                            j.qhat ? j.qhat + size_t(m) * ns : nullptr,
                            j.qhatf ? j.qhatf + size_t(m) * ns : nullptr);
}

__global__ void __launch_bounds__(kThreads) k_sym_ones(const SymJob* jj, int m0) {
  const SymJob& j = *jj;
  const int m = m0 + blockIdx.y;
  const size_t ns = size_t(j.Nc) + 1;
  for (size_t k = size_t(blockIdx.x) * kThreads + threadIdx.x; k < ns; k += size_t(gridDim.x) * kThreads) {
    if (j.qhat) j.qhat[size_t(m) * ns + k] = 1.0;
    if (j.qhatf) j.qhatf[size_t(m) * ns + k] = 1.0f;
  }
}

// ------------------------------------------------------------- host launchers
static size_t plan_lds(const Plan& pl) {
  const size_t a = size_t(2) * pl.CT * pl.N1, b = size_t(4) * pl.N2;
  return (a > b ? a : b) * sizeof(double2);
}

size_t level_lds_bytes(const Prob& h) {
  const size_t tab = size_t((3 * h.nexp + 1) / 2) * sizeof(double2);
  return tab + plan_lds(h.pl);
}

hipError_t launch_init_state(const Prob& h, const Prob* d, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(h.pl.ntiles), dim3(kThreads), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_to_natural(const Prob& h, const Prob* d, const double* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_to_natural, dim3(h.pl.ntiles), dim3(kThreads), 0, s, d, src, dst);
  return hipGetLastError();
}

hipError_t launch_kbar(const double* kappa, int n, int M, int td, double* kbar, hipStream_t s) {
  hipLaunchKernelGGL(k_kbar, dim3(M), dim3(kThreads), 0, s, kappa, n, td, kbar);
  return hipGetLastError();
}

size_t symbols_lds_bytes(const SymJob& job) {
  const size_t lc = plan_lds(job.plc), lr = plan_lds(job.plr);
  return lc > lr ? lc : lr;
}

hipError_t launch_symbols(const SymJob& job, const SymJob* d, int m0, int cnt, hipStream_t s) {
  if (job.identity) {
    hipLaunchKernelGGL(k_sym_ones, dim3(64, cnt), dim3(kThreads), 0, s, d, m0);
    return hipGetLastError();
  }
  const size_t lc = plan_lds(job.plc), lr = plan_lds(job.plr);
  hipLaunchKernelGGL(k_sym_a, dim3(job.plc.ntiles, cnt), dim3(kThreads), lc, s, d, m0);
  hipLaunchKernelGGL(k_sym_b, dim3(job.plc.nunits, cnt), dim3(kThreads), lc, s, d);
  hipLaunchKernelGGL(k_sym_c, dim3(job.plc.ntiles, cnt), dim3(kThreads), lc, s, d);
  hipLaunchKernelGGL(k_sym_d, dim3(job.plr.ntiles, cnt), dim3(kThreads), lr, s, d);
  hipLaunchKernelGGL(k_sym_e, dim3(job.plr.nunits, cnt), dim3(kThreads), lr, s, d, m0);
  return hipGetLastError();
}

hipError_t launch_levels(const Prob* probs, int nprob, int total_wg, size_t lds_bytes, int m_begin,
                         int m_end, unsigned long long timeout_ticks, int* abort_flag, hipStream_t s) {
  void* args[] = {(void*)&probs, (void*)&nprob, (void*)&m_begin, (void*)&m_end, (void*)&timeout_ticks,
                  (void*)&abort_flag};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_levels), dim3(total_wg), dim3(kThreads),
                                    args, static_cast<unsigned int>(lds_bytes), s);
}

}  // namespace fids
