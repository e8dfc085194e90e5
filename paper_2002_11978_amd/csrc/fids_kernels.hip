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

#include <algorithm>
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
          // w^2 and w^3 from w: one twiddle read instead of three (the
          // transform is bound by LDS bandwidth; each product adds about an
          // ulp, measured 2.1e-16 against 1.7e-16 relative at 256 points)
          Cx<R> w1 = tw[k * tstep];
          if (sign > 0) w1 = cconj<R>(w1);
          const Cx<R> w2 = cmul<R>(w1, w1), w3 = cmul<R>(w2, w1);
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
  const int total = pl.CT * pl.N1;
  const Cx<R>* res = lds_fft<R>(buf, buf + total, pl.N1, pl.log1, pl.CT, -1, tw_n1<R>(pl));
  const int c0 = tile * pl.CT, logCT = ilog2(pl.CT);
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int c = idx & (pl.CT - 1), k1 = idx >> logCT;
    Cx<R> v = res[c * pl.N1 + k1];
    const unsigned e = unsigned((c0 + c) * k1) * unsigned(pl.rootmul);
    if (e) v = cmul<R>(v, tw_root<R>(pl, e));
    T[k1 * pl.N2 + c0 + c] = v;
  }
}

// Column pass C: load T[k1*N2 + n2] for the tile, inverse N1-point FFTs;
// afterwards buf[c*N1 + n1] = Nc * z'[N2*n1 + c0 + c].
template <typename R>
__device__ __forceinline__ void tileC_load_ifft(const Plan& pl, int tile, const Cx<R>* T, Cx<R>* buf) {
  const int c0 = tile * pl.CT, logCT = ilog2(pl.CT);
  const int total = pl.CT * pl.N1;
  __syncthreads();
  // kLoadBatch loads per thread in flight before their LDS stores (both are
  // generic pointers, so the compiler keeps a load behind an earlier store)
  for (int base = threadIdx.x; base < total; base += kLoadBatch * kThreads) {
    R vx[kLoadBatch], vy[kLoadBatch];
#pragma unroll
    for (int q = 0; q < kLoadBatch; ++q) {
      const int idx = min(base + q * kThreads, total - 1);   // in range; stored only below total
      const Cx<R> v = T[(idx >> logCT) * pl.N2 + c0 + (idx & (pl.CT - 1))];
      vx[q] = v.x;
      vy[q] = v.y;
    }
#pragma unroll
    for (int q = 0; q < kLoadBatch; ++q) {
      const int idx = base + q * kThreads;
      if (idx < total) buf[(idx & (pl.CT - 1)) * pl.N1 + (idx >> logCT)] = mk<R>(vx[q], vy[q]);
    }
  }
  __syncthreads();
  const Cx<R>* res = lds_fft<R>(buf, buf + total, pl.N1, pl.log1, pl.CT, +1, tw_n1<R>(pl));
  if (res != buf) {
    for (int idx = threadIdx.x; idx < total; idx += kThreads) buf[idx] = res[idx];
    __syncthreads();
  }
}

template <typename R, typename RS>
__device__ __forceinline__ void rowB_point(const Plan& pl, int idx, int u0, const Cx<R>* b0, Cx<R>* b1,
                                           const RS* S, R s0, R s1, bool have_s, int mode, double* spec,
                                           float* specf);
constexpr int kSymRegs = 4;   // kTileCap / kThreads

// row k1 of side s (0 or 1) of row-pair unit u: (u, N1-u), and (0, N1/2) for u = 0.
__device__ __forceinline__ int unit_row(const Plan& pl, int u, int side) {
  return side == 0 ? u : (u == 0 ? (pl.N1 >> 1) : pl.N1 - u);
}

// Row pass B of a real-packed transform over row group `grp` (RU units, 2 RU
// rows).  Forward N2-point FFTs give Z[k1 + N1 k2]; each Z[k] is paired with
// Z[Nc-k] (the other row of its unit) to split the spectrum X of the real
// length-L input,
//   X[k] = E + W_L^k O,  X[k+Nc] = E - W_L^k O,
//   E = (Z[k] + Z*[Nc-k])/2,  O = -i (Z[k] - Z*[Nc-k])/2.
// mode 0: multiply by the real even symbol S (S[k], S[Nc-k]), repack for the
// inverse, inverse N2-point FFTs, twiddle W_Nc^{-n2 k1}, store T.
// mode 1: write Re X[k] (k < Nc) and Re X[Nc] to spec / specf.
// buf has room for 4 RU N2 points.
template <typename R, typename RS>
__device__ __forceinline__ void rowB_real(const Plan& pl, int grp, const Cx<R>* Tin, Cx<R>* Tout, const RS* S,
                                          Cx<R>* buf, int mode, double* spec, float* specf) {
  const int N1 = pl.N1, N2 = pl.N2, Nc = pl.Nc;
  const int nrow = 2 * pl.RU, u0 = grp * pl.RU;
  const int tot = nrow * N2;
  Cx<R>* b0 = buf;
  Cx<R>* b1 = buf + tot;
  // the symbol values of this thread's points are fetched with the rows so
  // that their latency overlaps (at most kTileCap / kThreads points each)
  R sv0[kSymRegs], sv1[kSymRegs];
  __syncthreads();
#pragma unroll
  for (int b = 0; b < kSymRegs; ++b) {
    const int idx = threadIdx.x + b * kThreads;
    if (idx < tot) {
      const int q = idx >> pl.log2, n2 = idx & (N2 - 1);
      const int k1 = unit_row(pl, u0 + (q >> 1), q & 1);
      b0[idx] = Tin[k1 * N2 + n2];
      if (mode == 0) {
        const int k = k1 + N1 * n2;
        sv0[b] = R(S[k]);
        sv1[b] = R(S[Nc - k]);
      }
    }
  }
  for (int idx = threadIdx.x + kSymRegs * kThreads; idx < tot; idx += kThreads) {
    const int q = idx >> pl.log2, n2 = idx & (N2 - 1);
    b0[idx] = Tin[unit_row(pl, u0 + (q >> 1), q & 1) * N2 + n2];
  }
  __syncthreads();
  {
    Cx<R>* res = lds_fft<R>(b0, b1, N2, pl.log2, nrow, -1, tw_n2<R>(pl));
    if (res != b0) { b1 = b0; b0 = res; }   // b0: spectrum rows, b1: free
  }
#pragma unroll
  for (int b = 0; b < kSymRegs; ++b) {
    const int idx = threadIdx.x + b * kThreads;
    if (idx < tot) rowB_point<R, RS>(pl, idx, u0, b0, b1, S, sv0[b], sv1[b], true, mode, spec, specf);
  }
  for (int idx = threadIdx.x + kSymRegs * kThreads; idx < tot; idx += kThreads)
    rowB_point<R, RS>(pl, idx, u0, b0, b1, S, R(0), R(0), false, mode, spec, specf);
  if (mode != 0) return;
  __syncthreads();
  const Cx<R>* res = lds_fft<R>(b1, b0, N2, pl.log2, nrow, +1, tw_n2<R>(pl));
  for (int idx = threadIdx.x; idx < tot; idx += kThreads) {
    const int q = idx >> pl.log2, n2 = idx & (N2 - 1);
    const int k1 = unit_row(pl, u0 + (q >> 1), q & 1);
    Cx<R> v = res[idx];
    const unsigned e = unsigned(n2 * k1) * unsigned(pl.rootmul);
    if (e) v = cmulc<R>(v, tw_root<R>(pl, e));
    Tout[k1 * N2 + n2] = v;
  }
}

// One point of the row pass: split the spectrum, apply the symbol (mode 0)
// or write the real spectrum (mode 1).
template <typename R, typename RS>
__device__ __forceinline__ void rowB_point(const Plan& pl, int idx, int u0, const Cx<R>* b0, Cx<R>* b1,
                                           const RS* S, R s0, R s1, bool have_s, int mode, double* spec,
                                           float* specf) {
  const int N1 = pl.N1, N2 = pl.N2, Nc = pl.Nc;
  {
    const int q = idx >> pl.log2, k2 = idx & (N2 - 1);
    const int u = u0 + (q >> 1);
    const int k1 = unit_row(pl, u, q & 1);
    const int k = k1 + N1 * k2;
    const int pq = (u == 0) ? q : (q ^ 1);
    const int pk2 = (k1 == 0) ? ((N2 - k2) & (N2 - 1)) : (N2 - 1 - k2);
    const Cx<R> Zk = b0[idx];
    const Cx<R> Zt = cconj<R>(b0[pq * N2 + pk2]);
    const Cx<R> E = cscale<R>(cadd<R>(Zk, Zt), R(0.5));
    const Cx<R> D = csub<R>(Zk, Zt);
    const Cx<R> O = mk<R>(R(0.5) * D.y, R(-0.5) * D.x);
    const Cx<R> W = tw_root<R>(pl, unsigned(k));
    const Cx<R> WO = cmul<R>(W, O);
    const Cx<R> X0 = cadd<R>(E, WO), X1 = csub<R>(E, WO);
    if (mode == 0) {
      if (!have_s) { s0 = R(S[k]); s1 = R(S[Nc - k]); }
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
}

// Row pass B of a complex transform (row group of RU units): forward N2-point
// FFTs, multiply by the complex symbol Sc[k1 + N1 k2], inverse, twiddle, store.
__device__ __forceinline__ void rowB_complex(const Plan& pl, int grp, double2* T, const double2* Sc,
                                             double2* buf) {
  const int N1 = pl.N1, N2 = pl.N2;
  const int nrow = 2 * pl.RU, u0 = grp * pl.RU;
  const int tot = nrow * N2;
  __syncthreads();
  for (int idx = threadIdx.x; idx < tot; idx += kThreads) {
    const int q = idx >> pl.log2, n2 = idx & (N2 - 1);
    buf[idx] = T[unit_row(pl, u0 + (q >> 1), q & 1) * N2 + n2];
  }
  __syncthreads();
  double2* res = lds_fft<double>(buf, buf + tot, N2, pl.log2, nrow, -1, pl.tw2);
  double2* oth = (res == buf) ? buf + tot : buf;
  for (int idx = threadIdx.x; idx < tot; idx += kThreads) {
    const int q = idx >> pl.log2, k2 = idx & (N2 - 1);
    const int k1 = unit_row(pl, u0 + (q >> 1), q & 1);
    res[idx] = cmul<double>(res[idx], Sc[k1 + N1 * k2]);
  }
  __syncthreads();
  res = lds_fft<double>(res, oth, N2, pl.log2, nrow, +1, pl.tw2);
  for (int idx = threadIdx.x; idx < tot; idx += kThreads) {
    const int q = idx >> pl.log2, n2 = idx & (N2 - 1);
    const int k1 = unit_row(pl, u0 + (q >> 1), q & 1);
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

// Reduce `cnt` consecutive slots starting at `s0` into out[0..cnt) (LDS).
__device__ __forceinline__ void reduce_range(const Prob& p, int s0, int cnt, double* out) {
  const int nt = p.pl.ntiles;
  for (int b = 0; b < cnt; b += 8) {
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      double s = 0;
      if (b + i < cnt)
        for (int t = threadIdx.x; t < nt; t += kThreads) s += p.part[(s0 + b + i) * nt + t];
      v[i] = s;
    }
    block_sum<8>(v);
    if (threadIdx.x == 0)
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (b + i < cnt) out[b + i] = v[i];
  }
  __syncthreads();
}

template <int NV>
__device__ __forceinline__ void write_partials(const Prob& p, int tile, const int (&slot)[NV], double (&v)[NV]) {
  block_sum<NV>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) p.part[slot[i] * p.pl.ntiles + tile] = v[i];
}

// ------------------------------------------------------------- group barrier
// All workgroups of one problem meet here.  Every workgroup owns one 128-byte
// arrival slot holding the number of barriers it has reached.  Thread 0
// publishes the workgroup's writes with an agent-scope release fence and
// stores the new count into its own slot (a plain relaxed store: no
// read-modify-write, so arrivals do not queue behind one another on a shared
// counter); wave 0 then polls every slot of the group with relaxed loads, one
// per lane, until all have reached that count, and takes one acquire fence
// (on gfx950 every agent-scope acquire invalidates the caches, so polling
// with acquiring loads would do that on every probe).  Measured on MI355X
// with 64 workgroups exchanging 16 KiB each: 3.6 us per phase against 5.2 us
// for a counter with a generation word, 2.1 against 3.4 us with no data.
// The counts only grow, so a workgroup that has already moved on to the next
// barrier still satisfies the test of this one.  A wall-clock timeout or an
// abort raised by another workgroup makes every waiter return false, so the
// launch always drains.
__device__ __forceinline__ bool group_barrier(const Prob& p, int rank, unsigned& gen, unsigned long long timeout,
                                              int* abort_flag) {
  __shared__ int s_ok;
  __syncthreads();
  if (p.ng == 1) return true;
  const unsigned g = gen + 1u;
  gen = g;
  if (threadIdx.x < 64) {   // wave 0
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&p.bar[rank * kBarSlotWords], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    const unsigned long long t0 = wall_clock64();
    for (;;) {
      bool here = true;
      for (int i = threadIdx.x; i < p.ng; i += 64)
        here &= int(__hip_atomic_load(&p.bar[i * kBarSlotWords], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - g) >= 0;
      if (__all(here)) break;
      __builtin_amdgcn_s_sleep(1);
      // the decision to give up is lane 0's, taken by the whole wave
      int stop = 0;
      if (threadIdx.x == 0) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          stop = 1;
        } else if (wall_clock64() - t0 > timeout) {
          __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          stop = 1;
        }
      }
      if (__builtin_amdgcn_readfirstlane(stop)) { ok = 0; break; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) s_ok = ok;
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
// streaming (non-temporal) access for the SOE history, touched once per level
__device__ __forceinline__ double2 ld2nt(const double* a, size_t off) {
  return make_double2(__builtin_nontemporal_load(a + off), __builtin_nontemporal_load(a + off + 1));
}
__device__ __forceinline__ void st2nt(double* a, size_t off, double2 v) {
  __builtin_nontemporal_store(v.x, a + off);
  __builtin_nontemporal_store(v.y, a + off + 1);
}
__device__ __forceinline__ void st2(double* a, int off, double2 v) { *reinterpret_cast<double2*>(a + off) = v; }
// Element i of the solver's vectors is an unknown (not padding): i < n and,
// in 2-D, a node of its row (rows of stride S hold nx nodes).  S is even, so
// the pair (i0, i0 + 1) of an item never spans two rows: when i0 is padding,
// so is i0 + 1.
// Branch-free: 1-D has vmask 0 and vlim 1, so the row test always holds.
__device__ __forceinline__ bool valid_at(const Prob& p, int i) {
  return (i < p.n) & ((i & p.vmask) < p.vlim);
}
// index of unknown i in the caller's (natural) arrays: i, or i + nx j for the node (i, j) at i + S j
__device__ __forceinline__ int nat_at(const Prob& p, int i) {
  return p.vmask == 0 ? i : (i & p.vmask) + p.nx * (i >> p.lsx);
}
__device__ __forceinline__ double2 nat2(const double* a, int i0, const Prob& p) {
  return make_double2(valid_at(p, i0) ? a[nat_at(p, i0)] : 0.0, valid_at(p, i0 + 1) ? a[nat_at(p, i0 + 1)] : 0.0);
}
__device__ __forceinline__ double2 mask2(double2 v, int i0, const Prob& p) {
  return make_double2(valid_at(p, i0) ? v.x : 0.0, valid_at(p, i0 + 1) ? v.y : 0.0);
}
template <typename R> __device__ __forceinline__ Cx<R> tocx(double2 v) { return mk<R>(R(v.x), R(v.y)); }
// Input of a P^{-1} application: with the kappa-scaled preconditioner
// P = K_m C_m, P^{-1} v = C_m^{-1} K_m^{-1} v, and C_m^{-1} = kbar_m (b_m' I + kbar_m s(A))^{-1}
// reuses the Strang symbol, so v is scaled by kbar_m / kappa_i^m (dsc, tile-major).
// Conjugate gradients apply the same operator to the original residual r: the
// symmetrised system's residual is K_m^{-1} r and its preconditioner
// P^{(m)} / kbar_m, so z = kbar_m (b_m' I + kbar_m s(A))^{-1} K_m^{-1} r.
__device__ __forceinline__ bool kscaled(const Prob& p) {
  return p.precond == FIDS_STRANG_K || p.solver == FIDS_PCG;
}
__device__ __forceinline__ double2 pc_in(const Prob& p, int off, double2 v) {
  if (!kscaled(p)) return v;
  const double2 d = *reinterpret_cast<const double2*>(p.dsc + off);
  return make_double2(v.x * d.x, v.y * d.y);
}
template <typename R> __device__ __forceinline__ double2 fromcx(Cx<R> v) { return make_double2(double(v.x), double(v.y)); }

// views of the problem in the preconditioner precision R
template <typename R> __device__ __forceinline__ Cx<R>* pT(const Prob& p);
template <> __device__ __forceinline__ double2* pT<double>(const Prob& p) { return p.T; }
template <> __device__ __forceinline__ float2* pT<float>(const Prob& p) { return p.Tf; }
template <typename R> __device__ __forceinline__ const R* pQ(const Prob& p, int m);
template <> __device__ __forceinline__ const double* pQ<double>(const Prob& p, int m) {
  return p.qhat + size_t(m) * (p.pl.Nc + 1);
}
template <> __device__ __forceinline__ const float* pQ<float>(const Prob& p, int m) {
  return p.qhatf + size_t(m) * (p.pl.Nc + 1);
}
// FGMRES Z basis, stored in the preconditioner precision
template <typename R> __device__ __forceinline__ double2 z_get(const Prob& p, int i, int off);
template <> __device__ __forceinline__ double2 z_get<double>(const Prob& p, int i, int off) {
  return ld2(p.zd + size_t(i) * p.vlen, off);
}
template <> __device__ __forceinline__ double2 z_get<float>(const Prob& p, int i, int off) {
  const float2 v = *reinterpret_cast<const float2*>(p.zf + size_t(i) * p.vlen + off);
  return make_double2(double(v.x), double(v.y));
}
// store z and return the stored (rounded) value
template <typename R> __device__ __forceinline__ double2 z_put(const Prob& p, int i, int off, double2 v);
template <> __device__ __forceinline__ double2 z_put<double>(const Prob& p, int i, int off, double2 v) {
  st2(p.zd + size_t(i) * p.vlen, off, v);
  return v;
}
template <> __device__ __forceinline__ double2 z_put<float>(const Prob& p, int i, int off, double2 v) {
  const float2 f = make_float2(float(v.x), float(v.y));
  *reinterpret_cast<float2*>(p.zf + size_t(i) * p.vlen + off) = f;
  return make_double2(double(f.x), double(f.y));
}

// ------------------------------------------------------------- level state
// Vector roles in Prob::vec (VV doubles as the FGMRES vector w).
enum { VB = 0, VR, VRH, VP, VV, VS, VT, VPH, VSH };

struct Ctl {
  int rank;        // this workgroup's place in its problem's group
  unsigned gen;    // group barriers this workgroup has passed (its arrival slot)
  unsigned long long timeout;
  int* abort_flag;
  int hist_lo;     // >= 0: store u^k at uhist[k - hist_lo]; < 0: keep no states
  int ckpt_on;     // forward: write the segment snapshots
  int pending;     // adjoint: the kappa gradient of level m+1 waits in T
  unsigned sym_seen;  // symbols known to be built up to this level (Prob::symflag)
};

// FGMRES small state in LDS: hraw (J+1)J, R J*J, and 8 vectors of J+1.
constexpr int kSmallDoubles = ((kMaxRestart + 1) * kMaxRestart + kMaxRestart * kMaxRestart + 8 * (kMaxRestart + 1) + 1) / 2 * 2;

// LDS carve-up of the level kernel.
struct Lds {
  double* tab;      // 3 * nexp SOE factors
  double* small;    // FGMRES Hessenberg state
  double2* bd;      // FP64 tile / row buffer
  float2* bf;       // FP32 tile / row buffer
  Plan pl;          // the problem's plan with its twiddle tables copied to LDS
};
template <typename R> __device__ __forceinline__ Cx<R>* lbuf(const Lds& L);
template <> __device__ __forceinline__ double2* lbuf<double>(const Lds& L) { return L.bd; }
template <> __device__ __forceinline__ float2* lbuf<float>(const Lds& L) { return L.bf; }

#define BARRIER()                                                     \
  do {                                                                \
    if (!group_barrier(p, ctl.rank, ctl.gen, ctl.timeout, ctl.abort_flag)) { \
      return FIDS_EDEVICE;                                            \
    }                                                                 \
  } while (0)

__device__ __forceinline__ void write_info(const Prob& p, int rank, int m, int iters, int matvecs, double relres,
                                           int status, int fp64_iters = 0) {
  if (rank == 0 && threadIdx.x == 0) {
    fids_step_info in;
    in.m = m;
    in.iters = iters;
    in.matvecs = matvecs;
    in.relres = relres;
    in.pc_fp64_iters = fp64_iters;
    in.flags = (status == FIDS_OK && relres > p.tol) ? FIDS_LEVEL_ABOVE_TOL : 0;
    p.info[m - 1] = in;
    p.status[0] = status;
    if (status == FIDS_OK) p.status[1] = m;
  }
}

__device__ __forceinline__ bool bad(double v) { return !isfinite(v); }

// Rounding level of a true residual r = b - (b_m' x + kappa .* A x) formed in
// FP64, relative to ||b||: a circulant product through length-L transforms
// carries an error of about u log2(L) ||A|| ||x|| (u the unit roundoff, ||A||
// <= ||A||_inf), scaled by kappa <= kmax_m, plus u b_m' ||x|| from the shift
// and u ||b|| from the subtraction.  A level whose true residual stops
// improving above the tolerance is accepted only below
// max(kPcgSlack tol, this level); above it the level has not converged.
__device__ __forceinline__ double floor_bound(const Prob& p, int m, double xx, double bnorm) {
  constexpr double u = 1.1102230246251565e-16;   // 2^-53
  const double lg = double(31 - __clz(p.L));
  const double e = u * ((lg * p.kmax[m] * p.anorm + p.beta[m]) * sqrt(xx) / bnorm + 1.0);
  return fmax(kPcgSlack * p.tol, p.floor_scale * e);
}

// ------------------------------------------------------------- phases
// Wait until *addr >= target (thread 0 polls with relaxed loads, sleeping
// `nap` x 64 cycles between polls, then takes one agent-scope acquire fence,
// as in group_barrier); false on timeout, abort, or the solver group's stop
// flag.
template <int NAP>
__device__ __forceinline__ bool wait_ge(const Prob& p, const unsigned* addr, unsigned target, const Ctl& ctl) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(NAP);
      if (__hip_atomic_load(ctl.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          __hip_atomic_load(&p.status[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
      if (wall_clock64() - t0 > ctl.timeout) {
        __hip_atomic_store(ctl.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Waits until the symbol stream has built level m's symbol, kbar and kmax
// (Prob::symflag >= m; thread 0 polls with relaxed loads, then one acquire
// fence as in group_barrier) and remembers the level it saw, so that the
// levels of a chunk already built pass without a probe.  False on timeout,
// abort, or the solver group's stop flag.
__device__ __forceinline__ bool wait_symbols(const Prob& p, int m, Ctl& ctl) {
  __shared__ unsigned s_seen;
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    unsigned v;
    const unsigned long long t0 = wall_clock64();
    while ((v = __hip_atomic_load(p.symflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < unsigned(m)) {
      __builtin_amdgcn_s_sleep(8);
      if (__hip_atomic_load(ctl.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          __hip_atomic_load(&p.status[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
      if (wall_clock64() - t0 > ctl.timeout) {
        __hip_atomic_store(ctl.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_seen = v;
    s_ok = ok;
  }
  __syncthreads();
  ctl.sym_seen = s_seen;
  return s_ok != 0;
}

// Direct history, helper step k (concurrent with the solve of level k): the
// part of level k+1's sum that does not involve u^k,
//   S^{k+1} = sum_{j<k} w_{k+1,j} u^j,
// over chunks of j (partial c covers j in [k c / djc, k (c+1) / djc)) and
// element blocks of kThreads active items.  u^j for j <= k-2 was stored when
// level j+1 ran; u^{k-1} is still in the ring (its stored copy is written by
// level k concurrently).  The solver group adds the chunks and w_{k+1,k} u^k.
__device__ __forceinline__ void direct_helper_step(const Prob& p, int hr, int k) {
  const Plan& pl = p.pl;
  const int per_tile = p.dact * pl.CT;
  const int nact = pl.ntiles * per_tile;
  const int blk = 2 * pl.CT * pl.N1;
  const int logCT = ilog2(pl.CT);
  const double* wrow = p.dhw + size_t(k) * size_t(k + 1) / 2;
  double* P = p.dpart + size_t((k + 1) & 1) * size_t(p.djc) * p.vlen;
  const double* ulast = p.u[(k - 1) % kRing];
  const int units = p.dec * p.djc;
  for (int un = hr; un < units; un += p.nh) {
    const int eb = un % p.dec, c = un / p.dec;
    const int j0 = int(int64_t(k) * c / p.djc), j1 = int(int64_t(k) * (c + 1) / p.djc);
    const int a = eb * kThreads + threadIdx.x;
    if (a >= nact) continue;
    const int tile = a / per_tile, idx = a - tile * per_tile;
    const int i0 = 2 * (pl.N2 * (idx >> logCT) + tile * pl.CT + (idx & (pl.CT - 1)));
    if (!valid_at(p, i0)) continue;
    const int off = tile * blk + 2 * idx;
    const int js = min(j1, k - 1);
    double2 s = make_double2(0.0, 0.0);
    const double* up = p.uhist + size_t(j0) * p.vlen + off;
#pragma unroll 8
    for (int j = j0; j < js; ++j, up += p.vlen) {
      const double2 uj = *reinterpret_cast<const double2*>(up);
      s.x += wrow[j] * uj.x;
      s.y += wrow[j] * uj.y;
    }
    if (j1 == k) {
      const double2 uj = ld2(ulast, off);
      s.x += wrow[k - 1] * uj.x;
      s.y += wrow[k - 1] * uj.y;
    }
    st2(P + size_t(c) * p.vlen, off, s);
  }
}

// SOE helper workgroup `hr` of nh: for steps k = k0..k1 it advances the
// history F^{(k)} = e^{-s tau_k} F^{(k-1)} + theta_k (u^{k-1} - u^{k-2}) over its
// slice of the elements and forms the next level's history sum
// H1^{k+1} = sum_j g w_j e^{-s_j tau_{k+1}} F_j^{(k)}, so that level k+1 only needs
// h = H1^{k+1} + c_{k+1} (u^k - u^{k-1}) (the recurrence split exactly).  Step k
// starts once level k-1 is complete and every helper has finished step k-1;
// it runs concurrently with the solve of level k.
__device__ __forceinline__ int helper_loop(const Prob& p, int hr, int k0, int k1, const Ctl& ctl, double* tab) {
  const Plan& pl = p.pl;
  const int nexp = p.nexp;
  const int blk = 2 * pl.CT * pl.N1;
  const int npairs = p.vlen / 2;
  const int per = (npairs + p.nh - 1) / p.nh;
  const int q0 = hr * per, q1 = min(npairs, q0 + per);
  const int logCT = ilog2(pl.CT);
  double* th = tab;
  double* de = tab + nexp;
  double* dn = tab + 2 * nexp;
  unsigned* myflag = p.hflag + size_t(hr) * 64;
  for (int k = k0; k <= k1; ++k) {
    // helper 0 watches the solver group and the other helpers, then releases
    // each helper through its own flag line (few pollers per address)
    if (hr == 0) {
      if (!wait_ge<8>(p, &p.sync2[64], unsigned(k - 1), ctl)) return FIDS_EDEVICE;
      if (!wait_ge<8>(p, &p.sync2[0], unsigned(k - 2) * unsigned(p.nh), ctl)) return FIDS_EDEVICE;
      for (int h = threadIdx.x; h < p.nh; h += kThreads)
        __hip_atomic_store(p.hflag + size_t(h) * 64, unsigned(k), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else if (!wait_ge<127>(p, myflag, unsigned(k), ctl)) {
      return FIDS_EDEVICE;
    }
    if (p.history == FIDS_HISTORY_DIRECT) {
      direct_helper_step(p, hr, k);
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_fetch_add(&p.sync2[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    const bool next = k + 1 <= p.M;
    for (int j = threadIdx.x; j < nexp; j += kThreads) {
      th[j] = p.theta[size_t(k) * nexp + j];
      de[j] = p.decay[size_t(k) * nexp + j];
      dn[j] = next ? p.gw[j] * p.decay[size_t(k + 1) * nexp + j] : 0.0;
    }
    __syncthreads();
    const double* um1 = p.u[(k - 1) % kRing];
    const double* um2 = p.u[(k - 2 + kRing) % kRing];
    double* H = p.H1 + size_t((k + 1) & 1) * p.vlen;
    for (int q = q0 + threadIdx.x; q < q1; q += kThreads) {
      const int tile = (2 * q) / blk, lp = (2 * q) % blk;
      const int idx = lp >> 1;
      const int i0 = 2 * (pl.N2 * (idx >> logCT) + tile * pl.CT + (idx & (pl.CT - 1)));
      if (!valid_at(p, i0)) continue;
      const int off = 2 * q;
      const double2 a1 = ld2(um1, off), a2 = ld2(um2, off);
      const double2 d = make_double2(a1.x - a2.x, a1.y - a2.y);
      double* Fp = p.F + size_t(tile) * nexp * blk + lp;
      double2 h = make_double2(0.0, 0.0);
      for (int j = 0; j < nexp; ++j) {
        double2 fj = ld2nt(Fp, size_t(j) * blk);
        fj.x = de[j] * fj.x + th[j] * d.x;
        fj.y = de[j] * fj.y + th[j] * d.y;
        st2nt(Fp, size_t(j) * blk, fj);
        h.x += dn[j] * fj.x;
        h.y += dn[j] * fj.y;
      }
      if (next) st2(H, off, h);
    }
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&p.sync2[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  return FIDS_OK;
}

// Lagrange weights at v of polynomial extrapolation through npts earlier
// levels at distances d_k = v - v_k > 0 (k = 1..npts, nearest first):
// w_k = prod_{j != k} d_j / (d_j - d_k).  Forward and adjoint solves
// extrapolate in v = (t / T)^gamma (the adjoint backward in time).
__device__ __forceinline__ void extrap_weights(const double* d, int npts, double* w) {
  for (int k = 0; k < kRing; ++k) {
    double v = 0.0;
    if (k < npts) {
      v = 1.0;
      for (int j = 0; j < npts; ++j)
        if (j != k) v *= d[j] / (d[j] - d[k]);
    }
    w[k] = v;
  }
}

// Right-hand side of level m (eq. 3.16gu with the SOE history):
//   b = b_m' u^{m-1} - h^m + f^m,  h^m = sum_j g w_j F_j^{(m)};
// with helpers h^m = H1^m + c_m (u^{m-1} - u^{m-2}); without them the solver
// group advances F here.  kappa^m is copied tile-major.
// Initial guess x0 = 0, or polynomial extrapolation in v = (t / T)^gamma
// through the last x0_mode + 1 states (linear, quadratic, cubic; fewer near
// m = 1): the solution behaves like u^0 + c t^gamma near t = 0, linear in v.
// Then one of
//   fused (FGMRES, x0_mode >= 1, m >= 3): A x0 = sum_k w_k A u^{m-k} from the
//     stored products, r0 = b - b_m' x0 - kappa .* A x0, partials (b,b),
//     (r0,r0), column pass of P^{-1} on r0;
//   warm: column pass of A on x0 (the residual follows after the row pass);
//   cold: r0 = b (BiCGSTAB also r^ = p = b), column pass of P^{-1} on b.
template <typename RP>
__device__ __forceinline__ void phase_rhs(const Prob& p, int m, int rank, const Lds& L, bool fused,
                                          const Ctl& ctl) {
  const Plan& pl = L.pl;
  const int nexp = p.nexp;
  const bool self_soe = p.nh == 0;
  const bool direct = p.history == FIDS_HISTORY_DIRECT;
  const double* dw = direct ? p.dhw + size_t(m - 1) * size_t(m) / 2 : nullptr;
  double* th = L.tab;
  double* de = L.tab + nexp;
  double* gw = L.tab + 2 * nexp;
  if (self_soe) {
    __syncthreads();
    for (int j = threadIdx.x; j < nexp; j += kThreads) {
      th[j] = p.theta[size_t(m) * nexp + j];
      de[j] = p.decay[size_t(m) * nexp + j];
      gw[j] = p.gw[j];
    }
    __syncthreads();
  }
  const double bm = p.beta[m];
  const double cm = p.soec[m];
  // extrapolation coordinate v_m = (t_m / T)^gamma (linear through two levels: x0 = u^{m-1} + rho d)
  const double rho = (m >= 2) ? (p.xv[m] - p.xv[m - 1]) / (p.xv[m - 1] - p.xv[m - 2]) : 0.0;
  const bool warm = p.x0_mode != 0;
  const bool bicg = p.solver == FIDS_BICGSTAB;
  const double* um1 = p.u[(m - 1) % kRing];
  const double* um2 = p.u[(m - 2 + kRing) % kRing];
  double* x = p.u[m % kRing];              // holds u^{m-kRing} until x0 is stored
  const double* fm = p.f + size_t(m - 1) * p.nn;
  const double* km = p.kappa + (p.kappa_td ? size_t(m - 1) * p.nn : 0);
  const double* H1m = p.H1 + size_t(m & 1) * p.vlen;
  const bool kscale = kscaled(p);
  const double kb = kscale ? p.kbar[m] : 0.0;
  // extrapolation: npts earlier states u^{m-1}, ..., u^{m-npts} with weights w[]
  // (the fused residual also needs their stored A u^{m-k}, kept from level 1 on)
  const int npts = !warm ? 0 : min(p.x0_mode + 1, fused ? m - 1 : m);
  double w[kRing];
  {
    double d[kRing];
    for (int k = 0; k < kRing; ++k)
      d[k] = (m - 1 - k >= 0) ? p.xv[m] - p.xv[m - 1 - k] : 1.0;   // v_m - v_{m-1-k} (used for k < npts)
    extrap_weights(d, npts, w);
  }
  const int blk = 2 * pl.CT * pl.N1;
  // snapshot of the state entering level m = kC + 1 (k >= 1), taken while it
  // streams through this phase: u^{m-1..m-kRing}, A u^{m-1..m-kRing}, F^{(m-1)}
  const bool snap = ctl.ckpt_on && p.ckpt != nullptr && m >= 2 && (m - 1) % p.ckpt_every == 0;
  double* ck = snap ? p.ckpt + size_t((m - 1) / p.ckpt_every - 1) * size_t(nexp + 2 * kRing) * p.vlen : nullptr;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    double acc[3] = {0.0, 0.0, 0.0};   // (b,b), (r0,r0), kappa entries not > 0
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 b = make_double2(0.0, 0.0), x0 = make_double2(0.0, 0.0), r0 = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        const double2 a1 = ld2(um1, off);
        double2 h = make_double2(0.0, 0.0);
        double2 d = make_double2(0.0, 0.0);
        double2 dsum = make_double2(0.0, 0.0);   // direct scheme: sum_{k<m} w_k u^k
        if (direct) {
          dsum = make_double2(dw[m - 1] * a1.x, dw[m - 1] * a1.y);
          if (p.nh > 0 && m >= 3) {          // the helpers' chunks of sum_{k<m-1} w_k u^k
            const double* P = p.dpart + size_t(m & 1) * size_t(p.djc) * p.vlen + off;
            for (int c = 0; c < p.djc; ++c) {
              const double2 s = *reinterpret_cast<const double2*>(P + size_t(c) * p.vlen);
              dsum.x += s.x;
              dsum.y += s.y;
            }
          } else {
            for (int k = 0; k < m - 1; ++k) {
              const double2 uk = ld2(p.uhist + size_t(k) * p.vlen, off);
              dsum.x += dw[k] * uk.x;
              dsum.y += dw[k] * uk.y;
            }
          }
          if (m >= 2) {
            const double2 a2 = ld2(um2, off);
            d = make_double2(a1.x - a2.x, a1.y - a2.y);
          }
        } else if (m >= 2) {
          const double2 a2 = ld2(um2, off);
          if (snap)
            for (int k = 0; k < kRing; ++k) {
              st2(ck + size_t(k) * p.vlen, off, ld2(p.u[(m - 1 - k + 2 * kRing) % kRing], off));
              if (fused) st2(ck + size_t(kRing + k) * p.vlen, off, ld2(p.AU + size_t((m - 1 - k + 2 * kRing) % kRing) * p.vlen, off));
            }
          d = make_double2(a1.x - a2.x, a1.y - a2.y);
          if (self_soe) {
            double* Fp = p.F + size_t(tile) * nexp * blk + 2 * idx;
            double* Fc = snap ? ck + size_t(2 * kRing) * p.vlen + size_t(tile) * nexp * blk + 2 * idx : nullptr;
            // the loads of kSoeBatch nodes are issued together: a store to F_j
            // would otherwise hold back the load of F_{j+1} (same base
            // pointer), one memory round trip per node; same arithmetic order
            int j = 0;
            for (; j + kSoeBatch <= nexp; j += kSoeBatch) {
              double2 fb[kSoeBatch];
#pragma unroll
              for (int q = 0; q < kSoeBatch; ++q) fb[q] = ld2(Fp, (j + q) * blk);
#pragma unroll
              for (int q = 0; q < kSoeBatch; ++q) {
                double2 fj = fb[q];
                if (snap) st2(Fc, (j + q) * blk, fj);
                fj.x = de[j + q] * fj.x + th[j + q] * d.x;
                fj.y = de[j + q] * fj.y + th[j + q] * d.y;
                st2(Fp, (j + q) * blk, fj);
                h.x += gw[j + q] * fj.x;
                h.y += gw[j + q] * fj.y;
              }
            }
            for (; j < nexp; ++j) {
              double2 fj = ld2(Fp, j * blk);
              if (snap) st2(Fc, j * blk, fj);
              fj.x = de[j] * fj.x + th[j] * d.x;
              fj.y = de[j] * fj.y + th[j] * d.y;
              st2(Fp, j * blk, fj);
              h.x += gw[j] * fj.x;
              h.y += gw[j] * fj.y;
            }
          } else {
            h = make_double2(cm * d.x, cm * d.y);
            if (m >= 3) {
              const double2 hh = ld2(H1m, off);
              h.x += hh.x;
              h.y += hh.y;
            }
          }
        }
        const double2 fv = nat2(fm, i0, p);
        const double2 kk = nat2(km, i0, p);
        b = direct ? mask2(make_double2(dsum.x + fv.x, dsum.y + fv.y), i0, p)
                   : mask2(make_double2(bm * a1.x - h.x + fv.x, bm * a1.y - h.y + fv.y), i0, p);
        if (npts == 2) {
          x0 = mask2(make_double2(a1.x + rho * d.x, a1.y + rho * d.y), i0, p);
        } else if (npts > 0) {
          x0 = make_double2(0.0, 0.0);
          for (int k = 0; k < npts; ++k) {
            const double2 uk = ld2(p.u[(m - 1 - k + 2 * kRing) % kRing], off);
            x0.x += w[k] * uk.x;
            x0.y += w[k] * uk.y;
          }
          x0 = mask2(x0, i0, p);
        }
        if (fused) {
          double2 ax = make_double2(0.0, 0.0);
          if (npts == 2) {
            const double2 A1 = ld2(p.AU + size_t((m - 1) % kRing) * p.vlen, off);
            const double2 A2 = ld2(p.AU + size_t((m - 2 + kRing) % kRing) * p.vlen, off);
            ax = make_double2((1.0 + rho) * A1.x - rho * A2.x, (1.0 + rho) * A1.y - rho * A2.y);
          } else {
            for (int k = 0; k < npts; ++k) {
              const double2 Ak = ld2(p.AU + size_t((m - 1 - k + 2 * kRing) % kRing) * p.vlen, off);
              ax.x += w[k] * Ak.x;
              ax.y += w[k] * Ak.y;
            }
          }
          st2(p.AU + size_t(m % kRing) * p.vlen, off, mask2(ax, i0, p));
          r0 = mask2(make_double2(b.x - (bm * x0.x + kk.x * ax.x), b.y - (bm * x0.y + kk.y * ax.y)), i0, p);
        }
        st2(p.kap, off, kk);
        acc[2] += (kk.x > 0.0 ? 0.0 : 1.0) + (valid_at(p, i0 + 1) && !(kk.y > 0.0) ? 1.0 : 0.0);
        if (kscale) st2(p.dsc, off, mask2(make_double2(kb / kk.x, kb / kk.y), i0, p));
        if (ctl.hist_lo >= 0) st2(p.uhist + size_t(m - 1 - ctl.hist_lo) * p.vlen, off, a1);
      }
      st2(p.vec[VB], off, b);
      st2(x, off, x0);
      acc[0] += b.x * b.x + b.y * b.y;
      if (fused) {
        st2(p.vec[VR], off, r0);
        acc[1] += r0.x * r0.x + r0.y * r0.y;
        lbuf<RP>(L)[sl] = tocx<RP>(pc_in(p, off, r0));
      } else if (warm) {
        L.bd[sl] = x0;
      } else {
        st2(p.vec[VR], off, b);
        if (bicg) { st2(p.vec[VRH], off, b); st2(p.vec[VP], off, b); }
        lbuf<RP>(L)[sl] = tocx<RP>(pc_in(p, off, b));
      }
    }
    const int sls[3] = {SL_BB, SL_RR, SL_KB};
    write_partials<3>(p, tile, sls, acc);
    if (warm && !fused) tileA_fft_store<double>(pl, tile, L.bd, p.T);
    else tileA_fft_store<RP>(pl, tile, lbuf<RP>(L), pT<RP>(p));
  }
}

// Row pass of a symbol over all row groups of the problem.
template <typename R, typename RS>
__device__ __forceinline__ void phase_rows(const Prob& p, int rank, const RS* S, Cx<R>* T, Cx<R>* buf,
                                           const Lds& L) {
  for (int g = rank; g < L.pl.nrg; g += p.ng) rowB_real<R, RS>(L.pl, g, T, T, S, buf, 0, nullptr, nullptr);
}

// Residual r = b - (b_m' x + kappa .* A x) after the row pass of A on x;
// stores r (and r^ = p = r for BiCGSTAB) and A x (as A u^m), partial (r, r),
// then the column pass of P^{-1} on r.
template <typename RP>
__device__ __forceinline__ void phase_r0(const Prob& p, int m, int rank, const Lds& L) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  const double bm = p.beta[m];
  const double* x = p.u[m % kRing];
  double* Aum = p.AU + size_t(m % kRing) * p.vlen;   // A x is kept as A u^m
  const bool bicg = p.solver == FIDS_BICGSTAB;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, L.bd);
    double acc[2] = {0.0, 0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 r = make_double2(0.0, 0.0), y = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        y = mask2(cscale<double>(L.bd[sl], inv), i0, p);
        const double2 xx = ld2(x, off), kk = ld2(p.kap, off), b = ld2(p.vec[VB], off);
        r = mask2(make_double2(b.x - (bm * xx.x + kk.x * y.x), b.y - (bm * xx.y + kk.y * y.y)), i0, p);
        acc[1] += xx.x * xx.x + xx.y * xx.y;
      }
      st2(Aum, off, y);
      st2(p.vec[VR], off, r);
      if (bicg) { st2(p.vec[VRH], off, r); st2(p.vec[VP], off, r); }
      acc[0] += r.x * r.x + r.y * r.y;
      lbuf<RP>(L)[sl] = tocx<RP>(pc_in(p, off, r));
    }
    const int sl_rr[2] = {SL_RR, SL_XX};
    write_partials<2>(p, tile, sl_rr, acc);
    tileA_fft_store<RP>(pl, tile, lbuf<RP>(L), pT<RP>(p));
  }
}

// ------------------------------------------------------------- adjoint
// The transposed system of level m, (b_m' I + A K_m) lambda = ubar^m, equals
// K_m^{-1} (b_m' I + K_m A) K_m lambda = ubar^m, so it is solved as the forward
// system with right-hand side K_m ubar^m: y = (b_m' I + K_m A)^{-1} K_m ubar^m,
// lambda^m = y / kappa^m, with the forward preconditioner and solver.

// Finishes dJ/dkappa^{m+1} = -lambda^{m+1} .* A u^{m+1} from the buffer the
// column pass C just left (A u^{m+1} scaled by Nc): a row of the caller's
// [M][n] array for time-dependent kappa, else the tile-major running sum.
__device__ __forceinline__ void adj_grad_item(const Prob& p, int mg, int i0, int off, double2 y) {
  const double2 lm = ld2(p.lam, off);
  const double2 g = make_double2(-lm.x * y.x, -lm.y * y.y);
  if (p.kappa_td) {
    if (p.g_kappa) {
      double* row = p.g_kappa + size_t(mg - 1) * p.nn;
      row[nat_at(p, i0)] = g.x;
      if (valid_at(p, i0 + 1)) row[nat_at(p, i0 + 1)] = g.y;
    }
  } else {
    const double2 a = ld2(p.gk, off);
    st2(p.gk, off, mask2(make_double2(a.x + g.x, a.y + g.y), i0, p));
  }
}

// Right-hand side of adjoint level m: b = kappa^m .* ubar^m, initial guess 0 or
// the extrapolation y^{m+1} + rho (y^{m+1} - y^{m+2}), rho = tau_{m+1}/tau_{m+2}
// (x0_mode 1), or the quadratic one through y^{m+3}, y^{m+2}, y^{m+1}
// (x0_mode 2, m + 3 <= M); then the column pass of A on x0 (warm) or of P^{-1}
// on b (cold).  First the pending gradient of level m+1 (column pass C of
// A u^{m+1}).
template <typename RP>
__device__ __forceinline__ void phase_adj_rhs(const Prob& p, int m, int rank, const Lds& L, const Ctl& ctl) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  const bool warm = p.x0_mode != 0;
  const bool bicg = p.solver == FIDS_BICGSTAB;
  const double* ub = p.ubar[m % 3];
  const double* y1 = p.u[(m + 1) % kRing];
  const double* y2 = p.u[(m + 2) % kRing];
  double* x = p.u[m % kRing];
  const double rho = (m + 2 <= p.M) ? (p.xv[m + 1] - p.xv[m]) / (p.xv[m + 2] - p.xv[m + 1]) : 0.0;
  // backward in time: y^{m+1}, ..., y^{m+npts} at distances v_{m+k} - v_m
  const int npts = !warm ? 0 : min(p.x0_mode + 1, p.M - m);
  double w[kRing];
  {
    double d[kRing];
    for (int k = 0; k < kRing; ++k) d[k] = (m + 1 + k <= p.M) ? p.xv[m + 1 + k] - p.xv[m] : 1.0;
    extrap_weights(d, npts, w);
  }
  const double* km = p.kappa + (p.kappa_td ? size_t(m - 1) * p.nn : 0);
  const bool kscale = kscaled(p);
  const double kb = kscale ? p.kbar[m] : 0.0;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    if (ctl.pending) tileC_load_ifft<double>(pl, tile, p.T, L.bd);
    double acc[2] = {0.0, 0.0};   // (b,b), kappa entries not > 0
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 b = make_double2(0.0, 0.0), x0 = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        if (ctl.pending) adj_grad_item(p, m + 1, i0, off, cscale<double>(L.bd[sl], inv));
        const double2 kk = nat2(km, i0, p);
        const double2 u = ld2(ub, off);
        b = mask2(make_double2(kk.x * u.x, kk.y * u.y), i0, p);
        if (npts == 2) {
          const double2 a1 = ld2(y1, off), a2 = ld2(y2, off);
          x0 = mask2(make_double2(a1.x + rho * (a1.x - a2.x), a1.y + rho * (a1.y - a2.y)), i0, p);
        } else if (npts > 0) {
          for (int k = 0; k < npts; ++k) {
            const double2 yk = ld2(p.u[(m + 1 + k) % kRing], off);   // y^{m+kRing} sits in x
            x0.x += w[k] * yk.x;
            x0.y += w[k] * yk.y;
          }
          x0 = mask2(x0, i0, p);
        }
        st2(p.kap, off, kk);
        acc[1] += (kk.x > 0.0 ? 0.0 : 1.0) + (valid_at(p, i0 + 1) && !(kk.y > 0.0) ? 1.0 : 0.0);
        if (kscale) st2(p.dsc, off, mask2(make_double2(kb / kk.x, kb / kk.y), i0, p));
      }
      st2(p.vec[VB], off, b);
      st2(x, off, x0);
      acc[0] += b.x * b.x + b.y * b.y;
      if (warm) {
        L.bd[sl] = x0;
      } else {
        st2(p.vec[VR], off, b);
        if (bicg) { st2(p.vec[VRH], off, b); st2(p.vec[VP], off, b); }
        lbuf<RP>(L)[sl] = tocx<RP>(pc_in(p, off, b));
      }
    }
    const int sls[2] = {SL_BB, SL_KB};
    write_partials<2>(p, tile, sls, acc);
    if (warm) tileA_fft_store<double>(pl, tile, L.bd, p.T);
    else tileA_fft_store<RP>(pl, tile, lbuf<RP>(L), pT<RP>(p));
  }
}

// After the solve of adjoint level m (y^m in u[m % kRing]):
//   lambda = y / kappa^m;  dJ/df^m = lambda;  ubar^{m-1} += b_m' lambda;
// the history recurrence in reverse (m >= 2; F^{(1)} = 0 has no inputs):
//   Fbar_j -= g w_j lambda;  rho = sum_j theta_{m,j} Fbar_j;  Fbar_j *= e^{-s_j tau_m};
//   ubar^{m-1} += rho;  ubar^{m-2} = -rho  (its first contribution);
// then the column pass of A on the forward state u^m.
__device__ __forceinline__ void phase_adj_post(const Prob& p, int m, int rank, const Lds& L, const Ctl& ctl) {
  const Plan& pl = L.pl;
  const int nexp = p.nexp;
  double* th = L.tab;
  double* de = L.tab + nexp;
  double* gw = L.tab + 2 * nexp;
  __syncthreads();
  for (int j = threadIdx.x; j < nexp; j += kThreads) {
    th[j] = p.theta[size_t(m) * nexp + j];
    de[j] = p.decay[size_t(m) * nexp + j];
    gw[j] = p.gw[j];
  }
  __syncthreads();
  const double bm = p.beta[m];
  const double* y = p.u[m % kRing];
  double* u1 = p.ubar[(m - 1) % 3];
  double* u2 = p.ubar[(m + 1) % 3];   // (m-2) mod 3
  const double* um = p.uhist + size_t(m - ctl.hist_lo) * p.vlen;
  double* gf = p.g_f ? p.g_f + size_t(m - 1) * p.nn : nullptr;
  const int blk = 2 * pl.CT * pl.N1;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 uv = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        const double2 yy = ld2(y, off), kk = ld2(p.kap, off);
        const double2 lm = make_double2(yy.x / kk.x, valid_at(p, i0 + 1) ? yy.y / kk.y : 0.0);
        st2(p.lam, off, lm);
        if (gf) {
          gf[nat_at(p, i0)] = lm.x;
          if (valid_at(p, i0 + 1)) gf[nat_at(p, i0 + 1)] = lm.y;
        }
        double2 a = ld2(u1, off);
        a.x += bm * lm.x;
        a.y += bm * lm.y;
        if (m >= 2) {
          double* Fp = p.F + size_t(tile) * nexp * blk + 2 * idx;
          double2 r = make_double2(0.0, 0.0);
          int j = 0;
          for (; j + kSoeBatch <= nexp; j += kSoeBatch) {   // loads issued together (see phase_rhs)
            double2 fv[kSoeBatch];
#pragma unroll
            for (int q = 0; q < kSoeBatch; ++q) fv[q] = ld2(Fp, (j + q) * blk);
#pragma unroll
            for (int q = 0; q < kSoeBatch; ++q) {
              double2 fb = fv[q];
              fb.x -= gw[j + q] * lm.x;
              fb.y -= gw[j + q] * lm.y;
              r.x += th[j + q] * fb.x;
              r.y += th[j + q] * fb.y;
              fb.x *= de[j + q];
              fb.y *= de[j + q];
              st2(Fp, (j + q) * blk, fb);
            }
          }
          for (; j < nexp; ++j) {
            double2 fb = ld2(Fp, j * blk);
            fb.x -= gw[j] * lm.x;
            fb.y -= gw[j] * lm.y;
            r.x += th[j] * fb.x;
            r.y += th[j] * fb.y;
            fb.x *= de[j];
            fb.y *= de[j];
            st2(Fp, j * blk, fb);
          }
          a.x += r.x;
          a.y += r.y;
          st2(u2, off, mask2(make_double2(-r.x, -r.y), i0, p));
        }
        st2(u1, off, mask2(a, i0, p));
        uv = mask2(ld2(um, off), i0, p);
      }
      L.bd[sl] = uv;
    }
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// Column pass C of A u^m after the last level of an adjoint launch: the
// gradient of that level (no level follows in this launch to absorb it).
__device__ __forceinline__ void phase_adj_flush(const Prob& p, int m, int rank, const Lds& L) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, L.bd);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      if (valid_at(p, i0)) adj_grad_item(p, m, i0, t.toff + 2 * idx, cscale<double>(L.bd[sl], inv));
    }
  }
}

// ------------------------------------------------------------- BiCGSTAB
// C pass of P^{-1}: z = crop(IFFT), store z into vec[dst], then A pass of A on z.
__device__ __forceinline__ void bi_C_then_A(const Prob& p, int rank, int dst, const Lds& L) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, L.bd);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const double2 z = mask2(cscale<double>(L.bd[sl], inv), i0, p);
      st2(p.vec[dst], t.toff + 2 * idx, z);
      L.bd[sl] = z;
    }
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// C pass of A: y = A z;  out = b_m' z + kappa .* y;  partials of dots.
// which = 0: v = M p^, partial (r^, v).   which = 1: t = M s^, partials (t,s), (t,t), (r^,t).
__device__ __forceinline__ void bi_C_matvec(const Prob& p, int m, int rank, int which, const Lds& L) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  const double bm = p.beta[m];
  const double* z = p.vec[which == 0 ? VPH : VSH];
  double* out = p.vec[which == 0 ? VV : VT];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, L.bd);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      if (!valid_at(p, i0)) continue;
      const int off = t.toff + 2 * idx;
      const double2 y = cscale<double>(L.bd[sl], inv);
      const double2 zz = ld2(z, off), kk = ld2(p.kap, off);
      const double2 o = mask2(make_double2(bm * zz.x + kk.x * y.x, bm * zz.y + kk.y * y.y), i0, p);
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
__device__ __forceinline__ void bi_s(const Prob& p, int rank, double alpha, const Lds& L) {
  const Plan& pl = L.pl;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    double acc[2] = {0.0, 0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 s = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        const double2 r = ld2(p.vec[VR], off), v = ld2(p.vec[VV], off), rh = ld2(p.vec[VRH], off);
        s = mask2(make_double2(r.x - alpha * v.x, r.y - alpha * v.y), i0, p);
        st2(p.vec[VS], off, s);
        acc[0] += s.x * s.x + s.y * s.y;
        acc[1] += rh.x * s.x + rh.y * s.y;
        s = pc_in(p, off, s);
      }
      L.bd[sl] = s;
    }
    const int sl[2] = {SL_SS, SL_RS};
    write_partials<2>(p, tile, sl, acc);
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// x += alpha p^ + omega s^; r = s - omega t; p = r + beta (p - omega v);
// partial (r,r); A pass of P^{-1} on p.
__device__ __forceinline__ void bi_update(const Prob& p, int m, int rank, double alpha, double omega, double beta,
                                          const Lds& L) {
  const Plan& pl = L.pl;
  double* x = p.u[m % kRing];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    double acc[1] = {0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 pn = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        const double2 ph = ld2(p.vec[VPH], off), sh = ld2(p.vec[VSH], off);
        const double2 s = ld2(p.vec[VS], off), tt = ld2(p.vec[VT], off);
        const double2 po = ld2(p.vec[VP], off), v = ld2(p.vec[VV], off);
        double2 xx = ld2(x, off);
        xx.x += alpha * ph.x + omega * sh.x;
        xx.y += alpha * ph.y + omega * sh.y;
        st2(x, off, mask2(xx, i0, p));
        const double2 r = mask2(make_double2(s.x - omega * tt.x, s.y - omega * tt.y), i0, p);
        st2(p.vec[VR], off, r);
        pn = mask2(make_double2(r.x + beta * (po.x - omega * v.x), r.y + beta * (po.y - omega * v.y)), i0, p);
        st2(p.vec[VP], off, pn);
        acc[0] += r.x * r.x + r.y * r.y;
        pn = pc_in(p, off, pn);
      }
      L.bd[sl] = pn;
    }
    const int sl[1] = {SL_RR};
    write_partials<1>(p, tile, sl, acc);
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// x += alpha p^ (half-iteration exit).
__device__ __forceinline__ void bi_half(const Prob& p, int m, int rank, double alpha) {
  const Plan& pl = p.pl;   // sizes only
  double* x = p.u[m % kRing];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      if (!valid_at(p, i0)) continue;
      const int off = t.toff + 2 * idx;
      const double2 ph = ld2(p.vec[VPH], off);
      double2 xx = ld2(x, off);
      xx.x += alpha * ph.x;
      xx.y += alpha * ph.y;
      st2(x, off, mask2(xx, i0, p));
    }
  }
}

// Level setup shared by both solvers: rhs, optional initial residual.
// bb = ||b||^2, rr0 = ||r0||^2.
__device__ __forceinline__ int level_start(const Prob& p, int m, int rank, Ctl& ctl, const Lds& L, bool fp32pc,
                                           double& bb, double& rr0) {
  // the helpers' history sum H1^m (step m-1) must be complete
  if (p.nh > 0 && m >= 3 && !wait_ge<8>(p, &p.sync2[0], unsigned(m - 2) * unsigned(p.nh), ctl)) return FIDS_EDEVICE;
  // FGMRES ends every level with A u^m from an explicit matvec, so the
  // residual of an extrapolated guess can be formed from the kept products.
  // PCG forms it by a matvec: its recurrences carry the initial residual's
  // rounding to the end, and the extrapolation weights (4, -6, 4, -1 for the
  // cubic) amplify that of the kept products several-fold.
  const bool fused = p.solver == FIDS_FGMRES && p.x0_mode != 0 && m >= 3 && !p.adjoint;
  if (p.adjoint) {
    if (fp32pc) phase_adj_rhs<float>(p, m, rank, L, ctl);
    else phase_adj_rhs<double>(p, m, rank, L, ctl);
  } else if (fp32pc) {
    phase_rhs<float>(p, m, rank, L, fused, ctl);
  } else {
    phase_rhs<double>(p, m, rank, L, fused, ctl);
  }
  BARRIER();
  double red3[3];
  {
    const int sl[3] = {SL_BB, SL_RR, SL_KB};
    reduce_slots<3>(p, sl, red3);
  }
  // the method needs kappa > 0 (the problem statement of (1.1)); a level with
  // kappa^m not > 0 somewhere (or NaN) is reported as FIDS_ENUMERIC
  if (red3[2] != 0.0) {
    write_info(p, rank, m, 0, 0, NAN, FIDS_ENUMERIC);
    return FIDS_ENUMERIC;
  }
  bb = red3[0];
  rr0 = fused ? red3[1] : bb;
  double red1[1];
  if (p.x0_mode != 0 && !fused) {
    phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
    BARRIER();
    if (fp32pc) phase_r0<float>(p, m, rank, L);
    else phase_r0<double>(p, m, rank, L);
    BARRIER();
    const int sl[1] = {SL_RR};
    reduce_slots<1>(p, sl, red1);
    rr0 = red1[0];
  }
  return FIDS_OK;
}

// One level of FIDS with right-preconditioned BiCGSTAB.
__device__ __forceinline__ int level_bicgstab(const Prob& p, int m, int rank, Ctl& ctl, const Lds& L) {
  const double* Q = pQ<double>(p, m);
  const double tol = p.tol;
  double bb, rho;
  {
    const int st = level_start(p, m, rank, ctl, L, false, bb, rho);
    if (st != FIDS_OK) return st;
  }
  if (bad(bb) || bad(rho)) { write_info(p, rank, m, 0, 0, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
  const double bnorm = sqrt(bb);
  const int mv0 = p.x0_mode != 0 ? 1 : 0;
  if (sqrt(rho) <= tol * bnorm) {
    write_info(p, rank, m, 0, mv0, bnorm > 0 ? sqrt(rho) / bnorm : 0.0, FIDS_OK);
    return FIDS_OK;
  }
  double alpha = 0, omega = 0, red1[1];
  int it = 0, mv = mv0;
  for (;;) {
    phase_rows<double, double>(p, rank, Q, p.T, L.bd, L);   // P^{-1} p
    BARRIER();
    bi_C_then_A(p, rank, VPH, L);                        // p^ ; A p^ (column pass)
    BARRIER();
    phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
    BARRIER();
    bi_C_matvec(p, m, rank, 0, L);                       // v = M p^
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
    bi_s(p, rank, alpha, L);                             // s = r - alpha v ; P^{-1} s (column pass)
    BARRIER();
    double red2[2];
    {
      const int sl[2] = {SL_SS, SL_RS};
      reduce_slots<2>(p, sl, red2);
    }
    const double ss = red2[0], rs = red2[1];
    if (bad(ss)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
    if (sqrt(ss) <= tol * bnorm) {
      bi_half(p, m, rank, alpha);
      BARRIER();
      write_info(p, rank, m, it + 1, mv, sqrt(ss) / bnorm, FIDS_OK);
      return FIDS_OK;
    }
    phase_rows<double, double>(p, rank, Q, p.T, L.bd, L);
    BARRIER();
    bi_C_then_A(p, rank, VSH, L);
    BARRIER();
    phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
    BARRIER();
    bi_C_matvec(p, m, rank, 1, L);                       // t = M s^
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
    bi_update(p, m, rank, alpha, omega, beta, L);        // x, r, p ; P^{-1} p (column pass)
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

// ------------------------------------------------------------- PCG
// Conjugate gradients on the symmetrised system S = K_m^{-1} M^{(m)} =
// b_m' K_m^{-1} + A (SPD) with right-hand side K_m^{-1} b and preconditioner
// C = P^{(m)} / kbar_m, in the one-reduction form of Chronopoulos and Gear
// (the recurrences for p and s = S p share one reduction of the two dots per
// iteration).  The vectors kept are those of the original system: r = b -
// M x (= K_m times the symmetrised residual), u = C^{-1} K_m^{-1} r, w = M u
// and s = M p, so every inner product of the symmetrised system carries the
// weight 1/kappa: (r_s, u) = sum r u / kappa, (S u, u) = sum w u / kappa.
// Per iteration: rows of P^{-1} | C pass -> u, A pass of A on u | rows of A |
// C pass -> w, dots | updates of p, s, x, r, A pass of P^{-1} on r: five
// group barriers, one matvec, one preconditioner application.

// C pass of A on u: w = b_m' u + kappa .* A u; partials (r,u)_K, (w,u)_K.
__device__ __forceinline__ void pcg_C_matvec(const Prob& p, int m, int rank, const Lds& L) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  const double bm = p.beta[m];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, L.bd);
    double acc[2] = {0.0, 0.0};
    for (int base = threadIdx.x; base < t.total; base += kVecBatch * kThreads) {
      double2 uu[kVecBatch], kv[kVecBatch], rv[kVecBatch];
#pragma unroll
      for (int q = 0; q < kVecBatch; ++q) {   // loads first (see pcg_update)
        const int idx = base + q * kThreads;
        int i0, sl;
        item(pl, t, idx, i0, sl);
        const int off = t.toff + 2 * idx;
        if (idx < t.total && valid_at(p, i0)) {
          uu[q] = ld2(p.vec[VPH], off);
          kv[q] = ld2(p.kap, off);
          rv[q] = ld2(p.vec[VR], off);
        }
      }
#pragma unroll
      for (int q = 0; q < kVecBatch; ++q) {
        const int idx = base + q * kThreads;
        int i0, sl;
        item(pl, t, idx, i0, sl);
        if (idx >= t.total || !valid_at(p, i0)) continue;
        const int off = t.toff + 2 * idx;
        const double2 y = cscale<double>(L.bd[sl], inv);
        const double2 u = uu[q], kk = kv[q], r = rv[q];
        const double2 w = mask2(make_double2(bm * u.x + kk.x * y.x, bm * u.y + kk.y * y.y), i0, p);
        st2(p.vec[VV], off, w);
        const double ix = 1.0 / kk.x, iy = valid_at(p, i0 + 1) ? 1.0 / kk.y : 0.0;
        acc[0] += (r.x * u.x) * ix + (r.y * u.y) * iy;
        acc[1] += (w.x * u.x) * ix + (w.y * u.y) * iy;
      }
    }
    const int sl[2] = {SL_RS, SL_TS};
    write_partials<2>(p, tile, sl, acc);
  }
}

// p = u + beta p, s = w + beta s (first iteration: p = u, s = w);
// x += alpha p, r -= alpha s; partial (r,r); A pass of P^{-1} on r.
__device__ __forceinline__ void pcg_update(const Prob& p, int m, int rank, double alpha, double beta, bool first,
                                           const Lds& L) {
  const Plan& pl = L.pl;
  double* x = p.u[m % kRing];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    double acc[1] = {0.0};
    // kVecBatch items per thread: all loads first (the stores to the same
    // vectors would otherwise hold back the next item's loads)
    for (int base = threadIdx.x; base < t.total; base += kVecBatch * kThreads) {
      double2 uu[kVecBatch], ww[kVecBatch], po[kVecBatch], so[kVecBatch], xo[kVecBatch], ro[kVecBatch];
      double2 dd[kVecBatch];
#pragma unroll
      for (int q = 0; q < kVecBatch; ++q) {
        const int idx = base + q * kThreads;
        int i0, sl;
        item(pl, t, idx, i0, sl);
        const int off = t.toff + 2 * idx;
        if (idx < t.total && valid_at(p, i0)) {
          uu[q] = ld2(p.vec[VPH], off);
          ww[q] = ld2(p.vec[VV], off);
          if (!first) { po[q] = ld2(p.vec[VP], off); so[q] = ld2(p.vec[VS], off); }
          xo[q] = ld2(x, off);
          ro[q] = ld2(p.vec[VR], off);
          dd[q] = ld2(p.dsc, off);
        }
      }
#pragma unroll
      for (int q = 0; q < kVecBatch; ++q) {
        const int idx = base + q * kThreads;
        if (idx >= t.total) continue;
        int i0, sl;
        item(pl, t, idx, i0, sl);
        const int off = t.toff + 2 * idx;
        double2 r = make_double2(0.0, 0.0);
        if (valid_at(p, i0)) {
          double2 pp = uu[q], ss = ww[q];
          if (!first) {
            pp = make_double2(pp.x + beta * po[q].x, pp.y + beta * po[q].y);
            ss = make_double2(ss.x + beta * so[q].x, ss.y + beta * so[q].y);
          }
          st2(p.vec[VP], off, pp);
          st2(p.vec[VS], off, ss);
          double2 xx = xo[q];
          xx.x += alpha * pp.x;
          xx.y += alpha * pp.y;
          st2(x, off, mask2(xx, i0, p));
          r = mask2(make_double2(ro[q].x - alpha * ss.x, ro[q].y - alpha * ss.y), i0, p);
          st2(p.vec[VR], off, r);
          acc[0] += r.x * r.x + r.y * r.y;
          r = make_double2(r.x * dd[q].x, r.y * dd[q].y);   // pc_in: PCG always scales by kbar / kappa
        }
        L.bd[sl] = r;
      }
    }
    const int sl[1] = {SL_RR};
    write_partials<1>(p, tile, sl, acc);
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// Column pass of A on the iterate x (the first pass of its true residual).
__device__ __forceinline__ void pcg_x_colA(const Prob& p, int m, int rank, const Lds& L) {
  const Plan& pl = L.pl;
  const double* x = p.u[m % kRing];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      L.bd[sl] = ld2(x, t.toff + 2 * idx);
    }
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// One level of FIDS with preconditioned conjugate gradients.  When the
// recursively updated residual meets the tolerance, the true residual
// b - M x is formed by an explicit matvec.  A true residual within kPcgSlack times the
// tolerance is accepted (the gap of a few tolerances is FP64 rounding: at
// n = 65535 every solver's true residual floor is about 2.5e-10 of ||b||);
// beyond that CG restarts from it (at most kPcgChecks times) and a level whose
// true residual stops improving is accepted at that attainable floor.  The
// true value is reported either way.
__device__ __forceinline__ int level_pcg(const Prob& p, int m, int rank, Ctl& ctl, const Lds& L) {
  const double* Q = pQ<double>(p, m);
  const double tol = p.tol;
  double bb, rr;
  {
    const int st = level_start(p, m, rank, ctl, L, false, bb, rr);
    if (st != FIDS_OK) return st;
  }
  if (bad(bb) || bad(rr)) { write_info(p, rank, m, 0, 0, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
  const double bnorm = sqrt(bb);
  int it = 0, mv = p.x0_mode != 0 ? 1 : 0;   // the residual of an extrapolated guess costs a matvec
  if (sqrt(rr) <= tol * bnorm) {
    write_info(p, rank, m, 0, mv, bnorm > 0 ? sqrt(rr) / bnorm : 0.0, FIDS_OK);
    return FIDS_OK;
  }
  double alpha = 0.0, gamma_old = 0.0, rr_true_prev = INFINITY;
  int cyc0 = 0, checks = 0;                // first iteration of the current CG cycle
  for (;;) {
    phase_rows<double, double>(p, rank, Q, p.T, L.bd, L);   // P^{-1} r
    BARRIER();
    bi_C_then_A(p, rank, VPH, L);                        // u ; A u (column pass)
    BARRIER();
    phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
    BARRIER();
    pcg_C_matvec(p, m, rank, L);                         // w = M u ; (r,u)_K, (w,u)_K
    BARRIER();
    ++mv;
    double red2[2];
    {
      const int sl[2] = {SL_RS, SL_TS};
      reduce_slots<2>(p, sl, red2);
    }
    const double g = red2[0], d = red2[1];
    if (bad(g) || bad(d)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
    const bool first = it == cyc0;
    const double beta = first ? 0.0 : g / gamma_old;
    const double den = first ? d : d - beta * g / alpha;
    // S and C are SPD: g > 0 and den = (p, S p) > 0 unless r = 0 or rounding took over
    if (!(g > 0.0) || !(den > 0.0)) {
      write_info(p, rank, m, it, mv, sqrt(rr) / bnorm, FIDS_ENOCONV);
      return FIDS_ENOCONV;
    }
    alpha = g / den;
    gamma_old = g;
    pcg_update(p, m, rank, alpha, beta, first, L);       // p, s, x, r ; P^{-1} r (column pass)
    BARRIER();
    ++it;
    double red1[1];
    const int sl1[1] = {SL_RR};
    reduce_slots<1>(p, sl1, red1);
    rr = red1[0];
    if (bad(rr)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
    if (sqrt(rr) <= tol * bnorm) {
      // true residual: A x, r = b - M x, P^{-1} column pass on r (for a restart)
      pcg_x_colA(p, m, rank, L);
      BARRIER();
      phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
      BARRIER();
      phase_r0<double>(p, m, rank, L);
      BARRIER();
      ++mv;
      double red2x[2];
      const int slx[2] = {SL_RR, SL_XX};
      reduce_slots<2>(p, slx, red2x);
      const double rt = red2x[0];
      if (bad(rt)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
      if (sqrt(rt) <= kPcgSlack * tol * bnorm) {
        write_info(p, rank, m, it, mv, sqrt(rt) / bnorm, FIDS_OK);
        return FIDS_OK;
      }
      if (++checks >= kPcgChecks || !(rt < 0.25 * rr_true_prev)) {
        // stalled: accepted at the FP64 floor only within its rounding level
        const bool ok = sqrt(rt) <= floor_bound(p, m, red2x[1], bnorm) * bnorm;
        write_info(p, rank, m, it, mv, sqrt(rt) / bnorm, ok ? FIDS_OK : FIDS_ENOCONV);
        return ok ? FIDS_OK : FIDS_ENOCONV;
      }
      rr_true_prev = rt;
      rr = rt;
      cyc0 = it;                             // restart from the true residual
    }
    if (it >= p.maxit) {
      write_info(p, rank, m, it, mv, sqrt(rr) / bnorm, FIDS_ENOCONV);
      return FIDS_ENOCONV;
    }
  }
}

// ------------------------------------------------------------- FGMRES
// Small Hessenberg state kept identically by every workgroup (LDS):
//   hraw[(J+1) x J] unrotated Arnoldi coefficients (row-major, stride J),
//   cs/sn[J] Givens rotations, g[J+1] rotated right-hand side,
//   gsave[J] g[j] before rotation j, cor[J+1] re-orthogonalisation
//   coefficients, y[J+1] least-squares solution / scratch.
struct Hess {
  double *hraw, *cs, *sn, *g, *gsave, *cor, *y, *col, *R;
  int J;
};
__device__ __forceinline__ Hess hess(const Lds& L, int J) {
  Hess H;
  H.J = J;
  H.hraw = L.small;
  H.cs = H.hraw + (J + 1) * J;
  H.sn = H.cs + J;
  H.g = H.sn + J;
  H.gsave = H.g + J + 1;
  H.cor = H.gsave + J;
  H.y = H.cor + J + 1;
  H.col = H.y + J + 1;
  H.R = H.col + J + 1;        // J x J
  return H;
}

// Apply rotations 0..j-1 to column j of hraw, form rotation j, update g.
// Thread 0 only (state in LDS); callers synchronise.
__device__ __forceinline__ void givens_col(const Hess& H, int j, bool redo) {
  double* col = H.col;
  for (int i = 0; i <= j + 1; ++i) col[i] = H.hraw[i * H.J + j];
  for (int k = 0; k < j; ++k) {
    const double a = col[k], b = col[k + 1];
    col[k] = H.cs[k] * a + H.sn[k] * b;
    col[k + 1] = -H.sn[k] * a + H.cs[k] * b;
  }
  if (!redo) H.gsave[j] = H.g[j];
  const double a = col[j], b = col[j + 1];
  const double r = hypot(a, b);
  const double c = r > 0 ? a / r : 1.0, s = r > 0 ? b / r : 0.0;
  H.cs[j] = c;
  H.sn[j] = s;
  const double gj = H.gsave[j];
  H.g[j] = c * gj;
  H.g[j + 1] = -s * gj;
}

// Back substitution R y = g for columns 0..jl (R rebuilt from hraw by the
// stored rotations).  Thread 0 only.
__device__ __forceinline__ void lsq_solve(const Hess& H, int jl) {
  double* col = H.col;
  const int J = H.J;
  for (int j = 0; j <= jl; ++j) {
    for (int i = 0; i <= j + 1; ++i) col[i] = H.hraw[i * J + j];
    for (int k = 0; k <= j; ++k) {
      const double a = col[k], b = col[k + 1];
      col[k] = H.cs[k] * a + H.sn[k] * b;
      col[k + 1] = -H.sn[k] * a + H.cs[k] * b;
    }
    for (int i = 0; i <= j; ++i) H.R[i * J + j] = col[i];
  }
  for (int i = jl; i >= 0; --i) {
    double s = H.g[i];
    for (int k = i + 1; k <= jl; ++k) s -= H.R[i * J + k] * H.y[k];
    H.y[i] = (H.R[i * J + i] != 0.0) ? s / H.R[i * J + i] : 0.0;
  }
}

// P1: C pass of A on z_j -> w = b_m' z_j + kappa .* A z_j (stored in VV);
// re-orthogonalisation of v_j (j >= 1) with cor[] from the previous step;
// partials (v_i, w), i <= j, and (w, w); then the column pass of P^{-1} on
// w - v_j.  Pipelining: z_{j+1} is formed in P3 by linearity from
// P^{-1}(w - v_j) before the Arnoldi coefficients are known.  The shift by
// v_j matters: with a good preconditioner w ~ v_j, and applying P^{-1} to w
// itself would amplify its rounding error (FP32 in the mixed form) by
// ||w|| / eta.
template <typename RP>
__device__ __forceinline__ void gm_P1(const Prob& p, int m, int rank, int j, const Lds& L, const Hess& H) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  const double bm = p.beta[m];
  const int vl = p.vlen;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<double>(pl, tile, p.T, L.bd);
    double accw[1] = {0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 w = make_double2(0.0, 0.0), sh = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        const double2 y = cscale<double>(L.bd[sl], inv);
        const double2 zz = z_get<RP>(p, j, off), kk = ld2(p.kap, off);
        w = mask2(make_double2(bm * zz.x + kk.x * y.x, bm * zz.y + kk.y * y.y), i0, p);
        double2 v = ld2(p.V + size_t(j) * vl, off);
        if (j >= 1) {
          for (int i = 0; i < j; ++i) {
            const double2 vi = ld2(p.V + size_t(i) * vl, off);
            v.x -= H.cor[i] * vi.x;
            v.y -= H.cor[i] * vi.y;
          }
          const double sc = 1.0 / H.cor[j];
          v = make_double2(v.x * sc, v.y * sc);
          st2(p.V + size_t(j) * vl, off, v);
        }
        sh = make_double2(w.x - v.x, w.y - v.y);
      }
      st2(p.vec[VV], off, w);
      accw[0] += w.x * w.x + w.y * w.y;
      lbuf<RP>(L)[sl] = tocx<RP>(valid_at(p, i0) ? pc_in(p, off, sh) : sh);
    }
    {
      const int sl[1] = {SL_GM + kMaxRestart + 1};
      write_partials<1>(p, tile, sl, accw);
    }
    // (v_i, w) in chunks of 8
    for (int i0b = 0; i0b <= j; i0b += 8) {
      double acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.0;
      for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
        int i0, sl;
        item(pl, t, idx, i0, sl);
        if (!valid_at(p, i0)) continue;
        const int off = t.toff + 2 * idx;
        const double2 w = ld2(p.vec[VV], off);
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (i0b + q <= j) {
            const double2 vi = ld2(p.V + size_t(i0b + q) * vl, off);
            acc[q] += vi.x * w.x + vi.y * w.y;
          }
      }
      block_sum<8>(acc);
      if (threadIdx.x == 0)
        for (int q = 0; q < 8 && i0b + q <= j; ++q) p.part[(SL_GM + i0b + q) * pl.ntiles + tile] = acc[q];
    }
    tileA_fft_store<RP>(pl, tile, lbuf<RP>(L), pT<RP>(p));
  }
}

// P3: C pass of P^{-1} on w - v_j -> y = P^{-1}(w - v_j);
//   z_{j+1} = (y + z_j - sum_{i<=j} h_ij z_i) / eta,  v_{j+1} = (w - sum h_ij v_i) / eta,
// stored; partials (v_i, v_{j+1}) i <= j and (v_{j+1}, v_{j+1}) for the
// re-orthogonalisation; then the column pass of A on z_{j+1}.
// For j = -1 (start of a cycle): z_0 = y / beta0, v_0 = r0 / beta0.
template <typename RP>
__device__ __forceinline__ void gm_P3(const Prob& p, int rank, int j, double eta, const Lds& L, const Hess& H) {
  const Plan& pl = L.pl;
  const double inv = 1.0 / double(pl.Nc);
  const int vl = p.vlen;
  const double ie = 1.0 / eta;
  const int jn = j + 1;
  const double* src = (j < 0) ? p.vec[VR] : p.vec[VV];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    tileC_load_ifft<RP>(pl, tile, pT<RP>(p), lbuf<RP>(L));
    double accv[1] = {0.0};
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 z = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        const double2 y = fromcx<RP>(lbuf<RP>(L)[sl]);
        z = make_double2(y.x * inv, y.y * inv);
        if (j >= 0) {
          const double2 zj = z_get<RP>(p, j, off);
          z.x += zj.x;
          z.y += zj.y;
        }
        v = ld2(src, off);
        for (int i = 0; i <= j; ++i) {
          const double h = H.hraw[i * H.J + j];
          const double2 zi = z_get<RP>(p, i, off);
          const double2 vi = ld2(p.V + size_t(i) * vl, off);
          z.x -= h * zi.x; z.y -= h * zi.y;
          v.x -= h * vi.x; v.y -= h * vi.y;
        }
        z = mask2(make_double2(z.x * ie, z.y * ie), i0, p);
        v = mask2(make_double2(v.x * ie, v.y * ie), i0, p);
        accv[0] += v.x * v.x + v.y * v.y;
      }
      L.bd[sl] = z_put<RP>(p, jn, off, z);
      st2(p.V + size_t(jn) * vl, off, v);
    }
    {
      const int sl[1] = {SL_GM + kMaxRestart + 1};
      write_partials<1>(p, tile, sl, accv);
    }
    for (int i0b = 0; i0b <= j; i0b += 8) {
      double acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.0;
      for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
        int i0, sl;
        item(pl, t, idx, i0, sl);
        if (!valid_at(p, i0)) continue;
        const int off = t.toff + 2 * idx;
        const double2 v = ld2(p.V + size_t(jn) * vl, off);
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (i0b + q <= j) {
            const double2 vi = ld2(p.V + size_t(i0b + q) * vl, off);
            acc[q] += vi.x * v.x + vi.y * v.y;
          }
      }
      block_sum<8>(acc);
      if (threadIdx.x == 0)
        for (int q = 0; q < 8 && i0b + q <= j; ++q) p.part[(SL_GM + i0b + q) * pl.ntiles + tile] = acc[q];
    }
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// F1: x += sum_{i<=jl} y_i z_i; column pass of A on x.
template <typename RP>
__device__ __forceinline__ void gm_F1(const Prob& p, int m, int rank, int jl, const Lds& L, const Hess& H) {
  const Plan& pl = L.pl;
  double* x = p.u[m % kRing];
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      const int off = t.toff + 2 * idx;
      double2 xx = make_double2(0.0, 0.0);
      if (valid_at(p, i0)) {
        xx = ld2(x, off);
        for (int i = 0; i <= jl; ++i) {
          const double2 zi = z_get<RP>(p, i, off);
          xx.x += H.y[i] * zi.x;
          xx.y += H.y[i] * zi.y;
        }
        xx = mask2(xx, i0, p);
        st2(x, off, xx);
      }
      L.bd[sl] = xx;
    }
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// Column pass of P^{-1} (FP64) on the residual VR: the start of a restart
// cycle that continues with the FP64 preconditioner.
__device__ __forceinline__ void phase_pc_col64(const Prob& p, int rank, const Lds& L) {
  const Plan& pl = L.pl;
  for (int tile = rank; tile < pl.ntiles; tile += p.ng) {
    const TileIdx t = tile_idx(pl, tile);
    for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
      int i0, sl;
      item(pl, t, idx, i0, sl);
      L.bd[sl] = valid_at(p, i0) ? pc_in(p, t.toff + 2 * idx, ld2(p.vec[VR], t.toff + 2 * idx)) : make_double2(0.0, 0.0);
    }
    tileA_fft_store<double>(pl, tile, L.bd, p.T);
  }
}

// Counters a level carries from one restart cycle to the next.
struct Cyc {
  double rr;          // ||r||^2 of the true residual in VR
  double xx;          // ||x||^2 of the iterate it belongs to (after a cycle)
  int it, mv, floor_hits, it64;
  bool est_conv;
};
constexpr int kFallback = 1;   // internal: continue the level with the FP64 preconditioner

// Restart cycles of flexible GMRES(J) with the preconditioner in precision RP,
// from the true residual r (VR, ||r||^2 = rr) whose P^{-1} column pass is in
// pT<RP>.  With the FP32 preconditioner, a level still unconverged after its
// first cycle continues with the FP64 preconditioner: flexible GMRES allows a
// different preconditioner in every cycle, and the FP32 transforms cannot
// resolve a preconditioner spectrum 1/(b_m' + kbar lambda_k) that spans more
// than about 1e5.
template <typename RP>
__device__ __forceinline__ int fgmres_cycles(const Prob& p, int m, int rank, Ctl& ctl, const Lds& L, const Hess& H,
                                             double bnorm, Cyc& c) {
  double rr = c.rr, xx = c.xx;
  int it = c.it, mv = c.mv, floor_hits = c.floor_hits, it64 = c.it64;
  bool est_conv = c.est_conv;
  const RP* Q = pQ<RP>(p, m);
  const double tol = p.tol;
  const int J = p.restart;
  double red1[1];
  for (;;) {                                   // restart cycles
    const double beta0 = sqrt(rr);
    if (est_conv && beta0 > tol * bnorm && ++floor_hits >= 2) {
      // the Arnoldi estimate met the tolerance twice but the true FP64
      // residual did not: accepted at that floor only within its rounding
      // level, with the true relative residual reported
      const int st = beta0 <= floor_bound(p, m, xx, bnorm) * bnorm ? FIDS_OK : FIDS_ENOCONV;
      write_info(p, rank, m, it, mv, beta0 / bnorm, st, it64);
      return st;
    }
    if (beta0 <= tol * bnorm) {
      write_info(p, rank, m, it, mv, bnorm > 0 ? beta0 / bnorm : 0.0, FIDS_OK, it64);
      return FIDS_OK;
    }
    if (it >= p.maxit) { write_info(p, rank, m, it, mv, beta0 / bnorm, FIDS_ENOCONV, it64); return FIDS_ENOCONV; }
    if constexpr (sizeof(RP) == 4) {
      if (p.qhat != nullptr && p.zd != nullptr && it >= J) {
        c.rr = rr; c.xx = xx; c.it = it; c.mv = mv; c.floor_hits = floor_hits; c.it64 = 0; c.est_conv = est_conv;
        return kFallback;
      }
    }
    const int it_cycle0 = it;
    if (threadIdx.x == 0) {
      for (int i = 0; i <= J; ++i) H.g[i] = 0.0;
      H.g[0] = beta0;
    }
    __syncthreads();
    phase_rows<RP, RP>(p, rank, Q, pT<RP>(p), lbuf<RP>(L), L);      // P^{-1} r0 (rows)
    BARRIER();
    gm_P3<RP>(p, rank, -1, beta0, L, H);                        // z_0, v_0; A z_0 (columns)
    BARRIER();
    phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
    BARRIER();
    int jl = 0;
    for (int j = 0;; ++j) {
      gm_P1<RP>(p, m, rank, j, L, H);                           // w = M z_j; dots; P^{-1} w (columns)
      BARRIER();
      ++it;
      ++mv;
      reduce_range(p, SL_GM, j + 1, H.y);                       // h_ij into y[] scratch
      {
        const int sl[1] = {SL_GM + kMaxRestart + 1};
        reduce_slots<1>(p, sl, red1);
      }
      double hs = 0.0;
      for (int i = 0; i <= j; ++i) hs += H.y[i] * H.y[i];
      if (bad(red1[0]) || bad(hs)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC, it64); return FIDS_ENUMERIC; }
      const double e2 = red1[0] - hs;
      const double eta = e2 > 0.0 ? sqrt(e2) : 0.0;
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int i = 0; i <= j; ++i) H.hraw[i * J + j] = H.y[i];
        H.hraw[(j + 1) * J + j] = eta;
        givens_col(H, j, false);
      }
      __syncthreads();
      const double est = fabs(H.g[j + 1]);
      jl = j;
      est_conv = est <= tol * bnorm;
      if (est_conv || j + 1 >= J || eta <= 1e-300 * bnorm || it >= p.maxit) break;
      phase_rows<RP, RP>(p, rank, Q, pT<RP>(p), lbuf<RP>(L), L);    // P^{-1} w (rows)
      BARRIER();
      gm_P3<RP>(p, rank, j, eta, L, H);                          // z_{j+1}, v_{j+1}; A z_{j+1} (columns)
      BARRIER();
      reduce_range(p, SL_GM, j + 1, H.cor);                      // c_i = (v_i, v_{j+1})
      {
        const int sl[1] = {SL_GM + kMaxRestart + 1};
        reduce_slots<1>(p, sl, red1);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double cs = 0.0;
        for (int i = 0; i <= j; ++i) cs += H.cor[i] * H.cor[i];
        const double s2 = red1[0] - cs;
        const double sc = s2 > 0.0 ? sqrt(s2) : 1.0;
        H.cor[j + 1] = sc;
        for (int i = 0; i <= j; ++i) H.hraw[i * J + j] += eta * H.cor[i];
        H.hraw[(j + 1) * J + j] = eta * sc;
        givens_col(H, j, true);
      }
      __syncthreads();
      phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);    // A z_{j+1} (rows)
      BARRIER();
    }
    if (sizeof(RP) == 8 && p.precision == FIDS_MIXED) it64 += it - it_cycle0;
    __syncthreads();
    if (threadIdx.x == 0) lsq_solve(H, jl);
    __syncthreads();
    gm_F1<RP>(p, m, rank, jl, L, H);                             // x += Z y; A x (columns)
    BARRIER();
    phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
    BARRIER();
    if (sizeof(RP) == 4) phase_r0<float>(p, m, rank, L);       // r = b - M x; P^{-1} r (columns)
    else phase_r0<double>(p, m, rank, L);
    BARRIER();
    ++mv;
    {
      double red2[2];
      const int sl[2] = {SL_RR, SL_XX};
      reduce_slots<2>(p, sl, red2);
      rr = red2[0];
      xx = red2[1];
    }
    if (bad(rr)) { write_info(p, rank, m, it, mv, NAN, FIDS_ENUMERIC, it64); return FIDS_ENUMERIC; }
  }
}

// One level of FIDS with flexible GMRES(J), right preconditioning, pipelined
// so that one Arnoldi step costs four group barriers.
template <typename RP>
__device__ __forceinline__ int level_fgmres(const Prob& p, int m, int rank, Ctl& ctl, const Lds& L) {
  const Hess H = hess(L, p.restart);
  double bb, rr;
  {
    const int st = level_start(p, m, rank, ctl, L, sizeof(RP) == 4, bb, rr);
    if (st != FIDS_OK) return st;
  }
  if (bad(bb) || bad(rr)) { write_info(p, rank, m, 0, 0, NAN, FIDS_ENUMERIC); return FIDS_ENUMERIC; }
  Cyc c{rr, 0.0, 0, (p.x0_mode != 0) ? 1 : 0, 0, 0, false};
  const int st = fgmres_cycles<RP>(p, m, rank, ctl, L, H, sqrt(bb), c);
  if constexpr (sizeof(RP) == 4) {
    if (st == kFallback) {
      // the FP32 cycles' state is dead here, so the FP64 cycles reuse its registers
      phase_pc_col64(p, rank, L);
      BARRIER();
      return fgmres_cycles<double>(p, m, rank, ctl, L, H, sqrt(bb), c);
    }
  }
  return st;
}

// Level solver variants; each kernel instance holds one, so that its register
// allocation follows that path alone.
enum { VAR_BICG = 0, VAR_GM64 = 1, VAR_GM32 = 2, VAR_PCG = 3, VAR_COUNT = 4 };

template <int VAR>
__device__ __forceinline__ int level_solve(const Prob& p, int m, int rank, Ctl& ctl, const Lds& L) {
  if constexpr (VAR == VAR_BICG) return level_bicgstab(p, m, rank, ctl, L);
  else if constexpr (VAR == VAR_PCG) return level_pcg(p, m, rank, ctl, L);
  else if constexpr (VAR == VAR_GM32) return level_fgmres<float>(p, m, rank, ctl, L);
  else return level_fgmres<double>(p, m, rank, ctl, L);
}

// Adjoint level m: transposed solve, reversed history step, A u^m for the
// kappa gradient (finished by the next level's right-hand side phase or by
// the flush after the launch's last level).
template <int VAR>
__device__ __forceinline__ int level_adjoint(const Prob& p, int m, int rank, Ctl& ctl, const Lds& L) {
  const int st = level_solve<VAR>(p, m, rank, ctl, L);
  if (st != FIDS_OK) return st;
  phase_adj_post(p, m, rank, L, ctl);
  BARRIER();
  phase_rows<double, double>(p, rank, p.ahat, p.T, L.bd, L);
  BARRIER();
  return FIDS_OK;
}

// One problem's levels inside the level kernel (workgroup `rank` of its group).
template <int VAR, bool ADJ>
__device__ __forceinline__ void run_member(const Prob& p, int rank, int m_begin, int m_end, int hist_lo,
                                           int ckpt_on, unsigned long long timeout, int* abort_flag,
                                           double2* dyn) {
  // LDS: [tab 3*nexp doubles][small][twiddles FP64][twiddles FP32][FP64 buffer][FP32 buffer]
  const int tab_c = (3 * p.nexp + 1) / 2;
  const int small_c = kSmallDoubles / 2;
  const int tile_pts = max(2 * p.pl.CT * p.pl.N1, 4 * p.pl.RU * p.pl.N2);
  const int nlo = p.pl.twmask + 1;
  const int ntw = p.pl.twn;               // twiddles copied to LDS (set with twres)
  const bool mixed = p.precision == FIDS_MIXED;
  Lds L;
  L.tab = reinterpret_cast<double*>(dyn);
  L.small = reinterpret_cast<double*>(dyn + tab_c);
  double2* twd = dyn + tab_c + small_c;
  float2* twf = reinterpret_cast<float2*>(twd + ntw);
  L.bd = twd + ntw + (mixed ? (ntw + 1) / 2 : 0);
  L.bf = reinterpret_cast<float2*>(L.bd + tile_pts);
  L.pl = p.pl;
  {
    const Plan& g = p.pl;
    for (int i = threadIdx.x; i < ntw; i += kThreads) {
      double2 v;
      float2 vf = make_float2(0.f, 0.f);
      if (i < g.N1) { v = g.tw1[i]; if (mixed) vf = g.tw1f[i]; }
      else if (i < g.N1 + g.N2) { v = g.tw2[i - g.N1]; if (mixed) vf = g.tw2f[i - g.N1]; }
      else if (i < g.N1 + g.N2 + nlo) { v = g.twlo[i - g.N1 - g.N2]; if (mixed) vf = g.twlof[i - g.N1 - g.N2]; }
      else { v = g.twhi[i - g.N1 - g.N2 - nlo]; if (mixed) vf = g.twhif[i - g.N1 - g.N2 - nlo]; }
      twd[i] = v;
      if (mixed) twf[i] = vf;
    }
    // tables not copied keep pointing at the global ones
    if (g.twres <= 1) {
      L.pl.tw1 = twd;
      L.pl.tw2 = twd + g.N1;
      L.pl.tw1f = twf;
      L.pl.tw2f = twf + g.N1;
    }
    if (g.twres == 0) {
      L.pl.twlo = twd + g.N1 + g.N2;
      L.pl.twhi = twd + g.N1 + g.N2 + nlo;
      L.pl.twlof = twf + g.N1 + g.N2;
      L.pl.twhif = twf + g.N1 + g.N2 + nlo;
    }
    __syncthreads();
  }
  Ctl ctl;
  ctl.rank = rank;
  // every workgroup of the group ends a launch with the same count
  ctl.gen = rank < p.ng ? __hip_atomic_load(&p.bar[rank * kBarSlotWords], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : 0u;
  ctl.timeout = timeout;
  ctl.abort_flag = abort_flag;
  ctl.hist_lo = hist_lo;
  ctl.ckpt_on = ckpt_on;
  ctl.pending = 0;
  ctl.sym_seen = 0;
  if constexpr (ADJ) {
    for (int m = m_begin; m >= m_end; --m) {
      ctl.pending = m < m_begin;
      const int st = level_adjoint<VAR>(p, m, rank, ctl, L);
      if (st != FIDS_OK) {
        if (rank == 0 && threadIdx.x == 0 && st == FIDS_EDEVICE) p.status[0] = FIDS_EDEVICE;
        return;
      }
    }
    phase_adj_flush(p, m_end, rank, L);
    return;
  }
  if (rank >= p.ng) {                         // SOE helper
    helper_loop(p, rank - p.ng, max(2, m_begin - 1), m_end - 1, ctl, L.tab);
    return;
  }
  for (int m = m_begin; m <= m_end; ++m) {
    int st = FIDS_OK;
    if (p.symflag && unsigned(m) > ctl.sym_seen && !wait_symbols(p, m, ctl)) st = FIDS_EDEVICE;
    if (st == FIDS_OK) st = level_solve<VAR>(p, m, rank, ctl, L);
    if (st != FIDS_OK) {
      if (rank == 0 && threadIdx.x == 0) {
        if (st == FIDS_EDEVICE) p.status[0] = FIDS_EDEVICE;
        __hip_atomic_store(&p.status[2], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      return;
    }
    // level m is complete in every workgroup of the group: publish it
    if (rank == 0 && threadIdx.x == 0)
      __hip_atomic_store(&p.sync2[64], unsigned(m), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  // keep u^{m_end} with the stored states (tile-local copy, no barrier needed)
  if (hist_lo >= 0) {
    const double* ue = p.u[m_end % kRing];
    double* dst = p.uhist + size_t(m_end - hist_lo) * p.vlen;
    for (int tile = rank; tile < L.pl.ntiles; tile += p.ng) {
      const TileIdx t = tile_idx(L.pl, tile);
      for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
        const int off = t.toff + 2 * idx;
        st2(dst, off, ld2(ue, off));
      }
    }
  }
}


// Persistent level kernel.  Forward descriptors advance m = m_begin..m_end;
// adjoint descriptors (ADJ) run m = m_begin down to m_end (m_begin >= m_end).
// Descriptors are sorted by their first workgroup g0; consecutive descriptors
// with the same g0 form a slot whose members the slot's workgroups run one
// after the other (packed batch members).
template <int VAR, bool ADJ>
__global__ void __launch_bounds__(kThreads) k_levels(const Prob* probs, int nprob, int m_begin, int m_end,
                                                     int hist_lo, int ckpt_on, unsigned long long timeout,
                                                     int* abort_flag) {
  extern __shared__ double2 dyn[];
  int last = 0;
  {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (int(blockIdx.x) >= probs[mid].g0) lo = mid;
      else hi = mid - 1;
    }
    last = lo;
  }
  const int first = probs[last].slot_first;
  for (int q = first; q <= last; ++q) {
    const Prob& p = probs[q];
    const int rank = int(blockIdx.x) - p.g0;
    if (rank < 0 || rank >= p.ng + p.nh) continue;
    run_member<VAR, ADJ>(p, rank, m_begin, m_end, hist_lo, ckpt_on, timeout, abort_flag, dyn);
    __syncthreads();
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
    const double2 v = nat2(p.phi, i0, p);
    st2(p.u[0], off, v);
    st2(p.u[kRing - 1], off, v);   // u^{-1} := u^0 (never weighted: extrapolation uses levels >= 0)
    if (p.store_states) st2(p.uhist, off, v);
  }
}

__global__ void __launch_bounds__(kThreads) k_to_natural(const Prob* pp, const double* src, double* dst) {
  const Prob& p = *pp;
  const Plan& pl = p.pl;
  const int tile = blockIdx.x;
  src += size_t(blockIdx.y) * p.vlen;
  dst += size_t(blockIdx.y) * p.nn;
  const TileIdx t = tile_idx(pl, tile);
  for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
    int i0, sl;
    item(pl, t, idx, i0, sl);
    const double2 v = ld2(src, t.toff + 2 * idx);
    if (valid_at(p, i0)) dst[nat_at(p, i0)] = v.x;
    if (valid_at(p, i0 + 1)) dst[nat_at(p, i0 + 1)] = v.y;
  }
}

__global__ void __launch_bounds__(kThreads) k_from_natural(const Prob* pp, const double* src, double* dst) {
  const Prob& p = *pp;
  const Plan& pl = p.pl;
  const int tile = blockIdx.x;
  const TileIdx t = tile_idx(pl, tile);
  for (int idx = threadIdx.x; idx < t.total; idx += kThreads) {
    int i0, sl;
    item(pl, t, idx, i0, sl);
    st2(dst, t.toff + 2 * idx, nat2(src, i0, p));
  }
}

__global__ void __launch_bounds__(kThreads) k_kbar(const double* kappa, int n, int m0, int td, double* kbar,
                                                   double* kmax) {
  __shared__ double red[kThreads / 64];
  const int m = m0 + int(blockIdx.x);
  const double* row = kappa + (td ? size_t(m - 1) * n : 0);
  double acc[1] = {0.0};
  double mx = -INFINITY;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    acc[0] += row[i];
    mx = fmax(mx, row[i]);
  }
  block_sum<1>(acc);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) mx = fmax(mx, red[w]);
    kbar[m] = acc[0] / double(n);
    kmax[m] = mx;
  }
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

__global__ void k_flag(unsigned* flag, unsigned value) {
  if (threadIdx.x == 0) __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------- host launchers
static size_t plan_lds(const Plan& pl) {
  const size_t a = size_t(2) * pl.CT * pl.N1, b = size_t(4) * pl.RU * pl.N2;
  return (a > b ? a : b) * sizeof(double2);
}

size_t level_lds_bytes(const Prob& h) {
  const size_t tab = size_t((3 * h.nexp + 1) / 2) * sizeof(double2);
  const size_t small = size_t(kSmallDoubles) * sizeof(double);
  const size_t bd = plan_lds(h.pl);
  const bool mixed = h.precision == FIDS_MIXED;
  const size_t bf = mixed ? bd / 2 : 0;
  const size_t ntw = size_t(h.pl.twn);
  const size_t tw = ntw * sizeof(double2) + (mixed ? ((ntw + 1) / 2) * sizeof(double2) : 0);
  return tab + small + tw + bd + bf;
}

hipError_t launch_init_state(const Prob& h, const Prob* d, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(h.pl.ntiles), dim3(kThreads), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_to_natural(const Prob& h, const Prob* d, const double* src, double* dst, hipStream_t s,
                             int64_t count) {
  for (int64_t k0 = 0; k0 < count; k0 += 65535) {
    const unsigned c = unsigned(std::min<int64_t>(65535, count - k0));
    hipLaunchKernelGGL(k_to_natural, dim3(h.pl.ntiles, c), dim3(kThreads), 0, s, d,
                       src + size_t(k0) * h.vlen, dst + size_t(k0) * h.n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_from_natural(const Prob& h, const Prob* d, const double* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_from_natural, dim3(h.pl.ntiles), dim3(kThreads), 0, s, d, src, dst);
  return hipGetLastError();
}

hipError_t launch_kbar(const double* kappa, int n, int m0, int cnt, int td, double* kbar, double* kmax,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_kbar, dim3(cnt), dim3(kThreads), 0, s, kappa, n, m0, td, kbar, kmax);
  return hipGetLastError();
}

hipError_t launch_flag(unsigned* flag, unsigned value, hipStream_t s) {
  hipLaunchKernelGGL(k_flag, dim3(1), dim3(64), 0, s, flag, value);
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
  hipLaunchKernelGGL(k_sym_b, dim3(job.plc.nrg, cnt), dim3(kThreads), lc, s, d);
  hipLaunchKernelGGL(k_sym_c, dim3(job.plc.ntiles, cnt), dim3(kThreads), lc, s, d);
  hipLaunchKernelGGL(k_sym_d, dim3(job.plr.ntiles, cnt), dim3(kThreads), lr, s, d);
  hipLaunchKernelGGL(k_sym_e, dim3(job.plr.nrg, cnt), dim3(kThreads), lr, s, d, m0);
  return hipGetLastError();
}

// The kernel instance of a descriptor's solver variant and direction.
static const void* level_kernel(const Prob& h) {
  static const void* const table[VAR_COUNT][2] = {
      {reinterpret_cast<const void*>(k_levels<VAR_BICG, false>), reinterpret_cast<const void*>(k_levels<VAR_BICG, true>)},
      {reinterpret_cast<const void*>(k_levels<VAR_GM64, false>), reinterpret_cast<const void*>(k_levels<VAR_GM64, true>)},
      {reinterpret_cast<const void*>(k_levels<VAR_GM32, false>), reinterpret_cast<const void*>(k_levels<VAR_GM32, true>)},
      {reinterpret_cast<const void*>(k_levels<VAR_PCG, false>), reinterpret_cast<const void*>(k_levels<VAR_PCG, true>)}};
  const int var = h.solver == FIDS_BICGSTAB ? VAR_BICG
                  : h.solver == FIDS_PCG    ? VAR_PCG
                                            : (h.precision == FIDS_MIXED ? VAR_GM32 : VAR_GM64);
  return table[var][h.adjoint ? 1 : 0];
}

hipError_t level_max_blocks(const Prob& h, size_t lds_bytes, int* per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, level_kernel(h), kThreads, lds_bytes);
}

hipError_t level_lds_cap(const Prob& h, size_t* cap) {
  int dev = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  hipFuncAttributes a{};
  if (e == hipSuccess) e = hipFuncGetAttributes(&a, level_kernel(h));
  if (e != hipSuccess) return e;
  const size_t st = a.sharedSizeBytes;
  *cap = size_t(per_cu) > st ? size_t(per_cu) - st : 0;
  return hipSuccess;
}

hipError_t set_level_lds_limit(const Prob& h, size_t bytes) {
  Prob a = h;
  a.adjoint = 0;
  hipError_t e = hipFuncSetAttribute(level_kernel(a), hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  if (e != hipSuccess) return e;
  a.adjoint = 1;
  return hipFuncSetAttribute(level_kernel(a), hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

hipError_t launch_levels_plain(const Prob& h, const Prob* probs, int nprob, int total_wg, size_t lds_bytes,
                               int m_begin, int m_end, hipStream_t s) {
  int hist_lo = -1, ckpt_on = 0;
  unsigned long long timeout_ticks = 0;
  int* abort_flag = nullptr;
  void* args[] = {(void*)&probs, (void*)&nprob, (void*)&m_begin, (void*)&m_end, (void*)&hist_lo,
                  (void*)&ckpt_on, (void*)&timeout_ticks, (void*)&abort_flag};
  return hipLaunchKernel(level_kernel(h), dim3(total_wg), dim3(kThreads), args, lds_bytes, s);
}

hipError_t launch_levels(const Prob& h, const Prob* probs, int nprob, int total_wg, size_t lds_bytes,
                         int m_begin, int m_end, int hist_lo, int ckpt_on, unsigned long long timeout_ticks,
                         int* abort_flag, hipStream_t s) {
  void* args[] = {(void*)&probs, (void*)&nprob, (void*)&m_begin, (void*)&m_end, (void*)&hist_lo,
                  (void*)&ckpt_on, (void*)&timeout_ticks, (void*)&abort_flag};
  return hipLaunchCooperativeKernel(level_kernel(h), dim3(total_wg), dim3(kThreads), args,
                                    static_cast<unsigned int>(lds_bytes), s);
}

}  // namespace fids
