// Host launchers for the gfx950 kernels (implemented in fids_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "fids_device.h"

namespace fids {

// LDS bytes a workgroup of the level kernel needs for problem descriptor `h`.
size_t level_lds_bytes(const Prob& h);

// Clears the state of one problem and sets u^0 = phi (tile-major).
hipError_t launch_init_state(const Prob& h, const Prob* d, hipStream_t s);

// Mean and largest entry of kappa^m for m = m0..m0+cnt-1 (rows m-1 of a
// [M][n] kappa, or its single row) into kbar[m] and kmax[m].
hipError_t launch_kbar(const double* kappa, int n, int m0, int cnt, int td, double* kbar, double* kmax,
                       hipStream_t s);

// Per-level preconditioner symbols for levels [m0, m0 + cnt).
hipError_t launch_symbols(const SymJob& job, const SymJob* d, int m0, int cnt, hipStream_t s);
// *flag = value (agent-scope release), ordered after the stream's earlier work.
hipError_t launch_flag(unsigned* flag, unsigned value, hipStream_t s);

// LDS bytes of the symbol kernels.
size_t symbols_lds_bytes(const SymJob& job);

// Advances every problem in `probs` (device array of `nprob` descriptors whose
// workgroup groups tile [0, total_wg)) over levels [m_begin, m_end] in one
// cooperative launch (adjoint descriptors: m_begin down to m_end).  The
// kernel instance follows the host copy `h` (all descriptors share its solver
// variant and direction).
// hist_lo >= 0 stores u^k at uhist[k - hist_lo] (forward) / reads it from
// there (adjoint); ckpt_on writes the forward segment snapshots.
hipError_t launch_levels(const Prob& h, const Prob* probs, int nprob, int total_wg, size_t lds_bytes,
                         int m_begin, int m_end, int hist_lo, int ckpt_on,
                         unsigned long long timeout_ticks, int* abort_flag, hipStream_t s);

// Ordinary (non-cooperative) launch for descriptors that all have one
// workgroup (ng = 1, no helpers): no workgroup ever waits for another, so the
// launch may be captured in a HIP graph.
hipError_t launch_levels_plain(const Prob& h, const Prob* probs, int nprob, int total_wg, size_t lds_bytes,
                               int m_begin, int m_end, hipStream_t s);

// Co-resident workgroups per CU of the level kernel instance of `h` (its
// solver variant and direction) for a given LDS size.
hipError_t level_max_blocks(const Prob& h, size_t lds_bytes, int* per_cu);

// Raises the dynamic-LDS limit of the forward and adjoint instances of `h`'s variant.
hipError_t set_level_lds_limit(const Prob& h, size_t bytes);
// Dynamic LDS a level-kernel workgroup may use on the current device (the
// CU's LDS less the kernel's static LDS).
hipError_t level_lds_cap(const Prob& h, size_t* cap);

// Natural-layout [n] array into a tile-major vector (zero padding).
hipError_t launch_from_natural(const Prob& h, const Prob* d, const double* src, double* dst, hipStream_t s);

// Copies u^m (tile-major) into a natural-layout [n] array.
// count vectors: src + k * vlen (tile-major) -> dst + k * n (natural), k < count
hipError_t launch_to_natural(const Prob& h, const Prob* d, const double* src, double* dst, hipStream_t s,
                             int64_t count = 1);

}  // namespace fids
