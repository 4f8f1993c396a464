// Per-edge accumulation of one step (Algorithm 2 lines 10-11, Eq. 9), shared by
// the kernels that carry it as extra workgroups.
#pragma once

#include "sc_internal.hpp"

namespace sc {

// gacc[k] += (Y[s][c] - Y[j][c]) / d_s for slot k = (s -> j) of the job's block,
// if l <= tau_k; Y is node-major with B columns, c = s - s0.
template <typename T, int B>
__device__ inline void accumulate_half(const AccJob& acc, const int32_t* __restrict__ slot_row,
                                       const int32_t* __restrict__ col,
                                       const double* __restrict__ inv_deg_d,
                                       const T* __restrict__ Y, int k) {
  if (k >= acc.kend) return;
  if (acc.rdiag) {   // recording job
    const int s = slot_row[k];
    const int c = s - acc.s0;
    const int64_t o = static_cast<int64_t>(k) * (kRecSteps + 1) + acc.ell;
    static_cast<T*>(acc.rdiag)[o] = Y[static_cast<size_t>(s) * B + c];
    static_cast<T*>(acc.roff)[o] = Y[static_cast<size_t>(col[k]) * B + c];
    return;
  }
  if (acc.ell > acc.tau[k]) return;
  const int s = slot_row[k];
  const int c = s - acc.s0;
  const int j = col[k];
  const double pss = static_cast<double>(Y[static_cast<size_t>(s) * B + c]);
  const double pjs = static_cast<double>(Y[static_cast<size_t>(j) * B + c]);
  acc.gacc[k] += (pss - pjs) * inv_deg_d[s];
}

}  // namespace sc
