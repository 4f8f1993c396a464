// Deterministic traversal kernels (Algorithm 2) for a block of B sources.
//
// Layout: the block state Y is node-major, Y[x * B + c] = p_l(x, s0 + c), so
// gathering a neighbour row reads B contiguous values.  Every reduction has a
// fixed order (no floating-point atomics), so results are bit-reproducible.
#include "sc_internal.hpp"

#include <cfloat>
#include <climits>

namespace sc {

namespace {

constexpr int kThreads = 64 * kWavesPerBlock;

inline unsigned grid_for(int64_t items, int per_block) {
  return static_cast<unsigned>((items + per_block - 1) / per_block);
}

// ------------------------------------------------------------------ closed-form l = 0, 1 terms
__global__ void k_gacc_init(int64_t nslots, const int32_t* __restrict__ slot_row,
                            const int32_t* __restrict__ col, const double* __restrict__ inv_deg,
                            const int32_t* __restrict__ tau, int include_l1,
                            double* __restrict__ gacc) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nslots) return;
  const int s = slot_row[k];
  const int j = col[k];
  double v = inv_deg[s];                          // l = 0: p_0(s,s)/d_s, p_0(j,s) = 0
  if (include_l1 && tau[k] >= 1)
    v -= inv_deg[j] * inv_deg[s];                 // l = 1: p_1(s,s) = 0, p_1(j,s) = 1/d_j
  gacc[k] = v;
}

// ------------------------------------------------------------------ truncation lengths
__device__ inline int odd_at_least(double f) {
  long long k = static_cast<long long>(ceil(f));
  if (k < 1) k = 1;
  if ((k & 1) == 0) ++k;
  return k > INT_MAX ? INT_MAX : static_cast<int>(k);
}

__global__ void k_tau(int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                      const int32_t* __restrict__ deg, int L, double eps_tau, double lam,
                      int max_L, int32_t* __restrict__ tau_slot, int32_t* __restrict__ tau_row) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  int tmax = 0;
  const double di = static_cast<double>(deg[x]);
  for (int k = rowptr[x]; k < rowptr[x + 1]; ++k) {
    int t;
    if (L > 0) {
      t = L;
    } else {
      const double dj = static_cast<double>(deg[col[k]]);
      const double num = 1.0 / di + 1.0 / dj - 2.0 / (di * dj);
      const double f = ceil(log(num / (eps_tau * (1.0 - lam * lam))) / log(1.0 / lam) - 1.0);
      t = odd_at_least(f);
      if (t > max_L) t = max_L;
    }
    tau_slot[k] = t;
    tmax = t > tmax ? t : tmax;
  }
  tau_row[x] = tmax;
}

// ------------------------------------------------------------------ indicator masks
// One wave per source column; lanes stride over N(s).
// anymask holds one bit per node: set when any column of the block marks it.
__global__ void k_mask_set(int n, int s0, int B, const int32_t* __restrict__ rowptr,
                           const int32_t* __restrict__ col, unsigned long long* mask,
                           unsigned* anymask, int clear) {
  const int c = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int s = s0 + c;
  if (c >= B || s >= n) return;
  const unsigned long long bit = 1ull << c;
  for (int k = rowptr[s] + lane; k < rowptr[s + 1]; k += 64) {
    const int u = col[k];
    if (clear) {
      // every bit still set belongs to this block, so whole words can be cleared
      mask[u] = 0ull;
      anymask[u >> 5] = 0u;
    } else {
      atomicOr(&mask[u], bit);
      atomicOr(&anymask[u >> 5], 1u << (u & 31));
    }
  }
}

// ------------------------------------------------------------------ wave helpers
template <typename T, int B>
__device__ inline T reduce_groups(T v) {
  // lanes c, c+B, c+2B, ... hold partial sums of column c; butterfly in a fixed order
#pragma unroll
  for (int off = B; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// wave-uniform broadcast of lane jj's value through a scalar register
__device__ inline float bcast(float v, int jj) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), jj));
}
__device__ inline double bcast(double v, int jj) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xFFFFFFFFll), jj);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), jj);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}

// ------------------------------------------------------------------ Y2 from masks
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_twohop(const Task* __restrict__ tasks, int ntasks,
                                                     const int32_t* __restrict__ col,
                                                     const T* __restrict__ inv_deg,
                                                     const unsigned long long* __restrict__ mask,
                                                     const unsigned* __restrict__ anymask,
                                                     T* __restrict__ Y, T* __restrict__ partials) {
  constexpr int G = 64 / B;
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (t >= ntasks) return;
  const Task tk = tasks[t];
  const int c = lane % B;
  const int gq = lane / B;
  T acc = T(0);
  for (int base = tk.beg; base < tk.end; base += 64) {
    const int cnt = min(64, tk.end - base);
    const int myu = lane < cnt ? col[base + lane] : 0;
    // the small bitmap filters out the neighbours no column marks
    const bool hit = lane < cnt && ((anymask[myu >> 5] >> (myu & 31)) & 1u);
    const unsigned long long mym = hit ? mask[myu] : 0ull;
    const T myw = hit ? inv_deg[myu] : T(0);
    if (__ballot(hit) == 0ull) continue;
    if (G == 1) {
      // one row per wave: broadcast each neighbour's mask and weight through
      // scalar registers
      const int mlo = static_cast<int>(mym & 0xFFFFFFFFull);
      const int mhi = static_cast<int>(mym >> 32);
      for (int jj = 0; jj < cnt; ++jj) {
        const unsigned long long mk =
            (static_cast<unsigned long long>(static_cast<unsigned>(__builtin_amdgcn_readlane(mhi, jj))) << 32) |
            static_cast<unsigned>(__builtin_amdgcn_readlane(mlo, jj));
        if ((mk >> c) & 1ull) acc += bcast(myw, jj);
      }
    } else {
      // uniform trip count: every lane takes part in each shuffle (a shuffle
      // from an inactive lane would read 0), the add is predicated instead
      for (int j0 = 0; j0 < cnt; j0 += G) {
        const int jj = j0 + gq;
        const unsigned long long mk = __shfl(mym, jj, 64);
        const T w = __shfl(myw, jj, 64);
        if (jj < cnt && ((mk >> c) & 1ull)) acc += w;
      }
    }
  }
  acc = reduce_groups<T, B>(acc);
  if (gq == 0) {
    if (tk.part < 0)
      Y[static_cast<size_t>(tk.row) * B + c] = acc * inv_deg[tk.row];
    else
      partials[static_cast<size_t>(tk.part) * B + c] = acc;
  }
}

// ------------------------------------------------------------------ dense propagation
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_propagate(const Task* __restrict__ tasks,
                                                        int ntasks,
                                                        const int32_t* __restrict__ col,
                                                        const T* __restrict__ inv_deg,
                                                        const T* __restrict__ Yp,
                                                        T* __restrict__ Yn,
                                                        T* __restrict__ partials) {
  constexpr int G = 64 / B;
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (t >= ntasks) return;
  const Task tk = tasks[t];
  const int c = lane % B;
  const int gq = lane / B;
  T acc = T(0);
  for (int base = tk.beg; base < tk.end; base += 64) {
    const int cnt = min(64, tk.end - base);
    const int myu = lane < cnt ? col[base + lane] : 0;
    if (G == 1) {
      int jj = 0;
      for (; jj + 8 <= cnt; jj += 8) {
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int u = __builtin_amdgcn_readlane(myu, jj + q);
          v[q] = Yp[static_cast<size_t>(u) * B + c];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q];
      }
      for (; jj < cnt; ++jj) {
        const int u = __builtin_amdgcn_readlane(myu, jj);
        acc += Yp[static_cast<size_t>(u) * B + c];
      }
    } else {
      for (int j0 = 0; j0 < cnt; j0 += G) {   // uniform trip count, see k_twohop
        const int jj = j0 + gq;
        const int u = __shfl(myu, jj, 64);
        if (jj < cnt) acc += Yp[static_cast<size_t>(u) * B + c];
      }
    }
  }
  acc = reduce_groups<T, B>(acc);
  if (gq == 0) {
    if (tk.part < 0)
      Yn[static_cast<size_t>(tk.row) * B + c] = acc * inv_deg[tk.row];
    else
      partials[static_cast<size_t>(tk.part) * B + c] = acc;
  }
}

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_fixup(const HeavyRow* __restrict__ heavy,
                                                    int nheavy, const T* __restrict__ inv_deg,
                                                    const T* __restrict__ partials,
                                                    T* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int h = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (h >= nheavy || lane >= B) return;
  const HeavyRow hr = heavy[h];
  T acc = T(0);
  for (int p = 0; p < hr.nparts; ++p) acc += partials[static_cast<size_t>(hr.part0 + p) * B + lane];
  Y[static_cast<size_t>(hr.row) * B + lane] = acc * inv_deg[hr.row];
}

// ------------------------------------------------------------------ per-step accumulation (Eq. 9)
template <typename T, int B>
__global__ void k_accumulate(int kbeg, int kend, int s0, int ell,
                             const int32_t* __restrict__ slot_row,
                             const int32_t* __restrict__ col, const double* __restrict__ inv_deg,
                             const T* __restrict__ Y, const int32_t* __restrict__ tau,
                             double* __restrict__ gacc) {
  const int k = kbeg + blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kend) return;
  if (ell > tau[k]) return;
  const int s = slot_row[k];
  const int c = s - s0;
  const int j = col[k];
  const double pss = static_cast<double>(Y[static_cast<size_t>(s) * B + c]);
  const double pjs = static_cast<double>(Y[static_cast<size_t>(j) * B + c]);
  gacc[k] += (pss - pjs) * inv_deg[s];
}

// ------------------------------------------------------------------ combine and traces
__global__ void k_combine(int64_t m, const int32_t* __restrict__ half_slot,
                          const double* __restrict__ gacc, double* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  out[e] = gacc[half_slot[e]] + gacc[half_slot[e + m]];
}

__global__ void k_trace(int64_t m, const int32_t* __restrict__ half_slot,
                        const int32_t* __restrict__ tau_slot, const int64_t* __restrict__ nr_slot,
                        int32_t* __restrict__ tau_out, int64_t* __restrict__ nr_out) {
  const int64_t h = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (h >= 2 * m) return;
  const int k = half_slot[h];
  if (tau_out && h < m) tau_out[h] = tau_slot[k];
  if (nr_out) nr_out[h] = nr_slot ? nr_slot[k] : 0;
}

// ------------------------------------------------------------------ Lanczos helpers
__global__ __launch_bounds__(kThreads) void k_nmat_spmv(int n, const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ sid,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (r >= n) return;
  double acc = 0.0;
  for (int k = rowptr[r] + lane; k < rowptr[r + 1]; k += 64) {
    const int u = col[k];
    acc += sid[u] * x[u];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[r] = sid[r] * acc;
}

__global__ __launch_bounds__(256) void k_multi_dot(const double* __restrict__ V, int64_t ld,
                                                   const double* __restrict__ w, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const double* vj = V + static_cast<size_t>(j) * ld;
  double acc = 0.0;
  for (int64_t x = threadIdx.x; x < n; x += 256) acc += vj[x] * w[x];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

__global__ void k_multi_axpy(const double* __restrict__ V, int ncols, int64_t ld,
                             const double* __restrict__ h, double* __restrict__ w, int64_t n) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= n) return;
  double acc = 0.0;
  for (int j = 0; j < ncols; ++j) acc += V[static_cast<size_t>(j) * ld + x] * h[j];
  w[x] -= acc;
}

}  // namespace

// ====================================================================== wrappers

hipError_t launch_gacc_init(const DeviceGraph& g, const int32_t* tau_slot, int include_l1,
                            double* gacc, hipStream_t st) {
  const int64_t ns = g.nslots;
  k_gacc_init<<<grid_for(ns, 256), 256, 0, st>>>(ns, g.slot_row, g.col, g.inv_deg_d, tau_slot,
                                                  include_l1, gacc);
  return hipGetLastError();
}

hipError_t launch_tau(const DeviceGraph& g, int L, double eps_tau, double lam, int max_L,
                      int32_t* tau_slot, int32_t* tau_row, hipStream_t st) {
  k_tau<<<grid_for(g.n, 256), 256, 0, st>>>(g.n, g.rowptr, g.col, g.deg, L, eps_tau, lam, max_L,
                                             tau_slot, tau_row);
  return hipGetLastError();
}

hipError_t launch_mask_set(const DeviceGraph& g, int s0, int B, unsigned long long* mask,
                           unsigned* anymask, bool clear, hipStream_t st) {
  k_mask_set<<<grid_for(B, kWavesPerBlock), kThreads, 0, st>>>(g.n, s0, B, g.rowptr, g.col, mask,
                                                               anymask, clear ? 1 : 0);
  return hipGetLastError();
}

#define SC_DISPATCH_B(B, CALL)             \
  switch (B) {                             \
    case 64: { constexpr int kB = 64; CALL; } break; \
    case 32: { constexpr int kB = 32; CALL; } break; \
    case 16: { constexpr int kB = 16; CALL; } break; \
    default: return hipErrorInvalidValue;  \
  }

template <typename T>
const T* inv_deg_of(const DeviceGraph& g);
template <>
const float* inv_deg_of<float>(const DeviceGraph& g) { return g.inv_deg_f; }
template <>
const double* inv_deg_of<double>(const DeviceGraph& g) { return g.inv_deg_d; }

template <typename T>
hipError_t launch_twohop(const DeviceGraph& g, int B, const unsigned long long* mask,
                         const unsigned* anymask, T* Y, T* partials, hipStream_t st) {
  SC_DISPATCH_B(B, (k_twohop<T, kB><<<grid_for(g.ntasks, kWavesPerBlock), kThreads, 0, st>>>(
                        g.tasks, g.ntasks, g.col, inv_deg_of<T>(g), mask, anymask, Y, partials)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_propagate(const DeviceGraph& g, int B, const T* Yp, T* Yn, T* partials,
                            hipStream_t st) {
  SC_DISPATCH_B(B, (k_propagate<T, kB><<<grid_for(g.ntasks, kWavesPerBlock), kThreads, 0, st>>>(
                        g.tasks, g.ntasks, g.col, inv_deg_of<T>(g), Yp, Yn, partials)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fixup(const DeviceGraph& g, int B, const T* partials, T* Y, hipStream_t st) {
  if (g.nheavy == 0) return hipSuccess;
  SC_DISPATCH_B(B, (k_fixup<T, kB><<<grid_for(g.nheavy, kWavesPerBlock), kThreads, 0, st>>>(
                        g.heavy, g.nheavy, inv_deg_of<T>(g), partials, Y)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_accumulate(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int ell,
                             const T* Y, const int32_t* tau_slot, double* gacc, hipStream_t st) {
  if (kend <= kbeg) return hipSuccess;
  SC_DISPATCH_B(B, (k_accumulate<T, kB><<<grid_for(kend - kbeg, 256), 256, 0, st>>>(
                        kbeg, kend, s0, ell, g.slot_row, g.col, g.inv_deg_d, Y, tau_slot, gacc)));
  return hipGetLastError();
}

hipError_t launch_combine(const DeviceGraph& g, const double* gacc, double* out,
                          hipStream_t st) {
  k_combine<<<grid_for(g.m, 256), 256, 0, st>>>(g.m, g.half_slot, gacc, out);
  return hipGetLastError();
}

hipError_t launch_trace(const DeviceGraph& g, const int32_t* tau_slot, const int64_t* nr_slot,
                        int32_t* tau_out, int64_t* nr_out, hipStream_t st) {
  if (!tau_out && !nr_out) return hipSuccess;
  k_trace<<<grid_for(2 * g.m, 256), 256, 0, st>>>(g.m, g.half_slot, tau_slot, nr_slot, tau_out,
                                                   nr_out);
  return hipGetLastError();
}

hipError_t launch_nmat_spmv(const DeviceGraph& g, const double* sid, const double* x, double* y,
                            hipStream_t st) {
  k_nmat_spmv<<<grid_for(g.n, kWavesPerBlock), kThreads, 0, st>>>(g.n, g.rowptr, g.col, sid, x, y);
  return hipGetLastError();
}

hipError_t launch_multi_dot(const double* V, int ncols, int64_t ld, const double* w, int64_t n,
                            double* out, hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  k_multi_dot<<<ncols, 256, 0, st>>>(V, ld, w, n, out);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(const double* V, int ncols, int64_t ld, const double* h, double* w,
                             int64_t n, hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  k_multi_axpy<<<grid_for(n, 256), 256, 0, st>>>(V, ncols, ld, h, w, n);
  return hipGetLastError();
}

template hipError_t launch_twohop<float>(const DeviceGraph&, int, const unsigned long long*,
                                         const unsigned*, float*, float*, hipStream_t);
template hipError_t launch_twohop<double>(const DeviceGraph&, int, const unsigned long long*,
                                          const unsigned*, double*, double*, hipStream_t);
template hipError_t launch_propagate<float>(const DeviceGraph&, int, const float*, float*,
                                            float*, hipStream_t);
template hipError_t launch_propagate<double>(const DeviceGraph&, int, const double*, double*,
                                             double*, hipStream_t);
template hipError_t launch_fixup<float>(const DeviceGraph&, int, const float*, float*,
                                        hipStream_t);
template hipError_t launch_fixup<double>(const DeviceGraph&, int, const double*, double*,
                                         hipStream_t);
template hipError_t launch_accumulate<float>(const DeviceGraph&, int, int, int, int, int,
                                             const float*, const int32_t*, double*, hipStream_t);
template hipError_t launch_accumulate<double>(const DeviceGraph&, int, int, int, int, int,
                                              const double*, const int32_t*, double*, hipStream_t);

}  // namespace sc
