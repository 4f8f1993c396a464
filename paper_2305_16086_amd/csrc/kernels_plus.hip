// TGT+ kernels (Section 4): candidate bound of Algorithm 3, walk counts of
// Eq. 13, and the random-walk tail estimator of Eq. 11.
//
// All floating-point reductions use fixed orders; the walk randomness is a
// pure function of (seed, i, j, r, side, step) so results do not depend on
// the thread schedule.
#include "philox.hpp"
#include "sc_internal.hpp"

#include <cfloat>
#include <climits>

namespace sc {

namespace {

constexpr int kThreads = 64 * kWavesPerBlock;

inline unsigned grid_for(int64_t items, int per_block) {
  return static_cast<unsigned>((items + per_block - 1) / per_block);
}

// (value desc, id asc) ordering of Algorithm 3 line 2
__device__ inline bool ranks_before(double va, int ia, double vb, int ib) {
  return va > vb || (va == vb && ia < ib);
}

__device__ inline bool adjacent(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                int a, int b) {
  int lo = rowptr[a], hi = rowptr[a + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int v = col[mid];
    if (v == b) return true;
    if (v < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return false;
}

// One workgroup per source column c of the block.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_colstats(int n, int s0, int gamma,
                                                  const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col,
                                                  const T* __restrict__ Y,
                                                  ColStats* __restrict__ cs) {
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ int so[256];
  __shared__ double top_v[kMaxGamma];
  __shared__ int top_i[kMaxGamma];
  __shared__ double red_a[256];
  __shared__ double red_b[256];

  const int c = blockIdx.x;
  const int s = s0 + c;
  const int tid = threadIdx.x;

  double lv[kMaxGamma];
  int li[kMaxGamma];
#pragma unroll
  for (int p = 0; p < kMaxGamma; ++p) {
    lv[p] = -DBL_MAX;
    li[p] = INT_MAX;
  }
  double last = -DBL_MAX;   // value at position gamma-1 of this thread's list
  double mx = -DBL_MAX, mn = DBL_MAX;
  for (int x = tid; x < n; x += 256) {
    const double q = static_cast<double>(Y[static_cast<size_t>(x) * B + c]);
    mx = fmax(mx, q);
    mn = fmin(mn, q);
    if (gamma > 0 && q > last) {
      // ids increase along this thread's scan, so an equal value never outranks
      double cv = q;
      int ci = x;
#pragma unroll
      for (int p = 0; p < kMaxGamma; ++p) {
        if (p < gamma && ranks_before(cv, ci, lv[p], li[p])) {
          const double tv = lv[p];
          const int ti = li[p];
          lv[p] = cv;
          li[p] = ci;
          cv = tv;
          ci = ti;
        }
      }
#pragma unroll
      for (int p = 0; p < kMaxGamma; ++p)
        if (p == gamma - 1) last = lv[p];
    }
  }

  // extremes over V
  red_a[tid] = mx;
  red_b[tid] = mn;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) {
      red_a[tid] = fmax(red_a[tid], red_a[tid + w]);
      red_b[tid] = fmin(red_b[tid], red_b[tid + w]);
    }
    __syncthreads();
  }
  const double maxV = red_a[0];
  const double minV = red_b[0];
  __syncthreads();

  // merge the per-thread candidate lists: gamma rounds of a workgroup argmax
  const int cnt = gamma < n ? gamma : n;
  int head = 0;
  for (int r = 0; r < cnt; ++r) {
    double hv = -DBL_MAX;
    int hi = INT_MAX;
#pragma unroll
    for (int p = 0; p < kMaxGamma; ++p)
      if (p == head) {
        hv = lv[p];
        hi = li[p];
      }
    sv[tid] = hv;
    si[tid] = hi;
    so[tid] = tid;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if (tid < w && ranks_before(sv[tid + w], si[tid + w], sv[tid], si[tid])) {
        sv[tid] = sv[tid + w];
        si[tid] = si[tid + w];
        so[tid] = so[tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      top_v[r] = sv[0];
      top_i[r] = si[0];
    }
    if (so[0] == tid) ++head;
    __syncthreads();
  }

  // rho bound: best candidate-pair edge, and q[c1] + q[c_gamma] for edges
  // leaving the candidate set (Algorithm 3 lines 3-5, safe reading)
  double best = -DBL_MAX;
  if (gamma > 0) {
    for (int p = tid; p < cnt * cnt; p += 256) {
      const int a = p / cnt, b = p % cnt;
      if (a < b && adjacent(rowptr, col, top_i[a], top_i[b])) best = fmax(best, top_v[a] + top_v[b]);
    }
  }
  // extremes over N(s)
  double nmx = -DBL_MAX, nmn = DBL_MAX;
  for (int k = rowptr[s] + tid; k < rowptr[s + 1]; k += 256) {
    const double q = static_cast<double>(Y[static_cast<size_t>(col[k]) * B + c]);
    nmx = fmax(nmx, q);
    nmn = fmin(nmn, q);
  }
  __syncthreads();
  red_a[tid] = nmx;
  red_b[tid] = nmn;
  sv[tid] = best;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) {
      red_a[tid] = fmax(red_a[tid], red_a[tid + w]);
      red_b[tid] = fmin(red_b[tid], red_b[tid + w]);
      sv[tid] = fmax(sv[tid], sv[tid + w]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    ColStats o;
    o.maxV = maxV;
    o.minV = minV;
    o.rho = gamma > 0 ? fmax(sv[0], top_v[0] + top_v[cnt - 1]) : 0.0;
    o.maxN = red_a[0];
    o.minN = red_b[0];
    cs[c] = o;
  }
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per slot k = (s -> j) of the block.
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_walk_counts(
    int kbeg, int kend, int s0, int tilde, int gamma, double coef, long long nr_cap,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ slot_row, const int32_t* __restrict__ deg, const T* __restrict__ Y,
    const ColStats* __restrict__ cs, const int32_t* __restrict__ tau, long long* __restrict__ nr,
    unsigned long long* __restrict__ work) {
  const int lane = threadIdx.x & 63;
  const int k = kbeg + blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (k >= kend) return;
  const int len = tau[k] - tilde;
  if (len <= 0) {
    if (lane == 0) nr[k] = 0;
    return;
  }
  const int s = slot_row[k];
  const int c = s - s0;
  const int j = col[k];
  double jmx = -DBL_MAX, jmn = DBL_MAX;
  for (int kk = rowptr[j] + lane; kk < rowptr[j + 1]; kk += 64) {
    const double q = static_cast<double>(Y[static_cast<size_t>(col[kk]) * B + c]);
    jmx = fmax(jmx, q);
    jmn = fmin(jmn, q);
  }
  jmx = wave_max(jmx);
  jmn = wave_min(jmn);
  if (lane != 0) return;
  const ColStats st = cs[c];
  double chi;
  if (gamma > 0) {
    // Lemma 4.3 bounds for both walks (both scored with q = p_tilde(., s)), Eq. 17
    const double lb_i = st.minN + (len - 1) * st.minV;
    const double ub_i = st.maxN * 0.5 + st.maxV * 0.5 + (len - 1) * st.rho * 0.5;
    const double lb_j = jmn + (len - 1) * st.minV;
    const double ub_j = jmx * 0.5 + st.maxV * 0.5 + (len - 1) * st.rho * 0.5;
    chi = ub_i + ub_j - lb_i - lb_j;
  } else {
    chi = 2.0 * len * (st.maxV - st.minV);   // Eq. 15
  }
  const double d = static_cast<double>(deg[s]);
  const double R = coef * chi * chi / (d * d);   // Eq. 13
  double r = ceil(R);
  if (!(r >= 1.0)) r = 1.0;
  long long w = r > static_cast<double>(nr_cap) ? nr_cap : static_cast<long long>(r);
  nr[k] = w;
  atomicAdd(&work[0], static_cast<unsigned long long>(w));
  atomicAdd(&work[1], static_cast<unsigned long long>(w) * 2ull * static_cast<unsigned long long>(len));
}

// One wave per slot; lanes take walk pairs r = lane, lane + 64, ...
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_walks(
    int kbeg, int kend, int s0, int tilde, unsigned k0, unsigned k1,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ slot_row, const int32_t* __restrict__ deg,
    const double* __restrict__ inv_deg, const T* __restrict__ Y, const int32_t* __restrict__ tau,
    const long long* __restrict__ nr, double* __restrict__ gacc) {
  const int lane = threadIdx.x & 63;
  const int k = kbeg + blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (k >= kend) return;
  const long long n_r = nr[k];
  if (n_r <= 0) return;
  const int len = tau[k] - tilde;
  const int s = slot_row[k];
  const int c = s - s0;
  const int j = col[k];
  double acc = 0.0;
  for (long long r = lane; r < n_r; r += 64) {
    double S[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int pos = side == 0 ? s : j;
      double sum = 0.0;
      U32x4 words;
      for (int t = 0; t < len; ++t) {
        if ((t & 3) == 0)
          words = philox4x32_10(static_cast<uint32_t>(s), static_cast<uint32_t>(j),
                                static_cast<uint32_t>(r),
                                (static_cast<uint32_t>(side) << 31) | static_cast<uint32_t>(t >> 2),
                                k0, k1);
        const uint32_t w = words.w[t & 3];
        const int d = deg[pos];
        pos = col[rowptr[pos] + static_cast<int>(pick_neighbour(w, static_cast<uint32_t>(d)))];
        sum += static_cast<double>(Y[static_cast<size_t>(pos) * B + c]);
      }
      S[side] = sum;
    }
    acc += (S[0] - S[1]) * inv_deg[s];   // X of Eq. 11
  }
  acc = wave_sum(acc);
  if (lane == 0) gacc[k] += acc / static_cast<double>(n_r);
}

}  // namespace

#define SC_DISPATCH_B(B, CALL)                        \
  switch (B) {                                        \
    case 64: { constexpr int kB = 64; CALL; } break;  \
    case 32: { constexpr int kB = 32; CALL; } break;  \
    case 16: { constexpr int kB = 16; CALL; } break;  \
    default: return hipErrorInvalidValue;             \
  }

template <typename T>
hipError_t launch_colstats(const DeviceGraph& g, int s0, int B, int gamma, const T* Y,
                           ColStats* cs, hipStream_t st) {
  int ncols = B;
  if (s0 + ncols > g.n) ncols = g.n - s0;
  if (ncols <= 0) return hipSuccess;
  if (gamma > kMaxGamma) return hipErrorInvalidValue;
  SC_DISPATCH_B(B, (k_colstats<T, kB><<<ncols, 256, 0, st>>>(g.n, s0, gamma, g.rowptr, g.col, Y,
                                                              cs)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_walk_counts(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int tilde,
                              int gamma, double coef, int64_t nr_cap, const T* Y,
                              const ColStats* cs, const int32_t* tau_slot, int64_t* nr_slot,
                              unsigned long long* work, hipStream_t st) {
  if (kend <= kbeg) return hipSuccess;
  SC_DISPATCH_B(B, (k_walk_counts<T, kB><<<grid_for(kend - kbeg, kWavesPerBlock), kThreads, 0,
                                          st>>>(
                        kbeg, kend, s0, tilde, gamma, coef, static_cast<long long>(nr_cap),
                        g.rowptr, g.col, g.slot_row, g.deg, Y, cs, tau_slot,
                        reinterpret_cast<long long*>(nr_slot), work)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_walks(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int tilde,
                        uint64_t seed, const T* Y, const int32_t* tau_slot,
                        const int64_t* nr_slot, double* gacc, hipStream_t st) {
  if (kend <= kbeg) return hipSuccess;
  const unsigned k0 = static_cast<unsigned>(seed & 0xFFFFFFFFull);
  const unsigned k1 = static_cast<unsigned>(seed >> 32);
  SC_DISPATCH_B(B, (k_walks<T, kB><<<grid_for(kend - kbeg, kWavesPerBlock), kThreads, 0, st>>>(
                        kbeg, kend, s0, tilde, k0, k1, g.rowptr, g.col, g.slot_row, g.deg,
                        g.inv_deg_d, Y, tau_slot, reinterpret_cast<const long long*>(nr_slot),
                        gacc)));
  return hipGetLastError();
}

template hipError_t launch_colstats<float>(const DeviceGraph&, int, int, int, const float*,
                                           ColStats*, hipStream_t);
template hipError_t launch_colstats<double>(const DeviceGraph&, int, int, int, const double*,
                                            ColStats*, hipStream_t);
template hipError_t launch_walk_counts<float>(const DeviceGraph&, int, int, int, int, int, int,
                                              double, int64_t, const float*, const ColStats*,
                                              const int32_t*, int64_t*, unsigned long long*,
                                              hipStream_t);
template hipError_t launch_walk_counts<double>(const DeviceGraph&, int, int, int, int, int, int,
                                               double, int64_t, const double*, const ColStats*,
                                               const int32_t*, int64_t*, unsigned long long*,
                                               hipStream_t);
template hipError_t launch_walks<float>(const DeviceGraph&, int, int, int, int, int, uint64_t,
                                        const float*, const int32_t*, const int64_t*, double*,
                                        hipStream_t);
template hipError_t launch_walks<double>(const DeviceGraph&, int, int, int, int, int, uint64_t,
                                         const double*, const int32_t*, const int64_t*, double*,
                                         hipStream_t);

}  // namespace sc
