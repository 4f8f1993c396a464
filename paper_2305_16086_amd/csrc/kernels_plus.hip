// TGT+ kernels (Section 4): candidate bound of Algorithm 3, walk counts of
// Eq. 13, and the random-walk tail estimator of Eq. 11.
//
// All floating-point reductions use fixed orders; the walk randomness is a
// pure function of (seed, i, j, r, side, step) so results do not depend on
// the thread schedule.
#include "philox.hpp"
#include "sc_internal.hpp"
#include "accumulate.hpp"

#include <cfloat>
#include <climits>

namespace sc {

namespace {

constexpr int kThreads = 64 * kWavesPerBlock;
constexpr int kWalkBlocks = 2048;   // persistent grid of the flattened walks

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


// Insert (v, id) into a list kept in (value desc, id asc) order; the last
// entry falls off.  Fully unrolled so the list stays in registers.
__device__ inline void list_insert(double (&lv)[kMaxGamma], int (&li)[kMaxGamma], int gamma,
                                   double v, int id) {
  double cv = v;
  int ci = id;
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
}

__device__ inline void list_last(const double (&lv)[kMaxGamma], const int (&li)[kMaxGamma],
                                 int gamma, double* v, int* id) {
#pragma unroll
  for (int p = 0; p < kMaxGamma; ++p)
    if (p == gamma - 1) {
      *v = lv[p];
      *id = li[p];
    }
}

// The per-column summary of Algorithm 3 runs in four passes over the block
// state Y (lanes are columns, rows are cut into kColParts chunks):
//  A  chunk maxima and minima (one coalesced read of Y);
//  B  per column: overall extremes and theta = the gamma-th largest chunk
//     maximum.  The gamma largest chunk maxima are gamma distinct entries, so
//     every entry of the column's top-gamma list is >= theta;
//  C  chunks whose maximum reaches theta keep their top-gamma entries >= theta
//     and register themselves with the column;
//  D  per column: merge the registered lists, test candidate pairs for edges
//     (Algorithm 3 lines 3-5, safe reading), extremes over N(s).
// Chunk p of column c: pmx/pmn[c*kColParts + p], lists pv/pi[(p*B + c)*gamma + r].

// Slot kbeg + i of a finished block: add its chunk sums in chunk order, divided
// by n_r (nothing when the block walked one slot per wave: ctl[1] == 0).
__device__ inline void walk_finish_slot(const FinishJob& f, int i) {
  if (f.ctl[1] == 0 || i >= f.kend - f.kbeg) return;
  const long long n_r = f.nr[f.kbeg + i];
  if (n_r <= 0) return;
  double acc = 0.0;
  for (long long c = f.chunk_off[i]; c < f.chunk_off[i + 1]; ++c) acc += f.part[c];
  f.gacc[f.kbeg + i] += acc / static_cast<double>(n_r);
}

// Workgroups after col_blocks carry the accumulation of the step held in Y
// (acc; Algorithm 2 lines 10-11) and then a previous block's walk finish (fin),
// saving launches.
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_colmax(int n, int rows_per_part, int nparts,
                                                     const T* __restrict__ Y,
                                                     T* __restrict__ pmx, T* __restrict__ pmn,
                                                     int col_blocks, AccJob acc, int acc_blocks,
                                                     FinishJob fin,
                                                     const int32_t* __restrict__ slot_row,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ inv_deg_d) {
  if (static_cast<int>(blockIdx.x) >= col_blocks) {
    const int t = static_cast<int>(blockIdx.x) - col_blocks;
    if (t < acc_blocks) {
      const int k = acc.kbeg + t * kThreads + threadIdx.x;
      accumulate_half<T, B>(acc, slot_row, col, inv_deg_d, Y, k);
    } else {
      walk_finish_slot(fin, (t - acc_blocks) * kThreads + static_cast<int>(threadIdx.x));
    }
    return;
  }
  constexpr int G = 64 / B;
  __shared__ T smx[kThreads], smn[kThreads];
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int c = lane % B;
  const int part = wave * G + lane / B;
  const int x0 = part * rows_per_part;
  const int x1 = min(n, x0 + rows_per_part);
  T mx = T(-1), mn = T(2);   // probabilities lie in [0, 1]: -1 / 2 mark an empty chunk
  for (int xb = x0; xb < x1; xb += 8) {
    T q[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
      q[r] = (xb + r < x1) ? Y[static_cast<size_t>(xb + r) * B + c] : T(-1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (xb + r < x1) {
        mx = q[r] > mx ? q[r] : mx;
        mn = q[r] < mn ? q[r] : mn;
      }
    }
  }
  // entry (local part pl, column c) sits at pl * B + c == threadIdx.x; store
  // column-major so each column's chunk values are contiguous
  smx[threadIdx.x] = mx;
  smn[threadIdx.x] = mn;
  __syncthreads();
  constexpr int kParts = kWavesPerBlock * G;   // parts of this workgroup
  const int cc = threadIdx.x / kParts;
  const int pl = threadIdx.x % kParts;
  const int p0 = blockIdx.x * kParts;
  pmx[static_cast<size_t>(cc) * nparts + p0 + pl] = smx[pl * B + cc];
  pmn[static_cast<size_t>(cc) * nparts + p0 + pl] = smn[pl * B + cc];
}

__device__ inline void wave_best(double& v, int& id, int& owner) {
  // (value desc, id asc) arg-best over the wave, fixed butterfly
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(id, off, 64);
    const int oo = __shfl_xor(owner, off, 64);
    if (ranks_before(ov, oi, v, id)) {
      v = ov;
      id = oi;
      owner = oo;
    }
  }
}

// Pass B: one workgroup of kThreshWaves waves per column.  Each wave takes
// kColParts / kThreshWaves chunk maxima, keeps its gamma largest (with
// multiplicity), and the first wave picks theta = the gamma-th largest of all
// from those lists.  Then the chunks whose maximum reaches theta (and is not
// empty) are listed in ascending chunk order: act[c*kColParts + k], nact[c].
constexpr int kThreshWaves = 4;

template <typename T, int B>
__global__ __launch_bounds__(64 * kThreshWaves) void k_colthresh(
    int gamma, int nparts, const T* __restrict__ pmx, const T* __restrict__ pmn,
    T* __restrict__ thr, int* __restrict__ nact, int* __restrict__ act, ColStats* __restrict__ cs) {
  constexpr int kPer = kColParts / (64 * kThreshWaves);
  __shared__ double s_top[kThreshWaves][kMaxGamma];
  __shared__ double s_mx[kThreshWaves], s_mn[kThreshWaves];
  __shared__ double s_theta;
  __shared__ int s_cnt[kThreshWaves];
  const int c = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double v[kPer];
  double mx = -DBL_MAX, mn = DBL_MAX;
  {
    double w[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {   // all loads issued before any use
      const int p = wave * (kPer * 64) + k * 64 + lane;
      const size_t o = static_cast<size_t>(c) * nparts + (p < nparts ? p : 0);
      v[k] = p < nparts ? static_cast<double>(pmx[o]) : -1.0;
      w[k] = p < nparts ? static_cast<double>(pmn[o]) : 2.0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      // empty chunks carry max -1 and min 2, outside [0, 1]
      mx = fmax(mx, v[k]);
      mn = fmin(mn, w[k]);
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    mn = fmin(mn, __shfl_xor(mn, off, 64));
  }
  // this wave's gamma largest chunk maxima
  {
    double r[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) r[k] = v[k];
    for (int q = 0; q < gamma; ++q) {
      double best = -1.0;
      int at = -1;
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (r[k] > best) {
          best = r[k];
          at = k;
        }
      double wbest = best;
      int wlane = lane;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(wbest, off, 64);
        const int ol = __shfl_xor(wlane, off, 64);
        if (ob > wbest || (ob == wbest && ol < wlane)) {
          wbest = ob;
          wlane = ol;
        }
      }
      if (lane == 0) s_top[wave][q] = wbest;
      if (lane == wlane) {
#pragma unroll
        for (int k = 0; k < kPer; ++k)
          if (k == at) r[k] = -1.0;
      }
    }
  }
  if (lane == 0) {
    s_mx[wave] = mx;
    s_mn[wave] = mn;
  }
  __syncthreads();
  if (wave == 0) {
    // theta over the kThreshWaves lists (lane = candidate)
    double cand = -1.0;
    if (lane < kThreshWaves * gamma) cand = s_top[lane / gamma][lane % gamma];
    double theta = -1.0;
    for (int q = 0; q < gamma; ++q) {
      double wbest = cand;
      int wlane = lane;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(wbest, off, 64);
        const int ol = __shfl_xor(wlane, off, 64);
        if (ob > wbest || (ob == wbest && ol < wlane)) {
          wbest = ob;
          wlane = ol;
        }
      }
      if (wbest < 0.0) {   // fewer than gamma non-empty chunks: keep every entry
        theta = -1.0;
        break;
      }
      theta = wbest;
      if (lane == wlane) cand = -1.0;
    }
    if (lane == 0) {
      s_theta = theta;
      double gmx = s_mx[0], gmn = s_mn[0];
      for (int q = 1; q < kThreshWaves; ++q) {
        gmx = fmax(gmx, s_mx[q]);
        gmn = fmin(gmn, s_mn[q]);
      }
      thr[c] = static_cast<T>(theta);
      cs[c].maxV = gmx;
      cs[c].minV = gmn;
    }
  }
  __syncthreads();
  // active chunks in ascending order
  const double theta = s_theta;
  unsigned long long bal[kPer];
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const T tv = static_cast<T>(theta);
    const bool on = v[k] >= 0.0 && static_cast<T>(v[k]) >= tv;
    bal[k] = __ballot(on);
    cnt += __popcll(bal[k]);
  }
  if (lane == 0) s_cnt[wave] = cnt;
  __syncthreads();
  int base = 0;
  for (int q = 0; q < wave; ++q) base += s_cnt[q];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if ((bal[k] >> lane) & 1ull) {
      const int idx = base + __popcll(bal[k] & ((1ull << lane) - 1ull));
      act[static_cast<size_t>(c) * kColParts + idx] = wave * (kPer * 64) + k * 64 + lane;
    }
    base += __popcll(bal[k]);
  }
  if (threadIdx.x == 64 * kThreshWaves - 1) nact[c] = base;
}

// Pass C: kScanWaves waves per column walk the column's active chunks; for
// each, the lanes take 64 rows at a time and the wave keeps the gamma best
// entries (value desc, id asc) that reach theta, in lanes 0..gamma-1.
constexpr int kScanWaves = 16;

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_colscan(int n, int rows_per_part, int gamma,
                                                      const T* __restrict__ Y,
                                                      const T* __restrict__ thr,
                                                      T* __restrict__ pv, int* __restrict__ pi,
                                                      const int* __restrict__ nact,
                                                      const int* __restrict__ act) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int c = gw / kScanWaves;
  const int wc = gw % kScanWaves;
  const int na = nact[c];
  const T th = thr[c];
  for (int k = wc; k < na; k += kScanWaves) {
    const int part = act[static_cast<size_t>(c) * kColParts + k];
    const int x0 = part * rows_per_part;
    const int x1 = min(n, x0 + rows_per_part);
    double lv = -DBL_MAX;   // list entry r sits in lane r (r < gamma)
    int li = INT_MAX;
    for (int xb = x0; xb < x1; xb += 64) {
      const int x = xb + lane;
      double bv = -DBL_MAX;
      int bi = INT_MAX;
      if (x < x1) {
        const T q = Y[static_cast<size_t>(x) * B + c];
        if (q >= th) {
          bv = static_cast<double>(q);
          bi = x;
        }
      }
      // new list = best gamma of (list, batch); each lane holds at most two entries
      double nv = -DBL_MAX;
      int ni = INT_MAX;
      bool list_used = false, batch_used = false;
      for (int r = 0; r < gamma; ++r) {
        const bool take_list = !list_used && (batch_used || ranks_before(lv, li, bv, bi));
        double cv = take_list ? lv : (batch_used ? -DBL_MAX : bv);
        int ci = take_list ? li : (batch_used ? INT_MAX : bi);
        if (list_used && batch_used) {
          cv = -DBL_MAX;
          ci = INT_MAX;
        }
        int owner = lane;
        wave_best(cv, ci, owner);
        if (ci == INT_MAX) break;   // no entries left
        if (lane == r) {
          nv = cv;
          ni = ci;
        }
        if (lane == owner) {
          if (take_list) list_used = true;
          else batch_used = true;
        }
      }
      lv = nv;
      li = ni;
    }
    if (lane < gamma) {
      const size_t o = static_cast<size_t>(part) * B + c;
      pv[o * gamma + lane] = static_cast<T>(lv);
      pi[o * gamma + lane] = li;
    }
  }
}


// one wave per column; the registered chunk order is arbitrary but the
// selection uses the total order (value desc, id asc), so the result is not
template <typename T, int B>
__global__ __launch_bounds__(64) void k_colmerge(int n, int s0, int gamma,
                                                 const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col,
                                                 const T* __restrict__ Y,
                                                 const T* __restrict__ pv,
                                                 const int* __restrict__ pi,
                                                 const int* __restrict__ nact,
                                                 const int* __restrict__ act,
                                                 ColStats* __restrict__ cs) {
  const int c = blockIdx.x;
  const int s = s0 + c;
  const int lane = threadIdx.x;
  double lv[kMaxGamma];
  int li[kMaxGamma];
#pragma unroll
  for (int p = 0; p < kMaxGamma; ++p) {
    lv[p] = -DBL_MAX;
    li[p] = INT_MAX;
  }
  double lastv = -DBL_MAX;
  int lasti = INT_MAX;
  const int na = nact[c];
  for (int k = lane; k < na; k += 64) {
    const size_t o = static_cast<size_t>(act[static_cast<size_t>(c) * kColParts + k]) * B + c;
    for (int r = 0; r < gamma; ++r) {
      const int id = pi[o * gamma + r];
      if (id == INT_MAX) break;
      const double v = static_cast<double>(pv[o * gamma + r]);
      if (!ranks_before(v, id, lastv, lasti)) break;   // partial lists are sorted
      list_insert(lv, li, gamma, v, id);
      list_last(lv, li, gamma, &lastv, &lasti);
    }
  }
  const int cnt = gamma < n ? gamma : n;
  double top_v = -DBL_MAX;   // lane r keeps the r-th candidate
  int top_i = INT_MAX;
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
    int owner = lane;
    wave_best(hv, hi, owner);
    if (lane == r) {
      top_v = hv;
      top_i = hi;
    }
    if (owner == lane) ++head;
  }
  double best = -DBL_MAX;
  if (gamma > 0) {
    // the cnt (cnt - 1) / 2 unordered candidate pairs, one per lane; each test
    // searches the shorter of the two neighbour lists (adjacency is symmetric)
    const int npairs = cnt * (cnt - 1) / 2;
    for (int p = 0; p < npairs; p += 64) {
      const int q = p + lane;
      int a = 0, b = 1, rem = q;
      while (a < cnt - 1 && rem >= cnt - 1 - a) {   // q -> (a, b), a < b, row by row
        rem -= cnt - 1 - a;
        ++a;
      }
      b = a + 1 + rem;
      const bool on = q < npairs;
      const int ia = __shfl(top_i, on ? a : 0, 64);
      const int ib = __shfl(top_i, on && b < 64 ? b : 0, 64);
      const double va = __shfl(top_v, on ? a : 0, 64);
      const double vb = __shfl(top_v, on && b < 64 ? b : 0, 64);
      if (on) {
        const int da = rowptr[ia + 1] - rowptr[ia];
        const int db = rowptr[ib + 1] - rowptr[ib];
        const bool adj = da <= db ? adjacent(rowptr, col, ia, ib) : adjacent(rowptr, col, ib, ia);
        if (adj) best = fmax(best, va + vb);
      }
    }
  }
  double nmx = -DBL_MAX, nmn = DBL_MAX;
  for (int k = rowptr[s] + lane; k < rowptr[s + 1]; k += 64) {
    const double q = static_cast<double>(Y[static_cast<size_t>(col[k]) * B + c]);
    nmx = fmax(nmx, q);
    nmn = fmin(nmn, q);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    best = fmax(best, __shfl_xor(best, off, 64));
    nmx = fmax(nmx, __shfl_xor(nmx, off, 64));
    nmn = fmin(nmn, __shfl_xor(nmn, off, 64));
  }
  const double first = __shfl(top_v, 0, 64);
  const double lastc = __shfl(top_v, cnt > 0 ? cnt - 1 : 0, 64);
  if (lane == 0) {
    cs[c].rho = gamma > 0 ? fmax(best, first + lastc) : 0.0;
    cs[c].maxN = nmx;
    cs[c].minN = nmn;
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

// One wave per slot k = (s -> j) of the block.  Three loads in flight per lane
// keep the kernel at 32 VGPRs, which is what the dense step's six waves per
// SIMD leave free on the other stream.
constexpr int kWcBatch = 3;
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_walk_counts(
    int kbeg, int kend, int s0, int tilde, int gamma, double coef, long long nr_cap,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ slot_row, const int32_t* __restrict__ deg, const T* __restrict__ Y,
    const ColStats* __restrict__ cs, const int32_t* __restrict__ tau, long long* __restrict__ nr) {
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
  const int je = rowptr[j + 1];
  for (int kb = rowptr[j] + lane; kb < je; kb += 64 * kWcBatch) {
    int u[kWcBatch];
#pragma unroll
    for (int q = 0; q < kWcBatch; ++q) u[q] = kb + 64 * q < je ? col[kb + 64 * q] : -1;
    T y[kWcBatch];
#pragma unroll
    for (int q = 0; q < kWcBatch; ++q) y[q] = u[q] >= 0 ? Y[static_cast<size_t>(u[q]) * B + c] : T(0);
#pragma unroll
    for (int q = 0; q < kWcBatch; ++q) {
      if (u[q] >= 0) {
        jmx = fmax(jmx, static_cast<double>(y[q]));
        jmn = fmin(jmn, static_cast<double>(y[q]));
      }
    }
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
}

// walk pairs and single-walk steps of slots [kbeg, kend): one atomic pair per
// workgroup (integer sums, so the totals do not depend on the order)
__global__ __launch_bounds__(256) void k_work_totals(int kbeg, int kend, int tilde,
                                                     const int32_t* __restrict__ tau,
                                                     const long long* __restrict__ nr,
                                                     unsigned long long* __restrict__ work) {
  __shared__ unsigned long long s0[256], s1[256];
  unsigned long long a = 0, b = 0;
  for (int k = kbeg + blockIdx.x * 256 + threadIdx.x; k < kend; k += gridDim.x * 256) {
    const long long w = nr[k];
    if (w > 0) {
      a += static_cast<unsigned long long>(w);
      b += static_cast<unsigned long long>(w) * 2ull * static_cast<unsigned long long>(tau[k] - tilde);
    }
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&work[0], s0[0]);
    atomicAdd(&work[1], s1[0]);
  }
}

// The walks of slot k = (s -> j) by one wave, lanes taking walk pairs r = lane,
// lane + 64, ...; gacc[k] += their mean (Eq. 11).
template <typename T, int B>
__device__ inline void slot_walks(int k, int lane, int s0, int tilde, unsigned k0, unsigned k1,
                                  const int32_t* __restrict__ rowptr,
                                  const int32_t* __restrict__ col,
                                  const int32_t* __restrict__ slot_row,
                                  const double* __restrict__ inv_deg, const T* __restrict__ Y,
                                  const int32_t* __restrict__ tau,
                                  const long long* __restrict__ nr, double* __restrict__ gacc) {
  const long long n_r = nr[k];
  if (n_r <= 0) return;
  const int len = tau[k] - tilde;
  const int s = slot_row[k];
  const int c = s - s0;
  const int j = col[k];
  double acc = 0.0;
  for (long long r = lane; r < n_r; r += 64) {
    // the two walks of the pair advance in lockstep so their loads overlap
    int pos0 = s, pos1 = j;
    double sum0 = 0.0, sum1 = 0.0;
    for (int t4 = 0; t4 < len; t4 += 4) {   // four steps per Philox draw
      const uint32_t hi = static_cast<uint32_t>(t4 >> 2);
      const U32x4 w0 = philox4x32_10(static_cast<uint32_t>(s), static_cast<uint32_t>(j),
                                     static_cast<uint32_t>(r), hi, k0, k1);
      const U32x4 w1 = philox4x32_10(static_cast<uint32_t>(s), static_cast<uint32_t>(j),
                                     static_cast<uint32_t>(r), (1u << 31) | hi, k0, k1);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (t4 + u >= len) break;
        const int b0 = rowptr[pos0], e0 = rowptr[pos0 + 1];
        const int b1 = rowptr[pos1], e1 = rowptr[pos1 + 1];
        pos0 = col[b0 + static_cast<int>(pick_neighbour(w0.w[u], static_cast<uint32_t>(e0 - b0)))];
        pos1 = col[b1 + static_cast<int>(pick_neighbour(w1.w[u], static_cast<uint32_t>(e1 - b1)))];
        sum0 += static_cast<double>(Y[static_cast<size_t>(pos0) * B + c]);
        sum1 += static_cast<double>(Y[static_cast<size_t>(pos1) * B + c]);
      }
    }
    acc += (sum0 - sum1) * inv_deg[s];   // X of Eq. 11
  }
  acc = wave_sum(acc);
  if (lane == 0) gacc[k] += acc / static_cast<double>(n_r);
}

// ---------------------------------------------------------------- flattened walks
// The walk pairs of a block's half-edges are cut into chunks of 64 pairs
// (chunk_off: exclusive prefix of ceil(n_r / 64) over the block's slots, one
// workgroup); waves take contiguous ranges of chunks, one pair per lane, and
// store each chunk's sum (fixed butterfly); a last pass adds a slot's chunk
// sums in chunk order.  ctl[0] = number of chunks, ctl[1] = 1 when they fit
// the partial-sum buffer (else the same grid walks one slot per wave).
constexpr int kScanThreads = 256;   // one small workgroup: schedules beside the traversal kernels
constexpr int kScanPer = 8;

__global__ __launch_bounds__(kScanThreads) void k_walk_scan(int kbeg, int kend,
                                                            const long long* __restrict__ nr,
                                                            long long* __restrict__ chunk_off,
                                                            long long capacity,
                                                            long long* __restrict__ ctl) {
  __shared__ long long wsum[kScanThreads / 64];
  __shared__ long long carry_s;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nk = kend - kbeg;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < nk; base += kScanThreads * kScanPer) {
    long long v[kScanPer];
    long long tsum = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      const int i = base + tid * kScanPer + q;
      const long long r = i < nk ? nr[kbeg + i] : 0;
      v[q] = r > 0 ? (r + 63) / 64 : 0;
      tsum += v[q];
    }
    // inclusive scan of the thread sums inside the wave
    long long x = tsum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const long long y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    long long wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += wsum[w];
    long long run = carry_s + wpre + x - tsum;   // exclusive prefix of this thread
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      const int i = base + tid * kScanPer + q;
      if (i < nk) chunk_off[i] = run;
      run += v[q];
    }
    __syncthreads();
    if (tid == kScanThreads - 1) carry_s = run;
    __syncthreads();
  }
  if (tid == 0) {
    chunk_off[nk] = carry_s;
    ctl[0] = carry_s;
    ctl[1] = carry_s <= capacity ? 1 : 0;
  }
}

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_walks_flat(
    int kbeg, int kend, int s0, int tilde, unsigned k0, unsigned k1,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ slot_row, const double* __restrict__ inv_deg,
    const T* __restrict__ Y, const int32_t* __restrict__ tau, const long long* __restrict__ nr,
    const long long* __restrict__ chunk_off, const long long* __restrict__ ctl,
    double* __restrict__ part, double* __restrict__ gacc) {
  const int lane = threadIdx.x & 63;
  const long long nwaves = static_cast<long long>(gridDim.x) * kWavesPerBlock;
  const long long w = static_cast<long long>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
  if (ctl[1] == 0) {
    // the chunks do not fit the partial-sum buffer: one wave per slot instead
    for (long long k = kbeg + w; k < kend; k += nwaves)
      slot_walks<T, B>(static_cast<int>(k), lane, s0, tilde, k0, k1, rowptr, col, slot_row,
                       inv_deg, Y, tau, nr, gacc);
    return;
  }
  const long long total = ctl[0];
  const long long per = (total + nwaves - 1) / nwaves;
  const long long c0 = w * per;
  const long long c1 = min(total, c0 + per);
  if (c0 >= c1) return;
  const int nk = kend - kbeg;
  // slot of chunk c0: the last i with chunk_off[i] <= c0 (and a chunk of its own)
  int lo = 0, hi = nk;   // chunk_off[lo] <= c0 < chunk_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= c0) lo = mid;
    else hi = mid;
  }
  int i = lo;
  long long next = chunk_off[i + 1];
  for (long long c = c0; c < c1; ++c) {
    while (c >= next) {   // move to the slot that owns chunk c (skips slots without walks)
      ++i;
      next = chunk_off[i + 1];
    }
    const int k = kbeg + i;
    const long long n_r = nr[k];
    const long long r = (c - chunk_off[i]) * 64 + lane;
    double x = 0.0;
    if (r < n_r) {
      const int len = tau[k] - tilde;
      const int s = slot_row[k];
      const int cc = s - s0;
      const int j = col[k];
      int pos0 = s, pos1 = j;
      double sum0 = 0.0, sum1 = 0.0;
      // four steps per Philox draw, the word of each step a compile-time index
      // (a run-time index would put the draw in scratch memory)
      for (int t4 = 0; t4 < len; t4 += 4) {
        const uint32_t h = static_cast<uint32_t>(t4 >> 2);
        const U32x4 w0 = philox4x32_10(static_cast<uint32_t>(s), static_cast<uint32_t>(j),
                                       static_cast<uint32_t>(r), h, k0, k1);
        const U32x4 w1 = philox4x32_10(static_cast<uint32_t>(s), static_cast<uint32_t>(j),
                                       static_cast<uint32_t>(r), (1u << 31) | h, k0, k1);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (t4 + u >= len) break;
          // the two walks of the pair advance in lockstep so their loads overlap
          const int b0 = rowptr[pos0], e0 = rowptr[pos0 + 1];
          const int b1 = rowptr[pos1], e1 = rowptr[pos1 + 1];
          pos0 = col[b0 + static_cast<int>(pick_neighbour(w0.w[u], static_cast<uint32_t>(e0 - b0)))];
          pos1 = col[b1 + static_cast<int>(pick_neighbour(w1.w[u], static_cast<uint32_t>(e1 - b1)))];
          sum0 += static_cast<double>(Y[static_cast<size_t>(pos0) * B + cc]);
          sum1 += static_cast<double>(Y[static_cast<size_t>(pos1) * B + cc]);
        }
      }
      x = (sum0 - sum1) * inv_deg[s];   // X of Eq. 11
    }
    x = wave_sum(x);
    if (lane == 0) part[c] = x;
  }
}

__global__ void k_walk_finish(FinishJob f) {
  walk_finish_slot(f, static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x));
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
                           ColStats* cs, void* scratch, hipStream_t st, const AccJob* acc,
                           const FinishJob* fin) {
  int ncols = B;
  if (s0 + ncols > g.n) ncols = g.n - s0;
  if (ncols <= 0) return fin ? launch_walk_finish(*fin, st) : hipSuccess;
  if (gamma > kMaxGamma || gamma < 0) return hipErrorInvalidValue;
  const int G = 64 / B;
  const int nparts = kColParts;
  const int waves = nparts / G;
  const int rows = (g.n + nparts - 1) / nparts;
  // scratch layout (see kColScratchBytes)
  char* base = static_cast<char*>(scratch);
  const size_t cells = static_cast<size_t>(nparts) * 64;
  T* pv = reinterpret_cast<T*>(base);
  int* pi = reinterpret_cast<int*>(base + cells * kMaxGamma * sizeof(double));
  T* pmx = reinterpret_cast<T*>(base + cells * kMaxGamma * (sizeof(double) + sizeof(int)));
  T* pmn = pmx + cells;
  int* act = reinterpret_cast<int*>(pmn + cells);             // [64][kColParts]
  int* nact = act + cells;                                     // [64]
  T* thr = reinterpret_cast<T*>(nact + 64);                    // [64]
  const int col_blocks = waves / kWavesPerBlock;
  const AccJob job = acc ? *acc : AccJob{};
  const int acc_blocks =
      acc_job_set(job) ? static_cast<int>(grid_for(job.kend - job.kbeg, kThreads)) : 0;
  const FinishJob fj = fin ? *fin : FinishJob{};
  const int fin_blocks =
      fj.gacc && fj.kend > fj.kbeg ? static_cast<int>(grid_for(fj.kend - fj.kbeg, kThreads)) : 0;
  SC_DISPATCH_B(B, (k_colmax<T, kB><<<col_blocks + acc_blocks + fin_blocks, kThreads, 0, st>>>(
                        g.n, rows, nparts, Y, pmx, pmn, col_blocks, job, acc_blocks, fj,
                        g.slot_row, g.col, g.inv_deg_d)));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SC_DISPATCH_B(B, (k_colthresh<T, kB><<<ncols, 64 * kThreshWaves, 0, st>>>(
                        gamma, nparts, pmx, pmn, thr, nact, act, cs)));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (gamma > 0) {
    SC_DISPATCH_B(B, (k_colscan<T, kB><<<grid_for(static_cast<int64_t>(ncols) * kScanWaves,
                                                  kWavesPerBlock), kThreads, 0, st>>>(
                          g.n, rows, gamma, Y, thr, pv, pi, nact, act)));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  SC_DISPATCH_B(B, (k_colmerge<T, kB><<<ncols, 64, 0, st>>>(g.n, s0, gamma, g.rowptr, g.col, Y,
                                                             pv, pi, nact, act, cs)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_walk_counts(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int tilde,
                              int gamma, double coef, int64_t nr_cap, const T* Y,
                              const ColStats* cs, const int32_t* tau_slot, int64_t* nr_slot,
                              hipStream_t st) {
  if (kend <= kbeg) return hipSuccess;
  SC_DISPATCH_B(B, (k_walk_counts<T, kB><<<grid_for(kend - kbeg, kWavesPerBlock), kThreads, 0,
                                          st>>>(
                        kbeg, kend, s0, tilde, gamma, coef, static_cast<long long>(nr_cap),
                        g.rowptr, g.col, g.slot_row, g.deg, Y, cs, tau_slot,
                        reinterpret_cast<long long*>(nr_slot))));
  return hipGetLastError();
}

hipError_t launch_work_totals(int kbeg, int kend, int tilde, const int32_t* tau_slot,
                              const int64_t* nr_slot, unsigned long long* work, hipStream_t st) {
  if (kend <= kbeg) return hipSuccess;
  unsigned blocks = grid_for(kend - kbeg, 256);
  if (blocks > 256) blocks = 256;
  k_work_totals<<<blocks, 256, 0, st>>>(kbeg, kend, tilde, tau_slot,
                                        reinterpret_cast<const long long*>(nr_slot), work);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_walks(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int tilde,
                        uint64_t seed, const T* Y, const int32_t* tau_slot,
                        const int64_t* nr_slot, double* gacc, const WalkScratch& ws,
                        hipStream_t st, FinishJob* defer) {
  if (defer) *defer = FinishJob{};
  if (kend <= kbeg) return hipSuccess;
  const unsigned k0 = static_cast<unsigned>(seed & 0xFFFFFFFFull);
  const unsigned k1 = static_cast<unsigned>(seed >> 32);
  const long long* nr = reinterpret_cast<const long long*>(nr_slot);
  long long* off = reinterpret_cast<long long*>(ws.chunk_off);
  long long* ctl = reinterpret_cast<long long*>(ws.ctl);
  if (!ws.chunk_off || !ws.part || !ws.ctl) return hipErrorInvalidValue;   // scratch required
  k_walk_scan<<<1, kScanThreads, 0, st>>>(kbeg, kend, nr, off, ws.capacity, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SC_DISPATCH_B(B, (k_walks_flat<T, kB><<<kWalkBlocks, kThreads, 0, st>>>(
                        kbeg, kend, s0, tilde, k0, k1, g.rowptr, g.col, g.slot_row, g.inv_deg_d,
                        Y, tau_slot, nr, off, ctl, ws.part, gacc)));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  FinishJob f;
  f.kbeg = kbeg;
  f.kend = kend;
  f.nr = nr_slot;
  f.chunk_off = ws.chunk_off;
  f.ctl = ws.ctl;
  f.part = ws.part;
  f.gacc = gacc;
  if (defer) {
    *defer = f;
    return hipSuccess;
  }
  return launch_walk_finish(f, st);
}

// The nodes visited by walk pair r of half-edge (i, j): thread 0 walks from i
// (side 0), thread 1 from j (side 1), with the counters and the neighbour pick
// of the walk kernels; nodes[side * len + t] is the node after step t + 1.
__global__ void k_walk_trace(int i, int j, unsigned r, int len, unsigned k0, unsigned k1,
                             const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             int32_t* __restrict__ nodes) {
  const int side = threadIdx.x;
  if (side > 1) return;
  int pos = side == 0 ? i : j;
  for (int t4 = 0; t4 < len; t4 += 4) {
    const U32x4 w = philox4x32_10(static_cast<uint32_t>(i), static_cast<uint32_t>(j), r,
                                  (side ? (1u << 31) : 0u) | static_cast<uint32_t>(t4 >> 2), k0, k1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (t4 + u >= len) break;
      const int b = rowptr[pos], e = rowptr[pos + 1];
      pos = col[b + static_cast<int>(pick_neighbour(w.w[u], static_cast<uint32_t>(e - b)))];
      nodes[static_cast<size_t>(side) * len + t4 + u] = pos;
    }
  }
}

hipError_t launch_walk_trace(const DeviceGraph& g, int i, int j, uint32_t r, int len,
                             uint64_t seed, int32_t* nodes, hipStream_t st) {
  const unsigned k0 = static_cast<unsigned>(seed & 0xFFFFFFFFull);
  const unsigned k1 = static_cast<unsigned>(seed >> 32);
  k_walk_trace<<<1, 64, 0, st>>>(i, j, r, len, k0, k1, g.rowptr, g.col, nodes);
  return hipGetLastError();
}

hipError_t launch_walk_finish(const FinishJob& f, hipStream_t st) {
  if (!f.gacc || f.kend <= f.kbeg) return hipSuccess;
  k_walk_finish<<<grid_for(f.kend - f.kbeg, 256), 256, 0, st>>>(f);
  return hipGetLastError();
}

template hipError_t launch_colstats<float>(const DeviceGraph&, int, int, int, const float*,
                                           ColStats*, void*, hipStream_t, const AccJob*,
                                           const FinishJob*);
template hipError_t launch_colstats<double>(const DeviceGraph&, int, int, int, const double*,
                                            ColStats*, void*, hipStream_t, const AccJob*,
                                            const FinishJob*);
template hipError_t launch_walk_counts<float>(const DeviceGraph&, int, int, int, int, int, int,
                                              double, int64_t, const float*, const ColStats*,
                                              const int32_t*, int64_t*, hipStream_t);
template hipError_t launch_walk_counts<double>(const DeviceGraph&, int, int, int, int, int, int,
                                               double, int64_t, const double*, const ColStats*,
                                               const int32_t*, int64_t*, hipStream_t);
template hipError_t launch_walks<float>(const DeviceGraph&, int, int, int, int, int, uint64_t,
                                        const float*, const int32_t*, const int64_t*, double*,
                                        const WalkScratch&, hipStream_t, FinishJob*);
template hipError_t launch_walks<double>(const DeviceGraph&, int, int, int, int, int, uint64_t,
                                         const double*, const int32_t*, const int64_t*, double*,
                                         const WalkScratch&, hipStream_t, FinishJob*);

}  // namespace sc
