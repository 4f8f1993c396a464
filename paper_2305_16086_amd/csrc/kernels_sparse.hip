// Per-source TGT+ (Algorithm 4) with a frontier-sparse traversal and the
// adaptive switch step of Eq. 14 (Section 4.2.1).
//
// One workgroup owns one source i at a time and keeps its column in a private
// slot of device memory, as 64-bit fixed point (unit 2^-63):
//
//   Q_l[y] = r_l[y] / d_y,   r_l[y] = p_l(i, y) (the walk distribution from i),
//
// so that by reversibility (Eq. 4) q[y] = p_l(y, i) = d_i * Q_l[y] * 2^-63.
// One step is a push over the support S_l: r_{l+1}[y] = sum over u in N(y) of
// Q_l[u], added with 64-bit integer atomics (exact and order-free, so the
// result does not depend on the schedule), then Q_{l+1}[y] = r_{l+1}[y] / d_y
// rounded to nearest.  The support list S_{l+1} collects the nodes whose
// accumulator was zero before their first addition.
//
// At every l the workgroup evaluates Algorithm 3 on q = p_l(., i) (top-gamma
// threshold by radix select, rho-hat over the candidate edges, extremes over
// N(i), N(j) and V), the walk counts of Eq. 13, and Eq. 14's two sides; the
// first l where the frontier volume exceeds the walk work becomes tilde_tau_i.
// The walks of a wave of sources then run flat over the whole GPU (chunks of
// 64 walk pairs, fixed-order sums), reading q from the sources' slots.
#include "philox.hpp"
#include "sc_internal.hpp"

#include <cfloat>
#include <climits>

namespace sc {

namespace {

constexpr int kT = kSrcThreads;           // threads of the per-source workgroup
constexpr int kTW = kT / 64;              // its waves
constexpr double kInvUnit = 1.0 / 9223372036854775808.0;   // 2^-63
constexpr int kWalkGrid = 2048;
constexpr int kLongRow = 2048;   // N(j) longer than this is scanned by the whole workgroup
constexpr int kLongList = 256;

__device__ inline int block_scan_excl(int v, int* s_w, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_w[wave] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kTW; ++w) {
    pre += w < wave ? s_w[w] : 0;
    tot += s_w[w];
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

template <typename V, typename Op>
__device__ inline V block_reduce(V v, V* s, Op op) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = op(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  V r = s[0];
#pragma unroll
  for (int w = 1; w < kTW; ++w) r = op(r, s[w]);
  __syncthreads();
  return r;
}

struct MaxU64 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a > b ? a : b; }
};
struct MinU64 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a < b ? a : b; }
};
struct AddU64 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; }
};
struct AddD {
  __device__ double operator()(double a, double b) const { return a + b; }
};

// Visit every (entry, neighbour) pair of the entries [0, cnt) of a node list
// that pass `keep`, edge-parallel over the workgroup: each pass loads 256
// entries, scans their degrees and spreads the neighbour slots over the
// threads (a hub's list is shared by all of them).  act(entry, value, y).
template <typename Keep, typename Act>
__device__ inline void for_each_edge(const int32_t* __restrict__ list, int cnt,
                                     const int32_t* __restrict__ rowptr,
                                     const int32_t* __restrict__ col, Keep keep, Act act,
                                     int* s_off, int* s_beg, uint64_t* s_val, int* s_w) {
  for (int base = 0; base < cnt; base += kT) {
    const int e = base + static_cast<int>(threadIdx.x);
    int du = 0, beg = 0;
    uint64_t val = 0;
    if (e < cnt) {
      const int u = list[e];
      if (keep(e, u, &val)) {
        beg = rowptr[u];
        du = rowptr[u + 1] - beg;
      }
    }
    int total = 0;
    const int off = block_scan_excl(du, s_w, &total);
    s_off[threadIdx.x] = off;
    s_beg[threadIdx.x] = beg;
    s_val[threadIdx.x] = val;
    __syncthreads();
    for (int x = threadIdx.x; x < total; x += kT) {
      int lo = 0, hi = kT - 1;   // last t with s_off[t] <= x (entries without edges share offsets)
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= x) lo = mid;
        else hi = mid - 1;
      }
      act(lo, s_val[lo], col[s_beg[lo] + (x - s_off[lo])]);
    }
    __syncthreads();
  }
}

// x in the sorted neighbour list col[b, e)
__device__ inline bool adjacent(const int32_t* __restrict__ col, int b, int e, int x) {
  while (b < e) {
    const int mid = (b + e) >> 1;
    const int v = col[mid];
    if (v == x) return true;
    if (v < x) b = mid + 1;
    else e = mid;
  }
  return false;
}

__device__ inline double wave_max_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_min_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kT) void k_src_head(SrcArgs a) {
  __shared__ int s_off[kT], s_beg[kT];
  __shared__ uint64_t s_val[kT];
  __shared__ int s_w[kTW];
  __shared__ uint64_t s_r64[kTW];
  __shared__ double s_rd[kTW];
  __shared__ unsigned s_hist[256];
  __shared__ unsigned long long s_bmin[256], s_bmax[256];
  __shared__ int s_cnt;
  __shared__ int s_long[kLongList];   // halves whose N(j) the whole workgroup scans
  __shared__ int s_nlong;
  __shared__ uint64_t s_sel[3];   // prefix, threshold, done flag
  __shared__ int s_rank;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int w = blockIdx.x;
  const int n = a.n;
  {
    // the final column of the slot's previous source, read by that wave's walks
    // (earlier in stream order), is zeroed here instead of by a launch of its own
    const int cnt_old = a.slot_ctl[2 * w];
    if (cnt_old > 0) {
      const size_t c = 2 * static_cast<size_t>(w) + static_cast<size_t>(a.slot_ctl[2 * w + 1]);
      uint64_t* Qo = a.Q + c * static_cast<size_t>(n);
      const int32_t* So = a.S + c * static_cast<size_t>(n);
      for (int e = tid; e < cnt_old; e += kT) Qo[So[e]] = 0;
    }
    __syncthreads();
  }
  const int64_t li = a.list_base + w;
  if (li >= a.nsrc) {
    if (tid == 0) {
      a.slot_ctl[2 * w] = 0;
      a.slot_ctl[2 * w + 1] = 0;
    }
    return;
  }
  const int i = a.srcs ? a.srcs[li] : static_cast<int>(li);
  const int rb = a.rowptr[i], re = a.rowptr[i + 1];
  const int di = re - rb;
  const int taup = a.tau_row[i];
  uint64_t* Qc = a.Q + static_cast<size_t>(2 * w) * n;
  uint64_t* Qn = Qc + n;
  int32_t* Sc = a.S + static_cast<size_t>(2 * w) * n;
  int32_t* Sn = Sc + n;
  int parity = 0;
  if (tid == 0) {
    const uint64_t one = 1ull << 63;
    Qc[i] = (one + static_cast<uint64_t>(di) / 2) / static_cast<uint64_t>(di);   // r_0 = e_i
    Sc[0] = i;
  }
  int cnt = 1;
  int ell = 0;
  uint64_t pushed = 0;
  __syncthreads();

  for (;;) {
    // ---- (1) the support: volume (Eq. 14 left side), extremes, select keys
    uint64_t vol = 0, qmx = 0, qmn = ~0ull;
    for (int e = tid; e < cnt; e += kT) {
      const int y = Sc[e];
      const uint64_t v = Qc[y];
      vol += static_cast<uint64_t>(a.rowptr[y + 1] - a.rowptr[y]);
      qmx = v > qmx ? v : qmx;
      qmn = v < qmn ? v : qmn;
      Qn[e] = v;   // keys of the radix select (Qn is all zero here)
    }
    vol = block_reduce(vol, s_r64, AddU64{});
    qmx = block_reduce(qmx, s_r64, MaxU64{});
    qmn = block_reduce(qmn, s_r64, MinU64{});
    const double maxV = static_cast<double>(qmx);
    const double minV = cnt == n ? static_cast<double>(qmn) : 0.0;   // zeros outside S

    // ---- (2)-(5) walk counts at this l (skipped where no half needs walks)
    // a forced switch step (tests, and a fixed tilde_tau option) skips Eq. 14 and
    // evaluates the walk counts only where it stops.  Eq. 14 itself is not
    // evaluated at l = 0: its left side is then d_i while each of the d_i halves
    // needs at least one walk pair, so it cannot switch there.
    const bool forced = a.force_tilde >= 0;
    const int stop_forced = forced ? (a.force_tilde < taup ? a.force_tilde : taup) : -1;
    const bool need = ell < taup && (forced ? ell == stop_forced : ell > 0);
    double rhs = 0.0;
    double rhoQ = 0.0;
    double maxNi = 0.0, minNi = 0.0;
    if (need) {
      // (2) threshold T = the gamma-th largest q (Algorithm 3 line 2); 0 when the
      // support has fewer than gamma nodes (the candidate list then holds zeros)
      uint64_t T = 0;
      if (a.gamma > 0 && cnt < a.gamma && cnt == n) T = qmn;   // every node is a candidate
      if (a.gamma > 0 && cnt >= a.gamma) {
        const int top = 63 - __clzll(static_cast<long long>(qmx | 1ull));
        int shift = (top / 8) * 8;
        uint64_t prefix = 0, pmask = shift + 8 >= 64 ? 0ull : ~((1ull << (shift + 8)) - 1);
        if (tid == 0) {
          s_rank = a.gamma;
          s_sel[2] = 0;
        }
        __syncthreads();
        for (; shift >= 0; shift -= 8) {
          for (int d = tid; d < 256; d += kT) {
            s_hist[d] = 0;
            s_bmin[d] = ~0ull;
            s_bmax[d] = 0;
          }
          __syncthreads();
          for (int e = tid; e < cnt; e += kT) {
            const uint64_t v = Qn[e];
            if ((v & pmask) == prefix) {
              const int d = static_cast<int>((v >> shift) & 255u);
              atomicAdd(&s_hist[d], 1u);
              atomicMin(&s_bmin[d], static_cast<unsigned long long>(v));
              atomicMax(&s_bmax[d], static_cast<unsigned long long>(v));
            }
          }
          __syncthreads();
          if (tid == 0) {
            int k = s_rank, d = 255;
            for (; d > 0; --d) {
              if (static_cast<int>(s_hist[d]) >= k) break;
              k -= static_cast<int>(s_hist[d]);
            }
            s_rank = k;
            s_sel[0] = prefix | (static_cast<uint64_t>(d) << shift);
            if (s_bmin[d] == s_bmax[d]) {   // one value left in the bucket
              s_sel[1] = s_bmin[d];
              s_sel[2] = 1;
            }
          }
          __syncthreads();
          prefix = s_sel[0];
          pmask |= 255ull << shift;
          if (s_sel[2]) break;
          __syncthreads();
        }
        T = s_sel[2] ? s_sel[1] : prefix;
        __syncthreads();
      }
      // (3) rho-hat (Eq. 16 bound, Algorithm 3 lines 3-5, safe reading): the best
      // candidate-pair edge against q[c_1] + q[c_gamma]
      if (a.gamma > 0) {
        const uint64_t thr = T > 0 ? T : 1;
        unsigned long long best = 0;
        for_each_edge(
            Sc, cnt, a.rowptr, a.col,
            [&](int, int u, uint64_t* val) {
              *val = Qc[u];
              return *val >= thr;
            },
            [&](int, uint64_t qc, int y) {
              const uint64_t qy = Qc[y];
              if (qy >= thr) {
                const unsigned long long s = qc + qy;
                best = s > best ? s : best;
              }
            },
            s_off, s_beg, s_val, s_w);
        best = block_reduce(static_cast<uint64_t>(best), s_r64, MaxU64{});
        rhoQ = fmax(static_cast<double>(best), maxV + static_cast<double>(T));
      }
      // (4) extremes over N(i)
      double mx = -DBL_MAX, mn = DBL_MAX;
      for (int k = rb + tid; k < re; k += kT) {
        const double v = static_cast<double>(Qc[a.col[k]]);
        mx = fmax(mx, v);
        mn = fmin(mn, v);
      }
      maxNi = block_reduce(mx, s_rd, [](double x, double y) { return fmax(x, y); });
      minNi = block_reduce(mn, s_rd, [](double x, double y) { return fmin(x, y); });
      // (5) per half (i, j): extremes over N(j), chi (Eq. 17 / Eq. 15), n_r (Eq. 13)
      double part = 0.0;
      auto count_walks = [&](int k, int len, double jmx, double jmn) {
        double chiQ;
        if (a.gamma > 0) {
          const double lb_i = minNi + (len - 1) * minV;
          const double ub_i = maxNi * 0.5 + maxV * 0.5 + (len - 1) * rhoQ * 0.5;
          const double lb_j = jmn + (len - 1) * minV;
          const double ub_j = jmx * 0.5 + maxV * 0.5 + (len - 1) * rhoQ * 0.5;
          chiQ = ub_i + ub_j - lb_i - lb_j;
        } else {
          chiQ = 2.0 * len * (maxV - minV);
        }
        // q = d_i Q 2^-63 and Eq. 13 divides chi^2 by d_i^2: d_i cancels
        const double chi = chiQ * kInvUnit;
        double r = ceil(a.coef * chi * chi);
        if (!(r >= 1.0)) r = 1.0;
        const long long nr = r > static_cast<double>(a.nr_cap) ? a.nr_cap : static_cast<long long>(r);
        a.nr_slot[k] = nr;
        part += a.rule == 0 ? static_cast<double>(nr) : 2.0 * len * static_cast<double>(nr);
      };
      if (tid == 0) s_nlong = 0;
      __syncthreads();
      for (int k = rb + wave; k < re; k += kTW) {
        const int len = a.tau_slot[k] - ell;
        if (len <= 0) {
          if (lane == 0) a.nr_slot[k] = 0;
          continue;
        }
        if (a.gamma > 0) {
          const int j = a.col[k];
          const int jb = a.rowptr[j], je = a.rowptr[j + 1];
          double jmx, jmn;
          if (je - jb > kLongRow && static_cast<int64_t>(cnt) * 16 >= je - jb) {
            // a hub's list: left to the whole workgroup below (or scanned here
            // when the list of such halves is full)
            int slot = -1;
            if (lane == 0) slot = atomicAdd(&s_nlong, 1);
            slot = __shfl(slot, 0, 64);
            if (slot < kLongList) {
              if (lane == 0) s_long[slot] = k;
              continue;
            }
          }
          if (static_cast<int64_t>(cnt) * 16 < je - jb) {
            // a short support against a long N(j) (a hub): visit the support and
            // test adjacency to j instead; q is zero off the support, so the
            // extremes over N(j) are those of the support nodes in N(j), with
            // the minimum 0 unless they fill N(j)
            double mx = 0.0, mn = DBL_MAX;
            int hits = 0;
            for (int e = lane; e < cnt; e += 64) {
              const int y = Sc[e];
              const int yb = a.rowptr[y], ye = a.rowptr[y + 1];
              const bool in_j = ye - yb < je - jb ? adjacent(a.col, yb, ye, j)
                                                  : adjacent(a.col, jb, je, y);
              if (in_j) {
                const double v = static_cast<double>(Qc[y]);
                mx = fmax(mx, v);
                mn = fmin(mn, v);
                ++hits;
              }
            }
            jmx = wave_max_d(mx);
            mn = wave_min_d(mn);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) hits += __shfl_xor(hits, off, 64);
            jmn = hits < je - jb ? 0.0 : mn;
          } else {
            double mx = -DBL_MAX, mn = DBL_MAX;
            for (int q = jb + lane; q < je; q += 64) {
              const double v = static_cast<double>(Qc[a.col[q]]);
              mx = fmax(mx, v);
              mn = fmin(mn, v);
            }
            jmx = wave_max_d(mx);
            jmn = wave_min_d(mn);
          }
          if (lane == 0) count_walks(k, len, jmx, jmn);
        } else if (lane == 0) {
          count_walks(k, len, 0.0, 0.0);
        }
      }
      __syncthreads();
      const int nlong = s_nlong < kLongList ? s_nlong : kLongList;
      for (int t = 0; t < nlong; ++t) {   // hubs' lists, all threads at once
        const int k = s_long[t];
        const int j = a.col[k];
        double mx = -DBL_MAX, mn = DBL_MAX;
        for (int q = a.rowptr[j] + tid; q < a.rowptr[j + 1]; q += kT) {
          const double v = static_cast<double>(Qc[a.col[q]]);
          mx = fmax(mx, v);
          mn = fmin(mn, v);
        }
        mx = block_reduce(mx, s_rd, [](double x, double y) { return fmax(x, y); });
        mn = block_reduce(mn, s_rd, [](double x, double y) { return fmin(x, y); });
        if (tid == 0) count_walks(k, a.tau_slot[k] - ell, mx, mn);
      }
      rhs = block_reduce(part, s_rd, AddD{});
    }
    // ---- (6) Eq. 14: switch when the next push costs more than the walks
    const bool done = forced ? ell >= stop_forced
                             : (ell >= taup || (need && static_cast<double>(vol) > rhs));
    if (done) {
      // clear the select keys, record the outcome
      for (int e = tid; e < cnt; e += kT) Qn[e] = 0;
      unsigned long long wk = 0, ws = 0;
      const int64_t pbase = (a.hoff ? a.hoff[li] : static_cast<int64_t>(rb)) - a.pos_base;
      for (int k = rb + tid; k < re; k += kT) {
        const int len = a.tau_slot[k] - ell;
        const long long nr = len > 0 ? a.nr_slot[k] : 0;
        if (len <= 0) a.nr_slot[k] = 0;
        const int64_t p = pbase + (k - rb);
        a.pos_slot[p] = k;
        a.pos_w[p] = w;
        a.nr_pos[p] = nr;
        wk += static_cast<unsigned long long>(nr);
        ws += static_cast<unsigned long long>(nr) * 2ull * static_cast<unsigned long long>(len > 0 ? len : 0);
      }
      wk = block_reduce(static_cast<uint64_t>(wk), s_r64, AddU64{});
      ws = block_reduce(static_cast<uint64_t>(ws), s_r64, AddU64{});
      if (tid == 0) {
        a.tilde_row[i] = ell;
        a.slot_ctl[2 * w] = cnt;
        a.slot_ctl[2 * w + 1] = parity;
        atomicAdd(&a.totals[0], wk);
        atomicAdd(&a.totals[1], ws);
        atomicAdd(&a.totals[2], static_cast<unsigned long long>(pushed));
        atomicMin(&a.totals[3], static_cast<unsigned long long>(ell));
        atomicMax(&a.totals[4], static_cast<unsigned long long>(ell));
      }
      return;
    }

    // ---- (7) push l -> l + 1: r_{l+1}[y] = sum over u in N(y) of Q_l[u]
    for (int e = tid; e < cnt; e += kT) Qn[e] = 0;   // the select keys
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    for_each_edge(
        Sc, cnt, a.rowptr, a.col,
        [&](int, int u, uint64_t* val) {
          *val = Qc[u];
          return *val != 0;
        },
        [&](int, uint64_t qv, int y) {
          const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long*>(&Qn[y]),
                                                   static_cast<unsigned long long>(qv));
          if (old == 0) Sn[atomicAdd(&s_cnt, 1)] = y;
        },
        s_off, s_beg, s_val, s_w);
    pushed += vol;
    const int cntn = s_cnt;
    // ---- (8) Q_{l+1}[y] = r_{l+1}[y] / d_y (rounded to nearest); (9) clear Q_l
    for (int e = tid; e < cntn; e += kT) {
      const int y = Sn[e];
      const uint64_t d = static_cast<uint64_t>(a.rowptr[y + 1] - a.rowptr[y]);
      Qn[y] = (Qn[y] + d / 2) / d;
    }
    for (int e = tid; e < cnt; e += kT) Qc[Sc[e]] = 0;
    __syncthreads();
    // ---- (10) step l + 1 of Eq. 9: g(i, j) += (p(i,i) - p(j,i)) / d_i = (Q[i] - Q[j]) 2^-63
    const double qi = static_cast<double>(Qn[i]);
    for (int k = rb + tid; k < re; k += kT)
      if (ell + 1 <= a.tau_slot[k])
        a.gacc[k] += (qi - static_cast<double>(Qn[a.col[k]])) * kInvUnit;
    __syncthreads();
    uint64_t* tq = Qc;
    Qc = Qn;
    Qn = tq;
    int32_t* ts = Sc;
    Sc = Sn;
    Sn = ts;
    cnt = cntn;
    parity ^= 1;
    ++ell;
  }
}

// ---------------------------------------------------------------- walks of a wave
// chunk_off[p] = exclusive prefix of ceil(nr_pos[p] / 64); ctl = {chunks, fits}
__global__ __launch_bounds__(256) void k_src_scan(int64_t P, const int64_t* __restrict__ nr_pos,
                                                  int64_t* __restrict__ chunk_off, int64_t capacity,
                                                  int64_t* __restrict__ ctl) {
  __shared__ int64_t s_w[4];
  __shared__ int64_t s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int kPer = 8;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < P; base += 256 * kPer) {
    int64_t v[kPer];
    int64_t ts = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int64_t p = base + tid * kPer + q;
      const int64_t r = p < P ? nr_pos[p] : 0;
      v[q] = r > 0 ? (r + 63) / 64 : 0;
      ts += v[q];
    }
    int64_t x = ts;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    int64_t pre = 0;
    for (int q = 0; q < wave; ++q) pre += s_w[q];
    int64_t run = s_carry + pre + x - ts;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int64_t p = base + tid * kPer + q;
      if (p < P) chunk_off[p] = run;
      run += v[q];
    }
    __syncthreads();
    if (tid == 255) s_carry = run;
    __syncthreads();
  }
  if (tid == 0) {
    chunk_off[P] = s_carry;
    ctl[0] = s_carry;
    ctl[1] = s_carry <= capacity ? 1 : 0;
  }
}

// One walk pair of half-edge (i, j): the sums of Q over W_i and W_j (Eq. 11
// numerator in units of 2^-63 / d_i), Philox counters as the other walk kernels.
__device__ inline double walk_pair(int i, int j, long long r, int len, unsigned k0, unsigned k1,
                                   const int32_t* __restrict__ rowptr,
                                   const int32_t* __restrict__ col,
                                   const uint64_t* __restrict__ Qs) {
  int p0 = i, p1 = j;
  double s0 = 0.0, s1 = 0.0;
  for (int t4 = 0; t4 < len; t4 += 4) {
    const uint32_t h = static_cast<uint32_t>(t4 >> 2);
    const U32x4 w0 = philox4x32_10(static_cast<uint32_t>(i), static_cast<uint32_t>(j),
                                   static_cast<uint32_t>(r), h, k0, k1);
    const U32x4 w1 = philox4x32_10(static_cast<uint32_t>(i), static_cast<uint32_t>(j),
                                   static_cast<uint32_t>(r), (1u << 31) | h, k0, k1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (t4 + u >= len) break;
      const int b0 = rowptr[p0], e0 = rowptr[p0 + 1];
      const int b1 = rowptr[p1], e1 = rowptr[p1 + 1];
      p0 = col[b0 + static_cast<int>(pick_neighbour(w0.w[u], static_cast<uint32_t>(e0 - b0)))];
      p1 = col[b1 + static_cast<int>(pick_neighbour(w1.w[u], static_cast<uint32_t>(e1 - b1)))];
      s0 += static_cast<double>(Qs[p0]);
      s1 += static_cast<double>(Qs[p1]);
    }
  }
  return (s0 - s1) * kInvUnit;   // X of Eq. 11
}

__global__ __launch_bounds__(256) void k_src_walks(SrcWalkArgs a) {
  const int lane = threadIdx.x & 63;
  const long long nwaves = static_cast<long long>(gridDim.x) * 4;
  const long long wv = static_cast<long long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const size_t n = static_cast<size_t>(a.n);
  auto slot_q = [&](int w) {
    return a.Q + (2 * static_cast<size_t>(w) + static_cast<size_t>(a.slot_ctl[2 * w + 1])) * n;
  };
  if (a.cend < 0 && a.ctl[1] == 0) {
    // the chunks do not fit the partial-sum buffer: one wave per half-edge
    for (long long p = wv; p < a.P; p += nwaves) {
      const long long nr = a.nr_pos[p];
      if (nr <= 0) continue;
      const int k = a.pos_slot[p];
      const int i = a.slot_row[k], j = a.col[k];
      const int len = a.tau_slot[k] - a.tilde_row[i];
      const uint64_t* Qs = slot_q(a.pos_w[p]);
      double acc = 0.0;
      for (long long r = lane; r < nr; r += 64)
        acc += walk_pair(i, j, r, len, a.k0, a.k1, a.rowptr, a.col, Qs);
      acc = wave_sum_d(acc);
      if (lane == 0) a.gacc[k] += acc / static_cast<double>(nr);
    }
    return;
  }
  // chunks [cb, ce): a batch given by the host, or all of them
  const long long cb = a.cend < 0 ? 0 : a.cbeg;
  const long long ce = a.cend < 0 ? a.ctl[0] : a.cend;
  const long long per = (ce - cb + nwaves - 1) / nwaves;
  const long long c0 = cb + wv * per;
  const long long c1 = min(ce, c0 + per);
  if (c0 >= c1) return;
  long long lo = 0, hi = a.P;   // chunk_off[lo] <= c0 < chunk_off[hi]
  while (hi - lo > 1) {
    const long long mid = (lo + hi) >> 1;
    if (a.chunk_off[mid] <= c0) lo = mid;
    else hi = mid;
  }
  long long p = lo;
  long long next = a.chunk_off[p + 1];
  for (long long c = c0; c < c1; ++c) {
    while (c >= next) {
      ++p;
      next = a.chunk_off[p + 1];
    }
    const int k = a.pos_slot[p];
    const long long nr = a.nr_pos[p];
    const long long r = (c - a.chunk_off[p]) * 64 + lane;
    double x = 0.0;
    if (r < nr) {
      const int i = a.slot_row[k], j = a.col[k];
      const int len = a.tau_slot[k] - a.tilde_row[i];
      x = walk_pair(i, j, r, len, a.k0, a.k1, a.rowptr, a.col, slot_q(a.pos_w[p]));
    }
    x = wave_sum_d(x);
    if (lane == 0) a.part[c - cb] = x;
  }
}

// The half's chunks inside this batch: [lo, hi), stored from part[lo - cb].
__device__ inline bool finish_range(const SrcWalkArgs& a, long long p, long long* cb,
                                    long long* lo, long long* hi) {
  if (a.nr_pos[p] <= 0) return false;
  *cb = a.cend < 0 ? 0 : a.cbeg;
  *lo = max(a.chunk_off[p], *cb);
  *hi = a.cend < 0 ? a.chunk_off[p + 1] : min(a.chunk_off[p + 1], a.cend);
  return *lo < *hi;
}

// gacc[k] += (chunk sums of half p in chunk order) / n_r, one thread per half
// with at most finish_seg chunks in the batch
__global__ __launch_bounds__(256) void k_src_finish(SrcWalkArgs a) {
  const long long p = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
  if (p >= a.P || (a.cend < 0 && a.ctl[1] == 0)) return;
  long long cb, lo, hi;
  if (!finish_range(a, p, &cb, &lo, &hi) || hi - lo > a.finish_seg) return;
  double s = 0.0;
  for (long long c = lo; c < hi; ++c) s += a.part[c - cb];
  a.gacc[a.pos_slot[p]] += s / static_cast<double>(a.nr_pos[p]);
}

// The same for the halves with more chunks: a workgroup per half, each thread
// summing one fixed segment of ceil(chunks / 256) in order, then the 256
// segment sums in order (the order depends only on the chunk count)
__global__ __launch_bounds__(256) void k_src_finish_long(SrcWalkArgs a) {
  __shared__ double s_seg[256];
  if (a.cend < 0 && a.ctl[1] == 0) return;
  const int tid = threadIdx.x;
  for (long long p = blockIdx.x; p < a.P; p += gridDim.x) {
    long long cb, lo, hi;
    if (!finish_range(a, p, &cb, &lo, &hi) || hi - lo <= a.finish_seg) continue;
    const long long seg = (hi - lo + 255) / 256;
    const long long c0 = lo + tid * seg;
    const long long c1 = min(hi, c0 + seg);
    double s = 0.0;
    for (long long c = c0; c < c1; ++c) s += a.part[c - cb];
    s_seg[tid] = s;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int q = 0; q < 256; ++q) t += s_seg[q];
      a.gacc[a.pos_slot[p]] += t / static_cast<double>(a.nr_pos[p]);
    }
    __syncthreads();
  }
}

// zero the slot's final column over its support list
__global__ __launch_bounds__(256) void k_src_clear(int n, int nslots_used, uint64_t* __restrict__ Q,
                                                   const int32_t* __restrict__ S,
                                                   const int32_t* __restrict__ slot_ctl) {
  const int w = blockIdx.x;
  if (w >= nslots_used) return;
  const int cnt = slot_ctl[2 * w];
  const int par = slot_ctl[2 * w + 1];
  uint64_t* Qs = Q + (2 * static_cast<size_t>(w) + par) * static_cast<size_t>(n);
  const int32_t* Ss = S + (2 * static_cast<size_t>(w) + par) * static_cast<size_t>(n);
  for (int e = threadIdx.x; e < cnt; e += 256) Qs[Ss[e]] = 0;
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* __restrict__ p, int64_t count,
                                                  uint64_t value) {
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < count;
       k += static_cast<int64_t>(gridDim.x) * 256)
    p[k] = value;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t count,
                                                  uint32_t value) {
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < count;
       k += static_cast<int64_t>(gridDim.x) * 256)
    p[k] = value;
}

// smallest and largest row truncation (tau_row) into mm[0] / mm[1]
__global__ __launch_bounds__(256) void k_tau_range(int n, const int32_t* __restrict__ tau_row,
                                                   unsigned long long* __restrict__ mm) {
  unsigned long long lo = ~0ull, hi = 0;
  for (int x = blockIdx.x * 256 + threadIdx.x; x < n; x += gridDim.x * 256) {
    const unsigned long long t = static_cast<unsigned long long>(tau_row[x]);
    lo = t < lo ? t : lo;
    hi = t > hi ? t : hi;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long a = __shfl_xor(lo, off, 64);
    const unsigned long long b = __shfl_xor(hi, off, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&mm[0], lo);
    atomicMax(&mm[1], hi);
  }
}

// vol[x] = sum over the neighbours j of x of d_j (one wave per node)
__global__ __launch_bounds__(256) void k_nbr_volume(int n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    int64_t* __restrict__ vol) {
  const int x = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (x >= n) return;
  int64_t v = 0;
  for (int k = rowptr[x] + lane; k < rowptr[x + 1]; k += 64) {
    const int j = col[k];
    v += rowptr[j + 1] - rowptr[j];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) vol[x] = v;
}

inline unsigned fill_grid(int64_t count) {
  const int64_t g = (count + 255) / 256;
  return static_cast<unsigned>(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_fill_u64(uint64_t* p, int64_t count, uint64_t value, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill_u64<<<fill_grid(count), 256, 0, st>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill_u32<<<fill_grid(count), 256, 0, st>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_nbr_volume(const DeviceGraph& g, int64_t* vol, hipStream_t st) {
  k_nbr_volume<<<static_cast<unsigned>((g.n + 3) / 4), 256, 0, st>>>(g.n, g.rowptr, g.col, vol);
  return hipGetLastError();
}

hipError_t launch_tau_range(int n, const int32_t* tau_row, unsigned long long* mm, hipStream_t st) {
  k_tau_range<<<fill_grid(n) < 1024 ? fill_grid(n) : 1024, 256, 0, st>>>(n, tau_row, mm);
  return hipGetLastError();
}

hipError_t launch_src_head(const SrcArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  k_src_head<<<grid, kT, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_src_scan(const SrcWalkArgs& a, hipStream_t st) {
  if (a.P <= 0) return hipSuccess;
  k_src_scan<<<1, 256, 0, st>>>(a.P, a.nr_pos, a.chunk_off, a.capacity, a.ctl);
  return hipGetLastError();
}

hipError_t launch_src_walk_batch(const SrcWalkArgs& a, hipStream_t st) {
  if (a.P <= 0) return hipSuccess;
  k_src_walks<<<kWalkGrid, 256, 0, st>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_src_finish<<<static_cast<unsigned>((a.P + 255) / 256), 256, 0, st>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_src_finish_long<<<static_cast<unsigned>(std::min<int64_t>(a.P, 1024)), 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_src_clear(const SrcWalkArgs& a, int nslots_used, hipStream_t st) {
  k_src_clear<<<nslots_used, 256, 0, st>>>(a.n, nslots_used, a.Qw, a.S, a.slot_ctl);
  return hipGetLastError();
}

__global__ void k_gather_i32(const int32_t* __restrict__ src, const int32_t* __restrict__ idx,
                             int32_t* __restrict__ dst, int64_t n) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x < n) dst[x] = src[idx[x]];
}

hipError_t launch_gather_i32(const int32_t* src, const int32_t* idx, int32_t* dst, int64_t n,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_gather_i32<<<static_cast<unsigned>((n + 255) / 256), 256, 0, st>>>(src, idx, dst, n);
  return hipGetLastError();
}

hipError_t launch_src_walks(const SrcWalkArgs& a, hipStream_t st) {
  hipError_t e = launch_src_scan(a, st);
  if (e == hipSuccess) e = launch_src_walk_batch(a, st);
  return e;
}

}  // namespace sc
