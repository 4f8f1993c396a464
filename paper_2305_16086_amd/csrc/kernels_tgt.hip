// Deterministic traversal kernels (Algorithm 2) for a block of B sources.
//
// Layout: the block state Y is node-major, Y[x * B + c] = p_l(x, s0 + c), so
// gathering a neighbour row reads B contiguous values.  Every floating-point
// reduction has a fixed order (no floating-point atomics), so results are
// bit-reproducible.  A row with at most kChunk neighbours is one wave's task;
// a heavier row is one workgroup's task (its four waves take interleaved
// 64-slot pieces and add their sums in wave order through LDS); a row above
// kGiant neighbours is cut into workgroup chunks whose partial sums a fix-up
// pass adds in chunk order.
#include "sc_internal.hpp"
#include "accumulate.hpp"
#include <hip/hip_ext.h>
#include "tau.hpp"

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
// One wave per row: the lanes stride over the row's slots (hub rows too) and a
// butterfly max gives the row's longest truncation.
__global__ __launch_bounds__(kThreads) void k_tau(int n, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ deg, int L,
                                                  double eps_tau, double lam, int max_L,
                                                  int32_t* __restrict__ tau_slot,
                                                  int32_t* __restrict__ tau_row,
                                                  unsigned long long* __restrict__ capped) {
  const int x = blockIdx.x * kWavesPerBlock + static_cast<int>(threadIdx.x) / 64;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  if (x >= n) return;   // uniform per wave
  int tmax = 0;
  int ncap = 0;
  const double di = static_cast<double>(deg[x]);
  const int end = rowptr[x + 1];
  for (int k = rowptr[x] + lane; k < end; k += 64) {
    int t = tau_uncapped(L, di, static_cast<double>(deg[col[k]]), eps_tau, lam);
    if (L <= 0 && t > max_L) {
      t = max_L;
      ++ncap;
    }
    tau_slot[k] = t;
    tmax = t > tmax ? t : tmax;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(tmax, off, 64);
    tmax = o > tmax ? o : tmax;
    ncap += __shfl_xor(ncap, off, 64);
  }
  if (lane == 0) {
    tau_row[x] = tmax;
    if (capped && ncap > 0) atomicAdd(capped, static_cast<unsigned long long>(ncap));
  }
}

// ------------------------------------------------------------------ CalTau (Algorithm 1)
// One wave per row x; for every slot (x -> j) the lanes hold the eigenpairs
// k = 2 .. omega-1 (1-based; up to kMaxOmega / 64 per lane) and the sums of
// Eq. 7 and Eq. 8 close with a fixed butterfly, so both halves of an edge get
// the same tau.  lam[omega], phi[n][omega] node-major, pair 1 the trivial one.
__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kThreads) void k_caltau(
    int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ deg, const double* __restrict__ lam,
    const double* __restrict__ phi, int omega, double eps_tau, int max_L,
    int32_t* __restrict__ tau_slot, int32_t* __restrict__ tau_row,
    unsigned long long* __restrict__ capped) {
  constexpr int P = kMaxOmega / 64;
  const int x = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (x >= n) return;
  bool on[P];
  double lk[P], ax[P];
  const double dx = static_cast<double>(deg[x]);
  const double sx = sqrt(dx);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int k = lane + 64 * p;   // 0-based index; the captured pairs are 1 .. omega-2
    on[p] = k >= 1 && k <= omega - 2;
    lk[p] = on[p] ? lam[k] : 0.0;
    ax[p] = on[p] ? phi[static_cast<size_t>(x) * omega + k] / sx : 0.0;
  }
  const double lw = fabs(lam[omega - 1]);
  const double shrink = 1.0 - lw * lw;
  const double log_inv = log(1.0 / lw);
  int tmax = 0;
  int ncap = 0;   // slots of this row cut to max_L (same on every lane)
  for (int s = rowptr[x]; s < rowptr[x + 1]; ++s) {
    const int j = col[s];
    const double dj = static_cast<double>(deg[j]);
    const double sj = sqrt(dj);
    double coef[P], pw[P], sq[P];
    double ups = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int k = lane + 64 * p;
      const double a = on[p] ? ax[p] - phi[static_cast<size_t>(j) * omega + k] / sj : 0.0;
      const double w = a * a;
      ups += w * (1.0 + lk[p]);
      coef[p] = on[p] ? w / (1.0 - lk[p]) : 0.0;
      sq[p] = lk[p] * lk[p];
      pw[p] = sq[p];   // lambda_k^(t+1) at t = 1
    }
    ups = wave_sum_d(ups);                                 // Eq. 7
    const double num = 1.0 / dx + 1.0 / dj - 2.0 / (dx * dj) - ups;
    int t = 1;
    while (t <= max_L) {
      double dl = 0.0;
#pragma unroll
      for (int p = 0; p < P; ++p) dl += coef[p] * pw[p];
      const double delta = wave_sum_d(dl);                 // Eq. 8 at t
      bool more;                                           // t <= Eq. 6 (Algorithm 1 line 5)
      if (eps_tau - delta <= 0.0) {
        more = true;                                       // Eq. 6 = +infinity
      } else if (num <= 0.0) {
        more = false;                                      // Eq. 6 = -infinity
      } else {
        const double f = ceil(log(num / ((eps_tau - delta) * shrink)) / log_inv - 1.0);
        more = static_cast<double>(t) <= f;
      }
      if (!more) break;
      t += 2;
#pragma unroll
      for (int p = 0; p < P; ++p) pw[p] *= sq[p];
    }
    const int tau = t > max_L ? max_L : t;
    if (lane == 0) tau_slot[s] = tau;
    ncap += t > max_L ? 1 : 0;
    tmax = tau > tmax ? tau : tmax;
  }
  if (lane == 0) {
    tau_row[x] = tmax;
    if (capped && ncap > 0) atomicAdd(capped, static_cast<unsigned long long>(ncap));
  }
}

// Ritz vectors of the Lanczos basis: phi[x][1 + c] = sum_i V[i + 1][x] Y[i][c]
// for c < p (Y: steps x p32 row-major, zero-padded to a multiple of 32
// columns); column 0 of phi is V's column 0 (the trivial eigenvector).

__global__ __launch_bounds__(256) void k_ritz(int64_t n, int64_t ld, const double* __restrict__ V,
                                              int steps, const double* __restrict__ Y, int p32,
                                              int p, int omega, double* __restrict__ phi) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (x >= n) return;
  const int c0 = blockIdx.y * kRitzCols;
  double acc[kRitzCols];
#pragma unroll
  for (int c = 0; c < kRitzCols; ++c) acc[c] = 0.0;
  for (int i = 0; i < steps; ++i) {
    const double v = V[static_cast<size_t>(i + 1) * ld + x];
    const double* yr = Y + static_cast<size_t>(i) * p32 + c0;
#pragma unroll
    for (int c = 0; c < kRitzCols; ++c) acc[c] += v * yr[c];
  }
#pragma unroll
  for (int c = 0; c < kRitzCols; ++c)
    if (c0 + c < p) phi[static_cast<size_t>(x) * omega + 1 + c0 + c] = acc[c];
  if (blockIdx.y == 0) phi[static_cast<size_t>(x) * omega] = V[x];
}

// ------------------------------------------------------------------ indicator masks
// Waves [0, B) mark bit c of mask[u] (and the node's bit in anymask) for every
// u in N(s_set + c) in buffer `buf`; waves [B, 2B) clear what block s_clear
// marked in the other buffer.  Each buffer only ever holds one block's bits,
// so clearing may zero whole words.
__device__ inline void mask_update_wave(int w, int lane, int n, const MaskJob& mj,
                                        const int32_t* __restrict__ rowptr,
                                        const int32_t* __restrict__ col) {
  if (w >= 2 * mj.B) return;
  const bool set = w < mj.B;
  const int c = set ? w : w - mj.B;
  const int sb = set ? mj.s_set : mj.s_clear;
  const int s = sb + c;
  if (sb < 0 || s >= n) return;
  const int b = set ? mj.buf : 1 - mj.buf;
  unsigned long long* mk = mj.mask + static_cast<size_t>(b) * mj.mwords;
  unsigned* am = mj.anymask + static_cast<size_t>(b) * mj.awords;
  const unsigned long long bit = 1ull << c;
  for (int k = rowptr[s] + lane; k < rowptr[s + 1]; k += 64) {
    const int u = col[k];
    if (set) {
      atomicOr(&mk[u], bit);
      atomicOr(&am[u >> 5], 1u << (u & 31));
    } else {
      mk[u] = 0ull;
      am[u >> 5] = 0u;
    }
  }
}

__global__ void k_mask_update(int n, MaskJob mj, const int32_t* __restrict__ rowptr,
                              const int32_t* __restrict__ col) {
  mask_update_wave(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6), threadIdx.x & 63, n, mj,
                   rowptr, col);
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

// Pointers the row kernels need (passed by value).
template <typename T>
struct RowArgs {
  const Task* tasks;          // wave tasks: one light row each (used when B < 64)
  int ntasks;
  const Task* ptasks;         // wave tasks: runs of consecutive light rows (B = 64)
  int nptasks;
  const int32_t* rowptr;
  const Task* wg_tasks;       // workgroup tasks (heavy rows, giant-row chunks)
  int nwg;
  int row_blocks;             // nwg + workgroups of wave tasks
  const int32_t* col;
  const T* inv_deg;
  T* partials;
  // fused accumulation of the previous step (workgroups after row_blocks)
  const int32_t* slot_row;
  const double* inv_deg_d;
  AccJob acc;
  // rows known to be zero in Yp (nz[u] == 0, B = 64 only)
  const uint8_t* nz;
  // the next block's mask update (workgroups after the accumulation)
  int acc_blocks;
  MaskJob mj;
  int n;
};

// gacc[k] += (Y[s][c] - Y[j][c]) / d_s for slot k = (s -> j), l <= tau_k (Eq. 9)
template <typename T, int B>
__device__ inline void accumulate_slot(const RowArgs<T>& a, const T* Y, int k) {
  accumulate_half<T, B>(a.acc, a.slot_row, a.col, a.inv_deg_d, Y, k);
}

// Sum over the 64-slot pieces first, first + step, ... of [beg, end) of the
// neighbour rows of Yp (column c); lanes c, c+B, ... share a column and are
// combined at the end.
template <typename T, int B, bool kSkip = false>
__device__ inline T gather_pieces(const RowArgs<T>& a, const T* __restrict__ Yp, int beg, int end,
                                  int first, int step, int lane, int c, int gq) {
  constexpr int G = 64 / B;
  constexpr int kBatch = sizeof(T) == 4 ? 32 : 16;   // gathers in flight per lane
  static_assert(!kSkip || G == 1, "zero-row skipping needs one column per lane");
  T acc = T(0);
  for (int base = beg + 64 * first; base < end; base += 64 * step) {
    const int cnt = min(64, end - base);
    const int myu = lane < cnt ? a.col[base + lane] : 0;
    if (kSkip) {
      // gather only the slots whose row is nonzero, in slot order: the skipped
      // rows are exact zeros, so the sum is that of the full slot loop
      unsigned long long rem = __ballot(lane < cnt && a.nz[myu]);
      while (rem) {
        T v[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          v[q] = T(0);
          if (rem) {
            const int l = __builtin_ctzll(rem);
            rem &= rem - 1ull;
            const int u = __builtin_amdgcn_readlane(myu, l);
            v[q] = Yp[static_cast<size_t>(u) * B + c];
          }
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) acc += v[q];
      }
    } else if (G == 1) {
      for (int jj = 0; jj < cnt; jj += kBatch) {
        T v[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          const int l = jj + q;   // wave-uniform
          const int u = __builtin_amdgcn_readlane(myu, l & 63);
          v[q] = l < cnt ? Yp[static_cast<size_t>(u) * B + c] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) acc += v[q];
      }
    } else {
      // uniform trip count: every lane takes part in each shuffle (a shuffle
      // from an inactive lane would read 0), the add is predicated instead
      for (int j0 = 0; j0 < cnt; j0 += G) {
        const int jj = j0 + gq;
        const int u = __shfl(myu, jj, 64);
        if (jj < cnt) acc += Yp[static_cast<size_t>(u) * B + c];
      }
    }
  }
  return reduce_groups<T, B>(acc);
}

// Same traversal for the two-hop step: neighbour u contributes 1/d_u to column
// c when bit c of mask[u] is set (u is a neighbour of source c).
template <typename T, int B>
__device__ inline T twohop_pieces(const RowArgs<T>& a, const unsigned long long* __restrict__ mask,
                                  const unsigned* __restrict__ anymask, int beg, int end,
                                  int first, int step, int lane, int c, int gq) {
  constexpr int G = 64 / B;
  T acc = T(0);
  for (int base = beg + 64 * first; base < end; base += 64 * step) {
    const int cnt = min(64, end - base);
    const int myu = lane < cnt ? a.col[base + lane] : 0;
    // the small bitmap filters out the neighbours no column marks
    const bool hit = lane < cnt && ((anymask[myu >> 5] >> (myu & 31)) & 1u);
    const unsigned long long mym = hit ? mask[myu] : 0ull;
    const T myw = hit ? a.inv_deg[myu] : T(0);
    if (__ballot(hit) == 0ull) continue;
    if (G == 1) {
      const int mlo = static_cast<int>(mym & 0xFFFFFFFFull);
      const int mhi = static_cast<int>(mym >> 32);
      unsigned long long ph = __ballot(hit);   // only marked slots contribute, in slot order
      while (ph) {
        const int jj = __builtin_ctzll(ph);
        ph &= ph - 1ull;
        const unsigned long long mk =
            (static_cast<unsigned long long>(static_cast<unsigned>(__builtin_amdgcn_readlane(mhi, jj))) << 32) |
            static_cast<unsigned>(__builtin_amdgcn_readlane(mlo, jj));
        if ((mk >> c) & 1ull) acc += bcast(myw, jj);
      }
    } else {
      for (int j0 = 0; j0 < cnt; j0 += G) {
        const int jj = j0 + gq;
        const unsigned long long mk = __shfl(mym, jj, 64);
        const T w = __shfl(myw, jj, 64);
        if (jj < cnt && ((mk >> c) & 1ull)) acc += w;
      }
    }
  }
  return reduce_groups<T, B>(acc);
}

// A run of consecutive light rows with at most 64 slots in total (B = 64):
// one coalesced load of their neighbour lists, all gathers in flight, and the
// row sums closed in slot order (the same order as the one-row path).
template <typename T, int B>
__device__ inline void gather_run(const RowArgs<T>& a, const T* __restrict__ Yp, const Task& tk,
                                  int lane, T* __restrict__ Yn) {
  constexpr int kBatch = sizeof(T) == 4 ? 32 : 16;
  const int nrows = tk.part;
  const int cnt = tk.end - tk.beg;
  const int myu = lane < cnt ? a.col[tk.beg + lane] : 0;
  const int myend = lane < nrows ? a.rowptr[tk.row + lane + 1] - tk.beg : 0;
  const T myinv = lane < nrows ? a.inv_deg[tk.row + lane] : T(0);
  T acc = T(0);
  int ri = 0;
  int bnd = __builtin_amdgcn_readlane(myend, 0);
  for (int jj = 0; jj < cnt; jj += kBatch) {
    T v[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int l = jj + q;
      const int u = __builtin_amdgcn_readlane(myu, l & 63);
      v[q] = l < cnt ? Yp[static_cast<size_t>(u) * B + lane] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int l = jj + q;
      if (l < cnt) {
        acc += v[q];
        if (l + 1 == bnd) {
          Yn[static_cast<size_t>(tk.row + ri) * B + lane] = acc * bcast(myinv, ri);
          acc = T(0);
          ++ri;
          bnd = __builtin_amdgcn_readlane(myend, ri & 63);
        }
      }
    }
  }
}

template <typename T, int B>
__device__ inline void twohop_run(const RowArgs<T>& a, const unsigned long long* __restrict__ mask,
                                  const unsigned* __restrict__ anymask, const Task& tk, int lane,
                                  T* __restrict__ Y, uint8_t* __restrict__ nzw) {
  const int nrows = tk.part;
  const int cnt = tk.end - tk.beg;
  const int myu = lane < cnt ? a.col[tk.beg + lane] : 0;
  const int myend = lane < nrows ? a.rowptr[tk.row + lane + 1] - tk.beg : 0;
  const T myinv = lane < nrows ? a.inv_deg[tk.row + lane] : T(0);
  const bool hit = lane < cnt && ((anymask[myu >> 5] >> (myu & 31)) & 1u);
  const unsigned long long mym = hit ? mask[myu] : 0ull;
  const T myw = hit ? a.inv_deg[myu] : T(0);
  const unsigned long long hits = __ballot(hit);
  const int mlo = static_cast<int>(mym & 0xFFFFFFFFull);
  const int mhi = static_cast<int>(mym >> 32);
  // row by row, visiting only the slots some column marks (in slot order, so
  // the sums are those of the full slot loop: the other slots add nothing)
  int rbeg = 0;
  for (int ri = 0; ri < nrows; ++ri) {
    const int rend = __builtin_amdgcn_readlane(myend, ri);
    const unsigned long long below_end = rend >= 64 ? ~0ull : ((1ull << rend) - 1ull);
    const unsigned long long below_beg = (1ull << rbeg) - 1ull;   // rbeg < 64
    unsigned long long rh = hits & below_end & ~below_beg;
    T acc = T(0);
    while (rh) {
      const int l = __builtin_ctzll(rh);
      rh &= rh - 1ull;
      const unsigned long long mk =
          (static_cast<unsigned long long>(static_cast<unsigned>(__builtin_amdgcn_readlane(mhi, l))) << 32) |
          static_cast<unsigned>(__builtin_amdgcn_readlane(mlo, l));
      if ((mk >> lane) & 1ull) acc += bcast(myw, l);
    }
    Y[static_cast<size_t>(tk.row + ri) * B + lane] = acc * bcast(myinv, ri);
    if (nzw) {
      const bool any = __ballot(acc != T(0)) != 0ull;
      if (lane == 0) nzw[tk.row + ri] = any ? 1 : 0;
    }
    rbeg = rend;
  }
}

// Workgroup task: the four waves' sums are added in wave order; a whole row
// is scaled by 1/d and stored, a giant-row chunk goes to its partial row.
template <typename T, int B>
__device__ inline void wg_finish(const RowArgs<T>& a, const Task& tk, T sum, int wave, int lane,
                                 T* __restrict__ Y) {
  __shared__ T red[kWavesPerBlock][64];
  red[wave][lane] = sum;
  __syncthreads();
  if (wave == 0 && lane < B) {
    T tot = red[0][lane];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) tot += red[w][lane];
    if (tk.part < 0)
      Y[static_cast<size_t>(tk.row) * B + lane] = tot * a.inv_deg[tk.row];
    else
      a.partials[static_cast<size_t>(tk.part) * B + lane] = tot;
  }
}

// ------------------------------------------------------------------ Y2 from masks
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_twohop(RowArgs<T> a,
                                                     const unsigned long long* __restrict__ mask,
                                                     const unsigned* __restrict__ anymask,
                                                     T* __restrict__ Y, uint8_t* __restrict__ nzw) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c = lane % B;
  const int gq = lane / B;
  if (static_cast<int>(blockIdx.x) < a.nwg) {
    const Task tk = a.wg_tasks[blockIdx.x];
    const T sum = twohop_pieces<T, B>(a, mask, anymask, tk.beg, tk.end, wave, kWavesPerBlock, lane, c, gq);
    wg_finish<T, B>(a, tk, sum, wave, lane, Y);   // heavy rows keep their flag (1)
    return;
  }
  const int t = (blockIdx.x - a.nwg) * kWavesPerBlock + wave;
  if (B == 64) {
    if (t >= a.nptasks) return;
    const Task tk = a.ptasks[t];
    if (tk.end - tk.beg <= 64) {
      twohop_run<T, B>(a, mask, anymask, tk, lane, Y, nzw);
      return;
    }
    const T sum = twohop_pieces<T, B>(a, mask, anymask, tk.beg, tk.end, 0, 1, lane, c, gq);
    Y[static_cast<size_t>(tk.row) * B + c] = sum * a.inv_deg[tk.row];
    if (nzw) {
      const bool any = __ballot(sum != T(0)) != 0ull;
      if (lane == 0) nzw[tk.row] = any ? 1 : 0;
    }
    return;
  }
  if (t >= a.ntasks) return;
  const Task tk = a.tasks[t];
  const T sum = twohop_pieces<T, B>(a, mask, anymask, tk.beg, tk.end, 0, 1, lane, c, gq);
  if (gq == 0) Y[static_cast<size_t>(tk.row) * B + c] = sum * a.inv_deg[tk.row];
}

// gather_run when the rows flagged zero in nz are exact zeros: only the slots
// of nonzero rows are gathered; each row's sum still closes in slot order and
// rows whose slots are all skipped are written as zeros.
template <typename T, int B>
__device__ inline void gather_run_skip(const RowArgs<T>& a, const T* __restrict__ Yp,
                                       const Task& tk, int lane, T* __restrict__ Yn) {
  constexpr int kBatch = sizeof(T) == 4 ? 32 : 16;
  const int nrows = tk.part;
  const int cnt = tk.end - tk.beg;
  const int myu = lane < cnt ? a.col[tk.beg + lane] : 0;
  const int myend = lane < nrows ? a.rowptr[tk.row + lane + 1] - tk.beg : 0;
  const T myinv = lane < nrows ? a.inv_deg[tk.row + lane] : T(0);
  unsigned long long rem = __ballot(lane < cnt && a.nz[myu]);
  T acc = T(0);
  int ri = 0;
  int bnd = __builtin_amdgcn_readlane(myend, 0);
  while (rem) {
    T v[kBatch];
    int sl[kBatch];   // wave-uniform slot of each gather, 64 = none
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      v[q] = T(0);
      sl[q] = 64;
      if (rem) {
        const int l = __builtin_ctzll(rem);
        rem &= rem - 1ull;
        const int u = __builtin_amdgcn_readlane(myu, l);
        v[q] = Yp[static_cast<size_t>(u) * B + lane];
        sl[q] = l;
      }
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      if (sl[q] < 64) {
        while (bnd <= sl[q]) {   // close the rows that end before this slot
          Yn[static_cast<size_t>(tk.row + ri) * B + lane] = acc * bcast(myinv, ri);
          acc = T(0);
          ++ri;
          bnd = __builtin_amdgcn_readlane(myend, ri & 63);
        }
        acc += v[q];
      }
    }
  }
  for (; ri < nrows; ++ri) {
    Yn[static_cast<size_t>(tk.row + ri) * B + lane] = acc * bcast(myinv, ri);
    acc = T(0);
  }
}

// ------------------------------------------------------------------ dense propagation
// Workgroups [0, nwg): heavy rows and giant-row chunks; then wave tasks; then
// the accumulation of the step held in Yp (fused, saves a launch).  Register
// use is held to 6 waves per SIMD: more waves with shallower gather batches run
// the kernel faster alone but slow the concurrent tail of the block pipeline.
// kSkip (B = 64): rows with nz[u] == 0 are exact zeros in Yp and are not gathered.
template <typename T, int B, bool kSkip>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_propagate(RowArgs<T> a, const T* __restrict__ Yp,
                                                        T* __restrict__ Yn) {
  if (static_cast<int>(blockIdx.x) >= a.row_blocks) {
    const int t = blockIdx.x - a.row_blocks;
    if (t < a.acc_blocks) {
      accumulate_slot<T, B>(a, Yp, a.acc.kbeg + t * kThreads + threadIdx.x);
    } else {
      mask_update_wave((t - a.acc_blocks) * kWavesPerBlock + (threadIdx.x >> 6),
                       threadIdx.x & 63, a.n, a.mj, a.rowptr, a.col);
    }
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c = lane % B;
  const int gq = lane / B;
  if (static_cast<int>(blockIdx.x) < a.nwg) {
    const Task tk = a.wg_tasks[blockIdx.x];
    const T sum =
        gather_pieces<T, B, kSkip>(a, Yp, tk.beg, tk.end, wave, kWavesPerBlock, lane, c, gq);
    wg_finish<T, B>(a, tk, sum, wave, lane, Yn);
    return;
  }
  const int t = (blockIdx.x - a.nwg) * kWavesPerBlock + wave;
  if (B == 64) {
    if (t >= a.nptasks) return;
    const Task tk = a.ptasks[t];
    if (tk.end - tk.beg <= 64) {
      if (kSkip)
        gather_run_skip<T, B>(a, Yp, tk, lane, Yn);
      else
        gather_run<T, B>(a, Yp, tk, lane, Yn);
      return;
    }
    const T sum = gather_pieces<T, B, kSkip>(a, Yp, tk.beg, tk.end, 0, 1, lane, c, gq);
    Yn[static_cast<size_t>(tk.row) * B + c] = sum * a.inv_deg[tk.row];
    return;
  }
  if (t >= a.ntasks) return;
  const Task tk = a.tasks[t];
  const T sum = gather_pieces<T, B>(a, Yp, tk.beg, tk.end, 0, 1, lane, c, gq);
  if (gq == 0) Yn[static_cast<size_t>(tk.row) * B + c] = sum * a.inv_deg[tk.row];
}

// Giant rows: Y[row] = inv_deg[row] * (sum of the chunk partials in chunk order).
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_fixup(const HeavyRow* __restrict__ giant, int ngiant,
                                                    const T* __restrict__ inv_deg,
                                                    const T* __restrict__ partials,
                                                    T* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int h = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (h >= ngiant || lane >= B) return;
  const HeavyRow hr = giant[h];
  T acc = T(0);
  for (int p = 0; p < hr.nparts; ++p) acc += partials[static_cast<size_t>(hr.part0 + p) * B + lane];
  Y[static_cast<size_t>(hr.row) * B + lane] = acc * inv_deg[hr.row];
}

// standalone accumulation (the last step of a block)
template <typename T, int B>
__global__ void k_accumulate(RowArgs<T> a, const T* __restrict__ Y) {
  accumulate_slot<T, B>(a, Y, a.acc.kbeg + blockIdx.x * blockDim.x + threadIdx.x);
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
                      int32_t* tau_slot, int32_t* tau_row, hipStream_t st,
                      unsigned long long* capped) {
  k_tau<<<grid_for(g.n, kWavesPerBlock), kThreads, 0, st>>>(
      g.n, g.rowptr, g.col, g.deg, L, eps_tau, lam, max_L, tau_slot, tau_row, capped);
  return hipGetLastError();
}

hipError_t launch_caltau(const DeviceGraph& g, const double* lam, const double* phi, int omega,
                         double eps_tau, int max_L, int32_t* tau_slot, int32_t* tau_row,
                         hipStream_t st, unsigned long long* capped) {
  if (omega < 2 || omega > kMaxOmega) return hipErrorInvalidValue;
  k_caltau<<<grid_for(g.n, kWavesPerBlock), kThreads, 0, st>>>(
      g.n, g.rowptr, g.col, g.deg, lam, phi, omega, eps_tau, max_L, tau_slot, tau_row, capped);
  return hipGetLastError();
}

hipError_t launch_ritz(int64_t n, int64_t ld, const double* V, int steps, const double* Y,
                       int p32, int p, int omega, double* phi, hipStream_t st) {
  if (p32 % kRitzCols != 0 || p > p32 || 1 + p > omega) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(p32 / kRitzCols));
  k_ritz<<<grid, 256, 0, st>>>(n, ld, V, steps, Y, p32, p, omega, phi);
  return hipGetLastError();
}

MaskJob mask_job(const DeviceGraph& g, int s_set, int s_clear, int B, int buf,
                 unsigned long long* mask, unsigned* anymask) {
  MaskJob mj;
  mj.s_set = s_set;
  mj.s_clear = s_clear;
  mj.B = B;
  mj.buf = buf;
  mj.mwords = g.n;
  mj.awords = (g.n + 31) / 32;
  mj.mask = mask;
  mj.anymask = anymask;
  return mj;
}

hipError_t launch_mask_update(const DeviceGraph& g, int s_set, int s_clear, int B, int buf,
                              unsigned long long* mask, unsigned* anymask, hipStream_t st) {
  k_mask_update<<<grid_for(2 * B, kWavesPerBlock), kThreads, 0, st>>>(
      g.n, mask_job(g, s_set, s_clear, B, buf, mask, anymask), g.rowptr, g.col);
  return hipGetLastError();
}

#define SC_DISPATCH_B(B, CALL)                        \
  switch (B) {                                        \
    case 64: { constexpr int kB = 64; CALL; } break;  \
    case 32: { constexpr int kB = 32; CALL; } break;  \
    case 16: { constexpr int kB = 16; CALL; } break;  \
    default: return hipErrorInvalidValue;             \
  }

template <typename T>
const T* inv_deg_of(const DeviceGraph& g);
template <>
const float* inv_deg_of<float>(const DeviceGraph& g) { return g.inv_deg_f; }
template <>
const double* inv_deg_of<double>(const DeviceGraph& g) { return g.inv_deg_d; }

template <typename T>
RowArgs<T> row_args(const DeviceGraph& g, int B, T* partials, const AccJob& acc) {
  RowArgs<T> a;
  a.tasks = g.tasks;
  a.ntasks = g.ntasks;
  a.ptasks = g.ptasks;
  a.nptasks = g.nptasks;
  a.rowptr = g.rowptr;
  a.wg_tasks = g.wg_tasks;
  a.nwg = g.nwg;
  a.row_blocks = g.nwg + static_cast<int>(grid_for(B == 64 ? g.nptasks : g.ntasks, kWavesPerBlock));
  a.col = g.col;
  a.inv_deg = inv_deg_of<T>(g);
  a.partials = partials;
  a.slot_row = g.slot_row;
  a.inv_deg_d = g.inv_deg_d;
  a.acc = acc;
  a.nz = nullptr;
  a.acc_blocks = 0;
  a.mj = MaskJob{};
  a.n = g.n;
  return a;
}

inline int acc_blocks(const AccJob& acc) {
  return acc_job_set(acc) ? static_cast<int>(grid_for(acc.kend - acc.kbeg, kThreads))
                                          : 0;
}

template <typename T>
hipError_t launch_fixup(const DeviceGraph& g, int B, const T* partials, T* Y, hipStream_t st) {
  if (g.ngiant == 0) return hipSuccess;
  SC_DISPATCH_B(B, (k_fixup<T, kB><<<grid_for(g.ngiant, kWavesPerBlock), kThreads, 0, st>>>(
                        g.giant, g.ngiant, inv_deg_of<T>(g), partials, Y)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_twohop(const DeviceGraph& g, int B, const unsigned long long* mask,
                         const unsigned* anymask, T* Y, T* partials, uint8_t* nz, hipStream_t st) {
  const RowArgs<T> a = row_args<T>(g, B, partials, AccJob{});
  SC_DISPATCH_B(B, (k_twohop<T, kB><<<a.row_blocks, kThreads, 0, st>>>(a, mask, anymask, Y,
                                                                        B == 64 ? nz : nullptr)));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_fixup<T>(g, B, partials, Y, st);
}

template <typename T>
hipError_t launch_propagate_rows(const DeviceGraph& g, int B, const T* Yp, T* Yn, T* partials,
                                 const AccJob& acc, hipStream_t st, const uint8_t* nz,
                                 hipEvent_t ev_start, hipEvent_t ev_stop, const MaskJob* mj) {
  RowArgs<T> a = row_args<T>(g, B, partials, acc);
  a.acc_blocks = acc_blocks(acc);
  int mask_blocks = 0;
  if (mj && mj->B > 0) {
    a.mj = *mj;
    mask_blocks = static_cast<int>(grid_for(2 * mj->B, kWavesPerBlock));
  }
  const int blocks = a.row_blocks + a.acc_blocks + mask_blocks;
  if (B == 64 && nz) {
    a.nz = nz;
    hipExtLaunchKernelGGL(k_propagate<T, 64, true>, dim3(blocks), dim3(kThreads), 0, st,
                          ev_start, ev_stop, 0, a, Yp, Yn);
  } else {
    SC_DISPATCH_B(B, (hipExtLaunchKernelGGL(k_propagate<T, kB, false>, dim3(blocks),
                                            dim3(kThreads), 0, st, ev_start, ev_stop, 0, a, Yp,
                                            Yn)));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_propagate(const DeviceGraph& g, int B, const T* Yp, T* Yn, T* partials,
                            const AccJob& acc, hipStream_t st) {
  const hipError_t e = launch_propagate_rows<T>(g, B, Yp, Yn, partials, acc, st, nullptr);
  if (e != hipSuccess) return e;
  return launch_fixup<T>(g, B, partials, Yn, st);
}

template <typename T>
hipError_t launch_accumulate(const DeviceGraph& g, int B, const T* Y, const AccJob& acc,
                             hipStream_t st) {
  const int blocks = acc_blocks(acc);
  if (blocks == 0) return hipSuccess;
  const RowArgs<T> a = row_args<T>(g, B, nullptr, acc);
  SC_DISPATCH_B(B, (k_accumulate<T, kB><<<blocks, kThreads, 0, st>>>(a, Y)));
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
                                         const unsigned*, float*, float*, uint8_t*, hipStream_t);
template hipError_t launch_twohop<double>(const DeviceGraph&, int, const unsigned long long*,
                                          const unsigned*, double*, double*, uint8_t*, hipStream_t);
template hipError_t launch_propagate_rows<float>(const DeviceGraph&, int, const float*, float*,
                                                float*, const AccJob&, hipStream_t, const uint8_t*,
                                                hipEvent_t, hipEvent_t, const MaskJob*);
template hipError_t launch_propagate_rows<double>(const DeviceGraph&, int, const double*, double*,
                                                 double*, const AccJob&, hipStream_t,
                                                 const uint8_t*, hipEvent_t, hipEvent_t,
                                                 const MaskJob*);
template hipError_t launch_fixup<float>(const DeviceGraph&, int, const float*, float*, hipStream_t);
template hipError_t launch_fixup<double>(const DeviceGraph&, int, const double*, double*, hipStream_t);
template hipError_t launch_propagate<float>(const DeviceGraph&, int, const float*, float*,
                                            float*, const AccJob&, hipStream_t);
template hipError_t launch_propagate<double>(const DeviceGraph&, int, const double*, double*,
                                             double*, const AccJob&, hipStream_t);
template hipError_t launch_accumulate<float>(const DeviceGraph&, int, const float*,
                                             const AccJob&, hipStream_t);
template hipError_t launch_accumulate<double>(const DeviceGraph&, int, const double*,
                                              const AccJob&, hipStream_t);

}  // namespace sc
