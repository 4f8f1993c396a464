// Batched persistent traversal: Algorithm 2 for many graphs in one launch.
//
// A work item is one source block [s0, s0 + B) of one graph.  A persistent
// workgroup takes items from an atomic ticket counter (items are sorted by
// estimated cost, longest first) and runs every step l = 2..tmax of its item
// by itself: the two block states Y_(l-1), Y_l (node-major, Y[x * B + c] =
// p_l(x, s0 + c), plus a zero row at index n) sit in LDS when they fit,
// otherwise in a per-workgroup slab of device memory.  Steps are separated by
// workgroup barriers only; nothing crosses workgroups, so no grid-wide
// synchronisation exists and every wave reaches the exit once the ticket
// counter passes the item count.
//
// Rows are read through a sliced layout: the rows of a graph sorted by degree
// (descending) form groups of 64, and a group's neighbour lists are stored
// column-major in 32-bit words, word w of row i at nb[off + w * 64 + i]
// holding slots K w .. K w + K - 1 (K = 2: 16-bit ids, for graphs below 65535
// nodes; K = 1: 32-bit ids), so one load instruction fetches a word of 64
// consecutive rows; lanes past their row's degree read the zero row n.  A lane owns (row, V consecutive columns) and
// adds the row's neighbour values in the order the single-graph kernels use
// for the same B (sequential for B = 64; G = 64 / B interleaved partial sums
// combined as a butterfly for B = 16, 32; heavy rows in four interleaved
// 64-slot pieces; giant rows in chunks), so with B in {16, 32, 64} a graph's
// results are bitwise equal to the single-graph path.
#include "sc_internal.hpp"
#include "tau.hpp"

namespace sc {

namespace {

template <typename T, int V>
struct alignas(sizeof(T) * V) Pack {
  T v[V];
};

template <typename T, int V>
__device__ inline Pack<T, V> load_pack(const T* p) {
  return *reinterpret_cast<const Pack<T, V>*>(p);
}

// Pointers the hot loop reads are cast to the global address space so that
// their loads are global (not flat) loads: flat loads also count against the
// LDS counter, which would make every wait for an LDS gather wait for the
// prefetched neighbour words as well.
#define SC_GLOBAL __attribute__((address_space(1)))
template <typename P>
__device__ inline const SC_GLOBAL P* gptr(const P* p) {
  return (const SC_GLOBAL P*)p;
}

__device__ inline int wave_max_i(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

template <typename T>
__device__ inline const T* grp_inv_of(const BatchGraph& g);
template <>
__device__ inline const float* grp_inv_of<float>(const BatchGraph& g) { return g.grp_invf; }
template <>
__device__ inline const double* grp_inv_of<double>(const BatchGraph& g) { return g.grp_invd; }

template <typename T>
__device__ inline const T* inv_of(const BatchGraph& g);
template <>
__device__ inline const float* inv_of<float>(const BatchGraph& g) { return g.inv_f; }
template <>
__device__ inline const double* inv_of<double>(const BatchGraph& g) { return g.inv_d; }

// Butterfly combination of G partial sums, as the lanes of a group combine
// them in the single-graph kernels (own value first).
template <typename T, int G, int V>
__device__ inline void tree(T (&acc)[G][V], T (&out)[V]) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1)
#pragma unroll
    for (int g = 0; g < G; g += 2 * off)
#pragma unroll
      for (int e = 0; e < V; ++e) acc[g][e] = acc[g][e] + acc[g + off][e];
#pragma unroll
  for (int e = 0; e < V; ++e) out[e] = acc[0][e];
}

// Where a lane's row keeps its neighbour ids: the first kBatchSlots in its
// record, the rest column-major in nb from its column base.
struct RowIds {
  const SC_GLOBAL uint32_t* rec;   // record words 4 ..
  const SC_GLOBAL uint32_t* col;   // nb + column base
};

// Slot t of a lane's row (K = 2: two 16-bit ids per word, low half first).
template <int K>
__device__ inline int slot_index(const RowIds& r, int t) {
  const uint32_t w = t < kBatchSlots ? r.rec[t / K] : r.col[((t - kBatchSlots) / K) * 64];
  return K == 1 ? static_cast<int>(w) : static_cast<int>((w >> (16 * (t & 1))) & 0xFFFFu);
}

// Neighbour slots [b, e) of one lane's row taken in the workgroup-task order:
// four interleaved 64-slot pieces (piece p belongs to part p mod 4), each part
// with G interleaved partial sums, parts added in order.
template <typename T, int B, int V, int G, int K>
__device__ inline void chunk_sum(const RowIds& ids, const T* Y, int cv, int b, int e, T (&tot)[V]) {
#pragma unroll 1
  for (int w = 0; w < kWavesPerBlock; ++w) {
    T acc[G][V];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int q = 0; q < V; ++q) acc[g][q] = T(0);
    for (int pb = b + 64 * w; pb < e; pb += 64 * kWavesPerBlock) {
      const int pe = min(pb + 64, e);
      for (int t0 = pb; t0 < pe; t0 += G) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int t = t0 + g;
          if (t < pe) {
            const Pack<T, V> p = load_pack<T, V>(Y + static_cast<size_t>(slot_index<K>(ids, t)) * B + cv);
#pragma unroll
            for (int q = 0; q < V; ++q) acc[g][q] += p.v[q];
          }
        }
      }
    }
    T r[V];
    tree<T, G, V>(acc, r);
#pragma unroll
    for (int q = 0; q < V; ++q) tot[q] = (w == 0) ? r[q] : tot[q] + r[q];
  }
}

// Rows of more than kChunk neighbours (and lanes sharing their pass) in the
// order of the single-graph workgroup tasks; giant rows chunk by chunk.
template <typename T, int B, int V, int G, int K>
__device__ inline void heavy_sum(const RowIds& ids, const T* Yp, int cv, int d, T (&out)[V]) {
  if (d <= kChunk) {
    T acc[G][V];
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
      for (int q = 0; q < V; ++q) acc[gg][q] = T(0);
    for (int t0 = 0; t0 < d; t0 += G) {
#pragma unroll
      for (int gg = 0; gg < G; ++gg) {
        const int t = t0 + gg;
        if (t < d) {
          const Pack<T, V> pk = load_pack<T, V>(Yp + static_cast<size_t>(slot_index<K>(ids, t)) * B + cv);
#pragma unroll
          for (int q = 0; q < V; ++q) acc[gg][q] += pk.v[q];
        }
      }
    }
    tree<T, G, V>(acc, out);
  } else if (d <= kGiant) {
    chunk_sum<T, B, V, G, K>(ids, Yp, cv, 0, d, out);
  } else {
#pragma unroll
    for (int q = 0; q < V; ++q) out[q] = T(0);
    for (int b = 0; b < d; b += kGiantChunk) {
      T c[V];
      chunk_sum<T, B, V, G, K>(ids, Yp, cv, b, min(b + kGiantChunk, d), c);
#pragma unroll
      for (int q = 0; q < V; ++q) out[q] += c[q];
    }
  }
}

// Slots per gather batch; group widths are padded to a multiple of it.
static_assert(kBatchSlots == 8, "gather_batch is written for 8 slots");

// One batch of 8 slots (8 / K words): every slot inside the padded group width
// holds a real neighbour or the zero row n, so no slot needs a mask; slot s
// goes to partial sum s mod G (the single-graph order).
template <typename T, int B, int V, int G, int K, bool kFirst>
__device__ inline void gather_batch(const uint32_t* wd, const T* Yp, int cv, T (&acc)[G][V]) {
  int u[kBatchSlots];
#pragma unroll
  for (int s = 0; s < kBatchSlots; ++s)
    u[s] = K == 1 ? static_cast<int>(wd[s]) : static_cast<int>((wd[s / 2] >> (16 * (s & 1))) & 0xFFFFu);
  Pack<T, V> pk[kBatchSlots];
#pragma unroll
  for (int s = 0; s < kBatchSlots; ++s) pk[s] = load_pack<T, V>(Yp + static_cast<uint32_t>(u[s] * B + cv));
  // the first batch starts each partial sum at its first value (0 + v == v)
#pragma unroll
  for (int s = 0; s < kBatchSlots; ++s)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      if (kFirst && s < G)
        acc[s][e] = pk[s].v[e];
      else
        acc[s % G][e] += pk[s].v[e];
    }
}

// A row record: (row, degree, column base, 0) and the first kBatchSlots ids.
template <int K>
struct Rec {
  static constexpr int kWords = 4 + kBatchSlots / K;
  uint32_t w[kWords];
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int K>
__device__ inline Rec<K> load_rec(const SC_GLOBAL uint32_t* rec, uint32_t r) {
  Rec<K> out;
  const SC_GLOBAL u32x4* p = (const SC_GLOBAL u32x4*)(rec + r * static_cast<uint32_t>(Rec<K>::kWords));
#pragma unroll
  for (int j = 0; j < Rec<K>::kWords / 4; ++j) {
    const u32x4 v = p[j];
    out.w[4 * j] = v.x;
    out.w[4 * j + 1] = v.y;
    out.w[4 * j + 2] = v.z;
    out.w[4 * j + 3] = v.w;
  }
  return out;
}

// One pass: the rows of one record per lane, gathered from Yp into Yn.
template <typename T, int B, int K>
__device__ __forceinline__ void row_pass(const Rec<K>& rc, T sc, uint32_t ri, int n,
                                         const SC_GLOBAL uint32_t* __restrict__ recs,
                                         const SC_GLOBAL uint32_t* __restrict__ nbw,
                                         const T* Yp, T* Yn, int cv) {
  constexpr int V = (B * sizeof(T) < 16) ? B : static_cast<int>(16 / sizeof(T));
  constexpr int G = B >= 16 ? 64 / B : 1;
  constexpr bool kEmul = B >= 16;     // single-graph kernels exist for these widths
  constexpr int kW = kBatchSlots / K; // words per batch
  const int x = static_cast<int>(rc.w[0]);
  const int d = static_cast<int>(rc.w[1]);
  const uint32_t cb = rc.w[2];
  const int wmax = __builtin_amdgcn_readfirstlane(d);
  T out[V];
  if (kEmul && wmax > kChunk) {
    const RowIds ids{recs + ri * static_cast<uint32_t>(Rec<K>::kWords) + 4, nbw + cb};
    heavy_sum<T, B, V, G, K>(ids, Yp, cv, d, out);
  } else {
    T acc[G][V];
    gather_batch<T, B, V, G, K, true>(rc.w + 4, Yp, cv, acc);
    for (int t0 = kBatchSlots; t0 < wmax; t0 += kBatchSlots) {
      uint32_t wd[kW];
#pragma unroll
      for (int w = 0; w < kW; ++w) wd[w] = nbw[cb + static_cast<uint32_t>(((t0 - kBatchSlots) / K + w) * 64)];
      gather_batch<T, B, V, G, K, false>(wd, Yp, cv, acc);
    }
    tree<T, G, V>(acc, out);
  }
  if (x < n) {
    Pack<T, V> o;
#pragma unroll
    for (int e = 0; e < V; ++e) o.v[e] = out[e] * sc;
    *reinterpret_cast<Pack<T, V>*>(Yn + static_cast<uint32_t>(x * B + cv)) = o;
  }
}

// Propagation of one graph's block state: Yn = P Yp for all rows.  Each wave
// walks its passes (group gi = wave, wave + NW, ...; LR passes per group) and
// loads the next pass's row records (which carry the first neighbour ids)
// before it gathers the current pass; two register sets alternate.  Rows are
// sorted by degree, so a pass's width is the degree of its first row (lane 0).
template <typename T, int B, int NT, int K>
__device__ inline void rows_step(const BatchGraph& g, const T* Yp, T* Yn) {
  constexpr int V = (B * sizeof(T) < 16) ? B : static_cast<int>(16 / sizeof(T));
  constexpr int LR = B / V;           // lanes per row
  constexpr int RPP = 64 / LR;        // rows per pass
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = g.n;
  const SC_GLOBAL uint32_t* __restrict__ nbw = gptr(g.nb);
  const SC_GLOBAL uint32_t* __restrict__ recs = gptr(g.rec);
  const SC_GLOBAL T* __restrict__ ginv = gptr(grp_inv_of<T>(g));
  const int cv = (lane % LR) * V;
  const int nq = wave < g.ngroups ? ((g.ngroups - 1 - wave) / NW + 1) * LR : 0;
  // record index of pass q for this lane
  auto rec_index = [&](int q) -> uint32_t {
    return static_cast<uint32_t>((wave + (q / LR) * NW) * 64 + (q % LR) * RPP + lane / LR);
  };
  Rec<K> ra, rb;
  T ia = T(0), ib = T(0);
  uint32_t ja = 0, jb = 0;
  if (nq > 0) {
    ja = rec_index(0);
    ra = load_rec<K>(recs, ja);
    ia = ginv[ja];
  }
  // the loads for pass q + 1 are issued unconditionally (the last pass is
  // reloaded at the end) so that the wait for pass q counts exactly
  for (int q = 0; q < nq; q += 2) {
    jb = rec_index(min(q + 1, nq - 1));
    rb = load_rec<K>(recs, jb);
    ib = ginv[jb];
    row_pass<T, B, K>(ra, ia, ja, n, recs, nbw, Yp, Yn, cv);
    if (q + 1 >= nq) break;
    ja = rec_index(min(q + 2, nq - 1));
    ra = load_rec<K>(recs, ja);
    ia = ginv[ja];
    row_pass<T, B, K>(rb, ib, jb, n, recs, nbw, Yp, Yn, cv);
  }
}

constexpr int kAccRegs = 2;   // accumulation slots kept in registers per thread

// One item: block [s0, s0 + B) of graph g, all steps.
template <typename T, int B, int NT, int K>
__device__ __forceinline__ void run_item(const BatchGraph& g, int s0, T* Y0, T* Y1, int* s_tmax) {
  const int tid = threadIdx.x;
  const int n = g.n;
  const int ncols = min(B, n - s0);
  const int kbeg = g.rowptr[s0];
  const int kend = g.rowptr[s0 + ncols];
  const T* __restrict__ inv = inv_of<T>(g);
  // largest truncation of the block's sources
  if (tid < 64) {
    int t = tid < ncols ? g.tau_row[s0 + tid] : 0;
    t = wave_max_i(t);
    if (tid == 0) *s_tmax = t;
  }
  // zero state (and the zero row of the second buffer)
  const int64_t elems = static_cast<int64_t>(n + 1) * B;
  for (int64_t k = tid; k < elems; k += NT) Y0[k] = T(0);
  for (int k = tid; k < B; k += NT) Y1[static_cast<size_t>(n) * B + k] = T(0);
  __syncthreads();
  const int tmax = *s_tmax;
  if (tmax < 2) return;   // the l = 0, 1 terms are closed-form (initial gacc)
  // l = 1: p_1(x, s) = 1/d_x for x in N(s)
  for (int k = kbeg + tid; k < kend; k += NT) {
    const int s = g.slot_row[k];
    const int x = g.col[k];
    Y0[static_cast<size_t>(x) * B + (s - s0)] = inv[x];
  }
  // accumulation slots kept in registers
  int rs[kAccRegs], rj[kAccRegs], rt[kAccRegs];
  double rinv[kAccRegs], racc[kAccRegs];
#pragma unroll
  for (int r = 0; r < kAccRegs; ++r) {
    const int k = kbeg + tid + r * NT;
    rt[r] = -1;
    rs[r] = rj[r] = 0;
    rinv[r] = racc[r] = 0.0;
    if (k < kend) {
      rs[r] = g.slot_row[k];
      rj[r] = g.col[k];
      rt[r] = g.tau_slot[k];
      rinv[r] = g.inv_d[rs[r]];
      racc[r] = g.gacc[k];
    }
  }
  __syncthreads();
  T* Yp = Y0;
  T* Yn = Y1;
  for (int ell = 2; ell <= tmax; ++ell) {
    rows_step<T, B, NT, K>(g, Yp, Yn);
    __syncthreads();
    // gacc[k] += (p_l(s,s) - p_l(j,s)) / d_s for l <= tau_k (Eq. 9)
#pragma unroll
    for (int r = 0; r < kAccRegs; ++r) {
      if (ell <= rt[r]) {
        const int c = rs[r] - s0;
        const double pss = static_cast<double>(Yn[static_cast<size_t>(rs[r]) * B + c]);
        const double pjs = static_cast<double>(Yn[static_cast<size_t>(rj[r]) * B + c]);
        racc[r] += (pss - pjs) * rinv[r];
      }
    }
    for (int k = kbeg + kAccRegs * NT + tid; k < kend; k += NT) {
      if (ell > g.tau_slot[k]) continue;
      const int s = g.slot_row[k];
      const int c = s - s0;
      const int j = g.col[k];
      const double pss = static_cast<double>(Yn[static_cast<size_t>(s) * B + c]);
      const double pjs = static_cast<double>(Yn[static_cast<size_t>(j) * B + c]);
      g.gacc[k] += (pss - pjs) * g.inv_d[s];
    }
    T* t = Yp;
    Yp = Yn;
    Yn = t;
  }
#pragma unroll
  for (int r = 0; r < kAccRegs; ++r)
    if (rt[r] >= 0) g.gacc[kbeg + tid + r * NT] = racc[r];
}

template <typename T, int NT, bool kLds, int B>
__global__ __launch_bounds__(NT) void k_batch(const BatchGraph* __restrict__ graphs,
                                              const BatchItem* __restrict__ items, int nitems,
                                              int* __restrict__ ticket, T* __restrict__ slabs,
                                              int64_t slab_elems) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  __shared__ int s_tmax;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(ticket, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= nitems) return;
    const BatchItem w = items[it];
    const BatchGraph g = graphs[w.graph];
    T* Y0 = kLds ? reinterpret_cast<T*>(smem) : slabs + static_cast<int64_t>(blockIdx.x) * slab_elems;
    T* Y1 = Y0 + static_cast<int64_t>(g.n + 1) * B;
    if (g.narrow)
      run_item<T, B, NT, 2>(g, w.s0, Y0, Y1, &s_tmax);
    else
      run_item<T, B, NT, 1>(g, w.s0, Y0, Y1, &s_tmax);
  }
}

__global__ void k_fill_i32(int32_t* p, int count, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// index of the graph holding global index i: off[g] <= i < off[g + 1]
__device__ inline int graph_of(const int64_t* __restrict__ off, int G, int64_t i) {
  int lo = 0, hi = G;   // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void k_batch_prologue(const BatchGraph* __restrict__ graphs,
                                 const int64_t* __restrict__ node_off, int G, int64_t total,
                                 int32_t* mm, unsigned long long* capped) {
  const int64_t X = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  int tlo = INT_MAX, thi = 0;
  int ncap = 0;
  if (X < total) {
    const int gi = graph_of(node_off, G, X);
    const BatchGraph& g = graphs[gi];
    if (g.active) {
      const int x = static_cast<int>(X - node_off[gi]);
      const double di = static_cast<double>(g.deg[x]);
      const double eps_tau = g.eps;
      int tmax = 0;
      for (int k = g.rowptr[x]; k < g.rowptr[x + 1]; ++k) {
        const int j = g.col[k];
        int t;
        if (g.L < 0) {
          t = g.tau_slot[k];   // CalTau wrote it (and counted its own capped slots)
        } else {
          t = tau_uncapped(g.L, di, static_cast<double>(g.deg[j]), eps_tau, g.lam);
          if (g.L == 0 && t > g.max_L) {
            t = g.max_L;
            ++ncap;
          }
          const_cast<int32_t*>(g.tau_slot)[k] = t;
        }
        tmax = t > tmax ? t : tmax;
        double v = g.inv_d[x];                       // l = 0: p_0(x,x)/d_x
        if (t >= 1) v -= g.inv_d[j] * g.inv_d[x];    // l = 1: -p_1(j,x)/d_x
        g.gacc[k] = v;
      }
      const_cast<int32_t*>(g.tau_row)[x] = tmax;
      tlo = tmax;
      thi = tmax;
    }
  }
  if (mm) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      tlo = min(tlo, __shfl_xor(tlo, off, 64));
      thi = max(thi, __shfl_xor(thi, off, 64));
      ncap += __shfl_xor(ncap, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      if (tlo != INT_MAX) atomicMin(&mm[0], tlo);
      atomicMax(&mm[1], thi);
      if (capped && ncap > 0) atomicAdd(capped, static_cast<unsigned long long>(ncap));
    }
  }
}

__global__ void k_batch_combine(const BatchGraph* __restrict__ graphs,
                                const int64_t* __restrict__ edge_off, int G, int64_t total) {
  const int64_t E = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (E >= total) return;
  const int gi = graph_of(edge_off, G, E);
  const BatchGraph& g = graphs[gi];
  if (!g.active) return;
  const int e = static_cast<int>(E - edge_off[gi]);
  g.out[e] = g.gacc[g.half_slot[e]] + g.gacc[g.half_slot[e + g.m]];
}

template <typename T, int NT, bool kLds, int B>
const void* batch_kernel() {
  return reinterpret_cast<const void*>(&k_batch<T, NT, kLds, B>);
}

template <typename T, int NT, bool kLds>
const void* batch_kernel_b(int B) {
  switch (B) {
    case 1: return batch_kernel<T, NT, kLds, 1>();
    case 2: return batch_kernel<T, NT, kLds, 2>();
    case 4: return batch_kernel<T, NT, kLds, 4>();
    case 8: return batch_kernel<T, NT, kLds, 8>();
    case 16: return batch_kernel<T, NT, kLds, 16>();
    case 32: return batch_kernel<T, NT, kLds, 32>();
    case 64: return batch_kernel<T, NT, kLds, 64>();
    default: return nullptr;
  }
}

template <typename T, int NT, bool kLds, int B>
void launch_one(int grid, size_t dyn, const BatchGraph* graphs, const BatchItem* items, int nitems,
                int* ticket, T* slabs, int64_t slab_elems, hipStream_t st) {
  k_batch<T, NT, kLds, B><<<grid, NT, dyn, st>>>(graphs, items, nitems, ticket, slabs, slab_elems);
}

template <typename T, int NT, bool kLds>
hipError_t launch_b(int B, int grid, size_t dyn, const BatchGraph* graphs, const BatchItem* items,
                    int nitems, int* ticket, T* slabs, int64_t slab_elems, hipStream_t st) {
  switch (B) {
    case 1: launch_one<T, NT, kLds, 1>(grid, dyn, graphs, items, nitems, ticket, slabs, slab_elems, st); break;
    case 2: launch_one<T, NT, kLds, 2>(grid, dyn, graphs, items, nitems, ticket, slabs, slab_elems, st); break;
    case 4: launch_one<T, NT, kLds, 4>(grid, dyn, graphs, items, nitems, ticket, slabs, slab_elems, st); break;
    case 8: launch_one<T, NT, kLds, 8>(grid, dyn, graphs, items, nitems, ticket, slabs, slab_elems, st); break;
    case 16: launch_one<T, NT, kLds, 16>(grid, dyn, graphs, items, nitems, ticket, slabs, slab_elems, st); break;
    case 32: launch_one<T, NT, kLds, 32>(grid, dyn, graphs, items, nitems, ticket, slabs, slab_elems, st); break;
    case 64: launch_one<T, NT, kLds, 64>(grid, dyn, graphs, items, nitems, ticket, slabs, slab_elems, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

template <typename T>
const void* batch_kernel_ptr(int nt, bool lds, int B) {
  if (!lds) return batch_kernel_b<T, 256, false>(B);   // slab states: 256-thread workgroups
  switch (nt) {
    case 256: return batch_kernel_b<T, 256, true>(B);
    case 512: return batch_kernel_b<T, 512, true>(B);
    case 1024: return batch_kernel_b<T, 1024, true>(B);
    default: return nullptr;
  }
}

template <typename T>
hipError_t launch_batch(int nt, bool lds, int B, int grid, size_t dyn_lds, const BatchGraph* graphs,
                        const BatchItem* items, int nitems, int* ticket, T* slabs,
                        int64_t slab_elems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (!lds) {
    if (nt != 256) return hipErrorInvalidValue;
    return launch_b<T, 256, false>(B, grid, 0, graphs, items, nitems, ticket, slabs, slab_elems, st);
  }
  switch (nt) {
    case 256: return launch_b<T, 256, true>(B, grid, dyn_lds, graphs, items, nitems, ticket, slabs, slab_elems, st);
    case 512: return launch_b<T, 512, true>(B, grid, dyn_lds, graphs, items, nitems, ticket, slabs, slab_elems, st);
    case 1024: return launch_b<T, 1024, true>(B, grid, dyn_lds, graphs, items, nitems, ticket, slabs, slab_elems, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_i32(int32_t* p, int count, int value, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill_i32<<<(count + 255) / 256, 256, 0, st>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_batch_prologue(const BatchGraph* graphs, const int64_t* node_off, int G,
                                 int64_t total_rows, int32_t* mm, unsigned long long* capped,
                                 hipStream_t st) {
  if (total_rows <= 0) return hipSuccess;
  k_batch_prologue<<<static_cast<unsigned>((total_rows + 255) / 256), 256, 0, st>>>(
      graphs, node_off, G, total_rows, mm, capped);
  return hipGetLastError();
}

hipError_t launch_batch_combine(const BatchGraph* graphs, const int64_t* edge_off, int G,
                                int64_t total_edges, hipStream_t st) {
  if (total_edges <= 0) return hipSuccess;
  k_batch_combine<<<static_cast<unsigned>((total_edges + 255) / 256), 256, 0, st>>>(
      graphs, edge_off, G, total_edges);
  return hipGetLastError();
}

template const void* batch_kernel_ptr<float>(int, bool, int);
template const void* batch_kernel_ptr<double>(int, bool, int);
template hipError_t launch_batch<float>(int, bool, int, int, size_t, const BatchGraph*,
                                        const BatchItem*, int, int*, float*, int64_t,
                                        hipStream_t);
template hipError_t launch_batch<double>(int, bool, int, int, size_t, const BatchGraph*,
                                         const BatchItem*, int, int*, double*, int64_t,
                                         hipStream_t);

}  // namespace sc
