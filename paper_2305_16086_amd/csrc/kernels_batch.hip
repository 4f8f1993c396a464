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
// column-major, nb[off + t * 64 + i] = t-th neighbour of the group's row i
// (the zero row n past the row's degree), so one load instruction fetches
// slot t of consecutive rows.  A lane owns (row, V consecutive columns) and
// adds the row's neighbour values in the order the single-graph kernels use
// for the same B (sequential for B = 64; G = 64 / B interleaved partial sums
// combined as a butterfly for B = 16, 32; heavy rows in four interleaved
// 64-slot pieces; giant rows in chunks), so with B in {16, 32, 64} a graph's
// results are bitwise equal to the single-graph path.
#include "sc_internal.hpp"

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

__device__ inline int wave_max_i(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

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

// Neighbour slots [b, e) of one lane's row taken in the workgroup-task order:
// four interleaved 64-slot pieces (piece p belongs to part p mod 4), each part
// with G interleaved partial sums, parts added in order.
template <typename T, int B, int V, int G>
__device__ inline void chunk_sum(const int32_t* __restrict__ nb, const T* Y, int cv, int b, int e,
                                 T (&tot)[V]) {
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
            const Pack<T, V> p = load_pack<T, V>(Y + static_cast<size_t>(nb[t * 64]) * B + cv);
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

// Propagation of one graph's block state: Yn = P Yp for all rows.
template <typename T, int B, int NT>
__device__ inline void rows_step(const BatchGraph& g, const T* Yp, T* Yn) {
  constexpr int V = (B * sizeof(T) < 16) ? B : static_cast<int>(16 / sizeof(T));
  constexpr int LR = B / V;           // lanes per row
  constexpr int RPP = 64 / LR;        // rows per pass
  constexpr int G = B >= 16 ? 64 / B : 1;
  constexpr bool kEmul = B >= 16;     // single-graph kernels exist for these widths
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = g.n;
  const T* __restrict__ inv = inv_of<T>(g);
  const int cv = (lane % LR) * V;
  for (int gi = wave; gi < g.ngroups; gi += NW) {
    const int2 gd = g.grp[gi];
#pragma unroll 1
    for (int p = 0; p < LR; ++p) {
      const int i = p * RPP + lane / LR;
      const int2 rd = g.grp_rows[gi * 64 + i];
      const int x = rd.x;
      const int d = rd.y;
      const int wmax = wave_max_i(d);
      const int32_t* __restrict__ nb = g.nb + gd.x + i;
      T out[V];
      if (kEmul && wmax > kChunk) {
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
                const Pack<T, V> pk = load_pack<T, V>(Yp + static_cast<size_t>(nb[t * 64]) * B + cv);
#pragma unroll
                for (int q = 0; q < V; ++q) acc[gg][q] += pk.v[q];
              }
            }
          }
          tree<T, G, V>(acc, out);
        } else if (d <= kGiant) {
          chunk_sum<T, B, V, G>(nb, Yp, cv, 0, d, out);
        } else {
#pragma unroll
          for (int q = 0; q < V; ++q) out[q] = T(0);
          for (int b = 0; b < d; b += kGiantChunk) {
            T c[V];
            chunk_sum<T, B, V, G>(nb, Yp, cv, b, min(b + kGiantChunk, d), c);
#pragma unroll
            for (int q = 0; q < V; ++q) out[q] += c[q];
          }
        }
      } else {
        // light rows: slot t goes to partial sum t mod G; padding reads the zero row
        constexpr int kU = 8;
        T acc[G][V];
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
          for (int q = 0; q < V; ++q) acc[gg][q] = T(0);
        for (int t0 = 0; t0 < wmax; t0 += kU) {
          int u[kU];
#pragma unroll
          for (int q = 0; q < kU; ++q) u[q] = (t0 + q < wmax) ? nb[(t0 + q) * 64] : n;
#pragma unroll
          for (int q = 0; q < kU; ++q) {
            const Pack<T, V> pk = load_pack<T, V>(Yp + static_cast<size_t>(u[q]) * B + cv);
#pragma unroll
            for (int e = 0; e < V; ++e) acc[q % G][e] += pk.v[e];
          }
        }
        tree<T, G, V>(acc, out);
      }
      if (x < n) {
        const T s = inv[x];
        Pack<T, V> o;
#pragma unroll
        for (int q = 0; q < V; ++q) o.v[q] = out[q] * s;
        *reinterpret_cast<Pack<T, V>*>(Yn + static_cast<size_t>(x) * B + cv) = o;
      }
    }
  }
}

constexpr int kAccRegs = 2;   // accumulation slots kept in registers per thread

// One item: block [s0, s0 + B) of graph g, all steps.
template <typename T, int B, int NT>
__device__ void run_item(const BatchGraph& g, int s0, T* Y0, T* Y1, int* s_tmax) {
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
    rows_step<T, B, NT>(g, Yp, Yn);
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

template <typename T, int NT, bool kLds>
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
    T* Y1 = Y0 + static_cast<int64_t>(g.n + 1) * g.B;
    switch (g.B) {
      case 1: run_item<T, 1, NT>(g, w.s0, Y0, Y1, &s_tmax); break;
      case 2: run_item<T, 2, NT>(g, w.s0, Y0, Y1, &s_tmax); break;
      case 4: run_item<T, 4, NT>(g, w.s0, Y0, Y1, &s_tmax); break;
      case 8: run_item<T, 8, NT>(g, w.s0, Y0, Y1, &s_tmax); break;
      case 16: run_item<T, 16, NT>(g, w.s0, Y0, Y1, &s_tmax); break;
      case 32: run_item<T, 32, NT>(g, w.s0, Y0, Y1, &s_tmax); break;
      default: run_item<T, 64, NT>(g, w.s0, Y0, Y1, &s_tmax); break;
    }
  }
}

__global__ void k_fill_i32(int32_t* p, int count, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// min / max of tau_row over a range (integer atomics: order-independent)
__global__ void k_tau_range(const int32_t* __restrict__ tau_row, int64_t count, int32_t* mm) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  atomicMin(&mm[0], tau_row[i]);
  atomicMax(&mm[1], tau_row[i]);
}

template <typename T, int NT, bool kLds>
const void* batch_kernel() {
  return reinterpret_cast<const void*>(&k_batch<T, NT, kLds>);
}

}  // namespace

template <typename T>
const void* batch_kernel_ptr(int nt, bool lds) {
  if (!lds) return batch_kernel<T, 256, false>();   // slab states: 256-thread workgroups
  switch (nt) {
    case 256: return batch_kernel<T, 256, true>();
    case 512: return batch_kernel<T, 512, true>();
    case 1024: return batch_kernel<T, 1024, true>();
    default: return nullptr;
  }
}

template <typename T>
hipError_t launch_batch(int nt, bool lds, int grid, size_t dyn_lds, const BatchGraph* graphs,
                        const BatchItem* items, int nitems, int* ticket, T* slabs,
                        int64_t slab_elems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (!lds) {
    if (nt != 256) return hipErrorInvalidValue;
    k_batch<T, 256, false><<<grid, 256, 0, st>>>(graphs, items, nitems, ticket, slabs, slab_elems);
    return hipGetLastError();
  }
  switch (nt) {
    case 256:
      k_batch<T, 256, true><<<grid, 256, dyn_lds, st>>>(graphs, items, nitems, ticket, slabs, slab_elems);
      break;
    case 512:
      k_batch<T, 512, true><<<grid, 512, dyn_lds, st>>>(graphs, items, nitems, ticket, slabs, slab_elems);
      break;
    case 1024:
      k_batch<T, 1024, true><<<grid, 1024, dyn_lds, st>>>(graphs, items, nitems, ticket, slabs, slab_elems);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int count, int value, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill_i32<<<(count + 255) / 256, 256, 0, st>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_tau_range(const int32_t* tau_row, int64_t count, int32_t* mm, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_tau_range<<<static_cast<unsigned>((count + 255) / 256), 256, 0, st>>>(tau_row, count, mm);
  return hipGetLastError();
}

template const void* batch_kernel_ptr<float>(int, bool);
template const void* batch_kernel_ptr<double>(int, bool);
template hipError_t launch_batch<float>(int, bool, int, size_t, const BatchGraph*,
                                        const BatchItem*, int, int*, float*, int64_t,
                                        hipStream_t);
template hipError_t launch_batch<double>(int, bool, int, size_t, const BatchGraph*,
                                         const BatchItem*, int, int*, double*, int64_t,
                                         hipStream_t);

}  // namespace sc
