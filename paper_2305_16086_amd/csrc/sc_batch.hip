// Batched all-edge SC: many graphs, one persistent launch per LDS class,
// optional hipGraph replay, and a measured choice of the block width B per
// graph-size bucket.  Each graph's result is TGT (Algorithm 2) with the
// truncation of Theorem 3.2 (or a given L), exactly as sc_all_edges_ex.
#include "sc_host.hpp"

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using sc::fail;

namespace {

constexpr int kClasses = 4;         // LDS <= budget/4, <= budget/2, <= budget, device slab
constexpr int kThreadChoices = 3;   // workgroup sizes 256, 512, 1024
constexpr int kLaunchMax = kClasses * 7 * kThreadChoices;   // launches per (class, B, threads)
constexpr int kClassThreads[kClasses] = {256, 512, 1024, 256};
constexpr size_t kStaticLds = 64;   // the kernel's own __shared__ words (rounded up)
constexpr size_t kSlabCap = size_t(8) << 30;   // device memory for slab states

struct TuneEntry {
  int lg_n, lg_d, precision, block;
  int threads;   // workgroup size of the persistent launch, 0: the LDS class's default
};

int threads_index(int nt) { return nt == 1024 ? 2 : nt == 512 ? 1 : 0; }

int lg_floor(double x) { return x < 1.0 ? 0 : static_cast<int>(std::floor(std::log2(x))); }

}  // namespace

struct sc_batch {
  int device = 0;
  std::vector<sc_graph*> graphs;
  std::vector<int64_t> node_off, slot_off, edge_off;   // [G + 1]
  std::vector<int32_t> dmin;                           // smallest degree per graph
  // sliced neighbour lists (built once)
  std::vector<uint32_t*> nb;
  std::vector<int32_t> narrow;
  std::vector<uint32_t*> rec;
  std::vector<float*> grp_invf;
  std::vector<double*> grp_invd;
  std::vector<int32_t> ngroups;
  // run buffers (batch-wide, indexed by the offsets)
  int32_t* tau_slot = nullptr;
  int32_t* tau_row = nullptr;
  double* gacc = nullptr;
  double* out_dev = nullptr;       // host-output runs: results before the copy
  double* out_pinned = nullptr;    // pinned staging of out_dev
  sc::BatchGraph* d_graphs = nullptr;
  int64_t* d_node_off = nullptr;   // [G + 1]
  int64_t* d_edge_off = nullptr;   // [G + 1]
  sc::BatchItem* d_items = nullptr;
  size_t items_cap = 0;
  int32_t* d_misc = nullptr;       // [0, kLaunchMax): tickets; [kLaunchMax, +2): tau min / max;
                                   // [kLaunchMax + 2, +2): capped half-edges (one 64-bit word)
  int32_t* h_misc = nullptr;       // pinned copy of the tau range and the capped count
  void* slabs = nullptr;
  size_t slab_bytes = 0;
  size_t lds_budget = 0;
  int cus = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t hgraph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string exec_key;            // arguments the captured graph was made for
  std::vector<TuneEntry> tune;

  void drop_exec() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (hgraph) (void)hipGraphDestroy(hgraph);
    exec = nullptr;
    hgraph = nullptr;
    exec_key.clear();
  }

  void release() {
    drop_exec();
    for (auto* g : graphs) {
      if (g) {
        g->release();
        delete g;
      }
    }
    graphs.clear();
    for (auto*& p : nb) sc::dev_free(p);
    for (auto*& p : rec) sc::dev_free(p);
    for (auto*& p : grp_invf) sc::dev_free(p);
    for (auto*& p : grp_invd) sc::dev_free(p);
    sc::dev_free(tau_slot);
    sc::dev_free(tau_row);
    sc::dev_free(gacc);
    sc::dev_free(out_dev);
    if (out_pinned) (void)hipHostFree(out_pinned);
    out_pinned = nullptr;
    if (h_misc) (void)hipHostFree(h_misc);
    h_misc = nullptr;
    sc::dev_free(d_graphs);
    sc::dev_free(d_node_off);
    sc::dev_free(d_edge_off);
    sc::dev_free(d_items);
    sc::dev_free(d_misc);
    if (slabs) (void)sc::tracked_free(slabs);
    slabs = nullptr;
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
  }
};

namespace {

// Rows sorted by degree (descending, ties by id) in groups of 64: per row a
// record (row, degree, column base, 0, first kBatchSlots neighbour ids) and
// the remaining ids column-major in nb, two 16-bit ids per word when n <
// 65535; padded with the zero row n; 1/degree per record in invf / invd.
int build_slices(const sc::HostCSR& h, std::vector<uint32_t>& rec, std::vector<uint32_t>& nb,
                 std::vector<float>& invf, std::vector<double>& invd, int* narrow) {
  const int n = h.n;
  const int K = n < 65535 ? 2 : 1;
  const int KS = sc::kBatchSlots;
  const int RW = 4 + KS / K;
  *narrow = K == 2 ? 1 : 0;
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return h.deg[a] > h.deg[b]; });
  const int ngroups = (n + 63) / 64;
  const uint32_t pad_word = K == 2 ? (static_cast<uint32_t>(n) << 16) | static_cast<uint32_t>(n)
                                   : static_cast<uint32_t>(n);
  std::vector<int64_t> base(ngroups);
  int64_t off = 0;
  for (int gi = 0; gi < ngroups; ++gi) {
    const int64_t width = h.deg[order[gi * 64]];
    const int64_t padded = (width + KS - 1) / KS * KS;
    base[gi] = off;
    off += (padded - KS) / K * 64;
    if (off > INT32_MAX - sc::kBatchWordPad) return fail(SC_EINVAL, "batch graph too large");
  }
  nb.assign(static_cast<size_t>(off) + sc::kBatchWordPad, pad_word);
  rec.assign(static_cast<size_t>(ngroups) * 64 * RW, pad_word);
  invf.assign(static_cast<size_t>(ngroups) * 64, 0.0f);
  invd.assign(static_cast<size_t>(ngroups) * 64, 0.0);
  auto put = [&](uint32_t& w, int t, uint32_t id) {
    if (K == 1) {
      w = id;
    } else {
      const int sh = 16 * (t & 1);
      w = (w & ~(0xFFFFu << sh)) | (id << sh);
    }
  };
  for (int gi = 0; gi < ngroups; ++gi) {
    for (int i = 0; i < 64; ++i) {
      const size_t r = static_cast<size_t>(gi) * 64 + i;
      uint32_t* rr = &rec[r * RW];
      const bool real = gi * 64 + i < n;
      const int x = real ? order[gi * 64 + i] : n;
      const int dx = real ? h.deg[x] : 0;
      rr[0] = static_cast<uint32_t>(x);
      rr[1] = static_cast<uint32_t>(dx);
      rr[2] = static_cast<uint32_t>(base[gi] + i);
      rr[3] = 0;
      if (!real) continue;
      invf[r] = h.inv_f[x];
      invd[r] = h.inv_d[x];
      for (int t = 0; t < dx; ++t) {
        const uint32_t id = static_cast<uint32_t>(h.col[h.rowptr[x] + t]);
        if (t < KS)
          put(rr[4 + t / K], t, id);
        else
          put(nb[static_cast<size_t>(base[gi] + i) + static_cast<size_t>((t - KS) / K) * 64], t, id);
      }
    }
  }
  return SC_OK;
}

size_t state_bytes(int n, int B, size_t tsize) {
  return 2 * static_cast<size_t>(n + 1) * B * tsize;
}

bool valid_block(int B) {
  return B == 1 || B == 2 || B == 4 || B == 8 || B == 16 || B == 32 || B == 64;
}

// Block width when neither the options nor a tuning entry fix it: the widest
// block whose states fit a quarter of the LDS (four workgroups per CU), else
// the widest that fits at all, else 8 in a device slab.
int default_block(const sc_batch* b, int gi, size_t tsize) {
  const int n = b->graphs[gi]->d.n;
  for (int B = 64; B >= 1; B >>= 1)
    if (state_bytes(n, B, tsize) + kStaticLds <= b->lds_budget / 4) return B;
  for (int B = 64; B >= 1; B >>= 1)
    if (state_bytes(n, B, tsize) + kStaticLds <= b->lds_budget) return B;
  return 8;
}

void bucket_of(const sc_batch* b, int gi, int* lg_n, int* lg_d) {
  const sc_graph* g = b->graphs[gi];
  *lg_n = lg_floor(static_cast<double>(g->d.n));
  *lg_d = lg_floor(static_cast<double>(g->d.nslots) / static_cast<double>(g->d.n));
}

int block_for(const sc_batch* b, int gi, const sc_options& o, int* threads = nullptr) {
  const size_t tsize = o.precision == 1 ? sizeof(double) : sizeof(float);
  if (threads) *threads = 0;
  if (o.block > 0) return o.block;
  int ln, ld;
  bucket_of(b, gi, &ln, &ld);
  for (const TuneEntry& e : b->tune)
    if (e.lg_n == ln && e.lg_d == ld && e.precision == o.precision) {
      if (threads) *threads = e.threads;
      return e.block;
    }
  return default_block(b, gi, tsize);
}

int class_of(const sc_batch* b, int n, int B, size_t tsize) {
  const size_t need = state_bytes(n, B, tsize) + kStaticLds;
  if (need <= b->lds_budget / 4) return 0;
  if (need <= b->lds_budget / 2) return 1;
  if (need <= b->lds_budget) return 2;
  return 3;
}

// One persistent launch: the items of one (LDS class, block width, workgroup size).
struct Launch {
  int cls, B, nt;
  int off, count;     // items [off, off + count) of the plan
  size_t dyn;         // dynamic LDS bytes
  int grid;
  double cost;        // estimated, for the launch order
};

// Everything a run needs, prepared on the host before any device work.
struct Plan {
  std::vector<int> graphs;             // subset, in batch order
  std::vector<int> L;                  // odd L per graph of the subset (0 = automatic)
  std::vector<double> lam;             // lambda* per graph of the subset (automatic only)
  std::vector<int> spectral;           // 1: CalTau with the graph's spectrum (automatic only)
  std::vector<int> spec_version;       // the spectrum's version when spectral
  std::vector<int> block;              // B per graph of the subset
  std::vector<int> threads;            // workgroup size per graph (0: class default)
  std::vector<sc::BatchItem> items;    // grouped by launch
  std::vector<Launch> launches;        // most expensive first
  int64_t slab_elems = 0;
  int max_L = 255;
  double eps = 0.0;
};

template <typename T>
int plan_run(sc_batch* b, double eps, const int32_t* L, const sc_options& o,
             const std::vector<int>& subset, const std::vector<int>* blocks,
             const std::vector<int>* threads, Plan& P) {
  const size_t tsize = sizeof(T);
  P.graphs = subset;
  P.eps = eps;
  P.max_L = o.max_L > 0 ? o.max_L : 255;
  if (P.max_L % 2 == 0) --P.max_L;
  const size_t ng = subset.size();
  P.L.resize(ng);
  P.lam.assign(ng, 0.0);
  P.spectral.assign(ng, 0);
  P.spec_version.assign(ng, 0);
  P.block.resize(ng);
  P.threads.assign(ng, 0);
  std::vector<double> est(ng);
  for (size_t q = 0; q < ng; ++q) {
    const int gi = subset[q];
    sc_graph* g = b->graphs[gi];
    const int Lg = L ? L[gi] : 0;
    if (Lg < 0) return fail(SC_EINVAL, "L must be >= 0 for every graph");
    int nt = 0;
    const int B = blocks ? (*blocks)[q] : block_for(b, gi, o, &nt);
    if (threads) nt = (*threads)[q];
    if (!valid_block(B)) return fail(SC_EINVAL, "batch block must be 1, 2, 4, 8, 16, 32 or 64");
    if (nt != 0 && nt != 256 && nt != 512 && nt != 1024)
      return fail(SC_EINVAL, "batch workgroup size must be 256, 512 or 1024");
    P.block[q] = B;
    P.threads[q] = nt;
    if (Lg > 0) {
      P.L[q] = (Lg % 2 == 1) ? Lg : Lg + 1;
      est[q] = P.L[q];
    } else if ((o.flags & SC_TAU_SPECTRAL) && g->spec_omega >= 2) {
      // CalTau (Algorithm 1) with the graph's own spectrum; lam = |lambda_omega| for the
      // cost estimate only
      P.L[q] = 0;
      P.spectral[q] = 1;
      P.spec_version[q] = g->spec_version;
      P.lam[q] = std::fabs(g->spec_lam_h[1]);
      const double lam = std::max(1e-3, std::min(P.lam[q], 0.999999));
      const double t = std::ceil(std::log(1.0 / (eps * (1.0 - lam * lam))) / std::log(1.0 / lam));
      est[q] = std::min<double>(P.max_L, std::max(1.0, t));
    } else {
      double lam = o.lambda_star;
      if (!(lam > 0.0)) {
        const int rc = sc::graph_lambda_star(g, nullptr, &lam);
        if (rc) return rc;
      }
      if (!(lam > 0.0 && lam < 1.0)) return fail(SC_EINVAL, "lambda* must lie in (0, 1)");
      P.L[q] = 0;
      P.lam[q] = lam;
      // cost estimate only: the bound at num = 1 (no smaller than any edge's)
      const double t = std::ceil(std::log(1.0 / (eps * (1.0 - lam * lam))) / std::log(1.0 / lam));
      est[q] = std::min<double>(P.max_L, std::max(1.0, t));
    }
  }
  // items grouped by (class, B), longest first inside each group
  struct Cand {
    double cost;
    int key;          // class * 7 + log2 B
    sc::BatchItem it;
  };
  std::vector<Cand> cand;
  std::vector<double> key_cost(kLaunchMax, 0.0);
  std::vector<size_t> key_lds(kLaunchMax, 0);
  for (size_t q = 0; q < ng; ++q) {
    const int gi = subset[q];
    const sc_graph* g = b->graphs[gi];
    const int n = g->d.n, B = P.block[q];
    const int cls = class_of(b, n, B, tsize);
    // device slabs always use 256-thread workgroups
    const int nt = cls == 3 ? 256 : (P.threads[q] > 0 ? P.threads[q] : kClassThreads[cls]);
    const int key = (cls * 7 + __builtin_ctz(static_cast<unsigned>(B))) * kThreadChoices +
                    threads_index(nt);
    const double cost = est[q] * (static_cast<double>(g->d.nslots) + n) * std::sqrt(double(B));
    for (int s0 = 0; s0 < n; s0 += B) cand.push_back({cost, key, sc::BatchItem{gi, s0}});
    key_cost[key] += cost * ((n + B - 1) / B);
    if (cls == 3)   // rounded to 64 elements: every workgroup's slab stays 256-byte aligned
      P.slab_elems = std::max<int64_t>(P.slab_elems, (int64_t(state_bytes(n, B, tsize) / tsize) + 63) / 64 * 64);
    else
      key_lds[key] = std::max(key_lds[key], state_bytes(n, B, tsize));
  }
  if (cand.size() > static_cast<size_t>(INT32_MAX)) return fail(SC_EINVAL, "too many items");
  // launches in decreasing total cost; items of a launch longest first
  std::vector<int> order;
  for (int k = 0; k < kLaunchMax; ++k)
    if (key_cost[k] > 0.0) order.push_back(k);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key_cost[x] > key_cost[y]; });
  std::vector<int> rank(kLaunchMax, 0);
  for (size_t r = 0; r < order.size(); ++r) rank[order[r]] = static_cast<int>(r);
  std::stable_sort(cand.begin(), cand.end(), [&](const Cand& x, const Cand& y) {
    return x.key != y.key ? rank[x.key] < rank[y.key] : x.cost > y.cost;
  });
  P.items.resize(cand.size());
  for (size_t i = 0; i < cand.size(); ++i) P.items[i] = cand[i].it;
  int off = 0;
  for (int k : order) {
    Launch l;
    const int ti = k % kThreadChoices;
    l.nt = ti == 2 ? 1024 : ti == 1 ? 512 : 256;
    l.cls = (k / kThreadChoices) / 7;
    l.B = 1 << ((k / kThreadChoices) % 7);
    l.off = off;
    l.count = 0;
    for (size_t i = off; i < cand.size() && cand[i].key == k; ++i) ++l.count;
    off += l.count;
    l.dyn = l.cls < 3 ? key_lds[k] : 0;
    l.cost = key_cost[k];
    // grid: resident workgroups (occupancy), at most one per item
    const int nt = l.nt;
    const bool lds = l.cls < 3;
    const void* fn = sc::batch_kernel_ptr<T>(nt, lds, l.B);
    if (lds) HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(l.dyn)));
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, l.dyn));
    if (per_cu < 1) per_cu = 1;
    int64_t grid = int64_t(per_cu) * b->cus;
    if (!lds) {
      const size_t sb = static_cast<size_t>(P.slab_elems) * tsize;
      grid = std::min<int64_t>(grid, std::max<int64_t>(1, int64_t(kSlabCap / sb)));
    }
    l.grid = static_cast<int>(std::min<int64_t>(grid, l.count));
    P.launches.push_back(l);
  }
  return SC_OK;
}

// Device tables and buffers for plan P (host -> device copies, synchronous).
template <typename T>
int stage_plan(sc_batch* b, const Plan& P, double* const* outs) {
  const size_t tsize = sizeof(T);
  const int G = static_cast<int>(b->graphs.size());
  std::vector<sc::BatchGraph> tab(G);
  for (int gi = 0; gi < G; ++gi) {
    const sc_graph* g = b->graphs[gi];
    sc::BatchGraph& d = tab[gi];
    d.n = g->d.n;
    d.B = 0;
    d.ngroups = b->ngroups[gi];
    d.narrow = b->narrow[gi];
    d.rowptr = g->d.rowptr;
    d.col = g->d.col;
    d.slot_row = g->d.slot_row;
    d.tau_slot = b->tau_slot + b->slot_off[gi];
    d.tau_row = b->tau_row + b->node_off[gi];
    d.inv_f = g->d.inv_deg_f;
    d.inv_d = g->d.inv_deg_d;
    d.nb = b->nb[gi];
    d.rec = b->rec[gi];
    d.grp_invf = b->grp_invf[gi];
    d.grp_invd = b->grp_invd[gi];
    d.gacc = b->gacc + b->slot_off[gi];
    d.deg = g->d.deg;
    d.half_slot = g->d.half_slot;
    d.m = static_cast<int32_t>(g->d.m);
    d.max_L = P.max_L;
    d.eps = P.eps;
  }
  for (size_t q = 0; q < P.graphs.size(); ++q) {
    sc::BatchGraph& d = tab[P.graphs[q]];
    d.B = P.block[q];
    d.L = P.spectral[q] ? -1 : P.L[q];   // -1: tau written by CalTau before the prologue
    d.lam = P.lam[q];
    d.out = outs[q];
    d.active = 1;
  }
  HIP_TRY(hipMemcpy(b->d_graphs, tab.data(), G * sizeof(sc::BatchGraph), hipMemcpyHostToDevice));
  if (P.items.size() > b->items_cap) {
    sc::dev_free(b->d_items);
    HIP_TRY(sc::dev_alloc(&b->d_items, P.items.size()));
    b->items_cap = P.items.size();
  }
  if (!P.items.empty())
    HIP_TRY(hipMemcpy(b->d_items, P.items.data(), P.items.size() * sizeof(sc::BatchItem),
                      hipMemcpyHostToDevice));
  int slab_grid = 0;
  for (const Launch& l : P.launches)
    if (l.cls == 3) slab_grid = std::max(slab_grid, l.grid);
  if (slab_grid > 0) {
    const size_t need = static_cast<size_t>(slab_grid) * P.slab_elems * tsize;
    if (need > b->slab_bytes) {
      if (b->slabs) (void)sc::tracked_free(b->slabs);
      b->slabs = nullptr;
      b->slab_bytes = 0;
      HIP_TRY(sc::tracked_malloc(&b->slabs, need));
      b->slab_bytes = need;
    }
  }
  return SC_OK;
}

// Device work of plan P on stream st (no allocation, no host synchronisation,
// no memset: safe to capture).  outs[q]: device output of graph P.graphs[q].
// The tau range and the capped count are always computed, so a recorded graph
// serves runs with and without statistics alike.
template <typename T>
int enqueue_run(sc_batch* b, const Plan& P, hipStream_t st, hipEvent_t kb, hipEvent_t ke) {
  const int G = static_cast<int>(b->graphs.size());
  int32_t* mm = b->d_misc + kLaunchMax;
  auto* capped = reinterpret_cast<unsigned long long*>(b->d_misc + kLaunchMax + 2);
  HIP_TRY(sc::launch_fill_i32(b->d_misc, kLaunchMax, 0, st));
  HIP_TRY(sc::launch_fill_i32(mm, 1, INT32_MAX, st));
  HIP_TRY(sc::launch_fill_i32(mm + 1, 3, 0, st));   // tau max and the 64-bit capped count
  for (size_t q = 0; q < P.graphs.size(); ++q) {
    if (!P.spectral[q]) continue;
    const int gi = P.graphs[q];
    const sc_graph* g = b->graphs[gi];
    HIP_TRY(sc::launch_caltau(g->d, g->spec_lam, g->spec_phi, g->spec_omega, P.eps, P.max_L,
                              b->tau_slot + b->slot_off[gi], b->tau_row + b->node_off[gi], st,
                              capped));
  }
  HIP_TRY(sc::launch_batch_prologue(b->d_graphs, b->d_node_off, G, b->node_off[G], mm, capped,
                                    st));
  if (kb) HIP_TRY(hipEventRecord(kb, st));
  for (size_t li = 0; li < P.launches.size(); ++li) {
    const Launch& l = P.launches[li];
    HIP_TRY(sc::launch_batch<T>(l.nt, l.cls < 3, l.B, l.grid, l.dyn, b->d_graphs,
                                b->d_items + l.off, l.count, b->d_misc + li,
                                static_cast<T*>(b->slabs), P.slab_elems, st));
  }
  if (ke) HIP_TRY(hipEventRecord(ke, st));
  HIP_TRY(sc::launch_batch_combine(b->d_graphs, b->d_edge_off, G, b->edge_off[G], st));
  return SC_OK;
}

std::string run_key(const Plan& P, const sc_options& o, double* const* outs, bool host_out) {
  std::string k;
  char buf[96];
  uint64_t eb;
  std::memcpy(&eb, &P.eps, sizeof(eb));
  std::snprintf(buf, sizeof(buf), "%d|%" PRIx64 "|%d|%d|%u|%p|", o.precision, eb, P.max_L,
                host_out ? 1 : 0, o.flags, o.stream);
  k += buf;
  for (size_t q = 0; q < P.graphs.size(); ++q) {
    uint64_t lb;
    std::memcpy(&lb, &P.lam[q], sizeof(lb));
    std::snprintf(buf, sizeof(buf), "%d,%d,%d,%d,%" PRIx64 ",%d,%p;", P.graphs[q], P.L[q],
                  P.block[q], P.threads[q], lb, P.spectral[q] ? P.spec_version[q] : -1,
                  host_out ? nullptr : static_cast<void*>(outs[q]));
    k += buf;
  }
  return k;
}

template <typename T>
int run_batch(sc_batch* b, double eps, const int32_t* L, const sc_options& o,
              const std::vector<int>& subset, const std::vector<int>* blocks,
              const std::vector<int>* threads, double* const* out,
              sc_stats* st_user, float* kernel_ms) {
  hipStream_t st = static_cast<hipStream_t>(o.stream);
  const bool dev_ptrs = (o.flags & SC_DEVICE_PTRS) != 0;
  const bool replay = (o.flags & SC_GRAPH_REPLAY) != 0;
  const bool timing = (o.flags & SC_TIME_KERNELS) != 0 || kernel_ms != nullptr;
  Plan P;
  int rc = plan_run<T>(b, eps, L, o, subset, blocks, threads, P);
  if (rc) return rc;
  // device outputs per graph
  std::vector<double*> outs(P.graphs.size());
  for (size_t q = 0; q < P.graphs.size(); ++q)
    outs[q] = dev_ptrs ? out[P.graphs[q]] : b->out_dev + b->edge_off[P.graphs[q]];
  const std::string key = run_key(P, o, outs.data(), !dev_ptrs);
  const bool reuse = replay && b->exec && key == b->exec_key;
  if (!reuse) {
    b->drop_exec();
    rc = stage_plan<T>(b, P, outs.data());
    if (rc) return rc;
  }
  hipEvent_t t0 = nullptr, t1 = nullptr, kb = nullptr, ke = nullptr;
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  if (timing && !replay) {   // timing only: no system-scope fence around the kernels
    HIP_TRY(hipEventCreateWithFlags(&kb, hipEventDisableSystemFence));
    HIP_TRY(hipEventCreateWithFlags(&ke, hipEventDisableSystemFence));
  }
  struct EvGuard {
    hipEvent_t* e[4];
    ~EvGuard() {
      for (auto* p : e)
        if (*p) (void)hipEventDestroy(*p);
    }
  } guard{{&t0, &t1, &kb, &ke}};
  const bool want_range = st_user != nullptr;
  int64_t total_m = 0;
  for (int gi : P.graphs) total_m += b->graphs[gi]->d.m;
  HIP_TRY(hipEventRecord(t0, st));
  if (replay) {
    if (!reuse) {
      // record on the batch's own stream; the graph is then launched on st
      HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
      rc = enqueue_run<T>(b, P, b->cap_stream, nullptr, nullptr);
      if (!dev_ptrs && rc == SC_OK) {
        for (int gi : P.graphs) {
          const hipError_t e = hipMemcpyAsync(
              b->out_pinned + b->edge_off[gi], b->out_dev + b->edge_off[gi],
              b->graphs[gi]->d.m * sizeof(double), hipMemcpyDeviceToHost, b->cap_stream);
          if (e != hipSuccess) {
            rc = fail(SC_EHIP, std::string("capture copy: ") + hipGetErrorString(e));
            break;
          }
        }
      }
      hipGraph_t gr = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->cap_stream, &gr);
      if (rc) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
      }
      if (ec != hipSuccess) return fail(SC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
      b->hgraph = gr;
      const hipError_t ei = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        b->drop_exec();
        return fail(SC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
      }
      b->exec_key = key;
    }
    HIP_TRY(hipGraphLaunch(b->exec, st));
  } else {
    rc = enqueue_run<T>(b, P, st, kb, ke);
    if (rc) return rc;
    if (!dev_ptrs)
      for (int gi : P.graphs)
        HIP_TRY(hipMemcpyAsync(b->out_pinned + b->edge_off[gi], b->out_dev + b->edge_off[gi],
                               b->graphs[gi]->d.m * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (want_range)
    HIP_TRY(hipMemcpyAsync(b->h_misc, b->d_misc + kLaunchMax, 4 * sizeof(int32_t),
                           hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(t1, st));
  if (!dev_ptrs || want_range || timing) HIP_TRY(hipEventSynchronize(t1));
  if (!dev_ptrs)
    for (int gi : P.graphs)
      std::memcpy(out[gi], b->out_pinned + b->edge_off[gi], b->graphs[gi]->d.m * sizeof(double));
  float kms = 0.0f;
  if (kb && ke) HIP_TRY(hipEventElapsedTime(&kms, kb, ke));
  if (kernel_ms) *kernel_ms = kms;
  if (st_user) {
    sc_stats s{};
    s.L_used = b->h_misc[1];
    s.L_min = b->h_misc[0];
    unsigned long long capped_h = 0;
    std::memcpy(&capped_h, b->h_misc + 2, sizeof(capped_h));
    s.L_capped = static_cast<int64_t>(capped_h / 2);   // both halves of an edge share tau
    s.tilde_tau = -1;
    s.tilde_min = -1;
    s.tilde_max = -1;
    s.lambda_converged = -1;
    int B0 = P.block.empty() ? 0 : P.block[0];
    for (int B : P.block)
      if (B != B0) B0 = -1;
    s.block = B0;
    for (double l : P.lam) s.lambda_star = std::max(s.lambda_star, l);
    s.prop_launches = static_cast<int64_t>(P.launches.size());
    s.prop_timed = kb && ke ? s.prop_launches : 0;
    s.prop_ms = kms;
    float tms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&tms, t0, t1));
    s.total_ms = tms;
    *st_user = s;
  }
  (void)total_m;
  return SC_OK;
}

int run_dispatch(sc_batch* b, double eps, const int32_t* L, const sc_options& o,
                 const std::vector<int>& subset, const std::vector<int>* blocks,
                 const std::vector<int>* threads,
                 double* const* out, sc_stats* st, float* kernel_ms) {
  if (!(eps > 0.0 && eps < 1.0)) return fail(SC_EINVAL, "eps must lie in (0, 1)");
  if (o.method != SC_TGT) return fail(SC_ENOTIMPL, "batches run TGT (method 0) only");
  if (o.precision != 0 && o.precision != 1) return fail(SC_EINVAL, "precision must be 0 or 1");
  if (o.block != 0 && !valid_block(o.block))
    return fail(SC_EINVAL, "batch block must be 0 or 1, 2, 4, 8, 16, 32, 64");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b->device) return fail(SC_EINVAL, "current device differs from the batch's device");
  return o.precision == 1
             ? run_batch<double>(b, eps, L, o, subset, blocks, threads, out, st, kernel_ms)
             : run_batch<float>(b, eps, L, o, subset, blocks, threads, out, st, kernel_ms);
}

}  // namespace

extern "C" int sc_build_batch(int G, const int64_t* n, const int64_t* m,
                              const int64_t* const* u_host, const int64_t* const* v_host,
                              unsigned flags, sc_batch** out) {
  if (!out) return fail(SC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (G < 1 || !n || !m || !u_host || !v_host) return fail(SC_EINVAL, "bad batch arguments");
  if (flags & (SC_DEGREE_ORDER | SC_BFS_ORDER))
    return fail(SC_EINVAL, "SC_DEGREE_ORDER and SC_BFS_ORDER apply to sc_build_graph only");
  sc_batch* b = new (std::nothrow) sc_batch();
  if (!b) return fail(SC_ENOMEM, "host allocation failed");
  auto bail = [&](int rc) {
    b->release();
    delete b;
    return rc;
  };
  (void)hipGetDevice(&b->device);
  b->node_off.assign(G + 1, 0);
  b->slot_off.assign(G + 1, 0);
  b->edge_off.assign(G + 1, 0);
  b->nb.assign(G, nullptr);
  b->rec.assign(G, nullptr);
  b->grp_invf.assign(G, nullptr);
  b->grp_invd.assign(G, nullptr);
  b->ngroups.assign(G, 0);
  b->narrow.assign(G, 0);
  b->dmin.assign(G, 0);
  b->graphs.assign(G, nullptr);
  for (int gi = 0; gi < G; ++gi) {
    sc::HostCSR h;
    int rc = sc::build_host_csr(n[gi], m[gi], u_host[gi], v_host[gi], flags, h);
    if (rc) {
      fail(rc, "graph " + std::to_string(gi) + ": " + sc_last_error());
      return bail(rc);
    }
    std::vector<uint32_t> nbh, rech;
    std::vector<float> invf;
    std::vector<double> invd;
    rc = build_slices(h, rech, nbh, invf, invd, &b->narrow[gi]);
    if (rc) return bail(rc);
    b->ngroups[gi] = (h.n + 63) / 64;
    b->dmin[gi] = *std::min_element(h.deg.begin(), h.deg.end());
    hipError_t e = sc::dev_alloc(&b->nb[gi], nbh.size());
    if (e == hipSuccess) e = hipMemcpy(b->nb[gi], nbh.data(), nbh.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sc::dev_alloc(&b->rec[gi], rech.size());
    if (e == hipSuccess) e = hipMemcpy(b->rec[gi], rech.data(), rech.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sc::dev_alloc(&b->grp_invf[gi], invf.size());
    if (e == hipSuccess)
      e = hipMemcpy(b->grp_invf[gi], invf.data(), invf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = sc::dev_alloc(&b->grp_invd[gi], invd.size());
    if (e == hipSuccess)
      e = hipMemcpy(b->grp_invd[gi], invd.data(), invd.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess)
      return bail(fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP,
                       std::string("batch upload: ") + hipGetErrorString(e)));
    b->node_off[gi + 1] = b->node_off[gi] + h.n;
    b->slot_off[gi + 1] = b->slot_off[gi] + h.nslots;
    b->edge_off[gi + 1] = b->edge_off[gi] + h.m;
    rc = sc::graph_from_csr(h, &b->graphs[gi]);
    if (rc) return bail(rc);
  }
  hipError_t e = sc::dev_alloc(&b->tau_slot, b->slot_off[G]);
  if (e == hipSuccess) e = sc::dev_alloc(&b->tau_row, b->node_off[G]);
  if (e == hipSuccess) e = sc::dev_alloc(&b->gacc, b->slot_off[G]);
  if (e == hipSuccess) e = sc::dev_alloc(&b->out_dev, b->edge_off[G]);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->out_pinned),
                                         std::max<int64_t>(1, b->edge_off[G]) * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_misc), 4 * sizeof(int32_t));
  if (e == hipSuccess) e = sc::dev_alloc(&b->d_graphs, G);
  if (e == hipSuccess) e = sc::dev_alloc(&b->d_node_off, G + 1);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_node_off, b->node_off.data(), (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sc::dev_alloc(&b->d_edge_off, G + 1);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_edge_off, b->edge_off.data(), (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sc::dev_alloc(&b->d_misc, kLaunchMax + 4);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  int lds = 0, cus = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess)
    return bail(fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP,
                     std::string("batch buffers: ") + hipGetErrorString(e)));
  b->lds_budget = static_cast<size_t>(lds);
  b->cus = std::max(1, cus);
  *out = b;
  return SC_OK;
}

extern "C" int sc_batch_size(const sc_batch* b, int* G) {
  if (!b || !G) return fail(SC_EINVAL, "NULL argument");
  *G = static_cast<int>(b->graphs.size());
  return SC_OK;
}

extern "C" int sc_batch_graph(sc_batch* b, int i, sc_graph** g) {
  if (!b || !g) return fail(SC_EINVAL, "NULL argument");
  if (i < 0 || i >= static_cast<int>(b->graphs.size())) return fail(SC_EINVAL, "graph index out of range");
  *g = b->graphs[i];
  return SC_OK;
}

extern "C" void sc_free_batch(sc_batch* b) {
  if (!b) return;
  b->release();
  delete b;
}

extern "C" int sc_batch_blocks(const sc_batch* b, const sc_options* o, int32_t* blocks) {
  if (!b || !o || !blocks) return fail(SC_EINVAL, "NULL argument");
  if (o->block != 0 && !valid_block(o->block))
    return fail(SC_EINVAL, "batch block must be 0 or 1, 2, 4, 8, 16, 32, 64");
  for (size_t gi = 0; gi < b->graphs.size(); ++gi) blocks[gi] = block_for(b, static_cast<int>(gi), *o);
  return SC_OK;
}

extern "C" int sc_batch_all_edges(sc_batch* b, double eps, const int32_t* L,
                                  const sc_options* o, double* const* out, sc_stats* st) {
  if (!b || !o || !out) return fail(SC_EINVAL, "NULL argument");
  for (size_t gi = 0; gi < b->graphs.size(); ++gi)
    if (!out[gi]) return fail(SC_EINVAL, "NULL output pointer");
  std::vector<int> all(b->graphs.size());
  std::iota(all.begin(), all.end(), 0);
  return run_dispatch(b, eps, L, *o, all, nullptr, nullptr, out, st, nullptr);
}

// ---------------------------------------------------------------------- autotuner

extern "C" int sc_batch_autotune(sc_batch* b, double eps, const int32_t* L, const sc_options* o,
                                 const char* json_path) {
  if (!b || !o) return fail(SC_EINVAL, "NULL argument");
  if (o->method != SC_TGT) return fail(SC_ENOTIMPL, "batches run TGT (method 0) only");
  if (o->flags & SC_TAU_SPECTRAL)
    return fail(SC_ENOTIMPL, "batches use the lambda*-bound (SC_TAU_SPECTRAL not supported)");
  const size_t tsize = o->precision == 1 ? sizeof(double) : sizeof(float);
  // buckets present, each with its graphs (largest first)
  struct Bucket {
    int ln, ld;
    std::vector<int> graphs;
  };
  std::vector<Bucket> buckets;
  for (size_t gi = 0; gi < b->graphs.size(); ++gi) {
    int ln, ld;
    bucket_of(b, static_cast<int>(gi), &ln, &ld);
    auto it = std::find_if(buckets.begin(), buckets.end(),
                           [&](const Bucket& k) { return k.ln == ln && k.ld == ld; });
    if (it == buckets.end()) {
      buckets.push_back({ln, ld, {}});
      it = buckets.end() - 1;
    }
    it->graphs.push_back(static_cast<int>(gi));
  }
  sc_options so = *o;
  so.flags &= ~(SC_GRAPH_REPLAY | SC_TIME_KERNELS);
  so.flags |= SC_DEVICE_PTRS;
  std::vector<TuneEntry> found;
  std::string json = "{\n  \"format\": \"sc-batch-tuning-1\",\n  \"entries\": [\n";
  for (size_t bi = 0; bi < buckets.size(); ++bi) {
    Bucket& k = buckets[bi];
    std::stable_sort(k.graphs.begin(), k.graphs.end(),
                     [&](int x, int y) { return b->graphs[x]->d.n > b->graphs[y]->d.n; });
    if (k.graphs.size() > 8) k.graphs.resize(8);
    std::vector<double*> outs(b->graphs.size(), nullptr);
    for (int gi : k.graphs) outs[gi] = b->out_dev + b->edge_off[gi];
    int nmax = 0;
    for (int gi : k.graphs) nmax = std::max(nmax, b->graphs[gi]->d.n);
    int best = -1, best_nt = 0;
    float best_ms = 0.0f;
    std::string trials;
    auto trial = [&](int B, int nt, float* ms) -> int {
      std::vector<int> blocks(k.graphs.size(), B), threads(k.graphs.size(), nt);
      int rc = run_dispatch(b, eps, L, so, k.graphs, &blocks, &threads, outs.data(), nullptr, ms);
      if (rc) return rc;   // the first run warms up (lambda*, attributes, caches)
      rc = run_dispatch(b, eps, L, so, k.graphs, &blocks, &threads, outs.data(), nullptr, ms);
      if (rc) return rc;
      char buf[64];
      std::snprintf(buf, sizeof(buf), "%s{\"block\": %d, \"threads\": %d, \"ms\": %.4f}",
                    trials.empty() ? "" : ", ", B, nt, *ms);
      trials += buf;
      return SC_OK;
    };
    // block width with the LDS class's workgroup size
    for (int B = 1; B <= 64; B <<= 1) {
      const bool fits = state_bytes(nmax, B, tsize) + kStaticLds <= b->lds_budget;
      if (!fits && B > 8) continue;   // device-slab states: narrow blocks only
      float ms = 0.0f;
      const int rc = trial(B, 0, &ms);
      if (rc) return rc;
      if (best < 0 || ms < best_ms) {
        best = B;
        best_ms = ms;
      }
    }
    // then the workgroup size for that width (states in LDS only)
    if (state_bytes(nmax, best, tsize) + kStaticLds <= b->lds_budget) {
      for (int nt : {256, 512, 1024}) {
        float ms = 0.0f;
        const int rc = trial(best, nt, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
          best_nt = nt;
          best_ms = ms;
        }
      }
    }
    found.push_back({k.ln, k.ld, o->precision, best, best_nt});
    char head[192];
    std::snprintf(head, sizeof(head),
                  "    {\"lg_n\": %d, \"lg_d\": %d, \"precision\": %d, \"block\": %d, \"threads\": %d, "
                  "\"graphs\": %zu, \"trials\": [",
                  k.ln, k.ld, o->precision, best, best_nt, k.graphs.size());
    json += head + trials + "]}" + (bi + 1 < buckets.size() ? ",\n" : "\n");
  }
  json += "  ]\n}\n";
  // replace entries of this precision
  b->tune.erase(std::remove_if(b->tune.begin(), b->tune.end(),
                               [&](const TuneEntry& e) { return e.precision == o->precision; }),
                b->tune.end());
  b->tune.insert(b->tune.end(), found.begin(), found.end());
  b->drop_exec();
  if (json_path && *json_path) {
    FILE* f = std::fopen(json_path, "w");
    if (!f) return fail(SC_EINVAL, std::string("cannot write ") + json_path);
    std::fputs(json.c_str(), f);
    std::fclose(f);
  }
  return SC_OK;
}

extern "C" int sc_batch_load_tuning(sc_batch* b, const char* json_path) {
  if (!b || !json_path) return fail(SC_EINVAL, "NULL argument");
  FILE* f = std::fopen(json_path, "r");
  if (!f) return fail(SC_EINVAL, std::string("cannot read ") + json_path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  if (text.find("\"sc-batch-tuning-1\"") == std::string::npos)
    return fail(SC_EINVAL, "not a batch tuning file");
  std::vector<TuneEntry> found;
  size_t pos = 0;
  while ((pos = text.find("{\"lg_n\":", pos)) != std::string::npos) {
    TuneEntry e{};
    if (std::sscanf(text.c_str() + pos, "{\"lg_n\": %d, \"lg_d\": %d, \"precision\": %d, \"block\": %d",
                    &e.lg_n, &e.lg_d, &e.precision, &e.block) != 4 ||
        !valid_block(e.block) || (e.precision != 0 && e.precision != 1))
      return fail(SC_EINVAL, "malformed tuning entry");
    // optional workgroup size (0 = the LDS class's default)
    const size_t end = text.find('}', pos);
    const size_t th = text.find("\"threads\":", pos);
    if (th != std::string::npos && th < end &&
        (std::sscanf(text.c_str() + th, "\"threads\": %d", &e.threads) != 1 ||
         (e.threads != 0 && e.threads != 256 && e.threads != 512 && e.threads != 1024)))
      return fail(SC_EINVAL, "malformed tuning entry");
    found.push_back(e);
    ++pos;
  }
  b->tune = found;
  b->drop_exec();
  return SC_OK;
}
