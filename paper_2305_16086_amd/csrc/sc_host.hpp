// Host-side pieces shared by the translation units of libsc: error reporting,
// the graph handle, work buffers and the per-block traversal driver.
#pragma once

#include "sc_internal.hpp"

#include <string>
#include <vector>

namespace sc {

// Records the message for sc_last_error() and returns code.
int fail(int code, const std::string& msg);

// Every device allocation of the library goes through these two calls, which
// keep the live byte count.  When the environment variable
// SC_DEVICE_BYTES_LIMIT holds a positive number, an allocation that would
// take the live bytes above it fails with hipErrorOutOfMemory (a device-memory
// budget; also how the out-of-memory paths are tested).
hipError_t tracked_malloc_bytes(void** p, size_t bytes);
hipError_t tracked_free(void* p);
size_t tracked_live_bytes();

template <typename P>
hipError_t tracked_malloc(P** p, size_t bytes) {
  void* q = nullptr;
  const hipError_t e = tracked_malloc_bytes(&q, bytes);
  *p = static_cast<P*>(q);
  return e;
}

template <typename P>
hipError_t dev_alloc(P** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return tracked_malloc(p, count * sizeof(P));
}

template <typename P>
void dev_free(P*& p) {
  if (p) (void)tracked_free(p);
  p = nullptr;
}

// The per-graph block pipeline synchronises its two streams once per group of
// blocks; groups cycle through kPipeGroups sets of Y pairs, so the traversal of
// group q reuses the pairs of group q - kPipeGroups once that group's tails are
// done.  A group holds up to kMaxGroupBlocks blocks (fewer when the Y pairs of
// the larger pipeline would not fit kPipeBudgetBytes).
constexpr int kPipeGroups = 3;
constexpr int kMaxGroupBlocks = 4;
constexpr int kMaxPipe = kPipeGroups * kMaxGroupBlocks;   // Y pairs at most
constexpr size_t kPipeBudgetBytes = size_t(2) << 30;

// runs f when the scope ends (releases buffers on every return path)
template <typename F>
struct ScopeExit {
  F& f;
  ~ScopeExit() { f(); }
};

}  // namespace sc

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      return ::sc::fail(e_ == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP,           \
                        std::string(#expr) + ": " + hipGetErrorString(e_));        \
    }                                                                              \
  } while (0)

struct sc_graph {
  sc::DeviceGraph d;
  int device = 0;
  std::vector<int32_t> rowptr_h;
  std::vector<int32_t> deg_h;
  // SC_DEGREE_ORDER: the caller's node x is stored as rank_h[x]; stored node y is
  // the caller's label_h[y] (both empty when the graph keeps the caller's ids)
  std::vector<int32_t> rank_h;
  std::vector<int32_t> label_h;
  int32_t* rank_d = nullptr;            // device copy of rank_h
  double lambda_star = -1.0;
  int lambda_converged = -1;            // of the cached lambda* (see sc_stats)
  // spectrum for CalTau (Algorithm 1): spec_omega eigenpairs of D^-1/2 A D^-1/2,
  // |lambda| descending after the trivial pair; phi node-major [n][spec_omega]
  int spec_omega = 0;
  int spec_version = 0;                 // bumped on every change (keys the cached plan)
  double* spec_lam = nullptr;           // device [spec_omega]
  double* spec_phi = nullptr;           // device [n * spec_omega]
  std::vector<double> spec_lam_h;

  // work buffers, grown on demand
  void* Y[2 * sc::kMaxPipe] = {};          // one ping-pong pair per block in flight
  size_t ybytes = 0;
  int ypairs = 0;                          // pairs allocated (kPipeGroups x group size)
  hipStream_t tail_stream = nullptr;   // per-block tails overlap the next traversal
  // [0] stream joins, [1 + q] traversal of the group in set q done,
  // [1 + kPipeGroups + q] its tails done
  hipEvent_t pipe_ev[1 + 2 * sc::kPipeGroups] = {};
  void* partials = nullptr;
  size_t pbytes = 0;
  unsigned long long* mask = nullptr;   // 2 x n words (two alternating buffers)
  uint8_t* nz = nullptr;                // [n] nonzero rows of the two-hop state (1: unknown)
  unsigned* anymask = nullptr;          // 2 x ceil(n/32) words, one bit per node
  int mask_pending_s0 = -1;             // block whose bits are still set
  int mask_pending_buf = 0;
  int mask_pending_B = 0;
  double* gacc = nullptr;
  int32_t* tau_slot = nullptr;
  int32_t* tau_row = nullptr;
  int64_t* nr_slot = nullptr;
  sc::ColStats* cs = nullptr;
  void* colscratch = nullptr;  // sc::kColScratchBytes
  unsigned long long* work = nullptr;
  unsigned long long* plan_work = nullptr;   // [2 x 64] walk totals per candidate switch step
  sc::WalkScratch walk;                      // flattened walks (chunk offsets, chunk sums)
  // cached switch-step plan (the cost model depends only on these inputs)
  struct PlanKey {
    double eps;
    int L, max_L;
    double lam;
    int B, tsize, gamma;
    double delta;
    int tau_policy;   // 0: lambda*-bound, else the spectrum version used by CalTau
    bool operator==(const PlanKey& o) const {
      return eps == o.eps && L == o.L && max_L == o.max_L && lam == o.lam && B == o.B &&
             tsize == o.tsize && gamma == o.gamma && delta == o.delta &&
             tau_policy == o.tau_policy;
    }
  };
  PlanKey plan_key{};
  int plan_tilde = -1;
  bool plan_valid = false;
  // per-source TGT+ (SC_PER_SOURCE): workgroup-slot columns and the wave buffers
  struct SourceBuffers {
    uint64_t* Q = nullptr;          // [2 * slots * n] 64-bit fixed-point columns
    int32_t* S = nullptr;           // [2 * slots * n] support lists
    size_t qcap = 0;
    bool clean = false;             // Q is all zero (every call that finished leaves it so)
    int32_t* slot_ctl = nullptr;
    size_t ctl_cap = 0;
    int32_t* tilde_row = nullptr;
    size_t tilde_cap = 0;
    int32_t* pos_slot = nullptr;
    size_t pos_cap = 0;
    int32_t* pos_w = nullptr;
    size_t posw_cap = 0;
    int64_t* nr_pos = nullptr;
    size_t nrp_cap = 0;
    int64_t* chunk_off = nullptr;
    size_t co_cap = 0;
    double* part = nullptr;
    size_t part_cap = 0;
    int64_t* ctl = nullptr;
    size_t ctl2_cap = 0;
    unsigned long long* totals = nullptr;
    size_t tot_cap = 0;
    int32_t* list = nullptr;
    size_t list_cap = 0;
    int64_t* hoff = nullptr;
    size_t hoff_cap = 0;
    std::vector<int64_t> nbr_vol_h;   // per node: sum of its neighbours' degrees (wave order)
  } src;
  double* out_dev = nullptr;
  int32_t* tau_out_dev = nullptr;
  int64_t* nr_out_dev = nullptr;
  // learned closure buffers
  void* rdiag = nullptr;
  void* roff = nullptr;
  size_t rbytes = 0;
  float* feat = nullptr;       // [m][16]
  float* zpred = nullptr;      // [m]
  double* cl_s0 = nullptr;     // [m] x 4: s0, uK, lo, hi
  unsigned char* fb = nullptr; // [m]
  int* block_flag = nullptr;   // [nblocks of width 16]
  std::vector<hipEvent_t> events;

  void release();
};

namespace sc {

// CSR and task lists of one graph, built and validated on the host.
struct HostCSR {
  int32_t n = 0;
  int64_t m = 0, nslots = 0;
  std::vector<int32_t> rowptr, col, deg, slot_row, slot_half, half_slot;
  std::vector<Task> tasks, ptasks, wg_tasks;
  std::vector<HeavyRow> giant;
  int32_t nparts = 0;
  std::vector<float> inv_f;
  std::vector<double> inv_d;
};

int build_host_csr(int64_t n, int64_t m, const int64_t* u, const int64_t* v, unsigned flags,
                   HostCSR& out);
int upload_csr(const HostCSR& h, DeviceGraph& d);
// New handle owning an upload of h (h.rowptr and h.deg are moved into it).
int graph_from_csr(HostCSR& h, sc_graph** out);
// One Lanczos run from start vector number `seed`; *converged = 1 when the
// extreme Ritz pairs passed the residual test (or the Krylov space closed).
// TGT+ with the frontier-sparse traversal and the per-source switch step of
// Eq. 14 (SC_PER_SOURCE).
int run_per_source(sc_graph* g, double eps, int L, const sc_options& o, double* out,
                   sc_stats* st);

int lanczos_lambda_star(const DeviceGraph& d, const int32_t* deg_host, hipStream_t st, double* out,
                        int* converged = nullptr, uint64_t seed = 0);
// Lanczos for the omega eigenpairs of largest |lambda| (stores the converged prefix in g)
int lanczos_spectrum(sc_graph* g, int omega, int max_iter, double tol, hipStream_t st, int* kept,
                     double* worst);

int ensure_buffers(sc_graph* g, int B, size_t tsize);
int ensure_pipeline(sc_graph* g);
int ensure_closure_buffers(sc_graph* g, size_t tsize);
int compute_lambda_star(sc_graph* g, hipStream_t st, double* out);
int graph_lambda_star(sc_graph* g, hipStream_t st, double* out);

template <typename T>
__global__ void k_init_low(int n, int s0, int B, int ell, const int32_t* __restrict__ rowptr,
                           const int32_t* __restrict__ col, const T* __restrict__ inv_deg,
                           T* __restrict__ Y) {
  const int c = blockIdx.x;
  const int s = s0 + c;
  if (s >= n) return;
  if (ell == 0) {
    if (threadIdx.x == 0) Y[static_cast<size_t>(s) * B + c] = T(1);
    return;
  }
  for (int k = rowptr[s] + threadIdx.x; k < rowptr[s + 1]; k += blockDim.x) {
    const int x = col[k];
    Y[static_cast<size_t>(x) * B + c] = inv_deg[x];   // p_1(x, s) = 1/d_x for x in N(s)
  }
}

template <typename T>
inline const T* inv_deg_host_sel(const DeviceGraph& g);
template <>
inline const float* inv_deg_host_sel<float>(const DeviceGraph& g) { return g.inv_deg_f; }
template <>
inline const double* inv_deg_host_sel<double>(const DeviceGraph& g) { return g.inv_deg_d; }

// Drives the launches of one source block [s0, s0+B).
template <typename T>
struct Runner {
  sc_graph* g;
  int B;
  hipStream_t st;
  bool timing;
  sc_stats stats{};
  size_t ev_used = 0;
  int cur = 0;            // index of the Y buffer holding the latest step
  int po = 0;             // first buffer of the Y pair in use (2 * pair)
  T* rdiag = nullptr;     // optional per-slot recordings of p_l(s,s), p_l(j,s)
  T* roff = nullptr;
  int record_to = -1;     // record steps 2..record_to

  T* Yb(int i) { return static_cast<T*>(g->Y[po + i]); }
  T* parts() { return static_cast<T*>(g->partials); }

  // odd: the sampled launches cycle through the dense steps of a block
  static constexpr int64_t kTimeEvery = 15;

  // timing-only events: no system-scope fence (a fence writes back and
  // invalidates the caches)
  int event_pair(hipEvent_t* a, hipEvent_t* b) {
    while (g->events.size() < ev_used + 2) {
      hipEvent_t e;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      g->events.push_back(e);
    }
    *a = g->events[ev_used];
    *b = g->events[ev_used + 1];
    ev_used += 2;
    return SC_OK;
  }

  // algorithmic bytes of one dense propagation launch: the state read once and
  // written once, the CSR column array, the task list and the degree vector
  double step_bytes() const {
    const double n = g->d.n, S = static_cast<double>(g->rowptr_h[g->d.n]);
    return 2.0 * n * B * sizeof(T) + 4.0 * S + 16.0 * (g->d.ntasks + g->d.nwg) + sizeof(T) * n;
  }

  AccJob pending_acc;     // accumulation of the latest step, not yet launched

  // recordings of step ell next to an accumulation (without one, the
  // recording is the pending job itself and rides on the next launch)
  int record_step(int s0, int kbeg, int kend, int ell, bool acc) {
    if (acc && rdiag && ell <= record_to)
      HIP_TRY(launch_record<T>(g->d, kbeg, kend, s0, B, ell, Yb(cur), rdiag, roff, st));
    return SC_OK;
  }

  // launches the pending accumulation on its own
  int flush_acc() {
    if (acc_job_set(pending_acc))
      HIP_TRY(launch_accumulate<T>(g->d, B, Yb(cur), pending_acc, st));
    pending_acc = AccJob{};
    return SC_OK;
  }

  // clears the neighbour bits a traversal left set
  int flush_masks() {
    if (g->mask_pending_s0 >= 0) {
      HIP_TRY(launch_mask_update(g->d, -1, g->mask_pending_s0, g->mask_pending_B,
                                 1 - g->mask_pending_buf, g->mask, g->anymask, st));
      g->mask_pending_s0 = -1;
    }
    return SC_OK;
  }

  // traverse the block from l = 2 up to l = lend (l = 0, 1 are closed form);
  // the accumulation of step l rides on the launch of step l + 1, the last one
  // stays pending (flush_acc or a fused consumer launches it).  With next_s0 >= 0
  // the first dense step also sets the masks of block next_s0 and clears this
  // block's (the two-hop step, the only reader, is done by then).
  int traverse(int s0, int kbeg, int kend, int lend, bool acc, double* gacc, int next_s0 = -1) {
    pending_acc = AccJob{};
    if (lend < 2) return SC_OK;
    int buf;
    if (g->mask_pending_s0 == s0 && g->mask_pending_B == B) {
      buf = g->mask_pending_buf;   // a buffer only ever holds one block's bits: these are s0's
    } else {
      buf = g->mask_pending_s0 >= 0 ? 1 - g->mask_pending_buf : 0;
      if (g->mask_pending_s0 >= 0 && g->mask_pending_B != B) {
        int rc0 = flush_masks();
        if (rc0) return rc0;
      }
      HIP_TRY(launch_mask_update(g->d, s0, g->mask_pending_s0, B, buf, g->mask, g->anymask, st));
      g->mask_pending_s0 = s0;
      g->mask_pending_buf = buf;
      g->mask_pending_B = B;
    }
    unsigned long long* mk = g->mask + static_cast<size_t>(buf) * g->d.n;
    unsigned* am = g->anymask + static_cast<size_t>(buf) * ((g->d.n + 31) / 32);
    cur = 0;
    HIP_TRY(launch_twohop<T>(g->d, B, mk, am, Yb(cur), parts(), g->nz, st));
    auto job = [&](int ell) {
      AccJob j;
      if (acc) {
        j.kbeg = kbeg;
        j.kend = kend;
        j.s0 = s0;
        j.ell = ell;
        j.tau = g->tau_slot;
        j.gacc = gacc;
      } else if (rdiag && ell <= record_to) {
        j.kbeg = kbeg;
        j.kend = kend;
        j.s0 = s0;
        j.ell = ell;
        j.rdiag = rdiag;
        j.roff = roff;
      }
      return j;
    };
    pending_acc = job(2);
    int rc = record_step(s0, kbeg, kend, 2, acc);
    if (rc) return rc;
    for (int ell = 3; ell <= lend; ++ell) {
      hipEvent_t a = nullptr, b = nullptr;
      // the first dense step skips the rows the two-hop step left at zero (B = 64);
      // the later ones gather every neighbour row and are the launches the stats
      // count.  Every kTimeEvery-th of those is timed by events that take the
      // row-gather kernel's own start and end (the kernel the roofline is taken
      // on); the others run without events.
      const bool skip = ell == 3 && B == 64;
      const bool timed = timing && !skip && stats.prop_launches % kTimeEvery == 0;
      if (timed) {
        rc = event_pair(&a, &b);
        if (rc) return rc;
      }
      MaskJob mj;
      const bool carry = ell == 3 && next_s0 >= 0;
      if (carry) mj = mask_job(g->d, next_s0, s0, B, 1 - buf, g->mask, g->anymask);
      // a and b (when timed) take the kernel's own start and end times
      HIP_TRY(launch_propagate_rows<T>(g->d, B, Yb(cur), Yb(1 - cur), parts(), pending_acc, st,
                                       skip ? g->nz : nullptr, a, b, carry ? &mj : nullptr));
      if (carry) {
        g->mask_pending_s0 = next_s0;
        g->mask_pending_buf = 1 - buf;
      }
      HIP_TRY(launch_fixup<T>(g->d, B, parts(), Yb(1 - cur), st));
      if (!skip) {
        ++stats.prop_launches;
        stats.prop_bytes += step_bytes();
      }
      cur = 1 - cur;
      pending_acc = job(ell);
      rc = record_step(s0, kbeg, kend, ell, acc);
      if (rc) return rc;
    }
    return SC_OK;
  }

  // one more dense step without accumulation (switch-step planning)
  int advance() {
    HIP_TRY(launch_propagate<T>(g->d, B, Yb(cur), Yb(1 - cur), parts(), AccJob{}, st));
    cur = 1 - cur;
    return SC_OK;
  }

  // state at l = 0 (indicators) or l = 1 (one hop) when the walk tail starts that early
  int init_low(int s0, int ell) {
    HIP_TRY(hipMemsetAsync(Yb(0), 0, g->ybytes, st));
    cur = 0;
    k_init_low<T><<<B, 64, 0, st>>>(g->d.n, s0, B, ell, g->d.rowptr, g->d.col,
                                    inv_deg_host_sel<T>(g->d), Yb(0));
    HIP_TRY(hipGetLastError());
    return SC_OK;
  }

  // a block's source range, slot range and largest truncation
  void block_range(int b, const std::vector<int32_t>& tau_row, int* s0, int* kbeg, int* kend,
                   int* tmax) const {
    const int64_t n = g->d.n;
    *s0 = b * B;
    const int s1 = static_cast<int>(std::min<int64_t>(n, static_cast<int64_t>(*s0) + B));
    *kbeg = g->rowptr_h[*s0];
    *kend = g->rowptr_h[s1];
    int t = 0;
    for (int x = *s0; x < s1; ++x) t = std::max(t, tau_row[x]);
    *tmax = t;
  }
};

// learned closure run (method SC_LEARNED)
int run_learned(sc_graph* g, double eps, const sc_options& o, double* out_user, sc_stats* st);

}  // namespace sc
