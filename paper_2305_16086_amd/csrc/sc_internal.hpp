// Internal declarations shared by the host orchestration and the kernel
// translation units of libsc.  Not part of the public ABI (see include/sc.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sc.h"

namespace sc {

// Row tasks of the gather kernels: a row with at most kChunk slots is one
// wave's task, a row with up to kGiant slots one workgroup's task, and a
// giant row is cut into workgroup chunks of kGiantChunk slots whose partial
// sums a fix-up pass adds in chunk order (deterministic, no atomics).
constexpr int kChunk = 256;
constexpr int kGiant = 4096;
constexpr int kGiantChunk = 1024;
constexpr int kWavesPerBlock = 4;     // 256-thread workgroups
constexpr int kMaxGamma = 16;         // candidate lists kept in registers

struct Task {
  int32_t row;
  int32_t beg;      // first CSR slot
  int32_t end;      // one past the last CSR slot
  int32_t part;     // -1: whole row; else index of this chunk's partial-sum row
};

struct HeavyRow {
  int32_t row;
  int32_t part0;    // first partial row
  int32_t nparts;   // number of chunks
  int32_t pad;
};

// Per-column summary of q = p_tilde(., s_c) used by Algorithm 3 / Lemma 4.3.
struct ColStats {
  double maxV, minV;     // max / min over all nodes
  double rho;            // upper bound on rho_i (Eq. 16), safe reading of Alg. 3
  double maxN, minN;     // max / min over N(s_c)
};

// Per-edge accumulation job of one source block: slots [kbeg, kend) of the
// block starting at s0 gain the step-ell term (gacc == nullptr: no job).  With
// rdiag set instead, the job records p_ell(s,s) and p_ell(j,s) of every slot
// into rdiag / roff (T[slots][L0 + 1], the learned closure's recordings).
struct AccJob {
  int kbeg = 0, kend = 0, s0 = 0, ell = 0;
  const int32_t* tau = nullptr;
  double* gacc = nullptr;
  void* rdiag = nullptr;
  void* roff = nullptr;
};
inline bool acc_job_set(const AccJob& a) { return (a.gacc || a.rdiag) && a.kend > a.kbeg; }

// Neighbour-bit update of the two-hop masks: set the bits of block s_set in
// buffer buf, clear those of block s_clear in buffer 1 - buf (s_* < 0: none).
struct MaskJob {
  int s_set = -1, s_clear = -1, B = 0, buf = 0;
  int64_t mwords = 0, awords = 0;
  unsigned long long* mask = nullptr;
  unsigned* anymask = nullptr;
};

struct DeviceGraph {
  int32_t n = 0;
  int64_t m = 0;                 // input edges (halves 0..2m-1)
  int64_t nslots = 0;            // CSR slots (2 x distinct edges)
  int32_t* rowptr = nullptr;     // [n+1]
  int32_t* col = nullptr;        // [2m] neighbours, ascending per row
  int32_t* deg = nullptr;        // [n]
  int32_t* slot_row = nullptr;   // [2m] row of each slot
  int32_t* slot_half = nullptr;  // [2m] slot -> half id (e, or e + m for (v_e -> u_e))
  int32_t* half_slot = nullptr;  // [2m] half id -> slot
  float* inv_deg_f = nullptr;    // [n]
  double* inv_deg_d = nullptr;   // [n]
  Task* tasks = nullptr;         // [ntasks] wave tasks: rows with <= kChunk slots
  int32_t ntasks = 0;
  Task* ptasks = nullptr;        // [nptasks] wave tasks for B = 64: runs of consecutive light
  int32_t nptasks = 0;           //   rows with <= 64 slots in total (part = row count)
  Task* wg_tasks = nullptr;      // [nwg] workgroup tasks: heavy rows, giant-row chunks
  int32_t nwg = 0;
  HeavyRow* giant = nullptr;     // [ngiant] rows cut into chunks
  int32_t ngiant = 0;
  int32_t nparts = 0;            // total partial rows
};

// One graph of a batch as the persistent kernel sees it (device pointers).
// Rows sorted by degree (descending) form groups of 64.  Row i of group gi
// has a record rec[(gi * 64 + i) * RW ...] of RW = 4 + 8 / K words: (row,
// degree, cb, 0) followed by its first kBatchSlots neighbour ids, K = 2 ids
// of 16 bits per word when narrow (n < 65535), else K = 1; its slots from
// kBatchSlots on sit column-major in nb, word w at nb[cb + w * 64].  Rows are
// padded with the zero row n up to their group's largest degree rounded up
// to kBatchSlots; records past the last row read (n, 0, 0, 0, n ...).
struct BatchGraph {
  int32_t n = 0;
  int32_t B = 0;                    // source-block width of this graph's items
  int32_t ngroups = 0;
  int32_t narrow = 0;               // 1: two 16-bit ids per neighbour word
  const int32_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const int32_t* slot_row = nullptr;
  const int32_t* tau_slot = nullptr;
  const int32_t* tau_row = nullptr;
  const float* inv_f = nullptr;
  const double* inv_d = nullptr;
  const uint32_t* rec = nullptr;
  const uint32_t* nb = nullptr;
  const float* grp_invf = nullptr;  // 1/degree of the records' rows (0 past the last)
  const double* grp_invd = nullptr;
  double* gacc = nullptr;
  // truncation and output of the run (prologue / epilogue kernels)
  const int32_t* deg = nullptr;
  const int32_t* half_slot = nullptr;
  double* out = nullptr;            // device output, m doubles
  int32_t m = 0;
  int32_t L = 0;                    // odd uniform truncation, 0: Theorem 3.2, -1: tau_slot
                                    // and tau_row already hold CalTau's lengths
  int32_t max_L = 0;
  int32_t active = 0;               // 1: graph takes part in the run
  double eps = 0.0;
  double lam = 0.0;
};

constexpr int kBatchSlots = 8;          // neighbour slots per gather batch (group widths padded to it)
constexpr int kBatchWordPad = 8 * 64;   // spare words after the last group

struct BatchItem {
  int32_t graph;
  int32_t s0;
};

// --------------------------------------------------------------- kernels (launch wrappers)
// All wrappers enqueue on `st` and return the hipError_t of the launch.

// gacc[k] = 1/d_s - [tau_k >= 1] * 1/(d_s d_j): the l = 0 and l = 1 terms of
// Eq. 9, whose probabilities are known in closed form (p_0 = e_s,
// p_1(s,s) = 0, p_1(j,s) = 1/d_j).
// include_l1 = 0 leaves the l = 1 term to the walk tail (TGT+ with tilde_tau = 0).
hipError_t launch_gacc_init(const DeviceGraph& g, const int32_t* tau_slot, int include_l1,
                            double* gacc, hipStream_t st);

// tau per slot: uniform L (odd) when L > 0, else the lambda* bound of
// Theorem 3.2 with Upsilon = Delta = 0.  Also the per-row maximum.
// CalTau (Algorithm 1, Eq. 6-8) for every slot with the omega eigenpairs of
// D^-1/2 A D^-1/2 of largest |lambda| (lam[omega], phi[n][omega] node-major on
// the device, pair 0 the trivial one); tau capped at the odd max_L.
constexpr int kMaxOmega = 256;
// capped (may be null): += half-edges whose automatic tau was cut to max_L.
hipError_t launch_caltau(const DeviceGraph& g, const double* lam, const double* phi, int omega,
                         double eps_tau, int max_L, int32_t* tau_slot, int32_t* tau_row,
                         hipStream_t st, unsigned long long* capped = nullptr);
// Ritz vectors phi[x][1..p] = V[:, 1..steps] Y (Y: steps x p32 row-major, p32 a multiple of
// kRitzCols), phi[x][0] = V[x]
constexpr int kRitzCols = 32;
hipError_t launch_ritz(int64_t n, int64_t ld, const double* V, int steps, const double* Y,
                       int p32, int p, int omega, double* phi, hipStream_t st);
hipError_t launch_tau(const DeviceGraph& g, int L, double eps_tau, double lam, int max_L,
                      int32_t* tau_slot, int32_t* tau_row, hipStream_t st,
                      unsigned long long* capped = nullptr);

// Mark block s_set's neighbour bits in mask buffer `buf` and clear block
// s_clear's bits (s_clear < 0: none) in the other buffer.  mask: 2 x n words,
// anymask: 2 x ceil(n/32) words.
hipError_t launch_mask_update(const DeviceGraph& g, int s_set, int s_clear, int B, int buf,
                              unsigned long long* mask, unsigned* anymask, hipStream_t st);

// Y2 = P P Y0 for the indicator block via the neighbour masks.  With B = 64
// and nz, nz[x] = (row x of Y2 has a nonzero) for rows of at most kChunk
// neighbours (heavier rows are left as they are, 1).
template <typename T>
hipError_t launch_twohop(const DeviceGraph& g, int B, const unsigned long long* mask,
                         const unsigned* anymask, T* Y, T* partials, uint8_t* nz, hipStream_t st);

// The two launches of launch_propagate, separately: the row gathers (giant
// rows leave chunk sums in partials) and the giant-row fix-up.  With B = 64
// and nz, neighbours u with nz[u] == 0 are not gathered (their rows of Yp are
// exact zeros, so every sum is unchanged).  Non-null ev_start / ev_stop take
// the start and end times of the row-gather kernel itself.
// mj (may be null): a mask update carried by extra workgroups of the same launch.
template <typename T>
hipError_t launch_propagate_rows(const DeviceGraph& g, int B, const T* Yp, T* Yn, T* partials,
                                 const AccJob& acc, hipStream_t st, const uint8_t* nz = nullptr,
                                 hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
                                 const MaskJob* mj = nullptr);
MaskJob mask_job(const DeviceGraph& g, int s_set, int s_clear, int B, int buf,
                 unsigned long long* mask, unsigned* anymask);
template <typename T>
hipError_t launch_fixup(const DeviceGraph& g, int B, const T* partials, T* Y, hipStream_t st);

// Yn = P Yp (dense block gather); `acc` (may be empty) accumulates the step in Yp.
template <typename T>
hipError_t launch_propagate(const DeviceGraph& g, int B, const T* Yp, T* Yn, T* partials,
                            const AccJob& acc, hipStream_t st);

// gacc[k] += (Y[s][c] - Y[j][c]) / d_s for the job's slots with l <= tau_k.
template <typename T>
hipError_t launch_accumulate(const DeviceGraph& g, int B, const T* Y, const AccJob& acc,
                             hipStream_t st);

// Last pass of a block's flattened walks: gacc[k] += (slot k's chunk sums in
// chunk order) / n_r.  It may ride on a later launch of the same stream that
// comes before the next block's walks (which reuse chunk_off, part and ctl).
struct FinishJob {
  int kbeg = 0, kend = 0;
  const int64_t* nr = nullptr;
  const int64_t* chunk_off = nullptr;
  const int64_t* ctl = nullptr;
  const double* part = nullptr;
  double* gacc = nullptr;   // null: no job
};

// Algorithm 3 summary per column of the block (top-gamma, rho bound, extremes).
// scratch: kColScratchBytes of device memory.
constexpr int kColParts = 2048;  // row chunks of the coalesced first pass (multiple of 4 * 64/B)
constexpr size_t kColScratchBytes =
    static_cast<size_t>(kColParts) * 64 *
        (kMaxGamma * (sizeof(double) + sizeof(int)) + 2 * sizeof(double) + sizeof(int)) +
    64 * (sizeof(int) + sizeof(double));
// acc / fin (optional): an accumulation step and a previous block's walk
// finish carried by the first launch as extra workgroups.
template <typename T>
hipError_t launch_colstats(const DeviceGraph& g, int s0, int B, int gamma, const T* Y,
                           ColStats* cs, void* scratch, hipStream_t st,
                           const AccJob* acc = nullptr, const FinishJob* fin = nullptr);

// n_r per slot (Eq. 13 with chi of Eq. 17 / Eq. 15); 0 where tau_k <= tilde.
template <typename T>
hipError_t launch_walk_counts(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int tilde,
                              int gamma,
                              double coef, int64_t nr_cap, const T* Y, const ColStats* cs,
                              const int32_t* tau_slot, int64_t* nr_slot, hipStream_t st);

// work[0] += walk pairs, work[1] += single-walk steps over slots [kbeg, kend)
hipError_t launch_work_totals(int kbeg, int kend, int tilde, const int32_t* tau_slot,
                              const int64_t* nr_slot, unsigned long long* work, hipStream_t st);

// Scratch of the flattened walks (required by launch_walks).
struct WalkScratch {
  int64_t* chunk_off = nullptr;   // [slots of a block + 1]
  double* part = nullptr;         // [capacity] chunk sums
  int64_t capacity = 0;
  int64_t* ctl = nullptr;         // [2]
};


// Walk tail: gacc[k] += mean_r X_r (Eq. 11) for the block's slots (ws must hold
// the chunk buffers; blocks whose chunks do not fit walk one slot per wave).
// With defer, the last pass is not launched but returned in *defer (gacc null
// when there is none); the caller runs it with launch_walk_finish or carries
// it on launch_colstats.
template <typename T>
hipError_t launch_walks(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int tilde,
                        uint64_t seed, const T* Y, const int32_t* tau_slot,
                        const int64_t* nr_slot, double* gacc, const WalkScratch& ws,
                        hipStream_t st, FinishJob* defer = nullptr);
hipError_t launch_walk_finish(const FinishJob& job, hipStream_t st);
// the nodes of walk pair r of half-edge (i, j) over len steps: nodes[0, len)
// from i, nodes[len, 2 len) from j (device memory)
hipError_t launch_walk_trace(const DeviceGraph& g, int i, int j, uint32_t r, int len,
                             uint64_t seed, int32_t* nodes, hipStream_t st);

// out[e] = gacc[slot(u_e->v_e)] + gacc[slot(v_e->u_e)] (Algorithm 2 line 12).
hipError_t launch_combine(const DeviceGraph& g, const double* gacc, double* out,
                          hipStream_t st);

// Trace outputs in input order.
hipError_t launch_trace(const DeviceGraph& g, const int32_t* tau_slot, const int64_t* nr_slot,
                        int32_t* tau_out, int64_t* nr_out, hipStream_t st);

// --------------------------------------------------------------- per-source TGT+
// Frontier-sparse traversal with the per-source switch step of Eq. 14, one
// workgroup per source (kernels_sparse.hip).  Columns are 64-bit fixed point
// Q[y] = p_l(i, y) / d_y in units of 2^-63, one pair of n-word columns and one
// pair of n-entry support lists per workgroup slot.
constexpr int kSrcThreads = 256;

struct SrcArgs {
  int32_t n = 0;
  const int32_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const int32_t* tau_slot = nullptr;
  const int32_t* tau_row = nullptr;
  const int32_t* srcs = nullptr;   // source list (null: node k is entry k)
  const int64_t* hoff = nullptr;   // [nsrc + 1] prefix of the listed sources' degrees (null: rowptr)
  int64_t list_base = 0;           // first list entry of this launch (workgroup w takes entry base + w)
  int64_t nsrc = 0;                // list length
  int64_t pos_base = 0;            // hoff[list_base]: positions are relative to it
  uint64_t* Q = nullptr;           // [2 * slots * n], all zero between sources
  int32_t* S = nullptr;            // [2 * slots * n]
  int32_t* slot_ctl = nullptr;     // [2 * slots]: final support size, which column holds it
  int32_t* tilde_row = nullptr;    // [n] switch step per source
  int64_t* nr_slot = nullptr;      // [2m] walk pairs per CSR slot
  double* gacc = nullptr;          // [2m] per-half sums (l = 0 term already in)
  int32_t* pos_slot = nullptr;     // [positions] CSR slot of each position
  int32_t* pos_w = nullptr;        // [positions] workgroup slot holding its source's column
  int64_t* nr_pos = nullptr;       // [positions] walk pairs
  unsigned long long* totals = nullptr;   // walk pairs, walk steps, pushed entries, min / max tilde
  double coef = 0.0;               // 8 ln(2m / delta) / eps^2 (Eq. 13)
  int64_t nr_cap = 0;
  int gamma = 10;
  int rule = 0;                    // 0: Eq. 14 as printed (walk pairs), 1: walk steps
  int force_tilde = -1;            // >= 0: switch at min(force_tilde, tau_p) instead
};

struct SrcWalkArgs {
  int32_t n = 0;
  int64_t P = 0;                   // positions of this wave
  const int32_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const int32_t* slot_row = nullptr;
  const int32_t* tau_slot = nullptr;
  const int32_t* tilde_row = nullptr;
  const uint64_t* Q = nullptr;
  uint64_t* Qw = nullptr;          // same memory, cleared after the walks
  const int32_t* S = nullptr;
  const int32_t* slot_ctl = nullptr;
  const int32_t* pos_slot = nullptr;
  const int32_t* pos_w = nullptr;
  const int64_t* nr_pos = nullptr;
  int64_t* chunk_off = nullptr;    // [P + 1]
  int64_t* ctl = nullptr;          // [2]
  double* part = nullptr;          // [capacity]
  int64_t capacity = 0;
  double* gacc = nullptr;
  unsigned k0 = 0, k1 = 0;         // Philox key
  // a batch of chunks [cbeg, cend) set by the host (part holds the batch from
  // index 0); cend < 0: all chunks at once, or one wave per half when they do
  // not fit the buffer (ctl[1] == 0)
  int64_t cbeg = 0, cend = -1;
  // a half with more chunks than this in the batch is summed by a whole
  // workgroup (fixed segments, then the segment sums in order)
  int64_t finish_seg = 4096;
};

hipError_t launch_src_head(const SrcArgs& a, int grid, hipStream_t st);
// plain fills (kernels, so that a captured sequence holds no memset nodes)
hipError_t launch_fill_u64(uint64_t* p, int64_t count, uint64_t value, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t st);
// vol[x] = sum of the degrees of x's neighbours (the first push of source x)
hipError_t launch_nbr_volume(const DeviceGraph& g, int64_t* vol, hipStream_t st);
// mm[0] = min(mm[0], min tau_row), mm[1] = max(mm[1], max tau_row)
hipError_t launch_tau_range(int n, const int32_t* tau_row, unsigned long long* mm, hipStream_t st);
// scan, walks and finish of a wave (its columns are cleared by the next head
// that takes the slot, or by launch_src_clear after the last wave)
hipError_t launch_src_walks(const SrcWalkArgs& a, hipStream_t st);
// the same in parts: the chunk scan (ctl[0] = chunks), one batch of walks with
// its finish pass; and the clearing of every used slot's final column
hipError_t launch_src_scan(const SrcWalkArgs& a, hipStream_t st);
hipError_t launch_src_walk_batch(const SrcWalkArgs& a, hipStream_t st);
hipError_t launch_src_clear(const SrcWalkArgs& a, int nslots_used, hipStream_t st);
// dst[x] = src[idx[x]] for x < n (per-node results of a renumbered graph, in the
// caller's ids)
hipError_t launch_gather_i32(const int32_t* src, const int32_t* idx, int32_t* dst, int64_t n,
                             hipStream_t st);

// --------------------------------------------------------------- learned closure
constexpr int kMlpParams = 5313;
constexpr int kFeat = 16;
constexpr int kRecSteps = 8;   // L0

template <typename T>
hipError_t launch_record_init(const DeviceGraph& g, T* rdiag, T* roff, hipStream_t st);
template <typename T>
hipError_t launch_record(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int ell,
                         const T* Y, T* rdiag, T* roff, hipStream_t st);
// Recordings of steps ell - 1 and ell of a block from the state at ell - 1
// (no dense step for ell); 3 <= ell <= kRecSteps.
template <typename T>
hipError_t launch_record_last(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int ell,
                              const T* Y, T* rdiag, T* roff, hipStream_t st);
template <typename T>
hipError_t launch_features(const DeviceGraph& g, const T* rdiag, const T* roff, double lam,
                           float* X, double* s0, double* uK, double* lo, double* hi,
                           hipStream_t st);
hipError_t launch_targets(int64_t m, const double* s_ref, const double* s0, const double* uK,
                          float* z, float* w, hipStream_t st);
hipError_t launch_norm_stats(const float* X, int64_t N, float* norm, hipStream_t st);
hipError_t launch_feature_range(const float* X, int64_t N, float* fmin, float* fmax,
                                hipStream_t st);
hipError_t launch_mlp_train_step(const float* theta, const float* norm, const float* X,
                                 const float* z, const float* w, const int64_t* idx,
                                 int64_t nbatch, float inv_count, float* grads, float* lossp,
                                 float* grad, float* loss_out, hipStream_t st);
hipError_t launch_adam(float* theta, const float* grad, float* m1, float* m2, float lr,
                       float b1, float b2, float eps, int step, hipStream_t st);
hipError_t launch_mlp_infer(const float* theta, const float* norm, const float* X, int64_t N,
                            int bf16, float* y, hipStream_t st);
hipError_t launch_closure_apply(const DeviceGraph& g, const float* zpred, const double* s0,
                                const double* uK, const double* lo, const double* hi,
                                const float* X, const float* fmin, const float* fmax, double eps,
                                int B, int force, double* out, unsigned char* fb,
                                int* block_flag, unsigned long long* count, hipStream_t st);
hipError_t launch_combine_masked(const DeviceGraph& g, const double* gacc,
                                 const unsigned char* fb, double* out, hipStream_t st);

// --------------------------------------------------------------- Lanczos helpers
hipError_t launch_nmat_spmv(const DeviceGraph& g, const double* sid, const double* x,
                            double* y, hipStream_t st);
hipError_t launch_multi_dot(const double* V, int ncols, int64_t ld, const double* w,
                            int64_t n, double* out, hipStream_t st);
hipError_t launch_multi_axpy(const double* V, int ncols, int64_t ld, const double* h,
                             double* w, int64_t n, hipStream_t st);

// Persistent batch kernel for items of block width B: workgroups of nt
// threads (256, 512, 1024) take items from *ticket (zero before the launch)
// until it passes nitems.  lds: block states in dyn_lds bytes of dynamic
// LDS, else in slabs of slab_elems elements per workgroup (nt = 256).
template <typename T>
hipError_t launch_batch(int nt, bool lds, int B, int grid, size_t dyn_lds, const BatchGraph* graphs,
                        const BatchItem* items, int nitems, int* ticket, T* slabs,
                        int64_t slab_elems, hipStream_t st);
template <typename T>
const void* batch_kernel_ptr(int nt, bool lds, int B);
hipError_t launch_fill_i32(int32_t* p, int count, int value, hipStream_t st);
// Truncation per slot and row, and the closed-form l = 0, 1 terms, for every
// row of the active graphs (node_off: G + 1 prefix of node counts); with mm,
// mm[0] / mm[1] take the min / max of the rows' truncations; capped (may be
// null) += half-edges whose automatic length was cut to max_L.
hipError_t launch_batch_prologue(const BatchGraph* graphs, const int64_t* node_off, int G,
                                 int64_t total_rows, int32_t* mm, unsigned long long* capped,
                                 hipStream_t st);
// out[e] = g(u_e, v_e) + g(v_e, u_e) for every edge of the active graphs.
hipError_t launch_batch_combine(const BatchGraph* graphs, const int64_t* edge_off, int G,
                                int64_t total_edges, hipStream_t st);

}  // namespace sc
