/*
 * sc.h - all-edge spanning centrality (AESC) on AMD MI355X (gfx950).
 *
 * Spanning centrality s(e) of an edge e of a connected undirected graph is the
 * fraction of spanning trees that contain e (Definition 2.1); it equals the
 * effective resistance between the endpoints (Section 2.3).  This library
 * returns an estimate s^(e) for every edge with |s^(e) - s(e)| <= eps
 * (Definition 2.2, Eq. 1) using the truncated series of Eq. 2:
 *
 *   s_tau(e_ij) = sum_{l=0..tau} p_l(i,i)/d_i + p_l(j,j)/d_j - 2 p_l(j,i)/d_i
 *
 * with p_l(x,i) = (D^-1 A)^l [x,i] (Table 1), computed either by
 * deterministic traversal of every source column (TGT, Algorithm 2) or by a
 * traversal head plus a random-walk tail (TGT+, Algorithm 4).
 *
 * Conventions for every entry point:
 *   - return value: SC_OK (0) or a negative SC_E* code; no C++ exception
 *     crosses this boundary;
 *   - on error no output buffer is written and partial allocations are freed;
 *     sc_last_error() returns a text description of the calling thread's
 *     last error;
 *   - a graph handle is not thread-safe; distinct handles are independent;
 *   - pointers named *_host are host memory; "out" and the optional trace
 *     arrays are host memory unless SC_DEVICE_PTRS is set in the options'
 *     flags, in which case they are device memory on the handle's device
 *     and results are stream-ordered on the options' stream;
 *   - with host outputs every call returns after the results are written;
 *   - sc_all_edges_ex runs the per-block tails (candidate summary, walk
 *     counts, walks, the last step's accumulation) on a second stream owned
 *     by the handle; it waits for the options' stream before its first
 *     launch and the options' stream waits for it before the combine, so
 *     the call stays ordered on the options' stream.
 */
#ifndef SC_H
#define SC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
enum {
  SC_OK = 0,
  SC_EINVAL = -1,        /* bad argument (size, range, eps not in (0,1), L < 0, ...) */
  SC_ESELFLOOP = -2,     /* an edge (i,i): A must be 0/1 off the diagonal (Section 2.1) */
  SC_EDUP = -3,          /* the same undirected edge twice (without SC_MERGE_DUPS) */
  SC_EDISCONNECTED = -4, /* SC is defined for connected graphs (Definition 2.1) */
  SC_EBIPARTITE = -5,    /* the series needs a non-bipartite graph (Section 2.1) */
  SC_ENOMEM = -6,        /* device or host allocation failed */
  SC_EHIP = -7,          /* a HIP runtime call failed (text in sc_last_error) */
  SC_ENOTIMPL = -8       /* option combination not supported */
};

/* build flags (sc_build_graph) */
#define SC_MERGE_DUPS 0x2u   /* merge repeated edges instead of failing with SC_EDUP */
#define SC_DEGREE_ORDER 0x4u /* store the nodes renumbered by descending degree (ties by id)
                                for the locality of the walks and traversals; see
                                sc_build_graph (sc_build_graph only) */
#define SC_BFS_ORDER 0x8u    /* store the nodes renumbered in breadth-first order from the
                                highest-degree node, for the locality of the source blocks;
                                see sc_build_graph (sc_build_graph only) */

/* run flags (sc_options.flags) */
#define SC_DEVICE_PTRS 0x1u  /* out / trace arrays are device pointers */
#define SC_TIME_KERNELS 0x4u /* time a sample of propagation launches with HIP events */
#define SC_GRAPH_REPLAY 0x8u /* sc_batch_all_edges: record the device work as a hipGraph
                                on the first call, replay it on later identical calls */
#define SC_TAU_SPECTRAL 0x10u /* automatic truncation (L = 0) by CalTau, Algorithm 1, with
                                 the graph's spectrum (sc_compute_spectrum / sc_set_spectrum)
                                 instead of the lambda*-bound; SC_TGT and SC_TGT_PLUS */
#define SC_PER_SOURCE 0x20u   /* SC_TGT_PLUS only: Algorithm 4 source by source, each with a
                                 frontier-sparse traversal and its own switch step by Eq. 14
                                 (Section 4.2.1), instead of dense blocks of sources with one
                                 switch step per call; see sc_all_edges_ex */

/* methods (sc_options.method) */
#define SC_TGT 0       /* Algorithm 2: traversal to tau for every source */
#define SC_TGT_PLUS 1  /* Algorithm 4: traversal to tilde_tau, then random walks */
#define SC_LEARNED 2   /* learned tail closure after L0 = 8 steps, TGT as fallback */

typedef struct sc_graph sc_graph;   /* opaque: device CSR, maps, work buffers */
typedef struct sc_mlp sc_mlp;       /* opaque: tail-closure network on the device */

typedef struct sc_options {
  int method;          /* SC_TGT or SC_TGT_PLUS                                      */
  int precision;       /* 0: FP32 propagation, 1: FP64 propagation; sums always FP64 */
  int block;           /* source-block width B (columns per pass): 0 = default      */
  int gamma;           /* candidate count of Algorithm 3; < 0 means 10 (Section 5.1) */
  double delta;        /* TGT+ failure probability; <= 0 means 1/n (Section 5.1)     */
  uint64_t seed;       /* Philox4x32-10 key for the walks                            */
  int tilde_tau;       /* TGT+ switch step: < 0 = chosen by the cost model          */
  int max_L;           /* cap on automatic truncation lengths (<= 0: 255)            */
  double lambda_star;  /* > 0: use this value of max_{k>=2}|lambda_k|; else computed  */
  unsigned flags;      /* SC_DEVICE_PTRS | SC_TIME_KERNELS                           */
  void* stream;        /* hipStream_t to run on; NULL = the null stream             */
  /* optional trace outputs (NULL = not wanted); same memory kind as out */
  int32_t* tau_out;        /* [m]  truncation tau_ij used per input edge             */
  int32_t* tilde_tau_out;  /* [n]  switch step per source node (TGT: tau_p)          */
  int64_t* nr_out;         /* [2m] walk pairs per half-edge: [0,m) = (u_e -> v_e),
                                   [m,2m) = (v_e -> u_e)                            */
  /* SC_LEARNED only */
  const sc_mlp* mlp;       /* trained network (required)                              */
  int infer_bf16;          /* 1: BF16 MFMA inference (default), 0: FP32               */
  int force_fallback;      /* 1: every edge takes the fallback traversal              */
  /* SC_PER_SOURCE only */
  const int32_t* sources;  /* host list of nsources distinct source nodes, or NULL for all;
                              only the halves (i, j) with i listed are computed, so out[e]
                              is the full estimate only where both endpoints are listed
                              (the others hold the l = 0 term of an unlisted half)      */
  int64_t nsources;
  int switch_rule;         /* 0: Eq. 14 as printed (frontier volume against walk pairs);
                              1: against single-walk steps, 2 (tau_ij - l) per pair      */
} sc_options;

typedef struct sc_stats {
  int L_used;              /* largest truncation used                                  */
  int L_min;               /* smallest truncation used                                 */
  int tilde_tau;           /* TGT+ switch step used (uniform over sources), else -1   */
  int block;               /* source-block width used                                  */
  double lambda_star;      /* value used for automatic truncation (0 if not needed)   */
  int64_t walks;           /* walk pairs simulated                                    */
  int64_t walk_steps;      /* single-walk steps simulated                             */
  int64_t prop_launches;   /* dense propagation launches that gather every neighbour
                              row (at block width 64 the first dense step after the
                              two-hop step skips zero rows and is not counted)      */
  double prop_ms;          /* sum of the timed propagation launches (SC_TIME_KERNELS) */
  double prop_bytes;       /* algorithmic bytes of the counted propagation launches   */
  double total_ms;         /* wall time of the call on the stream                     */
  int64_t fallback_edges;  /* SC_LEARNED: edges computed by the fallback traversal    */
  int64_t prop_timed;      /* launches whose times prop_ms sums (SC_TIME_KERNELS times
                              every 15th counted launch with events that take the
                              kernel's own start and end)                          */
  double host_ms;          /* host time spent issuing the block loop (the GPU work
                              queued behind it runs meanwhile)                     */
  int64_t L_capped;        /* edges whose automatic truncation was cut to max_L: the
                              error bound of Theorem 3.2 does not cover them (always 0
                              with a fixed L; SC_LEARNED: of the fallback truncation) */
  int32_t lambda_converged;/* 1: lambda* from Lanczos runs whose extreme Ritz pairs
                              passed the residual test; 0: a run reached its step limit
                              first (the value is then an estimate only); -1: lambda*
                              given by the caller or not needed                      */
  int32_t tilde_min;       /* smallest per-source switch step (TGT+), else -1         */
  int32_t tilde_max;       /* largest per-source switch step (TGT+), else -1          */
  int32_t reserved_;
  int64_t push_edges;      /* SC_PER_SOURCE: neighbour-list entries pushed by the
                              frontier-sparse traversal, else 0                     */
} sc_stats;

/* Fill *o with defaults: TGT, FP32, gamma 10, delta 1/n, seed 0x5C5C, auto tilde_tau. */
void sc_default_options(sc_options* o);

/*
 * Build a graph handle from an undirected edge list (Section 2.1: simple,
 * unweighted).  u_host/v_host: m node ids each in [0, n), int64, host
 * memory, copied (the caller keeps ownership).  Edge e = (u_host[e],
 * v_host[e]); results are reported per e in this order.  Checks: ids in
 * range (SC_EINVAL), no self-loops (SC_ESELFLOOP), no repeated edge
 * (SC_EDUP unless SC_MERGE_DUPS), connected (SC_EDISCONNECTED), not
 * bipartite (SC_EBIPARTITE).  With SC_MERGE_DUPS repeated edges report the
 * same value.  The CSR, degree and half-edge maps are uploaded to the
 * current HIP device.  n >= 2, 1 <= m, 2m < 2^31.
 * Node orders (at most one of the two flags; SC_EINVAL for both):
 * SC_DEGREE_ORDER stores node x as its rank by descending degree (ties by
 * ascending x), so the rows that walks and pushes visit most share cache
 * lines; SC_BFS_ORDER stores the nodes in the order a breadth-first search
 * visits them, started at the highest-degree node (the lowest id among
 * equals) and taking each node's neighbours in ascending id, so a block of
 * consecutive sources lies close together in the graph (nodes it cannot
 * reach keep ascending id after the others; such a graph is rejected as
 * disconnected anyway).  The graph is the same; every node id the API takes
 * or returns stays the caller's (source lists, tilde_tau_out, spectra, walk
 * traces) and per-edge results keep the input order.  A flagged handle
 * computes exactly what an unflagged handle built on the renumbered edge
 * list computes (same sums, same walks: the Philox counters and the
 * neighbour order are those of the renumbered graph), so its results differ
 * from an unflagged handle's on the caller's labels by rounding order and
 * the walks' randomness only.  Costs up to 24 bytes per edge of host memory
 * during the build and 4 bytes per node of device memory.
 */
int sc_build_graph(int64_t n, int64_t m, const int64_t* u_host, const int64_t* v_host,
                   unsigned flags, sc_graph** out);

/* Node and edge counts of a handle. */
int sc_graph_size(const sc_graph* g, int64_t* n, int64_t* m);

/* Release a handle and all device memory it owns.  NULL is allowed. */
void sc_free_graph(sc_graph* g);

/*
 * lambda* = max_{k>=2} |lambda_k| of D^-1/2 A D^-1/2 (Lemma 3.1), the rate in
 * the truncation bound of Theorem 3.2 (Algorithm 1 line 1).  Computed once by
 * Lanczos on the GPU (deflated of the top eigenvector sqrt(d)/sqrt(2m)) and
 * cached in the handle.  The value returned is an upper estimate: the
 * extreme Ritz value plus its residual norm.
 */
int sc_lambda_star(sc_graph* g, double* lam);

/*
 * Walk trace (a check of the walk stream, not part of a run): the nodes that
 * walk pair r of half-edge (i -> j) visits over `length` steps, exactly as the
 * TGT+ walk kernels take them (Algorithm 4's walks, estimator of Eq. 11).
 * Step t of the walk from side s (0: from i, 1: from j) draws word (t-1) mod 4
 * of Philox4x32-10 with counter (i, j, r, s * 2^31 + floor((t-1)/4)) and key
 * (seed mod 2^32, seed / 2^32), and moves to neighbour floor(word * d / 2^32)
 * of the current node's row (neighbours in ascending id order).
 * nodes_host (host, 2 * length int32, caller-owned): nodes_host[t-1] is the
 * node after step t from i, nodes_host[length + t-1] the same from j.
 * i and j need not be adjacent.  On a handle built with SC_DEGREE_ORDER or
 * SC_BFS_ORDER the walk is the renumbered graph's (counters and rows in its
 * ids), and i, j and the nodes returned are the caller's ids.  Errors: SC_EINVAL for ids out of range,
 * r outside [0, 2^32), length outside [0, 2^20]; SC_ENOMEM / SC_EHIP from the
 * device (nodes_host is then not written).
 */
int sc_walk_trace(sc_graph* g, int32_t i, int32_t j, int64_t r, int32_t length, uint64_t seed,
                  int32_t* nodes_host);

/* ---- spectrum for CalTau (Algorithm 1, Theorem 3.2, Eq. 6-8) ----------------
 * The omega eigenpairs (lambda_k, phi_k) of N = D^-1/2 A D^-1/2 of largest
 * |lambda|: lambda[0] = 1 with phi_0 = sqrt(d / 2m), then |lambda| descending.
 * phi is node-major: phi[x * omega + k].  CalTau uses pairs 2 .. omega-1
 * (1-based) exactly and bounds the others by |lambda_omega|; the bound holds if
 * no eigenvalue left out is larger in magnitude than |lambda_omega|.
 * The graph keeps one spectrum (replaced by every set/compute call). */

/* Lanczos with full re-orthogonalisation on the device (the trivial pair
 * deflated), checked every 25 steps, stopping when the omega - 1 Ritz pairs of
 * largest |theta| have residual estimates <= tol (<= 0: 1e-8) or after max_iter
 * steps (<= 0: 2048; also capped by n - 1 and a 16 GiB basis).  Keeps the
 * longest prefix of pairs within tol: *omega_kept (<= omega) and their largest
 * residual estimate *max_residual (either may be NULL).  A single-vector Krylov
 * space finds one vector per repeated eigenvalue, so graphs with repeated
 * eigenvalues among the top ones need sc_set_spectrum instead.
 * omega in [2, 256] (clamped to n).  SC_EINVAL if no pair converges. */
int sc_compute_spectrum(sc_graph* g, int omega, int max_iter, double tol, int* omega_kept,
                        double* max_residual);

/* Load a spectrum computed elsewhere: lambda[omega], phi[n * omega] (host, node-major,
 * copied).  SC_EINVAL unless 2 <= omega <= min(n, 256), lambda[0] = 1, the others in
 * (-1, 1) and ordered by |lambda| descending. */
int sc_set_spectrum(sc_graph* g, int omega, const double* lambda, const double* phi);

/* *omega = stored pair count (0: none); lambda[omega] and phi[n * omega] (host) are
 * filled when not NULL. */
int sc_get_spectrum(const sc_graph* g, int* omega, double* lambda, double* phi);

/*
 * All-edge SC with default options (FP32 propagation, TGT when L > 0 or
 * TGT+ with automatic truncation when L == 0).
 *   eps : absolute error target, in (0, 1) (Definition 2.2).
 *   L   : > 0  every edge uses tau = L rounded up to odd (Eq. 5 parity);
 *         == 0 per-edge tau_ij from Theorem 3.2 with lambda* (Eq. 6 with
 *              Upsilon = Delta = 0), at eps for TGT and eps/2 for TGT+
 *              (Algorithm 4 line 2);
 *         < 0 SC_EINVAL.
 *   out : m doubles, host memory, input edge order.
 */
int sc_all_edges(sc_graph* g, double eps, int L, double* out);

/*
 * All-edge SC with explicit options; st (may be NULL) receives statistics.
 * TGT (Algorithm 2): for every source i and l = 1..tau_ij every half-edge
 * (i,j) gains (p_l(i,i) - p_l(j,i))/d_i (Eq. 9); s = g(i,j) + g(j,i).
 * TGT+ (Algorithm 4): the traversal stops at tilde_tau; each half-edge with
 * tau_ij > tilde_tau adds the mean of n_r samples of X (Eq. 11), n_r from
 * Eq. 13 with chi from Algorithm 3 / Eq. 17 (Eq. 15 when gamma == 0).
 * Random walks follow the Philox4x32-10 counter scheme documented in the
 * implementation (counter = (i, j, r, side*2^31 + step/4), key = seed).
 * Environment (read by the library, all optional): SC_COST_GATHER_BW,
 * SC_COST_STEP_FIXED, SC_COST_SKIP_FRAC, SC_COST_TAIL_FIXED,
 * SC_COST_TAIL_PER_NODE, SC_COST_WALK_STEP and SC_COST_OVERLAP override the
 * constants of the switch-step cost model (bytes/s, s, fraction of a dense
 * step, s, s per node, s per walk step, share);
 * SC_WALK_CHUNK_CAPACITY caps the
 * walk chunk-sum buffer when it is first allocated (blocks whose walks do not
 * fit then walk one slot per wave; used by the tests).
 */
int sc_all_edges_ex(sc_graph* g, double eps, int L, const sc_options* o, double* out,
                    sc_stats* st);
/*
 * With SC_PER_SOURCE (TGT+): every source i starts at p_0(., i) = e_i and,
 * at l = 1, 2, ... (at l = 0 the volume d_i cannot exceed the d_i halves' walk
 * pairs), tests Eq. 14: the volume of the nodes with p_l(v, i) != 0
 * against the walk pairs (switch_rule 0) or walk steps (1) that stopping at l
 * would need (Eq. 13 with chi of Algorithm 3 at q = p_l(., i)); the first l
 * where the volume is larger, or l = max_j tau_ij, is tilde_tau_i (recorded in
 * tilde_tau_out).  Steps are pushed over the support only.  tilde_tau >= 0 in
 * the options forces min(tilde_tau, max_j tau_ij) for every source instead.
 * Any gamma >= 0 is accepted.  The traversal keeps 64-bit fixed-point columns
 * (unit 2^-63) and sums them with integer atomics, so results are
 * reproducible; precision and block are ignored.  Per-source columns take
 * 24 n bytes per workgroup slot (up to 2048 slots, within half the free
 * device memory, the handle's slot buffers from earlier calls counted as free,
 * and at most 128 GiB, or SC_SOURCE_SLOT_BYTES); the handle keeps them for
 * later calls until sc_free_graph.  st: tilde_min / tilde_max,
 * push_edges, walks, walk_steps; with SC_TIME_KERNELS, prop_ms is the time of
 * the waves' walk phases (events on the stream), prop_launches = prop_timed =
 * waves and prop_bytes = 20 bytes per single-walk step (row bounds, neighbour
 * id, column entry).  Environment (tests): SC_SOURCE_PART_CAPACITY caps the
 * walk chunk-sum buffer (smaller walk batches), SC_SOURCE_FINISH_SEG the chunk
 * count of a half above which a workgroup sums its chunk sums (default 4096).
 */

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops that forbid allocation): per-source TGT+, as sc_all_edges_ex
 * with method SC_TGT_PLUS and SC_PER_SOURCE, with every work buffer carved
 * from a static device array of 128 MiB per GPU (held by each GPU the library
 * runs on until the process ends) instead of allocated.
 *   out, and the optional tau_out / tilde_tau_out / nr_out of o: device
 *   pointers on the handle's device (SC_DEVICE_PTRS is implied); results are
 *   stream-ordered on o->stream.
 *   o: method SC_TGT_PLUS (else SC_ENOTIMPL); no source list (SC_EINVAL);
 *   the automatic truncation needs lambda* already known, from
 *   o->lambda_star or an earlier sc_lambda_star / run on the handle (SC_EINVAL
 *   otherwise, since computing it allocates), or a fixed L, or
 *   SC_TAU_SPECTRAL with a stored spectrum.
 *   st (may be NULL): as sc_all_edges_ex; asking for it synchronises the stream
 *   (total_ms is then host time).
 * Graphs whose buffers do not fit the array (about 20 bytes per half-edge plus
 * 24 bytes per node and workgroup slot) are refused with SC_EINVAL.  The array
 * is shared by every call on a GPU and keeps the last call's contents: calls
 * that overlap on one GPU race.  No memory is allocated; fills are kernels.
 */
int sc_all_edges_static(sc_graph* g, double eps, int L, const sc_options* o, double* out,
                        sc_stats* st);

/* ------------------------------------------------------------------ learned closure
 *
 * Not in the paper: an optional form that stops the traversal after L0 = 8
 * steps, truncates at the odd tau0 = 7 and predicts the remaining tail.  The
 * series terms of Eq. 2 have the spectral form of Eq. 18 with non-negative
 * weights, so the pair sums u_k = t_2k + t_2k+1 are a non-negative mixture of
 * geometric sequences; hence the tail lies in [u3 r/(1-r), u3 l2/(1-l2)] with
 * r = u3/u2 and l2 = lambda*^2.  The network (16 -> 64 -> 64 -> 1, silu)
 * predicts z = tail/u3 and the prediction is clamped to that interval, so the
 * error of every edge is at most u3 (hi - lo); edges where that exceeds eps,
 * or whose features leave the training range, are recomputed by TGT with the
 * truncation of Theorem 3.2.  Arrays named X, z, w, y below are DEVICE
 * pointers: X is row-major [N][16] float, z, w, y are [N] float.
 */
typedef struct sc_train_options {
  int epochs;          /* passes over the data (default 20)            */
  int batch;           /* samples per Adam step (default 4096)         */
  float lr;            /* Adam step size (default 2e-3)                */
  uint64_t seed;       /* shuffling seed                               */
  void* stream;        /* hipStream_t, NULL = null stream             */
} sc_train_options;

void sc_default_train_options(sc_train_options* t);

/* New network with seeded fan-in-scaled uniform weights and zero biases. */
int sc_mlp_create(uint64_t seed, sc_mlp** out);
void sc_mlp_free(sc_mlp* net);

/* Copy parameters (5313 floats: W1[64][16], b1[64], W2[64][64], b2[64],
 * W3[64], b3), feature normalisation (32 floats: mean[16], 1/std[16]) and
 * feature range (32 floats: min[16], max[16]) to / from host memory; any
 * pointer may be NULL.  Setting a range enables the out-of-range fallback. */
int sc_mlp_get(const sc_mlp* net, float* params, float* norm, float* range);
int sc_mlp_set(sc_mlp* net, const float* params, const float* norm, const float* range);

/* Write the network (parameters, normalisation and feature range) to a file
 * (binary, little-endian, with a checksum; the layout is documented in the
 * implementation).  Adam's moments are not saved.  Errors: SC_EINVAL when the
 * file cannot be written.  The network is unchanged. */
int sc_mlp_save(const sc_mlp* net, const char* path);

/* New network from a file written by sc_mlp_save on the current device;
 * *out is NULL on error (SC_EINVAL: missing file, wrong size, header or
 * checksum, NaN values). */
int sc_mlp_load(const char* path, sc_mlp** out);

/* Training data of one graph: features X [m][16] (from the first 8 steps),
 * targets z = (s_Lref - s_7)/u3 and weights w (0 where u3 = 0), with s_Lref
 * from TGT at the uniform odd truncation L_ref (e.g. 201).  Device pointers. */
int sc_closure_dataset(sc_graph* g, int L_ref, int precision, float* X, float* z, float* w,
                       void* stream);

/* Features and certified interval of every edge (device pointers; any of the
 * double arrays may be NULL): s0 = s_7, uK = u3, [lo, hi] as above. */
int sc_closure_features(sc_graph* g, int precision, float* X, double* s0, double* uK,
                        double* lo, double* hi, void* stream);

/* Mean squared error training with Adam on N samples; the first call fits the
 * normalisation and the feature range on X.  loss_per_epoch (host, may be
 * NULL) receives the mean weighted loss of every epoch. */
int sc_mlp_train(sc_mlp* net, const float* X, const float* z, const float* w, int64_t N,
                 const sc_train_options* t, float* loss_per_epoch);

/* Gradient of the mean weighted squared error over all N samples (host
 * outputs: grad[5313], loss[1]); the normalisation in use is applied. */
int sc_mlp_grad(sc_mlp* net, const float* X, const float* z, const float* w, int64_t N,
                float* grad_host, float* loss_host, void* stream);

/* y = network(X) for N samples, BF16 MFMA (bf16 = 1) or FP32 (bf16 = 0). */
int sc_mlp_predict(const sc_mlp* net, const float* X, int64_t N, int bf16, float* y,
                   void* stream);

/* ------------------------------------------------------------------ batches
 *
 * Not in the paper: many independent graphs through TGT (Algorithm 2) in one
 * persistent launch.  Every graph's result is what sc_all_edges_ex gives for
 * it with method SC_TGT and the same eps, L, precision and (for B in
 * {16, 32, 64}) block: tau per edge from Theorem 3.2 with that graph's own
 * lambda* (Eq. 6 with Upsilon = Delta = 0, capped at max_L) or a fixed odd L,
 * and s(i,j) = g(i,j) + g(j,i) with the per-half-edge sums of Eq. 9.
 * A work item is one source block of one graph; a workgroup runs all of its
 * steps with the block's state in LDS when it fits (else in a device slab),
 * taking items from an atomic ticket counter, longest first.
 */
typedef struct sc_batch sc_batch;

/* Build G graph handles at once (each validated as by sc_build_graph; the
 * error text names the failing graph) plus the sliced neighbour lists the
 * batch kernel reads.  n[g], m[g]: sizes; u_host[g], v_host[g]: the m[g]
 * edge endpoints of graph g (int64, host, copied).  flags as sc_build_graph,
 * except SC_DEGREE_ORDER and SC_BFS_ORDER (SC_EINVAL). */
int sc_build_batch(int G, const int64_t* n, const int64_t* m, const int64_t* const* u_host,
                   const int64_t* const* v_host, unsigned flags, sc_batch** out);

/* Number of graphs. */
int sc_batch_size(const sc_batch* b, int* G);

/* Graph i of the batch as an ordinary handle (borrowed: owned and freed by
 * the batch; usable with every sc_graph call). */
int sc_batch_graph(sc_batch* b, int i, sc_graph** g);

/* Release the batch, its graphs and all device memory.  NULL is allowed. */
void sc_free_batch(sc_batch* b);

/*
 * All-edge SC of every graph.  L: NULL (all automatic) or G ints, L[g] as
 * the L argument of sc_all_edges (0 automatic, > 0 fixed odd-rounded).
 * o: method must be SC_TGT; precision, max_L, lambda_star (applied to every
 * graph when > 0), stream and flags as for sc_all_edges_ex; with
 * SC_TAU_SPECTRAL every automatic graph that holds a spectrum
 * (sc_compute_spectrum / sc_set_spectrum on sc_batch_graph) takes CalTau
 * (Algorithm 1), the others the lambda*-bound; block: 0 = the
 * tuned width of the graph's size bucket (sc_batch_autotune /
 * sc_batch_load_tuning), else a built-in choice; or 1, 2, 4, 8, 16, 32, 64
 * for every graph.  SC_GRAPH_REPLAY records the device work (truncation,
 * initial terms, the persistent launches, the per-graph combination and,
 * for host outputs, the copy to pinned staging) as a hipGraph and replays it
 * while the arguments (and output pointers) stay the same.
 * out: G pointers; out[g] receives m[g] doubles in graph g's input edge
 * order (host memory, or device memory with SC_DEVICE_PTRS).
 * st (may be NULL): L_used / L_min over all graphs, L_capped (edges of all
 * graphs whose automatic length was cut to max_L), block (-1 when mixed),
 * largest lambda* (|lambda_2| of the spectrum for CalTau graphs),
 * prop_launches = persistent launches, prop_ms = their time
 * (SC_TIME_KERNELS, not with SC_GRAPH_REPLAY), total_ms.
 */
int sc_batch_all_edges(sc_batch* b, double eps, const int32_t* L, const sc_options* o,
                       double* const* out, sc_stats* st);

/* The block width every graph would use under o (host int[G]). */
int sc_batch_blocks(const sc_batch* b, const sc_options* o, int32_t* blocks_host);

/*
 * Measure the persistent launch for each size bucket (floor(log2 n),
 * floor(log2 2m/n)) of the batch, on up to 8 of its largest graphs: first
 * every B in {1, ..., 64} whose state fits the LDS (B <= 8 in device slabs
 * otherwise) with the default workgroup size of its LDS class, then the
 * workgroup sizes 256, 512 and 1024 threads for the fastest B (states in
 * LDS); keep the fastest per bucket for o->precision and write the table with
 * all timings as JSON to json_path (NULL: keep it in the handle only).  The
 * computed values do not depend on the choice beyond rounding.
 */
int sc_batch_autotune(sc_batch* b, double eps, const int32_t* L, const sc_options* o,
                      const char* json_path);

/* Load a table written by sc_batch_autotune (replaces the handle's table). */
int sc_batch_load_tuning(sc_batch* b, const char* json_path);

/* Text for an error code; never NULL. */
const char* sc_strerror(int code);

/* Text of the calling thread's last error; never NULL. */
const char* sc_last_error(void);

/* Library version string. */
const char* sc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SC_H */
