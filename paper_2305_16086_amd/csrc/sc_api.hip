// Host side of libsc: graph ingest and validation, the truncation policy,
// the TGT / TGT+ orchestration over source blocks, and lambda* by Lanczos.
//
// Every piece of arithmetic of the method runs in the kernels of
// kernels_tgt.hip / kernels_plus.hip; this file only builds the CSR, sizes
// buffers, chooses launch parameters and sequences the launches.

#include <algorithm>
#include <limits>
#include <chrono>
#include <mutex>
#include <unordered_map>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "sc_host.hpp"

namespace sc {

namespace {
thread_local std::string g_last_error = "no error";
}  // namespace

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

namespace {
std::mutex g_alloc_mu;
std::unordered_map<void*, size_t> g_alloc_sizes;
size_t g_alloc_live = 0;
}  // namespace

hipError_t tracked_malloc_bytes(void** p, size_t bytes) {
  *p = nullptr;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (const char* lim = std::getenv("SC_DEVICE_BYTES_LIMIT")) {
    const double cap = std::atof(lim);
    if (cap > 0.0 && static_cast<double>(g_alloc_live) + static_cast<double>(bytes) > cap)
      return hipErrorOutOfMemory;
  }
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  g_alloc_sizes[*p] = bytes;
  g_alloc_live += bytes;
  return hipSuccess;
}

hipError_t tracked_free(void* p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_alloc_sizes.find(p);
    if (it != g_alloc_sizes.end()) {
      g_alloc_live -= it->second;
      g_alloc_sizes.erase(it);
    }
  }
  return hipFree(p);
}

size_t tracked_live_bytes() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc_live;
}

}  // namespace sc

using sc::dev_alloc;
using sc::dev_free;
using sc::fail;

void sc_graph::release() {
  dev_free(d.rowptr);
  dev_free(d.col);
  dev_free(d.deg);
  dev_free(d.slot_row);
  dev_free(d.slot_half);
  dev_free(d.half_slot);
  dev_free(d.inv_deg_f);
  dev_free(d.inv_deg_d);
  dev_free(d.tasks);
  dev_free(d.wg_tasks);
  dev_free(d.ptasks);
  dev_free(d.giant);
  dev_free(rank_d);
  for (auto& y : Y) {
    if (y) (void)sc::tracked_free(y);
    y = nullptr;
  }
  if (tail_stream) (void)hipStreamDestroy(tail_stream);
  tail_stream = nullptr;
  for (auto& e : pipe_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (partials) (void)sc::tracked_free(partials);
  partials = nullptr;
  dev_free(mask);
  dev_free(anymask);
  dev_free(gacc);
  dev_free(tau_slot);
  dev_free(tau_row);
  dev_free(nr_slot);
  dev_free(spec_lam);
  dev_free(spec_phi);
  dev_free(cs);
  if (colscratch) (void)sc::tracked_free(colscratch);
  colscratch = nullptr;
  dev_free(work);
  dev_free(plan_work);
  dev_free(nz);
  dev_free(walk.chunk_off);
  dev_free(walk.part);
  dev_free(walk.ctl);
  walk.capacity = 0;
  dev_free(out_dev);
  dev_free(tau_out_dev);
  dev_free(nr_out_dev);
  if (rdiag) (void)sc::tracked_free(rdiag);
  if (roff) (void)sc::tracked_free(roff);
  sc::dev_free(src.Q);
  sc::dev_free(src.S);
  sc::dev_free(src.slot_ctl);
  sc::dev_free(src.tilde_row);
  sc::dev_free(src.pos_slot);
  sc::dev_free(src.pos_w);
  sc::dev_free(src.nr_pos);
  sc::dev_free(src.chunk_off);
  sc::dev_free(src.part);
  sc::dev_free(src.ctl);
  sc::dev_free(src.totals);
  sc::dev_free(src.list);
  sc::dev_free(src.hoff);
  src = SourceBuffers{};
  rdiag = roff = nullptr;
  rbytes = 0;
  dev_free(feat);
  dev_free(zpred);
  dev_free(cl_s0);
  dev_free(fb);
  dev_free(block_flag);
  for (auto& e : events) (void)hipEventDestroy(e);
  events.clear();
}

// ====================================================================== graph build

int sc::build_host_csr(int64_t n, int64_t m, const int64_t* u, const int64_t* v, unsigned flags,
                       HostCSR& out) {
  if (!u || !v) return fail(SC_EINVAL, "edge arrays are NULL");
  if (n < 2 || m < 1) return fail(SC_EINVAL, "need n >= 2 and m >= 1");
  if (n >= (1ll << 31) || 2 * m >= (1ll << 31))
    return fail(SC_EINVAL, "n and 2m must be below 2^31");
  for (int64_t e = 0; e < m; ++e) {
    if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n)
      return fail(SC_EINVAL, "edge " + std::to_string(e) + " has a node id out of [0, n)");
    if (u[e] == v[e]) return fail(SC_ESELFLOOP, "edge " + std::to_string(e) + " is a self-loop");
  }
  const int32_t N = static_cast<int32_t>(n);
  const int64_t H = 2 * m;
  std::vector<int32_t> hsrc, hdst;
  std::vector<int32_t> order, tmp;
  try {
    hsrc.resize(H);
    hdst.resize(H);
    order.resize(H);
    tmp.resize(H);
  } catch (const std::bad_alloc&) {
    return fail(SC_ENOMEM, "host allocation failed");
  }
  for (int64_t e = 0; e < m; ++e) {
    hsrc[e] = static_cast<int32_t>(u[e]);
    hdst[e] = static_cast<int32_t>(v[e]);
    hsrc[e + m] = static_cast<int32_t>(v[e]);
    hdst[e + m] = static_cast<int32_t>(u[e]);
  }
  // two stable counting sorts: by neighbour, then by source -> rows sorted by neighbour
  std::vector<int64_t> cnt(static_cast<size_t>(N) + 1);
  auto counting_sort = [&](const std::vector<int32_t>& key, const std::vector<int32_t>& in,
                           std::vector<int32_t>& outv) {
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t i = 0; i < H; ++i) ++cnt[key[in[i]] + 1];
    for (int32_t x = 0; x < N; ++x) cnt[x + 1] += cnt[x];
    for (int64_t i = 0; i < H; ++i) outv[cnt[key[in[i]]]++] = in[i];
  };
  std::iota(order.begin(), order.end(), 0);
  counting_sort(hdst, order, tmp);
  counting_sort(hsrc, tmp, order);

  // rows, duplicates
  std::vector<int32_t> rowptr(N + 1, 0), col, slot_half, half_slot(H);
  col.reserve(H);
  slot_half.reserve(H);
  int64_t i = 0;
  for (int32_t x = 0; x < N; ++x) {
    rowptr[x] = static_cast<int32_t>(col.size());
    while (i < H && hsrc[order[i]] == x) {
      const int32_t h = order[i];
      if (!col.empty() && static_cast<int64_t>(col.size()) > rowptr[x] && col.back() == hdst[h]) {
        if (!(flags & SC_MERGE_DUPS)) {
          const int64_t e = h % m;
          return fail(SC_EDUP, "edge " + std::to_string(e) + " repeats an earlier edge");
        }
        half_slot[h] = static_cast<int32_t>(col.size()) - 1;
      } else {
        half_slot[h] = static_cast<int32_t>(col.size());
        col.push_back(hdst[h]);
        slot_half.push_back(h);
      }
      ++i;
    }
  }
  rowptr[N] = static_cast<int32_t>(col.size());
  const int64_t S = static_cast<int64_t>(col.size());
  std::vector<int32_t> deg(N), slot_row(S);
  for (int32_t x = 0; x < N; ++x) {
    deg[x] = rowptr[x + 1] - rowptr[x];
    for (int32_t k = rowptr[x]; k < rowptr[x + 1]; ++k) slot_row[k] = x;
  }

  // connected and non-bipartite (BFS 2-colouring)
  {
    std::vector<int8_t> colour(N, -1);
    std::vector<int32_t> queue;
    queue.reserve(N);
    queue.push_back(0);
    colour[0] = 0;
    bool odd_cycle = false;
    for (size_t qh = 0; qh < queue.size(); ++qh) {
      const int32_t x = queue[qh];
      for (int32_t k = rowptr[x]; k < rowptr[x + 1]; ++k) {
        const int32_t y = col[k];
        if (colour[y] < 0) {
          colour[y] = static_cast<int8_t>(1 - colour[x]);
          queue.push_back(y);
        } else if (colour[y] == colour[x]) {
          odd_cycle = true;
        }
      }
    }
    if (static_cast<int64_t>(queue.size()) != N)
      return fail(SC_EDISCONNECTED, "graph is not connected");
    if (!odd_cycle) return fail(SC_EBIPARTITE, "graph is bipartite");
  }

  // gather tasks: workgroup tasks (heavy rows, giant-row chunks) first, then
  // wave tasks for the light rows
  std::vector<sc::Task> tasks, wg_tasks;
  std::vector<sc::HeavyRow> giant;
  int32_t nparts = 0;
  for (int32_t x = 0; x < N; ++x) {
    if (deg[x] > sc::kGiant) {
      sc::HeavyRow hr{x, nparts, 0, 0};
      for (int32_t b = rowptr[x]; b < rowptr[x + 1]; b += sc::kGiantChunk) {
        wg_tasks.push_back({x, b, std::min(b + sc::kGiantChunk, rowptr[x + 1]), nparts++});
        ++hr.nparts;
      }
      giant.push_back(hr);
    } else if (deg[x] > sc::kChunk) {
      wg_tasks.push_back({x, rowptr[x], rowptr[x + 1], -1});
    } else {
      tasks.push_back({x, rowptr[x], rowptr[x + 1], -1});
    }
  }
  // runs of consecutive light rows, at most 64 slots per run (rows with more
  // than 64 slots stay alone)
  std::vector<sc::Task> ptasks;
  for (int32_t x = 0; x < N;) {
    if (deg[x] > sc::kChunk) {
      ++x;
      continue;
    }
    int32_t y = x + 1;
    if (deg[x] <= 64)
      while (y < N && deg[y] <= sc::kChunk && rowptr[y + 1] - rowptr[x] <= 64) ++y;
    ptasks.push_back({x, rowptr[x], rowptr[y], y - x});
    x = y;
  }

  std::vector<float> inv_f(N);
  std::vector<double> inv_d(N);
  for (int32_t x = 0; x < N; ++x) {
    inv_f[x] = 1.0f / static_cast<float>(deg[x]);
    inv_d[x] = 1.0 / static_cast<double>(deg[x]);
  }
  out.n = N;
  out.m = m;
  out.nslots = S;
  out.rowptr = std::move(rowptr);
  out.col = std::move(col);
  out.deg = std::move(deg);
  out.slot_row = std::move(slot_row);
  out.slot_half = std::move(slot_half);
  out.half_slot = std::move(half_slot);
  out.tasks = std::move(tasks);
  out.ptasks = std::move(ptasks);
  out.wg_tasks = std::move(wg_tasks);
  out.giant = std::move(giant);
  out.nparts = nparts;
  out.inv_f = std::move(inv_f);
  out.inv_d = std::move(inv_d);
  return SC_OK;
}

int sc::upload_csr(const HostCSR& h, DeviceGraph& d) {
  d.n = h.n;
  d.m = h.m;
  d.nslots = h.nslots;
  d.ntasks = static_cast<int32_t>(h.tasks.size());
  d.nptasks = static_cast<int32_t>(h.ptasks.size());
  d.nwg = static_cast<int32_t>(h.wg_tasks.size());
  d.ngiant = static_cast<int32_t>(h.giant.size());
  d.nparts = h.nparts;
  auto up = [&](auto** dst, const auto& src) -> hipError_t {
    hipError_t e = dev_alloc(dst, src.size());
    if (e != hipSuccess) return e;
    if (src.empty()) return hipSuccess;
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(src[0]), hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(&d.rowptr, h.rowptr);
  if (e == hipSuccess) e = up(&d.col, h.col);
  if (e == hipSuccess) e = up(&d.deg, h.deg);
  if (e == hipSuccess) e = up(&d.slot_row, h.slot_row);
  if (e == hipSuccess) e = up(&d.slot_half, h.slot_half);
  if (e == hipSuccess) e = up(&d.half_slot, h.half_slot);
  if (e == hipSuccess) e = up(&d.inv_deg_f, h.inv_f);
  if (e == hipSuccess) e = up(&d.inv_deg_d, h.inv_d);
  if (e == hipSuccess) e = up(&d.tasks, h.tasks);
  if (e == hipSuccess) e = up(&d.wg_tasks, h.wg_tasks);
  if (e == hipSuccess) e = up(&d.ptasks, h.ptasks);
  if (e == hipSuccess) e = up(&d.giant, h.giant);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP,
                std::string("graph upload: ") + hipGetErrorString(e));
  return SC_OK;
}

int sc::graph_from_csr(HostCSR& h, sc_graph** out) {
  sc_graph* g = new (std::nothrow) sc_graph();
  if (!g) return fail(SC_ENOMEM, "host allocation failed");
  (void)hipGetDevice(&g->device);
  const int rc = sc::upload_csr(h, g->d);
  if (rc) {
    g->release();
    delete g;
    return rc;
  }
  g->rowptr_h = std::move(h.rowptr);
  g->deg_h = std::move(h.deg);
  *out = g;
  return SC_OK;
}

namespace {

// Breadth-first visiting order of the nodes (ids valid, n >= 1): started at
// the highest-degree node (lowest id among equals), each node's neighbours
// taken in ascending id; unreached nodes follow in ascending id.
void bfs_order(int64_t n, int64_t m, const int64_t* u, const int64_t* v, std::vector<int32_t>& label) {
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    ++off[u[e] + 1];
    ++off[v[e] + 1];
  }
  for (int64_t x = 0; x < n; ++x) off[x + 1] += off[x];
  std::vector<int32_t> adj(static_cast<size_t>(2 * m));
  {
    // rows in edge order, then transposed: walking the rows in ascending x and
    // appending x to each neighbour's row leaves every row in ascending id
    std::vector<int32_t> first(static_cast<size_t>(2 * m));
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t e = 0; e < m; ++e) {
      first[pos[u[e]]++] = static_cast<int32_t>(v[e]);
      first[pos[v[e]]++] = static_cast<int32_t>(u[e]);
    }
    pos.assign(off.begin(), off.end() - 1);
    for (int64_t x = 0; x < n; ++x)
      for (int64_t k = off[x]; k < off[x + 1]; ++k) adj[pos[first[k]]++] = static_cast<int32_t>(x);
  }
  int64_t s = 0;
  for (int64_t x = 1; x < n; ++x)
    if (off[x + 1] - off[x] > off[s + 1] - off[s]) s = x;
  std::vector<unsigned char> seen(n, 0);
  label.clear();
  label.reserve(n);
  seen[s] = 1;
  label.push_back(static_cast<int32_t>(s));
  for (size_t q = 0; q < label.size(); ++q) {
    const int32_t x = label[q];
    for (int64_t k = off[x]; k < off[x + 1]; ++k) {
      const int32_t y = adj[k];
      if (!seen[y]) {
        seen[y] = 1;
        label.push_back(y);
      }
    }
  }
  for (int64_t x = 0; x < n; ++x)
    if (!seen[x]) label.push_back(static_cast<int32_t>(x));
}

}  // namespace

extern "C" int sc_build_graph(int64_t n, int64_t m, const int64_t* u, const int64_t* v,
                              unsigned flags, sc_graph** out) {
  if (!out) return fail(SC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  const unsigned order_flags = flags & (SC_DEGREE_ORDER | SC_BFS_ORDER);
  if (order_flags == (SC_DEGREE_ORDER | SC_BFS_ORDER))
    return fail(SC_EINVAL, "SC_DEGREE_ORDER and SC_BFS_ORDER exclude each other");
  const unsigned build_flags = flags & ~(SC_DEGREE_ORDER | SC_BFS_ORDER);
  sc::HostCSR h;
  bool ranges_ok = order_flags && u && v && n >= 2 && n < (1ll << 31) && m >= 1 &&
                   2 * m < (1ll << 31);
  for (int64_t e = 0; ranges_ok && e < m; ++e)
    ranges_ok = u[e] >= 0 && u[e] < n && v[e] >= 0 && v[e] < n;
  if (!ranges_ok) {
    // the caller's ids (or input errors, reported by the build)
    const int rc = sc::build_host_csr(n, m, u, v, build_flags, h);
    if (rc) return rc;
    return sc::graph_from_csr(h, out);
  }
  // renumber (stored node y is the caller's label[y]); the edge order is kept
  std::vector<int32_t> rank, label;
  std::vector<int64_t> u2, v2;
  try {
    if (order_flags == SC_BFS_ORDER) {
      bfs_order(n, m, u, v, label);
    } else {   // descending degree, ties by ascending id
      std::vector<int64_t> deg(n, 0);
      for (int64_t e = 0; e < m; ++e) {
        ++deg[u[e]];
        ++deg[v[e]];
      }
      label.resize(n);
      std::iota(label.begin(), label.end(), 0);
      std::stable_sort(label.begin(), label.end(),
                       [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
    }
    rank.resize(n);
    for (int64_t y = 0; y < n; ++y) rank[label[y]] = static_cast<int32_t>(y);
    u2.resize(m);
    v2.resize(m);
    for (int64_t e = 0; e < m; ++e) {
      u2[e] = rank[u[e]];
      v2[e] = rank[v[e]];
    }
  } catch (const std::bad_alloc&) {
    return fail(SC_ENOMEM, "host allocation failed");
  }
  int rc = sc::build_host_csr(n, m, u2.data(), v2.data(), build_flags, h);
  if (rc) return rc;
  u2 = std::vector<int64_t>();
  v2 = std::vector<int64_t>();
  sc_graph* g = nullptr;
  rc = sc::graph_from_csr(h, &g);
  if (rc) return rc;
  const hipError_t e = sc::dev_alloc(&g->rank_d, static_cast<size_t>(n));
  const hipError_t e2 = e == hipSuccess ? hipMemcpy(g->rank_d, rank.data(), n * sizeof(int32_t),
                                                    hipMemcpyHostToDevice)
                                        : e;
  if (e2 != hipSuccess) {
    sc_free_graph(g);
    return fail(e2 == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP,
                std::string("graph upload: ") + hipGetErrorString(e2));
  }
  g->rank_h = std::move(rank);
  g->label_h = std::move(label);
  *out = g;
  return SC_OK;
}

extern "C" int sc_graph_size(const sc_graph* g, int64_t* n, int64_t* m) {
  if (!g) return fail(SC_EINVAL, "graph is NULL");
  if (n) *n = g->d.n;
  if (m) *m = g->d.m;
  return SC_OK;
}

extern "C" void sc_free_graph(sc_graph* g) {
  if (!g) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  g->release();
  (void)hipSetDevice(cur);
  delete g;
}

// ====================================================================== lambda* by Lanczos

namespace {

__global__ void k_scale_into(const double* __restrict__ w, double s, double* __restrict__ dst,
                             int64_t n) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x < n) dst[x] = w[x] * s;
}

// Lanczos start for N = D^-1/2 A D^-1/2: column 0 of V holds the top
// eigenvector sqrt(d / 2m) (eigenvalue 1, deflated by the re-orthogonalisation),
// column 1 a fixed pseudo-random unit vector orthogonal to it; sid = 1/sqrt(d).
hipError_t lanczos_start(const sc::DeviceGraph& dg, const int32_t* deg_host, double* V, int64_t ld,
                         double* sid, hipStream_t st, uint64_t seed = 0) {
  const int64_t n = dg.n;
  std::vector<double> hv(n), sidh(n);
  const double two_m = static_cast<double>(dg.nslots);
  for (int64_t x = 0; x < n; ++x) {
    hv[x] = std::sqrt(deg_host[x] / two_m);
    sidh[x] = 1.0 / std::sqrt(static_cast<double>(deg_host[x]));
  }
  std::vector<double> v0(n);
  uint64_t z = 0x9E3779B97F4A7C15ull * (2 * seed + 1);
  double dot = 0.0;
  for (int64_t x = 0; x < n; ++x) {
    z += 0x9E3779B97F4A7C15ull;
    uint64_t r = z;
    r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
    r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
    r ^= r >> 31;
    v0[x] = (static_cast<double>(r >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
    dot += v0[x] * hv[x];
  }
  double nrm = 0.0;
  for (int64_t x = 0; x < n; ++x) {
    v0[x] -= dot * hv[x];
    nrm += v0[x] * v0[x];
  }
  nrm = std::sqrt(nrm);
  for (int64_t x = 0; x < n; ++x) v0[x] /= nrm;
  hipError_t e = hipMemcpy(V, hv.data(), n * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(V + ld, v0.data(), n * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(sid, sidh.data(), n * sizeof(double), hipMemcpyHostToDevice);
  (void)st;
  return e;
}

// Eigenvalues of the symmetric tridiagonal matrix (diagonal d[0..k), off-diagonal
// e[0..k-1)) by implicit QL iterations with Wilkinson-type shifts (Wilkinson and
// Reinsch; Golub and Van Loan, implicit symmetric tridiagonal QR).  d receives
// the eigenvalues (unordered).  zt (k x k), if given, receives the eigenvectors
// as rows (zt[c * k + i] = component i of the vector of d[c]); zlast, if given,
// their last components only.
// Returns false if an eigenvalue needs more than 60 iterations.
bool tridiag_eigen(std::vector<double>& d, std::vector<double> e, std::vector<double>* zt,
                   std::vector<double>* zlast) {
  const int k = static_cast<int>(d.size());
  e.resize(k, 0.0);
  e[k - 1] = 0.0;
  if (zt) {
    zt->assign(static_cast<size_t>(k) * k, 0.0);
    for (int i = 0; i < k; ++i) (*zt)[static_cast<size_t>(i) * k + i] = 1.0;
  }
  if (zlast) {
    zlast->assign(k, 0.0);
    (*zlast)[k - 1] = 1.0;
  }
  const double ulp = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < k; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < k - 1; ++m)   // first negligible off-diagonal at or after l
        if (std::fabs(e[m]) <= ulp * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
      if (m == l) break;
      if (iter == 60) return false;
      // shift from the leading 2 x 2 block, then chase the bulge from m up to l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double sn = 1.0, cs = 1.0, p = 0.0;
      bool split = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = sn * e[i];
        const double b = cs * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {   // the matrix splits: deflate and restart from l
          d[i + 1] -= p;
          e[m] = 0.0;
          split = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * sn + 2.0 * cs * b;
        p = sn * r;
        d[i + 1] = g + p;
        g = cs * r - b;
        if (zt) {   // rotate vectors i and i + 1 (two contiguous rows)
          double* ri = zt->data() + static_cast<size_t>(i) * k;
          double* rj = ri + k;
          for (int q = 0; q < k; ++q) {
            const double t = rj[q];
            rj[q] = sn * ri[q] + cs * t;
            ri[q] = cs * ri[q] - sn * t;
          }
        }
        if (zlast) {
          const double t = (*zlast)[i + 1];
          (*zlast)[i + 1] = sn * (*zlast)[i] + cs * t;
          (*zlast)[i] = cs * (*zlast)[i] - sn * t;
        }
      }
      if (split) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

// extreme Ritz estimate: max over the two ends of |theta| + residual, where the
// residual of a Ritz pair is |beta_last * (last component of its vector)|
// (eigenvalues and last components by implicit QL, O(k^2) per check)
double ritz_bound(const std::vector<double>& alpha, const std::vector<double>& beta, int k,
                  double beta_last, double* worst_res) {
  std::vector<double> d(alpha.begin(), alpha.begin() + k), zl;
  std::vector<double> e(beta.begin(), beta.begin() + std::min<size_t>(beta.size(), k));
  if (!tridiag_eigen(d, e, nullptr, &zl)) {
    *worst_res = 1.0;   // no answer: report as unconverged
    return 1.0;
  }
  int imax = 0, imin = 0;
  for (int i = 1; i < k; ++i) {
    if (d[i] > d[imax]) imax = i;
    if (d[i] < d[imin]) imin = i;
  }
  const double rmax = std::fabs(beta_last * zl[imax]);
  const double rmin = std::fabs(beta_last * zl[imin]);
  *worst_res = std::max(rmax, rmin);
  return std::max(std::fabs(d[imax]) + rmax, std::fabs(d[imin]) + rmin);
}

}  // namespace

int sc::compute_lambda_star(sc_graph* g, hipStream_t st, double* out) {
  // two Lanczos runs from independent start vectors; the larger estimate is kept
  // (a start vector nearly orthogonal to the extreme eigenvector would make one
  // run under-estimate), converged only if both runs passed the residual test
  double a = 0.0, b = 0.0;
  int ca = 0, cb = 0;
  int rc = lanczos_lambda_star(g->d, g->deg_h.data(), st, &a, &ca, 0);
  if (rc != SC_OK) return rc;
  rc = lanczos_lambda_star(g->d, g->deg_h.data(), st, &b, &cb, 1);
  if (rc != SC_OK) return rc;
  *out = std::max(a, b);
  g->lambda_converged = (ca && cb) ? 1 : 0;
  return SC_OK;
}

int sc::lanczos_lambda_star(const DeviceGraph& dg, const int32_t* deg_host, hipStream_t st,
                            double* out, int* converged, uint64_t seed) {
  using namespace sc;
  const int64_t n = dg.n;
  // up to 600 steps, the basis held to 4 GiB
  const int64_t kcap = std::max<int64_t>(40, (int64_t(1) << 29) / std::max<int64_t>(n, 1) - 2);
  const int kmax = static_cast<int>(std::min<int64_t>({n - 1, 600, kcap}));
  if (converged) *converged = 0;
  const int64_t ld = n;
  double *V = nullptr, *w = nullptr, *h = nullptr, *sid = nullptr;
  auto cleanup = [&]() {
    dev_free(V);
    dev_free(w);
    dev_free(h);
    dev_free(sid);
  };
  const ScopeExit<decltype(cleanup)> guard{cleanup};   // also on early error returns
  hipError_t e = dev_alloc(&V, static_cast<size_t>(kmax + 2) * ld);
  if (e == hipSuccess) e = dev_alloc(&w, n);
  if (e == hipSuccess) e = dev_alloc(&h, kmax + 2);
  if (e == hipSuccess) e = dev_alloc(&sid, n);
  if (e != hipSuccess) {
    cleanup();
    return fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP, "lanczos allocation failed");
  }
  HIP_TRY(lanczos_start(dg, deg_host, V, ld, sid, st, seed));

  std::vector<double> alpha, beta, hh(kmax + 2);
  double result = -1.0;
  const unsigned grid = static_cast<unsigned>((n + 255) / 256);
  for (int j = 1; j <= kmax; ++j) {
    const double* vj = V + static_cast<size_t>(j) * ld;
    HIP_TRY(sc::launch_nmat_spmv(dg, sid, vj, w, st));
    double a_j = 0.0;
    for (int pass = 0; pass < 2; ++pass) {   // full re-orthogonalisation, twice
      HIP_TRY(sc::launch_multi_dot(V, j + 1, ld, w, n, h, st));
      HIP_TRY(hipMemcpyAsync(hh.data(), h, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      a_j += hh[j];
      HIP_TRY(sc::launch_multi_axpy(V, j + 1, ld, h, w, n, st));
    }
    HIP_TRY(sc::launch_multi_dot(w, 1, ld, w, n, h, st));
    HIP_TRY(hipMemcpyAsync(hh.data(), h, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double b_j = std::sqrt(std::max(hh[0], 0.0));
    alpha.push_back(a_j);
    const bool exhausted = b_j < 1e-12 || j == kmax;
    if ((j % 20 == 0) || exhausted) {
      double res = 0.0;
      const double bound = ritz_bound(alpha, beta, j, exhausted ? 0.0 : b_j, &res);
      result = bound;
      if (b_j < 1e-12 || res < 1e-9) {   // Krylov space exhausted, or both ends converged
        if (converged) *converged = 1;
        break;
      }
      if (exhausted) break;
    }
    beta.push_back(b_j);
    k_scale_into<<<grid, 256, 0, st>>>(w, 1.0 / b_j, V + static_cast<size_t>(j + 1) * ld, n);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  cleanup();
  if (!(result > 0.0) || !(result < 1.0))
    return fail(SC_EINVAL, "lambda* estimate outside (0, 1): " + std::to_string(result) +
                               " (graph bipartite or too small?)");
  *out = result;
  return SC_OK;
}

int sc::graph_lambda_star(sc_graph* g, hipStream_t st, double* lam) {
  if (g->lambda_star <= 0.0) {
    double v = 0.0;
    const int rc = compute_lambda_star(g, st, &v);
    if (rc != SC_OK) return rc;
    g->lambda_star = v;
  }
  *lam = g->lambda_star;
  return SC_OK;
}

// Lanczos with full re-orthogonalisation (twice) on N = D^-1/2 A D^-1/2 with
// the trivial eigenvector deflated.  Every 25 steps the Ritz values of the
// tridiagonal matrix are checked: the run stops when the omega - 1 of largest
// |theta| have residual estimates |beta_j y_j| <= tol (or after max_iter steps,
// or when the Krylov space is exhausted).  The longest prefix (|theta|
// descending) of pairs within tol is kept, with the trivial pair in front.
int sc::lanczos_spectrum(sc_graph* g, int omega, int max_iter, double tol, hipStream_t st,
                         int* kept, double* worst) {
  const sc::DeviceGraph& dg = g->d;
  const int64_t n = dg.n;
  const int64_t ld = n;
  // the basis is held whole: at most ~16 GiB of it
  const int64_t cap = std::max<int64_t>(omega + 8, (int64_t(16) << 30) / (8 * n) - 2);
  const int kmax = static_cast<int>(std::min<int64_t>({n - 1, static_cast<int64_t>(max_iter), cap}));
  double *V = nullptr, *w = nullptr, *h = nullptr, *sid = nullptr, *Yd = nullptr;
  auto cleanup = [&]() {
    dev_free(V);
    dev_free(w);
    dev_free(h);
    dev_free(sid);
    dev_free(Yd);
  };
  const ScopeExit<decltype(cleanup)> guard{cleanup};   // also on early error returns
  hipError_t e = dev_alloc(&V, static_cast<size_t>(kmax + 2) * ld);
  if (e == hipSuccess) e = dev_alloc(&w, n);
  if (e == hipSuccess) e = dev_alloc(&h, kmax + 2);
  if (e == hipSuccess) e = dev_alloc(&sid, n);
  if (e == hipSuccess) e = lanczos_start(dg, g->deg_h.data(), V, ld, sid, st);
  if (e != hipSuccess) {
    cleanup();
    return fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP, "spectrum: allocation failed");
  }
  const int want = omega - 1;
  // Ritz pairs ordered by |theta| descending (ties: theta descending)
  auto order_of = [](const std::vector<double>& th) {
    std::vector<int> idx(th.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = static_cast<int>(i);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) {
      const double fa = std::fabs(th[a]), fb = std::fabs(th[b]);
      return fa > fb || (fa == fb && th[a] > th[b]);
    });
    return idx;
  };
  std::vector<double> alpha, beta, hh(kmax + 2);
  const unsigned grid = static_cast<unsigned>((n + 255) / 256);
  int steps = 0;
  double b_last = 0.0;
  for (int j = 1; j <= kmax; ++j) {
    const double* vj = V + static_cast<size_t>(j) * ld;
    HIP_TRY(sc::launch_nmat_spmv(dg, sid, vj, w, st));
    double a_j = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      HIP_TRY(sc::launch_multi_dot(V, j + 1, ld, w, n, h, st));
      HIP_TRY(hipMemcpyAsync(hh.data(), h, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      a_j += hh[j];
      HIP_TRY(sc::launch_multi_axpy(V, j + 1, ld, h, w, n, st));
    }
    HIP_TRY(sc::launch_multi_dot(w, 1, ld, w, n, h, st));
    HIP_TRY(hipMemcpyAsync(hh.data(), h, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double b_j = std::sqrt(std::max(hh[0], 0.0));
    alpha.push_back(a_j);
    steps = j;
    b_last = b_j;
    const bool exhausted = b_j < 1e-12 || j == kmax;
    if (exhausted) break;
    if (j % 25 == 0 && j >= want) {
      std::vector<double> th = alpha, zl;
      if (!tridiag_eigen(th, beta, nullptr, &zl)) break;
      const std::vector<int> idx = order_of(th);
      bool done = true;
      for (int c = 0; c < want && done; ++c) done = std::fabs(b_j * zl[idx[c]]) <= tol;
      if (done) break;
    }
    beta.push_back(b_j);
    k_scale_into<<<grid, 256, 0, st>>>(w, 1.0 / b_j, V + static_cast<size_t>(j + 1) * ld, n);
    HIP_TRY(hipGetLastError());
  }
  // Ritz pairs of the final tridiagonal matrix
  std::vector<double> th = alpha, Z;
  beta.resize(steps - 1);
  if (!tridiag_eigen(th, beta, &Z, nullptr)) {
    cleanup();
    return fail(SC_EINVAL, "spectrum: tridiagonal eigenvalues did not converge");
  }
  const std::vector<int> idx = order_of(th);
  const bool exact = b_last < 1e-12;   // invariant subspace: the Ritz pairs are eigenpairs
  int p = 0;
  double wres = 0.0;
  while (p < want && p < steps) {
    const double r = exact ? 0.0 : std::fabs(b_last * Z[static_cast<size_t>(idx[p]) * steps + steps - 1]);
    if (r > tol) break;
    wres = std::max(wres, r);
    ++p;
  }
  if (p == 0) {
    cleanup();
    return fail(SC_EINVAL, "spectrum: no Ritz pair reached the tolerance (raise max_iter)");
  }
  const int om = p + 1;
  const int p32 = (p + kRitzCols - 1) / kRitzCols * kRitzCols;
  std::vector<double> Y(static_cast<size_t>(steps) * p32, 0.0);
  for (int i = 0; i < steps; ++i)
    for (int c = 0; c < p; ++c) Y[static_cast<size_t>(i) * p32 + c] = Z[static_cast<size_t>(idx[c]) * steps + i];
  std::vector<double> lam(om);
  lam[0] = 1.0;
  for (int c = 0; c < p; ++c) lam[1 + c] = th[idx[c]];
  double* lam_d = nullptr;
  double* phi_d = nullptr;
  e = dev_alloc(&Yd, Y.size());
  if (e == hipSuccess) e = dev_alloc(&lam_d, om);
  if (e == hipSuccess) e = dev_alloc(&phi_d, static_cast<size_t>(n) * om);
  if (e == hipSuccess) e = hipMemcpy(Yd, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(lam_d, lam.data(), om * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sc::launch_ritz(n, ld, V, steps, Yd, p32, p, om, phi_d, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) {
    dev_free(lam_d);
    dev_free(phi_d);
    return fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP,
                std::string("spectrum: ") + hipGetErrorString(e));
  }
  dev_free(g->spec_lam);
  dev_free(g->spec_phi);
  g->spec_lam = lam_d;
  g->spec_phi = phi_d;
  g->spec_omega = om;
  g->spec_lam_h = lam;
  ++g->spec_version;
  *kept = om;
  *worst = wres;
  return SC_OK;
}

extern "C" int sc_compute_spectrum(sc_graph* g, int omega, int max_iter, double tol,
                                   int* omega_kept, double* max_residual) {
  if (!g) return fail(SC_EINVAL, "graph is NULL");
  if (omega < 2 || omega > sc::kMaxOmega) return fail(SC_EINVAL, "omega must lie in [2, 256]");
  if (omega > g->d.n) omega = static_cast<int>(g->d.n);
  if (max_iter <= 0) max_iter = 2048;
  if (!(tol > 0.0)) tol = 1e-8;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != g->device) (void)hipSetDevice(g->device);
  int kept = 0;
  double worst = 0.0;
  const int rc = sc::lanczos_spectrum(g, omega, max_iter, tol, nullptr, &kept, &worst);
  if (cur != g->device) (void)hipSetDevice(cur);
  if (rc) return rc;
  if (omega_kept) *omega_kept = kept;
  if (max_residual) *max_residual = worst;
  return SC_OK;
}

extern "C" int sc_set_spectrum(sc_graph* g, int omega, const double* lambda, const double* phi) {
  if (!g || !lambda || !phi) return fail(SC_EINVAL, "NULL argument");
  if (omega < 2 || omega > sc::kMaxOmega || omega > g->d.n)
    return fail(SC_EINVAL, "omega must lie in [2, min(n, 256)]");
  if (std::fabs(lambda[0] - 1.0) > 1e-8)
    return fail(SC_EINVAL, "lambda[0] must be the trivial eigenvalue 1");
  for (int k = 1; k < omega; ++k) {
    if (!(std::fabs(lambda[k]) < 1.0))
      return fail(SC_EINVAL, "non-trivial eigenvalues must lie in (-1, 1)");
    if (k >= 2 && std::fabs(lambda[k]) > std::fabs(lambda[k - 1]) * (1.0 + 1e-12))
      return fail(SC_EINVAL, "eigenvalues must be ordered by |lambda| descending");
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != g->device) (void)hipSetDevice(g->device);
  const size_t cells = static_cast<size_t>(g->d.n) * omega;
  std::vector<double> stored;   // rows in the stored node order (renumbered graphs)
  if (!g->rank_h.empty()) {
    try {
      stored.resize(cells);
    } catch (const std::bad_alloc&) {
      if (cur != g->device) (void)hipSetDevice(cur);
      return fail(SC_ENOMEM, "host allocation failed");
    }
    for (int64_t x = 0; x < g->d.n; ++x)
      std::memcpy(stored.data() + static_cast<size_t>(g->rank_h[x]) * omega,
                  phi + static_cast<size_t>(x) * omega, omega * sizeof(double));
  }
  const double* phi_src = stored.empty() ? phi : stored.data();
  double* lam_d = nullptr;
  double* phi_d = nullptr;
  hipError_t e = sc::dev_alloc(&lam_d, omega);
  if (e == hipSuccess) e = sc::dev_alloc(&phi_d, cells);
  if (e == hipSuccess) e = hipMemcpy(lam_d, lambda, omega * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(phi_d, phi_src, cells * sizeof(double), hipMemcpyHostToDevice);
  if (cur != g->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    sc::dev_free(lam_d);
    sc::dev_free(phi_d);
    return fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP,
                std::string("set spectrum: ") + hipGetErrorString(e));
  }
  sc::dev_free(g->spec_lam);
  sc::dev_free(g->spec_phi);
  g->spec_lam = lam_d;
  g->spec_phi = phi_d;
  g->spec_omega = omega;
  g->spec_lam_h.assign(lambda, lambda + omega);
  ++g->spec_version;
  return SC_OK;
}

extern "C" int sc_get_spectrum(const sc_graph* g, int* omega, double* lambda, double* phi) {
  if (!g || !omega) return fail(SC_EINVAL, "NULL argument");
  *omega = g->spec_omega;
  if (g->spec_omega == 0) return SC_OK;
  if (lambda) std::memcpy(lambda, g->spec_lam_h.data(), g->spec_omega * sizeof(double));
  if (phi) {
    const int omega_s = g->spec_omega;
    const size_t cells = static_cast<size_t>(g->d.n) * omega_s;
    std::vector<double> stored;   // rows in the stored node order (renumbered graphs)
    if (!g->rank_h.empty()) {
      try {
        stored.resize(cells);
      } catch (const std::bad_alloc&) {
        return fail(SC_ENOMEM, "host allocation failed");
      }
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    const hipError_t e = hipMemcpy(stored.empty() ? phi : stored.data(), g->spec_phi,
                                   cells * sizeof(double), hipMemcpyDeviceToHost);
    if (cur != g->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(SC_EHIP, std::string("get spectrum: ") + hipGetErrorString(e));
    for (int64_t x = 0; !stored.empty() && x < g->d.n; ++x)
      std::memcpy(phi + static_cast<size_t>(x) * omega_s,
                  stored.data() + static_cast<size_t>(g->rank_h[x]) * omega_s,
                  omega_s * sizeof(double));
  }
  return SC_OK;
}

extern "C" int sc_lambda_star(sc_graph* g, double* lam) {
  if (!g || !lam) return fail(SC_EINVAL, "NULL argument");
  return sc::graph_lambda_star(g, nullptr, lam);
}

extern "C" int sc_walk_trace(sc_graph* g, int32_t i, int32_t j, int64_t r, int32_t length,
                             uint64_t seed, int32_t* nodes_host) {
  if (!g || (!nodes_host && length > 0)) return fail(SC_EINVAL, "NULL argument");
  if (i < 0 || j < 0 || i >= g->d.n || j >= g->d.n) return fail(SC_EINVAL, "node id out of range");
  if (r < 0 || r > 0xFFFFFFFFll) return fail(SC_EINVAL, "walk index must lie in [0, 2^32)");
  if (length < 0 || length > (1 << 20)) return fail(SC_EINVAL, "length must lie in [0, 2^20]");
  if (length == 0) return SC_OK;
  const bool renumbered = !g->rank_h.empty();
  if (renumbered) {   // the stored nodes
    i = g->rank_h[i];
    j = g->rank_h[j];
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != g->device) (void)hipSetDevice(g->device);
  int32_t* d = nullptr;
  int rc = SC_OK;
  {
    auto body = [&]() -> int {
      HIP_TRY(sc::dev_alloc(&d, 2 * static_cast<size_t>(length)));
      HIP_TRY(sc::launch_walk_trace(g->d, i, j, static_cast<uint32_t>(r), length, seed, d, nullptr));
      HIP_TRY(hipMemcpy(nodes_host, d, 2 * static_cast<size_t>(length) * sizeof(int32_t),
                        hipMemcpyDeviceToHost));
      return SC_OK;
    };
    rc = body();
  }
  sc::dev_free(d);
  if (cur != g->device) (void)hipSetDevice(cur);
  if (rc == SC_OK && renumbered)   // back to the caller's ids
    for (int64_t t = 0; t < 2 * static_cast<int64_t>(length); ++t) nodes_host[t] = g->label_h[nodes_host[t]];
  return rc;
}

// ====================================================================== all-edge SC

extern "C" void sc_default_options(sc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = SC_TGT;
  o->precision = 0;
  o->block = 0;
  o->gamma = 10;
  o->delta = 0.0;
  o->seed = 0x5C5Cull;
  o->tilde_tau = -1;
  o->max_L = 255;
  o->lambda_star = 0.0;
  o->mlp = nullptr;
  o->infer_bf16 = 1;
  o->force_fallback = 0;
  o->sources = nullptr;
  o->nsources = 0;
  o->switch_rule = 0;
}

namespace sc {

int ensure_buffers(sc_graph* g, int B, size_t tsize) {
  using namespace sc;
  const int64_t n = g->d.n;
  const int64_t S = static_cast<int64_t>(g->rowptr_h[n]);
  const size_t yb = static_cast<size_t>(n) * B * tsize;
  // blocks per pipeline group: as many as the budget allows (at least one)
  int group = sc::kMaxGroupBlocks;
  while (group > 1 && 2 * sc::kPipeGroups * group * yb > sc::kPipeBudgetBytes) group /= 2;
  const int pairs = sc::kPipeGroups * group;
  if (yb > g->ybytes || pairs != g->ypairs) {
    for (auto& y : g->Y) {
      if (y) (void)sc::tracked_free(y);
      y = nullptr;
    }
    g->ybytes = 0;
    g->ypairs = 0;
    for (int i = 0; i < 2 * pairs; ++i) HIP_TRY(sc::tracked_malloc(&g->Y[i], yb));
    g->ybytes = yb;
    g->ypairs = pairs;
  }
  if (!g->nz) {
    HIP_TRY(dev_alloc(&g->nz, n));
    HIP_TRY(hipMemset(g->nz, 1, n));
  }
  const size_t pb = static_cast<size_t>(std::max(g->d.nparts, 1)) * B * tsize;
  if (pb > g->pbytes) {
    if (g->partials) (void)sc::tracked_free(g->partials);
    g->partials = nullptr;
    g->pbytes = 0;
    HIP_TRY(sc::tracked_malloc(&g->partials, pb));
    g->pbytes = pb;
  }
  if (!g->mask) {
    HIP_TRY(dev_alloc(&g->mask, 2 * n));
    HIP_TRY(hipMemset(g->mask, 0, 2 * n * sizeof(unsigned long long)));
    HIP_TRY(dev_alloc(&g->anymask, 2 * ((n + 31) / 32)));
    HIP_TRY(hipMemset(g->anymask, 0, 2 * ((n + 31) / 32) * sizeof(unsigned)));
    g->mask_pending_s0 = -1;
  }
  if (!g->gacc) HIP_TRY(dev_alloc(&g->gacc, S));
  if (!g->tau_slot) HIP_TRY(dev_alloc(&g->tau_slot, S));
  if (!g->tau_row) HIP_TRY(dev_alloc(&g->tau_row, n));
  if (!g->nr_slot) HIP_TRY(dev_alloc(&g->nr_slot, S));
  if (!g->cs) HIP_TRY(dev_alloc(&g->cs, 64));
  if (!g->colscratch) HIP_TRY(sc::tracked_malloc(&g->colscratch, sc::kColScratchBytes));
  if (!g->work) HIP_TRY(dev_alloc(&g->work, 4));   // [0..1] walk totals, [2] capped halves
  if (!g->plan_work) HIP_TRY(dev_alloc(&g->plan_work, 2 * 64));
  if (!g->out_dev) HIP_TRY(dev_alloc(&g->out_dev, g->d.m));
  return SC_OK;
}

int ensure_pipeline(sc_graph* g) {
  if (!g->tail_stream) HIP_TRY(hipStreamCreateWithFlags(&g->tail_stream, hipStreamNonBlocking));
  for (auto& e : g->pipe_ev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return SC_OK;
}

}  // namespace sc

namespace {

using sc::Runner;

// Switch-step cost model.  The traversal of a block runs on the critical
// stream, its tail (candidate summary, walk counts, walks) on the tail stream,
// so a block costs about max(traversal, tail) plus an interference share of
// the shorter one.  Constants are whole-GPU rates measured on MI355X; the
// environment can override them for tuning.
struct CostModel {
  double gather_bw;     // bytes/s of neighbour-row gathers in a dense step
  double step_fixed;    // s of fixed cost per dense step
  double twohop_frac;   // two-hop step cost relative to a dense step
  double skip_frac;     // first dense step (zero rows skipped, B = 64) relative to a dense step
  double tail_fixed;    // s of a block's tail launches besides the walks (their
                        // chain of small launches under the traversal's load) ...
  double tail_per_node; // ... plus this many s per node (passes over the block state)
  double walk_step;     // s per single-walk step
  double overlap;       // share of the shorter stream that still costs time
};

CostModel cost_model() {
  CostModel c{7.5e12, 3.0e-6, 0.3, 0.6, 5.5e-5, 3.5e-10, 2.5e-11, 0.25};
  if (const char* s = std::getenv("SC_COST_GATHER_BW")) c.gather_bw = std::atof(s);
  if (const char* s = std::getenv("SC_COST_STEP_FIXED")) c.step_fixed = std::atof(s);
  if (const char* s = std::getenv("SC_COST_SKIP_FRAC")) c.skip_frac = std::atof(s);
  if (const char* s = std::getenv("SC_COST_TAIL_FIXED")) c.tail_fixed = std::atof(s);
  if (const char* s = std::getenv("SC_COST_TAIL_PER_NODE")) c.tail_per_node = std::atof(s);
  if (const char* s = std::getenv("SC_COST_WALK_STEP")) c.walk_step = std::atof(s);
  if (const char* s = std::getenv("SC_COST_OVERLAP")) c.overlap = std::atof(s);
  return c;
}

template <typename T>
int run_method(sc_graph* g, double eps, int L, const sc_options& o, double* out_user,
               sc_stats* st_user) {
  const int64_t n = g->d.n, m = g->d.m;
  hipStream_t st = static_cast<hipStream_t>(o.stream);
  const int B = o.block > 0 ? o.block : 64;
  if (B != 16 && B != 32 && B != 64) return fail(SC_EINVAL, "block must be 16, 32 or 64");
  const bool plus = o.method == SC_TGT_PLUS;
  const int gamma = o.gamma < 0 ? 10 : o.gamma;
  if (gamma > sc::kMaxGamma) return fail(SC_EINVAL, "gamma above 16 is not supported");
  int max_L = o.max_L > 0 ? o.max_L : 255;
  if (max_L % 2 == 0) --max_L;
  int rc = sc::ensure_buffers(g, B, sizeof(T));
  if (rc) return rc;
  const bool dev_ptrs = (o.flags & SC_DEVICE_PTRS) != 0;

  Runner<T> R{g, B, st, (o.flags & SC_TIME_KERNELS) != 0};
  R.stats.block = B;
  R.stats.tilde_tau = -1;
  R.stats.tilde_min = -1;
  R.stats.tilde_max = -1;
  R.stats.lambda_converged = -1;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  auto destroy_events = [&]() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  const sc::ScopeExit<decltype(destroy_events)> ev_guard{destroy_events};   // every return path
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  HIP_TRY(hipEventRecord(t0, st));

  // truncation policy: uniform L, CalTau with the graph's spectrum (Algorithm 1),
  // or the lambda*-bound (Algorithm 1 line 1)
  double lam = 0.0;
  int Lodd = 0;
  const bool spectral = L == 0 && (o.flags & SC_TAU_SPECTRAL) != 0;
  if (spectral && g->spec_omega < 2)
    return fail(SC_EINVAL, "SC_TAU_SPECTRAL needs a spectrum (sc_compute_spectrum or sc_set_spectrum)");
  if (L > 0) {
    Lodd = (L % 2 == 1) ? L : L + 1;
  } else if (spectral) {
    lam = std::fabs(g->spec_lam_h[1]);
  } else {
    if (o.lambda_star > 0.0) {
      lam = o.lambda_star;
    } else {
      rc = sc::graph_lambda_star(g, st, &lam);
      if (rc) return rc;
      R.stats.lambda_converged = g->lambda_converged;
    }
    if (!(lam > 0.0 && lam < 1.0)) return fail(SC_EINVAL, "lambda* must lie in (0, 1)");
  }
  R.stats.lambda_star = lam;
  const double eps_tau = plus ? eps / 2.0 : eps;
  unsigned long long* capped = g->work + 2;
  HIP_TRY(hipMemsetAsync(capped, 0, sizeof(unsigned long long), st));
  if (spectral)
    HIP_TRY(sc::launch_caltau(g->d, g->spec_lam, g->spec_phi, g->spec_omega, eps_tau, max_L,
                              g->tau_slot, g->tau_row, st, capped));
  else
    HIP_TRY(sc::launch_tau(g->d, Lodd, eps_tau, lam, max_L, g->tau_slot, g->tau_row, st, capped));
  std::vector<int32_t> tau_row(n);
  unsigned long long capped_h = 0;
  HIP_TRY(hipMemcpyAsync(tau_row.data(), g->tau_row, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&capped_h, capped, sizeof(capped_h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  R.stats.L_capped = static_cast<int64_t>(capped_h / 2);   // both halves of an edge share tau
  int Lmax = 0, Lmin = 1 << 30;
  for (int64_t x = 0; x < n; ++x) {
    Lmax = std::max(Lmax, tau_row[x]);
    Lmin = std::min(Lmin, tau_row[x]);
  }
  R.stats.L_used = Lmax;
  R.stats.L_min = Lmin;

  const int nblocks = static_cast<int>((n + B - 1) / B);
  auto block_range = [&](int b, int* s0, int* kbeg, int* kend, int* tmax) {
    R.block_range(b, tau_row, s0, kbeg, kend, tmax);
  };

  int tilde = Lmax;
  double coef = 0.0;
  const int64_t nr_cap = (1ll << 31) - 1;
  if (plus && !g->walk.chunk_off) {
    // flattened walks: chunk offsets per slot, chunk sums (a block whose chunks
    // do not fit runs the per-slot kernel instead)
    const int64_t S = g->rowptr_h[n];
    HIP_TRY(sc::dev_alloc(&g->walk.chunk_off, S + 1));
    HIP_TRY(sc::dev_alloc(&g->walk.ctl, 2));
    g->walk.capacity = std::min<int64_t>(int64_t(1) << 22, 4 * S + 65536);
    if (const char* cap = std::getenv("SC_WALK_CHUNK_CAPACITY"))   // smaller buffer (tests)
      g->walk.capacity = std::max<int64_t>(1, std::min<int64_t>(g->walk.capacity, std::atoll(cap)));
    HIP_TRY(sc::dev_alloc(&g->walk.part, g->walk.capacity));
  }
  if (plus) {
    const double delta = o.delta > 0.0 ? o.delta : 1.0 / static_cast<double>(n);
    // Eq. 13 constant; m counts distinct edges
    coef = 8.0 * std::log(static_cast<double>(g->d.nslots) / delta) / (eps * eps);
    HIP_TRY(hipMemsetAsync(g->nr_slot, 0, g->rowptr_h[n] * sizeof(int64_t), st));
    const sc_graph::PlanKey key{eps,  L,     max_L, lam, B, static_cast<int>(sizeof(T)), gamma,
                                delta, spectral ? g->spec_version : 0};
    if (o.tilde_tau >= 0) {
      tilde = std::min(o.tilde_tau, Lmax);
    } else if (g->plan_valid && g->plan_key == key) {
      tilde = g->plan_tilde;   // the switch step depends only on the graph and these options
    } else {
      // sample blocks: walk steps at every candidate switch point
      const CostModel cm = cost_model();
      const double dense = cm.step_fixed + static_cast<double>(g->d.nslots) * B * sizeof(T) / cm.gather_bw;
      const double tail0 = cm.tail_fixed + cm.tail_per_node * static_cast<double>(n);
      const int nsamp = std::min(nblocks, 4);
      std::vector<double> cost(Lmax + 1, 0.0);
      for (int si = 0; si < nsamp; ++si) {
        const int b = static_cast<int>((si + 0.5) * nblocks / nsamp);
        int s0, kbeg, kend, tmax;
        block_range(b, &s0, &kbeg, &kend, &tmax);
        std::vector<unsigned long long> wk(2 * (Lmax + 1), 0ull);
        HIP_TRY(hipMemsetAsync(g->plan_work, 0, 2 * 64 * sizeof(unsigned long long), st));
        if (tmax >= 3) {
          rc = R.traverse(s0, kbeg, kend, 2, false, nullptr);
          if (rc) return rc;
          for (int ell = 2; ell < tmax && ell <= Lmax && ell < 64; ++ell) {
            if (ell > 2) {
              rc = R.advance();
              if (rc) return rc;
            }
            HIP_TRY(sc::launch_colstats<T>(g->d, s0, B, gamma, R.Yb(R.cur), g->cs, g->colscratch, st));
            HIP_TRY(sc::launch_walk_counts<T>(g->d, kbeg, kend, s0, B, ell, gamma, coef, nr_cap,
                                              R.Yb(R.cur), g->cs, g->tau_slot, g->nr_slot, st));
            HIP_TRY(sc::launch_work_totals(kbeg, kend, ell, g->tau_slot, g->nr_slot,
                                           g->plan_work + 2 * ell, st));
          }
          HIP_TRY(hipMemcpyAsync(wk.data(), g->plan_work,
                                 std::min<size_t>(wk.size(), 2 * 64) * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, st));
          HIP_TRY(hipStreamSynchronize(st));
        }
        for (int ell = 2; ell <= Lmax; ++ell) {
          const int steps = std::min(ell, tmax);
          const double first = B == 64 ? cm.skip_frac : 1.0;   // l = 3
          const double trav =
              steps >= 2 ? cm.step_fixed +
                               dense * (cm.twohop_frac + (steps >= 3 ? first + (steps - 3) : 0.0))
                         : 0.0;
          // switch points beyond the 64 counter slots are not candidates
          const double tail =
              ell < tmax ? (ell < 64 ? tail0 + static_cast<double>(wk[2 * ell + 1]) * cm.walk_step
                                     : 1e30)
                         : cm.step_fixed;
          cost[ell] += std::max(trav, tail) + cm.overlap * std::min(trav, tail);
        }
      }
      tilde = Lmax;
      for (int ell = 2; ell <= Lmax; ++ell)
        if (cost[ell] < cost[tilde]) tilde = ell;
      HIP_TRY(hipMemsetAsync(g->nr_slot, 0, g->rowptr_h[n] * sizeof(int64_t), st));
      g->plan_key = key;
      g->plan_tilde = tilde;
      g->plan_valid = true;
    }
    R.stats.tilde_tau = tilde;
    R.stats.tilde_min = tilde;
    R.stats.tilde_max = tilde;
  }
  HIP_TRY(sc::launch_gacc_init(g->d, g->tau_slot, (plus && tilde < 1) ? 0 : 1, g->gacc, st));
  R.ev_used = 0;
  R.stats.prop_launches = 0;
  R.stats.prop_bytes = 0.0;

  unsigned long long* work = g->work;
  HIP_TRY(hipMemsetAsync(work, 0, 2 * sizeof(unsigned long long), st));
  // Block pipeline: the traversal of block b runs on the caller's stream, its
  // tail (last accumulation, candidate summary, walk counts, walks) on the
  // tail stream, overlapping the traversals of the next blocks.  The streams
  // meet once per group of G blocks: the tails of a group wait for the whole
  // group's traversal, and the traversal of group q waits for the tails of
  // group q - kPipeGroups, whose Y pairs it reuses (block i of the launched
  // sequence takes pair i mod (kPipeGroups G)).  Blocks touch disjoint slots
  // of gacc and nr_slot.
  rc = sc::ensure_pipeline(g);
  if (rc) return rc;
  hipStream_t sb = g->tail_stream;
  HIP_TRY(hipEventRecord(g->pipe_ev[0], st));
  HIP_TRY(hipStreamWaitEvent(sb, g->pipe_ev[0], 0));
  const auto host0 = std::chrono::steady_clock::now();
  constexpr int Q = sc::kPipeGroups;
  const int D = g->ypairs;
  const int G = D / Q;
  bool tail_recorded[Q] = {};
  // the last pass of a block's walks rides on the next candidate summary's
  // first launch (same stream, before the next walks reuse the chunk buffers)
  sc::FinishJob fin;
  // a traversed block whose tail is not yet enqueued
  struct TailJob {
    int s0, kbeg, kend, tmax, pair, cur;
    sc::AccJob acc;
  };
  std::vector<TailJob> group_jobs;
  group_jobs.reserve(G);
  auto enqueue_tails = [&](int qset) -> int {
    HIP_TRY(hipEventRecord(g->pipe_ev[1 + qset], st));
    HIP_TRY(hipStreamWaitEvent(sb, g->pipe_ev[1 + qset], 0));
    R.st = sb;
    for (const TailJob& tj : group_jobs) {
      R.po = 2 * tj.pair;
      R.cur = tj.cur;
      R.pending_acc = tj.acc;
      // the last step's accumulation rides on the candidate summary's first
      // launch when there is one (same state, same stream)
      const bool fuse_acc = plus && tj.tmax > tilde && tilde >= 2;
      if (!fuse_acc) {
        const int rc1 = R.flush_acc();
        if (rc1) return rc1;
      }
      if (plus && tj.tmax > tilde) {
        if (tilde < 2) {
          const int rc1 = R.init_low(tj.s0, tilde);
          if (rc1) return rc1;
        }
        HIP_TRY(sc::launch_colstats<T>(g->d, tj.s0, B, gamma, R.Yb(R.cur), g->cs, g->colscratch,
                                       sb, fuse_acc ? &R.pending_acc : nullptr, &fin));
        R.pending_acc = sc::AccJob{};
        fin = sc::FinishJob{};
        HIP_TRY(sc::launch_walk_counts<T>(g->d, tj.kbeg, tj.kend, tj.s0, B, tilde, gamma, coef,
                                          nr_cap, R.Yb(R.cur), g->cs, g->tau_slot, g->nr_slot,
                                          sb));
        HIP_TRY(sc::launch_walks<T>(g->d, tj.kbeg, tj.kend, tj.s0, B, tilde, o.seed,
                                    R.Yb(R.cur), g->tau_slot, g->nr_slot, g->gacc, g->walk, sb,
                                    &fin));
      }
    }
    group_jobs.clear();
    HIP_TRY(hipEventRecord(g->pipe_ev[1 + Q + qset], sb));
    tail_recorded[qset] = true;
    R.st = st;
    return SC_OK;
  };
  int launched = 0;   // blocks traversed so far
  for (int b = 0; b < nblocks; ++b) {
    int s0, kbeg, kend, tmax;
    block_range(b, &s0, &kbeg, &kend, &tmax);
    const int lend = plus ? std::min(tmax, tilde) : tmax;
    // a block whose edges all stop at tau <= 1 has only the l = 0, 1 terms,
    // which the accumulator initialisation already holds: no launch, no events
    if (lend < 2 && !(plus && tmax > tilde)) continue;
    const int pair = launched % D;
    const int qset = (launched / G) % Q;
    if (launched % G == 0 && tail_recorded[qset])
      HIP_TRY(hipStreamWaitEvent(st, g->pipe_ev[1 + Q + qset], 0));
    R.st = st;
    R.po = 2 * pair;
    rc = R.traverse(s0, kbeg, kend, lend, true, g->gacc, b + 1 < nblocks ? s0 + B : -1);
    if (rc) return rc;
    group_jobs.push_back(TailJob{s0, kbeg, kend, tmax, pair, R.cur, R.pending_acc});
    R.pending_acc = sc::AccJob{};
    ++launched;
    if (launched % G == 0) {
      rc = enqueue_tails(qset);
      if (rc) return rc;
    }
  }
  if (!group_jobs.empty()) {
    rc = enqueue_tails(((launched - 1) / G) % Q);
    if (rc) return rc;
  }
  R.stats.host_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host0).count();
  HIP_TRY(sc::launch_walk_finish(fin, sb));
  HIP_TRY(hipEventRecord(g->pipe_ev[0], sb));
  HIP_TRY(hipStreamWaitEvent(st, g->pipe_ev[0], 0));
  R.po = 0;
  rc = R.flush_masks();
  if (rc) return rc;
  double* out_dev = dev_ptrs ? out_user : g->out_dev;
  HIP_TRY(sc::launch_combine(g->d, g->gacc, out_dev, st));
  HIP_TRY(hipEventRecord(t1, st));

  // traces
  int32_t* tau_o = nullptr;
  int64_t* nr_o = nullptr;
  if (o.tau_out) {
    if (!dev_ptrs && !g->tau_out_dev) HIP_TRY(dev_alloc(&g->tau_out_dev, m));
    tau_o = dev_ptrs ? o.tau_out : g->tau_out_dev;
  }
  if (o.nr_out) {
    if (!dev_ptrs && !g->nr_out_dev) HIP_TRY(dev_alloc(&g->nr_out_dev, 2 * m));
    nr_o = dev_ptrs ? o.nr_out : g->nr_out_dev;
  }
  HIP_TRY(sc::launch_trace(g->d, g->tau_slot, plus ? g->nr_slot : nullptr, tau_o, nr_o, st));
  std::vector<int32_t> tilde_h;
  if (o.tilde_tau_out) {
    tilde_h.resize(n);
    for (int64_t x = 0; x < n; ++x)   // in the caller's ids
      tilde_h[x] = plus ? tilde : tau_row[g->rank_h.empty() ? x : g->rank_h[x]];
    if (dev_ptrs)
      HIP_TRY(hipMemcpyAsync(o.tilde_tau_out, tilde_h.data(), n * sizeof(int32_t),
                             hipMemcpyHostToDevice, st));
    else
      std::memcpy(o.tilde_tau_out, tilde_h.data(), n * sizeof(int32_t));
  }
  unsigned long long wk[2] = {0, 0};
  if (plus) {
    HIP_TRY(sc::launch_work_totals(0, static_cast<int>(g->d.nslots), tilde, g->tau_slot,
                                   g->nr_slot, work, st));
    HIP_TRY(hipMemcpyAsync(wk, work, sizeof(wk), hipMemcpyDeviceToHost, st));
  }
  if (!dev_ptrs) {
    HIP_TRY(hipMemcpyAsync(out_user, out_dev, m * sizeof(double), hipMemcpyDeviceToHost, st));
    if (o.tau_out)
      HIP_TRY(hipMemcpyAsync(o.tau_out, tau_o, m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (o.nr_out)
      HIP_TRY(hipMemcpyAsync(o.nr_out, nr_o, 2 * m * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
  R.stats.total_ms = ms;
  R.stats.walks = plus ? static_cast<int64_t>(wk[0]) : 0;
  R.stats.walk_steps = plus ? static_cast<int64_t>(wk[1]) : 0;
  if (R.timing) {
    double tot = 0.0;
    for (size_t i = 0; i + 1 < R.ev_used; i += 2) {
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, g->events[i], g->events[i + 1]));
      tot += t;
    }
    R.stats.prop_ms = tot;
    R.stats.prop_timed = static_cast<int64_t>(R.ev_used / 2);
  }
  if (st_user) *st_user = R.stats;
  return SC_OK;
}

}  // namespace

extern "C" int sc_all_edges_ex(sc_graph* g, double eps, int L, const sc_options* o, double* out,
                               sc_stats* st) {
  if (!g) return fail(SC_EINVAL, "graph is NULL");
  if (!out) return fail(SC_EINVAL, "out is NULL");
  if (!(eps > 0.0 && eps < 1.0)) return fail(SC_EINVAL, "eps must lie in (0, 1)");
  if (L < 0) return fail(SC_EINVAL, "L must be >= 0");
  sc_options opt;
  if (o)
    opt = *o;
  else
    sc_default_options(&opt);
  if (opt.method != SC_TGT && opt.method != SC_TGT_PLUS && opt.method != SC_LEARNED)
    return fail(SC_EINVAL, "unknown method");
  if (opt.precision != 0 && opt.precision != 1) return fail(SC_EINVAL, "precision must be 0 or 1");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != g->device) (void)hipSetDevice(g->device);
  if (opt.method == SC_LEARNED && (opt.flags & SC_TAU_SPECTRAL))
    return fail(SC_ENOTIMPL, "SC_TAU_SPECTRAL is not supported with SC_LEARNED");
  const bool per_source = (opt.flags & SC_PER_SOURCE) != 0;
  if (per_source && opt.method != SC_TGT_PLUS)
    return fail(SC_ENOTIMPL, "SC_PER_SOURCE runs TGT+ (method 1) only");
  if (opt.sources && !per_source) return fail(SC_EINVAL, "a source list needs SC_PER_SOURCE");
  int rc;
  if (per_source)
    rc = sc::run_per_source(g, eps, L, opt, out, st);
  else if (opt.method == SC_LEARNED)
    rc = sc::run_learned(g, eps, opt, out, st);
  else
    rc = opt.precision == 1 ? run_method<double>(g, eps, L, opt, out, st)
                            : run_method<float>(g, eps, L, opt, out, st);
  if (cur != g->device) (void)hipSetDevice(cur);
  return rc;
}

extern "C" int sc_all_edges(sc_graph* g, double eps, int L, double* out) {
  sc_options o;
  sc_default_options(&o);
  o.method = L == 0 ? SC_TGT_PLUS : SC_TGT;
  return sc_all_edges_ex(g, eps, L, &o, out, nullptr);
}

extern "C" const char* sc_strerror(int code) {
  switch (code) {
    case SC_OK: return "ok";
    case SC_EINVAL: return "invalid argument";
    case SC_ESELFLOOP: return "self-loop in edge list";
    case SC_EDUP: return "duplicate edge";
    case SC_EDISCONNECTED: return "graph is not connected";
    case SC_EBIPARTITE: return "graph is bipartite";
    case SC_ENOMEM: return "out of memory";
    case SC_EHIP: return "HIP runtime error";
    case SC_ENOTIMPL: return "not implemented";
    default: return "unknown error code";
  }
}

extern "C" const char* sc_last_error(void) { return sc::g_last_error.c_str(); }

extern "C" const char* sc_version(void) { return "sc-mi355x 0.1 (gfx950)"; }
