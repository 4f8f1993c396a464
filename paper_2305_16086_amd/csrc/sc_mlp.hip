// Host side of the learned tail closure: the network object, its training
// loop (kernels in kernels_closure.hip), the dataset builder and the
// SC_LEARNED run with its certified fallback.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "sc_host.hpp"

using sc::dev_alloc;
using sc::dev_free;
using sc::fail;

struct sc_mlp {
  int device = 0;
  float* theta = nullptr;  // [5313]
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* norm = nullptr;   // [32] mean, 1/std
  float* range = nullptr;  // [32] min, max
  bool has_norm = false;
  bool has_range = false;
  int step = 0;
  float* grads = nullptr;  // [tiles][5313]
  size_t grads_tiles = 0;
  float* lossp = nullptr;  // [tiles]
  float* grad = nullptr;   // [5313]
  float* losses = nullptr; // [steps of an epoch]
  size_t losses_cap = 0;
  int64_t* idx = nullptr;
  size_t idx_cap = 0;

  void release() {
    dev_free(theta);
    dev_free(m1);
    dev_free(m2);
    dev_free(norm);
    dev_free(range);
    dev_free(grads);
    dev_free(lossp);
    dev_free(grad);
    dev_free(losses);
    dev_free(idx);
  }
};

namespace {

constexpr int kP = sc::kMlpParams;

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& x) { return static_cast<double>(splitmix64(x) >> 11) * (1.0 / 9007199254740992.0); }

int ensure_train_scratch(sc_mlp* net, int64_t batch, int64_t n) {
  const size_t tiles = static_cast<size_t>((batch + 63) / 64);
  if (tiles > net->grads_tiles) {
    dev_free(net->grads);
    dev_free(net->lossp);
    HIP_TRY(dev_alloc(&net->grads, tiles * kP));
    HIP_TRY(dev_alloc(&net->lossp, tiles));
    net->grads_tiles = tiles;
  }
  if (static_cast<size_t>(n) > net->idx_cap) {
    dev_free(net->idx);
    HIP_TRY(dev_alloc(&net->idx, n));
    net->idx_cap = n;
  }
  const size_t steps = static_cast<size_t>((n + batch - 1) / batch);
  if (steps > net->losses_cap) {
    dev_free(net->losses);
    HIP_TRY(dev_alloc(&net->losses, steps));
    net->losses_cap = steps;
  }
  return SC_OK;
}

}  // namespace

extern "C" void sc_default_train_options(sc_train_options* t) {
  if (!t) return;
  std::memset(t, 0, sizeof(*t));
  t->epochs = 20;
  t->batch = 4096;
  t->lr = 2e-3f;
  t->seed = 0xC105Eull;
  t->stream = nullptr;
}

extern "C" int sc_mlp_create(uint64_t seed, sc_mlp** out) {
  if (!out) return fail(SC_EINVAL, "out is NULL");
  *out = nullptr;
  sc_mlp* net = new (std::nothrow) sc_mlp();
  if (!net) return fail(SC_ENOMEM, "host allocation failed");
  (void)hipGetDevice(&net->device);
  std::vector<float> th(kP, 0.0f);
  uint64_t s = seed;
  auto fill = [&](int off, int rows, int cols) {
    const double lim = std::sqrt(3.0 / cols);
    for (int i = 0; i < rows * cols; ++i) th[off + i] = static_cast<float>((2.0 * uniform01(s) - 1.0) * lim);
  };
  fill(0, 64, 16);                       // W1
  fill(64 * 16 + 64, 64, 64);            // W2
  fill(64 * 16 + 64 + 64 * 64 + 64, 1, 64);   // W3
  std::vector<float> nrm(32, 0.0f);
  for (int f = 0; f < 16; ++f) nrm[16 + f] = 1.0f;
  hipError_t e = dev_alloc(&net->theta, kP);
  if (e == hipSuccess) e = dev_alloc(&net->m1, kP);
  if (e == hipSuccess) e = dev_alloc(&net->m2, kP);
  if (e == hipSuccess) e = dev_alloc(&net->norm, 32);
  if (e == hipSuccess) e = dev_alloc(&net->range, 32);
  if (e == hipSuccess) e = dev_alloc(&net->grad, kP);
  if (e == hipSuccess) e = hipMemcpy(net->theta, th.data(), kP * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(net->m1, 0, kP * sizeof(float));
  if (e == hipSuccess) e = hipMemset(net->m2, 0, kP * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(net->norm, nrm.data(), 32 * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    net->release();
    delete net;
    return fail(e == hipErrorOutOfMemory ? SC_ENOMEM : SC_EHIP, std::string("sc_mlp_create: ") + hipGetErrorString(e));
  }
  *out = net;
  return SC_OK;
}

extern "C" void sc_mlp_free(sc_mlp* net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  net->release();
  delete net;
}

extern "C" int sc_mlp_get(const sc_mlp* net, float* params, float* norm, float* range) {
  if (!net) return fail(SC_EINVAL, "net is NULL");
  if (params) HIP_TRY(hipMemcpy(params, net->theta, kP * sizeof(float), hipMemcpyDeviceToHost));
  if (norm) HIP_TRY(hipMemcpy(norm, net->norm, 32 * sizeof(float), hipMemcpyDeviceToHost));
  if (range) {
    if (net->has_range) {
      HIP_TRY(hipMemcpy(range, net->range, 32 * sizeof(float), hipMemcpyDeviceToHost));
    } else {
      for (int f = 0; f < 16; ++f) {
        range[f] = -INFINITY;
        range[16 + f] = INFINITY;
      }
    }
  }
  return SC_OK;
}

extern "C" int sc_mlp_set(sc_mlp* net, const float* params, const float* norm, const float* range) {
  if (!net) return fail(SC_EINVAL, "net is NULL");
  if (params) {
    HIP_TRY(hipMemcpy(net->theta, params, kP * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(net->m1, 0, kP * sizeof(float)));
    HIP_TRY(hipMemset(net->m2, 0, kP * sizeof(float)));
    net->step = 0;
  }
  if (norm) {
    HIP_TRY(hipMemcpy(net->norm, norm, 32 * sizeof(float), hipMemcpyHostToDevice));
    net->has_norm = true;
  }
  if (range) {
    HIP_TRY(hipMemcpy(net->range, range, 32 * sizeof(float), hipMemcpyHostToDevice));
    net->has_range = true;
  }
  return SC_OK;
}

extern "C" int sc_mlp_grad(sc_mlp* net, const float* X, const float* z, const float* w, int64_t N,
                           float* grad_host, float* loss_host, void* stream) {
  if (!net || !X || !z || N <= 0) return fail(SC_EINVAL, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ensure_train_scratch(net, N, N);
  if (rc) return rc;
  std::vector<int64_t> id(N);
  for (int64_t i = 0; i < N; ++i) id[i] = i;
  HIP_TRY(hipMemcpyAsync(net->idx, id.data(), N * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(sc::launch_mlp_train_step(net->theta, net->norm, X, z, w, net->idx, N,
                                    1.0f / static_cast<float>(N), net->grads, net->lossp,
                                    net->grad, net->losses, st));
  if (grad_host) HIP_TRY(hipMemcpyAsync(grad_host, net->grad, kP * sizeof(float), hipMemcpyDeviceToHost, st));
  if (loss_host) HIP_TRY(hipMemcpyAsync(loss_host, net->losses, sizeof(float), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SC_OK;
}

extern "C" int sc_mlp_train(sc_mlp* net, const float* X, const float* z, const float* w, int64_t N,
                            const sc_train_options* topt, float* loss_per_epoch) {
  if (!net || !X || !z || N <= 0) return fail(SC_EINVAL, "bad arguments");
  sc_train_options t;
  if (topt)
    t = *topt;
  else
    sc_default_train_options(&t);
  if (t.epochs < 0 || t.batch <= 0 || !(t.lr > 0.0f)) return fail(SC_EINVAL, "bad training options");
  hipStream_t st = static_cast<hipStream_t>(t.stream);
  int rc = ensure_train_scratch(net, t.batch, N);
  if (rc) return rc;
  if (!net->has_norm) {
    HIP_TRY(sc::launch_norm_stats(X, N, net->norm, st));
    net->has_norm = true;
  }
  if (!net->has_range) {
    HIP_TRY(sc::launch_feature_range(X, N, net->range, net->range + 16, st));
    net->has_range = true;
  }
  std::vector<int64_t> perm(N);
  const int64_t steps = (N + t.batch - 1) / t.batch;
  std::vector<float> losses(steps);
  for (int ep = 0; ep < t.epochs; ++ep) {
    for (int64_t i = 0; i < N; ++i) perm[i] = i;
    uint64_t s = t.seed + 0x1000193ull * static_cast<uint64_t>(ep + 1);
    for (int64_t i = N - 1; i > 0; --i) {
      const int64_t j = static_cast<int64_t>(splitmix64(s) % static_cast<uint64_t>(i + 1));
      std::swap(perm[i], perm[j]);
    }
    HIP_TRY(hipMemcpyAsync(net->idx, perm.data(), N * sizeof(int64_t), hipMemcpyHostToDevice, st));
    for (int64_t b = 0; b < steps; ++b) {
      const int64_t nb = std::min<int64_t>(t.batch, N - b * t.batch);
      HIP_TRY(sc::launch_mlp_train_step(net->theta, net->norm, X, z, w, net->idx + b * t.batch, nb,
                                        1.0f / static_cast<float>(nb), net->grads, net->lossp,
                                        net->grad, net->losses + b, st));
      ++net->step;
      HIP_TRY(sc::launch_adam(net->theta, net->grad, net->m1, net->m2, t.lr, 0.9f, 0.999f, 1e-8f,
                              net->step, st));
    }
    HIP_TRY(hipMemcpyAsync(losses.data(), net->losses, steps * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (loss_per_epoch) {
      double acc = 0.0;
      for (int64_t b = 0; b < steps; ++b) acc += losses[b];
      loss_per_epoch[ep] = static_cast<float>(acc / static_cast<double>(steps));
    }
  }
  return SC_OK;
}

extern "C" int sc_mlp_predict(const sc_mlp* net, const float* X, int64_t N, int bf16, float* y,
                              void* stream) {
  if (!net || !X || !y || N < 0) return fail(SC_EINVAL, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(sc::launch_mlp_infer(net->theta, net->norm, X, N, bf16, y, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SC_OK;
}

// ====================================================================== weights file
//
// Layout (little-endian): 8-byte magic "SCMLPW01", u32 parameter count (5313),
// u32 flags (bit 0: normalisation set, bit 1: feature range set), then
// float32 params[5313], norm[32], range[32], then the u64 FNV-1a hash of every
// byte before it.

namespace {

constexpr char kMagic[8] = {'S', 'C', 'M', 'L', 'P', 'W', '0', '1'};

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

constexpr size_t kFileBytes = 8 + 4 + 4 + sizeof(float) * (kP + 64) + 8;

}  // namespace

extern "C" int sc_mlp_save(const sc_mlp* net, const char* path) {
  if (!net || !path) return fail(SC_EINVAL, "net or path is NULL");
  std::vector<unsigned char> buf(kFileBytes);
  std::vector<float> vals(kP + 64);
  const int rc = sc_mlp_get(net, vals.data(), vals.data() + kP, vals.data() + kP + 32);
  if (rc != SC_OK) return rc;
  const uint32_t count = kP;
  const uint32_t flags = (net->has_norm ? 1u : 0u) | (net->has_range ? 2u : 0u);
  unsigned char* p = buf.data();
  std::memcpy(p, kMagic, 8);
  std::memcpy(p + 8, &count, 4);
  std::memcpy(p + 12, &flags, 4);
  std::memcpy(p + 16, vals.data(), sizeof(float) * vals.size());
  const uint64_t h = fnv1a(buf.data(), kFileBytes - 8);
  std::memcpy(p + kFileBytes - 8, &h, 8);
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(SC_EINVAL, std::string("cannot open for writing: ") + path);
  const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
  const int c = std::fclose(f);
  if (w != buf.size() || c != 0) return fail(SC_EINVAL, std::string("write failed: ") + path);
  return SC_OK;
}

extern "C" int sc_mlp_load(const char* path, sc_mlp** out) {
  if (!path || !out) return fail(SC_EINVAL, "path or out is NULL");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(SC_EINVAL, std::string("cannot open: ") + path);
  std::vector<unsigned char> buf(kFileBytes + 1);
  const size_t r = std::fread(buf.data(), 1, buf.size(), f);
  std::fclose(f);
  if (r != kFileBytes) return fail(SC_EINVAL, std::string("not a weights file (size): ") + path);
  uint32_t count = 0, flags = 0;
  uint64_t h = 0;
  std::memcpy(&count, buf.data() + 8, 4);
  std::memcpy(&flags, buf.data() + 12, 4);
  std::memcpy(&h, buf.data() + kFileBytes - 8, 8);
  if (std::memcmp(buf.data(), kMagic, 8) != 0 || count != static_cast<uint32_t>(kP) || (flags & ~3u))
    return fail(SC_EINVAL, std::string("not a weights file (header): ") + path);
  if (fnv1a(buf.data(), kFileBytes - 8) != h)
    return fail(SC_EINVAL, std::string("weights file corrupted (checksum): ") + path);
  std::vector<float> vals(kP + 64);
  std::memcpy(vals.data(), buf.data() + 16, sizeof(float) * vals.size());
  for (float x : vals)
    if (std::isnan(x)) return fail(SC_EINVAL, std::string("weights file holds NaN: ") + path);
  sc_mlp* net = nullptr;
  int rc = sc_mlp_create(0, &net);
  if (rc != SC_OK) return rc;
  rc = sc_mlp_set(net, vals.data(), (flags & 1u) ? vals.data() + kP : nullptr,
                  (flags & 2u) ? vals.data() + kP + 32 : nullptr);
  if (rc != SC_OK) {
    sc_mlp_free(net);
    return rc;
  }
  *out = net;
  return SC_OK;
}

// ====================================================================== closure data and run

int sc::ensure_closure_buffers(sc_graph* g, size_t tsize) {
  const int64_t S = g->d.nslots, m = g->d.m;
  const size_t rb = static_cast<size_t>(S) * (kRecSteps + 1) * tsize;
  if (rb > g->rbytes) {
    if (g->rdiag) (void)sc::tracked_free(g->rdiag);
    if (g->roff) (void)sc::tracked_free(g->roff);
    g->rdiag = g->roff = nullptr;
    g->rbytes = 0;
    HIP_TRY(sc::tracked_malloc(&g->rdiag, rb));
    HIP_TRY(sc::tracked_malloc(&g->roff, rb));
    g->rbytes = rb;
  }
  if (!g->feat) HIP_TRY(dev_alloc(&g->feat, static_cast<size_t>(m) * kFeat));
  if (!g->zpred) HIP_TRY(dev_alloc(&g->zpred, m));
  if (!g->cl_s0) HIP_TRY(dev_alloc(&g->cl_s0, 4 * static_cast<size_t>(m)));
  if (!g->fb) HIP_TRY(dev_alloc(&g->fb, m));
  if (!g->block_flag) HIP_TRY(dev_alloc(&g->block_flag, (g->d.n + 15) / 16 + 1));
  return SC_OK;
}

namespace {

// the first L0 steps of every block with per-slot recordings, then the features
template <typename T>
int record_and_features(sc_graph* g, int B, hipStream_t st, double lam, float* X, double* s0,
                        double* uK, double* lo, double* hi, sc::Runner<T>& R) {
  HIP_TRY(sc::launch_record_init<T>(g->d, static_cast<T*>(g->rdiag), static_cast<T*>(g->roff), st));
  R.rdiag = static_cast<T*>(g->rdiag);
  R.roff = static_cast<T*>(g->roff);
  R.record_to = sc::kRecSteps;
  const int64_t n = g->d.n;
  const int nblocks = static_cast<int>((n + B - 1) / B);
  std::vector<int32_t> dummy_tau(n, sc::kRecSteps);
  for (int b = 0; b < nblocks; ++b) {
    int s0b, kbeg, kend, tmax;
    R.block_range(b, dummy_tau, &s0b, &kbeg, &kend, &tmax);
    // the next block's neighbour masks ride on this block's first dense step
    // steps 2 .. L0 - 1 (recordings ride on the next launch), then steps
    // L0 - 1 and L0 recorded from the state at L0 - 1 (no full last step)
    const int rc = R.traverse(s0b, kbeg, kend, sc::kRecSteps - 1, false, nullptr,
                              b + 1 < nblocks ? s0b + B : -1);
    if (rc) return rc;
    R.pending_acc = sc::AccJob{};
    if (kend > kbeg)
      HIP_TRY(sc::launch_record_last<T>(g->d, kbeg, kend, s0b, B, sc::kRecSteps, R.Yb(R.cur),
                                        R.rdiag, R.roff, st));
  }
  {
    const int rc = R.flush_masks();
    if (rc) return rc;
  }
  R.rdiag = nullptr;
  R.roff = nullptr;
  HIP_TRY(sc::launch_features<T>(g->d, static_cast<const T*>(g->rdiag), static_cast<const T*>(g->roff),
                                 lam, X, s0, uK, lo, hi, st));
  return SC_OK;
}

template <typename T>
int closure_features_t(sc_graph* g, hipStream_t st, float* X, double* s0, double* uK, double* lo,
                       double* hi) {
  const int B = 64;
  int rc = sc::ensure_buffers(g, B, sizeof(T));
  if (rc) return rc;
  rc = sc::ensure_closure_buffers(g, sizeof(T));
  if (rc) return rc;
  double lam = 0.0;
  rc = sc::graph_lambda_star(g, st, &lam);
  if (rc) return rc;
  const int64_t m = g->d.m;
  double* base = g->cl_s0;
  sc::Runner<T> R{g, B, st, false};
  return record_and_features<T>(g, B, st, lam, X ? X : g->feat, s0 ? s0 : base,
                                uK ? uK : base + m, lo ? lo : base + 2 * m, hi ? hi : base + 3 * m, R);
}

template <typename T>
int learned_t(sc_graph* g, double eps, const sc_options& o, double* out_user, sc_stats* st_user) {
  const int64_t n = g->d.n, m = g->d.m;
  hipStream_t st = static_cast<hipStream_t>(o.stream);
  const int B = o.block > 0 ? o.block : 64;
  if (B != 16 && B != 32 && B != 64) return fail(SC_EINVAL, "block must be 16, 32 or 64");
  if (!o.mlp) return fail(SC_EINVAL, "SC_LEARNED needs options.mlp");
  const sc_mlp* net = o.mlp;
  const bool dev_ptrs = (o.flags & SC_DEVICE_PTRS) != 0;
  int rc = sc::ensure_buffers(g, B, sizeof(T));
  if (rc) return rc;
  rc = sc::ensure_closure_buffers(g, sizeof(T));
  if (rc) return rc;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  auto destroy_events = [&]() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  const sc::ScopeExit<decltype(destroy_events)> ev_guard{destroy_events};   // every return path
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  HIP_TRY(hipEventRecord(t0, st));
  double lam = o.lambda_star;
  int converged = -1;
  if (!(lam > 0.0)) {
    rc = sc::graph_lambda_star(g, st, &lam);
    if (rc) return rc;
    converged = g->lambda_converged;
  }
  int max_L = o.max_L > 0 ? o.max_L : 255;
  if (max_L % 2 == 0) --max_L;
  // fallback truncation: Theorem 3.2 at eps (its cut edges counted in work[2])
  unsigned long long* capped = g->work + 2;
  HIP_TRY(hipMemsetAsync(capped, 0, sizeof(unsigned long long), st));
  HIP_TRY(sc::launch_tau(g->d, 0, eps, lam, max_L, g->tau_slot, g->tau_row, st, capped));
  std::vector<int32_t> tau_row(n);
  unsigned long long capped_h = 0;
  HIP_TRY(hipMemcpyAsync(tau_row.data(), g->tau_row, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&capped_h, capped, sizeof(capped_h), hipMemcpyDeviceToHost, st));
  HIP_TRY(sc::launch_gacc_init(g->d, g->tau_slot, 1, g->gacc, st));

  sc::Runner<T> R{g, B, st, (o.flags & SC_TIME_KERNELS) != 0};
  R.stats.block = B;
  R.stats.tilde_tau = -1;
  R.stats.tilde_min = -1;
  R.stats.tilde_max = -1;
  R.stats.lambda_star = lam;
  R.stats.lambda_converged = converged;
  double* s0 = g->cl_s0;
  double* uK = s0 + m;
  double* lo = s0 + 2 * m;
  double* hi = s0 + 3 * m;
  rc = record_and_features<T>(g, B, st, lam, g->feat, s0, uK, lo, hi, R);
  if (rc) return rc;
  HIP_TRY(sc::launch_mlp_infer(net->theta, net->norm, g->feat, m, o.infer_bf16 ? 1 : 0, g->zpred, st));
  const int nblocks = static_cast<int>((n + B - 1) / B);
  HIP_TRY(hipMemsetAsync(g->block_flag, 0, (g->d.n + 15) / 16 * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(g->work, 0, 2 * sizeof(unsigned long long), st));
  double* out_dev = dev_ptrs ? out_user : g->out_dev;
  HIP_TRY(sc::launch_closure_apply(g->d, g->zpred, s0, uK, lo, hi, g->feat,
                                   net->has_range ? net->range : nullptr,
                                   net->has_range ? net->range + 16 : nullptr, eps, B,
                                   o.force_fallback ? 1 : 0, out_dev, g->fb, g->block_flag,
                                   g->work, st));
  std::vector<int> flags(nblocks);
  unsigned long long cnt[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(flags.data(), g->block_flag, nblocks * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(cnt, g->work, sizeof(cnt), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int Lmax = sc::kRecSteps;
  if (cnt[0] > 0) {
    for (int b = 0; b < nblocks; ++b) {
      if (!flags[b]) continue;
      int s0b, kbeg, kend, tmax;
      R.block_range(b, tau_row, &s0b, &kbeg, &kend, &tmax);
      Lmax = std::max(Lmax, tmax);
      rc = R.traverse(s0b, kbeg, kend, tmax, true, g->gacc);
      if (rc) return rc;
      rc = R.flush_acc();
      if (rc) return rc;
    }
    rc = R.flush_masks();
    if (rc) return rc;
    HIP_TRY(sc::launch_combine_masked(g->d, g->gacc, g->fb, out_dev, st));
  }
  HIP_TRY(hipEventRecord(t1, st));
  if (!dev_ptrs) HIP_TRY(hipMemcpyAsync(out_user, out_dev, m * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
  R.stats.total_ms = ms;
  R.stats.L_capped = static_cast<int64_t>(capped_h / 2);   // of the fallback truncation
  R.stats.L_used = Lmax;
  R.stats.L_min = sc::kRecSteps;
  R.stats.fallback_edges = static_cast<int64_t>(cnt[0]);
  if (R.timing) {
    double tot = 0.0;
    for (size_t i = 0; i + 1 < R.ev_used; i += 2) {
      float tt = 0.0f;
      HIP_TRY(hipEventElapsedTime(&tt, g->events[i], g->events[i + 1]));
      tot += tt;
    }
    R.stats.prop_ms = tot;
    R.stats.prop_timed = static_cast<int64_t>(R.ev_used / 2);
  }
  if (st_user) *st_user = R.stats;
  return SC_OK;
}

template <typename T>
int dataset_t(sc_graph* g, int L_ref, hipStream_t st, float* X, float* z, float* w) {
  const int64_t m = g->d.m;
  int rc = closure_features_t<T>(g, st, X, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  // reference sums at the uniform truncation L_ref (Algorithm 2)
  double* s_ref = nullptr;
  HIP_TRY(dev_alloc(&s_ref, m));
  sc_options o;
  sc_default_options(&o);
  o.method = SC_TGT;
  o.precision = sizeof(T) == 8 ? 1 : 0;
  o.flags = SC_DEVICE_PTRS;
  o.stream = st;
  rc = sc_all_edges_ex(g, 0.5, L_ref, &o, s_ref, nullptr);
  if (rc) {
    dev_free(s_ref);
    return rc;
  }
  const hipError_t e = sc::launch_targets(m, s_ref, g->cl_s0, g->cl_s0 + m, z, w, st);
  (void)hipStreamSynchronize(st);
  dev_free(s_ref);
  HIP_TRY(e);
  return SC_OK;
}

}  // namespace

int sc::run_learned(sc_graph* g, double eps, const sc_options& o, double* out, sc_stats* st) {
  return o.precision == 1 ? learned_t<double>(g, eps, o, out, st) : learned_t<float>(g, eps, o, out, st);
}

extern "C" int sc_closure_features(sc_graph* g, int precision, float* X, double* s0, double* uK,
                                   double* lo, double* hi, void* stream) {
  if (!g || !X) return fail(SC_EINVAL, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = precision == 1 ? closure_features_t<double>(g, st, X, s0, uK, lo, hi)
                          : closure_features_t<float>(g, st, X, s0, uK, lo, hi);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  return SC_OK;
}

extern "C" int sc_closure_dataset(sc_graph* g, int L_ref, int precision, float* X, float* z,
                                  float* w, void* stream) {
  if (!g || !X || !z || L_ref < sc::kRecSteps) return fail(SC_EINVAL, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return precision == 1 ? dataset_t<double>(g, L_ref, st, X, z, w)
                        : dataset_t<float>(g, L_ref, st, X, z, w);
}
