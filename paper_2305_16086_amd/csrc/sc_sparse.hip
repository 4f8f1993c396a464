// Host side of per-source TGT+ (SC_PER_SOURCE): Algorithm 4 with the
// adaptive switch step of Eq. 14 decided per source by the kernels of
// kernels_sparse.hip.  Sources are processed in waves of as many workgroup
// slots as the column memory allows; each wave is one head launch (traversal,
// CalChi, walk counts, Eq. 14) followed by the wave's flattened walks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "sc_host.hpp"

using sc::dev_alloc;
using sc::dev_free;
using sc::fail;

namespace {

constexpr int kMaxSlots = 2048;
constexpr int64_t kPartCapacity = int64_t(1) << 24;   // chunk sums of one wave (128 MiB)

// grow a device array to at least `count` elements
template <typename P>
hipError_t grow(P** p, size_t* cap, size_t count) {
  if (*p && *cap >= count) return hipSuccess;
  dev_free(*p);
  *cap = 0;
  const hipError_t e = dev_alloc(p, count);
  if (e == hipSuccess) *cap = count;
  return e;
}

}  // namespace

int sc::run_per_source(sc_graph* g, double eps, int L, const sc_options& o, double* out_user,
                       sc_stats* st_user) {
  const int64_t n = g->d.n, m = g->d.m;
  const int64_t S2 = g->d.nslots;
  hipStream_t st = static_cast<hipStream_t>(o.stream);
  const bool dev_ptrs = (o.flags & SC_DEVICE_PTRS) != 0;
  const int gamma = o.gamma < 0 ? 10 : o.gamma;
  if (o.switch_rule != 0 && o.switch_rule != 1) return fail(SC_EINVAL, "switch_rule must be 0 or 1");
  int max_L = o.max_L > 0 ? o.max_L : 255;
  if (max_L % 2 == 0) --max_L;

  sc_stats stats{};
  stats.tilde_tau = -1;
  stats.tilde_min = -1;
  stats.tilde_max = -1;
  stats.block = 1;
  stats.lambda_converged = -1;

  // ---- source list (validated before anything is written)
  const int64_t nsrc = o.sources ? o.nsources : n;
  if (o.sources && (o.nsources <= 0 || o.nsources > n))
    return fail(SC_EINVAL, "nsources must lie in [1, n]");
  std::vector<int64_t> hoff;
  if (o.sources) {
    std::vector<unsigned char> seen(n, 0);
    hoff.resize(nsrc + 1);
    hoff[0] = 0;
    for (int64_t k = 0; k < nsrc; ++k) {
      const int32_t s = o.sources[k];
      if (s < 0 || s >= n) return fail(SC_EINVAL, "source id out of range");
      if (seen[s]) return fail(SC_EINVAL, "source listed twice");
      seen[s] = 1;
      hoff[k + 1] = hoff[k] + (g->rowptr_h[s + 1] - g->rowptr_h[s]);
    }
  }
  auto hoff_at = [&](int64_t k) -> int64_t {
    return o.sources ? hoff[k] : static_cast<int64_t>(g->rowptr_h[k]);
  };

  // ---- slots: two n-word columns and two n-entry lists each
  const size_t per_slot = static_cast<size_t>(n) * (2 * sizeof(uint64_t) + 2 * sizeof(int32_t));
  size_t budget = 0;
  if (const char* b = std::getenv("SC_SOURCE_SLOT_BYTES")) budget = static_cast<size_t>(std::atof(b));
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    budget = std::min<size_t>(fr / 3, size_t(48) << 30);
  }
  int W = static_cast<int>(std::min<int64_t>(
      {static_cast<int64_t>(kMaxSlots), nsrc, std::max<int64_t>(1, static_cast<int64_t>(budget / per_slot))}));
  int64_t Pmax = 0;
  for (int64_t b = 0; b < nsrc; b += W) Pmax = std::max(Pmax, hoff_at(std::min(nsrc, b + W)) - hoff_at(b));

  // ---- buffers
  auto& sb = g->src;
  if (!g->gacc) HIP_TRY(dev_alloc(&g->gacc, S2));
  if (!g->tau_slot) HIP_TRY(dev_alloc(&g->tau_slot, S2));
  if (!g->tau_row) HIP_TRY(dev_alloc(&g->tau_row, n));
  if (!g->nr_slot) HIP_TRY(dev_alloc(&g->nr_slot, S2));
  if (!g->out_dev) HIP_TRY(dev_alloc(&g->out_dev, m));
  if (!g->work) HIP_TRY(dev_alloc(&g->work, 4));
  const size_t qwords = static_cast<size_t>(2) * W * n;
  if (!sb.Q || sb.qcap < qwords) {
    dev_free(sb.Q);
    dev_free(sb.S);
    sb.qcap = 0;
    HIP_TRY(dev_alloc(&sb.Q, qwords));
    HIP_TRY(dev_alloc(&sb.S, qwords));
    sb.qcap = qwords;
    sb.clean = false;
  }
  HIP_TRY(grow(&sb.slot_ctl, &sb.ctl_cap, static_cast<size_t>(2) * W));
  HIP_TRY(grow(&sb.tilde_row, &sb.tilde_cap, static_cast<size_t>(n)));
  HIP_TRY(grow(&sb.pos_slot, &sb.pos_cap, static_cast<size_t>(Pmax)));
  HIP_TRY(grow(&sb.pos_w, &sb.posw_cap, static_cast<size_t>(Pmax)));
  HIP_TRY(grow(&sb.nr_pos, &sb.nrp_cap, static_cast<size_t>(Pmax)));
  HIP_TRY(grow(&sb.chunk_off, &sb.co_cap, static_cast<size_t>(Pmax) + 1));
  HIP_TRY(grow(&sb.part, &sb.part_cap, static_cast<size_t>(kPartCapacity)));
  HIP_TRY(grow(&sb.ctl, &sb.ctl2_cap, size_t(2)));
  HIP_TRY(grow(&sb.totals, &sb.tot_cap, size_t(5)));
  int32_t* d_src = nullptr;
  int64_t* d_hoff = nullptr;
  if (o.sources) {
    HIP_TRY(grow(&sb.list, &sb.list_cap, static_cast<size_t>(nsrc)));
    HIP_TRY(grow(&sb.hoff, &sb.hoff_cap, static_cast<size_t>(nsrc) + 1));
    d_src = sb.list;
    d_hoff = sb.hoff;
  }

  hipEvent_t t0 = nullptr, t1 = nullptr;
  auto destroy_events = [&]() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  const sc::ScopeExit<decltype(destroy_events)> ev_guard{destroy_events};
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  HIP_TRY(hipEventRecord(t0, st));
  if (o.sources) {
    HIP_TRY(hipMemcpyAsync(d_src, o.sources, nsrc * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_hoff, hoff.data(), (nsrc + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  }

  // ---- truncation (Theorem 3.2 at eps / 2, Algorithm 4 line 2)
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
      const int rc = sc::graph_lambda_star(g, st, &lam);
      if (rc) return rc;
      stats.lambda_converged = g->lambda_converged;
    }
    if (!(lam > 0.0 && lam < 1.0)) return fail(SC_EINVAL, "lambda* must lie in (0, 1)");
  }
  stats.lambda_star = lam;
  const double eps_tau = eps / 2.0;
  unsigned long long* capped = g->work + 2;
  HIP_TRY(hipMemsetAsync(capped, 0, sizeof(unsigned long long), st));
  if (spectral)
    HIP_TRY(sc::launch_caltau(g->d, g->spec_lam, g->spec_phi, g->spec_omega, eps_tau, max_L,
                              g->tau_slot, g->tau_row, st, capped));
  else
    HIP_TRY(sc::launch_tau(g->d, Lodd, eps_tau, lam, max_L, g->tau_slot, g->tau_row, st, capped));

  // ---- per-call state: l = 0 terms, no walks, clean columns
  if (!sb.clean) HIP_TRY(hipMemsetAsync(sb.Q, 0, qwords * sizeof(uint64_t), st));
  sb.clean = false;   // set again once the call has finished
  HIP_TRY(hipMemsetAsync(g->nr_slot, 0, S2 * sizeof(int64_t), st));
  HIP_TRY(hipMemsetAsync(sb.tilde_row, 0xFF, n * sizeof(int32_t), st));
  HIP_TRY(sc::launch_gacc_init(g->d, g->tau_slot, 0, g->gacc, st));
  const unsigned long long tot0[5] = {0, 0, 0, ~0ull, 0};
  HIP_TRY(hipMemcpyAsync(sb.totals, tot0, sizeof(tot0), hipMemcpyHostToDevice, st));

  const double delta = o.delta > 0.0 ? o.delta : 1.0 / static_cast<double>(n);
  SrcArgs a;
  a.n = static_cast<int32_t>(n);
  a.rowptr = g->d.rowptr;
  a.col = g->d.col;
  a.tau_slot = g->tau_slot;
  a.tau_row = g->tau_row;
  a.srcs = d_src;
  a.hoff = d_hoff;
  a.nsrc = nsrc;
  a.Q = sb.Q;
  a.S = sb.S;
  a.slot_ctl = sb.slot_ctl;
  a.tilde_row = sb.tilde_row;
  a.nr_slot = g->nr_slot;
  a.gacc = g->gacc;
  a.pos_slot = sb.pos_slot;
  a.pos_w = sb.pos_w;
  a.nr_pos = sb.nr_pos;
  a.totals = sb.totals;
  a.coef = 8.0 * std::log(static_cast<double>(S2) / delta) / (eps * eps);   // Eq. 13, 2m = slots
  a.nr_cap = (int64_t(1) << 31) - 1;
  a.gamma = gamma;
  a.rule = o.switch_rule;
  a.force_tilde = o.tilde_tau;

  SrcWalkArgs wa;
  wa.n = static_cast<int32_t>(n);
  wa.rowptr = g->d.rowptr;
  wa.col = g->d.col;
  wa.slot_row = g->d.slot_row;
  wa.tau_slot = g->tau_slot;
  wa.tilde_row = sb.tilde_row;
  wa.Q = sb.Q;
  wa.Qw = sb.Q;
  wa.S = sb.S;
  wa.slot_ctl = sb.slot_ctl;
  wa.pos_slot = sb.pos_slot;
  wa.pos_w = sb.pos_w;
  wa.nr_pos = sb.nr_pos;
  wa.chunk_off = sb.chunk_off;
  wa.ctl = sb.ctl;
  wa.part = sb.part;
  wa.capacity = kPartCapacity;
  if (const char* c = std::getenv("SC_SOURCE_PART_CAPACITY"))   // smaller buffer (tests)
    wa.capacity = std::max<int64_t>(1, std::min<int64_t>(kPartCapacity, std::atoll(c)));
  wa.gacc = g->gacc;
  wa.k0 = static_cast<unsigned>(o.seed & 0xFFFFFFFFull);
  wa.k1 = static_cast<unsigned>(o.seed >> 32);

  const auto host0 = std::chrono::steady_clock::now();
  for (int64_t b = 0; b < nsrc; b += W) {
    const int cnt = static_cast<int>(std::min<int64_t>(W, nsrc - b));
    a.list_base = b;
    a.pos_base = hoff_at(b);
    HIP_TRY(sc::launch_src_head(a, cnt, st));
    wa.P = hoff_at(b + cnt) - hoff_at(b);
    HIP_TRY(sc::launch_src_walks(wa, cnt, st));
  }
  stats.host_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host0).count();
  double* out_dev = dev_ptrs ? out_user : g->out_dev;
  HIP_TRY(sc::launch_combine(g->d, g->gacc, out_dev, st));
  HIP_TRY(hipEventRecord(t1, st));

  // ---- traces and statistics
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
  HIP_TRY(sc::launch_trace(g->d, g->tau_slot, g->nr_slot, tau_o, nr_o, st));
  if (o.tilde_tau_out)
    HIP_TRY(hipMemcpyAsync(o.tilde_tau_out, sb.tilde_row, n * sizeof(int32_t),
                           dev_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  unsigned long long tot[5] = {};
  unsigned long long capped_h = 0;
  HIP_TRY(hipMemcpyAsync(tot, sb.totals, sizeof(tot), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&capped_h, capped, sizeof(capped_h), hipMemcpyDeviceToHost, st));
  std::vector<int32_t> tau_row_h(n);
  HIP_TRY(hipMemcpyAsync(tau_row_h.data(), g->tau_row, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (!dev_ptrs) {
    HIP_TRY(hipMemcpyAsync(out_user, out_dev, m * sizeof(double), hipMemcpyDeviceToHost, st));
    if (o.tau_out)
      HIP_TRY(hipMemcpyAsync(o.tau_out, tau_o, m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (o.nr_out)
      HIP_TRY(hipMemcpyAsync(o.nr_out, nr_o, 2 * m * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  sb.clean = true;
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
  stats.total_ms = ms;
  stats.walks = static_cast<int64_t>(tot[0]);
  stats.walk_steps = static_cast<int64_t>(tot[1]);
  stats.push_edges = static_cast<int64_t>(tot[2]);
  stats.tilde_min = tot[3] == ~0ull ? -1 : static_cast<int32_t>(tot[3]);
  stats.tilde_max = static_cast<int32_t>(tot[4]);
  if (stats.tilde_min >= 0 && stats.tilde_min == stats.tilde_max) stats.tilde_tau = stats.tilde_min;
  stats.L_capped = static_cast<int64_t>(capped_h / 2);
  int Lmax = 0, Lmin = std::numeric_limits<int>::max();
  for (int64_t x = 0; x < n; ++x) {
    Lmax = std::max(Lmax, tau_row_h[x]);
    Lmin = std::min(Lmin, tau_row_h[x]);
  }
  stats.L_used = Lmax;
  stats.L_min = Lmin;
  if (st_user) *st_user = stats;
  return SC_OK;
}
