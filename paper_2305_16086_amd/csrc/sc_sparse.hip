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
#include <mutex>
#include <type_traits>
#include <vector>

#include "sc_host.hpp"

using sc::dev_alloc;
using sc::dev_free;
using sc::fail;

namespace {

constexpr int kMaxSlots = 2048;
constexpr int64_t kPartCapacity = int64_t(1) << 24;   // chunk sums of one wave (128 MiB)

// totals: walk pairs, walk steps, pushed entries, min / max switch step,
// capped half-edges, min / max row truncation
constexpr int kTotals = 8;

// Device buffers of one call.
struct SrcBufs {
  double* gacc = nullptr;
  int32_t* tau_slot = nullptr;
  int32_t* tau_row = nullptr;
  int64_t* nr_slot = nullptr;
  uint64_t* Q = nullptr;
  int32_t* S = nullptr;
  int32_t* slot_ctl = nullptr;
  int32_t* tilde_row = nullptr;
  int32_t* pos_slot = nullptr;
  int32_t* pos_w = nullptr;
  int64_t* nr_pos = nullptr;
  int64_t* chunk_off = nullptr;
  double* part = nullptr;
  int64_t part_capacity = 0;
  int64_t* ctl = nullptr;
  unsigned long long* totals = nullptr;
  int32_t* list = nullptr;    // source list (null: all)
  int64_t* hoff = nullptr;
  bool Q_clean = false;       // Q is known to be all zero
  int W = 1;
};

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

// largest half-edge count of a wave of W consecutive list entries
int64_t wave_positions(int64_t nsrc, int W, const std::vector<int64_t>* hoff,
                       const std::vector<int32_t>& rowptr_h) {
  auto at = [&](int64_t k) -> int64_t { return hoff ? (*hoff)[k] : int64_t(rowptr_h[k]); };
  int64_t pm = 0;
  for (int64_t b = 0; b < nsrc; b += W) pm = std::max(pm, at(std::min(nsrc, b + W)) - at(b));
  return pm;
}

// lambda* for the automatic truncation: given, cached or (allow_compute) computed
int truncation_rate(sc_graph* g, int L, const sc_options& o, bool allow_compute, hipStream_t st,
                    double* lam, int* converged) {
  *lam = 0.0;
  *converged = -1;
  const bool spectral = L == 0 && (o.flags & SC_TAU_SPECTRAL) != 0;
  if (spectral && g->spec_omega < 2)
    return fail(SC_EINVAL, "SC_TAU_SPECTRAL needs a spectrum (sc_compute_spectrum or sc_set_spectrum)");
  if (L > 0) return SC_OK;
  if (spectral) {
    *lam = std::fabs(g->spec_lam_h[1]);
    return SC_OK;
  }
  if (o.lambda_star > 0.0) {
    *lam = o.lambda_star;
  } else if (g->lambda_star > 0.0 || allow_compute) {
    const int rc = sc::graph_lambda_star(g, st, lam);
    if (rc) return rc;
    *converged = g->lambda_converged;
  } else {
    return fail(SC_EINVAL, "lambda* is not known yet (computing it allocates): pass "
                           "lambda_star in the options or call sc_lambda_star first");
  }
  if (!(*lam > 0.0 && *lam < 1.0)) return fail(SC_EINVAL, "lambda* must lie in (0, 1)");
  return SC_OK;
}

// The device work of one call on stream st: truncation, the l = 0 terms, the
// waves, the edge combine and the traces.  No allocation, no synchronisation,
// no memset (fills are kernels).
int enqueue_per_source(sc_graph* g, double eps, int L, const sc_options& o, double lam,
                       const SrcBufs& B, int64_t nsrc, const std::vector<int64_t>* hoff,
                       double* out_dev, int32_t* tau_o, int64_t* nr_o, hipStream_t st,
                       const std::vector<hipEvent_t>* walk_ev = nullptr,
                       bool batch_walks = false) {
  const int64_t n = g->d.n;
  const int64_t S2 = g->d.nslots;
  int max_L = o.max_L > 0 ? o.max_L : 255;
  if (max_L % 2 == 0) --max_L;
  const int Lodd = L > 0 ? ((L % 2 == 1) ? L : L + 1) : 0;
  const bool spectral = L == 0 && (o.flags & SC_TAU_SPECTRAL) != 0;
  const double eps_tau = eps / 2.0;   // Algorithm 4 line 2
  auto* tot = B.totals;
  const unsigned long long init[kTotals] = {0, 0, 0, ~0ull, 0, 0, ~0ull, 0};
  for (int k = 0; k < kTotals; ++k) HIP_TRY(sc::launch_fill_u64(reinterpret_cast<uint64_t*>(tot + k), 1, init[k], st));
  if (spectral)
    HIP_TRY(sc::launch_caltau(g->d, g->spec_lam, g->spec_phi, g->spec_omega, eps_tau, max_L,
                              B.tau_slot, B.tau_row, st, tot + 5));
  else
    HIP_TRY(sc::launch_tau(g->d, Lodd, eps_tau, lam, max_L, B.tau_slot, B.tau_row, st, tot + 5));
  HIP_TRY(sc::launch_tau_range(static_cast<int>(n), B.tau_row, tot + 6, st));
  if (!B.Q_clean)
    HIP_TRY(sc::launch_fill_u64(B.Q, static_cast<int64_t>(2) * B.W * n, 0, st));
  HIP_TRY(sc::launch_fill_u64(reinterpret_cast<uint64_t*>(B.nr_slot), S2, 0, st));
  // no slot holds a column to clear yet (the heads clear their slot's last one)
  HIP_TRY(sc::launch_fill_u32(reinterpret_cast<uint32_t*>(B.slot_ctl), 2 * static_cast<int64_t>(B.W),
                              0, st));
  HIP_TRY(sc::launch_fill_u32(reinterpret_cast<uint32_t*>(B.tilde_row), n, 0xFFFFFFFFu, st));
  HIP_TRY(sc::launch_gacc_init(g->d, B.tau_slot, 0, B.gacc, st));

  const double delta = o.delta > 0.0 ? o.delta : 1.0 / static_cast<double>(n);
  sc::SrcArgs a;
  a.n = static_cast<int32_t>(n);
  a.rowptr = g->d.rowptr;
  a.col = g->d.col;
  a.tau_slot = B.tau_slot;
  a.tau_row = B.tau_row;
  a.srcs = B.list;
  a.hoff = B.list ? B.hoff : nullptr;
  a.nsrc = nsrc;
  a.Q = B.Q;
  a.S = B.S;
  a.slot_ctl = B.slot_ctl;
  a.tilde_row = B.tilde_row;
  a.nr_slot = B.nr_slot;
  a.gacc = B.gacc;
  a.pos_slot = B.pos_slot;
  a.pos_w = B.pos_w;
  a.nr_pos = B.nr_pos;
  a.totals = tot;
  a.coef = 8.0 * std::log(static_cast<double>(S2) / delta) / (eps * eps);   // Eq. 13, 2m = slots
  a.nr_cap = (int64_t(1) << 31) - 1;
  a.gamma = o.gamma < 0 ? 10 : o.gamma;
  a.rule = o.switch_rule;
  a.force_tilde = o.tilde_tau;

  sc::SrcWalkArgs wa;
  wa.n = static_cast<int32_t>(n);
  wa.rowptr = g->d.rowptr;
  wa.col = g->d.col;
  wa.slot_row = g->d.slot_row;
  wa.tau_slot = B.tau_slot;
  wa.tilde_row = B.tilde_row;
  wa.Q = B.Q;
  wa.Qw = B.Q;
  wa.S = B.S;
  wa.slot_ctl = B.slot_ctl;
  wa.pos_slot = B.pos_slot;
  wa.pos_w = B.pos_w;
  wa.nr_pos = B.nr_pos;
  wa.chunk_off = B.chunk_off;
  wa.ctl = B.ctl;
  wa.part = B.part;
  wa.capacity = B.part_capacity;
  wa.gacc = B.gacc;
  wa.k0 = static_cast<unsigned>(o.seed & 0xFFFFFFFFull);
  wa.k1 = static_cast<unsigned>(o.seed >> 32);
  if (const char* f = std::getenv("SC_SOURCE_FINISH_SEG"))   // smaller segments (tests)
    wa.finish_seg = std::max<int64_t>(1, std::atoll(f));

  auto at = [&](int64_t k) -> int64_t { return hoff ? (*hoff)[k] : int64_t(g->rowptr_h[k]); };
  int64_t wave = 0;
  for (int64_t b = 0; b < nsrc; b += B.W, ++wave) {
    const int cnt = static_cast<int>(std::min<int64_t>(B.W, nsrc - b));
    a.list_base = b;
    a.pos_base = at(b);
    HIP_TRY(sc::launch_src_head(a, cnt, st));
    wa.P = at(b + cnt) - at(b);
    if (walk_ev) HIP_TRY(hipEventRecord((*walk_ev)[2 * wave], st));
    if (batch_walks && wa.P > 0) {
      // the host reads the wave's chunk count and walks them in batches of the
      // buffer's capacity, so no half is left to a single wave however many
      // walks it has
      HIP_TRY(sc::launch_src_scan(wa, st));
      int64_t total = 0;
      HIP_TRY(hipMemcpyAsync(&total, B.ctl, sizeof(total), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      for (int64_t c = 0; c < total; c += wa.capacity) {
        sc::SrcWalkArgs wb = wa;
        wb.cbeg = c;
        wb.cend = std::min(total, c + wa.capacity);
        HIP_TRY(sc::launch_src_walk_batch(wb, st));
      }
    } else {
      HIP_TRY(sc::launch_src_walks(wa, st));
    }
    if (walk_ev) HIP_TRY(hipEventRecord((*walk_ev)[2 * wave + 1], st));
  }
  // the final columns of the slots' last sources (the first wave used the most slots)
  HIP_TRY(sc::launch_src_clear(wa, static_cast<int>(std::min<int64_t>(B.W, nsrc)), st));
  HIP_TRY(sc::launch_combine(g->d, B.gacc, out_dev, st));
  HIP_TRY(sc::launch_trace(g->d, B.tau_slot, B.nr_slot, tau_o, nr_o, st));
  return SC_OK;
}

void fill_stats(const unsigned long long (&t)[kTotals], sc_stats* s) {
  s->walks = static_cast<int64_t>(t[0]);
  s->walk_steps = static_cast<int64_t>(t[1]);
  s->push_edges = static_cast<int64_t>(t[2]);
  s->tilde_min = t[3] == ~0ull ? -1 : static_cast<int32_t>(t[3]);
  s->tilde_max = static_cast<int32_t>(t[4]);
  s->tilde_tau = (s->tilde_min >= 0 && s->tilde_min == s->tilde_max) ? s->tilde_min : -1;
  s->L_capped = static_cast<int64_t>(t[5] / 2);   // both halves of an edge share tau
  s->L_min = static_cast<int>(t[6]);
  s->L_used = static_cast<int>(t[7]);
  s->block = 1;
}

}  // namespace

int sc::run_per_source(sc_graph* g, double eps, int L, const sc_options& o, double* out_user,
                       sc_stats* st_user) {
  const int64_t n = g->d.n, m = g->d.m;
  const int64_t S2 = g->d.nslots;
  hipStream_t st = static_cast<hipStream_t>(o.stream);
  const bool dev_ptrs = (o.flags & SC_DEVICE_PTRS) != 0;
  if (o.switch_rule != 0 && o.switch_rule != 1) return fail(SC_EINVAL, "switch_rule must be 0 or 1");

  // ---- source list (validated before anything is written), ordered by the
  // volume of the source's neighbourhood, largest first: a wave lasts as long as
  // its slowest source, so sources of similar cost share waves
  const int64_t nsrc = o.sources ? o.nsources : n;
  if (o.sources && (o.nsources <= 0 || o.nsources > n))
    return fail(SC_EINVAL, "nsources must lie in [1, n]");
  std::vector<int32_t> order(nsrc);
  if (o.sources) {
    std::vector<unsigned char> seen(n, 0);
    for (int64_t k = 0; k < nsrc; ++k) {
      const int32_t s = o.sources[k];
      if (s < 0 || s >= n) return fail(SC_EINVAL, "source id out of range");
      if (seen[s]) return fail(SC_EINVAL, "source listed twice");
      seen[s] = 1;
      order[k] = g->rank_h.empty() ? s : g->rank_h[s];   // the stored node
    }
  } else {
    for (int64_t k = 0; k < nsrc; ++k) order[k] = static_cast<int32_t>(k);
  }
  auto& sb0 = g->src;
  if (sb0.nbr_vol_h.empty()) {
    int64_t* vol = nullptr;
    HIP_TRY(dev_alloc(&vol, n));
    const hipError_t e1 = sc::launch_nbr_volume(g->d, vol, st);
    sb0.nbr_vol_h.resize(n);
    const hipError_t e2 = e1 == hipSuccess ? hipMemcpyAsync(sb0.nbr_vol_h.data(), vol, n * sizeof(int64_t),
                                                            hipMemcpyDeviceToHost, st)
                                           : e1;
    const hipError_t e3 = e2 == hipSuccess ? hipStreamSynchronize(st) : e2;
    dev_free(vol);
    if (e3 != hipSuccess) {
      sb0.nbr_vol_h.clear();
      return fail(SC_EHIP, std::string("neighbourhood volumes: ") + hipGetErrorString(e3));
    }
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return sb0.nbr_vol_h[x] > sb0.nbr_vol_h[y];
  });
  std::vector<int64_t> hoff(nsrc + 1);
  hoff[0] = 0;
  for (int64_t k = 0; k < nsrc; ++k)
    hoff[k + 1] = hoff[k] + (g->rowptr_h[order[k] + 1] - g->rowptr_h[order[k]]);
  const std::vector<int64_t>* hp = &hoff;

  // ---- slots: two n-word columns and two n-entry lists each
  const size_t per_slot = static_cast<size_t>(n) * (2 * sizeof(uint64_t) + 2 * sizeof(int32_t));
  size_t budget = 0;
  if (const char* b = std::getenv("SC_SOURCE_SLOT_BYTES")) budget = static_cast<size_t>(std::atof(b));
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    // the slot columns and lists the handle already holds are reused or
    // replaced, so they count as free
    const size_t held = g->src.qcap * (sizeof(uint64_t) + sizeof(int32_t));
    budget = std::min<size_t>((fr + held) / 2, size_t(128) << 30);
  }
  SrcBufs B;
  B.W = static_cast<int>(std::min<int64_t>({static_cast<int64_t>(kMaxSlots), nsrc,
                                            std::max<int64_t>(1, static_cast<int64_t>(budget / per_slot))}));
  const int64_t Pmax = wave_positions(nsrc, B.W, hp, g->rowptr_h);

  // ---- buffers owned by the handle
  auto& sb = g->src;
  if (!g->gacc) HIP_TRY(dev_alloc(&g->gacc, S2));
  if (!g->tau_slot) HIP_TRY(dev_alloc(&g->tau_slot, S2));
  if (!g->tau_row) HIP_TRY(dev_alloc(&g->tau_row, n));
  if (!g->nr_slot) HIP_TRY(dev_alloc(&g->nr_slot, S2));
  if (!g->out_dev) HIP_TRY(dev_alloc(&g->out_dev, m));
  const size_t qwords = static_cast<size_t>(2) * B.W * n;
  if (!sb.Q || sb.qcap < qwords) {
    dev_free(sb.Q);
    dev_free(sb.S);
    sb.qcap = 0;
    sb.clean = false;
    HIP_TRY(dev_alloc(&sb.Q, qwords));
    HIP_TRY(dev_alloc(&sb.S, qwords));
    sb.qcap = qwords;
  }
  HIP_TRY(grow(&sb.slot_ctl, &sb.ctl_cap, static_cast<size_t>(2) * B.W));
  HIP_TRY(grow(&sb.tilde_row, &sb.tilde_cap, static_cast<size_t>(n)));
  HIP_TRY(grow(&sb.pos_slot, &sb.pos_cap, static_cast<size_t>(Pmax)));
  HIP_TRY(grow(&sb.pos_w, &sb.posw_cap, static_cast<size_t>(Pmax)));
  HIP_TRY(grow(&sb.nr_pos, &sb.nrp_cap, static_cast<size_t>(Pmax)));
  HIP_TRY(grow(&sb.chunk_off, &sb.co_cap, static_cast<size_t>(Pmax) + 1));
  HIP_TRY(grow(&sb.part, &sb.part_cap, static_cast<size_t>(kPartCapacity)));
  HIP_TRY(grow(&sb.ctl, &sb.ctl2_cap, size_t(2)));
  HIP_TRY(grow(&sb.totals, &sb.tot_cap, size_t(kTotals)));
  HIP_TRY(grow(&sb.list, &sb.list_cap, static_cast<size_t>(nsrc)));
  HIP_TRY(grow(&sb.hoff, &sb.hoff_cap, static_cast<size_t>(nsrc) + 1));
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
  B.gacc = g->gacc;
  B.tau_slot = g->tau_slot;
  B.tau_row = g->tau_row;
  B.nr_slot = g->nr_slot;
  B.Q = sb.Q;
  B.S = sb.S;
  B.slot_ctl = sb.slot_ctl;
  B.tilde_row = sb.tilde_row;
  B.pos_slot = sb.pos_slot;
  B.pos_w = sb.pos_w;
  B.nr_pos = sb.nr_pos;
  B.chunk_off = sb.chunk_off;
  B.part = sb.part;
  B.part_capacity = kPartCapacity;
  if (const char* c = std::getenv("SC_SOURCE_PART_CAPACITY"))   // smaller buffer (tests)
    B.part_capacity = std::max<int64_t>(1, std::min<int64_t>(kPartCapacity, std::atoll(c)));
  B.ctl = sb.ctl;
  B.totals = sb.totals;
  B.list = sb.list;
  B.hoff = sb.hoff;
  B.Q_clean = sb.clean;

  hipEvent_t t0 = nullptr, t1 = nullptr;
  auto destroy_events = [&]() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  const sc::ScopeExit<decltype(destroy_events)> ev_guard{destroy_events};
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  HIP_TRY(hipEventRecord(t0, st));
  double lam = 0.0;
  int conv = -1;
  int rc = truncation_rate(g, L, o, true, st, &lam, &conv);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(B.list, order.data(), nsrc * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.hoff, hoff.data(), (nsrc + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  sb.clean = false;   // set again once the call has finished
  double* out_dev = dev_ptrs ? out_user : g->out_dev;
  // SC_TIME_KERNELS: the walk phase of every wave between two timing events
  std::vector<hipEvent_t> walk_ev;
  auto destroy_walk_events = [&]() {
    for (hipEvent_t e : walk_ev)
      if (e) (void)hipEventDestroy(e);
  };
  const sc::ScopeExit<decltype(destroy_walk_events)> wev_guard{destroy_walk_events};
  const int64_t waves = (nsrc + B.W - 1) / B.W;
  if (o.flags & SC_TIME_KERNELS) {
    walk_ev.assign(static_cast<size_t>(2 * waves), nullptr);
    for (auto& e : walk_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  const auto host0 = std::chrono::steady_clock::now();
  rc = enqueue_per_source(g, eps, L, o, lam, B, nsrc, hp, out_dev, tau_o, nr_o, st,
                          walk_ev.empty() ? nullptr : &walk_ev, true);
  if (rc) return rc;
  const double host_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host0).count();
  HIP_TRY(hipEventRecord(t1, st));
  const bool renumbered = g->rank_d != nullptr;
  std::vector<int32_t> tilde_h;   // stored order, for a host output of a renumbered graph
  if (o.tilde_tau_out) {
    if (renumbered && dev_ptrs) {
      HIP_TRY(sc::launch_gather_i32(B.tilde_row, g->rank_d, o.tilde_tau_out, n, st));
    } else if (renumbered) {
      tilde_h.resize(n);
      HIP_TRY(hipMemcpyAsync(tilde_h.data(), B.tilde_row, n * sizeof(int32_t),
                             hipMemcpyDeviceToHost, st));
    } else {
      HIP_TRY(hipMemcpyAsync(o.tilde_tau_out, B.tilde_row, n * sizeof(int32_t),
                             dev_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    }
  }
  unsigned long long tot[kTotals] = {};
  HIP_TRY(hipMemcpyAsync(tot, B.totals, sizeof(tot), hipMemcpyDeviceToHost, st));
  if (!dev_ptrs) {
    HIP_TRY(hipMemcpyAsync(out_user, out_dev, m * sizeof(double), hipMemcpyDeviceToHost, st));
    if (o.tau_out)
      HIP_TRY(hipMemcpyAsync(o.tau_out, tau_o, m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (o.nr_out)
      HIP_TRY(hipMemcpyAsync(o.nr_out, nr_o, 2 * m * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  sb.clean = true;
  if (!tilde_h.empty())
    for (int64_t x = 0; x < n; ++x) o.tilde_tau_out[x] = tilde_h[g->rank_h[x]];
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
  if (st_user) {
    sc_stats s{};
    fill_stats(tot, &s);
    s.lambda_star = lam;
    s.lambda_converged = conv;
    s.total_ms = ms;
    s.host_ms = host_ms;
    if (!walk_ev.empty()) {
      // the walks' algorithmic bytes: per single-walk step the row bounds
      // (8 B), the neighbour id (4 B) and the column entry (8 B)
      double wms = 0.0;
      for (int64_t w = 0; w < waves; ++w) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, walk_ev[2 * w], walk_ev[2 * w + 1]));
        wms += t;
      }
      s.prop_ms = wms;
      s.prop_launches = waves;
      s.prop_timed = waves;
      s.prop_bytes = 20.0 * static_cast<double>(s.walk_steps);
    }
    *st_user = s;
  }
  return SC_OK;
}
// ====================================================================== no-allocation entry point
//
// Every buffer of sc_all_edges_static lives in this array.  In host code its
// name is only a stand-in for the symbol: the device address, one per GPU,
// comes from hipGetSymbolAddress on the first call with that device current.

namespace {

constexpr size_t kStaticScratchBytes = size_t(128) << 20;
constexpr int64_t kStaticPartCapacity = int64_t(1) << 18;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};
// Layout of the last run on each device and whether it finished: its columns
// (Q) were then left all zero, but only a run with the same layout may rely on it
struct Layout {
  int64_t n = -1, slots = -1;
  int W = -1;
  bool clean = false;
};
Layout g_scratch_last[kMaxDevices];

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Carve the buffers of a run with W slots from base (null: only measure).
// Returns the bytes used.
size_t carve(unsigned char* base, int64_t n, int64_t S2, int W, int64_t P, SrcBufs* B) {
  size_t off = 0;
  auto take = [&](auto** p, size_t bytes) {
    if (base) *p = reinterpret_cast<std::remove_reference_t<decltype(**p)>*>(base + off);
    off += up256(bytes);
  };
  SrcBufs dummy;
  SrcBufs& b = B ? *B : dummy;
  take(&b.gacc, sizeof(double) * S2);
  take(&b.tau_slot, sizeof(int32_t) * S2);
  take(&b.nr_slot, sizeof(int64_t) * S2);
  take(&b.tau_row, sizeof(int32_t) * n);
  take(&b.tilde_row, sizeof(int32_t) * n);
  take(&b.totals, sizeof(unsigned long long) * kTotals);
  take(&b.ctl, sizeof(int64_t) * 2);
  take(&b.slot_ctl, sizeof(int32_t) * 2 * W);
  take(&b.pos_slot, sizeof(int32_t) * std::max<int64_t>(P, 1));
  take(&b.pos_w, sizeof(int32_t) * std::max<int64_t>(P, 1));
  take(&b.nr_pos, sizeof(int64_t) * std::max<int64_t>(P, 1));
  take(&b.chunk_off, sizeof(int64_t) * (P + 1));
  take(&b.part, sizeof(double) * kStaticPartCapacity);
  take(&b.Q, sizeof(uint64_t) * 2 * static_cast<size_t>(W) * n);
  take(&b.S, sizeof(int32_t) * 2 * static_cast<size_t>(W) * n);
  b.part_capacity = kStaticPartCapacity;
  if (const char* c = std::getenv("SC_SOURCE_PART_CAPACITY"))   // smaller buffer (tests)
    b.part_capacity = std::max<int64_t>(1, std::min<int64_t>(kStaticPartCapacity, std::atoll(c)));
  b.W = W;
  return off;
}

}  // namespace

extern "C" int sc_all_edges_static(sc_graph* g, double eps, int L, const sc_options* o,
                                   double* out, sc_stats* st) {
  if (!g) return fail(SC_EINVAL, "graph is NULL");
  if (!o) return fail(SC_EINVAL, "options are NULL");
  if (!out) return fail(SC_EINVAL, "out is NULL");
  if (!(eps > 0.0 && eps < 1.0)) return fail(SC_EINVAL, "eps must lie in (0, 1)");
  if (L < 0) return fail(SC_EINVAL, "L must be >= 0");
  if (o->method != SC_TGT_PLUS) return fail(SC_ENOTIMPL, "sc_all_edges_static runs TGT+ only");
  if (o->sources) return fail(SC_EINVAL, "sc_all_edges_static takes no source list");
  if (o->switch_rule != 0 && o->switch_rule != 1) return fail(SC_EINVAL, "switch_rule must be 0 or 1");
  if (g->device < 0 || g->device >= kMaxDevices) return fail(SC_EINVAL, "device index out of range");
  const int64_t n = g->d.n, S2 = g->d.nslots;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != g->device) (void)hipSetDevice(g->device);
  struct Restore {
    int dev, cur;
    ~Restore() {
      if (cur != dev) (void)hipSetDevice(cur);
    }
  } restore{g->device, cur};
  hipStream_t stream = static_cast<hipStream_t>(o->stream);

  // the largest slot count whose buffers fit the array
  int W = static_cast<int>(std::min<int64_t>(kMaxSlots, n));
  size_t need = 0;
  for (;;) {
    const int64_t P = wave_positions(n, W, nullptr, g->rowptr_h);
    need = carve(nullptr, n, S2, W, P, nullptr);
    if (need <= kStaticScratchBytes || W == 1) break;
    W = std::max(1, W / 2);
  }
  if (need > kStaticScratchBytes)
    return fail(SC_EINVAL, "graph too large for sc_all_edges_static: it needs " +
                               std::to_string(need) + " bytes of scratch, the static array holds " +
                               std::to_string(kStaticScratchBytes));
  double lam = 0.0;
  int conv = -1;
  int rc = truncation_rate(g, L, *o, false, stream, &lam, &conv);
  if (rc) return rc;

  std::lock_guard<std::mutex> lk(g_scratch_mu);
  unsigned char*& base = g_scratch_ptr[g->device];
  if (!base) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    base = static_cast<unsigned char*>(p);
    g_scratch_last[g->device] = Layout{};
  }
  SrcBufs B;
  carve(base, n, S2, W, wave_positions(n, W, nullptr, g->rowptr_h), &B);
  // the columns are cleared unless the last run on this GPU finished with the same layout
  Layout& last = g_scratch_last[g->device];
  B.Q_clean = last.clean && last.n == n && last.slots == S2 && last.W == W;
  last = Layout{n, S2, W, false};
  const auto host0 = std::chrono::steady_clock::now();
  rc = enqueue_per_source(g, eps, L, *o, lam, B, n, nullptr, out, o->tau_out, o->nr_out, stream);
  if (rc) return rc;
  if (o->tilde_tau_out) {
    if (g->rank_d)
      HIP_TRY(sc::launch_gather_i32(B.tilde_row, g->rank_d, o->tilde_tau_out, n, stream));
    else
      HIP_TRY(hipMemcpyAsync(o->tilde_tau_out, B.tilde_row, n * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, stream));
  }
  last.clean = true;   // in stream order, the call's last clear zeroes every column it used
  if (st) {
    unsigned long long tot[kTotals] = {};
    HIP_TRY(hipMemcpyAsync(tot, B.totals, sizeof(tot), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    sc_stats s{};
    fill_stats(tot, &s);
    s.lambda_star = lam;
    s.lambda_converged = conv;
    s.host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host0).count();
    s.total_ms = s.host_ms;
    *st = s;
  }
  return SC_OK;
}
