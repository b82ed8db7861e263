// dtb_api.cpp - host side of the C ABI declared in include/dtb.h:
// validation, the device layout of the property and connection tables
// (Sec. V-D), handle lifetime, step sequencing and reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "dtb_internal.h"

using namespace dtb;

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;

dtb_status fail(dtb_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      return fail(DTB_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    }                                                                                   \
  } while (0)

// parallel loop over [0, n) in contiguous chunks on host threads
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 65536) nt = 1;
  if (nt == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned q = 0; q < nt; ++q) {
    const int64_t a = q * chunk, b = std::min<int64_t>(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=, &fn] { fn(a, b); });
  }
  for (auto& x : th) x.join();
}

// first index in [0, n) for which bad(i) holds, or -1 (parallel scan)
int64_t find_first(int64_t n, const std::function<bool(int64_t)>& bad) {
  std::atomic<int64_t> first(INT64_MAX);
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      if (i >= first.load(std::memory_order_relaxed)) return;
      if (bad(i)) {
        int64_t cur = first.load();
        while (i < cur && !first.compare_exchange_weak(cur, i)) {
        }
        return;
      }
    }
  });
  const int64_t f = first.load();
  return f == INT64_MAX ? -1 : f;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Poisson(lambda) inversion thresholds T_k = floor(F(k) 2^32) while below
// 2^32 - 1, with F accumulated from p_0 = exp(-lambda), p_k = p_{k-1} lambda / k.
int poisson_thresholds(double lambda, uint32_t* T, int cap) {
  const double two32 = 4294967296.0;
  double pk = std::exp(-lambda), F = pk;
  for (int k = 0; k < cap; ++k) {
    const double x = std::floor(F * two32);
    if (x >= 4294967295.0) return k;
    T[k] = uint32_t(x);
    pk = pk * lambda / double(k + 1);
    F = F + pk;
  }
  return -1;
}

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

bool finite_f(float x) { return std::isfinite(x); }
}  // namespace

namespace dtb {
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace dtb

struct dtb_net {
  DeviceNet d;
  hipStream_t stream = nullptr;
  int64_t t = 0;                 // steps taken (host mirror of the device step)
  float dt_ms = 1.f;
  bool failed = false;           // sticky HIP failure
  int64_t force_head = 0;        // step index of the first pending forced bitmap
  int64_t force_pending = 0;     // forced steps not yet consumed
  std::vector<int64_t> region_n; // neurons per population
  std::vector<void*> allocs;
  bool own_stream = false;       // created by the library (caller passed NULL)
  // members of a batched partition: first row and first population of each
  std::vector<int64_t> member_row0;
  std::vector<int32_t> member_region0;
  std::vector<int32_t> member_id;
  std::vector<uint64_t> member_seed;
  // captured step sequence replayed by dtb_run
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int32_t graph_steps = 0;
  // kernel timing: event pairs per kernel kind, reused after each read
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool[kTimedKernels];
  size_t ev_used[kTimedKernels] = {};
  // remote in-edge block (J_inter): its delivery tests run on a second
  // stream, forked from and joined back into the handle's stream every step
  bool remote = false;
  hipStream_t comm = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipEvent_t bg_fork = nullptr, bg_join = nullptr;  // the background counts on the second stream
  int64_t rq_head = 0;     // queue row of the first pending remote step
  int64_t rq_pending = 0;  // remote steps pushed and not yet consumed
  uint32_t read_epoch = 0; // spike-list rebuilds so far (their look-back epochs)
};

namespace {

dtb_status check_net(dtb_net* net) {
  if (!net) return fail(DTB_ERR_INVALID, "null handle");
  if (net->failed) return fail(DTB_ERR_STATE, "handle is in a failed state after an earlier HIP error");
  return DTB_OK;
}

dtb_status hip_fail(dtb_net* net, hipError_t e, const char* what) {
  net->failed = true;
  return fail(DTB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
dtb_status dalloc(dtb_net* net, T** p, size_t count) {
  void* q = nullptr;
  const size_t bytes = std::max<size_t>(1, count * sizeof(T));
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? DTB_ERR_OOM : DTB_ERR_HIP,
                "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
  }
  net->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return DTB_OK;
}

dtb_status validate(const dtb_desc* s) {
  if (!s) return fail(DTB_ERR_INVALID, "desc is NULL");
  if (s->n < 1 || s->n > kMaxNeurons)
    return fail(DTB_ERR_INVALID, "n must be in [1, " + std::to_string(kMaxNeurons) + "]");
  if (s->n_regions < 1) return fail(DTB_ERR_INVALID, "n_regions must be >= 1");
  if (s->max_delay < 1 || s->max_delay > kMaxDelay)
    return fail(DTB_ERR_INVALID, "max_delay must be in [1, 31]");
  if (s->n_ptypes < 1 || s->n_ptypes > 65536) return fail(DTB_ERR_INVALID, "n_ptypes must be in [1, 65536]");
  if (s->nnz < 0 || s->nnz > INT32_MAX) return fail(DTB_ERR_INVALID, "nnz must be in [0, 2^31-1]");
  if (!s->row_ptr || !s->is_inh || !s->region || !s->ptype || !s->ptypes || !s->V0)
    return fail(DTB_ERR_INVALID, "a required array pointer is NULL");
  if (s->nnz > 0 && (!s->col || !s->w || !s->delay))
    return fail(DTB_ERR_INVALID, "col/w/delay must be non-NULL when nnz > 0");
  if (s->wtype != DTB_W_F32 && s->wtype != DTB_W_BF16) return fail(DTB_ERR_INVALID, "unknown wtype");
  if (s->record_steps < 1) return fail(DTB_ERR_INVALID, "record_steps must be >= 1");
  if (s->gather_bundle_syn != 0 && (s->gather_bundle_syn < 4096 || s->gather_bundle_syn > kBundleMaxSyn))
    return fail(DTB_ERR_INVALID, "gather_bundle_syn must be 0 or in [4096, 2^20-1]");
  if (s->gather_unroll < 0 || s->gather_unroll > 3) return fail(DTB_ERR_INVALID, "gather_unroll must be 0 .. 3");
  if (s->gather_fuse < 0 || s->gather_fuse > 2) return fail(DTB_ERR_INVALID, "gather_fuse must be 0 .. 2");
  if (s->gather_events < 0 || s->gather_events > 2) return fail(DTB_ERR_INVALID, "gather_events must be 0 .. 2");
  if (!(s->dt_ms > 0.f) || !finite_f(s->dt_ms)) return fail(DTB_ERR_INVALID, "dt_ms must be finite and > 0");
  for (int u = 0; u < 4; ++u) {
    if (!(s->tau_ms[u] > 0.f) || !finite_f(s->tau_ms[u]))
      return fail(DTB_ERR_INVALID, "tau_ms[" + std::to_string(u) + "] must be finite and > 0");
    if (!finite_f(s->E[u])) return fail(DTB_ERR_INVALID, "E[" + std::to_string(u) + "] must be finite");
  }
  if (!(s->bg_w >= 0.f) || !finite_f(s->bg_w)) return fail(DTB_ERR_INVALID, "bg_w must be finite and >= 0");
  if (!(s->bg_lambda >= 0.0) || !(s->bg_lambda <= 400.0))
    return fail(DTB_ERR_INVALID, "bg_lambda must be in [0, 400]");
  if (s->row_ptr[0] != 0) return fail(DTB_ERR_INVALID, "row_ptr[0] must be 0");
  if (s->row_ptr[s->n] != s->nnz) return fail(DTB_ERR_INVALID, "row_ptr[n] must equal nnz");
  const int64_t n = s->n;
  int64_t bad = find_first(n, [&](int64_t i) { return s->row_ptr[i + 1] < s->row_ptr[i]; });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "row_ptr decreases at row " + std::to_string(bad));
  bad = find_first(s->nnz, [&](int64_t k) { return s->col[k] < 0 || int64_t(s->col[k]) >= n; });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "col out of range at synapse " + std::to_string(bad));
  bad = find_first(s->nnz, [&](int64_t k) { return s->delay[k] < 1 || s->delay[k] > s->max_delay; });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "delay out of [1, max_delay] at synapse " + std::to_string(bad));
  bad = find_first(s->nnz, [&](int64_t k) { return !(s->w[k] >= 0.f) || !finite_f(s->w[k]); });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "weight not finite and >= 0 at synapse " + std::to_string(bad));
  bad = find_first(n, [&](int64_t i) {
    return s->is_inh[i] > 1 || s->region[i] < 0 || s->region[i] >= s->n_regions ||
           int(s->ptype[i]) >= s->n_ptypes || !finite_f(s->V0[i]);
  });
  if (bad >= 0)
    return fail(DTB_ERR_INVALID, "neuron " + std::to_string(bad) + ": is_inh, region, ptype or V0 invalid");
  for (int p = 0; p < s->n_ptypes; ++p) {
    const dtb_ptype& q = s->ptypes[p];
    const float vals[] = {q.C, q.gL, q.EL, q.Vth, q.Vreset, q.tref_ms, q.Iext, q.g[0], q.g[1], q.g[2], q.g[3]};
    for (float v : vals)
      if (!finite_f(v)) return fail(DTB_ERR_INVALID, "ptype " + std::to_string(p) + " has a non-finite field");
    if (!(q.C > 0.f) || q.gL < 0.f || !(q.Vreset < q.Vth) || q.tref_ms < 0.f || q.g[0] < 0.f ||
        q.g[1] < 0.f || q.g[2] < 0.f || q.g[3] < 0.f)
      return fail(DTB_ERR_INVALID, "ptype " + std::to_string(p) +
                                       ": need C > 0, gL >= 0, Vreset < Vth, tref >= 0, g >= 0");
    if (std::lround(double(q.tref_ms) / double(s->dt_ms)) > 255)
      return fail(DTB_ERR_INVALID, "ptype " + std::to_string(p) + ": tref / dt must be <= 255 steps");
  }
  return DTB_OK;
}

dtb_status upload(dtb_net* net, void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, net->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy H2D");
  return DTB_OK;
}

// Run fn(b) for b in [0, n) on host threads with dynamic scheduling.
void parallel_items(int64_t n, const std::function<void(int64_t)>& fn) {
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<int64_t> next(0);
  auto work = [&] {
    for (int64_t b = next++; b < n; b = next++) fn(b);
  };
  if (nt == 1 || n < 2) {
    work();
    return;
  }
  std::vector<std::thread> th;
  for (unsigned q = 0; q < nt; ++q) th.emplace_back(work);
  for (auto& x : th) x.join();
}

// The connection table (Sec. V-D) in the gather's layout: rows cut into
// bundles, each bundle's synapses once in CSR order (weights, sign bit =
// inhibitory source) and once sorted by (delay, source) as 64-entry tiles of
// (source delta, CSR position) lookups (see dtb_internal.h).
// One in-edge block: n rows given by row_ptr / col / w / delay, sources
// marked inhibitory by src_inh[col]; bundle_syn as gather_bundle_syn.
struct BlockInput {
  int64_t n, nnz;
  const int64_t* row_ptr;
  const int32_t* col;
  const float* w;
  const uint8_t* delay;
  const uint8_t* src_inh;
  int32_t bundle_syn;
  bool events;      // spike-driven delivery table instead of the sorted lookup tiles
  int64_t n_src;    // sources (the event table's rows)
};

// Synapse k's stored weight as the row sums take it: |w| with the sign bit
// marking an inhibitory source, as FP32 bits, or as BF16 bits (w rounded
// to nearest even) in the high half.
uint32_t weight_bits(const BlockInput* s, int64_t k, bool bf16) {
  const bool inh = s->src_inh[s->col[k]] != 0;
  if (bf16) return uint32_t((f32_to_bf16_rne(s->w[k]) & 0x7FFFu) | (inh ? 0x8000u : 0u)) << 16;
  uint32_t u;
  std::memcpy(&u, &s->w[k], 4);
  return (u & 0x7FFFFFFFu) | (inh ? 0x80000000u : 0u);
}

// The spike-driven delivery table of a block: every synapse as the pair
// (bundle << kPosBits | position in its bundle, its weight bits), grouped by
// source and, inside a source, by delay, otherwise in CSR order (a stable
// counting sort on host threads): the deliveries of source m through delay
// d are entries [soff[m (D+1) + d - 1], soff[m (D+1) + d]).  Plus the
// per-bundle buckets the step's deliveries are sorted into.
dtb_status build_events(dtb_net* net, ConnBlock& cb, const BlockInput* s, const std::vector<Bundle>& bl) {
  const int D = net->d.max_delay;
  const bool bf16 = net->d.wtype == DTB_W_BF16;
  const int64_t nb = int64_t(bl.size()), nnz = s->nnz, ns = s->n_src;
  if (nb > kEventMaxBundles)
    return fail(DTB_ERR_UNSUPPORTED, "spike-driven delivery takes at most " + std::to_string(kEventMaxBundles) +
                                         " bundles (" + std::to_string(nb) + " here): raise gather_bundle_syn");
  const unsigned T = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // thread q takes bundles [cut[q], cut[q+1]) with about nnz / T synapses
  std::vector<int64_t> cut(T + 1, nb);
  cut[0] = 0;
  {
    int64_t b = 0, acc = 0;
    for (unsigned q = 1; q < T; ++q) {
      const int64_t goal = nnz * int64_t(q) / int64_t(T);
      while (b < nb && acc + bl[b].nsyn <= goal) acc += bl[b++].nsyn;
      cut[q] = b;
    }
  }
  auto on_threads = [&](const std::function<void(unsigned)>& fn) {
    std::vector<std::thread> th;
    for (unsigned q = 0; q < T; ++q) th.emplace_back([&fn, q] { fn(q); });
    for (auto& x : th) x.join();
  };
  std::vector<std::vector<uint32_t>> hist(T);
  on_threads([&](unsigned q) {
    hist[q].assign(size_t(ns), 0u);
    for (int64_t b = cut[q]; b < cut[q + 1]; ++b)
      for (int64_t k = bl[b].syn0; k < bl[b].syn0 + bl[b].nsyn; ++k) hist[q][s->col[k]]++;
  });
  // run starts per source, then each thread's place inside every run
  std::vector<uint32_t> start(size_t(ns) + 1, 0u);
  parallel_for(ns, [&](int64_t a, int64_t b) {
    for (int64_t m = a; m < b; ++m) {
      uint32_t c = 0;
      for (unsigned q = 0; q < T; ++q) c += hist[q][m];
      start[m + 1] = c;
    }
  });
  for (int64_t m = 0; m < ns; ++m) start[m + 1] += start[m];
  parallel_for(ns, [&](int64_t a, int64_t b) {
    for (int64_t m = a; m < b; ++m) {
      uint32_t o = start[m];
      for (unsigned q = 0; q < T; ++q) {
        const uint32_t c = hist[q][m];
        hist[q][m] = o;
        o += c;
      }
    }
  });
  // entry (low word) and weight bits (high word) of each pair
  std::vector<uint64_t> ent(size_t(std::max<int64_t>(1, nnz)));
  std::vector<uint8_t> dl(size_t(std::max<int64_t>(1, nnz)));
  on_threads([&](unsigned q) {
    for (int64_t b = cut[q]; b < cut[q + 1]; ++b)
      for (int64_t k = bl[b].syn0; k < bl[b].syn0 + bl[b].nsyn; ++k) {
        const uint32_t o = hist[q][s->col[k]]++;
        ent[o] = uint64_t((uint32_t(b) << kPosBits) | uint32_t(k - bl[b].syn0)) |
                 (uint64_t(weight_bits(s, k, bf16)) << 32);
        dl[o] = s->delay[k];
      }
  });
  std::vector<std::vector<uint32_t>>().swap(hist);
  // inside each source's run: stable by delay, and the (source, delay) runs
  std::vector<uint32_t> soff(size_t(ns) * (D + 1));
  parallel_for(ns, [&](int64_t a, int64_t b) {
    std::vector<uint64_t> tmp;
    uint32_t c[kMaxDelay + 2];
    for (int64_t m = a; m < b; ++m) {
      const uint32_t r0 = start[m], r1 = start[m + 1];
      std::fill(c, c + D + 2, 0u);
      for (uint32_t o = r0; o < r1; ++o) c[dl[o]]++;
      uint32_t* so = &soff[size_t(m) * (D + 1)];
      so[0] = r0;
      for (int d = 1; d <= D; ++d) so[d] = so[d - 1] + c[d];
      tmp.assign(ent.begin() + r0, ent.begin() + r1);
      uint32_t at[kMaxDelay + 1];
      for (int d = 1; d <= D; ++d) at[d] = so[d - 1];
      for (uint32_t o = r0; o < r1; ++o) ent[at[dl[o]]++] = tmp[o - r0];
    }
  });
  std::vector<uint8_t>().swap(dl);
  dtb_status st;
  if ((st = dalloc(net, &cb.ev_ent, 2 * std::max<int64_t>(1, nnz))) ||
      (st = dalloc(net, &cb.ev_soff, std::max<int64_t>(1, ns * (D + 1)))) ||
      (st = dalloc(net, &cb.evbuf, 2 * std::max<int64_t>(1, nnz))) || (st = dalloc(net, &cb.ev_cursor, nb)))
    return st;
  if ((st = upload(net, cb.ev_ent, ent.data(), size_t(nnz) * 8)) ||
      (st = upload(net, cb.ev_soff, soff.data(), soff.size() * 4)))
    return st;
  // every bucket starts empty: its cursor at the bundle's first synapse
  std::vector<uint32_t> cur(static_cast<size_t>(nb));
  for (int64_t b = 0; b < nb; ++b) cur[size_t(b)] = uint32_t(bl[size_t(b)].syn0);
  return upload(net, cb.ev_cursor, cur.data(), cur.size() * 4);
}

dtb_status build_block(dtb_net* net, ConnBlock& cb, const BlockInput* s) {
  const DeviceNet& d = net->d;
  const int64_t n = s->n;
  const std::vector<int64_t>& mrow = net->member_row0;
  // 1. bundles of consecutive rows
  const int64_t max_rows = std::min<int64_t>(65536, std::max<int64_t>(64, (n + 511) / 512));
  const int64_t max_syn = s->bundle_syn ? int64_t(s->bundle_syn) : kBundleDefaultSyn;
  std::vector<Bundle> bl;
  size_t mq = 0;  // member of row r
  for (int64_t r = 0; r < n;) {
    while (mq + 1 < mrow.size() && mrow[mq + 1] <= r) ++mq;
    const int64_t mend = mq + 1 < mrow.size() ? mrow[mq + 1] : n;  // bundles never cross members
    Bundle b{};
    b.row0 = r;
    b.syn0 = s->row_ptr[r];
    b.member_row0 = mrow[mq];
    b.member = net->member_id[mq];
    b.seed = net->member_seed[mq];
    while (r < mend && r - b.row0 < max_rows && s->row_ptr[r + 1] - b.syn0 <= max_syn) ++r;
    // with the default size, a longer row still gets a bundle of its own
    if (r == b.row0 && !s->bundle_syn && s->row_ptr[r + 1] - b.syn0 <= kBundleMaxSyn) ++r;
    if (r == b.row0)
      return fail(DTB_ERR_UNSUPPORTED, "row " + std::to_string(r) + " has more than " +
                                           std::to_string(max_syn) + " synapses (gather_bundle_syn)");
    b.row1 = r;
    b.nsyn = int32_t(s->row_ptr[r] - b.syn0);
    bl.push_back(b);
  }
  const int64_t nb = int64_t(bl.size());
  // 2. per bundle: sort by (delay, source, position) and cut into tiles
  // (the sweep's lookup stream; the spike-driven delivery does without)
  std::vector<std::vector<uint32_t>> btiles(nb), bheads(nb);
  if (!s->events) parallel_items(nb, [&](int64_t q) {
    const Bundle& b = bl[q];
    std::vector<uint64_t> key(size_t(b.nsyn));
    for (int32_t p = 0; p < b.nsyn; ++p) {
      const int64_t k = b.syn0 + p;
      key[p] = (uint64_t(s->delay[k] - 1) << 46) | (uint64_t(uint32_t(s->col[k])) << 20) | uint64_t(p);
    }
    std::sort(key.begin(), key.end());
    std::vector<uint32_t>& T = btiles[q];
    std::vector<uint32_t>& H = bheads[q];
    T.reserve(size_t(b.nsyn) + size_t(b.nsyn) / 16 + kTile);
    const uint32_t pad = uint32_t(b.nsyn);  // delta 0, position one past the last synapse
    int c = 0;
    uint32_t prev = 0, d1 = 0;
    for (uint64_t kk : key) {
      const uint32_t kd = uint32_t(kk >> 46), src = uint32_t((kk >> 20) & 0x3FFFFFFu);
      const uint32_t pos = uint32_t(kk & kPosMask);
      // a gap wider than one delta is bridged by skip entries (largest delta,
      // aimed at the padding bit) while that is cheaper than a fresh tile
      if (c > 0 && c < kTile && kd == d1 && src - prev > kMaxDelta && src - prev <= kMaxDelta * kMaxSkips) {
        while (src - prev > kMaxDelta && c < kTile) {
          T.push_back((kMaxDelta << kPosBits) | pad);
          prev += kMaxDelta;
          ++c;
        }
      }
      if (c == 0 || c == kTile || kd != d1 || src - prev > kMaxDelta) {
        while (c > 0 && c < kTile) {
          T.push_back(pad);
          ++c;
        }
        H.push_back(src | (kd << 26));
        prev = src;
        d1 = kd;
        c = 0;
      }
      T.push_back(((src - prev) << kPosBits) | pos);
      prev = src;
      ++c;
    }
    while (c > 0 && c < kTile) {
      T.push_back(pad);
      ++c;
    }
    // store each tile plane-major: lane l of a wavefront holds sorted entries
    // l, 64 + l, 128 + l, 192 + l, so each of its four bitmap loads covers 64
    // consecutive sources
    uint32_t tmp[kTile];
    for (size_t t0 = 0; t0 < T.size(); t0 += kTile) {
      for (int e = 0; e < kTile; ++e) tmp[(e & 63) * 4 + (e >> 6)] = T[t0 + e];
      std::copy(tmp, tmp + kTile, T.begin() + t0);
    }
  });
  int64_t ntiles = 0, hwords = 0;
  int32_t hw = 2 * (kGatherThreads / 64);  // the block totals reuse the hit bitmap's words
  for (int64_t q = 0; q < nb; ++q) {
    bl[q].tile0 = ntiles;
    bl[q].ntiles = int32_t(bheads[q].size());
    bl[q].hbit0 = 32 * hwords;  // each bundle's hit words start on a word of their own
    hwords += (bl[q].nsyn >> 5) + 1;
    ntiles += bl[q].ntiles;
    hw = std::max(hw, int32_t(bl[q].nsyn >> 5) + 1);
  }
  cb.n_bundles = nb;
  cb.n_tiles = ntiles;
  cb.hit_words = hw;
  cb.hit_total_words = hwords;
  // contiguous bundle ranges per XCD with about equal work: tiles of the
  // lookup stream (sweep) or synapses (spike-driven)
  int64_t xf[9];
  {
    auto work = [&](int64_t q) { return s->events ? int64_t(bl[q].nsyn) : int64_t(bl[q].ntiles); };
    int64_t tot = 0;
    for (int64_t q = 0; q < nb; ++q) tot += work(q);
    xf[0] = 0;
    int64_t acc = 0, q = 0;
    for (int x = 1; x < 8; ++x) {
      const int64_t goal = (tot * x + 7) / 8;
      while (q < nb && acc + work(q) <= goal) acc += work(q++);
      xf[x] = q;
    }
    xf[8] = nb;
    cb.xcd_max = 0;
    for (int x = 0; x < 8; ++x) cb.xcd_max = std::max(cb.xcd_max, xf[x + 1] - xf[x]);
  }
  // the bundle of each 1024-row block's first row (bundles are consecutive row ranges)
  const int64_t nblk = (n + 1023) / 1024;
  std::vector<int32_t> blk(size_t(std::max<int64_t>(1, nblk)), 0);
  {
    int64_t q = 0;
    for (int64_t b = 0; b < nblk; ++b) {
      while (bl[q].row1 <= b * 1024) ++q;
      blk[b] = int32_t(q);
    }
  }
  dtb_status st;
  const size_t wsz = d.wtype == DTB_W_BF16 ? 2 : 4;
  if ((st = dalloc(net, &cb.bundles, nb)) || (st = dalloc(net, &cb.tiles, std::max<int64_t>(1, ntiles) * kTile)) ||
      (st = dalloc(net, &cb.hitbuf, std::max<int64_t>(1, hwords))) ||
      (st = dalloc(net, &cb.block_bundle, int64_t(blk.size()))) || (st = dalloc(net, &cb.xcd_first, 9)) ||
      (st = dalloc(net, &cb.theads, std::max<int64_t>(1, ntiles))) || (st = dalloc(net, &cb.row_ptr, n + 1)))
    return st;
  {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(1, size_t(s->nnz) * wsz));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(DTB_ERR_OOM, "hipMalloc of weights failed");
    }
    net->allocs.push_back(q);
    cb.wts = q;
  }
  if ((st = upload(net, cb.bundles, bl.data(), nb * sizeof(Bundle))) ||
      (st = upload(net, cb.block_bundle, blk.data(), blk.size() * sizeof(int32_t))) ||
      (st = upload(net, cb.xcd_first, xf, sizeof(xf))) ||
      (st = upload(net, cb.row_ptr, s->row_ptr, (n + 1) * sizeof(int64_t))))
    return st;
  for (int64_t q = 0; q < nb; ++q) {
    if (bl[q].ntiles == 0) continue;
    if ((st = upload(net, cb.tiles + bl[q].tile0 * kTile, btiles[q].data(), btiles[q].size() * 4)) ||
        (st = upload(net, cb.theads + bl[q].tile0, bheads[q].data(), bheads[q].size() * 4)))
      return st;
    std::vector<uint32_t>().swap(btiles[q]);
    std::vector<uint32_t>().swap(bheads[q]);
  }
  if (s->events && (st = build_events(net, cb, s, bl))) return st;
  // 3. weights in CSR order with the sign bit marking an inhibitory source
  const int64_t chunk = int64_t(1) << 26;
  std::vector<uint8_t> hwt;
  for (int64_t k0 = 0; k0 < s->nnz; k0 += chunk) {
    const int64_t k1 = std::min<int64_t>(s->nnz, k0 + chunk);
    hwt.assign(size_t(k1 - k0) * wsz, 0);
    parallel_for(k1 - k0, [&](int64_t a, int64_t b) {
      for (int64_t q = a; q < b; ++q) {
        const uint32_t u = weight_bits(s, k0 + q, wsz == 2);
        if (wsz == 4) {
          std::memcpy(&hwt[q * 4], &u, 4);
        } else {
          const uint16_t h = uint16_t(u >> 16);
          std::memcpy(&hwt[q * 2], &h, 2);
        }
      }
    });
    if ((st = upload(net, static_cast<uint8_t*>(cb.wts) + k0 * wsz, hwt.data(), hwt.size()))) return st;
  }
  return DTB_OK;
}

dtb_status build_connections(dtb_net* net, const dtb_desc* s) {
  BlockInput in{s->n, s->nnz, s->row_ptr, s->col, s->w, s->delay, s->is_inh, s->gather_bundle_syn,
                net->d.events != 0, s->n};
  return build_block(net, net->d.loc, &in);
}

// launch `fn`, bracketed by a pair of events when timing is on
template <typename F>
hipError_t timed(dtb_net* net, int kind, F fn, hipStream_t st = nullptr) {
  if (!net->timing) return fn();
  if (!st) st = net->stream;
  auto& pool = net->ev_pool[kind];
  if (net->ev_used[kind] == pool.size()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    pool.emplace_back(a, b);
  }
  auto& pr = pool[net->ev_used[kind]++];
  hipError_t e = hipEventRecord(pr.first, st);
  if (e == hipSuccess) e = fn();
  if (e == hipSuccess) e = hipEventRecord(pr.second, st);
  return e;
}

// Kernel arguments are captured by value in a graph: parameter changes drop it.
void drop_graph(dtb_net* net) {
  if (net->graph_exec) (void)hipGraphExecDestroy(net->graph_exec);
  if (net->graph) (void)hipGraphDestroy(net->graph);
  net->graph_exec = nullptr;
  net->graph = nullptr;
  net->graph_steps = 0;
}

// The step's Poisson background counts go to the second stream: forked
// after the neuron update is enqueued (the previous step's row sums, their
// only reader, are done by then) and joined before this step's gather, so
// the ALU-bound draw shares the CUs with the latency-bound compaction and
// bucketing (one bucketing workgroup per CU leaves room beside it).
bool background_on(const DeviceNet& d) { return !d.ou_on && d.loc.n_bundles > 0; }

hipError_t fork_background(dtb_net* net, bool capturing) {
  if (!background_on(net->d)) return hipSuccess;
  hipError_t e = hipEventRecord(net->bg_fork, net->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(net->comm, net->bg_fork, 0);
  if (e == hipSuccess)
    e = capturing ? launch_background(net->d, net->comm)
                  : timed(net, 8, [&] { return launch_background(net->d, net->comm); }, net->comm);
  if (e == hipSuccess) e = hipEventRecord(net->bg_join, net->comm);
  return e;
}

hipError_t join_background(dtb_net* net) {
  return background_on(net->d) ? hipStreamWaitEvent(net->stream, net->bg_join, 0) : hipSuccess;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

int dtb_abi_version(void) { return DTB_ABI_VERSION; }

const char* dtb_last_error(void) { return g_err.c_str(); }

int64_t dtb_bitmap_words(int64_t n) { return n <= 0 ? 0 : (n + 31) / 32; }

void dtb_destroy(dtb_net* net) {
  if (!net) return;
  (void)hipStreamSynchronize(net->stream);
  if (net->comm) {
    (void)hipStreamSynchronize(net->comm);
    (void)hipStreamDestroy(net->comm);
  }
  if (net->fork_ev) (void)hipEventDestroy(net->fork_ev);
  if (net->join_ev) (void)hipEventDestroy(net->join_ev);
  if (net->bg_fork) (void)hipEventDestroy(net->bg_fork);
  if (net->bg_join) (void)hipEventDestroy(net->bg_join);
  for (auto& pool : net->ev_pool)
    for (auto& pr : pool) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  if (net->graph_exec) (void)hipGraphExecDestroy(net->graph_exec);
  if (net->graph) (void)hipGraphDestroy(net->graph);
  for (void* p : net->allocs) (void)hipFree(p);
  if (net->own_stream) (void)hipStreamDestroy(net->stream);
  delete net;
}

// Build a handle from a validated description; `net` already carries the
// member table (one member for a plain partition).
static dtb_status create_impl(const dtb_desc* desc, dtb_net* net, void* hip_stream, dtb_net** out) {
  dtb_status st;
  {
    hipError_t e = gather_set_lds_limit();
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(DTB_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
  }
  net->stream = static_cast<hipStream_t>(hip_stream);
  if (!net->stream) {
    // graph capture needs a non-default stream: use a private blocking stream,
    // which the legacy default stream still orders against
    hipError_t e = hipStreamCreate(&net->stream);
    if (e != hipSuccess) {
      delete net;
      return fail(DTB_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    net->own_stream = true;
  }
  {
    hipError_t e = hipStreamCreate(&net->comm);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&net->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&net->join_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&net->bg_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&net->bg_join, hipEventDisableTiming);
    if (e != hipSuccess) {
      dtb_destroy(net);
      return fail(DTB_ERR_HIP, std::string("second stream: ") + hipGetErrorString(e));
    }
  }
  net->dt_ms = desc->dt_ms;
  DeviceNet& d = net->d;
  d.dt_ms = desc->dt_ms;
  d.n = desc->n;
  d.n_pad = round_up(desc->n, kNeuronPad);
  d.words = dtb_bitmap_words(desc->n);
  d.words_pad = d.n_pad / 32;
  d.nnz = desc->nnz;
  d.n_regions = desc->n_regions;
  d.max_delay = desc->max_delay;
  d.n_ptypes = desc->n_ptypes;
  d.member = desc->member;
  d.wtype = desc->wtype;
  d.unroll = desc->gather_unroll ? desc->gather_unroll : kGatherUnroll;
  d.fuse = desc->gather_fuse ? desc->gather_fuse : 1;
  d.events = desc->gather_events == 2 ? 1 : 0;
  d.id_slots = d.events ? desc->max_delay + 1 : 1;
  d.rec = desc->record_steps;
  d.slots = std::max(d.rec, d.max_delay) + 1;
  d.bg_w = desc->bg_w;
  d.seed = desc->seed;
  d.compact_blocks = (d.words_pad + kCompactWords * kCompactBlock - 1) / (kCompactWords * kCompactBlock);
  for (int u = 0; u < 4; ++u) {
    d.a[u] = float(std::exp(-double(desc->dt_ms) / double(desc->tau_ms[u])));
    d.E[u] = desc->E[u];
  }
  std::vector<uint32_t> T(kMaxPoisson);
  d.poisson_K = poisson_thresholds(desc->bg_lambda, T.data(), kMaxPoisson);
  if (d.poisson_K < 0) {
    dtb_destroy(net);
    return fail(DTB_ERR_INVALID, "bg_lambda needs more than 512 inversion-table entries");
  }
  const int64_t slots = int64_t(d.slots);
  d.poisson_cap = std::max(1, d.poisson_K);
  if ((st = dalloc(net, &d.V, d.n_pad)) || (st = dalloc(net, &d.V0, d.n_pad)) || (st = dalloc(net, &d.bgc, d.n_pad)) ||
      (st = dalloc(net, &d.j, 4 * d.n_pad)) ||
      (st = dalloc(net, &d.ref, d.n_pad)) || (st = dalloc(net, &d.ptype, d.n_pad)) ||
      (st = dalloc(net, &d.region, d.n_pad)) ||
      (st = dalloc(net, &d.ptab, d.n_ptypes)) || (st = dalloc(net, &d.gain, 4 * d.n_regions)) ||
      (st = dalloc(net, &d.poisson, std::max(1, d.poisson_K))) ||
      (st = dalloc(net, &d.raster, slots * d.words_pad)) ||
      (st = dalloc(net, &d.counts, slots * d.n_regions)) || (st = dalloc(net, &d.ev, slots * kStripes * 2)) ||
      (st = dalloc(net, &d.totals, 4)) || (st = dalloc(net, &d.ids, int64_t(d.id_slots) * d.n_pad)) ||
      (st = dalloc(net, &d.id_count, d.id_slots)) || (st = dalloc(net, &d.cstatus, d.compact_blocks)) ||
      (st = dalloc(net, &d.cticket, 1)) || (st = dalloc(net, &d.force, (d.rec + 1) * d.words_pad)) ||
      (st = dalloc(net, &d.bad, 1)) || (st = dalloc(net, &d.step, 2)) ||
      (st = dalloc(net, &d.inv_nr_dt, d.n_regions)) || (st = dalloc(net, &d.bold, 4 * d.n_regions)) ||
      (st = dalloc(net, &d.bold_y, d.n_regions)) || (st = dalloc(net, &d.rd_at, 2)) ||
      (st = dalloc(net, &d.rd_ids, d.n_pad)) || (st = dalloc(net, &d.rd_count, 1)) ||
      (st = dalloc(net, &d.rd_status, d.compact_blocks)) || (st = dalloc(net, &d.rd_ticket, 1)) ||
      (st = dalloc(net, &d.rd_total, 1))) {
    dtb_destroy(net);
    return st;
  }
  if (d.events) {
    // gathered run offsets for up to an eighth of the neurons spiking in a step
    d.run_cap = std::max<int64_t>(64, (d.n_pad / 8 + 63) / 64 * 64);
    if ((st = dalloc(net, &d.run_off, int64_t(d.id_slots) * (d.max_delay + 1) * d.run_cap)) ||
        (st = dalloc(net, &d.run_n, d.id_slots))) {
      dtb_destroy(net);
      return st;
    }
  }
  auto zero = [&](void* p, size_t bytes) { return hipMemsetAsync(p, 0, bytes, net->stream); };
  hipError_t e = hipSuccess;
  for (auto pr : std::vector<std::pair<void*, size_t>>{
           {d.j, 4 * d.n_pad * sizeof(float)}, {d.ref, size_t(d.n_pad)},
           {d.raster, slots * d.words_pad * 4}, {d.counts, slots * d.n_regions * 4},
           {d.ev, slots * kStripes * 2 * 8}, {d.totals, 32}, {d.id_count, size_t(d.id_slots) * 4},
           {d.cstatus, d.compact_blocks * 8}, {d.cticket, 4}, {d.bad, 4}, {d.ptype, d.n_pad * 2},
           {d.region, d.n_pad * 4}, {d.V, d.n_pad * 4}, {d.step, 16}, {d.bold, size_t(d.n_regions) * 16},
           {d.bold_y, size_t(d.n_regions) * 4}, {d.rd_status, d.compact_blocks * 8}, {d.rd_count, 4},
           {d.run_n, d.run_n ? size_t(d.id_slots) * 4 : 0}}) {
    if (e == hipSuccess && pr.second) e = zero(pr.first, pr.second);
  }
  if (e != hipSuccess) {
    st = fail(DTB_ERR_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    dtb_destroy(net);
    return st;
  }
  // property table: derived per-type constants
  std::vector<PType> pt(d.n_ptypes);
  for (int p = 0; p < d.n_ptypes; ++p) {
    const dtb_ptype& q = desc->ptypes[p];
    pt[p].dtC = float(double(desc->dt_ms) / double(q.C));
    pt[p].gL = q.gL;
    pt[p].EL = q.EL;
    pt[p].Vth = q.Vth;
    pt[p].Vreset = q.Vreset;
    pt[p].Iext = q.Iext;
    for (int u = 0; u < 4; ++u) pt[p].g[u] = q.g[u];
    pt[p].nref = int32_t(std::lround(double(q.tref_ms) / double(desc->dt_ms)));
    pt[p].pad = 0;
  }
  std::vector<float> gain(4 * d.n_regions, 1.0f);
  net->region_n.assign(d.n_regions, 0);
  for (int64_t i = 0; i < d.n; ++i) net->region_n[desc->region[i]]++;
  std::vector<float> inr(d.n_regions, 0.f);
  for (int r = 0; r < d.n_regions; ++r)
    if (net->region_n[r] > 0) inr[r] = float(1.0 / (double(net->region_n[r]) * double(desc->dt_ms) * 1e-3));
  if ((st = upload(net, d.ptab, pt.data(), pt.size() * sizeof(PType))) ||
      (st = upload(net, d.gain, gain.data(), gain.size() * 4)) ||
      (st = upload(net, d.inv_nr_dt, inr.data(), inr.size() * 4)) ||
      (st = upload(net, d.poisson, T.data(), std::max(1, d.poisson_K) * 4)) ||
      (st = upload(net, d.V, desc->V0, d.n * 4)) || (st = upload(net, d.V0, desc->V0, d.n * 4)) ||
      (st = upload(net, d.ptype, desc->ptype, d.n * 2)) ||
      (st = upload(net, d.region, desc->region, d.n * 4)) || (st = build_connections(net, desc))) {
    dtb_destroy(net);
    return st;
  }
  *out = net;
  return DTB_OK;
}

dtb_status dtb_create(const dtb_desc* desc, void* hip_stream, dtb_net** out) {
  if (!out) return fail(DTB_ERR_INVALID, "out is NULL");
  *out = nullptr;
  dtb_status st = validate(desc);
  if (st) return st;
  dtb_net* net = new (std::nothrow) dtb_net();
  if (!net) return fail(DTB_ERR_OOM, "host allocation failed");
  net->member_row0 = {0};
  net->member_region0 = {0, desc->n_regions};
  net->member_id = {desc->member};
  net->member_seed = {desc->seed};
  return create_impl(desc, net, hip_stream, out);
}

dtb_status dtb_create_batch(const dtb_desc* members, int32_t n_members, void* hip_stream, dtb_net** out) {
  if (!out) return fail(DTB_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!members || n_members < 1) return fail(DTB_ERR_INVALID, "need at least one member");
  const dtb_desc& m0 = members[0];
  int64_t n = 0, nnz = 0;
  int64_t R = 0, P = 0;
  int32_t D = 0;
  for (int32_t m = 0; m < n_members; ++m) {
    const dtb_desc& q = members[m];
    dtb_status st = validate(&q);
    if (st) return fail(st, "member " + std::to_string(m) + ": " + g_err);
    bool same = q.dt_ms == m0.dt_ms && q.bg_w == m0.bg_w && q.bg_lambda == m0.bg_lambda &&
                q.wtype == m0.wtype && q.record_steps == m0.record_steps;
    for (int u = 0; u < 4; ++u) same = same && q.E[u] == m0.E[u] && q.tau_ms[u] == m0.tau_ms[u];
    if (!same)
      return fail(DTB_ERR_UNSUPPORTED, "member " + std::to_string(m) +
                                           ": E, tau, dt, background rate and weight, wtype and record_steps must match member 0");
    n += q.n;
    nnz += q.nnz;
    R += q.n_regions;
    P += q.n_ptypes;
    D = std::max(D, q.max_delay);
  }
  if (n > kMaxNeurons) return fail(DTB_ERR_INVALID, "members exceed the neuron limit together");
  if (nnz > INT32_MAX) return fail(DTB_ERR_INVALID, "members exceed 2^31-1 synapses together");
  if (R > INT32_MAX || P > 65536) return fail(DTB_ERR_INVALID, "members exceed the population / type limits");
  // the batch is one block-diagonal partition
  std::vector<int64_t> row_ptr(n + 1);
  std::vector<int32_t> col(nnz), region(n);
  std::vector<float> w(nnz), V0(n);
  std::vector<uint8_t> delay(nnz), is_inh(n);
  std::vector<uint16_t> ptype(n);
  std::vector<dtb_ptype> ptypes(P);
  dtb_net* net = new (std::nothrow) dtb_net();
  if (!net) return fail(DTB_ERR_OOM, "host allocation failed");
  int64_t i0 = 0, k0 = 0;
  int32_t r0 = 0, p0 = 0;
  for (int32_t m = 0; m < n_members; ++m) {
    const dtb_desc& q = members[m];
    net->member_row0.push_back(i0);
    net->member_region0.push_back(r0);
    net->member_id.push_back(q.member);
    net->member_seed.push_back(q.seed);
    parallel_for(q.nnz, [&](int64_t a, int64_t b) {
      for (int64_t k = a; k < b; ++k) {
        col[k0 + k] = int32_t(q.col[k] + i0);
        w[k0 + k] = q.w[k];
        delay[k0 + k] = q.delay[k];
      }
    });
    for (int64_t i = 0; i < q.n; ++i) {
      row_ptr[i0 + i] = q.row_ptr[i] + k0;
      region[i0 + i] = q.region[i] + r0;
      ptype[i0 + i] = uint16_t(q.ptype[i] + p0);
      is_inh[i0 + i] = q.is_inh[i];
      V0[i0 + i] = q.V0[i];
    }
    for (int32_t p = 0; p < q.n_ptypes; ++p) ptypes[p0 + p] = q.ptypes[p];
    i0 += q.n;
    k0 += q.nnz;
    r0 += q.n_regions;
    p0 += q.n_ptypes;
  }
  row_ptr[n] = nnz;
  net->member_region0.push_back(r0);
  dtb_desc all = m0;
  all.n = n;
  all.nnz = nnz;
  all.n_regions = int32_t(R);
  all.n_ptypes = int32_t(P);
  all.max_delay = D;
  all.row_ptr = row_ptr.data();
  all.col = col.data();
  all.w = w.data();
  all.delay = delay.data();
  all.is_inh = is_inh.data();
  all.region = region.data();
  all.ptype = ptype.data();
  all.ptypes = ptypes.data();
  all.V0 = V0.data();
  all.member = 0;
  return create_impl(&all, net, hip_stream, out);
}

dtb_status dtb_batch_info(dtb_net* net, int32_t* n_members, int64_t* neuron_offset, int32_t* region_offset,
                          int32_t cap) {
  dtb_status st = check_net(net);
  if (st) return st;
  const int32_t M = int32_t(net->member_row0.size());
  if (n_members) *n_members = M;
  for (int32_t m = 0; m <= std::min(M, cap); ++m) {
    if (neuron_offset) neuron_offset[m] = m < M ? net->member_row0[m] : net->d.n;
    if (region_offset) region_offset[m] = net->member_region0[m];
  }
  return DTB_OK;
}

dtb_status dtb_set_gains(dtb_net* net, const float* gains, int src_on_device) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (!gains) return fail(DTB_ERR_INVALID, "gains is NULL");
  const size_t bytes = size_t(net->d.n_regions) * 16;
  if (!src_on_device) {
    for (int64_t q = 0; q < int64_t(net->d.n_regions) * 4; ++q)
      if (!(gains[q] >= 0.f) || !finite_f(gains[q]))
        return fail(DTB_ERR_INVALID, "gain " + std::to_string(q) + " is not finite and >= 0");
  }
  hipError_t e = hipMemcpyAsync(net->d.gain, gains, bytes,
                                src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, net->stream);
  if (e == hipSuccess && !src_on_device) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy gains");
  return DTB_OK;
}

dtb_status dtb_read_bold(dtb_net* net, float* y, float* sfvq, int dst_on_device) {
  dtb_status st = check_net(net);
  if (st) return st;
  const DeviceNet& d = net->d;
  if (sfvq && dst_on_device) return fail(DTB_ERR_UNSUPPORTED, "the hemodynamic state is read into host memory");
  if (y) {
    hipError_t e = hipMemcpyAsync(y, d.bold_y, size_t(d.n_regions) * 4,
                                  dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, net->stream);
    if (e == hipSuccess && !dst_on_device) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy bold");
  }
  if (sfvq) {
    hipError_t e = hipMemcpyAsync(sfvq, d.bold, size_t(d.n_regions) * 16, hipMemcpyDeviceToHost, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy bold state");
    for (int64_t r = 0; r < d.n_regions; ++r)
      for (int c = 1; c < 4; ++c) sfvq[4 * r + c] += 1.f;  // stored as deviations from rest
  }
  return DTB_OK;
}

dtb_status dtb_set_timing(dtb_net* net, int enable) {
  dtb_status st = check_net(net);
  if (st) return st;
  net->timing = enable != 0;
  return DTB_OK;
}

dtb_status dtb_read_timing(dtb_net* net, double* ms, int64_t* launches) {
  dtb_status st = check_net(net);
  if (st) return st;
  hipError_t e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipStreamSynchronize");
  for (int k = 0; k < kTimedKernels; ++k) {
    double sum = 0.0;
    for (size_t q = 0; q < net->ev_used[k]; ++q) {
      float x = 0.f;
      e = hipEventElapsedTime(&x, net->ev_pool[k][q].first, net->ev_pool[k][q].second);
      if (e != hipSuccess) return hip_fail(net, e, "hipEventElapsedTime");
      sum += x;
    }
    if (ms) ms[k] = sum;
    if (launches) launches[k] = int64_t(net->ev_used[k]);
    net->ev_used[k] = 0;
  }
  return DTB_OK;
}

dtb_status dtb_step(dtb_net* net, int32_t n_steps) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (n_steps < 0) return fail(DTB_ERR_INVALID, "n_steps must be >= 0");
  DeviceNet& d = net->d;
  for (int32_t q = 0; q < n_steps; ++q) {
    const int64_t t = net->t;
    if (net->remote && net->rq_pending == 0)
      return fail(DTB_ERR_STATE, "no remote spikes pushed for step " + std::to_string(t));
    const uint32_t* forced = nullptr;
    if (net->force_pending > 0) {
      forced = d.force + (net->force_head % (d.rec + 1)) * d.words_pad;
      net->force_head++;
      net->force_pending--;
    }
    hipError_t e = hipSuccess;
    if (net->remote) {
      // the arrival of this step's remote spikes on the second stream (the
      // pushed bitmap from the queue into the remote ring: where an exchange
      // would land them), concurrent with the update, compaction and J_intra
      const uint32_t* row = d.rqueue + (net->rq_head % (d.rec + 1)) * d.rwords_pad;
      e = hipEventRecord(net->fork_ev, net->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(net->comm, net->fork_ev, 0);
      if (e == hipSuccess)
        e = launch_copy_words(d.rraster + (t % d.slots) * d.rwords_pad, row, d.rwords_pad, net->comm);
      if (e == hipSuccess) e = hipEventRecord(net->join_ev, net->comm);
      if (e != hipSuccess) return hip_fail(net, e, "remote block launch");
      net->rq_head++;
      net->rq_pending--;
    }
    if (e == hipSuccess) e = timed(net, 0, [&] { return launch_neuron_update(d, forced, net->stream); });
    if (e == hipSuccess) e = fork_background(net, false);
    if (e == hipSuccess) e = timed(net, 1, [&] { return launch_compact(d, net->stream); });
    // the gather workgroups also sum their rows (fuse == 1) unless a remote
    // block is set: then both blocks' hit bits go to k_sums (local, then
    // remote)
    const bool fuse = !net->remote && d.fuse == 1;
    if (d.events) {
      // spike-driven delivery: the step's deliveries into per-bundle buckets,
      // then each bundle's hit bitmap from its bucket
      if (e == hipSuccess) e = timed(net, 7, [&] { return launch_spike_runs(d, net->stream); });
      if (e == hipSuccess) e = timed(net, 6, [&] { return launch_events(d, net->stream); });
      if (e == hipSuccess) e = join_background(net);
      if (e == hipSuccess) e = timed(net, 2, [&] { return launch_gather_events(d, fuse, net->stream); });
    } else {
      if (e == hipSuccess) e = join_background(net);
      if (e == hipSuccess)
        e = timed(net, 2, [&] { return launch_gather(d, d.loc, d.raster, d.words_pad, fuse, net->stream); });
    }
    if (e == hipSuccess && net->remote) {
      // J_inter after J_intra, once the remote spikes are in (the paper's
      // computing-thread order); its delivery tests OR into their own hit
      // buffer
      e = hipStreamWaitEvent(net->stream, net->join_ev, 0);
      if (e == hipSuccess)
        e = timed(net, 5, [&] { return launch_gather(d, d.rem, d.rraster, d.rwords_pad, false, net->stream); });
    }
    if (e == hipSuccess && !fuse) e = timed(net, 3, [&] { return launch_sums(d, net->stream); });
    if (e == hipSuccess) e = timed(net, 4, [&] { return launch_finalize(d, net->stream); });
    if (e != hipSuccess) return hip_fail(net, e, "kernel launch");
    net->t = t + 1;
  }
  return DTB_OK;
}

dtb_status dtb_run(dtb_net* net, int32_t n_steps) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (n_steps < 0) return fail(DTB_ERR_INVALID, "n_steps must be >= 0");
  if (net->force_pending) return fail(DTB_ERR_STATE, "teacher forcing is pending: use dtb_step");
  if (net->remote)
    return fail(DTB_ERR_UNSUPPORTED, "a remote in-edge block takes one pushed bitmap per step: use dtb_step");
  if (n_steps == 0) return DTB_OK;
  DeviceNet& d = net->d;
  hipError_t e = hipSuccess;
  if (!net->graph_exec || net->graph_steps != n_steps) {
    if (net->graph_exec) (void)hipGraphExecDestroy(net->graph_exec);
    if (net->graph) (void)hipGraphDestroy(net->graph);
    net->graph_exec = nullptr;
    net->graph = nullptr;
    e = hipStreamBeginCapture(net->stream, hipStreamCaptureModeThreadLocal);
    for (int32_t q = 0; q < n_steps && e == hipSuccess; ++q) {
      e = launch_neuron_update(d, nullptr, net->stream);
      if (e == hipSuccess) e = fork_background(net, true);
      if (e == hipSuccess) e = launch_compact(d, net->stream);
      if (d.events) {
        if (e == hipSuccess) e = launch_spike_runs(d, net->stream);
        if (e == hipSuccess) e = launch_events(d, net->stream);
      }
      if (e == hipSuccess) e = join_background(net);
      if (e == hipSuccess) {
        e = d.events ? launch_gather_events(d, d.fuse == 1, net->stream)
                     : launch_gather(d, d.loc, d.raster, d.words_pad, d.fuse == 1, net->stream);
      }
      if (e == hipSuccess && d.fuse != 1) e = launch_sums(d, net->stream);
      if (e == hipSuccess) e = launch_finalize(d, net->stream);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(net->stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&net->graph_exec, g, nullptr, nullptr, 0);
    net->graph = g;
    if (e != hipSuccess) return hip_fail(net, e, "graph capture of the step sequence");
    net->graph_steps = n_steps;
  }
  e = hipGraphLaunch(net->graph_exec, net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipGraphLaunch");
  net->t += n_steps;
  return DTB_OK;
}

dtb_status dtb_reset(dtb_net* net) {
  dtb_status st = check_net(net);
  if (st) return st;
  DeviceNet& d = net->d;
  const size_t slots = size_t(d.slots);
  hipError_t e = hipMemcpyAsync(d.V, d.V0, d.n_pad * 4, hipMemcpyDeviceToDevice, net->stream);
  for (auto pr : std::vector<std::pair<void*, size_t>>{
           {d.j, 4 * d.n_pad * sizeof(float)}, {d.ref, size_t(d.n_pad)}, {d.raster, slots * d.words_pad * 4},
           {d.counts, slots * d.n_regions * 4}, {d.ev, slots * kStripes * 2 * 8}, {d.totals, 32},
           {d.id_count, size_t(d.id_slots) * 4}, {d.cstatus, d.compact_blocks * 8}, {d.cticket, 4}, {d.bad, 4},
           {d.step, 16},
           {d.bold, size_t(d.n_regions) * 16}, {d.bold_y, size_t(d.n_regions) * 4},
           {d.run_n, d.run_n ? size_t(d.id_slots) * 4 : 0}}) {
    if (e == hipSuccess && pr.second) e = hipMemsetAsync(pr.first, 0, pr.second, net->stream);
  }
  if (e == hipSuccess && d.ou_on) e = launch_fill(d.ou, d.n_pad, d.ou_mu, net->stream);
  if (e == hipSuccess && net->remote) e = launch_copy_words(d.rraster, nullptr, slots * d.rwords_pad, net->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "reset");
  net->t = 0;
  net->force_pending = 0;
  net->force_head = 0;
  net->rq_pending = 0;
  net->rq_head = 0;
  return DTB_OK;
}

dtb_status dtb_set_background(dtb_net* net, double bg_lambda, float bg_w) {
  dtb_status st = check_net(net);
  if (st) return st;
  // validate and build the table before touching the handle: a rejected
  // call leaves the drive as it was
  if (!(bg_lambda >= 0.0) || !(bg_lambda <= 400.0)) return fail(DTB_ERR_INVALID, "bg_lambda must be in [0, 400]");
  if (!(bg_w >= 0.f) || !finite_f(bg_w)) return fail(DTB_ERR_INVALID, "bg_w must be finite and >= 0");
  std::vector<uint32_t> T(kMaxPoisson);
  const int K = poisson_thresholds(bg_lambda, T.data(), kMaxPoisson);
  if (K < 0) return fail(DTB_ERR_INVALID, "bg_lambda needs more than 512 inversion-table entries");
  DeviceNet& d = net->d;
  if (K > d.poisson_cap) {
    uint32_t* q = nullptr;
    if ((st = dalloc(net, &q, K))) return st;
    d.poisson = q;
    d.poisson_cap = K;
  }
  // the table is read by kernels already queued: replace it in stream order
  if (K > 0 && (st = upload(net, d.poisson, T.data(), size_t(K) * 4))) return st;
  drop_graph(net);
  d.ou_on = 0;
  d.poisson_K = K;
  d.bg_w = bg_w;
  return DTB_OK;
}

dtb_status dtb_set_background_ou(dtb_net* net, float mu, float sigma, float tau_ms) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (!finite_f(mu) || !finite_f(sigma) || !(sigma >= 0.f) || !finite_f(tau_ms) || !(tau_ms > 0.f))
    return fail(DTB_ERR_INVALID, "need finite mu, sigma >= 0 and tau_ms > 0");
  DeviceNet& d = net->d;
  drop_graph(net);
  if (!d.ou && (st = dalloc(net, &d.ou, d.n_pad))) return st;
  const double a = std::exp(-double(d.dt_ms) / double(tau_ms));
  d.ou_mu = mu;
  d.ou_a = float(a);
  d.ou_s = float(double(sigma) * std::sqrt(1.0 - a * a));
  d.ou_on = 1;
  d.poisson_K = 0;  // the Poisson drive is off
  hipError_t e = launch_fill(d.ou, d.n_pad, mu, net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "OU current fill");
  return DTB_OK;
}

dtb_status dtb_force_spikes(dtb_net* net, const uint32_t* bits, int32_t n_steps) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (n_steps < 0 || (n_steps > 0 && !bits)) return fail(DTB_ERR_INVALID, "bad bits / n_steps");
  DeviceNet& d = net->d;
  if (net->force_pending + n_steps > d.rec)
    return fail(DTB_ERR_INVALID, "more forced steps pending than record_steps");
  if (net->force_pending == 0) net->force_head = 0;
  std::vector<uint32_t> row(d.words_pad, 0u);
  for (int32_t q = 0; q < n_steps; ++q) {
    std::memcpy(row.data(), bits + size_t(q) * d.words, d.words * 4);
    const int64_t slot = (net->force_head + net->force_pending) % (d.rec + 1);
    hipError_t e = hipMemcpyAsync(d.force + slot * d.words_pad, row.data(), d.words_pad * 4,
                                  hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy forced spikes");
    net->force_pending++;
  }
  return DTB_OK;
}

dtb_status dtb_set_remote_block(dtb_net* net, int64_t n_remote, int64_t nnz, const int64_t* row_ptr,
                                const int32_t* col, const float* w, const uint8_t* delay,
                                const uint8_t* remote_is_inh) {
  dtb_status st = check_net(net);
  if (st) return st;
  DeviceNet& d = net->d;
  if (net->remote) return fail(DTB_ERR_STATE, "the remote block is already set");
  if (net->t != 0) return fail(DTB_ERR_STATE, "set the remote block before the first step (or after dtb_reset)");
  if (net->member_row0.size() != 1) return fail(DTB_ERR_UNSUPPORTED, "a remote block needs a single-member handle");
  if (n_remote < 1 || n_remote > (int64_t(1) << 26) - 1)
    return fail(DTB_ERR_INVALID, "n_remote must be in [1, 2^26 - 1]");
  if (nnz < 0 || !row_ptr || (nnz > 0 && (!col || !w || !delay)) || !remote_is_inh)
    return fail(DTB_ERR_INVALID, "null remote block array");
  if (row_ptr[0] != 0 || row_ptr[d.n] != nnz) return fail(DTB_ERR_INVALID, "row_ptr must run from 0 to nnz");
  int64_t bad = find_first(d.n, [&](int64_t i) { return row_ptr[i + 1] < row_ptr[i]; });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "row_ptr decreases at row " + std::to_string(bad));
  bad = find_first(nnz, [&](int64_t k) { return col[k] < 0 || int64_t(col[k]) >= n_remote; });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "remote col out of range at synapse " + std::to_string(bad));
  bad = find_first(nnz, [&](int64_t k) { return delay[k] < 1 || delay[k] > d.max_delay; });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "delay out of [1, max_delay] at synapse " + std::to_string(bad));
  bad = find_first(nnz, [&](int64_t k) { return !(finite_f(w[k]) && w[k] >= 0.f); });
  if (bad >= 0) return fail(DTB_ERR_INVALID, "weight not finite and >= 0 at synapse " + std::to_string(bad));
  BlockInput in{d.n, nnz, row_ptr, col, w, delay, remote_is_inh, 0, false, n_remote};
  if ((st = build_block(net, d.rem, &in))) return st;
  d.n_remote = n_remote;
  d.rwords_pad = round_up(n_remote, kNeuronPad) / 32;
  if ((st = dalloc(net, &d.rraster, int64_t(d.slots) * d.rwords_pad)) ||
      (st = dalloc(net, &d.rqueue, (d.rec + 1) * d.rwords_pad)))
    return st;
  hipError_t e = launch_copy_words(d.rraster, nullptr, int64_t(d.slots) * d.rwords_pad, net->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "remote block set-up");
  drop_graph(net);
  net->remote = true;
  net->rq_head = 0;
  net->rq_pending = 0;
  return DTB_OK;
}

dtb_status dtb_push_remote_spikes(dtb_net* net, const uint32_t* bits, int32_t n_steps) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (!net->remote) return fail(DTB_ERR_STATE, "no remote block set");
  if (n_steps < 0 || (n_steps > 0 && !bits)) return fail(DTB_ERR_INVALID, "bad bits / n_steps");
  DeviceNet& d = net->d;
  if (net->rq_pending + n_steps > d.rec)
    return fail(DTB_ERR_INVALID, "more remote steps pending than record_steps");
  if (net->rq_pending == 0) net->rq_head = 0;
  const int64_t rw = dtb_bitmap_words(d.n_remote);
  const uint32_t tail = (d.n_remote & 31) ? (1u << (d.n_remote & 31)) - 1u : ~0u;
  std::vector<uint32_t> rows(size_t(n_steps) * d.rwords_pad, 0u);
  for (int32_t q = 0; q < n_steps; ++q) {
    uint32_t* r = rows.data() + size_t(q) * d.rwords_pad;
    std::memcpy(r, bits + size_t(q) * rw, size_t(rw) * 4);
    r[rw - 1] &= tail;  // bits past n_remote are not neurons
  }
  for (int32_t q = 0; q < n_steps; ++q) {
    const int64_t slot = (net->rq_head + net->rq_pending) % (d.rec + 1);
    hipError_t e = hipMemcpyAsync(d.rqueue + slot * d.rwords_pad, rows.data() + size_t(q) * d.rwords_pad,
                                  d.rwords_pad * 4, hipMemcpyHostToDevice, net->stream);
    if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy remote spikes");
    net->rq_pending++;
  }
  hipError_t e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy remote spikes");
  return DTB_OK;
}

dtb_status dtb_enkf_analysis(int32_t n_members, int32_t n_params, int32_t n_obs, float* X, const float* Y,
                             const float* y_obs, const float* r_var, float inflation, uint64_t seed, int64_t iter,
                             float lo, float hi, void* hip_stream) {
  if (!X || !Y || !y_obs || !r_var) return fail(DTB_ERR_INVALID, "null EnKF array");
  if (n_members < 2 || n_params < 1 || n_obs < 1 || n_obs > kEnkfMaxObs)
    return fail(DTB_ERR_INVALID, "EnKF needs n_members >= 2, n_params >= 1, 1 <= n_obs <= 64");
  if (!(inflation >= 1.f) || !finite_f(inflation) || !(lo <= hi) || !finite_f(lo) || !finite_f(hi))
    return fail(DTB_ERR_INVALID, "EnKF needs a finite inflation >= 1 and finite lo <= hi");
  EnkfVar rv{};
  for (int o = 0; o < n_obs; ++o) {
    if (!(r_var[o] > 0.f) || !finite_f(r_var[o])) return fail(DTB_ERR_INVALID, "r_var must be finite and > 0");
    rv.r[o] = r_var[o];
  }
  if (enkf_lds_bytes(n_members, n_params, n_obs) > size_t(160) * 1024)
    return fail(DTB_ERR_UNSUPPORTED, "EnKF sizes exceed the 160 KB of LDS (8 (P + O + O^2 + P O + M O) bytes)");
  hipError_t e = launch_enkf(n_members, n_params, n_obs, X, Y, y_obs, rv, double(inflation), seed, iter, lo, hi,
                             static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(DTB_ERR_HIP, std::string("EnKF launch: ") + hipGetErrorString(e));
  return DTB_OK;
}

static dtb_status window(dtb_net* net, int64_t t0, int64_t t1) {
  if (t0 < 0 || t1 < t0 || t1 > net->t || t0 < net->t - net->d.rec)
    return fail(DTB_ERR_INVALID, "window [" + std::to_string(t0) + ", " + std::to_string(t1) +
                                     ") outside the recorded steps");
  return DTB_OK;
}

static dtb_status copy_out(dtb_net* net, void* dst, const void* src, size_t bytes, int on_device) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                net->stream);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy read");
  return DTB_OK;
}

// Rows t0 .. t1-1 of a per-step ring (row of step t at slot t mod slots,
// src_pitch bytes apart, `width` bytes each) into dst rows dst_pitch bytes
// apart: at most two strided copies (the window wraps the ring at most once).
static dtb_status copy_ring_window(dtb_net* net, void* dst, size_t dst_pitch, const void* ring, size_t src_pitch,
                                   size_t width, int64_t t0, int64_t t1, int on_device) {
  const int64_t S = net->d.slots;
  hipError_t e = hipSuccess;
  for (int64_t t = t0; t < t1 && e == hipSuccess;) {
    const int64_t slot = t % S;
    const int64_t rows = std::min<int64_t>(t1 - t, S - slot);
    e = hipMemcpy2DAsync(static_cast<char*>(dst) + size_t(t - t0) * dst_pitch, dst_pitch,
                         static_cast<const char*>(ring) + size_t(slot) * src_pitch, src_pitch, width, size_t(rows),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, net->stream);
    t += rows;
  }
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy2D read");
  return DTB_OK;
}

dtb_status dtb_read_spikes(dtb_net* net, int64_t t0, int64_t t1, uint32_t* dst, int dst_on_device) {
  dtb_status st = check_net(net);
  if (st || (st = window(net, t0, t1))) return st;
  if (!dst && t1 > t0) return fail(DTB_ERR_INVALID, "dst is NULL");
  const DeviceNet& d = net->d;
  if (t1 == t0 || d.words == 0) return DTB_OK;
  return copy_ring_window(net, dst, size_t(d.words) * 4, d.raster, size_t(d.words_pad) * 4, size_t(d.words) * 4, t0,
                          t1, dst_on_device);
}

dtb_status dtb_read_spike_ids(dtb_net* net, int64_t t, int32_t* ids, int64_t cap, int64_t* count) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (!count || cap < 0 || (cap > 0 && !ids)) return fail(DTB_ERR_INVALID, "bad ids / cap / count");
  if ((st = window(net, t, t + 1))) return st;
  DeviceNet& d = net->d;
  const int64_t islot = t % d.id_slots;  // step t's list, while it is the last step
  const int32_t* src_ids = d.ids + islot * d.n_pad;
  const int32_t* src_count = d.id_count + islot;
  if (t != net->t - 1) {
    // an earlier step: rebuild its list from the step's ring slot with the
    // same compaction kernel, on the read's own look-back words
    const int64_t at[2] = {net->read_epoch, t % d.slots};
    hipError_t e = hipMemcpyAsync(d.rd_at, at, sizeof(at), hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d.rd_ticket, 0, 4, net->stream);
    if (e == hipSuccess)
      e = launch_compact_read(d, d.rd_at, d.rd_ids, d.rd_count, d.rd_status, d.rd_ticket, d.rd_total, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);  // `at` lives until here
    if (e != hipSuccess) return hip_fail(net, e, "spike-list rebuild");
    net->read_epoch++;
    src_ids = d.rd_ids;
    src_count = d.rd_count;
  }
  int32_t c = 0;
  if ((st = copy_out(net, &c, src_count, 4, 0))) return st;
  *count = c;
  const int64_t m = std::min<int64_t>(c, cap);
  if (m > 0 && (st = copy_out(net, ids, src_ids, size_t(m) * 4, 0))) return st;
  return DTB_OK;
}

dtb_status dtb_read_state(dtb_net* net, int32_t field, float* dst, int dst_on_device) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (!dst) return fail(DTB_ERR_INVALID, "dst is NULL");
  const DeviceNet& d = net->d;
  if (field == DTB_V) return copy_out(net, dst, d.V, d.n * 4, dst_on_device);
  if (field == DTB_I_OU) {
    if (d.ou_on) return copy_out(net, dst, d.ou, d.n * 4, dst_on_device);
    if (dst_on_device) {
      hipError_t e = hipMemsetAsync(dst, 0, d.n * 4, net->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
      if (e != hipSuccess) return hip_fail(net, e, "hipMemsetAsync");
    } else {
      std::memset(dst, 0, d.n * 4);
    }
    return DTB_OK;
  }
  if (field >= DTB_J_AMPA && field <= DTB_J_GABAB)
    return copy_out(net, dst, d.j + (field - 1) * d.n_pad, d.n * 4, dst_on_device);
  if (field == DTB_REF) {
    std::vector<uint8_t> r(d.n);
    if ((st = copy_out(net, r.data(), d.ref, d.n, 0))) return st;
    std::vector<float> f(r.begin(), r.end());
    if (dst_on_device) {
      hipError_t e = hipMemcpy(dst, f.data(), d.n * 4, hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(net, e, "hipMemcpy");
    } else {
      std::memcpy(dst, f.data(), d.n * 4);
    }
    return DTB_OK;
  }
  return fail(DTB_ERR_INVALID, "unknown field");
}

dtb_status dtb_read_region_counts(dtb_net* net, int64_t t0, int64_t t1, int32_t* dst) {
  dtb_status st = check_net(net);
  if (st || (st = window(net, t0, t1))) return st;
  if (!dst && t1 > t0) return fail(DTB_ERR_INVALID, "dst is NULL");
  const DeviceNet& d = net->d;
  if (t1 == t0) return DTB_OK;
  const size_t row = size_t(d.n_regions) * 4;
  return copy_ring_window(net, dst, row, d.counts, row, row, t0, t1, 0);
}

dtb_status dtb_read_region_rates(dtb_net* net, int64_t t0, int64_t t1, float* hz) {
  dtb_status st = check_net(net);
  if (st || (st = window(net, t0, t1))) return st;
  if (!hz) return fail(DTB_ERR_INVALID, "hz is NULL");
  const int R = net->d.n_regions;
  std::vector<int32_t> c(size_t(std::max<int64_t>(1, t1 - t0)) * R, 0);
  if (t1 > t0 && (st = dtb_read_region_counts(net, t0, t1, c.data()))) return st;
  for (int r = 0; r < R; ++r) {
    int64_t s = 0;
    for (int64_t q = 0; q < t1 - t0; ++q) s += c[q * R + r];
    const double denom = double(net->region_n[r]) * double(t1 - t0) * double(net->dt_ms) * 1e-3;
    hz[r] = denom > 0 ? float(double(s) / denom) : 0.f;
  }
  return DTB_OK;
}

dtb_status dtb_read_step_events(dtb_net* net, int64_t t0, int64_t t1, int64_t* ev_rec, int64_t* ev_bg) {
  dtb_status st = check_net(net);
  if (st || (st = window(net, t0, t1))) return st;
  const DeviceNet& d = net->d;
  if (t1 == t0) return DTB_OK;
  // each slot's final totals are its first (rec, bg) pair
  std::vector<int64_t> v(size_t(t1 - t0) * 2);
  if ((st = copy_ring_window(net, v.data(), 16, d.ev, size_t(kStripes) * 2 * 8, 16, t0, t1, 0))) return st;
  for (int64_t t = t0; t < t1; ++t) {
    if (ev_rec) ev_rec[t - t0] = v[2 * (t - t0)];
    if (ev_bg) ev_bg[t - t0] = v[2 * (t - t0) + 1];
  }
  return DTB_OK;
}

dtb_status dtb_read_counters(dtb_net* net, int64_t* steps, int64_t* spikes, int64_t* ev_rec, int64_t* ev_bg) {
  dtb_status st = check_net(net);
  if (st) return st;
  int64_t v[4];
  if ((st = copy_out(net, v, net->d.totals, 32, 0))) return st;
  if (steps) *steps = v[3];
  if (spikes) *spikes = v[0];
  if (ev_rec) *ev_rec = v[1];
  if (ev_bg) *ev_bg = v[2];
  return DTB_OK;
}

// ------------------------------------------------------ checkpoint / resume
}  // extern "C"

namespace {
struct SaveHeader {
  char magic[8];
  int32_t abi, wtype;
  int64_t n, n_pad, words_pad, slots, n_regions, rec, members, n_remote, rwords_pad;
  int64_t t, total_bytes;
  int32_t poisson_K, ou_on;
  float bg_w, ou_mu, ou_a, ou_s;
};
constexpr char kSaveMagic[8] = {'D', 'T', 'B', 'S', 'T', 'A', 'T', '1'};

// the handle's dynamic state, in file order: (device pointer, bytes)
std::vector<std::pair<void*, size_t>> state_sections(const dtb_net* net, int32_t ou_on) {
  const DeviceNet& d = net->d;
  const size_t slots = size_t(d.slots), R = size_t(d.n_regions), np = size_t(d.n_pad);
  std::vector<std::pair<void*, size_t>> v = {
      {d.V, np * 4},           {d.j, 4 * np * 4},
      {d.ref, np},             {d.gain, 4 * R * 4},
      {d.raster, slots * size_t(d.words_pad) * 4},
      {d.counts, slots * R * 4}, {d.ev, slots * kStripes * 2 * 8},
      {d.totals, 4 * 8},       {d.step, 2 * 8},
      {d.bold, 4 * R * 4},     {d.bold_y, R * 4}};
  if (ou_on) v.emplace_back(d.ou, np * 4);
  if (net->remote) v.emplace_back(d.rraster, slots * size_t(d.rwords_pad) * 4);
  return v;
}
}  // namespace

extern "C" {

dtb_status dtb_save(dtb_net* net, void* host_buf, size_t cap, size_t* used) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (!used) return fail(DTB_ERR_INVALID, "used is NULL");
  const DeviceNet& d = net->d;
  if (net->force_pending || net->rq_pending)
    return fail(DTB_ERR_STATE, "teacher forcing or remote spikes are pending: step them first");
  const int32_t ou_on = d.ou_on && d.ou ? 1 : 0;
  const auto sec = state_sections(net, ou_on);
  size_t total = sizeof(SaveHeader) + size_t(d.poisson_K) * 4;
  for (auto& x : sec) total += x.second;
  *used = total;
  if (!host_buf) return DTB_OK;  // size query
  if (cap < total) return fail(DTB_ERR_INVALID, "buffer smaller than the state (" + std::to_string(total) + " B)");
  SaveHeader h{};
  std::memcpy(h.magic, kSaveMagic, 8);
  h.abi = DTB_ABI_VERSION;
  h.wtype = d.wtype;
  h.n = d.n;
  h.n_pad = d.n_pad;
  h.words_pad = d.words_pad;
  h.slots = d.slots;
  h.n_regions = d.n_regions;
  h.rec = d.rec;
  h.members = int64_t(net->member_row0.size());
  h.n_remote = net->remote ? d.n_remote : 0;
  h.rwords_pad = net->remote ? d.rwords_pad : 0;
  h.t = net->t;
  h.total_bytes = int64_t(total);
  h.poisson_K = d.poisson_K;
  h.ou_on = ou_on;
  h.bg_w = d.bg_w;
  h.ou_mu = d.ou_mu;
  h.ou_a = d.ou_a;
  h.ou_s = d.ou_s;
  uint8_t* out = static_cast<uint8_t*>(host_buf);
  std::memcpy(out, &h, sizeof(h));
  size_t off = sizeof(h);
  hipError_t e = hipSuccess;
  if (d.poisson_K > 0)
    e = hipMemcpyAsync(out + off, d.poisson, size_t(d.poisson_K) * 4, hipMemcpyDeviceToHost, net->stream);
  off += size_t(d.poisson_K) * 4;
  for (auto& x : sec) {
    if (e == hipSuccess) e = hipMemcpyAsync(out + off, x.first, x.second, hipMemcpyDeviceToHost, net->stream);
    off += x.second;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "save");
  return DTB_OK;
}

dtb_status dtb_load(dtb_net* net, const void* host_buf, size_t len) {
  dtb_status st = check_net(net);
  if (st) return st;
  if (!host_buf || len < sizeof(SaveHeader)) return fail(DTB_ERR_INVALID, "buffer too short for a saved state");
  SaveHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  DeviceNet& d = net->d;
  if (std::memcmp(h.magic, kSaveMagic, 8) != 0 || h.abi != DTB_ABI_VERSION)
    return fail(DTB_ERR_INVALID, "not a saved state of this library version");
  if (h.wtype != d.wtype || h.n != d.n || h.n_pad != d.n_pad || h.words_pad != d.words_pad || h.slots != d.slots ||
      h.n_regions != d.n_regions || h.rec != d.rec || h.members != int64_t(net->member_row0.size()) ||
      h.n_remote != (net->remote ? d.n_remote : 0) || h.rwords_pad != (net->remote ? d.rwords_pad : 0))
    return fail(DTB_ERR_INVALID, "the saved state belongs to a handle of another shape");
  if (h.total_bytes < 0 || size_t(h.total_bytes) > len) return fail(DTB_ERR_INVALID, "truncated saved state");
  if (h.poisson_K < 0 || h.poisson_K > kMaxPoisson || h.t < 0 || h.ou_on < 0 || h.ou_on > 1)
    return fail(DTB_ERR_INVALID, "corrupt saved state header");
  size_t total = sizeof(SaveHeader) + size_t(h.poisson_K) * 4;
  for (auto& x : state_sections(net, h.ou_on)) total += x.second;  // sizes only (d.ou may not exist yet)
  if (size_t(h.total_bytes) != total) return fail(DTB_ERR_INVALID, "saved state size does not match");
  // background settings (kernel arguments: the captured graph is dropped)
  drop_graph(net);
  if (h.poisson_K > d.poisson_cap) {
    uint32_t* q = nullptr;
    if ((st = dalloc(net, &q, h.poisson_K))) return st;
    d.poisson = q;
    d.poisson_cap = h.poisson_K;
  }
  if (h.ou_on && !d.ou && (st = dalloc(net, &d.ou, d.n_pad))) return st;
  const uint8_t* in = static_cast<const uint8_t*>(host_buf);
  size_t off = sizeof(h);
  hipError_t e = hipSuccess;
  if (h.poisson_K > 0)
    e = hipMemcpyAsync(d.poisson, in + off, size_t(h.poisson_K) * 4, hipMemcpyHostToDevice, net->stream);
  off += size_t(h.poisson_K) * 4;
  for (auto& x : state_sections(net, h.ou_on)) {
    if (e == hipSuccess) e = hipMemcpyAsync(x.first, in + off, x.second, hipMemcpyHostToDevice, net->stream);
    off += x.second;
  }
  // compaction look-back words and the failure flag start clean
  if (e == hipSuccess) e = hipMemsetAsync(d.cstatus, 0, size_t(d.compact_blocks) * 8, net->stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.cticket, 0, 4, net->stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.bad, 0, 4, net->stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.id_count, 0, size_t(d.id_slots) * 4, net->stream);
  // the rebuilt lists have no gathered run offsets: their spikes' runs are
  // read from the table directly
  if (e == hipSuccess && d.run_n) e = hipMemsetAsync(d.run_n, 0, size_t(d.id_slots) * 4, net->stream);
  // the spike-id lists still needed (the last step's; with spike-driven
  // delivery the last D steps') are rebuilt from the restored bitmaps
  const int64_t keep = d.id_slots == 1 ? 1 : int64_t(d.max_delay);
  for (int64_t q = std::max<int64_t>(0, h.t - keep); q < h.t && e == hipSuccess; ++q) {
    const int64_t at[2] = {net->read_epoch++, q % d.slots};
    const int64_t sl = q % d.id_slots;
    e = hipMemcpyAsync(d.rd_at, at, sizeof(at), hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d.rd_ticket, 0, 4, net->stream);
    if (e == hipSuccess)
      e = launch_compact_read(d, d.rd_at, d.ids + sl * d.n_pad, d.id_count + sl, d.rd_status, d.rd_ticket,
                              d.rd_total, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);  // `at` lives until here
  }
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "load");
  d.poisson_K = h.poisson_K;
  d.bg_w = h.bg_w;
  d.ou_on = h.ou_on;
  d.ou_mu = h.ou_mu;
  d.ou_a = h.ou_a;
  d.ou_s = h.ou_s;
  net->t = h.t;
  net->force_pending = 0;
  net->force_head = 0;
  net->rq_pending = 0;
  net->rq_head = 0;
  return DTB_OK;
}

// ------------------------------------------------------- launch autotuner
}  // extern "C"

namespace {

struct TuneEntry {
  int32_t bundle_syn = 0, unroll = 0, fuse = 0, events = 0;
  double ms = 0.0;
};

// Cache file: one JSON object, one entry per line,
//   "<arch>|n=<n>,nnz=<nnz>,members=<m>,w=<f32|bf16>,D=<D>":
//       {"bundle_syn": b, "unroll": u, "fuse": f, "events": v, "ms_per_step": ms}
// Lines that do not parse are dropped when the file is rewritten.
std::map<std::string, TuneEntry> read_tune_cache(const char* path) {
  std::map<std::string, TuneEntry> db;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    if (a == std::string::npos) continue;
    const size_t b = line.find('"', a + 1);
    if (b == std::string::npos) continue;
    TuneEntry e;
    const char* rest = line.c_str() + b + 1;
    if (std::sscanf(rest, " : {\"bundle_syn\": %d, \"unroll\": %d, \"fuse\": %d, \"events\": %d, \"ms_per_step\": %lf",
                    &e.bundle_syn, &e.unroll, &e.fuse, &e.events, &e.ms) == 5)
      db[line.substr(a + 1, b - a - 1)] = e;
  }
  return db;
}

bool write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& db) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\n";
    size_t q = 0;
    for (const auto& kv : db) {
      char buf[224];
      std::snprintf(buf, sizeof(buf),
                    ": {\"bundle_syn\": %d, \"unroll\": %d, \"fuse\": %d, \"events\": %d, \"ms_per_step\": %.6f}",
                    kv.second.bundle_syn, kv.second.unroll, kv.second.fuse, kv.second.events, kv.second.ms);
      f << "\"" << kv.first << "\"" << buf << (++q < db.size() ? ",\n" : "\n");
    }
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

dtb_status dtb_autotune(const dtb_desc* members, int32_t n_members, void* hip_stream, const char* cache_path,
                        const int32_t* bundle_cands, int32_t n_cands, int32_t burnin, int32_t steps,
                        dtb_tune_result* out) {
  if (!out) return fail(DTB_ERR_INVALID, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!members || n_members < 1) return fail(DTB_ERR_INVALID, "need at least one member");
  if (n_cands < 0 || n_cands > DTB_TUNE_MAX_BUNDLES || (n_cands > 0 && !bundle_cands))
    return fail(DTB_ERR_INVALID, "n_cands must be in [0, " + std::to_string(DTB_TUNE_MAX_BUNDLES) + "]");
  for (int32_t q = 0; q < n_cands; ++q)
    if (bundle_cands[q] < 4096 || int64_t(bundle_cands[q]) > kBundleMaxSyn)
      return fail(DTB_ERR_INVALID, "bundle candidate " + std::to_string(q) + " outside [4096, 2^20-1]");
  if (burnin < 0 || steps < 1) return fail(DTB_ERR_INVALID, "need burnin >= 0 and steps >= 1");
  int64_t n = 0, nnz = 0;
  int32_t D = 0;
  for (int32_t m = 0; m < n_members; ++m) {
    n += members[m].n;
    nnz += members[m].nnz;
    D = std::max(D, members[m].max_delay);
  }
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fail(DTB_ERR_HIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  const std::string key = arch + "|n=" + std::to_string(n) + ",nnz=" + std::to_string(nnz) +
                          ",members=" + std::to_string(n_members) +
                          ",w=" + (members[0].wtype == DTB_W_BF16 ? "bf16" : "f32") + ",D=" + std::to_string(D);
  if (cache_path) {
    const auto db = read_tune_cache(cache_path);
    const auto it = db.find(key);
    if (it != db.end()) {
      out->bundle_syn = it->second.bundle_syn;
      out->unroll = it->second.unroll;
      out->fuse = it->second.fuse;
      out->events = it->second.events;
      out->ms_per_step = float(it->second.ms);
      out->from_cache = 1;
      return DTB_OK;
    }
  }
  // candidate bundle sizes: the caller's, or the largest bundle and sizes
  // whose bundle count fills whole rounds of the CUs (one workgroup per CU)
  std::vector<int32_t> cands(bundle_cands, bundle_cands + n_cands);
  if (cands.empty()) {
    cands.push_back(int32_t(kBundleMaxSyn));
    const double L = n > 0 ? double(nnz) / double(n) : 1.0;
    const int64_t ncu = std::max(1, prop.multiProcessorCount);
    const int64_t k0 = std::max<int64_t>(1, (nnz + kBundleMaxSyn * ncu - 1) / (kBundleMaxSyn * ncu));
    for (int64_t k = k0; k < k0 + 3 && int32_t(cands.size()) < DTB_TUNE_MAX_BUNDLES; ++k) {
      const int64_t rows = (n + k * ncu - 1) / (k * ncu);
      const int64_t b = int64_t(double(rows) * L + 0.5);
      if (b >= 4096 && b <= kBundleMaxSyn && std::find(cands.begin(), cands.end(), int32_t(b)) == cands.end())
        cands.push_back(int32_t(b));
    }
  }
  // the spike-driven delivery also tries sizes whose bundles leave room in
  // the LDS for their carried weights (hit bitmaps of at most 2^19 bits)
  std::vector<int32_t> ev_cands = cands;
  if (n_cands == 0) {
    constexpr int64_t kCarrySyn = (int64_t(1) << 19) - 1;
    const double L = n > 0 ? double(nnz) / double(n) : 1.0;
    const int64_t ncu = std::max(1, prop.multiProcessorCount);
    const int64_t k0 = std::max<int64_t>(1, (nnz + kCarrySyn * ncu - 1) / (kCarrySyn * ncu));
    for (int64_t k = k0; k < k0 + 3; ++k) {
      const int64_t rows = (n + k * ncu - 1) / (k * ncu);
      const int64_t b = int64_t(double(rows) * L + 0.5);
      if (b >= 4096 && b <= kCarrySyn && std::find(ev_cands.begin(), ev_cands.end(), int32_t(b)) == ev_cands.end())
        ev_cands.push_back(int32_t(b));
    }
  }
  std::vector<dtb_desc> ds(members, members + n_members);
  std::vector<uint8_t> saved;
  hipEvent_t ea = nullptr, eb = nullptr;
  e = hipEventCreate(&ea);
  if (e == hipSuccess) e = hipEventCreate(&eb);
  if (e != hipSuccess) {
    if (ea) (void)hipEventDestroy(ea);
    return fail(DTB_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
  }
  dtb_status st = DTB_OK;
  // per candidate bundle size: the sweep with 1..3 tiles per round and either
  // placement of the row sums, then the spike-driven delivery with either
  // placement (when the bundles fit its 4096 ids)
  for (size_t c = 0; c < ev_cands.size() && st == DTB_OK; ++c) {
    for (int32_t mode = c < cands.size() ? 1 : 2; mode <= 2 && st == DTB_OK; ++mode) {
      for (auto& x : ds) {
        x.gather_bundle_syn = ev_cands[c];
        x.gather_unroll = 0;
        x.gather_fuse = 0;
        x.gather_events = mode;
      }
      dtb_net* net = nullptr;
      st = n_members == 1 ? dtb_create(ds.data(), hip_stream, &net)
                          : dtb_create_batch(ds.data(), n_members, hip_stream, &net);
      if (st == DTB_ERR_UNSUPPORTED && mode == 2) {  // too many bundles for the event table
        st = DTB_OK;
        continue;
      }
      if (st) break;
      if (saved.empty()) {
        // one burned-in state shared by every candidate: each times the same steps
        size_t used = 0;
        if (!(st = dtb_step(net, burnin)) && !(st = dtb_save(net, nullptr, 0, &used))) {
          saved.resize(used);
          st = dtb_save(net, saved.data(), saved.size(), &used);
        }
      }
      const int32_t nv = mode == 1 ? 6 : 2;
      for (int32_t v = 0; v < nv && st == DTB_OK; ++v) {
        const int32_t u = mode == 1 ? 1 + v % 3 : 0, fz = mode == 1 ? 1 + v / 3 : 1 + v;
        net->d.unroll = u ? u : kGatherUnroll;
        net->d.fuse = fz;
        drop_graph(net);
        if ((st = dtb_load(net, saved.data(), saved.size()))) break;
        e = hipEventRecord(ea, net->stream);
        if (e == hipSuccess && (st = dtb_step(net, steps))) break;
        if (e == hipSuccess) e = hipEventRecord(eb, net->stream);
        if (e == hipSuccess) e = hipEventSynchronize(eb);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
        if (e != hipSuccess) {
          st = fail(DTB_ERR_HIP, std::string("autotune timing: ") + hipGetErrorString(e));
          break;
        }
        const int q = out->n_tried++;
        out->tried_bundle[q] = ev_cands[c];
        out->tried_unroll[q] = u;
        out->tried_fuse[q] = fz;
        out->tried_events[q] = mode;
        out->tried_ms[q] = ms / float(steps);
        if (q == 0 || out->tried_ms[q] < out->ms_per_step) {
          out->bundle_syn = ev_cands[c];
          out->unroll = u;
          out->fuse = fz;
          out->events = mode;
          out->ms_per_step = out->tried_ms[q];
        }
      }
      dtb_destroy(net);
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (st) return st;
  if (cache_path) {
    auto db = read_tune_cache(cache_path);
    db[key] = TuneEntry{out->bundle_syn, out->unroll, out->fuse, out->events, double(out->ms_per_step)};
    if (!write_tune_cache(cache_path, db))
      return fail(DTB_ERR_INVALID, std::string("cannot write the tuning cache ") + cache_path);
  }
  return DTB_OK;
}

dtb_status dtb_sync(dtb_net* net) {
  dtb_status st = check_net(net);
  if (st) return st;
  hipError_t e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) return hip_fail(net, e, "hipStreamSynchronize");
  int32_t bad = 0;
  if ((st = copy_out(net, &bad, net->d.bad, 4, 0))) return st;
  if (bad) {
    e = hipMemsetAsync(net->d.bad, 0, 4, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) return hip_fail(net, e, "hipMemset");
    return fail(DTB_ERR_NUMERIC, "non-finite membrane potential or gate produced");
  }
  return DTB_OK;
}

}  // extern "C"
