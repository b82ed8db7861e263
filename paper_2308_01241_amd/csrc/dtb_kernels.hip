// dtb_kernels.hip - gfx950 kernels of one partition step.
//
// A step t is, in stream order (the computing cycle of Sec. V-B / VI-C):
//   k_neuron_update  membrane update of Eq. (1) by forward Euler (Sec. VI-A),
//                    threshold / reset / refractory, wavefront ballot into
//                    the step's spike bitmap (a slot of the delay ring of
//                    bitmaps), per-population spike counts;
//   k_background     (on the library's second stream, joined before the
//                    gather) the step's Poisson counts that stand in for the
//                    spikes of other partitions (J_inter), one Philox block
//                    per eight neurons;
//   k_compact        ascending spike-id list from the bitmap (ballot
//                    popcounts, block scan, decoupled look-back);
//   k_spike_runs,    spike-driven delivery only: the table run offsets of
//   k_events         the step's spikes, then the deliveries of the spikes of
//                    the last D steps bucketed per bundle;
//   k_gather         the hit bitmap per bundle of J_intra - from the pull
//                    over each row's in-edges through the delay ring, in
//                    (delay, source) order, or from the bundle's bucket;
//                    then, in the same workgroup, per row: delivered weights
//                    in CSR order, the background count, the gate update
//                    (jump + exact decay);
//   k_sums           the per-row part alone, when a remote in-edge block
//                    is gathered too (local, then remote, then background);
//   k_finalize       per-step event totals, BOLD, ring slot, step counter.
//
// Everything is FP32 except the integer work (ids, delays, ballots, counts,
// RNG).  The file is compiled with -ffp-contract=off: every fused
// multiply-add below is written out, so the arithmetic is the source's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dtb_internal.h"

namespace dtb {
namespace {

// ------------------------------------------------------------------ RNG
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 64x64 -> 128-bit products, key bumped by the Weyl constants between rounds.
// the four output words of counter (c0, c1, c2, c3), key (k0, k1)
__device__ inline void philox_block(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                                    uint64_t (&out)[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t y0 = hi1 ^ c1 ^ k0, y2 = hi0 ^ c3 ^ k1;
    c0 = y0;
    c1 = lo1;
    c2 = y2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// the high 32 bits of output word 0; *w1 (if given) receives output word 1
__device__ inline uint64_t philox_hi32_word0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                             uint64_t k0, uint64_t k1, uint64_t* w1 = nullptr) {
  uint64_t out[4];
  philox_block(c0, c1, c2, c3, k0, k1, out);
  if (w1) *w1 = out[1];
  return out[0] >> 32;
}

__device__ inline int poisson_count(uint32_t u, const uint32_t* __restrict__ T, int K) {
  int c = 0;
  while (c < K && u >= T[c]) ++c;
  return c;
}

// ------------------------------------------------------------- background
// The step's Poisson background counts, eight neurons per Philox block:
// group g of a member network's neurons (its neurons 8g .. 8g + 7) draws
// counter (t, g, member, 0), key (the member's seed, 0); the block's four
// words give eight 32-bit values (a word's high half, then its low half),
// neuron 8g + j takes value j and inverts it against the table (staged in
// LDS).  One workgroup per bundle (a bundle lies inside one member); a group
// that straddles two bundles is drawn by both, identically, and each writes
// its own rows.  A group inside the bundle whose first row is a multiple of
// eight writes its eight counts with one 16-byte store.
constexpr int kBgThreads = 256;
__global__ __launch_bounds__(kBgThreads) void k_background(const int64_t* __restrict__ step,
                                                          const Bundle* __restrict__ bundles,
                                                          const uint32_t* __restrict__ T, int K,
                                                          uint16_t* __restrict__ bgc) {
  __shared__ uint32_t s_T[kMaxPoisson];
  for (int c = threadIdx.x; c < K; c += kBgThreads) s_T[c] = T[c];
  __syncthreads();
  const Bundle B = bundles[blockIdx.x];
  const int64_t t = step[0];
  const int64_t g0 = (B.row0 - B.member_row0) >> 3, g1 = (B.row1 - 1 - B.member_row0) >> 3;
  for (int64_t g = g0 + threadIdx.x; g <= g1; g += kBgThreads) {
    uint64_t w[4];
    philox_block(uint64_t(t), uint64_t(g), uint64_t(B.member), 0ull, B.seed, 0ull, w);
    uint32_t c[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) c[j] = uint32_t(poisson_count((j & 1) ? uint32_t(w[j >> 1]) : uint32_t(w[j >> 1] >> 32), s_T, K));
    const int64_t r0 = B.member_row0 + 8 * g;
    if ((r0 & 7) == 0 && r0 >= B.row0 && r0 + 8 <= B.row1) {
      uint4 q;
      q.x = c[0] | (c[1] << 16);
      q.y = c[2] | (c[3] << 16);
      q.z = c[4] | (c[5] << 16);
      q.w = c[6] | (c[7] << 16);
      *reinterpret_cast<uint4*>(bgc + r0) = q;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (r0 + j >= B.row0 && r0 + j < B.row1) bgc[r0 + j] = uint16_t(c[j]);
    }
  }
}

// ----------------------------------------------------------- neuron update
// 1024 neurons per block, kNpt per thread: thread x of the block takes
// neurons x, x + 1024/kNpt, ...; all their loads are issued before any
// arithmetic, so each wavefront keeps kNpt neurons' worth of loads in
// flight.  A wavefront's 64 consecutive neurons of one part form two words
// of the step's spike bitmap (one ballot).
template <int kNpt>
__global__ __launch_bounds__(1024 / kNpt) void k_neuron_update(
    int64_t n, int64_t n_pad, const int64_t* __restrict__ step, float* __restrict__ V, const float* __restrict__ j,
    uint8_t* __restrict__ ref, const uint16_t* __restrict__ ptype, const int32_t* __restrict__ region,
    const PType* __restrict__ ptab, const float* __restrict__ gain, const float* __restrict__ ou,
    float E0, float E1, float E2, float E3, const uint32_t* __restrict__ forced,
    uint32_t* __restrict__ raster, int64_t words_pad, int32_t* __restrict__ counts, int32_t n_regions,
    uint32_t* __restrict__ cticket, int32_t* __restrict__ bad) {
  constexpr int kT = 1024 / kNpt;       // threads per block
  constexpr int kW = kT / 64;           // wavefronts per block
  __shared__ int s_reg[16];             // per 64-neuron run of the block, in neuron order
  __shared__ int s_cnt[16];
  const int64_t slot = step[1];  // step[0] = t, step[1] = t mod ring slots
  uint32_t* __restrict__ raster_slot = raster + slot * words_pad;
  int32_t* __restrict__ counts_slot = counts + slot * n_regions;
  const int64_t base = int64_t(blockIdx.x) * 1024;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool valid[kNpt];
  float v[kNpt], x0[kNpt], x1[kNpt], x2[kNpt], x3[kNpt], xo[kNpt];
  int rr[kNpt], pt[kNpt], rg[kNpt];
#pragma unroll
  for (int h = 0; h < kNpt; ++h) {
    const int64_t i = base + h * kT + threadIdx.x;
    valid[h] = i < n;
    v[h] = x0[h] = x1[h] = x2[h] = x3[h] = xo[h] = 0.f;
    rr[h] = pt[h] = rg[h] = 0;
    if (valid[h]) {
      v[h] = V[i];
      rr[h] = ref[i];
      pt[h] = ptype[i];
      rg[h] = region[i];
      x0[h] = j[i];
      x1[h] = j[n_pad + i];
      x2[h] = j[2 * n_pad + i];
      x3[h] = j[3 * n_pad + i];
      if (ou) xo[h] = ou[i];
    }
  }
#pragma unroll
  for (int h = 0; h < kNpt; ++h) {
    const int64_t i = base + h * kT + threadIdx.x;
    int s = 0;
    if (valid[h]) {
      const PType p = ptab[pt[h]];
      const float* gn = gain + 4 * rg[h];
      const float vv = v[h];
      const int r = rr[h];
      float vt = 0.f;
      if (r <= 0) {
        // I = (Iext + I_ou) + sum_u (g_u gain_u) j_u (E_u - V) - gL (V - EL);  V~ = V + dt/C I
        float I = p.Iext;
        if (ou) I = I + xo[h];
        I = __fmaf_rn((p.g[0] * gn[0]) * x0[h], E0 - vv, I);
        I = __fmaf_rn((p.g[1] * gn[1]) * x1[h], E1 - vv, I);
        I = __fmaf_rn((p.g[2] * gn[2]) * x2[h], E2 - vv, I);
        I = __fmaf_rn((p.g[3] * gn[3]) * x3[h], E3 - vv, I);
        I = __fmaf_rn(-p.gL, vv - p.EL, I);
        vt = __fmaf_rn(p.dtC, I, vv);
      }
      if (forced) s = (forced[i >> 5] >> (i & 31)) & 1u;
      else s = (r <= 0 && vt >= p.Vth) ? 1 : 0;
      float nv;
      int nr;
      if (s) {
        nv = p.Vreset;
        nr = p.nref;
      } else if (r > 0) {
        nv = p.Vreset;
        nr = r - 1;
      } else {
        nv = vt;
        nr = 0;
      }
      V[i] = nv;
      ref[i] = (uint8_t)nr;
      if (!isfinite(nv)) atomicOr(bad, 1);
    }
    // the wavefront's 64 spike predicates are 64 consecutive bits of the bitmap
    const uint64_t m = __ballot(s);
    const int run = h * kW + wave;  // 64-neuron run of the block
    const int64_t first = base + int64_t(run) * 64;
    if (lane == 0) {
      raster_slot[first >> 5] = uint32_t(m);
      raster_slot[(first >> 5) + 1] = uint32_t(m >> 32);
    }
    // population counts: one entry per run when it lies in one population
    const int reg = rg[h];
    const int r0 = __shfl(reg, 0);
    const int uniform = __all((!valid[h] || reg == r0) ? 1 : 0);
    if (uniform) {
      if (lane == 0) {
        s_reg[run] = r0;
        s_cnt[run] = __popcll(m);
      }
    } else {
      if (s) atomicAdd(&counts_slot[reg], 1);
      if (lane == 0) {
        s_reg[run] = -1;
        s_cnt[run] = 0;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int cur = -1, acc = 0;
    for (int w = 0; w < 16; ++w) {
      if (s_reg[w] < 0 || s_cnt[w] == 0) continue;
      if (s_reg[w] == cur) {
        acc += s_cnt[w];
      } else {
        if (cur >= 0) atomicAdd(&counts_slot[cur], acc);
        cur = s_reg[w];
        acc = s_cnt[w];
      }
    }
    if (cur >= 0) atomicAdd(&counts_slot[cur], acc);
    if (blockIdx.x == 0) *cticket = 0u;  // compaction of this step starts after us
  }
}

// ---------------------------------------------------------------- compaction
// Each thread owns 32 * kCompactWords neurons (kCompactWords bitmap words),
// so a block covers 65,536 neurons and the look-back chain stays short.
// Blocks take a dynamic ticket so that a block only waits on blocks that
// are already running.
// Look-back status word: epoch (32) | flag (2: 1 aggregate, 2 prefix) | value (30);
// one wavefront inspects 64 predecessors per round.
__device__ inline uint64_t pack_status(uint32_t epoch, uint32_t flag, uint32_t value) {
  return (uint64_t(epoch) << 32) | (uint64_t(flag) << 30) | uint64_t(value);
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(kCompactBlock) void k_compact(
    const int64_t* __restrict__ step, const uint32_t* __restrict__ raster, int64_t words, int64_t n_blocks,
    int32_t* __restrict__ ids, int32_t* __restrict__ id_count, int32_t id_slots, int64_t id_stride,
    uint64_t* __restrict__ status, uint32_t* __restrict__ ticket, int64_t* __restrict__ spike_total) {
  __shared__ uint32_t s_bid;
  __shared__ int s_wave[kCompactBlock / 64];
  __shared__ int s_excl;
  const uint32_t epoch = uint32_t(uint64_t(step[0]) + 1u);  // never 0 for a live step
  const uint32_t* __restrict__ bits = raster + step[1] * words;
  // the list of step t goes to slot t mod id_slots (one slot, or one per delay)
  const int64_t islot = step[0] % id_slots;
  ids += islot * id_stride;
  id_count += islot;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_bid = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t bid = s_bid;
  const int64_t w0 = (bid * kCompactBlock + tid) * kCompactWords;
  uint32_t wv[kCompactWords];
  int c = 0;
#pragma unroll
  for (int q = 0; q < kCompactWords; ++q) {
    wv[q] = w0 + q < words ? bits[w0 + q] : 0u;
    c += __popc(wv[q]);
  }
  int x = c;  // inclusive scan across the wavefront
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  int wave_off = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < kCompactBlock / 64; ++w) {
    if (w < wave) wave_off += s_wave[w];
    agg += s_wave[w];
  }
  if (wave == 0) {
    uint32_t excl = 0;
    if (bid == 0) {
      if (lane == 0)
        __hip_atomic_store(&status[0], pack_status(epoch, 2, uint32_t(agg)), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(&status[bid], pack_status(epoch, 1, uint32_t(agg)), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      int64_t top = bid - 1;  // lane l inspects predecessor top - l
      while (true) {
        const int64_t idx = top - lane;
        const uint64_t st = idx >= 0 ? __hip_atomic_load(&status[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)
                                     : pack_status(epoch, 2, 0);
        const uint32_t flag = uint32_t(st >> 30) & 3u;
        const bool ready = uint32_t(st >> 32) == epoch && flag != 0;
        const uint64_t incl = __ballot(ready && flag == 2);
        const uint64_t wait = __ballot(!ready);
        const int f = incl ? __ffsll((unsigned long long)incl) - 1 : 64;   // nearest inclusive prefix
        const uint64_t need = f >= 63 ? ~0ull : ((2ull << f) - 1ull);        // lanes 0 .. f
        if (wait & need) continue;                                           // a predecessor is still running
        excl += wave_sum_u32(lane <= f ? (uint32_t(st) & 0x3FFFFFFFu) : 0u);
        if (f < 64) break;
        top -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(&status[bid], pack_status(epoch, 2, excl + uint32_t(agg)), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_excl = int(excl);
      if (bid == n_blocks - 1) {
        *id_count = int(excl) + agg;
        atomicAdd(reinterpret_cast<unsigned long long*>(spike_total), (unsigned long long)(excl + agg));
      }
    }
  }
  __syncthreads();
  int off = s_excl + wave_off + x - c;
#pragma unroll
  for (int q = 0; q < kCompactWords; ++q) {
    uint32_t a = wv[q];
    const int32_t base = int32_t((w0 + q) * 32);
    while (a) {
      ids[off++] = base + (__ffs(a) - 1);
      a &= a - 1u;
    }
  }
}

// ------------------------------------------------------------------ gather
// The pull over each row's in-edges (J_intra).
//  k_gather - one workgroup (16 wavefronts) per bundle of rows.  Phase 1,
//    the delivery tests: the bundle's lookup stream is sorted by (delay,
//    source); a wavefront takes 256-entry tiles (four planes of 64
//    consecutive entries, one entry per lane), rebuilds the sources by
//    prefix sums of the 12-bit deltas,
//    reads the spike bit of step t - d + 1 from that step's slot of the
//    delay ring (monotone addresses, so the cache lines of the bitmaps are
//    swept rather than hit at random) and sets the synapse's bit in the LDS
//    hit bitmap (integer OR: order-free).  Phase 2, when the partition has
//    no other in-edge block: the same workgroup sums its rows from that
//    bitmap, adds their background and updates their gates (fused_rows).
//    With a remote block, the bitmap goes to the hit buffer in one
//    coalesced pass instead, for
//  k_sums - one thread per row visits the row's set hit bits (local block,
//    then remote block) in ascending position, which is its CSR order,
//    loads only those weights and accumulates E and I in FP32 - the fixed
//    per-neuron summation order - then adds the background count and
//    updates the four gates.  Both paths add the same terms in the same
//    order, so their results are identical.
// Gather workgroups are mapped XCD-aware: the blocks an XCD receives
// (blockIdx congruent mod 8) take a contiguous range of bundles, so bundles
// of the same population (same source set) share that XCD's L2; the eight
// ranges hold about equal numbers of tiles.
// Inclusive prefix sum over the 64 lanes of a wavefront with DPP row shifts
// (within each 16-lane row) and the row broadcasts of lanes 15 and 31.
__device__ inline uint32_t wave_incl_scan_dpp(uint32_t x) {
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x111, 0xF, 0xF, true));   // row_shr:1
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x112, 0xF, 0xF, true));   // row_shr:2
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x114, 0xF, 0xF, true));   // row_shr:4
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x118, 0xF, 0xF, true));   // row_shr:8
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x142, 0xA, 0xF, false));  // row_bcast:15
  x += uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x143, 0xC, 0xF, false));  // row_bcast:31
  return x;
}

// ------------------------------------------------------- spike-driven delivery
// The deliveries of step t through every delay d = 1..D: each spike m of
// step t - d + 1 (that step's id list) delivers through its synapses of
// delay d, entries [soff[m (D+1) + d - 1], soff[m (D+1) + d]) of the event
// table, each naming (bundle, position in the bundle) and carrying the
// synapse's weight.  The (delay, spike)
// pairs are cut into equal shares, one per workgroup.  A workgroup works in
// rounds: each thread takes the next kEvRuns pairs, a block prefix sum of
// their run lengths places the runs' entries one after another, and up to
// kEvStage of them are staged in LDS (entry k read by thread k mod T, so
// the loads of a run are adjacent, and all of a thread's loads issued
// before any is used); they are counted per bundle, sorted by bundle in
// LDS, each bundle's share reserved in its bucket with one global atomic,
// and written out bundle by bundle as (position, weight) pairs, so a bucket
// receives contiguous pieces.  A run that does not fit continues in the
// next round.  The order inside a bucket is free: its consumer orders the
// deliveries by position itself, and every synapse delivers at most once
// per step, so a bundle's bucket (room for all its synapses) never
// overflows.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));  // an event-table or bucket pair

constexpr int kEvStage = 5120;   // entries staged per round
constexpr int kEvRuns = 2;       // (delay, spike) pairs a thread takes per round
constexpr int kEvJ = kEvStage / kEventThreads;  // staged entries per thread per round, at most
static_assert(kEvStage % kEventThreads == 0, "every staged entry has its thread");
static_assert(2 * kEvStage * 8 + 3 * kEventMaxBundles * 4 + 2 * kEventThreads * kEvRuns * 4 + 1024 <= 160 * 1024,
              "the bucketing kernel's LDS fits a CU");

__device__ inline uint32_t block_incl_scan(uint32_t x, uint32_t* s_w, uint32_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t v = wave_incl_scan_dpp(x);
  if (lane == 63) s_w[w] = v;
  __syncthreads();
  uint32_t add = 0, all = 0;
#pragma unroll
  for (int q = 0; q < kEventThreads / 64; ++q) {
    const uint32_t y = s_w[q];
    if (q < w) add += y;
    all += y;
  }
  __syncthreads();  // s_w is reused by the next scan
  total = all;
  return v + add;
}

// the last index p in [0, n) with a[p] <= k (a non-decreasing, a[0] <= k)
template <typename T>
__device__ inline int last_at_most(const T* a, int n, T k) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The run offsets of the step's spikes, gathered once: spike k of step t's
// id list gets soff[m (D+1) + d], d = 0..D, at run_off[slot][d][k] (for
// k < cap), so the bucketing of the next D steps reads them as coalesced
// rows instead of a scattered cache line per (spike, delay).
constexpr int kRunThreads = 256;
__global__ __launch_bounds__(kRunThreads) void k_spike_runs(const int64_t* __restrict__ step,
                                                           const int32_t* __restrict__ ids,
                                                           const int32_t* __restrict__ id_count, int32_t id_slots,
                                                           int64_t id_stride, int32_t D,
                                                           const uint32_t* __restrict__ soff,
                                                           uint32_t* __restrict__ run_off,
                                                           int32_t* __restrict__ run_n, int64_t cap) {
  const int64_t sl = step[0] % id_slots;
  const int64_t cnt = min(int64_t(id_count[sl]), cap);
  const int32_t* __restrict__ li = ids + sl * id_stride;
  uint32_t* __restrict__ out = run_off + sl * int64_t(D + 1) * cap;
  for (int64_t k = int64_t(blockIdx.x) * kRunThreads + threadIdx.x; k < cnt;
       k += int64_t(gridDim.x) * kRunThreads) {
    const uint32_t* __restrict__ row = soff + int64_t(li[k]) * (D + 1);
    // the whole row is requested before any of it is stored; past D the
    // last entry is read and stored again (branch-free, so the stores do
    // not wait on one another)
    uint32_t v[kMaxDelay + 1];
#pragma unroll
    for (int d = 0; d <= kMaxDelay; ++d) v[d] = row[min(d, D)];
#pragma unroll
    for (int d = 0; d <= kMaxDelay; ++d) out[int64_t(min(d, D)) * cap + k] = v[d];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) run_n[sl] = int32_t(cnt);
}

__global__ __launch_bounds__(kEventThreads) void k_events(
    const int64_t* __restrict__ step, const int32_t* __restrict__ ids, const int32_t* __restrict__ id_count,
    int32_t id_slots, int64_t id_stride, int32_t D, const uint32_t* __restrict__ soff,
    const uint32_t* __restrict__ run_off, const int32_t* __restrict__ run_n, int64_t run_cap,
    const u32x2* __restrict__ ent, int32_t n_bundles, uint32_t* __restrict__ cursor,
    u32x2* __restrict__ evbuf) {
  constexpr int kRuns = kEventThreads * kEvRuns;  // pairs per round
  extern __shared__ u32x2 s_dyn2[];
  u32x2* s_stage = s_dyn2;                      // [kEvStage] the round's entries, in run order
  u32x2* s_sorted = s_stage + kEvStage;         // [kEvStage] the same, by bundle
  uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_sorted + kEvStage);  // [n_bundles] entries per bundle this round
  uint32_t* s_off = s_cnt + n_bundles;          // [n_bundles] their places in s_sorted
  uint32_t* s_gb = s_off + n_bundles;           // [n_bundles] their first place in the bucket
  __shared__ int64_t s_pre[kMaxDelay + 1];      // first pair of each delay
  __shared__ int64_t s_base[kMaxDelay];         // its id list
  __shared__ int64_t s_roff[kMaxDelay];         // its gathered run offsets (delay d's row)
  __shared__ int32_t s_rn[kMaxDelay];           // how many of its spikes have them
  __shared__ uint32_t s_ex[kRuns];              // staged entries before each pair's run
  __shared__ uint32_t s_a[kRuns];               // table index of each pair's next entry
  __shared__ uint32_t s_w[kEventThreads / 64];
  __shared__ int64_t s_cur;                     // next pair of the share
  __shared__ uint32_t s_coff;                   // entries of that pair already done
  const int tid = threadIdx.x;
  const int64_t t = step[0];
  if (tid == 0) {
    int64_t acc = 0;
    for (int d = 1; d <= D; ++d) {
      const int64_t e = t - d + 1;  // spikes of step e arrive now through delay d
      const int64_t sl = e >= 0 ? e % id_slots : 0;
      s_pre[d - 1] = acc;
      s_base[d - 1] = sl * id_stride;
      s_roff[d - 1] = (sl * (D + 1) + (d - 1)) * run_cap;
      s_rn[d - 1] = e >= 0 ? run_n[sl] : 0;
      acc += e >= 0 ? int64_t(id_count[sl]) : 0;
    }
    s_pre[D] = acc;
  }
  for (int b = tid; b < n_bundles; b += kEventThreads) s_cnt[b] = 0u;
  __syncthreads();
  const int64_t R = s_pre[D];
  const int64_t per = (R + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = min(R, int64_t(blockIdx.x) * per), r1 = min(R, r0 + per);
  if (tid == 0) {
    s_cur = r0;
    s_coff = 0u;
  }
  __syncthreads();
  while (true) {
    const int64_t cur = s_cur;
    const uint32_t coff = s_coff;
    if (cur >= r1) break;  // the same for every thread
    // this thread's pairs cur + kEvRuns tid + h and their runs of entries
    // (the gathered offsets of all the thread's pairs are requested before
    // any is used; a spike without them reads its id and the table after)
    uint32_t a[kEvRuns], len[kEvRuns];
    int dl[kEvRuns];
    int64_t kk[kEvRuns];
    bool valid[kEvRuns], gathered[kEvRuns];
#pragma unroll
    for (int h = 0; h < kEvRuns; ++h) {
      const int64_t i = cur + kEvRuns * tid + h;
      valid[h] = i < r1;
      dl[h] = valid[h] ? last_at_most(s_pre, D, i) : 0;  // delay dl + 1
      kk[h] = valid[h] ? i - s_pre[dl[h]] : 0;            // the spike's place in its list
      gathered[h] = valid[h] && kk[h] < s_rn[dl[h]];
    }
#pragma unroll
    for (int h = 0; h < kEvRuns; ++h) {
      const int64_t o = s_roff[dl[h]] + kk[h];
      a[h] = gathered[h] ? run_off[o] : 0u;
      len[h] = gathered[h] ? run_off[o + run_cap] : 0u;
    }
#pragma unroll
    for (int h = 0; h < kEvRuns; ++h) {
      if (valid[h] && !gathered[h]) {
        const int64_t m = ids[s_base[dl[h]] + kk[h]];
        a[h] = soff[m * (D + 1) + dl[h]];
        len[h] = soff[m * (D + 1) + dl[h] + 1];
      }
    }
#pragma unroll
    for (int h = 0; h < kEvRuns; ++h) len[h] -= a[h];
    if (tid == 0) {
      a[0] += coff;
      len[0] -= coff;
    }
    uint32_t total = 0, mine = 0;
#pragma unroll
    for (int h = 0; h < kEvRuns; ++h) mine += len[h];
    uint32_t ex = block_incl_scan(mine, s_w, total) - mine;
#pragma unroll
    for (int h = 0; h < kEvRuns; ++h) {
      s_ex[kEvRuns * tid + h] = ex;
      s_a[kEvRuns * tid + h] = a[h];
      ex += len[h];
    }
    const uint32_t K = min(total, uint32_t(kEvStage));
    __syncthreads();
    // stage entries [0, K): entry k belongs to the last run starting at or
    // before k; all of a thread's loads are issued before any is used
    u32x2 ev[kEvJ];
#pragma unroll
    for (int j = 0; j < kEvJ; ++j) {
      const uint32_t k = tid + uint32_t(j) * kEventThreads;
      ev[j] = u32x2{0u, 0u};
      if (k < K) {
        const int o = last_at_most(s_ex, kRuns, k);
        ev[j] = ent[s_a[o] + (k - s_ex[o])];
      }
    }
#pragma unroll
    for (int j = 0; j < kEvJ; ++j) {
      const uint32_t k = tid + uint32_t(j) * kEventThreads;
      if (k < K) {
        s_stage[k] = ev[j];
        atomicAdd(&s_cnt[ev[j].x >> kPosBits], 1u);
      }
    }
    if (tid == 0) {
      if (total <= uint32_t(kEvStage)) {
        s_cur = cur + min(int64_t(kRuns), r1 - cur);
        s_coff = 0u;
      } else {  // the run holding entry K - 1 continues in the next round
        const int o = last_at_most(s_ex, kRuns, K - 1);
        const uint32_t run_len = (o + 1 < kRuns ? s_ex[o + 1] : total) - s_ex[o];
        const uint32_t done = K - s_ex[o];
        if (done == run_len) {
          s_cur = cur + o + 1;
          s_coff = 0u;
        } else {
          s_cur = cur + o;
          s_coff = (o == 0 ? coff : 0u) + done;
        }
      }
    }
    __syncthreads();
    // places by bundle: exclusive prefix of the counts (each thread sums a
    // stripe of consecutive bundles), and each bundle's piece of its bucket
    const int per_t = (n_bundles + kEventThreads - 1) / kEventThreads;
    const int b0 = min(n_bundles, tid * per_t), b1 = min(n_bundles, b0 + per_t);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += s_cnt[b];
    uint32_t all = 0;
    uint32_t run = block_incl_scan(sum, s_w, all) - sum;
    for (int b = b0; b < b1; ++b) {
      const uint32_t c = s_cnt[b];
      s_off[b] = run;
      run += c;
      if (c) s_gb[b] = atomicAdd(&cursor[b], c);
    }
    __syncthreads();
    for (uint32_t k = tid; k < K; k += kEventThreads) {
      const u32x2 e = s_stage[k];
      s_sorted[atomicAdd(&s_off[e.x >> kPosBits], 1u)] = e;
    }
    __syncthreads();
    // written bundle by bundle: consecutive places of a bundle are adjacent in its bucket
    for (uint32_t k = tid; k < K; k += kEventThreads) {
      const u32x2 e = s_sorted[k];
      const uint32_t b = e.x >> kPosBits;
      evbuf[s_gb[b] + (k - (s_off[b] - s_cnt[b]))] = u32x2{e.x & kPosMask, e.y};
    }
    __syncthreads();
    for (int b = b0; b < b1; ++b) s_cnt[b] = 0u;
    __syncthreads();
  }
}

// Data touched once per step (lookup tiles, row pointers, gates, weights)
// is loaded and stored non-temporally so that it does not push the delayed
// spike bitmaps, which every bundle re-reads, out of the L2 of its XCD.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ inline T stream_load(const T* p) {
#if DTB_GATHER_NT
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <typename T>
__device__ inline void stream_store(T* p, T v) {
#if DTB_GATHER_NT
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

// One round of delivery tests over kU tiles already in registers: rebuild
// the sources (a wavefront prefix sum of the deltas per plane of 64 entries,
// on top of the tile's first source) and issue the kU x 4 bitmap loads, each
// over 64 consecutive sources.  (Four consecutive entries per lane instead
// - one prefix sum per tile - was measured slower: each load then spans a
// whole tile's sources, so its lanes touch about four times as many cache
// lines.)
template <int kU>
__device__ inline void gather_lookups(const u32x4 (&tv)[kU], const uint32_t (&h)[kU], const uint32_t* bitmaps,
                                      int64_t words_pad, int32_t t_mod, int32_t slots, uint32_t wmax,
                                      uint32_t (&src)[kU][4], uint32_t (&word)[kU][4]) {
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    // plane c holds sorted entries 64 c .. 64 c + 63, one per lane
    const uint32_t e[4] = {tv[u].x, tv[u].y, tv[u].z, tv[u].w};
    uint32_t incl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) incl[c] = wave_incl_scan_dpp(e[c] >> kPosBits);
    uint32_t base = h[u] & 0x3FFFFFFu;  // the tile's first source
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      src[u][c] = base + incl[c];
      base += uint32_t(__builtin_amdgcn_readlane(int(incl[c]), 63));  // the plane's total
    }
    // spikes of step t - d + 1 arrive now; steps before 0 map to unwritten (zero) slots
    int32_t slot = t_mod - int32_t(h[u] >> 26);
    if (slot < 0) slot += slots;
    const uint32_t* bm = bitmaps + int64_t(slot) * words_pad;
#pragma unroll
    for (int c = 0; c < 4; ++c) word[u][c] = bm[min(src[u][c] >> 5, wmax)];
  }
}

// Set the LDS hit bit of every synapse whose source spiked.  The wavefront
// skips an entry index (uniform branch) when none of its lanes has a hit.
// Padding entries point at the bit one past the bundle's last synapse,
// which the sums never read, and a tile processed twice sets the same bits
// again, so neither needs a test here.
template <int kU>
__device__ inline void gather_hits(const u32x4 (&tv)[kU], const uint32_t (&src)[kU][4],
                                   const uint32_t (&word)[kU][4], uint32_t* s_hits) {
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const uint32_t e[4] = {tv[u].x, tv[u].y, tv[u].z, tv[u].w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t hit = __builtin_amdgcn_ubfe(word[u][c], src[u][c], 1u);
      if (__builtin_amdgcn_ballot_w64(hit != 0u)) {
        asm volatile("");  // keeps this wavefront-uniform skip a scalar branch of its own
        if (hit) atomicOr(&s_hits[(e[c] & kPosMask) >> 5], 1u << (e[c] & 31u));
      }
    }
  }
}

// ------------------------------------------------------------ row sums
// A row's delivered weights are added in ascending CSR position - the row's
// fixed summation order - kWalkHits hits at a time, their weights loaded
// together; then its background input and its gates are updated.  The same
// code serves the gather with fused sums (hits read from the bundle's LDS
// hit bitmap) and k_sums (hits read from the hit buffers).
constexpr int kWalkHits = 4;

// gather modes: hit bits out to the hit buffer (k_sums follows), or the
// rows summed in the same workgroup from LDS, with FP32 or BF16 weights
constexpr int kHitsOut = 0, kSumF32 = 1, kSumBF16 = 2;

// what a row's tail reads and writes besides its sums
struct RowTail {
  float* j;                 // [4][n_pad] gates
  int64_t n_pad;
  float a0, a1, a2, a3;     // exp(-dt / tau_u)
  float bg_w;               // background weight
  const uint16_t* bgc;      // the step's background count per row (Poisson background)
  float* ou;                // I_ou [n_pad], or null for the Poisson background
  float ou_mu, ou_a, ou_s;  // OU mean, exp(-dt / tau), sigma sqrt(1 - a^2)
  int32_t* bad;             // non-finite flag
};

// the CSR side of an in-edge block: row pointers and signed weights
struct RowsCsr {
  const int64_t* row_ptr;
  const void* wts;
};

// weights of nh hits at CSR positions base + hp[q], as FP32 bit patterns
// (a BF16 weight is the high half of its FP32 value; sign = inhibitory)
template <bool kBF16>
__device__ inline void load_weights(const void* wts, int64_t base, const int (&hp)[kWalkHits], int nh,
                                    uint32_t (&x)[kWalkHits]) {
  const float* wf = reinterpret_cast<const float*>(wts) + base;
  const uint16_t* wb = reinterpret_cast<const uint16_t*>(wts) + base;
#pragma unroll
  for (int q = 0; q < kWalkHits; ++q)
    if (q < nh) x[q] = kBF16 ? uint32_t(stream_load(wb + hp[q])) << 16 : __float_as_uint(stream_load(wf + hp[q]));
}

__device__ inline void walk_add(const uint32_t (&x)[kWalkHits], int nh, float& dE, float& dI) {
#pragma unroll
  for (int q = 0; q < kWalkHits; ++q) {
    if (q < nh) {
      const float wv = __uint_as_float(x[q] & 0x7FFFFFFFu);
      if (x[q] >> 31) dI += wv;
      else dE += wv;
    }
  }
}

// Row rr's tail at step t after its delivered sums dE / dI: the background
// count of the step (k_background) joins the excitatory sum - or, with the
// OU background, I_ou takes one exact OU step instead - then the four gates
// decay and jump.  Returns the row's background events.
__device__ inline uint32_t row_finish(const RowTail& A, int64_t t, int64_t rr, int64_t mrow0, int32_t member,
                                      uint64_t seed, float dE, float dI, const float (&jv)[4]) {
  const int c = A.ou ? 0 : int(A.bgc[rr]);
  const float de = __fmaf_rn(float(c), A.bg_w, dE);
  const float ja = __fmaf_rn(A.a0, jv[0], de);
  const float jb = __fmaf_rn(A.a1, jv[1], de);
  const float jc = __fmaf_rn(A.a2, jv[2], dI);
  const float jd = __fmaf_rn(A.a3, jv[3], dI);
  A.j[rr] = ja;
  A.j[A.n_pad + rr] = jb;
  A.j[2 * A.n_pad + rr] = jc;
  A.j[3 * A.n_pad + rr] = jd;
  if (!(isfinite(ja) && isfinite(jb) && isfinite(jc) && isfinite(jd))) atomicOr(A.bad, 1);
  if (A.ou) {
    // I_ou <- mu + a (I_ou - mu) + s xi, xi by Box-Muller on Philox stream 1
    uint64_t w1 = 0;
    const uint32_t h0 = uint32_t(philox_hi32_word0(uint64_t(t), uint64_t(rr - mrow0), uint64_t(member), 1ull,
                                                   seed, 0ull, &w1));
    const uint32_t h1 = uint32_t(w1 >> 32);
    // the draw in FP64 (u1, u2 exact), rounded once: a float u1 cannot
    // resolve ln u1 near 1
    const double u1 = (double(h0) + 1.0) * 2.3283064365386962890625e-10;  // (0, 1]
    const double u2 = double(h1) * 2.3283064365386962890625e-10;          // [0, 1)
    const float xi = float(sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2));
    const float xo = A.ou[rr];
    const float y = __fmaf_rn(A.ou_s, xi, __fmaf_rn(A.ou_a, xo - A.ou_mu, A.ou_mu));
    A.ou[rr] = y;
    if (!isfinite(y)) atomicOr(A.bad, 1);
  }
  return uint32_t(c);
}

// A row's walk over bits [p0, p0 + len) of a bundle's LDS hit bitmap, in
// ascending position.
struct LdsWalk {
  int w, w1;
  uint32_t bits, last;
};

__device__ inline void lds_walk_init(const uint32_t* s_hits, int p0, int len, LdsWalk& R) {
  if (len <= 0) {
    R.w = 0;
    R.w1 = -1;
    R.bits = R.last = 0u;
    return;
  }
  R.w = p0 >> 5;
  R.w1 = (p0 + len - 1) >> 5;
  R.bits = s_hits[R.w] & (~0u << (p0 & 31));
  R.last = ~0u >> (31 - ((p0 + len - 1) & 31));
}

// the next up to kWalkHits hit positions of the row (fewer: the row is done)
__device__ inline int lds_walk_collect(const uint32_t* s_hits, LdsWalk& R, int (&hp)[kWalkHits]) {
  int nh = 0;
  while (nh < kWalkHits) {
    if (R.w == R.w1) R.bits &= R.last;
    if (R.bits) {
      hp[nh++] = (R.w << 5) + (__ffs(R.bits) - 1);
      R.bits &= R.bits - 1u;
    } else if (R.w < R.w1) {
      R.bits = s_hits[++R.w];
    } else {
      break;
    }
  }
  return nh;
}

// Rows of a bundle summed from its LDS hit bitmap by one workgroup: each
// thread takes kFuseRows rows at a time (rows tid, tid + T, ... of the
// bundle, T = threads), walks their bits, requests all their first
// kWalkHits weights together and adds each row's weights in its CSR order;
// a row with more hits continues alone.  Then each row's background and
// gates.  One row at a time measured fastest (2 and 4 rows in flight per
// thread: 0.2 % and 3 % slower at 7 Hz, 2 % and 6 % at 30 Hz): the phase
// is bound by the weight lines it fetches, not by load latency.
constexpr int kFuseRows = 1;

template <bool kBF16>
__device__ inline void fused_rows(const uint32_t* s_hits, const Bundle& B, const RowsCsr& rows, const RowTail& A,
                                  int64_t t, int tid, uint32_t& ev, uint32_t& evb) {
  for (int64_t rb = B.row0 + tid; rb < B.row1; rb += int64_t(kFuseRows) * kGatherThreads) {
    int64_t r[kFuseRows];
    bool valid[kFuseRows];
    float jv[kFuseRows][4], dE[kFuseRows], dI[kFuseRows];
    LdsWalk W[kFuseRows];
#pragma unroll
    for (int h = 0; h < kFuseRows; ++h) {
      r[h] = rb + int64_t(h) * kGatherThreads;
      valid[h] = r[h] < B.row1;
      dE[h] = dI[h] = 0.f;
      int64_t k0 = 0, k1 = 0;
      jv[h][0] = jv[h][1] = jv[h][2] = jv[h][3] = 0.f;
      if (valid[h]) {
        k0 = rows.row_ptr[r[h]];
        k1 = rows.row_ptr[r[h] + 1];
        jv[h][0] = A.j[r[h]];
        jv[h][1] = A.j[A.n_pad + r[h]];
        jv[h][2] = A.j[2 * A.n_pad + r[h]];
        jv[h][3] = A.j[3 * A.n_pad + r[h]];
      }
      lds_walk_init(s_hits, int(k0 - B.syn0), int(k1 - k0), W[h]);
    }
    int hp[kFuseRows][kWalkHits], nh[kFuseRows];
    uint32_t x[kFuseRows][kWalkHits];
#pragma unroll
    for (int h = 0; h < kFuseRows; ++h) nh[h] = lds_walk_collect(s_hits, W[h], hp[h]);
#pragma unroll
    for (int h = 0; h < kFuseRows; ++h) load_weights<kBF16>(rows.wts, B.syn0, hp[h], nh[h], x[h]);
#pragma unroll
    for (int h = 0; h < kFuseRows; ++h) {
      walk_add(x[h], nh[h], dE[h], dI[h]);
      ev += uint32_t(nh[h]);
      while (nh[h] == kWalkHits) {
        nh[h] = lds_walk_collect(s_hits, W[h], hp[h]);
        load_weights<kBF16>(rows.wts, B.syn0, hp[h], nh[h], x[h]);
        walk_add(x[h], nh[h], dE[h], dI[h]);
        ev += uint32_t(nh[h]);
      }
    }
#pragma unroll
    for (int h = 0; h < kFuseRows; ++h)
      if (valid[h]) evb += row_finish(A, t, r[h], B.member_row0, B.member, B.seed, dE[h], dI[h], jv[h]);
  }
}

// where a bundle's delivery tests come from: the sweep of its (delay,
// source)-sorted lookup stream over the delayed spike bitmaps, or its
// bucket of the step's spike-driven deliveries (k_events)
constexpr int kFromSweep = 0, kFromEvents = 1;

// pairs of its bucket a thread of the fused spike-driven sums keeps in
// registers between setting their hit bits and placing their weights
constexpr int kEvKeep = 16;

// a bundle's bucket of deliveries: bundle b's (position, weight bits) pairs
// at evbuf + syn0, up to cursor[b]; with the row sums fused, the LDS after
// the hit bitmap (hit_words words, the largest bundle's) holds the group
// prefix counts and up to weight_cap delivered weights (-1: no room even
// for the prefix counts)
struct EventSrc {
  u32x2* evbuf;
  uint32_t* cursor;
  int32_t hit_words, weight_cap;
};

// the number of set hit bits below position p of a bundle's bitmap: the
// count before p's group of kEvGroupWords words, then the words of the
// group before p's, then p's word below p
__device__ inline uint32_t hit_rank(const uint32_t* s_hits, const uint32_t* s_pre, uint32_t p) {
  const uint32_t w = p >> 5, g = w / kEvGroupWords;
  uint32_t r = s_pre[g];
  for (uint32_t q = g * kEvGroupWords; q < w; ++q) r += uint32_t(__popc(s_hits[q]));
  return r + uint32_t(__popc(s_hits[w] & ((1u << (p & 31u)) - 1u)));
}

// Rows of a bundle summed from its bucket's carried weights (phase 1 has
// set the bucket's hit bits): every delivery's weight is put at its rank
// among the set bits, which orders the bundle's delivered weights by
// position, so row r's are places [rank(p0), rank(p1)) with [p0, p1) its
// CSR positions, added in its CSR order as the bitmap walk adds them (the
// same sums, bit for bit) - without fetching a weight line per delivery.
// The places are LDS or, for a bucket larger than the LDS holds (glob), the
// unused part of the bundle's bucket right after its pairs (a few hundred
// KB per bundle, so it stays in L2).  Then each
// row's background and gates.  Every thread of the block calls this (block
// scan and barriers inside).
template <int kKeep>
__device__ inline void carried_rows(uint32_t* s_hits, uint32_t* s_scan, const u32x2 (&kept)[kKeep], const Bundle& B,
                                    const RowsCsr& rows, const RowTail& A, const EventSrc& E, int cnt, bool glob,
                                    int64_t t, int tid, uint32_t& ev, uint32_t& evb) {
  static_assert(kGatherThreads == kEventThreads, "block_incl_scan takes kEventThreads threads");
  uint32_t* s_pre = s_hits + E.hit_words;
  const u32x2* __restrict__ bk = E.evbuf + B.syn0;
  uint32_t* const wt_glob = reinterpret_cast<uint32_t*>(E.evbuf + B.syn0 + cnt);
  uint32_t* const wt_lds = s_pre + ev_groups(E.hit_words);
  const int hw = (B.nsyn >> 5) + 1;
  const int ng = ev_groups(hw);
  // exclusive prefix of the groups' counts (thread tid sums a stripe of groups)
  const int per = (ng + kGatherThreads - 1) / kGatherThreads;
  const int g0 = min(ng, tid * per), g1 = min(ng, g0 + per);
  uint32_t sum = 0;
  for (int q = g0 * kEvGroupWords; q < min(hw, g1 * kEvGroupWords); ++q) sum += uint32_t(__popc(s_hits[q]));
  uint32_t all = 0;
  uint32_t run = block_incl_scan(sum, s_scan, all) - sum;
  for (int g = g0; g < g1; ++g) {
    s_pre[g] = run;
    for (int q = g * kEvGroupWords; q < min(hw, (g + 1) * kEvGroupWords); ++q) run += uint32_t(__popc(s_hits[q]));
  }
  __syncthreads();
  // every delivery's weight at its rank: the pairs kept in registers, then
  // the rest (each loop written for one memory, so LDS stays LDS)
  auto place = [&](uint32_t* wt) {
#pragma unroll
    for (int j = 0; j < kKeep; ++j)
      if (tid + j * kGatherThreads < cnt) wt[hit_rank(s_hits, s_pre, kept[j].x)] = kept[j].y;
    for (int q = tid + kKeep * kGatherThreads; q < cnt; q += kGatherThreads) {
      const u32x2 e = bk[q];
      wt[hit_rank(s_hits, s_pre, e.x)] = e.y;
    }
  };
  if (glob) place(wt_glob);
  else place(wt_lds);
  __syncthreads();
  // the rows; each row's pointers and gates are requested one row ahead
  int64_t k0n = 0, k1n = 0;
  float jn[4] = {0.f, 0.f, 0.f, 0.f};
  auto fetch = [&](int64_t r) {
    if (r < B.row1) {
      k0n = rows.row_ptr[r];
      k1n = rows.row_ptr[r + 1];
      jn[0] = A.j[r];
      jn[1] = A.j[A.n_pad + r];
      jn[2] = A.j[2 * A.n_pad + r];
      jn[3] = A.j[3 * A.n_pad + r];
    }
  };
  fetch(B.row0 + tid);
  for (int64_t r = B.row0 + tid; r < B.row1; r += kGatherThreads) {
    const int64_t k0 = k0n, k1 = k1n;
    const float jv[4] = {jn[0], jn[1], jn[2], jn[3]};
    fetch(r + kGatherThreads);
    const uint32_t a = hit_rank(s_hits, s_pre, uint32_t(k0 - B.syn0));
    const uint32_t b = hit_rank(s_hits, s_pre, uint32_t(k1 - B.syn0));
    float dE = 0.f, dI = 0.f;
    auto add = [&](const uint32_t* wt) {
      for (uint32_t k = a; k < b; ++k) {
        const uint32_t x = wt[k];
        const float wv = __uint_as_float(x & 0x7FFFFFFFu);
        if (x >> 31) dI += wv;
        else dE += wv;
      }
    };
    if (glob) add(wt_glob);
    else add(wt_lds);
    ev += b - a;
    evb += row_finish(A, t, r, B.member_row0, B.member, B.seed, dE, dI, jv);
  }
}

template <int kU, int kMode, int kSrc>
__global__ __launch_bounds__(kGatherThreads) __attribute__((amdgpu_waves_per_eu(kU == 1 && kMode == kHitsOut ? 8 : 4)))
void k_gather(const int64_t* __restrict__ xcd_first, const int64_t* __restrict__ step, const Bundle* __restrict__ bundles,
              const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ theads,
              const uint32_t* __restrict__ bitmaps, int64_t words_pad, int32_t slots,
              uint32_t* __restrict__ hitbuf, int64_t* __restrict__ ev_ring, RowsCsr rows, RowTail A, EventSrc E) {
  extern __shared__ uint32_t s_hits[];
  __shared__ uint32_t s_red[2][kGatherThreads / 64];
  __shared__ int32_t s_count;
  const int32_t t_mod = int32_t(step[1]);
  int64_t* __restrict__ ev_slot = ev_ring + int64_t(t_mod) * kStripes * 2;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int x = int(blockIdx.x % 8);
  const int64_t bi = xcd_first[x] + blockIdx.x / 8;
  if (bi >= xcd_first[x + 1]) return;  // whole block leaves together
  const Bundle B = bundles[bi];
  const int hw = (B.nsyn >> 5) + 1;  // includes the padding bit at position nsyn
  for (int q = tid; q < hw; q += kGatherThreads) s_hits[q] = 0u;
  if (kSrc == kFromEvents && tid == 0) s_count = int32_t(E.cursor[bi] - uint32_t(B.syn0));
  __syncthreads();

  u32x2 kept[kSrc == kFromEvents && kMode != kHitsOut ? kEvKeep : 1];
  if constexpr (kSrc == kFromEvents) {
    // ---- phase 1 from the bucket: each delivery sets its synapse's bit
    // (positions < nsyn, each at most once per step); the bucket is emptied
    // for the next step once every thread has read its count
    const int cnt = s_count;
    const u32x2* __restrict__ bk = E.evbuf + B.syn0;
    int q0 = tid;
    if constexpr (kMode != kHitsOut) {
      // the thread's first kEvKeep pairs stay in registers for the carried
      // weights; the loads of the rest stay cacheable (read again there)
#pragma unroll
      for (int j = 0; j < kEvKeep; ++j) {
        const int q = tid + j * kGatherThreads;
        kept[j] = q < cnt ? stream_load(bk + q) : u32x2{0u, 0u};
      }
#pragma unroll
      for (int j = 0; j < kEvKeep; ++j) {
        const uint32_t p = kept[j].x;
        if (tid + j * kGatherThreads < cnt) atomicOr(&s_hits[p >> 5], 1u << (p & 31u));
      }
      q0 = tid + kEvKeep * kGatherThreads;
    }
    for (int q = q0; q < cnt; q += kGatherThreads) {
      const uint32_t p = kMode != kHitsOut ? bk[q].x : stream_load(bk + q).x;
      atomicOr(&s_hits[p >> 5], 1u << (p & 31u));
    }
    if (tid == 0) E.cursor[bi] = uint32_t(B.syn0);
  } else {
  // ---- phase 1: delivery tests in (delay, source) order
  // Software pipeline over rounds of kU tiles per wavefront.  In the stage
  // that takes the hits of round r, the bitmap words of round r+1 are
  // requested and the tiles of round r+3 are fetched, while those of round
  // r+2 are still on their way: two rounds of lookups and two of tiles are
  // in flight per wavefront, and since loads return in order no wait ever
  // has to drain the newer ones.  Four tile sets and two lookup sets
  // rotate (the loop body is four stages).  Tile indices past the end are
  // clamped to the last tile, which then is processed again (the OR is
  // idempotent), so every load is unconditional.
  constexpr int kS = (kGatherThreads / 64) * kU;  // tiles per round of the workgroup
  const int nt = B.ntiles;
  const u32x4* tp = reinterpret_cast<const u32x4*>(tiles + B.tile0 * kTile) + lane;
  const uint32_t* hp = theads + B.tile0;
  const uint32_t wmax = uint32_t(words_pad - 1);
  u32x4 t0[kU], t1[kU], t2[kU], t3[kU];
  uint32_t h0[kU], h1[kU], h2[kU], h3[kU];
  uint32_t sa[kU][4], sb[kU][4];  // sources of the rounds being looked up
  uint32_t xa[kU][4], xb[kU][4];  // their bitmap words
  auto fetch = [&](u32x4 (&tv)[kU], uint32_t (&h)[kU], int qb) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int qc = min(qb + u * (kGatherThreads / 64), nt - 1);
      tv[u] = stream_load(tp + int64_t(qc) * 64);
      h[u] = __builtin_amdgcn_readfirstlane(hp[qc]);
    }
  };
  auto lookups = [&](const u32x4 (&tv)[kU], const uint32_t (&h)[kU], uint32_t (&src)[kU][4],
                     uint32_t (&word)[kU][4]) {
    gather_lookups<kU>(tv, h, bitmaps, words_pad, t_mod, slots, wmax, src, word);
  };
  if (wave < nt) {  // nt > 0 here, so every clamped index lies in the bundle
    // stage j takes the hits of one round; the loop runs whole groups of
    // four stages (a break inside the group would make the compiler drain
    // every load at the loop head), the remaining rounds follow it
    const int rounds = (nt - wave + kS - 1) / kS;
    int q0 = wave;
    fetch(t0, h0, q0);
    fetch(t1, h1, q0 + kS);
    fetch(t2, h2, q0 + 2 * kS);
    lookups(t0, h0, sa, xa);
    for (int g = rounds >> 2; g > 0; --g, q0 += 4 * kS) {
      lookups(t1, h1, sb, xb);
      fetch(t3, h3, q0 + 3 * kS);
      gather_hits<kU>(t0, sa, xa, s_hits);
      lookups(t2, h2, sa, xa);
      fetch(t0, h0, q0 + 4 * kS);
      gather_hits<kU>(t1, sb, xb, s_hits);
      lookups(t3, h3, sb, xb);
      fetch(t1, h1, q0 + 5 * kS);
      gather_hits<kU>(t2, sa, xa, s_hits);
      lookups(t0, h0, sa, xa);
      fetch(t2, h2, q0 + 6 * kS);
      gather_hits<kU>(t3, sb, xb, s_hits);
    }
    const int rem = rounds & 3;
    if (rem > 0) {
      lookups(t1, h1, sb, xb);
      gather_hits<kU>(t0, sa, xa, s_hits);
      if (rem > 1) {
        lookups(t2, h2, sa, xa);
        gather_hits<kU>(t1, sb, xb, s_hits);
        if (rem > 2) gather_hits<kU>(t2, sa, xa, s_hits);
      }
    }
  }
  }  // sweep
  __syncthreads();

  uint32_t ev = 0, evb = 0;
  if constexpr (kMode == kHitsOut) {
    // ---- hand the delivery tests to the sums: the bundle's hit words, and
    // the delivered events (set bits below the padding bit at nsyn)
    uint32_t* __restrict__ dst = hitbuf + (B.hbit0 >> 5);
    for (int q = tid; q < hw; q += kGatherThreads) {
      const uint32_t w = s_hits[q];
      stream_store(dst + q, w);
      ev += uint32_t(__popc(q == hw - 1 ? w & ((1u << (B.nsyn & 31)) - 1u) : w));
    }
  } else {
    // ---- phase 2: the sums of the bundle's rows from the hit bitmap still
    // in LDS (row r's CSR positions [row_ptr[r] - syn0, row_ptr[r+1] -
    // syn0)), then their background and gates.  The delivered events are
    // the hits the rows visit.
    // The carried weights, placed in LDS when they fit, else in the free
    // part of the bucket (room for them when the bucket is at most 2/3
    // full); the weight of each hit from the CSR when the LDS cannot even
    // hold the prefix counts or the bucket is fuller than that.
    if (kSrc == kFromEvents && E.weight_cap >= 0 &&
        (s_count <= E.weight_cap || 3 * int64_t(s_count) <= 2 * int64_t(B.nsyn)))
      carried_rows(s_hits, s_red[0], kept, B, rows, A, E, s_count, s_count > E.weight_cap, step[0], tid, ev, evb);
    else
      fused_rows<kMode == kSumBF16>(s_hits, B, rows, A, step[0], tid, ev, evb);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ev += __shfl_down(ev, off);
    evb += __shfl_down(evb, off);
  }
  if (lane == 0) {
    s_red[0][tid >> 6] = ev;
    s_red[1][tid >> 6] = evb;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t r = 0, rb = 0;
    for (int w = 0; w < kGatherThreads / 64; ++w) {
      r += s_red[0][w];
      rb += s_red[1][w];
    }
    int64_t* dsts = ev_slot + 2 * (blockIdx.x & (kStripes - 1));
    if (r) atomicAdd(reinterpret_cast<unsigned long long*>(dsts), (unsigned long long)r);
    if (rb) atomicAdd(reinterpret_cast<unsigned long long*>(dsts + 1), (unsigned long long)rb);
  }
}

// ------------------------------------------------------------------- sums
// One thread per neuron (row): the delivered weights in the row's CSR order
// (the fixed per-neuron summation order) - the local block, then the remote
// block if there is one - then the step's background count (drawn by
// k_background), then the four gates (exact decay + jump).  A row's delivery tests are the
// bits hbit0 + (k - syn0) of its bundle in the block's hit buffer.
constexpr int kSumsRowsPerBlock = 1024;  // rows per workgroup (the block table's granularity)

// the tables one in-edge block hands to the sums
struct SumBlock {
  const Bundle* bundles;
  const int32_t* block_bundle;
  const int64_t* row_ptr;
  const void* wts;
  const uint32_t* hitbuf;
};

// adds row r's delivered weights of one block to (dE, dI) in CSR order;
// A row's walk over one block's hit bits [bit0, bit0 + len), in ascending
// order: the first kWalkWords words are loaded together (a row of
// in-degree 100 spans at most 5), then the window slides one word at a
// time; hits are taken kWalkHits at a time and their weights loaded
// together.
constexpr int kWalkWords = 5;

struct RowWalk {
  int64_t k0, bit0, w, w1;
  int len;
  uint32_t bits, last;
  uint32_t win[kWalkWords];
};

// the row's bundle, CSR range and first hit words
__device__ inline const Bundle* walk_init(const SumBlock& S, int64_t r, RowWalk& R) {
  int32_t b = S.block_bundle[r / kSumsRowsPerBlock];
  while (r >= S.bundles[b].row1) ++b;  // bundles are consecutive row ranges
  const Bundle* B = S.bundles + b;
  const int64_t k0 = S.row_ptr[r], k1 = S.row_ptr[r + 1];
  R.k0 = k0;
  R.len = int(k1 - k0);
  R.bit0 = B->hbit0 + (k0 - B->syn0);
  R.w = R.bit0 >> 5;
  R.w1 = (R.bit0 + R.len - 1) >> 5;
#pragma unroll
  for (int q = 0; q < kWalkWords; ++q) R.win[q] = R.len > 0 && R.w + q <= R.w1 ? S.hitbuf[R.w + q] : 0u;
  R.bits = R.win[0] & (~0u << (R.bit0 & 31));
  R.last = ~0u >> (31 - int((R.bit0 + R.len - 1) & 31));
  return B;
}

// the next up to kWalkHits hit offsets of the row (fewer: the row is done)
__device__ inline int walk_collect(const SumBlock& S, RowWalk& R, int (&hp)[kWalkHits]) {
  int nh = 0;
  if (R.len <= 0) return 0;
  while (nh < kWalkHits) {
    if (R.w == R.w1) R.bits &= R.last;
    if (R.bits) {
      hp[nh++] = int((R.w << 5) + (__ffs(R.bits) - 1) - R.bit0);
      R.bits &= R.bits - 1u;
    } else if (R.w < R.w1) {
      ++R.w;
#pragma unroll
      for (int q = 0; q + 1 < kWalkWords; ++q) R.win[q] = R.win[q + 1];
      R.win[kWalkWords - 1] = R.w + kWalkWords - 1 <= R.w1 ? S.hitbuf[R.w + kWalkWords - 1] : 0u;
      R.bits = R.win[0];
    } else {
      break;
    }
  }
  return nh;
}

template <bool kBF16>
__device__ inline void walk_load(const SumBlock& S, const RowWalk& R, const int (&hp)[kWalkHits], int nh,
                                 uint32_t (&x)[kWalkHits]) {
  load_weights<kBF16>(S.wts, R.k0, hp, nh, x);
}

// adds the delivered weights of one block to the kRows rows of a thread,
// each row in its CSR order; the rows' first batches of loads are issued
// together
template <bool kBF16, int kRows>
__device__ inline void block_rows_sum(const SumBlock& S, const int64_t (&r)[kRows], const bool (&valid)[kRows],
                                      float (&dE)[kRows], float (&dI)[kRows], const Bundle* (&B)[kRows]) {
  RowWalk R[kRows];
#pragma unroll
  for (int h = 0; h < kRows; ++h) {
    if (valid[h]) B[h] = walk_init(S, r[h], R[h]);
    else R[h].len = 0;
  }
  int hp[kRows][kWalkHits];
  int nh[kRows];
  uint32_t x[kRows][kWalkHits];
#pragma unroll
  for (int h = 0; h < kRows; ++h) nh[h] = walk_collect(S, R[h], hp[h]);
#pragma unroll
  for (int h = 0; h < kRows; ++h) walk_load<kBF16>(S, R[h], hp[h], nh[h], x[h]);
#pragma unroll
  for (int h = 0; h < kRows; ++h) {
    walk_add(x[h], nh[h], dE[h], dI[h]);
    while (nh[h] == kWalkHits) {
      nh[h] = walk_collect(S, R[h], hp[h]);
      walk_load<kBF16>(S, R[h], hp[h], nh[h], x[h]);
      walk_add(x[h], nh[h], dE[h], dI[h]);
    }
  }
}

template <bool kBF16, int kRows>
__global__ __launch_bounds__(kSumsRowsPerBlock / kRows) void k_sums(
    int64_t n, const int64_t* __restrict__ step, SumBlock loc, SumBlock rem, int has_rem, RowTail A,
    int64_t* __restrict__ ev_ring) {
  constexpr int kT = kSumsRowsPerBlock / kRows;  // threads per block
  __shared__ uint32_t s_bg[kT / 64];
  const int64_t t = step[0];
  int64_t* __restrict__ ev_slot = ev_ring + int64_t(step[1]) * kStripes * 2;
  const int tid = threadIdx.x, lane = tid & 63;
  int64_t r[kRows];
  bool valid[kRows];
  float dE[kRows], dI[kRows], jv[kRows][4];
  const Bundle* B[kRows];
#pragma unroll
  for (int h = 0; h < kRows; ++h) {
    r[h] = int64_t(blockIdx.x) * kSumsRowsPerBlock + h * kT + tid;
    valid[h] = r[h] < n;
    dE[h] = dI[h] = 0.f;
    B[h] = nullptr;
    if (valid[h]) {
      jv[h][0] = A.j[r[h]];
      jv[h][1] = A.j[A.n_pad + r[h]];
      jv[h][2] = A.j[2 * A.n_pad + r[h]];
      jv[h][3] = A.j[3 * A.n_pad + r[h]];
    }
  }
  block_rows_sum<kBF16, kRows>(loc, r, valid, dE, dI, B);
  if (has_rem) {
    const Bundle* Br[kRows];
    block_rows_sum<kBF16, kRows>(rem, r, valid, dE, dI, Br);
  }
  uint32_t evb = 0;
#pragma unroll
  for (int h = 0; h < kRows; ++h) {
    if (!valid[h]) continue;
    evb += row_finish(A, t, r[h], B[h]->member_row0, B[h]->member, B[h]->seed, dE[h], dI[h], jv[h]);
  }
  // block total of background events, one striped atomic per block
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) evb += __shfl_down(evb, off);
  if (lane == 0) s_bg[tid >> 6] = evb;
  __syncthreads();
  if (tid == 0) {
    int64_t tot = 0;
    for (int q = 0; q < kT / 64; ++q) tot += s_bg[q];
    int64_t* dst = ev_slot + 2 * (blockIdx.x & (kStripes - 1)) + 1;
    if (tot) atomicAdd(reinterpret_cast<unsigned long long*>(dst), (unsigned long long)tot);
  }
}

// ---------------------------------------------------------------- finalize
// Last kernel of a step: reduce the striped event counters of step t into
// the totals, advance the per-population Balloon-Windkessel hemodynamics
// by one Euler step with the population rates of step t, clear the ring
// slot step t+1 will fill, and advance the device step counter.
//
// Balloon-Windkessel (Friston et al. 2000; the BOLD model of Sec. V-E) is
// integrated in FP32 for the deviations from rest x = (s, f-1, v-1, q-1),
// which keeps the small increments of a 1 ms step representable:
//   ds = eps u - kappa s - gamma (f-1)        df = s
//   tau0 dv = f - v^(1/alpha)                 tau0 dq = f E(f)/E0 - v^(1/alpha) q / v
//   E(f) = 1 - (1-E0)^(1/f),  y = V0 [-k1 (q-1) + k2 (v-q)/v - k3 (v-1)]
struct BoldParams {
  float kappa, gamma, tau0, inv_alpha, E0, log1mE0, V0, eps, k1, k2, k3, rate_scale;
};

__global__ __launch_bounds__(256) void k_finalize(
    int64_t* __restrict__ step, int32_t slots, int64_t* __restrict__ ev, int32_t* __restrict__ counts,
    int32_t n_regions, int64_t* __restrict__ totals, const float* __restrict__ inv_nr_dt, float dt_s,
    float* __restrict__ bold, float* __restrict__ bold_y, BoldParams bp) {
  const int tid = threadIdx.x;
  const int64_t t = step[0];
  const int32_t slot = int32_t(step[1]);
  const int32_t next = slot + 1 == slots ? 0 : slot + 1;
  int64_t* ev_slot = ev + int64_t(slot) * kStripes * 2;
  int64_t* ev_next = ev + int64_t(next) * kStripes * 2;
  __syncthreads();
  if (tid < 64) {
    int64_t r = ev_slot[2 * tid], b = ev_slot[2 * tid + 1];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      r += __shfl_down(r, off);
      b += __shfl_down(b, off);
    }
    if (tid == 0) {
      ev_slot[0] = r;
      ev_slot[1] = b;
      totals[1] += r;
      totals[2] += b;
      totals[3] += 1;
    }
  }
  const int32_t* c = counts + int64_t(slot) * n_regions;
  for (int q = tid; q < n_regions; q += 256) {
    const float u = float(c[q]) * inv_nr_dt[q] / bp.rate_scale;  // population rate (Hz) / scale
    float* x = bold + 4 * q;
    const float s = x[0], fm = x[1], vm = x[2], qm = x[3];
    const float f = 1.f + fm, v = 1.f + vm, qq = 1.f + qm;
    const float vpow = expf(bp.inv_alpha * log1pf(vm));           // v^(1/alpha)
    const float Ef = 1.f - expf(bp.log1mE0 / f);                   // 1 - (1-E0)^(1/f)
    const float ds = bp.eps * u - bp.kappa * s - bp.gamma * fm;
    const float dv = (fm - (vpow - 1.f)) / bp.tau0;
    const float dq = (f * Ef / bp.E0 - vpow * qq / v) / bp.tau0;
    const float ns = __fmaf_rn(dt_s, ds, s);
    const float nf = __fmaf_rn(dt_s, s, fm);
    const float nv = __fmaf_rn(dt_s, dv, vm);
    const float nq = __fmaf_rn(dt_s, dq, qm);
    x[0] = ns;
    x[1] = nf;
    x[2] = nv;
    x[3] = nq;
    bold_y[q] = bp.V0 * (-bp.k1 * nq + bp.k2 * (nv - nq) / (1.f + nv) - bp.k3 * nv);
  }
  if (tid < 64) {
    ev_next[2 * tid] = 0;
    ev_next[2 * tid + 1] = 0;
  }
  int32_t* cn = counts + int64_t(next) * n_regions;
  for (int q = tid; q < n_regions; q += 256) cn[q] = 0;
  __syncthreads();
  if (tid == 0) {
    step[0] = t + 1;
    step[1] = next;
  }
}

}  // namespace

hipError_t launch_neuron_update(const DeviceNet& d, const uint32_t* forced, hipStream_t s) {
  const unsigned grid = unsigned(d.n_pad / 1024);
  hipLaunchKernelGGL(k_neuron_update<kUpdateNpt>, dim3(grid), dim3(1024 / kUpdateNpt), 0, s, d.n, d.n_pad, d.step,
                     d.V, d.j, d.ref,
                     d.ptype, d.region, d.ptab, d.gain, d.ou_on ? d.ou : nullptr, d.E[0], d.E[1], d.E[2], d.E[3],
                     forced, d.raster,
                     d.words_pad, d.counts, d.n_regions, d.cticket, d.bad);
  return hipGetLastError();
}

hipError_t launch_background(const DeviceNet& d, hipStream_t s) {
  if (d.ou_on || d.loc.n_bundles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_background, dim3(unsigned(d.loc.n_bundles)), dim3(kBgThreads), 0, s, d.step, d.loc.bundles,
                     d.poisson, d.poisson_K, d.bgc);
  return hipGetLastError();
}

hipError_t launch_compact(const DeviceNet& d, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(unsigned(d.compact_blocks)), dim3(kCompactBlock), 0, s, d.step, d.raster,
                     d.words_pad, d.compact_blocks, d.ids, d.id_count, d.id_slots, d.n_pad, d.cstatus, d.cticket,
                     d.totals);
  return hipGetLastError();
}

// the spike list of an earlier step, rebuilt from its ring slot: at[0] + 1 is
// the look-back epoch of this read, at[1] the slot; the read's own status
// words, ticket (zeroed by the caller) and spike-total sink
hipError_t launch_compact_read(const DeviceNet& d, const int64_t* at, int32_t* ids, int32_t* count,
                               uint64_t* status, uint32_t* ticket, int64_t* total, hipStream_t s) {
  hipLaunchKernelGGL(k_compact, dim3(unsigned(d.compact_blocks)), dim3(kCompactBlock), 0, s, at, d.raster,
                     d.words_pad, d.compact_blocks, ids, count, 1, 0, status, ticket, total);
  return hipGetLastError();
}

namespace {

RowTail row_tail(const DeviceNet& d) {
  return RowTail{d.j, d.n_pad, d.a[0], d.a[1], d.a[2], d.a[3], d.bg_w, d.bgc,
                 d.ou_on ? d.ou : nullptr, d.ou_mu, d.ou_a, d.ou_s, d.bad};
}

template <int kU, int kMode, int kSrc>
void launch_gather_as(const DeviceNet& d, const ConnBlock& cb, const uint32_t* bitmaps, int64_t words_pad,
                      hipStream_t s) {
  const unsigned grid = unsigned(cb.xcd_max * 8);
  // the fused spike-driven sums take the carried weights when they fit
  const int cap = kSrc == kFromEvents && kMode != kHitsOut ? ev_weight_cap(cb.hit_words) : -1;
  const size_t lds = cap >= 0 ? size_t(kEvLdsBytes) : size_t(cb.hit_words) * 4;
  hipLaunchKernelGGL((k_gather<kU, kMode, kSrc>), dim3(grid), dim3(kGatherThreads), lds, s, cb.xcd_first, d.step,
                     cb.bundles, cb.tiles, cb.theads, bitmaps, words_pad, d.slots, cb.hitbuf, d.ev,
                     RowsCsr{cb.row_ptr, cb.wts}, row_tail(d),
                     EventSrc{reinterpret_cast<u32x2*>(cb.evbuf), cb.ev_cursor, cb.hit_words, cap});
}

template <int kMode>
void launch_gather_mode(const DeviceNet& d, const ConnBlock& cb, const uint32_t* bitmaps, int64_t words_pad,
                        hipStream_t s) {
  switch (d.unroll) {
    case 1: launch_gather_as<1, kMode, kFromSweep>(d, cb, bitmaps, words_pad, s); break;
    case 2: launch_gather_as<2, kMode, kFromSweep>(d, cb, bitmaps, words_pad, s); break;
    default: launch_gather_as<3, kMode, kFromSweep>(d, cb, bitmaps, words_pad, s); break;
  }
}

template <int kU, int kMode, int kSrc>
hipError_t set_lds_limit_one(int bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather<kU, kMode, kSrc>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace

hipError_t launch_gather(const DeviceNet& d, const ConnBlock& cb, const uint32_t* bitmaps, int64_t words_pad,
                         bool fuse_sums, hipStream_t s) {
  if (cb.n_bundles == 0) return hipSuccess;
  if (!fuse_sums) launch_gather_mode<kHitsOut>(d, cb, bitmaps, words_pad, s);
  else if (d.wtype == DTB_W_BF16) launch_gather_mode<kSumBF16>(d, cb, bitmaps, words_pad, s);
  else launch_gather_mode<kSumF32>(d, cb, bitmaps, words_pad, s);
  return hipGetLastError();
}

hipError_t launch_spike_runs(const DeviceNet& d, hipStream_t s) {
  const ConnBlock& cb = d.loc;
  if (cb.n_bundles == 0) return hipSuccess;
  const unsigned rgrid = unsigned(std::min<int64_t>(2048, std::max<int64_t>(1, (d.run_cap + kRunThreads - 1) / kRunThreads)));
  hipLaunchKernelGGL(k_spike_runs, dim3(rgrid), dim3(kRunThreads), 0, s, d.step, d.ids, d.id_count, d.id_slots,
                     d.n_pad, d.max_delay, cb.ev_soff, d.run_off, d.run_n, d.run_cap);
  return hipGetLastError();
}

hipError_t launch_events(const DeviceNet& d, hipStream_t s) {
  const ConnBlock& cb = d.loc;
  if (cb.n_bundles == 0) return hipSuccess;
  const size_t lds = 2 * size_t(kEvStage) * 8 + 3 * size_t(cb.n_bundles) * 4;
  hipLaunchKernelGGL(k_events, dim3(kEventGrid), dim3(kEventThreads), lds, s, d.step, d.ids,
                     d.id_count, d.id_slots, d.n_pad, d.max_delay, cb.ev_soff, d.run_off, d.run_n, d.run_cap,
                     reinterpret_cast<const u32x2*>(cb.ev_ent), int32_t(cb.n_bundles), cb.ev_cursor,
                     reinterpret_cast<u32x2*>(cb.evbuf));
  return hipGetLastError();
}

hipError_t launch_gather_events(const DeviceNet& d, bool fuse_sums, hipStream_t s) {
  const ConnBlock& cb = d.loc;
  if (cb.n_bundles == 0) return hipSuccess;
  if (!fuse_sums) launch_gather_as<1, kHitsOut, kFromEvents>(d, cb, nullptr, 0, s);
  else if (d.wtype == DTB_W_BF16) launch_gather_as<1, kSumBF16, kFromEvents>(d, cb, nullptr, 0, s);
  else launch_gather_as<1, kSumF32, kFromEvents>(d, cb, nullptr, 0, s);
  return hipGetLastError();
}

hipError_t gather_set_lds_limit() {
  const int bytes = kHitWords * 4;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_events),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     2 * kEvStage * 8 + 3 * kEventMaxBundles * 4);
  for (hipError_t x : {set_lds_limit_one<1, kHitsOut, kFromSweep>(bytes), set_lds_limit_one<2, kHitsOut, kFromSweep>(bytes),
                       set_lds_limit_one<3, kHitsOut, kFromSweep>(bytes), set_lds_limit_one<1, kSumF32, kFromSweep>(bytes),
                       set_lds_limit_one<2, kSumF32, kFromSweep>(bytes), set_lds_limit_one<3, kSumF32, kFromSweep>(bytes),
                       set_lds_limit_one<1, kSumBF16, kFromSweep>(bytes), set_lds_limit_one<2, kSumBF16, kFromSweep>(bytes),
                       set_lds_limit_one<3, kSumBF16, kFromSweep>(bytes), set_lds_limit_one<1, kHitsOut, kFromEvents>(bytes),
                       set_lds_limit_one<1, kSumF32, kFromEvents>(std::max(bytes, kEvLdsBytes)),
                       set_lds_limit_one<1, kSumBF16, kFromEvents>(std::max(bytes, kEvLdsBytes))})
    if (e == hipSuccess) e = x;
  return e;
}

hipError_t launch_sums(const DeviceNet& d, hipStream_t s) {
  const unsigned grid = unsigned((d.n + kSumsRowsPerBlock - 1) / kSumsRowsPerBlock);
  constexpr int kT = kSumsRowsPerBlock / kSumsRows;
  const SumBlock loc{d.loc.bundles, d.loc.block_bundle, d.loc.row_ptr, d.loc.wts, d.loc.hitbuf};
  const SumBlock rem{d.rem.bundles, d.rem.block_bundle, d.rem.row_ptr, d.rem.wts, d.rem.hitbuf};
  const int has_rem = d.rem.n_bundles > 0 ? 1 : 0;
  if (d.wtype == DTB_W_BF16)
    hipLaunchKernelGGL((k_sums<true, kSumsRows>), dim3(grid), dim3(kT), 0, s, d.n, d.step, loc, rem, has_rem,
                       row_tail(d), d.ev);
  else
    hipLaunchKernelGGL((k_sums<false, kSumsRows>), dim3(grid), dim3(kT), 0, s, d.n, d.step, loc, rem, has_rem,
                       row_tail(d), d.ev);
  return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(256) void k_copy_words(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                                    int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) dst[i] = src ? src[i] : 0u;
}
}  // namespace

// dst[0, n) = src[0, n), or zeros when src is null
hipError_t launch_copy_words(uint32_t* dst, const uint32_t* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_words, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(256) void k_fill(float* __restrict__ dst, int64_t n, float v) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) dst[i] = v;
}
}  // namespace

hipError_t launch_fill(float* dst, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

hipError_t launch_finalize(const DeviceNet& d, hipStream_t s) {
  const float E0 = 0.34f;
  BoldParams bp{0.65f, 0.41f, 0.98f, 1.f / 0.32f, E0, std::log(1.f - E0), 0.02f, 0.5f,
                7.f * E0, 2.f, 2.f * E0 - 0.2f, 100.f};
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, d.step, d.slots, d.ev, d.counts, d.n_regions,
                     d.totals, d.inv_nr_dt, d.dt_ms * 1e-3f, d.bold, d.bold_y, bp);
  return hipGetLastError();
}

// ----------------------------------------------------------------- EnKF
// Analysis step of an ensemble Kalman filter over the per-population
// hyper-parameters (the assimilation of Sec. V-E that adapts the
// hyper-parameters by tracking BOLD signals; the filter itself is a stand-in
// for the method the paper defers to its companion work).  One workgroup,
// FP64 throughout: the matrices are tiny and the ensemble is read from L2.
// LDS: xbar [P], ybar [O], C [O][O] (C_yy + R, then its Cholesky factor),
// K [P][O] (C_xy), Z [M][O] (innovations, then (C_yy + R)^-1 d).
namespace {
__device__ inline double bm_normal(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3) {
  uint64_t w1 = 0;
  const uint32_t h0 = uint32_t(philox_hi32_word0(c0, c1, c2, c3, seed, 0ull, &w1));
  const double u1 = (double(h0) + 1.0) * 2.3283064365386962890625e-10;        // (0, 1]
  const double u2 = double(uint32_t(w1 >> 32)) * 2.3283064365386962890625e-10;  // [0, 1)
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2);
}

__global__ __launch_bounds__(256) void k_enkf(int M, int P, int O, float* __restrict__ X,
                                              const float* __restrict__ Y, const float* __restrict__ yobs,
                                              EnkfVar rvar, double infl, uint64_t seed, int64_t iter, float lo,
                                              float hi) {
  extern __shared__ double sm[];
  double* xbar = sm;
  double* ybar = xbar + P;
  double* C = ybar + O;
  double* K = C + O * O;
  double* Z = K + P * O;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double inv = 1.0 / double(M - 1);
  for (int p = tid; p < P; p += nt) {
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += double(X[int64_t(m) * P + p]);
    xbar[p] = s / double(M);
  }
  for (int o = tid; o < O; o += nt) {
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += double(Y[int64_t(m) * O + o]);
    ybar[o] = s / double(M);
  }
  __syncthreads();
  // ensemble covariances (divisor M - 1); the parameter anomalies inflated
  for (int q = tid; q < O * O; q += nt) {
    const int a = q / O, b = q % O;
    double s = 0.0;
    for (int m = 0; m < M; ++m)
      s += (double(Y[int64_t(m) * O + a]) - ybar[a]) * (double(Y[int64_t(m) * O + b]) - ybar[b]);
    C[q] = s * inv + (a == b ? double(rvar.r[a]) : 0.0);
  }
  for (int q = tid; q < P * O; q += nt) {
    const int p = q / O, o = q % O;
    double s = 0.0;
    for (int m = 0; m < M; ++m)
      s += infl * (double(X[int64_t(m) * P + p]) - xbar[p]) * (double(Y[int64_t(m) * O + o]) - ybar[o]);
    K[q] = s * inv;
  }
  // innovations against perturbed observations y + sqrt(r) xi,
  // xi ~ N(0, 1) on Philox counter (iter, m, o, 2)
  for (int q = tid; q < M * O; q += nt) {
    const int m = q / O, o = q % O;
    const double xi = bm_normal(seed, uint64_t(iter), uint64_t(m), uint64_t(o), 2ull);
    Z[q] = double(yobs[o]) + sqrt(double(rvar.r[o])) * xi - double(Y[q]);
  }
  __syncthreads();
  // Cholesky factor of C_yy + R, lower triangle in place, column by column
  for (int k = 0; k < O; ++k) {
    if (tid == 0) {
      double d = C[k * O + k];
      for (int j = 0; j < k; ++j) d -= C[k * O + j] * C[k * O + j];
      C[k * O + k] = sqrt(d);
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < O; i += nt) {
      double s = C[i * O + k];
      for (int j = 0; j < k; ++j) s -= C[i * O + j] * C[k * O + j];
      C[i * O + k] = s / C[k * O + k];
    }
    __syncthreads();
  }
  // each member's z = (L L^T)^-1 d: forward, then backward substitution
  for (int m = tid; m < M; m += nt) {
    double* z = Z + int64_t(m) * O;
    for (int i = 0; i < O; ++i) {
      double s = z[i];
      for (int j = 0; j < i; ++j) s -= C[i * O + j] * z[j];
      z[i] = s / C[i * O + i];
    }
    for (int i = O - 1; i >= 0; --i) {
      double s = z[i];
      for (int j = i + 1; j < O; ++j) s -= C[j * O + i] * z[j];
      z[i] = s / C[i * O + i];
    }
  }
  __syncthreads();
  // x_m <- xbar + infl (x_m - xbar) + C_xy z_m, clamped to [lo, hi]
  for (int q = tid; q < M * P; q += nt) {
    const int m = q / P, p = q % P;
    double u = 0.0;
    for (int o = 0; o < O; ++o) u += K[p * O + o] * Z[int64_t(m) * O + o];
    const double x = xbar[p] + infl * (double(X[q]) - xbar[p]) + u;
    X[q] = float(fmin(fmax(x, double(lo)), double(hi)));
  }
}
}  // namespace

size_t enkf_lds_bytes(int M, int P, int O) {
  return size_t(8) * (size_t(P) + size_t(O) + size_t(O) * O + size_t(P) * O + size_t(M) * O);
}

hipError_t launch_enkf(int M, int P, int O, float* X, const float* Y, const float* yobs, const EnkfVar& rvar,
                       double infl, uint64_t seed, int64_t iter, float lo, float hi, hipStream_t s) {
  const size_t lds = enkf_lds_bytes(M, P, O);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_enkf),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_enkf, dim3(1), dim3(256), lds, s, M, P, O, X, Y, yobs, rvar, infl, seed, iter, lo, hi);
  return hipGetLastError();
}

}  // namespace dtb
