// dtb_kernels.hip - gfx950 kernels of one partition step.
//
// A step t is, in stream order (the computing cycle of Sec. V-B / VI-C):
//   k_neuron_update  membrane update of Eq. (1) by forward Euler (Sec. VI-A),
//                    threshold / reset / refractory, spike into the delay
//                    ring, wavefront ballot into the step's spike bitmap,
//                    per-population spike counts;
//   k_compact        ascending spike-id list from the bitmap (ballot
//                    popcounts, block scan, decoupled look-back);
//   k_gather         pull over each row's in-edges in CSR order through the
//                    delay ring (J_intra), plus the Poisson count that stands
//                    in for the spikes of other partitions (J_inter), then
//                    the gate update (jump + exact exponential decay);
//   k_finalize       per-step event totals.
//
// Everything is FP32 except the integer work (ids, delays, ballots, counts,
// RNG).  The file is compiled with -ffp-contract=off: every fused
// multiply-add below is written out, so the arithmetic is the source's.
#include <hip/hip_runtime.h>

#include "dtb_internal.h"

namespace dtb {
namespace {

// ------------------------------------------------------------------ RNG
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 64x64 -> 128-bit products, key bumped by the Weyl constants between rounds.
__device__ inline uint64_t philox_hi32_word0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                             uint64_t k0, uint64_t k1) {
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
  return c0 >> 32;
}

__device__ inline int poisson_count(uint32_t u, const uint32_t* __restrict__ T, int K) {
  int c = 0;
  while (c < K && u >= T[c]) ++c;
  return c;
}

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// ----------------------------------------------------------- neuron update
// One thread per neuron, 1024 threads (16 wavefronts) per block.
__global__ __launch_bounds__(1024) void k_neuron_update(
    int64_t n, int64_t n_pad, int64_t t, float* __restrict__ V, const float* __restrict__ j,
    uint8_t* __restrict__ ref, const uint16_t* __restrict__ ptype, const int32_t* __restrict__ region,
    uint32_t* __restrict__ ring, const PType* __restrict__ ptab, const float* __restrict__ gain,
    float E0, float E1, float E2, float E3, const uint32_t* __restrict__ forced,
    uint32_t* __restrict__ raster_slot, int32_t* __restrict__ counts_slot, uint32_t* __restrict__ cticket,
    int32_t* __restrict__ bad) {
  __shared__ int s_reg[16];
  __shared__ int s_cnt[16];
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool valid = i < n;
  int s = 0, reg = 0;
  if (valid) {
    const float v = V[i];
    const int r = ref[i];
    const PType p = ptab[ptype[i]];
    reg = region[i];
    const float* gn = gain + 4 * reg;
    float vt = 0.f;
    if (r <= 0) {
      // I = Iext + sum_u (g_u gain_u) j_u (E_u - V) - gL (V - EL);  V~ = V + dt/C I
      float I = p.Iext;
      I = __fmaf_rn((p.g[0] * gn[0]) * j[i], E0 - v, I);
      I = __fmaf_rn((p.g[1] * gn[1]) * j[n_pad + i], E1 - v, I);
      I = __fmaf_rn((p.g[2] * gn[2]) * j[2 * n_pad + i], E2 - v, I);
      I = __fmaf_rn((p.g[3] * gn[3]) * j[3 * n_pad + i], E3 - v, I);
      I = __fmaf_rn(-p.gL, v - p.EL, I);
      vt = __fmaf_rn(p.dtC, I, v);
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
    const uint32_t bit = 1u << (uint32_t(t) & 31u);
    const uint32_t h = ring[i];
    ring[i] = s ? (h | bit) : (h & ~bit);
  }
  // the wavefront's 64 spike predicates are 64 consecutive bits of the bitmap
  const uint64_t m = __ballot(s);
  const int64_t wave_first = int64_t(blockIdx.x) * 1024 + wave * 64;
  if (lane == 0) {
    raster_slot[wave_first >> 5] = uint32_t(m);
    raster_slot[(wave_first >> 5) + 1] = uint32_t(m >> 32);
  }
  // population counts: one entry per wavefront when it lies in one population
  const int r0 = __shfl(reg, 0);
  const int uniform = __all((!valid || reg == r0) ? 1 : 0);
  if (uniform) {
    if (lane == 0) {
      s_reg[wave] = r0;
      s_cnt[wave] = __popcll(m);
    }
  } else {
    if (s) atomicAdd(&counts_slot[reg], 1);
    if (lane == 0) {
      s_reg[wave] = -1;
      s_cnt[wave] = 0;
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
// Each thread owns 64 neurons (two bitmap words).  Blocks take a dynamic
// ticket so that a block only waits on blocks that are already running.
// Look-back status word: epoch (32) | flag (2: 1 aggregate, 2 prefix) | value (30).
__device__ inline uint64_t pack_status(uint32_t epoch, uint32_t flag, uint32_t value) {
  return (uint64_t(epoch) << 32) | (uint64_t(flag) << 30) | uint64_t(value);
}

__global__ __launch_bounds__(kCompactBlock) void k_compact(
    const uint32_t* __restrict__ bits, int64_t words, int64_t n_blocks, uint32_t epoch,
    int32_t* __restrict__ ids, int32_t* __restrict__ id_count, uint64_t* __restrict__ status,
    uint32_t* __restrict__ ticket, int64_t* __restrict__ spike_total) {
  __shared__ uint32_t s_bid;
  __shared__ int s_wave[kCompactBlock / 64];
  __shared__ int s_excl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_bid = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t bid = s_bid;
  const int64_t w0 = (bid * kCompactBlock + tid) * 2;
  uint32_t a = w0 < words ? bits[w0] : 0u;
  uint32_t b = w0 + 1 < words ? bits[w0 + 1] : 0u;
  const int c = __popc(a) + __popc(b);
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
  if (tid == 0) {
    uint32_t excl = 0;
    if (bid == 0) {
      __hip_atomic_store(&status[0], pack_status(epoch, 2, uint32_t(agg)), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&status[bid], pack_status(epoch, 1, uint32_t(agg)), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
      int64_t p = bid - 1;
      while (true) {
        const uint64_t st = __hip_atomic_load(&status[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t flag = uint32_t(st >> 30) & 3u;
        if (uint32_t(st >> 32) != epoch || flag == 0) continue;  // predecessor still running
        excl += uint32_t(st) & 0x3FFFFFFFu;
        if (flag == 2) break;
        --p;
      }
      __hip_atomic_store(&status[bid], pack_status(epoch, 2, excl + uint32_t(agg)), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    s_excl = int(excl);
    if (bid == n_blocks - 1) {
      *id_count = int(excl) + agg;
      atomicAdd(reinterpret_cast<unsigned long long*>(spike_total), (unsigned long long)(excl + agg));
    }
  }
  __syncthreads();
  int off = s_excl + wave_off + x - c;
  const int32_t base = int32_t(w0 * 32);
  while (a) {
    const int q = __ffs(a) - 1;
    ids[off++] = base + q;
    a &= a - 1u;
  }
  while (b) {
    const int q = __ffs(b) - 1;
    ids[off++] = base + 32 + q;
    b &= b - 1u;
  }
}

// ------------------------------------------------------------------ gather
// One wavefront per SELL-64 slice (64 consecutive rows), one lane per row.
// Lane `l` walks its row in CSR order k = 0, 1, ...: the slice stores entry
// (k, l) at slice_off + 64 k + l, so the wavefront's loads of one k are one
// contiguous 256-byte segment.  A synapse delivers when bit (t - d + 1) & 31
// of its presynaptic neuron's ring word is set.
template <bool kBF16>
__global__ __launch_bounds__(256) void k_gather(
    int64_t n, int64_t n_slices, int64_t n_pad, int64_t t, int32_t member, uint64_t seed,
    const uint32_t* __restrict__ syn, const void* __restrict__ wts_v, const int64_t* __restrict__ slice_off,
    const int32_t* __restrict__ slice_len, const int32_t* __restrict__ row_len,
    const uint32_t* __restrict__ ring, float* __restrict__ j, float a0, float a1, float a2, float a3,
    float bg_w, const uint32_t* __restrict__ poisson, int K, int64_t* __restrict__ ev_slot,
    int32_t* __restrict__ bad) {
  __shared__ int64_t s_ev[4][2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t slice = int64_t(blockIdx.x) * 4 + wave;
  uint32_t ev = 0, evb = 0;
  if (slice < n_slices) {
    const int64_t row = slice * kSlice + lane;
    const int64_t base = slice_off[slice];
    const int L = slice_len[slice];
    const int len = row_len[row];
    const uint32_t* sp = syn + base + lane;
    const float* wf = reinterpret_cast<const float*>(wts_v) + base + lane;
    const uint16_t* wb = reinterpret_cast<const uint16_t*>(wts_v) + base + lane;
    const uint32_t tt = uint32_t(t);
    float dE = 0.f, dI = 0.f;
    int k = 0;
    for (; k + 8 <= L; k += 8) {
      uint32_t wd[8], h[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) wd[u] = sp[int64_t(k + u) * kSlice];
#pragma unroll
      for (int u = 0; u < 8; ++u) h[u] = (k + u < len) ? ring[wd[u] & kColMask] : 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t hit = (h[u] >> ((tt - ((wd[u] >> kColBits) & 31u)) & 31u)) & 1u;
        if (hit) {
          const int64_t o = int64_t(k + u) * kSlice;
          const float w = kBF16 ? bf16_to_f32(wb[o]) : wf[o];
          if (wd[u] >> 31) dI += w;
          else dE += w;
          ++ev;
        }
      }
    }
    for (; k < L; ++k) {
      const uint32_t wd = sp[int64_t(k) * kSlice];
      const uint32_t h = (k < len) ? ring[wd & kColMask] : 0u;
      if ((h >> ((tt - ((wd >> kColBits) & 31u)) & 31u)) & 1u) {
        const int64_t o = int64_t(k) * kSlice;
        const float w = kBF16 ? bf16_to_f32(wb[o]) : wf[o];
        if (wd >> 31) dI += w;
        else dE += w;
        ++ev;
      }
    }
    if (row < n) {
      // background Poisson count: Philox4x64-10, key (seed, 0), counter (t, i, member, 0)
      const uint32_t u = uint32_t(philox_hi32_word0(uint64_t(t), uint64_t(row), uint64_t(member), 0ull, seed, 0ull));
      const int c = poisson_count(u, poisson, K);
      evb = uint32_t(c);
      dE = __fmaf_rn(float(c), bg_w, dE);
      float* jr = j + row;
      const float ja = __fmaf_rn(a0, jr[0], dE);
      const float jn = __fmaf_rn(a1, jr[n_pad], dE);
      const float jga = __fmaf_rn(a2, jr[2 * n_pad], dI);
      const float jgb = __fmaf_rn(a3, jr[3 * n_pad], dI);
      jr[0] = ja;
      jr[n_pad] = jn;
      jr[2 * n_pad] = jga;
      jr[3 * n_pad] = jgb;
      if (!(isfinite(ja) && isfinite(jn) && isfinite(jga) && isfinite(jgb))) atomicOr(bad, 1);
    }
  }
  // block totals of delivered events, then one striped atomic per block
  uint32_t e = ev, eb = evb;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_down(e, off);
    eb += __shfl_down(eb, off);
  }
  if (lane == 0) {
    s_ev[wave][0] = e;
    s_ev[wave][1] = eb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t r = s_ev[0][0] + s_ev[1][0] + s_ev[2][0] + s_ev[3][0];
    const int64_t bgs = s_ev[0][1] + s_ev[1][1] + s_ev[2][1] + s_ev[3][1];
    int64_t* dst = ev_slot + 2 * (blockIdx.x & (kStripes - 1));
    if (r) atomicAdd(reinterpret_cast<unsigned long long*>(dst), (unsigned long long)r);
    if (bgs) atomicAdd(reinterpret_cast<unsigned long long*>(dst + 1), (unsigned long long)bgs);
  }
}

// ---------------------------------------------------------------- finalize
// Reduce the striped event counters of step t, add them to the totals, and
// clear the ring slot that step t+1 will fill.
__global__ __launch_bounds__(64) void k_finalize(int64_t* __restrict__ ev_slot, int64_t* __restrict__ ev_next,
                                                 int32_t* __restrict__ counts_next, int32_t n_regions,
                                                 int64_t* __restrict__ totals) {
  const int lane = threadIdx.x;
  int64_t r = ev_slot[2 * lane], b = ev_slot[2 * lane + 1];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    r += __shfl_down(r, off);
    b += __shfl_down(b, off);
  }
  __syncthreads();
  if (lane == 0) {
    ev_slot[0] = r;
    ev_slot[1] = b;
    totals[1] += r;
    totals[2] += b;
    totals[3] += 1;
  }
  ev_next[2 * lane] = 0;
  ev_next[2 * lane + 1] = 0;
  for (int q = lane; q < n_regions; q += 64) counts_next[q] = 0;
}

}  // namespace

hipError_t launch_neuron_update(const DeviceNet& d, int64_t t, const uint32_t* forced, hipStream_t s) {
  const int64_t slot = t % (d.rec + 1);
  const unsigned grid = unsigned(d.n_pad / 1024);
  hipLaunchKernelGGL(k_neuron_update, dim3(grid), dim3(1024), 0, s, d.n, d.n_pad, t, d.V, d.j, d.ref,
                     d.ptype, d.region, d.ring, d.ptab, d.gain, d.E[0], d.E[1], d.E[2], d.E[3], forced,
                     d.raster + slot * d.words_pad, d.counts + slot * d.n_regions, d.cticket, d.bad);
  return hipGetLastError();
}

hipError_t launch_compact(const DeviceNet& d, int64_t t, hipStream_t s) {
  const int64_t slot = t % (d.rec + 1);
  hipLaunchKernelGGL(k_compact, dim3(unsigned(d.compact_blocks)), dim3(kCompactBlock), 0, s,
                     d.raster + slot * d.words_pad, d.words_pad, d.compact_blocks,
                     uint32_t(uint64_t(t) + 1u), d.ids, d.id_count, d.cstatus, d.cticket, d.totals);
  return hipGetLastError();
}

hipError_t launch_gather(const DeviceNet& d, int64_t t, hipStream_t s) {
  const int64_t slot = t % (d.rec + 1);
  const unsigned grid = unsigned((d.n_slices + 3) / 4);
  int64_t* evs = d.ev + slot * kStripes * 2;
  if (d.wtype == DTB_W_BF16)
    hipLaunchKernelGGL(k_gather<true>, dim3(grid), dim3(256), 0, s, d.n, d.n_slices, d.n_pad, t, d.member,
                       d.seed, d.syn, d.wts, d.slice_off, d.slice_len, d.row_len, d.ring, d.j, d.a[0], d.a[1],
                       d.a[2], d.a[3], d.bg_w, d.poisson, d.poisson_K, evs, d.bad);
  else
    hipLaunchKernelGGL(k_gather<false>, dim3(grid), dim3(256), 0, s, d.n, d.n_slices, d.n_pad, t, d.member,
                       d.seed, d.syn, d.wts, d.slice_off, d.slice_len, d.row_len, d.ring, d.j, d.a[0], d.a[1],
                       d.a[2], d.a[3], d.bg_w, d.poisson, d.poisson_K, evs, d.bad);
  return hipGetLastError();
}

hipError_t launch_finalize(const DeviceNet& d, int64_t t, hipStream_t s) {
  const int64_t slot = t % (d.rec + 1), next = (t + 1) % (d.rec + 1);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, d.ev + slot * kStripes * 2,
                     d.ev + next * kStripes * 2, d.counts + next * d.n_regions, d.n_regions, d.totals);
  return hipGetLastError();
}

}  // namespace dtb
