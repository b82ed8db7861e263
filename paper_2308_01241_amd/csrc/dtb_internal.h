// dtb_internal.h - device data layout of one partition and the kernel
// launchers shared by the host API (dtb_api.cpp) and the kernels
// (dtb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dtb.h"

namespace dtb {

constexpr int kMaxDelay = 31;
constexpr int64_t kMaxNeurons = (int64_t(1) << 26) - 1;
constexpr int kNeuronPad = 1024;    // neuron arrays padded to this multiple
constexpr int kStripes = 64;        // striped event counters per step
constexpr int kMaxPoisson = 512;    // entries of the background inversion table
constexpr int kCompactBlock = 256;  // threads of the compaction kernel
constexpr int kCompactWords = 8;    // bitmap words per compaction thread

// ---- gather layout ("bundles") --------------------------------------------
// Rows are cut into bundles of consecutive rows holding at most
// kBundleMaxSyn synapses.  One workgroup owns a bundle.  A bundle's synapses
// are stored twice:
//  * the weight stream, in CSR order (= the fixed summation order), the sign
//    bit marking an inhibitory presynaptic neuron;
//  * the lookup stream: the same synapses sorted by (delay, source), cut into
//    tiles of 256 entries stored plane-major (a wavefront loads one tile as
//    one 16-byte load per lane: lane l holds sorted entries l, 64+l, 128+l,
//    192+l).  Entry = source delta (12 bits,
//    relative to the previous entry of the tile; the first entry has delta 0)
//    << 20 | position of the synapse in the bundle's CSR range (20 bits).
//    Padding entries (the tail of a tile) have delta 0 and position nsyn,
//    one past the bundle's last synapse: a bit the sums never read.  A
//    source gap wider than 4095 inside a tile is bridged by skip entries
//    (delta 4095, position nsyn) when it needs at most 64 of them; a wider
//    gap, or a new delay, starts a new tile.
//    Tile header = first source of the tile (26 bits) | (delay - 1) << 26.
constexpr int kTile = 256;
constexpr int kPosBits = 20;
constexpr uint32_t kPosMask = (1u << kPosBits) - 1u;
constexpr uint32_t kMaxDelta = (1u << (32 - kPosBits)) - 1u;  // 4095
constexpr uint32_t kMaxSkips = 64;  // widest gap bridged by skip entries: 64 deltas
constexpr int64_t kBundleMaxSyn = int64_t(kPosMask);         // synapses 0 .. 2^20 - 2, padding at nsyn
constexpr int kHitWords = int(kBundleMaxSyn >> 5) + 1;       // LDS hit bitmap words of the largest bundle

// Gather launch shape: threads per workgroup, the default lookup tiles per
// wavefront per round (the kernel is compiled for 1, 2 and 3; the handle
// picks one) and whether the data each step reads once is loaded
// non-temporally.  The default bundle fills the LDS hit bitmap (128 KB of
// the CU's 160 KB): one 1024-thread workgroup per CU.  With one tile per
// round the kernel fits 64 VGPRs, so two workgroups share a CU when their
// bundles leave the LDS for it.
#ifndef DTB_GATHER_THREADS
#define DTB_GATHER_THREADS 1024
#endif
// rows per thread of the sums kernel (1 or 2; two rows' loads in flight per
// thread cost more registers than they hide latency: 0.535 vs 0.488 ms)
#ifndef DTB_SUMS_ROWS
#define DTB_SUMS_ROWS 1
#endif
constexpr int kSumsRows = DTB_SUMS_ROWS;
static_assert(kSumsRows == 1 || kSumsRows == 2, "rows per sums thread: 1 or 2");

// neurons per thread of the neuron update (1, 2 or 4)
#ifndef DTB_UPDATE_NPT
#define DTB_UPDATE_NPT 2
#endif
constexpr int kUpdateNpt = DTB_UPDATE_NPT;
static_assert(kUpdateNpt == 1 || kUpdateNpt == 2 || kUpdateNpt == 4, "neurons per thread: 1, 2 or 4");

#ifndef DTB_GATHER_UNROLL
#define DTB_GATHER_UNROLL 3
#endif
#ifndef DTB_GATHER_NT
#define DTB_GATHER_NT 1
#endif
#ifndef DTB_GATHER_BUNDLE_SYN
#define DTB_GATHER_BUNDLE_SYN 1048575
#endif
constexpr int kGatherThreads = DTB_GATHER_THREADS;
constexpr int kTimedKernels = 9;  // neuron update, compaction, gather, sums, finalize, remote gather, events,
                                  // spike runs, background
constexpr int kGatherUnroll = DTB_GATHER_UNROLL;
constexpr int64_t kBundleDefaultSyn = DTB_GATHER_BUNDLE_SYN;
static_assert(kBundleDefaultSyn <= kBundleMaxSyn, "bundle positions are 20 bits");

struct Bundle {
  int64_t row0, row1;   // rows [row0, row1)
  int64_t member_row0;  // first row of the member network the bundle belongs to
  uint64_t seed;        // the member's background seed (Philox key)
  int32_t member;       // member id (background counter)
  int32_t pad;
  int64_t syn0;         // CSR index of the bundle's first synapse
  int64_t tile0;        // first tile of the bundle's lookup stream
  int32_t ntiles;       // tiles of the lookup stream
  int32_t nsyn;         // synapses of the bundle
  int64_t hbit0;        // bit of the hit buffer that holds the bundle's synapse 0 (a multiple of 32)
};

// One in-edge block in the gather's layout: the rows' synapses cut into
// bundles, their lookup tiles, the per-bundle hit words written by the
// delivery tests, and the CSR row pointers and signed weights the sums read.
// A partition has its local block (sources = its own neurons) and, with
// dtb_set_remote_block, a remote block (sources = neurons of other
// partitions, replayed).
struct ConnBlock {
  int64_t n_bundles = 0, n_tiles = 0;
  int32_t hit_words = 1;            // LDS words of the largest bundle's hit bitmap
  int64_t hit_total_words = 0;
  int64_t xcd_max = 0;              // most bundles of one XCD
  Bundle* bundles = nullptr;        // [n_bundles]
  int32_t* block_bundle = nullptr;  // [ceil(n / 1024)] bundle of each 1024-row block's first row
  int64_t* xcd_first = nullptr;     // [9] bundles [xcd_first[x], xcd_first[x+1]) go to XCD x (equal tiles)
  uint32_t* tiles = nullptr;        // [n_tiles][kTile] lookup entries
  uint32_t* theads = nullptr;       // [n_tiles] tile headers
  uint32_t* hitbuf = nullptr;       // [hit_total_words] delivery-test results: per bundle, one bit per
                                    // synapse in CSR order (from bit hbit0), rewritten every step
  int64_t* row_ptr = nullptr;       // [n + 1]
  void* wts = nullptr;              // [nnz] float or bf16, sign bit = inhibitory source
  // spike-driven delivery (gather_events = 2; local block only): the
  // synapses grouped by source and, within a source, by delay, each as the
  // pair (bundle << kPosBits | position in the bundle, weight bits as the
  // row sums take them: FP32 bits or BF16 bits << 16, sign = inhibitory);
  // a step's deliveries are bucketed per bundle into evbuf as pairs
  // (position, weight bits) (bundle b's bucket at its syn0, room for all
  // its synapses), filled up to ev_cursor[b] (syn0 while empty)
  uint32_t* ev_ent = nullptr;       // [nnz][2]
  uint32_t* ev_soff = nullptr;      // [n_src][D + 1]: (m, d) = [soff[m (D+1) + d - 1], soff[m (D+1) + d])
  uint32_t* evbuf = nullptr;        // [nnz][2]
  uint32_t* ev_cursor = nullptr;    // [n_bundles]
};

constexpr int kEventMaxBundles = 1 << (32 - kPosBits);  // bundle ids fit the 12 high bits of an entry
constexpr int kEventThreads = 1024;  // threads of the bucketing kernel
constexpr int kEventGrid = 256;      // its workgroups (one per CU: its LDS staging takes most of a CU's)
// LDS of the spike-driven row sums: a bundle's hit bitmap, the hit counts
// before every group of kEvGroupWords bitmap words, and the delivered
// weights in position order (as many as fit the rest)
constexpr int kEvLdsBytes = 160 * 1024 - 1024;
constexpr int kEvGroupWords = 4;
__host__ __device__ constexpr int ev_groups(int hit_words) { return (hit_words + kEvGroupWords - 1) / kEvGroupWords; }
// (-1: not even the bitmap and the prefix counts fit)
__host__ __device__ constexpr int ev_weight_cap(int hit_words) {
  return kEvLdsBytes / 4 - hit_words - ev_groups(hit_words) >= 0 ? kEvLdsBytes / 4 - hit_words - ev_groups(hit_words)
                                                                   : -1;
}

// Derived per-type constants in the order the neuron update reads them.
struct PType {
  float dtC;      // dt / C (rounded once from FP64)
  float gL, EL, Vth, Vreset, Iext;
  float g[4];
  int32_t nref;   // round(tref / dt)
  int32_t pad;
};

struct DeviceNet {
  // sizes
  int64_t n = 0, n_pad = 0, words = 0, words_pad = 0, nnz = 0;
  int32_t n_regions = 0, max_delay = 0, n_ptypes = 0, member = 0;
  int32_t wtype = 0, rec = 0;       // rec = record_steps
  int32_t unroll = 3;               // gather lookup tiles per wavefront per round (1 .. 3)
  int32_t fuse = 1;                 // row sums in the gather's workgroups (1) or in k_sums (2)
  int32_t events = 0;               // 1: the local block's deliveries are spike-driven (event table)
  int32_t id_slots = 1;             // spike-id lists kept: D + 1 with events (one per delay), else 1
  int32_t slots = 0;                // spike-bitmap ring slots: max(rec, D) + 1
  int32_t poisson_K = 0, poisson_cap = 1;
  int64_t compact_blocks = 0;
  float a[4] = {0, 0, 0, 0};        // exp(-dt / tau_u)
  float E[4] = {0, 0, 0, 0};        // reversal potentials
  float bg_w = 0.f;
  uint64_t seed = 0;
  // Ornstein-Uhlenbeck background (off while ou is null or ou_on == 0)
  int32_t ou_on = 0;
  float ou_mu = 0.f, ou_a = 0.f, ou_s = 0.f;  // mean, exp(-dt / tau), sigma sqrt(1 - a^2)
  float* ou = nullptr;              // [n_pad] I_ou
  uint16_t* bgc = nullptr;          // [n_pad] the step's Poisson background count per neuron
  // neuron state (SoA) and tables
  float* V = nullptr;               // [n_pad]
  float* V0 = nullptr;              // [n_pad] initial potentials (for dtb_reset)
  float* j = nullptr;               // [4][n_pad]
  uint8_t* ref = nullptr;           // [n_pad]
  uint16_t* ptype = nullptr;        // [n_pad]
  int32_t* region = nullptr;        // [n_pad]
  PType* ptab = nullptr;            // [n_ptypes]
  float* gain = nullptr;            // [n_regions][4]
  uint32_t* poisson = nullptr;      // [poisson_K]
  // connection tables: local sources, and the optional remote-source block
  ConnBlock loc, rem;
  int64_t n_remote = 0, rwords_pad = 0;  // remote neurons; words of one remote bitmap (padded)
  uint32_t* rraster = nullptr;      // [slots][rwords_pad] remote spike bitmaps: the remote delay ring
  uint32_t* rqueue = nullptr;       // [rec + 1][rwords_pad] pushed remote bitmaps not yet consumed
  // history and outputs
  uint32_t* raster = nullptr;       // [slots][words_pad] spike bitmaps: the delay ring
  int32_t* counts = nullptr;        // [slots][n_regions]
  int64_t* ev = nullptr;            // [slots][kStripes][2] striped (rec, bg); [slot][0][*] final
  int64_t* totals = nullptr;        // [4]: spikes, ev_rec, ev_bg, steps
  int32_t* ids = nullptr;           // [id_slots][n_pad] ascending spike ids: step t's list in slot t mod id_slots
  int32_t* id_count = nullptr;      // [id_slots]
  // spike-driven delivery: the event-table run offsets of each listed spike
  // (its soff row), delay-major per slot, for the first run_n[slot] spikes
  int64_t run_cap = 0;              // spikes per slot with gathered offsets
  uint32_t* run_off = nullptr;      // [id_slots][D + 1][run_cap]
  int32_t* run_n = nullptr;         // [id_slots]
  // spike list of an earlier recorded step, rebuilt on request from its
  // ring slot: [0] epoch - 1, [1] slot | ids | count | look-back status words,
  // ticket, spike-total sink
  int64_t* rd_at = nullptr;         // [2]
  int32_t* rd_ids = nullptr;        // [n_pad]
  int32_t* rd_count = nullptr;      // [1]
  uint64_t* rd_status = nullptr;    // [compact_blocks]
  uint32_t* rd_ticket = nullptr;    // [1]
  int64_t* rd_total = nullptr;      // [1]
  uint64_t* cstatus = nullptr;      // [compact_blocks] look-back status words
  uint32_t* cticket = nullptr;      // [1] dynamic block ticket
  uint32_t* force = nullptr;        // [rec + 1][words_pad] pending forced bitmaps
  int32_t* bad = nullptr;           // [1] non-finite flag
  int64_t* step = nullptr;          // [2] device step counter: t, t mod slots
  float* inv_nr_dt = nullptr;       // [n_regions] 1 / (neurons of the population * dt in s)
  float* bold = nullptr;            // [n_regions][4] Balloon-Windkessel state (deviations from rest)
  float* bold_y = nullptr;          // [n_regions] BOLD signal after the last step
  float dt_ms = 1.f;
};

// launchers (dtb_kernels.hip); all enqueue on `s`
// Every kernel reads the step t from d.step, so a sequence of launches can be
// captured once and replayed; k_finalize (last of a step) advances it.
hipError_t launch_neuron_update(const DeviceNet& d, const uint32_t* forced, hipStream_t s);
// the step's Poisson background counts of the local rows (none with the OU
// current); after the neuron update, before the row sums read them
hipError_t launch_background(const DeviceNet& d, hipStream_t s);
hipError_t launch_compact(const DeviceNet& d, hipStream_t s);
hipError_t launch_compact_read(const DeviceNet& d, const int64_t* at, int32_t* ids, int32_t* count,
                               uint64_t* status, uint32_t* ticket, int64_t* total, hipStream_t s);
hipError_t launch_sums(const DeviceNet& d, hipStream_t s);
// delivery tests of one in-edge block; with fuse_sums the same workgroups
// then sum their bundles' rows and update background and gates (no k_sums
// needed: the partition has no other block), otherwise the hit bits go to
// the block's hit buffer for launch_sums
hipError_t launch_gather(const DeviceNet& d, const ConnBlock& cb, const uint32_t* bitmaps, int64_t words_pad,
                         bool fuse_sums, hipStream_t s);
// spike-driven delivery of the local block: the table run offsets of the
// step's spikes gathered once (k_spike_runs, after the compaction), the
// deliveries of the spikes of steps t .. t-D+1 through their delays bucketed
// per bundle (k_events), then per bundle the hit bitmap from its bucket and,
// like launch_gather, the row sums or the hit words (k_gather on the buckets)
hipError_t launch_spike_runs(const DeviceNet& d, hipStream_t s);
hipError_t launch_events(const DeviceNet& d, hipStream_t s);
hipError_t launch_gather_events(const DeviceNet& d, bool fuse_sums, hipStream_t s);
// observation-error variances of one EnKF analysis, passed by value
constexpr int kEnkfMaxObs = 64;
struct EnkfVar {
  float r[kEnkfMaxObs];
};
size_t enkf_lds_bytes(int M, int P, int O);
hipError_t launch_enkf(int M, int P, int O, float* X, const float* Y, const float* yobs, const EnkfVar& rvar,
                       double infl, uint64_t seed, int64_t iter, float lo, float hi, hipStream_t s);
hipError_t launch_copy_words(uint32_t* dst, const uint32_t* src, int64_t n, hipStream_t s);
hipError_t launch_finalize(const DeviceNet& d, hipStream_t s);
hipError_t launch_fill(float* dst, int64_t n, float v, hipStream_t s);
hipError_t gather_set_lds_limit();

}  // namespace dtb
