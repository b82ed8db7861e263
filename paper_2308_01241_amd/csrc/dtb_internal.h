// dtb_internal.h - device data layout of one partition and the kernel
// launchers shared by the host API (dtb_api.cpp) and the kernels
// (dtb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/dtb.h"

namespace dtb {

// Packed synapse word of the connection table (Sec. V-D), one per synapse:
//   bits  0..25  presynaptic neuron id (n < 2^26)
//   bits 26..30  delay - 1             (1 <= delay <= 31)
//   bit  31      presynaptic neuron is inhibitory
constexpr uint32_t kColBits = 26;
constexpr uint32_t kColMask = (1u << kColBits) - 1u;
constexpr int kMaxDelay = 31;
constexpr int64_t kMaxNeurons = (int64_t(1) << kColBits) - 1;
constexpr int kSlice = 64;          // rows per SELL slice = one wavefront
constexpr int kNeuronPad = 1024;    // neuron arrays padded to this multiple
constexpr int kStripes = 64;        // striped event counters per step
constexpr int kMaxPoisson = 512;    // entries of the background inversion table
constexpr int kCompactBlock = 256;  // threads of the compaction kernel
constexpr int kCompactPerBlock = kCompactBlock * 64;  // neurons per compaction block

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
  int64_t n = 0, n_pad = 0, words = 0, n_slices = 0, total_slots = 0;
  int32_t n_regions = 0, max_delay = 0, n_ptypes = 0, member = 0;
  int32_t wtype = 0, rec = 0;       // rec = record_steps; rings hold rec + 1 slots
  int32_t poisson_K = 0;
  int64_t compact_blocks = 0;
  float a[4] = {0, 0, 0, 0};        // exp(-dt / tau_u)
  float E[4] = {0, 0, 0, 0};        // reversal potentials
  float bg_w = 0.f;
  uint64_t seed = 0;
  // neuron state (SoA) and tables
  float* V = nullptr;               // [n_pad]
  float* j = nullptr;               // [4][n_pad]
  uint8_t* ref = nullptr;           // [n_pad]
  uint16_t* ptype = nullptr;        // [n_pad]
  int32_t* region = nullptr;        // [n_pad]
  uint32_t* ring = nullptr;         // [n_pad] delay ring: bit (t & 31) holds s^t
  PType* ptab = nullptr;            // [n_ptypes]
  float* gain = nullptr;            // [n_regions][4]
  uint32_t* poisson = nullptr;      // [poisson_K]
  // connection table, SELL-64
  uint32_t* syn = nullptr;          // [total_slots] packed words
  void* wts = nullptr;              // [total_slots] float or bf16 (uint16)
  int64_t* slice_off = nullptr;     // [n_slices]
  int32_t* slice_len = nullptr;     // [n_slices]
  int32_t* row_len = nullptr;       // [n_pad]
  // history and outputs
  uint32_t* raster = nullptr;       // [rec + 1][words_pad] spike bitmaps
  int32_t* counts = nullptr;        // [rec + 1][n_regions]
  int64_t* ev = nullptr;            // [rec + 1][kStripes][2] striped (rec, bg); [slot][0][*] final
  int64_t* totals = nullptr;        // [4]: spikes, ev_rec, ev_bg, steps
  int32_t* ids = nullptr;           // [n_pad] ascending spike ids of the last step
  int32_t* id_count = nullptr;      // [1]
  uint64_t* cstatus = nullptr;      // [compact_blocks] look-back status words
  uint32_t* cticket = nullptr;      // [1] dynamic block ticket
  uint32_t* force = nullptr;        // [rec + 1][words_pad] pending forced bitmaps
  int32_t* bad = nullptr;           // [1] non-finite flag
  int64_t words_pad = 0;
};

// launchers (dtb_kernels.hip); all enqueue on `s`
hipError_t launch_neuron_update(const DeviceNet& d, int64_t t, const uint32_t* forced, hipStream_t s);
hipError_t launch_compact(const DeviceNet& d, int64_t t, hipStream_t s);
hipError_t launch_gather(const DeviceNet& d, int64_t t, hipStream_t s);
hipError_t launch_finalize(const DeviceNet& d, int64_t t, hipStream_t s);

}  // namespace dtb
