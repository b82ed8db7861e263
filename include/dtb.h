/*
 * dtb.h - C ABI of the MI355X partition simulator for the conductance-based
 * leaky integrate-and-fire network of "Digital Twin Brain" (arXiv 2308.01241).
 *
 * One handle holds one partition of the network on one GPU: the neuron
 * property table and connection table of Sec. V-D, the neuron state of
 * Sec. III-B Eq. (1), and the integer delay ring that carries spikes between
 * steps.  A step is the computing cycle of Sec. V-B / VI-C: membrane update
 * and spike collection, then the weighted sum over presynaptic spikes
 * (J_intra) with the spikes of other partitions (J_inter) replaced by a seeded
 * Poisson count, then the gate update.  Time stepping is forward Euler with
 * dt = 1 ms (Sec. VI-A); gates jump and decay exponentially (Sec. III-B),
 * integrated exactly between jumps.
 *
 * Conventions shared by every entry point
 *  - No C++ types or exceptions cross this boundary; every call returns a
 *    dtb_status and never aborts.  dtb_last_error() describes the last
 *    failure of the calling thread.
 *  - Input arrays are borrowed only for the duration of the call that takes
 *    them and are deep-copied; the library never keeps or frees caller memory.
 *  - All GPU work is ordered on the hipStream_t given at creation (a
 *    void* here; NULL = a private blocking stream of the handle, which the
 *    legacy default stream orders against).  Parts of a step (the
 *    background draw, a remote block's landing) run on a private second
 *    stream of the handle, forked from that stream and joined back into it
 *    within the same step, so its order and its synchronization cover them.
 *    Reads into device memory are stream-ordered; reads into host memory
 *    synchronize the stream.
 *  - Neuron ids are 0..n-1.  Spike bitmaps hold neuron i at bit (i & 31) of
 *    32-bit word (i >> 5); a step's bitmap has dtb_bitmap_words(n) words.
 *  - Errors found while validating inputs return DTB_ERR_INVALID with a
 *    message naming the first offending index.  A failing HIP call returns
 *    DTB_ERR_HIP and makes the handle's error sticky: every later call on it
 *    returns DTB_ERR_STATE until it is destroyed.
 */
#ifndef DTB_H
#define DTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DTB_ABI_VERSION 14

typedef enum {
  DTB_OK = 0,
  DTB_ERR_INVALID = -1,     /* an argument or an input array failed validation */
  DTB_ERR_OOM = -2,         /* device or host allocation failed */
  DTB_ERR_HIP = -3,         /* a HIP runtime call failed (handle becomes sticky-failed) */
  DTB_ERR_STATE = -4,       /* call not valid in the handle's current state */
  DTB_ERR_NUMERIC = -5,     /* non-finite membrane potential or gate detected */
  DTB_ERR_UNSUPPORTED = -6  /* valid request outside what the library implements */
} dtb_status;

typedef enum { DTB_W_F32 = 0, DTB_W_BF16 = 1 } dtb_wtype;

typedef enum {
  DTB_V = 0,        /* membrane potential, mV (float32) */
  DTB_J_AMPA = 1,   /* gating variables j_u of Eq. (1) (float32) */
  DTB_J_NMDA = 2,
  DTB_J_GABAA = 3,
  DTB_J_GABAB = 4,
  DTB_REF = 5,      /* remaining refractory steps (returned as float32) */
  DTB_I_OU = 6      /* Ornstein-Uhlenbeck background current (float32; 0 while the
                       Poisson drive is selected) */
} dtb_field;

/* One row of the neuron property table (Sec. V-D): the configurable
 * parameters of Eq. (1).  Units: C in the same unit as the conductances
 * times ms, potentials in mV, tref in ms. */
typedef struct dtb_ptype {
  float C, gL, EL, Vth, Vreset, tref_ms, Iext;
  float g[4]; /* channel conductances g_u: AMPA, NMDA, GABAa, GABAb */
} dtb_ptype;

/* Network description.  The connection table of Sec. V-D is given as an
 * in-edge CSR (rows = post-synaptic neurons of this partition, a pull
 * layout); the order of a row's entries is the fixed order in which the
 * step sums that row. */
typedef struct dtb_desc {
  int64_t n;                 /* neurons, 1 .. 2^26-1 */
  int32_t n_regions;         /* populations whose spike counts are reported, >= 1 */
  int32_t max_delay;         /* D, largest synaptic delay in steps, 1 .. 31 */
  int32_t n_ptypes;          /* rows of the property table, 1 .. 65536 */
  int32_t member;            /* ensemble member id (enters the background counter) */
  int64_t nnz;               /* synapses, 0 .. 2^31-1; must equal row_ptr[n] */
  const int64_t* row_ptr;    /* [n+1], row_ptr[0] = 0, non-decreasing */
  const int32_t* col;        /* [nnz] presynaptic neuron, 0 .. n-1 */
  const float* w;            /* [nnz] weight (jump of the post gates), finite, >= 0 */
  const uint8_t* delay;      /* [nnz] delay d in steps, 1 .. max_delay; a spike of step e
                                is summed in step e+d-1 and first moves V in step e+d */
  const uint8_t* is_inh;     /* [n] 0 = excitatory (drives AMPA, NMDA), 1 = inhibitory
                                (drives GABAa, GABAb) */
  const int32_t* region;     /* [n] population id, 0 .. n_regions-1 */
  const uint16_t* ptype;     /* [n] row of the property table */
  const dtb_ptype* ptypes;   /* [n_ptypes]: C > 0, gL >= 0, Vreset < Vth, tref >= 0, g >= 0 */
  const float* V0;           /* [n] initial membrane potential */
  float E[4];                /* reversal potentials E_u (mV) */
  float tau_ms[4];           /* gate decay constants tau_u (ms), > 0 */
  float dt_ms;               /* time step (ms), > 0 */
  float bg_w;                /* weight of one background event (excitatory), >= 0 */
  double bg_lambda;          /* mean background Poisson count per neuron-step, 0 .. 400 */
  uint64_t seed;             /* background seed: Philox4x64-10 key (seed, 0) */
  int32_t wtype;             /* dtb_wtype: storage precision of w (accumulation is FP32) */
  int32_t record_steps;      /* steps of raster / counts history kept on device, >= 1 */
  int32_t gather_bundle_syn; /* launch shape of the gather: most synapses per workgroup
                                (4096 .. 2^20-1; 0 = library default, 2^20-1); a row longer
                                than a non-default value is rejected.  A tuning knob:
                                results do not depend on it */
  int32_t gather_unroll;     /* launch shape of the gather: lookup tiles per wavefront per
                                round, 1 .. 3 (0 = library default, 3).  A tuning knob:
                                results do not depend on it */
  int32_t gather_fuse;       /* where the row sums run: 1 = in the gather's workgroups, from
                                the bundle's hit bitmap still in LDS; 2 = in a separate
                                kernel over the hit buffer (always so while a remote in-edge
                                block is set); 0 = library default, 1.  A tuning knob: both
                                add the same terms in the same order */
  int32_t gather_events;     /* how the local block's delivery tests are found: 1 = the pull
                                sweep of each bundle's (delay, source)-sorted synapses over the
                                delayed spike bitmaps; 2 = spike-driven: the step's spikes of
                                the last D steps (their id lists) each deliver through their
                                out-synapses of the matching delay, bucketed per bundle with
                                the synapse's weight, which then sets the same hit bits; with
                                the row sums fused, a bundle whose bucket fits the LDS beside
                                its hit bitmap sums the carried weights (ordered by position),
                                a larger one loads them from the CSR (needs at most 4096
                                bundles, DTB_ERR_UNSUPPORTED otherwise; costs 16 B of device
                                memory per synapse: the event table and the buckets); 0 =
                                library default, 1.  A tuning knob: both find the same hits
                                and add the same weights in the same order, so the results
                                are identical */
} dtb_desc;

/* ------------------------------------------------------------ library */

int dtb_abi_version(void);

/* Text of the last failure on the calling thread; valid until the next call
 * on that thread.  Never NULL. */
const char* dtb_last_error(void);

/* Words in one step's spike bitmap: ceil(n / 32). */
int64_t dtb_bitmap_words(int64_t n);

/* --------------------------------------------------------- partition */

typedef struct dtb_net dtb_net;

/* Build a partition from the property and connection tables (Sec. V-D) and
 * initialise it (steps (2)-(3) of Sec. VI-A): V = V0, gates 0, no refractory
 * neuron, empty delay ring, t = 0.  Copies every input.  hip_stream: the
 * hipStream_t all work of this handle is enqueued on.
 * Errors: DTB_ERR_INVALID (validation), DTB_ERR_OOM, DTB_ERR_HIP. */
dtb_status dtb_create(const dtb_desc* desc, void* hip_stream, dtb_net** out);

/* Advance n_steps steps of the computing cycle of Sec. V-B / VI-C
 * (asynchronous on the handle's stream).  n_steps >= 0. */
dtb_status dtb_step(dtb_net* net, int32_t n_steps);

/* Return to the initial state of dtb_create (V = V0, gates 0, no refractory
 * neuron, empty delay ring, counters 0, t = 0), keeping the tables, the
 * background settings and any gains.  Re-running after a reset with the same
 * settings reproduces the first run exactly (the background draws are keyed
 * by step, neuron and member).  Drops pending teacher forcing. */
dtb_status dtb_reset(dtb_net* net);

/* Change the background drive standing in for J_inter (Sec. V-B): mean
 * Poisson count per neuron-step (0 .. 400) and event weight (finite, >= 0).
 * Takes effect from the next step; selects the Poisson drive (leaves the
 * Ornstein-Uhlenbeck one of dtb_set_background_ou). */
dtb_status dtb_set_background(dtb_net* net, double bg_lambda, float bg_w);

/* Select the paper's own background model (Sec. III-B: every neuron receives
 * an uncorrelated Ornstein-Uhlenbeck input current I_ou that keeps the
 * network active) instead of the Poisson count.  I_ou is added to I_ext in
 * the membrane equation (I = (I_ext + I_ou) + sum_u ...); after the step's
 * gates, I_ou <- mu + a (I_ou - mu) + sigma sqrt(1 - a^2) xi with
 * a = exp(-dt / tau_ms), the exact discretisation of the OU process, and
 * xi ~ N(0, 1) by Box-Muller from Philox4x64-10, key (seed, 0), counter
 * (t, i, member, 1): u1 = (hi32(word 0) + 1) / 2^32, u2 = hi32(word 1) / 2^32,
 * xi = sqrt(-2 ln u1) cos(2 pi u2).  Every neuron's I_ou is set to mu now
 * (also by dtb_reset while selected).  mu and sigma (>= 0) in the units of
 * I_ext, tau_ms > 0, all finite; the Poisson drive is off while selected.
 * Takes effect from the next step. */
dtb_status dtb_set_background_ou(dtb_net* net, float mu, float sigma, float tau_ms);

/* Teacher forcing (a test hook for the accuracy check of Sec. VII-B): the
 * next n_steps steps take their spikes from bits (host, [n_steps] bitmaps
 * of dtb_bitmap_words(n) words) instead of the threshold test.  A forced bit
 * decides the spike, the reset and the ring entry; an unforced neuron that
 * is not refractory keeps the integrated V even above threshold.  Queues
 * after any forcing still pending; at most record_steps pending steps. */
dtb_status dtb_force_spikes(dtb_net* net, const uint32_t* bits, int32_t n_steps);

/* J_inter (Sec. V-B, the equation splitting the input of neuron i into
 * J_intra over presynaptic neurons on the same GPU and J_inter over those on
 * other GPUs): give the partition a second in-edge block whose sources are
 * n_remote neurons of other partitions, and replay their spikes
 * (dtb_push_remote_spikes) in place of the exchange.  The block is a CSR
 * over the n local rows: row_ptr int64 [n+1] (row_ptr[0] = 0,
 * row_ptr[n] = nnz, non-decreasing), col int32 [nnz] in [0, n_remote),
 * w float32 [nnz] finite >= 0, delay uint8 [nnz] in [1, max_delay] ms,
 * remote_is_inh uint8 [n_remote] (nonzero = the remote source is
 * inhibitory, its weight goes to the GABA gates).  Host arrays, copied (the
 * caller keeps ownership).  Each row's input is then the local in-edges in
 * CSR order, then the remote ones in CSR order, then the background; a
 * delivered remote spike counts as a recurrent event.  Every step then
 * lands the step's remote bitmap in a remote ring on a second stream of the
 * library's (where an exchange would deliver it), concurrent with the
 * update, compaction and local delivery tests, and runs the remote block's
 * delivery tests after the local ones once that has arrived (the paper's
 * order: J_intra, then J_inter, then the j and I update).  Only on a single-member handle before its first step
 * (or right after dtb_reset); once per handle (DTB_ERR_STATE otherwise);
 * n_remote in [1, 2^26 - 1].  dtb_run is unavailable on such a handle. */
dtb_status dtb_set_remote_block(dtb_net* net, int64_t n_remote, int64_t nnz, const int64_t* row_ptr,
                                const int32_t* col, const float* w, const uint8_t* delay,
                                const uint8_t* remote_is_inh);

/* Queue the remote spikes of the next n_steps steps: bits (host,
 * [n_steps][dtb_bitmap_words(n_remote)] uint32; bit m of step q = remote
 * neuron m spiked at that step; bits past n_remote are ignored).  Each
 * dtb_step consumes one queued step and fails with DTB_ERR_STATE when none
 * is queued; at most record_steps pending steps; dtb_reset drops them.
 * Synchronizes the handle's stream. */
dtb_status dtb_push_remote_spikes(dtb_net* net, const uint32_t* bits, int32_t n_steps);

/* Spike bitmaps of steps [t0, t1) (the "spikes sequence" of Sec. V-B),
 * [t1-t0][dtb_bitmap_words(n)] uint32 into dst.  Requires
 * now - record_steps <= t0 <= t1 <= now (now = steps taken). */
dtb_status dtb_read_spikes(dtb_net* net, int64_t t0, int64_t t1, uint32_t* dst,
                           int dst_on_device);

/* Ascending ids of the neurons that spiked in step t (the compacted spike
 * list that a partition sends after collecting its spikes, Sec. V-B), at
 * most cap of them into ids (host, int32); *count receives the total (may
 * exceed cap).  t must lie in the recorded window (now - record_steps <= t
 * < now, DTB_ERR_INVALID otherwise).  The list of the most recent step is
 * the one the step built; an earlier step's list is rebuilt from that
 * step's spike bitmap by the same compaction kernel.  Synchronizes the
 * stream. */
dtb_status dtb_read_spike_ids(dtb_net* net, int64_t t, int32_t* ids, int64_t cap, int64_t* count);

/* Current value of one state field for all n neurons (float32 [n]). */
dtb_status dtb_read_state(dtb_net* net, int32_t field, float* dst, int dst_on_device);

/* Per-population spike counts of steps [t0, t1): int32 [t1-t0][n_regions],
 * host dst.  Same window rule as dtb_read_spikes. */
dtb_status dtb_read_region_counts(dtb_net* net, int64_t t0, int64_t t1, int32_t* dst);

/* Population firing rates over [t0, t1) (the population-wise rates that feed
 * the BOLD model of Sec. V-E): hz[r] = spikes of r / (n_r (t1-t0) dt / 1000);
 * float32 [n_regions], host dst.  Empty populations report 0. */
dtb_status dtb_read_region_rates(dtb_net* net, int64_t t0, int64_t t1, float* hz);

/* Per-step delivered recurrent events and background events of steps
 * [t0, t1): int64 [t1-t0] each (either pointer may be NULL), host dst. */
dtb_status dtb_read_step_events(dtb_net* net, int64_t t0, int64_t t1, int64_t* ev_rec,
                                int64_t* ev_bg);

/* Totals since creation: steps taken, spikes, delivered recurrent synaptic
 * events (a spike crossing one synapse), background events.  Any pointer may
 * be NULL.  Synchronizes the stream. */
dtb_status dtb_read_counters(dtb_net* net, int64_t* steps, int64_t* spikes, int64_t* ev_rec,
                             int64_t* ev_bg);

/* Kernel timing (a measurement aid for the statistics interface of
 * Sec. VI-C): while enabled, every kernel launch of dtb_step is bracketed by
 * a pair of hipEvents recorded on the handle's stream.  dtb_read_timing
 * synchronizes, returns the summed durations in ms and the number of timed
 * launches per kernel, in the order neuron update, compaction, gather
 * (delivery tests, with the row sums when they run there), sums (per-row
 * sums, background, gates), finalize, remote gather (the remote block's
 * delivery tests, timed on the second stream), events (the bucketing of
 * spike-driven deliveries), spike runs (the gathering of the step's table run
 * offsets for the bucketing), background (the step's Poisson background
 * counts) (double [9], int64 [9]; either may be NULL), and clears them. */
dtb_status dtb_set_timing(dtb_net* net, int enable);
dtb_status dtb_read_timing(dtb_net* net, double* ms, int64_t* launches);

/* ------------------------------------------------- batched ensemble */

/* Build one handle that advances n_members independent networks together
 * (the ensemble of brain samples that the paper's data assimilation runs on
 * disjoint node sets, Sec. V-E).  The members become one block-diagonal
 * partition: member m's neurons, populations and property-table rows follow
 * member m-1's.  Each member keeps its own background counter (t, i, member,
 * 0) under its own seed, i its own neuron index and member its desc's
 * `member` field, so a member advanced in a batch computes exactly what it
 * computes alone.  Members may differ in size, connectivity, populations,
 * property table, V0 and seed; E, tau_ms, dt_ms, bg_lambda, bg_w, wtype and
 * record_steps must be equal (DTB_ERR_UNSUPPORTED otherwise).  Inputs are
 * copied. */
dtb_status dtb_create_batch(const dtb_desc* members, int32_t n_members, void* hip_stream,
                            dtb_net** out);

/* Member table of a handle: *n_members, and for m = 0 .. min(cap, n_members)
 * the first neuron (int64) and first population (int32) of member m (entry
 * n_members holds the totals).  A plain partition is one member. */
dtb_status dtb_batch_info(dtb_net* net, int32_t* n_members, int64_t* neuron_offset,
                          int32_t* region_offset, int32_t cap);

/* Per-population gains on the four channel conductances (the population
 * hyper-parameters of the assimilation, Sec. V-E): g_u of every neuron of
 * population r is multiplied by gains[4 r + u].  float32 [n_regions][4],
 * finite and >= 0 (checked for host sources).  Default 1. */
dtb_status dtb_set_gains(dtb_net* net, const float* gains, int src_on_device);

/* Advance n_steps steps as one captured HIP graph (captured on the first
 * call with a given n_steps, replayed afterwards); same results as
 * dtb_step(n_steps).  Not available while teacher forcing is pending. */
dtb_status dtb_run(dtb_net* net, int32_t n_steps);

/* Launch-shape autotuner for the batched ensemble and the plain partition
 * (the block and tile shapes of the gather, chosen by timing them on the
 * real network): builds the network of `members` (n_members == 1: a plain
 * partition, else a batch as dtb_create_batch) once per candidate bundle
 * size (gather_bundle_syn; bundle_cands [n_cands], each in [4096, 2^20-1],
 * or n_cands = 0 for the library's list: the largest bundle and the sizes
 * whose bundle count fills whole rounds of the GPU's compute units), times
 * `steps` steps with hipEvents for each lookup-tiles-per-round value 1..3
 * (gather_unroll) and each placement of the row sums 1..2 (gather_fuse) of
 * the sweep, and for each placement with spike-driven delivery
 * (gather_events = 2, when the bundles fit it; with the library's list also
 * at up to three sizes of at most 2^19 - 1 synapses, whose buckets' weights
 * fit the LDS), and reports the fastest.  Every timing starts from the
 * same state - the first candidate's state after `burnin` steps, saved once
 * and loaded before each timing - so all candidates time the same steps
 * (the shapes change only the schedule, never a result).  The members'
 * own gather_bundle_syn / gather_unroll / gather_fuse / gather_events are
 * ignored.
 * cache_path (may be NULL): a JSON file of tuned shapes keyed by
 * "<gfx arch>|n=..,nnz=..,members=..,w=<f32|bf16>,D=..", one entry per line
 * ({"bundle_syn": b, "unroll": u, "fuse": f, "events": v, "ms_per_step": ms});
 * a key already present is returned without timing (from_cache = 1),
 * otherwise the winner is added (the file is rewritten through a temporary
 * file; DTB_ERR_INVALID if it cannot be written).  Work runs on hip_stream
 * (NULL: a private stream per candidate); the call blocks until it is done.
 * Errors: DTB_ERR_INVALID (arguments, see above), and whatever creating or
 * stepping the candidate networks returns. */
#define DTB_TUNE_MAX_BUNDLES 8
typedef struct dtb_tune_result {
  int32_t bundle_syn, unroll, fuse, events; /* the fastest shape (unroll 0 with events 2) */
  float ms_per_step;            /* its time per step (from the cache when from_cache) */
  int32_t from_cache;           /* 1: taken from cache_path without timing */
  int32_t n_tried;              /* shapes timed: per candidate 3 x 2 sweeps + 2 spike-driven,
                                   per extra spike-driven size 2 */
  int32_t tried_bundle[8 * DTB_TUNE_MAX_BUNDLES];
  int32_t tried_unroll[8 * DTB_TUNE_MAX_BUNDLES];
  int32_t tried_fuse[8 * DTB_TUNE_MAX_BUNDLES];
  int32_t tried_events[8 * DTB_TUNE_MAX_BUNDLES];
  float tried_ms[8 * DTB_TUNE_MAX_BUNDLES];
} dtb_tune_result;
dtb_status dtb_autotune(const dtb_desc* members, int32_t n_members, void* hip_stream, const char* cache_path,
                        const int32_t* bundle_cands, int32_t n_cands, int32_t burnin, int32_t steps,
                        dtb_tune_result* out);

/* Balloon-Windkessel BOLD signal per population after the last step (the
 * hemodynamic readout of Sec. V-E, integrated with the population rates of
 * every step): y float32 [n_regions] (host or device), and optionally the
 * state (s, f, v, q) float32 [n_regions][4] (host only).  Either may be NULL. */
dtb_status dtb_read_bold(dtb_net* net, float* y, float* sfvq, int dst_on_device);

/* ------------------------------------------------------- surrogate */

/* A small dense network that predicts population rates and BOLD from
 * population hyper-parameters, to screen assimilation proposals (Sec. V-E)
 * before they are simulated.  Layers: n_in -> n_hidden x hidden (exact-erf
 * GELU) -> n_out (linear).  Matrix products on MFMA with bfloat16 operands
 * and FP32 accumulation; parameters, Adam state and gradients FP32.
 * Parameters are one flat float32 vector, layer by layer: W [out][in]
 * row-major then b [out] (dtb_mlp_num_params entries).  Initial weights are
 * uniform(-1/sqrt(in), 1/sqrt(in)) from `seed`, biases 0. */
typedef struct dtb_mlp dtb_mlp;
dtb_status dtb_mlp_create(int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out, uint64_t seed,
                          void* hip_stream, dtb_mlp** out);
int64_t dtb_mlp_num_params(const dtb_mlp* mlp);
/* get = 1 copies the parameters out; get = 0 sets them (and resets Adam). */
dtb_status dtb_mlp_params(dtb_mlp* mlp, float* buf, int get, int on_device);
/* fp32 = 1: every matrix operand stays FP32 (MFMA 16x16x4 f32; same tiles,
 * epilogues and accumulation order) - the check of the kernels' logic
 * against an unrounded reference; fp32 = 0 (the default): bfloat16
 * operands.  Parameters and Adam state are unaffected. */
dtb_status dtb_mlp_set_operands(dtb_mlp* mlp, int fp32);
/* Y [batch][n_out] = f(X [batch][n_in]); on_device tells where X and Y live. */
dtb_status dtb_mlp_forward(dtb_mlp* mlp, const float* X, int32_t batch, float* Y, int on_device);
/* loss = mean over all entries of (f(X) - T)^2; grads [num_params] its
 * gradient (either output may be NULL).  Loss is written to host memory. */
dtb_status dtb_mlp_grad(dtb_mlp* mlp, const float* X, const float* T, int32_t batch, float* loss,
                        float* grads, int on_device);
/* One Adam step (Kingma & Ba; beta 0.9 / 0.999, eps 1e-8) on that loss. */
dtb_status dtb_mlp_train_step(dtb_mlp* mlp, const float* X, const float* T, int32_t batch, float lr,
                              float* loss, int on_device);
void dtb_mlp_destroy(dtb_mlp* mlp);

/* Indices of the k smallest of n scores (ties: smaller index first; NaN
 * last), 1 <= k <= n <= 4096, in ascending order of score. */
dtb_status dtb_topk(const float* score, int32_t n, int32_t k, int32_t* idx, void* hip_stream,
                    int on_device);

/* dtb_topk for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same selection as dtb_topk with on_device = 0: score [n] and idx [k] are
 * host arrays, 1 <= k <= n <= 4096 (DTB_ERR_INVALID otherwise, naming the
 * limit).  The scores and indices are staged through a static device array
 * of 32 KB (4096 scores + 4096 indices), one per GPU the library runs on,
 * held until the process ends; its address is looked up once per device.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); it copies the scores in, sorts, copies the indices out and
 * synchronizes hip_stream (NULL: the current device's null stream).  All
 * calls on one GPU share that array, so calls that overlap on one GPU
 * race: serialize them (one stream, or wait for the previous call). */
dtb_status dtb_topk_noalloc(const float* score, int32_t n, int32_t k, int32_t* idx, void* hip_stream);

/* ------------------------------------------------- assimilation */

/* One analysis step of an ensemble Kalman filter over hyper-parameters: the
 * iteration of Sec. V-E that adapts the per-population hyper-parameters of
 * an ensemble of simulated brain models by tracking BOLD signals (the
 * paper defers the filter itself to its companion work; this stochastic
 * EnKF with perturbed observations stands in for it).  Device arrays:
 * X float32 [n_members][n_params] (in/out; e.g. the gains of a batched
 * handle, [member][population][channel]), Y float32 [n_members][n_obs] (each
 * member's predicted observation, e.g. dtb_read_bold of the batch),
 * y_obs float32 [n_obs].  Host array r_var float32 [n_obs]: observation-error
 * variances, finite and > 0.  With anomalies A = inflation (X - mean X) and
 * B = Y - mean Y, C_xy = A^T B / (M-1), C_yy = B^T B / (M-1):
 *   X_m <- mean X + A_m + C_xy (C_yy + R)^-1 (y_obs + sqrt(r) xi_m - Y_m),
 * clamped to [lo, hi], xi_m,o ~ N(0, 1) by Box-Muller on Philox4x64-10, key
 * (seed, 0), counter (iter, m, o, 2) (u1 = (hi32(word 0) + 1) / 2^32,
 * u2 = hi32(word 1) / 2^32).  FP64 inside, one workgroup, asynchronous on
 * hip_stream.  A parameter with no spread across members is left exactly
 * as it is; parameters equal in every member stay equal.  Sizes:
 * n_members >= 2, n_params >= 1, 1 <= n_obs <= 64 and
 * 8 (P + O + O^2 + P O + M O) <= 160 KB (DTB_ERR_UNSUPPORTED otherwise);
 * inflation >= 1 and lo <= hi, all finite (DTB_ERR_INVALID otherwise). */
dtb_status dtb_enkf_analysis(int32_t n_members, int32_t n_params, int32_t n_obs, float* X, const float* Y,
                             const float* y_obs, const float* r_var, float inflation, uint64_t seed, int64_t iter,
                             float lo, float hi, void* hip_stream);

/* ------------------------------------------------- partitioning */

/* Neuron-to-GPU partition minimising the heaviest inter-GPU traffic
 * (Sec. V-C, Eq. (2): F(P) = max_j sum_{i != j} D_ij) subject to a disjoint
 * cover and a per-GPU capacity on the summed vertex sizes (the constraint
 * after Eq. (2)).  Host only; needs no GPU.  Vertices are groups of neurons
 * (a population or a piece of one): size double [n_vert] (>= 0, e.g.
 * bytes), neurons double [n_vert] (> 0), spikes double [n_vert] (spikes per
 * step, >= 0); synapses between vertices as a CSR by source: e_ptr int64
 * [n_vert+1], e_dst int32 [ne], e_syn double [ne] (synapse counts, >= 0).
 * Traffic: a spike of a neuron of u on GPU i goes to GPU j != i once if the
 * neuron has a target there, probability 1 - exp(-c_uj / n_u) with c_uj
 * the synapses from u onto j's vertices, so
 * D_ij = bytes_per_spike sum_{u on i} s_u (1 - exp(-c_uj / n_u)).
 * Start: init int32 [n_vert] if given, else the greedy fill (one GPU at a
 * time, the unassigned vertex most connected to it, up to an even share of
 * the total size); then up to refine_rounds single-vertex moves into or out
 * of the most loaded GPU, or swaps with its strongest senders, each lowering
 * F (refine_rounds = 0 evaluates the start).  Outputs: part int32 [n_vert],
 * *F_out, D_out double [n_gpu][n_gpu] (diagonal 0; either may be NULL).
 * Cost: the greedy fill scans the unassigned vertices for every placement
 * (O(n_vert^2)) and each move re-evaluates F (O(n_gpu^2)); meant for up to
 * ~10^4 vertices (1,319 vertices on 64 GPUs take 0.3 s).  Errors: DTB_ERR_INVALID
 * (bad arrays, an init beyond the capacity), DTB_ERR_UNSUPPORTED (a vertex
 * or the total beyond the capacity, n_vert n_gpu > 2^28). */
dtb_status dtb_partition(int64_t n_vert, const double* size, const double* neurons, const double* spikes,
                         const int64_t* e_ptr, const int32_t* e_dst, const double* e_syn, int32_t n_gpu,
                         double capacity, double bytes_per_spike, const int32_t* init, int32_t refine_rounds,
                         int32_t* part, double* F_out, double* D_out);

/* ------------------------------------------------- checkpoint / resume */

/* Save the handle's dynamic state into host memory so that a run can be
 * resumed later (a checkpoint of the simulation; the paper keeps the state
 * variables in GPU memory for the whole run, Sec. V-B): V, gates, refractory
 * counters, OU currents, gains, the spike-bitmap ring (and the remote ring),
 * population counts, event counters and totals, the last spike-id list, the
 * step counter, the BOLD state, and the background settings.  The network
 * tables are not saved: a state is loaded into a handle created from the
 * same description (and given the same remote block).  host_buf NULL asks
 * for the size only (*used); otherwise cap must be at least that size
 * (DTB_ERR_INVALID, *used set).  Not while teacher forcing or pushed
 * remote spikes are pending (DTB_ERR_STATE).  Synchronizes the stream. */
dtb_status dtb_save(dtb_net* net, void* host_buf, size_t cap, size_t* used);

/* Restore a state written by dtb_save (host buffer of len bytes) into a
 * handle of the same shape (DTB_ERR_INVALID otherwise: other sizes, record
 * steps, weight type, member count or remote block, a truncated or foreign
 * buffer).  The next step continues the saved run exactly; pending teacher
 * forcing and remote spikes are dropped.  Synchronizes the stream. */
dtb_status dtb_load(dtb_net* net, const void* host_buf, size_t len);

/* Wait for the handle's stream; report asynchronous failures (DTB_ERR_NUMERIC
 * when a non-finite V or gate was produced since the last check). */
dtb_status dtb_sync(dtb_net* net);

/* Release everything the handle owns.  NULL-safe. */
void dtb_destroy(dtb_net* net);

#ifdef __cplusplus
}
#endif
#endif /* DTB_H */
