/*
 * dtb_oracle.c - plain FP64 CPU reference of one partition step of the
 * conductance-based LIF network.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the simulator's product path links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the GPU library.
 *
 * What it computes (paper: Sec. III-B Eq. (1) for the neuron, Sec. V-B and
 * the time anchors of Sec. VI-C for the order inside a step, Sec. VI-A for
 * forward Euler with a 1 ms step):
 *
 *   state before step t: V^t, gates j_u^t (u = AMPA, NMDA, GABAa, GABAb),
 *   refractory counter ref^t, and the spikes s^{t'} of all t' < t.
 *
 *   1. if ref^t > 0:  V^{t+1} = V_reset, ref^{t+1} = ref^t - 1, s^t = 0
 *      else:          Vt = V^t + dt/C [ -gL (V^t - EL)
 *                                       + sum_u g_u gain_u j_u^t (E_u - V^t) + Iext ]
 *                     s^t = [Vt >= Vth]; spike -> V^{t+1} = V_reset,
 *                     ref^{t+1} = n_ref = round(T_ref / dt); else V^{t+1} = Vt.
 *   2. the spikes s^t enter the delay ring buffer.
 *   3. pull over the in-edges k of row i, in CSR order:
 *        dE_i = sum_{k: m_k exc} w_k s^{t-d_k+1}_{m_k} + w_bg c_i^t
 *        dI_i = sum_{k: m_k inh} w_k s^{t-d_k+1}_{m_k}
 *      (a spike sent at step e through delay d is gathered in step e+d-1 and
 *      first moves V in step e+d; d = 1 is the paper's one-step exchange).
 *      c_i^t is the background Poisson count standing in for the spikes of
 *      other partitions (J_inter of Sec. V-B).
 *   4. gates: jump and exponential decay (Sec. III-B), exact between jumps:
 *        j_u^{t+1} = exp(-dt/tau_u) j_u^t + dE_i (AMPA, NMDA) or dI_i (GABAs).
 *   5. per-region spike counts of step t.
 *
 * Background draws: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), key
 * (seed, 0), one block per eight neurons: counter (t, floor(i / 8), member,
 * 0); its four output words give eight 32-bit values (word 0's high half,
 * word 0's low half, word 1's high half, ...), and neuron i takes value
 * i mod 8, u, which is turned into a Poisson(lambda) count by inversion against the table
 * T_k = floor(F(k) 2^32) (F the Poisson CDF, entries kept while below
 * 2^32 - 1): c = #{k : u >= T_k}.
 *
 * Alternative background (the paper's own, Sec. III-B): an uncorrelated
 * Ornstein-Uhlenbeck current I_ou per neuron, added to Iext in step 1
 * (I = (Iext + I_ou) + sum_u ...), advanced after step 4 by the exact
 * discretisation I_ou <- mu + a (I_ou - mu) + sigma sqrt(1 - a^2) xi,
 * a = exp(-dt / tau); xi by Box-Muller from Philox counter (t, i, member, 1):
 * u1 = (hi32(word 0) + 1) 2^-32, u2 = hi32(word 1) 2^-32,
 * xi = sqrt(-2 ln u1) cos(2 pi u2).  The Poisson drive is off meanwhile.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ Philox */

static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, x0, &hi0, &lo0);
    mulhilo64(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * Poisson(lambda) inversion table T_k = floor(F(k) 2^32), k = 0, 1, ...,
 * kept while T_k < 2^32 - 1 (the first saturated entry ends the table, so a
 * draw u counts c = #{k < K : u >= T_k}; lambda = 0 gives K = 0, c = 0).
 * F(k) is accumulated from p_0 = exp(-lambda), p_k = p_{k-1} lambda / k.
 * Returns K, or -1 if cap entries are not enough.
 */
int ora_poisson_table(double lambda, uint32_t* T, int cap) {
  if (!(lambda >= 0.0) || !(lambda < 700.0) || cap < 1) return -1;
  const double two32 = 4294967296.0;
  double p = exp(-lambda), F = p;
  for (int k = 0; k < cap; k++) {
    double x = floor(F * two32);
    if (x >= 4294967295.0) return k;
    T[k] = (uint32_t)x;
    p = p * lambda / (double)(k + 1);
    F = F + p;
  }
  return -1;
}

static inline int poisson_count(uint32_t u, const uint32_t* T, int K) {
  int c = 0;
  while (c < K && u >= T[c]) c++;
  return c;
}

uint32_t ora_bg_uniform(uint64_t seed, int64_t t, int64_t i, int64_t member) {
  uint64_t ctr[4] = {(uint64_t)t, (uint64_t)(i >> 3), (uint64_t)member, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  ora_philox4x64_10(ctr, key, out);
  const int j = (int)(i & 7);
  const uint64_t w = out[j >> 1];
  return (j & 1) ? (uint32_t)w : (uint32_t)(w >> 32);
}

/* standard normal draw of the OU background: Box-Muller on Philox stream 1 */
double ora_ou_normal(uint64_t seed, int64_t t, int64_t i, int64_t member) {
  uint64_t ctr[4] = {(uint64_t)t, (uint64_t)i, (uint64_t)member, 1};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  ora_philox4x64_10(ctr, key, out);
  const double u1 = ((double)(out[0] >> 32) + 1.0) * 0x1p-32;
  const double u2 = (double)(out[1] >> 32) * 0x1p-32;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2);
}

/* standard normals out[i][j] = Box-Muller on Philox counter (c0, i, j, c3),
   i < n1, j < n2 (the perturbed observations of the EnKF use c3 = 2) */
void ora_normals(uint64_t seed, int64_t c0, int64_t n1, int64_t n2, int64_t c3, double* out) {
  uint64_t key[2] = {seed, 0};
  for (int64_t i = 0; i < n1; i++)
    for (int64_t j = 0; j < n2; j++) {
      uint64_t ctr[4] = {(uint64_t)c0, (uint64_t)i, (uint64_t)j, (uint64_t)c3};
      uint64_t w[4];
      ora_philox4x64_10(ctr, key, w);
      const double u1 = ((double)(w[0] >> 32) + 1.0) * 0x1p-32;
      const double u2 = (double)(w[1] >> 32) * 0x1p-32;
      out[i * n2 + j] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2);
    }
}

/* ------------------------------------------------------------- network */

typedef struct {
  int64_t n;
  int32_t n_regions, max_delay, n_ptypes, member;
  const int64_t* row_ptr;
  const int32_t* col;
  const float* w;
  const uint8_t* delay;
  const uint8_t* is_inh;
  const int32_t* region;
  const uint16_t* ptype;
  const float* ptypes; /* [n_ptypes][11]: C gL EL Vth Vreset tref Iext gA gN gGa gGb */
  const float* V0;
  double E[4], tau_ms[4], dt_ms;
  double bg_lambda, bg_w;
  uint64_t seed;
  const double* gain; /* [n_regions][4] or NULL (all ones) */
} ora_input;

typedef struct {
  ora_input in;
  double a[4];
  /* per parameter type */
  double *C, *gL, *EL, *Vth, *Vreset, *Iext, *g; /* g: [n_ptypes][4] */
  int32_t* nref;
  uint32_t T[512];
  int K;
  /* state */
  int64_t t;
  double* V;
  double* j; /* [4][n] */
  int32_t* ref;
  uint8_t* ring; /* [max_delay][n] */
  double* gain;  /* [n_regions][4] */
  /* Ornstein-Uhlenbeck background (ou_on) */
  int ou_on;
  double ou_mu, ou_a, ou_s;
  double* ou; /* [n] */
  /* remote in-edge block (J_inter of Sec. V-B): sources are n_remote neurons
     of other partitions whose spikes are given step by step */
  int64_t n_remote;
  int64_t* r_row_ptr; /* [n+1] */
  int32_t* r_col;
  float* r_w;
  uint8_t* r_delay;
  uint8_t* r_inh;     /* [n_remote] */
  uint8_t* r_ring;    /* [max_delay][n_remote] */
  int64_t r_given;    /* step whose remote spikes are in the ring (-1: none) */
} ora_net;

void ora_destroy(ora_net* h) {
  if (!h) return;
  free(h->C); free(h->gL); free(h->EL); free(h->Vth); free(h->Vreset); free(h->Iext);
  free(h->g); free(h->nref); free(h->V); free(h->j); free(h->ref); free(h->ring); free(h->gain);
  free(h->ou);
  free(h->r_row_ptr); free(h->r_col); free(h->r_w); free(h->r_delay); free(h->r_inh); free(h->r_ring);
  free(h);
}

/* returns NULL on invalid input or allocation failure */
ora_net* ora_create(const ora_input* in) {
  if (!in || in->n <= 0 || in->n_regions <= 0 || in->max_delay < 1 || in->n_ptypes < 1 ||
      !(in->dt_ms > 0.0))
    return NULL;
  ora_net* h = (ora_net*)calloc(1, sizeof(ora_net));
  if (!h) return NULL;
  h->in = *in;
  const int64_t n = in->n;
  const int P = in->n_ptypes;
  for (int u = 0; u < 4; u++) h->a[u] = exp(-in->dt_ms / in->tau_ms[u]);
  h->C = malloc(sizeof(double) * P); h->gL = malloc(sizeof(double) * P);
  h->EL = malloc(sizeof(double) * P); h->Vth = malloc(sizeof(double) * P);
  h->Vreset = malloc(sizeof(double) * P); h->Iext = malloc(sizeof(double) * P);
  h->g = malloc(sizeof(double) * P * 4); h->nref = malloc(sizeof(int32_t) * P);
  h->V = malloc(sizeof(double) * n); h->j = calloc((size_t)n * 4, sizeof(double));
  h->ref = calloc((size_t)n, sizeof(int32_t));
  h->ring = calloc((size_t)n * in->max_delay, 1);
  h->gain = malloc(sizeof(double) * in->n_regions * 4);
  if (!h->C || !h->gL || !h->EL || !h->Vth || !h->Vreset || !h->Iext || !h->g || !h->nref ||
      !h->V || !h->j || !h->ref || !h->ring || !h->gain) {
    ora_destroy(h);
    return NULL;
  }
  for (int p = 0; p < P; p++) {
    const float* r = in->ptypes + 11 * p;
    h->C[p] = r[0]; h->gL[p] = r[1]; h->EL[p] = r[2]; h->Vth[p] = r[3]; h->Vreset[p] = r[4];
    h->nref[p] = (int32_t)lround((double)r[5] / in->dt_ms);
    h->Iext[p] = r[6];
    for (int u = 0; u < 4; u++) h->g[4 * p + u] = r[7 + u];
  }
  for (int r = 0; r < in->n_regions; r++)
    for (int u = 0; u < 4; u++) h->gain[4 * r + u] = in->gain ? in->gain[4 * r + u] : 1.0;
  h->K = ora_poisson_table(in->bg_lambda, h->T, 512);
  if (h->K < 0) { ora_destroy(h); return NULL; }
  for (int64_t i = 0; i < n; i++) h->V[i] = in->V0[i];
  h->t = 0;
  return h;
}

int64_t ora_time(const ora_net* h) { return h->t; }

/* select the OU background (every I_ou set to mu); returns -1 on bad input */
int ora_set_ou(ora_net* h, double mu, double sigma, double tau_ms) {
  if (!(sigma >= 0.0) || !(tau_ms > 0.0) || !isfinite(mu) || !isfinite(sigma) || !isfinite(tau_ms)) return -1;
  if (!h->ou) {
    h->ou = malloc(sizeof(double) * h->in.n);
    if (!h->ou) return -1;
  }
  h->ou_on = 1;
  h->ou_mu = mu;
  h->ou_a = exp(-h->in.dt_ms / tau_ms);
  h->ou_s = sigma * sqrt(1.0 - h->ou_a * h->ou_a);
  h->K = 0; /* no Poisson drive */
  for (int64_t i = 0; i < h->in.n; i++) h->ou[i] = mu;
  return 0;
}

/* Add the remote in-edge block: CSR over the n local rows (row_ptr [n+1],
   col [nnz] in [0, n_remote), w, delay in [1, max_delay]) and the remote
   sources' inhibitory flags.  The arrays are copied.  From then on every step
   needs ora_give_remote first.  Returns -1 on bad input or a second call. */
int ora_set_remote(ora_net* h, int64_t n_remote, const int64_t* row_ptr, const int32_t* col,
                   const float* w, const uint8_t* delay, const uint8_t* inh) {
  const int64_t n = h->in.n;
  if (h->r_row_ptr || n_remote < 1 || row_ptr[0] != 0) return -1;
  const int64_t nnz = row_ptr[n];
  for (int64_t i = 0; i < n; i++)
    if (row_ptr[i + 1] < row_ptr[i]) return -1;
  for (int64_t k = 0; k < nnz; k++)
    if (col[k] < 0 || col[k] >= n_remote || delay[k] < 1 || delay[k] > h->in.max_delay) return -1;
  h->r_row_ptr = malloc(sizeof(int64_t) * (n + 1));
  h->r_col = malloc(sizeof(int32_t) * (nnz + 1));
  h->r_w = malloc(sizeof(float) * (nnz + 1));
  h->r_delay = malloc(nnz + 1);
  h->r_inh = malloc(n_remote);
  h->r_ring = calloc((size_t)n_remote * h->in.max_delay, 1);
  if (!h->r_row_ptr || !h->r_col || !h->r_w || !h->r_delay || !h->r_inh || !h->r_ring) return -1;
  memcpy(h->r_row_ptr, row_ptr, sizeof(int64_t) * (n + 1));
  memcpy(h->r_col, col, sizeof(int32_t) * nnz);
  memcpy(h->r_w, w, sizeof(float) * nnz);
  memcpy(h->r_delay, delay, nnz);
  memcpy(h->r_inh, inh, n_remote);
  h->n_remote = n_remote;
  h->r_given = -1;
  return 0;
}

/* The spikes [n_remote] (0/1) the remote sources emit at the coming step. */
int ora_give_remote(ora_net* h, const uint8_t* spikes) {
  if (!h->r_row_ptr) return -1;
  uint8_t* slot = h->r_ring + (size_t)(h->t % h->in.max_delay) * h->n_remote;
  for (int64_t m = 0; m < h->n_remote; m++) slot[m] = spikes[m] ? 1 : 0;
  h->r_given = h->t;
  return 0;
}

int ora_set_gain(ora_net* h, const double* gain) {
  for (int r = 0; r < h->in.n_regions; r++)
    for (int u = 0; u < 4; u++) h->gain[4 * r + u] = gain[4 * r + u];
  return 0;
}

/*
 * One step.  forced: optional [n] spike raster of this step that replaces the
 * threshold test (teacher forcing: the forced bit decides spike, reset and
 * ring entry).  rows/n_rows: optional subset of neurons whose state is
 * advanced (requires forced, since the spikes of the others are unknown).
 * Outputs (each optional): spikes [n], margin [n] = Vt - Vth for
 * non-refractory neurons (signed: >= 0 is the threshold test's own spike,
 * also when forced; NAN for refractory ones), region_counts [n_regions],
 * ev_rec / ev_bg (delivered recurrent / background events of the rows).
 */
int ora_step(ora_net* h, const uint8_t* forced, const int64_t* rows, int64_t n_rows,
             uint8_t* spikes, double* margin, int64_t* region_counts, int64_t* ev_rec,
             int64_t* ev_bg) {
  const ora_input* in = &h->in;
  const int64_t n = in->n;
  const int D = in->max_delay;
  const int64_t t = h->t;
  if (rows && !forced) return -1;
  if (h->r_row_ptr && h->r_given != t) return -2; /* remote spikes of step t not given */
  const int64_t nr = rows ? n_rows : n;
  uint8_t* slot_now = h->ring + (size_t)(t % D) * n;

  /* 1. neuron update (all neurons, or the subset) */
#pragma omp parallel for schedule(static) if (nr > 16384)
  for (int64_t q = 0; q < nr; q++) {
    const int64_t i = rows ? rows[q] : q;
    const int p = in->ptype[i];
    const int reg = in->region[i];
    const double V = h->V[i];
    const int r = h->ref[i];
    double Vt = NAN;
    if (r <= 0) {
      double I = h->Iext[p];
      if (h->ou_on) I += h->ou[i];
      for (int u = 0; u < 4; u++)
        I += h->g[4 * p + u] * h->gain[4 * reg + u] * h->j[(size_t)u * n + i] * (in->E[u] - V);
      Vt = V + in->dt_ms / h->C[p] * (-h->gL[p] * (V - h->EL[p]) + I);
    }
    int s;
    if (forced) s = forced[i] ? 1 : 0;
    else s = (r <= 0 && Vt >= h->Vth[p]) ? 1 : 0;
    if (s) { h->V[i] = h->Vreset[p]; h->ref[i] = h->nref[p]; }
    else if (r > 0) { h->V[i] = h->Vreset[p]; h->ref[i] = r - 1; }
    else { h->V[i] = Vt; h->ref[i] = 0; }
    if (margin) margin[i] = (r <= 0) ? Vt - h->Vth[p] : NAN;
    if (!forced) slot_now[i] = (uint8_t)s;
  }
  /* 2. spikes of this step into the ring (teacher forcing: the given raster) */
  if (forced) {
#pragma omp parallel for schedule(static) if (n > 16384)
    for (int64_t i = 0; i < n; i++) slot_now[i] = forced[i] ? 1 : 0;
  }
  if (spikes) memcpy(spikes, slot_now, (size_t)n);

  /* 3.-4. pull gather over in-edges in CSR order, background, gate update */
  int64_t er = 0, eb = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : er, eb) if (nr > 1024)
  for (int64_t q = 0; q < nr; q++) {
    const int64_t i = rows ? rows[q] : q;
    double dE = 0.0, dI = 0.0;
    for (int64_t k = in->row_ptr[i]; k < in->row_ptr[i + 1]; k++) {
      const int32_t m = in->col[k];
      const int64_t te = t - (int64_t)in->delay[k] + 1;
      const int64_t sl = ((te % D) + D) % D;
      if (h->ring[(size_t)sl * n + m]) {
        if (in->is_inh[m]) dI += (double)in->w[k];
        else dE += (double)in->w[k];
        er++;
      }
    }
    /* J_inter: the remote in-edges, after the local ones, in CSR order */
    if (h->r_row_ptr) {
      for (int64_t k = h->r_row_ptr[i]; k < h->r_row_ptr[i + 1]; k++) {
        const int32_t m = h->r_col[k];
        const int64_t te = t - (int64_t)h->r_delay[k] + 1;
        const int64_t sl = ((te % D) + D) % D;
        if (h->r_ring[(size_t)sl * h->n_remote + m]) {
          if (h->r_inh[m]) dI += (double)h->r_w[k];
          else dE += (double)h->r_w[k];
          er++;
        }
      }
    }
    const int c = poisson_count(ora_bg_uniform(in->seed, t, i, in->member), h->T, h->K);
    dE += in->bg_w * (double)c;
    eb += c;
    h->j[0 * (size_t)n + i] = h->a[0] * h->j[0 * (size_t)n + i] + dE;
    h->j[1 * (size_t)n + i] = h->a[1] * h->j[1 * (size_t)n + i] + dE;
    h->j[2 * (size_t)n + i] = h->a[2] * h->j[2 * (size_t)n + i] + dI;
    h->j[3 * (size_t)n + i] = h->a[3] * h->j[3 * (size_t)n + i] + dI;
    if (h->ou_on)
      h->ou[i] = h->ou_mu + h->ou_a * (h->ou[i] - h->ou_mu) +
                 h->ou_s * ora_ou_normal(in->seed, t, i, in->member);
  }
  if (ev_rec) *ev_rec = er;
  if (ev_bg) *ev_bg = eb;

  /* 5. region spike counts of step t */
  if (region_counts) {
    memset(region_counts, 0, sizeof(int64_t) * in->n_regions);
    for (int64_t i = 0; i < n; i++) region_counts[in->region[i]] += slot_now[i];
  }
  h->t = t + 1;
  return 0;
}

/* field: 0 = V, 1..4 = gates AMPA NMDA GABAa GABAb, 5 = refractory counter,
   6 = OU current (0 while the Poisson drive is selected) */
int ora_get(const ora_net* h, int field, double* out) {
  const int64_t n = h->in.n;
  if (field == 6) {
    for (int64_t i = 0; i < n; i++) out[i] = h->ou_on ? h->ou[i] : 0.0;
    return 0;
  }
  if (field == 0) memcpy(out, h->V, sizeof(double) * n);
  else if (field >= 1 && field <= 4) memcpy(out, h->j + (size_t)(field - 1) * n, sizeof(double) * n);
  else if (field == 5) for (int64_t i = 0; i < n; i++) out[i] = h->ref[i];
  else return -1;
  return 0;
}

int ora_set(ora_net* h, int field, const double* src) {
  const int64_t n = h->in.n;
  if (field == 0) memcpy(h->V, src, sizeof(double) * n);
  else if (field >= 1 && field <= 4) memcpy(h->j + (size_t)(field - 1) * n, src, sizeof(double) * n);
  else if (field == 5) for (int64_t i = 0; i < n; i++) h->ref[i] = (int32_t)src[i];
  else return -1;
  return 0;
}

int ora_poisson_K(const ora_net* h) { return h->K; }
double ora_decay(const ora_net* h, int u) { return h->a[u]; }

int ora_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_set_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
#else
  (void)nt;
#endif
}
