// dtb_partition.cpp - the neuron-to-GPU partitioner of Sec. V-C (host only).
//
// Objective (Eq. (2)): F(P) = max_j sum_{i != j} D_ij, the heaviest traffic
// any GPU receives, subject to a disjoint cover of the vertices and a
// per-GPU capacity on the summed vertex sizes.  Vertices are groups of
// neurons (a population or a piece of one); D_ij is the spike traffic from
// GPU i to GPU j per step: a spike of a neuron of vertex u on GPU i is sent
// to GPU j once if the neuron has at least one target there.  With c_uj the
// synapses from u to vertices on j and n_u the neurons of u, a neuron of u
// has targets on j with probability 1 - exp(-c_uj / n_u) (its out-synapses
// fall on targets independently), so
//     D_ij = b * sum_{u on i} s_u (1 - exp(-c_uj / n_u)),
// with s_u the spikes of u per step and b the bytes per spike.
//
// Method: the paper's greedy assignment (fill one GPU at a time with the
// unassigned vertex most strongly connected to it, up to an even share of
// the total size), then a local search on the GPU receiving the most
// traffic - single vertices moved into or out of it, or swapped with a
// strong sender - while that lowers F.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dtb.h"

namespace dtb {
void set_error(const std::string& msg);
}

namespace {

struct Part {
  int64_t n;
  int32_t N;
  const double *size, *nn, *spk;
  double b;
  std::vector<int64_t> optr, iptr;  // out- and in-edges (CSR)
  std::vector<int32_t> odst, isrc;
  std::vector<double> osyn, isyn;
  std::vector<int32_t> part;
  std::vector<double> c;     // [n][N] synapses from u to GPU j
  std::vector<double> D;     // [N][N] traffic i -> j (diagonal unused)
  std::vector<double> load;  // [N] summed sizes

  double contrib(int64_t u, int32_t j) const {
    return b * spk[u] * (1.0 - std::exp(-c[size_t(u) * N + j] / nn[u]));
  }
  void recompute() {
    std::fill(c.begin(), c.end(), 0.0);
    std::fill(D.begin(), D.end(), 0.0);
    std::fill(load.begin(), load.end(), 0.0);
    for (int64_t u = 0; u < n; ++u) {
      load[part[u]] += size[u];
      for (int64_t e = optr[u]; e < optr[u + 1]; ++e) c[size_t(u) * N + part[odst[e]]] += osyn[e];
    }
    for (int64_t u = 0; u < n; ++u)
      for (int32_t j = 0; j < N; ++j)
        if (j != part[u]) D[size_t(part[u]) * N + j] += contrib(u, j);
  }
  double colsum(int32_t j) const {
    double s = 0.0;
    for (int32_t i = 0; i < N; ++i)
      if (i != j) s += D[size_t(i) * N + j];
    return s;
  }
  double F(int32_t* arg = nullptr) const {
    double f = -1.0;
    for (int32_t j = 0; j < N; ++j) {
      const double s = colsum(j);
      if (s > f) {
        f = s;
        if (arg) *arg = j;
      }
    }
    return std::max(f, 0.0);
  }
  double total() const {
    double s = 0.0;
    for (double x : D) s += x;
    return s;
  }
  // move vertex u to GPU g, keeping c, D and load current
  void move(int64_t u, int32_t g) {
    const int32_t a = part[u];
    if (a == g) return;
    for (int32_t j = 0; j < N; ++j)
      if (j != a) D[size_t(a) * N + j] -= contrib(u, j);
    for (int64_t e = iptr[u]; e < iptr[u + 1]; ++e) {
      const int32_t w = isrc[e];
      if (w == u) continue;
      const int32_t pw = part[w];
      double* cw = &c[size_t(w) * N];
      if (a != pw) D[size_t(pw) * N + a] -= contrib(w, a);
      if (g != pw) D[size_t(pw) * N + g] -= contrib(w, g);
      cw[a] -= isyn[e];
      cw[g] += isyn[e];
      if (a != pw) D[size_t(pw) * N + a] += contrib(w, a);
      if (g != pw) D[size_t(pw) * N + g] += contrib(w, g);
    }
    for (int64_t e = optr[u]; e < optr[u + 1]; ++e)
      if (odst[e] == u) {
        c[size_t(u) * N + a] -= osyn[e];
        c[size_t(u) * N + g] += osyn[e];
      }
    part[u] = g;
    load[a] -= size[u];
    load[g] += size[u];
    for (int32_t j = 0; j < N; ++j)
      if (j != g) D[size_t(g) * N + j] += contrib(u, j);
  }
};

}  // namespace

extern "C" dtb_status dtb_partition(int64_t n_vert, const double* size, const double* neurons,
                                    const double* spikes, const int64_t* e_ptr, const int32_t* e_dst,
                                    const double* e_syn, int32_t n_gpu, double capacity, double bytes_per_spike,
                                    const int32_t* init, int32_t refine_rounds, int32_t* part, double* F_out,
                                    double* D_out) {
  auto bad = [](dtb_status st, const std::string& m) {
    dtb::set_error(m);
    return st;
  };
  if (n_vert < 1 || n_gpu < 1 || !size || !neurons || !spikes || !e_ptr || !part)
    return bad(DTB_ERR_INVALID, "partition: n_vert, n_gpu >= 1 and non-null arrays required");
  if ((int64_t(n_vert) * n_gpu) > (int64_t(1) << 28))
    return bad(DTB_ERR_UNSUPPORTED, "partition: n_vert * n_gpu above 2^28");
  if (!(capacity > 0.0) || !std::isfinite(capacity) || !(bytes_per_spike > 0.0) || refine_rounds < 0)
    return bad(DTB_ERR_INVALID, "partition: capacity, bytes_per_spike > 0 and refine_rounds >= 0 required");
  if (e_ptr[0] != 0) return bad(DTB_ERR_INVALID, "partition: e_ptr[0] must be 0");
  const int64_t ne = e_ptr[n_vert];
  if (ne > 0 && (!e_dst || !e_syn)) return bad(DTB_ERR_INVALID, "partition: null edge arrays");
  for (int64_t u = 0; u < n_vert; ++u) {
    if (e_ptr[u + 1] < e_ptr[u]) return bad(DTB_ERR_INVALID, "partition: e_ptr decreases");
    if (!(neurons[u] > 0.0) || !(size[u] >= 0.0) || !(spikes[u] >= 0.0) || !std::isfinite(size[u]) ||
        !std::isfinite(spikes[u]) || !std::isfinite(neurons[u]))
      return bad(DTB_ERR_INVALID, "partition: vertex " + std::to_string(u) + " has a bad size / neurons / spikes");
    if (size[u] > capacity) return bad(DTB_ERR_UNSUPPORTED, "partition: a vertex exceeds the capacity");
  }
  for (int64_t e = 0; e < ne; ++e)
    if (e_dst[e] < 0 || e_dst[e] >= n_vert || !(e_syn[e] >= 0.0) || !std::isfinite(e_syn[e]))
      return bad(DTB_ERR_INVALID, "partition: bad edge " + std::to_string(e));
  Part P;
  P.n = n_vert;
  P.N = n_gpu;
  P.size = size;
  P.nn = neurons;
  P.spk = spikes;
  P.b = bytes_per_spike;
  P.optr.assign(e_ptr, e_ptr + n_vert + 1);
  P.odst.assign(e_dst, e_dst + ne);
  P.osyn.assign(e_syn, e_syn + ne);
  // in-edges
  P.iptr.assign(size_t(n_vert) + 1, 0);
  for (int64_t e = 0; e < ne; ++e) P.iptr[e_dst[e] + 1]++;
  for (int64_t v = 0; v < n_vert; ++v) P.iptr[v + 1] += P.iptr[v];
  P.isrc.resize(size_t(ne));
  P.isyn.resize(size_t(ne));
  {
    std::vector<int64_t> at(P.iptr.begin(), P.iptr.end() - 1);
    for (int64_t u = 0; u < n_vert; ++u)
      for (int64_t e = e_ptr[u]; e < e_ptr[u + 1]; ++e) {
        const int64_t q = at[e_dst[e]]++;
        P.isrc[q] = int32_t(u);
        P.isyn[q] = e_syn[e];
      }
  }
  P.part.assign(size_t(n_vert), -1);
  P.c.assign(size_t(n_vert) * n_gpu, 0.0);
  P.D.assign(size_t(n_gpu) * n_gpu, 0.0);
  P.load.assign(size_t(n_gpu), 0.0);
  double tot = 0.0;
  for (int64_t u = 0; u < n_vert; ++u) tot += size[u];
  if (tot > capacity * n_gpu) return bad(DTB_ERR_UNSUPPORTED, "partition: total size exceeds n_gpu * capacity");

  if (init) {
    for (int64_t u = 0; u < n_vert; ++u) {
      if (init[u] < 0 || init[u] >= n_gpu) return bad(DTB_ERR_INVALID, "partition: init out of range");
      P.part[u] = init[u];
    }
  } else {
    // greedy fill, one GPU at a time: seed with the largest unassigned
    // vertex, then take the unassigned vertex with the most synapses to or
    // from the GPU's vertices while the GPU stays within an even share
    const double share = std::min(capacity, tot / n_gpu);
    std::vector<double> conn(size_t(n_vert), 0.0);
    int64_t left = n_vert;
    for (int32_t g = 0; g < n_gpu && left > 0; ++g) {
      std::fill(conn.begin(), conn.end(), 0.0);
      double fill = 0.0;
      const bool last = g == n_gpu - 1;
      while (left > 0) {
        int64_t best = -1;
        for (int64_t u = 0; u < n_vert; ++u) {
          if (P.part[u] >= 0) continue;
          const double lim = last ? capacity : share;
          if (fill + size[u] > lim * (1.0 + 1e-12) && fill > 0.0) continue;
          if (best < 0 || conn[u] > conn[best] || (conn[u] == conn[best] && size[u] > size[best])) best = u;
        }
        if (best < 0) break;
        if (!last && fill > 0.0 && fill + size[best] > share * (1.0 + 1e-12)) break;
        P.part[best] = g;
        fill += size[best];
        --left;
        for (int64_t e = e_ptr[best]; e < e_ptr[best + 1]; ++e) conn[e_dst[e]] += e_syn[e];
        for (int64_t e = P.iptr[best]; e < P.iptr[best + 1]; ++e) conn[P.isrc[e]] += P.isyn[e];
        if (fill >= share && !last) break;
      }
    }
    if (left > 0) {
      // place what the even shares left over on the least-loaded GPU that has room
      std::vector<double> fill(size_t(n_gpu), 0.0);
      for (int64_t u = 0; u < n_vert; ++u)
        if (P.part[u] >= 0) fill[P.part[u]] += size[u];
      for (int64_t u = 0; u < n_vert; ++u) {
        if (P.part[u] >= 0) continue;
        int32_t g = -1;
        for (int32_t q = 0; q < n_gpu; ++q)
          if (fill[q] + size[u] <= capacity && (g < 0 || fill[q] < fill[g])) g = q;
        if (g < 0) return bad(DTB_ERR_UNSUPPORTED, "partition: the greedy fill found no room (raise capacity)");
        P.part[u] = g;
        fill[g] += size[u];
      }
    }
  }
  P.recompute();
  for (int32_t g = 0; g < n_gpu; ++g)
    if (P.load[g] > capacity * (1.0 + 1e-12)) return bad(DTB_ERR_INVALID, "partition: init exceeds the capacity");

  // local search on the GPU with the heaviest incoming traffic
  for (int32_t round = 0; round < refine_rounds; ++round) {
    int32_t js = 0;
    const double f0 = P.F(&js);
    const double t0 = P.total();
    bool improved = false;
    auto try_move = [&](int64_t u, int32_t g) {
      const int32_t a = P.part[u];
      if (g == a || P.load[g] + size[u] > capacity) return false;
      P.move(u, g);
      const double f1 = P.F();
      if (f1 < f0 * (1.0 - 1e-12) || (f1 <= f0 && P.total() < t0 * (1.0 - 1e-12))) return true;
      P.move(u, a);
      return false;
    };
    // candidates: vertices elsewhere sending the most to js (move into js),
    // then vertices on js (move to the GPU that takes them best)
    std::vector<std::pair<double, int64_t>> cand;
    for (int64_t u = 0; u < n_vert; ++u)
      if (P.part[u] != js) cand.emplace_back(-P.contrib(u, js), u);
    std::sort(cand.begin(), cand.end());
    for (size_t q = 0; q < cand.size() && q < 64 && !improved; ++q) improved = try_move(cand[q].second, js);
    for (int64_t u = 0; u < n_vert && !improved; ++u) {
      if (P.part[u] != js) continue;
      for (int32_t g = 0; g < n_gpu && !improved; ++g) improved = try_move(u, g);
    }
    // then swaps of a vertex on js with one of the strongest senders to js,
    // which keep both GPUs within the capacity when single moves cannot
    for (int64_t u = 0; u < n_vert && !improved; ++u) {
      if (P.part[u] != js) continue;
      for (size_t q = 0; q < cand.size() && q < 64 && !improved; ++q) {
        const int64_t v = cand[q].second;
        const int32_t g = P.part[v];
        if (g == js || P.load[js] - size[u] + size[v] > capacity || P.load[g] - size[v] + size[u] > capacity)
          continue;
        P.move(u, g);
        P.move(v, js);
        const double f1 = P.F();
        if (f1 < f0 * (1.0 - 1e-12) || (f1 <= f0 && P.total() < t0 * (1.0 - 1e-12))) {
          improved = true;
        } else {
          P.move(v, g);
          P.move(u, js);
        }
      }
    }
    if (!improved) break;
    if ((round & 63) == 63) P.recompute();  // drop accumulated rounding of the incremental updates
  }
  P.recompute();
  for (int64_t u = 0; u < n_vert; ++u) part[u] = P.part[u];
  if (F_out) *F_out = P.F();
  if (D_out)
    for (int32_t i = 0; i < n_gpu; ++i)
      for (int32_t j = 0; j < n_gpu; ++j) D_out[size_t(i) * n_gpu + j] = i == j ? 0.0 : P.D[size_t(i) * n_gpu + j];
  return DTB_OK;
}
