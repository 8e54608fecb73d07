// Host planner.  Paper passages followed:
//   * MaxCut cost and QAOA ansatz: Section II (eq. qaoa1), U_C = exp(-i gamma C).
//   * light cone of an edge term: Section II (local terms; gates outside the
//     backward light cone cancel).
//   * tensors of states and gates, diagonal gates without new indices:
//     Sections III.A and IV.B (eq. example, the rank-2 ZZ tensor).
//   * bucket elimination and the role of the order: Section III.B (eq. tn).
#include "plan.hpp"

#include <algorithm>
#include <map>
#include <queue>
#include <functional>
#include <iterator>
#include <cstring>
#include <cmath>
#include <climits>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <set>

namespace qtn {

std::string validate_graph(int32_t n, int32_t m, const int32_t* edges, int32_t p) {
  if (n < 1) return "n_vertices must be >= 1";
  if (m < 0) return "n_edges must be >= 0";
  if (p < 1) return "p must be >= 1";
  if (p > 16) return "p must be <= 16";
  if (m > 0 && !edges) return "edges is NULL";
  std::set<std::pair<int, int>> seen;
  for (int e = 0; e < m; ++e) {
    int u = edges[2 * e], v = edges[2 * e + 1];
    if (u < 0 || v < 0 || u >= n || v >= n) return "edge " + std::to_string(e) + " has a vertex id out of range";
    if (u == v) return "edge " + std::to_string(e) + " is a self-loop";
    if (!seen.insert({std::min(u, v), std::max(u, v)}).second)
      return "edge " + std::to_string(e) + " is a duplicate";
  }
  return "";
}

// ---------------------------------------------------------------- light cones
// Qubit q at graph distance d(q) <= p from {j,k} keeps its mixers of layers
// 1..m_q with m_q = p - d(q); the ZZ gate of layer l on (u,w) survives iff
// min(d_u, d_w) <= p - l.  Each qubit carries ket indices a_{q,0..m_q-1}, bra
// indices b_{q,0..m_q-1} and one index t_q shared by ket and bra (the identity
// and the observable between them are diagonal).
void build_cones(Plan& P) {
  const int n = P.n, p = P.p;
  std::vector<std::vector<int>> adj(n);
  for (auto& e : P.edges) {
    adj[e.first].push_back(e.second);
    adj[e.second].push_back(e.first);
  }
  for (auto& a : adj) std::sort(a.begin(), a.end());
  P.cones.assign(P.edges.size(), Cone());
  std::vector<int> dist(n, -1), local(n, -1);
  for (size_t ei = 0; ei < P.edges.size(); ++ei) {
    Cone& C = P.cones[ei];
    const int j = P.edges[ei].first, k = P.edges[ei].second;
    C.j = j;
    C.k = k;
    std::vector<int> qs = {j, k};
    dist[j] = dist[k] = 0;
    for (size_t h = 0; h < qs.size(); ++h) {
      int u = qs[h];
      if (dist[u] == p) continue;
      for (int w : adj[u])
        if (dist[w] < 0) {
          dist[w] = dist[u] + 1;
          qs.push_back(w);
        }
    }
    const int nq = (int)qs.size();
    C.n_qubits = nq;
    for (int i = 0; i < nq; ++i) local[qs[i]] = i;
    // index ids
    std::vector<int> top(nq), m(nq), a0(nq), b0(nq);
    int nid = 0;
    for (int i = 0; i < nq; ++i) {
      m[i] = p - dist[qs[i]];
      top[i] = nid++;
      a0[i] = nid;
      nid += m[i];
      b0[i] = nid;
      nid += m[i];
    }
    C.n_idx = nid;
    auto K = [&](int i, int s) { return s < m[i] ? a0[i] + s : top[i]; };
    auto B = [&](int i, int s) { return s < m[i] ? b0[i] + s : top[i]; };
    auto& L = C.leaves;
    for (int i = 0; i < nq; ++i) {
      L.push_back({LK_PLUS, K(i, 0), -1});
      L.push_back({LK_PLUS, B(i, 0), -1});
      for (int l = 1; l <= m[i]; ++l) {
        L.push_back({lk_mx(l - 1), K(i, l - 1), K(i, l)});
        L.push_back({lk_mxb(l - 1), B(i, l - 1), B(i, l)});
      }
    }
    for (int i = 0; i < nq; ++i) {
      int u = qs[i];
      for (int w : adj[u]) {
        if (local[w] < 0 || w <= u) continue;
        int iw = local[w];
        int dmin = std::min(dist[u], dist[w]);
        for (int l = 1; l <= p; ++l) {
          if (dmin > p - l) continue;
          L.push_back({lk_zz(l - 1), K(i, l - 1), K(iw, l - 1)});
          L.push_back({lk_zzb(l - 1), B(i, l - 1), B(iw, l - 1)});
        }
      }
    }
    L.push_back({LK_ZOBS, top[0], -1});
    L.push_back({LK_ZOBS, top[1], -1});
    for (int u : qs) {
      dist[u] = -1;
      local[u] = -1;
    }
  }
}

void build_amplitude(Plan& P) {
  const int n = P.n, p = P.p;
  P.cones.assign(1, Cone());
  Cone& C = P.cones[0];
  C.j = C.k = -1;
  C.n_qubits = n;
  // index a(q, s), s = 0..p: the wire of qubit q after s mixer layers
  auto A = [&](int q, int s) { return q * (p + 1) + s; };
  C.n_idx = n * (p + 1);
  auto& L = C.leaves;
  for (int q = 0; q < n; ++q) {
    L.push_back({LK_PLUS, A(q, 0), -1});
    for (int l = 1; l <= p; ++l) L.push_back({lk_mx(l - 1), A(q, l - 1), A(q, l)});
    L.push_back({lk_proj0(p), A(q, p), -1});
  }
  for (auto& e : P.edges)
    for (int l = 1; l <= p; ++l) L.push_back({lk_zz(l - 1), A(e.first, l - 1), A(e.second, l - 1)});
}

// ---------------------------------------------------------------- ordering
// Greedy elimination on the interaction graph (indices adjacent iff they share
// a leaf).  min-degree: fewest neighbours; min-fill: fewest new edges among
// the neighbours.  Deterministic runs break ties by the smaller degree, then
// the lowest index id.  Randomized runs (the paper's order finder is a
// randomized greedy with repeats and a temperature, Section V) pick among the
// candidates with weights exp(-(score - min score) / temperature), and the
// cheapest of all runs is kept.  Cost of an order: sum over buckets of
// 2^|union| (the work of the contraction).
namespace {

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct OrderRun {
  std::vector<int> order;
  int width = 0;
  double cost = 0;
};

OrderRun order_run(const Cone& C, int kind, bool randomized, double temperature, uint64_t seed) {
  const int n = C.n_idx;
  const int nw = (n + 63) / 64;
  std::vector<uint64_t> adj((size_t)n * nw, 0);
  auto row = [&](int v) { return adj.data() + (size_t)v * nw; };
  auto setb = [&](uint64_t* r, int b) { r[b >> 6] |= 1ull << (b & 63); };
  for (auto& l : C.leaves)
    if (l.b >= 0) {
      setb(row(l.a), l.b);
      setb(row(l.b), l.a);
    }
  std::vector<char> alive(n, 1);
  std::vector<int64_t> prim(n, 0), deg(n, 0);
  auto degree = [&](int v) {
    int d = 0;
    const uint64_t* r = row(v);
    for (int w = 0; w < nw; ++w) d += __builtin_popcountll(r[w]);
    return d;
  };
  auto fill = [&](int v) {
    const uint64_t* r = row(v);
    int64_t f = 0;
    for (int w = 0; w < nw; ++w) {
      uint64_t bits = r[w];
      while (bits) {
        int a = (w << 6) + __builtin_ctzll(bits);
        bits &= bits - 1;
        const uint64_t* ra = row(a);
        for (int x = 0; x < nw; ++x) {
          uint64_t miss = r[x] & ~ra[x];
          if (x == (a >> 6)) miss &= ~(1ull << (a & 63));
          f += __builtin_popcountll(miss);
        }
      }
    }
    return f / 2;
  };
  auto rescore = [&](int v) {
    deg[v] = degree(v);
    prim[v] = kind == 1 ? fill(v) : deg[v];
  };
  for (int v = 0; v < n; ++v) rescore(v);
  OrderRun R;
  R.order.reserve(n);
  std::vector<int> nb, touched, cand;
  std::vector<double> wts;
  std::vector<char> mark(n, 0);
  uint64_t rng = seed;
  for (int step = 0; step < n; ++step) {
    int v = -1;
    if (!randomized) {
      for (int x = 0; x < n; ++x)
        if (alive[x] && (v < 0 || prim[x] < prim[v] || (prim[x] == prim[v] && deg[x] < deg[v]))) v = x;
    } else {
      int64_t mn = INT64_MAX;
      for (int x = 0; x < n; ++x)
        if (alive[x]) mn = std::min(mn, prim[x]);
      cand.clear();
      wts.clear();
      double tot = 0;
      const double T = std::max(temperature, 1e-12);
      for (int x = 0; x < n; ++x) {
        if (!alive[x]) continue;
        const double d = (double)(prim[x] - mn) / T;
        if (d > 30.0) continue;
        const double wgt = std::exp(-d);
        cand.push_back(x);
        wts.push_back(wgt);
        tot += wgt;
      }
      double r = (double)(splitmix64(rng) >> 11) * (1.0 / 9007199254740992.0) * tot;
      v = cand.back();
      for (size_t i = 0; i < cand.size(); ++i) {
        r -= wts[i];
        if (r <= 0) {
          v = cand[i];
          break;
        }
      }
    }
    nb.clear();
    uint64_t* rv = row(v);
    for (int w = 0; w < nw; ++w) {
      uint64_t bits = rv[w];
      while (bits) {
        nb.push_back((w << 6) + __builtin_ctzll(bits));
        bits &= bits - 1;
      }
    }
    R.width = std::max(R.width, (int)nb.size());
    R.cost += std::ldexp(1.0, (int)nb.size() + 1);
    for (int a : nb) {
      uint64_t* ra = row(a);
      for (int w = 0; w < nw; ++w) ra[w] |= rv[w];
      ra[a >> 6] &= ~(1ull << (a & 63));
      ra[v >> 6] &= ~(1ull << (v & 63));
    }
    std::fill(rv, rv + nw, 0);
    alive[v] = 0;
    R.order.push_back(v);
    touched.clear();
    for (int a : nb)
      if (!mark[a]) {
        mark[a] = 1;
        touched.push_back(a);
      }
    if (kind == 1) {
      const size_t n1 = touched.size();
      for (size_t t = 0; t < n1; ++t) {
        const uint64_t* ra = row(touched[t]);
        for (int w = 0; w < nw; ++w) {
          uint64_t bits = ra[w];
          while (bits) {
            int b = (w << 6) + __builtin_ctzll(bits);
            bits &= bits - 1;
            if (!mark[b]) {
              mark[b] = 1;
              touched.push_back(b);
            }
          }
        }
      }
    }
    for (int a : touched) {
      mark[a] = 0;
      rescore(a);
    }
  }
  return R;
}

void order_one(Cone& C, const OrderOptions& O, uint64_t cone_seed) {
  OrderRun best = order_run(C, O.kind, false, 0.0, 0);
  uint64_t s = O.seed ^ (cone_seed * 0xD1B54A32D192ED03ull);
  for (int r = 0; r < O.repeats; ++r) {
    OrderRun R = order_run(C, O.kind, true, O.temperature, splitmix64(s));
    if (R.cost < best.cost || (R.cost == best.cost && R.width < best.width)) best = std::move(R);
  }
  C.order = std::move(best.order);
  C.width = best.width;
}


// ---------------------------------------------------------------- cost model
// Index structure of the single-amplitude network <0...0|gamma beta> under the
// four constructions the paper compares (Section IV, Figures diag_costs and
// diag_costs_vs_n, Tables I and II).  Circuit: |0> and H on every qubit, then
// per layer the cost gates of every edge and the mixer of every qubit, then
// <0| on every qubit.  "ZZ" circuits use one two-qubit ZZ(gamma) gate per edge
// and one X rotation per qubit; the others decompose them as CNOT, Z rotation
// on the target, CNOT and H, Z rotation, H.  Without the diagonal
// simplification every gate gives each qubit it acts on a fresh index (a
// 2-index tensor per one-qubit gate, 4 indices per two-qubit gate); with it,
// a gate keeps the index of every qubit it acts on diagonally (Z rotations and
// ZZ on both of their qubits, CNOT on its control), so the ZZ phase becomes a
// rank-2 tensor on the two current indices.  Indices are numbered in the order
// the construction creates them (a two-qubit gate numbers its first qubit's
// new index first), the numbering of the exported elimination order.
struct IndexNet {
  int n_idx = 0;
  std::vector<std::vector<int>> tensors;
};

IndexNet variant_network(int n, const std::vector<std::pair<int32_t, int32_t>>& edges, int p, int variant) {
  const bool diag = variant == 1 || variant == 3;
  const bool zz = variant == 2 || variant == 3;
  IndexNet T;
  std::vector<int> cur(n);
  for (int q = 0; q < n; ++q) {
    cur[q] = T.n_idx++;
    T.tensors.push_back({cur[q]});  // |0>
  }
  auto one_qubit = [&](int q, bool keeps) {  // a one-qubit gate
    if (keeps) {
      T.tensors.push_back({cur[q]});
    } else {
      const int nw = T.n_idx++;
      T.tensors.push_back({cur[q], nw});
      cur[q] = nw;
    }
  };
  for (int q = 0; q < n; ++q) one_qubit(q, false);  // H
  for (int l = 0; l < p; ++l) {
    for (auto& e : edges) {
      const int u = e.first, w = e.second;
      if (zz) {
        if (diag) {
          T.tensors.push_back({cur[u], cur[w]});
        } else {
          const int nu = T.n_idx++, nw = T.n_idx++;
          T.tensors.push_back({cur[u], cur[w], nu, nw});
          cur[u] = nu;
          cur[w] = nw;
        }
      } else {
        for (int g = 0; g < 3; ++g) {
          if (g == 1) {
            one_qubit(w, diag);  // Z rotation on the target
            continue;
          }
          // CNOT(u -> w): the control keeps its index under the diagonal
          // simplification; otherwise the control's new index is numbered first
          if (diag) {
            const int nw = T.n_idx++;
            T.tensors.push_back({cur[u], cur[w], nw});
            cur[w] = nw;
          } else {
            const int nu = T.n_idx++, nw = T.n_idx++;
            T.tensors.push_back({cur[u], cur[w], nu, nw});
            cur[u] = nu;
            cur[w] = nw;
          }
        }
      }
    }
    for (int q = 0; q < n; ++q) {
      if (zz) {
        one_qubit(q, false);  // X rotation
      } else {
        one_qubit(q, false);  // H
        one_qubit(q, diag);   // Z rotation
        one_qubit(q, false);  // H
      }
    }
  }
  for (int q = 0; q < n; ++q) T.tensors.push_back({cur[q]});  // <0|
  return T;
}

}  // namespace

CostEstimate cost_model(int n, const std::vector<std::pair<int32_t, int32_t>>& edges, int p, int variant,
                        const OrderOptions& O, std::vector<int>* order_out) {
  const IndexNet T = variant_network(n, edges, p, variant);
  // the orderer works on the interaction graph: a tensor links every pair of
  // its indices
  Cone C;
  C.n_idx = T.n_idx;
  for (const auto& t : T.tensors)
    for (size_t i = 0; i < t.size(); ++i)
      for (size_t j = i + 1; j < t.size(); ++j) C.leaves.push_back({0, t[i], t[j]});
  order_one(C, O, 1);
  // bucket elimination along the order: width and sum of 2^|union|
  std::vector<int> pos(T.n_idx);
  for (int s = 0; s < T.n_idx; ++s) pos[C.order[s]] = s;
  std::vector<std::vector<std::vector<int>>> pending(T.n_idx);  // tensors waiting at each bucket
  auto place = [&](const std::vector<int>& t) {
    int first = t[0];
    for (int x : t)
      if (pos[x] < pos[first]) first = x;
    pending[pos[first]].push_back(t);
  };
  for (const auto& t : T.tensors) place(t);
  CostEstimate R;
  R.n_indices = T.n_idx;
  R.n_tensors = (int)T.tensors.size();
  double ops = 0;
  for (int s = 0; s < T.n_idx; ++s) {
    std::vector<int> uni;
    for (const auto& t : pending[s]) uni.insert(uni.end(), t.begin(), t.end());
    std::sort(uni.begin(), uni.end());
    uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
    if (uni.empty()) continue;
    ops += std::ldexp(1.0, (int)uni.size());
    std::vector<int> out;
    for (int x : uni)
      if (pos[x] != s) out.push_back(x);
    R.width = std::max(R.width, (int)out.size());
    if (!out.empty()) place(out);
  }
  R.log2_ops = ops > 0 ? std::log2(ops) : 0.0;
  if (order_out) *order_out = C.order;
  return R;
}

// Symbolic bucket elimination (Section III.B): the bucket of v holds every
// tensor whose earliest-eliminated index is v; its output carries the union of
// their indices without v and goes to the bucket of its earliest index.
static void buckets_one(Cone& C) {
  const int n = C.n_idx;
  std::vector<int> pos(n);
  for (int s = 0; s < n; ++s) pos[C.order[s]] = s;
  C.plain.assign(n, Bucket());
  std::vector<std::vector<int>> out_idx(n);
  for (size_t li = 0; li < C.leaves.size(); ++li) {
    const Leaf& l = C.leaves[li];
    int first = l.b < 0 ? l.a : (pos[l.a] < pos[l.b] ? l.a : l.b);
    C.plain[pos[first]].leaves.push_back((int)li);
  }
  std::vector<std::vector<int>> pending(n);  // producer buckets waiting at each bucket
  int width = 0;
  for (int s = 0; s < n; ++s) {
    Bucket& Bk = C.plain[s];
    Bk.v = C.order[s];
    Bk.in_bkt = pending[s];
    std::vector<int> uni = {Bk.v};
    for (int li : Bk.leaves) {
      uni.push_back(C.leaves[li].a);
      if (C.leaves[li].b >= 0) uni.push_back(C.leaves[li].b);
    }
    for (int pb : Bk.in_bkt)
      for (int x : out_idx[pb]) uni.push_back(x);
    std::sort(uni.begin(), uni.end(), [&](int a, int b) { return pos[a] < pos[b]; });
    uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
    Bk.uni = uni;
    auto bit_of = [&](int idx) {
      for (size_t t = 0; t < uni.size(); ++t)
        if (uni[t] == idx) return (int)t;
      return -1;
    };
    Bk.lam_mask = 0;
    for (int li : Bk.leaves) {
      Bk.lam_mask |= 1u << bit_of(C.leaves[li].a);
      if (C.leaves[li].b >= 0) Bk.lam_mask |= 1u << bit_of(C.leaves[li].b);
    }
    Bk.in_mask.clear();
    for (int pb : Bk.in_bkt) {
      uint32_t mk = 0;
      for (int x : out_idx[pb]) mk |= 1u << bit_of(x);
      Bk.in_mask.push_back(mk);
    }
    out_idx[s].assign(uni.begin() + 1, uni.end());
    width = std::max(width, (int)uni.size() - 1);
    if (uni.size() == 1) {
      Bk.consumer = -1;
    } else {
      Bk.consumer = pos[uni[1]];
      pending[Bk.consumer].push_back(s);
    }
  }
  C.width = width;
}


// Contraction steps of a cone from its plain buckets.  In elimination order,
// a bucket (with the buckets already merged into it) joins its consumer while
// the merged union stays within merge_bits bits and the merged step has at
// most MAXIN inputs: for buckets this small every step costs about the same
// fixed time, so fewer steps are faster.  At any size it joins a consumer that
// adds no index to its union (its output is then never written): a marginal
// of its output always, one that adds inputs when the merged step suits the
// wide executor.  A merged step is the union of its
// members' tensors summed over all of their eliminated indices (the same
// contraction, Section III.B, taken several indices at a time).
static void group_buckets(Cone& C, int merge_bits, int merge_lam_bits) {
  const std::vector<Bucket>& Pl = C.plain;
  const int n = (int)Pl.size();
  std::vector<int> pos(C.n_idx);
  for (int s = 0; s < n; ++s) pos[C.order[s]] = s;
  std::vector<int> root(n), gsize(n), gelim(n, 1), gnin(n), glam(n), gfirst(n);
  std::vector<std::vector<int>> gleafidx(n);  // indices carried by the group's leaves
  std::vector<std::vector<int>> ginputs(n);   // producer groups (their roots) feeding the group
  for (int b = 0; b < n; ++b) {
    root[b] = b;
    gsize[b] = Pl[b].nbits();
    gnin[b] = (int)Pl[b].in_bkt.size();
    glam[b] = Pl[b].lam_mask ? 1 : 0;
    gfirst[b] = Pl[b].v;
    ginputs[b] = Pl[b].in_bkt;
    for (int li : Pl[b].leaves) {
      gleafidx[b].push_back(C.leaves[li].a);
      if (C.leaves[li].b >= 0) gleafidx[b].push_back(C.leaves[li].b);
    }
    std::sort(gleafidx[b].begin(), gleafidx[b].end());
    gleafidx[b].erase(std::unique(gleafidx[b].begin(), gleafidx[b].end()), gleafidx[b].end());
  }
  std::function<int(int)> find = [&](int x) { return root[x] == x ? x : (root[x] = find(root[x])); };
  if (merge_bits > 0)
    for (int b = 0; b < n; ++b) {
      const int t = Pl[b].consumer;  // b is still its group's root; t has not been merged anywhere yet
      if (t < 0) continue;
      const int size = gsize[t] + gelim[b];
      const int nin = gnin[t] - 1 + gnin[b];
      const int lam = glam[t] | glam[b];
      if (nin + lam > MAXIN) continue;
      // the merged leaf-product table (built and differentiated per entry)
      // stays small
      std::vector<int> li;
      std::set_union(gleafidx[t].begin(), gleafidx[t].end(), gleafidx[b].begin(), gleafidx[b].end(),
                     std::back_inserter(li));
      if ((int)li.size() > merge_lam_bits) continue;
      // At any size, when the consumer carries no index beyond b's output
      // (the merged union is b's own), the merge saves writing b's output
      // and reading it back (forward and adjoint):
      //  * a marginal of b's output (no input added): always;
      //  * with the consumer's other inputs (or leaf table) added: when the
      //    merged step still suits the wide executor -- at most 4 inputs,
      //    at most one of them without the step's first eliminated index
      //    (its adjoint passes then have at most two such inputs, the output
      //    adjoint being the other).
      bool wide_ok = false;
      if (size <= gsize[b]) {
        if (nin + lam <= gnin[b] + glam[b]) {
          wide_ok = true;
        } else if (nin + lam <= 4) {
          const int first = pos[gfirst[t]] < pos[gfirst[b]] ? gfirst[t] : gfirst[b];
          auto holds = [&](const std::vector<int>& ix) { return std::find(ix.begin(), ix.end(), first) != ix.end(); };
          int singles = 0;
          for (int g : {b, t})
            for (int x : ginputs[g])
              if (x != b && !holds(std::vector<int>(Pl[x].uni.begin() + 1, Pl[x].uni.end()))) ++singles;
          if (lam && !holds(li)) ++singles;
          wide_ok = singles <= 1;
        }
      }
      if (size > merge_bits && !wide_ok) continue;
      gleafidx[t] = li;
      root[b] = t;
      gsize[t] = size;
      gelim[t] += gelim[b];
      gnin[t] = nin;
      glam[t] = lam;
      if (pos[gfirst[b]] < pos[gfirst[t]]) gfirst[t] = gfirst[b];
      std::vector<int> ins;
      for (int x : ginputs[t])
        if (x != b) ins.push_back(x);
      ins.insert(ins.end(), ginputs[b].begin(), ginputs[b].end());
      ginputs[t] = ins;
    }
  std::vector<int> idx(n, -1);
  int ng = 0;
  for (int b = 0; b < n; ++b)
    if (find(b) == b) idx[b] = ng++;
  C.buckets.assign(ng, Bucket());
  C.scalars.clear();
  std::vector<std::vector<int>> members(ng);
  for (int b = 0; b < n; ++b) members[idx[find(b)]].push_back(b);
  for (int r = 0; r < n; ++r) {
    if (idx[r] < 0) continue;
    Bucket& G = C.buckets[idx[r]];
    const std::vector<int>& mem = members[idx[r]];
    G.v = Pl[mem[0]].v;
    G.n_elim = (int)mem.size();
    std::vector<int> uni;
    for (int m : mem) uni.push_back(Pl[m].v);
    uni.insert(uni.end(), Pl[r].uni.begin() + 1, Pl[r].uni.end());
    std::sort(uni.begin(), uni.end(), [&](int a, int b) { return pos[a] < pos[b]; });
    G.uni = uni;
    auto bit_of = [&](int x) {
      for (size_t t = 0; t < uni.size(); ++t)
        if (uni[t] == x) return (int)t;
      return -1;
    };
    for (int m : mem) {
      G.leaves.insert(G.leaves.end(), Pl[m].leaves.begin(), Pl[m].leaves.end());
      for (int pb : Pl[m].in_bkt) {
        const int g = find(pb);
        if (g == r) continue;
        G.in_bkt.push_back(idx[g]);
        uint32_t mk = 0;
        for (size_t q = 1; q < Pl[g].uni.size(); ++q) mk |= 1u << bit_of(Pl[g].uni[q]);
        G.in_mask.push_back(mk);
      }
    }
    G.lam_mask = 0;
    for (int li : G.leaves) {
      G.lam_mask |= 1u << bit_of(C.leaves[li].a);
      if (C.leaves[li].b >= 0) G.lam_mask |= 1u << bit_of(C.leaves[li].b);
    }
    G.consumer = Pl[r].consumer < 0 ? -1 : idx[find(Pl[r].consumer)];
    if (G.consumer < 0) C.scalars.push_back(idx[r]);
  }
}

void order_cones(Plan& P, const OrderOptions& O, int n_threads) {
  const size_t nc = P.cones.size();
  n_threads = std::max(1, std::min<int>(n_threads, (int)nc));
  std::vector<std::thread> th;
  for (int t = 0; t < n_threads; ++t)
    th.emplace_back([&, t]() {
      for (size_t c = t; c < nc; c += n_threads) {
        order_one(P.cones[c], O, (uint64_t)c + 1);
        buckets_one(P.cones[c]);
      }
    });
  for (auto& x : th) x.join();
  P.max_width = 0;
  for (auto& C : P.cones) P.max_width = std::max(P.max_width, C.width);
  P.order_kind = O.kind;
  P.ordered = true;
}

// ---------------------------------------------------------------- arena layout
static int64_t align_elems(int64_t off, int64_t size) {
  int64_t a = size >= 64 ? 64 : 2;
  return (off + a - 1) / a * a;
}

// ---------------------------------------------------------------- op programs
namespace {

struct Ctx {
  Plan& P;
  int elem_bytes;
};

// Split the non-pair union bits of a contraction op into lanes, loop and
// blocks (see OpDesc).  seq: the op runs inside one workgroup, so no summed
// bit may become a block bit (no atomics).
void partition_bits_as(OpDesc& d, int nbits, uint32_t out_mask, bool seq, bool wide, const TuneParams& T);

// Inputs of a contraction op without the eliminated index (bit 0), if they
// are its first 0, 1 or 2 inputs (the wide executor loads them as single
// elements, the others as pairs); -1 otherwise.
int wide_singles(const OpDesc& d) {
  int k = 0;
  while (k < d.n_in && !(d.in_mask[k] & 1u)) ++k;
  for (int i = k; i < d.n_in; ++i)
    if (!(d.in_mask[i] & 1u)) return -1;
  return k <= 2 ? k : -1;
}

// Splits the union bits of a contraction op into lanes, per-thread outputs,
// the summation loop and blocks.  Ops outside sequential programs with at
// most 4 inputs, of which at most the first two lack the eliminated index, go
// to the wide executor when every block range they are given (a tile of
// tile_blocks blocks, or all blocks) holds at least one block per sub-block.
void partition_bits(OpDesc& d, int nbits, uint32_t out_mask, bool seq, const TuneParams& T0) {
  const TuneParams T = T0.for_bits(nbits);
  bool wide = !seq && d.n_in <= 4 && wide_singles(d) >= 0;
  if (wide) {
    partition_bits_as(d, nbits, out_mask, seq, true, T);
    const int64_t nsub = std::max(1, T.threads >> d.nl);
    const int64_t nblk = int64_t(1) << d.nb;
    if (std::min<int64_t>(std::max(1, T.tile_blocks), nblk) >= nsub) {
      d.flags |= F_WIDE;
      return;
    }
  }
  partition_bits_as(d, nbits, out_mask, seq, false, T);
}

void partition_bits_as(OpDesc& d, int nbits, uint32_t out_mask, bool seq, bool wide, const TuneParams& T) {
  std::vector<int> freeb, sumb;
  for (int u = 1; u < nbits; ++u) ((out_mask >> u) & 1 ? freeb : sumb).push_back(u);
  const int max_lanes = std::min({T.lane_cap, MAXLANE, 31 - __builtin_clz((unsigned)std::max(T.threads, 1))});
  std::vector<int> lanes, unroll, loop, blocks;
  size_t fi = 0, si = 0;
  d.lane_sum = 0;
  std::vector<int> rfree, rsum;
  if (wide && T.lane_low) {
    // wide ops: lanes on the lowest union bits, summed or not.  Every tensor
    // keeps its indices in elimination order, so neighbouring lanes read
    // neighbouring elements of every input; summed lane bits are combined
    // across lanes (shuffles, LDS above bit 5) before the store
    for (int u = 1; u < nbits; ++u) {
      const bool fr = (out_mask >> u) & 1;
      if ((int)lanes.size() < max_lanes) {
        if (!fr) d.lane_sum |= 1u << lanes.size();
        lanes.push_back(u);
      } else {
        (fr ? rfree : rsum).push_back(u);
      }
    }
  } else {
    // lanes: the lowest output bits (coalesced stores and, since every tensor
    // keeps its indices in elimination order, mostly coalesced loads); small
    // outputs fill the remaining lanes with summed bits (shuffle / LDS reduce)
    while (fi < freeb.size() && (int)lanes.size() < max_lanes) lanes.push_back(freeb[fi++]);
    while (si < sumb.size() && (int)lanes.size() < max_lanes) {
      d.lane_sum |= 1u << lanes.size();
      lanes.push_back(sumb[si++]);
    }
    rfree.assign(freeb.begin() + fi, freeb.end());
    rsum.assign(sumb.begin() + si, sumb.end());
  }
  if (!seq) {
    // several outputs per thread: more loads in flight, block offsets amortised
    // (bounded by the register budget of the kernel variant for this input count)
    const int nin = d.n_in;
    int cap;
    if (wide)  // per-thread outputs only where nothing is summed beyond the lanes (and the pair)
      cap = rsum.empty() ? (T.elem_bytes == 8 ? 2 : 1) : 0;
    else
      cap = std::min(T.unroll_cap, (T.elem_bytes == 8 && nin <= 2) ? 1 : 0);
    while ((int)unroll.size() < cap && rfree.size() > unroll.size() + 2) unroll.push_back(rfree[unroll.size()]);
    rfree.erase(rfree.begin(), rfree.begin() + unroll.size());
  }
  int nk;
  if (seq) {
    nk = (int)rsum.size();
  } else {
    // keep enough blocks to fill the chip: 2^(lanes + blocks) >= 2^par_bits threads
    const int need = std::max(0, T.par_bits - (int)lanes.size() - (int)rfree.size());
    nk = std::max(0, (int)rsum.size() - need);
    nk = std::min(nk, T.loop_cap);
    nk = std::max(nk, std::min((int)rsum.size(), 3));
  }
  loop.assign(rsum.begin(), rsum.begin() + nk);
  // block bits: the bits that large inputs lack vary fastest, so the blocks
  // that re-read the same input data run close together (and, with the
  // XCD-contiguous block mapping, on the same L2)
  std::vector<std::pair<double, int>> keyed;
  for (int u : rfree) {
    double w = 0;
    for (int i = 0; i < d.n_in; ++i)
      if (!((d.in_mask[i] >> u) & 1)) {
        const int r = __builtin_popcount(d.in_mask[i]);
        if (r >= 16) w += std::ldexp(1.0, r);
      }
    keyed.push_back({-w, u});
  }
  std::stable_sort(keyed.begin(), keyed.end());
  bool atomic = false;
  if (wide) {
    // wide ops: summed block bits vary fastest, so consecutive block steps of
    // a workgroup add into the same outputs and the executor carries its
    // partial sums across them (one atomic per output and run of steps)
    for (size_t t = nk; t < rsum.size(); ++t) {
      blocks.push_back(rsum[t]);
      atomic = true;
    }
    for (auto& kv : keyed) blocks.push_back(kv.second);
  } else {
    for (auto& kv : keyed) blocks.push_back(kv.second);
    for (size_t t = nk; t < rsum.size(); ++t) {
      blocks.push_back(rsum[t]);
      atomic = true;
    }
  }
  d.nl = (int)lanes.size();
  d.nu = (int)unroll.size();
  d.nk = (int)loop.size();
  d.nb = (int)blocks.size();
  int z = 0;
  for (int u : lanes) d.zbit[z++] = (uint8_t)u;
  for (int u : unroll) d.zbit[z++] = (uint8_t)u;
  for (int u : loop) d.zbit[z++] = (uint8_t)u;
  for (int u : blocks) d.zbit[z++] = (uint8_t)u;
  for (; z < 32; ++z) d.zbit[z] = 0;
  d.flags = (atomic ? F_ATOMIC : 0) | ((d.lane_sum >> 6) ? F_LDSRED : 0);
  auto lshift = [](uint32_t m, uint32_t u) -> uint8_t {
    return ((m >> u) & 1u) ? (uint8_t)__builtin_popcount(m & ((1u << u) - 1u)) : LSH_NONE;
  };
  for (int i = 0; i <= MAXIN; ++i)
    for (int j = 0; j < MAXLANE; ++j) {
      const uint32_t m = i == MAXIN ? out_mask : (i < d.n_in ? d.in_mask[i] : 0u);
      d.lsh[i][j] = j < d.nl ? lshift(m, d.zbit[j]) : LSH_NONE;
    }
}

// Bit split of an OP_ADJOINT op (inputs already set: the output adjoint, then
// every input of the bucket; output i is the adjoint of input i).  The loop
// bits are taken from one group of union bits that the same outputs hold:
// those outputs ("holders") get one value per loop step, combined across the
// lanes they sum and written at once, so every bit a holder sums must be a
// lane; the other outputs sum the loop bits in registers and write once per
// run of block steps that flip only bits they lack.  Lanes (at most 6, one
// wavefront) are the lowest union bits; among the groups of the other bits,
// the largest whose holders sum no bit outside the lanes is taken (so
// holders never need atomics).  An output that sums a block bit is added with atomics
// into zeroed memory.  Returns false (the bucket keeps one op per input
// adjoint) for a single input (its adjoint does not read it, so it need not
// be kept), more than 3 inputs, an input without the eliminated index, no
// group of at least 2 bits, or too few blocks per tile.
bool fused_adjoint_bits(OpDesc& d, int nbits, uint32_t all, const TuneParams& T0) {
  const TuneParams T = T0.for_bits(nbits);
  if (d.n_in < 3 || d.n_in > 4 || (d.in_mask[0] & 1u)) return false;
  d.adj_sel = 0;
  for (int i = 1; i < d.n_in; ++i) {
    if (!(d.in_mask[i] & 1u)) return false;
    d.adj_sel |= 1u << i;
  }
  const int max_lanes = std::min({T.lane_cap, 6, 31 - __builtin_clz((unsigned)std::max(T.threads, 1))});
  // lanes: the lowest union bits (neighbouring lanes read neighbouring
  // elements of every input)
  uint32_t lanes = 0;
  for (int u = 1; u < nbits && __builtin_popcount(lanes) < max_lanes; ++u) lanes |= 1u << u;
  // group the other bits by the set of outputs that hold them
  std::map<uint32_t, uint32_t> groups;  // holders -> bits
  for (int u = 1; u < nbits; ++u) {
    if ((lanes >> u) & 1u) continue;
    uint32_t h = 0;
    for (int i = 1; i < d.n_in; ++i) h |= ((d.in_mask[i] >> u) & 1u) << i;
    groups[h] |= 1u << u;
  }
  uint32_t best_bits = 0;
  for (const auto& g : groups) {
    uint32_t req = 0;  // bits some holder sums
    for (int i = 1; i < d.n_in; ++i)
      if ((g.first >> i) & 1u) req |= all & ~d.in_mask[i] & ~1u;
    if ((req & ~lanes) || __builtin_popcount(g.second) < 2) continue;
    if (__builtin_popcount(g.second) > __builtin_popcount(best_bits)) best_bits = g.second;
  }
  if (!best_bits) return false;
  std::vector<int> lane_v, loopable, others;
  for (int u = 1; u < nbits; ++u) {
    if ((lanes >> u) & 1u)
      lane_v.push_back(u);
    else
      (((best_bits >> u) & 1u) ? loopable : others).push_back(u);
  }
  const int nl = (int)lane_v.size();
  const int need = std::max(0, T.par_bits - nl - (int)others.size());
  int nk = std::max(0, (int)loopable.size() - need);
  nk = std::min(nk, T.loop_cap);
  nk = std::max(nk, std::min((int)loopable.size(), 3));
  const int nb = nbits - 1 - nl - nk;
  const int64_t nsub = std::max(1, T.threads >> nl);
  if (std::min<int64_t>(std::max(1, T.tile_blocks), int64_t(1) << nb) < nsub) return false;
  d.nl = nl;
  d.nu = 0;
  d.nk = nk;
  d.nb = nb;
  int z = 0;
  for (int u : lane_v) d.zbit[z++] = (uint8_t)u;
  for (int u : loopable) d.zbit[z++] = (uint8_t)u;  // loop bits, then block bits of the same group
  for (int u : others) d.zbit[z++] = (uint8_t)u;
  for (; z < 32; ++z) d.zbit[z] = 0;
  uint32_t blockbits = 0;
  for (int q = nl + nk; q < nbits - 1; ++q) blockbits |= 1u << d.zbit[q];
  bool atomic = false;
  for (int i = 1; i < d.n_in; ++i) atomic |= (blockbits & ~d.in_mask[i]) != 0;
  d.lane_sum = 0;
  d.out_mask = 0;
  d.out_off = 0;
  d.flags = F_WIDE | (atomic ? F_ATOMIC : 0);
  for (int i = 0; i <= MAXIN; ++i)
    for (int j = 0; j < MAXLANE; ++j) {
      const uint32_t m = i < d.n_in ? d.in_mask[i] : 0u;
      const uint32_t u = d.zbit[j];
      d.lsh[i][j] = (j < d.nl && ((m >> u) & 1u)) ? (uint8_t)__builtin_popcount(m & ((1u << u) - 1u)) : LSH_NONE;
    }
  return true;
}

// Bit split of an OP_ADJOINT op summed per tile in LDS (F_TILE), for buckets
// whose inputs each lack part of the union (no group of loop bits works for
// them): a workgroup takes one tile at a time (a value of the block bits) and
// walks the tile bits with all its threads, the lowest tile bits being the
// lanes of the whole workgroup and the rest a per-thread loop.  Every output
// sums its share of the tile in LDS (shuffles within a wavefront, then LDS
// atomics) and writes it once per tile: stored when it sums no block bit,
// else added with atomics into zeroed memory.  Tile bits: every bit summed by
// an output with more than 6 indices (those outputs are then stored), the
// lowest union bits that fit (contiguous reads), then the lowest others up to
// the workgroup size; the tile sums must fit kTileLdsBytes.
constexpr int64_t kTileLdsBytes = 24 * 1024;

bool tile_adjoint_bits(OpDesc& d, int nbits, uint32_t all, const TuneParams& T) {
  if (d.n_in < 3 || d.n_in > 4 || (d.in_mask[0] & 1u)) return false;
  const int lt = 31 - __builtin_clz((unsigned)std::max(T.threads, 64));
  d.adj_sel = 0;
  uint32_t tile = 0;
  for (int i = 1; i < d.n_in; ++i) {
    if (!(d.in_mask[i] & 1u) || d.in_mask[i] == all) return false;
    d.adj_sel |= 1u << i;
    if (__builtin_popcount(d.in_mask[i]) > 6) tile |= all & ~d.in_mask[i] & ~1u;
  }
  const int64_t budget = kTileLdsBytes / (2 * T.elem_bytes);  // pairs
  auto need = [&](uint32_t t) {
    int64_t s = 0;
    for (int i = 1; i < d.n_in; ++i) s += int64_t(1) << __builtin_popcount(t & d.in_mask[i]);
    return s;
  };
  if (need(tile) > budget) return false;
  for (int u = 1; u < std::min(nbits, 5); ++u)
    if (need(tile | (1u << u)) <= budget) tile |= 1u << u;
  for (int u = 1; u < nbits && __builtin_popcount(tile) < lt; ++u)
    if (need(tile | (1u << u)) <= budget) tile |= 1u << u;
  if (__builtin_popcount(tile) < lt || __builtin_popcount(tile) > lt + 12) return false;
  d.nl = lt;
  d.nu = 0;
  d.nk = __builtin_popcount(tile) - lt;
  d.nb = nbits - 1 - __builtin_popcount(tile);
  int z = 0;
  for (int u = 1; u < nbits; ++u)
    if ((tile >> u) & 1u) d.zbit[z++] = (uint8_t)u;  // lanes, then the loop
  uint32_t blockbits = 0;
  for (int u = 1; u < nbits; ++u)
    if (!((tile >> u) & 1u)) {
      d.zbit[z++] = (uint8_t)u;
      blockbits |= 1u << u;
    }
  for (; z < 32; ++z) d.zbit[z] = 0;
  bool atomic = false;
  for (int i = 1; i < d.n_in; ++i) atomic |= (blockbits & ~d.in_mask[i]) != 0;
  d.lane_sum = 0;
  d.out_mask = 0;
  d.out_off = 0;
  d.aux0 = (int32_t)(2 * need(tile));
  d.flags = F_WIDE | F_TILE | (atomic ? F_ATOMIC : 0);
  for (int i = 0; i <= MAXIN; ++i)
    for (int j = 0; j < MAXLANE; ++j) {
      const uint32_t m = i < d.n_in ? d.in_mask[i] : 0u;
      const uint32_t u = d.zbit[j];
      d.lsh[i][j] = (j < d.nl && ((m >> u) & 1u)) ? (uint8_t)__builtin_popcount(m & ((1u << u) - 1u)) : LSH_NONE;
    }
  return true;
}

// Bit split of an OP_ADJOINT op run by the outer-product executor
// (F_OUTER), for buckets whose inputs each lack a different part of the
// union, so that no group of loop bits suits the fused executor.  Lanes: the
// lowest union bits, as there.  The other bits are grouped by the set of
// outputs holding them.  The loop takes one group and the register slots
// one bit of another: an output lacking the loop bits sums over them in
// its slots, one lacking the slot bits adds its slots at each flush.  Among
// all such pairs the one whose outputs are left with the fewest partial sums
// to add with atomics (the block bits each output lacks, weighted by its
// size) is taken.  An output holding both loop and slot bits is flushed for
// every element, so it must sum lane bits only.  Loop length as in the fused
// rule.  Returns false when no pair qualifies or the block range is smaller
// than a workgroup step.
bool outer_adjoint_bits(OpDesc& d, int nbits, uint32_t all, const TuneParams& T0) {
  const TuneParams T = T0.for_bits(nbits);
  // complex64 only: with complex128 pairs the slots would lower the occupancy
  // of the whole persistent kernel
  if (T.elem_bytes != 8 || d.n_in < 3 || d.n_in > 4 || (d.in_mask[0] & 1u)) return false;
  d.adj_sel = 0;
  for (int i = 1; i < d.n_in; ++i) {
    if (!(d.in_mask[i] & 1u)) return false;
    d.adj_sel |= 1u << i;
  }
  const int max_lanes = std::min({T.lane_cap, 6, 31 - __builtin_clz((unsigned)std::max(T.threads, 1))});
  uint32_t lanes = 0;
  for (int u = 1; u < nbits && __builtin_popcount(lanes) < max_lanes; ++u) lanes |= 1u << u;
  std::map<uint32_t, uint32_t> groups;  // holders -> bits
  for (int u = 1; u < nbits; ++u) {
    if ((lanes >> u) & 1u) continue;
    uint32_t h = 0;
    for (int i = 1; i < d.n_in; ++i) h |= ((d.in_mask[i] >> u) & 1u) << i;
    groups[h] |= 1u << u;
  }
  const uint32_t outs = d.adj_sel;
  const int nl = __builtin_popcount(lanes);
  // the lowest bits of a group first (neighbouring elements)
  auto take = [](uint32_t bits, int n) {
    uint32_t r = 0;
    for (int u = 0; u < 32 && n > 0; ++u)
      if ((bits >> u) & 1u) {
        r |= 1u << u;
        --n;
      }
    return r;
  };
  double best = -1;
  uint32_t best_slot = 0, best_loop = 0;
  for (const auto& g2 : groups) {
    if (g2.first == outs) continue;  // every output holds it: nothing sums over it
    for (const auto& g1 : groups) {
      if (g1.first == g2.first || g1.first == outs) continue;
      bool ok = true;
      for (int i = 1; i < d.n_in; ++i)
        if (((g1.first & g2.first) >> i) & 1u)
          ok &= !(all & ~d.in_mask[i] & ~lanes & ~1u);
      if (!ok) continue;
      const int ki = 1;  // register budget of the persistent kernel
      const uint32_t slot = take(g1.second, ki);
      const int rest = nbits - 1 - nl - ki;  // loop and block bits
      const int loopable = __builtin_popcount(g2.second);
      int nk = std::max(0, std::min(loopable, rest - T.par_bits + nl));
      nk = std::min(nk, T.loop_cap);
      nk = std::max(nk, std::min(loopable, 3));
      if (nk < 1) continue;
      const uint32_t loop = take(g2.second, nk);
      const uint32_t blocks = all & ~1u & ~lanes & ~slot & ~loop;
      const int nb = __builtin_popcount(blocks);
      const int64_t nsub = std::max(1, T.threads >> nl);
      if (std::min<int64_t>(std::max(1, T.tile_blocks), int64_t(1) << nb) < nsub) continue;
      double cost = 0;  // partial sums written per output element, weighted by size
      for (int i = 1; i < d.n_in; ++i)
        cost += std::ldexp(1.0, __builtin_popcount(d.in_mask[i]) + __builtin_popcount(blocks & ~d.in_mask[i]));
      if (best < 0 || cost < best) {
        best = cost;
        best_slot = slot;
        best_loop = loop;
      }
    }
  }
  if (best < 0) return false;
  const int ki = __builtin_popcount(best_slot), nk = __builtin_popcount(best_loop);
  d.nl = nl;
  d.nu = ki;
  d.nk = nk;
  d.nb = nbits - 1 - nl - ki - nk;
  int z = 0;
  for (int u = 1; u < nbits; ++u)
    if ((lanes >> u) & 1u) d.zbit[z++] = (uint8_t)u;
  for (int u = 1; u < nbits; ++u)
    if ((best_slot >> u) & 1u) d.zbit[z++] = (uint8_t)u;
  for (int u = 1; u < nbits; ++u)
    if ((best_loop >> u) & 1u) d.zbit[z++] = (uint8_t)u;
  uint32_t blockbits = 0;
  for (int u = 1; u < nbits; ++u)
    if (!(((lanes | best_slot | best_loop) >> u) & 1u)) {
      d.zbit[z++] = (uint8_t)u;
      blockbits |= 1u << u;
    }
  for (; z < 32; ++z) d.zbit[z] = 0;
  bool atomic = false;
  for (int i = 1; i < d.n_in; ++i) atomic |= (blockbits & ~d.in_mask[i]) != 0;
  d.lane_sum = 0;
  d.out_mask = 0;
  d.out_off = 0;
  d.flags = F_WIDE | F_OUTER | (atomic ? F_ATOMIC : 0);
  for (int i = 0; i <= MAXIN; ++i)
    for (int j = 0; j < MAXLANE; ++j) {
      const uint32_t m = i < d.n_in ? d.in_mask[i] : 0u;
      const uint32_t u = d.zbit[j];
      d.lsh[i][j] = (j < d.nl && ((m >> u) & 1u)) ? (uint8_t)__builtin_popcount(m & ((1u << u) - 1u)) : LSH_NONE;
    }
  return true;
}

OpDesc blank(int kind, int cone) {
  OpDesc d;
  std::memset(&d, 0, sizeof(d));
  d.kind = kind;
  d.cone = cone;
  return d;
}

}  // namespace

// F_SYNC marks the ops of a cone program that must wait for the whole
// workgroup before they start, because they read or overwrite data written by
// an op since the previous barrier, or overwrite data read since then (dead
// buffers are reused).  Independent consecutive ops
// (e.g. the buckets of unrelated branches of the elimination tree) run
// without one.
static void mark_barriers(Plan& P) {
  struct Rng {
    int space;
    int64_t lo, hi;
  };
  auto overlaps = [](const std::vector<Rng>& v, const Rng& x) {
    for (const Rng& r : v)
      if (r.space == x.space && x.lo < r.hi && r.lo < x.hi) return true;
    return false;
  };
  auto run = [&](int32_t lo, int32_t hi, std::vector<Rng>& dirty, std::vector<Rng>& rdset) {
    for (int32_t o = lo; o < hi; ++o) {
      OpDesc& d = P.ops[o];
      std::vector<Rng> rd, wr;
      auto opnd = [&](int, int64_t goff, int64_t size) -> Rng { return {0, goff, goff + size}; };
      if (d.kind == OP_CONTRACT) {
        for (int i = 0; i < d.n_in; ++i)
          rd.push_back(opnd(i, d.in_off[i], int64_t(1) << __builtin_popcount(d.in_mask[i])));
        wr.push_back(opnd(MAXIN, d.out_off, int64_t(1) << __builtin_popcount(d.out_mask)));
      } else if (d.kind == OP_ADJOINT) {
        for (int i = 0; i < d.n_in; ++i) {
          const int64_t sz = int64_t(1) << __builtin_popcount(d.in_mask[i]);
          rd.push_back({0, d.in_off[i], d.in_off[i] + sz});
          if ((d.adj_sel >> i) & 1u) wr.push_back({0, d.adj_off[i], d.adj_off[i] + sz});
        }
      } else if (d.kind == OP_RESULT) {
        for (int i = 0; i < d.n_in; ++i) rd.push_back(opnd(i, d.in_off[i], 1));
        if (d.flags & F_GRAD)
          for (int i = 0; i < d.n_in; ++i) wr.push_back(opnd(d.n_in + i, d.in_off[d.n_in + i], 1));
      } else if (d.kind == OP_ZERO) {
        wr.push_back({0, d.out_off, d.out_off + d.in_off[0]});
      }
      bool need = false;
      for (const Rng& r : rd) need |= overlaps(dirty, r);
      for (const Rng& r : wr) need |= overlaps(dirty, r) || overlaps(rdset, r);
      if (need) {
        d.flags |= F_SYNC;
        dirty.clear();
        rdset.clear();
      } else {
        d.flags &= ~F_SYNC;
      }
      dirty.insert(dirty.end(), wr.begin(), wr.end());
      rdset.insert(rdset.end(), rd.begin(), rd.end());
    }
  };
  for (size_t c = 0; c < P.cones.size(); ++c) {
    std::vector<Rng> dirty, rdset;
    run(P.cone_fwd_lo[c], P.cone_fwd_hi[c] + 1, dirty, rdset);  // forward program ends with its result op
    dirty.clear();
    rdset.clear();
    run(P.cone_fwd_lo[c], P.cone_fwd_hi[c], dirty, rdset);  // gradient program: forward ops, then the adjoint range
    run(P.cone_adj_lo[c], P.cone_adj_hi[c], dirty, rdset);
  }
}

namespace {

// One cone's programs with buffer codes as operands.
struct ConeProg {
  std::vector<OpDesc> fwd, adj, leaf, lgrad;
  OpDesc result;
};

int64_t buf_size(const Cone& C, int64_t code) {
  const Bucket& B = C.buckets[code_bucket(code)];
  switch (code_kind(code)) {
    case BK_LAM:
    case BK_LAMADJ: return int64_t(1) << B.lam_rank();
    default: return std::max<int64_t>(int64_t(1) << B.out_rank(), 2);
  }
}

// Forward program (leaf tables, buckets in elimination order, result) and
// adjoint program (result with seeds, buckets in reverse order: the adjoint of
// every intermediate input and of the leaf-product table; recomputation of
// dropped outputs right before they are needed; zeroing right before ops
// that accumulate).  The paper defines the forward contraction (Section
// III.B); the adjoint is the reverse sweep of the same buckets.
std::string emit_cone(Plan& P, size_t c, ConeProg& G) {
  Cone& C = P.cones[c];
  const TuneParams& T = P.tune;
  const int eb = T.elem_bytes;
  G = ConeProg();
  if (C.width > MAXBITS - 1) return "contraction width " + std::to_string(C.width) + " exceeds 30";
  if (C.scalars.size() > MAXIN / 2) return "more than 4 disconnected components in one light cone";
  const size_t nb = C.buckets.size();
  if (C.recompute.size() != nb) C.recompute.assign(nb, 0);
  C.fwd_bytes_alg = C.bwd_bytes_alg = C.fwd_flops = C.rec_bytes = 0;
  std::vector<int32_t> ref_lo(nb, -1), ref_n(nb, 0);
  for (size_t b = 0; b < nb; ++b) {
    const Bucket& Bk = C.buckets[b];
    if (!Bk.lam_mask) continue;
    OpDesc d = blank(OP_LEAF, (int)c);
    d.nbits = Bk.lam_rank();
    d.out_off = buf_code(BK_LAM, (int)b);
    d.aux0 = (int32_t)P.leafrefs.size();
    for (int li : Bk.leaves) {
      const Leaf& l = C.leaves[li];
      auto lbit = [&](int idx) {
        int u = 0;
        while (Bk.uni[u] != idx) ++u;
        return __builtin_popcount(Bk.lam_mask & ((1u << u) - 1));
      };
      LeafRef r;
      r.kind = (int16_t)l.kind;
      r.pa = (int8_t)lbit(l.a);
      r.pb = (int8_t)(l.b >= 0 ? lbit(l.b) : -1);
      P.leafrefs.push_back(r);
    }
    // leaves of one angle next to each other: the leaf gradient sums them
    // before its single atomic per angle
    std::stable_sort(P.leafrefs.begin() + d.aux0, P.leafrefs.end(),
                     [](const LeafRef& a, const LeafRef& b) { return a.kind < b.kind; });
    d.aux1 = (int32_t)P.leafrefs.size() - d.aux0;
    ref_lo[b] = d.aux0;
    ref_n[b] = d.aux1;
    G.leaf.push_back(d);
  }
  // inputs [from, n_in) without the eliminated index (bit 0) first, the
  // order the wide executor takes them in (single elements, then pairs)
  auto singles_first = [](OpDesc& d, int from) {
    int64_t off[MAXIN];
    uint32_t msk[MAXIN];
    int k = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int i = from; i < d.n_in; ++i)
        if (bool(d.in_mask[i] & 1u) == bool(pass)) {
          off[k] = d.in_off[i];
          msk[k] = d.in_mask[i];
          ++k;
        }
    for (int i = from; i < d.n_in; ++i) {
      d.in_off[i] = off[i - from];
      d.in_mask[i] = msk[i - from];
    }
  };
  // forward contraction of bucket b, writing `out` (its output or a
  // recomputation, which reads the recomputed values of inputs that were
  // dropped too)
  auto fwd_op = [&](size_t b, int64_t out, double* bytes, double* flops) -> OpDesc {
    const Bucket& Bk = C.buckets[b];
    const int nbits = Bk.nbits();
    const bool rec = code_kind(out) == BK_REC;
    OpDesc d = blank(OP_CONTRACT, (int)c);
    d.nbits = nbits;
    int ni = 0;
    double in_elems = 0;
    for (size_t t = 0; t < Bk.in_bkt.size(); ++t) {
      const int pb = Bk.in_bkt[t];
      d.in_off[ni] = buf_code(rec && C.recompute[pb] ? BK_REC : BK_OUT, pb);
      d.in_mask[ni] = Bk.in_mask[t];
      in_elems += std::ldexp(1.0, __builtin_popcount(Bk.in_mask[t]));
      ++ni;
    }
    if (Bk.lam_mask) {
      d.in_off[ni] = buf_code(BK_LAM, (int)b);
      d.in_mask[ni] = Bk.lam_mask;
      ++ni;
    }
    d.n_in = ni;
    singles_first(d, 0);
    d.out_mask = ((nbits >= 32 ? 0u : (1u << nbits)) - 1u) & ~Bk.elim_mask();
    d.out_off = out;
    partition_bits(d, nbits, d.out_mask, nbits <= T.seq_max_bits, T);
    const double outn = std::ldexp(1.0, Bk.out_rank());
    if (bytes) *bytes += (in_elems + outn) * eb;
    if (flops) *flops += 6.0 * std::max(0, ni - 1) * std::ldexp(1.0, nbits) + 2.0 * outn;
    return d;
  };
  // an op whose partial sums meet in atomics (summed bits among its block
  // bits: merged steps split across work items) needs a zeroed output
  auto push_zeroed = [&](std::vector<OpDesc>& prog, const OpDesc& d) {
    if (d.flags & F_ATOMIC) {
      OpDesc z = blank(OP_ZERO, (int)c);
      z.out_off = d.out_off;
      z.in_off[0] = int64_t(1) << __builtin_popcount(d.out_mask);
      prog.push_back(z);
    }
    prog.push_back(d);
  };
  for (size_t b = 0; b < nb; ++b) {
    const Bucket& Bk = C.buckets[b];
    if (Bk.in_bkt.size() + (Bk.lam_mask ? 1 : 0) > (size_t)MAXIN) return "bucket with more than 8 inputs";
    push_zeroed(G.fwd, fwd_op(b, buf_code(BK_OUT, (int)b), &C.fwd_bytes_alg, &C.fwd_flops));
  }
  G.result = blank(OP_RESULT, (int)c);
  G.result.n_in = (int)C.scalars.size();
  for (size_t s = 0; s < C.scalars.size(); ++s) {
    G.result.in_off[s] = buf_code(BK_OUT, C.scalars[s]);
    G.result.in_off[C.scalars.size() + s] = buf_code(BK_ADJ, C.scalars[s]);
  }
  OpDesc rg = G.result;
  rg.flags = F_GRAD;
  G.adj.push_back(rg);
  // a dropped output is recomputed once, right before its first use in the
  // adjoint sweep, after the dropped outputs it reads (recursively); the
  // recomputed value then lives until its last use
  std::vector<char> made(nb, 0);
  std::function<void(int)> ensure = [&](int b) {
    if (!C.recompute[b] || made[b]) return;
    for (int pb : C.buckets[b].in_bkt) ensure(pb);
    push_zeroed(G.adj, fwd_op(b, buf_code(BK_REC, b), &C.rec_bytes, nullptr));
    made[b] = 1;
  };
  for (size_t bb = nb; bb-- > 0;) {
    const Bucket& Bk = C.buckets[bb];
    const int nbits = Bk.nbits();
    const bool seq = nbits <= T.seq_max_bits;
    const uint32_t all = ((nbits >= 32 ? 0u : (1u << nbits)) - 1u);
    const int nin = (int)Bk.in_bkt.size();
    // inputs dropped after the forward sweep are recomputed before their use
    for (int t = 0; t < nin; ++t) ensure(Bk.in_bkt[t]);
    auto in_code = [&](int t) {
      const int pb = Bk.in_bkt[t];
      return buf_code(C.recompute[pb] ? BK_REC : BK_OUT, pb);
    };
    double stored = 0;
    for (int t = 0; t < nin; ++t) stored += std::ldexp(1.0, __builtin_popcount(Bk.in_mask[t]));
    C.bwd_bytes_alg += (std::ldexp(1.0, Bk.out_rank()) + stored) * eb;
    auto add_common = [&](OpDesc& d, int skip_t, bool with_lam) {
      int ni = 0;
      d.in_off[ni] = buf_code(BK_ADJ, (int)bb);
      d.in_mask[ni] = all & ~Bk.elim_mask();
      ++ni;
      if (with_lam && Bk.lam_mask) {
        d.in_off[ni] = buf_code(BK_LAM, (int)bb);
        d.in_mask[ni] = Bk.lam_mask;
        ++ni;
      }
      for (int t = 0; t < nin; ++t) {
        if (t == skip_t) continue;
        d.in_off[ni] = in_code(t);
        d.in_mask[ni] = Bk.in_mask[t];
        ++ni;
      }
      d.n_in = ni;
    };
    auto push_adj = [&](OpDesc& d) { push_zeroed(G.adj, d); };
    auto push_leafgrad = [&]() {
      OpDesc g = blank(OP_LEAFGRAD, (int)c);
      g.nbits = Bk.lam_rank();
      g.in_off[0] = buf_code(BK_LAMADJ, (int)bb);
      g.aux0 = ref_lo[bb];
      g.aux1 = ref_n[bb];
      G.lgrad.push_back(g);
    };
    if (!seq && T.fuse_adjoint) {
      OpDesc d = blank(OP_ADJOINT, (int)c);
      d.nbits = nbits;
      add_common(d, -1, true);
      if (fused_adjoint_bits(d, nbits, all, T) || (T.fuse_adjoint == 3 && outer_adjoint_bits(d, nbits, all, T)) ||
          (T.fuse_adjoint == 2 && tile_adjoint_bits(d, nbits, all, T))) {
        int i = 1;
        if (Bk.lam_mask) d.adj_off[i++] = buf_code(BK_LAMADJ, (int)bb);
        for (int t = 0; t < nin; ++t) d.adj_off[i++] = buf_code(BK_ADJ, Bk.in_bkt[t]);
        // outputs summed with atomics (those that sum a block bit) start from zero
        uint32_t blockbits = 0;
        for (int q = d.nl + d.nu + d.nk; q < nbits - 1; ++q) blockbits |= 1u << d.zbit[q];
        for (int k = 1; k < d.n_in; ++k)
          if (blockbits & ~d.in_mask[k]) {
            OpDesc z = blank(OP_ZERO, (int)c);
            z.out_off = d.adj_off[k];
            z.in_off[0] = int64_t(1) << __builtin_popcount(d.in_mask[k]);
            G.adj.push_back(z);
          }
        G.adj.push_back(d);
        for (int t = 0; t < nin; ++t) C.bwd_bytes_alg += std::ldexp(1.0, __builtin_popcount(Bk.in_mask[t])) * eb;
        if (Bk.lam_mask) push_leafgrad();
        continue;
      }
    }
    for (int t = 0; t < nin; ++t) {
      OpDesc d = blank(OP_CONTRACT, (int)c);
      d.nbits = nbits;
      add_common(d, t, true);
      if (d.n_in > MAXIN) return "adjoint op with more than 8 inputs";
      singles_first(d, 1);
      d.out_mask = Bk.in_mask[t];
      d.out_off = buf_code(BK_ADJ, Bk.in_bkt[t]);
      partition_bits(d, nbits, d.out_mask, seq, T);
      push_adj(d);
      C.bwd_bytes_alg += std::ldexp(1.0, __builtin_popcount(Bk.in_mask[t])) * eb;
    }
    if (Bk.lam_mask) {
      OpDesc d = blank(OP_CONTRACT, (int)c);
      d.nbits = nbits;
      add_common(d, -1, false);
      if (d.n_in > MAXIN) return "adjoint op with more than 8 inputs";
      singles_first(d, 1);
      d.out_mask = Bk.lam_mask;
      d.out_off = buf_code(BK_LAMADJ, (int)bb);
      partition_bits(d, nbits, d.out_mask, seq, T);
      push_adj(d);
      push_leafgrad();
    }
  }
  return "";
}

// Lifetimes over the gradient program and first-fit placement.  Arena of a
// cone: [leaf tables][their adjoints][everything else, reused by lifetime].
int64_t alloc_cone(Cone& C, const ConeProg& G) {
  std::unordered_map<int64_t, size_t> idx;
  C.bufs.clear();
  auto touch = [&](int64_t code, int t) {
    if (!is_code(code)) return;
    auto it = idx.find(code);
    if (it == idx.end()) {
      idx[code] = C.bufs.size();
      BufLife B;
      B.code = code;
      B.size = buf_size(C, code);
      B.def = B.last = t;
      C.bufs.push_back(B);
    } else {
      C.bufs[it->second].last = std::max(C.bufs[it->second].last, t);
    }
  };
  auto scan = [&](const OpDesc& d, int t) {
    switch (d.kind) {
      case OP_CONTRACT:
        for (int i = 0; i < d.n_in; ++i) touch(d.in_off[i], t);
        touch(d.out_off, t);
        break;
      case OP_ADJOINT:
        for (int i = 0; i < d.n_in; ++i) {
          touch(d.in_off[i], t);
          if ((d.adj_sel >> i) & 1u) touch(d.adj_off[i], t);
        }
        break;
      case OP_RESULT:
        for (int i = 0; i < 2 * d.n_in; ++i) touch(d.in_off[i], t);
        break;
      case OP_ZERO: touch(d.out_off, t); break;
      case OP_LEAF: touch(d.out_off, t); break;
      case OP_LEAFGRAD: touch(d.in_off[0], t); break;
      default: break;
    }
  };
  int t = 0;
  for (const OpDesc& d : G.leaf) scan(d, t);
  for (const OpDesc& d : G.fwd) scan(d, ++t);
  scan(G.result, ++t);  // forward-only result: same position as the seeding result
  for (const OpDesc& d : G.adj) scan(d, t++);
  for (const OpDesc& d : G.lgrad) scan(d, t);
  // pinned blocks
  int64_t off = 0;
  for (BufLife& B : C.bufs)
    if (code_kind(B.code) == BK_LAM) {
      off = align_elems(off, B.size);
      B.off = off;
      off += B.size;
    }
  const int64_t lam_size = off;
  off = align_elems(off, 64);
  for (BufLife& B : C.bufs)
    if (code_kind(B.code) == BK_LAMADJ) {
      off = align_elems(off, B.size);
      B.off = off;
      off += B.size;
    }
  const int64_t base0 = align_elems(off, 64);
  C.dyn_start = base0;
  std::vector<size_t> order;
  for (size_t i = 0; i < C.bufs.size(); ++i) {
    const int k = code_kind(C.bufs[i].code);
    if (k != BK_LAM && k != BK_LAMADJ) order.push_back(i);
  }
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return C.bufs[a].def < C.bufs[b].def; });
  int64_t peak = base0;
  std::vector<size_t> live;
  for (size_t bi : order) {
    BufLife& B = C.bufs[bi];
    live.erase(std::remove_if(live.begin(), live.end(), [&](size_t x) { return C.bufs[x].last < B.def; }),
               live.end());
    std::vector<std::pair<int64_t, int64_t>> used;
    for (size_t x : live) used.push_back({C.bufs[x].off, C.bufs[x].off + C.bufs[x].size});
    std::sort(used.begin(), used.end());
    const int64_t al = B.size >= 64 ? 64 : 2;
    int64_t cand = base0;
    for (auto& u : used) {
      if (cand + B.size <= u.first) break;
      cand = std::max(cand, align_elems(u.second, al >= 64 ? B.size : 2));
    }
    B.off = cand;
    peak = std::max(peak, cand + B.size);
    live.push_back(bi);
  }
  C.lam_size = lam_size;
  C.arena_elems = align_elems(peak, 64);
  return C.arena_elems;
}

// Absolute arena offset of a coded operand: a leaf table or its adjoint in
// the cone's pinned part, anything else in its dynamic region.
int64_t resolve_off(const Plan& P, const Cone& C, const std::unordered_map<int64_t, int64_t>& where, int64_t v) {
  if (!is_code(v)) return v;
  const int64_t off = where.at(v);
  const int k = code_kind(v);
  if (k == BK_LAM || k == BK_LAMADJ) return C.base + off;
  return P.dyn_off + C.dyn_base + (off - C.dyn_start);
}

}  // namespace

// LDS-resident light cones.  When every step of a cone's gradient program is
// narrow and its tensors fit the LDS window, the batched sweep runs the whole
// program in one workgroup with every intermediate in LDS, from compact
// SmallOps: the cone's leaf-product block (built by the leaf launch) is copied
// in first, the adjoints of the leaf tables go straight to global memory (the
// leaf-gradient launch reads them there), and every other tensor stays in LDS.
// Buffers are placed first-fit by lifetime over that program, after the leaf
// block (the forward-only program is its prefix with a plain result, so the
// same placement serves it).  Ops between two barriers are independent of each
// other: each is given to one wavefront of the workgroup (balanced by size),
// so a workgroup of several wavefronts runs them side by side.  The per-op
// programs stay in P.ops for the plain per-op path.
static void small_programs(Plan& P, const std::vector<ConeProg>& progs) {
  const TuneParams& T = P.tune;
  const size_t nc = P.cones.size();
  const int64_t budget = (int64_t)T.lds_kb * 1024 / std::max(1, T.elem_bytes);
  const int nwaves = std::max(1, T.lds_threads / 64);
  P.cone_lds.assign(nc, 0);
  P.small.clear();
  P.small_fwd_lo.assign(nc, 0);
  P.small_fwd_hi.assign(nc, 0);
  P.small_grad_lo.assign(nc, 0);
  P.small_grad_hi.assign(nc, 0);
  P.lds_elems = 0;
  if (budget <= 0) return;
  for (size_t c = 0; c < nc; ++c) {
    const Cone& C = P.cones[c];
    const ConeProg& G = progs[c];
    std::unordered_map<int64_t, int64_t> goff;  // arena offsets (relative to the cone) of its buffers
    for (const BufLife& B : C.bufs) goff[B.code] = B.off;
    // gradient program: forward steps, the seeding result, adjoint steps
    std::vector<const OpDesc*> prog;
    bool ok = C.lam_size <= budget;
    for (const OpDesc& d : G.fwd) prog.push_back(&d);
    const size_t fwd_end = prog.size();
    for (const OpDesc& d : G.adj) prog.push_back(&d);
    for (const OpDesc* d : prog) {
      if (d->kind == OP_CONTRACT) {
        ok = ok && d->nbits <= 15 && d->nbits <= T.seq_max_bits && d->n_in <= 8 && !(d->flags & F_ATOMIC);
        for (int i = 0; i < d->n_in; ++i) ok = ok && is_code(d->in_off[i]) && code_kind(d->in_off[i]) != BK_LAMADJ;
        ok = ok && is_code(d->out_off) && code_kind(d->out_off) != BK_LAM;
      } else if (d->kind != OP_RESULT) {
        ok = false;  // zeroing, fused adjoints: wide steps
      }
    }
    if (!ok) continue;
    auto gout = [&](int64_t code) { return code_kind(code) == BK_LAMADJ; };
    // lifetimes over the program; the leaf block sits at LDS offset 0 as in the arena
    struct L {
      int64_t size;
      int def = -1, last = -1;
      int64_t off = -1;
    };
    std::unordered_map<int64_t, L> bufs;
    auto touch = [&](int64_t code, int t) {
      if (code_kind(code) == BK_LAM || gout(code)) return;
      L& B = bufs[code];
      if (B.def < 0) {
        B.def = t;
        B.size = int64_t(1) << C.buckets[code_bucket(code)].out_rank();
      }
      B.last = std::max(B.last, t);
    };
    for (size_t t = 0; t < prog.size(); ++t) {
      const OpDesc& d = *prog[t];
      if (d.kind == OP_CONTRACT) {
        for (int i = 0; i < d.n_in; ++i) touch(d.in_off[i], (int)t);
        touch(d.out_off, (int)t);
      } else if (d.kind == OP_RESULT) {
        for (int i = 0; i < 2 * d.n_in; ++i) touch(d.in_off[i], (int)t);
      }
    }
    std::vector<int64_t> order;
    for (auto& kv : bufs) order.push_back(kv.first);
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return bufs[a].def != bufs[b].def ? bufs[a].def < bufs[b].def : a < b;
    });
    const int64_t base0 = C.lam_size;
    int64_t peak = base0;
    std::vector<int64_t> live;
    for (int64_t code : order) {
      L& B = bufs[code];
      live.erase(std::remove_if(live.begin(), live.end(), [&](int64_t x) { return bufs[x].last < B.def; }),
                 live.end());
      std::vector<std::pair<int64_t, int64_t>> used;
      for (int64_t x : live) used.push_back({bufs[x].off, bufs[x].off + bufs[x].size});
      std::sort(used.begin(), used.end());
      int64_t cand = base0;
      for (auto& u : used) {
        if (cand + B.size <= u.first) break;
        cand = std::max(cand, u.second);
      }
      B.off = cand;
      peak = std::max(peak, cand + B.size);
      live.push_back(code);
    }
    if (peak > budget || peak > 65535) continue;
    auto lds = [&](int64_t code) -> uint16_t {
      return (uint16_t)(code_kind(code) == BK_LAM ? goff.at(code) : bufs.at(code).off);
    };
    struct Rng {
      int64_t lo, hi;
    };
    auto range = [&](int64_t code) -> Rng {
      if (code_kind(code) == BK_LAM) {
        const int64_t o = goff.at(code);
        return {o, o + (int64_t(1) << C.buckets[code_bucket(code)].lam_rank())};
      }
      return {bufs.at(code).off, bufs.at(code).off + bufs.at(code).size};
    };
    auto emit = [&](const OpDesc& d, bool grad_result) {
      SmallOp s;
      std::memset(&s, 0, sizeof(s));
      s.cone = (int32_t)c;
      if (d.kind == OP_CONTRACT) {
        s.kind = S_CONTRACT;
        s.n_in = (uint8_t)d.n_in;
        s.nbits = (uint8_t)d.nbits;
        s.n_out = (uint8_t)__builtin_popcount(d.out_mask);
        // dimensions: output bits, then summed bits, each in union order
        int dims[16], nd = 0;
        for (int u = 0; u < d.nbits; ++u)
          if ((d.out_mask >> u) & 1u) dims[nd++] = u;
        for (int u = 0; u < d.nbits; ++u)
          if (!((d.out_mask >> u) & 1u)) dims[nd++] = u;
        for (int i = 0; i < d.n_in; ++i) {
          uint64_t sh = ~uint64_t(0);
          for (int j = 0; j < nd; ++j)
            if ((d.in_mask[i] >> dims[j]) & 1u) {
              const uint64_t r = (uint64_t)__builtin_popcount(d.in_mask[i] & ((1u << dims[j]) - 1u));
              sh &= ~(uint64_t(0xf) << (4 * j));
              sh |= r << (4 * j);
            }
          s.shift[i] = sh;
          s.in_off[i] = lds(d.in_off[i]);
        }
        if (gout(d.out_off)) {
          s.flags |= SF_GOUT;
          s.gout = C.base + goff.at(d.out_off);
        } else {
          s.out_off = lds(d.out_off);
        }
      } else {  // OP_RESULT
        s.kind = S_RESULT;
        s.n_in = (uint8_t)d.n_in;
        for (int i = 0; i < d.n_in; ++i) s.in_off[i] = lds(d.in_off[i]);
        if (grad_result) {
          s.flags |= SF_GRAD;
          for (int i = 0; i < d.n_in; ++i) s.in_off[4 + i] = lds(d.in_off[d.n_in + i]);
        }
      }
      return s;
    };
    // one program: the leaf-block copy, then the ops; barriers from the LDS
    // read / write sets since the last one; the ops of one stage (between
    // barriers) spread over the wavefronts, largest first onto the least loaded
    auto emit_range = [&](const std::vector<std::pair<const OpDesc*, bool>>& ops) {
      SmallOp cp;
      std::memset(&cp, 0, sizeof(cp));
      cp.kind = S_COPYIN;
      cp.cone = (int32_t)c;
      cp.gout = C.lam_base;
      cp.aux1 = (int32_t)C.lam_size;
      P.small.push_back(cp);
      std::vector<Rng> dirty, rdset;
      auto hit = [](const std::vector<Rng>& v, const Rng& x) {
        for (const Rng& r : v)
          if (x.lo < r.hi && r.lo < x.hi) return true;
        return false;
      };
      dirty.push_back({0, C.lam_size});  // the copy-in
      std::vector<size_t> stage;         // indices into P.small of the open stage
      auto close_stage = [&]() {
        std::vector<double> load(nwaves, 0.0);
        std::vector<size_t> by_size(stage);
        auto cost = [&](size_t k) {
          const SmallOp& o = P.small[k];
          return o.kind == S_CONTRACT ? std::ldexp(1.0, o.nbits) * o.n_in + 256.0 : 64.0;
        };
        std::stable_sort(by_size.begin(), by_size.end(), [&](size_t a, size_t b) { return cost(a) > cost(b); });
        // the stage's largest op is shared by every wavefront when it costs
        // more than the others together and its outer output walk has at
        // least two steps (more than 64 output elements)
        size_t first = 0;
        if (nwaves > 1 && !by_size.empty()) {
          SmallOp& o = P.small[by_size[0]];
          double rest = 0;
          for (size_t i = 1; i < by_size.size(); ++i) rest += cost(by_size[i]);
          if (o.kind == S_CONTRACT && o.n_out >= 7 && cost(by_size[0]) > rest) {
            o.flags |= SF_SPLIT;
            o.wave = 0;
            // the executor's split: contiguous chunks of the 2^(n_out-6) outer steps
            const int nouter = 1 << (o.n_out - 6), chunk = (nouter + nwaves - 1) / nwaves;
            for (int w = 0; w < nwaves; ++w) {
              const int h0 = std::min(nouter, w * chunk), h1 = std::min(nouter, h0 + chunk);
              load[w] += cost(by_size[0]) * (h1 - h0) / nouter;
            }
            first = 1;
          }
        }
        for (size_t i = first; i < by_size.size(); ++i) {
          const size_t k = by_size[i];
          const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
          P.small[k].wave = (uint8_t)w;
          load[w] += cost(k);
        }
        stage.clear();
      };
      for (auto& pr : ops) {
        const OpDesc& d = *pr.first;
        std::vector<Rng> rd, wr;
        if (d.kind == OP_CONTRACT) {
          for (int i = 0; i < d.n_in; ++i) rd.push_back(range(d.in_off[i]));
          if (!gout(d.out_off)) wr.push_back(range(d.out_off));
        } else {
          for (int i = 0; i < d.n_in; ++i) rd.push_back(range(d.in_off[i]));
          if (pr.second)
            for (int i = 0; i < d.n_in; ++i) wr.push_back(range(d.in_off[d.n_in + i]));
        }
        bool need = false;
        for (const Rng& r : rd) need |= hit(dirty, r);
        for (const Rng& r : wr) need |= hit(dirty, r) || hit(rdset, r);
        SmallOp so = emit(d, pr.second);
        if (need) {
          close_stage();
          so.flags |= SF_SYNC;
          dirty.clear();
          rdset.clear();
        }
        dirty.insert(dirty.end(), wr.begin(), wr.end());
        rdset.insert(rdset.end(), rd.begin(), rd.end());
        stage.push_back(P.small.size());
        P.small.push_back(so);
      }
      close_stage();
    };
    std::vector<std::pair<const OpDesc*, bool>> fwd, grad;
    for (size_t t = 0; t < fwd_end; ++t) fwd.push_back({prog[t], false});
    fwd.push_back({&G.result, false});
    for (size_t t = 0; t < prog.size(); ++t) grad.push_back({prog[t], prog[t]->kind == OP_RESULT});
    P.small_fwd_lo[c] = (int32_t)P.small.size();
    emit_range(fwd);
    P.small_fwd_hi[c] = (int32_t)P.small.size();
    P.small_grad_lo[c] = (int32_t)P.small.size();
    emit_range(grad);
    P.small_grad_hi[c] = (int32_t)P.small.size();
    P.cone_lds[c] = 1;
    P.lds_elems = std::max(P.lds_elems, peak);
  }
}

static bool admit_cones(Plan& P, int64_t area);

std::string build_programs(Plan& P, int elem_bytes) {
  P.tune.elem_bytes = elem_bytes;
  P.ops.clear();
  P.leafrefs.clear();
  const size_t nc = P.cones.size();
  P.cone_fwd_lo.assign(nc, 0);
  P.cone_fwd_hi.assign(nc, 0);
  P.cone_adj_lo.assign(nc, 0);
  P.cone_adj_hi.assign(nc, 0);
  std::vector<ConeProg> progs(nc);
  int64_t total = 0;
  for (size_t c = 0; c < nc; ++c) {
    group_buckets(P.cones[c], P.tune.merge_bits, P.tune.merge_lam_bits);
    P.cones[c].recompute.assign(P.cones[c].buckets.size(), 0);
    std::string err = emit_cone(P, c, progs[c]);
    if (!err.empty()) return err;
    total += alloc_cone(P.cones[c], progs[c]);
    P.cones[c].keep_all_elems = P.cones[c].arena_elems;
  }
  // memory budget: every cone's pinned part (leaf tables and their
  // adjoints, written before and read after the sweep) side by side, the
  // dynamic regions in a shared area that the batched sweep admits cones
  // into; a cone whose dynamic region alone exceeds the area drops bucket
  // outputs after the forward sweep (largest first, kept when the region
  // shrinks) and recomputes them in the adjoint sweep
  int64_t pinned = 0;
  for (size_t c = 0; c < nc; ++c) pinned += align_elems(P.cones[c].dyn_start, 64);
  const int64_t area = P.mem_budget > 0 ? P.mem_budget - align_elems(pinned, 64) : 0;
  if (P.mem_budget > 0) {
    if (area <= 0) return "the memory budget does not hold the leaf tables";
    for (size_t c = 0; c < nc; ++c) {
      Cone& C = P.cones[c];
      if (C.arena_elems - C.dyn_start <= area) continue;
      std::vector<int> cand;
      for (size_t b = 0; b < C.buckets.size(); ++b)
        if (C.buckets[b].consumer >= 0 && C.buckets[b].out_rank() >= 4) cand.push_back((int)b);
      std::stable_sort(cand.begin(), cand.end(),
                       [&](int a, int b) { return C.buckets[a].out_rank() > C.buckets[b].out_rank(); });
      for (int b : cand) {
        if (C.arena_elems - C.dyn_start <= area) break;
        const int64_t before = C.arena_elems;
        C.recompute[b] = 1;
        std::string err = emit_cone(P, c, progs[c]);
        if (!err.empty()) return err;
        alloc_cone(C, progs[c]);
        if (C.arena_elems >= before) {  // no gain: keep the output
          C.recompute[b] = 0;
          err = emit_cone(P, c, progs[c]);
          if (!err.empty()) return err;
          alloc_cone(C, progs[c]);
        }
      }
      if (C.arena_elems - C.dyn_start > area)
        return "the gradient sweep does not fit the memory budget even with recomputation";
    }
  }
  // assemble the op list (operands still coded)
  std::vector<OpDesc> leaf_ops, lgrad_ops;
  for (size_t c = 0; c < nc; ++c) {
    ConeProg& G = progs[c];
    P.cone_fwd_lo[c] = (int32_t)P.ops.size();
    P.ops.insert(P.ops.end(), G.fwd.begin(), G.fwd.end());
    P.cone_fwd_hi[c] = (int32_t)P.ops.size();
    P.ops.push_back(G.result);
    P.cone_adj_lo[c] = (int32_t)P.ops.size();
    P.ops.insert(P.ops.end(), G.adj.begin(), G.adj.end());
    P.cone_adj_hi[c] = (int32_t)P.ops.size();
    leaf_ops.insert(leaf_ops.end(), G.leaf.begin(), G.leaf.end());
    lgrad_ops.insert(lgrad_ops.end(), G.lgrad.begin(), G.lgrad.end());
  }
  P.leaf_lo = (int32_t)P.ops.size();
  P.ops.insert(P.ops.end(), leaf_ops.begin(), leaf_ops.end());
  P.leaf_hi = (int32_t)P.ops.size();
  P.lgrad_lo = P.leaf_hi;
  // leaf gradients of tables with at most 8 leaves first: they run in a
  // kernel of their own whose smaller register footprint fits more
  // wavefronts per SIMD
  std::stable_partition(lgrad_ops.begin(), lgrad_ops.end(), [](const OpDesc& d) { return d.aux1 <= 8; });
  P.ops.insert(P.ops.end(), lgrad_ops.begin(), lgrad_ops.end());
  P.lgrad_hi = (int32_t)P.ops.size();
  P.lgrad_mid = P.lgrad_lo;
  while (P.lgrad_mid < P.lgrad_hi && P.ops[P.lgrad_mid].aux1 <= 8) ++P.lgrad_mid;
  // pinned parts side by side, then the dynamic area
  int64_t off = 0;
  for (size_t c = 0; c < nc; ++c) {
    Cone& C = P.cones[c];
    C.base = off;
    C.lam_base = off;
    off += align_elems(C.dyn_start, 64);
  }
  P.dyn_off = align_elems(off, 64);
  small_programs(P, progs);
  // dynamic regions: under a budget, placed by the admission schedule of the
  // batched sweep; else side by side.  LDS-resident cones use none in the
  // batched sweep (the plain path runs one cone at a time): offset 0.
  P.cone_pred.clear();
  int64_t dyn_end = 0;
  if (P.mem_budget > 0) {
    P.sched_workers = std::max(1, P.sched_workers);
    if (!admit_cones(P, area)) return "the gradient sweep does not fit the memory budget even with recomputation";
    for (size_t c = 0; c < nc; ++c)
      dyn_end = std::max(dyn_end, P.cones[c].dyn_base + P.cones[c].arena_elems - P.cones[c].dyn_start);
  } else {
    for (size_t c = 0; c < nc; ++c) {
      Cone& C = P.cones[c];
      const int64_t n = C.arena_elems - C.dyn_start;
      C.dyn_base = P.cone_lds[c] ? 0 : dyn_end;
      dyn_end = std::max(dyn_end, C.dyn_base + n);
      if (!P.cone_lds[c]) dyn_end = align_elems(dyn_end, 64);
    }
  }
  P.arena_grad = P.arena_fwd = align_elems(P.dyn_off + dyn_end, 64);
  // the LDS window also holds the tile sums of LDS-tiled adjoints
  for (const OpDesc& d : P.ops)
    if (d.kind == OP_ADJOINT && (d.flags & F_TILE)) P.lds_elems = std::max<int64_t>(P.lds_elems, d.aux0);
  {
    std::vector<std::unordered_map<int64_t, int64_t>> where(nc);
    for (size_t c = 0; c < nc; ++c)
      for (const BufLife& B : P.cones[c].bufs) where[c][B.code] = B.off;
    for (OpDesc& d : P.ops) {
      const Cone& C = P.cones[d.cone];
      const auto& W = where[d.cone];
      switch (d.kind) {
        case OP_CONTRACT:
          for (int i = 0; i < d.n_in; ++i) d.in_off[i] = resolve_off(P, C, W, d.in_off[i]);
          d.out_off = resolve_off(P, C, W, d.out_off);
          break;
        case OP_ADJOINT:
          for (int i = 0; i < d.n_in; ++i) {
            d.in_off[i] = resolve_off(P, C, W, d.in_off[i]);
            if ((d.adj_sel >> i) & 1u) d.adj_off[i] = resolve_off(P, C, W, d.adj_off[i]);
          }
          break;
        case OP_RESULT:
          for (int i = 0; i < 2 * d.n_in; ++i) d.in_off[i] = resolve_off(P, C, W, d.in_off[i]);
          break;
        case OP_ZERO:
        case OP_LEAF: d.out_off = resolve_off(P, C, W, d.out_off); break;
        case OP_LEAFGRAD: d.in_off[0] = resolve_off(P, C, W, d.in_off[0]); break;
        default: break;
      }
    }
  }
  mark_barriers(P);
  return "";
}

// Invariants of an OP_ADJOINT op that its executor relies on.
static std::string validate_adjoint_op(const Plan& P, const OpDesc& d) {
  const uint32_t all = (uint32_t)((uint64_t(1) << d.nbits) - 1);
  if (d.nbits <= P.tune.seq_max_bits || !(d.flags & F_WIDE)) return "adjoint op not wide";
  if (d.n_in < 3 || d.n_in > 4) return "adjoint op with a bad input count";
  const bool tiled = d.flags & F_TILE;
  const bool outer = d.flags & F_OUTER;
  if (tiled && outer) return "adjoint op both tiled and outer";
  if ((outer ? d.nu != 1 : d.nu != 0) || d.nl < 1 ||
      d.nl + d.nu + d.nk + d.nb != d.nbits - 1)
    return "adjoint op bit partition";
  if (outer && (d.nk < 1 || P.tune.elem_bytes != 8)) return "outer adjoint op without loop bits or not complex64";
  if (tiled ? (1 << d.nl) != P.tune.threads : d.nl > 6) return "adjoint op lane count";
  if (d.adj_sel != (((1u << d.n_in) - 1u) & ~1u)) return "adjoint op output selection";
  if ((d.in_mask[0] & 1u) || (d.in_mask[0] & ~all)) return "adjoint op output adjoint mask";
  for (int i = 1; i < d.n_in; ++i)
    if (!(d.in_mask[i] & 1u) || (d.in_mask[i] & ~all)) return "adjoint op input mask";
  uint32_t seen = 0, lanes = 0, slots = 0, loop = 0, blocks = 0;
  for (int z = 0; z < d.nbits - 1; ++z) {
    const uint32_t u = d.zbit[z];
    if (u < 1 || (int)u >= d.nbits || (seen >> u) & 1) return "adjoint op bad zbit";
    seen |= 1u << u;
    (z < d.nl ? lanes : z < d.nl + d.nu ? slots : z < d.nl + d.nu + d.nk ? loop : blocks) |= 1u << u;
  }
  bool atomic = false;
  int64_t tile_elems = 0;
  for (int i = 1; i < d.n_in; ++i) {
    const uint32_t held = d.in_mask[i] & loop;
    if (tiled) {
      if (d.in_mask[i] == all) return "LDS-tiled adjoint with an output holding the whole union";
      tile_elems += int64_t(2) << __builtin_popcount(d.in_mask[i] & (lanes | loop));
    } else if (outer) {
      if (held != 0 && held != loop) return "adjoint op output holds part of the loop bits";
      if (held && (d.in_mask[i] & slots) && (all & ~d.in_mask[i] & ~lanes & ~1u))
        return "outer adjoint op output flushed per element sums a non-lane bit";
    } else {
      if (held != 0 && held != loop) return "adjoint op output holds part of the loop bits";
      if (held && (all & ~d.in_mask[i] & ~lanes & ~1u)) return "adjoint op loop holder sums a non-lane bit";
    }
    atomic |= (blocks & ~d.in_mask[i]) != 0;
  }
  if (tiled && (tile_elems != d.aux0 || d.aux0 > P.lds_elems)) return "LDS-tiled adjoint tile size";
  if (atomic != bool(d.flags & F_ATOMIC)) return "adjoint op atomic flag mismatch";
  const int64_t nsub = std::max(1, P.tune.threads >> d.nl);
  if (std::min<int64_t>(std::max(1, P.tune.for_bits(d.nbits).tile_blocks), int64_t(1) << d.nb) < nsub)
    return "adjoint op block range smaller than a workgroup step";
  for (int i = 0; i < d.n_in; ++i) {
    const int64_t sz = int64_t(1) << __builtin_popcount(d.in_mask[i]);
    if (d.in_off[i] < 0 || d.in_off[i] + sz > P.arena_grad) return "adjoint op input range out of bounds";
    if (i > 0 && (d.adj_off[i] < 0 || d.adj_off[i] + sz > P.arena_grad)) return "adjoint op output out of bounds";
    if (i > 0 && (d.adj_off[i] & 1)) return "adjoint op output pair not aligned";
    for (int k = 0; k < d.n_in; ++k)
      if (k > 0 && d.adj_off[k] < d.in_off[i] + sz &&
          d.in_off[i] < d.adj_off[k] + (int64_t(1) << __builtin_popcount(d.in_mask[k])))
        return "adjoint op output overlaps an input";
    for (int j = 0; j < MAXLANE; ++j) {
      const uint32_t m = d.in_mask[i];
      const uint32_t st = j < d.nl && ((m >> d.zbit[j]) & 1) ? (1u << __builtin_popcount(m & ((1u << d.zbit[j]) - 1))) : 0u;
      const uint32_t got = d.lsh[i][j] == LSH_NONE ? 0u : (1u << d.lsh[i][j]);
      if (st != got) return "adjoint op lane shift table mismatch";
    }
  }
  return "";
}

// The wait structure of a stored work queue.  A cone's items, in queue
// order, form runs of equal op ranges (its segments; a wide op's items share
// one run).  Every run after a cone's first, and the first run of a cone that
// waits for other cones' memory, waits on one node; the items that release
// that node are exactly the preceding run (and the last runs of the cones it
// waits for), all earlier in the queue, and the node's initial count is their
// number.  Runs that wait on nothing have no releasing items.
static std::string validate_queue(const Plan& P, bool grad) {
  const auto& items = grad ? P.items_grad : P.items_fwd;
  const auto& init = grad ? P.node_init_grad : P.node_init_fwd;
  const auto& succ = grad ? P.succ_grad : P.succ_fwd;
  const std::string q = grad ? "gradient queue: " : "forward queue: ";
  const size_t nc = P.cones.size(), ni = items.size(), nn = init.size();
  std::vector<std::vector<int32_t>> rel(nn);  // items that release each node
  for (size_t i = 0; i < ni; ++i) {
    const QItem& I = items[i];
    if (I.op_lo < 0 || I.op_hi > (int32_t)P.ops.size() || I.op_lo >= I.op_hi) return q + "bad op range";
    if (I.succ_lo < 0 || I.succ_hi < I.succ_lo || I.succ_hi > (int32_t)succ.size()) return q + "bad successor range";
    for (int32_t s = I.succ_lo; s < I.succ_hi; ++s) {
      if (succ[s] < 0 || succ[s] >= (int32_t)nn) return q + "successor node out of range";
      rel[succ[s]].push_back((int32_t)i);
    }
    if (I.node < -1 || I.node >= (int32_t)nn) return q + "wait node out of range";
  }
  for (size_t n = 0; n < nn; ++n)
    if ((int32_t)rel[n].size() != init[n]) return q + "node " + std::to_string(n) + " count != releasing items";
  // runs per cone
  auto same_run = [](const QItem& a, const QItem& b) {
    return a.op_lo == b.op_lo && a.op_hi == b.op_hi && a.op2_lo == b.op2_lo && a.op2_hi == b.op2_hi;
  };
  std::vector<std::vector<std::vector<int32_t>>> runs(nc);
  for (size_t i = 0; i < ni; ++i) {
    auto& r = runs[P.ops[items[i].op_lo].cone];
    if (r.empty() || !same_run(items[r.back().back()], items[i])) r.emplace_back();
    r.back().push_back((int32_t)i);
  }
  const bool gated = P.cone_pred.size() == nc;
  for (size_t c = 0; c < nc; ++c) {
    for (size_t k = 0; k < runs[c].size(); ++k) {
      std::vector<int32_t> need;
      if (k > 0) need = runs[c][k - 1];
      if (k == 0 && gated)
        for (int a : P.cone_pred[c])
          if (!runs[a].empty()) need.insert(need.end(), runs[a].back().begin(), runs[a].back().end());
      const int32_t node = items[runs[c][k][0]].node;
      for (int32_t i : runs[c][k])
        if (items[i].node != node) return q + "items of one segment wait on different nodes";
      if (need.empty()) {
        if (node >= 0 && init[node] != 0) return q + "cone " + std::to_string(c) + " waits on unrelated items";
        continue;
      }
      if (node < 0) return q + "cone " + std::to_string(c) + " segment " + std::to_string(k) + " does not wait";
      std::vector<int32_t> got = rel[node];
      std::sort(got.begin(), got.end());
      std::sort(need.begin(), need.end());
      if (got != need) return q + "cone " + std::to_string(c) + " segment " + std::to_string(k) + " waits on the wrong items";
      if (need.back() >= runs[c][k][0]) return q + "an item waits on a later item";
    }
  }
  return "";
}

std::string validate_plan(const Plan& P) {
  auto S = [](auto... a) {
    std::string r;
    ((r += std::to_string(a), r += ' '), ...);
    return r;
  };
  struct Iv {
    int64_t lo, hi;
  };
  std::vector<Iv> iv;
  for (size_t c = 0; c < P.cones.size(); ++c) {
    const Cone& C = P.cones[c];
    const int n = C.n_idx;
    if ((int)C.order.size() != n) return "cone " + S(c) + "order length != index count";
    std::vector<int> pos(n, -1);
    for (int s = 0; s < n; ++s) {
      int v = C.order[s];
      if (v < 0 || v >= n || pos[v] >= 0) return "cone " + S(c) + "order is not a permutation";
      pos[v] = s;
    }
    const int nb = (int)C.buckets.size();
    std::vector<int> leaf_seen(C.leaves.size(), 0), consumed(nb, 0), elim_seen(n, 0);
    int width = 0;
    for (int b = 0; b < nb; ++b) {
      const Bucket& B = C.buckets[b];
      if (B.uni.empty() || B.n_elim < 1 || B.n_elim > (int)B.uni.size() || B.uni[0] != B.v)
        return "cone " + S(c, b) + "bucket index mismatch";
      if (B.nbits() > MAXBITS) return "cone " + S(c, b) + "union too wide";
      for (size_t t = 1; t < B.uni.size(); ++t)
        if (pos[B.uni[t]] <= pos[B.uni[t - 1]]) return "cone " + S(c, b) + "union not in elimination order";
      for (int q = 0; q < B.n_elim; ++q) elim_seen[B.uni[q]]++;
      if (b > 0 && pos[C.buckets[b - 1].uni[C.buckets[b - 1].n_elim - 1]] >= pos[B.uni[B.n_elim - 1]])
        return "cone " + S(c, b) + "steps not in elimination order";
      const uint32_t all = (uint32_t)((uint64_t(1) << B.uni.size()) - 1);
      uint32_t cover = 0;
      for (int li : B.leaves) {
        leaf_seen[li]++;
        const Leaf& L = C.leaves[li];
        for (int idx : {L.a, L.b}) {
          if (idx < 0) continue;
          auto it = std::find(B.uni.begin(), B.uni.end(), idx);
          if (it == B.uni.end()) return "cone " + S(c, b) + "leaf index outside the union";
          const uint32_t bit = 1u << (it - B.uni.begin());
          if (!(B.lam_mask & bit)) return "cone " + S(c, b) + "leaf bit missing from the leaf-product mask";
          cover |= bit;
        }
      }
      for (size_t t = 0; t < B.in_bkt.size(); ++t) {
        const int pb = B.in_bkt[t];
        if (pb < 0 || pb >= b) return "cone " + S(c, b) + "producer is not earlier";
        const Bucket& Pb = C.buckets[pb];
        if (Pb.consumer != b) return "cone " + S(c, b) + "producer's consumer mismatch";
        consumed[pb]++;
        uint32_t mk = 0;
        for (size_t q = Pb.n_elim; q < Pb.uni.size(); ++q) {
          auto it = std::find(B.uni.begin(), B.uni.end(), Pb.uni[q]);
          if (it == B.uni.end()) return "cone " + S(c, b) + "input index outside the union";
          mk |= 1u << (it - B.uni.begin());
        }
        if (mk != B.in_mask[t] || (mk & B.elim_mask()) == 0) return "cone " + S(c, b) + "input mask mismatch";
        cover |= mk;
      }
      if (cover != all) return "cone " + S(c, b) + "union larger than its inputs";
      width = std::max(width, B.out_rank());
      if ((B.out_rank() == 0) != (B.consumer == -1)) return "cone " + S(c, b) + "scalar / consumer mismatch";
    }
    for (size_t li = 0; li < C.leaves.size(); ++li)
      if (leaf_seen[li] != 1) return "cone " + S(c, li) + "leaf not absorbed exactly once";
    for (int v = 0; v < n; ++v)
      if (elim_seen[v] != 1) return "cone " + S(c, v) + "index not eliminated exactly once";
    for (int b = 0; b < nb; ++b)
      if ((C.buckets[b].consumer >= 0) != (consumed[b] == 1)) return "cone " + S(c, b) + "output not consumed once";
    if (width > C.width) return "cone " + S(c) + "width above the order's width";
    // arena placement: in the cone's region, and buffers alive at the same
    // time never overlap
    std::vector<const BufLife*> bl;
    for (const BufLife& B : C.bufs) {
      if (B.off < 0 || B.off + B.size > C.arena_elems) return "cone " + S(c) + "buffer outside the cone's arena";
      bl.push_back(&B);
    }
    std::sort(bl.begin(), bl.end(), [](const BufLife* a, const BufLife* b) { return a->def < b->def; });
    for (size_t i = 0; i < bl.size(); ++i)
      for (size_t j = i + 1; j < bl.size() && bl[j]->def <= bl[i]->last; ++j) {
        const BufLife& A = *bl[i];
        const BufLife& B = *bl[j];
        if (A.off < B.off + B.size && B.off < A.off + A.size)
          return "cone " + S(c) + "buffers with overlapping lifetimes share memory";
      }
    if (C.base < 0 || C.base + C.dyn_start > P.dyn_off) return "cone " + S(c) + "pinned part out of bounds";
    if (C.dyn_base < 0 || P.dyn_off + C.dyn_base + (C.arena_elems - C.dyn_start) > P.arena_grad)
      return "cone " + S(c) + "dynamic region out of bounds";
    iv.push_back({C.base, C.base + C.dyn_start});
  }
  // pinned parts never overlap; dynamic regions of cones run from the work
  // queue overlap only when one cone waits (through its predecessors) for the
  // other
  std::sort(iv.begin(), iv.end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
  for (size_t i = 1; i < iv.size(); ++i)
    if (iv[i].lo < iv[i - 1].hi) return "pinned parts of two cones overlap";
  {
    const size_t nc = P.cones.size();
    const bool gated = P.cone_pred.size() == nc;
    std::vector<std::vector<char>> anc;  // anc[c][a]: c waits for a, directly or not
    if (gated) {
      anc.assign(nc, std::vector<char>(nc, 0));
      std::vector<int> done(nc, 0);
      std::function<void(int)> visit = [&](int c) {
        if (done[c]) return;
        done[c] = 1;
        for (int a : P.cone_pred[c]) {
          if (a < 0 || a >= (int)nc || a == c) return;
          visit(a);
          anc[c][a] = 1;
          for (size_t x = 0; x < nc; ++x) anc[c][x] |= anc[a][x];
        }
      };
      for (size_t c = 0; c < nc; ++c) visit((int)c);
    }
    std::vector<std::pair<Iv, int>> dv;
    for (size_t c = 0; c < nc; ++c) {
      const Cone& C = P.cones[c];
      if (!P.cone_lds.empty() && P.cone_lds[c]) continue;
      if (C.arena_elems > C.dyn_start) dv.push_back({{C.dyn_base, C.dyn_base + C.arena_elems - C.dyn_start}, (int)c});
    }
    std::sort(dv.begin(), dv.end(), [](const std::pair<Iv, int>& a, const std::pair<Iv, int>& b) {
      return a.first.lo < b.first.lo;
    });
    for (size_t i = 0; i < dv.size(); ++i)
      for (size_t j = i + 1; j < dv.size() && dv[j].first.lo < dv[i].first.hi; ++j) {
        const int a = dv[i].second, b = dv[j].second;
        if (!gated || !(anc[a][b] || anc[b][a]))
          return "dynamic regions of cones " + S(a, b) + "overlap without an order between them";
      }
  }
  for (size_t o = 0; o < P.ops.size(); ++o) {
    const OpDesc& d = P.ops[o];
    if (d.kind == OP_ADJOINT) {
      const std::string e = validate_adjoint_op(P, d);
      if (!e.empty()) return "op " + S(o) + e;
      continue;
    }
    if (d.kind != OP_CONTRACT) continue;
    if (d.nl + d.nu + d.nk + d.nb != d.nbits - 1) return "op " + S(o) + "bit partition does not cover the union";
    if (d.flags & F_WIDE) {
      if (d.nu > (P.tune.elem_bytes == 8 ? 2 : 1)) return "op " + S(o) + "too many unroll bits";
      if (d.n_in > 4) return "op " + S(o) + "wide op with more than 4 inputs";
      if (wide_singles(d) < 0) return "op " + S(o) + "wide op with inputs without the eliminated index after a pair";
      const int64_t nsub = std::max(1, P.tune.threads >> d.nl);
      if (std::min<int64_t>(std::max(1, P.tune.for_bits(d.nbits).tile_blocks), int64_t(1) << d.nb) < nsub)
        return "op " + S(o) + "wide op block range smaller than a workgroup step";
      if (d.nbits <= P.tune.seq_max_bits) return "op " + S(o) + "wide op inside a sequential program";
    } else if (d.nu > ((P.tune.elem_bytes == 8 && d.n_in <= 2) ? 1 : 0)) {
      return "op " + S(o) + "too many unroll bits";
    }
    uint32_t seen = 0;
    bool summed_block = false;
    for (int z = 0; z < d.nbits - 1; ++z) {
      const uint32_t u = d.zbit[z];
      if (u < 1 || (int)u >= d.nbits || (seen >> u) & 1) return "op " + S(o) + "bad zbit";
      seen |= 1u << u;
      if (z >= d.nl && z < d.nl + d.nu && !((d.out_mask >> u) & 1)) return "op " + S(o) + "summed unroll bit";
      if (z >= d.nl + d.nu + d.nk && !((d.out_mask >> u) & 1)) summed_block = true;
    }
    for (int z = 0; z < 32; ++z)
      if ((d.lane_sum >> z) & 1)
        if (z >= d.nl || (d.out_mask >> d.zbit[z]) & 1) return "op " + S(o) + "bad lane reduction bit";
    for (int z = 0; z < d.nl; ++z)
      if (!((d.lane_sum >> z) & 1) && !((d.out_mask >> d.zbit[z]) & 1)) return "op " + S(o) + "unreduced summed lane bit";
    if (bool(d.lane_sum >> 6) != bool(d.flags & F_LDSRED)) return "op " + S(o) + "LDS reduction flag mismatch";
    if (summed_block != bool(d.flags & F_ATOMIC)) return "op " + S(o) + "atomic flag mismatch";
    for (int i = 0; i < d.n_in; ++i)
      if (d.in_off[i] < 0 || d.in_off[i] + (int64_t(1) << __builtin_popcount(d.in_mask[i])) > P.arena_grad)
        return "op " + S(o) + "input range out of bounds";
    if (d.out_off < 0 || d.out_off + (int64_t(1) << __builtin_popcount(d.out_mask)) > P.arena_grad)
      return "op " + S(o) + "output range out of bounds";
    for (int i = 0; i <= MAXIN; ++i) {
      if (i < MAXIN && i >= d.n_in) continue;
      const uint32_t m = i == MAXIN ? d.out_mask : d.in_mask[i];
      for (int j = 0; j < MAXLANE; ++j) {
        const uint32_t st = j < d.nl && ((m >> d.zbit[j]) & 1) ? (1u << __builtin_popcount(m & ((1u << d.zbit[j]) - 1))) : 0u;
        const uint32_t got = d.lsh[i][j] == LSH_NONE ? 0u : (1u << d.lsh[i][j]);
        if (st != got) return "op " + S(o) + "lane shift table mismatch";
      }
    }
  }
  // leaf gradients: tables of at most 8 leaves first (their kernel only has
  // the variants up to 8 leaves), then the others
  if (P.lgrad_mid < P.lgrad_lo || P.lgrad_mid > P.lgrad_hi) return "leaf-gradient split outside its range";
  for (int32_t o = P.lgrad_lo; o < P.lgrad_hi; ++o) {
    const OpDesc& d = P.ops[o];
    if (d.kind != OP_LEAFGRAD) return "op " + S(o) + "not a leaf gradient";
    if ((o < P.lgrad_mid) != (d.aux1 <= 8)) return "op " + S(o) + "leaf gradient in the wrong launch";
  }
  // LDS-resident programs: every operand inside the window; each input's
  // dimensions map one to one onto its element bits
  for (size_t c = 0; c < P.cones.size(); ++c) {
    if (!P.cone_lds[c]) continue;
    for (int r = 0; r < 2; ++r) {
      const int32_t lo = r ? P.small_grad_lo[c] : P.small_fwd_lo[c], hi = r ? P.small_grad_hi[c] : P.small_fwd_hi[c];
      if (lo >= hi || hi > (int32_t)P.small.size()) return "cone " + S(c) + "empty LDS program";
      for (int32_t k = lo; k < hi; ++k) {
        const SmallOp& d = P.small[k];
        auto in_window = [&](int64_t off, int64_t n) { return off >= 0 && off + n <= P.lds_elems; };
        if (d.cone != (int32_t)c) return "LDS op " + S(k) + "of another cone";
        if ((d.flags & SF_SPLIT) && (d.kind != S_CONTRACT || d.n_out < 7)) return "LDS op " + S(k) + "split op shape";
        if (d.kind == S_CONTRACT) {
          if (d.nbits > 15 || d.n_out > d.nbits || d.n_in < 1 || d.n_in > 8) return "LDS op " + S(k) + "shape";
          if (d.flags & SF_GOUT) {
            if (d.gout < 0 || d.gout + (int64_t(1) << d.n_out) > P.arena_grad)
              return "LDS op " + S(k) + "global output out of the arena";
          } else if (!in_window(d.out_off, int64_t(1) << d.n_out)) {
            return "LDS op " + S(k) + "output out of the window";
          }
          for (int i = 0; i < d.n_in; ++i) {
            uint32_t seen = 0;
            int rank = 0;
            for (int j = 0; j < d.nbits; ++j) {
              const int sh = (int)((d.shift[i] >> (4 * j)) & 0xf);
              if (sh == 0xf) continue;
              if (sh >= d.nbits || ((seen >> sh) & 1u)) return "LDS op " + S(k) + "input dimension map";
              seen |= 1u << sh;
              ++rank;
            }
            for (int j = d.nbits; j < 16; ++j)
              if (((d.shift[i] >> (4 * j)) & 0xf) != 0xf) return "LDS op " + S(k) + "dimension beyond the union";
            if (seen != (1u << rank) - 1u) return "LDS op " + S(k) + "input element bits not contiguous";
            if (!in_window(d.in_off[i], int64_t(1) << rank)) return "LDS op " + S(k) + "input out of the window";
          }
        } else if (d.kind == S_COPYIN) {
          if (k != lo || !in_window(0, d.aux1) || d.gout != P.cones[c].lam_base || d.aux1 != P.cones[c].lam_size)
            return "LDS op " + S(k) + "leaf-block copy";
        } else if (d.kind == S_RESULT) {
          if (d.n_in > 4) return "LDS op " + S(k) + "more than 4 scalars";
          for (int i = 0; i < d.n_in; ++i)
            if (!in_window(d.in_off[i], 1) || ((d.flags & SF_GRAD) && !in_window(d.in_off[4 + i], 1)))
              return "LDS op " + S(k) + "scalar out of the window";
        } else {
          return "LDS op " + S(k) + "unknown kind";
        }
      }
    }
  }
  for (int g = 0; g < 2; ++g) {
    const std::string e = validate_queue(P, g == 1);
    if (!e.empty()) return e;
  }
  return "";
}

void build_items(Plan& P, bool grad) {
  Queue q;
  build_queue(P, grad, nullptr, q);
  (grad ? P.items_grad : P.items_fwd) = std::move(q.items);
  (grad ? P.node_init_grad : P.node_init_fwd) = std::move(q.init);
  (grad ? P.succ_grad : P.succ_fwd) = std::move(q.succ);
  // LDS-resident cones: one workgroup each, the longest programs first
  auto& sm = grad ? P.small_items_grad : P.small_items_fwd;
  sm.clear();
  std::vector<std::pair<int32_t, int32_t>> r;
  for (size_t c = 0; c < P.cones.size(); ++c)
    if (!P.cone_lds.empty() && P.cone_lds[c])
      r.push_back(grad ? std::make_pair(P.small_grad_lo[c], P.small_grad_hi[c])
                       : std::make_pair(P.small_fwd_lo[c], P.small_fwd_hi[c]));
  std::stable_sort(r.begin(), r.end(), [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
    return a.second - a.first > b.second - b.first;
  });
  for (auto& x : r) {
    sm.push_back(x.first);
    sm.push_back(x.second);
  }
}

// A cone's program as a chain of segments: a segment is up to two physical op
// ranges run in sequence by one workgroup (a cone's gradient program is its
// forward range followed by its adjoint range), or one wide op split into
// items of per_item blocks.  Durations are estimates for the list schedule: a
// fixed cost per item and per op plus bytes at a nominal per-workgroup rate.
struct Seg {
  int32_t r[4];
  bool wide;
  int64_t nblocks;
  int64_t per_item;  // blocks per item of a wide op
  int32_t n_items() const { return wide ? (int32_t)((nblocks + per_item - 1) / per_item) : 1; }
};
struct Chains {
  std::vector<std::vector<Seg>> segs;
  std::vector<std::vector<double>> item_us, span;  // per segment: one item's duration; remaining chain length
};

static void cone_chains(const Plan& P, bool grad, const std::function<bool(int32_t)>& keep, Chains& ch) {
  const TuneParams& T = P.tune;
  const size_t nc = P.cones.size();
  // LDS-resident cones run in their own kernel, not from the queue
  auto in_queue = [&](size_t c) { return P.cone_lds.empty() || !P.cone_lds[c]; };
  ch.segs.assign(nc, {});
  ch.item_us.assign(nc, {});
  ch.span.assign(nc, {});
  auto& segs = ch.segs;
  for (size_t c = 0; c < nc; ++c) {
    if (!in_queue(c)) continue;
    std::vector<std::pair<int32_t, int32_t>> ranges;
    if (grad) {
      ranges.push_back({P.cone_fwd_lo[c], P.cone_fwd_hi[c]});
      ranges.push_back({P.cone_adj_lo[c], P.cone_adj_hi[c]});
    } else {
      ranges.push_back({P.cone_fwd_lo[c], P.cone_fwd_hi[c] + 1});
    }
    Seg cur{{-1, -1, -1, -1}, false, 1, 1};
    int nr = 0;  // physical ranges used by the open narrow segment
    auto close = [&]() {
      if (nr) segs[c].push_back(cur);
      cur = Seg{{-1, -1, -1, -1}, false, 1, 1};
      nr = 0;
    };
    for (auto& rg : ranges) {
      bool open_here = false;
      for (int32_t o = rg.first; o < rg.second; ++o) {
        const OpDesc& d = P.ops[o];
        if (keep && !keep(o)) {
          // a skipped op ends the open narrow range here
          open_here = false;
          continue;
        }
        const bool contract = d.kind == OP_CONTRACT || d.kind == OP_ADJOINT;
        const bool wide = contract && d.nbits > T.seq_max_bits;
        if (wide) {
          close();
          open_here = false;
          // tiles of an LDS-tiled adjoint: about 2^16 union elements per item
          const int tb = T.for_bits(d.nbits).tile_blocks;
          const int64_t per = (d.flags & F_TILE) ? std::min<int64_t>(std::max(1, tb),
                                                                       int64_t(1) << std::max(0, 16 - d.nl - d.nk))
                                                 : std::max(1, tb);
          segs[c].push_back(Seg{{o, o + 1, -1, -1}, true, int64_t(1) << d.nb, per});
        } else {
          if (!open_here) {
            if (nr == 2) close();
            cur.r[2 * nr] = o;
            cur.r[2 * nr + 1] = o + 1;
            ++nr;
            open_here = true;
          } else {
            cur.r[2 * nr - 1] = o + 1;
          }
        }
      }
    }
    close();
  }
  auto op_bytes = [&](const OpDesc& d) -> double {
    double b = 0;
    if (d.kind == OP_CONTRACT) {
      b = std::ldexp(1.0, __builtin_popcount(d.out_mask));
      for (int i = 0; i < d.n_in; ++i) b += std::ldexp(1.0, __builtin_popcount(d.in_mask[i]));
    } else if (d.kind == OP_ADJOINT) {
      for (int i = 0; i < d.n_in; ++i)
        b += std::ldexp(1.0, __builtin_popcount(d.in_mask[i])) * (((d.adj_sel >> i) & 1u) ? 2 : 1);
    } else if (d.kind == OP_ZERO) {
      b = (double)d.in_off[0];
    }
    return b * T.elem_bytes;
  };
  // bytes per microsecond of one workgroup, by kind of work (measured on
  // MI355X for 256-thread workgroups, four resident per compute unit)
  auto rate = [](const OpDesc& d) -> double {
    if (d.kind == OP_ADJOINT) return 7.0e3;
    if (d.kind != OP_CONTRACT) return 2.0e3;
    const bool adj = !(d.in_mask[0] & 1u);
    const bool red = __builtin_popcount(d.out_mask) < d.nbits - (adj ? 0 : 1);
    return adj ? (red ? 2.6e3 : 6.2e3) : 3.7e3;
  };
  for (size_t c = 0; c < nc; ++c) {
    for (const Seg& g : segs[c]) {
      double t = 2.0;
      if (g.wide) {
        const OpDesc& d = P.ops[g.r[0]];
        t += op_bytes(d) / (double)g.n_items() / rate(d);
      } else {
        for (int r = 0; r < 2; ++r)
          if (g.r[2 * r] >= 0)
            for (int32_t o = g.r[2 * r]; o < g.r[2 * r + 1]; ++o) t += 4.0 + op_bytes(P.ops[o]) / 1.7e3;
      }
      ch.item_us[c].push_back(t);
    }
    ch.span[c].assign(segs[c].size() + 1, 0.0);
    for (size_t s = segs[c].size(); s-- > 0;) ch.span[c][s] = ch.span[c][s + 1] + ch.item_us[c][s];
  }
}

// Memory admission under a workspace budget.  Cones run from the work queue
// share a dynamic area of `area` elements: the list schedule of the gradient
// program is simulated with a first-fit allocator, a cone is admitted (its
// first segment released) once its dynamic region fits, and its region is
// freed when its last segment ends.  Sets every queued cone's dyn_base and
// its predecessors: the cones that last held any part of its region (the
// queue makes it wait for them).  LDS-resident cones keep no region in the
// batched sweep; they get offset 0 (the plain per-op path runs one cone at a
// time).  Returns false if some cone's region exceeds the area.
static bool admit_cones(Plan& P, int64_t area) {
  const size_t nc = P.cones.size();
  Chains ch;
  cone_chains(P, true, nullptr, ch);
  P.cone_pred.assign(nc, {});
  struct Piece {
    int64_t lo, hi;
    int owner, last;  // owner -1: free
  };
  std::vector<Piece> mem{{0, area, -1, -1}};
  auto dyn = [&](size_t c) { return P.cones[c].arena_elems - P.cones[c].dyn_start; };
  for (size_t c = 0; c < nc; ++c) {
    P.cones[c].dyn_base = 0;
    if (dyn(c) > area) return false;
  }
  auto alloc = [&](int c, int64_t size) -> bool {
    for (size_t i = 0; i < mem.size(); ++i) {
      if (mem[i].owner >= 0) continue;
      // a run of free pieces from i covering size (64-element aligned start)
      const int64_t lo = (mem[i].lo + 63) / 64 * 64;
      if (lo >= mem[i].hi) continue;
      size_t j = i;
      while (j < mem.size() && mem[j].owner < 0 && mem[j].hi < lo + size) ++j;
      if (j == mem.size() || mem[j].owner >= 0) {
        i = j;
        continue;
      }
      const int64_t hi = lo + size;
      // split the first and last pieces, mark the covered ones
      std::vector<Piece> out(mem.begin(), mem.begin() + i);
      if (mem[i].lo < lo) out.push_back({mem[i].lo, lo, -1, mem[i].last});
      std::vector<int> pred;
      for (size_t k = i; k <= j; ++k) {
        const int64_t a = std::max(mem[k].lo, lo), b = std::min(mem[k].hi, hi);
        if (a < b && mem[k].last >= 0) pred.push_back(mem[k].last);
      }
      out.push_back({lo, hi, c, c});
      if (mem[j].hi > hi) out.push_back({hi, mem[j].hi, -1, mem[j].last});
      out.insert(out.end(), mem.begin() + j + 1, mem.end());
      mem.swap(out);
      std::sort(pred.begin(), pred.end());
      pred.erase(std::unique(pred.begin(), pred.end()), pred.end());
      P.cone_pred[c] = pred;
      P.cones[c].dyn_base = lo;
      return true;
    }
    return false;
  };
  auto release = [&](int c) {
    for (Piece& m : mem)
      if (m.owner == c) m.owner = -1;
  };
  struct Ready {
    double prio;
    int32_t cone, seg, item;
    bool operator<(const Ready& o) const {
      if (prio != o.prio) return prio < o.prio;
      if (cone != o.cone) return cone > o.cone;
      return item > o.item;
    }
  };
  struct Done {
    double t;
    int32_t cone, seg;
    bool operator<(const Done& o) const { return t > o.t; }
  };
  std::priority_queue<Ready> ready;
  std::priority_queue<Done> running;
  std::vector<std::vector<int32_t>> left(nc);
  auto release_seg = [&](size_t c, size_t s) {
    const int32_t k = ch.segs[c][s].n_items();
    left[c][s] = k;
    for (int32_t it = 0; it < k; ++it) ready.push({ch.span[c][s], (int32_t)c, (int32_t)s, it});
  };
  std::vector<int> pending;  // queued cones not yet admitted, longest chain first
  for (size_t c = 0; c < nc; ++c) {
    left[c].assign(ch.segs[c].size(), 0);
    if (!ch.segs[c].empty()) pending.push_back((int)c);
  }
  std::stable_sort(pending.begin(), pending.end(), [&](int a, int b) { return ch.span[a][0] > ch.span[b][0]; });
  auto admit = [&]() {
    std::vector<int> rest;
    for (int c : pending) {
      if (alloc(c, dyn(c)))
        release_seg(c, 0);
      else
        rest.push_back(c);
    }
    pending.swap(rest);
  };
  admit();
  double now = 0;
  int free_w = std::max(1, P.sched_workers);
  for (;;) {
    while (free_w > 0 && !ready.empty()) {
      const Ready r = ready.top();
      ready.pop();
      running.push({now + ch.item_us[r.cone][r.seg], r.cone, r.seg});
      --free_w;
    }
    if (running.empty()) break;
    const Done d = running.top();
    running.pop();
    now = d.t;
    ++free_w;
    if (--left[d.cone][d.seg] == 0) {
      if ((size_t)d.seg + 1 < ch.segs[d.cone].size()) {
        release_seg(d.cone, d.seg + 1);
      } else {
        release(d.cone);
        admit();
      }
    }
  }
  return pending.empty();
}

void build_queue(const Plan& P, bool grad, const std::function<bool(int32_t)>& keep, Queue& q) {
  auto& items = q.items;
  auto& init = q.init;
  auto& succ = q.succ;
  items.clear();
  init.clear();
  succ.clear();
  const size_t nc = P.cones.size();
  Chains ch;
  cone_chains(P, grad, keep, ch);
  const auto& segs = ch.segs;
  // memory admission: cone c starts after its predecessors end.  A filtered
  // queue may leave a predecessor without items: c then waits for that
  // cone's own predecessors, transitively.
  const bool gated = P.cone_pred.size() == nc;
  std::vector<std::vector<int>> pred(nc);
  if (gated) {
    std::vector<char> done(nc, 0);
    std::function<void(int)> eff = [&](int c) {
      if (done[c]) return;
      done[c] = 1;
      std::vector<int> r;
      for (int a : P.cone_pred[c]) {
        if (!segs[a].empty()) {
          r.push_back(a);
        } else {
          eff(a);
          r.insert(r.end(), pred[a].begin(), pred[a].end());
        }
      }
      std::sort(r.begin(), r.end());
      r.erase(std::unique(r.begin(), r.end()), r.end());
      pred[c] = r;
    };
    for (size_t c = 0; c < nc; ++c) eff((int)c);
  }
  std::vector<std::vector<int32_t>> after(nc);  // cones that wait for this one
  for (size_t c = 0; c < nc; ++c)
    for (int a : pred[c]) after[a].push_back((int32_t)c);
  std::vector<std::vector<int32_t>> node_of(nc);
  int32_t nn = 0;
  for (size_t c = 0; c < nc; ++c)
    for (size_t s = 0; s < segs[c].size(); ++s) node_of[c].push_back(nn++);
  init.assign(nn, 0);
  for (size_t c = 0; c < nc; ++c)
    for (size_t s = 1; s < segs[c].size(); ++s) init[node_of[c][s]] = segs[c][s - 1].n_items();
  // a gated cone's first node also counts its predecessors' last items
  std::vector<int32_t> waits(nc, 0);
  for (size_t c = 0; c < nc; ++c)
    for (int a : pred[c])
      if (!segs[c].empty()) {
        init[node_of[c][0]] += segs[a].back().n_items();
        ++waits[c];
      }
  // Queue order: a list schedule of the segments on the resident workgroups,
  // longest remaining chain first; an item enters the queue only when its
  // predecessor segment (and, for a cone's first segment, its predecessor
  // cones) has finished in the schedule, so every item waits only on items
  // earlier in the queue.
  const int workers = std::max(1, P.sched_workers);
  struct Ready {
    double prio;
    int32_t cone, seg, item;
    bool operator<(const Ready& o) const {
      if (prio != o.prio) return prio < o.prio;
      if (cone != o.cone) return cone > o.cone;
      return item > o.item;
    }
  };
  struct Done {
    double t;
    int32_t cone, seg;
    bool operator<(const Done& o) const { return t > o.t; }
  };
  std::priority_queue<Ready> ready;
  std::priority_queue<Done> running;
  std::vector<std::vector<int32_t>> left(nc);  // unfinished items per segment
  auto release = [&](size_t c, size_t s) {
    const int32_t k = segs[c][s].n_items();
    left[c][s] = k;
    for (int32_t it = 0; it < k; ++it) ready.push({ch.span[c][s], (int32_t)c, (int32_t)s, it});
  };
  // the simulation counts waits down: whether a cone's first node waits is
  // fixed before it starts
  const std::vector<int32_t> gate_of = waits;
  for (size_t c = 0; c < nc; ++c) {
    left[c].assign(segs[c].size(), 0);
    if (!segs[c].empty() && waits[c] == 0) release(c, 0);
  }
  double now = 0;
  int free_w = workers;
  for (;;) {
    while (free_w > 0 && !ready.empty()) {
      const Ready r = ready.top();
      ready.pop();
      const Seg& g = segs[r.cone][r.seg];
      const int32_t node = node_of[r.cone][r.seg];
      const bool has_next = (size_t)r.seg + 1 < segs[r.cone].size();
      int32_t slo = (int32_t)succ.size();
      if (has_next) succ.push_back(node_of[r.cone][r.seg + 1]);
      if (!has_next)
        for (int32_t c2 : after[r.cone])
          if (!segs[c2].empty()) succ.push_back(node_of[c2][0]);
      const int32_t shi = (int32_t)succ.size();
      const int32_t wait_node = (r.seg > 0 || gate_of[r.cone] > 0) ? node : -1;
      if (!g.wide) {
        items.push_back({g.r[0], g.r[1], g.r[2], g.r[3], 0, -1, wait_node, slo, shi, {0, 0, 0}});
      } else {
        const int64_t tb = g.per_item;
        const int64_t b = (int64_t)r.item * tb;
        items.push_back({g.r[0], g.r[1], -1, -1, (int32_t)b, (int32_t)std::min<int64_t>(g.nblocks, b + tb), wait_node,
                         slo, shi, {0, 0, 0}});
      }
      running.push({now + ch.item_us[r.cone][r.seg], r.cone, r.seg});
      --free_w;
    }
    if (running.empty()) break;
    const Done d = running.top();
    running.pop();
    now = d.t;
    ++free_w;
    if (--left[d.cone][d.seg] == 0) {
      if ((size_t)d.seg + 1 < segs[d.cone].size()) {
        release(d.cone, d.seg + 1);
      } else {
        for (int32_t c2 : after[d.cone])
          if (--waits[c2] == 0 && !segs[c2].empty()) release(c2, 0);
      }
    }
  }
}

}  // namespace qtn
