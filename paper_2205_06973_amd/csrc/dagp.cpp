// dagp.cpp -- acyclic recursive-bisection partitioner with a merge phase.
//
// Sec. IV.B.3 describes the paper's dagP: compute the working set of the
// graph; while it exceeds L_m (= k), split the graph into two roughly
// balanced parts (node counts, imbalance up to 1.5) with an *acyclic*
// bisection and recurse into both; finally merge parts on the part-graph as
// long as a merge keeps the part-graph acyclic and the merged working set
// within L_m.  The objective throughout is the number of parts under the
// working-set limit, not the edge cut; working sets are updated
// incrementally by counting, per qubit, the gates of each side that use it
// (the in-edge counting of Sec. IV.B.3 amounts to the same thing, because
// every gate has as many in-edges as out-edges, one per qubit).
//
// This implementation (written from that description; the underlying
// multilevel partitioner is not reproduced):
//   * an acyclic bisection of a convex gate set V is a down-set V0 (closed
//     under predecessors inside V) and its complement V1, so every edge goes
//     V0 -> V1 and running V0's parts before V1's respects the DAG;
//   * initial cut: the best prefix cut of several topological orders of V
//     (the circuit order and seeded random depth-first orders), scored by
//     L(V0) + L(V1) within the balance window;
//   * refinement: greedy moves of a maximal gate of V0 to V1, or a minimal
//     gate of V1 to V0, that lower L(V0) + L(V1) and keep the balance;
//   * merge phase: for parts in topological order, merge with a later part
//     when the union fits k and no other part lies on a path between them
//     (so the contracted graph stays acyclic); parts are then renumbered in
//     a topological order.
//   * coarsening (the agglomerative clustering that precedes the bisection):
//     in circuit order, a gate joins the cluster holding all of its
//     predecessors when the union stays within k qubits and the cluster
//     within a size cap; otherwise it starts a cluster.  A gate that joins
//     has no predecessor outside its cluster, so every edge between
//     clusters enters a cluster at the gate that started it, from a cluster
//     started earlier: the cluster graph is acyclic.  The bisection and its
//     refinement then run on clusters (a cluster's qubits = the union of its
//     gates'), the leaves are expanded back to gates, and the merge phase
//     runs on gates.  Restarts with and without coarsening (two caps) keep
//     the fewest parts.
#include <algorithm>
#include <numeric>

#include "hisv_internal.h"

namespace hisv {

namespace {

struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int below(int n) { return (int)(next() % (uint64_t)n); }
};

// The bisection works on items -- gates, or clusters of gates after
// coarsening -- each with a qubit mask, joined by an item DAG.
struct Ctx {
  const std::vector<uint64_t>* mask;  // qubits of each item
  const Dag* dag;                     // item DAG
  int n, k;
  uint64_t pad;  // qubits every part holds anyway (multi-level tiles)
  Rng rng;
  std::vector<int> side;   // scratch: -1 outside V, 0 / 1 inside
  std::vector<int> cnt0, cnt1;
  std::vector<std::vector<int>> parts;  // leaves (item ids), in execution order
};

uint64_t mask_of(const Ctx& c, const std::vector<int>& V) {
  uint64_t m = 0;
  for (int v : V) m |= (*c.mask)[v];
  return m;
}

// Topological order of the convex set V (listed in circuit order): random
// depth-first emission, as for the DFS strategy.
void order_of(Ctx& c, const std::vector<int>& V, bool natural, std::vector<int>* out) {
  if (natural) {
    *out = V;
    return;
  }
  std::vector<int> indeg(V.size());
  std::vector<int> stack;
  // local index of each gate (side[] holds index + 2 while ordering)
  for (size_t i = 0; i < V.size(); ++i) c.side[V[i]] = (int)i + 2;
  for (size_t i = 0; i < V.size(); ++i) {
    int d = 0;
    for (int p : c.dag->pred[V[i]]) d += c.side[p] >= 2;
    indeg[i] = d;
    if (!d) stack.push_back((int)i);
  }
  for (int i = (int)stack.size() - 1; i > 0; --i) std::swap(stack[i], stack[c.rng.below(i + 1)]);
  out->clear();
  std::vector<int> ready;
  while (!stack.empty()) {
    const int li = stack.back();
    stack.pop_back();
    out->push_back(V[li]);
    ready.clear();
    for (int s : c.dag->succ[V[li]]) {
      const int ls = c.side[s] - 2;
      if (ls >= 0 && --indeg[ls] == 0) ready.push_back(ls);
    }
    for (int i = (int)ready.size() - 1; i > 0; --i) std::swap(ready[i], ready[c.rng.below(i + 1)]);
    for (int r : ready) stack.push_back(r);
  }
  for (int v : V) c.side[v] = -1;
}

// Best balanced prefix cut of `ord` by L(prefix) + L(suffix); returns the
// cut position (prefix length) and its cost.
std::pair<int, int> best_prefix_cut(const Ctx& c, const std::vector<int>& ord, int lo, int hi) {
  const int N = (int)ord.size();
  std::vector<uint64_t> suf(N + 1, 0);
  for (int i = N - 1; i >= 0; --i) suf[i] = suf[i + 1] | (*c.mask)[ord[i]];
  uint64_t pre = 0;
  int best = -1, best_cost = 1 << 30;
  for (int i = 1; i < N; ++i) {
    pre |= (*c.mask)[ord[i - 1]];
    if (i < lo || i > hi) continue;
    const int cost = __builtin_popcountll(pre & ~c.pad) + __builtin_popcountll(suf[i] & ~c.pad);
    if (cost < best_cost) {
      best_cost = cost;
      best = i;
    }
  }
  return {best, best_cost};
}

// Greedy refinement of a down-set bisection (side[v] in {0,1} for v in V).
void refine(Ctx& c, const std::vector<int>& V, int lo, int hi) {
  std::fill(c.cnt0.begin(), c.cnt0.end(), 0);
  std::fill(c.cnt1.begin(), c.cnt1.end(), 0);
  int n0 = 0;
  for (int v : V) {
    for (uint64_t m = (*c.mask)[v]; m; m &= m - 1) (c.side[v] ? c.cnt1 : c.cnt0)[__builtin_ctzll(m)]++;
    n0 += c.side[v] == 0;
  }
  for (int pass = 0; pass < 8; ++pass) {
    bool moved = false;
    for (int v : V) {
      const int s = c.side[v];
      if (s == 0 && n0 - 1 < lo) continue;
      if (s == 1 && n0 + 1 > hi) continue;
      // legality: a gate leaves V0 only if none of its successors in V stays
      // in V0; it leaves V1 only if none of its predecessors in V is in V1
      bool legal = true;
      if (s == 0) {
        for (int w : c.dag->succ[v])
          if (c.side[w] == 0) { legal = false; break; }
      } else {
        for (int w : c.dag->pred[v])
          if (c.side[w] == 1) { legal = false; break; }
      }
      if (!legal) continue;
      const uint64_t vm = (*c.mask)[v];
      std::vector<int>& from = s ? c.cnt1 : c.cnt0;
      std::vector<int>& to = s ? c.cnt0 : c.cnt1;
      int gain = 0;
      for (uint64_t m = vm & ~c.pad; m; m &= m - 1) {  // pad qubits: held by both sides anyway
        const int q = __builtin_ctzll(m);
        if (from[q] == 1) ++gain;  // qubit leaves the source side
        if (to[q] == 0) --gain;    // qubit joins the destination side
      }
      if (gain <= 0) continue;
      for (uint64_t m = vm; m; m &= m - 1) {
        from[__builtin_ctzll(m)]--;
        to[__builtin_ctzll(m)]++;
      }
      c.side[v] = 1 - s;
      n0 += s ? 1 : -1;
      moved = true;
    }
    if (!moved) break;
  }
}

void bisect_rec(Ctx& c, std::vector<int> V, int depth) {
  if (V.empty()) return;
  if (__builtin_popcountll(mask_of(c, V) | c.pad) <= c.k || V.size() == 1 || depth > 60) {
    c.parts.push_back(std::move(V));
    return;
  }
  const int N = (int)V.size();
  // balance window: each side holds between 1/4 and 3/4 of the gates
  // (imbalance ratio 1.5); tiny sets may split anywhere
  int lo = std::max(1, N / 4), hi = std::min(N - 1, N - N / 4);
  if (N < 8) {
    lo = 1;
    hi = N - 1;
  }
  std::vector<int> ord, best_ord;
  int best_cut = -1, best_cost = 1 << 30;
  const int tries = 8;
  for (int t = 0; t < tries; ++t) {
    order_of(c, V, t == 0, &ord);
    auto [cut, cost] = best_prefix_cut(c, ord, lo, hi);
    if (cut > 0 && cost < best_cost) {
      best_cost = cost;
      best_cut = cut;
      best_ord = ord;
    }
  }
  if (best_cut < 0) {  // cannot happen for N >= 2; keep the set whole
    c.parts.push_back(std::move(V));
    return;
  }
  for (int i = 0; i < N; ++i) c.side[best_ord[i]] = i < best_cut ? 0 : 1;
  refine(c, V, lo, hi);
  std::vector<int> V0, V1;
  for (int v : V) (c.side[v] ? V1 : V0).push_back(v);  // V is in item (topological) order
  for (int v : V) c.side[v] = -1;
  if (V0.empty() || V1.empty()) {
    c.parts.push_back(std::move(V));
    return;
  }
  bisect_rec(c, std::move(V0), depth + 1);
  bisect_rec(c, std::move(V1), depth + 1);
}

// Merge phase on the part-graph, then topological renumbering.
int merge_and_number(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t pad,
                     std::vector<std::vector<int>>& parts, std::vector<int32_t>* out) {
  const int P = (int)parts.size();
  std::vector<int> pid(gates.size());
  std::vector<uint64_t> mask(P, 0);
  for (int p = 0; p < P; ++p)
    for (int v : parts[p]) {
      pid[v] = p;
      mask[p] |= gates[v].mask();
    }
  // union-find over parts; part-graph kept as adjacency bitsets of leaders
  std::vector<int> leader(P);
  std::iota(leader.begin(), leader.end(), 0);
  auto find = [&](int x) {
    while (leader[x] != x) x = leader[x] = leader[leader[x]];
    return x;
  };
  const int W = (P + 63) / 64;
  std::vector<std::vector<uint64_t>> succ(P, std::vector<uint64_t>(W, 0));
  for (int v = 0; v < (int)gates.size(); ++v)
    for (int w : dag.succ[v])
      if (pid[v] != pid[w]) succ[pid[v]][pid[w] >> 6] |= 1ull << (pid[w] & 63);
  std::vector<char> alive(P, 1);
  // reach(a, b): is b reachable from a in the current contracted graph,
  // through at least one node other than a and b (when skip_direct)?
  std::vector<int> stack;
  std::vector<char> seen(P);
  auto reach_via_other = [&](int a, int b) {
    std::fill(seen.begin(), seen.end(), 0);
    stack.clear();
    for (int w = 0; w < W; ++w)
      for (uint64_t m = succ[a][w]; m; m &= m - 1) {
        const int s = w * 64 + __builtin_ctzll(m);
        if (s != b && alive[s] && !seen[s]) {
          seen[s] = 1;
          stack.push_back(s);
        }
      }
    while (!stack.empty()) {
      const int x = stack.back();
      stack.pop_back();
      if (x == b) return true;
      for (int w = 0; w < W; ++w)
        for (uint64_t m = succ[x][w]; m; m &= m - 1) {
          const int s = w * 64 + __builtin_ctzll(m);
          if (alive[s] && !seen[s]) {
            seen[s] = 1;
            stack.push_back(s);
          }
        }
    }
    return false;
  };
  bool merged_any = true;
  while (merged_any) {
    merged_any = false;
    for (int a = 0; a < P; ++a) {
      if (!alive[a]) continue;
      // prefer partners sharing the most qubits
      std::vector<std::pair<int, int>> cand;
      for (int b = a + 1; b < P; ++b)
        if (alive[b] && __builtin_popcountll(mask[a] | mask[b] | pad) <= k)
          cand.push_back({-__builtin_popcountll(mask[a] & mask[b] & ~pad), b});
      std::sort(cand.begin(), cand.end());
      for (auto [negov, b] : cand) {
        (void)negov;
        if (!alive[b] || __builtin_popcountll(mask[a] | mask[b] | pad) > k) continue;
        if (reach_via_other(a, b) || reach_via_other(b, a)) continue;
        // merge b into a
        alive[b] = 0;
        leader[b] = a;
        mask[a] |= mask[b];
        for (int w = 0; w < W; ++w) succ[a][w] |= succ[b][w];
        succ[a][a >> 6] &= ~(1ull << (a & 63));
        succ[a][b >> 6] &= ~(1ull << (b & 63));
        for (int x = 0; x < P; ++x)
          if (alive[x] && (succ[x][b >> 6] >> (b & 63) & 1)) {
            succ[x][b >> 6] &= ~(1ull << (b & 63));
            if (x != a) succ[x][a >> 6] |= 1ull << (a & 63);
          }
        merged_any = true;
      }
    }
  }
  // topological numbering of the surviving parts (Kahn, smallest id first)
  std::vector<int> indeg(P, 0);
  for (int x = 0; x < P; ++x)
    if (alive[x])
      for (int w = 0; w < W; ++w)
        for (uint64_t m = succ[x][w]; m; m &= m - 1) indeg[w * 64 + __builtin_ctzll(m)]++;
  std::vector<int> ready, number(P, -1);
  for (int x = 0; x < P; ++x)
    if (alive[x] && !indeg[x]) ready.push_back(x);
  int next = 0;
  while (!ready.empty()) {
    std::sort(ready.begin(), ready.end(), std::greater<int>());
    const int x = ready.back();
    ready.pop_back();
    number[x] = next++;
    for (int w = 0; w < W; ++w)
      for (uint64_t m = succ[x][w]; m; m &= m - 1) {
        const int s = w * 64 + __builtin_ctzll(m);
        if (--indeg[s] == 0) ready.push_back(s);
      }
  }
  out->assign(gates.size(), -1);
  for (int v = 0; v < (int)gates.size(); ++v) (*out)[v] = number[find(pid[v])];
  return next;
}

// Coarsening: clusters of gates (cluster_of per gate; clusters numbered in
// circuit order of the gate that started them, a topological order of the
// cluster graph), their qubit masks, gate lists and the cluster DAG.
// cap = most gates a cluster takes.
struct Coarse {
  std::vector<int> cluster_of;
  std::vector<uint64_t> mask;
  std::vector<std::vector<int>> members;  // gate ids, circuit order
  Dag dag;
};

Coarse coarsen(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t pad, int cap) {
  Coarse cz;
  const int G = (int)gates.size();
  cz.cluster_of.assign(G, -1);
  for (int v = 0; v < G; ++v) {
    int c = -1;
    bool one = !dag.pred[v].empty();
    for (int p : dag.pred[v]) {
      const int pc = cz.cluster_of[p];
      if (c < 0) c = pc;
      else if (pc != c) one = false;
    }
    const uint64_t gm = gates[v].mask();
    if (one && c >= 0 && (int)cz.members[c].size() < cap &&
        __builtin_popcountll(cz.mask[c] | gm | pad) <= k) {
      cz.cluster_of[v] = c;
      cz.mask[c] |= gm;
      cz.members[c].push_back(v);
    } else {
      cz.cluster_of[v] = (int)cz.mask.size();
      cz.mask.push_back(gm);
      cz.members.push_back({v});
    }
  }
  const int C = (int)cz.mask.size();
  cz.dag.G = C;
  cz.dag.succ.assign(C, {});
  cz.dag.pred.assign(C, {});
  for (int v = 0; v < G; ++v)
    for (int w : dag.succ[v]) {
      const int a = cz.cluster_of[v], b = cz.cluster_of[w];
      if (a == b) continue;
      if (std::find(cz.dag.succ[a].begin(), cz.dag.succ[a].end(), b) == cz.dag.succ[a].end()) {
        cz.dag.succ[a].push_back(b);
        cz.dag.pred[b].push_back(a);
      }
    }
  return cz;
}

}  // namespace

int partition_dagp(const std::vector<Gate>& gates, const Dag& dag, int n, int k, uint64_t seed,
                   std::vector<int32_t>* part, uint64_t pad) {
  // seeded restarts of (coarsening +) bisection + merge; keep the fewest
  // parts.  cap 1 = no coarsening (every gate its own item).
  const int G = (int)gates.size();
  std::vector<uint64_t> gmask(G);
  for (int v = 0; v < G; ++v) gmask[v] = gates[v].mask();
  const int caps[] = {1, 4, 16};
  std::vector<Coarse> levels;
  for (int cap : caps) levels.push_back(cap > 1 ? coarsen(gates, dag, k, pad, cap) : Coarse{});
  int best = -1;
  std::vector<int32_t> cand;
  for (int r = 0; r < 6; ++r) {
    for (size_t l = 0; l < levels.size(); ++l) {
      const bool coarse = caps[l] > 1;
      const Coarse& cz = levels[l];
      const std::vector<uint64_t>* im = coarse ? &cz.mask : &gmask;
      const Dag* id = coarse ? &cz.dag : &dag;
      const int items = (int)im->size();
      Ctx c{im, id, n, k, pad, Rng((seed ^ 0xda6bull) + 7919ull * r + 104729ull * l), {}, {}, {}, {}};
      c.side.assign(items, -1);
      c.cnt0.assign(64, 0);
      c.cnt1.assign(64, 0);
      std::vector<int> all(items);
      std::iota(all.begin(), all.end(), 0);
      if (items) bisect_rec(c, std::move(all), 0);
      if (coarse) {  // leaves back to gates, in circuit order
        for (std::vector<int>& leaf : c.parts) {
          std::vector<int> gs;
          for (int cl : leaf) gs.insert(gs.end(), cz.members[cl].begin(), cz.members[cl].end());
          std::sort(gs.begin(), gs.end());
          leaf.swap(gs);
        }
      }
      const int np = merge_and_number(gates, dag, k, pad, c.parts, &cand);
      if (best < 0 || np < best) {
        best = np;
        part->swap(cand);
      }
    }
  }
  return best;
}

}  // namespace hisv
