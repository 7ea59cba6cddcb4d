// partition.cpp -- gate DAG and topological-order cutoff partitioners.
//
// Sec. IV.A: vertices are gates; an edge runs from a gate to the next gate
// on each of its qubits (the per-qubit entry and exit vertices carry no
// computation and stay implicit).  A part's working set is the number of
// distinct qubits of its gates.  Sec. IV.B.1 (Nat) cuts the circuit order
// into consecutive segments, closing a segment just before the gate that
// would take its working set above k; Sec. IV.B.2 (DFS) applies the same
// cutoff to several random depth-first topological orders and keeps the
// one with the fewest parts.  Consecutive segments of any topological order
// form an acyclic part-graph, and numbering them in order numbers the
// part-graph topologically.
#include <algorithm>
#include <climits>
#include <thread>

#include "hisv_internal.h"

namespace hisv {

Dag build_dag(const std::vector<Gate>& gates) {
  Dag d;
  d.G = (int)gates.size();
  d.succ.assign(d.G, {});
  d.pred.assign(d.G, {});
  std::vector<int> last(64, -1);
  for (int j = 0; j < d.G; ++j) {
    const Gate& g = gates[j];
    const int qs[2] = {g.q0, g.q1};
    for (int t = 0; t < g.arity(); ++t) {
      const int i = last[qs[t]];
      if (i >= 0 && std::find(d.succ[i].begin(), d.succ[i].end(), j) == d.succ[i].end()) {
        d.succ[i].push_back(j);
        d.pred[j].push_back(i);
      }
      last[qs[t]] = j;
    }
  }
  return d;
}

int cutoff_partition(const std::vector<Gate>& gates, const std::vector<int>& order, int k,
                     std::vector<int32_t>* part, uint64_t pad) {
  part->assign(gates.size(), -1);
  uint64_t cur = 0;
  int pid = -1;
  for (int gi : order) {
    const uint64_t m = gates[gi].mask();
    if (pid < 0 || __builtin_popcountll(cur | m | pad) > k) {
      ++pid;
      cur = 0;
    }
    cur |= m;
    (*part)[gi] = pid;
  }
  return pid + 1;
}

int partition_nat(const std::vector<Gate>& gates, int k, std::vector<int32_t>* part, uint64_t pad) {
  std::vector<int> order(gates.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  return cutoff_partition(gates, order, k, part, pad);
}

namespace {
// splitmix64: a small seeded generator for the random DFS orders.
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
  template <typename V>
  void shuffle(V& v) {
    for (int i = (int)v.size() - 1; i > 0; --i) std::swap(v[i], v[below(i + 1)]);
  }
};

// A random depth-first topological order: a ready vertex is emitted, its
// newly ready successors are pushed in random order on a stack, and the
// next vertex comes from the top of the stack, so the order follows chains
// of dependent gates before moving on.
void random_dfs_order(const Dag& dag, Rng& rng, std::vector<int>* order) {
  order->clear();
  std::vector<int> indeg(dag.G);
  std::vector<int> stack;
  for (int v = 0; v < dag.G; ++v) {
    indeg[v] = (int)dag.pred[v].size();
    if (!indeg[v]) stack.push_back(v);
  }
  rng.shuffle(stack);
  std::vector<int> ready;
  while (!stack.empty()) {
    const int v = stack.back();
    stack.pop_back();
    order->push_back(v);
    ready.clear();
    for (int s : dag.succ[v])
      if (--indeg[s] == 0) ready.push_back(s);
    rng.shuffle(ready);
    for (int s : ready) stack.push_back(s);
  }
}
}  // namespace

int partition_dfs(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t seed,
                  int trials, std::vector<int32_t>* part, uint64_t pad) {
  int best = partition_nat(gates, k, part, pad);
  std::vector<int> order;
  std::vector<int32_t> cand;
  for (int t = 1; t < trials; ++t) {
    Rng rng(seed * 0x100000001B3ull + (uint64_t)t);
    random_dfs_order(dag, rng, &order);
    const int np = cutoff_partition(gates, order, k, &cand, pad);
    if (np < best) {
      best = np;
      part->swap(cand);
    }
  }
  return best;
}

// Greedy growth over the ready set.  A part takes, one at a time, a ready
// gate (all its predecessors placed) that still fits, preferring the one
// that adds the fewest new qubits; when no ready gate fits, the part is
// closed.  The placed gates form a topological order and every part is a
// contiguous piece of it, so the part-graph is acyclic (as for the cutoff
// of Sec. IV.B.1-2).  Ties go to the lowest gate index in trial 0 and to a
// seeded random key in the other trials; the fewest parts win.
int partition_greedy(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t seed,
                     int trials, std::vector<int32_t>* part, uint64_t pad) {
  const int G = (int)gates.size();
  int best = -1;
  std::vector<int32_t> cand(G);
  std::vector<int> indeg(G), ready;
  std::vector<uint64_t> key(G);
  for (int t = 0; t < std::max(1, trials); ++t) {
    Rng rng(seed * 0x100000001B3ull + 0x9e37ull + (uint64_t)t);
    for (int i = 0; i < G; ++i) key[i] = t == 0 ? (uint64_t)i : rng.next();
    ready.clear();
    for (int i = 0; i < G; ++i) {
      indeg[i] = (int)dag.pred[i].size();
      if (!indeg[i]) ready.push_back(i);
    }
    int np = 0, placed = 0;
    while (placed < G) {
      uint64_t cur = pad;
      ++np;
      for (;;) {
        int pick = -1, pick_new = 65;
        for (int r = 0; r < (int)ready.size(); ++r) {
          const int i = ready[r];
          const uint64_t m = gates[i].mask();
          if (__builtin_popcountll(cur | m) > k) continue;
          const int nw = __builtin_popcountll(m & ~cur);
          if (nw < pick_new || (nw == pick_new && key[i] < key[ready[pick]])) {
            pick = r;
            pick_new = nw;
          }
        }
        if (pick < 0) break;
        const int i = ready[pick];
        ready[pick] = ready.back();
        ready.pop_back();
        cur |= gates[i].mask();
        cand[i] = np - 1;
        ++placed;
        for (int s : dag.succ[i])
          if (--indeg[s] == 0) ready.push_back(s);
      }
    }
    if (best < 0 || np < best) {
      best = np;
      *part = cand;
    }
  }
  return best;
}

namespace {
// One closure-partition run (see partition_closure).
class ClosureRun {
 public:
  ClosureRun(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t pad)
      : dag_(dag), k_(k), pad_(pad), G_(dag.G) {
    mask_.resize(G_);
    weight_.resize(G_);
    for (int i = 0; i < G_; ++i) {
      mask_[i] = gates[i].mask();
      weight_[i] = __builtin_popcountll(mask_[i]) > 1 ? 1 : 0;
    }
    tin_.assign(G_, 0);
    tstamp_.assign(G_, 0);
  }

  // Parts of one run with tie-break keys from `rng` (none: the first
  // candidate wins ties).
  int run(Rng* rng, std::vector<int32_t>* part) {
    part->assign(G_, -1);
    indeg_.resize(G_);
    ready_.clear();
    for (int i = 0; i < G_; ++i) {
      indeg_[i] = (int)dag_.pred[i].size();
      if (!indeg_[i]) ready_.push_back(i);
    }
    int placed = 0, np = 0;
    std::vector<int> take;
    while (placed < G_) {
      const uint64_t Q = choose(rng);
      take.clear();
      eval(Q, &take, nullptr);
      if (take.empty()) return -1;  // cannot happen: every gate fits k with the padding
      for (int i : take) {
        (*part)[i] = np;
        for (int s : dag_.succ[i]) --indeg_[s];
      }
      placed += (int)take.size();
      ++np;
      // the new front: untaken ready gates, then successors that became ready
      next_.clear();
      for (int i : ready_)
        if ((*part)[i] < 0) next_.push_back(i);
      for (int i : take)
        for (int s : dag_.succ[i])
          if (!indeg_[s] && (*part)[s] < 0) next_.push_back(s);
      std::sort(next_.begin(), next_.end());
      next_.erase(std::unique(next_.begin(), next_.end()), next_.end());
      ready_.swap(next_);
    }
    return np;
  }

 private:
  // Weight of the closure of Q from the current front: the unplaced gates
  // on qubits in Q whose predecessors are placed or in the closure.  Lists
  // the closure in `take` and the gates just outside it (all predecessors
  // placed or taken, some qubit outside Q) in `front`.
  int eval(uint64_t Q, std::vector<int>* take, std::vector<int>* front) {
    if (++stamp_ == 0) {
      std::fill(tstamp_.begin(), tstamp_.end(), 0u);
      stamp_ = 1;
    }
    stack_.clear();
    for (int i : ready_) {
      if (!(mask_[i] & ~Q)) stack_.push_back(i);
      else if (front) front->push_back(i);
    }
    int w = 0;
    while (!stack_.empty()) {
      const int i = stack_.back();
      stack_.pop_back();
      w += weight_[i];
      if (take) take->push_back(i);
      for (int s : dag_.succ[i]) {
        if (tstamp_[s] != stamp_) {
          tstamp_[s] = stamp_;
          tin_[s] = indeg_[s];
        }
        if (--tin_[s] == 0) {
          if (!(mask_[s] & ~Q)) stack_.push_back(s);
          else if (front) front->push_back(s);
        }
      }
    }
    return w;
  }

  uint64_t choose(Rng* rng) {
    // grow: add the qubits of the frontier gate whose closure weighs most;
    // ties to fewer qubits, then to the earlier frontier gate (trial 0) or
    // the lower random key
    uint64_t Q = pad_;
    for (;;) {
      front_.clear();
      eval(Q, nullptr, &front_);
      uint64_t best = Q;
      int64_t best_s = INT64_MIN;
      uint64_t best_key = 0;
      for (size_t r = 0; r < front_.size(); ++r) {
        const int f = front_[r];
        const uint64_t c = Q | mask_[f];
        if (c == Q || __builtin_popcountll(c) > k_) continue;
        const int64_t sc = ((int64_t)eval(c, nullptr, nullptr) << 8) - __builtin_popcountll(c);
        const uint64_t key = rng ? rng->next() : (uint64_t)r;
        if (sc > best_s || (sc == best_s && key < best_key)) {
          best_s = sc;
          best = c;
          best_key = key;
        }
      }
      if (best == Q) break;
      Q = best;
    }
    // improve: exchange one qubit (never a padding qubit) while the closure
    // gains weight; the candidates to bring in are the frontier's qubits
    int cur = eval(Q, nullptr, nullptr);
    for (int round = 0; round < 4 * k_; ++round) {
      front_.clear();
      eval(Q, nullptr, &front_);
      uint64_t in = 0;
      for (int f : front_) in |= mask_[f];
      in &= ~Q;
      bool moved = false;
      for (uint64_t out = Q & ~pad_; out && !moved; out &= out - 1) {
        const uint64_t qo = out & (0 - out);
        for (uint64_t cand = in; cand; cand &= cand - 1) {
          const uint64_t Q2 = (Q & ~qo) | (cand & (0 - cand));
          const int w = eval(Q2, nullptr, nullptr);
          if (w > cur) {
            Q = Q2;
            cur = w;
            moved = true;
            break;
          }
        }
      }
      if (!moved) break;
    }
    return Q;
  }

  const Dag& dag_;
  const int k_;
  const uint64_t pad_;
  const int G_;
  std::vector<uint64_t> mask_;
  std::vector<int> weight_, indeg_, ready_, next_, front_, stack_, tin_;
  std::vector<uint32_t> tstamp_;
  uint32_t stamp_ = 0;
};
}  // namespace

// Closure partition.  A part is fixed by its qubit set Q (at most k qubits
// with the padding): it takes every unplaced gate on qubits in Q whose
// predecessors are placed or taken -- the closure of Q from the current
// front.  Q grows from the padding by the frontier gate whose qubits give
// the closure with the most two-qubit gates (fewer qubits on ties), then
// exchanges one qubit at a time, lowest bits first, while that count grows.
// One-qubit gates do not count: any later part on their qubit takes them,
// and counting them measured 2% more parts on random circuits.  Parts are
// taken in order, so every edge runs forward and the part-graph is acyclic
// (Sec. IV.A condition ii).  Trial 0 breaks the remaining ties to the
// first frontier gate (ready gates in index order, then the gates the
// closure frees, as it frees them), later trials by a seeded random key;
// the fewest parts win, ties to the lowest trial.
int partition_closure(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t seed,
                      int trials, std::vector<int32_t>* part, uint64_t pad) {
  const int T = std::max(1, trials);
  const int nthreads = std::max(1, std::min({T, 8, (int)std::thread::hardware_concurrency()}));
  std::vector<int> best_np(nthreads, -1);
  std::vector<int> best_t(nthreads, -1);
  std::vector<std::vector<int32_t>> best_part(nthreads);
  auto worker = [&](int w) {
    ClosureRun run(gates, dag, k, pad);
    std::vector<int32_t> cand;
    for (int t = w; t < T; t += nthreads) {
      Rng rng(seed * 0x100000001B3ull + 0x51ull + (uint64_t)t);
      const int np = run.run(t == 0 ? nullptr : &rng, &cand);
      if (np > 0 && (best_np[w] < 0 || np < best_np[w])) {
        best_np[w] = np;
        best_t[w] = t;
        best_part[w] = cand;
      }
    }
  };
  if (nthreads == 1 || gates.size() < 64) {
    for (int w = 0; w < nthreads; ++w) worker(w);
  } else {
    std::vector<std::thread> pool;
    for (int w = 0; w < nthreads; ++w) pool.emplace_back(worker, w);
    for (auto& th : pool) th.join();
  }
  int bw = -1;
  for (int w = 0; w < nthreads; ++w)
    if (best_np[w] > 0 && (bw < 0 || best_np[w] < best_np[bw] ||
                           (best_np[w] == best_np[bw] && best_t[w] < best_t[bw])))
      bw = w;
  if (bw < 0) return partition_nat(gates, k, part, pad);
  part->swap(best_part[bw]);
  return best_np[bw];
}

std::string check_partition(const std::vector<Gate>& gates, const Dag& dag,
                            const std::vector<int32_t>& part, int k, uint64_t pad) {
  const int G = (int)gates.size();
  if ((int)part.size() != G) return "assignment length differs from the gate count";
  if (G == 0) return "";
  int P = 0;
  for (int i = 0; i < G; ++i) {
    if (part[i] < 0) return "negative part id";
    P = std::max(P, part[i] + 1);
  }
  if (P > G) return "more parts than gates";
  std::vector<uint64_t> mask(P, 0);
  std::vector<int> cnt(P, 0);
  for (int i = 0; i < G; ++i) {
    mask[part[i]] |= gates[i].mask();
    cnt[part[i]]++;
  }
  for (int p = 0; p < P; ++p) {
    if (!cnt[p]) return "part " + std::to_string(p) + " is empty";
    if (__builtin_popcountll(mask[p] | pad) > k)
      return "part " + std::to_string(p) + (pad ? " with the padding qubits" : "") +
             " uses more than k qubits";
  }
  // Every cross-part edge must go from a lower to a higher id: then the ids
  // are a topological order of the part-graph, which is therefore acyclic.
  for (int i = 0; i < G; ++i)
    for (int j : dag.succ[i])
      if (part[i] > part[j])
        return "edge from part " + std::to_string(part[i]) + " back to part " +
               std::to_string(part[j]);
  return "";
}

}  // namespace hisv
