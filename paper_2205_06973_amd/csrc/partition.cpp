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
#include <atomic>
#include <memory>
#include <stdexcept>
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
// Closure parts and the beam search over them (see partition_closure).
class ClosureSearch {
 public:
  // The parts taken so far, newest first (shared between beam nodes).
  struct History {
    mutable std::shared_ptr<const History> prev;
    std::vector<int> gates;
    ~History() {  // unlink a long chain iteratively, not by recursion
      std::shared_ptr<const History> p = std::move(prev);
      while (p && p.use_count() == 1) p = std::move(p->prev);
    }
  };
  // A partial partition: the gates placed so far.  Its size is O(G / 64 +
  // front), so extending a beam node costs little on long circuits.
  struct Node {
    std::vector<uint64_t> placed;          // bit per gate
    std::vector<int> ready;                // unplaced gates whose predecessors are placed, ascending
    std::shared_ptr<const History> parts;  // the parts, newest first
    int count = 0;                         // gates placed
    int nparts = 0;
    int weight = 0;                        // two-qubit gates placed
    uint64_t key = 0;                      // XOR of the placed gates' random keys
    bool is_placed(int i) const { return placed[i >> 6] >> (i & 63) & 1; }
  };

  ClosureSearch(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t pad)
      : dag_(dag), k_(k), pad_(pad), G_(dag.G) {
    mask_.resize(G_);
    weight_.resize(G_);
    for (int i = 0; i < G_; ++i) {
      mask_[i] = gates[i].mask();
      weight_[i] = __builtin_popcountll(mask_[i]) > 1 ? 1 : 0;
    }
    tin_.assign(G_, 0);
    tstamp_.assign(G_, 0);
    zkey_.resize(G_);
    Rng rng(0x5a17u);
    for (int i = 0; i < G_; ++i) zkey_[i] = rng.next();
  }

  Node root() const {
    Node r;
    r.placed.assign((G_ + 63) / 64, 0);
    for (int i = 0; i < G_; ++i)
      if (dag_.pred[i].empty()) r.ready.push_back(i);
    return r;
  }

  // part id per gate of a complete partition
  static void assign(const Node& nd, std::vector<int32_t>* part) {
    int id = nd.nparts;
    for (const History* h = nd.parts.get(); h; h = h->prev.get()) {
      --id;
      for (int i : h->gates) (*part)[i] = id;
    }
  }

  // Up to m distinct qubit sets for the next part of `nd`: the m best
  // first steps of the growth, each grown and improved (m = 1: the plain
  // closure rule).
  void candidates(const Node& nd, int m, std::vector<uint64_t>* out) {
    cur_ = &nd;
    out->clear();
    front_.clear();
    eval(pad_, nullptr, &front_);
    struct Seed {
      int64_t sc;
      uint64_t set;
    };
    std::vector<Seed> seeds;  // in front order, so the stable sort breaks ties to the earlier gate
    for (int f : front_) {
      const uint64_t c = pad_ | mask_[f];
      if (c == pad_ || __builtin_popcountll(c) > k_) continue;
      bool dup = false;
      for (const Seed& e : seeds) dup |= e.set == c;
      if (dup) continue;
      seeds.push_back({score(c), c});
    }
    std::stable_sort(seeds.begin(), seeds.end(), [](const Seed& x, const Seed& y) { return x.sc > y.sc; });
    if (seeds.empty()) seeds.push_back({0, pad_});
    for (size_t i = 0; i < seeds.size() && (int)out->size() < m; ++i) {
      const uint64_t Q = improve(grow(seeds[i].set));
      if (std::find(out->begin(), out->end(), Q) == out->end()) out->push_back(Q);
    }
  }

  // `nd` with the closure of Q placed as its next part.
  Node apply(const Node& nd, uint64_t Q) {
    cur_ = &nd;
    take_.clear();
    eval(Q, &take_, nullptr);
    Node r;
    r.placed = nd.placed;
    r.count = nd.count + (int)take_.size();
    r.nparts = nd.nparts + 1;
    r.weight = nd.weight;
    r.key = nd.key;
    for (int i : take_) {
      r.placed[i >> 6] |= uint64_t(1) << (i & 63);
      r.weight += weight_[i];
      r.key ^= zkey_[i];
    }
    auto h = std::make_shared<History>();
    h->prev = nd.parts;
    h->gates = take_;
    r.parts = std::move(h);
    for (int i : nd.ready)
      if (!r.is_placed(i)) r.ready.push_back(i);
    for (int i : take_)
      for (int s : dag_.succ[i]) {
        if (r.is_placed(s)) continue;
        bool ok = true;
        for (int q : dag_.pred[s]) ok &= r.is_placed(q);
        if (ok) r.ready.push_back(s);
      }
    std::sort(r.ready.begin(), r.ready.end());
    r.ready.erase(std::unique(r.ready.begin(), r.ready.end()), r.ready.end());
    return r;
  }

  int gates() const { return G_; }

 private:
  // Two-qubit weight of the closure of Q from the current node's front: the
  // unplaced gates on qubits in Q whose predecessors are placed or taken.
  // Lists the closure in `take` and the gates just outside it (predecessors
  // placed or taken, a qubit outside Q) in `front`, in the order found.
  int eval(uint64_t Q, std::vector<int>* take, std::vector<int>* front) {
    if (++stamp_ == 0) {
      std::fill(tstamp_.begin(), tstamp_.end(), 0u);
      stamp_ = 1;
    }
    stack_.clear();
    for (int i : cur_->ready) {
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
        if (tstamp_[s] != stamp_) {  // its unplaced predecessors (at most one per qubit)
          tstamp_[s] = stamp_;
          int u = 0;
          for (int q : dag_.pred[s]) u += !cur_->is_placed(q);
          tin_[s] = u;
        }
        if (--tin_[s] == 0) {
          if (!(mask_[s] & ~Q)) stack_.push_back(s);
          else if (front) front->push_back(s);
        }
      }
    }
    return w;
  }

  // closure weight first, then fewer qubits
  int64_t score(uint64_t Q) { return ((int64_t)eval(Q, nullptr, nullptr) << 8) - __builtin_popcountll(Q); }

  // Add the qubits of the frontier gate whose closure scores best (ties to
  // the earlier frontier gate) while any fits.
  uint64_t grow(uint64_t Q) {
    for (;;) {
      front_.clear();
      eval(Q, nullptr, &front_);
      uint64_t best = Q;
      int64_t best_s = INT64_MIN;
      for (int f : front_) {
        const uint64_t c = Q | mask_[f];
        if (c == Q || __builtin_popcountll(c) > k_) continue;
        const int64_t sc = score(c);
        if (sc > best_s) {
          best_s = sc;
          best = c;
        }
      }
      if (best == Q) return Q;
      Q = best;
    }
  }

  // Exchange one qubit (never a padding qubit; lowest bits first) for one of
  // the frontier's while the closure gains weight.
  uint64_t improve(uint64_t Q) {
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
  const Node* cur_ = nullptr;
  std::vector<uint64_t> mask_, zkey_;
  std::vector<int> weight_, front_, take_, stack_, tin_;
  std::vector<uint32_t> tstamp_;
  uint32_t stamp_ = 0;
};
}  // namespace

// Closure partition.  A part is fixed by its qubit set Q (at most k qubits
// with the padding): it takes every unplaced gate on qubits in Q whose
// predecessors are placed or taken -- the closure of Q from the current
// front.  Q grows from the padding by the frontier gate whose qubits give
// the closure with the most two-qubit gates (fewer qubits, then the earlier
// frontier gate on ties), then exchanges one qubit at a time while that
// count grows.  One-qubit gates do not count: any later part on their qubit
// takes them, and counting them measured 2% more parts on random circuits.
// Parts are taken in order, so every edge runs forward and the part-graph
// is acyclic (Sec. IV.A condition ii).
//
// `width` > 1 runs a beam search: each of the `width` best partial
// partitions (most two-qubit gates placed, then most gates) is extended by
// up to six parts -- the growth started from each of its six best first
// gates -- and the first partition to place every gate wins, unless the
// plain rule (width 1) needs fewer parts.  The result does not depend on
// the number of host threads.
int partition_closure(const std::vector<Gate>& gates, const Dag& dag, int k, int width,
                      std::vector<int32_t>* part, uint64_t pad) {
  using Node = ClosureSearch::Node;
  if (dag.G == 0) {
    part->clear();
    return 0;
  }
  const int B = std::max(1, width);
  const int M = B > 1 ? 6 : 1;
  // the beam's expansions run on up to 8 host threads (hs_tune "host_threads")
  const int want = host_threads();
  const int T = std::max(1, std::min(B, want > 0 ? want : std::min(8, (int)std::thread::hardware_concurrency())));
  std::vector<ClosureSearch> cs(T, ClosureSearch(gates, dag, k, pad));
  std::vector<Node> beam{cs[0].root()};
  std::vector<std::vector<Node>> grown(B);
  std::vector<std::vector<uint64_t>> qs(T);
  int result = -1;
  bool done = false;

  // nodes are taken from a shared counter; node i's expansions go to
  // grown[i] whichever thread makes them, so the result is the same
  std::atomic<size_t> next_node{0};
  auto expand = [&](int t) {
    for (size_t i; (i = next_node.fetch_add(1, std::memory_order_relaxed)) < beam.size();) {
      cs[t].candidates(beam[i], M, &qs[t]);
      grown[i].clear();
      for (uint64_t Q : qs[t]) grown[i].push_back(cs[t].apply(beam[i], Q));
    }
  };
  // the best `B` distinct expansions become the next beam; the first that
  // places every gate ends the search
  auto select = [&]() {
    next_node.store(0, std::memory_order_relaxed);
    std::vector<Node> next;
    for (size_t i = 0; i < beam.size(); ++i)
      for (auto& nd : grown[i]) next.push_back(std::move(nd));
    std::stable_sort(next.begin(), next.end(), [](const Node& x, const Node& y) {
      return x.weight != y.weight ? x.weight > y.weight : x.count > y.count;
    });
    for (auto& nd : next)
      if (nd.count == dag.G) {
        part->assign(dag.G, -1);
        ClosureSearch::assign(nd, part);
        result = nd.nparts;
        done = true;
        return;
      }
    if (next.empty()) {  // cannot happen: every gate fits k with the padding
      done = true;
      return;
    }
    beam.clear();
    for (auto& nd : next) {
      bool dup = false;
      for (const auto& b : beam)
        if (b.key == nd.key && b.count == nd.count && b.placed == nd.placed) {
          dup = true;
          break;
        }
      if (dup) continue;
      beam.push_back(std::move(nd));
      if ((int)beam.size() == B) break;
    }
  };

  auto alone = [&]() {
    while (!done) {
      expand(0);
      select();
    }
  };
  if (T == 1) {
    alone();
  } else {
    // a spinning barrier: a level's work is a fraction of a millisecond,
    // about what waking a sleeping thread costs
    struct Barrier {
      std::atomic<int> count{0};
      std::atomic<uint64_t> gen{0};
      const int n;
      explicit Barrier(int n_) : n(n_) {}
      void wait() {
        const uint64_t g = gen.load(std::memory_order_acquire);
        if (count.fetch_add(1, std::memory_order_acq_rel) == n - 1) {
          count.store(0, std::memory_order_relaxed);
          gen.fetch_add(1, std::memory_order_release);
        } else {
          while (gen.load(std::memory_order_acquire) == g) std::this_thread::yield();
        }
      }
    } bar(T);
    // an exception on any thread ends the search for all of them (after the
    // level's barrier) and is raised again on the calling thread
    std::atomic<int> failed{HS_OK};
    auto team = [&](int t) {
      for (;;) {
        hs_status rc = guarded([&] {
          expand(t);
          return HS_OK;
        });
        if (rc != HS_OK) failed.store(rc);
        bar.wait();
        if (t == 0) {
          if (failed.load() == HS_OK && (rc = guarded([&] {
                                           select();
                                           return HS_OK;
                                         })) != HS_OK)
            failed.store(rc);
          if (failed.load() != HS_OK) done = true;
        }
        bar.wait();
        if (done) return;
      }
    };
    // the helpers start only once all of them exist; if one cannot be
    // started, the others leave and the search runs on this thread alone
    std::atomic<int> go{0};
    std::vector<std::thread> pool;
    pool.reserve(T - 1);
    try {
      for (int t = 1; t < T; ++t)
        pool.emplace_back([&, t] {
          while (go.load(std::memory_order_acquire) == 0) std::this_thread::yield();
          if (go.load(std::memory_order_acquire) > 0) team(t);
        });
    } catch (...) {
      go.store(-1, std::memory_order_release);
      for (auto& th : pool) th.join();
      pool.clear();
    }
    if (pool.size() + 1 == (size_t)T) {
      go.store(1, std::memory_order_release);
      team(0);
      for (auto& th : pool) th.join();
      if (failed.load() == HS_E_NOMEM) throw std::bad_alloc();
      if (failed.load() != HS_OK) throw std::runtime_error("closure search failed on a host thread");
    } else {
      alone();
    }
  }
  if (result < 0) return partition_nat(gates, k, part, pad);
  if (B > 1) {  // never more parts than the plain rule
    std::vector<int32_t> plain;
    const int np = partition_closure(gates, dag, k, 1, &plain, pad);
    if (np < result) {
      part->swap(plain);
      result = np;
    }
  }
  return result;
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
