// Host runner for the partitioners under AddressSanitizer / UBSan or
// ThreadSanitizer (test infrastructure; links the library's partitioning
// sources, not the library).
//
//   partition_runner <circuit.txt> <jobs.txt>
//
// circuit.txt: "n G" then G lines "kind q0 q1" (q1 = -1 for one-qubit
// gates).  jobs.txt: lines "strategy k seed trials pad_qubits" with strategy
// one of nat dfs dagp greedy closure.  For each job it prints "parts" and
// whether the partition passes the exact validity check ("ok" or the
// violation).
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hisv_internal.h"

namespace hisv {
// the library's hs_tune("host_threads"): four helper threads here
int host_threads() { return 4; }
int serve_chunk_parts() { return 8; }
}  // namespace hisv

using namespace hisv;

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: partition_runner circuit.txt jobs.txt\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "r");
  if (!f) return 3;
  int n = 0, G = 0;
  if (std::fscanf(f, "%d %d", &n, &G) != 2) return 4;
  std::vector<Gate> gates(G);
  for (Gate& g : gates) {
    g = Gate{};
    if (std::fscanf(f, "%d %d %d", &g.kind, &g.q0, &g.q1) != 3) return 5;
  }
  std::fclose(f);
  const Dag dag = build_dag(gates);
  FILE* j = std::fopen(argv[2], "r");
  if (!j) return 6;
  char name[32];
  int k = 0, trials = 0, padq = 0;
  unsigned long long seed = 0;
  while (std::fscanf(j, "%31s %d %llu %d %d", name, &k, &seed, &trials, &padq) == 5) {
    const uint64_t pad = padq ? (uint64_t(1) << padq) - 1 : 0;
    std::vector<int32_t> part;
    int parts = -1;
    const std::string s = name;
    if (s == "nat") parts = partition_nat(gates, k, &part, pad);
    else if (s == "dfs") parts = partition_dfs(gates, dag, k, seed, trials, &part, pad);
    else if (s == "dagp") parts = partition_dagp(gates, dag, n, k, seed, &part, pad);
    else if (s == "greedy") parts = partition_greedy(gates, dag, k, seed, trials, &part, pad);
    else if (s == "closure") parts = partition_closure(gates, dag, k, trials, &part, pad);
    else return 7;
    const std::string why = check_partition(gates, dag, part, k, pad);
    std::printf("%s %d %llu %d %d %d %s\n", name, k, seed, trials, padq, parts,
                why.empty() ? "ok" : why.c_str());
  }
  std::fclose(j);
  return 0;
}
