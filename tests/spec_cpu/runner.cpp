// Host runner for generated part kernels (test infrastructure).
//
//   runner <state.bin> <launches.txt>
//
// state.bin holds the 2^n interleaved amplitudes (complex64 or complex128,
// matching the kernels) and is updated in place.  Each line of
// launches.txt is "part grid block tiles xcd": kernel `part` (declared by
// the included parts.inc as part_kernel(int)) runs with `grid` workgroups
// of `block` threads over `tiles` tiles.  The state lives in its own heap
// block, so AddressSanitizer reports any access outside it.
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "prelude.h"
#include "parts.inc"  // generated: the kernels and `launch_part(part, state, tiles, xcd)`

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: runner state.bin launches.txt\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  std::fseek(f, 0, SEEK_END);
  const long bytes = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  std::vector<unsigned char> state(bytes);
  if (std::fread(state.data(), 1, bytes, f) != (size_t)bytes) return 4;
  std::fclose(f);
  FILE* l = std::fopen(argv[2], "r");
  if (!l) return 5;
  int part;
  unsigned grid, block, xcd;
  unsigned long long tiles;
  while (std::fscanf(l, "%d %u %u %llu %u", &part, &grid, &block, &tiles, &xcd) == 5) {
    gridDim.x = grid;
    for (unsigned b = 0; b < grid; ++b) {
      std::barrier<> bar(block);
      cpu_block_barrier = &bar;
      std::vector<std::thread> th;
      for (unsigned t = 0; t < block; ++t)
        th.emplace_back([&, b, t] {
          blockIdx.x = b;
          threadIdx.x = t;
          launch_part(part, state.data(), tiles, xcd);
        });
      for (auto& x : th) x.join();
    }
  }
  std::fclose(l);
  f = std::fopen(argv[1], "wb");
  if (!f || std::fwrite(state.data(), 1, bytes, f) != (size_t)bytes) return 6;
  std::fclose(f);
  return 0;
}
