// CPU stand-ins for the HIP constructs used by the generated part kernels,
// so the exact kernel source can run on the host (test infrastructure).
// Every GPU thread of a workgroup is a std::thread; a workgroup's threads run
// concurrently and meet at a std::barrier where the kernel calls
// __syncthreads(); workgroups run one after another, so a function-static
// array stands in for the workgroup's LDS.
#pragma once
#include <barrier>
#include <cstdint>

#define __device__
#define __global__
#define __launch_bounds__(x)
#define __shared__ static
#define __restrict__

struct cpu_dim3 {
  unsigned x = 0, y = 0, z = 0;
};
inline thread_local cpu_dim3 threadIdx;
inline thread_local cpu_dim3 blockIdx;
inline cpu_dim3 gridDim;
inline std::barrier<>* cpu_block_barrier = nullptr;

inline void __syncthreads() { cpu_block_barrier->arrive_and_wait(); }
#define __builtin_amdgcn_readfirstlane(v) (v)
