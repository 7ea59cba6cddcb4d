// kernels.hip -- gfx950 kernels of the partitioned state-vector path.
//
//   part_pass_kernel   Alg. 1 (Sec. III.C) for one part, in place: each
//                      workgroup gathers tiles (one outer setting each) from
//                      HBM into registers with coalesced loads, runs the
//                      part's register stages (LDS re-layouts in between) and
//                      scatters the tile back -- one HBM read and one write
//                      per amplitude per part.
//   gate_pass_1q/2q    the non-hierarchical case (Sec. III.A-B): one full
//                      sweep of the state per gate.
//   set_basis, norm, probabilities/amplitude readout, copy probe.
//
// Amplitudes are interleaved complex (float2 / double2), index bit q =
// qubit q.  complex64 states compute in FP32, complex128 in FP64; the norm
// and probabilities are accumulated in FP64 for both.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <map>
#include <type_traits>

#include "hisv_internal.h"

namespace hisv {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

// ---------------------------------------------------------------------------
// register operations (one lane's 2^RB amplitudes; bit positions compile-time)
// ---------------------------------------------------------------------------
template <int N>
using IC = std::integral_constant<int, N>;

template <int RB, typename F>
__device__ __forceinline__ void for_bit(int b, F&& f) {
  switch (b) {
    case 0: if constexpr (RB > 0) { f(IC<0>{}); break; } else __builtin_unreachable();
    case 1: if constexpr (RB > 1) { f(IC<1>{}); break; } else __builtin_unreachable();
    case 2: if constexpr (RB > 2) { f(IC<2>{}); break; } else __builtin_unreachable();
    case 3: if constexpr (RB > 3) { f(IC<3>{}); break; } else __builtin_unreachable();
    case 4: if constexpr (RB > 4) { f(IC<4>{}); break; } else __builtin_unreachable();
    case 5: if constexpr (RB > 5) { f(IC<5>{}); break; } else __builtin_unreachable();
    default: __builtin_unreachable();
  }
}

template <int RB, typename F>
__device__ __forceinline__ void for_pair(int b0, int b1, F&& f) {
  for_bit<RB>(b0, [&](auto B0) __attribute__((always_inline)) {
    for_bit<RB>(b1, [&](auto B1) __attribute__((always_inline)) {
      if constexpr (decltype(B0)::value != decltype(B1)::value) f(B0, B1);
      else __builtin_unreachable();
    });
  });
}

// A lane's 2^RB amplitudes (re at 2j, im at 2j+1).  Every access below has
// a compile-time index, so the array is split into independent scalars that
// stay in VGPRs.  (A vector value did the same but must occupy one
// contiguous register range, which cost extra register copies per op:
// 1,643 against 1,109 moves in the complex64 kernel, 2.4% on a 28-qubit
// layered circuit.)
template <typename T, int RB>
struct RegV {
  T v[2 << RB];
  __device__ __forceinline__ T& operator[](int i) { return v[i]; }
  __device__ __forceinline__ const T& operator[](int i) const { return v[i]; }
};

// Every register operation reads one register set (a) and writes every
// register of another (b).  The interpreter alternates the two sets from op
// to op, so the switch over op kinds leaves its results where the next op
// reads them.  (Updating one set in place made the compiler assign each
// case's results to fresh registers and copy the whole set back after
// every op: 32 moves per op for complex64 with 16 amplitudes a lane.)
template <typename T>
__device__ __forceinline__ void cmul(cplx<T>& v, T cr, T ci) {
  const cplx<T> p = v;
  v.x = p.x * cr - p.y * ci;
  v.y = p.x * ci + p.y * cr;
}

// A register copy.  The empty asm keeps the compiler from merging the
// copies of different cases (different register indices) into copies
// through a selected address, which would move the register set to memory.
template <typename T, int RB>
__device__ __forceinline__ void cp_at(const RegV<T, RB>& a, RegV<T, RB>& b, int j, int k) {
  T x = a[2 * k], y = a[2 * k + 1];
  asm volatile("" : "+v"(x), "+v"(y));
  b[2 * j] = x;
  b[2 * j + 1] = y;
}

template <typename T, int RB>
__device__ __forceinline__ void cmul_at(const RegV<T, RB>& a, RegV<T, RB>& b, int j, T cr, T ci) {
  const T px = a[2 * j], py = a[2 * j + 1];
  b[2 * j] = px * cr - py * ci;
  b[2 * j + 1] = px * ci + py * cr;
}

template <typename T, int RB, int B>
__device__ __forceinline__ void r_u(const RegV<T, RB>& a, RegV<T, RB>& b, const T* __restrict__ c) {
  const T u00r = c[0], u00i = c[1], u01r = c[2], u01i = c[3];
  const T u10r = c[4], u10i = c[5], u11r = c[6], u11i = c[7];
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const T px = a[2 * j], py = a[2 * j + 1], qx = a[2 * k], qy = a[2 * k + 1];
    b[2 * j] = u00r * px - u00i * py + u01r * qx - u01i * qy;
    b[2 * j + 1] = u00r * py + u00i * px + u01r * qy + u01i * qx;
    b[2 * k] = u10r * px - u10i * py + u11r * qx - u11i * qy;
    b[2 * k + 1] = u10r * py + u10i * px + u11r * qy + u11i * qx;
  }
}

template <typename T, int RB, int B>
__device__ __forceinline__ void r_r(const RegV<T, RB>& a, RegV<T, RB>& b, const T* __restrict__ c) {
  const T u00 = c[0], u01 = c[1], u10 = c[2], u11 = c[3];
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const T px = a[2 * j], py = a[2 * j + 1], qx = a[2 * k], qy = a[2 * k + 1];
    b[2 * j] = u00 * px + u01 * qx;
    b[2 * j + 1] = u00 * py + u01 * qy;
    b[2 * k] = u10 * px + u11 * qx;
    b[2 * k + 1] = u10 * py + u11 * qy;
  }
}

template <typename T, int RB, int B>
__device__ __forceinline__ void r_d(const RegV<T, RB>& a, RegV<T, RB>& b, const T* __restrict__ c) {
  const T d0r = c[0], d0i = c[1], d1r = c[2], d1i = c[3];
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    if (j & (1 << B)) cmul_at<T, RB>(a, b, j, d1r, d1i);
    else cmul_at<T, RB>(a, b, j, d0r, d0i);
  }
}

template <typename T, int RB, int B>
__device__ __forceinline__ void r_d1(const RegV<T, RB>& a, RegV<T, RB>& b, const T* __restrict__ c) {
  const T d1r = c[0], d1i = c[1];
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    if (j & (1 << B)) cmul_at<T, RB>(a, b, j, d1r, d1i);
    else cp_at<T, RB>(a, b, j, j);
  }
}

template <typename T, int RB, int B>
__device__ __forceinline__ void r_x(const RegV<T, RB>& a, RegV<T, RB>& b) {
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) cp_at<T, RB>(a, b, j, j ^ (1 << B));
}

template <typename T, int RB, int C, int G>
__device__ __forceinline__ void r_cx(const RegV<T, RB>& a, RegV<T, RB>& b) {
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) cp_at<T, RB>(a, b, j, (j & (1 << C)) ? j ^ (1 << G) : j);
}

template <typename T, int RB, int B0, int B1>
__device__ __forceinline__ void r_swap(const RegV<T, RB>& a, RegV<T, RB>& b) {
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    const int k = ((j >> B0 & 1) != (j >> B1 & 1)) ? j ^ (1 << B0) ^ (1 << B1) : j;
    cp_at<T, RB>(a, b, j, k);
  }
}

template <typename T, int RB, int B0, int B1>
__device__ __forceinline__ void r_cz(const RegV<T, RB>& a, RegV<T, RB>& b) {
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    if ((j & (1 << B0)) && (j & (1 << B1))) {
      b[2 * j] = -a[2 * j];
      b[2 * j + 1] = -a[2 * j + 1];
    } else {
      cp_at<T, RB>(a, b, j, j);
    }
  }
}

template <typename T, int RB, int B0, int B1>
__device__ __forceinline__ void r_cp(const RegV<T, RB>& a, RegV<T, RB>& b, const T* __restrict__ c) {
  const T cr = c[0], ci = c[1];
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    if ((j & (1 << B0)) && (j & (1 << B1))) cmul_at<T, RB>(a, b, j, cr, ci);
    else cp_at<T, RB>(a, b, j, j);
  }
}

// Dense 4 x 4 on bits B0 < B1: y = M x over every quad of amplitudes that
// differ only in those bits (index within the quad = bit B0 + 2 bit B1).
template <typename T, int RB, int B0, int B1>
__device__ __forceinline__ void r_u2(const RegV<T, RB>& a, RegV<T, RB>& b, const T* __restrict__ c) {
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    if ((j >> B0 & 1) || (j >> B1 & 1)) continue;
    const int ix[4] = {j, j | (1 << B0), j | (1 << B1), j | (1 << B0) | (1 << B1)};
    T xr[4], xi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xr[q] = a[2 * ix[q]];
      xi[q] = a[2 * ix[q] + 1];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T* m = c + 8 * i;
      T yr = m[0] * xr[0] - m[1] * xi[0];
      T yi = m[0] * xi[0] + m[1] * xr[0];
#pragma unroll
      for (int k = 1; k < 4; ++k) {
        yr += m[2 * k] * xr[k] - m[2 * k + 1] * xi[k];
        yi += m[2 * k] * xi[k] + m[2 * k + 1] * xr[k];
      }
      b[2 * ix[i]] = yr;
      b[2 * ix[i] + 1] = yi;
    }
  }
}

// b = op(a).
template <typename T, int RB>
__device__ __forceinline__ void apply_op(const RegV<T, RB>& a, RegV<T, RB>& b,
                                         const OpDesc<T>* __restrict__ op) {
  const int kind = __builtin_amdgcn_readfirstlane(op->kind);
  const int b0 = __builtin_amdgcn_readfirstlane(op->b0);
  const int b1 = __builtin_amdgcn_readfirstlane(op->b1);
  const T* c = op->c;
  switch (kind) {
    case OP_U: for_bit<RB>(b0, [&](auto B) __attribute__((always_inline)) { r_u<T, RB, decltype(B)::value>(a, b, c); }); break;
    case OP_R: for_bit<RB>(b0, [&](auto B) __attribute__((always_inline)) { r_r<T, RB, decltype(B)::value>(a, b, c); }); break;
    case OP_D: for_bit<RB>(b0, [&](auto B) __attribute__((always_inline)) { r_d<T, RB, decltype(B)::value>(a, b, c); }); break;
    case OP_D1: for_bit<RB>(b0, [&](auto B) __attribute__((always_inline)) { r_d1<T, RB, decltype(B)::value>(a, b, c); }); break;
    case OP_X: for_bit<RB>(b0, [&](auto B) __attribute__((always_inline)) { r_x<T, RB, decltype(B)::value>(a, b); }); break;
    case OP_CX:
      for_pair<RB>(b0, b1, [&](auto B0, auto B1) __attribute__((always_inline)) {
        r_cx<T, RB, decltype(B0)::value, decltype(B1)::value>(a, b);
      });
      break;
    case OP_CZ:
      for_pair<RB>(b0, b1, [&](auto B0, auto B1) __attribute__((always_inline)) {
        r_cz<T, RB, decltype(B0)::value, decltype(B1)::value>(a, b);
      });
      break;
    case OP_CP:
      for_pair<RB>(b0, b1, [&](auto B0, auto B1) __attribute__((always_inline)) {
        r_cp<T, RB, decltype(B0)::value, decltype(B1)::value>(a, b, c);
      });
      break;
    case OP_SWAP:
      for_pair<RB>(b0, b1, [&](auto B0, auto B1) __attribute__((always_inline)) {
        r_swap<T, RB, decltype(B0)::value, decltype(B1)::value>(a, b);
      });
      break;
    case OP_U2:
      if constexpr (RB >= 2) {
        for_pair<RB>(b0, b1, [&](auto B0, auto B1) __attribute__((always_inline)) {
          if constexpr (decltype(B0)::value < decltype(B1)::value)
            r_u2<T, RB, decltype(B0)::value, decltype(B1)::value>(a, b, c);
          else
            __builtin_unreachable();
        });
        break;
      } else {
        __builtin_unreachable();
      }
    default: __builtin_unreachable();
  }
}

// LDS swizzle width: the bank window holds 2^sw amplitudes (128 B).
template <typename T>
constexpr int lds_sw() { return sizeof(T) == 4 ? 4 : 3; }

// Sum of the per-bit offsets selected by the bits of v (global offsets);
// masks rather than branches, since v is per lane.
template <int N>
__device__ __forceinline__ uint64_t bit_sum(const uint64_t* w, uint32_t v) {
  uint64_t s = 0;
#pragma unroll
  for (int c = 0; c < N; ++c) s += w[c] & (uint64_t(0) - uint64_t(v >> c & 1u));
  return s;
}

// XOR of the per-bit LDS offsets selected by the bits of v.
template <int N>
__device__ __forceinline__ uint32_t bit_xor(const uint32_t* w, uint32_t v) {
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < N; ++c) s ^= w[c] & (0u - (v >> c & 1u));
  return s;
}

// Base index of a tile: the outer setting `tile` with a zero bit inserted at
// every tile qubit (Alg. 1: the amplitudes of one outer setting).
__device__ __forceinline__ uint64_t tile_base32(uint64_t tile, const int32_t* tq, int m) {
  uint64_t b = tile;
  for (int i = 0; i < m; ++i) {
    const int q = tq[i];
    const uint64_t low = b & ((uint64_t(1) << q) - 1);
    b = ((b >> q) << (q + 1)) | low;
  }
  return b;
}

// Move the tile between HBM and registers.  `p` is the lane's address of
// register 0; register j adds the (uniform) offsets of its register bits.
template <typename T, int RB, bool STORE>
__device__ __forceinline__ void tile_io(cplx<T>* p, RegV<T, RB>& a, const uint64_t* reg) {
#pragma unroll
  for (int j = 0; j < (1 << RB); ++j) {
    cplx<T>* q = p + bit_sum<RB>(reg, (uint32_t)j);
    if constexpr (STORE) {
      cplx<T> v;
      v.x = a[2 * j];
      v.y = a[2 * j + 1];
      *q = v;
    } else {
      const cplx<T> v = *q;
      a[2 * j] = v.x;
      a[2 * j + 1] = v.y;
    }
  }
}

// ---------------------------------------------------------------------------
// part-pass kernel (Alg. 1 for one part), interpreting the part's ops
// ---------------------------------------------------------------------------
template <typename T, int RB>
__global__ void __launch_bounds__(1024)
part_pass_kernel(cplx<T>* __restrict__ st, const IPart* __restrict__ pd,
                 const IStage* __restrict__ sd, const OpDesc<T>* __restrict__ ops, uint32_t xcd) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NR = 1 << RB;
  const int m = pd->m;
  const int ne = pd->n_stages;
  const uint64_t tiles = pd->tiles;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool active = lane < (1u << pd->lb);

  // Tile-independent parts of the addresses.  Bits a layout lacks have zero
  // offsets, so lanes beyond the tile's lane bits stay in bounds.
  uint64_t ld_lane = bit_sum<kLaneBits>(pd->load.lane, lane) +
                           bit_sum<kMaxWaveBits>(pd->load.wave, wave);
  uint64_t sv_lane = bit_sum<kLaneBits>(pd->store.lane, lane) +
                           bit_sum<kMaxWaveBits>(pd->store.wave, wave);
  const uint32_t slot0 = bit_xor<kLaneBits>(sd[0].lane, lane) ^ bit_xor<kMaxWaveBits>(sd[0].wave, wave);
  // opaque: each stays one register value (otherwise the compiler keeps the
  // per-bit terms live across the tile loop and re-adds them per tile)
  asm volatile("" : "+v"(ld_lane), "+v"(sv_lane));

  // Tiles of this workgroup: with xcd set (grid and tile count multiples of
  // 8), XCD x = blockIdx % 8 sweeps the contiguous run [x T/8, (x+1) T/8).
  uint64_t tile = blockIdx.x, step = gridDim.x, end = tiles;
  if (xcd) {
    const uint64_t per = tiles >> 3;
    const uint32_t x = blockIdx.x & 7u;
    tile = x * per + (blockIdx.x >> 3);
    step = gridDim.x >> 3;
    end = (x + 1) * per;
  }
  // (no software prefetch of the next tile: with up to 1024 threads a lane
  // has 128 VGPRs, and a second tile's registers would spill)
  RegV<T, RB> a, b;
  for (; tile < end; tile += step) {
    cplx<T>* const base = st + tile_base32(tile, pd->tq, m);
    if (active) tile_io<T, RB, false>(base + ld_lane, a, pd->load.reg);
    // ---- execute: stages, re-laid out through LDS where the layout changes
    uint32_t slot = slot0;  // this lane's LDS offset in the current layout
    // an opaque copy of the lane index: keeps the per-bit lane masks of the
    // re-layouts from being hoisted out of the tile loop into live registers
    uint32_t ln = lane;
    asm volatile("" : "+v"(ln));
    for (int s = 1; s < ne; ++s) {
      const IStage& e = sd[s];
      if (e.transition) {
        const IStage& f = sd[s - 1];
        __syncthreads();
        if (active) {
#pragma unroll
          for (int j = 0; j < NR; ++j) {
            cplx<T> v;
            v.x = a[2 * j];
            v.y = a[2 * j + 1];
            *reinterpret_cast<cplx<T>*>(smem_raw + (slot ^ bit_xor<RB>(f.reg, (uint32_t)j))) = v;
          }
        }
        __syncthreads();
        slot = bit_xor<kLaneBits>(e.lane, ln) ^ bit_xor<kMaxWaveBits>(e.wave, wave);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          const cplx<T> v =
              *reinterpret_cast<const cplx<T>*>(smem_raw + (slot ^ bit_xor<RB>(e.reg, (uint32_t)j)));
          a[2 * j] = v.x;
          a[2 * j + 1] = v.y;
        }
      }
      // two ops an iteration: a -> b, then b -> a
      const int o1 = e.op_end;
      int o = e.op_begin;
      for (; o + 1 < o1; o += 2) {
        apply_op<T, RB>(a, b, ops + o);
        apply_op<T, RB>(b, a, ops + o + 1);
      }
      if (o < o1) {
        apply_op<T, RB>(a, b, ops + o);
        a = b;
      }
    }
    // ---- scatter (last entry is the store layout)
    if (active) tile_io<T, RB, true>(base + sv_lane, a, pd->store.reg);
  }
}

// ---------------------------------------------------------------------------
// fused part-pass kernel: one dense unitary per part on matrix cores
// ---------------------------------------------------------------------------
// For a part on w qubits (w = 4 or 5) every outer setting is a column of X
// (2^w rows, one per setting of the part's qubits); Y = U X for all columns.
// A wavefront takes 16 columns at a time -- the settings of the 4 lowest
// other qubits, so column runs are contiguous -- and computes the complex
// product as four real products on 16x16x4 MFMA tiles:
//   Yr = Ur Xr - Ui Xi,  Yi = Ur Xi + Ui Xr.
// (Gauss's three-product form, T3 = (Ur + Ui)(Xr + Xi), measured no faster
// for w = 4, 5 on 30-qubit states: those widths wait on memory, not on the
// matrix cores.)
// Operand layouts of the 16x16x4 MFMA (64 lanes, l = lane):
//   A[i][k]: i = l % 16, k = l / 16;   B[k][j]: j = l % 16, k = l / 16;
//   D[i][j] (4 registers v): j = l % 16 and
//     i = 4 * (l / 16) + v  for the FP32 instruction,
//     i = l / 16 + 4 * v    for the FP64 instruction
// (checked on gfx950 with a probe that feeds lane numbers through A and B).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// deposit the low bits of v onto the listed qubits
__device__ __forceinline__ uint64_t deposit(uint32_t v, const int8_t* q, int count) {
  uint64_t g = 0;
  for (int b = 0; b < count; ++b) g |= uint64_t((v >> b) & 1u) << q[b];
  return g;
}

// U arrives in fragment order: fragment f = rb * (2^w / 4) + ks holds, in lane
// l, U[16 rb + l % 16][4 ks + l / 16]; the real parts of all fragments come
// first, then the imaginary parts.  For w <= 5 a wave keeps all of U in
// registers (complex128 at w = 5 excepted); wider U (64x64, 128x128) is read
// fragment by fragment from the L2-resident copy -- one contiguous wave load
// per fragment.  In
// FP32 a wave then takes two tiles (32 columns) so that each fragment feeds
// eight matrix-core products, halving the L2 traffic for U.
template <typename T, int W>
constexpr int fused_tiles_per_wave() {
  return (W >= 6 && sizeof(T) == 4) ? 2 : 1;
}

template <typename T, int W, bool PIPE>
__global__ void __launch_bounds__(256)
fused_pass_kernel(cplx<T>* __restrict__ st, const FusedDesc* __restrict__ fd, const T* __restrict__ umat,
                  uint32_t xcd) {
  using v4 = typename Mfma<T>::v4;
  constexpr int R = 1 << W;   // rows of U
  constexpr int RBK = R / 16; // 16-row blocks
  constexpr int KS = R / 4;   // K steps of 4
  constexpr int NF = RBK * KS;
  // U in registers for w <= 5, except complex128 at w = 5 (96 more VGPRs:
  // one wave per SIMD), which reads U from the L1/L2-resident copy instead
  constexpr bool kRegU = W <= 4 || (W == 5 && sizeof(T) == 4);
  constexpr bool kPipe = PIPE && W <= 5;  // software-pipelined (see below)
  constexpr int CG = fused_tiles_per_wave<T, W>();
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t i16 = lane & 15, g4 = lane >> 4;
  const int m = fd->m;
  const uint64_t tiles = fd->tiles;
  const T* Ur = umat + fd->u_off;
  const T* Ui = Ur + NF * 64;
  T ur[kRegU ? RBK : 1][kRegU ? KS : 1], ui[kRegU ? RBK : 1][kRegU ? KS : 1],
      nui[kRegU ? RBK : 1][kRegU ? KS : 1];
  if (kRegU) {
#pragma unroll
    for (int rb = 0; rb < (kRegU ? RBK : 1); ++rb)
#pragma unroll
      for (int ks = 0; ks < (kRegU ? KS : 1); ++ks) {
        const int f = rb * KS + ks;
        ur[rb][ks] = Ur[f * 64 + lane];
        ui[rb][ks] = Ui[f * 64 + lane];
        nui[rb][ks] = -ui[rb][ks];
      }
  }
  // The qubit lists (sq[8], pq[4], tq[12]: 24 contiguous bytes of the
  // descriptor) as six uniform dwords, read once: byte loads inside the tile
  // loop would be vector loads followed by a full wait on every memory
  // operation in flight, prefetched tiles and stores included.
  static_assert(offsetof(FusedDesc, sq) % 4 == 0 && offsetof(FusedDesc, pq) == offsetof(FusedDesc, sq) + 8 &&
                    offsetof(FusedDesc, tq) == offsetof(FusedDesc, sq) + 12 && sizeof(FusedDesc::tq) == 12,
                "the qubit lists must be 24 contiguous bytes on a dword boundary");
  uint32_t qw[6];
  {
    const uint32_t* q32 = reinterpret_cast<const uint32_t*>(fd->sq);
#pragma unroll
    for (int i = 0; i < 6; ++i) qw[i] = __builtin_amdgcn_readfirstlane(q32[i]);
  }
  // qubit of list byte b (sq: 0-7, pq: 8-11, tq: 12-23); b is a constant
  auto qb = [&](int b) -> int { return (int)(int8_t)(qw[b >> 2] >> (8 * (b & 3))); };
  // deposit the low `count` bits of v onto the qubits of bytes first..
  auto dep = [&](uint32_t v, int first, int count) -> uint64_t {
    uint64_t g = 0;
#pragma unroll
    for (int b = 0; b < count; ++b) g |= uint64_t((v >> b) & 1u) << qb(first + b);
    return g;
  };
  // base index of a tile: a zero bit inserted at every tile qubit (ascending)
  auto base_of = [&](uint64_t t) -> uint64_t {
#pragma unroll
    for (int i = 0; i < 12; ++i)
      if (i < m) {
        const int q = qb(12 + i);
        t = ((t >> q) << (q + 1)) | (t & ((uint64_t(1) << q) - 1));
      }
    return t;
  };
  // lane parts of the addresses: B rows k = 4*ks + g4 (slots 0-1 from the
  // lane); D rows i = 16*rb + 4*g4 + v (FP32: slots 2-3 from the lane) or
  // 16*rb + 4*v + g4 (FP64: slots 0-1 from the lane); columns j = i16 on
  // the column qubits
  constexpr bool f64 = sizeof(T) == 8;
  const uint64_t col = dep(i16, 8, 4);
  const uint64_t lane_ld = col + dep(g4, 0, 2);
  const uint64_t lane_st = f64 ? lane_ld : col + dep(g4 << 2, 0, W);
  uint64_t row_ld[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) row_ld[ks] = dep(4 * ks, 0, W);
  // a workgroup's 4 waves take 4 * CG consecutive tiles; with xcd set (grid
  // and group count multiples of 8) XCD x = blockIdx % 8 sweeps a contiguous
  // run
  const uint64_t groups = (tiles + 4 * CG - 1) / (4 * CG);
  uint64_t g = blockIdx.x, step = gridDim.x, end = groups;
  if (xcd) {
    const uint64_t per = groups >> 3;
    const uint32_t x = blockIdx.x & 7u;
    g = x * per + (blockIdx.x >> 3);
    step = gridDim.x >> 3;
    end = (x + 1) * per;
  }
  // wave-uniform: tile indices, bases and the valid flags stay in scalar
  // registers (address arithmetic on the SALU, stores under a scalar branch)
  const uint64_t wave_tile = (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * CG;
  // X of this wave's tiles in group gg (zero columns past the last tile)
  // (branch-free: a wave past the last tile reads tile 0 and discards its
  // products, so no load sits in a conditional block or feeds a select --
  // either would make the wave wait for the load right away)
  // tiles is a power of two (2^(n-m)): a tile index is in range when no bit
  // at or above log2(tiles) is set -- a 64-bit test the scalar unit has (it
  // has no 64-bit ordered compare)
  const uint64_t past = ~(tiles - 1);
  auto load = [&](uint64_t gg, T (&xr)[CG][KS], T (&xi)[CG][KS], uint64_t (&base)[CG], bool (&valid)[CG]) {
    const uint64_t tile0 = gg * 4 * CG + wave_tile;
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      valid[c] = ((tile0 + c) & past) == 0;
      base[c] = base_of(valid[c] ? tile0 + c : 0);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const cplx<T> v = st[base[c] + row_ld[ks] + lane_ld];
        xr[c][ks] = v.x;
        xi[c][ks] = v.y;
      }
    }
  };
  // Y = U X on the matrix cores, stored in place
  auto product = [&](const T (&xr)[CG][KS], const T (&xi)[CG][KS], const uint64_t (&base)[CG],
                     const bool (&valid)[CG]) {
    constexpr int kRbUnroll = kRegU ? RBK : 1;
#pragma unroll kRbUnroll
    for (int rb = 0; rb < RBK; ++rb) {
      v4 yr[CG], yi[CG];
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        yr[c] = v4{0, 0, 0, 0};
        yi[c] = v4{0, 0, 0, 0};
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        T ar, ai, nai;
        if (kRegU) {
          ar = ur[kRegU ? rb : 0][kRegU ? ks : 0];
          ai = ui[kRegU ? rb : 0][kRegU ? ks : 0];
          nai = nui[kRegU ? rb : 0][kRegU ? ks : 0];
        } else {
          const int f = rb * KS + ks;
          ar = Ur[f * 64 + lane];
          ai = Ui[f * 64 + lane];
          nai = -ai;
        }
#pragma unroll
        for (int c = 0; c < CG; ++c) {
          yr[c] = Mfma<T>::mma(ar, xr[c][ks], yr[c]);
          yr[c] = Mfma<T>::mma(nai, xi[c][ks], yr[c]);
          yi[c] = Mfma<T>::mma(ar, xi[c][ks], yi[c]);
          yi[c] = Mfma<T>::mma(ai, xr[c][ks], yi[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        if (!valid[c]) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cplx<T> o;
          o.x = yr[c][v];
          o.y = yi[c][v];
          st[base[c] + dep(16 * rb + (f64 ? 4 * v : v), 0, W) + lane_st] = o;
        }
      }
    }
  };
  T xr[CG][KS], xi[CG][KS];
  uint64_t base[CG];
  bool valid[CG];
  if (kPipe) {
    // w <= 5: a persistent grid, software-pipelined per wave -- the next
    // group's loads are issued before this group's products, so each wave
    // overlaps its own HBM traffic with its matrix-core work (loads, products
    // and stores of one tile would otherwise run as three serial phases).
    // Two register sets alternate (no copies between iterations, which
    // would wait for the loads), and the loads are unconditional: past the
    // end a wave re-reads its current group, whose products it discards.
    T yr2[CG][KS], yi2[CG][KS];
    uint64_t base2[CG];
    bool valid2[CG];
    if (g < end) load(g, xr, xi, base, valid);
    while (g < end) {
      const uint64_t g1 = g + step;
      load(g1 < end ? g1 : g, yr2, yi2, base2, valid2);
      product(xr, xi, base, valid);
      if (g1 >= end) break;
      const uint64_t g2 = g1 + step;
      load(g2 < end ? g2 : g1, xr, xi, base, valid);
      product(yr2, yi2, base2, valid2);
      g = g2;
    }
  } else {
    for (; g < end; g += step) {
      load(g, xr, xi, base, valid);
      product(xr, xi, base, valid);
    }
  }
}

// ---------------------------------------------------------------------------
// gate-per-pass baseline: one sweep of the whole state per gate
// ---------------------------------------------------------------------------
template <typename T>
struct M2 {
  T c[8];
};

// Work items [first, end) with stride `step` of a thread in a streaming
// kernel.  With xcd set (grid a multiple of 8, count a multiple of 8), XCD
// x = blockIdx % 8 sweeps the contiguous eighth [x count/8, (x+1) count/8).
struct Walk {
  uint64_t first, step, end;
};
__device__ __forceinline__ Walk stream_walk(uint64_t count, uint32_t xcd) {
  if (!xcd)
    return {(uint64_t)blockIdx.x * blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x, count};
  const uint64_t per = count >> 3;
  const uint32_t x = blockIdx.x & 7u;
  return {x * per + (uint64_t)(blockIdx.x >> 3) * blockDim.x + threadIdx.x,
          (uint64_t)(gridDim.x >> 3) * blockDim.x, (x + 1) * per};
}

template <typename T>
__global__ void __launch_bounds__(256)
gate_pass_1q(cplx<T>* __restrict__ st, int q, uint64_t npairs, M2<T> u, uint32_t xcd) {
  const Walk w = stream_walk(npairs, xcd);
  const uint64_t lowmask = (uint64_t(1) << q) - 1;
  for (uint64_t p = w.first; p < w.end; p += w.step) {
    const uint64_t i0 = ((p >> q) << (q + 1)) | (p & lowmask);
    const uint64_t i1 = i0 | (uint64_t(1) << q);
    const cplx<T> x = st[i0], y = st[i1];
    cplx<T> r0, r1;
    r0.x = u.c[0] * x.x - u.c[1] * x.y + u.c[2] * y.x - u.c[3] * y.y;
    r0.y = u.c[0] * x.y + u.c[1] * x.x + u.c[2] * y.y + u.c[3] * y.x;
    r1.x = u.c[4] * x.x - u.c[5] * x.y + u.c[6] * y.x - u.c[7] * y.y;
    r1.y = u.c[4] * x.y + u.c[5] * x.x + u.c[6] * y.y + u.c[7] * y.x;
    st[i0] = r0;
    st[i1] = r1;
  }
}

// kind: 0 CX(q0 control, q1 target), 1 CZ, 2 CP(c0, c1), 3 SWAP
template <typename T>
__global__ void __launch_bounds__(256)
gate_pass_2q(cplx<T>* __restrict__ st, int q0, int q1, int kind, uint64_t nquads, T cr, T ci,
             uint32_t xcd) {
  const int lo = min(q0, q1), hi = max(q0, q1);
  const Walk w = stream_walk(nquads, xcd);
  const uint64_t m0 = uint64_t(1) << q0, m1 = uint64_t(1) << q1;
  for (uint64_t p = w.first; p < w.end; p += w.step) {
    uint64_t i = ((p >> lo) << (lo + 1)) | (p & ((uint64_t(1) << lo) - 1));
    i = ((i >> hi) << (hi + 1)) | (i & ((uint64_t(1) << hi) - 1));
    // a[b] with bit 0 of b = qubit q0, bit 1 = qubit q1
    cplx<T> a0 = st[i], a1 = st[i | m0], a2 = st[i | m1], a3 = st[i | m0 | m1];
    if (kind == 0) {
      const cplx<T> t = a1; a1 = a3; a3 = t;
    } else if (kind == 1) {
      a3.x = -a3.x; a3.y = -a3.y;
    } else if (kind == 2) {
      cmul(a3, cr, ci);
    } else {
      const cplx<T> t = a1; a1 = a2; a2 = t;
    }
    st[i] = a0; st[i | m0] = a1; st[i | m1] = a2; st[i | m0 | m1] = a3;
  }
}

// ---------------------------------------------------------------------------
// init, readout, probe
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) set_basis_kernel(cplx<T>* __restrict__ st, uint64_t N, uint64_t x) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    cplx<T> v;
    v.x = (i == x) ? T(1) : T(0);
    v.y = T(0);
    st[i] = v;
  }
}

constexpr int kNormBlocks = 1024;
constexpr int kNormThreads = 256;

// Fixed-shape two-level FP64 reduction: thread t of block b sums |a_i|^2 for
// i = b*256 + t + k*(1024*256), k = 0, 1, ...; each block reduces its 256
// partial sums by a fixed binary tree; one block then reduces the 1024
// block sums by the same tree.  The order never depends on the device.
template <typename T>
__global__ void __launch_bounds__(kNormThreads)
norm_partial(const cplx<T>* __restrict__ st, uint64_t N, double* __restrict__ part) {
  __shared__ double sh[kNormThreads];
  double acc = 0.0;
  const uint64_t stride = (uint64_t)kNormBlocks * kNormThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kNormThreads + threadIdx.x; i < N; i += stride) {
    const cplx<T> v = st[i];
    acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kNormThreads) norm_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kNormThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kNormBlocks; i += kNormThreads) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kNormThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// probs = 0: widen amplitudes to complex128; probs = 1: |a|^2 in FP64.
template <typename T>
__global__ void __launch_bounds__(256)
readout_kernel(const cplx<T>* __restrict__ st, uint64_t first, uint64_t count, int probs,
               double* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const cplx<T> v = st[first + i];
    const double re = (double)v.x, im = (double)v.y;
    if (probs) {
      out[i] = re * re + im * im;
    } else {
      out[2 * i] = re;
      out[2 * i + 1] = im;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
gather_kernel(const cplx<T>* __restrict__ st, const uint64_t* __restrict__ idx, uint64_t count,
              double* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const cplx<T> v = st[idx[i]];
    out[2 * i] = (double)v.x;
    out[2 * i + 1] = (double)v.y;
  }
}

__global__ void __launch_bounds__(256)
copy_probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return fail(HS_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct DevInfo {
  int cus = 0;
};

static std::mutex g_dev_mu;
static std::map<int, DevInfo> g_dev;

static hs_status device_info(int dev, DevInfo* out) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev.find(dev);
  if (it != g_dev.end()) {
    *out = it->second;
    return HS_OK;
  }
  DevInfo d;
  HIP_TRY(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
  g_dev[dev] = d;
  *out = d;
  return HS_OK;
}

static inline hipStream_t stream_of(State* s) { return (hipStream_t)s->stream; }

// streaming grid: enough blocks of 256 to fill the device a few times over
static hs_status stream_grid(int dev, uint64_t work, unsigned* grid) {
  DevInfo d;
  hs_status rc = device_info(dev, &d);
  if (rc) return rc;
  const uint64_t want = (work + 255) / 256;
  *grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)d.cus * 16));
  return HS_OK;
}

hs_status dev_set_basis(State* s, uint64_t x) {
  HIP_TRY(hipSetDevice(s->device));
  const uint64_t N = uint64_t(1) << s->n;
  unsigned grid;
  if (hs_status rc = stream_grid(s->device, N, &grid)) return rc;
  if (s->dtype == HS_C64)
    hipLaunchKernelGGL(set_basis_kernel<float>, dim3(grid), dim3(256), 0, stream_of(s),
                       (cplx<float>*)s->ptr, N, x);
  else
    hipLaunchKernelGGL(set_basis_kernel<double>, dim3(grid), dim3(256), 0, stream_of(s),
                       (cplx<double>*)s->ptr, N, x);
  HIP_TRY(hipGetLastError());
  return HS_OK;
}

// Grid of a gate sweep over `work` items: one item per thread up to 2^31
// threads, XCD-contiguous runs when the grid and the item count allow.
static void sweep_grid(uint64_t work, unsigned* grid, uint32_t* xcd) {
  uint64_t g = std::max<uint64_t>(1, std::min<uint64_t>((work + 255) / 256, (uint64_t(1) << 31) / 256));
  *xcd = 0;
  if (work % 8 == 0 && g >= 8) {
    g &= ~uint64_t(7);
    *xcd = 1;
  }
  *grid = (unsigned)g;
}

template <typename T>
static hs_status gate_pass_t(State* s, const Gate& g) {
  const uint64_t N = uint64_t(1) << s->n;
  unsigned grid;
  uint32_t xcd;
  if (g.arity() == 1) {
    sweep_grid(N / 2, &grid, &xcd);
    cd u[4];
    gate_matrix(g, u);
    M2<T> m;
    for (int i = 0; i < 4; ++i) {
      m.c[2 * i] = (T)u[i].real();
      m.c[2 * i + 1] = (T)u[i].imag();
    }
    hipLaunchKernelGGL(gate_pass_1q<T>, dim3(grid), dim3(256), 0, stream_of(s),
                       (cplx<T>*)s->ptr, g.q0, N / 2, m, xcd);
  } else {
    if (s->n < 2) return fail(HS_E_ARG, "two-qubit gate on a 1-qubit state");
    sweep_grid(N / 4, &grid, &xcd);
    int kind = 0;
    T cr = 0, ci = 0;
    switch (g.kind) {
      case HS_CX: kind = 0; break;
      case HS_CZ: kind = 1; break;
      case HS_CP: kind = 2; cr = (T)cos(g.p[0]); ci = (T)sin(g.p[0]); break;
      case HS_SWAP: kind = 3; break;
      default: return fail(HS_E_ARG, "unknown two-qubit kind %d", g.kind);
    }
    hipLaunchKernelGGL(gate_pass_2q<T>, dim3(grid), dim3(256), 0, stream_of(s),
                       (cplx<T>*)s->ptr, g.q0, g.q1, kind, N / 4, cr, ci, xcd);
  }
  HIP_TRY(hipGetLastError());
  return HS_OK;
}

hs_status dev_gate_pass(State* s, const Gate& g) {
  HIP_TRY(hipSetDevice(s->device));
  return s->dtype == HS_C64 ? gate_pass_t<float>(s, g) : gate_pass_t<double>(s, g);
}

// ---- uploaded plan ----------------------------------------------------------
struct DevicePlan {
  int device = 0;
  // descriptors from the stream-ordered allocator (serving): freed with
  // hipFreeAsync on free_stream, so a teardown never waits for the device
  bool async_alloc = false;
  void* free_stream = nullptr;
  // recorded after the asynchronous descriptor copies on free_stream; a
  // launch on another stream waits for it on the device
  hipEvent_t upload_done = nullptr;
  IPart* parts = nullptr;
  IStage* stages = nullptr;
  void* ops = nullptr;
  std::vector<PartDesc> h_parts;     // host copy (absolute offsets)
  std::vector<int> rb;               // register bits of the kernel per part
  std::vector<unsigned> grid;        // grid per part
  std::vector<uint8_t> xcd;          // XCD-contiguous tile runs
  // fused path (uploaded on first use)
  bool fused_ready = false;
  FusedDesc* fparts = nullptr;
  void* fmat = nullptr;
  std::vector<FusedDesc> h_fparts;
  std::vector<unsigned> fgrid;
  std::vector<uint8_t> fxcd;
  std::vector<uint8_t> fpipe;  // software-pipelined kernel (persistent grid)
};

// Best effort: called from destructors, where an error cannot be returned.
void device_plan_free(DevicePlan* d) {
  if (!d) return;
  (void)hipSetDevice(d->device);
  for (void* ptr : {(void*)d->parts, (void*)d->stages, d->ops}) {
    if (!ptr) continue;
    if (d->async_alloc) (void)hipFreeAsync(ptr, (hipStream_t)d->free_stream);
    else (void)hipFree(ptr);
  }
  if (d->fparts) (void)hipFree(d->fparts);
  if (d->fmat) (void)hipFree(d->fmat);
  if (d->upload_done) (void)hipEventDestroy(d->upload_done);
  delete d;
}

// Host copies of a plan's descriptors, kept until the asynchronous copies
// from them have run (a host function on the copy stream deletes them).
template <typename T>
struct HostDescriptors {
  std::vector<IPart> parts;
  std::vector<IStage> stages;
  std::vector<OpDesc<T>> ops;
  static void release(void* p) { delete static_cast<HostDescriptors*>(p); }
};

template <typename T, int RB>
static hs_status resident_per_cu(int block, size_t lds, int* per_cu) {
  if (lds > 65536)
    HIP_TRY(hipFuncSetAttribute((const void*)part_pass_kernel<T, RB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, part_pass_kernel<T, RB>, block, lds));
  if (*per_cu < 1) return fail(HS_E_UNSUPPORTED, "part kernel cannot be resident (block %d, lds %zu)",
                               block, lds);
  return HS_OK;
}

template <typename T>
static hs_status resident_rb(int rb, int block, size_t lds, int* per_cu) {
  switch (rb) {
    case 1: return resident_per_cu<T, 1>(block, lds, per_cu);
    case 2: return resident_per_cu<T, 2>(block, lds, per_cu);
    case 3: return resident_per_cu<T, 3>(block, lds, per_cu);
    case 4: return resident_per_cu<T, 4>(block, lds, per_cu);
    default: return fail(HS_E_UNSUPPORTED, "no kernel with %d register bits", rb);
  }
}

// Grid of one part-pass launch for launch shape `ls`: one workgroup per tile,
// or a persistent grid sized by occupancy; XCD-contiguous tile runs need the
// grid and the tile count to be multiples of 8.
static void part_grid(const LaunchShape& ls, uint64_t tiles, int block, int per_cu, int cus,
                      unsigned* grid, uint8_t* xcd) {
  uint64_t g = tiles;
  if (ls.per_cu > 0) g = std::min<uint64_t>(tiles, (uint64_t)ls.per_cu * per_cu * cus);
  g = std::max<uint64_t>(1, std::min<uint64_t>(g, (uint64_t(1) << 31) / (uint64_t)block));
  *xcd = 0;
  if (ls.xcd && tiles % 8 == 0 && g >= 8) {
    g &= ~uint64_t(7);
    *xcd = 1;
  }
  *grid = (unsigned)g;
}

// Interpreter tables of one layout (host side of IStage / IoOffsets).
template <typename T>
static IStage interp_stage(const StageDesc& e, const PartDesc& d) {
  IStage o{};
  const int sw = lds_sw<T>();
  auto slot = [&](int c) { return lds_slot(1u << e.pos[c], sw) * (uint32_t)sizeof(cplx<T>); };
  for (int c = 0; c < d.lb; ++c) o.lane[c] = slot(c);
  for (int c = 0; c < d.wb; ++c) o.wave[c] = slot(d.lb + c);
  for (int r = 0; r < d.rb; ++r) o.reg[r] = slot(d.lb + d.wb + r);
  o.op_begin = e.op_begin;
  o.op_end = e.op_end;
  o.transition = e.transition;
  return o;
}

static IoOffsets interp_io(const StageDesc& e, const PartDesc& d) {
  IoOffsets o{};
  auto off = [&](int c) { return uint64_t(1) << d.tq[e.pos[c]]; };
  for (int c = 0; c < d.lb; ++c) o.lane[c] = off(c);
  for (int c = 0; c < d.wb; ++c) o.wave[c] = off(d.lb + c);
  for (int r = 0; r < d.rb; ++r) o.reg[r] = off(d.lb + d.wb + r);
  return o;
}

// Upload a plan's interpreter descriptors.  stream = NULL: hipMalloc and
// blocking copies; otherwise the stream-ordered allocator and asynchronous
// copies on `stream`, waited for before returning.
template <typename T>
static hs_status upload_plan(Plan* p, int dtype, int dev, DevicePlan** out, hipStream_t stream,
                             const PinnedStaging* pin = nullptr) {
  std::vector<PartDesc> hparts;
  std::vector<IPart> parts;
  std::vector<IStage> stages;
  std::vector<OpDesc<T>> ops;
  auto dp = std::make_unique<DevicePlan>();
  dp->device = dev;
  DevInfo dinfo;
  if (hs_status rc = device_info(dev, &dinfo)) return rc;
  for (const CompiledPart& cp : p->comp[dtype]) {
    PartDesc d = cp.desc;
    if (d.rb > kMaxRegBits || d.wb > kMaxWaveBits || d.lb > kLaneBits || cp.stages.size() < 2)
      return fail(HS_E_UNSUPPORTED, "part layout outside the interpreter's limits");
    d.stage_off = (int)stages.size();
    d.lds_bytes = cp.lds_round_trips ? (int)((size_t(1) << d.m) * sizeof(cplx<T>)) : 0;
    const int op0 = (int)ops.size();
    for (const StageDesc& e : cp.stages) {
      IStage is = interp_stage<T>(e, d);
      is.op_begin += op0;
      is.op_end += op0;
      stages.push_back(is);
    }
    IPart ip{};
    ip.load = interp_io(cp.stages.front(), d);
    ip.store = interp_io(cp.stages.back(), d);
    ip.tiles = d.tiles;
    ip.m = d.m;
    ip.lb = d.lb;
    ip.n_stages = d.n_stages;
    for (int i = 0; i < kMaxTile; ++i) ip.tq[i] = d.tq[i];
    for (const HostOp& h : cp.ops) {
      OpDesc<T> o{};
      o.kind = h.kind;
      o.b0 = h.b0;
      o.b1 = h.b1;
      for (int i = 0; i < 32; ++i) o.c[i] = (T)h.c[i];
      ops.push_back(o);
    }
    hparts.push_back(d);
    parts.push_back(ip);
    dp->rb.push_back(cp.rb_kernel);
    const int block = 64 << d.wb;
    int per_cu = 0;
    if (hs_status rc = resident_rb<T>(cp.rb_kernel, block, (size_t)d.lds_bytes, &per_cu)) return rc;
    unsigned g = 1;
    uint8_t x = 0;
    part_grid(cp.launch, d.tiles, block, per_cu, dinfo.cus, &g, &x);
    dp->grid.push_back(g);
    dp->xcd.push_back(x);
  }
  if (ops.empty()) ops.push_back(OpDesc<T>{});
  if (parts.empty()) parts.push_back(IPart{});
  if (stages.empty()) stages.push_back(IStage{});
  if (stream) {
    // Nothing here waits for the device: the stream may share a hardware
    // queue with long-running part kernels, and a host wait would hold the
    // caller (a serving thread) until they drain.  The host copies live
    // until a host function after the copies deletes them, and launches
    // elsewhere wait for upload_done on the device.
    dp->async_alloc = true;
    dp->free_stream = stream;
    const size_t b_parts = parts.size() * sizeof(IPart), b_stages = stages.size() * sizeof(IStage),
                 b_ops = ops.size() * sizeof(OpDesc<T>);
    // pinned staging, when it is free and large enough: the copies are then
    // plain DMA with nothing to stage on the host
    const size_t o_stages = (b_parts + 255) & ~size_t(255), o_ops = (o_stages + b_stages + 255) & ~size_t(255);
    if (pin && pin->ptr && o_ops + b_ops <= pin->bytes && hipEventQuery((hipEvent_t)pin->busy) == hipSuccess) {
      char* h = static_cast<char*>(pin->ptr);
      std::memcpy(h, parts.data(), b_parts);
      std::memcpy(h + o_stages, stages.data(), b_stages);
      std::memcpy(h + o_ops, ops.data(), b_ops);
      HIP_TRY(hipMallocAsync((void**)&dp->parts, b_parts, stream));
      HIP_TRY(hipMallocAsync((void**)&dp->stages, b_stages, stream));
      HIP_TRY(hipMallocAsync(&dp->ops, b_ops, stream));
      HIP_TRY(hipMemcpyAsync(dp->parts, h, b_parts, hipMemcpyHostToDevice, stream));
      HIP_TRY(hipMemcpyAsync(dp->stages, h + o_stages, b_stages, hipMemcpyHostToDevice, stream));
      HIP_TRY(hipMemcpyAsync(dp->ops, h + o_ops, b_ops, hipMemcpyHostToDevice, stream));
      HIP_TRY(hipEventRecord((hipEvent_t)pin->busy, stream));  // the staging is free again once this passes
      HIP_TRY(hipEventCreateWithFlags(&dp->upload_done, hipEventDisableTiming));
      HIP_TRY(hipEventRecord(dp->upload_done, stream));
      dp->h_parts = hparts;
      *out = dp.release();
      return HS_OK;
    }
    auto host = std::make_unique<HostDescriptors<T>>();
    host->parts = std::move(parts);
    host->stages = std::move(stages);
    host->ops = std::move(ops);
    HIP_TRY(hipMallocAsync((void**)&dp->parts, host->parts.size() * sizeof(IPart), stream));
    HIP_TRY(hipMallocAsync((void**)&dp->stages, host->stages.size() * sizeof(IStage), stream));
    HIP_TRY(hipMallocAsync(&dp->ops, host->ops.size() * sizeof(OpDesc<T>), stream));
    HIP_TRY(hipMemcpyAsync(dp->parts, host->parts.data(), host->parts.size() * sizeof(IPart),
                           hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dp->stages, host->stages.data(), host->stages.size() * sizeof(IStage),
                           hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dp->ops, host->ops.data(), host->ops.size() * sizeof(OpDesc<T>),
                           hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventCreateWithFlags(&dp->upload_done, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(dp->upload_done, stream));
    if (hipLaunchHostFunc(stream, HostDescriptors<T>::release, host.get()) == hipSuccess) {
      host.release();  // deleted by the host function
    } else {
      (void)hipGetLastError();
      HIP_TRY(hipStreamSynchronize(stream));  // fallback: wait, then free here
    }
  } else {
    HIP_TRY(hipMalloc(&dp->parts, parts.size() * sizeof(IPart)));
    HIP_TRY(hipMalloc(&dp->stages, stages.size() * sizeof(IStage)));
    HIP_TRY(hipMalloc(&dp->ops, ops.size() * sizeof(OpDesc<T>)));
    HIP_TRY(hipMemcpy(dp->parts, parts.data(), parts.size() * sizeof(IPart), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dp->stages, stages.data(), stages.size() * sizeof(IStage), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dp->ops, ops.data(), ops.size() * sizeof(OpDesc<T>), hipMemcpyHostToDevice));
  }
  dp->h_parts = hparts;
  *out = dp.release();
  return HS_OK;
}

template <typename T>
static hs_status launch_part(State* s, DevicePlan* dp, int part) {
  const PartDesc& d = dp->h_parts[part];
  const int block = 64 << d.wb;
  const unsigned grid = dp->grid[part];
  const size_t lds = (size_t)d.lds_bytes;
  cplx<T>* st = (cplx<T>*)s->ptr;
  const IPart* pd = dp->parts + part;
  const IStage* sd = dp->stages + d.stage_off;
  const OpDesc<T>* ops = (const OpDesc<T>*)dp->ops;
  hipStream_t str = stream_of(s);
  const uint32_t xcd = dp->xcd[part];
#define HS_LAUNCH_PART(RB_)                                                                     \
  hipLaunchKernelGGL((part_pass_kernel<T, RB_>), dim3(grid), dim3(block), lds, str, st, pd, sd, ops, \
                     xcd);                                                                      \
  break;
  switch (dp->rb[part]) {
    case 1: HS_LAUNCH_PART(1)
    case 2: HS_LAUNCH_PART(2)
    case 3: HS_LAUNCH_PART(3)
    case 4: HS_LAUNCH_PART(4)
    default: return fail(HS_E_UNSUPPORTED, "no kernel with %d register bits", dp->rb[part]);
  }
#undef HS_LAUNCH_PART
  HIP_TRY(hipGetLastError());
  return HS_OK;
}

static hs_status device_plan(State* s, Plan* p, DevicePlan** out) {
  const int dt = (int)s->dtype;
  auto it = p->dev[dt].find(s->device);
  if (it != p->dev[dt].end()) {
    *out = it->second;
    return HS_OK;
  }
  DevicePlan* dp = nullptr;
  hs_status rc = dt == HS_C64 ? upload_plan<float>(p, dt, s->device, &dp, nullptr)
                              : upload_plan<double>(p, dt, s->device, &dp, nullptr);
  if (rc) return rc;
  p->dev[dt][s->device] = dp;
  *out = dp;
  return HS_OK;
}

hs_status dev_plan_upload_async(Plan* p, hs_dtype dtype, int device, void* stream, const PinnedStaging* pin) {
  HIP_TRY(hipSetDevice(device));
  std::lock_guard<std::mutex> lk(p->mu);
  const int dt = (int)dtype;
  if (p->dev[dt].count(device)) return HS_OK;
  DevicePlan* dp = nullptr;
  hs_status rc = dt == HS_C64 ? upload_plan<float>(p, dt, device, &dp, (hipStream_t)stream, pin)
                              : upload_plan<double>(p, dt, device, &dp, (hipStream_t)stream, pin);
  if (rc) {
    device_plan_free(dp);
    return rc;
  }
  p->dev[dt][device] = dp;
  return HS_OK;
}

hs_status dev_plan_stream_wait(Plan* p, hs_dtype dtype, int device, void* stream) {
  HIP_TRY(hipSetDevice(device));
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->dev[(int)dtype].find(device);
    if (it == p->dev[(int)dtype].end()) return fail(HS_E_STATE, "plan not uploaded for this device");
    ev = it->second->upload_done;
  }
  if (ev) HIP_TRY(hipStreamWaitEvent((hipStream_t)stream, ev, 0));
  return HS_OK;
}

hs_status dev_run_part(State* s, Plan* p, int part) {
  HIP_TRY(hipSetDevice(s->device));
  DevicePlan* dp = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (hs_status rc = device_plan(s, p, &dp)) return rc;
  }
  return s->dtype == HS_C64 ? launch_part<float>(s, dp, part) : launch_part<double>(s, dp, part);
}

template <typename T>
static hs_status upload_fused(Plan* p, DevicePlan* dp) {
  std::vector<FusedDesc> fds;
  std::vector<T> mats;
  for (const FusedPart& f : p->fused) {
    FusedDesc d{};
    d.w = f.w;
    d.m = f.m;
    d.tiles = f.tiles;
    d.u_off = (int32_t)mats.size();
    std::memcpy(d.sq, f.sq, sizeof d.sq);
    std::memcpy(d.pq, f.pq, sizeof d.pq);
    std::memcpy(d.tq, f.tq, sizeof d.tq);
    // fragment order (see fused_pass_kernel): real parts, then imaginary
    const int R = 1 << f.w;
    for (int part_im = 0; part_im < 2 && f.w > 0; ++part_im)
      for (int rb = 0; rb < R / 16; ++rb)
        for (int ks = 0; ks < R / 4; ++ks)
          for (int l = 0; l < 64; ++l) {
            const cd z = f.u[(size_t)(16 * rb + l % 16) * R + 4 * ks + l / 16];
            mats.push_back((T)(part_im ? z.imag() : z.real()));
          }
    fds.push_back(d);
    // one workgroup of four wavefronts per 4 * (tiles per wave) tiles,
    // XCD-contiguous runs
    uint64_t per_wg = 4;
    switch (f.w) {
      case 6: per_wg *= fused_tiles_per_wave<T, 6>(); break;
      case 7: per_wg *= fused_tiles_per_wave<T, 7>(); break;
      default: break;
    }
    const uint64_t groups = (f.tiles + per_wg - 1) / per_wg;
    uint64_t g = std::max<uint64_t>(1, std::min<uint64_t>(groups, (uint64_t(1) << 31) / 256));
    // w = 4, 5: launch shape from hs_tune("fused_shape"): 0 = one tile group
    // per workgroup; 1 = software-pipelined kernel, 2 = plain kernel, each
    // on a persistent grid of as many workgroups as the device keeps
    // resident (U is then read once per workgroup, not once per group).
    // By default (-1) the measured best per width and precision: on 30-qubit
    // states the persistent plain kernel for complex64 w = 5 (1.31 sweeps
    // against 1.40), one group per workgroup otherwise (complex64 w = 4:
    // 1.13-1.23 against 1.28-1.32; complex128 w = 4 / 5: 0.93-1.09 / 1.19-1.21
    // against 1.02-1.19 / 1.22-1.27).
    int shape = (f.w == 4 || f.w == 5) ? fused_launch_shape() : 0;
    if (shape < 0) shape = (sizeof(T) == 4 && f.w == 5) ? 2 : 0;
    if (shape) {
      int per_cu = 0;
      const void* fn = nullptr;
      if (f.w == 4)
        fn = shape == 1 ? (const void*)fused_pass_kernel<T, 4, true> : (const void*)fused_pass_kernel<T, 4, false>;
      else
        fn = shape == 1 ? (const void*)fused_pass_kernel<T, 5, true> : (const void*)fused_pass_kernel<T, 5, false>;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
      DevInfo di;
      if (hs_status rc = device_info(dp->device, &di)) return rc;
      g = std::max<uint64_t>(1, std::min<uint64_t>(g, (uint64_t)std::max(1, per_cu) * di.cus));
    }
    dp->fpipe.push_back(shape == 1 ? 1 : 0);
    uint8_t x = 0;
    if (groups % 8 == 0 && g >= 8) {
      g &= ~uint64_t(7);
      x = 1;
    }
    dp->fgrid.push_back((unsigned)g);
    dp->fxcd.push_back(x);
  }
  if (mats.empty()) mats.push_back(T(0));
  if (fds.empty()) fds.push_back(FusedDesc{});
  HIP_TRY(hipMalloc(&dp->fparts, fds.size() * sizeof(FusedDesc)));
  HIP_TRY(hipMalloc(&dp->fmat, mats.size() * sizeof(T)));
  HIP_TRY(hipMemcpy(dp->fparts, fds.data(), fds.size() * sizeof(FusedDesc), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dp->fmat, mats.data(), mats.size() * sizeof(T), hipMemcpyHostToDevice));
  dp->h_fparts = fds;
  dp->fused_ready = true;
  return HS_OK;
}

template <typename T>
static hs_status launch_fused(State* s, DevicePlan* dp, int part) {
  const FusedDesc& d = dp->h_fparts[part];
  cplx<T>* st = (cplx<T>*)s->ptr;
  const FusedDesc* fd = dp->fparts + part;
  const T* um = (const T*)dp->fmat;
  hipStream_t str = stream_of(s);
  const dim3 grid(dp->fgrid[part]);
  const uint32_t xcd = dp->fxcd[part];
  const bool pipe = dp->fpipe[part] != 0;
  switch (d.w) {
    case 4:
      if (pipe) hipLaunchKernelGGL((fused_pass_kernel<T, 4, true>), grid, dim3(256), 0, str, st, fd, um, xcd);
      else hipLaunchKernelGGL((fused_pass_kernel<T, 4, false>), grid, dim3(256), 0, str, st, fd, um, xcd);
      break;
    case 5:
      if (pipe) hipLaunchKernelGGL((fused_pass_kernel<T, 5, true>), grid, dim3(256), 0, str, st, fd, um, xcd);
      else hipLaunchKernelGGL((fused_pass_kernel<T, 5, false>), grid, dim3(256), 0, str, st, fd, um, xcd);
      break;
    case 6: hipLaunchKernelGGL((fused_pass_kernel<T, 6, false>), grid, dim3(256), 0, str, st, fd, um, xcd); break;
    case 7: hipLaunchKernelGGL((fused_pass_kernel<T, 7, false>), grid, dim3(256), 0, str, st, fd, um, xcd); break;
    default: return fail(HS_E_UNSUPPORTED, "part %d has no fused form", part);
  }
  HIP_TRY(hipGetLastError());
  return HS_OK;
}

hs_status dev_run_fused(State* s, Plan* p, int part) {
  HIP_TRY(hipSetDevice(s->device));
  DevicePlan* dp = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (hs_status rc = device_plan(s, p, &dp)) return rc;
    if (!dp->fused_ready) {
      hs_status rc = s->dtype == HS_C64 ? upload_fused<float>(p, dp) : upload_fused<double>(p, dp);
      if (rc) return rc;
    }
  }
  return s->dtype == HS_C64 ? launch_fused<float>(s, dp, part) : launch_fused<double>(s, dp, part);
}

// ---- readout ----------------------------------------------------------------
static hs_status ensure_scratch(State* s, size_t bytes) {
  if (s->scratch_bytes >= bytes) return HS_OK;
  if (s->scratch) HIP_TRY(hipFree(s->scratch));
  s->scratch = nullptr;
  s->scratch_bytes = 0;
  HIP_TRY(hipMalloc(&s->scratch, bytes));
  s->scratch_bytes = bytes;
  return HS_OK;
}

hs_status dev_norm(State* s, double* out) {
  HIP_TRY(hipSetDevice(s->device));
  if (hs_status rc = ensure_scratch(s, (kNormBlocks + 8) * sizeof(double))) return rc;
  double* part = (double*)s->scratch;
  double* res = part + kNormBlocks;
  const uint64_t N = uint64_t(1) << s->n;
  if (s->dtype == HS_C64)
    hipLaunchKernelGGL(norm_partial<float>, dim3(kNormBlocks), dim3(kNormThreads), 0, stream_of(s),
                       (const cplx<float>*)s->ptr, N, part);
  else
    hipLaunchKernelGGL(norm_partial<double>, dim3(kNormBlocks), dim3(kNormThreads), 0, stream_of(s),
                       (const cplx<double>*)s->ptr, N, part);
  hipLaunchKernelGGL(norm_final, dim3(1), dim3(kNormThreads), 0, stream_of(s), part, res);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, stream_of(s)));
  HIP_TRY(hipStreamSynchronize(stream_of(s)));
  return HS_OK;
}

// ---- the norm without allocation -------------------------------------------
// The norm's partial sums live in a file-scope device array instead of the
// state's lazily allocated scratch, so this path never calls the allocator.
// Each device holds its own copy; host code uses only the address that
// hipGetSymbolAddress reports for the current device (the array's name is a
// host-side stand-in, not a device address).  Every call on a device shares
// that device's copy: calls that overlap on one device race.  Nothing in it
// must start at zero: norm_partial writes every one of its kNormBlocks
// partial sums (zero for a block with no amplitudes) before norm_final
// reads them, and norm_final writes the result slot.
constexpr int kNoAllocDoubles = kNormBlocks + 8;  // 8,256 bytes per device
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`, looked up once per device with
// that device current.
static hs_status noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return fail(HS_E_ARG, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    HIP_TRY(hipSetDevice(device));
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[device] = (double*)ptr;
  }
  *out = g_noalloc_ptr[device];
  return HS_OK;
}

hs_status dev_norm_noalloc(State* s, double* out) {
  HIP_TRY(hipSetDevice(s->device));
  static_assert(kNormBlocks + 1 <= kNoAllocDoubles, "partials and result must fit the array");
  double* part = nullptr;
  if (hs_status rc = noalloc_scratch(s->device, &part)) return rc;
  double* res = part + kNormBlocks;
  const uint64_t N = uint64_t(1) << s->n;
  if (s->dtype == HS_C64)
    hipLaunchKernelGGL(norm_partial<float>, dim3(kNormBlocks), dim3(kNormThreads), 0, stream_of(s),
                       (const cplx<float>*)s->ptr, N, part);
  else
    hipLaunchKernelGGL(norm_partial<double>, dim3(kNormBlocks), dim3(kNormThreads), 0, stream_of(s),
                       (const cplx<double>*)s->ptr, N, part);
  hipLaunchKernelGGL(norm_final, dim3(1), dim3(kNormThreads), 0, stream_of(s), part, res);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, stream_of(s)));
  HIP_TRY(hipStreamSynchronize(stream_of(s)));
  return HS_OK;
}

hs_status dev_read(State* s, uint64_t first, uint64_t count, double* out, bool probs) {
  HIP_TRY(hipSetDevice(s->device));
  const uint64_t chunk = uint64_t(1) << 22;
  if (hs_status rc = ensure_scratch(s, std::max<size_t>(chunk * 16, (kNormBlocks + 8) * 8))) return rc;
  const int per = probs ? 1 : 2;
  for (uint64_t done = 0; done < count;) {
    const uint64_t c = std::min(chunk, count - done);
    unsigned grid;
    if (hs_status rc = stream_grid(s->device, c, &grid)) return rc;
    if (s->dtype == HS_C64)
      hipLaunchKernelGGL(readout_kernel<float>, dim3(grid), dim3(256), 0, stream_of(s),
                         (const cplx<float>*)s->ptr, first + done, c, probs ? 1 : 0, (double*)s->scratch);
    else
      hipLaunchKernelGGL(readout_kernel<double>, dim3(grid), dim3(256), 0, stream_of(s),
                         (const cplx<double>*)s->ptr, first + done, c, probs ? 1 : 0, (double*)s->scratch);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out + done * per, s->scratch, c * per * sizeof(double),
                           hipMemcpyDeviceToHost, stream_of(s)));
    HIP_TRY(hipStreamSynchronize(stream_of(s)));
    done += c;
  }
  return HS_OK;
}

// Amplitudes at host-given indices (validated < 2^n by the caller), widened
// to complex128, in chunks through the state's scratch buffer.
hs_status dev_read_at(State* s, const uint64_t* idx, uint64_t count, double* out) {
  HIP_TRY(hipSetDevice(s->device));
  const uint64_t chunk = uint64_t(1) << 21;  // 16 MiB of indices + 32 MiB of output
  if (hs_status rc = ensure_scratch(s, chunk * 24)) return rc;
  uint64_t* didx = (uint64_t*)s->scratch;
  double* dout = (double*)((char*)s->scratch + chunk * 8);
  for (uint64_t done = 0; done < count;) {
    const uint64_t c = std::min(chunk, count - done);
    unsigned grid;
    if (hs_status rc = stream_grid(s->device, c, &grid)) return rc;
    HIP_TRY(hipMemcpyAsync(didx, idx + done, c * sizeof(uint64_t), hipMemcpyHostToDevice, stream_of(s)));
    if (s->dtype == HS_C64)
      hipLaunchKernelGGL(gather_kernel<float>, dim3(grid), dim3(256), 0, stream_of(s),
                         (const cplx<float>*)s->ptr, didx, c, dout);
    else
      hipLaunchKernelGGL(gather_kernel<double>, dim3(grid), dim3(256), 0, stream_of(s),
                         (const cplx<double>*)s->ptr, didx, c, dout);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out + 2 * done, dout, c * 2 * sizeof(double), hipMemcpyDeviceToHost,
                           stream_of(s)));
    HIP_TRY(hipStreamSynchronize(stream_of(s)));
    done += c;
  }
  return HS_OK;
}

hs_status dev_copy_probe(const void* src, void* dst, size_t bytes, void* stream) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  unsigned grid;
  const uint64_t n16 = bytes / 16;
  if (hs_status rc = stream_grid(dev, n16, &grid)) return rc;
  hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                     (const uint4*)src, (uint4*)dst, n16);
  HIP_TRY(hipGetLastError());
  return HS_OK;
}

hs_status dev_sync(State* s) {
  HIP_TRY(hipSetDevice(s->device));
  HIP_TRY(hipStreamSynchronize(stream_of(s)));
  return HS_OK;
}

}  // namespace hisv
