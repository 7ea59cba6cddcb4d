// layout.h -- device-visible descriptors of a compiled part and the index
// maps shared by the host part compiler and the part-pass kernel.
//
// Alg. 1 (Sec. III.C) gathers, for every setting of the qubits outside a
// part, the 2^w amplitudes addressed by the part's qubits.  On the GPU one
// gathered sub-state is a *tile*: the part's qubits plus the lowest other
// qubits as padding (the padding rule of the multi-level scheme in Sec. IV,
// used here so that every tile row is a contiguous run of memory), m qubits
// in all, 2^m amplitudes.  A workgroup holds a tile in registers, 2^RB
// amplitudes per lane; the tile's m bits are split between lane bits,
// wave bits and register bits by a *layout*.  A gate can only run on bits
// that are register bits, so the part's gates are cut into *stages*
// (a second-level partition with limit RB, Sec. IV multi-level
// partitioning); between stages the tile is re-laid out through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hisv {

constexpr int kMaxTile = 16;   // widest tile (qubits)
constexpr int kMaxFusedQubits = 7;  // widest dense unitary of the fused path (128 x 128)
constexpr int kLaneBits = 6;   // 64-wide wavefronts

// A layout: pos[c] is the tile bit carried by coordinate bit c, where the
// coordinates of an amplitude are (lane, wave, register index j) packed as
// c in [0, lb) lane bits, [lb, lb+wb) wave bits, [lb+wb, m) register bits.
struct alignas(16) StageDesc {
  int8_t pos[kMaxTile];
  int32_t op_begin;    // ops [op_begin, op_end) run in this layout
  int32_t op_end;
  int32_t transition;  // 1: re-lay the tile out through LDS before the ops
  int32_t pad;
};

struct alignas(16) PartDesc {
  int32_t m, lb, wb, rb;   // tile bits; lane, wave and register bits (m = lb+wb+rb)
  int32_t n_stages;        // entries in the stage table: load, stages..., store
  int32_t stage_off;       // index of the load entry in the stage table
  int32_t lds_bytes;       // 0 when no entry needs a transition
  int32_t pad0;
  uint64_t tiles;          // 2^(n-m)
  int8_t tq[kMaxTile];     // tile bit -> global qubit, ascending
};

// Register-level operations produced by the part compiler.  Coefficients
// are in the state's precision; matrices are row-major complex (re, im).
enum OpKind : int32_t {
  OP_U = 0,     // dense 2x2 on b0: c = u00 u01 u10 u11 (8 reals)
  OP_R = 1,     // real 2x2 on b0: c[0..3] = u00 u01 u10 u11
  OP_D = 2,     // diagonal on b0: c = d0, d1 (4 reals)
  OP_D1 = 3,    // diag(1, d1) on b0: c[0..1] = d1
  OP_X = 4,     // swap the pair on b0
  OP_CX = 5,    // control b0, target b1
  OP_CZ = 6,    // negate where b0 = b1 = 1
  OP_CP = 7,    // multiply by c[0..1] where b0 = b1 = 1
  OP_SWAP = 8,  // exchange bits b0 and b1
  OP_U2 = 9,    // dense 4x4 on b0 < b1, row/column index = bit b0 + 2 bit b1:
                // c = 16 complex entries, row-major (32 reals)
  OP_NUM = 10
};

template <typename T>
struct alignas(16) OpDesc {
  int32_t kind, b0, b1, pad;
  T c[32];
};

// Descriptors of the interpreter kernel (part_pass_kernel), built from the
// compiled part at upload, per dtype.  Every per-bit quantity is a 32- or
// 64-bit word, so the kernel reads them with scalar loads and a lane builds
// its own offsets from them with a few ALU operations per bit.  Entries for
// bits a layout does not have are zero.
constexpr int kMaxWaveBits = 4;  // 1024-thread workgroups
constexpr int kMaxRegBits = 4;   // widest interpreter register stage

// Global offsets (in amplitudes) of the coordinate bits of a load or store
// layout: an amplitude's index is the tile base plus the offsets of its
// lane, wave and register bits.
struct alignas(16) IoOffsets {
  uint64_t lane[kLaneBits];
  uint64_t wave[kMaxWaveBits];
  uint64_t reg[kMaxRegBits];
};

// One entry of the stage table: swizzled LDS byte offsets of the layout's
// coordinate bits (XOR-combined: lds_slot is linear over XOR) and the ops
// that run in it.
struct alignas(16) IStage {
  uint32_t lane[kLaneBits];
  uint32_t wave[kMaxWaveBits];
  uint32_t reg[kMaxRegBits];
  int32_t op_begin, op_end;
  int32_t transition;  // 1: re-lay the tile out through LDS before the ops
  int32_t pad;
};

struct alignas(16) IPart {
  IoOffsets load, store;
  uint64_t tiles;       // 2^(n-m)
  int32_t m, lb, n_stages, pad;
  int32_t tq[kMaxTile];  // tile bit -> global qubit, ascending
};

// A fused part on the device: U (2^w x 2^w, real block then imaginary
// block, row-major, in the state's precision) starts at element u_off of the
// plan's matrix buffer.
struct alignas(16) FusedDesc {
  int32_t w, m;
  uint64_t tiles;
  int32_t u_off, pad;
  int8_t sq[8];
  int8_t pq[4];
  int8_t tq[12];
};

// Tile index of coordinate bits `coord` under layout `pos` (bits < m).
__host__ __device__ inline uint32_t tile_index(const int8_t* pos, int m, uint32_t coord) {
  uint32_t t = 0;
  for (int c = 0; c < m; ++c) t |= ((coord >> c) & 1u) << pos[c];
  return t;
}

// LDS slot of tile index t.  XOR-folding the higher bits into the low
// `sw` bits spreads lanes whose tile indices share low bits over distinct
// banks for every layout whose lane bits are a run of consecutive tile
// bits.  The map is linear over XOR, so the slot of (a ^ b) is
// slot(a) ^ slot(b) and a lane's base and a register's offset can be
// swizzled separately.
__host__ __device__ inline uint32_t lds_slot(uint32_t t, int sw) {
  const uint32_t mask = (1u << sw) - 1u;
  uint32_t f = 0;
  for (uint32_t h = t >> sw; h; h >>= sw) f ^= h & mask;
  return t ^ f;
}

// Insert a zero bit at every tile qubit position: outer setting -> global
// base index of the tile (Alg. 1: the amplitudes of one outer setting).
__host__ __device__ inline uint64_t tile_base(uint64_t tile, const int8_t* tq, int m) {
  uint64_t b = tile;
  for (int i = 0; i < m; ++i) {
    const int q = tq[i];
    const uint64_t low = b & ((uint64_t(1) << q) - 1);
    b = ((b >> q) << (q + 1)) | low;
  }
  return b;
}

// Global index offset of tile index t (tile bit i -> qubit tq[i]).
__host__ __device__ inline uint64_t tile_to_global(uint32_t t, const int8_t* tq, int m) {
  uint64_t g = 0;
  for (int i = 0; i < m; ++i) g |= uint64_t((t >> i) & 1u) << tq[i];
  return g;
}

}  // namespace hisv
