// compile.cpp -- compile a part into the descriptors of the part-pass kernel.
//
// Alg. 1 (Sec. III.C) for one part p with qubit set S_p: for every setting
// of the qubits outside the part, gather the amplitudes addressed by S_p,
// run the part's gates, scatter back.  The kernel gathers a *tile*:
//   T_p = S_p plus the lowest qubits not in S_p, m qubits in all.
// Padding with low qubits is the rule of the multi-level scheme (Sec. IV:
// a part with fewer qubits than the level's limit takes extra qubits for
// spatial locality); here it makes each tile a set of contiguous runs of
// at least 2^contig amplitudes, so global loads and stores coalesce.
//
// Inside the tile the part's gates (circuit order, Sec. IV.A) are cut by the
// natural cutoff (Sec. IV.B.1) with limit rb into stages, each of which
// runs entirely on register bits; this is the second level of the
// multi-level partitioning of Sec. IV, mapped to LDS (level 1: the tile) and
// registers (level 2: the stage).  Each stage's register bits are its
// qubits, padded with high tile bits; its lane bits are the lowest
// remaining tile bits (so that lanes touch neighbouring LDS slots and, in
// the load and store layouts, neighbouring global addresses).
//
// Within a stage, runs of one-qubit gates on the same bit with no other
// gate on that bit in between are multiplied into one 2x2 in FP64 (gates on
// different bits commute, so the product can be applied where the run ends).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hisv_internal.h"

namespace hisv {

int max_tile_qubits(const CompileOptions& opt) {
  return std::min(std::min(kMaxTile, opt.max_m), kLaneBits + opt.max_wb + opt.rb);
}

namespace {

struct Layout {
  int8_t pos[kMaxTile];
};

// Layout with the given register bits (ascending); lanes take the lowest
// other tile bits, waves the rest.
Layout make_layout(int m, int lb, int wb, uint32_t regs) {
  Layout L;
  std::memset(L.pos, 0, sizeof L.pos);
  int c = 0;
  int lane_left = lb;
  std::vector<int> waves;
  for (int t = 0; t < m; ++t) {
    if (regs >> t & 1) continue;
    if (lane_left) {
      L.pos[c++] = (int8_t)t;
      --lane_left;
    } else {
      waves.push_back(t);
    }
  }
  for (int t : waves) L.pos[c++] = (int8_t)t;
  for (int t = 0; t < m; ++t)
    if (regs >> t & 1) L.pos[c++] = (int8_t)t;
  (void)wb;
  return L;
}

// Pad `regs` to exactly rb tile bits: first with bits of `keep` (the
// previous layout's register bits, highest first), then with the highest
// free tile bits.  Keeping register bits across stages lets consecutive
// layouts coincide (no re-layout) or share a register bit (a re-layout can
// then run in two halves through half the LDS).
uint32_t pad_regs(uint32_t regs, int m, int rb, uint32_t keep = 0) {
  for (int t = m - 1; t >= 0 && __builtin_popcount(regs) < rb; --t)
    if (keep >> t & 1) regs |= 1u << t;
  for (int t = m - 1; t >= 0 && __builtin_popcount(regs) < rb; --t) regs |= 1u << t;
  return regs;
}

bool lanes_are_low(const Layout& L, int lb) {
  for (int c = 0; c < lb; ++c)
    if (L.pos[c] != c) return false;
  return true;
}

// Number of leading lane bits that are tile bits 0, 1, 2, ... (the length,
// in bits, of the contiguous global run each group of lanes touches).
int low_run(const Layout& L, int lb) {
  int c = 0;
  while (c < lb && L.pos[c] == c) ++c;
  return c;
}

bool same_layout(const Layout& a, const Layout& b, int m) {
  return std::memcmp(a.pos, b.pos, (size_t)m) == 0;
}

bool is_exact(const cd& z, double re, double im) { return z.real() == re && z.imag() == im; }

void matmul2(const cd a[4], const cd b[4], cd out[4]) {  // out = a * b
  cd r[4];
  r[0] = a[0] * b[0] + a[1] * b[2];
  r[1] = a[0] * b[1] + a[1] * b[3];
  r[2] = a[2] * b[0] + a[3] * b[2];
  r[3] = a[2] * b[1] + a[3] * b[3];
  for (int i = 0; i < 4; ++i) out[i] = r[i];
}

void emit_1q(int b, const cd u[4], std::vector<HostOp>* ops) {
  HostOp op{};
  op.b0 = b;
  op.b1 = -1;
  const bool diag = is_exact(u[1], 0, 0) && is_exact(u[2], 0, 0);
  if (diag) {
    if (is_exact(u[0], 1, 0) && is_exact(u[3], 1, 0)) return;  // identity
    if (is_exact(u[0], 1, 0)) {
      op.kind = OP_D1;
      op.c[0] = u[3].real();
      op.c[1] = u[3].imag();
    } else {
      op.kind = OP_D;
      op.c[0] = u[0].real(); op.c[1] = u[0].imag();
      op.c[2] = u[3].real(); op.c[3] = u[3].imag();
    }
  } else if (is_exact(u[0], 0, 0) && is_exact(u[3], 0, 0) && is_exact(u[1], 1, 0) &&
             is_exact(u[2], 1, 0)) {
    op.kind = OP_X;
  } else if (u[0].imag() == 0 && u[1].imag() == 0 && u[2].imag() == 0 && u[3].imag() == 0) {
    op.kind = OP_R;
    for (int i = 0; i < 4; ++i) op.c[i] = u[i].real();
  } else {
    op.kind = OP_U;
    for (int i = 0; i < 4; ++i) {
      op.c[2 * i] = u[i].real();
      op.c[2 * i + 1] = u[i].imag();
    }
  }
  ops->push_back(op);
}

// Kind emit_1q gives u (-1: identity, no op).
int kind_1q(const cd u[4]) {
  if (is_exact(u[1], 0, 0) && is_exact(u[2], 0, 0)) {
    if (is_exact(u[0], 1, 0) && is_exact(u[3], 1, 0)) return -1;
    return is_exact(u[0], 1, 0) ? OP_D1 : OP_D;
  }
  if (is_exact(u[0], 0, 0) && is_exact(u[3], 0, 0) && is_exact(u[1], 1, 0) && is_exact(u[2], 1, 0))
    return OP_X;
  if (u[0].imag() == 0 && u[1].imag() == 0 && u[2].imag() == 0 && u[3].imag() == 0) return OP_R;
  return OP_U;
}

// Estimated VALU instructions per wavefront for one op on A = 2^rb
// amplitudes a lane: its arithmetic or register moves, plus what every op
// costs the interpreter (moving the sub-state back into the loop's
// registers, and the dispatch).
int op_cost(int kind, int A) {
  int c = 0;
  switch (kind) {
    case -1: return 0;
    case OP_U: c = 8 * A; break;
    case OP_R: case OP_D: c = 4 * A; break;
    case OP_D1: case OP_X: c = 2 * A; break;
    case OP_CX: case OP_CP: case OP_SWAP: c = A; break;
    case OP_CZ: c = A / 2; break;
    case OP_U2: c = 16 * A; break;
    default: c = 8 * A;
  }
  return c + A + 10;
}

// 4 x 4 matrices, basis index i = bit(b0) + 2 bit(b1), row-major.
void matmul4(const cd a[16], const cd b[16], cd out[16]) {  // out = a * b
  cd r[16];
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k) {
      cd z = 0;
      for (int j = 0; j < 4; ++j) z += a[4 * i + j] * b[4 * j + k];
      r[4 * i + k] = z;
    }
  for (int i = 0; i < 16; ++i) out[i] = r[i];
}

// The same operator with the roles of the two bits exchanged.
void swap_bits4(const cd a[16], cd out[16]) {
  auto sg = [](int i) { return (i >> 1) | ((i & 1) << 1); };
  cd r[16];
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k) r[4 * sg(i) + sg(k)] = a[4 * i + k];
  for (int i = 0; i < 16; ++i) out[i] = r[i];
}

// u0 on bit 0 and u1 on bit 1 of the 4 x 4 index (u1 (x) u0).
void kron2(const cd u0[4], const cd u1[4], cd out[16]) {
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k) out[4 * i + k] = u0[2 * (i & 1) + (k & 1)] * u1[2 * (i >> 1) + (k >> 1)];
}

// A two-qubit gate on (q0 -> bit 0, q1 -> bit 1); CX: q0 controls.
hs_status gate4(const Gate& g, cd out[16]) {
  for (int i = 0; i < 16; ++i) out[i] = 0;
  switch (g.kind) {
    case HS_CX: out[0] = out[4 * 2 + 2] = out[4 * 1 + 3] = out[4 * 3 + 1] = 1; break;
    case HS_CZ: out[0] = out[5] = out[10] = 1; out[15] = -1; break;
    case HS_CP: out[0] = out[5] = out[10] = 1; out[15] = cd(cos(g.p[0]), sin(g.p[0])); break;
    case HS_SWAP: out[0] = out[4 * 1 + 2] = out[4 * 2 + 1] = out[15] = 1; break;
    default: return fail(HS_E_ARG, "unknown two-qubit kind %d", g.kind);
  }
  return HS_OK;
}

void set_u2(HostOp* op, const cd m[16]) {
  for (int i = 0; i < 16; ++i) {
    op->c[2 * i] = m[i].real();
    op->c[2 * i + 1] = m[i].imag();
  }
}

void get_u2(const HostOp& op, cd m[16]) {
  for (int i = 0; i < 16; ++i) m[i] = cd(op.c[2 * i], op.c[2 * i + 1]);
}

// Left-multiply the U2 op by `m`, given on (r0 -> bit 0, r1 -> bit 1).
void u2_apply_after(HostOp* op, int r0, const cd m[16]) {
  cd mm[16], cur[16];
  if (r0 == op->b0) {
    for (int i = 0; i < 16; ++i) mm[i] = m[i];
  } else {
    swap_bits4(m, mm);
  }
  get_u2(*op, cur);
  matmul4(mm, cur, cur);
  set_u2(op, cur);
}

// Register-stage cut: seeded DFS orders tried per part.
constexpr uint64_t kStageSeed = 0x5eed;
constexpr int kStageTrials = 32;

}  // namespace

hs_status compile_part(int n, const std::vector<Gate>& pg, const CompileOptions& opt,
                       CompiledPart* out) {
  if (pg.empty()) return fail(HS_E_ARG, "empty part");
  uint64_t S = 0;
  for (const Gate& g : pg) S |= g.mask();
  const int C = std::min(opt.contig, n);
  const uint64_t need = S | ((C >= 64) ? ~0ull : ((1ull << C) - 1));
  int m = std::max(__builtin_popcountll(need),
                   std::min(n, std::max(kLaneBits + opt.rb,
                                        std::min(opt.min_tile, max_tile_qubits(opt)))));
  if (m > max_tile_qubits(opt))
    return fail(HS_E_UNSUPPORTED, "part needs a %d-qubit tile; the kernel holds at most %d",
                m, max_tile_qubits(opt));
  const int rb = std::min(opt.rb, m);
  const int lb = std::min(kLaneBits, m - rb);
  const int wb = m - rb - lb;
  if (wb > opt.max_wb) return fail(HS_E_UNSUPPORTED, "tile needs %d wave bits", wb);

  // tile qubits: S plus the lowest qubits outside S
  uint64_t T = S;
  for (int q = 0; q < n && __builtin_popcountll(T) < m; ++q) T |= 1ull << q;
  int8_t tq[kMaxTile] = {0};
  int bit_of[64];
  for (int q = 0, t = 0; q < n; ++q) {
    bit_of[q] = -1;
    if (T >> q & 1) {
      tq[t] = (int8_t)q;
      bit_of[q] = t++;
    }
  }

  // Second level of the multi-level partition (Sec. IV): the part's gates
  // are cut into register stages of at most rb qubits by the DFS
  // partitioner (Sec. IV.B.2; its first trial is the circuit order) and by
  // the greedy one; the cut with fewer stages, hence fewer LDS re-layouts,
  // is kept (DFS on ties).  Stages run in creation order, a topological
  // order of the stage graph; a stage's gates keep circuit order.
  struct Stage {
    uint32_t bits = 0;
    std::vector<int> gates;
  };
  for (const Gate& g : pg)
    if (g.arity() > rb) return fail(HS_E_UNSUPPORTED, "gate wider than the register stage");
  std::vector<int32_t> stage_of, greedy_of;
  const Dag pdag = build_dag(pg);
  int nst = partition_dfs(pg, pdag, rb, kStageSeed, kStageTrials, &stage_of);
  const int ngr = partition_greedy(pg, pdag, rb, kStageSeed, kStageTrials, &greedy_of);
  if (ngr < nst) {
    nst = ngr;
    stage_of.swap(greedy_of);
  }
  std::vector<Stage> st(nst);
  for (int i = 0; i < (int)pg.size(); ++i) {
    Stage& S = st[stage_of[i]];
    S.bits |= 1u << bit_of[pg[i].q0];
    if (pg[i].q1 >= 0) S.bits |= 1u << bit_of[pg[i].q1];
    S.gates.push_back(i);
  }

  out->desc = PartDesc{};
  out->desc.m = m;
  out->desc.lb = lb;
  out->desc.wb = wb;
  out->desc.rb = rb;
  out->desc.tiles = uint64_t(1) << (n - m);
  std::memcpy(out->desc.tq, tq, sizeof tq);
  out->rb_kernel = rb;
  out->stages.clear();
  out->ops.clear();

  std::vector<Layout> lay;
  uint32_t prev_regs = pad_regs(0u, m, rb);  // the registers of a fresh load layout
  for (const Stage& s : st) {
    const uint32_t regs = pad_regs(s.bits, m, rb, prev_regs);
    lay.push_back(make_layout(m, lb, wb, regs));
    prev_regs = regs;
  }
  // load and store layouts: lanes on tile bits 0..lb-1 (contiguous global runs)
  auto io_layout = [&](const Layout& near) {
    if (lanes_are_low(near, lb) || low_run(near, lb) >= std::min(opt.min_run, lb)) return near;
    return make_layout(m, lb, wb, pad_regs(0u, m, rb));
  };
  const Layout load = io_layout(lay.front());
  const Layout store = io_layout(lay.back());

  auto push_entry = [&](const Layout& L, const Layout* prev) {
    StageDesc e{};
    std::memcpy(e.pos, L.pos, sizeof e.pos);
    e.transition = (prev && !same_layout(L, *prev, m)) ? 1 : 0;
    e.op_begin = e.op_end = (int)out->ops.size();
    out->stages.push_back(e);
    return &out->stages.back();
  };
  int trips = 0;
  push_entry(load, nullptr);
  const Layout* prev = &load;
  for (size_t s = 0; s < st.size(); ++s) {
    StageDesc* e = push_entry(lay[s], prev);
    trips += e->transition;
    // register index of each tile bit in this layout
    int reg_of[kMaxTile];
    for (int t = 0; t < kMaxTile; ++t) reg_of[t] = -1;
    for (int r = 0; r < rb; ++r) reg_of[lay[s].pos[lb + wb + r]] = r;
    cd pend[kMaxTile][4];
    bool has[kMaxTile] = {false};
    // latest op on each register bit in this stage (-1: none): a dense
    // 4 x 4 op that is still the latest on a bit absorbs later gates there
    int last[kMaxTile];
    for (int r = 0; r < kMaxTile; ++r) last[r] = -1;
    const int A = 1 << rb;
    auto open_u2 = [&](int r) { return opt.fuse2 && last[r] >= 0 && out->ops[last[r]].kind == OP_U2; };
    const cd I2[4] = {1, 0, 0, 1};
    auto flush = [&](int r) {
      if (!has[r]) return;
      has[r] = false;
      if (open_u2(r)) {
        HostOp& o = out->ops[last[r]];
        cd m[16];
        kron2(r == o.b0 ? pend[r] : I2, r == o.b0 ? I2 : pend[r], m);
        u2_apply_after(&o, o.b0, m);
        return;
      }
      const size_t before = out->ops.size();
      emit_1q(r, pend[r], &out->ops);
      if (out->ops.size() > before) last[r] = (int)before;
    };
    // cost of applying r's pending one-qubit gates on their own
    auto pend_cost = [&](int r) { return (!has[r] || open_u2(r)) ? 0 : op_cost(kind_1q(pend[r]), A); };
    for (int i : st[s].gates) {
      const Gate& g = pg[i];
      const int r0 = reg_of[bit_of[g.q0]];
      if (g.arity() == 1) {
        cd u[4];
        gate_matrix(g, u);
        if (has[r0]) {
          matmul2(u, pend[r0], pend[r0]);
        } else {
          for (int j = 0; j < 4; ++j) pend[r0][j] = u[j];
          has[r0] = true;
        }
        continue;
      }
      const int r1 = reg_of[bit_of[g.q1]];
      if (opt.fuse2) {
        cd m[16], pm[16];
        if (hs_status rc = gate4(g, m)) return rc;
        kron2(has[r0] ? pend[r0] : I2, has[r1] ? pend[r1] : I2, pm);
        matmul4(m, pm, m);  // the pending one-qubit gates come first
        const int gk = g.kind == HS_CX ? OP_CX : g.kind == HS_CZ ? OP_CZ : g.kind == HS_CP ? OP_CP : OP_SWAP;
        if (open_u2(r0) && last[r0] == last[r1]) {  // same pair: absorb
          u2_apply_after(&out->ops[last[r0]], r0, m);
          has[r0] = has[r1] = false;
          continue;
        }
        if (op_cost(OP_U2, A) < pend_cost(r0) + pend_cost(r1) + op_cost(gk, A)) {
          HostOp op{};
          op.kind = OP_U2;
          op.b0 = std::min(r0, r1);
          op.b1 = std::max(r0, r1);
          cd mm[16];
          if (r0 < r1) {
            for (int j = 0; j < 16; ++j) mm[j] = m[j];
          } else {
            swap_bits4(m, mm);
          }
          set_u2(&op, mm);
          has[r0] = has[r1] = false;
          last[r0] = last[r1] = (int)out->ops.size();
          out->ops.push_back(op);
          continue;
        }
      }
      flush(r0);
      flush(r1);
      last[r0] = last[r1] = (int)out->ops.size();
      HostOp op{};
      op.b0 = r0;
      op.b1 = r1;
      switch (g.kind) {
        case HS_CX: op.kind = OP_CX; break;
        case HS_CZ: op.kind = OP_CZ; break;
        case HS_CP:
          op.kind = OP_CP;
          op.c[0] = cos(g.p[0]);
          op.c[1] = sin(g.p[0]);
          break;
        case HS_SWAP: op.kind = OP_SWAP; break;
        default: return fail(HS_E_ARG, "unknown two-qubit kind %d", g.kind);
      }
      out->ops.push_back(op);
    }
    for (int r = 0; r < rb; ++r) flush(r);
    out->stages.back().op_end = (int)out->ops.size();
    prev = &lay[s];
  }
  StageDesc* e = push_entry(store, prev);
  trips += e->transition;
  out->desc.n_stages = (int)out->stages.size();
  out->desc.lds_bytes = 0;  // set per dtype at upload
  out->lds_round_trips = trips;
  return HS_OK;
}

}  // namespace hisv

namespace hisv {

// ---- fused path: one dense unitary per part -----------------------------------
//
// U_p = product of the part's gates (circuit order), built in FP64 by
// applying each gate to every column of the identity as a state of the
// part's qubits (inner slot b = the b-th smallest part qubit, the slot order
// of Alg. 1's worked example).  Parts narrower than 4 qubits take the lowest
// other qubits as extra slots (U acts as the identity on them).
hs_status compile_fused(int n, const std::vector<Gate>& pg, FusedPart* out) {
  uint64_t S = 0;
  for (const Gate& g : pg) S |= g.mask();
  for (int q = 0; q < n && __builtin_popcountll(S) < 4; ++q) S |= 1ull << q;
  const int w = __builtin_popcountll(S);
  if (w > kMaxFusedQubits)
    return fail(HS_E_UNSUPPORTED, "fused path takes parts of at most %d qubits (got %d)", kMaxFusedQubits, w);
  if (n < w + 4) return fail(HS_E_UNSUPPORTED, "fused path needs n >= %d", w + 4);
  FusedPart f;
  f.w = w;
  f.m = w + 4;
  f.tiles = uint64_t(1) << (n - f.m);
  int slot[64];
  for (int q = 0, b = 0; q < n; ++q) {
    slot[q] = -1;
    if (S >> q & 1) {
      f.sq[b] = (int8_t)q;
      slot[q] = b++;
    }
  }
  uint64_t T = S;
  for (int q = 0, c = 0; q < n && c < 4; ++q)
    if (!(S >> q & 1)) {
      f.pq[c++] = (int8_t)q;
      T |= 1ull << q;
    }
  for (int q = 0, t = 0; q < n; ++q)
    if (T >> q & 1) f.tq[t++] = (int8_t)q;
  const int R = 1 << w;
  f.u.assign((size_t)R * R, cd(0.0, 0.0));
  for (int i = 0; i < R; ++i) f.u[(size_t)i * R + i] = 1.0;
  // apply a gate to every column: column c is a 2^w state vector
  for (const Gate& g : pg) {
    const int a = slot[g.q0];
    if (g.arity() == 1) {
      cd m[4];
      gate_matrix(g, m);
      for (int c = 0; c < R; ++c)
        for (int r0 = 0; r0 < R; ++r0) {
          if (r0 >> a & 1) continue;
          const int r1 = r0 | (1 << a);
          const cd x = f.u[(size_t)r0 * R + c], y = f.u[(size_t)r1 * R + c];
          f.u[(size_t)r0 * R + c] = m[0] * x + m[1] * y;
          f.u[(size_t)r1 * R + c] = m[2] * x + m[3] * y;
        }
      continue;
    }
    const int b = slot[g.q1];
    const cd ph = g.kind == HS_CP ? std::polar(1.0, g.p[0]) : cd(-1.0, 0.0);
    for (int c = 0; c < R; ++c)
      for (int r = 0; r < R; ++r) {
        const bool ba = r >> a & 1, bb = r >> b & 1;
        cd& v = f.u[(size_t)r * R + c];
        switch (g.kind) {
          case HS_CX:  // control a, target b: swap the pair with a = 1
            if (ba && !bb) std::swap(v, f.u[(size_t)(r | (1 << b)) * R + c]);
            break;
          case HS_CZ:
          case HS_CP:
            if (ba && bb) v *= ph;
            break;
          case HS_SWAP:
            if (ba && !bb) std::swap(v, f.u[(size_t)(r ^ (1 << a) ^ (1 << b)) * R + c]);
            break;
          default: return fail(HS_E_ARG, "unknown two-qubit kind %d", g.kind);
        }
      }
  }
  *out = std::move(f);
  return HS_OK;
}

}  // namespace hisv

namespace hisv {

// Relative cost of a part on the interpreter kernel (one HBM sweep of the
// state = 1), fitted to per-part timings of 30-qubit states (random,
// layered and dressed-pair circuits; 820 parts, mean |log error| 0.05): a
// smooth maximum of the sweep (+0.04 / 0.02 per LDS re-layout, complex64 /
// complex128) and the vector-ALU work -- 0.0065 / 0.005 sweep per flop per
// amplitude (Sec. III.A's counting), plus 0.005 per register op for
// complex128 (the dispatch; the register ops no longer copy the sub-state
// back).  Used by AUTO only.
double lds_part_cost(const CompiledPart& cp, hs_dtype dt) {
  static const double flops[OP_NUM] = {14, 6, 6, 3, 0, 0, 0.5, 1.5, 0, 30};
  const bool f32 = dt == HS_C64;
  const double mem = 1.0 + (f32 ? 0.04 : 0.02) * cp.lds_round_trips;
  double f = 0;
  for (const HostOp& op : cp.ops) f += flops[op.kind];
  const double alu = (f32 ? 0.0065 : 0.005) * f + (f32 ? 0.0 : 0.005) * (double)cp.ops.size();
  return std::cbrt(mem * mem * mem + alu * alu * alu);
}

// The specialized kernels keep the sweep near the HBM rate while a part's
// arithmetic is light: an LDS re-layout costs about 0.03 sweep, and
// register permutations (X, CX, SWAP) are free (compile-time renames).
// Heavier parts become vector-ALU bound.  Per-part timings of 30-qubit
// states (random, layered and dressed-pair circuits, both precisions) fit
// a smooth maximum of the sweep and 0.0045 sweep per flop per amplitude
// (Sec. III.A's counting: a dense 2 x 2 is 14 flops per amplitude): flat at
// ~1.1 sweeps below ~200 flops per amplitude, 1.6-1.7 at 350, 2.1-2.3 at
// 500, 4.2-4.8 at 1,000.
double spec_part_cost(const CompiledPart& cp, hs_dtype dt) {
  static const double flops[OP_NUM] = {14, 6, 6, 3, 0, 0, 0.5, 1.5, 0, 30};
  const double mem = (dt == HS_C64 ? 1.05 : 1.0) + 0.03 * cp.lds_round_trips;
  double f = 0;
  for (const HostOp& op : cp.ops) f += flops[op.kind];
  const double alu = 0.0045 * f;
  return std::sqrt(std::sqrt(mem * mem * mem * mem + alu * alu * alu * alu));
}

// The fused kernel does 8 * 2^w flops per amplitude on matrix cores against
// 2 * s bytes of HBM traffic (s = 8 or 16 bytes per amplitude).  Per-part timings on
// 30-qubit states (random, layered and dressed-pair circuits), in sweeps:
// w = 6 and 7 are matrix-core bound; w <= 5 overlap their loads with the
// products only in part.  Complex64 parts that hold one of qubits 0..3 (the
// 16 columns of a wave are then not one contiguous run) cost ~0.1 more.
double fused_part_cost(const FusedPart& f, hs_dtype dt) {
  static const double c64[8] = {0, 0, 0, 0, 1.17, 1.29, 2.13, 3.37};
  static const double c128[8] = {0, 0, 0, 0, 1.10, 1.25, 1.69, 2.92};
  if (f.w < 4 || f.w > 7) return 1e30;
  const bool coalesced = f.pq[0] == 0 && f.pq[1] == 1 && f.pq[2] == 2 && f.pq[3] == 3;
  if (dt == HS_C64) return c64[f.w] + (coalesced ? 0.0 : 0.1);
  return c128[f.w];
}

}  // namespace hisv
