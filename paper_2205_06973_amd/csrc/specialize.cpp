// specialize.cpp -- per-part specialized part-pass kernels, built at plan time.
//
// The part-pass kernel in kernels.hip interprets a part's descriptors: every
// register operation is dispatched at run time on its kind and bit
// positions.  For long-running plans this file instead turns each compiled
// part (tile qubits, load / stage / store layouts, register operations and
// their coefficients) into straight-line HIP source -- register indices, LDS
// offsets and coefficients become compile-time constants -- compiles it with
// hipRTC for gfx950 and caches the resulting kernel.  The computation is the
// same Alg. 1 sweep (gather the tile, run the stages, scatter it back).  By
// default a launch has one workgroup per tile and each XCD sweeps a
// contiguous eighth of the tiles; a persistent grid that keeps the next
// tile's loads in flight is the alternative shape.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstring>
#include <functional>
#include <sstream>

#include "hisv_internal.h"

namespace hisv {

namespace {

std::string lit(double v, bool f32) {
  char buf[64];
  if (f32) {
    const float x = (float)v;
    if (x == 0.0f) return std::signbit(x) ? "(-0.0f)" : "0.0f";
    snprintf(buf, sizeof buf, "(%af)", x);
  } else {
    if (v == 0.0) return std::signbit(v) ? "(-0.0)" : "0.0";
    snprintf(buf, sizeof buf, "(%a)", v);
  }
  return buf;
}

// value of coordinate bits -> tile index, for the register bits of a layout
uint32_t reg_tile_offset(const StageDesc& e, int lb, int wb, int rb, int j) {
  uint32_t t = 0;
  for (int r = 0; r < rb; ++r)
    if (j >> r & 1) t |= 1u << e.pos[lb + wb + r];
  return t;
}

uint32_t slot(uint32_t t, int sw) {
  const uint32_t mask = (1u << sw) - 1u;
  uint32_t f = 0;
  for (uint32_t h = t >> sw; h; h >>= sw) f ^= h & mask;
  return t ^ f;
}

struct Emit {
  std::ostringstream o;
  bool f32;
  int rb;
  std::string T() const { return f32 ? "float" : "double"; }
};

// a[j] register names: ar<j>, ai<j>
void emit_op(Emit& E, const HostOp& op) {
  const int N = 1 << E.rb;
  auto& o = E.o;
  const bool f = E.f32;
  auto L = [&](double v) { return lit(v, f); };
  switch (op.kind) {
    case OP_U: {
      const double* c = op.c;
      for (int j = 0; j < N; ++j) {
        if (j >> op.b0 & 1) continue;
        const int k = j | (1 << op.b0);
        o << "  { const " << E.T() << " px = ar" << j << ", py = ai" << j << ", qx = ar" << k
          << ", qy = ai" << k << ";\n"
          << "    ar" << j << " = " << L(c[0]) << "*px - " << L(c[1]) << "*py + " << L(c[2]) << "*qx - "
          << L(c[3]) << "*qy;\n"
          << "    ai" << j << " = " << L(c[0]) << "*py + " << L(c[1]) << "*px + " << L(c[2]) << "*qy + "
          << L(c[3]) << "*qx;\n"
          << "    ar" << k << " = " << L(c[4]) << "*px - " << L(c[5]) << "*py + " << L(c[6]) << "*qx - "
          << L(c[7]) << "*qy;\n"
          << "    ai" << k << " = " << L(c[4]) << "*py + " << L(c[5]) << "*px + " << L(c[6]) << "*qy + "
          << L(c[7]) << "*qx; }\n";
      }
      break;
    }
    case OP_R: {
      const double* c = op.c;
      for (int j = 0; j < N; ++j) {
        if (j >> op.b0 & 1) continue;
        const int k = j | (1 << op.b0);
        o << "  { const " << E.T() << " px = ar" << j << ", py = ai" << j << ", qx = ar" << k
          << ", qy = ai" << k << ";\n"
          << "    ar" << j << " = " << L(c[0]) << "*px + " << L(c[1]) << "*qx; ai" << j << " = "
          << L(c[0]) << "*py + " << L(c[1]) << "*qy;\n"
          << "    ar" << k << " = " << L(c[2]) << "*px + " << L(c[3]) << "*qx; ai" << k << " = "
          << L(c[2]) << "*py + " << L(c[3]) << "*qy; }\n";
      }
      break;
    }
    case OP_D:
    case OP_D1:
    case OP_CP:
    case OP_CZ: {
      for (int j = 0; j < N; ++j) {
        double cr, ci;
        if (op.kind == OP_D) {
          const bool one = j >> op.b0 & 1;
          cr = one ? op.c[2] : op.c[0];
          ci = one ? op.c[3] : op.c[1];
        } else if (op.kind == OP_D1) {
          if (!(j >> op.b0 & 1)) continue;
          cr = op.c[0];
          ci = op.c[1];
        } else {
          if (!((j >> op.b0 & 1) && (j >> op.b1 & 1))) continue;
          if (op.kind == OP_CZ) {
            o << "  ar" << j << " = -ar" << j << "; ai" << j << " = -ai" << j << ";\n";
            continue;
          }
          cr = op.c[0];
          ci = op.c[1];
        }
        o << "  { const " << E.T() << " px = ar" << j << ", py = ai" << j << ";\n"
          << "    ar" << j << " = px*" << L(cr) << " - py*" << L(ci) << "; ai" << j << " = px*" << L(ci)
          << " + py*" << L(cr) << "; }\n";
      }
      break;
    }
    case OP_X:
    case OP_CX:
    case OP_SWAP: {
      for (int j = 0; j < N; ++j) {
        int k;
        if (op.kind == OP_X) {
          if (j >> op.b0 & 1) continue;
          k = j | (1 << op.b0);
        } else if (op.kind == OP_CX) {
          if (!(j >> op.b0 & 1) || (j >> op.b1 & 1)) continue;
          k = j | (1 << op.b1);
        } else {
          if (!(j >> op.b0 & 1) || (j >> op.b1 & 1)) continue;
          k = j ^ (1 << op.b0) ^ (1 << op.b1);
        }
        o << "  { const " << E.T() << " tx = ar" << j << ", ty = ai" << j << "; ar" << j << " = ar" << k
          << "; ai" << j << " = ai" << k << "; ar" << k << " = tx; ai" << k << " = ty; }\n";
      }
      break;
    }
    case OP_U2: {
      const double* c = op.c;
      for (int j = 0; j < N; ++j) {
        if ((j >> op.b0 & 1) || (j >> op.b1 & 1)) continue;
        const int ix[4] = {j, j | (1 << op.b0), j | (1 << op.b1), j | (1 << op.b0) | (1 << op.b1)};
        o << "  { const " << E.T();
        for (int q = 0; q < 4; ++q)
          o << (q ? ", " : " ") << "x" << q << "r = ar" << ix[q] << ", x" << q << "i = ai" << ix[q];
        o << ";\n";
        for (int i = 0; i < 4; ++i) {
          o << "    ar" << ix[i] << " =";
          for (int k = 0; k < 4; ++k)
            o << (k ? " + " : " ") << L(c[8 * i + 2 * k]) << "*x" << k << "r - " << L(c[8 * i + 2 * k + 1])
              << "*x" << k << "i";
          o << ";\n    ai" << ix[i] << " =";
          for (int k = 0; k < 4; ++k)
            o << (k ? " + " : " ") << L(c[8 * i + 2 * k]) << "*x" << k << "i + " << L(c[8 * i + 2 * k + 1])
              << "*x" << k << "r";
          o << ";\n";
        }
        o << "  }\n";
      }
      break;
    }
    default: break;
  }
}

// Global index contributed by the lane and wave bits of layout e.
void emit_thread_offsets(Emit& E, const StageDesc& e, const PartDesc& d, const char* lane_var,
                         const char* wave_var, const char* out_lane, const char* out_wave) {
  auto& o = E.o;
  // 64-bit: lanes may carry any tile qubit (up to n - 1)
  o << "    const unsigned long long " << out_lane << " = 0ull";
  for (int c = 0; c < d.lb; ++c)
    o << " | ((unsigned long long)((" << lane_var << " >> " << c << ") & 1u) << "
      << (int)d.tq[e.pos[c]] << ")";
  o << ";\n    const unsigned long long " << out_wave << " = 0ull";
  for (int c = 0; c < d.wb; ++c)
    o << " | ((unsigned long long)((" << wave_var << " >> " << c << ") & 1u) << "
      << (int)d.tq[e.pos[d.lb + c]] << ")";
  o << ";\n";
}

void emit_io(Emit& E, const StageDesc& e, const PartDesc& d, bool store, const char* prefix,
             const char* base) {
  auto& o = E.o;
  const int N = 1 << E.rb;
  for (int j = 0; j < N; ++j) {
    uint64_t g = 0;
    const uint32_t t = reg_tile_offset(e, d.lb, d.wb, E.rb, j);
    for (int i = 0; i < d.m; ++i)
      if (t >> i & 1) g |= uint64_t(1) << d.tq[i];
    if (store)
      o << "      " << base << "[" << g << "ull] = make_v(ar" << j << ", ai" << j << ");\n";
    else
      o << "      { const V v = " << base << "[" << g << "ull]; " << prefix << "r" << j << " = v.x; "
        << prefix << "i" << j << " = v.y; }\n";
  }
}

// Tile bits removed from LDS indices when a re-layout runs in 2^s rounds:
// round h moves only the amplitudes whose split bits equal h, so the LDS
// holds 2^(m-s) amplitudes.  Any tile bit can split: as a register bit of a
// layout it selects half of each thread's registers, as a wave or lane bit
// half of the threads.  Register bits are cheapest (no idle threads), then
// wave bits (whole wavefronts wait), then lane bits.
std::vector<int> split_bits(const StageDesc& from, const StageDesc& to, const PartDesc& d, int s) {
  auto cost = [&](const StageDesc& e, int t) {
    for (int c = 0; c < d.m; ++c)
      if (e.pos[c] == t) return c >= d.lb + d.wb ? 0 : (c >= d.lb ? 1 : 2);
    return 3;
  };
  std::vector<std::pair<int, int>> cand;
  for (int t = 0; t < d.m; ++t) cand.push_back({cost(from, t) + cost(to, t), -t});
  std::sort(cand.begin(), cand.end());
  std::vector<int> out;
  for (int i = 0; i < s && i < (int)cand.size(); ++i) out.push_back(-cand[i].second);
  std::sort(out.begin(), out.end());
  return out;
}

// tile index with the split bits removed
uint32_t compress(uint32_t x, const std::vector<int>& sb) {
  for (int i = (int)sb.size() - 1; i >= 0; --i) {
    const int t = sb[i];
    x = (x & ((1u << t) - 1u)) | ((x >> (t + 1)) << t);
  }
  return x;
}

void emit_transition(Emit& E, const StageDesc& from, const StageDesc& to, const PartDesc& d, int sw,
                     int nsplit) {
  auto& o = E.o;
  const int N = 1 << E.rb;
  const int tb = d.lb + d.wb;
  const std::vector<int> sb = split_bits(from, to, d, nsplit);
  auto is_split = [&](int t) { return std::find(sb.begin(), sb.end(), t) != sb.end(); };
  auto cpos = [&](int t) {
    int c = t;
    for (int b : sb) c -= b < t;
    return c;
  };
  // LDS slot of this thread's coordinates (split bits dropped)
  auto thread_slot = [&](const StageDesc& e, const char* name) {
    o << "    const unsigned " << name << " = sl(0u";
    for (int c = 0; c < tb; ++c)
      if (!is_split(e.pos[c]))
        o << " | (((thr >> " << c << ") & 1u) << " << cpos(e.pos[c]) << ")";
    o << ");\n";
  };
  // condition on this thread's coordinates for round h ("" = always)
  auto thread_cond = [&](const StageDesc& e, int h) {
    std::string c;
    for (int i = 0; i < (int)sb.size(); ++i)
      for (int k = 0; k < tb; ++k)
        if (e.pos[k] == sb[i])
          c += (c.empty() ? "" : " && ") + std::string("((thr >> ") + std::to_string(k) + ") & 1u) == " +
               std::to_string(h >> i & 1) + "u";
    return c;
  };
  // does register j of layout e belong to round h?
  auto reg_in_round = [&](const StageDesc& e, int j, int h) {
    for (int i = 0; i < (int)sb.size(); ++i)
      for (int r = 0; r < E.rb; ++r)
        if (e.pos[tb + r] == sb[i] && (j >> r & 1) != (h >> i & 1)) return false;
    return true;
  };
  o << "    {\n";
  thread_slot(from, "wb_");
  thread_slot(to, "rb_");
  // split rounds read into their own temporaries (s*), never into the
  // prefetch registers (n*) that hold the next tile's amplitudes
  const std::string dst = sb.empty() ? "a" : "s";
  for (int h = 0; h < (1 << sb.size()); ++h) {
    o << "    __syncthreads();\n";
    std::string wc = thread_cond(from, h);
    if (d.lb < 6) wc = wc.empty() ? "active" : "active && " + wc;
    o << "    if (" << (wc.empty() ? "true" : wc) << ") {\n";
    for (int j = 0; j < N; ++j)
      if (reg_in_round(from, j, h))
        o << "      lds[wb_ ^ " << slot(compress(reg_tile_offset(from, d.lb, d.wb, E.rb, j), sb), sw)
          << "u] = make_v(ar" << j << ", ai" << j << ");\n";
    o << "    }\n    __syncthreads();\n";
    const std::string rc = thread_cond(to, h);
    o << "    if (" << (rc.empty() ? "true" : rc) << ") {\n";
    for (int j = 0; j < N; ++j)
      if (reg_in_round(to, j, h))
        o << "      { const V v = lds[rb_ ^ "
          << slot(compress(reg_tile_offset(to, d.lb, d.wb, E.rb, j), sb), sw) << "u]; " << dst << "r"
          << j << " = v.x; " << dst << "i" << j << " = v.y; }\n";
    o << "    }\n";
  }
  if (!sb.empty())
    for (int j = 0; j < N; ++j) o << "    ar" << j << " = sr" << j << "; ai" << j << " = si" << j << ";\n";
  o << "    }\n";
}

}  // namespace

std::string specialize_part_source(const CompiledPart& cp, hs_dtype dt, const std::string& name,
                                   bool standalone) {
  Emit E;
  E.f32 = dt == HS_C64;
  E.rb = cp.rb_kernel;
  const PartDesc& d = cp.desc;
  const int N = 1 << E.rb;
  const int sw = E.f32 ? 4 : 3;
  const int ne = (int)cp.stages.size();
  auto& o = E.o;
  const std::string T = E.T();
  const bool pf = cp.launch.prefetch && cp.launch.per_cu > 0;
  // LDS re-layouts run in 2^nsplit rounds so that the tile's LDS image stays
  // within the limit (more workgroups per CU)
  const size_t vbytes = E.f32 ? 8 : 16;
  int nsplit = 0;
  while (cp.lds_round_trips && ((size_t(1) << (d.m - nsplit)) * vbytes) > cp.launch.lds_limit &&
         nsplit < 2)
    ++nsplit;
  // hipRTC predefines the HIP language keywords; an offline hipcc build of
  // the same source (used to inspect it) takes them from the runtime header
  if (standalone) o << "#ifndef __HIPCC_RTC__\n#include <hip/hip_runtime.h>\n#endif\n";
  o << "typedef " << T << " T;\n"
    << "typedef struct __attribute__((aligned(" << 2 * (E.f32 ? 4 : 8) << "))) { T x, y; } V;\n"
    << "static __device__ inline __attribute__((always_inline)) V make_v(T x, T y) { V v; v.x = x; v.y = y; return v; }\n"
    << "static __device__ inline __attribute__((always_inline)) unsigned sl(unsigned t) { unsigned f = 0u, h = t >> " << sw
    << "; while (h) { f ^= h & " << ((1 << sw) - 1) << "u; h >>= " << sw << "; } return t ^ f; }\n";
  o << "extern \"C\" __global__ void __launch_bounds__(" << (64 << d.wb) << ") " << name
    << "(V* __restrict__ st, unsigned long long tiles, unsigned xcd) {\n";
  if (cp.lds_round_trips) o << "  __shared__ V lds[" << (1u << (d.m - nsplit)) << "];\n";
  o << "  const unsigned lane = threadIdx.x & 63u;\n"
    << "  const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n"
    << "  const unsigned thr = lane | (wave << " << d.lb << ");\n"
    << "  const bool active = lane < " << (1u << d.lb) << "u;\n"
    << "  (void)thr; (void)active;\n";
  o << "  " << T << " ";
  for (int j = 0; j < N; ++j) o << "ar" << j << ", ai" << j << (j + 1 < N ? ", " : ";\n");
  if (pf) {  // the next tile's amplitudes (persistent grid with prefetch)
    o << "  " << T << " ";
    for (int j = 0; j < N; ++j) o << "nr" << j << ", ni" << j << (j + 1 < N ? ", " : ";\n");
  }
  if (nsplit) {  // destinations of split re-layout rounds
    o << "  " << T << " ";
    for (int j = 0; j < N; ++j) o << "sr" << j << ", si" << j << (j + 1 < N ? ", " : ";\n");
  }
  // tile base: insert a zero bit at every tile qubit (ascending)
  o << "  auto base_of = [&](unsigned long long t) -> unsigned long long {\n    unsigned long long b = t;\n";
  for (int i = 0; i < d.m; ++i) {
    const int q = d.tq[i];
    o << "    b = ((b >> " << q << ") << " << (q + 1) << ") | (b & " << ((uint64_t(1) << q) - 1) << "ull);\n";
  }
  o << "    return b;\n  };\n";
  // load layout offsets
  o << "  {\n";
  emit_thread_offsets(E, cp.stages[0], d, "lane", "wave", "lo_ld", "wo_ld");
  emit_thread_offsets(E, cp.stages[ne - 1], d, "lane", "wave", "lo_st", "wo_st");
  // tiles walked by this workgroup: with xcd set (grid and tiles multiples
  // of 8), XCD x = blockIdx % 8 owns the contiguous run [x T/8, (x+1) T/8)
  o << "  unsigned long long tile = blockIdx.x, step = gridDim.x, end = tiles;\n"
    << "  if (xcd) {\n"
    << "    const unsigned long long per = tiles >> 3;\n"
    << "    tile = (unsigned long long)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);\n"
    << "    step = gridDim.x >> 3;\n"
    << "    end = (unsigned long long)((blockIdx.x & 7u) + 1u) * per;\n"
    << "  }\n";
  if (pf) {
    o << "  if (tile < end && active) {\n"
      << "    const V* p = st + base_of(tile) + wo_ld + lo_ld;\n";
    emit_io(E, cp.stages[0], d, false, "a", "p");
    o << "  }\n";
  }
  o << "  for (; tile < end; tile += step) {\n"
    << "    const unsigned long long tb = base_of(tile);\n";
  if (pf) {
    o << "    const unsigned long long nt = tile + step;\n"
      << "    if (nt < end && active) {\n"
      << "      const V* p = st + base_of(nt) + wo_ld + lo_ld;\n";
    emit_io(E, cp.stages[0], d, false, "n", "p");
    o << "    }\n";
  } else {
    o << "    if (active) {\n"
      << "      const V* p = st + tb + wo_ld + lo_ld;\n";
    emit_io(E, cp.stages[0], d, false, "a", "p");
    o << "    }\n";
  }
  for (int s = 1; s < ne; ++s) {
    const StageDesc& e = cp.stages[s];
    if (e.transition) emit_transition(E, cp.stages[s - 1], e, d, sw, nsplit);
    for (int i = e.op_begin; i < e.op_end; ++i) emit_op(E, cp.ops[i]);
  }
  o << "    if (active) {\n"
    << "      V* p = st + tb + wo_st + lo_st;\n";
  emit_io(E, cp.stages[ne - 1], d, true, "a", "p");
  o << "    }\n";
  if (pf)
    for (int j = 0; j < N; ++j) o << "    ar" << j << " = nr" << j << "; ai" << j << " = ni" << j << ";\n";
  o << "  }\n  }\n}\n";
  return o.str();
}

// ---- compile / cache / launch ----------------------------------------------------

struct SpecKernel {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  int block = 64;
  int per_cu = 1;  // resident workgroups per CU (occupancy)
  int cus = 1;
};

namespace {
std::mutex g_spec_mu;
// keyed by (device, full generated source): a hash alone could map two
// different parts onto one kernel
std::map<std::pair<int, std::string>, std::shared_ptr<SpecKernel>> g_spec;

hs_status rtc_compile(const std::string& src, const std::string& name, std::vector<char>* code) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), (name + ".hip").c_str(), 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS)
    return fail(HS_E_HIP, "hiprtcCreateProgram failed");
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops"};
  hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return fail(HS_E_HIP, "hipRTC failed for %s: %s", name.c_str(), log.substr(0, 400).c_str());
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code->resize(n);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  return HS_OK;
}
}  // namespace

// Compile and load the specialized kernels of every part of a plan for
// `dtype` on `device`; returns one kernel per part.  Kernels already in the
// cache (same device, same generated source) are reused; the others are
// built together as ONE hipRTC program, each part's code in a namespace of
// its own under a distinct kernel name: hipRTC serialises compilations
// within a process, and one program of many kernels pays the per-program
// front-end and code-object costs once instead of once per part.
hs_status specialize_plan(const std::vector<CompiledPart>& parts, hs_dtype dt, int device,
                          std::vector<std::shared_ptr<SpecKernel>>* out) {
  const int P = (int)parts.size();
  std::vector<std::string> src(P);
  out->assign(P, nullptr);
  std::vector<int> todo;
  for (int i = 0; i < P; ++i) src[i] = specialize_part_source(parts[i], dt, "part_pass_spec");
  {
    std::lock_guard<std::mutex> lk(g_spec_mu);
    for (int i = 0; i < P; ++i) {
      auto it = g_spec.find({device, src[i]});
      if (it != g_spec.end()) (*out)[i] = it->second;
      else todo.push_back(i);
    }
  }
  // dedupe identical sources among the parts still to build
  std::map<std::string, int> first;
  std::vector<int> build;
  for (int i : todo)
    if (first.emplace(src[i], i).second) build.push_back(i);
  if (!build.empty()) {
    std::string prog = "#ifndef __HIPCC_RTC__\n#include <hip/hip_runtime.h>\n#endif\n";
    for (size_t b = 0; b < build.size(); ++b)
      prog += "namespace part" + std::to_string(b) + " {\n" +
              specialize_part_source(parts[build[b]], dt, "part_pass_spec_" + std::to_string(b), false) +
              "}\n";
    std::vector<char> code;
    if (hs_status rc = rtc_compile(prog, "parts", &code)) return rc;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
      return fail(HS_E_HIP, "device attribute query failed");
    // the module stays loaded for the life of the process, like the cache
    hipModule_t mod = nullptr;
    if (hipModuleLoadData(&mod, code.data()) != hipSuccess) return fail(HS_E_HIP, "hipModuleLoadData failed");
    std::lock_guard<std::mutex> lk(g_spec_mu);
    for (size_t b = 0; b < build.size(); ++b) {
      const int i = build[b];
      auto k = std::make_shared<SpecKernel>();
      k->mod = mod;
      const std::string fname = "part_pass_spec_" + std::to_string(b);
      if (hipModuleGetFunction(&k->fn, mod, fname.c_str()) != hipSuccess)
        return fail(HS_E_HIP, "hipModuleGetFunction(%s) failed", fname.c_str());
      k->block = 64 << parts[i].desc.wb;
      int per_cu = 0;
      if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k->fn, k->block, 0) != hipSuccess ||
          per_cu < 1)
        return fail(HS_E_HIP, "occupancy query failed for a specialized part");
      k->per_cu = per_cu;
      k->cus = cus;
      g_spec[{device, src[i]}] = k;
    }
  }
  std::lock_guard<std::mutex> lk(g_spec_mu);
  for (int i : todo) (*out)[i] = g_spec[{device, src[i]}];
  return HS_OK;
}

hs_status launch_specialized(const SpecKernel& k, const CompiledPart& cp, void* state, void* stream) {
  uint64_t tiles = cp.desc.tiles;
  uint64_t grid = tiles;
  if (cp.launch.per_cu > 0)
    grid = std::min<uint64_t>(tiles, (uint64_t)cp.launch.per_cu * k.per_cu * k.cus);
  // keep the launch's thread count within 31 bits; the kernel loops over the rest
  grid = std::max<uint64_t>(1, std::min<uint64_t>(grid, (uint64_t(1) << 31) / (uint64_t)k.block));
  unsigned xcd = 0;
  if (cp.launch.xcd && tiles % 8 == 0 && grid >= 8) {
    grid &= ~uint64_t(7);
    xcd = 1;
  }
  unsigned g = (unsigned)grid;
  void* args[] = {&state, &tiles, &xcd};
  hipError_t e = hipModuleLaunchKernel(k.fn, g, 1, 1, k.block, 1, 1, 0, (hipStream_t)stream,
                                       args, nullptr);
  if (e != hipSuccess) return fail(HS_E_HIP, "hipModuleLaunchKernel: %s", hipGetErrorString(e));
  return HS_OK;
}

}  // namespace hisv
