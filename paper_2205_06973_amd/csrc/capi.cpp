// capi.cpp -- the extern "C" entry points declared in include/hisv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "hisv_internal.h"

namespace hisv {
const char* last_error();
}

using namespace hisv;

struct hs_state_ : State {};
struct hs_circuit_ : Circuit {};
struct hs_plan_ : Plan {};

#define CHECK_ARG(cond, ...) \
  do {                       \
    if (!(cond)) return fail(HS_E_ARG, __VA_ARGS__); \
  } while (0)

namespace hisv {

Plan::~Plan() {
  for (std::thread& t : spec_threads)
    if (t.joinable()) t.join();
  for (int d = 0; d < 2; ++d)
    for (auto& kv : dev[d]) device_plan_free(kv.second);
}

// Tunable knobs (hs_tune), read when a plan is compiled.  Register bits per
// lane: the interpreter kernel keeps the sub-state plus dispatch temporaries
// in at most 128 VGPRs (complex64: 2^4, complex128: 2^3 amplitudes).  The
// specialized kernels hold 2^5 / 2^4: the widest tiles (14 / 13 qubits) then
// take 512 threads, so two workgroups share a CU (1024-thread workgroups of
// the narrower widths measured 15-20% slower per pass); k <= 7 parts run at
// the same rate either way.
static std::mutex g_tune_mu;
static int g_rb[2][2] = {{4, 3}, {5, 4}};     // [specialized][dtype]
static int g_contig = 6;
static int g_min_run[2][2] = {{4, 4}, {3, 3}};  // [specialized][dtype]
// [specialized]: both paths default to one workgroup per tile, XCD-contiguous
static LaunchShape g_launch[2];
static int g_min_tile[2] = {0, 0};             // [specialized]
// Dense 4 x 4 ops: they save the interpreter's per-op dispatch and register
// moves; the specialized kernels have neither, so they keep gate-sized ops.
static bool g_fuse2[2] = {true, false};        // [specialized]
// fused w = 4, 5 launch shape: 0 = one tile group per workgroup, 1 =
// software-pipelined kernel on a persistent grid, 2 = plain kernel on a
// persistent grid, -1 = the measured best per width and precision
static int g_fused_shape = -1;
static int g_host_threads = 0;
static int g_serve_chunk = 8;

int fused_launch_shape() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_fused_shape;
}

int host_threads() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_host_threads;
}

int serve_chunk_parts() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_serve_chunk;
}

CompileOptions default_options(hs_dtype dtype, bool spec) {
  CompileOptions o;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  o.rb = g_rb[spec][dtype];
  o.contig = g_contig;
  o.min_run = g_min_run[spec][dtype];
  o.launch = g_launch[spec];
  o.min_tile = g_min_tile[spec];
  o.fuse2 = g_fuse2[spec];
  if (dtype == HS_C64) {
    o.swizzle = 4;
    o.max_m = 14;  // 2^14 x 8 B = 128 KiB of LDS
  } else {
    o.swizzle = 3;
    o.max_m = 13;  // 2^13 x 16 B = 128 KiB of LDS
  }
  return o;
}

hs_status plan_build(int n, const std::vector<Gate>& gates, int k,
                     const std::vector<int32_t>& part_of_gate, Plan* p, uint64_t pad) {
  p->n = n;
  p->k = k;
  p->pad = pad;
  p->gates = gates;
  p->dag = build_dag(gates);
  p->part_of_gate = part_of_gate;
  const std::string err = check_partition(gates, p->dag, part_of_gate, k, pad);
  if (!err.empty()) return fail(HS_E_BAD_PARTITION, "invalid partition: %s", err.c_str());
  int P = 0;
  for (int32_t v : part_of_gate) P = std::max(P, v + 1);
  p->parts.assign(P, {});
  p->masks.assign(P, 0);
  for (size_t i = 0; i < gates.size(); ++i) {
    p->parts[part_of_gate[i]].push_back((int)i);
    p->masks[part_of_gate[i]] |= gates[i].mask();
  }
  return HS_OK;
}

// Fused forms of every part (w = 0 where a part is wider than the kernel).
hs_status plan_compile_fused(Plan* p) {
  std::lock_guard<std::mutex> lk(p->mu);
  if (p->fused_built) return HS_OK;
  std::vector<FusedPart> fused(p->parts.size());
  std::vector<Gate> pg;
  for (size_t i = 0; i < p->parts.size(); ++i) {
    pg.clear();
    for (int gi : p->parts[i]) pg.push_back(p->gates[gi]);
    if (compile_fused(p->n, pg, &fused[i]) != HS_OK) fused[i] = FusedPart{};
  }
  clear_error();
  p->fused.swap(fused);
  p->fused_built = true;
  return HS_OK;
}

static hs_status compile_all(Plan* p, const CompileOptions& opt, std::vector<CompiledPart>* out) {
  std::vector<CompiledPart> comp(p->parts.size());
  std::vector<Gate> pg;
  for (size_t i = 0; i < p->parts.size(); ++i) {
    pg.clear();
    for (int gi : p->parts[i]) pg.push_back(p->gates[gi]);
    if (hs_status rc = compile_part(p->n, pg, opt, &comp[i])) return rc;
    comp[i].launch = opt.launch;
  }
  out->swap(comp);
  return HS_OK;
}

hs_status plan_compile(Plan* p, hs_dtype dtype) {
  std::lock_guard<std::mutex> lk(p->mu);
  if (p->compiled[dtype]) return HS_OK;
  if (hs_status rc = compile_all(p, default_options(dtype, false), &p->comp[dtype])) return rc;
  p->compiled[dtype] = true;
  return HS_OK;
}

hs_status plan_compile_spec(Plan* p, hs_dtype dtype) {
  std::lock_guard<std::mutex> lk(p->mu);
  if (p->scompiled[dtype]) return HS_OK;
  if (hs_status rc = compile_all(p, default_options(dtype, true), &p->scomp[dtype])) return rc;
  p->scompiled[dtype] = true;
  return HS_OK;
}

const std::vector<CompiledPart>& compiled_parts(const Plan* p, hs_dtype dtype, hs_exec exec) {
  return exec == HS_EXEC_PART_SPEC ? p->scomp[dtype] : p->comp[dtype];
}

}  // namespace hisv

extern "C" {

const char* hs_version(void) { return "hisv 0.1 (gfx950)"; }

const char* hs_last_error(void) { return hisv::last_error(); }

hs_status hs_device_count(int* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(out, "null output");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) n = 0;
    *out = n;
    return HS_OK;
  });
}

hs_status hs_tune(const char* key, int value) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(key, "null key");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::string k(key);
    int spec = 0;
    if (k.rfind("spec_", 0) == 0) {
      spec = 1;
      k = k.substr(5);
    }
    if (k == "rb_c64" || k == "rb_c128") {
      // the interpreter kernel (<= 1024 threads, 128 VGPRs a lane) spills beyond
      // 2^4 complex64 / 2^3 complex128 amplitudes a lane
      const int hi = spec ? 5 : (k == "rb_c64" ? 4 : 3);
      CHECK_ARG(value >= 1 && value <= hi, "register bits must be 1..%d", hi);
      g_rb[spec][k == "rb_c64" ? 0 : 1] = value;
    } else if (k == "contig" && !spec) {
      CHECK_ARG(value >= 0 && value <= 8, "contig must be 0..8");
      g_contig = value;
    } else if (k == "min_run_c64" || k == "min_run_c128") {
      CHECK_ARG(value >= 0 && value <= 6, "min_run must be 0..6");
      g_min_run[spec][k == "min_run_c64" ? 0 : 1] = value;
    } else if (k == "xcd" || (k == "prefetch" && spec)) {
      CHECK_ARG(value == 0 || value == 1, "%s must be 0 or 1", k.c_str());
      (k == "xcd" ? g_launch[spec].xcd : g_launch[spec].prefetch) = value != 0;
    } else if (k == "fuse2") {
      CHECK_ARG(value == 0 || value == 1, "fuse2 must be 0 or 1");
      g_fuse2[spec] = value != 0;
    } else if (k == "fused_shape" && !spec) {
      CHECK_ARG(value >= -1 && value <= 2, "fused_shape must be -1, 0, 1 or 2");
      g_fused_shape = value;
    } else if (k == "serve_chunk" && !spec) {
      CHECK_ARG(value >= 1 && value <= 4096, "serve_chunk must be 1..4096");
      g_serve_chunk = value;
    } else if (k == "host_threads" && !spec) {
      CHECK_ARG(value >= 0 && value <= 64, "host_threads must be 0..64");
      g_host_threads = value;
    } else if (k == "min_tile") {
      CHECK_ARG(value >= 0 && value <= 16, "min_tile must be 0..16");
      g_min_tile[spec] = value;
    } else if (k == "lds_limit_kib" && spec) {
      CHECK_ARG(value >= 16 && value <= 160, "lds_limit_kib must be 16..160");
      g_launch[spec].lds_limit = (size_t)value * 1024;
    } else if (k == "grid") {
      CHECK_ARG(value >= 0 && value <= 64, "grid must be 0 (one workgroup per tile) or 1..64");
      g_launch[spec].per_cu = value;
    } else {
      return fail(HS_E_ARG, "unknown tuning key '%s'", key);
    }
    return HS_OK;
  });
}

static hs_status check_exec(hs_exec exec);

hs_status hs_max_part_qubits(hs_dtype dtype, hs_exec exec, int* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(out, "null output");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype %d", (int)dtype);
    if (hs_status rc = check_exec(exec)) return rc;
    if (exec == HS_EXEC_GATE_PER_PASS) {
      *out = 64;
    } else if (exec == HS_EXEC_PART_FUSED) {
      *out = kMaxFusedQubits;
    } else {
      const CompileOptions o = default_options(dtype, exec == HS_EXEC_PART_SPEC);
      *out = max_tile_qubits(o) - o.contig;
    }
    return HS_OK;
  });
}

// ---- states ------------------------------------------------------------------

static hs_status new_state(int n, hs_dtype dtype, void* stream, hs_state* out) {
  CHECK_ARG(out, "null output");
  CHECK_ARG(n >= 1 && n <= 40, "n = %d outside [1, 40]", n);
  CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype %d", (int)dtype);
  auto* s = new hs_state_();
  s->n = n;
  s->dtype = dtype;
  s->bytes = (size_t(1) << n) * amp_bytes(dtype);
  s->stream = stream;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(HS_E_HIP, "no HIP device");
  }
  *out = s;
  return HS_OK;
}

hs_status hs_state_create(int n, hs_dtype dtype, void* hip_stream, hs_state* out) {
  return guarded([&]() -> hs_status {
    hs_state s = nullptr;
    if (hs_status rc = new_state(n, dtype, hip_stream, &s)) return rc;
    hipError_t e = hipMalloc(&s->ptr, s->bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // clear the sticky error of the failed allocation
      delete s;
      return fail(HS_E_NOMEM, "hipMalloc(%zu): %s", (size_t(1) << n) * amp_bytes(dtype),
                  hipGetErrorString(e));
    }
    s->owned = true;
    *out = s;
    return HS_OK;
  });
}

hs_status hs_state_wrap(int n, hs_dtype dtype, void* dev_ptr, size_t bytes, void* hip_stream,
                        hs_state* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(dev_ptr, "null device pointer");
    CHECK_ARG(n >= 1 && n <= 40, "n = %d outside [1, 40]", n);
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype %d", (int)dtype);
    CHECK_ARG(bytes == (size_t(1) << n) * amp_bytes(dtype), "buffer of %zu bytes is not 2^%d amplitudes",
              bytes, n);
    CHECK_ARG(((uintptr_t)dev_ptr % amp_bytes(dtype)) == 0, "device pointer not aligned to an amplitude");
    hs_state s = nullptr;
    if (hs_status rc = new_state(n, dtype, hip_stream, &s)) return rc;
    s->ptr = dev_ptr;
    s->owned = false;
    *out = s;
    return HS_OK;
  });
}

hs_status hs_state_set_basis(hs_state s, uint64_t x) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s, "null state");
    CHECK_ARG(x < (uint64_t(1) << s->n), "basis index outside the state");
    return dev_set_basis(s, x);
  });
}

hs_status hs_state_info(hs_state s, int* n, hs_dtype* dtype, void** dev_ptr) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s, "null state");
    if (n) *n = s->n;
    if (dtype) *dtype = s->dtype;
    if (dev_ptr) *dev_ptr = s->ptr;
    return HS_OK;
  });
}

hs_status hs_state_destroy(hs_state s) {
  return guarded([&]() -> hs_status {
    if (!s) return HS_OK;
    // release everything even if the device reports an error; report the
    // first one (a failed wait means work on the state did not complete)
    hipError_t e = hipSetDevice(s->device);
    const hipError_t w = s->stream ? hipStreamSynchronize((hipStream_t)s->stream) : hipDeviceSynchronize();
    if (e == hipSuccess) e = w;
    if (s->owned && s->ptr) {
      const hipError_t f = hipFree(s->ptr);
      if (e == hipSuccess) e = f;
    }
    if (s->scratch) {
      const hipError_t f = hipFree(s->scratch);
      if (e == hipSuccess) e = f;
    }
    delete s;
    if (e != hipSuccess) return fail(HS_E_HIP, "state teardown: %s", hipGetErrorString(e));
    return HS_OK;
  });
}

// ---- circuits ----------------------------------------------------------------

hs_status hs_circuit_load(int n, const hs_gate* gates, size_t count, hs_circuit* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(out, "null output");
    CHECK_ARG(n >= 1 && n <= 40, "n = %d outside [1, 40]", n);
    CHECK_ARG(gates || count == 0, "null gate array");
    auto c = std::make_unique<hs_circuit_>();
    c->n = n;
    c->gates.reserve(count);
    for (size_t i = 0; i < count; ++i)
      if (hs_status rc = expand_gate(n, gates[i], &c->gates)) return rc;
    *out = c.release();
    return HS_OK;
  });
}

hs_status hs_circuit_info(hs_circuit c, int* n, size_t* count) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(c, "null circuit");
    if (n) *n = c->n;
    if (count) *count = c->gates.size();
    return HS_OK;
  });
}

hs_status hs_circuit_destroy(hs_circuit c) {
  return guarded([&]() -> hs_status {
    delete c;
    return HS_OK;
  });
}

// ---- plans -------------------------------------------------------------------

// CLOSURE keeps up to `trials` partial partitions and their expansions: a
// bound on the beam keeps a mistyped width from reserving gigabytes.
constexpr int kMaxBeam = 65536;

hs_status hs_partition(hs_circuit c, int k, hs_strategy strategy, uint64_t seed, int trials,
                       hs_plan* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(c && out, "null argument");
    CHECK_ARG(k >= 1, "k = %d < 1", k);
    for (const Gate& g : c->gates)
      if (g.arity() > k) return fail(HS_E_ARITY_GT_K, "a %d-qubit gate does not fit k = %d", g.arity(), k);
    std::vector<int32_t> part;
    const Dag dag = build_dag(c->gates);
    switch (strategy) {
      case HS_PART_NAT: partition_nat(c->gates, k, &part); break;
      case HS_PART_DFS:
        CHECK_ARG(trials >= 1, "DFS needs trials >= 1");
        partition_dfs(c->gates, dag, k, seed, trials, &part);
        break;
      case HS_PART_DAGP: partition_dagp(c->gates, dag, c->n, k, seed, &part); break;
      case HS_PART_GREEDY:
        CHECK_ARG(trials >= 1, "GREEDY needs trials >= 1");
        partition_greedy(c->gates, dag, k, seed, trials, &part);
        break;
      case HS_PART_CLOSURE:
        CHECK_ARG(trials >= 1 && trials <= kMaxBeam, "CLOSURE beam width %d outside [1, %d]", trials,
                  kMaxBeam);
        partition_closure(c->gates, dag, k, trials, &part);
        break;
      default: return fail(HS_E_ARG, "unknown strategy %d", (int)strategy);
    }
    auto p = std::make_unique<hs_plan_>();
    if (hs_status rc = plan_build(c->n, c->gates, k, part, p.get())) return rc;
    *out = p.release();
    return HS_OK;
  });
}

// Multi-level: level 1 bounds each part together with the padding qubits
// 0..pad_qubits-1 by the tile; level 2 (register stages) is the compile step.
hs_status hs_partition_multilevel(hs_circuit c, int tile_qubits, int pad_qubits,
                                  hs_strategy strategy, uint64_t seed, int trials, hs_plan* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(c && out, "null argument");
    CHECK_ARG(pad_qubits >= 0 && pad_qubits <= 64, "pad_qubits = %d outside [0, 64]", pad_qubits);
    const int np = std::min(pad_qubits, c->n);
    const uint64_t pad = np >= 64 ? ~uint64_t(0) : (uint64_t(1) << np) - 1;
    CHECK_ARG(tile_qubits >= 1, "tile_qubits = %d < 1", tile_qubits);
    for (const Gate& g : c->gates)
      if (__builtin_popcountll(g.mask() | pad) > tile_qubits)
        return fail(HS_E_ARITY_GT_K, "a gate and the %d padding qubits do not fit %d tile qubits", np,
                    tile_qubits);
    std::vector<int32_t> part;
    const Dag dag = build_dag(c->gates);
    switch (strategy) {
      case HS_PART_NAT: partition_nat(c->gates, tile_qubits, &part, pad); break;
      case HS_PART_DFS:
        CHECK_ARG(trials >= 1, "DFS needs trials >= 1");
        partition_dfs(c->gates, dag, tile_qubits, seed, trials, &part, pad);
        break;
      case HS_PART_DAGP: partition_dagp(c->gates, dag, c->n, tile_qubits, seed, &part, pad); break;
      case HS_PART_GREEDY:
        CHECK_ARG(trials >= 1, "GREEDY needs trials >= 1");
        partition_greedy(c->gates, dag, tile_qubits, seed, trials, &part, pad);
        break;
      case HS_PART_CLOSURE:
        CHECK_ARG(trials >= 1 && trials <= kMaxBeam, "CLOSURE beam width %d outside [1, %d]", trials,
                  kMaxBeam);
        partition_closure(c->gates, dag, tile_qubits, trials, &part, pad);
        break;
      default: return fail(HS_E_ARG, "unknown strategy %d", (int)strategy);
    }
    auto p = std::make_unique<hs_plan_>();
    if (hs_status rc = plan_build(c->n, c->gates, tile_qubits, part, p.get(), pad)) return rc;
    *out = p.release();
    return HS_OK;
  });
}

hs_status hs_plan_from_assignment(hs_circuit c, int k, const int32_t* part_of_gate, size_t count,
                                  hs_plan* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(c && out, "null argument");
    CHECK_ARG(part_of_gate || c->gates.empty(), "null assignment");
    CHECK_ARG(count == c->gates.size(), "assignment has %zu entries, the circuit %zu gates", count,
              c->gates.size());
    CHECK_ARG(k >= 1, "k = %d < 1", k);
    std::vector<int32_t> part(part_of_gate, part_of_gate + c->gates.size());
    auto p = std::make_unique<hs_plan_>();
    if (hs_status rc = plan_build(c->n, c->gates, k, part, p.get())) return rc;
    *out = p.release();
    return HS_OK;
  });
}

hs_status hs_plan_num_parts(hs_plan p, int* parts) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p && parts, "null argument");
    *parts = (int)p->parts.size();
    return HS_OK;
  });
}

hs_status hs_plan_part_of_gate(hs_plan p, int32_t* out, size_t cap, size_t* count) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    if (count) *count = p->part_of_gate.size();
    if (!out) return HS_OK;
    CHECK_ARG(cap >= p->part_of_gate.size(), "buffer of %zu entries for %zu gates", cap,
              p->part_of_gate.size());
    std::copy(p->part_of_gate.begin(), p->part_of_gate.end(), out);
    return HS_OK;
  });
}

hs_status hs_plan_part_info(hs_plan p, int part, uint64_t* qubit_mask, int* num_gates) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    CHECK_ARG(part >= 0 && part < (int)p->parts.size(), "part %d out of range", part);
    if (qubit_mask) *qubit_mask = p->masks[part];
    if (num_gates) *num_gates = (int)p->parts[part].size();
    return HS_OK;
  });
}

hs_status hs_plan_validate(hs_plan p) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    const std::string err = check_partition(p->gates, p->dag, p->part_of_gate, p->k, p->pad);
    if (!err.empty()) return fail(HS_E_BAD_PARTITION, "invalid partition: %s", err.c_str());
    return HS_OK;
  });
}

static hs_status compile_for(Plan* p, hs_dtype dtype, hs_exec exec) {
  return exec == HS_EXEC_PART_SPEC ? plan_compile_spec(p, dtype) : plan_compile(p, dtype);
}

hs_status hs_plan_part_layout(hs_plan p, int part, hs_dtype dtype, hs_exec exec, int* tile_qubits,
                              int* stages, int* lds_round_trips) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    CHECK_ARG(part >= 0 && part < (int)p->parts.size(), "part %d out of range", part);
    if (hs_status rc = compile_for(p, dtype, exec)) return rc;
    const CompiledPart& cp = compiled_parts(p, dtype, exec)[part];
    if (tile_qubits) *tile_qubits = cp.desc.m;
    if (stages) *stages = cp.desc.n_stages - 2;
    if (lds_round_trips) *lds_round_trips = cp.lds_round_trips;
    return HS_OK;
  });
}

hs_status hs_plan_part_descriptors(hs_plan p, int part, hs_dtype dtype, hs_exec exec, int32_t* header,
                                   int32_t* entries, int entries_cap, double* ops, int ops_cap) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p && header, "null argument");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    CHECK_ARG(part >= 0 && part < (int)p->parts.size(), "part %d out of range", part);
    if (hs_status rc = compile_for(p, dtype, exec)) return rc;
    const CompiledPart& cp = compiled_parts(p, dtype, exec)[part];
    const PartDesc& d = cp.desc;
    header[0] = d.m;
    header[1] = d.lb;
    header[2] = d.wb;
    header[3] = d.rb;
    header[4] = d.n_stages;
    header[5] = cp.lds_round_trips;
    header[6] = (int)cp.ops.size();
    header[7] = p->n - d.m;
    for (int i = 0; i < kMaxTile; ++i) header[8 + i] = d.tq[i];
    if (entries && entries_cap >= d.n_stages) {
      for (int s = 0; s < d.n_stages; ++s) {
        const StageDesc& e = cp.stages[s];
        int32_t* o = entries + 20 * s;
        for (int i = 0; i < kMaxTile; ++i) o[i] = e.pos[i];
        o[16] = e.op_begin;
        o[17] = e.op_end;
        o[18] = e.transition;
        o[19] = 0;
      }
    }
    if (ops && ops_cap >= (int)cp.ops.size()) {
      for (size_t i = 0; i < cp.ops.size(); ++i) {
        double* o = ops + 35 * i;
        o[0] = cp.ops[i].kind;
        o[1] = cp.ops[i].b0;
        o[2] = cp.ops[i].b1;
        for (int j = 0; j < 32; ++j) o[3 + j] = cp.ops[i].c[j];
      }
    }
    return HS_OK;
  });
}

// The plan's specialized kernels for `dtype` on `device`, built if need be.
// The build runs under the plan's build lock only, so the interpreter and
// AUTO keep launching parts (they take p->mu briefly) while hipRTC works.
static hs_status ensure_spec(Plan* p, hs_dtype dtype, int device,
                             std::vector<std::shared_ptr<SpecKernel>>** out) {
  if (hs_status rc = plan_compile_spec(p, dtype)) return rc;
  std::lock_guard<std::mutex> build(p->spec_build_mu);
  {
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->spec[dtype].find(device);
    if (it != p->spec[dtype].end()) {
      *out = &it->second;
      return HS_OK;
    }
  }
  // scomp[dtype] no longer changes once compiled
  std::vector<std::shared_ptr<SpecKernel>> ks;
  if (hs_status rc = specialize_plan(p->scomp[dtype], dtype, device, &ks)) return rc;
  std::lock_guard<std::mutex> lk(p->mu);
  *out = &p->spec[dtype].emplace(device, std::move(ks)).first->second;
  return HS_OK;
}

hs_status hs_plan_part_source(hs_plan p, int part, hs_dtype dtype, char* buf, size_t cap, size_t* len) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    CHECK_ARG(part >= 0 && part < (int)p->parts.size(), "part %d out of range", part);
    if (hs_status rc = plan_compile_spec(p, dtype)) return rc;
    const std::string src = specialize_part_source(p->scomp[dtype][part], dtype, "part_pass_spec");
    if (len) *len = src.size();
    if (!buf) return HS_OK;
    CHECK_ARG(cap > src.size(), "buffer of %zu bytes is too small", cap);
    std::memcpy(buf, src.c_str(), src.size() + 1);
    return HS_OK;
  });
}

hs_status hs_plan_specialize(hs_plan p, hs_dtype dtype) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(HS_E_HIP, "no HIP device");
    std::vector<std::shared_ptr<SpecKernel>>* ks = nullptr;
    return ensure_spec(p, dtype, dev, &ks);
  });
}

hs_status hs_plan_specialize_async(hs_plan p, hs_dtype dtype) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(HS_E_HIP, "no HIP device");
    // the descriptors first, on the caller's thread (host work, milliseconds),
    // so that a compile error is reported here
    if (hs_status rc = plan_compile_spec(p, dtype)) return rc;
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->spec[dtype].count(dev)) return HS_OK;
    p->spec_async_rc[dtype] = HS_OK;
    p->spec_async_msg[dtype].clear();
    Plan* plan = p;
    p->spec_threads.emplace_back([plan, dtype, dev]() {
      std::vector<std::shared_ptr<SpecKernel>>* ks = nullptr;
      hs_status rc = guarded([&] {
        return hipSetDevice(dev) == hipSuccess ? ensure_spec(plan, dtype, dev, &ks)
                                               : fail(HS_E_HIP, "hipSetDevice failed");
      });
      if (rc != HS_OK) {
        std::lock_guard<std::mutex> g(plan->mu);
        plan->spec_async_rc[dtype] = rc;
        guarded([&] {  // the message, if there is memory for it
          plan->spec_async_msg[dtype] = hs_last_error();
          return HS_OK;
        });
      }
    });
    return HS_OK;
  });
}

hs_status hs_plan_specialize_wait(hs_plan p, hs_dtype dtype) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p, "null plan");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    // join the background builds started so far (each joined by one caller)
    std::vector<std::thread> ts;
    {
      std::lock_guard<std::mutex> lk(p->mu);
      ts.swap(p->spec_threads);
    }
    for (std::thread& t : ts) t.join();
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->spec_async_rc[dtype] != HS_OK)
      return fail(p->spec_async_rc[dtype], "background build failed: %s", p->spec_async_msg[dtype].c_str());
    return HS_OK;
  });
}

hs_status hs_plan_specialized(hs_plan p, hs_dtype dtype, int* ready) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p && ready, "null argument");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(HS_E_HIP, "no HIP device");
    std::lock_guard<std::mutex> lk(p->mu);
    *ready = p->spec[dtype].count(dev) ? 1 : 0;
    return HS_OK;
  });
}

static hs_status run_spec_parts(hs_state s, Plan* p, int first, int last) {
  std::vector<std::shared_ptr<SpecKernel>>* ks = nullptr;
  if (hipSetDevice(s->device) != hipSuccess) return fail(HS_E_HIP, "hipSetDevice failed");
  if (hs_status rc = ensure_spec(p, s->dtype, s->device, &ks)) return rc;
  for (int i = first; i < last; ++i)
    if (hs_status rc = launch_specialized(*(*ks)[i], p->scomp[s->dtype][i], s->ptr, s->stream))
      return rc;
  return HS_OK;
}

hs_status hs_plan_destroy(hs_plan p) {
  return guarded([&]() -> hs_status {
    delete p;
    return HS_OK;
  });
}

// ---- simulation --------------------------------------------------------------

static hs_status check_exec(hs_exec exec) {
  if (exec == HS_EXEC_GATE_PER_PASS || exec == HS_EXEC_PART_LDS || exec == HS_EXEC_AUTO ||
      exec == HS_EXEC_PART_SPEC || exec == HS_EXEC_PART_FUSED)
    return HS_OK;
  return fail(HS_E_ARG, "unknown exec mode %d", (int)exec);
}

// Parts [first, last) on the interpreter LDS kernel, the fused kernel, or
// (AUTO) whichever the cost model prefers per part.  AUTO's gate-by-gate side
// is the specialized kernels when hs_plan_specialize has built them for this
// dtype and device (no hipRTC work starts here), else the interpreter.
// AUTO's choice for part i: the fused kernel when the part has a fused form
// and its cost (in HBM sweeps) is below the gate-by-gate kernel's -- the
// specialized kernel's when the plan is specialized, else the interpreter's.
static bool auto_picks_fused(Plan* p, hs_dtype dt, int i, bool specialized) {
  const double gate_cost = specialized ? spec_part_cost(p->scomp[dt][i], dt) : lds_part_cost(p->comp[dt][i], dt);
  return p->fused[i].w && fused_part_cost(p->fused[i], dt) < gate_cost;
}

static hs_status run_parts(hs_state s, Plan* p, int first, int last, hs_exec exec) {
  if (hs_status rc = plan_compile(p, s->dtype)) return rc;
  if (exec != HS_EXEC_PART_LDS)
    if (hs_status rc = plan_compile_fused(p)) return rc;
  std::vector<std::shared_ptr<SpecKernel>>* ks = nullptr;
  if (exec == HS_EXEC_AUTO) {
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->spec[s->dtype].find(s->device);
    if (it != p->spec[s->dtype].end()) ks = &it->second;
  }
  for (int i = first; i < last; ++i) {
    bool fused = false;
    if (exec == HS_EXEC_PART_FUSED) {
      if (!p->fused[i].w)
        return fail(HS_E_UNSUPPORTED, "part %d uses more than %d qubits: no fused form", i,
                    kMaxFusedQubits);
      fused = true;
    } else if (exec == HS_EXEC_AUTO) {
      fused = auto_picks_fused(p, s->dtype, i, ks != nullptr);
    }
    hs_status rc;
    if (fused) {
      rc = dev_run_fused(s, p, i);
    } else if (ks) {
      if (hipSetDevice(s->device) != hipSuccess) return fail(HS_E_HIP, "hipSetDevice failed");
      rc = launch_specialized(*(*ks)[i], p->scomp[s->dtype][i], s->ptr, s->stream);
    } else {
      rc = dev_run_part(s, p, i);
    }
    if (rc) return rc;
  }
  return HS_OK;
}

hs_status hs_simulate_part(hs_state s, hs_plan p, int part, hs_exec exec) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && p, "null argument");
    CHECK_ARG(p->n == s->n, "plan is for %d qubits, state has %d", p->n, s->n);
    CHECK_ARG(part >= 0 && part < (int)p->parts.size(), "part %d out of range", part);
    if (hs_status rc = check_exec(exec)) return rc;
    if (exec == HS_EXEC_GATE_PER_PASS) {
      for (int gi : p->parts[part])
        if (hs_status rc = dev_gate_pass(s, p->gates[gi])) return rc;
      return HS_OK;
    }
    if (exec == HS_EXEC_PART_SPEC) return run_spec_parts(s, p, part, part + 1);
    return run_parts(s, p, part, part + 1, exec);
  });
}

hs_status hs_plan_auto_choice(hs_plan p, hs_dtype dtype, int32_t* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p && out, "null argument");
    CHECK_ARG(dtype == HS_C64 || dtype == HS_C128, "bad dtype");
    if (hs_status rc = plan_compile(p, dtype)) return rc;
    if (hs_status rc = plan_compile_fused(p)) return rc;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) device = -1;
    bool specialized = false;
    {
      std::lock_guard<std::mutex> lk(p->mu);
      specialized = p->spec[dtype].count(device) > 0;
    }
    for (int i = 0; i < (int)p->parts.size(); ++i) out[i] = auto_picks_fused(p, dtype, i, specialized) ? 1 : 0;
    return HS_OK;
  });
}

hs_status hs_simulate(hs_state s, hs_plan p, hs_exec exec) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && p, "null argument");
    CHECK_ARG(p->n == s->n, "plan is for %d qubits, state has %d", p->n, s->n);
    if (hs_status rc = check_exec(exec)) return rc;
    if (exec == HS_EXEC_GATE_PER_PASS) {
      for (const Gate& g : p->gates)
        if (hs_status rc = dev_gate_pass(s, g)) return rc;
      return HS_OK;
    }
    if (exec == HS_EXEC_PART_SPEC) return run_spec_parts(s, p, 0, (int)p->parts.size());
    return run_parts(s, p, 0, (int)p->parts.size(), exec);
  });
}

hs_status hs_plan_part_unitary(hs_plan p, int part, int* w, double* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(p && w, "null argument");
    CHECK_ARG(part >= 0 && part < (int)p->parts.size(), "part %d out of range", part);
    if (hs_status rc = plan_compile_fused(p)) return rc;
    const FusedPart& f = p->fused[part];
    *w = f.w;
    if (!f.w) return fail(HS_E_UNSUPPORTED, "part %d has no fused form", part);
    if (out) {
      for (int b = 0; b < f.w; ++b) out[b] = f.sq[b];
      double* u = out + f.w;
      for (size_t i = 0; i < f.u.size(); ++i) {
        u[2 * i] = f.u[i].real();
        u[2 * i + 1] = f.u[i].imag();
      }
    }
    return HS_OK;
  });
}

hs_status hs_simulate_gate_per_pass(hs_state s, hs_circuit c) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && c, "null argument");
    CHECK_ARG(c->n == s->n, "circuit is for %d qubits, state has %d", c->n, s->n);
    for (const Gate& g : c->gates)
      if (hs_status rc = dev_gate_pass(s, g)) return rc;
    return HS_OK;
  });
}

// ---- readout -----------------------------------------------------------------

hs_status hs_read_amplitudes(hs_state s, uint64_t first, uint64_t count, double* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && (out || count == 0), "null argument");
    const uint64_t N = uint64_t(1) << s->n;
    CHECK_ARG(first <= N && count <= N - first, "range outside the state");
    if (!count) return HS_OK;
    return dev_read(s, first, count, out, false);
  });
}

hs_status hs_read_amplitudes_at(hs_state s, const uint64_t* idx, uint64_t count, double* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && ((idx && out) || count == 0), "null argument");
    const uint64_t N = uint64_t(1) << s->n;
    for (uint64_t i = 0; i < count; ++i)
      CHECK_ARG(idx[i] < N, "index %llu outside the state", (unsigned long long)idx[i]);
    if (!count) return HS_OK;
    return dev_read_at(s, idx, count, out);
  });
}

hs_status hs_probabilities(hs_state s, uint64_t first, uint64_t count, double* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && (out || count == 0), "null argument");
    const uint64_t N = uint64_t(1) << s->n;
    CHECK_ARG(first <= N && count <= N - first, "range outside the state");
    if (!count) return HS_OK;
    return dev_read(s, first, count, out, true);
  });
}

hs_status hs_norm(hs_state s, double* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && out, "null argument");
    return dev_norm(s, out);
  });
}

hs_status hs_norm_noalloc(hs_state s, double* out) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s && out, "null argument");
    CHECK_ARG(s->ptr, "state has no device memory");
    return dev_norm_noalloc(s, out);
  });
}

hs_status hs_sync(hs_state s) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(s, "null state");
    return dev_sync(s);
  });
}

hs_status hs_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream) {
  return guarded([&]() -> hs_status {
    CHECK_ARG(src && dst, "null pointer");
    CHECK_ARG(bytes % 16 == 0, "bytes must be a multiple of 16");
    return dev_copy_probe(src, dst, bytes, hip_stream);
  });
}

}  // extern "C"
