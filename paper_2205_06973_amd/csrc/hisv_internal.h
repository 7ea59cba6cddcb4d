// hisv_internal.h -- host-side types shared by the library's translation units.
#pragma once

#include <stdint.h>

#include <complex>
#include <exception>
#include <map>
#include <new>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "../../include/hisv.h"
#include "layout.h"

namespace hisv {

using cd = std::complex<double>;

// ---- errors ---------------------------------------------------------------
hs_status fail(hs_status code, const char* fmt, ...);
void clear_error();

// No exception crosses the C boundary or ends a library thread: each entry
// point and each thread body runs inside guarded(), which returns a failed
// allocation as HS_E_NOMEM and any other exception (a thread that could not
// be started, ...) as HS_E_INTERNAL.
template <class F>
hs_status guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(HS_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HS_E_INTERNAL, "%s", e.what());
  } catch (...) {
    return fail(HS_E_INTERNAL, "unexpected exception");
  }
}

// ---- gates (Sec. II.A) ----------------------------------------------------
struct Gate {
  int kind, q0, q1;
  double p[3];
  int arity() const { return q1 < 0 ? 1 : 2; }
  uint64_t mask() const {
    return (uint64_t(1) << q0) | (q1 >= 0 ? (uint64_t(1) << q1) : 0);
  }
};

bool kind_is_1q(int kind);
bool kind_is_2q(int kind);
hs_status validate_gate(int n, const hs_gate& g, Gate* out);
// Validate a gate and append it, or the one- and two-qubit gates that
// replace a three-qubit kind, to *out.
hs_status expand_gate(int n, const hs_gate& g, std::vector<Gate>* out);
// 2x2 matrix (row-major) of a one-qubit gate, in FP64.
void gate_matrix(const Gate& g, cd u[4]);

struct Circuit {
  int n = 0;
  std::vector<Gate> gates;
};

// ---- partitioning (Sec. IV) -------------------------------------------------
struct Dag {
  int G = 0;
  std::vector<std::vector<int>> succ, pred;  // wire dependencies, no duplicates
};
Dag build_dag(const std::vector<Gate>& gates);

// Contiguous cutoff of `order` (a topological order) into parts of at most k
// qubits; part_of_gate is indexed by gate id.  Returns the number of parts.
// `pad` = qubits every part holds anyway (the padding of a multi-level tile):
// a part's qubits together with them must number at most k.
int cutoff_partition(const std::vector<Gate>& gates, const std::vector<int>& order, int k,
                     std::vector<int32_t>* part_of_gate, uint64_t pad = 0);
int partition_nat(const std::vector<Gate>& gates, int k, std::vector<int32_t>* part,
                  uint64_t pad = 0);
int partition_dfs(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t seed,
                  int trials, std::vector<int32_t>* part, uint64_t pad = 0);
int partition_dagp(const std::vector<Gate>& gates, const Dag& dag, int n, int k,
                   uint64_t seed, std::vector<int32_t>* part, uint64_t pad = 0);
int partition_greedy(const std::vector<Gate>& gates, const Dag& dag, int k, uint64_t seed,
                     int trials, std::vector<int32_t>* part, uint64_t pad = 0);
// hs_tune("host_threads"): threads a partition search may use (0 = up to 8,
// as the host has them).
int host_threads();
// hs_tune("serve_chunk"): parts a serving request enqueues at a time.
int serve_chunk_parts();
int partition_closure(const std::vector<Gate>& gates, const Dag& dag, int k, int width,
                      std::vector<int32_t>* part, uint64_t pad = 0);
// Exact validity check; returns "" when valid, else the first violation.
std::string check_partition(const std::vector<Gate>& gates, const Dag& dag,
                            const std::vector<int32_t>& part, int k, uint64_t pad = 0);

// ---- part compilation (kernel descriptors) --------------------------------------
struct HostOp {
  int kind, b0, b1;
  double c[32];  // OP_U2: 4 x 4 complex; the others use the first 8
};

// How a part-pass grid walks the tiles of a part.  Workgroup b of a launch
// runs on XCD b % 8 and each XCD has its own L2; the hardware sustains more
// HBM bandwidth when every XCD sweeps one contiguous run of tiles than when
// consecutive tiles are dealt round-robin over the XCDs.
struct LaunchShape {
  bool xcd = true;        // XCD x takes tiles [x T/8, (x+1) T/8)
  int per_cu = 0;         // 0: one workgroup per tile; g > 0: a persistent grid of
                          // g x (resident workgroups per CU) x CUs
  bool prefetch = false;  // persistent grid: keep the next tile's loads in flight
  // specialized kernels: LDS re-layouts run in 2 or 4 rounds when the tile's
  // LDS image exceeds this many bytes (two workgroups then share a CU)
  size_t lds_limit = 65536;
};

struct CompiledPart {
  PartDesc desc;                    // stage_off relative to this part's stages
  std::vector<StageDesc> stages;    // load, stages..., store (op ranges relative)
  std::vector<HostOp> ops;
  int rb_kernel = 0;
  int lds_round_trips = 0;
  LaunchShape launch;
};

// A part applied as one dense unitary on matrix cores (the fused path):
// U acts on the qubits sq[0..w) (bit b of a row/column index = qubit sq[b]),
// columns of the batched product are the settings of the 4 column qubits.
struct FusedPart {
  int w = 0;                  // 4 or 5
  int m = 0;                  // tile = w + 4 qubits
  uint64_t tiles = 0;         // 2^(n - m)
  int8_t sq[8] = {0};
  int8_t pq[4] = {0};
  int8_t tq[12] = {0};        // sq and pq together, ascending
  std::vector<cd> u;          // 2^w x 2^w, row-major
};
hs_status compile_fused(int n, const std::vector<Gate>& part_gates, FusedPart* out);

struct CompileOptions {
  int rb = 4;        // register bits per lane (2^rb amplitudes per lane)
  int contig = 6;    // tile always holds qubits 0..contig-1 (coalesced runs)
  int max_wb = 4;    // at most 2^max_wb wavefronts per workgroup
  int swizzle = 4;   // LDS swizzle width (bits)
  int max_m = 14;    // widest tile whose 2^m amplitudes fit the LDS
  int min_run = 6;   // load/store straight in a stage layout whose lanes cover
                     // at least qubits 0..min_run-1 (runs of 2^min_run amplitudes)
  int min_tile = 0;  // pad tiles with the lowest free qubits up to this many
                     // (longer contiguous runs per tile); 0 = lanes + registers
  bool fuse2 = false;  // merge two-qubit gates with their one-qubit neighbours
                       // into dense 4 x 4 ops where that saves instructions
  LaunchShape launch;
};

// Compile one part (its gates in circuit order) on an n-qubit state.
hs_status compile_part(int n, const std::vector<Gate>& part_gates, const CompileOptions& opt,
                       CompiledPart* out);
int max_tile_qubits(const CompileOptions& opt);

// ---- plan -------------------------------------------------------------------
struct DevicePlan;  // uploaded descriptors (kernels.hip)
void device_plan_free(DevicePlan* d);
struct SpecKernel;  // a part's specialized kernel (specialize.cpp)

struct Plan {
  int n = 0, k = 0;
  uint64_t pad = 0;  // multi-level plans: qubits counted in every part's bound
  std::vector<Gate> gates;
  Dag dag;
  std::vector<int32_t> part_of_gate;
  std::vector<std::vector<int>> parts;  // gate ids per part, circuit order
  std::vector<uint64_t> masks;
  // per dtype: compiled descriptors + uploaded copy (per device)
  std::mutex mu;
  bool compiled[2] = {false, false};
  std::vector<CompiledPart> comp[2];    // for the interpreter kernel
  bool scompiled[2] = {false, false};
  std::vector<CompiledPart> scomp[2];   // for the specialized kernels
  std::map<int, DevicePlan*> dev[2];
  std::map<int, std::vector<std::shared_ptr<SpecKernel>>> spec[2];  // per device
  // one kernel build at a time per plan (held across the hipRTC build; the
  // maps above are guarded by mu alone, so launches never wait for a build)
  std::mutex spec_build_mu;
  std::vector<std::thread> spec_threads;  // background builds, joined by ~Plan
  hs_status spec_async_rc[2] = {HS_OK, HS_OK};
  std::string spec_async_msg[2];
  bool fused_built = false;
  std::vector<FusedPart> fused;  // w = 0 where a part has no fused form
  ~Plan();
};

hs_status plan_build(int n, const std::vector<Gate>& gates, int k,
                     const std::vector<int32_t>& part_of_gate, Plan* p, uint64_t pad = 0);
CompileOptions default_options(hs_dtype dtype, bool spec = false);
hs_status plan_compile(Plan* p, hs_dtype dtype);
hs_status plan_compile_spec(Plan* p, hs_dtype dtype);
// the compiled parts of a path (PART_SPEC -> specialized, else interpreter)
const std::vector<CompiledPart>& compiled_parts(const Plan* p, hs_dtype dtype, hs_exec exec);

// ---- state --------------------------------------------------------------------
struct State {
  int n = 0;
  hs_dtype dtype = HS_C64;
  void* ptr = nullptr;
  size_t bytes = 0;
  bool owned = false;
  int device = 0;
  void* stream = nullptr;   // hipStream_t
  void* scratch = nullptr;  // device scratch for readout (lazily allocated)
  size_t scratch_bytes = 0;
};

inline size_t amp_bytes(hs_dtype d) { return d == HS_C64 ? 8 : 16; }

// ---- device side (kernels.hip) ------------------------------------------------
hs_status dev_set_basis(State* s, uint64_t x);
hs_status dev_gate_pass(State* s, const Gate& g);
hs_status dev_run_part(State* s, Plan* p, int part);
// Upload the plan's interpreter descriptors for `dtype` on `device` with the
// stream-ordered allocator on `stream`, without waiting for the copies; the
// plan later frees them with hipFreeAsync on that stream, never with a
// device-wide wait.  A launch on another stream first calls
// dev_plan_stream_wait, which makes that stream wait for the copies.
// Pinned host staging for those copies (one per preparing thread): used
// when large enough and `busy` (recorded after its last copies) has passed;
// otherwise the copies go from pageable memory.
struct PinnedStaging {
  void* ptr = nullptr;
  size_t bytes = 0;
  void* busy = nullptr;  // hipEvent_t
};
hs_status dev_plan_upload_async(Plan* p, hs_dtype dtype, int device, void* stream,
                                const PinnedStaging* pin = nullptr);
hs_status dev_plan_stream_wait(Plan* p, hs_dtype dtype, int device, void* stream);
hs_status dev_run_fused(State* s, Plan* p, int part);
hs_status plan_compile_fused(Plan* p);
// hs_tune("fused_shape"): the fused w = 4, 5 kernels' launch shape, read when
// a plan's fused descriptors are uploaded
int fused_launch_shape();
// relative cost (one HBM sweep = 1) of a part on each path, for AUTO
double spec_part_cost(const CompiledPart& cp, hs_dtype dt);
double lds_part_cost(const CompiledPart& cp, hs_dtype dt);
double fused_part_cost(const FusedPart& f, hs_dtype dt);
hs_status dev_norm(State* s, double* out);
// the same reduction with its partial sums in a static device array (no allocation)
hs_status dev_norm_noalloc(State* s, double* out);
hs_status dev_read(State* s, uint64_t first, uint64_t count, double* out, bool probs);
hs_status dev_read_at(State* s, const uint64_t* idx, uint64_t count, double* out);
hs_status dev_copy_probe(const void* src, void* dst, size_t bytes, void* stream);
hs_status dev_sync(State* s);

// ---- specialized part kernels (specialize.cpp) ------------------------------------
// standalone = true: a complete translation unit (the runtime header guard
// included); false: only the part's own declarations, to be wrapped in a
// namespace of a multi-kernel program
std::string specialize_part_source(const CompiledPart& cp, hs_dtype dt, const std::string& name,
                                   bool standalone = true);
hs_status specialize_plan(const std::vector<CompiledPart>& parts, hs_dtype dt, int device,
                          std::vector<std::shared_ptr<SpecKernel>>* out);
hs_status launch_specialized(const SpecKernel& k, const CompiledPart& cp, void* state, void* stream);

}  // namespace hisv
