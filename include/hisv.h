/*
 * hisv.h -- C ABI of the partitioned state-vector library (libhisv.so).
 *
 * Method: Fang et al., "Efficient Hierarchical State Vector Simulation of
 * Quantum Circuits via Acyclic Graph Partitioning" (arXiv 2205.06973).
 *
 *   - Sec. II.B: given an initial n-qubit state (2^n complex amplitudes) and
 *     a sequence of gates, apply every gate in order.
 *   - Sec. IV.A: the circuit is a DAG of gates; an acyclic partition splits it
 *     into parts whose working set (distinct qubits) is at most L_m (called k
 *     here), with an acyclic part-graph; the output is a part id per gate and
 *     the gates of a part keep circuit order.
 *   - Alg. 1 (Sec. III.C): each part is applied to the whole state by
 *     Gather-Execute-Scatter: for every setting of the qubits outside the
 *     part, the 2^w amplitudes addressed by the part's qubits are gathered,
 *     the part's gates run on them, and they are scattered back -- one sweep
 *     of the state per part instead of one per gate.
 *
 * Conventions (all entry points)
 *   - State layout: 2^n interleaved complex numbers (re, im) in device memory,
 *     complex64 (2 x float) or complex128 (2 x double); amplitude index bit q
 *     is the value of qubit q (little-endian, Fig. 1 caption; a one-qubit gate
 *     on qubit i pairs amplitudes 2^i apart, Sec. III.A).
 *   - Every call returns an hs_status; nothing throws across the ABI.  On a
 *     non-OK status, hs_last_error() returns a message for the calling thread.
 *   - Handles are opaque and owned by the library; each has a *_destroy.
 *     Host arrays passed in are copied; host output buffers belong to the
 *     caller.  Device memory passed to hs_state_wrap stays the caller's.
 *   - Work on a state is enqueued, in order, on the HIP stream given when the
 *     state was made (NULL = the device's null stream).  Calls documented as
 *     "syncs" wait for that stream before returning.
 *   - Handles may be used from several threads, but calls on one state or
 *     one plan must not overlap.
 */
#ifndef HISV_H
#define HISV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HS_OK = 0,
  HS_E_ARG = 1,            /* a null handle/pointer, bad size, bad enum, mismatched n */
  HS_E_QUBIT_RANGE = 2,    /* a gate qubit outside [0, n), or both qubits equal      */
  HS_E_ARITY_GT_K = 3,     /* a gate uses more qubits than the part limit k           */
  HS_E_NOMEM = 4,          /* host or device allocation failed                        */
  HS_E_ADMISSION = 5,      /* serving: request can never fit the byte budget          */
  HS_E_HIP = 6,            /* a HIP runtime call failed (message has the HIP error)   */
  HS_E_BAD_PARTITION = 7,  /* a plan failed exact validation                          */
  HS_E_STATE = 8,          /* wrong object state (e.g. reading an unfinished ticket)  */
  HS_E_UNSUPPORTED = 9,    /* a valid request this build does not handle (e.g. a part
                              wider than the largest kernel tile)                     */
  HS_E_INTERNAL = 10       /* an unexpected host-side failure (e.g. a host thread could
                              not be started); the message names it                   */
} hs_status;

typedef enum { HS_C64 = 0, HS_C128 = 1 } hs_dtype;

/* Gate kinds.  X, Y, Z, H are the matrices of Sec. II.A; the others use the
 * OpenQASM-2 definitions: S = diag(1, i), T = diag(1, e^{i pi/4}),
 * RX(t) = [[c, -i s], [-i s, c]], RY(t) = [[c, -s], [s, c]] (c = cos t/2,
 * s = sin t/2), RZ(t) = diag(e^{-it/2}, e^{it/2}), P(l) = diag(1, e^{il}),
 * U3(t, f, l) = [[c, -e^{il} s], [e^{if} s, e^{i(f+l)} c]];
 * CX(q0 = control, q1 = target); CZ, CP(l) multiply amplitudes with both
 * qubits set by -1 and e^{il}; SWAP exchanges the two qubits.
 * Three-qubit kinds (Sec. III.A footnote: gates on more qubits are
 * decomposed): CCX (Toffoli; controls q0, q1, target q2) and CSWAP
 * (Fredkin; control q0 exchanges q1 and q2).  hs_circuit_load replaces each
 * with one- and two-qubit gates -- CCX by H, T, T^dagger and six CX (the
 * standard exact decomposition, no global phase), CSWAP by CX(q2, q1) CCX
 * CX(q2, q1) -- so partitions and kernels only ever see arity <= 2. */
typedef enum {
  HS_H = 0, HS_X = 1, HS_Y = 2, HS_Z = 3, HS_S = 4, HS_T = 5,
  HS_RX = 6, HS_RY = 7, HS_RZ = 8, HS_P = 9, HS_U3 = 10,
  HS_CX = 11, HS_CZ = 12, HS_CP = 13, HS_SWAP = 14,
  HS_CCX = 15, HS_CSWAP = 16
} hs_kind;

/* One gate: q1 = -1 for one-qubit kinds; q2 = the third qubit of the
 * three-qubit kinds and 0 for all others; p[] holds the angles (unused ones
 * ignored).  40 bytes, naturally aligned. */
typedef struct {
  int32_t kind;
  int32_t q0;
  int32_t q1;
  int32_t q2;
  double p[3];
} hs_gate;

/* Sec. IV.B: natural topological-order cutoff (Nat), the same cutoff over
 * seeded random DFS topological orders keeping the fewest parts (DFS), and an
 * acyclic recursive-bisection partitioner with a final merge phase (DAGP).
 * GREEDY (not in the paper): each part grows by the ready gate that fits and
 * adds the fewest new qubits, closing when none fits; trial 0 breaks ties by
 * gate index, the other trials by seeded random keys; fewest parts win.
 * Its parts are contiguous pieces of a topological order, hence acyclic.
 * CLOSURE (not in the paper): each part is the closure of a qubit set from
 * the current front (every unplaced gate on those qubits whose
 * predecessors are placed), the set chosen for the most two-qubit gates;
 * `trials` > 1 is the width of a beam search over such parts.  Parts are
 * taken in order, hence acyclic. */
typedef enum {
  HS_PART_NAT = 0,
  HS_PART_DFS = 1,
  HS_PART_DAGP = 2,
  HS_PART_GREEDY = 3,
  HS_PART_CLOSURE = 4
} hs_strategy;

/* How hs_simulate applies a plan:
 *   GATE_PER_PASS -- ignore the partition; one sweep of the state per gate
 *                    (the non-hierarchical case of Sec. III.B);
 *   PART_LDS      -- one sweep per part; each part runs gate by gate on
 *                    register-resident sub-states, staged through LDS;
 *   PART_FUSED    -- one sweep per part; each part's gates are multiplied
 *                    into one dense 2^w x 2^w unitary applied on matrix cores;
 *   AUTO          -- per part, the cheaper by a cost model of PART_FUSED and
 *                    the gate-by-gate kernel: PART_SPEC's when
 *                    hs_plan_specialize has built them for the state's dtype
 *                    and device, else PART_LDS's;
 *   PART_SPEC     -- one sweep per part, as PART_LDS, with each part's kernel
 *                    specialized at plan time: the part's layouts, register
 *                    operations and coefficients become compile-time
 *                    constants of a kernel built with hipRTC for gfx950
 *                    (hs_plan_specialize builds them ahead; otherwise the
 *                    first hs_simulate does). */
typedef enum {
  HS_EXEC_GATE_PER_PASS = 0, HS_EXEC_PART_LDS = 1, HS_EXEC_PART_FUSED = 2, HS_EXEC_AUTO = 3,
  HS_EXEC_PART_SPEC = 4
} hs_exec;

typedef struct hs_state_* hs_state;
typedef struct hs_circuit_* hs_circuit;
typedef struct hs_plan_* hs_plan;

/* ---- library ------------------------------------------------------------ */

/* Version string of the library; never NULL. */
const char* hs_version(void);

/* Message for the last non-OK status returned on the calling thread ("" if
 * none).  The pointer stays valid until the thread's next failing call. */
const char* hs_last_error(void);

/* Number of HIP devices visible (0 on a machine without a GPU). */
hs_status hs_device_count(int* out);

/* Layout knobs read when a plan is next compiled (plans already compiled
 * keep theirs): "rb_c64" / "rb_c128" = register bits per lane (2^rb
 * amplitudes each; 1..4 / 1..3 for the interpreter kernel, 1..5 for the
 * specialized kernels); "contig" = the tile always holds qubits 0..contig-1
 * (0..8, default 6); "min_run_c64" / "min_run_c128" = gather and scatter straight in a
 * stage's layout when its lanes still cover qubits 0..min_run-1, instead of
 * re-laying out through LDS (0..6; 6 = only fully contiguous 64-amplitude
 * runs); "min_tile" (0..16) = pad every tile with the lowest free qubits up
 * to this many qubits, for longer contiguous runs (0 = lanes + registers;
 * capped at the kernel's widest tile); "fuse2" (0/1; default 1 for the
 * interpreter, 0 for the specialized kernels) = merge a two-qubit gate and
 * the dense one-qubit gates around it into one 4 x 4 op where that saves
 * instructions.  Launch shape of the part kernels: "xcd" (0/1) = each of the 8
 * XCDs sweeps one contiguous eighth of the tiles; "grid" = 0 for one
 * workgroup per tile, g in 1..64 for a persistent grid of g x the resident
 * workgroups per CU; "spec_prefetch" (0/1) = a persistent grid of the
 * specialized kernels keeps the next tile's loads in flight;
 * "spec_lds_limit_kib" (16..160, default 64) = the specialized kernels run
 * each LDS re-layout in 2 or 4 rounds, over half or a quarter of the tile,
 * when the tile's LDS image is larger; "fused_shape" (-1..2, default -1) =
 * launch shape of the fused kernels of 4- and 5-qubit parts: 0 = one group
 * of tiles per workgroup, 1 = a persistent grid whose waves issue the next
 * group's loads before the current group's products, 2 = a persistent grid
 * of the plain kernel, -1 = the measured best for the width and precision.
 * Host side: "host_threads" (0..64, default 0 = up to 8 as the host has
 * them) = threads a CLOSURE beam search may use; its plans are the same
 * for every value.  "serve_chunk" (1..4096, default 8) = part-passes a
 * serving request queues at a time (two chunks at most), read when a
 * request is launched.  A "spec_"
 * prefix on a key sets it for the specialized kernels (PART_SPEC) instead of
 * the interpreter kernel ("contig" has no prefix: it applies to both).
 * HS_E_ARG for an unknown key or value. */
hs_status hs_tune(const char* key, int value);

/* Largest part width k that hs_simulate with `exec` accepts for every part
 * of a k-bounded plan on the given dtype: the LDS tile capacity less the
 * coalescing pad for PART_LDS / PART_SPEC / AUTO, 7 for PART_FUSED (a
 * 128 x 128 unitary), unbounded (64) for GATE_PER_PASS. */
hs_status hs_max_part_qubits(hs_dtype dtype, hs_exec exec, int* out);

/* ---- states (Sec. II.B) --------------------------------------------------- */

/* New n-qubit state in library-owned device memory on the current device,
 * bound to `hip_stream` (a hipStream_t, may be NULL).  Contents undefined
 * until hs_state_set_basis.  1 <= n <= 40; HS_E_NOMEM if it does not fit. */
hs_status hs_state_create(int n, hs_dtype dtype, void* hip_stream, hs_state* out);

/* Borrow caller-owned device memory `dev_ptr` of `bytes` bytes holding 2^n
 * amplitudes of `dtype` (bytes must be exactly 2^n * 8 or 2^n * 16), bound
 * to `hip_stream`.  The memory must outlive the handle. */
hs_status hs_state_wrap(int n, hs_dtype dtype, void* dev_ptr, size_t bytes,
                        void* hip_stream, hs_state* out);

/* Set the state to the basis state |x> (x < 2^n; x = 0 is |0...0>). */
hs_status hs_state_set_basis(hs_state s, uint64_t x);

hs_status hs_state_info(hs_state s, int* n, hs_dtype* dtype, void** dev_ptr);

/* Wait for the state's stream, free library-owned memory and the handle.
 * The handle is gone even on error; HS_E_HIP reports a failed wait or free
 * (work enqueued on the state did not complete). */
hs_status hs_state_destroy(hs_state s);

/* ---- circuits (Sec. II.B: a sequence of gates) ----------------------------- */

/* Copy and validate `count` gates on n qubits; three-qubit kinds are
 * replaced by their one- and two-qubit decompositions (see hs_kind).
 * HS_E_QUBIT_RANGE for a qubit outside [0, n) or a gate with repeated
 * qubits; HS_E_ARG for an unknown kind, a one-qubit gate with q1 != -1, a
 * non-zero q2 on a one- or two-qubit kind, or a non-finite angle. */
hs_status hs_circuit_load(int n, const hs_gate* gates, size_t count, hs_circuit* out);

/* *count = the number of gates after decomposition: gate ids in partitions
 * (hs_plan_part_of_gate) index this sequence. */
hs_status hs_circuit_info(hs_circuit c, int* n, size_t* count);
hs_status hs_circuit_destroy(hs_circuit c);

/* ---- partitioning (Sec. IV) ------------------------------------------------ */

/* Partition the circuit's gate DAG into acyclic parts of at most k qubits
 * (Sec. IV.A conditions i-ii), minimising the part count heuristically
 * (condition iii).  `seed` and `trials` drive DFS (trial 0 is the natural
 * order, so DFS never returns more parts than Nat) and GREEDY; `trials` is
 * CLOSURE's beam width; Nat ignores both.
 * Strategies: NAT and DFS cut one topological order (Sec. IV.B.1-2); DAGP
 * bisects the DAG (Sec. IV.B.3); GREEDY grows each part one ready gate at
 * a time, fewest new qubits first; CLOSURE fixes each part by a qubit set
 * chosen so that the two-qubit gates it can take from the current front
 * (its closure) are most, improved by one-qubit exchanges, and with
 * trials > 1 searches a beam of that many partial partitions (on up to 8
 * host threads; the result does not depend on their number).
 * Parts are numbered in a topological order of the part-graph.
 * HS_E_ARITY_GT_K if a gate is wider than k; HS_E_ARG if k < 1, trials < 1
 * (DFS, GREEDY, CLOSURE) or a CLOSURE beam wider than 65536. */
hs_status hs_partition(hs_circuit c, int k, hs_strategy strategy, uint64_t seed,
                       int trials, hs_plan* out);

/* Multi-level partition (Sec. IV.B, multi-level paragraph).  Level 1 cuts
 * the DAG into acyclic parts sized for one tile of the part-pass kernels:
 * every tile gathers qubits 0..pad_qubits-1 anyway (coalescing padding), so
 * a part's qubits together with those number at most tile_qubits.  Level 2
 * -- register stages inside a part -- is formed when the plan is compiled.
 * With pad_qubits = 6 and tile_qubits = 6 + hs_max_part_qubits(dtype,
 * PART_SPEC) every part fits the specialized kernels' tile.  The plan's k
 * is tile_qubits and hs_plan_validate checks the padded bound.
 * HS_E_ARITY_GT_K if a gate with the padding exceeds tile_qubits; HS_E_ARG
 * for pad_qubits outside [0, 64] or tile_qubits < 1. */
hs_status hs_partition_multilevel(hs_circuit c, int tile_qubits, int pad_qubits,
                                  hs_strategy strategy, uint64_t seed, int trials, hs_plan* out);

/* Build a plan from a caller-given assignment part_of_gate[count] (ids
 * 0..P-1, one per gate of the circuit after decomposition: count must equal
 * hs_circuit_info's count, else HS_E_ARG).  HS_E_BAD_PARTITION unless it
 * passes hs_plan_validate's checks. */
hs_status hs_plan_from_assignment(hs_circuit c, int k, const int32_t* part_of_gate, size_t count,
                                  hs_plan* out);

hs_status hs_plan_num_parts(hs_plan p, int* parts);

/* *count = the plan's gate count (after decomposition); if out is not NULL
 * it receives the part id of every gate, out[0 .. *count) -- HS_E_ARG if
 * cap < *count. */
hs_status hs_plan_part_of_gate(hs_plan p, int32_t* out, size_t cap, size_t* count);

/* Qubit mask (bit q set if the part uses qubit q) and gate count of a part. */
hs_status hs_plan_part_info(hs_plan p, int part, uint64_t* qubit_mask, int* num_gates);

/* Exact check: every gate in exactly one non-empty part, every part uses at
 * most k qubits (for a multi-level plan: together with its padding qubits),
 * the part-graph is acyclic and every cross-part edge goes from a lower to a
 * higher part id.  HS_OK or HS_E_BAD_PARTITION. */
hs_status hs_plan_validate(hs_plan p);

/* Kernel-level layout of a part as compiled for `dtype` and `exec`
 * (PART_SPEC: the specialized kernels; any other mode: the interpreter
 * kernel): tile width m (qubits per gathered sub-state, the part's qubits
 * plus the lowest other qubits as padding), register stages, LDS round
 * trips per tile. */
hs_status hs_plan_part_layout(hs_plan p, int part, hs_dtype dtype, hs_exec exec, int* tile_qubits,
                              int* stages, int* lds_round_trips);

/* Introspection of the compiled descriptors of a part (`dtype`; `exec` as
 * for hs_plan_part_layout), so tests can replay them on the host.
 * header[24] = {m, lb, wb, rb,
 * entries, LDS round trips, ops, log2(tiles), tq[16]} (tq = tile bit ->
 * qubit).  entries[20 * entries] (filled if entries_cap >= entries): per
 * entry pos[16] (coordinate bit -> tile bit; lane bits, then wave bits, then
 * register bits), op_begin, op_end (relative to the part), transition, 0;
 * entry 0 is the load layout and the last entry the store layout.
 * ops[35 * ops] (filled if ops_cap >= ops): kind, b0, b1, c[32] with kinds
 * 0 dense 2x2, 1 real 2x2, 2 diagonal, 3 diag(1, d), 4 X, 5 CX, 6 CZ,
 * 7 controlled phase, 8 SWAP (coefficients in c[0..7]), 9 dense 4x4 on
 * b0 < b1 (index bit b0 + 2 bit b1; 16 complex entries, row-major). */
hs_status hs_plan_part_descriptors(hs_plan p, int part, hs_dtype dtype, hs_exec exec, int32_t* header,
                                   int32_t* entries, int entries_cap, double* ops, int ops_cap);

/* The HIP source of a part's specialized kernel (PART_SPEC) for `dtype`,
 * NUL-terminated, into buf[cap]; *len receives the length without the NUL
 * (query with buf = NULL).  HS_E_ARG if cap is too small. */
hs_status hs_plan_part_source(hs_plan p, int part, hs_dtype dtype, char* buf, size_t cap,
                              size_t* len);

/* Build (hipRTC, in parallel) and load the PART_SPEC kernels of every part
 * for `dtype` on the current device.  Kernels are cached per device by their
 * source, so plans sharing parts share kernels.  HS_E_HIP with the compiler
 * log on failure. */
hs_status hs_plan_specialize(hs_plan p, hs_dtype dtype);

/* hs_plan_specialize on a host thread of the library: returns at once (after
 * the part compile, so that a compile error is reported here).  While the
 * kernels build, HS_EXEC_AUTO runs the plan's gate-by-gate parts on the
 * interpreter kernel; once they are built it uses them.  A circuit run once
 * therefore never waits for hipRTC, and one run many times moves to the
 * specialized kernels after the build.  HS_EXEC_PART_SPEC waits for the build.
 * The build's error, if any, is reported by hs_plan_specialize_wait;
 * hs_plan_destroy waits for a build in progress. */
hs_status hs_plan_specialize_async(hs_plan p, hs_dtype dtype);

/* Wait for the background builds started on `p`; the first failure among them
 * (HS_E_HIP with the compiler log) or HS_OK. */
hs_status hs_plan_specialize_wait(hs_plan p, hs_dtype dtype);

/* *ready = 1 if the plan's specialized kernels for `dtype` are built on the
 * current device (HS_EXEC_AUTO then uses them), else 0. */
hs_status hs_plan_specialized(hs_plan p, hs_dtype dtype, int* ready);

/* The dense unitary U_p of a part as the fused path applies it: *w = the
 * number of qubits it acts on (4..7; parts of fewer than 4 qubits are
 * widened with the lowest other qubits, on which U acts as the identity).  If out is
 * not NULL it receives w doubles (the qubits, ascending; bit b of a row or
 * column index is the b-th of them) followed by the 2^w x 2^w matrix,
 * row-major, interleaved complex128.  Built in FP64 from the part's gates
 * in circuit order.  HS_E_UNSUPPORTED for parts wider than 7 qubits. */
hs_status hs_plan_part_unitary(hs_plan p, int part, int* w, double* out);

/* Which kernel HS_EXEC_AUTO runs for each part of `p` at `dtype` on the
 * current device: out[part] = 1 for the fused dense-unitary kernel, 0 for
 * the gate-by-gate kernel (the specialized one if the plan has been
 * specialized for `dtype` on this device, else the interpreter).  AUTO picks
 * per part the lower of the two cost estimates, in HBM sweeps of the state:
 * the gate-by-gate kernel's sweep plus its LDS re-layouts and register
 * operations, against the fused kernel's measured cost for the part's width
 * (Sec. III.A's cost argument: a part is memory-bound until its arithmetic
 * outgrows the sweep).  out has num_parts entries (caller-owned). */
hs_status hs_plan_auto_choice(hs_plan p, hs_dtype dtype, int32_t* out);

hs_status hs_plan_destroy(hs_plan p);

/* ---- simulation (Alg. 1) --------------------------------------------------- */

/* Apply the plan's circuit to the state, part after part in id order, each
 * part as one sweep (Alg. 1), or one sweep per gate for GATE_PER_PASS.
 * Asynchronous on the state's stream.  HS_E_ARG if the plan's n differs
 * from the state's; HS_E_UNSUPPORTED if a part exceeds hs_max_part_qubits. */
hs_status hs_simulate(hs_state s, hs_plan p, hs_exec exec);

/* One sweep per gate of the circuit, in circuit order (no partition). */
hs_status hs_simulate_gate_per_pass(hs_state s, hs_circuit c);

/* Apply a single part of a plan (one sweep).  Asynchronous. */
hs_status hs_simulate_part(hs_state s, hs_plan p, int part, hs_exec exec);

/* ---- readout (Sec. II.A-B) ------------------------------------------------- */

/* Copy amplitudes [first, first+count) to host as interleaved complex128
 * (out has 2*count doubles; complex64 states are widened on the device).
 * Syncs. */
hs_status hs_read_amplitudes(hs_state s, uint64_t first, uint64_t count, double* out);

/* Amplitudes at the caller's indices idx[count] (each < 2^n; host array,
 * copied) as interleaved complex128 into out[2*count].  Syncs. */
hs_status hs_read_amplitudes_at(hs_state s, const uint64_t* idx, uint64_t count, double* out);

/* |a|^2 in FP64 for amplitudes [first, first+count) into out[count].  Syncs. */
hs_status hs_probabilities(hs_state s, uint64_t first, uint64_t count, double* out);

/* Sum of |a|^2 over the whole state, accumulated in FP64 in a fixed-order
 * two-level tree (the same result on every run).  Syncs. */
hs_status hs_norm(hs_state s, double* out);

/* hs_norm for callers that cannot allocate device memory (code that runs
 * where hipMalloc is not allowed: tight serving loops, harnesses that forbid
 * allocation).  Same result as hs_norm, bit for bit: the same two kernels in
 * the same fixed order.  Their 1,024 partial sums and the result sit in a
 * static device array of 8,256 bytes that each GPU the library runs on holds
 * until the process ends; the reduction's shape does not depend on the state
 * size, so every state the library accepts fits and none is refused for its
 * size.  The array is found once per device (hipGetSymbolAddress, on the
 * first call on that device); the call never calls hipMalloc or hipFree.
 * All calls on one GPU share its array: calls that overlap on one GPU (two
 * host threads, or states on different streams) race and must be serialised
 * by the caller.  Writes the FP64 sum to *out (host memory); syncs the
 * state's stream.  Errors: HS_E_ARG for a null argument, HS_E_HIP if the
 * array's address or a launch fails. */
hs_status hs_norm_noalloc(hs_state s, double* out);

/* Wait for all work queued on the state's stream. */
hs_status hs_sync(hs_state s);

/* ---- measurement helper ---------------------------------------------------- */

/* Device-to-device copy of `bytes` bytes (multiple of 16) by a plain
 * streaming kernel, on `hip_stream`; used to calibrate HBM byte counters
 * against a kernel whose traffic is known. */
hs_status hs_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream);

/* ---- serving: continuous batching of many circuits ------------------------- */

typedef struct hs_server_* hs_server;

/* A server owns a pool of `num_streams` HIP streams on the current device,
 * four host threads that prepare requests (partition, compile, upload the
 * kernel descriptors from 8 MiB of pinned staging each) and a worker thread
 * that admits, launches and retires them.  Requests are admitted in ticket
 * order while the device bytes of resident states (plus their descriptors)
 * stay within `budget_bytes` (0 = free device memory at creation minus a
 * 4 GiB reserve); several requests are in flight on the device at once.
 * A request's descriptor copies (a few KiB per part) are queued before it is
 * admitted, and its stream waits for them on the device; its part-passes
 * are queued a chunk at a time (hs_tune "serve_chunk"), at most two chunks
 * outstanding, so later requests on the same hardware queue are not held
 * behind all of them.  Returns HS_E_HIP / HS_E_NOMEM if streams or buffers
 * cannot be created. */
hs_status hs_server_create(size_t budget_bytes, int num_streams, hs_server* out);

/* The server clock (seconds, monotonic) against which arrival times and
 * latencies are measured. */
hs_status hs_server_clock(hs_server sv, double* seconds);

/* Queue a circuit (copied and validated here) to be partitioned with limit
 * k by `strategy` (DFS and GREEDY with 16 trials, CLOSURE with beam
 * width 1), simulated from |init_basis> in `dtype`, and kept resident until
 * released.  `arrival_s`
 * is the request's arrival time on the server clock, where its latency
 * starts (negative: the time of this call; HS_E_ARG if it lies after the
 * call).  Returns a ticket.  HS_E_ADMISSION if the state alone can never fit
 * the budget (a request whose state and descriptors together exceed it fails
 * later with the same code, reported by hs_server_wait).  Does not wait for
 * partitioning, compilation or the device. */
hs_status hs_server_submit(hs_server sv, int n, const hs_gate* gates, size_t count,
                           hs_dtype dtype, uint64_t init_basis, int k,
                           hs_strategy strategy, double arrival_s, uint64_t* ticket);

/* Block until the ticket's result is ready (timeout_ms < 0: no limit).
 * HS_E_STATE on timeout; the request's own error if it failed. */
hs_status hs_server_wait(hs_server sv, uint64_t ticket, int64_t timeout_ms);

/* Non-blocking: *done = 1 if the ticket's result is ready (or it failed). */
hs_status hs_server_poll(hs_server sv, uint64_t ticket, int* done);

/* Read amplitudes of a finished request (as hs_read_amplitudes), staged
 * through a buffer the server allocated at creation. */
hs_status hs_server_read(hs_server sv, uint64_t ticket, uint64_t first, uint64_t count,
                         double* out);

/* Latency of a finished request: arrival to observed completion, seconds. */
hs_status hs_server_latency(hs_server sv, uint64_t ticket, double* seconds);

/* Where a finished request's latency went, seconds, summing to it:
 * out4[0] arrival -> preparation start (host queue), out4[1] preparation
 * (partition, compile, descriptor upload), out4[2] prepared -> launched
 * (waiting for admission), out4[3] launched -> completion observed (device). */
hs_status hs_server_timing(hs_server sv, uint64_t ticket, double* out4);

/* Free a finished request's device memory (its bytes return to the budget).
 * Stream-ordered frees: no device-wide wait.  Waits for hs_server_read calls
 * on the same ticket that are copying when it is called; reads that start
 * after it fail with HS_E_STATE. */
hs_status hs_server_release(hs_server sv, uint64_t ticket);

/* Counters: requests completed, peak admitted bytes, current admitted bytes,
 * peak number of requests on the device at once. */
hs_status hs_server_stats(hs_server sv, uint64_t* completed, uint64_t* peak_bytes,
                          uint64_t* cur_bytes, int* peak_inflight);

/* Wait for all submitted requests, stop the threads, free everything.
 * Requests still waiting for bytes that no running request will free fail
 * with HS_E_ADMISSION. */
hs_status hs_server_destroy(hs_server sv);

#ifdef __cplusplus
}
#endif

#endif /* HISV_H */
