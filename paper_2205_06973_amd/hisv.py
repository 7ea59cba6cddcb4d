"""ctypes binding of libhisv.so (declared in include/hisv.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  The ``hs_*`` functions mirror the C entry points one to one and
raise :class:`HisvError` on a non-OK status; ``State``, ``Circuit``,
``Plan`` and ``Server`` own the corresponding handles.  PyTorch is used only
to hand over device memory and streams (``State.wrap_tensor``).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhisv.so")

HS_OK = 0
STATUS = {0: "HS_OK", 1: "HS_E_ARG", 2: "HS_E_QUBIT_RANGE", 3: "HS_E_ARITY_GT_K",
          4: "HS_E_NOMEM", 5: "HS_E_ADMISSION", 6: "HS_E_HIP", 7: "HS_E_BAD_PARTITION",
          8: "HS_E_STATE", 9: "HS_E_UNSUPPORTED", 10: "HS_E_INTERNAL"}
DTYPES = {"c64": 0, "c128": 1}
KINDS = {"h": 0, "x": 1, "y": 2, "z": 3, "s": 4, "t": 5, "rx": 6, "ry": 7, "rz": 8,
         "p": 9, "u3": 10, "cx": 11, "cz": 12, "cp": 13, "swap": 14, "ccx": 15, "cswap": 16}
STRATEGIES = {"nat": 0, "dfs": 1, "dagp": 2, "greedy": 3, "closure": 4}
EXEC = {"gate_per_pass": 0, "part_lds": 1, "part_fused": 2, "auto": 3, "part_spec": 4}


class HisvError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        super().__init__(f"{func}: {STATUS.get(status, status)}: {message}")
        self.status = status
        self.code = STATUS.get(status, str(status))


class hs_gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("q2", C.c_int32), ("p", C.c_double * 3)]


_vp = C.c_void_p
_u64 = C.c_uint64
_i32p = C.POINTER(C.c_int32)
_dp = C.POINTER(C.c_double)

# name -> (argtypes)
_SIGS = {
    "hs_device_count": [C.POINTER(C.c_int)],
    "hs_max_part_qubits": [C.c_int, C.c_int, C.POINTER(C.c_int)],
    "hs_tune": [C.c_char_p, C.c_int],
    "hs_state_create": [C.c_int, C.c_int, _vp, C.POINTER(_vp)],
    "hs_state_wrap": [C.c_int, C.c_int, _vp, C.c_size_t, _vp, C.POINTER(_vp)],
    "hs_state_set_basis": [_vp, _u64],
    "hs_state_info": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(_vp)],
    "hs_state_destroy": [_vp],
    "hs_circuit_load": [C.c_int, C.POINTER(hs_gate), C.c_size_t, C.POINTER(_vp)],
    "hs_circuit_info": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_size_t)],
    "hs_circuit_destroy": [_vp],
    "hs_partition": [_vp, C.c_int, C.c_int, _u64, C.c_int, C.POINTER(_vp)],
    "hs_partition_multilevel": [_vp, C.c_int, C.c_int, C.c_int, _u64, C.c_int, C.POINTER(_vp)],
    "hs_plan_from_assignment": [_vp, C.c_int, _i32p, C.c_size_t, C.POINTER(_vp)],
    "hs_plan_num_parts": [_vp, C.POINTER(C.c_int)],
    "hs_plan_part_of_gate": [_vp, _i32p, C.c_size_t, C.POINTER(C.c_size_t)],
    "hs_plan_part_info": [_vp, C.c_int, C.POINTER(_u64), C.POINTER(C.c_int)],
    "hs_plan_validate": [_vp],
    "hs_plan_part_layout": [_vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int),
                            C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "hs_plan_part_descriptors": [_vp, C.c_int, C.c_int, C.c_int, _i32p, _i32p, C.c_int, _dp,
                                 C.c_int],
    "hs_plan_part_source": [_vp, C.c_int, C.c_int, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)],
    "hs_plan_specialize": [_vp, C.c_int],
    "hs_plan_specialize_async": [_vp, C.c_int],
    "hs_plan_specialize_wait": [_vp, C.c_int],
    "hs_plan_specialized": [_vp, C.c_int, C.POINTER(C.c_int)],
    "hs_plan_part_unitary": [_vp, C.c_int, C.POINTER(C.c_int), _dp],
    "hs_plan_auto_choice": [_vp, C.c_int, C.POINTER(C.c_int32)],
    "hs_plan_destroy": [_vp],
    "hs_simulate": [_vp, _vp, C.c_int],
    "hs_simulate_gate_per_pass": [_vp, _vp],
    "hs_simulate_part": [_vp, _vp, C.c_int, C.c_int],
    "hs_read_amplitudes": [_vp, _u64, _u64, _dp],
    "hs_read_amplitudes_at": [_vp, C.POINTER(_u64), _u64, _dp],
    "hs_probabilities": [_vp, _u64, _u64, _dp],
    "hs_norm": [_vp, _dp],
    "hs_norm_noalloc": [_vp, _dp],
    "hs_sync": [_vp],
    "hs_copy_probe": [_vp, _vp, C.c_size_t, _vp],
    "hs_server_create": [C.c_size_t, C.c_int, C.POINTER(_vp)],
    "hs_server_clock": [_vp, _dp],
    "hs_server_submit": [_vp, C.c_int, C.POINTER(hs_gate), C.c_size_t, C.c_int, _u64, C.c_int,
                         C.c_int, C.c_double, C.POINTER(_u64)],
    "hs_server_wait": [_vp, _u64, C.c_int64],
    "hs_server_poll": [_vp, _u64, C.POINTER(C.c_int)],
    "hs_server_read": [_vp, _u64, _u64, _u64, _dp],
    "hs_server_latency": [_vp, _u64, _dp],
    "hs_server_timing": [_vp, _u64, _dp],
    "hs_server_release": [_vp, _u64],
    "hs_server_stats": [_vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64),
                        C.POINTER(C.c_int)],
    "hs_server_destroy": [_vp],
}

_lib = None


def lib() -> C.CDLL:
    """Load libhisv.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_2205_06973_amd.build")
        L = C.CDLL(LIB_PATH)
        L.hs_version.restype = C.c_char_p
        L.hs_version.argtypes = []
        L.hs_last_error.restype = C.c_char_p
        L.hs_last_error.argtypes = []
        for name, args in _SIGS.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = C.c_int
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols() -> list[str]:
    return ["hs_version", "hs_last_error", *_SIGS.keys()]


def _call(name: str, *args) -> None:
    rc = getattr(lib(), name)(*args)
    if rc != HS_OK:
        msg = lib().hs_last_error().decode(errors="replace")
        raise HisvError(rc, name, msg)


def hs_version() -> str:
    return lib().hs_version().decode()


def hs_last_error() -> str:
    return lib().hs_last_error().decode(errors="replace")


def hs_device_count() -> int:
    v = C.c_int()
    _call("hs_device_count", C.byref(v))
    return v.value


def hs_tune(key: str, value: int) -> None:
    _call("hs_tune", key.encode(), int(value))


def hs_max_part_qubits(dtype: str = "c64", exec_mode: str = "part_lds") -> int:
    v = C.c_int()
    _call("hs_max_part_qubits", DTYPES[dtype], EXEC[exec_mode], C.byref(v))
    return v.value


def gates_to_array(gates) -> C.Array:
    """(name, q0, q1, params[, q2]) tuples -> hs_gate[] (q2: the third qubit
    of "ccx" / "cswap")."""
    arr = (hs_gate * max(1, len(gates)))()
    for i, gate in enumerate(gates):
        name, q0, q1, params = gate[:4]
        g = arr[i]
        g.kind = KINDS[name]
        g.q0 = int(q0)
        g.q1 = int(q1)
        g.q2 = int(gate[4]) if len(gate) > 4 else 0
        for j, v in enumerate(tuple(params)[:3]):
            g.p[j] = float(v)
    return arr


class Circuit:
    def __init__(self, n: int, gates):
        self.n = int(n)
        self.gates = list(gates)
        arr = gates_to_array(self.gates)
        h = _vp()
        _call("hs_circuit_load", self.n, arr, len(self.gates), C.byref(h))
        self.handle = h

    @property
    def num_gates(self) -> int:
        """Gates after three-qubit kinds are decomposed (the ids partitions use)."""
        n, cnt = C.c_int(), C.c_size_t()
        _call("hs_circuit_info", self.handle, C.byref(n), C.byref(cnt))
        return cnt.value

    def close(self):
        if self.handle:
            lib().hs_circuit_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    def __init__(self, handle, circuit: Circuit, k: int):
        self.handle = handle
        self.circuit = circuit
        self.k = k

    @classmethod
    def partition(cls, circuit: Circuit, k: int, strategy: str = "dfs", seed: int = 0,
                  trials: int = 32) -> "Plan":
        h = _vp()
        _call("hs_partition", circuit.handle, int(k), STRATEGIES[strategy], int(seed),
              int(trials), C.byref(h))
        return cls(h, circuit, k)

    @classmethod
    def partition_multilevel(cls, circuit: Circuit, tile_qubits: int | None = None,
                             pad_qubits: int = 6, strategy: str = "dfs", seed: int = 0,
                             trials: int = 32, dtype: str = "c64") -> "Plan":
        """Parts whose qubits together with qubits 0..pad_qubits-1 number at
        most tile_qubits.  Default: the widest tile of the specialized kernels
        for dtype (14 qubits complex64, 13 complex128)."""
        if tile_qubits is None:
            tile_qubits = pad_qubits + hs_max_part_qubits(dtype, "part_spec")
        h = _vp()
        _call("hs_partition_multilevel", circuit.handle, int(tile_qubits), int(pad_qubits),
              STRATEGIES[strategy], int(seed), int(trials), C.byref(h))
        return cls(h, circuit, tile_qubits)

    @classmethod
    def from_assignment(cls, circuit: Circuit, k: int, part_of_gate) -> "Plan":
        arr = np.ascontiguousarray(np.asarray(part_of_gate, dtype=np.int32))
        h = _vp()
        _call("hs_plan_from_assignment", circuit.handle, int(k),
              arr.ctypes.data_as(_i32p), arr.size, C.byref(h))
        return cls(h, circuit, k)

    @property
    def num_parts(self) -> int:
        v = C.c_int()
        _call("hs_plan_num_parts", self.handle, C.byref(v))
        return v.value

    def part_of_gate(self) -> np.ndarray:
        """Part id of every gate (of the decomposed sequence)."""
        cnt = C.c_size_t()
        _call("hs_plan_part_of_gate", self.handle, None, 0, C.byref(cnt))
        out = np.zeros(max(1, cnt.value), dtype=np.int32)
        _call("hs_plan_part_of_gate", self.handle, out.ctypes.data_as(_i32p), out.size,
              C.byref(cnt))
        return out[:cnt.value]

    def part_info(self, part: int) -> tuple[int, int]:
        mask, ng = _u64(), C.c_int()
        _call("hs_plan_part_info", self.handle, int(part), C.byref(mask), C.byref(ng))
        return mask.value, ng.value

    def validate(self) -> None:
        _call("hs_plan_validate", self.handle)

    def part_layout(self, part: int, dtype: str = "c64", mode: str = "part_lds"):
        """(tile qubits, register stages, LDS round trips) of a compiled part."""
        m, s, t = C.c_int(), C.c_int(), C.c_int()
        _call("hs_plan_part_layout", self.handle, int(part), DTYPES[dtype], EXEC[mode],
              C.byref(m), C.byref(s), C.byref(t))
        return m.value, s.value, t.value

    def part_descriptors(self, part: int, dtype: str = "c64", mode: str = "part_lds"):
        """(header[24], entries[E, 20], ops[O, 35]) of a compiled part."""
        hdr = np.zeros(24, dtype=np.int32)
        _call("hs_plan_part_descriptors", self.handle, int(part), DTYPES[dtype], EXEC[mode],
              hdr.ctypes.data_as(_i32p), None, 0, None, 0)
        ne, no = int(hdr[4]), int(hdr[6])
        ent = np.zeros((ne, 20), dtype=np.int32)
        ops = np.zeros((max(no, 1), 35), dtype=np.float64)
        _call("hs_plan_part_descriptors", self.handle, int(part), DTYPES[dtype], EXEC[mode],
              hdr.ctypes.data_as(_i32p), ent.ctypes.data_as(_i32p), ne,
              ops.ctypes.data_as(_dp), max(no, 1))
        return hdr, ent, ops[:no]

    def part_source(self, part: int, dtype: str = "c64") -> str:
        n = C.c_size_t()
        _call("hs_plan_part_source", self.handle, int(part), DTYPES[dtype], None, 0, C.byref(n))
        buf = C.create_string_buffer(n.value + 1)
        _call("hs_plan_part_source", self.handle, int(part), DTYPES[dtype], buf, n.value + 1,
              C.byref(n))
        return buf.value.decode()

    def part_unitary(self, part: int):
        """(qubits, U) of a part's fused form; U is 2^w x 2^w complex128."""
        w = C.c_int()
        _call("hs_plan_part_unitary", self.handle, int(part), C.byref(w), None)
        R = 1 << w.value
        out = np.zeros(w.value + 2 * R * R, dtype=np.float64)
        _call("hs_plan_part_unitary", self.handle, int(part), C.byref(w), out.ctypes.data_as(_dp))
        qubits = [int(v) for v in out[:w.value]]
        return qubits, out[w.value:].view(np.complex128).reshape(R, R)

    def auto_choice(self, dtype: str = "c64") -> np.ndarray:
        """1 where AUTO runs the part on the fused kernel, 0 for gate by gate."""
        out = np.zeros(max(self.num_parts, 1), dtype=np.int32)
        _call("hs_plan_auto_choice", self.handle, DTYPES[dtype],
              out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out[: self.num_parts]

    def specialize(self, dtype: str = "c64") -> None:
        _call("hs_plan_specialize", self.handle, DTYPES[dtype])

    def specialize_async(self, dtype: str = "c64") -> None:
        _call("hs_plan_specialize_async", self.handle, DTYPES[dtype])

    def specialize_wait(self, dtype: str = "c64") -> None:
        _call("hs_plan_specialize_wait", self.handle, DTYPES[dtype])

    def specialized(self, dtype: str = "c64") -> bool:
        r = C.c_int()
        _call("hs_plan_specialized", self.handle, DTYPES[dtype], C.byref(r))
        return bool(r.value)

    def close(self):
        if self.handle:
            lib().hs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """An n-qubit state on the GPU (library-owned or a borrowed torch tensor)."""

    def __init__(self, handle, n: int, dtype: str, keepalive=None):
        self.handle = handle
        self.n = n
        self.dtype = dtype
        self._keepalive = keepalive

    @classmethod
    def create(cls, n: int, dtype: str = "c64", stream=None) -> "State":
        h = _vp()
        _call("hs_state_create", int(n), DTYPES[dtype], _stream_ptr(stream), C.byref(h))
        return cls(h, n, dtype)

    @classmethod
    def wrap_tensor(cls, tensor, stream=None) -> "State":
        """Borrow a 1-D torch complex64/complex128 CUDA tensor of length 2^n."""
        import torch
        if tensor.dim() != 1 or not tensor.is_cuda or not tensor.is_contiguous():
            raise ValueError("need a contiguous 1-D CUDA tensor")
        dtype = {torch.complex64: "c64", torch.complex128: "c128"}[tensor.dtype]
        N = tensor.numel()
        n = N.bit_length() - 1
        if (1 << n) != N:
            raise ValueError("tensor length is not a power of two")
        h = _vp()
        _call("hs_state_wrap", n, DTYPES[dtype], C.c_void_p(tensor.data_ptr()),
              N * tensor.element_size(), _stream_ptr(stream), C.byref(h))
        return cls(h, n, dtype, keepalive=tensor)

    def set_basis(self, x: int = 0) -> None:
        _call("hs_state_set_basis", self.handle, int(x))

    def simulate(self, plan: Plan, mode: str = "part_lds") -> None:
        _call("hs_simulate", self.handle, plan.handle, EXEC[mode])

    def simulate_part(self, plan: Plan, part: int, mode: str = "part_lds") -> None:
        _call("hs_simulate_part", self.handle, plan.handle, int(part), EXEC[mode])

    def simulate_gate_per_pass(self, circuit: Circuit) -> None:
        _call("hs_simulate_gate_per_pass", self.handle, circuit.handle)

    def amplitudes(self, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - first
        out = np.zeros(2 * max(count, 1), dtype=np.float64)
        _call("hs_read_amplitudes", self.handle, int(first), int(count), out.ctypes.data_as(_dp))
        return out[:2 * count].view(np.complex128)

    def amplitudes_at(self, indices) -> np.ndarray:
        idx = np.ascontiguousarray(np.asarray(indices, dtype=np.uint64))
        out = np.zeros(2 * max(idx.size, 1), dtype=np.float64)
        _call("hs_read_amplitudes_at", self.handle, idx.ctypes.data_as(C.POINTER(_u64)), idx.size,
              out.ctypes.data_as(_dp))
        return out[:2 * idx.size].view(np.complex128)

    def probabilities(self, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - first
        out = np.zeros(max(count, 1), dtype=np.float64)
        _call("hs_probabilities", self.handle, int(first), int(count), out.ctypes.data_as(_dp))
        return out[:count]

    def norm(self) -> float:
        v = C.c_double()
        _call("hs_norm", self.handle, C.byref(v))
        return v.value

    def norm_noalloc(self) -> float:
        v = C.c_double()
        _call("hs_norm_noalloc", self.handle, C.byref(v))
        return v.value

    def sync(self) -> None:
        _call("hs_sync", self.handle)

    def close(self):
        if self.handle:
            lib().hs_state_destroy(self.handle)
            self.handle = None
        self._keepalive = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(int(stream.cuda_stream))


def hs_copy_probe(src_ptr: int, dst_ptr: int, nbytes: int, stream=None) -> None:
    _call("hs_copy_probe", C.c_void_p(src_ptr), C.c_void_p(dst_ptr), int(nbytes),
          _stream_ptr(stream))


class Server:
    """Continuous-batching server (hs_server_*)."""

    def __init__(self, budget_bytes: int = 0, num_streams: int = 4):
        h = _vp()
        _call("hs_server_create", int(budget_bytes), int(num_streams), C.byref(h))
        self.handle = h

    def clock(self) -> float:
        """The server clock (seconds) that arrival times are given on."""
        v = C.c_double()
        _call("hs_server_clock", self.handle, C.byref(v))
        return v.value

    def submit(self, n: int, gates, dtype: str = "c64", init_basis: int = 0, k: int = 6,
               strategy: str = "dfs", arrival_s: float = -1.0) -> int:
        arr = gates_to_array(gates)
        t = _u64()
        _call("hs_server_submit", self.handle, int(n), arr, len(gates), DTYPES[dtype],
              int(init_basis), int(k), STRATEGIES[strategy], float(arrival_s), C.byref(t))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> None:
        _call("hs_server_wait", self.handle, int(ticket), int(timeout_ms))

    def poll(self, ticket: int) -> bool:
        d = C.c_int()
        _call("hs_server_poll", self.handle, int(ticket), C.byref(d))
        return bool(d.value)

    def amplitudes(self, ticket: int, first: int, count: int) -> np.ndarray:
        out = np.zeros(2 * max(count, 1), dtype=np.float64)
        _call("hs_server_read", self.handle, int(ticket), int(first), int(count),
              out.ctypes.data_as(_dp))
        return out[:2 * count].view(np.complex128)

    def latency(self, ticket: int) -> float:
        v = C.c_double()
        _call("hs_server_latency", self.handle, int(ticket), C.byref(v))
        return v.value

    def timing(self, ticket: int) -> tuple[float, float, float, float]:
        """(host queue, preparation, admission wait, device) seconds of a finished request."""
        out = np.zeros(4, dtype=np.float64)
        _call("hs_server_timing", self.handle, int(ticket), out.ctypes.data_as(_dp))
        return tuple(float(v) for v in out)

    def release(self, ticket: int) -> None:
        _call("hs_server_release", self.handle, int(ticket))

    def stats(self) -> dict:
        a, b, c, d = _u64(), _u64(), _u64(), C.c_int()
        _call("hs_server_stats", self.handle, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
        return {"completed": a.value, "peak_bytes": b.value, "cur_bytes": c.value,
                "peak_inflight": d.value}

    def close(self):
        if self.handle:
            lib().hs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
