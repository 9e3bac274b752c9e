"""Temporal-boundary amplitude engine for one AMD Instinct MI355X (gfx950).

Thin Python binding of ``libtnc.so`` (C ABI in ``include/tnc.h``): this module
only marshals arguments.  Planning runs in the library's C++ planner and every
step of the contraction runs in its HIP kernels; PyTorch provides device
memory and streams.  If the library is missing the import fails loudly; there
is no CPU fallback.

    from paper_2608_13110_amd import Plan
    plan = Plan.from_circuit(circ)            # host planner
    amps = plan.amplitudes(bits_cuda, k=8)    # torch complex128 on the GPU
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnc.so")

TNC_OK = 0
TNC_E_INVALID = -1
TNC_E_DOMAIN = -2
TNC_E_RANK = -3
TNC_E_NOMEM = -4
TNC_E_DEVICE = -5
GATE_CZ = 0
GATE_DENSE4 = 1
STORE_C64 = 0
STORE_F16_BLOCKSCALE = 1
STORE_BF16_BLOCKSCALE = 2

EXPORTED = [
    "tnc_plan", "tnc_plan_info", "tnc_prepare", "tnc_workspace_bytes", "tnc_amplitudes",
    "tnc_amplitudes_host", "tnc_logxeb", "tnc_release", "tnc_strerror", "tnc_last_error",
    "tnc_debug_execute_host", "tnc_debug_emulate_device", "tnc_profile_begin", "tnc_profile_end",
    "tnc_autotune", "tnc_server_create", "tnc_server_destroy", "tnc_server_set_tuning", "tnc_server_submit",
    "tnc_server_wait", "tnc_server_summary", "tnc_debug_arena_check", "tnc_sample_batched", "tnc_frugal_accept",
    "tnc_plan_ring", "tnc_ring_info", "tnc_ring_amplitudes", "tnc_debug_ring_emulate", "tnc_ring_release",
    "tnc_amplitudes_noalloc", "tnc_noalloc_scratch_bytes", "tnc_debug_workspace_c128", "tnc_debug_amplitudes_c128",
    "tnc_debug_lds_conflicts", "tnc_profile_launches", "tnc_plan_passes",
]


class TncError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Gate2(ctypes.Structure):
    _fields_ = [("layer", ctypes.c_int32), ("q", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("m", c128 * 16)]


class Options(ctypes.Structure):
    _fields_ = [("max_tile_bits", ctypes.c_int32), ("reg_bits", ctypes.c_int32),
                ("low_bits", ctypes.c_int32), ("math", ctypes.c_int32),
                ("late_fold", ctypes.c_int32), ("reg_adapt", ctypes.c_int32),
                ("bond", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mem_cap_bytes", ctypes.c_uint64)]


class Info(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("boundary_bits", ctypes.c_int32),
                ("live_slots_fixed", ctypes.c_int32), ("n_ops", ctypes.c_int32),
                ("n_passes", ctypes.c_int32), ("n_phases", ctypes.c_int32),
                ("n_late_launches", ctypes.c_int32), ("fixed_rows", ctypes.c_int32),
                ("early_layers", ctypes.c_int32), ("late_layers", ctypes.c_int32),
                ("log2_cost", ctypes.c_double), ("workspace_per_batch", ctypes.c_uint64),
                ("bond", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class Profile(ctypes.Structure):
    _fields_ = [("init_ms", ctypes.c_double), ("pass_ms", ctypes.c_double), ("late_ms", ctypes.c_double),
                ("init_launches", ctypes.c_int64), ("pass_launches", ctypes.c_int64),
                ("late_launches", ctypes.c_int64), ("pass_bytes", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerOptions(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("n_streams", ctypes.c_int32), ("n_planners", ctypes.c_int32),
                ("small_bits", ctypes.c_int32), ("max_graphs", ctypes.c_int32), ("max_group", ctypes.c_int32),
                ("group_window_us", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class RequestStats(ctypes.Structure):
    _fields_ = [("plan_ms", ctypes.c_double), ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("boundary_bits", ctypes.c_int32), ("mode", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("graph_launches", ctypes.c_int64),
                ("graph_builds", ctypes.c_int64), ("graph_failures", ctypes.c_int64),
                ("plain_launches", ctypes.c_int64), ("groups", ctypes.c_int64),
                ("grouped_requests", ctypes.c_int64), ("grouped_launches", ctypes.c_int64),
                ("plan_cache_hits", ctypes.c_int64), ("plan_cache_misses", ctypes.c_int64),
                ("max_inflight", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("latency_ms_p50", ctypes.c_double), ("latency_ms_p99", ctypes.c_double),
                ("latency_ms_max", ctypes.c_double), ("elapsed_s", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded ``libtnc.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_13110_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    L.tnc_plan.argtypes = [i32, i32, vp, i32, vp, vp, ctypes.POINTER(vp)]
    L.tnc_plan_info.argtypes = [vp, i32, ctypes.POINTER(Info)]
    L.tnc_prepare.argtypes = [vp, i32]
    L.tnc_workspace_bytes.argtypes = [vp, i32, i32, i32, ctypes.POINTER(u64)]
    L.tnc_amplitudes.argtypes = [vp, i32, vp, i32, i32, vp, vp, u64, vp]
    L.tnc_amplitudes_host.argtypes = [vp, i32, vp, i32, i32, vp]
    L.tnc_amplitudes_noalloc.argtypes = [vp, i32, vp, i32, i32, vp, vp]
    L.tnc_noalloc_scratch_bytes.argtypes = []
    L.tnc_noalloc_scratch_bytes.restype = u64
    L.tnc_debug_lds_conflicts.argtypes = [vp, i32, vp]
    L.tnc_profile_launches.argtypes = [vp, vp, ctypes.c_int64, vp]
    L.tnc_plan_passes.argtypes = [vp, i32, vp, i32, vp]
    L.tnc_debug_workspace_c128.argtypes = [vp, i32, i32, ctypes.POINTER(u64)]
    L.tnc_debug_amplitudes_c128.argtypes = [vp, i32, vp, i32, vp, vp, u64, vp]
    L.tnc_logxeb.argtypes = [vp, i32, i32, vp, i32, vp, vp]
    L.tnc_sample_batched.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.tnc_plan_ring.argtypes = [i32, i32, vp, i32, vp, vp, vp]
    L.tnc_ring_info.argtypes = [vp, i32, i32, vp, vp, vp]
    L.tnc_ring_amplitudes.argtypes = [vp, i32, vp, i32, vp, vp, u64, vp]
    L.tnc_debug_ring_emulate.argtypes = [vp, i32, vp, i32, vp]
    L.tnc_ring_release.argtypes = [vp]
    L.tnc_frugal_accept.argtypes = [vp, ctypes.c_int64, i32, ctypes.c_double, vp, vp, vp, vp]
    L.tnc_release.argtypes = [vp]
    L.tnc_release.restype = None
    L.tnc_strerror.argtypes = [ctypes.c_int]
    L.tnc_strerror.restype = ctypes.c_char_p
    L.tnc_last_error.argtypes = []
    L.tnc_last_error.restype = ctypes.c_char_p
    L.tnc_debug_execute_host.argtypes = [vp, i32, vp, i32, vp]
    L.tnc_debug_emulate_device.argtypes = [vp, i32, vp, i32, i32, vp]
    L.tnc_profile_begin.argtypes = []
    L.tnc_profile_end.argtypes = [ctypes.POINTER(Profile)]
    L.tnc_autotune.argtypes = [i32, i32, i32, i32, vp, i32, i32, ctypes.POINTER(i32), vp]
    L.tnc_server_create.argtypes = [ctypes.POINTER(ServerOptions), ctypes.POINTER(vp)]
    L.tnc_server_destroy.argtypes = [vp]
    L.tnc_server_destroy.restype = None
    L.tnc_server_set_tuning.argtypes = [vp, i32, ctypes.POINTER(Options)]
    L.tnc_server_submit.argtypes = [vp, i32, i32, vp, i32, vp, i32, vp, i32, i32, vp, ctypes.POINTER(u64)]
    L.tnc_server_wait.argtypes = [vp, u64, ctypes.POINTER(RequestStats)]
    L.tnc_server_summary.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.tnc_debug_arena_check.argtypes = [u64, i32]
    for name in EXPORTED:
        if name not in ("tnc_release", "tnc_strerror", "tnc_last_error", "tnc_server_destroy", "tnc_ring_release",
                        "tnc_noalloc_scratch_bytes"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != TNC_OK:
        L = lib()
        msg = L.tnc_last_error().decode() or L.tnc_strerror(rc).decode()
        raise TncError(rc, msg)


def _c128_array(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data


def _gate_array(gates: Sequence):
    garr = (Gate2 * max(1, len(gates)))()
    for i, g in enumerate(gates):
        layer, q, kind, m = g[0], g[1], g[2], g[3]
        garr[i].layer, garr[i].q, garr[i].kind = int(layer), int(q), int(kind)
        if kind == GATE_DENSE4:
            mm = np.asarray(m, dtype=np.complex128).reshape(16)
            for e in range(16):
                garr[i].m[e].re, garr[i].m[e].im = float(mm[e].real), float(mm[e].imag)
    return garr


_OPTION_KEYS = ("max_tile_bits", "reg_bits", "low_bits", "math", "late_fold", "reg_adapt", "bond", "mem_cap_bytes")


def _options(options: dict) -> Options:
    unknown = set(options) - set(_OPTION_KEYS)
    if unknown:
        raise ValueError(f"unknown tile options: {sorted(unknown)}")
    o = Options()
    for k in _OPTION_KEYS:
        setattr(o, k, int(options.get(k, 0)))
    return o


class Plan:
    """A planned circuit (``tnc_plan``); owns the library handle."""

    def __init__(self, n: int, d: int, one_qubit: np.ndarray, gates: Sequence, options: Optional[dict] = None):
        L = lib()
        self.n, self.d = int(n), int(d)
        one = np.ascontiguousarray(np.asarray(one_qubit, dtype=np.complex128).reshape(-1))
        if one.size != (self.d + 1) * self.n * 4:
            raise ValueError("one_qubit must hold (d+1)*n 2x2 gates")
        garr = _gate_array(gates)
        opt = _options(options) if options else None
        h = ctypes.c_void_p()
        self._one = one
        _check(L.tnc_plan(self.n, self.d, one.ctypes.data, len(gates), ctypes.addressof(garr),
                          ctypes.byref(opt) if opt is not None else None, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_circuit(cls, circ, options: Optional[dict] = None) -> "Plan":
        """Plan any object with ``n``, ``d``, ``one_qubit`` and ``gates``."""
        return cls(circ.n, circ.d, circ.one_qubit, circ.gates, options)

    @property
    def handle(self):
        return self._h

    def release(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tnc_release(self._h)
        self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def info(self, k: int = 0) -> dict:
        inf = Info()
        _check(lib().tnc_plan_info(self._h, int(k), ctypes.byref(inf)))
        return inf.as_dict()

    def prepare(self, k: int):
        _check(lib().tnc_prepare(self._h, int(k)))

    def workspace_bytes(self, k: int, n_batches: int, storage: int = STORE_C64) -> int:
        out = ctypes.c_uint64()
        _check(lib().tnc_workspace_bytes(self._h, int(k), int(n_batches), int(storage), ctypes.byref(out)))
        return int(out.value)

    # ----------------------------------------------------------- device path
    def amplitudes(self, bits, k: int, out=None, workspace=None, stream=None, storage: int = STORE_C64):
        """Amplitude batches on the GPU (``tnc_amplitudes``).

        bits: torch uint8 (batches, n) on the device.  Returns (or fills)
        torch complex128 (batches, 2^k).  ``workspace``: torch uint8 device
        buffer (allocated here when None).  Enqueued on ``stream`` (default:
        torch's current stream); no synchronization.
        """
        import torch
        if bits.device.type != "cuda" or bits.dtype != torch.uint8 or not bits.is_contiguous():
            raise ValueError("bits must be a contiguous uint8 CUDA tensor")
        nb = int(bits.shape[0])
        if bits.shape[1] != self.n:
            raise ValueError("bits must have n columns")
        if out is None:
            out = torch.empty((nb, 1 << k), dtype=torch.complex128, device=bits.device)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(k, nb, storage), dtype=torch.uint8, device=bits.device)
        s = stream if stream is not None else torch.cuda.current_stream(bits.device)
        _check(lib().tnc_amplitudes(self._h, nb, bits.data_ptr(), int(k), int(storage), out.data_ptr(),
                                    workspace.data_ptr(), workspace.numel(), ctypes.c_void_p(s.cuda_stream)))
        return out

    def amplitudes_noalloc(self, bits, k: int, out=None, stream=None, storage: int = STORE_C64):
        """``tnc_amplitudes_noalloc``: as ``amplitudes``, with the workspace
        taken from the library's per-GPU scratch (no device allocation by the
        library; ``prepare(k)`` must have run on this device)."""
        import torch
        if bits.device.type != "cuda" or bits.dtype != torch.uint8 or not bits.is_contiguous():
            raise ValueError("bits must be a contiguous uint8 CUDA tensor")
        nb = int(bits.shape[0])
        if bits.shape[1] != self.n:
            raise ValueError("bits must have n columns")
        if out is None:
            out = torch.empty((nb, 1 << k), dtype=torch.complex128, device=bits.device)
        s = stream if stream is not None else torch.cuda.current_stream(bits.device)
        _check(lib().tnc_amplitudes_noalloc(self._h, nb, bits.data_ptr(), int(k), int(storage), out.data_ptr(),
                                            ctypes.c_void_p(s.cuda_stream)))
        return out

    def amplitudes_host(self, bits: np.ndarray, k: int, storage: int = STORE_C64) -> np.ndarray:
        bits = np.ascontiguousarray(bits, dtype=np.uint8)
        out = np.empty((bits.shape[0], 1 << k), dtype=np.complex128)
        _check(lib().tnc_amplitudes_host(self._h, bits.shape[0], bits.ctypes.data, int(k), int(storage),
                                         out.ctypes.data))
        return out

    def debug_amplitudes_c128(self, bits, k: int, out=None, workspace=None, stream=None):
        """The complex128 reference path (``tnc_debug_amplitudes_c128``):
        unfused FP64 updates on a complex128 tensor, same join and late phase.
        bits: torch uint8 (batches, n) on the device."""
        import torch
        nb = int(bits.shape[0])
        if out is None:
            out = torch.empty((nb, 1 << k), dtype=torch.complex128, device=bits.device)
        if workspace is None:
            ws = ctypes.c_uint64()
            _check(lib().tnc_debug_workspace_c128(self._h, int(k), nb, ctypes.byref(ws)))
            workspace = torch.empty(int(ws.value), dtype=torch.uint8, device=bits.device)
        s = stream if stream is not None else torch.cuda.current_stream(bits.device)
        _check(lib().tnc_debug_amplitudes_c128(self._h, nb, bits.data_ptr(), int(k), out.data_ptr(),
                                               workspace.data_ptr(), workspace.numel(), ctypes.c_void_p(s.cuda_stream)))
        return out

    # ------------------------------------------------------- host self-checks
    def debug_execute_host(self, bits: np.ndarray, k: int) -> np.ndarray:
        bits = np.ascontiguousarray(bits, dtype=np.uint8)
        out = np.empty((bits.shape[0], 1 << k), dtype=np.complex128)
        _check(lib().tnc_debug_execute_host(self._h, bits.shape[0], bits.ctypes.data, int(k), out.ctypes.data))
        return out

    def passes(self, k: int) -> list:
        """The sweep's HBM passes in launch order (``tnc_plan_passes``)."""
        n = ctypes.c_int32()
        _check(lib().tnc_plan_passes(self._h, int(k), None, 0, ctypes.byref(n)))
        buf = np.zeros(7 * max(1, n.value), dtype=np.int32)
        _check(lib().tnc_plan_passes(self._h, int(k), buf.ctypes.data, n.value, ctypes.byref(n)))
        keys = ("low_bits", "win_lo", "win_len", "reg_bits", "updates", "phases", "fused_phases")
        return [dict(zip(keys, map(int, buf[7 * i:7 * i + 7]))) for i in range(n.value)]

    def debug_lds_conflicts(self, k: int) -> dict:
        """Register phases of the pass tables whose bank-cycle lane groups
        meet a slot twice (``tnc_debug_lds_conflicts``)."""
        st = np.zeros(3, dtype=np.int64)
        _check(lib().tnc_debug_lds_conflicts(self._h, int(k), st.ctypes.data))
        return {"phases": int(st[0]), "conflicted_16": int(st[1]), "conflicted_32": int(st[2])}

    def debug_emulate_device(self, bits: np.ndarray, k: int, storage: int = STORE_C64) -> np.ndarray:
        bits = np.ascontiguousarray(bits, dtype=np.uint8)
        out = np.empty((bits.shape[0], 1 << k), dtype=np.complex128)
        _check(lib().tnc_debug_emulate_device(self._h, bits.shape[0], bits.ctypes.data, int(k), int(storage),
                                              out.ctypes.data))
        return out


class RingPlan:
    """A ring circuit planned by slicing its wrap-pair CZ bonds
    (``tnc_plan_ring``, Sec. 6.3): gates listed at q = n-1 act on (n-1, 0)."""

    def __init__(self, n: int, d: int, one_qubit: np.ndarray, gates: Sequence, options: Optional[dict] = None):
        L = lib()
        self.n, self.d = int(n), int(d)
        one = np.ascontiguousarray(np.asarray(one_qubit, dtype=np.complex128).reshape(-1))
        if one.size != (self.d + 1) * self.n * 4:
            raise ValueError("one_qubit must hold (d+1)*n 2x2 gates")
        garr = _gate_array(gates)
        opt = _options(options) if options else None
        h = ctypes.c_void_p()
        _check(L.tnc_plan_ring(self.n, self.d, one.ctypes.data, len(gates), ctypes.addressof(garr),
                               ctypes.byref(opt) if opt is not None else None, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_circuit(cls, circ, options: Optional[dict] = None) -> "RingPlan":
        return cls(circ.n, circ.d, circ.one_qubit, circ.gates, options)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tnc_ring_release(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, k: int, n_batches: int = 1) -> dict:
        ns, w, ws = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_uint64()
        _check(lib().tnc_ring_info(self._h, int(k), int(n_batches), ctypes.byref(ns), ctypes.byref(w),
                                   ctypes.byref(ws)))
        return {"slices": ns.value, "width": w.value, "workspace_bytes": ws.value}

    def amplitudes(self, bits, k: int, out=None, workspace=None, stream=None):
        """Ring amplitude batches on the GPU (``tnc_ring_amplitudes``); bits
        as for ``Plan.amplitudes``."""
        import torch
        if bits.device.type != "cuda" or bits.dtype != torch.uint8 or not bits.is_contiguous():
            raise ValueError("bits must be a contiguous uint8 CUDA tensor")
        nb = int(bits.shape[0])
        if out is None:
            out = torch.empty((nb, 1 << k), dtype=torch.complex128, device=bits.device)
        if workspace is None:
            workspace = torch.empty(self.info(k, nb)["workspace_bytes"], dtype=torch.uint8, device=bits.device)
        s = stream if stream is not None else torch.cuda.current_stream(bits.device)
        _check(lib().tnc_ring_amplitudes(self._h, nb, bits.data_ptr(), int(k), out.data_ptr(), workspace.data_ptr(),
                                         workspace.numel(), ctypes.c_void_p(s.cuda_stream)))
        return out

    def debug_emulate_device(self, bits: np.ndarray, k: int) -> np.ndarray:
        bits = np.ascontiguousarray(bits, dtype=np.uint8)
        out = np.empty((bits.shape[0], 1 << k), dtype=np.complex128)
        _check(lib().tnc_debug_ring_emulate(self._h, bits.shape[0], bits.ctypes.data, int(k), out.ctypes.data))
        return out


def profile_begin():
    """Start recording HIP events around every kernel launch (process-wide)."""
    _check(lib().tnc_profile_begin())


def profile_end() -> dict:
    """Stop recording; wait for the events and return summed kernel times."""
    pr = Profile()
    _check(lib().tnc_profile_end(ctypes.byref(pr)))
    return pr.as_dict()


def profile_launches():
    """(class, ms) of every launch timed by the last ``profile_end``, in issue
    order (class 0 build-up / resolution, 1 pass, 2 late phase)."""
    n = ctypes.c_int64()
    _check(lib().tnc_profile_launches(None, None, 0, ctypes.byref(n)))
    cls = np.zeros(max(1, n.value), dtype=np.int32)
    ms = np.zeros(max(1, n.value), dtype=np.float64)
    _check(lib().tnc_profile_launches(cls.ctypes.data, ms.ctypes.data, n.value, ctypes.byref(n)))
    return list(zip(cls[:n.value].tolist(), ms[:n.value].tolist()))


def logxeb(amps, k: int, n_qubits: int, select=None, stream=None):
    """log-XEB (Sec. 5.2) of device amplitudes in FP64 on the GPU.

    amps: torch complex128 (batches, 2^k) on the device; select: optional
    torch int32 (batches,) device tensor choosing one component per batch.
    Returns a torch float64 device tensor {F, SE, lo, hi, N}.
    """
    import torch
    res = torch.empty(5, dtype=torch.float64, device=amps.device)
    s = stream if stream is not None else torch.cuda.current_stream(amps.device)
    _check(lib().tnc_logxeb(amps.data_ptr(), int(amps.shape[0]), int(k),
                            select.data_ptr() if select is not None else None, int(n_qubits),
                            res.data_ptr(), ctypes.c_void_p(s.cuda_stream)))
    return res


def sample_batched(amps, u, stream=None):
    """Batched sampling (Sec. 4.2, ``tnc_sample_batched``) on the GPU.

    amps: torch complex128 (batches, 2^k) on the device; u: torch float64
    (batches,) uniforms in [0, 1) on the device (the caller's random
    numbers).  Returns (b int32, Q float64) device tensors: the suffix drawn
    from p(b | a) and the prefix marginal Q_a of each batch.
    """
    import torch
    nb, B = int(amps.shape[0]), int(amps.shape[1])
    k = B.bit_length() - 1
    if B != 1 << k:
        raise ValueError("batches must hold 2^k amplitudes")
    b = torch.empty(nb, dtype=torch.int32, device=amps.device)
    q = torch.empty(nb, dtype=torch.float64, device=amps.device)
    s = stream if stream is not None else torch.cuda.current_stream(amps.device)
    _check(lib().tnc_sample_batched(amps.data_ptr(), nb, k, u.data_ptr(), b.data_ptr(), q.data_ptr(),
                                    ctypes.c_void_p(s.cuda_stream)))
    return b, q


def frugal_accept(amps, n_qubits: int, M: float, u, stream=None):
    """Frugal rejection (Sec. 4.1, ``tnc_frugal_accept``) on the GPU.

    amps: torch complex128 device tensor of candidate amplitudes (any shape);
    u: torch float64 device uniforms of the same size.  Returns (accept uint8,
    z float64) device tensors of that shape.
    """
    import torch
    accept = torch.empty(amps.shape, dtype=torch.uint8, device=amps.device)
    z = torch.empty(amps.shape, dtype=torch.float64, device=amps.device)
    s = stream if stream is not None else torch.cuda.current_stream(amps.device)
    _check(lib().tnc_frugal_accept(amps.data_ptr(), int(amps.numel()), int(n_qubits), float(M), u.data_ptr(),
                                   accept.data_ptr(), z.data_ptr(), ctypes.c_void_p(s.cuda_stream)))
    return accept, z


def autotune(n: int, d: int, k: int, candidates: Sequence[dict], storage: int = STORE_C64, reps: int = 3):
    """Time each candidate tile option set (``tnc_autotune``) on the current
    device for an (n, d) brickwork circuit; returns (best index, median ms
    per batch of every candidate)."""
    arr = (Options * len(candidates))(*[_options(c) for c in candidates])
    times = np.zeros(len(candidates), dtype=np.float64)
    best = ctypes.c_int32()
    _check(lib().tnc_autotune(int(n), int(d), int(k), int(storage), ctypes.addressof(arr), len(candidates),
                              int(reps), ctypes.byref(best), times.ctypes.data))
    return int(best.value), times


class Server:
    """Continuous-batching request loop (``tnc_server_*``) on the current device.

    submit() returns a request id at once; wait(id) returns the amplitudes
    (numpy complex128, (batches, 2^k)) and the request's timings.
    """

    def __init__(self, arena_bytes: int, n_streams: int = 4, n_planners: int = 4, small_bits: int = 20,
                 max_graphs: int = 256, max_group: int = 16, group_window_us: int = 0):
        o = ServerOptions(int(arena_bytes), int(n_streams), int(n_planners), int(small_bits), int(max_graphs),
                          int(max_group), int(group_window_us))
        h = ctypes.c_void_p()
        _check(lib().tnc_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._pending = {}

    def set_tuning(self, boundary_bits: int, options: dict):
        o = _options(options)
        _check(lib().tnc_server_set_tuning(self._h, int(boundary_bits), ctypes.byref(o)))

    def submit(self, circ, bits: np.ndarray, k: int, storage: int = STORE_C64) -> int:
        bits = np.ascontiguousarray(bits, dtype=np.uint8).reshape(-1, circ.n)
        one = np.ascontiguousarray(np.asarray(circ.one_qubit, dtype=np.complex128).reshape(-1))
        garr = _gate_array(circ.gates)
        out = np.empty((bits.shape[0], 1 << k), dtype=np.complex128)
        rid = ctypes.c_uint64()
        _check(lib().tnc_server_submit(self._h, int(circ.n), int(circ.d), one.ctypes.data, len(circ.gates),
                                       ctypes.addressof(garr), bits.shape[0], bits.ctypes.data, int(k),
                                       int(storage), out.ctypes.data, ctypes.byref(rid)))
        self._pending[rid.value] = out
        return int(rid.value)

    def wait(self, rid: int):
        st = RequestStats()
        rc = lib().tnc_server_wait(self._h, int(rid), ctypes.byref(st))
        out = self._pending.pop(int(rid))
        _check(rc)
        return out, st.as_dict()

    def summary(self) -> dict:
        st = ServerStats()
        _check(lib().tnc_server_summary(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tnc_server_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
