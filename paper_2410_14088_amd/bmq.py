"""Thin Python binding of the C ABI in ``include/bmq.h`` (argument
marshalling only: every step of the stage loop runs in the HIP library).

PyTorch provides device memory (the arena and I/O tensors) and the stream.
The library is loaded from ``_build/libbmq.so`` next to this file; if it is
missing, :func:`lib` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BMQ_SO selects another build of the same library (the sanitized one)
SO = os.environ.get("BMQ_SO") or os.path.join(HERE, "_build", "libbmq.so")

SV_DOMAIN_LIN, SV_DOMAIN_LOG, SV_DOMAIN_RAW = 0, 1, 2
SV_FLAG_NO_SCRATCH = 1
SV_FLAG_NO_MFMA = 2
SV_FLAG_GATE_PER_STAGE = 4
SV_FLAG_DIAGONAL_FREE = 8
SV_FLAG_COMMUTE = 16
SV_FLAG_GROUP_SCRATCH = 32
SV_FLAG_REMAP = 64
SV_CHUNK_SLOT_BYTES = 576
KIND = {k: i for i, k in enumerate(
    ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U3", "CX", "CZ", "CP", "RZZ"])}
ERRORS = {-1: "SV_ERR_INVALID", -2: "SV_ERR_OOM", -3: "SV_ERR_CAPACITY", -4: "SV_ERR_HIP",
          -5: "SV_ERR_CORRUPT", -6: "SV_ERR_UNSUPPORTED", -7: "SV_ERR_TIMEOUT"}


class BmqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class sv_gate_t(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q", C.c_int32 * 2), ("pad", C.c_int32), ("p", C.c_double * 3)]


class sv_config_t(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("block_qubits", C.c_int32), ("inner_size", C.c_int32),
                ("fuse_qubits", C.c_int32), ("domain", C.c_int32), ("tile_qubits", C.c_int32),
                ("eb", C.c_double), ("pool_bytes", C.c_uint64), ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class sv_tune_space_t(C.Structure):
    _fields_ = [("n_tiles", C.c_int32), ("tiles", C.c_int32 * 4), ("n_fuse", C.c_int32), ("fuse", C.c_int32 * 5),
                ("n_inner", C.c_int32), ("inner", C.c_int32 * 6), ("probe_gates", C.c_uint64)]


class sv_fidelity_t(C.Structure):
    _fields_ = [("overlap2", C.c_double), ("fidelity", C.c_double), ("overlap_re", C.c_double),
                ("overlap_im", C.c_double), ("max_abs_err", C.c_double), ("norm2", C.c_double),
                ("ref_norm2", C.c_double)]


class sv_stage_stats_t(C.Structure):
    _fields_ = [("bytes_in", C.c_uint64), ("bytes_out", C.c_uint64), ("bytes_out_host", C.c_uint64),
                ("inter_bytes", C.c_uint64), ("dir_bytes", C.c_uint64),
                ("scratch_bytes", C.c_uint64), ("zero_chunks_out", C.c_uint64),
                ("mode_hist", C.c_uint64 * 4), ("passes", C.c_uint32), ("n_ops", C.c_uint32),
                ("n_gates", C.c_uint32), ("n_inner", C.c_uint32), ("ms", C.c_float), ("launches", C.c_uint32)]


EXPORTS = ["sv_last_error", "stage_plan", "plan_info", "plan_stage", "plan_gate_order", "plan_stage_ops", "plan_op", "plan_destroy",
           "sv_mem_required", "sv_create", "sv_destroy", "sv_attach_host_pool", "sv_host_alloc", "sv_host_free", "sv_reset", "stage_apply_compressed",
           "sv_fidelity", "sv_sample", "sv_export", "sv_amplitudes", "sv_footprint", "sv_check", "sv_directory",
           "sv_block_stream", "sv_debug_dump", "codec_workspace", "codec_encode", "codec_encode_noalloc", "codec_decode",
           "codec_encode_chunks", "codec_decode_chunks", "sv_block_features",
           "sv_block_labels", "mlp_forward", "mlp_work_floats", "mlp_loss_grad", "mlp_adam_update",
           "sv_graph_capture", "sv_graph_launch", "sv_graph_sync", "sv_graph_destroy", "sv_autotune",
           "sv_autotune_space", "plan_layout", "plan_gate", "sv_pipe_required", "sv_pipe_create", "sv_pipe_reset", "sv_pipe_apply",
           "sv_pipe_load", "sv_pipe_footprint", "sv_pipe_destroy",
           "sv_batch_workspace", "sv_batch_apply", "sv_persistent_workspace", "sv_persistent_apply",
           "sv_graph_capture_persistent",
           "sv_plan_features", "sv_plan_labels", "mlp_predict_work", "mlp_predict_bytes", "sv_admit"]
SV_FEATURES, SV_MLP_NPARAM = 32, 6597

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise RuntimeError(f"HIP library {SO} is not built; run __graft_entry__.build()")
        L = C.CDLL(SO)
        P, V = C.POINTER, C.c_void_p
        L.sv_last_error.restype = C.c_char_p
        L.stage_plan.argtypes = [V, C.c_size_t, P(sv_config_t), P(V)]
        L.plan_info.argtypes = [V, P(C.c_size_t), P(C.c_size_t), P(C.c_size_t)]
        L.plan_gate_order.argtypes = [V, P(C.c_uint32), C.c_size_t]
        L.plan_stage_ops.argtypes = [V, C.c_size_t, P(C.c_size_t), P(C.c_size_t)]
        L.plan_op.argtypes = [V, C.c_size_t, P(C.c_int32), P(C.c_int32), P(C.c_int32), V, C.c_size_t]
        L.plan_stage.argtypes = [V, C.c_size_t, P(C.c_size_t), P(C.c_size_t), P(C.c_int32),
                                 P(C.c_int32), P(C.c_int32)]
        L.plan_destroy.argtypes = [V]
        L.plan_destroy.restype = None
        L.sv_mem_required.argtypes = [P(sv_config_t), P(C.c_uint64)]
        L.sv_create.argtypes = [P(sv_config_t), V, C.c_uint64, V, P(V)]
        L.sv_destroy.argtypes = [V]
        L.sv_destroy.restype = None
        L.sv_reset.argtypes = [V]
        L.sv_attach_host_pool.argtypes = [V, V, C.c_uint64]
        L.sv_host_alloc.argtypes = [C.c_uint64, P(V)]
        L.sv_host_free.argtypes = [V]
        L.stage_apply_compressed.argtypes = [V, V, C.c_size_t, C.c_size_t, V]
        L.sv_fidelity.argtypes = [V, V, V, V, P(sv_fidelity_t)]
        L.sv_sample.argtypes = [V, C.c_uint64, C.c_uint64, V]
        L.sv_export.argtypes = [V, C.c_uint64, C.c_uint64, V]
        L.sv_amplitudes.argtypes = [V, V, C.c_uint64, V]
        L.sv_footprint.argtypes = [V, P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
        L.sv_check.argtypes = [V, P(C.c_uint64)]
        L.sv_directory.argtypes = [V, P(C.c_void_p), P(C.c_uint64)]
        L.sv_block_stream.argtypes = [V, C.c_uint64, V, C.c_uint64, P(C.c_uint64)]
        L.sv_debug_dump.argtypes = [V, C.c_uint64, C.c_uint64, V, V, V, V]
        L.codec_workspace.argtypes = [C.c_uint64, P(C.c_uint64)]
        L.codec_encode.argtypes = [V, V, C.c_uint64, P(sv_config_t), V, C.c_uint64, P(C.c_uint64), V, C.c_uint64, V]
        L.codec_decode.argtypes = [V, C.c_uint64, P(sv_config_t), C.c_uint64, V, V, V, C.c_uint64, V]
        L.codec_encode_noalloc.argtypes = [V, V, C.c_uint64, P(sv_config_t), V, C.c_uint64, P(C.c_uint64), V]
        L.codec_encode_chunks.argtypes = [V, V, C.c_uint64, P(sv_config_t), V, V, V]
        L.codec_decode_chunks.argtypes = [V, C.c_uint64, P(sv_config_t), V, V, V]
        L.sv_block_features.argtypes = [V, V, C.c_size_t, V]
        L.sv_graph_capture.argtypes = [V, V, C.c_size_t, C.c_size_t, P(V)]
        L.sv_batch_workspace.argtypes = [V, V, C.c_size_t, P(C.c_uint64)]
        L.sv_batch_apply.argtypes = [V, V, C.c_size_t, V, C.c_uint64, V]
        L.sv_persistent_workspace.argtypes = [V, V, C.c_size_t, P(C.c_uint64)]
        L.sv_persistent_apply.argtypes = [V, V, C.c_size_t, V, C.c_uint64, C.c_uint32, V]
        L.sv_graph_capture_persistent.argtypes = [V, V, V, C.c_uint64, C.c_uint32, P(V)]
        L.sv_autotune.argtypes = [V, C.c_size_t, P(sv_config_t), V, C.c_uint64, V, C.c_size_t, P(sv_config_t),
                                  P(C.c_float)]
        L.sv_autotune_space.argtypes = [V, C.c_size_t, P(sv_config_t), V, C.c_uint64, V, P(sv_tune_space_t),
                                        P(sv_config_t), P(C.c_float)]
        L.plan_layout.argtypes = [V, P(C.c_int32), C.c_size_t]
        L.plan_gate.argtypes = [V, C.c_size_t, P(C.c_int32), P(C.c_int32), P(C.c_double)]
        L.sv_pipe_required.argtypes = [P(sv_config_t), C.c_int32, P(C.c_uint64), P(C.c_uint64)]
        L.sv_pipe_create.argtypes = [P(sv_config_t), C.c_int32, V, C.c_uint64, V, C.c_uint64, V, P(V)]
        L.sv_pipe_reset.argtypes = [V]
        L.sv_pipe_apply.argtypes = [V, V, C.c_size_t, C.c_size_t, V]
        L.sv_pipe_load.argtypes = [V, V]
        L.sv_pipe_footprint.argtypes = [V] + [P(C.c_uint64)] * 5
        L.sv_pipe_destroy.argtypes = [V]
        L.sv_pipe_destroy.restype = None
        L.sv_graph_launch.argtypes = [V, V]
        L.sv_graph_sync.argtypes = [V]
        L.sv_graph_destroy.argtypes = [V]
        L.sv_graph_destroy.restype = None
        L.sv_block_labels.argtypes = [V, V, V]
        L.mlp_forward.argtypes = [V, V, C.c_uint32, V, V]
        L.mlp_work_floats.argtypes = [C.c_uint32]
        L.mlp_work_floats.restype = C.c_uint64
        L.mlp_loss_grad.argtypes = [V, V, V, V, C.c_uint32, V, V, V, V]
        L.mlp_adam_update.argtypes = [V, V, V, V, C.c_uint32, C.c_float, V]
        L.sv_plan_features.argtypes = [V, V, C.c_size_t, V]
        L.sv_plan_labels.argtypes = [V, V, V]
        L.mlp_predict_work.argtypes = [V, P(C.c_uint64)]
        L.mlp_predict_bytes.argtypes = [V, V, V, C.c_uint64, V, V]
        L.sv_admit.argtypes = [V, C.c_size_t, V, C.c_double, C.c_uint64, V, V, V]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise BmqError(rc, lib().sv_last_error().decode())


@dataclass
class Config:
    n: int
    b: int
    inner: int = 2
    fuse: int = 2
    domain: int = SV_DOMAIN_LIN
    eb: float = 1e-6
    tile: int = 0
    pool_bytes: int = 0
    flags: int = 0

    def c(self) -> sv_config_t:
        return sv_config_t(self.n, self.b, self.inner, self.fuse, self.domain, self.tile,
                           float(self.eb), int(self.pool_bytes), int(self.flags), 0)


def gate_array(gates) -> "C.Array":
    arr = (sv_gate_t * max(1, len(gates)))()
    for i, (k, q, p) in enumerate(gates):
        arr[i].kind = KIND[k]
        arr[i].q[0] = q[0]
        arr[i].q[1] = q[1] if len(q) > 1 else 0
        for j, v in enumerate(p):
            arr[i].p[j] = float(v)
    return arr


def _ptr(t) -> int:
    return t.data_ptr()


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class HostBuffer:
    """Page-locked host memory of exactly nbytes (sv_host_alloc), freed by
    close() or when the object goes away; the user keeps it alive while a
    state or pipeline uses it."""

    def __init__(self, nbytes: int):
        p = C.c_void_p()
        _check(lib().sv_host_alloc(int(nbytes), C.byref(p)))
        self.ptr, self.nbytes = p.value, int(nbytes)
        # kept here: at interpreter exit the module's globals may already be gone
        self._free, self._vp = lib().sv_host_free, C.c_void_p

    def data_ptr(self) -> int:
        return self.ptr

    def close(self):
        if getattr(self, "ptr", None):
            self._free(self._vp(self.ptr))
            self.ptr = None

    def __del__(self):
        self.close()


class Plan:
    """stage_plan: Algorithm 1 stages, tile passes and fused operations."""

    def __init__(self, gates: Sequence, cfg: Config):
        self.cfg = cfg
        arr = gate_array(gates)
        h = C.c_void_p()
        _check(lib().stage_plan(C.cast(arr, C.c_void_p), len(gates), C.byref(cfg.c()), C.byref(h)))
        self.h = h
        ns = self.info()["stages"]
        # gates as applied (more than the input with SV_FLAG_REMAP's swaps)
        self.n_gates = self.stage(ns - 1)["gates"][1] if ns else 0

    def layout(self):
        """Bit position of each logical qubit after the plan (identity unless SV_FLAG_REMAP)."""
        arr = (C.c_int32 * self.cfg.n)()
        _check(lib().plan_layout(self.h, arr, self.cfg.n))
        return list(arr)

    def gates(self):
        """The plan's gates as applied: (kind, positions, params), in plan order."""
        names = {v: k for k, v in KIND.items()}
        out = []
        for k in range(self.n_gates):
            kind, q, prm = C.c_int32(), (C.c_int32 * 2)(), (C.c_double * 3)()
            _check(lib().plan_gate(self.h, k, C.byref(kind), q, prm))
            qs = (q[0],) if q[1] < 0 else (q[0], q[1])
            out.append((names[kind.value], qs, tuple(prm)))
        return out

    def info(self):
        a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(lib().plan_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(stages=a.value, ops=b.value, passes=c.value)

    def stage(self, s: int):
        g0, g1 = C.c_size_t(), C.c_size_t()
        inner = (C.c_int32 * 8)()
        ni, npass = C.c_int32(), C.c_int32()
        _check(lib().plan_stage(self.h, s, C.byref(g0), C.byref(g1), inner, C.byref(ni), C.byref(npass)))
        return dict(gates=(g0.value, g1.value), inner=list(inner[:ni.value]), passes=npass.value)

    def gate_order(self):
        """Input index of each of the plan's gates (identity unless SV_FLAG_COMMUTE or
        SV_FLAG_REMAP; 0xFFFFFFFF for a remapping swap gate)."""
        arr = (C.c_uint32 * max(1, self.n_gates))()
        _check(lib().plan_gate_order(self.h, arr, self.n_gates))
        return list(arr[:self.n_gates])

    def stage_ops(self, s: int):
        """Fused operations of stage s in application order: (type, qubits,
        values) with values a complex64 matrix (dense) or phase vector."""
        import numpy as np
        b, e = C.c_size_t(), C.c_size_t()
        _check(lib().plan_stage_ops(self.h, s, C.byref(b), C.byref(e)))
        out = []
        for i in range(b.value, e.value):
            t, k = C.c_int32(), C.c_int32()
            qs = (C.c_int32 * 16)()
            _check(lib().plan_op(self.h, i, C.byref(t), C.byref(k), qs, None, 0))
            n = (1 << k.value) ** (2 if t.value == 0 else 1)
            buf = np.zeros(n, dtype=np.complex64)
            _check(lib().plan_op(self.h, i, None, None, None, C.c_void_p(buf.ctypes.data), n))
            vals = buf.reshape(1 << k.value, 1 << k.value) if t.value == 0 else buf
            out.append(("dense" if t.value == 0 else "diag", list(qs[:k.value]), vals))
        return out

    def stage_gates(self, s: int):
        """Input indices of stage s's gates, in the order they are applied."""
        g0, g1 = self.stage(s)["gates"]
        return self.gate_order()[g0:g1]

    @property
    def n_stages(self) -> int:
        return self.info()["stages"]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.plan_destroy(self.h)
            self.h = None


class State:
    """A compressed state vector in a torch-owned device arena."""

    def __init__(self, cfg: Config, device: str = "cuda:0"):
        import torch
        self.cfg = cfg
        need = C.c_uint64()
        _check(lib().sv_mem_required(C.byref(cfg.c()), C.byref(need)))
        self.arena = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=device)
        base = _ptr(self.arena)
        off = (-base) % 256
        h = C.c_void_p()
        _check(lib().sv_create(C.byref(cfg.c()), C.c_void_p(base + off), int(need.value), _stream(), C.byref(h)))
        self.h = h

    def apply(self, plan: Plan, first: int = 0, count: Optional[int] = None, stats: bool = False):
        if count is None:
            count = plan.n_stages - first
        st = (sv_stage_stats_t * max(1, count))() if stats else None
        _check(lib().stage_apply_compressed(self.h, plan.h, first, count,
                                            C.cast(st, C.c_void_p) if stats else None))
        if not stats:
            return None
        out = []
        for s in st[:count]:
            out.append(dict(bytes_in=s.bytes_in, bytes_out=s.bytes_out, bytes_out_host=s.bytes_out_host,
                            inter_bytes=s.inter_bytes, dir_bytes=s.dir_bytes,
                            scratch_bytes=s.scratch_bytes, zero_chunks_out=s.zero_chunks_out,
                            mode_hist=list(s.mode_hist), passes=s.passes, n_ops=s.n_ops,
                            n_gates=s.n_gates, n_inner=s.n_inner, ms=s.ms, launches=s.launches))
        return out

    def reset(self):
        _check(lib().sv_reset(self.h))

    def capture(self, plan: Plan, first: int = 0, count: Optional[int] = None) -> "Graph":
        """Record stages [first, first+count) as a HIP graph (nothing runs)."""
        if count is None:
            count = plan.n_stages - first
        h = C.c_void_p()
        _check(lib().sv_graph_capture(self.h, plan.h, first, count, C.byref(h)))
        return Graph(h, self, plan)

    def capture_persistent(self, plan: Plan, wait_limit_us: int = 0) -> "Graph":
        """Record the whole-circuit queue launch of plan as a HIP graph
        (sv_graph_capture_persistent); the workspace lives with the graph."""
        import torch
        sa = (C.c_void_p * 1)(self.h.value)
        pa = (C.c_void_p * 1)(plan.h.value)
        need = C.c_uint64()
        _check(lib().sv_persistent_workspace(sa, pa, 1, C.byref(need)))
        ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=self.arena.device)
        off = (-_ptr(ws)) % 256
        h = C.c_void_p()
        _check(lib().sv_graph_capture_persistent(self.h, plan.h, C.c_void_p(_ptr(ws) + off), int(need.value),
                                                 int(wait_limit_us), C.byref(h)))
        g = Graph(h, self, plan)
        g.workspace = ws
        return g

    def graph_sync(self):
        _check(lib().sv_graph_sync(self.h))

    def fidelity_full(self, ref=None) -> dict:
        """sv_fidelity against ref: None (norm only), a torch complex128 device
        tensor, a host numpy complex128 array (streamed by the library) or
        another State.  Returns every field of sv_fidelity_t."""
        out = sv_fidelity_t()
        host = dev = other = None
        if isinstance(ref, State):
            other = ref.h
        elif isinstance(ref, np.ndarray):
            if ref.dtype != np.complex128 or ref.size != (1 << self.cfg.n):
                raise ValueError("host reference must be 2^n complex128")
            ref = np.ascontiguousarray(ref)
            host = C.c_void_p(ref.ctypes.data)
        elif ref is not None:
            dev = C.c_void_p(_ptr(ref))
        _check(lib().sv_fidelity(self.h, host, dev, other, C.byref(out)))
        return {k: getattr(out, k) for k, _ in sv_fidelity_t._fields_}

    def fidelity(self, ref=None):
        """(|<ref|psi>|^2, max |psi - ref|, |psi|^2): the plain squared
        overlap, with reference and state as they are (see fidelity_full
        for the normalised value)."""
        r = self.fidelity_full(ref)
        return r["overlap2"], r["max_abs_err"], r["norm2"]

    def sample(self, k: int, seed: int) -> np.ndarray:
        """k indices drawn from |psi(x)|^2 (sv_sample), as a host uint64 array."""
        out = np.zeros(max(1, k), dtype=np.uint64)
        _check(lib().sv_sample(self.h, int(k), int(seed) & (2 ** 64 - 1), C.c_void_p(out.ctypes.data)))
        return out[:k]

    def export(self, start: int = 0, count: Optional[int] = None):
        import torch
        if count is None:
            count = (1 << self.cfg.n) - start
        out = torch.empty(count, dtype=torch.complex64, device=self.arena.device)
        _check(lib().sv_export(self.h, start, count, C.c_void_p(_ptr(out))))
        return out

    def amplitudes(self, idx):
        import torch
        idx = idx.to(device=self.arena.device, dtype=torch.int64).contiguous()
        out = torch.empty(idx.numel(), dtype=torch.complex64, device=self.arena.device)
        _check(lib().sv_amplitudes(self.h, C.c_void_p(_ptr(idx)), idx.numel(), C.c_void_p(_ptr(out))))
        return out

    def footprint(self):
        """(record bytes, of those in the host pool, directory bytes)"""
        r, h, d = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib().sv_footprint(self.h, C.byref(r), C.byref(h), C.byref(d)))
        return r.value, h.value, d.value

    def check(self) -> int:
        """Validate the chunk directory on the device; returns the number of
        bad entries (0), or raises BmqError (SV_ERR_CORRUPT, state poisoned)."""
        nb = C.c_uint64()
        _check(lib().sv_check(self.h, C.byref(nb)))
        return nb.value

    def directory(self):
        """(device address, entries) of the live copy's chunk directory."""
        ptr, n = C.c_void_p(), C.c_uint64()
        _check(lib().sv_directory(self.h, C.byref(ptr), C.byref(n)))
        return ptr.value, n.value

    def attach_host_pool(self, nbytes: int, exact: bool = False):
        """Second memory level: a pinned host buffer of nbytes (0 detaches);
        a pinned torch tensor, or with exact an sv_host_alloc buffer of
        exactly nbytes (torch's pinned allocator rounds up to a power of two)."""
        import torch
        if nbytes:
            buf = HostBuffer(int(nbytes)) if exact else torch.empty(int(nbytes), dtype=torch.uint8, pin_memory=True)
            _check(lib().sv_attach_host_pool(self.h, C.c_void_p(buf.data_ptr()), int(nbytes)))
        else:
            buf = None
            _check(lib().sv_attach_host_pool(self.h, None, 0))
        self.host_pool = buf

    def block_stream(self, block: int) -> bytes:
        nb = C.c_uint64()
        rc = lib().sv_block_stream(self.h, block, None, 0, C.byref(nb))
        if rc != 0 and nb.value == 0:
            _check(rc)
        buf = (C.c_uint8 * nb.value)()
        _check(lib().sv_block_stream(self.h, block, C.cast(buf, C.c_void_p), nb.value, C.byref(nb)))
        return bytes(buf)

    def debug_dump(self, re=None, im=None, start: int = 0, count: Optional[int] = None, dec_re=None, dec_im=None):
        """Test hook: later stages store the values they are about to encode
        (re, im) and the values their first pass decoded (dec_re, dec_im)
        for amplitudes [start, start+count); all None turns it off."""
        if count is None:
            count = (1 << self.cfg.n) - start
        p = lambda t: C.c_void_p(_ptr(t)) if t is not None else None
        _check(lib().sv_debug_dump(self.h, start, count, p(re), p(im), p(dec_re), p(dec_im)))

    @property
    def n_blocks(self) -> int:
        return 1 << (self.cfg.n - self.cfg.b)

    def block_features(self, plan: Plan, stage: int):
        """Predictor features of every block for the upcoming `stage`: [blocks][32]."""
        import torch
        out = torch.empty((self.n_blocks, SV_FEATURES), dtype=torch.float32, device=self.arena.device)
        _check(lib().sv_block_features(self.h, plan.h, stage, C.c_void_p(_ptr(out))))
        return out

    def plan_features(self, plan: Plan, stage: int):
        """Planning form of the block features (sv_plan_features): [blocks][32]."""
        import torch
        out = torch.empty((self.n_blocks, SV_FEATURES), dtype=torch.float32, device=self.arena.device)
        _check(lib().sv_plan_features(self.h, plan.h, stage, C.c_void_p(_ptr(out))))
        return out

    def plan_labels(self):
        """Planning form of the labels (sv_plan_labels): (log2 bytes per amplitude, mode)."""
        import torch
        lb = torch.empty(self.n_blocks, dtype=torch.float32, device=self.arena.device)
        md = torch.empty(self.n_blocks, dtype=torch.int32, device=self.arena.device)
        _check(lib().sv_plan_labels(self.h, C.c_void_p(_ptr(lb)), C.c_void_p(_ptr(md))))
        return lb, md

    def block_labels(self):
        """(log2 stream bytes, most frequent plane mode) per block of the current state."""
        import torch
        lb = torch.empty(self.n_blocks, dtype=torch.float32, device=self.arena.device)
        md = torch.empty(self.n_blocks, dtype=torch.int32, device=self.arena.device)
        _check(lib().sv_block_labels(self.h, C.c_void_p(_ptr(lb)), C.c_void_p(_ptr(md))))
        return lb, md

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sv_destroy(self.h)
            self.h = None
        pool = getattr(self, "host_pool", None)
        if pool is not None and hasattr(pool, "close"):   # a HostBuffer, freed once no state uses it
            pool.close()

    def __del__(self):
        self.close()


def autotune(gates, cfg: Config, probe_stages: int = 0, device: str = "cuda:0"):
    """Measure tile / fusion candidates on the device; returns (best Config,
    {(tile, fuse): ms})."""
    import torch
    need = C.c_uint64()
    _check(lib().sv_mem_required(C.byref(cfg.c()), C.byref(need)))
    arena = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=device)
    base = _ptr(arena)
    off = (-base) % 256
    arr = gate_array(gates)
    best = sv_config_t()
    ms = (C.c_float * 20)()
    _check(lib().sv_autotune(C.cast(arr, C.c_void_p), len(gates), C.byref(cfg.c()), C.c_void_p(base + off),
                             int(need.value), _stream(), probe_stages, C.byref(best), ms))
    table = {(10 + i // 5, 1 + i % 5): ms[i] for i in range(20) if ms[i] == ms[i]}
    out = Config(n=best.n_qubits, b=best.block_qubits, inner=best.inner_size, fuse=best.fuse_qubits,
                 domain=best.domain, eb=best.eb, tile=best.tile_qubits, pool_bytes=best.pool_bytes, flags=best.flags)
    return out, table


def _stats_list(st, count):
    return [dict(bytes_in=s.bytes_in, bytes_out=s.bytes_out, bytes_out_host=s.bytes_out_host,
                 inter_bytes=s.inter_bytes, dir_bytes=s.dir_bytes, scratch_bytes=s.scratch_bytes,
                 zero_chunks_out=s.zero_chunks_out, mode_hist=list(s.mode_hist), passes=s.passes, n_ops=s.n_ops,
                 n_gates=s.n_gates, n_inner=s.n_inner, ms=s.ms, launches=s.launches) for s in st[:count]]


class Pipe:
    """Host-resident compressed state (sv_pipe_*): block images in a pinned
    host store, each stage's SV groups moved through the device on `streams`
    streams (copy in, decompress / apply / recompress, copy out)."""

    def __init__(self, cfg: Config, streams: int = 2, host_bytes: Optional[int] = None, device: str = "cuda:0"):
        import torch
        self.cfg, self.streams = cfg, streams
        dev, hmin = C.c_uint64(), C.c_uint64()
        _check(lib().sv_pipe_required(C.byref(cfg.c()), streams, C.byref(dev), C.byref(hmin)))
        self.ws = torch.empty(int(dev.value) + 256, dtype=torch.uint8, device=device)
        if host_bytes is None:
            host_bytes = int(1.4 * (8 << cfg.n)) + int(hmin.value)
        self.host = torch.empty(int(host_bytes) + 256, dtype=torch.uint8, pin_memory=True)
        wo = (-_ptr(self.ws)) % 256
        ho = (-self.host.data_ptr()) % 256
        self.h = C.c_void_p()
        _check(lib().sv_pipe_create(C.byref(cfg.c()), streams, C.c_void_p(_ptr(self.ws) + wo), int(dev.value),
                                    C.c_void_p(self.host.data_ptr() + ho), int(host_bytes), _stream(),
                                    C.byref(self.h)))

    def apply(self, plan: Plan, first: int = 0, count: Optional[int] = None, stats: bool = False):
        if count is None:
            count = plan.n_stages - first
        st = (sv_stage_stats_t * max(1, count))() if stats else None
        _check(lib().sv_pipe_apply(self.h, plan.h, first, count, C.cast(st, C.c_void_p) if stats else None))
        return _stats_list(st, count) if stats else None

    def reset(self):
        _check(lib().sv_pipe_reset(self.h))

    def load(self, state: "State"):
        """Copy the host-resident state into a device State of the same configuration."""
        _check(lib().sv_pipe_load(self.h, state.h))

    def footprint(self) -> dict:
        v = [C.c_uint64() for _ in range(5)]
        _check(lib().sv_pipe_footprint(self.h, *[C.byref(x) for x in v]))
        return dict(record_bytes=v[0].value, image_bytes=v[1].value, host_used=v[2].value, h2d_bytes=v[3].value,
                    d2h_bytes=v[4].value)

    def close(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.sv_pipe_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        self.close()


def autotune_space(gates, cfg: Config, tiles=(12,), fuse=(1, 2, 3, 4, 5), inner=None, probe_gates: int = 0,
                   device: str = "cuda:0"):
    """Measure every (tile, fusion width, inner size) candidate on the first
    probe_gates gates (sv_autotune_space); returns (best Config,
    {(tile, fuse, inner): ms})."""
    import torch
    inner = (cfg.inner,) if inner is None else tuple(inner)
    sp = sv_tune_space_t()
    sp.n_tiles, sp.n_fuse, sp.n_inner = len(tiles), len(fuse), len(inner)
    for i, v in enumerate(tiles):
        sp.tiles[i] = v
    for i, v in enumerate(fuse):
        sp.fuse[i] = v
    for i, v in enumerate(inner):
        sp.inner[i] = v
    sp.probe_gates = probe_gates
    need = C.c_uint64(0)
    for m in inner:                         # group-sized scratch grows with the inner size
        nm = C.c_uint64()
        _check(lib().sv_mem_required(C.byref(dataclasses.replace(cfg, inner=m).c()), C.byref(nm)))
        need = nm if nm.value > need.value else need
    arena = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=device)
    base = _ptr(arena)
    off = (-base) % 256
    arr = gate_array(gates)
    best = sv_config_t()
    total = len(tiles) * len(fuse) * len(inner)
    ms = (C.c_float * total)()
    _check(lib().sv_autotune_space(C.cast(arr, C.c_void_p), len(gates), C.byref(cfg.c()), C.c_void_p(base + off),
                                   int(need.value), _stream(), C.byref(sp), C.byref(best), ms))
    del arena
    table = {}
    for it, t in enumerate(tiles):
        for ifu, f in enumerate(fuse):
            for ii, m in enumerate(inner):
                v = ms[(it * len(fuse) + ifu) * len(inner) + ii]
                if v == v:
                    table[(t, f, m)] = v
    out = Config(n=best.n_qubits, b=best.block_qubits, inner=best.inner_size, fuse=best.fuse_qubits,
                 domain=best.domain, eb=best.eb, tile=best.tile_qubits, pool_bytes=best.pool_bytes, flags=best.flags)
    return out, table


def batch_apply(states, plans):
    """Run every circuit's stages together (sv_batch_apply)."""
    import torch
    n = len(states)
    sa = (C.c_void_p * n)(*[st.h.value for st in states])
    pa = (C.c_void_p * n)(*[pl.h.value for pl in plans])
    need = C.c_uint64()
    _check(lib().sv_batch_workspace(sa, pa, n, C.byref(need)))
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=states[0].arena.device)
    base = _ptr(ws)
    off = (-base) % 256
    _check(lib().sv_batch_apply(sa, pa, n, C.c_void_p(base + off), int(need.value), _stream()))


def persistent_apply(states, plans, wait_limit_us: int = 0):
    """Run every circuit's stages in one persistent launch per tile size
    (sv_persistent_apply); wait_limit_us bounds each device-side wait
    (0 = the library default)."""
    import torch
    n = len(states)
    sa = (C.c_void_p * n)(*[st.h.value for st in states])
    pa = (C.c_void_p * n)(*[pl.h.value for pl in plans])
    need = C.c_uint64()
    _check(lib().sv_persistent_workspace(sa, pa, n, C.byref(need)))
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=states[0].arena.device)
    base = _ptr(ws)
    off = (-base) % 256
    _check(lib().sv_persistent_apply(sa, pa, n, C.c_void_p(base + off), int(need.value), int(wait_limit_us),
                                     _stream()))


class Graph:
    """A captured stage loop; replay with launch()."""

    def __init__(self, h, state: "State", plan: Plan):
        self.h, self.state, self.plan = h, state, plan

    def launch(self):
        _check(lib().sv_graph_launch(self.state.h, self.h))

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sv_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def codec_encode_chunks(re, im, cfg: Config):
    """Encode device float32 planes (whole chunks); returns (slots uint8 tensor, sizes int32 tensor)."""
    import torch
    n = re.numel()
    nch = (n + 63) // 64
    slots = torch.zeros(max(1, nch) * SV_CHUNK_SLOT_BYTES, dtype=torch.uint8, device=re.device)
    sizes = torch.zeros(max(1, nch), dtype=torch.int32, device=re.device)
    _check(lib().codec_encode_chunks(C.c_void_p(_ptr(re)), C.c_void_p(_ptr(im)), n, C.byref(cfg.c()),
                                     C.c_void_p(_ptr(slots)), C.c_void_p(_ptr(sizes)), _stream()))
    return slots, sizes


def codec_decode_chunks(slots, n: int, cfg: Config):
    import torch
    re = torch.empty(max(1, n), dtype=torch.float32, device=slots.device)
    im = torch.empty(max(1, n), dtype=torch.float32, device=slots.device)
    _check(lib().codec_decode_chunks(C.c_void_p(_ptr(slots)), n, C.byref(cfg.c()),
                                     C.c_void_p(_ptr(re)), C.c_void_p(_ptr(im)), _stream()))
    return re[:n], im[:n]


def _workspace(n: int, device):
    import torch
    need = C.c_uint64()
    _check(lib().codec_workspace(n, C.byref(need)))
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=device)
    off = (-_ptr(ws)) % 256
    return ws, C.c_void_p(_ptr(ws) + off), int(need.value)


def codec_encode(re, im, cfg: Config, cap: Optional[int] = None):
    """The canonical block stream of device float32 planes (codec_encode);
    returns a device uint8 tensor holding exactly the stream."""
    import torch
    n = re.numel()
    if cap is None:
        cap = 16 + (n // 64) * SV_CHUNK_SLOT_BYTES
    dst = torch.empty(max(cap, 4), dtype=torch.uint8, device=re.device)
    ws, wp, wb = _workspace(n, re.device)
    nb = C.c_uint64()
    _check(lib().codec_encode(C.c_void_p(_ptr(re)), C.c_void_p(_ptr(im)), n, C.byref(cfg.c()), C.c_void_p(_ptr(dst)),
                              int(cap), C.byref(nb), wp, wb, _stream()))
    return dst[:nb.value]


def codec_encode_noalloc(re, im, cfg: Config, cap: Optional[int] = None):
    """codec_encode with the library's static scratch (no workspace)."""
    import torch
    n = re.numel()
    if cap is None:
        cap = 16 + (n // 64) * SV_CHUNK_SLOT_BYTES
    dst = torch.empty(max(cap, 4), dtype=torch.uint8, device=re.device)
    nb = C.c_uint64()
    _check(lib().codec_encode_noalloc(C.c_void_p(_ptr(re)), C.c_void_p(_ptr(im)), n, C.byref(cfg.c()),
                                      C.c_void_p(_ptr(dst)), int(cap), C.byref(nb), _stream()))
    return dst[:nb.value]


def codec_decode(stream, n: int, cfg: Config):
    """Inverse of codec_encode: (re, im) device float32 planes of n values."""
    import torch
    stream = stream.contiguous()
    re = torch.empty(n, dtype=torch.float32, device=stream.device)
    im = torch.empty(n, dtype=torch.float32, device=stream.device)
    ws, wp, wb = _workspace(n, stream.device)
    _check(lib().codec_decode(C.c_void_p(_ptr(stream)), stream.numel(), C.byref(cfg.c()), n,
                              C.c_void_p(_ptr(re)), C.c_void_p(_ptr(im)), wp, wb, _stream()))
    torch.cuda.current_stream().synchronize()
    return re, im


def slots_to_stream(slots_host: np.ndarray, sizes_host: np.ndarray, n: int, domain: int, eb: float) -> bytes:
    """Concatenate per-chunk records into the canonical block stream (16-byte
    header + records in order).  Pure byte framing, no codec arithmetic."""
    import struct
    nch = (n + 63) // 64
    hdr = bytes([0x51, 1, domain, 6]) + struct.pack("<fII", float(np.float32(eb)), n, nch)
    parts = [hdr]
    for c in range(nch):
        parts.append(slots_host[c * SV_CHUNK_SLOT_BYTES: c * SV_CHUNK_SLOT_BYTES + int(sizes_host[c])].tobytes())
    return b"".join(parts)


# ---------------------------------------------------------------- block predictor

def mlp_forward(params, X):
    """[B][5] outputs of the block predictor for device features X [B][32]."""
    import torch
    X = X.contiguous()
    out = torch.empty((X.shape[0], 5), dtype=torch.float32, device=X.device)
    _check(lib().mlp_forward(C.c_void_p(_ptr(params)), C.c_void_p(_ptr(X)), X.shape[0],
                             C.c_void_p(_ptr(out)), _stream()))
    return out


def mlp_loss_grad(params, X, y, mode):
    """(mean loss [1], gradient [SV_MLP_NPARAM]) on device tensors."""
    import torch
    B = X.shape[0]
    work = torch.empty(int(lib().mlp_work_floats(B)), dtype=torch.float32, device=X.device)
    grad = torch.empty(SV_MLP_NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    X, y, mode = X.contiguous(), y.contiguous(), mode.to(torch.int32).contiguous()
    _check(lib().mlp_loss_grad(C.c_void_p(_ptr(params)), C.c_void_p(_ptr(X)), C.c_void_p(_ptr(y)),
                               C.c_void_p(_ptr(mode)), B, C.c_void_p(_ptr(work)), C.c_void_p(_ptr(grad)),
                               C.c_void_p(_ptr(loss)), _stream()))
    return loss, grad


def mlp_adam_update(params, grad, m, v, step: int, lr: float):
    _check(lib().mlp_adam_update(C.c_void_p(_ptr(params)), C.c_void_p(_ptr(grad)), C.c_void_p(_ptr(m)),
                                 C.c_void_p(_ptr(v)), step, float(lr), _stream()))


def predict_bytes(params, plan: "Plan"):
    """mlp_predict_bytes: predicted stream bytes after every stage of plan,
    from |0...0> (numpy float64 array, one entry per stage)."""
    import torch
    need = C.c_uint64()
    _check(lib().mlp_predict_work(plan.h, C.byref(need)))
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=params.device)
    off = (-_ptr(ws)) % 256
    ns = plan.n_stages
    out = np.zeros(max(1, ns), dtype=np.float64)
    _check(lib().mlp_predict_bytes(C.c_void_p(_ptr(params)), plan.h, C.c_void_p(_ptr(ws) + off), int(need.value),
                                   C.c_void_p(out.ctypes.data), _stream()))
    return out[:ns]


def admit(cfgs, peak_bytes, margin: float, budget: int):
    """sv_admit: (admitted flags, pool bytes, arena bytes) per configuration;
    peak_bytes None = worst-case pools (no predictor)."""
    n = len(cfgs)
    arr = (sv_config_t * max(1, n))(*[c.c() for c in cfgs])
    adm = np.zeros(max(1, n), dtype=np.uint8)
    pools = np.zeros(max(1, n), dtype=np.uint64)
    arenas = np.zeros(max(1, n), dtype=np.uint64)
    pk = None if peak_bytes is None else np.ascontiguousarray(peak_bytes, dtype=np.float64)
    _check(lib().sv_admit(C.cast(arr, C.c_void_p), n, C.c_void_p(pk.ctypes.data) if pk is not None else None,
                          float(margin), int(budget), C.c_void_p(adm.ctypes.data), C.c_void_p(pools.ctypes.data),
                          C.c_void_p(arenas.ctypes.data)))
    return adm[:n].astype(bool), pools[:n], arenas[:n]


class Predictor:
    """Block-size / mode predictor trained online (device parameters and Adam
    moments; every step runs in the library's kernels)."""

    def __init__(self, params_host: np.ndarray, device: str = "cuda:0", lr: float = 1e-3):
        import torch
        self.params = torch.from_numpy(np.asarray(params_host, dtype=np.float32).copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.lr = lr

    def predict(self, X):
        return mlp_forward(self.params, X)

    def train_step(self, X, y, mode):
        loss, grad = mlp_loss_grad(self.params, X, y, mode)
        self.step += 1
        mlp_adam_update(self.params, grad, self.m, self.v, self.step, self.lr)
        return loss
