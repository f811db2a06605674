"""ctypes loader for the oracle's C code (test infrastructure only).

``build()`` compiles ``codec_ref.c`` and ``sim_ref.c`` with gcc into
``oracle/_build/liboracle.so``; ``lib()`` loads it, building it first only if
it is missing.  Compiled with ``-ffp-contract=off`` and no fast-math so every
float32 operation of the codec rounds exactly as written.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
DEFAULT_SO = os.path.join(BUILD, "liboracle.so")
SO = os.environ.get("ORACLE_SO") or DEFAULT_SO      # ORACLE_SO: another build (the sanitized one)
SOURCES = ["codec_ref.c", "sim_ref.c"]

_lib = None


def build(sanitize: bool = False) -> str:
    """Build liboracle.so; with sanitize, liboracle_sanitized.so with
    AddressSanitizer and UndefinedBehaviorSanitizer (load it with
    ORACLE_SO=<path> and gcc's libasan / libubsan preloaded)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    out = os.path.join(BUILD, "liboracle_sanitized.so") if sanitize else DEFAULT_SO
    tmp = out + ".tmp"
    extra = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined"] if sanitize else []
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math"] + extra + ["-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO) and SO == DEFAULT_SO:
            build()
        L = C.CDLL(SO)
        P = C.c_void_p
        L.o_log2.restype = C.c_float
        L.o_log2.argtypes = [C.c_float]
        L.o_exp2.restype = C.c_float
        L.o_exp2.argtypes = [C.c_float]
        L.o_encode_block.restype = C.c_size_t
        L.o_encode_block.argtypes = [P, P, C.c_uint64, C.c_int, C.c_double, P, C.c_size_t]
        L.o_decode_block.restype = C.c_int
        L.o_decode_block.argtypes = [P, C.c_size_t, P, P, C.c_uint64]
        L.o_encode_chunk.restype = C.c_size_t
        L.o_encode_chunk.argtypes = [P, P, C.c_int, C.c_int, C.c_float, P]
        L.o_codes.restype = None
        L.o_codes.argtypes = [P, C.c_uint64, C.c_int, C.c_double, P, P]
        L.o_log2_vec.argtypes = [P, P, C.c_uint64]
        L.o_log_decode_vec.argtypes = [P, C.c_int, P, C.c_uint64]
        L.o_step_shift.restype = C.c_int
        L.o_step_shift.argtypes = [C.c_float]
        L.o_exp2_vec.argtypes = [P, P, C.c_uint64]
        L.o_gate_matrix.restype = C.c_int
        L.o_gate_matrix.argtypes = [C.c_int, P, P]
        L.o_simulate.argtypes = [P, C.c_int, P, P, P, C.c_int64]
        L.o_apply_circuit.argtypes = [P, C.c_int, P, P, P, C.c_int64]
        L.o_overlap.argtypes = [P, P, C.c_int, C.c_int64, P]
        L.o_qft_ry_amplitudes.argtypes = [C.c_int, P, P, C.c_int64, P]
        L.o_qft_ry_state.argtypes = [C.c_int, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- codec
def log2_own(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().o_log2_vec(_p(x), _p(y), x.size)
    return y


def exp2_own(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().o_exp2_vec(_p(x), _p(y), x.size)
    return y


def step_shift(eb: float) -> int:
    """s such that the quantization step is 2^-s (largest power of two <= 2 eb)."""
    return lib().o_step_shift(float(np.float32(eb)))


def log_decode(k: np.ndarray, s: int) -> np.ndarray:
    k = np.ascontiguousarray(k, dtype=np.int32)
    y = np.empty(k.size, dtype=np.float32)
    lib().o_log_decode_vec(_p(k), s, _p(y), k.size)
    return y


def encode_block(re: np.ndarray, im: np.ndarray, domain: int, eb: float) -> bytes:
    re = np.ascontiguousarray(re, dtype=np.float32)
    im = np.ascontiguousarray(im, dtype=np.float32)
    assert re.shape == im.shape and re.ndim == 1
    n = re.size
    cap = 16 + ((n + 63) // 64) * (8 + 512) + 64
    buf = np.zeros(cap, dtype=np.uint8)
    sz = lib().o_encode_block(_p(re), _p(im), n, domain, eb, _p(buf), cap)
    if sz == 0:
        raise RuntimeError("oracle encode: buffer too small")
    return buf[:sz].tobytes()


def decode_block(stream: bytes, n: int):
    src = np.frombuffer(stream, dtype=np.uint8).copy()
    re = np.zeros(n, dtype=np.float32)
    im = np.zeros(n, dtype=np.float32)
    rc = lib().o_decode_block(_p(src), src.size, _p(re), _p(im), n)
    if rc != 0:
        raise ValueError("oracle decode: malformed stream")
    return re, im


def codes(x: np.ndarray, domain: int, eb: float):
    x = np.ascontiguousarray(x, dtype=np.float32)
    k = np.zeros(x.size, dtype=np.int32)
    fail = np.zeros(x.size, dtype=np.uint8)
    lib().o_codes(_p(x), x.size, domain, eb, _p(k), _p(fail))
    return k, fail.astype(bool)


# ---------------------------------------------------------------- simulator
def _gate_arrays(gates, kind_code):
    m = len(gates)
    kinds = np.zeros(m, dtype=np.int32)
    qs = np.zeros(2 * m, dtype=np.int32)
    ps = np.zeros(3 * m, dtype=np.float64)
    for i, (k, q, p) in enumerate(gates):
        kinds[i] = kind_code[k]
        for j, qq in enumerate(q):
            qs[2 * i + j] = qq
        for j, pp in enumerate(p):
            ps[3 * i + j] = pp
    return kinds, qs, ps


KIND_CODE = {k: i for i, k in enumerate(
    ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U3", "CX", "CZ", "CP", "RZZ"])}


def simulate(n: int, gates) -> np.ndarray:
    """FP64 state after ``gates`` applied to |0..0> (complex128, 2^n)."""
    kinds, qs, ps = _gate_arrays(gates, KIND_CODE)
    st = np.empty(2 << n, dtype=np.float64)
    lib().o_simulate(_p(st), n, _p(kinds), _p(qs), _p(ps), len(gates))
    return st.view(np.complex128)


def apply_circuit(state: np.ndarray, n: int, gates) -> np.ndarray:
    kinds, qs, ps = _gate_arrays(gates, KIND_CODE)
    st = np.ascontiguousarray(state, dtype=np.complex128).copy()
    lib().o_apply_circuit(_p(st.view(np.float64)), n, _p(kinds), _p(qs), _p(ps), len(gates))
    return st


def gate_matrix(kind: str, params) -> np.ndarray:
    p = np.zeros(3, dtype=np.float64)
    p[:len(params)] = params
    u = np.zeros(32, dtype=np.float64)
    nq = lib().o_gate_matrix(KIND_CODE[kind], _p(p), _p(u))
    m = u.view(np.complex128)
    return m[:4].reshape(2, 2).copy() if nq == 1 else m.reshape(4, 4).copy()


def overlap(a: np.ndarray, b: np.ndarray):
    """Returns (<a|b>, |a|^2, |b|^2, max componentwise |a-b|)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if b.dtype == np.complex64:
        bb, b32 = np.ascontiguousarray(b), 1
    else:
        bb, b32 = np.ascontiguousarray(b, dtype=np.complex128), 0
    out = np.zeros(5, dtype=np.float64)
    lib().o_overlap(_p(a.view(np.float64)), _p(bb), b32, a.size, _p(out))
    return complex(out[0], out[1]), out[2], out[3], out[4]


def qft_ry_amplitudes(n: int, theta: np.ndarray, idx: np.ndarray) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ix = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.zeros(2 * ix.size, dtype=np.float64)
    lib().o_qft_ry_amplitudes(n, _p(th), _p(ix), ix.size, _p(out))
    return out.view(np.complex128)


def qft_ry_state(n: int, theta: np.ndarray) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.zeros(2 << n, dtype=np.float64)
    lib().o_qft_ry_state(n, _p(th), _p(out))
    return out.view(np.complex128)
