"""FP64 numpy oracle for small states (test infrastructure only).

* :func:`gate_matrix` -- the textbook matrices of the gate set.  Qubit q is
  bit q of the amplitude index; a two-qubit matrix is indexed by
  ``2*bit(q0) + bit(q1)``, the row order of the paper's 4x4 update rule
  (Section 2.1).
* :func:`simulate` -- apply gates one by one to a tensor of shape (2,)*n with
  ``numpy.tensordot`` (a second, independent simulator beside the C one).
* :func:`dense_unitary` -- the whole circuit as one 2^n x 2^n matrix built
  from Kronecker products (brute force, n <= 10).
* closed forms: :func:`ghz_state`, :func:`qft_basis_state`,
  :func:`qft_ry_state`, :func:`qaoa_ring_amplitude` (ring transfer matrix).
* :func:`fidelity2` -- |<a|b>|^2 / (|a|^2 |b|^2); the paper reports the
  unsquared |<psi_ideal|psi_sim>| (Section 5.3).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

DIAGONAL = {"Z", "S", "T", "RZ", "CZ", "CP", "RZZ"}


def gate_matrix(kind: str, p: Sequence[float] = ()) -> np.ndarray:
    c = lambda a: math.cos(a / 2)
    s = lambda a: math.sin(a / 2)
    e = lambda a: complex(math.cos(a), math.sin(a))
    if kind == "H":
        return np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2)
    if kind == "X":
        return np.array([[0, 1], [1, 0]], dtype=complex)
    if kind == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=complex)
    if kind == "Z":
        return np.diag([1, -1]).astype(complex)
    if kind == "S":
        return np.diag([1, 1j]).astype(complex)
    if kind == "T":
        return np.diag([1, e(math.pi / 4)]).astype(complex)
    if kind == "RX":
        return np.array([[c(p[0]), -1j * s(p[0])], [-1j * s(p[0]), c(p[0])]], dtype=complex)
    if kind == "RY":
        return np.array([[c(p[0]), -s(p[0])], [s(p[0]), c(p[0])]], dtype=complex)
    if kind == "RZ":
        return np.diag([e(-p[0] / 2), e(p[0] / 2)])
    if kind == "U3":
        th, ph, la = p
        return np.array([[c(th), -e(la) * s(th)],
                         [e(ph) * s(th), e(ph + la) * c(th)]], dtype=complex)
    if kind == "CX":
        m = np.eye(4, dtype=complex)
        m[2:, 2:] = [[0, 1], [1, 0]]
        return m
    if kind == "CZ":
        return np.diag([1, 1, 1, -1]).astype(complex)
    if kind == "CP":
        return np.diag([1, 1, 1, e(p[0])])
    if kind == "RZZ":
        g = p[0]
        return np.diag([e(-g / 2), e(g / 2), e(g / 2), e(-g / 2)])
    raise ValueError(kind)


def dagger(gate):
    """Inverse of a gate as a short list of gates of the set (mirror echo):
    S^dagger = Z S, T^dagger = Z S T, U3(t,p,l)^dagger = U3(-t,-l,-p)."""
    k, q, p = gate
    if k in ("H", "X", "Y", "Z", "CX", "CZ"):
        return [(k, q, ())]
    if k == "S":
        return [("Z", q, ()), ("S", q, ())]
    if k == "T":
        return [("Z", q, ()), ("S", q, ()), ("T", q, ())]
    if k in ("RX", "RY", "RZ", "CP", "RZZ"):
        return [(k, q, (-p[0],))]
    if k == "U3":
        th, ph, la = p
        return [("U3", q, (-th, -la, -ph))]
    raise ValueError(f"no dagger form for {k}")


def inverse_circuit(gates):
    out = []
    for g in reversed(gates):
        out += dagger(g)
    return out


def apply_gate(psi: np.ndarray, n: int, kind: str, qubits, params) -> np.ndarray:
    """psi has shape (2,)*n with axis n-1-q holding qubit q."""
    u = gate_matrix(kind, params)
    k = len(qubits)
    axes = [n - 1 - q for q in qubits]
    ut = u.reshape((2,) * (2 * k))
    out = np.tensordot(ut, psi, axes=(list(range(k, 2 * k)), axes))
    # tensordot puts the gate's output axes first; move them back in place
    return np.moveaxis(out, list(range(k)), axes)


def simulate(n: int, gates, psi0: np.ndarray | None = None) -> np.ndarray:
    if psi0 is None:
        psi = np.zeros(2 ** n, dtype=complex)
        psi[0] = 1.0
    else:
        psi = np.array(psi0, dtype=complex)
    t = psi.reshape((2,) * n)
    for kind, q, p in gates:
        t = apply_gate(t, n, kind, q, p)
    return t.reshape(-1)


def embed(u: np.ndarray, qubits, n: int) -> np.ndarray:
    """The 2^n x 2^n matrix of a 1- or 2-qubit gate, built from Kronecker
    products of single-qubit operators (brute force)."""
    I2 = np.eye(2, dtype=complex)
    dim = 2 ** n
    if len(qubits) == 1:
        ops = [I2] * n
        ops[qubits[0]] = u
        m = np.array([[1.0 + 0j]])
        for q in range(n - 1, -1, -1):     # most significant qubit first
            m = np.kron(m, ops[q])
        return m
    # two-qubit: expand u = sum_{ab,cd} u[ab,cd] |a><c| (x) |b><d|
    qa, qb = qubits
    m = np.zeros((dim, dim), dtype=complex)
    for r in range(4):
        for c in range(4):
            if u[r, c] == 0:
                continue
            A = np.zeros((2, 2), dtype=complex); A[r >> 1, c >> 1] = 1
            B = np.zeros((2, 2), dtype=complex); B[r & 1, c & 1] = 1
            ops = [I2] * n
            ops[qa] = A
            ops[qb] = B
            t = np.array([[1.0 + 0j]])
            for q in range(n - 1, -1, -1):
                t = np.kron(t, ops[q])
            m += u[r, c] * t
    return m


def dense_unitary(n: int, gates) -> np.ndarray:
    U = np.eye(2 ** n, dtype=complex)
    for kind, q, p in gates:
        U = embed(gate_matrix(kind, p), q, n) @ U
    return U


def fidelity2(a: np.ndarray, b: np.ndarray) -> float:
    ov = np.vdot(a, b)
    return float(abs(ov) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))


# ------------------------------------------------------------ closed forms
def ghz_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=complex)
    psi[0] = psi[-1] = 1 / math.sqrt(2)
    return psi


def bitrev(y: np.ndarray, n: int) -> np.ndarray:
    r = np.zeros_like(y)
    for b in range(n):
        r |= ((y >> b) & 1) << (n - 1 - b)
    return r


def qft_basis_state(n: int, x: int) -> np.ndarray:
    """Swap-free QFT of |x>: psi(y) = 2^{-n/2} exp(2 pi i x rev_n(y) / 2^n)."""
    y = np.arange(2 ** n, dtype=np.int64)
    ph = 2 * np.pi * ((x * bitrev(y, n)) % (2 ** n)) / 2 ** n
    return np.exp(1j * ph) / 2 ** (n / 2)


def qft_ry_state(n: int, theta) -> np.ndarray:
    """Swap-free QFT of the product state prod_q Ry(theta_q)|0>:
    psi(y) = 2^{-n/2} prod_i (cos(t_i/2) + sin(t_i/2) e^{2 pi i 2^i rev_n(y)/2^n})."""
    y = np.arange(2 ** n, dtype=np.int64)
    rv = bitrev(y, n)
    psi = np.ones(2 ** n, dtype=complex)
    for i in range(n):
        ph = 2 * np.pi * ((rv << i) % (2 ** n)) / 2 ** n
        psi *= math.cos(theta[i] / 2) + math.sin(theta[i] / 2) * np.exp(1j * ph)
    return psi / 2 ** (n / 2)


def qaoa_ring_amplitude(n: int, gammas, betas, x: int) -> complex:
    """<x| prod_l [RX(beta_l)^n RZZring(gamma_l)] H^n |0>, by a path sum over
    Z-basis worldlines w_i in {0,1}^p at each site, contracted around the ring
    as a trace of 2^p x 2^p transfer matrices (cost O(n 8^p) per amplitude)."""
    p = len(gammas)
    W = 2 ** p
    rx = [np.array([[math.cos(b / 2), -1j * math.sin(b / 2)],
                    [-1j * math.sin(b / 2), math.cos(b / 2)]]) for b in betas]
    # bond weight between neighbouring worldlines
    B = np.zeros((W, W), dtype=complex)
    for w in range(W):
        for v in range(W):
            ang = 0.0
            for l in range(p):
                zz = 1 - 2 * (((w >> l) & 1) ^ ((v >> l) & 1))
                ang += -gammas[l] / 2 * zz
            B[w, v] = complex(math.cos(ang), math.sin(ang))
    T = np.eye(W, dtype=complex)
    for i in range(n):
        xi = (x >> i) & 1
        a = np.zeros(W, dtype=complex)
        for w in range(W):
            amp = 1.0 + 0j
            for l in range(p):
                src = (w >> l) & 1
                dst = ((w >> (l + 1)) & 1) if l + 1 < p else xi
                amp *= rx[l][dst, src]
            a[w] = amp
        T = T @ (np.diag(a) @ B)
    return complex(np.trace(T) / 2 ** (n / 2))
