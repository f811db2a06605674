"""Seeded synthetic circuit generators.

This module only draws random numbers and lists gates: it holds none of the
method's arithmetic (no gate matrices, no state, no codec).  Both the CPU
oracle and the HIP path consume its output, so it is the single source of
inputs for parity tests and the benchmark.

A gate is a tuple ``(kind, qubits, params)``:

* ``kind``   -- one of :data:`GATE_KINDS`
* ``qubits`` -- tuple of qubit indices; qubit q is bit q of the amplitude
  index (qubit 0 is the least significant bit, as in the paper's update rules
  of Section 2.1).  For two-qubit gates the matrix index is
  ``2*bit(qubits[0]) + bit(qubits[1])``, the row order of the paper's 4x4
  update in Section 2.1.
* ``params`` -- tuple of angles in radians (length 0..3).

The paper evaluates on a public circuit suite that is not available here; the
families below (random U3+CZ layers, QFT on an Ry product state, QAOA on a
ring) are synthetic stand-ins with the shapes of its qft / qaoa / dense
entangling workloads.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

Gate = Tuple[str, Tuple[int, ...], Tuple[float, ...]]

# kind -> (number of qubits, number of params)
GATE_KINDS = {
    "H": (1, 0), "X": (1, 0), "Y": (1, 0), "Z": (1, 0), "S": (1, 0), "T": (1, 0),
    "RX": (1, 1), "RY": (1, 1), "RZ": (1, 1), "U3": (1, 3),
    "CX": (2, 0), "CZ": (2, 0), "CP": (2, 1), "RZZ": (2, 1),
}
# numeric codes used at the C boundary (sv_gate_t.kind)
KIND_CODE = {k: i for i, k in enumerate(
    ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U3", "CX", "CZ", "CP", "RZZ"])}


def random_layers(n: int, depth: int, seed: int, n_pairs: int = 8) -> List[Gate]:
    """Random-layer circuit: per layer U3 on every qubit (ascending q, angles
    (theta, phi, lambda) ~ U[0, 2pi) drawn per qubit in that order), then CZ on
    ``min(n_pairs, n//2)`` disjoint pairs taken from a seeded permutation."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    npairs = min(n_pairs, n // 2)
    for _ in range(depth):
        for q in range(n):
            th, ph, la = rng.uniform(0.0, 2.0 * math.pi, size=3)
            gates.append(("U3", (q,), (float(th), float(ph), float(la))))
        perm = rng.permutation(n)
        for i in range(npairs):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            gates.append(("CZ", (a, b), ()))
    return gates


def qft_on_ry(n: int, seed: int) -> Tuple[List[Gate], np.ndarray]:
    """Ry(theta_q) product state (theta_q ~ U[0, pi), ascending q) followed by
    the QFT ladder without final swaps: for t = n-1 .. 0: H(t), then
    CP(pi / 2**(t-s)) on (s, t) for s = t-1 .. 0.  Returns (gates, thetas)."""
    rng = np.random.default_rng(seed)
    thetas = rng.uniform(0.0, math.pi, size=n)
    gates: List[Gate] = [("RY", (q,), (float(thetas[q]),)) for q in range(n)]
    gates += qft_ladder(n)
    return gates, thetas


def qft_ladder(n: int) -> List[Gate]:
    gates: List[Gate] = []
    for t in range(n - 1, -1, -1):
        gates.append(("H", (t,), ()))
        for s in range(t - 1, -1, -1):
            gates.append(("CP", (s, t), (math.pi / float(2 ** (t - s)),)))
    return gates


def qaoa_ring(n: int, p: int, seed: int) -> Tuple[List[Gate], np.ndarray, np.ndarray]:
    """H on all qubits, then p layers of RZZ(gamma_l) on ring edges
    (i, i+1 mod n) for ascending i followed by RX(beta_l) on all qubits.
    gamma_1..gamma_p then beta_1..beta_p ~ U[0, pi).  Returns
    (gates, gammas, betas)."""
    rng = np.random.default_rng(seed)
    gammas = rng.uniform(0.0, math.pi, size=p)
    betas = rng.uniform(0.0, math.pi, size=p)
    gates: List[Gate] = [("H", (q,), ()) for q in range(n)]
    for l in range(p):
        for i in range(n):
            gates.append(("RZZ", (i, (i + 1) % n), (float(gammas[l]),)))
        for q in range(n):
            gates.append(("RX", (q,), (float(betas[l]),)))
    return gates, gammas, betas


def ghz(n: int) -> List[Gate]:
    """Textbook GHZ preparation: H(0) then CX(q-1, q) for q = 1..n-1."""
    return [("H", (0,), ())] + [("CX", (q - 1, q), ()) for q in range(1, n)]


def mirror(gates: Sequence[Gate]) -> List[Gate]:
    """The circuit followed by its inverse (gates reversed, each inverted), so
    the state returns to |0...0> up to a global phase.  S and T are undone by
    RZ(-pi/2) and RZ(-pi/4), which differ from their inverses by a global
    phase only."""
    inv = []
    for k, q, p in reversed(list(gates)):
        if k in ("H", "X", "Y", "Z", "CX", "CZ"):
            inv.append((k, q, ()))
        elif k in ("RX", "RY", "RZ", "CP", "RZZ"):
            inv.append((k, q, (-p[0],)))
        elif k == "U3":
            inv.append(("U3", q, (-p[0], -p[2], -p[1])))
        elif k == "S":
            inv.append(("RZ", q, (-math.pi / 2,)))
        elif k == "T":
            inv.append(("RZ", q, (-math.pi / 4,)))
        else:
            raise ValueError(k)
    return list(gates) + inv


# --------------------------------------------------------------------------
# The five workload configurations.  Each returns a dict with the circuit and
# the simulation parameters (qubits n, block qubits b, inner size, fuse width,
# codec domain and absolute error bound eb).
# --------------------------------------------------------------------------

LIN, LOG = 0, 1


def config(idx: int, n: int | None = None, **over) -> dict:
    if idx == 0:
        nn = 16 if n is None else n
        d = dict(name=f"random-{nn}q-d20", n=nn, b=min(10, nn - 2), inner=2,
                 fuse=2, domain=LIN, eb=1e-6,
                 gates=random_layers(nn, 20, 1000))
    elif idx == 1:
        nn = 30 if n is None else n
        g, th = qft_on_ry(nn, 1001)
        d = dict(name=f"qft-ry-{nn}q", n=nn, b=min(22, nn - 2), inner=2,
                 fuse=4, domain=LOG, eb=1e-5, gates=g, thetas=th)
    elif idx == 2:
        nn = 33 if n is None else n
        d = dict(name=f"random-{nn}q-d16", n=nn, b=min(24, nn - 2), inner=2,
                 fuse=5, domain=LOG, eb=1e-5,
                 gates=random_layers(nn, 16, 1002))
    elif idx == 3:
        nn = 36 if n is None else n
        g, ga, be = qaoa_ring(nn, 3, 1003)
        d = dict(name=f"qaoa-ring-{nn}q-p3", n=nn, b=min(24, nn - 2), inner=2,
                 fuse=4, domain=LOG, eb=1e-5, gates=g, gammas=ga, betas=be)
    else:
        raise ValueError("config index must be 0..3 (config 4 is batch_mix)")
    d.update(over)
    return d


def batch_mix(count: int = 512, seed0: int = 5000, nmin: int = 18, nmax: int = 26):
    """Uneven batch: circuit j uses seed seed0+j; n_j ~ U{nmin..nmax}, family
    ~ U{random, qft, qaoa}, depth d_j ~ U{8..24}; qaoa uses
    p = max(1, round(d_j/8)), qft ignores depth."""
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        nj = int(rng.integers(nmin, nmax + 1))
        fam = ["random", "qft", "qaoa"][int(rng.integers(0, 3))]
        dj = int(rng.integers(8, 25))
        s = seed0 + j
        if fam == "random":
            g = random_layers(nj, dj, s)
        elif fam == "qft":
            g, _ = qft_on_ry(nj, s)
        else:
            g, _, _ = qaoa_ring(nj, max(1, int(round(dj / 8))), s)
        out.append(dict(name=f"{fam}-{nj}q", n=nj, family=fam, depth=dj, gates=g))
    return out


def mlp_init_params(seed: int) -> np.ndarray:
    """Seeded initial parameters of the block predictor (32 -> 64 -> 64 -> 5):
    hidden-layer weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)) drawn layer by
    layer in row-major order, output layer and biases zero (so the untrained
    predictor says "same size as now, all modes equally likely"); float32,
    packed W1 b1 W2 b2 W3 b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 32), (64, 64)):
        lim = math.sqrt(6.0 / cols)
        parts.append(rng.uniform(-lim, lim, size=rows * cols))
        parts.append(np.zeros(rows))
    parts.append(np.zeros(5 * 64 + 5))
    return np.concatenate(parts).astype(np.float32)


def count_gates(gates: Sequence[Gate]) -> int:
    return len(gates)
