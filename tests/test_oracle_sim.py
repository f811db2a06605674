"""Pins for the FP64 simulator oracle (CPU only).

Every check ties the oracle to something other than itself: textbook gate
matrices, closed-form states (GHZ, QFT of a basis state and of an Ry product
state, QAOA ring amplitudes by a transfer matrix), brute-force Kronecker
unitaries, norm preservation and the mirror echo U^dagger U |0> = |0>.
The C and numpy simulators are two independent codings of the paper's
update rules (Section 2.1) and must also agree with each other.
"""
import math

import numpy as np
import pytest

from oracle import native as N
from oracle import sim
from paper_2410_14088_amd import circuits as C

ALL_KINDS = [("H", 1, 0), ("X", 1, 0), ("Y", 1, 0), ("Z", 1, 0), ("S", 1, 0), ("T", 1, 0),
             ("RX", 1, 1), ("RY", 1, 1), ("RZ", 1, 1), ("U3", 1, 3),
             ("CX", 2, 0), ("CZ", 2, 0), ("CP", 2, 1), ("RZZ", 2, 1)]


def mixed_circuit(n, m, seed):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(m):
        k, nq, npar = ALL_KINDS[rng.integers(len(ALL_KINDS))]
        q = tuple(int(x) for x in rng.choice(n, nq, replace=False))
        p = tuple(float(x) for x in rng.uniform(0, 2 * math.pi, npar))
        gates.append((k, q, p))
    return gates


def test_gate_matrices_unitary_and_textbook():
    for k, nq, npar in ALL_KINDS:
        p = tuple(np.linspace(0.3, 1.1, npar))
        u = sim.gate_matrix(k, p)
        assert np.allclose(u.conj().T @ u, np.eye(2 ** nq), atol=1e-14)
        # the C oracle builds its own matrices
        assert np.allclose(N.gate_matrix(k, p), u, atol=1e-15)
    h = sim.gate_matrix("H")
    assert np.allclose(h @ np.array([1, 0]), np.array([1, 1]) / math.sqrt(2))
    # CX with control q0 = index bit 1, target q1 = index bit 0: |10> -> |11>
    cx = sim.gate_matrix("CX")
    assert np.allclose(cx @ np.array([0, 0, 1, 0]), np.array([0, 0, 0, 1]))
    assert np.allclose(sim.gate_matrix("RZZ", (0.7,)),
                       np.diag(np.exp(-0.35j * np.array([1, -1, -1, 1]))))


def test_qubit_is_index_bit():
    # X on qubit 2 of |0..0> sets amplitude index 4 (paper: qubit k <-> bit k)
    st = N.simulate(4, [("X", (2,), ())])
    assert abs(st[4] - 1) < 1e-15 and np.sum(np.abs(st) ** 2) == pytest.approx(1)
    # CX(control 0, target 3) on |0001> gives |1001>
    st = N.simulate(4, [("X", (0,), ()), ("CX", (0, 3), ())])
    assert abs(st[9] - 1) < 1e-15


def test_c_and_numpy_simulators_agree_with_kronecker_bruteforce():
    n = 6
    g = mixed_circuit(n, 60, 11)
    a = N.simulate(n, g)
    b = sim.simulate(n, g)
    U = sim.dense_unitary(n, g)
    e0 = np.zeros(2 ** n, dtype=complex)
    e0[0] = 1
    c = U @ e0
    assert np.abs(a - b).max() < 1e-13
    assert np.abs(a - c).max() < 1e-13
    assert np.allclose(U.conj().T @ U, np.eye(2 ** n), atol=1e-12)


def test_ghz_closed_form():
    for n in (3, 8, 14):
        st = N.simulate(n, C.ghz(n))
        assert np.abs(st - sim.ghz_state(n)).max() < 1e-15


def test_qft_of_basis_state_closed_form():
    n = 7
    for x in (0, 1, 37, 127):
        prep = [("X", (q,), ()) for q in range(n) if (x >> q) & 1]
        st = sim.simulate(n, prep + C.qft_ladder(n))
        assert np.abs(st - sim.qft_basis_state(n, x)).max() < 1e-13


def test_qft_ry_closed_form():
    n = 10
    g, th = C.qft_on_ry(n, 1001)
    st = N.simulate(n, g)
    assert np.abs(st - sim.qft_ry_state(n, th)).max() < 1e-13
    assert np.abs(st - N.qft_ry_state(n, th)).max() < 1e-13
    idx = np.array([0, 5, 513, 1023], dtype=np.uint64)
    assert np.abs(N.qft_ry_amplitudes(n, th, idx) - st[idx.astype(np.int64)]).max() < 1e-13


def test_qaoa_ring_transfer_matrix_and_symmetries():
    n = 8
    g, ga, be = C.qaoa_ring(n, 3, 1003)
    st = N.simulate(n, g)
    amps = np.array([sim.qaoa_ring_amplitude(n, ga, be, x) for x in range(2 ** n)])
    assert np.abs(st - amps).max() < 1e-13
    full = 2 ** n - 1
    x = np.arange(2 ** n)
    assert np.abs(st - st[full ^ x]).max() < 1e-13            # global bit flip
    rot = ((x << 1) | (x >> (n - 1))) & full                   # cyclic shift
    assert np.abs(st - st[rot]).max() < 1e-13


def test_norm_preserved_and_mirror_echo():
    n = 12
    g = mixed_circuit(n, 200, 5)
    st = N.simulate(n, g)
    assert abs(np.vdot(st, st).real - 1) < 1e-12
    back = N.apply_circuit(st, n, sim.inverse_circuit(g))
    assert abs(back[0] - 1) < 1e-12 and np.abs(back[1:]).max() < 1e-12


def test_overlap_and_fidelity():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    b = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    ov, na, nb, mx = N.overlap(a, b)
    assert abs(ov - np.vdot(a, b)) < 1e-10
    assert na == pytest.approx(np.vdot(a, a).real)
    assert mx == pytest.approx(max(np.abs(a.real - b.real).max(), np.abs(a.imag - b.imag).max()))
    assert sim.fidelity2(a, 2j * a) == pytest.approx(1.0)
    ov32, *_ = N.overlap(a, b.astype(np.complex64))
    assert abs(ov32 - np.vdot(a, b.astype(np.complex64))) < 1e-5


def test_swapped_two_qubit_convention_is_detected():
    # a plausible mistake (reading the 4x4 index as 2*bit(q1)+bit(q0)) changes
    # the result; the Kronecker brute force catches it
    n = 4
    g = [("H", (0,), ()), ("CX", (0, 2), ())]
    good = sim.dense_unitary(n, g)[:, 0]
    swapped = sim.dense_unitary(n, [("H", (0,), ()), ("CX", (2, 0), ())])[:, 0]
    assert np.abs(N.simulate(n, g) - good).max() < 1e-14
    assert np.abs(good - swapped).max() > 0.1


def test_generators_deterministic():
    a = C.random_layers(16, 20, 1000)
    b = C.random_layers(16, 20, 1000)
    assert a == b and len(a) == 20 * (16 + 8)
    g, th = C.qft_on_ry(30, 1001)
    assert len(g) == 30 + 30 + 30 * 29 // 2 and th.min() >= 0 and th.max() < math.pi
    gq, _, _ = C.qaoa_ring(36, 3, 1003)
    assert len(gq) == 36 + 3 * 72
    # the paper's 33-qubit QFT count: 33 H + 528 controlled phases; with each
    # controlled phase decomposed into 5 basic gates this is the 2,673 gates
    # it quotes in Section 4.1
    assert len(C.qft_ladder(33)) == 33 + 528 and 33 + 5 * 528 == 2673


def test_mirror_returns_to_zero_state():
    from paper_2410_14088_amd import circuits as C
    for gates in (C.random_layers(8, 4, seed=3), C.qft_on_ry(7, seed=4)[0], C.qaoa_ring(8, 2, seed=5)[0],
                  [("S", (0,), ()), ("T", (1,), ()), ("H", (1,), ()), ("RZZ", (0, 2), (0.3,)),
                   ("CX", (2, 0), ()), ("RX", (1,), (0.7,)), ("Y", (2,), ())]):
        n = 1 + max(q for _, qs, _ in gates for q in qs)
        psi = sim.simulate(n, C.mirror(gates))
        assert abs(abs(psi[0]) - 1) < 1e-12
