"""Pins for the Algorithm 1 partition oracle (CPU only).

* invariants of Algorithm 1 (Section 4.1): the stages concatenate to the
  circuit in order, none is empty, each touches at most max(inner, 2) global
  indices, and each is maximal (its successor's first gate would overflow it);
* a brute-force greedy written differently (by trying every cut point);
* the SV-group structure of the Fig. 5 example (n = 6, b = 2, inner {3, 5},
  outer {2, 4}: 4 groups of 4 blocks);
* the paper's central claim that groups are independent: simulating every
  group of every stage as a separate small state reproduces the full
  simulation exactly;
* the same for the diagonal-free variant: a diagonal gate on an outer index
  acts inside each group as a phase fixed by that group's outer bits, and
  every non-diagonal gate of a stage stays within the group's qubits.
"""
import numpy as np
import pytest

from oracle import planner as P
from oracle import sim
from paper_2410_14088_amd import circuits as C


def circuits():
    yield C.random_layers(10, 6, 3), 10
    yield C.qft_on_ry(10, 4)[0], 10
    yield C.qaoa_ring(10, 2, 5)[0], 10
    yield C.ghz(10), 10


@pytest.mark.parametrize("b", [3, 5, 7])
@pytest.mark.parametrize("inner", [0, 2, 3, 4])
def test_alg1_invariants(b, inner):
    T = max(inner, 2)
    for gates, n in circuits():
        st = P.partition(gates, b, inner)
        assert st[0][0] == 0 and st[-1][1] == len(gates)
        for (a0, a1), (b0, b1) in zip(st, st[1:]):
            assert a1 == b0
        for s0, s1 in st:
            assert s1 > s0
            assert len(P.inner_indices(gates, (s0, s1), b)) <= T
        for (s0, s1), (t0, _) in zip(st, st[1:]):
            g = set(P.inner_indices(gates, (s0, s1), b)) | P.global_qubits(gates[t0][1], b)
            assert len(g) > T                      # maximal: next gate overflows


def brute_partition(gates, b, T):
    """Greedy by exhaustive search of the longest admissible next stage."""
    out, i = [], 0
    while i < len(gates):
        best = i + 1
        for j in range(i + 1, len(gates) + 1):
            g = set()
            for _, q, _ in gates[i:j]:
                g |= {x for x in q if x >= b}
            if len(g) <= T:
                best = j
            else:
                break
        out.append((i, best))
        i = best
    return out


def test_alg1_matches_bruteforce_greedy():
    for gates, n in circuits():
        for b in (2, 4, 6):
            for inner in (1, 2, 3):
                assert P.partition(gates, b, inner) == brute_partition(gates, b, max(inner, 2))


def test_fig5_group_structure():
    n, b = 6, 2
    gr = P.groups(n, b, [3, 5])
    assert len(gr) == 4 and all(len(g) == 4 for g in gr)
    allb = sorted(x for g in gr for x in g)
    assert allb == list(range(16))
    for g in gr:
        # blocks of a group agree on the outer indices 2 and 4 (block bits 0, 2)
        outer = {((blk >> 0) & 1, (blk >> 2) & 1) for blk in g}
        assert len(outer) == 1


def simulate_by_groups(n, b, inner_size, gates):
    psi = np.zeros(2 ** n, dtype=complex)
    psi[0] = 1
    for s in P.partition(gates, b, inner_size):
        inner = P.inner_indices(gates, s, b)
        m = len(inner)
        # relabel: local qubits stay, inner global qubit inner[i] -> b + i
        relabel = {q: q for q in range(b)}
        relabel.update({q: b + i for i, q in enumerate(inner)})
        sub_gates = [(k, tuple(relabel[x] for x in q), p) for k, q, p in gates[s[0]:s[1]]]
        for blocks in P.groups(n, b, inner):
            idx = np.concatenate([np.arange(2 ** b) + (blk << b) for blk in blocks])
            sub = sim.simulate(b + m, sub_gates, psi[idx])
            psi[idx] = sub
    return psi


@pytest.mark.parametrize("inner", [2, 3])
def test_groups_are_independent(inner):
    n, b = 8, 4
    for gates in (C.random_layers(n, 3, 8), C.qft_on_ry(n, 2)[0], C.qaoa_ring(n, 2, 1)[0]):
        ref = sim.simulate(n, gates)
        got = simulate_by_groups(n, b, inner, gates)
        assert np.abs(ref - got).max() < 1e-12


def simulate_by_groups_diag_free(n, b, inner_size, gates):
    """Groups of the diagonal-free partition simulated one by one: diagonal
    gates as phases read off each amplitude's full index (outer bits
    included), every other gate on the group's relabelled qubits only (a
    non-diagonal gate on an outer index has no relabelling and fails)."""
    psi = np.zeros(2 ** n, dtype=complex)
    psi[0] = 1
    for s in P.partition(gates, b, inner_size, diag_free=True):
        inner = P.inner_indices(gates, s, b, diag_free=True)
        relabel = {q: q for q in range(b)}
        relabel.update({q: b + i for i, q in enumerate(inner)})
        for blocks in P.groups(n, b, inner):
            idx = np.concatenate([np.arange(2 ** b) + (blk << b) for blk in blocks])
            sub = psi[idx].copy()
            for k, q, p in gates[s[0]:s[1]]:
                if k in P.DIAGONAL:
                    d = np.diag(sim.gate_matrix(k, p))
                    sel = (idx >> q[0]) & 1 if len(q) == 1 else 2 * ((idx >> q[0]) & 1) + ((idx >> q[1]) & 1)
                    sub = sub * d[sel]
                else:
                    sub = sim.simulate(b + len(inner), [(k, tuple(relabel[x] for x in q), p)], sub)
            psi[idx] = sub
    return psi


@pytest.mark.parametrize("inner", [2, 3])
def test_diagonal_free_groups_are_independent(inner):
    n, b = 8, 4
    for gates in (C.random_layers(n, 3, 8), C.qft_on_ry(n, 2)[0], C.qaoa_ring(n, 2, 1)[0],
                  C.qaoa_ring(n, 1, 4)[0] + C.qft_on_ry(n, 3)[0]):
        assert len(P.partition(gates, b, inner, diag_free=True)) <= len(P.partition(gates, b, inner))
        ref = sim.simulate(n, gates)
        got = simulate_by_groups_diag_free(n, b, inner, gates)
        assert np.abs(ref - got).max() < 1e-12


def test_diagonal_free_groups_catch_a_misread_gate():
    # reading H as diagonal (a plausible slip) lets it onto outer indices and
    # the group decomposition no longer reproduces the circuit
    n, b = 8, 4
    gates = C.qft_on_ry(n, 2)[0]
    saved = set(P.DIAGONAL)
    try:
        P.DIAGONAL.add("H")
        got = simulate_by_groups_diag_free(n, b, 2, gates)
        assert np.abs(sim.simulate(n, gates) - got).max() > 1e-2
    finally:
        P.DIAGONAL.clear()
        P.DIAGONAL.update(saved)


# ---------------------------------------------------------------- commutation
def _flat(stages):
    return [i for st in stages for i in st]


def _commute_cases():
    n = 8
    yield n, C.random_layers(n, 4, 21)
    yield n, C.qft_on_ry(n, 6)[0]
    yield n, C.qaoa_ring(n, 2, 8)[0]
    yield n, C.mirror(C.random_layers(n, 3, 22))
    yield n, C.ghz(n) + C.qft_ladder(n)


@pytest.mark.parametrize("diag_free", [False, True])
@pytest.mark.parametrize("inner", [2, 3])
def test_commute_partition_reorders_validly(inner, diag_free):
    b = 4
    for n, gates in _commute_cases():
        stages = P.partition_commute(gates, b, inner, diag_free)
        order = _flat(stages)
        assert sorted(order) == list(range(len(gates))) and all(stages)
        for st in stages:
            glob = set()
            for i in st:
                glob |= P.pairing_globals(gates[i], b, diag_free)
            assert len(glob) <= max(inner, 2)
        assert len(stages) <= len(P.partition(gates, b, inner, diag_free=diag_free))
        # the reordered circuit is the same unitary: same final state
        ref = sim.simulate(n, gates)
        assert np.abs(sim.simulate(n, [gates[i] for i in order]) - ref).max() < 1e-12
        # and its stages are independent groups (diagonal gates on outer
        # indices as phases when diag_free)
        re = [gates[i] for i in order]
        psi = np.zeros(2 ** n, dtype=complex)
        psi[0] = 1
        start = 0
        for st in stages:
            seg = re[start:start + len(st)]
            start += len(st)
            inner_q = sorted(set().union(*[P.pairing_globals(g, b, diag_free) for g in seg]))
            relabel = {q: q for q in range(b)}
            relabel.update({q: b + k for k, q in enumerate(inner_q)})
            for blocks in P.groups(n, b, inner_q):
                idx = np.concatenate([np.arange(2 ** b) + (blk << b) for blk in blocks])
                sub = psi[idx].copy()
                for k, q, p in seg:
                    if diag_free and k in P.DIAGONAL:
                        d = np.diag(sim.gate_matrix(k, p))
                        sel = (idx >> q[0]) & 1 if len(q) == 1 else 2 * ((idx >> q[0]) & 1) + ((idx >> q[1]) & 1)
                        sub = sub * d[sel]
                    else:
                        sub = sim.simulate(b + len(inner_q), [(k, tuple(relabel[x] for x in q), p)], sub)
                psi[idx] = sub
        assert np.abs(psi - ref).max() < 1e-12


def test_commute_partition_packs_random_layers():
    # a layer's single-qubit gates and disjoint CZs commute: far fewer stages
    gates = C.random_layers(12, 8, 5)
    assert len(P.partition_commute(gates, 6, 2)) * 2 < len(P.partition(gates, 6, 2))


def test_commute_test_catches_a_wrong_rule():
    # a commutation rule that lets gates sharing a qubit pass each other (a
    # plausible slip) changes the circuit: the reordered state differs
    n, b = 8, 4
    gates = C.random_layers(n, 4, 21)
    saved = P.commute
    try:
        P.commute = lambda g, h: True
        order = _flat(P.partition_commute(gates, b, 2))
        assert np.abs(sim.simulate(n, [gates[i] for i in order]) - sim.simulate(n, gates)).max() > 1e-3
    finally:
        P.commute = saved


# ---- qubit remapping (Algorithm 1 with swaps of inner and local positions)

def _unpermute(psi_out, n, phys):
    """psi(x) = psi_out(pi(x)), pi moving bit L of x to bit phys[L]."""
    x = np.arange(2 ** n, dtype=np.int64)
    y = np.zeros_like(x)
    for L, p in enumerate(phys):
        y |= ((x >> L) & 1) << p
    return psi_out[y]


def _remap_cases():
    yield C.random_layers(10, 6, 3), 10, 4
    yield C.qft_on_ry(10, 4)[0], 10, 4
    yield C.qaoa_ring(10, 2, 5)[0], 10, 4
    yield C.random_layers(9, 4, 11), 9, 3


@pytest.mark.parametrize("inner", [2, 3])
def test_remap_rewrite_is_exact(inner):
    """The physical circuit (relabelled gates plus the inserted swaps) applied
    to |0...0> equals the input circuit's state with its qubits moved to
    their final positions, to rounding (FP64 oracle simulator)."""
    for gates, n, b in _remap_cases():
        stages, out, src, phys = P.partition_remap(gates, n, b, inner)
        ref = sim.simulate(n, gates)
        got = _unpermute(sim.simulate(n, out), n, phys)
        assert np.abs(ref - got).max() < 1e-12
        # every input gate appears once, in order; swaps are CX triples
        assert [i for i in src if i >= 0] == list(range(len(gates)))
        sw = [g for g, i in zip(out, src) if i < 0]
        assert len(sw) % 3 == 0 and all(g[0] == "CX" for g in sw)
        assert sorted(phys) == list(range(n))


@pytest.mark.parametrize("inner", [2, 3])
def test_remap_stages_are_algorithm1_stages(inner):
    """Each stage of the physical circuit holds at most the threshold of
    global positions, is a valid Algorithm 1 stage (its groups are
    independent: simulating every group alone reproduces the state), and a
    stage is only closed where the next gate would overflow it."""
    T = max(inner, 2)
    for gates, n, b in _remap_cases():
        stages, out, src, phys = P.partition_remap(gates, n, b, inner)
        assert stages[0][0] == 0 and stages[-1][1] == len(out)
        assert all(s[0] < s[1] for s in stages)
        assert all(a[1] == c[0] for a, c in zip(stages, stages[1:]))
        for s in stages:
            assert len(P.inner_indices(out, s, b)) <= T
        for s, t in zip(stages, stages[1:]):
            # the gate that opened the next stage (after the swaps) overflows this one
            nxt = out[t[0]]
            assert len(set(P.inner_indices(out, s, b)) | P.global_qubits(nxt[1], b)) > T
        psi = np.zeros(2 ** n, dtype=complex)
        psi[0] = 1
        for s in stages:
            inner_q = P.inner_indices(out, s, b)
            relabel = {q: q for q in range(b)}
            relabel.update({q: b + i for i, q in enumerate(inner_q)})
            sub = [(k, tuple(relabel[x] for x in q), p) for k, q, p in out[s[0]:s[1]]]
            for blocks in P.groups(n, b, inner_q):
                idx = np.concatenate([np.arange(2 ** b) + (blk << b) for blk in blocks])
                psi[idx] = sim.simulate(b + len(inner_q), sub, psi[idx])
        assert np.abs(psi - sim.simulate(n, out)).max() < 1e-12


def test_remap_cuts_stages():
    """Fewer stages than Algorithm 1 on the QFT, the random layers and the
    QAOA ring at the configurations' shapes (counts of the planner only)."""
    for gates, n, b in ((C.qft_on_ry(20, 7)[0], 20, 12), (C.random_layers(18, 8, 2), 18, 10),
                        (C.qaoa_ring(18, 3, 4)[0], 18, 10)):
        base = len(P.partition(gates, b, 2))
        st = P.partition_remap(gates, n, b, 2)[0]
        assert len(st) < base, (len(st), base)


def test_remap_check_catches_dropped_swaps():
    """The exactness pin fails for a rewrite that relabels the gates but
    leaves the swaps out (a plausible mistake)."""
    gates, n, b = C.qft_on_ry(10, 4)[0], 10, 4
    stages, out, src, phys = P.partition_remap(gates, n, b, 2)
    assert any(i < 0 for i in src)
    broken = [g for g, i in zip(out, src) if i >= 0]
    got = _unpermute(sim.simulate(n, broken), n, phys)
    assert np.abs(sim.simulate(n, gates) - got).max() > 1e-3
