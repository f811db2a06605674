"""Circuit partition oracle (test infrastructure only).

Paper Section 4.1, Algorithm 1: the circuit is cut, in gate order, into
stages; a gate joins the current stage unless the set of global indices
(qubits >= b, the high c = n - b bits of the amplitude index) touched by
the stage plus that gate would exceed ``threshold = max(inner size, 2)``, in
which case the current stage is closed first.  The global indices a stage
touches are its *inner* indices; the other global indices are *outer*.  All
blocks that agree on the outer bits form one SV group; a stage with m inner
indices has 2^(c-m) independent groups of 2^m blocks each.

Readings where the pseudo-code is silent: "exceed" means strictly greater
than the threshold; a stage is never emitted empty; a gate that alone touches
more global indices than the threshold is rejected; gates are never
reordered.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple


# Gates whose matrix is diagonal in the computational basis (Section 2.1):
# each amplitude is multiplied by a phase fixed by its own index bits.
DIAGONAL = {"Z", "S", "T", "RZ", "CZ", "CP", "RZZ"}


def global_qubits(qubits, b: int):
    return {q for q in qubits if q >= b}


def pairing_globals(gate, b: int, diag_free: bool = False):
    """Global indices on which a gate pairs amplitudes of different blocks.
    With diag_free a diagonal gate pairs none: its phase for amplitude i
    depends on i alone, so the two-block update case of Section 3 never
    arises for it."""
    kind, q, _ = gate
    if diag_free and kind in DIAGONAL:
        return set()
    return global_qubits(q, b)


def partition(gates: Sequence, b: int, inner_size: int, per_gate: bool = False,
              diag_free: bool = False) -> List[Tuple[int, int]]:
    """Algorithm 1.  Returns stages as half-open gate index ranges.

    per_gate: the basic workflow that Section 3 describes before Algorithm 1
    (the state is decompressed, updated and recompressed once per gate), i.e.
    one stage per gate, kept for comparison.
    diag_free: diagonal gates add no global index to a stage (see
    pairing_globals)."""
    threshold = max(inner_size, 2)
    if per_gate:
        for i, (_, q, _) in enumerate(gates):
            if len(global_qubits(q, b)) > threshold:
                raise ValueError(f"gate {i} touches more than {threshold} global qubits")
        return [(i, i + 1) for i in range(len(gates))]
    stages: List[Tuple[int, int]] = []
    start = 0
    cur_globals: set = set()
    for i, gate in enumerate(gates):
        g = pairing_globals(gate, b, diag_free)
        if len(g) > threshold:
            raise ValueError(f"gate {i} touches {len(g)} global qubits > {threshold}")
        if len(cur_globals | g) > threshold:
            if i > start:                 # never emit an empty stage
                stages.append((start, i))
            start = i
            cur_globals = set()
        cur_globals |= g
    if len(gates) > start:
        stages.append((start, len(gates)))
    return stages


def commute(g, h) -> bool:
    """Sufficient commutation test: disjoint qubits, or both gates diagonal
    (diagonal matrices commute)."""
    (kg, qg, _), (kh, qh, _) = g, h
    return not set(qg) & set(qh) or (kg in DIAGONAL and kh in DIAGONAL)


def partition_commute(gates: Sequence, b: int, inner_size: int, diag_free: bool = False) -> List[List[int]]:
    """Algorithm 1 with commutation.  Each stage sweeps the remaining gates in
    input order and takes a gate when the stage's global indices stay within
    the threshold and the gate commutes with every gate this sweep has
    deferred so far (the ones it overtakes); the deferred gates are the next
    sweep.  Returns each stage as the list of input gate indices it applies,
    in order."""
    threshold = max(inner_size, 2)
    for i, gate in enumerate(gates):
        if len(pairing_globals(gate, b, diag_free)) > threshold:
            raise ValueError(f"gate {i} touches more than {threshold} global qubits")
    remaining = list(range(len(gates)))
    stages: List[List[int]] = []
    while remaining:
        stage: List[int] = []
        cur: set = set()
        deferred: List[int] = []
        for i in remaining:
            g = pairing_globals(gates[i], b, diag_free)
            if len(cur | g) <= threshold and all(commute(gates[i], gates[j]) for j in deferred):
                stage.append(i)
                cur |= g
            else:
                deferred.append(i)
        stages.append(stage)
        remaining = deferred
    return stages


NEVER = 1 << 62


def partition_remap(gates: Sequence, n: int, b: int, inner_size: int, diag_free: bool = False):
    """Algorithm 1 with qubit remapping (Section 4.1: fewer stages, so fewer
    compressions).  Logical qubit L sits at physical bit position phys[L] of
    the amplitude index (identity at the start); a gate acts on the
    positions of its qubits, and Algorithm 1 counts the global positions
    (>= b).  When the next gate would exceed the threshold, before the stage
    is closed, every inner (global) position pg of the stage, in ascending
    order, whose logical qubit L is used again is offered a swap: the local
    position l whose logical qubit is next used last (ties: the lowest l) is
    taken if that use comes strictly later than L's next use, and the stage
    ends with SWAP(l, pg) written as CX(l, pg) CX(pg, l) CX(l, pg).  Both
    positions are already in the stage (pg inner, l local), so the swap
    adds no global index, and L stays local while it is used (Belady's rule:
    keep the qubits needed soonest in the block).  The gate that closed the
    stage and all later ones are mapped through the new positions.

    Returns (stages as half-open ranges of the output gate list, the output
    gates on physical positions, the input index of each output gate (-1 for
    the swap gates), phys: logical qubit -> physical position at the end).
    The output circuit applied to |0...0> gives psi_out(pi(x)) = psi(x), pi
    moving bit L of x to bit phys[L]."""
    threshold = max(inner_size, 2)
    log_at = list(range(n))              # physical position -> logical qubit
    phys = list(range(n))                # logical qubit -> physical position
    uses = [[] for _ in range(n)]
    for i, (_, q, _) in enumerate(gates):
        for x in q:
            uses[x].append(i)

    def next_use(L, i):
        for u in uses[L]:
            if u >= i:
                return u
        return NEVER

    out, src, stages = [], [], []
    start, cur = 0, set()
    for i, (kind, q, prm) in enumerate(gates):
        gq = pairing_globals((kind, tuple(phys[x] for x in q), prm), b, diag_free)
        if len(gq) > threshold:
            raise ValueError(f"gate {i} touches {len(gq)} global qubits > {threshold}")
        if len(cur | gq) > threshold and len(out) > start:
            for pg in sorted(cur):
                nu = next_use(log_at[pg], i)
                if nu == NEVER:
                    continue
                best, best_nu = None, nu
                for l in range(b):
                    v = next_use(log_at[l], i)
                    if v > best_nu:
                        best, best_nu = l, v
                if best is None:
                    continue
                for a, c in ((best, pg), (pg, best), (best, pg)):
                    out.append(("CX", (a, c), ()))
                    src.append(-1)
                la, lg = log_at[best], log_at[pg]
                log_at[best], log_at[pg] = lg, la
                phys[lg], phys[la] = best, pg
            stages.append((start, len(out)))
            start, cur = len(out), set()
            gq = pairing_globals((kind, tuple(phys[x] for x in q), prm), b, diag_free)
        cur |= gq
        out.append((kind, tuple(phys[x] for x in q), prm))
        src.append(i)
    if len(out) > start:
        stages.append((start, len(out)))
    return stages, out, src, phys


def permute_index(x, phys):
    """pi(x): bit L of x moved to bit phys[L]."""
    y = 0
    for L, p in enumerate(phys):
        y |= ((x >> L) & 1) << p
    return y


def inner_indices(gates: Sequence, stage: Tuple[int, int], b: int, diag_free: bool = False) -> List[int]:
    s = set()
    for gate in gates[stage[0]:stage[1]]:
        s |= pairing_globals(gate, b, diag_free)
    return sorted(s)


def groups(n: int, b: int, inner: Sequence[int]) -> List[List[int]]:
    """SV groups of a stage: group g deposits its bits, in ascending order,
    into the outer global positions; within a group the blocks are ordered by
    their inner bits ascending.  Returns block ids (global index >> b)."""
    c = n - b
    inner_rel = [q - b for q in inner]
    outer_rel = [j for j in range(c) if j not in inner_rel]
    out = []
    for g in range(2 ** len(outer_rel)):
        base = 0
        for i, pos in enumerate(outer_rel):
            base |= ((g >> i) & 1) << pos
        blocks = []
        for m in range(2 ** len(inner_rel)):
            blk = base
            for i, pos in enumerate(inner_rel):
                blk |= ((m >> i) & 1) << pos
            blocks.append(blk)
        out.append(blocks)
    return out
