"""CPU check of the planner's gate fusion against the oracle (no GPU).

For every stage of a plan, the stage's fused operations as the library built
them (plan_stage_ops / plan_op: complex64 dense matrices and diagonal phase
tables, in application order) are applied to a random state with numpy and
compared with the oracle's FP64 simulation of the stage's gates (in the
plan's gate order, which is the input order unless gates were reordered by
commutation).  This covers the gate matrices and their qubit convention, the
embedding of gates into fused operations, their products, the deferral of
diagonal gates past commuting gates, and the tile passes of multi-pass
stages.  Tolerance: the operations are rounded once to complex64, so the
error is a few float32 ulps of the state's scale.
"""
import numpy as np
import pytest

from oracle import sim
from paper_2410_14088_amd import circuits as C


@pytest.fixture(scope="module")
def bmq():
    import os
    from paper_2410_14088_amd import bmq as B
    if not os.path.exists(B.SO):
        from paper_2410_14088_amd import build
        build.build()
    B.lib()
    return B


def apply_op(psi, n, kind, qs, vals):
    """Operation qubit j is bit j of the operation's index."""
    k = len(qs)
    t = psi.reshape([2] * n)
    axes = [n - 1 - q for q in reversed(qs)]
    t = np.moveaxis(t, axes, list(range(n - k, n)))
    shp = t.shape
    m = t.reshape(-1, 1 << k)
    m = m @ vals.astype(complex).T if kind == "dense" else m * vals.astype(complex)[None, :]
    return np.moveaxis(m.reshape(shp), list(range(n - k, n)), axes).reshape(-1)


def circuits_for(n):
    yield "random+qft", C.random_layers(n, 3, 31) + C.qft_ladder(n)
    yield "qft-on-ry", C.config(1, n=n)["gates"]
    yield "qaoa", C.qaoa_ring(n, 2, 7)[0]
    yield "mirror", C.mirror(C.random_layers(n, 2, 32))


@pytest.mark.parametrize("flags", [0, 8, 16, 24, 64])
@pytest.mark.parametrize("fuse,tile", [(1, 10), (2, 10), (4, 10), (5, 11), (4, 12)])
def test_fused_operations_equal_the_gates(bmq, flags, fuse, tile):
    n, b = 12, 7
    rng = np.random.default_rng(fuse * 100 + tile + flags)
    for name, gates in circuits_for(n):
        cfg = bmq.Config(n=n, b=b, inner=2, fuse=fuse, domain=1, eb=1e-5, tile=tile, flags=flags)
        plan = bmq.Plan(gates, cfg)
        order = plan.gate_order()
        # with remapping the stages apply the physical circuit (relabelled
        # gates and swaps, checked against the oracle planner in test_abi)
        applied = plan.gates() if flags & bmq.SV_FLAG_REMAP else [gates[i] for i in order]
        for s in range(plan.n_stages):
            g0, g1 = plan.stage(s)["gates"]
            psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
            ref = sim.simulate(n, applied[g0:g1], psi)
            got = psi.copy()
            for kind, qs, vals in plan.stage_ops(s):
                if kind == "dense":
                    assert len(qs) <= max(fuse, 2)      # a 2-qubit gate is one operation at any width
                got = apply_op(got, n, kind, qs, vals)
            scale = np.abs(ref).max()
            err = np.abs(got - ref).max() / scale
            assert err < 2e-6, (name, s, err)


def test_fusion_check_catches_a_wrong_order(bmq):
    # applying one stage's operations in reverse order (a plausible slip in a
    # fusion that reorders gates) must fail the comparison
    n, b = 12, 7
    gates = C.random_layers(n, 3, 31) + C.qft_ladder(n)
    plan = bmq.Plan(gates, bmq.Config(n=n, b=b, inner=2, fuse=4, domain=1, eb=1e-5, tile=10))
    rng = np.random.default_rng(0)
    worst = 0.0
    for s in range(plan.n_stages):
        ops = plan.stage_ops(s)
        if len(ops) < 2:
            continue
        g0, g1 = plan.stage(s)["gates"]
        psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        ref = sim.simulate(n, gates[g0:g1], psi)
        got = psi.copy()
        for kind, qs, vals in reversed(ops):
            got = apply_op(got, n, kind, qs, vals)
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    assert worst > 1e-2
