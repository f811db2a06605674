"""CPU checks of the C ABI: the library loads, exports every function that
include/bmq.h declares, and its host-only planner (stage_plan) reproduces
Algorithm 1's stages from the independent oracle planner.  No GPU needed:
planning makes no HIP calls."""
import os
import re

import numpy as np
import pytest

from oracle import planner as OP
from paper_2410_14088_amd import circuits as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bmq():
    from paper_2410_14088_amd import bmq as B
    if not os.path.exists(B.SO):
        from paper_2410_14088_amd import build
        build.build()
    B.lib()
    return B


def header_functions():
    txt = open(os.path.join(ROOT, "include", "bmq.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)))


def test_exports_every_declared_symbol(bmq):
    names = header_functions()
    assert "stage_apply_compressed" in names and "sv_create" in names
    L = bmq.lib()
    for nm in names:
        assert hasattr(L, nm), f"{nm} not exported"
    assert sorted(bmq.EXPORTS) == names


@pytest.mark.parametrize("inner", [0, 2, 3, 4])
def test_planner_matches_oracle_alg1(bmq, inner):
    cases = [(C.config(0)["gates"], 16, 10), (C.config(1, n=20)["gates"], 20, 14),
             (C.qaoa_ring(16, 3, 2)[0], 16, 11), (C.random_layers(18, 5, 9), 18, 12)]
    for gates, n, b in cases:
        cfg = bmq.Config(n=n, b=b, inner=inner, fuse=4, domain=1, eb=1e-5)
        plan = bmq.Plan(gates, cfg)
        want = OP.partition(gates, b, inner)
        assert plan.n_stages == len(want)
        for s, (g0, g1) in enumerate(want):
            st = plan.stage(s)
            assert st["gates"] == (g0, g1)
            assert st["inner"] == OP.inner_indices(gates, (g0, g1), b)
            assert st["passes"] >= 1


@pytest.mark.parametrize("inner", [2, 4])
def test_gate_per_stage_plan(bmq, inner):
    # the per-gate workflow: one stage per gate, its inner indices are the
    # gate's own global qubits, and one gate per fused operation
    for gates, n, b in [(C.config(0)["gates"], 16, 10), (C.qaoa_ring(16, 2, 5)[0], 16, 12)]:
        cfg = bmq.Config(n=n, b=b, inner=inner, fuse=4, domain=1, eb=1e-5, flags=bmq.SV_FLAG_GATE_PER_STAGE)
        plan = bmq.Plan(gates, cfg)
        want = OP.partition(gates, b, inner, per_gate=True)
        assert want == [(i, i + 1) for i in range(len(gates))]
        assert plan.n_stages == len(gates)
        for s in range(0, len(gates), 7):
            st = plan.stage(s)
            assert st["gates"] == want[s]
            assert st["inner"] == sorted(q for q in gates[s][1] if q >= b)
        assert len(OP.partition(gates, b, inner)) < len(gates)     # Algorithm 1 groups gates


@pytest.mark.parametrize("inner", [0, 2, 3])
def test_diagonal_free_plan_matches_oracle(bmq, inner):
    cases = [(C.config(1, n=20)["gates"], 20, 14), (C.qaoa_ring(16, 3, 2)[0], 16, 11),
             (C.config(0)["gates"], 16, 10), (C.random_layers(18, 5, 9) + C.qft_ladder(18), 18, 12)]
    for gates, n, b in cases:
        cfg = bmq.Config(n=n, b=b, inner=inner, fuse=4, domain=1, eb=1e-5, flags=bmq.SV_FLAG_DIAGONAL_FREE)
        plan = bmq.Plan(gates, cfg)
        want = OP.partition(gates, b, inner, diag_free=True)
        assert plan.n_stages == len(want)
        for s, (g0, g1) in enumerate(want):
            st = plan.stage(s)
            assert st["gates"] == (g0, g1)
            assert st["inner"] == OP.inner_indices(gates, (g0, g1), b, diag_free=True)
        assert len(want) <= len(OP.partition(gates, b, inner))


@pytest.mark.parametrize("flags", [16, 24])
@pytest.mark.parametrize("inner", [0, 2, 3])
def test_commute_plan_matches_oracle(bmq, inner, flags):
    cases = [(C.config(0)["gates"], 16, 10), (C.qaoa_ring(16, 3, 2)[0], 16, 11),
             (C.mirror(C.random_layers(18, 5, 9)), 18, 12), (C.config(1, n=20)["gates"], 20, 14)]
    for gates, n, b in cases:
        cfg = bmq.Config(n=n, b=b, inner=inner, fuse=4, domain=1, eb=1e-5, flags=flags)
        plan = bmq.Plan(gates, cfg)
        want = OP.partition_commute(gates, b, inner, diag_free=bool(flags & bmq.SV_FLAG_DIAGONAL_FREE))
        assert plan.n_stages == len(want)
        order = plan.gate_order()
        assert sorted(order) == list(range(len(gates)))
        for s, st_want in enumerate(want):
            g0, g1 = plan.stage(s)["gates"]
            assert order[g0:g1] == st_want
            assert plan.stage(s)["inner"] == sorted(set().union(
                *[OP.pairing_globals(gates[i], b, bool(flags & 8)) for i in st_want]))
    # without the flag the plan order is the input order
    plan = bmq.Plan(C.config(0)["gates"], bmq.Config(n=16, b=10))
    assert plan.gate_order() == list(range(len(C.config(0)["gates"])))


@pytest.mark.parametrize("flags", [64, 72])
@pytest.mark.parametrize("inner", [2, 3])
def test_remap_plan_matches_oracle(bmq, inner, flags):
    """SV_FLAG_REMAP: the host planner's stages, physical gates, input
    indices and final layout equal the oracle planner's partition_remap."""
    cases = [(C.config(0)["gates"], 16, 10), (C.qaoa_ring(16, 3, 2)[0], 16, 11),
             (C.config(1, n=20)["gates"], 20, 12), (C.random_layers(18, 6, 9), 18, 12)]
    for gates, n, b in cases:
        cfg = bmq.Config(n=n, b=b, inner=inner, fuse=4, domain=1, eb=1e-5, flags=flags)
        plan = bmq.Plan(gates, cfg)
        stages, out, src, phys = OP.partition_remap(gates, n, b, inner, diag_free=bool(flags & 8))
        assert plan.n_stages == len(stages)
        assert [plan.stage(s)["gates"] for s in range(plan.n_stages)] == stages
        got = plan.gates()
        assert [(k, q) for k, q, _ in got] == [(k, tuple(q)) for k, q, _ in out]
        assert all(np.allclose(a[2][:len(b_[2])], b_[2]) for a, b_ in zip(got, out))
        assert plan.gate_order() == [i if i >= 0 else 0xFFFFFFFF for i in src]
        assert plan.layout() == phys
        assert [plan.stage(s)["inner"] for s in range(plan.n_stages)] == \
            [OP.inner_indices(out, st, b, bool(flags & 8)) for st in stages]
    # fewer stages than Algorithm 1 on the QFT
    g = C.config(1, n=20)["gates"]
    assert bmq.Plan(g, bmq.Config(n=20, b=12, flags=64)).n_stages < bmq.Plan(g, bmq.Config(n=20, b=12)).n_stages
    for bad in (64 | 16, 64 | 4):
        with pytest.raises(bmq.BmqError):
            bmq.Plan(g, bmq.Config(n=20, b=12, flags=bad))


def test_diagonal_free_partition_pins():
    # a circuit of diagonal gates only is one stage, whatever qubits it
    # touches; a non-diagonal gate on a third global qubit still cuts
    b = 8
    diag = [("CP", (9, 12), (0.3,)), ("RZZ", (10, 11), (0.2,)), ("CZ", (8, 13), ()), ("T", (14,), ())]
    assert OP.partition(diag, b, 2, diag_free=True) == [(0, 4)]
    assert len(OP.partition(diag, b, 2)) == 4
    mix = [("H", (9,), ()), ("CP", (9, 12), (0.3,)), ("H", (10,), ()), ("RZZ", (11, 13), (0.1,)), ("X", (11,), ())]
    assert OP.partition(mix, b, 2, diag_free=True) == [(0, 4), (4, 5)]
    assert OP.inner_indices(mix, (0, 4), b, diag_free=True) == [9, 10]
    # the QFT's phase ladders are diagonal: 30 qubits on 2^22 blocks go from
    # dozens of stages to a handful
    d = C.config(1, n=30)
    assert len(OP.partition(d["gates"], 22, 2, diag_free=True)) <= 8 < len(OP.partition(d["gates"], 22, 2))


def test_config_stage_counts(bmq):
    d = C.config(0)
    assert bmq.Plan(d["gates"], bmq.Config(n=16, b=10)).n_stages == len(OP.partition(d["gates"], 10, 2))


@pytest.mark.parametrize("bad", [dict(n=9), dict(n=41), dict(b=5), dict(b=17), dict(fuse=0),
                                 dict(fuse=6), dict(domain=3), dict(domain=-1), dict(eb=0.0), dict(eb=-1.0),
                                 dict(tile=9), dict(tile=14), dict(eb=float("nan")), dict(flags=128),
                                 dict(flags=0x80000000)])
def test_invalid_configs_rejected(bmq, bad):
    kw = dict(n=16, b=10, inner=2, fuse=2, domain=0, eb=1e-6)
    kw.update(bad)
    with pytest.raises(bmq.BmqError) as e:
        bmq.Plan(C.ghz(16), bmq.Config(**kw))
    assert e.value.code == -1


def test_invalid_gates_rejected(bmq):
    cfg = bmq.Config(n=12, b=8)
    for g in ([("CX", (3, 3), ())], [("H", (12,), ())], [("X", (-1,), ())]):
        with pytest.raises(bmq.BmqError):
            bmq.Plan(g, cfg)


def test_no_scratch_flag_shrinks_the_arena(bmq):
    import ctypes as C_
    need = []
    for flags in (0, bmq.SV_FLAG_NO_SCRATCH):
        v = C_.c_uint64()
        bmq._check(bmq.lib().sv_mem_required(C_.byref(bmq.Config(n=24, b=16, flags=flags).c()), C_.byref(v)))
        need.append(v.value)
    assert need[0] - need[1] >= 2 * 4 * (1 << 24)       # two float32 scratch planes


def test_plan_views_reject_bad_arguments(bmq):
    import ctypes as C_
    L = bmq.lib()
    gates = C.config(0)["gates"]
    plan = bmq.Plan(gates, bmq.Config(n=16, b=10, flags=bmq.SV_FLAG_COMMUTE))
    order = (C_.c_uint32 * len(gates))()
    assert L.plan_gate_order(plan.h, order, len(gates) - 1) == -1          # wrong length
    assert L.plan_gate_order(None, order, len(gates)) == -1
    assert L.plan_gate_order(plan.h, order, len(gates)) == 0
    assert sorted(order) == list(range(len(gates)))
    b, e = C_.c_size_t(), C_.c_size_t()
    assert L.plan_stage_ops(plan.h, plan.n_stages, C_.byref(b), C_.byref(e)) == -1
    assert L.plan_stage_ops(plan.h, 0, C_.byref(b), C_.byref(e)) == 0 and e.value > b.value
    n_ops = plan.info()["ops"]
    t, k = C_.c_int32(), C_.c_int32()
    assert L.plan_op(plan.h, n_ops, C_.byref(t), C_.byref(k), None, None, 0) == -1
    assert L.plan_op(plan.h, 0, C_.byref(t), C_.byref(k), None, None, 0) == 0
    small = (C_.c_float * 2)()
    assert k.value >= 1 and L.plan_op(plan.h, 0, None, None, None, small, 1) == -1   # capacity below 2^k values
    # the state-level views refuse a NULL handle without touching a device
    nb = C_.c_uint64()
    assert L.sv_check(None, C_.byref(nb)) == -1
    ptr, n = C_.c_void_p(), C_.c_uint64()
    assert L.sv_directory(None, C_.byref(ptr), C_.byref(n)) == -1
    # exact pinned host allocations: bad arguments are refused before any
    # HIP call and leave the output untouched; freeing NULL does nothing
    p = C_.c_void_p(1)
    assert L.sv_host_alloc(0, C_.byref(p)) == -1 and p.value == 1
    assert L.sv_host_alloc(64, None) == -1
    assert L.sv_host_free(None) == 0


def test_admission_under_a_budget(bmq):
    """sv_admit (host only): worst-case pools without a predictor; predicted
    peaks shrink the pools (never beyond the worst case), so more circuits
    fit the same budget; first fit in order."""
    cfgs = [bmq.Config(n=n, b=n - 8, domain=1, eb=1e-5, flags=bmq.SV_FLAG_NO_SCRATCH) for n in (24, 25, 24, 23, 24, 23)]
    big = 1 << 62
    adm, pools, arenas = bmq.admit(cfgs, None, 0.1, big)
    assert adm.all()
    need = [bmq.C.c_uint64() for _ in cfgs]
    for c, x in zip(cfgs, need):
        bmq._check(bmq.lib().sv_mem_required(bmq.C.byref(c.c()), bmq.C.byref(x)))
    assert list(arenas) == [x.value for x in need]              # worst case = the default arena
    peaks = [0.7 * (8 << c.n) for c in cfgs]                   # a compression ratio of about 1.4
    adm_p, pools_p, arenas_p = bmq.admit(cfgs, peaks, 0.1, big)
    assert (pools_p < pools).all() and (arenas_p < arenas).all()
    budget = int(arenas[:3].sum())
    adm_w = bmq.admit(cfgs, None, 0.1, budget)[0]
    adm_p = bmq.admit(cfgs, peaks, 0.1, budget)[0]
    assert adm_w.sum() == 3 and adm_p.sum() > adm_w.sum()
    huge = [64.0 * (8 << c.n) for c in cfgs]                   # capped at the worst case
    assert (bmq.admit(cfgs, huge, 0.1, big)[1] == pools).all()
    with pytest.raises(bmq.BmqError):
        bmq.admit(cfgs, peaks, -1.0, big)
