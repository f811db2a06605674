"""Persistent multi-stage launch (sv_persistent_apply) on the GPU.

One launch per tile size runs every stage of every circuit: workgroups take
(pass, tile) items from a device queue and a tile waits for its circuit's
previous pass through an atomic done-counter.  It must leave every state with
exactly the records of the per-pass launches, for one circuit and for a mix,
with multi-pass stages, without scratch planes and with records in the host
pool.  The bounded wait is exercised from the host with a tiny limit: the
launch then aborts, finishes, reports SV_ERR_TIMEOUT and poisons its states,
and the device keeps working."""
import time

import numpy as np
import pytest

from oracle import native as N

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"
LIMIT_US = 5_000_000          # any wait longer than this aborts the launch (and fails the test)


def _make(d, **kw):
    cfg = bmq.Config(n=d["n"], b=d["b"], inner=d.get("inner", 2), fuse=d["fuse"], domain=d["domain"], eb=d["eb"],
                     tile=d.get("tile", 0), **kw)
    return bmq.Plan(d["gates"], cfg), bmq.State(cfg, DEV)


def _same(a, b, tag):
    # record and directory bytes (where the records live may differ)
    fa, fb = a.footprint(), b.footprint()
    assert (fa[0], fa[2]) == (fb[0], fb[2]), tag
    for k in range(a.n_blocks):
        assert a.block_stream(k) == b.block_stream(k), (tag, k)


def _qft(n, tile, **kw):
    g, _ = C.qft_on_ry(n, 1001)
    return dict(gates=g, n=n, b=n - 4, fuse=4, domain=1, eb=1e-5, tile=tile, **kw)


def test_single_circuit_equals_per_pass_launches():
    d = C.config(0)
    d = dict(gates=d["gates"], n=d["n"], b=d["b"], fuse=d["fuse"], domain=d["domain"], eb=d["eb"])
    p, s = _make(d)
    s.apply(p)
    p2, s2 = _make(d)
    print("persistent: 16-qubit random layers, LIN", flush=True)
    bmq.persistent_apply([s2], [p2], wait_limit_us=LIMIT_US)
    _same(s, s2, "random-16")
    ref = torch.from_numpy(np.ascontiguousarray(N.simulate(d["n"], d["gates"]))).to(DEV)
    f2, _, _ = s2.fidelity(ref)
    assert f2 >= 0.99


@pytest.mark.parametrize("flags", [0, 1])
def test_multi_pass_stages(flags):
    # 18-qubit QFT on 2^10-amplitude tiles: the ladder stages need several
    # passes (through the scratch planes, or recompressed without them)
    d = _qft(18, 10)
    p, s = _make(d, flags=flags)
    stats = s.apply(p, stats=True)
    assert max(x["passes"] for x in stats) > 1
    p2, s2 = _make(d, flags=flags)
    print(f"persistent: 18-qubit QFT, tile 10, flags {flags}", flush=True)
    bmq.persistent_apply([s2], [p2], wait_limit_us=LIMIT_US)
    _same(s, s2, f"qft-18-flags{flags}")


def test_mix_of_circuits_and_tile_sizes():
    mix = []
    for j, d in enumerate(C.batch_mix(10, seed0=7100, nmin=12, nmax=16)):
        mix.append(dict(gates=d["gates"], n=d["n"], b=d["n"] - 4, domain=j % 2, eb=1e-5 if j % 2 else 1e-6,
                        fuse=2 + j % 4, tile=10 if j % 3 == 0 else 0))
    mix.append(dict(gates=C.ghz(14), n=14, b=8, domain=1, eb=1e-5, fuse=2, tile=0))
    eager, states, plans = [], [], []
    for d in mix:
        p, s = _make(d)
        s.apply(p)
        eager.append(s)
        p2, s2 = _make(d)
        plans.append(p2)
        states.append(s2)
    print(f"persistent: mix of {len(mix)} circuits, tiles 10 and 12", flush=True)
    bmq.persistent_apply(states, plans, wait_limit_us=LIMIT_US)
    for i, (a, b) in enumerate(zip(eager, states)):
        _same(a, b, f"mix-{i}")
    # a second call continues from the current state
    for a, p in zip(eager[:3], plans[:3]):
        a.apply(p)
    bmq.persistent_apply(states[:3], plans[:3], wait_limit_us=LIMIT_US)
    for i in range(3):
        _same(eager[i], states[i], f"again-{i}")


def test_host_pool_records():
    d = C.config(0)
    d = dict(gates=d["gates"], n=d["n"], b=d["b"], fuse=d["fuse"], domain=1, eb=1e-5)
    p, s = _make(d)
    st = s.apply(p, stats=True)
    peak = max(x["bytes_out"] for x in st)
    p2, s2 = _make(d, pool_bytes=peak // 4)
    s2.attach_host_pool(4 * peak)
    print("persistent: device pool capped, records spill to the host pool", flush=True)
    bmq.persistent_apply([s2], [p2], wait_limit_us=LIMIT_US)
    _same(s, s2, "host-pool")
    assert s2.footprint()[1] > 0


def test_overflow_is_reported():
    d = C.config(0)
    d = dict(gates=d["gates"], n=d["n"], b=d["b"], fuse=d["fuse"], domain=1, eb=1e-5)
    p, s = _make(d, pool_bytes=4096)
    with pytest.raises(bmq.BmqError) as e:
        bmq.persistent_apply([s], [p], wait_limit_us=LIMIT_US)
    assert e.value.code == -3


def test_wait_limit_aborts_and_device_recovers():
    # 2^12 tiles per pass on 2^10-amplitude tiles: a tile of the second pass
    # is claimed while about a thousand tiles of the first are in flight, so
    # with a 1 us limit its wait runs out and the launch aborts
    d = _qft(22, 10)
    p, s = _make(d)
    print("persistent: 22-qubit QFT with a 1 us wait limit (abort expected)", flush=True)
    t0 = time.perf_counter()
    with pytest.raises(bmq.BmqError) as e:
        bmq.persistent_apply([s], [p], wait_limit_us=1)
    assert e.value.code == -7
    assert time.perf_counter() - t0 < 5.0
    with pytest.raises(bmq.BmqError):
        bmq.persistent_apply([s], [p], wait_limit_us=LIMIT_US)          # poisoned until reset
    s.reset()
    print("persistent: same state after reset", flush=True)
    bmq.persistent_apply([s], [p], wait_limit_us=LIMIT_US)
    pe, se = _make(d)
    se.apply(pe)
    _same(se, s, "after-abort")
