"""Two-level memory (device pool + pinned host pool) and the scratch-free
stage mode, on the GPU.  Placement must not change a single byte of the
state: streams with a small device pool spilling to the host equal those of
a run that fits the device, and the scratch-free mode stays within the
fidelity bound of its extra compressions."""
import numpy as np
import pytest

from oracle import native as N

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"


def _run(gates, n, b, pool_bytes=0, host=0, flags=0, fuse=2, inner=2, tile=0, eb=1e-5, exact=False):
    cfg = bmq.Config(n=n, b=b, inner=inner, fuse=fuse, domain=1, eb=eb, pool_bytes=pool_bytes, flags=flags,
                     tile=tile)
    plan = bmq.Plan(gates, cfg)
    sv = bmq.State(cfg, DEV)
    if host:
        sv.attach_host_pool(host, exact=exact)
    stats = sv.apply(plan, stats=True)
    return sv, plan, stats


def test_host_spill_is_bit_exact():
    d = C.config(0)
    n, b = d["n"], d["b"]
    print("reference run (device pool only)", flush=True)
    ref, _, st_ref = _run(d["gates"], n, b)
    peak = max(s["bytes_out"] for s in st_ref)
    print(f"spill run: device pool {peak // 4} bytes, peak state {peak}", flush=True)
    sv, _, st = _run(d["gates"], n, b, pool_bytes=peak // 4, host=4 * peak)
    assert max(s["bytes_out_host"] for s in st) > 0
    assert [s["bytes_out"] for s in st] == [s["bytes_out"] for s in st_ref]
    for k in range(sv.n_blocks):
        assert sv.block_stream(k) == ref.block_stream(k), k
    rec, host, _ = sv.footprint()
    assert rec == ref.footprint()[0] and 0 < host <= rec
    assert torch.equal(sv.export(), ref.export())
    f = N.simulate(n, d["gates"])
    fr = torch.from_numpy(np.ascontiguousarray(f)).to(DEV)
    assert sv.fidelity(fr) == ref.fidelity(fr)


def test_host_pool_of_exact_size_is_bit_exact():
    # a host pool from sv_host_alloc, of a size that is no power of two
    d = C.config(0)
    n, b = d["n"], d["b"]
    ref, _, st_ref = _run(d["gates"], n, b)
    peak = max(s["bytes_out"] for s in st_ref)
    host = 3 * peak + 4096 + 256
    print(f"spill run: device pool {peak // 4} bytes, exact host pool {host} bytes", flush=True)
    sv, _, st = _run(d["gates"], n, b, pool_bytes=peak // 4, host=host, exact=True)
    assert isinstance(sv.host_pool, bmq.HostBuffer) and sv.host_pool.nbytes == host
    assert max(s["bytes_out_host"] for s in st) > 0
    for k in range(sv.n_blocks):
        assert sv.block_stream(k) == ref.block_stream(k), k
    sv.close()
    assert sv.host_pool.ptr is None                # freed with the state


def test_both_levels_full_reports_capacity():
    d = C.config(0)
    _, _, st_ref = _run(d["gates"], d["n"], d["b"])
    peak = max(s["bytes_out"] for s in st_ref)
    with pytest.raises(bmq.BmqError) as e:
        _run(d["gates"], d["n"], d["b"], pool_bytes=peak // 4, host=peak // 4)
    assert e.value.code == -3


def test_detach_refused_while_host_holds_records():
    d = C.config(0)
    _, _, st_ref = _run(d["gates"], d["n"], d["b"])
    peak = max(s["bytes_out"] for s in st_ref)
    sv, _, _ = _run(d["gates"], d["n"], d["b"], pool_bytes=peak // 4, host=4 * peak)
    assert sv.footprint()[1] > 0
    with pytest.raises(bmq.BmqError):
        sv.attach_host_pool(0)
    sv.reset()
    sv.attach_host_pool(0)          # the reset state lives in the device pool


def test_no_scratch_mode_recompresses_between_passes():
    n, b = 18, 12
    gates = C.random_layers(n, 6, seed=31)
    print("scratch run", flush=True)
    a, plan, st_a = _run(gates, n, b, fuse=4, inner=4, tile=10)
    multi = [i for i, s in enumerate(st_a) if s["passes"] > 1]
    assert multi, "the circuit must have multi-pass stages"
    print(f"no-scratch run ({len(multi)} multi-pass stages)", flush=True)
    s, _, st_s = _run(gates, n, b, fuse=4, inner=4, tile=10, flags=bmq.SV_FLAG_NO_SCRATCH)
    assert all(x["scratch_bytes"] == 0 for x in st_s)
    assert all(st_s[i]["inter_bytes"] > 0 for i in multi)
    ref = torch.from_numpy(np.ascontiguousarray(N.simulate(n, gates))).to(DEV)
    fa, ma, _ = a.fidelity(ref)
    fs, ms, _ = s.fidelity(ref)
    assert fa >= 0.99 and fs >= 0.99
    # the angle bound holds for the normalised F^2
    fa, fs = a.fidelity_full(ref)["fidelity"], s.fidelity_full(ref)["fidelity"]
    # each compression moves the state by at most 2^eb - 1 relative per
    # amplitude; the extra passes add compressions, not more than that
    comp = len(st_s) + sum(x["passes"] - 1 for x in st_s)
    eps = 2 ** 1e-5 - 1
    print(f"F2 scratch {fa:.10f} no-scratch {fs:.10f} (compressions {comp}), max err {ma:.2e} {ms:.2e}", flush=True)
    assert fs >= np.cos(comp * np.arcsin(eps * 1.0001)) ** 2 - 1e-4


@pytest.mark.parametrize("fuse", [4, 5])
def test_mfma_and_vector_dense_paths_agree(fuse):
    """Dense 4- and 5-qubit operations on the matrix cores vs vector FMAs:
    both within the fidelity bound against FP64, and close to each other."""
    n, b = 18, 12
    gates = C.random_layers(n, 8, seed=40 + fuse)
    ref = torch.from_numpy(np.ascontiguousarray(N.simulate(n, gates))).to(DEV)
    out = []
    for flags in (0, bmq.SV_FLAG_NO_MFMA):
        sv, plan, st = _run(gates, n, b, fuse=fuse, flags=flags)
        f2, mx, _ = sv.fidelity(ref)
        print(f"fuse {fuse} flags {flags}: F2 {f2:.10f} max err {mx:.2e}", flush=True)
        assert f2 >= 0.9999 and mx < 1e-4
        out.append(sv.export())
    assert float((out[0] - out[1]).abs().max()) < 1e-5


@pytest.mark.parametrize("which", ["qft20", "random16-t10"])
def test_group_scratch_matches_full_scratch(which):
    """SV_FLAG_GROUP_SCRATCH: multi-pass stages run group by group on
    scratch planes sized for one SV group; every record equals the run with
    whole-state scratch planes, the arena shrinks, and a captured graph of the
    group launches replays to the same records."""
    if which == "qft20":
        n, b, tile, fuse = 20, 12, 12, 4
        gates = C.qft_on_ry(n, 7)[0]
    else:
        d = C.config(0)
        n, b, tile, fuse, gates = d["n"], d["b"], 10, 2, d["gates"]
    full, plan, st_full = _run(gates, n, b, fuse=fuse, tile=tile)
    grp, gplan, st_grp = _run(gates, n, b, fuse=fuse, tile=tile, flags=bmq.SV_FLAG_GROUP_SCRATCH)
    multi = [s["passes"] for s in st_grp if s["passes"] > 1]
    print(f"{which}: {len(st_grp)} stages, {len(multi)} multi-pass; arenas {full.arena.numel()} vs "
          f"{grp.arena.numel()} bytes", flush=True)
    assert multi, "the test needs multi-pass stages"
    assert grp.arena.numel() < full.arena.numel()
    assert [s["bytes_out"] for s in st_grp] == [s["bytes_out"] for s in st_full]
    for k in range(grp.n_blocks):
        assert grp.block_stream(k) == full.block_stream(k), k
    # the same stage loop captured in a graph (group launches included)
    grp.reset()
    g = grp.capture(gplan)
    for rep in range(3):
        grp.reset()
        g.launch()
        grp.graph_sync()
        torch.cuda.synchronize()
        for k in range(grp.n_blocks):
            assert grp.block_stream(k) == full.block_stream(k), (rep, k)
    g.close()
    # batched and queue launches need whole-state scratch for multi-pass stages
    grp.reset()
    with pytest.raises(bmq.BmqError) as e:
        bmq.batch_apply([grp], [gplan])
    assert e.value.code == -6
    # a plan whose stages span more qubits than the group scratch holds
    wide = bmq.Plan(gates, bmq.Config(n=n, b=b, inner=5, fuse=fuse, domain=1, eb=1e-5, tile=tile,
                                      flags=bmq.SV_FLAG_GROUP_SCRATCH))
    if any(wide.stage(s)["passes"] > 1 and len(wide.stage(s)["inner"]) > 2 for s in range(wide.n_stages)):
        grp.reset()
        with pytest.raises(bmq.BmqError) as e:
            grp.apply(wide)
        assert e.value.code == -1
