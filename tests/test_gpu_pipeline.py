"""The host-resident pipeline (the paper's deployment, Section 4.2 and
Fig. 6) on the GPU: the compressed state lives in pinned host memory as block
images and every stage moves each SV group through the device on S streams.
Its records must equal, bit for bit, those of the same plan run on a
device-resident state, for any number of streams."""
import numpy as np
import pytest

from oracle import native as N

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"


def _case(which):
    if which == "random16":
        d = C.config(0)
        return d["n"], d["b"], d["gates"], 2, 0
    n = 20
    return n, 12, C.qft_on_ry(n, 7)[0], 4, 0


@pytest.mark.parametrize("which", ["random16", "qft20"])
@pytest.mark.parametrize("streams", [1, 2, 4])
def test_pipeline_matches_device_resident(which, streams):
    n, b, gates, fuse, tile = _case(which)
    cfg = bmq.Config(n=n, b=b, inner=2, fuse=fuse, domain=bmq.SV_DOMAIN_LOG, eb=1e-5, tile=tile)
    plan = bmq.Plan(gates, cfg)
    print(f"{which}: {plan.n_stages} stages, {plan.info()['passes']} passes, {streams} streams", flush=True)
    ref = bmq.State(cfg, DEV)
    st_ref = ref.apply(plan, stats=True)
    pipe = bmq.Pipe(cfg, streams=streams)
    st = pipe.apply(plan, stats=True)
    fp = pipe.footprint()
    # every stage's copies: its images in and out
    assert all(s["bytes_in"] > 0 and s["bytes_out"] > 0 for s in st)
    assert fp["h2d_bytes"] == sum(s["bytes_in"] for s in st)
    assert fp["record_bytes"] == ref.footprint()[0]
    out = bmq.State(cfg, DEV)
    pipe.load(out)
    for k in range(out.n_blocks):
        assert out.block_stream(k) == ref.block_stream(k), k
    assert torch.equal(out.export(), ref.export())
    if which == "random16":
        f = torch.from_numpy(np.ascontiguousarray(N.simulate(n, gates))).to(DEV)
        f2, maxerr, _ = out.fidelity(f)
        assert f2 >= 0.99
    # a second run from |0...0> reuses the host store in place
    used = fp["host_used"]
    pipe.reset()
    pipe.apply(plan)
    pipe.load(out)
    for k in range(out.n_blocks):
        assert out.block_stream(k) == ref.block_stream(k), k
    assert pipe.footprint()["host_used"] <= used * 1.01 + 4096
    pipe.close()


def test_pipeline_stage_ranges_and_limits():
    n, b, gates, fuse, tile = _case("random16")
    cfg = bmq.Config(n=n, b=b, inner=2, fuse=fuse, domain=bmq.SV_DOMAIN_LOG, eb=1e-5)
    plan = bmq.Plan(gates, cfg)
    ref = bmq.State(cfg, DEV)
    ref.apply(plan)
    pipe = bmq.Pipe(cfg, streams=2)
    half = plan.n_stages // 2
    pipe.apply(plan, 0, half)
    pipe.apply(plan, half, plan.n_stages - half)
    out = bmq.State(cfg, DEV)
    pipe.load(out)
    for k in range(out.n_blocks):
        assert out.block_stream(k) == ref.block_stream(k), k
    # stages wider than the staging holds
    wide = bmq.Plan(gates, bmq.Config(n=n, b=b, inner=4, fuse=fuse, domain=bmq.SV_DOMAIN_LOG, eb=1e-5))
    if any(len(wide.stage(s)["inner"]) > 2 for s in range(wide.n_stages)):
        pipe.reset()
        with pytest.raises(bmq.BmqError) as e:
            pipe.apply(wide)
        assert e.value.code == -1
    pipe.close()
    # a host store too small for the state: capacity error, then poisoned
    small = bmq.Pipe(cfg, streams=1, host_bytes=(1 << (n - b)) * 8 * (1 << (b - 6)) * 5 // 4 + 65536)
    with pytest.raises(bmq.BmqError) as e:
        small.apply(plan)
    assert e.value.code == -3
    with pytest.raises(bmq.BmqError):
        small.apply(plan)
    small.reset()
    small.close()
