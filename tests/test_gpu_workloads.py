"""Mid-size runs of the benchmark workloads on the GPU: the random-layer
mirror circuit with 5-qubit fused operations on the matrix cores (exact
fidelity from amplitude 0) and the QFT on an Ry product with 4-qubit fusion
(sampled closed form)."""
import numpy as np
import pytest

from oracle import native as N

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"


def _bound(stats, eb=1e-5):
    # each compression moves the state by at most an angle arcsin(2^eb - 1)
    comp = sum(s["passes"] for s in stats)
    return np.cos(comp * np.arcsin((2 ** eb - 1) * 1.0001)) ** 2


@pytest.mark.parametrize("flags", [0, 2])
def test_random_mirror_24q_fuse5(flags):
    n = 24
    gates = C.mirror(C.random_layers(n, 8, seed=1002))
    cfg = bmq.Config(n=n, b=16, inner=2, fuse=5, domain=1, eb=1e-5, flags=flags)
    plan = bmq.Plan(gates, cfg)
    sv = bmq.State(cfg, DEV)
    print(f"random mirror n={n} flags={flags}: {len(gates)} gates, {plan.n_stages} stages", flush=True)
    st = sv.apply(plan, stats=True)
    _, _, norm2 = sv.fidelity(None)
    a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
    f2 = abs(a0) ** 2 / norm2
    print(f"  F2={f2:.10f} bound={_bound(st):.10f} norm2={norm2:.10f}", flush=True)
    assert f2 >= _bound(st) - 1e-5


def test_qft_24q_fuse4_sampled():
    n = 24
    d = C.config(1, n=n)
    cfg = bmq.Config(n=n, b=n - 8, inner=2, fuse=4, domain=1, eb=1e-5)
    plan = bmq.Plan(d["gates"], cfg)
    sv = bmq.State(cfg, DEV)
    st = sv.apply(plan, stats=True)
    idx = np.random.default_rng(3).integers(0, 1 << n, 8192).astype(np.uint64)
    want = N.qft_ry_amplitudes(n, d["thetas"], idx)
    got = sv.amplitudes(torch.from_numpy(idx.astype(np.int64))).cpu().numpy().astype(np.complex128)
    f2 = abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real)
    err = np.abs(got - want).max()
    print(f"qft n={n}: F2(sampled)={f2:.12f} max abs err={err:.3e}", flush=True)
    assert f2 >= _bound(st) - 1e-6
    # each compression adds an error vector of norm <= (2^eb - 1) |psi| and the
    # gates preserve norms, so no amplitude can be off by more than the sum
    comp = sum(s["passes"] for s in st)
    assert err <= comp * (2 ** 1e-5 - 1) * 1.01 + 1e-6


def test_config2_full_size_mirror():
    """33-qubit random layers (depth 16) followed by their inverse, 2^24-
    amplitude blocks, 5-qubit fused operations on the matrix cores, LOG
    eb=1e-5: the launch configuration the benchmark times.  A mirror circuit
    returns to |0...0>, so F^2 = |psi(0)|^2 / |psi|^2 is exact at any size."""
    d = C.config(2)
    n = d["n"]
    gates = C.mirror(d["gates"])
    cfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=5, domain=1, eb=1e-5)
    plan = bmq.Plan(gates, cfg)
    print(f"cfg2 mirror n={n}: {len(gates)} gates, {plan.n_stages} stages", flush=True)
    sv = bmq.State(cfg, DEV)
    st = sv.apply(plan, stats=True)
    _, _, norm2 = sv.fidelity(None)
    a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
    f2 = abs(a0) ** 2 / norm2
    print(f"  F2={f2:.10f} bound={_bound(st):.10f} norm2={norm2:.10f} "
          f"peak ratio={(8 << n) / max(s['bytes_out'] for s in st):.3f}", flush=True)
    assert f2 >= 0.99
    assert f2 >= _bound(st) - 1e-5
    sv.close()
    del sv
    torch.cuda.empty_cache()


def test_config3_qaoa_32q_host_spill_sampled():
    """QAOA ring p=3 at 32 qubits (the largest size whose closed-form check
    stays cheap), scratch-free, device pools capped at a quarter of the
    complex64 state so that most records live in the pinned host pool:
    sampled amplitudes against the oracle's transfer-matrix closed form."""
    from oracle import sim as S
    n = 32
    gates, gammas, betas = C.qaoa_ring(n, 3, 1003)
    pool = int(0.25 * (8 << n)) & ~255
    cfg = bmq.Config(n=n, b=n - 8, inner=2, fuse=4, domain=1, eb=1e-5, pool_bytes=pool,
                     flags=bmq.SV_FLAG_NO_SCRATCH)
    plan = bmq.Plan(gates, cfg)
    sv = bmq.State(cfg, DEV)
    sv.attach_host_pool(2 * (8 << n))
    print(f"cfg3 qaoa n={n}: {len(gates)} gates, {plan.n_stages} stages, device pool {pool} bytes", flush=True)
    st = sv.apply(plan, stats=True)
    rec, host, _ = sv.footprint()
    assert host > 0 and max(s["bytes_out_host"] for s in st) > 0
    idx = np.random.default_rng(11).integers(0, 1 << n, 48).astype(np.uint64)
    want = np.array([S.qaoa_ring_amplitude(n, gammas, betas, int(x)) for x in idx])
    got = sv.amplitudes(torch.from_numpy(idx.astype(np.int64))).cpu().numpy().astype(np.complex128)
    err = np.abs(got - want).max()
    f2 = abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real)
    print(f"  host bytes={host} of {rec}; sampled F2={f2:.10f} max abs err={err:.3e}", flush=True)
    assert f2 >= 0.99
    # each compression adds an error vector of norm <= (2^eb - 1) |psi| and
    # the gates preserve norms: no amplitude is off by more than the sum
    comp = sum(s["passes"] for s in st)
    assert err <= comp * (2 ** 1e-5 - 1) * 1.01
    sv.close()
    del sv
    torch.cuda.empty_cache()
