"""GPU parity of the checker and of the codec at full size.

* sv_fidelity's FP64 reductions (<ref|psi>, |psi|^2, |ref|^2, max |psi -
  ref|) equal the oracle's overlap of the exported state, for a host, a
  device and a compressed reference;
* sv_sample draws x from |psi(x)|^2 (chi-square against the exported
  state), and the importance-sampled fidelity estimate it feeds (Section
  5.3 fidelity; used where the reference is known only amplitude by
  amplitude) agrees with the exact value;
* at the 30- and 33-qubit configurations, two whole SV blocks per stage:
  records equal the CPU codec's stream of the values the stage encoded,
  and the next stage's decoder produces exactly the CPU decoder's values.
"""
import math

import numpy as np
import pytest

from oracle import native as N

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"


def _state(n, b, gates, domain=1, eb=1e-3, fuse=3):
    cfg = bmq.Config(n=n, b=b, inner=2, fuse=fuse, domain=domain, eb=eb)
    plan = bmq.Plan(gates, cfg)
    sv = bmq.State(cfg, DEV)
    sv.apply(plan)
    return sv


def _close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


def test_fidelity_reduction_matches_oracle_overlap():
    n, b = 16, 10
    gates = C.random_layers(n, 6, 4242)
    # a coarse bound, so that the state differs measurably from the reference
    sv = _state(n, b, gates, eb=2e-3)
    ref = N.simulate(n, gates)
    psi = sv.export().cpu().numpy()
    ov, nref, npsi, mx = N.overlap(ref, psi)
    print(f"oracle: <ref|psi>={ov} |ref|^2={nref} |psi|^2={npsi} max={mx}", flush=True)
    assert abs(ov) ** 2 / (nref * npsi) < 1 - 1e-9     # not a trivially perfect state
    for kind, r in (("host", ref), ("device", torch.from_numpy(ref).to(DEV))):
        f = sv.fidelity_full(r)
        print(kind, f, flush=True)
        assert _close(f["overlap_re"], ov.real) and _close(f["overlap_im"], ov.imag, rel=1e-9)
        assert _close(f["norm2"], npsi) and _close(f["ref_norm2"], nref)
        assert f["max_abs_err"] == pytest.approx(mx, rel=0, abs=0)
        assert _close(f["overlap2"], abs(ov) ** 2)
        assert _close(f["fidelity"], abs(ov) ** 2 / (nref * npsi))
    # a second compressed state as the reference (no compression: RAW)
    raw = _state(n, b, gates, domain=2, eb=1.0)
    rv = raw.export().cpu().numpy()
    ov2, nr2, np2, mx2 = N.overlap(rv.astype(np.complex128), psi)
    f = sv.fidelity_full(raw)
    assert _close(f["overlap_re"], ov2.real) and _close(f["norm2"], np2) and _close(f["ref_norm2"], nr2)
    assert f["max_abs_err"] == mx2
    f0 = sv.fidelity_full(None)
    assert _close(f0["norm2"], npsi) and math.isnan(f0["overlap2"])


def test_fidelity_rejects_two_references():
    n, b = 12, 8
    sv = _state(n, b, C.random_layers(n, 1, 1))
    ref = np.zeros(1 << n, np.complex128)
    rc = bmq.lib().sv_fidelity(sv.h, bmq.C.c_void_p(ref.ctypes.data), None, sv.h,
                               bmq.C.byref(bmq.sv_fidelity_t()))
    assert rc == -1


@pytest.mark.parametrize("n,b", [(12, 8), (18, 12)])
def test_sample_distribution(n, b):
    sv = _state(n, b, C.random_layers(n, 4, 31 + n), eb=1e-5)
    psi = sv.export().cpu().numpy().astype(np.complex128)
    p = np.abs(psi) ** 2
    p /= p.sum()
    k = 200000
    idx = sv.sample(k, seed=12345)
    assert idx.dtype == np.uint64 and idx.size == k and int(idx.max()) < (1 << n)
    assert np.all(p[idx.astype(np.int64)] > 0)
    # chi-square over 64-amplitude chunks (enough expected counts per cell)
    cells = 1 << (n - 6)
    width = (1 << n) // cells
    obs = np.bincount(idx.astype(np.int64) // width, minlength=cells).astype(np.float64)
    exp = p.reshape(cells, width).sum(1) * k
    m = exp > 0
    chi2 = float(((obs[m] - exp[m]) ** 2 / exp[m]).sum())
    dof = int(m.sum()) - 1
    print(f"n={n}: chi2={chi2:.1f} dof={dof}", flush=True)
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    # a different seed draws different samples; the same seed the same ones
    assert not np.array_equal(idx[:100], sv.sample(100, seed=1))
    assert np.array_equal(idx[:1000], sv.sample(1000, seed=12345))


def importance_sampled_f2(sv, ref_amp, k, seed):
    """F^2 = |<psi|ref>|^2 / (|psi|^2 |ref|^2) estimated from x ~ |psi(x)|^2:
    <psi|ref> = |psi|^2 E[ref(x) / psi(x)] (|ref| = 1 assumed).  Returns the
    estimate and its standard error (delta method on the sample mean)."""
    idx = sv.sample(k, seed)
    g = sv.amplitudes(torch.from_numpy(idx.astype(np.int64))).cpu().numpy().astype(np.complex128)
    o = ref_amp(idx)
    norm2 = sv.fidelity(None)[2]
    r = o / g
    m = np.mean(r)
    var = np.mean(np.abs(r - m) ** 2)
    return abs(m) ** 2 * norm2, 2 * norm2 * abs(m) * math.sqrt(var / k)


@pytest.mark.parametrize("eb", [2e-3, 1e-5])
def test_importance_sampled_fidelity_estimate(eb):
    n, b = 20, 14
    gates = C.random_layers(n, 8, 2024)
    sv = _state(n, b, gates, eb=eb, fuse=4)
    ref = N.simulate(n, gates)
    exact = sv.fidelity_full(ref)["fidelity"]
    est, se = importance_sampled_f2(sv, lambda x: ref[x.astype(np.int64)], 1 << 16, 99)
    print(f"eb={eb}: F2 exact={exact:.12f} estimate={est:.12f} +- {se:.2e}", flush=True)
    assert abs(est - exact) <= 5 * se + 1e-9
    assert se < 1e-3                                    # a usable estimate, not a wide band


def _full_size_blocks(cfgid, fuse, stages, nblk=2):
    d = C.config(cfgid)
    n, b = d["n"], d["b"]
    cfg = bmq.Config(n=n, b=b, inner=2, fuse=fuse, domain=1, eb=1e-5)
    plan = bmq.Plan(d["gates"], cfg)
    sv = bmq.State(cfg, DEV)
    blk0 = 3
    cnt = nblk << b
    pre = [torch.empty(cnt, dtype=torch.float32, device=DEV) for _ in range(4)]
    sv.debug_dump(pre[0], pre[1], start=blk0 << b, count=cnt, dec_re=pre[2], dec_im=pre[3])
    prev = None
    for s in range(stages):
        print(f"cfg{cfgid} n={n} stage {s}", flush=True)
        sv.apply(plan, s, 1)
        if prev is not None:
            dre, dim = pre[2].cpu().numpy(), pre[3].cpu().numpy()
            for j in range(nblk):
                lo, hi = j << b, (j + 1) << b
                assert np.array_equal(dre[lo:hi].view(np.uint32), prev[j][0].view(np.uint32)), f"stage {s}"
                assert np.array_equal(dim[lo:hi].view(np.uint32), prev[j][1].view(np.uint32)), f"stage {s}"
        xre, xim = pre[0].cpu().numpy(), pre[1].cpu().numpy()
        prev = []
        for j in range(nblk):
            lo, hi = j << b, (j + 1) << b
            gpu = sv.block_stream(blk0 + j)
            cpu = N.encode_block(xre[lo:hi], xim[lo:hi], 1, 1e-5)
            assert gpu == cpu, f"stage {s} block {blk0 + j}: streams differ"
            prev.append(N.decode_block(cpu, hi - lo))
    sv.close()
    del sv
    torch.cuda.empty_cache()


def test_full_size_blocks_config1():
    """30-qubit QFT on an Ry product, 2^22-amplitude blocks: 4 stages."""
    _full_size_blocks(1, 4, 4)


def test_full_size_blocks_config2():
    """33-qubit random layers, 2^24-amplitude blocks, 5-qubit fusion: 3 stages."""
    _full_size_blocks(2, 5, 3)
