"""Memory planning with the block predictor (Section 3 feasibility analysis,
Section 4.4 two-level memory management): the predictor, trained online on
block statistics the simulator generates, is rolled over a circuit's plan to
predict its peak compressed size; the peak sizes each circuit's device pools
and decides which circuits of a batch fit a device budget.

* the rollout kernels agree with a float64 rollout of the oracle network;
* with vs without the predictor: under the same budget the predicted pools
  admit more circuits than worst-case pools, every admitted circuit runs
  without a capacity error (or is re-run with worst-case pools), and its
  records are byte-identical to a worst-case run (pool sizes never change a
  byte); the naive alternative -- the size a circuit has before it runs --
  would overflow."""
import numpy as np
import pytest

from oracle import mlp as M
from oracle import native as N

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"


def _cfg(n, fuse=4):
    return bmq.Config(n=n, b=n - 8, inner=2, fuse=fuse, domain=1, eb=1e-5, flags=bmq.SV_FLAG_NO_SCRATCH)


def test_rollout_matches_float64_oracle():
    n = 16
    gates = C.random_layers(n, 6, 4)
    cfg = _cfg(n)
    plan = bmq.Plan(gates, cfg)
    params = C.mlp_init_params(3) + np.random.default_rng(1).normal(0, 0.02, bmq.SV_MLP_NPARAM).astype(np.float32)
    got = bmq.predict_bytes(torch.from_numpy(params).to(DEV), plan)
    b, ns = cfg.b, plan.n_stages
    order = plan.gate_order()
    sfs = []
    for s in range(ns):
        g0, g1 = plan.stage(s)["gates"]
        sfs.append(M.stage_features([gates[order[k]] for k in range(g0, g1)], b, len(plan.stage_ops(s)), s, ns, 1e-5))
    e = np.zeros(1 << b, np.float32)
    e[0] = 1
    z = np.zeros(1 << b, np.float32)
    X = np.array([M.block_features(N.encode_block(e if k == 0 else z, z, 1, 1e-5), sfs[0])
                  for k in range(1 << (n - b))])
    # planning form: log2 bytes per amplitude, features 1..24 of an all-zero block
    X[:, 0] -= b
    X[:, 1:25] = 0.0
    X[:, 1] = X[:, 21] = 1.0
    want = []
    for s in range(ns):
        out = M.forward(params.astype(np.float64), X)[0]
        out[:, 0] = np.clip(out[:, 0], -3.0, np.float32(3.1292830))
        want.append(np.exp2(out[:, 0] + b).sum())
        X[:, 0] = out[:, 0]
        if s + 1 < ns:
            X[:, 25:32] = sfs[s + 1]
    want = np.array(want)
    print(f"rollout: {ns} stages, max |log2 ratio| {np.abs(np.log2(got / want)).max():.2e}", flush=True)
    assert np.abs(np.log2(got / want)).max() < 1e-3


def _train(pred, circuits, rounds=4):
    """Online training, stage by stage (planning features before a stage,
    labels after it, `rounds` Adam steps), then calibration: the largest
    actual / predicted peak over the same circuits."""
    peaks, plans = [], []
    for d in circuits:
        cfg = _cfg(d["n"])
        plan = bmq.Plan(d["gates"], cfg)
        sv = bmq.State(cfg, DEV)
        peak = 0.0
        for s in range(plan.n_stages):
            X = sv.plan_features(plan, s)
            sv.apply(plan, s, 1)
            y, mode = sv.plan_labels()
            for _ in range(rounds):
                pred.train_step(X, y, mode)
            peak = max(peak, float(torch.exp2(y.double() + cfg.b).sum()))
        peaks.append(peak)
        plans.append(plan)
        sv.close()
    tp = np.array([float(bmq.predict_bytes(pred.params, p).max()) for p in plans])
    ratio = np.array(peaks) / tp
    calib = max(1.0, float(ratio.max()))
    print(f"training: actual / predicted peak on the training circuits {ratio.min():.3f}..{ratio.max():.3f}, "
          f"calibration {calib:.3f}", flush=True)
    return calib


def _run(d, pool):
    cfg = _cfg(d["n"])
    cfg.pool_bytes = int(pool)
    plan = bmq.Plan(d["gates"], cfg)
    sv = bmq.State(cfg, DEV)
    try:
        st = sv.apply(plan, stats=True)
    except bmq.BmqError as e:
        assert e.code == -3
        sv.close()
        return None, None
    return sv, st


def test_predicted_pools_admit_more_circuits_than_worst_case():
    mix = C.batch_mix(28, seed0=7000, nmin=20, nmax=24)
    train, test = mix[:12], mix[12:]
    pred = bmq.Predictor(C.mlp_init_params(11), DEV, lr=2e-3)
    calib = _train(pred, train)
    cfgs = [_cfg(d["n"]) for d in test]
    peaks = []
    for d, c in zip(test, cfgs):
        peaks.append(float(bmq.predict_bytes(pred.params, bmq.Plan(d["gates"], c)).max()) * calib)
    peaks = np.array(peaks)
    # actual peaks (stream bytes: record bodies + two 4-byte headers per chunk)
    actual, naive, ref_streams = [], [], []
    for d in test:
        sv, st = _run(d, 0)
        nch = 1 << (d["n"] - 6)
        actual.append(max(s["bytes_out"] for s in st) + 8 * nch)
        naive.append(st[0]["bytes_in"] + 8 * nch)             # the size before the circuit runs
        ref_streams.append([sv.block_stream(k) for k in range(sv.n_blocks)])
        sv.close()
    actual, naive = np.array(actual, np.float64), np.array(naive, np.float64)
    err = np.log2(peaks / actual)
    print(f"predicted / actual peak: log2 mean {err.mean():+.3f} max |.| {np.abs(err).max():.3f}; "
          f"before-run size / actual: {np.median(naive / actual):.2e}", flush=True)
    assert np.abs(err).max() < 1.0
    margin = 0.1
    worst = bmq.admit(cfgs, None, margin, 1 << 62)[2].sum()
    budget = int(0.6 * worst)
    adm_w, pool_w, _ = bmq.admit(cfgs, None, margin, budget)
    adm_p, pool_p, arena_p = bmq.admit(cfgs, peaks, margin, budget)
    adm_n = bmq.admit(cfgs, naive, margin, budget)[0]
    print(f"budget {budget}: admitted worst-case {adm_w.sum()}, predicted {adm_p.sum()}, "
          f"before-run size {adm_n.sum()} of {len(test)}", flush=True)
    assert adm_p.sum() > adm_w.sum()
    assert arena_p[adm_p].sum() <= budget
    # the admitted circuits with their predicted pools: no capacity error
    # except a re-run with worst-case pools, records identical either way
    fallbacks = 0
    for i in np.flatnonzero(adm_p):
        sv, st = _run(test[i], pool_p[i])
        if sv is None:
            fallbacks += 1
            sv, st = _run(test[i], 0)
        assert [sv.block_stream(k) for k in range(sv.n_blocks)] == ref_streams[i]
        sv.close()
    # the before-run size admits everything and overflows on most circuits
    over = sum(_run(test[i], p)[0] is None for i, p in zip(np.flatnonzero(adm_n), bmq.admit(cfgs, naive, margin, budget)[1][adm_n]))
    print(f"fallbacks with predicted pools {fallbacks} of {adm_p.sum()}; overflows with before-run sizes "
          f"{over} of {adm_n.sum()}", flush=True)
    assert fallbacks <= max(1, adm_p.sum() // 4)
    assert over > fallbacks
