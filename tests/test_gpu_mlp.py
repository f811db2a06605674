"""Block predictor on the GPU against the float64 oracle: forward, loss and
gradient, Adam, features and labels of a real compressed state, and online
training over the stages of a circuit (with vs without the predictor)."""
import math

import numpy as np
import pytest

from oracle import mlp as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 32)).astype(np.float32)
    y = (rng.normal(size=B) * 3 + 12).astype(np.float32)
    mode = rng.integers(0, 4, size=B).astype(np.int32)
    return X, y, mode


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("B", [1, 63, 257])
def test_forward_loss_grad_match_oracle(B):
    print(f"mlp B={B}", flush=True)
    X, y, mode = _batch(B, 100 + B)
    p = C.mlp_init_params(7)
    p[2048:2112] = 0.05        # positive first-layer biases so that most units fire
    out = bmq.mlp_forward(_dev(p), _dev(X)).cpu().numpy()
    want, _ = M.forward(p, X)
    assert np.abs(out - want).max() <= 1e-5 * max(1.0, np.abs(want).max())
    loss, g = bmq.mlp_loss_grad(_dev(p), _dev(X), _dev(y), _dev(mode))
    wl, wg = M.grad(p, X.astype(np.float64), y.astype(np.float64), mode)
    assert abs(float(loss.item()) - wl) <= 1e-5 * max(1.0, abs(wl))
    g = g.cpu().numpy()
    assert np.abs(g - wg).max() <= 1e-5 * max(1.0, np.abs(wg).max()), np.abs(g - wg).max()


def test_adam_matches_oracle_and_is_deterministic():
    p = C.mlp_init_params(3)
    rng = np.random.default_rng(4)
    grads = [rng.normal(size=p.size).astype(np.float32) for _ in range(5)]
    dp, dm, dv = _dev(p), torch.zeros(p.size, device=DEV), torch.zeros(p.size, device=DEV)
    op, om, ov = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for t, g in enumerate(grads, start=1):
        bmq.mlp_adam_update(dp, _dev(g), dm, dv, t, 1e-2)
        op, om, ov = M.adam(op, g.astype(np.float64), om, ov, t, 1e-2)
    assert np.abs(dp.cpu().numpy() - op).max() < 1e-5
    # same inputs, same bits
    loss1, g1 = bmq.mlp_loss_grad(dp, *[_dev(a) for a in _batch(300, 1)])
    loss2, g2 = bmq.mlp_loss_grad(dp, *[_dev(a) for a in _batch(300, 1)])
    assert torch.equal(g1, g2) and torch.equal(loss1, loss2)


def test_invalid_arguments():
    p = _dev(C.mlp_init_params(0))
    X = torch.zeros((0, 32), device=DEV)
    with pytest.raises(bmq.BmqError):
        bmq.mlp_loss_grad(p, X, torch.zeros(0, device=DEV), torch.zeros(0, dtype=torch.int32, device=DEV))
    with pytest.raises(bmq.BmqError):
        bmq.mlp_adam_update(p, p, p.clone(), p.clone(), 0, 1e-3)


def _sim(n, b, gates, fuse=2):
    cfg = bmq.Config(n=n, b=b, inner=2, fuse=fuse, domain=1, eb=1e-5)
    plan = bmq.Plan(gates, cfg)
    return cfg, plan, bmq.State(cfg, DEV)


def test_features_and_labels_match_streams():
    n, b = 16, 10
    d = C.config(0)
    cfg, plan, sv = _sim(n, b, d["gates"])
    ns = plan.n_stages
    n_ops = [st["n_ops"] for st in sv.apply(plan, stats=True)]
    for s in (0, 3, ns // 2, ns - 1):
        print(f"features stage {s}", flush=True)
        sv.reset()
        sv.apply(plan, 0, s)
        feats = sv.block_features(plan, s).cpu().numpy()
        g0, g1 = plan.stage(s)["gates"]
        sf = M.stage_features(d["gates"][g0:g1], b, n_ops[s], s, ns, 1e-5)
        for k in range(sv.n_blocks):
            want = M.block_features(sv.block_stream(k), sf)
            assert np.abs(feats[k] - want).max() <= 2e-7 * max(1.0, abs(want[0])), (s, k)
        lb, md = sv.block_labels()
        lb, md = lb.cpu().numpy(), md.cpu().numpy()
        for k in range(sv.n_blocks):
            wl, wm = M.block_label(sv.block_stream(k))
            assert abs(lb[k] - wl) <= 1e-6 * wl and md[k] == wm


@pytest.mark.parametrize("family", ["random", "qft"])
def test_online_training_over_stages(family):
    """Train on (features before a stage, labels after it), stage by stage of
    a 20-qubit circuit.  The loss falls and the mode is predicted; the size
    error on the last ten stages is reported next to the no-predictor
    assumption that a block keeps its current size (the untrained
    predictor's answer)."""
    n, b = 20, 12
    gates = C.random_layers(n, 12, seed=77) if family == "random" else C.qft_on_ry(n, seed=78)[0]
    cfg, plan, sv = _sim(n, b, gates, fuse=3)
    pred = bmq.Predictor(C.mlp_init_params(5), DEV, lr=1e-3)
    ns = plan.n_stages
    first = None
    errs = []
    for s in range(ns):
        X = sv.block_features(plan, s)
        out = pred.predict(X)
        if s == 0:
            assert torch.equal(out[:, 0], X[:, 0])          # untrained: no change predicted
        sv.apply(plan, s, 1)
        y, mode = sv.block_labels()
        if s >= ns - 10:
            acc = float((out[:, 1:].argmax(dim=1) == mode).float().mean())
            errs.append((float((out[:, 0] - y).abs().mean()), float((X[:, 0] - y).abs().mean()), acc))
        for _ in range(4):
            loss = float(pred.train_step(X, y, mode).item())
            first = loss if first is None else first
    e = np.array(errs)
    print(f"{family}: stages={ns} loss {first:.3f} -> {loss:.4f}; last ten stages mean |log2 bytes error| "
          f"with {e[:, 0].mean():.4f} without {e[:, 1].mean():.4f}, mode accuracy {e[:, 2].mean():.3f}", flush=True)
    assert loss < 0.5 * first
    assert e[:, 2].mean() >= 0.9
    assert e[:, 0].mean() < 0.25
