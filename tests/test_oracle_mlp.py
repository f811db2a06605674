"""Pins of the block-predictor oracle (CPU only): finite-difference
gradients, closed-form special cases of the loss and of Adam, and features
of hand-derived streams."""
import math
import struct

import numpy as np

from oracle import mlp as M
from paper_2410_14088_amd import circuits as C

GOLDEN = __file__.rsplit("/", 1)[0] + "/golden/"


def _data(B=7, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 32))
    y = rng.normal(size=B) * 3 + 10
    mode = rng.integers(0, 4, size=B)
    return X, y, mode


def test_layout_size():
    assert M.NPARAM == 6597 == C.mlp_init_params(0).size


def test_gradient_matches_central_differences():
    X, y, mode = _data()
    p = C.mlp_init_params(11).astype(np.float64)
    p += np.random.default_rng(5).normal(size=p.size) * 0.05     # non-zero biases
    _, g = M.grad(p, X, y, mode)
    idx = np.concatenate([np.arange(0, 6597, 97), [2048, 2111, 2112, 6208, 6271, 6272, 6591, 6592, 6596]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss(p + e, X, y, mode) - M.loss(p - e, X, y, mode)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_hand_set_network_closed_form():
    # W1[0,0] = W2[0,0] = W3[0,0] = 1, everything else 0: out0 = x0 + relu(relu(x0))
    # (skip connection plus the network), logits 0 -> cross entropy log 4
    p = np.zeros(M.NPARAM)
    P = M.unpack(p)
    P["W1"][0, 0] = 1.0
    P["W2"][0, 0] = 1.0
    P["W3"][0, 0] = 1.0
    flat = np.concatenate([P[n].reshape(-1) for n, _ in M.SHAPES])
    X = np.zeros((3, 32))
    X[:, 0] = [2.0, -1.0, 0.5]
    out, _ = M.forward(flat, X)
    assert np.allclose(out[:, 0], [4.0, -1.0, 1.0]) and np.all(out[:, 1:] == 0)
    y = np.array([1.0, 1.0, 1.0])
    want = np.mean(0.5 * (np.array([4.0, -1.0, 1.0]) - 1) ** 2) + math.log(4)
    assert abs(M.loss(flat, X, y, [0, 1, 3]) - want) < 1e-12
    # gradient of b3[0] is the mean residual; of the logit biases softmax - onehot
    _, g = M.grad(flat, X, y, [0, 1, 3])
    b3 = g[6592:]
    assert abs(b3[0] - np.mean([3.0, -2.0, 0.0])) < 1e-12
    assert np.allclose(b3[1:], (np.full(4, 0.25) * 3 - np.array([1, 1, 0, 1])) / 3)


def test_dead_relu_units_get_no_gradient():
    X, y, mode = _data()
    p = C.mlp_init_params(2).astype(np.float64)
    P = M.unpack(p)
    P["b1"][5] = -1e6          # unit 5 of layer 1 never fires
    flat = np.concatenate([P[n].reshape(-1) for n, _ in M.SHAPES])
    _, g = M.grad(flat, X, y, mode)
    assert np.all(g[5 * 32:6 * 32] == 0) and g[2048 + 5] == 0


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    new, m, v = M.adam(p, g, np.zeros(4), np.zeros(4), 1, 0.01)
    # after one step the bias-corrected moments are g and g^2
    assert np.allclose(new, -0.01 * g / (np.abs(g) + M.EPS))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(9)
    X = rng.normal(size=(64, 32))
    y = X[:, 0] * 2 + 12
    mode = (X[:, 1] > 0).astype(int)
    p = C.mlp_init_params(4).astype(np.float64)
    m = v = np.zeros_like(p)
    l0 = M.loss(p, X, y, mode)
    for t in range(1, 201):
        _, g = M.grad(p, X, y, mode)
        p, m, v = M.adam(p, g, m, v, t, 3e-3)
    assert M.loss(p, X, y, mode) < 0.1 * l0


def _hexstream(name):
    return bytes.fromhex(open(GOLDEN + name).read().split()[0])


def test_features_of_golden_streams():
    sf = np.arange(7) / 10
    # LIN ramp: re LZ w=2 (anchor 4 + payload 16 bytes), im ZERO; record 28 bytes
    f = M.block_features(_hexstream("lin_ramp_chunk.hex"), sf)
    want = np.zeros(32)
    want[0] = math.log2(28)
    want[1], want[2] = 0.5, 0.5          # one ZERO plane, one LZ plane
    want[5] = 1.0                        # width 2 -> bin 0
    want[23] = 2 / 32
    want[25:] = sf
    assert np.allclose(f, want, atol=0, rtol=1e-15), f
    assert M.block_label(_hexstream("lin_ramp_chunk.hex")) == (math.log2(28), 0)
    # LOG alternating powers of two: re LZ w=10, mixed signs (mask 8 bytes),
    # anchor 4, payload 80 -> record 100 bytes
    f = M.block_features(_hexstream("log_alternating_pow2_chunk.hex"), sf)
    want = np.zeros(32)
    want[0] = math.log2(100)
    want[1], want[2] = 0.5, 0.5
    want[7] = 1.0                        # width 10 -> bin 2
    want[22] = 1.0
    want[23] = 10 / 32
    want[25:] = sf
    assert np.allclose(f, want, atol=0, rtol=1e-15), f


def test_features_of_all_zero_block():
    nch = 16
    s = bytes([0x51, 1, 1, 6]) + struct.pack("<fII", 1e-5, 64 * nch, nch) + b"\0" * (8 * nch)
    f = M.block_features(s, np.zeros(7))
    assert f[0] == math.log2(8 * nch) and f[1] == 1.0 and f[21] == 1.0 and f[2:21].sum() == 0
    assert M.block_label(s) == (math.log2(8 * nch), 0)


def test_stage_features():
    gates = [("H", (0,), ()), ("CZ", (1, 12), ()), ("RZ", (3,), (0.1,)), ("U3", (11,), (1, 2, 3))]
    f = M.stage_features(gates, b=10, n_ops=3, stage=2, n_stages=8, eb=1e-5)
    assert np.allclose(f, [2 / 64, 2 / 64, 2 / 64, 3 / 10, 3 / 16, 0.25, math.log2(1e-5) / 32])
