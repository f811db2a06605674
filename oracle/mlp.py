"""Block-predictor oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this
module.  It shares no code with the HIP library.

What it computes, in float64 numpy, written from the definitions:
  * the multilayer perceptron 32 -> 64 -> 64 -> 5 with ReLU after the two
    hidden layers (parameters packed as W1[64][32] b1[64] W2[64][64] b2[64]
    W3[5][64] b3[5], row = output unit), whose size output 0 also adds
    input 0 (the block's current log2 bytes);
  * the loss per sample 0.5 (out0 - y)^2 + logsumexp(out1..4) - out[1 + mode],
    averaged over the batch, and its gradient by back-propagation;
  * one Adam step (Kingma and Ba) with bias correction;
  * the per-block features and labels that feed it, read from the canonical
    block stream (16-byte header, then per chunk two 32-bit headers and the
    record body).

The predictor answers the paper's observation that a block's compression
ratio is unknown before compression, which complicates memory planning
(Section 3 feasibility analysis; Section 4.4 two-level memory management).
"""
from __future__ import annotations

import math
import struct

import numpy as np

IN, H, OUT = 32, 64, 5
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)), ("b3", (OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def unpack(params):
    """Split the flat parameter vector into named float64 arrays."""
    p = np.asarray(params, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def forward(params, X):
    """Outputs [B][5] and the activations needed by the backward pass."""
    P = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ P["W3"].T + P["b3"]
    out[:, 0] += X[:, 0]          # skip connection: current log2 bytes
    return out, (h1, h2)


def loss(params, X, y, mode):
    """Mean over the batch of squared error (halved) plus cross entropy."""
    out, _ = forward(params, X)
    y = np.asarray(y, dtype=np.float64)
    mode = np.clip(np.asarray(mode), 0, 3)
    logits = out[:, 1:]
    mx = logits.max(axis=1, keepdims=True)
    lse = mx[:, 0] + np.log(np.exp(logits - mx).sum(axis=1))
    per = 0.5 * (out[:, 0] - y) ** 2 + lse - logits[np.arange(len(y)), mode]
    return float(per.mean())


def grad(params, X, y, mode):
    """(loss, gradient) by back-propagation through the three layers."""
    P = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mode = np.clip(np.asarray(mode), 0, 3)
    B = len(y)
    out, (h1, h2) = forward(params, X)
    logits = out[:, 1:]
    mx = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - mx)
    soft = e / e.sum(axis=1, keepdims=True)
    onehot = np.zeros_like(soft)
    onehot[np.arange(B), mode] = 1.0
    d_out = np.concatenate([(out[:, :1] - y[:, None]), soft - onehot], axis=1) / B
    g = {"W3": d_out.T @ h2, "b3": d_out.sum(axis=0)}
    d_h2 = (d_out @ P["W3"]) * (h2 > 0)
    g["W2"] = d_h2.T @ h1
    g["b2"] = d_h2.sum(axis=0)
    d_h1 = (d_h2 @ P["W2"]) * (h1 > 0)
    g["W1"] = d_h1.T @ X
    g["b1"] = d_h1.sum(axis=0)
    flat = np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])
    return loss(params, X, y, mode), flat


def adam(params, g, m, v, t, lr):
    """One Adam step t >= 1; returns (params, m, v)."""
    m = BETA1 * np.asarray(m, np.float64) + (1 - BETA1) * g
    v = BETA2 * np.asarray(v, np.float64) + (1 - BETA2) * g * g
    mh = m / (1 - BETA1 ** t)
    vh = v / (1 - BETA2 ** t)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + EPS), m, v


# ---------------------------------------------------------------- stream statistics

def _body_bytes(h: int, other: int) -> int:
    """Body bytes a plane with header h contributes (anchor, masks, payload)."""
    mode, w = h & 3, (h >> 2) & 63
    packed = mode in (1, 2)
    n = 4 if mode == 1 else 0
    if packed:
        n += 8 * (((h >> 8) & 3) == 2) + 8 * (((h >> 10) & 3) == 2) + 8 * w
    elif mode == 3:
        n += 256
    return n


def stream_records(stream: bytes):
    """Per chunk (hdr_re, hdr_im, record bytes) of a canonical block stream."""
    if len(stream) < 16 or stream[0] != 0x51:
        raise ValueError("not a block stream")
    n_chunks = struct.unpack_from("<I", stream, 12)[0]
    out, o = [], 16
    for _ in range(n_chunks):
        h0, h1 = struct.unpack_from("<II", stream, o)
        size = 8 + _body_bytes(h0, h1) + _body_bytes(h1, h0)
        out.append((h0, h1, size))
        o += size
    if o != len(stream):
        raise ValueError("stream length does not match its records")
    return out


def block_features(stream: bytes, stage_feats) -> np.ndarray:
    """The 32 predictor features of one block (float64)."""
    recs = stream_records(stream)
    nc = len(recs)
    f = np.zeros(32)
    total = sum(r[2] for r in recs)
    f[0] = math.log2(total)
    modes = np.zeros(4)
    wh = np.zeros((2, 8))
    packed = np.zeros(2)
    wsum = np.zeros(2)
    zero = mixed = 0
    for h0, h1, _ in recs:
        zero += (h0 | h1) == 0
        for p, h in enumerate((h0, h1)):
            m, w = h & 3, (h >> 2) & 63
            modes[m] += 1
            if m in (1, 2):
                wh[p, min(w >> 2, 7)] += 1
                packed[p] += 1
                wsum[p] += w
                mixed += ((h >> 8) & 3) == 2
    f[1:5] = modes / (2 * nc)
    f[5:13] = wh[0] / max(packed[0], 1)
    f[13:21] = wh[1] / max(packed[1], 1)
    f[21] = zero / nc
    f[22] = mixed / max(packed.sum(), 1)
    f[23] = wsum[0] / (32 * max(packed[0], 1))
    f[24] = wsum[1] / (32 * max(packed[1], 1))
    f[25:32] = stage_feats
    return f


def block_label(stream: bytes):
    """(log2 stream bytes without the 16-byte header, most frequent plane
    mode with ties to the lower mode)."""
    recs = stream_records(stream)
    modes = np.zeros(4, dtype=np.int64)
    for h0, h1, _ in recs:
        modes[h0 & 3] += 1
        modes[h1 & 3] += 1
    return math.log2(sum(r[2] for r in recs)), int(np.argmax(modes))


def stage_features(stage_gates, b: int, n_ops: int, stage: int, n_stages: int, eb: float,
                   diagonal=("Z", "S", "T", "RZ", "CZ", "CP", "RZZ")) -> np.ndarray:
    """Features 25..31 of a stage: gate counts, global and local qubits,
    fused operations, position in the circuit, error bound."""
    nd = sum(1 for k, _, _ in stage_gates if k not in diagonal)
    dg = len(stage_gates) - nd
    glob = sum(1 for _, q, _ in stage_gates if any(x >= b for x in q))
    local = {x for _, q, _ in stage_gates for x in q if x < b}
    return np.array([nd / 64, dg / 64, glob / 64, len(local) / b, n_ops / 16, stage / n_stages,
                     math.log2(eb) / 32])
