"""Pins for the CPU reference codec (CPU only).

The codec follows paper Section 4.3 / Algorithm 2 (sign bitmap, log2
transform, absolute-error-bounded lossy encode, bitmap pre-scan) with an
SZ-style linear-scaling quantizer and Lorenzo predictor.  Pins:

* the own log2/exp2 against libm (error bounds) and exact at powers of two;
* two hand-derived golden records (tests/golden, derivation in its README);
* the point-wise bound: |x'-x| <= eb (LIN) and |x'/x - 1| <= 2^eb - 1 plus
  the transform error (LOG, Eq. 1-2), on random and adversarial inputs;
* the stream layout decoded by an independent pure-Python parser written
  from the format definition;
* try-all optimality: the chosen mode is never larger than any alternative
  sized independently from the per-value codes.
"""
import math
import os
import struct

import numpy as np
import pytest

from oracle import native as N

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LIN, LOG = 0, 1
# Error bounds of the own transforms, each measured exhaustively over every
# float32 its argument can take (tests below): E_LOG2 bounds |p - log2 m| for
# the significand part p of log2|x| = e + p (m = the significand folded into
# [sqrt(1/2), sqrt(2)]; e is exact), E_EXP2 bounds |2^f_own / 2^f - 1| for
# every fraction f = r 2^-s, |r| <= 2^(s-1), s <= 22, that decoding forms.
E_LOG2 = 6.3e-8
E_EXP2 = 8.2e-8


def log_rel_bound(eb, v=0.0):
    """Relative bound of the LOG domain (Eq. 1-2): the code k = e 2^s +
    rint(p 2^s) is within delta/2 <= eb of e + p, p within E_LOG2 of the
    exact significand log, and the decoded 2^(k delta) within E_EXP2
    relative; log2|x| is never rounded as a whole, so the bound does not
    grow with |log2 x| (v is accepted for the call sites and unused)."""
    return 2.0 ** (eb + E_LOG2) * (1 + E_EXP2) - 1


def test_log2_significand_part_exhaustive():
    # every float32 significand in [sqrt(1/2), sqrt(2)]: there e = 0 and the
    # own log2 returns p itself
    lo, hi = np.float32(math.sqrt(0.5)), np.float32(math.sqrt(2.0))
    x = np.arange(lo.view(np.uint32), hi.view(np.uint32) + 1, dtype=np.uint32).view(np.float32)
    err = np.abs(N.log2_own(x).astype(np.float64) - np.log2(x.astype(np.float64)))
    assert err.max() <= E_LOG2
    assert err.max() > 0.5 * E_LOG2          # the constant is the fit's, not a loose guess


def test_exp2_fraction_exhaustive():
    # s = 22 gives every fraction the decoder forms for any s <= 22 (the
    # grid k 2^-s is a subset of the 2^-22 grid)
    s = 22
    k = np.arange(-(1 << (s - 1)), (1 << (s - 1)) + 1, dtype=np.int32)
    y = N.log_decode(k, s).astype(np.float64)
    rel = np.abs(y / np.exp2(k.astype(np.float64) * 2.0 ** -s) - 1)
    assert rel.max() <= E_EXP2 and rel.max() > 0.5 * E_EXP2


def test_log_bound_catches_whole_log2_rounding():
    """Planted mistake (on the CPU): a codec that rounded log2|x| to float32
    as a whole before quantizing -- k = rint(fl32(e + p) 2^s) -- loses up to
    half an ulp of |log2 x| on top of eb.  With eb = delta/2 exactly (eb a
    power of two) and magnitudes down to 2^-40 the pin must reject it."""
    eb = 2.0 ** -17
    s = N.step_shift(eb)
    assert 2.0 ** -s == 2 * eb
    rng = np.random.default_rng(21)
    x = (2.0 ** rng.uniform(-40, -20, 200000)).astype(np.float32)
    v32 = N.log2_own(x)                                  # e + p rounded once
    k_bad = np.rint(v32.astype(np.float64) * 2.0 ** s).astype(np.int32)
    rel_bad = np.abs(N.log_decode(k_bad, s).astype(np.float64) / x - 1)
    assert np.any(rel_bad > log_rel_bound(eb))
    # the codec as defined stays inside the same pin on the same values
    st = N.encode_block(x[:199936], x[:199936][::-1].copy(), LOG, eb)
    r2, _ = N.decode_block(st, 199936)
    assert np.all(np.abs(r2.astype(np.float64) / x[:199936] - 1) <= log_rel_bound(eb))


def test_lin_codes_beyond_2_24_need_no_correction():
    """LIN codes with 2^24 < |k| < 2^30: v 2^s is then an integer-valued
    float32, so rint, the product k 2^-s and the verify step are exact and
    the one-step correction toward v never runs; the codes equal v 2^s."""
    eb = 2.0 ** -20
    s = N.step_shift(eb)
    rng = np.random.default_rng(3)
    k = rng.integers(2 ** 24 + 1, 2 ** 30 - 1, 4096) * rng.choice([-1, 1], 4096)
    x = (k.astype(np.float64) * 2.0 ** -s).astype(np.float32)
    codes, fail = N.codes(x, LIN, eb)
    assert not fail.any()
    assert np.array_equal(codes.astype(np.float64), x.astype(np.float64) * 2.0 ** s)
    assert np.all(np.abs(codes.astype(np.int64)) > 2 ** 24)
    _check_bound(x, x[::-1].copy(), LIN, eb)


def test_log2_exp2_against_libm():
    rng = np.random.default_rng(0)
    x = (2.0 ** rng.uniform(-125, 126, 200000)).astype(np.float32)
    x = x[np.isfinite(x) & (x > 0)]
    v = np.log2(x.astype(np.float64))
    err = np.abs(N.log2_own(x).astype(np.float64) - v)
    # fit error plus one float32 rounding of the result
    assert np.all(err <= E_LOG2 + np.abs(v) * 2.0 ** -24)
    p2 = (2.0 ** np.arange(-126, 127)).astype(np.float32)
    assert np.array_equal(N.log2_own(p2), np.arange(-126, 127).astype(np.float32))
    y = rng.uniform(-120, 120, 200000).astype(np.float32)
    r = np.abs(N.exp2_own(y).astype(np.float64) / np.exp2(y.astype(np.float64)) - 1)
    assert r.max() < E_EXP2
    ints = np.arange(-120, 121).astype(np.float32)
    assert np.array_equal(N.exp2_own(ints), (2.0 ** np.arange(-120, 121)).astype(np.float32))


def _golden(name):
    return bytes.fromhex(open(os.path.join(GOLD, name)).read().strip())


def test_golden_lin_ramp():
    eb = 2.0 ** -10
    re = (np.arange(64) * 2.0 ** -9).astype(np.float32)
    im = np.zeros(64, np.float32)
    s = N.encode_block(re, im, LIN, eb)
    assert s == _golden("lin_ramp_chunk.hex")
    r2, i2 = N.decode_block(s, 64)
    assert np.array_equal(r2, re) and np.array_equal(i2, im)


def test_golden_log_alternating_powers_of_two():
    eb = 2.0 ** -10
    j = np.arange(64)
    re = ((-1.0) ** j * 2.0 ** (-j)).astype(np.float32)
    im = np.zeros(64, np.float32)
    s = N.encode_block(re, im, LOG, eb)
    assert s == _golden("log_alternating_pow2_chunk.hex")
    r2, i2 = N.decode_block(s, 64)
    assert np.array_equal(r2, re) and np.array_equal(i2, im)


def _check_bound(re, im, domain, eb):
    s = N.encode_block(re, im, domain, eb)
    r2, i2 = N.decode_block(s, re.size)
    for x, y in ((re, r2), (im, i2)):
        x64, y64 = x.astype(np.float64), y.astype(np.float64)
        fin = np.isfinite(x64)
        assert np.array_equal(np.isnan(x64), np.isnan(y64))
        if domain == LIN:
            assert np.all(np.abs(x64[fin] - y64[fin]) <= np.float32(eb))
        else:
            tiny = np.abs(x64) < 2.0 ** -126
            # zero class decodes to exactly 0; a VERBATIM chunk keeps the bits
            t = tiny & fin
            assert np.all((y64[t] == 0.0) | (y64[t] == x64[t]))
            m = fin & ~tiny
            rel = np.abs(y64[m] / x64[m] - 1)
            v = np.log2(np.abs(x64[m]))
            assert np.all(rel <= log_rel_bound(float(np.float32(eb)), v))
            assert np.all(np.sign(y64[m]) == np.sign(x64[m]))
    return s


@pytest.mark.parametrize("domain", [LIN, LOG])
@pytest.mark.parametrize("eb", [1e-6, 1e-5, 1e-3, math.log2(1.001), 2.0 ** -17])
def test_pointwise_bound_random(domain, eb):
    rng = np.random.default_rng(int(eb * 1e9) + domain)
    n = 64 * 37 + 13           # several chunks and a ragged tail
    scale = 2.0 ** rng.uniform(-40, 0, n)
    re = (rng.standard_normal(n) * scale).astype(np.float32)
    im = (rng.standard_normal(n) * scale).astype(np.float32)
    _check_bound(re, im, domain, eb)


@pytest.mark.parametrize("domain", [LIN, LOG])
def test_adversarial_inputs(domain):
    eb = 1e-5
    ebf = np.float32(eb)
    delta = np.float32(2) * ebf
    ks = np.arange(-40, 40)
    half = ((ks + 0.5) * delta.astype(np.float64)).astype(np.float32)   # k + 1/2 boundaries
    specials = np.array([0.0, -0.0, 1e-45, -1e-45, 1.1754942e-38, -1.1754942e-38,
                         1.0, -1.0, 0.5, -0.5, 3.4e38, -3.4e38], np.float32)
    alt = np.where(np.arange(64) % 2, 1e-3, -1e-3).astype(np.float32)
    eq = np.full(64, 0.123456, np.float32)
    re = np.concatenate([half, specials, alt, eq, np.zeros(64, np.float32)])
    im = np.concatenate([specials, half, eq, alt, -np.ones(64, np.float32) * 1e-40])
    n = min(re.size, im.size)
    _check_bound(re[:n], im[:n], domain, eb)


def test_zero_and_verbatim_are_exact():
    z = np.zeros(128, np.float32)
    s = N.encode_block(z, z, LOG, 1e-5)
    assert s[16:] == bytes(16)                # two ZERO records of 8 bytes
    x = np.linspace(-1, 1, 64).astype(np.float32)
    x[7] = np.nan
    x[9] = np.inf
    s = N.encode_block(x, x.copy(), LIN, 1e-5)
    h0, h1 = struct.unpack_from("<II", s, 16)
    assert h0 == 3 and h1 == 3                # VERBATIM
    r2, i2 = N.decode_block(s, 64)
    assert np.array_equal(r2.view(np.uint32), x.view(np.uint32))


def test_eq2_relative_bound_regime_of_the_paper():
    # Eq. 2: b_a = log2(1 + b_r); the paper runs b_r = 1e-3
    br = 1e-3
    ba = math.log2(1 + br)
    assert ba == pytest.approx(1.441974e-3, rel=1e-6)
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(4096) * 2.0 ** rng.uniform(-30, 0, 4096)).astype(np.float32)
    s = N.encode_block(x, x[::-1].copy(), LOG, ba)
    r2, _ = N.decode_block(s, x.size)
    rel = np.abs(r2.astype(np.float64) / x - 1)
    assert rel.max() <= br * (1 + 2e-3)


# ---------------------------------------------------------------- parser
def py_parse(stream):
    """Independent pure-Python reading of the block stream format."""
    magic, ver, dom, l2 = stream[:4]
    eb, nv, nc = struct.unpack_from("<fII", stream, 4)
    assert (magic, ver, l2) == (0x51, 1, 6)
    pos = 16
    recs = []
    for _ in range(nc):
        h = struct.unpack_from("<II", stream, pos)
        pos += 8
        planes = []
        for c in range(2):
            planes.append(dict(mode=h[c] & 3, w=(h[c] >> 2) & 63, sc=(h[c] >> 8) & 3, zc=(h[c] >> 10) & 3))
        for c in range(2):
            if planes[c]["mode"] == 1:
                planes[c]["anchor"] = struct.unpack_from("<i", stream, pos)[0]
                pos += 4
        for c in range(2):
            if planes[c]["mode"] in (1, 2):
                if planes[c]["sc"] == 2:
                    planes[c]["smask"] = struct.unpack_from("<Q", stream, pos)[0]
                    pos += 8
                if planes[c]["zc"] == 2:
                    planes[c]["zmask"] = struct.unpack_from("<Q", stream, pos)[0]
                    pos += 8
        for c in range(2):
            p = planes[c]
            if p["mode"] in (1, 2):
                nb = 8 * p["w"]
                bits = int.from_bytes(stream[pos:pos + nb], "little")
                p["fields"] = [(bits >> (j * p["w"])) & ((1 << p["w"]) - 1) for j in range(64)]
                pos += nb
            elif p["mode"] == 3:
                p["raw"] = struct.unpack_from("<64I", stream, pos)
                pos += 256
        recs.append(planes)
    assert pos == len(stream)
    return dom, eb, nv, recs


def unzz(z):
    return (z >> 1) ^ -(z & 1)


def zz(d):
    """zigzag: 0, -1, 1, -2, 2, ... -> 0, 1, 2, 3, 4, ..."""
    return 2 * d if d >= 0 else -2 * d - 1


@pytest.mark.parametrize("domain", [LIN, LOG])
def test_stream_matches_independent_parser_and_codes(domain):
    rng = np.random.default_rng(4 + domain)
    n = 64 * 9
    re = (rng.standard_normal(n) * 1e-3).astype(np.float32)
    im = (rng.standard_normal(n) * 1e-3).astype(np.float32)
    re[64:128] = 0                                 # an all-zero plane chunk
    im[130:140] = 0                                # a mixed-zero chunk
    eb = 1e-5
    s = N.encode_block(re, im, domain, eb)
    dom, ebf, nv, recs = py_parse(s)
    assert dom == domain and nv == n and ebf == np.float32(eb)
    kre, fre = N.codes(re, domain, eb)
    kim, fim = N.codes(im, domain, eb)
    for ci, planes in enumerate(recs):
        for c, (k, x) in enumerate(((kre, re), (kim, im))):
            p = planes[c]
            ks = k[ci * 64:(ci + 1) * 64].astype(np.int64)
            xs = x[ci * 64:(ci + 1) * 64]
            if domain == LOG:
                zero = (xs.view(np.uint32) & 0x7F800000) == 0
            else:
                zero = np.zeros(64, bool)
            if p["mode"] == 0:
                assert np.all(zero) if domain == LOG else np.all(ks == 0)
                continue
            assert p["mode"] in (1, 2)
            # substitute codes of zeros the way the format defines
            nz = np.flatnonzero(~zero)
            kp = ks.copy()
            last = ks[nz[0]]
            for j in range(64):
                if not zero[j]:
                    last = ks[j]
                kp[j] = last
            if p["mode"] == 1:
                dec = p["anchor"] + np.cumsum([0] + [unzz(f) for f in p["fields"][1:]])
            else:
                dec = np.array([unzz(f) for f in p["fields"]])
            assert np.array_equal(dec, kp)
            # try-all: the chosen size is the minimum over the alternatives
            masks = 8 * ((p["sc"] == 2) + (p["zc"] == 2))
            d = np.diff(kp, prepend=kp[0])
            w_lz = max(int(zz(int(v))).bit_length() for v in d)
            w_q0 = max(int(zz(int(v))).bit_length() for v in kp)
            sizes = {1: 4 + masks + 8 * w_lz, 2: masks + 8 * w_q0}
            chosen = sizes[p["mode"]]
            assert chosen <= min(sizes.values()) and chosen <= 256
            assert p["w"] == (w_lz if p["mode"] == 1 else w_q0)
            if domain == LOG:
                negs = (xs.view(np.uint32) >> 31).astype(bool) & ~zero
                smask = sum(1 << j for j in range(64) if negs[j])
                if p["sc"] == 2:
                    assert p["smask"] == smask
                else:
                    assert p["sc"] == (1 if smask else 0)
                zmask = sum(1 << j for j in range(64) if zero[j])
                if p["zc"] == 2:
                    assert p["zmask"] == zmask
                else:
                    assert zmask == 0


def _float_literals(text):
    import re
    return [float(v) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f\b", text)]


def test_polynomial_coefficients_are_the_documented_fit():
    """The oracle's and the device code's log2/exp2 coefficients are the
    float32-rounded least-squares Chebyshev fits that
    tests/golden/fit_codec_polys.py derives (same values on both sides)."""
    import importlib.util
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("fit_codec_polys", os.path.join(here, "golden", "fit_codec_polys.py"))
    fitmod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fitmod)
    logc, expc = fitmod.log2_coefficients(), fitmod.exp2_coefficients()
    assert len(logc) == 9 and len(expc) == 7
    root = os.path.dirname(here)
    oracle = open(os.path.join(root, "oracle", "codec_ref.c")).read()
    c_log = _float_literals(oracle[oracle.index("static const float C[9]"):])[:9]
    c_exp = _float_literals(oracle[oracle.index("static const float E[7]"):])[:7]
    assert c_log == logc and c_exp == expc
    # the device code evaluates the same polynomials by Horner's rule,
    # highest coefficient first
    dev = open(os.path.join(root, "paper_2410_14088_amd", "csrc", "bmq_kernels.hip")).read()
    enc = dev[dev.index("float pp = "):]
    d_log = _float_literals(enc[:enc.index("const uint32_t jb")])
    dec = dev[dev.index("float log_decode_h"):]
    d_exp = _float_literals(dec[dec.index("float p = "):dec.index("__builtin_amdgcn_ldexpf")])
    assert d_log == logc[::-1]
    assert d_exp[0] == expc[6] and d_exp[1:] == expc[5::-1] and len(d_exp) == 7
