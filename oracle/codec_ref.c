/*
 * CPU reference codec -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is part of the oracle: only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the HIP
 * library and is written to be read against the paper, not to be fast.
 *
 * What it computes (paper Section 4.3, Algorithm 2 and Eqs. 1-2):
 *   - LOG domain: sign bitmap (1 = negative), negate negatives, f(x)=log2(x),
 *     then an absolute-error-bounded lossy encode of f(x) with bound eb.  By
 *     Eq. 2 this gives a point-wise relative bound b_r = 2^eb - 1.
 *     Zeros (and subnormals) cannot go through log2; they are flagged in a
 *     zero bitmap and decode to exactly 0.
 *   - LIN domain: the same lossy encode applied to x itself (the literal
 *     point-wise absolute bound).
 *   - The bitmap pre-scan of Section 4.3: per 64-value chunk the sign and zero
 *     bitmaps are classified all-0 / all-1 / mixed and only mixed chunks keep
 *     their 64-bit mask.
 *   - The lossy encode is a prediction-plus-quantization coder (linear-scaling
 *     quantization with a Lorenzo predictor, the SZ family the paper cites in
 *     Section 2.2) with fixed-length packing per chunk.
 *
 * Quantization step.  The absolute bound eb on f(x) admits any step
 * delta <= 2 eb; the codec takes the largest power of two, delta = 2^-s, so
 * that scaling by 2^s is exact in binary floating point and rounding to the
 * nearest code never leaves an error above delta/2 <= eb.  In the LOG domain
 * the code is formed from the two parts of log2|x| = e + p (e the binary
 * exponent, p = log2 of the significand folded into [sqrt(1/2), sqrt(2)]):
 * k = e 2^s + rint(p 2^s), so log2|x| is never rounded to float32 as a whole.
 *
 * Stream format (little-endian), one "record" per chunk of 64 values of a
 * complex block (two planes: re, im):
 *   u32 hdr_re, u32 hdr_im
 *       hdr bits [1:0] mode (0 ZERO, 1 LZ, 2 Q0, 3 VERBATIM)
 *           bits [7:2] width w (LZ/Q0 only, 0..32)
 *           bits [9:8] sign class (LOG, LZ/Q0 only: 0 all >=0, 1 all <0, 2 mixed)
 *           bits [11:10] zero class (LOG, LZ/Q0 only: 0 none, 2 mixed)
 *   i32 anchor_re   if mode_re == LZ
 *   i32 anchor_im   if mode_im == LZ
 *   u64 sign_re, u64 zero_re, u64 sign_im, u64 zero_im   each only if mixed
 *   payload_re, payload_im: LZ/Q0 -> 64 fields of w bits, LSB-first (8*w
 *       bytes); VERBATIM -> 64 raw float32 (256 bytes); ZERO -> nothing.
 * A block stream is a 16-byte header (u8 0x51, u8 version 1, u8 domain,
 * u8 log2 chunk = 6, u32 eb bits, u32 n_values, u32 n_chunks) followed by the
 * records of its chunks in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CH 64
enum { M_ZERO = 0, M_LZ = 1, M_Q0 = 2, M_VERB = 3 };
enum { DOM_LIN = 0, DOM_LOG = 1 };

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* 2^i for an integer i in the float32 normal range, built from its bits. */
static float pow2i(int i) { return u2f((uint32_t)(i + 127) << 23); }

/* Quantization exponent s: delta = 2^-s is the largest power of two that is
 * <= 2*eb (eb as float32). */
int o_step_shift(float ebf)
{
    int ex;
    (void)frexpf(2.0f * ebf, &ex);   /* 2 eb = m 2^ex, m in [1/2, 1) */
    return 1 - ex;                   /* 2^(ex-1) <= 2 eb < 2^ex */
}

/* Split a positive normal float32 x into log2 x = e + p: the significand m is
 * folded into [sqrt(1/2), sqrt(2)], t = m - 1 (exact), and
 * p = log2(1 + t) ~ t * P(t) with P a degree-8 Chebyshev fit of
 * log2(1+t)/t on that interval, evaluated by Horner's rule with fused
 * multiply-adds and one final rounding of t * P. */
void o_log2_split(float x, int *e_out, float *p_out)
{
    static const float C[9] = {
        1.4426950216293335f, -0.7213473320007324f, 0.48091059923171997f,
        -0.36070483922958374f, 0.2879183292388916f, -0.23892034590244293f,
        0.21566985547542572f, -0.20742103457450867f, 0.12614846229553223f};
    uint32_t u = f2u(x);
    int ef = (int)(u >> 23);
    uint32_t mant = u & 0x007FFFFFu;
    float m;
    if (mant > 0x003504F3u) {           /* 1.mant > sqrt(2): use m/2 */
        m = u2f(mant | 0x3F000000u);
        *e_out = ef - 126;
    } else {
        m = u2f(mant | 0x3F800000u);
        *e_out = ef - 127;
    }
    float t = m - 1.0f;
    float p = C[8];
    for (int i = 7; i >= 0; --i) p = fmaf(p, t, C[i]);
    *p_out = t * p;
}

/* log2 as one float32 (e + p rounded once), for pinning against libm. */
float o_log2(float x)
{
    int e;
    float p;
    o_log2_split(x, &e, &p);
    return (float)e + p;
}

/* 2^f for f in [-1/2, 1/2]: degree-6 Chebyshev fit, Horner with fmaf. */
static float exp2_frac(float f)
{
    static const float E[7] = {
        1.0f, 0.6931471824645996f, 0.24022650718688965f, 0.05550327152013779f,
        0.00961802527308464f, 0.0013400432653725147f, 0.00015469732170458883f};
    float p = E[6];
    for (int k = 5; k >= 0; --k) p = fmaf(p, f, E[k]);
    return p;
}

/* 2^(i + f) with the integer power applied as two exact scalings. */
static float scale2(float p, int i)
{
    if (i < -250) i = -250;
    if (i > 250) i = 250;
    int i1 = i >> 1, i2 = i - i1;
    return (p * pow2i(i1)) * pow2i(i2);
}

/* 2^y for a float32 y (nearest integer i, f = y - i), for pinning. */
float o_exp2(float y)
{
    float fi = rintf(y);
    return scale2(exp2_frac(y - fi), (int)fi);
}

/* magnitude of a LOG-domain code k with step 2^-s: 2^(k 2^-s), with the
 * nearest integer i = round(k / 2^s) taken in integers and the remainder
 * f = (k - i 2^s) 2^-s in [-1/2, 1/2) exact in float32 */
float o_log_decode(int32_t k, int s)
{
    int32_t half = (int32_t)1 << (s - 1);
    int32_t i = (int32_t)(((int64_t)k + half) >> s);
    int32_t r = k - (int32_t)((uint32_t)i << s);
    float f = (float)r * pow2i(-s);
    return scale2(exp2_frac(f), i);
}

static uint32_t zigzag(int32_t d) { return ((uint32_t)d << 1) ^ (d < 0 ? 0xFFFFFFFFu : 0u); }
static int32_t unzigzag(uint32_t z) { return (int32_t)((z >> 1) ^ (0u - (z & 1u))); }
static int bitlen(uint32_t v) { int b = 0; while (v) { ++b; v >>= 1; } return b; }

/* Quantize v with step delta = 2^-s and verify |v - k delta| <= eb in float32
 * (try the neighbour toward v once if not).  Returns 0 on failure (the chunk
 * then falls back to VERBATIM). */
int o_quantize(float v, float ebf, int s, int32_t *kout)
{
    float delta = pow2i(-s), r = pow2i(s);
    float t = v * r;
    if (!(fabsf(t) < 1073741824.0f)) return 0;
    int32_t k = (int32_t)rintf(t);
    float q = (float)k * delta;
    if (!(fabsf(v - q) <= ebf)) {
        k += (v > q) ? 1 : -1;
        q = (float)k * delta;
        if (!(fabsf(v - q) <= ebf)) return 0;
    }
    *kout = k;
    return 1;
}

/* Code of one value; returns 0 if it cannot be coded (VERBATIM), sets *zero
 * for LOG-domain zeros and subnormals. */
static int code_value(float x, int domain, float ebf, int s, int32_t *k, int *zero, int *neg)
{
    *zero = 0;
    *neg = 0;
    *k = 0;
    if (s < -100 || s > 100) return 0;            /* step outside float32's range */
    if (domain == DOM_LIN) return o_quantize(x, ebf, s, k);
    if (s < 1 || s > 22) return 0;                /* LOG codes must fit 30 bits */
    uint32_t u = f2u(x);
    uint32_t ef = (u >> 23) & 0xFFu;
    if (ef == 0) { *zero = 1; return 1; }        /* 0 or subnormal */
    if (ef >= 254) return 0;                     /* |x| >= 2^127, inf, nan */
    *neg = (int)(u >> 31);
    int e;
    float p;
    o_log2_split(u2f(u & 0x7FFFFFFFu), &e, &p);
    int32_t j;
    if (!o_quantize(p, ebf, s, &j)) return 0;
    *k = (int32_t)((uint32_t)e << s) + j;
    return 1;
}

typedef struct {
    uint32_t hdr;
    int32_t anchor;
    int has_smask, has_zmask;
    uint64_t smask, zmask;
    uint32_t fields[CH];   /* zz values (LZ/Q0) or raw bits (VERBATIM) */
    int w;
    int mode;
} plane_rec;

/* Encode one plane of one chunk: x[0..nvalid-1] valid, the rest absent. */
static void encode_plane_chunk(const float *x, int nvalid, int domain, float ebf, int s,
                               plane_rec *out)
{
    int32_t k[CH];
    int zero[CH], neg[CH];
    int ok = 1;
    memset(out, 0, sizeof(*out));
    memset(zero, 0, sizeof(zero));
    memset(neg, 0, sizeof(neg));

    /* 1. transform and quantize (Algorithm 2: sign bitmap, |x|, log2) */
    for (int j = 0; j < nvalid; ++j)
        if (!code_value(x[j], domain, ebf, s, &k[j], &zero[j], &neg[j])) ok = 0;

    /* raw bits for VERBATIM */
    uint32_t raw[CH];
    for (int j = 0; j < CH; ++j) raw[j] = (j < nvalid) ? f2u(x[j]) : 0u;

    if (!ok) {
        out->mode = M_VERB;
        memcpy(out->fields, raw, sizeof(raw));
        out->hdr = M_VERB;
        return;
    }

    /* 2. ZERO test */
    int allzero = 1;
    for (int j = 0; j < nvalid; ++j) {
        if (domain == DOM_LOG) { if (!zero[j]) allzero = 0; }
        else if (k[j] != 0) allzero = 0;
    }
    if (allzero) { out->mode = M_ZERO; out->hdr = 0; return; }

    /* 3. LOG: zeros take the code of the last non-zero value before them (or
     *    of the first non-zero value), so their residual is 0; the pre-scan
     *    classifies the sign and zero bitmaps. */
    int32_t kp[CH];
    int sc = 0, zc = 0;
    uint64_t smask = 0, zmask = 0;
    if (domain == DOM_LOG) {
        int first = -1;
        for (int j = 0; j < nvalid; ++j) if (!zero[j]) { first = j; break; }
        int32_t last = k[first];
        for (int j = 0; j < nvalid; ++j) {
            if (!zero[j]) last = k[j];
            kp[j] = last;
        }
        int nneg = 0, nnz = 0, nz = 0;
        for (int j = 0; j < nvalid; ++j) {
            if (zero[j]) { ++nz; zmask |= (uint64_t)1 << j; }
            else { ++nnz; if (neg[j]) { ++nneg; smask |= (uint64_t)1 << j; } }
        }
        sc = (nneg == 0) ? 0 : (nneg == nnz ? 1 : 2);
        zc = (nz == 0) ? 0 : 2;
    } else {
        for (int j = 0; j < nvalid; ++j) kp[j] = k[j];
    }
    for (int j = nvalid; j < CH; ++j) kp[j] = kp[nvalid - 1];

    /* 4. predictors: Lorenzo (previous value) with anchor, and none (Q0) */
    uint32_t zlz[CH], zq0[CH], orlz = 0, orq0 = 0;
    for (int j = 0; j < CH; ++j) {
        int32_t d = (j == 0) ? 0 : (int32_t)((uint32_t)kp[j] - (uint32_t)kp[j - 1]);
        zlz[j] = zigzag(d);
        zq0[j] = zigzag(kp[j]);
        orlz |= zlz[j];
        orq0 |= zq0[j];
    }
    int wlz = bitlen(orlz), wq0 = bitlen(orq0);
    size_t masks = 8u * (size_t)((sc == 2) + (zc == 2));
    size_t s_lz = 4 + masks + 8u * (size_t)wlz;
    size_t s_q0 = masks + 8u * (size_t)wq0;
    size_t s_vb = 256;

    /* 5. try all, ties broken in the order LZ < Q0 < VERBATIM */
    int mode = M_LZ;
    size_t best = s_lz;
    if (s_q0 < best) { mode = M_Q0; best = s_q0; }
    if (s_vb < best) { mode = M_VERB; best = s_vb; }

    out->mode = mode;
    if (mode == M_VERB) {
        memcpy(out->fields, raw, sizeof(raw));
        out->hdr = M_VERB;
        return;
    }
    out->w = (mode == M_LZ) ? wlz : wq0;
    out->anchor = kp[0];
    memcpy(out->fields, (mode == M_LZ) ? zlz : zq0, sizeof(zlz));
    out->has_smask = (sc == 2);
    out->has_zmask = (zc == 2);
    out->smask = smask;
    out->zmask = zmask;
    out->hdr = (uint32_t)mode | ((uint32_t)out->w << 2) | ((uint32_t)sc << 8) | ((uint32_t)zc << 10);
}

/* Pack 64 fields of w bits LSB-first: field j occupies stream bits
 * [j*w, j*w + w); stream bit p is bit (p mod 8) of byte p/8. */
static void pack_fields(const uint32_t *f, int w, uint8_t *dst)
{
    memset(dst, 0, 8u * (size_t)w);
    for (int j = 0; j < CH; ++j)
        for (int b = 0; b < w; ++b)
            if ((f[j] >> b) & 1u) {
                size_t p = (size_t)j * (size_t)w + (size_t)b;
                dst[p >> 3] |= (uint8_t)(1u << (p & 7));
            }
}

static uint32_t unpack_field(const uint8_t *src, int w, int j)
{
    uint32_t v = 0;
    for (int b = 0; b < w; ++b) {
        size_t p = (size_t)j * (size_t)w + (size_t)b;
        if ((src[p >> 3] >> (p & 7)) & 1u) v |= 1u << b;
    }
    return v;
}

static void put32(uint8_t **p, uint32_t v) { memcpy(*p, &v, 4); *p += 4; }
static void put64(uint8_t **p, uint64_t v) { memcpy(*p, &v, 8); *p += 8; }

/* Encode one complex chunk into dst; returns the record size in bytes. */
size_t o_encode_chunk(const float *re, const float *im, int nvalid, int domain,
                      float ebf, uint8_t *dst)
{
    int s = o_step_shift(ebf);
    plane_rec P[2];
    encode_plane_chunk(re, nvalid, domain, ebf, s, &P[0]);
    encode_plane_chunk(im, nvalid, domain, ebf, s, &P[1]);
    uint8_t *p = dst;
    put32(&p, P[0].hdr);
    put32(&p, P[1].hdr);
    for (int c = 0; c < 2; ++c) if (P[c].mode == M_LZ) put32(&p, (uint32_t)P[c].anchor);
    for (int c = 0; c < 2; ++c) {
        if (P[c].mode != M_LZ && P[c].mode != M_Q0) continue;
        if (P[c].has_smask) put64(&p, P[c].smask);
        if (P[c].has_zmask) put64(&p, P[c].zmask);
    }
    for (int c = 0; c < 2; ++c) {
        if (P[c].mode == M_LZ || P[c].mode == M_Q0) {
            pack_fields(P[c].fields, P[c].w, p);
            p += 8u * (size_t)P[c].w;
        } else if (P[c].mode == M_VERB) {
            for (int j = 0; j < CH; ++j) put32(&p, P[c].fields[j]);
        }
    }
    return (size_t)(p - dst);
}

/* Size of a record from its two headers (format parse, no arithmetic). */
static size_t record_size_from_headers(uint32_t h0, uint32_t h1)
{
    size_t s = 8;
    uint32_t h[2] = {h0, h1};
    for (int c = 0; c < 2; ++c) {
        int mode = (int)(h[c] & 3u), w = (int)((h[c] >> 2) & 63u);
        int sc = (int)((h[c] >> 8) & 3u), zc = (int)((h[c] >> 10) & 3u);
        if (mode == M_LZ) s += 4;
        if (mode == M_LZ || mode == M_Q0) s += 8u * (size_t)((sc == 2) + (zc == 2)) + 8u * (size_t)w;
        if (mode == M_VERB) s += 256;
    }
    return s;
}

/* Decode one record; returns its size, or 0 on a malformed header. */
size_t o_decode_chunk(const uint8_t *src, int nvalid, int domain, float ebf,
                      float *re, float *im)
{
    int s = o_step_shift(ebf);
    float delta = pow2i(-s);
    uint32_t h[2];
    memcpy(&h[0], src, 4);
    memcpy(&h[1], src + 4, 4);
    const uint8_t *p = src + 8;
    int mode[2], w[2], sc[2], zc[2];
    int32_t anchor[2] = {0, 0};
    uint64_t sm[2] = {0, 0}, zm[2] = {0, 0};
    for (int c = 0; c < 2; ++c) {
        mode[c] = (int)(h[c] & 3u);
        w[c] = (int)((h[c] >> 2) & 63u);
        sc[c] = (int)((h[c] >> 8) & 3u);
        zc[c] = (int)((h[c] >> 10) & 3u);
        if (w[c] > 32 || sc[c] == 3 || zc[c] == 1 || zc[c] == 3) return 0;
        if ((h[c] >> 12) != 0) return 0;
        if ((mode[c] == M_ZERO || mode[c] == M_VERB) && (h[c] >> 2) != 0) return 0;
    }
    for (int c = 0; c < 2; ++c) if (mode[c] == M_LZ) { memcpy(&anchor[c], p, 4); p += 4; }
    for (int c = 0; c < 2; ++c) {
        if (mode[c] != M_LZ && mode[c] != M_Q0) continue;
        if (sc[c] == 2) { memcpy(&sm[c], p, 8); p += 8; }
        if (zc[c] == 2) { memcpy(&zm[c], p, 8); p += 8; }
    }
    for (int c = 0; c < 2; ++c) {
        float *x = c ? im : re;
        if (mode[c] == M_ZERO) {
            for (int j = 0; j < nvalid; ++j) x[j] = 0.0f;
        } else if (mode[c] == M_VERB) {
            for (int j = 0; j < CH; ++j) { uint32_t u; memcpy(&u, p + 4 * j, 4); if (j < nvalid) x[j] = u2f(u); }
            p += 256;
        } else {
            int32_t k = anchor[c];
            for (int j = 0; j < CH; ++j) {
                uint32_t z = unpack_field(p, w[c], j);
                int32_t kj;
                if (mode[c] == M_LZ) {
                    if (j > 0) k = (int32_t)((uint32_t)k + (uint32_t)unzigzag(z));
                    kj = k;
                } else {
                    kj = unzigzag(z);
                }
                if (j >= nvalid) continue;
                if (domain == DOM_LIN) {
                    x[j] = (float)kj * delta;
                } else {
                    int isz = (zc[c] == 2) ? (int)((zm[c] >> j) & 1u) : 0;
                    int isn = (sc[c] == 2) ? (int)((sm[c] >> j) & 1u) : (sc[c] == 1);
                    if (isz) x[j] = 0.0f;
                    else { float mag = o_log_decode(kj, s); x[j] = isn ? -mag : mag; }
                }
            }
            p += 8u * (size_t)w[c];
        }
    }
    return (size_t)(p - src);
}

/* Encode a block of n values (planes re, im) into a canonical block stream.
 * Returns the stream size, or 0 if cap is too small. */
size_t o_encode_block(const float *re, const float *im, uint64_t n, int domain,
                      double eb, uint8_t *dst, size_t cap)
{
    float ebf = (float)eb;
    uint64_t nch = (n + CH - 1) / CH;
    uint8_t rec[8 + 8 + 32 + 512];
    if (cap < 16) return 0;
    uint8_t *p = dst;
    uint32_t ebbits = f2u(ebf);
    p[0] = 0x51; p[1] = 1; p[2] = (uint8_t)domain; p[3] = 6;
    memcpy(p + 4, &ebbits, 4);
    uint32_t nv = (uint32_t)n, nc = (uint32_t)nch;
    memcpy(p + 8, &nv, 4);
    memcpy(p + 12, &nc, 4);
    p += 16;
    for (uint64_t c = 0; c < nch; ++c) {
        int nvalid = (int)((n - c * CH) < CH ? (n - c * CH) : CH);
        size_t s = o_encode_chunk(re + c * CH, im + c * CH, nvalid, domain, ebf, rec);
        if ((size_t)(p - dst) + s > cap) return 0;
        memcpy(p, rec, s);
        p += s;
    }
    return (size_t)(p - dst);
}

/* Decode a canonical block stream; returns 0 on success, -1 on malformed. */
int o_decode_block(const uint8_t *src, size_t len, float *re, float *im, uint64_t n)
{
    if (len < 16 || src[0] != 0x51 || src[1] != 1 || src[3] != 6) return -1;
    int domain = src[2];
    uint32_t ebbits, nv, nc;
    memcpy(&ebbits, src + 4, 4);
    memcpy(&nv, src + 8, 4);
    memcpy(&nc, src + 12, 4);
    if (nv != (uint32_t)n || nc != (uint32_t)((n + CH - 1) / CH)) return -1;
    float ebf = u2f(ebbits);
    const uint8_t *p = src + 16;
    for (uint64_t c = 0; c < nc; ++c) {
        if ((size_t)(p - src) + 8 > len) return -1;
        uint32_t h0, h1;
        memcpy(&h0, p, 4);
        memcpy(&h1, p + 4, 4);
        size_t need = record_size_from_headers(h0, h1);
        if ((size_t)(p - src) + need > len) return -1;
        int nvalid = (int)((n - c * CH) < CH ? (n - c * CH) : CH);
        size_t s = o_decode_chunk(p, nvalid, domain, ebf, re + c * CH, im + c * CH);
        if (s == 0 || s != need) return -1;
        p += s;
    }
    return ((size_t)(p - src) == len) ? 0 : -1;
}

/* Per-value quantization codes of one plane, for the code-level parity
 * checks: writes k (0 for LOG zeros) and a "cannot be coded" flag. */
void o_codes(const float *x, uint64_t n, int domain, double eb, int32_t *k, uint8_t *fail)
{
    float ebf = (float)eb;
    int s = o_step_shift(ebf);
    for (uint64_t i = 0; i < n; ++i) {
        int z, ng;
        int32_t kk = 0;
        int ok = code_value(x[i], domain, ebf, s, &kk, &z, &ng);
        k[i] = kk;
        fail[i] = (uint8_t)!ok;
    }
}

/* Vectorised transforms for pinning o_log2/o_exp2 against libm. */
void o_log2_vec(const float *x, float *y, uint64_t n) { for (uint64_t i = 0; i < n; ++i) y[i] = o_log2(x[i]); }
void o_exp2_vec(const float *x, float *y, uint64_t n) { for (uint64_t i = 0; i < n; ++i) y[i] = o_exp2(x[i]); }
void o_log_decode_vec(const int32_t *k, int s, float *y, uint64_t n) { for (uint64_t i = 0; i < n; ++i) y[i] = o_log_decode(k[i], s); }
