// gfx950 kernels of the compressed stage loop.
//
// Layout in HBM (two copies, used in ping-pong by consecutive stages):
//   directory: one u64 per 64-amplitude chunk:
//              bits 39:0  byte offset of the chunk's record body in the pool
//              bits 51:40 header of the real plane, bits 63:52 of the imaginary
//              plane.  0 means an all-zero chunk (both planes ZERO, no body);
//              all ones marks a body lost to a pool overflow.
//   pool:      record bodies appended by workgroups (one atomic bump per tile).
// A header holds mode (1:0: ZERO, LZ, Q0, VERBATIM), width w (7:2), sign class
// (9:8: 0 all >= 0, 1 all < 0, 2 mixed) and zero class (11:10: 0 none, 2
// mixed).  A body holds [i32 anchor_re] [i32 anchor_im] [u64 sign_re]
// [u64 zero_re] [u64 sign_im] [u64 zero_im] payload_re payload_im; LZ/Q0
// payloads are 64 fields of w bits, LSB-first (8w bytes), VERBATIM payloads 64
// raw float32.  The canonical record of a chunk is its two 32-bit headers
// followed by its body.
//
// The codec is the point-wise error-bounded compressor of Section 4.3
// (Algorithm 2): LOG domain = sign bitmap + log2 of the magnitude + absolute
// bound eb on the logarithm (relative bound 2^eb - 1, Eq. 1-2); the bitmap
// pre-scan classifies each 64-bit chunk of the sign/zero bitmaps with wave
// votes and keeps only mixed chunks.  The lossy part is linear-scaling
// quantization with a Lorenzo predictor and fixed-width packing per chunk.
// The quantization step is the largest power of two 2^-s <= 2 eb, so scaling
// is exact; in the LOG domain the code is e 2^s + rint(p 2^s) for
// log2|x| = e + p.  Every float32 step is written out (no contraction, own
// log2 and exp2), so codes and streams are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <stdint.h>

#include "bmq_internal.h"

namespace bmq {

// ------------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// DPP controls of the GFX9 family
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

// inclusive prefix sum over the 64 lanes (wrapping 32-bit arithmetic)
__device__ __forceinline__ uint32_t wave_scan_add(uint32_t v)
{
    v += dpp<DPP_ROW_SHR1, 0xf>(v);
    v += dpp<DPP_ROW_SHR2, 0xf>(v);
    v += dpp<DPP_ROW_SHR4, 0xf>(v);
    v += dpp<DPP_ROW_SHR8, 0xf>(v);
    v += dpp<DPP_ROW_BCAST15, 0xa>(v);
    v += dpp<DPP_ROW_BCAST31, 0xc>(v);
    return v;
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// A wave-uniform 64-bit value made scalar.  readfirstlane returns a signed
// int, so each half is zero-extended explicitly.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | (uint64_t)rfl((uint32_t)v);
}

__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t zigzag(int32_t d) { return ((uint32_t)d << 1) ^ (uint32_t)(d >> 31); }
__device__ __forceinline__ int32_t unzigzag(uint32_t z) { return (int32_t)((z >> 1) ^ (0u - (z & 1u))); }
__device__ __forceinline__ uint32_t bitlen(uint32_t v) { return v ? 32u - (uint32_t)__clz((int)v) : 0u; }

// ------------------------------------------------------------------ codec arithmetic

// 2^(k 2^-s) from kh = k + 2^(s-1): nearest integer i = round(k / 2^s) =
// kh >> s in integers, remainder f = (k - i 2^s) 2^-s in [-1/2, 1/2),
// computed as (kh mod 2^s) 2^-s - 1/2 (both steps exact: a power-of-two
// scaling of an integer below 2^22, then a difference of two multiples of
// 2^-s below 1 in magnitude), 2^f by the degree-6 Chebyshev fit, 2^i
// applied as two exact power-of-two scalings.  The caller adds 2^(s-1) to
// the code (folded into the Lorenzo start for LZ planes).
__device__ __forceinline__ float log_decode_h(int32_t kh, int s, float delta)
{
    // |k| < 2^30 and 1 <= s <= 22, so k + 2^(s-1) cannot overflow 32 bits
    const int32_t i = kh >> s;
    const uint32_t m = (uint32_t)kh & ((1u << s) - 1u);
    const float f = __builtin_fmaf((float)m, delta, -0.5f);
    float p = 0.00015469732170458883f;
    p = __builtin_fmaf(p, f, 0.0013400432653725147f);
    p = __builtin_fmaf(p, f, 0.00961802527308464f);
    p = __builtin_fmaf(p, f, 0.05550327152013779f);
    p = __builtin_fmaf(p, f, 0.24022650718688965f);
    p = __builtin_fmaf(p, f, 0.6931471824645996f);
    p = __builtin_fmaf(p, f, 1.0f);
    // p 2^i rounded once: one v_ldexp_f32.  For i in the normal range this
    // is the exact scaling p * 2^i; beyond it the result is what the two
    // half scalings (p 2^(i/2) exact, then one rounding) give: a subnormal
    // rounded once, zero below, infinity above.
    return __builtin_amdgcn_ldexpf(p, i);
}

// quantize v with step 2^-s and verify |v - k 2^-s| <= eb in float32 (one
// retry toward v); false if the bound cannot be met
__device__ __forceinline__ bool quantize(float v, const CodecParams &cp, int32_t &k)
{
    const float t = v * cp.scale;
    if (!(__builtin_fabsf(t) < 1073741824.0f)) return false;
    int32_t kk = (int32_t)__builtin_rintf(t);
    float q = (float)kk * cp.delta;
    if (!(__builtin_fabsf(v - q) <= cp.ebf)) {
        kk += (v > q) ? 1 : -1;
        q = (float)kk * cp.delta;
        if (!(__builtin_fabsf(v - q) <= cp.ebf)) return false;
    }
    k = kk;
    return true;
}

__device__ __forceinline__ const uint8_t *body_ptr(const uint8_t *dev, const uint8_t *host, uint64_t cap,
                                                   uint64_t off)
{
    return off < cap ? dev + off : host + (off - cap);
}

// bits of v deposited at positions q[0..nq) (bit i of v -> position q[i])
template <class P>
__device__ __forceinline__ uint64_t deposit(uint64_t v, P q, int nq)
{
    uint64_t r = 0;
    for (int i = 0; i < nq; ++i) r |= ((v >> i) & 1ull) << q[i];
    return r;
}

// ------------------------------------------------------------------ fused operations

// Dense 2^K x 2^K complex operation on the LDS tile.  Every thread takes
// groups of 2^K amplitudes whose indices differ only in the operation's bits.
// Read of operation data that no kernel writes while it runs: through the
// constant address space, so that a wave-uniform index becomes a scalar load
// into SGPRs instead of a vector load the compiler hoists into VGPRs.
__device__ __forceinline__ float2 const_ld(const float2 *p, int i)
{
    const __attribute__((address_space(4))) float *c = (const __attribute__((address_space(4))) float *)p;
    return make_float2(c[2 * i], c[2 * i + 1]);
}

// Tile layout in LDS: amplitude e of the tile sits at word e + e / 16, one
// pad word after every 16, so that the four lanes that encode one chunk
// (16 consecutive amplitudes each) and the 16 chunks of a wave hit 64
// different banks.
__device__ __forceinline__ uint32_t tix(uint32_t e) { return e + (e >> 4); }

template <int K, int TILE, int NT>
__device__ __forceinline__ void apply_dense(float *sre, float *sim, const OpDesc &op, const float2 *__restrict__ M,
                                            int tid)
{
    constexpr int D = 1 << K;
    constexpr int UNR = K <= 3 ? D : 1;
    int pos[K], sp[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { pos[j] = op.pos[j]; sp[j] = pos[j]; }
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j + 1 < K - i; ++j)
            if (sp[j] > sp[j + 1]) { const int t = sp[j]; sp[j] = sp[j + 1]; sp[j + 1] = t; }
    // UG groups per step: all their amplitudes are read before any is
    // written, so the LDS reads of a step are issued together instead of one
    // group waiting on the previous group's stores
    constexpr int NG = TILE >> K, IT = (NG + NT - 1) / NT;
    constexpr int UGMAX = K < 4 ? (16 >> K) : 1, UG = IT < UGMAX ? IT : UGMAX;
    static_assert(IT % UG == 0, "whole steps");
#pragma unroll 1
    for (int s0 = 0; s0 < IT; s0 += UG) {
        uint32_t i0[UG];
        bool ok[UG];
        float ar[UG][D], ai[UG][D];
#pragma unroll
        for (int u = 0; u < UG; ++u) {
            const int g = tid + (s0 + u) * NT;
            ok[u] = (NG % NT == 0) || g < NG;
            uint32_t x = (uint32_t)(ok[u] ? g : 0);
#pragma unroll
            for (int j = 0; j < K; ++j) x = ((x >> sp[j]) << (sp[j] + 1)) | (x & ((1u << sp[j]) - 1u));
            i0[u] = x;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                uint32_t o = 0;
#pragma unroll
                for (int j = 0; j < K; ++j) o |= (uint32_t)((c >> j) & 1) << pos[j];
                ar[u][c] = sre[tix(x + o)];
                ai[u][c] = sim[tix(x + o)];
            }
        }
#pragma unroll UNR
        for (int r = 0; r < D; ++r) {
            uint32_t o = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) o |= (uint32_t)((r >> j) & 1) << pos[j];
#pragma unroll
            for (int u = 0; u < UG; ++u) {
                float br = 0.0f, bi = 0.0f;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const float2 m = const_ld(M, r * D + c);
                    br = __builtin_fmaf(m.x, ar[u][c], br);
                    br = __builtin_fmaf(-m.y, ai[u][c], br);
                    bi = __builtin_fmaf(m.x, ai[u][c], bi);
                    bi = __builtin_fmaf(m.y, ar[u][c], bi);
                }
                if (ok[u]) {
                    sre[tix(i0[u] + o)] = br;
                    sim[tix(i0[u] + o)] = bi;
                }
            }
        }
    }
}

// Dense operation of K = 4 or 5 qubits on the matrix cores.  Over a tile the
// operation is the real product [Re out; Im out] = A [Re in; Im in] with the
// 2D x 2D block matrix A = [[Re M, -Im M], [Im M, Re M]] (D = 2^K) and one
// column per group of D amplitudes.  v_mfma_f32_32x32x2_f32 multiplies a
// 32 x 2 slice of A (lane l: row l % 32, column l / 32) by a 2 x 32 slice of
// the columns (lane l: row l / 32, column l % 32) into a 32 x 32 block (lane
// l, register v: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32), full
// float32 arithmetic.  Each wave takes column blocks of 32 groups; a group's
// amplitudes are read from LDS before any of them is written back, and the
// groups of different waves are disjoint, so the update is in place.
typedef float floatx16 __attribute__((ext_vector_type(16)));

// element (i, k) of A for a D x D complex matrix M (row major)
template <int D>
__device__ __forceinline__ float block_elem(const float2 *__restrict__ M, int i, int k)
{
    const int r = i & (D - 1), c = k & (D - 1);
    const float2 m = M[r * D + c];
    if (i < D) return k < D ? m.x : -m.y;
    return k < D ? m.y : m.x;
}

template <int K, int TILE, int NT>
__device__ __forceinline__ void apply_dense_mfma(float *sre, float *sim, const OpDesc &op, const float2 *__restrict__ M,
                                                 int tid)
{
    constexpr int D = 1 << K, G = TILE >> K, RB = 2 * D / 32, STEPS = D;   // row blocks, k-steps of 2
    static_assert(G % 32 == 0, "column blocks of 32 groups");
    const int lane = tid & 63, wave = tid >> 6;
    const int hi = lane >> 5, col = lane & 31;
    int pos[K], sp[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { pos[j] = op.pos[j]; sp[j] = pos[j]; }
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j + 1 < K - i; ++j)
            if (sp[j] > sp[j + 1]) { const int t = sp[j]; sp[j] = sp[j + 1]; sp[j + 1] = t; }
    // amplitude offset of row r of a group: r's bits deposited at the op positions
    auto row_off = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) o |= (uint32_t)((r >> j) & 1) << pos[j];
        return o;
    };
    // NB column blocks at a time give the matrix core independent chains
    // (one 32 x 32 block per instruction chain would wait on each result)
    constexpr int NW = NT / 64;
    constexpr int NB = (RB == 1 && (G / 32) % (2 * NW) == 0) ? 2 : 1;
    for (int cb = wave * 32 * NB; cb < G; cb += NW * 32 * NB) {
        uint32_t base[NB];
        floatx16 acc[NB][RB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            base[u] = (uint32_t)(cb + 32 * u + col);
#pragma unroll
            for (int j = 0; j < K; ++j)
                base[u] = ((base[u] >> sp[j]) << (sp[j] + 1)) | (base[u] & ((1u << sp[j]) - 1u));
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[u][rb][v] = 0.0f;
        }
#pragma unroll 4
        for (int st = 0; st < STEPS; ++st) {
            const int k = 2 * st + hi;                     // k < D exactly when st < D / 2
            const uint32_t ro = row_off(k & (D - 1));
            float bv[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const uint32_t idx = tix(base[u] | ro);
                bv[u] = (st < D / 2) ? sre[idx] : sim[idx];
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float av = block_elem<D>(M, rb * 32 + col, k);
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    acc[u][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[u], acc[u][rb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int i = rb * 32 + 8 * (v >> 2) + 4 * hi + (v & 3);   // output row of A
                    const uint32_t idx = tix(base[u] | row_off(i & (D - 1)));
                    if (i < D) sre[idx] = acc[u][rb][v];
                    else sim[idx] = acc[u][rb][v];
                }
    }
}

// Diagonal operation: multiply every amplitude by a phase from a 2^k table
// staged in LDS.  The table index of amplitude i = tid + m NT splits into a
// per-thread part (bits of tid and the tile-constant bits) and a per-m part
// built from wave-uniform words, so each amplitude costs one OR and a lookup.
template <int T, int NT>
__device__ __forceinline__ void apply_diag(float *sre, float *sim, const OpDesc &op, const float2 *__restrict__ tab, uint64_t base,
                           float2 *s_tab, int tid)
{
    constexpr int TILE = 1 << T;
    constexpr int LNT = __builtin_ctz(NT);
    constexpr int MB = T - LNT;
    const int k = op.k;
    for (int i = tid; i < (1 << k); i += NT) s_tab[i] = tab[i];
    uint32_t it = 0;
    uint32_t W[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) W[b] = 0;
    for (int j = 0; j < k; ++j) {
        const int p = op.pos[j];
        if (p < 0) {
            it |= (uint32_t)((base >> op.gq[j]) & 1ull) << j;
        } else if (p < LNT) {
            it |= (uint32_t)((tid >> p) & 1) << j;
        } else {
#pragma unroll
            for (int b = 0; b < MB; ++b)
                if (p == LNT + b) W[b] |= 1u << j;
        }
    }
    __syncthreads();
    // G amplitudes per step, all read (phase, real, imaginary) before any is
    // written back, so the step's LDS reads are in flight together
    constexpr int M = TILE / NT, G = M < 8 ? M : 8;
#pragma unroll
    for (int m0 = 0; m0 < M; m0 += G) {
        float2 ph[G];
        float ar[G], ai[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int m = m0 + u;
            uint32_t idx = it;
#pragma unroll
            for (int b = 0; b < MB; ++b)
                if ((m >> b) & 1) idx |= W[b];
            const int i = tid + (tid >> 4) + m * (NT + NT / 16);      // tix(tid + m NT), NT a multiple of 16
            ph[u] = s_tab[idx];
            ar[u] = sre[i];
            ai[u] = sim[i];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int i = tid + (tid >> 4) + (m0 + u) * (NT + NT / 16);
            sre[i] = __builtin_fmaf(ph[u].x, ar[u], -ph[u].y * ai[u]);
            sim[i] = __builtin_fmaf(ph[u].x, ai[u], ph[u].y * ar[u]);
        }
    }
}

// ------------------------------------------------------------------ pass kernel
//
// One workgroup = one tile of 2^T amplitudes: qubits 0..5 (one codec chunk)
// plus T-6 more qubits chosen by the planner.  The tile is decoded (or read
// from scratch) into LDS, every fused operation of the pass is applied in
// LDS, and the tile is re-encoded (or written to scratch).  Each wave owns a
// contiguous run of CPW chunks; lane i of a wave stands for its chunk i in
// all per-chunk bookkeeping (directory entries, headers, layouts, offsets), so
// that the bookkeeping of a wave's chunks costs one vector instruction, not
// one scalar sequence per chunk.

// Layout of a record body from its two 12-bit headers (see the file head),
// computed for one chunk per lane.
struct Layout {
    uint32_t m0, m1, w0, w1;                       // modes, widths (w <= 32)
    bool lz0, lz1, hs0, hz0, hs1, hz1;             // anchor / sign mask / zero mask present
    uint32_t off_sm0, off_zm0, off_sm1, off_zm1;   // byte offsets in the body
    uint32_t off_p0, off_p1, size;
};

__device__ __forceinline__ Layout layout_of(uint32_t h0, uint32_t h1)
{
    Layout L;
    L.m0 = h0 & 3u;
    L.m1 = h1 & 3u;
    L.w0 = min((h0 >> 2) & 63u, 32u);
    L.w1 = min((h1 >> 2) & 63u, 32u);
    const bool pk0 = L.m0 == M_LZ || L.m0 == M_Q0, pk1 = L.m1 == M_LZ || L.m1 == M_Q0;
    L.lz0 = L.m0 == M_LZ;
    L.lz1 = L.m1 == M_LZ;
    L.hs0 = pk0 && ((h0 >> 8) & 3u) == 2u;
    L.hz0 = pk0 && ((h0 >> 10) & 3u) == 2u;
    L.hs1 = pk1 && ((h1 >> 8) & 3u) == 2u;
    L.hz1 = pk1 && ((h1 >> 10) & 3u) == 2u;
    uint32_t o = 4u * ((uint32_t)L.lz0 + (uint32_t)L.lz1);
    L.off_sm0 = o; o += 8u * L.hs0;
    L.off_zm0 = o; o += 8u * L.hz0;
    L.off_sm1 = o; o += 8u * L.hs1;
    L.off_zm1 = o; o += 8u * L.hz1;
    L.off_p0 = o; o += (L.m0 == M_VERB) ? 256u : (pk0 ? 8u * L.w0 : 0u);
    L.off_p1 = o; o += (L.m1 == M_VERB) ? 256u : (pk1 ? 8u * L.w1 : 0u);
    L.size = o;
    return L;
}

// ------------------------------------------------------------------ quad-lane encoder
//
// In the pass kernel each chunk is encoded by four consecutive lanes of a
// wave (a quad); lane q holds values 16q..16q+15 and works through them one
// after another.  The chunk-wide facts the format needs (any failed code, any
// non-zero, sign and zero classes, the widest residual) are OR reductions
// over the quad (two DPP quad permutations each), the zero substitution and
// the Lorenzo residual across quarter boundaries need the previous lanes'
// last codes, and every decision is then per lane, so a wave encodes 16
// chunks with no scalar per-chunk work.  The result is byte for byte the
// record encode_plane produces.

// DPP quad permutations: broadcast lane i of the quad, swap neighbours
constexpr int QB0 = 0x00, QB1 = 0x55, QB2 = 0xAA, QB3 = 0xFF, QX1 = 0xB1, QX2 = 0x4E;
constexpr int QPREV = 0x90;     // lane q takes lane q - 1 (lane 0 itself)

template <int CTRL>
__device__ __forceinline__ uint32_t qperm(uint32_t v)
{
    uint32_t r = dpp<CTRL, 0xf>(v);
    // The permuted copy is pinned to its own register: when the compiler
    // folded a DPP move into a following subtraction (v_subrev_u32_dpp) the
    // device returned the negated difference, so only commutative
    // operations may absorb a DPP source.
    asm volatile("" : "+v"(r));
    return r;
}

__device__ __forceinline__ uint32_t quad_or(uint32_t v)
{
    v |= qperm<QX1>(v);
    v |= qperm<QX2>(v);
    return v;
}

struct QuadPlane {
    uint32_t hdr;       // plane header (same in the four lanes)
    int32_t anchor;     // LZ anchor (lane 0)
    uint32_t nzb, negb; // this lane's 16 non-zero / negative bits
    uint32_t w;         // field width
    int32_t kfirst;     // this lane's first code after the zero substitution
    int32_t kp[16];     // after encode_quad: the zigzagged Lorenzo residuals of this lane's codes
                        // (after the zero substitution; residual 0 for the chunk's first value),
                        // or the 16 raw values of a VERBATIM plane
};

// A VERBATIM plane keeps the lane's 16 raw values, in place of its codes.
__device__ __forceinline__ void verbatim_quad(const float *x, QuadPlane &P)
{
    P.hdr = M_VERB;
#pragma unroll
    for (int j = 0; j < 16; ++j) P.kp[j] = (int32_t)__float_as_uint(x[j]);
}

// Encode one plane of a chunk; x points at this lane's 16 values (LDS).
template <int DOM>
__device__ __forceinline__ void encode_quad(const float *x, const CodecParams &cp, int q, QuadPlane &P)
{
    constexpr bool log_dom = DOM == 1;
    if (DOM == 2) {                                    // no compression: every chunk raw
        P.nzb = 0xFFFFu;
        P.negb = 0;
        P.anchor = 0;
        P.w = 0;
        P.kfirst = 0;
        verbatim_quad(x, P);
        return;
    }
    uint32_t nzb = 0xFFFFu, negb = 0, bad = 0, anynz = 0;
    // LOG codes are kept with a constant offset kbias (mod 2^32, below): the
    // Lorenzo residuals do not see it, and the few steps that need a code
    // itself (the chunk's first code, the extremes for Q0) remove it once
    uint32_t kbias = 0;
    if (log_dom) {
        // rint(x 2^s) for |x 2^s| < 2^22 by one rounding addition: x + 1.5
        // 2^(23-s) falls in [2^(23-s), 2^(24-s)), where floats are 2^-s
        // apart, so the sum is x rounded to a multiple of 2^-s (ties to
        // even, as 1.5 2^23 is even) and its bits are ((150 - s) << 23) +
        // 2^22 + rint(x 2^s).  The integer work is uniform (scalar).
        const uint32_t mbits = ((uint32_t)(150 - cp.s) << 23) | 0x00400000u;
        const float magic = __uint_as_float(mbits);
        kbias = (127u << cp.s) + mbits;
        uint32_t amax = 0;
        nzb = 0;
#pragma unroll
        for (int j = 15; j >= 0; --j) {
            const uint32_t u = __float_as_uint(x[j]);
            const uint32_t a = u & 0x7FFFFFFFu;
            amax = max(amax, a);
            // bits j of the masks, shifted in from the top value down:
            // alignbit(m, v, 31) = (m << 1) | (v >> 31); a + 0x7F800000
            // has its top bit set exactly when the exponent field is not
            // zero (zero and subnormals: bit clear)
            nzb = __builtin_amdgcn_alignbit(nzb, a + 0x7F800000u, 31);
            negb = __builtin_amdgcn_alignbit(negb, u, 31);
            // log2|x| = e + p, the significand folded into [sqrt(1/2),
            // sqrt(2)], t = m - 1 exactly and p = t P(t) with P the degree-8
            // Chebyshev fit of log2(1+t)/t (Horner, fused multiply-adds,
            // one final rounding of t P).  Adding 0x4AFB0C carries into
            // the exponent exactly when the significand exceeds 0x3504F3, so
            // one integer add folds the significand into [sqrt(1/2), sqrt(2)]
            const uint32_t ix = a + 0x004AFB0Cu;
            const float t = __uint_as_float((ix & 0x007FFFFFu) + 0x3F3504F4u) - 1.0f;
            float pp = 0.12614846229553223f;
            pp = __builtin_fmaf(pp, t, -0.20742103457450867f);
            pp = __builtin_fmaf(pp, t, 0.21566985547542572f);
            pp = __builtin_fmaf(pp, t, -0.23892034590244293f);
            pp = __builtin_fmaf(pp, t, 0.2879183292388916f);
            pp = __builtin_fmaf(pp, t, -0.36070483922958374f);
            pp = __builtin_fmaf(pp, t, 0.48091059923171997f);
            pp = __builtin_fmaf(pp, t, -0.7213473320007324f);
            pp = __builtin_fmaf(pp, t, 1.4426950216293335f);
            // |t P| <= 1/2, so |t P 2^s| <= 2^21 for s <= 22
            const uint32_t jb = __float_as_uint((t * pp) + magic);
            // code (e << s) + rint(t P 2^s) with e = (ix >> 23) - 127, plus kbias
            P.kp[j] = (int32_t)(((ix >> 23) << cp.s) + jb);   // zeros are substituted below
        }
        negb &= nzb;                                   // zeros count as non-negative
        bad = amax >= 0x7F000000u || !cp.code_ok;      // exponent field 254 or 255
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            int32_t k = 0;
            bad |= !quantize(x[j], cp, k);
            anynz |= k != 0;
            P.kp[j] = k;
        }
        bad |= !cp.code_ok;
    }
    // the lane's first and last non-zero codes (LIN has no zeros)
    int32_t first = P.kp[0], last = P.kp[15];
    const bool seen = nzb != 0u;
    if (nzb != 0xFFFFu) {
        bool sn = false;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if ((nzb >> j) & 1u) {
                first = sn ? first : P.kp[j];
                last = P.kp[j];
                sn = true;
            }
    }
    // chunk facts: bit 0 any failed code, 1 any non-zero code (LIN), 2 any
    // non-zero value, 3 a non-zero value that is not negative (sign class
    // not all-negative); bits 16..31 any zero value, bits 4..15 unused
    const uint32_t zb = ~nzb & 0xFFFFu;
    const uint32_t f = quad_or(bad | (anynz << 1) | ((nzb != 0u) << 2) | ((negb != nzb) << 3) |
                               ((negb != 0u) << 4) | (zb << 16));
    P.nzb = nzb;
    P.negb = negb;
    P.anchor = 0;
    P.w = 0;
    P.kfirst = 0;
    if (f & 1u) { verbatim_quad(x, P); return; }
    const bool allzero = log_dom ? !(f & 4u) : !(f & 2u);
    if (allzero) { P.hdr = M_ZERO; return; }
    // zeros take the code of the last non-zero value at or before them, else
    // the chunk's first non-zero code: carry-in from the previous lanes.
    // Waves whose planes hold no zero (a wave-uniform test) take the
    // previous lane's last code directly (lane 0's carry is never used).
    int32_t carry;
    if (__builtin_amdgcn_ballot_w64(nzb != 0xFFFFu) == 0u) {
        carry = (int32_t)qperm<QPREV>((uint32_t)last);
    } else {
        const uint32_t hs = seen ? 1u : 0u;
        const uint32_t h0 = qperm<QB0>(hs), h1 = qperm<QB1>(hs), h2 = qperm<QB2>(hs);
        const int32_t f0 = (int32_t)qperm<QB0>((uint32_t)first), f1 = (int32_t)qperm<QB1>((uint32_t)first);
        const int32_t f2 = (int32_t)qperm<QB2>((uint32_t)first), f3 = (int32_t)qperm<QB3>((uint32_t)first);
        const int32_t l0 = (int32_t)qperm<QB0>((uint32_t)last), l1 = (int32_t)qperm<QB1>((uint32_t)last);
        const int32_t l2 = (int32_t)qperm<QB2>((uint32_t)last);
        const int32_t cfirst = h0 ? f0 : (h1 ? f1 : (h2 ? f2 : f3));
        carry = cfirst;
        if (q >= 1 && h0) carry = l0;
        if (q >= 2 && h1) carry = l1;
        if (q >= 3 && h2) carry = l2;
    }
    // zigzag(v) grows with |v| on each side of zero, so the widest field of a
    // mode is the zigzag of the smallest or of the largest value
    // from here on the lane keeps its Lorenzo residuals, zigzagged (the LZ
    // fields), in place of its codes; its first code (after the zero
    // substitution) rebuilds the codes if the chunk takes Q0.  The widest
    // field of a mode has the highest bit of the OR of its fields.
    // LOG codes carry kbias and lie in [0, 2^32) as unsigned values in the
    // order of the codes (the offset moves them away from both ends), LIN
    // codes are plain signed values: the extremes are taken in the matching
    // order and the offset removed from them once
    uint32_t kmin = log_dom ? 0xFFFFFFFFu : (uint32_t)INT32_MAX, kmax = log_dom ? 0u : (uint32_t)INT32_MIN;
    uint32_t orl = 0;
    int32_t prev = carry;
    if (nzb != 0xFFFFu) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int32_t kp = ((nzb >> j) & 1u) ? P.kp[j] : prev;
            if (j == 0) P.kfirst = kp;
            const int32_t d = (j == 0 && q == 0) ? 0 : (int32_t)((uint32_t)kp - (uint32_t)prev);
            P.kp[j] = (int32_t)zigzag(d);
            orl |= (uint32_t)P.kp[j];
            if (log_dom) {
                kmin = min(kmin, (uint32_t)kp);
                kmax = max(kmax, (uint32_t)kp);
            } else {
                kmin = (uint32_t)min((int32_t)kmin, kp);
                kmax = (uint32_t)max((int32_t)kmax, kp);
            }
            prev = kp;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int32_t kp = P.kp[j];
            if (j == 0) P.kfirst = kp;
            const int32_t d = (j == 0 && q == 0) ? 0 : (int32_t)((uint32_t)kp - (uint32_t)prev);
            P.kp[j] = (int32_t)zigzag(d);
            orl |= (uint32_t)P.kp[j];
            if (log_dom) {
                kmin = min(kmin, (uint32_t)kp);
                kmax = max(kmax, (uint32_t)kp);
            } else {
                kmin = (uint32_t)min((int32_t)kmin, kp);
                kmax = (uint32_t)max((int32_t)kmax, kp);
            }
            prev = kp;
        }
    }
    P.kfirst = (int32_t)((uint32_t)P.kfirst - kbias);
    const uint32_t orq = zigzag((int32_t)(kmin - kbias)) | zigzag((int32_t)(kmax - kbias));
    const uint32_t wl = bitlen(quad_or(orl)), wq = bitlen(quad_or(orq));
    uint32_t sc = 0, zc = 0;
    if (log_dom) {
        sc = !(f & 16u) ? 0u : ((f & 8u) ? 2u : 1u);
        zc = (f >> 16) ? 2u : 0u;
    }
    const uint32_t masks = 8u * ((sc == 2u) + (zc == 2u));
    const uint32_t s_lz = 4u + masks + 8u * wl, s_q0 = masks + 8u * wq;
    uint32_t mode = M_LZ, best = s_lz;
    if (s_q0 < best) { mode = M_Q0; best = s_q0; }
    if (256u < best) { verbatim_quad(x, P); return; }
    P.w = (mode == M_LZ) ? wl : wq;
    P.hdr = mode | (P.w << 2) | (sc << 8) | (zc << 10);
    P.anchor = P.kfirst;
}

// Decode one plane of a chunk, four lanes per chunk: lane q produces values
// 16q..16q+15 into dst[0..15] (LDS).  Its fields start at bit 16 w q of the
// payload; field j is cut from the two words holding it.  Lorenzo residuals
// are summed within the lane, and the quad's exclusive scan of the lane
// totals plus the anchor gives each lane its starting code.  The same
// integer and float32 steps as decode_value, so the values are identical.
template <int DOM>
__device__ __forceinline__ void decode_quad(uint32_t h, int32_t anchor, const uint8_t *body, uint32_t off_sm,
                                            uint32_t off_zm, uint32_t off_p, float *dst, int q, bool act,
                                            const CodecParams &cp)
{
    const uint32_t mode = h & 3u;
    if (mode == M_ZERO) {
        if (act)
#pragma unroll
            for (int j = 0; j < 16; ++j) dst[j] = 0.0f;
        return;
    }
    const uint32_t *pay = (const uint32_t *)(body + off_p);
    if (mode == M_VERB) {
        if (act)
#pragma unroll
            for (int j = 0; j < 16; ++j) dst[j] = __uint_as_float(pay[16 * q + j]);
        return;
    }
    const uint32_t w = min((h >> 2) & 63u, 32u);
    const uint32_t sc = (h >> 8) & 3u, zc = (h >> 10) & 3u;
    const uint32_t negb = (sc == 2u) ? (uint32_t)*(const uint16_t *)(body + off_sm + 2 * q) : (sc == 1u ? 0xFFFFu : 0u);
    const uint32_t zb = (zc == 2u) ? (uint32_t)*(const uint16_t *)(body + off_zm + 2 * q) : 0u;
    const uint32_t fmask = w >= 32u ? ~0u : ((1u << w) - 1u);
    const uint32_t o = 16u * w * (uint32_t)q;
    int32_t k[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t oj = o + (uint32_t)j * w;
        // word index through an opaque copy, so that the address is one
        // shift and one scaled 64-bit add (left alone, the compiler turns
        // (oj >> 5) * 4 into a shift and a mask before the add)
        uint32_t wi = oj >> 5;
        asm volatile("" : "+v"(wi));
        uint32_t v[2];                                  // the two words holding the field, one load
        __builtin_memcpy(v, pay + wi, 8);
        // the pair shifted right by oj mod 32 (alignbit takes the low 5 bits)
        const uint32_t f = __builtin_amdgcn_alignbit(v[1], v[0], oj) & fmask;
        k[j] = unzigzag(f);
    }
    if (mode == M_LZ) {
        if (q == 0) k[0] = 0;                           // the first residual is the anchor's
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            acc += (uint32_t)k[j];
            k[j] = (int32_t)acc;
        }
        const uint32_t t0 = qperm<QB0>(acc), t1 = qperm<QB1>(acc), t2 = qperm<QB2>(acc);
        // LOG: the 2^(s-1) that log_decode_h expects rides on the start
        uint32_t start = (uint32_t)anchor + (DOM == 1 ? 1u << (cp.s - 1) : 0u);
        if (q >= 1) start += t0;
        if (q >= 2) start += t1;
        if (q >= 3) start += t2;
#pragma unroll
        for (int j = 0; j < 16; ++j) k[j] = (int32_t)(start + (uint32_t)k[j]);
    } else if (DOM == 1) {
#pragma unroll
        for (int j = 0; j < 16; ++j) k[j] = (int32_t)((uint32_t)k[j] + (1u << (cp.s - 1)));
    }
    if (!act) return;
    if (DOM != 1) {
#pragma unroll
        for (int j = 0; j < 16; ++j) dst[j] = (float)k[j] * cp.delta;
        return;
    }
    // the magnitude is positive: the sign bit comes from the sign mask, and
    // a flagged zero clears every bit (+0).  Waves whose planes flag no zero
    // (a wave-uniform test) skip the zero step.
    if (__builtin_amdgcn_ballot_w64(zb != 0u) == 0u) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t mag = __float_as_uint(log_decode_h(k[j], cp.s, cp.delta));
            dst[j] = __uint_as_float(((negb << (31 - j)) & 0x80000000u) | mag);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t mag = __float_as_uint(log_decode_h(k[j], cp.s, cp.delta));
        const uint32_t sgn = negb << (31 - j);
        const uint32_t keep = ~(uint32_t)__builtin_amdgcn_sbfe((int)zb, j, 1);
        dst[j] = __uint_as_float(((sgn & 0x80000000u) | mag) & keep);
    }
}

// The wave's output stream is assembled in LDS before it goes to memory, in
// a staging region whose words are addressed from one base (no per-word
// choice of region).  In the pass kernel the records of the wave's first
// half of chunks go to its tile rows of the real plane and those of the
// second half to its rows of the imaginary plane (free once its chunks are
// encoded); each half holds at most half the chunks' worst-case records.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4 lds_u32x4;
struct Staging {
    lds_u32 *p;          // staging word 0
    __device__ __forceinline__ lds_u32 *word(uint32_t i) const { return p + i; }
};
__device__ __forceinline__ Staging make_staging(uint32_t *st)
{
    return Staging{(lds_u32 *)st};
}

// Stage this lane's part of a plane's payload, which starts at stream word
// pw: packed planes as 16 w-bit fields from bit 16 w q of the payload
// (LSB-first), VERBATIM planes as the 16 raw values from word 16 q.  Field j
// of a packed plane sits at stream bit 32 pw + 16 w q + j w and is ORed into
// the one or two staging words it overlaps (the staging words are zero
// beforehand), so the fields need no per-lane word assembly and a word that
// two neighbouring lanes share needs no merging.  The second OR of a field
// that ends inside its first word adds nothing; its word is at most the
// stream's last word + 1, which still lies in the staging rows.
__device__ __forceinline__ void stage_quad_payload(const QuadPlane &P, const Staging &S, uint32_t pw, int q)
{
    const uint32_t mode = P.hdr & 3u;
    if (mode == M_VERB) {
#pragma unroll
        for (int j = 0; j < 16; ++j) *S.word(pw + 16 * q + j) = (uint32_t)P.kp[j];
        return;
    }
    const uint32_t w = P.w;
    if (mode == M_ZERO || w == 0u) return;
    // bit positions relative to word pw (its multiple of 32 changes no
    // shift): field j at bit 16 w q + j w; Q0 fields are the codes
    // themselves, i.e. residuals against a predecessor of 0
    lds_u32 *const pl = S.p + pw;
    const uint32_t b0 = 16u * w * (uint32_t)q;
    uint32_t fld[16];
    if (mode == M_Q0) {
        // Q0 fields are the codes themselves: rebuilt from the residuals
        uint32_t k = (uint32_t)P.kfirst;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (j) k += (uint32_t)unzigzag((uint32_t)P.kp[j]);
            fld[j] = zigzag((int32_t)k);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) fld[j] = (uint32_t)P.kp[j];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t b = b0 + (uint32_t)j * w;
        const uint64_t t = (uint64_t)fld[j] << (b & 31u);
        uint32_t wi = b >> 5;                           // opaque, as in the decoder: shift + scaled add
        asm volatile("" : "+v"(wi));
        lds_u32 *const wp = pl + wi;
        __hip_atomic_fetch_or(wp, (uint32_t)t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        __hip_atomic_fetch_or(wp + 1, (uint32_t)(t >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
}

// Stage one chunk's record body (anchors, mixed sign / zero masks, both
// payloads) at byte offset rel of the staging area, whose words are zero
// beforehand; the four lanes of the chunk's quad call it together.
__device__ __forceinline__ void stage_record(const QuadPlane &P0, const QuadPlane &P1, const Layout &Lv,
                                             const Staging &S, uint32_t rel, int q)
{
    if (q == 0) {
        if (Lv.lz0) *S.word(rel >> 2) = (uint32_t)P0.anchor;
        if (Lv.lz1) *S.word((rel >> 2) + (Lv.lz0 ? 1 : 0)) = (uint32_t)P1.anchor;
    }
    // each lane stages its 16 bits (bytes 2q, 2q + 1) of the mixed masks
    const uint32_t mw = (uint32_t)q >> 1, mh = (uint32_t)q & 1u;
    if (Lv.hs0) ((lds_u16 *)S.word(((rel + Lv.off_sm0) >> 2) + mw))[mh] = (uint16_t)P0.negb;
    if (Lv.hz0) ((lds_u16 *)S.word(((rel + Lv.off_zm0) >> 2) + mw))[mh] = (uint16_t)(~P0.nzb);
    if (Lv.hs1) ((lds_u16 *)S.word(((rel + Lv.off_sm1) >> 2) + mw))[mh] = (uint16_t)P1.negb;
    if (Lv.hz1) ((lds_u16 *)S.word(((rel + Lv.off_zm1) >> 2) + mw))[mh] = (uint16_t)(~P1.nzb);
    stage_quad_payload(P0, S, (rel + Lv.off_p0) >> 2, q);
    stage_quad_payload(P1, S, (rel + Lv.off_p1) >> 2, q);
}

// Zero staging words [0, nw) (the whole wave, 16 bytes per lane and step).
__device__ __forceinline__ void zero_staging(const Staging &S, uint32_t nw)
{
    for (uint32_t w4 = 4u * (uint32_t)lane_id(); w4 < nw; w4 += 256u) {
        if (w4 + 4u <= nw) *(lds_u32x4 *)S.word(w4) = u32x4{0u, 0u, 0u, 0u};
        else
            for (uint32_t wd = w4; wd < nw; ++wd) *S.word(wd) = 0u;
    }
}

// Copy staging words [0, nw) to dst (4-byte aligned), 16 bytes per lane
// and step (the staging base is 16-byte aligned).
__device__ __forceinline__ void copy_staging(const Staging &S, uint32_t nw, uint32_t *dst)
{
    for (uint32_t w4 = 4u * (uint32_t)lane_id(); w4 < nw; w4 += 256u) {
        if (w4 + 4u <= nw) {
            const u32x4 v = *(const lds_u32x4 *)S.word(w4);
            __builtin_memcpy(dst + w4, &v, 16);
        } else {
            for (uint32_t wd = w4; wd < nw; ++wd) dst[wd] = *S.word(wd);
        }
    }
}

// Decode one chunk record (headers h0, h1; body at `body`) four lanes per
// chunk: lane q writes values 16q..16q+15 of the real plane to dre[0..15]
// and of the imaginary plane to dim[0..15] (LDS or registers).  The one
// decoder of the library: the stage loop, export, sampled amplitudes,
// reductions and the stand-alone codec all decode through it.
template <int DOM>
__device__ __forceinline__ void decode_record(uint32_t h0, uint32_t h1, const uint8_t *body, const CodecParams &cp,
                                              int q, bool act, float *dre, float *dim)
{
    const Layout Lv = layout_of(h0, h1);
    const int32_t an0 = Lv.lz0 ? *(const int32_t *)body : 0;
    const int32_t an1 = Lv.lz1 ? *(const int32_t *)(body + (Lv.lz0 ? 4 : 0)) : 0;
    decode_quad<DOM>(h0, an0, body, Lv.off_sm0, Lv.off_zm0, Lv.off_p0, dre, q, act, cp);
    decode_quad<DOM>(h1, an1, body, Lv.off_sm1, Lv.off_zm1, Lv.off_p1, dim, q, act, cp);
}

// Decode the chunk of directory entry e (a lost chunk reads as zero).
template <int DOM>
__device__ __forceinline__ void decode_entry(uint64_t e, const uint8_t *pool, const uint8_t *host, uint64_t cap,
                                             const CodecParams &cp, int q, bool act, float *dre, float *dim)
{
    if (e == kDirInvalid) e = 0;
    const uint32_t h0 = (uint32_t)(e >> 40) & 0xFFFu, h1 = (uint32_t)(e >> 52);
    decode_record<DOM>(h0, h1, body_ptr(pool, host, cap, e & kDirOffsetMask), cp, q, act, dre, dim);
}

template <int T, int NT>
struct __attribute__((aligned(16))) PassLds {
    static constexpr int TILE = 1 << T, NCH = TILE / kChunk, NW = NT / 64;
    float re[TILE + TILE / 16];           // tile, padded layout (tix)
    float im[TILE + TILE / 16];
    float2 tab[1 << kMaxDiagQubits];      // apply phase: diagonal table
};

__device__ __forceinline__ CodecParams copy_cp(const CodecParams &c) { return c; }

template <class C>
__device__ __forceinline__ CodecParams copy_cp(const C &c)
{
    CodecParams r;
    r.domain = c.domain;
    r.s = c.s;
    r.ebf = c.ebf;
    r.delta = c.delta;
    r.scale = c.scale;
    r.code_ok = c.code_ok;
    return r;
}

// A is PassArgs, or PassArgs in the constant address space (arguments that a
// batched launch reads from device memory with scalar loads)
// DUMP: the test hooks (sv_debug_dump) are compiled in; only the per-pass
// kernel has them (batched, persistent and captured launches refuse dumps)
template <int T, int NT, int DOM, bool DUMP, class A>
__device__ __forceinline__ void pass_body(const A &a, uint32_t tile)
{
    using L = PassLds<T, NT>;
    constexpr int NCH = L::NCH, NW = L::NW, CPW = NCH / NW;
    static_assert(CPW >= 4 && CPW <= 16 && CPW % 4 == 0, "chunks per wave");
    __shared__ L s;

    // the thread index through an opaque copy: when the body runs in a loop
    // over work items, nothing derived from it can be hoisted out of the
    // loop and kept live (and spilled) across items
    uint32_t tid_u;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid_u) : "v"((uint32_t)threadIdx.x));
    const int tid = (int)tid_u;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const CodecParams cp = copy_cp(a.cp);
    const uint64_t base = deposit((uint64_t)tile, a.nontile, a.n_nontile) | a.fixed;
    const int c0 = wave * CPW;


    // ---- load
    if (a.in_mode == IO_COMPRESSED) {
        __builtin_amdgcn_s_setprio(2);                  // the loads leave ahead of other waves' arithmetic
        // four lanes per chunk (see decode_quad)
        const int qc = lane >> 2, q = lane & 3;
        const bool act = qc < CPW;
        const int c = c0 + (act ? qc : 0);
        const uint64_t gch = base | deposit((uint64_t)c, a.tileq + 6, T - 6);
        const uint64_t dch = a.dir_packed ? (deposit((uint64_t)tile, a.snontile, a.n_nontile) |
                                             deposit((uint64_t)c, a.stileq + 6, T - 6)) : gch;
        const uint64_t e = act ? a.dir_in[dch >> 6] : 0ull;
        const uint32_t t0 = tix((uint32_t)(c << 6) + 16u * (uint32_t)q);
        decode_entry<DOM>(e, a.pool_in, a.host_in, a.pool_cap, cp, q, act, s.re + t0, s.im + t0);
        if (DUMP && a.dumpd_re && act && gch - a.dump_lo < a.dump_n) {   // test hook: values as decoded
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                a.dumpd_re[gch - a.dump_lo + 16 * q + j] = s.re[t0 + j];
                a.dumpd_im[gch - a.dump_lo + 16 * q + j] = s.im[t0 + j];
            }
        }
        __builtin_amdgcn_s_setprio(0);
    } else {
        __builtin_amdgcn_s_setprio(2);                  // as for the decoder's loads
        // 16 bytes per lane and plane: lane 16 r + u takes amplitudes
        // 4u..4u+3 of chunk c0 + 4i + r (c0 is a multiple of CPW, itself a
        // multiple of 4, so the chunk index bits of c0, 4i and r are
        // disjoint and deposit separately)
        const int r = lane >> 4, u = lane & 15;
        const uint64_t gl = deposit((uint64_t)tile, a.snontile, a.n_nontile) |
                            deposit((uint64_t)(c0 | r), a.stileq + 6, T - 6);
#pragma unroll
        for (int i = 0; i < CPW / 4; ++i) {
            const uint64_t g = (gl | deposit((uint64_t)(4 * i), a.stileq + 6, T - 6)) + 4u * (uint32_t)u;
            const float4 vr = *(const float4 *)(a.scr_re + g);
            const float4 vi = *(const float4 *)(a.scr_im + g);
            const uint32_t e = tix((uint32_t)((c0 + 4 * i + r) << 6) + 4u * (uint32_t)u);
            s.re[e] = vr.x; s.re[e + 1] = vr.y; s.re[e + 2] = vr.z; s.re[e + 3] = vr.w;
            s.im[e] = vi.x; s.im[e + 1] = vi.y; s.im[e + 2] = vi.z; s.im[e + 3] = vi.w;
        }
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();

    // ---- apply the pass's fused operations
    for (int o = a.op_begin; o < a.op_end; ++o) {
        const OpDesc &op = a.ops[o];
        const float2 *data = a.opdata + op.data;
        if (op.type == OP_DIAG) {
            apply_diag<T, NT>(s.re, s.im, op, data, base, s.tab, tid);
        } else {
            switch (op.k) {
            case 1: apply_dense<1, L::TILE, NT>(s.re, s.im, op, data, tid); break;
            case 2: apply_dense<2, L::TILE, NT>(s.re, s.im, op, data, tid); break;
            case 3: apply_dense<3, L::TILE, NT>(s.re, s.im, op, data, tid); break;
            case 4:
                if (a.mfma) apply_dense_mfma<4, L::TILE, NT>(s.re, s.im, op, data, tid);
                else apply_dense<4, L::TILE, NT>(s.re, s.im, op, data, tid);
                break;
            default:
                if (a.mfma) apply_dense_mfma<5, L::TILE, NT>(s.re, s.im, op, data, tid);
                else apply_dense<5, L::TILE, NT>(s.re, s.im, op, data, tid);
                break;
            }
        }
        __syncthreads();
    }

    // ---- store
    if (a.out_mode == IO_SCRATCH) {
        // 16 bytes per lane and plane, as the scratch load above
        const int r = lane >> 4, u = lane & 15;
        const uint64_t gl = deposit((uint64_t)tile, a.snontile, a.n_nontile) |
                            deposit((uint64_t)(c0 | r), a.stileq + 6, T - 6);
#pragma unroll
        for (int i = 0; i < CPW / 4; ++i) {
            const uint64_t g = (gl | deposit((uint64_t)(4 * i), a.stileq + 6, T - 6)) + 4u * (uint32_t)u;
            const uint32_t e = tix((uint32_t)((c0 + 4 * i + r) << 6) + 4u * (uint32_t)u);
            *(float4 *)(a.scr_re + g) = make_float4(s.re[e], s.re[e + 1], s.re[e + 2], s.re[e + 3]);
            *(float4 *)(a.scr_im + g) = make_float4(s.im[e], s.im[e + 1], s.im[e + 2], s.im[e + 3]);
        }
        return;
    }

    // ---- encode: four lanes per chunk, lane q holding values 16q..16q+15
    // (see encode_quad); one allocation per wave
    const int qc = lane >> 2, q = lane & 3;
    const bool act = qc < CPW;
    const int c = c0 + (act ? qc : 0);
    const uint64_t g = base | deposit((uint64_t)c, a.tileq + 6, T - 6);   // chunk's first amplitude
    const uint64_t dch = a.dir_packed ? (deposit((uint64_t)tile, a.snontile, a.n_nontile) |
                                         deposit((uint64_t)c, a.stileq + 6, T - 6)) : g;   // its directory index
    const uint32_t t0 = tix((uint32_t)(c << 6) + 16u * (uint32_t)q);
    if (DUMP && a.dump_re && act && g - a.dump_lo < a.dump_n) {          // test hook: values about to be encoded
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            a.dump_re[g - a.dump_lo + 16 * q + j] = s.re[t0 + j];
            a.dump_im[g - a.dump_lo + 16 * q + j] = s.im[t0 + j];
        }
    }
    QuadPlane P0, P1;
    encode_quad<DOM>(s.re + t0, cp, q, P0);
    encode_quad<DOM>(s.im + t0, cp, q, P1);
    const uint32_t h0 = act ? P0.hdr : 0u, h1 = act ? P1.hdr : 0u;
    const Layout Lv = layout_of(h0, h1);
    const uint32_t size = (q == 0) ? Lv.size : 0u;
    const uint32_t incl = wave_scan_add(size);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t seg = (a.seg_base + tile * NW + (uint32_t)wave) & (uint32_t)(a.n_seg - 1);
    unsigned long long *cnt = a.counters + seg * C_NUM;
    // the wave's allocation: issued now, its result is needed only for the
    // copy-out, so the record staging below runs while it is in flight
    unsigned long long got = 0;
    if (lane == 0 && total) got = atomicAdd(&cnt[C_CURSOR], (unsigned long long)total);
    // the chunk's body offset in the wave's stream, from its quad's lane 0
    const uint32_t rel = qperm<QB0>(incl - size);
    // assemble the wave's bodies in its own LDS rows: chunks [0, CPW/2) in
    // its rows of the real plane, the rest in its rows of the imaginary
    // plane (record offsets relative to the region's first record)
    constexpr int H = CPW / 2 > 0 ? CPW / 2 : 1;
    static_assert(H * 512 + 4 <= CPW * 68 * 4, "half of the worst-case records fit one plane's rows");
    const uint32_t sh = (uint32_t)__builtin_amdgcn_readlane((int)incl, 4 * H - 1);   // bytes of chunks < H
    const Staging S0 = make_staging((uint32_t *)(s.re + tix((uint32_t)c0 << 6)));
    const Staging S1 = make_staging((uint32_t *)(s.im + tix((uint32_t)c0 << 6)));
    const bool upper = qc >= H;
    if (total) {
        wave_sync_lds();                              // every lane has read its values
        // zero the stream's staging words (the payload fields are ORed in)
        zero_staging(S0, sh >> 2);
        zero_staging(S1, (total - sh) >> 2);
        wave_sync_lds();
        if (act && (h0 | h1)) stage_record(P0, P1, Lv, upper ? S1 : S0, upper ? rel - sh : rel, q);
        wave_sync_lds();
    }
    const uint64_t b = uniform_u64(got);
    uint64_t wave_off = (uint64_t)seg * a.seg_cap + b;       // directory offset of the wave's first body
    bool overflow = false;
    if (total && b + total > a.seg_cap) {
        // segment full: the wave's bodies go to the host pool, or are lost;
        // either way its share of the segment's cursor holds no bytes
        unsigned long long goth = 0;
        if (lane == 0 && a.host_cap) goth = atomicAdd(&a.counters[C_HOST_CURSOR], (unsigned long long)total);
        const uint64_t hb = uniform_u64(goth);
        overflow = !a.host_cap || hb + total > a.host_cap;
        wave_off = a.pool_cap + hb;
        if (lane == 0) {
            atomicAdd(&cnt[C_SPILLED], (unsigned long long)total);
            if (!overflow) atomicAdd(&cnt[C_HOST_BYTES], (unsigned long long)total);
        }
    }
    if (lane == 0 && overflow) atomicOr(&cnt[C_OVERFLOW], 1ull);
    const uint64_t off = wave_off + rel;
    if (!overflow && total) {
        // copy the staged stream out
        uint32_t *dst = (uint32_t *)body_ptr(a.pool_out, a.host_out, a.pool_cap, wave_off);
        copy_staging(S0, sh >> 2, dst);
        copy_staging(S1, (total - sh) >> 2, dst + (sh >> 2));
    }
    if (act && q == 0)
        a.dir_out[dch >> 6] = (h0 | h1) == 0u ? 0ull
                           : (overflow ? kDirInvalid : (off | ((uint64_t)h0 << 40) | ((uint64_t)h1 << 52)));

    // mode histogram: 8-bit counts per mode packed in one word, summed over the wave
    const uint32_t hw = (act && q == 0) ? ((1u << (8 * (h0 & 3u))) + (1u << (8 * (h1 & 3u)))) : 0u;
    const uint32_t zw = (act && q == 0 && (h0 | h1) == 0u) ? 1u : 0u;
    const uint32_t hsum = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_add(hw), 63);
    const uint32_t zsum = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_add(zw), 63);
    // each wave adds its counts to its own segment's counters (no barrier:
    // the waves of a tile finish independently); LZ planes are not counted
    // (the runtime takes them as the rest), so a wave of LZ planes only, the
    // common case, issues none of these atomics
    if (lane == 0) {
        if (zsum) atomicAdd(&cnt[C_ZERO_CHUNKS], (unsigned long long)zsum);
        if (hsum & 0xFFu) atomicAdd(&cnt[C_MODE0], (unsigned long long)(hsum & 0xFFu));
        if (hsum >> 16)
            atomicAdd(&cnt[C_MODE0 + 2], (unsigned long long)((hsum >> 16) & 0xFFu) | ((unsigned long long)(hsum >> 24) << 32));
    }
}

template <int T, int NT, int DOM>
__global__ __launch_bounds__(NT, 1024 / NT) void pass_kernel(PassArgs a)
{
    pass_body<T, NT, DOM, true, PassArgs>(a, blockIdx.x);
}

// One launch over the tiles of several states (independent circuits): state
// i owns blocks [first_block[i], first_block[i + 1]) and its own arguments.
template <int T, int NT, int DOM>
__global__ __launch_bounds__(NT, 1024 / NT) void pass_kernel_batch(const PassArgs *__restrict__ args,
                                                                   const uint32_t *__restrict__ first_block, int n)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first_block[mid] <= blockIdx.x) lo = mid;
        else hi = mid;
    }
    typedef const __attribute__((address_space(4))) PassArgs CArgs;
    pass_body<T, NT, DOM, false, CArgs>(((CArgs *)args)[lo], blockIdx.x - first_block[lo]);
}

// Whole-circuit launch over a work queue: every stage of every circuit in
// one launch.  Each workgroup takes the next (pass, tile-run) item from a
// single device counter, runs it with the same pass body as the per-pass
// launches, and counts its finished items of a pass into that pass's
// done-counter when it moves on to an item of another pass (or runs out of
// items): one release and one atomic per workgroup and pass, not per item.
// An item of a pass that depends on an earlier pass (the previous pass of
// the same circuit) first waits until every item of that pass is counted:
// the per-circuit stage barrier of an atomic done-counter.
// Items are handed out in queue order, only to running workgroups, and a
// dependency always precedes its dependants.  A workgroup publishes its
// finished items before it waits on anything and never waits on a pass it
// holds uncounted items of, and the claim it takes while running an item
// is always later in the queue than that item; so every item a waiting
// workgroup depends on is finished or held by a workgroup that is running
// or about to run it, the earliest unfinished item never waits, and the
// queue always drains whatever number of workgroups is resident.  Every
// wait is bounded (pa.limit_ticks of the constant-rate clock); a wait that
// runs out raises the abort flag, after which every workgroup leaves at its
// next claim or wait, so the grid always finishes.
template <int T, int NT, int DOM>
__global__ __launch_bounds__(NT, 1024 / NT) void pass_kernel_queue(PersistArgs pa)
{
    __shared__ uint32_t s_item, s_go;
    typedef const __attribute__((address_space(4))) PassArgs CArgs;
    uint32_t *const next = pa.sync, *const abort_flag = pa.sync + 1, *const done = pa.sync + kSyncHead;
    int acquired = -1;
    int pend_pass = -1;             // pass of the finished, not yet counted items (same in every thread)
    uint32_t pend_n = 0;
    uint32_t claim = 0;             // thread 0: the next item, claimed while the current one runs
    if (threadIdx.x == 0) claim = atomicAdd(next, 1u);
    for (;;) {
        if (threadIdx.x == 0)
            s_item = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? pa.total : claim;
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();                                // s_item is rewritten only after every thread read it
        int lo = 0;
        if (it < pa.total) {
            int hi = (int)pa.n_pass;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pa.first_item[mid] <= it) lo = mid;
                else hi = mid;
            }
        }
        if (pend_n && (it >= pa.total || lo != pend_pass)) {
            // publish: every wave's records and directory entries of the
            // counted items are visible device-wide (or system-wide) first
            if (pa.system_scope) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0) {
                if (pa.system_scope)
                    __hip_atomic_fetch_add(done + pend_pass, pend_n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                else __hip_atomic_fetch_add(done + pend_pass, pend_n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            pend_n = 0;
        }
        if (it >= pa.total) return;
        const int d = pa.dep[lo];
        if (d >= 0 && d != acquired) {
            if (threadIdx.x == 0) {
                const uint32_t need = pa.first_item[d + 1] - pa.first_item[d];
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                uint32_t go = 1, nap = 1;
                while (__hip_atomic_load(done + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                        __builtin_amdgcn_s_memrealtime() - t0 > pa.limit_ticks) {
                        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        go = 0;
                        break;
                    }
                    for (uint32_t z = 0; z < nap; ++z) __builtin_amdgcn_s_sleep(4);
                    nap = nap < 4u ? 2u * nap : 4u;
                }
                s_go = go;
            }
            __syncthreads();
            if (!s_go) return;
            if (pa.system_scope) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            acquired = d;
        }
        if (threadIdx.x == 0) claim = atomicAdd(next, 1u);
        const uint32_t tpi = pa.tiles_per_item[lo];
        const uint32_t tile0 = (it - pa.first_item[lo]) * tpi;
        for (uint32_t u = 0; u < tpi; ++u) pass_body<T, NT, DOM, false, CArgs>(((CArgs *)pa.args)[lo], tile0 + u);
        pend_pass = lo;
        ++pend_n;
    }
}

// ------------------------------------------------------------------ utility kernels

__global__ void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Per-block statistics of the compressed state, read from the directory
// headers only (no decode): one workgroup per SV block.  Integer counts are
// summed with LDS atomics (exact, so the result does not depend on order) and
// turned into the predictor's 32 features, or into the labels of a block
// (log2 of its stream bytes, most frequent plane mode).
//   features: [0] log2 bytes  [1..4] mode fractions over planes
//             [5..12] / [13..20] width histograms (bins of 4 bits) of the
//             real / imaginary packed planes  [21] all-zero chunk fraction
//             [22] mixed-sign fraction of packed planes  [23], [24] mean
//             width / 32 of packed real / imaginary planes  [25..31] stage
//             features supplied by the host
enum { BS_MODE = 0, BS_WH_RE = 4, BS_WH_IM = 12, BS_PACKED_RE = 20, BS_PACKED_IM = 21, BS_ZERO = 22,
       BS_MIXED = 23, BS_WSUM_RE = 24, BS_WSUM_IM = 25, BS_N = 26 };

__global__ void block_stats_kernel(const uint64_t *dir, uint64_t chunks_per_block, StageFeats sf,
                                   float *feats, float *label_bytes, int32_t *label_mode)
{
    __shared__ uint32_t cnt[BS_N];
    __shared__ unsigned long long body;
    if (threadIdx.x < BS_N) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) body = 0;
    __syncthreads();
    uint32_t c[BS_N];
#pragma unroll
    for (int i = 0; i < BS_N; ++i) c[i] = 0;
    unsigned long long bytes = 0;
    const uint64_t c0 = (uint64_t)blockIdx.x * chunks_per_block;
    for (uint64_t j = threadIdx.x; j < chunks_per_block; j += blockDim.x) {
        uint64_t e = dir[c0 + j];
        if (e == kDirInvalid) e = 0;
        const uint32_t h0 = (uint32_t)(e >> 40) & 0xFFFu, h1 = (uint32_t)(e >> 52);
        const Layout L = layout_of(h0, h1);
        bytes += L.size;
        c[BS_MODE + L.m0]++;
        c[BS_MODE + L.m1]++;
        c[BS_ZERO] += (h0 | h1) == 0u;
        const bool pk0 = L.m0 == M_LZ || L.m0 == M_Q0, pk1 = L.m1 == M_LZ || L.m1 == M_Q0;
        if (pk0) {
            c[BS_WH_RE + min(L.w0 >> 2, 7u)]++;
            c[BS_PACKED_RE]++;
            c[BS_WSUM_RE] += L.w0;
            c[BS_MIXED] += ((h0 >> 8) & 3u) == 2u;
        }
        if (pk1) {
            c[BS_WH_IM + min(L.w1 >> 2, 7u)]++;
            c[BS_PACKED_IM]++;
            c[BS_WSUM_IM] += L.w1;
            c[BS_MIXED] += ((h1 >> 8) & 3u) == 2u;
        }
    }
#pragma unroll
    for (int i = 0; i < BS_N; ++i)
        if (c[i]) atomicAdd(&cnt[i], c[i]);
    if (bytes) atomicAdd(&body, bytes);
    __syncthreads();
    if (threadIdx.x != 0) return;
    // a chunk's record is its two 32-bit headers plus its body
    const double total = (double)body + 8.0 * (double)chunks_per_block;
    const float lb = (float)::log2(total);
    if (label_bytes) {
        uint32_t best = 0;
        for (uint32_t m = 1; m < 4; ++m)
            if (cnt[BS_MODE + m] > cnt[BS_MODE + best]) best = m;
        label_bytes[blockIdx.x] = lb;
        label_mode[blockIdx.x] = (int32_t)best;
    }
    if (feats) {
        float *f = feats + (uint64_t)blockIdx.x * 32u;
        const float planes = (float)(2 * chunks_per_block);
        const float pre = (float)max(cnt[BS_PACKED_RE], 1u), pim = (float)max(cnt[BS_PACKED_IM], 1u);
        f[0] = lb;
        for (int m = 0; m < 4; ++m) f[1 + m] = (float)cnt[BS_MODE + m] / planes;
        for (int i = 0; i < 8; ++i) {
            f[5 + i] = (float)cnt[BS_WH_RE + i] / pre;
            f[13 + i] = (float)cnt[BS_WH_IM + i] / pim;
        }
        f[21] = (float)cnt[BS_ZERO] / (float)chunks_per_block;
        f[22] = (float)cnt[BS_MIXED] / (float)max(cnt[BS_PACKED_RE] + cnt[BS_PACKED_IM], 1u);
        f[23] = (float)cnt[BS_WSUM_RE] / (32.0f * pre);
        f[24] = (float)cnt[BS_WSUM_IM] / (32.0f * pim);
        for (int i = 0; i < 7; ++i) f[25 + i] = sf.v[i];
    }
}

// ------------------------------------------------------------------ directory check
// A directory entry is 0 (an all-zero chunk) or two well-formed plane
// headers for the state's codec domain plus the offset of a record that lies
// inside the pool the offset names (the device pool below cap, else the host
// pool half).  Counts the entries that are neither.
__device__ __forceinline__ bool header_ok(uint32_t h, int domain)
{
    const uint32_t mode = h & 3u, w = (h >> 2) & 63u, sc = (h >> 8) & 3u, zc = (h >> 10) & 3u;
    if (mode == M_ZERO || mode == M_VERB) return (h >> 2) == 0u;
    if (domain == 2) return false;                     // no packed plane without the codec
    if (w > 32u || sc == 3u || zc == 1u || zc == 3u) return false;
    return domain == 1 || (sc | zc) == 0u;             // LIN planes carry no sign or zero class
}

__global__ void check_dir_kernel(const uint64_t *__restrict__ dir, uint64_t n, uint64_t pool_cap, uint64_t host_cap,
                                 int domain, unsigned long long *bad)
{
    unsigned long long nb = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = dir[i];
        if (e == 0) continue;
        const uint32_t h0 = (uint32_t)(e >> 40) & 0xFFFu, h1 = (uint32_t)(e >> 52);
        bool ok = e != kDirInvalid && (h0 | h1) != 0u && header_ok(h0, domain) && header_ok(h1, domain);
        if (ok) {
            const uint64_t off = e & kDirOffsetMask, size = layout_of(h0, h1).size;
            ok = off < pool_cap ? size <= pool_cap - off
                                : (off - pool_cap <= host_cap && size <= host_cap - (off - pool_cap));
        }
        nb += ok ? 0u : 1u;
    }
    if (nb) atomicAdd(bad, nb);
}

// |0...0>: chunk 0 holds amplitude 1 at index 0, encoded by the stage loop's
// quad-lane encoder; every other chunk is zero (directory entry 0, no body).
// One wave.
template <int DOM>
__global__ void init_state_kernel(uint64_t *dir, uint8_t *pool, unsigned long long *counters, CodecParams cp)
{
    __shared__ __align__(16) uint32_t stage[kSlotBytes / 4];
    const int lane = lane_id(), q = lane & 3;
    float xr[16], xi[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        xr[j] = (lane == 0 && j == 0) ? 1.0f : 0.0f;
        xi[j] = 0.0f;
    }
    QuadPlane P0, P1;
    encode_quad<DOM>(xr, cp, q, P0);
    encode_quad<DOM>(xi, cp, q, P1);
    const bool act = lane < 4;
    const uint32_t h0 = act ? P0.hdr : 0u, h1 = act ? P1.hdr : 0u;
    const Layout Lv = layout_of(h0, h1);
    const uint32_t size = rfl(Lv.size);
    const Staging S = make_staging(stage);
    zero_staging(S, kSlotBytes / 4);
    wave_sync_lds();
    if (act && (h0 | h1)) stage_record(P0, P1, Lv, S, 0u, q);
    wave_sync_lds();
    copy_staging(S, size >> 2, (uint32_t *)pool);
    if (lane == 0) {
        dir[0] = (h0 | h1) ? (((uint64_t)h0 << 40) | ((uint64_t)h1 << 52)) : 0ull;
        counters[C_CURSOR] = size;
    }
}

// Loop of a wave over runs of 16 consecutive items (chunks, indices), one
// quad per item: `b0` is the run's first item.
#define BMQ_WAVE_RUNS(b0, n)                                                                                   \
    for (uint64_t b0 = 16ull * ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); b0 < (n);     \
         b0 += 16ull * (uint64_t)gridDim.x * (blockDim.x >> 6))

// Decode chunks [chunk0, chunk0 + n_chunks) into dst (complex64).
template <int DOM>
__global__ void export_kernel(const uint64_t *dir, PoolView pv, CodecParams cp, uint64_t chunk0,
                              uint64_t n_chunks, float2 *dst)
{
    const int lane = lane_id(), q = lane & 3;
    BMQ_WAVE_RUNS(b0, n_chunks) {
        const uint64_t c = b0 + (uint64_t)(lane >> 2);
        const bool act = c < n_chunks;
        float vr[16], vi[16];
        decode_entry<DOM>(act ? dir[chunk0 + c] : 0ull, pv.dev, pv.host, pv.cap, cp, q, act, vr, vi);
        if (act) {
            float2 *o = dst + c * 64 + 16 * q;
#pragma unroll
            for (int j = 0; j < 16; ++j) o[j] = make_float2(vr[j], vi[j]);
        }
    }
}

// Amplitudes at idx[0..k): the quad of index j decodes its chunk and the
// lane holding the amplitude writes it (NaN for an index outside the state).
template <int DOM>
__global__ void amplitudes_kernel(const uint64_t *dir, PoolView pv, CodecParams cp, const uint64_t *idx,
                                  uint64_t k, uint64_t n_chunks, float2 *dst)
{
    const int lane = lane_id(), q = lane & 3;
    BMQ_WAVE_RUNS(b0, k) {
        const uint64_t j = b0 + (uint64_t)(lane >> 2);
        const bool act = j < k;
        const uint64_t x = act ? idx[j] : 0ull;
        const bool inside = (x >> 6) < n_chunks;
        float vr[16], vi[16];
        decode_entry<DOM>(act && inside ? dir[x >> 6] : 0ull, pv.dev, pv.host, pv.cap, cp, q, act && inside, vr, vi);
        const uint32_t sel = (uint32_t)(x & 63u);
        if (act && inside && (int)(sel >> 4) == q) {
            float r = 0.0f, i = 0.0f;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj)
                if ((uint32_t)jj == (sel & 15u)) { r = vr[jj]; i = vi[jj]; }
            dst[j] = make_float2(r, i);
        }
        if (act && !inside && q == 0) dst[j] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
    }
}

// ------------------------------------------------------------------ FP64 reductions
//
// <ref|psi>, |psi|^2, |ref|^2 and max |psi - ref| (componentwise) over
// chunks [chunk0, chunk0 + n_chunks).  The reference is a complex128 array
// (rv.c128, its element 0 = amplitude 64 chunk0) or a second compressed
// state (rv.dir / rv.pv / rv.cp).  Block b adds its five partials into
// partials[5b..5b+4] (the maximum by fmax), so that a host reference can be
// streamed slice by slice; partials are zeroed before the first slice.

__device__ __forceinline__ double wave_sum_f64(double x)
{
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

template <int DOM, int REF, int RDOM>
__global__ __launch_bounds__(256) void fidelity_partial_kernel(const uint64_t *dir, PoolView pv, CodecParams cp,
                                                               uint64_t chunk0, uint64_t n_chunks, RefView rv,
                                                               double *partials)
{
    __shared__ double sh[5][4];
    const int lane = lane_id(), q = lane & 3, wave = (int)(threadIdx.x >> 6);
    double sr = 0, si = 0, np = 0, nr = 0, mx = 0;
    BMQ_WAVE_RUNS(b0, n_chunks) {
        const uint64_t c = b0 + (uint64_t)(lane >> 2);
        const bool act = c < n_chunks;
        float vr[16], vi[16];
        decode_entry<DOM>(act ? dir[chunk0 + c] : 0ull, pv.dev, pv.host, pv.cap, cp, q, act, vr, vi);
        float wr[16], wi[16];
        if (REF == REF_STATE)
            decode_entry<RDOM>(act ? rv.dir[chunk0 + c] : 0ull, rv.pv.dev, rv.pv.host, rv.pv.cap, rv.cp, q, act, wr,
                               wi);
        if (!act) continue;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const double pr = vr[j], pi = vi[j];
            np += pr * pr + pi * pi;
            if (REF != REF_NONE) {
                double rr, ri;
                if (REF == REF_C128) {
                    const double2 r = rv.c128[c * 64 + 16 * q + j];
                    rr = r.x;
                    ri = r.y;
                } else {
                    rr = wr[j];
                    ri = wi[j];
                }
                sr += rr * pr + ri * pi;
                si += rr * pi - ri * pr;
                nr += rr * rr + ri * ri;
                mx = fmax(mx, fmax(fabs(pr - rr), fabs(pi - ri)));
            }
        }
    }
    double v[5] = {sr, si, np, nr, mx};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double x = v[k];
        for (int m = 32; m >= 1; m >>= 1) {
            const double y = __shfl_xor(x, m, 64);
            x = (k == 4) ? fmax(x, y) : x + y;
        }
        if (lane == 0) sh[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int k = (int)threadIdx.x;
        double x = sh[k][0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) x = (k == 4) ? fmax(x, sh[k][w]) : x + sh[k][w];
        double *p = partials + (uint64_t)blockIdx.x * 5 + k;
        *p = (k == 4) ? fmax(*p, x) : *p + x;
    }
}

__global__ void fidelity_final_kernel(const double *partials, int n, double *out5)
{
    if (threadIdx.x < 5) {
        const int q = (int)threadIdx.x;
        double x = partials[q];
        for (int i = 1; i < n; ++i)
            x = (q == 4) ? fmax(x, partials[(uint64_t)i * 5 + q]) : x + partials[(uint64_t)i * 5 + q];
        out5[q] = x;
    }
}

// ------------------------------------------------------------------ sampling x ~ |psi(x)|^2
//
// Two levels: |psi|^2 of each group of chunks_per_group chunks (one
// workgroup per group), then, per sample, a wave walks the chosen group's
// chunks in index order with a running FP64 sum until it passes the
// sample's residual (the host draws the uniforms and picks the group from
// the groups' prefix sums).
template <int DOM>
__global__ __launch_bounds__(256) void group_norm_kernel(const uint64_t *dir, PoolView pv, CodecParams cp,
                                                         uint32_t chunks_per_group, double *gnorm)
{
    __shared__ double sh[4];
    const int lane = lane_id(), q = lane & 3, wave = (int)(threadIdx.x >> 6);
    const uint64_t c0 = (uint64_t)blockIdx.x * chunks_per_group;
    double acc = 0;
    for (uint32_t b0 = 16u * (uint32_t)wave; b0 < chunks_per_group; b0 += 64u) {
        const uint32_t cc = b0 + (uint32_t)(lane >> 2);
        const bool act = cc < chunks_per_group;
        float vr[16], vi[16];
        decode_entry<DOM>(act ? dir[c0 + cc] : 0ull, pv.dev, pv.host, pv.cap, cp, q, act, vr, vi);
        if (act)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc += (double)vr[j] * vr[j] + (double)vi[j] * vi[j];
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) sh[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) gnorm[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <int DOM>
__global__ __launch_bounds__(256) void sample_kernel(const uint64_t *dir, PoolView pv, CodecParams cp,
                                                     uint32_t chunks_per_group, const uint32_t *grp,
                                                     const double *resid, uint64_t k, uint64_t *out)
{
    const int lane = lane_id(), q = lane & 3;
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t i = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < k; i += nw) {
        const uint64_t c0 = (uint64_t)grp[i] * chunks_per_group;
        const double r = resid[i];
        double acc = 0;
        uint64_t pick = c0 * 64, last_nz = c0 * 64;
        bool found = false;
        for (uint32_t b0 = 0; b0 < chunks_per_group && !found; b0 += 16u) {
            const uint32_t cc = b0 + (uint32_t)(lane >> 2);
            const bool act = cc < chunks_per_group;
            float vr[16], vi[16];
            decode_entry<DOM>(act ? dir[c0 + cc] : 0ull, pv.dev, pv.host, pv.cap, cp, q, act, vr, vi);
            double p[16], s = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                p[j] = act ? (double)vr[j] * vr[j] + (double)vi[j] * vi[j] : 0.0;
                s += p[j];
            }
            // inclusive scan of the lane sums in lane order (= amplitude order)
            double incl = s;
            for (int d = 1; d < 64; d <<= 1) {
                const double y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            const double tot = __shfl(incl, 63, 64);
            const uint64_t base = (c0 + cc) * 64 + 16u * (uint32_t)q;
            if (acc + tot > r) {
                const uint64_t over = __ballot(acc + incl > r);
                const int L = __ffsll((long long)over) - 1;
                uint64_t mine = base;
                if (lane == L) {
                    double a2 = acc + (incl - s);
                    int hit = -1, lastp = 0;
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        a2 += p[j];
                        if (p[j] > 0.0) lastp = j;
                        if (hit < 0 && a2 > r) hit = j;
                    }
                    mine = base + (uint64_t)(hit >= 0 ? hit : lastp);
                }
                pick = __shfl(mine, L, 64);
                found = true;
            } else {
                const uint64_t nzl = __ballot(s > 0.0);
                if (nzl) {
                    const int Lh = 63 - __clzll((long long)nzl);
                    int lastp = 0;
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        if (p[j] > 0.0) lastp = j;
                    last_nz = __shfl(base + (uint64_t)lastp, Lh, 64);
                }
                acc += tot;
            }
        }
        if (lane == 0) out[i] = found ? pick : last_nz;
    }
}

// ------------------------------------------------------------------ stand-alone codec
//
// The stage loop's encoder and decoder on caller arrays of whole chunks.
// Slot form: chunk i's record (its two 32-bit headers, then its body) at
// slots + i kSlotBytes.  Stream form: the canonical block stream -- a
// 16-byte header (u8 0x51, u8 version 1, u8 domain, u8 log2 chunk = 6,
// u32 eb bits, u32 n_values, u32 n_chunks) followed by the records in chunk
// order.

__device__ __forceinline__ void load16(const float *p, bool act, float *x)
{
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = act ? p[j] : 0.0f;
}

template <int DOM>
__global__ __launch_bounds__(256) void codec_slots_encode_kernel(const float *re, const float *im, uint64_t nch,
                                                                 CodecParams cp, uint8_t *slots, uint32_t *sizes)
{
    constexpr uint32_t SW = kSlotBytes / 4;                 // words per slot
    __shared__ __align__(16) uint32_t stage[4][16 * SW];
    const int lane = lane_id(), q = lane & 3, qc = lane >> 2, wave = (int)(threadIdx.x >> 6);
    const Staging S = make_staging(stage[wave]);
    BMQ_WAVE_RUNS(b0, nch) {
        const uint64_t c = b0 + (uint64_t)qc;
        const bool act = c < nch;
        float xr[16], xi[16];
        load16(re + c * 64 + 16 * q, act, xr);
        load16(im + c * 64 + 16 * q, act, xi);
        QuadPlane P0, P1;
        encode_quad<DOM>(xr, cp, q, P0);
        encode_quad<DOM>(xi, cp, q, P1);
        const uint32_t h0 = act ? P0.hdr : 0u, h1 = act ? P1.hdr : 0u;
        const Layout Lv = layout_of(h0, h1);
        wave_sync_lds();                                    // the previous run's copy-out is done
        zero_staging(S, 16 * SW);
        wave_sync_lds();
        if (act && q == 0) {
            *S.word((uint32_t)qc * SW) = h0;
            *S.word((uint32_t)qc * SW + 1u) = h1;
        }
        if (act && (h0 | h1)) stage_record(P0, P1, Lv, S, (uint32_t)qc * kSlotBytes + 8u, q);
        wave_sync_lds();
        const uint64_t nv = nch - b0 < 16 ? nch - b0 : 16;
        copy_staging(S, (uint32_t)nv * SW, (uint32_t *)(slots + b0 * kSlotBytes));
        if (act && q == 0) sizes[c] = 8u + Lv.size;
    }
}

template <int DOM>
__global__ __launch_bounds__(256) void codec_slots_decode_kernel(const uint8_t *slots, uint64_t nch, CodecParams cp,
                                                                 float *re, float *im)
{
    const int lane = lane_id(), q = lane & 3;
    BMQ_WAVE_RUNS(b0, nch) {
        const uint64_t c = b0 + (uint64_t)(lane >> 2);
        const bool act = c < nch;
        const uint8_t *rec = slots + (act ? c : 0) * kSlotBytes;
        const uint32_t h0 = act ? (*(const uint32_t *)rec & 0xFFFu) : 0u;
        const uint32_t h1 = act ? (*(const uint32_t *)(rec + 4) & 0xFFFu) : 0u;
        float vr[16], vi[16];
        decode_record<DOM>(h0, h1, rec + 8, cp, q, act, vr, vi);
        if (act)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                re[c * 64 + 16 * q + j] = vr[j];
                im[c * 64 + 16 * q + j] = vi[j];
            }
    }
}

// stream pass 1: record bytes (headers + body) of every chunk
template <int DOM>
__global__ __launch_bounds__(256) void codec_size_kernel(const float *re, const float *im, uint64_t nch,
                                                         CodecParams cp, uint32_t *sizes)
{
    const int lane = lane_id(), q = lane & 3;
    BMQ_WAVE_RUNS(b0, nch) {
        const uint64_t c = b0 + (uint64_t)(lane >> 2);
        const bool act = c < nch;
        float xr[16], xi[16];
        load16(re + c * 64 + 16 * q, act, xr);
        load16(im + c * 64 + 16 * q, act, xi);
        QuadPlane P0, P1;
        encode_quad<DOM>(xr, cp, q, P0);
        encode_quad<DOM>(xi, cp, q, P1);
        const Layout Lv = layout_of(act ? P0.hdr : 0u, act ? P1.hdr : 0u);
        if (act && q == 0) sizes[c] = 8u + Lv.size;
    }
}

// exclusive prefix sum of sizes[0..n) into off[0..n), the total into off[n];
// one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void scan_sizes_kernel(const uint32_t *sizes, uint64_t n, uint64_t *off)
{
    __shared__ uint32_t wsum[16];
    __shared__ unsigned long long carry;
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t base = 0; base < n; base += 1024) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < n ? sizes[i] : 0u;
        const uint32_t incl = wave_scan_add(v);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < 16; ++w) {
            before += w < wave ? wsum[w] : 0u;
            all += wsum[w];
        }
        const unsigned long long cbase = carry;
        if (i < n) off[i] = cbase + before + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = cbase + all;
        __syncthreads();
    }
    if (threadIdx.x == 0) off[n] = carry;
}

// stream pass 2: each wave stages the records of its 16 chunks (contiguous
// in the stream) and copies them to their place; nothing is written when
// the stream does not fit cap bytes
template <int DOM>
__global__ __launch_bounds__(256) void codec_write_kernel(const float *re, const float *im, uint64_t nch,
                                                          CodecParams cp, const uint64_t *off, uint8_t *dst,
                                                          uint64_t cap, uint32_t ebbits)
{
    constexpr uint32_t SW = kSlotBytes / 4;
    __shared__ __align__(16) uint32_t stage[4][16 * SW];
    if (16u + off[nch] > cap) return;
    const int lane = lane_id(), q = lane & 3, qc = lane >> 2, wave = (int)(threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        uint32_t *h = (uint32_t *)dst;
        h[0] = 0x51u | (1u << 8) | ((uint32_t)DOM << 16) | (6u << 24);
        h[1] = ebbits;
        h[2] = (uint32_t)(nch * 64);
        h[3] = (uint32_t)nch;
    }
    const Staging S = make_staging(stage[wave]);
    BMQ_WAVE_RUNS(b0, nch) {
        const uint64_t c = b0 + (uint64_t)qc;
        const bool act = c < nch;
        float xr[16], xi[16];
        load16(re + c * 64 + 16 * q, act, xr);
        load16(im + c * 64 + 16 * q, act, xi);
        QuadPlane P0, P1;
        encode_quad<DOM>(xr, cp, q, P0);
        encode_quad<DOM>(xi, cp, q, P1);
        const uint32_t h0 = act ? P0.hdr : 0u, h1 = act ? P1.hdr : 0u;
        const Layout Lv = layout_of(h0, h1);
        const uint32_t rsz = (act && q == 0) ? 8u + Lv.size : 0u;
        const uint32_t incl = wave_scan_add(rsz);
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        const uint32_t rel = qperm<QB0>(incl - rsz);
        wave_sync_lds();
        zero_staging(S, total >> 2);
        wave_sync_lds();
        if (act && q == 0) {
            *S.word(rel >> 2) = h0;
            *S.word((rel >> 2) + 1u) = h1;
        }
        if (act && (h0 | h1)) stage_record(P0, P1, Lv, S, rel + 8u, q);
        wave_sync_lds();
        copy_staging(S, total >> 2, (uint32_t *)(dst + 16 + uniform_u64(off[b0])));
    }
}

// One lane walks the stream's records (a record's size follows from its two
// headers) and writes each chunk's record offset; *bad is set when a header
// is malformed for the domain or a record does not lie inside the stream.
__global__ void codec_walk_kernel(const uint8_t *src, uint64_t bytes, uint64_t nch, int domain, uint64_t *off,
                                  uint32_t *bad)
{
    if (threadIdx.x != 0) return;
    uint64_t o = 16;
    for (uint64_t c = 0; c < nch; ++c) {
        if (o + 8 > bytes) { *bad = 1u; return; }
        const uint32_t h0 = *(const uint32_t *)(src + o), h1 = *(const uint32_t *)(src + o + 4);
        if ((h0 >> 12) || (h1 >> 12) || !header_ok(h0, domain) || !header_ok(h1, domain)) { *bad = 1u; return; }
        off[c] = o;
        o += 8u + layout_of(h0, h1).size;
    }
    if (o != bytes) *bad = 1u;
}

template <int DOM>
__global__ __launch_bounds__(256) void codec_read_kernel(const uint8_t *src, const uint64_t *off, uint64_t nch,
                                                         CodecParams cp, float *re, float *im)
{
    const int lane = lane_id(), q = lane & 3;
    BMQ_WAVE_RUNS(b0, nch) {
        const uint64_t c = b0 + (uint64_t)(lane >> 2);
        const bool act = c < nch;
        const uint8_t *rec = src + (act ? off[c] : 16ull);
        const uint32_t h0 = act ? *(const uint32_t *)rec : 0u, h1 = act ? *(const uint32_t *)(rec + 4) : 0u;
        float vr[16], vi[16];
        decode_record<DOM>(h0, h1, rec + 8, cp, q, act, vr, vi);
        if (act)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                re[c * 64 + 16 * q + j] = vr[j];
                im[c * 64 + 16 * q + j] = vi[j];
            }
    }
}

// ------------------------------------------------------------------ launchers

static inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap = 65536)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_pass(const PassArgs &a, hipStream_t s)
{
    const uint64_t tiles = 1ull << a.n_nontile;
    if (tiles > 0x7FFFFFFFull) return hipErrorInvalidValue;
    const dim3 grid((unsigned)tiles);
    const int key = a.t * 3 + a.cp.domain;
    switch (key) {
#define BMQ_PASS(T, NT, D) \
    case T * 3 + D: hipLaunchKernelGGL((pass_kernel<T, NT, D>), grid, dim3(NT), 0, s, a); break;
    BMQ_PASS(10, 256, 0) BMQ_PASS(10, 256, 1) BMQ_PASS(10, 256, 2)
    BMQ_PASS(11, 256, 0) BMQ_PASS(11, 256, 1) BMQ_PASS(11, 256, 2)
    BMQ_PASS(12, 256, 0) BMQ_PASS(12, 256, 1) BMQ_PASS(12, 256, 2)
    BMQ_PASS(13, 512, 0) BMQ_PASS(13, 512, 1) BMQ_PASS(13, 512, 2)
#undef BMQ_PASS
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pass_queue(int t, int domain, const PersistArgs &pa, hipStream_t s)
{
    if (pa.total == 0) return hipSuccess;
    const dim3 grid(std::min(pa.total, pa.max_grid));
    switch (t * 3 + domain) {
#define BMQ_PASS(T, NT, D) \
    case T * 3 + D: hipLaunchKernelGGL((pass_kernel_queue<T, NT, D>), grid, dim3(NT), 0, s, pa); break;
    BMQ_PASS(10, 256, 0) BMQ_PASS(10, 256, 1) BMQ_PASS(10, 256, 2)
    BMQ_PASS(11, 256, 0) BMQ_PASS(11, 256, 1) BMQ_PASS(11, 256, 2)
    BMQ_PASS(12, 256, 0) BMQ_PASS(12, 256, 1) BMQ_PASS(12, 256, 2)
    BMQ_PASS(13, 512, 0) BMQ_PASS(13, 512, 1) BMQ_PASS(13, 512, 2)
#undef BMQ_PASS
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pass_batch(int t, int domain, const PassArgs *args_dev, const uint32_t *first_block_dev, int n,
                             uint32_t blocks, hipStream_t s)
{
    const dim3 grid(blocks);
    const int key = t * 3 + domain;
    switch (key) {
#define BMQ_PASS(T, NT, D) \
    case T * 3 + D: \
        hipLaunchKernelGGL((pass_kernel_batch<T, NT, D>), grid, dim3(NT), 0, s, args_dev, first_block_dev, n); \
        break;
    BMQ_PASS(10, 256, 0) BMQ_PASS(10, 256, 1) BMQ_PASS(10, 256, 2)
    BMQ_PASS(11, 256, 0) BMQ_PASS(11, 256, 1) BMQ_PASS(11, 256, 2)
    BMQ_PASS(12, 256, 0) BMQ_PASS(12, 256, 1) BMQ_PASS(12, 256, 2)
    BMQ_PASS(13, 512, 0) BMQ_PASS(13, 512, 1) BMQ_PASS(13, 512, 2)
#undef BMQ_PASS
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_check_dir(const uint64_t *dir, uint64_t n, uint64_t pool_cap, uint64_t host_cap, int domain,
                            unsigned long long *bad, hipStream_t s)
{
    hipLaunchKernelGGL(check_dir_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, dir, n, pool_cap, host_cap,
                       domain, bad);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ group staging (host-resident pipeline)

__global__ void rebase_dir_kernel(uint64_t *dir, uint64_t n, uint32_t cpb, const uint64_t *body_off)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = dir[i];
        if (e) dir[i] = e + body_off[i / cpb];
    }
}

// body bytes of a chunk from its directory entry
__device__ __forceinline__ uint32_t entry_body_bytes(uint64_t e)
{
    if (e == 0) return 0;
    return layout_of((uint32_t)(e >> 40) & 0xFFFu, (uint32_t)(e >> 52)).size;
}

// one workgroup (256 threads) per segment of seg <= 1024 chunks; thread t
// takes chunks 4t..4t+3 of the segment
__global__ __launch_bounds__(256) void pack_sizes_kernel(const uint64_t *dir, uint64_t n, uint32_t seg, uint32_t *rel,
                                                         uint64_t *segsum)
{
    __shared__ uint32_t s_wave[4];
    const uint64_t c0 = (uint64_t)blockIdx.x * seg;
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    uint32_t sz[4], tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t i = 4u * t + (uint32_t)k;
        sz[k] = (i < seg && c0 + i < n) ? entry_body_bytes(dir[c0 + i]) : 0u;
        tot += sz[k];
    }
    const uint32_t incl = wave_scan_add(tot);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t off = incl - tot;
    for (uint32_t w = 0; w < wave; ++w) off += s_wave[w];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t i = 4u * t + (uint32_t)k;
        if (i < seg && c0 + i < n) rel[c0 + i] = off;
        off += sz[k];
    }
    if (t == 255) segsum[blockIdx.x] = off;
}

// one thread: the segments of each block scanned in place, then the images
__global__ void pack_offsets_kernel(uint64_t *segsum, uint32_t cpb, uint32_t seg, uint32_t n_blocks, uint64_t *img_off)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const uint32_t spb = cpb / seg;
    uint64_t img = 0;
    for (uint32_t j = 0; j < n_blocks; ++j) {
        uint64_t acc = 0;
        for (uint32_t k = 0; k < spb; ++k) {
            const uint64_t v = segsum[(uint64_t)j * spb + k];
            segsum[(uint64_t)j * spb + k] = acc;
            acc += v;
        }
        img_off[j] = img;
        img_off[n_blocks + 1 + j] = acc;
        img += (8ull * cpb + acc + 15ull) & ~15ull;
    }
    img_off[n_blocks] = img;
}

// four lanes per chunk: lane 0 writes the image's directory entry, the quad
// copies the body word by word
__global__ __launch_bounds__(256) void pack_write_kernel(const uint64_t *dir, const uint8_t *pool, uint32_t cpb,
                                                         uint32_t seg, uint64_t n, const uint32_t *rel,
                                                         const uint64_t *segsum, const uint64_t *img_off, uint8_t *img)
{
    const uint64_t c = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const uint32_t q = threadIdx.x & 3u;
    if (c >= n) return;
    const uint64_t e = dir[c];
    const uint64_t j = c / cpb, cl = c % cpb;
    const uint64_t r = segsum[c / seg] + rel[c];                 // body offset within the block's body area
    uint8_t *const im = img + img_off[j];
    if (q == 0) ((uint64_t *)im)[cl] = e ? ((e & ~kDirOffsetMask) | r) : 0ull;
    const uint32_t nb = entry_body_bytes(e);
    const uint32_t *src = (const uint32_t *)(pool + (e & kDirOffsetMask));
    uint32_t *dst = (uint32_t *)(im + 8ull * cpb + r);
    for (uint32_t w = q; w < nb / 4u; w += 4u) dst[w] = src[w];
}

hipError_t launch_rebase_dir(uint64_t *dir, uint64_t n_entries, uint32_t chunks_per_block, const uint64_t *body_off,
                             hipStream_t s)
{
    if (n_entries == 0) return hipSuccess;
    hipLaunchKernelGGL(rebase_dir_kernel, dim3(grid_for(n_entries, 256, 16384)), dim3(256), 0, s, dir, n_entries,
                       chunks_per_block, body_off);
    return hipGetLastError();
}

hipError_t launch_pack_sizes(const uint64_t *dir, uint64_t n_chunks, uint32_t seg, uint32_t *rel, uint64_t *segsum,
                             hipStream_t s)
{
    if (seg == 0 || seg > 1024 || n_chunks % seg) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pack_sizes_kernel, dim3((unsigned)(n_chunks / seg)), dim3(256), 0, s, dir, n_chunks, seg, rel,
                       segsum);
    return hipGetLastError();
}

hipError_t launch_pack_offsets(uint64_t *segsum, uint32_t chunks_per_block, uint32_t seg, uint32_t n_blocks,
                               uint64_t *img_off, hipStream_t s)
{
    if (seg == 0 || chunks_per_block % seg) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pack_offsets_kernel, dim3(1), dim3(64), 0, s, segsum, chunks_per_block, seg, n_blocks, img_off);
    return hipGetLastError();
}

hipError_t launch_pack_write(const uint64_t *dir, const uint8_t *pool, uint32_t chunks_per_block, uint32_t seg,
                             uint64_t n_chunks, const uint32_t *rel, const uint64_t *segsum, const uint64_t *img_off,
                             uint8_t *img, hipStream_t s)
{
    if (n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(pack_write_kernel, dim3((unsigned)((4 * n_chunks + 255) / 256)), dim3(256), 0, s, dir, pool,
                       chunks_per_block, seg, n_chunks, rel, segsum, img_off, img);
    return hipGetLastError();
}

// D = the codec domain (0 LIN, 1 LOG, 2 RAW) as a constant inside the body
#define BMQ_DOM_SWITCH(dom, ...)                          \
    switch (dom) {                                        \
    case 0: { constexpr int D = 0; __VA_ARGS__; } break;  \
    case 1: { constexpr int D = 1; __VA_ARGS__; } break;  \
    case 2: { constexpr int D = 2; __VA_ARGS__; } break;  \
    default: return hipErrorInvalidValue;                 \
    }

hipError_t launch_init_state(uint64_t *dir, uint64_t n_chunks, uint8_t *pool, unsigned long long *counters,
                             CodecParams cp, hipStream_t s)
{
    hipError_t e = launch_fill_u64(dir, n_chunks, 0ull, s);
    if (e != hipSuccess) return e;
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(init_state_kernel<D>, dim3(1), dim3(64), 0, s, dir, pool, counters, cp))
    return hipGetLastError();
}

// runs of 16 items per wave, 4 waves per workgroup
static inline unsigned grid_runs(uint64_t items, unsigned cap = 65536) { return grid_for((items + 15) / 16, 4, cap); }

hipError_t launch_export(const uint64_t *dir, const PoolView &pv, CodecParams cp, uint64_t chunk0,
                         uint64_t n_chunks, float2 *dst, hipStream_t s)
{
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(export_kernel<D>, dim3(grid_runs(n_chunks)), dim3(256), 0, s, dir,
                                                 pv, cp, chunk0, n_chunks, dst))
    return hipGetLastError();
}

hipError_t launch_amplitudes(const uint64_t *dir, const PoolView &pv, CodecParams cp, const uint64_t *idx,
                             uint64_t k, uint64_t n_chunks, float2 *dst, hipStream_t s)
{
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(amplitudes_kernel<D>, dim3(grid_runs(k)), dim3(256), 0, s, dir, pv,
                                                 cp, idx, k, n_chunks, dst))
    return hipGetLastError();
}

template <int DOM, int REF, int RDOM>
static void fid_launch(unsigned grid, const uint64_t *dir, const PoolView &pv, CodecParams cp, uint64_t chunk0,
                       uint64_t n, const RefView &rv, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL((fidelity_partial_kernel<DOM, REF, RDOM>), dim3(grid), dim3(256), 0, s, dir, pv, cp, chunk0, n,
                       rv, partials);
}

hipError_t launch_fidelity_partial(const uint64_t *dir, const PoolView &pv, CodecParams cp, uint64_t chunk0,
                                   uint64_t n_chunks, const RefView &rv, double *partials, int n_partials,
                                   hipStream_t s)
{
    const unsigned g = (unsigned)n_partials;
    if (rv.kind == REF_NONE) {
        BMQ_DOM_SWITCH(cp.domain, (fid_launch<D, REF_NONE, 0>(g, dir, pv, cp, chunk0, n_chunks, rv, partials, s)))
    } else if (rv.kind == REF_C128) {
        BMQ_DOM_SWITCH(cp.domain, (fid_launch<D, REF_C128, 0>(g, dir, pv, cp, chunk0, n_chunks, rv, partials, s)))
    } else {
        switch (rv.cp.domain) {
        case 0: BMQ_DOM_SWITCH(cp.domain, (fid_launch<D, REF_STATE, 0>(g, dir, pv, cp, chunk0, n_chunks, rv, partials, s))) break;
        case 1: BMQ_DOM_SWITCH(cp.domain, (fid_launch<D, REF_STATE, 1>(g, dir, pv, cp, chunk0, n_chunks, rv, partials, s))) break;
        case 2: BMQ_DOM_SWITCH(cp.domain, (fid_launch<D, REF_STATE, 2>(g, dir, pv, cp, chunk0, n_chunks, rv, partials, s))) break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_fidelity_final(const double *partials, int n_partials, double *out5, hipStream_t s)
{
    hipLaunchKernelGGL(fidelity_final_kernel, dim3(1), dim3(64), 0, s, partials, n_partials, out5);
    return hipGetLastError();
}

hipError_t launch_group_norm(const uint64_t *dir, const PoolView &pv, CodecParams cp, uint32_t chunks_per_group,
                             uint64_t n_groups, double *gnorm, hipStream_t s)
{
    if (n_groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(group_norm_kernel<D>, dim3((unsigned)n_groups), dim3(256), 0, s, dir,
                                                 pv, cp, chunks_per_group, gnorm))
    return hipGetLastError();
}

hipError_t launch_sample(const uint64_t *dir, const PoolView &pv, CodecParams cp, uint32_t chunks_per_group,
                         const uint32_t *grp, const double *resid, uint64_t k, uint64_t *out, hipStream_t s)
{
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(sample_kernel<D>, dim3(grid_for(k, 4, 16384)), dim3(256), 0, s, dir,
                                                 pv, cp, chunks_per_group, grp, resid, k, out))
    return hipGetLastError();
}

hipError_t launch_codec_slots_encode(const float *re, const float *im, uint64_t nch, CodecParams cp,
                                     uint8_t *slots, uint32_t *sizes, hipStream_t s)
{
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(codec_slots_encode_kernel<D>, dim3(grid_runs(nch)), dim3(256), 0, s,
                                                 re, im, nch, cp, slots, sizes))
    return hipGetLastError();
}

hipError_t launch_codec_slots_decode(const uint8_t *slots, uint64_t nch, CodecParams cp, float *re, float *im,
                                     hipStream_t s)
{
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(codec_slots_decode_kernel<D>, dim3(grid_runs(nch)), dim3(256), 0, s,
                                                 slots, nch, cp, re, im))
    return hipGetLastError();
}

hipError_t launch_codec_stream_encode(const float *re, const float *im, uint64_t nch, CodecParams cp,
                                      uint32_t *sizes, uint64_t *off, uint8_t *dst, uint64_t cap, uint32_t ebbits,
                                      hipStream_t s)
{
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(codec_size_kernel<D>, dim3(grid_runs(nch)), dim3(256), 0, s, re, im,
                                                 nch, cp, sizes))
    hipLaunchKernelGGL(scan_sizes_kernel, dim3(1), dim3(1024), 0, s, sizes, nch, off);
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(codec_write_kernel<D>, dim3(grid_runs(nch)), dim3(256), 0, s, re, im,
                                                 nch, cp, off, dst, cap, ebbits))
    return hipGetLastError();
}

hipError_t launch_codec_stream_decode(const uint8_t *src, uint64_t bytes, uint64_t nch, CodecParams cp,
                                      uint64_t *off, uint32_t *bad, hipStream_t s)
{
    hipLaunchKernelGGL(codec_walk_kernel, dim3(1), dim3(64), 0, s, src, bytes, nch, cp.domain, off, bad);
    return hipGetLastError();
}

hipError_t launch_codec_read(const uint8_t *src, const uint64_t *off, uint64_t nch, CodecParams cp, float *re,
                             float *im, hipStream_t s)
{
    BMQ_DOM_SWITCH(cp.domain, hipLaunchKernelGGL(codec_read_kernel<D>, dim3(grid_runs(nch)), dim3(256), 0, s, src,
                                                 off, nch, cp, re, im))
    return hipGetLastError();
}

hipError_t launch_block_stats(const uint64_t *dir, uint64_t chunks_per_block, uint64_t n_blocks,
                              const StageFeats &sf, float *feats, float *label_bytes, int32_t *label_mode,
                              hipStream_t s)
{
    hipLaunchKernelGGL(block_stats_kernel, dim3((unsigned)n_blocks), dim3(256), 0, s, dir, chunks_per_block, sf,
                       feats, label_bytes, label_mode);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free scratch
//
// Device scratch of codec_encode_noalloc: a file-scope array that every GPU
// the library runs on holds until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): its device address is looked up once per device with that
// device current and kept.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **ptr)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace bmq
