/*
 * CPU reference state-vector simulator -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 (complex128) simulation with no compression, no blocking and no
 * fusion: gates are applied one at a time in circuit order with the update
 * rules of paper Section 2.1 (a 2x2 matrix on every amplitude pair whose
 * indices differ only in bit k; a 4x4 matrix on every quadruple whose indices
 * differ only in bits q and k, rows ordered 0q0k, 0q1k, 1q0k, 1q1k).
 * Qubit q is bit q of the amplitude index.  Parallelised over independent
 * pairs/quadruples with OpenMP only; the arithmetic per pair is the textbook
 * matrix-vector product.
 *
 * Gate kinds (codes match the boundary's sv_gate_t.kind):
 *   0 H, 1 X, 2 Y, 3 Z, 4 S, 5 T, 6 RX, 7 RY, 8 RZ, 9 U3,
 *   10 CX (control q0, target q1), 11 CZ, 12 CP(lambda), 13 RZZ(gamma)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;

static void gate_matrix(int kind, const double *p, cplx *u /* 16 entries, row major */, int *nq)
{
    const double s2 = 1.0 / sqrt(2.0);
    memset(u, 0, 16 * sizeof(cplx));
    *nq = 1;
    switch (kind) {
    case 0: u[0] = s2; u[1] = s2; u[2] = s2; u[3] = -s2; break;
    case 1: u[1] = 1; u[2] = 1; break;
    case 2: u[1] = -I; u[2] = I; break;
    case 3: u[0] = 1; u[3] = -1; break;
    case 4: u[0] = 1; u[3] = I; break;
    case 5: u[0] = 1; u[3] = cexp(I * M_PI / 4); break;
    case 6: { double c = cos(p[0] / 2), s = sin(p[0] / 2);
              u[0] = c; u[1] = -I * s; u[2] = -I * s; u[3] = c; } break;
    case 7: { double c = cos(p[0] / 2), s = sin(p[0] / 2);
              u[0] = c; u[1] = -s; u[2] = s; u[3] = c; } break;
    case 8: u[0] = cexp(-I * p[0] / 2); u[3] = cexp(I * p[0] / 2); break;
    case 9: { double c = cos(p[0] / 2), s = sin(p[0] / 2);
              u[0] = c; u[1] = -cexp(I * p[2]) * s;
              u[2] = cexp(I * p[1]) * s; u[3] = cexp(I * (p[1] + p[2])) * c; } break;
    case 10: *nq = 2; u[0] = 1; u[5] = 1; u[11] = 1; u[14] = 1; break;
    case 11: *nq = 2; u[0] = 1; u[5] = 1; u[10] = 1; u[15] = -1; break;
    case 12: *nq = 2; u[0] = 1; u[5] = 1; u[10] = 1; u[15] = cexp(I * p[0]); break;
    case 13: *nq = 2; u[0] = cexp(-I * p[0] / 2); u[5] = cexp(I * p[0] / 2);
             u[10] = cexp(I * p[0] / 2); u[15] = cexp(-I * p[0] / 2); break;
    default: *nq = 0; break;
    }
}

/* insert a zero bit at position q of x */
static uint64_t ins0(uint64_t x, int q) { return ((x >> q) << (q + 1)) | (x & ((1ull << q) - 1)); }

int o_gate_matrix(int kind, const double *p, double *u_interleaved)
{
    cplx u[16];
    int nq;
    gate_matrix(kind, p, u, &nq);
    for (int i = 0; i < 16; ++i) { u_interleaved[2 * i] = creal(u[i]); u_interleaved[2 * i + 1] = cimag(u[i]); }
    return nq;
}

void o_apply_gate(double *state /* interleaved complex128, 2^n */, int n,
                  int kind, const int *q, const double *p)
{
    cplx u[16];
    int nq;
    cplx *psi = (cplx *)state;
    gate_matrix(kind, p, u, &nq);
    if (nq == 1) {
        int k = q[0];
        int64_t half = (int64_t)1 << (n - 1);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < half; ++i) {
            uint64_t i0 = ins0((uint64_t)i, k), i1 = i0 | (1ull << k);
            cplx a0 = psi[i0], a1 = psi[i1];
            psi[i0] = u[0] * a0 + u[1] * a1;
            psi[i1] = u[2] * a0 + u[3] * a1;
        }
    } else if (nq == 2) {
        int qa = q[0], qb = q[1];
        int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
        int64_t quarter = (int64_t)1 << (n - 2);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < quarter; ++i) {
            uint64_t base = ins0(ins0((uint64_t)i, lo), hi);
            uint64_t idx[4];
            cplx a[4];
            for (int r = 0; r < 4; ++r) {
                uint64_t ba = (uint64_t)(r >> 1), bb = (uint64_t)(r & 1);
                idx[r] = base | (ba << qa) | (bb << qb);
                a[r] = psi[idx[r]];
            }
            for (int r = 0; r < 4; ++r) {
                cplx acc = 0;
                for (int c = 0; c < 4; ++c) acc += u[4 * r + c] * a[c];
                psi[idx[r]] = acc;
            }
        }
    }
}

/* Run a whole circuit from |0...0> (paper Section 4.2: the first element is 1,
 * all others 0).  kinds[g], qubits[2g..2g+1], params[3g..3g+2]. */
void o_simulate(double *state, int n, const int *kinds, const int *qubits,
                const double *params, int64_t n_gates)
{
    int64_t dim = (int64_t)1 << n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < 2 * dim; ++i) state[i] = 0.0;
    state[0] = 1.0;
    for (int64_t g = 0; g < n_gates; ++g)
        o_apply_gate(state, n, kinds[g], qubits + 2 * g, params + 3 * g);
}

/* Apply a gate list to an existing state (used for the mirror-echo pin). */
void o_apply_circuit(double *state, int n, const int *kinds, const int *qubits,
                     const double *params, int64_t n_gates)
{
    for (int64_t g = 0; g < n_gates; ++g)
        o_apply_gate(state, n, kinds[g], qubits + 2 * g, params + 3 * g);
}

/* <a|b>, |a|^2, |b|^2 in FP64 over interleaved complex128 (b may be float32
 * interleaved when b32 != 0). */
void o_overlap(const double *a, const void *b, int b32, int64_t dim, double *out /* re, im, na, nb, maxabs */)
{
    double sre = 0, sim = 0, na = 0, nb = 0, mx = 0;
    #pragma omp parallel for reduction(+:sre,sim,na,nb) reduction(max:mx) schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        double ar = a[2 * i], ai = a[2 * i + 1], br, bi;
        if (b32) { br = ((const float *)b)[2 * i]; bi = ((const float *)b)[2 * i + 1]; }
        else { br = ((const double *)b)[2 * i]; bi = ((const double *)b)[2 * i + 1]; }
        sre += ar * br + ai * bi;
        sim += ar * bi - ai * br;
        na += ar * ar + ai * ai;
        nb += br * br + bi * bi;
        double dr = fabs(ar - br), di = fabs(ai - bi);
        double d = dr > di ? dr : di;
        if (d > mx) mx = d;
    }
    out[0] = sre; out[1] = sim; out[2] = na; out[3] = nb; out[4] = mx;
}

/* QFT-on-Ry closed form (no final swaps): psi(y) = 2^{-n/2} prod_i
 * (cos(t_i/2) + sin(t_i/2) exp(2 pi i 2^i rev_n(y) / 2^n)), evaluated for a
 * list of indices.  Derivation: the product state sum_x prod_i a_i(x_i)|x>
 * maps under the swap-free QFT to 2^{-n/2} sum_y exp(2 pi i x rev(y)/2^n). */
void o_qft_ry_amplitudes(int n, const double *theta, const uint64_t *idx, int64_t k, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < k; ++j) {
        uint64_t y = idx[j], rev = 0;
        for (int b = 0; b < n; ++b) if ((y >> b) & 1ull) rev |= 1ull << (n - 1 - b);
        cplx acc = 1.0;
        for (int i = 0; i < n; ++i) {
            /* phase = 2 pi * frac(2^i * rev / 2^n), reduced exactly in integers */
            uint64_t num = (rev << i) & ((1ull << n) - 1);
            double ph = 2.0 * M_PI * (double)num / (double)(1ull << n);
            acc *= cos(theta[i] / 2) + sin(theta[i] / 2) * cexp(I * ph);
        }
        acc *= pow(2.0, -0.5 * n);
        out[2 * j] = creal(acc);
        out[2 * j + 1] = cimag(acc);
    }
}

/* Full QFT-on-Ry state by the closed form (interleaved complex128). */
void o_qft_ry_state(int n, const double *theta, double *out)
{
    int64_t dim = (int64_t)1 << n;
    const int64_t B = 1 << 16;
    for (int64_t s = 0; s < dim; s += B) {
        int64_t cnt = dim - s < B ? dim - s : B;
        uint64_t idx[1 << 16];
        for (int64_t j = 0; j < cnt; ++j) idx[j] = (uint64_t)(s + j);
        o_qft_ry_amplitudes(n, theta, idx, cnt, out + 2 * s);
    }
}
