// Block-size / mode predictor: a 32 -> 64 -> 64 -> 5 multilayer perceptron
// with ReLU hidden layers, trained online with Adam.  The paper notes that
// the compression ratio of a block cannot be known before it is compressed,
// which makes memory hard to plan (Section 3, Section 4.4); the predictor
// estimates, per SV block and before a stage runs, log2 of the block's
// compressed bytes after the stage (output 0) and logits of its most frequent
// codec mode (outputs 1..4).  Output 0 adds feature 0 (the block's current
// log2 bytes) to the network's first output, so an untrained predictor
// already predicts that a block keeps its size and training learns the change.
//
// Parameters (float32, one device array of SV_MLP_NPARAM):
//   W1[64][32] b1[64] W2[64][64] b2[64] W3[5][64] b3[5]   (row = output unit)
// Loss per sample: 0.5 (out0 - y)^2 + logsumexp(out1..4) - out[1 + mode],
// averaged over the batch.  Every reduction runs in a fixed order (no
// floating-point atomics), so results are reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "../../include/bmq.h"
#include "bmq_internal.h"

namespace {

constexpr int IN = SV_MLP_IN, H = SV_MLP_HIDDEN, OUT = SV_MLP_OUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + OUT * H, NPARAM = OFF_B3 + OUT;
static_assert(NPARAM == SV_MLP_NPARAM, "parameter layout");

// per-sample work record: h1[64] h2[64] out[5] d_h1[64] d_h2[64] d_out[5] loss
constexpr int W_H1 = 0, W_H2 = W_H1 + H, W_OUT = W_H2 + H, W_DH1 = W_OUT + OUT, W_DH2 = W_DH1 + H,
              W_DOUT = W_DH2 + H, W_LOSS = W_DOUT + OUT, W_REC = W_LOSS + 1;

// forward pass of one sample per workgroup of 64 threads (thread = hidden unit)
__device__ void forward_sample(const float *__restrict__ P, const float *__restrict__ x, float *h1s, float *h2s,
                               float *outs)
{
    const int j = (int)threadIdx.x;
    float z = P[OFF_B1 + j];
    for (int k = 0; k < IN; ++k) z = __builtin_fmaf(P[OFF_W1 + j * IN + k], x[k], z);
    h1s[j] = z > 0.0f ? z : 0.0f;
    __syncthreads();
    z = P[OFF_B2 + j];
    for (int i = 0; i < H; ++i) z = __builtin_fmaf(P[OFF_W2 + j * H + i], h1s[i], z);
    h2s[j] = z > 0.0f ? z : 0.0f;
    __syncthreads();
    if (j < OUT) {
        z = P[OFF_B3 + j];
        for (int i = 0; i < H; ++i) z = __builtin_fmaf(P[OFF_W3 + j * H + i], h2s[i], z);
        outs[j] = j == 0 ? x[0] + z : z;     // size output: skip connection from feature 0
    }
    __syncthreads();
}

__global__ __launch_bounds__(64) void mlp_forward_kernel(const float *P, const float *X, float *out)
{
    __shared__ float xs[IN], h1[H], h2[H], o[OUT];
    const uint64_t s = blockIdx.x;
    if (threadIdx.x < IN) xs[threadIdx.x] = X[s * IN + threadIdx.x];
    __syncthreads();
    forward_sample(P, xs, h1, h2, o);
    if (threadIdx.x < OUT) out[s * OUT + threadIdx.x] = o[threadIdx.x];
}

// forward + backward of one sample: activations and deltas go to its work record
__global__ __launch_bounds__(64) void mlp_backward_kernel(const float *P, const float *X, const float *y_bytes,
                                                          const int32_t *y_mode, uint32_t batch, float *work)
{
    __shared__ float xs[IN], h1[H], h2[H], o[OUT], dout[OUT], dh2[H];
    const uint64_t s = blockIdx.x;
    const int j = (int)threadIdx.x;
    if (j < IN) xs[j] = X[s * IN + j];
    __syncthreads();
    forward_sample(P, xs, h1, h2, o);
    float *w = work + s * W_REC;
    const float inv_b = 1.0f / (float)batch;
    if (j == 0) {
        const int32_t m = min(max(y_mode[s], 0), OUT - 2);   // mode classes 0..3
        const float r = o[0] - y_bytes[s];
        float mx = o[1];
        for (int c = 2; c < OUT; ++c) mx = o[c] > mx ? o[c] : mx;
        float e[OUT - 1], se = 0.0f;
        for (int c = 0; c < OUT - 1; ++c) {
            e[c] = expf(o[1 + c] - mx);
            se += e[c];
        }
        const float lse = mx + logf(se);
        dout[0] = r * inv_b;
        for (int c = 0; c < OUT - 1; ++c) dout[1 + c] = (e[c] / se - (c == m ? 1.0f : 0.0f)) * inv_b;
        w[W_LOSS] = 0.5f * r * r + (lse - o[1 + m]);
    }
    __syncthreads();
    // d h2_j = sum_o W3[o][j] d out_o, gated by ReLU
    float z = 0.0f;
    for (int c = 0; c < OUT; ++c) z = __builtin_fmaf(P[OFF_W3 + c * H + j], dout[c], z);
    dh2[j] = h2[j] > 0.0f ? z : 0.0f;
    __syncthreads();
    z = 0.0f;
    for (int i = 0; i < H; ++i) z = __builtin_fmaf(P[OFF_W2 + i * H + j], dh2[i], z);
    w[W_H1 + j] = h1[j];
    w[W_H2 + j] = h2[j];
    w[W_DH1 + j] = h1[j] > 0.0f ? z : 0.0f;
    w[W_DH2 + j] = dh2[j];
    if (j < OUT) {
        w[W_OUT + j] = o[j];
        w[W_DOUT + j] = dout[j];
    }
}

// one thread per parameter: gradient = sum over the batch in sample order;
// thread NPARAM sums the loss
__global__ void mlp_grad_kernel(const float *X, const float *work, uint32_t batch, float *grad, float *loss)
{
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p > NPARAM) return;
    float g = 0.0f;
    if (p == NPARAM) {
        for (uint32_t s = 0; s < batch; ++s) g += work[(uint64_t)s * W_REC + W_LOSS];
        *loss = g / (float)batch;
        return;
    }
    int dsrc, asrc = -1, aoff = 0;
    bool from_x = false;
    if (p < OFF_B1) { dsrc = W_DH1 + p / IN; from_x = true; aoff = p % IN; }
    else if (p < OFF_W2) { dsrc = W_DH1 + (p - OFF_B1); }
    else if (p < OFF_B2) { dsrc = W_DH2 + (p - OFF_W2) / H; asrc = W_H1 + (p - OFF_W2) % H; }
    else if (p < OFF_W3) { dsrc = W_DH2 + (p - OFF_B2); }
    else if (p < OFF_B3) { dsrc = W_DOUT + (p - OFF_W3) / H; asrc = W_H2 + (p - OFF_W3) % H; }
    else { dsrc = W_DOUT + (p - OFF_B3); }
    for (uint32_t s = 0; s < batch; ++s) {
        const float *w = work + (uint64_t)s * W_REC;
        const float a = from_x ? X[(uint64_t)s * IN + aoff] : (asrc >= 0 ? w[asrc] : 1.0f);
        g = __builtin_fmaf(w[dsrc], a, g);
    }
    grad[p] = g;
}

struct AdamArgs {
    float lr, beta1, beta2, eps, c1, c2;   // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
};

__global__ void mlp_adam_kernel(float *P, const float *grad, float *m, float *v, AdamArgs a)
{
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= NPARAM) return;
    const float g = grad[p];
    const float mm = a.beta1 * m[p] + (1.0f - a.beta1) * g;
    const float vv = a.beta2 * v[p] + (1.0f - a.beta2) * (g * g);
    m[p] = mm;
    v[p] = vv;
    const float mh = mm * a.c1, vh = vv * a.c2;
    P[p] = P[p] - a.lr * mh / (sqrtf(vh) + a.eps);
}

// ---- rollout of the predictor over a circuit (memory planning)

// X[i] <- the features of row 1 for every row i >= 2 (blocks 1.. of |0...0>
// are identical all-zero blocks; rows 0 and 1 were computed from the state)
__global__ void replicate_rows_kernel(float *X, uint32_t n_blocks)
{
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 2ull * IN; t < (uint64_t)n_blocks * IN;
         t += (uint64_t)gridDim.x * blockDim.x)
        X[t] = X[IN + (t % IN)];
}

// Planning form of block features (or labels): feature 0 becomes log2 bytes
// per amplitude (less b), features 1..24 the values of an all-zero block
// (ZERO-mode fraction 1, all-zero chunk fraction 1, the rest 0), the state
// features a rollout cannot advance
__global__ void plan_form_kernel(float *X, float *y, uint32_t n_blocks, float b)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_blocks; i += gridDim.x * blockDim.x) {
        if (X) {
            float *x = X + (uint64_t)i * IN;
            x[0] -= b;
            for (int k = 1; k <= 24; ++k) x[k] = (k == 1 || k == 21) ? 1.0f : 0.0f;
        }
        if (y) y[i] -= b;
    }
}

// One rollout step: total[0] += sum over blocks of 2^out0 (the predicted
// stream bytes after the stage; fixed summation order: one workgroup, lanes
// in index order, then a tree), then feature 0 <- out0 and the stage
// features <- those of the next stage.
__global__ __launch_bounds__(256) void rollout_step_kernel(float *X, const float *out, uint32_t n_blocks,
                                                           bmq::StageFeats next, double b, double *total)
{
    __shared__ double part[256];
    double acc = 0.0;
    // a chunk's record is 8 to 8 + 552 bytes: the size per amplitude lies
    // between 2^-3 and 2^log2(560/64); predictions are held to that range
    const float lo = -3.0f, hi = 3.1292830f;
    for (uint32_t i = threadIdx.x; i < n_blocks; i += 256) {
        const float y = fminf(fmaxf(out[(uint64_t)i * OUT], lo), hi);
        acc += exp2((double)y + b);
        X[(uint64_t)i * IN] = y;
#pragma unroll
        for (int k = 0; k < 7; ++k) X[(uint64_t)i * IN + 25 + k] = next.v[k];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = part[0];
}

}  // namespace

namespace bmq {
hipError_t launch_replicate_rows(float *X, uint32_t n_blocks, hipStream_t s)
{
    if (n_blocks <= 2) return hipSuccess;
    const uint64_t work = (uint64_t)n_blocks * IN;
    hipLaunchKernelGGL(replicate_rows_kernel, dim3((unsigned)std::min<uint64_t>((work + 255) / 256, 16384)), dim3(256),
                       0, s, X, n_blocks);
    return hipGetLastError();
}
hipError_t launch_rollout_step(float *X, const float *out, uint32_t n_blocks, const StageFeats &next, int b,
                               double *total, hipStream_t s)
{
    hipLaunchKernelGGL(rollout_step_kernel, dim3(1), dim3(256), 0, s, X, out, n_blocks, next, (double)b, total);
    return hipGetLastError();
}
hipError_t launch_plan_form(float *X, float *y, uint32_t n_blocks, int b, hipStream_t s)
{
    hipLaunchKernelGGL(plan_form_kernel, dim3((unsigned)std::min<uint32_t>((n_blocks + 255) / 256, 4096u)), dim3(256),
                       0, s, X, y, n_blocks, (float)b);
    return hipGetLastError();
}
}  // namespace bmq

namespace bmq {

uint64_t mlp_work_floats(uint32_t batch) { return (uint64_t)batch * W_REC; }

hipError_t launch_mlp_forward(const float *P, const float *X, uint32_t batch, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(batch), dim3(64), 0, s, P, X, out);
    return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float *P, const float *X, const float *y_bytes, const int32_t *y_mode,
                                uint32_t batch, float *work, float *grad, float *loss, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(batch), dim3(64), 0, s, P, X, y_bytes, y_mode, batch, work);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, s, X, work, batch, grad,
                       loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *P, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t s)
{
    const AdamArgs a{lr, beta1, beta2, eps, c1, c2};
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, grad, m, v, a);
    return hipGetLastError();
}

}  // namespace bmq
