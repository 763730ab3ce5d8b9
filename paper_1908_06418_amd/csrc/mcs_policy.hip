// Learned branching policy: a 16 -> 64 -> 64 -> 1 ReLU network that scores a
// candidate vertex at a search node.  The search uses the scores to choose v
// within the selected class and the order of its partners w; it never prunes
// on them, so answers are unchanged (the paper's Solve explores or bounds
// every child regardless of order).
//
// Parameters are float32 "master" values packed as W1[64][16], b1[64],
// W2[64][64], b2[64], w3[64], b3.  Inputs are half precision.  Every multiply
// uses the half-rounded weights with float32 accumulation -- the same
// arithmetic the search applies at inference (mcs_policy_score).
//
// Training kernels: per-block partial gradients over 64 rows (one row per
// lane, activations kept in registers, outer products through LDS), a
// deterministic cross-block reduction, and an SGD step.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcs_policy.h"

namespace mcs {

__device__ __forceinline__ float h2f(uint16_t h) { return __half2float(__ushort_as_half(h)); }
__device__ __forceinline__ float round_half(float x) { return __half2float(__float2half(x)); }

// Stage the half-rounded weights of the network into LDS as floats.
__device__ void stage_weights(const float *P, float *s) {
    for (int i = threadIdx.x; i < kPolicyParams; i += blockDim.x)
        s[i] = round_half(P[i]);
    __syncthreads();
}

// Forward pass of one row (x in registers) with the staged weights.
__device__ __forceinline__ float row_forward(const float *s, const float x[kPolicyF], float a1[64],
                                             float a2[64]) {
    const float *W1 = s + kOffW1, *b1 = s + kOffB1, *W2 = s + kOffW2, *b2 = s + kOffB2,
                *w3 = s + kOffW3;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        float acc = b1[j];
#pragma unroll
        for (int f = 0; f < kPolicyF; ++f)
            acc += W1[j * kPolicyF + f] * x[f];
        a1[j] = acc;
    }
    float z = s[kOffB3];
    for (int j = 0; j < 64; ++j) {
        float acc = b2[j];
#pragma unroll 16
        for (int i = 0; i < 64; ++i)
            acc += W2[j * 64 + i] * fmaxf(a1[i], 0.f);
        a2[j] = acc;
        z += w3[j] * fmaxf(acc, 0.f);
    }
    return z;
}

__global__ void __launch_bounds__(64) policy_forward_kernel(const uint16_t *X, int rows,
                                                            const float *P, float *logits) {
    __shared__ float s[kPolicyParams];
    stage_weights(P, s);
    const int r = blockIdx.x * 64 + threadIdx.x;
    if (r >= rows)
        return;
    float x[kPolicyF], a1[64], a2[64];
#pragma unroll
    for (int f = 0; f < kPolicyF; ++f)
        x[f] = h2f(X[(size_t)r * kPolicyF + f]);
    logits[r] = row_forward(s, x, a1, a2);
}

// One block = 64 rows.  Writes this block's share of the gradient of the mean
// binary cross-entropy (already divided by the total row count) and of the
// summed loss to partials[block][kPolicyParams + 1].  Thread t owns hidden
// unit t of both layers when summing over the block's rows.
__global__ void __launch_bounds__(64) policy_partial_kernel(const uint16_t *X, const float *y,
                                                            int rows, const float *P,
                                                            float *partials) {
    __shared__ float s[kPolicyParams];
    __shared__ float sh[64][65];   // h1, later h2, of each row (padded)
    __shared__ float sd2[64][65];  // dL/da2 of each row
    __shared__ float sx[64][kPolicyF + 1];
    __shared__ float sdz[64];
    __shared__ float sloss[64];
    stage_weights(P, s);
    const int t = threadIdx.x;
    const int r = blockIdx.x * 64 + t;
    const bool live = r < rows;
    float x[kPolicyF], a1[64], a2[64];
#pragma unroll
    for (int f = 0; f < kPolicyF; ++f) {
        x[f] = live ? h2f(X[(size_t)r * kPolicyF + f]) : 0.f;
        sx[t][f] = x[f];
    }
    const float z = row_forward(s, x, a1, a2);
    const float yy = live ? y[r] : 0.f;
    // stable form of the binary cross-entropy of sigmoid(z) against y
    const float loss = fmaxf(z, 0.f) - z * yy + log1pf(__expf(-fabsf(z)));
    const float sig = 1.f / (1.f + __expf(-z));
    const float dz = live ? (sig - yy) / (float)rows : 0.f;
    sloss[t] = live ? loss : 0.f;
    sdz[t] = dz;
    const float *W2 = s + kOffW2, *w3 = s + kOffW3;
    for (int j = 0; j < 64; ++j) {
        sh[t][j] = fmaxf(a1[j], 0.f);
        sd2[t][j] = a2[j] > 0.f ? dz * w3[j] : 0.f;
    }
    __syncthreads();
    float *out = partials + (size_t)blockIdx.x * (kPolicyParams + 1);
    {
        float gb1 = 0.f, gb2 = 0.f;
        float gW1[kPolicyF];
#pragma unroll
        for (int f = 0; f < kPolicyF; ++f)
            gW1[f] = 0.f;
        for (int q = 0; q < 64; ++q) {
            // dL/da1 of row q at unit t: masked by h1 > 0 (i.e. a1 > 0)
            float d1 = 0.f;
            if (sh[q][t] > 0.f)
                for (int j = 0; j < 64; ++j)
                    d1 += sd2[q][j] * W2[j * 64 + t];
            gb1 += d1;
#pragma unroll
            for (int f = 0; f < kPolicyF; ++f)
                gW1[f] += d1 * sx[q][f];
            gb2 += sd2[q][t];
        }
#pragma unroll
        for (int f = 0; f < kPolicyF; ++f)
            out[kOffW1 + t * kPolicyF + f] = gW1[f];
        out[kOffB1 + t] = gb1;
        out[kOffB2 + t] = gb2;
        for (int i = 0; i < 64; ++i) {
            float g = 0.f;
            for (int q = 0; q < 64; ++q)
                g += sd2[q][t] * sh[q][i];
            out[kOffW2 + t * 64 + i] = g;
        }
    }
    __syncthreads();
    for (int j = 0; j < 64; ++j)
        sh[t][j] = fmaxf(a2[j], 0.f);
    __syncthreads();
    {
        float g = 0.f;
        for (int q = 0; q < 64; ++q)
            g += sdz[q] * sh[q][t];
        out[kOffW3 + t] = g;
    }
    if (t == 0) {
        float gb3 = 0.f, l = 0.f;
        for (int q = 0; q < 64; ++q) {
            gb3 += sdz[q];
            l += sloss[q];
        }
        out[kOffB3] = gb3;
        out[kPolicyParams] = l;
    }
}

// grads[i] = sum over blocks; loss = summed loss / rows.  Fixed order.
__global__ void __launch_bounds__(256) policy_reduce_kernel(const float *partials, int blocks,
                                                            int rows, float *grads, float *loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kPolicyParams)
        return;
    float acc = 0.f;
    for (int b = 0; b < blocks; ++b)
        acc += partials[(size_t)b * (kPolicyParams + 1) + i];
    if (i < kPolicyParams)
        grads[i] = acc;
    else if (loss)
        *loss = acc / (float)rows;
}

__global__ void __launch_bounds__(256) policy_sgd_kernel(float *P, const float *G, float lr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kPolicyParams)
        P[i] -= lr * G[i];
}

__global__ void __launch_bounds__(256) policy_pack_half_kernel(const float *P, uint16_t *H) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kPolicyParams)
        H[i] = __half_as_ushort(__float2half(P[i]));
}

}  // namespace mcs

// ---- C ABI (declared in include/mcs.h) -------------------------------------

#include "mcs.h"

namespace {
mcs_status launch_status(hipError_t e) { return e == hipSuccess ? MCS_OK : MCS_E_DEVICE; }
}  // namespace

extern "C" {

int32_t mcs_policy_param_count(void) { return mcs::kPolicyParams; }

size_t mcs_policy_workspace_size(int32_t rows) {
    if (rows <= 0)
        return 0;
    size_t blocks = ((size_t)rows + 63) / 64;
    return blocks * (mcs::kPolicyParams + 1) * sizeof(float);
}

mcs_status mcs_policy_forward(const uint16_t *x, int32_t rows, const float *params, float *logits,
                              void *stream) {
    if (rows < 0 || (rows > 0 && (!x || !params || !logits)))
        return MCS_E_INVALID;
    if (rows == 0)
        return MCS_OK;
    hipLaunchKernelGGL(mcs::policy_forward_kernel, dim3((rows + 63) / 64), dim3(64), 0,
                       (hipStream_t)stream, x, rows, params, logits);
    return launch_status(hipGetLastError());
}

mcs_status mcs_policy_grad(const uint16_t *x, const float *y, int32_t rows, const float *params,
                           float *grads, float *loss, void *workspace, size_t bytes,
                           void *stream) {
    if (rows <= 0 || !x || !y || !params || !grads)
        return MCS_E_INVALID;
    if (!workspace || bytes < mcs_policy_workspace_size(rows))
        return MCS_E_WORKSPACE;
    int blocks = (rows + 63) / 64;
    hipStream_t s = (hipStream_t)stream;
    float *partials = (float *)workspace;
    hipLaunchKernelGGL(mcs::policy_partial_kernel, dim3(blocks), dim3(64), 0, s, x, y, rows,
                       params, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return MCS_E_DEVICE;
    hipLaunchKernelGGL(mcs::policy_reduce_kernel, dim3((mcs::kPolicyParams + 1 + 255) / 256),
                       dim3(256), 0, s, partials, blocks, rows, grads, loss);
    return launch_status(hipGetLastError());
}

mcs_status mcs_policy_sgd(float *params, const float *grads, float lr, void *stream) {
    if (!params || !grads)
        return MCS_E_INVALID;
    hipLaunchKernelGGL(mcs::policy_sgd_kernel, dim3((mcs::kPolicyParams + 255) / 256), dim3(256),
                       0, (hipStream_t)stream, params, grads, lr);
    return launch_status(hipGetLastError());
}

mcs_status mcs_policy_pack_half(const float *params, uint16_t *half_params, void *stream) {
    if (!params || !half_params)
        return MCS_E_INVALID;
    hipLaunchKernelGGL(mcs::policy_pack_half_kernel, dim3((mcs::kPolicyParams + 255) / 256),
                       dim3(256), 0, (hipStream_t)stream, params, half_params);
    return launch_status(hipGetLastError());
}

}  // extern "C"
