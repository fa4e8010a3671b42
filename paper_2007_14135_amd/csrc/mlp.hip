// Learned proposal network: covariance features, MLP forward/backward on the BF16 matrix cores,
// binary cross-entropy and Adam.
//
// The network is 272 -> 512 -> 512 -> 180 with ReLU hidden units and sigmoid outputs; its input
// is the upper triangle of R (Eq. 3) scaled by M / trace(R).  Master weights, Adam moments and
// activations are FP32 in memory; every GEMM rounds its operands to bfloat16 when it stages them
// through LDS and accumulates in FP32 on v_mfma_f32_32x32x16_bf16.  All reductions run in a fixed
// order (no floating-point atomics), so a training step is deterministic.
#include <float.h>
#include <math.h>

#include "internal.h"

namespace nssdoa {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTM = 64, kTN = 64, kTK = 64;   // workgroup tile; each of 4 waves owns 32 x 32

// C(m, n) = act( alpha * sum_k A(m, k) B(k, n) + bias(n) ), element (m, k) of A at
// A[m * sam + k * sak], (k, n) of B at B[k * sbk + n * sbn], C row-major with leading dimension ldc.
// relu_in_a / relu_in_b: the operand is read through max(., 0) (a layer consumes ReLU of a
// stored pre-activation).  mask: optional, C is multiplied by (mask(m, n) > 0) (ReLU derivative).
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const float* __restrict__ A,
                                                        int64_t sam, int64_t sak, int relu_in_a,
                                                        const float* __restrict__ B, int64_t sbk,
                                                        int64_t sbn, int relu_in_b, float alpha,
                                                        const float* __restrict__ bias,
                                                        const float* __restrict__ mask, int64_t ldm,
                                                        int relu_out, float* __restrict__ C, int64_t ldc) {
    __shared__ __bf16 As[kTM][kTK + 8];
    __shared__ __bf16 Bs[kTN][kTK + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int h = lane >> 5, r32 = lane & 31;
    floatx16 acc = {0.0f};
    for (int k0 = 0; k0 < K; k0 += kTK) {
        __syncthreads();
        for (int e = tid; e < kTM * kTK; e += 256) {
            const int mm = e / kTK, kk = e - mm * kTK;
            const int m = m0 + mm, k = k0 + kk;
            float a = 0.0f;
            if (m < M && k < K) {
                a = A[(int64_t)m * sam + (int64_t)k * sak];
                if (relu_in_a) a = fmaxf(a, 0.0f);
            }
            As[mm][kk] = (__bf16)a;
        }
        for (int e = tid; e < kTN * kTK; e += 256) {
            const int nn = e / kTK, kk = e - nn * kTK;
            const int n = n0 + nn, k = k0 + kk;
            float b = (n < N && k < K) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.0f;
            if (relu_in_b) b = fmaxf(b, 0.0f);
            Bs[nn][kk] = (__bf16)b;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kTK / 16; ++s) {
            bf16x8 a, b;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                a[t] = As[wm * 32 + r32][16 * s + 8 * h + t];
                b[t] = Bs[wn * 32 + r32][16 * s + 8 * h + t];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
    }
    // register r of lane h*32+j: row 8(r/4) + 4h + r%4, column j of the wave's 32 x 32 block
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const int n = n0 + wn * 32 + r32;
        if (m < M && n < N) {
            float v = alpha * acc[r];
            if (bias) v += bias[n];
            if (mask && !(mask[(int64_t)m * ldm + n] > 0.0f)) v = 0.0f;
            if (relu_out) v = fmaxf(v, 0.0f);
            C[(int64_t)m * ldc + n] = v;
        }
    }
}

// out[n] = sum_m X[m * ld + n] over m = 0..rows-1, in order (bias gradients).
__global__ void colsum_kernel(int rows, int cols, const float* __restrict__ X, int64_t ld,
                              float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    float s = 0.0f;
    for (int m = 0; m < rows; ++m) s += X[(int64_t)m * ld + n];
    out[n] = s;
}

// Binary cross-entropy with logits: per row partial sums of max(z,0) - z y + log(1 + exp(-|z|)),
// and the gradient dZ = (sigmoid(z) - y) / (rows * cols).
__global__ void bce_kernel(int rows, int cols, const float* __restrict__ Z, const float* __restrict__ Y,
                           float* __restrict__ dZ, float* __restrict__ row_loss) {
    __shared__ float red[256];
    const int m = blockIdx.x;
    float s = 0.0f;
    const float inv = 1.0f / ((float)rows * (float)cols);
    for (int n = threadIdx.x; n < cols; n += blockDim.x) {
        const float z = Z[(int64_t)m * cols + n], y = Y[(int64_t)m * cols + n];
        s += fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
        dZ[(int64_t)m * cols + n] = (1.0f / (1.0f + expf(-z)) - y) * inv;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) row_loss[m] = red[0];
}

// loss = sum(row_loss) / (rows * cols), one thread, fixed order.
__global__ void loss_finish_kernel(int rows, int cols, const float* __restrict__ row_loss,
                                   float* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int m = 0; m < rows; ++m) s += row_loss[m];
    *loss = (float)(s / ((double)rows * (double)cols));
}

// Adam with bias correction; t counts from 1.  a1 = 1 - b1, a2 = 1 - b2 and the bias corrections
// c1 = 1 - b1^t, c2 = 1 - b2^t come from the host, formed in FP64 and rounded once: formed in FP32
// from the rounded b2 = 0.999f they would carry a relative error near 5e-5 (cancellation).
__global__ void adam_kernel(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float a1, float a2, float eps,
                            float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + a1 * gi;
    const float vi = b2 * v[i] + a2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Features of frame flist[row] (frame `row` when flist is NULL): upper triangle of
// R * M / trace(R), row-major, (re, im) interleaved.
__global__ void features_kernel(const int32_t* __restrict__ flist, int n, const FrameDev* __restrict__ frames,
                                const char* __restrict__ ws, float* __restrict__ out, int nfeat) {
    const int row = blockIdx.x;
    if (row >= n) return;
    const FrameDev& fr = frames[flist ? flist[row] : row];
    const int M = fr.M;
    const double2* R = reinterpret_cast<const double2*>(ws + fr.ws_R);
    __shared__ double trs;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < M; ++i) t += R[i * M + i].x;
        trs = (double)M / t;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < M * (M + 1) / 2; e += blockDim.x) {
        int i = 0, r = e;
        while (r >= M - i) { r -= M - i; ++i; }
        const int j = i + r;
        const double2 v = R[i * M + j];
        if (2 * e + 1 < nfeat) {
            out[(int64_t)row * nfeat + 2 * e] = (float)(v.x * trs);
            out[(int64_t)row * nfeat + 2 * e + 1] = (float)(v.y * trs);
        }
    }
}

}  // namespace

hipError_t launch_gemm_bf16(int M, int N, int K, const float* A, int64_t sam, int64_t sak, int relu_in_a,
                            const float* B, int64_t sbk, int64_t sbn, int relu_in_b, float alpha,
                            const float* bias, const float* mask, int64_t ldm, int relu_out, float* C,
                            int64_t ldc, hipStream_t s) {
    dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, M, N, K, A, sam, sak, relu_in_a, B, sbk, sbn,
                       relu_in_b, alpha, bias, mask, ldm, relu_out, C, ldc);
    return hipGetLastError();
}

hipError_t launch_colsum(int rows, int cols, const float* X, int64_t ld, float* out, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, s, rows, cols, X, ld, out);
    return hipGetLastError();
}

hipError_t launch_bce(int rows, int cols, const float* Z, const float* Y, float* dZ, float* row_loss,
                      float* loss, hipStream_t s) {
    hipLaunchKernelGGL(bce_kernel, dim3(rows), dim3(256), 0, s, rows, cols, Z, Y, dZ, row_loss);
    hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(64), 0, s, rows, cols, row_loss, loss);
    return hipGetLastError();
}

hipError_t launch_adam(int n, float* p, const float* g, float* m, float* v, float lr, int t, hipStream_t s) {
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, (double)t)), c2 = (float)(1.0 - pow(b2, (double)t));
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, p, g, m, v, lr, (float)b1, (float)b2,
                       (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
    return hipGetLastError();
}

hipError_t launch_features(const int32_t* flist, int n, const FrameDev* frames, const char* ws, float* out,
                           int nfeat, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(n), dim3(128), 0, s, flist, n, frames, ws, out, nfeat);
    return hipGetLastError();
}

}  // namespace nssdoa
