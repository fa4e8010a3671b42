// Alternative forms of the Table 2 Step-5 scan, for measuring what the factored form buys: every
// grid point in plain FP32 on the vector ALUs, without the FP64 re-evaluation of low-Q points.
//   factored   Q = ||B^H a||^2, the form of the library's scans (C = B B^H, Table 3), a sum of
//              squares;
//   quadratic  Q = Re a^H C a with C = B B^H formed in FP64 and rounded to FP32: the form
//              Table 2 Step-5 writes, M^2 terms that cancel down to Q near a null;
//   complement Q = ||a||^2 - ||E_s^H a||^2 (MUSIC: C = I - E_s E_s^H), D terms subtracted from M.
// One workgroup per (frame, chunk of 4096 grid points): the frame's operand (B, C or E_s) is read
// from the estimate's workspace into LDS in FP32, then each thread forms its points' FP32 steering vector
// (phase in cycles formed and reduced in FP64, then FP32 sincospi, as the steering tables) and Q,
// and writes P = 1 / max(Q, FLT_MIN).
#include <float.h>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {

constexpr int kFormPoints = 256;

template <int MB>
__global__ __launch_bounds__(kFormPoints) void scan_form_kernel(const PointItem* __restrict__ items,
                                                                const FrameDev* __restrict__ frames,
                                                                const double* __restrict__ pos,
                                                                const char* __restrict__ ws, int form,
                                                                float* __restrict__ spec) {
    __shared__ float2 op[MB * MB];       // B (M x K), C (M x M) or E_s (M x D), column-major
    const PointItem it = items[blockIdx.x];
    const FrameDev& fr = frames[it.frame];
    const int M = fr.M, tid = threadIdx.x;
    const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
    const double2* U = reinterpret_cast<const double2*>(ws + fr.ws_evecs);   // row-major, column r = e_r
    int ncol;
    if (form == NSSDOA_FORM_QUADRATIC) {
        ncol = M;
        for (int e = tid; e < M * M; e += blockDim.x) {
            const int j = e / M, i = e - j * M;            // C[i][j] = sum_k b_ik conj(b_jk)
            double re = 0.0, im = 0.0;
            for (int k = 0; k < fr.K; ++k) {
                const double2 bi = B[(size_t)k * M + i], bj = B[(size_t)k * M + j];
                re = fma(bi.x, bj.x, fma(bi.y, bj.y, re));
                im = fma(bi.y, bj.x, fma(-bi.x, bj.y, im));
            }
            op[j * M + i] = make_float2((float)re, (float)im);
        }
    } else if (form == NSSDOA_FORM_COMPLEMENT) {
        ncol = fr.D;
        for (int e = tid; e < M * fr.D; e += blockDim.x) {
            const int r = e / M, i = e - r * M;
            const double2 u = U[(size_t)i * M + r];
            op[r * M + i] = make_float2((float)u.x, (float)u.y);
        }
    } else {
        ncol = fr.K;
        for (int e = tid; e < M * fr.K; e += blockDim.x) {
            const double2 b = B[e];
            op[e] = make_float2((float)b.x, (float)b.y);
        }
    }
    __syncthreads();
    const int lend = min(fr.L, it.l0 + kRefineChunk);
    for (int l = it.l0 + tid; l < lend; l += blockDim.x) {
        const double* ps = pos + fr.pos_off;
        const Dir3 d = grid_dir(fr, l);
        float ar[MB], ai[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            ar[m] = 0.0f;
            ai[m] = 0.0f;
            if (m < M) {
                const double c = phase_cycles(ps + 3 * m, d);
                sincospif((float)(2.0 * (c - rint(c))), &ai[m], &ar[m]);
            }
        }
        float Q = 0.0f;
        if (form == NSSDOA_FORM_QUADRATIC) {
            // Re sum_i conj(a_i) (C a)_i
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                if (i >= M) break;
                float yr = 0.0f, yi = 0.0f;
#pragma unroll
                for (int j = 0; j < MB; ++j) {
                    if (j < M) {
                        const float2 c = op[j * M + i];
                        yr = fmaf(c.x, ar[j], fmaf(-c.y, ai[j], yr));
                        yi = fmaf(c.x, ai[j], fmaf(c.y, ar[j], yi));
                    }
                }
                Q = fmaf(ar[i], yr, fmaf(ai[i], yi, Q));
            }
        } else {
            float s = 0.0f;
            for (int k = 0; k < ncol; ++k) {
                float yr = 0.0f, yi = 0.0f;
#pragma unroll
                for (int m = 0; m < MB; ++m) {
                    if (m < M) {
                        const float2 b = op[k * M + m];        // conj(b) a
                        yr = fmaf(b.x, ar[m], fmaf(b.y, ai[m], yr));
                        yi = fmaf(b.x, ai[m], fmaf(-b.y, ar[m], yi));
                    }
                }
                s = fmaf(yr, yr, fmaf(yi, yi, s));
            }
            if (form == NSSDOA_FORM_COMPLEMENT) {
                float a2 = 0.0f;
#pragma unroll
                for (int m = 0; m < MB; ++m) a2 = fmaf(ar[m], ar[m], fmaf(ai[m], ai[m], a2));
                Q = a2 - s;
            } else {
                Q = s;
            }
        }
        spec[fr.spec_off_user + l] = 1.0f / fmaxf(Q, FLT_MIN);
    }
}

}  // namespace

hipError_t launch_scan_form(int bucket_M, const PointItem* items, int n_items, const FrameDev* frames,
                            const double* pos, const char* ws, int form, float* spec, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (bucket_M) {
        case 8: hipLaunchKernelGGL(scan_form_kernel<8>, dim3(n_items), dim3(kFormPoints), 0, s, items, frames, pos, ws, form, spec); break;
        case 16: hipLaunchKernelGGL(scan_form_kernel<16>, dim3(n_items), dim3(kFormPoints), 0, s, items, frames, pos, ws, form, spec); break;
        case 32: hipLaunchKernelGGL(scan_form_kernel<32>, dim3(n_items), dim3(kFormPoints), 0, s, items, frames, pos, ws, form, spec); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nssdoa
