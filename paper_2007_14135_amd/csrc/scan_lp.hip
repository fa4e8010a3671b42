// Step-5 (Table 2) with 16-bit operands: the same real-embedded contraction as the FP32 scan,
// T = Bemb x S with inner dimension 2M, on v_mfma_f32_32x32x16_{bf16,f16} (FP32 accumulation).
//
// Operand layout (D[i][j] += sum_k A[i][k] B[k][j], i, j < 32, k < 16): lane h*32+i holds
// A[i][8h .. 8h+7] and lane h*32+j holds B[8h .. 8h+7][j]; MFMA step s covers inner indices
// 16s .. 16s+15, so a lane holds inner k = 16s + 8h + t (t = 0..7) at step s.  The result layout
// is that of the FP32 32x32 instruction (register r of lane h*32+j: row 8(r/4) + 4h + r%4, column
// j), so the per-frame reduction over 8-row blocks is the same as in the FP32 scan.
// Steering values are formed as in the FP32 scan (phase in FP64, reduced, FP32 sincospi) and
// rounded once to the operand type; embedded B tiles are rounded by the eigen kernel.
// Points whose Q is below max(lowq_tau ||B||_F^2, the frame's 16-bit floor lp_lowq_floor, which
// the eigen kernel stores after ||B||_F^2) go to the FP64 re-evaluation list.
#include <float.h>

#include "internal.h"

namespace nssdoa {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

template <typename T> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf16x8 type; };
template <> struct Vec8<_Float16> { typedef halfx8 type; };

__device__ inline floatx16 mfma16(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ inline floatx16 mfma16(halfx8 a, halfx8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Steering operand of one lane for one 32-angle column tile: inner k = 16s + 8h + t is Re a_k for
// k < M and Im a_(k-M) otherwise.
template <int M, typename T>
__device__ inline void steering16(const double* __restrict__ p, const Dir3& d, int h,
                                  typename Vec8<T>::type* st) {
    constexpr int S = M / 8;
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = 16 * s + 8 * h + t;
            const int m = k < M ? k : k - M;
            const double c = phase_cycles(p + 3 * m, d);   // cycles
            float sn, cs;
            sincospif((float)(2.0 * (c - rint(c))), &sn, &cs);
            st[s][t] = (T)(k < M ? cs : sn);
        }
    }
}

template <int M, typename T>
__global__ __launch_bounds__(256) void scan_lp_kernel(const ScanItem* __restrict__ items,
                                                      const GroupDev* __restrict__ groups,
                                                      const FrameDev* __restrict__ frames,
                                                      const int32_t* __restrict__ blkframe,
                                                      const double* __restrict__ pos,
                                                      char* __restrict__ ws,
                                                      float* __restrict__ spec, int use_user,
                                                      float lowq_tau, LowqList lql) {
    typedef typename Vec8<T>::type V;
    constexpr int S = M / 8;
    const ScanItem it = items[blockIdx.x];
    const GroupDev& g = groups[it.group];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const int base = it.angle_tile * kScanAnglesPerWG + wave * kScanAnglesPerWave;

    V st0[S], st1[S];
    {
        const double* p = pos + g.pos_off;
        const int j = lane & 31;
        steering16<M, T>(p, grid_dir(g, base + j), h, st0);
        steering16<M, T>(p, grid_dir(g, base + 32 + j), h, st1);
    }

    const V* emb = reinterpret_cast<const V*>(ws + g.ws_emb) + (size_t)lane * S;
    const int4* blk4 = reinterpret_cast<const int4*>(blkframe + g.blk_off);
    float q0 = 0.0f, q1 = 0.0f;
    int cur = -1;
    __shared__ ScanLowq lq;                 // low-Q points, published after the loop
    if (threadIdx.x == 0) lq.n = 0;
    __syncthreads();

    auto flush = [&](int f) {
        const float t0 = q0 + __shfl_xor(q0, 32);
        const float t1 = q1 + __shfl_xor(q1, 32);
        const float v = (lane < 32) ? t0 : t1;
        const int l = base + lane;
        const FrameDev& fd = frames[f];
        const bool in = l < g.L;
        if (in) {
            float* out = spec + (use_user ? fd.spec_off_user : fd.spec_off_ws);
            out[l] = 1.0f / fmaxf(v, FLT_MIN);
        }
        const double* qr = reinterpret_cast<const double*>(ws + fd.ws_qref);
        const float thr = fmaxf(lowq_tau * (float)qr[0], (float)qr[1]);
        scan_lowq_collect(in && v < thr, f, wave * kScanAnglesPerWave + lane, lq,
                          reinterpret_cast<int*>(ws + fd.ws_lowq));
    };

    V b[S];
    if (it.t0 < it.t1) {
#pragma unroll
        for (int s = 0; s < S; ++s) b[s] = emb[(size_t)it.t0 * 64 * S + s];
    }
    for (int t = it.t0; t < it.t1; ++t) {
        V bn[S];
        if (t + 1 < it.t1) {
#pragma unroll
            for (int s = 0; s < S; ++s) bn[s] = emb[(size_t)(t + 1) * 64 * S + s];
        }
        floatx16 a0 = {0.0f}, a1 = {0.0f};
#pragma unroll
        for (int s = 0; s < S; ++s) {
            a0 = mfma16(b[s], st0[s], a0);
            a1 = mfma16(b[s], st1[s], a1);
        }
        const int4 fb = blk4[t];
        const int fbk[4] = {fb.x, fb.y, fb.z, fb.w};
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
            const int f = fbk[gq];
            if (f != cur) {
                if (cur >= 0) flush(cur);
                cur = f;
                q0 = 0.0f;
                q1 = 0.0f;
            }
            q0 += a0[4 * gq] * a0[4 * gq] + a0[4 * gq + 1] * a0[4 * gq + 1] +
                  a0[4 * gq + 2] * a0[4 * gq + 2] + a0[4 * gq + 3] * a0[4 * gq + 3];
            q1 += a1[4 * gq] * a1[4 * gq] + a1[4 * gq + 1] * a1[4 * gq + 1] +
                  a1[4 * gq + 2] * a1[4 * gq + 2] + a1[4 * gq + 3] * a1[4 * gq + 3];
        }
#pragma unroll
        for (int s = 0; s < S; ++s) b[s] = bn[s];
    }
    if (cur >= 0) flush(cur);
    __syncthreads();
    scan_lowq_publish(lq, it.angle_tile * kScanAnglesPerWG, lql.count, lql.list, lql.cap, frames, ws);
}

template <int M, typename T>
hipError_t launch_mt(const ScanItem* items, int n_items, const GroupDev* groups, const FrameDev* frames,
                     const int32_t* blkframe, const double* pos, char* ws, float* spec, int use_user,
                     float tau, LowqList lq, hipStream_t s) {
    hipLaunchKernelGGL((scan_lp_kernel<M, T>), dim3(n_items), dim3(256), 0, s, items, groups, frames,
                       blkframe, pos, ws, spec, use_user, tau, lq);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(int M, const ScanItem* items, int n_items, const GroupDev* groups, const FrameDev* frames,
                    const int32_t* blkframe, const double* pos, char* ws, float* spec, int use_user,
                    float tau, LowqList lq, hipStream_t s) {
    switch (M) {
        case 8: return launch_mt<8, T>(items, n_items, groups, frames, blkframe, pos, ws, spec, use_user, tau, lq, s);
        case 16: return launch_mt<16, T>(items, n_items, groups, frames, blkframe, pos, ws, spec, use_user, tau, lq, s);
        case 32: return launch_mt<32, T>(items, n_items, groups, frames, blkframe, pos, ws, spec, use_user, tau, lq, s);
        case 64: return launch_mt<64, T>(items, n_items, groups, frames, blkframe, pos, ws, spec, use_user, tau, lq, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_scan_lp(bool f16, int M, const ScanItem* items, int n_items, const GroupDev* groups,
                          const FrameDev* frames, const int32_t* blkframe, const double* pos, char* ws,
                          float* spec, int use_user, float tau, LowqList lq, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (f16) return launch_t<_Float16>(M, items, n_items, groups, frames, blkframe, pos, ws, spec, use_user, tau, lq, s);
    return launch_t<__bf16>(M, items, n_items, groups, frames, blkframe, pos, ws, spec, use_user, tau, lq, s);
}

}  // namespace nssdoa
