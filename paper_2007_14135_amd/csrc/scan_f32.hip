// Step-5 (Table 2): pseudo-spectrum scan P(theta_l) = 1 / ||B^H a(theta_l)||^2 to FP32 accuracy on
// the matrix cores, for every frame of a group that shares one array geometry and one grid:
// scan_f32_kernel on FP32 operands, scan_split16_kernel (further down) on FP16 hi/lo parts of the
// same FP32 operands.
//
// Real embedding: with a = ar + j ai and a column b of B,
//   Re(b^H a) = br.ar + bi.ai,   Im(b^H a) = -bi.ar + br.ai,
// so the complex contraction becomes the real product T = Bemb (rows) x S (columns) with inner
// dimension 2M, Bemb holding two rows (re-row, im-row) per column of B and S the embedded
// steering vectors (ar; ai).  Frames of a group are stacked along the rows; each frame owns a
// multiple of 8 rows (zero padded), so every 8-row block belongs to exactly one frame and
// Q_f(l) = sum of T^2 over the frame's rows.
//
// MFMA mapping (v_mfma_f32_32x32x2f32, D[i][j] += A[i][k] B[k][j], i, j < 32, k < 2):
//   A operand = Bemb rows (lane h*32+i holds row i, inner 2s+h), B operand = steering
//   (lane h*32+j holds angle j, inner 2s+h), s = 0..M-1 covers the 2M inner values.
//   The accumulator register r of lane h*32+j holds row 8*(r/4) + 4h + r%4 of angle j, so the
//   sum of squares of registers 4g..4g+3 is the half of 8-row block g held by this lane; the
//   other half is in lane j + 32(1-h) and is added once per frame at the write.
// Each wave owns 64 angles (two 32-angle column tiles sharing every A operand); a workgroup of
// four waves owns 256 angles and one chunk of whole frames, whose B tiles it stages in LDS once
// (all four waves read every tile).  Steering values come from the
// group's table (built once per batch by steer_table_kernel: the phase in cycles formed and
// reduced to [-1/2, 1/2] in FP64, then FP32 sincospi), loaded once per work item.  Points whose
// FP32 Q is below lowq_tau ||B||_F^2 are listed in LDS and published to the batch's low-Q list
// after the matrix-core loop.
#include <float.h>

#include "internal.h"

namespace nssdoa {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// One thread per (angle, element): a_m(theta_l) into the group's steering table (see internal.h).
__global__ void steer_table_kernel(const double* __restrict__ pos, GroupDev g, int Lpad, float* __restrict__ T) {
    const int M = g.M;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Lpad * M) return;
    const int l = t / M, m = t - l * M;
    float s = 0.0f, co = 0.0f;
    if (l < g.L) {
        const double c = phase_cycles(pos + 3 * m, grid_dir(g, l));   // cycles
        sincospif((float)(2.0 * (c - rint(c))), &s, &co);
    }
    const int h = m & 1, j = m >> 1;
    T[(size_t)(2 * l + h) * M + j] = co;
    T[(size_t)(2 * l + h) * M + M / 2 + j] = s;
}

// One thread per (angle, element): the FP16 split steering table of P parts (layout in
// internal.h) from the same FP32 values as steer_table_kernel.
template <int P>
__global__ void steer_split_kernel(const double* __restrict__ pos, GroupDev g, int Lpad, _Float16* __restrict__ T) {
    const int M = g.M;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Lpad * M) return;
    const int l = t / M, m = t - l * M;
    float s = 0.0f, co = 0.0f;
    if (l < g.L) {
        const double c = phase_cycles(pos + 3 * m, grid_dir(g, l));   // cycles
        sincospif((float)(2.0 * (c - rint(c))), &s, &co);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {            // inner k = m (Re a_m) and k = M + m (Im a_m)
        const int k = c == 0 ? m : M + m;
        float v = (c == 0 ? co : s) * kSplitSteerScale;             // exact: a power of two
        const int s16 = k >> 4, h = (k >> 3) & 1, tt = k & 7;
#pragma unroll
        for (int part = 0; part < P; ++part) {
            const _Float16 x = (_Float16)v;
            v -= (float)x;                                           // exact in FP32
            T[((size_t)2 * P * l + 2 * part + h) * M + 8 * s16 + tt] = x;
        }
    }
}

// Sum over the two 32-row halves of a column tile pair: lanes 0-31 return q0(l) + q0(l + 32) and
// lanes 32-63 return q1(l - 32) + q1(l) (one v_permlane32_swap: the upper half of q0 trades
// places with the lower half of q1).
__device__ inline float halves_sum(float q0, float q1) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(q0), __float_as_uint(q1), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The steering operand of lane h*32 + j for grid index l: M contiguous floats of the table.
template <int M>
__device__ inline void steering_load(const float* __restrict__ T, int l, int h, float* st) {
    const float4* src = reinterpret_cast<const float4*>(T + (size_t)(2 * l + h) * M);
#pragma unroll
    for (int v = 0; v < M / 4; ++v) {
        const float4 x = src[v];
        st[4 * v] = x.x; st[4 * v + 1] = x.y; st[4 * v + 2] = x.z; st[4 * v + 3] = x.w;
    }
}

template <int M>
__global__ __launch_bounds__(256) void scan_f32_kernel(const ScanItem* __restrict__ items,
                                                       const GroupDev* __restrict__ groups,
                                                       const FrameDev* __restrict__ frames,
                                                       const int32_t* __restrict__ blkframe,
                                                       const float* __restrict__ steer,
                                                       char* __restrict__ ws,
                                                       float* __restrict__ spec, int use_user,
                                                       float lowq_tau, LowqList lql) {
    const ScanItem it = items[blockIdx.x];
    const GroupDev& g = groups[it.group];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const int base = it.angle_tile * kScanAnglesPerWG + wave * kScanAnglesPerWave;
    const int gL = g.L;

    float st0[M], st1[M];
    {
        const float* T = steer + g.steer_off;
        const int j = lane & 31;
        steering_load<M>(T, base + j, h, st0);
        steering_load<M>(T, base + 32 + j, h, st1);
    }

    // the work item's B tiles, staged once in LDS for the four waves (they share every row), and
    // per 8-row block its frame with that frame's output row, low-Q threshold and flag
    extern __shared__ float4 embs[];
    __shared__ ScanLowq lq;
    __shared__ __align__(16) int bfr[kScanMaxBlocks];
    __shared__ float bthr[kScanMaxBlocks];
    __shared__ int64_t bso[kScanMaxBlocks];
    __shared__ int* bflag[kScanMaxBlocks];
    constexpr int kTile4 = 64 * M / 4;                       // float4 per 32-row tile
    const int nblk = (it.t1 - it.t0) * 4;
    if (threadIdx.x == 0) lq.n = 0;
    {
        const float4* src = reinterpret_cast<const float4*>(ws + g.ws_emb) + (size_t)it.t0 * kTile4;
        const int n4 = (it.t1 - it.t0) * kTile4;
        for (int i = threadIdx.x; i < n4; i += blockDim.x) embs[i] = src[i];
        for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
            const int f = blkframe[g.blk_off + it.t0 * 4 + i];
            bfr[i] = f;
            if (f >= 0) {
                const FrameDev& fd = frames[f];
                bso[i] = use_user ? fd.spec_off_user : fd.spec_off_ws;
                bthr[i] = lowq_tau * (float)*reinterpret_cast<const double*>(ws + fd.ws_qref);
                bflag[i] = reinterpret_cast<int*>(ws + fd.ws_lowq);
            }
        }
    }
    __syncthreads();
    float q0 = 0.0f, q1 = 0.0f;
    int cur = -1, curf = -1;                     // a block and the frame being summed (-1: padding)

    auto flush = [&](int bi) {
        const float v = halves_sum(q0, q1);
        const int l = base + lane;          // col tile lane/32, angle lane%32
        const bool in = l < gL;
        if (in) spec[bso[bi] + l] = __builtin_amdgcn_rcpf(fmaxf(v, FLT_MIN));
        scan_lowq_collect(in && v < bthr[bi], bfr[bi], wave * kScanAnglesPerWave + lane, lq, bflag[bi]);
    };

    for (int t = it.t0; t < it.t1; ++t) {
        float b[M];
        const float4* src = embs + (t - it.t0) * kTile4 + lane;
#pragma unroll
        for (int v = 0; v < M / 4; ++v) {
            const float4 x = src[v * 64];
            b[4 * v] = x.x; b[4 * v + 1] = x.y; b[4 * v + 2] = x.z; b[4 * v + 3] = x.w;
        }
        floatx16 a0 = {0.0f}, a1 = {0.0f};
#pragma unroll
        for (int s = 0; s < M; ++s) {
            a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(b[s], st0[s], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(b[s], st1[s], a1, 0, 0, 0);
        }
        const int b0 = (t - it.t0) * 4;
        const int4 fb = *reinterpret_cast<const int4*>(bfr + b0);
        const int fbk[4] = {fb.x, fb.y, fb.z, fb.w};
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
            const int f = fbk[gq];
            if (f != curf) {
                if (curf >= 0) flush(cur);
                cur = b0 + gq;
                curf = f;
                q0 = 0.0f;
                q1 = 0.0f;
            }
            q0 += a0[4 * gq] * a0[4 * gq] + a0[4 * gq + 1] * a0[4 * gq + 1] +
                  a0[4 * gq + 2] * a0[4 * gq + 2] + a0[4 * gq + 3] * a0[4 * gq + 3];
            q1 += a1[4 * gq] * a1[4 * gq] + a1[4 * gq + 1] * a1[4 * gq + 1] +
                  a1[4 * gq + 2] * a1[4 * gq + 2] + a1[4 * gq + 3] * a1[4 * gq + 3];
        }
    }
    if (curf >= 0) flush(cur);
    __syncthreads();
    scan_lowq_publish(lq, it.angle_tile * kScanAnglesPerWG, lql.count, lql.list, lql.cap, frames, ws);
}

// The FP16 split scan (C64 default): the same work items, per-frame reduction and low-Q
// collection as scan_f32_kernel, on v_mfma_f32_32x32x16_f16; each wave reads the B tiles from L2
// itself, one tile ahead, instead of staging them in LDS.  Each FP32 product a b of the
// real-embedded contraction is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b of the operands'
// FP16 parts (B tiles scaled per frame by 2^e, steering by 2^13, both exact), accumulated in FP32;
// the frame's Q is the sum of squares times its scale 2^-2e 2^-26 (qref[1]).
// Operand layout (D[i][j] += sum_k A[i][k] B[k][j], k < 16 per step s): lane h*32+i holds
// A[i][16s + 8h .. 16s + 8h + 7] (B rows) and lane h*32+j holds B[16s + 8h .. +7][j] (steering);
// the result layout is that of the FP32 32x32 instruction.
// Products of the parts that the split keeps: with P = 2, hi hi + hi lo + lo hi; with P = 3,
// every pair of parts whose orders add up to at most 2 (hi hi, hi mid, mid hi, hi lo, lo hi,
// mid mid), so the dropped products are below 2^-33 of |a b| (their orders add up to 3 or more).
// Word 3 of a raw (untyped) buffer resource on gfx9-family GPUs: 32-bit data format, no swizzle.
constexpr int kRawBufferFlags = 0x00020000;
// s_waitcnt operand on gfx9-family GPUs waiting for vmcnt = 0 only (expcnt 7, lgkmcnt 15 left
// unconstrained, vmcnt bits [3:0] and [15:14] zero).
constexpr int kWaitVmcnt0 = 0x0F70;

template <int P>
__device__ __forceinline__ void split_mfma(const halfx8* bp, const halfx8* s0, const halfx8* s1, floatx16& a0,
                                           floatx16& a1) {
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (i + j <= P - 1) {
                a0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(bp[i], s0[j], a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(bp[i], s1[j], a1, 0, 0, 0);
            }
}

template <int M, int P>
__global__ __launch_bounds__(256) void scan_split16_kernel(const ScanItem* __restrict__ items,
                                                           const GroupDev* __restrict__ groups,
                                                           const FrameDev* __restrict__ frames,
                                                           const int32_t* __restrict__ blkframe,
                                                           const float* __restrict__ steer,
                                                           char* __restrict__ ws,
                                                           float* __restrict__ spec, int use_user,
                                                           float lowq_tau, LowqList lql) {
    constexpr int S = M / 8;                                 // 16-deep MFMA steps over 2M
    const ScanItem it = items[blockIdx.x];
    const GroupDev& g = groups[it.group];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const int base = it.angle_tile * kScanAnglesPerWG + wave * kScanAnglesPerWave;
    const int gL = g.L;

    halfx8 st0[S][P], st1[S][P];             // steering parts of the two column tiles
    {
        const _Float16* T = reinterpret_cast<const _Float16*>(steer + g.steer_x16_off);
        const int j = lane & 31;
        const halfx8* p0 = reinterpret_cast<const halfx8*>(T + ((size_t)2 * P * (base + j) + h) * M);
        const halfx8* p1 = reinterpret_cast<const halfx8*>(T + ((size_t)2 * P * (base + 32 + j) + h) * M);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int q = 0; q < P; ++q) {
                st0[s][q] = p0[2 * S * q + s];   // part q is 2qM halves further
                st1[s][q] = p1[2 * S * q + s];
            }
    }

    __shared__ ScanLowq lq;
    __shared__ int bovf[kScanMaxBlocks];          // a frame's low-Q entries did not fit in lq
    constexpr int kTile8 = P * S * 64;                       // halfx8 per 32-row tile (all parts)
    const int nblk = (it.t1 - it.t0) * 4;
    // B tiles: each wave reads them from global memory (L2) itself, one tile ahead, into two
    // operand buffers used in turn
    const halfx8* emb = reinterpret_cast<const halfx8*>(ws + g.ws_emb) + lane;
    halfx8 opA[S][P], opB[S][P];
    if (it.t0 < it.t1) {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int q = 0; q < P; ++q) opA[s][q] = emb[(size_t)it.t0 * kTile8 + (q * S + s) * 64];
    }
    // LDS state behind a barrier that waits for no global load
    if (threadIdx.x == 0) lq.n = 0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) bovf[i] = 0;
    __syncthreads();
    // Per-block parameters in registers, block i of the item in lane i % 64 of set i / 64 (at
    // most kScanMaxBlocks = 128 blocks), read with readlane: its frame, output offset, Q scale and
    // low-Q threshold.  Every wave loads its own copy; nothing waits for them before the first
    // tile's epilogue.
    static_assert(kScanMaxBlocks <= 128, "two lane sets of block parameters");
    int pf[2];
    int64_t pso[2];
    float pqs[2], pthr[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = lane + 64 * k;
        pf[k] = -1;
        pso[k] = 0;
        pqs[k] = 0.0f;
        pthr[k] = 0.0f;
        if (i < nblk) {
            const int f = blkframe[g.blk_off + it.t0 * 4 + i];
            pf[k] = f;
            if (f >= 0) {
                const FrameDev& fd = frames[f];
                const double* qr = reinterpret_cast<const double*>(ws + fd.ws_qref);
                pso[k] = use_user ? fd.spec_off_user : fd.spec_off_ws;
                pthr[k] = lowq_tau * (float)qr[0];
                pqs[k] = (float)qr[1];
            }
        }
    }
    auto lane_i32 = [&](const int (&x)[2], int b) { return __builtin_amdgcn_readlane(b < 64 ? x[0] : x[1], b & 63); };
    auto lane_f32 = [&](const float (&x)[2], int b) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b < 64 ? x[0] : x[1]), b & 63));
    };
    auto lane_i64 = [&](const int64_t (&x)[2], int b) {
        const int64_t v = b < 64 ? x[0] : x[1];
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, b & 63);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), b & 63);
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    float q0 = 0.0f, q1 = 0.0f;
    int curf = -1;                               // the frame being summed (-1: none yet)
    // the frame's output offset, Q scale and low-Q threshold, read when the frame starts
    int64_t c_so = 0;
    float c_qs = 0.0f, c_thr = 0.0f;
    int c_blk = 0;

    // Spectrum writes are software-pipelined: a tile's finished frames (at most one per 8-row
    // block) are held in registers and stored at the start of the next iteration, before the B
    // prefetch and the matrix instructions, with a buffer store per block (a zero-length record
    // where no frame ends, angles past the grid outside the record).  Each iteration begins
    // with one wait for everything issued in the previous one (its operands and stores), so the
    // loads and stores it issues stay in flight behind its matrix and epilogue work.
    const int l = base + lane;               // col tile lane/32, angle lane%32
    float pv[4];
    __amdgpu_buffer_rsrc_t prs[4];
    const __amdgpu_buffer_rsrc_t none = __builtin_amdgcn_make_buffer_rsrc(spec, (short)0, 0, kRawBufferFlags);
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
        pv[gq] = 0.0f;
        prs[gq] = none;
    }
    auto finish = [&](int gq) {               // the frame summed so far ends before block gq
        const float v = halves_sum(q0, q1) * c_qs;
        scan_lowq_collect(l < gL && v < c_thr, curf, wave * kScanAnglesPerWave + lane, lq, &bovf[c_blk]);
        const uint64_t addr = reinterpret_cast<uint64_t>(spec + c_so);
        float* rowp = reinterpret_cast<float*>(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32)) << 32) |
                                               (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)addr));
        pv[gq] = __builtin_amdgcn_rcpf(fmaxf(v, FLT_MIN));
        prs[gq] = __builtin_amdgcn_make_buffer_rsrc(rowp, (short)0, 4 * gL, kRawBufferFlags);
    };

    // One tile: its operands are in `cur`, the next tile's go to `nxt`.
    auto tile = [&](int t, halfx8 (&cur)[S][P], halfx8 (&nxt)[S][P]) {
        // this tile's operands and the previous tile's stores, all issued one iteration ago
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __builtin_amdgcn_sched_barrier(0);
        // the previous tile's frames
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(pv[gq]), prs[gq], 4 * l, 0, 0);
            prs[gq] = none;
        }
        __builtin_amdgcn_sched_barrier(0);
        {
            // the next tile (the last one reloads itself: a fixed number of loads per tile), in
            // flight during this tile's matrix instructions and epilogue
            const int tn = min(t + 1, it.t1 - 1);
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int q = 0; q < P; ++q) nxt[s][q] = emb[(size_t)tn * kTile8 + (q * S + s) * 64];
        }
        __builtin_amdgcn_sched_barrier(0);
        floatx16 a0 = {0.0f}, a1 = {0.0f};
#pragma unroll
        for (int s = 0; s < S; ++s) split_mfma<P>(cur[s], st0[s], st1[s], a0, a1);
        __builtin_amdgcn_sched_barrier(0);
        const int b0 = (t - it.t0) * 4;
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
            const int f = lane_i32(pf, b0 + gq);
            if (f != curf) {
                if (curf >= 0) finish(gq);
                curf = f;
                q0 = 0.0f;
                q1 = 0.0f;
                if (f >= 0) {
                    c_so = lane_i64(pso, b0 + gq);
                    c_qs = lane_f32(pqs, b0 + gq);
                    c_thr = lane_f32(pthr, b0 + gq);
                    c_blk = b0 + gq;
                }
            }
            q0 += a0[4 * gq] * a0[4 * gq] + a0[4 * gq + 1] * a0[4 * gq + 1] +
                  a0[4 * gq + 2] * a0[4 * gq + 2] + a0[4 * gq + 3] * a0[4 * gq + 3];
            q1 += a1[4 * gq] * a1[4 * gq] + a1[4 * gq + 1] * a1[4 * gq + 1] +
                  a1[4 * gq + 2] * a1[4 * gq + 2] + a1[4 * gq + 3] * a1[4 * gq + 3];
        }
    };
    for (int t = it.t0; t < it.t1; t += 2) {
        tile(t, opA, opB);
        if (t + 1 >= it.t1) break;
        tile(t + 1, opB, opA);
    }
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(pv[gq]), prs[gq], 4 * l, 0, 0);
        prs[gq] = none;
    }
    if (curf >= 0) {                          // the last frame of the work item
        finish(0);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(pv[0]), prs[0], 4 * l, 0, 0);
    }
    __syncthreads();
    if (wave == 0) {                          // low-Q overflow flags of the item's frames
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = lane + 64 * k;
            if (i < nblk && bovf[i] && pf[k] >= 0) *reinterpret_cast<int*>(ws + frames[pf[k]].ws_lowq) = 1;
        }
    }
    scan_lowq_publish(lq, it.angle_tile * kScanAnglesPerWG, lql.count, lql.list, lql.cap, frames, ws);
}

template <int M>
hipError_t launch_split(int parts, const ScanItem* items, int n_items, const GroupDev* groups,
                        const FrameDev* frames, const int32_t* blkframe, const float* steer, char* ws, float* spec,
                        int use_user, float tau, LowqList lq, hipStream_t s) {
    if (parts == 3)
        hipLaunchKernelGGL((scan_split16_kernel<M, 3>), dim3(n_items), dim3(256), 0, s, items, groups, frames,
                           blkframe, steer, ws, spec, use_user, tau, lq);
    else
        hipLaunchKernelGGL((scan_split16_kernel<M, 2>), dim3(n_items), dim3(256), 0, s, items, groups, frames,
                           blkframe, steer, ws, spec, use_user, tau, lq);
    return hipGetLastError();
}

template <int M>
hipError_t launch_m(const ScanItem* items, int n_items, int max_tiles, const GroupDev* groups,
                    const FrameDev* frames, const int32_t* blkframe, const float* steer, char* ws, float* spec,
                    int use_user, float tau, LowqList lq, hipStream_t s) {
    const size_t lds = (size_t)max_tiles * 64 * M * sizeof(float);
    hipLaunchKernelGGL(scan_f32_kernel<M>, dim3(n_items), dim3(256), lds, s, items, groups, frames,
                       blkframe, steer, ws, spec, use_user, tau, lq);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_steer_table(const double* pos, const GroupDev& g, float* table, hipStream_t s) {
    const int Lpad = steer_table_rows(g.L);
    const int64_t n = (int64_t)Lpad * g.M;
    hipLaunchKernelGGL(steer_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, g, Lpad, table);
    return hipGetLastError();
}

hipError_t launch_steer_table_split16(int parts, const double* pos, const GroupDev& g, float* table, hipStream_t s) {
    const int Lpad = steer_table_rows(g.L);
    const int64_t n = (int64_t)Lpad * g.M;
    if (parts == 3)
        hipLaunchKernelGGL(steer_split_kernel<3>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, g, Lpad,
                           reinterpret_cast<_Float16*>(table));
    else
        hipLaunchKernelGGL(steer_split_kernel<2>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, g, Lpad,
                           reinterpret_cast<_Float16*>(table));
    return hipGetLastError();
}

hipError_t launch_scan_split16(int parts, int M, const ScanItem* items, int n_items, int max_tiles,
                               const GroupDev* groups, const FrameDev* frames, const int32_t* blkframe,
                               const float* steer, char* ws, float* spec, int use_user, float tau, LowqList lq,
                               hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (max_tiles * 4 > kScanMaxBlocks || (parts != 2 && parts != 3)) return hipErrorInvalidValue;
    switch (M) {
        case 8: return launch_split<8>(parts, items, n_items, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        case 16: return launch_split<16>(parts, items, n_items, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        case 32: return launch_split<32>(parts, items, n_items, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        case 64: return launch_split<64>(parts, items, n_items, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scan_f32(int M, const ScanItem* items, int n_items, int max_tiles, const GroupDev* groups,
                           const FrameDev* frames, const int32_t* blkframe, const float* steer,
                           char* ws, float* spec, int use_user, float tau, LowqList lq, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if ((size_t)max_tiles * 64 * M * sizeof(float) > kScanLdsBytes) return hipErrorInvalidValue;
    switch (M) {
        case 8: return launch_m<8>(items, n_items, max_tiles, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        case 16: return launch_m<16>(items, n_items, max_tiles, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        case 32: return launch_m<32>(items, n_items, max_tiles, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        case 64: return launch_m<64>(items, n_items, max_tiles, groups, frames, blkframe, steer, ws, spec, use_user, tau, lq, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nssdoa
