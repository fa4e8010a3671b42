// Windowed estimation: the Table 2 Step-5 scan and the Step-6 peak search restricted to angle
// windows chosen from per-bin scores (the learned proposal network's logits, or any caller
// scores).  Every kernel here reads the per-frame work that the proposal kernel wrote on the
// device, so the host issues the whole sequence without waiting for it.
//
// proposal_kernel, one wave per frame: bin b covers [-90 + b w, -90 + (b+1) w) deg with
//   w = 180 / n_bins.  The topk best bins (ties to the lower bin; after the first D of them only
//   those scoring at least the floor; optionally only local maxima of the score curve) give
//   windows centre +- half width, snapped to the frame's grid, sorted and merged.  A frame whose best score is below
//   the threshold falls back to one window over its whole grid.  It also counts the frame's
//   64-angle scan items and 4096-point peak chunks.
// prefix_kernel, one workgroup: exclusive prefix sums of per-frame counts (a block scan);
// expand_kernel, one wave per frame: the frame's scan items and peak chunks written out at those
//   offsets, so that the kernels below read their work item with one load.
// scan_win_kernel<M, PARTS>, grid-stride over 64-angle items, one wave per item: one frame's
//   angles in one window, contracted on the matrix cores with the frame's own 8-row blocks of the
//   packed B tiles (the operands, steering tables and epilogue of the group scans: FP32 operands,
//   or FP16 split operands of 2 or 3 parts with 3 or 6 products per FP32-accuracy product).
// lowq_win_kernel<MB>, grid-stride over 64-entry slices of the frames' low-Q lists: FP64
//   re-evaluation of the listed points.
// winpeaks_kernel<MB>, grid-stride over 4096-point chunks of the windows, one workgroup per
//   chunk: the chunk's best D + extra plateau winners to its candidate slots.  Values outside a
//   window are unknown, so a window's end points are never peaks.
// rescue_kernel, one thread per frame, after the peak selection: a frame whose windows held fewer
//   than D peaks (a proposal that missed a source, or a peak whose plateau reaches a window end)
//   gets one window over its whole grid and is searched again by the same kernels; every other
//   frame gets no work in that second pass and keeps its peaks.
#include <float.h>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
constexpr int kHaloW = 16;

__device__ inline double qnan_d() { return __longlong_as_double(0x7ff8000000000000LL); }

// window of bin b: centre c, start index ceil((c - hw - start) / step - 1e-9), end (exclusive)
// floor((c + hw - start) / step + 1e-9) + 1, every operation rounded separately
__device__ inline void window_of_bin(int b, double width, double hw, double start, double step, int L,
                                     int* l0, int* l1) {
#pragma clang fp contract(off)
    const double c = -90.0 + ((double)b + 0.5) * width;
    const double lo = (c - hw - start) / step - 1e-9;
    const double hi = (c + hw - start) / step + 1e-9;
    *l0 = (int)fmax(ceil(lo), 0.0);
    *l1 = (int)fmin(floor(hi) + 1.0, (double)L);
}

__global__ __launch_bounds__(64) void proposal_kernel(const FrameDev* __restrict__ frames, int n_frames,
                                                      const float* __restrict__ scores, int n_bins, int topk,
                                                      double half_window, float threshold, float floor,
                                                      int local_max, char* __restrict__ ws, LearnedLayout lay,
                                                      uint32_t* __restrict__ status) {
    const int f = blockIdx.x;
    if (f >= n_frames) return;
    const FrameDev& fr = frames[f];
    const int lane = threadIdx.x;
    __shared__ float sc[kMaxBins];
    __shared__ int chosen[kMaxWindows];
    const float* z = scores + (size_t)f * n_bins;
    for (int b = lane; b < n_bins; b += 64) sc[b] = z[b];
    __syncthreads();
    if (local_max) {
        // only local maxima of the score curve stay eligible (NaN counts as -inf): above the left
        // neighbour, and the run of equal scores starting here ends lower or at the last bin;
        // every other bin becomes NaN.  The best score is a local maximum, so the threshold test
        // is unchanged.
        constexpr int kPer = kMaxBins / 64;
        float keep[kPer];
        auto val = [&](int b) { const float x = sc[b]; return x == x ? x : -INFINITY; };
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int b = lane + 64 * k;
            keep[k] = __int_as_float(0x7fc00000);
            if (b >= n_bins || sc[b] != sc[b]) continue;
            const float v = sc[b];
            if (b > 0 && !(v > val(b - 1))) continue;
            int e = b;
            while (e + 1 < n_bins && val(e + 1) == v) ++e;
            if (e + 1 == n_bins || val(e + 1) < v) keep[k] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (lane + 64 * k < n_bins) sc[lane + 64 * k] = keep[k];
        __syncthreads();
    }
    // best score (the fallback test) and the topk best bins; NaN scores never win
    float best = -INFINITY;
    int nch = 0;
    for (int r = 0; r < topk; ++r) {
        float v = -INFINITY;
        int bi = 1 << 30;
        for (int b = lane; b < n_bins; b += 64)
            if (sc[b] > v || (sc[b] == v && b < bi)) { v = sc[b]; bi = b; }
        for (int o = 32; o > 0; o >>= 1) {
            const float v2 = __shfl_xor(v, o);
            const int b2 = __shfl_xor(bi, o);
            if (v2 > v || (v2 == v && b2 < bi)) { v = v2; bi = b2; }
        }
        if (r == 0) best = v;
        if (bi >= n_bins) break;          // uniform: every lane holds the reduced value
        if (r >= fr.D && !(v >= floor)) break;   // bins beyond the source count need the floor
        if (lane == 0) {
            chosen[nch] = bi;
            sc[bi] = __int_as_float(0x7fc00000);   // NaN: never chosen again
        }
        ++nch;
        __syncthreads();
    }
    if (lane != 0) return;
    int* W = reinterpret_cast<int*>(ws + lay.off_win) + (size_t)f * kWinStride;
    int nw = 0;
    if (status[f] & NSSDOA_ST_NONFINITE_INPUT) {
        nw = 0;                           // nothing to scan
    } else if (!(best >= threshold)) {
        W[1] = 0;
        W[2] = fr.L;
        nw = 1;
        status[f] |= NSSDOA_ST_FALLBACK_USED;
    } else {
        const double width = 180.0 / (double)n_bins;
        int l0s[kMaxWindows], l1s[kMaxWindows];
        for (int i = 0; i < nch; ++i) {
            int a, e;
            window_of_bin(chosen[i], width, half_window, fr.grid_start, fr.grid_step, fr.L, &a, &e);
            int j = i;                    // insertion by (start, end)
            while (j > 0 && (l0s[j - 1] > a || (l0s[j - 1] == a && l1s[j - 1] > e))) {
                l0s[j] = l0s[j - 1];
                l1s[j] = l1s[j - 1];
                --j;
            }
            l0s[j] = a;
            l1s[j] = e;
        }
        for (int i = 0; i < nch; ++i) {
            if (l1s[i] <= l0s[i]) continue;
            if (nw > 0 && l0s[i] <= W[2 * nw]) {
                W[2 * nw] = max(W[2 * nw], l1s[i]);
            } else {
                W[1 + 2 * nw] = l0s[i];
                W[2 + 2 * nw] = l1s[i];
                ++nw;
            }
        }
    }
    W[0] = nw;
    int items = 0, chunks = 0;
    for (int i = 0; i < nw; ++i) {
        const int len = W[2 + 2 * i] - W[1 + 2 * i];
        items += (len + kScanAnglesPerWave - 1) / kScanAnglesPerWave;
        chunks += (len + kRefineChunk - 1) / kRefineChunk;
    }
    reinterpret_cast<int*>(ws + lay.off_items)[f] = items;
    reinterpret_cast<int*>(ws + lay.off_chunks)[f] = chunks;
}

// low-Q slices per frame: ceil(min(count, capacity) / 64)
__global__ void lowq_count_kernel(const FrameDev* __restrict__ frames, int n_frames, char* __restrict__ ws,
                                  LearnedLayout lay) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < n_frames; f += gridDim.x * blockDim.x) {
        const FrameDev& fr = frames[f];
        const int n = min(*reinterpret_cast<const int*>(ws + fr.ws_lowq), fr.lowq_cap);
        reinterpret_cast<int*>(ws + lay.off_lowq)[f] = (n + 63) / 64;
    }
}

__global__ void rescue_kernel(const FrameDev* __restrict__ frames, const int32_t* __restrict__ flist, int n_list,
                              const int32_t* __restrict__ npeaks, uint32_t* __restrict__ status,
                              char* __restrict__ ws, LearnedLayout lay, int32_t* __restrict__ rescue) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_list; i += gridDim.x * blockDim.x) {
        const int f = flist[i];
        const FrameDev& fr = frames[f];
        const uint32_t st = status[f];
        const bool again = !(st & (NSSDOA_ST_NONFINITE_INPUT | NSSDOA_ST_FALLBACK_USED)) && npeaks[f] < fr.D;
        int* W = reinterpret_cast<int*>(ws + lay.off_win) + (size_t)f * kWinStride;
        int items = 0, chunks = 0;
        if (again) {
            W[0] = 1;
            W[1] = 0;
            W[2] = fr.L;
            items = (fr.L + kScanAnglesPerWave - 1) / kScanAnglesPerWave;
            chunks = (fr.L + kRefineChunk - 1) / kRefineChunk;
            status[f] = (st & ~(NSSDOA_ST_FEWER_PEAKS | NSSDOA_ST_PEAK_OVERFLOW)) | NSSDOA_ST_FALLBACK_USED;
        } else {
            W[0] = 0;
        }
        reinterpret_cast<int*>(ws + lay.off_items)[f] = items;
        reinterpret_cast<int*>(ws + lay.off_chunks)[f] = chunks;
        *reinterpret_cast<int*>(ws + fr.ws_lowq) = 0;      // the second pass's low-Q list
        rescue[i] = again ? f : -1;
    }
}

// off[i] = sum of cnt[0..i-1] for i = 0..n (off has n + 1 entries), for one or two arrays.
__global__ __launch_bounds__(1024) void prefix_kernel(int n, const int* __restrict__ cnt_a, int* __restrict__ off_a,
                                                      const int* __restrict__ cnt_b, int* __restrict__ off_b) {
    __shared__ int sa[1024], sb[1024];
    const int tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
    int a = 0, b = 0;
    for (int i = i0; i < i1; ++i) {
        a += cnt_a[i];
        if (cnt_b) b += cnt_b[i];
    }
    sa[tid] = a;
    sb[tid] = b;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {          // inclusive Hillis-Steele scan
        const int xa = tid >= d ? sa[tid - d] : 0;
        const int xb = tid >= d ? sb[tid - d] : 0;
        __syncthreads();
        sa[tid] += xa;
        sb[tid] += xb;
        __syncthreads();
    }
    int ra = sa[tid] - a, rb = sb[tid] - b;       // exclusive
    for (int i = i0; i < i1; ++i) {
        off_a[i] = ra;
        ra += cnt_a[i];
        if (cnt_b) {
            off_b[i] = rb;
            rb += cnt_b[i];
        }
    }
    if (tid == 1023) {
        off_a[n] = sa[1023];
        if (cnt_b) off_b[n] = sb[1023];
    }
}

// One wave per frame: the frame's scan items and peak chunks, at its prefix-sum offsets.
__global__ void expand_kernel(const FrameDev* __restrict__ frames, int n_frames, char* __restrict__ ws,
                              LearnedLayout lay) {
    const int f = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (f >= n_frames) return;                     // uniform per wave
    const int lane = threadIdx.x & 63;
    const int* W = reinterpret_cast<const int*>(ws + lay.off_win) + (size_t)f * kWinStride;
    int ki = reinterpret_cast<const int*>(ws + lay.off_item_off)[f];
    int kc = reinterpret_cast<const int*>(ws + lay.off_chunk_off)[f];
    int2* sitems = reinterpret_cast<int2*>(ws + lay.off_scan_items);
    int4* citems = reinterpret_cast<int4*>(ws + lay.off_chunk_items);
    const int nw = W[0];
    for (int w = 0; w < nw; ++w) {
        const int l0 = W[1 + 2 * w], l1 = W[2 + 2 * w];
        const int n = (l1 - l0 + kScanAnglesPerWave - 1) / kScanAnglesPerWave;
        for (int k = lane; k < n; k += 64) {
            const int a0 = l0 + k * kScanAnglesPerWave;
            const int cnt = min(kScanAnglesPerWave, l1 - a0);
            sitems[ki + k] = make_int2(f, a0 | (cnt << 24));
        }
        const int nc = (l1 - l0 + kRefineChunk - 1) / kRefineChunk;
        for (int k = lane; k < nc; k += 64) citems[kc + k] = make_int4(f, l0 + k * kRefineChunk, l0, l1);
        ki += n;
        kc += nc;
    }
}

// largest f with off[f] <= item (off non-decreasing, off[0] = 0 <= item < off[n])
__device__ inline int find_frame(const int* __restrict__ off, int n, int item) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int M>
__device__ inline void steering_load_w(const float* __restrict__ T, int l, int h, float* st) {
    const float4* src = reinterpret_cast<const float4*>(T + (size_t)(2 * l + h) * M);
#pragma unroll
    for (int v = 0; v < M / 4; ++v) {
        const float4 x = src[v];
        st[4 * v] = x.x; st[4 * v + 1] = x.y; st[4 * v + 2] = x.z; st[4 * v + 3] = x.w;
    }
}

// FP32-accuracy products of the split parts kept (see scan_split16_kernel): P = 2 or 3.
template <int P>
__device__ __forceinline__ void win_split_mfma(const halfx8* bp, const halfx8* s0, const halfx8* s1, floatx16& a0,
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

// PARTS: 0 = FP32 operands, 2 or 3 = FP16 split operands of that many parts
template <int M, int PARTS>
__global__ __launch_bounds__(256) void scan_win_kernel(const FrameDev* __restrict__ frames, int n_frames,
                                                       const GroupDev* __restrict__ groups,
                                                       const int32_t* __restrict__ blkframe,
                                                       const float* __restrict__ steer, char* __restrict__ ws,
                                                       LearnedLayout lay, float* __restrict__ spec, int use_user,
                                                       float lowq_tau) {
    constexpr int S = M / 8;                     // 16-deep steps of the FP16 split
    const int lane = threadIdx.x & 63, h = lane >> 5, j = lane & 31;
    const int* ioff = reinterpret_cast<const int*>(ws + lay.off_item_off);
    const int total = ioff[n_frames];
    const int nwaves = gridDim.x * (blockDim.x >> 6);
    const int2* sitems = reinterpret_cast<const int2*>(ws + lay.off_scan_items);
    for (int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); item < total; item += nwaves) {
        const int2 it = sitems[item];
        const int f = it.x;
        const int a0 = it.y & 0xFFFFFF, a1 = a0 + (it.y >> 24);
        const FrameDev& fr = frames[f];
        const GroupDev& g = groups[fr.group];
        const double* qr = reinterpret_cast<const double*>(ws + fr.ws_qref);
        const int t0 = fr.emb_row0 >> 5, t1 = ((fr.emb_row0 + 2 * fr.K - 1) >> 5) + 1;
        float q0 = 0.0f, q1 = 0.0f;
        auto fold = [&](const floatx16& acc0, const floatx16& acc1, int t) {
            const int4 fb = reinterpret_cast<const int4*>(blkframe + g.blk_off)[t];
            const int fbk[4] = {fb.x, fb.y, fb.z, fb.w};
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                if (fbk[gq] != f) continue;
                q0 += acc0[4 * gq] * acc0[4 * gq] + acc0[4 * gq + 1] * acc0[4 * gq + 1] +
                      acc0[4 * gq + 2] * acc0[4 * gq + 2] + acc0[4 * gq + 3] * acc0[4 * gq + 3];
                q1 += acc1[4 * gq] * acc1[4 * gq] + acc1[4 * gq + 1] * acc1[4 * gq + 1] +
                      acc1[4 * gq + 2] * acc1[4 * gq + 2] + acc1[4 * gq + 3] * acc1[4 * gq + 3];
            }
        };
        if constexpr (PARTS > 0) {
            constexpr int P = PARTS;
            halfx8 st0[S][P], st1[S][P];
            const _Float16* T = reinterpret_cast<const _Float16*>(steer + g.steer_x16_off);
            const halfx8* p0 = reinterpret_cast<const halfx8*>(T + ((size_t)2 * P * (a0 + j) + h) * M);
            const halfx8* p1 = reinterpret_cast<const halfx8*>(T + ((size_t)2 * P * (a0 + 32 + j) + h) * M);
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2)
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    st0[s2][q] = p0[2 * S * q + s2];
                    st1[s2][q] = p1[2 * S * q + s2];
                }
            const halfx8* emb = reinterpret_cast<const halfx8*>(ws + g.ws_emb) + lane;   // [tile][part][S][64]
            for (int t = t0; t < t1; ++t) {
                halfx8 bp[S][P];
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2)
#pragma unroll
                    for (int q = 0; q < P; ++q) bp[s2][q] = emb[((size_t)t * P * S + q * S + s2) * 64];
                floatx16 acc0 = {0.0f}, acc1 = {0.0f};
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) win_split_mfma<P>(bp[s2], st0[s2], st1[s2], acc0, acc1);
                fold(acc0, acc1, t);
            }
        } else {
            float st0[M], st1[M];
            const float* T = steer + g.steer_off;
            steering_load_w<M>(T, a0 + j, h, st0);
            steering_load_w<M>(T, a0 + 32 + j, h, st1);
            const float4* emb = reinterpret_cast<const float4*>(ws + g.ws_emb) + lane;   // [tile][M/4][64]
            for (int t = t0; t < t1; ++t) {
                float b[M];
                const float4* src = emb + (size_t)t * (16 * M);
#pragma unroll
                for (int v = 0; v < M / 4; ++v) {
                    const float4 x = src[v * 64];
                    b[4 * v] = x.x; b[4 * v + 1] = x.y; b[4 * v + 2] = x.z; b[4 * v + 3] = x.w;
                }
                floatx16 acc0 = {0.0f}, acc1 = {0.0f};
#pragma unroll
                for (int s2 = 0; s2 < M; ++s2) {
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(b[s2], st0[s2], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(b[s2], st1[s2], acc1, 0, 0, 0);
                }
                fold(acc0, acc1, t);
            }
        }
        const float u0 = q0 + __shfl_xor(q0, 32), u1 = q1 + __shfl_xor(q1, 32);
        const float v = ((lane < 32) ? u0 : u1) * (PARTS > 0 ? (float)qr[1] : 1.0f);
        const int l = a0 + lane;
        const bool in = l < a1;
        if (in) {
            float* out = spec + (use_user ? fr.spec_off_user : fr.spec_off_ws);
            out[l] = 1.0f / fmaxf(v, FLT_MIN);
        }
        const float thr = lowq_tau * (float)qr[0];
        lowq_append(in && v < thr, l, reinterpret_cast<int*>(ws + fr.ws_lowq), fr.lowq_cap);
    }
}

template <int MB>
__global__ __launch_bounds__(256) void lowq_win_kernel(const FrameDev* __restrict__ frames, int n_frames,
                                                       const double* __restrict__ pos,
                                                       const double2* __restrict__ cis, char* __restrict__ ws,
                                                       LearnedLayout lay, float* __restrict__ spec, int use_user) {
    const int lane = threadIdx.x & 63;
    const int* qoff = reinterpret_cast<const int*>(ws + lay.off_lowq_off);
    const int total = qoff[n_frames];
    const int nwaves = gridDim.x * (blockDim.x >> 6);
    for (int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); item < total; item += nwaves) {
        const int f = find_frame(qoff, n_frames, item);
        const FrameDev& fr = frames[f];
        const int* list = reinterpret_cast<const int*>(ws + fr.ws_lowq);
        const int n = min(list[0], fr.lowq_cap);
        const int i = (item - qoff[f]) * 64 + lane;
        if (i >= n) continue;
        const int l = list[1 + i];
        const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
        const double Q = q64_eval<MB>(pos + fr.pos_off, fr.M, fr.K, B,
                                      grid_dir(fr, l), cis);
        float* P = spec + (use_user ? fr.spec_off_user : fr.spec_off_ws);
        P[l] = (float)(1.0 / fmax(Q, (double)FLT_MIN));
    }
}

template <int MB>
__global__ __launch_bounds__(256) void winpeaks_kernel(const FrameDev* __restrict__ frames, int n_frames,
                                                       const double* __restrict__ pos,
                                                       const double2* __restrict__ cis, char* __restrict__ ws,
                                                       LearnedLayout lay, int extra, double lowq_tau,
                                                       double plateau_rel, float* __restrict__ spec,
                                                       int use_user) {
    __shared__ double v[kRefineChunk + 2 * kHaloW];
    __shared__ int rlist[kRefineChunk + 2 * kHaloW];
    __shared__ double lval[kRefineChunk / 2];
    __shared__ int lidx[kRefineChunk / 2];
    __shared__ double bmax[(kRefineChunk + 2 * kHaloW) / kPlateauBlock + 1];
    __shared__ double bmin[(kRefineChunk + 2 * kHaloW) / kPlateauBlock + 1];
    __shared__ int lcount, rcount;
    const int tid = threadIdx.x;
    const int* coff = reinterpret_cast<const int*>(ws + lay.off_chunk_off);
    const int total = coff[n_frames];
    const int4* citems = reinterpret_cast<const int4*>(ws + lay.off_chunk_items);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int4 ci = citems[item];
        const int f = ci.x, c0 = ci.y, wl0 = ci.z, wl1 = ci.w;
        const FrameDev& fr = frames[f];
        const int C = fr.D + extra;
        CandSlot* slots = reinterpret_cast<CandSlot*>(ws + fr.ws_cand) + (size_t)(item - coff[f]) * C;
        const int nown = min(kRefineChunk, wl1 - c0), span = nown + 2 * kHaloW;
        float* P = spec + (use_user ? fr.spec_off_user : fr.spec_off_ws);
        __syncthreads();                  // the previous chunk's LDS is no longer read
        if (tid == 0) {
            lcount = 0;
            rcount = 0;
        }
        for (int e = tid; e < span; e += blockDim.x) {
            const int l = c0 - kHaloW + e;
            v[e] = (l >= wl0 && l < wl1) ? (double)P[l] : qnan_d();
        }
        __syncthreads();
        // a frame whose low-Q list overflowed re-evaluates its low-Q points here
        if (*reinterpret_cast<const int*>(ws + fr.ws_lowq) > fr.lowq_cap) {
            const double pthr = 1.0 / (lowq_tau * *reinterpret_cast<const double*>(ws + fr.ws_qref));
            for (int e = tid; e < span; e += blockDim.x) {
                const double x = v[e];
                if (x == x && !(x < pthr)) rlist[atomicAdd(&rcount, 1)] = e;
            }
            __syncthreads();
            const int nr = rcount;
            const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
            for (int i = tid; i < nr; i += blockDim.x) {
                const int e = rlist[i];
                const int l = c0 - kHaloW + e;
                const double Q = q64_eval<MB>(pos + fr.pos_off, fr.M, fr.K, B,
                                              grid_dir(fr, l), cis);
                const double x = 1.0 / fmax(Q, (double)FLT_MIN);
                v[e] = x;
                if (e >= kHaloW && e < kHaloW + nown) P[l] = (float)x;
            }
            __syncthreads();
        }
        for (int o = tid; o < nown; o += blockDim.x) {
            const int e = o + kHaloW;
            const double x = v[e];
            if (!(x > v[e - 1])) continue;
            int r = e + 1;
            while (r < span && v[r] == x) ++r;
            bool peak = false;
            if (r < span) {
                peak = v[r] < x;
            } else {
                // the run of equal values is longer than the halo: follow it inside the window
                for (int rl = c0 - kHaloW + r; rl < wl1; ++rl) {
                    const double y = (double)P[rl];
                    if (y != x) {
                        peak = y < x;
                        break;
                    }
                }
            }
            if (peak) {
                const int s = atomicAdd(&lcount, 1);
                if (s < kRefineChunk / 2) {
                    lval[s] = x;
                    lidx[s] = c0 + o;
                }
            }
        }
        __syncthreads();
        const int n = min(lcount, kRefineChunk / 2);
        auto val = [&](int g) -> double {
            if (g < wl0 || g >= wl1) return qnan_d();
            const int e = g - (c0 - kHaloW);
            return (e >= 0 && e < span) ? v[e] : (double)P[g];
        };
        uint32_t* flag = reinterpret_cast<uint32_t*>(rlist);
        prefilter_losers(n, lval, [&](int i) { return lidx[i] - (c0 - kHaloW); }, v, span, plateau_rel, bmax, bmin,
                         flag);
        chunk_candidates(n, lval, lidx, flag, &rcount, plateau_rel, val, slots, C);
    }
}

}  // namespace

hipError_t launch_proposals(const FrameDev* frames, int n_frames, const float* scores, int n_bins, int topk,
                            double half_window, float threshold, float floor, int local_max, char* ws,
                            const LearnedLayout& lay, uint32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(proposal_kernel, dim3(n_frames), dim3(64), 0, s, frames, n_frames, scores, n_bins, topk,
                       half_window, threshold, floor, local_max, ws, lay, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_expand(frames, n_frames, ws, lay, s);
}

hipError_t launch_expand(const FrameDev* frames, int n_frames, char* ws, const LearnedLayout& lay, hipStream_t s) {
    hipLaunchKernelGGL(prefix_kernel, dim3(1), dim3(1024), 0, s, n_frames,
                       reinterpret_cast<const int*>(ws + lay.off_items), reinterpret_cast<int*>(ws + lay.off_item_off),
                       reinterpret_cast<const int*>(ws + lay.off_chunks),
                       reinterpret_cast<int*>(ws + lay.off_chunk_off));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(expand_kernel, dim3((n_frames + 3) / 4), dim3(256), 0, s, frames, n_frames, ws, lay);
    return hipGetLastError();
}

hipError_t launch_rescue(const FrameDev* frames, const int32_t* frame_list, int n_list, const int32_t* npeaks,
                         uint32_t* status, char* ws, const LearnedLayout& lay, int32_t* rescue, hipStream_t s) {
    if (n_list <= 0) return hipSuccess;
    hipLaunchKernelGGL(rescue_kernel, dim3((n_list + 255) / 256), dim3(256), 0, s, frames, frame_list, n_list, npeaks,
                       status, ws, lay, rescue);
    return hipGetLastError();
}

hipError_t launch_scan_windows(int parts, int M, const FrameDev* frames, int n_frames, const GroupDev* groups,
                               const int32_t* blkframe, const float* steer, char* ws, const LearnedLayout& lay,
                               float* spec, int use_user, float lowq_tau, int n_wg, hipStream_t s) {
#define NSSDOA_WIN_CASE(MM)                                                                                   \
    case MM:                                                                                               \
        if (parts == 3)                                                                                    \
            hipLaunchKernelGGL((scan_win_kernel<MM, 3>), dim3(n_wg), dim3(256), 0, s, frames, n_frames,     \
                               groups, blkframe, steer, ws, lay, spec, use_user, lowq_tau);                 \
        else if (parts == 2)                                                                               \
            hipLaunchKernelGGL((scan_win_kernel<MM, 2>), dim3(n_wg), dim3(256), 0, s, frames, n_frames,     \
                               groups, blkframe, steer, ws, lay, spec, use_user, lowq_tau);                 \
        else                                                                                               \
            hipLaunchKernelGGL((scan_win_kernel<MM, 0>), dim3(n_wg), dim3(256), 0, s, frames, n_frames,     \
                               groups, blkframe, steer, ws, lay, spec, use_user, lowq_tau);                 \
        return hipGetLastError();
    switch (M) {
        NSSDOA_WIN_CASE(8)
        NSSDOA_WIN_CASE(16)
        NSSDOA_WIN_CASE(32)
        NSSDOA_WIN_CASE(64)
        default: return hipErrorInvalidValue;
    }
#undef NSSDOA_WIN_CASE
}

hipError_t launch_window_peaks(int bucket_M, const FrameDev* frames, int n_frames, const double* pos,
                               const double2* cis, char* ws, const LearnedLayout& lay, int extra, double lowq_tau,
                               double plateau_rel, float* spec, int use_user, int n_wg, hipStream_t s) {
    hipLaunchKernelGGL(lowq_count_kernel, dim3((n_frames + 255) / 256), dim3(256), 0, s, frames, n_frames, ws, lay);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prefix_kernel, dim3(1), dim3(1024), 0, s, n_frames,
                       reinterpret_cast<const int*>(ws + lay.off_lowq), reinterpret_cast<int*>(ws + lay.off_lowq_off),
                       nullptr, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
#define NSSDOA_WP_CASE(MB)                                                                                  \
    case MB:                                                                                             \
        hipLaunchKernelGGL(lowq_win_kernel<MB>, dim3(n_wg), dim3(256), 0, s, frames, n_frames, pos, cis, ws, \
                           lay, spec, use_user);                                                           \
        if ((e = hipGetLastError()) != hipSuccess) return e;                                               \
        hipLaunchKernelGGL(winpeaks_kernel<MB>, dim3(n_wg), dim3(256), 0, s, frames, n_frames, pos, cis, ws, \
                           lay, extra, lowq_tau, plateau_rel, spec, use_user);                             \
        return hipGetLastError();
    switch (bucket_M) {
        NSSDOA_WP_CASE(8)
        NSSDOA_WP_CASE(16)
        NSSDOA_WP_CASE(32)
        NSSDOA_WP_CASE(64)
        default: return hipErrorInvalidValue;
    }
#undef NSSDOA_WP_CASE
}

}  // namespace nssdoa
