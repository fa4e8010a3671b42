// Step-6 (Table 2): peak search and selection, preceded for FP32 spectra by the FP64
// re-evaluation of low-Q points.
//
// lowq_kernel: the scan appends, per frame, every grid point whose FP32 ||B^H a||^2 is below
//  tau ||B||_F^2 (the spectrum peaks, where FP32 rounding is largest relative to Q); one thread
//  per listed point recomputes it in FP64 and writes the rounded value back.  Work items are
//  256-entry slices of the lists, so the FP64 work is spread over the whole GPU whatever the
//  per-frame counts are.
// localmax_kernel, one workgroup per (frame, chunk of 4096 grid points):
//  1. loads the chunk plus a halo of 16 points on each side into LDS (a frame whose list
//     overflowed re-evaluates its low-Q points here instead);
//  2. finds the local maxima of its own points: P[l] > P[l-1] and the run of values equal to
//     P[l] ends in a strictly smaller value (the run is reported at its first index); grid ends
//     are not peaks unless the grid is circular;
//  3. writes its best D + extra maxima by (value desc, index asc) to the chunk's reserved slots,
//     unused slots get index -1.  Slots are per chunk, so no atomics cross workgroups and the
//     result does not depend on scheduling.
// select_kernel, one workgroup per frame:
//  4. ranks the chunk candidates and keeps the best D + extra;
//  5. evaluates a window of +-halfwidth points around each in FP64 (16 lanes per point),
//     sliding a window that holds no interior FP64 local maximum uphill; in windowed
//     estimation points outside the scan windows are left unknown (NaN);
//  6. ranks the distinct FP64 local maxima of the windows by (value desc, index asc) and writes
//     the first D; slots beyond the number found get idx = -1 and NaN.
#include <float.h>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {

constexpr int kHalo = 16;
constexpr int kLocalCap = kRefineChunk / 2;
constexpr int kMaxSel = 96;      // D + extra <= 63 + 16 < 96
constexpr int kMaxWin = 33;      // 2 * 16 + 1
constexpr int kMaxFinal = 1024;
constexpr int kMaxClimb = 32;    // slides of an FP64 window toward a flat peak's maximum

struct Cand {
    double v;
    int32_t idx;
    int32_t pad;
};

__device__ inline double qnan() { return __longlong_as_double(0x7ff8000000000000LL); }

// l lies in one of the windows W = {count, [l0, l1) pairs}
__device__ inline bool in_windows(const int32_t* W, int l) {
    bool in = false;
    for (int i = 0; i < W[0]; ++i) in |= (l >= W[1 + 2 * i]) && (l < W[2 + 2 * i]);
    return in;
}

template <int MB>
__global__ __launch_bounds__(256) void lowq_kernel(const PointItem* __restrict__ items,
                                                   const FrameDev* __restrict__ frames,
                                                   const double* __restrict__ pos,
                                                   const double2* __restrict__ cis,
                                                   const char* __restrict__ ws, float* __restrict__ spec,
                                                   int use_user, const uint32_t* __restrict__ status) {
    const PointItem it = items[blockIdx.x];
    const FrameDev& fr = frames[it.frame];
    const int* list = reinterpret_cast<const int*>(ws + fr.ws_lowq);
    const int n = min(list[0], fr.lowq_cap);
    const int i = it.l0 + (int)threadIdx.x;
    if (i >= n || (status[it.frame] & NSSDOA_ST_NONFINITE_INPUT)) return;
    const int l = list[1 + i];
    const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
    const double Q = q64_eval<MB>(pos + fr.pos_off, fr.M, fr.K, B, grid_angle(fr.grid_start, fr.grid_step, l), cis);
    float* P = spec + (use_user ? fr.spec_off_user : fr.spec_off_ws);
    P[l] = (float)(1.0 / fmax(Q, (double)FLT_MIN));
}

template <int MB, typename TS>
__global__ __launch_bounds__(256) void localmax_kernel(const PointItem* __restrict__ items,
                                                     const FrameDev* __restrict__ frames,
                                                     const double* __restrict__ pos,
                                                     const double2* __restrict__ cis,
                                                     char* __restrict__ ws, TS* __restrict__ spec,
                                                     PeakParams prm,
                                                     const uint32_t* __restrict__ status) {
    __shared__ double v[kRefineChunk + 2 * kHalo];
    __shared__ int rlist[kRefineChunk + 2 * kHalo];
    __shared__ double lval[kLocalCap];
    __shared__ int lidx[kLocalCap];
    __shared__ int lcount, rcount;

    const PointItem it = items[blockIdx.x];
    const int f = it.frame;
    const FrameDev& fr = frames[f];
    const int tid = threadIdx.x;
    const int L = fr.L, l0 = it.l0;
    const int nown = min(kRefineChunk, L - l0);
    const int span = nown + 2 * kHalo;
    const bool circ = fr.circular != 0;
    const int C = fr.D + prm.extra;
    TS* P = spec + (prm.use_user_spec ? fr.spec_off_user : fr.spec_off_ws);
    Cand* slots = reinterpret_cast<Cand*>(ws + fr.ws_cand) + (size_t)(l0 / kRefineChunk) * C;

    if (status[f] & NSSDOA_ST_NONFINITE_INPUT) {
        for (int o = tid; o < nown; o += blockDim.x) P[l0 + o] = (TS)qnan();
        for (int s = tid; s < C; s += blockDim.x) {
            slots[s].v = qnan();
            slots[s].idx = -1;
        }
        return;
    }

    // FP32 spectra were re-evaluated by lowq_kernel unless the frame's list overflowed
    const bool overflow = prm.refine_lowq && *reinterpret_cast<const int*>(ws + fr.ws_lowq) > fr.lowq_cap;
    double pthr = INFINITY;
    if (overflow) pthr = 1.0 / (prm.lowq_tau * *reinterpret_cast<const double*>(ws + fr.ws_qref));
    const double* ps = pos + fr.pos_off;
    const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
    if (tid == 0) {
        lcount = 0;
        rcount = 0;
    }
    // load the chunk and its halo; points beyond a non-circular grid end hold NaN, which
    // compares false both ways
    {
        // every load of this thread is issued before the first LDS store
        constexpr int kPer = (kRefineChunk + 2 * kHalo + 255) / 256;
        double xs[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * 256;
            const int l = l0 - kHalo + e;
            double x = qnan();
            if (e < span) {
                if (l >= 0 && l < L) x = (double)P[l];
                else if (circ) x = (double)P[((l % L) + L) % L];
            }
            xs[u] = x;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * 256;
            if (e < span) v[e] = xs[u];
        }
    }
    __syncthreads();
    if (overflow) {
        // list the low-Q points, then re-evaluate them in FP64 one per thread
        for (int e = tid; e < span; e += blockDim.x) {
            const double x = v[e];
            if (x == x && !(x < pthr)) rlist[atomicAdd(&rcount, 1)] = e;
        }
        __syncthreads();
        const int nr = rcount;
        for (int i = tid; i < nr; i += blockDim.x) {
            const int e = rlist[i];
            int l = l0 - kHalo + e;
            if (l < 0 || l >= L) l = ((l % L) + L) % L;
            const double Q = q64_eval<MB>(ps, fr.M, fr.K, B, grid_angle(fr.grid_start, fr.grid_step, l), cis);
            const double x = 1.0 / fmax(Q, (double)FLT_MIN);
            v[e] = x;
            if (e >= kHalo && e < kHalo + nown) P[l] = (TS)x;
        }
        __syncthreads();
    }

    for (int o = tid; o < nown; o += blockDim.x) {
        const int l = l0 + o;
        if (!circ && (l == 0 || l == L - 1)) continue;
        const int e = o + kHalo;
        const double x = v[e];
        if (!(x > v[e - 1])) continue;
        int r = e + 1;
        while (r < span && v[r] == x) ++r;
        bool peak = false;
        if (r < span) {
            peak = v[r] < x;
        } else {
            // the run of equal values is longer than the halo: follow it in the stored spectrum
            int rl = l0 - kHalo + r, steps = 0;
            for (;;) {
                if (rl >= L) {
                    if (!circ) break;
                    rl -= L;
                }
                const double y = (double)P[rl];
                if (y != x) {
                    peak = y < x;
                    break;
                }
                if (++steps >= L) break;
                ++rl;
            }
        }
        if (peak) {
            const int slot = atomicAdd(&lcount, 1);
            if (slot < kLocalCap) {
                lval[slot] = x;
                lidx[slot] = l;
            }
        }
    }
    __syncthreads();
    const int n = min(lcount, kLocalCap);
    for (int i = tid; i < n; i += blockDim.x) {
        const double vi = lval[i];
        const int li = lidx[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += (lval[j] > vi) || (lval[j] == vi && lidx[j] < li);
        if (rank < C) {
            slots[rank].v = vi;
            slots[rank].idx = li;
        }
    }
    for (int s = n + tid; s < C; s += blockDim.x) {
        slots[s].v = qnan();
        slots[s].idx = -1;
    }
}

template <int MB>
__global__ __launch_bounds__(256) void select_kernel(const int32_t* __restrict__ flist,
                                                     const FrameDev* __restrict__ frames,
                                                     const double* __restrict__ pos,
                                                     const double2* __restrict__ cis,
                                                     const char* __restrict__ ws, PeakParams prm,
                                                     nssdoa_peak* __restrict__ peaks,
                                                     int32_t* __restrict__ npeaks,
                                                     uint32_t* __restrict__ status) {
    __shared__ double cval[kSelCap];
    __shared__ int cidx[kSelCap];
    __shared__ int sel[kMaxSel];
    __shared__ double win[kMaxSel * kMaxWin];
    __shared__ double fval[kMaxFinal];
    __shared__ int fidx[kMaxFinal];
    __shared__ int rankpos[kMaxSel];
    __shared__ int act[kMaxSel], climb[kMaxSel];
    __shared__ int ccount, fcount, nuniq, nact;
    __shared__ double2 asteer[4 * 4 * MB];      // q64_group scratch: 4 waves x 4 groups x MB

    const int f = flist[blockIdx.x];
    const FrameDev& fr = frames[f];
    const int tid = threadIdx.x;
    const int L = fr.L, D = fr.D;
    const bool circ = fr.circular != 0;
    nssdoa_peak* out = peaks + (size_t)f * prm.max_D;
    uint32_t st = status[f];

    if (st & NSSDOA_ST_NONFINITE_INPUT) {
        for (int r = tid; r < prm.max_D; r += blockDim.x) {
            out[r].idx = -1;
            out[r].reserved = 0;
            out[r].angle_deg = qnan();
            out[r].value = qnan();
        }
        if (tid == 0) {
            npeaks[f] = 0;
            status[f] = st | NSSDOA_ST_FEWER_PEAKS;
        }
        return;
    }

    // 4. gather the chunk candidates and keep the best C
    const int Cc = D + prm.extra;
    const int n_chunks = prm.chunk_count ? prm.chunk_count[f] : (L + kRefineChunk - 1) / kRefineChunk;
    const int total = n_chunks * Cc;
    const Cand* slots = reinterpret_cast<const Cand*>(ws + fr.ws_cand);
    if (tid == 0) {
        ccount = 0;
        fcount = 0;
        nuniq = 0;
    }
    __syncthreads();
    for (int i = tid; i < total; i += blockDim.x) {
        const Cand c = slots[i];
        if (c.idx >= 0) {
            const int s = atomicAdd(&ccount, 1);
            cval[s] = c.v;
            cidx[s] = c.idx;
        }
    }
    __syncthreads();
    const int nc = ccount;
    const int C = min(nc, Cc);
    for (int i = tid; i < nc; i += blockDim.x) {
        const double vi = cval[i];
        const int li = cidx[i];
        int rank = 0;
        for (int j = 0; j < nc; ++j) rank += (cval[j] > vi) || (cval[j] == vi && cidx[j] < li);
        if (rank < C) sel[rank] = li;
    }
    __syncthreads();

    // 5. FP64 windows around the kept candidates.  A window without an interior FP64 local
    //    maximum (the FP32 maximum of a very flat peak can lie farther from the FP64 one than the
    //    half width) slides toward its higher end by W - 2 points, keeping two points of overlap,
    //    until it holds one or kMaxClimb slides are done.
    const double* ps = pos + fr.pos_off;
    const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
    const int w = prm.halfwidth, W = 2 * w + 1;
    for (int i = tid; i < C; i += blockDim.x) act[i] = i;
    if (tid == 0) nact = C;
    __syncthreads();
    for (int iter = 0;; ++iter) {
        const int na = nact;
        {
            // 16 lanes per window point: 16 points per pass of the 256-thread workgroup
            const int grp = tid >> 4, j = tid & 15;
            double2* a = asteer + (tid >> 6) * 4 * MB;
            for (int e0 = 0; e0 < na * W; e0 += 16) {
                const int e = e0 + grp;
                const bool valid = e < na * W;
                const int c = valid ? act[e / W] : 0, o = valid ? e - (e / W) * W : 0;
                int l = valid ? sel[c] + o - w : 0;
                if (circ) l = ((l % L) + L) % L;
                bool inside = valid && (circ || (l >= 0 && l < L));
                if (inside && prm.windows) inside = in_windows(prm.windows + (size_t)f * kWinStride, l);
                const double Q = q64_group<MB>(ps, fr.M, fr.K, B,
                                               grid_angle(fr.grid_start, fr.grid_step, inside ? l : 0), cis, a);
                if (valid && j == 0) win[c * kMaxWin + o] = inside ? 1.0 / fmax(Q, 1e-300) : qnan();
            }
        }
        __syncthreads();
        if (iter == kMaxClimb) break;
        // one thread per active window: interior local maximum present? otherwise slide uphill
        for (int i = tid; i < na; i += blockDim.x) {
            const int c = act[i];
            const double* wv = win + c * kMaxWin;
            bool interior = false;
            for (int o = 1; o < W - 1 && !interior; ++o) {
                const double x = wv[o];
                if (!(x > wv[o - 1])) continue;
                int r = o + 1;
                while (r < W && wv[r] == x) ++r;
                interior = r < W && wv[r] < x;
            }
            int move = 0;
            if (!interior) {
                if (wv[W - 1] > wv[0] || (wv[W - 1] == wv[W - 1] && wv[0] != wv[0])) move = W - 2;
                else if (wv[0] > wv[W - 1] || (wv[0] == wv[0] && wv[W - 1] != wv[W - 1])) move = -(W - 2);
            }
            climb[i] = move;
        }
        __syncthreads();
        if (tid == 0) {
            int n2 = 0;
            for (int i = 0; i < na; ++i) {
                if (climb[i] == 0) continue;
                const int c = act[i];
                sel[c] += climb[i];
                act[n2++] = c;
            }
            nact = n2;
        }
        __syncthreads();
        if (nact == 0) break;
    }

    // 6. FP64 local maxima inside the windows (interior points: both neighbours known)
    for (int e = tid; e < C * W; e += blockDim.x) {
        const int c = e / W, o = e - c * W;
        if (o == 0 || o == W - 1) continue;
        int l = sel[c] + o - w;
        if (circ) l = ((l % L) + L) % L;
        else if (l <= 0 || l >= L - 1) continue;
        const double* wv = win + c * kMaxWin;
        const double x = wv[o];
        if (!(x > wv[o - 1])) continue;
        int r = o + 1;
        while (r < W && wv[r] == x) ++r;
        if (r < W && wv[r] < x) {
            const int s = atomicAdd(&fcount, 1);
            if (s < kMaxFinal) {
                fval[s] = x;
                fidx[s] = l;
            }
        }
    }
    __syncthreads();
    const int nf = min(fcount, kMaxFinal);
    for (int i = tid; i < nf; i += blockDim.x) {
        const int li = fidx[i];
        bool dup = false;
        for (int j = 0; j < i; ++j) dup |= (fidx[j] == li);
        if (dup) continue;
        atomicAdd(&nuniq, 1);
        const double vi = fval[i];
        int rank = 0;
        for (int j = 0; j < nf; ++j) {
            const int lj = fidx[j];
            bool djdup = false;
            for (int k = 0; k < j; ++k) djdup |= (fidx[k] == lj);
            if (djdup) continue;
            rank += (fval[j] > vi) || (fval[j] == vi && lj < li);
        }
        if (rank < D) rankpos[rank] = i;
    }
    __syncthreads();
    const int nout = min(nuniq, D);
    for (int r = tid; r < prm.max_D; r += blockDim.x) {
        if (r < nout) {
            const int i = rankpos[r];
            out[r].idx = fidx[i];
            out[r].reserved = 0;
            out[r].angle_deg = grid_angle(fr.grid_start, fr.grid_step, fidx[i]);
            out[r].value = fval[i];
        } else {
            out[r].idx = -1;
            out[r].reserved = 0;
            out[r].angle_deg = qnan();
            out[r].value = qnan();
        }
    }
    if (tid == 0) {
        npeaks[f] = nout;
        if (nout < D) st |= NSSDOA_ST_FEWER_PEAKS;
        status[f] = st;
    }
}

template <int MB>
hipError_t launch_mb(bool f64, const PointItem* lowq_items, int n_lowq, const PointItem* items, int n_items,
                     const int32_t* flist, int n_frames, const FrameDev* frames, const double* pos,
                     const double2* cis, char* ws, void* spec, const PeakParams& p, nssdoa_peak* peaks,
                     int32_t* npeaks, uint32_t* status, hipStream_t s) {
    if (!f64 && p.refine_lowq && n_lowq > 0) {
        hipLaunchKernelGGL((lowq_kernel<MB>), dim3(n_lowq), dim3(256), 0, s, lowq_items, frames, pos, cis, ws,
                           static_cast<float*>(spec), p.use_user_spec, status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_items > 0) {
        if (f64)
            hipLaunchKernelGGL((localmax_kernel<MB, double>), dim3(n_items), dim3(256), 0, s, items, frames, pos,
                               cis, ws, static_cast<double*>(spec), p, status);
        else
            hipLaunchKernelGGL((localmax_kernel<MB, float>), dim3(n_items), dim3(256), 0, s, items, frames, pos,
                               cis, ws, static_cast<float*>(spec), p, status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_frames > 0)
        hipLaunchKernelGGL((select_kernel<MB>), dim3(n_frames), dim3(256), 0, s, flist, frames, pos, cis, ws, p,
                           peaks, npeaks, status);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_peaks(bool f64, int bucket_M, const PointItem* lowq_items, int n_lowq_items,
                        const PointItem* items, int n_items, const int32_t* frame_list,
                        int n_frames, const FrameDev* frames, const double* pos,
                        const double2* cis, char* ws, void* spec, const PeakParams& p,
                        void* peaks, int32_t* npeaks, uint32_t* status, hipStream_t s) {
    nssdoa_peak* pk = static_cast<nssdoa_peak*>(peaks);
#define NSSDOA_PEAKS_CASE(MB)                                                                       \
    case MB:                                                                                     \
        return launch_mb<MB>(f64, lowq_items, n_lowq_items, items, n_items, frame_list, n_frames,   \
                             frames, pos, cis, ws, spec, p, pk, npeaks, status, s);
    switch (bucket_M) {
        NSSDOA_PEAKS_CASE(8)
        NSSDOA_PEAKS_CASE(16)
        NSSDOA_PEAKS_CASE(32)
        NSSDOA_PEAKS_CASE(64)
        default: return hipErrorInvalidValue;
    }
#undef NSSDOA_PEAKS_CASE
}

}  // namespace nssdoa
