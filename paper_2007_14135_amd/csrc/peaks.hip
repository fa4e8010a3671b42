// Step-6 (Table 2): peak search and selection, preceded for FP32 spectra by the FP64
// re-evaluation of low-Q points.
//
// lowq_refine_kernel: the matrix-core scans publish every grid point whose FP32 ||B^H a||^2 is
//  below tau ||B||_F^2 (the spectrum peaks, where FP32 rounding is largest relative to Q) to one
//  list per batch; one thread per listed point recomputes it in FP64 and writes the rounded value
//  back, so the FP64 work is spread over the whole GPU whatever the per-frame counts are.
// localmax_kernel, one workgroup per (frame, chunk of 4096 grid points):
//  1. loads the chunk plus a halo of 16 points on each side into LDS (lowq_refine_kernel has
//     re-evaluated the low-Q points in FP64; for a frame whose scan list overflowed this kernel
//     re-evaluates every point at or above 1 / (lowq_tau ||B||_F^2) itself, writes the chunk's
//     own points back to the spectrum and uses the same rounded values for the halo);
//  2. finds the local maxima of its own points: P[l] > P[l-1] and the run of values equal to
//     P[l] ends in a strictly smaller value (the run is reported at its first index); grid ends
//     are not peaks unless the grid is circular;
//  3. keeps the maxima that win their plateau (chunk_candidates) and writes the best D + extra
//     by (value desc, index asc), with their plateau extents, to the chunk's reserved slots;
//     unused slots get index -1.  Slots are per chunk, so no atomics cross workgroups and the
//     result does not depend on scheduling.
// select_kernel, one workgroup per frame:
//  4. orders the chunk candidates by (value desc, index asc);
//  5. takes them in that order, in batches, and evaluates each one's plateau +- halfwidth points
//     in FP64 (16 lanes per point), listing the FP64 local maxima interior to these spans (in
//     windowed estimation points outside the scan windows are unknown, NaN); it stops once D
//     distinct FP64 maxima are known and the next candidate, raised by the plateau depth, is
//     below the D-th of them;
//  6. ranks the distinct FP64 local maxima by (value desc, index asc) and writes the first D;
//     slots beyond the number found get idx = -1 and NaN.
#include <float.h>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {

constexpr int kHalo = 16;
constexpr int kLocalCap = kRefineChunk / 2;
constexpr int kMaxSel = 96;      // D + extra <= 63 + 16 < 96
constexpr int kMaxFinal = 1024;
constexpr int kSpanCap = 2048;   // FP64 points evaluated per batch of candidates
constexpr int kMaxBatch = 96;    // candidates per batch (D + extra of them, at most)


__device__ inline double qnan() { return __longlong_as_double(0x7ff8000000000000LL); }

// l lies in one of the windows W = {count, [l0, l1) pairs}
__device__ inline bool in_windows(const int32_t* W, int l) {
    bool in = false;
    for (int i = 0; i < W[0]; ++i) in |= (l >= W[1 + 2 * i]) && (l < W[2 + 2 * i]);
    return in;
}

// FP64 re-evaluation of the batch's low-Q list (published by the matrix-core scans), one point
// per thread over a fixed grid: the list's length is known only on the device.
template <int MB>
__global__ __launch_bounds__(256) void lowq_refine_kernel(LowqList lq, const FrameDev* __restrict__ frames,
                                                          const double* __restrict__ pos,
                                                          const double2* __restrict__ cis,
                                                          const char* __restrict__ ws, float* __restrict__ spec,
                                                          int use_user) {
    const int n = min(*lq.count, lq.cap);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int2 e = lq.list[i];
        const FrameDev& fr = frames[e.x];
        const double Q = q64_eval<MB>(pos + fr.pos_off, fr.M, fr.K, reinterpret_cast<const double2*>(ws + fr.ws_B),
                                      grid_dir(fr, e.y), cis);
        float* out = spec + (use_user ? fr.spec_off_user : fr.spec_off_ws);
        out[e.y] = (float)(1.0 / fmax(Q, (double)FLT_MIN));
    }
}

// True when the local-maximum candidate x at v-index e (P[l] > P[l-1], P[l+1] == x) is a peak:
// the run of values equal to x ends in a strictly smaller value.  Runs longer than the halo
// are followed in the stored spectrum.
template <typename TS>
__device__ bool equal_run_ends_lower(const TS* v, int e, int span, double x, const TS* P, int l0, int L, bool circ) {
    int r = e + 1;
    while (r < span && (double)v[r] == x) ++r;
    if (r < span) return (double)v[r] < x;
    int rl = l0 - kHalo + r, steps = 0;
    for (;;) {
        if (rl >= L) {
            if (!circ) return false;
            rl -= L;
        }
        const double y = (double)P[rl];
        if (y != x) return y < x;
        if (++steps >= L) return false;
        ++rl;
    }
}

constexpr int kLmThreads = 512;       // threads of a local-maximum workgroup

template <int MB, typename TS>
__global__ __launch_bounds__(kLmThreads, 4) void localmax_kernel(const PointItem* __restrict__ items,
                                                     const FrameDev* __restrict__ frames,
                                                     const double* __restrict__ pos,
                                                     const double2* __restrict__ cis,
                                                     char* __restrict__ ws, TS* __restrict__ spec,
                                                     PeakParams prm,
                                                     const uint32_t* __restrict__ status) {
    constexpr int kSpanMax = kRefineChunk + 2 * kHalo;
    constexpr int kPerT = kRefineChunk / kLmThreads;   // own points per thread in the maximum test
    static_assert(kSpanMax * sizeof(int) >= kLocalCap * sizeof(double), "union layout");
    __shared__ TS v[kSpanMax];
    // the low-Q point list of an overflowed frame, then (once it is used) the local maxima's values
    __shared__ double rl_union[kSpanMax * sizeof(int) / sizeof(double) + 1];
    __shared__ int lidx[kLocalCap];
    __shared__ uint32_t flag[kLocalCap];
    __shared__ double bmax[kSpanMax / kPlateauBlock + 1];
    __shared__ double bmin[kSpanMax / kPlateauBlock + 1];
    __shared__ int lcount, rcount;
    int* rlist = reinterpret_cast<int*>(rl_union);
    double* lval = rl_union;

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
    CandSlot* slots = reinterpret_cast<CandSlot*>(ws + fr.ws_cand) + (size_t)(l0 / kRefineChunk) * C;

    // Every global load is issued before the first one is used: the frame status, ||B||_F^2 and
    // the chunk with its halo (points beyond a non-circular grid end hold NaN, which compares
    // false both ways).
    const uint32_t fst = status[f];
    const int overflow = prm.refine_lowq ? *reinterpret_cast<const int*>(ws + fr.ws_lowq) : 0;
    const double* qrp = reinterpret_cast<const double*>(ws + fr.ws_qref);
    const double qref = prm.refine_lowq ? qrp[0] : 0.0;
    const double qfloor = prm.refine_lowq && prm.lp_floor ? qrp[1] : 0.0;
    constexpr int kPer = (kSpanMax + kLmThreads - 1) / kLmThreads;
    TS xs[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * kLmThreads;
        const int l = l0 - kHalo + e;
        TS x = (TS)qnan();
        if (e < span) {
            if (l >= 0 && l < L) x = P[l];
            else if (circ) x = P[((l % L) + L) % L];
        }
        xs[u] = x;
    }
    if (fst & NSSDOA_ST_NONFINITE_INPUT) {
        for (int o = tid; o < nown; o += blockDim.x) P[l0 + o] = (TS)qnan();
        for (int s = tid; s < C; s += blockDim.x) {
            slots[s].v = qnan();
            slots[s].idx = -1;
        }
        return;
    }
    if (tid == 0) {
        lcount = 0;
        rcount = 0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * kLmThreads;
        if (e < span) v[e] = xs[u];
    }
    __syncthreads();
    if (overflow) {
        // list the low-Q points (one LDS atomic per wave), then re-evaluate them in FP64, one per
        // thread; the halo gets the same rounded values the neighbouring chunk writes
        const double pthr = 1.0 / fmax(prm.lowq_tau * qref, qfloor);
        const int lane = tid & 63;
        for (int e0 = 0; e0 < span; e0 += blockDim.x) {
            const int e = e0 + tid;
            const double x = e < span ? (double)v[e] : qnan();
            const bool low = x == x && !(x < pthr);
            const unsigned long long mask = __ballot(low);
            if (mask) {
                const int leader = __ffsll((long long)mask) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&rcount, __popcll(mask));
                base = __shfl(base, leader);
                if (low) rlist[base + __popcll(mask & ((1ull << lane) - 1ull))] = e;
            }
        }
        __syncthreads();
        const int nr = rcount;
        const double* ps = pos + fr.pos_off;
        const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
        for (int i = tid; i < nr; i += blockDim.x) {
            const int e = rlist[i];
            int l = l0 - kHalo + e;
            if (l < 0 || l >= L) l = ((l % L) + L) % L;
            const double Q = q64_eval<MB>(ps, fr.M, fr.K, B, grid_dir(fr, l), cis);
            const TS x = (TS)(1.0 / fmax(Q, (double)FLT_MIN));
            v[e] = x;
            if (e >= kHalo && e < kHalo + nown) P[l] = x;
        }
        __syncthreads();
    }

    // 2. local maxima: thread t tests its own points o = 8 t .. 8 t + 7 from registers (one
    // aligned vector read of them plus their two neighbours), first as two bit masks: points
    // above their left neighbour and above / equal to their right one
    {
        const int o0 = tid * kPerT;
        if (o0 < nown) {
            TS w[kPerT + 2];                             // v-indices kHalo + o0 - 1 .. kHalo + o0 + kPerT
            w[0] = v[kHalo + o0 - 1];
#pragma unroll
            for (int k = 0; k < kPerT; ++k) w[k + 1] = v[kHalo + o0 + k];
            w[kPerT + 1] = v[kHalo + o0 + kPerT];
            const int lo_ok = circ ? 0 : 1 - l0;        // first own o that may be a peak
            const int hi_ok = circ ? nown : min(nown, L - 1 - l0);   // one past the last
            uint32_t above = 0, level = 0;
#pragma unroll
            for (int k = 0; k < kPerT; ++k) {
                const int o = o0 + k;
                const bool ok = o >= lo_ok && o < hi_ok && w[k + 1] > w[k];
                above |= (uint32_t)(ok && w[k + 2] < w[k + 1]) << k;
                level |= (uint32_t)(ok && w[k + 2] == w[k + 1]) << k;
            }
            while (level) {                              // a run of equal values: follow it
                const int k = __builtin_ctz(level);
                level &= level - 1;
                if (equal_run_ends_lower(v, kHalo + o0 + k, span, (double)v[kHalo + o0 + k], P, l0, L, circ))
                    above |= 1u << k;
            }
            while (above) {
                const int k = __builtin_ctz(above);
                above &= above - 1;
                const int slot = atomicAdd(&lcount, 1);
                if (slot < kLocalCap) {
                    lval[slot] = (double)v[kHalo + o0 + k];
                    lidx[slot] = l0 + o0 + k;
                }
            }
        }
    }
    __syncthreads();
    // 3. plateau winners, best C to the chunk's slots
    const int n = min(lcount, kLocalCap);
    auto val = [&](int g) -> double {
        const int e = g - (l0 - kHalo);
        if (e >= 0 && e < span) return (double)v[e];
        if (circ) return (double)P[((g % L) + L) % L];
        return (g >= 0 && g < L) ? (double)P[g] : qnan();
    };
    prefilter_losers(n, lval, [&](int i) { return lidx[i] - (l0 - kHalo); }, v, span, prm.plateau_rel, bmax, bmin,
                     flag);
    chunk_candidates(n, lval, lidx, flag, &rcount, prm.plateau_rel, val, slots, C);
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
    // candidate slots in dynamic LDS, sized for the launch's largest frame (prm.sel_cap): values,
    // indices, plateau spans and the value order
    extern __shared__ double sel_dyn[];
    double* cval = sel_dyn;
    int* cidx = reinterpret_cast<int*>(cval + prm.sel_cap);
    uint32_t* cspan = reinterpret_cast<uint32_t*>(cidx + prm.sel_cap);
    int* ord = reinterpret_cast<int*>(cspan + prm.sel_cap);
    __shared__ double buf[kSpanCap];
    __shared__ int sp_lo[kMaxBatch], sp_off[kMaxBatch + 1];
    __shared__ double fval[kMaxFinal];
    __shared__ int fidx[kMaxFinal];
    __shared__ int rankpos[kMaxSel];
    __shared__ int ccount, fcount, nuniq, nproc, nbatch, done;
    __shared__ double dth;
    __shared__ double2 asteer[4 * 4 * MB];      // q64_group scratch: 4 waves x 4 groups x MB

    const int f = flist[blockIdx.x];
    if (f < 0) return;                          // a frame with nothing to select (uniform)
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
            out[r].polar_deg = qnan();
        }
        if (tid == 0) {
            npeaks[f] = 0;
            status[f] = st | NSSDOA_ST_FEWER_PEAKS;
        }
        return;
    }

    // 4. gather the chunk candidates and order them by (value desc, index asc)
    const int Cc = D + prm.extra;
    const int n_chunks = prm.chunk_count ? prm.chunk_count[f] : (L + kRefineChunk - 1) / kRefineChunk;
    const int total = n_chunks * Cc;
    const CandSlot* slots = reinterpret_cast<const CandSlot*>(ws + fr.ws_cand);
    if (tid == 0) {
        ccount = 0;
        fcount = 0;
        nuniq = 0;
        nproc = 0;
        dth = 0.0;
    }
    __syncthreads();
    for (int i = tid; i < total; i += blockDim.x) {
        const CandSlot c = slots[i];
        if (c.idx >= 0) {
            const int s = atomicAdd(&ccount, 1);
            cval[s] = c.v;
            cidx[s] = c.idx;
            cspan[s] = c.span;
        }
    }
    __syncthreads();
    const int nc = ccount;
    for (int i = tid; i < nc; i += blockDim.x) {
        const double vi = cval[i];
        const int li = cidx[i];
        int rank = 0;
        for (int k = 0; k < nc; ++k) rank += (cval[k] > vi) || (cval[k] == vi && cidx[k] < li);
        ord[rank] = i;
    }
    __syncthreads();

    // 5. FP64 evaluation of each candidate's plateau +- halfwidth, in batches taken in candidate
    //    order, until D distinct FP64 maxima are known and the next candidate cannot beat the D-th
    //    (a plateau's FP64 values exceed its candidate's value by less than plateau_rel)
    const double* ps = pos + fr.pos_off;
    const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
    const int w = prm.halfwidth;
    const int grp = tid >> 4, j = tid & 15;
    double2* a = asteer + (tid >> 6) * 4 * MB;
    const int32_t* W = prm.windows ? prm.windows + (size_t)f * kWinStride : nullptr;
    for (;;) {
        if (tid == 0) {
            int stop = nproc >= nc;
            if (!stop && nuniq >= D && cval[ord[nproc]] * (1.0 + prm.plateau_rel) < dth) stop = 1;
            int nb = 0, tot = 0;
            // the first batch holds the best D candidates: for well separated peaks it is all
            // the FP64 work there is
            const int cap = min(nproc == 0 ? D : Cc, kMaxBatch);
            while (!stop && nproc + nb < nc && nb < cap) {
                const int i = ord[nproc + nb];
                const int l = cidx[i];
                int lo = l - (int)(cspan[i] >> 16) - w, hi = l + (int)(cspan[i] & 0xFFFFu) + w;
                if (!circ) {
                    lo = max(lo, 0);
                    hi = min(hi, L - 1);
                }
                if (hi - lo + 1 > kSpanCap) {          // a very long plateau: its central part
                    lo = max(lo, l - kSpanCap / 2);
                    hi = lo + kSpanCap - 1;
                }
                const int len = hi - lo + 1;
                if (tot + len > kSpanCap) break;
                sp_lo[nb] = lo;
                sp_off[nb] = tot;
                tot += len;
                ++nb;
            }
            sp_off[nb] = tot;
            nbatch = nb;
            nproc += nb;
            done = stop || nb == 0;
        }
        __syncthreads();
        if (done) break;
        const int nb = nbatch, tot = sp_off[nb];
        // 16 lanes per point: 16 points per pass of the 256-thread workgroup
        for (int e0 = 0; e0 < tot; e0 += 16) {
            const int e = e0 + grp;
            const bool valid = e < tot;
            int b = 0;
            if (valid)
                while (sp_off[b + 1] <= e) ++b;
            int l = valid ? sp_lo[b] + (e - sp_off[b]) : 0;
            if (circ) l = ((l % L) + L) % L;
            bool inside = valid && (circ || (l >= 0 && l < L));
            if (inside && W) inside = in_windows(W, l);
            const double Q = q64_group<MB>(ps, fr.M, fr.K, B,
                                           grid_dir(fr, inside ? l : 0), cis, a);
            if (valid && j == 0) buf[e] = inside ? 1.0 / fmax(Q, 1e-300) : qnan();
        }
        __syncthreads();
        // FP64 local maxima interior to the spans (both neighbours and the plateau run known)
        for (int e = tid; e < tot; e += blockDim.x) {
            int b = 0;
            while (sp_off[b + 1] <= e) ++b;
            const int beg = sp_off[b], end = sp_off[b + 1];
            if (e == beg || e == end - 1) continue;
            int l = sp_lo[b] + (e - beg);
            if (circ) l = ((l % L) + L) % L;
            else if (l <= 0 || l >= L - 1) continue;
            const double x = buf[e];
            if (!(x > buf[e - 1])) continue;
            int r = e + 1;
            while (r < end && buf[r] == x) ++r;
            if (r < end && buf[r] < x) {
                const int s = atomicAdd(&fcount, 1);
                if (s < kMaxFinal) {
                    fval[s] = x;
                    fidx[s] = l;
                }
            }
        }
        if (tid == 0) nuniq = 0;
        __syncthreads();
        // distinct maxima so far and the D-th best value
        const int nf = min(fcount, kMaxFinal);
        for (int i = tid; i < nf; i += blockDim.x) {
            const int li = fidx[i];
            bool dup = false;
            for (int k = 0; k < i; ++k) dup |= (fidx[k] == li);
            if (dup) continue;
            atomicAdd(&nuniq, 1);
            const double vi = fval[i];
            int rank = 0;
            for (int k = 0; k < nf; ++k) {
                const int lk = fidx[k];
                bool kdup = false;
                for (int q = 0; q < k; ++q) kdup |= (fidx[q] == lk);
                if (kdup) continue;
                rank += (fval[k] > vi) || (fval[k] == vi && lk < li);
            }
            if (rank == D - 1) dth = vi;
        }
        __syncthreads();
    }

    // 6. rank the distinct FP64 maxima by (value desc, index asc) and write the first D
    const int nf = min(fcount, kMaxFinal);
    for (int i = tid; i < nf; i += blockDim.x) {
        const int li = fidx[i];
        bool dup = false;
        for (int k = 0; k < i; ++k) dup |= (fidx[k] == li);
        if (dup) continue;
        const double vi = fval[i];
        int rank = 0;
        for (int k = 0; k < nf; ++k) {
            const int lk = fidx[k];
            bool kdup = false;
            for (int q = 0; q < k; ++q) kdup |= (fidx[q] == lk);
            if (kdup) continue;
            rank += (fval[k] > vi) || (fval[k] == vi && lk < li);
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
            out[r].polar_deg = 90.0;
        } else {
            out[r].idx = -1;
            out[r].reserved = 0;
            out[r].angle_deg = qnan();
            out[r].value = qnan();
            out[r].polar_deg = qnan();
        }
    }
    if (tid == 0) {
        npeaks[f] = nout;
        if (nout < D) st |= NSSDOA_ST_FEWER_PEAKS;
        if (fcount > kMaxFinal) st |= NSSDOA_ST_PEAK_OVERFLOW;
        status[f] = st;
    }
}

template <int MB>
hipError_t launch_mb(bool f64, const PointItem* items, int n_items, const int32_t* flist, int n_frames,
                     const FrameDev* frames, const double* pos, const double2* cis, char* ws, void* spec,
                     const PeakParams& p, nssdoa_peak* peaks, int32_t* npeaks, uint32_t* status, hipStream_t s) {
    if (n_items > 0) {
        if (f64)
            hipLaunchKernelGGL((localmax_kernel<MB, double>), dim3(n_items), dim3(kLmThreads), 0, s, items, frames, pos,
                               cis, ws, static_cast<double*>(spec), p, status);
        else
            hipLaunchKernelGGL((localmax_kernel<MB, float>), dim3(n_items), dim3(kLmThreads), 0, s, items, frames, pos,
                               cis, ws, static_cast<float*>(spec), p, status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_frames > 0) {
        if (p.sel_cap < 1 || p.sel_cap > kSelCap) return hipErrorInvalidValue;
        const size_t lds = (size_t)p.sel_cap * (sizeof(double) + 3 * sizeof(int));
        hipLaunchKernelGGL((select_kernel<MB>), dim3(n_frames), dim3(256), lds, s, flist, frames, pos, cis, ws, p,
                           peaks, npeaks, status);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lowq_refine(int bucket_M, LowqList lq, const FrameDev* frames, const double* pos,
                              const double2* cis, const char* ws, float* spec, int use_user, int n_wg,
                              hipStream_t s) {
    if (!lq.count || lq.cap <= 0 || n_wg <= 0) return hipSuccess;
    switch (bucket_M) {
        case 8: hipLaunchKernelGGL(lowq_refine_kernel<8>, dim3(n_wg), dim3(256), 0, s, lq, frames, pos, cis, ws, spec, use_user); break;
        case 16: hipLaunchKernelGGL(lowq_refine_kernel<16>, dim3(n_wg), dim3(256), 0, s, lq, frames, pos, cis, ws, spec, use_user); break;
        case 32: hipLaunchKernelGGL(lowq_refine_kernel<32>, dim3(n_wg), dim3(256), 0, s, lq, frames, pos, cis, ws, spec, use_user); break;
        case 64: hipLaunchKernelGGL(lowq_refine_kernel<64>, dim3(n_wg), dim3(256), 0, s, lq, frames, pos, cis, ws, spec, use_user); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_peaks(bool f64, int bucket_M, const PointItem* items, int n_items, const int32_t* frame_list,
                        int n_frames, const FrameDev* frames, const double* pos, const double2* cis, char* ws,
                        void* spec, const PeakParams& p, void* peaks, int32_t* npeaks, uint32_t* status,
                        hipStream_t s) {
    nssdoa_peak* pk = static_cast<nssdoa_peak*>(peaks);
#define NSSDOA_PEAKS_CASE(MB)                                                                       \
    case MB:                                                                                     \
        return launch_mb<MB>(f64, items, n_items, frame_list, n_frames, frames, pos, cis, ws, spec, p, pk, \
                             npeaks, status, s);
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
