// Step-6 (Table 2): peak search and selection, preceded for FP32 spectra by the FP64
// re-evaluation of low-Q points.
//
// One workgroup per frame:
//  1. FP32 spectra: every point with P >= 1 / (tau * ||B||_F^2), i.e. Q below tau times its
//     typical size, is recomputed in FP64 and written back (these are the spectrum peaks, where
//     FP32 rounding is largest relative to Q).
//  2. Local maxima over the spectrum: P[l] > P[l-1] and the run of values equal to P[l] ends
//     in a strictly smaller value; the run is reported at its first index.  Grid ends are not
//     peaks unless the grid is circular.  Candidates go to an LDS list.
//  3. The D + extra best candidates by (value desc, index asc) are kept.
//  4. Each kept candidate's window of +-halfwidth points is evaluated in FP64.
//  5. Local maxima of the FP64 windows are ranked by (FP64 value desc, index asc) and the first
//     D are written.  Slots beyond the number found get idx = -1 and NaN.
#include <float.h>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {

constexpr int kMaxSel = 96;      // D + extra <= 64 + 16 < 96
constexpr int kMaxWin = 33;      // 2 * 16 + 1
constexpr int kMaxFinal = 512;

template <int MB, typename TS>
__global__ __launch_bounds__(256) void peaks_kernel(const int32_t* __restrict__ flist,
                                                    const FrameDev* __restrict__ frames,
                                                    const double* __restrict__ pos,
                                                    const char* __restrict__ ws,
                                                    TS* __restrict__ spec, PeakParams prm,
                                                    nssdoa_peak* __restrict__ peaks,
                                                    int32_t* __restrict__ npeaks,
                                                    uint32_t* __restrict__ status) {
    __shared__ double cval[kCandCap];
    __shared__ int cidx[kCandCap];
    __shared__ int sel[kMaxSel];
    __shared__ double win[kMaxSel * kMaxWin];
    __shared__ double fval[kMaxFinal];
    __shared__ int fidx[kMaxFinal];
    __shared__ int ccount, fcount;

    const int f = flist[blockIdx.x];
    const FrameDev& fr = frames[f];
    const int tid = threadIdx.x;
    const int L = fr.L, D = fr.D, M = fr.M, K = fr.K;
    const bool circ = fr.circular != 0;
    TS* P = spec + (prm.use_user_spec ? fr.spec_off_user : fr.spec_off_ws);
    const double* ps = pos + fr.pos_off;
    const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
    nssdoa_peak* out = peaks + (size_t)f * prm.max_D;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    uint32_t st = status[f];

    if (st & NSSDOA_ST_NONFINITE_INPUT) {
        for (int l = tid; l < L; l += blockDim.x) P[l] = (TS)nan;
        for (int r = tid; r < prm.max_D; r += blockDim.x) {
            out[r].idx = -1;
            out[r].reserved = 0;
            out[r].angle_deg = nan;
            out[r].value = nan;
        }
        if (tid == 0) {
            npeaks[f] = 0;
            status[f] = st | NSSDOA_ST_FEWER_PEAKS;
        }
        return;
    }

    // 1. FP64 re-evaluation of low-Q points of an FP32 spectrum
    if (prm.refine_lowq) {
        const double qref = *reinterpret_cast<const double*>(ws + fr.ws_qref);
        const double pthr = 1.0 / (prm.lowq_tau * qref);
        for (int l = tid; l < L; l += blockDim.x) {
            const double v = (double)P[l];
            if (!(v < pthr)) {
                const double Q = q64_eval<MB>(ps, M, K, B, grid_angle(fr.grid_start, fr.grid_step, l));
                P[l] = (TS)(1.0 / fmax(Q, (double)FLT_MIN));
            }
        }
    }
    if (tid == 0) {
        ccount = 0;
        fcount = 0;
    }
    __syncthreads();

    // 2. local maxima with the plateau rule
    for (int l = tid; l < L; l += blockDim.x) {
        if (!circ && (l == 0 || l == L - 1)) continue;
        const double v = (double)P[l];
        const double vl = (double)P[l == 0 ? L - 1 : l - 1];
        if (!(v > vl)) continue;
        int r = l + 1, steps = 0;
        bool peak = false;
        for (;;) {
            int rr = r;
            if (rr >= L) {
                if (!circ) break;          // the run reaches the last point: not a peak
                rr -= L;
            }
            const double vr = (double)P[rr];
            if (vr != v) {
                peak = vr < v;
                break;
            }
            if (++steps >= L) break;
            ++r;
        }
        if (peak) {
            const int slot = atomicAdd(&ccount, 1);
            if (slot < kCandCap) {
                cval[slot] = v;
                cidx[slot] = l;
            }
        }
    }
    __syncthreads();

    // 3. keep the best C candidates
    const int nc = min(ccount, kCandCap);
    if (ccount > kCandCap) st |= NSSDOA_ST_PEAK_OVERFLOW;
    const int C = min(nc, D + prm.extra);
    for (int i = tid; i < nc; i += blockDim.x) {
        const double vi = cval[i];
        const int li = cidx[i];
        int rank = 0;
        for (int j = 0; j < nc; ++j) {
            const double vj = cval[j];
            rank += (vj > vi) || (vj == vi && cidx[j] < li);
        }
        if (rank < C) sel[rank] = li;
    }
    __syncthreads();

    // 4. FP64 windows
    const int w = prm.halfwidth, W = 2 * w + 1;
    for (int e = tid; e < C * W; e += blockDim.x) {
        const int c = e / W, o = e - c * W;
        int l = sel[c] + o - w;
        double v = nan;
        if (circ) {
            l = ((l % L) + L) % L;
            v = 1.0 / fmax(q64_eval<MB>(ps, M, K, B, grid_angle(fr.grid_start, fr.grid_step, l)), 1e-300);
        } else if (l >= 0 && l < L) {
            v = 1.0 / fmax(q64_eval<MB>(ps, M, K, B, grid_angle(fr.grid_start, fr.grid_step, l)), 1e-300);
        }
        win[c * kMaxWin + o] = v;
    }
    __syncthreads();

    // 5. FP64 local maxima inside the windows (interior points with both neighbours known)
    for (int e = tid; e < C * W; e += blockDim.x) {
        const int c = e / W, o = e - c * W;
        if (o == 0 || o == W - 1) continue;
        int l = sel[c] + o - w;
        if (circ) l = ((l % L) + L) % L;
        else if (l <= 0 || l >= L - 1) continue;
        const double* wv = win + c * kMaxWin;
        const double v = wv[o];
        if (!(v > wv[o - 1])) continue;
        int r = o + 1;
        while (r < W && wv[r] == v) ++r;
        if (r < W && wv[r] < v) {
            const int slot = atomicAdd(&fcount, 1);
            if (slot < kMaxFinal) {
                fval[slot] = v;
                fidx[slot] = l;
            }
        }
    }
    __syncthreads();

    // 6. rank the distinct FP64 peaks and write the first D
    const int nf = min(fcount, kMaxFinal);
    __shared__ int nuniq;
    __shared__ int rankpos[kMaxSel];
    if (tid == 0) nuniq = 0;
    __syncthreads();
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
            const double vj = fval[j];
            rank += (vj > vi) || (vj == vi && lj < li);
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
            out[r].angle_deg = nan;
            out[r].value = nan;
        }
    }
    if (tid == 0) {
        npeaks[f] = nout;
        if (nout < D) st |= NSSDOA_ST_FEWER_PEAKS;
        status[f] = st;
    }
}

template <typename TS>
hipError_t launch_t(int max_M, const int32_t* flist, int n, const FrameDev* frames, const double* pos,
                    const char* ws, TS* spec, const PeakParams& p, nssdoa_peak* peaks,
                    int32_t* npeaks, uint32_t* status, hipStream_t s) {
    if (max_M <= 8)
        hipLaunchKernelGGL((peaks_kernel<8, TS>), dim3(n), dim3(256), 0, s, flist, frames, pos, ws, spec, p, peaks, npeaks, status);
    else if (max_M <= 16)
        hipLaunchKernelGGL((peaks_kernel<16, TS>), dim3(n), dim3(256), 0, s, flist, frames, pos, ws, spec, p, peaks, npeaks, status);
    else if (max_M <= 32)
        hipLaunchKernelGGL((peaks_kernel<32, TS>), dim3(n), dim3(256), 0, s, flist, frames, pos, ws, spec, p, peaks, npeaks, status);
    else
        hipLaunchKernelGGL((peaks_kernel<64, TS>), dim3(n), dim3(256), 0, s, flist, frames, pos, ws, spec, p, peaks, npeaks, status);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_peaks(bool f64, int max_M, const int32_t* frame_list, int n_frames,
                        const FrameDev* frames, const double* pos, const char* ws, void* spec,
                        const PeakParams& p, void* peaks, int32_t* npeaks, uint32_t* status,
                        hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    nssdoa_peak* pk = static_cast<nssdoa_peak*>(peaks);
    if (f64)
        return launch_t<double>(max_M, frame_list, n_frames, frames, pos, ws, static_cast<double*>(spec), p, pk, npeaks, status, s);
    return launch_t<float>(max_M, frame_list, n_frames, frames, pos, ws, static_cast<float*>(spec), p, pk, npeaks, status, s);
}

}  // namespace nssdoa
