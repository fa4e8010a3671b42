// Step-6 (Table 2) on 2-D grids (azimuth x polar angle of Eq. 2, the scans of the paper's
// experiments, Section 5): a grid point is a peak when it lies above its 8 neighbours inside the
// grid -- strictly above each neighbour that precedes it in row-major order, at least equal to
// each one that follows, and strictly above at least one -- with the azimuth axis wrapping on a
// circular grid; the D largest peaks (ties to the lower index) are selected.
//
// peak2d_mark_kernel<MB, TS>, one thread per grid point of a 2-D frame (items of 256 points):
//   FP64 spectra (complex128 batches) are tested as they are.  FP32 spectra are rounded: a point
//   whose FP64 value is a peak is at least (1 - kRel) times each neighbour in FP32 (kRel is
//   above twice the scan's relative error after the FP64 re-evaluation of low-Q points), so only
//   such candidates are re-evaluated, with their 8 neighbours, in FP64 and tested exactly (every
//   point is, in a frame whose scan overflowed its low-Q list, or where the FP32 value is NaN).
//   The point's FP64 value is written to the frame's peak map if it is a peak, -1 otherwise.
// peak2d_select_kernel, one workgroup per 2-D frame: gathers the mapped peaks into LDS (at most
//   kCap2d; more sets NSSDOA_ST_PEAK_OVERFLOW), ranks them by (value desc, index asc) and writes
//   the first D with their azimuth and polar angle.
#include <float.h>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {

constexpr double kRel = 2e-4;
constexpr int kCap2d = 1024;

__device__ inline double qnan2() { return __longlong_as_double(0x7ff8000000000000LL); }

// In-grid neighbour k (0..7) of point (j, i): its linear index, or -1 outside the grid.
__device__ inline int neighbour(int k, int j, int i, int E, int A, bool circ) {
    const int dj = k < 3 ? -1 : k < 5 ? 0 : 1;
    const int di = k < 3 ? k - 1 : k == 3 ? -1 : k == 4 ? 1 : k - 6;
    const int jj = j + dj;
    int ii = i + di;
    if (circ) ii = ii < 0 ? ii + A : ii >= A ? ii - A : ii;
    if (jj < 0 || jj >= E || ii < 0 || ii >= A) return -1;
    return jj * A + ii;
}

// The peak rule on values v0 (the point, linear index l) and vn[k] of its neighbours nb[k].
__device__ inline bool peak_rule(double v0, int l, const int* nb, const double* vn) {
    bool ok = true, above = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (nb[k] < 0) continue;
        ok &= nb[k] < l ? v0 > vn[k] : v0 >= vn[k];
        above |= v0 > vn[k];
    }
    return ok && above;
}

template <int MB, typename TS>
__global__ __launch_bounds__(256) void peak2d_mark_kernel(const PointItem* __restrict__ items,
                                                          const FrameDev* __restrict__ frames,
                                                          const double* __restrict__ pos,
                                                          const double2* __restrict__ cis,
                                                          char* __restrict__ ws, const TS* __restrict__ spec,
                                                          int use_user, const uint32_t* __restrict__ status) {
    const PointItem it = items[blockIdx.x];
    const FrameDev& fr = frames[it.frame];
    const int l = it.l0 + (int)threadIdx.x;
    if (l >= fr.L) return;
    double* map = reinterpret_cast<double*>(ws + fr.ws_cand);
    if (status[it.frame] & NSSDOA_ST_NONFINITE_INPUT) {
        map[l] = -1.0;
        return;
    }
    const TS* P = spec + (use_user ? fr.spec_off_user : fr.spec_off_ws);
    const int A = fr.n_az, E = fr.L / fr.n_az;
    const int j = l / A, i = l - j * A;
    const bool circ = fr.circular != 0;
    int nb[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nb[k] = neighbour(k, j, i, E, A, circ);
    const double v0 = (double)P[l];
    double vn[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) vn[k] = nb[k] >= 0 ? (double)P[nb[k]] : 0.0;
    double out = -1.0;
    if (sizeof(TS) == sizeof(double)) {
        if (peak_rule(v0, l, nb, vn)) out = v0;
    } else {
        // a frame whose low-Q list overflowed has FP32 values near its nulls: every point is a
        // candidate then
        bool cand = *reinterpret_cast<const int*>(ws + fr.ws_lowq) != 0 || v0 != v0;
        if (!cand) {
            cand = true;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (nb[k] >= 0) cand &= v0 >= vn[k] * (1.0 - kRel);
        }
        if (cand) {
            const double* ps = pos + fr.pos_off;
            const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
            const double w0 = 1.0 / fmax(q64_eval<MB>(ps, fr.M, fr.K, B, grid_dir(fr, l), cis), 1e-300);
            double wn[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                wn[k] = nb[k] >= 0 ? 1.0 / fmax(q64_eval<MB>(ps, fr.M, fr.K, B, grid_dir(fr, nb[k]), cis), 1e-300)
                                   : 0.0;
            if (peak_rule(w0, l, nb, wn)) out = w0;
        }
    }
    map[l] = out;
}

__global__ __launch_bounds__(256) void peak2d_select_kernel(const int32_t* __restrict__ flist,
                                                            const FrameDev* __restrict__ frames,
                                                            const char* __restrict__ ws, int max_D,
                                                            nssdoa_peak* __restrict__ peaks,
                                                            int32_t* __restrict__ npeaks,
                                                            uint32_t* __restrict__ status) {
    __shared__ double cval[kCap2d];
    __shared__ int cidx[kCap2d];
    __shared__ int rankpos[64];
    __shared__ int count;
    const int f = flist[blockIdx.x];
    const FrameDev& fr = frames[f];
    const int tid = threadIdx.x;
    if (tid == 0) count = 0;
    __syncthreads();
    const double* map = reinterpret_cast<const double*>(ws + fr.ws_cand);
    uint32_t st = status[f];
    const bool nonfinite = (st & NSSDOA_ST_NONFINITE_INPUT) != 0;
    if (!nonfinite) {
        for (int l = tid; l < fr.L; l += blockDim.x) {
            const double v = map[l];
            if (v >= 0.0) {
                const int slot = atomicAdd(&count, 1);
                if (slot < kCap2d) {
                    cval[slot] = v;
                    cidx[slot] = l;
                }
            }
        }
    }
    __syncthreads();
    const int n = min(count, kCap2d);
    const int D = fr.D;
    for (int a = tid; a < n; a += blockDim.x) {
        const double va = cval[a];
        const int la = cidx[a];
        int rank = 0;
        for (int b = 0; b < n; ++b) rank += cval[b] > va || (cval[b] == va && cidx[b] < la);
        if (rank < D) rankpos[rank] = a;
    }
    __syncthreads();
    const int nout = min(n, D);
    nssdoa_peak* out = peaks + (size_t)f * max_D;
    for (int r = tid; r < max_D; r += blockDim.x) {
        if (r < nout) {
            const int a = rankpos[r];
            const int l = cidx[a];
            const int jj = l / fr.n_az, ii = l - jj * fr.n_az;
            out[r].idx = l;
            out[r].reserved = 0;
            out[r].angle_deg = grid_angle(fr.grid_start, fr.grid_step, ii);
            out[r].value = cval[a];
            out[r].polar_deg = grid_angle(fr.el_start, fr.el_step, jj);
        } else {
            out[r].idx = -1;
            out[r].reserved = 0;
            out[r].angle_deg = qnan2();
            out[r].value = qnan2();
            out[r].polar_deg = qnan2();
        }
    }
    if (tid == 0) {
        npeaks[f] = nout;
        if (nout < D) st |= NSSDOA_ST_FEWER_PEAKS;
        if (count > kCap2d) st |= NSSDOA_ST_PEAK_OVERFLOW;
        status[f] = st;
    }
}

}  // namespace

int peak2d_map_bytes_per_point() { return (int)sizeof(double); }

hipError_t launch_peaks2d(bool f64, int bucket_M, const PointItem* items, int n_items, const int32_t* flist,
                          int n_frames, const FrameDev* frames, const double* pos, const double2* cis, char* ws,
                          const void* spec, int use_user, int max_D, nssdoa_peak* peaks, int32_t* npeaks,
                          uint32_t* status, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    if (max_D < 1 || max_D > 64) return hipErrorInvalidValue;
#define NSSDOA_P2D_CASE(MB)                                                                                    \
    case MB:                                                                                                \
        if (f64)                                                                                            \
            hipLaunchKernelGGL((peak2d_mark_kernel<MB, double>), dim3(n_items), dim3(256), 0, s, items, frames, \
                               pos, cis, ws, static_cast<const double*>(spec), use_user, status);             \
        else                                                                                                \
            hipLaunchKernelGGL((peak2d_mark_kernel<MB, float>), dim3(n_items), dim3(256), 0, s, items, frames,  \
                               pos, cis, ws, static_cast<const float*>(spec), use_user, status);              \
        break;
    switch (bucket_M) {
        NSSDOA_P2D_CASE(8)
        NSSDOA_P2D_CASE(16)
        NSSDOA_P2D_CASE(32)
        NSSDOA_P2D_CASE(64)
        default: return hipErrorInvalidValue;
    }
#undef NSSDOA_P2D_CASE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(peak2d_select_kernel, dim3(n_frames), dim3(256), 0, s, flist, frames, ws, max_D, peaks,
                       npeaks, status);
    return hipGetLastError();
}

}  // namespace nssdoa
