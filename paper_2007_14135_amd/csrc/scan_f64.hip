// Step-5 (Table 2) in FP64 for complex128 batches: one thread per (frame, grid angle) evaluates
// ||B^H a(theta)||^2 with FP64 steering (phase reduced before sincospi) and FP64 accumulation,
// and writes P = 1 / max(Q, 1e-300).
#include "internal.h"

namespace nssdoa {
namespace {

template <int MB>
__global__ __launch_bounds__(256) void scan_f64_kernel(const PointItem* __restrict__ items,
                                                       const FrameDev* __restrict__ frames,
                                                       const double* __restrict__ pos,
                                                       const double2* __restrict__ cis,
                                                       const char* __restrict__ ws,
                                                       double* __restrict__ spec, int use_user) {
    const PointItem it = items[blockIdx.x];
    const FrameDev& fr = frames[it.frame];
    const int l = it.l0 + (int)threadIdx.x;
    if (l >= fr.L) return;
    const double2* B = reinterpret_cast<const double2*>(ws + fr.ws_B);
    const double Q = q64_eval<MB>(pos + fr.pos_off, fr.M, fr.K, B,
                                  grid_dir(fr, l), cis);
    double* out = spec + (use_user ? fr.spec_off_user : fr.spec_off_ws);
    out[l] = 1.0 / fmax(Q, 1e-300);
}

}  // namespace

hipError_t launch_scan_f64(const PointItem* items, int n_items, int max_M,
                           const FrameDev* frames, const double* pos, const double2* cis,
                           const char* ws, double* spec, int use_user, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (max_M <= 8)
        hipLaunchKernelGGL(scan_f64_kernel<8>, dim3(n_items), dim3(256), 0, s, items, frames, pos, cis, ws, spec, use_user);
    else if (max_M <= 16)
        hipLaunchKernelGGL(scan_f64_kernel<16>, dim3(n_items), dim3(256), 0, s, items, frames, pos, cis, ws, spec, use_user);
    else if (max_M <= 32)
        hipLaunchKernelGGL(scan_f64_kernel<32>, dim3(n_items), dim3(256), 0, s, items, frames, pos, cis, ws, spec, use_user);
    else
        hipLaunchKernelGGL(scan_f64_kernel<64>, dim3(n_items), dim3(256), 0, s, items, frames, pos, cis, ws, spec, use_user);
    return hipGetLastError();
}

}  // namespace nssdoa
