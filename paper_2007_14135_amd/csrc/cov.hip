// Step-1 (Eq. 3): partial sample covariances  sum_n x_i[n] conj(x_j[n])  over snapshot chunks.
//
// One workgroup per (frame, snapshot chunk).  The chunk is staged through LDS in tiles of
// 1024 complex values converted to FP64; each thread owns a 4x4 block of the upper block
// triangle of R for a strided subset of the tile's snapshots and accumulates in FP64.  For
// complex64 input every product of two FP32 values is exact in FP64, so the only rounding is
// the FP64 accumulation.  The per-thread partials are reduced across snapshot subsets in a fixed
// order and written to the workspace; the eigen kernel adds the chunks in order and divides by
// N, so the result does not depend on scheduling.
#include "internal.h"

namespace nssdoa {
namespace {

constexpr int kTileElems = 1024;   // complex values staged per LDS tile
constexpr int kThreads = 256;

template <typename TIn>
__device__ inline double2 load_c(const TIn* p);
template <>
__device__ inline double2 load_c<float2>(const float2* p) {
    float2 v = *p;
    return make_double2((double)v.x, (double)v.y);
}
template <>
__device__ inline double2 load_c<double2>(const double2* p) {
    return *p;
}

template <typename TIn>
__global__ __launch_bounds__(kThreads) void cov_kernel(const CovItem* __restrict__ items,
                                                       const FrameDev* __restrict__ frames,
                                                       const TIn* __restrict__ X,
                                                       char* __restrict__ ws) {
    __shared__ double2 xs[kTileElems];
    __shared__ double2 red[kThreads];

    const CovItem it = items[blockIdx.x];
    const FrameDev& fr = frames[it.frame];
    const int M = fr.M;
    const int T = (M + 3) >> 2;              // 4-row blocks
    const int PT = T * (T + 1) / 2;          // upper block-triangle pairs
    const int G = kThreads / PT;             // snapshot subsets
    const int M4 = T * 4;
    const int NT = kTileElems / M4;          // snapshots per LDS tile
    const int tid = threadIdx.x;
    const bool active = tid < PT * G;
    const int tp = tid % PT;
    const int g = tid / PT;

    // (ti, tj), ti <= tj, from the pair index tp (row-major over the upper block triangle)
    int ti = 0, rem = tp;
    while (rem >= T - ti) { rem -= T - ti; ++ti; }
    const int tj = ti + rem;

    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);

    const TIn* xf = X + fr.x_off;
    // Tiles are staged through registers: the next tile's loads are in flight while the current
    // tile is being accumulated.  Thread tid stages elements e = tid + u * 256 (m = e / NT).
    constexpr int kPer = kTileElems / kThreads;
    int em[kPer], en[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * kThreads;
        em[u] = e / NT;
        en[u] = e - em[u] * NT;
    }
    double2 pre[kPer];
    auto fetch = [&](int nb) {
        const int cnt = min(NT, it.n1 - nb);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            pre[u] = make_double2(0.0, 0.0);
            if (em[u] < M && en[u] < cnt) pre[u] = load_c<TIn>(xf + (size_t)em[u] * fr.ldx + nb + en[u]);
        }
    };
    fetch(it.n0);
    for (int nb = it.n0; nb < it.n1; nb += NT) {
        const int cnt = min(NT, it.n1 - nb);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (em[u] < M4) xs[tid + u * kThreads] = pre[u];
        __syncthreads();
        if (nb + NT < it.n1) fetch(nb + NT);
        if (active) {
            for (int n = g; n < cnt; n += G) {
                double2 xi[4], xj[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    xi[a] = xs[(4 * ti + a) * NT + n];
                    xj[a] = xs[(4 * tj + a) * NT + n];
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        // x_i conj(x_j) = (ar br + ai bi) + j (ai br - ar bi)
                        acc[a][b].x = fma(xi[a].x, xj[b].x, acc[a][b].x);
                        acc[a][b].x = fma(xi[a].y, xj[b].y, acc[a][b].x);
                        acc[a][b].y = fma(xi[a].y, xj[b].x, acc[a][b].y);
                        acc[a][b].y = fma(-xi[a].x, xj[b].y, acc[a][b].y);
                    }
            }
        }
    }

    // Reduce the G snapshot subsets in a fixed order, one accumulator entry at a time.
    double2* out = reinterpret_cast<double2*>(ws + fr.ws_partial) + (size_t)it.chunk * M * M;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            __syncthreads();
            red[tid] = active ? acc[a][b] : make_double2(0.0, 0.0);
            __syncthreads();
            if (tid < PT) {
                double2 s = red[tid];
                for (int q = 1; q < G; ++q) {
                    double2 v = red[q * PT + tid];
                    s.x += v.x;
                    s.y += v.y;
                }
                const int i = 4 * ti + a, j = 4 * tj + b;
                if (i < M && j < M) out[i * M + j] = s;
            }
        }
}

}  // namespace

hipError_t launch_cov(bool c128, const CovItem* items, int n_items, const FrameDev* frames,
                      const void* X, char* ws, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (c128)
        hipLaunchKernelGGL(cov_kernel<double2>, dim3(n_items), dim3(kThreads), 0, s, items, frames,
                           static_cast<const double2*>(X), ws);
    else
        hipLaunchKernelGGL(cov_kernel<float2>, dim3(n_items), dim3(kThreads), 0, s, items, frames,
                           static_cast<const float2*>(X), ws);
    return hipGetLastError();
}

}  // namespace nssdoa
