// Step-1 (Eq. 3): partial sample covariances  sum_n x_i[n] conj(x_j[n])  over snapshot chunks.
//
// Two kernels compute the same partial sums; both accumulate in FP64.
//
// cov_mfma_kernel (M <= 32): the real-embedded Gram on the FP64 matrix cores, from two real
// products instead of three.  With P = Xi Xr^T and Z = Xr + Xi, Im R = P - P^T and
// Re R = Xr Xr^T + Xi Xi^T = Z Z^T - P - P^T, so per 16-row block pair two 16x16x4 products are
// accumulated (Z Z^T over I <= J, P over all pairs).  Products of two FP32 values (P) are exact
// in FP64; z = xr + xi rounds by at most u|z| (u = 2^-53; exact unless the exponents of xr and
// xi differ by more than 29) and z_i z_j by at most u|z_i z_j|, so with |z| <= sqrt(2)|x| and
// Cauchy-Schwarz over the snapshots the real part of R gains at most 6u sqrt(R_ii R_jj) beyond
// the FP64 accumulation's own rounding; integer-valued data stays exact.  Lane l holds element
// l%16 of snapshot group l/16: that one register is both the A operand (A[i][k], i = l%16,
// k = l/16) and the B operand (B[k][j], j = l%16) of v_mfma_f64_16x16x4f64, whose result
// register r of lane l is D[l/16 + 4r][l%16].  Each wave owns every fourth 16-snapshot block of the chunk and keeps
// three blocks of loads in flight (raw complex64 read as aligned float4 when the layout allows)
// while the matrix cores run; the four waves are reduced in LDS in fixed order.
//
// cov_kernel (any M): the chunk is staged through LDS in tiles of
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
                                                       char* __restrict__ ws, int* reset) {
    __shared__ double2 xs[kTileElems + 64];     // rows padded by one element (bank conflicts)
    __shared__ double2 red[kThreads];

    const CovItem it = items[blockIdx.x];
    if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0;   // the batch's low-Q count
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
            if (em[u] < M4) xs[em[u] * (NT + 1) + en[u]] = pre[u];
        __syncthreads();
        if (nb + NT < it.n1) fetch(nb + NT);
        if (active) {
            for (int n = g; n < cnt; n += G) {
                double2 xi[4], xj[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    xi[a] = xs[(4 * ti + a) * (NT + 1) + n];
                    xj[a] = xs[(4 * tj + a) * (NT + 1) + n];
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

typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename TIn, int RB>   // RB = 16-row blocks (M <= 16 RB)
__global__ __launch_bounds__(256) void cov_mfma_kernel(const CovItem* __restrict__ items,
                                                       const FrameDev* __restrict__ frames,
                                                       const TIn* __restrict__ X,
                                                       char* __restrict__ ws, int* reset) {
    constexpr int NP = RB * (RB + 1) / 2;          // symmetric block pairs (I <= J)
    constexpr int NX = RB * RB;                    // all block pairs of Xi Xr^T
    __shared__ double sre[4][RB * 16][RB * 16 + 1];
    __shared__ double sim[4][RB * 16][RB * 16 + 1];

    const CovItem it = items[blockIdx.x];
    if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0;   // the batch's low-Q count
    const FrameDev& fr = frames[it.frame];
    const int M = fr.M;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mi = lane & 15, q = lane >> 4;       // element in a row block, snapshot group

    doublex4 dzz[NP], dir[NX];
#pragma unroll
    for (int t = 0; t < NP; ++t) dzz[t] = doublex4{0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < NX; ++t) dir[t] = doublex4{0, 0, 0, 0};

    const TIn* xf = X + fr.x_off;
    // per row block b: this lane's element row and whether it exists
    const TIn* rowp[RB];
    bool rowok[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const int m = b * 16 + mi;
        rowok[b] = m < M;
        rowp[b] = xf + (size_t)(rowok[b] ? m : 0) * fr.ldx;
    }
    // one 16-snapshot step of the two products from lane (mi, q)'s four snapshots n + 4q + u
    auto mfma_step = [&](const double (&xr)[RB], const double (&xi)[RB]) {
        double z[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) z[b] = xr[b] + xi[b];
        int t = 0;
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = I; J < RB; ++J, ++t)
                dzz[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[I], z[J], dzz[t], 0, 0, 0);
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = 0; J < RB; ++J)
                dir[I * RB + J] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[I], xr[J], dir[I * RB + J], 0, 0, 0);
    };
    const int first = it.n0 + 16 * wave;           // this wave's blocks: first + 64 k
    const int nblk = first < it.n1 ? (it.n1 - first + 63) / 64 : 0;
    bool vec = false;
    if constexpr (sizeof(TIn) == 8) {
        // complex64 frames whose rows and chunks start on 16-byte boundaries and whose chunk is
        // whole 16-snapshot blocks: the four snapshots of a lane are two aligned float4, kept
        // raw in a ring of three blocks in flight per wave
        vec = ((fr.x_off | fr.ldx | it.n0) & 1) == 0 && ((it.n1 - it.n0) & 15) == 0 &&
              (reinterpret_cast<uintptr_t>(X) & 15) == 0;
    }
    if (vec) {
        struct Raw { float4 a[RB][2]; };
        auto load_raw = [&](int n, Raw& r) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    r.a[b][h] = rowok[b] ? *reinterpret_cast<const float4*>(rowp[b] + n + 4 * q + 2 * h)
                                         : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        };
        auto process = [&](const Raw& r) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                double xr[RB], xi[RB];
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const float4 v = r.a[b][u >> 1];
                    xr[b] = (double)((u & 1) ? v.z : v.x);
                    xi[b] = (double)((u & 1) ? v.w : v.y);
                }
                mfma_step(xr, xi);
            }
        };
        Raw r0, r1, r2;
        if (nblk > 0) load_raw(first, r0);
        if (nblk > 1) load_raw(first + 64, r1);
        if (nblk > 2) load_raw(first + 128, r2);
        for (int k = 0; k < nblk; k += 3) {
            process(r0);
            if (k + 3 < nblk) load_raw(first + 64 * (k + 3), r0);
            if (k + 1 < nblk) {
                process(r1);
                if (k + 4 < nblk) load_raw(first + 64 * (k + 4), r1);
            }
            if (k + 2 < nblk) {
                process(r2);
                if (k + 5 < nblk) load_raw(first + 64 * (k + 5), r2);
            }
        }
    } else {
        double2 cur[RB][4], nxt[RB][4];
        auto fetch = [&](int n, double2 (&dst)[RB][4]) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int nn = n + 4 * q + u;
                    dst[b][u] = (rowok[b] && nn < it.n1) ? load_c<TIn>(rowp[b] + nn) : make_double2(0.0, 0.0);
                }
        };
        int n = first;
        if (n < it.n1) fetch(n, cur);
        for (; n < it.n1; n += 64) {
            if (n + 64 < it.n1) fetch(n + 64, nxt);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                double xr[RB], xi[RB];
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    xr[b] = cur[b][u].x;
                    xi[b] = cur[b][u].y;
                }
                mfma_step(xr, xi);
            }
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int u = 0; u < 4; ++u) cur[b][u] = nxt[b][u];
        }
    }

    // scatter this wave's sums to LDS: Z Z^T over I <= J, P = Xi Xr^T over all block pairs
    {
        int t = 0;
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = I; J < RB; ++J, ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    sre[wave][I * 16 + q + 4 * r][J * 16 + mi] = dzz[t][r];
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = 0; J < RB; ++J)
#pragma unroll
                for (int r = 0; r < 4; ++r) sim[wave][I * 16 + q + 4 * r][J * 16 + mi] = dir[I * RB + J][r];
    }
    __syncthreads();
    double2* out = reinterpret_cast<double2*>(ws + fr.ws_partial) + (size_t)it.chunk * M * M;
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        const int i = e / M, j = e - i * M;
        if (i > j) continue;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const double pij = sim[w][i][j], pji = sim[w][j][i];
            re += sre[w][i][j] - (pij + pji);    // Re R_ij = (Z Z^T - P - P^T)_ij
            im += pij - pji;                     // Im R_ij = sum xi_i xr_j - xr_i xi_j
        }
        out[i * M + j] = make_double2(re, im);
    }
}

}  // namespace

hipError_t launch_cov(bool c128, int max_M, const CovItem* items, int n_items, const FrameDev* frames,
                      const void* X, char* ws, int* reset, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (max_M <= 32) {
        if (c128) {
            if (max_M <= 16)
                hipLaunchKernelGGL((cov_mfma_kernel<double2, 1>), dim3(n_items), dim3(256), 0, s, items, frames,
                                   static_cast<const double2*>(X), ws, reset);
            else
                hipLaunchKernelGGL((cov_mfma_kernel<double2, 2>), dim3(n_items), dim3(256), 0, s, items, frames,
                                   static_cast<const double2*>(X), ws, reset);
        } else {
            if (max_M <= 16)
                hipLaunchKernelGGL((cov_mfma_kernel<float2, 1>), dim3(n_items), dim3(256), 0, s, items, frames,
                                   static_cast<const float2*>(X), ws, reset);
            else
                hipLaunchKernelGGL((cov_mfma_kernel<float2, 2>), dim3(n_items), dim3(256), 0, s, items, frames,
                                   static_cast<const float2*>(X), ws, reset);
        }
        return hipGetLastError();
    }
    if (c128)
        hipLaunchKernelGGL(cov_kernel<double2>, dim3(n_items), dim3(kThreads), 0, s, items, frames,
                           static_cast<const double2*>(X), ws, reset);
    else
        hipLaunchKernelGGL(cov_kernel<float2>, dim3(n_items), dim3(kThreads), 0, s, items, frames,
                           static_cast<const float2*>(X), ws, reset);
    return hipGetLastError();
}

}  // namespace nssdoa
