// Steps 2-4 (Table 2 Step-2, Table 3): FP64 Hermitian eigendecomposition of R and the
// noise-subspace matrix B with C = B B^H.
//
// One workgroup per frame.  The workgroup first adds the frame's partial covariances in chunk
// order and divides by N (Eq. 3).  Three eigensolvers:
//
// * For M <= 16 (the default there): one wave per frame, Householder reduction with the matrix
//   and the unitary factor in registers, Sturm-count multisection for the eigenvalues and
//   inverse iteration for the eigenvectors (described before evd_small_kernel).
// * Householder + implicit QL (the default for M > 16).  R is reduced to a real symmetric tridiagonal matrix
//   T = Q^H R Q with Q = H_0 H_1 ... H_{M-2}, H_k = I - tau_k v_k v_k^H chosen so that H_k^H maps
//   the part of column k below the diagonal onto a real multiple of its first unit vector (the
//   two-sided update of the trailing block is the rank-2 form A -= v w^H + w v^H,
//   w = tau A v - |tau|^2 (v^H A v) / 2 v).  T is diagonalised by implicit QL sweeps with
//   Wilkinson's shift (a bulge chased from the bottom of the unreduced block to its top with
//   Givens rotations, the rotations accumulated into Z; the block splits where
//   |e_i| <= tol (|d_i| + |d_{i+1}|)), one wave running the sequential rotation chain while each
//   lane updates one row of Z.  The eigenvectors are V = Q Z, applied reflector by reflector to
//   the columns of Z.  About 3 M^2 / 2 dependent rotations per frame, against 8-10 Jacobi sweeps
//   of M - 1 dependent steps that each need a workgroup barrier.
// * Cyclic Jacobi.  Complex Jacobi rotations in round-robin order: M/2 disjoint pivot pairs per
//   step, M-1 steps per sweep, so every step is one fully parallel two-sided update of the 2x2
//   blocks of A and one update of V; each wave computes the step's M/2 rotations once into LDS
//   and its tasks read them there.  A rotation for pivot (p, q) first removes the phase of r_pq
//   with diag(1, exp(-j arg r_pq)) and then applies the real rotation [[c, s], [-s, c]] with
//   t = sgn(theta) / (|theta| + sqrt(theta^2+1)), theta = (r_qq - r_pp) / (2 |r_pq|).  Sweeps
//   stop when every |r_pq| <= tol * sqrt(r_pp r_qq), a relative criterion that also keeps
//   eigenvalues far below ||R|| accurate to working precision relative to themselves.
//
// Eigenvalues are then ranked in descending order and B is built for the requested method, in
// FP64 and (for the matrix-core scans) as the packed real-embedded operand tiles of the scan.
#include <float.h>

#include <algorithm>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {


__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Block-wide reductions: butterfly inside each wave, then one LDS pass over the wave results.
__device__ inline double block_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) red[wid] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < nw; ++w) r = fmax(r, red[w]);
    __syncthreads();
    return r;
}

__device__ inline double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) red[wid] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < nw; ++w) r += red[w];
    __syncthreads();
    return r;
}

// FP64 reciprocal square root and reciprocal: hardware estimate plus two Newton steps.
__device__ __forceinline__ double rsq64(double x) {
    double r = __builtin_amdgcn_rsq(x);
    r = fma(0.5 * r, fma(-x, r * r, 1.0), r);
    r = fma(0.5 * r, fma(-x, r * r, 1.0), r);
    return r;
}
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// rsqrt to working precision in one step: from the hardware estimate r0 (relative error near
// 2^-24), h = 1 - x r0^2 and r = r0 (1 + h/2 + 3h^2/8), which leaves an O(h^3) error.
__device__ __forceinline__ double rsq_full(double x) {
    const double r0 = __builtin_amdgcn_rsq(x);
    const double h = fma(-(x * r0), r0, 1.0);
    return fma(r0 * h, fma(h, 0.375, 0.5), r0);
}
// reciprocal to about 2^-48 (one Newton step), enough for a QL shift
__device__ __forceinline__ double rcp_approx(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// x rounded to the nearest FP16 value (ties to even): x is first rounded to FP32 with round to
// odd (truncated, and the last bit set when inexact), which keeps 13 bits beyond FP16's 11, so
// the hardware's round to nearest from FP32 then rounds as if from x itself.
__device__ __forceinline__ _Float16 f64_to_f16(double x) {
    const float f = (float)x;
    const double back = (double)f;
    uint32_t u = __float_as_uint(f);
    if (back != x) {
        if (fabs(back) > fabs(x)) u -= 1u;     // rounded away from zero: step back toward it
        u |= 1u;
    }
    return (_Float16)__uint_as_float(u);
}

// Cross-lane moves of doubles (two 32-bit DPP moves or lane reads).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int kDppRowMirror = 0x140;     // lane i <- lane 15 - i within each row of 16
constexpr int kDppRowHalfMirror = 0x141; // lane i <- lane 7 - i within each half row

// Sum over each aligned group of four lanes, in all four (the group must be active).
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_f64<kDppQuadXor1>(v);
    return v + dpp_f64<kDppQuadXor2>(v);
}
// Sum over the 64 lanes of a fully active wave; every lane gets the same value.
__device__ __forceinline__ double wave_sum(double v) {
    v = quad_sum(v);
    v += dpp_f64<kDppRowHalfMirror>(v);
    v += dpp_f64<kDppRowMirror>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
// Maximum over the 64 lanes of a fully active wave; every lane gets the same value.
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<kDppQuadXor1>(v));
    v = fmax(v, dpp_f64<kDppQuadXor2>(v));
    v = fmax(v, dpp_f64<kDppRowHalfMirror>(v));
    v = fmax(v, dpp_f64<kDppRowMirror>(v));
    return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}
// Block-wide sum of q and maximum of mx over fully active waves, in one LDS exchange (red: two
// doubles per wave).
__device__ inline void block_sum_max(double& q, double& mx, double* red) {
    q = wave_sum(q);
    mx = wave_max(mx);
    const int nw = (blockDim.x + 63) >> 6;
    if (nw == 1) return;
    if ((threadIdx.x & 63) == 0) {
        red[2 * (threadIdx.x >> 6)] = q;
        red[2 * (threadIdx.x >> 6) + 1] = mx;
    }
    __syncthreads();
    q = red[0];
    mx = red[1];
    for (int w = 1; w < nw; ++w) {
        q += red[2 * w];
        mx = fmax(mx, red[2 * w + 1]);
    }
    __syncthreads();
}
// Block-wide sum of fully active waves: wave sums, then (with several waves) one LDS pass.
__device__ inline double block_sum_fast(double v, double* red) {
    v = wave_sum(v);
    const int nw = (blockDim.x + 63) >> 6;
    if (nw == 1) return v;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < nw; ++w) r += red[w];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------------------------
// The default eigensolver for M <= kSmallM (evd_small_kernel): four waves per frame, one per SIMD
// of the compute unit, thread t owning entry (t / 16, t % 16) of the matrices.
//   1. R = (sum of the chunk partials, in chunk order) / N (load_covariance).
//   2. Householder reduction T = Q^H R Q with R and Q one entry per thread.  H_k = I - tau_k u_k
//      u_k^H maps column k below the diagonal onto a real multiple beta_k of its first unit
//      vector; the reflector is kept unnormalised, u = (alpha - beta, x), tau = (beta - alpha) /
//      (beta |alpha - beta|^2) (the usual v = u / (alpha - beta) with tau (beta - alpha) / beta).
//      The sixteen threads of row k form it from row k alone (column k is its conjugate): the
//      norm by a reduction within their row of lanes, beta and 1/beta from one reciprocal square
//      root; u goes to LDS.  Every thread then forms its row's part of y = A u and z = Q u (row
//      reductions), y goes to LDS for the columns and the waves' parts of gamma = u^H y meet in
//      LDS; the trailing block takes the rank-2 update A -= u w^H + w u^H with w = tau y -
//      |tau|^2 gamma / 2 u, and Q <- Q H_k = Q - tau z u^H, so V = Q Z needs no separate
//      back-transformation.  Two barriers per step.
//   3. Eigenvalues of T by Sturm counts: the number of eigenvalues below x is the number of
//      sign changes along the leading principal minors p_i of T - x I, whose three-term
//      recurrence needs no division (T is scaled by a power of two to a norm in [1/2, 1), the
//      minors are rescaled by powers of two every fourth row, and a minor that vanishes is
//      replaced by -2^-60 times its predecessor: a negative pivot far below rounding).  A coarse
//      pass counts at 256 points across the Gershgorin interval, then 17-section: the sixteen
//      lanes of eigenvalue j count at the sixteen inner points of its interval, down to
//      2 eps ||T||.
//   4. Eigenvectors of T by inverse iteration (one wave): lane j solves (T - lambda_j I) x = b
//      twice by LU with partial pivoting (a zero pivot is replaced by eps ||T||) from a
//      pseudo-random start, and the vectors are orthonormalised by modified Gram-Schmidt within
//      clusters of close eigenvalues.  If that moved some vector towards another by more than
//      16 eps ||T|| / |lambda_j - lambda_k| (nearly dependent vectors of a tight cluster, where
//      the projection mixes in what the solves had not yet removed), every vector is solved
//      once more and orthonormalised again.
//   5. V = Q Z; ranking, B and the scan operands as for the other solvers.
constexpr int kSmallM = 16;
constexpr int kSmallThreads = kSmallM * kSmallM;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over each aligned row of 16 lanes, in all 16 (the row must be active).
__device__ __forceinline__ double row16_sum(double v) {
    v = quad_sum(v);
    v += dpp_f64<kDppRowHalfMirror>(v);
    return v + dpp_f64<kDppRowMirror>(v);
}

// Step 2 (see above).  A: R in LDS (row stride ld); on return the thread holds Q[r][c] in qm,
// T is in dq (diagonal) and eq (off-diagonal, eq[M-1] = 0).  ubuf, ybuf: 16 entries; sc: two
// complex scalars; gpart: one double per wave.
__device__ void tridiag_block(int M, const double2* A, int ld, double* dq, double* eq, double2* ubuf, double2* ybuf,
                              double2* sc, double* gpart, double2& qm) {
    const int tid = threadIdx.x, r = tid >> 4, c = tid & 15, lane = tid & 63;
    double2 a = (r < M && c < M) ? A[r * ld + c] : make_double2(0.0, 0.0);
    qm = make_double2((r == c && r < M) ? 1.0 : 0.0, 0.0);
    for (int k = 0; k < M - 1; ++k) {
        if (r == k) {
            // the sixteen lanes of row k: ||A[k][k+2:]||^2, alpha = A[k+1][k] = conj(A[k][k+1])
            const double xn2 = row16_sum(c > k + 1 ? fma(a.x, a.x, a.y * a.y) : 0.0);
            const int l0 = 16 * (k & 3);             // row k: lanes l0 .. l0 + 15 of wave k / 4
            const double2 alpha = make_double2(readlane_f64(a.x, l0 + k + 1), -readlane_f64(a.y, l0 + k + 1));
            const double dk = readlane_f64(a.x, l0 + k);
            double beta = alpha.x;
            double2 tau = make_double2(0.0, 0.0), u1 = make_double2(0.0, 0.0);
            if (xn2 > 0.0 || alpha.y != 0.0) {
                const double s2 = fma(alpha.x, alpha.x, fma(alpha.y, alpha.y, xn2));
                const double rs = rsq_full(s2);
                beta = -copysign(s2 * rs, alpha.x);
                u1 = make_double2(alpha.x - beta, alpha.y);
                const double rt = rcp64(beta * fma(u1.x, u1.x, u1.y * u1.y));
                tau = make_double2((beta - alpha.x) * rt, -alpha.y * rt);
            }
            // u_{k+1} = alpha - beta, u_c = A[c][k] = conj(A[k][c]) for c > k + 1, 0 elsewhere
            ubuf[c] = (c == k + 1) ? u1 : (c > k + 1 && c < M) ? cconj(a) : make_double2(0.0, 0.0);
            if (c == 0) {
                sc[0] = tau;
                dq[k] = dk;
                eq[k] = beta;
            }
        }
        __syncthreads();
        const double2 tau = sc[0];
        if (tau.x == 0.0 && tau.y == 0.0) continue;      // uniform: H_k = I
        const double2 ur = ubuf[r], uc = ubuf[c];
        // row parts of y = A u and z = Q u
        double2 y = make_double2(fma(a.x, uc.x, -a.y * uc.y), fma(a.x, uc.y, a.y * uc.x));
        double2 z = make_double2(fma(qm.x, uc.x, -qm.y * uc.y), fma(qm.x, uc.y, qm.y * uc.x));
        y.x = row16_sum(y.x);
        y.y = row16_sum(y.y);
        z.x = row16_sum(z.x);
        z.y = row16_sum(z.y);
        if (c == 0) ybuf[r] = y;
        // gamma = sum over rows r > k of Re(conj(u_r) y_r): the wave's four rows, then the waves
        double g = (r > k) ? fma(ur.x, y.x, ur.y * y.y) : 0.0;
        g = (readlane_f64(g, 0) + readlane_f64(g, 16)) + (readlane_f64(g, 32) + readlane_f64(g, 48));
        if (lane == 0) gpart[tid >> 6] = g;
        __syncthreads();
        const double gam = (gpart[0] + gpart[1]) + (gpart[2] + gpart[3]);
        const double h = 0.5 * fma(tau.x, tau.x, tau.y * tau.y) * gam;
        const double2 yc = ybuf[c];
        const double2 wr = (r > k && r < M) ? csub(cmul(tau, y), cscale(h, ur)) : make_double2(0.0, 0.0);
        const double2 wc = (c > k && c < M) ? csub(cmul(tau, yc), cscale(h, uc)) : make_double2(0.0, 0.0);
        const double2 tz = cmul(tau, z);
        // A -= u w^H + w u^H;  Q -= (tau Q u) u^H
        a.x -= fma(ur.x, wc.x, ur.y * wc.y) + fma(wr.x, uc.x, wr.y * uc.y);
        a.y -= fma(ur.y, wc.x, -ur.x * wc.y) + fma(wr.y, uc.x, -wr.x * uc.y);
        qm.x -= fma(tz.x, uc.x, tz.y * uc.y);
        qm.y -= fma(tz.y, uc.x, -tz.x * uc.y);
    }
    if (r == M - 1 && c == M - 1) {
        dq[M - 1] = a.x;
        eq[M - 1] = 0.0;
    }
}

// Eigenvalues of T below x: sign changes along p_0 = 1, p_{i+1} = (dp_i - x) p_i - e2_i p_{i-1}
// (dp: scaled diagonal padded with decoupled rows above every point counted, e2_i: squared
// scaled coupling of rows i - 1 and i, e2_0 = 0).
__device__ __forceinline__ int sturm_count(const double (&dp)[kSmallM], const double (&e2)[kSmallM], double x) {
    double p0 = 0.0, p1 = 1.0;
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kSmallM; ++i) {
        double pn = fma(dp[i] - x, p1, -e2[i] * p0);
        pn = pn != 0.0 ? pn : -0x1p-60 * p1;
        cnt += (pn < 0.0) != (p1 < 0.0);
        p0 = p1;
        p1 = pn;
        if ((i & 3) == 3) {
            const int ex = __builtin_amdgcn_frexp_exp(p1);
            p1 = __builtin_amdgcn_ldexp(p1, -ex);
            p0 = __builtin_amdgcn_ldexp(p0, -ex);
        }
    }
    return cnt;
}

// Step 3, all four waves: eigenvalue j of T (ascending, j < M) to lamv[j]; returns the
// Gershgorin bound tnorm of ||T|| (0 when T = 0: every eigenvalue is then 0).  first: 64 ints.
__device__ double eigvals_block(int M, const double (&d)[kSmallM], const double (&e)[kSmallM], double* lamv,
                                int* first) {
    constexpr int MB = kSmallM;
    constexpr double eps = 0x1p-52;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int grp = lane >> 4, p = lane & 15, j = 4 * wv + grp;
    double gl = INFINITY, gu = -INFINITY;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        if (i < M) {
            const double r = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
            gl = fmin(gl, d[i] - r);
            gu = fmax(gu, d[i] + r);
        }
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    if (!(tnorm > 0.0)) {
        if (tid < M) lamv[tid] = 0.0;
        return 0.0;
    }
    // scale by 2^-ex: ||T|| bound in [1/2, 1); rows beyond M sit at 4, above every point
    const int ex = __builtin_amdgcn_frexp_exp(tnorm);
    double dp[MB], e2[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        dp[i] = i < M ? __builtin_amdgcn_ldexp(d[i], -ex) : 4.0;
        const double es = (i > 0 && i < M) ? __builtin_amdgcn_ldexp(e[i - 1], -ex) : 0.0;
        e2[i] = es * es;
    }
    const double tn = __builtin_amdgcn_ldexp(tnorm, -ex);
    const double pad = 2.1 * (tn * eps * M + 0x1p-57);
    const double tol = 2.0 * eps * tn + 0x1p-58;
    // coarse pass: thread t counts at the point t + 1 of 257 across the Gershgorin interval;
    // eigenvalue j lies above the last point below which at most j eigenvalues lie
    const double g0 = __builtin_amdgcn_ldexp(gl, -ex) - pad;
    const double gw = (__builtin_amdgcn_ldexp(gu, -ex) + pad) - g0;
    constexpr double kInv257 = 1.0 / 257.0;
    const int cc = sturm_count(dp, e2, g0 + gw * ((double)(tid + 1) * kInv257));
    for (int jj = 0; jj < M; ++jj) {
        const unsigned long long bal = __ballot(cc > jj);
        if (lane == jj) first[wv * 16 + jj] = bal ? __builtin_ctzll(bal) : 64;
    }
    __syncthreads();
    int kf = 256;
    if (j < M) {
#pragma unroll
        for (int w = 3; w >= 0; --w) {
            const int f = first[w * 16 + j];
            kf = f < 64 ? 64 * w + f : kf;
        }
    }
    double lo = kf == 0 ? g0 : g0 + gw * ((double)kf * kInv257);
    double hi = kf == 256 ? g0 + gw : g0 + gw * ((double)(kf + 1) * kInv257);
    const int its = min(64, max(1, (int)ceil(log2(gw * kInv257 / tol) / log2(17.0)) + 1));
    // 17-section: lane p of eigenvalue j's row of lanes counts at point p + 1 of 17
    constexpr double kInv17 = 1.0 / 17.0;
    for (int it = 0; it < its; ++it) {
        const double w = hi - lo;
        const int cnt = sturm_count(dp, e2, lo + w * ((double)(p + 1) * kInv17));
        // the first point below which more than j eigenvalues lie bounds eigenvalue j above
        const unsigned long long bal = __ballot(cnt > j);
        const uint32_t bits = (uint32_t)(bal >> (16 * grp)) & 0xFFFFu;
        const int k = bits ? __builtin_ctz(bits) : 16;
        const double nlo = k == 0 ? lo : lo + w * ((double)k * kInv17);
        const double nhi = k == 16 ? hi : lo + w * ((double)(k + 1) * kInv17);
        lo = nlo;
        hi = nhi;
    }
    if (p == 0 && j < M) lamv[j] = __builtin_amdgcn_ldexp(0.5 * (lo + hi), ex);
    return tnorm;
}

// Deterministic pseudo-random start of inverse iteration, in [-1, 1).
__device__ __forceinline__ double ii_start(int i, int j) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u + (uint32_t)j * 0x85EBCA77u + 0x165667B1u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (double)h * 0x1p-31 - 1.0;
}

// Step 4, one wave (every lane calls it), for eigenvalue lam in lane j < M.  With finish false:
// the two solves from the pseudo-random start, normalised, as row j of Zr (row stride
// kSmallM + 1), and the cluster index of eigenvalue j in cid[j].  With finish true: from those
// rows, Gram-Schmidt within clusters and, where needed, one more solve and Gram-Schmidt;
// eigenvector j as column j of Zs (row-major, kSmallM columns).
__device__ void tridiag_eigvecs(int M, const double (&d)[kSmallM], const double (&e)[kSmallM], double lam,
                                double tnorm, double* Zr, double* Zs, double* bk, int* cid, bool finish) {
    constexpr int MB = kSmallM;
    constexpr double eps = 0x1p-52;
    const int lane = threadIdx.x & 63;
    double z[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) z[i] = (tnorm == 0.0 && i == lane) ? 1.0 : 0.0;
    if (tnorm > 0.0) {
        // LU with partial pivoting of T - lam I (lanes j < M; rows i, i+1 per step)
        const double epsp = eps * tnorm;
        double mul[MB], ru1[MB], u2[MB], u3[MB];
        uint32_t piv = 0;
        double u = d[0] - lam, v = e[0];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            mul[i] = 0.0;
            ru1[i] = 0.0;
            u2[i] = 0.0;
            u3[i] = 0.0;
            if (i < M - 1) {
                const double ei = e[i], ai1 = d[i + 1] - lam, ei1 = (i + 1 < MB) ? e[i + 1] : 0.0;
                const bool sw = fabs(u) < fabs(ei);
                const double den = sw ? ei : (u == 0.0 ? epsp : u);
                const double rden = rcp64(den);
                const double m = (sw ? u : ei) * rden;
                ru1[i] = rden;
                u2[i] = sw ? ai1 : v;
                u3[i] = sw ? ei1 : 0.0;
                const double nu = sw ? fma(-m, ai1, v) : fma(-m, v, ai1);
                v = sw ? -m * ei1 : ei1;
                u = nu;
                mul[i] = m;
                piv |= (uint32_t)sw << i;
            } else if (i == M - 1) {
                ru1[i] = rcp64(fabs(u) < epsp ? (u < 0.0 ? -epsp : epsp) : u);
            }
        }
        // x = (T - lam I)^-1 b for b scaled to unit max norm
        auto solve = [&](double (&x)[MB]) {
            double b[MB];
            double mx = 0.0;
#pragma unroll
            for (int i = 0; i < MB; ++i) mx = fmax(mx, fabs(x[i]));
            const double s = mx > 0.0 ? 1.0 / mx : 1.0;
#pragma unroll
            for (int i = 0; i < MB; ++i) b[i] = x[i] * s;
#pragma unroll
            for (int i = 0; i < MB - 1; ++i) {
                if (i < M - 1) {
                    const bool sw = (piv >> i) & 1u;
                    const double bi = b[i], bi1 = b[i + 1];
                    b[i] = sw ? bi1 : bi;
                    b[i + 1] = sw ? fma(-mul[i], bi1, bi) : fma(-mul[i], bi, bi1);
                }
            }
            double x1 = 0.0, x2 = 0.0;
#pragma unroll
            for (int i = MB - 1; i >= 0; --i) {
                if (i < M) {
                    const double xi = (b[i] - u2[i] * x1 - u3[i] * x2) * ru1[i];
                    x[i] = xi;
                    x2 = x1;
                    x1 = xi;
                } else {
                    x[i] = 0.0;
                }
            }
        };
        // dot products with four partial sums (MB is a multiple of 4)
        auto dot = [&](const double (&x)[MB], const double (&y)[MB]) {
            double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < MB; ++i) a[i & 3] = fma(x[i], y[i], a[i & 3]);
            return (a[0] + a[1]) + (a[2] + a[3]);
        };
        auto normalise = [&](double (&x)[MB]) {
            const double n2 = dot(x, x);
            const double r = n2 > 0.0 ? rsq_full(n2) : 0.0;
#pragma unroll
            for (int i = 0; i < MB; ++i) x[i] *= r;
        };
        // clusters: maximal runs of eigenvalues (ascending) less than 1e-3 ||T|| apart; bit k of
        // cend is set when eigenvalue k ends its cluster.  Vectors of different clusters are
        // orthogonal to about eps ||T|| / gap already, so Gram-Schmidt runs within clusters.
        const double lam_next = __shfl_down(lam, 1);
        const unsigned long long cend =
            __ballot(lane < M && (lane == M - 1 || lam_next - lam > 1e-3 * tnorm)) | (1ull << (M - 1));
        // Modified Gram-Schmidt within each cluster, in lane order, with four lanes per vector:
        // lane 4 j + g holds components 4 g .. 4 g + 3 of vector j (moved there through Zs, one
        // row per vector); the pivot vector reaches every lane through LDS (bk).  mix: the
        // largest |<z_k, z_j>| |lambda_j - lambda_k| removed from vector j (the change of its
        // eigen-residual); weak: a vector whose norm fell below 1/sqrt(2) before normalisation
        // (it was nearly dependent on the ones before it).
        const int jq = lane >> 2, g = lane & 3;
        const double lamq = __shfl(lam, jq);
        double zq[4];
        double mix = 0.0;
        bool weak = false;
        auto to_quads = [&]() {
            if (lane < M) {
#pragma unroll
                for (int i = 0; i < MB; ++i) Zr[lane * (MB + 1) + i] = z[i];
            }
            wave_sync();
#pragma unroll
            for (int t = 0; t < 4; ++t) zq[t] = Zr[jq * (MB + 1) + 4 * g + t];
            wave_sync();
        };
        auto from_quads = [&]() {
#pragma unroll
            for (int t = 0; t < 4; ++t) Zr[jq * (MB + 1) + 4 * g + t] = zq[t];
            wave_sync();
#pragma unroll
            for (int i = 0; i < MB; ++i) z[i] = Zr[lane * (MB + 1) + i];
            wave_sync();
        };
        auto mgs = [&]() {
            for (int k = 0; k < M; ++k) {
                if ((cend >> k) & 1ull) {            // last of its cluster: only normalised
                    if (jq == k) {
                        const double n2 = quad_sum(fma(zq[0], zq[0], fma(zq[1], zq[1], fma(zq[2], zq[2], zq[3] * zq[3]))));
                        weak |= n2 < 0.5;
                        const double rn = n2 > 0.0 ? rsq_full(n2) : 0.0;
#pragma unroll
                        for (int t = 0; t < 4; ++t) zq[t] *= rn;
                    }
                    continue;
                }
                const int ce = k + 2 + __builtin_ctzll(cend >> (k + 1));   // cluster end, exclusive
                if (jq == k) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) bk[4 * g + t] = zq[t];
                }
                wave_sync();
                double zk[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) zk[t] = bk[4 * g + t];
                const double n2 = quad_sum(fma(zk[0], zk[0], fma(zk[1], zk[1], fma(zk[2], zk[2], zk[3] * zk[3]))));
                const double lk = readlane_f64(lam, k);
                weak |= n2 < 0.5;
                const double rn = n2 > 0.0 ? rsq_full(n2) : 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) zk[t] *= rn;
                if (jq == k) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) zq[t] = zk[t];
                } else if (jq > k && jq < ce) {
                    const double dt = quad_sum(fma(zk[0], zq[0], fma(zk[1], zq[1], fma(zk[2], zq[2], zk[3] * zq[3]))));
                    mix = fmax(mix, fabs(dt) * fabs(lamq - lk));
#pragma unroll
                    for (int t = 0; t < 4; ++t) zq[t] = fma(-dt, zk[t], zq[t]);
                }
                wave_sync();
            }
        };
        if (!finish) {
            if (lane < M) {
#pragma unroll
                for (int i = 0; i < MB; ++i) z[i] = i < M ? ii_start(i, lane) : 0.0;
                solve(z);
                solve(z);
                normalise(z);
#pragma unroll
                for (int i = 0; i < MB; ++i) Zr[lane * (MB + 1) + i] = z[i];
            }
            if (lane < MB) cid[lane] = __builtin_popcountll(cend & ((1ull << lane) - 1ull));
            return;
        }
        if (lane < M) {
#pragma unroll
            for (int i = 0; i < MB; ++i) z[i] = Zr[lane * (MB + 1) + i];
        }
        to_quads();
        mgs();
        if (__ballot(jq < M && (weak || mix > 16.0 * epsp))) {
            from_quads();
            if (lane < M) {
                solve(z);
                normalise(z);
            }
            to_quads();
            mgs();
        }
        // Z[i][j] = component i of vector j
        if (jq < M) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * g + t < M) Zs[(4 * g + t) * MB + jq] = zq[t];
        }
    } else if (lane < MB) {
        // T = 0: the unit vectors, one cluster
        if (!finish) {
#pragma unroll
            for (int i = 0; i < MB; ++i) Zr[lane * (MB + 1) + i] = z[i];
            cid[lane] = 0;
        } else if (lane < M) {
#pragma unroll
            for (int i = 0; i < MB; ++i)
                if (i < M) Zs[i * MB + lane] = z[i];
        }
    }
}

struct Rot {
    int p, q;
    double c, s, t;   // t = tan * |r_pq|, the shift of the two diagonal entries
    double2 e;        // exp(-j arg r_pq)
};

// Pivot pair k of round-robin step `step` and its rotation, from the current matrix A.
// Position 0 holds index 0, position i >= 1 holds ((i - 1 + step) mod (Mp - 1)) + 1, and pair k
// joins positions k and Mp-1-k.  The rotation first removes the phase of r_pq, then applies
// [[c, s], [-s, c]] with t = sgn(theta) / (|theta| + sqrt(theta^2 + 1)),
// theta = (r_qq - r_pp) / (2 |r_pq|); it is the identity when |r_pq| is below threshold.
__device__ __forceinline__ Rot rotation(const double2* __restrict__ A, int ld, int M, int Mp, int step,
                                        int k, double tol2, double floor2) {
    const int n1 = Mp - 1;                       // 0 <= k - 1 + step < 2 (Mp - 1): no division
    int xa = k - 1 + step;
    xa -= (xa >= n1) ? n1 : 0;
    const int ia = (k == 0) ? 0 : xa + 1;
    int xb = n1 - k - 1 + step;
    xb -= (xb >= n1) ? n1 : 0;
    const int ib = xb + 1;
    Rot r;
    r.p = min(ia, ib);
    r.q = max(ia, ib);
    r.c = 1.0;
    r.s = 0.0;
    r.t = 0.0;
    r.e = make_double2(1.0, 0.0);
    if (r.q < M) {
        const double2 apq = A[r.p * ld + r.q];
        const double app = A[r.p * ld + r.p].x, aqq = A[r.q * ld + r.q].x;
        const double ab2 = apq.x * apq.x + apq.y * apq.y;
        if (ab2 > tol2 * fmax(fabs(app * aqq), floor2) && ab2 > 0.0) {
            const double rab = rsq64(ab2);
            r.e = make_double2(apq.x * rab, -apq.y * rab);
            const double th = 0.5 * (aqq - app) * rab;
            const double h = fma(th, th, 1.0);
            const double t = (th >= 0.0 ? 1.0 : -1.0) * rcp64(fabs(th) + h * rsq64(h));
            r.c = rsq64(fma(t, t, 1.0));
            r.s = t * r.c;
            r.t = t * (ab2 * rab);
        }
    }
    return r;
}

// A step's rotation as stored in LDS: one copy per wave, written by lanes 0..np-1.
struct RotL {
    double c, s, t, ex, ey;
    int32_t p, q;
};

__device__ __forceinline__ Rot load_rot(const RotL& x) {
    Rot r;
    r.p = x.p;
    r.q = x.q;
    r.c = x.c;
    r.s = x.s;
    r.t = x.t;
    r.e = make_double2(x.ex, x.ey);
    return r;
}

constexpr int kMaxTasksPerThread = 3;
constexpr int kMaxPairChecks = 2;   // off-diagonal pairs checked per thread and sweep

// Step-1 completion: R = (sum of chunk partials, in chunk order) / N, Hermitian by construction,
// into A (row stride ld, padded to Mp x Mp with zeros) and the workspace; `bad` is set when R is
// not finite.
__device__ void load_covariance(const FrameDev& fr, char* __restrict__ ws, double2* __restrict__ A, int ld,
                                int Mp, int* bad) {
    const int M = fr.M, tid = threadIdx.x, bd = blockDim.x;
    const double2* part = reinterpret_cast<const double2*>(ws + fr.ws_partial);
    double2* Rout = reinterpret_cast<double2*>(ws + fr.ws_R);
    const double dN = (double)fr.N;
    const int nch = fr.n_chunks;
    for (int e = tid; e < Mp * Mp; e += bd) {
        const int i = e / Mp, j = e - i * Mp;
        if (i < M && j < M) {
            if (i <= j) {
                double2 s = make_double2(0.0, 0.0);
                for (int c0 = 0; c0 < nch; c0 += 8) {
                    double2 v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        v[u] = (c0 + u < nch) ? part[(size_t)(c0 + u) * M * M + i * M + j] : make_double2(0.0, 0.0);
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        s.x += v[u].x;
                        s.y += v[u].y;
                    }
                }
                s.x = s.x / dN;
                s.y = (i == j) ? 0.0 : s.y / dN;
                if (!isfinite(s.x) || !isfinite(s.y)) *bad = 1;
                A[i * ld + j] = s;
                A[j * ld + i] = cconj(s);
                Rout[i * M + j] = s;
                Rout[j * M + i] = cconj(s);
            }
        } else {
            A[i * ld + j] = make_double2(0.0, 0.0);
        }
    }
}

// Everything after the eigenpairs: eigenvalue i is lamv[i * lstride] and its eigenvector column
// i of V (row stride ld).  Ranks the eigenvalues (Table 2 Step-2: descending, ties keep the lower
// index first), writes them and the eigenvectors, builds B (Table 3 Step-3/4) in Bs (LDS, M x K
// column-major, which must not overlap V; lamv is read before B is written), ||B||_F^2, the embedded operand tiles of the
// scan, and the frame status.  With bad set the outputs are NaN and B is zero.
__device__ void finish_frame(const FrameDev& fr, int fidx, const EvdParams& prm, const GroupDev* __restrict__ groups,
                             char* __restrict__ ws, uint32_t* __restrict__ status, const double* lamv, int lstride,
                             const double2* V, int ld, double2* Bs, int bad, uint32_t st, int* perm, double* lam,
                             double* red) {
    const int tid = threadIdx.x, bd = blockDim.x;
    const int M = fr.M, K = fr.K;
    double* evals = reinterpret_cast<double*>(ws + fr.ws_evals);
    double2* evecs = reinterpret_cast<double2*>(ws + fr.ws_evecs);
    double2* Bout = reinterpret_cast<double2*>(ws + fr.ws_B);
    double* qref = reinterpret_cast<double*>(ws + fr.ws_qref);
    double bmax = 0.0;                        // largest |Re|, |Im| of B (0 when bad: B is zero)
    if (bad) {
        st |= NSSDOA_ST_NONFINITE_INPUT;
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        for (int e = tid; e < M; e += bd) evals[e] = nan;
        for (int e = tid; e < M * M; e += bd) evecs[e] = make_double2(nan, nan);
        for (int e = tid; e < M * K; e += bd) Bs[e] = make_double2(0.0, 0.0);
        if (tid == 0) {
            *qref = nan;
            if (prm.write_emb == 2 || prm.write_emb == 3) qref[1] = nan;
        }
    } else {
        if (M <= 16 && bd >= 256) {
            // thread (i, j) = (tid / 16, tid % 16) compares eigenvalues i and j; the rank of i is
            // the count over its row of 16 lanes
            const int i = tid >> 4, j = tid & 15;
            const double li = i < M ? lamv[i * lstride] : 0.0, lj = j < M ? lamv[j * lstride] : 0.0;
            const unsigned long long bal = __ballot(i < M && j < M && (lj > li || (lj == li && j < i)));
            if (tid < 256 && i < M && j == 0) {
                perm[__builtin_popcount((uint32_t)(bal >> (tid & 48)) & 0xFFFFu)] = i;
                lam[i] = li;
            }
        } else if (tid < M) {
            const double li = lamv[tid * lstride];
            int r = 0;
            for (int j = 0; j < M; ++j) {
                const double lj = lamv[j * lstride];
                r += (lj > li) || (lj == li && j < tid);
            }
            perm[r] = tid;
            lam[tid] = li;
        }
        __syncthreads();
        for (int e = tid; e < M; e += bd) evals[e] = lam[perm[e]];
        for (int e = tid; e < M * M; e += bd) {
            const int i = e / M, r = e - i * M;
            evecs[e] = V[i * ld + perm[r]];
        }
        if (fr.alg == kMUSIC || fr.alg == kEV) {
            for (int e = tid; e < M * K; e += bd) {
                const int k = e / M, m = e - k * M;
                double2 v = V[m * ld + perm[fr.D + k]];
                if (fr.alg == kEV) {
                    const double l = lam[perm[fr.D + k]];
                    v = cscale(l > 0.0 ? 1.0 / sqrt(l) : 0.0, v);
                }
                Bs[e] = v;
            }
            // EV weights 1/sqrt(lambda): a noise eigenvalue at the rounding level of ||R|| (below
            // M 2^-52 lambda_1) is zero to working precision
            if (fr.alg == kEV && lam[perm[M - 1]] <= (double)M * 0x1p-52 * fmax(lam[perm[0]], 0.0))
                st |= NSSDOA_ST_DEGENERATE;
        } else if (fr.alg == kPHD) {
            for (int m = tid; m < M; m += bd) Bs[m] = V[m * ld + perm[M - 1]];
        } else {   // MN: d = P_n e_1 / (P_n)_11 with P_n = E_n E_n^H
            double pn11 = 0.0;
            for (int k = fr.D; k < M; ++k) {
                const double2 u0 = V[0 * ld + perm[k]];
                pn11 += u0.x * u0.x + u0.y * u0.y;
            }
            const bool degen = !(pn11 > 1e-300);
            if (degen) st |= NSSDOA_ST_DEGENERATE;
            for (int m = tid; m < M; m += bd) {
                double2 d = make_double2(0.0, 0.0);
                for (int k = fr.D; k < M; ++k) {
                    const double2 u0 = V[0 * ld + perm[k]];
                    d = cadd(d, cmul(V[m * ld + perm[k]], cconj(u0)));
                }
                Bs[m] = degen ? make_double2(0.0, 0.0) : cscale(1.0 / pn11, d);
            }
        }
        __syncthreads();
        double q = 0.0, mx = 0.0;
        for (int e = tid; e < M * K; e += bd) {
            q += Bs[e].x * Bs[e].x + Bs[e].y * Bs[e].y;
            mx = fmax(mx, fmax(fabs(Bs[e].x), fabs(Bs[e].y)));
        }
        block_sum_max(q, mx, red);
        bmax = mx;
        if (tid == 0) {
            *qref = q;
            // 16-bit scans: the Q below which a point is re-evaluated in FP64 at the least
            if (prm.write_emb == 2 || prm.write_emb == 3) qref[1] = lp_lowq_floor(M, K, q, prm.write_emb == 3);
        }
    }
    __syncthreads();
    for (int e = tid; e < M * K; e += bd) Bout[e] = Bs[e];

    if (prm.write_emb) {
        // Real embedding of B for the scan: column k gives two rows over the inner index
        // kk in [0, 2M):  re-row (Re b, Im b) and im-row (-Im b, Re b), so that the row dot the
        // embedded steering (Re a, Im a) is Re(b^H a) and Im(b^H a).  Rows are packed per 32-row
        // tile in the operand order of the scan's MFMA:
        //   FP32 (32x32x2):        lane h*32+i holds inner kk = 2s + h of row i as value s, stored
        //                          [M/4][64 lanes][4 values] so that lane-contiguous float4 reads
        //                          are conflict-free in LDS and coalesced in global memory;
        //   BF16/FP16 (32x32x16):  [64 lanes][M values], lane h*32+i holds inner kk = 16s + 8h + t
        //                          at position 8s + t;
        //   FP16 split (32x32x16): [part][M/8][64 lanes][8 values] with the lane mapping of the
        //                          16-bit tiles, part 0 = hi = fp16(2^e v), part 1 = lo =
        //                          fp16(2^e v - hi); 2^e puts the largest |component| of B in
        //                          [2^12, 2^13) and the scan's Q scale 2^-2e / 2^26 goes to qref[1].
        const GroupDev& g = groups[fr.group];
        const int rows = fr.emb_rows, inner = 2 * M;
        double bscale = 1.0;
        if (prm.write_emb >= 4) {
            const double mx = bmax;
            if (mx > 0.0 && isfinite(mx)) bscale = ldexp(1.0, 12 - ilogb(mx));
            if (tid == 0) {
                const double sab = (double)kSplitSteerScale * bscale;
                qref[1] = 1.0 / (sab * sab);
            }
        }
        if (prm.write_emb >= 4) {
            // FP16 split of P parts from the FP64 values: part p = fp16(x_p), x_(p+1) = x_p - part p
            // (exact in FP64); eight consecutive inner indices (one lane's 16-byte operand) per thread
            typedef _Float16 halfx8v __attribute__((ext_vector_type(8)));
            halfx8v* o8 = reinterpret_cast<halfx8v*>(ws + g.ws_emb);
            const int P = prm.write_emb == 5 ? 3 : 2;
            // half of a lane's operand (four inner indices) per thread
            typedef _Float16 halfx4v __attribute__((ext_vector_type(4)));
            halfx4v* o4 = reinterpret_cast<halfx4v*>(o8);
            for (int u2 = tid; u2 < rows * (inner / 4); u2 += bd) {
                const int u = u2 >> 1, hf = u2 & 1;
                const int rl = u / (inner / 8), kk0 = (u - rl * (inner / 8)) * 8;
                const int col = rl >> 1, re = kk0 < M, m0 = (re ? kk0 : kk0 - M) + 4 * hf;
                halfx4v part4[3];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    double vd = 0.0;
                    if (col < K) {
                        const double2 bv = Bs[col * M + m0 + t];
                        vd = (rl & 1) == 0 ? (re ? bv.x : bv.y) : (re ? -bv.y : bv.x);
                    }
                    vd *= bscale;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const _Float16 x = f64_to_f16(vd);
                        part4[q][t] = x;
                        vd -= (double)x;
                    }
                }
                const int r = fr.emb_row0 + rl, tile = r >> 5, i = r & 31;
                const size_t o0 = ((size_t)tile * P * (M / 8) + (kk0 >> 4)) * 64 + ((kk0 >> 3) & 1) * 32 + i;
                for (int q = 0; q < P; ++q) o4[2 * (o0 + (size_t)q * (M / 8) * 64) + hf] = part4[q];
            }
        } else
        for (int e = tid; e < rows * inner; e += bd) {
            const int rl = e / inner, kk = e - rl * inner;
            const int col = rl >> 1;
            float v = 0.0f;
            if (col < K) {
                const double2 b = Bs[col * M + (kk < M ? kk : kk - M)];
                if ((rl & 1) == 0) v = (float)(kk < M ? b.x : b.y);
                else v = (float)(kk < M ? -b.y : b.x);
            }
            const int r = fr.emb_row0 + rl;
            const int tile = r >> 5, i = r & 31;
            if (prm.write_emb == 1) {
                const int h = kk & 1, s2 = kk >> 1;
                reinterpret_cast<float*>(ws + g.ws_emb)[((size_t)tile * (M / 4) + (s2 >> 2)) * 256 +
                                                        (h * 32 + i) * 4 + (s2 & 3)] = v;
            } else {
                const int s16 = kk >> 4, h = (kk >> 3) & 1, t = kk & 7;
                const size_t o = ((size_t)tile * 64 + h * 32 + i) * M + s16 * 8 + t;
                if (prm.write_emb == 2) reinterpret_cast<__bf16*>(ws + g.ws_emb)[o] = (__bf16)v;
                else reinterpret_cast<_Float16*>(ws + g.ws_emb)[o] = (_Float16)v;
            }
        }
    }
    if (tid == 0) status[fidx] = st;
}

template <bool DB>
__global__ __launch_bounds__(DB ? 256 : 1024) void evd_kernel(const int32_t* __restrict__ flist,
                                                   const FrameDev* __restrict__ frames, EvdParams prm,
                                                   const GroupDev* __restrict__ groups,
                                                   char* __restrict__ ws,
                                                   uint32_t* __restrict__ status) {
    extern __shared__ double2 lds[];
    __shared__ int perm[64];
    __shared__ double red[32];
    __shared__ double lam[64];
    __shared__ int bad;

    const int fidx = flist[blockIdx.x];
    const FrameDev& fr = frames[fidx];
    const int tid = threadIdx.x, bd = blockDim.x;
    const int M = fr.M, Mp = M + (M & 1), ld = Mp + 1, np = Mp / 2;
    double2* A = lds;
    double2* V = lds + Mp * ld;
    double2* A2 = DB ? lds + 2 * Mp * ld : lds;   // second copy of A when double buffered
    RotL* rotw = reinterpret_cast<RotL*>(lds + (DB ? 3 : 2) * Mp * ld) + (threadIdx.x >> 6) * np;

    if (tid == 0) {
        bad = 0;
        if (prm.write_emb) *reinterpret_cast<int*>(ws + fr.ws_lowq) = 0;   // low-Q list of the scan
    }
    __syncthreads();
    load_covariance(fr, ws, A, ld, Mp, &bad);
    for (int e = tid; e < Mp * Mp; e += bd) {
        const int i = e / Mp, j = e - i * Mp;
        V[i * ld + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();

    uint32_t st = 0;
    if (!bad) {
        const double tol2 = prm.tol * prm.tol;
        // Entries below 1e-2 * tol * trace(R) are rounding noise of a positive semi-definite R:
        // the relative test r_pq^2 <= tol^2 r_pp r_qq is floored there so that exactly singular
        // R (N < M, noise-free models) still converges.
        double tr = 0.0;
        for (int e = tid; e < M; e += bd) tr += fabs(A[e * ld + e].x);
        tr = block_sum(tr, red);
        const double floor2 = (1e-2 * tr) * (1e-2 * tr);
        const int nA = np * np, nT = nA + Mp * np;
        // task coordinates of this thread, fixed for the whole solve: an A task is a 2x2 block
        // (pair k, pair l), a V task is (row i, pair l)
        int tk[kMaxTasksPerThread], tl[kMaxTasksPerThread];
#pragma unroll
        for (int u = 0; u < kMaxTasksPerThread; ++u) {
            const int task = tid + u * bd;
            if (task < nA) {
                tk[u] = task / np;
                tl[u] = task - tk[u] * np;
            } else {
                const int t2 = task - nA;
                tk[u] = t2 / np;
                tl[u] = t2 - tk[u] * np;
            }
        }
        // off-diagonal pairs (i < j) checked by this thread each sweep, indices fixed up front
        const int npairs = M * (M - 1) / 2;
        int ci[kMaxPairChecks], cj[kMaxPairChecks];
#pragma unroll
        for (int u = 0; u < kMaxPairChecks; ++u) {
            int t = tid + u * bd, i = 0;
            while (t >= M - 1 - i && i < M - 1) { t -= M - 1 - i; ++i; }
            ci[u] = i;
            cj[u] = i + 1 + t;
        }
        bool converged = false;
        for (int sweep = 0; sweep <= prm.max_iter; ++sweep) {
            int above = 0;
#pragma unroll
            for (int v = 0; v < kMaxPairChecks; ++v) {
                if (tid + v * bd < npairs) {
                    const int i = ci[v], j = cj[v];
                    const double2 a = A[i * ld + j];
                    const double num = a.x * a.x + a.y * a.y;
                    above |= num > tol2 * fmax(fabs(A[i * ld + i].x * A[j * ld + j].x), floor2);
                }
            }
            if (!__syncthreads_or(above)) {
                converged = true;
                break;
            }
            if (sweep == prm.max_iter) break;
            for (int step = 0; step < Mp - 1; ++step) {
                // The step's np rotations from the current A, one copy per wave (no block-wide
                // barrier: each wave reads only its own copy).
                if ((tid & 63) < np) {
                    const Rot r = rotation(A, ld, M, Mp, step, tid & 63, tol2, floor2);
                    RotL& o = rotw[tid & 63];
                    o.c = r.c;
                    o.s = r.s;
                    o.t = r.t;
                    o.ex = r.e.x;
                    o.ey = r.e.y;
                    o.p = r.p;
                    o.q = r.q;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // Each task reads the rotations it needs, reads its block and computes the new
                // values.  Double buffered: written at once to the other copy.  In place: kept in
                // registers until every thread has read, then written.
                double2 keep[kMaxTasksPerThread][4];
                int kp[kMaxTasksPerThread][4];
#pragma unroll
                for (int u = 0; u < kMaxTasksPerThread; ++u) {
                    const int task = tid + u * bd;
                    if (task < nA) {
                        const int k = tk[u], l = tl[u];
                        const Rot r1 = load_rot(rotw[k]);
                        const Rot r2 = (l == k) ? r1 : load_rot(rotw[l]);
                        const double2 b11 = A[r1.p * ld + r2.p], b12 = A[r1.p * ld + r2.q];
                        const double2 b21 = A[r1.q * ld + r2.p], b22 = A[r1.q * ld + r2.q];
                        double2 o11, o12, o21, o22;
                        if (k == l) {
                            // diagonal block: the rotation annihilates r_pq exactly
                            if (r1.s == 0.0) {
                                o11 = b11; o12 = b12; o21 = b21; o22 = b22;
                            } else {
                                o11 = make_double2(b11.x - r1.t, 0.0);
                                o22 = make_double2(b22.x + r1.t, 0.0);
                                o12 = make_double2(0.0, 0.0);
                                o21 = o12;
                            }
                        } else {
                            // right: B J_l with J = [[c, s], [-s e, c e]]
                            const double2 se2 = cscale(r2.s, r2.e), ce2 = cscale(r2.c, r2.e);
                            const double2 x11 = csub(cscale(r2.c, b11), cmul(b12, se2));
                            const double2 x12 = cadd(cscale(r2.s, b11), cmul(b12, ce2));
                            const double2 x21 = csub(cscale(r2.c, b21), cmul(b22, se2));
                            const double2 x22 = cadd(cscale(r2.s, b21), cmul(b22, ce2));
                            // left: J_k^H (B J_l) with J^H = [[c, -s conj(e)], [s, c conj(e)]]
                            const double2 se1 = cscale(r1.s, cconj(r1.e)), ce1 = cscale(r1.c, cconj(r1.e));
                            o11 = csub(cscale(r1.c, x11), cmul(se1, x21));
                            o12 = csub(cscale(r1.c, x12), cmul(se1, x22));
                            o21 = cadd(cscale(r1.s, x11), cmul(ce1, x21));
                            o22 = cadd(cscale(r1.s, x12), cmul(ce1, x22));
                        }
                        if (DB) {
                            A2[r1.p * ld + r2.p] = o11;
                            A2[r1.p * ld + r2.q] = o12;
                            A2[r1.q * ld + r2.p] = o21;
                            A2[r1.q * ld + r2.q] = o22;
                        } else {
                            keep[u][0] = o11; keep[u][1] = o12; keep[u][2] = o21; keep[u][3] = o22;
                            kp[u][0] = r1.p * ld + r2.p; kp[u][1] = r1.p * ld + r2.q;
                            kp[u][2] = r1.q * ld + r2.p; kp[u][3] = r1.q * ld + r2.q;
                        }
                    } else if (task < nT) {
                        // V <- V J_l on row i: no other task touches these two entries this step
                        const int i = tk[u], l = tl[u];
                        const Rot r = load_rot(rotw[l]);
                        const double2 v1 = V[i * ld + r.p], v2 = V[i * ld + r.q];
                        V[i * ld + r.p] = csub(cscale(r.c, v1), cmul(v2, cscale(r.s, r.e)));
                        V[i * ld + r.q] = cadd(cscale(r.s, v1), cmul(v2, cscale(r.c, r.e)));
                    }
                }
                if (!DB) {
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < kMaxTasksPerThread; ++u) {
                        if (tid + u * bd < nA) {
#pragma unroll
                            for (int w = 0; w < 4; ++w) A[kp[u][w]] = keep[u][w];
                        }
                    }
                }
                __syncthreads();
                if (DB) {
                    double2* t = A;
                    A = A2;
                    A2 = t;
                }
            }
        }
        if (!converged) st |= NSSDOA_ST_EVD_NOT_CONVERGED;
    }
    __syncthreads();
    // eigenvalue i = A[i][i].x; B is staged over the first copy of A (finish_frame reads the
    // eigenvalues before it writes B)
    finish_frame(fr, fidx, prm, groups, ws, status, &A[0].x, 2 * (ld + 1), V, ld, lds, bad, st, perm, lam, red);
}

// Householder tridiagonalisation, implicit QL and back-transformation.  LDS: region 0
// (Mp x ld complex) holds R, then Z (real values in .x), then V = Q Z; region 1 holds v_k in
// column k, rows k+1..M-1, and later B.
__global__ __launch_bounds__(256) void evd_ql_kernel(const int32_t* __restrict__ flist,
                                                     const FrameDev* __restrict__ frames, EvdParams prm,
                                                     const GroupDev* __restrict__ groups,
                                                     char* __restrict__ ws,
                                                     uint32_t* __restrict__ status) {
    extern __shared__ double2 lds[];
    __shared__ int perm[64];
    __shared__ double red[32];
    __shared__ double lam[64];
    __shared__ double dq[64], eq[64];      // diagonal and off-diagonal of T (eq[i] couples i, i+1)
    __shared__ double2 tq[64];             // tau_k
    __shared__ double2 vb[64], wb[64];     // the current reflector v and the vector w of its update
    __shared__ int bad;

    const int fidx = flist[blockIdx.x];
    const FrameDev& fr = frames[fidx];
    const int tid = threadIdx.x, bd = blockDim.x;
    const int M = fr.M, Mp = M + (M & 1), ld = Mp + 1;
    double2* A = lds;
    double2* Hv = lds + Mp * ld;

    if (tid == 0) {
        bad = 0;
        if (prm.write_emb) *reinterpret_cast<int*>(ws + fr.ws_lowq) = 0;   // low-Q list of the scan
    }
    __syncthreads();
    load_covariance(fr, ws, A, ld, Mp, &bad);
    __syncthreads();

    uint32_t st = 0;
    // four lanes per matrix row (or column) in the parallel phases
    const int grp = tid >> 2, q = tid & 3, gstep = bd >> 2;
    if (!bad) {
        // T = Q^H R Q.  Step k reflects rows/columns k+1..M-1 so that column k below the
        // subdiagonal vanishes and the subdiagonal entry becomes the real beta.
        for (int k = 0; k < M - 1; ++k) {
            const int m = M - 1 - k;
            const double2* col = A + (k + 1) * ld + k;          // col[i * ld] = A[k+1+i][k]
            double part = 0.0;
            for (int i = 1 + tid; i < m; i += bd) {
                const double2 x = col[i * ld];
                part = fma(x.x, x.x, fma(x.y, x.y, part));
            }
            const double xn2 = block_sum_fast(part, red);
            const double2 alpha = col[0];
            double beta = alpha.x;
            double2 tau = make_double2(0.0, 0.0), scl = make_double2(0.0, 0.0);
            if (xn2 > 0.0 || alpha.y != 0.0) {
                // beta = -sgn(Re alpha) ||(alpha, x)||, tau = (beta - alpha) / beta,
                // v = (1, x / (alpha - beta)): then H^H (alpha, x) = (beta, 0)
                beta = -copysign(sqrt(fma(alpha.x, alpha.x, fma(alpha.y, alpha.y, xn2))), alpha.x);
                tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                const double2 den = make_double2(alpha.x - beta, alpha.y);
                const double dn2 = fma(den.x, den.x, den.y * den.y);
                scl = make_double2(den.x / dn2, -den.y / dn2);
            }
            for (int i = tid; i < m; i += bd) {
                const double2 v = (i == 0) ? make_double2(1.0, 0.0) : cmul(col[i * ld], scl);
                Hv[(k + 1 + i) * ld + k] = v;
                vb[i] = v;
            }
            if (tid == 0) {
                dq[k] = A[k * ld + k].x;
                eq[k] = beta;
                tq[k] = tau;
            }
            __syncthreads();
            if (tau.x == 0.0 && tau.y == 0.0) continue;        // uniform: H_k = I
            // y = B v for the trailing block B, gamma = v^H y (real), w = tau y - |tau|^2 gamma / 2 v
            double gp = 0.0;
            for (int r = grp; r < m; r += gstep) {
                const double2* arow = A + (k + 1 + r) * ld + k + 1;
                double2 acc = make_double2(0.0, 0.0);
                for (int j = q; j < m; j += 4) {
                    const double2 a = arow[j], v = vb[j];
                    acc.x = fma(a.x, v.x, fma(-a.y, v.y, acc.x));
                    acc.y = fma(a.x, v.y, fma(a.y, v.x, acc.y));
                }
                acc.x = quad_sum(acc.x);
                acc.y = quad_sum(acc.y);
                if (q == 0) {
                    const double2 v = vb[r];
                    gp = fma(v.x, acc.x, fma(v.y, acc.y, gp));
                    wb[r] = acc;
                }
            }
            const double gam = block_sum_fast(gp, red);
            const double h = 0.5 * fma(tau.x, tau.x, tau.y * tau.y) * gam;
            for (int r = grp; r < m; r += gstep) {
                if (q == 0) wb[r] = csub(cmul(tau, wb[r]), cscale(h, vb[r]));
            }
            __syncthreads();
            // B -= v w^H + w v^H
            for (int r = grp; r < m; r += gstep) {
                const double2 vi = vb[r], wi = wb[r];
                double2* arow = A + (k + 1 + r) * ld + k + 1;
                for (int j = q; j < m; j += 4) {
                    const double2 vj = vb[j], wj = wb[j];
                    double2 a = arow[j];
                    a.x -= fma(vi.x, wj.x, vi.y * wj.y) + fma(wi.x, vj.x, wi.y * vj.y);
                    a.y -= fma(vi.y, wj.x, -vi.x * wj.y) + fma(wi.y, vj.x, -wi.x * vj.y);
                    arow[j] = a;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            dq[M - 1] = A[(M - 1) * ld + M - 1].x;
            eq[M - 1] = 0.0;
        }
        __syncthreads();
        for (int e = tid; e < Mp * Mp; e += bd) {
            const int i = e / Mp, j = e - i * Mp;
            A[i * ld + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);      // Z = I
        }
        __syncthreads();

        // Implicit QL on (dq, eq) in the first M lanes of wave 0.  Lane j keeps d_j and e_j in
        // registers (the others read them with readlane) and row j of Z in LDS; every lane runs
        // the rotation chain, whose values are uniform.
        if (tid < M) {
            const int lane = tid;
            double dl = dq[lane], el = eq[lane];
            double2* zrow = A + lane * ld;
            const double tol = prm.tol;
            for (int l = 0; l < M; ++l) {
                for (int it = 0;; ++it) {
                    // the block [l, m]: m is the first index >= l whose e_m is negligible
                    const double dnx = __shfl_down(dl, 1);
                    const bool split = (lane == M - 1) || fabs(el) <= tol * (fabs(dl) + fabs(dnx));
                    const unsigned long long bal = __ballot(split && lane >= l);
                    const int m = __builtin_ctzll(bal);
                    if (m == l) break;
                    if (it == prm.max_iter) {
                        st |= NSSDOA_ST_EVD_NOT_CONVERGED;
                        break;
                    }
                    // shift: the eigenvalue of the leading 2x2 of the block nearer to d_l (its
                    // precision only affects the convergence rate)
                    const double d_l = readlane_f64(dl, l), e_l = readlane_f64(el, l);
                    const double d_m = readlane_f64(dl, m);
                    double g = (readlane_f64(dl, l + 1) - d_l) * rcp_approx(2.0 * e_l);
                    const double g21 = fma(g, g, 1.0);
                    double r = g21 * rsq_full(g21);
                    g = d_m - d_l + e_l * rcp_approx(g + copysign(r, g));
                    double s = 1.0, c = 1.0, p = 0.0;
                    int i = m - 1;
                    double di1 = d_m, di = readlane_f64(dl, i), ei = readlane_f64(el, i);
                    double zc = zrow[m].x, zi = zrow[i].x;   // column i+1 (carried) and column i
                    bool early = false;
                    for (; i >= l; --i) {
                        const int in = i > 0 ? i - 1 : 0;      // the next rotation's index
                        const double dn = readlane_f64(dl, in), en = readlane_f64(el, in);
                        const double zn = zrow[in].x;
                        const double f = s * ei, b = c * ei;
                        const double t = fma(f, f, g * g);
                        if (t == 0.0) {
                            early = true;
                            break;
                        }
                        const double rr = rsq_full(t);
                        const double enew = t * rr;
                        s = f * rr;
                        c = g * rr;
                        g = di1 - p;
                        r = fma(di - g, s, 2.0 * c * b);
                        p = s * r;
                        const double dnew = g + p;
                        g = fma(c, r, -b);
                        el = (lane == i + 1) ? enew : el;
                        dl = (lane == i + 1) ? dnew : dl;
                        zrow[i + 1].x = fma(s, zi, c * zc);
                        zc = fma(c, zi, -s * zc);
                        di1 = di;
                        di = dn;
                        ei = en;
                        zi = zn;
                    }
                    zrow[i + 1].x = zc;
                    if (early) {                                // the chase vanished: restart
                        dl = (lane == i + 1) ? di1 - p : dl;
                        el = (lane == m) ? 0.0 : el;
                        continue;
                    }
                    dl = (lane == l) ? di1 - p : dl;
                    el = (lane == l) ? g : (lane == m) ? 0.0 : el;
                }
            }
            dq[lane] = dl;
        }
        __syncthreads();

        // V = H_0 (H_1 (... H_{M-2} Z)); H_k Z = Z - tau_k v_k (v_k^H Z).  Four lanes own one
        // column of Z for all reflectors, so no barrier is needed between them.
        for (int j = grp; j < M; j += gstep) {
            for (int k = M - 2; k >= 0; --k) {
                const double2 tau = tq[k];
                if (tau.x == 0.0 && tau.y == 0.0) continue;
                const int m = M - 1 - k;
                double2 sa = make_double2(0.0, 0.0);
                for (int i = q; i < m; i += 4) {
                    const double2 v = Hv[(k + 1 + i) * ld + k], z = A[(k + 1 + i) * ld + j];
                    sa.x = fma(v.x, z.x, fma(v.y, z.y, sa.x));
                    sa.y = fma(v.x, z.y, fma(-v.y, z.x, sa.y));
                }
                sa.x = quad_sum(sa.x);
                sa.y = quad_sum(sa.y);
                const double2 ts = cmul(tau, sa);
                for (int i = q; i < m; i += 4) {
                    const double2 v = Hv[(k + 1 + i) * ld + k];
                    A[(k + 1 + i) * ld + j] = csub(A[(k + 1 + i) * ld + j], cmul(v, ts));
                }
            }
        }
        __syncthreads();
    }
    finish_frame(fr, fidx, prm, groups, ws, status, dq, 1, A, ld, Hv, bad, st, perm, lam, red);
}

// The default solver for M <= kSmallM: four waves per frame (see the description of steps 1-5
// above).  LDS: R and then Q and V (row stride kSmallM + 1), Z, B.
__global__ __launch_bounds__(kSmallThreads) void evd_small_kernel(const int32_t* __restrict__ flist,
                                                                  const FrameDev* __restrict__ frames, EvdParams prm,
                                                                  const GroupDev* __restrict__ groups,
                                                                  char* __restrict__ ws,
                                                                  uint32_t* __restrict__ status) {
    constexpr int MB = kSmallM, ld = kSmallM + 1;
    __shared__ double2 As[MB * ld];
    __shared__ double2 Bs[MB * MB];
    __shared__ double Zs[MB * MB];
    __shared__ double Zr[MB * (MB + 1)];
    __shared__ double Es[MB * MB];
    __shared__ int cid[MB];
    __shared__ double2 ubuf[MB], ybuf[MB], sc[2];
    __shared__ double dq[MB], eq[MB], lamv[MB], gpart[4], bk[MB];
    __shared__ int first[64];
    __shared__ int perm[64];
    __shared__ double red[32];
    __shared__ double lam[64];
    __shared__ int bad;

    const int fidx = flist[blockIdx.x];
    const FrameDev& fr = frames[fidx];
    const int tid = threadIdx.x, r = tid >> 4, c = tid & 15;
    const int M = fr.M;
    if (tid == 0) {
        bad = 0;
        if (prm.write_emb) *reinterpret_cast<int*>(ws + fr.ws_lowq) = 0;   // low-Q list of the scan
    }
    __syncthreads();
    load_covariance(fr, ws, As, ld, MB, &bad);
    __syncthreads();
    if (!bad) {
        double2 qm;
        tridiag_block(M, As, ld, dq, eq, ubuf, ybuf, sc, gpart, qm);
        __syncthreads();
        // Q over R (R is no longer read)
        if (r < M && c < M) As[r * ld + c] = qm;
        double d[MB], e[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            d[i] = i < M ? dq[i] : 0.0;
            e[i] = i < M - 1 ? eq[i] : 0.0;
        }
        const double tnorm = eigvals_block(M, d, e, lamv, first);
        __syncthreads();
        const double lj = tid < M ? lamv[tid] : 0.0;
        if (tid < 64) tridiag_eigvecs(M, d, e, lj, tnorm, Zr, Zs, bk, cid, false);
        __syncthreads();
        // Orthonormalisation within clusters in one symmetric step: with the Gram matrix
        // G = I + E of a cluster's vectors, z_j <- z_j - 1/2 sum_k E_jk z_k is Z (I + E)^(-1/2) up
        // to O(|E|^2), taken when every |E_jk| <= 1e-10 and |E_jk| |lambda_j - lambda_k| <=
        // 16 eps ||T|| (the change of the eigen-residuals); otherwise the wave runs Gram-Schmidt.
        {
            const int j = r, k = c;
            double ejk = 0.0;
            bool far = false;
            if (j < M && k < M && cid[j] == cid[k]) {
                double gjk = 0.0;
#pragma unroll
                for (int i = 0; i < MB; ++i) gjk = fma(Zr[j * (MB + 1) + i], Zr[k * (MB + 1) + i], gjk);
                ejk = (j == k) ? gjk - 1.0 : gjk;
                if (j != k)
                    far = !(fabs(ejk) <= 1e-10) ||
                          !(fabs(ejk) * fabs(lamv[j] - lamv[k]) <= 16.0 * 0x1p-52 * tnorm);
            }
            Es[j * MB + k] = ejk;
            if (__syncthreads_or(far)) {
                if (tid < 64) tridiag_eigvecs(M, d, e, lj, tnorm, Zr, Zs, bk, cid, true);
            } else if (j < M && k < M) {
                // thread (j, i = c): component i of the corrected vector j
                double zv = Zr[j * (MB + 1) + k];
                double corr = 0.0;
                for (int kk = 0; kk < M; ++kk) corr = fma(Es[j * MB + kk], Zr[kk * (MB + 1) + k], corr);
                Zs[k * MB + j] = fma(-0.5, corr, zv);
            }
        }
        __syncthreads();
        // V = Q Z (Z real), over Q
        double2 v = make_double2(0.0, 0.0);
        if (r < M && c < M) {
            for (int i = 0; i < M; ++i) {
                const double2 qi = As[r * ld + i];
                const double zt = Zs[i * MB + c];
                v.x = fma(qi.x, zt, v.x);
                v.y = fma(qi.y, zt, v.y);
            }
        }
        __syncthreads();
        if (r < M && c < M) As[r * ld + c] = v;
        __syncthreads();
    }
    finish_frame(fr, fidx, prm, groups, ws, status, lamv, 1, As, ld, Bs, bad, 0u, perm, lam, red);
}

}  // namespace

hipError_t launch_evd(const int32_t* frame_list, int n_frames, int max_M, const EvdParams& p,
                      const FrameDev* frames, const GroupDev* groups, char* ws, uint32_t* status,
                      hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    if (max_M < 2 || max_M > 64) return hipErrorInvalidValue;
    const int Mp = max_M + (max_M & 1);
    if (p.method == NSSDOA_EIG_AUTO && max_M <= kSmallM) {
        hipLaunchKernelGGL(evd_small_kernel, dim3(n_frames), dim3(kSmallThreads), 0, s, frame_list, frames, p, groups,
                           ws, status);
        return hipGetLastError();
    }
    if (p.method != NSSDOA_EIG_JACOBI) {
        const int threads = max_M <= 16 ? 64 : max_M <= 32 ? 128 : 256;
        const size_t lds = (size_t)2 * Mp * (Mp + 1) * sizeof(double2);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)evd_ql_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(evd_ql_kernel, dim3(n_frames), dim3(threads), lds, s, frame_list, frames, p, groups, ws,
                           status);
        return hipGetLastError();
    }
    // Jacobi: one thread per 2x2 block update and per V row-pair update of a step:
    // 3 Mp^2 / 4 tasks, at most kMaxTasksPerThread per thread
    const int tasks = 3 * Mp * Mp / 4;
    const bool db = Mp <= 32;     // a second copy of A fits in LDS: one barrier per step
    const int threads = std::min(db ? 256 : 1024, std::max(64, (tasks + 63) / 64 * 64));
    if (tasks > threads * kMaxTasksPerThread) return hipErrorInvalidValue;
    if (max_M * (max_M - 1) / 2 > threads * kMaxPairChecks) return hipErrorInvalidValue;
    const size_t lds = (size_t)(db ? 3 : 2) * Mp * (Mp + 1) * sizeof(double2) +
                       (size_t)(threads / 64) * (Mp / 2) * sizeof(RotL);
    const void* fn = db ? (const void*)evd_kernel<true> : (const void*)evd_kernel<false>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (db)
        hipLaunchKernelGGL(evd_kernel<true>, dim3(n_frames), dim3(threads), lds, s, frame_list, frames, p,
                           groups, ws, status);
    else
        hipLaunchKernelGGL(evd_kernel<false>, dim3(n_frames), dim3(threads), lds, s, frame_list, frames, p,
                           groups, ws, status);
    return hipGetLastError();
}

}  // namespace nssdoa
