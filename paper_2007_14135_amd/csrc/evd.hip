// Steps 2-4 (Table 2 Step-2, Table 3): FP64 Hermitian eigendecomposition by cyclic Jacobi and
// the noise-subspace matrix B with C = B B^H.
//
// One workgroup per frame.  The workgroup first adds the frame's partial covariances in chunk
// order and divides by N (Eq. 3), then diagonalises R in LDS with complex Jacobi rotations in
// round-robin order: M/2 disjoint pivot pairs per step, M-1 steps per sweep, so every step is
// one fully parallel two-sided update of the 2x2 blocks of A and one update of V.  A rotation
// for pivot (p, q) first removes the phase of r_pq with diag(1, exp(-j arg r_pq)) and then
// applies the real rotation [[c, s], [-s, c]] with t = sgn(theta) / (|theta| + sqrt(theta^2+1)),
// theta = (r_qq - r_pp) / (2 |r_pq|).  Sweeps stop when every |r_pq| <= tol * sqrt(r_pp r_qq),
// the relative criterion that keeps small (noise) eigenvalues accurate.  Eigenvalues are then
// ranked in descending order and B is built for the requested method, in FP64 and (for the FP32
// scan) as the packed real-embedded FP32 operand tiles of the scan kernel.
#include <float.h>

#include "nssdoa.h"
#include "internal.h"

namespace nssdoa {
namespace {

constexpr int kMaxPairs = 32;

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ inline double block_max(double v, double* red) {
    const int tid = threadIdx.x, bd = blockDim.x;
    red[tid] = v;
    __syncthreads();
    for (int s = bd >> 1; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline double block_sum(double v, double* red) {
    const int tid = threadIdx.x, bd = blockDim.x;
    red[tid] = v;
    __syncthreads();
    for (int s = bd >> 1; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void evd_kernel(const FrameDev* __restrict__ frames, EvdParams prm,
                                                  const GroupDev* __restrict__ groups,
                                                  char* __restrict__ ws,
                                                  uint32_t* __restrict__ status) {
    extern __shared__ double2 lds[];
    __shared__ int pr[kMaxPairs], qr[kMaxPairs], perm[64];
    __shared__ double rc[kMaxPairs], rs[kMaxPairs], rt[kMaxPairs];
    __shared__ double2 re[kMaxPairs];
    __shared__ double red[256];
    __shared__ int bad;

    const FrameDev& fr = frames[blockIdx.x];
    const int tid = threadIdx.x, bd = blockDim.x;
    const int M = fr.M, Mp = M + (M & 1), ld = Mp + 1, np = Mp / 2;
    double2* A = lds;
    double2* V = lds + Mp * ld;

    if (tid == 0) bad = 0;
    __syncthreads();

    // Step-1 completion: R = (sum of chunk partials) / N, Hermitian by construction.
    const double2* part = reinterpret_cast<const double2*>(ws + fr.ws_partial);
    double2* Rout = reinterpret_cast<double2*>(ws + fr.ws_R);
    const double dN = (double)fr.N;
    for (int e = tid; e < Mp * Mp; e += bd) {
        const int i = e / Mp, j = e - i * Mp;
        V[i * ld + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        if (i < M && j < M) {
            if (i <= j) {
                double2 s = make_double2(0.0, 0.0);
                for (int c = 0; c < fr.n_chunks; ++c) {
                    double2 v = part[(size_t)c * M * M + i * M + j];
                    s.x += v.x;
                    s.y += v.y;
                }
                s.x = s.x / dN;
                s.y = (i == j) ? 0.0 : s.y / dN;
                if (!isfinite(s.x) || !isfinite(s.y)) bad = 1;
                A[i * ld + j] = s;
                A[j * ld + i] = cconj(s);
                Rout[i * M + j] = s;
                Rout[j * M + i] = cconj(s);
            }
        } else {
            A[i * ld + j] = make_double2(0.0, 0.0);
        }
    }
    __syncthreads();

    uint32_t st = 0;
    const int K = fr.K;
    double* evals = reinterpret_cast<double*>(ws + fr.ws_evals);
    double2* evecs = reinterpret_cast<double2*>(ws + fr.ws_evecs);
    double2* Bout = reinterpret_cast<double2*>(ws + fr.ws_B);
    double* qref = reinterpret_cast<double*>(ws + fr.ws_qref);
    double2* Bs = A;   // B is staged over A once the eigenpairs are extracted

    if (bad) {
        st |= NSSDOA_ST_NONFINITE_INPUT;
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        for (int e = tid; e < M; e += bd) evals[e] = nan;
        for (int e = tid; e < M * M; e += bd) evecs[e] = make_double2(nan, nan);
        __syncthreads();
        for (int e = tid; e < M * K; e += bd) Bs[e] = make_double2(0.0, 0.0);
        if (tid == 0) *qref = nan;
    } else {
        const double tol2 = prm.tol * prm.tol;
        // Entries below 1e-2 * tol * trace(R) are rounding noise of a positive semi-definite R:
        // the relative test r_pq^2 <= tol^2 r_pp r_qq is floored there so that exactly singular
        // R (N < M, noise-free models) still converges.
        double tr = 0.0;
        for (int e = tid; e < M; e += bd) tr += fabs(A[e * ld + e].x);
        tr = block_sum(tr, red);
        const double floor2 = (1e-2 * tr) * (1e-2 * tr);
        bool converged = false;
        for (int sweep = 0; sweep <= prm.max_sweeps; ++sweep) {
            // relative off-diagonal size: max |r_pq|^2 / max(r_pp r_qq, floor^2)
            double mx = 0.0;
            for (int e = tid; e < M * M; e += bd) {
                const int i = e / M, j = e - i * M;
                if (i < j) {
                    const double2 a = A[i * ld + j];
                    const double den = fmax(fabs(A[i * ld + i].x * A[j * ld + j].x), floor2);
                    const double num = a.x * a.x + a.y * a.y;
                    const double r = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
                    mx = fmax(mx, r);
                }
            }
            mx = block_max(mx, red);
            if (mx <= tol2) {
                converged = true;
                break;
            }
            if (sweep == prm.max_sweeps) break;
            for (int step = 0; step < Mp - 1; ++step) {
                if (tid < np) {
                    // round-robin: position 0 holds index 0, position i >= 1 holds
                    // ((i - 1 + step) mod (Mp - 1)) + 1; pair k joins positions k and Mp-1-k.
                    const int k = tid;
                    const int ia = (k == 0) ? 0 : ((k - 1 + step) % (Mp - 1)) + 1;
                    const int kb = Mp - 1 - k;
                    const int ib = ((kb - 1 + step) % (Mp - 1)) + 1;
                    const int p = min(ia, ib), q = max(ia, ib);
                    pr[k] = p;
                    qr[k] = q;
                    double c = 1.0, s = 0.0, t = 0.0;
                    double2 e = make_double2(1.0, 0.0);
                    if (q < M) {
                        const double2 apq = A[p * ld + q];
                        const double app = A[p * ld + p].x, aqq = A[q * ld + q].x;
                        const double ab = hypot(apq.x, apq.y);
                        if (ab > prm.tol * sqrt(fmax(fabs(app * aqq), floor2)) && ab > 0.0) {
                            e = make_double2(apq.x / ab, -apq.y / ab);     // exp(-j arg r_pq)
                            const double th = (aqq - app) / (2.0 * ab);
                            t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                            c = 1.0 / sqrt(1.0 + t * t);
                            s = t * c;
                            t = t * ab;
                        }
                    }
                    rc[k] = c;
                    rs[k] = s;
                    rt[k] = t;
                    re[k] = e;
                }
                __syncthreads();
                const int nA = np * np, nV = Mp * np;
                for (int task = tid; task < nA + nV; task += bd) {
                    if (task < nA) {
                        const int k = task / np, l = task - k * np;
                        const int p1 = pr[k], q1 = qr[k];
                        if (k == l) {
                            if (rs[k] != 0.0) {
                                A[p1 * ld + p1] = make_double2(A[p1 * ld + p1].x - rt[k], 0.0);
                                A[q1 * ld + q1] = make_double2(A[q1 * ld + q1].x + rt[k], 0.0);
                                A[p1 * ld + q1] = make_double2(0.0, 0.0);
                                A[q1 * ld + p1] = make_double2(0.0, 0.0);
                            }
                        } else {
                            const int p2 = pr[l], q2 = qr[l];
                            const double c1 = rc[k], s1 = rs[k], c2 = rc[l], s2 = rs[l];
                            const double2 e1 = re[k], e2 = re[l];
                            const double2 b11 = A[p1 * ld + p2], b12 = A[p1 * ld + q2];
                            const double2 b21 = A[q1 * ld + p2], b22 = A[q1 * ld + q2];
                            // right: B J_l, J = [[c, s], [-s e, c e]]
                            const double2 se2 = cscale(s2, e2), ce2 = cscale(c2, e2);
                            const double2 r11 = csub(cscale(c2, b11), cmul(b12, se2));
                            const double2 r12 = cadd(cscale(s2, b11), cmul(b12, ce2));
                            const double2 r21 = csub(cscale(c2, b21), cmul(b22, se2));
                            const double2 r22 = cadd(cscale(s2, b21), cmul(b22, ce2));
                            // left: J_k^H (B J_l), J^H = [[c, -s conj(e)], [s, c conj(e)]]
                            const double2 se1 = cscale(s1, cconj(e1)), ce1 = cscale(c1, cconj(e1));
                            A[p1 * ld + p2] = csub(cscale(c1, r11), cmul(se1, r21));
                            A[p1 * ld + q2] = csub(cscale(c1, r12), cmul(se1, r22));
                            A[q1 * ld + p2] = cadd(cscale(s1, r11), cmul(ce1, r21));
                            A[q1 * ld + q2] = cadd(cscale(s1, r12), cmul(ce1, r22));
                        }
                    } else {
                        const int t2 = task - nA;
                        const int i = t2 / np, l = t2 - i * np;
                        const int p = pr[l], q = qr[l];
                        const double c = rc[l], s = rs[l];
                        const double2 e = re[l];
                        const double2 v1 = V[i * ld + p], v2 = V[i * ld + q];
                        V[i * ld + p] = csub(cscale(c, v1), cmul(v2, cscale(s, e)));
                        V[i * ld + q] = cadd(cscale(s, v1), cmul(v2, cscale(c, e)));
                    }
                }
                __syncthreads();
            }
        }
        if (!converged) st |= NSSDOA_ST_EVD_NOT_CONVERGED;

        // Table 2 Step-2 ordering: eigenvalues descending (ties keep the lower index first).
        if (tid < M) {
            const double li = A[tid * ld + tid].x;
            int r = 0;
            for (int j = 0; j < M; ++j) {
                const double lj = A[j * ld + j].x;
                r += (lj > li) || (lj == li && j < tid);
            }
            perm[r] = tid;
        }
        __syncthreads();
        for (int e = tid; e < M; e += bd) evals[e] = A[perm[e] * ld + perm[e]].x;
        for (int e = tid; e < M * M; e += bd) {
            const int i = e / M, r = e - i * M;
            evecs[e] = V[i * ld + perm[r]];
        }
        // the noise eigenvalues are needed after A is overwritten by B
        double lam_k = 0.0;
        if (tid < M) lam_k = A[perm[tid] * ld + perm[tid]].x;
        __syncthreads();
        if (tid < M) red[tid] = lam_k;
        __syncthreads();

        // Table 3, Step-3/4: B with C = B B^H
        if (fr.alg == kMUSIC || fr.alg == kEV) {
            for (int e = tid; e < M * K; e += bd) {
                const int k = e / M, m = e - k * M;
                double2 v = V[m * ld + perm[fr.D + k]];
                if (fr.alg == kEV) {
                    const double l = red[fr.D + k];
                    v = cscale(l > 0.0 ? 1.0 / sqrt(l) : 0.0, v);
                }
                Bs[e] = v;
            }
            if (fr.alg == kEV && red[M - 1] <= 0.0) st |= NSSDOA_ST_DEGENERATE;
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
        double q = 0.0;
        for (int e = tid; e < M * K; e += bd) q += Bs[e].x * Bs[e].x + Bs[e].y * Bs[e].y;
        q = block_sum(q, red);
        if (tid == 0) *qref = q;
    }
    __syncthreads();
    for (int e = tid; e < M * K; e += bd) Bout[e] = Bs[e];

    if (prm.write_emb) {
        // Real embedding of B for the FP32 scan: column k gives two rows over the inner index
        // kk in [0, 2M):  re-row (Re b, Im b) and im-row (-Im b, Re b), so that the row dot the
        // embedded steering (Re a, Im a) is Re(b^H a) and Im(b^H a).  Rows are packed per
        // 32-row tile as [64 lanes][M floats]: lane h*32+i holds inner kk = 2s+h of row i.
        const GroupDev& g = groups[fr.group];
        float* emb = reinterpret_cast<float*>(ws + g.ws_emb);
        const int rows = fr.emb_rows, inner = 2 * M;
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
            const int tile = r >> 5, i = r & 31, h = kk & 1, s = kk >> 1;
            emb[((size_t)tile * 64 + h * 32 + i) * M + s] = v;
        }
    }
    if (tid == 0) status[blockIdx.x] = st;
}

}  // namespace

hipError_t launch_evd(const FrameDev* frames, int n_frames, int max_M, const EvdParams& p,
                      const GroupDev* groups, char* ws, uint32_t* status, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    const int Mp = max_M + (max_M & 1);
    const size_t lds = (size_t)2 * Mp * (Mp + 1) * sizeof(double2);
    const int threads = max_M <= 16 ? 64 : 256;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)evd_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(evd_kernel, dim3(n_frames), dim3(threads), lds, s, frames, p, groups, ws, status);
    return hipGetLastError();
}

}  // namespace nssdoa
