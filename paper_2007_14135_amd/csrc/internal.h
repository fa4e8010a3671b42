// Internal declarations shared by the HIP kernels and the host side of libnssdoa.
// Device descriptors are plain structs uploaded once per batch; every kernel reads them with
// uniform (scalar) loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <float.h>

#include "nssdoa.h"

namespace nssdoa {

constexpr double kDeg2Rad = 0.017453292519943295;   // pi / 180, the same constant numpy uses
constexpr int kScanWaves = 4;                       // waves per scan workgroup
constexpr int kScanAnglesPerWave = 64;              // two 32-angle MFMA column tiles
constexpr int kScanAnglesPerWG = kScanWaves * kScanAnglesPerWave;
constexpr int kRefineChunk = 4096;                  // grid points per refine/local-maximum workgroup
constexpr int kSelCap = 4096;                       // chunk candidates gathered per frame
constexpr int kMaxWindows = 16;                     // scan windows per frame (windowed estimation)
constexpr int kWinStride = 1 + 2 * kMaxWindows;     // int32 per frame: count, then [l0, l1) pairs
constexpr int kMaxBins = 256;                       // proposal bins

enum Alg : int32_t { kPHD = 0, kMUSIC = 1, kEV = 2, kMN = 3 };

// Per-frame descriptor.  Byte offsets (ws_*) are relative to the workspace base.
struct FrameDev {
    int32_t M, N, D, K;         // K = columns of B (M - D for MUSIC/EV, 1 for PHD/MN)
    int32_t group;              // index of the (array, grid) group
    int32_t n_chunks;           // covariance partial sums
    int32_t emb_row0;           // first row of this frame in its group's packed FP32 B tiles
    int32_t emb_rows;           // rows reserved there (>= 2K, multiple of 8)
    int64_t x_off, ldx;         // snapshot addressing, complex elements
    int64_t spec_off_user;      // element offset in the caller's spectrum buffer
    int64_t spec_off_ws;        // element offset in the workspace spectrum
    int64_t ws_partial;         // n_chunks * M*M complex128 partial covariances
    int64_t ws_R;               // M*M complex128
    int64_t ws_evals;           // M double
    int64_t ws_evecs;           // M*M complex128
    int64_t ws_B;               // M*K complex128, column-major
    int64_t ws_qref;            // 1 double
    int64_t ws_cand;            // ceil(L / kRefineChunk) * (D + extra) candidate slots of 16 bytes
    int64_t ws_lowq;            // int32, then lowq_cap int32 grid indices with low FP32 Q: the windowed
                                // scan keeps a count and the list there; the full scans keep only a
                                // flag, set when a work item's LDS list of low-Q points overflowed
    double grid_start, grid_step;
    int32_t L, circular;        // L: grid points of the frame (n_az * n_polar for a 2-D grid)
    int32_t pos_off;            // offset (doubles) of this frame's 3*M positions
    int32_t alg;
    int32_t lowq_cap;           // capacity of the low-Q list (a multiple of 256)
    int32_t is2d;               // 2-D grid: azimuth x polar angle, row-major (one row per polar angle)
    int32_t n_az;               // azimuth points per row (L for a 1-D grid)
    int32_t pad3;
    double el_start, el_step;   // 2-D grid: polar angle phi_j = el_start + j * el_step
};

// Frames that share an array geometry and a scan grid: their spectra are one GEMM.
struct GroupDev {
    int32_t M, L;
    int32_t pos_off, n_tiles;   // packed FP32 B tiles of 32 rows
    double grid_start, grid_step;
    int64_t ws_emb;             // byte offset of n_tiles 32-row MFMA operand tiles of 64 M values
    int32_t blk_off;            // offset of this group's 8-row-block -> frame table
    int32_t pad;
    int64_t steer_off;          // FP32 scans: float offset of the group's steering table, else -1
    int64_t steer_x16_off;      // FP16 split scan: float offset of the group's split table, else -1
    int32_t is2d, n_az;         // as in FrameDev
    double el_start, el_step;
};

// Split steering table of a group for the FP16 split scans of P parts (P = 2: the bytes of the
// FP32 table; P = 3: 1.5 times them): for grid index l, part p < P and h = 0, 1, the M halves at
// ((2 P l + 2 p + h) M + 8 s + t) hold part p of 2^13 v for the inner index k = 16 s + 8 h + t of
// the real-embedded steering vector (v = Re a_k for k < M, Im a_(k-M) otherwise, the FP32 value
// of the FP32 table): x_0 = 2^13 v, part p = fp16(x_p), x_(p+1) = x_p - part p (exact in FP32).
constexpr float kSplitSteerScale = 8192.0f;

// Low-Q floor of the 16-bit scans.  With both operands rounded to 16 bits (unit roundoff u:
// 2^-8 bfloat16, 2^-11 FP16, from their 8 and 11 significant bits), FP32 steering values and
// FP32 accumulation over 2M terms, each y_k = b_k^H a is off by at most c ||b_k|| + e0, c = sqrt(2) sqrt(M) (2u + u^2 + (2M + 4) 2^-24),
// e0 = sqrt(2) M 2^-25 (FP16 subnormals; 0 for bfloat16), so with S = ||B||_F^2 and K columns
// E = c sqrt(S) + e0 sqrt(K) bounds the error of the vector B^H a and |dQ| <= 2 E sqrt(Q) + E^2.
// That relative bound exceeds 1 exactly where Q < (1 + sqrt 2)^2 E^2; such a point scans to
// Q_scan < (2 + sqrt 2)^2 E^2 < 12 E^2, so every point scanned below 12 E^2 is re-evaluated in
// FP64 and the bound holds, with a relative error below 1, at every point that is not.
__host__ __device__ inline double lp_lowq_floor(int M, int K, double S, bool f16) {
    const double u = f16 ? 0x1p-11 : 0x1p-8;
    const double c = sqrt(2.0 * M) * (2.0 * u + u * u + (2.0 * M + 4.0) * 0x1p-24);
    const double e0 = f16 ? sqrt(2.0) * M * 0x1p-25 : 0.0;
    const double E = c * sqrt(S) + e0 * sqrt((double)K);
    return 12.0 * E * E;
}

// Steering table of a group for the FP32 scans: for grid index l (rounded up to whole 256-angle
// tiles) and h = 0, 1, the M floats T[(2 l + h) M + k] are Re a_{2k+h}(theta_l) for k < M/2 and
// Im a_{2(k-M/2)+h}(theta_l) for k >= M/2: the steering operand of MFMA lane h*32 + j for angle
// l, as contiguous 16-byte loads.  Values: phase in cycles formed and reduced to [-1/2, 1/2] in
// FP64, then FP32 sincospi.
// Rows: whole 256-angle tiles of the group scan plus 64 more for a windowed item that starts at
// the last grid point (points beyond the grid hold zeros and are never written out).
inline int steer_table_rows(int L) {
    return (L + kScanAnglesPerWG - 1) / kScanAnglesPerWG * kScanAnglesPerWG + kScanAnglesPerWave;
}
inline int64_t steer_table_floats(int M, int L) { return (int64_t)steer_table_rows(L) * 2 * M; }

struct CovItem { int32_t frame, chunk, n0, n1; };
struct ScanItem { int32_t group, angle_tile, t0, t1; };       // t1 exclusive, whole frames
struct PointItem { int32_t frame, l0; };                      // FP64 scan: 256 angles

struct EvdParams {
    double tol;
    int32_t max_iter;           // Jacobi: sweeps; QL: iterations per eigenvalue
    int32_t method;             // nssdoa_eig_method
    int32_t write_emb;          // packed B tiles for the scan: 0 none, 1 FP32, 2 BF16, 3 FP16,
                                // 4 FP16 split of 2 parts, 5 FP16 split of 3 parts
};

struct PeakParams {
    double lowq_tau;            // FP32 spectra: FP64 re-evaluation below tau * qref
    int32_t halfwidth;          // FP64 window around each candidate
    int32_t extra;              // candidates beyond D
    int32_t max_D;              // peak slots per frame
    int32_t refine_lowq;        // 1 for FP32 spectra
    int32_t lp_floor;           // 16-bit scans: the threshold is at least the frame's 16-bit floor
    int32_t use_user_spec;      // spectrum lives in the caller's buffer
    int32_t sel_cap;            // candidate slots of the launch's largest frame (<= kSelCap)
    // windowed estimation (both NULL otherwise): candidate chunks per frame, and the per-frame
    // window tables (kWinStride int32 each); grid points outside every window count as unknown
    const int32_t* chunk_count;
    const int32_t* windows;
    double plateau_rel;         // relative depth of a candidate's plateau (see plateau_walk)
};

// Byte offsets, inside the workspace, of the windowed-estimation tables (after the batch's own
// regions).  off_feat and off_scores are used by the learned path only.
struct LearnedLayout {
    int64_t off_feat;           // n_frames x n_feat float
    int64_t off_scores;         // n_frames x n_bins float (network logits)
    int64_t off_win;            // n_frames x kWinStride int32
    int64_t off_items;          // n_frames int32: 64-angle scan items
    int64_t off_chunks;         // n_frames int32: 4096-point peak chunks
    int64_t off_lowq;           // n_frames int32: 64-entry low-Q slices
    int64_t off_item_off;       // n_frames + 1 int32 exclusive prefix sums of the three counts
    int64_t off_chunk_off;
    int64_t off_lowq_off;
    int64_t off_scan_items;     // int2 {frame, first angle | angles << 24} per 64-angle scan item
    int64_t off_chunk_items;    // int4 {frame, first point, window start, window end} per chunk
    int64_t off_rescue;         // n_frames int32: frames searched again over the whole grid, or -1
};

// Upper bounds of the windowed work lists of one frame (a fallback frame scans its whole grid).
inline int64_t max_scan_items(int L) { return (L + kScanAnglesPerWave - 1) / kScanAnglesPerWave + kMaxWindows; }
inline int64_t max_chunk_items(int L) { return (L + kRefineChunk - 1) / kRefineChunk + kMaxWindows; }

// Scan angle theta_l = start + l * step with the product and the sum rounded separately
// (contraction into one fused multiply-add is switched off here).
__device__ inline double grid_angle(double start, double step, int l) {
#pragma clang fp contract(off)
    const double prod = step * (double)l;
    return start + prod;
}

// Direction of grid index l as the three factors of Eq. 2's phase: the phase of element m in
// cycles is x_m u + y_m v + z_m w.  A 1-D grid lies in the horizontal plane (phi = 90 deg, taken
// as sin phi = 1 and cos phi = 0 exactly): u = sin theta, v = cos theta, w = 0.  A 2-D grid is
// row-major, l = j n_az + i: theta_i = start + i step, phi_j = el_start + j el_step, and
// u = sin theta sin phi, v = cos theta sin phi, w = cos phi.  Any descriptor with the FrameDev /
// GroupDev grid fields works.
struct Dir3 { double u, v, w; };

template <typename G>
__device__ inline Dir3 grid_dir(const G& g, int l) {
    Dir3 d;
    if (!g.is2d) {
        sincos(grid_angle(g.grid_start, g.grid_step, l) * kDeg2Rad, &d.u, &d.v);
        d.w = 0.0;
        return d;
    }
    const int j = l / g.n_az, i = l - j * g.n_az;
    double sth, cth, sph, cph;
    sincos(grid_angle(g.grid_start, g.grid_step, i) * kDeg2Rad, &sth, &cth);
    sincos(grid_angle(g.el_start, g.el_step, j) * kDeg2Rad, &sph, &cph);
    d.u = sth * sph;
    d.v = cth * sph;
    d.w = cph;
    return d;
}

// Phase of element m in cycles for direction d (positions: x, y, z in wavelengths).
__device__ __forceinline__ double phase_cycles(const double* __restrict__ pm, const Dir3& d) {
    return fma(pm[2], d.w, fma(pm[0], d.u, pm[1] * d.v));
}

constexpr int kCisTable = 257;   // exp(j 2 pi k / 256) for k = -128..128

// exp(j 2 pi r) in FP64 for |r| <= 1/2: r = k/256 + d with |d| <= 1/512; exp(j 2 pi k/256) comes
// from a correctly rounded table and exp(j 2 pi d) from its Taylor series to degree 9
// (|2 pi d| <= pi/256, truncation below 1e-25).
__device__ __forceinline__ double2 cis2pi(double r, const double2* __restrict__ cis) {
    const double kd = rint(r * 256.0);
    const double x = fma(kd, -1.0 / 256.0, r) * 6.283185307179586;
    const double x2 = x * x;
    double c = fma(x2, 1.0 / 40320.0, -1.0 / 720.0);
    c = fma(c, x2, 1.0 / 24.0);
    c = fma(c, x2, -0.5);
    c = fma(c, x2, 1.0);
    double s = fma(x2, 1.0 / 362880.0, -1.0 / 5040.0);
    s = fma(s, x2, 1.0 / 120.0);
    s = fma(s, x2, -1.0 / 6.0);
    s = fma(s * x2, x, x);
    const double2 t = cis[(int)kd + 128];
    return make_double2(t.x * c - t.y * s, fma(t.x, s, t.y * c));
}

// ||B^H a(d)||^2 in FP64 for one direction d (Eq. 2, Table 3 Step-4 in factored form).  B is
// M x K complex128, column-major.  The phase in cycles is reduced to [-1/2, 1/2] before
// exp(j 2 pi .) so that its rounding does not grow with the aperture.
template <int MB>
__device__ __forceinline__ double q64_eval(const double* __restrict__ pos, int M, int K,
                                           const double2* __restrict__ B, const Dir3& d,
                                           const double2* __restrict__ cis) {
    double ar[MB], ai[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        ar[m] = 0.0;
        ai[m] = 0.0;
        if (m < M) {
            const double c = phase_cycles(pos + 3 * m, d);
            const double2 a = cis2pi(c - rint(c), cis);
            ar[m] = a.x;
            ai[m] = a.y;
        }
    }
    double Q = 0.0;
    int k = 0;
    for (; k + 4 <= K; k += 4) {
        double yr[4] = {0.0, 0.0, 0.0, 0.0}, yi[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (m < M) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double2 b = B[(size_t)(k + u) * M + m];
                    // conj(b) * a = (br ar + bi ai) + j (br ai - bi ar)
                    yr[u] = fma(b.x, ar[m], fma(b.y, ai[m], yr[u]));
                    yi[u] = fma(b.x, ai[m], fma(-b.y, ar[m], yi[u]));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) Q += yr[u] * yr[u] + yi[u] * yi[u];
    }
    for (; k < K; ++k) {
        double yr = 0.0, yi = 0.0;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (m < M) {
                const double2 b = B[(size_t)k * M + m];
                yr = fma(b.x, ar[m], fma(b.y, ai[m], yr));
                yi = fma(b.x, ai[m], fma(-b.y, ar[m], yi));
            }
        }
        Q += yr * yr + yi * yi;
    }
    return Q;
}

// The same quantity evaluated by a group of 16 lanes of one wave (lanes 16g..16g+15 share one
// direction): lane j forms a_m for m = j, j+16, ... into LDS (`a` holds 4 * MB entries per wave),
// then forms y_k = b_k^H a for k = j, j+16, ..., and the 16 partial sums of |y_k|^2 are added
// with a butterfly.  Every lane of the wave must call it; the result is in all 16 lanes.
template <int MB>
__device__ __forceinline__ double q64_group(const double* __restrict__ pos, int M, int K,
                                            const double2* __restrict__ B, const Dir3& d,
                                            const double2* __restrict__ cis, double2* a) {
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    for (int m = j; m < M; m += 16) {
        const double c = phase_cycles(pos + 3 * m, d);
        a[g * MB + m] = cis2pi(c - rint(c), cis);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double q = 0.0;
    for (int k = j; k < K; k += 16) {
        const double2* bk = B + (size_t)k * M;
        double yr = 0.0, yi = 0.0;
#pragma unroll 8
        for (int m = 0; m < M; ++m) {
            const double2 b = bk[m];
            const double2 am = a[g * MB + m];
            yr = fma(b.x, am.x, fma(b.y, am.y, yr));
            yi = fma(b.x, am.y, fma(-b.y, am.x, yi));
        }
        q += yr * yr + yi * yi;
    }
    q += __shfl_xor(q, 8, 16);
    q += __shfl_xor(q, 4, 16);
    q += __shfl_xor(q, 2, 16);
    q += __shfl_xor(q, 1, 16);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();   // `a` may be reused by the caller's next call
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return q;
}

// ---------------------------------------------------------------------------------------------
// Peak candidates.  On a fine grid a broad maximum of P is flatter than the scan's rounding, so
// the rounded spectrum shows many small local maxima around it.  A local maximum x at l is kept
// only if it wins its plateau, the contiguous points around l with values >= x (1 - rel): no
// point of the plateau holds a larger value, nor an equal one at a lower index.  Each broad
// maximum then gives one candidate, which carries its plateau's extent; the exact maximum lies
// in the plateau when rel exceeds the spectrum's relative error.
constexpr int kMaxPlateau = 4096;   // points walked on each side of a candidate

struct CandSlot {
    double v;                   // value at idx (NaN for an unused slot)
    int32_t idx;                // grid index, -1 for an unused slot
    uint32_t span;              // plateau points left of idx << 16 | points right of idx
};

// Walk the plateau of the local maximum x at grid index l through val(g) (NaN: unknown, ends the
// walk).  Returns false when the plateau holds a better point, else its extent in *span.  The 64
// lanes of a wave walk together, 64 points per step (every lane must call it with the same
// arguments); the first point that ends the plateau or beats x decides.
template <typename F>
__device__ inline bool plateau_walk(double x, int l, double rel, F val, uint32_t* span) {
    const int lane = threadIdx.x & 63;
    const double thr = x - x * rel;
    int ext[2] = {kMaxPlateau, kMaxPlateau};
    for (int side = 0; side < 2; ++side) {
        for (int base = 1; base <= kMaxPlateau; base += 64) {
            const int k = base + lane;
            bool stop = true, beat = false;
            if (k <= kMaxPlateau) {
                const double y = val(side == 0 ? l - k : l + k);
                stop = !(y >= thr);
                // on the left an equal value wins (lower index); on the right it does not
                beat = !stop && (side == 0 ? y >= x : y > x);
            }
            const unsigned long long sb = __ballot(stop), bb = __ballot(beat);
            if (sb | bb) {
                const int first = __ffsll((long long)(sb | bb)) - 1;
                if ((bb >> first) & 1ull) return false;
                ext[side] = base + first - 1;
                break;
            }
        }
    }
    *span = ((uint32_t)ext[0] << 16) | (uint32_t)ext[1];
    return true;
}

// Extrema of the 32-point blocks of v[0..span): bmax[b], bmin[b] for b < ceil(span / 32); a block
// holding a NaN gets bmin = NaN.  Every thread of the workgroup calls it; thread b scans block b.
constexpr int kPlateauBlock = 32;
template <typename TV>
__device__ inline void block_extrema(const TV* v, int span, double* bmax, double* bmin) {
    const int nb = (span + kPlateauBlock - 1) / kPlateauBlock;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const int e0 = b * kPlateauBlock, e1 = min(span, e0 + kPlateauBlock);
        double hi = -INFINITY, lo = INFINITY;
#pragma unroll
        for (int j = 0; j < kPlateauBlock; ++j) {
            const int e = e0 + ((j + b) & (kPlateauBlock - 1));   // rotated start: no bank conflicts
            if (e >= e1) continue;
            const double x = (double)v[e];
            hi = fmax(hi, x);
            lo = (x < lo || x != x) ? x : lo;               // NaN sticks
        }
        bmax[b] = hi;
        bmin[b] = lo;
    }
}

// True when the local maximum x at v-index e certainly loses its plateau: the 32-point block
// holding e and its two neighbours contain a larger value and no value below x (1 - rel) or NaN,
// so the plateau walk would reach that larger value.
__device__ inline bool plateau_prefilter(int e, double x, double rel, int span, const double* bmax,
                                         const double* bmin) {
    const int b = e / kPlateauBlock, nb = (span + kPlateauBlock - 1) / kPlateauBlock;
    if (b < 1 || b + 1 >= nb) return false;
    const double hi = fmax(bmax[b - 1], fmax(bmax[b], bmax[b + 1]));
    const double lo0 = bmin[b - 1], lo1 = bmin[b], lo2 = bmin[b + 1];
    const double thr = x - x * rel;
    return hi > x && lo0 >= thr && lo1 >= thr && lo2 >= thr;
}

constexpr uint32_t kLoser = 0xFFFFFFFFu;       // flag of a local maximum that lost its plateau
constexpr int kPrefilterMin = 8;               // local maxima in a chunk worth the block extrema

// Marks in flag[0..n) (kLoser or 0) the local maxima of a chunk that plateau_prefilter drops,
// when the chunk has more than kPrefilterMin of them (a fine grid, where rounding makes many);
// v_index(i) gives the v-index of local maximum i.  Every thread of the workgroup calls it.
template <typename FI, typename TV>
__device__ inline void prefilter_losers(int n, const double* lval, FI v_index, const TV* v, int span,
                                        double rel, double* bmax, double* bmin, uint32_t* flag) {
    const int tid = threadIdx.x;
    const bool use = n > kPrefilterMin;
    if (use) {
        block_extrema(v, span, bmax, bmin);
        __syncthreads();
    }
    for (int i = tid; i < n; i += blockDim.x)
        flag[i] = (use && plateau_prefilter(v_index(i), lval[i], rel, span, bmax, bmin)) ? kLoser : 0u;
    __syncthreads();
}

// The best C plateau winners among the n local maxima (lval, lidx) of a chunk, by (value desc,
// index asc), to slots[0..C); unused slots get idx -1.  flag: n ints of LDS holding kLoser for
// maxima already known to lose (prefilter_losers), else 0; cnt: one LDS int.  Every thread of the
// workgroup calls it; each wave walks one local maximum at a time, then every winner finds its
// rank among the winners.
template <typename F>
__device__ inline void chunk_candidates(int n, const double* lval, const int* lidx, uint32_t* flag, int* cnt,
                                        double rel, F val, CandSlot* slots, int C) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = tid >> 6, nwaves = blockDim.x >> 6;
    for (int i = wave; i < n; i += nwaves) {
        if (flag[i] == kLoser) continue;             // uniform: one i per wave
        uint32_t sp = 0;
        const bool win = plateau_walk(lval[i], lidx[i], rel, val, &sp);
        if (lane == 0) flag[i] = win ? sp : kLoser;  // a span never has all bits set
    }
    __syncthreads();
    if (tid == 0) *cnt = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
        const uint32_t fi = flag[i];
        if (fi == kLoser) continue;
        atomicAdd(cnt, 1);
        const double vi = lval[i];
        const int li = lidx[i];
        int rank = 0;
        for (int k = 0; k < n; ++k)
            rank += flag[k] != kLoser && ((lval[k] > vi) || (lval[k] == vi && lidx[k] < li));
        if (rank < C) {
            slots[rank].v = vi;
            slots[rank].idx = li;
            slots[rank].span = fi;
        }
    }
    __syncthreads();
    const int m = *cnt;
    for (int s = m + tid; s < C; s += blockDim.x) {
        slots[s].v = __longlong_as_double(0x7ff8000000000000LL);
        slots[s].idx = -1;
        slots[s].span = 0;
    }
}

// Appends grid index l to a frame's low-Q list (int count, then entries) when `low`, with one
// atomic per wave: every lane of the wave calls it for the same list; entries beyond `cap` are
// only counted.
__device__ inline void lowq_append(bool low, int l, int* cnt, int cap) {
    const unsigned long long mask = __ballot(low);
    if (mask == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt, __popcll(mask));
    base = __shfl(base, leader);
    if (low) {
        const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (slot < cap) cnt[1 + slot] = l;
    }
}

// Low-Q points of a matrix-core scan work item (Q = ||B^H a||^2 below lowq_tau ||B||_F^2, where
// its FP32 value has a large relative error), collected in LDS while the scan runs and published
// after its matrix-core loop to the batch's list, which lowq_refine_kernel re-evaluates in FP64
// (balanced over the whole GPU: low-Q points cluster around the peaks of a few frames).  Entry:
// frame << 8 | angle within the work item's 256 angles.
constexpr int kScanLowqCap = 1024;
struct ScanLowq {
    int n;
    int base;
    int list[kScanLowqCap];
};

// Every lane of a wave calls it for one frame's 64 angles; lanes with `low` append their entry
// (one LDS atomic per wave).  When the list is full the frame's flag is set instead, and the
// peak search re-evaluates that frame's low-Q points itself.
__device__ inline void scan_lowq_collect(bool low, int f, int a, ScanLowq& q, int* frame_flag) {
    const unsigned long long mask = __ballot(low);
    if (mask == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&q.n, __popcll(mask));
    base = __shfl(base, leader);
    if (low) {
        const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (slot < kScanLowqCap) q.list[slot] = (f << 8) | a;
        else *frame_flag = 1;
    }
}

// Reserves room for the work item's entries in the batch list (count, then (frame, grid index)
// pairs) with one atomic and writes them; entries beyond the list's capacity set their frame's
// flag.  Called by every thread after a workgroup barrier.
__device__ inline void scan_lowq_publish(ScanLowq& q, int angle0, int* count, int2* list, int cap,
                                         const FrameDev* __restrict__ frames, char* __restrict__ ws) {
    const int n = min(q.n, kScanLowqCap);
    if (threadIdx.x == 0) q.base = n > 0 ? atomicAdd(count, n) : 0;
    __syncthreads();
    const int base = q.base;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ent = q.list[i];
        const int f = ent >> 8, l = angle0 + (ent & 255);
        if (base + i < cap) list[base + i] = make_int2(f, l);
        else *reinterpret_cast<int*>(ws + frames[f].ws_lowq) = 1;
    }
}

// Host-side launchers (defined next to their kernels).
hipError_t launch_cov(bool c128, int max_M, const CovItem* items, int n_items, const FrameDev* frames,
                      const void* X, char* ws, int* reset, hipStream_t s);
hipError_t launch_evd(const int32_t* frame_list, int n_frames, int max_M, const EvdParams& p,
                      const FrameDev* frames, const GroupDev* groups, char* ws, uint32_t* status,
                      hipStream_t s);
hipError_t launch_steer_table(const double* pos, const GroupDev& g, float* table, hipStream_t s);
hipError_t launch_steer_table_split16(int parts, const double* pos, const GroupDev& g, float* table, hipStream_t s);
constexpr size_t kScanLdsBytes = 65536;            // B tiles of one FP32 scan work item in LDS
constexpr int kScanMaxBlocks = kScanLdsBytes / (64 * 8 * 4) * 4;   // 8-row blocks of one, M >= 8
// Low-Q list of a batch: an int count (reset by the covariance launch), then cap (frame, index).
struct LowqList {
    int* count;
    int2* list;
    int cap;
};
hipError_t launch_scan_f32(int M, const ScanItem* items, int n_items, int max_tiles, const GroupDev* groups,
                           const FrameDev* frames, const int32_t* blkframe, const float* steer,
                           char* ws, float* spec, int use_user_spec, float lowq_tau, LowqList lq, hipStream_t s);
hipError_t launch_scan_split16(int parts, int M, const ScanItem* items, int n_items, int max_tiles,
                               const GroupDev* groups, const FrameDev* frames, const int32_t* blkframe,
                               const float* steer, char* ws, float* spec, int use_user, float tau, LowqList lq,
                               hipStream_t s);
hipError_t launch_scan_lp(bool f16, int M, const ScanItem* items, int n_items, const GroupDev* groups,
                          const FrameDev* frames, const int32_t* blkframe, const double* pos, char* ws,
                          float* spec, int use_user, float lowq_tau, LowqList lq, hipStream_t s);
hipError_t launch_lowq_refine(int bucket_M, LowqList lq, const FrameDev* frames, const double* pos,
                              const double2* cis, const char* ws, float* spec, int use_user, int n_wg,
                              hipStream_t s);
hipError_t launch_scan_f64(const PointItem* items, int n_items, int max_M,
                           const FrameDev* frames, const double* pos, const double2* cis,
                           const char* ws, double* spec, int use_user_spec, hipStream_t s);
hipError_t launch_peaks(bool f64, int bucket_M, const PointItem* items, int n_items, const int32_t* frame_list,
                        int n_frames, const FrameDev* frames, const double* pos, const double2* cis, char* ws,
                        void* spec, const PeakParams& p, void* peaks, int32_t* npeaks, uint32_t* status,
                        hipStream_t s);
hipError_t launch_scan_form(int bucket_M, const PointItem* items, int n_items, const FrameDev* frames,
                            const double* pos, const char* ws, int form, float* spec, hipStream_t s);

// 2-D grids: items of 256 points of the frames in flist (one M bucket), then one selection per
// frame; each frame's ws_cand region holds an FP64 peak map of L doubles.
constexpr int kPeak2dItem = 256;
hipError_t launch_peaks2d(bool f64, int bucket_M, const PointItem* items, int n_items, const int32_t* flist,
                          int n_frames, const FrameDev* frames, const double* pos, const double2* cis, char* ws,
                          const void* spec, int use_user, int max_D, nssdoa_peak* peaks, int32_t* npeaks,
                          uint32_t* status, hipStream_t s);

hipError_t launch_gemm_bf16(int M, int N, int K, const float* A, int64_t sam, int64_t sak, int relu_in_a,
                            const float* B, int64_t sbk, int64_t sbn, int relu_in_b, float alpha,
                            const float* bias, const float* mask, int64_t ldm, int relu_out, float* C,
                            int64_t ldc, hipStream_t s);
hipError_t launch_colsum(int rows, int cols, const float* X, int64_t ld, float* out, hipStream_t s);
hipError_t launch_bce(int rows, int cols, const float* Z, const float* Y, float* dZ, float* row_loss,
                      float* loss, hipStream_t s);
hipError_t launch_adam(int n, float* p, const float* g, float* m, float* v, float lr, int t, hipStream_t s);
hipError_t launch_features(const int32_t* flist, int n, const FrameDev* frames, const char* ws, float* out,
                           int nfeat, hipStream_t s);

hipError_t launch_proposals(const FrameDev* frames, int n_frames, const float* scores, int n_bins, int topk,
                            double half_window, float threshold, float floor, int local_max, char* ws,
                            const LearnedLayout& lay, uint32_t* status, hipStream_t s);
hipError_t launch_rescue(const FrameDev* frames, const int32_t* frame_list, int n_list, const int32_t* npeaks,
                         uint32_t* status, char* ws, const LearnedLayout& lay, int32_t* rescue, hipStream_t s);
hipError_t launch_expand(const FrameDev* frames, int n_frames, char* ws, const LearnedLayout& lay, hipStream_t s);
hipError_t launch_scan_windows(int parts, int M, const FrameDev* frames, int n_frames, const GroupDev* groups,
                               const int32_t* blkframe, const float* steer, char* ws, const LearnedLayout& lay,
                               float* spec, int use_user, float lowq_tau, int n_wg, hipStream_t s);
hipError_t launch_window_peaks(int bucket_M, const FrameDev* frames, int n_frames, const double* pos,
                               const double2* cis, char* ws, const LearnedLayout& lay, int extra, double lowq_tau,
                               double plateau_rel, float* spec, int use_user, int n_wg, hipStream_t s);

// Network dimensions and its forward pass for `rows` feature rows into logits[rows][out]
// (processed in slices of the network's max_batch rows).
void mlp_dims(nssdoa_mlp n, int32_t* in, int32_t* width, int32_t* out, int32_t* max_batch);
hipError_t mlp_forward_rows(nssdoa_mlp n, const float* feats, int rows, float* logits, hipStream_t s);

}  // namespace nssdoa
