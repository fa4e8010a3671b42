/*
 * nssdoa.h -- C ABI of the MI355X noise-subspace narrowband DOA library (libnssdoa.so).
 *
 * The library estimates directions of arrival with the four noise-subspace methods of
 * Eray & Temizel, "Performance Analysis of Noise Subspace-based Narrowband Direction-of-Arrival
 * (DOA) Estimation Algorithms on CPU and GPU" (arXiv 2007.14135): PHD, MUSIC, EV and MN.
 * Per frame of complex snapshots it runs the common code structure of Table 2 on the GPU:
 *   Step-1  sample covariance R = X X^H / N                              (Eq. 3)
 *   Step-2  Hermitian eigendecomposition, eigenvalues descending         (Table 2, Step-2)
 *   Step-3/4 noise-subspace selection; the Step-4 matrix C is kept in
 *           factored form C = B B^H                                      (Table 3)
 *   Step-5  pseudo-spectrum P(theta) = 1 / (a^H C a) = 1 / ||B^H a||^2
 *           over a uniform azimuth grid, steering vectors of Eq. 2       (Table 2, Step-5)
 *   Step-6  peak search and selection of the D strongest peaks           (Table 2, Step-6)
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns nssdoa_status; NSSDOA_OK (0) on success.  No C++ exception crosses the
 *   ABI.  nssdoa_last_error() returns a message describing the last failure on this thread.
 * - Argument errors are detected on the host, synchronously, before any device work, and
 *   return NSSDOA_EINVAL.  Problems that depend on the data (non-finite input, a degenerate
 *   noise subspace, fewer peaks than sources) never fail a call: they set per-frame status bits.
 * - "host" pointers are ordinary CPU memory; "device" pointers are GPU memory of the current
 *   HIP device (for example the data_ptr() of a torch tensor on that device).
 * - The caller owns every buffer it passes and the stream.  The library never frees caller
 *   memory.  Plans and batches own only their internal device tables and free them on destroy.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Device work is
 *   enqueued on it and the call returns; results are valid once the stream has been
 *   synchronised.  Two calls that share a workspace or an output buffer must not overlap.
 * - Directions are azimuth angles in degrees, measured from +y toward +x in the horizontal plane
 *   (phi = 90 deg in Eq. 2).  Element positions are in wavelengths.
 */
#ifndef NSSDOA_H
#define NSSDOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NSSDOA_OK = 0,
    NSSDOA_EINVAL = 1,        /* invalid argument (checked on the host before device work)  */
    NSSDOA_EUNSUPPORTED = 2,  /* valid request this build does not implement                */
    NSSDOA_ENOMEM = 3,        /* a device or host allocation of the library failed          */
    NSSDOA_EDEVICE = 4,       /* a HIP runtime call failed (no device, launch failure, ...) */
    NSSDOA_ESTATE = 5         /* object used in a state that does not allow the call        */
} nssdoa_status;

/* Table 3: the four noise-subspace methods.  Their Step-4 matrices factor as C = B B^H with
 * PHD  B = e_min (eigenvector of the smallest eigenvalue), K = 1 column;
 * MUSIC B = E_n (eigenvectors D+1..M), K = M - D columns;
 * EV   B = E_n diag(lambda_n^(-1/2)), K = M - D columns;
 * MN   B = P_n e_1 / (e_1^H P_n e_1) with P_n = E_n E_n^H, K = 1 column. */
typedef enum { NSSDOA_PHD = 0, NSSDOA_MUSIC = 1, NSSDOA_EV = 2, NSSDOA_MN = 3 } nssdoa_alg;

/* Arithmetic of the spectrum scan (Step-5).  The covariance is always accumulated in FP64, and
 * the eigensolve, noise-subspace matrices and peak refinement are always FP64.
 * C128: complex128 snapshots, FP64 scan, double spectrum.
 * C64 : complex64 snapshots, FP32 scan on the matrix cores with FP32 accumulation; float
 *       spectrum.
 * BF16, F16: complex64 snapshots, scan operands rounded to bfloat16 / IEEE half on the matrix
 *       cores with FP32 accumulation; float spectrum.
 * For C64, BF16 and F16 every point whose scanned ||B^H a||^2 is below lowq_tau * ||B||_F^2 (the
 * neighbourhoods of the spectrum peaks) is re-evaluated in FP64 before the peak search.  For BF16
 * and F16 the threshold is at least 12 E^2, E = c ||B||_F + e0 sqrt(K) with
 * c = sqrt(2M) (2u + u^2 + (2M + 4) 2^-24), u = 2^-8 (BF16) or 2^-11 (F16), e0 = sqrt(2) M 2^-25
 * (F16) or 0 (BF16): E bounds the error of the 16-bit B^H a, so every point where the relative
 * bound 2E/sqrt(Q) + E^2/Q on the scanned Q reaches 1 is re-evaluated in FP64. */
typedef enum { NSSDOA_C128 = 0, NSSDOA_C64 = 1, NSSDOA_BF16 = 2, NSSDOA_F16 = 3 } nssdoa_prec;

/* Per-frame status bits written to status[] by nssdoa_estimate. */
#define NSSDOA_ST_NONFINITE_INPUT   0x1u  /* R has a NaN/Inf entry; no peaks, spectrum is NaN      */
#define NSSDOA_ST_EVD_NOT_CONVERGED 0x2u  /* eigensolver stopped at eig_max_iter above eig_tol     */
#define NSSDOA_ST_DEGENERATE        0x4u  /* EV: a noise eigenvalue <= M 2^-52 lambda_1 (zero to
                                             working precision); MN: (P_n)_11 <= 1e-300            */
#define NSSDOA_ST_FEWER_PEAKS       0x8u  /* fewer than D local maxima; unused slots idx = -1      */
#define NSSDOA_ST_PEAK_OVERFLOW     0x10u /* more local maxima than the candidate buffer holds     */
#define NSSDOA_ST_FALLBACK_USED     0x20u /* windowed estimation scanned the whole grid (best score
                                             below the threshold, or the windows held fewer than D
                                             peaks); informational                               */

/* An array geometry: M elements at host positions pos_wl[3*m + {0,1,2}] = (x, y, z) in
 * wavelengths (Eq. 2).  The plan copies the positions; the caller may free them afterwards. */
typedef struct {
    int32_t M;            /* elements, 2 <= M <= 64; 8, 16, 32 or 64 for the C64/BF16/F16 scans */
    int32_t reserved;     /* must be 0                                                         */
    const double* pos_wl; /* host, 3*M doubles                                                 */
} nssdoa_array;

/* A uniform scan grid (the AngleSer of Table 2, Step-5).
 * 1-D (n_polar = 0): azimuths theta_l = start_deg + l * step_deg for l = 0..L-1, each computed
 *   from l in FP64, in the horizontal plane (phi = 90 deg of Eq. 2, taken as sin phi = 1 and
 *   cos phi = 0 exactly).  circular != 0 makes the first and last points neighbours for the peak
 *   search (a full 360 deg grid); otherwise neither end can be a peak.
 * 2-D (n_polar >= 1): the L azimuths above times n_polar polar angles phi_j = polar_start_deg +
 *   j * polar_step_deg (Eq. 2's phi, measured from +z; 90 deg is the horizontal plane), the
 *   azimuth x elevation scans of the paper's experiments (Section 5, Tables 8 and 10).  A frame's
 *   spectrum then holds L * n_polar values, row-major with one row per polar angle: point
 *   j * L + i is (theta_i, phi_j).  Peaks are the points above their 8 neighbours inside the
 *   grid: strictly above each neighbour that precedes them in that order, at least equal to
 *   each one that follows, and strictly above at least one (a plateau is reported at its first
 *   point; grid edges can hold peaks); the azimuth axis wraps when circular != 0, the polar axis
 *   never does.  2-D grids are supported with NSSDOA_C64 and NSSDOA_C128 by nssdoa_estimate,
 *   nssdoa_estimate_noalloc and graph capture (EUNSUPPORTED otherwise). */
typedef struct {
    double start_deg;
    double step_deg;      /* > 0                                                               */
    int32_t L;            /* azimuth points, >= 3                                              */
    int32_t circular;
    double polar_start_deg;  /* 2-D grids: first polar angle, finite                          */
    double polar_step_deg;   /* 2-D grids: > 0                                                */
    int32_t n_polar;      /* 0: 1-D grid; 1..4096: polar angles of a 2-D grid; L * n_polar <=
                             2^24                                                              */
    int32_t reserved;     /* must be 0                                                         */
} nssdoa_grid;

/* One frame of snapshots.  X_N of Eq. 3 is M x N with one column per snapshot; it is stored
 * element-major: snapshot n of element m is complex element x_off + m * ldx + n of the X buffer
 * (complex64 or complex128 interleaved re, im).  spec_off is the element offset of this frame's
 * L spectrum values in the spectrum buffer (ignored when no spectrum buffer is passed). */
typedef struct {
    int32_t array_id;     /* index into the plan's arrays                                      */
    int32_t grid_id;      /* index into the plan's grids                                       */
    int32_t N;            /* snapshots, >= 1                                                   */
    int32_t D;            /* sources, 1 <= D < M                                               */
    int64_t x_off;        /* >= 0                                                              */
    int64_t ldx;          /* >= N                                                              */
    int64_t spec_off;     /* >= 0                                                              */
} nssdoa_frame;

/* One selected peak (Table 2, Step-6): grid index, its direction and the FP64 spectrum value. */
typedef struct {
    int32_t idx;          /* grid index (j * L + i on a 2-D grid), or -1 for an unused slot    */
    int32_t reserved;
    double angle_deg;     /* azimuth theta, NaN for an unused slot                             */
    double value;         /* P at idx evaluated in FP64, NaN for an unused slot                */
    double polar_deg;     /* polar angle phi: 90 on a 1-D grid, NaN for an unused slot         */
} nssdoa_peak;

/* Hermitian eigensolver of Step-2 (Table 2).  All run in FP64 with one workgroup per frame and
 * start from the Householder reduction of R to a real symmetric tridiagonal T (except Jacobi).
 *   NSSDOA_EIG_AUTO:   M <= 16: eigenvalues of T by bisection (Sturm counts, to 2 eps ||T||),
 *                      eigenvectors by inverse iteration with modified Gram-Schmidt
 *                      orthonormalisation; larger M: as NSSDOA_EIG_QL.  The default.
 *   NSSDOA_EIG_QL:     implicit QL with Wilkinson's shift on T; the block splits where
 *                      |e_i| <= eig_tol * (|d_i| + |d_{i+1}|); at most eig_max_iter QL iterations
 *                      per eigenvalue.
 *   NSSDOA_EIG_JACOBI: cyclic complex Jacobi on R; stops when |r_pq| <= eig_tol * sqrt(r_pp r_qq)
 *                      for all p < q, at most eig_max_iter sweeps.  Slower, but small eigenvalues
 *                      are accurate relative to themselves.
 * Eigenvalue errors of AUTO and QL are of the order of eps ||R||. */
typedef enum { NSSDOA_EIG_AUTO = 0, NSSDOA_EIG_QL = 1, NSSDOA_EIG_JACOBI = 2 } nssdoa_eig_method;

/* Matrix-core kernel of the C64 (FP32-accuracy) scans of Step-5 (Table 2).  All three form the
 * real-embedded product of the B tiles and the FP32 steering values and accumulate in FP32.
 *   NSSDOA_C64_SCAN_SPLIT16: every FP32 operand x is split into FP16 parts x = hi + lo + r with
 *                            |r| <= 2^-22 |x| + 2^-25 (2^-25: half the FP16 subnormal spacing),
 *                            after an exact power-of-two scaling per frame (B) and per steering
 *                            table that puts the largest magnitudes near 2^13, and a b is formed
 *                            as hi_a hi_b + hi_a lo_b + lo_a hi_b on the FP16 matrix cores
 *                            (v_mfma_f32_32x32x16_f16); the neglected terms are below
 *                            2^-20 |a b| + 2^-25 (|a| + |b|), the order of the FP32 accumulation
 *                            error of the sums they enter: 22-bit operands, the fastest.
 *   NSSDOA_C64_SCAN_FP32:    FP32 operands on v_mfma_f32_32x32x2f32.
 *   NSSDOA_C64_SCAN_SPLIT16X3: three FP16 parts per operand, x = hi + mid + lo + r (each part the
 *                            FP16 rounding of what the earlier parts leave): 33 significant bits,
 *                            so after the same power-of-two scaling every FP32 steering value is
 *                            reproduced exactly where |2^13 v| >= 1/2 and to within 2^-25 below,
 *                            and B (split from its FP64 values) to within 2^-33 |x| + 2^-25, both
 *                            below the FP32 rounding the FP32-operand kernel applies to them; a b
 *                            is formed from the six products of parts whose orders add up to at
 *                            most two (hi hi, hi mid, mid hi, hi lo, lo hi, mid mid; the dropped
 *                            ones are below 2^-33 |a b|), accumulated in FP32 on the FP16 matrix
 *                            cores.  At least as accurate as the FP32-operand kernel.  The default.
 * The windowed and learned estimators use the same kernel choice. */
typedef enum { NSSDOA_C64_SCAN_SPLIT16X3 = 0, NSSDOA_C64_SCAN_FP32 = 1, NSSDOA_C64_SCAN_SPLIT16 = 2 } nssdoa_c64_scan;

/* Tunables; pass NULL to nssdoa_plan_create for the defaults given here. */
typedef struct {
    double eig_tol;           /* QL / Jacobi tolerance (see nssdoa_eig_method), (0, 1); 1e-15  */
    int32_t eig_max_iter;     /* QL iterations per eigenvalue / Jacobi sweeps, 1..1000; 30     */
    int32_t refine_halfwidth; /* FP64 re-evaluation window around each candidate peak, 1..16; 4 */
    double lowq_tau;          /* C64: FP64 re-evaluation below lowq_tau * ||B||_F^2, >= 0; 5e-4 */
    int32_t extra_candidates; /* local maxima kept beyond D for the FP64 re-pick, 0..16; 4     */
    int32_t scan_rows;        /* rows of stacked B per matrix-core scan work item: 0 = default
                                 (384 for C64, 4096 for BF16/F16), else a multiple of 32 in
                                 [32, 16384].  A tuning knob: it moves frames' rows within the
                                 32-row MFMA tiles, so FP32 spectra may change in their last
                                 bits; peaks are re-picked in FP64.  C64 work items hold at most
                                 65536 / (8 M) rows with FP32 operands, 1024 with FP16 split ones */
    int32_t eig_method;       /* nssdoa_eig_method; NSSDOA_EIG_AUTO                            */
    int32_t c64_scan;         /* nssdoa_c64_scan: matrix-core kernel of the C64 scans;
                                 NSSDOA_C64_SCAN_SPLIT16X3 (0)                                  */
} nssdoa_options;

typedef struct nssdoa_plan_s* nssdoa_plan;
typedef struct nssdoa_batch_s* nssdoa_batch;

/* Intermediate results a caller (or a test) may read from the workspace after nssdoa_estimate. */
typedef enum {
    NSSDOA_WS_COV = 0,     /* R, M x M complex128, row-major, full Hermitian                    */
    NSSDOA_WS_EVALS = 1,   /* lambda, M doubles, descending                                     */
    NSSDOA_WS_EVECS = 2,   /* U, M x M complex128, row-major, column k pairs with lambda_k      */
    NSSDOA_WS_B = 3,       /* B, M x K complex128, column-major (column k contiguous)            */
    NSSDOA_WS_QREF = 4,    /* ||B||_F^2, one double                                             */
    NSSDOA_WS_SPECTRUM = 5 /* the internal spectrum (used when no spectrum buffer is passed)    */
} nssdoa_ws_item;

/* Stages of nssdoa_estimate, for nssdoa_stage_time. */
typedef enum {
    NSSDOA_STAGE_COVARIANCE = 0, /* Step-1                                                     */
    NSSDOA_STAGE_EIGEN = 1,      /* Step-2..4: covariance reduction, Jacobi, B                 */
    NSSDOA_STAGE_SCAN = 2,       /* Step-5                                                     */
    NSSDOA_STAGE_PEAKS = 3,      /* low-Q FP64 re-evaluation and Step-6                        */
    NSSDOA_STAGE_PROPOSAL = 4,   /* windowed estimation: features, network, windows            */
    NSSDOA_STAGE_COUNT = 5
} nssdoa_stage;

/* Create a plan holding array geometries and scan grids (host work only, no device call).
 * arrays[n_arrays] and grids[n_grids] are host arrays, copied.  options may be NULL.
 * EINVAL: NULL plan/arrays/grids, n_arrays or n_grids < 1, M < 2 or M > 64, L < 3,
 * step <= 0 or non-finite, non-finite positions, an option out of its stated range. */
nssdoa_status nssdoa_plan_create(nssdoa_plan* plan, const nssdoa_array* arrays, int32_t n_arrays,
                                 const nssdoa_grid* grids, int32_t n_grids,
                                 const nssdoa_options* options);

/* Free a plan.  Every batch created from it must have been destroyed first (ESTATE otherwise).
 * NULL is accepted and ignored. */
nssdoa_status nssdoa_plan_destroy(nssdoa_plan plan);

/* Validate a set of frames for one algorithm and scan precision, group the frames that share an
 * array and a grid, and upload the schedule to the current device (the batch owns it).  For
 * C64 it also computes, once, the steering vectors of every group's grid (Eq. 2) into a table the
 * batch owns: (L rounded up to 256, plus 64) * 2M floats per group; the call waits for them. 
 * frames[n_frames] is a host array, copied.  max_D is the peak slots per frame in the outputs.
 * EINVAL: NULL pointers, n_frames < 1, unknown array/grid ids, N < 1, D < 1, D >= M, D > max_D,
 * ldx < N, negative offsets, max_D > 64, a grid longer than 4096 * floor(4096 / (D +
 * extra_candidates)) points (the peak candidate capacity); for C64, BF16 and F16 the array's M
 * must be 8, 16, 32 or 64.
 * EDEVICE/ENOMEM: device upload failed. */
nssdoa_status nssdoa_batch_create(nssdoa_batch* batch, nssdoa_plan plan, nssdoa_alg alg,
                                  nssdoa_prec prec, const nssdoa_frame* frames, int32_t n_frames,
                                  int32_t max_D);

/* Free a batch (waits for nothing: the caller must not destroy a batch whose work is in flight).
 * ESTATE while graphs captured from it or pipelines built on it exist.  NULL is accepted and
 * ignored. */
nssdoa_status nssdoa_batch_destroy(nssdoa_batch batch);

/* Bytes of device workspace nssdoa_estimate needs for this batch. */
nssdoa_status nssdoa_workspace_size(nssdoa_batch batch, size_t* bytes);

/* Byte offset, inside the workspace, of `item` for frame `frame` (see nssdoa_ws_item). */
nssdoa_status nssdoa_workspace_offset(nssdoa_batch batch, nssdoa_ws_item item, int32_t frame,
                                      size_t* offset);

/* Run Steps 1-6 for every frame of the batch on `stream`.
 *   X         device, complex64 (C64) or complex128 (C128) snapshots addressed by the frames
 *   x_elems   complex elements in X; every frame must satisfy x_off + (M-1)*ldx + N <= x_elems
 *   spectrum  device, float (C64) or double (C128); frame f's L values at frames[f].spec_off.
 *             May be NULL: the spectrum then lives in the workspace only.
 *   spectrum_elems  elements in spectrum; every frame must satisfy spec_off + L <= spectrum_elems
 *             (ignored when spectrum is NULL)
 *   peaks     device, n_frames * max_D entries, best first per frame
 *   npeaks    device, n_frames int32: number of valid peaks per frame (<= D)
 *   status    device, n_frames uint32: NSSDOA_ST_* bits
 *   workspace device, at least nssdoa_workspace_size bytes, 256-byte aligned; its contents on
 *             entry do not matter
 * EINVAL: NULL X/peaks/npeaks/status/workspace, a frame outside X or the spectrum, workspace
 * too small or not 256-byte aligned. */
nssdoa_status nssdoa_estimate(nssdoa_batch batch, const void* X, size_t x_elems, void* spectrum,
                              size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks,
                              uint32_t* status, void* workspace, size_t workspace_bytes,
                              void* stream);

/* nssdoa_estimate without a caller workspace and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace is one array of the library's code object per device,
 * of nssdoa_noalloc_workspace_limit bytes (64 MiB), held by every device the library runs on
 * until the process ends; its address on a device is looked up by the first nssdoa_batch_create
 * (or nssdoa_estimate_noalloc) call made with that device current.  The call itself allocates
 * nothing (no hipMalloc, no events) and computes exactly what nssdoa_estimate computes with the
 * same arguments.  Every call on one device shares that device's array, which keeps the last
 * call's contents: two calls that may overlap on one device (different streams, or different
 * host threads) race on it and must be serialised by the caller.  Stage timing does not apply.
 * EINVAL: as nssdoa_estimate, or a batch whose workspace (nssdoa_workspace_size) exceeds the
 * array; EDEVICE: the array's address could not be obtained. */
nssdoa_status nssdoa_estimate_noalloc(nssdoa_batch batch, const void* X, size_t x_elems, void* spectrum,
                                      size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks,
                                      uint32_t* status, void* stream);

/* Size in bytes of the workspace array of nssdoa_estimate_noalloc. */
nssdoa_status nssdoa_noalloc_workspace_limit(size_t* bytes);

/* Graph capture: record the launch sequence of one nssdoa_estimate call with these arguments
 * (validated as for nssdoa_estimate) into a HIP graph, captured on a stream of the library's own.
 * nssdoa_graph_launch replays it on `stream` as one graph launch: the same computation on the
 * same buffers, whose contents may change between launches.  No memory is allocated per launch.
 * The batch must outlive the graph (nssdoa_batch_destroy returns ESTATE while graphs of it
 * exist).  Stage timing does not apply to graph launches.
 * EINVAL: as nssdoa_estimate; EDEVICE: capture or instantiation failed. */
typedef struct nssdoa_graph_s* nssdoa_graph;
nssdoa_status nssdoa_graph_create(nssdoa_graph* graph, nssdoa_batch batch, const void* X, size_t x_elems,
                                  void* spectrum, size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks,
                                  uint32_t* status, void* workspace, size_t workspace_bytes);
nssdoa_status nssdoa_graph_launch(nssdoa_graph graph, void* stream);
nssdoa_status nssdoa_graph_destroy(nssdoa_graph graph);

/* Streaming pipeline (the continuously working system of Section 5.3, with the pinned host
 * buffers of Table 9's third step): batches of snapshots that arrive in host memory, laid out as
 * the batch's frames address them, each copied to the device, estimated and its results copied
 * back on one of `depth` slots.  A slot owns a stream, device copies of X, the workspace and the
 * outputs, and a completion event, so the copy-in of one batch overlaps the estimate of the one
 * before and the copy-out of the one before that.  Host buffers should be pinned (hipHostMalloc,
 * or a torch tensor with pin_memory): from pageable memory the copies are staged by the runtime
 * and do not overlap.
 * create: EINVAL for depth outside [1, 8]; allocates the slots (ENOMEM/EDEVICE on failure).  The
 *   batch must outlive the pipeline (nssdoa_batch_destroy returns ESTATE while it exists).
 * submit: waits on the host until the slot it takes (slots in turn) has finished its previous
 *   batch, enqueues copy-in of X_host (the batch's x extent), the estimate, and copy-out of the
 *   peaks, peak counts and status (and of the spectrum into spectrum_host unless it is NULL:
 *   nssdoa_estimate's spectrum layout, frames at their spec_off), and returns a ticket.  The host
 *   buffers of a submission must not be touched until nssdoa_pipeline_wait(ticket) returns.
 * wait: blocks until the ticket's results are in its host buffers.  EINVAL for a ticket never
 *   issued.
 * destroy: waits for every slot, then frees them. */
typedef struct nssdoa_pipeline_s* nssdoa_pipeline;
nssdoa_status nssdoa_pipeline_create(nssdoa_pipeline* pipeline, nssdoa_batch batch, int32_t depth);
nssdoa_status nssdoa_pipeline_submit(nssdoa_pipeline pipeline, const void* X_host, void* spectrum_host,
                                     nssdoa_peak* peaks_host, int32_t* npeaks_host, uint32_t* status_host,
                                     int64_t* ticket);
nssdoa_status nssdoa_pipeline_wait(nssdoa_pipeline pipeline, int64_t ticket);
nssdoa_status nssdoa_pipeline_destroy(nssdoa_pipeline pipeline);

/* Per-stage device timing.  stage_mask selects stages (bit 1 << NSSDOA_STAGE_*; 0 = off, -1 =
 * all); while set, nssdoa_estimate records HIP events around those stages on its stream (each
 * pair costs a few microseconds of stream time).  nssdoa_stage_time waits for them and returns
 * the summed milliseconds and the number of launches of `stage` since timing was (re)set. */
nssdoa_status nssdoa_set_timing(nssdoa_batch batch, int32_t stage_mask);
nssdoa_status nssdoa_stage_time(nssdoa_batch batch, nssdoa_stage stage, double* total_ms,
                                int64_t* launches);

/* ---------------------------------------------------------------------------------------------
 * Learned proposal network (not part of the paper's method: a batched front end that restricts
 * the Table 2 Step-5 scan to windows).  A 3-layer perceptron in -> width -> width -> out with
 * ReLU hidden units maps covariance features to per-bin logits; its GEMMs round operands to
 * bfloat16 and accumulate in FP32 on the matrix cores.  Parameters are FP32 (master copy) with
 * Adam moments; all of it lives in device memory owned by the nssdoa_mlp object.
 * ------------------------------------------------------------------------------------------- */
typedef struct nssdoa_mlp_s* nssdoa_mlp;

/* Allocate a network with zero parameters and zero Adam state; max_batch bounds the rows of
 * forward and training calls (activation buffers are sized for it).  The activation buffers
 * belong to the network object and every call that runs it (nssdoa_mlp_forward,
 * nssdoa_mlp_train_step, nssdoa_estimate_learned) reuses them: calls that use one network must
 * not overlap (one stream at a time, or the caller orders them); give each concurrent stream
 * its own network (nssdoa_mlp_save / nssdoa_mlp_load copy one).
 * EINVAL: NULL mlp, a size outside [1, 65536], max_batch outside [1, 2^20]. */
nssdoa_status nssdoa_mlp_create(nssdoa_mlp* mlp, int32_t in, int32_t width, int32_t out, int32_t max_batch);
nssdoa_status nssdoa_mlp_destroy(nssdoa_mlp mlp);

/* Number of parameters: width*in + width + width*width + width + out*width + out, stored in the
 * order W1 (width x in, row-major), b1, W2, b2, W3 (out x width), b3. */
nssdoa_status nssdoa_mlp_param_count(nssdoa_mlp mlp, size_t* count);

/* Checkpoint blob (host memory): eight int32 header words (magic, version, in, width, out, Adam
 * step, 0, 0) followed by the FP32 parameters, first moments and second moments, each in the
 * parameter order above.  save with blob == NULL returns the size in *bytes; otherwise *bytes
 * must be at least that size and receives it.  load requires the exact size and a matching
 * header.  Both synchronise the device.  Initial weights are loaded this way (the caller draws
 * them). */
nssdoa_status nssdoa_mlp_save(nssdoa_mlp mlp, void* blob, size_t* bytes);
nssdoa_status nssdoa_mlp_load(nssdoa_mlp mlp, const void* blob, size_t bytes);

/* Proposal features of every frame of a batch, as nssdoa_estimate_learned computes them: the
 * upper triangle i <= j of R * M / trace(R), row-major, real and imaginary parts interleaved
 * (M (M + 1) FP32 values per frame; the trace summed in index order and the scale M / trace
 * formed in FP64, each product rounded to FP32), from the covariances R (Eq. 3) that the last
 * nssdoa_estimate (or _noalloc: then pass nothing else) left in `workspace`; enqueued on `stream`,
 * so it must follow that call on the same stream.  feats: device [n_frames][n_feat] float.
 * EINVAL: NULL pointers, a workspace smaller than nssdoa_workspace_size or not 256-byte aligned,
 * n_feat != M (M + 1); EUNSUPPORTED: frames of different M. */
nssdoa_status nssdoa_features(nssdoa_batch batch, const void* workspace, size_t workspace_bytes, float* feats,
                              int32_t n_feat, void* stream);

/* Alternative forms of the Step-5 scan, as measured ablations of the factored form: after
 * nssdoa_estimate on `workspace`, the spectrum of every frame again, in plain FP32 on the vector
 * ALUs and without the FP64 re-evaluation of low-Q points, with Q formed as
 *   NSSDOA_FORM_FACTORED:   ||B^H a||^2 (the library's form, a sum of squares);
 *   NSSDOA_FORM_QUADRATIC:  Re a^H C a, C = B B^H formed in FP64 then rounded to FP32 (Table 2
 *                           Step-5 as printed: M^2 terms that cancel down to Q near a null);
 *   NSSDOA_FORM_COMPLEMENT: ||a||^2 - ||E_s^H a||^2 with the D signal eigenvectors (MUSIC only).
 * P = 1 / max(Q, FLT_MIN) is written to `spectrum` (float) at each frame's spec_off; steering
 * vectors are FP32 values of phases reduced in FP64.  Peaks are not searched.
 * EINVAL: NULL pointers, an unknown form, a workspace or spectrum smaller than the batch needs;
 * EUNSUPPORTED: a batch that is not NSSDOA_C64, has 2-D grids or M > 32, or the complement form
 * for another method than MUSIC. */
typedef enum { NSSDOA_FORM_FACTORED = 0, NSSDOA_FORM_QUADRATIC = 1, NSSDOA_FORM_COMPLEMENT = 2 } nssdoa_scan_form_kind;
nssdoa_status nssdoa_scan_form(nssdoa_batch batch, int32_t form, const void* workspace, size_t workspace_bytes,
                               float* spectrum, size_t spectrum_elems, void* stream);

/* Logits of `batch` feature rows: feats device [batch][in] FP32, logits device [batch][out]. */
nssdoa_status nssdoa_mlp_forward(nssdoa_mlp mlp, const float* feats, int32_t batch, float* logits,
                                 void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the mean binary
 * cross-entropy with logits between the network output and `targets` (device [batch][out], 0/1).
 * loss: device, one float, receives the loss before the update.  EINVAL: NULL pointers, batch
 * outside [1, max_batch], lr outside [0, 1e3). */
nssdoa_status nssdoa_mlp_train_step(nssdoa_mlp mlp, const float* feats, const float* targets,
                                    int32_t batch, float lr, float* loss, void* stream);

/* Host copy of the gradients of the last training step (count = nssdoa_mlp_param_count). */
nssdoa_status nssdoa_mlp_gradients(nssdoa_mlp mlp, float* host, size_t count);

/* ---------------------------------------------------------------------------------------------
 * Windowed estimation: Steps 1-4 for every frame as in nssdoa_estimate, then the Step-5 scan and
 * the Step-6 peak search only inside angle windows proposed from per-bin scores.
 *
 * Bins: n_bins bins of width w = 180 / n_bins deg; bin b covers [-90 + b w, -90 + (b+1) w) and its
 * centre is c_b = -90 + (b + 1/2) w.  Per frame the topk best scores (ties to the lower bin; NaN
 * never chosen; after the frame's first D bins only those scoring at least the window floor; with
 * local_max_bins != 0 only local maxima of the score curve: a bin above its left neighbour whose run
 * of equal scores ends lower or at the last bin, NaN counting as -inf) give
 * windows [c_b - half_window_deg, c_b + half_window_deg], snapped inward to the
 * frame's grid: grid indices ceil((c_b - hw - start) / step - 1e-9) .. floor((c_b + hw - start) /
 * step + 1e-9), clipped to [0, L), each operation rounded in FP64; overlapping or touching windows
 * merge.  If the frame's best score is below the threshold (or NaN) the frame falls back to one
 * window over its whole grid and gets NSSDOA_ST_FALLBACK_USED.  Windows never wrap around a
 * circular grid.  A frame whose windows hold fewer than D peaks (a proposal that missed a source,
 * or a peak whose plateau reaches a window's end) is searched again, on the device within the same
 * call, with one window over its whole grid, and also gets NSSDOA_ST_FALLBACK_USED: its peaks are
 * then those of the whole grid.
 * Within the windows everything is as in nssdoa_estimate (FP32 scan, FP64 re-evaluation of
 * low-Q points, FP64 re-pick around the candidates) except that spectrum values outside every
 * window are unknown: the first and last points of a window are never peaks, and a peak's
 * neighbours and plateau must lie inside its window.  Spectrum values outside the windows are
 * not written; a frame with NSSDOA_ST_NONFINITE_INPUT gets no windows and no spectrum values.
 *
 * Requirements beyond nssdoa_estimate (EUNSUPPORTED otherwise): the batch was created with
 * NSSDOA_C64, and all its frames have the same M.  EINVAL: topk outside [1, 16], n_bins outside
 * [1, 256], half_window_deg outside (0, 180], a NaN threshold, a frame whose grid of L points
 * gives (ceil(L / 4096) + topk) * (D + extra_candidates) > 4096 candidate slots, a workspace
 * smaller than nssdoa_windowed_workspace_size.
 * ------------------------------------------------------------------------------------------- */

/* Bytes of device workspace windowed estimation needs for this batch: with mlp == NULL for
 * nssdoa_estimate_windowed, with the network for nssdoa_estimate_learned. */
nssdoa_status nssdoa_windowed_workspace_size(nssdoa_batch batch, nssdoa_mlp mlp, size_t* bytes);

/* Windowed estimation with caller scores: scores is device [n_frames][n_bins] float, row f for
 * frame f; a frame falls back to the full grid when its best score < score_threshold; a chosen bin
 * beyond the frame's first D gets a window only when its score >= window_floor (-INFINITY: every
 * one of the topk; EINVAL if NaN).  The other arguments are those of nssdoa_estimate. */
nssdoa_status nssdoa_estimate_windowed(nssdoa_batch batch, const void* X, size_t x_elems, const float* scores,
                                       int32_t n_bins, int32_t topk, double half_window_deg,
                                       float score_threshold, float window_floor, int32_t local_max_bins,
                                       void* spectrum, size_t spectrum_elems, nssdoa_peak* peaks,
                                       int32_t* npeaks, uint32_t* status, void* workspace, size_t workspace_bytes,
                                       void* stream);

/* Windowed estimation with the learned proposal: per frame the features (upper triangle i <= j
 * of R * M / trace(R), row-major, real and imaginary parts interleaved: M (M + 1) values, which
 * must equal the network's input size) go through the network; its outputs are the bin logits
 * (n_bins = the network's output size).  A frame falls back to the full grid when
 * sigmoid(best logit) < fallback_score, i.e. best logit < log(p / (1 - p)); fallback_score in
 * [0, 1] (0: never, 1: always).  A chosen bin beyond the frame's first D gets a window only when
 * sigmoid(its logit) >= window_score, in [0, 1] (0: every one of the topk); local_max_bins as for
 * nssdoa_estimate_windowed, on the logits.  The network's
 * activation buffers are reused, so two calls that use one network must not overlap. */
nssdoa_status nssdoa_estimate_learned(nssdoa_batch batch, nssdoa_mlp mlp, const void* X, size_t x_elems,
                                      int32_t topk, double half_window_deg, double fallback_score,
                                      double window_score, int32_t local_max_bins, void* spectrum,
                                      size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks,
                                      uint32_t* status, void* workspace, size_t workspace_bytes, void* stream);

/* Static description of a status code, and the last failure message on this thread. */
const char* nssdoa_status_string(nssdoa_status status);
const char* nssdoa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NSSDOA_H */
