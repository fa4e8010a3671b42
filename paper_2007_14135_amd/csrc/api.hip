// Host side of libnssdoa: argument validation, batch scheduling, workspace layout and the
// launch sequence of nssdoa_estimate.  See include/nssdoa.h for the contract of every call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nssdoa.h"
#include "internal.h"

using namespace nssdoa;

// Workspace of nssdoa_estimate_noalloc: one array per device in the library's code object, so
// that call needs no allocation.  Host code never passes `scratch` itself to a kernel (in host
// code the name is a stand-in, not a device address); it uses the address hipGetSymbolAddress
// returns for the current device, looked up once per device and kept in g_scratch_addr.
static constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

namespace {

thread_local std::string g_last_error;

nssdoa_status fail(nssdoa_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
nssdoa_status fail(nssdoa_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

}  // namespace

nssdoa_status nssdoa_internal_fail(nssdoa_status st, const char* msg) {
    g_last_error = msg;
    return st;
}

namespace {

nssdoa_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? NSSDOA_ENOMEM : NSSDOA_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

// Device address of the no-allocation workspace on the current device (looked up on the first
// call for that device, then cached).
nssdoa_status scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(NSSDOA_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0)
            return fail(NSSDOA_EDEVICE, "scratch array at an unaligned address");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return NSSDOA_OK;
}

// Grid points of a grid: L azimuths, times n_polar polar angles for a 2-D grid.
inline int64_t grid_points(const nssdoa_grid& g) { return (int64_t)g.L * std::max(1, g.n_polar); }
constexpr int64_t kMaxGrid2dPoints = (int64_t)1 << 24;
constexpr int kMaxPolar = 4096;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
inline int round_up(int v, int a) { return (v + a - 1) / a * a; }

constexpr int kChunkRows = 384;      // rows of stacked B per FP32 scan work item (12 tiles)
constexpr int kChunkRowsLP = 4096;   // rows per 16-bit scan work item (128 tiles)
constexpr int kCovTargetItems = 2048;
constexpr int64_t kLowqListMax = 1 << 22;     // entries of a batch's low-Q list
constexpr int kLowqRefineGrid = 1024;         // workgroups of the low-Q re-evaluation
constexpr double kPlateauRelScan = 1e-4;   // > the FP32 scan's relative error above the low-Q cut


}  // namespace

struct nssdoa_plan_s {
    std::vector<int32_t> M;
    std::vector<std::vector<double>> pos;
    std::vector<nssdoa_grid> grids;
    nssdoa_options opt;
    int live_batches = 0;
};

struct StageEvents {
    int stage;
    hipEvent_t a, b;
};

// Work-item order of one scan launch for the eight XCDs of the MI355X, which take workgroups
// round-robin (workgroup i runs on XCD i mod 8 up to a fixed offset) and each have their own L2:
// the angle tiles are split into eight contiguous ranges of about equal work, range x goes to
// the items at positions x, x + 8, x + 16, ..., and within a range the row chunks of one angle
// tile follow each other.  Each XCD then reads its eighth of the steering table once and keeps
// the B tiles of all chunks in its L2, instead of every chunk pass re-reading the whole table.
constexpr int kXcds = 8;
static void xcd_order(std::vector<ScanItem>& items, size_t i, size_t j) {
    if (j - i < 2 * (size_t)kXcds) return;
    std::vector<ScanItem> its(items.begin() + i, items.begin() + j);
    std::stable_sort(its.begin(), its.end(), [](const ScanItem& x, const ScanItem& y) {
        return x.group != y.group ? x.group < y.group : x.angle_tile < y.angle_tile;
    });
    const size_t total = its.size();
    std::vector<std::vector<ScanItem>> q(kXcds);
    size_t k = 0;
    for (int x = 0; x < kXcds; ++x) {
        const size_t end = total * (size_t)(x + 1) / kXcds;
        // keep an angle tile's chunks together: extend the range to the end of its tile
        size_t e = std::max(end, k);
        while (e < total && e > k && its[e].group == its[e - 1].group && its[e].angle_tile == its[e - 1].angle_tile) ++e;
        if (x == kXcds - 1) e = total;
        for (; k < e; ++k) q[x].push_back(its[k]);
    }
    std::vector<size_t> pos(kXcds, 0);
    size_t out = i;
    while (out < j) {
        for (int x = 0; x < kXcds && out < j; ++x) {
            int y = x;
            if (pos[y] >= q[y].size()) {          // this range is done: take from the fullest one
                y = 0;
                for (int z = 1; z < kXcds; ++z)
                    if (q[z].size() - pos[z] > q[y].size() - pos[y]) y = z;
            }
            items[out++] = q[y][pos[y]++];
        }
    }
}

struct nssdoa_batch_s {
    nssdoa_plan plan = nullptr;
    nssdoa_alg alg;
    nssdoa_prec prec;
    int32_t n_frames = 0, max_D = 0, max_M = 0;
    std::vector<FrameDev> frames;
    std::vector<GroupDev> groups;
    std::vector<CovItem> cov_items;
    std::vector<ScanItem> scan_items;           // sorted by group M
    std::vector<std::pair<int, std::pair<int, int>>> scan_ranges;   // M -> [begin, end)
    std::vector<int> scan_max_tiles;                                // per range: largest t1 - t0
    std::vector<PointItem> point_items;
    std::vector<int32_t> blk;
    std::vector<double> pos;
    std::vector<int32_t> peak_list;             // frames grouped by M bucket (8, 16, 32, 64)
    std::vector<std::pair<int, std::pair<int, int>>> peak_ranges;   // bucket M -> [begin, end)
    std::vector<PointItem> refine_items;        // (frame, chunk start), grouped like peak_list
    std::vector<std::pair<int, int>> refine_ranges;                 // per bucket [begin, end)
    std::vector<int> peak_selcap;               // per bucket: candidate slots of its largest frame
    // 2-D grids: frames (in peak_list, after the 1-D ones) and 256-point items (in refine_items)
    std::vector<std::pair<int, std::pair<int, int>>> p2d_ranges;    // bucket M -> [begin, end) of peak_list
    std::vector<std::pair<int, int>> p2d_iranges;                   // per bucket [begin, end) of refine_items
    bool any2d = false;
    size_t ws_bytes = 0;
    int64_t ws_lowq_all = -1;                   // the scans' low-Q list (count, then cap entries)
    int32_t lowq_all_cap = 0;
    size_t spec_elem = 4;
    size_t x_extent = 0;       // complex elements of X the frames address
    size_t spec_extent = 0;    // elements of the caller's spectrum the frames address
    // device copies
    char* dev = nullptr;
    FrameDev* d_frames = nullptr;
    GroupDev* d_groups = nullptr;
    CovItem* d_cov = nullptr;
    ScanItem* d_scan = nullptr;
    PointItem* d_points = nullptr;
    int32_t* d_blk = nullptr;
    double* d_pos = nullptr;
    int32_t* d_plist = nullptr;
    PointItem* d_refine = nullptr;
    double2* d_cis = nullptr;
    float* d_steer = nullptr;                   // steering tables of the C64 scans (batch-owned)
    int split_parts = 0;                        // C64 scans on FP16 split operands of 2 or 3 parts (0: FP32)
    int live_graphs = 0;                        // graphs and pipelines that use the batch
    // timing
    uint32_t timing = 0;                        // stages with HIP events (bit 1 << stage)
    std::vector<StageEvents> pending;
    double stage_ms[NSSDOA_STAGE_COUNT] = {0, 0, 0, 0};
    int64_t stage_n[NSSDOA_STAGE_COUNT] = {0, 0, 0, 0};
};

extern "C" {

const char* nssdoa_status_string(nssdoa_status s) {
    switch (s) {
        case NSSDOA_OK: return "ok";
        case NSSDOA_EINVAL: return "invalid argument";
        case NSSDOA_EUNSUPPORTED: return "unsupported";
        case NSSDOA_ENOMEM: return "out of memory";
        case NSSDOA_EDEVICE: return "device error";
        case NSSDOA_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char* nssdoa_last_error(void) { return g_last_error.c_str(); }

nssdoa_status nssdoa_plan_create(nssdoa_plan* plan, const nssdoa_array* arrays, int32_t n_arrays,
                                 const nssdoa_grid* grids, int32_t n_grids,
                                 const nssdoa_options* options) {
    if (!plan) return fail(NSSDOA_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!arrays || n_arrays < 1) return fail(NSSDOA_EINVAL, "need at least one array");
    if (!grids || n_grids < 1) return fail(NSSDOA_EINVAL, "need at least one grid");
    nssdoa_options opt;
    opt.eig_tol = 1e-15;
    opt.eig_max_iter = 30;
    opt.refine_halfwidth = 4;
    opt.lowq_tau = 5e-4;
    opt.extra_candidates = 4;
    opt.scan_rows = 0;
    opt.eig_method = NSSDOA_EIG_AUTO;
    opt.c64_scan = NSSDOA_C64_SCAN_SPLIT16X3;
    if (options) {
        opt = *options;
        if (!(opt.eig_tol > 0.0 && opt.eig_tol < 1.0))
            return fail(NSSDOA_EINVAL, "eig_tol must be in (0, 1)");
        if (opt.eig_max_iter < 1 || opt.eig_max_iter > 1000)
            return fail(NSSDOA_EINVAL, "eig_max_iter must be in [1, 1000]");
        if (opt.eig_method != NSSDOA_EIG_AUTO && opt.eig_method != NSSDOA_EIG_QL && opt.eig_method != NSSDOA_EIG_JACOBI)
            return fail(NSSDOA_EINVAL, "eig_method must be NSSDOA_EIG_AUTO, NSSDOA_EIG_QL or NSSDOA_EIG_JACOBI");
        if (opt.refine_halfwidth < 1 || opt.refine_halfwidth > 16)
            return fail(NSSDOA_EINVAL, "refine_halfwidth must be in [1, 16]");
        if (!(opt.lowq_tau >= 0.0) || !isfinite(opt.lowq_tau))
            return fail(NSSDOA_EINVAL, "lowq_tau must be finite and >= 0");
        if (opt.extra_candidates < 0 || opt.extra_candidates > 16)
            return fail(NSSDOA_EINVAL, "extra_candidates must be in [0, 16]");
        if (opt.scan_rows != 0 && (opt.scan_rows < 32 || opt.scan_rows > 16384 || opt.scan_rows % 32 != 0))
            return fail(NSSDOA_EINVAL, "scan_rows must be 0 or a multiple of 32 in [32, 16384]");
        if (opt.c64_scan != NSSDOA_C64_SCAN_SPLIT16 && opt.c64_scan != NSSDOA_C64_SCAN_FP32 &&
            opt.c64_scan != NSSDOA_C64_SCAN_SPLIT16X3)
            return fail(NSSDOA_EINVAL, "c64_scan must be NSSDOA_C64_SCAN_SPLIT16X3, _FP32 or _SPLIT16");
    }
    auto* p = new (std::nothrow) nssdoa_plan_s();
    if (!p) return fail(NSSDOA_ENOMEM, "host allocation failed");
    for (int a = 0; a < n_arrays; ++a) {
        const nssdoa_array& ar = arrays[a];
        if (ar.M < 2 || ar.M > 64) {
            delete p;
            return fail(NSSDOA_EINVAL, "array %d: M=%d outside [2, 64]", a, ar.M);
        }
        if (!ar.pos_wl || ar.reserved != 0) {
            delete p;
            return fail(NSSDOA_EINVAL, "array %d: NULL positions or nonzero reserved", a);
        }
        std::vector<double> v(ar.pos_wl, ar.pos_wl + 3 * ar.M);
        for (double x : v)
            if (!isfinite(x)) {
                delete p;
                return fail(NSSDOA_EINVAL, "array %d: non-finite position", a);
            }
        p->M.push_back(ar.M);
        p->pos.push_back(std::move(v));
    }
    for (int g = 0; g < n_grids; ++g) {
        const nssdoa_grid& gr = grids[g];
        if (gr.L < 3) {
            delete p;
            return fail(NSSDOA_EINVAL, "grid %d: L=%d < 3", g, gr.L);
        }
        if (!(gr.step_deg > 0.0) || !isfinite(gr.step_deg) || !isfinite(gr.start_deg)) {
            delete p;
            return fail(NSSDOA_EINVAL, "grid %d: step must be finite and > 0", g);
        }
        if (gr.reserved != 0 || gr.n_polar < 0 || gr.n_polar > kMaxPolar) {
            delete p;
            return fail(NSSDOA_EINVAL, "grid %d: n_polar=%d outside [0, %d] or nonzero reserved", g, gr.n_polar,
                        kMaxPolar);
        }
        if (gr.n_polar > 0) {
            if (!(gr.polar_step_deg > 0.0) || !isfinite(gr.polar_step_deg) || !isfinite(gr.polar_start_deg)) {
                delete p;
                return fail(NSSDOA_EINVAL, "grid %d: polar step must be finite and > 0", g);
            }
            if (grid_points(gr) > kMaxGrid2dPoints) {
                delete p;
                return fail(NSSDOA_EINVAL, "grid %d: %lld points exceed the 2-D grid limit of %lld", g,
                            (long long)grid_points(gr), (long long)kMaxGrid2dPoints);
            }
        }
        p->grids.push_back(gr);
    }
    p->opt = opt;
    *plan = p;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_plan_destroy(nssdoa_plan plan) {
    if (!plan) return NSSDOA_OK;
    if (plan->live_batches > 0)
        return fail(NSSDOA_ESTATE, "plan still has %d live batches", plan->live_batches);
    delete plan;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_batch_destroy(nssdoa_batch batch) {
    if (!batch) return NSSDOA_OK;
    if (batch->live_graphs > 0)
        return fail(NSSDOA_ESTATE, "batch still has %d live graphs or pipelines", batch->live_graphs);
    for (auto& e : batch->pending) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    if (batch->dev) (void)hipFree(batch->dev);
    if (batch->plan) batch->plan->live_batches--;
    delete batch;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_batch_create(nssdoa_batch* out, nssdoa_plan plan, nssdoa_alg alg,
                                  nssdoa_prec prec, const nssdoa_frame* frames, int32_t n_frames,
                                  int32_t max_D) {
    if (!out) return fail(NSSDOA_EINVAL, "batch is NULL");
    *out = nullptr;
    if (!plan) return fail(NSSDOA_EINVAL, "plan is NULL");
    if (!frames || n_frames < 1) return fail(NSSDOA_EINVAL, "need at least one frame");
    if (alg < NSSDOA_PHD || alg > NSSDOA_MN) return fail(NSSDOA_EINVAL, "unknown algorithm %d", (int)alg);
    if (prec < NSSDOA_C128 || prec > NSSDOA_F16) return fail(NSSDOA_EINVAL, "unknown precision %d", (int)prec);
    if (max_D < 1 || max_D > 64) return fail(NSSDOA_EINVAL, "max_D=%d outside [1, 64]", max_D);
    const int n_arr = (int)plan->M.size(), n_grid = (int)plan->grids.size();
    for (int f = 0; f < n_frames; ++f) {
        const nssdoa_frame& fr = frames[f];
        if (fr.array_id < 0 || fr.array_id >= n_arr)
            return fail(NSSDOA_EINVAL, "frame %d: unknown array_id %d", f, fr.array_id);
        if (fr.grid_id < 0 || fr.grid_id >= n_grid)
            return fail(NSSDOA_EINVAL, "frame %d: unknown grid_id %d", f, fr.grid_id);
        const int M = plan->M[fr.array_id];
        if (fr.N < 1) return fail(NSSDOA_EINVAL, "frame %d: N=%d < 1", f, fr.N);
        if (fr.D < 1 || fr.D >= M) return fail(NSSDOA_EINVAL, "frame %d: D=%d outside [1, M-1] (M=%d)", f, fr.D, M);
        if (fr.D > max_D) return fail(NSSDOA_EINVAL, "frame %d: D=%d > max_D=%d", f, fr.D, max_D);
        if (fr.ldx < fr.N) return fail(NSSDOA_EINVAL, "frame %d: ldx < N", f);
        if (fr.x_off < 0 || fr.spec_off < 0) return fail(NSSDOA_EINVAL, "frame %d: negative offset", f);
        if (plan->grids[fr.grid_id].n_polar > 0) {
            if (prec != NSSDOA_C64 && prec != NSSDOA_C128)
                return fail(NSSDOA_EUNSUPPORTED, "frame %d: 2-D grids need NSSDOA_C64 or NSSDOA_C128", f);
        } else {
            const int64_t L = plan->grids[fr.grid_id].L;
            const int64_t slots = (L + kRefineChunk - 1) / kRefineChunk * (fr.D + plan->opt.extra_candidates);
            if (slots > kSelCap)
                return fail(NSSDOA_EINVAL, "frame %d: grid of %lld points with D + extra_candidates = %d "
                            "exceeds the peak candidate capacity (%d slots of %d-point chunks)", f,
                            (long long)L, fr.D + plan->opt.extra_candidates, kSelCap, kRefineChunk);
        }
        if (prec != NSSDOA_C128 && M != 8 && M != 16 && M != 32 && M != 64)
            return fail(NSSDOA_EINVAL, "frame %d: the matrix-core scans need M in {8, 16, 32, 64} (M=%d)", f, M);
    }

    auto* b = new (std::nothrow) nssdoa_batch_s();
    if (!b) return fail(NSSDOA_ENOMEM, "host allocation failed");
    b->plan = plan;
    b->alg = alg;
    b->prec = prec;
    b->n_frames = n_frames;
    b->max_D = max_D;
    b->spec_elem = prec == NSSDOA_C128 ? sizeof(double) : sizeof(float);
    b->split_parts = prec != NSSDOA_C64 ? 0 : plan->opt.c64_scan == NSSDOA_C64_SCAN_SPLIT16 ? 2
                   : plan->opt.c64_scan == NSSDOA_C64_SCAN_SPLIT16X3 ? 3 : 0;

    // positions table (one copy per array)
    std::vector<int> pos_off(n_arr);
    for (int a = 0; a < n_arr; ++a) {
        pos_off[a] = (int)b->pos.size();
        b->pos.insert(b->pos.end(), plan->pos[a].begin(), plan->pos[a].end());
    }

    // groups: frames sharing (array, grid), in order of first appearance
    std::map<std::pair<int, int>, int> gid;
    std::vector<std::vector<int>> gframes;
    b->frames.resize(n_frames);
    for (int f = 0; f < n_frames; ++f) {
        const nssdoa_frame& in = frames[f];
        auto key = std::make_pair(in.array_id, in.grid_id);
        auto it = gid.find(key);
        int g;
        if (it == gid.end()) {
            g = (int)b->groups.size();
            gid[key] = g;
            GroupDev gd;
            memset(&gd, 0, sizeof(gd));
            const nssdoa_grid& gr = plan->grids[in.grid_id];
            gd.M = plan->M[in.array_id];
            gd.L = (int32_t)grid_points(gr);
            gd.pos_off = pos_off[in.array_id];
            gd.grid_start = gr.start_deg;
            gd.grid_step = gr.step_deg;
            gd.is2d = gr.n_polar > 0;
            gd.n_az = gr.L;
            gd.el_start = gr.n_polar > 0 ? gr.polar_start_deg : 90.0;
            gd.el_step = gr.n_polar > 0 ? gr.polar_step_deg : 0.0;
            b->groups.push_back(gd);
            gframes.emplace_back();
        } else {
            g = it->second;
        }
        gframes[g].push_back(f);
        FrameDev& fd = b->frames[f];
        memset(&fd, 0, sizeof(fd));
        const nssdoa_grid& gr = plan->grids[in.grid_id];
        fd.M = plan->M[in.array_id];
        fd.N = in.N;
        fd.D = in.D;
        fd.K = (alg == NSSDOA_MUSIC || alg == NSSDOA_EV) ? fd.M - in.D : 1;
        fd.group = g;
        fd.x_off = in.x_off;
        fd.ldx = in.ldx;
        fd.spec_off_user = in.spec_off;
        fd.grid_start = gr.start_deg;
        fd.grid_step = gr.step_deg;
        fd.L = (int32_t)grid_points(gr);
        fd.circular = gr.circular ? 1 : 0;
        fd.is2d = gr.n_polar > 0;
        fd.n_az = gr.L;
        fd.el_start = gr.n_polar > 0 ? gr.polar_start_deg : 90.0;
        fd.el_step = gr.n_polar > 0 ? gr.polar_step_deg : 0.0;
        fd.pos_off = pos_off[in.array_id];
        fd.alg = (int32_t)alg;
        b->max_M = std::max(b->max_M, fd.M);
        b->x_extent = std::max(b->x_extent, (size_t)(in.x_off + (int64_t)(fd.M - 1) * in.ldx + in.N));
        b->spec_extent = std::max(b->spec_extent, (size_t)(in.spec_off + grid_points(gr)));
    }

    // covariance chunks over snapshots
    const int S_target = std::max(1, (kCovTargetItems + n_frames - 1) / n_frames);
    for (int f = 0; f < n_frames; ++f) {
        FrameDev& fd = b->frames[f];
        const int S = std::max(1, std::min(S_target, fd.N / 256));
        const int len = (fd.N + S - 1) / S;
        int c = 0;
        for (int n0 = 0; n0 < fd.N; n0 += len, ++c) b->cov_items.push_back({f, c, n0, std::min(fd.N, n0 + len)});
        fd.n_chunks = c;
    }

    // workspace: per-frame regions, then per-group packed B tiles, then the spectrum
    size_t off = 0;
    for (int f = 0; f < n_frames; ++f) {
        FrameDev& fd = b->frames[f];
        const size_t MM = (size_t)fd.M * fd.M;
        fd.ws_partial = (int64_t)off; off = align_up(off + (size_t)fd.n_chunks * MM * 16);
        fd.ws_R = (int64_t)off;       off = align_up(off + MM * 16);
        fd.ws_evals = (int64_t)off;   off = align_up(off + (size_t)fd.M * 8);
        fd.ws_evecs = (int64_t)off;   off = align_up(off + MM * 16);
        fd.ws_B = (int64_t)off;       off = align_up(off + (size_t)fd.M * fd.K * 16);
        fd.ws_qref = (int64_t)off;    off = align_up(off + 16);   // ||B||_F^2, then the FP16 split Q scale
        // candidate chunks: one per 4096 grid points, plus one per window of windowed estimation
        const int n_chunks = (fd.L + kRefineChunk - 1) / kRefineChunk + kMaxWindows;
        fd.ws_cand = (int64_t)off;
        if (fd.is2d)   // the FP64 peak map of a 2-D grid
            off = align_up(off + (size_t)fd.L * sizeof(double));
        else
            off = align_up(off + (size_t)n_chunks * (fd.D + plan->opt.extra_candidates) * 16);
        if (prec != NSSDOA_C128) {
            // low-Q list: room for an eighth of the grid (at least 256 points); a frame with more
            // low-Q points re-evaluates them in its local-maximum pass instead
            fd.lowq_cap = round_up(std::max(256, fd.L / 8), 256);
            fd.ws_lowq = (int64_t)off;  off = align_up(off + (size_t)(fd.lowq_cap + 1) * 4);
        }
    }
    if (prec != NSSDOA_C128) {
        // the matrix-core scans' list of low-Q points: an int count (padded to 256 bytes), then
        // (frame, grid index) pairs; its capacity is the sum of the frames' list capacities, at
        // most kLowqListMax (points beyond it are re-evaluated by their frame's peak search)
        int64_t cap = 0;
        for (const FrameDev& fd : b->frames) cap += fd.lowq_cap;
        b->lowq_all_cap = (int32_t)std::min<int64_t>(cap, kLowqListMax);
        b->ws_lowq_all = (int64_t)off;
        off = align_up(off + 256 + (size_t)b->lowq_all_cap * sizeof(int2));
    }
    int64_t steer_floats = 0;
    for (auto& gd : b->groups) gd.steer_off = gd.steer_x16_off = -1;
    if (prec != NSSDOA_C128) {
        const bool lp = prec != NSSDOA_C64;
        // rows of stacked B per scan work item: the 16-bit scans form their steering operands
        // per work item at a cost comparable to 64 tiles of their MFMA work, so they take
        // longer chunks
        const int chunk_rows_req = plan->opt.scan_rows > 0 ? plan->opt.scan_rows : lp ? kChunkRowsLP : kChunkRows;
        // bytes per operand value: 16-bit, FP32, or P FP16 parts
        const size_t emb_elem = lp ? 2 : b->split_parts ? 2 * b->split_parts : sizeof(float);
        for (size_t g = 0; g < b->groups.size(); ++g) {
            GroupDev& gd = b->groups[g];
            // the FP32 scan stages a work item's rows in LDS (8M bytes per row); the FP16 split
            // scan keeps only its per-block tables there (kScanMaxBlocks 8-row blocks)
            const int chunk_rows = lp ? chunk_rows_req
                                 : b->split_parts ? std::min(chunk_rows_req, kScanMaxBlocks * 8)
                                              : std::min(chunk_rows_req, (int)(kScanLdsBytes / (8 * gd.M)) / 32 * 32);
            int row = 0, chunk_start = 0, chunk_frames = 0;
            std::vector<std::pair<int, int>> chunks;
            int last_f = -1;
            for (int f : gframes[g]) {
                FrameDev& fd = b->frames[f];
                const int rows = round_up(2 * fd.K, 8);
                if (chunk_frames > 0 && (row - chunk_start) + rows > chunk_rows) {
                    const int end = round_up(row, 32);
                    b->frames[last_f].emb_rows += end - row;   // the last frame zero-fills the tail
                    chunks.push_back({chunk_start / 32, end / 32});
                    row = chunk_start = end;
                    chunk_frames = 0;
                }
                fd.emb_row0 = row;
                fd.emb_rows = rows;
                row += rows;
                ++chunk_frames;
                last_f = f;
            }
            const int end = round_up(row, 32);
            b->frames[last_f].emb_rows += end - row;
            chunks.push_back({chunk_start / 32, end / 32});
            gd.n_tiles = end / 32;
            gd.blk_off = (int)b->blk.size();
            b->blk.resize(b->blk.size() + (size_t)gd.n_tiles * 4, -1);
            for (int f : gframes[g]) {
                const FrameDev& fd = b->frames[f];
                for (int r = fd.emb_row0; r < fd.emb_row0 + round_up(2 * fd.K, 8); r += 8)
                    b->blk[gd.blk_off + r / 8] = f;
            }
            gd.ws_emb = (int64_t)off;
            off = align_up(off + (size_t)gd.n_tiles * 64 * gd.M * emb_elem);
            if (!lp) {
                gd.steer_off = steer_floats;
                steer_floats += (steer_table_floats(gd.M, gd.L) + 63) / 64 * 64;
                if (b->split_parts) {   // P FP16 parts: P / 2 times the bytes of the FP32 table
                    gd.steer_x16_off = steer_floats;
                    steer_floats += (steer_table_floats(gd.M, gd.L) * b->split_parts / 2 + 63) / 64 * 64;
                }
            }
            const int n_at = (gd.L + kScanAnglesPerWG - 1) / kScanAnglesPerWG;
            for (auto& ch : chunks)
                for (int at = 0; at < n_at; ++at)
                    b->scan_items.push_back({(int)g, at, ch.first, ch.second});
        }
        std::stable_sort(b->scan_items.begin(), b->scan_items.end(),
                         [&](const ScanItem& x, const ScanItem& y) { return b->groups[x.group].M < b->groups[y.group].M; });
        for (size_t i = 0; i < b->scan_items.size();) {
            const int M = b->groups[b->scan_items[i].group].M;
            size_t j = i;
            while (j < b->scan_items.size() && b->groups[b->scan_items[j].group].M == M) ++j;
            xcd_order(b->scan_items, i, j);
            b->scan_ranges.push_back({M, {(int)i, (int)j}});
            int mt = 0;
            for (size_t k = i; k < j; ++k) mt = std::max(mt, b->scan_items[k].t1 - b->scan_items[k].t0);
            b->scan_max_tiles.push_back(mt);
            i = j;
        }
    } else {
        for (int f = 0; f < n_frames; ++f)
            for (int l0 = 0; l0 < b->frames[f].L; l0 += 256) b->point_items.push_back({f, l0});
    }
    for (int f = 0; f < n_frames; ++f) {
        b->frames[f].spec_off_ws = (int64_t)((off - 0) / b->spec_elem);
        off += (size_t)b->frames[f].L * b->spec_elem;
    }
    off = align_up(off);
    b->ws_bytes = off;
    // the internal spectrum offsets above are relative to the workspace base in elements
    // (the region is aligned to the element size because every earlier region is 256-aligned)

    // frame lists and refine work items by M bucket
    for (int mb : {8, 16, 32, 64}) {
        const int begin = (int)b->peak_list.size();
        const int ibegin = (int)b->refine_items.size();
        for (int f = 0; f < n_frames; ++f) {
            const int M = b->frames[f].M;
            const int bucket = M <= 8 ? 8 : M <= 16 ? 16 : M <= 32 ? 32 : 64;
            if (bucket != mb || b->frames[f].is2d) continue;
            b->peak_list.push_back(f);
            for (int l0 = 0; l0 < b->frames[f].L; l0 += kRefineChunk) b->refine_items.push_back({f, l0});
        }
        if ((int)b->peak_list.size() > begin) {
            b->peak_ranges.push_back({mb, {begin, (int)b->peak_list.size()}});
            b->refine_ranges.push_back({ibegin, (int)b->refine_items.size()});
            // candidate slots per frame: (4096-point chunks + windows) x (D + extra), as ws_cand
            int cap = 1;
            for (int i = begin; i < (int)b->peak_list.size(); ++i) {
                const FrameDev& fd = b->frames[b->peak_list[i]];
                const int nch = (fd.L + kRefineChunk - 1) / kRefineChunk + kMaxWindows;
                cap = std::max(cap, nch * (fd.D + plan->opt.extra_candidates));
            }
            b->peak_selcap.push_back(std::min(cap, kSelCap));
        }
    }
    for (int mb : {8, 16, 32, 64}) {
        const int begin = (int)b->peak_list.size();
        const int ibegin = (int)b->refine_items.size();
        for (int f = 0; f < n_frames; ++f) {
            const int M = b->frames[f].M;
            const int bucket = M <= 8 ? 8 : M <= 16 ? 16 : M <= 32 ? 32 : 64;
            if (bucket != mb || !b->frames[f].is2d) continue;
            b->peak_list.push_back(f);
            for (int l0 = 0; l0 < b->frames[f].L; l0 += kPeak2dItem) b->refine_items.push_back({f, l0});
        }
        if ((int)b->peak_list.size() > begin) {
            b->p2d_ranges.push_back({mb, {begin, (int)b->peak_list.size()}});
            b->p2d_iranges.push_back({ibegin, (int)b->refine_items.size()});
            b->any2d = true;
        }
    }

    // upload the schedule
    size_t o_frames = 0;
    size_t o_groups = align_up(o_frames + b->frames.size() * sizeof(FrameDev));
    size_t o_cov = align_up(o_groups + b->groups.size() * sizeof(GroupDev));
    size_t o_scan = align_up(o_cov + b->cov_items.size() * sizeof(CovItem));
    size_t o_pts = align_up(o_scan + b->scan_items.size() * sizeof(ScanItem));
    size_t o_blk = align_up(o_pts + b->point_items.size() * sizeof(PointItem));
    size_t o_pos = align_up(o_blk + b->blk.size() * sizeof(int32_t));
    size_t o_pl = align_up(o_pos + b->pos.size() * sizeof(double));
    size_t o_ri = align_up(o_pl + b->peak_list.size() * sizeof(int32_t));
    size_t o_cis = align_up(o_ri + b->refine_items.size() * sizeof(PointItem));
    const size_t o_steer = align_up(o_cis + kCisTable * sizeof(double2));
    const size_t n_host = o_steer;                       // tables uploaded from the host
    size_t total = align_up(o_steer + (size_t)steer_floats * sizeof(float));
    std::vector<char> host(n_host, 0);
    auto put = [&](size_t o, const void* src, size_t n) { if (n) memcpy(host.data() + o, src, n); };
    put(o_frames, b->frames.data(), b->frames.size() * sizeof(FrameDev));
    put(o_groups, b->groups.data(), b->groups.size() * sizeof(GroupDev));
    put(o_cov, b->cov_items.data(), b->cov_items.size() * sizeof(CovItem));
    put(o_scan, b->scan_items.data(), b->scan_items.size() * sizeof(ScanItem));
    put(o_pts, b->point_items.data(), b->point_items.size() * sizeof(PointItem));
    put(o_blk, b->blk.data(), b->blk.size() * sizeof(int32_t));
    put(o_pos, b->pos.data(), b->pos.size() * sizeof(double));
    put(o_pl, b->peak_list.data(), b->peak_list.size() * sizeof(int32_t));
    put(o_ri, b->refine_items.data(), b->refine_items.size() * sizeof(PointItem));
    {
        // exp(j 2 pi k / 256), k = -128..128, from extended-precision host sin/cos
        std::vector<double2> cis(kCisTable);
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int k = -128; k <= 128; ++k) {
            const long double a = pi * (long double)k / 128.0L;
            cis[k + 128] = make_double2((double)cosl(a), (double)sinl(a));
        }
        put(o_cis, cis.data(), cis.size() * sizeof(double2));
    }
    // set-up of nssdoa_estimate_noalloc on this device: the address of its workspace array
    void* scratch_ws = nullptr;
    nssdoa_status sst = scratch_address(&scratch_ws);
    if (sst != NSSDOA_OK) {
        delete b;
        return sst;
    }
    hipError_t e = hipMalloc((void**)&b->dev, total);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipMalloc(batch tables)");
    }
    e = hipMemcpy(b->dev, host.data(), n_host, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(b->dev);
        delete b;
        return hip_fail(e, "hipMemcpy(batch tables)");
    }
    b->d_frames = reinterpret_cast<FrameDev*>(b->dev + o_frames);
    b->d_groups = reinterpret_cast<GroupDev*>(b->dev + o_groups);
    b->d_cov = reinterpret_cast<CovItem*>(b->dev + o_cov);
    b->d_scan = reinterpret_cast<ScanItem*>(b->dev + o_scan);
    b->d_points = reinterpret_cast<PointItem*>(b->dev + o_pts);
    b->d_blk = reinterpret_cast<int32_t*>(b->dev + o_blk);
    b->d_pos = reinterpret_cast<double*>(b->dev + o_pos);
    b->d_plist = reinterpret_cast<int32_t*>(b->dev + o_pl);
    b->d_refine = reinterpret_cast<PointItem*>(b->dev + o_ri);
    b->d_cis = reinterpret_cast<double2*>(b->dev + o_cis);
    b->d_steer = reinterpret_cast<float*>(b->dev + o_steer);
    // steering tables of the FP32 scans, computed once per batch on the device
    for (const GroupDev& gd : b->groups) {
        if (gd.steer_off < 0) continue;
        e = launch_steer_table(b->d_pos + gd.pos_off, gd, b->d_steer + gd.steer_off, nullptr);
        if (e == hipSuccess && gd.steer_x16_off >= 0)
            e = launch_steer_table_split16(b->split_parts, b->d_pos + gd.pos_off, gd, b->d_steer + gd.steer_x16_off,
                                           nullptr);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        (void)hipFree(b->dev);
        delete b;
        return hip_fail(e, "steering tables");
    }
    plan->live_batches++;
    *out = b;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_workspace_size(nssdoa_batch batch, size_t* bytes) {
    if (!batch || !bytes) return fail(NSSDOA_EINVAL, "NULL argument");
    *bytes = batch->ws_bytes;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_workspace_offset(nssdoa_batch batch, nssdoa_ws_item item, int32_t frame,
                                      size_t* offset) {
    if (!batch || !offset) return fail(NSSDOA_EINVAL, "NULL argument");
    if (frame < 0 || frame >= batch->n_frames) return fail(NSSDOA_EINVAL, "frame %d out of range", frame);
    const FrameDev& fd = batch->frames[frame];
    switch (item) {
        case NSSDOA_WS_COV: *offset = (size_t)fd.ws_R; break;
        case NSSDOA_WS_EVALS: *offset = (size_t)fd.ws_evals; break;
        case NSSDOA_WS_EVECS: *offset = (size_t)fd.ws_evecs; break;
        case NSSDOA_WS_B: *offset = (size_t)fd.ws_B; break;
        case NSSDOA_WS_QREF: *offset = (size_t)fd.ws_qref; break;
        case NSSDOA_WS_SPECTRUM: *offset = (size_t)fd.spec_off_ws * batch->spec_elem; break;
        default: return fail(NSSDOA_EINVAL, "unknown workspace item %d", (int)item);
    }
    return NSSDOA_OK;
}

nssdoa_status nssdoa_set_timing(nssdoa_batch batch, int32_t stage_mask) {
    if (!batch) return fail(NSSDOA_EINVAL, "batch is NULL");
    for (auto& e : batch->pending) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    batch->pending.clear();
    for (int s = 0; s < NSSDOA_STAGE_COUNT; ++s) {
        batch->stage_ms[s] = 0.0;
        batch->stage_n[s] = 0;
    }
    batch->timing = (uint32_t)stage_mask & ((1u << NSSDOA_STAGE_COUNT) - 1u);
    return NSSDOA_OK;
}

nssdoa_status nssdoa_stage_time(nssdoa_batch batch, nssdoa_stage stage, double* total_ms,
                                int64_t* launches) {
    if (!batch || !total_ms || !launches) return fail(NSSDOA_EINVAL, "NULL argument");
    if (stage < 0 || stage >= NSSDOA_STAGE_COUNT) return fail(NSSDOA_EINVAL, "unknown stage %d", (int)stage);
    for (auto& e : batch->pending) {
        hipError_t err = hipEventSynchronize(e.b);
        if (err != hipSuccess) return hip_fail(err, "hipEventSynchronize");
        float ms = 0.0f;
        err = hipEventElapsedTime(&ms, e.a, e.b);
        if (err != hipSuccess) return hip_fail(err, "hipEventElapsedTime");
        batch->stage_ms[e.stage] += ms;
        batch->stage_n[e.stage] += 1;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    batch->pending.clear();
    *total_ms = batch->stage_ms[stage];
    *launches = batch->stage_n[stage];
    return NSSDOA_OK;
}

}  // extern "C"

namespace {

// Arguments of windowed estimation; mlp != NULL selects the learned proposal (scores are the
// network's logits of the frames' covariance features).
struct WindowArgs {
    nssdoa_mlp mlp;
    const float* scores;
    int32_t n_bins;
    int32_t topk;
    double half_window;
    float threshold;
    float floor;               // bins beyond a frame's first D need at least this score
    int32_t local_max;         // only local maxima of the score curve are eligible
};

size_t windowed_layout(const nssdoa_batch_s* b, int n_feat, int n_bins, LearnedLayout* lay) {
    const size_t F = (size_t)b->n_frames;
    size_t off = align_up(b->ws_bytes);
    lay->off_feat = (int64_t)off;      off = align_up(off + F * n_feat * sizeof(float));
    lay->off_scores = (int64_t)off;    off = align_up(off + F * n_bins * sizeof(float));
    lay->off_win = (int64_t)off;       off = align_up(off + F * kWinStride * sizeof(int32_t));
    lay->off_items = (int64_t)off;     off = align_up(off + F * sizeof(int32_t));
    lay->off_chunks = (int64_t)off;    off = align_up(off + F * sizeof(int32_t));
    lay->off_lowq = (int64_t)off;      off = align_up(off + F * sizeof(int32_t));
    lay->off_item_off = (int64_t)off;  off = align_up(off + (F + 1) * sizeof(int32_t));
    lay->off_chunk_off = (int64_t)off; off = align_up(off + (F + 1) * sizeof(int32_t));
    lay->off_lowq_off = (int64_t)off;  off = align_up(off + (F + 1) * sizeof(int32_t));
    int64_t n_scan = 0, n_chunk = 0;
    for (const FrameDev& fd : b->frames) {
        n_scan += max_scan_items(fd.L);
        n_chunk += max_chunk_items(fd.L);
    }
    lay->off_scan_items = (int64_t)off;  off = align_up(off + (size_t)n_scan * 8);
    lay->off_chunk_items = (int64_t)off; off = align_up(off + (size_t)n_chunk * 16);
    lay->off_rescue = (int64_t)off;      off = align_up(off + F * sizeof(int32_t));
    return off;
}

// workgroups of a grid-stride launch: `per_cu` resident workgroups on every compute unit
int persistent_grid(int per_cu) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus * per_cu;
}

nssdoa_status check_windowed(nssdoa_batch batch, const WindowArgs& wa, int* n_feat, int* n_bins) {
    if (batch->prec != NSSDOA_C64)
        return fail(NSSDOA_EUNSUPPORTED, "windowed estimation runs the C64 scans: create the batch with NSSDOA_C64");
    if (batch->any2d) return fail(NSSDOA_EUNSUPPORTED, "windowed estimation scans 1-D grids only");
    const int M = batch->frames[0].M;
    for (const FrameDev& fd : batch->frames)
        if (fd.M != M) return fail(NSSDOA_EUNSUPPORTED, "windowed estimation needs one array size in the batch");
    if (wa.topk < 1 || wa.topk > kMaxWindows) return fail(NSSDOA_EINVAL, "topk=%d outside [1, %d]", wa.topk, kMaxWindows);
    if (!(wa.half_window > 0.0) || !(wa.half_window <= 180.0))
        return fail(NSSDOA_EINVAL, "half_window_deg must be in (0, 180]");
    if (wa.threshold != wa.threshold) return fail(NSSDOA_EINVAL, "threshold is NaN");
    *n_feat = 0;
    *n_bins = wa.n_bins;
    if (wa.mlp) {
        int32_t in, width, out, mb;
        mlp_dims(wa.mlp, &in, &width, &out, &mb);
        if (in != M * (M + 1))
            return fail(NSSDOA_EINVAL, "the network takes %d inputs, covariance features of M=%d are %d", in, M, M * (M + 1));
        *n_feat = in;
        *n_bins = out;
    } else if (!wa.scores) {
        return fail(NSSDOA_EINVAL, "scores is NULL");
    }
    if (*n_bins < 1 || *n_bins > kMaxBins) return fail(NSSDOA_EINVAL, "n_bins=%d outside [1, %d]", *n_bins, kMaxBins);
    for (int f = 0; f < batch->n_frames; ++f) {
        const FrameDev& fd = batch->frames[f];
        const int64_t slots = ((int64_t)(fd.L + kRefineChunk - 1) / kRefineChunk + wa.topk) *
                              (fd.D + batch->plan->opt.extra_candidates);
        if (slots > kSelCap)
            return fail(NSSDOA_EINVAL, "frame %d: %d windows on a grid of %d points exceed the peak candidate capacity",
                        f, wa.topk, fd.L);
    }
    return NSSDOA_OK;
}

nssdoa_status estimate_impl(nssdoa_batch batch, const void* X, size_t x_elems, void* spectrum,
                            size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks, uint32_t* status,
                            void* workspace, size_t workspace_bytes, void* stream, const WindowArgs* wa,
                            bool capturing = false) {
    if (!batch) return fail(NSSDOA_EINVAL, "batch is NULL");
    if (!X || !peaks || !npeaks || !status || !workspace)
        return fail(NSSDOA_EINVAL, "NULL X, peaks, npeaks, status or workspace");
    if (x_elems < batch->x_extent)
        return fail(NSSDOA_EINVAL, "X holds %zu complex elements, the frames address %zu", x_elems,
                    batch->x_extent);
    if (spectrum && spectrum_elems < batch->spec_extent)
        return fail(NSSDOA_EINVAL, "spectrum holds %zu elements, the frames address %zu",
                    spectrum_elems, batch->spec_extent);
    LearnedLayout lay;
    memset(&lay, 0, sizeof(lay));
    size_t need = batch->ws_bytes;
    int n_feat = 0, n_bins = 0;
    if (wa) {
        nssdoa_status st = check_windowed(batch, *wa, &n_feat, &n_bins);
        if (st != NSSDOA_OK) return st;
        need = windowed_layout(batch, n_feat, wa->mlp ? n_bins : 0, &lay);
    }
    if (workspace_bytes < need)
        return fail(NSSDOA_EINVAL, "workspace of %zu bytes < required %zu", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(NSSDOA_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    const int use_user = spectrum != nullptr;
    void* spec = use_user ? spectrum : static_cast<void*>(ws);
    const bool c128 = batch->prec == NSSDOA_C128;
    const nssdoa_options& opt = batch->plan->opt;

    hipEvent_t ev0 = nullptr;
    const uint32_t timing = capturing ? 0u : batch->timing;
    auto stage_begin = [&](int stage) -> nssdoa_status {
        if (!(timing & (1u << stage))) return NSSDOA_OK;
        // timing-only events: no system-scope fence (no cache writeback around the timed stage)
        hipError_t e = hipEventCreateWithFlags(&ev0, hipEventDisableSystemFence);
        if (e == hipSuccess) e = hipEventRecord(ev0, s);
        return e == hipSuccess ? NSSDOA_OK : hip_fail(e, "hipEventRecord");
    };
    auto stage_end = [&](int stage) -> nssdoa_status {
        if (!(timing & (1u << stage))) return NSSDOA_OK;
        hipEvent_t ev1;
        hipError_t e = hipEventCreateWithFlags(&ev1, hipEventDisableSystemFence);
        if (e == hipSuccess) e = hipEventRecord(ev1, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        batch->pending.push_back({stage, ev0, ev1});
        return NSSDOA_OK;
    };
    nssdoa_status st;
    hipError_t e;

    if ((st = stage_begin(NSSDOA_STAGE_COVARIANCE)) != NSSDOA_OK) return st;
    LowqList lql = {nullptr, nullptr, 0};
    if (batch->ws_lowq_all >= 0)
        lql = {reinterpret_cast<int*>(ws + batch->ws_lowq_all), reinterpret_cast<int2*>(ws + batch->ws_lowq_all + 256),
               batch->lowq_all_cap};
    e = launch_cov(c128, batch->max_M, batch->d_cov, (int)batch->cov_items.size(), batch->d_frames, X, ws, lql.count,
                   s);
    if (e != hipSuccess) return hip_fail(e, "covariance launch");
    if ((st = stage_end(NSSDOA_STAGE_COVARIANCE)) != NSSDOA_OK) return st;

    if ((st = stage_begin(NSSDOA_STAGE_EIGEN)) != NSSDOA_OK) return st;
    EvdParams ep;
    ep.tol = opt.eig_tol;
    ep.max_iter = opt.eig_max_iter;
    ep.method = opt.eig_method;
    // operand tiles of the scans: FP32, FP16 split, BF16, FP16
    ep.write_emb = c128 ? 0 : batch->prec == NSSDOA_C64 ? (batch->split_parts == 3 ? 5 : batch->split_parts ? 4 : 1)
                                                         : batch->prec == NSSDOA_BF16 ? 2 : 3;
    for (const auto* ranges : {&batch->peak_ranges, &batch->p2d_ranges}) {
        for (auto& r : *ranges) {
            e = launch_evd(batch->d_plist + r.second.first, r.second.second - r.second.first, r.first, ep,
                           batch->d_frames, batch->d_groups, ws, status, s);
            if (e != hipSuccess) return hip_fail(e, "eigen launch");
        }
    }
    if ((st = stage_end(NSSDOA_STAGE_EIGEN)) != NSSDOA_OK) return st;

    PeakParams pp;
    memset(&pp, 0, sizeof(pp));
    pp.lowq_tau = opt.lowq_tau;
    pp.halfwidth = opt.refine_halfwidth;
    pp.extra = opt.extra_candidates;
    pp.max_D = batch->max_D;
    pp.refine_lowq = c128 ? 0 : 1;
    pp.lp_floor = batch->prec == NSSDOA_BF16 || batch->prec == NSSDOA_F16;
    pp.use_user_spec = use_user;
    // plateau depth of the peak candidates: above the relative error of the scanned spectrum
    // (FP32 and 16-bit scans after the FP64 re-evaluation of low-Q points; FP64 scan)
    pp.plateau_rel = c128 ? 1e-10 : kPlateauRelScan;

    if (wa) {
        const int F = batch->n_frames, M = batch->frames[0].M;
        if ((st = stage_begin(NSSDOA_STAGE_PROPOSAL)) != NSSDOA_OK) return st;
        const float* scores = wa->scores;
        if (wa->mlp) {
            float* feats = reinterpret_cast<float*>(ws + lay.off_feat);
            float* logits = reinterpret_cast<float*>(ws + lay.off_scores);
            e = launch_features(nullptr, F, batch->d_frames, ws, feats, n_feat, s);
            if (e == hipSuccess) e = mlp_forward_rows(wa->mlp, feats, F, logits, s);
            if (e != hipSuccess) return hip_fail(e, "proposal network launch");
            scores = logits;
        }
        e = launch_proposals(batch->d_frames, F, scores, n_bins, wa->topk, wa->half_window, wa->threshold, wa->floor, wa->local_max, ws, lay,
                             status, s);
        if (e != hipSuccess) return hip_fail(e, "proposal launch");
        if ((st = stage_end(NSSDOA_STAGE_PROPOSAL)) != NSSDOA_OK) return st;

        if ((st = stage_begin(NSSDOA_STAGE_SCAN)) != NSSDOA_OK) return st;
        e = launch_scan_windows(batch->split_parts, M, batch->d_frames, F, batch->d_groups, batch->d_blk, batch->d_steer, ws, lay,
                                static_cast<float*>(spec), use_user, (float)opt.lowq_tau, persistent_grid(8), s);
        if (e != hipSuccess) return hip_fail(e, "windowed scan launch");
        if ((st = stage_end(NSSDOA_STAGE_SCAN)) != NSSDOA_OK) return st;

        if ((st = stage_begin(NSSDOA_STAGE_PEAKS)) != NSSDOA_OK) return st;
        const int bucket = M <= 8 ? 8 : M <= 16 ? 16 : M <= 32 ? 32 : 64;
        e = launch_window_peaks(bucket, batch->d_frames, F, batch->d_pos, batch->d_cis, ws, lay, opt.extra_candidates,
                                opt.lowq_tau, pp.plateau_rel, static_cast<float*>(spec), use_user,
                                persistent_grid(2), s);
        if (e != hipSuccess) return hip_fail(e, "windowed peak launch");
        pp.chunk_count = reinterpret_cast<const int32_t*>(ws + lay.off_chunks);
        pp.windows = reinterpret_cast<const int32_t*>(ws + lay.off_win);
        for (auto& r : batch->peak_ranges) {
            pp.sel_cap = batch->peak_selcap[&r - &batch->peak_ranges[0]];
            e = launch_peaks(false, r.first, nullptr, 0, batch->d_plist + r.second.first,
                             r.second.second - r.second.first, batch->d_frames, batch->d_pos, batch->d_cis, ws, spec,
                             pp, peaks, npeaks, status, s);
            if (e != hipSuccess) return hip_fail(e, "peak launch");
        }
        // second pass: frames whose windows held fewer than D peaks, over their whole grid (the
        // host enqueues it unconditionally; frames that need nothing get no work items)
        int32_t* rescue = reinterpret_cast<int32_t*>(ws + lay.off_rescue);
        for (auto& r : batch->peak_ranges) {
            e = launch_rescue(batch->d_frames, batch->d_plist + r.second.first, r.second.second - r.second.first,
                              npeaks, status, ws, lay, rescue + r.second.first, s);
            if (e != hipSuccess) return hip_fail(e, "rescue launch");
        }
        e = launch_expand(batch->d_frames, F, ws, lay, s);
        if (e == hipSuccess)
            e = launch_scan_windows(batch->split_parts, M, batch->d_frames, F, batch->d_groups, batch->d_blk,
                                    batch->d_steer, ws, lay, static_cast<float*>(spec), use_user,
                                    (float)opt.lowq_tau, persistent_grid(8), s);
        if (e == hipSuccess)
            e = launch_window_peaks(bucket, batch->d_frames, F, batch->d_pos, batch->d_cis, ws, lay,
                                    opt.extra_candidates, opt.lowq_tau, pp.plateau_rel, static_cast<float*>(spec),
                                    use_user, persistent_grid(2), s);
        if (e != hipSuccess) return hip_fail(e, "rescue scan launch");
        for (auto& r : batch->peak_ranges) {
            pp.sel_cap = batch->peak_selcap[&r - &batch->peak_ranges[0]];
            e = launch_peaks(false, r.first, nullptr, 0, rescue + r.second.first, r.second.second - r.second.first,
                             batch->d_frames, batch->d_pos, batch->d_cis, ws, spec, pp, peaks, npeaks, status, s);
            if (e != hipSuccess) return hip_fail(e, "rescue peak launch");
        }
        return stage_end(NSSDOA_STAGE_PEAKS);
    }

    if ((st = stage_begin(NSSDOA_STAGE_SCAN)) != NSSDOA_OK) return st;
    if (c128) {
        e = launch_scan_f64(batch->d_points, (int)batch->point_items.size(), batch->max_M, batch->d_frames,
                            batch->d_pos, batch->d_cis, ws, static_cast<double*>(spec), use_user, s);
        if (e != hipSuccess) return hip_fail(e, "FP64 scan launch");
    } else {
        for (auto& r : batch->scan_ranges) {
            if (batch->prec == NSSDOA_C64 && batch->split_parts)
                e = launch_scan_split16(batch->split_parts, r.first, batch->d_scan + r.second.first, r.second.second - r.second.first,
                                        batch->scan_max_tiles[&r - &batch->scan_ranges[0]],
                                        batch->d_groups, batch->d_frames, batch->d_blk, batch->d_steer, ws,
                                        static_cast<float*>(spec), use_user, (float)opt.lowq_tau, lql, s);
            else if (batch->prec == NSSDOA_C64)
                e = launch_scan_f32(r.first, batch->d_scan + r.second.first, r.second.second - r.second.first,
                                    batch->scan_max_tiles[&r - &batch->scan_ranges[0]],
                                    batch->d_groups, batch->d_frames, batch->d_blk, batch->d_steer, ws,
                                    static_cast<float*>(spec), use_user, (float)opt.lowq_tau, lql, s);
            else
                e = launch_scan_lp(batch->prec == NSSDOA_F16, r.first, batch->d_scan + r.second.first,
                                   r.second.second - r.second.first, batch->d_groups, batch->d_frames,
                                   batch->d_blk, batch->d_pos, ws, static_cast<float*>(spec), use_user,
                                   (float)opt.lowq_tau, lql, s);
            if (e != hipSuccess) return hip_fail(e, "scan launch");
        }
    }
    if ((st = stage_end(NSSDOA_STAGE_SCAN)) != NSSDOA_OK) return st;

    if ((st = stage_begin(NSSDOA_STAGE_PEAKS)) != NSSDOA_OK) return st;
    if (!c128) {
        const int bucket = batch->max_M <= 8 ? 8 : batch->max_M <= 16 ? 16 : batch->max_M <= 32 ? 32 : 64;
        e = launch_lowq_refine(bucket, lql, batch->d_frames, batch->d_pos, batch->d_cis, ws, static_cast<float*>(spec),
                               use_user, kLowqRefineGrid, s);
        if (e != hipSuccess) return hip_fail(e, "low-Q refine launch");
    }
    for (size_t i = 0; i < batch->peak_ranges.size(); ++i) {
        const auto& r = batch->peak_ranges[i];
        const auto& ri = batch->refine_ranges[i];
        pp.sel_cap = batch->peak_selcap[i];
        e = launch_peaks(c128, r.first, batch->d_refine + ri.first, ri.second - ri.first,
                         batch->d_plist + r.second.first, r.second.second - r.second.first,
                         batch->d_frames, batch->d_pos, batch->d_cis, ws, spec, pp, peaks, npeaks, status, s);
        if (e != hipSuccess) return hip_fail(e, "peak launch");
    }
    for (size_t i = 0; i < batch->p2d_ranges.size(); ++i) {
        const auto& r = batch->p2d_ranges[i];
        const auto& ri = batch->p2d_iranges[i];
        e = launch_peaks2d(c128, r.first, batch->d_refine + ri.first, ri.second - ri.first,
                           batch->d_plist + r.second.first, r.second.second - r.second.first, batch->d_frames,
                           batch->d_pos, batch->d_cis, ws, spec, use_user, batch->max_D, peaks, npeaks, status, s);
        if (e != hipSuccess) return hip_fail(e, "2-D peak launch");
    }
    return stage_end(NSSDOA_STAGE_PEAKS);
}

}  // namespace

extern "C" {

nssdoa_status nssdoa_estimate(nssdoa_batch batch, const void* X, size_t x_elems, void* spectrum,
                              size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks,
                              uint32_t* status, void* workspace, size_t workspace_bytes,
                              void* stream) {
    return estimate_impl(batch, X, x_elems, spectrum, spectrum_elems, peaks, npeaks, status, workspace,
                         workspace_bytes, stream, nullptr);
}

nssdoa_status nssdoa_estimate_noalloc(nssdoa_batch batch, const void* X, size_t x_elems, void* spectrum,
                                      size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks, uint32_t* status,
                                      void* stream) {
    if (!batch) return fail(NSSDOA_EINVAL, "batch is NULL");
    if (batch->ws_bytes > kNoallocScratchBytes)
        return fail(NSSDOA_EINVAL, "the batch needs %zu bytes of workspace, the no-allocation workspace holds %zu",
                    batch->ws_bytes, kNoallocScratchBytes);
    void* ws = nullptr;
    nssdoa_status st = scratch_address(&ws);
    if (st != NSSDOA_OK) return st;
    // no stage timing here: its events are created per call
    return estimate_impl(batch, X, x_elems, spectrum, spectrum_elems, peaks, npeaks, status, ws,
                         kNoallocScratchBytes, stream, nullptr, true);
}

nssdoa_status nssdoa_noalloc_workspace_limit(size_t* bytes) {
    if (!bytes) return fail(NSSDOA_EINVAL, "NULL argument");
    *bytes = kNoallocScratchBytes;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_features(nssdoa_batch batch, const void* workspace, size_t workspace_bytes, float* feats,
                              int32_t n_feat, void* stream) {
    if (!batch || !workspace || !feats) return fail(NSSDOA_EINVAL, "NULL batch, workspace or feats");
    if (workspace_bytes < batch->ws_bytes)
        return fail(NSSDOA_EINVAL, "workspace of %zu bytes < required %zu", workspace_bytes, batch->ws_bytes);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(NSSDOA_EINVAL, "workspace must be 256-byte aligned");
    const int M = batch->frames[0].M;
    for (const FrameDev& fd : batch->frames)
        if (fd.M != M) return fail(NSSDOA_EUNSUPPORTED, "features need one array size in the batch");
    if (n_feat != M * (M + 1)) return fail(NSSDOA_EINVAL, "n_feat=%d, the features of M=%d hold %d", n_feat, M, M * (M + 1));
    hipError_t e = launch_features(nullptr, batch->n_frames, batch->d_frames,
                                   static_cast<const char*>(workspace), feats, n_feat, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NSSDOA_OK : hip_fail(e, "features launch");
}

nssdoa_status nssdoa_scan_form(nssdoa_batch batch, int32_t form, const void* workspace, size_t workspace_bytes,
                               float* spectrum, size_t spectrum_elems, void* stream) {
    if (!batch || !workspace || !spectrum) return fail(NSSDOA_EINVAL, "NULL batch, workspace or spectrum");
    if (form != NSSDOA_FORM_FACTORED && form != NSSDOA_FORM_QUADRATIC && form != NSSDOA_FORM_COMPLEMENT)
        return fail(NSSDOA_EINVAL, "unknown scan form %d", form);
    if (batch->prec != NSSDOA_C64) return fail(NSSDOA_EUNSUPPORTED, "scan forms run on NSSDOA_C64 batches");
    if (batch->any2d || batch->max_M > 32)
        return fail(NSSDOA_EUNSUPPORTED, "scan forms run on 1-D grids with M <= 32");
    if (form == NSSDOA_FORM_COMPLEMENT && batch->alg != NSSDOA_MUSIC)
        return fail(NSSDOA_EUNSUPPORTED, "the complement form is the MUSIC matrix I - E_s E_s^H");
    if (workspace_bytes < batch->ws_bytes)
        return fail(NSSDOA_EINVAL, "workspace of %zu bytes < required %zu", workspace_bytes, batch->ws_bytes);
    if (spectrum_elems < batch->spec_extent)
        return fail(NSSDOA_EINVAL, "spectrum holds %zu elements, the frames address %zu", spectrum_elems,
                    batch->spec_extent);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (size_t i = 0; i < batch->peak_ranges.size(); ++i) {
        const auto& ri = batch->refine_ranges[i];
        hipError_t e = launch_scan_form(batch->peak_ranges[i].first, batch->d_refine + ri.first, ri.second - ri.first,
                                        batch->d_frames, batch->d_pos, static_cast<const char*>(workspace), form,
                                        spectrum, s);
        if (e != hipSuccess) return hip_fail(e, "scan form launch");
    }
    return NSSDOA_OK;
}

nssdoa_status nssdoa_windowed_workspace_size(nssdoa_batch batch, nssdoa_mlp mlp, size_t* bytes) {
    if (!batch || !bytes) return fail(NSSDOA_EINVAL, "NULL argument");
    int32_t in = 0, width = 0, out = 0, mb = 0;
    if (mlp) mlp_dims(mlp, &in, &width, &out, &mb);
    LearnedLayout lay;
    *bytes = windowed_layout(batch, in, out, &lay);
    return NSSDOA_OK;
}

nssdoa_status nssdoa_estimate_windowed(nssdoa_batch batch, const void* X, size_t x_elems, const float* scores,
                                       int32_t n_bins, int32_t topk, double half_window_deg, float score_threshold,
                                       float window_floor, int32_t local_max_bins, void* spectrum,
                                       size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks, uint32_t* status,
                                       void* workspace, size_t workspace_bytes, void* stream) {
    if (window_floor != window_floor) return fail(NSSDOA_EINVAL, "window_floor is NaN");
    WindowArgs wa{nullptr, scores, n_bins, topk, half_window_deg, score_threshold, window_floor, local_max_bins != 0};
    return estimate_impl(batch, X, x_elems, spectrum, spectrum_elems, peaks, npeaks, status, workspace,
                         workspace_bytes, stream, &wa);
}

nssdoa_status nssdoa_estimate_learned(nssdoa_batch batch, nssdoa_mlp mlp, const void* X, size_t x_elems,
                                      int32_t topk, double half_window_deg, double fallback_score,
                                      double window_score, int32_t local_max_bins, void* spectrum,
                                      size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks, uint32_t* status,
                                      void* workspace, size_t workspace_bytes, void* stream) {
    if (!mlp) return fail(NSSDOA_EINVAL, "mlp is NULL");
    if (!(fallback_score >= 0.0 && fallback_score <= 1.0))
        return fail(NSSDOA_EINVAL, "fallback_score must be in [0, 1]");
    if (!(window_score >= 0.0 && window_score <= 1.0))
        return fail(NSSDOA_EINVAL, "window_score must be in [0, 1]");
    // sigmoid(z) < p  <=>  z < log(p / (1 - p))
    auto logit = [](double p) { return p == 0.0 ? -INFINITY : p == 1.0 ? INFINITY : log(p) - log1p(-p); };
    WindowArgs wa{mlp, nullptr, 0, topk, half_window_deg, (float)logit(fallback_score), (float)logit(window_score),
                  local_max_bins != 0};
    return estimate_impl(batch, X, x_elems, spectrum, spectrum_elems, peaks, npeaks, status, workspace,
                         workspace_bytes, stream, &wa);
}

struct nssdoa_graph_s {
    nssdoa_batch batch = nullptr;
    hipGraphExec_t exec = nullptr;
};

nssdoa_status nssdoa_graph_create(nssdoa_graph* out, nssdoa_batch batch, const void* X, size_t x_elems,
                                  void* spectrum, size_t spectrum_elems, nssdoa_peak* peaks, int32_t* npeaks,
                                  uint32_t* status, void* workspace, size_t workspace_bytes) {
    if (!out) return fail(NSSDOA_EINVAL, "graph is NULL");
    *out = nullptr;
    if (!batch) return fail(NSSDOA_EINVAL, "batch is NULL");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate(capture)");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    nssdoa_status st = estimate_impl(batch, X, x_elems, spectrum, spectrum_elems, peaks, npeaks, status, workspace,
                                     workspace_bytes, cs, nullptr, true);
    const std::string msg = g_last_error;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st != NSSDOA_OK) {
        if (g) (void)hipGraphDestroy(g);
        g_last_error = msg;
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    auto* gr = new (std::nothrow) nssdoa_graph_s();
    if (!gr) {
        (void)hipGraphExecDestroy(exec);
        return fail(NSSDOA_ENOMEM, "host allocation failed");
    }
    gr->batch = batch;
    gr->exec = exec;
    batch->live_graphs++;
    *out = gr;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_graph_launch(nssdoa_graph graph, void* stream) {
    if (!graph) return fail(NSSDOA_EINVAL, "graph is NULL");
    hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NSSDOA_OK : hip_fail(e, "hipGraphLaunch");
}

nssdoa_status nssdoa_graph_destroy(nssdoa_graph graph) {
    if (!graph) return NSSDOA_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->batch) graph->batch->live_graphs--;
    delete graph;
    return NSSDOA_OK;
}

// ---------------------------------------------------------------------------------------------
// Streaming pipeline: batches of snapshots arriving in host memory, each copied in, estimated and
// its results copied out on one of `depth` slots; every slot has its own stream, device buffers
// and completion event, so the copy-in of one batch overlaps the estimate of the previous one and
// the copy-out of the one before.
struct PipeSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* dev = nullptr;                 // X, workspace, spectrum, peaks, npeaks, status
    void* X = nullptr;
    void* ws = nullptr;
    void* spec = nullptr;
    nssdoa_peak* peaks = nullptr;
    int32_t* npeaks = nullptr;
    uint32_t* status = nullptr;
    int64_t ticket = -1;                 // last submission on this slot, -1 if none
};

struct nssdoa_pipeline_s {
    nssdoa_batch batch = nullptr;
    std::vector<PipeSlot> slots;
    int64_t next = 0;
    size_t x_bytes = 0, ws_bytes = 0, spec_bytes = 0, peak_bytes = 0;
};

static void pipeline_free(nssdoa_pipeline pl) {
    for (PipeSlot& sl : pl->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.dev) (void)hipFree(sl.dev);
    }
    if (pl->batch) pl->batch->live_graphs--;
    delete pl;
}

nssdoa_status nssdoa_pipeline_create(nssdoa_pipeline* out, nssdoa_batch batch, int32_t depth) {
    if (!out) return fail(NSSDOA_EINVAL, "pipeline is NULL");
    *out = nullptr;
    if (!batch) return fail(NSSDOA_EINVAL, "batch is NULL");
    if (depth < 1 || depth > 8) return fail(NSSDOA_EINVAL, "depth=%d outside [1, 8]", depth);
    auto* pl = new (std::nothrow) nssdoa_pipeline_s();
    if (!pl) return fail(NSSDOA_ENOMEM, "host allocation failed");
    pl->batch = batch;
    batch->live_graphs++;                // the batch must outlive the pipeline
    const size_t celem = batch->prec == NSSDOA_C128 ? 16 : 8;
    pl->x_bytes = align_up(batch->x_extent * celem);
    pl->ws_bytes = align_up(batch->ws_bytes);
    pl->spec_bytes = align_up(batch->spec_extent * batch->spec_elem);
    pl->peak_bytes = align_up((size_t)batch->n_frames * batch->max_D * sizeof(nssdoa_peak));
    const size_t small = align_up((size_t)batch->n_frames * 4);
    const size_t total = pl->x_bytes + pl->ws_bytes + pl->spec_bytes + pl->peak_bytes + 2 * small;
    pl->slots.resize(depth);
    for (PipeSlot& sl : pl->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc((void**)&sl.dev, total);
        if (e != hipSuccess) {
            pipeline_free(pl);
            return hip_fail(e, "pipeline slot");
        }
        char* p = sl.dev;
        sl.X = p;                                       p += pl->x_bytes;
        sl.ws = p;                                      p += pl->ws_bytes;
        sl.spec = p;                                    p += pl->spec_bytes;
        sl.peaks = reinterpret_cast<nssdoa_peak*>(p);   p += pl->peak_bytes;
        sl.npeaks = reinterpret_cast<int32_t*>(p);      p += small;
        sl.status = reinterpret_cast<uint32_t*>(p);
    }
    *out = pl;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_pipeline_submit(nssdoa_pipeline pl, const void* X_host, void* spectrum_host, nssdoa_peak* peaks_host,
                                     int32_t* npeaks_host, uint32_t* status_host, int64_t* ticket) {
    if (!pl || !X_host || !peaks_host || !npeaks_host || !status_host || !ticket)
        return fail(NSSDOA_EINVAL, "NULL pipeline, X, peaks, npeaks, status or ticket");
    PipeSlot& sl = pl->slots[pl->next % (int64_t)pl->slots.size()];
    hipError_t e = hipSuccess;
    if (sl.ticket >= 0) {
        e = hipEventSynchronize(sl.done);             // the slot's previous batch has finished
        if (e != hipSuccess) return hip_fail(e, "pipeline wait");
    }
    nssdoa_batch b = pl->batch;
    const size_t celem = b->prec == NSSDOA_C128 ? 16 : 8;
    e = hipMemcpyAsync(sl.X, X_host, b->x_extent * celem, hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return hip_fail(e, "pipeline copy-in");
    nssdoa_status st = estimate_impl(b, sl.X, b->x_extent, spectrum_host ? sl.spec : nullptr,
                                     pl->spec_bytes / b->spec_elem, sl.peaks, sl.npeaks, sl.status, sl.ws, pl->ws_bytes,
                                     sl.stream, nullptr, true);
    if (st != NSSDOA_OK) return st;
    const size_t n = (size_t)b->n_frames;
    e = hipMemcpyAsync(peaks_host, sl.peaks, n * b->max_D * sizeof(nssdoa_peak), hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(npeaks_host, sl.npeaks, n * 4, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(status_host, sl.status, n * 4, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess && spectrum_host)
        e = hipMemcpyAsync(spectrum_host, sl.spec, b->spec_extent * b->spec_elem, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return hip_fail(e, "pipeline copy-out");
    sl.ticket = pl->next++;
    *ticket = sl.ticket;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_pipeline_wait(nssdoa_pipeline pl, int64_t ticket) {
    if (!pl) return fail(NSSDOA_EINVAL, "pipeline is NULL");
    if (ticket < 0 || ticket >= pl->next) return fail(NSSDOA_EINVAL, "ticket %lld was never issued", (long long)ticket);
    const PipeSlot& sl = pl->slots[ticket % (int64_t)pl->slots.size()];
    if (sl.ticket != ticket) return NSSDOA_OK;         // its slot was reused, which waited for it
    hipError_t e = hipEventSynchronize(sl.done);
    return e == hipSuccess ? NSSDOA_OK : hip_fail(e, "pipeline wait");
}

nssdoa_status nssdoa_pipeline_destroy(nssdoa_pipeline pl) {
    if (!pl) return NSSDOA_OK;
    pipeline_free(pl);
    return NSSDOA_OK;
}

}  // extern "C"
