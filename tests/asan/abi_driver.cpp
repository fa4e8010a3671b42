// Host AddressSanitizer driver for the C ABI (include/nssdoa.h).  Built against a copy of
// libnssdoa.so whose host code is instrumented (device code unchanged), it walks the calls a
// user makes, their argument checks and their error paths, and frees everything, so ASan sees
// every host allocation, copy and free of the library and LeakSanitizer sees what is left.
//
//   abi_driver cpu   no device needed: plan creation and its argument checks, status strings,
//                    and batch / network creation failing cleanly without a device
//   abi_driver gpu   the same argument checks, then every estimator on one small batch per
//                    precision (and a 2-D batch for C64 and C128): estimate,
//                    estimate_noalloc, graph capture and replay, stage timing, the streaming
//                    pipeline, workspace queries, scan forms, features, windowed and learned
//                    estimation, and the network's forward, training, gradients and checkpoint
//
// Exit status 0 when every call returned what it should; ASan aborts the process on an error.
// Numerical results are not checked here (the parity tests do that); only their shape.
#include <hip/hip_runtime_api.h>
#include <sanitizer/lsan_interface.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "nssdoa.h"

namespace {

int g_fail = 0;

void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s (last error: %s)\n", what, nssdoa_last_error());
        ++g_fail;
    }
}

#define EXPECT_STATUS(call, want) expect((call) == (want), #call " == " #want)

constexpr int kM = 16;

std::vector<double> ula(int M) {          // half-wavelength ULA along x
    std::vector<double> p(3 * M, 0.0);
    for (int m = 0; m < M; ++m) p[3 * m] = 0.5 * m;
    return p;
}

// Plan creation: one valid plan (returned) after a series of rejected arguments.
nssdoa_plan make_plan(const std::vector<double>& pos, bool with_2d) {
    nssdoa_array arr = {kM, 0, pos.data()};
    nssdoa_grid grids[2];
    std::memset(grids, 0, sizeof(grids));
    grids[0].start_deg = -90.0;
    grids[0].step_deg = 0.1;
    grids[0].L = 1800;
    grids[1] = grids[0];
    grids[1].start_deg = 0.0;
    grids[1].step_deg = 2.0;
    grids[1].L = 180;
    grids[1].circular = 1;
    grids[1].polar_start_deg = 30.0;
    grids[1].polar_step_deg = 10.0;
    grids[1].n_polar = 4;
    nssdoa_plan plan = nullptr;

    EXPECT_STATUS(nssdoa_plan_create(nullptr, &arr, 1, grids, 1, nullptr), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_plan_create(&plan, nullptr, 1, grids, 1, nullptr), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_plan_create(&plan, &arr, 0, grids, 1, nullptr), NSSDOA_EINVAL);
    nssdoa_array bad = arr;
    bad.M = 65;
    EXPECT_STATUS(nssdoa_plan_create(&plan, &bad, 1, grids, 1, nullptr), NSSDOA_EINVAL);
    std::vector<double> nanpos = pos;
    nanpos[4] = NAN;
    bad = arr;
    bad.pos_wl = nanpos.data();
    EXPECT_STATUS(nssdoa_plan_create(&plan, &bad, 1, grids, 1, nullptr), NSSDOA_EINVAL);
    nssdoa_grid bg = grids[0];
    bg.step_deg = 0.0;
    EXPECT_STATUS(nssdoa_plan_create(&plan, &arr, 1, &bg, 1, nullptr), NSSDOA_EINVAL);
    bg = grids[0];
    bg.L = 2;
    EXPECT_STATUS(nssdoa_plan_create(&plan, &arr, 1, &bg, 1, nullptr), NSSDOA_EINVAL);
    nssdoa_options opt;
    std::memset(&opt, 0, sizeof(opt));
    opt.eig_tol = 1e-15;
    opt.eig_max_iter = 30;
    opt.refine_halfwidth = 17;                // out of range
    opt.lowq_tau = 5e-4;
    opt.extra_candidates = 4;
    EXPECT_STATUS(nssdoa_plan_create(&plan, &arr, 1, grids, 1, &opt), NSSDOA_EINVAL);
    opt.refine_halfwidth = 4;
    opt.c64_scan = 7;
    EXPECT_STATUS(nssdoa_plan_create(&plan, &arr, 1, grids, 1, &opt), NSSDOA_EINVAL);
    opt.c64_scan = 0;
    EXPECT_STATUS(nssdoa_plan_create(&plan, &arr, 1, grids, with_2d ? 2 : 1, &opt), NSSDOA_OK);
    expect(plan != nullptr, "plan created");
    return plan;
}

std::vector<nssdoa_frame> make_frames(int F, int N, int grid_id, int64_t L) {
    std::vector<nssdoa_frame> fr(F);
    for (int f = 0; f < F; ++f) {
        fr[f].array_id = 0;
        fr[f].grid_id = grid_id;
        fr[f].N = N;
        fr[f].D = 2;
        fr[f].x_off = (int64_t)f * kM * N;
        fr[f].ldx = N;
        fr[f].spec_off = (int64_t)f * L;
    }
    return fr;
}

void status_strings() {
    for (int s = 0; s <= 6; ++s) expect(nssdoa_status_string((nssdoa_status)s) != nullptr, "status string");
    expect(nssdoa_last_error() != nullptr, "last error string");
    size_t lim = 0;
    EXPECT_STATUS(nssdoa_noalloc_workspace_limit(&lim), NSSDOA_OK);
    expect(lim > 0, "noalloc limit");
    EXPECT_STATUS(nssdoa_noalloc_workspace_limit(nullptr), NSSDOA_EINVAL);
}

// Batch argument checks that fail on the host before any device work.
void batch_argument_errors(nssdoa_plan plan) {
    std::vector<nssdoa_frame> fr = make_frames(4, 64, 0, 1800);
    nssdoa_batch b = nullptr;
    EXPECT_STATUS(nssdoa_batch_create(nullptr, plan, NSSDOA_MUSIC, NSSDOA_C64, fr.data(), 4, 4), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_batch_create(&b, nullptr, NSSDOA_MUSIC, NSSDOA_C64, fr.data(), 4, 4), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_batch_create(&b, plan, NSSDOA_MUSIC, NSSDOA_C64, fr.data(), 0, 4), NSSDOA_EINVAL);
    std::vector<nssdoa_frame> bad = fr;
    bad[2].D = kM;
    EXPECT_STATUS(nssdoa_batch_create(&b, plan, NSSDOA_MUSIC, NSSDOA_C64, bad.data(), 4, 4), NSSDOA_EINVAL);
    bad = fr;
    bad[1].ldx = 3;
    EXPECT_STATUS(nssdoa_batch_create(&b, plan, NSSDOA_MUSIC, NSSDOA_C64, bad.data(), 4, 4), NSSDOA_EINVAL);
    bad = fr;
    bad[3].grid_id = 9;
    EXPECT_STATUS(nssdoa_batch_create(&b, plan, NSSDOA_MUSIC, NSSDOA_C64, bad.data(), 4, 4), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_batch_create(&b, plan, NSSDOA_MUSIC, NSSDOA_C64, fr.data(), 4, 65), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_batch_destroy(nullptr), NSSDOA_OK);
    EXPECT_STATUS(nssdoa_plan_destroy(nullptr), NSSDOA_OK);
    nssdoa_mlp m = nullptr;
    EXPECT_STATUS(nssdoa_mlp_create(&m, 0, 8, 8, 8), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_mlp_create(nullptr, 8, 8, 8, 8), NSSDOA_EINVAL);
}

// Host-only checks; without a device (no_device) valid batches and networks must also fail
// cleanly.
int run_host(bool no_device) {
    std::vector<double> pos = ula(kM);
    status_strings();
    nssdoa_plan plan = make_plan(pos, false);
    batch_argument_errors(plan);
    if (!no_device) {
        EXPECT_STATUS(nssdoa_plan_destroy(plan), NSSDOA_OK);
        return g_fail;
    }
    std::vector<nssdoa_frame> fr = make_frames(4, 64, 0, 1800);
    nssdoa_batch b = nullptr;
    const nssdoa_status sb = nssdoa_batch_create(&b, plan, NSSDOA_MUSIC, NSSDOA_C64, fr.data(), 4, 4);
    expect(sb == NSSDOA_EDEVICE || sb == NSSDOA_ENOMEM, "batch creation without a device fails");
    expect(b == nullptr, "no batch handle on failure");
    nssdoa_mlp m = nullptr;
    const nssdoa_status sm = nssdoa_mlp_create(&m, 8, 8, 8, 8);
    expect(sm == NSSDOA_EDEVICE || sm == NSSDOA_ENOMEM, "network creation without a device fails");
    EXPECT_STATUS(nssdoa_plan_destroy(plan), NSSDOA_OK);
    return g_fail;
}

#define HIP_OK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            std::fprintf(stderr, "HIP error %s at %s\n", hipGetErrorString(e_), #call); \
            std::exit(3);                                                         \
        }                                                                         \
    } while (0)

template <typename T>
T* dev_alloc(size_t n) {
    void* p = nullptr;
    HIP_OK(hipMalloc(&p, n * sizeof(T) + 256));
    return static_cast<T*>(p);
}

// Every estimator on one batch of F frames (1-D grid; for C64/C128 also one 2-D batch).
void gpu_batch(nssdoa_plan plan, nssdoa_prec prec, int grid_id, int64_t L, hipStream_t st) {
    const int F = 8, N = 128;
    const bool c128 = prec == NSSDOA_C128;
    const size_t xel = (size_t)F * kM * N;
    std::mt19937_64 rng(1234 + (int)prec + 10 * grid_id);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double> xh(2 * xel);
    for (auto& v : xh) v = nd(rng);
    std::vector<float> xf(xh.begin(), xh.end());
    void* X = c128 ? (void*)dev_alloc<double>(2 * xel) : (void*)dev_alloc<float>(2 * xel);
    HIP_OK(hipMemcpy(X, c128 ? (const void*)xh.data() : (const void*)xf.data(),
                     2 * xel * (c128 ? sizeof(double) : sizeof(float)), hipMemcpyHostToDevice));

    std::vector<nssdoa_frame> fr = make_frames(F, N, grid_id, L);
    nssdoa_batch b = nullptr;
    EXPECT_STATUS(nssdoa_batch_create(&b, plan, NSSDOA_MUSIC, prec, fr.data(), F, 4), NSSDOA_OK);
    if (!b) return;
    size_t ws_bytes = 0;
    EXPECT_STATUS(nssdoa_workspace_size(b, &ws_bytes), NSSDOA_OK);
    size_t off = 0;
    EXPECT_STATUS(nssdoa_workspace_offset(b, NSSDOA_WS_B, F - 1, &off), NSSDOA_OK);
    EXPECT_STATUS(nssdoa_workspace_offset(b, NSSDOA_WS_B, F, &off), NSSDOA_EINVAL);
    char* ws = dev_alloc<char>(ws_bytes);
    const size_t spel = (size_t)F * L;
    void* spec = c128 ? (void*)dev_alloc<double>(spel) : (void*)dev_alloc<float>(spel);
    nssdoa_peak* peaks = dev_alloc<nssdoa_peak>((size_t)F * 4);
    int32_t* npk = dev_alloc<int32_t>(F);
    uint32_t* sts = dev_alloc<uint32_t>(F);

    // argument checks of the estimate, then the estimate itself
    EXPECT_STATUS(nssdoa_estimate(b, nullptr, xel, spec, spel, peaks, npk, sts, ws, ws_bytes, st), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_estimate(b, X, xel - 1, spec, spel, peaks, npk, sts, ws, ws_bytes, st), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_estimate(b, X, xel, spec, spel, peaks, npk, sts, ws, ws_bytes - 1, st), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_estimate(b, X, xel, spec, spel - 1, peaks, npk, sts, ws, ws_bytes, st), NSSDOA_EINVAL);
    EXPECT_STATUS(nssdoa_set_timing(b, -1), NSSDOA_OK);
    EXPECT_STATUS(nssdoa_estimate(b, X, xel, spec, spel, peaks, npk, sts, ws, ws_bytes, st), NSSDOA_OK);
    double ms = 0.0;
    int64_t launches = 0;
    EXPECT_STATUS(nssdoa_stage_time(b, NSSDOA_STAGE_SCAN, &ms, &launches), NSSDOA_OK);
    expect(launches == 1, "one timed scan launch");
    EXPECT_STATUS(nssdoa_set_timing(b, 0), NSSDOA_OK);
    EXPECT_STATUS(nssdoa_estimate(b, X, xel, nullptr, 0, peaks, npk, sts, ws, ws_bytes, st), NSSDOA_OK);
    HIP_OK(hipStreamSynchronize(st));
    std::vector<int32_t> nh(F);
    HIP_OK(hipMemcpy(nh.data(), npk, F * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int f = 0; f < F; ++f) expect(nh[f] >= 0 && nh[f] <= 2, "peak count within D");

    // the no-allocation entry point, graph capture and replay
    const nssdoa_status sn = nssdoa_estimate_noalloc(b, X, xel, spec, spel, peaks, npk, sts, st);
    expect(sn == NSSDOA_OK || sn == NSSDOA_EINVAL, "estimate_noalloc");
    nssdoa_graph g = nullptr;
    EXPECT_STATUS(nssdoa_graph_create(&g, b, X, xel, spec, spel, peaks, npk, sts, ws, ws_bytes), NSSDOA_OK);
    if (g) {
        EXPECT_STATUS(nssdoa_batch_destroy(b), NSSDOA_ESTATE);   // a graph of it exists
        EXPECT_STATUS(nssdoa_graph_launch(g, st), NSSDOA_OK);
        EXPECT_STATUS(nssdoa_graph_launch(g, st), NSSDOA_OK);
        HIP_OK(hipStreamSynchronize(st));
        EXPECT_STATUS(nssdoa_graph_destroy(g), NSSDOA_OK);
    }

    // streaming pipeline from pinned host buffers
    if (grid_id == 0) {
        void* xp = nullptr;
        void* sp = nullptr;
        void* pp = nullptr;
        void* np = nullptr;
        void* tp = nullptr;
        const size_t xb = 2 * xel * (c128 ? sizeof(double) : sizeof(float));
        HIP_OK(hipHostMalloc(&xp, xb, 0));
        HIP_OK(hipHostMalloc(&sp, spel * (c128 ? sizeof(double) : sizeof(float)), 0));
        HIP_OK(hipHostMalloc(&pp, F * 4 * sizeof(nssdoa_peak), 0));
        HIP_OK(hipHostMalloc(&np, F * sizeof(int32_t), 0));
        HIP_OK(hipHostMalloc(&tp, F * sizeof(uint32_t), 0));
        std::memcpy(xp, c128 ? (const void*)xh.data() : (const void*)xf.data(), xb);
        nssdoa_pipeline pl = nullptr;
        EXPECT_STATUS(nssdoa_pipeline_create(&pl, b, 9), NSSDOA_EINVAL);
        EXPECT_STATUS(nssdoa_pipeline_create(&pl, b, 2), NSSDOA_OK);
        if (pl) {
            int64_t t0 = -1, t1 = -1;
            EXPECT_STATUS(nssdoa_pipeline_submit(pl, xp, sp, (nssdoa_peak*)pp, (int32_t*)np, (uint32_t*)tp, &t0),
                          NSSDOA_OK);
            EXPECT_STATUS(nssdoa_pipeline_wait(pl, t0), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_pipeline_submit(pl, xp, nullptr, (nssdoa_peak*)pp, (int32_t*)np, (uint32_t*)tp, &t1),
                          NSSDOA_OK);
            EXPECT_STATUS(nssdoa_pipeline_wait(pl, t1 + 5), NSSDOA_EINVAL);
            EXPECT_STATUS(nssdoa_pipeline_wait(pl, t1), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_pipeline_destroy(pl), NSSDOA_OK);
        }
        HIP_OK(hipHostFree(xp));
        HIP_OK(hipHostFree(sp));
        HIP_OK(hipHostFree(pp));
        HIP_OK(hipHostFree(np));
        HIP_OK(hipHostFree(tp));
    }

    if (prec == NSSDOA_C64 && grid_id == 0) {
        // scan forms and features on the estimate's workspace
        EXPECT_STATUS(nssdoa_estimate(b, X, xel, spec, spel, peaks, npk, sts, ws, ws_bytes, st), NSSDOA_OK);
        for (int form = 0; form < 3; ++form)
            EXPECT_STATUS(nssdoa_scan_form(b, form, ws, ws_bytes, (float*)spec, spel, st), NSSDOA_OK);
        EXPECT_STATUS(nssdoa_scan_form(b, 5, ws, ws_bytes, (float*)spec, spel, st), NSSDOA_EINVAL);
        const int nfeat = kM * (kM + 1);
        float* feats = dev_alloc<float>((size_t)F * nfeat);
        EXPECT_STATUS(nssdoa_features(b, ws, ws_bytes, feats, nfeat, st), NSSDOA_OK);
        EXPECT_STATUS(nssdoa_features(b, ws, ws_bytes, feats, nfeat + 1, st), NSSDOA_EINVAL);

        // windowed estimation on caller scores, then the learned path with a small network
        const int nbins = 180;
        std::vector<float> sc((size_t)F * nbins);
        for (auto& v : sc) v = (float)nd(rng);
        float* scores = dev_alloc<float>(sc.size());
        HIP_OK(hipMemcpy(scores, sc.data(), sc.size() * sizeof(float), hipMemcpyHostToDevice));
        nssdoa_mlp m = nullptr;
        EXPECT_STATUS(nssdoa_mlp_create(&m, nfeat, 64, nbins, F), NSSDOA_OK);
        size_t wws = 0;
        EXPECT_STATUS(nssdoa_windowed_workspace_size(b, m, &wws), NSSDOA_OK);
        char* wsw = dev_alloc<char>(wws);
        EXPECT_STATUS(nssdoa_estimate_windowed(b, X, xel, scores, nbins, 17, 1.0, 0.5f, -INFINITY, 0, spec, spel,
                                               peaks, npk, sts, wsw, wws, st),
                      NSSDOA_EINVAL);
        EXPECT_STATUS(nssdoa_estimate_windowed(b, X, xel, scores, nbins, 4, 1.0, 0.5f, -INFINITY, 1, spec, spel,
                                               peaks, npk, sts, wsw, wws, st),
                      NSSDOA_OK);
        if (m) {
            size_t np = 0, blob_bytes = 0;
            EXPECT_STATUS(nssdoa_mlp_param_count(m, &np), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_mlp_save(m, nullptr, &blob_bytes), NSSDOA_OK);
            std::vector<char> blob(blob_bytes);
            EXPECT_STATUS(nssdoa_mlp_save(m, blob.data(), &blob_bytes), NSSDOA_OK);
            // small random weights through the checkpoint format, then a forward pass
            float* pw = reinterpret_cast<float*>(blob.data() + 32);
            for (size_t i = 0; i < np; ++i) pw[i] = 0.05f * (float)nd(rng);
            EXPECT_STATUS(nssdoa_mlp_load(m, blob.data(), blob_bytes), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_mlp_load(m, blob.data(), blob_bytes - 4), NSSDOA_EINVAL);
            float* logits = dev_alloc<float>((size_t)F * nbins);
            EXPECT_STATUS(nssdoa_mlp_forward(m, feats, F, logits, st), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_estimate_learned(b, m, X, xel, 4, 1.0, 0.5, 0.05, 1, spec, spel, peaks, npk, sts,
                                                  wsw, wws, st),
                          NSSDOA_OK);
            // two training steps on 0/1 targets, gradients to the host
            std::vector<float> tg((size_t)F * nbins, 0.0f);
            for (int f = 0; f < F; ++f) tg[(size_t)f * nbins + (f * 37) % nbins] = 1.0f;
            float* targets = dev_alloc<float>(tg.size());
            HIP_OK(hipMemcpy(targets, tg.data(), tg.size() * sizeof(float), hipMemcpyHostToDevice));
            float* loss = dev_alloc<float>(1);
            EXPECT_STATUS(nssdoa_mlp_train_step(m, feats, targets, F, 1e-3f, loss, st), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_mlp_train_step(m, feats, targets, F, 1e-3f, loss, st), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_mlp_train_step(m, feats, targets, F + 1, 1e-3f, loss, st), NSSDOA_EINVAL);
            HIP_OK(hipStreamSynchronize(st));
            std::vector<float> grads(np);
            EXPECT_STATUS(nssdoa_mlp_gradients(m, grads.data(), np), NSSDOA_OK);
            EXPECT_STATUS(nssdoa_mlp_destroy(m), NSSDOA_OK);
            HIP_OK(hipFree(logits));
            HIP_OK(hipFree(targets));
            HIP_OK(hipFree(loss));
        }
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(hipFree(scores));
        HIP_OK(hipFree(feats));
        HIP_OK(hipFree(wsw));
    }

    HIP_OK(hipStreamSynchronize(st));
    EXPECT_STATUS(nssdoa_batch_destroy(b), NSSDOA_OK);
    HIP_OK(hipFree(X));
    HIP_OK(hipFree(ws));
    HIP_OK(hipFree(spec));
    HIP_OK(hipFree(peaks));
    HIP_OK(hipFree(npk));
    HIP_OK(hipFree(sts));
}

int run_gpu() {
    run_host(false);
    std::vector<double> pos = ula(kM);
    nssdoa_plan plan = make_plan(pos, true);
    hipStream_t st;
    HIP_OK(hipStreamCreate(&st));
    for (nssdoa_prec p : {NSSDOA_C64, NSSDOA_C128, NSSDOA_BF16, NSSDOA_F16}) {
        std::printf("gpu batch prec %d, 1-D grid\n", (int)p);
        std::fflush(stdout);
        gpu_batch(plan, p, 0, 1800, st);
    }
    for (nssdoa_prec p : {NSSDOA_C64, NSSDOA_C128}) {
        std::printf("gpu batch prec %d, 2-D grid\n", (int)p);
        std::fflush(stdout);
        gpu_batch(plan, p, 1, 180 * 4, st);
    }
    HIP_OK(hipStreamDestroy(st));
    EXPECT_STATUS(nssdoa_plan_destroy(plan), NSSDOA_OK);
    return g_fail;
}

}  // namespace

int main(int argc, char** argv) {
    const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
    const int fails = gpu ? run_gpu() : run_host(true);
    std::printf("abi_driver %s: %d failed checks\n", gpu ? "gpu" : "cpu", fails);
    std::fflush(stdout);
    // The leak check runs now, while the HIP runtime is loaded (it exits with ASan's exit code if
    // the library left anything behind); the process then ends without the runtime's teardown,
    // which the ASan runtime's device-memory hooks do not follow.
    __lsan_do_leak_check();
    std::_Exit(fails == 0 ? 0 : 1);
}
