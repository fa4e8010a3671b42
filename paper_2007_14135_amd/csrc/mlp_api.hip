// Host side of the learned proposal network: the nssdoa_mlp object, its checkpoint blob, the
// forward pass and one training step (forward, BCE, backward, Adam) on a stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "nssdoa.h"
#include "internal.h"

using namespace nssdoa;

namespace {
constexpr int32_t kBlobMagic = 0x50434c4d;   // "MLCP"
constexpr int32_t kBlobVersion = 1;
}  // namespace

// defined in api.hip
nssdoa_status nssdoa_internal_fail(nssdoa_status st, const char* msg);

struct nssdoa_mlp_s {
    int32_t in = 0, width = 0, out = 0, max_batch = 0;
    int32_t step = 0;                  // Adam steps taken
    size_t nparam = 0;
    size_t off_w[3], off_b[3];         // offsets (floats) of W_l (out_l x in_l) and b_l
    float* dev = nullptr;              // params | grads | m | v | activations
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *z1 = nullptr, *z2 = nullptr, *z3 = nullptr, *d3 = nullptr, *d2 = nullptr, *d1 = nullptr;
    float* row_loss = nullptr;
};

static nssdoa_status mlp_fail(hipError_t e, const char* what) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    return nssdoa_internal_fail(e == hipErrorOutOfMemory ? NSSDOA_ENOMEM : NSSDOA_EDEVICE, buf);
}

extern "C" {

nssdoa_status nssdoa_mlp_create(nssdoa_mlp* out, int32_t in, int32_t width, int32_t nout, int32_t max_batch) {
    if (!out) return nssdoa_internal_fail(NSSDOA_EINVAL, "mlp is NULL");
    *out = nullptr;
    if (in < 1 || width < 1 || nout < 1 || in > 65536 || width > 65536 || nout > 65536)
        return nssdoa_internal_fail(NSSDOA_EINVAL, "layer sizes must be in [1, 65536]");
    if (max_batch < 1 || max_batch > (1 << 20))
        return nssdoa_internal_fail(NSSDOA_EINVAL, "max_batch must be in [1, 2^20]");
    auto* n = new (std::nothrow) nssdoa_mlp_s();
    if (!n) return nssdoa_internal_fail(NSSDOA_ENOMEM, "host allocation failed");
    n->in = in;
    n->width = width;
    n->out = nout;
    n->max_batch = max_batch;
    const int fin[3] = {in, width, width}, fout[3] = {width, width, nout};
    size_t o = 0;
    for (int l = 0; l < 3; ++l) {
        n->off_w[l] = o;
        o += (size_t)fin[l] * fout[l];
        n->off_b[l] = o;
        o += (size_t)fout[l];
    }
    n->nparam = o;
    const size_t act = (size_t)max_batch * (3 * (size_t)width + 2 * (size_t)nout + 2 * (size_t)width) + max_batch;
    const size_t total = 4 * o + act;
    hipError_t e = hipMalloc((void**)&n->dev, total * sizeof(float));
    if (e != hipSuccess) {
        delete n;
        return mlp_fail(e, "hipMalloc(mlp)");
    }
    e = hipMemset(n->dev, 0, 4 * o * sizeof(float));
    if (e != hipSuccess) {
        (void)hipFree(n->dev);
        delete n;
        return mlp_fail(e, "hipMemset(mlp)");
    }
    n->p = n->dev;
    n->g = n->p + o;
    n->m = n->g + o;
    n->v = n->m + o;
    float* a = n->v + o;
    n->z1 = a; a += (size_t)max_batch * width;
    n->z2 = a; a += (size_t)max_batch * width;
    n->z3 = a; a += (size_t)max_batch * nout;
    n->d3 = a; a += (size_t)max_batch * nout;
    n->d2 = a; a += (size_t)max_batch * width;
    n->d1 = a; a += (size_t)max_batch * width;
    n->row_loss = a;
    *out = n;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_mlp_destroy(nssdoa_mlp n) {
    if (!n) return NSSDOA_OK;
    if (n->dev) (void)hipFree(n->dev);
    delete n;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_mlp_param_count(nssdoa_mlp n, size_t* count) {
    if (!n || !count) return nssdoa_internal_fail(NSSDOA_EINVAL, "NULL argument");
    *count = n->nparam;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_mlp_save(nssdoa_mlp n, void* blob, size_t* bytes) {
    if (!n || !bytes) return nssdoa_internal_fail(NSSDOA_EINVAL, "NULL argument");
    const size_t need = 8 * sizeof(int32_t) + 3 * n->nparam * sizeof(float);
    if (!blob) {
        *bytes = need;
        return NSSDOA_OK;
    }
    if (*bytes < need) return nssdoa_internal_fail(NSSDOA_EINVAL, "checkpoint buffer too small");
    int32_t hdr[8] = {kBlobMagic, kBlobVersion, n->in, n->width, n->out, n->step, 0, 0};
    char* b = static_cast<char*>(blob);
    memcpy(b, hdr, sizeof(hdr));
    float* f = reinterpret_cast<float*>(b + sizeof(hdr));
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(f, n->p, n->nparam * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(f + n->nparam, n->m, n->nparam * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(f + 2 * n->nparam, n->v, n->nparam * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return mlp_fail(e, "checkpoint copy");
    *bytes = need;
    return NSSDOA_OK;
}

nssdoa_status nssdoa_mlp_load(nssdoa_mlp n, const void* blob, size_t bytes) {
    if (!n || !blob) return nssdoa_internal_fail(NSSDOA_EINVAL, "NULL argument");
    const size_t need = 8 * sizeof(int32_t) + 3 * n->nparam * sizeof(float);
    if (bytes != need) return nssdoa_internal_fail(NSSDOA_EINVAL, "checkpoint size does not match the network");
    int32_t hdr[8];
    memcpy(hdr, blob, sizeof(hdr));
    if (hdr[0] != kBlobMagic || hdr[1] != kBlobVersion || hdr[2] != n->in || hdr[3] != n->width || hdr[4] != n->out ||
        hdr[5] < 0)
        return nssdoa_internal_fail(NSSDOA_EINVAL, "checkpoint header does not match the network");
    const float* f = reinterpret_cast<const float*>(static_cast<const char*>(blob) + sizeof(hdr));
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(n->p, f, n->nparam * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->m, f + n->nparam, n->nparam * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->v, f + 2 * n->nparam, n->nparam * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return mlp_fail(e, "checkpoint copy");
    n->step = hdr[5];
    return NSSDOA_OK;
}

nssdoa_status nssdoa_mlp_gradients(nssdoa_mlp n, float* host, size_t count) {
    if (!n || !host) return nssdoa_internal_fail(NSSDOA_EINVAL, "NULL argument");
    if (count != n->nparam) return nssdoa_internal_fail(NSSDOA_EINVAL, "gradient count does not match");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host, n->g, count * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? NSSDOA_OK : mlp_fail(e, "gradient copy");
}

}  // extern "C"

// Z1 = X W1^T + b1;  Z2 = relu(Z1) W2^T + b2;  Z3 = relu(Z2) W3^T + b3 into z3 (row stride out)
static hipError_t mlp_forward(nssdoa_mlp n, const float* X, int B, float* z3, hipStream_t s) {
    hipError_t e;
    e = launch_gemm_bf16(B, n->width, n->in, X, n->in, 1, 0, n->p + n->off_w[0], 1, n->in, 0, 1.0f,
                         n->p + n->off_b[0], nullptr, 0, 0, n->z1, n->width, s);
    if (e != hipSuccess) return e;
    e = launch_gemm_bf16(B, n->width, n->width, n->z1, n->width, 1, 1, n->p + n->off_w[1], 1, n->width, 0, 1.0f,
                         n->p + n->off_b[1], nullptr, 0, 0, n->z2, n->width, s);
    if (e != hipSuccess) return e;
    return launch_gemm_bf16(B, n->out, n->width, n->z2, n->width, 1, 1, n->p + n->off_w[2], 1, n->width, 0, 1.0f,
                            n->p + n->off_b[2], nullptr, 0, 0, z3, n->out, s);
}

namespace nssdoa {

void mlp_dims(nssdoa_mlp n, int32_t* in, int32_t* width, int32_t* out, int32_t* max_batch) {
    *in = n->in;
    *width = n->width;
    *out = n->out;
    *max_batch = n->max_batch;
}

hipError_t mlp_forward_rows(nssdoa_mlp n, const float* feats, int rows, float* logits, hipStream_t s) {
    for (int r0 = 0; r0 < rows; r0 += n->max_batch) {
        const int B = rows - r0 < n->max_batch ? rows - r0 : n->max_batch;
        hipError_t e = mlp_forward(n, feats + (size_t)r0 * n->in, B, logits + (size_t)r0 * n->out, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace nssdoa

extern "C" {

nssdoa_status nssdoa_mlp_forward(nssdoa_mlp n, const float* feats, int32_t batch, float* logits, void* stream) {
    if (!n || !feats || !logits) return nssdoa_internal_fail(NSSDOA_EINVAL, "NULL argument");
    if (batch < 1 || batch > n->max_batch) return nssdoa_internal_fail(NSSDOA_EINVAL, "batch outside [1, max_batch]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = mlp_forward(n, feats, batch, logits, s);
    return e == hipSuccess ? NSSDOA_OK : mlp_fail(e, "mlp forward");
}

nssdoa_status nssdoa_mlp_train_step(nssdoa_mlp n, const float* feats, const float* targets, int32_t batch,
                                    float lr, float* loss, void* stream) {
    if (!n || !feats || !targets || !loss) return nssdoa_internal_fail(NSSDOA_EINVAL, "NULL argument");
    if (batch < 1 || batch > n->max_batch) return nssdoa_internal_fail(NSSDOA_EINVAL, "batch outside [1, max_batch]");
    if (!(lr >= 0.0f) || !(lr < 1e3f)) return nssdoa_internal_fail(NSSDOA_EINVAL, "learning rate must be in [0, 1e3)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int B = batch, W = n->width, O = n->out, I = n->in;
    hipError_t e = mlp_forward(n, feats, B, n->z3, s);
    // loss and dZ3 = (sigmoid(Z3) - Y) / (B O)
    if (e == hipSuccess) e = launch_bce(B, O, n->z3, targets, n->d3, n->row_loss, loss, s);
    // layer 3: dW3 = dZ3^T relu(Z2), db3 = colsum(dZ3), dZ2 = (dZ3 W3) * (Z2 > 0)
    if (e == hipSuccess)
        e = launch_gemm_bf16(O, W, B, n->d3, 1, O, 0, n->z2, W, 1, 1, 1.0f, nullptr, nullptr, 0, 0,
                             n->g + n->off_w[2], W, s);
    if (e == hipSuccess) e = launch_colsum(B, O, n->d3, O, n->g + n->off_b[2], s);
    if (e == hipSuccess)
        e = launch_gemm_bf16(B, W, O, n->d3, O, 1, 0, n->p + n->off_w[2], W, 1, 0, 1.0f, nullptr, n->z2, W, 0,
                             n->d2, W, s);
    // layer 2: dW2 = dZ2^T relu(Z1), db2 = colsum(dZ2), dZ1 = (dZ2 W2) * (Z1 > 0)
    if (e == hipSuccess)
        e = launch_gemm_bf16(W, W, B, n->d2, 1, W, 0, n->z1, W, 1, 1, 1.0f, nullptr, nullptr, 0, 0,
                             n->g + n->off_w[1], W, s);
    if (e == hipSuccess) e = launch_colsum(B, W, n->d2, W, n->g + n->off_b[1], s);
    if (e == hipSuccess)
        e = launch_gemm_bf16(B, W, W, n->d2, W, 1, 0, n->p + n->off_w[1], W, 1, 0, 1.0f, nullptr, n->z1, W, 0,
                             n->d1, W, s);
    // layer 1: dW1 = dZ1^T X, db1 = colsum(dZ1)
    if (e == hipSuccess)
        e = launch_gemm_bf16(W, I, B, n->d1, 1, W, 0, feats, I, 1, 0, 1.0f, nullptr, nullptr, 0, 0,
                             n->g + n->off_w[0], I, s);
    if (e == hipSuccess) e = launch_colsum(B, W, n->d1, W, n->g + n->off_b[0], s);
    if (e == hipSuccess) e = launch_adam((int)n->nparam, n->p, n->g, n->m, n->v, lr, n->step + 1, s);
    if (e != hipSuccess) return mlp_fail(e, "mlp train step");
    n->step += 1;
    return NSSDOA_OK;
}

}  // extern "C"
