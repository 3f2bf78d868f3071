// C ABI of the learned initial weights (declared in include/muca.h).
//
// A small MLP maps (model one-hot, 8/L, E/N) to ln Omega(E) / N.  It is
// trained on weights that the multicanonical recursion itself converged to
// at small L (W = 1/Omega when the histogram is flat, Sec. 2) and seeds the
// weight iteration at larger L.  Training, gradients and prediction run in
// the HIP kernels of mlp_kernels.hip; the host only stages data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/muca.h"
#include "mlp_device.h"

using namespace muca;

namespace {
std::string g_mlp_error;
constexpr size_t kAlignM = 256;
constexpr int kLossChunk = 4096;
size_t alignm(size_t v) { return (v + kAlignM - 1) / kAlignM * kAlignM; }

struct MlpLayout {
    size_t p, pbf, m, v, grad, grad_part, loss_part, y, dy, z1, z2, z3, a0, a1, a2, a3, x, t, loss, total;
};

MlpLayout mlp_layout(int max_n) {
    MlpLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off = alignm(off + bytes); return r; };
    const size_t n = (size_t)max_n, tiles = (n + 63) / 64;
    L.p = take(4 * kMlpParams);
    L.pbf = take(2 * kMlpParams);
    L.m = take(4 * kMlpParams);
    L.v = take(4 * kMlpParams);
    L.grad = take(4 * kMlpParams);
    L.grad_part = take(4 * kMlpParams * tiles);
    L.loss_part = take(4 * tiles);
    L.y = take(4 * n);
    L.dy = take(4 * n);
    L.z1 = take(4 * n * kMlpHidden);
    L.z2 = take(4 * n * kMlpHidden);
    L.z3 = take(4 * n * kMlpHidden);
    L.a0 = take(2 * n * kMlpIn);
    L.a1 = take(2 * n * kMlpHidden);
    L.a2 = take(2 * n * kMlpHidden);
    L.a3 = take(2 * n * kMlpHidden);
    L.x = take(4 * n * kMlpIn);
    L.t = take(4 * n);
    L.loss = take(4 * kLossChunk);
    L.total = off;
    return L;
}

uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
}  // namespace

struct muca_mlp_s {
    std::string err;
    hipStream_t stream = nullptr;
    int max_n = 0;
    uint8_t *ws = nullptr;
    MlpLayout lay;
    MlpBuffers b{};
    float *d_x = nullptr, *d_t = nullptr, *d_loss = nullptr;
    std::vector<float> hx, hy;   // staged training data
    int step = 0;                // Adam steps taken
};

namespace {
muca_status mfail(muca_mlp m, muca_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (m) m->err = buf; else g_mlp_error = buf;
    return st;
}
#define MHIP(m, expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return mfail(m, MUCA_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

muca_status upload_data(muca_mlp m, int *n_out) {
    const int n = (int)m->hy.size();
    if (n <= 0) return mfail(m, MUCA_ESTATE, "no training data");
    if (n > m->max_n) return mfail(m, MUCA_EINVAL, "%d samples exceed the capacity %d", n, m->max_n);
    MHIP(m, hipMemcpyAsync(m->d_x, m->hx.data(), 4 * (size_t)n * kMlpIn, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->d_t, m->hy.data(), 4 * (size_t)n, hipMemcpyHostToDevice, m->stream));
    *n_out = n;
    return MUCA_OK;
}

// Features of bin k of a problem: model one-hot, 8/L, E/N.
void features(int model, int L, int k, float *x) {
    const double N = (double)L * L;
    const double E = (model == MUCA_ISING) ? -2.0 * N + 2.0 * k : -2.0 * N + k;
    x[0] = model == MUCA_ISING ? 1.0f : 0.0f;
    x[1] = model == MUCA_ISING ? 0.0f : 1.0f;
    x[2] = (float)(8.0 / L);
    x[3] = (float)(E / N);
}
}  // namespace

extern "C" {

muca_status mucaMlpWorkspaceSize(int32_t max_samples, size_t *bytes) {
    if (max_samples < 1 || max_samples > (1 << 22) || !bytes)
        return mfail(nullptr, MUCA_EINVAL, "max_samples must be 1..2^22");
    *bytes = mlp_layout(max_samples).total;
    return MUCA_OK;
}

muca_status mucaMlpCreate(muca_mlp *out, int32_t max_samples, uint64_t seed, void *d_workspace, size_t ws_bytes,
                          void *hip_stream) {
    if (!out) return mfail(nullptr, MUCA_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_samples < 1 || max_samples > (1 << 22)) return mfail(nullptr, MUCA_EINVAL, "max_samples must be 1..2^22");
    const MlpLayout L = mlp_layout(max_samples);
    if (!d_workspace) return mfail(nullptr, MUCA_EINVAL, "workspace is NULL");
    if (ws_bytes < L.total) return mfail(nullptr, MUCA_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (((uintptr_t)d_workspace) % kAlignM) return mfail(nullptr, MUCA_EINVAL, "workspace must be 256-byte aligned");
    muca_mlp m = new muca_mlp_s();
    m->stream = (hipStream_t)hip_stream;
    m->max_n = max_samples;
    m->ws = (uint8_t *)d_workspace;
    m->lay = L;
    uint8_t *w = m->ws;
    m->b.p = (float *)(w + L.p);
    m->b.pbf = (uint16_t *)(w + L.pbf);
    m->b.m = (float *)(w + L.m);
    m->b.v = (float *)(w + L.v);
    m->b.grad = (float *)(w + L.grad);
    m->b.grad_part = (float *)(w + L.grad_part);
    m->b.loss_part = (float *)(w + L.loss_part);
    m->b.y = (float *)(w + L.y);
    m->b.dy = (float *)(w + L.dy);
    m->b.z1 = (float *)(w + L.z1);
    m->b.z2 = (float *)(w + L.z2);
    m->b.z3 = (float *)(w + L.z3);
    m->b.a0 = (uint16_t *)(w + L.a0);
    m->b.a1 = (uint16_t *)(w + L.a1);
    m->b.a2 = (uint16_t *)(w + L.a2);
    m->b.a3 = (uint16_t *)(w + L.a3);
    m->d_x = (float *)(w + L.x);
    m->d_t = (float *)(w + L.t);
    m->d_loss = (float *)(w + L.loss);
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases
    std::vector<float> p(kMlpParams);
    uint64_t st = seed;
    auto fill = [&](int off, int count, int fan_in) {
        const double bound = 1.0 / std::sqrt((double)fan_in);
        for (int i = 0; i < count; ++i) {
            const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            p[off + i] = (float)((2.0 * u - 1.0) * bound);
        }
    };
    fill(0, 256, 4);
    fill(256, 64, 4);
    fill(320, 4096, 64);
    fill(4416, 64, 64);
    fill(4480, 4096, 64);
    fill(8576, 64, 64);
    fill(8640, 64, 64);
    fill(8704, 1, 64);
    muca_status rc = mucaMlpSetParams(m, p.data());
    if (rc) {
        g_mlp_error = m->err;
        delete m;
        return rc;
    }
    *out = m;
    return MUCA_OK;
}

muca_status mucaMlpSetParams(muca_mlp m, const float *params) {
    if (!m || !params) return MUCA_EINVAL;
    MHIP(m, hipMemcpyAsync(m->b.p, params, 4 * kMlpParams, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemsetAsync(m->b.m, 0, 4 * kMlpParams, m->stream));
    MHIP(m, hipMemsetAsync(m->b.v, 0, 4 * kMlpParams, m->stream));
    MHIP(m, mlp_launch_cast(m->b, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    m->step = 0;
    return MUCA_OK;
}

muca_status mucaMlpGetParams(muca_mlp m, float *params) {
    if (!m || !params) return MUCA_EINVAL;
    MHIP(m, hipMemcpyAsync(params, m->b.p, 4 * kMlpParams, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return MUCA_OK;
}

muca_status mucaMlpClearData(muca_mlp m) {
    if (!m) return MUCA_EINVAL;
    m->hx.clear();
    m->hy.clear();
    return MUCA_OK;
}

muca_status mucaMlpAddData(muca_mlp m, const float *x, const float *y, int32_t n) {
    if (!m || !x || !y || n < 0) return MUCA_EINVAL;
    if ((int64_t)m->hy.size() + n > m->max_n) return mfail(m, MUCA_EINVAL, "data would exceed %d samples", m->max_n);
    m->hx.insert(m->hx.end(), x, x + (size_t)n * kMlpIn);
    m->hy.insert(m->hy.end(), y, y + n);
    return MUCA_OK;
}

muca_status mucaMlpAddWeights(muca_mlp m, muca_ctx ctx, int32_t prob) {
    if (!m || !ctx) return MUCA_EINVAL;
    muca_problem def;
    muca_status st = mucaProblemInfo(ctx, prob, &def);
    if (st) return mfail(m, st, "%s", mucaLastError(ctx));
    if (def.model == MUCA_ISING_MAG) return mfail(m, MUCA_EINVAL, "the network learns weights over the energy only");
    const int N = def.L * def.L, nb = 2 * N + 1;
    std::vector<double> lnW(nb);
    std::vector<uint8_t> reach(nb);
    if ((st = mucaGet(ctx, MUCA_GET_LNW, prob, lnW.data(), 8 * (size_t)nb))) return mfail(m, st, "%s", mucaLastError(ctx));
    if ((st = mucaGet(ctx, MUCA_GET_REACH, prob, reach.data(), (size_t)nb))) return mfail(m, st, "%s", mucaLastError(ctx));
    // ln Omega = -lnW + c, with c fixed by sum_k Omega(k) = q^N (logsumexp over reachable bins)
    double mx = -INFINITY;
    for (int k = 0; k < nb; ++k)
        if (reach[k]) mx = std::max(mx, -lnW[k]);
    double s = 0.0;
    for (int k = 0; k < nb; ++k)
        if (reach[k]) s += std::exp(-lnW[k] - mx);
    const double q = def.model == MUCA_ISING ? 2.0 : (double)def.q;
    const double c = N * std::log(q) - (mx + std::log(s));
    std::vector<float> x, y;
    for (int k = 0; k < nb; ++k) {
        if (!reach[k]) continue;
        float f[kMlpIn];
        features(def.model, def.L, k, f);
        x.insert(x.end(), f, f + kMlpIn);
        y.push_back((float)((-lnW[k] + c) / N));
    }
    return mucaMlpAddData(m, x.data(), y.data(), (int32_t)y.size());
}

muca_status mucaMlpNumSamples(muca_mlp m, int32_t *n) {
    if (!m || !n) return MUCA_EINVAL;
    *n = (int32_t)m->hy.size();
    return MUCA_OK;
}

muca_status mucaMlpTrain(muca_mlp m, int32_t steps, float lr, float *loss_out) {
    if (!m || steps < 0 || !(lr > 0.0f)) return mfail(m, MUCA_EINVAL, "steps >= 0 and lr > 0 required");
    int n = 0;
    muca_status st = upload_data(m, &n);
    if (st) return st;
    for (int done = 0; done < steps;) {
        const int chunk = std::min(kLossChunk, steps - done);
        for (int i = 0; i < chunk; ++i) {
            MHIP(m, mlp_launch_forward(m->b, m->d_x, m->d_t, n, 1, m->stream));
            MHIP(m, mlp_launch_loss(m->b, n, m->d_loss, i, m->stream));
            MHIP(m, mlp_launch_backward(m->b, n, m->stream));
            m->step += 1;
            MHIP(m, mlp_launch_adam(m->b, n, m->step, lr, m->stream));
        }
        if (loss_out)
            MHIP(m, hipMemcpyAsync(loss_out + done, m->d_loss, 4 * (size_t)chunk, hipMemcpyDeviceToHost, m->stream));
        MHIP(m, hipStreamSynchronize(m->stream));
        done += chunk;
    }
    return MUCA_OK;
}

muca_status mucaMlpGradients(muca_mlp m, float *grad, float *loss) {
    if (!m || !grad) return MUCA_EINVAL;
    int n = 0;
    muca_status st = upload_data(m, &n);
    if (st) return st;
    MHIP(m, mlp_launch_forward(m->b, m->d_x, m->d_t, n, 1, m->stream));
    MHIP(m, mlp_launch_loss(m->b, n, m->d_loss, 0, m->stream));
    MHIP(m, mlp_launch_backward(m->b, n, m->stream));
    MHIP(m, mlp_launch_adam(m->b, n, 0, 0.0f, m->stream));   // sums the tile gradients only
    MHIP(m, hipMemcpyAsync(grad, m->b.grad, 4 * kMlpParams, hipMemcpyDeviceToHost, m->stream));
    if (loss) MHIP(m, hipMemcpyAsync(loss, m->d_loss, 4, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return MUCA_OK;
}

muca_status mucaMlpPredict(muca_mlp m, const float *x, int32_t n, float *y) {
    if (!m || !x || !y || n < 1) return MUCA_EINVAL;
    if (n > m->max_n) return mfail(m, MUCA_EINVAL, "%d samples exceed the capacity %d", n, m->max_n);
    MHIP(m, hipMemcpyAsync(m->d_x, x, 4 * (size_t)n * kMlpIn, hipMemcpyHostToDevice, m->stream));
    MHIP(m, mlp_launch_forward(m->b, m->d_x, nullptr, n, 0, m->stream));
    MHIP(m, hipMemcpyAsync(y, m->b.y, 4 * (size_t)n, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return MUCA_OK;
}

muca_status mucaMlpSetLogWeights(muca_mlp m, muca_ctx ctx, int32_t prob) {
    if (!m || !ctx) return MUCA_EINVAL;
    muca_problem def;
    muca_status st = mucaProblemInfo(ctx, prob, &def);
    if (st) return mfail(m, st, "%s", mucaLastError(ctx));
    if (def.model == MUCA_ISING_MAG) return mfail(m, MUCA_EINVAL, "the network predicts weights over the energy only");
    const int N = def.L * def.L, nb = 2 * N + 1;
    if (nb > m->max_n) return mfail(m, MUCA_EINVAL, "problem has %d bins > capacity %d", nb, m->max_n);
    std::vector<uint8_t> reach(nb);
    if ((st = mucaGet(ctx, MUCA_GET_REACH, prob, reach.data(), (size_t)nb))) return mfail(m, st, "%s", mucaLastError(ctx));
    std::vector<float> x((size_t)nb * kMlpIn), y(nb);
    for (int k = 0; k < nb; ++k) features(def.model, def.L, k, &x[(size_t)k * kMlpIn]);
    if ((st = mucaMlpPredict(m, x.data(), nb, y.data()))) return st;
    // W = 1/Omega: lnW = -N * (ln Omega / N); unreachable bins keep 0
    std::vector<double> lnW(nb, 0.0);
    for (int k = 0; k < nb; ++k)
        if (reach[k]) lnW[k] = -(double)N * (double)y[k];
    st = mucaSetLogWeights(ctx, prob, lnW.data(), nb);
    if (st) return mfail(m, st, "%s", mucaLastError(ctx));
    return MUCA_OK;
}

void mucaMlpDestroy(muca_mlp m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    delete m;
}

const char *mucaMlpLastError(muca_mlp m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

}  // extern "C"
