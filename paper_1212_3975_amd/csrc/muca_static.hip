// mucaReweightStatic: time-series reweighting (Eq. 2) of caller-held
// production data without any device allocation.  The reweighting kernel's
// inputs and outputs are staged in a file-scope device array instead of a
// context's workspace, so a caller that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc)
// can still reweight.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "../../include/muca.h"
#include "muca_device.h"

namespace muca {
namespace {

// Largest problem: Ising or Potts with L = 256, 2 * 256^2 + 1 bins.
constexpr int kStaticMaxBins = 2 * 256 * 256 + 1;
constexpr int kStaticMaxBetas = 4096;
constexpr size_t kSeg = 256;   // section alignment

constexpr size_t seg(size_t bytes) { return (bytes + kSeg - 1) / kSeg * kSeg; }
// Sections of the array: merged counts, |M| sums, lnW, betas, outputs [3][betas].
constexpr size_t kOffH = 0;
constexpr size_t kOffS = kOffH + seg(8 * (size_t)kStaticMaxBins);
constexpr size_t kOffW = kOffS + seg(8 * (size_t)kStaticMaxBins);
constexpr size_t kOffB = kOffW + seg(8 * (size_t)kStaticMaxBins);
constexpr size_t kOffO = kOffB + seg(8 * (size_t)kStaticMaxBetas);
constexpr size_t kStaticBytes = kOffO + seg(3 * 8 * (size_t)kStaticMaxBetas);   // 3,277,568 bytes
static_assert(kStaticBytes == 3277568, "size stated in muca.h");

// Every GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

muca_status fail_static(muca_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
muca_status fail_static(muca_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_context_free_error(buf);
    return st;
}

// The device address of `scratch` on the current device, looked up once per
// device with that device current.  The host-side name `scratch` is only a
// stand-in for the symbol and is never handed to a kernel or a copy.
muca_status scratch_of_current_device(unsigned char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_static(MUCA_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail_static(MUCA_EINVAL, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail_static(MUCA_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch[dev];
    return MUCA_OK;
}

}  // namespace
}  // namespace muca

using namespace muca;

extern "C" muca_status mucaReweightStatic(int32_t model, int32_t L, const double *lnW, const int64_t *cnt,
                                          const int64_t *sabs, int32_t n_bins, const double *betas, int32_t n_betas,
                                          double *e_per_site, double *c_v, double *abs_m_per_site,
                                          void *hip_stream) {
    if (model == MUCA_ISING) {
        if (L < 4 || L > 256 || (L & 1)) return fail_static(MUCA_EINVAL, "Ising needs even L in 4..256");
    } else if (model == MUCA_POTTS) {
        if (L < 3 || L > 256) return fail_static(MUCA_EINVAL, "Potts needs L in 3..256");
    } else {
        return fail_static(MUCA_EINVAL, "model must be MUCA_ISING or MUCA_POTTS");
    }
    const int N = L * L, nb = 2 * N + 1;
    if (n_bins != nb) return fail_static(MUCA_EINVAL, "n_bins must be 2N+1 = %d", nb);
    if (n_bins > kStaticMaxBins) return fail_static(MUCA_EINVAL, "at most %d bins", kStaticMaxBins);
    if (n_betas < 1 || n_betas > kStaticMaxBetas)
        return fail_static(MUCA_EINVAL, "n_betas must be 1..%d", kStaticMaxBetas);
    if (!lnW || !cnt || !betas || !e_per_site || !c_v || !abs_m_per_site || (model == MUCA_ISING && !sabs))
        return fail_static(MUCA_EINVAL, "NULL array");
    int64_t total = 0;
    for (int k = 0; k < nb; ++k) {
        if (!std::isfinite(lnW[k])) return fail_static(MUCA_EINVAL, "lnW[%d] is not finite", k);
        if (cnt[k] < 0) return fail_static(MUCA_EINVAL, "cnt[%d] is negative", k);
        total += cnt[k];
    }
    if (total == 0) return fail_static(MUCA_ESTATE, "no production data (every count is 0)");
    for (int j = 0; j < n_betas; ++j)
        if (!std::isfinite(betas[j])) return fail_static(MUCA_EINVAL, "betas[%d] is not finite", j);

    unsigned char *base = nullptr;
    muca_status st = scratch_of_current_device(&base);
    if (st) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    ProbDev p{};
    p.model = model;
    p.q = model == MUCA_ISING ? 2 : 0;
    p.L = L;
    p.N = N;
    p.nbins = nb;
    p.H = (int64_t *)(base + kOffH);
    p.S = (int64_t *)(base + kOffS);
    p.lnW = (const double *)(base + kOffW);
    double *d_betas = (double *)(base + kOffB);
    double *d_out = (double *)(base + kOffO);
#define SCHECK(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail_static(MUCA_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
    SCHECK(hipMemcpyAsync(p.H, cnt, 8 * (size_t)nb, hipMemcpyHostToDevice, s));
    // the kernel reads the |M| sums for Ising only (Potts gives NaN)
    if (model == MUCA_ISING) SCHECK(hipMemcpyAsync(p.S, sabs, 8 * (size_t)nb, hipMemcpyHostToDevice, s));
    SCHECK(hipMemcpyAsync((void *)p.lnW, lnW, 8 * (size_t)nb, hipMemcpyHostToDevice, s));
    SCHECK(hipMemcpyAsync(d_betas, betas, 8 * (size_t)n_betas, hipMemcpyHostToDevice, s));
    SCHECK(launch_reweight(p, d_betas, n_betas, d_out, s));
    SCHECK(hipMemcpyAsync(e_per_site, d_out, 8 * (size_t)n_betas, hipMemcpyDeviceToHost, s));
    SCHECK(hipMemcpyAsync(c_v, d_out + n_betas, 8 * (size_t)n_betas, hipMemcpyDeviceToHost, s));
    SCHECK(hipMemcpyAsync(abs_m_per_site, d_out + 2 * n_betas, 8 * (size_t)n_betas, hipMemcpyDeviceToHost, s));
    SCHECK(hipStreamSynchronize(s));
#undef SCHECK
    return MUCA_OK;
}
