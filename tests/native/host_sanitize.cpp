// Drives the library's entry points that need no GPU (mucaEqualHeight,
// mucaWorkspaceSize, mucaMlpWorkspaceSize, the error strings) over ordinary,
// degenerate and invalid inputs.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code: any out-of-bounds access,
// leak or undefined operation ends the run with an error report.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "muca.h"

static unsigned long long state = 88172645463325252ull;
static double uniform() {  // xorshift64, for test inputs only
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            failures++;                                                   \
        }                                                                 \
    } while (0)

static void touch_error() {
    const char *e = mucaLastError(nullptr);
    CHECK(e != nullptr);
    if (e) CHECK(std::strlen(e) < 4096);
}

int main() {
    int calls = 0, ok = 0;
    for (int model = 0; model < 4; ++model) {
        for (int L : {2, 3, 4, 8, 16}) {
            const int nb = 2 * L * L + 1;
            for (int trial = 0; trial < 60; ++trial) {
                int n = nb;
                if (trial % 7 == 0) n = nb - 1;
                if (trial % 11 == 0) n = 1;
                if (trial % 13 == 0) n = 0;
                std::vector<double> w(n > 0 ? n : 1), lnP(n > 0 ? n : 1);
                std::vector<int64_t> c(n > 0 ? n : 1);
                for (int k = 0; k < n; ++k) {
                    const double x = (double)k / nb;
                    // double wells of random depth, holes in the counts, a NaN now and then
                    w[k] = 40.0 * std::cos(4.0 * M_PI * x) * uniform() + 3.0 * x;
                    if (trial % 5 == 0 && k == n / 2) w[k] = NAN;
                    c[k] = (trial % 3 == 0 && uniform() < 0.6) ? 0 : (int64_t)(uniform() * 1000.0);
                    if (trial % 17 == 0) c[k] = 0;
                }
                double beta = 0.0, sigma = 0.0;
                int32_t kp[3] = {-7, -7, -7};
                const double lo = uniform() * 2.0 - 0.5;
                const double hi = (trial % 19 == 0) ? lo : uniform() * 2.0;
                const muca_status rc =
                    mucaEqualHeight(model, L, w.data(), c.data(), n, lo, hi, &beta, &sigma, kp, lnP.data());
                calls++;
                if (rc == MUCA_OK) {
                    ok++;
                    CHECK(model == MUCA_ISING || model == MUCA_POTTS);
                    CHECK(n == nb);
                    CHECK(0 <= kp[0] && kp[0] < kp[1] && kp[1] < kp[2] && kp[2] < n);
                    CHECK(std::isfinite(beta) && std::isfinite(sigma) && sigma >= 0.0);
                } else {
                    touch_error();
                }
            }
        }
    }
    {
        double b, s;
        int32_t kp[3];
        CHECK(mucaEqualHeight(MUCA_POTTS, 8, nullptr, nullptr, 129, 0.0, 1.0, &b, &s, kp, nullptr) != MUCA_OK);
        touch_error();
    }

    std::vector<muca_problem> probs;
    for (int i = 0; i < 40; ++i) {
        muca_problem p{};
        p.model = i % 4;
        p.q = (p.model == MUCA_POTTS) ? 2 + i % 8 : 2;
        p.L = 2 + 2 * (i % 12) + (i % 5 == 0);
        p.n_chains = (i % 9 == 0) ? 0 : 1 + i * 37;
        p.seed = (uint64_t)i;
        p.beta = 0.5;
        probs.push_back(p);
    }
    muca_options opt{};
    size_t bytes = 0;
    for (int cw : {-1, 0, 1, 17, 64, 65}) {
        opt.chains_per_wg = cw;
        for (int np : {0, 1, 5, 40}) {
            if (mucaWorkspaceSize(probs.data(), np, &opt, &bytes) != MUCA_OK) touch_error();
        }
        CHECK(mucaWorkspaceSize(nullptr, 3, &opt, &bytes) != MUCA_OK);
        touch_error();
    }
    size_t mb = 0;
    for (int n : {-5, 0, 1, 4096, 1 << 22, (1 << 22) + 1}) {
        const bool valid = n >= 1 && n <= (1 << 22);
        CHECK((mucaMlpWorkspaceSize(n, &mb) == MUCA_OK) == valid);
    }
    std::printf("equal-height calls %d, %d solved; failures %d\n", calls, ok, failures);
    return failures ? 1 : 0;
}
