// Host runtime and C ABI of the MUCA library (declared in include/muca.h).
//
// Per weight iteration the device runs the sweeps and the merge; the host
// applies the recursion W <- W / H in logarithms (Sec. 2) to the 2N+1 merged
// bins and rebuilds the acceptance tables, which are O(bins) steps.  They
// stay on the host on purpose: log and exp come from the C library in IEEE
// double (compiled without contraction or fast-math), so the weights and the
// tables are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/muca.h"
#include "muca_device.h"

using namespace muca;

namespace {

std::string g_init_error;

constexpr size_t kAlign = 256;
constexpr int kMaxBetas = 4096;
constexpr uint32_t kAlways = 0xFFFFFFFFu;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// floor(2^32 * min(1, exp(delta))) with the "always" value for results that
// would reach 2^32 - 1 (the threshold of the acceptance test).
uint32_t threshold(double delta) {
    if (delta >= 0.0) return kAlways;
    const double x = std::ldexp(std::exp(delta), 32);
    if (x >= 4294967295.0) return kAlways;
    return (uint32_t)std::floor(x);
}

// Bins that can occur: Ising (even L) every even k except 2 and 2N-2; Potts
// (q >= 3) every k except 1, 2, 3 and 5; multimagnetic every m = 0..N.
void reachable_mask(int model, int N, std::vector<uint8_t> &mask) {
    if (model == MUCA_ISING_MAG) {
        mask.assign(N + 1, 1);
        return;
    }
    mask.assign(2 * N + 1, 1);
    if (model == MUCA_ISING) {
        for (int k = 0; k <= 2 * N; ++k)
            if (k & 1) mask[k] = 0;
        mask[2] = 0;
        mask[2 * N - 2] = 0;
    } else {
        mask[1] = mask[2] = mask[3] = mask[5] = 0;
    }
}

struct ProbHost {
    muca_problem def;
    int N, nbins, trows, tcols;
    std::vector<double> lnW;
    std::vector<uint8_t> reach;
    int chains_per_wg = 0, spin_lds = 0, table_lds = 0;
    size_t off_spins, off_k, off_m, off_hist, off_sabs, off_tab, off_H, off_S, off_lnW, off_backup;
    size_t tab_stage_off;   // offset (in uint32 words) of this problem's table in the staging buffer
    muca_iter_stats last{};
    bool prod_alloc = false;   // production accumulators exist
    bool prod_data = false;    // a production sweep has run
};

}  // namespace

struct muca_ctx_s {
    std::string err;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int device = 0;
    int max_lds = 65536;
    muca_options opt{};
    std::vector<ProbHost> probs;
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    // shared device regions
    ProbDev *d_probs = nullptr;
    WorkItem *d_items = nullptr;
    MergeItem *d_merge = nullptr;
    uint32_t *d_sweep = nullptr;
    double *d_betas = nullptr;
    double *d_rw_out = nullptr;
    uint32_t *d_tables = nullptr;   // all device tables, contiguous
    int64_t *d_H = nullptr;         // all merged histograms, contiguous
    size_t tab_words = 0, h_words = 0;
    // host mirrors
    std::vector<ProbDev> h_probdev;
    std::vector<WorkItem> items;
    std::vector<MergeItem> merge_items;
    int n_producer_waves = 0;
    int lds_bytes = 0;
    uint32_t sweep = 0;
    // pinned staging
    int64_t *pin_H = nullptr;
    uint32_t *pin_tab = nullptr;
    // graph of one iteration
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t graph_sweeps = -1;
    int graph_status = 0;
    // timing of sweep launches
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timing;
    std::vector<hipEvent_t> event_pool;
};

namespace {

muca_status fail(muca_ctx ctx, muca_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_init_error = buf;
    return st;
}

#define HIPCHECK(ctx, expr)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, MUCA_EHIP, "%s failed: %s (line %d)", #expr, hipGetErrorString(e_), \
                        __LINE__);                                                               \
    } while (0)

muca_status validate(const muca_problem *pr, int32_t n, const muca_options *o) {
    if (!pr || n <= 0 || n > 64) return fail(nullptr, MUCA_EINVAL, "need 1..64 problems");
    for (int i = 0; i < n; ++i) {
        const muca_problem &p = pr[i];
        if (p.model == MUCA_ISING || p.model == MUCA_ISING_MAG) {
            if (p.L < 4 || p.L > 256 || (p.L & 1))
                return fail(nullptr, MUCA_EINVAL, "problem %d: Ising needs even L in 4..256", i);
            if (p.model == MUCA_ISING_MAG && !(p.beta >= 0.0 && p.beta <= 10.0))
                return fail(nullptr, MUCA_EINVAL, "problem %d: multimagnetic beta must be in [0, 10]", i);
        } else if (p.model == MUCA_POTTS) {
            if (p.L < 3 || p.L > 256) return fail(nullptr, MUCA_EINVAL, "problem %d: Potts needs L in 3..256", i);
            if (p.q < 3 || p.q > 8) return fail(nullptr, MUCA_EINVAL, "problem %d: Potts needs q in 3..8", i);
        } else {
            return fail(nullptr, MUCA_EINVAL, "problem %d: unknown model %d", i, p.model);
        }
        if (p.n_chains < 1 || p.n_chains > (1 << 20))
            return fail(nullptr, MUCA_EINVAL, "problem %d: n_chains must be 1..2^20", i);
    }
    if (o) {
        const int cw = o->chains_per_wg;
        if (cw < 0 || cw > 64) return fail(nullptr, MUCA_EINVAL, "chains_per_wg must be 0 (tune) or 1..64");
        if (o->rng_mode < 0 || o->rng_mode > 1 + kMaxProducerWaves)
            return fail(nullptr, MUCA_EINVAL, "rng_mode must be 0..%d", 1 + kMaxProducerWaves);
        if (o->spin_placement < 0 || o->spin_placement > 2 || o->table_placement < 0 || o->table_placement > 2)
            return fail(nullptr, MUCA_EINVAL, "placements must be 0..2");
        if (o->flat_rule < 0 || o->flat_rule > 1) return fail(nullptr, MUCA_EINVAL, "flat_rule must be 0 or 1");
        if (o->correction < 0 || o->correction > 1) return fail(nullptr, MUCA_EINVAL, "correction must be 0 or 1");
        if (o->update_norm < 0 || o->update_norm > 1) return fail(nullptr, MUCA_EINVAL, "update_norm must be 0 or 1");
    }
    return MUCA_OK;
}

muca_options defaults(const muca_options *o) {
    muca_options d{};
    if (o) d = *o;
    if (d.flat_ratio <= 0.0) d.flat_ratio = 0.5;
    if (d.tune_sweeps <= 0) d.tune_sweeps = 4;
    return d;
}

struct Layout {
    std::vector<ProbHost> probs;
    size_t off_probdev, off_items, off_merge, off_sweep, off_betas, off_rwout, off_tables, off_H, total;
    size_t tab_words, h_words;
    int max_items, n_merge;
};

int merge_items_for(int nbins) { return (nbins + 7) / 8; }

Layout plan_layout(const muca_problem *pr, int32_t n, const muca_options &o) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t r = off; off = align_up(off + bytes); return r; };
    L.tab_words = 0;
    L.h_words = 0;
    L.max_items = 0;
    L.n_merge = 0;
    for (int i = 0; i < n; ++i) {
        ProbHost h;
        h.def = pr[i];
        if (h.def.model != MUCA_POTTS) h.def.q = 2;
        if (h.def.model != MUCA_ISING_MAG) h.def.beta = 0.0;
        h.N = pr[i].L * pr[i].L;
        h.nbins = (h.def.model == MUCA_ISING_MAG) ? h.N + 1 : 2 * h.N + 1;
        h.trows = (h.def.model == MUCA_POTTS) ? h.nbins : h.N + 1;
        h.tcols = (h.def.model == MUCA_ISING) ? 5 : (h.def.model == MUCA_ISING_MAG) ? 10 : 9;
        const size_t C = (size_t)pr[i].n_chains;
        h.off_spins = take((size_t)h.N * C);
        h.off_k = take(4 * C);
        h.off_m = take(4 * C);
        h.off_hist = take(4 * (size_t)h.nbins * C);
        h.off_sabs = o.production ? take(8 * (size_t)h.nbins * C) : (size_t)-1;
        h.off_lnW = take(8 * (size_t)h.nbins);
        h.off_S = take(8 * (size_t)h.nbins);
        h.off_backup = take((size_t)h.N * C + 8 * C);
        h.tab_stage_off = L.tab_words;
        L.tab_words += (size_t)h.trows * h.tcols;
        L.tab_words = (L.tab_words + 63) / 64 * 64;
        h.off_H = L.h_words;   // words into the H region
        L.h_words += (size_t)h.nbins;
        L.max_items += (pr[i].n_chains + 3) / 4;
        L.n_merge += merge_items_for(h.nbins);
        L.probs.push_back(h);
    }
    L.off_probdev = take(sizeof(ProbDev) * n);
    L.off_items = take(sizeof(WorkItem) * L.max_items);
    L.off_merge = take(sizeof(MergeItem) * L.n_merge);
    L.off_sweep = take(2 * sizeof(uint32_t));   // sweep counter, status word
    L.off_betas = take(sizeof(double) * kMaxBetas);
    L.off_rwout = take(sizeof(double) * 3 * kMaxBetas);
    L.off_tables = take(4 * L.tab_words);
    L.off_H = take(8 * L.h_words);
    L.total = off;
    return L;
}

// Flatness statistics over reachable bins, and the recursion (Sec. 2-3).
void stats_of(const ProbHost &p, const int64_t *H, double ratio, int rule, muca_iter_stats &s) {
    s = muca_iter_stats{};
    s.k_lo = -1;
    s.k_hi = -1;
    int64_t hmin = INT64_MAX, hmax = 0, total = 0, nreach = 0;
    double sum = 0;
    bool covered = true;
    for (int k = 0; k < p.nbins; ++k) {
        total += H[k];
        if (H[k] > 0) {
            if (s.k_lo < 0) s.k_lo = k;
            s.k_hi = k;
            s.visited++;
        }
        if (p.reach[k]) {
            nreach++;
            hmin = std::min(hmin, H[k]);
            hmax = std::max(hmax, H[k]);
            sum += (double)H[k];
            if (H[k] <= 0) covered = false;
        }
    }
    const double avg = nreach ? sum / (double)nreach : 0.0;
    s.reachable = (int32_t)nreach;
    s.covered = covered;
    s.total = total;
    s.min_over_max = hmax > 0 ? (double)hmin / (double)hmax : 0.0;
    s.min_over_avg = avg > 0 ? (double)hmin / avg : 0.0;
    s.max_over_avg = avg > 0 ? (double)hmax / avg : 0.0;
    bool flat;
    if (rule == 0) {
        flat = covered && s.min_over_max >= ratio;
    } else {
        flat = covered;
        for (int k = 0; k < p.nbins && flat; ++k)
            if (p.reach[k] && ((double)H[k] < 0.5 * avg || (double)H[k] > 2.0 * avg)) flat = false;
    }
    s.flat = flat;
}

void recursion(ProbHost &p, const int64_t *H, int update_norm) {
    if (!update_norm) {
        for (int k = 0; k < p.nbins; ++k)
            if (H[k] > 0) p.lnW[k] -= std::log((double)H[k]);
        return;
    }
    // the update shifted to zero mean over the visited bins
    double sum = 0.0;
    int n = 0;
    for (int k = 0; k < p.nbins; ++k)
        if (H[k] > 0) {
            sum += std::log((double)H[k]);
            ++n;
        }
    const double mean = n > 0 ? sum / n : 0.0;
    for (int k = 0; k < p.nbins; ++k)
        if (H[k] > 0) p.lnW[k] -= std::log((double)H[k]) - mean;
}

// Correction function (Sec. 3): beyond each edge of the sampled region,
// continue lnW on a straight line through the edge bin and the reachable bin
// L reachable bins inward (or the other edge when the region is narrower).
void correction(ProbHost &p, const int64_t *H) {
    int lo = -1, hi = -1;
    for (int k = 0; k < p.nbins; ++k)
        if (H[k] > 0) {
            if (lo < 0) lo = k;
            hi = k;
        }
    if (lo < 0 || lo == hi) return;
    const int L = p.def.L;
    auto inward = [&](int edge, int dir) {
        int k = edge, count = 0;
        while (count < L) {
            const int nk = k + dir;
            if (nk < lo || nk > hi) break;
            k = nk;
            if (p.reach[k]) ++count;
        }
        return k;
    };
    const int in_lo = inward(lo, +1), in_hi = inward(hi, -1);
    if (in_lo != lo) {
        const double slope = (p.lnW[lo] - p.lnW[in_lo]) / (double)(lo - in_lo);
        for (int k = 0; k < lo; ++k)
            if (p.reach[k]) p.lnW[k] = p.lnW[lo] + slope * (double)(k - lo);
    }
    if (in_hi != hi) {
        const double slope = (p.lnW[hi] - p.lnW[in_hi]) / (double)(hi - in_hi);
        for (int k = hi + 1; k < p.nbins; ++k)
            if (p.reach[k]) p.lnW[k] = p.lnW[hi] + slope * (double)(k - hi);
    }
}

// Device-layout table of one problem (see muca_device.h).
void device_table(const ProbHost &p, uint32_t *out) {
    const int n = p.nbins;
    if (p.def.model == MUCA_ISING_MAG) {
        // row m (up spins), column j + 5u: an up spin (u = 1) goes to m - 1,
        // a down spin to m + 1; the flip changes k by dk = 2j - 4, E by 2 dk
        const double beta = p.def.beta;
        for (int m = 0; m < n; ++m)
            for (int u = 0; u < 2; ++u) {
                const int t = u ? m - 1 : m + 1;
                for (int j = 0; j < 5; ++j) {
                    const int dk = 2 * j - 4;
                    out[m * 10 + j + 5 * u] =
                        (t >= 0 && t < n) ? threshold((p.lnW[t] - p.lnW[m]) - beta * (double)(2 * dk)) : 0u;
                }
            }
    } else if (p.def.model == MUCA_ISING) {
        for (int r = 0; r < p.trows; ++r) {
            const int k = 2 * r;
            for (int j = 0; j < 5; ++j) {
                const int t = k + 2 * (j - 2);
                out[r * 5 + j] = (t >= 0 && t < n) ? threshold(p.lnW[t] - p.lnW[k]) : 0u;
            }
        }
    } else {
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < 9; ++j) {
                const int t = k + (j - 4);
                out[k * 9 + j] = (t >= 0 && t < n) ? threshold(p.lnW[t] - p.lnW[k]) : 0u;
            }
    }
}

void build_all_tables(muca_ctx ctx) {
    for (auto &p : ctx->probs) device_table(p, ctx->pin_tab + p.tab_stage_off);
}

ProbDev make_probdev(muca_ctx ctx, const ProbHost &h) {
    ProbDev d{};
    d.model = h.def.model;
    d.q = h.def.q;
    d.L = h.def.L;
    d.N = h.N;
    d.nbins = h.nbins;
    d.C = h.def.n_chains;
    d.trows = h.trows;
    d.tcols = h.tcols;
    d.seed_lo = (uint32_t)(h.def.seed & 0xFFFFFFFFull);
    d.seed_hi = (uint32_t)(h.def.seed >> 32);
    d.spin_lds = h.spin_lds;
    d.table_lds = h.table_lds;
    uint8_t *w = ctx->ws;
    d.spins = w + h.off_spins;
    d.k = (int32_t *)(w + h.off_k);
    d.m = (int32_t *)(w + h.off_m);
    d.hist = (int32_t *)(w + h.off_hist);
    d.sabs = (h.off_sabs == (size_t)-1) ? nullptr : (int64_t *)(w + h.off_sabs);
    d.table = ctx->d_tables + h.tab_stage_off;
    d.H = ctx->d_H + h.off_H;
    d.S = (int64_t *)(w + h.off_S);
    d.lnW = (const double *)(w + h.off_lnW);
    return d;
}

// Work items and LDS size for the current per-problem configuration.
muca_status plan_launch(muca_ctx ctx, const std::vector<int> &only) {
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));   // the previous upload may still read items
    ctx->items.clear();
    int lds = 0;
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        if (!only.empty() && std::find(only.begin(), only.end(), (int)pi) == only.end()) continue;
        const ProbHost &h = ctx->probs[pi];
        const int cw = h.chains_per_wg;
        for (int c0 = 0; c0 < h.def.n_chains; c0 += cw) {
            WorkItem it;
            it.prob = (int)pi;
            it.chain0 = c0;
            it.nchains = std::min(cw, h.def.n_chains - c0);
            it.spin_stride = (it.nchains + 3) / 4 * 4;
            ctx->items.push_back(it);
            lds = std::max(lds, lds_bytes_for(ctx->h_probdev[pi], it, ctx->n_producer_waves));
        }
    }
    if (lds > ctx->max_lds) return fail(ctx, MUCA_EINVAL, "launch needs %d LDS bytes > %d", lds, ctx->max_lds);
    ctx->lds_bytes = lds;
    HIPCHECK(ctx, hipMemcpyAsync(ctx->d_items, ctx->items.data(), sizeof(WorkItem) * ctx->items.size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    return MUCA_OK;
}

muca_status upload_probdev(muca_ctx ctx) {
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));   // the previous upload may still read h_probdev
    ctx->h_probdev.clear();
    for (auto &h : ctx->probs) ctx->h_probdev.push_back(make_probdev(ctx, h));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->d_probs, ctx->h_probdev.data(), sizeof(ProbDev) * ctx->h_probdev.size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    return MUCA_OK;
}

// Whether a placement fits in LDS for chains_per_wg chains.
bool fits(muca_ctx ctx, const ProbHost &h, int cw, int spin_lds, int table_lds, int nprod) {
    ProbDev d = make_probdev(ctx, h);
    d.spin_lds = spin_lds;
    d.table_lds = table_lds;
    WorkItem it{0, 0, std::min(cw, h.def.n_chains), (std::min(cw, h.def.n_chains) + 3) / 4 * 4};
    return lds_bytes_for(d, it, nprod) <= ctx->max_lds;
}

// The walkers count a launch's chunks in int32: the longest launch the
// current configuration allows.
int64_t max_sweeps_per_launch(muca_ctx ctx) {
    int64_t worst = 1;
    for (const WorkItem &it : ctx->items)
        worst = std::max<int64_t>(worst, chunks_per_sweep(ctx->h_probdev[it.prob], it, ctx->n_producer_waves));
    return (int64_t)INT32_MAX / worst;
}

muca_status check_sweeps(muca_ctx ctx, int64_t n_sweeps) {
    if (n_sweeps > (1 << 30)) return fail(ctx, MUCA_EINVAL, "n_sweeps out of range");
    const int64_t cap = max_sweeps_per_launch(ctx);
    if (n_sweeps > cap)
        return fail(ctx, MUCA_EINVAL, "n_sweeps %lld exceeds %lld, the most one launch of this configuration counts",
                    (long long)n_sweeps, (long long)cap);
    if ((uint64_t)ctx->sweep + (uint64_t)n_sweeps > 0xFFFFFFFFull)
        return fail(ctx, MUCA_ESTATE, "sweep counter would wrap");
    return MUCA_OK;
}

// The status word of the sweep launches (after the stream has drained): a
// walker whose bounded wait for its producer waves expired (or theirs for it)
// has left the chains in an invalid state.  The word stays set.
muca_status check_walk_status(muca_ctx ctx) {
    uint32_t w = 0;
    HIPCHECK(ctx, hipMemcpyAsync(&w, ctx->d_sweep + 1, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (w & kStatusWaitExpired)
        return fail(ctx, MUCA_EHIP, "a sweep's bounded wait between walker and producer waves expired; "
                                    "the chains' state is not valid");
    return MUCA_OK;
}

muca_status enqueue_sweep(muca_ctx ctx, int64_t n_sweeps, int record, bool timed) {
    SweepLaunch l;
    l.probs = ctx->d_probs;
    l.items = ctx->d_items;
    l.n_items = (int)ctx->items.size();
    l.n_producer_waves = ctx->n_producer_waves;
    l.lds_bytes = ctx->lds_bytes;
    l.n_sweeps = (int)n_sweeps;
    l.record = record;
    l.sweep_ctr = ctx->d_sweep;
    l.status = ctx->d_sweep + 1;
    l.wait_polls = ctx->opt.wait_polls == 0 ? (1u << 24) : ctx->opt.wait_polls < 0 ? 0u : (uint32_t)ctx->opt.wait_polls;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        if (ctx->event_pool.size() < 2) {
            hipEvent_t a, b;
            HIPCHECK(ctx, hipEventCreate(&a));
            HIPCHECK(ctx, hipEventCreate(&b));
            ctx->event_pool.push_back(a);
            ctx->event_pool.push_back(b);
        }
        e1 = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        e0 = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        HIPCHECK(ctx, hipEventRecord(e0, ctx->stream));
    }
    bool cstream = false;
    for (const WorkItem &it : ctx->items)
        cstream = cstream || walker_kind(ctx->h_probdev[it.prob], it, ctx->n_producer_waves) >= 8;
    HIPCHECK(ctx, launch_sweep(l, cstream, ctx->stream));
    if (timed) {
        HIPCHECK(ctx, hipEventRecord(e1, ctx->stream));
        ctx->timing.push_back({e0, e1});
    }
    return MUCA_OK;
}

// Candidate timing for the tuner: sweeps without recording, state restored after.
muca_status time_config(muca_ctx ctx, const std::vector<int> &only, int sweeps, float *ms) {
    muca_status st = upload_probdev(ctx);
    if (st) return st;
    if ((st = plan_launch(ctx, only))) return st;
    hipEvent_t a, b;
    HIPCHECK(ctx, hipEventCreate(&a));
    HIPCHECK(ctx, hipEventCreate(&b));
    // one untimed launch first (LDS staging, caches)
    if ((st = enqueue_sweep(ctx, 1, kRecNone, false))) return st;
    HIPCHECK(ctx, hipEventRecord(a, ctx->stream));
    if ((st = enqueue_sweep(ctx, sweeps, kRecNone, false))) return st;
    HIPCHECK(ctx, hipEventRecord(b, ctx->stream));
    HIPCHECK(ctx, hipEventSynchronize(b));
    HIPCHECK(ctx, hipEventElapsedTime(ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return MUCA_OK;
}

muca_status backup_state(muca_ctx ctx, bool restore) {
    for (auto &h : ctx->probs) {
        uint8_t *w = ctx->ws;
        const size_t C = h.def.n_chains, nsp = (size_t)h.N * C;
        uint8_t *bk = w + h.off_backup;
        if (!restore) {
            HIPCHECK(ctx, launch_copy_bytes(bk, w + h.off_spins, nsp, ctx->stream));
            HIPCHECK(ctx, launch_copy_bytes(bk + nsp, w + h.off_k, 4 * C, ctx->stream));
            HIPCHECK(ctx, launch_copy_bytes(bk + nsp + 4 * C, w + h.off_m, 4 * C, ctx->stream));
        } else {
            HIPCHECK(ctx, launch_copy_bytes(w + h.off_spins, bk, nsp, ctx->stream));
            HIPCHECK(ctx, launch_copy_bytes(w + h.off_k, bk + nsp, 4 * C, ctx->stream));
            HIPCHECK(ctx, launch_copy_bytes(w + h.off_m, bk + nsp + 4 * C, 4 * C, ctx->stream));
        }
    }
    return MUCA_OK;
}

// Picks chains per workgroup, random-number mode and placements.
muca_status configure(muca_ctx ctx) {
    const muca_options &o = ctx->opt;
    // rng candidates: own (0 producers) or 1..3 producer waves
    std::vector<int> rng_cands;
    if (o.rng_mode == 0) rng_cands = {0, 1, 2, 3, 4};
    else if (o.rng_mode == 1) rng_cands = {0};
    else rng_cands = {std::min(kMaxProducerWaves, std::max(1, o.rng_mode - 1))};
    std::vector<int> cw_cands;
    if (o.chains_per_wg) cw_cands = {o.chains_per_wg};
    else cw_cands = {16, 32, 64};
    const bool tune = (rng_cands.size() > 1 || cw_cands.size() > 1 || o.spin_placement == 0 ||
                       o.table_placement == 0);

    // placement per problem for a given cw / nprod: prefer LDS where it fits
    auto place = [&](ProbHost &h, int cw, int nprod) -> bool {
        int sl_c[2], tl_c[2], ns = 0, nt = 0;
        if (o.spin_placement != 2) sl_c[ns++] = 1;
        if (o.spin_placement != 1) sl_c[ns++] = 0;
        if (o.table_placement != 2) tl_c[nt++] = 1;
        if (o.table_placement != 1) tl_c[nt++] = 0;
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < ns; ++b)
                if (fits(ctx, h, cw, sl_c[b], tl_c[a], nprod)) {
                    h.chains_per_wg = cw;
                    h.spin_lds = sl_c[b];
                    h.table_lds = tl_c[a];
                    return true;
                }
        return false;
    };

    if (!tune) {
        ctx->n_producer_waves = rng_cands[0];
        for (auto &h : ctx->probs) {
            bool ok = false;
            for (int cw : cw_cands) if ((ok = place(h, cw, ctx->n_producer_waves))) break;
            if (!ok) return fail(ctx, MUCA_EINVAL, "no placement fits in LDS");
        }
        muca_status st = upload_probdev(ctx);
        if (st) return st;
        return plan_launch(ctx, {});
    }

    muca_status st = backup_state(ctx, false);
    if (st) return st;
    float best_total = 1e30f;
    std::vector<ProbHost> best_cfg;
    int best_nprod = 0;
    for (int nprod : rng_cands) {
        ctx->n_producer_waves = nprod;
        bool all_ok = true;
        for (size_t pi = 0; pi < ctx->probs.size() && all_ok; ++pi) {
            ProbHost &h = ctx->probs[pi];
            float best = 1e30f;
            ProbHost keep = h;
            bool any = false;
            // besides the fixed sizes, the most chains whose lattice and table both fit in LDS
            std::vector<int> cands = cw_cands;
            if (!o.chains_per_wg && o.spin_placement != 2 && o.table_placement != 2) {
                int top = 0;
                for (int cw = 64; cw >= 1 && !top; --cw)
                    if (fits(ctx, h, cw, 1, 1, nprod)) top = cw;
                if (top && std::find(cands.begin(), cands.end(), top) == cands.end()) cands.push_back(top);
            }
            for (int cw : cands) {
                if (!place(h, cw, nprod)) continue;
                float ms = 0;
                if ((st = time_config(ctx, {(int)pi}, o.tune_sweeps, &ms))) return st;
                if (ms < best) {
                    best = ms;
                    keep = h;
                    any = true;
                }
            }
            if (!any) all_ok = false;
            else h = keep;
        }
        if (!all_ok) continue;
        float ms = 0;
        if ((st = time_config(ctx, {}, o.tune_sweeps, &ms))) return st;
        if (ms < best_total) {
            best_total = ms;
            best_cfg = ctx->probs;
            best_nprod = nprod;
        }
    }
    if (best_cfg.empty()) return fail(ctx, MUCA_EINVAL, "no launch configuration fits");
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        ctx->probs[pi].chains_per_wg = best_cfg[pi].chains_per_wg;
        ctx->probs[pi].spin_lds = best_cfg[pi].spin_lds;
        ctx->probs[pi].table_lds = best_cfg[pi].table_lds;
    }
    ctx->n_producer_waves = best_nprod;
    if ((st = backup_state(ctx, true))) return st;
    if ((st = upload_probdev(ctx))) return st;
    return plan_launch(ctx, {});
}

muca_status upload_tables(muca_ctx ctx) {
    HIPCHECK(ctx, hipMemcpyAsync(ctx->d_tables, ctx->pin_tab, 4 * ctx->tab_words, hipMemcpyHostToDevice,
                                 ctx->stream));
    return MUCA_OK;
}

// Host half of an iteration: statistics, recursion and tables from pin_H.
void host_update(muca_ctx ctx, int update) {
    for (auto &p : ctx->probs) {
        const int64_t *H = ctx->pin_H + p.off_H;
        stats_of(p, H, ctx->opt.flat_ratio, ctx->opt.flat_rule, p.last);
        if (update) {
            recursion(p, H, ctx->opt.update_norm);
            if (ctx->opt.correction) correction(p, H);
            device_table(p, ctx->pin_tab + p.tab_stage_off);
        }
    }
}

void host_update_cb(void *arg) { host_update((muca_ctx)arg, 1); }

muca_status enqueue_merge(muca_ctx ctx, int production, hipStream_t s) {
    HIPCHECK(ctx, launch_merge(ctx->d_probs, ctx->d_merge, (int)ctx->merge_items.size(), production, 1, s));
    return MUCA_OK;
}

muca_status check_prob(muca_ctx ctx, int32_t prob) {
    if (!ctx) return MUCA_EINVAL;
    if (prob < 0 || prob >= (int)ctx->probs.size()) return fail(ctx, MUCA_EINVAL, "bad problem index %d", prob);
    return MUCA_OK;
}

// Equal-height analysis of a reweighted energy histogram (Sec. 5, Eq. 9).
// At inverse temperature beta, bin k with cnt_k > 0 carries
// a_k = ln cnt_k - lnW_k - beta E_k (the log of the canonical probability up to
// a constant).  The two peaks are the maxima of a on either side of the
// weighted mean bin; the minimum is taken between them.
struct PeakSplit {
    int ko = -1, km = -1, kd = -1;   // ordered peak, minimum, disordered peak
    double ao = 0, am = 0, ad = 0;
};

// a_k = ln cnt_k - lnW_k - beta E_k (the log canonical probability at beta up
// to a constant, Eq. 2) over the bins with data, in increasing k.
void log_canonical(const int64_t *cnt, const double *lnW, const double *E, int nb, double beta,
                   std::vector<int> &ks, std::vector<double> &a) {
    ks.clear();
    a.clear();
    for (int k = 0; k < nb; ++k)
        if (cnt[k] > 0) {
            ks.push_back(k);
            a.push_back(std::log((double)cnt[k]) - lnW[k] - beta * E[k]);
        }
}

// The bin separating the ordered from the disordered peak.  A point scores as
// the bottom of a double peak with its depth below the lower of the highest
// values on its two sides (itself included), less |ln(M_left / M_right)|, M
// the probability (sum of e^a) on each side, the point counted on both.  The
// two phases of a double peak carry comparable probability; an isolated bin
// at an edge or a dip in a tail does not, and scores below zero.  The split
// is the best point at the beta of the bracket where the best score is
// highest, over 65 equally spaced beta.  Fixed in k, it makes the peak-height
// difference continuous and increasing in beta.  False if no point scores
// above zero.
bool valley_split(const int64_t *cnt, const double *lnW, const double *E, int nb, double beta_lo, double beta_hi,
                  int &split) {
    std::vector<int> ks;
    std::vector<double> a, right, mright;
    double best = 0.0;
    split = -1;
    for (int i = 0; i <= 64; ++i) {
        const double beta = beta_lo + (beta_hi - beta_lo) * i / 64.0;
        log_canonical(cnt, lnW, E, nb, beta, ks, a);
        const int n = (int)a.size();
        if (n == 0) return false;
        double A = a[0];
        for (int j = 1; j < n; ++j) A = std::max(A, a[j]);
        right.assign(n, 0.0);
        mright.assign(n, 0.0);
        right[n - 1] = a[n - 1];
        mright[n - 1] = std::exp(a[n - 1] - A);
        for (int j = n - 2; j >= 0; --j) {
            right[j] = std::max(right[j + 1], a[j]);
            mright[j] = mright[j + 1] + std::exp(a[j] - A);
        }
        double left = -HUGE_VAL, mleft = 0.0, smax = -HUGE_VAL;
        int jmax = -1;
        for (int j = 0; j < n; ++j) {
            left = std::max(left, a[j]);
            mleft += std::exp(a[j] - A);
            const double sc = std::min(left, right[j]) - a[j] - std::fabs(std::log(mleft) - std::log(mright[j]));
            if (jmax < 0 || sc > smax) smax = sc, jmax = j;
        }
        if (smax > best) best = smax, split = ks[jmax];
    }
    return split >= 0;
}

// The ordered peak (largest a_k at k <= split), the disordered peak (largest
// a_k at k > split) and the smallest a_k between them, at beta.
bool split_peaks(const int64_t *cnt, const double *lnW, const double *E, int nb, double beta, int split,
                 PeakSplit &ps) {
    std::vector<int> ks;
    std::vector<double> a;
    log_canonical(cnt, lnW, E, nb, beta, ks, a);
    ps = PeakSplit();
    int io = -1, id = -1;
    for (int j = 0; j < (int)ks.size(); ++j) {
        if (ks[j] <= split) {
            if (io < 0 || a[j] > a[io]) io = j;
        } else {
            if (id < 0 || a[j] > a[id]) id = j;
        }
    }
    if (io < 0 || id < 0) return false;
    int im = io;
    for (int j = io; j <= id; ++j)
        if (a[j] < a[im]) im = j;
    ps.ko = ks[io], ps.ao = a[io];
    ps.kd = ks[id], ps.ad = a[id];
    ps.km = ks[im], ps.am = a[im];
    return true;
}

muca_status equal_height(muca_ctx ctx, int32_t model, int32_t L, const double *lnW, const int64_t *cnt,
                         int32_t n_bins, double beta_lo, double beta_hi, double *beta_out, double *sigma_out,
                         int32_t *k3, double *lnP) {
    if ((model != MUCA_ISING && model != MUCA_POTTS) || L < 2 || !lnW || !cnt || !beta_out || !sigma_out)
        return fail(ctx, MUCA_EINVAL, "bad arguments");
    const int N = L * L, nb = 2 * N + 1;
    if (n_bins != nb) return fail(ctx, MUCA_EINVAL, "n_bins must be 2N+1 = %d", nb);
    if (!(beta_lo < beta_hi)) return fail(ctx, MUCA_EINVAL, "need beta_lo < beta_hi");
    std::vector<double> E(nb);
    for (int k = 0; k < nb; ++k) E[k] = (double)(-2 * N + (model == MUCA_ISING ? 2 * k : k));
    int split = -1;
    if (!valley_split(cnt, lnW, E.data(), nb, beta_lo, beta_hi, split))
        return fail(ctx, MUCA_ESTATE, "histogram has no two peaks");
    PeakSplit lo_ps, hi_ps;
    if (!split_peaks(cnt, lnW, E.data(), nb, beta_lo, split, lo_ps) ||
        !split_peaks(cnt, lnW, E.data(), nb, beta_hi, split, hi_ps))
        return fail(ctx, MUCA_ESTATE, "histogram has no two peaks");
    // the ordered (low-energy) peak gains on the disordered one as beta grows
    if (!(lo_ps.ao - lo_ps.ad < 0.0 && hi_ps.ao - hi_ps.ad > 0.0))
        return fail(ctx, MUCA_ESTATE, "peak heights do not cross in [%g, %g]", beta_lo, beta_hi);
    double lo = beta_lo, hi = beta_hi;
    PeakSplit ps;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (!split_peaks(cnt, lnW, E.data(), nb, mid, split, ps)) return fail(ctx, MUCA_ESTATE, "lost the two peaks");
        if (ps.ao - ps.ad < 0.0) lo = mid;
        else hi = mid;
    }
    const double beta = 0.5 * (lo + hi);
    if (!split_peaks(cnt, lnW, E.data(), nb, beta, split, ps)) return fail(ctx, MUCA_ESTATE, "lost the two peaks");
    // a single peak splits into two neighbouring "maxima" with no bin between them
    if (!(ps.ko < ps.km && ps.km < ps.kd)) return fail(ctx, MUCA_ESTATE, "histogram has no two peaks");
    *beta_out = beta;
    *sigma_out = (0.5 * (ps.ao + ps.ad) - ps.am) / (2.0 * L);
    if (k3) k3[0] = ps.ko, k3[1] = ps.km, k3[2] = ps.kd;
    if (lnP) {
        // normalised log-probabilities at the equal-height beta, -inf where cnt = 0
        double A = -HUGE_VAL;
        for (int k = 0; k < nb; ++k)
            if (cnt[k] > 0) A = std::max(A, std::log((double)cnt[k]) - lnW[k] - beta * E[k]);
        double z = 0.0;
        for (int k = 0; k < nb; ++k)
            if (cnt[k] > 0) z += std::exp(std::log((double)cnt[k]) - lnW[k] - beta * E[k] - A);
        const double lz = A + std::log(z);
        for (int k = 0; k < nb; ++k)
            lnP[k] = (cnt[k] > 0) ? std::log((double)cnt[k]) - lnW[k] - beta * E[k] - lz : -HUGE_VAL;
    }
    return MUCA_OK;
}

void drop_graph(muca_ctx ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_sweeps = -1;
}

}  // namespace

void muca::set_context_free_error(const char *text) { g_init_error = text; }

extern "C" {

muca_status mucaWorkspaceSize(const muca_problem *problems, int32_t n, const muca_options *opts, size_t *bytes) {
    muca_status st = validate(problems, n, opts);
    if (st) return st;
    if (!bytes) return MUCA_EINVAL;
    muca_options o = defaults(opts);
    *bytes = plan_layout(problems, n, o).total;
    return MUCA_OK;
}

muca_status mucaInit(muca_ctx *out, const muca_problem *problems, int32_t n, const muca_options *opts,
                     void *d_workspace, size_t ws_bytes, void *hip_stream) {
    if (!out) return fail(nullptr, MUCA_EINVAL, "out is NULL");
    *out = nullptr;
    muca_status st = validate(problems, n, opts);
    if (st) return st;
    muca_options o = defaults(opts);
    Layout L = plan_layout(problems, n, o);
    if (!d_workspace) return fail(nullptr, MUCA_EINVAL, "workspace is NULL");
    if (ws_bytes < L.total)
        return fail(nullptr, MUCA_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (((uintptr_t)d_workspace) % kAlign) return fail(nullptr, MUCA_EINVAL, "workspace must be 256-byte aligned");

    muca_ctx ctx = new muca_ctx_s();
    ctx->opt = o;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->ws = (uint8_t *)d_workspace;
    ctx->ws_bytes = ws_bytes;
    ctx->probs = L.probs;
    ctx->tab_words = L.tab_words;
    ctx->h_words = L.h_words;
    auto bail = [&](muca_status s) {
        g_init_error = ctx->err;
        mucaDestroy(ctx);
        return s;
    };
#define INITCHECK(expr)                                                                                \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            fail(ctx, MUCA_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));                       \
            return bail(MUCA_EHIP);                                                                    \
        }                                                                                              \
    } while (0)
    INITCHECK(hipGetDevice(&ctx->device));
    int lds = 0;
    INITCHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    ctx->max_lds = lds;
    // raising the dynamic-LDS limit is best effort; plan_launch enforces the limit
    (void)configure_sweep_kernel(lds);
    (void)hipGetLastError();
    uint8_t *w = ctx->ws;
    ctx->d_probs = (ProbDev *)(w + L.off_probdev);
    ctx->d_items = (WorkItem *)(w + L.off_items);
    ctx->d_merge = (MergeItem *)(w + L.off_merge);
    ctx->d_sweep = (uint32_t *)(w + L.off_sweep);
    ctx->d_betas = (double *)(w + L.off_betas);
    ctx->d_rw_out = (double *)(w + L.off_rwout);
    ctx->d_tables = (uint32_t *)(w + L.off_tables);
    ctx->d_H = (int64_t *)(w + L.off_H);
    INITCHECK(hipHostMalloc((void **)&ctx->pin_H, 8 * std::max<size_t>(1, L.h_words), hipHostMallocDefault));
    INITCHECK(hipHostMalloc((void **)&ctx->pin_tab, 4 * std::max<size_t>(1, L.tab_words), hipHostMallocDefault));
    std::memset(ctx->pin_H, 0, 8 * L.h_words);

    for (auto &h : ctx->probs) {
        h.lnW.assign(h.nbins, 0.0);
        reachable_mask(h.def.model, h.N, h.reach);
        h.chains_per_wg = 64;
        h.spin_lds = 0;
        h.table_lds = 0;
        h.prod_alloc = (h.off_sabs != (size_t)-1);
    }
    if ((st = upload_probdev(ctx))) return bail(st);
    // zero accumulators, counter and tables; draw the initial state
    INITCHECK(launch_fill_u32(ctx->d_sweep, 0u, 2, ctx->stream));
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        const ProbHost &h = ctx->probs[pi];
        const ProbDev &d = ctx->h_probdev[pi];
        const size_t C = h.def.n_chains;
        INITCHECK(launch_fill_u32((uint32_t *)d.hist, 0u, (size_t)h.nbins * C, ctx->stream));
        if (d.sabs) INITCHECK(launch_fill_u32((uint32_t *)d.sabs, 0u, 2 * (size_t)h.nbins * C, ctx->stream));
        INITCHECK(launch_fill_u32((uint32_t *)d.S, 0u, 2 * (size_t)h.nbins, ctx->stream));
        INITCHECK(launch_fill_u32((uint32_t *)(w + h.off_lnW), 0u, 2 * (size_t)h.nbins, ctx->stream));
        INITCHECK(launch_init(d, 0, (int)C, ctx->stream));
        INITCHECK(launch_energy(d, ctx->stream));
    }
    INITCHECK(launch_fill_u32((uint32_t *)ctx->d_H, 0u, 2 * L.h_words, ctx->stream));
    build_all_tables(ctx);
    if ((st = upload_tables(ctx))) return bail(st);
    // merge work: 8 bins per workgroup
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        const int nb = ctx->probs[pi].nbins;
        for (int b = 0; b < nb; b += 8) ctx->merge_items.push_back({(int)pi, b, std::min(8, nb - b), 0});
    }
    INITCHECK(hipMemcpyAsync(ctx->d_merge, ctx->merge_items.data(), sizeof(MergeItem) * ctx->merge_items.size(),
                             hipMemcpyHostToDevice, ctx->stream));
    if ((st = configure(ctx))) return bail(st);
    INITCHECK(hipStreamSynchronize(ctx->stream));
#undef INITCHECK
    *out = ctx;
    return MUCA_OK;
}

muca_status mucaSetLogWeights(muca_ctx ctx, int32_t prob, const double *lnW, int32_t n_bins) {
    muca_status st = check_prob(ctx, prob);
    if (st) return st;
    ProbHost &p = ctx->probs[prob];
    if (!lnW || n_bins != p.nbins) return fail(ctx, MUCA_EINVAL, "lnW must have 2N+1 = %d entries", p.nbins);
    for (int k = 0; k < n_bins; ++k)
        if (!std::isfinite(lnW[k])) return fail(ctx, MUCA_EINVAL, "lnW[%d] is not finite", k);
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));   // staging may still feed a copy
    p.lnW.assign(lnW, lnW + n_bins);
    device_table(p, ctx->pin_tab + p.tab_stage_off);
    st = upload_tables(ctx);
    if (st) return st;
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return MUCA_OK;
}

muca_status mucaSweep(muca_ctx ctx, int64_t n_sweeps, int32_t record) {
    if (!ctx) return MUCA_EINVAL;
    if (n_sweeps < 0) return fail(ctx, MUCA_EINVAL, "n_sweeps out of range");
    if (record < 0 || record > 2) return fail(ctx, MUCA_EINVAL, "record must be 0, 1 or 2");
    if (record == kRecProd && !ctx->probs[0].prod_alloc)
        return fail(ctx, MUCA_ESTATE, "context was created without production accumulators");
    if (n_sweeps == 0) return MUCA_OK;
    muca_status st = check_sweeps(ctx, n_sweeps);
    if (st) return st;
    st = enqueue_sweep(ctx, n_sweeps, record, true);
    if (st) return st;
    HIPCHECK(ctx, launch_advance(ctx->d_sweep, (uint32_t)n_sweeps, ctx->stream));
    ctx->sweep += (uint32_t)n_sweeps;
    if (record == kRecProd)
        for (auto &p : ctx->probs) p.prod_data = true;
    return MUCA_OK;
}

muca_status mucaMergeUpdate(muca_ctx ctx, int32_t update, muca_iter_stats *out) {
    if (!ctx) return MUCA_EINVAL;
    muca_status st = enqueue_merge(ctx, 0, ctx->stream);
    if (st) return st;
    HIPCHECK(ctx, hipMemcpyAsync(ctx->pin_H, ctx->d_H, 8 * ctx->h_words, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    if ((st = check_walk_status(ctx))) return st;
    host_update(ctx, update);
    if (update) {
        if ((st = upload_tables(ctx))) return st;
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (out)
        for (size_t i = 0; i < ctx->probs.size(); ++i) out[i] = ctx->probs[i].last;
    return MUCA_OK;
}

muca_status mucaIterate(muca_ctx ctx, int64_t n_sweeps, muca_iter_stats *out) {
    if (!ctx) return MUCA_EINVAL;
    if (n_sweeps <= 0) return fail(ctx, MUCA_EINVAL, "n_sweeps out of range");
    muca_status cs = check_sweeps(ctx, n_sweeps);
    if (cs) return cs;
    if (!ctx->opt.use_graph) {
        muca_status st = mucaSweep(ctx, n_sweeps, kRecMuca);
        if (st) return st;
        return mucaMergeUpdate(ctx, 1, out);
    }
    if (ctx->graph_sweeps != n_sweeps) {
        drop_graph(ctx);
        if (!ctx->capture_stream) HIPCHECK(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        hipStream_t cs = ctx->capture_stream;
        HIPCHECK(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        hipStream_t keep = ctx->stream;
        ctx->stream = cs;
        muca_status st = enqueue_sweep(ctx, n_sweeps, kRecMuca, false);
        hipError_t e = hipSuccess;
        if (!st) e = launch_advance(ctx->d_sweep, (uint32_t)n_sweeps, cs);
        if (!st && e == hipSuccess) st = enqueue_merge(ctx, 0, cs);
        if (!st && e == hipSuccess)
            e = hipMemcpyAsync(ctx->pin_H, ctx->d_H, 8 * ctx->h_words, hipMemcpyDeviceToHost, cs);
        if (!st && e == hipSuccess) e = hipLaunchHostFunc(cs, host_update_cb, ctx);
        if (!st && e == hipSuccess)
            e = hipMemcpyAsync(ctx->d_tables, ctx->pin_tab, 4 * ctx->tab_words, hipMemcpyHostToDevice, cs);
        ctx->stream = keep;
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(ctx, MUCA_EHIP, "graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        ctx->graph = g;
        HIPCHECK(ctx, hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
        ctx->graph_sweeps = n_sweeps;
    }
    HIPCHECK(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->sweep += (uint32_t)n_sweeps;
    if ((cs = check_walk_status(ctx))) return cs;
    if (out)
        for (size_t i = 0; i < ctx->probs.size(); ++i) out[i] = ctx->probs[i].last;
    return MUCA_OK;
}

muca_status mucaClearProduction(muca_ctx ctx) {
    if (!ctx) return MUCA_EINVAL;
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        const ProbHost &h = ctx->probs[pi];
        const ProbDev &d = ctx->h_probdev[pi];
        HIPCHECK(ctx, launch_fill_u32((uint32_t *)d.hist, 0u, (size_t)h.nbins * h.def.n_chains, ctx->stream));
        if (d.sabs)
            HIPCHECK(ctx, launch_fill_u32((uint32_t *)d.sabs, 0u, 2 * (size_t)h.nbins * h.def.n_chains, ctx->stream));
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return MUCA_OK;
}

muca_status mucaReweight(muca_ctx ctx, int32_t prob, const double *betas, int32_t n_betas, double *e_per_site,
                         double *c_v, double *abs_m_per_site) {
    muca_status st = check_prob(ctx, prob);
    if (st) return st;
    if (!betas || n_betas <= 0 || n_betas > kMaxBetas)
        return fail(ctx, MUCA_EINVAL, "n_betas must be 1..%d", kMaxBetas);
    if (!e_per_site || !c_v || !abs_m_per_site) return fail(ctx, MUCA_EINVAL, "NULL output");
    ProbHost &p = ctx->probs[prob];
    if (p.def.model == MUCA_ISING_MAG) return fail(ctx, MUCA_EINVAL, "reweighting in beta needs weights over E");
    if (!p.prod_data) return fail(ctx, MUCA_ESTATE, "no production data");
    // merge the production accumulators (counts into H, |M| sums into S), keep them
    HIPCHECK(ctx, launch_merge(ctx->d_probs, ctx->d_merge, (int)ctx->merge_items.size(), 1, 0, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync((void *)ctx->h_probdev[prob].lnW, p.lnW.data(), 8 * p.nbins,
                                 hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->d_betas, betas, 8 * n_betas, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, launch_reweight(ctx->h_probdev[prob], ctx->d_betas, n_betas, ctx->d_rw_out, ctx->stream));
    std::vector<double> res(3 * (size_t)n_betas);
    HIPCHECK(ctx, hipMemcpyAsync(res.data(), ctx->d_rw_out, 8 * res.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(e_per_site, res.data(), 8 * n_betas);
    std::memcpy(c_v, res.data() + n_betas, 8 * n_betas);
    std::memcpy(abs_m_per_site, res.data() + 2 * n_betas, 8 * n_betas);
    return MUCA_OK;
}

muca_status mucaEqualHeight(int32_t model, int32_t L, const double *lnW, const int64_t *cnt, int32_t n_bins,
                            double beta_lo, double beta_hi, double *beta_eqh, double *sigma_od, int32_t *k_peaks,
                            double *lnP) {
    return equal_height(nullptr, model, L, lnW, cnt, n_bins, beta_lo, beta_hi, beta_eqh, sigma_od, k_peaks, lnP);
}

muca_status mucaInterfaceTension(muca_ctx ctx, int32_t prob, double beta_lo, double beta_hi, double *beta_eqh,
                                 double *sigma_od, int32_t *k_peaks, double *lnP) {
    muca_status st = check_prob(ctx, prob);
    if (st) return st;
    ProbHost &p = ctx->probs[prob];
    if (p.def.model == MUCA_ISING_MAG) return fail(ctx, MUCA_EINVAL, "the interface analysis needs weights over E");
    if (!p.prod_data) return fail(ctx, MUCA_ESTATE, "no production data");
    // merge the production accumulators (counts into H), keep them
    HIPCHECK(ctx, launch_merge(ctx->d_probs, ctx->d_merge, (int)ctx->merge_items.size(), 1, 0, ctx->stream));
    std::vector<int64_t> cnt(p.nbins);
    HIPCHECK(ctx, hipMemcpyAsync(cnt.data(), ctx->h_probdev[prob].H, 8 * (size_t)p.nbins, hipMemcpyDeviceToHost,
                                 ctx->stream));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return equal_height(ctx, p.def.model, p.def.L, p.lnW.data(), cnt.data(), p.nbins, beta_lo, beta_hi, beta_eqh,
                        sigma_od, k_peaks, lnP);
}

muca_status mucaGet(muca_ctx ctx, int32_t what, int32_t prob, void *dst, size_t bytes) {
    muca_status st = check_prob(ctx, prob);
    if (st) return st;
    if (!dst) return fail(ctx, MUCA_EINVAL, "dst is NULL");
    const ProbHost &p = ctx->probs[prob];
    const ProbDev &d = ctx->h_probdev[prob];
    const size_t C = p.def.n_chains, nb = p.nbins;
    auto need = [&](size_t n) -> muca_status {
        if (bytes != n) return fail(ctx, MUCA_EINVAL, "item %d of problem %d has %zu bytes, got %zu", what, prob, n, bytes);
        return MUCA_OK;
    };
    auto d2h = [&](const void *src, size_t n) -> muca_status {
        HIPCHECK(ctx, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
        return check_walk_status(ctx);
    };
    switch (what) {
    case MUCA_GET_H:
        if ((st = need(8 * nb))) return st;
        return d2h(d.H, 8 * nb);
    case MUCA_GET_LNW:
        if ((st = need(8 * nb))) return st;
        HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
        std::memcpy(dst, p.lnW.data(), 8 * nb);
        return MUCA_OK;
    case MUCA_GET_T: {
        // the words the walkers read: this problem's device table, copied back
        const size_t words = (size_t)p.trows * p.tcols;
        if ((st = need(4 * words))) return st;
        return d2h(d.table, 4 * words);
    }
    case MUCA_GET_SPINS:
        if ((st = need((size_t)p.N * C))) return st;
        return d2h(d.spins, (size_t)p.N * C);
    case MUCA_GET_K:
        if ((st = need(4 * C))) return st;
        return d2h(d.k, 4 * C);
    case MUCA_GET_M:
        if ((st = need(4 * C))) return st;
        return d2h(d.m, 4 * C);
    case MUCA_GET_CHAIN_H:
        if ((st = need(4 * nb * C))) return st;
        return d2h(d.hist, 4 * nb * C);
    case MUCA_GET_PROD_CNT:
    case MUCA_GET_PROD_ABSM: {
        if ((st = need(8 * nb))) return st;
        if (!d.sabs) return fail(ctx, MUCA_ESTATE, "no production accumulators");
        HIPCHECK(ctx, launch_merge(ctx->d_probs, ctx->d_merge, (int)ctx->merge_items.size(), 1, 0, ctx->stream));
        return d2h(what == MUCA_GET_PROD_CNT ? (const void *)d.H : (const void *)d.S, 8 * nb);
    }
    case MUCA_GET_SWEEP:
        if ((st = need(4))) return st;
        *(uint32_t *)dst = ctx->sweep;
        return MUCA_OK;
    case MUCA_GET_REACH:
        if ((st = need(nb))) return st;
        std::memcpy(dst, p.reach.data(), nb);
        return MUCA_OK;
    default:
        return fail(ctx, MUCA_EINVAL, "unknown item %d", what);
    }
}

muca_status mucaLaunchInfo(muca_ctx ctx, int32_t prob, muca_launch_info *info) {
    muca_status st = check_prob(ctx, prob);
    if (st) return st;
    if (!info) return MUCA_EINVAL;
    const ProbHost &p = ctx->probs[prob];
    *info = muca_launch_info{};
    info->chains_per_wg = p.chains_per_wg;
    info->rng_mode = ctx->n_producer_waves == 0 ? 1 : 1 + ctx->n_producer_waves;
    info->spin_placement = p.spin_lds ? 1 : 2;
    info->table_placement = p.table_lds ? 1 : 2;
    info->lds_bytes = ctx->lds_bytes;
    int n = 0;
    for (auto &it : ctx->items) n += (it.prob == prob);
    info->n_workgroups = n;
    info->fast_walker = uses_fast_walker(ctx->h_probdev[prob], ctx->n_producer_waves) ? 1 : 0;
    for (auto &it : ctx->items)
        if (it.prob == prob) {
            info->walker = walker_kind(ctx->h_probdev[prob], it, ctx->n_producer_waves);
            break;
        }
    return MUCA_OK;
}

muca_status mucaSweepTiming(muca_ctx ctx, double *avg_ms, int32_t *n_launches) {
    if (!ctx || !avg_ms || !n_launches) return MUCA_EINVAL;
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    double tot = 0;
    for (auto &pr : ctx->timing) {
        float ms = 0;
        HIPCHECK(ctx, hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
        ctx->event_pool.push_back(pr.first);
        ctx->event_pool.push_back(pr.second);
    }
    *n_launches = (int32_t)ctx->timing.size();
    *avg_ms = ctx->timing.empty() ? 0.0 : tot / ctx->timing.size();
    ctx->timing.clear();
    return MUCA_OK;
}

// Checkpoint blob: header, then per problem spins, k, m, lnW, per-chain histograms.
namespace {
struct CkptHeader {
    uint64_t magic, version, n_problems, sweep;
};
constexpr uint64_t kMagic = 0x4D5543414B505431ull;   // "MUCAKPT1"
size_t ckpt_bytes(muca_ctx ctx) {
    size_t b = sizeof(CkptHeader);
    for (auto &p : ctx->probs) {
        const size_t C = p.def.n_chains;
        b += sizeof(muca_problem) + (size_t)p.N * C + 8 * C + 8 * (size_t)p.nbins + 4 * (size_t)p.nbins * C;
    }
    return b;
}
}  // namespace

muca_status mucaCheckpoint(muca_ctx ctx, void *blob, size_t *bytes) {
    if (!ctx || !bytes) return MUCA_EINVAL;
    const size_t need = ckpt_bytes(ctx);
    if (!blob) {
        *bytes = need;
        return MUCA_OK;
    }
    if (*bytes < need) return fail(ctx, MUCA_EINVAL, "checkpoint needs %zu bytes", need);
    uint8_t *o = (uint8_t *)blob;
    CkptHeader h{kMagic, 2, ctx->probs.size(), ctx->sweep};   // 2: problems carry beta
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        const ProbHost &p = ctx->probs[pi];
        const ProbDev &d = ctx->h_probdev[pi];
        const size_t C = p.def.n_chains;
        std::memcpy(o, &p.def, sizeof(muca_problem));
        o += sizeof(muca_problem);
        HIPCHECK(ctx, hipMemcpyAsync(o, d.spins, (size_t)p.N * C, hipMemcpyDeviceToHost, ctx->stream));
        o += (size_t)p.N * C;
        HIPCHECK(ctx, hipMemcpyAsync(o, d.k, 4 * C, hipMemcpyDeviceToHost, ctx->stream));
        o += 4 * C;
        HIPCHECK(ctx, hipMemcpyAsync(o, d.m, 4 * C, hipMemcpyDeviceToHost, ctx->stream));
        o += 4 * C;
        std::memcpy(o, p.lnW.data(), 8 * (size_t)p.nbins);
        o += 8 * (size_t)p.nbins;
        HIPCHECK(ctx, hipMemcpyAsync(o, d.hist, 4 * (size_t)p.nbins * C, hipMemcpyDeviceToHost, ctx->stream));
        o += 4 * (size_t)p.nbins * C;
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    muca_status st = check_walk_status(ctx);
    if (st) return st;
    *bytes = need;
    return MUCA_OK;
}

muca_status mucaRestore(muca_ctx ctx, const void *blob, size_t bytes) {
    if (!ctx || !blob) return MUCA_EINVAL;
    if (bytes != ckpt_bytes(ctx)) return fail(ctx, MUCA_EINVAL, "checkpoint size mismatch");
    const uint8_t *in = (const uint8_t *)blob;
    CkptHeader h;
    std::memcpy(&h, in, sizeof h);
    in += sizeof h;
    if (h.magic != kMagic || h.version != 2 || h.n_problems != ctx->probs.size())
        return fail(ctx, MUCA_EINVAL, "not a checkpoint of this context");
    // validate every problem before touching state
    const uint8_t *scan = in;
    for (auto &p : ctx->probs) {
        muca_problem def;
        std::memcpy(&def, scan, sizeof def);
        if (def.model != p.def.model || def.L != p.def.L || def.n_chains != p.def.n_chains ||
            def.seed != p.def.seed || (def.model == MUCA_POTTS && def.q != p.def.q) ||
            (def.model == MUCA_ISING_MAG && def.beta != p.def.beta))
            return fail(ctx, MUCA_EINVAL, "checkpoint problem differs from the context");
        const size_t C = p.def.n_chains;
        // spins outside 0..q-1 would break the walkers' byte arithmetic and
        // with it the tracked k that indexes the histograms
        const uint8_t *sp = scan + sizeof(muca_problem);
        const size_t ns = (size_t)p.N * C;
        const uint8_t q = (uint8_t)p.def.q;
        for (size_t i = 0; i < ns; ++i)
            if (sp[i] >= q)
                return fail(ctx, MUCA_EINVAL, "checkpoint spin %u out of range 0..%u in problem %zu", (unsigned)sp[i],
                            (unsigned)(q - 1), (size_t)(&p - ctx->probs.data()));
        // log-weights feed the thresholds: a NaN or an infinity has no threshold
        const uint8_t *lw = sp + ns + 8 * C;
        for (int k = 0; k < p.nbins; ++k) {
            double v;
            std::memcpy(&v, lw + 8 * (size_t)k, 8);
            if (!std::isfinite(v))
                return fail(ctx, MUCA_EINVAL, "checkpoint lnW[%d] of problem %zu is not finite", k,
                            (size_t)(&p - ctx->probs.data()));
        }
        scan += sizeof(muca_problem) + ns + 8 * C + 8 * (size_t)p.nbins + 4 * (size_t)p.nbins * C;
    }
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        ProbHost &p = ctx->probs[pi];
        const ProbDev &d = ctx->h_probdev[pi];
        const size_t C = p.def.n_chains;
        in += sizeof(muca_problem);
        HIPCHECK(ctx, hipMemcpy(d.spins, in, (size_t)p.N * C, hipMemcpyHostToDevice));
        in += (size_t)p.N * C;
        // k and M are recomputed from the spins rather than trusted, so a
        // damaged blob cannot point a chain outside its table
        in += 8 * C;
        HIPCHECK(ctx, launch_energy(d, ctx->stream));
        std::memcpy(p.lnW.data(), in, 8 * (size_t)p.nbins);
        in += 8 * (size_t)p.nbins;
        HIPCHECK(ctx, hipMemcpy(d.hist, in, 4 * (size_t)p.nbins * C, hipMemcpyHostToDevice));
        in += 4 * (size_t)p.nbins * C;
    }
    ctx->sweep = (uint32_t)h.sweep;
    HIPCHECK(ctx, hipMemcpy(ctx->d_sweep, &ctx->sweep, 4, hipMemcpyHostToDevice));
    build_all_tables(ctx);
    muca_status st = upload_tables(ctx);
    if (st) return st;
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    return MUCA_OK;
}

muca_status mucaProblemInfo(muca_ctx ctx, int32_t prob, muca_problem *out) {
    muca_status st = check_prob(ctx, prob);
    if (st) return st;
    if (!out) return MUCA_EINVAL;
    *out = ctx->probs[prob].def;
    return MUCA_OK;
}

void mucaDestroy(muca_ctx ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto &pr : ctx->timing) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->pin_H) (void)hipHostFree(ctx->pin_H);
    if (ctx->pin_tab) (void)hipHostFree(ctx->pin_tab);
    delete ctx;
}

const char *mucaLastError(muca_ctx ctx) {
    if (!ctx) return g_init_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"
