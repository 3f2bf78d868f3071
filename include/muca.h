/*
 * muca.h -- C ABI of the MI355X multicanonical (MUCA) sampling library.
 *
 * The method (Zierenberg, Marenz, Janke, "Scaling properties of a parallel
 * implementation of the multicanonical algorithm"):
 *   - Sec. 2, Eq. (1): sample with weights W(E) instead of exp(-beta E); with
 *     W = 1/Omega the energy histogram is flat;
 *   - Sec. 2: the weights are found iteratively, W <- W / H, kept in logs;
 *   - Sec. 2, the parallel version: p independent chains share W, each fills its
 *     own histogram H_i, the histograms are summed, the new W is sent back;
 *   - Sec. 3, Eqs. (3)-(4): 2D Ising and q-state Potts models on an L x L
 *     periodic square lattice, sweeps of V = L^2 single-spin updates, a start
 *     at infinite temperature, updates only where H > 0;
 *   - Sec. 2, Eq. (2): time-series reweighting of production data.
 *
 * Conventions of this library (fixed where the paper is silent):
 *   - N = L*L.  Energies are binned by k = number of unsatisfied bonds,
 *     k = 0..2N, so there are 2N+1 bins; Ising E = -2N + 2k, Potts E = -2N + k.
 *   - Random numbers: Philox4x32-10, key = (seed & 0xffffffff, seed >> 32),
 *     counter = (site block, sweep, chain, stream).  Init draws word 0 of
 *     counter (site, 0, chain, 1).  Sweep s, site i: Ising uses word (i & 3)
 *     of counter (i >> 2, s, chain, 0); Potts uses words 2(i&1) (proposal)
 *     and 2(i&1)+1 (acceptance) of counter (i >> 1, s, chain, 0).
 *   - Sites are updated in order i = y*L + x, x fastest.  The Potts proposal
 *     is s' = (s + 1 + ((r * (q-1)) >> 32)) mod q (uniform over the q-1 other
 *     states).  A move with change dk is accepted iff T[k][dk] == 0xffffffff
 *     or u < T[k][dk], where T[k][dk] = floor(2^32 min(1, exp(lnW[k+dk] -
 *     lnW[k]))) and values >= 2^32 - 1 are stored as 0xffffffff.
 *   - Every chain adds one count to its histogram at the end of each
 *     recorded sweep.  The recursion is lnW[k] -= log(H[k]) where H[k] > 0,
 *     with no renormalisation.  The host evaluates log/exp with the C library
 *     in IEEE double, so histograms, weights and tables are reproducible bit
 *     for bit by any implementation of the same definitions.
 *
 * Errors: every call returns a muca_status; nothing throws across the ABI.
 * MUCA_EINVAL for bad arguments, MUCA_ENOMEM for a workspace that is too
 * small, MUCA_EHIP for a failed HIP call (text in mucaLastError), MUCA_ESTATE
 * for a call in the wrong state.  A context is not thread-safe.
 */
#ifndef MUCA_H_
#define MUCA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct muca_ctx_s *muca_ctx;

typedef enum {
    MUCA_OK = 0,
    MUCA_EINVAL = -1,
    MUCA_ENOMEM = -2,
    MUCA_EHIP = -3,
    MUCA_ESTATE = -4
} muca_status;

enum { MUCA_ISING = 0, MUCA_POTTS = 1, MUCA_ISING_MAG = 2 };
enum { MUCA_REC_NONE = 0, MUCA_REC_MUCA = 1, MUCA_REC_PROD = 2 };

/* One problem: a model on one lattice with n_chains chains sharing lnW.
 * Ising: L even, 4 <= L <= 256, q ignored.  Potts: 3 <= L <= 256, 3 <= q <= 8.
 * 1 <= n_chains <= 1<<20.  seed keys the generator (Sec. 2: same weights,
 * different random numbers per chain).
 *
 * MUCA_ISING_MAG is the multimagnetic Ising ensemble of Sec. 4: the Ising
 * lattice (same L rules, same random numbers and sweep order) sampled with
 * exp(-beta E) W(M), the weights over the magnetization M at the fixed inverse
 * temperature beta (0 <= beta <= 10; ignored by the other models).  Its bins
 * are m = number of up spins = (M + N) / 2, m = 0..N (N+1 bins, all
 * reachable), where the energy models use k = 0..2N.  A flip that changes k by
 * dk and m by dm is accepted with probability
 * min(1, exp((lnW[m+dm] - lnW[m]) - beta * 2 dk)), through the same integer
 * threshold rule as below (delta evaluated in that order, in IEEE double). */
typedef struct {
    int32_t model;
    int32_t q;
    int32_t L;
    int32_t n_chains;
    uint64_t seed;
    double beta;
} muca_problem;

/* Launch and iteration options; zero means "default / autotune".
 *   chains_per_wg    chains handled by one workgroup, 1..64 (0 = tune: 16,
 *                    32, 64 and the most chains, up to 64, whose lattice and
 *                    table both fit in LDS); a count whose arrays do not fit
 *                    in the requested placement makes mucaInit fail
 *   rng_mode         0 = tune, 1 = walker draws its own numbers,
 *                    2, 3, 4, 5 = one, two, three or four helper waves of the
 *                    workgroup draw them (and, for the fast walkers, form
 *                    the lattice terms the walker's updates cannot change)
 *   spin_placement   0 = tune, 1 = lattice in LDS, 2 = lattice in HBM
 *   table_placement  0 = tune, 1 = table in LDS, 2 = table in HBM
 *   use_graph        1 = mucaIterate replays one HIP graph per iteration
 *   production       1 = reserve production accumulators (|M| sums)
 *   flat_ratio       min/max threshold of the flatness test (default 0.5)
 *   flat_rule        0 = all reachable bins visited and min/max >= flat_ratio;
 *                    1 = all reachable bins visited and every entry within
 *                        [avg/2, 2 avg] (the rule of Sec. 3)
 *   tune_sweeps      sweeps per timed candidate when tuning (default 4)
 *   correction       1 = after each recursion, continue lnW linearly beyond
 *                    the sampled region [k_lo, k_hi] (bins with H > 0): below
 *                    k_lo with the slope between k_lo and the reachable bin L
 *                    reachable bins inward (or the far edge if the region is
 *                    narrower), likewise above k_hi (the correction function
 *                    of Sec. 3)
 *   update_norm      1 = the recursion's update over the visited bins is
 *                    shifted to zero mean: lnW(k) -= ln H(k) - <ln H> for
 *                    H(k) > 0, <ln H> the mean over those bins (a reading of
 *                    Sec. 2: dividing W by H fixes W only up to one constant
 *                    per iteration, since H may be normalized in any way; this
 *                    chooses the constant that keeps the visited region's mean
 *                    weight against the unvisited bins).  0 = raw counts
 *   wait_polls       polls of the bounded waits between a streamed walker
 *                    and its helper waves before they give up (0 = default,
 *                    2^24, a second or more; negative = none, so that every
 *                    wait gives up at once: a test of that path, after which
 *                    mucaMergeUpdate, mucaIterate, mucaGet and mucaCheckpoint
 *                    report MUCA_EHIP).  Not a step of the method. */
typedef struct {
    int32_t chains_per_wg;
    int32_t rng_mode;
    int32_t spin_placement;
    int32_t table_placement;
    int32_t use_graph;
    int32_t production;
    double flat_ratio;
    int32_t flat_rule;
    int32_t tune_sweeps;
    int32_t correction;
    int32_t wait_polls;
    int32_t update_norm;
    int32_t pad;
} muca_options;

/* Statistics of one weight iteration for one problem, from the merged
 * histogram H of that iteration (before the recursion is applied). */
typedef struct {
    int32_t k_lo, k_hi;       /* smallest / largest k with H > 0 */
    int32_t visited;          /* bins with H > 0 */
    int32_t reachable;        /* bins that can occur at all */
    int32_t covered;          /* every reachable bin has H > 0 */
    int32_t flat;             /* covered and the flatness rule holds */
    double min_over_max, min_over_avg, max_over_avg;  /* over reachable bins */
    int64_t total;            /* sum of H = chains * recorded sweeps */
} muca_iter_stats;

/* Selected launch configuration of one problem (after tuning). */
typedef struct {
    int32_t chains_per_wg, rng_mode, spin_placement, table_placement;
    int32_t lds_bytes, n_workgroups;
    int32_t fast_walker;   /* 1: a four-sites-per-step walker (Ising, multimagnetic or 8-Potts) runs it */
    int32_t walker;        /* walker of the problem's first work item: 0 generic, 1 byte-wise Ising or
                              multimagnetic, 2 packed Ising, 3 packed Ising on the compact table,
                              4 8-Potts, 5 8-Potts on the compact table, 6 streamed Ising,
                              7 streamed 8-Potts on the compact table, 8 streamed Ising on
                              the compact table, 9 streamed Ising on bit lattices (L = 64,
                              more than 16 chains per workgroup) */
} muca_launch_info;

/* Bytes of device workspace that mucaInit needs for these problems.  (Not a
 * step of the method: memory planning of this library.) */
muca_status mucaWorkspaceSize(const muca_problem *problems, int32_t n_problems,
                              const muca_options *opts, size_t *bytes);

/* Creates a context.  d_workspace: device memory of at least the size from
 * mucaWorkspaceSize, owned by the caller, must outlive the context.
 * hip_stream: the hipStream_t every call enqueues on (NULL = default stream).
 * Draws the initial spins (Sec. 3, infinite temperature), computes k and M,
 * sets lnW = 0, builds the tables and, if asked, tunes the launch. */
muca_status mucaInit(muca_ctx *out, const muca_problem *problems, int32_t n_problems,
                     const muca_options *opts, void *d_workspace, size_t ws_bytes,
                     void *hip_stream);

/* Replaces lnW of problem prob (n_bins = 2N+1 host doubles, copied) and
 * rebuilds its table: installs the weights W(E) of Eq. (1) directly, for
 * example a canonical exp(-beta E) or an estimate of 1/Omega that starts the
 * recursion of Sec. 2 elsewhere than at W = 1.  MUCA_EINVAL for a wrong n_bins
 * or a value that is not finite.  Synchronises. */
muca_status mucaSetLogWeights(muca_ctx ctx, int32_t prob, const double *lnW, int32_t n_bins);

/* Runs n_sweeps sweeps of every chain of every problem (Sec. 3), asynchronously
 * on the stream.  record: MUCA_REC_NONE (thermalisation), MUCA_REC_MUCA
 * (one histogram count per chain per sweep), MUCA_REC_PROD (count and |M|
 * per chain per sweep).  One call is one kernel launch, whose walkers count
 * its chunks of sites in 32 bits: MUCA_EINVAL, before anything is enqueued,
 * for n_sweeps > 2^30 or more sweeps than (2^31 - 1) / (chunks per sweep)
 * (chunks of 32 to 72 sites; for example 2^25 - 1 sweeps at Ising L = 64 with
 * the byte walker); MUCA_ESTATE if the 32-bit sweep counter would wrap. */
muca_status mucaSweep(muca_ctx ctx, int64_t n_sweeps, int32_t record);

/* Bins: "k" below stands for the problem's bin index (m for MUCA_ISING_MAG).
 *
 * Merges the per-chain histograms (H = sum_i H_i, Sec. 2) and clears them.
 * update = 1 also applies lnW <- lnW - ln H where H > 0 and rebuilds the
 * tables.  Writes one muca_iter_stats per problem to out (may be NULL).
 * Synchronises the stream. */
muca_status mucaMergeUpdate(muca_ctx ctx, int32_t update, muca_iter_stats *out);

/* One weight iteration: n_sweeps recorded sweeps, merge, recursion, new
 * tables (Fig. 1's loop body).  With use_graph the whole iteration is one
 * HIP graph launch.  Synchronises the stream; out as in mucaMergeUpdate.
 * n_sweeps is limited as in mucaSweep. */
muca_status mucaIterate(muca_ctx ctx, int64_t n_sweeps, muca_iter_stats *out);

/* Time-series reweighting, Eq. (2), of the production data of problem prob
 * (accumulated by MUCA_REC_PROD sweeps since the last mucaClearProduction)
 * to n_betas inverse temperatures.  Outputs (host arrays of n_betas doubles,
 * caller-owned): <E>/N, C_V = beta^2 (<E^2> - <E>^2)/N and <|M|>/N (Ising;
 * NaN for Potts).  Runs on the device in double precision; synchronises.
 * MUCA_EINVAL for a MUCA_ISING_MAG problem (its weights are not over E). */
muca_status mucaReweight(muca_ctx ctx, int32_t prob, const double *betas, int32_t n_betas,
                         double *e_per_site, double *c_v, double *abs_m_per_site);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * reweighting of mucaReweight on caller-held production data, with no
 * context and no allocation.  Its device staging (counts, |M| sums, lnW,
 * betas, outputs) lives in one static device array of 3,277,568 bytes per
 * GPU, kept until the process ends; the call allocates nothing.
 *   model, L     MUCA_ISING (even L, 4..256) or MUCA_POTTS (3..256)
 *   lnW, cnt     host arrays of n_bins = 2N+1 (log-weights of the production
 *                run, finite; merged counts, >= 0, not all 0)
 *   sabs         host int64[n_bins] of merged |M| sums (Ising; ignored and
 *                may be NULL for Potts)
 *   betas        host double[n_betas], 1 <= n_betas <= 4096
 *   outputs      host double[n_betas] each, as mucaReweight
 *   hip_stream   the stream to run on (NULL = default stream)
 * Results equal mucaReweight's on the same data bit for bit (same kernel).
 * Synchronises the stream.  Calls on one GPU share its static array: calls
 * that overlap in time on one GPU (other threads or streams) race; calls one
 * after the other do not, since each call writes every entry it reads.
 * MUCA_EINVAL for bad arguments or sizes beyond the maximum, MUCA_ESTATE for
 * all-zero counts, MUCA_EHIP for a failed HIP call; text in
 * mucaLastError(NULL). */
muca_status mucaReweightStatic(int32_t model, int32_t L, const double *lnW, const int64_t *cnt, const int64_t *sabs,
                               int32_t n_bins, const double *betas, int32_t n_betas, double *e_per_site,
                               double *c_v, double *abs_m_per_site, void *hip_stream);

/* Zeroes the per-chain production accumulators of every problem: starts a
 * new set of production measurements for Eq. (2) (Sec. 3 thermalises again
 * before production; the caller runs MUCA_REC_NONE sweeps for that).
 * Synchronises. */
muca_status mucaClearProduction(muca_ctx ctx);

/* Order-disorder interface tension from a reweighted energy histogram
 * (Sec. 5, Eq. 9): find the inverse temperature beta_eqh at which the
 * histogram reweighted to the canonical ensemble has its two peaks at the
 * same height, and return sigma_od = ln(P_max / P_min) / (2L) there.
 *
 * At beta, bin k with cnt[k] > 0 carries a_k = ln cnt[k] - lnW[k] - beta E_k
 * (E_k as in the conventions above; the log of the canonical probability up
 * to a constant; bins with cnt[k] = 0 are left out).  The peaks are split at
 * the histogram's valley, a bin fixed for the whole search: over 65 equally
 * spaced beta in [beta_lo, beta_hi], each bin scores its depth below the
 * lower of the highest a on its two sides less |ln(M_left / M_right)| (M the
 * sum of e^{a} on each side, the bin on both), and the split is the best bin
 * at the beta with the highest score.  Peaks: the maxima of a over k <= split
 * (ordered) and over k > split (disordered); minimum: the smallest a_k between
 * them (first index on ties).  beta_eqh is found by bisection of
 * a(ordered peak) - a(disordered peak), which grows with beta and must be < 0
 * at beta_lo and > 0 at beta_hi; ln(P_max/P_min) uses the mean of the two
 * peak heights.  Host computation in IEEE double with the C library's
 * log/exp.
 *
 *   model, L     MUCA_ISING or MUCA_POTTS and the lattice side; n_bins = 2N+1
 *   lnW, cnt     host arrays of n_bins (log-weights of the production run and
 *                its merged counts), caller-owned
 *   beta_eqh, sigma_od  outputs
 *   k_peaks      int32[3] or NULL: ordered peak, minimum, disordered peak bins
 *   lnP          double[n_bins] or NULL: the normalised log-probabilities at
 *                beta_eqh (-HUGE_VAL where cnt = 0)
 * Returns MUCA_EINVAL for bad arguments and MUCA_ESTATE when the histogram has
 * no two peaks (no bin of any beta in the bracket scores above zero, or at
 * beta_eqh no bin lies strictly between the peaks) or their heights do not
 * cross inside [beta_lo, beta_hi].
 * Needs no GPU and no context (errors: mucaLastError(NULL)). */
muca_status mucaEqualHeight(int32_t model, int32_t L, const double *lnW, const int64_t *cnt, int32_t n_bins,
                            double beta_lo, double beta_hi, double *beta_eqh, double *sigma_od, int32_t *k_peaks,
                            double *lnP);

/* mucaEqualHeight applied to problem prob's production data (merged counts of
 * the MUCA_REC_PROD sweeps since the last mucaClearProduction) and its current
 * log-weights.  MUCA_ESTATE without production data.  Synchronises. */
muca_status mucaInterfaceTension(muca_ctx ctx, int32_t prob, double beta_lo, double beta_hi, double *beta_eqh,
                                 double *sigma_od, int32_t *k_peaks, double *lnP);

/* Copies state of problem prob to host memory (bytes must match exactly).
 * Inspection of the sampler's state; not a step of the method.  MUCA_EINVAL
 * for an unknown item or a byte count that differs from the item's size:
 *   MUCA_GET_H        int64[2N+1]      merged histogram of the last merge
 *   MUCA_GET_LNW      double[2N+1]     current log-weights
 *   MUCA_GET_T        the acceptance table as the walkers read it, copied
 *                     back from device memory (entries as in the conventions;
 *                     targets outside the bin range hold 0):
 *                       Ising uint32[N+1][5], row k/2, column dk/2 + 2
 *                       (dk = -4..4 in steps of 2; odd k never occurs)
 *                       Potts uint32[2N+1][9], row k, column dk + 4
 *   MUCA_GET_SPINS    uint8[N][C]      spins, site-major, chain fastest
 *                                      (Ising 0/1 for s = -1/+1, Potts 0..q-1)
 *   MUCA_GET_K        int32[C]         unsatisfied bonds per chain
 *   MUCA_GET_M        int32[C]         Ising magnetisation per chain (0 Potts)
 *   MUCA_GET_CHAIN_H  int32[2N+1][C]   per-chain histograms (not yet merged)
 *   MUCA_GET_PROD_CNT int64[2N+1]      merged production counts
 *   MUCA_GET_PROD_ABSM int64[2N+1]     merged production |M| sums
 *   MUCA_GET_SWEEP    uint32[1]        sweeps done since init
 *   MUCA_GET_REACH    uint8[2N+1]      reachable-bin mask
 * For MUCA_ISING_MAG every per-bin item has N+1 bins (m = 0..N), T is
 * uint32[N+1][10], row m, column j + 5u (u = 1 when the spin to flip is up, so
 * that m' = m - 1, else m' = m + 1; the flip changes k by dk = 2j - 4), and
 * MUCA_GET_PROD_ABSM holds the sums of k (unsatisfied bonds) per m.
 * Synchronises the stream. */
enum {
    MUCA_GET_H = 0, MUCA_GET_LNW = 1, MUCA_GET_T = 2, MUCA_GET_SPINS = 3, MUCA_GET_K = 4,
    MUCA_GET_M = 5, MUCA_GET_CHAIN_H = 6, MUCA_GET_PROD_CNT = 7, MUCA_GET_PROD_ABSM = 8,
    MUCA_GET_SWEEP = 9, MUCA_GET_REACH = 10
};
muca_status mucaGet(muca_ctx ctx, int32_t what, int32_t prob, void *host_dst, size_t bytes);

/* Launch configuration chosen for problem prob (by this library's tuner; not
 * in the paper). */
muca_status mucaLaunchInfo(muca_ctx ctx, int32_t prob, muca_launch_info *info);

/* Average duration in milliseconds of the sweep-kernel launches enqueued by
 * mucaSweep / mucaIterate since the last call (HIP events on the context's
 * stream), and how many launches it covers.  Synchronises.  (Measurement of
 * this library; not in the paper.) */
muca_status mucaSweepTiming(muca_ctx ctx, double *avg_ms, int32_t *n_launches);

/* Checkpoint of the whole sampling state (spins, k, M, sweep counter, lnW,
 * per-chain histograms) into a caller-owned host buffer (resuming a run is not
 * a step of the method; the paper does not describe one).  With blob == NULL
 * only *bytes is set.  mucaRestore loads such a blob into a context created
 * with the same problems; the continued run equals an uninterrupted one bit
 * for bit.  Both synchronise.  Errors: MUCA_EINVAL for a buffer too small, a
 * blob of another size or context, a spin outside 0..q-1 or a log-weight that
 * is not finite, all found before any state changes (k and M are recomputed
 * from the spins, not read). */
muca_status mucaCheckpoint(muca_ctx ctx, void *blob, size_t *bytes);
muca_status mucaRestore(muca_ctx ctx, const void *blob, size_t bytes);

/* The problem definition of index prob (as validated, q = 2 for Ising).  Not
 * a step of the method. */
muca_status mucaProblemInfo(muca_ctx ctx, int32_t prob, muca_problem *out);

/* ---------------------------------------------------------------------
 * Learned initial weights.  An MLP 4 -> 64 -> 64 -> 64 -> 1 with tanh-form
 * GELU maps (Ising one-hot, Potts one-hot, 8/L, E/N) to ln Omega(E)/N.  Its
 * weights are BF16 in the matrix products with FP32 accumulation; FP32
 * master weights are updated by Adam (full batch, MSE loss).  Training data
 * come from weights the recursion converged to at small L: with a flat
 * histogram W = 1/Omega up to a constant (Sec. 2), fixed here by
 * sum_E Omega(E) = q^N.  The prediction seeds lnW = -N f(...) at larger L;
 * the recursion then continues from there.
 * --------------------------------------------------------------------- */
typedef struct muca_mlp_s *muca_mlp;

/* Workspace bytes for up to max_samples training samples (1..2^22). */
muca_status mucaMlpWorkspaceSize(int32_t max_samples, size_t *bytes);
/* Creates the network with seeded uniform(+-1/sqrt(fan_in)) weights.  The
 * workspace (caller-owned device memory, 256-byte aligned) must outlive it. */
muca_status mucaMlpCreate(muca_mlp *out, int32_t max_samples, uint64_t seed, void *d_workspace, size_t ws_bytes,
                          void *hip_stream);
/* FP32 master parameters (8705 floats: W1[64][4], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], W4[64], b4); setting them also resets Adam. */
muca_status mucaMlpSetParams(muca_mlp m, const float *params);
muca_status mucaMlpGetParams(muca_mlp m, float *params);
/* Training set: raw (x[n][4], y[n]) pairs, or every reachable bin of a
 * problem's current weights (features as above, target ln Omega / N). */
muca_status mucaMlpClearData(muca_mlp m);
muca_status mucaMlpAddData(muca_mlp m, const float *x, const float *y, int32_t n);
muca_status mucaMlpAddWeights(muca_mlp m, muca_ctx ctx, int32_t prob);
muca_status mucaMlpNumSamples(muca_mlp m, int32_t *n);
/* steps full-batch Adam steps (beta 0.9/0.999, eps 1e-8) at rate lr;
 * loss_out (host, steps floats, may be NULL) gets each step's MSE. */
muca_status mucaMlpTrain(muca_mlp m, int32_t steps, float lr, float *loss_out);
/* Gradient of the MSE on the training set at the current parameters
 * (8705 floats) and the loss, without updating anything. */
muca_status mucaMlpGradients(muca_mlp m, float *grad, float *loss);
/* Predictions for n inputs x[n][4] into y[n] (host arrays). */
muca_status mucaMlpPredict(muca_mlp m, const float *x, int32_t n, float *y);
/* Installs lnW[k] = -N f(model, 8/L, E_k/N) on the reachable bins of
 * problem prob (0 elsewhere) through mucaSetLogWeights. */
muca_status mucaMlpSetLogWeights(muca_mlp m, muca_ctx ctx, int32_t prob);
void mucaMlpDestroy(muca_mlp m);
const char *mucaMlpLastError(muca_mlp m);

/* Frees the context (not the workspace).  Safe on NULL.  Not a step of the
 * method. */
void mucaDestroy(muca_ctx ctx);

/* Last error text of ctx (or of the last failed mucaInit when ctx is NULL). */
const char *mucaLastError(muca_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* MUCA_H_ */
