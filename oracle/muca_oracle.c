/*
 * CPU oracle for parallel multicanonical (MUCA) sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * reads this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP library.
 *
 * What it computes, step by step, in plain loops:
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the
 *     published round function and key schedule;
 *   - the 2D periodic Ising model, Eq. (3), and the q-state Potts model,
 *     Eq. (4), with J = 1 and nearest neighbours on an L x L square lattice;
 *   - a start at infinite temperature (random spins, Sec. 3);
 *   - sequential single-spin Metropolis sweeps of V = L*L updates (Sec. 3)
 *     under multicanonical weights W(E) = exp(lnW), Eq. (1);
 *   - one energy histogram per chain, merged by summation (Sec. 2, parallel
 *     version: H = sum_i H_i);
 *   - the recursion W <- W / H kept in logarithms (Sec. 2), applied only to
 *     bins with a non-zero histogram entry (Sec. 3);
 *   - production accumulators for time-series reweighting, Eq. (2);
 *   - the multimagnetic Ising ensemble of Sec. 4 (weights over the
 *     magnetization at a fixed inverse temperature beta): the same sweeps
 *     with acceptance min(1, exp(-beta dE) W(M') / W(M)).
 *
 * Conventions fixed where the paper is silent:
 *   - energies are binned by k, the number of unsatisfied bonds, 0..2N
 *     (Ising E = -2N + 2k, Potts E = -2N + k);
 *   - the generator counter is (site block, sweep, chain, stream), the key is
 *     the 64-bit seed split into two 32-bit words;
 *   - acceptance compares a raw 32-bit draw u with the threshold
 *     T[k][dk] = floor(2^32 * min(1, exp(lnW[k+dk] - lnW[k]))), where the value
 *     0xFFFFFFFF means "always accept";
 *   - histograms are filled once per completed sweep.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off (no FMA contraction), so
 * that log/exp are glibc's and every double operation is rounded once.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { MODEL_ISING = 0, MODEL_POTTS = 1, MODEL_ISING_MAG = 2 };
enum { REC_NONE = 0, REC_MUCA = 1, REC_PROD = 2 };
enum { STREAM_SWEEP = 0, STREAM_INIT = 1 };

#define TCOLS 9 /* threshold-table columns: dk = -4..4, column dk + 4 */
/* Multimagnetic table: row m = number of up spins (M = 2m - N), column
 * j + 5u, where u = 1 if the spin to flip is up, j = 4 - (disagreeing
 * neighbours), so that the flip changes k by dk = 2j - 4 and m by -1 (up) or
 * +1 (down). */
#define TCOLS_MAG 10

/* ---------------------------------------------------------------------- */
/* Philox4x32-10                                                            */
/* ---------------------------------------------------------------------- */

/* One Philox round: two 32x32->64 products, the high halves xored with the
 * other two counter words and the key, the low halves passed through. */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k);
        /* Weyl key schedule: golden ratio and sqrt(3)-1 constants */
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static void draw_block(uint64_t seed, uint32_t c0, uint32_t sweep, uint32_t chain,
                       uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, sweep, chain, stream};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* ---------------------------------------------------------------------- */
/* Lattice helpers                                                          */
/* ---------------------------------------------------------------------- */

/* The four nearest neighbours of site i = y*L + x on the periodic lattice. */
static void neighbours(int L, int i, int nb[4])
{
    int x = i % L, y = i / L;
    nb[0] = y * L + (x + 1) % L;       /* right */
    nb[1] = y * L + (x + L - 1) % L;   /* left  */
    nb[2] = ((y + 1) % L) * L + x;     /* down  */
    nb[3] = ((y + L - 1) % L) * L + x; /* up    */
}

/* Ising spin value s = +1 for stored 1, -1 for stored 0. */
static int ising_value(uint8_t b) { return b ? 1 : -1; }

/* k = number of unsatisfied bonds (s_i != s_j) over the 2N bonds; for Ising
 * also the magnetization M = sum_i s_i. Counts each bond once (right, down). */
void orc_energy(int model, int L, const uint8_t *s, int32_t *k_out, int32_t *m_out)
{
    int N = L * L, k = 0, m = 0;
    for (int i = 0; i < N; ++i) {
        int nb[4];
        neighbours(L, i, nb);
        if (s[i] != s[nb[0]]) ++k;
        if (s[i] != s[nb[2]]) ++k;
        if (model != MODEL_POTTS) m += ising_value(s[i]);
    }
    *k_out = k;
    *m_out = m;
}

/* ---------------------------------------------------------------------- */
/* Reachable bins                                                           */
/* ---------------------------------------------------------------------- */

/* Which k can occur.  Ising (even L): every cut of the 4-regular torus is
 * even; a single flip breaks 4 bonds so k = 2 is impossible, and flipping one
 * sublattice maps k to 2N - k, so 2N - 2 is impossible too.  Potts (q >= 3,
 * L >= 3): a colour class that is neither empty nor everything has at least 4
 * boundary bonds, two classes give even k, three or more give k >= 6; so
 * k in {1, 2, 3, 5} cannot occur. */
void orc_reachable(int model, int q, int L, uint8_t *mask)
{
    int N = L * L;
    (void)q;
    if (model == MODEL_ISING_MAG) {
        /* bins m = 0..N: any number of up spins occurs */
        for (int m = 0; m <= N; ++m) mask[m] = 1;
        return;
    }
    for (int k = 0; k <= 2 * N; ++k) {
        int r;
        if (model == MODEL_ISING)
            r = (k % 2 == 0) && k != 2 && k != 2 * N - 2;
        else
            r = !(k == 1 || k == 2 || k == 3 || k == 5);
        mask[k] = (uint8_t)r;
    }
}

/* ---------------------------------------------------------------------- */
/* Brute-force density of states                                           */
/* ---------------------------------------------------------------------- */

/* Enumerates all q^N configurations (q = 2 for Ising) and counts, per k, the
 * configurations (omega) and, for Ising, the sum of |M| (sum_abs_m). */
void orc_bruteforce(int model, int q, int L, int64_t *omega, int64_t *sum_abs_m)
{
    int N = L * L, nbins = 2 * N + 1;
    int qq = (model == MODEL_ISING) ? 2 : q;
    uint8_t s[64];
    memset(s, 0, sizeof(s));
    for (int b = 0; b < nbins; ++b) { omega[b] = 0; sum_abs_m[b] = 0; }
    for (;;) {
        int32_t k, m;
        orc_energy(model, L, s, &k, &m);
        omega[k] += 1;
        sum_abs_m[k] += (m < 0) ? -m : m;
        /* odometer increment in base qq */
        int i = 0;
        while (i < N) {
            if (++s[i] < qq) break;
            s[i] = 0;
            ++i;
        }
        if (i == N) break;
    }
}

/* Canonical averages at inverse temperature beta by summing over every state:
 * <E>, <E^2>, <|M|> with E from Eq. (3) (Ising) or Eq. (4) (Potts). */
void orc_bruteforce_canonical(int model, int q, int L, double beta,
                              double *e_mean, double *e2_mean, double *absm_mean)
{
    int N = L * L;
    int qq = (model == MODEL_ISING) ? 2 : q;
    uint8_t s[64];
    memset(s, 0, sizeof(s));
    /* ground-state energy shift keeps the Boltzmann factors <= 1 */
    double e_ground = -2.0 * N;
    double z = 0, se = 0, se2 = 0, sm = 0;
    for (;;) {
        int32_t k, m;
        orc_energy(model, L, s, &k, &m);
        double E = (model == MODEL_ISING) ? (-2.0 * N + 2.0 * k) : (-2.0 * N + k);
        double w = exp(-beta * (E - e_ground));
        z += w;
        se += w * E;
        se2 += w * E * E;
        sm += w * (double)((m < 0) ? -m : m);
        int i = 0;
        while (i < N) {
            if (++s[i] < qq) break;
            s[i] = 0;
            ++i;
        }
        if (i == N) break;
    }
    *e_mean = se / z;
    *e2_mean = se2 / z;
    *absm_mean = sm / z;
}

/* Exact canonical distribution of the Ising magnetization at beta: for every
 * m = number of up spins, p_m = sum over states with m up spins of
 * exp(-beta E) / Z, and e_m = the mean of k over those states (weighted the
 * same way).  By enumeration of all 2^N states. */
void orc_bruteforce_mag(int L, double beta, double *p_m, double *k_mean)
{
    int N = L * L;
    uint8_t s[64];
    memset(s, 0, sizeof(s));
    double e_ground = -2.0 * N, z = 0;
    for (int b = 0; b <= N; ++b) { p_m[b] = 0; k_mean[b] = 0; }
    for (;;) {
        int32_t k, m;
        orc_energy(MODEL_ISING, L, s, &k, &m);
        double w = exp(-beta * ((-2.0 * N + 2.0 * k) - e_ground));
        z += w;
        p_m[(m + N) / 2] += w;
        k_mean[(m + N) / 2] += w * (double)k;
        int i = 0;
        while (i < N) {
            if (++s[i] < 2) break;
            s[i] = 0;
            ++i;
        }
        if (i == N) break;
    }
    for (int b = 0; b <= N; ++b) {
        if (p_m[b] > 0) k_mean[b] /= p_m[b];
        p_m[b] /= z;
    }
}

/* ---------------------------------------------------------------------- */
/* Initial state: infinite temperature                                     */
/* ---------------------------------------------------------------------- */

/* Random spins (beta = 0 start, Sec. 3).  Site i of chain c draws word 0 of
 * the block at counter (i, 0, c, STREAM_INIT).  Ising stores the top bit;
 * Potts maps the word to 0..q-1 by (w * q) >> 32.
 * Chains chain0 .. chain0 + n_chains - 1; spins: [n_chains][N] bytes. */
void orc_init(int model, int q, int L, int chain0, int n_chains, uint64_t seed,
              uint8_t *spins, int32_t *k, int32_t *m)
{
    int N = L * L;
    for (int c = 0; c < n_chains; ++c) {
        uint8_t *s = spins + (size_t)c * N;
        for (int i = 0; i < N; ++i) {
            uint32_t blk[4];
            draw_block(seed, (uint32_t)i, 0u, (uint32_t)(chain0 + c), STREAM_INIT, blk);
            if (model != MODEL_POTTS)
                s[i] = (uint8_t)(blk[0] >> 31);
            else
                s[i] = (uint8_t)(((uint64_t)blk[0] * (uint64_t)q) >> 32);
        }
        orc_energy(model, L, s, &k[c], &m[c]);
    }
}

/* ---------------------------------------------------------------------- */
/* Threshold table                                                          */
/* ---------------------------------------------------------------------- */

/* T[k][dk+4] = floor(2^32 * min(1, exp(lnW[k+dk] - lnW[k]))) for 0 <= k+dk <= 2N;
 * cells whose target lies outside the range are 0 (never used).  A value that
 * would reach 2^32 - 1 or more is stored as 0xFFFFFFFF, read as "always". */
static uint32_t threshold_of(double delta)
{
    if (delta >= 0.0) return 0xFFFFFFFFu;
    double x = ldexp(exp(delta), 32);
    return (x >= 4294967295.0) ? 0xFFFFFFFFu : (uint32_t)floor(x);
}

void orc_build_table(int n_bins, const double *lnW, uint32_t *T)
{
    for (int k = 0; k < n_bins; ++k) {
        for (int dk = -4; dk <= 4; ++dk) {
            int t = k + dk;
            uint32_t v = 0;
            if (t >= 0 && t < n_bins) v = threshold_of(lnW[t] - lnW[k]);
            T[(size_t)k * TCOLS + (dk + 4)] = v;
        }
    }
}

/* Multimagnetic table (layout above): the move from m to m' = m -+ 1 that
 * changes the energy by dE = 2 dk (E = -2N + 2k) is accepted with probability
 * min(1, exp(-beta dE) W(m') / W(m)); in logarithms
 * delta = (lnW[m'] - lnW[m]) - beta * dE.  Targets outside 0..N are 0. */
void orc_build_table_mag(int L, double beta, const double *lnW, uint32_t *T)
{
    int N = L * L;
    for (int m = 0; m <= N; ++m) {
        for (int u = 0; u < 2; ++u) {
            int t = u ? m - 1 : m + 1;
            for (int j = 0; j < 5; ++j) {
                int dk = 2 * j - 4;
                uint32_t v = 0;
                if (t >= 0 && t <= N) v = threshold_of((lnW[t] - lnW[m]) - beta * (double)(2 * dk));
                T[(size_t)m * TCOLS_MAG + j + 5 * u] = v;
            }
        }
    }
}

static int accept(uint32_t u, uint32_t t) { return t == 0xFFFFFFFFu || u < t; }

/* ---------------------------------------------------------------------- */
/* Sweeps                                                                   */
/* ---------------------------------------------------------------------- */

typedef struct {
    int model, q, L, n_bins;
    int chain0;              /* generator index of local chain 0 */
    int c_begin, c_end;
    uint64_t seed;
    uint32_t sweep0;
    int n_sweeps, record;
    const uint32_t *T;
    uint8_t *spins;
    int32_t *k, *m;
    int32_t *hist;    /* [n_chains][n_bins] */
    int64_t *sabs;    /* [n_chains][n_bins], production only */
} sweep_job;

/* One chain, one sequential sweep over sites 0..N-1 (x fastest). */
static void sweep_one_chain(const sweep_job *j, int c, uint32_t sweep)
{
    int L = j->L, N = L * L;
    uint8_t *s = j->spins + (size_t)c * N;
    int32_t k = j->k[c], m = j->m[c];
    uint32_t blk[4] = {0, 0, 0, 0};
    for (int i = 0; i < N; ++i) {
        int nb[4];
        neighbours(L, i, nb);
        int before = 0, after = 0;
        uint8_t s_new;
        uint32_t u;
        if (j->model != MODEL_POTTS) {
            /* four sites share one block: site i uses word i mod 4 */
            if ((i & 3) == 0) draw_block(j->seed, (uint32_t)(i >> 2), sweep, (uint32_t)(j->chain0 + c), STREAM_SWEEP, blk);
            u = blk[i & 3];
            s_new = (uint8_t)(s[i] ^ 1u);
        } else {
            /* two sites share one block: site i uses words 2(i mod 2), 2(i mod 2)+1 */
            if ((i & 1) == 0) draw_block(j->seed, (uint32_t)(i >> 1), sweep, (uint32_t)(j->chain0 + c), STREAM_SWEEP, blk);
            uint32_t r = blk[2 * (i & 1)];
            u = blk[2 * (i & 1) + 1];
            /* new state uniform over the q-1 others: offset 1 + floor(r (q-1) / 2^32) */
            uint32_t t = (uint32_t)(((uint64_t)r * (uint64_t)(j->q - 1)) >> 32);
            s_new = (uint8_t)((s[i] + 1u + t) % (uint32_t)j->q);
        }
        for (int n = 0; n < 4; ++n) {
            if (s[nb[n]] != s[i]) ++before;
            if (s[nb[n]] != s_new) ++after;
        }
        int dk = after - before;
        uint32_t tv;
        if (j->model == MODEL_ISING_MAG) {
            /* row: up spins (m + N) / 2; column by dk and the spin's value */
            tv = j->T[(size_t)((m + N) / 2) * TCOLS_MAG + (dk + 4) / 2 + (s[i] ? 5 : 0)];
        } else {
            tv = j->T[(size_t)k * TCOLS + (dk + 4)];
        }
        if (accept(u, tv)) {
            if (j->model != MODEL_POTTS) m += ising_value(s_new) - ising_value(s[i]);
            s[i] = s_new;
            k += dk;
        }
    }
    if (j->record != REC_NONE) {
        if (j->model == MODEL_ISING_MAG) {
            /* bin m (up spins); production adds the bond count k of the measurement */
            int b = (m + N) / 2;
            j->hist[(size_t)c * j->n_bins + b] += 1;
            if (j->record == REC_PROD) j->sabs[(size_t)c * j->n_bins + b] += k;
        } else {
            j->hist[(size_t)c * j->n_bins + k] += 1;
            if (j->record == REC_PROD) j->sabs[(size_t)c * j->n_bins + k] += (m < 0) ? -m : m;
        }
    }
    j->k[c] = k;
    j->m[c] = m;
}

static void *sweep_worker(void *arg)
{
    const sweep_job *j = (const sweep_job *)arg;
    for (int c = j->c_begin; c < j->c_end; ++c)
        for (int sw = 0; sw < j->n_sweeps; ++sw)
            sweep_one_chain(j, c, j->sweep0 + (uint32_t)sw);
    return NULL;
}

/* n_sweeps sweeps of chains chain0 .. chain0 + n_chains - 1, sweep numbers
 * sweep0, sweep0+1, ...  Chains are independent, so they are split
 * statically over n_threads. */
void orc_sweeps(int model, int q, int L, int chain0, int n_chains, uint64_t seed, uint32_t sweep0,
                int n_sweeps, int record, const uint32_t *T, uint8_t *spins, int32_t *k,
                int32_t *m, int32_t *hist, int64_t *sabs, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_chains) n_threads = n_chains;
    sweep_job *jobs = (sweep_job *)calloc((size_t)n_threads, sizeof(sweep_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    int per = n_chains / n_threads, rem = n_chains % n_threads, c0 = 0;
    for (int t = 0; t < n_threads; ++t) {
        sweep_job *j = &jobs[t];
        j->model = model; j->q = q; j->L = L; j->chain0 = chain0;
        j->n_bins = (model == MODEL_ISING_MAG) ? L * L + 1 : 2 * L * L + 1;
        j->c_begin = c0; j->c_end = c0 + per + (t < rem ? 1 : 0); c0 = j->c_end;
        j->seed = seed; j->sweep0 = sweep0; j->n_sweeps = n_sweeps; j->record = record;
        j->T = T; j->spins = spins; j->k = k; j->m = m; j->hist = hist; j->sabs = sabs;
    }
    for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, sweep_worker, &jobs[t]);
    sweep_worker(&jobs[0]);
    for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
}

/* ---------------------------------------------------------------------- */
/* Merge and recursion                                                      */
/* ---------------------------------------------------------------------- */

/* H[k] = sum over chains of the per-chain histograms (parallel version). */
void orc_merge(int n_chains, int n_bins, const int32_t *hist, int64_t *H)
{
    for (int b = 0; b < n_bins; ++b) H[b] = 0;
    for (int c = 0; c < n_chains; ++c)
        for (int b = 0; b < n_bins; ++b) H[b] += hist[(size_t)c * n_bins + b];
}

/* W <- W / H in logarithms, only where H > 0; no renormalisation. */
void orc_recursion(int n_bins, const int64_t *H, double *lnW)
{
    for (int b = 0; b < n_bins; ++b)
        if (H[b] > 0) lnW[b] -= log((double)H[b]);
}

/* The same recursion with the update over the visited bins shifted to zero
 * mean (a reading of Sec. 2: W / H fixes W only up to one constant per
 * iteration): ln H(b) minus its mean over the bins with H(b) > 0, the mean
 * summed in bin order. */
void orc_recursion_norm(int n_bins, const int64_t *H, double *lnW)
{
    double sum = 0.0;
    int n = 0;
    for (int b = 0; b < n_bins; ++b)
        if (H[b] > 0) {
            sum += log((double)H[b]);
            ++n;
        }
    const double mean = n > 0 ? sum / n : 0.0;
    for (int b = 0; b < n_bins; ++b)
        if (H[b] > 0) lnW[b] -= log((double)H[b]) - mean;
}
