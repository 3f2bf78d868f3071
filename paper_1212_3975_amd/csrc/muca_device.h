// Data shared by the host runtime and the HIP kernels of the MUCA library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

constexpr int kIsing = 0;
constexpr int kPotts = 1;
constexpr int kIsingMag = 2;   // Ising with weights over the magnetization at fixed beta
constexpr int kRecNone = 0;
constexpr int kRecMuca = 1;
constexpr int kRecProd = 2;

// Sites whose random words one producer pass stages in LDS per chain.
constexpr int kChunkSites = 64;
constexpr int kMaxChainsPerWG = 64;
constexpr int kMaxProducerWaves = 4;

// Device view of one problem.  Spins are site-major with the chain index
// fastest ([N][C]) so that the chains of a workgroup read consecutive bytes.
struct ProbDev {
    int32_t model, q, L, N;
    int32_t nbins, C, trows, tcols;   // table: trows x tcols uint32 words
    uint32_t seed_lo, seed_hi;
    int32_t spin_lds, table_lds;      // placement used by this problem's workgroups
    uint8_t *spins;                   // [N][C]
    int32_t *k;                       // [C]  unsatisfied bonds
    int32_t *m;                       // [C]  Ising magnetisation
    int32_t *hist;                    // [nbins][C] per-chain counts
    int64_t *sabs;                    // [nbins][C] per-chain |M| sums (or null)
    const uint32_t *table;            // device table, layout below
    int64_t *H;                       // [nbins] merged counts
    int64_t *S;                       // [nbins] merged |M| sums
    const double *lnW;                // [nbins] device copy for reweighting
};

// Device table layout.  Ising: row kk = k/2 (0..N), column j = dk/2 + 2
// (dk = -4..4 in steps of 2), 5 columns.  Potts: row k (0..2N), column
// j = dk + 4, 9 columns.  Entries are stored so that a move with draw u is
// accepted iff min(u, 0xfffffffe) < entry; the "always" value 0xffffffff
// then accepts every u, and every other entry t accepts exactly u < t.

// One workgroup's share of a sweep launch: chains [chain0, chain0+nchains)
// of problem prob.
struct WorkItem {
    int32_t prob, chain0, nchains, spin_stride;   // spin_stride: LDS bytes per site
};

// One workgroup's share of a merge launch: bins [bin0, bin0+nb) of prob.
struct MergeItem {
    int32_t prob, bin0, nb, pad;
};

struct SweepLaunch {
    const ProbDev *probs;
    const WorkItem *items;
    int32_t n_items;
    int32_t n_producer_waves;   // 0: the walker draws its own numbers
    int32_t lds_bytes;
    int32_t n_sweeps;
    int32_t record;
    const uint32_t *sweep_ctr;  // device word: sweep number of the first sweep
    uint32_t *status;           // device word, sticky: bit 0 set when a walker's bounded wait expired
    uint32_t wait_polls;        // polls of those bounded waits
};

// Bits of the sweep status word.
constexpr uint32_t kStatusWaitExpired = 1u;

// LDS bytes one work item needs (table, lattice, random-word ring).
int lds_bytes_for(const ProbDev &p, const WorkItem &it, int n_producer_waves);
// Chunks per sweep of the walker that runs this work item; a launch of S
// sweeps counts S times this many chunks in an int32.
int chunks_per_sweep(const ProbDev &p, const WorkItem &it, int n_producer_waves);
// Whether the sweep kernel takes one of the fast walkers (four sites per step:
// Ising, multimagnetic or 8-Potts) for this problem.
bool uses_fast_walker(const ProbDev &p, int n_producer_waves);
// The walker that runs a work item (the codes of muca_launch_info.walker).
int walker_kind(const ProbDev &p, const WorkItem &it, int n_producer_waves);
// Raises the dynamic-LDS limit of the sweep kernel.
hipError_t configure_sweep_kernel(int max_lds_bytes);

// Launchers (muca_kernels.hip).  All enqueue on `stream` and return the HIP status.
hipError_t launch_init(const ProbDev &p, int chain_begin, int n_chains, hipStream_t stream);
hipError_t launch_energy(const ProbDev &p, hipStream_t stream);
// streamed_compact_ising: some work item runs the streamed Ising walker on bit
// lattices (walker_kind 8 or 9); the launch then takes the kernel that
// contains it.
hipError_t launch_sweep(const SweepLaunch &l, bool streamed_compact_ising, hipStream_t stream);
hipError_t launch_advance(uint32_t *sweep_ctr, uint32_t n, hipStream_t stream);
hipError_t launch_merge(const ProbDev *probs, const MergeItem *items, int n_items, int production,
                        int clear, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t *dst, uint32_t value, size_t n, hipStream_t stream);
// Eq. (2) over the bins of p (reads p.model, p.N, p.nbins, p.H, p.S, p.lnW).
hipError_t launch_reweight(const ProbDev &p, const double *betas, int n_betas,
                           double *out /* [3][n_betas] */, hipStream_t stream);
hipError_t launch_copy_bytes(void *dst, const void *src, size_t n, hipStream_t stream);

// Error text of the calls that take no context (mucaLastError(NULL)).
void set_context_free_error(const char *text);

}  // namespace muca
