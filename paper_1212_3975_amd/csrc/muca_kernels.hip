// HIP kernels of the MUCA library for gfx950 (MI355X).
//
// Sweep kernel design.  A chain's sweep is strictly sequential (every update
// reads the chain's current energy bin k), so the only parallelism is across
// chains: one lane per chain.  A workgroup owns up to 64 chains of one
// problem.  Its first wave is the walker: lane c runs chain chain0 + c
// through the sites in order.  Optionally 1..3 more waves are producers:
// they draw the Philox words of a later chunk of sites for every chain into
// an LDS ring while the walker consumes the current chunk, so the walker
// issues no multiplies; for the fast walkers they also form the lattice
// terms of that chunk that the walker's updates can no longer change.  The
// lattice (uint8 per site, chain fastest) and the acceptance table can each
// live in LDS or in HBM; the host picks the placement per problem.
#include <type_traits>

#include "muca_device.h"

namespace muca {

// ------------------------------------------------------------------ Philox

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// products; key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ------------------------------------------------------------------ init

// Infinite-temperature start: site i of chain c takes word 0 of the block at
// counter (i, 0, c, 1).
__global__ void init_kernel(ProbDev p, int chain_begin, int n_chains) {
    const int64_t total = (int64_t)p.N * n_chains;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / n_chains);
        const int c = chain_begin + (int)(t % n_chains);
        const uint4 b = philox4x32_10((uint32_t)i, 0u, (uint32_t)c, 1u, p.seed_lo, p.seed_hi);
        uint8_t s;
        if (p.model != kPotts)
            s = (uint8_t)(b.x >> 31);
        else
            s = (uint8_t)(((uint64_t)b.x * (uint64_t)p.q) >> 32);
        p.spins[(int64_t)i * p.C + c] = s;
    }
}

// k (unsatisfied bonds, right and down bond of every site) and M of every chain.
__global__ void energy_kernel(ProbDev p) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.C) return;
    const int L = p.L;
    int k = 0, m = 0;
    for (int y = 0; y < L; ++y) {
        const int yd = (y + 1 == L) ? 0 : y + 1;
        for (int x = 0; x < L; ++x) {
            const int xr = (x + 1 == L) ? 0 : x + 1;
            const uint8_t s = p.spins[(int64_t)(y * L + x) * p.C + c];
            k += (s != p.spins[(int64_t)(y * L + xr) * p.C + c]);
            k += (s != p.spins[(int64_t)(yd * L + x) * p.C + c]);
            m += s ? 1 : -1;
        }
    }
    p.k[c] = k;
    p.m[c] = (p.model != kPotts) ? m : 0;
}

// ------------------------------------------------------------------ sweep

__host__ __device__ inline int round_up(int v, int a) { return (v + a - 1) / a * a; }

// LDS carve-up of one work item; identical on host (sizing) and device.
//   table  trows x tcols words
//   spins  ceil(N/4) x spin_stride words: word d of lane c holds sites
//          4d..4d+3 of that chain, one byte each
//   ring   two buffers of random words for kChunkSites sites: Ising one
//          uint4 (four acceptance words) per 4 sites and lane, Potts one uint4
//          (offset, word, offset, word) per 2 sites and lane
struct LdsPlan {
    int off_tab, off_spin, off_ring, total;
    int off_rows;   // packed Ising walker only: the ring of unpacked rows
    int off_ctr;    // streamed walkers only: progress counters
};
// The packed Ising walker: L = 64 with more than 16 chains per workgroup
// (32-bit table), and L = 96 and 128 with the compact table below.  A lane's
// lattice is L*L/32 dwords of bits (odd stride), its row ring four rows of L/4
// byte dwords (odd stride), and random words come in chunks of 32 sites.
constexpr int kPackedChunkDwords = 8;
__host__ __device__ constexpr int packed_bit_stride(int L) { return L * L / 32 + 1; }
__host__ __device__ constexpr int packed_row_stride(int L) { return L + 1; }
// Ising lattices whose 32-bit table does not fit in LDS beside their lattices:
// the walker keeps a compact table there (one u16 per pair of neighbouring
// rows, see run_ising_packed) and reads the full table in HBM only for the
// rare draws the compact entry cannot decide.
__host__ __device__ inline bool compact_ising(const ProbDev &p) {
    return p.model == kIsing && (p.L == 96 || p.L == 128);
}
__host__ __device__ inline int compact_table_bytes(const ProbDev &p) { return 2 + 4 * (p.N + 1); }
__host__ __device__ inline bool packed_ising(const ProbDev &p, const WorkItem &it) {
    return p.model == kIsing && ((p.L == 64 && it.nchains > 16) || compact_ising(p));
}
__host__ __device__ inline bool fast_ising_ok(const ProbDev &p, int n_producer_waves);
__host__ __device__ inline bool fast_potts_ok(const ProbDev &p, int n_producer_waves);
__host__ __device__ constexpr int fast_rows_per_chunk(int L) { return (64 + L - 1) / L; }
// Potts chunks: 64 sites or more up to 32 chains per workgroup, 32 or more
// beyond (its ring has three buffers of two uint4 per dword, so smaller chunks
// leave LDS for more chains; larger ones cost fewer barriers per site).
__host__ __device__ constexpr bool potts_wide(int nchains) { return nchains > 32; }
__host__ __device__ constexpr int potts_rows_per_chunk(int L, bool wide) {
    return wide ? (32 + L - 1) / L : (64 + L - 1) / L;
}
// 8-state Potts at L = 48: the fast Potts walker with a compact table (one u16
// per pair of rows (k, k+j), j = 1..4, see run_potts_fast), in chunks of one
// row whatever the chain count.
__host__ __device__ inline bool compact_potts(const ProbDev &p) { return p.model == kPotts && p.q == 8 && p.L == 48; }
constexpr int kPottsGuardBytes = 256;   // free LDS before the compact Potts table
__host__ __device__ inline int compact_potts_table_bytes(const ProbDev &p) { return 2 + 8 * (2 * p.N + 1); }
__host__ __device__ inline bool potts_wide_item(const ProbDev &p, const WorkItem &it) {
    return potts_wide(it.nchains) || compact_potts(p);
}
__host__ __device__ constexpr int fast_lane_stride(int L) { return ((L * L / 4) % 2) ? L * L / 4 : L * L / 4 + 1; }
// The streamed Ising walker (run_ising_stream): L = 64 with up to 16 chains
// per workgroup.  Its producers form every dword's complete bulk and hand it
// over through a per-lane ring of one row of 32-byte records (the dword's four
// acceptance words, then its column maps and row steps), with a 16-byte pad
// per lane so that the lanes' 16-byte reads fall in distinct banks.
constexpr int kStreamBatch = 4;   // dwords per progress report and per producer batch
constexpr int kStreamCheck = 1;   // batches the walker checks at once
constexpr int kStreamCtrWords = 8;
__host__ __device__ constexpr int stream_lane_words(int L) { return (L / 4) * 8 + 4; }
__host__ __device__ inline bool stream_ising(const ProbDev &p, const WorkItem &it) {
    return p.model == kIsing && p.L == 64 && it.nchains <= 16;
}
// The streamed compact Potts walker (run_potts_stream): 8-Potts L = 48 with up
// to 32 chains per workgroup; per lane a ring of one row of 48-byte records and
// a 16-byte pad.
constexpr int kPStreamBatch = 4;   // dwords per producer batch and progress report
__host__ __device__ constexpr int pstream_lane_words(int L) { return (L / 4) * 12 + 4; }
__host__ __device__ inline bool stream_potts(const ProbDev &p, const WorkItem &it) {
    return compact_potts(p) && it.nchains <= 32;
}
// The streamed compact Ising walker (run_ising_cstream): Ising L = 96 and 128
// with up to 32 chains per workgroup; bit lattices, the compact table after a
// 16-byte guard, per lane a ring of 48-byte records (one row at L = 96, 16
// dwords at L = 128, where a row would not fit beside the table) and a
// 16-byte pad.
// The same walker on the 32-bit table runs Ising L = 64 with 17 to 64 chains
// per workgroup (32-byte records, one row of them per lane).
constexpr int kCStreamGuard = 16;
__host__ __device__ constexpr int cstream_slots(int L) { return L / 4 > 24 ? 16 : L / 4; }
__host__ __device__ constexpr int cstream_lane_words(int L, bool compact) {
    return cstream_slots(L) * (compact ? 12 : 8) + 4;
}
__host__ __device__ inline bool stream_compact_ising(const ProbDev &p, const WorkItem &it) {
    return p.model == kIsing && (p.L == 96 || p.L == 128) && it.nchains <= 32;
}
__host__ __device__ inline bool stream_bit_ising(const ProbDev &p, const WorkItem &it) {
    return p.model == kIsing && p.L == 64 && it.nchains > 16;
}
__host__ __device__ inline LdsPlan lds_plan(const ProbDev &p, const WorkItem &it, int n_producer_waves) {
    LdsPlan l;
    l.off_tab = 0;
    const bool compact_i = compact_ising(p) && fast_ising_ok(p, n_producer_waves);
    const bool compact_p = compact_potts(p) && fast_potts_ok(p, n_producer_waves);
    const bool cstream = compact_i && stream_compact_ising(p, it);
    const int tab = !p.table_lds ? 0
                    : round_up(compact_i ? (cstream ? kCStreamGuard : 0) + compact_table_bytes(p)
                                         : compact_p ? kPottsGuardBytes + compact_potts_table_bytes(p)
                                                     : p.trows * p.tcols * 4,
                               16);
    l.off_spin = l.off_tab + tab;
    l.off_rows = 0;
    l.off_ctr = 0;
    if (cstream || (fast_ising_ok(p, n_producer_waves) && stream_bit_ising(p, it))) {
        // bit lattices with an odd dword stride; record rings; counters
        l.off_ring = l.off_spin + round_up(it.nchains * packed_bit_stride(p.L) * 4, 16);
        l.off_ctr = l.off_ring + it.nchains * cstream_lane_words(p.L, cstream) * 4;
        l.total = l.off_ctr + 4 * kStreamCtrWords;
        return l;
    }
    if (fast_ising_ok(p, n_producer_waves) && packed_ising(p, it)) {
        l.off_rows = l.off_spin + round_up(it.nchains * packed_bit_stride(p.L) * 4, 16);
        l.off_ring = l.off_rows + round_up(it.nchains * packed_row_stride(p.L) * 4, 16);
        l.total = l.off_ring + 2 * it.nchains * (kPackedChunkDwords + 1) * 16;
        return l;
    }
    if (fast_ising_ok(p, n_producer_waves) && stream_ising(p, it)) {
        // lane-major lattice with an odd dword stride; record rings; counters
        l.off_ring = l.off_spin + round_up(it.nchains * fast_lane_stride(p.L) * 4, 16);
        l.off_ctr = l.off_ring + it.nchains * stream_lane_words(p.L) * 4;
        l.total = l.off_ctr + 4 * kStreamCtrWords;
        return l;
    }
    if (fast_ising_ok(p, n_producer_waves)) {
        // lane-major lattice with an odd dword stride; ring [2][lane][chunk dwords + 1] uint4
        // of words followed by [2][lane][chunk dwords + 1] uint2 of lattice terms
        const int W = p.L / 4;
        const int cdw = fast_rows_per_chunk(p.L) * W;
        l.off_ring = l.off_spin + round_up(it.nchains * fast_lane_stride(p.L) * 4, 16);
        l.total = l.off_ring + 2 * it.nchains * (cdw + 1) * 24;
        return l;
    }
    if (fast_potts_ok(p, n_producer_waves) && stream_potts(p, it)) {
        // lane-major lattice with an odd dword stride; record rings; counters
        l.off_ring = l.off_spin + round_up(it.nchains * fast_lane_stride(p.L) * 4, 16);
        l.off_ctr = l.off_ring + it.nchains * pstream_lane_words(p.L) * 4;
        l.total = l.off_ctr + 4 * kStreamCtrWords;
        return l;
    }
    if (fast_potts_ok(p, n_producer_waves)) {
        // lane-major lattice; ring of three buffers: [3][lane][chunk dwords + 1] uint4 words
        // followed by [3][lane][chunk dwords + 1] uint4 lattice terms
        const int W = p.L / 4;
        const int cdw = potts_rows_per_chunk(p.L, potts_wide_item(p, it)) * W;
        l.off_ring = l.off_spin + round_up(it.nchains * fast_lane_stride(p.L) * 4, 16);
        l.total = l.off_ring + 3 * it.nchains * (cdw + 1) * 32;
        return l;
    }
    const int spn = p.spin_lds ? round_up((p.N + 3) / 4 * it.spin_stride * 4, 16) : 0;
    l.off_ring = l.off_spin + spn;
    const int words = (p.model == kPotts) ? 2 : 1;
    const int ring = n_producer_waves > 0 ? 2 * kChunkSites * it.spin_stride * 4 * words : 0;
    l.total = l.off_ring + ring;
    return l;
}

int lds_bytes_for(const ProbDev &p, const WorkItem &it, int n_producer_waves) {
    return lds_plan(p, it, n_producer_waves).total;
}

// Chunks one sweep of this work item takes in the walker that runs it (the
// unit of the walkers' int32 loop counters).
int chunks_per_sweep(const ProbDev &p, const WorkItem &it, int n_producer_waves) {
    if (fast_ising_ok(p, n_producer_waves)) {
        if (p.model == kIsing && packed_ising(p, it)) return p.L * (p.L / 4) / kPackedChunkDwords;
        return p.L / fast_rows_per_chunk(p.L);
    }
    if (fast_potts_ok(p, n_producer_waves)) return p.L / potts_rows_per_chunk(p.L, potts_wide_item(p, it));
    return (p.N + kChunkSites - 1) / kChunkSites;
}

// The fast Ising walker (and its multimagnetic variant) has compiled shapes
// for these sizes (Ising also 96 and 128, packed with the compact table) and
// needs both arrays in LDS and producer waves.
__host__ __device__ inline bool fast_ising_ok(const ProbDev &p, int n_producer_waves) {
    const bool size_ok = p.L == 16 || p.L == 24 || p.L == 32 || p.L == 48 || p.L == 64 || compact_ising(p);
    return (p.model == kIsing || p.model == kIsingMag) && size_ok && p.spin_lds && p.table_lds &&
           n_producer_waves > 0;
}
// The fast Potts walker: q = 8, compiled sizes (48 with the compact table),
// both arrays in LDS, producers.
__host__ __device__ inline bool fast_potts_ok(const ProbDev &p, int n_producer_waves) {
    const bool size_ok = p.L == 16 || p.L == 24 || p.L == 32 || compact_potts(p);
    return p.model == kPotts && p.q == 8 && size_ok && p.spin_lds && p.table_lds && n_producer_waves > 0;
}

bool uses_fast_walker(const ProbDev &p, int n_producer_waves) {
    return fast_ising_ok(p, n_producer_waves) || fast_potts_ok(p, n_producer_waves);
}

int walker_kind(const ProbDev &p, const WorkItem &it, int n_producer_waves) {
    if (fast_ising_ok(p, n_producer_waves)) {
        if (p.model == kIsing && stream_compact_ising(p, it)) return 8;
        if (p.model == kIsing && stream_bit_ising(p, it)) return 9;
        if (p.model == kIsing && packed_ising(p, it)) return compact_ising(p) ? 3 : 2;
        if (p.model == kIsing && stream_ising(p, it)) return 6;
        return 1;
    }
    if (fast_potts_ok(p, n_producer_waves)) return stream_potts(p, it) ? 7 : compact_potts(p) ? 5 : 4;
    return 0;
}

// Every access of the sweep kernel names its address space: LDS through
// 32-bit LDS addresses, device memory through address_space(1) pointers.
// Generic (flat) accesses would be slower and, because a flat access may go
// to either memory, would make the compiler wait for all outstanding LDS reads
// wherever one of them might still be pending.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4 lds_u4;
typedef __attribute__((address_space(1))) int32_t g_i32;
typedef __attribute__((address_space(1))) int64_t g_i64;
typedef __attribute__((address_space(1))) uint8_t g_u8;
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

__device__ __forceinline__ uint32_t lds_ld(uint32_t a) { return *(const lds_u32 *)(size_t)a; }
__device__ __forceinline__ void lds_st(uint32_t a, uint32_t v) { *(lds_u32 *)(size_t)a = v; }
__device__ __forceinline__ uint4 lds_ld4(uint32_t a) {
    const u32x4 v = *(const lds_u4 *)(size_t)a;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void lds_st4(uint32_t a, uint4 v) {
    u32x4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *(lds_u4 *)(size_t)a = w;
}

template <bool LDS>
struct SpinRef;
// Lattice in LDS: base = LDS byte address of the lane's bytes in dword 0, stride
// = bytes per dword row (4 * spin_stride); site i is byte i & 3 of dword i >> 2.
template <>
struct SpinRef<true> {
    uint32_t base;
    int stride;
    __device__ __forceinline__ uint32_t addr(int site) const {
        return base + (uint32_t)((site >> 2) * stride + (site & 3));
    }
    __device__ __forceinline__ uint8_t ld(int site) const { return *(const lds_u8 *)(size_t)addr(site); }
    __device__ __forceinline__ void st(int site, uint8_t v) const { *(lds_u8 *)(size_t)addr(site) = v; }
};
// Lattice in HBM: base = spins + chain, stride = C.
template <>
struct SpinRef<false> {
    g_u8 *base;
    int64_t stride;
    __device__ __forceinline__ uint8_t ld(int site) const { return base[(int64_t)site * stride]; }
    __device__ __forceinline__ void st(int site, uint8_t v) const { base[(int64_t)site * stride] = v; }
};

// Threshold table in LDS (LDS byte address) or in HBM.
template <bool LDS>
struct TabRef;
template <>
struct TabRef<true> {
    uint32_t base;
    __device__ __forceinline__ uint32_t ld(int idx) const { return lds_ld(base + 4u * (uint32_t)idx); }
};
template <>
struct TabRef<false> {
    const g_u32 *base;
    __device__ __forceinline__ uint32_t ld(int idx) const { return base[idx]; }
};

// Producer waves: stage the random words of chunk `t` (global chunk counter)
// for every chain of the work item into LDS buffer t & 1.  Acceptance words
// are stored as min(u, 0xfffffffe), so that the walker's single comparison
// "stored < T" means T == 0xffffffff or u < T.  Potts also stores the
// proposal offset floor(r (q-1) / 2^32).
template <int MODEL>
__device__ __forceinline__ void produce_chunk(const ProbDev &p, const WorkItem &it, uint32_t ring, int t, int nchunks,
                              uint32_t sweep0, int ptid, int nprod_threads) {
    const int sw = t / nchunks;
    const int chunk = t - sw * nchunks;
    const uint32_t sweep = sweep0 + (uint32_t)sw;
    const int i0 = chunk * kChunkSites;
    const int i1 = min(p.N, i0 + kChunkSites);
    constexpr int SPB = (MODEL == kPotts) ? 2 : 4;   // sites per Philox block
    const int nblk = (i1 - i0 + SPB - 1) / SPB;
    const int total = nblk * it.nchains;
    const int ls = it.spin_stride;
    const uint32_t r = ring + (uint32_t)((t & 1) * (kChunkSites / SPB) * ls) * 16u;   // LDS byte address
    const uint32_t qm1 = (uint32_t)(p.q - 1);
    for (int w = ptid; w < total; w += nprod_threads) {
        const int b = w / it.nchains;
        const int lane = w - b * it.nchains;
        const uint4 blk = philox4x32_10((uint32_t)(i0 / SPB + b), sweep, (uint32_t)(it.chain0 + lane), 0u,
                                        p.seed_lo, p.seed_hi);
        uint4 o;
        if (MODEL != kPotts) {
            o = make_uint4(min(blk.x, 0xFFFFFFFEu), min(blk.y, 0xFFFFFFFEu), min(blk.z, 0xFFFFFFFEu),
                           min(blk.w, 0xFFFFFFFEu));
        } else {
            o = make_uint4((uint32_t)(((uint64_t)blk.x * qm1) >> 32), min(blk.y, 0xFFFFFFFEu),
                           (uint32_t)(((uint64_t)blk.z * qm1) >> 32), min(blk.w, 0xFFFFFFFEu));
        }
        lds_st4(r + (uint32_t)(b * ls + lane) * 16u, o);
    }
}

// Walker state of one lane (one chain) in the generic walker.
struct WalkState {
    int row;        // table row: k/2 (Ising), k (Potts), up spins (multimagnetic)
    int m;          // Ising magnetisation
    int k;          // unsatisfied bonds (multimagnetic only; the row holds k otherwise)
    int x, y, i;    // current site
};

template <int MODEL, bool SPIN_LDS, bool TAB_LDS>
__device__ __forceinline__ void update_site(const ProbDev &p, const SpinRef<SPIN_LDS> &S,
                                            const TabRef<TAB_LDS> &tab, WalkState &st, uint32_t u, uint32_t tq) {
    const int L = p.L, N = p.N, i = st.i, x = st.x, y = st.y;
    const int il = (x == 0) ? i + L - 1 : i - 1;
    const int ir = (x == L - 1) ? i - L + 1 : i + 1;
    const int iu = (y == 0) ? i + N - L : i - L;
    const int id = (y == L - 1) ? i - N + L : i + L;
    const uint8_t s = S.ld(i);
    const uint8_t a = S.ld(il), b = S.ld(ir), c = S.ld(iu), d = S.ld(id);
    uint8_t snew;
    int col, drow, dk = 0;
    if (MODEL == kIsing) {
        snew = s ^ 1u;
        const int nd = (a != s) + (b != s) + (c != s) + (d != s);
        // dk = 4 - 2 nd bonds; table row moves by dk/2 = 2 - nd, column 4 - nd
        col = 4 - nd;
        drow = 2 - nd;
    } else if (MODEL == kIsingMag) {
        snew = s ^ 1u;
        const int nd = (a != s) + (b != s) + (c != s) + (d != s);
        // row: up spins, -1 when an up spin flips, +1 for a down spin; column
        // 4 - nd (+5 for an up spin); the flip changes k by 4 - 2 nd
        col = 4 - nd + (s ? 5 : 0);
        drow = s ? -1 : 1;
        dk = 4 - 2 * nd;
    } else {
        const uint32_t q = (uint32_t)p.q;
        uint32_t v = (uint32_t)s + 1u + tq;
        snew = (uint8_t)(v >= q ? v - q : v);
        const int before = (a != s) + (b != s) + (c != s) + (d != s);
        const int after = (a != snew) + (b != snew) + (c != snew) + (d != snew);
        drow = after - before;
        col = drow + 4;
    }
    const uint32_t t = tab.ld(st.row * (MODEL == kIsing ? 5 : MODEL == kIsingMag ? 10 : 9) + col);
    const bool acc = u < t;   // u arrives as min(u, 0xfffffffe)
    if (acc) {
        S.st(i, snew);
        st.row += drow;
        if (MODEL != kPotts) st.m += snew ? 2 : -2;
        if (MODEL == kIsingMag) st.k += dk;
    }
    st.i = i + 1;
    st.x = x + 1;
    if (st.x == L) {
        st.x = 0;
        st.y = y + 1;
    }
}

__device__ __forceinline__ uint32_t clampw(uint32_t u) { return min(u, 0xFFFFFFFEu); }

// The generic walker's pass over chunk t.
template <int MODEL, bool SPIN_LDS, bool TAB_LDS, bool OWN_RNG>
__device__ __forceinline__ void walk_chunk(const ProbDev &p, const WorkItem &it, const SpinRef<SPIN_LDS> &S,
                                           const TabRef<TAB_LDS> &tab, uint32_t ring, WalkState &st, int t,
                                           int nchunks, uint32_t sweep0, int lane, int record) {
    const int sw = t / nchunks;
    const int chunk = t - sw * nchunks;
    const uint32_t sweep = sweep0 + (uint32_t)sw;
    const int i0 = chunk * kChunkSites;
    const int i1 = min(p.N, i0 + kChunkSites);
    if (chunk == 0) {
        st.i = 0;
        st.x = 0;
        st.y = 0;
    }
    const uint32_t chain = (uint32_t)(it.chain0 + lane);
    if (OWN_RNG) {
        if (MODEL != kPotts) {
            // N is a multiple of 4 for even L: whole blocks of four sites
            for (int i = i0; i < i1; i += 4) {
                const uint4 b = philox4x32_10((uint32_t)(i >> 2), sweep, chain, 0u, p.seed_lo, p.seed_hi);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, clampw(b.x), 0u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, clampw(b.y), 0u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, clampw(b.z), 0u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, clampw(b.w), 0u);
            }
        } else {
            const uint32_t qm1 = (uint32_t)(p.q - 1);
            for (int i = i0; i < i1; i += 2) {
                const uint4 b = philox4x32_10((uint32_t)(i >> 1), sweep, chain, 0u, p.seed_lo, p.seed_hi);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, clampw(b.y),
                                                      (uint32_t)(((uint64_t)b.x * qm1) >> 32));
                if (i + 1 < i1)
                    update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, clampw(b.w),
                                                          (uint32_t)(((uint64_t)b.z * qm1) >> 32));
            }
        }
    } else {
        const int ls = it.spin_stride;
        if (MODEL != kPotts) {
            const uint32_t r = ring + (uint32_t)((t & 1) * (kChunkSites / 4) * ls + lane) * 16u;
            for (int i = i0; i < i1; i += 4) {
                const uint4 w = lds_ld4(r + (uint32_t)(((i - i0) >> 2) * ls) * 16u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, w.x, 0u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, w.y, 0u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, w.z, 0u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, w.w, 0u);
            }
        } else {
            const uint32_t r = ring + (uint32_t)((t & 1) * (kChunkSites / 2) * ls + lane) * 16u;
            for (int i = i0; i < i1; i += 2) {
                const uint4 w = lds_ld4(r + (uint32_t)(((i - i0) >> 1) * ls) * 16u);
                update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, w.y, w.x);
                if (i + 1 < i1) update_site<MODEL, SPIN_LDS, TAB_LDS>(p, S, tab, st, w.w, w.z);
            }
        }
    }
    if (i1 == p.N && record != kRecNone) {
        // bin: k (energy models) or up spins (multimagnetic); production adds
        // |M| per energy bin, or the bond count k per magnetization bin
        const int b = (MODEL == kIsing) ? 2 * st.row : st.row;
        const int c = it.chain0 + lane;
        ((g_i32 *)p.hist)[(int64_t)b * p.C + c] += 1;
        if (record == kRecProd)
            ((g_i64 *)p.sabs)[(int64_t)b * p.C + c] +=
                (MODEL == kIsingMag) ? (int64_t)st.k : (int64_t)(st.m < 0 ? -st.m : st.m);
    }
}

// ------------------------------------------------------------------ fast Ising walker
//
// Sites are handled four at a time: one dword holds four consecutive sites
// of a row (one byte each, 0/1).  With byte-wise xor and add, a few dword ops
// give for all four sites the number of disagreeing neighbours among up,
// down and right; the left neighbour is the only one an earlier update of
// the same sweep can still change, so each site gets two candidate counts,
// D0 (left neighbour kept) and D1 (left neighbour flipped), chosen by the
// previous site's acceptance.  A move with D disagreeing neighbours changes
// k by 2(2 - D): the table row moves by 2 - D rows (20 bytes each) and the
// move reads column 4 - D (byte offset 16 - 4D).  Both byte maps are applied
// to four sites at once with v_perm as a lookup table.
//
// The dependence from one site to the next is then only "select, compare":
// while site j is decided, the table words of site j+1 for both outcomes of
// site j are already in flight (row unchanged with D0, or row moved with D1).
//
// Layout: each lane's lattice is contiguous in LDS (row-major dwords, an odd
// dword stride between lanes so that lanes hit different banks); L is a
// compile-time constant, so every neighbour read is a fixed offset from one
// of a few row pointers.  The row above the current one is the walker's own
// output and stays in registers.  The producers fill, per chunk of rows, a
// ring [buffer][lane][dword] of uint4 random words followed by a ring of the
// dword's lattice terms that do not involve the row above (uint2 counts for
// Ising, uint4 for Potts).

__device__ __forceinline__ uint32_t ubyte(uint32_t v, int j) { return (v >> (8 * j)) & 0xFFu; }
__device__ __forceinline__ int32_t sbyte(uint32_t v, int j) { return (int32_t)(int8_t)(uint8_t)(v >> (8 * j)); }

struct FastBulk {
    uint32_t cur;      // old spins of the dword
    uint32_t a0, a1;   // bytes: column byte offset 16 - 4D for D0 / D1
    uint32_t e0, e1;   // bytes (int8): row byte step 40 - 20D for D0 / D1 (multimagnetic: +-40)
};

// The bulk of a dword in three pieces (so that a walker can spread it over
// the sites of the previous dword): the neighbour sums, the candidate counts
// D0 (left neighbour kept) and D1 (left neighbour flipped), and the byte maps.
struct BulkSums {
    uint32_t cur, s3, ml;   // old spins; up+down+right disagreements; left disagreement
};

__device__ __forceinline__ BulkSums bulk_sums(uint32_t cur, uint32_t prv, uint32_t nxt, uint32_t up, uint32_t dn) {
    // right neighbours: bytes cur1 cur2 cur3 nxt0; left (old): prv3 cur0 cur1 cur2
    const uint32_t rn = __builtin_amdgcn_alignbyte(nxt, cur, 1);
    const uint32_t lo = __builtin_amdgcn_alignbyte(cur, prv, 3);
    return BulkSums{cur, (cur ^ up) + (cur ^ dn) + (cur ^ rn), cur ^ lo};
}

struct BulkDiff {
    uint32_t cur, d0, d1;
};

template <bool ROW_START>
__device__ __forceinline__ BulkDiff bulk_diff(const BulkSums &q) {
    BulkDiff d;
    d.cur = q.cur;
    d.d0 = q.s3 + q.ml;
    d.d1 = q.s3 + (q.ml ^ 0x01010101u);
    // the first site of a row has its left neighbour at the row's end, which
    // this sweep has not visited yet: both candidates agree
    if (ROW_START) d.d1 = (d.d1 & 0xFFFFFF00u) | (d.d0 & 0xFFu);
    return d;
}

// Column byte offsets (16 - 4D) of both candidates.
template <bool MAG>
__device__ __forceinline__ void bulk_cols(const BulkDiff &d, FastBulk &b) {
    b.cur = d.cur;
    b.a0 = __builtin_amdgcn_perm(0u, 0x04080C10u, d.d0);           // 16,12,8,4,0
    b.a1 = __builtin_amdgcn_perm(0u, 0x04080C10u, d.d1);
    if (MAG) {
        // multimagnetic rows are up-spin counts of 40 bytes (ten columns): an
        // up spin reads the columns 5..9
        const uint32_t s20 = __builtin_amdgcn_perm(0u, 0x00001400u, d.cur);   // 0 / 20 per byte
        b.a0 += s20;
        b.a1 += s20;
    }
}

// Row byte steps (40 - 20D) of both candidates; multimagnetic rows move by
// -40 for an up spin and +40 for a down one, whatever the left neighbour did.
template <bool MAG>
__device__ __forceinline__ void bulk_steps(const BulkDiff &d, FastBulk &b) {
    if (MAG) {
        b.e0 = __builtin_amdgcn_perm(0u, 0x0000D828u, d.cur);                 // +40 / -40
        b.e1 = b.e0;
    } else {
        b.e0 = __builtin_amdgcn_perm(0xD8u, 0xEC001428u, d.d0);        // 40,20,0,-20,-40
        b.e1 = __builtin_amdgcn_perm(0xD8u, 0xEC001428u, d.d1);
    }
}

template <bool ROW_START, bool MAG = false>
__device__ __forceinline__ FastBulk fast_bulk(uint32_t cur, uint32_t prv, uint32_t nxt, uint32_t up, uint32_t dn) {
    const BulkDiff d = bulk_diff<ROW_START>(bulk_sums(cur, prv, nxt, up, dn));
    FastBulk b;
    bulk_cols<MAG>(d, b);
    bulk_steps<MAG>(d, b);
    return b;
}

// Walker state between sites: the table row before the previous site's move
// (R) and after it (C), the current site's table words for both outcomes of
// the previous site (tA kept, tB flipped), and that outcome (acc).
struct FastState {
    uint32_t R, C, tA, tB;
    bool acc;
};

// The four sites of one dword.  Each site is issued in fenced parts:
//   1. from the previous site's outcome, the row and the two table reads of
//      the next site (both outcomes of this one);
//   2. this site's decision, on the words read one site earlier;
//   3. independent work: a piece of the next dword's bulk;
//   4. the flip record of this site.
// The fences keep about a site of work between a table read and its use,
// which hides the LDS latency, and keep three or more instructions between a
// decision and the next read of it as a lane mask, which hides the latency
// of a compare result.  Pieces: work(0) loads, work(1) neighbour sums,
// work(2) candidate counts and column maps (site 3's reads need them),
// work(3) row steps.  Returns the accepted sites of the dword: FLIP << (STRIDE j)
// for an accepted site j.
// Row byte step of site j of a dword if it is accepted, for both outcomes of
// the previous site (Ising and multimagnetic: the step itself; Potts: dk
// rows of 36 bytes).
__device__ __forceinline__ int32_t row_step(const FastBulk &b, bool left_flipped, int j) {
    return left_flipped ? sbyte(b.e1, j) : sbyte(b.e0, j);
}

template <class Bulk, uint32_t FLIP, int STRIDE, class Work>
__device__ __forceinline__ uint32_t walk_dword(FastState &s, const Bulk &b, const Bulk &nb, const uint4 &u,
                                               Work &&work) {
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t Rj = s.acc ? s.C : s.R;
        const uint32_t Cj = Rj + (uint32_t)row_step(b, s.acc, j);
        const uint32_t a0 = (j < 3) ? ubyte(b.a0, j + 1) : ubyte(nb.a0, 0);
        const uint32_t a1 = (j < 3) ? ubyte(b.a1, j + 1) : ubyte(nb.a1, 0);
        const uint32_t nA = lds_ld(Rj + a0);
        const uint32_t nB = lds_ld(Cj + a1);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t tj = s.acc ? s.tB : s.tA;
        const uint32_t uj = (j == 0) ? u.x : (j == 1) ? u.y : (j == 2) ? u.z : u.w;
        s.acc = uj < tj;
        s.R = Rj;
        s.C = Cj;
        s.tA = nA;
        s.tB = nB;
        __builtin_amdgcn_sched_barrier(0);
        work(j);
        __builtin_amdgcn_sched_barrier(0);
        f |= s.acc ? (FLIP << (STRIDE * j)) : 0u;   // accepted: site j
        __builtin_amdgcn_sched_barrier(0);
    }
    return f;
}

// Bond count k of a lane-major LDS lattice (right and down bond of every site).
template <int L>
__device__ __forceinline__ int lattice_bonds(uint32_t sb) {
    constexpr int W = L / 4;
    int k = 0;
    for (int y = 0; y < L; ++y) {
        const uint32_t r = sb + (uint32_t)(y * W) * 4u, rd = sb + (uint32_t)((y + 1 == L ? 0 : y + 1) * W) * 4u;
        for (int w = 0; w < W; ++w) {
            const uint32_t cur = lds_ld(r + 4u * w), nxt = lds_ld(r + 4u * (w + 1 == W ? 0 : w + 1));
            k += __builtin_popcount(cur ^ __builtin_amdgcn_alignbyte(nxt, cur, 1)) +
                 __builtin_popcount(cur ^ lds_ld(rd + 4u * w));
        }
    }
    return k;
}

// Producer side of the Ising bulk for one dword: the candidate counts D0, D1
// over the down, right and left neighbours (without the row above, which the
// walker is updating, and without the right neighbour of a row's last site,
// the row's first site of this sweep).  At a row start both candidates agree.
__device__ __forceinline__ uint2 ising_pre(uint32_t cur, uint32_t prv, uint32_t nxt, uint32_t dn, bool row_start,
                                           bool row_end) {
    const uint32_t rn = __builtin_amdgcn_alignbyte(nxt, cur, 1);
    const uint32_t lo = __builtin_amdgcn_alignbyte(cur, prv, 3);
    const uint32_t s2 = (cur ^ dn) + ((cur ^ rn) & (row_end ? 0x00FFFFFFu : 0xFFFFFFFFu));
    const uint32_t ml = cur ^ lo;
    const uint32_t p0 = s2 + ml;
    uint32_t p1 = s2 + (ml ^ 0x01010101u);
    if (row_start) p1 = (p1 & 0xFFFFFF00u) | (p0 & 0xFFu);
    return make_uint2(p0, p1);
}

template <int L, bool MAG>
__device__ __forceinline__ void run_ising_fast(const ProbDev &p, const WorkItem &it, char *lds, const SweepLaunch &l,
                               uint32_t sweep0, const LdsPlan &plan) {
    // table row bytes: Ising rows k/2 of five words, multimagnetic rows m of ten
    constexpr uint32_t RB = MAG ? 40u : 20u;
    constexpr int W = L / 4;                  // dwords per row
    constexpr int NW = L * L / 4;             // dwords per lattice
    constexpr int RPC = fast_rows_per_chunk(L);
    constexpr int CDW = RPC * W;              // dwords per chunk
    constexpr int NCH = L / RPC;              // chunks per sweep
    constexpr int P = fast_lane_stride(L);    // dwords between lanes
    static_assert(L % RPC == 0 && W >= 4, "fast walker shape");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int nch = it.nchains;
    const bool active = (wave == 0) && (lane < nch);
    const uint32_t lbase = (uint32_t)(size_t)(__attribute__((address_space(3))) char *)lds;
    const uint32_t tab0 = lbase + (uint32_t)plan.off_tab;
    const uint32_t spin0 = lbase + (uint32_t)plan.off_spin;
    const uint32_t ring0 = lbase + (uint32_t)plan.off_ring;
    const uint32_t ringbuf = (uint32_t)nch * (CDW + 1) * 16u;   // bytes per ring buffer of words
    const uint32_t ringp0 = ring0 + 2u * ringbuf;                // [2][lane][CDW+1] uint2 lattice terms
    const uint32_t pbuf = (uint32_t)nch * (CDW + 1) * 8u;

    // stage the lattice: lane c's dword d = sites 4d..4d+3 of chain chain0 + c
    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const g_u8 *g = (const g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        const uint32_t v = (uint32_t)g[0] | ((uint32_t)g[p.C] << 8) | ((uint32_t)g[2 * (int64_t)p.C] << 16) |
                           ((uint32_t)g[3 * (int64_t)p.C] << 24);
        lds_st(spin0 + (uint32_t)(c * P + d) * 4u, v);
    }
    __syncthreads();

    const uint32_t sb = spin0 + (uint32_t)(lane * P) * 4u;   // this lane's lattice
    const uint32_t rb = ring0 + (uint32_t)(lane * (CDW + 1)) * 16u;
    const uint32_t rbp = ringp0 + (uint32_t)(lane * (CDW + 1)) * 8u;
    auto row_addr = [&](int y) -> uint32_t { return sb + (uint32_t)(y * W) * 4u; };

    FastState st{0, 0, 0, 0, false};
    FastBulk nb{0, 0, 0, 0, 0};
    // the row above the current row, as updated in this sweep (dword w of the
    // current row replaces it once written): the walker's own stores, kept in
    // registers
    uint32_t upr[W];
#pragma unroll
    for (int w = 0; w < W; ++w) upr[w] = 0;
    if (active) {
#pragma unroll
        for (int w = 0; w < W; ++w) upr[w] = lds_ld(row_addr(L - 1) + 4u * w);
        const int k = ((const g_i32 *)p.k)[it.chain0 + lane];
        st.R = MAG ? tab0 + RB * (uint32_t)((((const g_i32 *)p.m)[it.chain0 + lane] + L * L) / 2)
                   : tab0 + RB * (uint32_t)(k >> 1);
        st.C = st.R;
        const uint32_t r0 = row_addr(0), rl = row_addr(L - 1), r1 = row_addr(1);
        nb = fast_bulk<true, MAG>(lds_ld(r0), lds_ld(r0 + 4 * (W - 1)), lds_ld(r0 + 4), lds_ld(rl), lds_ld(r1));
        st.tA = lds_ld(st.R + ubyte(nb.a0, 0));
        st.tB = st.tA;
    }

    // producers: chunk t covers rows (t mod NCH) * RPC .. + RPC - 1 of sweep t / NCH.
    // One chunk ahead of the walker, the rows of the chunk and the row below it
    // hold their final values of the previous sweep (below the last row: row
    // 0 of this sweep), so the producers also form the lattice terms that do
    // not involve the row above.
    auto produce = [&](int t) {
        const int sw = t / NCH;
        const uint32_t sweep = sweep0 + (uint32_t)sw;
        const int ci = t - sw * NCH;
        const int blk0 = ci * CDW;   // Philox block of the chunk's first dword
        const uint32_t buf = ring0 + (uint32_t)(t & 1) * ringbuf;
        const uint32_t bp = ringp0 + (uint32_t)(t & 1) * pbuf;
        const int total = CDW * nch;
        for (int w = tid - 64; w < total; w += nthreads - 64) {
            const int c = w / CDW, q = w - c * CDW;
            const uint4 b = philox4x32_10((uint32_t)(blk0 + q), sweep, (uint32_t)(it.chain0 + c), 0u, p.seed_lo,
                                          p.seed_hi);
            lds_st4(buf + (uint32_t)(c * (CDW + 1) + q) * 16u,
                    make_uint4(min(b.x, 0xFFFFFFFEu), min(b.y, 0xFFFFFFFEu), min(b.z, 0xFFFFFFFEu),
                               min(b.w, 0xFFFFFFFEu)));
            const int r = q / W, x = q - r * W;
            const int y = ci * RPC + r;
            const uint32_t lb = spin0 + (uint32_t)(c * P) * 4u;
            const uint32_t rowb = lb + (uint32_t)(y * W) * 4u;
            const uint32_t cur = lds_ld(rowb + 4u * (uint32_t)x);
            const uint32_t prv = lds_ld(rowb + 4u * (uint32_t)(x == 0 ? W - 1 : x - 1));
            const uint32_t nxt = lds_ld(rowb + 4u * (uint32_t)(x + 1 == W ? x : x + 1));
            const uint32_t dn = lds_ld(lb + (uint32_t)(((y + 1 == L) ? 0 : y + 1) * W + x) * 4u);
            const uint2 pe = ising_pre(cur, prv, nxt, dn, x == 0, x + 1 == W);
            lds_st(bp + (uint32_t)(c * (CDW + 1) + q) * 8u, pe.x);
            lds_st(bp + (uint32_t)(c * (CDW + 1) + q) * 8u + 4u, pe.y);
        }
    };

    const int total_chunks = NCH * l.n_sweeps;
    if (wave > 0) produce(0);
    __syncthreads();
    uint4 u_next = make_uint4(0, 0, 0, 0);
    for (int t = 0; t < total_chunks; ++t) {
        if (wave == 0) {
            if (active) {
                const int ci = t % NCH;                 // chunk within the sweep
                const uint32_t ub = rb + (uint32_t)(t & 1) * ringbuf;
                const uint32_t pb = rbp + (uint32_t)(t & 1) * pbuf;
#pragma unroll
                for (int r = 0; r < RPC; ++r) {
                    const int y = ci * RPC + r;
                    const uint32_t vcur = row_addr(y);
                    // rows of the next row's bulk (wrapping into the next sweep)
                    const int yn = (y + 1 == L) ? 0 : y + 1;
                    const uint32_t vnc = row_addr(yn);
                    const uint32_t vnd = row_addr(yn + 1 == L ? 0 : yn + 1);
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const FastBulk b = nb;
                        // random words of this dword (prefetched one dword ahead inside the chunk)
                        const uint4 u = (r == 0 && w == 0) ? lds_ld4(ub) : u_next;
                        // the next dword's bulk, in pieces between this dword's sites
                        // (within the chunk from the producers' lattice terms; the next
                        // chunk's first dword, whose terms are still being formed, in full)
                        const bool in_chunk = (w + 1 < W) || (r + 1 < RPC);
                        uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, first = 0;
                        uint2 pe = make_uint2(0, 0);
                        BulkSums ns{0, 0, 0};
                        BulkDiff nd{0, 0, 0};
                        auto work = [&](int j) {
                            if (j == 0) {
                                if (r * W + w + 1 < CDW) u_next = lds_ld4(ub + (uint32_t)(r * W + w + 1) * 16u);
                                if (w + 1 < W) {
                                    q0 = lds_ld(vcur + 4 * (w + 1));                          // old dword w+1
                                    q3 = upr[w + 1];
                                    pe.x = lds_ld(pb + (uint32_t)(r * W + w + 1) * 8u);
                                    pe.y = lds_ld(pb + (uint32_t)(r * W + w + 1) * 8u + 4u);
                                    if (w + 2 == W) first = upr[0];   // the row's first dword, this sweep
                                } else if (in_chunk) {
                                    q0 = lds_ld(vnc);
                                    q3 = upr[0];                         // upper row: this one (new)
                                    pe.x = lds_ld(pb + (uint32_t)((r + 1) * W) * 8u);
                                    pe.y = lds_ld(pb + (uint32_t)((r + 1) * W) * 8u + 4u);
                                } else {
                                    // first dword of the next chunk: all neighbours here
                                    q0 = lds_ld(vnc);
                                    q1 = lds_ld(vnc + 4 * (W - 1));
                                    q2 = lds_ld(vnc + 4);
                                    q3 = upr[0];
                                    q4 = lds_ld(vnd);
                                }
                            } else if (j == 1) {
                                if (in_chunk) {
                                    const uint32_t xu = q0 ^ q3;
                                    uint32_t d0 = pe.x + xu, d1 = pe.y + xu;
                                    if (w + 2 == W) {
                                        const uint32_t cr = (q0 ^ (first << 24)) & 0xFF000000u;
                                        d0 += cr;
                                        d1 += cr;
                                    }
                                    nd = BulkDiff{q0, d0, d1};
                                } else {
                                    ns = bulk_sums(q0, q1, q2, q3, q4);
                                }
                            } else if (j == 2) {
                                if (!in_chunk) nd = bulk_diff<true>(ns);
                                bulk_cols<MAG>(nd, nb);
                            } else {
                                bulk_steps<MAG>(nd, nb);
                            }
                        };
                        const uint32_t f = walk_dword<FastBulk, 1u, 8>(st, b, nb, u, work);
                        upr[w] = b.cur ^ f;
                        lds_st(vcur + 4 * w, upr[w]);
                    }
                    if (y == L - 1 && l.record != kRecNone) {
                        const uint32_t Rk = st.acc ? st.C : st.R;
                        // bin: k (row k/2) or, multimagnetic, the up-spin count m (the row)
                        const int bin = MAG ? (int)((Rk - tab0) / RB) : 2 * (int)((Rk - tab0) / RB);
                        const int64_t cidx = (int64_t)bin * p.C + it.chain0 + lane;
                        g_i32 *h = (g_i32 *)p.hist;
                        h[cidx] += 1;
                        if (l.record == kRecProd) {
                            g_i64 *s = (g_i64 *)p.sabs;
                            if (MAG) {
                                s[cidx] += (int64_t)lattice_bonds<L>(sb);
                            } else {
                                int ones = 0;
                                for (int dd = 0; dd < NW; ++dd) ones += __builtin_popcount(lds_ld(sb + 4u * dd));
                                const int m = 2 * ones - L * L;
                                s[cidx] += (int64_t)(m < 0 ? -m : m);
                            }
                        }
                    }
                }
            }
        } else if (t + 1 < total_chunks) {
            produce(t + 1);
        }
        __syncthreads();
    }

    if (active) {
        const uint32_t Rk = st.acc ? st.C : st.R;
        ((g_i32 *)p.k)[it.chain0 + lane] = MAG ? lattice_bonds<L>(sb) : 2 * (int)((Rk - tab0) / RB);
        int ones = 0;
        for (int dd = 0; dd < NW; ++dd) ones += __builtin_popcount(lds_ld(sb + 4u * dd));
        ((g_i32 *)p.m)[it.chain0 + lane] = 2 * ones - L * L;
    }
    __syncthreads();
    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const uint32_t v = lds_ld(spin0 + (uint32_t)(c * P + d) * 4u);
        g_u8 *g = (g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        g[0] = (uint8_t)v;
        g[p.C] = (uint8_t)(v >> 8);
        g[2 * (int64_t)p.C] = (uint8_t)(v >> 16);
        g[3 * (int64_t)p.C] = (uint8_t)(v >> 24);
    }
}


// ------------------------------------------------------------------ streamed Ising walker
//
// The byte walker above still forms part of every dword's bulk itself: the
// terms of the row above, which it is updating in the same sweep.  But dword
// (y, w) needs only dword (y-1, w) of this sweep, which the walker finished a
// full row (L/4 dwords) before it reaches (y, w).  Here the producer waves
// form the complete bulk of every dword (column maps and row steps of both
// candidates, from the dword's old spins, its left, right and lower
// neighbours and the row above as this sweep left it) and hand it to the
// walker in a record beside the dword's four acceptance words.  The walker
// only decides sites, xors each dword's flips into the lattice and reports
// its progress.
//
// Walker and producers exchange progress through LDS counters instead of
// workgroup barriers:
//   - the walker publishes the number of dwords it has finished after every
//     batch of kStreamBatch dwords and after each row's first dword;
//   - producer wave i forms the batches i, i+np, i+2np, ... of every sweep (np
//     producer waves); the batches are published in order, on one counter of
//     the batches formed, each wave waiting for the previous batch's.
// A batch of row y may be formed once the walker has finished the batch's
// dwords of row y-1; a row's last batch also needs the row's first dword (the
// right neighbour of the row's last site, this sweep).  The producers read
// and count everything else (the old left, right and lower neighbours, the
// random words) before they wait.  The walker checks the next batch one
// dword before it first reads it (the counter was read a dword earlier, so
// the check costs no LDS wait).  Each side has several dwords of slack, so
// neither normally waits long.  Both sides wait with a bounded poll: if one
// expires the workgroup raises an abort word that ends every other wait, the
// walker rewrites its records to reject every move, the workgroup finishes
// with invalid chains and sets the launch's status word, which the host
// reports.  LDS operations of one wave are performed in order, so a counter
// written after data is never seen before that data.
//
// Records: per lane a ring of one row of 32-byte slots; slot w holds dword w
// of the row being formed (random words, then a0, a1, e0, e1).  Slot w of row
// y replaces slot w of row y-1 only after the walker has finished (y-1, w).

__device__ __forceinline__ uint32_t lds_ld_sync(uint32_t a) {
    return __hip_atomic_load((lds_u32 *)(size_t)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st_sync(uint32_t a, uint32_t v) {
    __hip_atomic_store((lds_u32 *)(size_t)a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_xor(uint32_t a, uint32_t v) {
    (void)__hip_atomic_fetch_xor((lds_u32 *)(size_t)a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Keeps the compiler from moving memory accesses across this point (the
// hardware keeps one wave's LDS operations in order by itself).
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// Counters of the streamed walker, LDS words from ctr: [0] batches formed
// (published in order), [1] dwords the walker has finished, [7] abort.
constexpr uint32_t kCtrFormed = 0u, kCtrDone = 4u, kCtrAbort = 28u;

// Bounded wait, wave-uniform: polls (up to `polls` times; 2^24 polls take a
// second or more) until the counter at ctr + off reaches want (wrap-safe).
// Returns false at once if the abort word is raised; raises it and returns
// false if the count is not reached.
__device__ __noinline__ bool stream_wait(uint32_t ctr, uint32_t off, uint32_t want, uint32_t polls) {
    for (uint32_t n = 0; n < polls; ++n) {
        if ((int32_t)(lds_ld_sync(ctr + off) - want) >= 0) {
            lds_order();
            return true;
        }
        if (lds_ld_sync(ctr + kCtrAbort)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    lds_st_sync(ctr + kCtrAbort, 1u);
    return false;
}

// The four sites of one dword for the streamed walker: as walk_dword, but
// with no bulk to interleave.  Between its compare and the next site's row
// select, which reads the compare as a lane mask, each site records the flip
// of the previous site, whose compare is a full site old, so that the select
// does not wait for a fresh compare.  The dword's last flip is recorded by the
// next dword's first site, which passes the previous dword's finished flip
// record to done() (bit 8 j for site j).  Returns the record of sites 0..2;
// site 3's outcome is s.acc.
template <class Work, class Done>
__device__ __forceinline__ uint32_t walk_dword_stream(FastState &s, const FastBulk &b, const FastBulk &nb,
                                                      const uint4 &u, uint32_t fprev, Work &&work, Done &&done) {
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t Rj = s.acc ? s.C : s.R;
        const uint32_t Cj = Rj + (uint32_t)row_step(b, s.acc, j);
        const uint32_t a0 = (j < 3) ? ubyte(b.a0, j + 1) : ubyte(nb.a0, 0);
        const uint32_t a1 = (j < 3) ? ubyte(b.a1, j + 1) : ubyte(nb.a1, 0);
        const uint32_t nA = lds_ld(Rj + a0);
        const uint32_t nB = lds_ld(Cj + a1);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t tj = s.acc ? s.tB : s.tA;
        const uint32_t uj = (j == 0) ? u.x : (j == 1) ? u.y : (j == 2) ? u.z : u.w;
        const bool prev = s.acc;
        s.acc = uj < tj;
        s.R = Rj;
        s.C = Cj;
        s.tA = nA;
        s.tB = nB;
        __builtin_amdgcn_sched_barrier(0);
        if (j == 0) {
            done(fprev | (prev ? 0x01000000u : 0u));
        } else {
            f |= prev ? (1u << (8 * (j - 1))) : 0u;
            asm volatile("" : "+v"(f));   // recorded here, not at the end of the dword
        }
        work(j);
        __builtin_amdgcn_sched_barrier(0);
    }
    return f;
}

template <int L>
__device__ __forceinline__ void run_ising_stream(const ProbDev &p, const WorkItem &it, char *lds, const SweepLaunch &l,
                                                 uint32_t sweep0, const LdsPlan &plan) {
    constexpr uint32_t RB = 20u;              // table row bytes
    constexpr int W = L / 4;                  // dwords per row
    constexpr int NW = L * L / 4;             // dwords per lattice
    constexpr int P = fast_lane_stride(L);    // lattice dwords between lanes
    constexpr int B = kStreamBatch;
    constexpr int BPR = W / B;                // batches per row
    constexpr int BPS = L * BPR;              // batches per sweep
    constexpr uint32_t RS = stream_lane_words(L) * 4u;   // ring bytes per lane
    // the walker checks batches c+1 .. c+K (K = kStreamCheck) in the last
    // dword of every K-th batch c: by then it has finished what every record
    // of those batches depends on (W >= (K+1) B + 1), a row's last batch
    // included (it also needs the row's first dword)
    constexpr int K = kStreamCheck;
    static_assert(W % (K * B) == 0 && W >= (K + 1) * B + 1, "streamed walker shape");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int np = nthreads / 64 - 1;         // producer waves
    const int nch = it.nchains;
    const bool active = (wave == 0) && (lane < nch);
    const uint32_t lbase = (uint32_t)(size_t)(__attribute__((address_space(3))) char *)lds;
    const uint32_t tab0 = lbase + (uint32_t)plan.off_tab;
    const uint32_t spin0 = lbase + (uint32_t)plan.off_spin;
    const uint32_t ring0 = lbase + (uint32_t)plan.off_ring;
    const uint32_t ctr = lbase + (uint32_t)plan.off_ctr;   // counters (see kCtrDone)

    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const g_u8 *g = (const g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        const uint32_t v = (uint32_t)g[0] | ((uint32_t)g[p.C] << 8) | ((uint32_t)g[2 * (int64_t)p.C] << 16) |
                           ((uint32_t)g[3 * (int64_t)p.C] << 24);
        lds_st(spin0 + (uint32_t)(c * P + d) * 4u, v);
    }
    if (tid < kStreamCtrWords) lds_st(ctr + 4u * (uint32_t)tid, 0u);
    __syncthreads();

    const int n_sweeps = l.n_sweeps;
    if (wave == 0) {
        if (active) {
            const uint32_t sb = spin0 + (uint32_t)(lane * P) * 4u;   // this lane's lattice
            const uint32_t rb = ring0 + (uint32_t)lane * RS;          // this lane's records
            auto row_addr = [&](int y) -> uint32_t { return sb + (uint32_t)(y * W) * 4u; };
            FastState st{0, 0, 0, 0, false};
            const int k0 = ((const g_i32 *)p.k)[it.chain0 + lane];
            st.R = tab0 + RB * (uint32_t)(k0 >> 1);
            st.C = st.R;
            // After a wait gives up, the walker rewrites its records to reject
            // every move (draws 2^32 - 1, column 0, no row step) and walks them
            // to the end of the row: nothing changes, every read stays in the
            // table, and the loops stay free of exits.
            auto neutralize = [&]() {
                for (int w = 0; w < W; ++w) {
                    lds_st4(rb + (uint32_t)w * 32u, make_uint4(~0u, ~0u, ~0u, ~0u));
                    lds_st4(rb + (uint32_t)w * 32u + 16u, make_uint4(0u, 0u, 0u, 0u));
                }
            };
            bool ok = stream_wait(ctr, kCtrFormed, 1u, l.wait_polls);   // batch 0 of the launch
            if (!ok) neutralize();
            uint4 u_next = lds_ld4(rb);
            const uint4 m0 = lds_ld4(rb + 16u);
            FastBulk nb{0, m0.x, m0.y, m0.z, m0.w};
            st.tA = lds_ld(st.R + ubyte(nb.a0, 0));
            st.tB = st.tA;
            uint32_t c = 0;        // batches walked before the current one (wraps)
            uint32_t formed = 0;   // batches formed, read a dword before the check
            uint32_t fpend = 0;    // flips of sites 0..2 of the last dword walked, not yet in the lattice
            uint32_t apend = sb;   // that dword's address (nothing pending before the first dword)
            for (int s = 0; s < n_sweeps && ok; ++s) {
                for (int y = 0; y < L && ok; ++y) {
                    const uint32_t vcur = row_addr(y);
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const int q = w % B;
                        // in a batch's last dword (every K-th batch): batches c + 1 (whose
                        // first record this dword's first site reads) .. c + K, none
                        // beyond the launch; the counter was read a dword earlier
                        const int qk = w % (K * B);
                        if (qk == B - 2) formed = lds_ld_sync(ctr + kCtrFormed);
                        if (qk == B - 1 && ok) {
                            const uint32_t f1 = __builtin_amdgcn_readfirstlane(formed);
                            uint32_t want = __builtin_amdgcn_readfirstlane(c) + (uint32_t)(K + 1);
                            if (y == L - 1 && s + 1 == n_sweeps) {
                                const int left = (W - 1 - w) / B;   // batches of the launch after this one
                                if (left < K) want = __builtin_amdgcn_readfirstlane(c) + (uint32_t)(left + 1);
                            }
                            if ((int32_t)(f1 - want) < 0) {
                                ok = stream_wait(ctr, kCtrFormed, want, l.wait_polls);
                                if (!ok) neutralize();
                            }
                            lds_order();
                        }
                        const FastBulk b = nb;
                        const uint4 u = u_next;
                        auto work = [&](int j) {
                            if (j == 0) {
                                const uint32_t slot = rb + (uint32_t)((w + 1) % W) * 32u;   // dword after this one
                                u_next = lds_ld4(slot);
                                const uint4 m = lds_ld4(slot + 16u);
                                nb = FastBulk{0, m.x, m.y, m.z, m.w};
                            }
                        };
                        // the previous dword's flips go into the lattice; after a
                        // batch's last dword, and after a row's first dword (which
                        // the row's last batch needs), the walker reports its progress
                        auto done = [&](uint32_t fp) {
                            lds_xor(apend, fp);
                            if (q == 0 || w == 1) {
                                lds_order();
                                lds_st_sync(ctr + kCtrDone, c * (uint32_t)B + (uint32_t)q);
                            }
                        };
                        fpend = walk_dword_stream(st, b, nb, u, fpend, work, done);
                        apend = vcur + 4u * (uint32_t)w;
                        if (q == B - 1) ++c;
                    }
                    if (y == L - 1 && l.record != kRecNone) {
                        const uint32_t Rk = st.acc ? st.C : st.R;
                        int bin = 2 * ((int32_t)(Rk - tab0) / (int32_t)RB);
                        bin = min(max(bin, 0), p.nbins - 1);   // in range even after an abort
                        const int64_t cidx = (int64_t)bin * p.C + it.chain0 + lane;
                        g_i32 *h = (g_i32 *)p.hist;
                        h[cidx] += 1;
                        if (l.record == kRecProd) {
                            g_i64 *sab = (g_i64 *)p.sabs;
                            int ones = 0;
                            for (int dd = 0; dd < NW; ++dd) ones += __builtin_popcount(lds_ld(sb + 4u * dd));
                            // the last dword's flips are still pending
                            const uint32_t old = lds_ld(apend);
                            const uint32_t fl = fpend | (st.acc ? 0x01000000u : 0u);
                            ones += __builtin_popcount(old ^ fl) - __builtin_popcount(old);
                            const int m = 2 * ones - L * L;
                            sab[cidx] += (int64_t)(m < 0 ? -m : m);
                        }
                    }
                }
            }
            lds_xor(apend, fpend | (st.acc ? 0x01000000u : 0u));
            const uint32_t Rk = st.acc ? st.C : st.R;
            ((g_i32 *)p.k)[it.chain0 + lane] = 2 * ((int32_t)(Rk - tab0) / (int32_t)RB);
            int ones = 0;
            for (int dd = 0; dd < NW; ++dd) ones += __builtin_popcount(lds_ld(sb + 4u * dd));
            ((g_i32 *)p.m)[it.chain0 + lane] = 2 * ones - L * L;
        }
    } else {
        // producer wave i: batch bb of every sweep with bb = i mod np; lane r
        // forms the record of chain r / B, dword r mod B of the batch (a wave's
        // 64 lanes cover a batch: stream_ising admits at most 16 chains)
        const int i = wave - 1;
        const int r = lane;
        const bool has = r < nch * B;
        const int cc = r / B, qq = r - cc * B;
        const uint32_t lb = spin0 + (uint32_t)(cc * P) * 4u;
        const uint32_t rbp = ring0 + (uint32_t)cc * RS;
        bool ok = true;
        for (int s = 0; s < n_sweeps && ok; ++s) {
            const uint32_t sweep = sweep0 + (uint32_t)s;
            for (int bb = i; bb < BPS; bb += np) {
                const uint32_t c = (uint32_t)s * (uint32_t)BPS + (uint32_t)bb;   // batch since the launch began
                const int y = bb / BPR, w0 = (bb - y * BPR) * B;
                const int x = w0 + qq;
                // everything that does not depend on the walker first: the random
                // words, and the counts over the old left, right and lower
                // neighbours (the right neighbour of a row's last site, the row's
                // first site of this sweep, excepted).  These dwords hold their
                // previous sweep's final values: the walker updates them only after
                // this batch is published, and it finished their previous sweep
                // (and, below the last row, row 0 of this sweep) long before this
                // wave's previous batch could be formed.
                const uint32_t rowb = lb + (uint32_t)(y * W) * 4u;
                uint4 u = make_uint4(0, 0, 0, 0);
                uint32_t cur = 0;
                uint2 pre = make_uint2(0, 0);
                if (has) {
                    const uint4 v = philox4x32_10((uint32_t)(y * W + x), sweep, (uint32_t)(it.chain0 + cc), 0u,
                                                  p.seed_lo, p.seed_hi);
                    u = make_uint4(min(v.x, 0xFFFFFFFEu), min(v.y, 0xFFFFFFFEu), min(v.z, 0xFFFFFFFEu),
                                   min(v.w, 0xFFFFFFFEu));
                    cur = lds_ld(rowb + 4u * (uint32_t)x);
                    const uint32_t prv = lds_ld(rowb + 4u * (uint32_t)(x == 0 ? W - 1 : x - 1));
                    const uint32_t nxt = lds_ld(rowb + 4u * (uint32_t)(x + 1 == W ? x : x + 1));
                    const uint32_t dn = lds_ld(lb + (uint32_t)((y + 1 == L ? 0 : y + 1) * W + x) * 4u);
                    pre = ising_pre(cur, prv, nxt, dn, x == 0, x + 1 == W);
                }
                // then the walker must have finished (y-1, w0+B-1) and, for a
                // row's last batch, (y, 0)
                const uint32_t g0 = c * (uint32_t)B;   // the batch's first dword since the launch began
                const uint32_t want = (w0 + B == W) ? g0 - (uint32_t)w0 + 1u : g0 + (uint32_t)(B - W);
                if (!stream_wait(ctr, kCtrDone, want, l.wait_polls)) {
                    ok = false;
                    break;
                }
                if (has) {
                    // the row above as this sweep left it
                    const uint32_t xu = cur ^ lds_ld(lb + (uint32_t)((y == 0 ? L - 1 : y - 1) * W + x) * 4u);
                    uint32_t d0 = pre.x + xu, d1 = pre.y + xu;
                    if (x + 1 == W) {
                        // right neighbour of the row's last site: the row's first site, this sweep
                        const uint32_t cr = (cur ^ (lds_ld(rowb) << 24)) & 0xFF000000u;
                        d0 += cr;
                        d1 += cr;
                    }
                    FastBulk fb;
                    bulk_cols<false>(BulkDiff{cur, d0, d1}, fb);
                    bulk_steps<false>(BulkDiff{cur, d0, d1}, fb);
                    const uint32_t slot = rbp + (uint32_t)x * 32u;
                    lds_st4(slot, u);
                    lds_st4(slot + 16u, make_uint4(fb.a0, fb.a1, fb.e0, fb.e1));
                }
                // publish in order: after batch c - 1 (formed by the previous wave)
                if (!stream_wait(ctr, kCtrFormed, c, l.wait_polls)) {
                    ok = false;
                    break;
                }
                if (lane == 0) lds_st_sync(ctr + kCtrFormed, c + 1u);
            }
        }
    }
    __syncthreads();
    if (tid == 0 && lds_ld_sync(ctr + kCtrAbort)) __hip_atomic_fetch_or(l.status, kStatusWaitExpired, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const uint32_t v = lds_ld(spin0 + (uint32_t)(c * P + d) * 4u);
        g_u8 *g = (g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        g[0] = (uint8_t)v;
        g[p.C] = (uint8_t)(v >> 8);
        g[2 * (int64_t)p.C] = (uint8_t)(v >> 16);
        g[3 * (int64_t)p.C] = (uint8_t)(v >> 24);
    }
}

// ------------------------------------------------------------------ packed Ising walker
//
// At L = 64 a byte per spin is 4 KB per chain: with the 80 KB table only 16
// chains fit in LDS, so a walker wave would run with a quarter of its lanes.
// Here each lattice is kept as bits (bit x of dwords y*L/32 .. y*L/32 + L/32-1
// is site (x, y)) and the byte-wise walker above reads a ring of four unpacked
// rows per lane.  While row y is updated, the ring holds row y-1 (already
// updated), row y (updated in place, a dword at a time) and row y+1 (old), and
// row y+2 is unpacked into the fourth slot, one dword per updated dword.  The
// flips are collected as one nibble per dword and xored into the packed row
// at the end of each chunk of 32 sites (one bit dword).  Rows wrap modulo L,
// so at row L-2 the already updated row 0 is unpacked for the next sweep.
// Random words come in chunks of 32 sites.  The site order, random words and
// acceptance rule are those of the byte walker.
//
// Compact table (L = 96, 128, where the 32-bit table would not leave room for
// the lattices).  For rows kk and kk+j (j = 1, 2) the two thresholds are
// T(kk -> kk+j) and T(kk+j -> kk), computed from lnW[kk+j] - lnW[kk] and its
// exact negative, so at least one of them is the "always" value.  One u16
// holds the other: bit 14 set when the move down (kk+j -> kk) is the one that
// can be rejected, bits 0..13 the top 14 bits of its threshold.  The entry of
// pair (kk, kk+j) sits at byte 4 kk + 2 j (after a 2-byte pad), so a move by
// d rows from row kk reads byte 4 kk + 2 d whatever the sign of d.  The walker
// decodes the entry per candidate by xoring bit 14 for a move down (making an
// up-rejectable entry >= 0x4000, i.e. always) and bit 15 for a move that keeps
// k (always), and compares it with the top 14 bits a of the clamped draw:
// a < t accepts, a > t rejects, and a == t (about one site in 2^14) cannot be
// decided from the prefix.  A dword with such a site is redone exactly: the
// full threshold comes from the 32-bit table in HBM and the draw is drawn
// again from the generator.  Every decision therefore equals the 32-bit rule.

template <int V>
struct IntConst {
    static constexpr int value = V;
};

__device__ __forceinline__ uint32_t spread_nibble(uint32_t n) {
    // bits 0..3 of n into bits 0, 8, 16, 24 (the partial products never overlap)
    return __umul24(n, 0x00204081u) & 0x01010101u;
}

typedef __attribute__((address_space(3))) uint16_t lds_u16;
__device__ __forceinline__ uint32_t lds_ld16(uint32_t a) { return *(const lds_u16 *)(size_t)a; }

// Compact entry of the pair (kk, kk+j) from the two 32-bit thresholds.
__device__ __forceinline__ uint16_t compact_entry(uint32_t t_up, uint32_t t_down) {
    if (t_up != 0xFFFFFFFFu) return (uint16_t)(t_up >> 18);
    if (t_down != 0xFFFFFFFFu) return (uint16_t)(0x4000u | (t_down >> 18));
    return 0x3FFFu;   // both always: an up move compares with the largest prefix, a tie decides exactly
}

// Bulk of one dword for the compact table: besides the old spins, the column
// codes (2 d + 4, d = 2 - D the row move), the row steps (4 d bytes) and the
// decode codes (byte 1 of the xor: 0x40 for a move down, 0x80 for d = 0) of
// both candidates.
struct CompactBulk {
    uint32_t cur, a0, a1, e0, e1, z0, z1;
};

__device__ __forceinline__ void compact_cols(const BulkDiff &d, CompactBulk &b) {
    b.cur = d.cur;
    b.a0 = __builtin_amdgcn_perm(0u, 0x02040608u, d.d0);   // D = 0..4 -> 8, 6, 4, 2, 0
    b.a1 = __builtin_amdgcn_perm(0u, 0x02040608u, d.d1);
}
__device__ __forceinline__ void compact_steps(const BulkDiff &d, CompactBulk &b) {
    b.e0 = __builtin_amdgcn_perm(0xF8u, 0xFC000408u, d.d0);   // 8, 4, 0, -4, -8
    b.e1 = __builtin_amdgcn_perm(0xF8u, 0xFC000408u, d.d1);
    b.z0 = __builtin_amdgcn_perm(0x40u, 0x40800000u, d.d0);   // 0, 0, 0x80, 0x40, 0x40
    b.z1 = __builtin_amdgcn_perm(0x40u, 0x40800000u, d.d1);
}
__device__ __forceinline__ int32_t row_step(const CompactBulk &b, bool left_flipped, int j) {
    return left_flipped ? sbyte(b.e1, j) : sbyte(b.e0, j);
}

// Walker state of the compact walkers: as FastState, with the previous
// site's outcome in a full word (a struct without padding stays in registers
// through the copies the exact redo makes).
struct CompactState {
    uint32_t R, C, tA, tB, acc;
};

// t with its byte 1 xored with byte j of codes (the compact walkers' decode of
// a table entry), in one SDWA instruction; j is a compile-time constant after
// unrolling.
__device__ __forceinline__ uint32_t xor_byte1(uint32_t t, uint32_t codes, int j) {
    uint32_t r = t;
    switch (j) {
    case 0:
        asm("v_xor_b32_sdwa %0, %1, %2 dst_sel:BYTE_1 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_1 src1_sel:BYTE_0"
            : "+v"(r) : "v"(t), "v"(codes));
        break;
    case 1:
        asm("v_xor_b32_sdwa %0, %1, %2 dst_sel:BYTE_1 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_1 src1_sel:BYTE_1"
            : "+v"(r) : "v"(t), "v"(codes));
        break;
    case 2:
        asm("v_xor_b32_sdwa %0, %1, %2 dst_sel:BYTE_1 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_1 src1_sel:BYTE_2"
            : "+v"(r) : "v"(t), "v"(codes));
        break;
    default:
        asm("v_xor_b32_sdwa %0, %1, %2 dst_sel:BYTE_1 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_1 src1_sel:BYTE_3"
            : "+v"(r) : "v"(t), "v"(codes));
        break;
    }
    return r;
}

// Walker state and flip record of an exactly recomputed dword: R, C, tA, tB,
// acc (0/1) and the flip record, as a vector so that the out-of-line redo
// returns it in registers (a returned struct can be placed in memory and drag
// the walker's state there with it).
typedef unsigned int u32x8 __attribute__((ext_vector_type(8)));
typedef u32x8 RedoResult;
__device__ __forceinline__ RedoResult redo_result(uint32_t R, uint32_t C, uint32_t tA, uint32_t tB, bool acc,
                                                  uint32_t f) {
    RedoResult r;
    r.s0 = R;
    r.s1 = C;
    r.s2 = tA;
    r.s3 = tB;
    r.s4 = acc ? 1u : 0u;
    r.s5 = f;
    r.s6 = 0u;
    r.s7 = 0u;
    return r;
}

// Exact recomputation of one dword of the compact walker (rare: some site of
// the dword drew a prefix equal to its entry's).  From the state at the
// dword's start (rows R, C and the previous site's outcome acc), each site is
// decided from its decoded entry where the prefix decides, else from the full
// threshold T32[kk][d + 2] in HBM and the site's draw regenerated from the
// generator (block blk of the sweep, word j).  Returns the state after the
// dword, with the next dword's first entries read for both outcomes (column
// codes na0, na1), and the flip record (bit j for an accepted site j).  Kept
// out of line so that the walker's state stays in registers on the fast path.
__device__ __noinline__ RedoResult redo_compact_dword(uint32_t R, uint32_t C, uint32_t acc_in, uint32_t ca0,
                                                      uint32_t ca1, uint32_t ce0, uint32_t ce1, uint32_t cz0,
                                                      uint32_t cz1, uint32_t na0, uint32_t na1, uint32_t u0,
                                                      uint32_t u1, uint32_t u2, uint32_t u3, uint32_t tab0,
                                                      const uint32_t *table, uint32_t blk, uint32_t sweep,
                                                      uint32_t chain, uint32_t seed_lo, uint32_t seed_hi) {
    const g_u32 *T = (const g_u32 *)table;
    bool acc = acc_in != 0;
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t Rj = acc ? C : R;
        const int32_t step = acc ? sbyte(ce1, j) : sbyte(ce0, j);
        const uint32_t code = acc ? ubyte(ca1, j) : ubyte(ca0, j);
        const uint32_t z = acc ? ubyte(cz1, j) : ubyte(cz0, j);
        const uint32_t t = lds_ld16(Rj + code) ^ (z << 8);
        const uint32_t a = (j == 0) ? u0 : (j == 1) ? u1 : (j == 2) ? u2 : u3;
        bool ok;
        if (a != t) {
            ok = a < t;
        } else {
            // full threshold: row kk = (Rj + 4 - tab0) / 4, column d + 2 with d = step / 4
            const int kk = (int)((Rj + 4u - tab0) >> 2);
            const uint32_t Tf = T[kk * 5 + 2 + (step >> 2)];
            const uint4 b = philox4x32_10(blk, sweep, chain, 0u, seed_lo, seed_hi);
            const uint32_t uu = (j == 0) ? b.x : (j == 1) ? b.y : (j == 2) ? b.z : b.w;
            ok = min(uu, 0xFFFFFFFEu) < Tf;
        }
        R = Rj;
        C = Rj + (uint32_t)step;
        acc = ok;
        if (ok) f |= 1u << j;
    }
    return redo_result(R, C, lds_ld16(R + na0), lds_ld16(C + na1), acc, f);
}

// The four sites of one dword against the compact table; as walk_dword, plus
// the decode of each candidate's entry and the detection of undecidable
// draws.  If any site of the dword drew a == t, the whole dword is recomputed
// exactly from the state at its start (redo_compact_dword; ex holds the
// table, the Philox block of the dword and the generator's key).
// r + byte 0 of codes in one SDWA instruction (the compiler otherwise masks the
// byte with a separate instruction when the word also feeds other uses).
__device__ __forceinline__ uint32_t add_byte0(uint32_t r, uint32_t codes) {
    uint32_t d;
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(d) : "v"(r), "v"(codes));
    return d;
}

struct CompactExact {
    uint32_t tab0;
    const uint32_t *table;
    uint32_t blk, sweep, chain, seed_lo, seed_hi;
};

__device__ __forceinline__ RedoResult compact_redo(uint32_t R0, uint32_t C0, bool acc0, const CompactBulk &b,
                                                   const CompactBulk &nb, const uint4 &u, const CompactExact &ex) {
    return redo_compact_dword(R0, C0, acc0 ? 1u : 0u, b.a0, b.a1, b.e0, b.e1, b.z0, b.z1,
                              __builtin_amdgcn_ubfe(nb.a0, 0u, 8u), __builtin_amdgcn_ubfe(nb.a1, 0u, 8u), u.x, u.y,
                              u.z, u.w, ex.tab0, ex.table, ex.blk, ex.sweep, ex.chain, ex.seed_lo, ex.seed_hi);
}

template <class Bulk, uint32_t FLIP, int STRIDE, class Work>
__device__ __forceinline__ uint32_t walk_dword_compact(CompactState &s, const Bulk &b, const Bulk &nb, const uint4 &u,
                                                       Work &&work, const CompactExact &ex) {
    const uint32_t R0 = s.R, C0 = s.C;   // the state at the dword's start, for an exact redo
    const bool acc0 = s.acc != 0u;
    bool acc = acc0;                     // the previous site's outcome, as a lane mask
    uint32_t f = 0;
    bool tie = false;
    bool eq = false;   // the previous site's tie, folded in a site later (its compare has long finished)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t Rj = acc ? s.C : s.R;
        const uint32_t Cj = Rj + (uint32_t)row_step(b, acc, j);
        uint32_t adA, adB;
        if (j < 3) {
            adA = Rj + ubyte(b.a0, j + 1);
            adB = Cj + ubyte(b.a1, j + 1);
        } else {
            adA = add_byte0(Rj, nb.a0);
            adB = add_byte0(Cj, nb.a1);
        }
        const uint32_t nA = lds_ld16(adA);
        const uint32_t nB = lds_ld16(adB);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t tA = xor_byte1(s.tA, b.z0, j);
        const uint32_t tB = xor_byte1(s.tB, b.z1, j);
        tie |= eq;
        const uint32_t tj = acc ? tB : tA;
        const uint32_t uj = (j == 0) ? u.x : (j == 1) ? u.y : (j == 2) ? u.z : u.w;
        acc = uj < tj;
        eq = uj == tj;
        s.R = Rj;
        s.C = Cj;
        s.tA = nA;
        s.tB = nB;
        __builtin_amdgcn_sched_barrier(0);
        work(j);
        __builtin_amdgcn_sched_barrier(0);
        f |= acc ? (FLIP << (STRIDE * j)) : 0u;
        __builtin_amdgcn_sched_barrier(0);
    }
    tie |= eq;
    s.acc = acc ? 1u : 0u;
    if (__builtin_amdgcn_ballot_w64(tie) != 0u) {
        // rare: the whole wave redoes the dword exactly (the redo agrees with
        // the fast path wherever the prefixes decide) and writes the flip
        // record in the walker's format (FLIP << STRIDE j for an accepted site j)
        const RedoResult r = compact_redo(R0, C0, acc0, b, nb, u, ex);
        s.R = r.s0;
        s.C = r.s1;
        s.tA = r.s2;
        s.tB = r.s3;
        s.acc = r.s4;
        f = r.s5;
    }
    return f;
}

template <int L, bool COMPACT>
__device__ __forceinline__ void run_ising_packed(const ProbDev &p, const WorkItem &it, char *lds, const SweepLaunch &l,
                                 uint32_t sweep0, const LdsPlan &plan) {
    constexpr int W = L / 4;                    // byte dwords per row
    constexpr int BPR = L / 32;                 // bit dwords per row = chunks per row
    constexpr int NB = L * BPR;                 // bit dwords per lattice
    constexpr int CDW = kPackedChunkDwords;     // byte dwords per chunk (one bit dword)
    constexpr int NCH = L * BPR;                // chunks per sweep
    constexpr int PB = packed_bit_stride(L), PR = packed_row_stride(L);
    constexpr uint32_t RB = COMPACT ? 4u : 20u;   // table row bytes
    static_assert(W == CDW * BPR, "packed walker shape");
    using Bulk = typename std::conditional<COMPACT, CompactBulk, FastBulk>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int nch = it.nchains;
    const bool active = (wave == 0) && (lane < nch);
    const uint32_t lbase = (uint32_t)(size_t)(__attribute__((address_space(3))) char *)lds;
    const uint32_t tab0 = lbase + (uint32_t)plan.off_tab;
    const uint32_t bits0 = lbase + (uint32_t)plan.off_spin;
    const uint32_t rows0 = lbase + (uint32_t)plan.off_rows;
    const uint32_t ring0 = lbase + (uint32_t)plan.off_ring;
    const uint32_t ringbuf = (uint32_t)nch * (CDW + 1) * 16u;
    // compact rows: entry (kk, j) sits at tab0 + 4 kk + 2 j (tab0 holds the
    // pad); R = tab0 + 4 kk - 4, so that R + (2 d + 4) is the entry a move by
    // d rows reads, for d = -2..2 (d = 0 reads a valid entry it ignores)
    auto row_of = [&](int kk) -> uint32_t { return COMPACT ? tab0 + 4u * (uint32_t)kk - 4u : tab0 + RB * (uint32_t)kk; };
    auto kk_of = [&](uint32_t R) -> int { return COMPACT ? (int)((R + 4u - tab0) >> 2) : (int)((R - tab0) / RB); };

    if constexpr (COMPACT) {
        // the pair table, from the 32-bit table in HBM (rows kk, columns dk/2 + 2)
        const g_u32 *T = (const g_u32 *)p.table;
        const int rows = p.N + 1;
        if (tid == 0) *(lds_u16 *)(size_t)tab0 = 0;
        for (int e = tid; e < 2 * rows; e += nthreads) {
            const int kk = e >> 1, j = (e & 1) + 1;
            uint16_t v = 0;
            if (kk + j < rows) v = compact_entry(T[kk * 5 + 2 + j], T[(kk + j) * 5 + 2 - j]);
            *(lds_u16 *)(size_t)(tab0 + 2u + 2u * (uint32_t)e) = v;
        }
    }
    // stage the lattice as bits: dword d of lane c holds sites 32d..32d+31
    for (int j = tid; j < NB * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const g_u8 *g = (const g_u8 *)p.spins + (int64_t)(32 * d) * p.C + it.chain0 + c;
        uint32_t v = 0;
        for (int b = 0; b < 32; ++b) v |= (uint32_t)g[(int64_t)b * p.C] << b;
        lds_st(bits0 + (uint32_t)(c * PB + d) * 4u, v);
    }
    __syncthreads();

    const uint32_t bl = bits0 + (uint32_t)(lane * PB) * 4u;   // this lane's bits
    const uint32_t rl = rows0 + (uint32_t)(lane * PR) * 4u;   // this lane's row ring
    const uint32_t rb = ring0 + (uint32_t)(lane * (CDW + 1)) * 16u;
    const uint32_t chain = (uint32_t)(it.chain0 + lane);
    auto slot = [&](int y) -> uint32_t { return rl + (uint32_t)((y & 3) * W) * 4u; };
    // byte dword w of row y, unpacked from the bits
    auto unpacked = [&](int y, int w) -> uint32_t {
        const uint32_t word = lds_ld(bl + (uint32_t)(BPR * y + (w >> 3)) * 4u);
        return spread_nibble(__builtin_amdgcn_ubfe(word, 4u * (uint32_t)(w & 7), 4u));
    };
    auto read_t = [&](uint32_t a) -> uint32_t { return COMPACT ? lds_ld16(a) : lds_ld(a); };
    auto make_bulk = [&](const BulkDiff &d, Bulk &b) {
        if constexpr (COMPACT) {
            compact_cols(d, b);
            compact_steps(d, b);
        } else {
            bulk_cols<false>(d, b);
            bulk_steps<false>(d, b);
        }
    };

    using State = typename std::conditional<COMPACT, CompactState, FastState>::type;
    State st{};
    Bulk nb{};
    if (active) {
        // ring: rows L-1, 0, 1 (row 2 is unpacked while row 0 is updated)
        for (int w = 0; w < W; ++w) {
            lds_st(slot(L - 1) + 4u * w, unpacked(L - 1, w));
            lds_st(slot(0) + 4u * w, unpacked(0, w));
            lds_st(slot(1) + 4u * w, unpacked(1, w));
        }
        const int k = ((const g_i32 *)p.k)[it.chain0 + lane];
        st.R = row_of(k >> 1);
        st.C = st.R;
        const uint32_t r0 = slot(0);
        make_bulk(bulk_diff<true>(bulk_sums(lds_ld(r0), lds_ld(r0 + 4 * (W - 1)), lds_ld(r0 + 4), lds_ld(slot(L - 1)),
                                            lds_ld(slot(1)))),
                  nb);
        st.tA = read_t(st.R + ubyte(nb.a0, 0));
        st.tB = st.tA;
    }

    // producers: chunk t covers dwords (t mod NCH) * CDW .. + CDW - 1 of sweep t / NCH;
    // the compact walker receives the top 14 bits of each clamped draw
    auto produce = [&](int t) __attribute__((always_inline)) {
        const int sw = t / NCH;
        const uint32_t sweep = sweep0 + (uint32_t)sw;
        const int blk0 = (t - sw * NCH) * CDW;
        const uint32_t buf = ring0 + (uint32_t)(t & 1) * ringbuf;
        const int total = CDW * nch;
        for (int w = tid - 64; w < total; w += nthreads - 64) {
            const int c = w / CDW, q = w - c * CDW;
            const uint4 b = philox4x32_10((uint32_t)(blk0 + q), sweep, (uint32_t)(it.chain0 + c), 0u, p.seed_lo,
                                          p.seed_hi);
            uint4 o = make_uint4(min(b.x, 0xFFFFFFFEu), min(b.y, 0xFFFFFFFEu), min(b.z, 0xFFFFFFFEu),
                                 min(b.w, 0xFFFFFFFEu));
            if (COMPACT) o = make_uint4(o.x >> 18, o.y >> 18, o.z >> 18, o.w >> 18);
            lds_st4(buf + (uint32_t)(c * (CDW + 1) + q) * 16u, o);
        }
    };

    const int total_chunks = NCH * l.n_sweeps;
    if (wave > 0) produce(0);
    __syncthreads();
    uint4 u_next = make_uint4(0, 0, 0, 0);
    // One chunk of 32 sites (bit dword H of row y); H is a compile-time
    // constant so that every dword index, LDS offset and flip word below is
    // fixed at compile time.
    auto walk_chunk = [&](auto HC, int t) __attribute__((always_inline)) {
        constexpr int H = decltype(HC)::value;
        const int sw = t / NCH;
        const int y = (t - sw * NCH) / BPR;
        const uint32_t sweep = sweep0 + (uint32_t)sw;
        const uint32_t ub = rb + (uint32_t)(t & 1) * ringbuf;
        const uint32_t vcur = slot(y), vnc = slot(y + 1), vnd = slot(y + 2), vup = slot(y + 3);
        const int y2 = (y + 2 == L) ? 0 : (y + 2 == L + 1) ? 1 : y + 2;   // row unpacked into vnd
        const uint32_t word_y2 = lds_ld(bl + (uint32_t)(BPR * y2 + H) * 4u);   // its chunk H
        uint32_t nxt_cache = lds_ld(vcur + 4 * (8 * H + 1));
        uint32_t fl = 0;   // flips of this chunk, one bit per site
#pragma unroll
        for (int q = 0; q < CDW; ++q) {
            const int w = 8 * H + q;
            const Bulk b = nb;
            const uint4 u = (q == 0) ? lds_ld4(ub) : u_next;
            // the next dword's bulk (and one dword of row y+2 into the ring),
            // in pieces between this dword's sites
            uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0;
            BulkSums ns{0, 0, 0};
            BulkDiff nd{0, 0, 0};
            auto work = [&](int j) __attribute__((always_inline)) {
                if (j == 0) {
                    if (q + 1 < CDW) u_next = lds_ld4(ub + (uint32_t)(q + 1) * 16u);
                    if (w + 1 < W) {
                        q0 = nxt_cache;
                        q1 = b.cur;
                        q2 = lds_ld(vcur + 4 * ((w + 2 < W) ? w + 2 : 0));
                        q3 = lds_ld(vup + 4 * (w + 1));
                        q4 = lds_ld(vnc + 4 * (w + 1));
                    } else {
                        q0 = lds_ld(vnc);
                        q1 = lds_ld(vnc + 4 * (W - 1));
                        q2 = lds_ld(vnc + 4);
                        q3 = lds_ld(vcur);
                        q4 = lds_ld(vnd);
                    }
                } else if (j == 1) {
                    ns = bulk_sums(q0, q1, q2, q3, q4);
                    if (w + 1 < W) nxt_cache = q2;
                } else if (j == 2) {
                    nd = (w + 1 < W) ? bulk_diff<false>(ns) : bulk_diff<true>(ns);
                    if constexpr (COMPACT) compact_cols(nd, nb);
                    else bulk_cols<false>(nd, nb);
                } else {
                    if constexpr (COMPACT) compact_steps(nd, nb);
                    else bulk_steps<false>(nd, nb);
                    // row y+2 into the ring (the slot of row y-2, no longer read)
                    lds_st(vnd + 4u * w, spread_nibble(__builtin_amdgcn_ubfe(word_y2, 4u * (uint32_t)q, 4u)));
                }
            };
            uint32_t nib;
            if constexpr (COMPACT) {
                const CompactExact ex{tab0, p.table, (uint32_t)(y * W + w), sweep, chain, p.seed_lo, p.seed_hi};
                nib = walk_dword_compact<CompactBulk, 1u, 1>(st, b, nb, u, work, ex);
            } else {
                nib = walk_dword<FastBulk, 1u, 1>(st, b, nb, u, work);
            }
            lds_st(vcur + 4 * w, b.cur ^ spread_nibble(nib));
            fl |= nib << (4 * q);
        }
        // chunk done: fold its flips into the bits of row y
        const uint32_t a0 = bl + (uint32_t)(BPR * y + H) * 4u;
        lds_st(a0, lds_ld(a0) ^ fl);
        if (H == BPR - 1 && y == L - 1 && l.record != kRecNone) {
            const uint32_t Rk = st.acc ? st.C : st.R;
            const int k = 2 * kk_of(Rk);
            const int64_t cidx = (int64_t)k * p.C + it.chain0 + lane;
            g_i32 *hh = (g_i32 *)p.hist;
            hh[cidx] += 1;
            if (l.record == kRecProd) {
                int ones = 0;
                for (int dd = 0; dd < NB; ++dd) ones += __builtin_popcount(lds_ld(bl + 4u * dd));
                const int m = 2 * ones - L * L;
                g_i64 *s = (g_i64 *)p.sabs;
                s[cidx] += (int64_t)(m < 0 ? -m : m);
            }
        }
    };
    // chunk H of a row, then the barrier that hands the next chunk's random
    // words over
    auto chunk_pass = [&](auto HC, int t) __attribute__((always_inline)) {
        constexpr int H = decltype(HC)::value;
        if (wave == 0) {
            if (active) walk_chunk(IntConst<H>{}, t + H);
        } else if (t + H + 1 < total_chunks) {
            produce(t + H + 1);
        }
        __syncthreads();
    };
    static_assert(BPR >= 2 && BPR <= 4, "packed walker rows of 2 to 4 chunks");
    for (int t = 0; t < total_chunks; t += BPR) {
        chunk_pass(IntConst<0>{}, t);
        chunk_pass(IntConst<1>{}, t);
        if constexpr (BPR > 2) chunk_pass(IntConst<2>{}, t);
        if constexpr (BPR > 3) chunk_pass(IntConst<3>{}, t);
    }

    if (active) {
        const uint32_t Rk = st.acc ? st.C : st.R;
        ((g_i32 *)p.k)[it.chain0 + lane] = 2 * kk_of(Rk);
        int ones = 0;
        for (int dd = 0; dd < NB; ++dd) ones += __builtin_popcount(lds_ld(bl + 4u * dd));
        ((g_i32 *)p.m)[it.chain0 + lane] = 2 * ones - L * L;
    }
    __syncthreads();
    // bits back to bytes in HBM
    for (int j = tid; j < NB * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const uint32_t v = lds_ld(bits0 + (uint32_t)(c * PB + d) * 4u);
        g_u8 *g = (g_u8 *)p.spins + (int64_t)(32 * d) * p.C + it.chain0 + c;
        for (int b = 0; b < 32; ++b) g[(int64_t)b * p.C] = (uint8_t)((v >> b) & 1u);
    }
}

// ------------------------------------------------------------------ streamed Ising walker on bit lattices
//
// The packed walker above unpacks rows, forms every dword's bulk and, at L =
// 96 and 128, decodes the compact table in one wave: about 110 (L = 64) and
// 139 (L = 96, 128) cycles per site.  Here, as in the streamed Ising and
// Potts walkers, the helper waves form each dword's complete record from the
// bit lattice once the walker has left the row above (the draws, or their
// 14-bit prefixes on the compact table, then column codes, row steps and,
// compact, decode codes of both candidates), and the walker only decides
// sites and xors each dword's flips, as a nibble, into the bit lattice.  On
// the compact table ties with the 14-bit entries are redone exactly
// (redo_compact_dword).

// The four sites of one dword: as walk_dword_pstream (compact decode, ties
// folded a site later), with one flip bit per site: bit b0 + j for site j.
// Returns the bits of sites 0..2; site 3's outcome is s.acc.
template <class Work, class Done>
__device__ __forceinline__ uint32_t walk_dword_cstream(FastState &s, const uint4 &m, const uint4 &z, const uint4 &nm,
                                                       const uint4 &u, uint32_t b0, bool &tie, Work &&work,
                                                       Done &&done) {
    uint32_t f = 0;
    bool eq = false;   // the previous site's tie, folded in a site later
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool acc = s.acc;
        const uint32_t Rj = acc ? s.C : s.R;
        const uint32_t Cj = Rj + (uint32_t)(acc ? sbyte(m.w, j) : sbyte(m.z, j));
        uint32_t adA, adB;
        if (j < 3) {
            adA = Rj + ubyte(m.x, j + 1);
            adB = Cj + ubyte(m.y, j + 1);
        } else {
            adA = add_byte0(Rj, nm.x);
            adB = add_byte0(Cj, nm.y);
        }
        const uint32_t nA = lds_ld16(adA);
        const uint32_t nB = lds_ld16(adB);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t tA = xor_byte1(s.tA, z.x, j);
        const uint32_t tB = xor_byte1(s.tB, z.y, j);
        tie |= eq;
        const uint32_t tj = acc ? tB : tA;
        const uint32_t uj = (j == 0) ? u.x : (j == 1) ? u.y : (j == 2) ? u.z : u.w;
        s.acc = uj < tj;
        eq = uj == tj;
        s.R = Rj;
        s.C = Cj;
        s.tA = nA;
        s.tB = nB;
        __builtin_amdgcn_sched_barrier(0);
        if (j == 0) {
            done(acc);
        } else {
            f |= acc ? (1u << (b0 + (uint32_t)(j - 1))) : 0u;
            asm volatile("" : "+v"(f));   // recorded here, not at the end of the dword
        }
        work(j);
        __builtin_amdgcn_sched_barrier(0);
    }
    tie |= eq;
    return f;
}

// The four sites of one dword on the 32-bit table (Ising L = 64): as
// walk_dword_stream, with one flip bit per site (bit b0 + j for site j).
template <class Work, class Done>
__device__ __forceinline__ uint32_t walk_dword_bstream(FastState &s, const uint4 &m, const uint4 &nm, const uint4 &u,
                                                       uint32_t b0, Work &&work, Done &&done) {
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool acc = s.acc;
        const uint32_t Rj = acc ? s.C : s.R;
        const uint32_t Cj = Rj + (uint32_t)(acc ? sbyte(m.w, j) : sbyte(m.z, j));
        uint32_t adA, adB;
        if (j < 3) {
            adA = Rj + ubyte(m.x, j + 1);
            adB = Cj + ubyte(m.y, j + 1);
        } else {
            adA = add_byte0(Rj, nm.x);
            adB = add_byte0(Cj, nm.y);
        }
        const uint32_t nA = lds_ld(adA);
        const uint32_t nB = lds_ld(adB);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t tj = acc ? s.tB : s.tA;
        const uint32_t uj = (j == 0) ? u.x : (j == 1) ? u.y : (j == 2) ? u.z : u.w;
        s.acc = uj < tj;
        s.R = Rj;
        s.C = Cj;
        s.tA = nA;
        s.tB = nB;
        __builtin_amdgcn_sched_barrier(0);
        if (j == 0) {
            done(acc);
        } else {
            f |= acc ? (1u << (b0 + (uint32_t)(j - 1))) : 0u;
            asm volatile("" : "+v"(f));   // recorded here, not at the end of the dword
        }
        work(j);
        __builtin_amdgcn_sched_barrier(0);
    }
    return f;
}

template <int L, bool COMPACT>
__device__ __forceinline__ void run_ising_cstream(const ProbDev &p, const WorkItem &it, char *lds, const SweepLaunch &l,
                                                  uint32_t sweep0, const LdsPlan &plan) {
    constexpr int W = L / 4;                  // byte dwords (four sites) per row
    constexpr int BPR = L / 32;               // bit dwords per row
    constexpr int NB = L * BPR;               // bit dwords per lattice
    constexpr int PB = packed_bit_stride(L);  // bit dwords between lanes
    constexpr int B = kStreamBatch;
    constexpr int BTR = W / B;                // batches per row
    constexpr int BPS = L * BTR;              // batches per sweep
    constexpr uint32_t RS = cstream_lane_words(L, COMPACT) * 4u;   // ring bytes per lane
    constexpr uint32_t RECB = COMPACT ? 48u : 32u;                 // record bytes
    constexpr int R = cstream_slots(L);                   // record slots per lane: dword x uses slot x mod R
    constexpr int HR = COMPACT ? 2 : 4;                   // records per helper lane and batch (32 or 64 chains)
    static_assert(W % B == 0 && W >= 2 * B + 1 && W % 8 == 0 && R >= 2 * B + 2, "streamed compact Ising walker shape");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int np = nthreads / 64 - 1;         // producer waves
    const int nch = it.nchains;
    const bool active = (wave == 0) && (lane < nch);
    const uint32_t lbase = (uint32_t)(size_t)(__attribute__((address_space(3))) char *)lds;
    const uint32_t tab0 = lbase + (uint32_t)plan.off_tab + (COMPACT ? kCStreamGuard : 0u);
    const uint32_t bits0 = lbase + (uint32_t)plan.off_spin;
    const uint32_t ring0 = lbase + (uint32_t)plan.off_ring;
    const uint32_t ctr = lbase + (uint32_t)plan.off_ctr;   // counters (see kCtrDone)
    // rows kk = k / 2: compact R = tab0 + 4 kk - 4 (see run_ising_packed), else
    // 20 kk (five words); the 32-bit table is already in LDS
    auto row_of = [&](int kk) -> uint32_t { return COMPACT ? tab0 + 4u * (uint32_t)kk - 4u : tab0 + 20u * (uint32_t)kk; };
    auto kk_of = [&](uint32_t R) -> int {
        return COMPACT ? (int)((int32_t)(R + 4u - tab0) >> 2) : (int)((int32_t)(R - tab0) / 20);
    };
    auto read_t = [&](uint32_t a) -> uint32_t { return COMPACT ? lds_ld16(a) : lds_ld(a); };

    if constexpr (COMPACT) {
        // the pair table, from the 32-bit table in HBM (rows kk, columns dk/2 + 2)
        const g_u32 *T = (const g_u32 *)p.table;
        const int rows = p.N + 1;
        if (tid == 0) *(lds_u16 *)(size_t)tab0 = 0;
        for (int e = tid; e < 2 * rows; e += nthreads) {
            const int kk = e >> 1, j = (e & 1) + 1;
            uint16_t v = 0;
            if (kk + j < rows) v = compact_entry(T[kk * 5 + 2 + j], T[(kk + j) * 5 + 2 - j]);
            *(lds_u16 *)(size_t)(tab0 + 2u + 2u * (uint32_t)e) = v;
        }
    }
    // the lattice as bits: dword d of lane c holds sites 32d..32d+31
    for (int j = tid; j < NB * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const g_u8 *g = (const g_u8 *)p.spins + (int64_t)(32 * d) * p.C + it.chain0 + c;
        uint32_t v = 0;
        for (int b = 0; b < 32; ++b) v |= (uint32_t)g[(int64_t)b * p.C] << b;
        lds_st(bits0 + (uint32_t)(c * PB + d) * 4u, v);
    }
    if (tid < kStreamCtrWords) lds_st(ctr + 4u * (uint32_t)tid, 0u);
    __syncthreads();

    const int n_sweeps = l.n_sweeps;
    if (wave == 0) {
        if (active) {
            const uint32_t bl = bits0 + (uint32_t)(lane * PB) * 4u;   // this lane's bits
            const uint32_t rb = ring0 + (uint32_t)lane * RS;          // this lane's records
            const uint32_t chain = (uint32_t)(it.chain0 + lane);
            FastState st{0, 0, 0, 0, false};
            const int k0 = ((const g_i32 *)p.k)[it.chain0 + lane];
            st.R = row_of(k0 >> 1);
            st.C = st.R;
            // After a wait gives up, the walker rewrites its records to reject
            // every move (draws 2^32 - 1, which no threshold exceeds and no
            // 14-bit entry equals; compact code 4, the row's own entry, or
            // column 0; no step, no decode).
            auto neutralize = [&]() {
                const uint32_t a = COMPACT ? 0x04040404u : 0u;
                for (int w = 0; w < R; ++w) {
                    lds_st4(rb + (uint32_t)w * RECB, make_uint4(~0u, ~0u, ~0u, ~0u));
                    lds_st4(rb + (uint32_t)w * RECB + 16u, make_uint4(a, a, 0u, 0u));
                    if (COMPACT) lds_st4(rb + (uint32_t)w * RECB + 32u, make_uint4(0u, 0u, 0u, 0u));
                }
            };
            bool ok = stream_wait(ctr, kCtrFormed, 1u, l.wait_polls);   // batch 0 of the launch
            if (!ok) neutralize();
            uint4 u_next = lds_ld4(rb);
            uint4 nm = lds_ld4(rb + 16u);
            uint4 nz = COMPACT ? lds_ld4(rb + 32u) : make_uint4(0, 0, 0, 0);
            st.tA = read_t(st.R + ubyte(nm.x, 0));
            st.tB = st.tA;
            uint32_t c = 0;        // batches walked before the current one (wraps)
            uint32_t formed = 0;   // batches formed, read a dword before the check
            uint32_t fpend = 0;    // flip bits of sites 0..2 of the last dword walked, not yet in the lattice
            uint32_t apend = bl;   // that dword's bit word (nothing pending before the first dword)
            for (int s = 0; s < n_sweeps && ok; ++s) {
                const uint32_t sweep = sweep0 + (uint32_t)s;
                for (int y = 0; y < L && ok; ++y) {
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const int q = w % B;
                        // in a batch's last dword: batch c + 1 (whose first record this
                        // dword's first site reads), none beyond the launch; the counter
                        // was read a dword earlier
                        if (q == B - 2) formed = lds_ld_sync(ctr + kCtrFormed);
                        if (q == B - 1 && ok) {
                            const uint32_t f1 = __builtin_amdgcn_readfirstlane(formed);
                            const bool last = (y == L - 1 && s + 1 == n_sweeps && w + 1 == W);
                            const uint32_t want = __builtin_amdgcn_readfirstlane(c) + (last ? 1u : 2u);
                            if ((int32_t)(f1 - want) < 0) {
                                ok = stream_wait(ctr, kCtrFormed, want, l.wait_polls);
                                if (!ok) neutralize();
                            }
                            lds_order();
                        }
                        const uint4 m = nm, z = nz;
                        const uint4 u = u_next;
                        auto work = [&](int j) {
                            if (j == 0) {
                                const uint32_t slot = rb + (uint32_t)(((w + 1) % W) % R) * RECB;   // dword after this one
                                u_next = lds_ld4(slot);
                                nm = lds_ld4(slot + 16u);
                                if (COMPACT) nz = lds_ld4(slot + 32u);
                            }
                        };
                        // the previous dword's flips go into the bit lattice (its site 3 is
                        // bit 4 ((w - 1) mod 8) + 3 of its word); after a batch's last dword,
                        // and after a row's first dword (which the row's last batch needs),
                        // the walker reports its progress
                        const uint32_t b3prev = 4u * (uint32_t)((w + 7) % 8) + 3u;
                        auto done = [&](bool acc3) {
                            lds_xor(apend, fpend | (acc3 ? (1u << b3prev) : 0u));
                            if (q == 0 || w == 1) {
                                lds_order();
                                lds_st_sync(ctr + kCtrDone, c * (uint32_t)B + (uint32_t)q);
                            }
                        };
                        uint32_t f;
                        if constexpr (!COMPACT) {
                            f = walk_dword_bstream(st, m, nm, u, 4u * (uint32_t)(w % 8), work, done);
                        } else {
                        const uint32_t R0 = st.R, C0 = st.C;
                        const bool acc0 = st.acc;
                        bool tie = false;
                        f = walk_dword_cstream(st, m, z, nm, u, 4u * (uint32_t)(w % 8), tie, work, done);
                        if (__builtin_amdgcn_ballot_w64(tie) != 0u) {
                            // rare: the whole wave redoes the dword exactly (the redo agrees
                            // with the fast path wherever the prefixes decide); its record
                            // has bit j for an accepted site j; site 3's outcome stays pending
                            const RedoResult r = redo_compact_dword(
                                R0, C0, acc0 ? 1u : 0u, m.x, m.y, m.z, m.w, z.x, z.y, __builtin_amdgcn_ubfe(nm.x, 0u, 8u),
                                __builtin_amdgcn_ubfe(nm.y, 0u, 8u), u.x, u.y, u.z, u.w, tab0, p.table,
                                (uint32_t)(y * W + w), sweep, chain, p.seed_lo, p.seed_hi);
                            st.R = r.s0;
                            st.C = r.s1;
                            st.tA = r.s2;
                            st.tB = r.s3;
                            st.acc = r.s4 != 0u;
                            f = (r.s5 & 7u) << (4u * (uint32_t)(w % 8));
                        }
                        }
                        fpend = f;
                        apend = bl + (uint32_t)(BPR * y + w / 8) * 4u;
                        if (q == B - 1) ++c;
                    }
                    if (y == L - 1 && l.record != kRecNone) {
                        const uint32_t Rk = st.acc ? st.C : st.R;
                        const int bin = min(max(2 * kk_of(Rk), 0), p.nbins - 1);   // in range even after an abort
                        const int64_t cidx = (int64_t)bin * p.C + it.chain0 + lane;
                        ((g_i32 *)p.hist)[cidx] += 1;
                        if (l.record == kRecProd) {
                            int ones = 0;
                            for (int dd = 0; dd < NB; ++dd) ones += __builtin_popcount(lds_ld(bl + 4u * dd));
                            // the last dword's flips are still pending
                            const uint32_t old = lds_ld(apend);
                            const uint32_t fl = fpend | (st.acc ? (1u << (4u * (uint32_t)((W - 1) % 8) + 3u)) : 0u);
                            ones += __builtin_popcount(old ^ fl) - __builtin_popcount(old);
                            const int mm = 2 * ones - L * L;
                            ((g_i64 *)p.sabs)[cidx] += (int64_t)(mm < 0 ? -mm : mm);
                        }
                    }
                }
            }
            lds_xor(apend, fpend | (st.acc ? (1u << (4u * (uint32_t)((W - 1) % 8) + 3u)) : 0u));
            const uint32_t Rk = st.acc ? st.C : st.R;
            ((g_i32 *)p.k)[it.chain0 + lane] = 2 * kk_of(Rk);
            int ones = 0;
            for (int dd = 0; dd < NB; ++dd) ones += __builtin_popcount(lds_ld(bl + 4u * dd));
            ((g_i32 *)p.m)[it.chain0 + lane] = 2 * ones - L * L;
        }
    } else {
        // producer wave i: batch bb of every sweep with bb = i mod np; lane r
        // forms the records r, r + 64, ... of the batch (chain r / B, dword r mod B)
        const int i = wave - 1;
        bool ok = true;
        for (int s = 0; s < n_sweeps && ok; ++s) {
            const uint32_t sweep = sweep0 + (uint32_t)s;
            for (int bb = i; bb < BPS; bb += np) {
                const uint32_t c = (uint32_t)s * (uint32_t)BPS + (uint32_t)bb;   // batch since the launch began
                const int y = bb / BTR, w0 = (bb - y * BTR) * B;
                // first what does not depend on the walker: the draws, and the
                // counts over the old left, right and lower neighbours (see the
                // streamed Ising walker)
                uint4 uu[HR];
                uint2 pre[HR];
                uint32_t cur[HR];
#pragma unroll
                for (int h = 0; h < HR; ++h) {
                    const int r = lane + 64 * h;
                    uu[h] = make_uint4(0, 0, 0, 0);
                    pre[h] = make_uint2(0, 0);
                    cur[h] = 0;
                    if (r < nch * B) {
                        const int cc = r / B, x = w0 + (r - cc * B);
                        const uint4 v = philox4x32_10((uint32_t)(y * W + x), sweep, (uint32_t)(it.chain0 + cc), 0u,
                                                      p.seed_lo, p.seed_hi);
                        uu[h] = make_uint4(min(v.x, 0xFFFFFFFEu), min(v.y, 0xFFFFFFFEu), min(v.z, 0xFFFFFFFEu),
                                           min(v.w, 0xFFFFFFFEu));
                        // the compact walker compares the top 14 bits
                        if (COMPACT) uu[h] = make_uint4(uu[h].x >> 18, uu[h].y >> 18, uu[h].z >> 18, uu[h].w >> 18);
                        const uint32_t lb = bits0 + (uint32_t)(cc * PB) * 4u;
                        const uint32_t rowb = lb + (uint32_t)(y * BPR) * 4u;
                        const uint32_t word = lds_ld(rowb + 4u * (uint32_t)(x / 8));
                        const uint32_t sh = 4u * (uint32_t)(x % 8);
                        cur[h] = spread_nibble((word >> sh) & 15u);
                        // left neighbour of site 0 (bit 31 of the previous word, or the
                        // row's last site at a row start) and right neighbour of site 3
                        const uint32_t lw = (x % 8 == 0) ? lds_ld(rowb + 4u * (uint32_t)((x == 0 ? W : x) / 8 - 1)) : word;
                        const uint32_t lbit = (lw >> ((sh + 31u) & 31u)) & 1u;
                        const uint32_t rw = (x % 8 == 7 && x + 1 < W) ? lds_ld(rowb + 4u * (uint32_t)(x / 8 + 1)) : word;
                        const uint32_t rbit = (rw >> ((sh + 4u) & 31u)) & 1u;
                        const uint32_t dw = lds_ld(lb + (uint32_t)(((y + 1 == L) ? 0 : y + 1) * BPR + x / 8) * 4u);
                        const uint32_t dn = spread_nibble((dw >> sh) & 15u);
                        pre[h] = ising_pre(cur[h], lbit << 24, rbit, dn, x == 0, x + 1 == W);
                    }
                }
                // then the walker must have finished (y-1, w0+B-1) and, for a
                // row's last batch, (y, 0); with fewer slots than dwords per row
                // it must also have finished the dwords whose records these
                // replace (x - R for dword x), which implies both
                const uint32_t g0 = c * (uint32_t)B;   // the batch's first dword since the launch began
                const uint32_t want = (R < W) ? g0 + (uint32_t)(B - R)
                                    : (w0 + B == W) ? g0 - (uint32_t)w0 + 1u : g0 + (uint32_t)(B - W);
                if (!stream_wait(ctr, kCtrDone, want, l.wait_polls)) {
                    ok = false;
                    break;
                }
#pragma unroll
                for (int h = 0; h < HR; ++h) {
                    const int r = lane + 64 * h;
                    if (r < nch * B) {
                        const int cc = r / B, x = w0 + (r - cc * B);
                        const uint32_t lb = bits0 + (uint32_t)(cc * PB) * 4u;
                        const uint32_t sh = 4u * (uint32_t)(x % 8);
                        // the row above as this sweep left it
                        const uint32_t uw = lds_ld(lb + (uint32_t)((y == 0 ? L - 1 : y - 1) * BPR + x / 8) * 4u);
                        const uint32_t xu = cur[h] ^ spread_nibble((uw >> sh) & 15u);
                        uint32_t d0 = pre[h].x + xu, d1 = pre[h].y + xu;
                        if (x + 1 == W) {
                            // right neighbour of the row's last site: the row's first site, this sweep
                            const uint32_t first = lds_ld(lb + (uint32_t)(y * BPR) * 4u) & 1u;
                            const uint32_t cr = (cur[h] ^ (first << 24)) & 0xFF000000u;
                            d0 += cr;
                            d1 += cr;
                        }
                        const uint32_t slot = ring0 + (uint32_t)cc * RS + (uint32_t)(x % R) * RECB;
                        lds_st4(slot, uu[h]);
                        if constexpr (COMPACT) {
                            CompactBulk fb;
                            compact_cols(BulkDiff{cur[h], d0, d1}, fb);
                            compact_steps(BulkDiff{cur[h], d0, d1}, fb);
                            lds_st4(slot + 16u, make_uint4(fb.a0, fb.a1, fb.e0, fb.e1));
                            lds_st4(slot + 32u, make_uint4(fb.z0, fb.z1, 0u, 0u));
                        } else {
                            FastBulk fb;
                            bulk_cols<false>(BulkDiff{cur[h], d0, d1}, fb);
                            bulk_steps<false>(BulkDiff{cur[h], d0, d1}, fb);
                            lds_st4(slot + 16u, make_uint4(fb.a0, fb.a1, fb.e0, fb.e1));
                        }
                    }
                }
                // publish in order: after batch c - 1 (formed by the previous wave)
                if (!stream_wait(ctr, kCtrFormed, c, l.wait_polls)) {
                    ok = false;
                    break;
                }
                if (lane == 0) lds_st_sync(ctr + kCtrFormed, c + 1u);
            }
        }
    }
    __syncthreads();
    if (tid == 0 && lds_ld_sync(ctr + kCtrAbort)) __hip_atomic_fetch_or(l.status, kStatusWaitExpired, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
    // bits back to bytes in HBM
    for (int j = tid; j < NB * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const uint32_t v = lds_ld(bits0 + (uint32_t)(c * PB + d) * 4u);
        g_u8 *g = (g_u8 *)p.spins + (int64_t)(32 * d) * p.C + it.chain0 + c;
        for (int b = 0; b < 32; ++b) g[(int64_t)b * p.C] = (uint8_t)((v >> b) & 1u);
    }
}

template <bool MAG, bool CS>
__device__ __forceinline__ bool run_fast_if_supported(const ProbDev &p, const WorkItem &it, char *lds,
                                                      const SweepLaunch &l, uint32_t sweep0, const LdsPlan &plan) {
    if constexpr (CS) {
        if (!MAG && stream_compact_ising(p, it)) {
            if (p.L == 96) run_ising_cstream<96, true>(p, it, lds, l, sweep0, plan);
            else run_ising_cstream<128, true>(p, it, lds, l, sweep0, plan);
            return true;
        }
        if (!MAG && stream_bit_ising(p, it)) {
            run_ising_cstream<64, false>(p, it, lds, l, sweep0, plan);
            return true;
        }
    }
    if (!MAG && packed_ising(p, it)) {
        switch (p.L) {
        case 64: run_ising_packed<64, false>(p, it, lds, l, sweep0, plan); return true;
        case 96: run_ising_packed<96, true>(p, it, lds, l, sweep0, plan); return true;
        case 128: run_ising_packed<128, true>(p, it, lds, l, sweep0, plan); return true;
        default: return false;
        }
    }
    if (!MAG && stream_ising(p, it)) {
        run_ising_stream<64>(p, it, lds, l, sweep0, plan);
        return true;
    }
    switch (p.L) {
    case 16: run_ising_fast<16, MAG>(p, it, lds, l, sweep0, plan); return true;
    case 24: run_ising_fast<24, MAG>(p, it, lds, l, sweep0, plan); return true;
    case 32: run_ising_fast<32, MAG>(p, it, lds, l, sweep0, plan); return true;
    case 48: run_ising_fast<48, MAG>(p, it, lds, l, sweep0, plan); return true;
    case 64: run_ising_fast<64, MAG>(p, it, lds, l, sweep0, plan); return true;
    default: return false;
    }
}

// ------------------------------------------------------------------ fast Potts walker (q = 8)
//
// Same scheme as the fast Ising walker.  Per dword of four sites the bulk
// step forms the proposals s' = (s + 1 + t) mod 8 and, with byte-wise xor and
// a v_perm lookup that maps 0 to 1 and 1..7 to 0, the equalities of every
// neighbour with s and with s'.  The energy change of a site is
// dk = sum_nb ([nb = s] - [nb = s']); the left neighbour's term has two
// candidates (its old state, or its proposal if it was accepted).  Bytes hold
// dk as int8 (for the row step, 36 bytes per row of nine columns) and the
// column byte offset 16 + 4 dk.  Proposal offsets are needed one dword ahead
// of the walker, across chunk boundaries, so the ring has three buffers and
// the producers run two chunks ahead.
//
// Two chunks ahead, the rows of a chunk and the row below it hold their
// final values of the previous sweep (or, below the last row, row 0 of this
// sweep), so the producers also form every term that does not involve the
// row above (which the walker is updating): with the proposals, the biased
// counts 0x80 + X - Y of both candidates without the up terms, and for the
// left neighbour's proposal of a dword's first site (drawn in the previous
// dword) a bit mask of the values equal to the site's state and to its
// proposal.  The walker adds the up terms, that first-site term, and at a
// row's last site the right neighbour, which is the row's first site of this
// sweep.

struct PottsBulk {
    uint32_t cur;      // old states
    uint32_t sp;       // proposals
    uint32_t a0, a1;   // bytes: column byte offset for candidates 0 / 1
    uint32_t k0, k1;   // bytes (int8): dk for candidates 0 / 1
};

__device__ __forceinline__ uint32_t eq8(uint32_t a, uint32_t b) {
    // per byte: 1 if equal (values 0..7), else 0
    return __builtin_amdgcn_perm(0u, 0x00000001u, a ^ b);
}

// Column byte offsets 4 (dk + 4) = 4 ((0x80 + dk) - 0x7c) of both candidates
// from the biased differences.
__device__ __forceinline__ void potts_maps_a(uint2 bd, PottsBulk &b) {
    b.a0 = (bd.x - 0x7C7C7C7Cu) << 2;
    b.a1 = (bd.y - 0x7C7C7C7Cu) << 2;
}

__device__ __forceinline__ void potts_steps(uint2 bd, PottsBulk &b) {
    b.k0 = bd.x ^ 0x80808080u;
    b.k1 = bd.y ^ 0x80808080u;
}

__device__ __forceinline__ int32_t row_step(const PottsBulk &b, bool left_flipped, int j) {
    return 36 * (left_flipped ? sbyte(b.k1, j) : sbyte(b.k0, j));
}

// Producer side of the Potts bulk for one dword: (B0, B1 - 1, T, sp) with
// B = (X | 0x80808080) - Y over the down, right and left terms (the right term
// of a row's last site and the left proposal term of a dword's first site
// left out), T a table of 1 + [v = s0] - [v = s'0] in two bits per value v of
// the first site's left proposal (all 1 at a row start, whose candidates
// agree), and the proposals sp.
__device__ __forceinline__ uint4 potts_pre(uint32_t cur, uint32_t prv, uint32_t nxt, uint32_t dn, uint32_t tq4,
                                           bool row_start, bool row_end) {
    const uint32_t sp = (cur + 0x01010101u + tq4) & 0x07070707u;
    const uint32_t rn = __builtin_amdgcn_alignbyte(nxt, cur, 1);
    const uint32_t lo = __builtin_amdgcn_alignbyte(cur, prv, 3);
    const uint32_t ln = sp << 8;   // left proposals of sites 1..3
    const uint32_t rmask = row_end ? 0x00FFFFFFu : 0xFFFFFFFFu;
    const uint32_t P2 = eq8(dn, cur) + (eq8(rn, cur) & rmask);
    const uint32_t Q2 = eq8(dn, sp) + (eq8(rn, sp) & rmask);
    const uint32_t lc = eq8(lo, cur), ls = eq8(lo, sp);
    uint32_t nc = eq8(ln, cur) & 0xFFFFFF00u, ns = eq8(ln, sp) & 0xFFFFFF00u;
    if (row_start) {
        nc |= lc & 0xFFu;
        ns |= ls & 0xFFu;
    }
    const uint32_t B0 = ((P2 + lc) | 0x80808080u) - (Q2 + ls);
    const uint32_t B1 = ((P2 + nc) | 0x80808080u) - (Q2 + ns);
    const uint32_t T = row_start ? 0x5555u : 0x5555u + (1u << (2u * (cur & 7u))) - (1u << (2u * (sp & 7u)));
    return make_uint4(B0, B1 - 1u, T, sp);
}

// Walker side: the up terms added to the producer's counts.
__device__ __forceinline__ uint2 potts_up(uint32_t cur, uint32_t up, const uint4 &pe) {
    const uint32_t eu = eq8(up, cur), es = eq8(up, pe.w);
    return make_uint2(pe.x + eu - es, pe.y + eu - es);
}

// A row's last site: its right neighbour is the row's first site, updated
// earlier in this sweep (byte 0 of first).
__device__ __forceinline__ uint2 potts_row_end(uint2 bd, uint32_t cur, uint32_t sp, uint32_t first) {
    const uint32_t t = first << 24;
    const uint32_t x3 = eq8(t, cur) & 0xFF000000u, y3 = eq8(t, sp) & 0xFF000000u;
    return make_uint2(bd.x + x3 - y3, bd.y + x3 - y3);
}

// A dword's first site with its left neighbour accepted: that neighbour holds
// its proposal v (byte 3 of sp_prv), looked up in the producer's table at bit
// 2v = sp_prv >> 23 (byte 2 of sp_prv is at most 7).  The table entry carries
// the +1 that the producer took off B1.
__device__ __forceinline__ uint32_t potts_left(uint32_t b1, uint32_t T, uint32_t sp_prv) {
    return b1 + __builtin_amdgcn_ubfe(T, sp_prv >> 23, 2u);
}

// Compact table of the Potts walker (L = 48): as for the Ising walker, the
// pair of rows (k, k+j), j = 1..4, has one rejectable direction, stored in a
// u16 (bit 14 set when it is the move down; bits 0..13 the top 14 bits of its
// threshold).  Entry (k, j) sits at byte 8 k + 2 j after a 2-byte pad, so a
// move by d reads 8 k + 2 d for d > 0 and 8 k + 6 d for d < 0.  With the row
// register R = tab0 + 8 k - 247 the column codes 247 + (2 d or 6 d) are
// 223..255, one v_perm lookup on dk + 4 (the selector 8 of dk = +4 copies bit
// 7 of byte 1 of the low source, which is set: 0xff).  The decode code (byte
// 1 of the xor) is 0x40 for a move down and 0x80 for dk = 0.  The walker
// keeps 256 bytes free before the table, so that every code addresses LDS
// inside the workgroup's allocation whatever the row.
constexpr uint32_t kPottsCompactBias = 247;
constexpr uint32_t kPottsCompactGuard = kPottsGuardBytes;

struct CompactPottsBulk {
    uint32_t cur, sp;   // old states, proposals
    uint32_t a0, a1;    // column codes of candidates 0 / 1
    uint32_t k0, k1;    // dk bytes (int8)
    uint32_t z0, z1;    // decode codes
};

__device__ __forceinline__ void potts_maps_c(uint2 bd, CompactPottsBulk &b) {
    const uint32_t i0 = bd.x - 0x7C7C7C7Cu, i1 = bd.y - 0x7C7C7C7Cu;   // dk + 4 per byte
    b.a0 = __builtin_amdgcn_perm(0xFDFBF9F7u, 0xF1EBE5DFu, i0);          // 223 229 235 241 247 249 251 253 255
    b.a1 = __builtin_amdgcn_perm(0xFDFBF9F7u, 0xF1EBE5DFu, i1);
    b.z0 = __builtin_amdgcn_perm(0x00000080u, 0x40404040u, i0);          // 0x40 x4, 0x80, 0 x4
    b.z1 = __builtin_amdgcn_perm(0x00000080u, 0x40404040u, i1);
}
__device__ __forceinline__ void potts_steps(uint2 bd, CompactPottsBulk &b) {
    b.k0 = bd.x ^ 0x80808080u;
    b.k1 = bd.y ^ 0x80808080u;
}
__device__ __forceinline__ int32_t row_step(const CompactPottsBulk &b, bool left_flipped, int j) {
    return 8 * (left_flipped ? sbyte(b.k1, j) : sbyte(b.k0, j));
}

// Exact recomputation of one dword of the compact Potts walker (see
// redo_compact_dword): rows R = tab0 + 8 k - 247, full thresholds
// T32[k][dk + 4], and the acceptance draws of dword dw: words 1 and 3 of the
// blocks 2 dw (sites 0, 1) and 2 dw + 1 (sites 2, 3).  The flip record holds
// 0xff in byte j for an accepted site j.
__device__ __noinline__ RedoResult redo_compact_potts(uint32_t R, uint32_t C, uint32_t acc_in, uint32_t ca0,
                                                      uint32_t ca1, uint32_t ck0, uint32_t ck1, uint32_t cz0,
                                                      uint32_t cz1, uint32_t na0, uint32_t na1, uint32_t u0,
                                                      uint32_t u1, uint32_t u2, uint32_t u3, uint32_t tab0,
                                                      const uint32_t *table, uint32_t dw, uint32_t sweep,
                                                      uint32_t chain, uint32_t seed_lo, uint32_t seed_hi) {
    const g_u32 *T = (const g_u32 *)table;
    bool acc = acc_in != 0;
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t Rj = acc ? C : R;
        const int32_t dk = acc ? sbyte(ck1, j) : sbyte(ck0, j);
        const uint32_t code = acc ? ubyte(ca1, j) : ubyte(ca0, j);
        const uint32_t z = acc ? ubyte(cz1, j) : ubyte(cz0, j);
        const uint32_t t = lds_ld16(Rj + code) ^ (z << 8);
        const uint32_t a = (j == 0) ? u0 : (j == 1) ? u1 : (j == 2) ? u2 : u3;
        bool ok;
        if (a != t) {
            ok = a < t;
        } else {
            const int k = (int)((Rj + kPottsCompactBias - tab0) >> 3);
            const uint32_t Tf = T[k * 9 + 4 + dk];
            const uint4 b = philox4x32_10(2u * dw + (uint32_t)(j >> 1), sweep, chain, 0u, seed_lo, seed_hi);
            ok = min((j & 1) ? b.w : b.y, 0xFFFFFFFEu) < Tf;
        }
        R = Rj;
        C = Rj + (uint32_t)(8 * dk);
        acc = ok;
        if (ok) f |= 0xFFu << (8 * j);
    }
    return redo_result(R, C, lds_ld16(R + na0), lds_ld16(C + na1), acc, f);
}

__device__ __forceinline__ RedoResult compact_redo(uint32_t R0, uint32_t C0, bool acc0, const CompactPottsBulk &b,
                                                   const CompactPottsBulk &nb, const uint4 &u, const CompactExact &ex) {
    return redo_compact_potts(R0, C0, acc0 ? 1u : 0u, b.a0, b.a1, b.k0, b.k1, b.z0, b.z1,
                              __builtin_amdgcn_ubfe(nb.a0, 0u, 8u), __builtin_amdgcn_ubfe(nb.a1, 0u, 8u), u.x, u.y,
                              u.z, u.w, ex.tab0, ex.table, ex.blk, ex.sweep, ex.chain, ex.seed_lo, ex.seed_hi);
}

template <int L, bool WIDE, bool COMPACT>
__device__ __forceinline__ void run_potts_fast(const ProbDev &p, const WorkItem &it, char *lds, const SweepLaunch &l,
                               uint32_t sweep0, const LdsPlan &plan) {
    constexpr int W = L / 4;
    constexpr int NW = L * L / 4;
    constexpr int RPC = potts_rows_per_chunk(L, WIDE);
    constexpr int CDW = RPC * W;
    constexpr int NCH = L / RPC;
    constexpr int P = fast_lane_stride(L);
    constexpr uint32_t ROWB = COMPACT ? 8u : 36u;   // table row: four u16 pairs, or nine words
    static_assert(L % RPC == 0 && W >= 4, "fast walker shape");
    using Bulk = typename std::conditional<COMPACT, CompactPottsBulk, PottsBulk>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int nch = it.nchains;
    const bool active = (wave == 0) && (lane < nch);
    const uint32_t lbase = (uint32_t)(size_t)(__attribute__((address_space(3))) char *)lds;
    const uint32_t tab0 = lbase + (uint32_t)plan.off_tab + (COMPACT ? kPottsCompactGuard : 0u);
    const uint32_t spin0 = lbase + (uint32_t)plan.off_spin;
    const uint32_t ringu0 = lbase + (uint32_t)plan.off_ring;                    // [3][lane][CDW+1] uint4
    auto row_of = [&](int k) -> uint32_t {
        return COMPACT ? tab0 + 8u * (uint32_t)k - kPottsCompactBias : tab0 + ROWB * (uint32_t)k;
    };
    auto k_of = [&](uint32_t R) -> int {
        return COMPACT ? (int)((R + kPottsCompactBias - tab0) >> 3) : (int)((R - tab0) / ROWB);
    };
    auto read_t = [&](uint32_t a) -> uint32_t { return COMPACT ? lds_ld16(a) : lds_ld(a); };
    auto maps = [&](uint2 bd, Bulk &b) {
        if constexpr (COMPACT) potts_maps_c(bd, b);
        else potts_maps_a(bd, b);
    };

    if constexpr (COMPACT) {
        // the pair table from the 32-bit table in HBM (rows k, columns dk + 4)
        const g_u32 *T = (const g_u32 *)p.table;
        const int rows = 2 * p.N + 1;
        if (tid == 0) *(lds_u16 *)(size_t)tab0 = 0;
        for (int e = tid; e < 4 * rows; e += nthreads) {
            const int k = e >> 2, j = (e & 3) + 1;
            uint16_t v = 0;
            if (k + j < rows) v = compact_entry(T[k * 9 + 4 + j], T[(k + j) * 9 + 4 - j]);
            *(lds_u16 *)(size_t)(tab0 + 2u + 2u * (uint32_t)e) = v;
        }
    }
    const uint32_t ubuf = (uint32_t)nch * (CDW + 1) * 16u;
    const uint32_t ringp0 = ringu0 + 3u * ubuf;                                 // [3][lane][CDW+1] uint4

    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const g_u8 *g = (const g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        const uint32_t v = (uint32_t)g[0] | ((uint32_t)g[p.C] << 8) | ((uint32_t)g[2 * (int64_t)p.C] << 16) |
                           ((uint32_t)g[3 * (int64_t)p.C] << 24);
        lds_st(spin0 + (uint32_t)(c * P + d) * 4u, v);
    }
    __syncthreads();   // the producers read the staged lattice

    // producers: chunk t covers rows (t mod NCH) * RPC .. + RPC - 1 of sweep t / NCH;
    // one work unit is one dword (two Philox blocks of two sites each)
    auto produce = [&](int t) {
        const int sw = t / NCH;
        const uint32_t sweep = sweep0 + (uint32_t)sw;
        const int ci = t - sw * NCH;
        const int dw0 = ci * CDW;
        const uint32_t bu = ringu0 + (uint32_t)(t % 3) * ubuf, bp = ringp0 + (uint32_t)(t % 3) * ubuf;
        const int total = CDW * nch;
        for (int w = tid - 64; w < total; w += nthreads - 64) {
            const int c = w / CDW, q = w - c * CDW;
            const uint32_t chain = (uint32_t)(it.chain0 + c);
            const uint4 b0 = philox4x32_10((uint32_t)(2 * (dw0 + q)), sweep, chain, 0u, p.seed_lo, p.seed_hi);
            const uint4 b1 = philox4x32_10((uint32_t)(2 * (dw0 + q) + 1), sweep, chain, 0u, p.seed_lo, p.seed_hi);
            const uint32_t t0 = (uint32_t)(((uint64_t)b0.x * 7u) >> 32), t1 = (uint32_t)(((uint64_t)b0.z * 7u) >> 32);
            const uint32_t t2 = (uint32_t)(((uint64_t)b1.x * 7u) >> 32), t3 = (uint32_t)(((uint64_t)b1.z * 7u) >> 32);
            const uint32_t off = (uint32_t)(c * (CDW + 1) + q);
            uint4 acc_words = make_uint4(min(b0.y, 0xFFFFFFFEu), min(b0.w, 0xFFFFFFFEu), min(b1.y, 0xFFFFFFFEu),
                                         min(b1.w, 0xFFFFFFFEu));
            // the compact walker compares the top 14 bits
            if (COMPACT) acc_words = make_uint4(acc_words.x >> 18, acc_words.y >> 18, acc_words.z >> 18, acc_words.w >> 18);
            lds_st4(bu + off * 16u, acc_words);
            // lattice terms of the dword (row y, dword x of chain c)
            const int r = q / W, x = q - r * W;
            const int y = ci * RPC + r;
            const uint32_t lb = spin0 + (uint32_t)(c * P) * 4u;
            const uint32_t rowb = lb + (uint32_t)(y * W) * 4u;
            const uint32_t cur = lds_ld(rowb + 4u * (uint32_t)x);
            const uint32_t prv = lds_ld(rowb + 4u * (uint32_t)(x == 0 ? W - 1 : x - 1));
            const uint32_t nxt = lds_ld(rowb + 4u * (uint32_t)(x + 1 == W ? x : x + 1));
            const uint32_t dn = lds_ld(lb + (uint32_t)(((y + 1 == L) ? 0 : y + 1) * W + x) * 4u);
            lds_st4(bp + off * 16u, potts_pre(cur, prv, nxt, dn, t0 | (t1 << 8) | (t2 << 16) | (t3 << 24), x == 0,
                                             x + 1 == W));
        }
    };

    const int total_chunks = NCH * l.n_sweeps;
    if (wave > 0) {
        produce(0);
        if (total_chunks > 1) produce(1);
    }
    __syncthreads();

    const uint32_t sb = spin0 + (uint32_t)(lane * P) * 4u;
    const uint32_t rbu = ringu0 + (uint32_t)(lane * (CDW + 1)) * 16u;
    const uint32_t rbp = ringp0 + (uint32_t)(lane * (CDW + 1)) * 16u;
    auto row_addr = [&](int y) -> uint32_t { return sb + (uint32_t)(y * W) * 4u; };

    using State = typename std::conditional<COMPACT, CompactState, FastState>::type;
    State st{};
    uint4 u_next = make_uint4(0, 0, 0, 0);
    Bulk nb{};
    // the row above, as updated in this sweep: the walker's own stores
    uint32_t upr[W];
#pragma unroll
    for (int w = 0; w < W; ++w) upr[w] = 0;
    if (active) {
#pragma unroll
        for (int w = 0; w < W; ++w) upr[w] = lds_ld(row_addr(L - 1) + 4u * w);
        const int k = ((const g_i32 *)p.k)[it.chain0 + lane];
        st.R = row_of(k);
        st.C = st.R;
        const uint32_t r0 = row_addr(0), rl = row_addr(L - 1);
        // dword 0 of chunk 0 (a row start): the producer's terms and the up row
        const uint4 pe0 = lds_ld4(rbp);
        const uint32_t c0 = lds_ld(r0);
        uint2 bd0 = potts_up(c0, lds_ld(rl), pe0);
        bd0.y += 1u;   // a row start: its table entry is 1 whatever the left proposal
        maps(bd0, nb);
        potts_steps(bd0, nb);
        nb.cur = c0;
        nb.sp = pe0.w;
        st.tA = read_t(st.R + ubyte(nb.a0, 0));
        st.tB = st.tA;
    }

    for (int t = 0; t < total_chunks; ++t) {
        if (wave == 0) {
            if (active) {
                const int sw = t / NCH;
                const int ci = t - sw * NCH;
                const uint32_t sweep = sweep0 + (uint32_t)sw;
                const uint32_t ub = rbu + (uint32_t)(t % 3) * ubuf;
                const uint32_t pb = rbp + (uint32_t)(t % 3) * ubuf;
                const uint32_t pbn = rbp + (uint32_t)((t + 1) % 3) * ubuf;   // next chunk's lattice terms
#pragma unroll
                for (int r = 0; r < RPC; ++r) {
                    const int y = ci * RPC + r;
                    const uint32_t vcur = row_addr(y);
                    const int yn = (y + 1 == L) ? 0 : y + 1;
                    const uint32_t vnc = row_addr(yn);
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const Bulk b = nb;
                        const uint4 u = (r == 0 && w == 0) ? lds_ld4(ub) : u_next;
                        // the next dword's bulk, in pieces between this dword's sites
                        uint32_t ncur = 0, nup = 0, first = 0;
                        uint4 pe = make_uint4(0, 0, 0, 0);
                        uint2 bd = make_uint2(0, 0);
                        auto work = [&](int j) {
                            if (j == 0) {
                                if (r * W + w + 1 < CDW) u_next = lds_ld4(ub + (uint32_t)(r * W + w + 1) * 16u);
                                if (w + 1 < W) {
                                    ncur = lds_ld(vcur + 4 * (w + 1));
                                    nup = upr[w + 1];
                                    pe = lds_ld4(pb + (uint32_t)(r * W + w + 1) * 16u);
                                    if (w + 2 == W) first = upr[0];   // the row's first dword, this sweep
                                } else {
                                    // first dword of the next row: its upper row is this one (new)
                                    ncur = lds_ld(vnc);
                                    nup = upr[0];
                                    pe = (r + 1 < RPC) ? lds_ld4(pb + (uint32_t)((r + 1) * W) * 16u) : lds_ld4(pbn);
                                }
                            } else if (j == 1) {
                                bd = potts_up(ncur, nup, pe);
                                if (w + 2 == W) bd = potts_row_end(bd, ncur, pe.w, first);
                            } else if (j == 2) {
                                bd.y = potts_left(bd.y, pe.z, b.sp);
                                maps(bd, nb);
                            } else {
                                potts_steps(bd, nb);
                                nb.cur = ncur;
                                nb.sp = pe.w;
                            }
                        };
                        uint32_t mask;
                        if constexpr (COMPACT) {
                            const CompactExact ex{tab0, p.table, (uint32_t)(y * W + w), sweep,
                                                  (uint32_t)(it.chain0 + lane), p.seed_lo, p.seed_hi};
                            mask = walk_dword_compact<Bulk, 0xFFu, 8>(st, b, nb, u, work, ex);
                        } else {
                            mask = walk_dword<Bulk, 0xFFu, 8>(st, b, nb, u, work);
                        }
                        upr[w] = (mask & b.sp) | (~mask & b.cur);
                        lds_st(vcur + 4 * w, upr[w]);
                    }
                    if (y == L - 1 && l.record != kRecNone) {
                        const uint32_t Rk = st.acc ? st.C : st.R;
                        const int k = k_of(Rk);
                        g_i32 *h = (g_i32 *)p.hist;
                        h[(int64_t)k * p.C + it.chain0 + lane] += 1;
                    }
                }
            }
        } else if (t + 2 < total_chunks) {
            produce(t + 2);
        }
        __syncthreads();
    }

    if (active) {
        const uint32_t Rk = st.acc ? st.C : st.R;
        ((g_i32 *)p.k)[it.chain0 + lane] = k_of(Rk);
        ((g_i32 *)p.m)[it.chain0 + lane] = 0;
    }
    __syncthreads();
    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const uint32_t v = lds_ld(spin0 + (uint32_t)(c * P + d) * 4u);
        g_u8 *g = (g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        g[0] = (uint8_t)v;
        g[p.C] = (uint8_t)(v >> 8);
        g[2 * (int64_t)p.C] = (uint8_t)(v >> 16);
        g[3 * (int64_t)p.C] = (uint8_t)(v >> 24);
    }
}

// ------------------------------------------------------------------ streamed compact Potts walker
//
// The fast Potts walker at L = 48 forms part of every dword's bulk itself
// (the terms of the row above, the first site's left proposal, the right
// neighbour of a row's last site) and decodes the compact table on top: about
// 150 cycles per site.  As for the streamed Ising walker, the producer waves
// here form each dword's complete record after the walker has left the row
// above, and the walker only decides sites.  A record holds:
//   - the four draws' 14-bit prefixes (the compact comparison);
//   - the column codes, row steps (8 dk bytes, the compact row stride) and
//     decode codes of both candidates of every site;
//   - the xor of the old states and the proposals, which the walker applies
//     to the accepted sites.
// The proposal of a dword's last site, which the next dword's first site sees
// as its left neighbour when it is accepted, is drawn again by the producer of
// that next dword (one more Philox block), so records never wait for each
// other.  Progress counters, in-order publishing, bounded waits and the
// abort path are those of the streamed Ising walker.  A dword with a draw
// equal to its decoded entry is redone exactly (redo_compact_potts).

// The four sites of one dword: as walk_dword_stream, with the compact decode
// and the detection of undecidable draws (tie).  The flip record holds 0xff
// in byte j for an accepted site j.
template <class Work, class Done>
__device__ __forceinline__ uint32_t walk_dword_pstream(FastState &s, const uint4 &m, const uint4 &z,
                                                       const uint4 &nm, const uint4 &u, uint32_t fprev, bool &tie,
                                                       Work &&work, Done &&done) {
    uint32_t f = 0;
    bool eq = false;   // the previous site's tie, folded in a site later (its compare has long finished)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool acc = s.acc;
        const uint32_t Rj = acc ? s.C : s.R;
        const uint32_t Cj = Rj + (uint32_t)(acc ? sbyte(m.w, j) : sbyte(m.z, j));
        uint32_t adA, adB;
        if (j < 3) {
            adA = Rj + ubyte(m.x, j + 1);
            adB = Cj + ubyte(m.y, j + 1);
        } else {
            adA = add_byte0(Rj, nm.x);
            adB = add_byte0(Cj, nm.y);
        }
        const uint32_t nA = lds_ld16(adA);
        const uint32_t nB = lds_ld16(adB);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t tA = xor_byte1(s.tA, z.x, j);
        const uint32_t tB = xor_byte1(s.tB, z.y, j);
        tie |= eq;
        const uint32_t tj = acc ? tB : tA;
        const uint32_t uj = (j == 0) ? u.x : (j == 1) ? u.y : (j == 2) ? u.z : u.w;
        s.acc = uj < tj;
        eq = uj == tj;
        s.R = Rj;
        s.C = Cj;
        s.tA = nA;
        s.tB = nB;
        __builtin_amdgcn_sched_barrier(0);
        if (j == 0) {
            done(fprev | (acc ? 0xFF000000u : 0u));
        } else {
            f |= acc ? (0xFFu << (8 * (j - 1))) : 0u;
            asm volatile("" : "+v"(f));   // recorded here, not at the end of the dword
        }
        work(j);
        __builtin_amdgcn_sched_barrier(0);
    }
    tie |= eq;
    return f;
}

// dk bytes from row-step bytes 8 dk (each byte shifted right by 3 with its sign)
__device__ __forceinline__ uint32_t pstream_dk(uint32_t e) {
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) r |= ((uint32_t)(sbyte(e, j) >> 3) & 0xFFu) << (8 * j);
    return r;
}

template <int L>
__device__ __forceinline__ void run_potts_stream(const ProbDev &p, const WorkItem &it, char *lds, const SweepLaunch &l,
                                                 uint32_t sweep0, const LdsPlan &plan) {
    constexpr int W = L / 4;                  // dwords per row
    constexpr int NW = L * L / 4;             // dwords per lattice
    constexpr int P = fast_lane_stride(L);    // lattice dwords between lanes
    constexpr int B = kPStreamBatch;
    constexpr int BPR = W / B;                // batches per row
    constexpr int BPS = L * BPR;              // batches per sweep
    constexpr uint32_t RS = pstream_lane_words(L) * 4u;   // ring bytes per lane
    constexpr uint32_t RECB = 48u;                        // record bytes
    static_assert(W % B == 0 && W >= 2 * B + 1, "streamed Potts walker shape");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int np = nthreads / 64 - 1;         // producer waves
    const int nch = it.nchains;
    const bool active = (wave == 0) && (lane < nch);
    const uint32_t lbase = (uint32_t)(size_t)(__attribute__((address_space(3))) char *)lds;
    const uint32_t tab0 = lbase + (uint32_t)plan.off_tab + kPottsCompactGuard;
    const uint32_t spin0 = lbase + (uint32_t)plan.off_spin;
    const uint32_t ring0 = lbase + (uint32_t)plan.off_ring;
    const uint32_t ctr = lbase + (uint32_t)plan.off_ctr;   // counters (see kCtrDone)

    // the pair table from the 32-bit table in HBM (rows k, columns dk + 4)
    {
        const g_u32 *T = (const g_u32 *)p.table;
        const int rows = 2 * p.N + 1;
        if (tid == 0) *(lds_u16 *)(size_t)tab0 = 0;
        for (int e = tid; e < 4 * rows; e += nthreads) {
            const int k = e >> 2, j = (e & 3) + 1;
            uint16_t v = 0;
            if (k + j < rows) v = compact_entry(T[k * 9 + 4 + j], T[(k + j) * 9 + 4 - j]);
            *(lds_u16 *)(size_t)(tab0 + 2u + 2u * (uint32_t)e) = v;
        }
    }
    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const g_u8 *g = (const g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        const uint32_t v = (uint32_t)g[0] | ((uint32_t)g[p.C] << 8) | ((uint32_t)g[2 * (int64_t)p.C] << 16) |
                           ((uint32_t)g[3 * (int64_t)p.C] << 24);
        lds_st(spin0 + (uint32_t)(c * P + d) * 4u, v);
    }
    if (tid < kStreamCtrWords) lds_st(ctr + 4u * (uint32_t)tid, 0u);
    __syncthreads();

    const int n_sweeps = l.n_sweeps;
    if (wave == 0) {
        if (active) {
            const uint32_t sb = spin0 + (uint32_t)(lane * P) * 4u;   // this lane's lattice
            const uint32_t rb = ring0 + (uint32_t)lane * RS;          // this lane's records
            auto row_addr = [&](int y) -> uint32_t { return sb + (uint32_t)(y * W) * 4u; };
            FastState st{0, 0, 0, 0, false};
            const int k0 = ((const g_i32 *)p.k)[it.chain0 + lane];
            st.R = tab0 + 8u * (uint32_t)k0 - kPottsCompactBias;
            st.C = st.R;
            // After a wait gives up, the walker rewrites its records to reject
            // every move (prefixes 2^32 - 1, which equal no entry; code 0, which
            // stays in the guard before the table; no step, no state change).
            auto neutralize = [&]() {
                for (int w = 0; w < W; ++w) {
                    lds_st4(rb + (uint32_t)w * RECB, make_uint4(~0u, ~0u, ~0u, ~0u));
                    lds_st4(rb + (uint32_t)w * RECB + 16u, make_uint4(0u, 0u, 0u, 0u));
                    lds_st4(rb + (uint32_t)w * RECB + 32u, make_uint4(0u, 0u, 0u, 0u));
                }
            };
            bool ok = stream_wait(ctr, kCtrFormed, 1u, l.wait_polls);   // batch 0 of the launch
            if (!ok) neutralize();
            uint4 u_next = lds_ld4(rb);
            uint4 nm = lds_ld4(rb + 16u);
            uint4 nz = lds_ld4(rb + 32u);
            st.tA = lds_ld16(st.R + ubyte(nm.x, 0));
            st.tB = st.tA;
            uint32_t c = 0;        // batches walked before the current one (wraps)
            uint32_t formed = 0;   // batches formed, read a dword before the check
            uint32_t fpend = 0;    // flips of sites 0..2 of the last dword walked, not yet in the lattice
            uint32_t xpend = 0;    // that dword's state xor (old ^ proposal)
            uint32_t apend = sb;   // that dword's address (nothing pending before the first dword)
            for (int s = 0; s < n_sweeps && ok; ++s) {
                const uint32_t sweep = sweep0 + (uint32_t)s;
                for (int y = 0; y < L && ok; ++y) {
                    const uint32_t vcur = row_addr(y);
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const int q = w % B;
                        // in a batch's last dword: batch c + 1 (whose first record this
                        // dword's first site reads), none beyond the launch; the counter
                        // was read a dword earlier
                        if (q == B - 2) formed = lds_ld_sync(ctr + kCtrFormed);
                        if (q == B - 1 && ok) {
                            const uint32_t f1 = __builtin_amdgcn_readfirstlane(formed);
                            const bool last = (y == L - 1 && s + 1 == n_sweeps && w + 1 == W);
                            const uint32_t want = __builtin_amdgcn_readfirstlane(c) + (last ? 1u : 2u);
                            if ((int32_t)(f1 - want) < 0) {
                                ok = stream_wait(ctr, kCtrFormed, want, l.wait_polls);
                                if (!ok) neutralize();
                            }
                            lds_order();
                        }
                        const uint4 m = nm, z = nz;
                        const uint4 u = u_next;
                        auto work = [&](int j) {
                            if (j == 0) {
                                const uint32_t slot = rb + (uint32_t)((w + 1) % W) * RECB;   // dword after this one
                                u_next = lds_ld4(slot);
                                nm = lds_ld4(slot + 16u);
                                nz = lds_ld4(slot + 32u);
                            }
                        };
                        // the previous dword's accepted sites take their proposals; after a
                        // batch's last dword, and after a row's first dword (which the
                        // row's last batch needs), the walker reports its progress
                        auto done = [&](uint32_t fp) {
                            lds_xor(apend, fp & xpend);
                            if (q == 0 || w == 1) {
                                lds_order();
                                lds_st_sync(ctr + kCtrDone, c * (uint32_t)B + (uint32_t)q);
                            }
                        };
                        const uint32_t R0 = st.R, C0 = st.C;
                        const bool acc0 = st.acc;
                        bool tie = false;
                        uint32_t f = walk_dword_pstream(st, m, z, nm, u, fpend, tie, work, done);
                        if (__builtin_amdgcn_ballot_w64(tie) != 0u) {
                            // rare (about one dword in 4096 per chain): the whole wave redoes
                            // the dword exactly (the redo agrees with the fast path wherever
                            // the prefixes decide) and writes the whole record (0xff in byte j
                            // for an accepted site j); site 3's outcome stays pending
                            const RedoResult r = redo_compact_potts(
                                R0, C0, acc0 ? 1u : 0u, m.x, m.y, pstream_dk(m.z), pstream_dk(m.w), z.x, z.y,
                                __builtin_amdgcn_ubfe(nm.x, 0u, 8u), __builtin_amdgcn_ubfe(nm.y, 0u, 8u), u.x, u.y,
                                u.z, u.w, tab0, p.table,
                                (uint32_t)(y * W + w), sweep, (uint32_t)(it.chain0 + lane), p.seed_lo, p.seed_hi);
                            st.R = r.s0;
                            st.C = r.s1;
                            st.tA = r.s2;
                            st.tB = r.s3;
                            st.acc = r.s4 != 0u;
                            f = r.s5 & 0x00FFFFFFu;
                        }
                        fpend = f;
                        xpend = z.z;
                        apend = vcur + 4u * (uint32_t)w;
                        if (q == B - 1) ++c;
                    }
                    if (y == L - 1 && l.record != kRecNone) {
                        const uint32_t Rk = st.acc ? st.C : st.R;
                        int bin = (int)((int32_t)(Rk + kPottsCompactBias - tab0) >> 3);
                        bin = min(max(bin, 0), p.nbins - 1);   // in range even after an abort
                        ((g_i32 *)p.hist)[(int64_t)bin * p.C + it.chain0 + lane] += 1;
                    }
                }
            }
            lds_xor(apend, (fpend | (st.acc ? 0xFF000000u : 0u)) & xpend);
            const uint32_t Rk = st.acc ? st.C : st.R;
            ((g_i32 *)p.k)[it.chain0 + lane] = (int)((int32_t)(Rk + kPottsCompactBias - tab0) >> 3);
            ((g_i32 *)p.m)[it.chain0 + lane] = 0;
        }
    } else {
        // producer wave i: batch bb of every sweep with bb = i mod np; lane r
        // forms the records r, r + 64 of the batch (chain r / B, dword r mod B)
        const int i = wave - 1;
        bool ok = true;
        for (int s = 0; s < n_sweeps && ok; ++s) {
            const uint32_t sweep = sweep0 + (uint32_t)s;
            for (int bb = i; bb < BPS; bb += np) {
                const uint32_t c = (uint32_t)s * (uint32_t)BPS + (uint32_t)bb;   // batch since the launch began
                const int y = bb / BPR, w0 = (bb - y * BPR) * B;
                // everything that does not depend on the walker first (see the
                // streamed Ising walker): draws, proposals and the terms of the
                // old left, right and lower neighbours
                uint4 uu[2], pe[2];
                uint32_t cur[2], spv[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = lane + 64 * h;
                    uu[h] = make_uint4(0, 0, 0, 0);
                    pe[h] = make_uint4(0, 0, 0, 0);
                    cur[h] = 0;
                    spv[h] = 0;
                    if (r < nch * B) {
                        const int cc = r / B, x = w0 + (r - cc * B);
                        const uint32_t chain = (uint32_t)(it.chain0 + cc);
                        const uint32_t dw = (uint32_t)(y * W + x);
                        const uint4 b0 = philox4x32_10(2u * dw, sweep, chain, 0u, p.seed_lo, p.seed_hi);
                        const uint4 b1 = philox4x32_10(2u * dw + 1u, sweep, chain, 0u, p.seed_lo, p.seed_hi);
                        const uint32_t t0 = (uint32_t)(((uint64_t)b0.x * 7u) >> 32);
                        const uint32_t t1 = (uint32_t)(((uint64_t)b0.z * 7u) >> 32);
                        const uint32_t t2 = (uint32_t)(((uint64_t)b1.x * 7u) >> 32);
                        const uint32_t t3 = (uint32_t)(((uint64_t)b1.z * 7u) >> 32);
                        uu[h] = make_uint4(min(b0.y, 0xFFFFFFFEu) >> 18, min(b0.w, 0xFFFFFFFEu) >> 18,
                                           min(b1.y, 0xFFFFFFFEu) >> 18, min(b1.w, 0xFFFFFFFEu) >> 18);
                        const uint32_t lb = spin0 + (uint32_t)(cc * P) * 4u;
                        const uint32_t rowb = lb + (uint32_t)(y * W) * 4u;
                        cur[h] = lds_ld(rowb + 4u * (uint32_t)x);
                        const uint32_t prv = lds_ld(rowb + 4u * (uint32_t)(x == 0 ? W - 1 : x - 1));
                        const uint32_t nxt = lds_ld(rowb + 4u * (uint32_t)(x + 1 == W ? x : x + 1));
                        const uint32_t dn = lds_ld(lb + (uint32_t)((y + 1 == L ? 0 : y + 1) * W + x) * 4u);
                        pe[h] = potts_pre(cur[h], prv, nxt, dn, t0 | (t1 << 8) | (t2 << 16) | (t3 << 24), x == 0,
                                          x + 1 == W);
                        if (x > 0) {
                            // the previous dword's last proposal: its old state (byte 3 of
                            // prv) moved by the draw of its second block
                            const uint4 bp = philox4x32_10(2u * dw - 1u, sweep, chain, 0u, p.seed_lo, p.seed_hi);
                            const uint32_t tp = (uint32_t)(((uint64_t)bp.z * 7u) >> 32);
                            spv[h] = (((prv >> 24) + 1u + tp) & 7u) << 24;
                        }
                    }
                }
                // then the walker must have finished (y-1, w0+B-1) and, for a
                // row's last batch, (y, 0)
                const uint32_t g0 = c * (uint32_t)B;   // the batch's first dword since the launch began
                const uint32_t want = (w0 + B == W) ? g0 - (uint32_t)w0 + 1u : g0 + (uint32_t)(B - W);
                if (!stream_wait(ctr, kCtrDone, want, l.wait_polls)) {
                    ok = false;
                    break;
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = lane + 64 * h;
                    if (r < nch * B) {
                        const int cc = r / B, x = w0 + (r - cc * B);
                        const uint32_t lb = spin0 + (uint32_t)(cc * P) * 4u;
                        // the row above as this sweep left it
                        const uint32_t up = lds_ld(lb + (uint32_t)((y == 0 ? L - 1 : y - 1) * W + x) * 4u);
                        uint2 bd = potts_up(cur[h], up, pe[h]);
                        if (x + 1 == W) bd = potts_row_end(bd, cur[h], pe[h].w, lds_ld(lb + (uint32_t)(y * W) * 4u));
                        if (x == 0) bd.y += 1u;   // a row start: both candidates agree
                        else bd.y = potts_left(bd.y, pe[h].z, spv[h]);
                        CompactPottsBulk cb;
                        potts_maps_c(bd, cb);
                        potts_steps(bd, cb);
                        const uint32_t e0 = (cb.k0 << 3) & 0xF8F8F8F8u, e1 = (cb.k1 << 3) & 0xF8F8F8F8u;
                        const uint32_t slot = ring0 + (uint32_t)cc * RS + (uint32_t)x * RECB;
                        lds_st4(slot, uu[h]);
                        lds_st4(slot + 16u, make_uint4(cb.a0, cb.a1, e0, e1));
                        lds_st4(slot + 32u, make_uint4(cb.z0, cb.z1, cur[h] ^ pe[h].w, 0u));
                    }
                }
                // publish in order: after batch c - 1 (formed by the previous wave)
                if (!stream_wait(ctr, kCtrFormed, c, l.wait_polls)) {
                    ok = false;
                    break;
                }
                if (lane == 0) lds_st_sync(ctr + kCtrFormed, c + 1u);
            }
        }
    }
    __syncthreads();
    if (tid == 0 && lds_ld_sync(ctr + kCtrAbort)) __hip_atomic_fetch_or(l.status, kStatusWaitExpired, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
    for (int j = tid; j < NW * nch; j += nthreads) {
        const int d = j / nch, c = j - d * nch;
        const uint32_t v = lds_ld(spin0 + (uint32_t)(c * P + d) * 4u);
        g_u8 *g = (g_u8 *)p.spins + (int64_t)(4 * d) * p.C + it.chain0 + c;
        g[0] = (uint8_t)v;
        g[p.C] = (uint8_t)(v >> 8);
        g[2 * (int64_t)p.C] = (uint8_t)(v >> 16);
        g[3 * (int64_t)p.C] = (uint8_t)(v >> 24);
    }
}

__device__ __forceinline__ bool run_potts_fast_if_supported(const ProbDev &p, const WorkItem &it, char *lds,
                                                            const SweepLaunch &l, uint32_t sweep0,
                                                            const LdsPlan &plan) {
    const bool wide = potts_wide_item(p, it);
    switch (p.L) {
    case 16: wide ? run_potts_fast<16, true, false>(p, it, lds, l, sweep0, plan)
                  : run_potts_fast<16, false, false>(p, it, lds, l, sweep0, plan); return true;
    case 24: wide ? run_potts_fast<24, true, false>(p, it, lds, l, sweep0, plan)
                  : run_potts_fast<24, false, false>(p, it, lds, l, sweep0, plan); return true;
    case 32: wide ? run_potts_fast<32, true, false>(p, it, lds, l, sweep0, plan)
                  : run_potts_fast<32, false, false>(p, it, lds, l, sweep0, plan); return true;
    case 48:
        if (stream_potts(p, it)) run_potts_stream<48>(p, it, lds, l, sweep0, plan);
        else run_potts_fast<48, true, true>(p, it, lds, l, sweep0, plan);
        return true;
    default: return false;
    }
}

// ------------------------------------------------------------------ work item driver

template <int MODEL, bool SPIN_LDS, bool TAB_LDS, bool CS>
__device__ __forceinline__ void run_item(const ProbDev &p, const WorkItem &it, char *lds, const SweepLaunch &l,
                                         uint32_t sweep0) {
    const LdsPlan plan = lds_plan(p, it, l.n_producer_waves);
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    const uint32_t lbase = (uint32_t)(size_t)(__attribute__((address_space(3))) char *)lds;
    // stage the table and the lattice
    TabRef<TAB_LDS> tab;
    if constexpr (TAB_LDS) {
        tab.base = lbase + (uint32_t)plan.off_tab;
        // the compact-table walkers build their own (smaller) table in LDS
        if (!(compact_ising(p) && fast_ising_ok(p, l.n_producer_waves)) &&
            !(compact_potts(p) && fast_potts_ok(p, l.n_producer_waves))) {
            const int n = p.trows * p.tcols;
            for (int j = tid; j < n; j += nthreads) lds_st(tab.base + 4u * (uint32_t)j, ((const g_u32 *)p.table)[j]);
        }
    } else {
        tab.base = (const g_u32 *)p.table;
    }
    if ((MODEL == kIsing || MODEL == kIsingMag) && SPIN_LDS && TAB_LDS && fast_ising_ok(p, l.n_producer_waves)) {
        if (run_fast_if_supported<MODEL == kIsingMag, CS>(p, it, lds, l, sweep0, plan)) return;
    }
    if (MODEL == kPotts && SPIN_LDS && TAB_LDS && fast_potts_ok(p, l.n_producer_waves)) {
        if (run_potts_fast_if_supported(p, it, lds, l, sweep0, plan)) return;
    }
    SpinRef<SPIN_LDS> S;
    const int ls = it.spin_stride;
    const uint32_t sp = lbase + (uint32_t)plan.off_spin;   // LDS lattice (SPIN_LDS)
    if constexpr (SPIN_LDS) {
        const int n = p.N * it.nchains;
        for (int j = tid; j < n; j += nthreads) {
            const int site = j / it.nchains, c = j - site * it.nchains;
            *(lds_u8 *)(size_t)(sp + (uint32_t)(((site >> 2) * ls + c) * 4 + (site & 3))) =
                ((const g_u8 *)p.spins)[(int64_t)site * p.C + it.chain0 + c];
        }
        S.base = sp + 4u * (uint32_t)lane;
        S.stride = 4 * ls;
    } else {
        S.base = (g_u8 *)p.spins + it.chain0 + lane;
        S.stride = p.C;
    }
    const uint32_t ring = lbase + (uint32_t)plan.off_ring;

    {
        const int nchunks = (p.N + kChunkSites - 1) / kChunkSites;
        const int total_chunks = nchunks * l.n_sweeps;
        const bool active = (wave == 0) && (lane < it.nchains);
        WalkState st;
        st.row = 0;
        st.m = 0;
        st.k = 0;
        st.x = st.y = st.i = 0;
        if (active) {
            const int k = ((const g_i32 *)p.k)[it.chain0 + lane];
            st.m = ((const g_i32 *)p.m)[it.chain0 + lane];
            st.k = k;
            st.row = (MODEL == kIsing) ? (k >> 1) : (MODEL == kIsingMag) ? (st.m + p.N) / 2 : k;
        }
        if (l.n_producer_waves == 0) {
            __syncthreads();
            if (active)
                for (int t = 0; t < total_chunks; ++t)
                    walk_chunk<MODEL, SPIN_LDS, TAB_LDS, true>(p, it, S, tab, ring, st, t, nchunks, sweep0, lane,
                                                               l.record);
        } else {
            const int ptid = tid - 64;
            const int nprod = nthreads - 64;
            if (wave > 0) produce_chunk<MODEL>(p, it, ring, 0, nchunks, sweep0, ptid, nprod);
            __syncthreads();
            for (int t = 0; t < total_chunks; ++t) {
                if (wave == 0) {
                    if (active)
                        walk_chunk<MODEL, SPIN_LDS, TAB_LDS, false>(p, it, S, tab, ring, st, t, nchunks, sweep0,
                                                                    lane, l.record);
                } else if (t + 1 < total_chunks) {
                    produce_chunk<MODEL>(p, it, ring, t + 1, nchunks, sweep0, ptid, nprod);
                }
                __syncthreads();
            }
        }
        if (active) {
            ((g_i32 *)p.k)[it.chain0 + lane] = (MODEL == kIsing) ? 2 * st.row : (MODEL == kIsingMag) ? st.k : st.row;
            ((g_i32 *)p.m)[it.chain0 + lane] = st.m;
        }
    }
    if constexpr (SPIN_LDS) {
        __syncthreads();
        const int n = p.N * it.nchains;
        for (int j = tid; j < n; j += nthreads) {
            const int site = j / it.nchains, c = j - site * it.nchains;
            ((g_u8 *)p.spins)[(int64_t)site * p.C + it.chain0 + c] =
                *(const lds_u8 *)(size_t)(sp + (uint32_t)(((site >> 2) * ls + c) * 4 + (site & 3)));
        }
    }
}

// One instantiation with the streamed Ising walkers on bit lattices (CS) and
// one without: their code, compiled into the same kernel, slows the other
// walkers by about 2 %, so launches without such items use the kernel
// without it.
template <bool CS>
__global__ void __launch_bounds__(64 * (1 + kMaxProducerWaves)) sweep_kernel(SweepLaunch l) {
    extern __shared__ __align__(16) char lds[];
    const WorkItem it = l.items[blockIdx.x];
    const ProbDev p = l.probs[it.prob];
    const uint32_t sweep0 = *l.sweep_ctr;
    if (p.model == kIsing) {
        if (p.spin_lds) {
            if (p.table_lds) run_item<kIsing, true, true, CS>(p, it, lds, l, sweep0);
            else run_item<kIsing, true, false, CS>(p, it, lds, l, sweep0);
        } else {
            if (p.table_lds) run_item<kIsing, false, true, CS>(p, it, lds, l, sweep0);
            else run_item<kIsing, false, false, CS>(p, it, lds, l, sweep0);
        }
    } else if (p.model == kIsingMag) {
        if (p.spin_lds) {
            if (p.table_lds) run_item<kIsingMag, true, true, CS>(p, it, lds, l, sweep0);
            else run_item<kIsingMag, true, false, CS>(p, it, lds, l, sweep0);
        } else {
            if (p.table_lds) run_item<kIsingMag, false, true, CS>(p, it, lds, l, sweep0);
            else run_item<kIsingMag, false, false, CS>(p, it, lds, l, sweep0);
        }
    } else {
        if (p.spin_lds) {
            if (p.table_lds) run_item<kPotts, true, true, CS>(p, it, lds, l, sweep0);
            else run_item<kPotts, true, false, CS>(p, it, lds, l, sweep0);
        } else {
            if (p.table_lds) run_item<kPotts, false, true, CS>(p, it, lds, l, sweep0);
            else run_item<kPotts, false, false, CS>(p, it, lds, l, sweep0);
        }
    }
}

__global__ void advance_kernel(uint32_t *ctr, uint32_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += n;
}

// ------------------------------------------------------------------ merge

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// H[k] = sum_c hist[k][c] (Sec. 2: the chains' histograms are summed), and
// the production |M| sums likewise; optionally clears what it read.
__global__ void __launch_bounds__(256) merge_kernel(const ProbDev *probs, const MergeItem *items, int production,
                                                     int clear) {
    __shared__ int64_t red[2][4];
    const MergeItem it = items[blockIdx.x];
    const ProbDev p = probs[it.prob];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int b = it.bin0; b < it.bin0 + it.nb; ++b) {
        int32_t *h = p.hist + (int64_t)b * p.C;
        int64_t s = 0, sa = 0;
        for (int c = tid; c < p.C; c += 256) {
            s += h[c];
            if (clear) h[c] = 0;
        }
        if (production && p.sabs) {
            int64_t *a = p.sabs + (int64_t)b * p.C;
            for (int c = tid; c < p.C; c += 256) {
                sa += a[c];
                if (clear) a[c] = 0;
            }
        }
        s = wave_sum(s);
        sa = wave_sum(sa);
        if (lane == 0) {
            red[0][wave] = s;
            red[1][wave] = sa;
        }
        __syncthreads();
        if (tid == 0) {
            p.H[b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
            if (production) p.S[b] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        }
        __syncthreads();
    }
}

__global__ void fill_u32_kernel(uint32_t *dst, uint32_t v, size_t n) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x)
        dst[j] = v;
}

__global__ void copy_bytes_kernel(uint8_t *dst, const uint8_t *src, size_t n) {
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x)
        dst[j] = src[j];
}

// ------------------------------------------------------------------ reweighting

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Eq. (2) over energy bins, one workgroup per beta: a bin with n_k
// measurements taken under weight W(E_k) contributes n_k exp(-beta E_k) / W(E_k).
// Outputs <E>/N, beta^2 var(E)/N and <|M|>/N into out[0..2][j].
__global__ void __launch_bounds__(256) reweight_kernel(ProbDev p, const double *betas, int n_betas, double *out) {
    __shared__ double red[4][4];
    const int j = blockIdx.x;
    if (j >= n_betas) return;
    const double beta = betas[j];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double N = (double)p.N;
    const double estep = (p.model == kIsing) ? 2.0 : 1.0;
    // pass 1: largest exponent
    double amax = -INFINITY;
    for (int b = tid; b < p.nbins; b += 256) {
        const int64_t n = p.H[b];
        if (n > 0) {
            const double E = -2.0 * N + estep * b;
            amax = fmax(amax, log((double)n) - p.lnW[b] - beta * E);
        }
    }
    amax = wave_max_d(amax);
    if (lane == 0) red[0][wave] = amax;
    __syncthreads();
    const double A = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
    __syncthreads();
    // pass 2: Z, sum w E, sum of |M| weights
    double z = 0, ze = 0, zm = 0;
    for (int b = tid; b < p.nbins; b += 256) {
        const int64_t n = p.H[b];
        if (n > 0) {
            const double E = -2.0 * N + estep * b;
            const double e0 = -p.lnW[b] - beta * E - A;
            const double w = exp(log((double)n) + e0);
            z += w;
            ze += w * E;
            if (p.model == kIsing) zm += (double)p.S[b] * exp(e0);
        }
    }
    z = wave_sum_d(z);
    ze = wave_sum_d(ze);
    zm = wave_sum_d(zm);
    if (lane == 0) {
        red[0][wave] = z;
        red[1][wave] = ze;
        red[2][wave] = zm;
    }
    __syncthreads();
    const double Z = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double ZE = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const double ZM = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    const double em = ZE / Z;
    __syncthreads();
    // pass 3: variance about the mean (two-pass)
    double zv = 0;
    for (int b = tid; b < p.nbins; b += 256) {
        const int64_t n = p.H[b];
        if (n > 0) {
            const double E = -2.0 * N + estep * b;
            const double w = exp(log((double)n) - p.lnW[b] - beta * E - A);
            zv += w * (E - em) * (E - em);
        }
    }
    zv = wave_sum_d(zv);
    if (lane == 0) red[3][wave] = zv;
    __syncthreads();
    if (tid == 0) {
        const double var = (red[3][0] + red[3][1] + red[3][2] + red[3][3]) / Z;
        out[j] = em / N;
        out[n_betas + j] = beta * beta * var / N;
        out[2 * n_betas + j] = (p.model == kIsing) ? ZM / Z / N : __builtin_nan("");
    }
}

// ------------------------------------------------------------------ launchers

static int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_init(const ProbDev &p, int chain_begin, int n_chains, hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, dim3(grid_for((int64_t)p.N * n_chains, 256)), dim3(256), 0, s, p, chain_begin,
                       n_chains);
    return hipGetLastError();
}

hipError_t launch_energy(const ProbDev &p, hipStream_t s) {
    hipLaunchKernelGGL(energy_kernel, dim3(grid_for(p.C, 64)), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t configure_sweep_kernel(int max_lds_bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_kernel<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_kernel<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
}

hipError_t launch_sweep(const SweepLaunch &l, bool streamed_compact_ising, hipStream_t s) {
    const int threads = 64 * (1 + l.n_producer_waves);
    if (streamed_compact_ising)
        hipLaunchKernelGGL(sweep_kernel<true>, dim3(l.n_items), dim3(threads), l.lds_bytes, s, l);
    else
        hipLaunchKernelGGL(sweep_kernel<false>, dim3(l.n_items), dim3(threads), l.lds_bytes, s, l);
    return hipGetLastError();
}

hipError_t launch_advance(uint32_t *ctr, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, ctr, n);
    return hipGetLastError();
}

hipError_t launch_merge(const ProbDev *probs, const MergeItem *items, int n_items, int production, int clear,
                        hipStream_t s) {
    hipLaunchKernelGGL(merge_kernel, dim3(n_items), dim3(256), 0, s, probs, items, production, clear);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *dst, uint32_t v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for((int64_t)n, 256)), dim3(256), 0, s, dst, v, n);
    return hipGetLastError();
}

hipError_t launch_copy_bytes(void *dst, const void *src, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(copy_bytes_kernel, dim3(grid_for((int64_t)n, 256)), dim3(256), 0, s, (uint8_t *)dst,
                       (const uint8_t *)src, n);
    return hipGetLastError();
}

hipError_t launch_reweight(const ProbDev &p, const double *betas, int n_betas, double *out, hipStream_t s) {
    hipLaunchKernelGGL(reweight_kernel, dim3(n_betas), dim3(256), 0, s, p, betas, n_betas, out);
    return hipGetLastError();
}

}  // namespace muca
