// kernels.h -- device data layout shared by the kernels and the host engine.
//
// Every matrix of an instance (one per lowered non-terminal) is a dense bit
// matrix over n x n, stored twice when the productions need both (Section 3,
// optimisation 2): R (row-major: row i holds bit j for pair (i, j)) and C
// (column-major: row j holds bit i).  A row is Wp = 64 * S words of 64 bits,
// cut into S segments of 64 words (4096 columns); one wave of 64 lanes owns
// one segment, one word per lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cflr {

constexpr uint32_t kWave = 64;        // lanes per wavefront (CDNA)
constexpr uint32_t kSegWords = 64;    // words per row segment
constexpr uint32_t kCountShards = 64;   // counters per instance for new pairs

// Product tiling.  The new pairs of an operand are sorted by (key tile,
// partner), the key being the row i of a pair (i, k) of dA or the column j
// of a pair (k, j) of dB, and the partner the other index k.  One work item
// is (production part, tile of kTileKeys keys, row segment, at most
// `chunk` pairs, by default kChunkPairs): a workgroup of kProdWaves waves keeps the accumulators
// of the tile's keys in LDS; a partner segment is read once per run of
// pairs that share it (within a window of 64 pairs), not once per pair.
constexpr uint32_t kTileKeys = 256;
constexpr uint32_t kProdWaves = 16;
constexpr uint32_t kKeysPerWave = kTileKeys / kProdWaves;  // keys each wave flushes
constexpr uint32_t kChunkPairs = 1u << 20;
static_assert(kSegWords % kProdWaves == 0, "each product wave takes whole words of a segment");
__host__ __device__ inline uint32_t key_tiles(uint32_t n) { return (n + kTileKeys - 1) / kTileKeys; }

// Key of an appended pair: bits 0..15 matrix, bits 16..29 instance slot.
// kHole marks an unused slot.
constexpr uint32_t kHole = 0xFFFFFFFFu;
constexpr uint32_t kMaxSlots = 0x3FFFu;
constexpr uint32_t kMaxMats = 0x10000u;
__host__ __device__ inline uint32_t pair_key(uint32_t slot, uint32_t mat) { return (slot << 16) | mat; }
__host__ __device__ inline uint32_t key_slot(uint32_t key) { return (key >> 16) & kMaxSlots; }
__host__ __device__ inline uint32_t key_mat(uint32_t key) { return key & 0xFFFFu; }

// Segment masks: word r of Rm has bit s % 64 set when segment s of row r of
// R may hold a pair; a clear bit means every segment s' with s' % 64 == s
// of that row is zero.  Bits are set together with the pairs (seeding and
// the product's flush) and never cleared, so at the start of a round the
// masks cover every pair derived before it; the product uses them to skip
// partner segments that are zero.  Cm is the same for the rows of C.
struct MatDev {
    uint64_t *R;    // row-major bits (always present)
    uint64_t *C;    // column-major copy (null when no production needs it)
    uint64_t *Rm;   // n mask words for R
    uint64_t *Cm;   // n mask words for C (null with C)
    uint32_t sort;  // kSortRows: new pairs needed in row order (the matrix
                    // stands in an a slot); kSortCols: in column order (b slot)
    uint16_t rrank;  // index among the instance's matrices sorted in row order
    uint16_t crank;  // index among those sorted in column order
};
constexpr uint32_t kSegCols = kSegWords * 64;  // columns per row segment
// mask bit of the segment holding column (or row) index x
__host__ __device__ inline uint64_t seg_flag(uint32_t x) { return 1ull << ((x / kSegCols) & 63); }
constexpr uint32_t kSortRows = 1u, kSortCols = 2u;

struct InstDev {
    uint32_t n;        // vertices
    uint32_t S;        // segments per row; Wp = 64 * S
    uint32_t bbase;    // first sort bucket of this instance: in the row-order
                       // counters, matrix x (row rank r), key tile t, partner
                       // segment s (partners s*4096 .. s*4096+4095) is bucket
                       // bbase + (r * key_tiles(n) + t) * S + s; the column-order
                       // counters use the column rank
    uint32_t mat_off;  // first MatDev of this instance
};

// Sort buckets of pair (i, j) of matrix M: row order by (key tile of i,
// partner segment of j), column order by (key tile of j, partner segment of i).
__host__ __device__ inline uint32_t row_bucket(const InstDev &I, const MatDev &M, uint32_t i, uint32_t j) {
    return (uint32_t)(I.bbase + ((uint64_t)M.rrank * key_tiles(I.n) + i / kTileKeys) * I.S + j / kSegCols);
}
__host__ __device__ inline uint32_t col_bucket(const InstDev &I, const MatDev &M, uint32_t i, uint32_t j) {
    return (uint32_t)(I.bbase + ((uint64_t)M.crank * key_tiles(I.n) + j / kTileKeys) * I.S + i / kSegCols);
}

// One (instance, production, part) of a round; part 0 = rows of the new
// pairs of a times B (row by row), part 1 = A times the new pairs of b
// (column by column).  The parts of a round run as two launches, every
// part 0 first: a pair that part 0 derives is in both copies of its matrix
// before part 1 starts, so the two parts never both report one pair.
struct EntryDev {
    uint32_t inst, c, a, b, part;
};


// A unit of product work: one key tile of one (instance, production, part),
// with everything a work item needs, so that it is read in one round trip.
struct UnitDev {
    EntryDev e;
    uint32_t tile;
    uint32_t rank;        // the sorted operand's rank in its order (row rank of a, column rank of b)
    uint32_t start, cnt;  // its new pairs in the sorted order (set by the prep each round)
    InstDev I;
};

// ------------------------------------------------------------ kernel arguments

struct ProductArgs {
    const MatDev *mats;
    const UnitDev *units;
    const uint64_t *item_prefix;  // exclusive prefix of items per unit; [nunit] = total
    uint32_t unit_lo, unit_hi;    // units of this launch (all of one part)
    const uint64_t *rs;           // new pairs (i, k) in (i tile, k) order, packed (i << 32) | k
    const uint64_t *cs;           // new pairs (k, j) in (j tile, k) order, packed (j << 32) | k
    uint32_t *ap_key, *ap_i, *ap_j;   // appended new pairs: (key, i, j)
    unsigned long long *ap_count;
    uint64_t ap_cap;
    uint32_t *inst_overflow;       // per instance: an append did not fit
    uint32_t *halt;                // any overflow: later kernels of the round skip
    unsigned long long *work_counter;  // items taken by this launch
    unsigned long long *inst_new;  // [slot * kCountShards + shard]: new pairs of the round
    // traffic accounting (STATS): first-touch bits per (matrix, layout, row, segment)
    uint32_t *touched;             // bit array
    const uint64_t *touched_off;   // per instance: bit offset of its matrices
    unsigned long long *algo_bytes;
    uint32_t chunk;  // pairs per work item at most (as in the prep)
    uint32_t *rcnt, *ccnt;  // sort counters: the new pairs are counted into their buckets
};

struct PrepArgs {
    UnitDev *units;
    uint32_t nunit;
    const uint32_t *rptr, *cptr;  // bucket starts of the two sort orders
    uint64_t *item_prefix;
    unsigned long long *work_counter0, *work_counter1;  // reset for the two launches
    const uint32_t *halt;
    uint32_t chunk;  // pairs per work item at most
    uint64_t ap_cap;  // sorted pairs the buffers hold (ranges are clamped to it)
};

struct SortArgs {
    const InstDev *inst;
    const MatDev *mats;
    const uint32_t *ap_key, *ap_i, *ap_j;
    const unsigned long long *ap_count;
    uint64_t ap_cap;
    uint32_t *rcnt, *ccnt;       // per bucket: counts -> inclusive scan -> starts (after scatter)
    uint64_t *rs_stage, *cs_stage;  // pairs grouped by bucket (second pass: ordered by partner)
    uint64_t *rs, *cs;
    const uint32_t *halt;
};

struct SeedArgs {
    MatDev *mats;  // this instance's matrices (device array)
    InstDev I;
    uint32_t inst;
    const uint32_t *src, *dst, *lab;
    uint64_t m;
    const uint32_t *lm_ptr, *lm_mat;  // graph label -> matrices with x -> label
    const uint32_t *eps_mat;
    uint32_t n_eps;
    uint32_t *ap_key, *ap_i, *ap_j;
    unsigned long long *ap_count;
    uint64_t ap_cap;
    unsigned long long *inst_new;
    uint32_t *inst_overflow;
    uint32_t *rcnt, *ccnt;  // sort counters (each seeded pair is counted)
};

// Per-instance round bookkeeping kept on the device, so that several rounds
// can be replayed (hipGraph) between host checks.
struct SlotStats {
    uint32_t rounds;               // rounds run until (and including) the empty one
    uint32_t done;                 // a round derived nothing: converged
    unsigned long long new_total;  // pairs derived by all rounds
    unsigned long long max_delta;  // most pairs derived in one round
};

// ------------------------------------------------------------------ launchers

// grid: workgroups of kProdWaves waves
hipError_t launch_product(const ProductArgs &A, uint32_t grid, bool stats, hipStream_t s);
hipError_t launch_prep(const PrepArgs &A, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *a, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *a, uint64_t n, unsigned long long v, hipStream_t s);
// zero the sort counters [0, len) of both orders (skipped once halted)
hipError_t launch_zero_counts(uint32_t *rcnt, uint32_t *ccnt, uint64_t len, const uint32_t *halt, hipStream_t s);
// counting sort of the appended pairs over buckets [0, nbuckets] (nbuckets + 1
// counters, already holding the counts): scan, scatter, order by partner
hipError_t launch_sort(const SortArgs &A, uint64_t nbuckets, uint32_t *bsum, uint32_t sort_grid,
                       hipStream_t s);
uint32_t scan_block_count(uint64_t nbuckets);
hipError_t launch_round_end(const uint32_t *active, unsigned long long *inst_new, SlotStats *st, uint32_t nslots,
                            const uint32_t *halt, hipStream_t s);
hipError_t launch_reset_appends(unsigned long long *ap_count, const uint32_t *halt, hipStream_t s);
hipError_t launch_purge_slot(uint32_t *ap_key, const unsigned long long *ap_count, uint64_t ap_cap,
                             uint32_t slot, uint32_t grid, hipStream_t s);
hipError_t launch_seed(const SeedArgs &A, hipStream_t s);
hipError_t launch_extract_all(const MatDev *mats, const InstDev &I, uint32_t slot, uint32_t nmat,
                              uint32_t *ap_key,
                              uint32_t *ap_i, uint32_t *ap_j, unsigned long long *ap_count,
                              uint64_t ap_cap, uint32_t *overflow, uint32_t *rcnt, uint32_t *ccnt,
                              hipStream_t s);
hipError_t launch_row_count(const uint64_t *R, uint32_t n, uint32_t S, uint32_t *cnt,
                            unsigned long long *total, hipStream_t s);
hipError_t launch_row_write(const uint64_t *R, uint32_t n, uint32_t S, const uint32_t *cnt,
                            uint64_t *off, uint32_t *src, uint32_t *dst, hipStream_t s);

}  // namespace cflr
