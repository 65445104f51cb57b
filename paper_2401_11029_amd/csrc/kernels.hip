// kernels.hip -- HIP kernels for gfx950 (CDNA4, wave64).
//
// One round of the semi-naive fixpoint (Section 3, optimisations 1 and 2):
// for every binary production c -> a b,
//
//     New_c = ((dA . B) U (A . dB)) \ M_c,      M_c <- M_c U New_c,
//
// where dA, dB are the pairs added to a and b in the previous round.  The
// paper's identity M.M = (M_old.dM) U (dM.M) U (M_old.M_old) is used with A in
// place of A_old in the second product; that only repeats dA.dB, which the
// first product already covers, and saves materialising M_old.
//
// Kernels:
//   product_kernel  persistent; one workgroup of 16 waves per work item =
//                   (instance, production, part, key tile of 256 rows or
//                   columns, row segment of 4096 columns, chunk of new pairs).
//                   The tile's accumulators live in LDS; part 0 ORs the B row
//                   segments named by the tile's dA pairs (i, k) into the
//                   accumulator of row i, part 1 the A column segments named
//                   by dB pairs (k, j) into that of column j, skipping
//                   partner segments whose mask says they are zero.  The
//                   flush masks each accumulator with M_c, ORs it in with
//                   64-bit atomics whose return value identifies the
//                   genuinely new bits, keeps the other layout and the
//                   segment masks in step, and appends the new pairs.
//   seed kernels    edges and eps rules -> initial pairs (Algorithm 1's
//                   seeding, and (i, i) for every x -> eps).
//   sort kernels    two-level counting sort of the appended pairs into row
//                   order and column order, grouped by (key tile, partner)
//                   (the next round's dA and dB).
//   readout         bit rows -> (i, j) pairs in (i, j) order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace cflr {

// ------------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t rdlane(uint32_t v, uint32_t l) {
    return __builtin_amdgcn_readlane(v, l);
}
__device__ __forceinline__ uint32_t first_lane(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t first_lane64(uint64_t v) {
    return ((uint64_t)first_lane((uint32_t)(v >> 32)) << 32) | first_lane((uint32_t)v);
}

// exclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t *total) {
    const uint32_t lane = lane_id();
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x += y;
    }
    *total = rdlane(x, 63);
    return x - v;
}

// 64-bit value of lane l (each lane its own l; every lane must take part)
__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t l) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, (int)l, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), (int)l, 64);
    return ((uint64_t)hi << 32) | lo;
}


__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    uint32_t t;
    wave_excl_scan(v, &t);
    return t;
}

// ----------------------------------------------------------- product kernel

// Matrices live in device global memory; loads through this type compile to
// global_load (not flat_load, which also counts against the LDS/scalar
// wait counter and serialises a batch of loads).
typedef const uint64_t __attribute__((address_space(1))) *global_u64;


// Slots of the append buffer are taken from the global counter in chunks
// per wave, so one device-scope atomic serves many flushes.  Unused slots of
// a chunk are marked as holes when the wave moves to a new chunk or exits.
constexpr uint32_t kSlotChunk = 1024;

struct SlotChunk {
    uint64_t pos = 0, end = 0;  // wave-uniform
    uint64_t bytes = 0;         // traffic accounting (lane 0), added once at exit
};

__device__ __forceinline__ void retire_chunk(const ProductArgs &A, SlotChunk &ch) {
    for (uint64_t x = ch.pos + lane_id(); x < ch.end; x += kWave) A.ap_key[x] = kHole;
    ch.pos = ch.end;
}

// Reserve `need` slots for this lane (wave-aggregated).  Returns false if
// the buffer is full: the instance is flagged, the caller leaves M
// untouched, and the host grows the buffer and re-runs the round.
__device__ __forceinline__ bool reserve_slots(const ProductArgs &A, SlotChunk &ch, uint32_t inst,
                                              uint32_t need, uint64_t *pos) {
    uint32_t total;
    uint32_t pre = wave_excl_scan(need, &total);
    *pos = 0;
    if (total == 0) return true;
    if (ch.pos + total > ch.end) {
        retire_chunk(A, ch);
        const uint64_t want = total > kSlotChunk ? total : kSlotChunk;
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(A.ap_count, (unsigned long long)want);
        base = first_lane64(base);
        if (base + want > A.ap_cap) {
            for (uint64_t x = base + lane_id(); x < A.ap_cap && x < base + want; x += kWave)
                A.ap_key[x] = kHole;
            if (lane_id() == 0) {
                atomicOr(&A.inst_overflow[inst], 1u);
                atomicOr(A.halt, 1u);
            }
            return false;
        }
        ch.pos = base;
        ch.end = base + want;
    }
    *pos = ch.pos + pre;
    ch.pos += total;
    return true;
}

template <bool STATS>
__device__ __forceinline__ bool first_touch(const ProductArgs &A, uint32_t inst, uint32_t mat,
                                            uint32_t layout, uint32_t row, uint32_t seg,
                                            const InstDev &I) {
    uint64_t bit = A.touched_off[inst] +
                   (((uint64_t)mat * 2 + layout) * I.n + row) * I.S + seg;
    uint32_t m = 1u << (bit & 31);
    uint32_t old = atomicOr(&A.touched[bit >> 5], m);
    return !(old & m);
}

// Append the candidates of one key: slots [base + pre_l, base + pre_l +
// popc(cand_l)) belong to lane l.  The wave fills them together, 64
// consecutive slots per pass: slot t goes to lane t % 64, which finds the
// lane and the bit that own it (binary searches over the lanes' prefix sums
// and over the bits of the word), so the stores are contiguous.  A
// candidate that turned out not to be new leaves a hole.  (The other layout
// is updated for the whole tile afterwards, other_layout_tile.)
template <bool COL>
__device__ __forceinline__ void append_key(const ProductArgs &A, uint32_t k, uint32_t key, uint32_t seg,
                                           uint64_t cand, uint64_t fresh, uint64_t base, uint32_t pre,
                                           uint32_t total) {
    const uint32_t lane = lane_id();
    for (uint32_t r = 0; r < total; r += kWave) {
        const uint32_t t = r + lane;
        uint32_t src = 0;  // last lane whose first slot is <= t
#pragma unroll
        for (uint32_t step = 32; step; step >>= 1) {
            const uint32_t probe = src + step;
            if ((uint32_t)__shfl(pre, probe, 64) <= t) src = probe;
        }
        const uint64_t word = shfl64(cand, src);
        const uint64_t fresh_bits = shfl64(fresh, src);
        uint32_t rank = t - (uint32_t)__shfl(pre, src, 64);
        uint32_t b = 0;  // position of the rank-th set bit of word
#pragma unroll
        for (uint32_t width = 32; width; width >>= 1) {
            const uint32_t c2 = (uint32_t)__popcll((word >> b) & ((1ull << width) - 1));
            if (rank >= c2) {
                rank -= c2;
                b += width;
            }
        }
        if (t < total) {
            const uint64_t slot = base + t;
            if ((fresh_bits >> b) & 1) {
                const uint32_t x = (seg * kSegWords + src) * 64 + b;  // the other index of the pair
                A.ap_key[slot] = k;
                A.ap_i[slot] = COL ? x : key;
                A.ap_j[slot] = COL ? key : x;
            } else {
                A.ap_key[slot] = kHole;
            }
        }
    }
}

// LDS of the product workgroup: the accumulators of the tile's keys for the
// item's row segment (kept all zero between items).
struct ProductShared {
    // rows padded by one word, so that the column reads of other_layout_tile
    // spread over the banks
    uint64_t acc[kTileKeys][kSegWords + 1];
    unsigned long long item;  // the workgroup's current item
    uint32_t unit;            // and its unit
    uint32_t next_window;     // windows of the item taken so far
};

// Zero the accumulator rows of the live keys of one flush group.
__device__ __forceinline__ void clear_rows(ProductShared &sh, uint32_t wave, uint32_t g0, uint32_t live) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t q = 0; q < 8; q++)
        if ((live >> q) & 1) sh.acc[wave + kProdWaves * (g0 + q)][lane] = 0;
}

// Transpose of a 64 x 64 bit block held one row per lane: afterwards lane b
// holds column b (bit l = bit b of lane l's row).  Six butterfly stages, each
// swapping the off-diagonal sub-blocks of size s between lanes l and l ^ s.
__device__ __forceinline__ uint64_t transpose64(uint64_t v) {
    const uint32_t lane = lane_id();
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (uint32_t st = 0; st < 6; st++) {
        const uint32_t s = 32u >> st;
        const uint64_t m = masks[st];
        const uint64_t p = shfl64(v, lane ^ s);
        v = (lane & s) ? (((p >> s) & m) | (v & ~m)) : ((v & m) | ((p & m) << s));
    }
    return v;
}

// The other layout's update for a whole tile, after the flush left each
// key's new bits in its accumulator row: wave w takes the column words
// 4w .. 4w + 3 of the segment; for each and each group of 64 keys it
// transposes the 64 x 64 block, so that lane b holds, for other index
// x = 64 (64 seg + word) + b, the word of its other-layout row that covers
// those 64 keys, and ORs it in with one atomic (instead of one per pair);
// the four key groups of x are adjacent words.  The same pass sets the
// other layout's segment mask of every x that gained a pair (read first,
// set only where missing) and zeroes what it read.
template <bool COL>
__device__ __forceinline__ void other_layout_tile(ProductShared &sh, const MatDev &Mc, uint32_t key0,
                                                  uint32_t seg, uint64_t Wp) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint64_t *other = COL ? Mc.R : Mc.C;
    uint64_t *other_mask = COL ? Mc.Rm : Mc.Cm;
    const uint64_t flag = seg_flag(key0);
#pragma unroll 1
    for (uint32_t r = 0; r < kSegWords / kProdWaves; r++) {
        const uint32_t w = wave * (kSegWords / kProdWaves) + r;
        const uint32_t x = (seg * kSegWords + w) * 64 + lane;
        uint64_t any = 0;
#pragma unroll
        for (uint32_t g = 0; g < kTileKeys / 64; g++) {
            uint64_t v = sh.acc[g * 64 + lane][w];
            if (!__ballot(v != 0)) continue;
            sh.acc[g * 64 + lane][w] = 0;
            v = transpose64(v);
            if (v) atomicOr((unsigned long long *)&other[(uint64_t)x * Wp + (key0 >> 6) + g], (unsigned long long)v);
            any |= v;
        }
        if (any && !(other_mask[x] & flag)) atomicOr((unsigned long long *)&other_mask[x], (unsigned long long)flag);
    }
}

// Flush of the wave's keys kl = wave + 16 q of the tile: each accumulator
// word holds candidate bits of row `key` (COL = false: pairs (key, j), the
// row-major copy is the authority) or of column `key` (COL = true: pairs
// (i, key), the column-major copy).  The authority segments of all the
// wave's keys are read at once, append slots are reserved once for the
// wave, and the returning 64-bit atomic ORs that tell which candidates are
// new are issued back to back (in groups of eight keys); then the new pairs
// are appended, set in the other layout and counted for the instance.  Every
// accumulator row is left zero, also after an overflow.
template <bool COL, bool STATS>
__device__ __forceinline__ void flush_keys(const ProductArgs &A, ProductShared &sh, SlotChunk &ch,
                                           uint32_t inst, const InstDev &I, const MatDev &Mc, uint32_t c,
                                           uint32_t key0, uint32_t seg, uint64_t Wp) {
    constexpr uint32_t kGroup = 8;  // keys whose round trips overlap
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t w = seg * kSegWords + lane;
    uint64_t *own = COL ? Mc.C : Mc.R;
    uint64_t *own_mask = COL ? Mc.Cm : Mc.Rm;
    const uint32_t k = pair_key(inst, c);
    uint32_t fresh = 0;
    bool failed = false;  // an append did not fit: later groups only clear their accumulators
#pragma unroll 1
    for (uint32_t g0 = 0; g0 < kKeysPerWave; g0 += kGroup) {
        uint64_t cand[kGroup], old[kGroup];
        uint32_t live = 0;  // keys with a non-zero accumulator (the same in every lane)
#pragma unroll
        for (uint32_t q = 0; q < kGroup; q++) {
            const uint32_t kl = wave + kProdWaves * (g0 + q);
            cand[q] = sh.acc[kl][lane];
            const uint64_t lanes = __ballot(cand[q] != 0);
            if (lanes) {
                live |= 1u << q;
                if (STATS && lane == 0 && first_touch<STATS>(A, inst, c, COL ? 1 : 0, key0 + kl, seg, I))
                    ch.bytes += 8ull * __popcll(lanes);
            }
        }
        if (!live) continue;
        if (failed) {
            clear_rows(sh, wave, g0, live);
            continue;
        }
#pragma unroll
        for (uint32_t q = 0; q < kGroup; q++) {
            old[q] = 0;
            if ((live >> q) & 1) old[q] = own[(uint64_t)(key0 + wave + kProdWaves * (g0 + q)) * Wp + w];
        }
        uint32_t need = 0;
#pragma unroll
        for (uint32_t q = 0; q < kGroup; q++) {
            cand[q] &= ~old[q];
            need += (uint32_t)__popcll(cand[q]);
        }
        // one reservation for the group's candidates (on overflow nothing
        // is set: the host re-runs the round with a larger buffer)
        uint32_t grand;
        const uint32_t pre_all = wave_excl_scan(need, &grand);
        uint64_t pos;
        if (!reserve_slots(A, ch, inst, need, &pos)) {
            failed = true;
            clear_rows(sh, wave, g0, live);
            continue;
        }
        if (!grand) {
            clear_rows(sh, wave, g0, live);
            continue;
        }
        uint64_t base = first_lane64(pos - pre_all);
#pragma unroll
        for (uint32_t q = 0; q < kGroup; q++)
            if (cand[q])
                old[q] = atomicOr((unsigned long long *)&own[(uint64_t)(key0 + wave + kProdWaves * (g0 + q)) * Wp + w],
                                  (unsigned long long)cand[q]);
#pragma unroll
        for (uint32_t q = 0; q < kGroup; q++) {
            const uint32_t kl = wave + kProdWaves * (g0 + q);
            uint32_t total;
            const uint32_t pre = wave_excl_scan((uint32_t)__popcll(cand[q]), &total);
            const uint64_t nw = cand[q] & ~old[q];
            // the row keeps the new bits for the other layout's update
            if ((live >> q) & 1) sh.acc[kl][lane] = nw;
            if (!total) continue;
            fresh += (uint32_t)__popcll(nw);
            const uint32_t key = key0 + kl;
            if (__ballot(nw != 0) && lane == 0)
                atomicOr((unsigned long long *)&own_mask[key], 1ull << (seg & 63));
            append_key<COL>(A, k, key, seg, cand[q], nw, base, pre, total);
            base += total;
        }
    }
    // count the new pairs into next round's sort buckets: in the key's own
    // order every pair of the item shares one bucket (key tile, this
    // segment); in the other order lane l's pairs share (tile of its 64
    // other indexes, segment of the key), four lanes per tile
    const uint32_t x0 = (seg * kSegWords + lane) * 64;  // lane's first other index
    const uint32_t need = Mc.sort;
    uint32_t group = fresh;
    group += (uint32_t)__shfl_xor((int)group, 1, 64);
    group += (uint32_t)__shfl_xor((int)group, 2, 64);
    fresh = wave_sum(fresh);
    if (!fresh) return;
    if (COL) {
        if ((need & kSortCols) && lane == 0) atomicAdd(&A.ccnt[col_bucket(I, Mc, x0, key0)], fresh);
        if ((need & kSortRows) && (lane & 3) == 0 && group) atomicAdd(&A.rcnt[row_bucket(I, Mc, x0, key0)], group);
    } else {
        if ((need & kSortRows) && lane == 0) atomicAdd(&A.rcnt[row_bucket(I, Mc, key0, x0)], fresh);
        if ((need & kSortCols) && (lane & 3) == 0 && group) atomicAdd(&A.ccnt[col_bucket(I, Mc, key0, x0)], group);
    }
    if (lane == 0) {
        const uint32_t shard = (blockIdx.x * kProdWaves + wave) % kCountShards;
        atomicAdd(&A.inst_new[(uint64_t)inst * kCountShards + shard], (unsigned long long)fresh);
        if (STATS) ch.bytes += 20ull * fresh;
    }
}

constexpr uint32_t kRunBatch = 8;  // partner segments in flight per wave
constexpr uint32_t kWinGroup = 4;  // windows a wave takes at once

// The runs of one window of 64 pairs (lane l holds key key_l and partner
// k_l; `heads` marks the first lane of each run, `todo` the runs whose
// partner segment may be non-zero): their partner segments are loaded, up to
// kRunBatch at a time, and ORed into the accumulators of the run's keys.
template <bool COL, bool STATS>
__device__ __forceinline__ void or_runs(const ProductArgs &A, ProductShared &sh, SlotChunk &ch,
                                        const EntryDev &E, const InstDev &I, uint32_t pm, global_u64 G,
                                        uint64_t Wp, uint32_t seg, uint32_t key, uint32_t k,
                                        uint64_t heads, uint32_t nvalid, uint64_t todo) {
    const uint32_t lane = lane_id();
    const uint32_t row_bytes = (key & (kTileKeys - 1)) * (uint32_t)sizeof(sh.acc[0]);
    char *acc_lane = (char *)&sh.acc[0][lane];
    while (todo) {
        // up to kRunBatch runs: their partner segments requested together
        uint32_t start[kRunBatch];
        uint64_t v[kRunBatch];
        uint32_t nb = 0;
#pragma unroll
        for (uint32_t q = 0; q < kRunBatch; q++) {
            start[q] = 64;
            v[q] = 0;
            if (todo) {
                start[q] = (uint32_t)__ffsll((unsigned long long)todo) - 1;
                todo &= todo - 1;
                nb = q + 1;
                const uint32_t kk = rdlane(k, start[q]);
                v[q] = G[(uint64_t)kk * Wp + seg * kSegWords + lane];
            }
        }
#pragma unroll
        for (uint32_t q = 0; q < kRunBatch; q++) {
            if (q >= nb) break;
            const uint64_t live = __ballot(v[q] != 0);
            if (!live) continue;
            if (STATS && lane == 0 &&
                first_touch<STATS>(A, E.inst, pm, COL ? 1 : 0, rdlane(k, start[q]), seg, I))
                ch.bytes += 8ull * __popcll(live);
            // the run ends where the next run starts (or the window's pairs end)
            const uint64_t later = start[q] == 63 ? 0 : heads & (~0ull << (start[q] + 1));
            const uint32_t end = later ? (uint32_t)__ffsll((unsigned long long)later) - 1 : nvalid;
            // every key of the unit's pairs lies in its tile (they are
            // bucketed by key tile, tiles start at multiples of kTileKeys); the mask
            // keeps the row inside the accumulators without a branch, and
            // the row's byte offset is read straight out of lane t
            for (uint32_t t = start[q]; t < end; t++)
                atomicOr((unsigned long long *)(acc_lane + rdlane(row_bytes, t)), (unsigned long long)v[q]);
        }
    }
}

// One work item: pairs [p0, p1) of one key tile, sorted by partner, against
// row segment `seg`.  COL = false: pairs (i, k) of dA, partner rows k of B
// (row-major); COL = true: pairs (j, k) of dB, partner rows k of A's
// column-major copy.  The waves take kWinGroup windows of 64 consecutive
// pairs at a time from an LDS counter; a wave requests a group's pairs, then
// (one group later) the segment masks of its run heads' partners, and (one
// group later again) loads its runs, so that two groups' requests are in
// flight while it ORs the runs of a third.  In a window, pairs with
// the same partner k are adjacent (a run): only runs whose partner segment
// may be non-zero load it, once per run, and OR it into the LDS accumulator
// of every key of the run (atomic OR in LDS, no return value); a loaded
// segment that is zero after all is skipped too.  After the last window the
// waves flush the tile's keys and zero their accumulators.  Every wave meets
// the two barriers of the item.
template <bool COL, bool STATS>
__device__ __forceinline__ void product_tile(const ProductArgs &A, ProductShared &sh, SlotChunk &ch,
                                             const EntryDev &E, const InstDev &I, uint32_t tile,
                                             uint32_t p0, uint32_t p1, uint32_t seg) {
    const uint32_t lane = lane_id();
    const uint64_t Wp = (uint64_t)I.S * kSegWords;
    const uint32_t pm = COL ? E.a : E.b;
    const MatDev Mp = A.mats[I.mat_off + pm];
    const global_u64 G = (global_u64)(COL ? Mp.C : Mp.R);
    const global_u64 Gm = (global_u64)(COL ? Mp.Cm : Mp.Rm);
    const uint64_t seg_bit = 1ull << (seg & 63);
    const uint64_t *pairs = COL ? A.cs : A.rs;
    const uint32_t key0 = tile * kTileKeys;
    const uint32_t nwin = (p1 - p0 + kWave - 1) / kWave;
    // Two-stage pipeline per wave: while the runs of the current group of
    // windows are ORed, the segment masks of the next group and the pairs of
    // the group after it are in flight.
    constexpr uint32_t P = kWinGroup;
    uint32_t wr = 0;  // group whose pairs are being loaded
    if (lane == 0) wr = atomicAdd(&sh.next_window, P);
    wr = first_lane(wr);
    uint64_t raw[P];
#pragma unroll
    for (uint32_t q = 0; q < P; q++) {
        const uint64_t x = (uint64_t)p0 + (uint64_t)(wr + q) * kWave + lane;
        raw[q] = ~0ull;
        if (x < p1) raw[q] = pairs[x];
    }
    uint32_t wn = wr;  // group decoded, masks in flight
    uint32_t kn[P], pn[P], nvn[P];
    uint64_t hn[P], mn[P];
#pragma unroll
    for (uint32_t q = 0; q < P; q++) {
        kn[q] = (uint32_t)(raw[q] >> 32);
        pn[q] = (uint32_t)raw[q];
        const bool valid = (uint64_t)p0 + (uint64_t)(wn + q) * kWave + lane < p1 && pn[q] < I.n;
        const uint32_t kprev = __shfl_up(pn[q], 1, 64);
        const bool head = valid && (lane == 0 || pn[q] != kprev);
        hn[q] = __ballot(head);
        nvn[q] = (uint32_t)__popcll(__ballot(valid));
        mn[q] = head ? Gm[pn[q]] : 0ull;
    }
    if (wn < nwin) {
        if (lane == 0) wr = atomicAdd(&sh.next_window, P);
        wr = first_lane(wr);
#pragma unroll
        for (uint32_t q = 0; q < P; q++) {
            const uint64_t x = (uint64_t)p0 + (uint64_t)(wr + q) * kWave + lane;
            raw[q] = ~0ull;
            if (x < p1) raw[q] = pairs[x];
        }
    }
    while (wn < nwin) {
        // the current group: its runs to load, from the gathered masks
        uint32_t kc[P], pc[P], nvc[P];
        uint64_t hc[P], tc[P];
#pragma unroll
        for (uint32_t q = 0; q < P; q++) {
            kc[q] = kn[q];
            pc[q] = pn[q];
            nvc[q] = nvn[q];
            hc[q] = hn[q];
            tc[q] = __ballot(((hn[q] >> lane) & 1) && (mn[q] & seg_bit));
        }
        if (STATS && seg == 0 && lane == 0) {
            // the pairs themselves, read once per production
            uint32_t taken = 0;
#pragma unroll
            for (uint32_t q = 0; q < P; q++) taken += nvc[q];
            ch.bytes += 8ull * taken;
        }
        // the next group: decoded, its masks requested
        wn = wr;
#pragma unroll
        for (uint32_t q = 0; q < P; q++) {
            kn[q] = (uint32_t)(raw[q] >> 32);
            pn[q] = (uint32_t)raw[q];
            const bool valid = (uint64_t)p0 + (uint64_t)(wn + q) * kWave + lane < p1 && pn[q] < I.n;
            const uint32_t kprev = __shfl_up(pn[q], 1, 64);
            const bool head = valid && (lane == 0 || pn[q] != kprev);
            hn[q] = __ballot(head);
            nvn[q] = (uint32_t)__popcll(__ballot(valid));
            mn[q] = head ? Gm[pn[q]] : 0ull;
        }
        // the group after it: its pairs requested
        if (wn < nwin) {
            if (lane == 0) wr = atomicAdd(&sh.next_window, P);
            wr = first_lane(wr);
#pragma unroll
            for (uint32_t q = 0; q < P; q++) {
                const uint64_t x = (uint64_t)p0 + (uint64_t)(wr + q) * kWave + lane;
                raw[q] = ~0ull;
                if (x < p1) raw[q] = pairs[x];
            }
        }
        // the current group's runs, while those are in flight
#pragma unroll
        for (uint32_t q = 0; q < P; q++)
            if (tc[q]) or_runs<COL, STATS>(A, sh, ch, E, I, pm, G, Wp, seg, kc[q], pc[q], hc[q], nvc[q], tc[q]);
    }
    __syncthreads();  // every window's ORs are in the accumulators
    flush_keys<COL, STATS>(A, sh, ch, E.inst, I, A.mats[I.mat_off + E.c], E.c, key0, seg, Wp);
    __syncthreads();  // every key's new bits are in its accumulator row
    other_layout_tile<COL>(sh, A.mats[I.mat_off + E.c], key0, seg, Wp);
    // the accumulators are zero again before the next item (its first
    // barrier orders this before any of its ORs)
}

template <bool STATS>
__global__ __launch_bounds__(kProdWaves * kWave) void product_kernel(ProductArgs A) {
    __shared__ ProductShared sh;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id(), wave = tid / kWave;
    const uint64_t first = A.item_prefix[A.unit_lo], total = A.item_prefix[A.unit_hi];
    SlotChunk ch;
    for (uint32_t x = tid; x < kTileKeys * kSegWords; x += kProdWaves * kWave) sh.acc[x / kSegWords][x % kSegWords] = 0;
    // items are taken from a counter, one atomic per workgroup and item; the
    // next one is requested when an item starts, so its round trip overlaps
    // the work.  After an overflow the round is re-run: stop early.
    unsigned long long nxt = 0;
    if (tid == 0) nxt = first + atomicAdd(A.work_counter, 1ull);
    while (true) {
        if (tid == 0) {
            unsigned long long it = nxt;
            if (__hip_atomic_load(A.halt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) it = total;
            sh.item = it;
            sh.next_window = 0;
            if (it < total) nxt = first + atomicAdd(A.work_counter, 1ull);
        }
        __syncthreads();
        const uint64_t item = first_lane64(sh.item);  // uniform: kept in scalar registers
        if (item >= total) break;
        if (wave == 0) {
            // the unit holding the item, item_prefix[lo] <= item < item_prefix[hi]:
            // a 64-way search, one round trip per factor of 64
            uint32_t lo = A.unit_lo, hi = A.unit_hi;
            while (hi - lo > 1) {
                const uint32_t step = (hi - lo + kWave - 1) / kWave;
                const uint32_t probe = lo + lane * step;
                const bool ok = probe < hi && A.item_prefix[probe] <= item;
                const uint64_t m = __ballot(ok);  // lane 0 (probe lo) is always set
                lo += (63 - (uint32_t)__clzll((unsigned long long)m)) * step;
                if (lo + step < hi) hi = lo + step;
            }
            if (lane == 0) sh.unit = lo;
        }
        __syncthreads();  // the unit is known; every thread has read the item
        const uint32_t u = first_lane(sh.unit);
        const UnitDev U = A.units[u];
        const uint64_t local = item - A.item_prefix[u];
        const uint32_t seg = (uint32_t)(local % U.I.S);
        const uint64_t chunk = local / U.I.S;
        const uint64_t end = (uint64_t)U.start + U.cnt;
        const uint64_t c0 = U.start + chunk * A.chunk;
        const uint64_t c1 = c0 + A.chunk < end ? c0 + A.chunk : end;
        if (U.e.part == 0)
            product_tile<false, STATS>(A, sh, ch, U.e, U.I, U.tile, (uint32_t)c0, (uint32_t)c1, seg);
        else
            product_tile<true, STATS>(A, sh, ch, U.e, U.I, U.tile, (uint32_t)c0, (uint32_t)c1, seg);
    }
    retire_chunk(A, ch);
    if (STATS && lane_id() == 0 && ch.bytes) atomicAdd(A.algo_bytes, (unsigned long long)ch.bytes);
}

// ------------------------------------------------------------- work table


// One workgroup of 1024 threads: pairs and items of every unit (entry, key
// tile) and the prefix sum of the items.
__global__ __launch_bounds__(1024) void prep_kernel(PrepArgs A) {
    // once a round has halted, its work table must survive for the host's
    // re-run of that round's product: a later captured round writes nothing
    if (*A.halt) return;
    __shared__ uint64_t part[1024];
    __shared__ uint64_t carry;
    const uint32_t t = threadIdx.x;
    if (t == 0) {
        carry = 0;
        *A.work_counter0 = 0;
        *A.work_counter1 = 0;
    }
    __syncthreads();
    for (uint32_t base = 0; base < A.nunit; base += 1024) {
        const uint32_t u = base + t;
        uint64_t items = 0;
        if (u < A.nunit) {
            UnitDev &U = A.units[u];
            const uint32_t *ptr = U.e.part == 0 ? A.rptr : A.cptr;
            const uint64_t b0 = U.I.bbase + ((uint64_t)U.rank * key_tiles(U.I.n) + U.tile) * U.I.S;
            uint64_t s = ptr[b0], f = ptr[b0 + U.I.S];
            if (f > A.ap_cap) f = A.ap_cap;
            if (s > f) s = f;
            U.start = s;
            U.cnt = f - s;
            items = ((uint64_t)(f - s) + A.chunk - 1) / A.chunk * U.I.S;
        }
        part[t] = items;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {  // inclusive scan (Hillis-Steele)
            uint64_t v = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += v;
            __syncthreads();
        }
        if (u < A.nunit) A.item_prefix[u] = carry + part[t] - items;
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
    if (t == 0) A.item_prefix[A.nunit] = carry;
}

// ------------------------------------------------------------- new-pair sort

__global__ void fill_u32_kernel(uint32_t *a, uint64_t n, uint32_t v) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        a[x] = v;
}

// fill that is skipped once an overflow has halted the round (inside a
// replayed round it must not destroy state the host's re-run still needs)
__global__ void fill_u32_unless_halted_kernel(uint32_t *a, uint64_t n, uint32_t v, const uint32_t *halt) {
    if (*halt) return;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        a[x] = v;
}

__global__ void fill_u64_kernel(unsigned long long *a, uint64_t n, unsigned long long v) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        a[x] = v;
}


// Runs of equal row ids among the 64 lanes of a wave (consecutive buffer
// positions): the appended pairs of one flush share their row (row part) or
// column (column part), so a run takes one atomic and one contiguous range.
struct LaneRun {
    bool head;       // first lane of its run
    uint32_t len;    // run length (head lanes)
    uint32_t first;  // head lane of this lane's run
};

__device__ __forceinline__ LaneRun lane_run(uint32_t rid) {
    const uint32_t lane = lane_id();
    const uint32_t prev = __shfl_up(rid, 1, 64);
    LaneRun r;
    r.head = lane == 0 || rid != prev;
    const uint64_t H = __ballot(r.head);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    r.first = 63 - __clzll((unsigned long long)(H & upto));
    const uint64_t above = H & ~upto;
    const uint32_t nxt = above ? (uint32_t)__ffsll((unsigned long long)above) - 1 : 64;
    r.len = nxt - lane;
    return r;
}

// Buckets of entry x in the two sort orders (kHole when the entry is a hole
// or its matrix needs that order for no production): row order groups pair
// (i, j) by (tile of i, segment of j), column order by (tile of j, segment
// of i); a second pass orders each bucket by the partner (j, resp. i).
__device__ __forceinline__ void entry_rows(const SortArgs &A, uint64_t x, uint64_t n, uint32_t *r, uint32_t *c,
                                           uint32_t *i, uint32_t *j) {
    *r = *c = kHole;
    if (x >= n) return;
    const uint32_t key = A.ap_key[x];
    if (key == kHole) return;
    const InstDev I = A.inst[key_slot(key)];
    const MatDev &M = A.mats[I.mat_off + key_mat(key)];
    const uint32_t need = M.sort;
    *i = A.ap_i[x];
    *j = A.ap_j[x];
    if (need & kSortRows) *r = row_bucket(I, M, *i, *j);
    if (need & kSortCols) *c = col_bucket(I, M, *i, *j);
}

__global__ __launch_bounds__(256) void scatter_kernel(SortArgs A) {
    if (*A.halt) return;
    uint64_t n = *A.ap_count;
    if (n > A.ap_cap) n = A.ap_cap;
    const uint32_t lane = lane_id();
    for (uint64_t x0 = blockIdx.x * (uint64_t)blockDim.x; x0 < n; x0 += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t r, c, i = 0, j = 0;
        entry_rows(A, x0 + threadIdx.x, n, &r, &c, &i, &j);
        const LaneRun rr = lane_run(r), cr = lane_run(c);
        // the counts hold inclusive ends; taking len off the end of a row
        // gives the run a contiguous range, and leaves the row's start
        uint32_t p0 = 0, q0 = 0;
        if (rr.head && r != kHole) p0 = atomicSub(&A.rcnt[r], rr.len) - rr.len;
        if (cr.head && c != kHole) q0 = atomicSub(&A.ccnt[c], cr.len) - cr.len;
        p0 = __shfl(p0, rr.first, 64) + (lane - rr.first);
        q0 = __shfl(q0, cr.first, 64) + (lane - cr.first);
        // (positions outside the buffer would mean counts that disagree with
        // the appended pairs; they are dropped rather than written)
        if (r != kHole && p0 < A.ap_cap) A.rs_stage[p0] = ((uint64_t)i << 32) | j;
        if (c != kHole && q0 < A.ap_cap) A.cs_stage[q0] = ((uint64_t)j << 32) | i;
    }
}

// Second pass: each bucket (key tile, partner segment) of each order is
// ordered by the partner (the low 32 bits of a packed pair; its offset in
// the segment, 12 bits) so that the pairs sharing a partner are adjacent;
// their relative order is arbitrary.  One workgroup per bucket: up to 256
// pairs are ranked by comparison in LDS, larger buckets by a counting sort
// over the 4096 partners of the segment (LDS histogram, block scan).
constexpr uint32_t kSegSortThreads = 1024, kSegSortSmall = 256;
__global__ __launch_bounds__(kSegSortThreads) void segsort_kernel(SortArgs A, uint32_t nbuckets) {
    if (*A.halt) return;
    __shared__ uint32_t hist[kSegCols];
    __shared__ uint64_t small[kSegSortSmall];
    __shared__ uint32_t wsum[kSegSortThreads / kWave];
    const uint32_t *ptr = blockIdx.y ? A.ccnt : A.rcnt;
    const uint64_t *src = blockIdx.y ? A.cs_stage : A.rs_stage;
    uint64_t *dst = blockIdx.y ? A.cs : A.rs;
    const uint32_t t = threadIdx.x, lane = lane_id(), wave = t / kWave;
    for (uint32_t b = blockIdx.x; b < nbuckets; b += gridDim.x) {
        uint32_t s = ptr[b], e = ptr[b + 1];
        if (e > A.ap_cap) e = (uint32_t)A.ap_cap;
        if (e <= s) continue;
        const uint32_t m = e - s;
        if (m <= kSegSortSmall) {
            if (t < m) small[t] = src[s + t];
            __syncthreads();
            if (t < m) {
                const uint64_t v = small[t];
                const uint32_t p = (uint32_t)v & (kSegCols - 1);
                uint32_t rank = 0;
                for (uint32_t u = 0; u < m; u++) {
                    const uint32_t pu = (uint32_t)small[u] & (kSegCols - 1);
                    rank += (pu < p || (pu == p && u < t)) ? 1u : 0u;
                }
                dst[s + rank] = v;
            }
            __syncthreads();
            continue;
        }
        for (uint32_t x = t; x < kSegCols; x += kSegSortThreads) hist[x] = 0;
        __syncthreads();
        for (uint32_t q = s + t; q < e; q += kSegSortThreads)
            atomicAdd(&hist[(uint32_t)src[q] & (kSegCols - 1)], 1u);
        __syncthreads();
        // exclusive scan of the histogram: four bins per thread
        constexpr uint32_t kPer = kSegCols / kSegSortThreads;
        uint32_t c[kPer], sum = 0;
#pragma unroll
        for (uint32_t z = 0; z < kPer; z++) {
            c[z] = hist[t * kPer + z];
            sum += c[z];
        }
        uint32_t wtot;
        const uint32_t wex = wave_excl_scan(sum, &wtot);
        if (lane == 0) wsum[wave] = wtot;
        __syncthreads();
        uint32_t off = wex;
        for (uint32_t w = 0; w < wave; w++) off += wsum[w];
#pragma unroll
        for (uint32_t z = 0; z < kPer; z++) {
            hist[t * kPer + z] = off;
            off += c[z];
        }
        __syncthreads();
        for (uint32_t q = s + t; q < e; q += kSegSortThreads) {
            const uint64_t v = src[q];
            dst[s + atomicAdd(&hist[(uint32_t)v & (kSegCols - 1)], 1u)] = v;
        }
        __syncthreads();
    }
}

// Inclusive scan of two u32 arrays (blockIdx.y selects), 3 phases.
constexpr uint32_t kScanThreads = 256, kScanItems = 16, kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(256) void scan_reduce_kernel(uint32_t *a0, uint32_t *a1, uint64_t n,
                                                          uint32_t *bsum, uint32_t nblk,
                                                          const uint32_t *halt) {
    if (halt && *halt) return;
    uint32_t *a = blockIdx.y ? a1 : a0;
    __shared__ uint32_t red[kScanThreads];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (uint32_t q = 0; q < kScanItems; q++) {
        uint64_t x = base + q * kScanThreads + threadIdx.x;
        if (x < n) s += a[x];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t d = kScanThreads / 2; d; d >>= 1) {
        if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.y * nblk + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void scan_blocks_kernel(uint32_t *bsum, uint32_t nblk,
                                                           const uint32_t *halt) {
    if (halt && *halt) return;
    uint32_t *b = bsum + blockIdx.x * nblk;  // exclusive scan of block sums
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    const uint32_t t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nblk; base += 1024) {
        uint32_t v = base + t < nblk ? b[base + t] : 0;
        part[t] = v;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            uint32_t u = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += u;
            __syncthreads();
        }
        if (base + t < nblk) b[base + t] = carry + part[t] - v;
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(uint32_t *a0, uint32_t *a1, uint64_t n,
                                                         const uint32_t *bsum, uint32_t nblk,
                                                         const uint32_t *halt) {
    if (halt && *halt) return;
    uint32_t *a = blockIdx.y ? a1 : a0;
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t tsum[kScanThreads];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    for (uint32_t q = 0; q < kScanItems; q++) {
        uint64_t x = base + q * kScanThreads + threadIdx.x;
        tile[q * kScanThreads + threadIdx.x] = x < n ? a[x] : 0;
    }
    __syncthreads();
    // each thread scans its own run of kScanItems consecutive elements
    uint32_t *mine = tile + threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (uint32_t q = 0; q < kScanItems; q++) {
        s += mine[q];
        mine[q] = s;
    }
    tsum[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t d = 1; d < kScanThreads; d <<= 1) {
        uint32_t u = threadIdx.x >= d ? tsum[threadIdx.x - d] : 0;
        __syncthreads();
        tsum[threadIdx.x] += u;
        __syncthreads();
    }
    uint32_t off = bsum[blockIdx.y * nblk + blockIdx.x] + tsum[threadIdx.x] - s;
    for (uint32_t q = 0; q < kScanItems; q++) mine[q] += off;
    __syncthreads();
    for (uint32_t q = 0; q < kScanItems; q++) {
        uint64_t x = base + q * kScanThreads + threadIdx.x;
        if (x < n) a[x] = tile[q * kScanThreads + threadIdx.x];
    }
}

// ------------------------------------------------------------------ seeding


// Set (i, j) in matrix x if absent; on success keep C in step and append it.
__device__ __forceinline__ void seed_pair(const SeedArgs &A, uint32_t x, uint32_t i, uint32_t j) {
    const uint64_t Wp = (uint64_t)A.I.S * kSegWords;
    const MatDev M = A.mats[x];
    uint64_t bit = 1ull << (j & 63);
    unsigned long long o = atomicOr((unsigned long long *)&M.R[(uint64_t)i * Wp + (j >> 6)], bit);
    if (o & bit) return;
    atomicOr((unsigned long long *)&M.Rm[i], (unsigned long long)seg_flag(j));
    if (M.C) {
        atomicOr((unsigned long long *)&M.C[(uint64_t)j * Wp + (i >> 6)], 1ull << (i & 63));
        atomicOr((unsigned long long *)&M.Cm[j], (unsigned long long)seg_flag(i));
    }
    unsigned long long p = atomicAdd(A.ap_count, 1ull);
    atomicAdd(&A.inst_new[(uint64_t)A.inst * kCountShards], 1ull);
    if (p < A.ap_cap) {
        A.ap_key[p] = pair_key(A.inst, x);
        A.ap_i[p] = i;
        A.ap_j[p] = j;
        if (M.sort & kSortRows) atomicAdd(&A.rcnt[row_bucket(A.I, M, i, j)], 1u);
        if (M.sort & kSortCols) atomicAdd(&A.ccnt[col_bucket(A.I, M, i, j)], 1u);
    } else {
        atomicOr(&A.inst_overflow[A.inst], 1u);
    }
}

__global__ void seed_edges_kernel(SeedArgs A) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < A.m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t l = A.lab[e];
        for (uint32_t q = A.lm_ptr[l]; q < A.lm_ptr[l + 1]; q++)
            seed_pair(A, A.lm_mat[q], A.src[e], A.dst[e]);
    }
}

__global__ void seed_eps_kernel(SeedArgs A) {
    uint64_t total = (uint64_t)A.n_eps * A.I.n;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t e = (uint32_t)(x / A.I.n), i = (uint32_t)(x % A.I.n);
        seed_pair(A, A.eps_mat[e], i, i);
    }
}

// Every pair of every matrix becomes "new" (the naive variant, where each
// round multiplies all of M).  Both layouts already hold these pairs.
__global__ __launch_bounds__(64) void extract_all_kernel(const MatDev *mats, InstDev I, uint32_t slot,
                                                         uint32_t nmat, uint32_t *ap_key, uint32_t *ap_i,
                                                         uint32_t *ap_j, unsigned long long *ap_count,
                                                         uint64_t ap_cap, uint32_t *overflow, uint32_t *rcnt,
                                                         uint32_t *ccnt) {
    const uint32_t lane = lane_id();
    const uint64_t Wp = (uint64_t)I.S * kSegWords;
    const uint64_t rows = (uint64_t)nmat * I.n * I.S;
    for (uint64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        uint32_t seg = (uint32_t)(r % I.S);
        uint64_t rr = r / I.S;
        uint32_t i = (uint32_t)(rr % I.n), x = (uint32_t)(rr / I.n);
        uint64_t v = mats[x].R[(uint64_t)i * Wp + seg * kSegWords + lane];
        uint32_t total;
        uint32_t pre = wave_excl_scan((uint32_t)__popcll(v), &total);
        if (!total) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(ap_count, (unsigned long long)total);
        base = first_lane64(base);
        uint64_t p = base + pre;
        while (v) {
            uint32_t b = __ffsll((unsigned long long)v) - 1;
            v &= v - 1;
            if (p < ap_cap) {
                const uint32_t j = (seg * kSegWords + lane) * 64 + b;
                ap_key[p] = pair_key(slot, x);
                ap_i[p] = i;
                ap_j[p] = j;
                if (mats[x].sort & kSortRows) atomicAdd(&rcnt[row_bucket(I, mats[x], i, j)], 1u);
                if (mats[x].sort & kSortCols) atomicAdd(&ccnt[col_bucket(I, mats[x], i, j)], 1u);
            } else {
                atomicOr(overflow, 1u);
            }
            p++;
        }
    }
}

// End of a round: fold each running instance's count of new pairs into its
// statistics; an instance whose round derived nothing is converged.
__global__ void round_end_kernel(const uint32_t *active, unsigned long long *inst_new, SlotStats *st,
                                 uint32_t nslots, const uint32_t *halt) {
    if (*halt) return;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < nslots; x += gridDim.x * blockDim.x) {
        if (!active[x]) continue;
        SlotStats v = st[x];
        unsigned long long n = 0;
        for (uint32_t q = 0; q < kCountShards; q++) {
            n += inst_new[(uint64_t)x * kCountShards + q];
            inst_new[(uint64_t)x * kCountShards + q] = 0;
        }
        if (v.done) continue;
        v.rounds++;
        if (n == 0) {
            v.done = 1;
        } else {
            v.new_total += n;
            if (n > v.max_delta) v.max_delta = n;
        }
        st[x] = v;
    }
}

// The appended pairs have been sorted: empty the buffer.  Skipped after an
// overflow, so the host still sees how many slots the round asked for.
__global__ void reset_appends_kernel(unsigned long long *ap_count, const uint32_t *halt) {
    if (!*halt) *ap_count = 0;
}

// Drop the pending pairs of a retired instance (their slot may be reused).
__global__ void purge_slot_kernel(uint32_t *ap_key, const unsigned long long *ap_count, uint64_t ap_cap,
                                  uint32_t slot) {
    uint64_t n = *ap_count;
    if (n > ap_cap) n = ap_cap;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t k = ap_key[x];
        if (k != kHole && key_slot(k) == slot) ap_key[x] = kHole;
    }
}

// ------------------------------------------------------------------ readout

__global__ __launch_bounds__(64) void row_count_kernel(const uint64_t *R, uint32_t n, uint32_t S,
                                                       uint32_t *cnt, unsigned long long *total) {
    const uint32_t lane = lane_id();
    const uint64_t Wp = (uint64_t)S * kSegWords;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        uint32_t c = 0;
        for (uint32_t s = 0; s < S; s++) c += (uint32_t)__popcll(R[(uint64_t)i * Wp + s * kSegWords + lane]);
        c = wave_sum(c);
        if (lane == 0) {
            cnt[i] = c;
            if (total) atomicAdd(total, (unsigned long long)c);
        }
    }
}

// off: exclusive start of each row in the output (64-bit: counts may pass 2^32)
__global__ __launch_bounds__(64) void row_write_kernel(const uint64_t *R, uint32_t n, uint32_t S,
                                                       const uint64_t *off, uint32_t *src,
                                                       uint32_t *dst) {
    const uint32_t lane = lane_id();
    const uint64_t Wp = (uint64_t)S * kSegWords;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        uint64_t pos = off[i];
        for (uint32_t s = 0; s < S; s++) {
            uint32_t w = s * kSegWords + lane;
            uint64_t v = R[(uint64_t)i * Wp + w];
            uint32_t total;
            uint32_t pre = wave_excl_scan((uint32_t)__popcll(v), &total);
            uint64_t p = pos + pre;
            while (v) {
                uint32_t b = __ffsll((unsigned long long)v) - 1;
                v &= v - 1;
                src[p] = i;
                dst[p] = w * 64 + b;
                p++;
            }
            pos += total;
        }
    }
}

// exclusive scan of u32 row counts into u64 offsets, one workgroup
__global__ __launch_bounds__(1024) void offsets_kernel(const uint32_t *cnt, uint32_t n, uint64_t *off) {
    __shared__ uint64_t part[1024];
    __shared__ uint64_t carry;
    const uint32_t t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += 1024) {
        uint64_t v = base + t < n ? cnt[base + t] : 0;
        part[t] = v;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            uint64_t u = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += u;
            __syncthreads();
        }
        if (base + t < n) off[base + t] = carry + part[t] - v;
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
}

// ------------------------------------------------------------ host launchers

#define CFLR_LAUNCH_CHECK()                                     \
    do {                                                        \
        hipError_t e_ = hipGetLastError();                      \
        if (e_ != hipSuccess) return e_;                        \
    } while (0)

hipError_t launch_product(const ProductArgs &A, uint32_t grid, bool stats, hipStream_t s) {
    if (stats) product_kernel<true><<<grid, kProdWaves * kWave, 0, s>>>(A);
    else product_kernel<false><<<grid, kProdWaves * kWave, 0, s>>>(A);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_prep(const PrepArgs &A, hipStream_t s) {
    prep_kernel<<<1, 1024, 0, s>>>(A);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fill_u32(uint32_t *a, uint64_t n, uint32_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    fill_u32_kernel<<<(uint32_t)g, 256, 0, s>>>(a, n, v);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fill_u64(unsigned long long *a, uint64_t n, unsigned long long v, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    fill_u64_kernel<<<(uint32_t)g, 256, 0, s>>>(a, n, v);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

// counting sort of the appended pairs; buckets [0, nbuckets] (nbuckets + 1 counters)
hipError_t launch_sort(const SortArgs &A, uint64_t nbuckets, uint32_t *bsum, uint32_t sort_grid,
                       hipStream_t s) {
    const uint64_t len = nbuckets + 1;
    uint32_t nblk = (uint32_t)((len + kScanTile - 1) / kScanTile);
    scan_reduce_kernel<<<dim3(nblk, 2), 256, 0, s>>>(A.rcnt, A.ccnt, len, bsum, nblk, A.halt);
    CFLR_LAUNCH_CHECK();
    scan_blocks_kernel<<<2, 1024, 0, s>>>(bsum, nblk, A.halt);
    CFLR_LAUNCH_CHECK();
    scan_apply_kernel<<<dim3(nblk, 2), 256, 0, s>>>(A.rcnt, A.ccnt, len, bsum, nblk, A.halt);
    CFLR_LAUNCH_CHECK();
    scatter_kernel<<<sort_grid, 256, 0, s>>>(A);
    CFLR_LAUNCH_CHECK();
    if (nbuckets) {
        const uint32_t g = (uint32_t)std::min<uint64_t>(nbuckets, sort_grid);
        segsort_kernel<<<dim3(g, 2), kSegSortThreads, 0, s>>>(A, (uint32_t)nbuckets);
        CFLR_LAUNCH_CHECK();
    }
    return hipSuccess;
}

hipError_t launch_zero_counts(uint32_t *rcnt, uint32_t *ccnt, uint64_t len, const uint32_t *halt, hipStream_t s) {
    if (!len) return hipSuccess;
    uint64_t g = (len + 255) / 256;
    if (g > 8192) g = 8192;
    fill_u32_unless_halted_kernel<<<(uint32_t)g, 256, 0, s>>>(rcnt, len, 0, halt);
    CFLR_LAUNCH_CHECK();
    fill_u32_unless_halted_kernel<<<(uint32_t)g, 256, 0, s>>>(ccnt, len, 0, halt);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

uint32_t scan_block_count(uint64_t nbuckets) {
    return (uint32_t)((nbuckets + 1 + kScanTile - 1) / kScanTile);
}

hipError_t launch_seed(const SeedArgs &A, hipStream_t s) {
    if (A.m) {
        uint64_t g = (A.m + 255) / 256;
        if (g > 16384) g = 16384;
        seed_edges_kernel<<<(uint32_t)g, 256, 0, s>>>(A);
        CFLR_LAUNCH_CHECK();
    }
    uint64_t e = (uint64_t)A.n_eps * A.I.n;
    if (e) {
        uint64_t g = (e + 255) / 256;
        if (g > 16384) g = 16384;
        seed_eps_kernel<<<(uint32_t)g, 256, 0, s>>>(A);
        CFLR_LAUNCH_CHECK();
    }
    return hipSuccess;
}

hipError_t launch_round_end(const uint32_t *active, unsigned long long *inst_new, SlotStats *st, uint32_t nslots,
                            const uint32_t *halt, hipStream_t s) {
    uint32_t g = (nslots + 255) / 256;
    round_end_kernel<<<g ? g : 1, 256, 0, s>>>(active, inst_new, st, nslots, halt);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_reset_appends(unsigned long long *ap_count, const uint32_t *halt, hipStream_t s) {
    reset_appends_kernel<<<1, 1, 0, s>>>(ap_count, halt);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_purge_slot(uint32_t *ap_key, const unsigned long long *ap_count, uint64_t ap_cap,
                             uint32_t slot, uint32_t grid, hipStream_t s) {
    purge_slot_kernel<<<grid, 256, 0, s>>>(ap_key, ap_count, ap_cap, slot);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_extract_all(const MatDev *mats, const InstDev &I, uint32_t slot, uint32_t nmat,
                              uint32_t *ap_key, uint32_t *ap_i, uint32_t *ap_j, unsigned long long *ap_count,
                              uint64_t ap_cap, uint32_t *overflow, uint32_t *rcnt, uint32_t *ccnt,
                              hipStream_t s) {
    uint64_t rows = (uint64_t)nmat * I.n * I.S;
    if (!rows) return hipSuccess;
    uint64_t g = rows < 65536 ? rows : 65536;
    extract_all_kernel<<<(uint32_t)g, 64, 0, s>>>(mats, I, slot, nmat, ap_key, ap_i, ap_j, ap_count, ap_cap,
                                                  overflow, rcnt, ccnt);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_row_count(const uint64_t *R, uint32_t n, uint32_t S, uint32_t *cnt,
                            unsigned long long *total, hipStream_t s) {
    if (!n) return hipSuccess;
    uint32_t g = n < 65536 ? n : 65536;
    row_count_kernel<<<g, 64, 0, s>>>(R, n, S, cnt, total);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_row_write(const uint64_t *R, uint32_t n, uint32_t S, const uint32_t *cnt,
                            uint64_t *off, uint32_t *src, uint32_t *dst, hipStream_t s) {
    if (!n) return hipSuccess;
    offsets_kernel<<<1, 1024, 0, s>>>(cnt, n, off);
    CFLR_LAUNCH_CHECK();
    uint32_t g = n < 65536 ? n : 65536;
    row_write_kernel<<<g, 64, 0, s>>>(R, n, S, off, src, dst);
    CFLR_LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace cflr
