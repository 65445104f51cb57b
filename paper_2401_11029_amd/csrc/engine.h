// engine.h -- host engine: context, device pool, instances and rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace cflr {

void hip_check(hipError_t e, const char *what);

// Caching device allocator: blocks are kept per size after release and
// handed out again, so repeated solves of one shape allocate once.
class DevPool {
   public:
    explicit DevPool(int device) : device_(device) {}
    ~DevPool();
    void *alloc(size_t bytes);
    void release(void *p);
    void trim();  // hand cached blocks back to the HIP runtime (hipFree)
    uint64_t held() const { return held_; }

   private:
    int device_;
    std::mutex mu_;
    std::multimap<size_t, void *> cache_;
    std::map<void *, size_t> live_;
    uint64_t held_ = 0;
};

// RAII device buffer from a pool
struct DevBuf {
    DevPool *pool = nullptr;
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(DevPool *p, size_t b) : pool(p), ptr(b ? p->alloc(b) : nullptr), bytes(b) {}
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        reset();
        pool = o.pool;
        ptr = o.ptr;
        bytes = o.bytes;
        o.ptr = nullptr;
        o.bytes = 0;
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (ptr && pool) pool->release(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace cflr

struct cflr_ctx {
    // one reference for the caller's handle plus one per graph, instance,
    // run and server using it; the context is torn down at zero, so objects
    // freed after cflr_ctx_destroy still find their pool and stream
    std::atomic<int> refs{1};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t num_cu = 0;
    std::unique_ptr<cflr::DevPool> pool;
    uint64_t delta_capacity_hint = 0;  // grown new-pair capacity, reused by later solves
    uint32_t grid_waves_tuned = 0;     // autotuned product grid (0 = not yet)
    uint32_t rounds_per_sync_tuned = 0;  // autotuned rounds per graph replay (batches)
    uint32_t chunk_pairs_tuned = 0;      // autotuned work-item size (dense engine)
    uint32_t sparse_heavy_tuned = 0;     // autotuned heavy-bucket threshold (sparse engine)
    uint32_t batch_running_cap = 0;      // graphs a batch ran at most when its new pairs last fit the
                                         // buffer's limit after a restart (0: no restart yet)
    // sizes the sparse engine grew to (new-pair buffer, list pool, hash
    // slots), the starting point of later sparse solves on this context
    uint64_t sparse_delta_hint = 0, sparse_pool_hint = 0, sparse_slots_hint = 0;
};

namespace cflr {

void ctx_retain(cflr_ctx *ctx);
void ctx_release(cflr_ctx *ctx);

// Holds a reference to a context for the lifetime of its owner.  Declare it
// as the owner's first member so that it is released after every buffer.
struct CtxRef {
    cflr_ctx *p = nullptr;
    CtxRef() = default;
    explicit CtxRef(cflr_ctx *c) : p(c) {
        if (p) ctx_retain(p);
    }
    CtxRef(const CtxRef &o) : CtxRef(o.p) {}
    CtxRef &operator=(const CtxRef &o) {
        if (this != &o) {
            if (o.p) ctx_retain(o.p);
            if (p) ctx_release(p);
            p = o.p;
        }
        return *this;
    }
    ~CtxRef() {
        if (p) ctx_release(p);
    }
};

}  // namespace cflr

struct cflr_graph {
    cflr::CtxRef hold;
    cflr_ctx *ctx = nullptr;
    uint32_t n = 0;
    uint64_t m = 0;
    cflr::DevBuf src, dst, lab;
    std::vector<std::string> label_names;
};

namespace cflr {

// Pair storage of a solve on the sparse engine (sparse.cpp, layout in
// sparse.h): the adjacency-list directory and the pool of list entries,
// kept for readout.
struct SparseStore {
    CtxRef hold;  // first member: released after the buffers
    cflr_ctx *ctx = nullptr;
    uint32_t n = 0, nlayouts = 0;
    DevBuf dir, pool;
    std::vector<uint32_t> row_layout;  // per matrix (kNone: none)
    // per matrix: ~0u, or the mirror whose rows hold its pairs transposed
    // (a user non-terminal without rows of its own is read out from them)
    std::vector<uint32_t> readout_mirror;
    // witnesses (single-path semantics), when the solve recorded them: the
    // pair set, a witness per slot, and the tables that name a witness in
    // the grammar text's symbols (per binary production its two operands;
    // per graph label its terminal)
    DevBuf hash, wit;
    uint64_t hash_slots = 0;
    std::vector<uint32_t> prod_sym, label_sym;
};

// One graph being solved (or solved): its matrices live in `arena` (dense
// storage) or in `sp` (sparse storage).
struct Instance {
    CtxRef hold;
    cflr_ctx *ctx = nullptr;
    Lowered low;  // copy: results outlive the grammar handle
    uint32_t n = 0, S = 0;
    uint64_t Wp = 0;
    DevBuf arena;
    std::vector<MatDev> mats;
    uint64_t footprint = 0;
    // seeding tables
    DevBuf lm_ptr, lm_mat, eps_mat;
    uint32_t n_eps = 0;
    uint64_t max_seeds = 0;
    const cflr_graph *graph = nullptr;
    // state
    uint32_t bbase = 0;  // first sort bucket
    uint32_t slot = 0;
    uint32_t rounds = 0;
    bool done = false;
    cflr_status status = CFLR_OK;
    std::string error;
    cflr_stats stats{};
    // readout cache
    std::vector<int64_t> counts;  // per user NT, -1 = unknown
    std::shared_ptr<SparseStore> sp;  // set when the sparse engine solved it
};

// Device bytes an instance of this grammar on n vertices will hold.
uint64_t instance_footprint(const Lowered &low, uint32_t n);
// Sort buckets of such an instance: per sorted matrix, key tiles x partner
// segments.
uint64_t instance_buckets(const Lowered &low, uint32_t n);
// (key tile, partner) slots of all its matrices: a batch admits instances
// while these sum to at most max(largest, 2^28), which keeps one round's new
// pairs inside the 2^32-entry new-pair buffer.
uint64_t instance_pair_slots(const Lowered &low, uint32_t n);

// dense = false: only the seeding tables (the sparse engine keeps its own
// storage).
std::shared_ptr<Instance> make_instance(cflr_ctx *ctx, const Lowered &low, const cflr_graph *g, bool dense = true);

// The sparse engine (sparse.cpp): solves one instance made with dense =
// false on `stream` (null: the context's); *timed_out when opts.max_rounds
// stopped it first.
void sparse_solve(cflr_ctx *ctx, const cflr_opts &opts, Instance &inst, bool *timed_out,
                  hipStream_t stream = nullptr);
// Binary productions a mirror plan of the sparse engine leaves without a
// product of their own (one of each mirror pair); 0 when the grammar has no
// mirror (cflr_opts.mirror).
uint32_t mirror_skipped(const Lowered &low);
void sparse_counts(Instance &inst);
// cflr_solve_noalloc: the sparse engine on the file-scope scratch region (no
// device allocation); results into the caller's device arrays.
void sparse_solve_noalloc(cflr_ctx *ctx, const Lowered &low, uint32_t n, uint64_t m, const uint32_t *src,
                          const uint32_t *dst, const uint32_t *label, const std::vector<std::string> &label_names,
                          const cflr_opts &o, uint32_t *out_src, uint32_t *out_dst, uint64_t capacity,
                          uint64_t *counts, cflr_stats *stats);
void sparse_copy(Instance &inst, uint32_t nt, uint32_t *src, uint32_t *dst, uint64_t count, bool on_device);
// The witnesses of nt's pairs, in the order of sparse_copy (count of them).
void sparse_witness(Instance &inst, uint32_t nt, uint32_t *left, uint32_t *right, uint32_t *mid, uint32_t *round,
                    uint64_t count, bool on_device);

// A set of instances advancing round by round together (the product
// launches of a round cover all of them).
class Run {
   public:
    // bucket_capacity: sort buckets for all instances admitted at once
    // (instance_buckets of each); below 2^32.  stream: where the rounds run
    // (null: the context's stream).
    Run(cflr_ctx *ctx, const cflr_opts &opts, uint64_t bucket_capacity, uint32_t max_instances,
        hipStream_t stream = nullptr);
    ~Run();
    // Admit an instance: assigns its sort buckets, seeds its pairs (they
    // become the next round's new pairs).  Between rounds only.  If it
    // throws, the run is unchanged (the instance is not admitted).
    void add(const std::shared_ptr<Instance> &inst);
    // Drop an instance (finished); between rounds only.
    void remove(Instance *inst);
    // One round over every admitted instance.  Instances whose round derived
    // nothing are marked done.  Returns the number still running.
    uint32_t round();
    // R rounds; with R > 1 they are captured once into a hipGraph and
    // replayed, with one host check per replay.  Returns the number running.
    uint32_t rounds(uint32_t R);
    size_t size() const { return insts_.size(); }
    const std::vector<std::shared_ptr<Instance>> &instances() const { return insts_; }
    double product_ms() const { return product_ms_; }
    uint64_t product_launches() const { return product_launches_; }
    uint64_t algo_bytes() const { return algo_bytes_; }
    uint32_t reruns() const { return reruns_; }
    uint64_t delta_capacity() const { return ap_cap_; }

   private:
    CtxRef hold_;  // first member: released after every buffer below
    void rebuild_tables();
    void ensure_capacity(uint64_t pairs, bool keep);
    void sort_appended();
    uint64_t alloc_buckets(uint64_t count);
    void free_buckets(uint64_t base, uint64_t count);
    void read_flags();
    uint64_t bucket_hi() const;
    void extract_all_pairs();
    // rerun: the product of an overflowing round again (the work table and
    // the counts of the pairs appended so far are kept)
    void enqueue_product(bool timed, bool rerun = false);
    void enqueue_round_end();
    void enqueue_round(bool timed);
    void recover();
    void log_round();

    cflr_ctx *ctx_;
    cflr_opts opts_;
    hipStream_t s_;
    std::vector<std::shared_ptr<Instance>> insts_;
    bool dirty_ = true;
    uint64_t bucket_cap_;
    uint32_t max_inst_;
    std::map<uint64_t, uint64_t> free_buckets_;  // base -> length
    // device tables
    DevBuf d_inst_, d_mats_, d_ent_, d_prefix_;
    DevBuf d_units_;
    uint32_t nent_ = 0, nunit_ = 0, unit_split_ = 0;  // units [0, unit_split_) are row parts
    DevBuf d_rcnt_, d_ccnt_, d_bsum_;
    DevBuf d_ap_key_, d_ap_i_, d_ap_j_, d_rs_, d_cs_, d_rs_stage_, d_cs_stage_;
    uint64_t ap_cap_ = 0;
    // most pairs the new-pair buffer may hold: 32-bit sort positions; the
    // environment variable CFLR_DENSE_PAIR_LIMIT lowers it (tests of what
    // callers do at the limit)
    uint64_t ap_limit_ = 0xFFFFFFF0ull;
    DevBuf d_counters_;  // [0] ap_count, [1] items taken (row parts), [2] algo_bytes, [3] halt (u32),
                         // [4] items taken (column parts)
    DevBuf d_inst_new_, d_inst_over_, d_active_, d_slot_stats_;
    SlotStats *h_stats_ = nullptr;
    hipGraphExec_t graph_exec_ = nullptr;
    uint64_t generation_ = 1, graph_gen_ = 0;
    uint32_t graph_rounds_ = 0;
    DevBuf d_touched_, d_touched_off_;
    uint64_t touched_bits_ = 0;
    // host mirrors (pinned)
    unsigned long long *h_new_ = nullptr;
    uint32_t *h_over_ = nullptr;
    unsigned long long *h_counters_ = nullptr;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    double product_ms_ = 0;
    uint64_t product_launches_ = 0;
    uint64_t algo_bytes_ = 0;
    uint32_t reruns_ = 0;
    uint32_t grid_ = 0;
    uint32_t round_no_ = 0;
    bool log_ = false;
};

void instance_counts(Instance &inst);
// keep only the row-major matrices of the user non-terminals (finished instances)
void compact_instance(Instance &in);
void set_last_error(const std::string &msg);
void copy_sync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
void instance_copy(Instance &inst, uint32_t nt, uint32_t *src, uint32_t *dst, uint64_t capacity,
                   bool on_device, uint64_t *written);

}  // namespace cflr

struct cflr_result {
    std::shared_ptr<cflr::Instance> inst;
};
