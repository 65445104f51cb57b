/*
 * cflr.h -- C interface of libcflr, a CFL-reachability solver for AMD
 * MI355X (gfx950).
 *
 * Problem (Section 1 of Muravev, "Optimization of the Context-Free Language
 * Reachability Matrix-Based Algorithm", arXiv 2401.11029): given a grammar
 * and an edge-labelled graph, find for every non-terminal x the pairs of
 * vertices (i, j) joined by a path whose label word x derives.  The answer is
 * Algorithm 1's Result, M_ij = { x : some path i -> j is derivable from x },
 * stored as one boolean |V| x |V| matrix per non-terminal.
 *
 * Method: the fixpoint of Algorithm 1 over the reachability semiring
 * (Definition 2), in its semi-naive form (Section 3, optimisation 1): every
 * round multiplies only the pairs that are new since the previous round,
 * row by row against row-major copies and column by column against
 * column-major copies (optimisation 2), masks the candidates against the
 * existing matrix and ORs the genuinely new ones in place (the requirement of
 * optimisation 3: a sparse union never rebuilds M).  Rounds repeat until no
 * matrix changes.
 *
 * Conventions (every entry point):
 *  - Every call returns a cflr_status; on failure cflr_last_error() holds a
 *    message.  No C++ exception crosses this interface.
 *  - Inputs are copied during the call; the caller keeps ownership of every
 *    array it passes.  Handles are owned by the library until their *_free.
 *  - Vertex ids are 0-based (the paper numbers them 1..n).
 *  - Edge labels are matched to grammar terminals by name; labels that no
 *    production uses are ignored.  Reversed ("bar") edges are never implied:
 *    a label such as a_bar is just another name.
 *  - Output covers every non-terminal of the grammar text (every left-hand
 *    side), in the order of first appearance; helpers the library adds are
 *    hidden.  Pairs are returned sorted by (i, j).
 *  - A context is used by one host thread at a time (the server below has a
 *    thread of its own and locks internally).
 */
#ifndef CFLR_H
#define CFLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cflr_status {
    CFLR_OK = 0,
    CFLR_EINVAL = 1,        /* bad argument (null pointer, vertex >= n, ...) */
    CFLR_EPARSE = 2,        /* grammar text does not parse */
    CFLR_ENOMEM = 3,        /* device or host memory exhausted */
    CFLR_EDEVICE = 4,       /* a HIP call failed */
    CFLR_PENDING = 5,       /* server: the request has not finished */
    CFLR_ETIMEOUT = 6,      /* server: wait timed out / round limit hit */
    CFLR_EUNSUPPORTED = 7   /* valid input the library cannot handle */
} cflr_status;

typedef struct cflr_ctx cflr_ctx;
typedef struct cflr_grammar cflr_grammar;
typedef struct cflr_graph cflr_graph;
typedef struct cflr_result cflr_result;
typedef struct cflr_server cflr_server;

/* Solver options.  Fill with cflr_opts_default() and change fields. */
typedef struct cflr_opts {
    uint32_t max_rounds;       /* stop with CFLR_ETIMEOUT after this many
                                  rounds; 0 = no limit */
    uint32_t semi_naive;       /* 1 (default): multiply only the new pairs of
                                  each round (optimisation 1); 0: multiply
                                  every pair every round (Algorithm 1 as
                                  printed; an ablation) */
    uint32_t kernel_timing;    /* 1: time every product launch with HIP
                                  events (cflr_stats.product_ms) */
    uint32_t count_traffic;    /* 1: count the algorithmic bytes of the
                                  product kernel (cflr_stats.algo_bytes);
                                  slower, for roofline accounting */
    uint64_t delta_capacity;   /* initial capacity of the new-pair buffer, in
                                  pairs; 0 = automatic.  The buffer grows on
                                  overflow (the round is then re-run). */
    uint32_t grid_waves;       /* waves of the persistent product kernel;
                                  0 = automatic (autotuned) */
    uint32_t rounds_per_sync;  /* rounds replayed per host check of the
                                  changed flag (batched and served forms);
                                  0 = automatic */
    uint32_t chunk_pairs;      /* new pairs of one key tile that one product
                                  work item takes at most (a tile with more
                                  is split, and each part flushes the tile's
                                  keys again); 0 = 2^20 */
    uint32_t storage;          /* single solves: CFLR_STORAGE_AUTO (default),
                                  _DENSE or _SPARSE (see cflr_solve) */
    uint32_t witness;          /* 1: record one derivation per pair for
                                  cflr_result_witness (single-path
                                  semantics); single solves on the sparse
                                  engine only (AUTO then picks it), grammars
                                  without right sides of three or more
                                  symbols.  0 (default): none */
    uint32_t mirror;           /* sparse engine: CFLR_MIRROR_AUTO (default)
                                  or CFLR_MIRROR_OFF (see below) */
    uint32_t sparse_heavy;     /* sparse engine: a bucket of new pairs (one
                                  matrix, one key vertex) whose products
                                  reach this many goes to the LDS bit-set
                                  kernel; 0 = automatic (autotuned, else
                                  128) */
} cflr_opts;

/* Mirror plans (cflr_opts.mirror; the sparse engine).  The analyses of the
   paper's appendix hold every edge with its reverse, (u, t, v) and
   (v, t_bar, u), and their grammars are closed under reversal: Fig. 4b's
   PT -> LPFS_i PT is the mirror of FT -> FT SPFL_i, and FT holds the
   transposes of PT's pairs.  Then every semi-naive round (Section 3,
   opt. 1) derives a set closed under mirroring, and the product of one
   production of each mirror pair gives the other's new pairs as
   transposes.  AUTO finds the mirror of the grammar (labels pair by name,
   t with t_bar; a label without a partner is its own reverse), checks it
   on the grammar exactly and on the seeds of the graph (every seeded pair's
   mirror must be seeded), and uses it when both hold; otherwise, and with
   OFF, every production has its own product.  The result is the same
   either way (cflr_stats.mirror says which plan ran). */
enum {
    CFLR_MIRROR_AUTO = 0,
    CFLR_MIRROR_OFF = 1
};

/* Storage engines of a single solve (cflr_opts.storage, cflr_stats.storage). */
enum {
    CFLR_STORAGE_AUTO = 0,   /* dense while its bit matrices take at most a
                                quarter of the device memory, else sparse */
    CFLR_STORAGE_DENSE = 1,  /* one n x n bit matrix per non-terminal (and a
                                column-major copy where a production needs one) */
    CFLR_STORAGE_SPARSE = 2  /* pairs: growable adjacency lists per matrix and
                                layout, a hash set for membership */
};

/* Per-solve statistics. */
typedef struct cflr_stats {
    uint32_t rounds;           /* product rounds until nothing changed */
    uint32_t reruns;           /* rounds re-run after a buffer overflow */
    uint64_t seed_pairs;       /* pairs set by edges and eps rules */
    uint64_t new_pairs;        /* pairs derived by the rounds */
    uint64_t total_pairs;      /* pairs over every user non-terminal */
    double fixpoint_ms;        /* seeding start to convergence (HIP events) */
    double product_ms;         /* sum of product-kernel times (kernel_timing) */
    uint64_t product_launches; /* product-kernel launches */
    uint64_t algo_bytes;       /* algorithmic bytes of the product kernels
                                  (count_traffic) */
    uint64_t device_bytes;     /* device memory held for this solve */
    uint64_t max_delta;        /* largest number of new pairs in one round */
    uint32_t storage;          /* engine that solved: CFLR_STORAGE_DENSE or _SPARSE */
    /* sparse storage, key-sorted product: its two kernels, for the heavy
       buckets (one workgroup and an LDS bit set per run of a bucket) and
       the light ones (a hash probe per product); one launch each a round */
    double heavy_ms;           /* heavy kernel time (kernel_timing) */
    uint64_t heavy_launches;   /* launches of each of the two */
    uint64_t heavy_algo_bytes; /* algorithmic bytes (count_traffic): 8 per
                                  sorted new pair, 4 per entry of each
                                  distinct partner list and output row read
                                  in a round, 16 per pair derived */
    double light_ms;           /* light kernel time (kernel_timing) */
    uint64_t light_algo_bytes; /* its algorithmic bytes, as heavy_algo_bytes */
    uint32_t mirror;           /* 1: the solve ran a mirror plan (see
                                  CFLR_MIRROR_AUTO) */
} cflr_stats;

void cflr_opts_default(cflr_opts *opts);

/* Thread-local message of the last failed call on this thread ("" if none).
   Owned by the library; valid until the next call on the same thread. */
const char *cflr_last_error(void);

/* Library version string, e.g. "cflr 0.1 gfx950". */
const char *cflr_version(void);

/* ---- context ----------------------------------------------------------
 * hip_device: HIP device ordinal.  hip_stream: a hipStream_t to issue all
 * work on (e.g. torch.cuda.current_stream().cuda_stream), or NULL for a
 * stream the context creates.  The stream must have default priority.
 * Errors: EINVAL (bad device), EDEVICE. */
cflr_status cflr_ctx_create(int hip_device, void *hip_stream, cflr_ctx **out);
void cflr_ctx_destroy(cflr_ctx *ctx);
/* Free and total device memory seen by the context, in bytes (blocks the
 * context's pool keeps for reuse count as used; cflr_ctx_trim frees them). */
cflr_status cflr_ctx_mem_info(cflr_ctx *ctx, uint64_t *free_bytes, uint64_t *total_bytes);
/* Hand the device blocks the context's pool keeps for reuse back to the HIP
 * runtime (results and graphs keep theirs).  Not while a server of the
 * context runs.  Errors: EINVAL. */
cflr_status cflr_ctx_trim(cflr_ctx *ctx);

/* ---- grammar (host only; needs no device) -----------------------------
 * Text format: one production per line, "LHS -> ALT | ALT ...", where ALT is
 * "eps" or a sequence of one or more symbols; "#" starts a comment.
 * Left-hand sides are the non-terminals; every other symbol is a terminal
 * (edge label).  Weak Chomsky normal form (Definition 1) is the case of
 * right sides of at most two non-terminals; the library normalises the rest
 * as the paper does for its CFPQ Data grammars (Figs. 4a-7a): a right side
 * y1 ... yk with k >= 3 becomes y1 H with hidden helper matrices for its
 * suffixes (shared between rules), a terminal t in a longer right side
 * becomes a wrapper non-terminal with T_t -> t, and unit rules x -> y are
 * removed by copying the productions of every non-terminal they reach.
 * Only the non-terminals of the text are results.
 * len: bytes of text (need not be NUL-terminated).
 * Errors: EINVAL (null), EPARSE (message names the line). */
cflr_status cflr_grammar_parse(const char *text, size_t len, cflr_grammar **out);
void cflr_grammar_free(cflr_grammar *g);
uint32_t cflr_grammar_num_nonterminals(const cflr_grammar *g);
/* Name of user non-terminal nt (0-based, first-appearance order); NULL if
   out of range.  Owned by the grammar. */
const char *cflr_grammar_nonterminal_name(const cflr_grammar *g, uint32_t nt);
/* Terminals of the grammar (the labels its rules name), 0-based in order of
   first appearance; in a witness (cflr_result_witness) terminal t has symbol
   number cflr_grammar_num_nonterminals(g) + t.  The name is owned by the
   grammar; NULL if out of range. */
uint32_t cflr_grammar_num_terminals(const cflr_grammar *g);
const char *cflr_grammar_terminal_name(const cflr_grammar *g, uint32_t t);

/* Shape of the lowered (strict WCNF) grammar the device works on. */
typedef struct cflr_grammar_info {
    uint32_t user_nonterminals;  /* non-terminals of the text */
    uint32_t wrappers;           /* T_t helpers for terminals in binary slots */
    uint32_t matrices;           /* user_nonterminals + wrappers + helpers */
    uint32_t binary;             /* binary productions after lowering */
    uint32_t terminal_rules;     /* x -> t after lowering */
    uint32_t eps_rules;          /* x -> eps after lowering */
    uint32_t terminals;          /* distinct terminal names */
    uint32_t helpers;            /* matrices for suffixes of right sides longer than two */
    uint32_t mirror_skipped;     /* binary productions whose product a mirror
                                    plan leaves out (CFLR_MIRROR_AUTO); 0: the
                                    grammar has no mirror */
} cflr_grammar_info;
cflr_status cflr_grammar_info_get(const cflr_grammar *g, cflr_grammar_info *out);

/* ---- graph --------------------------------------------------------------
 * Edge e is (src[e], label[e], dst[e]); label[e] < n_labels indexes
 * label_names (NUL-terminated strings).  src/dst/label are host pointers
 * when on_device == 0 and device pointers of ctx's device when on_device ==
 * 1; either way they are copied into device memory owned by the graph.
 * Duplicate edges and self-loops are allowed (set semantics).
 * Errors: EINVAL (null arrays with n_edges > 0, src/dst >= n_vertices,
 * label >= n_labels), ENOMEM, EDEVICE. */
cflr_status cflr_graph_create(cflr_ctx *ctx, uint32_t n_vertices, uint64_t n_edges,
                              const uint32_t *src, const uint32_t *dst,
                              const uint32_t *label, uint32_t n_labels,
                              const char *const *label_names, int on_device,
                              cflr_graph **out);
void cflr_graph_free(cflr_graph *g);

/* ---- solve ----------------------------------------------------------------
 * Runs the fixpoint of Algorithm 1 for one graph (its Data: the grammar and
 * the edge-labelled graph; its Result: every non-terminal's pairs), in the
 * semi-naive form of Section 3, optimisation 1 (each round multiplies only
 * the pairs new since the previous one), with row-major copies for the
 * matrices in b slots and column-major copies for those in a slots
 * (optimisation 2).  Storage (cflr_opts.storage): dense bit matrices, or
 * adjacency lists plus a hash set for membership, where adding a round's
 * new pairs never rebuilds a matrix (the aim of optimisation 3) and per
 * vertex use masks select the productions a new pair meets (the block
 * directory of optimisation 4).  opts may be NULL (defaults).  The result
 * holds the device storage until cflr_result_free.
 * Errors: EINVAL, ENOMEM (storage does not fit), EDEVICE, EUNSUPPORTED
 * (sparse storage with semi_naive = 0, more than 2^24 - 1 vertices or 65535
 * matrices; witnesses with dense storage or with a right side of three or
 * more symbols), ETIMEOUT (max_rounds reached; *out is still set and holds the
 * partial state, a subset of the fixpoint). */
cflr_status cflr_solve(cflr_ctx *ctx, const cflr_grammar *g, const cflr_graph *graph,
                       const cflr_opts *opts, cflr_result **out);

/* ---- solve without allocating ------------------------------------------
 * For callers that cannot allocate device memory: code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as cflr_solve on sparse storage, but every device structure lives
 * in one fixed region the library holds per device (a file-scope device
 * array of CFLR_NOALLOC_SCRATCH_BYTES, kept until the process ends): the
 * call makes no hipMalloc, hipFree, pinned-host or library allocation.
 * Inputs: the graph as device arrays src/dst/label (n_edges each, device of
 * ctx; label[e] < n_labels indexes label_names); the caller keeps them.
 * Outputs: counts (host array of cflr_grammar_num_nonterminals entries)
 * receives each user non-terminal's pair count; out_src/out_dst (device
 * arrays of `capacity` entries) receive the pairs, each non-terminal's
 * sorted by (i, j), one after another in non-terminal order.  stats
 * (nullable) as for cflr_result_stats.  opts may be NULL; storage is
 * ignored.  The region holds the lists of about 2^24 pair entries and a
 * hash set of 2^24 slots (roughly 10^7 pairs in all, fewer with many
 * non-terminals on many vertices).
 * Errors: EINVAL (null arguments, an edge with a vertex >= n_vertices or a
 * label >= n_labels, capacity below the total: counts are then written but
 * no pairs), ENOMEM (the solve needs more than the region holds; message
 * names the structure), ETIMEOUT (max_rounds), EUNSUPPORTED (also
 * opts->witness), EDEVICE.
 * Every call on one device shares that device's region and leaves the last
 * call's contents in it (each call clears what it needs): calls that
 * overlap on one device race, so serialise them. */
#define CFLR_NOALLOC_SCRATCH_BYTES (256ull << 20)
cflr_status cflr_solve_noalloc(cflr_ctx *ctx, const cflr_grammar *g, uint32_t n_vertices, uint64_t n_edges,
                               const uint32_t *src, const uint32_t *dst, const uint32_t *label,
                               uint32_t n_labels, const char *const *label_names, const cflr_opts *opts,
                               uint32_t *out_src, uint32_t *out_dst, uint64_t capacity, uint64_t *counts,
                               cflr_stats *stats);

/* Batched form: graphs[k] is solved with grammars[k] (the same grammar may be
 * passed for every k).  Admitted instances advance together: the product of
 * a round is two launches (row parts, then column parts) over every (graph,
 * production, tile of new pairs), so many uneven graphs share the device.
 * Graphs are admitted in order while their matrices fit in 70 % of the free
 * device memory and their (key tile, partner) slots -- key tiles of 256
 * vertices x n partners per matrix -- sum to at most the larger of
 * 2^28 and the largest single graph's; the others wait for retirements.
 * If the running graphs derive more new pairs in one round than the
 * new-pair buffer may hold (2^32; the dense engine's sort positions are 32
 * bits), they start again from scratch with at most half as many running
 * at once, and the context keeps that bound for its later batches.
 * outs: caller array of count pointers, each set to a result (or NULL on
 * failure).  Results are identical to cflr_solve of each graph alone.
 * Batches run on dense storage without witnesses (opts->witness and
 * storage = SPARSE give EUNSUPPORTED). */
cflr_status cflr_solve_batch(cflr_ctx *ctx, const cflr_grammar *const *grammars,
                             const cflr_graph *const *graphs, uint32_t count,
                             const cflr_opts *opts, cflr_result **outs);

/* Autotuner: solves graphs[0..count) (as cflr_solve_batch would, or as
 * cflr_solve for one graph) once per candidate and keeps the fastest in ctx
 * for every later solve on it that leaves those options at 0.  Candidates,
 * one option at a time with the others at the best so far: the product
 * grid ({16, 32, 48} waves per compute unit); for batches of more than one
 * graph the rounds per hipGraph replay ({2, 4, 8}); on dense storage the
 * pairs one work item takes at most (chunk_pairs: 2^18, 2^20, 2^22); on
 * sparse storage the products that make a bucket heavy (sparse_heavy: 64,
 * 128, 256).  Results are identical for every candidate (only the
 * interleaving of the atomics changes); they are discarded.
 * out_grid_waves / out_rounds_per_sync (nullable) receive those two
 * choices, out_best_ms (nullable) the best time; cflr_ctx_tuned gives them
 * all.  Errors: as cflr_solve_batch. */
cflr_status cflr_autotune(cflr_ctx *ctx, const cflr_grammar *const *grammars,
                          const cflr_graph *const *graphs, uint32_t count,
                          uint32_t *out_grid_waves, uint32_t *out_rounds_per_sync,
                          double *out_best_ms);

/* The options a context fills in for those a solve leaves at 0 (after
 * cflr_autotune; 0 where nothing was tuned): grid_waves, rounds_per_sync,
 * chunk_pairs, sparse_heavy; the other fields as cflr_opts_default.
 * Errors: EINVAL. */
cflr_status cflr_ctx_tuned(const cflr_ctx *ctx, cflr_opts *out);

/* ---- results --------------------------------------------------------------
 * Algorithm 1's Result, read per non-terminal: the set of pairs (i, j)
 * joined by a path whose word the non-terminal derives (Section 1).  nt
 * indexes the user non-terminals of the result's grammar (first-appearance
 * order).  A result stays valid after its context, grammar and graph are
 * freed.  Errors: EINVAL (null, nt out of range), EDEVICE.
 * cflr_result_count: *n_pairs = |pairs of nt|. */
cflr_status cflr_result_count(const cflr_result *r, uint32_t nt, uint64_t *n_pairs);
/* Copy the pairs of nt, sorted by (src, dst), into src/dst (capacity
 * entries each; host pointers when on_device == 0, device pointers of the
 * result's device when 1; owned by the caller).  *written = pairs copied.
 * EINVAL if capacity is smaller than the count (nothing is written). */
cflr_status cflr_result_copy(const cflr_result *r, uint32_t nt, uint32_t *src, uint32_t *dst,
                             uint64_t capacity, int on_device, uint64_t *written);
/* Single-path semantics (the footnote to Section 5: the same fixpoint over
 * a semiring that carries, for each pair, one derivation).  For a solve with
 * cflr_opts.witness = 1, one derivation of every pair of nt, in the order of
 * cflr_result_copy (arrays of capacity entries each; host or device
 * pointers as there; owned by the caller):
 *   x -> eps:      left = right = mid = CFLR_NONE (and i == j);
 *   x -> t (edge): left = symbol of terminal t, right = mid = CFLR_NONE;
 *   x -> y z:      left = symbol of y, right = symbol of z, mid = k such
 *                  that (i, k) is a pair of y and (k, j) one of z (for a
 *                  terminal, an edge);
 * where symbols number the non-terminals first, then the terminals
 * (cflr_grammar_num_terminals).  The rule is the grammar's own or, when x
 * reaches y' through unit rules, the rule of y' that derived the pair (x's
 * pair then rests on the same pair of y').  round[p] = the round that
 * derived the pair (0 for seeds); a derivation's premises come from earlier
 * rounds, so the rounds order the pairs into a well-founded derivation.
 * *written = entries written.  Errors: EINVAL (null, nt out of range,
 * capacity below the count, a solve without witnesses), EDEVICE. */
#define CFLR_NONE 0xFFFFFFFFu
cflr_status cflr_result_witness(const cflr_result *r, uint32_t nt, uint32_t *left, uint32_t *right,
                                uint32_t *mid, uint32_t *round, uint64_t capacity, int on_device,
                                uint64_t *written);
/* Statistics of the solve (rounds, pairs seeded and derived, times; see
 * cflr_stats).  Errors: EINVAL. */
cflr_status cflr_result_stats(const cflr_result *r, cflr_stats *out);
void cflr_result_free(cflr_result *r);

/* ---- server (continuous batching) --------------------------------------
 * A worker thread keeps the device busy with every admitted request: between
 * rounds it admits queued requests (in arrival order; one that does not fit
 * yet lets later ones pass) while the estimated device footprint of the
 * running ones plus the new one stays within hbm_budget_bytes, their
 * (key tile, partner) slots (key tiles of 256 vertices x n partners per
 * matrix) stay within hbm_budget_bytes / 16 (between 2^20 and 2^29), and
 * fewer than max_slots run in the request's class, and retires requests that
 * converged.  Requests whose footprint is at most hbm_budget_bytes / 64 form
 * the small class, the others the large one; each class runs its own rounds,
 * and the small class runs two round batches per batch of the large one, so
 * a small request does not wait for a large request's round for each of its
 * own.  Each round's product is two launches (row parts, then column parts)
 * over the class's running requests.  Requests may use different grammars.  Results are identical to
 * cflr_solve of the same input.  A request whose dense footprint exceeds
 * the budget goes to the sparse lane instead: a second thread
 * solves such requests one at a time on the sparse engine (cflr_stats.storage
 * = CFLR_STORAGE_SPARSE; mirror plans apply), on a stream of its own, beside
 * the two classes; its memory grows with its pairs and is not counted in
 * the budget.  When a class's running requests derive more new pairs in one
 * round than the dense engine's buffer may hold (2^32), or the buffer's
 * growth finds no memory, they start again from scratch at the front of
 * the queue and the class admits at most half as many from then on; a
 * request whose dense memory cannot be had while nothing else holds any
 * goes to the sparse lane.  Besides the budget the server holds, per class,
 * the sort's bucket counters (8 bytes per bucket, budget / 65536 buckets, at
 * least 2^20 and at most 2^26) and a new-pair buffer of 44 bytes per pair:
 * the large class's starts at the size earlier solves on ctx grew it to
 * (else 2^26 pairs), at most a quarter of the budget (44 bytes a pair; at
 * least 2^20 pairs), the small
 * class's at 2^22 pairs at most, unless opts->delta_capacity says
 * otherwise (each grows when a round overflows it).
 * It also admits a request only while the running requests' (key tile,
 * partner) slots -- key tiles of 256 vertices x n partners per matrix --
 * stay within hbm_budget_bytes / 16 (between 2^20 and 2^29).
 * The server runs its rounds on streams of its own on ctx's device, so the
 * caller's thread may read results and free handles (on ctx's stream) while
 * it runs; do not start other solves on ctx while the server lives.
 * Errors (every server call sets cflr_last_error): EINVAL, ENOMEM, EDEVICE,
 * EUNSUPPORTED (opts->witness). */
cflr_status cflr_server_create(cflr_ctx *ctx, uint64_t hbm_budget_bytes, uint32_t max_slots,
                               const cflr_opts *opts, cflr_server **out);
/* Queue a request; the grammar and graph must stay alive until its result is
 * returned.  *ticket identifies it. */
cflr_status cflr_server_submit(cflr_server *s, const cflr_grammar *g, const cflr_graph *graph,
                               uint64_t *ticket);
/* OK and *out set when finished (the caller then owns *out), PENDING if not
   yet, or the request's own error status. */
cflr_status cflr_server_poll(cflr_server *s, uint64_t ticket, cflr_result **out);
/* Block until finished or timeout_ns elapses (ETIMEOUT). */
cflr_status cflr_server_wait(cflr_server *s, uint64_t ticket, uint64_t timeout_ns,
                             cflr_result **out);
/* Times of a finished request, in seconds on the server's clock. */
cflr_status cflr_server_times(cflr_server *s, uint64_t ticket, double *submitted,
                              double *admitted, double *finished);
/* Stops the worker after the running requests finish; frees the server. */
void cflr_server_free(cflr_server *s);

#ifdef __cplusplus
}
#endif

#endif /* CFLR_H */
