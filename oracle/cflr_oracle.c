/*
 * cflr_oracle.c -- CPU reference solver for CFL-reachability.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this program; it exists so that tests can check the GPU path against
 * an independent implementation.  It shares no code with the GPU path.
 *
 * What it computes (Section 1; Algorithm 1's Result): for every non-terminal
 * x of the grammar,
 *
 *     R_x = { (i, j) : some path from vertex i to vertex j spells a word of
 *                      L(x) },
 *
 * the empty path included (so (i, i) is in R_x for every vertex i when x
 * derives the empty word).  The grammar is in weak Chomsky normal form
 * (Definition 1) relaxed as in the paper's appendix figures: a binary
 * right-hand side may hold terminals, a right-hand side may be a single
 * symbol (terminal or non-terminal), and a right-hand side may be longer
 * than two symbols (the CFPQ Data grammars, Figs. 4a-7a).  A long rule
 * x -> y1 y2 ... yk is read as a chain of prefixes: an internal symbol for
 * y1 y2, one for (y1 y2) y3, and so on, with x -> (y1 ... y(k-1)) yk, so a
 * fact of a prefix symbol says that a path spells a word of the prefix.
 * The internal symbols are never printed.
 *
 * How: the least set of facts (s, i, j) closed under the grammar, computed by
 * a worklist.  Terminal facts are the graph's edges.  Every fact is popped
 * once and combined with every fact already present:
 *
 *   popped (y, i, j), rule x -> y z : for each k with (z, j, k): add (x, i, k)
 *   popped (y, i, j), rule x -> z y : for each k with (z, k, i): add (x, k, j)
 *   popped (y, i, j), rule x -> y   : add (x, i, j)
 *   rule x -> eps                   : add (x, i, i) for every vertex i
 *
 * A fact added after another was popped is itself popped later and meets it
 * then, so at exhaustion the set is closed; every added fact has a
 * derivation, so it is also the least such set.  The sets "for each k with
 * (z, j, k)" are read from per-row sets of vertices: a small hash set of
 * vertex ids while the row is sparse, a bit set (one bit per vertex, read 64
 * at a time) once it holds more than n/64 vertices.  This is only a set
 * representation and changes nothing about which facts are produced.
 *
 * Usage:
 *   cflr_oracle GRAMMAR.txt GRAPH.cflg [--digest] [--pairs OUT]
 *               [--cert OUT] [--stats]
 *
 * --digest  prints "nt NAME COUNT SHA256" per non-terminal, where SHA256 is
 *           FIPS 180-4 SHA-256 over the pairs sorted by (i, j), each written
 *           as two little-endian u32.
 * --pairs   writes u32 K, then per non-terminal: u32 len, name, u64 count,
 *           count x (u32 i, u32 j) sorted by (i, j).
 * --cert    writes every fact in insertion order with the rule and midpoint
 *           that produced it (format in write_cert below).
 * --stats   prints "stats facts F seconds T" (T: fixpoint only, no I/O).
 */
#define _GNU_SOURCE
#include <errno.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static void die(const char *msg, const char *arg) {
    fprintf(stderr, "cflr_oracle: %s%s%s\n", msg, arg ? ": " : "", arg ? arg : "");
    exit(2);
}

static void *xcalloc(size_t n, size_t sz) {
    void *p = calloc(n ? n : 1, sz ? sz : 1);
    if (!p) die("out of memory", NULL);
    return p;
}

static void *xrealloc(void *p, size_t sz) {
    p = realloc(p, sz ? sz : 1);
    if (!p) die("out of memory", NULL);
    return p;
}

/* ------------------------------------------------------------------ grammar */

enum { R_EPS = 0, R_UNIT = 1, R_BIN = 2, R_EDGE = 3 };

typedef struct { uint32_t kind, lhs, r1, r2; } rule_t;

static char **sym_name;      /* symbol id -> name */
static int *sym_is_nt;       /* 1 if the symbol is some rule's left side,
                                2 for an internal prefix of a long rule */
static uint32_t nsym;
static rule_t *rules;
static uint32_t nrules;

static uint32_t sym_lookup(const char *s, int create) {
    for (uint32_t i = 0; i < nsym; i++)
        if (strcmp(sym_name[i], s) == 0) return i;
    if (!create) return UINT32_MAX;
    sym_name = xrealloc(sym_name, (nsym + 1) * sizeof *sym_name);
    sym_is_nt = xrealloc(sym_is_nt, (nsym + 1) * sizeof *sym_is_nt);
    sym_name[nsym] = strdup(s);
    sym_is_nt[nsym] = 0;
    return nsym++;
}

static void add_rule(uint32_t kind, uint32_t lhs, uint32_t r1, uint32_t r2) {
    rules = xrealloc(rules, (nrules + 1) * sizeof *rules);
    rules[nrules++] = (rule_t){kind, lhs, r1, r2};
}

static char *read_file(const char *path, size_t *len) {
    FILE *f = fopen(path, "rb");
    if (!f) die("cannot open", path);
    fseek(f, 0, SEEK_END);
    long sz = ftell(f);
    fseek(f, 0, SEEK_SET);
    char *buf = xcalloc((size_t)sz + 1, 1);
    if (sz > 0 && fread(buf, 1, (size_t)sz, f) != (size_t)sz) die("short read", path);
    fclose(f);
    *len = (size_t)sz;
    return buf;
}

/* Parse the text format: "LHS -> ALT | ALT ...", ALT = eps | s | s s. */
static void parse_grammar(const char *path) {
    size_t len;
    char *text = read_file(path, &len);
    /* pass 1: left sides, so that they are known as non-terminals */
    for (int pass = 0; pass < 2; pass++) {
        char *copy = strdup(text);
        char *save_line = NULL;
        for (char *line = strtok_r(copy, "\n", &save_line); line;
             line = strtok_r(NULL, "\n", &save_line)) {
            char *hash = strchr(line, '#');
            if (hash) *hash = 0;
            char *arrow = strstr(line, "->");
            char *p = line;
            while (*p == ' ' || *p == '\t' || *p == '\r') p++;
            if (!*p) continue;
            if (!arrow) die("line without '->'", line);
            *arrow = 0;
            char lhs[512];
            if (sscanf(line, "%511s", lhs) != 1) die("missing left side", NULL);
            char extra[8];
            if (sscanf(line, "%*s %7s", extra) == 1) die("two symbols on a left side", lhs);
            uint32_t x = sym_lookup(lhs, 1);
            if (pass == 0) { sym_is_nt[x] = 1; continue; }
            char *save_alt = NULL;
            for (char *alt = strtok_r(arrow + 2, "|", &save_alt); alt;
                 alt = strtok_r(NULL, "|", &save_alt)) {
                char *tok[256];
                int nt = 0;
                char *save_tok = NULL;
                for (char *t = strtok_r(alt, " \t\r", &save_tok); t;
                     t = strtok_r(NULL, " \t\r", &save_tok)) {
                    if (nt == 256) die("right side longer than 256 symbols", lhs);
                    tok[nt++] = t;
                }
                if (nt == 0) die("bad right side", lhs);
                if (nt == 1 && strcmp(tok[0], "eps") == 0) {
                    add_rule(R_EPS, x, 0, 0);
                } else if (nt == 1) {
                    add_rule(R_UNIT, x, sym_lookup(tok[0], 1), 0);
                } else {
                    for (int q = 0; q < nt; q++)
                        if (!strcmp(tok[q], "eps")) die("eps inside a longer right side", lhs);
                    /* prefix chain: p1 = tok0 tok1, p(q) = p(q-1) tok(q), x = p(nt-2) tok(nt-1) */
                    uint32_t left = sym_lookup(tok[0], 1);
                    for (int q = 1; q < nt - 1; q++) {
                        char name[64];
                        snprintf(name, sizeof name, "prefix %u.%d", nrules, q);
                        uint32_t p = sym_lookup(name, 1);
                        sym_is_nt[p] = 2;
                        add_rule(R_BIN, p, left, sym_lookup(tok[q], 1));
                        left = p;
                    }
                    add_rule(R_BIN, x, left, sym_lookup(tok[nt - 1], 1));
                }
            }
        }
        free(copy);
    }
    free(text);
}

/* -------------------------------------------------------------------- graph */

static uint32_t n_vert;
static uint64_t n_edge;
static uint32_t *e_src, *e_dst, *e_sym; /* e_sym: grammar symbol or UINT32_MAX */

static void read_graph(const char *path) {
    FILE *f = fopen(path, "rb");
    if (!f) die("cannot open", path);
    char magic[8];
    uint32_t L;
    if (fread(magic, 1, 8, f) != 8 || memcmp(magic, "CFLG0001", 8)) die("bad magic", path);
    if (fread(&n_vert, 4, 1, f) != 1 || fread(&n_edge, 8, 1, f) != 1 ||
        fread(&L, 4, 1, f) != 1) die("short header", path);
    uint32_t *lab_sym = xcalloc(L, sizeof *lab_sym);
    for (uint32_t l = 0; l < L; l++) {
        uint32_t k;
        if (fread(&k, 4, 1, f) != 1) die("short label table", path);
        char *s = xcalloc(k + 1, 1);
        if (k && fread(s, 1, k, f) != k) die("short label name", path);
        uint32_t id = sym_lookup(s, 0);
        /* labels that are not terminals of the grammar take part in nothing */
        lab_sym[l] = (id != UINT32_MAX && !sym_is_nt[id]) ? id : UINT32_MAX;
        free(s);
    }
    e_src = xcalloc(n_edge, 4);
    e_dst = xcalloc(n_edge, 4);
    e_sym = xcalloc(n_edge, 4);
    if (n_edge && (fread(e_src, 4, n_edge, f) != n_edge || fread(e_dst, 4, n_edge, f) != n_edge ||
                   fread(e_sym, 4, n_edge, f) != n_edge)) die("short edge arrays", path);
    for (uint64_t e = 0; e < n_edge; e++) {
        if (e_src[e] >= n_vert || e_dst[e] >= n_vert) die("edge endpoint out of range", path);
        if (e_sym[e] >= L) die("edge label out of range", path);
        e_sym[e] = lab_sym[e_sym[e]];
    }
    free(lab_sym);
    fclose(f);
}

/* --------------------------------------------------------------- fact store */

static uint32_t n_words;          /* words of a bit-set row: ceil(n / 64) */

/* A set of vertex ids (one row of one symbol's relation, or one column).
 * Sparse form: open addressing with linear probing over `cap` slots (a
 * power of two, at most half full), EMPTY marking a free slot.  Dense form
 * (bits != NULL): one bit per vertex.  A set turns dense when its count
 * passes n / 64, where the bit set takes no more memory than the slots. */
#define EMPTY UINT32_MAX
typedef struct {
    uint32_t count;
    uint32_t cap;
    uint32_t *slot;
    uint64_t *bits;
} vset_t;

static vset_t ***row_set;         /* row_set[s][i]: the j with (s, i, j) */
static vset_t ***col_set;         /* col_set[s][j]: the i with (s, i, j) */
static uint64_t *fact_count;      /* per symbol */

static uint32_t vhash(uint32_t v, uint32_t cap) { return (uint32_t)((v * 2654435761u) & (cap - 1)); }

static int vset_has(const vset_t *a, uint32_t v) {
    if (!a || !a->count) return 0;
    if (a->bits) return (int)((a->bits[v >> 6] >> (v & 63)) & 1);
    for (uint32_t h = vhash(v, a->cap);; h = (h + 1) & (a->cap - 1)) {
        if (a->slot[h] == v) return 1;
        if (a->slot[h] == EMPTY) return 0;
    }
}

static void vset_put_slot(uint32_t *slot, uint32_t cap, uint32_t v) {
    uint32_t h = vhash(v, cap);
    while (slot[h] != EMPTY) h = (h + 1) & (cap - 1);
    slot[h] = v;
}

/* Insert v (known to be absent). */
static void vset_insert(vset_t *a, uint32_t v) {
    a->count++;
    if (a->bits) {
        a->bits[v >> 6] |= 1ull << (v & 63);
        return;
    }
    if ((uint64_t)a->count * 64 > n_vert && n_words > 0) {
        /* dense from now on */
        a->bits = xcalloc(n_words, sizeof(uint64_t));
        for (uint32_t h = 0; h < a->cap; h++)
            if (a->slot[h] != EMPTY) a->bits[a->slot[h] >> 6] |= 1ull << (a->slot[h] & 63);
        a->bits[v >> 6] |= 1ull << (v & 63);
        free(a->slot);
        a->slot = NULL;
        a->cap = 0;
        return;
    }
    if (2ull * a->count > a->cap) {
        uint32_t ncap = a->cap ? 2 * a->cap : 4;
        uint32_t *ns = xcalloc(ncap, sizeof(uint32_t));
        memset(ns, 0xFF, (size_t)ncap * sizeof(uint32_t));
        for (uint32_t h = 0; h < a->cap; h++)
            if (a->slot[h] != EMPTY) vset_put_slot(ns, ncap, a->slot[h]);
        free(a->slot);
        a->slot = ns;
        a->cap = ncap;
    }
    vset_put_slot(a->slot, a->cap, v);
}

static vset_t *set_of(vset_t **sets, uint32_t r) {
    if (!sets[r]) sets[r] = xcalloc(1, sizeof(vset_t));
    return sets[r];
}

/* The members of a set, copied out (the set may grow while the caller
 * works through them); in increasing order when `sorted`. */
static uint32_t *snap_buf;
static uint64_t snap_cap;

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static uint32_t vset_snapshot(const vset_t *a, int sorted) {
    if (!a || !a->count) return 0;
    if (a->count > snap_cap) {
        snap_cap = 2ull * a->count;
        snap_buf = xrealloc(snap_buf, snap_cap * sizeof(uint32_t));
    }
    uint32_t k = 0;
    if (a->bits) {
        for (uint32_t w = 0; w < n_words; w++)
            for (uint64_t b = a->bits[w]; b; b &= b - 1) snap_buf[k++] = w * 64 + (uint32_t)__builtin_ctzll(b);
        return k;
    }
    for (uint32_t h = 0; h < a->cap; h++)
        if (a->slot[h] != EMPTY) snap_buf[k++] = a->slot[h];
    if (sorted) qsort(snap_buf, k, sizeof(uint32_t), cmp_u32);
    return k;
}

static uint32_t *stk_s, *stk_i, *stk_j;
static uint64_t stk_len, stk_cap;

static int want_cert;
static uint32_t *cert_s, *cert_i, *cert_j, *cert_rule, *cert_mid;
static uint64_t cert_len, cert_cap;

static void push(uint32_t s, uint32_t i, uint32_t j) {
    if (stk_len == stk_cap) {
        stk_cap = stk_cap ? 2 * stk_cap : 1024;
        stk_s = xrealloc(stk_s, stk_cap * 4);
        stk_i = xrealloc(stk_i, stk_cap * 4);
        stk_j = xrealloc(stk_j, stk_cap * 4);
    }
    stk_s[stk_len] = s;
    stk_i[stk_len] = i;
    stk_j[stk_len] = j;
    stk_len++;
}

/* Insert fact (s, i, j) produced by rule `rule` with midpoint `mid`. */
static void add_fact(uint32_t s, uint32_t i, uint32_t j, uint32_t rule, uint32_t mid) {
    vset_t *r = set_of(row_set[s], i);
    if (vset_has(r, j)) return;
    vset_insert(r, j);
    vset_insert(set_of(col_set[s], j), i);
    fact_count[s]++;
    push(s, i, j);
    if (want_cert) {
        if (cert_len == cert_cap) {
            cert_cap = cert_cap ? 2 * cert_cap : 1024;
            cert_s = xrealloc(cert_s, cert_cap * 4);
            cert_i = xrealloc(cert_i, cert_cap * 4);
            cert_j = xrealloc(cert_j, cert_cap * 4);
            cert_rule = xrealloc(cert_rule, cert_cap * 4);
            cert_mid = xrealloc(cert_mid, cert_cap * 4);
        }
        cert_s[cert_len] = s;
        cert_i[cert_len] = i;
        cert_j[cert_len] = j;
        cert_rule[cert_len] = rule;
        cert_mid[cert_len] = mid;
        cert_len++;
    }
}

/* Rules indexed by the symbol that triggers them. */
static uint32_t **by_left, *n_left;   /* x -> y z, keyed by y */
static uint32_t **by_right, *n_right; /* x -> z y, keyed by y */
static uint32_t **by_unit, *n_unit;   /* x -> y,   keyed by y */

static void index_rule(uint32_t ***tab, uint32_t **cnt, uint32_t key, uint32_t rule) {
    (*tab)[key] = xrealloc((*tab)[key], ((*cnt)[key] + 1) * sizeof(uint32_t));
    (*tab)[key][(*cnt)[key]++] = rule;
}

static void solve(void) {
    n_words = (n_vert + 63) / 64;
    row_set = xcalloc(nsym, sizeof *row_set);
    col_set = xcalloc(nsym, sizeof *col_set);
    for (uint32_t s = 0; s < nsym; s++) {
        row_set[s] = xcalloc(n_vert, sizeof(vset_t *));
        col_set[s] = xcalloc(n_vert, sizeof(vset_t *));
    }
    fact_count = xcalloc(nsym, sizeof *fact_count);
    by_left = xcalloc(nsym, sizeof *by_left);
    by_right = xcalloc(nsym, sizeof *by_right);
    by_unit = xcalloc(nsym, sizeof *by_unit);
    n_left = xcalloc(nsym, 4);
    n_right = xcalloc(nsym, 4);
    n_unit = xcalloc(nsym, 4);
    for (uint32_t r = 0; r < nrules; r++) {
        if (rules[r].kind == R_BIN) {
            index_rule(&by_left, &n_left, rules[r].r1, r);
            index_rule(&by_right, &n_right, rules[r].r2, r);
        } else if (rules[r].kind == R_UNIT) {
            index_rule(&by_unit, &n_unit, rules[r].r1, r);
        }
    }
    /* the edges are the terminal facts; then x -> eps gives every (x, i, i) */
    for (uint64_t e = 0; e < n_edge; e++)
        if (e_sym[e] != UINT32_MAX) add_fact(e_sym[e], e_src[e], e_dst[e], UINT32_MAX, UINT32_MAX);
    for (uint32_t r = 0; r < nrules; r++)
        if (rules[r].kind == R_EPS)
            for (uint32_t i = 0; i < n_vert; i++) add_fact(rules[r].lhs, i, i, r, UINT32_MAX);

    while (stk_len) {
        stk_len--;
        uint32_t y = stk_s[stk_len], i = stk_i[stk_len], j = stk_j[stk_len];
        for (uint32_t t = 0; t < n_unit[y]; t++) {
            uint32_t r = by_unit[y][t];
            add_fact(rules[r].lhs, i, j, r, UINT32_MAX);
        }
        /* x -> y z with (y, i, j): every (z, j, k) gives (x, i, k) */
        for (uint32_t t = 0; t < n_left[y]; t++) {
            uint32_t r = by_left[y][t], x = rules[r].lhs, z = rules[r].r2;
            const vset_t *zr = row_set[z][j];
            if (!zr || !zr->count) continue;
            const vset_t *xr = row_set[x][i];
            if (zr->bits && xr && xr->bits) {
                /* both dense: 64 candidates at a time */
                for (uint32_t w = 0; w < n_words; w++) {
                    uint64_t fresh = zr->bits[w] & ~xr->bits[w];
                    while (fresh) {
                        uint32_t k = w * 64 + (uint32_t)__builtin_ctzll(fresh);
                        fresh &= fresh - 1;
                        add_fact(x, i, k, r, j);
                    }
                }
                continue;
            }
            uint32_t cnt = vset_snapshot(zr, 0);
            for (uint32_t q = 0; q < cnt; q++) {
                uint32_t k = snap_buf[q];
                if (!vset_has(row_set[x][i], k)) add_fact(x, i, k, r, j);
            }
        }
        /* x -> z y with (y, i, j): every (z, k, i) gives (x, k, j) */
        for (uint32_t t = 0; t < n_right[y]; t++) {
            uint32_t r = by_right[y][t], x = rules[r].lhs, z = rules[r].r1;
            const vset_t *zc = col_set[z][i];
            if (!zc || !zc->count) continue;
            const vset_t *xc = col_set[x][j];
            if (zc->bits && xc && xc->bits) {
                for (uint32_t w = 0; w < n_words; w++) {
                    uint64_t fresh = zc->bits[w] & ~xc->bits[w];
                    while (fresh) {
                        uint32_t k = w * 64 + (uint32_t)__builtin_ctzll(fresh);
                        fresh &= fresh - 1;
                        add_fact(x, k, j, r, i);
                    }
                }
                continue;
            }
            uint32_t cnt = vset_snapshot(zc, 0);
            for (uint32_t q = 0; q < cnt; q++) {
                uint32_t k = snap_buf[q];
                if (!vset_has(col_set[x][j], k)) add_fact(x, k, j, r, i);
            }
        }
    }
}

/* ------------------------------------------------------------------ sha-256 */
/* FIPS 180-4, section 6.2. */

typedef struct {
    uint32_t h[8];
    uint8_t buf[64];
    uint64_t total;
    uint32_t fill;
} sha256_t;

static const uint32_t SHA_K[64] = {
    0x428a2f98, 0x71374491, 0xb5c0fbcf, 0xe9b5dba5, 0x3956c25b, 0x59f111f1, 0x923f82a4, 0xab1c5ed5,
    0xd807aa98, 0x12835b01, 0x243185be, 0x550c7dc3, 0x72be5d74, 0x80deb1fe, 0x9bdc06a7, 0xc19bf174,
    0xe49b69c1, 0xefbe4786, 0x0fc19dc6, 0x240ca1cc, 0x2de92c6f, 0x4a7484aa, 0x5cb0a9dc, 0x76f988da,
    0x983e5152, 0xa831c66d, 0xb00327c8, 0xbf597fc7, 0xc6e00bf3, 0xd5a79147, 0x06ca6351, 0x14292967,
    0x27b70a85, 0x2e1b2138, 0x4d2c6dfc, 0x53380d13, 0x650a7354, 0x766a0abb, 0x81c2c92e, 0x92722c85,
    0xa2bfe8a1, 0xa81a664b, 0xc24b8b70, 0xc76c51a3, 0xd192e819, 0xd6990624, 0xf40e3585, 0x106aa070,
    0x19a4c116, 0x1e376c08, 0x2748774c, 0x34b0bcb5, 0x391c0cb3, 0x4ed8aa4a, 0x5b9cca4f, 0x682e6ff3,
    0x748f82ee, 0x78a5636f, 0x84c87814, 0x8cc70208, 0x90befffa, 0xa4506ceb, 0xbef9a3f7, 0xc67178f2};

static uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

static void sha_block(sha256_t *c, const uint8_t *p) {
    uint32_t w[64];
    for (int t = 0; t < 16; t++)
        w[t] = (uint32_t)p[4 * t] << 24 | (uint32_t)p[4 * t + 1] << 16 | (uint32_t)p[4 * t + 2] << 8 | p[4 * t + 3];
    for (int t = 16; t < 64; t++) {
        uint32_t s0 = rotr(w[t - 15], 7) ^ rotr(w[t - 15], 18) ^ (w[t - 15] >> 3);
        uint32_t s1 = rotr(w[t - 2], 17) ^ rotr(w[t - 2], 19) ^ (w[t - 2] >> 10);
        w[t] = w[t - 16] + s0 + w[t - 7] + s1;
    }
    uint32_t a = c->h[0], b = c->h[1], cc = c->h[2], d = c->h[3];
    uint32_t e = c->h[4], f = c->h[5], g = c->h[6], h = c->h[7];
    for (int t = 0; t < 64; t++) {
        uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
        uint32_t ch = (e & f) ^ (~e & g);
        uint32_t t1 = h + S1 + ch + SHA_K[t] + w[t];
        uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
        uint32_t mj = (a & b) ^ (a & cc) ^ (b & cc);
        uint32_t t2 = S0 + mj;
        h = g; g = f; f = e; e = d + t1; d = cc; cc = b; b = a; a = t1 + t2;
    }
    c->h[0] += a; c->h[1] += b; c->h[2] += cc; c->h[3] += d;
    c->h[4] += e; c->h[5] += f; c->h[6] += g; c->h[7] += h;
}

static void sha_init(sha256_t *c) {
    static const uint32_t H0[8] = {0x6a09e667, 0xbb67ae85, 0x3c6ef372, 0xa54ff53a,
                                   0x510e527f, 0x9b05688c, 0x1f83d9ab, 0x5be0cd19};
    memcpy(c->h, H0, sizeof H0);
    c->total = 0;
    c->fill = 0;
}

static void sha_update(sha256_t *c, const void *data, size_t len) {
    const uint8_t *p = data;
    c->total += len;
    while (len) {
        uint32_t take = 64 - c->fill;
        if (take > len) take = (uint32_t)len;
        memcpy(c->buf + c->fill, p, take);
        c->fill += take;
        p += take;
        len -= take;
        if (c->fill == 64) { sha_block(c, c->buf); c->fill = 0; }
    }
}

static void sha_final(sha256_t *c, char hex[65]) {
    uint64_t bits = c->total * 8;
    uint8_t pad = 0x80;
    sha_update(c, &pad, 1);
    uint8_t zero = 0;
    while (c->fill != 56) sha_update(c, &zero, 1);
    uint8_t len[8];
    for (int t = 0; t < 8; t++) len[t] = (uint8_t)(bits >> (56 - 8 * t));
    sha_update(c, len, 8);
    for (int t = 0; t < 8; t++) sprintf(hex + 8 * t, "%08x", c->h[t]);
    hex[64] = 0;
}

/* ------------------------------------------------------------------- output */

static void le32(uint8_t *o, uint32_t v) {
    o[0] = (uint8_t)v; o[1] = (uint8_t)(v >> 8); o[2] = (uint8_t)(v >> 16); o[3] = (uint8_t)(v >> 24);
}

/* Visit the pairs of symbol s in (i, j) order. */
typedef void (*pair_fn)(void *ctx, uint32_t i, uint32_t j);
static void for_pairs(uint32_t s, pair_fn fn, void *ctx) {
    for (uint32_t i = 0; i < n_vert; i++) {
        uint32_t cnt = vset_snapshot(row_set[s][i], 1);
        for (uint32_t q = 0; q < cnt; q++) fn(ctx, i, snap_buf[q]);
    }
}

static void sha_pair(void *ctx, uint32_t i, uint32_t j) {
    uint8_t b[8];
    le32(b, i);
    le32(b + 4, j);
    sha_update((sha256_t *)ctx, b, 8);
}

static void file_pair(void *ctx, uint32_t i, uint32_t j) {
    uint32_t b[2] = {i, j};
    if (fwrite(b, 4, 2, (FILE *)ctx) != 2) die("write failed", NULL);
}

static void write_cert(const char *path) {
    /* u32 nsym; per symbol: u32 len, name, u32 is_nt
       u32 nrules; per rule: u32 kind, lhs, r1, r2
       u64 nfacts; per fact: u32 sym, i, j, rule (UINT32_MAX: edge), mid
       (UINT32_MAX: none) -- in insertion order */
    FILE *f = fopen(path, "wb");
    if (!f) die("cannot write", path);
    fwrite(&nsym, 4, 1, f);
    for (uint32_t s = 0; s < nsym; s++) {
        uint32_t k = (uint32_t)strlen(sym_name[s]);
        uint32_t nt = (uint32_t)sym_is_nt[s];
        fwrite(&k, 4, 1, f);
        fwrite(sym_name[s], 1, k, f);
        fwrite(&nt, 4, 1, f);
    }
    fwrite(&nrules, 4, 1, f);
    fwrite(rules, sizeof(rule_t), nrules, f);
    fwrite(&cert_len, 8, 1, f);
    for (uint64_t t = 0; t < cert_len; t++) {
        uint32_t rec[5] = {cert_s[t], cert_i[t], cert_j[t], cert_rule[t], cert_mid[t]};
        fwrite(rec, 4, 5, f);
    }
    fclose(f);
}

int main(int argc, char **argv) {
    if (argc < 3) die("usage: cflr_oracle GRAMMAR GRAPH [--digest] [--pairs OUT] [--cert OUT] [--stats]", NULL);
    int digest = 0, stats = 0;
    const char *pairs_path = NULL, *cert_path = NULL;
    for (int a = 3; a < argc; a++) {
        if (!strcmp(argv[a], "--digest")) digest = 1;
        else if (!strcmp(argv[a], "--stats")) stats = 1;
        else if (!strcmp(argv[a], "--pairs") && a + 1 < argc) pairs_path = argv[++a];
        else if (!strcmp(argv[a], "--cert") && a + 1 < argc) cert_path = argv[++a];
        else die("unknown argument", argv[a]);
    }
    want_cert = cert_path != NULL;
    parse_grammar(argv[1]);
    read_graph(argv[2]);

    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    solve();
    clock_gettime(CLOCK_MONOTONIC, &t1);
    double secs = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);

    uint64_t total = 0;
    for (uint32_t s = 0; s < nsym; s++) total += fact_count[s];
    if (stats) printf("stats facts %llu seconds %.6f\n", (unsigned long long)total, secs);
    if (digest) {
        for (uint32_t s = 0; s < nsym; s++) {
            if (sym_is_nt[s] != 1) continue;
            sha256_t c;
            sha_init(&c);
            for_pairs(s, sha_pair, &c);
            char hex[65];
            sha_final(&c, hex);
            printf("nt %s %llu %s\n", sym_name[s], (unsigned long long)fact_count[s], hex);
        }
    }
    if (pairs_path) {
        FILE *f = fopen(pairs_path, "wb");
        if (!f) die("cannot write", pairs_path);
        uint32_t k = 0;
        for (uint32_t s = 0; s < nsym; s++) k += (uint32_t)(sym_is_nt[s] == 1);
        fwrite(&k, 4, 1, f);
        for (uint32_t s = 0; s < nsym; s++) {
            if (sym_is_nt[s] != 1) continue;
            uint32_t len = (uint32_t)strlen(sym_name[s]);
            fwrite(&len, 4, 1, f);
            fwrite(sym_name[s], 1, len, f);
            fwrite(&fact_count[s], 8, 1, f);
            for_pairs(s, file_pair, f);
        }
        if (fclose(f)) die("write failed", pairs_path);
    }
    if (cert_path) write_cert(cert_path);
    fflush(stdout);
    return 0;
}
