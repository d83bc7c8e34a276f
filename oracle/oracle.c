/*
 * Plain CPU oracle for Poseidon-12 Merkle building over Goldilocks.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP path and must never be used as a
 * fallback for it.
 *
 * Everything here is the textbook definition, written for a reader to check
 * by eye against the paper (arXiv 2506.09505):
 *
 *   field   p = 2^64 - 2^32 + 1 (Sec. 2.4, Eq. 1); a+b, a-b, a*b are computed
 *           exactly in 128 bits and reduced with the C '%' operator.  None of
 *           the paper's fast reduction (Alg. 2) or add/sub tricks (Alg. 3-6)
 *           is used; they are what the GPU side implements.
 *   perm    Poseidon over a 12-element state (Sec. 2.4 "Poseidon Hash"):
 *           4 full, 22 partial, 4 full rounds, S-box x^7.  Each round r does
 *             state += C[r]; S-box (all 12 words in full rounds, word 0 in
 *             partial rounds); state = M * state   (dense 12x12, every round).
 *           Alg. 1 prints the same function in an optimised shape (sparse
 *           partial-round matrices S and moved constants); the oracle keeps
 *           the dense shape on purpose.
 *   sponge  rate 8, capacity 4: state = 0; for each chunk of 8 row words, add
 *           them into state[0..7] (a short last chunk adds zeros), permute;
 *           digest = state[0..3] (Sec. 2.4; Sec. 4.2 for 8-word leaves).
 *   tree    level 0 = digests of the rows; each parent = sponge of the 8-word
 *           concatenation left||right; an unpaired last node moves up
 *           unchanged; repeat to one root (Sec. 2.4 "Merkle Tree", Sec. 4.2).
 *
 * Parity unpinned: the permutation against the paper's own numbers (the paper
 * prints no round constants, matrix or test vectors).  Everything else is
 * pinned by closed forms and brute force in the CPU test suite.
 *
 * Layouts are those of the C ABI: leaves column-major (element (r, c) at
 * leaves[c*n_rows + r]), nodes level-major with 4 words per node.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define ORACLE_P 0xFFFFFFFF00000001ULL /* 2^64 - 2^32 + 1, Sec. 2.4 Eq. 1 */
#define WIDTH 12                       /* state words, Sec. 2.4            */
#define RATE 8                         /* absorbed chunk, Sec. 2.4         */
#define DIGEST 4                       /* digest words, Sec. 4.2           */
#define HALF_FULL 4                    /* HALF_FULL_ROUNDS, Sec. 2.4       */
#define PARTIAL 22                     /* PARTIAL_ROUNDS, Sec. 2.4         */
#define ROUNDS (2 * HALF_FULL + PARTIAL)

/* Round constants C[30][12] and the dense matrix M[12][12]: the instance
 * parameters, passed in by the caller (the paper prints no values). */
typedef struct {
    uint64_t rc[ROUNDS][WIDTH];
    uint64_t mds[WIDTH][WIDTH];
} oracle_params;

/* ---------------------------------------------------------------- field -- */

uint64_t oracle_fadd(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a + b) % ORACLE_P); }

uint64_t oracle_fsub(uint64_t a, uint64_t b) {
    return (uint64_t)(((u128)a + ORACLE_P - (b % ORACLE_P)) % ORACLE_P);
}

uint64_t oracle_fmul(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) % ORACLE_P); }

/* 128-bit value reduced mod p (the operation Alg. 2 computes). */
uint64_t oracle_reduce128(uint64_t hi, uint64_t lo) {
    u128 v = ((u128)hi << 64) | lo;
    return (uint64_t)(v % ORACLE_P);
}

uint64_t oracle_fpow(uint64_t a, uint64_t e) {
    uint64_t r = 1 % ORACLE_P, b = a % ORACLE_P;
    while (e) {
        if (e & 1) r = oracle_fmul(r, b);
        b = oracle_fmul(b, b);
        e >>= 1;
    }
    return r;
}

/* Element-wise field operations on arrays (for checking the device field
 * layer): op 0 a+b, 1 a-b, 2 (a 2^64 + b) mod p, 3 a^2, 4 a*b,
 * 5 a*(b mod 256), 6 a^7.  Each is the plain definition above. */
void oracle_field_array(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t n) {
    for (size_t i = 0; i < n; i++) {
        switch (op) {
            case 0: out[i] = oracle_fadd(a[i], b[i]); break;
            case 1: out[i] = oracle_fsub(a[i], b[i]); break;
            case 2: out[i] = oracle_reduce128(a[i], b[i]); break;
            case 3: out[i] = oracle_fmul(a[i], a[i]); break;
            case 4: out[i] = oracle_fmul(a[i], b[i]); break;
            case 5: out[i] = oracle_fmul(a[i], b[i] & 0xFF); break;
            case 6: out[i] = oracle_fpow(a[i], 7); break;
            default: out[i] = 0;
        }
    }
}

/* ---------------------------------------------------------- permutation -- */

static uint64_t sbox(uint64_t x) { return oracle_fpow(x, 7); }

static void permute_one(const oracle_params *prm, uint64_t s[WIDTH]) {
    for (int r = 0; r < ROUNDS; r++) {
        int full = (r < HALF_FULL) || (r >= HALF_FULL + PARTIAL);
        for (int i = 0; i < WIDTH; i++) s[i] = oracle_fadd(s[i], prm->rc[r][i]);
        if (full) {
            for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);
        } else {
            s[0] = sbox(s[0]);
        }
        uint64_t t[WIDTH];
        for (int i = 0; i < WIDTH; i++) {
            uint64_t acc = 0;
            for (int j = 0; j < WIDTH; j++) acc = oracle_fadd(acc, oracle_fmul(prm->mds[i][j], s[j]));
            t[i] = acc;
        }
        memcpy(s, t, sizeof t);
    }
}

/* Sponge over n words (Sec. 2.4): chunks of RATE added into state[0..7]. */
static void sponge(const oracle_params *prm, const uint64_t *words, size_t n, uint64_t out[DIGEST]) {
    uint64_t s[WIDTH] = {0};
    for (size_t k = 0; k < n; k += RATE) {
        for (size_t i = 0; i < RATE && k + i < n; i++) s[i] = oracle_fadd(s[i], words[k + i]);
        permute_one(prm, s);
    }
    memcpy(out, s, DIGEST * sizeof(uint64_t));
}

/* ----------------------------------------------------- thread fan-out -- */

typedef struct {
    void (*fn)(void *ctx, size_t i);
    void *ctx;
    size_t begin, end;
} job_t;

static void *run_job(void *arg) {
    job_t *j = (job_t *)arg;
    for (size_t i = j->begin; i < j->end; i++) j->fn(j->ctx, i);
    return NULL;
}

/* Runs fn(ctx, i) for i in [0, n) over `threads` POSIX threads. */
static void parallel_for(size_t n, int threads, void (*fn)(void *, size_t), void *ctx) {
    if (threads < 1) threads = 1;
    if ((size_t)threads > n) threads = (int)(n ? n : 1);
    if (threads == 1) {
        for (size_t i = 0; i < n; i++) fn(ctx, i);
        return;
    }
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    job_t *jobs = (job_t *)calloc((size_t)threads, sizeof(job_t));
    for (int t = 0; t < threads; t++) {
        jobs[t].fn = fn;
        jobs[t].ctx = ctx;
        jobs[t].begin = n * (size_t)t / (size_t)threads;
        jobs[t].end = n * (size_t)(t + 1) / (size_t)threads;
        pthread_create(&tid[t], NULL, run_job, &jobs[t]);
    }
    for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    free(tid);
    free(jobs);
}

/* ---------------------------------------------------------- entry points -- */

typedef struct {
    const oracle_params *prm;
    uint64_t *states;
} perm_ctx;

static void perm_item(void *c, size_t i) {
    perm_ctx *x = (perm_ctx *)c;
    permute_one(x->prm, x->states + i * WIDTH);
}

/* Permutes n states ([n][12], row-major) in place. */
void oracle_permute(const oracle_params *prm, uint64_t *states, size_t n, int threads) {
    perm_ctx c = {prm, states};
    parallel_for(n, threads, perm_item, &c);
}

typedef struct {
    const oracle_params *prm;
    const uint64_t *leaves;
    size_t n_rows, n_cols;
    uint64_t *digests;
} leaf_ctx;

static void leaf_item(void *c, size_t r) {
    leaf_ctx *x = (leaf_ctx *)c;
    uint64_t *row = (uint64_t *)malloc(x->n_cols * sizeof(uint64_t));
    for (size_t col = 0; col < x->n_cols; col++) row[col] = x->leaves[col * x->n_rows + r];
    sponge(x->prm, row, x->n_cols, x->digests + r * DIGEST);
    free(row);
}

/* Hashes rows r = 0..n_rows-1 of a column-major matrix to [n_rows][4]. */
void oracle_leaf_hash(const oracle_params *prm, const uint64_t *leaves, size_t n_rows, size_t n_cols,
                      uint64_t *digests, int threads) {
    leaf_ctx c = {prm, leaves, n_rows, n_cols, digests};
    parallel_for(n_rows, threads, leaf_item, &c);
}

typedef struct {
    const oracle_params *prm;
    const uint64_t *children;
    size_t n_children;
    uint64_t *parents;
} level_ctx;

static void level_item(void *c, size_t i) {
    level_ctx *x = (level_ctx *)c;
    if (2 * i + 1 < x->n_children) {
        sponge(x->prm, x->children + 2 * i * DIGEST, 2 * DIGEST, x->parents + i * DIGEST);
    } else { /* unpaired last node moves up unchanged */
        memcpy(x->parents + i * DIGEST, x->children + 2 * i * DIGEST, DIGEST * sizeof(uint64_t));
    }
}

/* One tree level: n_children digests -> ceil(n_children/2) parents. */
void oracle_merkle_level(const oracle_params *prm, const uint64_t *children, size_t n_children,
                         uint64_t *parents, int threads) {
    level_ctx c = {prm, children, n_children, parents};
    parallel_for((n_children + 1) / 2, threads, level_item, &c);
}

/* Nodes of a tree with n leaves: sum over levels of n_l, n_{l+1} = ceil(n_l/2). */
size_t oracle_merkle_num_nodes(size_t n) {
    if (n == 0) return 0;
    size_t total = n;
    while (n > 1) {
        n = (n + 1) / 2;
        total += n;
    }
    return total;
}

/* Whole tree: nodes_out gets every node, level-major, leaves' digests first. */
void oracle_merkle_build(const oracle_params *prm, const uint64_t *leaves, size_t n_rows, size_t n_cols,
                         uint64_t *nodes_out, int threads) {
    oracle_leaf_hash(prm, leaves, n_rows, n_cols, nodes_out, threads);
    size_t off = 0, n = n_rows;
    while (n > 1) {
        oracle_merkle_level(prm, nodes_out + off * DIGEST, n, nodes_out + (off + n) * DIGEST, threads);
        off += n;
        n = (n + 1) / 2;
    }
}
