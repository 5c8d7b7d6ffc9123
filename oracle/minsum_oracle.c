/*
 * Min-Sum LDPC decoding oracle: plain, slow, obviously correct CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the HIP library; it extracts its own neighbour
 * sets from the dense parity matrix.
 *
 * What it computes (A mapping of the Min-Sum decoder to reduction operations,
 * Sella & Heinis):
 *   - neighbour sets N_i (row support of H, ascending bit index) and M_j
 *     (column support, ascending check index), Sec. II-B;
 *   - Algorithm 1 (graph form of Min-Sum): the check update of eq. eta_update
 *     taken literally as a minimum and a sign product over k != j for every
 *     edge (O(d^2) per row, no min0/min1 shortcut), the bit update of
 *     eq. lambda_j, the slicer of eq. slice and the GF(2) syndrome H b = 0;
 *   - the pre-loop codeword test of the paper's kernel listing (Sec. IV), so
 *     a channel decision that is already a codeword stops with 0 iterations;
 *   - the paper's own termination variant (Sec. IV, the GPU experiments and
 *     the kernel-profile table): the codeword test runs only after every
 *     k-th iteration (k = 6 there); k = 1 tests after every iteration;
 *   - Algorithm 2 (map-reduce form, Sec. III) on dense m x n arrays, for the
 *     reformulation check only;
 *   - an optional normalised/offset check update (learned per-iteration,
 *     per-check-degree scale alpha and offset beta), which is not in the paper;
 *     alpha = 1, beta = 0 gives plain Min-Sum back bit for bit.
 *
 * Readings of the paper taken here (each is also a decision of the HIP path):
 *   - LLR polarity: a positive LLR favours bit 0 and the slicer outputs
 *     b = 1 iff s < 0.  The paper's text states the opposite polarity, but
 *     under that polarity its plain sign-product check rule is right only for
 *     checks of even degree; under the usual polarity it is right for every
 *     degree.  So the usual polarity is used and the check rule is kept
 *     exactly as printed (on even-degree codes the decisions are the paper's
 *     with the LLR signs flipped).
 *   - sign(v) = -1 if v < 0 else +1, decided by comparison, so sign(-0) = +1
 *     (the paper fixes sign(0) = 1 in Sec. III).
 *   - Iteration count: 0 when the channel decision is a codeword, t when the
 *     first zero syndrome follows iteration t, L when none does; `ok` reports
 *     whether the final decision is a codeword.
 *   - Bit update order: acc = +0; acc = acc + eta_ij for i in M_j ascending;
 *     s_j = acc + r_j.  Every operation is an IEEE binary32 operation with
 *     round-to-nearest-even; build with -ffp-contract=off and no fast-math.
 *   - Rows of degree 1 have no "other" bits, so their message is undefined:
 *     such an H is rejected (status -2).  Rows of degree 0 are always
 *     satisfied; bits of degree 0 keep s = r.
 *
 * Build:  gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared minsum_oracle.c
 *         -o liboracle.so -lpthread -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0 /* planted mistakes, used only by the pin-sensitivity tests */
#endif

/* ------------------------------------------------------------------------ */
/* Neighbour sets N_i and M_j from the dense matrix (Sec. II-B).            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t m, n;
    int64_t E;
    int32_t dmax;      /* largest row degree */
    int64_t *row_start; /* m + 1: edges of N_i are row_start[i] .. row_start[i+1]-1 */
    int32_t *row_bit;   /* E: the bit j of each edge, ascending within a row */
    int32_t *row_class; /* m: index of the row's degree among the sorted distinct degrees */
    int64_t *col_start; /* n + 1 */
    int64_t *col_edge;  /* E: the edge (i, j) for the members i of M_j, ascending i */
} tanner_t;

static void tanner_free(tanner_t *g) {
    free(g->row_start); free(g->row_bit); free(g->row_class);
    free(g->col_start); free(g->col_edge);
    memset(g, 0, sizeof(*g));
}

/* returns 0, or -2 if H holds a value other than 0/1 or a row of degree 1 */
static int tanner_build(const uint8_t *H, int32_t m, int32_t n, tanner_t *g) {
    memset(g, 0, sizeof(*g));
    g->m = m; g->n = n;
    int64_t E = 0;
    for (int64_t k = 0; k < (int64_t)m * n; ++k) {
        if (H[k] > 1) return -2;
        E += H[k];
    }
    g->E = E;
    g->row_start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
    g->row_bit = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
    g->row_class = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    g->col_start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->col_edge = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E ? E : 1));
    if (!g->row_start || !g->row_bit || !g->row_class || !g->col_start || !g->col_edge) {
        tanner_free(g);
        return -1;
    }
    int64_t e = 0;
    g->dmax = 0;
    for (int32_t i = 0; i < m; ++i) {
        g->row_start[i] = e;
        for (int32_t j = 0; j < n; ++j)
            if (H[(int64_t)i * n + j]) g->row_bit[e++] = j;
        int32_t d = (int32_t)(e - g->row_start[i]);
        if (d == 1) { tanner_free(g); return -2; }
        if (d > g->dmax) g->dmax = d;
    }
    g->row_start[m] = e;
    /* degree classes: rank of the row degree among the distinct nonzero row
     * degrees of H, ascending; rows of degree 0 carry no messages (class -1) */
    int32_t *present = (int32_t *)calloc((size_t)n + 2, sizeof(int32_t));
    if (!present) { tanner_free(g); return -1; }
    for (int32_t i = 0; i < m; ++i) present[g->row_start[i + 1] - g->row_start[i]] = 1;
    for (int32_t d = 1, rank = 0; d <= n; ++d) {
        const int32_t here = present[d];
        present[d] = rank;
        rank += here;
    }
    for (int32_t i = 0; i < m; ++i) {
        const int32_t d = (int32_t)(g->row_start[i + 1] - g->row_start[i]);
        g->row_class[i] = d ? present[d] : -1;
    }
    free(present);
    /* M_j: walk rows in ascending order so each column list is ascending in i */
    for (int64_t k = 0; k < E; ++k) g->col_start[g->row_bit[k] + 1]++;
    for (int32_t j = 0; j < n; ++j) g->col_start[j + 1] += g->col_start[j];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!fill) { tanner_free(g); return -1; }
    memcpy(fill, g->col_start, sizeof(int64_t) * ((size_t)n + 1));
    for (int32_t i = 0; i < m; ++i)
        for (int64_t k = g->row_start[i]; k < g->row_start[i + 1]; ++k)
            g->col_edge[fill[g->row_bit[k]]++] = k;
    free(fill);
    return 0;
}

/* The row-degree class table is sized by the caller; this reports it. */
static int32_t tanner_num_classes(const tanner_t *g) {
    int32_t c = 0;
    for (int32_t i = 0; i < g->m; ++i)
        if (g->row_class[i] + 1 > c) c = g->row_class[i] + 1;
    return c;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, one frame.                                                  */
/* ------------------------------------------------------------------------ */

static int hard_bit(float s) {
#if ORACLE_MUTANT == 5
    return s > 0.0f; /* planted: slicer polarity as printed, against the LLR convention */
#else
    return s < 0.0f; /* eq. slice under "positive favours 0"; s = +-0 gives 0 */
#endif
}

static float sgn(float v) { return v < 0.0f ? -1.0f : 1.0f; }

/* H b = 0 over GF(2): every row's XOR of its bits is 0 (eq. 1-2) */
static int syndrome_is_zero(const tanner_t *g, const float *s) {
    for (int32_t i = 0; i < g->m; ++i) {
        int x = 0;
        for (int64_t e = g->row_start[i]; e < g->row_start[i + 1]; ++e) x ^= hard_bit(s[g->row_bit[e]]);
        if (x) return 0;
    }
    return 1;
}

typedef struct {
    const float *alpha, *beta; /* [T][n_classes] or NULL for plain Min-Sum */
    int32_t T, n_classes;
} nms_t;

/* eq. eta_update for every edge of every row, each message from its own
 * minimum and sign product over the other bits of the row. */
static void check_update(const tanner_t *g, const float *s, float *eta, float *x,
                         const nms_t *w, int32_t t) {
    for (int32_t i = 0; i < g->m; ++i) {
        const int64_t e0 = g->row_start[i];
        const int32_t d = (int32_t)(g->row_start[i + 1] - e0);
        for (int32_t a = 0; a < d; ++a) {
#if ORACLE_MUTANT == 2
            x[a] = s[g->row_bit[e0 + a]]; /* planted: no extrinsic subtraction */
#elif ORACLE_MUTANT == 7
            x[a] = eta[e0 + a] - s[g->row_bit[e0 + a]]; /* planted: operands swapped */
#else
            x[a] = s[g->row_bit[e0 + a]] - eta[e0 + a]; /* lambda_k - eta_prev_ik */
#endif
        }
        for (int32_t a = 0; a < d; ++a) {
            float mu = INFINITY;
            float sigma = 1.0f;
            for (int32_t k = 0; k < d; ++k) {
                if (k == a) continue; /* only the other bits of the row, k != j */
                const float mag = fabsf(x[k]);
                if (mag < mu) mu = mag;
                sigma = sigma * sgn(x[k]);
            }
#if ORACLE_MUTANT == 3
            sigma = sigma * sgn(x[a]); /* planted: own sign kept in the product */
#elif ORACLE_MUTANT == 4
            if (fabsf(x[a]) < mu) mu = fabsf(x[a]); /* planted: own magnitude in the min */
#endif
            if (w->alpha) {
#if ORACLE_MUTANT == 11
                const int32_t c = i % w->n_classes; /* planted: class from the row index */
#else
                const int32_t c = g->row_class[i];
#endif
#if ORACLE_MUTANT == 8
                const int64_t tw = t % w->T; /* planted: the next iteration's weights */
#else
                const int64_t tw = t - 1;
#endif
                const float al = w->alpha[tw * w->n_classes + c];
                const float be = w->beta[tw * w->n_classes + c];
#if ORACLE_MUTANT == 9
                const float v = fmaf(al, mu, be); /* planted: offset added */
#else
                const float v = fmaf(al, mu, -be);
#endif
#if ORACLE_MUTANT == 10
                mu = v; /* planted: no clamp at zero */
#else
                mu = v > 0.0f ? v : 0.0f;
#endif
            }
            eta[e0 + a] = sigma * mu;
        }
    }
}

/* eq. lambda_j with the fixed order: +0, then eta_ij for i ascending, then r_j */
static void bit_update(const tanner_t *g, const float *r, const float *eta, float *s) {
    for (int32_t j = 0; j < g->n; ++j) {
        float acc = 0.0f;
        for (int64_t k = g->col_start[j]; k < g->col_start[j + 1]; ++k) acc = acc + eta[g->col_edge[k]];
#if ORACLE_MUTANT == 1
        s[j] = acc; /* planted: channel term dropped */
#else
        s[j] = acc + r[j];
#endif
    }
}

typedef struct {
    float *eta, *s, *x;
} scratch_t;

static void decode_frame(const tanner_t *g, const float *r, int32_t L, int early, const nms_t *w,
                         scratch_t *sc, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok) {
    for (int64_t e = 0; e < g->E; ++e) sc->eta[e] = 0.0f; /* eta = 0 before iteration 1 */
    for (int32_t j = 0; j < g->n; ++j) sc->s[j] = r[j];   /* lambda = r */
    int32_t it = L;
    int done = 0;
#if ORACLE_MUTANT == 6
    int skip_zero = 1; /* planted: no pre-loop codeword test */
#else
    int skip_zero = 0;
#endif
    /* early = the codeword-test period k (0: never test, run all L iterations) */
    if (early && !skip_zero && syndrome_is_zero(g, sc->s)) { it = 0; done = 1; }
    for (int32_t t = 1; !done && t <= L; ++t) {
        check_update(g, sc->s, sc->eta, sc->x, w, t);
        bit_update(g, r, sc->eta, sc->s);
        if (early && t % early == 0 && syndrome_is_zero(g, sc->s)) { it = t; done = 1; }
    }
    for (int32_t j = 0; j < g->n; ++j) {
        if (bits) bits[j] = (uint8_t)hard_bit(sc->s[j]);
        if (post) post[j] = sc->s[j];
    }
    if (iters) *iters = it;
    if (ok) *ok = (uint8_t)syndrome_is_zero(g, sc->s);
}

/* ------------------------------------------------------------------------ */
/* Batch driver: frames are independent, split into contiguous ranges.      */
/* ------------------------------------------------------------------------ */

typedef struct {
    const tanner_t *g;
    const float *llr;
    int32_t b0, b1, L, early;
    nms_t w;
    uint8_t *bits; float *post; int32_t *iters; uint8_t *ok;
    int status;
} job_t;

static void *run_job(void *p) {
    job_t *jb = (job_t *)p;
    const tanner_t *g = jb->g;
    scratch_t sc;
    sc.eta = (float *)malloc(sizeof(float) * (size_t)(g->E ? g->E : 1));
    sc.s = (float *)malloc(sizeof(float) * (size_t)(g->n ? g->n : 1));
    sc.x = (float *)malloc(sizeof(float) * (size_t)(g->dmax ? g->dmax : 1));
    if (!sc.eta || !sc.s || !sc.x) { jb->status = -1; goto out; }
    for (int32_t f = jb->b0; f < jb->b1; ++f) {
        const int64_t o = (int64_t)f * g->n;
        decode_frame(g, jb->llr + o, jb->L, jb->early, &jb->w, &sc,
                     jb->bits ? jb->bits + o : NULL, jb->post ? jb->post + o : NULL,
                     jb->iters ? jb->iters + f : NULL, jb->ok ? jb->ok + f : NULL);
    }
    jb->status = 0;
out:
    free(sc.eta); free(sc.s); free(sc.x);
    return NULL;
}

static int run_batch(const tanner_t *g, const float *llr, int32_t B, int32_t L, int32_t early,
                     const nms_t *w, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok,
                     int32_t nthreads) {
    if (nthreads <= 0) nthreads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > B) nthreads = B > 0 ? B : 1;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -1; }
    for (int32_t k = 0; k < nthreads; ++k) {
        job_t *jb = &jobs[k];
        jb->g = g; jb->llr = llr; jb->L = L; jb->early = early; jb->w = *w;
        jb->b0 = (int32_t)((int64_t)B * k / nthreads);
        jb->b1 = (int32_t)((int64_t)B * (k + 1) / nthreads);
        jb->bits = bits; jb->post = post; jb->iters = iters; jb->ok = ok;
    }
    int status = 0;
    if (nthreads == 1) {
        run_job(&jobs[0]);
        status = jobs[0].status;
    } else {
        for (int32_t k = 0; k < nthreads; ++k) pthread_create(&th[k], NULL, run_job, &jobs[k]);
        for (int32_t k = 0; k < nthreads; ++k) {
            pthread_join(th[k], NULL);
            if (jobs[k].status) status = jobs[k].status;
        }
    }
    free(jobs); free(th);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points.  All buffers are host memory, row-major:          */
/*   H m x n (0/1), llr B x n, bits B x n, post B x n, iters B, ok B.       */
/* Output pointers may be NULL.  early_exit: 0 runs all max_iter            */
/* iterations; k >= 1 tests for a codeword before the first iteration and   */
/* after every k-th one.  Returns 0, -1 (bad argument / no memory) or -2    */
/* (H not 0/1, or a row of degree 1).                                        */
/* ------------------------------------------------------------------------ */

int oracle_minsum_decode(const uint8_t *H, int32_t m, int32_t n, const float *llr, int32_t B,
                         int32_t max_iter, int32_t early_exit, uint8_t *bits, float *post,
                         int32_t *iters, uint8_t *ok, int32_t nthreads) {
    if (!H || m < 1 || n < 1 || B < 0 || max_iter < 0 || early_exit < 0 || (B > 0 && !llr)) return -1;
    tanner_t g;
    int st = tanner_build(H, m, n, &g);
    if (st) return st;
    nms_t w = {NULL, NULL, 0, 0};
    st = run_batch(&g, llr, B, max_iter, early_exit, &w, bits, post, iters, ok, nthreads);
    tanner_free(&g);
    return st;
}

/* Normalised/offset Min-Sum: the message magnitude mu of row i at iteration t
 * becomes max(fma(alpha[t-1][c], mu, -beta[t-1][c]), 0), c the rank of the
 * row's degree among the distinct row degrees of H (ascending).  Requires
 * max_iter <= T. */
int oracle_nms_decode(const uint8_t *H, int32_t m, int32_t n, const float *llr, int32_t B,
                      int32_t max_iter, int32_t early_exit, const float *alpha, const float *beta,
                      int32_t T, int32_t n_classes, uint8_t *bits, float *post, int32_t *iters,
                      uint8_t *ok, int32_t nthreads) {
    if (!H || m < 1 || n < 1 || B < 0 || max_iter < 0 || max_iter > T || early_exit < 0 || !alpha ||
        !beta || (B > 0 && !llr))
        return -1;
    tanner_t g;
    int st = tanner_build(H, m, n, &g);
    if (st) return st;
    if (tanner_num_classes(&g) != n_classes) { tanner_free(&g); return -1; }
    nms_t w = {alpha, beta, T, n_classes};
    st = run_batch(&g, llr, B, max_iter, early_exit, &w, bits, post, iters, ok, nthreads);
    tanner_free(&g);
    return st;
}

/* The sorted distinct row degrees of H; returns their count (or < 0). */
int32_t oracle_check_degrees(const uint8_t *H, int32_t m, int32_t n, int32_t *degrees, int32_t cap) {
    tanner_t g;
    int st = tanner_build(H, m, n, &g);
    if (st) return st;
    int32_t c = tanner_num_classes(&g);
    for (int32_t i = 0; i < m && degrees; ++i) {
        int32_t k = g.row_class[i];
        if (k < cap) degrees[k] = (int32_t)(g.row_start[i + 1] - g.row_start[i]);
    }
    tanner_free(&g);
    return c;
}

/* syndrome[b][i] = XOR of bits[b][j] over j in N_i */
int oracle_syndrome(const uint8_t *H, int32_t m, int32_t n, const uint8_t *bits, int32_t B,
                    uint8_t *syndrome) {
    if (!H || !bits || !syndrome || m < 1 || n < 1 || B < 0) return -1;
    for (int32_t f = 0; f < B; ++f)
        for (int32_t i = 0; i < m; ++i) {
            int x = 0;
            for (int32_t j = 0; j < n; ++j)
                if (H[(int64_t)i * n + j]) x ^= bits[(int64_t)f * n + j] & 1;
            syndrome[(int64_t)f * m + i] = (uint8_t)x;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (Sec. III), literally, on dense m x n arrays, one frame.      */
/* The masked entries are real zeros and take part in every reduction; the  */
/* argmin entry receives min1 and the others min0 (Observation 1; the       */
/* printed eq. etaCalculation has the two swapped).                          */
/* ------------------------------------------------------------------------ */

/* dense H b over the integers, then mod 2 (the listing's product-then-mod) */
static int dense_is_codeword(const uint8_t *H, int32_t m, int32_t n, const float *s) {
    for (int32_t i = 0; i < m; ++i) {
        int64_t acc = 0;
        for (int32_t j = 0; j < n; ++j) acc += (int64_t)H[(size_t)i * n + j] * hard_bit(s[j]);
        if (acc % 2) return 0;
    }
    return 1;
}

int oracle_minsum_dense(const uint8_t *H, int32_t m, int32_t n, const float *r, int32_t L,
                        int32_t early_exit, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok) {
    if (!H || !r || m < 1 || n < 1 || L < 0) return -1;
    for (int64_t k = 0; k < (int64_t)m * n; ++k)
        if (H[k] > 1) return -2;
    const size_t mn = (size_t)m * (size_t)n;
    float *lam = (float *)malloc(sizeof(float) * mn);
    float *eta = (float *)malloc(sizeof(float) * mn);
    float *s = (float *)malloc(sizeof(float) * (size_t)n);
    if (!lam || !eta || !s) { free(lam); free(eta); free(s); return -1; }
    for (size_t k = 0; k < mn; ++k) eta[k] = 0.0f;
    for (int32_t j = 0; j < n; ++j) s[j] = r[j];
    /* fan-out, eq. firstIterationFanOut */
    for (int32_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < n; ++j) lam[(size_t)i * n + j] = r[j] * (float)H[(size_t)i * n + j];

    int32_t it = L;
    int done = 0;
    if (early_exit && dense_is_codeword(H, m, n, s)) { it = 0; done = 1; }
    for (int32_t t = 1; !done && t <= L; ++t) {
        for (int32_t i = 0; i < m; ++i) {
            const float *row = lam + (size_t)i * n;
            const uint8_t *hr = H + (size_t)i * n;
            int32_t deg = 0;
            for (int32_t j = 0; j < n; ++j) deg += hr[j];
            if (deg == 0) { /* no messages; avoids 0 * inf below */
                for (int32_t j = 0; j < n; ++j) eta[(size_t)i * n + j] = 0.0f;
                continue;
            }
            float min0 = INFINITY, min1 = INFINITY;
            int32_t loc = -1;
            for (int32_t j = 0; j < n; ++j)
                if (hr[j] && fabsf(row[j]) < min0) { min0 = fabsf(row[j]); loc = j; }
            for (int32_t j = 0; j < n; ++j)
                if (hr[j] && j != loc && fabsf(row[j]) < min1) min1 = fabsf(row[j]);
            float sg = 1.0f; /* product over the whole row; masked zeros have sign +1 */
            for (int32_t j = 0; j < n; ++j) sg = sg * sgn(row[j]);
            for (int32_t j = 0; j < n; ++j) {
                const float mag = (j == loc) ? min1 : min0;
                eta[(size_t)i * n + j] = (float)hr[j] * (sgn(row[j]) * sg * mag);
            }
        }
        /* eq. sCalculation: column reduction over every i, then + r */
        for (int32_t j = 0; j < n; ++j) {
            float acc = 0.0f;
            for (int32_t i = 0; i < m; ++i) acc = acc + eta[(size_t)i * n + j];
            s[j] = acc + r[j];
        }
        if (early_exit && dense_is_codeword(H, m, n, s)) { it = t; done = 1; break; }
        /* later iterations: lambda(i,j) = s(j) H(i,j) - eta(i,j) */
        for (int32_t i = 0; i < m; ++i)
            for (int32_t j = 0; j < n; ++j)
                lam[(size_t)i * n + j] = s[j] * (float)H[(size_t)i * n + j] - eta[(size_t)i * n + j];
    }
    const int okv = dense_is_codeword(H, m, n, s);
    for (int32_t j = 0; j < n; ++j) {
        if (bits) bits[j] = (uint8_t)hard_bit(s[j]);
        if (post) post[j] = s[j];
    }
    if (iters) *iters = it;
    if (ok) *ok = (uint8_t)okv;
    free(lam); free(eta); free(s);
    return 0;
}
