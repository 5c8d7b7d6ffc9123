/*
 * FP64 oracle of the learned (normalised / offset) Min-Sum training
 * objective and its gradient.  TEST INFRASTRUCTURE ONLY: it may be loaded by
 * the tests and the benchmark's CPU-baseline leg, never by the product path.
 *
 * The paper decodes with plain Min-Sum (Algorithm 1).  The learned variant
 * replaces the message magnitude mu of eq. eta_update in iteration t by
 *     max(alpha[t-1][c] * mu - beta[t-1][c], 0)
 * where c is the rank of the check row's degree among the distinct nonzero
 * row degrees of H (ascending).  Training unrolls exactly T iterations (no
 * syndrome exit) and minimises
 *     loss = 1/(B n) * sum_frames sum_{t=1..T} sum_j softplus((2 c_j - 1) s_j^(t))
 * the binary cross-entropy of every iteration's posterior s^(t) against the
 * transmitted bits c (P(bit = 1) = sigmoid(-s) under "positive LLR favours 0").
 *
 * The plain definitions it follows:
 *   x_e   = s_j - eta_e (eta = 0 and s = r before iteration 1)
 *   mu_e  = min over the other edges k of row i of |x_k|
 *   sg_e  = product over the other edges of sign(x_k), sign(0) = +1
 *   v_e   = alpha mu_e - beta
 *   eta_e = sg_e * max(v_e, 0)
 *   s_j   = r_j + sum over the checks of bit j of eta_e
 * and the reverse sweep of the chain rule, where the derivative of mu_e goes
 * to the edge attaining the minimum over the other edges (the lowest edge
 * position on a tie), d|x|/dx = sign(x), the sign product is held constant and
 * the derivative of max(v, 0) is [v > 0].
 *
 * Two forwards feed the same reverse sweep:
 *   - double precision throughout (the training objective as a real
 *     function; the finite-difference pins check this mode);
 *   - the binary32 decoder's own forward (x, v = fma(alpha, mu, -beta) and the
 *     column sum +0, messages in ascending check order, then + r, each rounded
 *     to binary32, as the decoding oracle does), stored exactly in doubles.
 *     The reverse sweep then runs in double precision along the binary32
 *     forward's decisions: its argmin and second-minimum positions, its signs
 *     and its clip masks [v > 0].  This is the gradient a binary32 backward
 *     must approximate; near a tie of two magnitudes the double-precision
 *     forward can pick another minimum, so only this mode can be compared
 *     with a binary32 implementation entry by entry.
 * Alongside the gradient the sweep can return its magnitude bound: the same
 * sweep with every term replaced by its absolute value (|alpha|, |mu|,
 * |sigmoid|, sums of absolute values).  An implementation that rounds each
 * operation to binary32 differs from the exact sweep by at most
 * k u (magnitude bound) for k roundings along the longest dependency chain
 * and u = 2^-24 (forward error of sums and products).
 *
 * Build: compiled into liboracle.so together with minsum_oracle.c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t m, n, E, dmax, ncls;
    int32_t *rs;   /* m + 1 */
    int32_t *rb;   /* E: bit of each edge, ascending in a row */
    int32_t *rc;   /* m: degree class */
} rows_t;

static void rows_free(rows_t *g) {
    free(g->rs); free(g->rb); free(g->rc);
    memset(g, 0, sizeof(*g));
}

/* neighbour sets N_i of Sec. II-B from the dense matrix, and degree classes */
static int rows_build(const uint8_t *H, int32_t m, int32_t n, rows_t *g) {
    memset(g, 0, sizeof(*g));
    g->m = m; g->n = n;
    int64_t E = 0;
    for (int64_t k = 0; k < (int64_t)m * n; ++k) {
        if (H[k] > 1) return -2;
        E += H[k];
    }
    g->E = (int32_t)E;
    g->rs = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
    g->rb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
    g->rc = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *present = (int32_t *)calloc((size_t)n + 2, sizeof(int32_t));
    if (!g->rs || !g->rb || !g->rc || !present) { free(present); rows_free(g); return -1; }
    int32_t e = 0;
    for (int32_t i = 0; i < m; ++i) {
        g->rs[i] = e;
        for (int32_t j = 0; j < n; ++j)
            if (H[(int64_t)i * n + j]) g->rb[e++] = j;
        const int32_t d = e - g->rs[i];
        if (d == 1) { free(present); rows_free(g); return -2; }
        if (d > g->dmax) g->dmax = d;
        present[d] = 1;
    }
    g->rs[m] = e;
    int32_t rank = 0;
    for (int32_t d = 1; d <= n; ++d) {
        const int32_t here = present[d];
        present[d] = rank;
        rank += here;
    }
    g->ncls = rank;
    for (int32_t i = 0; i < m; ++i) {
        const int32_t d = g->rs[i + 1] - g->rs[i];
        g->rc[i] = d ? present[d] : -1;
    }
    free(present);
    return 0;
}

static double sgn(double v) { return v < 0.0 ? -1.0 : 1.0; }
static double softplus(double z) { return z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z)); }
static double sigmoid(double z) { return z >= 0.0 ? 1.0 / (1.0 + exp(-z)) : exp(z) / (1.0 + exp(z)); }

/* position (within the row) of the smallest |x| over the row's edges other
 * than `skip`, lowest position on a tie */
static int32_t argmin_other(const double *x, int32_t d, int32_t skip) {
    int32_t best = -1;
    for (int32_t k = 0; k < d; ++k) {
        if (k == skip) continue;
        if (best < 0 || fabs(x[k]) < fabs(x[best])) best = k;
    }
    return best;
}

/* v = alpha mu - beta of the clipped message magnitude: exact in double, or
 * the binary32 decoder's fused multiply-add rounded once to binary32 */
static double clip_arg(double al, double mu, double be, int f32) {
    if (f32) return (double)fmaf((float)al, (float)mu, -(float)be);
    return al * mu - be;
}

/* the scratch arrays of one frame */
typedef struct {
    double *xs;  /* (T+1) x E: x^(t) of every edge */
    double *ss;  /* (T+1) x n: s^(t), s^(0) = r */
    double *eta; /* E */
    double *gs, *gx, *gxn;    /* n, E, E */
    double *as, *ax, *axn;    /* magnitude bound of gs, gx, gxn */
} work_t;

/*
 * One frame: loss (not divided by B n) and, when galpha is non-NULL, its
 * gradient accumulated into galpha, gbeta ([T][ncls]) and gr ([n], may be
 * NULL); when aalpha is non-NULL also the magnitude bound of each gradient
 * entry into aalpha, abeta and ar (ar may be NULL).  target: n bits (NULL =
 * all-zero codeword).  f32: the forward in binary32 arithmetic (see the
 * file comment); post (may be NULL) receives s^(T).
 */
static double frame(const rows_t *g, const double *r, const uint8_t *target, const double *alpha,
                    const double *beta, int32_t T, int f32, double *galpha, double *gbeta, double *gr,
                    double *aalpha, double *abeta, double *ar, double scale, double *post, work_t *w) {
    const int32_t E = g->E, n = g->n, m = g->m;
    double *xs = w->xs, *ss = w->ss, *eta = w->eta;
    double loss = 0.0;
    for (int32_t e = 0; e < E; ++e) eta[e] = 0.0;
    for (int32_t j = 0; j < n; ++j) ss[j] = r[j];
    for (int32_t t = 1; t <= T; ++t) {
        double *x = xs + (size_t)t * E;
        const double *sp = ss + (size_t)(t - 1) * n;
        double *s = ss + (size_t)t * n;
        for (int32_t i = 0; i < m; ++i)
            for (int32_t e = g->rs[i]; e < g->rs[i + 1]; ++e)
                x[e] = f32 ? (double)((float)sp[g->rb[e]] - (float)eta[e]) : sp[g->rb[e]] - eta[e];
        for (int32_t i = 0; i < m; ++i) {
            const int32_t e0 = g->rs[i], d = g->rs[i + 1] - e0;
            if (d == 0) continue;
            const double al = alpha[(size_t)(t - 1) * g->ncls + g->rc[i]];
            const double be = beta[(size_t)(t - 1) * g->ncls + g->rc[i]];
            for (int32_t a = 0; a < d; ++a) {
                double mu = INFINITY, sg = 1.0;
                for (int32_t k = 0; k < d; ++k) {
                    if (k == a) continue;
                    if (fabs(x[e0 + k]) < mu) mu = fabs(x[e0 + k]);
                    sg *= sgn(x[e0 + k]);
                }
                const double v = clip_arg(al, mu, be, f32);
                eta[e0 + a] = sg * (v > 0.0 ? v : 0.0);
            }
        }
        if (f32) {
            /* eq. lambda_j in the decoder's order: +0, the messages of M_j in
             * ascending check order, then r_j, each addition in binary32 */
            for (int32_t j = 0; j < n; ++j) s[j] = 0.0;
            for (int32_t i = 0; i < m; ++i) /* rows ascending: each column's messages in ascending i */
                for (int32_t e = g->rs[i]; e < g->rs[i + 1]; ++e)
                    s[g->rb[e]] = (double)((float)s[g->rb[e]] + (float)eta[e]);
            for (int32_t j = 0; j < n; ++j) s[j] = (double)((float)s[j] + (float)r[j]);
        } else {
            for (int32_t j = 0; j < n; ++j) s[j] = r[j];
            for (int32_t i = 0; i < m; ++i)
                for (int32_t e = g->rs[i]; e < g->rs[i + 1]; ++e) s[g->rb[e]] += eta[e];
        }
        for (int32_t j = 0; j < n; ++j) {
            const double y = (target && target[j]) ? 1.0 : -1.0; /* 2c - 1 */
            loss += softplus(y * s[j]);
        }
    }
    if (post)
        for (int32_t j = 0; j < n; ++j) post[j] = ss[(size_t)T * n + j];
    if (!galpha) return loss;

    /* reverse sweep; the magnitude bound runs beside it with |.| of every term */
    double *gs = w->gs, *gx = w->gx, *gxn = w->gxn;
    double *as = w->as, *ax = w->ax, *axn = w->axn;
    const int bound = aalpha != NULL;
    for (int32_t e = 0; e < E; ++e) gxn[e] = axn[e] = 0.0; /* d loss / d x^(t+1) */
    for (int32_t t = T; t >= 1; --t) {
        const double *x = xs + (size_t)t * E;
        const double *s = ss + (size_t)t * n;
        /* d/ds^(t): the loss term of iteration t, and s^(t) inside x^(t+1) */
        for (int32_t j = 0; j < n; ++j) {
            const double y = (target && target[j]) ? 1.0 : -1.0;
            gs[j] = scale * y * sigmoid(y * s[j]);
            as[j] = fabs(gs[j]);
        }
        for (int32_t i = 0; i < m; ++i)
            for (int32_t e = g->rs[i]; e < g->rs[i + 1]; ++e) {
                gs[g->rb[e]] += gxn[e];
                as[g->rb[e]] += axn[e];
            }
        for (int32_t j = 0; j < n; ++j) { /* s^(t) = r + ... */
            if (gr) gr[j] += gs[j];
            if (bound && ar) ar[j] += as[j];
        }
        for (int32_t e = 0; e < E; ++e) gx[e] = ax[e] = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            const int32_t e0 = g->rs[i], d = g->rs[i + 1] - e0;
            if (d == 0) continue;
            const int32_t c = g->rc[i];
            const double al = alpha[(size_t)(t - 1) * g->ncls + c];
            const double be = beta[(size_t)(t - 1) * g->ncls + c];
            for (int32_t a = 0; a < d; ++a) {
                const int32_t e = e0 + a;
                /* eta^(t)_e enters s^(t) with + and x^(t+1)_e with - */
                const double geta = gs[g->rb[e]] - gxn[e];
                const double aeta = as[g->rb[e]] + axn[e];
                const int32_t ks = argmin_other(x + e0, d, a);
                const double mu = fabs(x[e0 + ks]);
                double sg = 1.0;
                for (int32_t k = 0; k < d; ++k)
                    if (k != a) sg *= sgn(x[e0 + k]);
                const double v = clip_arg(al, mu, be, f32);
                if (!(v > 0.0)) continue;
                const double gv = geta * sg;
                galpha[(size_t)(t - 1) * g->ncls + c] += gv * mu;
                gbeta[(size_t)(t - 1) * g->ncls + c] -= gv;
                gx[e0 + ks] += gv * al * sgn(x[e0 + ks]);
                if (bound) {
                    aalpha[(size_t)(t - 1) * g->ncls + c] += aeta * mu;
                    abeta[(size_t)(t - 1) * g->ncls + c] += aeta;
                    ax[e0 + ks] += aeta * fabs(al);
                }
            }
        }
        /* x^(t) = s^(t-1) - eta^(t-1): gx flows to both in the next step down */
        memcpy(gxn, gx, sizeof(double) * (size_t)E);
        memcpy(axn, ax, sizeof(double) * (size_t)E);
    }
    for (int32_t i = 0; i < m; ++i) /* x^(1) = r - 0 */
        for (int32_t e = g->rs[i]; e < g->rs[i + 1]; ++e) {
            if (gr) gr[g->rb[e]] += gxn[e];
            if (bound && ar) ar[g->rb[e]] += axn[e];
        }
    return loss;
}

/*
 * Mean loss over B frames and n bits and, if galpha != NULL, its gradient
 * with respect to alpha and beta ([T][ncls]) and, if gllr != NULL, the
 * channel LLRs ([B][n]).  targets: [B][n] bits or NULL (all-zero).
 * f32 = 0: double-precision forward; f32 = 1: the binary32 decoder's forward
 * (llr, alpha and beta must then hold binary32 values), the reverse sweep in
 * double along its decisions.  aalpha, abeta, allr (each may be NULL; allr
 * only with gllr): magnitude bounds of the gradient entries.  post: [B][n]
 * posteriors after iteration T, or NULL.
 * Returns 0, -1 (argument or memory) or -2 (bad H).
 */
int oracle_nms_train_loss_grad_ex(const uint8_t *H, int32_t m, int32_t n, const double *llr,
                                  const uint8_t *targets, int32_t B, const double *alpha, const double *beta,
                                  int32_t T, int32_t ncls, int32_t f32, double *loss, double *galpha,
                                  double *gbeta, double *gllr, double *aalpha, double *abeta, double *allr,
                                  double *post) {
    if (!H || !llr || !alpha || !beta || !loss || m < 1 || n < 1 || B < 1 || T < 1) return -1;
    if ((galpha == NULL) != (gbeta == NULL) || (aalpha == NULL) != (abeta == NULL)) return -1;
    if ((aalpha && !galpha) || (allr && (!gllr || !aalpha))) return -1;
    rows_t g;
    int st = rows_build(H, m, n, &g);
    if (st) return st;
    if (g.ncls != ncls) { rows_free(&g); return -1; }
    const size_t E = (size_t)(g.E ? g.E : 1);
    work_t w;
    w.xs = (double *)malloc(sizeof(double) * E * (size_t)(T + 1));
    w.ss = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(T + 1));
    w.eta = (double *)malloc(sizeof(double) * E);
    w.gs = (double *)malloc(sizeof(double) * (size_t)n);
    w.gx = (double *)malloc(sizeof(double) * E);
    w.gxn = (double *)malloc(sizeof(double) * E);
    w.as = (double *)malloc(sizeof(double) * (size_t)n);
    w.ax = (double *)malloc(sizeof(double) * E);
    w.axn = (double *)malloc(sizeof(double) * E);
    if (!w.xs || !w.ss || !w.eta || !w.gs || !w.gx || !w.gxn || !w.as || !w.ax || !w.axn) {
        free(w.xs); free(w.ss); free(w.eta); free(w.gs); free(w.gx); free(w.gxn);
        free(w.as); free(w.ax); free(w.axn); rows_free(&g);
        return -1;
    }
    const double scale = 1.0 / ((double)B * (double)n);
    if (galpha) {
        memset(galpha, 0, sizeof(double) * (size_t)T * (size_t)ncls);
        memset(gbeta, 0, sizeof(double) * (size_t)T * (size_t)ncls);
    }
    if (aalpha) {
        memset(aalpha, 0, sizeof(double) * (size_t)T * (size_t)ncls);
        memset(abeta, 0, sizeof(double) * (size_t)T * (size_t)ncls);
    }
    double total = 0.0;
    for (int32_t f = 0; f < B; ++f) {
        double *gr = gllr ? gllr + (size_t)f * n : NULL;
        double *ar = allr ? allr + (size_t)f * n : NULL;
        if (gr) memset(gr, 0, sizeof(double) * (size_t)n);
        if (ar) memset(ar, 0, sizeof(double) * (size_t)n);
        total += frame(&g, llr + (size_t)f * n, targets ? targets + (size_t)f * n : NULL, alpha, beta, T, f32 != 0,
                       galpha, gbeta, gr, aalpha, abeta, ar, scale, post ? post + (size_t)f * n : NULL, &w);
    }
    *loss = total * scale;
    free(w.xs); free(w.ss); free(w.eta); free(w.gs); free(w.gx); free(w.gxn);
    free(w.as); free(w.ax); free(w.axn);
    rows_free(&g);
    return 0;
}

/* The double-precision objective and gradient (no bounds, no posteriors). */
int oracle_nms_train_loss_grad(const uint8_t *H, int32_t m, int32_t n, const double *llr, const uint8_t *targets,
                               int32_t B, const double *alpha, const double *beta, int32_t T, int32_t ncls,
                               double *loss, double *galpha, double *gbeta, double *gllr) {
    return oracle_nms_train_loss_grad_ex(H, m, n, llr, targets, B, alpha, beta, T, ncls, 0, loss, galpha, gbeta,
                                         gllr, NULL, NULL, NULL, NULL);
}
