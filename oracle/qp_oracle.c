/*
 * Plain FP64 CPU oracle for the all-pairs posterior stage (stage I) of
 * QuickProbs 2 (Methods, opening paragraph: posterior probability matrices
 * for every sequence pair from a pair hidden Markov model and from a
 * partition function, then maximum-expected-accuracy scores).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; it exists so that tests, the smoke check and the CPU baseline
 * leg of the benchmark can compare the GPU path with an independent,
 * obviously correct implementation.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * Everything is computed in log space in double precision, single threaded,
 * with full (m+1) x (n+1) matrices per state -- no blocking, no scaling
 * tricks, no fusion.  The model readings (the paper only names the models)
 * are:
 *   - alignment = monotone sequence of match columns M(i,j), x-gap columns
 *     X(i) and y-gap columns Y(j); an X column is never adjacent to a Y
 *     column (classic pair-HMM topology, applied to both models);
 *   - begin and end behave as a match state (virtual M before the first and
 *     after the last column);
 *   - pair-HMM with G gap classes: M->M tau = 1 - 2*sum(delta_k),
 *     M->X_k = M->Y_k = delta_k, X_k->X_k = eps_k, X_k->M = 1 - eps_k;
 *     match emission in odds form e_ab = p_ab / (qx_a qy_b) with qx, qy the
 *     row and column marginals of the joint p (insert emissions cancel);
 *   - partition function: weight exp(score/T) with score = sum of s_ab over
 *     match columns + for every gap run (g_open + (L-1) g_ext); this is the
 *     same recurrence with M->M = 1, open = exp(g_open/T),
 *     extend = exp(g_ext/T), close = 1, emission exp(s_ab/T);
 *   - posterior P(i,j) = f_M(i,j) b_M(i,j) / Z for both models, combined as
 *     w * P_hmm + (1 - w) * P_pf;
 *   - expected accuracy: A(i,j) = max(A(i-1,j-1) + P(i,j), A(i-1,j),
 *     A(i,j-1)) on the dense combined matrix, EA = A(m,n) / min(m,n).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QPO_ALPHA 20
#define QPO_MAXG 4

/* One model in generic transition form (log weights). */
typedef struct {
    int G;                                   /* number of gap classes       */
    double l_mm;                             /* log M->M                    */
    double l_open[QPO_MAXG];                 /* log M->X_k (= M->Y_k)       */
    double l_ext[QPO_MAXG];                  /* log X_k->X_k                */
    double l_close[QPO_MAXG];                /* log X_k->M  (and X_k->end)  */
    double l_emit[QPO_ALPHA * QPO_ALPHA];    /* log match weight [x][y]     */
} qpo_model;

static const double NEG_INF = -INFINITY;

/* log(exp(a) + exp(b)) */
static double lse2(double a, double b) {
    if (a == NEG_INF) return b;
    if (b == NEG_INF) return a;
    if (a > b) return a + log1p(exp(b - a));
    return b + log1p(exp(a - b));
}

/* Forward and backward over one model; fills pm (m*n) with the posterior of
 * each match cell, returns log Z from the forward pass in *lz_f and from the
 * backward pass in *lz_b.  Matrices are (m+1) x (n+1), index i*(n+1)+j. */
static int run_model(const qpo_model* md, const uint8_t* x, int m, const uint8_t* y, int n,
                     double* pm, double* lz_f, double* lz_b) {
    const int W = n + 1;
    const size_t cells = (size_t)(m + 1) * (size_t)(n + 1);
    const int G = md->G;
    const int S = 1 + 2 * G;  /* M, X_1..X_G, Y_1..Y_G */
    double* f = (double*)malloc(sizeof(double) * cells * S);
    double* b = (double*)malloc(sizeof(double) * cells * S);
    if (!f || !b) { free(f); free(b); return -1; }
#define FM(i, j) f[((size_t)(i) * W + (j)) * S]
#define FX(k, i, j) f[((size_t)(i) * W + (j)) * S + 1 + (k)]
#define FY(k, i, j) f[((size_t)(i) * W + (j)) * S + 1 + G + (k)]
#define BM(i, j) b[((size_t)(i) * W + (j)) * S]
#define BX(k, i, j) b[((size_t)(i) * W + (j)) * S + 1 + (k)]
#define BY(k, i, j) b[((size_t)(i) * W + (j)) * S + 1 + G + (k)]
#define EMIT(i, j) md->l_emit[x[(i) - 1] * QPO_ALPHA + y[(j) - 1]]

    /* ---- forward ---- */
    for (int i = 0; i <= m; ++i) {
        for (int j = 0; j <= n; ++j) {
            /* match state: reached from (i-1, j-1) */
            double vm = NEG_INF;
            if (i == 0 && j == 0) {
                vm = 0.0; /* virtual begin state, weight 1 */
            } else if (i >= 1 && j >= 1) {
                double into = md->l_mm + FM(i - 1, j - 1);
                for (int k = 0; k < G; ++k) {
                    into = lse2(into, md->l_close[k] + FX(k, i - 1, j - 1));
                    into = lse2(into, md->l_close[k] + FY(k, i - 1, j - 1));
                }
                vm = EMIT(i, j) + into;
            }
            FM(i, j) = vm;
            for (int k = 0; k < G; ++k) {
                double vx = NEG_INF, vy = NEG_INF;
                if (i >= 1) vx = lse2(md->l_open[k] + FM(i - 1, j), md->l_ext[k] + FX(k, i - 1, j));
                if (j >= 1) vy = lse2(md->l_open[k] + FM(i, j - 1), md->l_ext[k] + FY(k, i, j - 1));
                FX(k, i, j) = vx;
                FY(k, i, j) = vy;
            }
        }
    }
    double zf = md->l_mm + FM(m, n);
    for (int k = 0; k < G; ++k) {
        zf = lse2(zf, md->l_close[k] + FX(k, m, n));
        zf = lse2(zf, md->l_close[k] + FY(k, m, n));
    }

    /* ---- backward ---- */
    for (int i = m; i >= 0; --i) {
        for (int j = n; j >= 0; --j) {
            /* t = weight of continuing with the match column (i+1, j+1), or
             * of ending when (i, j) is the last cell */
            double t = NEG_INF;
            if (i == m && j == n) t = 0.0;
            else if (i < m && j < n) t = EMIT(i + 1, j + 1) + BM(i + 1, j + 1);
            double vm = md->l_mm + t;
            for (int k = 0; k < G; ++k) {
                if (i < m) vm = lse2(vm, md->l_open[k] + BX(k, i + 1, j));
                if (j < n) vm = lse2(vm, md->l_open[k] + BY(k, i, j + 1));
            }
            BM(i, j) = vm;
            for (int k = 0; k < G; ++k) {
                double vx = md->l_close[k] + t;
                double vy = md->l_close[k] + t;
                if (i < m) vx = lse2(vx, md->l_ext[k] + BX(k, i + 1, j));
                if (j < n) vy = lse2(vy, md->l_ext[k] + BY(k, i, j + 1));
                BX(k, i, j) = vx;
                BY(k, i, j) = vy;
            }
        }
    }
    double zb = BM(0, 0);

    for (int i = 1; i <= m; ++i)
        for (int j = 1; j <= n; ++j)
            pm[(size_t)(i - 1) * n + (j - 1)] = exp(FM(i, j) + BM(i, j) - zf);

    *lz_f = zf;
    *lz_b = zb;
    free(f);
    free(b);
#undef FM
#undef FX
#undef FY
#undef BM
#undef BX
#undef BY
#undef EMIT
    return 0;
}

/* Pair-HMM tables from the raw joint emission and gap probabilities. */
static int make_hmm(qpo_model* md, const double* joint, int G, const double* delta, const double* eps) {
    if (G < 1 || G > QPO_MAXG) return -2;
    double qx[QPO_ALPHA] = {0}, qy[QPO_ALPHA] = {0};
    for (int a = 0; a < QPO_ALPHA; ++a)
        for (int c = 0; c < QPO_ALPHA; ++c) {
            qx[a] += joint[a * QPO_ALPHA + c];
            qy[c] += joint[a * QPO_ALPHA + c];
        }
    double tau = 1.0;
    for (int k = 0; k < G; ++k) tau -= 2.0 * delta[k];
    if (!(tau > 0.0)) return -2;
    md->G = G;
    md->l_mm = log(tau);
    for (int k = 0; k < G; ++k) {
        md->l_open[k] = log(delta[k]);
        md->l_ext[k] = log(eps[k]);
        md->l_close[k] = log(1.0 - eps[k]);
    }
    for (int a = 0; a < QPO_ALPHA; ++a)
        for (int c = 0; c < QPO_ALPHA; ++c)
            md->l_emit[a * QPO_ALPHA + c] = log(joint[a * QPO_ALPHA + c]) - log(qx[a]) - log(qy[c]);
    return 0;
}

/* Partition-function tables: Boltzmann weights of the scores at temperature T. */
static int make_pf(qpo_model* md, const double* score, double g_open, double g_ext, double T) {
    if (!(T > 0.0)) return -2;
    md->G = 1;
    md->l_mm = 0.0;
    md->l_open[0] = g_open / T;
    md->l_ext[0] = g_ext / T;
    md->l_close[0] = 0.0;
    for (int a = 0; a < QPO_ALPHA * QPO_ALPHA; ++a) md->l_emit[a] = score[a] / T;
    return 0;
}

/* Maximum expected accuracy score over monotone matchings of the dense
 * posterior matrix (m x n, row-major). */
static double mea_score(const double* P, int m, int n) {
    double* A = (double*)calloc((size_t)(m + 1) * (n + 1), sizeof(double));
    if (!A) return NAN;
    const int W = n + 1;
    for (int i = 1; i <= m; ++i)
        for (int j = 1; j <= n; ++j) {
            double v = A[(size_t)(i - 1) * W + (j - 1)] + P[(size_t)(i - 1) * n + (j - 1)];
            double up = A[(size_t)(i - 1) * W + j];
            double left = A[(size_t)i * W + (j - 1)];
            if (up > v) v = up;
            if (left > v) v = left;
            A[(size_t)i * W + j] = v;
        }
    double r = A[(size_t)m * W + n];
    free(A);
    return r;
}

/*
 * Posteriors of one pair.
 *   x[m], y[n]      residue codes 0..19 (m, n >= 1)
 *   joint[400]      pair-HMM joint emission p_ab (row = residue of x)
 *   G, delta, eps   pair-HMM gap classes
 *   score[400]      PF scores s_ab; g_open, g_ext PF gap scores; T temperature
 *   w_hmm           weight of the HMM posterior in the combination
 * Outputs (caller-allocated, any may be NULL except post):
 *   post[m*n]       combined posterior, row-major over (i, j)
 *   post_h, post_p  per-model posteriors
 *   stats[6]        log Z_hmm (fwd), log Z_hmm (bwd), log Z_pf (fwd),
 *                   log Z_pf (bwd), MEA score A(m,n), EA = A(m,n)/min(m,n)
 * Returns 0, or a negative value on bad arguments / allocation failure.
 */
int qpo_pair(const uint8_t* x, int m, const uint8_t* y, int n,
             const double* joint, int G, const double* delta, const double* eps,
             const double* score, double g_open, double g_ext, double T, double w_hmm,
             double* post, double* post_h, double* post_p, double* stats) {
    if (m < 1 || n < 1 || !x || !y || !post) return -1;
    for (int i = 0; i < m; ++i) if (x[i] >= QPO_ALPHA) return -1;
    for (int j = 0; j < n; ++j) if (y[j] >= QPO_ALPHA) return -1;
    qpo_model hmm, pf;
    if (make_hmm(&hmm, joint, G, delta, eps)) return -2;
    if (make_pf(&pf, score, g_open, g_ext, T)) return -2;
    size_t mn = (size_t)m * n;
    double* ph = post_h ? post_h : (double*)malloc(sizeof(double) * mn);
    double* pp = post_p ? post_p : (double*)malloc(sizeof(double) * mn);
    int rc = 0;
    double s[6] = {0};
    if (!ph || !pp) { rc = -3; goto done; }
    if (run_model(&hmm, x, m, y, n, ph, &s[0], &s[1])) { rc = -3; goto done; }
    if (run_model(&pf, x, m, y, n, pp, &s[2], &s[3])) { rc = -3; goto done; }
    for (size_t c = 0; c < mn; ++c) post[c] = w_hmm * ph[c] + (1.0 - w_hmm) * pp[c];
    s[4] = mea_score(post, m, n);
    s[5] = s[4] / (double)(m < n ? m : n);
    if (stats) memcpy(stats, s, sizeof(s));
done:
    if (!post_h) free(ph);
    if (!post_p) free(pp);
    return rc;
}

/* Posterior of a single model given in generic transition form (used by the
 * tests to exercise the shared recurrence with arbitrary coefficients). */
int qpo_model_posterior(const uint8_t* x, int m, const uint8_t* y, int n, int G, double l_mm,
                        const double* l_open, const double* l_ext, const double* l_close,
                        const double* l_emit, double* post, double* lz) {
    if (m < 1 || n < 1 || G < 1 || G > QPO_MAXG) return -1;
    qpo_model md;
    md.G = G;
    md.l_mm = l_mm;
    for (int k = 0; k < G; ++k) {
        md.l_open[k] = l_open[k];
        md.l_ext[k] = l_ext[k];
        md.l_close[k] = l_close[k];
    }
    memcpy(md.l_emit, l_emit, sizeof(md.l_emit));
    return run_model(&md, x, m, y, n, post, &lz[0], &lz[1]);
}

/* MEA score of an arbitrary dense matrix (exposed for tests). */
double qpo_mea(const double* P, int m, int n) { return mea_score(P, m, n); }
