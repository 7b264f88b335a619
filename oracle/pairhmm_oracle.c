/*
 * Pair-HMM forward/backward oracle: plain FP64 C, full DP matrices.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP kernels are
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never calls it.  It shares
 * no code, header, table or constant with the HIP library.
 *
 * What it computes (arXiv 2411.11547, Section II-A):
 *   M(i,j) = lam_ij * (alpha_i M(i-1,j-1) + beta_i (I(i-1,j-1) + D(i-1,j-1)))   Eq. (1)
 *   I(i,j) = delta_i M(i-1,j) + eps_i I(i-1,j)                                  Eq. (2)
 *   D(i,j) = zeta_i M(i,j-1)  + eps_i D(i,j-1)                                  Eq. (3)
 *   lam_ij = 1 - Q_i if r_i = h_j, else Q_i / 3                                 Eq. (4)
 *   M(i,0) = I(i,0) = D(i,0) = 0, M(0,j) = I(0,j) = 0, D(0,j) = 1/n             (init.)
 *   L = sum_{j=1..n} (M(m,j) + I(m,j))                                           (result)
 *
 * Readings of points the paper leaves open (each is a named convention):
 *   - Phred decoding: Q_i = 10^(-q/10); delta = 10^(-ins/10), zeta =
 *     10^(-del/10), eps = 10^(-gcp/10) (one gap-continuation value for I->I
 *     and D->D, as Eq. (2)-(3) share eps_i), alpha = 1 - delta - zeta,
 *     beta = 1 - eps (each state's out-transitions sum to one).
 *   - N (code 4) on either side counts as a match (wildcard), unless the
 *     caller asks for the literal reading (r_i == h_j only).
 *   - D(0,0) = 1/n like every other D(0,j); the zero rule covers i >= 1.
 *   - Transitions at cell (i,j) use the destination row's index i.
 *
 * Range: after row i is complete it may be divided by a power of two 2^s_i
 * (s_i from frexp of the row maximum) with s_i added to a running exponent.
 * Power-of-two scaling is exact, so results equal the unscaled recurrence
 * bit for bit wherever the unscaled one stays in range; it only keeps long,
 * low-quality pairs out of the subnormal range.
 *
 * Gradients: g_theta_i = d log10 L / d log10 theta_i for the seven per-position
 * parameters {alpha, beta, delta, eps, zeta, lam_match, lam_mismatch}; each is
 * the posterior expected number of uses of theta_i, i.e. a sum over the cells
 * of row i of forward value x transition x backward value, divided by L.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NCH 7 /* alpha, beta, delta, eps, zeta, lam_match, lam_mismatch */
enum { P_ALPHA, P_BETA, P_DELTA, P_EPS, P_ZETA, P_LMATCH, P_LMIS };
/* extended gradient channels: eps split into its I->I and D->D uses */
#define NEXT 8
enum { X_ALPHA, X_BETA, X_DELTA, X_EPS_I, X_EPS_D, X_ZETA, X_LMATCH, X_LMIS };

static double phred_to_prob(int q) { return pow(10.0, -(double)q / 10.0); }

/* Per read position i: the seven probabilities from Phred bytes. */
void oracle_params_from_phred(int m, const uint8_t *bq, const uint8_t *iq,
                              const uint8_t *dq, const uint8_t *gq, double *par)
{
    for (int i = 0; i < m; i++) {
        double Q = phred_to_prob(bq[i]);
        double delta = phred_to_prob(iq[i]);
        double zeta = phred_to_prob(dq[i]);
        double eps = phred_to_prob(gq[i]);
        double *p = par + (size_t)i * NCH;
        p[P_ALPHA] = 1.0 - delta - zeta;
        p[P_BETA] = 1.0 - eps;
        p[P_DELTA] = delta;
        p[P_EPS] = eps;
        p[P_ZETA] = zeta;
        p[P_LMATCH] = 1.0 - Q;
        p[P_LMIS] = Q / 3.0;
    }
}

/* Explicit-parameter mode: theta = 10^(log10 theta) for all seven. */
void oracle_params_from_log10(int m, const float *lg, double *par)
{
    for (size_t i = 0; i < (size_t)m * NCH; i++) par[i] = pow(10.0, (double)lg[i]);
}

static int is_match(uint8_t r, uint8_t h, int literal_n)
{
    if (literal_n) return r == h;
    return r == h || r == 4 || h == 4;
}

/* Full forward matrices.  Row i of X lives at X[i*(n+1) + j].  e[i] is the
 * cumulative power-of-two exponent of row i: true value = stored * 2^e[i].
 * Returns the stored row-m sum; *L_exp receives e[m]. */
static double forward_matrices(int m, int n, const uint8_t *r, const uint8_t *h,
                               const double *par, int rescale, int literal_n,
                               double *M, double *I, double *D, int *e)
{
    const size_t W = (size_t)n + 1;
    for (int j = 0; j <= n; j++) {
        M[j] = 0.0;
        I[j] = 0.0;
        D[j] = 1.0 / n;
    }
    e[0] = 0;
    for (int i = 1; i <= m; i++) {
        const double *p = par + (size_t)(i - 1) * NCH;
        double *Mi = M + i * W, *Ii = I + i * W, *Di = D + i * W;
        const double *Mu = M + (i - 1) * W, *Iu = I + (i - 1) * W, *Du = D + (i - 1) * W;
        Mi[0] = Ii[0] = Di[0] = 0.0;
        for (int j = 1; j <= n; j++) {
            double lam = is_match(r[i - 1], h[j - 1], literal_n) ? p[P_LMATCH] : p[P_LMIS];
            Mi[j] = lam * (p[P_ALPHA] * Mu[j - 1] + p[P_BETA] * (Iu[j - 1] + Du[j - 1]));
            Ii[j] = p[P_DELTA] * Mu[j] + p[P_EPS] * Iu[j];
            Di[j] = p[P_ZETA] * Mi[j - 1] + p[P_EPS] * Di[j - 1];
        }
        e[i] = e[i - 1];
        if (rescale) {
            double mx = 0.0;
            for (int j = 0; j <= n; j++) {
                if (Mi[j] > mx) mx = Mi[j];
                if (Ii[j] > mx) mx = Ii[j];
                if (Di[j] > mx) mx = Di[j];
            }
            if (mx > 0.0 && isfinite(mx)) {
                int s;
                frexp(mx, &s);
                for (int j = 0; j <= n; j++) {
                    Mi[j] = ldexp(Mi[j], -s);
                    Ii[j] = ldexp(Ii[j], -s);
                    Di[j] = ldexp(Di[j], -s);
                }
                e[i] += s;
            }
        }
    }
    double sum = 0.0;
    const double *Mm = M + (size_t)m * W, *Im = I + (size_t)m * W;
    for (int j = 1; j <= n; j++) sum += Mm[j] + Im[j];
    return sum;
}

static double to_log10(double sum, int exp2)
{
    return log10(sum) + (double)exp2 * log10(2.0);
}

/* log10 L of one pair; -inf if L == 0.  Returns NaN for m < 1 or n < 1. */
double oracle_forward(int m, int n, const uint8_t *r, const uint8_t *h, const double *par,
                      int rescale, int literal_n)
{
    if (m < 1 || n < 1) return NAN;
    size_t cells = (size_t)(m + 1) * (n + 1);
    double *buf = malloc(3 * cells * sizeof(double));
    int *e = malloc((size_t)(m + 1) * sizeof(int));
    if (!buf || !e) { free(buf); free(e); return NAN; }
    double s = forward_matrices(m, n, r, h, par, rescale, literal_n, buf, buf + cells,
                                buf + 2 * cells, e);
    double out = to_log10(s, e[m]);
    free(buf);
    free(e);
    return out;
}

/* Forward matrices exported for tests (no rescaling): M, I, D each (m+1)x(n+1). */
int oracle_forward_full(int m, int n, const uint8_t *r, const uint8_t *h, const double *par,
                        int literal_n, double *M, double *I, double *D)
{
    if (m < 1 || n < 1) return -1;
    int *e = malloc((size_t)(m + 1) * sizeof(int));
    if (!e) return -1;
    forward_matrices(m, n, r, h, par, 0, literal_n, M, I, D, e);
    free(e);
    return 0;
}

/*
 * Viterbi (max-product) form of the same model: every sum over predecessor
 * states in Eq. (1)-(3) becomes a maximum and the result formula takes the
 * largest M(m,j) or I(m,j) instead of their sum, which gives the probability
 * of the single most probable alignment path:
 *   V_M(i,j) = lam_ij * max(alpha_i V_M(i-1,j-1), beta_i V_I(i-1,j-1), beta_i V_D(i-1,j-1))
 *   V_I(i,j) = max(delta_i V_M(i-1,j), eps_i V_I(i-1,j))
 *   V_D(i,j) = max(zeta_i V_M(i,j-1), eps_i V_D(i,j-1))
 * with the forward initialisation.  Rows are rescaled by powers of two as in
 * the forward (exact, since max commutes with a positive scale).
 */
static double viterbi_matrices(int m, int n, const uint8_t *r, const uint8_t *h, const double *par,
                               int rescale, int literal_n, double *M, double *I, double *D, int *e)
{
    const size_t W = (size_t)n + 1;
    for (int j = 0; j <= n; j++) {
        M[j] = 0.0;
        I[j] = 0.0;
        D[j] = 1.0 / n;
    }
    e[0] = 0;
    for (int i = 1; i <= m; i++) {
        const double *p = par + (size_t)(i - 1) * NCH;
        double *Mi = M + i * W, *Ii = I + i * W, *Di = D + i * W;
        const double *Mu = M + (i - 1) * W, *Iu = I + (i - 1) * W, *Du = D + (i - 1) * W;
        Mi[0] = Ii[0] = Di[0] = 0.0;
        for (int j = 1; j <= n; j++) {
            double lam = is_match(r[i - 1], h[j - 1], literal_n) ? p[P_LMATCH] : p[P_LMIS];
            double best = fmax(p[P_ALPHA] * Mu[j - 1], fmax(p[P_BETA] * Iu[j - 1], p[P_BETA] * Du[j - 1]));
            Mi[j] = lam * best;
            Ii[j] = fmax(p[P_DELTA] * Mu[j], p[P_EPS] * Iu[j]);
            Di[j] = fmax(p[P_ZETA] * Mi[j - 1], p[P_EPS] * Di[j - 1]);
        }
        e[i] = e[i - 1];
        if (rescale) {
            double mx = 0.0;
            for (int j = 0; j <= n; j++) {
                if (Mi[j] > mx) mx = Mi[j];
                if (Ii[j] > mx) mx = Ii[j];
                if (Di[j] > mx) mx = Di[j];
            }
            if (mx > 0.0 && isfinite(mx)) {
                int s;
                frexp(mx, &s);
                for (int j = 0; j <= n; j++) {
                    Mi[j] = ldexp(Mi[j], -s);
                    Ii[j] = ldexp(Ii[j], -s);
                    Di[j] = ldexp(Di[j], -s);
                }
                e[i] += s;
            }
        }
    }
    double best = 0.0;
    const double *Mm = M + (size_t)m * W, *Im = I + (size_t)m * W;
    for (int j = 1; j <= n; j++) best = fmax(best, fmax(Mm[j], Im[j]));
    return best;
}

/* log10 of the best path's probability; -inf if no path has weight. */
double oracle_viterbi(int m, int n, const uint8_t *r, const uint8_t *h, const double *par, int rescale,
                      int literal_n)
{
    if (m < 1 || n < 1) return NAN;
    size_t cells = (size_t)(m + 1) * (n + 1);
    double *buf = malloc(3 * cells * sizeof(double));
    int *e = malloc((size_t)(m + 1) * sizeof(int));
    if (!buf || !e) { free(buf); free(e); return NAN; }
    double s = viterbi_matrices(m, n, r, h, par, rescale, literal_n, buf, buf + cells, buf + 2 * cells, e);
    double out = to_log10(s, e[m]);
    free(buf);
    free(e);
    return out;
}

/*
 * Backward (adjoint) pass and gradients of one pair.
 *
 * B_X(i,j) = dL/dX(i,j).  L takes M(m,j) and I(m,j) with weight one, so
 * B_M(m,j) = B_I(m,j) = 1 and B_D(m,j) = 0.  Each forward term in Eq. (1)-(3)
 * sends its coefficient back to its source cell:
 *   B_M(i,j) = alpha_{i+1} X + delta_{i+1} B_I(i+1,j) + zeta_i B_D(i,j+1)
 *   B_I(i,j) = beta_{i+1}  X + eps_{i+1}  B_I(i+1,j)
 *   B_D(i,j) = beta_{i+1}  X + eps_i      B_D(i,j+1)
 * with X = lam_{i+1,j+1} B_M(i+1,j+1), and anything with j > n or i > m zero.
 * The initial D(0,j) = 1/n feed M(1,j+1) with weight beta_1 lam_{1,j+1}, so
 * the backward total sum_{j=0..n-1} (1/n) beta_1 lam_{1,j+1} B_M(1,j+1) is L.
 *
 * grad_ext[(i-1)*8 + c] receives the eight extended channels of row i;
 * log10_total_fwd / log10_total_bwd receive log10 L both ways.
 * Rows are rescaled by powers of two in both passes.
 */
int oracle_backward(int m, int n, const uint8_t *r, const uint8_t *h, const double *par,
                    int literal_n, double *grad_ext, double *log10_total_fwd,
                    double *log10_total_bwd)
{
    if (m < 1 || n < 1) return -1;
    const size_t W = (size_t)n + 2; /* backward rows carry a j = n+1 zero column */
    const size_t FW = (size_t)n + 1;
    size_t fcells = (size_t)(m + 1) * FW, bcells = (size_t)(m + 2) * W;
    double *F = malloc(3 * fcells * sizeof(double));
    double *B = malloc(3 * bcells * sizeof(double));
    int *eF = malloc((size_t)(m + 1) * sizeof(int));
    int *eB = malloc((size_t)(m + 2) * sizeof(int));
    if (!F || !B || !eF || !eB) { free(F); free(B); free(eF); free(eB); return -1; }
    double *M = F, *I = F + fcells, *D = F + 2 * fcells;
    double *BM = B, *BI = B + bcells, *BD = B + 2 * bcells;

    double Ls = forward_matrices(m, n, r, h, par, 1, literal_n, M, I, D, eF);
    int Le = eF[m];
    *log10_total_fwd = to_log10(Ls, Le);

    /* row m+1 (outside the matrix) is all zero */
    for (size_t j = 0; j < W; j++) BM[(m + 1) * W + j] = BI[(m + 1) * W + j] = BD[(m + 1) * W + j] = 0.0;
    eB[m + 1] = 0;
    for (int i = m; i >= 1; i--) {
        double *bm = BM + i * W, *bi = BI + i * W, *bd = BD + i * W;
        const double *bmd = BM + (i + 1) * W, *bid = BI + (i + 1) * W;
        const double *p = par + (size_t)(i - 1) * NCH;
        bm[n + 1] = bi[n + 1] = bd[n + 1] = 0.0;
        bm[0] = bi[0] = bd[0] = 0.0; /* column 0 holds constants, not variables */
        if (i == m) {
            for (int j = n; j >= 1; j--) {
                bd[j] = 0.0;
                bm[j] = 1.0 + p[P_ZETA] * bd[j + 1];
                bi[j] = 1.0;
            }
            eB[i] = 0;
        } else {
            const double *pn = par + (size_t)i * NCH; /* row i+1 */
            for (int j = n; j >= 1; j--) {
                double X = 0.0;
                if (j + 1 <= n) {
                    double lam = is_match(r[i], h[j], literal_n) ? pn[P_LMATCH] : pn[P_LMIS];
                    X = lam * bmd[j + 1];
                }
                bm[j] = pn[P_ALPHA] * X + pn[P_DELTA] * bid[j] + p[P_ZETA] * bd[j + 1];
                bi[j] = pn[P_BETA] * X + pn[P_EPS] * bid[j];
                bd[j] = pn[P_BETA] * X + p[P_EPS] * bd[j + 1];
            }
            eB[i] = eB[i + 1];
            double mx = 0.0;
            for (int j = 1; j <= n; j++) {
                if (bm[j] > mx) mx = bm[j];
                if (bi[j] > mx) mx = bi[j];
                if (bd[j] > mx) mx = bd[j];
            }
            if (mx > 0.0 && isfinite(mx)) {
                int s;
                frexp(mx, &s);
                for (int j = 1; j <= n; j++) {
                    bm[j] = ldexp(bm[j], -s);
                    bi[j] = ldexp(bi[j], -s);
                    bd[j] = ldexp(bd[j], -s);
                }
                eB[i] += s;
            }
        }
    }

    /* backward total from the initial D(0, j) = 1/n (stored row 0 of D) */
    {
        const double *p1 = par;
        double t = 0.0;
        for (int j = 0; j <= n - 1; j++) {
            double lam = is_match(r[0], h[j], literal_n) ? p1[P_LMATCH] : p1[P_LMIS];
            t += D[j] * p1[P_BETA] * lam * BM[1 * W + j + 1];
        }
        *log10_total_bwd = to_log10(t, eF[0] + eB[1]);
    }

    /* gradients: for every row i, sums over j of forward x coefficient x backward / L */
    for (int i = 1; i <= m; i++) {
        const double *p = par + (size_t)(i - 1) * NCH;
        const double *Mu = M + (i - 1) * FW, *Iu = I + (i - 1) * FW, *Du = D + (i - 1) * FW;
        const double *Mi = M + i * FW, *Di = D + i * FW;
        const double *bm = BM + i * W, *bi = BI + i * W, *bd = BD + i * W;
        double sa = 0, sb = 0, sd = 0, sei = 0, sed = 0, sz = 0, slm = 0, slx = 0;
        for (int j = 1; j <= n; j++) {
            int match = is_match(r[i - 1], h[j - 1], literal_n);
            double lam = match ? p[P_LMATCH] : p[P_LMIS];
            sa += p[P_ALPHA] * lam * Mu[j - 1] * bm[j];
            sb += p[P_BETA] * lam * (Iu[j - 1] + Du[j - 1]) * bm[j];
            if (match) slm += Mi[j] * bm[j]; else slx += Mi[j] * bm[j];
            sd += p[P_DELTA] * Mu[j] * bi[j];
            sei += p[P_EPS] * Iu[j] * bi[j];
            sed += p[P_EPS] * Di[j - 1] * bd[j];
            sz += p[P_ZETA] * Mi[j - 1] * bd[j];
        }
        /* scale: row i-1 terms carry 2^(eF[i-1]+eB[i]), row i terms 2^(eF[i]+eB[i]); L = Ls 2^Le */
        int up = eF[i - 1] + eB[i] - Le, cur = eF[i] + eB[i] - Le;
        double *g = grad_ext + (size_t)(i - 1) * NEXT;
        g[X_ALPHA] = ldexp(sa / Ls, up);
        g[X_BETA] = ldexp(sb / Ls, up);
        g[X_DELTA] = ldexp(sd / Ls, up);
        g[X_EPS_I] = ldexp(sei / Ls, up);
        g[X_EPS_D] = ldexp(sed / Ls, cur);
        g[X_ZETA] = ldexp(sz / Ls, cur);
        g[X_LMATCH] = ldexp(slm / Ls, cur);
        g[X_LMIS] = ldexp(slx / Ls, cur);
    }
    free(F);
    free(B);
    free(eF);
    free(eB);
    return 0;
}

/* ------------------------------------------------------------------------
 * Batch loop: every pair of every batch, in output order (batch-major,
 * then read, then haplotype), spread over a pool of threads.  Parameters
 * come from Phred bytes, or from explicit log10 parameters [sum m x 7] when
 * log10_par is non-NULL.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t num_pairs;
    const int32_t *pair_read, *pair_hap;
    const int64_t *read_offset, *hap_offset;
    const uint8_t *read_bases, *bq, *iq, *dq, *gq, *hap_bases;
    const float *log10_par;
    int literal_n;
    int viterbi;       /* 1: max-product score instead of the forward likelihood */
    double *out;       /* forward: log10 L per pair */
    double *grad_ext;  /* backward: [sum over pairs of m x 8] or NULL */
    const int64_t *grad_offset; /* per pair, row offset into grad_ext */
    volatile int64_t next;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *jb = arg;
    for (;;) {
        int64_t k = __sync_fetch_and_add(&jb->next, 1);
        if (k >= jb->num_pairs) break;
        int32_t rr = jb->pair_read[k], hh = jb->pair_hap[k];
        int64_t ro = jb->read_offset[rr], ho = jb->hap_offset[hh];
        int m = (int)(jb->read_offset[rr + 1] - ro), n = (int)(jb->hap_offset[hh + 1] - ho);
        double *par = malloc((size_t)(m > 0 ? m : 1) * NCH * sizeof(double));
        if (!par) { jb->out[k] = NAN; continue; }
        if (jb->log10_par)
            oracle_params_from_log10(m, jb->log10_par + ro * NCH, par);
        else
            oracle_params_from_phred(m, jb->bq + ro, jb->iq + ro, jb->dq + ro, jb->gq + ro, par);
        if (jb->grad_ext) {
            double lf, lb;
            if (oracle_backward(m, n, jb->read_bases + ro, jb->hap_bases + ho, par, jb->literal_n,
                                jb->grad_ext + jb->grad_offset[k] * NEXT, &lf, &lb) != 0)
                lf = NAN;
            jb->out[k] = lf;
        } else if (jb->viterbi) {
            jb->out[k] = oracle_viterbi(m, n, jb->read_bases + ro, jb->hap_bases + ho, par, 1,
                                        jb->literal_n);
        } else {
            jb->out[k] = oracle_forward(m, n, jb->read_bases + ro, jb->hap_bases + ho, par, 1,
                                        jb->literal_n);
        }
        free(par);
    }
    return NULL;
}

static int run_pool(batch_job *jb, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    int started = 0;
    jb->next = 0;
    for (int t = 0; t < threads; t++) {
        if (pthread_create(&tid[t], NULL, batch_worker, jb) != 0) break;
        started++;
    }
    if (started == 0) batch_worker(jb);
    for (int t = 0; t < started; t++) pthread_join(tid[t], NULL);
    return started ? started : 1;
}

/* Forward over an explicit pair list; returns the number of threads used. */
int oracle_forward_pairs(int64_t num_pairs, const int32_t *pair_read, const int32_t *pair_hap,
                         const int64_t *read_offset, const uint8_t *read_bases,
                         const uint8_t *bq, const uint8_t *iq, const uint8_t *dq,
                         const uint8_t *gq, const int64_t *hap_offset,
                         const uint8_t *hap_bases, const float *log10_par, int literal_n,
                         int threads, double *out_log10)
{
    batch_job jb = {0};
    jb.num_pairs = num_pairs;
    jb.pair_read = pair_read;
    jb.pair_hap = pair_hap;
    jb.read_offset = read_offset;
    jb.hap_offset = hap_offset;
    jb.read_bases = read_bases;
    jb.bq = bq; jb.iq = iq; jb.dq = dq; jb.gq = gq;
    jb.hap_bases = hap_bases;
    jb.log10_par = log10_par;
    jb.literal_n = literal_n;
    jb.out = out_log10;
    return run_pool(&jb, threads);
}

/* Viterbi scores over an explicit pair list; returns the number of threads used. */
int oracle_viterbi_pairs(int64_t num_pairs, const int32_t *pair_read, const int32_t *pair_hap,
                         const int64_t *read_offset, const uint8_t *read_bases,
                         const uint8_t *bq, const uint8_t *iq, const uint8_t *dq,
                         const uint8_t *gq, const int64_t *hap_offset,
                         const uint8_t *hap_bases, const float *log10_par, int literal_n,
                         int threads, double *out_log10)
{
    batch_job jb = {0};
    jb.num_pairs = num_pairs;
    jb.pair_read = pair_read;
    jb.pair_hap = pair_hap;
    jb.read_offset = read_offset;
    jb.hap_offset = hap_offset;
    jb.read_bases = read_bases;
    jb.bq = bq; jb.iq = iq; jb.dq = dq; jb.gq = gq;
    jb.hap_bases = hap_bases;
    jb.log10_par = log10_par;
    jb.literal_n = literal_n;
    jb.viterbi = 1;
    jb.out = out_log10;
    return run_pool(&jb, threads);
}

/* Backward over an explicit pair list: grad_ext rows at grad_offset[k]. */
int oracle_backward_pairs(int64_t num_pairs, const int32_t *pair_read, const int32_t *pair_hap,
                          const int64_t *read_offset, const uint8_t *read_bases,
                          const uint8_t *bq, const uint8_t *iq, const uint8_t *dq,
                          const uint8_t *gq, const int64_t *hap_offset,
                          const uint8_t *hap_bases, const float *log10_par, int literal_n,
                          int threads, const int64_t *grad_offset, double *grad_ext,
                          double *out_log10)
{
    batch_job jb = {0};
    jb.num_pairs = num_pairs;
    jb.pair_read = pair_read;
    jb.pair_hap = pair_hap;
    jb.read_offset = read_offset;
    jb.hap_offset = hap_offset;
    jb.read_bases = read_bases;
    jb.bq = bq; jb.iq = iq; jb.dq = dq; jb.gq = gq;
    jb.hap_bases = hap_bases;
    jb.log10_par = log10_par;
    jb.literal_n = literal_n;
    jb.out = out_log10;
    jb.grad_ext = grad_ext;
    jb.grad_offset = grad_offset;
    return run_pool(&jb, threads);
}
