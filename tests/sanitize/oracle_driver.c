/* The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer:
 * single pairs (forward, Viterbi, backward, the full matrices) and the
 * threaded batch loops over random pairs of 1..40 x 1..60 bases, including
 * N codes and explicit log10 parameters.  Exits 0 when the forward and
 * backward totals agree and the batch loops equal the single-pair calls. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double oracle_forward(int m, int n, const uint8_t *r, const uint8_t *h, const double *par, int rescale,
                      int literal_n);
int oracle_forward_full(int m, int n, const uint8_t *r, const uint8_t *h, const double *par, int literal_n,
                        double *M, double *I, double *D);
double oracle_viterbi(int m, int n, const uint8_t *r, const uint8_t *h, const double *par, int rescale,
                      int literal_n);
int oracle_backward(int m, int n, const uint8_t *r, const uint8_t *h, const double *par, int literal_n,
                    double *grad_ext, double *log10_total_fwd, double *log10_total_bwd);
void oracle_params_from_phred(int m, const uint8_t *bq, const uint8_t *iq, const uint8_t *dq,
                              const uint8_t *gq, double *par);
int oracle_forward_pairs(int64_t num_pairs, const int32_t *pair_read, const int32_t *pair_hap,
                         const int64_t *read_offset, const uint8_t *read_bases, const uint8_t *bq,
                         const uint8_t *iq, const uint8_t *dq, const uint8_t *gq, const int64_t *hap_offset,
                         const uint8_t *hap_bases, const float *log10_par, int literal_n, int threads,
                         double *out_log10);
int oracle_viterbi_pairs(int64_t num_pairs, const int32_t *pair_read, const int32_t *pair_hap,
                         const int64_t *read_offset, const uint8_t *read_bases, const uint8_t *bq,
                         const uint8_t *iq, const uint8_t *dq, const uint8_t *gq, const int64_t *hap_offset,
                         const uint8_t *hap_bases, const float *log10_par, int literal_n, int threads,
                         double *out_log10);
int oracle_backward_pairs(int64_t num_pairs, const int32_t *pair_read, const int32_t *pair_hap,
                          const int64_t *read_offset, const uint8_t *read_bases, const uint8_t *bq,
                          const uint8_t *iq, const uint8_t *dq, const uint8_t *gq, const int64_t *hap_offset,
                          const uint8_t *hap_bases, const float *log10_par, int literal_n, int threads,
                          const int64_t *grad_offset, double *grad_ext, double *out_log10);

static uint64_t state = 12345;
static uint32_t rnd(uint32_t k)
{
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (uint32_t)(state >> 33) % k;
}

enum { NR = 12, NH = 9 };

int main(void)
{
    int64_t ro[NR + 1], ho[NH + 1];
    ro[0] = ho[0] = 0;
    for (int r = 0; r < NR; ++r) ro[r + 1] = ro[r] + 1 + rnd(40);
    for (int h = 0; h < NH; ++h) ho[h + 1] = ho[h] + 1 + rnd(60);
    uint8_t *rbases = malloc(ro[NR]), *bq = malloc(ro[NR]), *iq = malloc(ro[NR]), *dq = malloc(ro[NR]),
            *gq = malloc(ro[NR]), *hbases = malloc(ho[NH]);
    float *lg = malloc(sizeof(float) * ro[NR] * 7);
    for (int64_t i = 0; i < ro[NR]; ++i) {
        rbases[i] = (uint8_t)rnd(5);
        bq[i] = (uint8_t)(5 + rnd(36));
        iq[i] = (uint8_t)(20 + rnd(26));
        dq[i] = (uint8_t)(20 + rnd(26));
        gq[i] = (uint8_t)rnd(20);
    }
    for (int64_t j = 0; j < ho[NH]; ++j) hbases[j] = (uint8_t)rnd(5);
    double *par = malloc(sizeof(double) * ro[NR] * 7);
    oracle_params_from_phred((int)ro[NR], bq, iq, dq, gq, par);
    for (int64_t i = 0; i < ro[NR] * 7; ++i) lg[i] = (float)log10(par[i]);

    const int64_t P = (int64_t)NR * NH;
    int32_t pr[NR * NH], ph[NR * NH];
    int64_t goff[NR * NH + 1];
    goff[0] = 0;
    for (int64_t k = 0; k < P; ++k) {
        pr[k] = (int32_t)(k / NH);
        ph[k] = (int32_t)(k % NH);
        goff[k + 1] = goff[k] + (ro[pr[k] + 1] - ro[pr[k]]);
    }
    double *fw = malloc(sizeof(double) * P), *vt = malloc(sizeof(double) * P), *bw = malloc(sizeof(double) * P),
           *fwl = malloc(sizeof(double) * P);
    double *g = malloc(sizeof(double) * goff[P] * 8);
    int bad = 0;
    oracle_forward_pairs(P, pr, ph, ro, rbases, bq, iq, dq, gq, ho, hbases, NULL, 0, 4, fw);
    oracle_forward_pairs(P, pr, ph, ro, rbases, bq, iq, dq, gq, ho, hbases, lg, 1, 3, fwl);
    oracle_viterbi_pairs(P, pr, ph, ro, rbases, bq, iq, dq, gq, ho, hbases, NULL, 0, 2, vt);
    oracle_backward_pairs(P, pr, ph, ro, rbases, bq, iq, dq, gq, ho, hbases, NULL, 0, 4, goff, g, bw);
    for (int64_t k = 0; k < P; ++k) {
        const int r = pr[k], h = ph[k];
        const int m = (int)(ro[r + 1] - ro[r]), n = (int)(ho[h + 1] - ho[h]);
        const uint8_t *rr = rbases + ro[r], *hh = hbases + ho[h];
        const double *pp = par + ro[r] * 7;
        const double f = oracle_forward(m, n, rr, hh, pp, 1, 0);
        const double v = oracle_viterbi(m, n, rr, hh, pp, 1, 0);
        double ge[8 * 64], lf = 0, lb = 0;
        double *gx = m <= 64 ? ge : malloc(sizeof(double) * m * 8);
        oracle_backward(m, n, rr, hh, pp, 0, gx, &lf, &lb);
        if (m > 64) free(gx);
        if (m * n <= 4000) {
            double *M = malloc(sizeof(double) * 3 * (m + 1) * (n + 1));
            oracle_forward_full(m, n, rr, hh, pp, 0, M, M + (m + 1) * (n + 1), M + 2 * (m + 1) * (n + 1));
            free(M);
        }
        if (fabs(f - fw[k]) > 1e-12 || fabs(v - vt[k]) > 1e-12 || fabs(lf - lb) > 1e-9 * (1 + fabs(lf)) ||
            fabs(bw[k] - f) > 1e-9 * (1 + fabs(f)) || v > f + 1e-12 || !isfinite(fwl[k])) {
            fprintf(stderr, "pair %lld: forward %g/%g viterbi %g/%g backward totals %g %g\n", (long long)k, f,
                    fw[k], v, vt[k], lf, lb);
            ++bad;
        }
    }
    printf("oracle checks: %lld pairs, %d mismatches\n", (long long)P, bad);
    free(rbases); free(bq); free(iq); free(dq); free(gq); free(hbases); free(lg); free(par);
    free(fw); free(vt); free(bw); free(fwl); free(g);
    return bad ? 1 : 0;
}
