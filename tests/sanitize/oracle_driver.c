/*
 * Driver that exercises every entry point of the CPU oracle (test
 * infrastructure) so that it can be run under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  It checks two of the oracle's own identities on
 * small seeded inputs: the power-trace sum equals the matching definition
 * (brute force), and the listed subset terms add up to the power-trace sum.
 * Exit status 0 when every check passes.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_lhaf_dp_d(const double *A, int N, double *out);
int oracle_lhaf_pt_d(const double *A, int N, int nthreads, double *out, double *abs_sum);
int oracle_lhaf_dp_ld(const double *A, int N, long double *out);
int oracle_lhaf_pt_ld(const double *A, int N, int nthreads, long double *out, long double *abs_sum);
int oracle_term_d(const double *A, int N, unsigned long long mask, double *out);
int oracle_terms_d(const double *A, int N, const unsigned long long *masks, long long count, int nthreads,
                   double *out);
int oracle_charpoly_d(const double *M, int m, double *coef);
int oracle_power_traces_d(const double *M, int m, int K, double *p);
int oracle_max_threads(void);

static unsigned long long state = 0x9E3779B97F4A7C15ull;
static double rnd(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}

int main(void)
{
    int fails = 0;
    for (int N = 0; N <= 14; ++N) {
        double *A = calloc((size_t)(2 * N * N + 2), sizeof(double));
        for (int i = 0; i < N; ++i)
            for (int j = 0; j <= i; ++j) {
                const double re = rnd(), im = rnd();
                A[2 * (i * N + j)] = A[2 * (j * N + i)] = re;
                A[2 * (i * N + j) + 1] = A[2 * (j * N + i) + 1] = im;
            }
        double dp[2], pt[2], ab = 0.0;
        long double dpl[2], ptl[2], abl = 0.0L;
        if (oracle_lhaf_dp_d(A, N, dp) || oracle_lhaf_pt_d(A, N, 2, pt, &ab) || oracle_lhaf_dp_ld(A, N, dpl) ||
            oracle_lhaf_pt_ld(A, N, 1, ptl, &abl)) {
            printf("N=%d: oracle call failed\n", N);
            ++fails;
            free(A);
            continue;
        }
        const double err = hypot(dp[0] - pt[0], dp[1] - pt[1]);
        if (err > 1e-13 * (ab + 1.0)) {
            printf("N=%d: dp %g%+gi vs pt %g%+gi\n", N, dp[0], dp[1], pt[0], pt[1]);
            ++fails;
        }
        const long double errl = hypotl(dpl[0] - ptl[0], dpl[1] - ptl[1]);
        if (errl > 1e-16L * (abl + 1.0L)) {
            printf("N=%d: long double dp vs pt differ by %Lg\n", N, errl);
            ++fails;
        }
        const int n = (N + 1) / 2;
        if (N > 0) {
            const long long cnt = 1LL << n;
            unsigned long long *masks = malloc(sizeof(unsigned long long) * (size_t)cnt);
            double *t = malloc(sizeof(double) * 2 * (size_t)cnt);
            for (long long k = 0; k < cnt; ++k) masks[k] = (unsigned long long)k;
            double sr = 0.0, si = 0.0, one[2];
            if (oracle_terms_d(A, N, masks, cnt, 2, t) || oracle_term_d(A, N, masks[cnt - 1], one)) {
                printf("N=%d: terms failed\n", N);
                ++fails;
            } else {
                for (long long k = 0; k < cnt; ++k) {
                    sr += t[2 * k];
                    si += t[2 * k + 1];
                }
                if (hypot(sr - pt[0], si - pt[1]) > 1e-13 * (ab + 1.0) || one[0] != t[2 * (cnt - 1)]) {
                    printf("N=%d: terms do not add up\n", N);
                    ++fails;
                }
            }
            free(masks);
            free(t);
            double *coef = malloc(sizeof(double) * 2 * (size_t)(N + 1));
            double *p = malloc(sizeof(double) * 2 * (size_t)(N + 2));
            if (oracle_charpoly_d(A, N, coef) || oracle_power_traces_d(A, N, N + 2, p)) {
                printf("N=%d: charpoly failed\n", N);
                ++fails;
            } else if (fabs(coef[2 * N] - 1.0) > 1e-14 || coef[2 * N + 1] != 0.0) {
                printf("N=%d: characteristic polynomial not monic\n", N);
                ++fails;
            }
            free(coef);
            free(p);
        }
        free(A);
    }
    printf("%d failures, %d threads\n", fails, oracle_max_threads());
    return fails ? 1 : 0;
}
