/* Drives the CPU oracle through every exported routine on small seeded point
 * sets, for a build with AddressSanitizer and UndefinedBehaviorSanitizer: any
 * out-of-bounds access, use after free, leak or undefined operation aborts the
 * run.  It also checks the tree-walk product against the dense K~ it defines
 * (Section 2.1: K~ W by the up pass, the far coupling, the down pass and the
 * near field), so that a run that is clean but wrong fails too.
 * Test infrastructure: built and run by tests/test_sanitizers.py only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_h2 orc_h2;
orc_h2 *orc_build_ex(const double *X, int64_t N, int d, int kernel, double h, int m, double tol,
                     int rmax, int adm, double tau, int64_t S, uint64_t seed, int part, double budget);
orc_h2 *orc_points(const double *X, int64_t N, int d, int kernel, double h);
void orc_free(orc_h2 *H);
void orc_sizes(const orc_h2 *H, int64_t *out);
int orc_eval(const orc_h2 *H, const double *W, int64_t Q, double *Y, double *what_dump,
             double *yhat_dump, double *ynear_dump, double *yfar_dump);
int orc_dense_ktilde(const orc_h2 *H, double *Kt);
void orc_exact_rows(const orc_h2 *H, const int64_t *rows, int64_t nrows, const double *W, int64_t Q,
                    double *out);
int64_t orc_row_sample_public(const orc_h2 *H, int a, int64_t *out, int64_t cap);
int orc_pqr_id_public(double *A, int64_t mr, int nc, double tol, int rmax, int *k, int *piv,
                      double *Tcoef, double *rdiag);
int orc_split_centers(const orc_h2 *H, int a, double *out);
int orc_write(const orc_h2 *H, const char *path);
void orc_set_threads(int n);

static uint64_t st = 0x9e3779b97f4a7c15ull;
static double urand(void) /* xorshift64*, uniform in [0, 1) */
{
    st ^= st >> 12; st ^= st << 25; st ^= st >> 27;
    return (double)((st * 0x2545f4914f6cdd1dull) >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { fprintf(stderr, __VA_ARGS__); fputc('\n', stderr); fails++; } } while (0)

static void one(const char *name, int64_t N, int d, int kernel, double h, int m, double tol, int rmax,
                int adm, double tau, int64_t S, int part, double budget, int64_t Q, double bar,
                const char *path)
{
    double *X = malloc(sizeof(double) * (size_t)(N * d));
    for (int64_t i = 0; i < N * d; i++) X[i] = urand() * (i % d == 0 ? 4.0 : 1.0);
    orc_h2 *H = orc_build_ex(X, N, d, kernel, h, m, tol, rmax, adm, tau, S, 11, part, budget);
    CHECK(H != NULL, "%s: build failed", name);
    if (!H) { free(X); return; }
    int64_t sz[10];
    orc_sizes(H, sz);
    const int n = (int)sz[3];
    double *W = malloc(sizeof(double) * (size_t)(N * Q)), *Y = malloc(sizeof(double) * (size_t)(N * Q));
    for (int64_t i = 0; i < N * Q; i++) W[i] = urand() - 0.5;
    CHECK(orc_eval(H, W, Q, Y, NULL, NULL, NULL, NULL) == 0, "%s: eval failed", name);
    double *Kt = malloc(sizeof(double) * (size_t)(N * N));
    CHECK(orc_dense_ktilde(H, Kt) == 0, "%s: dense K~ failed", name);
    double num = 0, den = 0;
    for (int64_t i = 0; i < N; i++)
        for (int64_t q = 0; q < Q; q++) {
            double s = 0;
            for (int64_t j = 0; j < N; j++) s += Kt[i * N + j] * W[j * Q + q];
            num += (s - Y[i * Q + q]) * (s - Y[i * Q + q]);
            den += s * s;
        }
    CHECK(sqrt(num / den) < 1e-12, "%s: tree walk vs dense K~: %g", name, sqrt(num / den));
    int64_t rows[7] = {0, 1, N / 3, N / 2, N - 2, N - 1, 5};
    double *ex = malloc(sizeof(double) * 7 * (size_t)Q);
    orc_exact_rows(H, rows, 7, W, Q, ex);
    num = den = 0;
    for (int r = 0; r < 7; r++)
        for (int64_t q = 0; q < Q; q++) {
            double e = ex[r * Q + q] - Y[rows[r] * Q + q];
            num += e * e;
            den += ex[r * Q + q] * ex[r * Q + q];
        }
    CHECK(sqrt(num / den) < bar, "%s: sampled-row error %g", name, sqrt(num / den));
    int64_t *rs = malloc(sizeof(int64_t) * (size_t)N);
    for (int a = 0; a < n; a++) CHECK(orc_row_sample_public(H, a, rs, N) >= 0, "%s: sample of %d", name, a);
    CHECK(orc_row_sample_public(H, n, rs, N) == -1, "%s: sample of a missing node", name);
    double c[64];
    for (int a = 0; a < n; a++) (void)orc_split_centers(H, a, c);
    CHECK(orc_write(H, path) == 0, "%s: write failed", name);
    orc_free(H);
    orc_h2 *P = orc_points(X, N, d, kernel, h);
    orc_exact_rows(P, rows, 7, W, Q, ex);
    orc_free(P);
    free(rs); free(ex); free(Kt); free(W); free(Y); free(X);
}

int main(int argc, char **argv)
{
    const char *path = argc > 1 ? argv[1] : "oracle_asan.hmc";
    orc_set_threads(2);
    /* distance admissibility, Gaussian; HSS, Laplace; two-means with the budget
     * rule; a binding rank cap; a single leaf.  The last argument but one
     * bounds the sampled-row error against the exact K W: loose where the
     * rank cap or the budget structure (d = 8) limits the accuracy. */
    one("h2_gauss", 900, 3, 0, 0.8, 32, 1e-7, 40, 0, 2.0, 64, 0, 0.0, 5, 1e-2, path);
    one("hss_lap", 700, 2, 1, 1.5, 24, 1e-6, 30, 1, 0.0, 48, 0, 0.0, 3, 1e-2, path);
    one("h2b_twomeans", 800, 8, 0, 1.0, 32, 1e-5, 64, 2, 0.0, 64, 1, 0.03, 4, 0.2, path);
    one("rank_cap", 600, 3, 0, 0.5, 16, 0.0, 4, 0, 1.5, 32, 0, 0.0, 2, 0.2, path);
    one("one_leaf", 20, 3, 0, 1.0, 32, 1e-6, 16, 0, 2.0, 16, 0, 0.0, 1, 1e-12, path);
    /* a standalone ID of a rank-3 block (60 x 12, column-major) */
    double A[60 * 12], T[144], rd[13];
    int k = 0, piv[12];
    for (int j = 0; j < 12; j++)
        for (int i = 0; i < 60; i++) A[j * 60 + i] = sin(i * 0.1 * (j % 3 + 1)) + (j / 3) * cos(i * 0.07 * (j % 3 + 1));
    (void)orc_pqr_id_public(A, 60, 12, 1e-12, 12, &k, piv, T, rd);
    CHECK(k >= 1 && k <= 12, "pqr_id: rank %d", k);
    /* invalid arguments are refused, not read */
    double bad[6] = {0, 1, NAN, 3, 4, 5};
    CHECK(orc_build_ex(bad, 2, 3, 0, 1.0, 2, 1e-6, 4, 0, 2.0, 4, 1, 0, 0.0) == NULL, "NaN accepted");
    CHECK(orc_build_ex(bad, 0, 3, 0, 1.0, 2, 1e-6, 4, 0, 2.0, 4, 1, 0, 0.0) == NULL, "N = 0 accepted");
    if (fails) return 1;
    puts("oracle sanitizer run ok");
    return 0;
}
