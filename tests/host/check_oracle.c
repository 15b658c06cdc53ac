/* Host driver for the C oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * every entry point runs on small inputs whose buffers are sized exactly, and a
 * few closed forms are checked (equilateral triangle energy 11 nu / (8 r^9),
 * cube-corner 4-cliques, simplex volumes of the checksum walks).  Exit status 0
 * and "ok" on success.  Built together with oracle.c. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_edm_rows(const float *X, int64_t n, int64_t d, int64_t ldx, int64_t i0, int64_t i1, double *out);
void orc_edm_pairs(const float *X, int64_t d, int64_t ldx, const int64_t *I, const int64_t *J, int64_t m,
                   double *out);
double orc_at_energy(const float *X, int64_t n, int64_t ldx, double nu, int64_t i0, int64_t i1);
void orc_at_triplet_rows(const float *X, int64_t n, int64_t ldx, double nu, int64_t i0, int64_t i1, double *out);
void orc_at_grad(const float *X, int64_t n, int64_t ldx, double nu, double *G);
void orc_at_grad_rows(const float *X, int64_t n, int64_t ldx, double nu, const int64_t *idx, int64_t m,
                      double *G);
double orc_lj_energy(const float *X, int64_t n, int64_t ldx, double eps, double sigma, double rc);
void orc_lj_grad(const float *X, int64_t n, int64_t ldx, double eps, double sigma, double rc, double *G);
uint64_t orc_checksum_range(uint64_t v);
uint64_t orc_checksum_walk(int kind, int64_t n, int64_t *count);
int64_t orc_quad_contacts(const float *X, int64_t n, int64_t ldx, double rc);

static int fails = 0;
#define CHECK(c, msg)                              \
    do {                                           \
        if (!(c)) {                                \
            printf("check failed: %s\n", msg);     \
            ++fails;                               \
        }                                          \
    } while (0)

int main(void)
{
    const int64_t n = 37, ldx = 4;
    float *X = malloc(sizeof(float) * n * ldx);
    srand(7);
    for (int64_t i = 0; i < n * ldx; ++i) X[i] = (float)(rand() % 1000) / 100.0f;
    /* EDM rows: all rows of the packed triangle */
    double *D = malloc(sizeof(double) * n * (n + 1) / 2);
    orc_edm_rows(X, n, 3, ldx, 0, n, D);
    CHECK(D[0] == 0.0, "edm diagonal");
    int64_t I[3] = {0, 5, 36}, J[3] = {36, 5, 36};
    double Dp[3];
    orc_edm_pairs(X, 3, ldx, I, J, 3, Dp);
    CHECK(Dp[1] == 0.0 && Dp[2] == 0.0 && Dp[0] == D[36], "edm pairs");
    /* Axilrod-Teller: energy, packed terms, gradients */
    const double e = orc_at_energy(X, n, ldx, 1.0, 0, n);
    const int64_t m3 = n * (n - 1) * (n - 2) / 6;
    double *T = malloc(sizeof(double) * m3);
    orc_at_triplet_rows(X, n, ldx, 1.0, 0, n, T);
    double s = 0.0;
    for (int64_t q = 0; q < m3; ++q) s += T[q];
    CHECK(fabs(s - e) <= 1e-9 * fabs(e), "packed terms sum to the energy");
    double *G = malloc(sizeof(double) * n * 3);
    orc_at_grad(X, n, ldx, 1.0, G);
    int64_t idx[2] = {3, 30};
    double Gr[6];
    orc_at_grad_rows(X, n, ldx, 1.0, idx, 2, Gr);
    CHECK(fabs(Gr[0] - G[9]) <= 1e-9 * (fabs(G[9]) + 1e-30), "gradient rows");
    const float tri[9] = {0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.5f, 0.8660254f, 0.f};
    const double eq = orc_at_energy(tri, 3, 3, 1.0, 0, 3);
    CHECK(fabs(eq - 11.0 / 8.0) <= 1e-5, "equilateral triangle");
    /* Lennard-Jones */
    const double el = orc_lj_energy(X, n, ldx, 1.0, 1.0, 3.0);
    orc_lj_grad(X, n, ldx, 1.0, 1.0, 3.0, G);
    CHECK(isfinite(el), "lj energy");
    /* checksums: walks count the simplex volumes */
    int64_t c;
    const uint64_t w = orc_checksum_walk(2, 9, &c);
    CHECK(c == 165 && w == orc_checksum_range(165), "triplet walk");
    orc_checksum_walk(5, 9, &c);
    CHECK(c == 126, "quadruplet walk");
    /* 4-point contacts: cube corners below 1.01 sqrt(2) */
    float C[24];
    for (int k = 0; k < 8; ++k) {
        C[3 * k + 0] = (float)(k >> 2 & 1);
        C[3 * k + 1] = (float)(k >> 1 & 1);
        C[3 * k + 2] = (float)(k & 1);
    }
    CHECK(orc_quad_contacts(C, 8, 3, 1.01 * sqrt(2.0)) == 16, "cube corners");
    CHECK(orc_quad_contacts(X, n, ldx, 100.0) == n * (n - 1) * (n - 2) * (n - 3) / 24, "all in contact");
    free(X); free(D); free(T); free(G);
    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
