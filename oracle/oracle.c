/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain nested loops over the discrete orthogonal 2-simplex (pairs),
 * 3-simplex (triplets) and 4-simplex (quadruplets) in double precision.  It shares no code, header,
 * table or constant with the HIP library; only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  No product path calls it.
 *
 * Domains (paper Sec. I, eq. (1)-(2), read as the pairs / triplets form):
 *   EDM    : pairs i <= j < n           (n(n+1)/2 elements, diagonal included)
 *   LJ     : pairs i <  j < n           (n(n-1)/2 elements)
 *   AT     : triplets i < j < k < n     (n(n-1)(n-2)/6 elements)
 *   K4     : quadruplets i < j < k < l  (n(n-1)(n-2)(n-3)/24 elements)
 *
 * Every function takes FP32 inputs exactly as the GPU reads them and promotes
 * each coordinate to double before any arithmetic.  Sums over OpenMP threads are
 * combined in thread order, so a run with a fixed thread count is deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define PX(X, ldx, i, c) ((double)(X)[(int64_t)(i) * (ldx) + (c)])

int orc_max_threads(void) { return omp_get_max_threads(); }

/* Thread count for the parallel loops that follow (for single-core timings). */
void orc_set_threads(int k) { omp_set_num_threads(k > 0 ? k : 1); }

/* ------------------------------------------------------------------------ */
/* Packed Euclidean distance matrix (paper Sec. I and II: the EDM is a
 * 2-simplex problem; only the upper triangle is needed).  Output layout: the
 * row-major upper triangle with the diagonal, p(i,j) = i*n - i(i-1)/2 + (j-i).
 * This routine returns rows [i0, i1) contiguously, starting at p(i0, i0).      */
void orc_edm_rows(const float *X, int64_t n, int64_t d, int64_t ldx,
                  int64_t i0, int64_t i1, double *out)
{
    const int64_t base = i0 * n - (i0 * (i0 - 1)) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t row = i * n - (i * (i - 1)) / 2 - base;
        for (int64_t j = i; j < n; ++j) {
            double acc = 0.0;
            for (int64_t c = 0; c < d; ++c) {
                const double t = PX(X, ldx, i, c) - PX(X, ldx, j, c);
                acc += t * t;
            }
            out[row + (j - i)] = acc;
        }
    }
}

/* Squared distances of m arbitrary pairs (I[t], J[t]). */
void orc_edm_pairs(const float *X, int64_t d, int64_t ldx, const int64_t *I,
                   const int64_t *J, int64_t m, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < m; ++t) {
        double acc = 0.0;
        for (int64_t c = 0; c < d; ++c) {
            const double u = PX(X, ldx, I[t], c) - PX(X, ldx, J[t], c);
            acc += u * u;
        }
        out[t] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Axilrod-Teller triple-dipole energy (the triple-interaction n-body problem
 * the paper names as a 3-simplex workload, Sec. I).  Textbook angle form:
 *   E_ijk = nu * (1 + 3 cos(g_i) cos(g_j) cos(g_k)) / (r_ij r_jk r_ik)^3
 * with g_a the interior angle of the triangle at particle a.                  */
static double at_term_angle(const float *X, int64_t ldx, int64_t i, int64_t j,
                            int64_t k, double nu)
{
    double xi[3], xj[3], xk[3];
    for (int c = 0; c < 3; ++c) {
        xi[c] = PX(X, ldx, i, c);
        xj[c] = PX(X, ldx, j, c);
        xk[c] = PX(X, ldx, k, c);
    }
    double ij[3], ik[3], jk[3];
    for (int c = 0; c < 3; ++c) {
        ij[c] = xj[c] - xi[c];
        ik[c] = xk[c] - xi[c];
        jk[c] = xk[c] - xj[c];
    }
    const double rij = sqrt(ij[0] * ij[0] + ij[1] * ij[1] + ij[2] * ij[2]);
    const double rik = sqrt(ik[0] * ik[0] + ik[1] * ik[1] + ik[2] * ik[2]);
    const double rjk = sqrt(jk[0] * jk[0] + jk[1] * jk[1] + jk[2] * jk[2]);
    /* angle at i between (j - i) and (k - i) */
    const double ci = (ij[0] * ik[0] + ij[1] * ik[1] + ij[2] * ik[2]) / (rij * rik);
    /* angle at j between (i - j) and (k - j) */
    const double cj = (-ij[0] * jk[0] - ij[1] * jk[1] - ij[2] * jk[2]) / (rij * rjk);
    /* angle at k between (i - k) and (j - k) */
    const double ck = (ik[0] * jk[0] + ik[1] * jk[1] + ik[2] * jk[2]) / (rik * rjk);
    const double rr = rij * rjk * rik;
    return nu * (1.0 + 3.0 * ci * cj * ck) / (rr * rr * rr);
}

/* Energy of all triplets i<j<k whose smallest index i lies in [i0, i1). */
double orc_at_energy(const float *X, int64_t n, int64_t ldx, double nu,
                     int64_t i0, int64_t i1)
{
    const int nt = omp_get_max_threads();
    double *part = (double *)calloc((size_t)nt, sizeof(double));
#pragma omp parallel
    {
        double acc = 0.0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                for (int64_t k = j + 1; k < n; ++k)
                    acc += at_term_angle(X, ldx, i, j, k, nu);
        part[omp_get_thread_num()] = acc;
    }
    double e = 0.0;
    for (int t = 0; t < nt; ++t) e += part[t];
    free(part);
    return e;
}

/* Packed per-triplet energies, the 3-simplex analogue of the packed EDM: the
 * triplets i < j < k < n in lexicographic order.  Rows i in [i0, i1) are
 * written contiguously, starting with (i0, i0+1, i0+2), in exactly the order
 * of the triple loop (row i holds C(n-1-i, 2) elements).                       */
void orc_at_triplet_rows(const float *X, int64_t n, int64_t ldx, double nu,
                         int64_t i0, int64_t i1, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = i0; i < i1; ++i) {
        int64_t o = 0; /* elements of rows i0 .. i-1 */
        for (int64_t r = i0; r < i; ++r) o += (n - 1 - r) * (n - 2 - r) / 2;
        for (int64_t j = i + 1; j < n; ++j)
            for (int64_t k = j + 1; k < n; ++k)
                out[o++] = at_term_angle(X, ldx, i, j, k, nu);
    }
}

/* Analytic gradient of one Axilrod-Teller term with respect to the three
 * positions.  With s1=|x_j-x_i|^2, s2=|x_k-x_j|^2, s3=|x_i-x_k|^2 the term is
 *   E = nu (P - 3/8 T) P^(-5/2),  P = s1 s2 s3,  T = t1 t2 t3,
 *   t1 = s3-s1-s2, t2 = s1-s2-s3, t3 = s2-s3-s1
 * (the law of cosines turns each cosine into t_a / (2 r r)).  dE/ds_p follows
 * by the product rule; ds1/dx_i = -2(x_j-x_i), ds3/dx_i = 2(x_i-x_k), ...     */
static void at_term_grad(const double *xi, const double *xj, const double *xk,
                         double nu, double *gi, double *gj, double *gk)
{
    double a[3], b[3], c[3];
    for (int q = 0; q < 3; ++q) {
        a[q] = xj[q] - xi[q]; /* s1 = |a|^2 */
        b[q] = xk[q] - xj[q]; /* s2 = |b|^2 */
        c[q] = xi[q] - xk[q]; /* s3 = |c|^2 */
    }
    const double s1 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    const double s2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double s3 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    const double t1 = s3 - s1 - s2, t2 = s1 - s2 - s3, t3 = s2 - s3 - s1;
    const double P = s1 * s2 * s3, T = t1 * t2 * t3;
    const double N = P - 0.375 * T;
    const double Pm52 = pow(P, -2.5), Pm72 = pow(P, -3.5);
    /* dP/ds_p */
    const double dP1 = s2 * s3, dP2 = s1 * s3, dP3 = s1 * s2;
    /* dT/ds_p, using dt1/ds = (-1,-1,+1), dt2/ds = (+1,-1,-1), dt3/ds = (-1,+1,-1) */
    const double dT1 = -t2 * t3 + t1 * t3 - t1 * t2;
    const double dT2 = -t2 * t3 - t1 * t3 + t1 * t2;
    const double dT3 = t2 * t3 - t1 * t3 - t1 * t2;
    const double E1 = nu * ((dP1 - 0.375 * dT1) * Pm52 - 2.5 * N * Pm72 * dP1);
    const double E2 = nu * ((dP2 - 0.375 * dT2) * Pm52 - 2.5 * N * Pm72 * dP2);
    const double E3 = nu * ((dP3 - 0.375 * dT3) * Pm52 - 2.5 * N * Pm72 * dP3);
    for (int q = 0; q < 3; ++q) {
        gi[q] = -2.0 * E1 * a[q] + 2.0 * E3 * c[q];
        gj[q] = 2.0 * E1 * a[q] - 2.0 * E2 * b[q];
        gk[q] = 2.0 * E2 * b[q] - 2.0 * E3 * c[q];
    }
}

/* Full gradient dE/dx (n x 3, row-major) of the Axilrod-Teller energy. */
void orc_at_grad(const float *X, int64_t n, int64_t ldx, double nu, double *G)
{
    const int nt = omp_get_max_threads();
    double *priv = (double *)calloc((size_t)nt * (size_t)n * 3, sizeof(double));
#pragma omp parallel
    {
        double *g = priv + (size_t)omp_get_thread_num() * (size_t)n * 3;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            double xi[3] = {PX(X, ldx, i, 0), PX(X, ldx, i, 1), PX(X, ldx, i, 2)};
            for (int64_t j = i + 1; j < n; ++j) {
                double xj[3] = {PX(X, ldx, j, 0), PX(X, ldx, j, 1), PX(X, ldx, j, 2)};
                for (int64_t k = j + 1; k < n; ++k) {
                    double xk[3] = {PX(X, ldx, k, 0), PX(X, ldx, k, 1), PX(X, ldx, k, 2)};
                    double gi[3], gj[3], gk[3];
                    at_term_grad(xi, xj, xk, nu, gi, gj, gk);
                    for (int q = 0; q < 3; ++q) {
                        g[i * 3 + q] += gi[q];
                        g[j * 3 + q] += gj[q];
                        g[k * 3 + q] += gk[q];
                    }
                }
            }
        }
    }
    memset(G, 0, sizeof(double) * (size_t)n * 3);
    for (int t = 0; t < nt; ++t)
        for (int64_t q = 0; q < n * 3; ++q) G[q] += priv[(size_t)t * (size_t)n * 3 + q];
    free(priv);
}

/* Gradient with respect to the m selected particles only: for particle a,
 * the sum over every unordered pair {b, c} of other particles of the term's
 * derivative at a.  A different loop from orc_at_grad, for sampled checks at
 * sizes where the full O(n^3) gradient is too slow.                          */
void orc_at_grad_rows(const float *X, int64_t n, int64_t ldx, double nu,
                      const int64_t *idx, int64_t m, double *G)
{
    for (int64_t t = 0; t < m; ++t) {
        const int64_t a = idx[t];
        const double xa[3] = {PX(X, ldx, a, 0), PX(X, ldx, a, 1), PX(X, ldx, a, 2)};
        const int nt = omp_get_max_threads();
        double *part = (double *)calloc((size_t)nt * 3, sizeof(double));
#pragma omp parallel
        {
            double acc[3] = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
            for (int64_t b = 0; b < n; ++b) {
                if (b == a) continue;
                const double xb[3] = {PX(X, ldx, b, 0), PX(X, ldx, b, 1), PX(X, ldx, b, 2)};
                for (int64_t c = b + 1; c < n; ++c) {
                    if (c == a) continue;
                    const double xc[3] = {PX(X, ldx, c, 0), PX(X, ldx, c, 1), PX(X, ldx, c, 2)};
                    double ga[3], gb[3], gc[3];
                    at_term_grad(xa, xb, xc, nu, ga, gb, gc);
                    acc[0] += ga[0];
                    acc[1] += ga[1];
                    acc[2] += ga[2];
                }
            }
            double *p = part + 3 * omp_get_thread_num();
            p[0] = acc[0];
            p[1] = acc[1];
            p[2] = acc[2];
        }
        G[3 * t + 0] = G[3 * t + 1] = G[3 * t + 2] = 0.0;
        for (int q = 0; q < nt; ++q) {
            G[3 * t + 0] += part[3 * q + 0];
            G[3 * t + 1] += part[3 * q + 1];
            G[3 * t + 2] += part[3 * q + 2];
        }
        free(part);
    }
}

/* ------------------------------------------------------------------------ */
/* Lennard-Jones pairs (an n-body pair interaction on the 2-simplex, Sec. I):
 *   phi(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6)   for r < rc, else 0,
 * summed over i<j, with no shift and open boundaries.  Whether a pair lies
 * inside the cutoff is decided on the FP32 squared distance
 *   s32 = fl(fma(dz,dz, fma(dy,dy, dx*dx))),  d* = fl(x_j* - x_i*)
 * compared with fl(rc*rc), so that both sides take the same decision; the
 * energy and force themselves are evaluated in FP64.                        */
static int lj_inside(const float *X, int64_t ldx, int64_t i, int64_t j, float rc2)
{
    const float dx = X[j * ldx + 0] - X[i * ldx + 0];
    const float dy = X[j * ldx + 1] - X[i * ldx + 1];
    const float dz = X[j * ldx + 2] - X[i * ldx + 2];
    const float s = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    return s < rc2;
}

double orc_lj_energy(const float *X, int64_t n, int64_t ldx, double eps,
                     double sigma, double rc)
{
    const float rc2 = (float)(rc * rc);
    const int nt = omp_get_max_threads();
    double *part = (double *)calloc((size_t)nt, sizeof(double));
#pragma omp parallel
    {
        double acc = 0.0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                if (!lj_inside(X, ldx, i, j, rc2)) continue;
                double r2 = 0.0;
                for (int q = 0; q < 3; ++q) {
                    const double u = PX(X, ldx, j, q) - PX(X, ldx, i, q);
                    r2 += u * u;
                }
                const double r = sqrt(r2);
                const double sr6 = pow(sigma / r, 6.0);
                acc += 4.0 * eps * (sr6 * sr6 - sr6);
            }
        part[omp_get_thread_num()] = acc;
    }
    double e = 0.0;
    for (int t = 0; t < nt; ++t) e += part[t];
    free(part);
    return e;
}

/* dE/dx for the Lennard-Jones energy above: dphi/dr * (x_i - x_j)/r on i. */
void orc_lj_grad(const float *X, int64_t n, int64_t ldx, double eps, double sigma,
                 double rc, double *G)
{
    const float rc2 = (float)(rc * rc);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        double g[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
            if (!lj_inside(X, ldx, lo, hi, rc2)) continue;
            double u[3], r2 = 0.0;
            for (int q = 0; q < 3; ++q) {
                u[q] = PX(X, ldx, i, q) - PX(X, ldx, j, q);
                r2 += u[q] * u[q];
            }
            const double r = sqrt(r2);
            const double sr6 = pow(sigma / r, 6.0);
            /* dphi/dr = 4 eps (-12 sigma^12 / r^13 + 6 sigma^6 / r^7) */
            const double dphidr = 4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r;
            for (int q = 0; q < 3; ++q) g[q] += dphidr * u[q] / r;
        }
        G[3 * i + 0] = g[0];
        G[3 * i + 1] = g[1];
        G[3 * i + 2] = g[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Element checksums.  Each simplex element has an integer id, and the checksum
 * of a set of elements is the wrapping 64-bit sum of SplitMix64 (Steele, Lea and
 * Flood, OOPSLA 2014) finalisations of those ids.  The id maps are bijections
 * onto [0, V), so the checksum of a whole simplex is the sum over 0..V-1.
 *   pairs i<=j     : id = i*n - i(i-1)/2 + (j-i)       (packed row-major order)
 *   pairs i<j      : id = j(j-1)/2 + i
 *   triplets i<=j<=k: id = k(k+1)(k+2)/6 + j(j+1)/2 + i
 *   triplets i<j<k : id = k(k-1)(k-2)/6 + j(j-1)/2 + i
 *   quadruplets i<=j<=k<=l: id = l(l+1)(l+2)(l+3)/24 + k(k+1)(k+2)/6 + j(j+1)/2 + i
 *   quadruplets i<j<k<l   : id = l(l-1)(l-2)(l-3)/24 + k(k-1)(k-2)/6 + j(j-1)/2 + i
 */
static uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_mix64(uint64_t x) { return orc_splitmix64(x); }

/* Sum of mix(id) for id in [0, V): the checksum of a whole simplex. */
uint64_t orc_checksum_range(uint64_t v)
{
    const int nt = omp_get_max_threads();
    uint64_t *part = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
#pragma omp parallel
    {
        uint64_t acc = 0;
#pragma omp for schedule(static)
        for (int64_t t = 0; t < (int64_t)v; ++t) acc += orc_splitmix64((uint64_t)t);
        part[omp_get_thread_num()] = acc;
    }
    uint64_t s = 0;
    for (int t = 0; t < nt; ++t) s += part[t];
    free(part);
    return s;
}

/* Checksum of the elements a nested-loop walk visits: kind 0 = pairs i<=j,
 * 1 = pairs i<j, 2 = triplets i<=j<=k, 3 = triplets i<j<k, 4 = quadruplets
 * i<=j<=k<=l, 5 = quadruplets i<j<k<l.  This enumerates the elements and their
 * ids directly (no use of the bijection property).                           */
uint64_t orc_checksum_walk(int kind, int64_t n, int64_t *count)
{
    uint64_t s = 0;
    int64_t c = 0;
    if (kind == 0) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i; j < n; ++j) {
                s += orc_splitmix64((uint64_t)(i * n - (i * (i - 1)) / 2 + (j - i)));
                ++c;
            }
    } else if (kind == 1) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                s += orc_splitmix64((uint64_t)((j * (j - 1)) / 2 + i));
                ++c;
            }
    } else if (kind == 2) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i; j < n; ++j)
                for (int64_t k = j; k < n; ++k) {
                    s += orc_splitmix64((uint64_t)((k * (k + 1) * (k + 2)) / 6 + (j * (j + 1)) / 2 + i));
                    ++c;
                }
    } else if (kind == 3) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                for (int64_t k = j + 1; k < n; ++k) {
                    s += orc_splitmix64((uint64_t)((k * (k - 1) * (k - 2)) / 6 + (j * (j - 1)) / 2 + i));
                    ++c;
                }
    } else if (kind == 4) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i; j < n; ++j)
                for (int64_t k = j; k < n; ++k)
                    for (int64_t l = k; l < n; ++l) {
                        s += orc_splitmix64((uint64_t)((l * (l + 1) * (l + 2) * (l + 3)) / 24 +
                                                       (k * (k + 1) * (k + 2)) / 6 + (j * (j + 1)) / 2 + i));
                        ++c;
                    }
    } else {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                for (int64_t k = j + 1; k < n; ++k)
                    for (int64_t l = k + 1; l < n; ++l) {
                        s += orc_splitmix64((uint64_t)((l * (l - 1) * (l - 2) * (l - 3)) / 24 +
                                                       (k * (k - 1) * (k - 2)) / 6 + (j * (j - 1)) / 2 + i));
                        ++c;
                    }
    }
    if (count) *count = c;
    return s;
}

/* ------------------------------------------------------------------------ */
/* 4-point contacts on the 4-simplex: the number of quadruplets i < j < k < l
 * whose six pairs all lie within the contact radius rc (the 4-cliques of the
 * contact graph; the 4-point analogue of the correlation counts the paper
 * lists among simplex-shaped problems, Sec. I).  A pair is in contact when the
 * FP32 squared distance s32 = fl(fma(dz,dz, fma(dy,dy, dx*dx))), d* = fl(x_j* -
 * x_i*) for i < j, is below fl(rc*rc) -- the same decision rule as the LJ cutoff,
 * so both sides decide every pair identically and the count is exact.
 * Counting: forward neighbour lists N(i) = {j > i in contact} (sorted), then
 * for every i, j in N(i) the common list C = N(i) & N(j), and for every k in C
 * the size of C & N(k) (each l > k).                                         */
static int64_t isect(const int32_t *a, int64_t na, const int32_t *b, int64_t nb, int32_t *out)
{
    int64_t i = 0, j = 0, c = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else {
            if (out) out[c] = a[i];
            ++c; ++i; ++j;
        }
    }
    return c;
}

int64_t orc_quad_contacts(const float *X, int64_t n, int64_t ldx, double rc)
{
    if (n < 4) return 0;
    const float rc2 = (float)(rc * rc);
    int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) deg[i] += lj_inside(X, ldx, i, j, rc2);
    for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + deg[i];
    int32_t *adj = (int32_t *)malloc((size_t)(start[n] > 0 ? start[n] : 1) * sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = start[i];
        for (int64_t j = i + 1; j < n; ++j)
            if (lj_inside(X, ldx, i, j, rc2)) adj[c++] = (int32_t)j;
    }
    int64_t total = 0;
#pragma omp parallel reduction(+ : total)
    {
        int32_t *cij = (int32_t *)malloc((size_t)n * sizeof(int32_t));
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            const int32_t *ni = adj + start[i];
            const int64_t di = deg[i];
            for (int64_t a = 0; a < di; ++a) {
                const int32_t j = ni[a];
                const int64_t nc = isect(ni, di, adj + start[j], deg[j], cij);
                for (int64_t b = 0; b < nc; ++b) {
                    const int32_t k = cij[b];
                    total += isect(cij, nc, adj + start[k], deg[k], NULL);
                }
            }
        }
        free(cij);
    }
    free(adj);
    free(deg);
    free(start);
    return total;
}
