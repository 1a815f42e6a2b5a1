/*
 * gf_oracle_sun.c -- plain FP64 CPU oracle for Landau/Coulomb gauge fixing of
 * SU(N) lattice links by overrelaxation, N >= 2 (the paper's method for a
 * general number of colours: the local maximisation runs over all
 * N(N-1)/2 SU(2) subgroups).
 *
 * TEST INFRASTRUCTURE ONLY, like gf_oracle.c (same library): the HIP product
 * path never links, loads or calls it.
 *
 * Field layout: U[site][mu][row][col] as C99 double complex, N x N per link,
 * site = x + nx*(y + ny*(z + nz*t)), mu = 0..3 along x, y, z, t, periodic.
 * gauge = 0 Landau (mu = 0..3 in the functional), 1 Coulomb (mu = 0..2; the
 * temporal links are still rotated).
 *
 * Readings (the SU(3) readings of gf_oracle.c, written for general N):
 *  - subgroups (a, b), a < b, visited in lexicographic order
 *    (0,1), (0,2), ..., (0,N-1), (1,2), ..., (N-2,N-1), one pass each, K
 *    rebuilt from the links as updated by the previous subgroup; for N = 3
 *    this is (0,1), (0,2), (1,2);
 *  - the SU(2) solve and its exact principal power are oracle_su2_solve;
 *  - Delta(x) = A - (Tr A / N) 1 with A = M - M^dagger,
 *    M = sum_nu [U_nu(x - nu) - U_nu(x)]; theta = sum_x |Delta|^2 / (N V);
 *    F = sum_x sum_mu Re Tr U_mu(x) / (d N V);
 *  - reunitarisation: Gram-Schmidt of rows 0..N-2; the last row is the
 *    complex conjugate of its cofactors (the unique unit row completing an
 *    SU(N) matrix: U^dagger = adj U when det U = 1). For N = 3 that is
 *    conj(r0 x r1).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define NMAX 8

void oracle_su2_solve(const double b[4], double omega, double out[4]);

static long volume(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static long nbr(const int d[4], long s, int mu, int step)
{
    int c[4];
    long r = s;
    for (int k = 0; k < 4; k++) { c[k] = (int)(r % d[k]); r /= d[k]; }
    c[mu] = (c[mu] + step + d[mu]) % d[mu];
    return c[0] + (long)d[0] * (c[1] + (long)d[1] * (c[2] + (long)d[2] * c[3]));
}

static int parity(const int d[4], long s)
{
    int p = 0;
    for (int k = 0; k < 4; k++) { p += (int)(s % d[k]); s /= d[k]; }
    return p & 1;
}

static int ndirs(int gauge) { return gauge == 1 ? 3 : 4; }

static cplx *lnk(cplx *U, int n, long s, int mu) { return U + (s * 4 + mu) * n * n; }
static const cplx *clnk(const cplx *U, int n, long s, int mu) { return U + (s * 4 + mu) * n * n; }

/* r = a b (n x n), r may not alias a or b */
static void mmul(int n, const cplx *a, const cplx *b, cplx *r)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            cplx acc = 0;
            for (int k = 0; k < n; k++) acc += a[i * n + k] * b[k * n + j];
            r[i * n + j] = acc;
        }
}

static void mdag(int n, const cplx *a, cplx *r)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) r[i * n + j] = conj(a[j * n + i]);
}

/* determinant by Laplace expansion along the first row (the definition;
 * n <= NMAX - 1 here) */
static cplx det_laplace(int n, const cplx *a)
{
    if (n == 1) return a[0];
    cplx sub[NMAX * NMAX];
    cplx acc = 0;
    for (int j = 0; j < n; j++) {
        int m = 0;
        for (int i = 1; i < n; i++)
            for (int k = 0; k < n; k++)
                if (k != j) sub[m++] = a[i * n + k];
        cplx t = a[j] * det_laplace(n - 1, sub);
        acc += (j & 1) ? -t : t;
    }
    return acc;
}

/* ------------------------------------------------------------------ */
/* observables                                                         */
/* ------------------------------------------------------------------ */

static void divergence_n(const cplx *U, const int d[4], int n, int gauge, long s, cplx *A)
{
    cplx M[NMAX * NMAX];
    for (int e = 0; e < n * n; e++) M[e] = 0;
    for (int nu = 0; nu < ndirs(gauge); nu++) {
        const cplx *b = clnk(U, n, nbr(d, s, nu, -1), nu), *f = clnk(U, n, s, nu);
        for (int e = 0; e < n * n; e++) M[e] += b[e] - f[e];
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) A[i * n + j] = M[i * n + j] - conj(M[j * n + i]);
    cplx tr = 0;
    for (int i = 0; i < n; i++) tr += A[i * n + i];
    for (int i = 0; i < n; i++) A[i * n + i] -= tr / n;
}

void oracle_sun_quality(const cplx *U, const int d[4], int n, int gauge, double *F, double *theta)
{
    long V = volume(d);
    int nd = ndirs(gauge);
    double fsum = 0, tsum = 0;
    cplx D[NMAX * NMAX];
    for (long s = 0; s < V; s++) {
        for (int mu = 0; mu < nd; mu++) {
            const cplx *u = clnk(U, n, s, mu);
            for (int i = 0; i < n; i++) fsum += creal(u[i * n + i]);
        }
        divergence_n(U, d, n, gauge, s, D);
        for (int e = 0; e < n * n; e++) tsum += creal(D[e] * conj(D[e]));
    }
    *F = fsum / (nd * (double)n * V);
    *theta = tsum / ((double)n * V);
}

/* K(x) of eq. (5): sum over the functional's directions of
 * U_mu(x) + U_mu(x - mu)^dagger (n x n, row-major) */
void oracle_sun_staple(const cplx *U, const int d[4], int n, int gauge, long s, cplx *K)
{
    for (int e = 0; e < n * n; e++) K[e] = 0;
    for (int mu = 0; mu < ndirs(gauge); mu++) {
        const cplx *f = clnk(U, n, s, mu), *b = clnk(U, n, nbr(d, s, mu, -1), mu);
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) K[i * n + j] += f[i * n + j] + conj(b[j * n + i]);
    }
}

/* ------------------------------------------------------------------ */
/* local update                                                        */
/* ------------------------------------------------------------------ */

/* The embedded SU(2) element of the subgroup (a, b) that the overrelaxed
 * local solution picks at site s on the current field (n x n, written to G). */
void oracle_sun_subgroup_matrix(const cplx *U, const int d[4], int n, int gauge, long s, int a, int b,
                                double omega, cplx *G)
{
    cplx K[NMAX * NMAX];
    oracle_sun_staple(U, d, n, gauge, s, K);
    cplx kaa = K[a * n + a], kab = K[a * n + b], kba = K[b * n + a], kbb = K[b * n + b];
    double q[4] = {creal(kaa + kbb) / 2, cimag(kab + kba) / 2, creal(kab - kba) / 2, cimag(kaa - kbb) / 2};
    double g[4];
    oracle_su2_solve(q, omega, g);
    for (int e = 0; e < n * n; e++) G[e] = 0;
    for (int i = 0; i < n; i++) G[i * n + i] = 1;
    G[a * n + a] = g[0] + I * g[3];
    G[a * n + b] = g[2] + I * g[1];
    G[b * n + a] = -g[2] + I * g[1];
    G[b * n + b] = g[0] - I * g[3];
}

/* U_mu(x) <- G U_mu(x), U_mu(x - mu) <- U_mu(x - mu) G^dagger for all four mu */
void oracle_sun_apply(cplx *U, const int d[4], int n, long s, const cplx *G)
{
    cplx Gd[NMAX * NMAX], t[NMAX * NMAX];
    mdag(n, G, Gd);
    for (int mu = 0; mu < 4; mu++) {
        cplx *f = lnk(U, n, s, mu);
        mmul(n, G, f, t);
        memcpy(f, t, sizeof(cplx) * n * n);
        cplx *b = lnk(U, n, nbr(d, s, mu, -1), mu);
        mmul(n, b, Gd, t);
        memcpy(b, t, sizeof(cplx) * n * n);
    }
}

void oracle_sun_subgroup_update(cplx *U, const int d[4], int n, int gauge, long s, int a, int b, double omega)
{
    cplx G[NMAX * NMAX];
    oracle_sun_subgroup_matrix(U, d, n, gauge, s, a, b, omega, G);
    oracle_sun_apply(U, d, n, s, G);
}

void oracle_sun_site_update(cplx *U, const int d[4], int n, int gauge, long s, double omega)
{
    for (int a = 0; a < n; a++)
        for (int b = a + 1; b < n; b++) oracle_sun_subgroup_update(U, d, n, gauge, s, a, b, omega);
}

void oracle_sun_half_sweep(cplx *U, const int d[4], int n, int gauge, int par, double omega)
{
    long V = volume(d);
    for (long s = 0; s < V; s++)
        if (parity(d, s) == par) oracle_sun_site_update(U, d, n, gauge, s, omega);
}

void oracle_sun_sweep(cplx *U, const int d[4], int n, int gauge, double omega)
{
    oracle_sun_half_sweep(U, d, n, gauge, 0, omega);
    oracle_sun_half_sweep(U, d, n, gauge, 1, omega);
}

/* ------------------------------------------------------------------ */
/* reunitarisation                                                     */
/* ------------------------------------------------------------------ */

static void reunit_n(int n, cplx *u)
{
    for (int r = 0; r < n - 1; r++) {
        cplx *row = u + r * n;
        for (int q = 0; q < r; q++) {
            const cplx *prev = u + q * n;
            cplx p = 0;
            for (int j = 0; j < n; j++) p += conj(prev[j]) * row[j];
            for (int j = 0; j < n; j++) row[j] -= p * prev[j];
        }
        double nrm = 0;
        for (int j = 0; j < n; j++) nrm += creal(row[j] * conj(row[j]));
        nrm = sqrt(nrm);
        for (int j = 0; j < n; j++) row[j] /= nrm;
    }
    /* last row: conj of the cofactors C_{n-1,j} = (-1)^(n-1+j) minor */
    cplx sub[NMAX * NMAX];
    for (int j = 0; j < n; j++) {
        int m = 0;
        for (int i = 0; i < n - 1; i++)
            for (int k = 0; k < n; k++)
                if (k != j) sub[m++] = u[i * n + k];
        cplx c = det_laplace(n - 1, sub);
        if ((n - 1 + j) & 1) c = -c;
        u[(n - 1) * n + j] = conj(c);
    }
}

void oracle_sun_reunit(cplx *U, int n, long nlinks)
{
    for (long l = 0; l < nlinks; l++) reunit_n(n, U + l * n * n);
}

/* determinant of every n x n matrix in U (for tests) */
void oracle_sun_det(const cplx *U, int n, long nmat, cplx *out)
{
    for (long l = 0; l < nmat; l++) out[l] = det_laplace(n, U + l * n * n);
}

/* Alg. 1 (same schedule as oracle_fix): returns 1 if theta < eps at exit */
int oracle_sun_fix(cplx *U, const int d[4], int n, int gauge, double omega, double eps, int max_iter,
                   int reunit_every, int check_every, long start_sweep, int *iters, double *F, double *theta)
{
    if (check_every < 1) check_every = 1;
    long V = volume(d);
    oracle_sun_quality(U, d, n, gauge, F, theta);
    int it = 0, fresh = 1;
    while (it < max_iter) {
        if (fresh && *theta < eps) break;
        oracle_sun_sweep(U, d, n, gauge, omega);
        it++;
        if (reunit_every > 0 && (start_sweep + it) % reunit_every == 0) oracle_sun_reunit(U, n, 4 * V);
        fresh = (it % check_every == 0) || it == max_iter;
        if (fresh) oracle_sun_quality(U, d, n, gauge, F, theta);
    }
    *iters = it;
    return *theta < eps;
}
