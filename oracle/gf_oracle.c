/*
 * gf_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for
 * Landau/Coulomb gauge fixing of SU(3) lattice links by overrelaxation
 * (N. Cardoso, "Coulomb and Landau Gauge Fixing in GPUs using CUDA and
 * MILC", Lattice 2014, arXiv:1412.1498).
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library to check and to time against; the HIP
 * product path never links, loads or calls it, and it includes nothing from
 * the product.
 *
 * Field layout ("canonical", array of structures): U[site][mu][row][col] as
 * C99 double complex, site = x + nx*(y + ny*(z + nz*t)), mu = 0,1,2,3 along
 * x,y,z,t (t is the temporal direction), periodic boundary conditions.
 * gauge = 0 is Landau (directions mu = 0..3 enter the functional), gauge = 1
 * is Coulomb (mu = 0..2 enter; the temporal links are still rotated by g(x)).
 *
 * Readings of the paper taken here (where it is silent or terse):
 *  - g^omega is the exact principal power of the SU(2) solution: with
 *    g = (cos phi, n sin phi), phi in [0, pi], g^omega = (cos w phi, n sin w phi).
 *  - subgroups are visited in the order (0,1), (0,2), (1,2), one pass each,
 *    with K rebuilt from the links as updated by the previous subgroup.
 *  - a degenerate block (zero SU(2) projection) leaves the links unchanged;
 *    g = -1 is over-rotated about the third quaternion axis.
 *  - Delta(x) in the quality measure is literal: A = M - M^dagger with
 *    M = sum_nu [U_nu(x - nu) - U_nu(x)], minus (Tr A / 3) 1, no extra factor.
 *  - F is normalised by the number d of directions in the functional
 *    (d = 4 Landau, d = 3 Coulomb), so F = 1 on the unit field.
 *  - reunitarisation is Gram-Schmidt on rows 0 and 1, row 2 = conj(r0 x r1).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared -std=c99 -o liboracle.so gf_oracle.c -lm
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
typedef struct { cplx m[3][3]; } mat3;

/* ------------------------------------------------------------------ */
/* lattice geometry                                                    */
/* ------------------------------------------------------------------ */

static long volume(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void coords(const int d[4], long s, int c[4])
{
    c[0] = (int)(s % d[0]); s /= d[0];
    c[1] = (int)(s % d[1]); s /= d[1];
    c[2] = (int)(s % d[2]); s /= d[2];
    c[3] = (int)s;
}

static long site_of(const int d[4], const int c[4])
{
    return c[0] + (long)d[0] * (c[1] + (long)d[1] * (c[2] + (long)d[2] * c[3]));
}

/* periodic neighbour x + step * mu_hat, step = +1 or -1 */
static long neighbour(const int d[4], long s, int mu, int step)
{
    int c[4];
    coords(d, s, c);
    c[mu] = (c[mu] + step + d[mu]) % d[mu];
    return site_of(d, c);
}

static int parity_of(const int d[4], long s)
{
    int c[4];
    coords(d, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static mat3 *link(cplx *U, long s, int mu) { return (mat3 *)(U + (s * 4 + mu) * 9); }
static const mat3 *clink(const cplx *U, long s, int mu) { return (const mat3 *)(U + (s * 4 + mu) * 9); }

static int ndirs(int gauge) { return gauge == 1 ? 3 : 4; }

/* ------------------------------------------------------------------ */
/* 3x3 complex algebra                                                 */
/* ------------------------------------------------------------------ */

static mat3 mat_zero(void) { mat3 r; for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) r.m[i][j] = 0; return r; }
static mat3 mat_unit(void) { mat3 r = mat_zero(); r.m[0][0] = r.m[1][1] = r.m[2][2] = 1; return r; }

static mat3 mat_mul(const mat3 *a, const mat3 *b)
{
    mat3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx acc = 0;
            for (int k = 0; k < 3; k++) acc += a->m[i][k] * b->m[k][j];
            r.m[i][j] = acc;
        }
    return r;
}

static mat3 mat_dag(const mat3 *a)
{
    mat3 r;
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) r.m[i][j] = conj(a->m[j][i]);
    return r;
}

static void mat_acc(mat3 *r, const mat3 *a, double sign)
{
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) r->m[i][j] += sign * a->m[i][j];
}

static cplx mat_trace(const mat3 *a) { return a->m[0][0] + a->m[1][1] + a->m[2][2]; }

/* ------------------------------------------------------------------ */
/* observables: eqs. (1)-(3)                                           */
/* ------------------------------------------------------------------ */

/* Delta(x) of eq. (3): sum over the functional's directions of
 * [U_nu(x - nu) - U_nu(x)], minus its hermitian conjugate, minus the trace. */
static mat3 divergence(const cplx *U, const int d[4], int gauge, long s)
{
    mat3 M = mat_zero();
    for (int nu = 0; nu < ndirs(gauge); nu++) {
        mat_acc(&M, clink(U, neighbour(d, s, nu, -1), nu), +1.0);
        mat_acc(&M, clink(U, s, nu), -1.0);
    }
    mat3 Md = mat_dag(&M);
    mat3 A = M;
    mat_acc(&A, &Md, -1.0);
    cplx tr3 = mat_trace(&A) / 3.0;
    for (int i = 0; i < 3; i++) A.m[i][i] -= tr3;
    return A;
}

/* F (eq. 1, on the already transformed field, i.e. g = 1) and theta (eq. 2). */
void oracle_quality(const cplx *U, const int d[4], int gauge, double *F, double *theta)
{
    long V = volume(d);
    int nd = ndirs(gauge);
    double fsum = 0, tsum = 0;
    for (long s = 0; s < V; s++) {
        for (int mu = 0; mu < nd; mu++) fsum += creal(mat_trace(clink(U, s, mu)));
        mat3 D = divergence(U, d, gauge, s);
        mat3 Dd = mat_dag(&D);
        mat3 DDd = mat_mul(&D, &Dd);
        tsum += creal(mat_trace(&DDd));
    }
    *F = fsum / (nd * 3.0 * V);
    *theta = tsum / (3.0 * V);
}

/* Delta(x) per site, written as V blocks of 9 complex (for tests). */
void oracle_divergence_field(const cplx *U, const int d[4], int gauge, cplx *out)
{
    long V = volume(d);
    for (long s = 0; s < V; s++) {
        mat3 D = divergence(U, d, gauge, s);
        for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) out[s * 9 + 3 * i + j] = D.m[i][j];
    }
}

/* ------------------------------------------------------------------ */
/* local maximisation: eqs. (4)-(6) and overrelaxation                 */
/* ------------------------------------------------------------------ */

/* K(x) of eq. (5) with g = 1 on the neighbours (the field carries all gauge
 * transformations applied so far): sum_mu [U_mu(x) + U_mu(x - mu)^dagger]. */
void oracle_staple(const cplx *U, const int d[4], int gauge, long s, cplx *K_out)
{
    mat3 K = mat_zero();
    for (int mu = 0; mu < ndirs(gauge); mu++) {
        mat3 back = mat_dag(clink(U, neighbour(d, s, mu, -1), mu));
        mat_acc(&K, clink(U, s, mu), +1.0);
        mat_acc(&K, &back, +1.0);
    }
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) K_out[3 * i + j] = K.m[i][j];
}

/* SU(2) elements as quaternions (q0, q1, q2, q3) <->
 *     [[q0 + i q3,  q2 + i q1],
 *      [-q2 + i q1, q0 - i q3]].
 * The quaternion part of a 2x2 block k has
 *   b0 = Re(k00 + k11)/2, b1 = Im(k01 + k10)/2,
 *   b2 = Re(k01 - k10)/2, b3 = Im(k00 - k11)/2;
 * the rest of k does not contribute to Re Tr[g k] for any g in SU(2).
 *
 * Local solution, eq. (6): g = q^dagger (det q^dagger)^(-1/2) with q the
 * quaternion part, det q = |b|^2. Then the overrelaxed g^omega (exact
 * principal power). Result written to out[4]. */
void oracle_su2_solve(const double b[4], double omega, double out[4])
{
    double det = b[0] * b[0] + b[1] * b[1] + b[2] * b[2] + b[3] * b[3];
    if (det == 0.0) {               /* K block has no SU(2) part: keep links */
        out[0] = 1; out[1] = out[2] = out[3] = 0;
        return;
    }
    double nrm = sqrt(det);
    /* q^dagger / sqrt(det q^dagger): the conjugate quaternion, normalised */
    double g0 = b[0] / nrm, g1 = -b[1] / nrm, g2 = -b[2] / nrm, g3 = -b[3] / nrm;
    double vlen = sqrt(g1 * g1 + g2 * g2 + g3 * g3);
    double phi = atan2(vlen, g0);   /* g = (cos phi, n sin phi), phi in [0, pi] */
    double n1, n2, n3;
    if (vlen > 0) { n1 = g1 / vlen; n2 = g2 / vlen; n3 = g3 / vlen; }
    else { n1 = 0; n2 = 0; n3 = 1; }  /* g = +1 (phi = 0) or g = -1 (phi = pi) */
    out[0] = cos(omega * phi);
    out[1] = n1 * sin(omega * phi);
    out[2] = n2 * sin(omega * phi);
    out[3] = n3 * sin(omega * phi);
}

static const int SUBGROUP[3][2] = {{0, 1}, {0, 2}, {1, 2}};

/* One SU(2)-subgroup step at site s: find g in the subgroup acting on rows
 * and columns (a, b), over-relax it, and apply it to the eight links that
 * touch s: U_mu(x) <- G U_mu(x), U_mu(x - mu) <- U_mu(x - mu) G^dagger,
 * for all four mu (in both gauges). */
void oracle_subgroup_update(cplx *U, const int d[4], int gauge, long s, int sub, double omega)
{
    int a = SUBGROUP[sub][0], b = SUBGROUP[sub][1];
    cplx K[9];
    oracle_staple(U, d, gauge, s, K);
    cplx kaa = K[3 * a + a], kab = K[3 * a + b], kba = K[3 * b + a], kbb = K[3 * b + b];
    double q[4] = {creal(kaa + kbb) / 2, cimag(kab + kba) / 2, creal(kab - kba) / 2, cimag(kaa - kbb) / 2};
    double g[4];
    oracle_su2_solve(q, omega, g);

    mat3 G = mat_unit();
    G.m[a][a] = g[0] + I * g[3];
    G.m[a][b] = g[2] + I * g[1];
    G.m[b][a] = -g[2] + I * g[1];
    G.m[b][b] = g[0] - I * g[3];
    mat3 Gd = mat_dag(&G);

    for (int mu = 0; mu < 4; mu++) {
        mat3 *f = link(U, s, mu);
        *f = mat_mul(&G, f);
        mat3 *bk = link(U, neighbour(d, s, mu, -1), mu);
        *bk = mat_mul(bk, &Gd);
    }
}

void oracle_site_update(cplx *U, const int d[4], int gauge, long s, double omega)
{
    for (int sub = 0; sub < 3; sub++) oracle_subgroup_update(U, d, gauge, s, sub, omega);
}

/* Alg. 1, inner loops for one site parity: every site of that parity. The
 * order does not matter: a site reads and writes only the eight links
 * U_mu(x), U_mu(x - mu) that touch it, and no two sites of one parity touch
 * the same link, so the sites may also be shared among threads (OpenMP,
 * when built with it) with a result that does not depend on their number. */
void oracle_half_sweep(cplx *U, const int d[4], int gauge, int parity, double omega)
{
    long V = volume(d);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++)
        if (parity_of(d, s) == parity) oracle_site_update(U, d, gauge, s, omega);
}

/* Threads used by oracle_half_sweep (1 when built without OpenMP). n <= 0
 * leaves the current setting. Returns the number in effect. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Same, but visiting the sites of that parity in a caller-given order
 * (order[] lists site indices; entries of the other parity are skipped). */
void oracle_half_sweep_order(cplx *U, const int d[4], int gauge, int parity, double omega,
                             const long *order, long n)
{
    for (long k = 0; k < n; k++)
        if (parity_of(d, order[k]) == parity) oracle_site_update(U, d, gauge, order[k], omega);
}

/* ------------------------------------------------------------------ */
/* reunitarisation                                                     */
/* ------------------------------------------------------------------ */

static void reunit(mat3 *u)
{
    cplx *r0 = u->m[0], *r1 = u->m[1], *r2 = u->m[2];
    double n0 = sqrt(creal(r0[0] * conj(r0[0]) + r0[1] * conj(r0[1]) + r0[2] * conj(r0[2])));
    for (int j = 0; j < 3; j++) r0[j] /= n0;
    cplx p = conj(r0[0]) * r1[0] + conj(r0[1]) * r1[1] + conj(r0[2]) * r1[2];
    for (int j = 0; j < 3; j++) r1[j] -= p * r0[j];
    double n1 = sqrt(creal(r1[0] * conj(r1[0]) + r1[1] * conj(r1[1]) + r1[2] * conj(r1[2])));
    for (int j = 0; j < 3; j++) r1[j] /= n1;
    r2[0] = conj(r0[1] * r1[2] - r0[2] * r1[1]);
    r2[1] = conj(r0[2] * r1[0] - r0[0] * r1[2]);
    r2[2] = conj(r0[0] * r1[1] - r0[1] * r1[0]);
}

void oracle_reunit(cplx *U, long nlinks)
{
    for (long l = 0; l < nlinks; l++) reunit((mat3 *)(U + l * 9));
}

/* ------------------------------------------------------------------ */
/* Alg. 1 driver                                                       */
/* ------------------------------------------------------------------ */

/* One iteration of Alg. 1: even sites, then odd sites. */
void oracle_sweep(cplx *U, const int d[4], int gauge, double omega)
{
    oracle_half_sweep(U, d, gauge, 0, omega);
    oracle_half_sweep(U, d, gauge, 1, omega);
}

/* Alg. 1: compute F, theta; while theta >= eps (and fewer than max_iter
 * sweeps): sweep; reunitarise all links after every sweep whose global index
 * (start_sweep + sweeps done, counted from 1) is a multiple of reunit_every
 * (0 = never); recompute F, theta every check_every sweeps and after the
 * last allowed sweep. Returns 1 if theta < eps at exit, else 0. */
int oracle_fix(cplx *U, const int d[4], int gauge, double omega, double eps, int max_iter,
               int reunit_every, int check_every, long start_sweep,
               int *iters, double *F, double *theta)
{
    if (check_every < 1) check_every = 1;
    long V = volume(d);
    oracle_quality(U, d, gauge, F, theta);
    int it = 0, fresh = 1;
    while (it < max_iter) {
        if (fresh && *theta < eps) break;
        oracle_sweep(U, d, gauge, omega);
        it++;
        if (reunit_every > 0 && (start_sweep + it) % reunit_every == 0) oracle_reunit(U, 4 * V);
        fresh = (it % check_every == 0) || it == max_iter;
        if (fresh) oracle_quality(U, d, gauge, F, theta);
    }
    *iters = it;
    return *theta < eps;
}
