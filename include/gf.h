/*
 * gf.h -- C ABI of libgf, an MI355X (gfx950) library for Landau and Coulomb
 * gauge fixing of SU(3) lattice gauge fields by checkerboard overrelaxation.
 *
 * Method: N. Cardoso, "Coulomb and Landau Gauge Fixing in GPUs using CUDA and
 * MILC", Lattice 2014 (arXiv:1412.1498). The functional F_U[g] of eq. (1) is
 * maximised site by site: at each site the staple K(x) of eq. (5) is built,
 * the local SU(2) problem of eq. (6) is solved in each of the three SU(2)
 * subgroups of SU(3), the solution g is over-relaxed to g^omega and applied
 * to the eight links touching the site (Alg. 1). The quality theta of
 * eqs. (2)-(3) gates convergence.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Lattice dims are {nx, ny, nz, nt}; every dim must be even and >= 2.
 *   Directions mu = 0,1,2,3 run along x,y,z,t; boundaries are periodic.
 * - Site parity p = (x + y + z + t) mod 2; even sites (p = 0) are updated
 *   first in each sweep.
 * - Landau gauge uses mu = 0..3 in F, K and theta; Coulomb uses mu = 0..2
 *   (t is the temporal direction), but g(x) still rotates the temporal
 *   links. F is normalised by the number d of directions it sums (4 or 3), so
 *   F = 1 for the unit field. theta uses Delta(x) literally as in eq. (3):
 *   A = M - M^dagger, M = sum_nu [U_nu(x - nu) - U_nu(x)], minus (Tr A/3) 1.
 * - g^omega is the exact principal power of the SU(2) solution; subgroups
 *   are visited in the order (0,1), (0,2), (1,2).
 * - Precision: GF_F64 stores and updates links in double. GF_F32 stores and
 *   updates links in float, while the staple sums, the SU(2) solve with its
 *   power, reunitarisation and the F/theta reductions run in double (the
 *   8-real float form decodes and encodes links in float, with the hardware
 *   reciprocal and square root).
 * - Field pointers (U) are caller-owned DEVICE pointers, at least 16-byte
 *   aligned (GF_EINVAL otherwise; a torch tensor's data_ptr() is 256-byte
 *   aligned), in the internal layout below. The library never allocates,
 *   frees or keeps them beyond a call.
 * - Internal link layout. As in the paper's implementation section, sites
 *   are split by parity p = (x + y + z + t) mod 2 and numbered within a
 *   parity by h = (x + nx(y + ny(z + nz t))) / 2. The sites of one parity are
 *   grouped in blocks of 64 consecutive h; a block holds, for mu = 0..3 and
 *   each stored complex element e = 3 row + col, the 64 values of that element
 *   contiguously. The complex element e of U_mu at site (p, h) sits at
 *       (((p * nb + h / 64) * 4 + mu) * ne + e) * 64 + h % 64
 *   (units of one complex: float2 for F32, double2 for F64), with
 *   nb = ceil(V / 128) blocks per parity and ne = 9 (18-real storage) or 6
 *   (12-real storage, gf_params.storage = GF_STORE_12: rows 0 and 1 only, row
 *   2 rebuilt as conj(row0 x row1)) or 4 (8-real storage, GF_STORE_8:
 *   e = 0, 1, 2 hold U01, U02, U10 and e = 3 holds the pair (phase code of
 *   U00, phase code of U20), where the code of z with w = z/|z| is
 *   t = Im w / (1 + |Re w|) if Re w >= 0, else 2 - t (t >= 0) or -2 - t
 *   (t < 0), and 4 for z = 0; the rest follows from unitarity and det U = 1:
 *   |U00|^2 = 1 - n2, |U20|^2 = n2 - |U10|^2 with n2 = |U01|^2 + |U02|^2,
 *   U11 = -(conj(U00) U01 U10 + conj(U02) conj(U20)) / n2,
 *   U12 = (conj(U01) conj(U20) - conj(U00) U02 U10) / n2,
 *   U21 = -conj(U00 U12 - U02 U10), U22 = conj(U00 U11 - U01 U10); for a
 *   link with U01 = U02 = 0 exactly (then U10 = U20 = 0) e = 2 holds U11
 *   and the second code is that of U12, |U12|^2 = 1 - |U11|^2,
 *   U21 = -conj(U00 U12), U22 = conj(U00 U11)). The last block of a parity
 *   is padded.
 * - SU(N): a single-lattice context may also hold N = 2 or 4 colours (the
 *   paper's method for general N: all N(N-1)/2 SU(2) subgroups (a, b), a < b,
 *   in lexicographic order). Its links are full N x N matrices in the same
 *   layout with ne = N * N and e = N row + col; reunitarisation is
 *   Gram-Schmidt of rows 0..N-2 with the last row the complex conjugate of
 *   its cofactors; Delta(x) subtracts Tr A / N and F, theta are normalised by
 *   N. The su(3)-algebra entry points (gf_pack_alg, gf_unpack_alg,
 *   gf_functional, gf_functional_grad, gf_gauge_transform, gf_sd_step,
 *   gf_sd_fix) return GF_EUNSUPPORTED for N != 3; ensembles are SU(3).
 * - Canonical layout (pack/unpack only): [t][z][y][x][mu][row][col] complex
 *   in the context's precision (N x N per link).
 * - All work is enqueued on the context's HIP stream (the stream handle passed
 *   at creation; NULL = the default stream). Functions that return results to
 *   the host synchronise that stream; the others are asynchronous.
 * - Status codes: negative values are errors; no exception or abort crosses
 *   this ABI. After an error, gf_last_error() describes it.
 * - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GF_OK 0
#define GF_NOT_CONVERGED 1  /* informational: max_iter reached with theta >= eps */
#define GF_EINVAL (-1)      /* invalid argument; nothing was enqueued */
#define GF_ENOMEM (-2)      /* device or pinned host allocation failed */
#define GF_EDEVICE (-3)     /* a HIP call failed; gf_last_error() has its message */
#define GF_ENONFINITE (-4)  /* F or theta came out NaN or infinite */
#define GF_EUNSUPPORTED (-5)/* e.g. nc not in {2, 3, 4}; an SU(3)-only call on another N */

enum gf_gauge { GF_LANDAU = 0, GF_COULOMB = 1 };
enum gf_prec { GF_F64 = 0, GF_F32 = 1 };
enum gf_storage { GF_STORE_18 = 0, GF_STORE_12 = 1, GF_STORE_8 = 2 };

typedef struct gf_ctx gf_ctx;

/* Tunables and driver options. Zero-initialise or call gf_params_default. */
typedef struct gf_params {
    int check_every;        /* sweeps between F/theta evaluations in the fix
                               drivers (>= 1); default 1 */
    int reunit_every;       /* reunitarise every link after each sweep whose
                               global index is a multiple of this; 0 = never.
                               Default 20 (F64) / 10 (F32). Fused into the odd
                               half-sweep, so it costs no extra memory traffic */
    long long start_sweep;  /* global index of the last sweep already done
                               (sets the reunitarisation phase on resume) */
    int storage;            /* GF_STORE_18 (default), GF_STORE_12 or GF_STORE_8 */
    int lanes_per_site;     /* 0 = default (1; 2 for SU(4) and double SU(2)),
                               else 1, 2, 4 or 8 lanes per site (SU(4): >= 2) */
    int block_threads;      /* 0 = default, else 64, 128, 192 or 256 */
    int nontemporal;        /* 1 = streaming (non-temporal) link loads/stores,
                               0 = plain, -1 = default for the precision
                               (SU(2)/SU(4) kernels always stream) */
    int use_graph;          /* 1 = replay each check period as a hipGraph */
    int timing;             /* 1 = time every half-sweep with hipEvents */
    const char *log_path;   /* NULL = no log. Else the fix drivers (gf_fix,
                               gf_batch_fix, gf_sd_fix) append one JSON object
                               per line and per member at every F/theta
                               evaluation, the initial one included:
                               {"driver": "alg1" | "alg2", "call": k,
                                "member": i, "sweep" | "step": n, "F": F,
                                "theta": theta, "elapsed_s": s}, with k the
                               driver call's number in the context, n the
                               member's sweeps (Alg. 1) or steps (Alg. 2) so
                               far in that call and s the seconds since it
                               began. The context copies the path at creation
                               and opens the file (append) on first use;
                               flushed after every check. */
    int tile_order;         /* order in which a half-sweep's workgroups take
                               their tiles: 0 dispatch order, 1 XCD-contiguous
                               shares; -1 = default (0). Results do not depend
                               on it. */
} gf_params;

/* Fill *p with the defaults for precision prec. */
void gf_params_default(gf_params *p, int prec);

/* Create a context for one lattice. dims = {nx, ny, nz, nt}; nc is the
 * number of colours, 3, or 2 or 4 (SU(N) section above); gauge is GF_LANDAU
 * or GF_COULOMB; prec is GF_F64 or GF_F32; stream is a hipStream_t (NULL =
 * default stream); p may be NULL for defaults.
 * Returns GF_EINVAL for odd or non-positive dims, a bad enum or schedule,
 * GF_EUNSUPPORTED for nc not in {2, 3, 4} or 12-/8-real storage with nc != 3,
 * GF_ENOMEM / GF_EDEVICE on allocation failure (then *out is NULL). On
 * success the context owns its reduction scratch. */
int gf_create(gf_ctx **out, const int dims[4], int nc, int gauge, int prec, void *stream,
              const gf_params *p);

/* Create a context for an ensemble of n lattices fixed together (each with
 * its own dims[4*i..4*i+3] and gauge[i]; common precision and storage).
 * The single-lattice entry points require n == 1; the gf_batch_* ones
 * accept any n >= 1. */
int gf_batch_create(gf_ctx **out, int n, const int *dims, const int *gauge, int prec, void *stream,
                    const gf_params *p);

/* Release a context (waits for its stream, closes its log). NULL is
 * accepted. gf_batch_destroy is the same call under the ensemble's name:
 * single lattices and ensembles share the context type. */
int gf_destroy(gf_ctx *ctx);
int gf_batch_destroy(gf_ctx *ctx);

/* Human-readable description of the last error on ctx ("" if none); with
 * ctx = NULL, that of the last failed context-free call (gf_quality_noalloc)
 * on the calling thread. */
const char *gf_last_error(const gf_ctx *ctx);

/* Bytes of one field of member i in the internal layout:
 * 2 * nb * 4 * ne * 64 * sizeof(complex) (padding included). Members of an
 * ensemble differ in size, hence the member index; 0 for a single lattice.
 * Returns 0 for a NULL context or a member out of range. */
size_t gf_field_bytes(const gf_ctx *ctx, int member);

/* Convert member 0's field between the canonical layout U_aos (device) and
 * the internal layout U (device). 12-real storage drops row 2 on pack and
 * rebuilds it on unpack. Asynchronous. */
int gf_pack(gf_ctx *ctx, const void *U_aos, void *U);
int gf_unpack(gf_ctx *ctx, const void *U, void *U_aos);

/* One half-sweep of Alg. 1 (all sites of one parity, three subgroups each,
 * over-relaxation parameter omega in (0, 2)) on member 0. No
 * reunitarisation, no sweep counter change. Asynchronous. */
int gf_sweep(gf_ctx *ctx, void *U, int parity, double omega);

/* nsweeps full sweeps (even then odd half-sweep) on member 0, reunitarising
 * on the schedule of gf_params.reunit_every and advancing the context's
 * sweep counter. Asynchronous. */
int gf_sweeps(gf_ctx *ctx, void *U, double omega, int nsweeps);

/* Reunitarise every link of member 0 (Gram-Schmidt on rows 0, 1 in double,
 * row 2 = conj(row0 x row1)). Asynchronous. */
int gf_reunit(gf_ctx *ctx, void *U);

/* F (eq. 1, on the current field) and theta (eq. 2) of member 0, reduced in
 * double in a fixed order (bitwise reproducible for a given field).
 * Synchronises the stream. Returns GF_ENONFINITE if either is NaN or Inf. */
int gf_quality(gf_ctx *ctx, const void *U, double *F, double *theta);

/* Per time slice t = 0 .. nt-1 of member 0 (SU(3)): F_t and theta_t, the
 * sums of eqs. (1)-(2) over the nx ny nz sites of slice t normalised by
 * that slice volume (F_t by d N_c V_t, theta_t by N_c V_t), so that the mean
 * over t of theta_t is theta and that of F_t is F. For the Coulomb gauge
 * (Delta from the spatial links, one global theta gating convergence) this
 * is the per-slice diagnostic; it is defined for Landau too. F_t and theta_t
 * are host arrays of nt doubles. The first call allocates
 * 2 nt ceil(nx ny nz / 256) + 2 nt doubles of scratch (kept by the context).
 * Synchronises. GF_ENONFINITE if a value is NaN or Inf. */
int gf_quality_slices(gf_ctx *ctx, const void *U, double *F_t, double *theta_t);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): F and
 * theta of gf_quality for one SU(3) lattice without a context and without
 * any allocation. U is a field of the given dims, gauge, precision and
 * storage (GF_STORE_*) in the internal layout; out is a caller-owned DEVICE
 * array of 2 doubles receiving {F, theta}, bitwise those gf_quality returns
 * for the same field. Runs on the current device, asynchronously on stream
 * (a hipStream_t of that device; NULL = default stream), with no host
 * synchronisation and no allocating call (hipMalloc, hipFree, pinned
 * memory), so it may be captured into a graph. Its reduction scratch is a
 * fixed device array of the library (1 MiB per GPU, held until the process
 * ends), which limits the lattice to V <= 2^24 sites (65536 tiles of 256
 * sites; 48^3 x 96 fits): larger lattices return GF_EINVAL before any
 * device work, as do bad dims, gauge, precision, storage or pointers;
 * gf_last_error(NULL) then says why. All calls on one GPU share that array:
 * calls that may overlap in time on one GPU (several streams or threads)
 * race on it and must be ordered by the caller. */
int gf_quality_noalloc(const void *U, const int dims[4], int gauge, int prec, int storage, void *stream,
                       double *out);

/* Alg. 1 on member 0: compute F, theta; while theta >= eps and fewer than
 * max_iter sweeps were done: sweep (with scheduled reunitarisation) and
 * recompute F, theta every check_every sweeps and after the last allowed
 * sweep. *iters = sweeps done (0 if the initial theta < eps). Returns GF_OK
 * if theta < eps, GF_NOT_CONVERGED if max_iter was reached, or an error. */
int gf_fix(gf_ctx *ctx, void *U, double omega, double eps, int max_iter, int *iters, double *F,
           double *theta);

/* Alg. 1 on every member of an ensemble at once. U[i] is member i's field,
 * omega[i] its over-relaxation parameter. Each member stops sweeping as soon
 * as its own theta < eps at a check; results are bitwise those of gf_fix on
 * the member alone with the same parameters and schedule. iters, F, theta
 * are arrays of n. Returns GF_OK if every member converged, else
 * GF_NOT_CONVERGED (or an error). */
int gf_batch_fix(gf_ctx *ctx, void *const *U, const double *omega, double eps, int max_iter,
                 int *iters, double *F, double *theta);

/* F and theta of every member (arrays of n). Synchronises. */
int gf_batch_quality(gf_ctx *ctx, void *const *U, double *F, double *theta);

/* Time the candidate schedules (lanes per site, workgroup size,
 * non-temporal access, and for a single lattice the tile order) on a scratch copy of the members' fields U[i] and
 * keep the fastest in ctx. Every schedule gives bitwise the same links. If
 * cache_path is not NULL, a previous result for the same device, library
 * sources, colour number, precision, storage and lattice list is reused and
 * new results are appended. The context itself (single lattice or
 * ensemble) is the first argument, and the fields to time on and omega are
 * passed explicitly, because the timing runs real half-sweeps. Allocates
 * (and frees) a scratch copy of the fields. Synchronises. */
int gf_autotune(gf_ctx *ctx, void *const *U, double omega, const char *cache_path);

/* The schedule in use: lanes per site, workgroup threads, the
 * non-temporal flag and the tile order (NULL outputs are skipped). */
int gf_get_schedule(const gf_ctx *ctx, int *lanes_per_site, int *block_threads, int *nontemporal,
                    int *tile_order);

/* Total device time (ms) and number of the half-sweep launches timed since
 * the last call (needs gf_params.timing = 1). Synchronises. */
int gf_timing(gf_ctx *ctx, double *ms, long long *launches);

/* Set / read the global sweep counter (reunitarisation phase). */
int gf_set_sweep_count(gf_ctx *ctx, long long sweeps_done);
long long gf_get_sweep_count(const gf_ctx *ctx);

/* ---- differentiation: F as a function of a gauge transformation ------
 * g(x) = exp(S(x)), S(x) = i sum_a s_a(x) lambda_a / 2 (Gell-Mann lambda_a,
 * Tr lambda_a lambda_b = 2 delta_ab). s (and a gradient) is a DEVICE array
 * of 8 * 2 * nb * 64 reals of the context precision in the links' blocking:
 * component a (generator lambda_{a+1}) of site (p, h) at
 *     ((p * nb + h / 64) * 8 + a) * 64 + h % 64,
 * nb = ceil(V / 128) as for the links; the padding of a parity's last block
 * is neither read nor written. */

/* Convert s between the canonical layout [t][z][y][x][a] and the internal
 * one above. */
int gf_pack_alg(gf_ctx *ctx, const void *s_aos, void *s);
int gf_unpack_alg(gf_ctx *ctx, const void *s, void *s_aos);

/* F_U[g] of eq. (1) for g = exp(S(s)) (U itself is not modified).
 * Synchronises. */
int gf_functional(gf_ctx *ctx, const void *U, const void *s, double *F);

/* grad = dF * dF_U[g]/ds_a(x) at s, in the layout of s: the su(3)-valued
 * gradient of eq. (1) with respect to the gauge transformation.
 * Asynchronous. */
int gf_functional_grad(gf_ctx *ctx, const void *U, const void *s, double dF, void *grad);

/* Apply g = exp(S(s)): U_mu(x) <- g(x) U_mu(x) g(x + mu)^dagger for all mu.
 * Asynchronous. */
int gf_gauge_transform(gf_ctx *ctx, void *U, const void *s);

/* ---- steepest descent with Fourier acceleration (Alg. 2, eqs. 7-9) -----
 * One step on member 0: Delta(x) (eq. 3, the argument of eq. 7) is split
 * into its 8 real su(3) components, Fourier transformed over the lattice (4D
 * for Landau, 3D over x, y, z per time slice for Coulomb), multiplied by
 * p^2_max / p^2 with p^2 = sum 4 sin^2(pi k / L) over the transformed axes
 * (zero mode dropped), transformed back, and g(x) = reunit(1 + (alpha/2) X)
 * (first-order exponential, Gram-Schmidt) is applied to every link. The
 * transforms are the library's own (one pass per axis, in LDS); nx must be
 * at most 384 and ny, nz, nt at most 1024 (GF_EUNSUPPORTED otherwise, before
 * any device work). The first call allocates about 1.5x a field of scratch (kept
 * by the context). Asynchronous. alpha must be > 0 (0.08 in the paper). */
int gf_sd_step(gf_ctx *ctx, void *U, double alpha);

/* Alg. 2: F, theta; while theta >= eps and fewer than max_iter steps: steps,
 * with F, theta every check_every steps. Returns GF_OK / GF_NOT_CONVERGED. */
int gf_sd_fix(gf_ctx *ctx, void *U, double alpha, double eps, int max_iter, int *iters, double *F,
              double *theta);

/* ---- host-only checks (no device use) -----------------------------------
 * The SU(2) step of the sweep kernels evaluated on the host with the same
 * code: b = quaternion part (b0, b1, b2, b3) of a staple block, omega the
 * over-relaxation parameter; r receives g^omega as a quaternion (see the
 * conventions above). */
void gf_host_su2_step(const double b[4], double omega, double r[4]);

/* The kernels' own double-precision sine/cosine (valid for x in [0, 2 pi])
 * and arctangent: out = {sin x, cos x, atan2(y, x)}. */
void gf_host_trig(double x, double y, double out[3]);

/* The 8-real storage round trip on the host with the kernels' code: in is a
 * 3x3 complex matrix as 18 doubles (re, im of element 3 row + col); in
 * precision prec (GF_F32 first rounds it to float) it is compressed to the
 * 8 stored reals (written to stored) and reconstructed (written to out).
 * Returns GF_EINVAL for NULL pointers or a bad precision. */
int gf_host_link8(int prec, const double in[18], double stored[8], double out[18]);

/* Index check: complex offsets of element 0 of the eight links (18-real
 * storage) that the site (parity, h) of a dims lattice updates in a
 * half-sweep: out[0..3] = U_mu(x), out[4..7] = U_mu(x - mu). Returns
 * GF_EINVAL for bad arguments. */
int gf_site_links(const int dims[4], int parity, long long h, long long out[8]);

#ifdef __cplusplus
}
#endif

#endif /* GF_H */
