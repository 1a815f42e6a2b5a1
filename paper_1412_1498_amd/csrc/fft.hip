// fft.hip -- steepest descent with Fourier acceleration (Alg. 2, eqs. 7-9) on
// gfx950: Delta of eq. (3) as its eight real su(3) components, their lattice
// Fourier transform, the p2_max / p^2(k) filter, the inverse transform, and
// the step's gauge transformation g = reunit(1 + X) as a g field for
// k_gauge_transform.
//
// The components' spectrum is held as spec[t][a][z][y][kx] with kx = 0..nx/2
// (the real transform along x keeps half the spectrum, the other half being
// its complex conjugate). One pass per axis: x (real <-> half complex), with
// Delta computed in the forward x pass and g formed in the inverse one, so
// the components never go to memory in lattice space; then y, z and t
// (complex, in place). The multiplication by p2_max / p^2(k) is fused into
// the last forward pass, between its forward and inverse transform, so that
// pass writes back the filtered field already transformed back along its own
// axis.
//
// A workgroup loads a tile of pencils (for y, z, t: consecutive kx of one row,
// so every global access is a contiguous run) into LDS and transforms them by
// the mixed-radix Stockham algorithm (radix 4, 2, 3, 5 butterflies in
// registers, any larger prime by a direct sum), in place: one LDS read, one
// write and one twiddle per point and pass. The arithmetic is in double for
// both link precisions (a double FMA costs the same as a float one on this
// GPU); the spectrum is stored in the context precision between passes.
#include "fft.hpp"
#include "su3_device.hpp"
#include "tile_order.hpp"

namespace gf {

namespace {

// 16-byte aligned so that a value moves to and from LDS as one 128-bit
// access: as two 64-bit halves, consecutive lanes' values fell into the same
// banks and every LDS instruction of the transforms stalled on conflicts.
struct alignas(16) Cd {
    double x, y;
};

__device__ __forceinline__ Cd cmul(Cd a, Cd b) {
    Cd r;
    r.x = fma(a.x, b.x, -a.y * b.y);
    r.y = fma(a.x, b.y, a.y * b.x);
    return r;
}

__device__ __forceinline__ void cmac(Cd &acc, Cd a, Cd b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

// LDS of a transform tile: one buffer holding element j of pencil q at
// a[j * ld + q] (ld >= np pencils; the x transforms pad it so that a pencil's
// consecutive elements fall in different banks), transformed in place, and
// the n roots exp(2 pi i m / n).
struct Tile {
    Cd *a, *Wl;
    int ld;
    FastDiv dnp;  // division by the pencil count
};

__host__ __device__ inline int tile_lds_points(int n, int ld) { return n * ld + n; }

__device__ __forceinline__ Tile tile_setup(Cd *lds, const Cd *__restrict__ Wg, int n, int ld, const FastDiv &dnp) {
    Tile t;
    t.a = lds;
    t.ld = ld;
    t.dnp = dnp;
    t.Wl = lds + n * ld;
    return t;
}

// The n roots into the tile: called after the tile's own loads are issued,
// so their latency overlaps those instead of preceding them (lds_dft begins
// with a barrier).
__device__ __forceinline__ void load_roots(const Tile &t, const Cd *__restrict__ Wg, int n) {
    for (int m = threadIdx.x; m < n; m += blockDim.x) t.Wl[m] = Wg[m];
}

// w or its conjugate: the table holds exp(+2 pi i m / n); SIGN = -1 forward.
template <int SIGN>
__device__ __forceinline__ Cd root(Cd w) {
    if constexpr (SIGN < 0) w.y = -w.y;
    return w;
}

__device__ __forceinline__ Cd cadd(Cd a, Cd b) { return Cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ Cd csub(Cd a, Cd b) { return Cd{a.x - b.x, a.y - b.y}; }
// i s z for s = +-1
template <int S>
__device__ __forceinline__ Cd imul(Cd z) { return S > 0 ? Cd{-z.y, z.x} : Cd{z.y, -z.x}; }

// In-register R-point DFTs, X_s = sum_m v_m exp(SIGN 2 pi i m s / R).
template <int SIGN>
__device__ __forceinline__ void bfly2(Cd *v) {
    const Cd a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int SIGN>
__device__ __forceinline__ void bfly4(Cd *v) {
    const Cd t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const Cd t2 = cadd(v[1], v[3]), t3 = imul<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <int SIGN>
__device__ __forceinline__ void bfly3(Cd *v) {
    const double h = 0.86602540378443864676;  // sin(2 pi / 3)
    const Cd s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const Cd t = Cd{v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y};
    const Cd u = imul<SIGN>(Cd{h * d.x, h * d.y});
    v[0] = cadd(v[0], s);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
}

template <int SIGN>
__device__ __forceinline__ void bfly5(Cd *v) {
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;  // cos(2 pi/5), cos(4 pi/5)
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;   // sin(2 pi/5), sin(4 pi/5)
    const Cd a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const Cd a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const Cd p = Cd{v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    const Cd r = Cd{v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    const Cd u = imul<SIGN>(Cd{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    const Cd w = imul<SIGN>(Cd{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(p, u);
    v[4] = csub(p, u);
    v[2] = cadd(r, w);
    v[3] = csub(r, w);
}

// Butterflies per thread in a radix-R pass: a tile holds at most
// FFT_TILE_POINTS points, i.e. FFT_TILE_POINTS / R butterflies, over
// FFT_BLOCK threads; outputs per thread in a pass of any other radix.
constexpr int pass_b(int R) { return (FFT_TILE_POINTS / R + FFT_BLOCK - 1) / FFT_BLOCK; }
constexpr int PASS_OUT = (FFT_TILE_POINTS + FFT_BLOCK - 1) / FFT_BLOCK;
// Global loads per thread when a tile is filled (all issued before the first
// use, so a workgroup waits for one memory latency, not one per element).
constexpr int LOAD_C = (FFT_TILE_POINTS + FFT_BLOCK - 1) / FFT_BLOCK;

// One radix-R pass of the Stockham autosort algorithm over np pencils (element
// j of pencil q at [j * ld + q]), in place: Ns = product of the earlier
// radices; butterfly j reads j + r n/R, twiddles by
// exp(SIGN 2 pi i r (j mod Ns) / (Ns R)), and writes (j / Ns) Ns R + (j mod Ns) + r Ns.
// Every thread reads all its butterflies into registers before the barrier
// and writes them after it.
template <int SIGN, int R>
__device__ __forceinline__ void stockham_pass(Cd *buf, const Cd *Wl, int n, int Ns, int np, int ld,
                                              const FastDiv &dnp, const FastDiv &dns) {
    constexpr int B = pass_b(R);
    const int nb = n / R, tw = n / (Ns * R), total = nb * np;
    Cd v[B][R];
#pragma unroll
    for (int i = 0; i < B; i++) {
        const int bi = threadIdx.x + i * FFT_BLOCK;
        if (bi < total) {
            const int j = (int)fdiv((unsigned)bi, dnp), q = bi - j * np;
            const int k = j - (int)fdiv((unsigned)j, dns) * Ns;
#pragma unroll
            for (int r = 0; r < R; r++) v[i][r] = buf[(j + r * nb) * ld + q];
#pragma unroll
            for (int r = 1; r < R; r++) v[i][r] = cmul(v[i][r], root<SIGN>(Wl[r * k * tw]));
            if constexpr (R == 2) bfly2<SIGN>(v[i]);
            if constexpr (R == 3) bfly3<SIGN>(v[i]);
            if constexpr (R == 4) bfly4<SIGN>(v[i]);
            if constexpr (R == 5) bfly5<SIGN>(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < B; i++) {
        const int bi = threadIdx.x + i * FFT_BLOCK;
        if (bi < total) {
            const int j = (int)fdiv((unsigned)bi, dnp), q = bi - j * np;
            const int jh = (int)fdiv((unsigned)j, dns), k = j - jh * Ns;
            const int d = jh * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; r++) buf[(d + r * Ns) * ld + q] = v[i][r];
        }
    }
}

// A pass of any radix R (the primes above 5), in place: one output per
// thread and slot, the R-point sum over the root table.
template <int SIGN>
__device__ __forceinline__ void stockham_pass_any(Cd *buf, const Cd *Wl, int n, int Ns, int R, int np, int ld) {
    const int nb = n / R, tw = n / (Ns * R), nR = n / R, total = n * np;
    Cd o[PASS_OUT];
#pragma unroll
    for (int i = 0; i < PASS_OUT; i++) {
        const int idx = threadIdx.x + i * FFT_BLOCK;
        if (idx < total) {
            const int q = idx % np, rest = idx / np, j = rest % nb, s = rest / nb, k = j % Ns;
            Cd acc = {0.0, 0.0};
            for (int r = 0; r < R; r++) {
                Cd x = buf[(j + r * nb) * ld + q];
                if (r) x = cmul(x, root<SIGN>(Wl[r * k * tw]));
                cmac(acc, x, root<SIGN>(Wl[((r * s) % R) * nR]));
            }
            o[i] = acc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PASS_OUT; i++) {
        const int idx = threadIdx.x + i * FFT_BLOCK;
        if (idx < total) {
            const int q = idx % np, rest = idx / np, j = rest % nb, s = rest / nb, k = j % Ns;
            buf[((j / Ns) * Ns * R + k + s * Ns) * ld + q] = o[i];
        }
    }
}

// DFT of np pencils of length n held in t.a, in place. Begins and ends with
// a barrier.
template <int SIGN>
__device__ __forceinline__ void lds_dft(const Tile &t, const FftPlan &pl, int n, int np) {
    int Ns = 1;
    for (int f = 0; f < pl.nf; f++) {
        __syncthreads();
        const int R = pl.fac[f];
        if (R == 4) stockham_pass<SIGN, 4>(t.a, t.Wl, n, Ns, np, t.ld, t.dnp, pl.ns[f]);
        else if (R == 2) stockham_pass<SIGN, 2>(t.a, t.Wl, n, Ns, np, t.ld, t.dnp, pl.ns[f]);
        else if (R == 3) stockham_pass<SIGN, 3>(t.a, t.Wl, n, Ns, np, t.ld, t.dnp, pl.ns[f]);
        else if (R == 5) stockham_pass<SIGN, 5>(t.a, t.Wl, n, Ns, np, t.ld, t.dnp, pl.ns[f]);
        else stockham_pass_any<SIGN>(t.a, t.Wl, n, Ns, R, np, t.ld);
        Ns *= R;
    }
    __syncthreads();
}

__device__ __forceinline__ double lattice_p2(int k, int L) {
    if (L <= 0) return 0.0;
    const double s = sinpi((double)k / (double)L);
    return 4.0 * s * s;
}

}  // namespace

// The transform kernels ask for four waves per SIMD (at most 128 VGPRs): a
// pass's butterflies fit in that without spilling, and a CU then holds four
// workgroups to overlap one tile's memory phase with another's passes.

namespace {

// Delta(x) of eq. (3) at site (p, h) as its eight real su(3) components
// o_a = Tr[lambda_a Delta] / (2i): M = sum_mu [U_mu(x - mu) - U_mu(x)] in
// double, A = M - M^dagger, whose traceless part is Delta (the trace part
// drops out of these traces, so only Im of the diagonal and the off-diagonal
// entries of A enter).
template <typename R, int NE>
__device__ __forceinline__ void delta_components(const Geom &g, int nd, const gchar *U, int p, int h, double o[8]) {
    const SiteNbr nb = site_neighbours(g, p, h);
    double mr[9], mi[9];
#pragma unroll
    for (int e = 0; e < 9; e++) { mr[e] = 0.0; mi[e] = 0.0; }
    for (int mu = 0; mu < nd; mu++) {
        Mat<R> f, b;
        load_link<R, NE, false>(f, U, link_off(g, mu, p, h));
        load_link<R, NE, false>(b, U, link_off(g, mu, 1 - p, pick4(nb.hb, mu)));
#pragma unroll
        for (int e = 0; e < 9; e++) {
            mr[e] += (double)b.re[e] - (double)f.re[e];
            mi[e] += (double)b.im[e] - (double)f.im[e];
        }
    }
    double ar[9], ai[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            ar[3 * r + c] = mr[3 * r + c] - mr[3 * c + r];
            ai[3 * r + c] = mi[3 * r + c] + mi[3 * c + r];
        }
    const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
    o[0] = 0.5 * (ai[3] + ai[1]);
    o[1] = 0.5 * (ar[1] - ar[3]);
    o[2] = 0.5 * (ai[0] - ai[4]);
    o[3] = 0.5 * (ai[6] + ai[2]);
    o[4] = 0.5 * (ar[2] - ar[6]);
    o[5] = 0.5 * (ai[7] + ai[5]);
    o[6] = 0.5 * (ar[5] - ar[7]);
    o[7] = 0.5 * r3 * (ai[0] + ai[4] - 2.0 * ai[8]);
}

// g = reunit(1 + i H), H = sum_a s_a lambda_a (the first-order exponential
// of the step, Gram-Schmidt), in double.
__device__ __forceinline__ void step_matrix(const double s[8], Mat<double> &m) {
    const double r3 = 0.57735026918962576451;
    double hr[9], hi[9];
    hr[0] = s[2] + r3 * s[7];  hi[0] = 0.0;
    hr[4] = -s[2] + r3 * s[7]; hi[4] = 0.0;
    hr[8] = -2.0 * r3 * s[7];  hi[8] = 0.0;
    hr[1] = s[0]; hi[1] = -s[1];
    hr[3] = s[0]; hi[3] = s[1];
    hr[2] = s[3]; hi[2] = -s[4];
    hr[6] = s[3]; hi[6] = s[4];
    hr[5] = s[5]; hi[5] = -s[6];
    hr[7] = s[5]; hi[7] = s[6];
#pragma unroll
    for (int e = 0; e < 9; e++) {
        m.re[e] = (e % 4 == 0 ? 1.0 : 0.0) - hi[e];
        m.im[e] = hr[e];
    }
    reunitarise(m);
}

// (t, z, y) of the site rows of a tile, and z ny + y (row index within a
// time slice), kept in LDS so each is divided out once.
struct RowInfo {
    int t, z, y, zy;
};

__device__ __forceinline__ void row_info(RowInfo *ri, const Geom &g, long long sr0, int ys, long long srows) {
    for (int yl = threadIdx.x; yl < ys; yl += blockDim.x) {
        const long long sr = sr0 + yl;
        RowInfo r = {0, 0, 0, -1};
        if (sr < srows) {
            const int q = (int)(sr / g.ny);
            r.y = (int)(sr - (long long)q * g.ny);
            r.t = q / g.nz;
            r.z = q - r.t * g.nz;
            r.zy = r.z * g.ny + r.y;
        }
        ri[yl] = r;
    }
}

// spec[t][a][z][y][kx] index of component a, kx of a site row
__device__ __forceinline__ long long spec_index(const Geom &g, int nkx, const RowInfo &r, int a, int k) {
    return (((long long)r.t * 8 + a) * g.nz * g.ny + r.zy) * nkx + k;
}

}  // namespace

// Delta and its forward real transform along x, for ys site rows (lines
// along x at fixed y, z, t; consecutive in (t, z, y)). The eight components of
// a site row travel as four complex rows, components 2c + i (2c + 1) in
// pencil 4 yl + c; after the transform A[k] = (Z[k] + conj Z[-k]) / 2 and
// B[k] = (Z[k] - conj Z[-k]) / 2i are the two components' spectra. A site
// row holds both parities, so a site's x-backward link is the other
// parity's forward link of the same tile and its y-backward link that of the
// previous row.
template <typename R, int NE>
__global__ void __launch_bounds__(FFT_BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_sd_delta_fx(Geom g, int nd, const typename V2<R>::type *__restrict__ Uv, FftSite f, const Cd *__restrict__ Wg,
              typename V2<R>::type *__restrict__ spec, SlabOrder so) {
    extern __shared__ Cd lds[];
    const int nx = g.nx, nc = 4 * f.ys;
    const Tile t = tile_setup(lds, Wg, nx, nc + 1, f.dnc);
    load_roots(t, Wg, nx);
    RowInfo *ri = (RowInfo *)(t.Wl + nx);
    // slab order over tiles of ys site rows: a time slice is ny nz rows, so
    // the rows holding the t-backward links were read ny nz / ys tiles
    // before, in the same column block
    const long long sr0 = (long long)slab_tile(xcd_tile(blockIdx.x, gridDim.x), so) * f.ys;
    row_info(ri, g, sr0, f.ys, f.srows);
    __syncthreads();
    const gchar *U = as_global((const void *)Uv);
    for (int idx = threadIdx.x; idx < f.ys * nx; idx += blockDim.x) {
        const int yl = (int)fdiv((unsigned)idx, f.dn), x = idx - yl * nx;
        const RowInfo r = ri[yl];
        double o[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (r.zy >= 0) {
            const int lx = x + nx * (int)(sr0 + yl);  // x + nx (y + ny (z + nz t))
            delta_components<R, NE>(g, nd, U, (x + r.y + r.z + r.t) & 1, lx >> 1, o);
        }
#pragma unroll
        for (int c = 0; c < 4; c++) t.a[x * t.ld + yl * 4 + c] = Cd{o[2 * c], o[2 * c + 1]};
    }
    lds_dft<-1>(t, f.pl, nx, nc);
    for (int idx = threadIdx.x; idx < 8 * f.ys * f.nkx; idx += blockDim.x) {
        const int row = (int)fdiv((unsigned)idx, f.dnkx), k = idx - row * f.nkx;
        const int yl = row >> 3, a = row & 7;
        const RowInfo r = ri[yl];
        if (r.zy < 0) continue;
        const int cr = yl * 4 + (a >> 1);
        const Cd zk = t.a[k * t.ld + cr], zm = t.a[((nx - k) % nx) * t.ld + cr];
        typename V2<R>::type v;
        if (a & 1) {  // (zk - conj zm) / 2i
            v.x = (R)(0.5 * (zk.y + zm.y));
            v.y = (R)(-0.5 * (zk.x - zm.x));
        } else {      // (zk + conj zm) / 2
            v.x = (R)(0.5 * (zk.x + zm.x));
            v.y = (R)(0.5 * (zk.y - zm.y));
        }
        spec[spec_index(g, f.nkx, r, a, k)] = v;
    }
}

// Inverse real transform along x of ys site rows' eight component spectra
// (the rest of each by conjugate symmetry; the imaginary parts at kx = 0 and
// nx/2 are dropped, as for any real inverse transform), components 2c and
// 2c + 1 travelling as Z = A + i B; then every site's step matrix
// g = reunit(1 + i sum_a s_a lambda_a), written as the g field (gfield_off).
template <typename R>
__global__ void __launch_bounds__(FFT_BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_sd_fx_gfield(Geom g, FftSite f, const Cd *__restrict__ Wg, const typename V2<R>::type *__restrict__ spec,
               typename V2<R>::type *__restrict__ gf) {
    extern __shared__ Cd lds[];
    const int nx = g.nx, nc = 4 * f.ys, h = nx / 2;
    const Tile t = tile_setup(lds, Wg, nx, nc + 1, f.dnc);
    RowInfo *ri = (RowInfo *)(t.Wl + nx);
    const long long sr0 = (long long)xcd_tile(blockIdx.x, gridDim.x) * f.ys;
    row_info(ri, g, sr0, f.ys, f.srows);
    __syncthreads();
    // Every lane loads unconditionally (a pair that does not exist reads
    // element 0 and is zeroed afterwards): loads under a branch made the
    // compiler copy each result at the branch's end, which waited for it, so
    // only two loads were ever in flight.
    typename V2<R>::type va[LOAD_C], vb[LOAD_C];
    bool ok[LOAD_C];
#pragma unroll
    for (int i = 0; i < LOAD_C; i++) {  // nc nkx <= FFT_TILE_POINTS (pencil, frequency) pairs
        const int idx = threadIdx.x + i * FFT_BLOCK;
        const bool in = idx < nc * f.nkx;
        const int cr = in ? (int)fdiv((unsigned)idx, f.dnkx) : 0, k = idx - cr * f.nkx;
        const RowInfo r = ri[cr >> 2];
        ok[i] = in && r.zy >= 0;
        const int a = 2 * (cr & 3);
        const long long ia = ok[i] ? spec_index(g, f.nkx, r, a, k) : 0;
        const long long ib = ok[i] ? spec_index(g, f.nkx, r, a + 1, k) : 0;
        va[i] = spec[ia];
        vb[i] = spec[ib];
    }
    load_roots(t, Wg, nx);
#pragma unroll
    for (int i = 0; i < LOAD_C; i++) {
        const int idx = threadIdx.x + i * FFT_BLOCK;
        if (idx >= nc * f.nkx) continue;
        const int cr = (int)fdiv((unsigned)idx, f.dnkx), k = idx - cr * f.nkx;
        const double z = ok[i] ? 1.0 : 0.0;
        const Cd A = Cd{z * (double)va[i].x, z * (double)va[i].y}, B = Cd{z * (double)vb[i].x, z * (double)vb[i].y};
        if (k == 0 || k == h) {
            t.a[k * t.ld + cr] = Cd{A.x, B.x};
        } else {
            t.a[k * t.ld + cr] = Cd{A.x - B.y, A.y + B.x};
            t.a[(nx - k) * t.ld + cr] = Cd{A.x + B.y, B.x - A.y};
        }
    }
    lds_dft<1>(t, f.pl, nx, nc);
    for (int idx = threadIdx.x; idx < f.ys * nx; idx += blockDim.x) {
        const int yl = (int)fdiv((unsigned)idx, f.dn), x = idx - yl * nx;
        const RowInfo r = ri[yl];
        if (r.zy < 0) continue;
        double sv[8];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const Cd z = t.a[x * t.ld + yl * 4 + c];
            sv[2 * c] = z.x;
            sv[2 * c + 1] = z.y;
        }
        Mat<double> m;
        step_matrix(sv, m);
        const int lx = x + nx * (int)(sr0 + yl);
        const long long o = gfield_off(g, (x + r.y + r.z + r.t) & 1, lx >> 1, 0);
#pragma unroll
        for (int e = 0; e < 9; e++) {
            typename V2<R>::type v;
            v.x = (R)m.re[e];
            v.y = (R)m.im[e];
            gf[o + (long long)e * BLK] = v;
        }
    }
}

// Complex transform along one of y, z, t, in place. A workgroup takes np
// consecutive kx of one row (outer index = the other three of t, a, z, y).
// FILTER: forward transform, multiply by scale p2max / p^2(k) (0 at p^2 = 0),
// inverse transform.
template <typename R, bool FILTER>
__global__ void __launch_bounds__(FFT_BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_fft_axis(FftAxis f, const Cd *__restrict__ Wg, typename V2<R>::type *__restrict__ spec, int sign) {
    extern __shared__ Cd lds[];
    const int n = f.n, np = f.np;
    const Tile t = tile_setup(lds, Wg, n, np, f.dnp);
    // XCD-contiguous tile order: neighbouring tiles (the kx chunks of a row,
    // then the next row) share cache lines and meet in one L2
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int chunk = tile % f.nchunk;
    int o = tile / f.nchunk;
    const int d0 = o % f.r[0];
    o /= f.r[0];
    const int d1 = o % f.r[1], d2 = o / f.r[1];
    const int kx0 = chunk * np;
    const long long base = d0 * f.s[0] + d1 * f.s[1] + d2 * f.s[2] + kx0;
    {
        typename V2<R>::type v[LOAD_C];
#pragma unroll
        for (int i = 0; i < LOAD_C; i++) {
            const int idx = threadIdx.x + i * FFT_BLOCK;
            v[i].x = v[i].y = (R)0;
            if (idx < n * np) {
                const int j = (int)fdiv((unsigned)idx, f.dnp), q = idx - j * np;
                if (kx0 + q < f.nkx) v[i] = spec[base + j * f.s_ax + q];
            }
        }
        load_roots(t, Wg, n);
#pragma unroll
        for (int i = 0; i < LOAD_C; i++) {
            const int idx = threadIdx.x + i * FFT_BLOCK;
            if (idx < n * np) t.a[idx] = Cd{(double)v[i].x, (double)v[i].y};
        }
    }
    if (FILTER || sign < 0) lds_dft<-1>(t, f.pl, n, np);
    else lds_dft<1>(t, f.pl, n, np);
    Cd *res = t.a;
    if constexpr (FILTER) {
        // 4 sin^2(pi k / L) of this axis and of the tile's kx, once per workgroup
        double *p2ax = (double *)(t.Wl + n), *p2x = p2ax + n;
        for (int m = threadIdx.x; m < n + np; m += blockDim.x) {
            if (m < n) p2ax[m] = lattice_p2(m, f.Lax);
            else p2x[m - n] = lattice_p2(kx0 + m - n, f.Lx);
        }
        __syncthreads();
        const double p2o = lattice_p2(d0, f.L[0]) + lattice_p2(d1, f.L[1]) + lattice_p2(d2, f.L[2]);
        const double sp = f.scale * f.p2max;
        for (int idx = threadIdx.x; idx < n * np; idx += blockDim.x) {
            const int k = (int)fdiv((unsigned)idx, f.dnp), q = idx - k * np;
            const double p2 = p2o + p2ax[k] + p2x[q];
            const double fac = p2 > 0.0 ? sp / p2 : 0.0;
            res[idx].x *= fac;
            res[idx].y *= fac;
        }
        lds_dft<1>(t, f.pl, n, np);  // back along the same axis
    }
    for (int idx = threadIdx.x; idx < n * np; idx += blockDim.x) {
        const int j = (int)fdiv((unsigned)idx, f.dnp), q = idx - j * np;
        if (kx0 + q < f.nkx) {
            typename V2<R>::type v;
            v.x = (R)res[idx].x;
            v.y = (R)res[idx].y;
            spec[base + j * f.s_ax + q] = v;
        }
    }
}

// W[m] = exp(2 pi i m / n), m < n.
__global__ void __launch_bounds__(256) k_fft_roots(Cd *__restrict__ W, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    W[m] = Cd{c, s};
}

// Radices of a length: 4s first, then 2, 3, 5, then any other primes.
static FftPlan plan_length(int n) {
    FftPlan p{};
    int ns = 1;
    auto push = [&](int r) { p.ns[p.nf] = make_fastdiv((unsigned)ns); p.fac[p.nf++] = r; ns *= r; };
    while (n % 4 == 0) { push(4); n /= 4; }
    for (int r : {2, 3, 5})
        while (n % r == 0) { push(r); n /= r; }
    for (int r = 7; n > 1; r += 2)
        while (n % r == 0) { push(r); n /= r; }
    return p;
}

FftSite make_fft_site(const Geom &g) {
    FftSite f;
    f.n = g.nx;
    f.nkx = g.nx / 2 + 1;
    f.pl = plan_length(f.n);
    f.ys = FFT_TILE_POINTS / (4 * g.nx);  // site rows per workgroup (>= 1: nx <= FFT_MAX_NX)
    f.srows = (long long)g.nt * g.nz * g.ny;
    f.dn = make_fastdiv((unsigned)f.n);
    f.dnkx = make_fastdiv((unsigned)f.nkx);
    f.dnc = make_fastdiv((unsigned)(4 * f.ys));
    return f;
}

// axis: 1 = y, 2 = z, 3 = t. spec strides: kx 1, y nkx, z ny nkx, a nz ny nkx, t 8 nz ny nkx.
FftAxis make_fft_axis(const Geom &g, int axis, bool coulomb) {
    FftAxis f{};
    const long long nkx = g.nx / 2 + 1, sy = nkx, sz = g.ny * sy, sa = g.nz * sz, st = 8 * sa;
    f.nkx = (int)nkx;
    f.Lx = g.nx;
    if (axis == 1) {
        f.n = g.ny; f.s_ax = sy;
        f.r[0] = g.nz; f.s[0] = sz; f.L[0] = g.nz;
        f.r[1] = 8;    f.s[1] = sa; f.L[1] = 0;
        f.r[2] = g.nt; f.s[2] = st; f.L[2] = coulomb ? 0 : g.nt;
    } else if (axis == 2) {
        f.n = g.nz; f.s_ax = sz;
        f.r[0] = g.ny; f.s[0] = sy; f.L[0] = g.ny;
        f.r[1] = 8;    f.s[1] = sa; f.L[1] = 0;
        f.r[2] = g.nt; f.s[2] = st; f.L[2] = coulomb ? 0 : g.nt;
    } else {
        f.n = g.nt; f.s_ax = st;
        f.r[0] = g.ny; f.s[0] = sy; f.L[0] = g.ny;
        f.r[1] = g.nz; f.s[1] = sz; f.L[1] = g.nz;
        f.r[2] = 8;    f.s[2] = sa; f.L[2] = 0;
    }
    f.Lax = f.n;
    f.pl = plan_length(f.n);
    // kx chunks of at most FFT_TILE_POINTS / n, as even as possible
    const int cap = FFT_TILE_POINTS / f.n > 0 ? FFT_TILE_POINTS / f.n : 1;
    f.nchunk = (f.nkx + cap - 1) / cap;
    f.np = (f.nkx + f.nchunk - 1) / f.nchunk;
    f.dnp = make_fastdiv((unsigned)f.np);
    return f;
}

static size_t lds_bytes(int n, int np) { return (size_t)tile_lds_points(n, np) * sizeof(Cd); }

hipError_t launch_fft_roots(void *W, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_fft_roots, dim3((n + 255) / 256), dim3(256), 0, st, (Cd *)W, n);
    return hipGetLastError();
}

static size_t site_lds_bytes(const FftSite &f) {
    return lds_bytes(f.n, 4 * f.ys + 1) + (size_t)f.ys * sizeof(RowInfo);
}

hipError_t launch_sd_delta_fx(int prec, int nelem, int gauge, const Geom &g, const FftSite &f, const void *W,
                              const void *U, void *spec, hipStream_t st) {
    const dim3 grid((unsigned)((f.srows + f.ys - 1) / f.ys));
    const size_t sh = site_lds_bytes(f);
    const int nd = gauge == 0 ? 4 : 3;
    const Cd *w = (const Cd *)W;
    const SlabOrder so = make_slab_order(g.ny * g.nz, f.ys, (int)grid.x);
#define GF_L(R, NE)                                                                                   \
    hipLaunchKernelGGL((k_sd_delta_fx<R, NE>), grid, dim3(FFT_BLOCK), sh, st, g, nd,                 \
                       (const V2<R>::type *)U, f, w, (V2<R>::type *)spec, so)
    if (prec == 0) { if (nelem == 9) GF_L(double, 9); else if (nelem == 6) GF_L(double, 6); else GF_L(double, 4); }
    else { if (nelem == 9) GF_L(float, 9); else if (nelem == 6) GF_L(float, 6); else GF_L(float, 4); }
#undef GF_L
    return hipGetLastError();
}

hipError_t launch_sd_fx_gfield(int prec, const Geom &g, const FftSite &f, const void *W, const void *spec,
                               void *gfield, hipStream_t st) {
    const dim3 grid((unsigned)((f.srows + f.ys - 1) / f.ys));
    const size_t sh = site_lds_bytes(f);
    const Cd *w = (const Cd *)W;
    if (prec == 0)
        hipLaunchKernelGGL(k_sd_fx_gfield<double>, grid, dim3(FFT_BLOCK), sh, st, g, f, w,
                           (const V2<double>::type *)spec, (V2<double>::type *)gfield);
    else
        hipLaunchKernelGGL(k_sd_fx_gfield<float>, grid, dim3(FFT_BLOCK), sh, st, g, f, w,
                           (const V2<float>::type *)spec, (V2<float>::type *)gfield);
    return hipGetLastError();
}

hipError_t launch_fft_axis(int prec, const FftAxis &f, const void *W, void *spec, int sign, int filter,
                           hipStream_t st) {
    const dim3 grid((unsigned)((long long)f.r[0] * f.r[1] * f.r[2] * f.nchunk));
    // the filter's tables of the axis and kx terms (n + np doubles) follow the roots
    const size_t sh = lds_bytes(f.n, f.np) + (filter ? (size_t)(f.n + f.np) * sizeof(double) : 0);
    const Cd *w = (const Cd *)W;
    const int sg = sign < 0 ? -1 : 1;
#define GF_L(R, FL) \
    hipLaunchKernelGGL((k_fft_axis<R, FL>), grid, dim3(FFT_BLOCK), sh, st, f, w, (V2<R>::type *)spec, sg)
    if (prec == 0) { if (filter) GF_L(double, true); else GF_L(double, false); }
    else { if (filter) GF_L(float, true); else GF_L(float, false); }
#undef GF_L
    return hipGetLastError();
}

}  // namespace gf
