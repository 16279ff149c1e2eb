/*
 * Plain FP64 CPU oracle for the pseudospectral Navier-Stokes / MHD /
 * Boussinesq / Gross-Pitaevskii hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * Everything here is written to be checked by eye against the paper
 * (Rosenberg, Mininni, Reddy, Pouquet, "GPU parallelization of a hybrid
 * pseudospectral fluid turbulence framework using CUDA"):
 *
 *   - the discrete Fourier expansion and its sign convention:
 *     Sec. 2, eq. (fftsum) and the sentence after it (backward = sign change);
 *   - real-to-complex storage of (Nx/2+1) x Ny x Nz coefficients with the
 *     Hermitian relation for real data: Sec. 2, forward-transform steps;
 *   - the forward transform as x then y then z one-dimensional transforms and
 *     the backward transform as the same steps reversed: Sec. 2, steps 1-3;
 *   - products of the nonlinear terms in physical space, pressure by
 *     projection onto divergence-free fields: Sec. 2, paragraph after
 *     eq. (fftsum);
 *   - independent point counts N_i and box lengths L_i per direction
 *     (Sec. 2, paragraph after eq. fftsum): physical wavenumbers 2 pi p / L_i;
 *   - the incompressible Navier-Stokes equations (eq. mom + eq. divv with
 *     theta = 0), MHD (eq. uMHD, eq. bMHD), the Boussinesq equations
 *     (eq. mom, eq. temp, eq. divv) and the Gross-Pitaevskii equation
 *     (eq. gpe) of a complex wavefunction;
 *   - explicit Runge-Kutta time stepping of order 2-4: Sec. 2.
 *
 * Readings where the paper is silent (normalisation, dealiasing rule,
 * integrating factor, RK variant, shell binning) are the ones listed in the
 * design notes: forward transform carries 1/(Nx Ny Nz) so that
 * u(x) = sum_k uhat(k) exp(i k.x); backward is unscaled; cube truncation with
 * K_i = ceil(N_i/3) - 1 per axis for the quadratic products and
 * K_i = ceil(N_i/4) - 1 for the cubic product of eq. gpe (both chosen by the
 * caller and passed in); Lawson integrating factor with Heun RK2 / classical
 * RK4; shell n = floor(|k| / dk + 1/2) with dk = min_i 2 pi / L_i.
 *
 * The FFT is the textbook recursive mixed-radix Cooley-Tukey (Cooley & Tukey
 * 1965) over factors 2 and 3, with a naive O(n^2) DFT for any other factor.
 * No blocking, fusion or reordering beyond that.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* 1D transforms                                                             */
/* ------------------------------------------------------------------------ */

/* Naive DFT, the definition itself: X[k] = sum_j x[j] exp(sign 2 pi i j k / n). */
void ora_dft_naive(int n, const double *in, double *out, int sign)
{
    const cplx *x = (const cplx *)in;
    cplx *X = (cplx *)out;
    for (int k = 0; k < n; ++k) {
        cplx acc = 0;
        for (int j = 0; j < n; ++j) {
            long m = ((long)j * k) % n;
            double ang = sign * 2.0 * M_PI * (double)m / (double)n;
            acc += x[j] * (cos(ang) + I * sin(ang));
        }
        X[k] = acc;
    }
}

static int smallest_factor(int n)
{
    if (n % 2 == 0) return 2;
    if (n % 3 == 0) return 3;
    return n; /* anything else is done by the naive DFT */
}

/* Recursive decimation-in-time Cooley-Tukey.
 * in  : input sequence of length n with element stride s
 * out : contiguous output of length n
 * tw  : tw[m] = exp(sign 2 pi i m / L) for the top-level length L
 * step: L / n, so that w_n^j = tw[j * step]                                   */
static void fft_rec(const cplx *in, int s, cplx *out, int n, const cplx *tw, int step)
{
    if (n == 1) { out[0] = in[0]; return; }
    int p = smallest_factor(n);
    if (p == n) {
        for (int k = 0; k < n; ++k) {
            cplx acc = 0;
            for (int j = 0; j < n; ++j)
                acc += in[(long)j * s] * tw[(((long)j * k) % n) * step];
            out[k] = acc;
        }
        return;
    }
    int m = n / p;
    /* Y_q[k] = sum_{j<m} x[p j + q] w_m^{j k}, stored at out[q m + k] */
    for (int q = 0; q < p; ++q)
        fft_rec(in + (long)q * s, s * p, out + (long)q * m, m, tw, step * p);
    /* X[k + m t] = sum_q w_n^{q (k + m t)} Y_q[k]; the p outputs of a given k
     * occupy exactly the p slots its inputs came from, so it is done in place */
    cplx a[3];
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q) a[q] = out[(long)q * m + k];
        for (int t = 0; t < p; ++t) {
            cplx acc = 0;
            for (int q = 0; q < p; ++q)
                acc += tw[(((long)q * (k + (long)m * t)) % n) * step] * a[q];
            out[k + (long)m * t] = acc;
        }
    }
}

static cplx *roots_table(int n, int sign)
{
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int m = 0; m < n; ++m) {
        double ang = 2.0 * M_PI * (double)m / (double)n;
        tw[m] = cos(ang) + I * (sign * sin(ang));
    }
    return tw;
}

/* In-place 1D FFT of n complex numbers (interleaved re/im), unnormalised. */
void ora_fft1d(int n, double *data, int sign)
{
    cplx *x = (cplx *)data;
    cplx *tw = roots_table(n, sign);
    cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    fft_rec(x, 1, out, n, tw, 1);
    memcpy(x, out, sizeof(cplx) * (size_t)n);
    free(out);
    free(tw);
}

/* Transform every line of a 3D complex array along one axis.
 * Lines are gathered into a contiguous buffer, transformed and scattered back. */
static void c2c_axis(cplx *a, long nlines, int n, long stride,
                     long (*line_base)(long, const long *), const long *geo, int sign)
{
    cplx *tw = roots_table(n, sign);
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)n);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; ++l) {
            long b = line_base(l, geo);
            for (int j = 0; j < n; ++j) buf[j] = a[b + j * stride];
            fft_rec(buf, 1, out, n, tw, 1);
            for (int j = 0; j < n; ++j) a[b + j * stride] = out[j];
        }
        free(buf);
        free(out);
    }
    free(tw);
}

/* geo = {nz, ny, nxh}: complex array [nz][ny][nxh] */
static long base_y(long l, const long *g) { /* l over (z, kx) */
    long z = l / g[2], kx = l % g[2];
    return z * g[1] * g[2] + kx;
}
static long base_z(long l, const long *g) { /* l over (y, kx) */
    return l; /* y * nxh + kx is exactly the flat offset in the first plane */
}
static long base_x(long l, const long *g) { /* l over (z, y), full complex rows */
    return l * g[2];
}

/* ------------------------------------------------------------------------ */
/* 3D real <-> complex transforms (layout: real [nz][ny][nx], complex         */
/* [nz][ny][nx/2+1]; x fastest)                                               */
/* ------------------------------------------------------------------------ */

/* Forward: x, then y, then z, then scale by 1/(nx ny nz). */
void ora_r2c3(int nz, int ny, int nx, const double *in, double *out)
{
    long nxh = nx / 2 + 1;
    cplx *o = (cplx *)out;
    cplx *tw = roots_table(nx, -1);
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
        cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
#pragma omp for schedule(static)
        for (long l = 0; l < (long)nz * ny; ++l) {
            for (int j = 0; j < nx; ++j) buf[j] = in[l * nx + j];
            fft_rec(buf, 1, res, nx, tw, 1);
            for (long k = 0; k < nxh; ++k) o[l * nxh + k] = res[k];
        }
        free(buf);
        free(res);
    }
    free(tw);
    long geo[3] = {nz, ny, nxh};
    c2c_axis(o, (long)nz * nxh, ny, nxh, base_y, geo, -1);
    c2c_axis(o, (long)ny * nxh, nz, (long)ny * nxh, base_z, geo, -1);
    double scale = 1.0 / ((double)nx * ny * nz);
    long tot = (long)nz * ny * nxh;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < tot; ++i) o[i] *= scale;
}

/* Backward: z, then y, then x (the forward steps reversed), unscaled.  Along
 * x the half line is extended by X(nx-k) = conj X(k); the self-conjugate
 * points k = 0 and k = nx/2 keep only their real parts.                      */
void ora_c2r3(int nz, int ny, int nx, const double *in, double *out)
{
    long nxh = nx / 2 + 1;
    long tot = (long)nz * ny * nxh;
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
    memcpy(t, in, sizeof(cplx) * (size_t)tot);
    long geo[3] = {nz, ny, nxh};
    c2c_axis(t, (long)ny * nxh, nz, (long)ny * nxh, base_z, geo, +1);
    c2c_axis(t, (long)nz * nxh, ny, nxh, base_y, geo, +1);
    cplx *tw = roots_table(nx, +1);
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
        cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
#pragma omp for schedule(static)
        for (long l = 0; l < (long)nz * ny; ++l) {
            const cplx *h = t + l * nxh;
            for (int k = 0; k < nx; ++k) {
                if (k == 0) buf[k] = creal(h[0]);
                else if (2 * k == nx) buf[k] = creal(h[k]);
                else if (k < nxh) buf[k] = h[k];
                else buf[k] = conj(h[nx - k]);
            }
            fft_rec(buf, 1, res, nx, tw, 1);
            for (int j = 0; j < nx; ++j) out[l * nx + j] = creal(res[j]);
        }
        free(buf);
        free(res);
    }
    free(tw);
    free(t);
}

/* Full complex 3D transform [nz][ny][nx], unnormalised, for tests. */
void ora_c2c3(int nz, int ny, int nx, double *data, int sign)
{
    cplx *a = (cplx *)data;
    long geo[3] = {nz, ny, nx};
    c2c_axis(a, (long)nz * ny, nx, 1, base_x, geo, sign);
    c2c_axis(a, (long)nz * nx, ny, nx, base_y, geo, sign);
    c2c_axis(a, (long)ny * nx, nz, (long)ny * nx, base_z, geo, sign);
}

/* ------------------------------------------------------------------------ */
/* Wavenumbers, masks, projection                                             */
/* ------------------------------------------------------------------------ */

/* The grid of a run.  eq. (fftsum) expands every field over Nx x Ny x Nz
 * points of a box Lx x Ly x Lz whose sizes are independent per direction
 * (Sec. 2, paragraph after eq. fftsum): index p on an axis of n points is the
 * integer wavenumber wn(p, n), and the physical wavenumber is a p with
 * a = 2 pi / L.  kc* are the cube cutoffs per axis (< 0: nothing removed on
 * that axis); sphere = 1 keeps |k|^2 <= kcx^2 in integer wavenumbers (used on
 * isotropic grids only).                                                     */
typedef struct {
    int nx, ny, nz;
    double ax, ay, az;
    int kcx, kcy, kcz;
    int sphere;
} ora_grid;

/* Index -> integer wavenumber: p < n/2 -> p, else p - n (the Nyquist index
 * n/2 maps to -n/2 on the full axes; on the half x axis indices are 0..n/2). */
static int wn(int p, int n) { return p < n / 2 ? p : p - n; }

/* Dealiasing mask D(k) on integer wavenumbers. */
static int kept(const ora_grid *g, int kx, int ky, int kz)
{
    if (g->sphere) {
        if (g->kcx < 0) return 1;
        return (long)kx * kx + (long)ky * ky + (long)kz * kz <= (long)g->kcx * g->kcx;
    }
    return (g->kcx < 0 || abs(kx) <= g->kcx) && (g->kcy < 0 || abs(ky) <= g->kcy) &&
           (g->kcz < 0 || abs(kz) <= g->kcz);
}

/* Half-spectrum size and index: component c, mode (kz, ky, kx) at
 * c*NH + (z*ny + y)*(nx/2+1) + x.                                            */
static long nh_of(const ora_grid *g) { return (long)g->nz * g->ny * (g->nx / 2 + 1); }
static long np_of(const ora_grid *g) { return (long)g->nz * g->ny * g->nx; }
static long idx_of(const ora_grid *g, int z, int y, int x) { return ((long)z * g->ny + y) * (g->nx / 2 + 1) + x; }

/* Physical wavenumber vector of half-spectrum point (z, y, x). */
static void kvec(const ora_grid *g, int z, int y, int x, double *kx, double *ky, double *kz)
{
    *kx = g->ax * x;
    *ky = g->ay * wn(y, g->ny);
    *kz = g->az * wn(z, g->nz);
}

/* i k x v for a spectral vector field (3 components). */
static void spectral_curl(const ora_grid *g, const cplx *v, cplx *out)
{
    long nh = nh_of(g);
    int nxh = g->nx / 2 + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < nxh; ++x) {
                long i = idx_of(g, z, y, x);
                double kx, ky, kz;
                kvec(g, z, y, x, &kx, &ky, &kz);
                cplx vx = v[i], vy = v[nh + i], vz = v[2 * nh + i];
                out[i] = I * (ky * vz - kz * vy);
                out[nh + i] = I * (kz * vx - kx * vz);
                out[2 * nh + i] = I * (kx * vy - ky * vx);
            }
}

/* Pointwise cross product c = a x b of physical fields (3 components each),
 * accumulated into c when acc != 0. */
static void cross(long np, const double *a, const double *b, double *c, int acc)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < np; ++i) {
        double ax = a[i], ay = a[np + i], az = a[2 * np + i];
        double bx = b[i], by = b[np + i], bz = b[2 * np + i];
        double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
        if (acc) { c[i] += cx; c[np + i] += cy; c[2 * np + i] += cz; }
        else     { c[i]  = cx; c[np + i]  = cy; c[2 * np + i]  = cz; }
    }
}

static void c2r_vec(const ora_grid *g, const cplx *v, double *out)
{
    long np = np_of(g), nh = nh_of(g);
    for (int c = 0; c < 3; ++c) ora_c2r3(g->nz, g->ny, g->nx, (const double *)(v + c * nh), out + c * np);
}
static void r2c_vec(const ora_grid *g, const double *in, cplx *out)
{
    long np = np_of(g), nh = nh_of(g);
    for (int c = 0; c < 3; ++c) ora_r2c3(g->nz, g->ny, g->nx, in + c * np, (double *)(out + c * nh));
}

/* out = D(k) P(k) v  (P = I - k k^T / |k|^2, P(0) = 0), optionally + f. */
static void dealias_project(const ora_grid *g, cplx *v, const cplx *f)
{
    long nh = nh_of(g);
    int nxh = g->nx / 2 + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < nxh; ++x) {
                long i = idx_of(g, z, y, x);
                double kx, ky, kz;
                kvec(g, z, y, x, &kx, &ky, &kz);
                double k2 = kx * kx + ky * ky + kz * kz;
                cplx vx = v[i], vy = v[nh + i], vz = v[2 * nh + i];
                if (!kept(g, x, wn(y, g->ny), wn(z, g->nz)) || k2 == 0.0) {
                    vx = vy = vz = 0;
                } else {
                    cplx kv = (kx * vx + ky * vy + kz * vz) / k2;
                    vx -= kx * kv; vy -= ky * kv; vz -= kz * kv;
                }
                if (f) { vx += f[i]; vy += f[nh + i]; vz += f[2 * nh + i]; }
                v[i] = vx; v[nh + i] = vy; v[2 * nh + i] = vz;
            }
}

/* D(k) alone on nc components. */
static void dealias_only(const ora_grid *g, cplx *v, int nc)
{
    long nh = nh_of(g);
    int nxh = g->nx / 2 + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < nxh; ++x)
                if (!kept(g, x, wn(y, g->ny), wn(z, g->nz))) {
                    long i = idx_of(g, z, y, x);
                    for (int c = 0; c < nc; ++c) v[c * nh + i] = 0;
                }
}

/* ------------------------------------------------------------------------ */
/* Right-hand sides                                                          */
/* ------------------------------------------------------------------------ */

/* Navier-Stokes nonlinear operator, rotational form:
 *   N(u) = D P F[u x w] + f,  w = curl u computed spectrally as i k x uhat.
 * uhat, fhat, out: [3][nz][ny][nx/2+1] complex.  fhat may be NULL.          */
void ora_ns_rhs(const ora_grid *g, const double *uhat, const double *fhat, double *out)
{
    long nh = nh_of(g), np = np_of(g);
    const cplx *u = (const cplx *)uhat;
    cplx *w = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nh);
    double *ur = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    double *wr = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    double *nr = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    spectral_curl(g, u, w);
    c2r_vec(g, u, ur);
    c2r_vec(g, w, wr);
    cross(np, ur, wr, nr, 0);
    r2c_vec(g, nr, (cplx *)out);
    dealias_project(g, (cplx *)out, (const cplx *)fhat);
    free(w); free(ur); free(wr); free(nr);
}

/* MHD nonlinear operators (eq. uMHD, eq. bMHD in rotational form):
 *   N_u = D P F[u x w + j x b],   N_b = D (i k x F[u x b]),
 * with w = i k x uhat and j = i k x bhat.                                   */
void ora_mhd_rhs(const ora_grid *g, const double *uhat, const double *bhat, double *out_u, double *out_b)
{
    long nh = nh_of(g), np = np_of(g);
    const cplx *u = (const cplx *)uhat, *b = (const cplx *)bhat;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nh);
    double *ur = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    double *br = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    double *qr = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    double *nr = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    c2r_vec(g, u, ur);
    c2r_vec(g, b, br);
    spectral_curl(g, u, tmp);
    c2r_vec(g, tmp, qr);           /* w */
    cross(np, ur, qr, nr, 0);      /* u x w */
    spectral_curl(g, b, tmp);
    c2r_vec(g, tmp, qr);           /* j */
    cross(np, qr, br, nr, 1);      /* + j x b */
    r2c_vec(g, nr, (cplx *)out_u);
    dealias_project(g, (cplx *)out_u, NULL);
    cross(np, ur, br, nr, 0);      /* u x b */
    r2c_vec(g, nr, tmp);
    spectral_curl(g, tmp, (cplx *)out_b);
    dealias_only(g, (cplx *)out_b, 3);   /* D only: the curl is already solenoidal */
    free(tmp); free(ur); free(br); free(qr); free(nr);
}

/* Boussinesq operators (eq. mom with its buoyancy term, eq. temp, eq. divv).
 * Momentum in rotational form (the gradient part of u . grad u joins the
 * pressure and is removed by the projection); the scalar in advective form:
 *   N_u = D P (F[u x w] - nbv theta zhat) + f,
 *   N_t = D (-F[u . grad theta] + nbv w_z),
 * with w = i k x uhat, grad theta = c2r(i k thetahat) and w_z the z component
 * of the velocity coefficients.  thhat, out_t: [nz][ny][nx/2+1] complex.     */
void ora_bq_rhs(const ora_grid *g, double nbv, const double *uhat, const double *thhat,
                const double *fhat, double *out_u, double *out_t)
{
    long nh = nh_of(g), np = np_of(g);
    int nxh = g->nx / 2 + 1;
    const cplx *u = (const cplx *)uhat, *th = (const cplx *)thhat;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nh);
    double *ur = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    double *qr = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    double *nr = (double *)malloc(sizeof(double) * 3 * (size_t)np);
    cplx *ou = (cplx *)out_u, *ot = (cplx *)out_t;
    c2r_vec(g, u, ur);
    spectral_curl(g, u, tmp);
    c2r_vec(g, tmp, qr);           /* w */
    cross(np, ur, qr, nr, 0);      /* u x w */
    r2c_vec(g, nr, ou);
    for (long i = 0; i < nh; ++i) ou[2 * nh + i] -= nbv * th[i];   /* buoyancy */
    dealias_project(g, ou, (const cplx *)fhat);
    /* grad theta = i k thetahat, then u . grad theta in physical space */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < nxh; ++x) {
                long i = idx_of(g, z, y, x);
                double kx, ky, kz;
                kvec(g, z, y, x, &kx, &ky, &kz);
                tmp[i] = I * kx * th[i];
                tmp[nh + i] = I * ky * th[i];
                tmp[2 * nh + i] = I * kz * th[i];
            }
    c2r_vec(g, tmp, qr);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < np; ++i)
        nr[i] = -(ur[i] * qr[i] + ur[np + i] * qr[np + i] + ur[2 * np + i] * qr[2 * np + i]);
    ora_r2c3(g->nz, g->ny, g->nx, nr, out_t);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < nxh; ++x) {
                long i = idx_of(g, z, y, x);
                if (kept(g, x, wn(y, g->ny), wn(z, g->nz))) ot[i] += nbv * u[2 * nh + i];
                else ot[i] = 0;
            }
    free(tmp); free(ur); free(qr); free(nr);
}

/* Gross-Pitaevskii nonlinear operator (eq. gpe divided by i hbar): with
 * alpha = hbar / 2m and beta = g / hbar the equation reads
 *   d psi/dt = i alpha Lap psi - i beta |psi|^2 psi,
 * whose linear part -i alpha |k|^2 is taken by the integrating factor and
 * whose nonlinear part is  N(psi) = -i beta D F[|psi|^2 psi], the cube
 * product formed at the grid points.  psi is complex, so its coefficients
 * fill the whole [nz][ny][nx] spectrum (c2c transforms, forward scaled by
 * 1/(nx ny nz)).  On the x axis the cutoff applies to wn(x, nx).            */
static int kept_full(const ora_grid *g, int x, int y, int z)
{
    return kept(g, wn(x, g->nx), wn(y, g->ny), wn(z, g->nz));
}

void ora_gpe_rhs(const ora_grid *g, double beta, const double *psihat, double *out)
{
    long np = np_of(g);
    cplx *p = (cplx *)malloc(sizeof(cplx) * (size_t)np);
    cplx *o = (cplx *)out;
    memcpy(p, psihat, sizeof(cplx) * (size_t)np);
    ora_c2c3(g->nz, g->ny, g->nx, (double *)p, +1);        /* psi at the grid points */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < np; ++i) {
        double r2 = creal(p[i]) * creal(p[i]) + cimag(p[i]) * cimag(p[i]);
        o[i] = r2 * p[i];                                 /* |psi|^2 psi */
    }
    ora_c2c3(g->nz, g->ny, g->nx, out, -1);
    double scale = 1.0 / (double)np;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                long i = ((long)z * g->ny + y) * g->nx + x;
                o[i] = kept_full(g, x, y, z) ? -I * beta * scale * o[i] : 0;
            }
    free(p);
}

/* ------------------------------------------------------------------------ */
/* Time stepping: Lawson integrating factor + explicit Runge-Kutta            */
/* ------------------------------------------------------------------------ */

typedef struct {
    ora_grid g;
    int solver;      /* 0 = Navier-Stokes, 1 = MHD, 2 = Boussinesq, 3 = Gross-Pitaevskii */
    int rk_order;    /* 2 (Heun) or 4 (classical) */
    int linear_only; /* 1: nonlinear operator replaced by zero */
    double nu, eta, dt;   /* eta: magnetic (MHD) or scalar (Boussinesq) diffusivity;
                             Gross-Pitaevskii: nu = alpha (hbar / 2m), eta unused */
    double nbv;           /* Brunt-Vaisala frequency (Boussinesq); beta = g / hbar (Gross-Pitaevskii) */
} ora_params;

/* Evaluate the nonlinear operator(s) for the state (u, b) into (ku, kb). */
static void eval_rhs(const ora_params *p, const cplx *u, const cplx *b, const cplx *f,
                     cplx *ku, cplx *kb)
{
    const ora_grid *g = &p->g;
    long nh = nh_of(g);
    if (p->linear_only) {
        memset(ku, 0, sizeof(cplx) * (p->solver == 3 ? (size_t)np_of(g) : 3 * (size_t)nh));
        if (p->solver == 1 || p->solver == 2) memset(kb, 0, sizeof(cplx) * (p->solver == 2 ? 1 : 3) * (size_t)nh);
        return;
    }
    if (p->solver == 0)
        ora_ns_rhs(g, (const double *)u, (const double *)f, (double *)ku);
    else if (p->solver == 1)
        ora_mhd_rhs(g, (const double *)u, (const double *)b, (double *)ku, (double *)kb);
    else if (p->solver == 2)
        ora_bq_rhs(g, p->nbv, (const double *)u, (const double *)b, (const double *)f, (double *)ku, (double *)kb);
    else
        ora_gpe_rhs(g, p->nbv, (const double *)u, (double *)ku);
}

/* Integrating factor per mode of the half spectrum: E(k) = exp(-visc |k|^2 h / 2). */
static void if_table(const ora_grid *g, double visc, double h, cplx *E)
{
    int nxh = g->nx / 2 + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < nxh; ++x) {
                double kx, ky, kz;
                kvec(g, z, y, x, &kx, &ky, &kz);
                double k2 = kx * kx + ky * ky + kz * kz;
                E[idx_of(g, z, y, x)] = exp(-visc * k2 * h * 0.5);
            }
}

/* Integrating factor of the Gross-Pitaevskii linear part over the whole
 * spectrum: E(k) = exp(-i alpha |k|^2 h / 2).                               */
static void if_table_gpe(const ora_grid *g, double alpha, double h, cplx *E)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                double kx = g->ax * wn(x, g->nx), ky = g->ay * wn(y, g->ny), kz = g->az * wn(z, g->nz);
                double k2 = kx * kx + ky * ky + kz * kz;
                E[((long)z * g->ny + y) * g->nx + x] = cexp(-I * alpha * k2 * h * 0.5);
            }
}

/* One Lawson step for one field group given the already evaluated stages is
 * not separable from the others (the operator couples u with b or theta), so
 * the step below runs the stage loop over all fields together.  The second
 * group is b (3 components, diffusivity eta) or theta (1 component, eta read
 * as the scalar diffusivity kappa); the Gross-Pitaevskii state is the single
 * complex field psi over the whole spectrum.  Stage formulas:
 *   RK2 (Heun):  k1 = N(u);  k2 = N(E^2 (u + h k1));
 *                u+ = E^2 u + h/2 (E^2 k1 + k2)
 *   RK4:         k1 = N(u);  k2 = N(E (u + h/2 k1));  k3 = N(E u + h/2 k2);
 *                k4 = N(E^2 u + h E k3);
 *                u+ = E^2 u + h/6 (E^2 k1 + 2 E (k2 + k3) + k4)              */
int ora_step(const ora_params *p, double *uhat, double *bhat, const double *fhat, int nsteps)
{
    const ora_grid *g = &p->g;
    int gpe = p->solver == 3, two = p->solver == 1 || p->solver == 2;
    long nh = gpe ? np_of(g) : nh_of(g);   /* modes per component */
    long tots[2] = {(gpe ? 1 : 3) * nh, (p->solver == 2 ? 1 : 3) * nh};
    int nf = two ? 2 : 1;               /* field groups: u (and b or theta) */
    double h = p->dt;
    cplx *st[2] = {(cplx *)uhat, two ? (cplx *)bhat : NULL};
    cplx *E[2];
    cplx *k1[2], *k2[2], *k3[2], *k4[2], *v[2];
    for (int q = 0; q < nf; ++q) {
        long tot = tots[q];
        E[q] = (cplx *)malloc(sizeof(cplx) * (size_t)nh);
        if (gpe) if_table_gpe(g, p->nu, h, E[q]);
        else if_table(g, q == 0 ? p->nu : p->eta, h, E[q]);
        k1[q] = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
        k2[q] = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
        k3[q] = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
        k4[q] = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
        v[q] = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
    }
    if (!two) { k1[1] = k2[1] = k3[1] = k4[1] = v[1] = NULL; }
    const cplx *f = (const cplx *)fhat;

    for (int s = 0; s < nsteps; ++s) {
        if (p->rk_order == 2) {
            eval_rhs(p, st[0], st[1], f, k1[0], k1[1]);
            for (int q = 0; q < nf; ++q)
#pragma omp parallel for schedule(static)
                for (long i = 0; i < tots[q]; ++i) {
                    cplx e2 = E[q][i % nh] * E[q][i % nh];
                    v[q][i] = e2 * (st[q][i] + h * k1[q][i]);
                }
            eval_rhs(p, v[0], v[1], f, k2[0], k2[1]);
            for (int q = 0; q < nf; ++q)
#pragma omp parallel for schedule(static)
                for (long i = 0; i < tots[q]; ++i) {
                    cplx e2 = E[q][i % nh] * E[q][i % nh];
                    st[q][i] = e2 * st[q][i] + 0.5 * h * (e2 * k1[q][i] + k2[q][i]);
                }
        } else {
            eval_rhs(p, st[0], st[1], f, k1[0], k1[1]);
            for (int q = 0; q < nf; ++q)
#pragma omp parallel for schedule(static)
                for (long i = 0; i < tots[q]; ++i)
                    v[q][i] = E[q][i % nh] * (st[q][i] + 0.5 * h * k1[q][i]);
            eval_rhs(p, v[0], v[1], f, k2[0], k2[1]);
            for (int q = 0; q < nf; ++q)
#pragma omp parallel for schedule(static)
                for (long i = 0; i < tots[q]; ++i)
                    v[q][i] = E[q][i % nh] * st[q][i] + 0.5 * h * k2[q][i];
            eval_rhs(p, v[0], v[1], f, k3[0], k3[1]);
            for (int q = 0; q < nf; ++q)
#pragma omp parallel for schedule(static)
                for (long i = 0; i < tots[q]; ++i) {
                    cplx e = E[q][i % nh];
                    v[q][i] = e * e * st[q][i] + h * e * k3[q][i];
                }
            eval_rhs(p, v[0], v[1], f, k4[0], k4[1]);
            for (int q = 0; q < nf; ++q)
#pragma omp parallel for schedule(static)
                for (long i = 0; i < tots[q]; ++i) {
                    cplx e = E[q][i % nh];
                    st[q][i] = e * e * st[q][i]
                             + h / 6.0 * (e * e * k1[q][i] + 2.0 * e * (k2[q][i] + k3[q][i]) + k4[q][i]);
                }
        }
    }
    for (int q = 0; q < nf; ++q) {
        free(E[q]); free(k1[q]); free(k2[q]); free(k3[q]); free(k4[q]); free(v[q]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/* Weight of a stored half-spectrum mode in sums over the full spectrum:
 * 1 on the self-conjugate planes kx = 0 and kx = nx/2, otherwise 2.         */
static double hweight(int x, int nx) { return (x == 0 || 2 * x == nx) ? 1.0 : 2.0; }

/* Pairwise (cascade) summation of an array, the usual way to keep the
 * rounding error of a long sum at O(log n) ulps.                            */
static double pairwise(const double *a, long m)
{
    if (m <= 16) {
        double s = 0;
        for (long i = 0; i < m; ++i) s += a[i];
        return s;
    }
    long h = m / 2;
    return pairwise(a, h) + pairwise(a + h, m - h);
}

/* Energy of an nc-component field, E = 1/2 sum_k w |vhat|^2 = <|v|^2>/2
 * (kinetic or magnetic energy for nc = 3, scalar variance for nc = 1).
 * With k2w = 1 each mode is weighted by |k|^2 (enstrophy for a solenoidal
 * field: the mean of |curl v|^2 / 2; for a scalar <|grad theta|^2> / 2).    */
double ora_quad(const ora_grid *g, int nc, const double *vhat, int k2w)
{
    long nh = nh_of(g);
    int nxh = g->nx / 2 + 1;
    const cplx *v = (const cplx *)vhat;
    double *t = (double *)malloc(sizeof(double) * (size_t)nh);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nh; ++i) {
        int x = (int)(i % nxh), y = (int)((i / nxh) % g->ny), z = (int)(i / ((long)nxh * g->ny));
        double kx, ky, kz;
        kvec(g, z, y, x, &kx, &ky, &kz);
        double s = 0;
        for (int c = 0; c < nc; ++c) {
            cplx q = v[c * nh + i];
            s += creal(q) * creal(q) + cimag(q) * cimag(q);
        }
        t[i] = 0.5 * hweight(x, g->nx) * (k2w ? kx * kx + ky * ky + kz * kz : 1.0) * s;
    }
    double e = pairwise(t, nh);
    free(t);
    return e;
}

/* Shell of a mode: s = floor(|k| / dk + 1/2), dk = the smallest of the
 * per-axis wavenumber units 2 pi / L_i (|k| + 1/2 on a 2 pi box).           */
static double shell_unit(const ora_grid *g)
{
    double d = g->ax;
    if (g->ay < d) d = g->ay;
    if (g->az < d) d = g->az;
    return d;
}
static int shell_of(double k2, double dk) { return (int)floor(sqrt(k2) / dk + 0.5); }

/* Shell spectrum E(s) = 1/2 sum_{shell s} w |vhat|^2, s = 0..nshells-1, of
 * an nc-component field.  Modes beyond the last shell are ignored.          */
void ora_spectrum(const ora_grid *g, int nc, const double *vhat, double *Ek, int nshells)
{
    long nh = nh_of(g);
    int nxh = g->nx / 2 + 1;
    double dk = shell_unit(g);
    const cplx *v = (const cplx *)vhat;
    /* gather per-shell terms, then sum each shell pairwise */
    long *cnt = (long *)calloc((size_t)nshells, sizeof(long));
    int *sh = (int *)malloc(sizeof(int) * (size_t)nh);
    for (long i = 0; i < nh; ++i) {
        int x = (int)(i % nxh), y = (int)((i / nxh) % g->ny), z = (int)(i / ((long)nxh * g->ny));
        double kx, ky, kz;
        kvec(g, z, y, x, &kx, &ky, &kz);
        sh[i] = shell_of(kx * kx + ky * ky + kz * kz, dk);
        if (sh[i] < nshells) cnt[sh[i]]++;
    }
    double **terms = (double **)malloc(sizeof(double *) * (size_t)nshells);
    long *fill = (long *)calloc((size_t)nshells, sizeof(long));
    for (int s = 0; s < nshells; ++s) terms[s] = (double *)malloc(sizeof(double) * (size_t)(cnt[s] + 1));
    for (long i = 0; i < nh; ++i) {
        int s = sh[i];
        if (s >= nshells) continue;
        double a = 0;
        for (int c = 0; c < nc; ++c) {
            cplx q = v[c * nh + i];
            a += creal(q) * creal(q) + cimag(q) * cimag(q);
        }
        terms[s][fill[s]++] = 0.5 * hweight((int)(i % nxh), g->nx) * a;
    }
    for (int s = 0; s < nshells; ++s) {
        Ek[s] = pairwise(terms[s], fill[s]);
        free(terms[s]);
    }
    free(terms); free(fill); free(cnt); free(sh);
}

/* Gross-Pitaevskii invariants of a state on the whole spectrum:
 *   out[0] = particle number  N = sum_k |psihat|^2 = <|psi|^2>,
 *   out[1] = kinetic energy   alpha sum_k |k|^2 |psihat|^2 = alpha <|grad psi|^2>,
 *   out[2] = interaction      beta/2 <|psi|^4>   (grid average),
 * each pairwise-summed; H = out[1] + out[2] is the Hamiltonian of eq. gpe
 * in units of hbar.                                                          */
void ora_gpe_invariants(const ora_grid *g, double alpha, double beta, const double *psihat, double *out)
{
    long np = np_of(g);
    const cplx *v = (const cplx *)psihat;
    double *t0 = (double *)malloc(sizeof(double) * (size_t)np);
    double *t1 = (double *)malloc(sizeof(double) * (size_t)np);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)np);
    cplx *p = (cplx *)malloc(sizeof(cplx) * (size_t)np);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < np; ++i) {
        int x = (int)(i % g->nx), y = (int)((i / g->nx) % g->ny), z = (int)(i / ((long)g->nx * g->ny));
        double kx = g->ax * wn(x, g->nx), ky = g->ay * wn(y, g->ny), kz = g->az * wn(z, g->nz);
        double a2 = creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
        t0[i] = a2;
        t1[i] = alpha * (kx * kx + ky * ky + kz * kz) * a2;
    }
    memcpy(p, v, sizeof(cplx) * (size_t)np);
    ora_c2c3(g->nz, g->ny, g->nx, (double *)p, +1);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < np; ++i) {
        double r2 = creal(p[i]) * creal(p[i]) + cimag(p[i]) * cimag(p[i]);
        t2[i] = 0.5 * beta * r2 * r2 / (double)np;
    }
    out[0] = pairwise(t0, np);
    out[1] = pairwise(t1, np);
    out[2] = pairwise(t2, np);
    free(t0); free(t1); free(t2); free(p);
}
