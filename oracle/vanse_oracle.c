/*
 * vanse_oracle.c -- plain, slow, FP64 CPU reference of the consistent VANSE
 * lattice Boltzmann time step of Bukreev, Simonis, Kummerlaender, Jessberger
 * and Krause, "Consistent lattice Boltzmann methods for the volume averaged
 * Navier-Stokes equations" (arXiv:2208.09267).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * GPU library: the lattice tables below are this file's own copy, written
 * from the paper's Tables 1-2 (D2Q9, D3Q27) and the standard D3Q19 subset.
 *
 * Conventions
 *   - lattice units: dx = dt = 1, c_s^2 = 1/3 (follows from the weights of
 *     Tables 1-2: sum_i w_i xi_ix^2 = 1/3);
 *   - populations are stored cell-major ("AoS"): f[cell*Q + i], with
 *     cell = (z*ny + y)*nx + x, x fastest, periodic in every axis;
 *   - one step is the literal lattice Boltzmann equation (eq. lbe, Section
 *     "Lattice Boltzmann scheme for VANSE"): collide at x, then push the
 *     post-collision value to x + xi_i, into a second array;
 *   - compile with -O2 -ffp-contract=off and no fast-math, so every
 *     operation below is one IEEE binary64 round-to-nearest operation in
 *     the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_D2Q9 0
#define OR_D3Q19 1
#define OR_D3Q27 2

#define OR_OK 0
#define OR_EINVAL (-1)

/* ---------------------------------------------------------------------------
 * Lattice tables.  D2Q9: Table 1.  D3Q27: Table 2 (rest, 6 faces, 12 edges,
 * 8 corners).  D3Q19: rest + faces + edges of Table 2 with the standard
 * D3Q19 weights 1/3, 1/18, 1/36.
 * ------------------------------------------------------------------------ */
static const int C_D2Q9[9][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};

static const int C_D3Q27[27][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};

typedef struct {
    int d;                 /* spatial dimension */
    int q;                 /* number of discrete velocities */
    const int (*c)[3];     /* velocities */
    double w[27];          /* weights */
} or_lattice;

static int or_lattice_get(int lattice, or_lattice *L)
{
    int i;
    if (lattice == OR_D2Q9) {
        L->d = 2;
        L->q = 9;
        L->c = C_D2Q9;
        L->w[0] = 4.0 / 9.0;
        for (i = 1; i <= 4; ++i) L->w[i] = 1.0 / 9.0;
        for (i = 5; i <= 8; ++i) L->w[i] = 1.0 / 36.0;
        return OR_OK;
    }
    if (lattice == OR_D3Q19) {
        L->d = 3;
        L->q = 19;
        L->c = C_D3Q27;
        L->w[0] = 1.0 / 3.0;
        for (i = 1; i <= 6; ++i) L->w[i] = 1.0 / 18.0;
        for (i = 7; i <= 18; ++i) L->w[i] = 1.0 / 36.0;
        return OR_OK;
    }
    if (lattice == OR_D3Q27) {
        L->d = 3;
        L->q = 27;
        L->c = C_D3Q27;
        L->w[0] = 8.0 / 27.0;
        for (i = 1; i <= 6; ++i) L->w[i] = 2.0 / 27.0;
        for (i = 7; i <= 18; ++i) L->w[i] = 1.0 / 54.0;
        for (i = 19; i <= 26; ++i) L->w[i] = 1.0 / 216.0;
        return OR_OK;
    }
    return OR_EINVAL;
}

/* Exported copy of the tables, for the invariant tests. */
int oracle_lattice(int lattice, int *d, int *q, int *c_out, double *w_out)
{
    or_lattice L;
    int i, a;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    *d = L.d;
    *q = L.q;
    for (i = 0; i < L.q; ++i) {
        for (a = 0; a < 3; ++a) c_out[3 * i + a] = L.c[i][a];
        w_out[i] = L.w[i];
    }
    return OR_OK;
}

/* Quadrature weights of Table 3 for the volume-fraction cell integral,
 * indexed by the number of axes along which the volume fraction varies
 * (D1Q3, D2Q5, D3Q7; diagonals are not used).  Returns varpi_0 and
 * varpi_{i != 0}. */
int oracle_quad_weights(int n_axes, double *w0, double *wi)
{
    switch (n_axes) {
    case 1: *w0 = 1.0 / 2.0; *wi = 1.0 / 4.0; return OR_OK;
    case 2: *w0 = 1.0 / 3.0; *wi = 1.0 / 6.0; return OR_OK;
    case 3: *w0 = 1.0 / 6.0; *wi = 5.0 / 36.0; return OR_OK;
    default: return OR_EINVAL;
    }
}

static int popcount3(int m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1); }

/* quad_axes == OR_QUAD_NONE: no cell integral, I = phi, i.e. the density
 * sum f / phi of the earlier VANSE schemes the paper corrects (used only to
 * show what the correction changes). */
#define OR_QUAD_NONE 8

static int or_check(const or_lattice *L, const int64_t dims[3], int quad_axes)
{
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return OR_EINVAL;
    if (L->d == 2 && dims[2] != 1) return OR_EINVAL;
    if (quad_axes == OR_QUAD_NONE) return OR_OK;
    if (quad_axes < 0 || quad_axes > 7) return OR_EINVAL;
    if (L->d == 2 && (quad_axes & 4)) return OR_EINVAL;
    return OR_OK;
}

static int64_t wrap(int64_t a, int64_t n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* ---------------------------------------------------------------------------
 * Volume-fraction operators at one cell (Section "Lattice Boltzmann scheme
 * for VANSE"):
 *   I   = cell integral of phi, in the rearranged (Laplacian) form of
 *         eq. latDiffRuleIIre: phi + varpi_{i!=0} * lap(phi), with the
 *         lattice Laplacian sum_{alpha in quad axes} (phi(x+e) + phi(x-e)
 *         - 2 phi(x));
 *   g   = grad(phi) by central differences, (phi(x+e) - phi(x-e)) / 2.
 * ------------------------------------------------------------------------ */
static void or_eps_ops(const or_lattice *L, const int64_t dims[3], const double *eps,
                       int64_t x, int64_t y, int64_t z, int quad_mask, double *I,
                       double g[3])
{
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t cell = (z * ny + y) * nx + x;
    const double e = eps[cell];
    double ep[3], em[3];
    double S = 0.0, wi, w0;
    int a, n_axes = popcount3(quad_mask & 7);

    ep[0] = eps[(z * ny + y) * nx + wrap(x + 1, nx)];
    em[0] = eps[(z * ny + y) * nx + wrap(x - 1, nx)];
    ep[1] = eps[(z * ny + wrap(y + 1, ny)) * nx + x];
    em[1] = eps[(z * ny + wrap(y - 1, ny)) * nx + x];
    ep[2] = eps[(wrap(z + 1, nz) * ny + y) * nx + x];
    em[2] = eps[(wrap(z - 1, nz) * ny + y) * nx + x];

    for (a = 0; a < 3; ++a) {
        if (quad_mask & (1 << a)) {
            S = S + ep[a];
            S = S + em[a];
        }
    }
    if (quad_mask == OR_QUAD_NONE)
        *I = e;
    else {
        oracle_quad_weights(n_axes, &w0, &wi);
        *I = e + wi * (S - (double)(2 * n_axes) * e);
    }

    for (a = 0; a < 3; ++a) g[a] = (a < L->d) ? 0.5 * (ep[a] - em[a]) : 0.0;
}

/* Macroscopic quantities of one cell from its populations fc[0..Q-1]
 * (eqs. density, velocity, pressForce):
 *   M0 = sum_i f_i,  j = sum_i xi_i f_i,
 *   rho = M0 / I,  p = rho c_s^2,
 *   F = p grad(phi) + F_ext (+ a per-cell force),
 *   u = (j + F/2) / M0. */
static void or_macro(const or_lattice *L, const double *fc, double I, const double g[3],
                     const double fsum[3], double *M0_out, double *rho_out,
                     double *p_out, double j_out[3], double F_out[3], double u_out[3])
{
    double M0 = 0.0, j[3] = {0.0, 0.0, 0.0};
    double rho, p;
    int i, a;
    for (i = 0; i < L->q; ++i) {
        M0 = M0 + fc[i];
        for (a = 0; a < 3; ++a) j[a] = j[a] + (double)L->c[i][a] * fc[i];
    }
    rho = M0 / I;
    p = rho / 3.0;
    for (a = 0; a < 3; ++a) {
        if (a < L->d) {
            F_out[a] = p * g[a] + fsum[a];
            u_out[a] = (j[a] + 0.5 * F_out[a]) / M0;
        } else {
            F_out[a] = 0.0; /* a 2-D lattice carries no z component */
            u_out[a] = 0.0;
        }
        j_out[a] = j[a];
    }
    *M0_out = M0;
    *rho_out = rho;
    *p_out = p;
}

static void or_force_sum(const double *fext, const double *force, int64_t cell,
                         int64_t ncells, double out[3])
{
    int a;
    for (a = 0; a < 3; ++a) {
        out[a] = fext ? fext[a] : 0.0;
        if (force) out[a] = out[a] + force[a * ncells + cell];
    }
}

/* ---------------------------------------------------------------------------
 * One time step n -> n+1 (eq. lbe with the equilibrium of eq. feq, the
 * density of eq. density, the velocity of eq. velocity, the Guo forcing
 * term Omega^F and the pressure-correction force of eq. pressForce).
 *
 *   eps       volume fraction at the current time level t_n, per cell
 *   quad_axes bitmask of the axes used by the cell-integral quadrature
 *             (1 = x, 2 = y, 4 = z); 0 selects all d axes
 *   force     optional per-cell external force density, SoA [3][ncells]
 *   fext      constant external force density (may be NULL)
 *   fin/fout  populations at t_n / t_{n+1}, AoS [ncells][Q]; must differ
 * ------------------------------------------------------------------------ */
int oracle_step(int lattice, const int64_t dims[3], double tau, const double *eps,
                int quad_axes, const double *force, const double *fext,
                const double *fin, double *fout, int nthreads)
{
    or_lattice L;
    int64_t nx, ny, nz, ncells, row;
    double omega;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    if (or_check(&L, dims, quad_axes) != OR_OK) return OR_EINVAL;
    if (!(tau > 0.5) || !isfinite(tau) || fin == fout) return OR_EINVAL;
    if (quad_axes == 0) quad_axes = (L.d == 2) ? 3 : 7;
    nx = dims[0];
    ny = dims[1];
    nz = dims[2];
    ncells = nx * ny * nz;
    omega = 1.0 / tau;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (row = 0; row < ny * nz; ++row) {
        const int64_t z = row / ny, y = row % ny;
        int64_t x;
        for (x = 0; x < nx; ++x) {
            const int64_t cell = (z * ny + y) * nx + x;
            const double *fc = fin + cell * L.q;
            double I, g[3], fs[3], M0, rho, p, j[3], F[3], u[3], uu, uF;
            int i;
            or_eps_ops(&L, dims, eps, x, y, z, quad_axes, &I, g);
            or_force_sum(fext, force, cell, ncells, fs);
            or_macro(&L, fc, I, g, fs, &M0, &rho, &p, j, F, u);
            uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
            for (i = 0; i < L.q; ++i) {
                const int cx = L.c[i][0], cy = L.c[i][1], cz = L.c[i][2];
                const double cu = cx * u[0] + cy * u[1] + cz * u[2];
                const double cF = cx * F[0] + cy * F[1] + cz * F[2];
                const double feq =
                    L.w[i] * M0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                const double om =
                    (1.0 - 0.5 * omega) * L.w[i] * (3.0 * cF - 3.0 * uF + 9.0 * cu * cF);
                const double fstar = fc[i] - omega * (fc[i] - feq) + om;
                const int64_t dest =
                    (wrap(z + cz, nz) * ny + wrap(y + cy, ny)) * nx + wrap(x + cx, nx);
                fout[dest * L.q + i] = fstar;
            }
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Textbook BGK step with Guo forcing and no volume fraction: density
 * rho = sum f, u = (j + F/2)/rho, the same second-order equilibrium and the
 * same forcing term.  With phi == 1 the VANSE step above must reproduce this
 * bit for bit (I = 1 and grad(phi) = 0 exactly).  Written out separately on
 * purpose, with the same operation order for the shared terms.
 * ------------------------------------------------------------------------ */
int oracle_bgk_step(int lattice, const int64_t dims[3], double tau, const double *fext,
                    const double *fin, double *fout, int nthreads)
{
    or_lattice L;
    int64_t nx, ny, nz, row;
    double omega;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    if (or_check(&L, dims, 0) != OR_OK) return OR_EINVAL;
    if (!(tau > 0.5) || !isfinite(tau) || fin == fout) return OR_EINVAL;
    nx = dims[0];
    ny = dims[1];
    nz = dims[2];
    omega = 1.0 / tau;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (row = 0; row < ny * nz; ++row) {
        const int64_t z = row / ny, y = row % ny;
        int64_t x;
        for (x = 0; x < nx; ++x) {
            const int64_t cell = (z * ny + y) * nx + x;
            const double *fc = fin + cell * L.q;
            double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, F[3], u[3], uu, uF;
            int i, a;
            for (i = 0; i < L.q; ++i) {
                rho = rho + fc[i];
                for (a = 0; a < 3; ++a) j[a] = j[a] + (double)L.c[i][a] * fc[i];
            }
            for (a = 0; a < 3; ++a) {
                F[a] = (fext && a < L.d) ? fext[a] : 0.0;
                u[a] = (j[a] + 0.5 * F[a]) / rho;
            }
            uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
            for (i = 0; i < L.q; ++i) {
                const int cx = L.c[i][0], cy = L.c[i][1], cz = L.c[i][2];
                const double cu = cx * u[0] + cy * u[1] + cz * u[2];
                const double cF = cx * F[0] + cy * F[1] + cz * F[2];
                const double feq =
                    L.w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                const double om =
                    (1.0 - 0.5 * omega) * L.w[i] * (3.0 * cF - 3.0 * uF + 9.0 * cu * cF);
                const int64_t dest =
                    (wrap(z + cz, nz) * ny + wrap(y + cy, ny)) * nx + wrap(x + cx, nx);
                fout[dest * L.q + i] = fc[i] - omega * (fc[i] - feq) + om;
            }
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Single-cell kernels exposed for the moment-identity tests: the equilibrium
 * f^eq_i(M0, u) of eq. feq (with rho * I = M0) and the forcing term
 * Omega^F_i(u, F, tau).
 * ------------------------------------------------------------------------ */
int oracle_feq(int lattice, double M0, const double u[3], double *feq)
{
    or_lattice L;
    double uu;
    int i;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    uu = u[0] * u[0] + u[1] * u[1] + (L.d == 3 ? u[2] * u[2] : 0.0);
    for (i = 0; i < L.q; ++i) {
        const double cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
        feq[i] = L.w[i] * M0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
    return OR_OK;
}

int oracle_forcing(int lattice, double tau, const double u[3], const double F[3],
                   double *om)
{
    or_lattice L;
    double uF, omega = 1.0 / tau;
    int i;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    uF = u[0] * F[0] + u[1] * F[1] + (L.d == 3 ? u[2] * F[2] : 0.0);
    for (i = 0; i < L.q; ++i) {
        const double cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
        const double cF = L.c[i][0] * F[0] + L.c[i][1] * F[1] + L.c[i][2] * F[2];
        om[i] = (1.0 - 0.5 * omega) * L.w[i] * (3.0 * cF - 3.0 * uF + 9.0 * cu * cF);
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Initial populations (eq. equilibrium): f_i = w_i rho0 phi (...), i.e. the
 * equilibrium of M0 = rho0(x) * phi(x, 0) and u0(x).  rho0 == NULL means 1,
 * u0 == NULL means 0; u0 is SoA [d][ncells].
 * ------------------------------------------------------------------------ */
int oracle_init(int lattice, const int64_t dims[3], const double *eps0,
                const double *rho0, const double *u0, double *f)
{
    or_lattice L;
    int64_t ncells, cell;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    if (or_check(&L, dims, 0) != OR_OK) return OR_EINVAL;
    ncells = dims[0] * dims[1] * dims[2];
    for (cell = 0; cell < ncells; ++cell) {
        double u[3] = {0.0, 0.0, 0.0};
        const double r = rho0 ? rho0[cell] : 1.0;
        int a;
        if (u0)
            for (a = 0; a < L.d; ++a) u[a] = u0[a * ncells + cell];
        oracle_feq(lattice, r * eps0[cell], u, f + cell * L.q);
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Macroscopic output at time t_n: rho (effective density), p = rho c_s^2 and
 * the force-shifted velocity u, SoA u[d][ncells].  Same operators as the
 * step, applied to the current populations.
 * ------------------------------------------------------------------------ */
int oracle_moments(int lattice, const int64_t dims[3], const double *eps, int quad_axes,
                   const double *force, const double *fext, const double *f,
                   double *rho_out, double *p_out, double *u_out)
{
    or_lattice L;
    int64_t nx, ny, nz, ncells, z, y, x;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    if (or_check(&L, dims, quad_axes) != OR_OK) return OR_EINVAL;
    if (quad_axes == 0) quad_axes = (L.d == 2) ? 3 : 7;
    nx = dims[0];
    ny = dims[1];
    nz = dims[2];
    ncells = nx * ny * nz;
    for (z = 0; z < nz; ++z)
        for (y = 0; y < ny; ++y)
            for (x = 0; x < nx; ++x) {
                const int64_t cell = (z * ny + y) * nx + x;
                double I, g[3], fs[3], M0, rho, p, j[3], F[3], u[3];
                int a;
                or_eps_ops(&L, dims, eps, x, y, z, quad_axes, &I, g);
                or_force_sum(fext, force, cell, ncells, fs);
                or_macro(&L, f + cell * L.q, I, g, fs, &M0, &rho, &p, j, F, u);
                if (rho_out) rho_out[cell] = rho;
                if (p_out) p_out[cell] = p;
                if (u_out)
                    for (a = 0; a < L.d; ++a) u_out[a * ncells + cell] = u[a];
            }
    return OR_OK;
}

/* Neumaier's compensated summation, in a fixed serial order. */
typedef struct { double s, c; } or_ksum;
static void ksum_add(or_ksum *k, double v)
{
    const double t = k->s + v;
    if (fabs(k->s) >= fabs(v))
        k->c = k->c + ((k->s - t) + v);
    else
        k->c = k->c + ((v - t) + k->s);
    k->s = t;
}

/* Global diagnostics at t_n: out[0] = sum_x M0 (the volume-fraction weighted
 * mass, sum rho*I), out[1..3] = sum_x j, out[4..6] = sum_x F. */
int oracle_diagnostics(int lattice, const int64_t dims[3], const double *eps,
                       int quad_axes, const double *force, const double *fext,
                       const double *f, double *out)
{
    or_lattice L;
    or_ksum acc[7];
    int64_t nx, ny, nz, ncells, z, y, x;
    int k;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    if (or_check(&L, dims, quad_axes) != OR_OK) return OR_EINVAL;
    if (quad_axes == 0) quad_axes = (L.d == 2) ? 3 : 7;
    nx = dims[0];
    ny = dims[1];
    nz = dims[2];
    ncells = nx * ny * nz;
    memset(acc, 0, sizeof acc);
    for (z = 0; z < nz; ++z)
        for (y = 0; y < ny; ++y)
            for (x = 0; x < nx; ++x) {
                const int64_t cell = (z * ny + y) * nx + x;
                double I, g[3], fs[3], M0, rho, p, j[3], F[3], u[3];
                int a;
                or_eps_ops(&L, dims, eps, x, y, z, quad_axes, &I, g);
                or_force_sum(fext, force, cell, ncells, fs);
                or_macro(&L, f + cell * L.q, I, g, fs, &M0, &rho, &p, j, F, u);
                ksum_add(&acc[0], M0);
                for (a = 0; a < 3; ++a) {
                    ksum_add(&acc[1 + a], j[a]);
                    ksum_add(&acc[4 + a], F[a]);
                }
            }
    for (k = 0; k < 7; ++k) out[k] = acc[k].s + acc[k].c;
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Separable volume fraction driver: phi(x, t_n) = eps_mean + m(n) pert(x),
 * m(n) = cos(2 pi n / period) (period <= 0: m = 1).  Runs steps n0 ..
 * n0+nsteps-1 on f (in place from the caller's view; work is a second
 * population array of the same size).  eps_buf receives phi(t_n) of the last
 * time level touched (t_{n0+nsteps}) on return, for the moments call.
 * ------------------------------------------------------------------------ */
double oracle_modulation(int64_t n, double period)
{
    if (!(period > 0.0)) return 1.0;
    return cos(2.0 * M_PI * (double)n / period);
}

int oracle_eps_at(const int64_t dims[3], double eps_mean, const double *pert,
                  double period, int64_t n, double *eps_out)
{
    const int64_t ncells = dims[0] * dims[1] * dims[2];
    const double m = oracle_modulation(n, period);
    int64_t c;
    for (c = 0; c < ncells; ++c) eps_out[c] = eps_mean + m * (pert ? pert[c] : 0.0);
    return OR_OK;
}

int oracle_run_separable(int lattice, const int64_t dims[3], double tau, double eps_mean,
                         const double *pert, double period, int quad_axes,
                         const double *force, const double *fext, int64_t n0,
                         int64_t nsteps, double *f, double *work, double *eps_buf,
                         int nthreads)
{
    or_lattice L;
    int64_t n, ncells;
    double *a = f, *b = work;
    int rc = OR_OK;
    if (or_lattice_get(lattice, &L) != OR_OK) return OR_EINVAL;
    ncells = dims[0] * dims[1] * dims[2];
    for (n = n0; n < n0 + nsteps; ++n) {
        double *t;
        oracle_eps_at(dims, eps_mean, pert, period, n, eps_buf);
        rc = oracle_step(lattice, dims, tau, eps_buf, quad_axes, force, fext, a, b, nthreads);
        if (rc != OR_OK) return rc;
        t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, (size_t)(ncells * L.q) * sizeof(double));
    oracle_eps_at(dims, eps_mean, pert, period, n0 + nsteps, eps_buf);
    return rc;
}
