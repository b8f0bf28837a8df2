/*
 * vanse_mms.c -- method-of-manufactured-solutions harness for the CPU oracle
 * (Section "Numerical validation" of arXiv:2208.09267).
 *
 * TEST INFRASTRUCTURE ONLY (see vanse_oracle.c).
 *
 * The five examples of the paper are prescribed fields (phi, u, p) in
 * physical units on the periodic box [0, 2 m)^d with rho = 1 kg/m^3 and
 * nu = 0.1 m^2/s.  The manufactured force is the residual of the VANSE
 * momentum equation (eq. vansEquMom without the phi F term),
 *
 *   F_MMS = d_t(phi rho u) + div(phi rho u u) + phi grad p
 *           - nu div(phi rho (grad u + u grad)),
 *
 * and the lattice Boltzmann forcing carries F_MMS + F_PC.
 *
 * Example 5 is printed with a static phi and u = (0.5 + 1/phi)(1, 1, 1),
 * which violates the mass equation the examples are built to satisfy.  It is
 * read here as the travelling form of Examples 3 and 4 in three axes:
 * phi = 0.5 + 0.4 prod_a sin(pi (x_a - t/2)), p = prod_a sin(pi (x_a - t/2)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_step(int lattice, const int64_t dims[3], double tau, const double *eps,
                int quad_axes, const double *force, const double *fext,
                const double *fin, double *fout, int nthreads);
int oracle_init(int lattice, const int64_t dims[3], const double *eps0,
                const double *rho0, const double *u0, double *f);
int oracle_moments(int lattice, const int64_t dims[3], const double *eps, int quad_axes,
                   const double *force, const double *fext, const double *f,
                   double *rho_out, double *p_out, double *u_out);

#define MMS_L 2.0
#define MMS_NU 0.1

/* Spatial dimension, active (travelling) axes and quadrature axes of each
 * example.  Example 3 is one-dimensional in phi but its velocity has two
 * components, so it runs on a two-dimensional lattice with one row. */
int oracle_mms_info(int ex, int *dim, int *quad_axes, int *transient)
{
    switch (ex) {
    case 1: *dim = 2; *quad_axes = 3; *transient = 0; return 0;
    case 2: *dim = 3; *quad_axes = 7; *transient = 0; return 0;
    case 3: *dim = 2; *quad_axes = 1; *transient = 1; return 0;
    case 4: *dim = 2; *quad_axes = 3; *transient = 1; return 0;
    case 5: *dim = 3; *quad_axes = 7; *transient = 1; return 0;
    default: return -1;
    }
}

/* Exact fields of example ex at position X (3 components; unused ones are
 * ignored) and time t. */
int oracle_mms_fields_at(int ex, const double X[3], double t, double *phi, double u[3],
                         double *p)
{
    const double pi = M_PI;
    u[0] = u[1] = u[2] = 0.0;
    if (ex == 1) {
        const double sx = sin(pi * X[0]), cx = cos(pi * X[0]);
        const double sy = sin(pi * X[1]), cy = cos(pi * X[1]);
        *phi = 0.5 + 0.4 * sx * sy;
        u[0] = 2.0 * (-(sx * sx) * sy * cy);
        u[1] = 2.0 * ((sy * sy) * sx * cx);
        *p = sx * sy;
        return 0;
    }
    if (ex == 2) {
        const double sx = sin(pi * X[0]), cx = cos(pi * X[0]);
        const double sy = sin(pi * X[1]), cy = cos(pi * X[1]);
        const double sz = sin(pi * X[2]), cz = cos(pi * X[2]);
        *phi = 0.5 + 0.4 * sx * sy * sz;
        u[0] = (sx * sx) * sy * cy * sz * cz;
        u[1] = (sy * sy) * sx * cx * sz * cz;
        u[2] = -2.0 * (sz * sz) * sx * cx * sy * cy;
        *p = sx * sy * sz;
        return 0;
    }
    if (ex >= 3 && ex <= 5) {
        const int na = ex - 2; /* active axes: x; x,y; x,y,z */
        double prod = 1.0, psi;
        int a;
        for (a = 0; a < na; ++a) prod *= sin(pi * (X[a] - 0.5 * t));
        *phi = 0.5 + 0.4 * prod;
        psi = 0.5 + 1.0 / *phi;
        for (a = 0; a < na; ++a) u[a] = psi;
        *p = prod;
        return 0;
    }
    return -1;
}

/* F_MMS by nested central finite differences of the exact fields with step
 * h in space and time (the paper computes it with central differences). */
int oracle_mms_force_fd(int ex, const double X[3], double t, double nu, double h,
                        double F[3])
{
    double phi, u[3], p;
    double Y[3];
    int a, b, s;
    if (oracle_mms_fields_at(ex, X, t, &phi, u, &p) != 0) return -1;
    for (a = 0; a < 3; ++a) F[a] = 0.0;

    /* d_t(phi u) */
    {
        double php, upl[3], pp, phm, umi[3], pm;
        oracle_mms_fields_at(ex, X, t + h, &php, upl, &pp);
        oracle_mms_fields_at(ex, X, t - h, &phm, umi, &pm);
        for (a = 0; a < 3; ++a) F[a] += (php * upl[a] - phm * umi[a]) / (2.0 * h);
    }
    /* div(phi u u) and phi grad p */
    for (b = 0; b < 3; ++b) {
        double php, upl[3], pp, phm, umi[3], pm;
        memcpy(Y, X, sizeof Y);
        Y[b] = X[b] + h;
        oracle_mms_fields_at(ex, Y, t, &php, upl, &pp);
        Y[b] = X[b] - h;
        oracle_mms_fields_at(ex, Y, t, &phm, umi, &pm);
        for (a = 0; a < 3; ++a)
            F[a] += (php * upl[a] * upl[b] - phm * umi[a] * umi[b]) / (2.0 * h);
        F[b] += phi * (pp - pm) / (2.0 * h);
    }
    /* - nu div(phi (grad u + u grad)): outer difference over b of
     * phi (d_b u_a + d_a u_b), each evaluated by an inner difference. */
    for (b = 0; b < 3; ++b) {
        double V[2][3];
        for (s = 0; s < 2; ++s) {
            double Z[3], ph0, u0[3], p0, G[3][3]; /* G[k][a] = d_k u_a */
            int k;
            memcpy(Z, X, sizeof Z);
            Z[b] = X[b] + (s == 0 ? h : -h);
            oracle_mms_fields_at(ex, Z, t, &ph0, u0, &p0);
            for (k = 0; k < 3; ++k) {
                double W[3], php, upl[3], pp, phm, umi[3], pm;
                memcpy(W, Z, sizeof W);
                W[k] = Z[k] + h;
                oracle_mms_fields_at(ex, W, t, &php, upl, &pp);
                W[k] = Z[k] - h;
                oracle_mms_fields_at(ex, W, t, &phm, umi, &pm);
                for (a = 0; a < 3; ++a) G[k][a] = (upl[a] - umi[a]) / (2.0 * h);
            }
            for (a = 0; a < 3; ++a) V[s][a] = ph0 * (G[b][a] + G[a][b]);
        }
        for (a = 0; a < 3; ++a) F[a] -= nu * (V[0][a] - V[1][a]) / (2.0 * h);
    }
    return 0;
}

/* Closed form of F_MMS for the travelling examples 3-5.  With a the
 * indicator of the active axes, psi = 1/2 + 1/phi and u = psi a, the mass
 * equation holds exactly and the residual reduces to
 *   F_a = -a_a (a.grad phi)/phi^2 + phi d_a p
 *         + nu [ a_a (lap phi/phi - |grad phi|^2/phi^2)
 *              + sum_b a_b (d_a d_b phi/phi - d_a phi d_b phi/phi^2) ].
 * s[k], c[k] are sin and cos of pi (x_k - t/2) on the active axes. */
static void mms_force_travel(int na, const double *s, const double *c, double nu,
                             double F[3])
{
    const double pi = M_PI;
    double prod = 1.0, phi, dphi[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
    double d2[3][3], lap = 0.0, g2 = 0.0, adphi = 0.0;
    int a, b, k;
    for (a = 0; a < na; ++a) prod *= s[a];
    phi = 0.5 + 0.4 * prod;
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) d2[a][b] = 0.0;
    for (a = 0; a < na; ++a) {
        double rest = 1.0;
        for (k = 0; k < na; ++k)
            if (k != a) rest *= s[k];
        dp[a] = pi * c[a] * rest;
        dphi[a] = 0.4 * dp[a];
        for (b = 0; b < na; ++b) {
            if (b == a) {
                d2[a][a] = -0.4 * pi * pi * prod;
            } else {
                double rest2 = 1.0;
                for (k = 0; k < na; ++k)
                    if (k != a && k != b) rest2 *= s[k];
                d2[a][b] = 0.4 * pi * pi * c[a] * c[b] * rest2;
            }
        }
    }
    for (a = 0; a < na; ++a) {
        lap += d2[a][a];
        g2 += dphi[a] * dphi[a];
        adphi += dphi[a];
    }
    for (a = 0; a < 3; ++a) {
        const double act = (a < na) ? 1.0 : 0.0;
        double visc = act * (lap / phi - g2 / (phi * phi));
        for (b = 0; b < na; ++b) visc += d2[a][b] / phi - dphi[a] * dphi[b] / (phi * phi);
        F[a] = -act * adphi / (phi * phi) + phi * dp[a] + nu * visc;
    }
}

int oracle_mms_force_exact(int ex, const double X[3], double t, double nu, double F[3])
{
    double s[3], c[3];
    int a, na;
    if (ex < 3 || ex > 5) return -1;
    na = ex - 2;
    for (a = 0; a < na; ++a) {
        s[a] = sin(M_PI * (X[a] - 0.5 * t));
        c[a] = cos(M_PI * (X[a] - 0.5 * t));
    }
    mms_force_travel(na, s, c, nu, F);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Convergence run of one example at resolution N.
 *
 * Physical set-up: L = 2 m periodic, rho = 1, nu = 0.1, nodes at x_k = k dx,
 * dx = L/N.  Diffusive scaling with fixed tau: nu_lu = (tau - 1/2)/3 and
 * dt = nu_lu dx^2 / nu.  Unit conversions: u_lu = u dt/dx,
 * p_lu = 1/3 + p (dt/dx)^2, F_lu = F dt^2/dx.
 * Initial state: equilibrium of M0 = rho0 phi(x, 0), rho0 = 3 p_lu, u0.
 *
 * At n_samples evenly spaced times up to t_end, errs receives
 * [u L1, u L2, u Linf, p L1, p L2, p Linf] of the velocity (Euclidean norm
 * per node) and of the mean-free pressure, both in physical units, and
 * times the sample times.  Returns the number of steps run, or < 0.
 * ------------------------------------------------------------------------ */
int64_t oracle_mms_run_q(int ex, int lattice, int N, double tau, double t_end, int n_samples,
                         int nthreads, int quad_override, double *errs, double *times);

int64_t oracle_mms_run(int ex, int lattice, int N, double tau, double t_end, int n_samples,
                       int nthreads, double *errs, double *times)
{
    return oracle_mms_run_q(ex, lattice, N, tau, t_end, n_samples, nthreads, -1, errs, times);
}

/* As oracle_mms_run; quad_override >= 0 replaces the example's quadrature
 * axes (8 = no cell-integral correction, the ablation). */
int64_t oracle_mms_run_q(int ex, int lattice, int N, double tau, double t_end, int n_samples,
                         int nthreads, int quad_override, double *errs, double *times)
{
    int dim, quad, transient;
    int64_t dims[3], ncells, cell, nsteps, n;
    double dx, dt, nu_lu, us, ps, fs;
    double *eps = NULL, *force = NULL, *fa = NULL, *fb = NULL, *rho0 = NULL, *u0 = NULL;
    double *rho = NULL, *p = NULL, *u = NULL, *pex = NULL, *uex = NULL;
    double *sn = NULL, *cs = NULL;
    int q, k, next_sample = 1, rc = 0;

    if (oracle_mms_info(ex, &dim, &quad, &transient) != 0) return -1;
    if (quad_override >= 0) quad = quad_override;
    if (dim == 2 && lattice != 0) return -1;
    if (dim == 3 && lattice == 0) return -1;
    if (N < 2 || n_samples < 1 || !(tau > 0.5)) return -1;
    q = (lattice == 0) ? 9 : (lattice == 1 ? 19 : 27);
    dims[0] = N;
    dims[1] = (ex == 3) ? 1 : N;
    dims[2] = (dim == 3) ? N : 1;
    ncells = dims[0] * dims[1] * dims[2];
    dx = MMS_L / N;
    nu_lu = (tau - 0.5) / 3.0;
    dt = nu_lu * dx * dx / MMS_NU;
    nsteps = llround(t_end / dt);
    if (nsteps < n_samples) nsteps = n_samples;
    us = dt / dx;
    ps = (dt / dx) * (dt / dx);
    fs = dt * dt / dx;

    eps = malloc(sizeof(double) * ncells);
    force = malloc(sizeof(double) * 3 * ncells);
    fa = malloc(sizeof(double) * q * ncells);
    fb = malloc(sizeof(double) * q * ncells);
    rho0 = malloc(sizeof(double) * ncells);
    u0 = malloc(sizeof(double) * 3 * ncells);
    rho = malloc(sizeof(double) * ncells);
    p = malloc(sizeof(double) * ncells);
    u = malloc(sizeof(double) * 3 * ncells);
    pex = malloc(sizeof(double) * ncells);
    uex = malloc(sizeof(double) * 3 * ncells);
    sn = malloc(sizeof(double) * 3 * N);
    cs = malloc(sizeof(double) * 3 * N);
    if (!eps || !force || !fa || !fb || !rho0 || !u0 || !rho || !p || !u || !pex || !uex ||
        !sn || !cs) {
        rc = -2;
        goto done;
    }
    memset(force, 0, sizeof(double) * 3 * ncells);

    /* exact fields at t = 0 -> initial populations */
    for (cell = 0; cell < ncells; ++cell) {
        const int64_t x = cell % dims[0], y = (cell / dims[0]) % dims[1],
                      z = cell / (dims[0] * dims[1]);
        double X[3] = {x * dx, y * dx, z * dx}, ph, uu[3], pp;
        int a;
        oracle_mms_fields_at(ex, X, 0.0, &ph, uu, &pp);
        eps[cell] = ph;
        rho0[cell] = 3.0 * (1.0 / 3.0 + pp * ps);
        for (a = 0; a < 3; ++a) u0[a * ncells + cell] = uu[a] * us;
    }
    oracle_init(lattice, dims, eps, rho0, u0, fa);

    for (n = 0; n <= nsteps; ++n) {
        const double t = (double)n * dt;
        int do_sample = 0;
        /* phi(t_n) and F_MMS(t_n) in lattice units */
        if (transient || n == 0) {
            if (transient) {
                int a, i;
                for (a = 0; a < ex - 2; ++a)
                    for (i = 0; i < N; ++i) {
                        sn[a * N + i] = sin(M_PI * (i * dx - 0.5 * t));
                        cs[a * N + i] = cos(M_PI * (i * dx - 0.5 * t));
                    }
            }
            /* cells are independent: the same values in any thread count */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
            for (cell = 0; cell < ncells; ++cell) {
                const int64_t x = cell % dims[0], y = (cell / dims[0]) % dims[1],
                              z = cell / (dims[0] * dims[1]);
                const int64_t ix[3] = {x, y, z};
                double F[3];
                int a;
                if (transient) {
                    double s3[3], c3[3], prod = 1.0;
                    for (a = 0; a < ex - 2; ++a) {
                        s3[a] = sn[a * N + ix[a]];
                        c3[a] = cs[a * N + ix[a]];
                        prod *= s3[a];
                    }
                    eps[cell] = 0.5 + 0.4 * prod;
                    mms_force_travel(ex - 2, s3, c3, MMS_NU, F);
                } else {
                    double X[3] = {x * dx, y * dx, z * dx};
                    oracle_mms_force_fd(ex, X, t, MMS_NU, 1e-4, F);
                }
                for (a = 0; a < 3; ++a) force[a * ncells + cell] = F[a] * fs;
            }
        }
        if (next_sample <= n_samples && n == (nsteps * next_sample) / n_samples)
            do_sample = 1;
        if (do_sample) {
            double mp = 0.0, mpe = 0.0;
            double e[6] = {0, 0, 0, 0, 0, 0};
            oracle_moments(lattice, dims, eps, quad, force, NULL, fa, rho, p, u);
            for (cell = 0; cell < ncells; ++cell) {
                const int64_t x = cell % dims[0], y = (cell / dims[0]) % dims[1],
                              z = cell / (dims[0] * dims[1]);
                double X[3] = {x * dx, y * dx, z * dx}, ph, uu[3], pp;
                int a;
                oracle_mms_fields_at(ex, X, t, &ph, uu, &pp);
                pex[cell] = pp;
                for (a = 0; a < 3; ++a) uex[a * ncells + cell] = uu[a];
                mp += p[cell];
                mpe += pp;
            }
            mp /= (double)ncells;
            mpe /= (double)ncells;
            for (cell = 0; cell < ncells; ++cell) {
                double du2 = 0.0, dpv;
                int a;
                for (a = 0; a < dim; ++a) {
                    const double d = u[a * ncells + cell] / us - uex[a * ncells + cell];
                    du2 += d * d;
                }
                dpv = fabs((p[cell] - mp) / ps - (pex[cell] - mpe));
                e[0] += sqrt(du2);
                e[1] += du2;
                if (sqrt(du2) > e[2]) e[2] = sqrt(du2);
                e[3] += dpv;
                e[4] += dpv * dpv;
                if (dpv > e[5]) e[5] = dpv;
            }
            k = next_sample - 1;
            errs[6 * k + 0] = e[0] / ncells;
            errs[6 * k + 1] = sqrt(e[1] / ncells);
            errs[6 * k + 2] = e[2];
            errs[6 * k + 3] = e[3] / ncells;
            errs[6 * k + 4] = sqrt(e[4] / ncells);
            errs[6 * k + 5] = e[5];
            if (times) times[k] = t;
            ++next_sample;
        }
        if (n == nsteps) break;
        if (oracle_step(lattice, dims, tau, eps, quad, force, NULL, fa, fb, nthreads) != 0) {
            rc = -3;
            goto done;
        }
        {
            double *tmp = fa;
            fa = fb;
            fb = tmp;
        }
    }
done:
    free(eps); free(force); free(fa); free(fb); free(rho0); free(u0);
    free(rho); free(p); free(u); free(pex); free(uex); free(sn); free(cs);
    return rc < 0 ? rc : nsteps;
}
