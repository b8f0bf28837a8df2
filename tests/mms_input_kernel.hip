// mms_input_kernel.hip -- TEST INFRASTRUCTURE: device-side inputs of the
// travelling manufactured solutions (Examples 3-5 of the paper's numerical
// validation), so that a GPU convergence run can refresh phi(t_n) and
// F_MMS(t_n) every step with one launch.  Input generation only: it holds no
// lattice Boltzmann arithmetic and is not part of the library (tests load it
// with ctypes; tests/mms_inputs.py is the torch statement of the same fields,
// pinned against the symbolic residual, and a GPU test compares the two).
//
// Active axes A = x (Example 3), x, y (4), x, y, z (5); s_a, c_a = sin, cos
// of pi (x_a - t/2); P = prod_a s_a.
//   phi = 1/2 + 2/5 P,  p = P,  u_a = 1/2 + 1/phi on A,
//   F_a = -[a in A] (sum_b d_b phi)/phi^2 + phi d_a P
//         + nu ([a in A] (lap phi/phi - |grad phi|^2/phi^2)
//               + sum_{b in A} (d_a d_b phi/phi - d_a phi d_b phi/phi^2)).
#include <hip/hip_runtime.h>

#include <cmath>

namespace {

__global__ void __launch_bounds__(256) travel_fields(int na, int nx, int ny, int nz, double dx,
                                                     double t, double nu, double fscale,
                                                     double *__restrict__ phi_out,
                                                     double *__restrict__ force_out, int d)
{
    const long long n = (long long)nx * ny * nz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long long)nx * ny));
    const int idx[3] = {x, y, z};
    double s[3] = {1.0, 1.0, 1.0}, co[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < na; ++a) {
        const double arg = M_PI * (idx[a] * dx - 0.5 * t);
        s[a] = sin(arg);
        co[a] = cos(arg);
    }
    const double P = s[0] * s[1] * s[2];
    const double phi = 0.5 + 0.4 * P;
    // derivatives of P: dP[a] = pi c_a prod_{k != a} s_k, d2P[a][b]
    double dP[3] = {0.0, 0.0, 0.0}, d2P[3][3] = {{0.0}};
    for (int a = 0; a < na; ++a) {
        double r = M_PI * co[a];
        for (int k = 0; k < na; ++k)
            if (k != a) r *= s[k];
        dP[a] = r;
        for (int b = 0; b < na; ++b) {
            if (b == a) {
                d2P[a][a] = -M_PI * M_PI * P;
            } else {
                double q = M_PI * M_PI * co[a] * co[b];
                for (int k = 0; k < na; ++k)
                    if (k != a && k != b) q *= s[k];
                d2P[a][b] = q;
            }
        }
    }
    const double inv = 1.0 / phi, inv2 = inv * inv;
    double sum_dphi = 0.0, lap = 0.0, grad2 = 0.0;
    for (int b = 0; b < na; ++b) {
        sum_dphi += 0.4 * dP[b];
        lap += 0.4 * d2P[b][b];
        grad2 += 0.16 * dP[b] * dP[b];
    }
    phi_out[c] = phi;
    for (int a = 0; a < d; ++a) {
        double F = 0.0;
        if (a < na) {
            double visc = lap * inv - grad2 * inv2;
            for (int b = 0; b < na; ++b)
                visc += 0.4 * d2P[a][b] * inv - 0.16 * dP[a] * dP[b] * inv2;
            F = -sum_dphi * inv2 + phi * dP[a] + nu * visc;
        }
        force_out[(long long)a * n + c] = F * fscale;
    }
}

}  // namespace

// phi(t) [n] and fscale * F_MMS(t) SoA [d][n] (d = 2 for Examples 3-4, 3 for
// Example 5) at the nodes x_k = k dx of an nx x ny x nz lattice, x fastest.
// Asynchronous on `stream`.  Returns 0, or -1 for a bad example.
extern "C" int mms_travel_fields(int ex, int nx, int ny, int nz, double dx, double t, double nu,
                                 double fscale, double *phi, double *force, void *stream)
{
    if (ex < 3 || ex > 5 || nx < 1 || ny < 1 || nz < 1) return -1;
    const int d = ex == 5 ? 3 : 2;
    const long long n = (long long)nx * ny * nz;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    travel_fields<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(ex - 2, nx, ny, nz, dx, t,
                                                                       nu, fscale, phi, force, d);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
