// kernels.hip -- gfx950 kernels of the consistent VANSE lattice Boltzmann
// step (arXiv:2208.09267, Section "Lattice Boltzmann scheme for VANSE").
//
// Data layout in HBM: one population array per solve, SoA f[i][cell] with a
// plane stride padded to 128 elements, cells x fastest.  It is updated in
// place with the AA pattern (Bailey et al., 2009):
//   even time level n: cell x reads slot i of x and writes its post-collision
//                      value for direction i into slot opp(i) of x;
//   odd time level n:  cell x reads slot opp(i) of x - xi_i and writes into
//                      slot i of x + xi_i.
// Each slot is read and written by the same thread within a step, so one
// copy of f suffices and every step moves Q loads + Q stores per cell.
// After an odd step the layout is natural again.
//
// One thread updates one cell; a wave covers 64 consecutive cells of the
// flattened index, so every direction plane is read and written with
// coalesced (at most one line misaligned) 64-wide accesses.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "internal.h"
#include "lattice.h"

namespace vanse {

// ---------------------------------------------------------------------------
// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1, so
// lattice constants indexed by I stay constant expressions.
template <int I, int N, class Fn>
__device__ __forceinline__ void static_for(Fn &&fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1, N>(fn);
    }
}

// a*x + b*y + c*z for compile-time a, b, c in {-1, 0, 1}; zero terms vanish.
template <int A, int B, int C, class R>
__device__ __forceinline__ R dot3(R x, R y, R z)
{
    R s = R(0);
    if constexpr (A == 1) s = s + x;
    if constexpr (A == -1) s = s - x;
    if constexpr (B == 1) s = s + y;
    if constexpr (B == -1) s = s - y;
    if constexpr (C == 1) s = s + z;
    if constexpr (C == -1) s = s - z;
    return s;
}

template <int MODE> struct Storage;
template <> struct Storage<MODE_F64> { using T = double; using R = double; };
template <> struct Storage<MODE_F32S> { using T = float; using R = float; };
template <> struct Storage<MODE_F16S> { using T = __half; using R = float; };

// Decode a stored population into the arithmetic type: f_i itself (FP64), or
// the deviation g_i = f_i - w_i (shifted modes; FP16 stores g_i / w_i).
template <class L, int MODE, int I>
__device__ __forceinline__ typename Storage<MODE>::R decode(typename Storage<MODE>::T v)
{
    if constexpr (MODE == MODE_F16S)
        return float(L::w[I]) * __half2float(v);
    else
        return v;
}

template <class L, int MODE, int I>
__device__ __forceinline__ typename Storage<MODE>::T encode(typename Storage<MODE>::R v)
{
    if constexpr (MODE == MODE_F16S) {
        constexpr float inv_w = float(1.0 / L::w[I]);
        return __float2half_rn(v * inv_w);
    } else {
        return v;
    }
}

// ---------------------------------------------------------------------------
// Position of one cell and its periodic neighbours.
struct Cell {
    int c;
    int X[3];  // x-1, x, x+1 (wrapped)
    int Y[3];  // (y-1, y, y+1) * nx
    int Z[3];  // (z-1, z, z+1) * nx * ny
    __device__ __forceinline__ int at(int dx, int dy, int dz) const
    {
        return Z[dz + 1] + Y[dy + 1] + X[dx + 1];
    }
};

__device__ __forceinline__ Cell locate(const Geometry &g, int c)
{
    Cell k;
    k.c = c;
    const int x = c % g.nx;
    const int yz = c / g.nx;
    const int y = yz % g.ny;
    const int z = yz / g.ny;
    k.X[0] = (x == 0 ? g.nx : x) - 1;
    k.X[1] = x;
    k.X[2] = (x + 1 == g.nx) ? 0 : x + 1;
    k.Y[0] = ((y == 0 ? g.ny : y) - 1) * g.nx;
    k.Y[1] = y * g.nx;
    k.Y[2] = ((y + 1 == g.ny) ? 0 : y + 1) * g.nx;
    k.Z[0] = ((z == 0 ? g.nz : z) - 1) * g.nxy;
    k.Z[1] = z * g.nxy;
    k.Z[2] = ((z + 1 == g.nz) ? 0 : z + 1) * g.nxy;
    return k;
}

// Volume-fraction operators at one cell, at the current time level:
//   I = phi + varpi (sum_{quad axes} (phi(x+e) + phi(x-e)) - 2N phi)
//       (cell integral, eqs. quad / latDiffRuleIIre, Table 3)
//   g = (phi(x+e) - phi(x-e)) / 2  (central-difference gradient of the
//       pressure-correction force)
template <class L, class R>
__device__ __forceinline__ void eps_ops(const R *__restrict__ pert, R eps_mean, R m, R wq,
                                        R n2, int qmask, const Cell &k, R &I, R &gx, R &gy,
                                        R &gz)
{
    const R e0 = eps_mean + m * pert[k.c];
    const R xp = eps_mean + m * pert[k.at(1, 0, 0)];
    const R xm = eps_mean + m * pert[k.at(-1, 0, 0)];
    const R yp = eps_mean + m * pert[k.at(0, 1, 0)];
    const R ym = eps_mean + m * pert[k.at(0, -1, 0)];
    R zp = R(0), zm = R(0);
    if constexpr (L::D == 3) {
        zp = eps_mean + m * pert[k.at(0, 0, 1)];
        zm = eps_mean + m * pert[k.at(0, 0, -1)];
    }
    R S = R(0);
    if (qmask & 1) {
        S = S + xp;
        S = S + xm;
    }
    if (qmask & 2) {
        S = S + yp;
        S = S + ym;
    }
    if constexpr (L::D == 3) {
        if (qmask & 4) {
            S = S + zp;
            S = S + zm;
        }
    }
    I = e0 + wq * (S - n2 * e0);
    gx = R(0.5) * (xp - xm);
    gy = R(0.5) * (yp - ym);
    gz = (L::D == 3) ? R(0.5) * (zp - zm) : R(0);
}

// ---------------------------------------------------------------------------
// BGK collision with Guo forcing of one cell, in place on v[Q].
//   FP64:    v holds f_i; M0 = sum f.
//   shifted: v holds g_i = f_i - w_i; M0 = 1 + sum g (sum w = 1, sum w xi = 0),
//            and the equilibrium deviation f^eq_i - w_i =
//            w_i (dM0 + M0 (3 cu + 9/2 cu^2 - 3/2 uu)) keeps every stored and
//            relaxed quantity small.
template <class L, int MODE, class R>
__device__ __forceinline__ void collide(R (&v)[L::Q], R I, R gx, R gy, R gz, R omega,
                                        R fcoef, R Fex, R Fey, R Fez)
{
    constexpr bool shifted = (MODE != MODE_F64);
    R s0 = R(0), jx = R(0), jy = R(0), jz = R(0);
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        s0 = s0 + v[i];
        if constexpr (L::cx[i] == 1) jx = jx + v[i];
        if constexpr (L::cx[i] == -1) jx = jx - v[i];
        if constexpr (L::cy[i] == 1) jy = jy + v[i];
        if constexpr (L::cy[i] == -1) jy = jy - v[i];
        if constexpr (L::cz[i] == 1) jz = jz + v[i];
        if constexpr (L::cz[i] == -1) jz = jz - v[i];
    });
    const R M0 = shifted ? R(1) + s0 : s0;
    const R rho = M0 / I;               // eq. density
    const R p = rho / R(3);             // p = rho c_s^2
    const R Fx = p * gx + Fex;          // F_PC + F_ext (eq. pressForce)
    const R Fy = p * gy + Fey;
    const R Fz = (L::D == 3) ? p * gz + Fez : R(0);
    const R ux = (jx + R(0.5) * Fx) / M0;  // eq. velocity
    const R uy = (jy + R(0.5) * Fy) / M0;
    const R uz = (L::D == 3) ? (jz + R(0.5) * Fz) / M0 : R(0);
    const R uu = ux * ux + uy * uy + uz * uz;
    const R uF = ux * Fx + uy * Fy + uz * Fz;
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr R w = R(L::w[i]);
        const R cu = dot3<L::cx[i], L::cy[i], L::cz[i]>(ux, uy, uz);
        const R cF = dot3<L::cx[i], L::cy[i], L::cz[i]>(Fx, Fy, Fz);
        const R poly = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
        R feq;
        if constexpr (shifted)
            feq = w * (s0 + M0 * poly);
        else
            feq = w * M0 * (R(1) + poly);
        const R om = fcoef * w * (R(3) * cF - R(3) * uF + R(9) * cu * cF);
        v[i] = v[i] - omega * (v[i] - feq) + om;
    });
}

// ---------------------------------------------------------------------------
// One fused time step (the hot path): phi stencil, Q loads, collision,
// Q stores, for one cell per thread.
template <class L, int MODE, int PARITY>
__global__ void __launch_bounds__(256) step_kernel(StepArgs a)
{
    using T = typename Storage<MODE>::T;
    using R = typename Storage<MODE>::R;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.geo.ncells) return;
    const Cell k = locate(a.geo, c);
    R I, gx, gy, gz;
    eps_ops<L, R>(static_cast<const R *>(a.pert), R(a.eps_mean), R(a.m), R(a.wq), R(a.n2),
                  a.qmask, k, I, gx, gy, gz);

    T *__restrict__ f = static_cast<T *>(a.f);
    const long long S = a.geo.stride;
    R v[L::Q];
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (PARITY == 0) {
            v[i] = decode<L, MODE, i>(f[i * S + c]);
        } else {
            constexpr int o = opp<L>(i);
            v[i] = decode<L, MODE, i>(f[o * S + k.at(-L::cx[i], -L::cy[i], -L::cz[i])]);
        }
    });
    collide<L, MODE, R>(v, I, gx, gy, gz, R(a.omega), R(a.fcoef), R(a.F[0]), R(a.F[1]),
                        R(a.F[2]));
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (PARITY == 0) {
            constexpr int o = opp<L>(i);
            f[o * S + c] = encode<L, MODE, i>(v[i]);
        } else {
            f[i * S + k.at(L::cx[i], L::cy[i], L::cz[i])] = encode<L, MODE, i>(v[i]);
        }
    });
}

// ---------------------------------------------------------------------------
// FP64 view of one cell at time level n (parity = n & 1): populations in
// natural order and the macroscopic quantities of eqs. density, velocity and
// pressForce.  Used off the hot path (moments, diagnostics, export).
template <class L, int MODE>
__device__ __forceinline__ void load_natural(const StepArgs &a, const Cell &k, int parity,
                                             double (&fo)[L::Q])
{
    using T = typename Storage<MODE>::T;
    using R = typename Storage<MODE>::R;
    const T *__restrict__ f = static_cast<const T *>(a.f);
    const long long S = a.geo.stride;
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        T raw;
        if (parity == 0)
            raw = f[i * S + k.c];
        else
            raw = f[opp<L>(i) * S + k.at(-L::cx[i], -L::cy[i], -L::cz[i])];
        const R val = decode<L, MODE, i>(raw);
        if constexpr (MODE == MODE_F64)
            fo[i] = val;
        else
            fo[i] = L::w[i] + double(val);
    });
}

template <class L, int MODE>
__device__ __forceinline__ void macro_f64(const StepArgs &a, const Cell &k, int parity,
                                          double &M0, double (&j)[3], double &rho, double &p,
                                          double (&F)[3], double (&u)[3])
{
    using R = typename Storage<MODE>::R;
    R Ir, gxr, gyr, gzr;
    eps_ops<L, R>(static_cast<const R *>(a.pert), R(a.eps_mean), R(a.m), R(a.wq), R(a.n2),
                  a.qmask, k, Ir, gxr, gyr, gzr);
    const double I = Ir, g[3] = {double(gxr), double(gyr), double(gzr)};
    double fo[L::Q];
    load_natural<L, MODE>(a, k, parity, fo);
    M0 = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        M0 = M0 + fo[i];
        j[0] = j[0] + double(L::cx[i]) * fo[i];
        j[1] = j[1] + double(L::cy[i]) * fo[i];
        j[2] = j[2] + double(L::cz[i]) * fo[i];
    });
    rho = M0 / I;
    p = rho / 3.0;
    for (int d = 0; d < 3; ++d) {
        if (d < L::D) {
            F[d] = p * g[d] + a.F[d];
            u[d] = (j[d] + 0.5 * F[d]) / M0;
        } else {
            F[d] = 0.0;
            u[d] = 0.0;
        }
    }
}

template <class L, int MODE>
__global__ void __launch_bounds__(256) moments_kernel(StepArgs a, int parity,
                                                      double *__restrict__ rho_out,
                                                      double *__restrict__ p_out,
                                                      double *__restrict__ u_out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.geo.ncells) return;
    const Cell k = locate(a.geo, c);
    double M0, j[3], rho, p, F[3], u[3];
    macro_f64<L, MODE>(a, k, parity, M0, j, rho, p, F, u);
    if (rho_out) rho_out[c] = rho;
    if (p_out) p_out[c] = p;
    if (u_out)
        for (int d = 0; d < L::D; ++d) u_out[(long long)d * a.geo.ncells + c] = u[d];
}

template <class L, int MODE>
__global__ void __launch_bounds__(256) populations_kernel(StepArgs a, int parity,
                                                          double *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.geo.ncells) return;
    const Cell k = locate(a.geo, c);
    double fo[L::Q];
    load_natural<L, MODE>(a, k, parity, fo);
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        out[(long long)i * a.geo.ncells + c] = fo[i];
    });
}

// Initial state (eq. equilibrium): f_i = f_i^eq(M0 = rho0 phi(x, 0), u0),
// written in natural order (time level 0 is even).
template <class L, int MODE>
__global__ void __launch_bounds__(256) init_kernel(StepArgs a, const double *__restrict__ rho0,
                                                   const double *__restrict__ u0)
{
    using T = typename Storage<MODE>::T;
    using R = typename Storage<MODE>::R;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.geo.ncells) return;
    const R e = R(a.eps_mean) + R(a.m) * static_cast<const R *>(a.pert)[c];
    const double M0 = (rho0 ? rho0[c] : 1.0) * double(e);
    double u[3] = {0.0, 0.0, 0.0};
    if (u0)
        for (int d = 0; d < L::D; ++d) u[d] = u0[(long long)d * a.geo.ncells + c];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T *__restrict__ f = static_cast<T *>(a.f);
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const double cu = L::cx[i] * u[0] + L::cy[i] * u[1] + L::cz[i] * u[2];
        const double feq = L::w[i] * M0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        if constexpr (MODE == MODE_F64)
            f[i * a.geo.stride + c] = feq;
        else
            f[i * a.geo.stride + c] = encode<L, MODE, i>(R(feq - L::w[i]));
    });
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: a fixed grid of kReduceBlocks blocks, each
// accumulating a fixed strided subset of cells, a wave64 shuffle tree and a
// fixed-order combination of the waves; then one block combines the block
// partials in a fixed order.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&acc)[NV], double *__restrict__ out)
{
    __shared__ double lds[kReduceThreads / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int v = 0; v < NV; ++v) {
        double x = acc[v];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) lds[wave][v] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < kReduceThreads / 64; ++w) s += lds[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

template <class L, int MODE>
__global__ void __launch_bounds__(kReduceThreads) diag_kernel(StepArgs a, int parity,
                                                              double *__restrict__ partials)
{
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int c = blockIdx.x * kReduceThreads + threadIdx.x; c < a.geo.ncells;
         c += gridDim.x * kReduceThreads) {
        const Cell k = locate(a.geo, c);
        double M0, j[3], rho, p, F[3], u[3];
        macro_f64<L, MODE>(a, k, parity, M0, j, rho, p, F, u);
        acc[0] += M0;
        for (int d = 0; d < 3; ++d) {
            acc[1 + d] += j[d];
            acc[4 + d] += F[d];
        }
    }
    block_reduce<7>(acc, partials + 7 * blockIdx.x);
}

template <int NV>
__global__ void __launch_bounds__(kReduceThreads) finalize_kernel(const double *__restrict__ partials,
                                                                  int nblocks,
                                                                  double *__restrict__ out)
{
    double acc[NV];
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kReduceThreads)
        for (int v = 0; v < NV; ++v) acc[v] += partials[NV * b + v];
    block_reduce<NV>(acc, out);
}

// min, max and non-finite count of the stored phi perturbation.
template <class R>
__global__ void __launch_bounds__(kReduceThreads) pert_range_kernel(const R *__restrict__ pert,
                                                                    int n,
                                                                    double *__restrict__ partials)
{
    double lo = 1e300, hi = -1e300, bad = 0.0;
    for (int c = blockIdx.x * kReduceThreads + threadIdx.x; c < n;
         c += gridDim.x * kReduceThreads) {
        const double v = pert[c];
        if (!isfinite(v)) {
            bad += 1.0;
        } else {
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
    }
    __shared__ double s[3][kReduceThreads];
    s[0][threadIdx.x] = lo;
    s[1][threadIdx.x] = hi;
    s[2][threadIdx.x] = bad;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] += s[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = s[0][0];
        partials[3 * blockIdx.x + 1] = s[1][0];
        partials[3 * blockIdx.x + 2] = s[2][0];
    }
}

__global__ void __launch_bounds__(256) convert_pert_kernel(const double *__restrict__ src,
                                                           float *__restrict__ dst, int n)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) dst[c] = float(src[c]);
}

__global__ void __launch_bounds__(256) copy_kernel(const float4 *__restrict__ src,
                                                   float4 *__restrict__ dst, long long n)
{
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// Host-side launchers.
static inline unsigned blocks_for(long long n, int threads)
{
    return (unsigned)((n + threads - 1) / threads);
}

template <class Fn>
static hipError_t dispatch(int lattice, int mode, Fn &&fn)
{
    if (lattice == 0) {
        if (mode == MODE_F64) return fn(D2Q9{}, std::integral_constant<int, MODE_F64>{});
        if (mode == MODE_F32S) return fn(D2Q9{}, std::integral_constant<int, MODE_F32S>{});
        return fn(D2Q9{}, std::integral_constant<int, MODE_F16S>{});
    }
    if (mode == MODE_F64) return fn(D3Q19{}, std::integral_constant<int, MODE_F64>{});
    if (mode == MODE_F32S) return fn(D3Q19{}, std::integral_constant<int, MODE_F32S>{});
    return fn(D3Q19{}, std::integral_constant<int, MODE_F16S>{});
}

hipError_t launch_step(const Solver &s, const StepArgs &a, int parity)
{
    const unsigned nb = blocks_for(a.geo.ncells, s.block);
    return dispatch(s.lattice, s.mode, [&](auto lat, auto mode) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        if (parity == 0)
            step_kernel<L, M, 0><<<nb, s.block, 0, s.stream>>>(a);
        else
            step_kernel<L, M, 1><<<nb, s.block, 0, s.stream>>>(a);
        return hipGetLastError();
    });
}

hipError_t launch_init(const Solver &s, const double *rho0, const double *u0)
{
    StepArgs a = step_args(s, 0);
    const unsigned nb = blocks_for(a.geo.ncells, 256);
    return dispatch(s.lattice, s.mode, [&](auto lat, auto mode) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        init_kernel<L, M><<<nb, 256, 0, s.stream>>>(a, rho0, u0);
        return hipGetLastError();
    });
}

hipError_t launch_moments(const Solver &s, int parity, double m, double *rho, double *p,
                          double *u)
{
    StepArgs a = step_args(s, s.t);
    a.m = m;
    const unsigned nb = blocks_for(a.geo.ncells, 256);
    return dispatch(s.lattice, s.mode, [&](auto lat, auto mode) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        moments_kernel<L, M><<<nb, 256, 0, s.stream>>>(a, parity, rho, p, u);
        return hipGetLastError();
    });
}

hipError_t launch_populations(const Solver &s, int parity, double *f)
{
    StepArgs a = step_args(s, s.t);
    const unsigned nb = blocks_for(a.geo.ncells, 256);
    return dispatch(s.lattice, s.mode, [&](auto lat, auto mode) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        populations_kernel<L, M><<<nb, 256, 0, s.stream>>>(a, parity, f);
        return hipGetLastError();
    });
}

hipError_t launch_diagnostics(const Solver &s, int parity, double m, double *out_dev)
{
    StepArgs a = step_args(s, s.t);
    a.m = m;
    double *partials = s.scratch;
    hipError_t e = dispatch(s.lattice, s.mode, [&](auto lat, auto mode) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        diag_kernel<L, M><<<kReduceBlocks, kReduceThreads, 0, s.stream>>>(a, parity, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    finalize_kernel<7><<<1, kReduceThreads, 0, s.stream>>>(partials, kReduceBlocks, out_dev);
    return hipGetLastError();
}

hipError_t launch_convert_pert(const Solver &s, const double *src)
{
    convert_pert_kernel<<<blocks_for(s.geo.ncells, 256), 256, 0, s.stream>>>(
        src, static_cast<float *>(s.pert), s.geo.ncells);
    return hipGetLastError();
}

hipError_t launch_pert_range(const Solver &s, double *out_dev)
{
    if (s.mode == MODE_F64)
        pert_range_kernel<double><<<kReduceBlocks, kReduceThreads, 0, s.stream>>>(
            static_cast<const double *>(s.pert), s.geo.ncells, out_dev);
    else
        pert_range_kernel<float><<<kReduceBlocks, kReduceThreads, 0, s.stream>>>(
            static_cast<const float *>(s.pert), s.geo.ncells, out_dev);
    return hipGetLastError();
}

hipError_t launch_copy_probe(void *dst, const void *src, int64_t bytes, hipStream_t st)
{
    const long long n = bytes / 16;
    copy_kernel<<<4096, 256, 0, st>>>(static_cast<const float4 *>(src),
                                      static_cast<float4 *>(dst), n);
    return hipGetLastError();
}

}  // namespace vanse
