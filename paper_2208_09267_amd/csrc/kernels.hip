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

#include <algorithm>
#include <atomic>
#include <mutex>
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

// a*x + b*y + c*z for compile-time a, b, c in {-1, 0, 1}; zero terms vanish
// and the first nonzero term starts the sum (no 0 + x to evaluate).
template <int B, int C, class R>
__device__ __forceinline__ R add_terms(R s, R y, R z)
{
    if constexpr (B == 1) s = s + y;
    if constexpr (B == -1) s = s - y;
    if constexpr (C == 1) s = s + z;
    if constexpr (C == -1) s = s - z;
    return s;
}
template <int A, int B, int C, class R>
__device__ __forceinline__ R dot3(R x, R y, R z)
{
    if constexpr (A != 0) return add_terms<B, C>(A == 1 ? x : -x, y, z);
    else if constexpr (B != 0) return add_terms<0, C>(B == 1 ? y : -y, y, z);
    else if constexpr (C != 0) return C == 1 ? z : -z;
    else return R(0);
}

// Storage of one population: T is the raw element type in HBM, R the
// arithmetic type, and `shifted` / `scaled` / `unit_c` say what the stored
// value v_i is:
//   FP64        v_i = f_i                     (T = double)
//   FP32 shift  v_i = f_i - w_i               (T = float)
//   FP16 shift  v_i = f_i / (c w_i) - 1       (T = binary16 bits, decoded to float)
//   FX16 shift  v_i = f_i / (c w_i) - 1       (T = int16 bits: 2^15 v_i rounded to
//                                              nearest, saturated at +-32767)
// c is the solve's mean M0 at initialisation (StepArgs::shift): sum_i f_i is
// conserved, so v_i stays of the size of the relative deviations of M0 and u
// from their means, which the 16-bit codes resolve best near 0 (FP16: 11
// significant bits) or uniformly over 0 < f_i < 2 c w_i (FX16: rounding
// error at most 2^-16 c w_i).  The 16-bit modes step in units of c: their
// M0 is sum f / c, and the forces enter divided by c (StepArgs::Fk, fscale);
// u is the same in any unit of mass.
template <int MODE> struct Storage;
template <> struct Storage<MODE_F64> {
    using T = double;
    using R = double;
    static constexpr bool shifted = false, scaled = false, unit_c = false;
    static constexpr double unit = 1.0;   // decoded values are in units of `unit`
    static __device__ __forceinline__ R decode(T v) { return v; }
    static __device__ __forceinline__ T encode(R v) { return v; }
};
template <> struct Storage<MODE_F32S> {
    using T = float;
    using R = float;
    static constexpr bool shifted = true, scaled = false, unit_c = false;
    static constexpr double unit = 1.0;
    static __device__ __forceinline__ R decode(T v) { return v; }
    static __device__ __forceinline__ T encode(R v) { return v; }
};
template <> struct Storage<MODE_F16S> {
    using T = unsigned short;
    using R = float;
    static constexpr bool shifted = true, scaled = true, unit_c = true;
    static constexpr double unit = 1.0;
    static __device__ __forceinline__ R decode(T v) { return __half2float(__ushort_as_half(v)); }
    static __device__ __forceinline__ T encode(R v) { return __half_as_ushort(__float2half_rn(v)); }
};
template <> struct Storage<MODE_FX16S> {
    using T = unsigned short;
    using R = float;
    static constexpr bool shifted = true, scaled = true, unit_c = true;
    // the collision works on 2^15 v_i directly (the code's integer as a
    // float): a scaling by a power of two, exact, so its results are those
    // of decoding to v_i, with one multiplication per cell instead of one per
    // value and direction
    static constexpr double unit = 1.0 / 32768.0;
    static __device__ __forceinline__ R decode(T v) { return float((short)v); }
    // saturate at +-32767, then round to nearest even, so that an
    // out-of-range value reads back at the bound, which to_f64 reports as
    // not a number.  The clamp is the median of three, which takes a NaN
    // to -32767 (in IEEE mode its minimum of three drops a NaN operand).
    // Adding 1.5 * 2^23 to the clamped value leaves the nearest-even integer
    // in the low mantissa bits (the sum lies in [2^23, 2^24), where the
    // spacing is 1), so the low 16 bits of the sum's bit pattern are the
    // int16 code: the code of rounding, clamping and converting, in two
    // instructions instead of four.
    static __device__ __forceinline__ T encode(R v)
    {
        const float c = __builtin_amdgcn_fmed3f(v, -32767.0f, 32767.0f);
        return (unsigned short)__float_as_uint(c + 12582912.0f);
    }
};

// FP64 value of f_i from a stored population (off the hot path); c: the
// unit of the 16-bit modes.  An FX16 value at the bound of its range (the
// state left the range, or a NaN was stored) reads as NaN.
template <class L, int MODE, int I>
__device__ __forceinline__ double to_f64(typename Storage<MODE>::T raw, double c)
{
    using St = Storage<MODE>;
    if constexpr (MODE == MODE_FX16S) {
        if (raw == 0x7fffu || raw == 0x8000u || raw == 0x8001u) return __builtin_nan("");
    }
    const double v = double(St::decode(raw)) * St::unit;
    if constexpr (!St::shifted) return v;
    else if constexpr (!St::scaled) return L::w[I] + v;
    else if constexpr (!St::unit_c) return L::w[I] + L::w[I] * v;
    else return c * L::w[I] + c * L::w[I] * v;
}

// Unsigned division by a launch-invariant divisor d >= 1 for dividends
// n < 2^31: q = (n * m) >> s with s = 31 + ceil(log2 d), m = ceil(2^s / d)
// (the round-up multiplier of Granlund and Montgomery, 1994).
__device__ __forceinline__ unsigned fdiv(unsigned n, const FastDiv &f)
{
    return (unsigned)(((unsigned long long)n * f.m) >> f.s);
}

// The multiplier of make_fastdiv computed on the device (divisors < 2^31).
__device__ __forceinline__ FastDiv make_fastdiv_dev(unsigned d)
{
    FastDiv f;
    const unsigned l = d > 1 ? 32u - (unsigned)__clz((int)(d - 1)) : 0u;  // ceil(log2 d)
    f.s = 31 + l;
    f.m = (unsigned)(((1ull << f.s) + d - 1) / d);
    return f;
}

// Global memory access at a 32-bit byte offset from a base pointer.  With a
// wave-uniform base the compiler emits the scalar-base (saddr) form, so a
// lane carries one 32-bit offset instead of a 64-bit address.  The access
// goes through a global address-space pointer: pointers that a batched
// launch reads from its table in device memory carry no address space, and
// the compiler would otherwise use flat instructions, which also count
// against the LDS wait counter.
template <class T>
using global_t = __attribute__((address_space(1))) T;
template <class T, bool NT>
__device__ __forceinline__ T ld(const T *base, unsigned byte_off)
{
    const global_t<T> *p =
        (const global_t<T> *)(reinterpret_cast<const char *>(base) + byte_off);
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <class T, bool NT>
__device__ __forceinline__ void st(T *base, unsigned byte_off, T v)
{
    global_t<T> *p = (global_t<T> *)(reinterpret_cast<char *>(base) + byte_off);
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
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

// phi(x, t_n) = eps_mean + m(n) pert(x).  Every step kernel evaluates it
// through this one expression, so all launch forms round it alike.
template <class R>
__device__ __forceinline__ R phi_of(R eps_mean, R m, R pert)
{
    return eps_mean + m * pert;
}

// Volume-fraction operators at one cell, at the current time level:
//   I = phi + varpi (sum_{quad axes} (phi(x+e) + phi(x-e)) - 2N phi)
//       (cell integral, eqs. quad / latDiffRuleIIre, Table 3)
//   g = (phi(x+e) - phi(x-e)) / 2  (central-difference gradient of the
//       pressure-correction force)
// e[] holds phi at x, x+ex, x-ex, x+ey, x-ey, x+ez, x-ez.
template <class L, class R>
__device__ __forceinline__ void eps_combine(const R (&e)[7], R wq, R n2, int qmask, R &I,
                                            R &gx, R &gy, R &gz)
{
    R S = R(0);
    if (qmask & 1) S = e[1] + e[2];
    if (qmask & 2) {
        S = S + e[3];
        S = S + e[4];
    }
    if constexpr (L::D == 3) {
        if (qmask & 4) {
            S = S + e[5];
            S = S + e[6];
        }
    }
    I = e[0] + wq * (S - n2 * e[0]);
    gx = R(0.5) * (e[1] - e[2]);
    gy = R(0.5) * (e[3] - e[4]);
    gz = (L::D == 3) ? R(0.5) * (e[5] - e[6]) : R(0);
}

template <class L, class R>
__device__ __forceinline__ void eps_ops(const R *__restrict__ pert, R eps_mean, R m, R wq,
                                        R n2, int qmask, const Cell &k, R &I, R &gx, R &gy,
                                        R &gz)
{
    R e[7];
    e[0] = eps_mean + m * pert[k.c];
    e[1] = eps_mean + m * pert[k.at(1, 0, 0)];
    e[2] = eps_mean + m * pert[k.at(-1, 0, 0)];
    e[3] = eps_mean + m * pert[k.at(0, 1, 0)];
    e[4] = eps_mean + m * pert[k.at(0, -1, 0)];
    e[5] = e[6] = R(0);
    if constexpr (L::D == 3) {
        e[5] = eps_mean + m * pert[k.at(0, 0, 1)];
        e[6] = eps_mean + m * pert[k.at(0, 0, -1)];
    }
    eps_combine<L, R>(e, wq, n2, qmask, I, gx, gy, gz);
}

// ---------------------------------------------------------------------------
// BGK collision with Guo forcing of one cell, in place on the stored values
// v[Q] (f_i, f_i - w_i, or (f_i - w_i)/w_i by storage mode).
//
// Per cell: M0 = sum f (= 1 + sum (f - w) in the shifted modes, since
// sum w = 1 and sum w xi = 0; the 16-bit modes in units of c), rho = M0/I (eq. density), p = rho/3,
// F = p grad(phi) + F_ext (eq. pressForce), u = (j + F/2)/M0 (eq. velocity).
// The update f - (f - f^eq)/tau + Omega^F (eq. lbe with eq. feq, rho I = M0,
// and Guo's forcing term) is evaluated for each pair of opposite directions
// +-xi, whose equilibrium and forcing terms split into a part even in xi
// and a part odd in xi:
//   v'_{+-} = (1 - omega) v_{+-} + W [P0 + cu (a45 cu + b9 cF)]
//                                 +- W [c3 cu + d3 cF]
// with cu = xi.u, cF = xi.F, P0 = omega E - 3 k uF, a45 = 9/2 omega M0,
// b9 = 9 k, c3 = 3 omega M0, d3 = 3 k, k = 1 - omega/2, W = w_i (or 1 when
// the stored value is scaled by 1/w_i), and E = M0 (1 - 3/2 uu) for f, or
// dM0 - 3/2 uu M0 for the shifted values.
// First direction 1 .. H whose velocity has a nonzero component `axis`.
template <class L, int AXIS>
constexpr int first_dir()
{
    for (int i = 1; i <= L::H; ++i)
        if ((AXIS == 0 ? L::cx[i] : AXIS == 1 ? L::cy[i] : L::cz[i]) != 0) return i;
    return 0;
}

// sum_i R(w_i) - 1 for the weights as the collision rounds them (exact in
// double: the terms are at most 27 floats within 8 binades).
template <class L, class R>
constexpr double weight_excess()
{
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += (double)R(L::w[i]);
    return s - 1.0;
}

// F + Fc for a per-cell force value Fc stored in physical units: divided by c
// (times fscale = 1/c) in the 16-bit modes, which step in units of c.
template <class St, class R>
__device__ __forceinline__ R add_force(R F, R Fc, double fscale)
{
    if constexpr (St::unit_c) return F + R(fscale) * Fc;
    else return F + Fc;
}

template <class L, int MODE, class R>
__device__ __forceinline__ void collide(R (&v)[L::Q], R I, R gx, R gy, R gz, R omega,
                                        R fcoef, R Fex, R Fey, R Fez)
{
    using St = Storage<MODE>;
    constexpr int H = L::H;
    R s0, jx = R(0), jy = R(0), jz = R(0);
    if constexpr (St::scaled)
        s0 = R(L::w[0]) * v[0];
    else
        s0 = v[0];
    static_for<1, H + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int o = i + H;
        const R sp = v[i] + v[o];
        const R dm = v[i] - v[o];
        constexpr R w = St::scaled ? R(L::w[i]) : R(1);
        s0 = s0 + w * sp;
        // the first direction with a nonzero component starts each sum
        if constexpr (L::cx[i] != 0) {
            const R t = R(L::cx[i]) * w * dm;
            if constexpr (i == first_dir<L, 0>()) jx = t; else jx = jx + t;
        }
        if constexpr (L::cy[i] != 0) {
            const R t = R(L::cy[i]) * w * dm;
            if constexpr (i == first_dir<L, 1>()) jy = t; else jy = jy + t;
        }
        if constexpr (L::cz[i] != 0) {
            const R t = R(L::cz[i]) * w * dm;
            if constexpr (i == first_dir<L, 2>()) jz = t; else jz = jz + t;
        }
    });
    // sums of the stored values, in their units (FX16: 2^-15)
    if constexpr (St::unit != 1.0) {
        s0 = s0 * R(St::unit);
        jx = jx * R(St::unit);
        jy = jy * R(St::unit);
        jz = jz * R(St::unit);
    }
    const R M0 = St::shifted ? R(1) + s0 : s0;
    // eq. density and the 1/M0 of eq. velocity.  In the 16-bit modes, whose
    // rounding dominates the error, the hardware reciprocal (about 1 ulp of
    // FP32) replaces the two correctly rounded divisions: their step is bound
    // by its arithmetic, of which they are about a tenth.
    R rho, inv;
    if constexpr (St::scaled) {
        rho = M0 * __builtin_amdgcn_rcpf(I);
        inv = __builtin_amdgcn_rcpf(M0);
    } else {
        rho = M0 / I;
        inv = R(1) / M0;
    }
    const R p = rho * R(1.0 / 3.0);     // p = rho c_s^2
    const R Fx = p * gx + Fex;          // F_PC + F_ext (eq. pressForce)
    const R Fy = p * gy + Fey;
    const R Fz = (L::D == 3) ? p * gz + Fez : R(0);
    const R ux = (jx + R(0.5) * Fx) * inv;  // eq. velocity
    const R uy = (jy + R(0.5) * Fy) * inv;
    const R uz = (L::D == 3) ? (jz + R(0.5) * Fz) * inv : R(0);
    const R uu = ux * ux + uy * uy + uz * uz;
    const R uF = ux * Fx + uy * Fy + uz * Fz;

    const R om1 = R(1) - omega;
    const R E = St::shifted ? s0 - R(1.5) * uu * M0 : M0 * (R(1) - R(1.5) * uu);
    // the update's coefficients in the units of the stored values (exact:
    // 1/unit is a power of two)
    constexpr R IU = R(1.0 / St::unit);
    const R P0 = (omega * E - R(3) * fcoef * uF) * IU;
    const R a45 = R(4.5) * omega * M0 * IU;
    const R b9 = R(9) * fcoef * IU;
    const R c3 = R(3) * omega * M0 * IU;
    const R d3 = R(3) * fcoef * IU;
    {
        // The collision conserves M0: sum_i W_i (P0 + ...) = P0 in exact
        // arithmetic.  With the weights rounded to R their sum is 1 + delta
        // (FP32 D3Q19: delta = 1.49e-8), which in the shifted modes, where
        // P0 ~ omega (M0 - 1) is not small, would move the mass by delta P0
        // per cell and step, always the same way.  The rest population takes
        // back that excess (C0 P0).  FP64 stores f itself, and its weights'
        // excess (about 1e-16) is left alone.
        constexpr R W0 = St::scaled ? R(1) : R(L::w[0]);
        constexpr R C0 = St::shifted ? R(-weight_excess<L, R>() / (St::scaled ? L::w[0] : 1.0))
                                     : R(0);
        if constexpr (C0 != R(0))
            v[0] = om1 * v[0] + W0 * P0 + C0 * P0;
        else
            v[0] = om1 * v[0] + W0 * P0;
    }
    static_for<1, H + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int o = i + H;
        constexpr R W = St::scaled ? R(1) : R(L::w[i]);
        const R cu = dot3<L::cx[i], L::cy[i], L::cz[i]>(ux, uy, uz);
        const R cF = dot3<L::cx[i], L::cy[i], L::cz[i]>(Fx, Fy, Fz);
        const R sym = W * (P0 + cu * (a45 * cu + b9 * cF));
        const R anti = W * (c3 * cu + d3 * cF);
        v[i] = om1 * v[i] + sym + anti;
        v[o] = om1 * v[o] + sym - anti;
    });
}

// ---------------------------------------------------------------------------
// One fused time step of one cell (the hot path): Q population loads, the
// phi stencil, the collision and Q stores.  (x, y, z) is the cell; its
// periodic neighbour rows are the element offsets Yo (y-1, y, y+1) and Zo
// (z-1, z, z+1).  Every access is a row base (wave-uniform under ROW
// tiling) plus a 32-bit lane offset of x-1, x or x+1.
// NT: 0 plain accesses, 1 nontemporal loads and stores, 2 nontemporal stores.
template <class L, int MODE, int PARITY, int NT>
__device__ __forceinline__ void cell_step(const StepArgs &a, int x, int y, int z)
{
    using St = Storage<MODE>;
    using T = typename St::T;
    using R = typename St::R;
    const int nx = a.geo.nx, ny = a.geo.ny, nz = a.geo.nz;
    const int X[3] = {(x == 0 ? nx : x) - 1, x, (x + 1 == nx) ? 0 : x + 1};
    const int Yo[3] = {((y == 0 ? ny : y) - 1) * nx, y * nx, ((y + 1 == ny) ? 0 : y + 1) * nx};
    const int Zo[3] = {((z == 0 ? nz : z) - 1) * a.geo.nxy, z * a.geo.nxy,
                       ((z + 1 == nz) ? 0 : z + 1) * a.geo.nxy};

    auto load = [&](const T *plane, int dx, int dy, int dz) -> T {
        return ld<T, NT == 1>(plane + (Zo[dz + 1] + Yo[dy + 1]),
                         (unsigned)X[dx + 1] * (unsigned)sizeof(T));
    };
    auto store = [&](T *plane, int dx, int dy, int dz, T val) {
        st<T, NT != 0>(plane + (Zo[dz + 1] + Yo[dy + 1]), (unsigned)X[dx + 1] * (unsigned)sizeof(T),
                  val);
    };

    T *__restrict__ f = static_cast<T *>(a.f);
    const long long S = a.geo.stride;
    R v[L::Q];
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (PARITY == 0)
            v[i] = St::decode(load(f + i * S, 0, 0, 0));
        else
            v[i] = St::decode(load(f + opp<L>(i) * S, -L::cx[i], -L::cy[i], -L::cz[i]));
    });

    const R *__restrict__ pert = static_cast<const R *>(a.pert);
    const R em = R(a.eps_mean), mm = R(a.m);
    R e[7];
    e[0] = phi_of(em, mm, ld<R, false>(pert + (Zo[1] + Yo[1]), (unsigned)X[1] * sizeof(R)));
    e[1] = phi_of(em, mm, ld<R, false>(pert + (Zo[1] + Yo[1]), (unsigned)X[2] * sizeof(R)));
    e[2] = phi_of(em, mm, ld<R, false>(pert + (Zo[1] + Yo[1]), (unsigned)X[0] * sizeof(R)));
    e[3] = phi_of(em, mm, ld<R, false>(pert + (Zo[1] + Yo[2]), (unsigned)X[1] * sizeof(R)));
    e[4] = phi_of(em, mm, ld<R, false>(pert + (Zo[1] + Yo[0]), (unsigned)X[1] * sizeof(R)));
    e[5] = e[6] = R(0);
    if constexpr (L::D == 3) {
        e[5] = phi_of(em, mm, ld<R, false>(pert + (Zo[2] + Yo[1]), (unsigned)X[1] * sizeof(R)));
        e[6] = phi_of(em, mm, ld<R, false>(pert + (Zo[0] + Yo[1]), (unsigned)X[1] * sizeof(R)));
    }
    R I, gx, gy, gz;
    eps_combine<L, R>(e, R(a.wq), R(a.n2), a.qmask, I, gx, gy, gz);

    R Fex = R(a.Fk[0]), Fey = R(a.Fk[1]), Fez = R(a.Fk[2]);
    if (a.force) {  // per-cell force density, SoA [d][stride] (wave-uniform branch)
        const R *__restrict__ fc = static_cast<const R *>(a.force);
        const unsigned off = (unsigned)X[1] * (unsigned)sizeof(R);
        Fex = add_force<St>(Fex, ld<R, false>(fc + (Zo[1] + Yo[1]), off), a.fscale);
        Fey = add_force<St>(Fey, ld<R, false>(fc + a.geo.stride + (Zo[1] + Yo[1]), off), a.fscale);
        if constexpr (L::D == 3)
            Fez = add_force<St>(Fez, ld<R, false>(fc + 2 * a.geo.stride + (Zo[1] + Yo[1]), off),
                                a.fscale);
    }
    collide<L, MODE, R>(v, I, gx, gy, gz, R(a.omega), R(a.fcoef), Fex, Fey, Fez);

    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (PARITY == 0)
            store(f + opp<L>(i) * S, 0, 0, 0, St::encode(v[i]));
        else
            store(f + i * S, L::cx[i], L::cy[i], L::cz[i], St::encode(v[i]));
    });
}

// One time step of one solve.
// Tiled launch (the tile divides the lattice): a block covers tx consecutive
// cells of each of ty consecutive x-rows of one z-plane; every wave lies
// inside one row, so the y/z neighbour rows are wave-uniform (scalar
// registers), and the phi rows a block re-reads (y +- 1 inside the block)
// come from the CU's caches.  FLAT launch (any size): the lattice is flattened
// and divided with launch-invariant multipliers.
// XCD remap (flags & 2): the hardware deals blocks round-robin over the 8
// XCDs; the remap gives each XCD one contiguous range of blocks.
// Blocks of up to 1024 threads, except D3Q27 (27 populations per thread in
// registers), whose blocks are capped at 256 threads so that the compiler
// may hold them without spilling.
template <class L>
constexpr int max_block() { return L::Q > 19 ? 256 : 1024; }

template <class L, int MODE, int PARITY, bool ROW, int NT>
__global__ void __launch_bounds__(max_block<L>()) step_kernel(StepArgs a)
{
    unsigned b = blockIdx.x;
    if (a.flags & 2) {
        const unsigned q = a.nblocks >> 3, r = a.nblocks & 7, xcd = b & 7, idx = b >> 3;
        b = (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
    }
    if constexpr (ROW) {
        const unsigned rb = fdiv(b, a.fd_seg);
        const unsigned seg = b - rb * a.nseg;
        const unsigned zb = fdiv(rb, a.fd_nyb);
        const unsigned yb = rb - zb * a.nyb;
        // tx is a multiple of 64: all lanes of a wave share the row
        const unsigned ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> a.txlog);
        const int x = (int)(seg * a.tx + (threadIdx.x & (a.tx - 1)));
        const int y = (int)(yb * a.ty + ty);
        cell_step<L, MODE, PARITY, NT>(a, x, y, (int)zb);
    } else {
        const unsigned c = b * a.block + threadIdx.x;
        if (c >= (unsigned)a.geo.ncells) return;
        const unsigned yz = fdiv(c, a.fd_nx);
        const int x = (int)(c - yz * a.geo.nx);
        const int z = (int)fdiv(yz, a.fd_ny);
        const int y = (int)yz - z * a.geo.ny;
        cell_step<L, MODE, PARITY, NT>(a, x, y, z);
    }
}

// One time step of many independent solves in one launch.  Block b belongs
// to solve owner[b]; that solve's blocks are a contiguous range starting at
// members[s].block_begin and tile its flattened lattice.  Each solve has its
// own time level (parity t0[s] + j) and modulation mtab[j][s].  The per-cell
// arithmetic is cell_step, so every solve evolves exactly as it would alone.
template <class L, int MODE, bool NT>
__global__ void __launch_bounds__(256) batch_step_kernel(const BatchMember *__restrict__ members,
                                                         const unsigned *__restrict__ owner,
                                                         const double *__restrict__ mtab,
                                                         const long long *__restrict__ t0,
                                                         int j, int count)
{
    const unsigned s = owner[blockIdx.x];
    StepArgs a = members[s].a;
    a.m = mtab[(long long)j * count + s];
    const unsigned c = (blockIdx.x - members[s].block_begin) * a.block + threadIdx.x;
    if (c >= (unsigned)a.geo.ncells) return;
    const unsigned yz = fdiv(c, a.fd_nx);
    const int x = (int)(c - yz * a.geo.nx);
    const int z = (int)fdiv(yz, a.fd_ny);
    const int y = (int)yz - z * a.geo.ny;
    if ((t0[s] + j) & 1)
        cell_step<L, MODE, 1, NT ? 1 : 0>(a, x, y, z);
    else
        cell_step<L, MODE, 0, NT ? 1 : 0>(a, x, y, z);
}

// ---------------------------------------------------------------------------
// Two time steps in one launch (temporal blocking), 3-D lattices.
//
// Input: f at an even time level n in natural order (a.f).  Output: f at
// n + 2 in natural order in a second array (a.f2).  A block owns the interior
// tile of fty full x-rows (y0 .. y0+fty-1) of the z-planes z0 .. z1-1 and
// marches in z over the planes p = z0-1 .. z1:
//   1. step n on the fty + 2 rows y0-1 .. y0+fty of plane p (the two outer
//      rows are recomputed by the neighbouring tiles too): natural loads, the
//      phi stencil at m(n), collision -- the arithmetic of the even AA step;
//   2. each post-collision value f*_i(x) is pushed into an LDS slab at its
//      destination x + xi_i (slab [Q][nx * fty], indexed by direction and
//      destination cell of the tile; values leaving the tile rows are
//      dropped: the neighbouring tile computes them);
//   3. each interior cell reads back the values streaming into it; those with
//      xi_z = -1 complete plane p - 1, those with xi_z = 0 and +1 wait in
//      registers for planes p and p + 1;
//   4. step n + 1 on interior plane p - 1 (phi stencil at m(n+1)), results
//      pushed to x + xi_i of a.f2.
// The perturbation pert (phi = eps_mean + m pert) of the rows y0-2 ..
// y0+fty+1 is staged in an LDS ring of 5 planes (p-2 .. p+2), so the cell
// updates read no global memory.  Each halo cell's populations of plane p + 1
// are loaded as soon as its values of plane p have been read, and the pert
// rows of plane p + 3 before step 4 of plane p: they are in flight while the
// block computes, and no later global load waits behind them.  nx is a multiple of 64, so every wave lies in one x-row: row bases
// are scalar and a lane carries one 32-bit offset.  Per launch every
// population is loaded (fty + 2)/fty (fsz + 2)/fsz times and stored once for
// two lattice updates.  The cell arithmetic is the one of cell_step (phi_of,
// eps_combine, collide) and the intermediate values pass through the storage
// encoding as they would through HBM, so one launch is bitwise equal to two
// single steps.
// One tile (number b, y-fastest) of a two-step launch from a.f to a.f2 at
// modulations a.m, a.m2.  NXC / TYC: nx and fty as compile-time constants
// (0: read from a), so that the common tile shapes fold their index
// arithmetic.  GEN: any nx (waves may straddle x-rows: rows and row bases are
// per lane, accesses use 32-bit element offsets, which the host allows only
// when every array's byte size fits 32 bits) and a shorter last tile when fty
// does not divide ny; otherwise nx is a multiple of 64 and fty divides ny.
// XT (general tiles only): the tiles of a z-segment also split the x-rows
// into segments of a.ftx columns (a shorter last one), numbered x-fastest;
// such a tile adds a halo column on each side (its x-neighbours recompute
// them, as its outer rows), and its phi ring spans the tile's columns plus
// two on each side.  Its rows of at most 64 cells (a.ftx + 2 <= 64) each
// go to one wave, lane = column, so IPT and HPT count rows per wave: at most
// IPT * NT/64 interior rows, and HPT * NT/64 rows with the two outer ones.
// A member whose a.ftx covers its whole row (a.ftx >= nx) keeps
// the full-row indexing of the general tile (no halo columns: x wraps inside
// the row).  Needs nx >= 8 when a.ftx < nx.
template <class L, int MODE, int IPT, int HPT, int NXC, int TYC, bool GEN, int NT, bool XT = false>
__device__ __forceinline__ void fused2_tile(const StepArgs &a, unsigned b)
{
    static_assert(L::D == 3, "two-step launch: 3-D lattices only");
    static_assert(!XT || GEN, "x-split tiles are general tiles");
    using St = Storage<MODE>;
    using T = typename St::T;
    using R = typename St::R;
    constexpr int Q = L::Q;
    // every thread owns one interior cell per IPT (no repeats): stores need no
    // trash slot
    constexpr bool EXACT = !GEN && NXC > 0 && TYC > 0 && NXC * TYC == IPT * NT;
    constexpr int RING = 5;                 // pert planes p-2 .. p+2
    // pert values per thread and plane: exact for the compile-time tiles,
    // else a bound from the halo cells per thread ((rows + 4) / (rows + 2) <= 5/3)
    // (x-split tiles: (rows + 4)(cols + 4) <= (HPT NT/64 + 2) 66 <= 2 HPT NT)
    constexpr int PPT = (NXC > 0 && TYC > 0) ? ((TYC + 4) * NXC + NT - 1) / NT
                                             : (XT ? 2 * HPT : (5 * HPT + 2) / 3);
    extern __shared__ __align__(16) unsigned char fused_lds[];

    const int nx = NXC ? NXC : a.geo.nx, ny = a.geo.ny, nz = a.geo.nz, nxy = a.geo.nxy;
    const long long S = a.geo.stride;
    const unsigned bz = fdiv(b, a.fd_fnyb);
    const unsigned tb = b - bz * a.fnyb;  // tile within its z-segment
    unsigned yb = tb;
    int x0 = 0;                           // first interior column (x-split tiles)
    if constexpr (XT) {
        yb = fdiv(tb, a.fd_fnxb);
        x0 = (int)(tb - yb * a.fnxb) * (int)a.ftx;
    }
    const int y0 = (int)yb * (TYC ? TYC : (int)a.fty);
    const int TY = TYC ? TYC : (GEN ? min((int)a.fty, ny - y0) : (int)a.fty);
    // x-split: interior columns TX, halo row width HW = TX + 2, ring row width
    // RW = TX + 4; otherwise all three are nx (full rows, x wraps in the row)
    const bool xs = XT && (int)a.ftx < nx;
    const int TX = xs ? min((int)a.ftx, nx - x0) : nx;
    const int HW = xs ? TX + 2 : nx;
    const int RW = xs ? TX + 4 : nx;
    const int NI = TX * TY;          // interior cells of one plane of the tile
    const int HC = HW * (TY + 2);    // cells of one plane with the two outer rows
    const int PR = TY + 4;           // pert rows per plane: y0-2 .. y0+TY+1
    const int PC = PR * RW;
    T *__restrict__ slab = reinterpret_cast<T *>(fused_lds);
    R *__restrict__ ring =
        reinterpret_cast<R *>(fused_lds + ((size_t)Q * NI * sizeof(T) + 15) / 16 * 16);
    const int z0 = (int)bz * (int)a.fsz;
    const int z1 = min(z0 + (int)a.fsz, nz);
    const T *__restrict__ src = static_cast<const T *>(a.f);
    T *__restrict__ dst = static_cast<T *>(a.f2);
    const R *__restrict__ pert = static_cast<const R *>(a.pert);
    const R *__restrict__ fc = static_cast<const R *>(a.force);
    const R em = R(a.eps_mean);
    const int tid = threadIdx.x;

    // periodic index for v in [-n, 2n): neighbours and the halo of one tile
    auto wrap = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    // periodic plane index for any v >= -3 (the prologue and the prefetch
    // reach 2 planes below and 3 above the segment, also when nz < 3)
    auto zmod = [&](int v) { return (v + 3 * nz) % nz; };
    // x-row of a cell index of the tile: wave-uniform unless GEN
    auto row_of = [&](int idx) {
        const unsigned r = NXC ? (unsigned)idx / (unsigned)NXC : fdiv((unsigned)idx, a.fd_nx);
        if constexpr (GEN) return (int)r;
        else return (int)__builtin_amdgcn_readfirstlane(r);
    };
    // rows of halo, ring and interior cell indices: row widths HW, RW, TX
    // (x-split tiles: divisors of this tile, found once; otherwise nx)
    FastDiv fd_hw = a.fd_nx, fd_rw = a.fd_nx, fd_tx = a.fd_nx;
    if constexpr (XT) {
        if (xs) {
            fd_hw = make_fastdiv_dev((unsigned)HW);
            fd_rw = make_fastdiv_dev((unsigned)RW);
            fd_tx = make_fastdiv_dev((unsigned)TX);
        }
    }
    auto hrow = [&](int idx) { if constexpr (XT) return (int)fdiv((unsigned)idx, fd_hw); else return row_of(idx); };
    auto rrow = [&](int idx) { if constexpr (XT) return (int)fdiv((unsigned)idx, fd_rw); else return row_of(idx); };
    auto irow = [&](int idx) { if constexpr (XT) return (int)fdiv((unsigned)idx, fd_tx); else return row_of(idx); };
    // global column of halo column hx (x-split: x0 - 1 + hx, wrapped) and of
    // ring column c (x0 - 2 + c, wrapped); full rows: the column itself
    auto halo_x = [&](int hx) { return xs ? wrap(x0 - 1 + hx, nx) : hx; };
    auto ring_x = [&](int c) { return xs ? wrap(x0 - 2 + c, nx) : c; };
    // Cells of the tile handled by a thread.  Full rows: tile cells numbered
    // row by row, thread tid takes cell tid + pass * NT.  x-split tiles (HW <=
    // 64): one wave per row segment, lane = column, wave w takes row w + pass
    // * NW, so a wave's loads, LDS accesses and stores stay within one row
    // segment; lanes past the segment (and rows past the tile, which only
    // whole waves reach) repeat its last cell and are masked.
    constexpr int NW = NT / 64;
    const int lane = tid & 63, wv = tid >> 6;
    // halo cell of pass h: row hr (0 .. TY+1), column hx (0 .. HW-1), valid
    auto halo_cell = [&](int h, int &hr, int &hx, bool &valid) {
        if (xs) {
            const int r = wv + h * NW;
            valid = lane < HW && r < TY + 2;
            hr = min(r, TY + 1);
            hx = min(lane, HW - 1);
        } else {
            const int idx = min(tid + h * NT, HC - 1);
            valid = tid + h * NT < HC;
            hr = hrow(idx);
            hx = idx - hr * HW;
        }
    };
    // interior cell of pass k: row r (0 .. TY-1), column cx (0 .. TX-1), and
    // whether this thread owns it
    auto interior_cell = [&](int k, int &r, int &cx, bool &owned) {
        if (xs) {
            const int rr = wv + k * NW;
            owned = lane < TX && rr < TY;
            r = min(rr, TY - 1);
            cx = min(lane, TX - 1);
        } else {
            const int cell = min(tid + k * NT, NI - 1);
            owned = tid + k * NT < NI;
            r = irow(cell);
            cx = cell - r * TX;
        }
    };
    // element offset -> byte offset (GEN: 32-bit, checked on the host)
    auto boff = [](int elem, unsigned size) { return (unsigned)elem * size; };
    // Ring slot s holds the pert rows of one plane at ring + s * PC; plane q
    // lives in slot (q - z0 + 2) mod 5.  The loop keeps the slots of planes
    // p-2 .. p+2 in wave-uniform registers and rotates them per plane.
    // phi stencil, external + per-cell force and collision of one cell at
    // (x, y, z) (y, z wave-uniform unless GEN; r its ring row, c its ring
    // column: x itself for full rows, where the x-neighbours wrap in the row;
    // rm, r0, rp the ring planes of z - 1, z, z + 1) on the decoded values v,
    // at modulation mm
    auto update = [&](R (&v)[Q], int x, int y, int r, int c, const R *rm, const R *r0,
                      const R *rp, int z, R mm) {
        const int cm = xs ? c - 1 : (c == 0 ? nx : c) - 1;
        const int cp = xs ? c + 1 : ((c + 1 == nx) ? 0 : c + 1);
        const R *row = r0 + r * RW;
        R e[7];
        e[0] = phi_of(em, mm, row[c]);
        e[1] = phi_of(em, mm, row[cp]);
        e[2] = phi_of(em, mm, row[cm]);
        e[3] = phi_of(em, mm, row[RW + c]);
        e[4] = phi_of(em, mm, row[c - RW]);
        e[5] = phi_of(em, mm, rp[r * RW + c]);
        e[6] = phi_of(em, mm, rm[r * RW + c]);
        R I, gx, gy, gz;
        eps_combine<L, R>(e, R(a.wq), R(a.n2), a.qmask, I, gx, gy, gz);
        R Fex = R(a.Fk[0]), Fey = R(a.Fk[1]), Fez = R(a.Fk[2]);
        if (fc) {
            if constexpr (GEN) {
                const unsigned o = boff(z * nxy + y * nx + x, sizeof(R));
                Fex = add_force<St>(Fex, ld<R, false>(fc, o), a.fscale);
                Fey = add_force<St>(Fey, ld<R, false>(fc + S, o), a.fscale);
                Fez = add_force<St>(Fez, ld<R, false>(fc + 2 * S, o), a.fscale);
            } else {
                const R *row = fc + (z * nxy + y * nx);
                const unsigned ox = (unsigned)x * (unsigned)sizeof(R);
                Fex = add_force<St>(Fex, ld<R, false>(row, ox), a.fscale);
                Fey = add_force<St>(Fey, ld<R, false>(row + S, ox), a.fscale);
                Fez = add_force<St>(Fez, ld<R, false>(row + 2 * S, ox), a.fscale);
            }
        }
        collide<L, MODE, R>(v, I, gx, gy, gz, R(a.omega), R(a.fcoef), Fex, Fey, Fez);
    };
    // natural-order populations of the fty + 2 rows of plane p
    // natural-order populations of halo cell h (of the fty + 2 rows) of plane p
    auto load_cell = [&](T (&raw_h)[Q], int h, int p) {
        const int pz = zmod(p);
        int hr, hx;
        bool valid;
        halo_cell(h, hr, hx, valid);
        const int x = halo_x(hx);
        const int y = wrap(y0 + hr - 1, ny);
        if constexpr (GEN) {
            const unsigned o = boff(pz * nxy + y * nx + x, sizeof(T));
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                raw_h[i] = ld<T, false>(src + i * S, o);
            });
        } else {
            const T *base = src + (pz * nxy + y * nx);
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                raw_h[i] = ld<T, false>(base + i * S, (unsigned)x * (unsigned)sizeof(T));
            });
        }
    };
    // pert of the PR ring rows of plane q: into registers, then into the ring
    auto load_pert = [&](R (&ph)[PPT], int q) {
        const int qz = zmod(q);
        static_for<0, PPT>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int idx = min(tid + j * NT, PC - 1);
            const int r = rrow(idx);
            const int x = ring_x(idx - r * RW);
            const int y = ((y0 + r - 2) % ny + ny) % ny;
            if constexpr (GEN)
                ph[j] = ld<R, false>(pert, boff(qz * nxy + y * nx + x, sizeof(R)));
            else
                ph[j] = ld<R, false>(pert + (qz * nxy + y * nx), (unsigned)x * (unsigned)sizeof(R));
        });
    };
    auto store_pert = [&](const R (&ph)[PPT], int s) {
        static_for<0, PPT>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int idx = min(tid + j * NT, PC - 1);
            ring[s * PC + idx] = ph[j];  // repeats write the same value
        });
    };

    // Every iteration issues the same memory operations in the same order
    // (pert loads, population loads, Q * IPT stores), so the hardware wait
    // counts stay exact across the loop: threads past the end of the tile
    // repeat its last cell, and stores that must not land (those repeats, and
    // the two leading iterations that complete no plane) go to a trash slot.
    R up_prev[IPT][Q] = {};  // xi_z = +1 values for plane p - 1 (read at p - 2)
    R up_next[IPT][Q] = {};  // xi_z = +1 values for plane p (read at p - 1)
    R mid[IPT][Q] = {};      // xi_z = 0 values for plane p - 1 (read at p - 1)
    T raw[HPT][Q] = {};
    R ph[PPT] = {};
    T *__restrict__ trash = static_cast<T *>(a.trash);
    for (int q = z0 - 2; q <= z0; ++q) {
        load_pert(ph, q);
        store_pert(ph, q - (z0 - 2));
    }
    load_pert(ph, z0 + 1);
    static_for<0, HPT>([&](auto hc) { load_cell(raw[decltype(hc)::value], decltype(hc)::value, z0 - 1); });
    static_for<0, IPT * Q>([&](auto) { st<T, false>(trash, 0u, T(0)); });

    int s0 = 1;  // ring slot of plane p
    for (int p = z0 - 1; p <= z1; ++p) {
        const int pz = wrap(p, nz);
        const int sp1 = s0 == RING - 1 ? 0 : s0 + 1, sp2 = sp1 == RING - 1 ? 0 : sp1 + 1;
        const int sm1 = s0 == 0 ? RING - 1 : s0 - 1, sm2 = sm1 == 0 ? RING - 1 : sm1 - 1;
        const R *ring_m2 = ring + sm2 * PC, *ring_m1 = ring + sm1 * PC;
        const R *ring_0 = ring + s0 * PC, *ring_p1 = ring + sp1 * PC;
        __syncthreads();  // the slab and the ring slot of plane p - 3 are free
        store_pert(ph, sp2);
        static_for<0, HPT>([&](auto hc) {
            constexpr int h = decltype(hc)::value;
            int hr, hx;   // halo row and column (full rows: hx = x)
            bool valid = true;
            if constexpr (XT) {
                halo_cell(h, hr, hx, valid);
            } else {
                const int idx = min(tid + h * NT, HC - 1);
                hr = hrow(idx);
                hx = idx - hr * HW;
            }
            const int x = halo_x(hx);
            R v[Q];
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                v[i] = St::decode(raw[h][i]);
            });
            // the slot is free: its cell of plane p + 1 loads while this block
            // computes the rest of plane p
            load_cell(raw[h], h, p + 1);
            // a wave whose lanes all lie past the last halo cell only repeats
            // that cell (another wave computes it): it keeps the loads, so
            // every wave issues the same memory operations, and skips the
            // collision and the pushes
            constexpr bool FULL = !GEN && NXC > 0 && TYC > 0 && (h + 1) * NT <= (TYC + 2) * NXC;
            bool wave_on = (tid & ~63) + h * NT < HC;
            if constexpr (XT) {
                if (xs) wave_on = wv + h * NW < TY + 2;  // its row lies in the tile
            }
            if (FULL || wave_on) {
                update(v, x, wrap(y0 + hr - 1, ny), hr + 1, xs ? hx + 1 : x, ring_m1, ring_0,
                       ring_p1, pz, R(a.m));
                // destination rows hr - 1 + cy of the slab and columns x + cx
                // (full rows: wrapped in the row; x-split: hx - 1 + cx, kept
                // inside the tile)
                const int Ro[3] = {(hr - 2) * TX, (hr - 1) * TX, hr * TX};
                const int Xd[3] = {xs ? hx - 2 : (x == 0 ? nx : x) - 1, xs ? hx - 1 : x,
                                   xs ? hx : ((x + 1 == nx) ? 0 : x + 1)};
                static_for<0, Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    const int r = hr - 1 + L::cy[i];
                    bool in = (unsigned)r < (unsigned)TY;  // wave-uniform unless GEN
                    if constexpr (XT) in = in && valid && (unsigned)Xd[L::cx[i] + 1] < (unsigned)TX;
                    if (in)
                        slab[i * NI + Ro[L::cy[i] + 1] + Xd[L::cx[i] + 1]] = St::encode(v[i]);
                });
            }
        });
        __syncthreads();  // slab of plane p and ring plane p + 2 complete
        load_pert(ph, p + 3);
        // interior plane p - 1 is completed from p = z0 + 1 on; before that the
        // work is done on plane z0 (in range) and its results are discarded
        // (the ring slots it reads may not hold data yet)
        const int z = max(p - 1, z0);
        static_for<0, IPT>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            bool own;     // wave-uniform unless GEN
            int cell, r, cx;   // slab cell, interior row and column (full rows: cx = x)
            if constexpr (XT) {
                interior_cell(k, r, cx, own);
                own = own && p > z0;
                cell = r * TX + cx;
            } else {
                own = tid + k * NT < NI && p > z0;
                cell = min(tid + k * NT, NI - 1);
                r = irow(cell);
                cx = cell - r * TX;
            }
            R t[Q];
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                t[i] = St::decode(slab[i * NI + cell]);
            });
            const int x = x0 + cx;
            const int y = y0 + r;
            R w[Q];
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (L::cz[i] == 1) w[i] = up_prev[k][i];
                else if constexpr (L::cz[i] == 0) w[i] = mid[k][i];
                else w[i] = t[i];
            });
            update(w, x, y, r + 2, xs ? cx + 2 : x, ring_m2, ring_m1, ring_0, z, R(a.m2));
            // push to x + xi_i: wrapped rows (wave-uniform) and columns of a.f2
            const int Yo[3] = {((y == 0 ? ny : y) - 1) * nx, y * nx,
                               ((y + 1 == ny) ? 0 : y + 1) * nx};
            const int Zo[3] = {((z == 0 ? nz : z) - 1) * nxy, z * nxy,
                               ((z + 1 == nz) ? 0 : z + 1) * nxy};
            const unsigned Xo[3] = {(unsigned)((x == 0 ? nx : x) - 1) * (unsigned)sizeof(T),
                                    (unsigned)x * (unsigned)sizeof(T),
                                    (unsigned)((x + 1 == nx) ? 0 : x + 1) * (unsigned)sizeof(T)};
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                T *row = dst + i * S + (Zo[L::cz[i] + 1] + Yo[L::cy[i] + 1]);
                if constexpr (GEN) {
                    const unsigned o = boff(Zo[L::cz[i] + 1] + Yo[L::cy[i] + 1], sizeof(T)) +
                                       Xo[L::cx[i] + 1];
                    st<T, false>(own ? dst + i * S : trash, own ? o : 0u, St::encode(w[i]));
                } else if constexpr (EXACT) {
                    // every thread owns its cell; the leading iterations write
                    // their discarded results into the slots this thread
                    // rewrites when it completes plane z0
                    st<T, false>(row, Xo[L::cx[i] + 1], St::encode(w[i]));
                } else {
                    st<T, false>(own ? row : trash, own ? Xo[L::cx[i] + 1] : 0u,
                                 St::encode(w[i]));
                }
            });
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (L::cz[i] == 1) {
                    up_prev[k][i] = up_next[k][i];
                    up_next[k][i] = t[i];
                } else if constexpr (L::cz[i] == 0) {
                    mid[k][i] = t[i];
                }
            });
        });
        s0 = sp1;
    }
}


// Block b of a grid of n blocks -> tile number: the hardware deals blocks
// round-robin over the 8 XCDs; this gives each XCD one contiguous range of
// tiles, so y-neighbour tiles run on the same XCD at the same time and the
// rows both re-read can come from its L2.
__device__ __forceinline__ unsigned xcd_contiguous(unsigned b, unsigned n)
{
    const unsigned q = n >> 3, r = n & 7, xcd = b & 7, k = b >> 3;
    return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// Waves per SIMD the two-step kernel is compiled for: the compile-time D3Q19
// FP32 tiles with one interior and at most two halo cells per thread are
// held to 128 VGPRs (they fit without spilling) so that two 512-thread
// blocks share a CU.
template <class L, int MODE, int IPT, int HPT, int NXC, bool GEN, int NT>
constexpr int fused_waves_per_simd()
{
    return (std::is_same<L, D3Q19>::value && MODE == MODE_F32S && !GEN && NXC > 0 &&
            IPT == 1 && HPT <= 2 && NT == kFusedThreads) ? 4 : 1;
}

// Two-step launch of one solve, blocks of NT threads.
template <class L, int MODE, int IPT, int HPT, int NXC, int TYC, bool GEN, int NT>
__global__ void __launch_bounds__(NT, (fused_waves_per_simd<L, MODE, IPT, HPT, NXC, GEN, NT>()))
    fused2_kernel(StepArgs a)
{
    fused2_tile<L, MODE, IPT, HPT, NXC, TYC, GEN, NT>(a, xcd_contiguous(blockIdx.x, gridDim.x));
}

// Two-step launch of many solves: block b belongs to solve owner[b] (after
// the XCD-contiguous order), whose tiles are a contiguous range from
// members[s].block_begin.  Steps j and j + 1 of the chunk (modulations
// mtab[j][s], mtab[j + 1][s]); swap: the solve's current populations are in
// its second array (odd launch of a chunk).  GEN: general tiles, each member
// with its own rows; otherwise every member has the compile-time tile NXC x
// TYC of the single-solve launch.
template <class L, int MODE, int IPT, int HPT, int NXC, int TYC, bool GEN, int NT, bool XT>
__global__ void __launch_bounds__(NT, (fused_waves_per_simd<L, MODE, IPT, HPT, NXC, GEN, NT>()))
    batch_fused2_kernel(const BatchMember *__restrict__ members, const unsigned *__restrict__ owner,
                        const double *__restrict__ mtab, int j, int count, int swap)
{
    const unsigned b = xcd_contiguous(blockIdx.x, gridDim.x);
    const unsigned s = owner[b];
    StepArgs a = members[s].a;
    a.m = mtab[(long long)j * count + s];
    a.m2 = mtab[(long long)(j + 1) * count + s];
    if (swap) {
        void *t = a.f;
        a.f = a.f2;
        a.f2 = t;
    }
    fused2_tile<L, MODE, IPT, HPT, NXC, TYC, GEN, NT, XT>(a, b - members[s].block_begin);
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
    const T *__restrict__ f = static_cast<const T *>(a.f);
    const long long S = a.geo.stride;
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        T raw;
        if (parity == 0)
            raw = f[i * S + k.c];
        else
            raw = f[opp<L>(i) * S + k.at(-L::cx[i], -L::cy[i], -L::cz[i])];
        fo[i] = to_f64<L, MODE, i>(raw, a.shift);
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
    double Fc[3] = {0.0, 0.0, 0.0};
    if (a.force) {
        const R *fc = static_cast<const R *>(a.force);
        for (int d = 0; d < L::D; ++d) Fc[d] = double(fc[d * a.geo.stride + k.c]);
    }
    for (int d = 0; d < 3; ++d) {
        if (d < L::D) {
            F[d] = p * g[d] + (a.F[d] + Fc[d]);
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
        if constexpr (!Storage<MODE>::shifted)
            f[i * a.geo.stride + c] = feq;
        else if constexpr (!Storage<MODE>::scaled)
            f[i * a.geo.stride + c] = Storage<MODE>::encode(R(feq - L::w[i]));
        else
            f[i * a.geo.stride + c] =
                Storage<MODE>::encode(R((feq / (a.shift * L::w[i]) - 1.0) / Storage<MODE>::unit));
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

// sum over cells of rho0 phi(x, 0), phi formed in R as init_kernel forms it
// (the mean initial M0 is the unit of the 16-bit encodings)
template <class R>
__global__ void __launch_bounds__(kReduceThreads) init_mass_kernel(StepArgs a,
                                                                   const double *__restrict__ rho0,
                                                                   double *__restrict__ partials)
{
    double acc[1] = {0.0};
    for (int c = blockIdx.x * kReduceThreads + threadIdx.x; c < a.geo.ncells;
         c += gridDim.x * kReduceThreads) {
        const R e = R(a.eps_mean) + R(a.m) * static_cast<const R *>(a.pert)[c];
        acc[0] += (rho0 ? rho0[c] : 1.0) * double(e);
    }
    block_reduce<1>(acc, partials + blockIdx.x);
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

// min, max and non-finite count of n FP64 values (a caller's input array,
// checked before the library takes it over).
__global__ void __launch_bounds__(kReduceThreads) range_kernel(const double *__restrict__ src,
                                                               long long n,
                                                               double *__restrict__ partials)
{
    double lo = 1e300, hi = -1e300, bad = 0.0;
    for (long long c = (long long)blockIdx.x * kReduceThreads + threadIdx.x; c < n;
         c += (long long)gridDim.x * kReduceThreads) {
        const double v = src[c];
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

// Streaming copy, one 16-byte vector per thread: the best-performing plain
// copy shape on gfx950 (bandwidth calibration of the measurements).
__global__ void __launch_bounds__(256) copy_kernel(const float4 *__restrict__ src,
                                                   float4 *__restrict__ dst, long long n)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
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
    auto by_mode = [&](auto lat) {
        if (mode == MODE_F64) return fn(lat, std::integral_constant<int, MODE_F64>{});
        if (mode == MODE_F32S) return fn(lat, std::integral_constant<int, MODE_F32S>{});
        if (mode == MODE_F16S) return fn(lat, std::integral_constant<int, MODE_F16S>{});
        return fn(lat, std::integral_constant<int, MODE_FX16S>{});
    };
    if (lattice == 0) return by_mode(D2Q9{});
    if (lattice == 1) return by_mode(D3Q19{});
    return by_mode(D3Q27{});
}

hipError_t launch_step(const Solver &s, const StepArgs &a, int parity)
{
    const int nt = (a.flags & 1) ? 1 : ((a.flags & 8) ? 2 : 0);
    return dispatch(s.lattice, s.mode, [&](auto lat, auto mode) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        auto go = [&](auto row_c, auto nt_c) {
            constexpr bool ROW = decltype(row_c)::value;
            constexpr int NT = decltype(nt_c)::value;
            if (parity == 0)
                step_kernel<L, M, 0, ROW, NT><<<a.nblocks, a.block, 0, s.stream>>>(a);
            else
                step_kernel<L, M, 1, ROW, NT><<<a.nblocks, a.block, 0, s.stream>>>(a);
        };
        auto by_nt = [&](auto row_c) {
            if (nt == 1)
                go(row_c, std::integral_constant<int, 1>{});
            else if (nt == 2)
                go(row_c, std::integral_constant<int, 2>{});
            else
                go(row_c, std::integral_constant<int, 0>{});
        };
        if (a.row)
            by_nt(std::true_type{});
        else
            by_nt(std::false_type{});
        return hipGetLastError();
    });
}

size_t fused_lds_bytes(int q, int mode, int nx, int rows)
{
    const size_t elem = mode == MODE_F64 ? 8 : (mode == MODE_F32S ? 4 : 2);
    const size_t slab = ((size_t)q * nx * rows * elem + 15) / 16 * 16;
    const size_t ring = (size_t)5 * (rows + 4) * nx * (mode == MODE_F64 ? 8 : 4);
    return slab + ring;
}

bool fused_shape(int lattice, int mode, const Geometry &g, int rows, FusedShape *out)
{
    const int nx = g.nx;
    if (rows < 1 || rows > g.ny) return false;
    const long long ni = (long long)nx * rows, hc = ni + 2ll * nx;
    const long long i = (ni + kFusedThreads - 1) / kFusedThreads;
    const long long h = (hc + kFusedThreads - 1) / kFusedThreads;
    if (i > 4 || h > 8) return false;
    FusedShape sh;
    sh.ipt = (int)i;
    sh.hpt = (int)h;
    sh.gen = nx % 64 != 0 || g.ny % rows != 0;
    if (sh.gen) {
        // 32-bit byte offsets: every population plane, pert and force array
        if ((long long)g.ncells * 8 >= (1ll << 32)) return false;
        if (!fused_compiled_gen(lattice, mode, sh.ipt, sh.hpt)) return false;
    } else if (!fused_compiled(lattice, mode, sh.ipt, sh.hpt, fused_tile_nx(lattice, nx, rows))) {
        return false;
    }
    const int q = lattice == 0 ? 9 : (lattice == 1 ? 19 : 27);
    if (fused_lds_bytes(q, mode, nx, rows) > (size_t)kFusedMaxLds) return false;
    if (out) *out = sh;
    return true;
}

hipError_t launch_fused(const Solver &s, const StepArgs &a)
{
    FusedShape sh;
    if (!fused_shape(s.lattice, s.mode, a.geo, (int)a.fty, &sh)) return hipErrorInvalidValue;
    const int ipt = sh.ipt, hpt = sh.hpt;
    const bool gen = sh.gen;
    const size_t lds = fused_lds_bytes(s.q, s.mode, a.geo.nx, (int)a.fty);
    const unsigned nzb = (unsigned)((a.geo.nz + (int)a.fsz - 1) / (int)a.fsz);
    const unsigned nblocks = a.fnyb * nzb;
    hipError_t rc = hipErrorInvalidValue;
    bool launched = false;
    const int nx = a.geo.nx, ty = (int)a.fty;
    // one instantiation: IPT, HPT, (0 = runtime) compile-time nx / fty, GEN, threads
    auto go = [&](auto lat, auto mode, auto ic, auto hc, auto nxc, auto tyc, auto genc,
                  auto ntc) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        constexpr int I = decltype(ic)::value;
        constexpr int H = decltype(hc)::value;
        constexpr int NXC = decltype(nxc)::value;
        constexpr int TYC = decltype(tyc)::value;
        constexpr bool GEN = decltype(genc)::value;
        constexpr int NTC = decltype(ntc)::value;
        constexpr int LAT = std::is_same<L, D3Q19>::value ? 1 : 2;
        constexpr bool compiled =
            GEN ? (NXC == 0 && fused_compiled_gen(LAT, M, I, H)) : fused_compiled(LAT, M, I, H, NXC);
        if constexpr (compiled) {
            if (launched || GEN != gen || I != ipt || H != hpt) return;
            if (NXC && (NXC != nx || TYC != ty)) return;
            // (I, H) are the cells per thread of a 512-thread block; the
            // 1024-thread form of the same tile has half as many
            constexpr int KI = (I * kFusedThreads + NTC - 1) / NTC;
            constexpr int KH = (H * kFusedThreads + NTC - 1) / NTC;
            auto *fn = &fused2_kernel<L, M, KI, KH, NXC, TYC, GEN, NTC>;
            // slabs above 64 KiB need the kernel's LDS limit raised, once per device
            static std::atomic<unsigned long long> raised{0};
            int dev = 0;
            if ((rc = hipGetDevice(&dev)) != hipSuccess) return;
            const unsigned long long bit = 1ull << (dev & 63);
            if (lds > 65536 && !(raised.load() & bit)) {
                rc = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, kFusedMaxLds);
                if (rc != hipSuccess) return;
                raised.fetch_or(bit);
            }
            fn<<<nblocks, NTC, lds, s.stream>>>(a);
            rc = hipGetLastError();
            launched = true;
        }
    };
    auto shapes = [&](auto lat, auto mode) {
        using L = decltype(lat);
        using C0 = std::integral_constant<int, 0>;
        using C1 = std::integral_constant<int, 1>;
        using C2 = std::integral_constant<int, 2>;
        using C3 = std::integral_constant<int, 3>;
        using C4 = std::integral_constant<int, 4>;
        using C128 = std::integral_constant<int, 128>;
        using C256 = std::integral_constant<int, 256>;
        // compiled shapes of the common tiles (fused_tile_nx): 256-wide rows
        // x 2 or 4 rows, 128-wide rows x 4 rows (D3Q19); 256-wide x 2 or 4
        // rows (D3Q27)
        using F = std::false_type;
        using G = std::true_type;
        using N512 = std::integral_constant<int, kFusedThreads>;
        using N1024 = std::integral_constant<int, 2 * kFusedThreads>;
        if constexpr (std::is_same<L, D3Q19>::value) {
            // the 256 x 4 tile in 1024-thread blocks (one interior and two halo
            // cells per thread, 4 waves per SIMD; FP64 has no such tile)
            go(lat, mode, C2{}, C3{}, C256{}, C4{}, F{}, N1024{});
            go(lat, mode, C1{}, C2{}, C256{}, C2{}, F{}, N512{});
            go(lat, mode, C1{}, C2{}, C128{}, C4{}, F{}, N512{});
        } else {
            go(lat, mode, C2{}, C3{}, C256{}, C4{}, F{}, N512{});
            go(lat, mode, C1{}, C2{}, C256{}, C2{}, F{}, N512{});
        }
        go(lat, mode, C1{}, C1{}, C0{}, C0{}, F{}, N512{});
        go(lat, mode, C1{}, C2{}, C0{}, C0{}, F{}, N512{});
        go(lat, mode, C1{}, C3{}, C0{}, C0{}, F{}, N512{});
        go(lat, mode, C2{}, C2{}, C0{}, C0{}, F{}, N512{});
        go(lat, mode, C2{}, C3{}, C0{}, C0{}, F{}, N512{});
        go(lat, mode, C2{}, C4{}, C0{}, C0{}, F{}, N512{});
        go(lat, mode, C1{}, C1{}, C0{}, C0{}, G{}, N512{});
        go(lat, mode, C1{}, C2{}, C0{}, C0{}, G{}, N512{});
        go(lat, mode, C1{}, C3{}, C0{}, C0{}, G{}, N512{});
        go(lat, mode, C2{}, C2{}, C0{}, C0{}, G{}, N512{});
        go(lat, mode, C2{}, C3{}, C0{}, C0{}, G{}, N512{});
    };
    auto modes = [&](auto lat) {
        if (s.mode == MODE_F64) shapes(lat, std::integral_constant<int, MODE_F64>{});
        else if (s.mode == MODE_F32S) shapes(lat, std::integral_constant<int, MODE_F32S>{});
        else if (s.mode == MODE_F16S) shapes(lat, std::integral_constant<int, MODE_F16S>{});
        else shapes(lat, std::integral_constant<int, MODE_FX16S>{});
    };
    if (s.lattice == 1) modes(D3Q19{});
    else modes(D3Q27{});
    return rc;
}

int batch_fused_rows(const Solver &s, int threads)
{
    if (s.d != 3 || (long long)s.geo.ncells * 8 >= (1ll << 32)) return 0;
    const int nx = s.geo.nx;
    int rows;
    if (threads == kGenThreads768) {
        if (s.lattice != 1 || s.mode == MODE_F64) return 0;
        rows = kGenThreads768 / nx - 2;                 // 1 interior, 1 halo cell per thread
    } else if (s.mode == MODE_F64) {
        if (s.lattice != 1) return 0;
        rows = 512 / nx - 2;                            // 1 interior, 1 halo cell per thread
    } else {
        rows = std::min(512 / nx, 1024 / nx - 2);       // 1 interior, 2 halo cells per thread
    }
    rows = std::min(rows, s.geo.ny);
    return rows >= 1 ? rows : 0;
}

int batch_uniform_rows(int lattice, int mode, int nx, int ny)
{
    int rows = 0;
    if (lattice == 1 && nx == 256) rows = mode == MODE_F64 ? 2 : 4;
    else if (lattice == 1 && nx == 128) rows = 4;
    else if (lattice == 2 && nx == 256 && mode != MODE_F64) rows = 4;
    if (rows == 4 && nx == 256 && ny % 4 != 0) rows = mode == MODE_F64 ? 0 : 2;
    return (rows > 0 && ny % rows == 0) ? rows : 0;
}

size_t fused_lds_bytes_xt(int q, int mode, int cols, int rows)
{
    const size_t elem = mode == MODE_F64 ? 8 : (mode == MODE_F32S ? 4 : 2);
    const size_t slab = ((size_t)q * cols * rows * elem + 15) / 16 * 16;
    const size_t ring = (size_t)5 * (rows + 4) * (cols + 4) * (mode == MODE_F64 ? 8 : 4);
    return slab + ring;
}

// Rows and columns of a D3Q19 solve's tile in a batched launch with x-split
// members, whose kernel has one interior and one halo cell (FP64) or two and
// two (reduced storage) per thread: full rows where they fit (*cols = nx,
// as many rows as the cells per thread allow), unless split_above < nx;
// otherwise the fewest segments of at most 62 columns (a halo column on each
// side makes a row of at most 64: one wave per row) and as many rows as
// 8 waves hold (FP64 6, reduced 14).
bool batch_xt_tile(const Solver &s, int split_above, int *cols, int *rows)
{
    if (s.lattice != 1 || s.d != 3 || (long long)s.geo.ncells * 8 >= (1ll << 32)) return false;
    const int nx = s.geo.nx, ny = s.geo.ny;
    const int per = s.mode == MODE_F64 ? 1 : 2;        // interior and halo cells per thread
    const int full = std::min(per * kFusedThreads / nx - 2, ny);
    if (nx <= split_above || nx <= 62) {
        if (full < 1) return false;
        *cols = nx;
        *rows = full;
        return true;
    }
    const int k = (nx + 61) / 62;
    const int c = (nx + k - 1) / k;
    const int nw = kFusedThreads / 64;
    const int r = std::min(per * nw - 2, ny);
    if (fused_lds_bytes_xt(s.q, s.mode, c, r) > (size_t)kFusedMaxLds) return false;
    *cols = c;
    *rows = r;
    return true;
}

hipError_t launch_batch_fused(int lattice, int mode, int uni_nx, int uni_rows, bool xt, int gen_threads,
                              unsigned nblocks, size_t lds, const BatchMember *members,
                              const unsigned *owner, const double *mtab, int j, int count,
                              int swap, hipStream_t st)
{
    if (lattice == 0 || lds > (size_t)kFusedMaxLds) return hipErrorInvalidValue;
    hipError_t rc = hipErrorInvalidValue;
    bool launched = false;
    // one instantiation: IPT, HPT (of a 512-thread block), compile-time nx /
    // rows (0, 0: general tiles), threads per block
    auto go = [&](auto lat, auto m, auto ic, auto hc, auto nxc, auto tyc, auto ntc,
                  auto xtc) {
        using L = decltype(lat);
        constexpr int M = decltype(m)::value;
        constexpr int I = decltype(ic)::value;
        constexpr int H = decltype(hc)::value;
        constexpr int NXC = decltype(nxc)::value;
        constexpr int TYC = decltype(tyc)::value;
        constexpr int NTC = decltype(ntc)::value;
        constexpr bool XT = decltype(xtc)::value;
        constexpr int KI = (I * kFusedThreads + NTC - 1) / NTC;
        constexpr int KH = (H * kFusedThreads + NTC - 1) / NTC;
        constexpr bool GEN = NXC == 0;
        constexpr int LAT = std::is_same<L, D3Q19>::value ? 1 : 2;
        constexpr bool compiled =
            GEN ? fused_compiled_gen(LAT, M, I, H) : fused_compiled(LAT, M, I, H, NXC);
        if constexpr (compiled) {
            if (launched || NXC != uni_nx || TYC != uni_rows || XT != xt) return;
            if (GEN && !XT && NTC != gen_threads) return;
            auto *fn = &batch_fused2_kernel<L, M, KI, KH, NXC, TYC, GEN, NTC, XT>;
            static std::atomic<unsigned long long> raised{0};
            int dev = 0;
            if ((rc = hipGetDevice(&dev)) != hipSuccess) return;
            const unsigned long long bit = 1ull << (dev & 63);
            if (lds > 65536 && !(raised.load() & bit)) {
                rc = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, kFusedMaxLds);
                if (rc != hipSuccess) return;
                raised.fetch_or(bit);
            }
            fn<<<nblocks, NTC, lds, st>>>(members, owner, mtab, j, count, swap);
            rc = hipGetLastError();
            launched = true;
        }
    };
    (void)dispatch(lattice, mode, [&](auto lat, auto m) -> hipError_t {
        using L = decltype(lat);
        constexpr int M = decltype(m)::value;
        using C0 = std::integral_constant<int, 0>;
        using C1 = std::integral_constant<int, 1>;
        using C2 = std::integral_constant<int, 2>;
        using C3 = std::integral_constant<int, 3>;
        using C4 = std::integral_constant<int, 4>;
        using C128 = std::integral_constant<int, 128>;
        using C256 = std::integral_constant<int, 256>;
        if constexpr (L::D == 3) {
            // general tiles: one interior and two halo cells per thread (FP64:
            // one); the compile-time tiles of batch_uniform_rows
            using N512 = std::integral_constant<int, kFusedThreads>;
            using N1024 = std::integral_constant<int, 2 * kFusedThreads>;
            using F = std::false_type;
            using X = std::true_type;
            if constexpr (M == MODE_F64) go(lat, m, C1{}, C1{}, C0{}, C0{}, N512{}, F{});
            else go(lat, m, C1{}, C2{}, C0{}, C0{}, N512{}, F{});
            if constexpr (std::is_same<L, D3Q19>::value && M != MODE_F64) {
                // general tiles of batches of narrow members: 768-thread
                // blocks, one interior and one halo cell per thread
                using N768 = std::integral_constant<int, kGenThreads768>;
                go(lat, m, C1{}, C1{}, C0{}, C0{}, N768{}, F{});
            }
            if constexpr (std::is_same<L, D3Q19>::value) {
                // general tiles with x-split members
                if constexpr (M == MODE_F64) go(lat, m, C1{}, C1{}, C0{}, C0{}, N512{}, X{});
                else go(lat, m, C2{}, C2{}, C0{}, C0{}, N512{}, X{});
                go(lat, m, C2{}, C3{}, C256{}, C4{}, N1024{}, F{});
                go(lat, m, C1{}, C2{}, C256{}, C2{}, N512{}, F{});
                go(lat, m, C1{}, C2{}, C128{}, C4{}, N512{}, F{});
            } else {
                go(lat, m, C2{}, C3{}, C256{}, C4{}, N512{}, F{});
                go(lat, m, C1{}, C2{}, C256{}, C2{}, N512{}, F{});
            }
        }
        return hipSuccess;
    });
    return launched ? rc : hipErrorInvalidValue;
}

hipError_t launch_batch_step(int lattice, int mode, bool nt, unsigned nblocks, unsigned block,
                             const BatchMember *members, const unsigned *owner,
                             const double *mtab, const long long *t0, int j, int count,
                             hipStream_t st)
{
    return dispatch(lattice, mode, [&](auto lat, auto m) {
        using L = decltype(lat);
        constexpr int M = decltype(m)::value;
        if (nt)
            batch_step_kernel<L, M, true><<<nblocks, block, 0, st>>>(members, owner, mtab, t0, j,
                                                                    count);
        else
            batch_step_kernel<L, M, false><<<nblocks, block, 0, st>>>(members, owner, mtab, t0,
                                                                     j, count);
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

hipError_t launch_init_mass(const Solver &s, const double *rho0, double *out_dev)
{
    StepArgs a = step_args(s, 0);
    double *partials = s.scratch;
    if (s.mode == MODE_F64)
        init_mass_kernel<double><<<kReduceBlocks, kReduceThreads, 0, s.stream>>>(a, rho0, partials);
    else
        init_mass_kernel<float><<<kReduceBlocks, kReduceThreads, 0, s.stream>>>(a, rho0, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    finalize_kernel<1><<<1, kReduceThreads, 0, s.stream>>>(partials, kReduceBlocks, out_dev);
    return hipGetLastError();
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

// ---------------------------------------------------------------------------
// Reduction scratch of the allocation-free diagnostics: a fixed device array
// (one copy per GPU, held until the process ends) for the block partials and
// the combined sums.  Host code never passes the array's name to a kernel
// (in host code it is a stand-in, not a device address): the device address
// comes from hipGetSymbolAddress, taken once per device and kept below.
constexpr int kNoAllocScratchDoubles = 7 * kReduceBlocks + 64;
static __device__ __align__(256) double g_noalloc_scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's copy of the scratch array, looked up on the
// first call made with that device current.
static hipError_t noalloc_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_noalloc_scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_noalloc_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_noalloc_ptr[dev];
    return hipSuccess;
}

size_t noalloc_scratch_bytes() { return sizeof(double) * kNoAllocScratchDoubles; }

// The sums of launch_diagnostics over caller-owned FP64 inputs in natural
// order (f [Q][ncells], phi [ncells], force [d][ncells] or null): the same
// diag_kernel and finalize_kernel, with phi = 0 + 1 * phi and plane stride
// ncells, partials in the fixed scratch array.  Nothing is allocated.
hipError_t launch_diagnostics_noalloc(int lattice, const Geometry &g, const double *f,
                                      const double *phi, double wq, double n2, int qmask,
                                      const double F[3], const double *force, double *out,
                                      hipStream_t st)
{
    double *partials = nullptr;
    hipError_t e = noalloc_scratch(&partials);
    if (e != hipSuccess) return e;
    StepArgs a{};
    a.geo = g;
    a.f = const_cast<double *>(f);
    a.pert = phi;
    a.eps_mean = 0.0;
    a.shift = 1.0;
    a.m = 1.0;
    a.omega = 1.0;
    a.fcoef = 0.5;
    for (int d = 0; d < 3; ++d) a.F[d] = a.Fk[d] = F[d];
    a.fscale = 1.0;
    a.force = force;
    a.wq = wq;
    a.n2 = n2;
    a.qmask = qmask;
    e = dispatch(lattice, MODE_F64, [&](auto lat, auto mode) {
        using L = decltype(lat);
        constexpr int M = decltype(mode)::value;
        if constexpr (M == MODE_F64)
            diag_kernel<L, M><<<kReduceBlocks, kReduceThreads, 0, st>>>(a, 0, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    finalize_kernel<7><<<1, kReduceThreads, 0, st>>>(partials, kReduceBlocks, out);
    return hipGetLastError();
}

hipError_t launch_convert_pert(const Solver &s, const double *src)
{
    convert_pert_kernel<<<blocks_for(s.geo.ncells, 256), 256, 0, s.stream>>>(
        src, static_cast<float *>(s.pert), s.geo.ncells);
    return hipGetLastError();
}

hipError_t launch_convert(const double *src, float *dst, long long n, hipStream_t st)
{
    for (long long off = 0; off < n; off += (1ll << 30)) {
        const int m = (int)std::min<long long>(n - off, 1ll << 30);
        convert_pert_kernel<<<blocks_for(m, 256), 256, 0, st>>>(src + off, dst + off, m);
    }
    return hipGetLastError();
}

hipError_t launch_range(const double *src, long long n, double *partials, hipStream_t st)
{
    range_kernel<<<kReduceBlocks, kReduceThreads, 0, st>>>(src, n, partials);
    return hipGetLastError();
}

hipError_t launch_copy_probe(void *dst, const void *src, int64_t bytes, hipStream_t st)
{
    const long long n = bytes / 16;
    if (n == 0) return hipSuccess;
    if ((n + 255) / 256 > 0x7fffffffLL) return hipErrorInvalidValue;
    copy_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(static_cast<const float4 *>(src),
                                                             static_cast<float4 *>(dst), n);
    return hipGetLastError();
}

}  // namespace vanse
