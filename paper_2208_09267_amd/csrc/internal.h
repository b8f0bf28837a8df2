// internal.h -- solver state shared by the host API (api.hip) and the kernel
// launchers (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace vanse {

enum Mode { MODE_F64 = 0, MODE_F32S = 1, MODE_F16S = 2, MODE_FX16S = 3 };

// Launch-time view of one lattice: sizes and the population plane stride
// (elements between direction planes of the SoA population array).
struct Geometry {
    int nx, ny, nz;
    int nxy;
    int ncells;
    long long stride;
};

// Division by a launch-invariant divisor d (see fdiv in kernels.hip).
struct FastDiv {
    unsigned m;  // < 2^32 for every d >= 1
    unsigned s;
};

inline FastDiv make_fastdiv(unsigned d)
{
    unsigned l = 0;
    while ((1ull << l) < d) ++l;  // ceil(log2 d)
    FastDiv f;
    f.s = 31 + l;
    f.m = (unsigned)(((1ull << f.s) + d - 1) / d);
    return f;
}

// Everything one step of one solve needs, passed by value to the kernel.
struct StepArgs {
    Geometry geo;
    void *f;             // populations, SoA [Q][stride], storage type of the mode
    const void *pert;    // phi perturbation, double (FP64) or float (reduced)
    double eps_mean;     // phi = eps_mean + m * pert
    double shift;        // 16-bit modes: the unit c of the stored f_i / (c w_i) - 1
    double m;            // modulation m(n) of the current step
    double omega;        // 1 / tau
    double fcoef;        // 1 - omega / 2 (Guo forcing prefactor)
    double F[3];         // constant external force density
    double Fk[3];        // the same in the step kernels' units (16-bit modes: F / c)
    double fscale;       // per-cell force to the step kernels' units (16-bit modes: 1 / c)
    const void *force;   // optional per-cell force density, SoA [d][stride] (R), or null
    double wq;           // quadrature weight varpi_{i != 0}
    double n2;           // 2 * (number of quadrature axes)
    int qmask;           // quadrature axes bitmask
    // launch shape
    int row;             // 1: tiled (tile divides the lattice), 0: FLAT
    int flags;           // 1: nontemporal loads+stores, 2: XCD remap, 8: nontemporal stores
    unsigned block;      // threads per block
    unsigned nblocks;    // grid size
    unsigned tx, txlog;  // tiled: cells of one x-row segment per block (2^txlog, >= 64)
    unsigned ty;         // tiled: rows per block
    unsigned nseg;       // tiled: segments per x-row (nx / tx)
    unsigned nyb;        // tiled: row blocks per z-plane (ny / ty)
    FastDiv fd_nx, fd_ny, fd_seg, fd_nyb;
    // two-step launch (fused2_kernel): n -> n + 2 from f into f2
    void *f2;            // destination populations (natural order at n + 2)
    double m2;           // modulation m(n + 1) of the second step
    unsigned fty;        // full x-rows per tile
    unsigned fsz;        // z-planes per tile segment
    unsigned fnyb;       // tiles per z-segment (ny / fty; x-split tiles: times fnxb)
    FastDiv fd_fnyb;
    unsigned ftx;        // x-split general tiles: interior columns per tile (>= nx: full rows)
    unsigned fnxb;       //   and tiles per x-row
    FastDiv fd_fnxb;
    void *trash;         // 8-byte device slot for discarded stores
};

// One solve inside a batched launch (device-resident table).
struct BatchMember {
    StepArgs a;            // geometry, pointers and physics of the solve
    unsigned block_begin;  // first block of the solve in the batched grid
    unsigned nblocks;
};

struct Solver {
    int lattice = 0, mode = 0, d = 0, q = 0;
    Geometry geo{};
    double tau = 0.0;
    double eps_mean = 1.0, period = 0.0;
    double shift = 1.0;          // 16-bit modes: unit c of the encoding, set by vanse_init
    int qmask = 0;
    double F[3] = {0.0, 0.0, 0.0};
    bool porosity_set = false, initialized = false, unstable = false;
    // bumped by every setter of the step's physics (phi, forces), so that a
    // batch knows when its copy of the step parameters is stale
    unsigned long long gen = 0;
    int64_t t = 0;
    int tile_x = 256;            // step kernel tile: x-row segment per block
    int tile_y = 1;              //   and rows per block
    int flags = 0;               // step-kernel variant flags (StepArgs::flags)
    bool allow_row = true;       // use the tiled launch when the tile divides the lattice
    void *f = nullptr;           // populations (current time level)
    size_t f_bytes = 0;
    int fused_rows = 0;          // two-step launch: x-rows per tile (0 = off)
    int fused_planes = 0;        //   and z-planes per segment
    void *f_alt = nullptr;       // second population array of the two-step launch
    void *pert = nullptr;        // phi perturbation (double or float)
    size_t pert_bytes = 0;
    void *force = nullptr;       // per-cell force density (double or float), optional
    size_t force_bytes = 0;
    bool force_on = false;
    double *scratch = nullptr;   // reduction partials + results
    size_t scratch_bytes = 0;
    hipStream_t stream = nullptr;
    std::string err;
};

constexpr int kReduceBlocks = 1024;   // fixed grid of the reduction kernels
constexpr int kReduceThreads = 256;
// scratch (doubles): reduction partials [7 * kReduceBlocks], results [7], and
// from kTrashSlot on a slot that discarded kernel stores may write
constexpr int kTrashSlot = 7 * kReduceBlocks + 32;

double modulation(int64_t n, double period);
StepArgs step_args(const Solver &s, int64_t n);

// Kernel launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_step(const Solver &s, const StepArgs &a, int parity);
constexpr int kFusedThreads = 512;    // threads per block of the two-step launch
// general tiles of batches whose members are all narrow (nx <= 96, D3Q19,
// reduced storage): blocks of 768 threads, one interior and one halo cell
// per thread (145 VGPRs: 3 waves per SIMD, where the 512-thread tile with
// two halo cells per thread holds 193 VGPRs and 2 waves)
constexpr int kGenThreads768 = 768;
constexpr int kFusedMaxLds = 160 * 1024;
// Tile shapes of the two-step launch compiled into the library: ipt interior
// and hpt halo-plane cells per thread, kept to the combinations whose
// registers fit without spilling on gfx950.  nxc: nx when the tile is one of
// the compile-time tiles (fused_tile_nx), 0 for a runtime nx; D3Q27's
// 256-wide 4-row tile fits only with nx and rows folded in.
constexpr bool fused_compiled(int lattice, int mode, int ipt, int hpt, int nxc = 0)
{
    if (lattice == 0 || ipt < 1 || hpt < ipt) return false;
    if (lattice == 2)  // D3Q27: 27 populations per cell in registers
        return mode != MODE_F64 &&
               (ipt == 1 ? hpt <= 3 : (hpt <= 2 || (nxc == 256 && hpt == 3)));
    if (mode == MODE_F64) return ipt == 1 && hpt <= 2;
    return ipt <= 2 && hpt <= ipt + 2;
}
// nx if (nx, rows) is a compile-time tile of the two-step launch (D3Q19:
// 256 x 4, 256 x 2, 128 x 4; D3Q27: 256 x 4, 256 x 2), else 0.
constexpr int fused_tile_nx(int lattice, int nx, int rows)
{
    if (lattice == 1)
        return ((nx == 256 && (rows == 4 || rows == 2)) || (nx == 128 && rows == 4)) ? nx : 0;
    if (lattice == 2) return (nx == 256 && (rows == 4 || rows == 2)) ? nx : 0;
    return 0;
}
// The same for the general tile (any nx, shorter last tile), whose rows and
// row bases are per lane.
constexpr bool fused_compiled_gen(int lattice, int mode, int ipt, int hpt)
{
    if (lattice == 0 || ipt < 1 || hpt < ipt) return false;
    if (lattice == 2) return mode != MODE_F64 && ipt == 1 && hpt <= 2;
    if (mode == MODE_F64) return ipt == 1 && hpt == 1;
    return ipt == 1 ? hpt <= 3 : (ipt == 2 && hpt == 2);
}
// Two-step launch variant of a tile of `rows` full x-rows: ipt interior and
// hpt halo-plane cells per thread; gen: the general tile (nx not a multiple
// of 64 or rows not dividing ny; needs every array's byte size below 2^32).
struct FusedShape {
    int ipt = 0, hpt = 0;
    bool gen = false;
};
// false if the lattice/dtype has no such compiled shape or the LDS is too large.
bool fused_shape(int lattice, int mode, const Geometry &g, int rows, FusedShape *out);
// LDS of one block of the two-step launch: the population slab and the ring
// of 5 perturbation planes of rows + 4 x-rows.
size_t fused_lds_bytes(int q, int mode, int nx, int rows);
hipError_t launch_fused(const Solver &s, const StepArgs &a);
hipError_t launch_init(const Solver &s, const double *rho0, const double *u0);
// sum over cells of rho0 phi(x, 0) (the initial M0; rho0 NULL: 1), FP64, in
// the fixed order of the reductions, into out_dev[0] (device); uses the
// solver's reduction scratch.
hipError_t launch_init_mass(const Solver &s, const double *rho0, double *out_dev);
hipError_t launch_batch_step(int lattice, int mode, bool nt, unsigned nblocks, unsigned block,
                             const BatchMember *members, const unsigned *owner,
                             const double *mtab, const long long *t0, int j, int count,
                             hipStream_t st);
// Rows of a solve's general tile in the batched two-step launch with blocks
// of `threads` (kFusedThreads or kGenThreads768) threads (0: none).
int batch_fused_rows(const Solver &s, int threads = kFusedThreads);
// The tile of a D3Q19 solve in a batched two-step launch with x-split
// members: full rows (*cols = nx) when nx <= split_above or nx <= 62 (false
// if they do not fit), else segments of at most 62 columns, one wave per
// row; *rows rows.
bool batch_xt_tile(const Solver &s, int split_above, int *cols, int *rows);
// LDS of one block of an x-split tile (cols < nx): slab and a ring of 5
// perturbation planes of (rows + 4) x (cols + 4) values.
size_t fused_lds_bytes_xt(int q, int mode, int cols, int rows);
// Rows of the compile-time tile (nx a compile-time constant) that a batched
// two-step launch uses when every member has this nx and a multiple of the
// rows in y (0: none for this lattice, mode and size).
int batch_uniform_rows(int lattice, int mode, int nx, int ny);
// uni_nx, uni_rows: the members' common compile-time tile, or 0, 0 for
// general tiles (each member's own rows).
// xt: general tiles with x-split members (batch_xt_tile), D3Q19 only.
// gen_threads: block size of full-row general tiles (kFusedThreads, or
// kGenThreads768 for D3Q19 in the reduced modes).
hipError_t launch_batch_fused(int lattice, int mode, int uni_nx, int uni_rows, bool xt, int gen_threads,
                              unsigned nblocks, size_t lds, const BatchMember *members,
                              const unsigned *owner, const double *mtab, int j, int count,
                              int swap, hipStream_t st);
hipError_t launch_moments(const Solver &s, int parity, double m, double *rho, double *p,
                          double *u);
hipError_t launch_populations(const Solver &s, int parity, double *f);
hipError_t launch_diagnostics(const Solver &s, int parity, double m, double *out_dev);
// Allocation-free diagnostics over caller-owned natural-order FP64 inputs
// (plane stride g.stride == g.ncells); partials in a fixed per-device array.
hipError_t launch_diagnostics_noalloc(int lattice, const Geometry &g, const double *f,
                                      const double *phi, double wq, double n2, int qmask,
                                      const double F[3], const double *force, double *out,
                                      hipStream_t st);
size_t noalloc_scratch_bytes();
hipError_t launch_convert_pert(const Solver &s, const double *src);
hipError_t launch_convert(const double *src, float *dst, long long n, hipStream_t st);
// min, max and non-finite count of n FP64 values: per-block triples in
// partials[3 * kReduceBlocks]
hipError_t launch_range(const double *src, long long n, double *partials, hipStream_t st);
hipError_t launch_copy_probe(void *dst, const void *src, int64_t bytes, hipStream_t st);

}  // namespace vanse
