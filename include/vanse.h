/*
 * vanse.h -- C ABI of the MI355X (gfx950) implementation of the consistent
 * lattice Boltzmann scheme for the volume averaged Navier-Stokes equations
 * (VANSE) of Bukreev, Simonis, Kummerlaender, Jessberger and Krause,
 * arXiv:2208.09267, Section "Lattice Boltzmann scheme for VANSE".
 *
 * One solver handle owns one periodic lattice and advances it with the
 * fused per-cell step
 *
 *   I   = phi + varpi * lap(phi)                  cell integral of phi
 *                                                  (eqs. quad / latDiffRuleIIre,
 *                                                  Table 3 weights)
 *   rho = sum_i f_i / I                            eq. density
 *   p   = rho c_s^2,  F = p grad(phi) + F_ext      eq. pressForce (central
 *                                                  differences of phi)
 *   u   = (sum_i xi_i f_i + F/2) / sum_i f_i       eq. velocity
 *   f_i(x + xi_i, t + 1) = f_i - (f_i - f_i^eq)/tau + Omega^F_i
 *                                                  eq. lbe, eq. feq (with
 *                                                  rho I = sum f), Guo forcing
 *
 * in lattice units (dx = dt = 1, c_s^2 = 1/3).  The volume fraction is
 * phi(x, t_n) = eps_mean + m(n) eps_pert(x) with m(n) = cos(2 pi n / period)
 * (m = 1 when period <= 0); every term of step n uses phi at t_n.
 *
 * Conventions for every function below
 *   - Return value: VANSE_OK (0) or a negative VANSE_E* status.  No C++
 *     exception crosses the ABI.  vanse_last_error(h) describes the last
 *     failure on h.
 *   - Array arguments are DEVICE pointers owned by the caller (e.g. the data
 *     of contiguous torch tensors on the current GPU), FP64, x fastest:
 *     cell = (z*ny + y)*nx + x.  Vector fields are SoA: u[a*ncells + cell].
 *     The library never keeps a caller pointer past the call.
 *   - Work is enqueued on the handle's stream (vanse_set_stream; default the
 *     null stream) and is asynchronous unless stated otherwise.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef VANSE_H
#define VANSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vanse_solver *vanse_t;

/* Lattices: D2Q9 (Table 1), D3Q19 (the rest, face and edge groups of
 * Table 2 with weights 1/3, 1/18, 1/36) and D3Q27 (Table 2). */
enum { VANSE_D2Q9 = 0, VANSE_D3Q19 = 1, VANSE_D3Q27 = 2 };

/* quad_axes value that switches the cell-integral correction off: I = phi,
 * i.e. rho = sum f / phi (the density definition the paper corrects); for
 * ablation studies only. */
enum { VANSE_QUAD_NONE = 8 };

/* Population storage.  FP64: f_i in binary64, FP64 arithmetic.
 * FP32_SHIFTED: g_i = f_i - w_i in binary32, FP32 arithmetic in deviation
 * form.  FP16_SHIFTED: h_i = f_i / (c w_i) - 1 in binary16, FP32
 * arithmetic.  FX16_SHIFTED: the same h_i in 16-bit fixed point,
 * round(2^15 h_i) as int16, FP32 arithmetic: it holds 0 < f_i < 2 c w_i
 * with a rounding error of at most 2^-16 c w_i, where binary16 keeps 11
 * bits of h_i; a value at the bound of that range (a negative population,
 * or one above twice the mean-mass equilibrium) reads back as NaN and
 * vanse_diagnostics then reports EUNSTABLE.  c, the unit of both 16-bit
 * codes, is the mean of rho0 phi over the cells at vanse_init (the
 * conserved mass per cell, rounded to binary32), so that h_i carries only
 * the relative deviations of M0 and u from their means; these modes step
 * in units of c, with the forces divided by c.  In the reduced modes
 * eps_pert is held in binary32. */
enum { VANSE_FP64 = 0, VANSE_FP32_SHIFTED = 1, VANSE_FP16_SHIFTED = 2, VANSE_FX16_SHIFTED = 3 };

enum {
    VANSE_OK = 0,
    VANSE_EINVAL = -1,    /* bad argument (message in vanse_last_error)    */
    VANSE_ENOMEM = -2,    /* device allocation failed                      */
    VANSE_EDEVICE = -3,   /* HIP runtime error                             */
    VANSE_ESTATE = -4,    /* call out of order (e.g. step before init)     */
    VANSE_EUNSTABLE = -5  /* diagnostics saw a non-finite value (sticky)   */
};

/* Create a solver on the current HIP device.
 *   lattice  VANSE_D2Q9, VANSE_D3Q19 or VANSE_D3Q27
 *   dims     {nx, ny, nz}, each >= 1; nz must be 1 for D2Q9;
 *            nx*ny*nz < 2^31
 *   tau      BGK relaxation time, finite and > 1/2 (eq. lbe; the recovered
 *            viscosity is nu = (tau - 1/2) c_s^2)
 *   dtype    VANSE_FP64, VANSE_FP32_SHIFTED, VANSE_FP16_SHIFTED or
 *            VANSE_FX16_SHIFTED
 *   out      receives the handle
 * Allocates the single in-place population array (AA pattern), the phi
 * perturbation copy and the reduction scratch with hipMalloc; all are freed
 * by vanse_destroy.  Errors: EINVAL, ENOMEM, EDEVICE. */
int vanse_create(int lattice, const int64_t dims[3], double tau, int dtype, vanse_t *out);

/* Free every device allocation of h.  h may be NULL.  Synchronises h's
 * stream first. */
int vanse_destroy(vanse_t h);

/* Launch all later work of h on stream (a hipStream_t; NULL = null stream). */
int vanse_set_stream(vanse_t h, void *stream);

/* Volume fraction phi(x, t_n) = eps_mean + m(n) eps_pert(x), m(n) =
 * cos(2 pi n / period), period <= 0 meaning m == 1 (static field).
 *   eps_pert   device FP64 [ncells], or NULL for a uniform field; copied
 *              (converted to FP32 in the reduced modes), so the caller may
 *              free it on return
 *   quad_axes  bitmask of the axes the cell-integral quadrature runs over
 *              (1 = x, 2 = y, 4 = z; the D1Q3 / D2Q5 / D3Q7 choice of the
 *              paper, diagonals excluded); 0 selects all d axes;
 *              VANSE_QUAD_NONE drops the correction (I = phi)
 * Validates on the device that phi stays in (0, 1] for every reachable m and
 * that eps_pert is finite before anything is copied; synchronises.  A
 * rejected call leaves the solver as it was (its previous phi, if any, stays
 * in effect).  Errors: EINVAL, EDEVICE. */
int vanse_set_porosity(vanse_t h, double eps_mean, const double *eps_pert, double period,
                       int quad_axes);

/* Constant external force density F_ext (host array of 3 doubles, lattice
 * units), added to the pressure-correction force in sum_k F_k.  Components
 * beyond the lattice dimension must be 0.  Errors: EINVAL. */
int vanse_set_force(vanse_t h, const double F[3]);

/* Per-cell external force density (phase-interaction or manufactured-
 * solution forces; sum_k F_k of the Guo forcing term), added to F_ext and to
 * the pressure-correction force.  F: device FP64 SoA [d][ncells], copied
 * (to FP32 in the reduced modes; the first call allocates d planes);
 * NULL switches the field off.  Validates on the device that every value is
 * finite before anything is copied, and synchronises; a rejected call leaves
 * the solver as it was.  Errors: EINVAL, ENOMEM, EDEVICE. */
int vanse_set_force_field(vanse_t h, const double *F);

/* Initial populations (eq. equilibrium): f_i = f_i^eq of M0 = rho0 phi(x, 0)
 * and u0, with no non-equilibrium part.  rho0: device FP64 [ncells] or NULL
 * (1); u0: device FP64 SoA [d][ncells] or NULL (0).  Resets the time to 0.
 * The 16-bit modes first reduce rho0 phi to the unit c of their encoding
 * and synchronise (EINVAL if its mean is not finite and > 0; the solver is
 * then left as it was).  Requires vanse_set_porosity.  Errors: ESTATE,
 * EINVAL, EDEVICE. */
int vanse_init(vanse_t h, const double *rho0, const double *u0);

/* Advance n >= 0 time steps (asynchronous).  Errors: ESTATE, EINVAL,
 * EDEVICE. */
int vanse_step(vanse_t h, int64_t n);

/* Macroscopic fields at the current time t_n (eqs. density, velocity,
 * pressForce): rho [ncells], p [ncells], u SoA [d][ncells]; any may be NULL.
 * Computed in FP64 from the stored populations.  Asynchronous. */
int vanse_moments(vanse_t h, double *rho, double *p, double *u);

/* Global FP64 sums at t_n, in a fixed (deterministic) order, written to the
 * HOST array out[7]: out[0] = sum_x sum_i f_i (the phi-weighted mass
 * sum rho I), out[1..3] = sum_x sum_i xi_i f_i, out[4..6] = sum_x F.
 * Synchronises.  A non-finite sum (in FX16_SHIFTED also a population at the
 * bound of its range) makes h sticky-unstable: this and every later
 * vanse_step return EUNSTABLE. */
int vanse_diagnostics(vanse_t h, double out[7]);

/* Populations f_i(x, t_n) in FP64, natural order, SoA [Q][ncells] in this
 * library's direction order (vanse_lattice_info).  Asynchronous. */
int vanse_populations(vanse_t h, double *f);

/* Launch shape of the step kernel.  block: threads per block, 64, 128, 256,
 * 512 or 1024.  flags: bitwise OR of
 *   VANSE_TUNE_NONTEMPORAL  population loads and stores carry the nontemporal hint
 *   VANSE_TUNE_XCD_REMAP    each XCD processes one contiguous range of blocks
 *   VANSE_TUNE_FLAT         flattened tiling even when nx is a multiple of block
 *   VANSE_TUNE_NT_STORES    only the population stores carry the nontemporal hint
 * Without VANSE_TUNE_FLAT a block covers `block` consecutive cells of one
 * x-row when nx % block == 0.  Every setting computes bitwise-identical
 * results; only speed differs.  Errors: EINVAL. */
enum {
    VANSE_TUNE_NONTEMPORAL = 1,
    VANSE_TUNE_XCD_REMAP = 2,
    VANSE_TUNE_FLAT = 4,
    VANSE_TUNE_NT_STORES = 8,
    VANSE_TUNE_TWO_STEP = 16   /* batches only: see vanse_batch_set_tuning */
};
int vanse_set_tuning(vanse_t h, int block, int flags);

/* ---------------------------------------------------------------------------
 * Batched stepping: many independent solves advanced by one kernel launch per
 * time step.  The grid is a flattened table of blocks in which each solve owns
 * a contiguous range; each solve keeps its own size, tau, phi, force and time
 * level (and so its own AA parity).  The per-cell arithmetic is the same as
 * vanse_step's, so a solve evolves bitwise identically alone and in a batch.
 * Steps are issued in chunks; a full chunk replays a captured hipGraph. */
typedef struct vanse_batch *vanse_batch_t;

/* Create a batch over `count` >= 1 distinct, initialised solvers that share
 * lattice and dtype (host array of handles).  The batch does not own them:
 * they must outlive it.  A member may also be stepped alone between batch
 * calls, in stream order with the batch: the batch follows its time level
 * and, after two-step launches, its current population array (the batch
 * then rebuilds its tables once, synchronising its stream).  A member's
 * vanse_set_porosity, vanse_set_force or vanse_set_force_field after the
 * batch was built takes effect at the next batch call, which rebuilds the
 * tables the same way.  Allocates
 * small device tables (hipMalloc).  Errors: EINVAL, ESTATE, ENOMEM,
 * EDEVICE. */
int vanse_batch_create(const vanse_t *solvers, int count, vanse_batch_t *out);

/* Replace the members of b by `count` other (or the same) solvers of the
 * same lattice and dtype, keeping b's tuning and reusing its device tables
 * (grown when needed).  For request loops whose membership changes often.
 * Synchronises b's stream first.  Errors as vanse_batch_create. */
int vanse_batch_update(vanse_batch_t b, const vanse_t *solvers, int count);

/* Free the batch's tables and graph (not the solvers).  b may be NULL. */
int vanse_batch_destroy(vanse_batch_t b);

/* Launch later work of b on stream (NULL = null stream). */
int vanse_batch_set_stream(vanse_batch_t b, void *stream);

/* Threads per block (64, 128, 256) and flags of the batched kernel; chunk =
 * steps per captured graph (0: no graph, per-step launches).  Flags:
 *   VANSE_TUNE_NONTEMPORAL  nontemporal population loads and stores
 *   VANSE_TUNE_TWO_STEP     advance 3-D batches by the two-step launch (see
 *       vanse_set_fused): when every member has nx = 256 (rows: 4, or 2 in
 *       FP64 or when 4 does not divide ny) or nx = 128 (rows 4, D3Q19) and
 *       those rows divide its ny, all use that compile-time tile
 *       and their nz is split into equal segments of at most 64 planes (at
 *       most 32, 16 or 8 when a host-side estimate of the launch finds the
 *       batch too small to fill the GPU with 64); otherwise each
 *       member gets general tiles (any size) of as many x-rows as fit 512
 *       interior and 1024 (FP64: 512) halo-plane cells per 512-thread
 *       block, and its nz is split into equal segments of at most 32 planes
 *       (at most 24, 16, 12 or 8 when a host-side estimate of the launch
 *       finds the batch too small to fill the GPU with 32;
 *       vanse_batch_two_step_layout reports the result).  A D3Q19 batch in
 *       reduced storage whose members are all at most 96 cells wide takes
 *       768-thread blocks instead, with as many x-rows as fit 768
 *       halo-plane cells (more rows per tile).  On D3Q19, when a member's
 *       full rows do not fit a block (nx > 341; FP64 nx > 170), general
 *       tiles split the x-rows of wide members into the fewest segments of
 *       at most 62 columns, with a halo column on each side (one wave per
 *       row; vanse_batch_two_step_tiles reports them).  Every member gets a
 *       second population array (allocated here, kept by the member's
 *       solver: its population memory doubles).  Used for every group of 4
 *       steps of a chunk while all members sit at even time levels (two
 *       launches, so each member ends the group in its first array); other
 *       steps, and batches with a member that has no such tile (D3Q27 in
 *       FP64, or wider than 340 on D3Q27), use the single-step batched
 *       launch.
 * Results do not depend on any of these.  Errors: EINVAL, ENOMEM. */
int vanse_batch_set_tuning(vanse_batch_t b, int block, int flags, int chunk);

/* Advance every member n >= 0 steps (asynchronous).  Errors: EINVAL,
 * EUNSTABLE (a member is unstable), EDEVICE. */
int vanse_batch_step(vanse_batch_t b, int64_t n);

/* Autotune the batched launch shape: each candidate (block, flags: block
 * 64/128/256 with and without VANSE_TUNE_NONTEMPORAL, and, for 3-D batches
 * that fit it, VANSE_TUNE_TWO_STEP) runs `steps_per_trial` REAL steps of the
 * batch, timed with HIP events; then the two-step candidate (on
 * steps_per_trial rounded up to a multiple of 4, after one step to reach an
 * even level if the members share an odd one) and the best single-step
 * candidate (steps_per_trial rounded up to even) each run twice in a row,
 * the faster run of each counting; the fastest per step is kept and cached for batches of the same
 * lattice, dtype and size class (not cached when the members' time levels
 * differ in parity, which leaves the two-step candidate untried).  A cached
 * choice answers calls with at most the steps_per_trial that made it; a call
 * with longer trials runs them again and replaces it.  Members advance
 * the steps of every trial (0 if the choice came from the cache; *steps_run
 * tells).  Second population arrays allocated for the two-step trial stay
 * with the members.  Synchronises. */
int vanse_batch_autotune(vanse_batch_t b, int steps_per_trial, int *block, int *flags,
                         int64_t *steps_run);

/* The two-step layout in effect (VANSE_TUNE_TWO_STEP set by
 * vanse_batch_set_tuning or chosen by vanse_batch_autotune): for member k, in
 * the order the members were given, rows[k] full x-rows per tile and
 * planes[k] z-planes per segment (the last segment may be shorter).  rows
 * and planes are caller-owned host arrays of `count` ints; count must equal
 * the number of members (VANSE_EINVAL otherwise).  VANSE_ESTATE when no
 * two-step layout is in effect (the flag is not set, the lattice is 2-D, or a
 * member has no tile).  Host only: no GPU work. */
int vanse_batch_two_step_layout(vanse_batch_t b, int count, int *rows, int *planes);

/* As vanse_batch_two_step_layout, and cols[k]: the interior columns of member
 * k's tile (nx for tiles of full x-rows; fewer when the batch splits x-rows,
 * see vanse_batch_set_tuning).  Host only.  Errors: EINVAL, ESTATE. */
int vanse_batch_two_step_tiles(vanse_batch_t b, int count, int *cols, int *rows, int *planes);

/* Last error message of b (NULL: of the last failed vanse_batch_create). */
const char *vanse_batch_last_error(vanse_batch_t b);

/* Tile of the step kernel: a block covers tile_x consecutive cells (a power
 * of two in [64, 1024]) of each of tile_y consecutive x-rows of one z-plane;
 * tile_x * tile_y <= 1024 threads.  Used when the tile divides nx and ny (and
 * VANSE_TUNE_FLAT is not set), else the flattened launch with
 * tile_x * tile_y threads per block.  vanse_set_tuning resets the tile to
 * (block, 1).  Results are bitwise identical for every tile.
 * Errors: EINVAL. */
int vanse_set_tile(vanse_t h, int tile_x, int tile_y);

/* Two-step launch of vanse_step (3-D lattices, temporal blocking): one
 * launch advances two time levels.  It reads the populations at an even
 * level n from the solver's array and writes level n + 2 into a second
 * array of the same size (allocated here, so the population memory of the
 * solve doubles), keeping level n + 1 in LDS: the populations cross HBM
 * once per two lattice updates, plus the re-read halo of each tile.  A
 * block owns `rows` full x-rows of `planes` consecutive z-planes and
 * marches through them in z (halo: one x-row on each side and one plane at
 * each end of the segment).  vanse_step takes every pair of steps that
 * starts at an even level this way; a step left over (odd level, or odd n)
 * uses the single-step kernel.  Results are bitwise identical to single
 * steps.  Requires 1 <= rows <= ny, planes >= 1, and a tile shape compiled
 * into the library (the shapes whose registers fit without spilling): with
 * I = ceil(nx * rows / 512) interior and H = ceil(nx * (rows + 2) / 512)
 * halo cells per thread, when nx is a multiple of 64 and rows divides ny
 *   D3Q19, FP32/FP16 storage: I <= 2 and H <= I + 2
 *   D3Q19, FP64: I = 1 and H <= 2
 *   D3Q27, FP32/FP16 storage: I = 1 and H <= 3, or I = 2 and H = 2, or
 *       nx = 256 with rows = 4
 *   D3Q27, FP64: none (single steps only);
 * otherwise (the general tile: any nx, a shorter last tile in y, and
 * nx * ny * nz * 8 < 2^32)
 *   D3Q19, FP32/FP16 storage: I = 1 and H <= 3, or I = 2 and H = 2
 *   D3Q19, FP64: I = 1 and H = 1
 *   D3Q27, FP32/FP16 storage: I = 1 and H <= 2
 *   D3Q27, FP64: none;
 * and the block's LDS (Q * nx * rows stored populations plus 5 * (rows + 4)
 * * nx perturbation values) within 160 KiB.  Blocks have 512 threads, except
 * D3Q19's 256-wide 4-row tile in FP32/FP16 storage, which runs in blocks of
 * 1024 threads (one interior and two halo cells per thread).
 * rows = 0 switches the launch off and frees the second array.
 * Synchronises the solver's stream when it allocates or frees.
 * Errors: EINVAL, ENOMEM. */
int vanse_set_fused(vanse_t h, int rows, int planes);

/* Autotune the launch shape of vanse_step: each candidate (tiled 256-cell
 * row segments with 1, 2 or 4 rows per block where they divide the
 * lattice; flat launches of 256, 512 and 1024 threads; on 3-D lattices the
 * two-step launch of vanse_set_fused with 1, 2, 4 or 8 rows and 8, 16, 32
 * or 64 planes, and 128 when nz > 64, where its shape exists) runs
 * `steps_per_trial` REAL steps timed with HIP events, and the fastest is kept and cached for solves of the same
 * lattice, dtype and size class.  *fused_rows / *fused_planes report the
 * chosen two-step tile (0 / 0: single steps; the tile of the single-step
 * kernel is still reported and used for leftover steps).  The two-step
 * candidates need the second population array of vanse_set_fused: it is
 * allocated for the trials and freed again unless a two-step launch wins.
 * The solve advances (number of candidates) * steps_per_trial steps, or 0
 * when the choice came from the cache (*steps_run tells).  Synchronises.
 * Any output pointer may be NULL.  Errors: EINVAL, ESTATE, ENOMEM, EDEVICE. */
int vanse_autotune(vanse_t h, int steps_per_trial, int *tile_x, int *tile_y, int *flags,
                   int *fused_rows, int *fused_planes, int64_t *steps_run);

/* Current time level n (number of steps since vanse_init). */
int vanse_time(vanse_t h, int64_t *t);

/* Bytes of device memory held by h. */
int vanse_device_bytes(vanse_t h, int64_t *bytes);

/* Human-readable description of the last error on h (or of the last failed
 * vanse_create when h is NULL).  Never NULL; valid until the next call on
 * h. */
const char *vanse_last_error(vanse_t h);

/* This library's lattice tables: d, Q, xi (host int [Q][3]) and w (host
 * double [Q]), in the direction order used by vanse_populations. */
int vanse_lattice_info(int lattice, int *d, int *q, int *xi, double *w);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums of
 * vanse_diagnostics computed from caller-owned arrays by the same kernels,
 * with no handle and no allocation.
 *   lattice    VANSE_D2Q9, VANSE_D3Q19 or VANSE_D3Q27
 *   dims       {nx, ny, nz} as in vanse_create (nz = 1 for D2Q9); inputs of
 *              2^31 cells or more are rejected (EINVAL)
 *   f          device FP64 populations in natural order, SoA [Q][ncells], in
 *              this library's direction order (the layout vanse_populations
 *              writes)
 *   phi        device FP64 volume fraction at the time level of f [ncells]
 *   quad_axes  as in vanse_set_porosity
 *   F          host double[3] constant force density, or NULL (0)
 *   force      device FP64 per-cell force density SoA [d][ncells], or NULL
 *   out        DEVICE FP64 [7]: out[0] = sum_x sum_i f_i, out[1..3] =
 *              sum_x sum_i xi_i f_i, out[4..6] = sum_x F (pressure-correction
 *              plus external forces), in the fixed order of vanse_diagnostics
 *   stream     hipStream_t to launch on (NULL = null stream)
 * Asynchronous: nothing is synchronised, copied to the host or allocated;
 * the call may be captured into a graph.  The block partials go to a fixed
 * device array of the library (7 * 1024 + 64 doubles per GPU, whatever the
 * input size, held until the process ends) that every call on that GPU
 * overwrites completely: calls that overlap on one GPU (other streams, or
 * other threads) race on it and must be ordered by the caller.  Non-finite
 * inputs give non-finite sums (no sticky state: there is no handle).
 * Errors: EINVAL (message in vanse_last_error(NULL)), EDEVICE. */
int vanse_diagnostics_noalloc(int lattice, const int64_t dims[3], const double *f,
                              const double *phi, int quad_axes, const double F[3],
                              const double *force, double *out, void *stream);

/* Streaming copy of `bytes` bytes (multiple of 16) from src to dst on
 * stream: the achievable-bandwidth probe used to calibrate measurements.
 * Errors: EINVAL, EDEVICE. */
int vanse_copy_probe(void *dst, const void *src, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VANSE_H */
