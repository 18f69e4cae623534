/*
 * rsg.h -- C ABI of the MI355X real-space-grid Kohn-Sham library.
 *
 * The library applies the Kohn-Sham Hamiltonian
 *
 *     H = kin * Lap_h + V(r) + E * x_axis + sum_a sum_i |p_i^a> E_i^a <p_i^a|
 *
 * to a batch ("group of states") of orbitals sampled on a uniform grid
 * restricted to a spherical or cubic simulation box, and propagates the
 * batch in time with a 4th-order Taylor expansion of exp(-i dt H).
 *
 *   - Uniform grid, integrals as h^3-weighted grid sums, high-order finite
 *     differences for the Laplacian: section "Introduction".  Lap_h is the
 *     8th-order 25-point star; orbitals vanish outside the box.
 *   - Fields are linear arrays over the box points with the grid structure
 *     held separately; the basic object is a group of several states:
 *     section "Parallelization, optimizations and graphics processing units".
 *   - Non-local pseudopotential projectors: section "Magnetic response and
 *     gauge invariance in real-space grids" (separable form, 4 real
 *     projectors per atom).
 *   - Discrete evolution operator U(dt) applied step after step: section
 *     "Photoemission".
 *   - Optimal-control gradient eq. (qoctgradient) with a backward-propagated
 *     costate and a field parametrised by sine (Fourier) coefficients:
 *     section "Quantum optimal control".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Layout     An orbital batch is orbital-major, [nst][ldp] complex with
 *             interleaved re/im: orbital n holds its value at compact point
 *             i at element n*ldp + i.  ldp >= np; elements np..ldp-1 of each
 *             orbital are neither read nor written.  Compact point order is
 *             z-major, then y, then x, so each grid row of an orbital is
 *             contiguous.
 *  Dtypes     RSG_C128: complex128 (FP64) everywhere.
 *             RSG_C64_MIXED: the orbital batch the caller passes is still
 *             complex128; the Hamiltonian arithmetic (stencil, local
 *             potential, projectors) runs in FP32 on complex64 copies while
 *             the time-step accumulation of psi stays in FP64.
 *  Memory     Every pointer named *_dev, and every orbital/workspace
 *             pointer, is device memory owned by the caller.  Handles are
 *             opaque, owned by the library, released by rsg_*_destroy; a
 *             handle keeps its own copies of every table it was given.
 *  Streams    `stream` is a hipStream_t passed as void* (NULL = default
 *             stream).  Work is enqueued asynchronously on it; results in
 *             device memory are ready when the stream reaches them.
 *  Workspace  Entry points that need scratch device memory take (ws,
 *             ws_bytes); rsg_workspace_bytes() gives the size.
 *  Errors     0 on success, a negative RSG_E* code on failure.  Argument
 *             errors are detected before anything is enqueued.
 *             rsg_last_error() returns a thread-local message describing
 *             the last failure.  No C++ exception crosses this interface.
 */
#ifndef RSG_H
#define RSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RSG_OK = 0,
    RSG_EINVAL = -1,       /* null pointer, bad enum, negative size ... */
    RSG_ESHAPE = -2,       /* ldp < np, sizes inconsistent with the grid */
    RSG_EDTYPE = -3,       /* unknown dtype */
    RSG_EHIP = -4,         /* a HIP runtime call failed */
    RSG_ENOMEM = -5,       /* workspace too small or allocation failed */
    RSG_EUNSUPPORTED = -6  /* valid request the library does not serve */
};

enum { RSG_C128 = 0, RSG_C64_MIXED = 1 };
enum { RSG_BOX_CUBE = 0, RSG_BOX_SPHERE = 1 };

/* Operations for rsg_workspace_bytes. */
enum {
    RSG_OP_HPSI = 0,
    RSG_OP_STEP = 1,
    RSG_OP_REDUCE = 2,     /* rsg_dot, rsg_norm2, rsg_dipole_expectation */
    RSG_OP_ENERGY = 3,
    RSG_OP_ADJOINT = 4
};

typedef struct rsg_grid_s *rsg_grid_t;
typedef struct rsg_ham_s *rsg_ham_t;
typedef struct rsg_batch_s *rsg_batch_t;

/* ------------------------------------------------------------------ */
/* Grid                                                                */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t shape;   /* RSG_BOX_CUBE or RSG_BOX_SPHERE */
    int32_t n;       /* cube: points per axis (>= 1) */
    double radius;   /* sphere: radius in bohr (> 0) */
    double h;        /* grid spacing in bohr (> 0) */
} rsg_grid_desc;

/* Uniform grid restricted to the box ("Introduction"; "Parallelization,
 * optimizations and graphics processing units": linear arrays plus grid
 * metadata).  Sphere: the centre is a grid point and centred integer
 * offsets (i,j,k) are inside iff i^2+j^2+k^2 <= floor((radius/h)^2 + 1e-9).
 * Cube: n^3 points, positions h*(i - (n-1)/2) per axis.  The box membership
 * and compact numbering are computed by GPU kernels on `stream`; the call
 * returns once the point count is known.  Errors: RSG_EINVAL for a bad
 * descriptor, RSG_EHIP on a runtime failure. */
int rsg_grid_create(const rsg_grid_desc *desc, void *stream, rsg_grid_t *out);

/* The same box with row-aligned storage (a layout choice of this library;
 * the paper keeps fields as linear arrays over the box points, section
 * "Parallelization, optimizations and graphics processing units").  The
 * order of the points is unchanged, but every non-empty (y, z) row owns the
 * slots of its x-range widened to multiples of align, so that its slot at
 * x = 0 (mod align) starts a memory line: a stencil tile's row segment then
 * touches no partly used line at its start.  The extra "dead" slots (at
 * most 2 (align - 1) per row) hold no point.  align: a power of two in
 * 1..64 (1 gives rsg_grid_create's compact layout).  Every field on such a
 * grid has np slots (rsg_grid_info); callers keep zeros in the dead slots
 * of their inputs (reductions sum every slot), and every stencil output
 * (rsg_hpsi, the Taylor stages, the adjoint) writes zero there.  Projector
 * supports must name box points.  Grid-to-memory maps need align 1.
 * Errors as rsg_grid_create, RSG_EINVAL for a bad align. */
int rsg_grid_create_aligned(const rsg_grid_desc *desc, int32_t align, void *stream, rsg_grid_t *out);

/* Rectangular box of nx x ny x nz points (each 1..32767, fewer than 2^31 in
 * all), positions h*(i - (n_a - 1)/2) along axis a, compact order z, y, x,
 * row alignment as rsg_grid_create_aligned.  A box one point thick in y and
 * z holds a one-dimensional problem: the y and z taps of the star stencil
 * then reach only points outside the box (zero), so H is the
 * one-dimensional Hamiltonian plus the constant 2 kin c_0 / h^2 (times
 * e^{-2 i theta} under complex scaling).  Errors as rsg_grid_create. */
int rsg_grid_create_box(int32_t nx, int32_t ny, int32_t nz, double h, int32_t align, void *stream,
                        rsg_grid_t *out);

/* np: slots per field (the number of box points unless the grid is
 * row-aligned); dims: tight bounding box (x, y, z); h.  Any output pointer
 * may be NULL. */
int rsg_grid_info(rsg_grid_t g, int64_t *np, int32_t dims[3], double *h);

/* npoints: box points (np minus the dead slots); align: the grid's row
 * alignment.  Either pointer may be NULL. */
int rsg_grid_points(rsg_grid_t g, int64_t *npoints, int32_t *align);

/* Host copies over the np slots: ijk_host [np][3] int32 box coordinates
 * (0 <= ijk < dims; -1 for a dead slot), xyz_host [np][3] float64 positions
 * in bohr (0 for a dead slot). */
int rsg_grid_coords(rsg_grid_t g, int32_t *ijk_host);
int rsg_grid_positions(rsg_grid_t g, double *xyz_host);
int rsg_grid_destroy(rsg_grid_t g);

/* ------------------------------------------------------------------ */
/* Hamiltonian                                                         */
/* ------------------------------------------------------------------ */

/* One atom's separable projectors (4 real functions on its support S_a). */
typedef struct {
    int64_t n_support;   /* |S_a| >= 0 */
    const int32_t *idx;  /* device [n_support]: distinct compact indices */
    const double *p;     /* device [n_support][4]: p_i^a at those points */
    double E[4];         /* projector energies E_i^a (Hartree) */
} rsg_proj_desc;

/* H = kin*Lap_h + V + field*x_axis + sum_a sum_i |p_i^a> E_i^a h^3 <p_i^a|.
 * vloc_dev: device [np] float64 local potential (NULL = 0).  kin: -0.5 for
 * the Kohn-Sham kinetic energy.  dipole_axis: 0, 1, 2 (x, y, z) or -1.
 * The handle copies V and every projector table; the grid must outlive the
 * handle.  Errors: RSG_EINVAL (bad axis, null tables with n_support > 0,
 * index out of range), RSG_EHIP. */
int rsg_ham_create(rsg_grid_t g, const double *vloc_dev, double kin, int32_t dipole_axis,
                   int32_t natoms, const rsg_proj_desc *proj, rsg_ham_t *out);
int rsg_ham_destroy(rsg_ham_t H);

/* Mask boundary absorber (section "Photoemission", eq. (mask_split) and the
 * outgoing-flow propagation after it): with a mask set, every Taylor(4)
 * step of this Hamiltonian (rsg_propagate_step, rsg_propagate) ends with
 * psi <- M(r) psi, the part (1 - M) psi leaving the simulation box.
 * mask_dev: device [np] float64, real values (normally in [0, 1]); the
 * handle copies it.  NULL removes the mask.  The multiply is fused into the
 * last stage of the step (psi + (-i dt) H y, see rsg_propagate_step) and
 * its projector scatter.  The charge that leaves is
 * the drop of rsg_norm2 across a step.  rsg_adjoint_step, the control entry
 * points and rsg_batch_create reject a masked Hamiltonian
 * (RSG_EUNSUPPORTED).  Errors: RSG_EINVAL, RSG_EHIP. */
int rsg_ham_set_mask(rsg_ham_t H, const double *mask_dev);

/* Scratch device bytes an operation needs for a batch of nst orbitals with
 * orbital stride ldp (0 when the arguments are invalid). */
size_t rsg_workspace_bytes(rsg_ham_t H, int32_t op, int64_t nst, int64_t ldp, int32_t dtype);

/* hpsi = H psi at the given field value ("application of a Hamiltonian" as
 * a building block, section "Parallelization, optimizations and graphics
 * processing units").  psi and hpsi: device [nst][ldp] complex128, must not
 * overlap.  dtype RSG_C128 only.  ws: RSG_OP_HPSI bytes. */
int rsg_hpsi(rsg_ham_t H, const void *psi, void *hpsi, int64_t nst, int64_t ldp, int32_t dtype,
             double field, void *ws, size_t ws_bytes, void *stream);

/* One Taylor(4) step in place: psi <- sum_{k=0}^{4} (-i dt H)^k / k! psi,
 * with H taken at `field` (the field at the step midpoint); the discrete
 * evolution operator of section "Photoemission".  psi: device [nst][ldp]
 * complex128.  dtype RSG_C128 or RSG_C64_MIXED.  ws: RSG_OP_STEP bytes.
 * RSG_C128 without an absorber mask evaluates the polynomial as the product
 * of its four linear factors (1 + (i dt / r_k) H), r_k its roots: four
 * stages that each read only their input.  RSG_C64_MIXED and a masked step
 * use T4(z) = 1 + z prod_j (1 - z / s_j), s_j the roots of the cubic
 * 1 + z/2 + z^2/6 + z^3/24: three such stages from psi into complex64
 * (mixed) or complex128 work buffers, then psi_out = psi + (-i dt) H y, so
 * psi is read only by the first and the last stage and stays FP64. */
int rsg_propagate_step(rsg_ham_t H, void *psi, int64_t nst, int64_t ldp, int32_t dtype, double dt,
                       double field, void *ws, size_t ws_bytes, void *stream);

/* nsteps Taylor(4) steps; step n uses fields_dev[n] (device float64
 * [nsteps]) or zero field when fields_dev is NULL.  use_graph != 0 captures
 * the step sequence into a HIP graph once per distinct argument set and
 * replays it.  Same buffers as rsg_propagate_step. */
int rsg_propagate(rsg_ham_t H, void *psi, int64_t nst, int64_t ldp, int32_t dtype, double dt,
                  int64_t nsteps, const double *fields_dev, int32_t use_graph, void *ws,
                  size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Reductions: <a|b> = h^3 sum_r conj(a(r)) b(r), per orbital           */
/* (integration as a grid sum, section "Introduction").  Deterministic:  */
/* fixed two-pass order, identical results run to run.                 */
/* ------------------------------------------------------------------ */

/* Scratch bytes for rsg_dot / rsg_norm2 / rsg_dipole_expectation. */
size_t rsg_reduce_workspace_bytes(rsg_grid_t g, int64_t nst);

/* out_dev: device float64 [2*nst] (re, im per orbital). ws: RSG_OP_REDUCE. */
int rsg_dot(rsg_grid_t g, const void *a, const void *b, int64_t nst, int64_t ldp, double *out_dev,
            void *ws, size_t ws_bytes, void *stream);
/* out_dev: device float64 [nst], h^3 sum |a|^2. */
int rsg_norm2(rsg_grid_t g, const void *a, int64_t nst, int64_t ldp, double *out_dev, void *ws,
              size_t ws_bytes, void *stream);
/* out_dev: device float64 [2*nst], <psi_n|H psi_n> per orbital (the total
 * energy is the sum of the real parts). ws: RSG_OP_ENERGY bytes. */
int rsg_energy(rsg_ham_t H, const void *psi, int64_t nst, int64_t ldp, int32_t dtype, double field,
               double *out_dev, void *ws, size_t ws_bytes, void *stream);
/* out_dev: device float64 [nst], h^3 sum x_axis |a|^2 along the
 * Hamiltonian's dipole axis.  ws: RSG_OP_REDUCE bytes. */
int rsg_dipole_expectation(rsg_ham_t H, const void *a, int64_t nst, int64_t ldp, double *out_dev,
                           void *ws, size_t ws_bytes, void *stream);

/* rsg_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and the same result, bit for bit, with the partial sums in a
 * static device array of rsg_dot_noalloc_max_bytes() bytes (1 MiB) instead of
 * a caller workspace.  The call allocates nothing and synchronises nothing.
 * Limit: rsg_reduce_workspace_bytes(g, nst) must not exceed that size
 * (every grid up to 64 orbitals fits), else RSG_EUNSUPPORTED before
 * anything is enqueued.  Each GPU holds one such array for the life of the
 * process, shared by every call on that GPU: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 * Other arguments and errors as rsg_dot. */
int rsg_dot_noalloc(rsg_grid_t g, const void *a, const void *b, int64_t nst, int64_t ldp, double *out_dev,
                    void *stream);
size_t rsg_dot_noalloc_max_bytes(void);

/* ------------------------------------------------------------------ */
/* Optimal control (section "Quantum optimal control")                 */
/* ------------------------------------------------------------------ */

/* E(tau_n) = sum_{k=1}^{ncoef} c_k sin(k pi tau_n / T), tau_n = (step0 + n
 * + 1/2) dt, for n = 0..nsteps-1.  coef_dev device [ncoef], out_dev device
 * [nsteps]. */
int rsg_laser_field(const double *coef_dev, int32_t ncoef, double T, double dt, int64_t step0,
                    int64_t nsteps, double *out_dev, void *stream);

/* grad_dev[k-1] = sum_{n<nsteps} sin(k pi tau_n / T) g_dev[n]: the chain rule
 * from per-step field derivatives to the sine coefficients.  Fixed-order
 * sums. */
int rsg_laser_grad(const double *g_dev, int64_t nsteps, double T, double dt, int32_t ncoef,
                   double *grad_dev, void *stream);

/* One discrete adjoint step for psi_{n+1} = T4(-i dt H_n) psi_n with
 * H_n = H(field).  In: psi_n, lambda = lambda_{n+1}.  Out: lambda =
 * T4(+i dt H_n) lambda_{n+1} (the costate one step back), and
 * g_dev[0] = dJ/dE_n = 2 Re sum_{l=0}^{3} <H^l lambda_{n+1}| x_axis |w_l>,
 * w_l = sum_{m=0}^{3-l} a_{l+m+1} H^m psi_n, a_j = (-i dt)^j / j!: the
 * time-discrete form of eq. (qoctgradient).  Computed in the product form
 * of the step (see rsg_control_backward): the three stage outputs of psi_n
 * are recomputed, then four adjoint stages on lambda and one pass over the
 * four stage pairs; equal to the formulas above in exact arithmetic.
 * Needs a dipole axis.  ws: RSG_OP_ADJOINT bytes. */
int rsg_adjoint_step(rsg_ham_t H, const void *psi_n, void *lambda, int64_t nst, int64_t ldp,
                     double dt, double field, double *g_dev, void *ws, size_t ws_bytes,
                     void *stream);

/* Scratch bytes for rsg_control_forward / rsg_control_backward with these
 * sizes (the checkpoint store is separate and owned by the caller).  For a
 * handle whose steps run in product form (no absorber mask) the segment
 * store holds, per step, the state and its three stage outputs: about
 * 4 ckpt_every orbital batches. */
size_t rsg_control_workspace_bytes(rsg_ham_t H, int64_t nst, int64_t ldp, int64_t nsteps,
                                   int64_t ckpt_every);

/* The least scratch bytes the control entry points accept: the segment
 * store holds the states only (ckpt_every batches plus three), and each
 * adjoint step recomputes its three stage outputs, so the backward pass
 * runs 3 more stencil stages per step (about 25 % more stencil work).  Any
 * workspace of at least rsg_control_workspace_bytes takes the faster path. */
size_t rsg_control_workspace_bytes_min(rsg_ham_t H, int64_t nst, int64_t ldp, int64_t nsteps,
                                       int64_t ckpt_every);

/* Forward pass of the control problem: nsteps Taylor(4) steps of psi (in:
 * psi(0), out: psi(T), T = nsteps*dt) under the field of coef_dev, storing
 * psi at every step that is a multiple of ckpt_every (step 0 included) in
 * ckpt_dev [nsteps/ckpt_every + 1][nst][ldp] complex128.  J_dev[0] =
 * sum_n <psi_n(T)| x_axis |psi_n(T)>.  ckpt_dev may be NULL (no checkpoints
 * kept).  ws: rsg_control_workspace_bytes. */
int rsg_control_forward(rsg_ham_t H, void *psi, int64_t nst, int64_t ldp, double dt,
                        int64_t nsteps, const double *coef_dev, int32_t ncoef,
                        int64_t ckpt_every, void *ckpt_dev, double *J_dev, void *ws,
                        size_t ws_bytes, void *stream);

/* Backward pass: lambda_N = x_axis psi(T); segment by segment, newest
 * first, recompute the segment's states from its checkpoint, then take
 * adjoint steps back through it.  grad_dev [ncoef] = dJ/dc; g_steps_dev
 * [nsteps] (may be NULL) = dJ/dE_n.  psi_T: device [nst][ldp], unchanged.
 * ws: rsg_control_workspace_bytes.  Product-form steps psi_{n+1} = F4 F3
 * F2 F1 psi_n (F_k = 1 + a_k H, see rsg_propagate_step): the recompute
 * keeps each step's stage outputs y_1..y_3 (y_0 = psi_n), the costate
 * runs back through the adjoint factors, m_4 = lambda_{n+1}, m_{k-1} =
 * (1 + conj(a_k) H) m_k, lambda_n = m_0, and dJ/dE_n = 2 Re sum_k a_k
 * <m_k| x_axis |y_{k-1}>, as in rsg_adjoint_step. */
int rsg_control_backward(rsg_ham_t H, const void *psi_T, int64_t nst, int64_t ldp, double dt,
                         int64_t nsteps, const double *coef_dev, int32_t ncoef,
                         int64_t ckpt_every, const void *ckpt_dev, double *grad_dev,
                         double *g_steps_dev, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Stencil tile shapes and the autotuner                               */
/* ------------------------------------------------------------------ */

/* Tile of the z-marching stencil kernel: B orbitals (1) x TX x TY grid
 * columns per workgroup, marching along z in chunks of ZC planes (0 = whole
 * box), with PD planes in flight (1..2: pipelined march; 0: lean march).
 * PT = 1 launches the tiles of each z-chunk in Morton (Z-curve) order;
 * PT >= 2 launches them in PT x PT patches that share a z-range, so that
 * neighbouring workgroups march together; 0 = row order.  BO = 0 launches
 * the orbitals of a tile together, BO = 1 sweeps all tiles of one orbital
 * before the next, BO = G in 2..64 sweeps the tiles with G orbitals of each
 * tile side by side.  ZM = 0 marches each tile upward from its lowest plane;
 * ZM = 1 marches every tile outward from the box's centre plane (upward
 * above it, downward below it), longest tiles first within a z-chunk, so
 * that workgroups resident together cover neighbouring tiles at the same
 * plane; ZM = 2 aligns the z-chunks to multiples of ZC for every tile
 * (chunk-major order), so that workgroups launched together march the same
 * planes side by side. */
typedef struct {
    int32_t B, TX, TY, ZC, PD, PT, BO, ZM;
} rsg_tile;

/* Compiled tile shapes for a dtype (ZC = 0).  Writes up to max entries and
 * the total count. */
int rsg_tile_candidates(int32_t dtype, rsg_tile *out, int32_t max, int32_t *count);

/* Use tile t for batches of nst orbitals in dtype on this Hamiltonian.
 * RSG_EUNSUPPORTED if (B, TX, TY, PD) is not compiled. */
int rsg_set_tile(rsg_ham_t H, int64_t nst, int32_t dtype, const rsg_tile *t);
int rsg_get_tile(rsg_ham_t H, int64_t nst, int32_t dtype, rsg_tile *t);

/* Tile autotuner for the Taylor(4) step on psi (device [nst][ldp], left
 * unchanged).  Phase 1 times one of the middle Taylor stages (reads a work
 * buffer, writes the other) for every compiled tile
 * shape, z-chunk lengths {whole, 64, 32, and 16, 8, 4, 2, 1 when the batch
 * has few tiles}, PT {0, 1}, BO {0, 1, 2, 4} and ZM {0, 1} with HIP events (best of
 * reps launches after a warm-up launch; a stage under 0.2 ms is timed as the
 * mean of 16 back-to-back launches).  Phase 2 re-times the six fastest
 * on the stencil work of a whole step (the first stage plus three later
 * ones, 3 reps launches each), keeps the fastest for (nst, dtype) and
 * returns it in *best and that step time in *best_ms (either may be NULL).
 * ws: RSG_OP_STEP bytes (both work buffers are used).  Synchronises the
 * stream. */
int rsg_autotune(rsg_ham_t H, const void *psi, int64_t nst, int64_t ldp, int32_t dtype, void *ws,
                 size_t ws_bytes, int32_t reps, rsg_tile *best, double *best_ms, void *stream);

/* rsg_autotune with a tile cache in the text file cache_path, one line per
 * tuned case: "<key> | B TX TY ZC PD PT BO ZM | ms".  The key names the box
 * shape, its dimensions, point and slot counts, the row alignment, nst, the
 * dtype, complex scaling and mask use, and the device (architecture name
 * and compute-unit count).  If the file holds the key (the last such line
 * wins) the tile is set with no kernel launch and *cached = 1; otherwise
 * the autotuner runs as rsg_autotune does, its choice is appended to the
 * file and *cached = 0.  best, best_ms and cached may be NULL.  The file is
 * created if missing; concurrent writers may append the same key twice,
 * which is harmless.  Errors: those of rsg_autotune, and RSG_EINVAL when
 * the file cannot be written. */
int rsg_autotune_cache(rsg_ham_t H, const void *psi, int64_t nst, int64_t ldp, int32_t dtype, void *ws,
                       size_t ws_bytes, int32_t reps, const char *cache_path, rsg_tile *best, double *best_ms,
                       int32_t *cached, void *stream);

/* ------------------------------------------------------------------ */
/* Many independent systems                                            */
/* ------------------------------------------------------------------ */

/* One system of a batch: its Hamiltonian (and grid) and its orbitals,
 * device [nst][ldp] complex128, propagated in place.  No dipole field. */
typedef struct {
    rsg_ham_t ham;
    void *psi;
    int64_t nst, ldp;
} rsg_system_desc;

/* Scratch bytes rsg_batch_create needs for these systems. */
size_t rsg_batch_workspace_bytes(int32_t nsys, const rsg_system_desc *sys);

/* Group nsys independent systems (the group of states of section
 * "Parallelization, optimizations and graphics processing units", extended
 * across systems).  The systems fall into size classes by the width of their
 * tight box (narrower than 48 points, 48 to 79, 80 or more; empty classes
 * are dropped), and each class has its own stencil tile shape (initially
 * 32 x 8, depth 2).  Each stage of a Taylor(4) step of all systems runs as
 * one persistent stencil launch per class over a list of (system, tile,
 * z-range, orbital) items (largest systems first; cut into one segment per
 * XCD, each workgroup taking items from its own XCD's segment first and
 * then from the others), with one projector
 * gather launch and one scatter launch per colour for all systems.  ws
 * (rsg_batch_workspace_bytes) holds the work buffers and must outlive the
 * batch, as must every Hamiltonian and orbital array named in sys.  Results
 * are bitwise equal to propagating each system alone with its class's tile.
 * Errors: RSG_EINVAL, RSG_ESHAPE, RSG_ENOMEM, RSG_EUNSUPPORTED (a system
 * with a dipole axis, a mask or complex scaling), RSG_EHIP. */
int rsg_batch_create(int32_t nsys, const rsg_system_desc *sys, void *ws, size_t ws_bytes, void *stream,
                     rsg_batch_t *out);
/* The same call under the name of the plan/run pair below. */
int rsg_batch_plan_create(int32_t nsys, const rsg_system_desc *sys, void *ws, size_t ws_bytes, void *stream,
                          rsg_batch_t *out);
int rsg_batch_destroy(rsg_batch_t b);

/* Size classes: *nclass, and (if class_of_sys is not NULL) the class of
 * every system.  rsg_batch_set_classes replaces the classes: class_of_sys[i]
 * in 0..nclass-1 for every system, every class non-empty (RSG_EINVAL
 * otherwise); every class restarts with the 32 x 8 depth-2 tile. */
int rsg_batch_classes(rsg_batch_t b, int32_t *nclass, int32_t *class_of_sys);
int rsg_batch_set_classes(rsg_batch_t b, const int32_t *class_of_sys, void *stream);

/* Tile shape of every class (rsg_batch_set_tile) or of class c (FP64 shapes
 * of rsg_tile_candidates; PT and BO are ignored).  rsg_batch_get_tile
 * reports the tile of the class with the most grid-point x orbital work.
 * RSG_EUNSUPPORTED for a shape that is not compiled. */
int rsg_batch_set_tile(rsg_batch_t b, const rsg_tile *t, void *stream);
int rsg_batch_set_class_tile(rsg_batch_t b, int32_t c, const rsg_tile *t, void *stream);
int rsg_batch_get_tile(rsg_batch_t b, rsg_tile *t);
int rsg_batch_get_class_tile(rsg_batch_t b, int32_t c, rsg_tile *t);

/* Class c: its number of systems, its stencil work items per stage
 * (tiles x z-chunks x orbitals) and the workgroups its persistent launch
 * runs (at most nitems; each takes items until the list is exhausted). */
int rsg_batch_class_info(rsg_batch_t b, int32_t c, int32_t *nsys, int64_t *nitems, int32_t *grid);

/* At most max_workgroups persistent workgroups per stencil launch (0: as
 * many as are resident on the device, the default).  Fewer workgroups take
 * more items each; the results do not change.  Drops captured graphs. */
int rsg_batch_set_grid(rsg_batch_t b, int32_t max_workgroups);

/* Autotuner over the size classes: for each class, every compiled FP64 tile
 * shape x z-chunk {whole, 32} x z-march {upward, centre-out}, timed on that
 * class's persistent launch of a middle Taylor stage (best of reps after a
 * warm-up); the fastest per class is kept.  *best: the tile of the class
 * with the most work; *best_ms: the sum over classes of their best stage
 * times.  The orbitals are not modified.  Synchronises the stream. */
int rsg_batch_autotune(rsg_batch_t b, int32_t reps, rsg_tile *best, double *best_ms, void *stream);

/* nsteps Taylor(4) steps of every system at time step dt, zero field.
 * use_graph != 0 captures the launch sequence into a HIP graph once per
 * (dt, nsteps, stream) and replays it; needs a non-default stream. */
int rsg_batch_propagate(rsg_batch_t b, double dt, int64_t nsteps, int32_t use_graph, void *stream);
/* rsg_batch_propagate with graph capture: the run half of the plan/run pair. */
int rsg_batch_run(rsg_batch_t b, int64_t nsteps, double dt, void *stream);

/* ------------------------------------------------------------------ */
/* Complex scaling                                                     */
/* ------------------------------------------------------------------ */

/* Section "Complex scaling and resonances": under r -> r e^{i theta} the
 * Hamiltonian becomes H_theta = kin e^{-2 i theta} Lap_h + v(r e^{i theta}),
 * symmetric but not Hermitian; bound-state energies stay put, the continuum
 * rotates by -2 theta and resonances appear as eigenvalues eps - i Gamma/2.
 * After this call every H application of the handle (rsg_hpsi,
 * rsg_propagate_step, rsg_propagate, rsg_energy, rsg_shifted_solve with QMR)
 * uses kin e^{-2 i theta} and the local potential V + i V_im, where V is
 * the real part given at creation (the caller evaluates the continued
 * potential) and vim_dev (device [np] float64, copied; NULL = 0) its
 * imaginary part.  theta = 0 with vim_dev = NULL restores the Hermitian
 * operator.  Only the FP64 path is complex-scaled (RSG_C64_MIXED returns
 * RSG_EUNSUPPORTED).  The complex-scaled stencil runs the handle's tile at
 * pipeline depth 1 (8x8, 16x8, 16x16 and 32x16 are built; another tile runs
 * as 16x8).  Errors: RSG_EINVAL (theta not finite), RSG_EUNSUPPORTED
 * (the handle has projectors or an absorber mask; the adjoint, control,
 * batch and CG entry points reject a complex-scaled handle), RSG_EHIP. */
int rsg_ham_set_complex_scaling(rsg_ham_t H, double theta, const double *vim_dev);

/* Bilinear form without conjugation, out_dev[2n], out_dev[2n+1] = re, im of
 * h^3 sum_r a_n(r) b_n(r) (the matrix elements of complex scaling).  Same
 * arguments and errors as rsg_dot. */
int rsg_bilinear(rsg_grid_t g, const void *a, const void *b, int64_t nst, int64_t ldp, double *out_dev,
                 void *ws, size_t ws_bytes, void *stream);

/* Eigenvalues of the (complex-scaled) Hamiltonian nearest the targets
 * z_n (host [2*nst], re and im), one per orbital, by shifted inverse
 * iteration: psi_n <- (H - z_n)^{-1} psi_n with rsg_shifted_solve (QMR,
 * qmr_tol, qmr_maxiter), normalised to h^3 psi^T psi = 1, lambda_n = h^3
 * psi_n^T H psi_n, until every lambda changes by at most tol max(1,
 * |lambda|) or after max_outer iterations.  psi: device [nst][ldp]
 * complex128, start vectors in, eigenvectors out.  lambda: host [2*nst]
 * out; outer_iters: host [nst] or NULL.  ws: rsg_cs_eigs_workspace_bytes.
 * Synchronises the stream.  Errors: RSG_EINVAL (targets, tolerances, a
 * start vector of zero bilinear norm), RSG_ESHAPE, RSG_ENOMEM, RSG_EHIP. */
size_t rsg_cs_eigs_workspace_bytes(rsg_ham_t H, int64_t nst, int64_t ldp);
int rsg_cs_eigs(rsg_ham_t H, const double *target, void *psi, int64_t nst, int64_t ldp, int32_t max_outer,
                double tol, int32_t qmr_maxiter, double qmr_tol, double *lambda, int32_t *outer_iters, void *ws,
                size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Shifted-Hamiltonian solves                                          */
/* ------------------------------------------------------------------ */

/* Section "The Sternheimer formulation of linear-response", eq.
 * (sternheimer): each Sternheimer iteration
 * solves (H - eps_n +- omega + i eta) x_n = b_n for every occupied orbital;
 * the paper uses conjugate gradients for a real shift and the quasi-minimal
 * residual method (Freund and Nachtigal, Numer. Math. 60, 315 (1991)) for a
 * complex one.  Here sigma_n stands for the whole shift -eps_n +- omega +
 * i eta and the operator is the Hamiltonian without field (complex-scaled
 * or not), so A_n = H + sigma_n is complex symmetric and QMR needs one H
 * application per iteration; CG needs a Hermitian H. */
enum { RSG_SOLVE_CG = 0, RSG_SOLVE_QMR = 1 };

/* Workspace bytes of rsg_shifted_solve (6 batch buffers for QMR, 3 for CG,
 * the projector buffer, partial sums and per-orbital state); 0 on bad
 * arguments. */
size_t rsg_solve_workspace_bytes(rsg_ham_t H, int32_t method, int64_t nst, int64_t ldp);

/* Solves (H + sigma_n) x_n = b_n for n < nst.  shift: host [2*nst], re and
 * im of sigma_n (CG: im must be 0).  b, x: device orbital-major [nst][ldp]
 * complex128; x holds the initial guess on entry and the solution on exit;
 * b and x must not overlap.  Orbital n stops when ||b - A x|| <= tol ||b||
 * (the recurrence residual; ||b|| = 0 counts as 1), after maxiter
 * iterations or at a breakdown of the recurrence; all orbitals iterate
 * together and a stopped orbital is left untouched.  The host reads the
 * stop flags every check_every iterations (one synchronisation each) and
 * returns when all have stopped.  Outputs (host, [nst], each may be NULL):
 * iters, rel_res = ||r|| / ||b||, status = 0 converged, 1 iteration limit,
 * 2 breakdown.  ws: rsg_solve_workspace_bytes.  Synchronises the stream.
 * Errors: RSG_EINVAL (method, shift, tol, overlap), RSG_ESHAPE (nst
 * outside 1..65535, ldp < np), RSG_ENOMEM (workspace), RSG_EHIP. */
int rsg_shifted_solve(rsg_ham_t H, const double *shift, const void *b, void *x, int64_t nst, int64_t ldp,
                      int32_t method, double tol, int32_t maxiter, int32_t check_every, int32_t *iters,
                      double *rel_res, int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Grid-to-memory maps                                                 */
/* ------------------------------------------------------------------ */

/* Section "Parallelization, optimizations and graphics processing units",
 * figures gridmaps and gpu_laplacian: a grid function is a linear array and
 * the order in which grid points are stored in it is free.  A map is such an
 * order together with the neighbour table of the 25-point star stencil in
 * it, for a generic (gather-form) finite-difference Laplacian that works
 * with any order.  Kinds:
 *   RSG_MAP_STANDARD  the compact order (z, then y, then x fastest);
 *   RSG_MAP_BRICKS    the tight box cut into param^3 bricks, bricks in the
 *                     compact order of their corner, points inside a brick in
 *                     compact order;
 *   RSG_MAP_HILBERT   ascending 3D Hilbert index of the box coordinates
 *                     (x, y, z) on the enclosing 2^b cube, from the
 *                     axes-to-transpose transform of Skilling (AIP Conf.
 *                     Proc. 707, 2004), x the most significant axis of each
 *                     level.
 * The map holds a device table of 24 int32 per point (96 B/pt). */
typedef struct rsg_map_s *rsg_map_t;
enum { RSG_MAP_STANDARD = 0, RSG_MAP_BRICKS = 1, RSG_MAP_HILBERT = 2 };

/* Builds the order and the neighbour table on the host from the grid's row
 * table and uploads the table; param = brick edge (1..64) for
 * RSG_MAP_BRICKS, ignored otherwise.  The grid must outlive the map.
 * Errors: RSG_EINVAL (null argument, unknown kind, bad brick edge),
 * RSG_EUNSUPPORTED (a row-aligned grid), RSG_ENOMEM, RSG_EHIP. */
int rsg_map_create(rsg_grid_t g, int32_t kind, int32_t param, rsg_map_t *out);
int rsg_map_destroy(rsg_map_t m);

/* order_host[i] = compact index of the i-th point in map order (host
 * [np] int32, caller-owned).  A grid function f in compact order is
 * f[order] in map order. */
int rsg_map_order(rsg_map_t m, int32_t *order_host);

/* out = scale * sum over the 25 stencil taps of c_|m| psi(r + m h e_axis)
 * (the 8th-order star of rsg_hpsi's kinetic term, psi = 0 outside the box),
 * with psi and out both in map order and in the point-major batch layout
 * [np][ld] complex128 (orbital fastest, nst <= ld).  kin * Lap_h is
 * scale = kin / h^2.  Columns nst..ld-1 of out are not written; psi and out
 * must not overlap.  One thread per (point, orbital); consecutive
 * workgroups are kept on one XCD so that points close in the map share that
 * XCD's L2.  Errors: RSG_EINVAL, RSG_ESHAPE (nst < 1 or ld < nst),
 * RSG_EHIP. */
int rsg_map_laplacian(rsg_map_t m, const void *psi, void *out, int64_t nst, int64_t ld, double scale,
                      void *stream);

/* ------------------------------------------------------------------ */
/* Misc                                                                */
/* ------------------------------------------------------------------ */

/* Thread-local description of the last failure ("" if none). */
const char *rsg_last_error(void);

/* Library version string. */
const char *rsg_version(void);

/* Plain device copy of n bytes (16-byte aligned pointers, n % 16 == 0),
 * one read and one write per byte; used to calibrate HBM traffic counters
 * and to measure achievable copy bandwidth. */
int rsg_copy(const void *src, void *dst, size_t nbytes, void *stream);

/* Kernel timing.  While enabled, the library records a HIP event pair
 * around every launch of the stencil kernel on the launch stream; the
 * query returns the number of timed launches and their mean duration in
 * milliseconds (synchronising on the recorded events), then clears them. */
int rsg_timing_enable(int32_t on);
int rsg_timing_query(int64_t *count, double *mean_ms, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* RSG_H */
