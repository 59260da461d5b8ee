/*
 * sgrid — contiguous narrow-band sparse grids on MI355X (gfx950).
 *
 * C ABI of the hot path of "Contiguous Storage of Grid Data for
 * Heterogeneous Computing": 4x4x4 data packages of the activated coarse
 * cells held in one contiguous array per field, found through a
 * cell-to-package index map and a 27-entry neighbour-package table.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Domain: the cube [0, 4 M h)^3.  M = n_coarse coarse cells per axis of
 *    size l_c = 4h; N = 4M data points per axis, data point (i, j, k) at
 *    ((i, j, k) + 1/2) h.  Coarse cell (a, b, c) has linear index
 *    a + M b + M^2 c (x fastest).
 *  - Package ids: 0 is the negative (inside) far field, 1 the positive
 *    (outside) far field, 2 .. P+1 the P activated cells in ascending
 *    linear cell order (Sec. 5, Sec. 7.1 step 3).  P^ = P + 2.
 *  - A field is stored as [P^][64] values; inside a package the data index
 *    (i, j, k) in 0..3 is stored at i + 4 j + 16 k.  Rows 0 and 1 hold the
 *    far-field constants -B and +B with B = 16 h (sgrid_fill_far_field).
 *    Vector fields (the gradient) are three such arrays back to back,
 *    [3][P^][64].
 *  - Neighbour slot of the shift (dx, dy, dz) in {-1,0,1}^3 is
 *    (dx+1) + 3 (dy+1) + 9 (dz+1); slot 13 is the package itself.
 *    Neighbours outside the domain are package 1; the far-field packages
 *    neighbour themselves (Sec. 5.2, Sec. 7.1 step 5).
 *  - Memory: every pointer argument named *_dev, and every field, is device
 *    memory owned by the caller (16-byte aligned); the grid handle owns its
 *    index tables.  `stream` is a hipStream_t (NULL = default stream).
 *    Calls are asynchronous on that stream, except sgrid_build_packages,
 *    which synchronises once to learn P.
 *  - Errors: every call returns an sgrid_status and never aborts; the text of
 *    the last failure on the calling thread is sgrid_last_error().  Argument
 *    checks run before any device work.  Faults of kernels already queued
 *    surface at the next call that synchronises.
 */
#ifndef SGRID_H
#define SGRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGRID_OK = 0,
    SGRID_E_INVALID = 1,   /* null, misaligned or out-of-range argument */
    SGRID_E_NOMEM = 2,     /* device allocation failed */
    SGRID_E_HIP = 3,       /* a HIP runtime call or kernel launch failed */
    SGRID_E_CAPACITY = 4,  /* a size does not fit the 32-bit index tables */
    SGRID_E_STATE = 5      /* handle used in a state that does not allow the call */
} sgrid_status;

typedef enum { SGRID_F32 = 0, SGRID_F64 = 1 } sgrid_dtype;

typedef struct sgrid_grid sgrid_grid;
typedef struct sgrid_mlp sgrid_mlp;
typedef struct sgrid_batch sgrid_batch;

typedef struct {
    int32_t n_coarse;   /* M >= 1, M^3 + 2 < 2^32 */
    double h;           /* data spacing, > 0; l_c = 4h */
} sgrid_desc;

typedef struct {
    int32_t n_coarse;
    double h;
    int64_t n_packages;          /* P (activated, excluding the two far-field packages) */
    int64_t n_core;              /* core packages among them */
    const uint32_t *cell_pkg;    /* device [M^3]: package id of every coarse cell */
    const uint32_t *pkg_cell;    /* device [P^]: linear cell of each package, 0xFFFFFFFF for 0 and 1 */
    const uint8_t *pkg_type;     /* device [P^]: 0 far field, 1 core, 2 inner */
    const uint32_t *pkg_nbr;     /* device [P^][27]: neighbour package ids */
    const uint32_t *core_list;   /* device [n_core]: ids of the core packages, ascending */
    const uint32_t *sweep_order; /* device [P]: activated package ids in Morton (Z-curve) order of their
                                    coarse cells; the order of sweep variant 3 */
    const uint32_t *rank_map;    /* device [M * M * rank_row][4]: cell_pkg in compact form, one entry per
                                    32 cells of a row (row y + M z, cells x = 32 e .. 32 e + 31):
                                    {activated bits, negative-sign bits, activated cells before the
                                    entry, 0}; bit b is cell 32 e + b.  The probe reads it. */
    int32_t rank_row;            /* entries per row: ceil(M / 32) */
} sgrid_info;

/* Text of the last failure on this thread ("" if none). */
const char *sgrid_last_error(void);

/* Library version, as major * 10000 + minor * 100 + patch. */
int32_t sgrid_version(void);

/*
 * Activation, numbering and neighbour table (Sec. 4, Sec. 5, Sec. 7.1 steps
 * 1-3 and 5).  `coarse_sdf_dev` [M^3] is the signed distance at every coarse
 * cell centre.  A cell is core when |d| < l_c and inner when it is not core
 * but one of its 26 neighbours is; both are activated and numbered 2.. in
 * ascending linear order; every other cell maps to far field 0 (d < 0) or 1.
 * The result is bit-identical for identical inputs.  On success *out owns the
 * tables until sgrid_destroy.  Synchronises `stream` once (to learn P); the
 * tables are complete when `stream` reaches the end of the call, so work on
 * other streams must wait for it.  Memory comes from the library's caching
 * allocator (blocks of destroyed grids are reused).
 */
sgrid_status sgrid_build_packages(const sgrid_desc *desc, const float *coarse_sdf_dev,
                                  void *stream, sgrid_grid **out);

/*
 * Consistency (sign) correction of a layer's distances (Sec. 7.2: only the
 * signs of cells very close to the surface are used directly; the others
 * come from a diffusion outward from them), the coarse step on the mesh
 * cells.  `d_dev` [M^3] (M = desc->n_coarse, x fastest, FP32): core cells
 * (|d| < 4 desc->h) keep their value.  Every other cell gets its sign by
 * rounds of simultaneous updates: a cell without a sign takes one when a face
 * neighbour has one, positive if any such neighbour is positive, else
 * negative, until a round changes nothing; such cells are written as |d| with
 * that sign, and cells no diffusion reaches keep d.  `out_dev` [M^3] may be
 * `d_dev` (in place).  *rounds_out (nullable) receives the number of rounds
 * that decided a cell.  Synchronises `stream` once per 16 rounds; workspace
 * M^3 / 2 bytes from the library's caching allocator.  M <= 4096.
 */
sgrid_status sgrid_correct_signs(const sgrid_desc *desc, const float *d_dev, float *out_dev, void *stream,
                                 int32_t *rounds_out);

/*
 * The refined step of the sign correction (Sec. 7.2: on a refined layer the
 * correction is limited to inner cells or data packages), on phi_dev
 * [P^][64] in place.  The points of core packages keep their sign, as the
 * core cells do in sgrid_correct_signs, and so do the far-field packages
 * (rows 0 and 1 must hold -B and +B; a neighbour outside the domain is the
 * positive far field).  The points of inner packages get their sign by the
 * same rounds of diffusion over face neighbours (positive if any decided
 * neighbour is positive, else negative) and take |phi| with it; points no
 * diffusion reaches keep phi.  *rounds_out (nullable) receives the number of
 * rounds that decided a point.  Synchronises `stream` once per 16 rounds;
 * workspace 2 bytes per point from the caching allocator.
 */
sgrid_status sgrid_correct_package_signs(const sgrid_grid *grid, sgrid_dtype dtype, void *phi_dev, void *stream,
                                         int32_t *rounds_out);

/*
 * The next layer of the multi-resolution construction (Sec. 7: layers of
 * successively doubled resolution, each initialised from the one before;
 * Sec. 7.1 step 1: a finer layer evaluates distances only in the cells that
 * the coarser layer's core cells cover).  The new grid has 2M cells per axis
 * and spacing h / 2.  `child_sdf_dev` [n_core][8] (FP32, device) holds the
 * signed distance at the centres of the eight children of each core cell of
 * `coarse`, rows in core_list order, child b = bx + 2 by + 4 bz.  A fine cell
 * under a core parent is tagged with its own distance; any other fine cell
 * is not core and takes its parent's sign (the parent's distance is at least
 * the parent cell size).  Then inner tagging, numbering, neighbours and the
 * sweep order as for sgrid_build_packages; for a signed distance function
 * the tables equal those of sgrid_build_packages on the dense (2M)^3
 * sampling.  `coarse` must stay alive until the call returns (it is only
 * read).  Synchronises `stream` once.  child_sdf_dev may be NULL when
 * `coarse` has no core cell.
 */
sgrid_status sgrid_build_packages_refined(const sgrid_grid *coarse, const float *child_sdf_dev, void *stream,
                                          sgrid_grid **out);

/* Sizes and device views of the tables (valid until sgrid_destroy). */
sgrid_status sgrid_get_info(const sgrid_grid *grid, sgrid_info *out);

/* Frees the tables; waits for the device first.  NULL is accepted. */
sgrid_status sgrid_destroy(sgrid_grid *grid);

/* Writes -B to package 0 and +B to package 1 of `phi_dev` [P^][64] (B = 16h). */
sgrid_status sgrid_fill_far_field(const sgrid_grid *grid, sgrid_dtype dtype, void *phi_dev,
                                  void *stream);

/*
 * Upwind reinitialisation (the paper names level-set operations on the band
 * without fixing the scheme; this is the Sussman-Smereka-Osher iteration
 * with Godunov upwinding): n_iter Jacobi sweeps over every point of every
 * activated package, with
 *   S = phi / sqrt(phi^2 + h^2), dt = h / 2,
 *   per axis D- = (phi_p - phi_{p-e}) / h, D+ = (phi_{p+e} - phi_p) / h,
 *   S > 0: a^2 = max(max(D-,0)^2, min(D+,0)^2); S < 0: max(min(D-,0)^2, max(D+,0)^2),
 *   phi' = phi - dt S (sqrt(sum a^2) - 1).
 * Neighbours come through the neighbour table (Sec. 5.2); far-field rows are
 * read, never written.  `scratch_dev` is a second [P^][64] buffer of the same
 * dtype; the result is left in `phi_dev` for any n_iter >= 0.
 */
sgrid_status sgrid_reinitialize(const sgrid_grid *grid, sgrid_dtype dtype, void *phi_dev,
                                void *scratch_dev, int32_t n_iter, void *stream);

/*
 * Central-difference gradient (Sec. 7.3, Listing 5, with the plain average of
 * the two one-sided differences): g = (phi_{p+e} - phi_{p-e}) / (2h) at every
 * point of every activated package; rows 0 and 1 of every component are set
 * to 0.  `grad_dev` is [3][P^][64].
 */
sgrid_status sgrid_compute_gradient(const sgrid_grid *grid, sgrid_dtype dtype,
                                    const void *phi_dev, void *grad_dev, void *stream);

/*
 * The same gradient written with phi into one array of (phi, gx, gy, gz)
 * quadruples, [P^][64][4] in `dtype`, a layout for the packed probe: one
 * 16-byte gather per corner in FP32.  Inside a package the points are in
 * 2x2x2 blocks: point (i, j, k) is at 8 ((i>>1) + 2 (j>>1) + 4 (k>>1)) +
 * ((i&1) + 2 (j&1) + 4 (k&1)), so a cell inside one block is one 128-byte
 * line.  Far-field rows hold (+-B, 0, 0, 0).
 */
sgrid_status sgrid_compute_gradient_packed(const sgrid_grid *grid, sgrid_dtype dtype,
                                           const void *phi_dev, void *packed_dev, void *stream);

/*
 * Grid-to-particle probe (Sec. 8): trilinear interpolation of phi and of the
 * gradient at n particles, then normal = g / |g| (0 where g = 0).  Per axis
 * u = x / h, s = u - 1/2, i0 = clamp(floor(s), 0, N - 2), t = clamp(s - i0, 0, 1).
 * The particle's package is the coarse cell clamp(floor(u / 4), 0, M - 1) that
 * contains it; the eight corners are reached from it through the neighbour
 * table (index shifts in [-1, 4]), so a particle in a far-field cell reads that
 * far-field package everywhere.  `pos_dev` [n][3], `phi_out_dev` [n],
 * `normal_out_dev` [n][3], all in `dtype`.  n may be 0.  The grid must have
 * M <= 4096 (SGRID_E_INVALID otherwise; cell_pkg alone takes 256 GiB at
 * 4096), as for sgrid_probe_integral_field.
 */
sgrid_status sgrid_probe_particles(const sgrid_grid *grid, sgrid_dtype dtype, const void *phi_dev,
                                   const void *grad_dev, const void *pos_dev, int64_t n,
                                   void *phi_out_dev, void *normal_out_dev, void *stream);

/* sgrid_probe_particles on the packed (phi, g) array of sgrid_compute_gradient_packed. */
sgrid_status sgrid_probe_particles_packed(const sgrid_grid *grid, sgrid_dtype dtype, const void *packed_dev,
                                          const void *pos_dev, int64_t n, void *phi_out_dev,
                                          void *normal_out_dev, void *stream);

/*
 * Particle reordering for the probe (Sec. 8 probing is position-based random
 * access; the reordering is not in the paper).  Stable sort of n FP32
 * particles `pos_dev` [n][3] by the Morton (Z-order) code of their home
 * coarse cell (the probe's cell clamp(floor(x / 4h), 0, M - 1) per axis, bit
 * b of x, y, z at bits 3b, 3b + 1, 3b + 2), the order of the sweep worklist,
 * so that particles of one package are adjacent and neighbouring packages
 * close.  Writes pos_sorted_dev [n][3] with pos_sorted[i] = pos[perm[i]] and
 * perm_dev [n] (uint32): keys non-decreasing, equal keys in input order, so
 * the result is unique.  Probing pos_sorted gives each particle's values in
 * sorted order; perm maps them back.  `workspace_dev` (caller-owned,
 * 256-byte aligned, contents on return unspecified) of at least the bytes
 * sgrid_sort_particles_workspace_size returns (about 16.5 n bytes).
 * n in [0, 2^32 - 1]; pos and pos_sorted distinct.  Asynchronous on `stream`.
 */
sgrid_status sgrid_sort_particles_workspace_size(const sgrid_grid *grid, int64_t n, int64_t *bytes);
sgrid_status sgrid_sort_particles(const sgrid_grid *grid, const float *pos_dev, int64_t n, float *pos_sorted_dev,
                                  uint32_t *perm_dev, void *workspace_dev, int64_t workspace_bytes, void *stream);

/*
 * Near-surface kernel integrals (Sec. 8 names the integral with an SPH
 * smoothing kernel over the sparse grid).  At every data point p of every
 * core package, with query point q = x_p + (h/2)(1,1,1) and the 32 data points
 * j within 2h of q:
 *   out[0] = h^3 sum_j W(|q - x_j|) V_j,
 *   out[1+a] = h^4 sum_j W'(|q - x_j|) (q - x_j)_a / |q - x_j| V_j,
 * where W is the Wendland C2 kernel with smoothing length h, g_j the central
 * difference at j, and V_j the exact fraction of j's cell on the phi > 0 side
 * of the plane phi_j + g_j.(y - x_j).  FP32.  `out_dev` is [4][n_core * 64],
 * core packages in core_list order, local index i + 4j + 16k inside each.
 * With `model` non-NULL the surrogate network is evaluated instead and every
 * point whose gate fails falls back to the plain integral; the number of
 * fallback points is written to *n_fallback_dev when that pointer is non-NULL.
 * A point whose 32 taps all lie more than half a cell from the surface
 * (saturated: every V_j is 0 or 1) skips the network; it and every fallback
 * point get the plain kernel's bits.
 */
sgrid_status sgrid_compute_near_surface_integrals(const sgrid_grid *grid, const float *phi_dev,
                                                  const sgrid_mlp *model, float *out_dev,
                                                  uint32_t *n_fallback_dev, void *stream);

/*
 * The plain integrals of sgrid_compute_near_surface_integrals in factorised
 * form.  The cut fraction V_j depends on the point j alone (its value and its
 * central-difference gradient), so a first pass writes V at every data point
 * of every activated package into `vfrac_dev` ([P + 2][64] FP32, caller-owned
 * workspace, contents on return unspecified), and a second pass sums each
 * core point's 32 taps from it, so that no fraction is evaluated twice (the
 * direct kernel evaluates 7^3 per package for 64 points).  The result has the
 * bits of the direct plain kernel.  `out_dev` as there; phi, vfrac and out
 * must be distinct.  Asynchronous on `stream`.
 */
sgrid_status sgrid_compute_near_surface_integrals_factorised(const sgrid_grid *grid, const float *phi_dev,
                                                             float *vfrac_dev, float *out_dev, void *stream);

/*
 * The integral field for grid-to-particle coupling (Sec. 8: the kernel
 * integral evaluated on the sparse grid is interpolated trilinearly to the
 * particles and drives them as a surface force).  The integrals above, at
 * every data point of every activated package (core and inner), written to
 * `field_dev` [P + 2][64] float4 (K_W, h K_grad x, y, z) in the packed
 * blocked point order of sgrid_compute_gradient_packed.  Rows 0 and 1 are
 * the far-field packages' constants: (0, 0, 0, 0) for the negative side,
 * (c_full, 0, 0, 0) for the positive side, c_full = sum of the 32 kernel
 * weights (K_W of a support wholly on the phi > 0 side).  Inner packages'
 * windows reach into the far field, whose constant values they read like
 * any other neighbour.  FP32; `phi_dev` with its far-field rows filled.
 */
sgrid_status sgrid_compute_integral_field(const sgrid_grid *grid, const float *phi_dev, float *field_dev,
                                          void *stream);

/*
 * The integral field at particle positions: trilinear interpolation of the
 * four components over the eight data points around each particle, with the
 * home package and the index shift of sgrid_probe_particles (a particle
 * whose home cell is far field reads that package's constants).  `pos_dev`
 * [n][3] FP32, `out_dev` [n][4] float (16-byte aligned) receives
 * (K_W, h K_grad) unnormalised.
 */
sgrid_status sgrid_probe_integral_field(const sgrid_grid *grid, const float *field_dev, const float *pos_dev,
                                        int64_t n, float *out_dev, void *stream);

/* ------------------------------------------------------------------------
 * Surrogate network for the near-surface integrals (not in the paper: a
 * learned replacement of the plain integral above).  216 -> 128 -> 128 -> 4
 * MLP with tanh-approximated GELU; input the 6x6x6 window of phi / h at
 * offsets -2..3 around a core data point (x fastest), output
 * (K_W, h K_grad x, y, z).  Parameters are one packed FP32 vector of 44,804
 * values: W1[128][216], b1[128], W2[128][128], b2[128], W3[4][128], b3[4]
 * (row-major, y = W x + b).  Kernels use BF16 MFMA with FP32 accumulation;
 * the first layer splits its input into BF16 hi + lo parts.
 *
 * A model owns device buffers that its calls write (Adam moments, partial
 * gradients, the fallback list of the learned integrals).  Calls with one
 * model are ordered on the device: each records an event on its stream and a
 * call on another stream first waits for the previous call's event, so the
 * model can be used from several streams in turn.  The handle itself is not
 * thread-safe: calls with one model must not run concurrently on the host.
 * ------------------------------------------------------------------------ */

/* Creates a model on the current device from host parameters (copied). */
sgrid_status sgrid_mlp_create(const float *params_host, sgrid_mlp **out);
sgrid_status sgrid_mlp_destroy(sgrid_mlp *model);

/* Copies the FP32 parameters, Adam moments and step count to host buffers
 * (each nullable); synchronises the device. */
sgrid_status sgrid_mlp_get_params(const sgrid_mlp *model, float *params_host, float *adam_m_host,
                                  float *adam_v_host, int64_t *step);

/* Restores Adam moments and the step count (for resuming training). */
sgrid_status sgrid_mlp_set_state(sgrid_mlp *model, const float *adam_m_host, const float *adam_v_host,
                                 int64_t step);

/* Gate of the learned integrals: a non-saturated point takes the network's
 * output when the mean squared residual of its window after the best affine
 * fit (units of h^2) is <= tau and the predicted K_W lies in [kw_lo, kw_hi];
 * otherwise it falls back to the plain integral.  Default: tau = FLT_MAX,
 * [-0.05, 1.05]. */
sgrid_status sgrid_mlp_set_gate(sgrid_mlp *model, float tau, float kw_lo, float kw_hi);

/* y_dev [B][4] = network(x_dev [B][216]).  16-byte aligned device arrays. */
sgrid_status sgrid_mlp_forward(const sgrid_mlp *model, const float *x_dev, int64_t B, float *y_dev,
                               void *stream);

/* grad_dev [44804] = d(sum_b dy[b] . y[b]) / d(params) for x_dev [B][216],
 * dy_dev [B][4]; the sum over the batch is reduced in a fixed order, so
 * repeated calls give identical bits. */
sgrid_status sgrid_mlp_backward(sgrid_mlp *model, const float *x_dev, const float *dy_dev, int64_t B,
                                float *grad_dev, void *stream);

/* One Adam step (beta1 and beta2 the FP32 numbers nearest 0.9 and 0.999, eps
 * 1e-8, bias-corrected with the same betas) on the
 * loss sum_b sum_o w_o (y_bo - t_bo)^2 / B with w = loss_weights_host[4];
 * the loss before the step goes to *loss_dev (nullable, the sum over the
 * batch before dividing by B). */
sgrid_status sgrid_mlp_train_step(sgrid_mlp *model, const float *x_dev, const float *t_dev, int64_t B,
                                  const float *loss_weights_host, float lr, float *loss_dev, void *stream);

/* One Adam step (as in sgrid_mlp_train_step) on the model's parameters from
 * a caller's gradient grad_dev [44804] (device, FP32), e.g. one reduced over
 * several devices in data-parallel training.  Increments the step count. */
sgrid_status sgrid_mlp_apply_gradient(sgrid_mlp *model, const float *grad_dev, float lr, void *stream);

/* Network inputs of every core point in the integrals' output order:
 * x_dev [n_core * 64][216] (nullable) = window of phi / h; unsat_dev
 * [n_core * 64] (nullable) = 1 when some tap's cut fraction is strictly
 * between 0 and 1, else 0. */
sgrid_status sgrid_gather_windows(const sgrid_grid *grid, const float *phi_dev, float *x_dev,
                                  uint8_t *unsat_dev, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the learned
 * integrals of sgrid_compute_near_surface_integrals with a model, the same
 * kernels and results (outputs and fallback count), calling no hipMalloc or
 * hipFree.  Where that entry keeps its fallback list in a buffer the model
 * allocates, this one uses a fixed array of the library in every GPU's
 * memory: 8 MiB per device, held until the process ends, sized for one
 * chunk of 32,768 core packages; grids with more core packages are processed
 * in chunks, up to 2^26 core packages (32-bit point indices), beyond which the
 * call fails with SGRID_E_INVALID.  `model` must be non-NULL (the plain
 * integrals allocate nothing anyway); grid and model must live on the current
 * device.  *n_fallback_dev (nullable, device) receives the number of fallback
 * points.  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (on different streams, or from several host threads) race and
 * must be serialised by the caller.  The array's contents between calls are
 * unspecified; a call clears its counters itself.
 */
sgrid_status sgrid_compute_near_surface_integrals_noalloc(const sgrid_grid *grid, const float *phi_dev,
                                                          const sgrid_mlp *model, float *out_dev,
                                                          uint32_t *n_fallback_dev, void *stream);

/* ------------------------------------------------------------------------
 * Batched reinitialisation of many grids (shapes of uneven size) in one
 * persistent launch per iteration over a global package worklist, with the
 * iteration loop replayable as a HIP graph (not in the paper).
 *
 * The fields of the batch are the grids' [P_s + 2][64] FP32 arrays
 * concatenated in the order given: grid s starts at package row base_s
 * (sgrid_batch_info), its far-field rows first.  Each grid's result is
 * bit-identical to sgrid_reinitialize on that grid alone.
 * ------------------------------------------------------------------------ */

/* Builds the rebased face tables and the worklist of `n` grids (the grids
 * must stay alive while the batch is used).  Synchronises `stream`. */
sgrid_status sgrid_batch_create(const sgrid_grid *const *grids, int32_t n, void *stream, sgrid_batch **out);
sgrid_status sgrid_batch_destroy(sgrid_batch *batch);

/* Total package rows of the concatenated fields, worklist length, and the
 * first row of every grid (bases_host [n], nullable). */
sgrid_status sgrid_batch_info(const sgrid_batch *batch, int64_t *n_total, int64_t *n_work,
                              int64_t *bases_host);

/* Kernel choice: variant 0 = DPP lane exchange, 1 = LDS tile; workgroups per
 * compute unit of the persistent launch (1..16), or 0 for one wavefront per
 * four worklist entries (no persistence). */
sgrid_status sgrid_batch_set_config(sgrid_batch *batch, int32_t variant, int32_t blocks_per_cu);

/* Times every (variant, workgroups per CU in {1, 2, 4, 8, 16, 0}) candidate
 * with `reps` sweeps that read phi_dev and write scratch_dev (phi is not
 * modified), keeps the fastest as the batch's configuration and returns it;
 * us_table [2][6] (nullable) receives the microseconds per sweep in that
 * order. */
sgrid_status sgrid_batch_autotune(sgrid_batch *batch, const float *phi_dev, float *scratch_dev, int32_t reps,
                                  void *stream, int32_t *variant_out, int32_t *blocks_per_cu_out,
                                  float *us_table);

/* n_iter sweeps of the upwind reinitialisation over every grid of the batch;
 * with use_graph the iteration loop is captured once per (buffers, n_iter,
 * configuration) and replayed as a HIP graph.  The result is left in phi. */
sgrid_status sgrid_batch_reinitialize(sgrid_batch *batch, float *phi_dev, float *scratch_dev, int32_t n_iter,
                                      int32_t use_graph, void *stream);

/*
 * The two operations of the paper's timing test (Sec. 9, Tab. 1), over every
 * data point of every activated package:
 *   sgrid_sequential_update: phi += delta (the "small change to every active
 *     value"); far-field rows 0 and 1 untouched.
 *   sgrid_compute_laplacian: out = (sum of the six face neighbours - 6 phi) /
 *     h^2, the seven-point Laplacian, neighbours through the neighbour table
 *     (Sec. 5.2); out-of-band neighbours are their far-field constants; rows 0
 *     and 1 of out get 0.  phi and out are distinct [P^][64] arrays.
 * Asynchronous on `stream`; SGRID_E_INVALID for NULL or misaligned pointers.
 */
sgrid_status sgrid_sequential_update(const sgrid_grid *grid, sgrid_dtype dtype, void *phi_dev, double delta,
                                     void *stream);
sgrid_status sgrid_compute_laplacian(const sgrid_grid *grid, sgrid_dtype dtype, const void *phi_dev,
                                     void *out_dev, void *stream);

/*
 * Tuning knob for sgrid_reinitialize: sweep variant 0 exchanges the interior
 * neighbours between lanes (DPP row shifts), variant 1 stages each package
 * and its face halo in an LDS tile, variant 2 is variant 3 as a persistent
 * kernel whose wavefronts walk the Morton worklist in grid-stride rounds
 * with the next face row prefetched, variant 3 is variant 0 over the
 * packages in Morton order of their cells (spatial neighbours swept by the
 * same workgroup), variant 4
 * sweeps groups of 64 consecutive Morton-ordered packages per 1024-lane
 * workgroup and reads halo rows of in-group neighbours from LDS, variant 5
 * is variant 0 with the y / z neighbour rows exchanged through LDS instead of
 * DPP (no workgroup barrier), variant 6 is variant 0 as a persistent
 * grid-stride walk in package-id order with the next set's face row and own
 * rows loaded ahead, variant 7 holds the field in Morton (worklist) order
 * between the first and the last sweep of a call (the first sweep gathers it
 * from package-id order, the last scatters it back), so each sweep streams
 * contiguous rows.  `groups` (1, 2, 3, 4 or 8) is, for variants 0, 1, 3 and
 * 5, the number of four-package sets one wavefront processes, for variants 2
 * and 6 the number of workgroups per compute unit, and is ignored by variants
 * 4 and 7.  With variant 2, 3, 4 or 7 the gradient and Laplacian passes also
 * visit the packages in Morton order.  Process-wide; default (0, 1).  Safe to
 * call from any thread: each sweep, gradient or Laplacian call reads the
 * setting once, so a change reaches calls that start after it.  Results are
 * identical for every setting.
 */
sgrid_status sgrid_set_sweep_config(int32_t variant, int32_t groups);

/*
 * Autotuner of sgrid_reinitialize on the caller's grid: times the candidates
 * (variant, groups) = (0, 1), (0, 2), (2, 4), (3, 1), (3, 2), (5, 1), (7, 1)
 * with `reps` sweeps each (1..1000) that read phi and write scratch (phi is
 * not modified; scratch rows 2.. are overwritten; variant 7 is timed on its
 * steady-state sweep, worklist order to worklist order), makes the fastest
 * the process-wide configuration (as sgrid_set_sweep_config) and returns it.
 * us_table [7] (nullable) receives the microseconds per sweep in that order.
 * Synchronises the stream.  Results are identical for every candidate, so
 * tuning changes only speed.
 */
sgrid_status sgrid_autotune_sweep(const sgrid_grid *grid, sgrid_dtype dtype, const void *phi_dev,
                                  void *scratch_dev, int32_t reps, void *stream, int32_t *variant_out,
                                  int32_t *groups_out, float *us_table);

#ifdef __cplusplus
}
#endif

#endif /* SGRID_H */
