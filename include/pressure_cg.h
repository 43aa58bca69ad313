/*
 * pressure_cg.h -- C ABI of the MI355X matrix-free P1 pressure solver.
 *
 * The library solves, on one AMD Instinct MI355X (gfx950), the linear system
 * of the projection stage of the semi-implicit hybrid FV/FE scheme for all
 * Mach number flows (Busto, Rio-Martin, Vazquez-Cendon, Dumbser, arXiv
 * 2301.08357, Sec. 3.4, the weak problem for the pressure correction):
 *
 *     alpha * int dP z  +  beta * int c grad(dP) . grad(z)  =  rhs(z)
 *
 * for the P1 (piecewise linear, continuous) pressure correction dP on the
 * vertices of a triangle (2D) or tetrahedron (3D) mesh, for every P1 test
 * function z.  In the paper alpha = 1/(gamma-1), beta = dt^2 and c = H, the
 * enthalpy, piecewise constant per primal element (Sec. 3.3).  The mass
 * matrix is the consistent one (no lumping, Sec. 3.4).  The sign in front
 * of the stiffness integral is '+': it follows from Green's formula applied
 * to the strong pressure equation (Sec. 3) and it is the sign for which the
 * system is symmetric positive definite, as the paper states; the printed
 * weak form shows '-'.
 *
 * Dirichlet pressure nodes (Sec. 3.6: the exact value is imposed on the
 * boundary vertex) are eliminated symmetrically.  With P_I, P_B the 0/1
 * diagonal projectors on free and Dirichlet nodes the operator is
 *
 *     A_D = P_I (alpha M + beta K_c) P_I + P_B,
 *
 * symmetric positive definite when alpha >= 0, beta > 0, every c_e > 0 and
 * (alpha > 0 or at least one Dirichlet node).  An inhomogeneous value g is
 * imposed by passing rhs_B = g and rhs_I = f_I - A_IB g; the solver then
 * returns p_B = g exactly.
 *
 * With alpha = 0 and no Dirichlet node (the zero Mach number limit, where
 * the system becomes the pressure Poisson problem of the incompressible
 * scheme, Sec. 1 and 3.4) the operator is singular: its kernel is the
 * constants.  The handle detects this case and solves the weak problem posed
 * in V_0 = {z : int z = 0} (Sec. 3.4): with the lumped weights
 * m_i = int phi_i and |Omega| = sum_i m_i it replaces rhs by the compatible
 * rhs - (sum_i rhs_i / |Omega|) m, runs CG on it (the operator is positive
 * definite on the complement of the constants, and CG stays in it), and
 * returns the solution shifted so that int p_h = sum_i m_i p_i = 0.
 * Stopping test, iters, res_hist and true_relres then refer to the
 * projected rhs.
 *
 * The solve is the classical conjugate gradient method the paper names for
 * this system (abstract; Sec. 3.4), matrix-free: the operator is never
 * assembled.  Stopping test: ||r_k||_2 <= rtol * ||rhs||_2 (Euclidean norm
 * over all nodes); once it holds, the true residual ||rhs - A_D p|| is
 * computed and, if it is above rtol * ||rhs||, the residual is replaced by
 * the true one and the iteration resumes (at most twice).
 *
 * Conventions for every call:
 *  - Node vectors are in the caller's node order; any renumbering is
 *    internal.  Device vectors are FP64 arrays of n_nodes entries in device
 *    memory owned by the caller; they are read/written in stream order on
 *    the given stream (a hipStream_t passed as void*, NULL = default
 *    stream).
 *  - Host arrays passed to pressure_setup / pressure_update_coef /
 *    pressure_layout are copied before the call returns; the caller may
 *    free them afterwards.
 *  - A handle owns all the device memory it allocates until
 *    pressure_destroy.  One handle must not be used from two host threads
 *    at once; distinct handles are independent.
 *  - No exception crosses the ABI; every call returns a status code.
 */
#ifndef PRESSURE_CG_H
#define PRESSURE_CG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PM_OK 0               /* success                                          */
#define PM_NOT_CONVERGED 1    /* max_iter reached; the output holds the last iterate */
#define PM_PENDING 2          /* pressure_batch_step_poll: the step is still running */
#define PM_EINVAL (-1)        /* invalid argument (NULL, dim, index, rtol, c_e, NaN) */
#define PM_EDEGENERATE (-2)   /* an element has zero volume                       */
#define PM_ENOMEM (-3)        /* device or host allocation failed                 */
#define PM_EBREAKDOWN (-4)    /* CG breakdown: p.Ap <= 0 or not finite            */
#define PM_EHIP (-5)          /* a HIP runtime call failed                         */
#define PM_ETOOLARGE (-6)     /* beyond the static scratch of pressure_solve_noalloc */
#define PM_ETIMEOUT (-7)      /* a grid barrier of a persistent batched launch timed out */

/* Precision flags for pressure_setup / pressure_footprint. */
#define PM_FP64 1             /* FP64 operator data (always present)               */
#define PM_FP32_INNER 2       /* also keep FP32 operator data for pressure_solve_mixed */
/* Morton tile size of the tiled apply (bits 4..7 of flags).  0 = the
 * default, 128 nodes; a mesh that the tiled kernel cannot take at the
 * default size (a node in more than 63 elements, or a tile reaching more
 * than 1024 own and halo nodes) then runs on the node kernel, while an
 * explicit size returns PM_EINVAL for it.  pressure_tune_tile picks the
 * fastest size for a mesh. */
#define PM_TILE_MASK 0xF0
#define PM_TILE_256 0x10
#define PM_TILE_512 0x20
#define PM_TILE_128 0x30
/* Lumped (diagonal) mass matrix instead of the consistent one: M_L =
 * diag(m_i), m_i = int phi_i = sum over node i's elements of |T|/(d+1)
 * (the row sums of the consistent mass).  The paper solves with the
 * consistent mass (Sec. 3.4) and names mass lumping as what makes the
 * general-EOS pressure system amenable to nested Newton methods (Sec. 3);
 * with it the operator is P_I (alpha M_L + beta K_c) P_I + P_B (lumped first,
 * then the Dirichlet rows eliminated).  Applies to every call of the handle,
 * including the mixed, batched and V_0 solves. */
#define PM_MASS_LUMPED 0x100

/* Apply-kernel variants (pressure_set_variant). */
#define PM_VARIANT_AUTO 0     /* tiled when the mesh has tiles, else node           */
#define PM_VARIANT_NODE 1     /* one lane per node, element factors recomputed per incidence */
#define PM_VARIANT_TILED 2    /* Morton tiles: each element computed once per tile in LDS */

typedef struct pm_handle pm_handle;

/* A primal simplex mesh (the paper's Sec. 3.1: triangles T_k with vertices
 * V_j in 2D, tetrahedra in 3D).  All arrays are host memory.
 *   dim        2 (triangles) or 3 (tetrahedra)
 *   coords     n_nodes * dim doubles, row-major (x, y[, z]) per node
 *   elems      n_elems * (dim+1) vertex indices, 0-based; any orientation
 *              (elements with negative volume are reoriented)
 *   dirichlet  n_nodes bytes, nonzero = Dirichlet pressure node; NULL = none
 *   lattice    optional n_nodes * dim integer coordinates in [0, 2^21) used
 *              as Morton keys; NULL = coordinates quantised to 21 bits per
 *              axis over the bounding box.
 *   period     optional dim doubles: period[ax] > 0 makes the mesh periodic
 *              along axis ax with that length, 0 leaves the axis open; NULL
 *              = not periodic.  Periodic boundary conditions (Sec. 3.6): the
 *              caller provides a periodic mesh whose matching boundary
 *              vertices are already merged, so each pair (or group) of
 *              periodic images is one node, one pressure unknown, and the
 *              elements reference the merged nodes.  Every element then
 *              takes the minimum image of its edge vectors: along a periodic
 *              axis each component of x_k - x_0 is shifted by a multiple of
 *              the period into [-period/2, period/2].  This requires every
 *              element's extent along a periodic axis to stay below half the
 *              period (three or more cells across it).  Translations along
 *              the coordinate axes only. */
typedef struct {
    int32_t dim;
    int32_t reserved;
    int64_t n_nodes;
    int64_t n_elems;
    const double *coords;
    const int32_t *elems;
    const uint8_t *dirichlet;
    const int32_t *lattice;
    const double *period;
} pm_mesh;

/* Build the device-resident operator of one mesh (Sec. 3.4 operator with
 * alpha = mass_coef, beta = dt*dt, c = elem_coef).
 *   elem_coef  host, n_elems doubles, each finite and > 0 (c_e = H_e)
 *   mass_coef  alpha >= 0 (1/(gamma-1) in the paper)
 *   dt         > 0; the stiffness scale is beta = dt*dt
 *   flags      PM_FP64, optionally | PM_FP32_INNER, optionally one PM_TILE_*,
 *              optionally | PM_MASS_LUMPED; other bits give PM_EINVAL
 *   out        receives the handle (NULL on failure)
 * Validation: dim in {2,3}, n_nodes in [1, 2^31-1), n_elems in
 * [1, 2^29), indices in range, finite coordinates, nonzero element volume
 * (after the minimum image on periodic axes), each period finite and >= 0.
 * Errors: PM_EINVAL, PM_EDEGENERATE, PM_ENOMEM, PM_EHIP.  Synchronous. */
int pressure_setup(const pm_mesh *mesh, const double *elem_coef, double mass_coef, double dt,
                   int32_t flags, pm_handle **out);

/* New coefficients on the same mesh (a new Picard iterate H^{n+1,k} or a
 * new time step, Sec. 3.4).  elem_coef may be NULL to keep the current
 * c_e.  Same validation as pressure_setup.  Synchronous. */
int pressure_update_coef(pm_handle *h, const double *elem_coef, double mass_coef, double dt);

/* y = A_D x (both device, n_nodes doubles, caller order).  x and y must not
 * overlap.  Asynchronous on stream. */
int pressure_apply(pm_handle *h, const double *x_dev, double *y_dev, void *stream);

/* Solve A_D p = rhs by CG in FP64.
 *   rhs_dev     device, n_nodes doubles
 *   x0_dev      device initial guess (NULL = zero; its Dirichlet entries are
 *               replaced by rhs_B); the paper starts from the previous
 *               solution (Sec. 3.4)
 *   rtol        > 0, relative to ||rhs||_2
 *   max_iter    >= 0
 *   p_dev       device output, n_nodes doubles (may alias x0_dev)
 *   iters       host out: CG iterations performed
 *   res_hist    host out or NULL: ||r_k|| / ||rhs|| for k = 0..iters
 *               (capacity max_iter + 1)
 *   true_relres host out or NULL: ||rhs - A_D p|| / ||rhs|| at exit
 * Returns PM_OK, PM_NOT_CONVERGED, PM_EBREAKDOWN, PM_EINVAL or PM_EHIP.
 * rhs = 0 gives p = 0 after 0 iterations.  Synchronises the stream before
 * returning (the host outputs are final).
 * Each CG iteration is two launches (the operator apply fused with the
 * direction update, then the vector update), run in chunks between reads
 * of the solver state.  A mesh whose coordinates, vectors and element
 * contributions fit one workgroup's LDS (about (dim + 4) * n_nodes +
 * (dim + 1) * n_elems doubles; pressure_info entry 8 says whether a handle
 * qualifies) instead runs the whole solve (the start, every iteration and
 * the true residual) in a single launch of one workgroup, with the same
 * arithmetic and the same reduction order, so p, iters, res_hist and
 * true_relres are bit for bit those of the multi-launch form.  Timing
 * (pressure_timing_enable) keeps the multi-launch form.  Such a launch also
 * writes the history and the final state to pinned host memory held by the
 * handle (max_iter + 1 doubles, grown on demand, freed by pressure_destroy;
 * none is allocated inside pressure_solve_noalloc), so the call ends with one
 * stream synchronisation. */
int pressure_solve(pm_handle *h, const double *rhs_dev, const double *x0_dev, double rtol,
                   int32_t max_iter, double *p_dev, int32_t *iters, double *res_hist,
                   double *true_relres, void *stream);

/* Same system by FP64 defect correction around an FP32 inner CG: the outer
 * residual, the dot-product accumulation and the solution update are FP64;
 * the inner operator data, vectors and apply are FP32.  Requires a handle
 * built with PM_FP32_INNER.  Each correction step computes the FP64
 * residual r = rhs - A x, runs the FP32 CG on A d = r until its residual has
 * dropped by inner_rtol (in (0,1)), and adds d to x in FP64.  In the default
 * mode (PM_MIXED_KEEP_DIRECTION, see pressure_set_mixed_mode) the inner CG
 * is not restarted at a correction: its residual is replaced by the
 * rounded FP64 residual and its search direction is kept (the "reliable
 * update" form of mixed-precision CG, Clark et al., Comput. Phys. Commun.
 * 181 (2010) 1517), so the inner iteration count stays close to a plain
 * CG's; PM_MIXED_RESTART starts a fresh inner CG at every correction.
 * iters receives the total number of inner iterations and outer (may be
 * NULL) the number of corrections; res_hist (may be NULL, capacity
 * max_iter+1) receives the FP64 relative residual at each correction. */
int pressure_solve_mixed(pm_handle *h, const double *rhs_dev, const double *x0_dev, double rtol,
                         double inner_rtol, int32_t max_iter, double *p_dev, int32_t *iters,
                         int32_t *outer, double *res_hist, double *true_relres, void *stream);

/* pressure_solve without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and status codes as
 * pressure_solve, bit for bit the same results; the CG vectors, block
 * partials, solver state and residual history live in one static device
 * array of the library (about 26 MB: 6 vectors of PM_NOALLOC_MAX_NODES
 * doubles, the partials and PM_NOALLOC_MAX_ITER + 1 history entries), which
 * each GPU the library runs on holds until the process ends; its address
 * is looked up at pressure_setup.  The call allocates no device memory, no
 * events (handle timing is not recorded) and no host memory of its own.
 *   n_nodes > PM_NOALLOC_MAX_NODES or max_iter > PM_NOALLOC_MAX_ITER:
 *   PM_ETOOLARGE, nothing launched.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (from two host threads, or on two streams) race and must not be made.
 * The array keeps the last call's contents; the call clears what must start
 * at zero (the two direction buffers) itself. */
#define PM_NOALLOC_MAX_NODES 524288
#define PM_NOALLOC_MAX_ITER 65535
int pressure_solve_noalloc(pm_handle *h, const double *rhs_dev, const double *x0_dev, double rtol,
                           int32_t max_iter, double *p_dev, int32_t *iters, double *res_hist,
                           double *true_relres, void *stream);

/* Inner-solve mode of pressure_solve_mixed for this handle. */
#define PM_MIXED_KEEP_DIRECTION 0
#define PM_MIXED_RESTART 1
int pressure_set_mixed_mode(pm_handle *h, int32_t mode);

/* Device bytes pressure_setup would allocate for this mesh (operator
 * data, CG vectors and scratch), for admission control.  Host only. */
int pressure_footprint(const pm_mesh *mesh, int32_t flags, uint64_t *bytes);

/* Release every device allocation of the handle.  NULL is ignored. */
void pressure_destroy(pm_handle *h);

/* Static text for a status code. */
const char *pressure_strerror(int status);

/* Host-only: the integer layout pressure_setup builds (no GPU needed).
 *   node_new2old  n_nodes    : old id of internal node i (Morton order:
 *                 nodes sorted by (interleaved 21-bit key with x in the
 *                 lowest bit, old id))
 *   elem_new2old  n_elems    : old id of internal element e (sorted by
 *                 (smallest internal vertex id, old id))
 *   elems_new     n_elems*(dim+1) : oriented connectivity, internal ids
 *   n2e_off       n_nodes+1  : node-to-element offsets
 *   n2e_ent       n_elems*(dim+1) : entries 4*e + a (element e, local
 *                 vertex a), ascending e per node
 * Any output pointer may be NULL.  Errors as pressure_setup. */
int pressure_layout(const pm_mesh *mesh, int32_t *node_new2old, int32_t *elem_new2old,
                    int32_t *elems_new, int32_t *n2e_off, int32_t *n2e_ent);

/* Select the apply kernel used by pressure_apply / pressure_solve.  Both
 * kernels give the same bits.  PM_VARIANT_TILED returns PM_EINVAL for a
 * handle without tiles (see PM_TILE_MASK); PM_EINVAL also for an unknown
 * variant. */
int pressure_set_variant(pm_handle *h, int32_t variant);

/* Kernel timing with HIP events on the solve stream.  enable != 0 starts
 * recording the duration of a sample of the operator-apply launches inside
 * pressure_solve, iterations 1, 33, 65, ... of each solve that ran a full
 * iteration (and resets the totals); pressure_timing_read returns the
 * number of recorded launches and their summed duration in milliseconds.
 * Each sampled launch gets two event records. */
int pressure_timing_enable(pm_handle *h, int32_t enable);
int pressure_timing_read(pm_handle *h, int64_t *launches, double *total_ms);

/* Sizes and bytes of the operator data of a handle:
 *   info[0] n_nodes, [1] n_elems, [2] free nodes, [3] dim,
 *   [4] algorithmic bytes of one FP64 apply (x read, y written, coordinates,
 *       connectivity, element coefficient: each once),
 *   [5] device bytes held by the handle, [6] number of tiles, [7] element
 *       instances over all tiles, [8] 1 if pressure_solve runs its CG
 *       iterations in one launch (a mesh small enough for one workgroup's
 *       LDS, on the tiled kernel with timing off; see pressure_solve), else 0.
 * Entries past n_info are not written. */
int pressure_info(pm_handle *h, int64_t *info, int32_t n_info);

/* ------------------------------------------------------------------------
 * Batched solves: many independent meshes (2D and 3D mixed) solved together.
 * Each CG iteration of all meshes is two kernel launches (the operator apply
 * of every (mesh, tile slot), then the vector update of every (mesh, node
 * slot)); chunks of iterations are captured once in a HIP graph and
 * replayed, and meshes that have converged skip their slots.  Optionally
 * (pressure_batch_set_persistent) each chunk is one cooperative launch of a
 * persistent kernel whose phases meet at grid barriers.  This is the
 * same classical CG as pressure_solve (paper Sec. 3.4), run for many systems
 * at once.
 */
typedef struct pm_batch pm_batch;

/* Group n handles (all from pressure_setup on the current device, each with
 * the default or 128-node tiles) into a batch.
 *   params   NULL for the defaults, else int32_t[3]:
 *            params[0] Morton tiles per apply slot (>= 1, default 4),
 *            params[1] nodes per lane of an update slot (>= 1, default 8),
 *            params[2] launch index of the batch's first step (>= 1,
 *                      default 1); a batch rebuilt over a changed set of
 *                      handles continues the solves in flight when it starts
 *                      at the old batch's pressure_batch_next_index.
 * Joining a batch sets each handle's launch grids to the batch's; single
 * pressure_solve calls on the handle then use the same grids, so a mesh's
 * batched result equals its single-mesh result bit for bit.  The handles
 * must outlive the batch and must not be used while a batched solve runs.
 * Errors: PM_EINVAL (n < 1, NULL handle, unsupported tile size or mesh
 * shape, handles on different devices), PM_ENOMEM, PM_EHIP. */
int pressure_batch_create(pm_handle *const *handles, int32_t n, const int32_t *params, pm_batch **out);

/* A batch of mixed-precision solves (pressure_solve_mixed for every mesh):
 * the FP32 inner CG iterations of all meshes run in the batched launches;
 * when a mesh's inner solve has dropped its residual by inner_rtol (in
 * (0,1)) the next step computes that mesh's FP64 correction and residual
 * and, unless it has converged, continues its inner solve (in the handle's
 * pressure_set_mixed_mode).  Every handle must be built with PM_FP32_INNER;
 * params and errors as pressure_batch_create.  pressure_batch_solve, _begin,
 * _step and _finish then run mixed solves (iters counts inner iterations;
 * done[m] is set when mesh m's whole solve has finished), and each result
 * equals pressure_solve_mixed on the same handle bit for bit. */
int pressure_batch_create_mixed(pm_handle *const *handles, int32_t n, const int32_t *params, double inner_rtol,
                                pm_batch **out);

/* Solve all meshes of the batch.  rhs_dev, x0_dev and p_dev are host arrays
 * of n device pointers (x0_dev may be NULL, or hold NULL entries, for a zero
 * initial guess); iters, true_relres and status are host arrays of n
 * (status[m] is the PM_* code of mesh m).  rtol and max_iter apply to every
 * mesh.  Returns PM_OK when every mesh converged, PM_NOT_CONVERGED if some
 * did not, or the first error.  Synchronises the stream before returning. */
int pressure_batch_solve(pm_batch *b, const double *const *rhs_dev, const double *const *x0_dev, double rtol,
                         int32_t max_iter, double *const *p_dev, int32_t *iters, double *true_relres,
                         int32_t *status, void *stream);

/* Continuous batching: solves start and finish independently while the
 * batch steps.  pressure_batch_begin starts the solve of mesh m (0-based)
 * at the next step (rhs_dev, x0_dev as in pressure_solve; the solve must not
 * be in flight); pressure_batch_step advances every solve in flight by one
 * chunk of iterations and writes done[m] (host, n entries: nonzero = mesh m
 * idle or finished); pressure_batch_finish computes mesh m's true residual,
 * writes its solution to p_dev and returns its status (mesh m must be
 * finished; rhs_dev and rtol as passed to begin).  A solve's arithmetic does
 * not depend on the step at which it starts or on the other solves in
 * flight, so each result equals the same solve run alone, bit for bit.
 * The batch runs on a stream of its own: _begin and _step start after the
 * work already queued on `stream`, _finish's output is ready in `stream`
 * order, and _step returns with the batch's work complete.  A step launches
 * blocks only for the meshes in flight (begun, and not yet stopped or
 * finished): with every mesh in flight it replays the captured graph,
 * otherwise it launches the same iterations directly over the slots of
 * those meshes. */
int pressure_batch_begin(pm_batch *b, int32_t m, const double *rhs_dev, const double *x0_dev, double rtol,
                         int32_t max_iter, void *stream);
int pressure_batch_step(pm_batch *b, int32_t *done, void *stream);

/* pressure_batch_step in two halves, so that one host thread can keep the
 * steps of several batches (each on its own stream) running on the device
 * at once: _launch queues the step after the work already queued on
 * `stream` and returns without waiting; _wait waits for it and writes
 * done[] as pressure_batch_step does.  Between the two no other call may be
 * made on the batch but _poll (PM_EINVAL: a second _launch, _begin, _finish,
 * _step, _solve; _wait without a _launch).  Errors as pressure_batch_step. */
int pressure_batch_step_launch(pm_batch *b, void *stream);
int pressure_batch_step_wait(pm_batch *b, int32_t *done);

/* _wait without blocking: PM_PENDING (nothing written) while the step
 * queued by _launch still runs, else what _wait returns. */
int pressure_batch_step_poll(pm_batch *b, int32_t *done);
int pressure_batch_finish(pm_batch *b, int32_t m, const double *rhs_dev, double rtol, double *p_dev, int32_t *iters,
                          double *true_relres, void *stream);

/* Launch index of the batch's next step (see pressure_batch_create). */
int pressure_batch_next_index(pm_batch *b, int32_t *k);

/* Number of CG iterations captured per graph replay (default 16, even, 2..256);
 * 0 disables graph capture (iterations are launched one by one). */
int pressure_batch_set_graph(pm_batch *b, int32_t iterations_per_replay);

/* Launch form of the batch's steps.  persistent = 0 (default): two
 * launches per CG iteration, chunks replayed from the captured graph.
 * persistent = 1: each step is ONE cooperative launch of a persistent
 * kernel, as many blocks as can be resident on the device, that runs the
 * step's iterations (pressure_batch_set_graph's count, 8 if 0) over the
 * slots of the meshes in flight; inside it the phases (apply of every
 * slot, update of every slot) are separated by grid barriers instead of
 * kernel boundaries.  With every mesh in flight the launch is replayed from
 * a HIP graph captured at the first such step (launched directly if the
 * runtime does not capture it).  The arithmetic is the same, so results equal the
 * two-launch form bit for bit.  Each barrier wait is bounded (2 s); if one
 * times out the step returns PM_ETIMEOUT and the solves in flight are lost
 * (begin them again).  Errors: PM_EINVAL. */
int pressure_batch_set_persistent(pm_batch *b, int32_t persistent);

/* Time limit of each grid-barrier wait of the persistent form, in
 * microseconds (0: the default, 2 s; at most 600 s).  A wait that exceeds
 * it ends the step with PM_ETIMEOUT.  Errors: PM_EINVAL. */
int pressure_batch_set_barrier_limit(pm_batch *b, int64_t microseconds);

/* Release the batch (not its handles).  NULL is ignored. */
void pressure_batch_destroy(pm_batch *b);

/* ------------------------------------------------------------------------
 * Autotuners.  Each times short runs of the real CG iterations on the
 * caller's own operators (right-hand side of ones; a tolerance no run can
 * meet, so every candidate runs the same iterations) and returns the
 * fastest candidate with its time per iteration.  cache_path (NULL = no
 * cache) names a text file of earlier choices, one line each, keyed by a
 * 64-bit hash of the tuner, the device (architecture name and compute-unit
 * count), the library build and the mesh sizes: a key that is present is
 * returned at once (with the time recorded for it); a new choice is
 * appended.  Errors: PM_EINVAL (arguments), PM_ENOMEM, PM_EHIP, and those of
 * the calls the tuner makes.
 */

/* Launch shape of a batch over n handles: Morton tiles per apply slot in
 * {1, 2, 4, 8} and nodes per lane of an update slot in {2, 4, 8, 16}, each
 * candidate timed over `iters` iterations (rounded up to whole 16-iteration
 * graph replays) of a batched solve of all n meshes.  params_out[0..1] take
 * the choice (params[0..1] of pressure_batch_create).  The runs overwrite
 * the handles' solver state and set their launch grids as
 * pressure_batch_create does; create the batch afterwards. */
int pressure_batch_tune(pm_handle *const *handles, int32_t n, int32_t iters, const char *cache_path,
                        int32_t *params_out, double *ms_per_iter);

/* Morton tile size of one mesh: the mesh is set up with each of
 * PM_TILE_128, PM_TILE_256 and PM_TILE_512 (sizes whose tables do not fit
 * the kernel are skipped) and `iters` CG iterations of each are timed.
 * *flags_out receives `flags` with the fastest PM_TILE_* bits.  Arguments as
 * pressure_setup; the key hashes dim, n_nodes, n_elems and the precision
 * flags. */
int pressure_tune_tile(const pm_mesh *mesh, const double *elem_coef, double mass_coef, double dt, int32_t flags,
                       int32_t iters, const char *cache_path, int32_t *flags_out, double *ms_per_iter);

/* ------------------------------------------------------------------------
 * The projection stage around the solve (Sec. 3.3 pre-projection, Sec. 3.4
 * projection with its Picard loop, and the momentum update of eq.
 * momentum_dt_p).
 *
 * Dual mesh (Sec. 2, face-type dual cells): one dual cell C_f per face
 * (3D) or edge (2D) f of the primal mesh, made of the sub-elements T_kf
 * that join f to the barycenters of the one or two primal elements T_k that
 * share it; |T_kf| = |T_k|/(d+1).  Dual cells are numbered by the sorted
 * tuples of their vertices' internal node indices (the Morton order that
 * pressure_layout reports as node_new2old) in lexicographic order, so that
 * dual-cell arrays are laid out in the order the kernels visit elements;
 * pressure_dual_faces lists each cell's vertices and elements in the
 * caller's numbering.
 * With merged periodic vertices the two images of a seam face are one
 * interior face, as Sec. 3.6 combines matching dual boundary cells.
 */

/* Number of dual cells and of boundary faces (faces of one element).
 * Built on the host at the first call and kept by the handle. */
int pressure_dual_count(pm_handle *h, int64_t *n_faces, int64_t *n_boundary);

/* The dual cells: face_vertices (host, n_faces * dim: ascending caller node
 * ids of face f) and face_elems (host, n_faces * 2: the caller element ids
 * sharing f, ascending, -1 for none).  Either may be NULL. */
int pressure_dual_faces(pm_handle *h, int32_t *face_vertices, int32_t *face_elems);

/* One projection stage (all device arrays in caller numbering, FP64; node
 * vectors n_nodes, element vectors n_elems, dual-cell vectors n_faces, and
 * vector fields n_faces * dim, row-major per cell):
 *   rho_dev    rho^{n+1} on the dual cells (from the transport stage), > 0
 *   we_dev     the intermediate total energy density tilde W_E on the dual cells
 *   wu_dev     the intermediate momentum double-tilde W_u on the dual cells
 *   p_dev      P^n at the primal vertices, > 0
 *   pb_dev     P^{n+1} prescribed at the Dirichlet vertices (read there only),
 *              or NULL for P^{n+1}_B = P^n_B
 *   bflux_dev  H W^{n+1} . eta (outward normal momentum times enthalpy) on
 *              the boundary faces (read there only), or NULL for 0 (walls)
 *   dp0_dev    initial guess of the first pressure correction (the paper
 *              starts from the previous solution), or NULL for 0
 *   gamma > 1, dt > 0, n_picard >= 1 (N_Pic; the paper suggests 2),
 *   rtol, max_iter as pressure_solve, for every Picard iteration.
 * Steps:
 *  1. Pre-projection (Sec. 3.3): W_k = sum_f W_f |T_kf|/|T_k|, i.e. the mean
 *     over the d+1 faces of T_k, for rho, tilde W_E and double-tilde W_u;
 *     (rho K)_k = |W_u,k|^2 / (2 rho_k) with the first momentum guess
 *     W_u^{n+1,1} = double-tilde W_u; H_f = gamma/(gamma-1) P_f / rho_f on
 *     the dual cells, P_f the mean of the face's vertex pressures, and
 *     H_k = the mean of H_f over the faces of T_k.
 *  2. For k = 1 .. n_picard: the operator takes c_e = H_k, alpha =
 *     1/(gamma-1), beta = dt^2 (the handle's mass matrix, consistent or
 *     lumped); the right-hand side of the weak problem (Sec. 3.4) is, for a
 *     free vertex i,
 *       b_i = sum_{T_k ni i} [ (W_E,k - (rho K)_k) |T_k|/(d+1)
 *                              + dt H_k W_u,k . grad(phi_i)|_k |T_k| ]
 *             - alpha (M P^n)_i - (A g)_i
 *             - dt sum_{boundary faces f ni i} bflux_f |f| / d,
 *     g = P^{n+1}_B - P^n_B on the Dirichlet vertices (zero elsewhere, and
 *     the lift A g uses the operator before elimination); b_i = g_i on a
 *     Dirichlet vertex.  CG solves for dP (warm start: dp0, then the
 *     previous Picard iterate); P^{n+1,k+1} = P^n + dP; the per-element
 *     momentum W_u,k - dt grad(dP)|_k gives (rho K)_k, and P^{n+1,k+1}
 *     gives H_f and H_k as in step 1.
 *  3. Momentum update on the dual cells: W_u,f^{n+1} = double-tilde W_u,f
 *     - dt grad(dP)_f, grad(dP)_f = sum_k |T_kf| grad(dP)|_k / |C_f| over
 *     the elements of f.
 * Outputs: p_out (n_nodes) P^{n+1}; wu_out (n_faces * dim) W_u^{n+1};
 * h_out (n_elems, may be NULL) H^{n+1} per element; iters (host, n_picard
 * entries, may be NULL) the CG iterations of each Picard iteration.
 * The handle's operator is left with the coefficients of H^{n+1}.
 * Returns PM_OK, or the first non-OK status of a CG solve (PM_NOT_CONVERGED,
 * PM_EBREAKDOWN: a non-positive enthalpy makes the system indefinite),
 * PM_EINVAL or PM_EHIP.  The first call on a handle (of this function,
 * pressure_transport, pressure_post_projection or the dual-cell queries)
 * builds the dual cells on the host and allocates their device data: about
 * 14 doubles and 21 bytes of indices per element, 16 bytes per dual cell
 * and 5 doubles per node, kept until pressure_destroy.  Synchronises the
 * stream before returning. */
int pressure_projection(pm_handle *h, const double *rho_dev, const double *we_dev, const double *wu_dev,
                        const double *p_dev, const double *pb_dev, const double *bflux_dev,
                        const double *dp0_dev, double gamma, double dt, int32_t n_picard, double rtol,
                        int32_t max_iter, double *p_out, double *wu_out, double *h_out, int32_t *iters,
                        void *stream);

/* Post-projection (Sec. 3.5, eq. WEupdatek and the weighted average back to
 * the dual cells): the total energy per primal element
 *   W_E,k = W_E,k~ - dt/|T_k| sum_{faces l of T_k} H_l W_u,l^{n+1} . A_kl,
 * W_E,k~ the mean of tilde W_E over the faces of T_k (as in the
 * pre-projection), A_kl the outward area vector of face l, W_u,l^{n+1} the
 * momentum of the dual cell of l and H_l = gamma/(gamma-1) P_l / rho_l with
 * P_l the mean of the face's vertex pressures P^{n+1}; then
 * W_E,f^{n+1} = sum_k |T_kf| W_E,k / |C_f|.  Interior faces cancel between
 * their two elements, so the total energy changes only through the primal
 * boundary.  Arrays as in pressure_projection (caller face numbering):
 * rho_dev rho^{n+1}, we_dev tilde W_E, wu_dev W_u^{n+1} (n_faces * dim), p_dev
 * P^{n+1} at the vertices; we_out (n_faces) W_E^{n+1}, not aliasing we_dev.
 * Synchronises the stream before returning. */
int pressure_post_projection(pm_handle *h, const double *rho_dev, const double *we_dev, const double *wu_dev,
                             const double *p_dev, double gamma, double dt, double *we_out, void *stream);

/* One explicit transport step on the dual cells, first order (Sec. 3.2,
 * eq. discrf_mass, discrf_momentum and discrf_energy, with the viscous
 * terms of eq. visc_mom and visc_toten and the heat flux):
 *   rho_f^{n+1}  = rho_f - dt/|C_f| sum_j phi_rho(f, j)
 *   W_u,f        = W_u,f - dt/|C_f| ( sum_j phi_u(f, j) + int_{C_f} grad P^n
 *                                     - sum_j int_{Gamma_fj} tau eta )
 *                  + dt rho_f g
 *   W_E,f        = W_E,f - dt/|C_f| ( sum_j phi_E(f, j)
 *                                     - sum_j int_{Gamma_fj} (tau u) . eta
 *                                     + sum_j int_{Gamma_fj} Q . eta )
 *                  + dt g . W_u,f
 * over the dual faces Gamma_fj inside the one or two primal elements of f
 * (in element k the cells of faces a and b meet on the simplex that joins
 * the barycenter of T_k to the primal vertices the two faces share; its
 * area vector from a to b is eta_ab = |T_k| d/(d+1) (grad phi_a - grad
 * phi_b)).  phi is the modified Rusanov flux of eq. flux:
 *   phi = (Z(W_f, eta) + Z(W_j, eta))/2 - alpha_RS (Wr_j - Wr_f)/2,
 *   Z(W, eta) = (W_u . eta, W_u (U . eta), rho K (U . eta)), U = W_u/rho,
 *   Wr = (rho, W_u, rho K), rho K = |W_u|^2 / (2 rho),
 *   alpha_RS = max(|U_f . eta|, |U_j . eta|) + c_alpha |eta|
 * (the sound speed does not enter: the pressure is implicit).  The viscous
 * stress tau = mu (grad u + grad u^T - 2/3 div u I) is constant on each
 * primal element, from the Galerkin (Crouzeix-Raviart) gradient of the face
 * velocities u_f = W_u,f / rho_f: grad u = -d sum_a u_{f_a} (x) grad phi_a;
 * in the energy term u on Gamma_fj is the mean of the two cells' velocities;
 * The heat flux Q = -lambda grad Theta is constant on each primal element
 * too: Theta_f = P_f / (rho_f R) on the cells, P_f the mean of the face's
 * vertex pressures P^n, and the same Galerkin gradient (eq. heatflux,
 * stateequation; Sec. 3.2, heat flux term).  mu = lambda = 0 gives the
 * Euler step.  The pressure
 * force int_{C_f} grad P^n = sum_k |T_k|/(d+1) grad P^n|_k is exact for the
 * P1 pressure.  Boundary faces of the primal mesh carry no convective flux
 * (impermeable walls).  Arrays are device, caller face numbering as in
 * pressure_dual_faces: rho_dev, we_dev, rho_out, we_out n_faces; wu_dev,
 * wu_out n_faces * dim; p_dev n_nodes (P^n at the vertices).  gravity is
 * host, dim doubles, or NULL for none; c_alpha >= 0; mu >= 0; lambda >= 0
 * (thermal conductivity); r_gas > 0 (R = c_p - c_v, read only when
 * lambda > 0); dt > 0; otherwise PM_EINVAL.  Primal boundary faces carry no
 * viscous or heat flux either (stress-free, adiabatic walls).  Outputs must
 * not alias inputs.  One pass per dual cell: each cell evaluates the fluxes
 * across its 2d (2D: 4, 3D: 6) dual faces itself; the two cells of a dual
 * face obtain exactly opposite fluxes, so the scheme stays conservative.
 * The first call on a handle also allocates 64 bytes per dual cell (the
 * element records of both sides of each cell), kept until pressure_destroy.
 * Synchronises the stream before returning. */
int pressure_transport(pm_handle *h, const double *rho_dev, const double *wu_dev, const double *we_dev,
                       const double *p_dev, const double *gravity, double c_alpha, double mu, double lambda,
                       double r_gas, double dt, double *rho_out, double *wu_out, double *we_out, void *stream);

/* The same transport step at second order in space and time, by the LADER
 * method of Sec. 3.2.1 (Steps 1-4); arguments, outputs and errors as
 * pressure_transport.  Only the convective fluxes change:
 *  1. on every primal element the Galerkin (Crouzeix-Raviart) gradients of
 *     rho and of each momentum component, grad W = -d sum_a W_{f_a} grad
 *     phi_a over the element's d+1 dual cells; for the side of cell i on the
 *     dual face Gamma_ij (inside the centred element T_ij) and each scalar,
 *     the gradient of the upwind element T_ijL (the other primal element of
 *     cell i; T_ij itself for a boundary cell) when |grad W . (N_ij - N_i)|
 *     is not larger than with T_ij's gradient (ENO), else T_ij's; N_ij the
 *     barycentre of Gamma_ij, N_i that of cell i's primal face;
 *  2. the extrapolated state W_i + (N_ij - N_i) . grad W;
 *  3. its evolution by dt/2: the printed Step 3 divides by a length L_ij it
 *     does not define and adds the two sides' fluxes across one eta_ij; it
 *     is read as the Cauchy-Kovalevskaya form of the mass and momentum
 *     equations written with the chosen gradients, d rho/dt = -div W_u,
 *     d W_u/dt = -div(W_u (x) U) - grad P^n|_{T_ij} + rho g (the pressure and
 *     gravity terms are the printed ones);
 *  4. the Rusanov flux of eq. flux_lmnt_lader at the evolved states of the
 *     two sides (rho K from the evolved rho and W_u).
 * The pressure force, gravity sources and the viscous and heat-flux terms
 * are those of pressure_transport (first order in time).  The step runs
 * per primal element: each side of each dual face is evolved once, the two
 * sides of a dual face see opposite fluxes (conservative), and a cell adds
 * the sums of its two elements.  The first call on a handle also allocates
 * (d + d^2) doubles per primal element for the gradients and 24 doubles
 * per primal element for the per-side sums, kept until pressure_destroy;
 * it does not allocate pressure_transport's element records.  Synchronises
 * the stream before returning. */
int pressure_transport_lader(pm_handle *h, const double *rho_dev, const double *wu_dev, const double *we_dev,
                             const double *p_dev, const double *gravity, double c_alpha, double mu, double lambda,
                             double r_gas, double dt, double *rho_out, double *wu_out, double *we_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PRESSURE_CG_H */
