/*
 * femx -- matrix-free finite element actions on AMD Instinct MI355X (gfx950), FP64.
 *
 * C ABI of the library.  The operation is the matrix-free action of a finite element
 * operator on affine simplex meshes, or on curved cells with a P2 geometry
 * (fem_plan_create_curved, paper Sec. 2.4) (paper Sec. 2.2, the action written as a sum of cell
 * integrals through the local-to-global maps and the reference-cell substitution, then
 * replaced by quadrature; Sec. 2.3, the generic action kernel: gather, Jacobian and
 * determinant, evaluation at quadrature points, pointwise form, quadrature contraction,
 * scatter-add).  Forms follow App. A: mass, Laplace, Helmholtz, linear elasticity, and the
 * hyperelastic residual with a compressible neo-Hookean or St Venant-Kirchhoff energy.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Reference simplex {xi >= 0, sum xi <= 1}; P_k Lagrange basis with equispaced nodes
 *   xi = alpha/k, |alpha| <= k.  Local node order (the columns of cell_nodes): first
 *   coordinate fastest, i.e. 2D  for j in 0..k: for i in 0..k-j: (i, j);
 *   3D  for l: for j: for i (i + j + l <= k).  n_loc = C(k + d, d).
 * - Geometry (fem_plan_create) is affine: J = [x_1 - x_0 | ... | x_d - x_0] from the
 *   cell's vertices in cell_verts order; integrals use |det J| (cells with det J < 0 in 3D
 *   are valid).  Curved plans evaluate J at every quadrature point instead.
 * - Quadrature: a rule exact to quad_degree on the reference simplex, from one of two
 *   families: FEM_QUAD_CONICAL, the conical-product (collapsed Gauss-Jacobi) rule with
 *   ceil((quad_degree + 1)/2) points per direction (any degree); FEM_QUAD_SYMMETRIC, fully
 *   symmetric rules (points on orbits of the simplex's symmetry group, one weight per
 *   orbit, positive weights, points inside), each an isolated root of its moment
 *   equations solved by Gauss-Newton iteration at plan creation: triangles of degree <= 2, 4, 6,
 *   8, 10, 12 (1, 3, 6, 12, 16, 25, 33 points), tetrahedra of degree <= 2, 5, 6, 8 (1, 4,
 *   14, 24, 50 points);
 *   a degree without its own rule takes the next tabulated one.  A plan uses the
 *   symmetric rule when one is built for its degree, else the conical rule
 *   (fem_plan_set_quadrature switches).  On affine cells the linear forms' operators do
 *   not depend on the rule once it integrates their polynomial integrands exactly; the
 *   hyperelastic operators, and every form on curved cells, do.
 * - Vectors are node-major interleaved: component c of node n at index n * ncomp + c,
 *   ncomp = 1 for the scalar forms (mass, Laplace, Helmholtz) and d for the vector forms
 *   (elasticity, neo-Hookean, St Venant-Kirchhoff).
 * - Host arrays are read during the call only.  Device arrays (u, v, y, g) are caller-
 *   owned device memory (e.g. PyTorch CUDA tensors); the library never frees them.
 * - Kernels are enqueued on the caller's HIP stream (hipStream_t passed as void*, NULL =
 *   the default stream); fem_action and fem_action_vjp do not synchronise.
 * - Every function returns FEM_OK (0) or a negative status; fem_last_error() returns a
 *   thread-local message for the last failure.  No C++ exception crosses the ABI.
 * - Results are deterministic: the scatter-add never uses atomics; it runs in colour order
 *   or in a fixed per-patch order (fem_plan_set_strategy).
 * - A plan owns a small device scratch area (partial sums of nodes shared by patches):
 *   calls on one plan (or on batches holding it) that overlap in time on different streams
 *   race on it.
 */
#ifndef FEM_ACTION_H
#define FEM_ACTION_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* quadrature families */
#define FEM_QUAD_CONICAL 0
#define FEM_QUAD_SYMMETRIC 1

/* form ids */
#define FEM_MASS 0        /* a(u, v) = int u v                                        */
#define FEM_ELASTICITY 1  /* a(u, v) = int sigma(u) : eps(v),
                             sigma = lambda tr(eps) I + 2 mu eps,  params {lambda, mu} */
#define FEM_NEOHOOKEAN 2  /* r(u; v) = int P(F) : grad v,  F = I + grad u,
                             P = mu (F - F^{-T}) + lambda ln(det F) F^{-T}
                             (energy mu/2 (tr F^T F - d) - mu ln J + lambda/2 ln^2 J),
                             params {lambda, mu}                                     */
#define FEM_LAPLACE 4     /* a(u, v) = int grad u . grad v  (scalar)                  */
#define FEM_HELMHOLTZ 5   /* a(u, v) = int grad u . grad v + u v  (scalar, paper App. A) */
#define FEM_SVK 3         /* St Venant-Kirchhoff residual (paper App. A hyperelastic law):
                             r(u; v) = int F S : grad v,  E = (F^T F - I)/2,
                             S = lambda tr(E) I + 2 mu E  (energy lambda/2 tr^2 E + mu E:E),
                             params {lambda, mu}                                     */

/* status codes */
#define FEM_OK 0
#define FEM_E_ARG (-1)          /* null pointer, negative size, bad layout argument     */
#define FEM_E_UNSUPPORTED (-2)  /* form / dimension / degree / quadrature not built     */
#define FEM_E_INDEX (-3)        /* a map entry is outside [0, n_vert) or [0, n_node)     */
#define FEM_E_INVERTED (-4)     /* det J == 0, or det J < 0 for a 2D cell               */
#define FEM_E_HIP (-5)          /* a HIP runtime call failed (message has the HIP error) */
#define FEM_E_NOMEM (-6)        /* device or host allocation failed                     */

typedef struct fem_plan fem_plan;

/*
 * Build a plan: validates the mesh, tabulates the reference basis at the quadrature
 * points (paper Sec. 2.2, tabulated-values equation), colours the cells (greedy first-
 * fit in ascending cell id; two cells conflict when they share a node of cell_nodes),
 * and uploads colour-sorted copies of the maps and the coordinates to the current HIP
 * device.  Synchronous; allocates device memory owned by the plan.
 *
 *   form         FEM_MASS, FEM_ELASTICITY, FEM_NEOHOOKEAN, FEM_SVK, FEM_LAPLACE or
 *                FEM_HELMHOLTZ
 *   dim          2 (triangles) or 3 (tetrahedra)
 *   degree       polynomial degree k: 1..8 in 2D, 1..6 in 3D (batches and curved cells:
 *                up to 6 in 2D, 4 in 3D)
 *   quad_degree  degree the rule integrates exactly: 0..20
 *   coords       HOST f64 [n_vert][dim]
 *   cell_verts   HOST i32 [n_cell][dim+1]   vertex ids, the affine map's vertex order
 *   cell_nodes   HOST i32 [n_cell][n_loc]   node ids in the local order above
 *   n_node       number of nodes; vectors have n_node * ncomp entries
 *   params       HOST f64 [n_params]: {lambda, mu} for the vector forms, unused for the
 *                scalar forms (mass, Laplace, Helmholtz)
 * Errors: FEM_E_ARG, FEM_E_UNSUPPORTED, FEM_E_INDEX, FEM_E_INVERTED, FEM_E_HIP,
 * FEM_E_NOMEM.  On error *out is set to NULL and nothing is leaked.
 */
int fem_plan_create(fem_plan **out, int form, int dim, int degree, int quad_degree,
                    int64_t n_vert, const double *coords, int64_t n_cell,
                    const int32_t *cell_verts, const int32_t *cell_nodes, int64_t n_node,
                    const double *params, int n_params);

/*
 * A plan on curved (non-affine) cells: every cell carries the 6 (triangle) or 10
 * (tetrahedron) nodes of a P2 geometry, and the map x(xi) = sum_g x_g phiG_g(xi) is
 * differentiated at every quadrature point, so J, J^{-1} and |det J| are evaluated per
 * point instead of once per cell (paper Sec. 2.4, non-affine geometry: the coordinates are
 * handled like a vector trial function).
 *   n_gnode      number of geometry nodes;  gcoords HOST f64 [n_gnode][dim]
 *   cell_gnodes  HOST i32 [n_cell][6 or 10]: the cell's geometry nodes in the P2 local
 *                order (reference lattice points alpha/2, first coordinate fastest, as for
 *                cell_nodes), so local nodes 0, 2, 5 (2D) or 0, 2, 5, 9 (3D) are the
 *                vertices
 *   other arguments as fem_plan_create (the solution degree is independent of the
 *   geometry degree: isoparametric for degree 2, sub- or super-parametric otherwise).
 * det J is checked at every point of the rule (FEM_E_INVERTED where it is zero, not
 * finite, changes sign within a cell, or is negative in 2D); between the points the map is
 * not checked.  Curved plans run one lane per cell, or lane triples for the 3D vector forms
 * (FEM_E_UNSUPPORTED for the other lane splits), and cannot join a batch.  Errors as fem_plan_create.
 */
int fem_plan_create_curved(fem_plan **out, int form, int dim, int degree, int quad_degree,
                           int64_t n_gnode, const double *gcoords, int64_t n_cell,
                           const int32_t *cell_gnodes, const int32_t *cell_nodes, int64_t n_node,
                           const double *params, int n_params);

/* Release a plan and its device memory (NULL is a no-op, FEM_OK).  Synchronises the device
 * before freeing so that no enqueued launch still reads the plan's arrays.  Errors:
 * FEM_E_ARG, with the plan left intact, while a batch (fem_batch_create) holds it. */
int fem_plan_destroy(fem_plan *plan);

/*
 * y = A(u): the operator action (paper Sec. 2.3, generic action kernel; App. A forms).
 * For FEM_NEOHOOKEAN and FEM_SVK this is the nonlinear residual r(u).
 *   u  DEVICE f64 [n_node * ncomp]  input
 *   y  DEVICE f64 [n_node * ncomp]  output, overwritten (not accumulated); must not alias u
 * Asynchronous on `stream`.  Errors: FEM_E_ARG (null plan/pointer), FEM_E_HIP (launch).
 * Non-finite output for FEM_NEOHOOKEAN if det F <= 0 at a quadrature point.
 */
int fem_action(const fem_plan *plan, const double *u, double *y, void *stream);

/*
 * y = A(u) for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result as fem_action, bit for bit, but the shared nodes' partial sums of the patch
 * strategy go to a static device buffer of FEM_NOALLOC_SCRATCH_DOUBLES doubles (16 MiB)
 * that the library holds on each device it runs on until the process ends, instead of the
 * plan's own buffer.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine) and does no kernel timing (fem_plan_set_timing does not apply).  Every
 * partial slot is written before it is read in each call, so nothing needs clearing.
 * Every call on one device shares that device's buffer: calls that overlap on one GPU
 * (concurrent streams, or threads) race and give wrong results; calls ordered on one
 * stream do not.  Colour-strategy plans and meshes without shared nodes use no scratch.
 *   u, y as fem_action.
 * Errors: FEM_E_UNSUPPORTED when the plan's partial sums (its shared partial slots times
 * ncomp) exceed the buffer; otherwise as fem_action.
 */
#define FEM_NOALLOC_SCRATCH_DOUBLES 2097152
int fem_action_noalloc(const fem_plan *plan, const double *u, double *y, void *stream);

/*
 * g = (dA/du)^T v: vector-Jacobian product of the action at u.  For the hyperelastic forms
 * (FEM_NEOHOOKEAN, FEM_SVK) the tangent of the residual is contracted with grad v at every
 * quadrature point, F being recomputed from u (nothing is stored between the forward and
 * this call).  For the linear forms A is symmetric and independent of u, so g = A v and u
 * is ignored.
 *   u, v  DEVICE f64 [n_node * ncomp] inputs;  g DEVICE f64 [n_node * ncomp] output,
 *   overwritten; g must alias neither u nor v.  Asynchronous.  Errors as fem_action, and
 *   FEM_E_UNSUPPORTED for a hyperelastic form when the configuration's tangent kernel
 *   spills registers to scratch memory (such kernels are not run: two heavily spilling
 *   ones returned wrong values); the plan's default configuration, every configuration the
 *   tuner keeps and the matrix-core kernel (lanes_per_cell 4) are free of such spills.
 *   Also FEM_E_UNSUPPORTED when the patch kernel's tangent, which stages u and v, needs
 *   more than 160 KB of LDS per workgroup for the plan's largest patch (plan creation and
 *   fem_plan_set_strategy check the action's need only): 3D P6 on full-size meshes.
 */
int fem_action_vjp(const fem_plan *plan, const double *u, const double *v, double *g,
                   void *stream);

/*
 * (dA/du) w: the tangent (linearised) action at u applied to w -- the operator the paper
 * times for its hyperelastic cases.  The hyperelastic tangents have major symmetry, so
 * this equals fem_action_vjp(plan, u, w) and runs the same kernels; for the linear forms
 * it is A w.  Arguments and errors as fem_action_vjp.
 */
int fem_action_jvp(const fem_plan *plan, const double *u, const double *w, double *out,
                   void *stream);

/*
 * One-shot y = A(u) from the mesh arrays alone: builds a temporary plan with the
 * arguments of fem_plan_create (default launch configuration), runs fem_action on
 * `stream`, waits for it and destroys the plan.  Synchronous and slow (plan building
 * dominates); for repeated actions on one mesh create a plan once.  Errors: those of
 * fem_plan_create and fem_action.
 */
int fem_action_once(int form, int dim, int degree, int quad_degree, int64_t n_vert,
                    const double *coords, int64_t n_cell, const int32_t *cell_verts,
                    const int32_t *cell_nodes, int64_t n_node, const double *params,
                    int n_params, const double *u, double *y, void *stream);

/* Plan properties (all outputs optional, pass NULL to skip). */
int fem_plan_info(const fem_plan *plan, int *n_loc, int *ncomp, int *n_quad, int *n_colours,
                  int64_t *n_dof);

/* Colour of every cell in the caller's cell order: HOST i32 [n_cell] out. */
int fem_plan_colouring(const fem_plan *plan, int32_t *colour);

/*
 * The plan's colouring on the host alone (no device needed): greedy first-fit over cells
 * in ascending id, a cell taking the smallest colour not held by an earlier cell that
 * shares one of its nodes.  The paper scatters with atomic adds (Sec. 4.1, single cell
 * per work-item; Sec. 4.2, tiled kernel); the colouring replaces them so that the sum
 * into each node runs in a fixed order.
 *   cell_nodes HOST i32 [n_cell][n_loc] (n_loc <= 64);  colour HOST i32 [n_cell] out;
 *   n_colours  HOST out (may be NULL).
 * Errors: FEM_E_ARG (sizes, nulls), FEM_E_INDEX, FEM_E_UNSUPPORTED (> 1024 colours).
 */
int fem_colouring(int64_t n_cell, int n_loc, const int32_t *cell_nodes, int64_t n_node,
                  int32_t *colour, int32_t *n_colours);

/*
 * Reference tables as used by the kernels (for testing the tabulation; paper Sec. 2.2,
 * tabulated-values equation): HOST outputs points [n_quad][dim], weights [n_quad],
 * phi [n_quad][n_loc], dphi [n_quad][n_loc][dim] (derivatives in the reference coordinates
 * xi), for the rule of `family` (FEM_QUAD_*).  Call with points == NULL to get n_quad and
 * n_loc only.  Errors: FEM_E_UNSUPPORTED (no such rule), FEM_E_ARG.
 */
int fem_reference_tables(int dim, int degree, int quad_degree, int family, int *n_quad,
                         int *n_loc, double *points, double *weights, double *phi,
                         double *dphi);

/* Switch the plan's quadrature family (FEM_QUAD_*) and re-tabulate.  Synchronises.
 * Errors: FEM_E_UNSUPPORTED (no rule of that family for the plan's degree), FEM_E_ARG. */
int fem_plan_set_quadrature(fem_plan *plan, int family);

/* Launch tuning of the colour strategy: cells per workgroup (64, 128 or 256); 0 restores
 * the default.  Errors: FEM_E_ARG for any other value. */
int fem_plan_set_block(fem_plan *plan, int cells_per_block);

/*
 * Scatter strategy (both are deterministic; they sum in different fixed orders, so their
 * results agree to rounding, and each is bitwise reproducible run to run):
 *   FEM_SCATTER_COLOUR  one launch per colour of the greedy colouring; a lane owning a
 *                       cell read-add-writes its nodes (no two cells of a launch share one).
 *   FEM_SCATTER_PATCH   one launch over patches of `patch_cells` consecutive cells along a
 *                       Morton curve of the cell centroids.  A workgroup stages its patch's
 *                       nodal values in LDS and sums its cells' vectors into the patch's
 *                       nodes in a fixed order; nodes no other patch holds are stored, the
 *                       others leave as partial sums that a second, small kernel adds in
 *                       patch order.  The default.  The P2 mass form on triangles with
 *                       256-cell coloured patches runs a pipelined variant: as many
 *                       workgroups as stay resident take the patches in turn, the next
 *                       patch's loads in flight during this one's work (same results).
 *   lanes_per_cell  1; 2 (2D vector forms: lane c of a pair owns component c); 3 (3D vector
 *                   forms: lane triples, 21 per wavefront); 4 (affine cells, every form:
 *                   the FP64 matrix-core kernel, where both contractions of the
 *                   quadrature loop run as 16x16x4 MFMA tiles over 16 cells per wavefront
 *                   and the pointwise form on the vector ALU, each cell's points and nodes
 *                   spread over four lanes; coloured sums only).
 *   patch_cells     64, 128 or 256 with 1 or 2 lanes (at most 256 lanes per workgroup);
 *                   21, 42, 63 or 84 with 3; 64 with 4.
 *   sum_mode        FEM_SUM_ELEMENT: every cell vector to an LDS element buffer, each node
 *                   summing its slots in ascending (cell, local node); FEM_SUM_COLOURED:
 *                   cells coloured inside the patch (first-fit, or DSatur where that
 *                   needs two colours fewer) accumulate into an LDS node buffer colour by
 *                   colour (smaller LDS, one barrier per colour).
 *   0 for lanes_per_cell, patch_cells or sum_mode picks the plan's default (three lanes
 *   for 3D vector forms of degree >= 3 when the patch size allows it, one otherwise;
 *   coloured sums; 42 cells for lane triples, else the largest patch whose element buffer
 *   would fit 64 KB).
 * Rebuilding patches synchronises the device.  Errors: FEM_E_ARG, FEM_E_UNSUPPORTED (a lane
 * split the form lacks, or more than 160 KB of LDS), FEM_E_HIP, FEM_E_NOMEM.
 */
#define FEM_SCATTER_COLOUR 0
#define FEM_SCATTER_PATCH 1
#define FEM_SUM_ELEMENT 1
#define FEM_SUM_COLOURED 2
int fem_plan_set_strategy(fem_plan *plan, int strategy, int patch_cells, int lanes_per_cell,
                          int sum_mode);
int fem_plan_get_strategy(const fem_plan *plan, int *strategy, int *patch_cells,
                          int *lanes_per_cell, int *sum_mode);

/* The plan's quadrature family (FEM_QUAD_*) and number of points.  Errors: FEM_E_ARG. */
int fem_plan_get_quadrature(const fem_plan *plan, int *family, int *n_points);

/*
 * Kernel timing, a measurement aid.  With timing on, every fem_action / fem_action_vjp
 * call on the plan times its main kernel with a pair of HIP events on the caller's stream:
 * for the patch strategy the events are attached to the patch kernel's dispatch
 * (hipExtLaunchKernel), so they read the kernel's own start and end; for the colour
 * strategy they bracket the run of colour launches.  The shared-node fixup and the zeroing
 * of untouched nodes fall outside.  fem_plan_get_timing waits
 * for the recorded events and returns the summed milliseconds and the number of bracketed
 * calls since timing was last switched on or off (either resets both).  The events are the
 * plan's and are destroyed with it.  Errors: FEM_E_ARG, FEM_E_HIP.
 */
int fem_plan_set_timing(fem_plan *plan, int enable);
int fem_plan_get_timing(fem_plan *plan, double *kernel_ms, int64_t *calls);

/*
 * Autotuner: time every launch configuration of the plan on the caller's vectors and keep
 * the fastest on the plan.  Candidates: the colour strategy with 64/128/256 cells per
 * workgroup; the patch strategy with 64/128/256 cells per patch and one lane per cell,
 * 64/128 with lane pairs (2D vector forms), 42/63/84 with lane triples (3D vector forms),
 * each with both sum modes; and the matrix-core kernel (affine cells, 64 cells per patch,
 * coloured sums): the matrix cores on or off.  The configuration the plan had on entry is kept unless a
 * candidate is more than 3% faster.  Timing follows the paper's protocol (Sec. 6.2.1): 5 warm-up runs,
 * then timed runs until 15 are collected or 0.2 s accumulates, arithmetic mean, HIP
 * events on `stream`.  Synchronises; may rebuild the plan's patches (host work).
 *   u, v   DEVICE inputs (v only for vjp != 0, which tunes fem_action_vjp instead)
 *   y      DEVICE scratch output of n_dof doubles (overwritten)
 *   cache_path  HOST path of a JSON cache to update (NULL: none).  fem_plan_create applies
 *          a cached configuration when the environment variable FEM_TUNE_CACHE names the
 *          file.  Keys: device architecture, form, dimension, degree, quadrature degree
 *          and rule family, round(log2(cell count)), and for the hyperelastic forms the
 *          direction (the VJP's entry is its own; plan creation applies the action's).
 *   results HOST f64 [max_results][6] out: strategy, cells per patch, lanes per cell,
 *          cells per workgroup (colour), sum mode, mean milliseconds; n_results HOST out.
 *   max_timed  0: time every candidate; k > 0: only the cost model's k best
 *          (fem_tune_predict) plus the entry configuration.
 * Errors: FEM_E_ARG, FEM_E_HIP, FEM_E_NOMEM.
 */
int fem_tune(fem_plan *plan, const double *u, const double *v, double *y, int vjp,
             const char *cache_path, void *stream, double *results, int max_results,
             int *n_results, int max_timed);

/*
 * The autotuner's cost model (paper Sec. 5, the heuristic performance model, adapted to
 * gfx950): an analytic time for every candidate of fem_tune, from the plan's sizes and the
 * compiled kernels' register counts, with no launch -- FP64 VALU time derated for low
 * occupancy (registers, LDS), memory time of the footprint plus shared-node partials or
 * colour scatters, and barrier / launch counts.  fem_tune with max_timed = k > 0 times only
 * the model's k best candidates (and the plan's entry configuration).
 *   results HOST f64 [max_results][6] out: as fem_tune's, the last column predicted ms.
 * Errors: FEM_E_ARG.
 */
int fem_tune_predict(const fem_plan *plan, int vjp, double *results, int max_results,
                     int *n_results);

/*
 * Batched actions over many meshes (y_i = A_i(u_i) for every plan of the batch) in a few
 * launches recorded once into a HIP graph.  The paper launches one kernel per mesh and
 * names small meshes as an open problem (Sec. 7); here the plans are grouped by kernel
 * variant (form, dimension, degree, lanes per cell, cells per patch), each group is one
 * launch over all patches of its meshes, and one launch sums every mesh's shared nodes.
 *
 * fem_batch_create: plans HOST [n] (each switched to the patch strategy if it is not on
 *   it).  The batch holds its plans until fem_batch_destroy: meanwhile fem_plan_destroy,
 *   fem_plan_set_strategy, fem_plan_set_quadrature and fem_tune on any of them fail with
 *   FEM_E_ARG and leave the plan unchanged (the batch keeps pointers to its arrays);
 *   u, y HOST arrays [n] of DEVICE pointers, mesh i reading u[i] and writing y[i] (no two
 *   meshes may share an output).  Synchronous.
 * fem_batch_set_vectors: rebind the vectors (synchronous; the graph is re-recorded at the
 *   next run).
 * fem_batch_run: enqueue the whole batch on `stream`; use_graph != 0 replays the recorded
 *   graph (recording it on the first call, on a private stream), 0 launches eagerly.  Both
 *   produce bitwise the same result as fem_action on each plan with the same strategy.
 * fem_batch_info: meshes, launch groups, total patches, total (shared node, component)
 *   items summed by the fixup launch (all optional).
 * Errors: FEM_E_ARG, FEM_E_UNSUPPORTED, FEM_E_HIP, FEM_E_NOMEM.
 */
typedef struct fem_batch fem_batch;
int fem_batch_create(fem_batch **out, int n, fem_plan *const *plans, const double *const *u,
                     double *const *y);
int fem_batch_set_vectors(fem_batch *batch, const double *const *u, double *const *y);
int fem_batch_run(fem_batch *batch, void *stream, int use_graph);
int fem_batch_info(const fem_batch *batch, int *n_mesh, int *n_groups, int64_t *n_patches,
                   int64_t *n_shared);
void fem_batch_destroy(fem_batch *batch);

/*
 * Host-only check of the patch layout the library would build for this mesh (no device
 * needed): every (cell, local node) contribution is summed exactly once into the node the
 * map names, every index the kernels follow lies inside its buffer, and every shared node's
 * partial slots are written once.  The same check runs inside fem_plan_create when the
 * environment variable FEM_CHECK=1 is set.
 *   stats HOST i64 [8] out (may be NULL): cells per patch, patches, most distinct nodes in a
 *         patch, (patch, node) pairs, shared nodes, partial slots, LDS bytes per workgroup
 *         for the forward kernel in the default sum mode, most sub-colours in a patch.
 * Errors: FEM_E_ARG (including a layout violation), FEM_E_INDEX, FEM_E_INVERTED,
 * FEM_E_UNSUPPORTED.
 */
int fem_check_patch_layout(int form, int dim, int degree, int64_t n_vert, const double *coords,
                           int64_t n_cell, const int32_t *cell_verts, const int32_t *cell_nodes,
                           int64_t n_node, int patch_cells, int64_t *stats);

/*
 * The main kernel the plan's current configuration launches for fem_action (vjp = 0) or
 * fem_action_vjp (vjp != 0): its registers per lane (hipFuncGetAttributes numRegs), its
 * scratch (spill) bytes per lane, and 1 if it is the variant with wave-priority hints
 * around its memory phases.  That variant of a coloured-sum patch kernel on affine cells
 * runs only where its compiled form uses no scratch memory; the environment variable
 * FEM_WAVE_PRIORITY=0 turns the hints off everywhere.  All outputs HOST, may be NULL.
 * Errors: FEM_E_ARG, FEM_E_HIP (no device).
 */
int fem_plan_kernel_info(const fem_plan *plan, int vjp, int *regs, int *scratch_bytes,
                         int *wave_priority);

/*
 * Measurement aids (the roofline's bandwidth input, paper Sec. 6.1: peak bandwidth is
 * measured, not assumed).
 * fem_stream_copy: dst[i] = src[i] for i < n, a STREAM-style copy that reads each byte of
 *   src once and writes each byte of dst once (16-byte accesses, grid-stride).
 *   src, dst  DEVICE f64 [n], 16-byte aligned, not overlapping.  Asynchronous on `stream`.
 * fem_stream_read: reads src[0..n) once and writes one partial sum per workgroup to
 *   sink[0..FEM_STREAM_SINK): a read-only pass that evicts the caches (L2 and the
 *   memory-side cache) without leaving dirty lines to be written back later.
 *   src DEVICE f64 [n], 16-byte aligned; sink DEVICE f64 [n_sink >= FEM_STREAM_SINK].
 * Errors: FEM_E_ARG (nulls, misalignment, overlap, short sink), FEM_E_HIP.
 */
#define FEM_STREAM_SINK 65536
int fem_stream_copy(const double *src, double *dst, int64_t n, void *stream);
int fem_stream_read(const double *src, int64_t n, double *sink, int64_t n_sink, void *stream);

/* Thread-local message of the last failing call ("" if none). */
const char *fem_last_error(void);

/* ABI version: major * 10000 + minor * 100 + patch. */
int fem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FEM_ACTION_H */
