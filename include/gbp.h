/*
 * gbp.h -- C ABI of the Geodesic-BP hot path for AMD Instinct MI355X (gfx950).
 *
 * Geodesic-BP (Grandits et al., arXiv 2308.08410) computes cardiac activation
 * times with the anisotropic eikonal equation on a tetrahedral mesh (Sec. 2.1,
 * Eq. (anisotropic_eikonal_eq)), differentiates them with respect to the model
 * parameters by back-propagation along geodesic parents (Sec. 2.3), and maps
 * them to body-surface ECGs with a precomputed lead-field operator (Sec. 2.4).
 *
 * General conventions (every entry point):
 *   - Array arguments are caller-owned, contiguous, row-major.  "device" means
 *     memory allocated with hipMalloc (e.g. a PyTorch tensor on the GPU);
 *     "host" means ordinary CPU memory.  Nothing passed in is retained after
 *     the call returns, except that a plan keeps its own copies of the mesh.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it.  gbp_eikonal_forward and gbp_eikonal_backward wait for
 *     it: how many relaxation rounds and adjoint levels a solve needs is known
 *     only on the device, so the host reads the device's convergence flag (one
 *     batch of launches behind, so that the device does not idle) and returns
 *     when the solve is done, with its statistics and error code.  Their _async
 *     variants enqueue a fixed budget of launches and return at once (for graph
 *     capture and streams the caller does not want to block on); the ECG, loss
 *     and Adam calls are fully asynchronous.
 *   - Outputs are overwritten, never accumulated into.
 *   - Return value: GBP_OK (0) or a negative GBP_ERR_* code; gbp_last_error()
 *     then returns a message (thread-local, valid until the next call).
 *   - Symmetric 3x3 tensors are packed as 6 floats (xx, yy, zz, xy, xz, yz).
 *     Gradients with respect to such a tensor store the off-diagonal entries
 *     doubled (dL/dA_xy + dL/dA_yx), so that sum_k A6[k]*dA6[k] = <A, dL/dA>_F.
 *   - Floating point is FP32 on the device.
 */
#ifndef GBP_H
#define GBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GBP_OK = 0,
    GBP_ERR_ARG = -1,             /* bad size, pointer or index */
    GBP_ERR_DEGENERATE_TET = -2,  /* an element with (near) zero volume */
    GBP_ERR_NOT_SPD = -3,         /* a velocity tensor that is not positive definite */
    GBP_ERR_NONFINITE = -4,       /* NaN or Inf in an input that must be finite */
    GBP_ERR_NOT_CONVERGED = -5,   /* iteration cap reached; outputs are still written */
    GBP_ERR_HIP = -6,             /* a HIP runtime call failed */
    GBP_ERR_NOMEM = -7            /* device or host allocation failed */
};

/* Opaque per-mesh plan: node/element reordering, adjacency, device workspace. */
typedef struct gbp_plan_s *gbp_plan;

typedef struct {
    float eps_rel;     /* change threshold: a node counts as changed when its value
                          drops by more than eps_rel*max(1,|T|); 0 -> 2^-20 */
    int max_rounds;    /* cap on global relaxation rounds; 0 -> 20000 */
    int reorder;       /* 0 -> default (locality reordering on), -1 -> keep caller order */
    int reserved[5];   /* must be zero */
} gbp_options;

typedef struct {
    int rounds;            /* global relaxation rounds executed */
    int converged;         /* 1 when the change set emptied before max_rounds */
    int64_t face_solves;   /* local problems evaluated */
    int64_t node_updates;  /* node value decreases by more than the threshold */
    int unreached;         /* nodes left at +inf (not connected to any root) */
    int reserved[3];
} gbp_stats;

/*
 * gbp_plan_create -- analyse a P1 tetrahedral mesh (Sec. 2.1: vertices V,
 * elements E_j, patches omega_i of elements around each vertex).
 *   xyz   host  float [n_v*3]  vertex coordinates
 *   tets  host  int32 [n_e*4]  vertex ids of each element (0-based)
 *   opt   host  may be NULL (defaults)
 *   out   host  receives the plan; destroy with gbp_plan_destroy.
 * Errors: GBP_ERR_ARG (sizes, ids out of range, repeated vertex in an element),
 * GBP_ERR_NONFINITE (coordinates), GBP_ERR_DEGENERATE_TET (|volume| below
 * 1e-7 of the cube of the element's longest edge), GBP_ERR_NOMEM, GBP_ERR_HIP.
 * Uses the current HIP device; all later calls with this plan must run there.
 */
int gbp_plan_create(const float *xyz, int n_v, const int32_t *tets, int n_e,
                    const gbp_options *opt, gbp_plan *out);
void gbp_plan_destroy(gbp_plan plan);
int gbp_plan_sizes(gbp_plan plan, int *n_v, int *n_e);

/*
 * gbp_eikonal_forward -- activation times phi at the vertices: the fixed point
 * of the Hopf-Lax rule phi_i = min over elements E_j around v_i of the local
 * minimum phi*_{j\i} = min_{x in face opposite v_i} phi(x) + ||v_i - x||
 * (Sec. 2.1 Eq. (hopflax_global), Eq. (hopflax_local); solved on each face in
 * barycentric form, Sec. 2.2 Eq. (upwind_eq_lsqr)), with phi = t_r at the roots
 * (initial conditions X_0, Sec. 2.1).  Iterated to convergence as in Alg. 2.
 *   D          device float [n_e*6]  velocity tensor per element (the paper's M,
 *                                    units length^2/time^2); a step e inside E_j
 *                                    costs sqrt(e^T D_eff^{-1} e)
 *   vscale     device float [n_v] or NULL (all ones): nodal velocity scale; the
 *                                    element uses D_eff = sbar^2 D with sbar the
 *                                    mean of its four nodal scales
 *   root_node  device int32 [n_roots]   vertex of each initial condition
 *   root_t     device float [n_roots]   its onset time; duplicates take the min
 *   T_init     device float [n_v] or NULL.  NULL: cold start from +inf.
 *              Non-NULL: a guess; the solve then uses the two-sided update
 *              (every node re-takes the minimum over its faces, roots also
 *              min with their onset), which converges to the same fixed point
 *              from any finite or infinite guess: the guess is taken as +inf on
 *              every connected component of the mesh that holds no root (there
 *              the two-sided update would raise the values without end).  With
 *              gbp_plan_set_warm_order on, the guess instead orders a cold
 *              solve (see there).
 *   T_out      device float [n_v]  (may alias T_init)
 *   stats      host, may be NULL
 * Unreached vertices get +inf.  Errors: GBP_ERR_ARG (root id out of range,
 * n_roots < 0), GBP_ERR_NONFINITE / GBP_ERR_NOT_SPD (D, vscale <= 0 or
 * non-finite, non-finite onsets), GBP_ERR_NOT_CONVERGED (T_out still written).
 */
int gbp_eikonal_forward(gbp_plan plan, const float *D, const float *vscale,
                        const int32_t *root_node, const float *root_t, int n_roots,
                        const float *T_init, float *T_out, gbp_stats *stats, void *stream);

/*
 * gbp_eikonal_backward -- vector-Jacobian product of the forward solve
 * (Sec. 2.3, Eq. (dto_grad)): with the geodesic parents frozen (the
 * minimising element and barycentric weights alpha of each vertex, recomputed
 * here from the converged T, never stored), L = sum_i dL_dT[i] T[i] has
 *   dL/dt_r  = lambda at the root's vertex if root r is active (its onset is
 *              not beaten by the upwind value, Sec. 2.5), else 0,
 *   dL/dD_j  = sum over vertices i parented by E_j of
 *              lambda_i * (-sbar_j^-2 D_j^-1 e e^T D_j^-1 / (2 h)),
 *   dL/ds_n  = 1/4 sum_{j containing n} sum_i lambda_i * (-h / sbar_j),
 * where e = sum_k alpha_k (v_k - v_i), h = sqrt(e^T D_eff,j^-1 e) and lambda
 * solves lambda = dL_dT + P^T lambda (P: parent weights).
 *   D, vscale, root_node, root_t, n_roots: as passed to the forward
 *   T          device float [n_v]   converged forward output
 *   dL_dT      device float [n_v]   incoming gradient (ignored at +inf nodes)
 *   dL_dD      device float [n_e*6] or NULL   (off-diagonals doubled)
 *   dL_dvscale device float [n_v]   or NULL
 *   dL_droot_t device float [n_roots] or NULL
 * The element metric, scales and onsets are rebuilt from D, vscale and the roots,
 * or kept from the previous call on the plan (see gbp_plan_set_input_reuse).
 * Errors: as the forward; GBP_ERR_NOT_CONVERGED if the adjoint did not settle.
 */
int gbp_eikonal_backward(gbp_plan plan, const float *D, const float *vscale,
                         const int32_t *root_node, const float *root_t, int n_roots,
                         const float *T, const float *dL_dT, float *dL_dD,
                         float *dL_dvscale, float *dL_droot_t, void *stream);

/*
 * gbp_eikonal_forward_async / gbp_eikonal_backward_async -- gbp_eikonal_forward
 * and gbp_eikonal_backward enqueued on `stream` with fixed launch budgets and no
 * host synchronisation (graph-capturable; the same kernels and results):
 *   round_budget  relaxation rounds (>= 1); rounds after convergence return at once
 *   level_budget  adjoint levels (>= 1); gs_budget Gauss-Seidel sweeps (>= 0) for
 *                 vertices on or above parent-graph cycles
 * Whether the budgets sufficed and the input errors the kernels found (root ids
 * out of range, non-finite inputs, D not positive definite) are kept on the
 * device: gbp_plan_status reads them (it synchronises), gbp_plan_forward_work the
 * work done.  Budgets come from a synchronous call on similar inputs
 * (gbp_plan_last_counts, gbp_backward_info) with a margin.  Errors returned here:
 * GBP_ERR_ARG (sizes, pointers, budgets), GBP_ERR_NOMEM, GBP_ERR_HIP.
 */
int gbp_eikonal_forward_async(gbp_plan plan, const float *D, const float *vscale,
                              const int32_t *root_node, const float *root_t, int n_roots,
                              const float *T_init, float *T_out, int round_budget, void *stream);
int gbp_eikonal_backward_async(gbp_plan plan, const float *D, const float *vscale,
                               const int32_t *root_node, const float *root_t, int n_roots,
                               const float *T, const float *dL_dT, float *dL_dD,
                               float *dL_dvscale, float *dL_droot_t, int level_budget,
                               int gs_budget, void *stream);

/*
 * gbp_plan_set_local_solver / gbp_plan_get_local_solver -- the local solver of
 * the forward's relaxation rounds:
 *   solver          0: exact minimum (all KKT candidates of the local problem,
 *                      Sec. 2.2 Eq. (upwind_eq_lsqr), predicated; the default)
 *                   1: n_f iterations of FISTA (Alg. 1) from alpha = 1/3, step
 *                      1/L per face with L from Eq. (lipschitz_est)
 *   n_f             FISTA iterations, 1..100000 (solver 1)
 *   lipschitz_mode  0: the lower bound h_ = sigma_min(A)/(3 sqrt 3) of Eq.
 *                      (lipschitz_est); 1: the tightened h_ = h(alpha*_0)/1.1 of
 *                      Sec. 2.5 (default)
 * FISTA values are feasible points, so they are never below the exact minimum:
 * the solve converges to activation times at or above the exact scheme's, closer
 * with more iterations.  The backward always uses the exact parents.
 * Errors: GBP_ERR_ARG for values outside those ranges, GBP_ERR_NOMEM.
 */
int gbp_plan_set_local_solver(gbp_plan plan, int solver, int n_f, int lipschitz_mode);
int gbp_plan_get_local_solver(gbp_plan plan, int *solver, int *n_f, int *lipschitz_mode);

/*
 * gbp_plan_set_fista_tolerance / gbp_plan_get_fista_tolerance -- iterations per
 * face for the FISTA solver from its rate, Eq. (fista_convergence), as Sec. 2.5
 * proposes (n_f per element): after k iterations from alpha = 1/3 the value is
 * at most 2 L ||alpha_0 - alpha*||^2 / (k+1)^2 above the minimum, and
 * ||alpha_0 - alpha*||^2 <= 2/3 on the simplex, so a face with step constant L
 * runs the least k with k + 1 >= sqrt(4 L / (3 tau)), at least 1 and at most the
 * n_f of gbp_plan_set_local_solver (FP32: product, quotient, root, each rounded).
 *   tau  value tolerance of a local problem (time units); 0 (the default): every
 *        face runs n_f iterations
 * The error bound holds with the step constant of Eq. (lipschitz_est)
 * (lipschitz_mode 0); with the tightened one it is the same rule on a smaller L.
 * Errors: GBP_ERR_ARG for a negative or non-finite tau.
 */
/*
 * gbp_plan_set_hold / gbp_plan_get_hold -- bucketed hold-back of the cold forward
 * (Delta-stepping on the active list of Alg. 2).  Bucket b holds the values in
 * [t_min + b delta, t_min + (b+1) delta), t_min the smallest onset.  A vertex whose
 * value drops beyond the current bucket plus `window` buckets does not propagate
 * yet; it waits in its bucket's list.  The buckets open in increasing order: one
 * per round whenever the active list is shorter than open_below vertices (0: half
 * of what one round's grid takes at once), and the next non-empty one whenever the
 * list is empty.  Only the order of the relaxation changes: the solve reaches the
 * same fixed point, with fewer re-evaluations of vertices whose first values were
 * too high, in more rounds.  delta = 0 (the default) turns it off.  Warm
 * (two-sided) solves do not hold.  Allocates 5 n_v / 4 ints of device memory on
 * first use (per plan).
 * Errors: GBP_ERR_ARG (delta negative or non-finite, window outside 0..32,
 * open_below < 0), GBP_ERR_NOMEM.
 */
int gbp_plan_set_hold(gbp_plan plan, float delta, int window, int open_below);
int gbp_plan_get_hold(gbp_plan plan, float *delta, int *window, int *open_below);

/*
 * gbp_plan_set_warm_order / gbp_plan_get_warm_order -- what a forward does with
 * T_init.  on = 0 (the default): the two-sided warm update from T_init.  on = 1:
 * the forward solves cold (from +inf, one-sided update, as with T_init NULL)
 * and uses T_init only as an ordering guess for the hold-back: a vertex whose
 * value has dropped is keyed by min(value, guess), so a value still above its
 * guess waits until the front reaches the guess (Delta-stepping keyed by a
 * prediction of the solution, e.g. the last iteration's times or the learned
 * warm start's).  The fixed point is the cold solve's for any guess (NaN reads as
 * +inf); the guess only changes the work.  With the hold-back off
 * (gbp_plan_set_hold delta = 0) the guess is ignored.  T_init may alias T_out.
 * Allocates n_v floats of device memory on first use (per plan).
 * Errors: GBP_ERR_ARG (on not 0 or 1), GBP_ERR_NOMEM.
 */
int gbp_plan_set_warm_order(gbp_plan plan, int on);
int gbp_plan_get_warm_order(gbp_plan plan, int *on);

/*
 * gbp_plan_set_input_reuse -- lets gbp_eikonal_backward and gbp_parent_map keep
 * what the last forward (or other call) on this plan built from its inputs: the
 * element metric D_eff^-1 per element, the nodal scales and the root onsets.
 * They are kept when the call passes the same D, vscale, root_node and root_t
 * pointers and root count as that call; otherwise they are rebuilt as always.
 * The caller promises that the arrays behind those pointers have not changed in
 * between (as with tensors saved for a backward pass).  Input errors of the
 * call that built them are still reported.
 *   on  1: allow, 0: always rebuild (the default)
 * Errors: GBP_ERR_ARG for on outside {0, 1}.
 */
int gbp_plan_set_input_reuse(gbp_plan plan, int on);

int gbp_plan_set_fista_tolerance(gbp_plan plan, float tau);
int gbp_plan_get_fista_tolerance(gbp_plan plan, float *tau);

/*
 * gbp_fista_iterations -- the per-face counts of gbp_plan_set_fista_tolerance
 * for n step constants (Eq. (fista_convergence)).
 *   lip    device float [n]  step constants L
 *   tau    tolerance (>= 0; 0 gives n_max everywhere)
 *   n_max  cap, 1..100000
 *   n_f    device int [n]    the counts
 * Errors: GBP_ERR_ARG (sizes, tau, n_max, missing pointers), GBP_ERR_HIP.
 */
int gbp_fista_iterations(const float *lip, int n, float tau, int n_max, int *n_f, void *stream);

/*
 * gbp_local_solve -- n independent local problems (Sec. 2.2 Eq.
 * (upwind_eq_lsqr)): min over the simplex of <alpha, Phi> + sqrt(alpha^T Q alpha).
 *   Q6       device float [n*6]  Q = E^T D_eff^-1 E packed (q00, q11, q22, q01, q02, q12)
 *   Phi      device float [n*3]  face values (+inf: unreached, weight zero)
 *   solver   0 exact, 1 FISTA (Alg. 1) with n_f iterations
 *   lip      device float [n] or NULL: FISTA step constants; NULL computes them
 *            with lipschitz_mode as in gbp_plan_set_local_solver
 *   value    device float [n]      the minimum (FISTA: the value at alpha_{n_f})
 *   alpha    device float [n*3] or NULL   the minimiser (FISTA: alpha_{n_f})
 *   lip_out  device float [n] or NULL     the step constants used (solver 1)
 * Errors: GBP_ERR_ARG (sizes, solver, n_f, mode, missing pointers), GBP_ERR_HIP.
 */
int gbp_local_solve(const float *Q6, const float *Phi, int n, int solver, int n_f,
                    const float *lip, int lipschitz_mode, float *value, float *alpha,
                    float *lip_out, void *stream);

/*
 * gbp_lead_field -- lead weights B = K Z on the device (Sec. 2.4 with unit
 * conductivity, G_i = I): K the P1 stiffness of the plan's mesh,
 * K_ab = sum over elements of |E| grad(l_a) . grad(l_b), and Z[n, l] =
 * 1 / |x_n - e_l| the lead field of a point electrode at e_l.  The result is
 * the W of gbp_ecg_forward.
 *   electrodes  device float [n_leads*3]
 *   W           device float [n_v*n_leads]  (caller vertex order, row-major)
 * FP64 arithmetic, deterministic.  Errors: GBP_ERR_ARG (n_leads outside
 * 1..256, missing pointers), GBP_ERR_HIP.
 */
int gbp_lead_field(gbp_plan plan, const float *electrodes, int n_leads, float *W, void *stream);

/*
 * Triangle meshes (d = 2, the setting of the paper's 2-D study, Sec. 3.1): the
 * forward and backward of the tetrahedral path with a segment as the local
 * simplex (Sec. 2.2 Eq. (upwind_eq_lsqr) with d = 2).  Mesh arrays are host
 * pointers, per-call arrays device pointers, as for tetrahedra.
 *
 * gbp_tri_plan_create -- xy [n_v*2] coordinates, tris [n_t*3] vertex ids.
 *   Errors: GBP_ERR_ARG (ids out of range, a repeated vertex), GBP_ERR_NONFINITE,
 *   GBP_ERR_DEGENERATE_TET (|2 area| below 1e-7 of the longest edge squared),
 *   GBP_ERR_NOMEM, GBP_ERR_HIP.
 * gbp_tri_forward -- activation times (Alg. 2, exact local solves in FP32):
 *   D [n_t*3] velocity tensor per triangle packed (xx, yy, xy), vscale [n_v] or
 *   NULL (D_eff = sbar^2 D, sbar the mean of the three nodal scales), vertex
 *   roots and onsets as gbp_eikonal_forward; T_out [n_v].  Synchronous (the
 *   convergence check reads the queue length every 8 rounds).  Errors: as
 *   gbp_eikonal_forward.
 * gbp_tri_backward -- vector-Jacobian product along the FP64 geodesic parents:
 *   dL_dD [n_t*3] (off-diagonal doubled) / dL_dvscale [n_v] / dL_droot_t
 *   [n_roots], each may be NULL; the formulas of gbp_eikonal_backward with
 *   d sbar / d s = 1/3.  The adjoint is the leaves-first level walk of
 *   gbp_eikonal_backward (each vertex finished once its children are, in a
 *   fixed order); the vertices that parent-graph cycles leave unfinished take
 *   Gauss-Seidel sweeps to a relative change of 1e-7.  Errors: as
 *   gbp_eikonal_backward.
 * gbp_tri_backward_info -- the last backward's level count, the vertices the
 *   walk left to the sweeps, and the sweeps taken (any pointer may be NULL).
 */
typedef struct gbp_tri_plan_s *gbp_tri_plan;
int gbp_tri_plan_create(const float *xy, int n_v, const int32_t *tris, int n_t, gbp_tri_plan *out);
void gbp_tri_plan_destroy(gbp_tri_plan plan);
int gbp_tri_forward(gbp_tri_plan plan, const float *D, const float *vscale, const int32_t *root_node,
                    const float *root_t, int n_roots, float *T_out, gbp_stats *stats, void *stream);
int gbp_tri_backward(gbp_tri_plan plan, const float *D, const float *vscale,
                     const int32_t *root_node, const float *root_t, int n_roots, const float *T,
                     const float *dL_dT, float *dL_dD, float *dL_dvscale, float *dL_droot_t,
                     void *stream);
int gbp_tri_backward_info(gbp_tri_plan plan, int *levels, int *cyclic, int *sweeps);

/*
 * gbp_point_roots -- initial conditions at points inside elements (Sec. 2.3
 * Eq. (upwind_xi)): a root at the point x_r of element E_k with onset t_r
 * gives each vertex v of E_k the onset t_r + sqrt((v - x_r)^T D_eff,k^-1 (v - x_r))
 * (the step cost of the forward in that element).  The 4 n_roots results are
 * vertex roots for gbp_eikonal_forward / gbp_eikonal_backward (a vertex named
 * by several takes the smallest onset).
 *   D, vscale  as for the forward (D_eff,k = sbar_k^2 D_k)
 *   root_tet   device int32 [n_roots]     caller element id holding each point
 *   root_xyz   device float [n_roots*3]   the points
 *   root_t     device float [n_roots]     onsets
 *   node_out   device int32 [4*n_roots]   caller vertex ids, root r at 4r..4r+3 in
 *                                         the element's vertex order
 *   t_out      device float [4*n_roots]   their onsets
 * Asynchronous.  An element id out of range gives vertex ids -1 (the forward
 * then returns GBP_ERR_ARG); non-finite points or onsets give non-finite
 * onsets (the forward returns GBP_ERR_NONFINITE).  Errors here: GBP_ERR_ARG
 * (n_roots < 0, missing pointers), GBP_ERR_HIP.
 */
int gbp_point_roots(gbp_plan plan, const float *D, const float *vscale, const int32_t *root_tet,
                    const float *root_xyz, const float *root_t, int n_roots, int32_t *node_out,
                    float *t_out, void *stream);

/*
 * gbp_point_roots_backward -- chain rule of gbp_point_roots (the gradient of
 * Sec. 2.3: d onset / d x_r = -D_eff^-1 e / |e|, e = v - x_r; d onset / d t_r = 1;
 * and the metric's dependence on D_k and the nodal scales, as in the backward).
 *   dL_donset     device float [4*n_roots]  e.g. gbp_eikonal_backward's
 *                                           dL_droot_t for the vertex roots
 *   dL_droot_t    device float [n_roots]    or NULL, overwritten
 *   dL_droot_xyz  device float [n_roots*3]  or NULL, overwritten
 *   dL_dD         device float [n_e*6]      or NULL, ACCUMULATED (off-diagonals
 *                                           doubled, as in the backward)
 *   dL_dvscale    device float [n_v]        or NULL, ACCUMULATED
 * A vertex at the point itself contributes to dL_droot_t only.  Roots sharing
 * an element or a vertex accumulate in unspecified order (rounding only).
 * Elements out of range give zero gradients.  Errors: as gbp_point_roots.
 */
int gbp_point_roots_backward(gbp_plan plan, const float *D, const float *vscale,
                             const int32_t *root_tet, const float *root_xyz, int n_roots,
                             const float *dL_donset, float *dL_droot_t, float *dL_droot_xyz,
                             float *dL_dD, float *dL_dvscale, void *stream);

/*
 * gbp_locate_points -- the element holding each point (for roots given by
 * position): the lowest caller element id whose barycentric coordinates of the
 * point are all >= -tol (FP32), or -1 if none.
 *   points   device float [n_points*3];  tet_out  device int32 [n_points]
 * Brute force over all elements (n_e x n_points tests).  Errors: GBP_ERR_ARG
 * (n_points < 0, tol < 0, missing pointers), GBP_ERR_HIP.
 */
int gbp_locate_points(gbp_plan plan, const float *points, int n_points, float tol,
                      int32_t *tet_out, void *stream);

/*
 * gbp_backward_info -- diagnostics of the last gbp_eikonal_backward on this
 * plan.  The adjoint walks the parent graph leaves-first in levels; two vertices
 * that are each other's weighted parents (possible in anisotropic media, where
 * a face vertex may be later than the vertex it updates) are solved together as
 * a 2x2 system.  `levels` is the number of levels walked, `cyclic` the number of
 * vertices the walk could not finish (on or above a longer cycle), and
 * `gs_sweeps` the Gauss-Seidel sweeps used to finish those.  Any pointer may be
 * NULL.
 */
int gbp_backward_info(gbp_plan plan, int *levels, int *cyclic, int *gs_sweeps);

/*
 * gbp_parent_map -- the geodesic parents used by the backward pass, exposed
 * for inspection: for every vertex the minimising element (Sec. 2.3: the
 * element whose face carries the upwind point), the three face vertices and
 * their barycentric weights alpha (zero off the support).
 *   par_tet   device int32 [n_v]    element id (caller numbering), -1 for a
 *                                   vertex that is its own parent (active root)
 *                                   or unreached
 *   par_node  device int32 [n_v*3]  face vertices (caller numbering), -1 if none
 *   par_alpha device float [n_v*3]  weights
 *   best      device float [n_v] or NULL: minimum upwind value per vertex
 */
int gbp_parent_map(gbp_plan plan, const float *D, const float *vscale,
                   const int32_t *root_node, const float *root_t, int n_roots,
                   const float *T, int32_t *par_tet, int32_t *par_node, float *par_alpha,
                   float *best, void *stream);

/* Action-potential template and time grid (Sec. 2.4 Eq. (tanh_waveform), read
 * with K0 the resting and K1 the peak potential):
 *   U(xi) = K0 + (K1 - K0) / (1 + exp(-4 xi / tau)),  t_s = t0 + s*dt, s < n_steps. */
typedef struct {
    float K0, K1, tau, t0, dt;
    int n_steps;
} gbp_ap;

/*
 * gbp_ecg_forward -- lead-field ECG (Sec. 2.4): ecg[s*L + l] =
 *   sum_n W[n*L + l] * U(t_s - T[n]).  W is the discretised lead-field operator
 *   B (one column per lead).  Vertices with T = +inf stay at rest (U = K0).
 *   T   device float [n_v];  W device float [n_v*L];  ecg device float [n_steps*L]
 *   1 <= L <= 256, 1 <= n_steps <= 2^20 (the kernels take tiles of 16 leads and
 *   chunks of 992 steps; the paper's 31 leads are two tiles).  Uses a
 *   library-owned scratch buffer per device (grown on demand, which frees the old
 *   one): forward calls that overlap on one device, on different streams or host
 *   threads, race on it, and a captured graph would keep a buffer that a later,
 *   larger call frees.  For either, use gbp_ecg_forward_batched with a batch of
 *   one instance (the batch owns its scratch).
 */
int gbp_ecg_forward(const float *T, int n_v, const float *W, int L, const gbp_ap *ap,
                    float *ecg, void *stream);

/*
 * gbp_ecg_forward_noalloc -- gbp_ecg_forward for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results, with the scratch in a
 * fixed-size array that the library holds in each GPU's memory (129 KB, for any
 * call within gbp_ecg_forward's limits: the lead tiles and time chunks reuse it
 * in stream order).  The call allocates and frees nothing.  Every call on one GPU
 * shares that GPU's array (the kernels clear it first): calls that overlap on one
 * GPU, on different streams or host threads, race on it.  Arguments, limits and
 * errors as gbp_ecg_forward; GBP_ERR_HIP if the array's address cannot be found.
 */
int gbp_ecg_forward_noalloc(const float *T, int n_v, const float *W, int L, const gbp_ap *ap,
                            float *ecg, void *stream);

/*
 * gbp_ecg_backward -- dL_dT[n] = -sum_s U'(t_s - T[n]) sum_l dL_decg[s*L+l] W[n*L+l]
 * (Sec. 2.4: the gradient of V_l is -B^T U' times the gradient of phi).
 *   dL_decg device float [n_steps*L];  dL_dT device float [n_v] (overwritten)
 * Limits as gbp_ecg_forward; no scratch (the tiles and chunks add into dL_dT in
 * launch order, so the result is deterministic).
 */
int gbp_ecg_backward(const float *T, int n_v, const float *W, int L, const gbp_ap *ap,
                     const float *dL_decg, float *dL_dT, void *stream);

/*
 * gbp_ecg_loss -- objective of Sec. 2.4 Eq. (inverse_ecg) with the time
 * integral as a rectangle rule: loss = sum (ecg - target)^2 / n and
 * dL_decg = 2 (ecg - target) / n, n = number of entries.
 *   ecg, target device float [n];  loss device float [1];  dL_decg device [n] or NULL
 */
int gbp_ecg_loss(const float *ecg, const float *target, int n, float *loss, float *dL_decg,
                 void *stream);

/*
 * gbp_adam_step -- one Adam update (the optimiser of Sec. 2.4) on n parameters:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * All arrays device float [n]; step >= 1.  Optional bounds: if lo < hi the
 * result is clamped to [lo, hi].
 */
int gbp_adam_step(float *param, const float *grad, float *m, float *v, int n, float lr,
                  float beta1, float beta2, float eps, int step, float lo, float hi,
                  void *stream);

/*
 * Kernel timing for diagnostics and roofline reports.  While enabled, each
 * launch of the library's kernels is bracketed by two HIP events recorded on the
 * stream the kernel runs on; gbp_profile_read synchronises those events and
 * returns, for one kernel family, the number of timed launches and their summed
 * duration in milliseconds.  Families: "metric", "fim_sweep", "parent",
 * "child_lists", "adj_level", "grad", "ecg_fwd", "ecg_bwd", "aux".
 * Enabling adds host overhead per launch; leave it off for throughput runs.
 * gbp_profile_read returns GBP_ERR_ARG for an unknown family name.
 */
int gbp_profile_enable(int on);
void gbp_profile_reset(void);
int gbp_profile_read(const char *kernel, int64_t *launches, double *total_ms);

/*
 * gbp_plan_status -- synchronises `stream` and reports the device-side status of
 * the last call on the plan: the error code its inputs raised (GBP_OK if none),
 * whether the last forward converged within its rounds, whether the last
 * backward settled, and the rounds / levels that carried work.  Needed after the
 * budgeted (graph-captured) calls, which do not synchronise.
 */
int gbp_plan_status(gbp_plan plan, int *err_code, int *forward_converged,
                    int *backward_settled, int *rounds, int *levels, void *stream);

/*
 * gbp_plan_forward_work -- synchronises `stream` and returns the work of the last
 * forward on the plan, synchronous or budgeted (e.g. inside a replayed step):
 * local problems evaluated and vertex value changes beyond the threshold.
 * Either pointer may be NULL.
 */
int gbp_plan_forward_work(gbp_plan plan, int64_t *face_solves, int64_t *node_updates,
                          void *stream);

/*
 * gbp_plan_set_launch / gbp_plan_get_launch -- launch configuration of the
 * relaxation rounds and adjoint levels (chosen by an autotuner):
 *   lanes        lanes per vertex in a relaxation round: 8, 16 or 32
 *   sweep_blocks grid of a relaxation round, 64..2048
 *   level_blocks grid of an adjoint level (a scan of all vertices, at most 8 per
 *                thread, so at least n_v / 2048 blocks are used), 16..2048
 *   sync_batch   launches between convergence checks in synchronous calls, 1..64
 * Results do not depend on the configuration beyond rounding order.
 * Errors: GBP_ERR_ARG for values outside those ranges.
 */
int gbp_plan_set_launch(gbp_plan plan, int lanes, int sweep_blocks, int level_blocks,
                        int sync_batch);
int gbp_plan_get_launch(gbp_plan plan, int *lanes, int *sweep_blocks, int *level_blocks,
                        int *sync_batch);

/*
 * Layout of the cold/warm relaxation queue (chosen by the autotuner).
 * split = 1 (default): the vertex range (Morton order) is cut into 512 regions,
 * region r is queued in sub-queue r mod 8, and the blocks the hardware places on
 * XCD x serve sub-queue x, so each XCD's L2 caches a fixed eighth of the mesh.
 * split = 0: one queue served by every block.  Results are the same fixed point.
 * Errors: GBP_ERR_ARG.
 */
int gbp_plan_set_queue_split(gbp_plan plan, int split);
int gbp_plan_get_queue_split(gbp_plan plan, int *split);
/* Rounds and levels that carried work in the last synchronous forward/backward. */
int gbp_plan_last_counts(gbp_plan plan, int *rounds, int *levels);

/*
 * Batches.  Many meshes solve together as one plan over their disjoint union
 * (the instances are its connected components, vertices numbered instance by
 * instance); a batch descriptor records where each instance's vertices start
 * so that the ECG and the misfit are evaluated per instance.  The batch owns the
 * ECG forward's scratch (n_inst * ~130 KB at most), so batched ECG calls are
 * graph-capturable; calls with one batch must not overlap.
 *   offsets  host int32 [n_inst+1], offsets[0] = 0, non-decreasing; instance i
 *            owns vertices [offsets[i], offsets[i+1]) of the union
 *   max_steps largest n_steps the batch will be used with (<= 2^20)
 * Errors: GBP_ERR_ARG, GBP_ERR_NOMEM, GBP_ERR_HIP.
 */
typedef struct gbp_batch_s *gbp_batch;
int gbp_batch_create(const int32_t *offsets, int n_inst, int max_steps, gbp_batch *out);
void gbp_batch_destroy(gbp_batch batch);
int gbp_batch_sizes(gbp_batch batch, int *n_inst, int *n_total);

/*
 * gbp_ecg_forward_batched / gbp_ecg_backward_batched -- Sec. 2.4 per instance:
 *   ecg[i][s][l] = sum over vertices n of instance i of W[n*L+l] U(t_s - T[n])
 *   T, W, dL_dT over the union (vertex order of the offsets); ecg and dL_decg
 *   device float [n_inst*n_steps*L].  Enqueue only (graph-capturable).
 */
int gbp_ecg_forward_batched(gbp_batch batch, const float *T, const float *W, int L,
                            const gbp_ap *ap, float *ecg, void *stream);
int gbp_ecg_backward_batched(gbp_batch batch, const float *T, const float *W, int L,
                             const gbp_ap *ap, const float *dL_decg, float *dL_dT,
                             void *stream);
/*
 * gbp_ecg_loss_batched -- per instance i: loss[i] = mean over its n_per entries of
 * (ecg - target)^2 and dL_decg = 2 (ecg - target) / n_per (so the gradient of
 * sum_i loss[i]).  ecg, target, dL_decg device float [n_inst*n_per]; loss device
 * float [n_inst].
 */
int gbp_ecg_loss_batched(const float *ecg, const float *target, int n_inst, int n_per,
                         float *loss, float *dL_decg, void *stream);

/*
 * gbp_adam_step_dev -- gbp_adam_step with the step number read from device memory
 * (*step >= 1), so that a captured graph can advance it; the caller (or
 * gbp_counter_add) increments it.
 */
int gbp_adam_step_dev(float *param, const float *grad, float *m, float *v, int n, float lr,
                      float beta1, float beta2, float eps, const int *step, float lo, float hi,
                      void *stream);
int gbp_counter_add(int *counter, int delta, void *stream);

/*
 * One Geodesic-BP iteration captured in a HIP graph (the batched, graph-launched
 * form).  gbp_step_create records, on a private capture stream, the budgeted
 * forward (cold, or warm from the previous iteration's T), the batched ECG,
 * misfit, ECG backward, budgeted adjoint and Adam on the velocity scale and the
 * root onsets, then instantiates the graph; gbp_step_launch replays it on
 * `stream`.  All buffers named in the descriptor are caller-owned device memory
 * that must stay allocated while the step exists; the step owns its scratch
 * (gradients, Adam moments, the step counter).  Budgets come from a synchronous
 * run (gbp_plan_last_counts) with a margin; gbp_plan_status tells whether they
 * sufficed.  Calls on one plan must not overlap.
 */
typedef struct {
    gbp_plan plan;
    gbp_batch batch;            /* instances of the plan's union mesh */
    const float *D;             /* [n_e*6] */
    float *vscale;              /* [n_v], updated by Adam */
    const int32_t *root_node;   /* [n_roots] union vertex ids */
    float *root_t;              /* [n_roots], updated by Adam */
    int n_roots;
    const float *W;             /* [n_v*L] */
    int L;
    gbp_ap ap;
    const float *target;        /* [n_inst*n_steps*L] */
    float *T;                   /* [n_v] activation times (output; warm-start input) */
    float *ecg;                 /* [n_inst*n_steps*L] output */
    float *loss;                /* [n_inst] output */
    float lr_vscale, lr_root_t, vscale_lo, vscale_hi;
    int round_budget, level_budget, gs_budget;
    int warm;                   /* 1: forward warm-started from T: two-sided update,
                                   or (plan's warm order on at creation) a cold
                                   solve ordered by T */
    int reserved[4];            /* must be zero */
} gbp_step_desc;
typedef struct gbp_step_s *gbp_step;
int gbp_step_create(const gbp_step_desc *desc, gbp_step *out);
int gbp_step_launch(gbp_step step, void *stream);
void gbp_step_destroy(gbp_step step);
/*
 * gbp_step_gradients -- copies, on `stream`, the gradients the last replay of the
 * step computed before its Adam updates (at the parameters that replay started
 * from): dL_dT [n_v] (ECG backward), dL_dvscale [n_v] and dL_droot_t [n_roots]
 * (eikonal backward), L the sum of the instances' misfits.  Device buffers, each
 * may be NULL.  Errors: GBP_ERR_ARG (no step), GBP_ERR_HIP.
 */
int gbp_step_gradients(gbp_step step, float *dL_dT, float *dL_dvscale, float *dL_droot_t,
                       void *stream);

/*
 * gbp_step_get_state / gbp_step_set_state -- the fit's optimiser state that a
 * step owns (Adam's first and second moments of the velocity scales and of the
 * onsets, and the Adam step counter, Sec. 2.4), for checkpointing and resuming
 * a fit: a step created from the same parameters, given the state saved after
 * iteration k, continues with iteration k + 1.
 *   m_vscale, v_vscale  device float [n_v]
 *   m_root_t, v_root_t  device float [n_roots] (ignored when n_roots == 0)
 *   counter             host int: the next update's index (>= 1; 1 before any)
 * Synchronous on `stream`.  Errors: GBP_ERR_ARG (NULL buffer, counter < 1).
 */
int gbp_step_get_state(gbp_step step, float *m_vscale, float *v_vscale, float *m_root_t,
                       float *v_root_t, int *counter, void *stream);
int gbp_step_set_state(gbp_step step, const float *m_vscale, const float *v_vscale,
                       const float *m_root_t, const float *v_root_t, int counter, void *stream);

/*
 * Learned warm start (an extension beyond the paper, which solves every
 * forward from scratch): a multilayer perceptron 16 -> 256 -> 256 -> 256 -> 256
 * -> 1 with ReLU activations predicts activation times from per-vertex
 * features; its prediction is gbp_eikonal_forward's T_init (the two-sided
 * update, or the ordering guess of gbp_plan_set_warm_order), whose fixed point
 * is the cold solution whatever the guess.
 *
 * Precision: features and hidden weights are bf16, products accumulate in
 * fp32 on the matrix cores, hidden activations are stored as bf16; the output
 * layer, master weights, gradients and Adam moments are fp32.  Backward rounds
 * the back-propagated activations' gradients to bf16 at each layer.
 * Parameter vector (fp32, gbp_mlp_num_params entries, this order): W1[256][16],
 * b1[256], W2[256][256], b2, W3[256][256], b3, W4[256][256], b4, w5[256], b5[1]
 * (row-major, W_l maps layer l-1 to layer l).
 *
 * gbp_mlp_create: allocates a network for training batches of up to max_rows
 *   rows (1 <= max_rows <= 2^21),
 *   He-normal weights from `seed` (column 16 of W1, the pad feature, is zero),
 *   zero biases and moments.  Errors: GBP_ERR_ARG, GBP_ERR_NOMEM, GBP_ERR_HIP.
 * gbp_mlp_set_params / gbp_mlp_get_params: host fp32 copies of the parameter
 *   vector (and of the last gradient); synchronous on `stream`.
 * gbp_mlp_features: X[r][16] (bf16 bit patterns, device) for the vertices
 *   rows[r] (device int32, or NULL for rows r = 0..n_rows-1, n_rows <= n_v) of a
 *   mesh given by xyz[n_v*3] and unit fibre directions fibre[n_v*3] (device,
 *   user order); a row id outside [0, n_v) gives zero features and a NaN target:
 *     0-2   (x - c) / len_scale
 *     3-5   fibre direction
 *     6-13  the 8 values |x - x_r| / len_scale + t_r / time_scale over the roots
 *           (root_xyz[n_roots*3], root_t[n_roots], device; 1 <= n_roots <= 8,
 *           fewer than 8 repeat root 0), sorted ascending
 *     14    vscale[i] (device, or NULL for 1)
 *     15    0
 *   norm: HOST float[5] = {cx, cy, cz, len_scale, time_scale}.  With T (device
 *   [n_v]) and target (device [n_rows]) non-NULL, also target[r] = T[rows[r]] /
 *   time_scale (training data).  Errors: GBP_ERR_ARG.
 * gbp_mlp_forward: y[m] = out_scale * MLP(X) for 1 <= m <= 2^27 rows (device;
 *   not limited by max_rows: the whole network runs in one kernel per 64 or 128
 *   rows with the activations kept on chip, rounded as in gbp_mlp_gradient's
 *   forward pass); non-finite predictions are written as +inf, which the
 *   warm-started solve treats as no information.  X must be 16-byte aligned
 *   (rows are read in 16-byte pieces).  Errors: GBP_ERR_ARG (rows, NULL,
 *   alignment).
 * gbp_mlp_gradient: forward, mean squared error against target[m] (device),
 *   written to *loss (device, may be NULL), and the parameter gradient (kept in
 *   the network; read with gbp_mlp_get_params); m <= max_rows, X 16-byte
 *   aligned.  Deterministic: every sum runs in a fixed order (per-tile and
 *   per-split partials, then a fixed-order reduction), so equal inputs give
 *   bitwise-equal gradients.  Errors: GBP_ERR_ARG (rows, NULL, alignment).
 * gbp_mlp_train_step: gbp_mlp_gradient followed by one Adam step (beta 0.9,
 *   0.999, eps 1e-8, bias-corrected) with learning rate lr on the fp32 masters
 *   and a refresh of their bf16 copies.
 * gbp_mlp_get_state / gbp_mlp_set_state: host fp32 copies of Adam's moments
 *   (gbp_mlp_num_params entries each) and the number of Adam steps taken, for
 *   checkpointing and resuming training (with gbp_mlp_get/set_params);
 *   synchronous on `stream`.  Errors: GBP_ERR_ARG (NULL buffer, step < 0).
 * All calls on one network are stream-ordered and must not overlap.
 */
typedef struct gbp_mlp_s *gbp_mlp;
int gbp_mlp_create(int max_rows, uint64_t seed, gbp_mlp *out);
void gbp_mlp_destroy(gbp_mlp mlp);
int gbp_mlp_num_params(gbp_mlp mlp);
int gbp_mlp_set_params(gbp_mlp mlp, const float *params, void *stream);
int gbp_mlp_get_params(gbp_mlp mlp, float *params, float *grads, void *stream);
int gbp_mlp_get_state(gbp_mlp mlp, float *m, float *v, int *step, void *stream);
int gbp_mlp_set_state(gbp_mlp mlp, const float *m, const float *v, int step, void *stream);
int gbp_mlp_features(const float *xyz, const float *fibre, const float *vscale, int n_v,
                     const int32_t *rows, int n_rows, const float *root_xyz,
                     const float *root_t, int n_roots, const float *norm, const float *T,
                     uint16_t *X, float *target, void *stream);
int gbp_mlp_forward(gbp_mlp mlp, const uint16_t *X, int m, float out_scale, float *y,
                    void *stream);
int gbp_mlp_gradient(gbp_mlp mlp, const uint16_t *X, int m, const float *target, float *loss,
                     void *stream);
int gbp_mlp_train_step(gbp_mlp mlp, const uint16_t *X, int m, const float *target, float lr,
                       float *loss, void *stream);

const char *gbp_last_error(void);
const char *gbp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GBP_H */
