/*
 * bemfmm.h - C ABI of the MI355X (gfx950) FMM-accelerated Burton-Miller
 * collocation boundary-element library.
 *
 * What is computed
 * ----------------
 * The paper (Isakari, Kondo, Takahashi, Matsumoto, "A level-set-based
 * topology optimisation for acoustic-elastic coupled problems with a fast
 * BEM-FEM solver") solves the boundary integral equation of Sec. 2.3
 * (Eq. danseibie2) for the 3-D Helmholtz kernel G = exp(ik|x|)/(4 pi |x|),
 * discretised with piecewise-constant triangles and collocation; its acoustic
 * block is I/2 - D (Eq. renritupu), applied by an FMM inside every GMRES
 * iteration (solver step 2(c), Sec. 2.3).  This library applies the
 * Burton-Miller combination of that equation with its normal derivative,
 *
 *     y = (I/2 - K - alpha H) p + (S + alpha K' + (alpha/2) I) q,
 *
 * where, for element j and collocation point x_i (centroid of element i),
 * S_ij = int_j G, K_ij = int_j dG/dn_y, K'_ij = int_j dG/dn_x and
 * H_ij = finite-part int_j d2G/dn_x dn_y; n is the unit normal pointing into
 * the fluid.  alpha = 0 gives the paper's own operator I/2 - D (D = K) with
 * S applied to q = dp/dn.  Regular pairs use the 3-point degree-2 triangle
 * rule; pairs with |x_i - c_j| < eta * (longest edge of j) are integrated
 * accurately; self terms use closed edge reductions.
 *
 * Conventions
 * -----------
 * - Vectors are DEVICE pointers to contiguous complex128 (interleaved re, im,
 *   the PyTorch layout), in the caller's element order; nrhs columns are
 *   stored one after the other with stride n_tri.  The caller owns them.
 * - Mesh arrays in bem_problem are HOST pointers, copied at plan creation.
 * - Calls are ordered on the given HIP stream (hipStream_t passed as void*,
 *   NULL = the default stream).  Matvecs are asynchronous; solves
 *   synchronise before returning.
 * - Errors: every call returns a bem_status; on failure bem_last_error()
 *   returns a thread-local message.  Invalid input is rejected before any
 *   kernel launch.  No call allocates on behalf of the caller except
 *   bem_plan_create.
 * - A plan may hold several problems (meshes / wavenumbers); `prob` selects
 *   one.  The tree, lists, near-field coefficients and translation
 *   operators of a problem are built once and reused by forward and adjoint
 *   products and solves (the paper reuses them between its state and
 *   adjoint solves, Sec. 2.5, steps 6-7).
 * - Thread safety: calls on the same plan must not overlap.
 */
#ifndef BEMFMM_H
#define BEMFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_plan bem_plan; /* opaque */

typedef enum {
  BEM_OK = 0,
  BEM_E_INVALID = -1,   /* bad argument or mesh; nothing was launched        */
  BEM_E_OOM = -2,       /* device allocation failed                          */
  BEM_E_HIP = -3,       /* a HIP runtime call failed                         */
  BEM_E_NOCONV = -4,    /* GMRES hit max_iter; x holds the last iterate      */
  BEM_E_BREAKDOWN = -5, /* GMRES breakdown without convergence               */
  BEM_E_NAN = -6        /* NaN/Inf met in a solve                            */
} bem_status;

/* Arithmetic of the far field, near field and their corrections.  Vectors
 * at the boundary are complex128 in both cases; the self (diagonal) terms
 * and the I/2, alpha/2 identities are always applied in float64. */
typedef enum { BEM_C128 = 0, BEM_C64 = 1 } bem_prec;

typedef struct {
  const double* vert;  /* host, n_vert x 3, row-major                       */
  int64_t n_vert;
  const int32_t* tri;  /* host, n_tri x 3, counter-clockwise seen from the
                          fluid (right-hand normal into the fluid)         */
  int64_t n_tri;
  double k;            /* wavenumber, > 0                                   */
  double alpha_re;     /* Burton-Miller coupling alpha (i/k typical; 0 =    */
  double alpha_im;     /*   the paper's conventional equation)              */
  double near_eta;     /* near-pair radius factor eta (<= 0 -> 2)           */
  int32_t leaf_cap;    /* uniform leaf level = smallest level >= 2 whose
                          fullest leaf holds <= leaf_cap elements (<=0->64) */
  int32_t leaf_level;  /* > 0 forces the leaf level instead; < 0 tunes it:
                          the occupancy-rule level and its two neighbours
                          are built and timed on a float32 product at plan
                          creation, and the fastest is kept              */
  int32_t order64;     /* expansion order of the float64 far field: > 0
                          fixed; 0: per level ceil(k sqrt(3) h) + 8 + s, at
                          least 12 + s (s: calibration shift, see
                          fmm_tol); < 0: the same with minimum -order64    */
  int32_t order32;     /* same for the float32 far field (+3, at least 7)  */
  double fmm_tol;      /* target relative L2 error of the float64 product
                          against the exact discrete operator (the paper
                          fixes its truncation numerically to an error
                          target, Sec. 3).  > 0: at plan creation the
                          product is applied to seeded random densities and
                          compared on 128 sampled rows with those rows
                          summed directly in float64, and likewise on a
                          plane-wave density (smooth: its far field adds up
                          coherently and errs more); the level rule is
                          shifted, up or down, until the larger of the two
                          sampled errors is below 0.7 fmm_tol.  <= 0: the
                          rule unshifted.  Ignored when order64 > 0.      */
  double fmm_tol32;    /* same for the float32 product, whose orders are
                          only raised above the rule (<= 0: the rule)     */
  int32_t p_max;       /* largest expansion order (<= 0 -> 40, > 40 invalid) */
  int32_t m2l_rot;     /* multipole-to-local variant per level (the paper's
                          low-frequency FMM fixes none, Sec. 2.3): 0 dense
                          or rotation-based (point-and-shoot: rotate the
                          multipole onto the translation axis, translate
                          along it, rotate back; ~3.3 (p+1)^3 instead of
                          (p+1)^4 operations per pair, ahead as the orders
                          grow with k times the box size), whichever the
                          plan times faster on the level; 1 dense only;
                          2 rotation-based on every level of order <= 23;
                          else BEM_E_INVALID.  Products agree to rounding. */
} bem_problem;

typedef struct {
  double tol;          /* relative residual ||b - A x|| / ||b|| target       */
  int32_t restart;     /* GMRES restart length m (<= 0 -> 50)                */
  int32_t max_iter;    /* total Arnoldi steps (<= 0 -> 2000)                 */
  int32_t mode;        /* 0: float64 operator throughout;
                          1: mixed precision - inner GMRES on the float32
                             operator, outer residuals and corrections in
                             float64 (iterative refinement)                 */
  double inner_tol;    /* mode 1: relative residual reduction asked of the
                          first inner solve (<= 0 -> 1e-3); later ones ask
                          for half the reduction still needed, >= 1e-6      */
  int32_t use_x0;      /* nonzero: x holds the initial guess on entry       */
} bem_gmres_opts;

typedef struct {
  int32_t iterations;  /* Arnoldi steps (all precisions)                     */
  int32_t matvec64;    /* float64 operator applications                     */
  int32_t matvec32;    /* float32 operator applications                     */
  int32_t restarts;    /* GMRES restarts (mode 0) / refinement steps (mode 1)*/
  double resid;        /* final true relative residual (float64 operator)   */
  int32_t converged;
  int32_t n_hist;      /* entries written to hist                           */
  double hist[512];    /* residual estimates per Arnoldi step (truncated)   */
} bem_gmres_info;

typedef struct {
  int64_t n_tri;
  int32_t leaf_level;
  int32_t n_leaves;
  int64_t n_near;          /* near pairs (off-diagonal accurate entries)     */
  int64_t n_p2p_pairs;     /* (target, source element) pairs in the U lists */
  int64_t n_m2l[22];       /* multipole-to-local pairs per level             */
  int32_t order64[22];     /* expansion order per level                      */
  int32_t order32[22];
  double box_size[22];
  int64_t device_bytes;    /* device memory held by this problem             */
  double tuned_ms;         /* leaf_level < 0: float32 product time (ms) of the
                              kept leaf level; 0 otherwise                   */
  int32_t m2l_tile32[22];  /* pairs per tile of the float32 M2L per level   */
  int32_t schedule[2];     /* stream schedule of the float64 / float32
                              products, chosen by timing at plan creation:
                              0 leaf-level M2L beside the upward pass, 1 it
                              before the upward pass, 2 as 1 with the near
                              field started after it, 3 as 0 with the near
                              field started after the upward pass, 4 as 0
                              with the near field started after the leaf
                              multipoles, behind the leaf-level M2L, 5
                              every stage on the caller's stream, one after
                              another                                       */
  int32_t p2p_grid[2];     /* near-field workgroups (float64 / float32): 0 one
                              per leaf, else a grid-stride launch of that
                              many (chosen with the schedule)               */
  int32_t m2l_grid[2];     /* leaf-level M2L workgroups, same convention    */
  int32_t direct_depth[2]; /* levels above the leaves reached by direct
                              leaf <-> ancestor translations in one launch
                              (0: level-by-level chains); chosen by timing  */
  double fmm_err64;        /* sampled relative error of the float64 / float32 */
  double fmm_err32;        /* product on white-noise densities, measured at
                              plan creation (see fmm_tol; 0: direct sum)    */
  double fmm_err64_smooth; /* the same on a plane-wave density             */
  double fmm_err32_smooth;
  int32_t far_cut[2];      /* orders dropped from the multipole side of the M2L
                              translations across three boxes, float64 / float32
                              (chosen by the calibration: they converge much
                              faster than those across two)                    */
  int64_t n_m2l_far[22];   /* of the multipole-to-local pairs per level, those
                              across three boxes (Chebyshev distance 3)        */
  int32_t m2l_rot64[22];   /* 1 where the level's float64 / float32 M2L is */
  int32_t m2l_rot32[22];   /* rotation-based (see bem_problem.m2l_rot)     */
} bem_plan_stats;

/* Build a plan for n_probs problems: everything the products of Sec. 2.3
 * (the FMM of solver step 2(c)) need that does not depend on the densities,
 * built once and reused by every forward and adjoint product and solve (the
 * paper reuses its tree, near-field integrals and translation operators
 * between the state and adjoint solves, Sec. 2.5 steps 6-7).  Uploads the
 * meshes and runs, on the device: element geometry and quadrature points
 * (constant elements with collocation, Sec. 2.3), Morton keys and a stable
 * radix sort, the uniform-depth octree and its U/V lists, the near-pair
 * list with accurate near-singular integrals and self terms, and the
 * translation, multipole and local operators in float64 and float32.
 * Rejects NULL pointers, n_tri < 1, indices out of range, non-finite
 * coordinates, zero-area triangles, k <= 0 (BEM_E_INVALID). */
int bem_plan_create(const bem_problem* probs, int n_probs, void* stream, bem_plan** out);
int bem_plan_destroy(bem_plan* plan);
int bem_plan_get_stats(const bem_plan* plan, int prob, bem_plan_stats* stats);

/* y = (I/2 - K - alpha H) p + (S + alpha K' + (alpha/2) I) q  (Burton-Miller
 * combination of the boundary integral equation of Sec. 2.3).  p or q may
 * be NULL (treated as zero); y must not alias p or q.  nrhs >= 1 columns. */
int bem_fmm_matvec(bem_plan* plan, int prob, int prec, const void* p, const void* q,
                   void* y, int nrhs, void* stream);

/* bem_fmm_matvec without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): same arguments, operator, kernels and results, but the
 * product's own buffers (sorted densities, near-field sums, expansions of
 * every level, per-pair M2L results) are laid out in the library's static
 * device array of 64 MiB per device (held until the process ends) instead of
 * the plan's buffers.  BEM_E_INVALID, with a message naming the sizes, when a
 * problem's buffers need more than that (about N <= 5000 in float64 and
 * N <= 20000 in float32 on spheres).  All calls on one device share that
 * device's array: calls that overlap on one device (other streams, other
 * threads) race.  Stage profiling is skipped for these calls. */
int bem_fmm_matvec_noalloc(bem_plan* plan, int prob, int prec, const void* p, const void* q,
                           void* y, int nrhs, void* stream);

/* Exact algebraic adjoint of bem_fmm_matvec: the operator of the adjoint
 * problem (Sec. 2.2, Eq. danseiajohel, which the paper solves with the same
 * boundary operator as the state problem), conjugate-transposed in its
 * discrete form, with the same tree, near field and operators as the
 * forward product (reused, Sec. 2.5 steps 6-7):
 *     u = (I/2 - K - alpha H)^H y,   w = (S + alpha K' + (alpha/2) I)^H y.
 * Device complex128 vectors, nrhs columns of stride n_tri; u or w may be
 * NULL (not both; w = NULL leaves out the w terms); outputs must not alias
 * y.  BEM_E_INVALID for bad arguments. */
int bem_fmm_matvec_adjoint(bem_plan* plan, int prob, int prec, const void* y, void* u,
                           void* w, int nrhs, void* stream);

/* Solve A(sigma) x = b by restarted GMRES (the paper's iterative solver,
 * Sec. 2.3 step 2 and Sec. 3), with A(sigma) = (I/2 - K - alpha H) +
 * (S + alpha K' + (alpha/2) I) diag(sigma).  sigma (device complex128,
 * n_tri) may be NULL (rigid scatterer, q = 0).  adjoint != 0 solves
 * A(sigma)^H x = b instead.  x0 = 0 unless opts->use_x0.  Exit on the true
 * relative residual recomputed with the float64 operator.  Synchronises. */
int bem_gmres_solve(bem_plan* plan, int prob, const void* sigma, int adjoint, const void* b,
                    void* x, const bem_gmres_opts* opts, bem_gmres_info* info, void* stream);

/* Batched solves: n_sys systems, system i being problem probs[i] with
 * sigma[i] (may be NULL, or sigma itself NULL for all rigid), adjoint[i]
 * (NULL = all forward), right-hand side b[i] and solution x[i] (device
 * complex128, distinct x).  probs, sigma, adjoint, b, x and infos are HOST
 * arrays (of device pointers).  All systems advance in lockstep, one float64
 * residual or one Arnoldi step per system per tick, with one host
 * synchronisation per tick; each stage of a tick's products and each phase
 * of its orthogonalisation is one launch over all systems (near field and
 * leaf-level M2L on the plan's side streams).  The systems' Krylov and
 * product buffers are kept by the plan for later calls (freed with it).
 * Same options and exit test as bem_gmres_solve (mode 1: GMRES(m) on the
 * float32 operator inside each refinement step, restarted from the float64
 * residual).
 * Returns BEM_OK when every system converged, else the first failing status;
 * infos[i] (may be NULL) reports each system.  Ordered after prior work on
 * `stream`; synchronises before returning. */
int bem_gmres_solve_batch(bem_plan* plan, int n_sys, const int32_t* probs,
                          const void* const* sigma, const int32_t* adjoint, const void* const* b,
                          void* const* x, const bem_gmres_opts* opts, bem_gmres_info* infos,
                          void* stream);

/* Right-hand side of a plane wave exp(i k d.x) of unit amplitude:
 * b_i = p_inc(x_i) + alpha dp_inc/dn(x_i) (device complex128 out). */
int bem_plane_wave_rhs(bem_plan* plan, int prob, const double* dir3, void* b, void* stream);

/* Right-hand side of point sources of intensity A_m at y_m (the source term
 * of the paper's forward problem, Eq. hel, whose incident field is
 * p_inc = sum_m A_m G(x - y_m)):  b_i = p_inc(x_i) + alpha dp_inc/dn(x_i).
 * src: device float64 n_src x 3 (off the boundary); amp: device complex128
 * n_src; b: device complex128 n_tri out (caller order).  n_src >= 1. */
int bem_point_source_rhs(bem_plan* plan, int prob, const double* src, const void* amp, int n_src,
                         void* b, void* stream);

/* Field at exterior points by the integral representation (solver step 5,
 * Sec. 2.3): out_m = inc_m + sum_j [int_j dG/dn_y p_j - int_j G q_j] with the
 * 3-point rule, inc_m = exp(i k d.x_m) if dir3 != NULL else 0.  pts: device
 * float64 n_pts x 3; p, q, out device complex128 (q may be NULL). */
int bem_eval_field(bem_plan* plan, int prob, const void* p, const void* q, const double* pts,
                   int n_pts, const double* dir3, void* out, void* stream);

/* Total field and its gradient at exterior points (solver step 5, the
 * integral representation; 3-point rule, so points should lie more than an
 * element size off the boundary):
 *   out_m  = inc(x_m) + sum_j [int_j dG/dn_y p_j - int_j G q_j],
 *   grad_m = grad of the same (3 complex per point, x y z),
 * inc = exp(i k d.x) if dir3 != NULL, plus sum_s A_s G(x - y_s) for point
 * sources (src: device float64 n_src x 3, amp: device complex128 n_src; src
 * NULL for none).  p, q (q may be NULL): device complex128 boundary data;
 * pts: device float64 n_pts x 3; out: device complex128 n_pts; grad (may be
 * NULL): device complex128 3 n_pts.  Summed directly over the elements
 * (cost n_pts x n_tri). */
int bem_eval_field_grad(bem_plan* plan, int prob, const void* p, const void* q,
                        const double* pts, int n_pts, const double* dir3, const double* src,
                        const void* amp, int n_src, void* out, void* grad, void* stream);

/* A fixed set of evaluation points (the design-domain lattice on which the
 * topology loop of Sec. 3 evaluates the state and adjoint fields, step 8)
 * sorted into an octree on the grid of problem `prob`'s tree, with the
 * translations from the problem's boxes into the point boxes, for one
 * precision (BEM_C128 or BEM_C64).  Created once per point set and problem,
 * reused by every evaluation; it refers to the plan, so destroy it first.
 * pts: host float64 n_pts x 3 (row-major, copied).  Every point must lie
 * within two widths of the tree's root cube from that cube (per axis);
 * BEM_E_INVALID otherwise (and for non-finite coordinates or prec 2).  A
 * problem without a far field (leaves not wider than the near radius) keeps
 * the points for the direct sum. */
typedef struct bem_field_points bem_field_points;
int bem_field_points_create(bem_plan* plan, int prob, int prec, const double* pts,
                            int64_t n_pts, void* stream, bem_field_points** out);
int bem_field_points_destroy(bem_field_points* fp);

typedef struct {
  int64_t n_pts;
  int32_t levels;                    /* deepest level (the problem's leaf level) */
  int32_t n_box[22];     /* point boxes per level */
  int64_t n_m2l[22];     /* translations into point boxes per level */
  int32_t order[22];     /* expansion orders (the problem's) */
  int64_t n_leaf;                    /* point boxes evaluated (leaves) */
  int64_t n_near_pairs;              /* point x element pairs summed directly */
  int64_t device_bytes;
  int64_t n_m2l_far[22];             /* of the translations, those across three
                                        boxes or more                         */
  int32_t far_cut;                   /* input orders cut from those (0: the
                                        point-box translations use full orders) */
  int32_t m2l_rot[22];               /* 1 where the level's translations into
                                        point boxes are rotation-based (the
                                        problem's own M2L of the precision is,
                                        or bem_problem.m2l_rot = 2)            */
} bem_field_points_stats;
int bem_field_points_get_stats(const bem_field_points* fp, bem_field_points_stats* st);

/* bem_eval_field_grad on the point set of `fp` (outputs in the order the
 * points were given), with the boundary sums split by the FMM: translations
 * of the problem's multipoles into the point boxes, local expansions
 * evaluated with their gradient at the points, and the 3-point rule summed
 * directly over the touching leaves.  It differs from the direct sum by the
 * expansions' truncation (the products' tolerance).  Arguments as
 * bem_eval_field_grad; stream-ordered, the set's buffers are reused by the
 * next call (overlapping calls on one set race). */
int bem_eval_field_grad_fmm(bem_field_points* fp, const void* p, const void* q,
                            const double* dir3, const double* src, const void* amp, int n_src,
                            void* out, void* grad, void* stream);

/* Fluid and solid constants of the topological derivative: densities
 * rho_f, rho_s, bulk moduli lam_f, lam_s, angular frequency omega (time
 * factor exp(-i omega t)).  rho_s = lam_s = +INFINITY is the sound-hard
 * (rigid) limit. */
typedef struct {
  double rho_f, lam_f, rho_s, lam_s, omega;
} bem_material;

/* Topological derivative for the appearance of a small elastic sphere in
 * the fluid (Sec. 2.2, Eq. danseitpoderi) at n_pts points, from the state
 * field p, grad p and the adjoint field pt, grad pt there (as from
 * bem_eval_field_grad; the adjoint field is the one radiated by point
 * sources of intensity df/dp at the observation points, Eq. danseiajohel):
 *   T = Re[3 (rho_s - rho_f) / (2 rho_s + rho_f) grad p . grad pt
 *          - (lam_s - lam_f) / (lam_s lam_f) rho_f omega^2 p pt].
 * Device arrays: p, pt complex128 n_pts; grad_p, grad_pt complex128 3 n_pts;
 * T float64 n_pts out. */
int bem_topological_derivative(int n_pts, const void* p, const void* grad_p, const void* pt,
                               const void* grad_pt, const bem_material* mat, double* T,
                               void* stream);

/* Adjoint of bem_eval_field's boundary part: rp_j = sum_m conj(int_j dG/dn_y
 * (x_m)) c_m, rq_j = -sum_m conj(int_j G(x_m)) c_m.  rq may be NULL. */
int bem_eval_field_adjoint(bem_plan* plan, int prob, const double* pts, int n_pts,
                           const void* c, void* rp, void* rq, void* stream);

/* Objective J = sum_m |p(x_m)|^2 of the plane-wave problem with admittance
 * boundary q = sigma p, sigma = -i k beta (beta device complex128, n_tri),
 * and its gradient grad_e = dJ/dRe(beta_e) + i dJ/dIm(beta_e) by the discrete
 * adjoint: one forward solve, one adjoint solve (conjugate-transposed FMM
 * operator), one adjoint product.  grad may be NULL (objective only).
 * p_out (may be NULL) receives the boundary pressure.  Synchronises. */
int bem_objective_grad(bem_plan* plan, int prob, const void* beta, const double* dir3,
                       const double* pts, int n_pts, const bem_gmres_opts* opts, double* J,
                       void* grad, void* p_out, bem_gmres_info* info_fwd,
                       bem_gmres_info* info_adj, void* stream);

/* The two halves of bem_objective_grad, for callers that need J without its
 * gradient (line searches) or that take the gradient later (reverse-mode
 * differentiation: the adjoint solve is the backward pass).
 *
 * Forward half, the state problem (Sec. 2.3, Eq. danseibie2 with the
 * admittance boundary q = sigma p): one solve of A(sigma) p = b for the
 * plane wave, the field p_obs at the points (solver step 5) and
 * J = sum |p_obs|^2 (Eq. obj with f = |p|^2).  p_out (device complex128,
 * n_tri) and pobs_out (device complex128, n_pts) receive p and p_obs; either
 * may be NULL.  Synchronises. */
int bem_objective_forward(bem_plan* plan, int prob, const void* beta, const double* dir3,
                          const double* pts, int n_pts, const bem_gmres_opts* opts, double* J,
                          void* p_out, void* pobs_out, bem_gmres_info* info, void* stream);

/* Backward half, the adjoint problem (Sec. 2.2, Eq. danseiajohel, here the
 * discrete adjoint of the collocation system): from the forward half's p and
 * p_obs (device complex128), one solve with the conjugate-transposed operator
 * A(sigma)^H, one adjoint product, and grad_e = dJ/dRe(beta_e) +
 * i dJ/dIm(beta_e) (pairing of Eq. danseideltaJ) into grad (device
 * complex128, n_tri, must not alias an input).  The tree, near field and
 * operators are those of the forward solve (reused, Sec. 2.5 steps 6-7).
 * Synchronises. */
int bem_objective_backward(bem_plan* plan, int prob, const void* beta, const void* p,
                           const void* pobs, const double* pts, int n_pts,
                           const bem_gmres_opts* opts, void* grad, bem_gmres_info* info,
                           void* stream);

/* Morton keys (uint64, caller order) and the sorted permutation (int32:
 * sorted position -> caller index) of a problem, copied to device buffers
 * the caller owns (n_tri entries each; either may be NULL). */
int bem_tree_export(bem_plan* plan, int prob, void* keys, void* perm, void* stream);

/* Leaf boxes: box keys (uint64, level-L keys) and [start, end) ranges in
 * sorted order; device buffers of n_leaves entries (any may be NULL). */
int bem_leaves_export(bem_plan* plan, int prob, void* box_keys, void* start, void* end,
                      void* stream);

/* Interaction lists of the octree (the FMM's partition of the element pairs,
 * Sec. 3): at tree level `level` (2 .. leaf level) the level's non-empty box
 * keys (uint64, level keys, ascending; *n_boxes of them) and its
 * multipole-to-local (V list) pairs as (destination, source) indices into
 * those keys (int32, *n_pairs each; grouped by translation vector); at the
 * leaf level also the near-field (U) lists, CSR over the leaves (u_ptr:
 * *n_boxes + 1 int32, u_idx: *n_u int32 leaf indices).  Device buffers
 * (any may be NULL: sizes only); the sizes go to the host integers (any may
 * be NULL).  Level outside 2 .. leaf level: BEM_E_INVALID; a plan without a
 * far field (direct sum) has no V pairs.  Synchronises the stream. */
int bem_lists_export(bem_plan* plan, int prob, int level, void* box_keys, void* v_dst,
                     void* v_src, void* u_ptr, void* u_idx, int64_t* n_boxes,
                     int64_t* n_pairs, int64_t* n_u, void* stream);

/* Near-field pairs of problem `prob` (the pairs whose rule-point integrals
 * are replaced by accurate ones, Sec. 2.3 discretisation): CSR by target in
 * sorted element order (bem_tree_export's perm maps a sorted index to the
 * caller's), ptr: n + 1 int32, col: *n_near int32 source indices (sorted
 * order).  Device buffers (either may be NULL: size only); *n_near on the
 * host (may be NULL).  Synchronises the stream. */
int bem_near_export(bem_plan* plan, int prob, void* ptr, void* col, int64_t* n_near,
                    void* stream);

/* Overrides the choices made by timing at plan creation for problem `prob`
 * and precision prec (BEM_C128 / BEM_C64), see bem_plan_stats: stream
 * schedule (0..5), near-field and leaf-level M2L grids (0: one workgroup per
 * leaf / tile, else a grid-stride launch of that many) and direct
 * translation depth (0 .. the depth built).  A negative value keeps the
 * current choice.  Products agree up to rounding whatever the choice.
 * BEM_E_INVALID for a bad index, precision or value. */
int bem_plan_set_tuning(bem_plan* plan, int prob, int prec, int schedule, int p2p_grid,
                        int m2l_grid, int direct_depth);

/* Stage timing with HIP events recorded on the call's stream.  After
 * bem_profile_start, every product records an event pair around each stage;
 * bem_profile_stop synchronises and returns, per slot, the summed
 * milliseconds and the number of timed stage executions.  Slot =
 * stage + 16 * (float32 ? 1 : 0) + 32 * (adjoint ? 1 : 0), stage: 0 gather,
 * 1 P2P (with the near-field corrections), 2 P2M (adjoint: L2P^H), 3 M2M,
 * 4 M2L of the levels above the leaves, 5 L2L, 6 leaf finish (sums of the
 * leaf-level M2L, L2P, P2P sums, diagonal, scatter), 7 reduction of 4,
 * 8 M2L of the leaf level, 9 unused (the reduction of 8 is part of 6).
 * ms and calls hold BEM_PROFILE_SLOTS entries (host).
 * bem_profile_leaf_m2l_start times only stage 8, with timing events attached
 * to its launches (nothing is recorded on any stream between kernels), so a
 * timed region keeps its schedule; bem_profile_stop ends either mode.
 * BEM_E_INVALID for a bad plan, problem or output pointer. */
#define BEM_PROFILE_SLOTS 64
int bem_profile_start(bem_plan* plan, int prob);
/* As bem_profile_start, but the products then run every stage on the
 * call's stream one after another (no side streams), so each stage is timed
 * alone on the GPU; products keep their values.  Ended by bem_profile_stop. */
int bem_profile_serial_start(bem_plan* plan, int prob);
int bem_profile_leaf_m2l_start(bem_plan* plan, int prob);
int bem_profile_stop(bem_plan* plan, int prob, double* ms, int32_t* calls);

/* BEM-FEM coupled operator of an elastic scatterer (Sec. 2.3: the weak form
 * of the body, Eq. fem_2, with linear tetrahedra; the coupled system,
 * Eq. renritupu; its Schur form, Eqs. kousokuu and GMRES).  The body is a
 * tetrahedral mesh (nodes: host, n_nodes x 3; tets: host, n_tets x 4 node
 * indices) whose boundary faces are the problem's triangles: tri (host,
 * n_tri x 3, the problem's element order) gives their node indices, normals
 * (v1 - v0) x (v2 - v0) pointing into the fluid.  Isotropic material lambda,
 * mu (mu > 0, 3 lambda + 2 mu > 0), density rho_s; fluid density rho_f;
 * angular frequency omega (> 0; the problem's k = omega / c_f).  At creation
 * the device assembles K - omega^2 M densely (3 n_nodes <= BEM_FEM_MAX_DOF
 * unknowns), solves it against the boundary load N by a blocked LU with
 * partial pivoting (in place of the paper's multi-frontal factorisation)
 * and keeps C = -rho_f omega^2 Tc (K - omega^2 M)^-1 N
 * (n_tri x n_tri, float64, row-major, the problem's element order): q = C p
 * is dp/dn on the fluid side for the boundary pressure p (momentum balance
 * dp/dn = rho_f omega^2 u.n at the collocation points), and its transpose
 * for the adjoint (2 n_tri^2 doubles of device memory while the coupling
 * lives; the factorisation's workspace, 8 (3 n_nodes) (3 n_nodes + n_tri)
 * bytes, only during creation).  The coupling keeps a pointer to its plan's
 * problem: destroy it before the plan.  Products and solves on one coupling
 * share a work vector, so calls on different streams must not overlap.
 * BEM_E_INVALID for a bad plan, problem (more than 65535 triangles),
 * material or size, or a mesh with
 * an index out of range, a tetrahedron of zero volume or a boundary
 * triangle of zero area; BEM_E_NAN
 * when K - omega^2 M is singular to working precision (omega^2 an eigenvalue
 * of the free body: C comes out non-finite; near such a frequency C is
 * large but finite and is kept). */
#define BEM_FEM_MAX_DOF 24576
typedef struct bem_coupling bem_coupling;
int bem_coupling_create(bem_plan* plan, int prob, const double* nodes, int64_t n_nodes,
                        const int32_t* tets, int64_t n_tets, const int32_t* tri, double lambda,
                        double mu, double rho_s, double rho_f, double omega, void* stream,
                        bem_coupling** out);
int bem_coupling_destroy(bem_coupling* c);
/* C copied into C_out (device, n_tri x n_tri float64). */
int bem_coupling_get_matrix(const bem_coupling* c, void* C_out, void* stream);
/* out = C v (transpose != 0: C^T v), v and out device complex128 of n_tri:
 * the body's response alone (dp/dn for the boundary pressure v, Eq.
 * kousokuu), e.g. to recover the normal derivative after a coupled solve.
 * BEM_E_INVALID for a null pointer or out == v. */
int bem_coupling_apply(const bem_coupling* c, int transpose, const void* v, void* out,
                       void* stream);
/* y = (I/2 - K - alpha H) p + (S + alpha K' + alpha/2 I) C p: the coupled
 * operator (alpha = 0: the paper's Eq. GMRES), float64 (BEM_C128) or the
 * float32 far field (BEM_C64) as bem_fmm_matvec; p, y device complex128. */
int bem_coupled_matvec(bem_coupling* c, int prec, const void* p, void* y, void* stream);
/* GMRES on the coupled operator (adjoint != 0: on its conjugate transpose,
 * the adjoint problem of Sec. 2.2 solved the same way), options and status
 * as bem_gmres_solve. */
int bem_coupled_solve(bem_coupling* c, int adjoint, const void* b, void* x,
                      const bem_gmres_opts* opts, bem_gmres_info* info, void* stream);

const char* bem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BEMFMM_H */
