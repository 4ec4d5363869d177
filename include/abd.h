/*
 * abd.h - C ABI of the MI355X (gfx950) affine-body-dynamics contact path.
 *
 * Method: Lan, Kaufman, Li, Jiang, Yang, "Affine Body Dynamics: Fast, Stable
 * and Intersection-free Simulation of Stiff Materials" (ABD).  Every stiff
 * body carries 12 affine DOFs q = (p, a1, a2, a3) with a_i the rows of A
 * (sec. 3); its surface vertices move as x = A xbar + p (Eq. kinematic).
 * One Newton iteration of the incremental potential (sec. 4) evaluates the
 * orthogonality potential (Eq. orthogonality), the clamped log barrier on
 * point-triangle (PT) and edge-edge (EE) pairs of different bodies
 * (Eq. barrier, Eq. clamped-b), culled by box overlap (sec. 4.2), assembles
 * J^T H J into 12x12 body blocks (sec. 4.3), solves, and limits the step by
 * linear CCD (sec. 4.1).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers (caller-owned, contiguous, row-major
 *    as documented) unless marked "host".  The library never frees them.
 *  - Calls are enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and return after enqueueing, except calls documented as "syncs": those
 *    need a count or scalar on the host and synchronise `stream` first.
 *  - "accumulated" outputs are added to (callers zero them first).
 *  - Return value: ABD_OK or a negative ABD_E_* code; abd_last_error gives
 *    the message.  No exception crosses the ABI.  One context per host
 *    thread; calls on one context are not thread-safe.
 *  - The library allocates only its own workspace (inside the context,
 *    grown on demand, released by abd_destroy).
 */
#ifndef ABD_H
#define ABD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ABD_OK = 0,
  ABD_E_INVALID = -1,        /* null pointer, bad size, bad index, non-finite input */
  ABD_E_CAPACITY = -2,       /* output capacity too small; required count returned */
  ABD_E_INTERSECT = -3,      /* a pair at zero distance (intersecting input) */
  ABD_E_NOT_CONVERGED = -4,  /* Newton iteration cap reached */
  ABD_E_LINESEARCH = -5,     /* no energy decrease after max_ls halvings */
  ABD_E_PCG = -6,            /* PCG breakdown (non-positive curvature) or cap */
  ABD_E_HIP = -7             /* HIP runtime error */
};

/* Distance case codes written by abd_classify (vertex slots: PT pair =
 * (p, t0, t1, t2), EE pair = (a0, a1, b0, b1)).
 *   PT: 0,1,2 point-point with t0,t1,t2; 3 point-edge (t0,t1);
 *       4 point-edge (t1,t2); 5 point-edge (t0,t2); 6 point-face.
 *   EE: 16 + 3k + c for the endpoint-vs-segment side k (0: a0 vs b,
 *       1: a1 vs b, 2: b0 vs a, 3: b1 vs a) with c = 0/1 the segment's
 *       first/second endpoint, c = 2 its interior; 28 line-line.      */

typedef struct abd_ctx abd_ctx;

/* Scene geometry (device arrays; counts are host values).  Bodies are
 * contiguous ranges of vertices, triangles and edges.  Vertex, triangle and
 * edge indices are global.  Sub-scenes (batched mode) are contiguous body
 * ranges; pairs never cross sub-scenes.  A context keeps tables derived
 * from body_scene (and from the joint arrays) between calls, keyed by the
 * array's address and the counts: their contents must not change while a
 * context uses the scene. */
typedef struct abd_scene {
  int32_t n_bodies, n_verts, n_tris, n_edges, n_scenes;
  const double *xbar;           /* [n_verts][3] body-frame rest positions */
  const int32_t *vert_body;     /* [n_verts] */
  const int32_t *tris;          /* [n_tris][3] */
  const int32_t *tri_body;      /* [n_tris] */
  const int32_t *edges;         /* [n_edges][2], first < second */
  const int32_t *edge_body;     /* [n_edges] */
  const int32_t *body_vert_off; /* [n_bodies+1] */
  const int32_t *body_tri_off;  /* [n_bodies+1] */
  const int32_t *body_edge_off; /* [n_bodies+1] */
  const uint8_t *body_fixed;    /* [n_bodies], 1 = Dirichlet (never moves) */
  const int32_t *body_scene;    /* [n_bodies] sub-scene id, non-decreasing */
  const double *mass;           /* [n_bodies][10] from abd_body_mass (may be NULL
                                   for calls that do not use it) */
  const double *volume;         /* [n_bodies] from abd_body_mass */
  /* Joints (sec. 5.3: q maps linearly to a virtual tetrahedron's vertices,
   * which are material points, so fixing them is a linear equality):
   * joint j makes body a's body-frame point coincide with body b's point
   * (b = -1: with a fixed world point), enforced by the penalty
   * dt^2 kappa_j / 2 |x_a - x_b|^2 in the incremental potential.  A hinge
   * is two joints on its axis.  a and b in one sub-scene.  The arrays are
   * read once per context and scene (they must not change while used). */
  int32_t n_joints;
  const int32_t *joint_body;    /* [n_joints][2] (a, b) */
  const double *joint_point;    /* [n_joints][2][3] point of a; of b (world point when b = -1) */
} abd_scene;

/* Method parameters (host struct). */
typedef struct abd_params {
  double dt;          /* time step */
  double dhat;        /* barrier activation distance (Eq. clamped-b) */
  double kappa_b;     /* barrier stiffness (Eq. barrier) */
  double kappa_o;     /* orthogonality stiffness, times body volume (Eq. orthogonality) */
  double mu, eps_v;   /* friction coefficient and static-velocity threshold */
  double gravity[3];
  double newton_tol;  /* converged when max_k |J_k p|_inf <= newton_tol * dt */
  double pcg_rtol;    /* PCG stop: |r| <= pcg_rtol |b| */
  double ccd_s;       /* ACCD gap fraction s */
  double ccd_tmax;    /* ACCD maximal step fraction */
  int32_t ccd_max_iter, max_newton, max_pcg, max_ls;
  /* the body's rigidity potential, times kappa_o, the body volume and the
   * weight (dt^2 in the incremental potential): 0 the orthogonality
   * potential V_perp (Eq. ortho-energy, the paper's choice); 1 ARAP,
   * |A - R(A)|_F^2 with R the polar rotation; 2 neo-Hookean with
   * mu = lambda = 1, 1/2 (|A|_F^2 - 3) - ln J + 1/2 (ln J)^2, J = det A
   * (infinite for J <= 0) -- the alternatives sec. 3.2 names */
  int32_t rigidity;
  double kappa_j;     /* joint penalty stiffness (N/m; used when the scene has joints) */
  /* Adaptive barrier stiffness (IPC's rule; the paper's kappa of sec. 4,
   * Eq. barrier, has no value): 0 keeps kappa_b fixed; 1 makes abd_time_step
   * set, per scene at q^t, kappa = clamp(-(g_E . g_B) / |g_B|^2, kappa_b,
   * kappa_max) (g_B the barrier gradient at kappa = 1, g_E that of inertia,
   * rigidity potential and joints, over the free DOFs; kappa_b when
   * g_B = 0), and double it (up to kappa_max) before a Newton iteration
   * whose closest active pair is nearer than kappa_eps_d and nearer than at
   * the iteration before.  abd_newton_step and the adjoint entry points
   * reject 1 (ABD_E_INVALID). */
  int32_t kappa_adaptive;
  double kappa_max;
  double kappa_eps_d;  /* m */
} abd_params;

/* Per-iteration statistics (host struct). */
typedef struct abd_stats {
  int64_t n_pt, n_ee;             /* pairs tested for activity at the current
                                     iterate: the last accepted step's swept
                                     candidates, else the candidates at it */
  int64_t n_active_pt, n_active_ee;
  int64_t n_pt_swept, n_ee_swept; /* candidates over the step's sweep */
  int64_t n_offdiag;              /* off-diagonal blocks of the system */
  int32_t pcg_iters, ls_halvings, converged, newton_iters;
  double alpha_ccd, alpha;        /* CCD bound and accepted step */
  double disp;                    /* max_k |J_k p|_inf of the Newton direction */
  double energy0, energy1;        /* E(q), E(q + alpha p) */
  double t_barrier_ms, t_ccd_ms, t_candidates_ms, t_solve_ms, t_total_ms;
  int64_t n_friction;             /* lagged friction pairs in use */
  int64_t scene_newton_iters;     /* time step: Newton iterations summed over sub-scenes */
  int32_t newly_converged;        /* sub-scenes that converged in this iteration */
  int32_t pad_;
} abd_stats;

int abd_create(abd_ctx **ctx, int device);
int abd_destroy(abd_ctx *ctx);
const char *abd_last_error(const abd_ctx *ctx);

/* Mass properties (sec. 3.1, Eq. mass: M = int rho J^T J).  For every free
 * body: mass[b] = (m, h_x, h_y, h_z, S_xx, S_xy, S_xz, S_yy, S_yz, S_zz) with
 * m = int rho, h = int rho xbar, S = int rho xbar xbar^T over the closed,
 * outward-oriented surface (divergence theorem), and volume[b]; zeros for
 * fixed bodies.  density: [n_bodies]. */
int abd_body_mass(abd_ctx *ctx, const abd_scene *sc, const double *density, double *mass, double *volume,
                  hipStream_t stream);

/* Kinematic map (sec. 3, Eq. kinematic): x_k = A_b xbar_k + p_b for every
 * vertex, component i evaluated as p_i + ((a_i0 xbar_0 + a_i1 xbar_1) +
 * a_i2 xbar_2) without fused multiply-add, so results are bit-reproducible.
 * q: [n_bodies][12]; x: [n_verts][3]. */
int abd_vertex_map(abd_ctx *ctx, const abd_scene *sc, const double *q, double *x, hipStream_t stream);

/* Candidate pairs (sec. 4.2).  A primitive's box spans its vertices at x0
 * and x1 (x1 = NULL: x0 only); a pair is a candidate iff the primitives lie
 * on different bodies of one sub-scene, not both fixed, and on every axis
 * lo_a <= hi_b + inflate and lo_b <= hi_a + inflate.  Whole-body boxes and
 * their pairwise intersections (i-AABBs) cull exactly for this predicate.
 * Output: pt [cap_pt][2] = (vertex, triangle) of either body against the
 * other; ee [cap_ee][2] = (edge_lo, edge_hi).  Order: grouped by body pair
 * (min body, max body) ascending; inside a group PT pairs by (vertex,
 * triangle) and EE pairs by (edge_lo, edge_hi) ascending.  Syncs; *n_pt and
 * *n_ee (host) receive the counts; ABD_E_CAPACITY if either exceeds its
 * capacity (outputs then undefined, counts valid). */
int abd_candidates(abd_ctx *ctx, const abd_scene *sc, const double *x0, const double *x1, double inflate,
                   int32_t *pt, int64_t cap_pt, int64_t *n_pt, int32_t *ee, int64_t cap_ee, int64_t *n_ee,
                   hipStream_t stream);

/* Candidates at x (x1 = NULL, same inflate) taken from the swept
 * candidates (spt, see) of a segment x0 -> x1 that contains x (x a convex
 * combination of x0 and x1 vertex by vertex, as every Newton iterate on
 * the search line is): each static box lies in the swept box, so the
 * result is the swept list filtered by the same box test, in the same
 * canonical order, equal to abd_candidates at x.  (A vertex of x computed
 * from an intermediate q may round outside the swept box by an ulp; a pair
 * whose static boxes touch only within that rounding can then be missing:
 * its primitives are dhat apart up to rounding, so its barrier is zero.)
 * Syncs; counts and ABD_E_CAPACITY as abd_candidates. */
int abd_candidates_within(abd_ctx *ctx, const abd_scene *sc, const double *x, double inflate, const int32_t *spt,
                          int64_t n_spt, const int32_t *see, int64_t n_see, int32_t *pt, int64_t cap_pt,
                          int64_t *n_pt, int32_t *ee, int64_t cap_ee, int64_t *n_ee, hipStream_t stream);

/* Off-diagonal block pattern of the global Hessian (sec. 4.3): sorted unique
 * body pairs (a < b, both free) touched by the given pairs and by the
 * scene's joints between two bodies.  keys: [cap][2].  Syncs; *n_keys (host)
 * receives the count (ABD_E_CAPACITY when it exceeds cap). */
int abd_offdiag_pattern(abd_ctx *ctx, const abd_scene *sc, const int32_t *pt, int64_t n_pt, const int32_t *ee,
                        int64_t n_ee, int32_t *keys, int64_t cap, int64_t *n_keys, hipStream_t stream);

/* Narrow phase (sec. 4, distances of Eq. barrier): per pair the distance
 * case (codes above), the squared distance num/den of that case, and
 * active = (num < dhat^2 den), i.e. d < dhat decided without division.
 * is_ee selects the pair kind.  Outputs [n]; any may be NULL. */
int abd_classify(abd_ctx *ctx, const abd_scene *sc, const double *x, double dhat, const int32_t *pairs, int64_t n,
                 int is_ee, uint8_t *type, double *d2, uint8_t *active, hipStream_t stream);

/* Barrier term (Eq. barrier, Eq. clamped-b; EE pairs mollified by
 * m(c) = (2 - c/eps) c/eps, c = |(a1-a0)x(b1-b0)|^2, eps = 1e-3 |abar|^2
 * |bbar|^2): energy kappa_b sum m B(d); per active pair the local 12x12
 * Hessian, PSD-projected when project_psd != 0; J^T g and J^T H J reduced
 * into grad [n_bodies][12], diag [n_bodies][144] and off [n_keys][144]
 * (block (a,b) of keys[k] = (a,b), row-major 12x12, rows = DOFs of a).
 * energy [1], grad, diag, off are accumulated; diag/off may be NULL
 * (gradient only).  Contributions to fixed bodies are dropped.  Any pair
 * order is accepted.  ABD_E_INTERSECT is raised asynchronously: it is
 * reported by the next syncing call. */
int abd_barrier_grad_hess(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x,
                          const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, const int32_t *keys,
                          int64_t n_keys, double *energy, double *grad, double *diag, double *off, int project_psd,
                          hipStream_t stream);

/* Barrier energy only (line search): accumulates kappa_b sum m B(d) into
 * energy [1]; +inf when a pair is at zero distance. */
int abd_barrier_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt,
                       int64_t n_pt, const int32_t *ee, int64_t n_ee, double *energy, hipStream_t stream);

/* Barrier energy only, allocating nothing: for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same kernels, same summation
 * order and same result as abd_barrier_energy (accumulates into energy [1]),
 * but its scratch (per-pair energies and the reduction's partials) is a
 * fixed array in the library, one per GPU, held until the process ends:
 * n_pt + n_ee <= ABD_NOALLOC_MAX_PAIRS, else ABD_E_CAPACITY and nothing is
 * launched.  Calls on one GPU share that array, so calls that overlap on
 * one GPU (different streams or threads) race; serialise them.  Calls no
 * hipMalloc, hipFree or allocating library routine, and records no
 * profiling events. */
#define ABD_NOALLOC_MAX_PAIRS (1 << 20)
int abd_barrier_energy_noalloc(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x,
                               const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *energy,
                               hipStream_t stream);

/* CCD step bound (sec. 4.1: linear trajectories x0 + t dx, additive CCD):
 * per pair a conservative safe fraction t in [0, ccd_tmax] (t_pt [n_pt],
 * t_ee [n_ee], either may be NULL) and alpha [n_scenes] = min(1, min t)
 * over each sub-scene's pairs.  (Environment ABD_CCD_MAX_BLOCKS caps the
 * kernel's grid; the results do not depend on it.) */
int abd_ccd_max_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x0, const double *dx,
                     const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *t_pt, double *t_ee,
                     double *alpha, hipStream_t stream);

/* Orthogonality potential (Eq. orthogonality / ortho-energy / ortho-poly),
 * or the alternative rigidity potential prm->rigidity selects (ARAP or
 * neo-Hookean, sec. 3.2), scaled by `weight` (dt^2 inside the incremental
 * potential): energy [1], grad [n_bodies][12], diag [n_bodies][144]
 * accumulated; the 9x9 A-block of the Hessian PSD-projected when
 * project_psd != 0.  grad and diag may both be NULL (energy only).  Fixed
 * bodies skipped. */
int abd_orthogonality(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, double weight,
                      double *energy, double *grad, double *diag, int project_psd, hipStream_t stream);

/* Inertia term of the incremental potential (sec. 4): energy 1/2 |q - q~|_M^2,
 * gradient M (q - q~), Hessian M, accumulated; fixed bodies skipped. */
int abd_inertia(abd_ctx *ctx, const abd_scene *sc, const double *q, const double *q_tilde, double *energy,
                double *grad, double *diag, hipStream_t stream);

/* q~ = q + dt qdot + dt^2 M^-1 f with gravity (M^-1 f = (g, 0, 0, 0));
 * fixed bodies: q~ = q. */
int abd_q_tilde(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *qdot,
                double *q_tilde, hipStream_t stream);

/* Block-Jacobi preconditioned CG on the symmetric block matrix (diag +
 * off/off^T) restricted to free bodies: solves H p = rhs, p = 0 on fixed
 * bodies.  Sub-scenes are independent systems (no off-diagonal block joins
 * two of them): each runs its own CG scalars and stops on its own
 * |r| <= rtol |b|.  The iterations run in Chronopoulos-Gear form (one
 * kernel per iteration); the result is then checked on a freshly computed
 * residual b - H p, and a sub-scene that fails the check continues in the
 * classical form (environment ABD_PCG_CG=0: classical form only).
 * x0 (may be NULL = zero, may alias p): initial guess.  Syncs; *iters
 * (host) receives the largest iteration count over the sub-scenes (both
 * forms counted).  Error ABD_E_PCG: a diagonal block not positive definite
 * or a non-positive curvature in the classical form. */
int abd_pcg_solve(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off, const int32_t *keys,
                  int64_t n_keys, const double *rhs, const double *x0, double *p, double rtol, int32_t max_iter,
                  int32_t *iters, hipStream_t stream);

/* One projected-Newton iteration on q (in/out) towards the minimiser of
 * the incremental potential with target q_tilde: direction p = -H^-1 g;
 * a sub-scene with max_k |J_k p|_inf <= newton_tol dt (vertices of the
 * scene) is converged and keeps its q; every other sub-scene takes the CCD
 * bound over the swept candidates of x(q) -> x(q+p) as its first step
 * length and halves it until its energy E_s(q + alpha_s p) <= E_s(q).
 * Sub-scenes are independent problems: own convergence test, CCD bound,
 * line search and PCG scalars.  scene_done (device u8 [n_scenes], in/out,
 * may be NULL = none done): scenes marked non-zero are skipped (zero
 * direction, q unchanged); scenes converging in this call are marked.
 * stats->converged is set when every sub-scene is done.  Syncs.  stats
 * (host) may be NULL. */
int abd_newton_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q, const double *q_tilde,
                    uint8_t *scene_done, abd_stats *stats, hipStream_t stream);

/* One implicit-Euler time step: q~ from (q, qdot), Newton iterations until
 * every sub-scene has converged (ABD_E_NOT_CONVERGED after max_newton), then
 * qdot = (q_new - q_old) / dt.  q, qdot [n_bodies][12] in/out.  Syncs.
 * stats (host, may be NULL) receives totals of the step (newton_iters: the
 * iterations of the slowest sub-scene; scene_newton_iters: summed over
 * sub-scenes). */
int abd_time_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q, double *qdot,
                  abd_stats *stats, hipStream_t stream);

/* Reverse mode of one time step (the differentiability claimed in the
 * conclusion, sec. 6; implicit function theorem on the optimality condition
 * grad_q E(q^{t+1}; q~, q^t) = 0).  Given the forward step's start (q_t,
 * qdot_t) and result q_next, and the loss gradients qbar_next, qdbar_next
 * with respect to (q^{t+1}, qdot^{t+1}): solves H l = qbar_next +
 * qdbar_next/dt with H the unprojected Hessian of the incremental potential
 * at q_next (barrier, orthogonality, inertia and, when mu > 0, the friction
 * lagged at q_t; it may be indefinite), to relative residual rtol, with
 * the diagonal blocks of the projected Hessian as block-Jacobi
 * preconditioner: first by preconditioned conjugate gradients (as
 * abd_pcg_solve); if CG meets non-positive curvature or reaches its
 * iteration cap, again by MINRES (residual in the preconditioner's norm),
 * which needs symmetry only (environment ABD_ADJ_MINRES=1: MINRES alone).  Then it writes
 * qbar_t = M l + H_D l - C_lag^T l - qdbar_next/dt and qdbar_t = dt M l
 * (H_D the friction Hessian; C_lag the derivative of the friction gradient
 * through the lagged normal force, tangent basis and closest-point weights,
 * which are functions of q_t).  Zero on fixed bodies.  All arrays
 * [n_bodies][12]; outputs must not alias inputs.  Syncs; *pcg_iters (host,
 * may be NULL) receives the iteration count: CG's, plus MINRES's when CG
 * failed. */
int abd_adjoint_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q_t,
                     const double *qdot_t, const double *q_next, const double *qbar_next, const double *qdbar_next,
                     double rtol, double *qbar_t, double *qdbar_t, int32_t *pcg_iters, hipStream_t stream);

/* n_steps time steps from (q, qdot) (device [n_bodies][12], in/out),
 * keeping (q, qdot) before every checkpoint_every-th step, and after the
 * last step, in checkpoints (device, caller-owned,
 * [ceil(n_steps / checkpoint_every) + 1][2][n_bodies][12], may be NULL) for
 * abd_rollout_backward.  *newton_iters (host, may be NULL)
 * receives the Newton iterations summed over the steps.  Syncs. */
int abd_rollout_forward(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q, double *qdot,
                        int32_t n_steps, int32_t checkpoint_every, double *checkpoints, int64_t *newton_iters,
                        hipStream_t stream);

/* Gradient of a loss of the state after n_steps time steps from (q0, qdot0):
 * given qbar_T, qdbar_T (the loss gradient with respect to q^n and qdot^n),
 * writes qbar_0, qdbar_0.  The states every checkpoint_every steps come
 * from checkpoints (as written by abd_rollout_forward with the same
 * arguments) or, when it is NULL, from running the forward steps again
 * (context workspace); then per segment, last first, the segment's steps
 * are re-run (not with checkpoint_every = 1: every state is kept) and
 * abd_adjoint_step is applied backwards.  Syncs. */
int abd_rollout_backward(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q0,
                         const double *qdot0, int32_t n_steps, int32_t checkpoint_every, const double *checkpoints,
                         const double *qbar_T, const double *qdbar_T, double rtol, double *qbar_0, double *qdbar_0,
                         hipStream_t stream);

/* Lagged friction (sec. 4, friction potential V_F = sum of mu lambda f0 over
 * the active contact pairs; lagging as in IPC): quantities held fixed over a
 * time step are taken at the step-start positions xt.
 *
 * abd_friction_lag: for each pair (PT pairs then EE pairs, one combined
 * index i in [0, n_pt + n_ee)) at positions xt: lambda [n] = kappa_b m |B'(d)|
 * (m the EE mollifier of abd_barrier_grad_hess; 0 for inactive pairs, i.e.
 * d >= dhat, whose T and w are zero), the closest-point weights w [n][4]
 * over the pair's vertex slots (r = sum_k w_k x_k is the closest-point
 * difference; w = (1, -1) on the two closest vertices for point-point
 * cases, (1, -(1-t), -t) for a point against an edge, (1, -b0, -b1, -b2)
 * with barycentric b for point-face, (1-s, s, -(1-t), -t) for line-line) and
 * the tangent basis T [n][6] = (t1, t2): with n = r/|r| and e_a the
 * coordinate axis of smallest |n_a| (first on ties), t1 = n x e_a normalised,
 * t2 = n x t1. */
int abd_friction_lag(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *xt,
                     const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *lam, double *T,
                     double *w, hipStream_t stream);

/* Friction energy, gradient and Hessian at x of lagged pairs (arrays as
 * written by abd_friction_lag at xt; pairs with lambda <= 0 contribute
 * nothing): u = T^T sum_k w_k (x_k - xt_k), energy mu lambda f0(|u|) with
 * f0(y) = -y^3/(3 eps^2) + y^2/eps + eps/3 for y < eps = eps_v dt, else y;
 * local gradient and Hessian (exact, PSD) mapped by J^T . J and accumulated
 * like abd_barrier_grad_hess (energy [1] may be NULL; diag/off may be NULL;
 * keys must cover the pairs' body pairs). */
int abd_friction_grad_hess(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x,
                           const double *xt, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
                           const double *lam, const double *T, const double *w, const int32_t *keys, int64_t n_keys,
                           double *energy, double *grad, double *diag, double *off, hipStream_t stream);

/* Friction energy only (line search), accumulated into energy [1]. */
int abd_friction_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const double *xt,
                        const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, const double *lam,
                        const double *T, const double *w, double *energy, hipStream_t stream);

/* Friction state of a time step, held by the context: begin_step lags the
 * active pairs at x(q) (candidates within dhat, lambda > 0 kept, in
 * candidate order) and makes every later abd_newton_step include their
 * friction potential (when prm->mu > 0) and their body pairs in the
 * off-diagonal pattern, until end_step.  abd_time_step begins (when
 * mu > 0) and ends its own state.  begin_step syncs; *n_pairs (host, may be
 * NULL) receives the number of lagged pairs. */
int abd_friction_begin_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                            int64_t *n_pairs, hipStream_t stream);
int abd_friction_end_step(abd_ctx *ctx);

/* The per-scene barrier stiffness of the last adaptive time step on this
 * context (its final value), copied to kappa_out [n_scenes] (host).  Syncs;
 * ABD_E_INVALID when no adaptive step has run. */
int abd_barrier_stiffness(abd_ctx *ctx, const abd_scene *sc, double *kappa_out);

/* Launch shapes of the hot kernels (the autotuner's table).  No entry
 * changes a result: every kernel computes the same values and lists pairs
 * in the same order for any table.  Defaults {16, 1, 256, 1024, 256, 16, 64, 1}.
 *   tile_rows       rows per pair-culling tile (one wave): 8, 16, 32, 64
 *   barrier_waves   waves per block of the barrier kernel: 1, 2, 4
 *   ccd_block       threads per block of the CCD kernel: 64, 128, 256
 *   ccd_max_blocks  grid cap of the persistent CCD kernel: 64 .. 16384
 *   energy_block    threads per block of the energy-only kernel: 64 .. 1024 (powers of 2)
 *   pcg_short, pcg_long  shortest and longest PCG graph replay
 *                   (iterations; replays are powers of two between them,
 *                   chosen per solve to cover the last solve's count):
 *                   even, 2 <= pcg_short <= pcg_long <= 256
 *   cull_levels     i-AABB culling (sec. 4.2, Fig. iBVH): 1, the single
 *                   i-AABB per overlapping body pair; 3, inside each
 *                   i-AABB, three-level binary AABB trees over the culled
 *                   column primitives (blocks of 256 in index order, their
 *                   128-halves, their 64-chunks), which each tile of rows
 *                   descends with its own box, testing only the chunks it
 *                   reaches.  Both give the same candidate pairs in the
 *                   same order. */
typedef struct {
  int32_t tile_rows, barrier_waves, ccd_block, ccd_max_blocks, energy_block, pcg_short, pcg_long;
  int32_t cull_levels;
} abd_tune;

/* The context's launch-shape table: get, or set (ABD_E_INVALID for a value
 * outside the sets above; the table is then unchanged). */
int abd_tune_get(const abd_ctx *ctx, abd_tune *out);
int abd_tune_set(abd_ctx *ctx, const abd_tune *in);

/* Autotuner over the table above on the caller's workload: coordinate
 * descent, one entry at a time in the order of the struct, keeping for each
 * the value (among a fixed candidate set) whose n_steps time steps from the
 * start state (q, qdot [n_bodies][12], device; restored before every trial
 * run and on return) take the least host wall time between stream
 * synchronisations, best of `reps` runs; an entry changes only when a
 * candidate is faster by more than 1 %.  Leaves the picked table set in ctx
 * and copies it to *out (host); *best_ms_per_step (host, may be NULL) gets
 * its time per step.  Syncs.  Errors of the time steps are returned. */
int abd_autotune(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q, double *qdot, int n_steps,
                 int reps, abd_tune *out, double *best_ms_per_step, hipStream_t stream);

/* Kernel timing with HIP events on the calls' streams, for measurement:
 * abd_profile(enable, reset) switches recording on/off (reset clears the
 * totals); abd_profile_query returns, for one instrumented kernel
 * ("barrier_local", "friction_local", "assemble_chunks", "energy_only", "accd",
 * "pair_tiles_write", "pcg_round"), the summed duration in ms, the number of
 * launches and the work units processed (active pairs, records, pairs,
 * pairs, tiles; friction pairs for "friction_local"; for "pcg_round", one
 * replay of the captured PCG iterations,
 * the algorithmic HBM bytes of the iterations it executed); and, with zero
 * time and only in mode 2 (enable = 2, which adds a reduction per candidate
 * search), "box_tests" / "box_tests_single_level": per candidate-search
 * call, the primitive-pair box tests run with the table's i-AABB culling,
 * and the tests a single-level cull would run.  Two host-side entries
 * count work done on the host inside calls, with host wall time in ms:
 * "ws_grow" (a workspace buffer grown: synchronise, free, allocate, clear;
 * units = bytes asked for) and "pcg_capture" (a PCG graph captured and
 * instantiated; units = iterations in it).
 * Query synchronises the device. */
int abd_profile(abd_ctx *ctx, int enable, int reset);
int abd_profile_query(abd_ctx *ctx, const char *kernel, double *ms, int64_t *launches, int64_t *units);

#ifdef __cplusplus
}
#endif
#endif /* ABD_H */
