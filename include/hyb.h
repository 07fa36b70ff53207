/*
 * hyb.h - C ABI of the MI355X hybridised trace solver.
 *
 * The library solves the hybridised velocity / Exner-pressure system of one
 * semi-implicit timestep of a compatible finite element dynamical core, the
 * method of Betteridge, Cotter, Gibson, Griffith, Melvin and Mueller,
 * "Hybridised multigrid preconditioners for a compatible finite element
 * dynamical core":
 *
 *   [ A    K ] [ X      ]   [ R_X ]      A = [[M2b - Q22b, Gb], [Q32b + M3rho M3^-1 Db, M3Pi]]
 *   [ C^T  0 ] [ lambda ] = [ 0   ]      (Sec. 2.4, hybridisable system and its block form)
 *
 * by static condensation S lambda = B_lambda with S = C^T A^-1 K and
 * B_lambda = C^T A^-1 R_X (Sec. 2.4, Eqs. of S and B_lambda), a flexible
 * GMRES solve of that trace system preconditioned by the non-nested
 * two-level cycle (Sec. 2.5, Alg. 2 with LineSmooth, Alg. 1, and a pressure
 * multigrid V-cycle on the approximate Schur complement H of Sec. 2.3), and
 * the cellwise recovery X = A^-1 (R_X - K lambda) (Sec. 2.4, Eq. of the
 * recovery).  Lowest order (p = 0): six outward-flux broken Raviart-Thomas
 * dofs and one Exner-pressure dof per cell, one trace dof per facet.
 *
 * Layout (every per-cell or per-facet array is structure-of-arrays):
 *   ncol columns, nlev layers; cell c = k * ncol + col (k = 0 at the ground).
 *   Local faces of a cell: 0 W, 1 E, 2 S, 3 N (vertical facets, the "edges"
 *   of the horizontal mesh), 4 B, 5 T (horizontal facets).
 *   Trace vector (ntrace = (nlev+1)*ncol + nlev*nedge entries): first the
 *   horizontal facets, index k*ncol + col for k = 0..nlev (the bottom of layer
 *   k), then the vertical facets, index (nlev+1)*ncol + k*nedge + e.
 *   Broken velocity arrays are [6][nlev][ncol]; cell arrays are [nlev][ncol];
 *   theta / projected Exner fields on the vertically continuous points are
 *   [nlev+1][ncol].
 *
 * Ownership: the caller allocates and frees every array it passes.  Mesh
 * tables are HOST pointers, copied at hyb_create.  All field and vector
 * arguments of the other calls are DEVICE pointers (FP64); the library keeps
 * its own workspace (cell factors, trace stencil, multigrid hierarchy,
 * Krylov basis), allocated by hyb_create / hyb_assemble_local / hyb_condense
 * and freed by hyb_destroy.  Calls enqueue work on the context's stream and
 * return without synchronising, except hyb_solve, which reads one small
 * vector back to the host per iteration for its stopping test (the step's
 * Gram-Schmidt coefficients, read while the GPU runs the step's update).
 *
 * Errors: every call returns HYB_OK (0) or a negative code; no exception or
 * abort crosses the ABI.  hyb_last_error gives the text of the last error of
 * a context.  One context per stream and host thread.
 */
#ifndef HYB_H
#define HYB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYB_OK 0
#define HYB_EINVAL (-1)        /* null pointer, bad size or parameter */
#define HYB_ESTATE (-2)        /* call out of order (e.g. solve before condense) */
#define HYB_EHIP (-3)          /* HIP runtime error; text in hyb_last_error */
#define HYB_ENOMEM (-4)        /* device allocation failed */
#define HYB_NOT_CONVERGED 1    /* hyb_solve: maxit reached above rtol */
#define HYB_BREAKDOWN 2        /* hyb_solve: NaN/Inf or a zero Arnoldi vector before convergence */
#define HYB_STAGNATED 3        /* hyb_solve: two restart cycles in a row each left more than 99.9 %
                                  of the true residual (e.g. a tolerance below its rounding floor) */

#define HYB_PREC_FP64 0        /* every step in FP64 */
#define HYB_PREC_MIXED 1       /* FP32 preconditioner and preconditioned basis, FP64 outer Krylov */
#define HYB_PREC_MFMA_FP32 2   /* order 1 only: S_K condensed on FP32 MFMA (FP32 accumulation) */
#define HYB_PREC_MFMA_BF16X 3  /* order 1 only: S_K condensed on BF16 MFMA, operands split hi + lo */

#define HYB_GEOM_BOX 0         /* periodic box of axis-aligned cells dx x dy x dz[k] */
#define HYB_GEOM_SHELL 1       /* extruded cubed sphere: curved cells between spheres (below) */

typedef struct hyb_ctx hyb_ctx;

/* Horizontal mesh of one multigrid level (host arrays). */
typedef struct {
  int32_t ncol;              /* columns */
  const int32_t *col_edge;   /* [4][ncol]: edge of local face f (0..3) of a column */
  const int32_t *edge_col;   /* [2][2*ncol]: column the edge normal leaves (0) / enters (1) */
  const int32_t *edge_lf;    /* [2][2*ncol]: local face index of the edge in those columns */
  const int32_t *parent;     /* [ncol of the next finer level]; NULL on level 0 */
} hyb_level;

/* Extruded mesh plus its 2x2-agglomerated multigrid levels (levels[0] = the mesh itself; each
   coarser level keeps the local face orientation of its children; no vertical coarsening).
   geom = HYB_GEOM_BOX: a periodic box, cells dx x dy x dz[k] (dz host [nlev]).
   geom = HYB_GEOM_SHELL (order 0 only): an extruded cubed sphere.  corners (host [4][3][ncol]) are
   the unit vectors of the column corners, corner q = I + 2 J at the column's local coordinates
   (I, J) in {0, 1}^2 (local faces W at I = 0, E at I = 1, S at J = 0, N at J = 1, the frame
   right-handed seen from outside); radius (host [nlev + 1]) the radii of the layer interfaces.
   A cell is the image of the unit cube under x = r(zeta) p / |p|, r(zeta) = radius[k] +
   zeta (radius[k+1] - radius[k]), p the bilinear interpolation of the corners: the vertical is
   radial, the side faces lie on great-circle planes.  dx, dy and dz are ignored.  hyb_create returns
   HYB_EINVAL for non-finite corners, radii that do not increase, order 1, or a column whose frame
   turns the other way ((c1 - c0) x (c2 - c0) pointing inwards). */
typedef struct {
  int32_t nlev;
  int32_t nlevels;           /* multigrid levels, >= 1 */
  const hyb_level *levels;   /* [nlevels] */
  double dx, dy;
  const double *dz;          /* host [nlev] */
  int32_t order;             /* 0: RT0 / Q0 / one trace dof per facet; 1: RT1 / DG1 / Q1 trace (below) */
  int32_t geom;              /* HYB_GEOM_BOX or HYB_GEOM_SHELL */
  const double *corners;     /* HYB_GEOM_SHELL: host [4][3][ncol] */
  const double *radius;      /* HYB_GEOM_SHELL: host [nlev + 1], increasing */
} hyb_mesh;

typedef struct {
  /* linearisation (Sec. 2.1): time step, off-centring weights, c_p, gas constant R */
  double dt, tau_u, tau_rho, tau_theta, cp, rd;
  /* LineSmooth / two-level cycle (Alg. 1 / Alg. 2): relaxation, pre and post sweeps */
  double omega;
  int32_t n_pre, n_post;
  /* pressure multigrid (Sec. 2.3): block-Jacobi relaxation, sweeps per level, coarsest sweeps */
  double omega_p;
  int32_t mg_pre, mg_post, mg_coarse_sweeps;
  /* flexible GMRES restart length and arithmetic of the preconditioner (HYB_PREC_*) */
  int32_t restart;
  int32_t precision;
  /* 1: hyb_solve and hyb_precondition append the learned coarse correction (hyb_nn_*) after every
     two-level cycle; learned_tau > 0: a correction d is kept only if ||r' - S d|| < learned_tau ||r'|| */
  int32_t learned;
  double learned_tau;
  /* coarsest multigrid level: 0 = mg_coarse_sweeps damped block-Jacobi sweeps (omega_p); 1 = the
     Chebyshev semi-iteration with mg_coarse_sweeps steps (one column solve each), preconditioned by
     the same column operator H_z and tuned to eigenvalues of H_z^-1 H in [cheb_lo, cheb_hi]
     (0 < cheb_lo < cheb_hi; eigenvalues stay below 2 when H has non-positive couplings and positive
     row sums, as the pressure operators here do) */
  int32_t mg_coarse_cheb;
  double cheb_lo, cheb_hi;
  /* rotation rate about the +z axis (1/s): the Coriolis term tau_u dt <w . 2 Omega x u> of the
     velocity mass form (Sec. 2.2), on HYB_GEOM_SHELL meshes (0 on the box); read at
     hyb_assemble_local.  The lumped velocity mass of the preconditioner leaves it out. */
  double omega_rot;
  /* coarse correction of the two-level cycle (Alg. 2): 0 = one pressure-multigrid V-cycle (the
     paper's Configuration 3c, the default); 1 = none: the preconditioner is n_pre + n_post
     LineSmooth sweeps from zero (Alg. 1 alone, the paper's hybridised single-level Configuration 2);
     2 = BiCGStab on the coarse pressure system, preconditioned by one V-cycle, from zero until the
     coarse residual drops by coarse_rtol (at most 200 steps; the paper's Configurations 3a with
     1e-14 and 3b with 1e-2; order 0 and HYB_PREC_FP64 only, HYB_EINVAL otherwise) */
  int32_t coarse_mode;
  double coarse_rtol;
  /* LineSmooth's column matrices S^zz (Alg. 1): 0 = each column's own (the default); 1 = cached
     per 2x2 patch of columns (the patches of the first multigrid coarsening; needs at least 2
     levels): every column of a patch uses the mean of the patch's S^zz, whose LU factors are kept
     once per patch (the future-work variant of Sec. 4.2; order 0 only, HYB_EINVAL otherwise) */
  int32_t smoother_patch;
  /* the network's training passes (hyb_nn_forward and the loss / gradient / train-step calls):
     0 = BF16 activations and backpropagated fields on BF16 matrix cores (16x16x32 products, FP32
     accumulation; the default); 1 = FP32 activations on the vector units, kept as a reference for
     the BF16 path.  The stage inside hyb_solve always runs the BF16 inference passes. */
  int32_t nn_fp32;
  /* switches for tests (0 in normal use): HYB_DEBUG_ZERO_GAMMA takes Gamma as zero, so the coarse
     correction of Alg. 2 adds nothing and the cycle is its LineSmooth sweeps alone;
     HYB_DEBUG_NAN_STAGE fills the learned stage's network output with NaN, so every correction
     falls back to the plain cycle; HYB_DEBUG_UNPAIRED_RESTRICT makes the multigrid restriction
     read every child through the children map even where the children of a coarse column come as
     two pairs of adjacent columns (the results are the same bits) */
  int32_t debug;
} hyb_params;

#define HYB_DEBUG_ZERO_GAMMA 1
#define HYB_DEBUG_NAN_STAGE 2
#define HYB_DEBUG_UNPAIRED_RESTRICT 4

typedef struct {
  int32_t iters;        /* FGMRES iterations (preconditioner applications) */
  int32_t status;       /* HYB_OK, HYB_NOT_CONVERGED, HYB_BREAKDOWN or HYB_STAGNATED */
  int32_t restarts;
  double rel_res;       /* true ||B - S lambda||_2 / ||B||_2 at exit, computed in FP64 */
  double *history;      /* optional host array: Arnoldi residual estimate per iteration */
  int32_t history_cap;
  int32_t history_len;
  int32_t fallbacks;    /* learned corrections dropped (output not finite, or rejected by the residual test) */
} hyb_info;

/* Order 1 (the paper's p = 1 row of its table of unknowns; Sec. 2.2 forms with n = 4 point Gauss
   rules and q32 / m3^rho / m3^Pi at the W3 nodes; Sec. 2.4 hybridisation): broken RT1 velocity, 36
   dofs per cell ordered as the outward normal components at the 2x2 Gauss points of faces W, E, S,
   N, B, T (24; face point i = 2 t1 + t2 in the face's tangential coordinates (y,z), (x,z), (x,y)),
   then the mid-plane interior values (12); DG1 pressure nodal at the 2x2x2 Gauss points (8, index
   4 i + 2 j + k); Q1 trace nodal at the 2x2 face Gauss points, trace dof 4 F + i for facet F in
   the order-0 numbering.  Cell fields are the same inputs; right-hand sides and recovered fields
   are r_ub / u_b [36][nlev][ncol] and r_pi / pi [8][nlev][ncol]; trace vectors have 4 x the
   order-0 length (hyb_sizes).  The two-level preconditioner at order 1 uses the DG0 coarse space
   with the order-0 pressure operator H on the same mesh (an internal order-0 context), P setting
   the 4 dofs of a facet to the average of its cells, Gamma = H 1 / (P^T S P 1), and LineSmooth
   with 4x4 block-tridiagonal column solves on the horizontal facets and point Jacobi on the
   vertical ones; hyb_solve is FGMRES with it (FP64).  params.precision chooses the arithmetic of
   the condensation of S_K (HYB_PREC_FP64 or the MFMA modes, whose S_K is stored in FP32) or the
   mixed form (HYB_PREC_MIXED: S_K condensed in FP64 for the outer operator, its FP32 copy in the
   preconditioner's applications of S); after changing it call hyb_condense(ctx, NULL, ...) again.  hyb_restrict and the learned stage return HYB_ESTATE at order 1. */

/* Create a context for one mesh.  stream: a hipStream_t (NULL = default stream).
   Fails with HYB_EINVAL on inconsistent tables (every edge must appear on
   two distinct (column, face) pairs; each coarse column must have 4 children). */
int hyb_create(const hyb_mesh *mesh, const hyb_params *params, void *stream, hyb_ctx **out);

/* Replace the solver parameters (not the physics: dt, tau_*, cp, rd are read by
   hyb_assemble_local).  Sec. 3.2 and App. B tune n_pre, n_post, omega, omega_p. */
int hyb_set_params(hyb_ctx *ctx, const hyb_params *params);

/* Cell matrices A_K (7x7) and the diagonal of K_K (C_K is the identity for
   outward-flux dofs) of every cell, from the bilinear forms of Sec. 2.2
   (Eq. of the bilinear forms; q32, M3^rho and M3^Pi by the one-point rule
   at the cell centre) and the hybrid forms of Sec. 2.4.  theta_w and
   exner_hat_w: [nlev+1][ncol] values of theta* and the projected Exner
   pressure on the bottom/top facet points (linear in the vertical inside a
   cell); exner_c, rho_c: [nlev][ncol] cell values.  theta* must be single
   valued on every facet for the hybridised solution to equal the mixed one. */
int hyb_assemble_local(hyb_ctx *ctx, const double *theta_w, const double *exner_hat_w,
                       const double *exner_c, const double *rho_c);

/* Static condensation (Sec. 2.4).  With r_ub == NULL (first call after
   hyb_assemble_local): factor every A_K, form S = C^T A^-1 K as an 11-point
   stencil per trace row and set up the preconditioner (lumped mass, H on
   every multigrid level, Gamma of Eq. of the scaling matrix).  With r_ub
   given: B_lambda = C^T A^-1 R_X for R_X = (r_ub [6][nlev][ncol] broken
   velocity residual, r_pi [nlev][ncol] pressure residual); b_lambda [ntrace]. */
int hyb_condense(hyb_ctx *ctx, const double *r_ub, const double *r_pi, double *b_lambda);

/* y = S x for trace vectors x, y [ntrace] (x and y must not alias). */
int hyb_trace_apply(hyb_ctx *ctx, const double *x, double *y);

/* z = M(r): one application of the two-level cycle (Alg. 2) from zero:
   LineSmooth (n_pre), residual, restriction P^T scaled by Gamma, one pressure
   multigrid V-cycle on H, prolongation by facet averaging, LineSmooth
   (n_post); with params.learned = 1 followed by the learned stage (below).
   r, z [ntrace], must not alias. */
int hyb_precondition(hyb_ctx *ctx, const double *r, double *z);

/* Flexible GMRES on S lambda = B_lambda, right preconditioned by Alg. 2.
   lambda [ntrace] is the initial guess on entry and the solution on exit.
   Stops when the FP64 relative residual ||B - S lambda|| / ||B|| <= rtol or
   after maxit iterations.  Returns HYB_OK, HYB_NOT_CONVERGED, HYB_BREAKDOWN, HYB_STAGNATED
   or a negative error; info (may be NULL) gets iterations and residuals. */
int hyb_solve(hyb_ctx *ctx, const double *b_lambda, double *lambda, double rtol, int32_t maxit,
              hyb_info *info);

/* hyb_solve for callers that cannot allocate memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid allocation): the same FGMRES with the same kernels, arguments and
   results, but no allocation of any kind during the call.  The Krylov basis is the context's own
   (allocated by hyb_condense / hyb_set_params for the current restart length; HYB_ESTATE if it is
   not); the reduction partials and dot products go to a static 2 MiB device array of the library
   instead of the context's buffers, which bounds the restart length (HYB_EINVAL with the sizes
   beyond it: (2 * 2048 + 4) (restart + 2) doubles must fit, restart <= 61).  Order 0 only, without
   the learned stage, the Krylov coarse solve (coarse_mode 2) or profiling (HYB_EINVAL /
   HYB_ESTATE otherwise).  The array is shared by every context on the device: calls that overlap
   on one device (different streams or host threads) race and must be serialised by the caller. */
int hyb_solve_noalloc(hyb_ctx *ctx, const double *b_lambda, double *lambda, double rtol, int32_t maxit,
                      hyb_info *info);

/* Cellwise recovery X = A^-1 (R_X - K lambda) (Sec. 2.4): u_b [6][nlev][ncol]
   outward fluxes of the broken velocity, pi [nlev][ncol] Exner pressure. */
int hyb_recover(hyb_ctx *ctx, const double *r_ub, const double *r_pi, const double *lambda,
                double *u_b, double *pi);

/* ----- The whole linear solve of a time step: theta' and rho' around the 2x2 system -----
   Elimination before the solve (order 0, box or cubed sphere; HYB_ESTATE before
   hyb_assemble_local, whose reference state it uses).  Sec. 2.1: theta' eliminated from the
   linearised equations, which moves r_theta into the momentum right-hand side
   (r_u - tau_u dt c_p z_hat d(Pihat*) / dz r_theta) and the equation of state (r_Pi + r_theta / theta*);
   Sec. 2.2: rho' = M3^-1 (R_rho - D u) eliminated from the 3x3 matrix system, which adds
   M3^rho M3^-1 R_rho to the pressure right-hand side.  Inputs: r_ub [6][nlev][ncol] the broken
   momentum dual vector (as for hyb_condense), r_rho and r_pi [nlev][ncol] cell values of the
   density and equation-of-state residuals, r_theta [nlev+1][ncol] the potential-temperature
   residual on the horizontal facets (the W_theta nodes).  Outputs: r_ub_bar [6][nlev][ncol] and
   r_pi_bar [nlev][ncol] (the pressure dual vector), the right-hand side hyb_condense and
   hyb_recover take.  r_ub_bar may be r_ub and r_pi_bar may be r_pi (in place). */
int hyb_eliminate(hyb_ctx *ctx, const double *r_ub, const double *r_rho, const double *r_theta, const double *r_pi,
                  double *r_ub_bar, double *r_pi_bar);

/* Back-substitution after hyb_recover (Sec. 2.1, 2.2): rho [nlev][ncol] = r_rho - tau_rho dt rho*
   (sum of the cell's outward fluxes u_b) / |K|, and theta [2][nlev][ncol] the potential
   temperature increment at each cell's bottom (index 0) and top (1) W_theta node,
   r_theta - tau_theta dt (z_hat . u) d(theta*) / dz with the vertical velocity of the cell's own
   broken velocity there (theta' jumps across a horizontal facet where d(theta*) / dz does).
   Outputs must not alias inputs (HYB_EINVAL). */
int hyb_back_substitute(hyb_ctx *ctx, const double *r_rho, const double *r_theta, const double *u_b, double *rho,
                        double *theta);

/* ----- Configuration 1 of the paper: the unhybridised system (Sec. 2.2, 2.3) -----
   The velocity / Exner-pressure system of Sec. 2.2 on the same assembled cells (order 0 only;
   HYB_EINVAL otherwise; HYB_ESTATE before hyb_condense, whose setup it uses: the lumped
   velocity mass and the pressure multigrid hierarchy).  A mixed vector has ntrace + ncell FP64
   entries in device memory: first the velocity on every facet of the trace numbering in the
   facet's global orientation (+z for horizontal facets; for vertical facets the normal leaving
   the first column of the edge), the ground and lid facets, which carry no velocity dof, held
   at zero; then the Exner pressure of every cell ([nlev][ncol]).  These calls are FP64 whatever
   hyb_params.precision says, and do not use the learned stage. */

/* b = the mixed right-hand side from the broken one: R_u on facet F is the sum over the two
   cells of F of the orientation sign times r_ub of that cell face (Sec. 2.4), R_Pi = r_pi.
   r_ub [6][nlev][ncol], r_pi [nlev][ncol] as for hyb_condense; b [ntrace + ncell]. */
int hyb_mixed_rhs(hyb_ctx *ctx, const double *r_ub, const double *r_pi, double *b);

/* y = the mixed operator of Sec. 2.2 (velocity block M2 - Q22 with the Coriolis term on a
   rotating sphere, gradient G including the facet term of the form g, divergence rows
   Q32 + M3rho M3^-1 D, M3Pi) applied to x; y is zero on the ground and lid facets.  x and y
   [ntrace + ncell], distinct. */
int hyb_mixed_apply(hyb_ctx *ctx, const double *x, double *y);

/* z = the approximate-Schur preconditioner of Sec. 2.3 applied to r: Step 1 the pressure
   right-hand side with the lumped velocity mass, Step 2 one pressure multigrid V-cycle from
   zero (the same cycle and parameters as the coarse step of Alg. 2), Step 3 the velocity from
   the lumped mass.  r and z [ntrace + ncell], distinct; z is zero on the ground and lid.
   Uses the level-0 multigrid work vectors, like hyb_precondition. */
int hyb_mixed_precondition(hyb_ctx *ctx, const double *r, double *z);

/* Flexible GMRES(restart) on the mixed system, right preconditioned by hyb_mixed_precondition
   (the paper's Configuration 1).  x [ntrace + ncell] is the initial guess on entry and the
   solution on exit.  Stops when ||b - A x|| / ||b|| <= rtol (the unweighted 2-norm of the
   mixed residual) or after maxit iterations; returns as hyb_solve.  Allocates on its first
   call a second Krylov basis of (2 restart + 1) (ntrace + ncell) doubles, kept until
   hyb_destroy. */
int hyb_mixed_solve(hyb_ctx *ctx, const double *b, double *x, double rtol, int32_t maxit,
                    hyb_info *info);

/* Sizes of the trace system: ntrace, and the bytes of device workspace held. */
int hyb_sizes(const hyb_ctx *ctx, int64_t *ntrace, int64_t *ncell, int64_t *workspace_bytes);

/* Kernel timing with HIP events on the context's stream, for measurement.
   hyb_profile(ctx, 1) clears the counters and starts recording every launch
   of the named kernel families; hyb_profile(ctx, 0) stops.  hyb_profile_read
   synchronises the stream and returns the number of launches and their total
   duration in milliseconds for one family: "smooth_rows" (LineSmooth residual
   rows from a nonzero iterate), "smooth_rows0" (first presmoothing sweep),
   "thomas" (LineSmooth column solves), "trace_apply", "mg_smooth",
   "restrict", "prolong", "krylov", "cell_solve". */
int hyb_profile(hyb_ctx *ctx, int32_t enable);
/* As hyb_profile(ctx, 1), but recording one family only (the others launch without
   events, so the timing of the rest of the path is not disturbed).  HYB_EINVAL for an
   unknown family name. */
int hyb_profile_family(hyb_ctx *ctx, const char *family);
int hyb_profile_read(hyb_ctx *ctx, const char *family, int64_t *launches, double *total_ms);

/* Restriction of a trace vector r [ntrace] to cells [nlev][ncol] (device FP64 arrays): mode 0
   Gamma P^T r (the scaled right-hand side of the coarse level in Alg. 2), mode 1 the facet average
   P^T r / P^T 1, mode 2 H_KK times the facet average (H_KK: diagonal of the pressure operator H),
   mode 3 P^T r (P: the facet-average prolongation of Alg. 2).  HYB_EINVAL for another mode. */
int hyb_restrict(hyb_ctx *ctx, const double *r, double *cells, int32_t mode);

/* Learned coarse correction (not part of the paper): a network of three 3D convolutions on cell
   fields (3 -> 16 -> 16 -> 1 channels; taps = the 3x3 horizontal neighbourhood of a column in its
   own frame times 5 vertical offsets, zero padded at ground and lid and where a cube vertex leaves
   no corner neighbour; ReLU after the first two), BF16 weights with FP32 accumulation.  Input
   channel 0 is the field x; channels 1 and 2 are static fields of the assembled mesh, the same for
   every sample: log(h / dz) with h = sqrt(|K| / dz) the cell's horizontal size, and the height of
   the cell centre over the height of the lid (network calls need hyb_assemble_local first).  With params.learned = 1, hyb_solve and hyb_precondition follow every
   two-level cycle z = M(v) with r' = v - S z, c = Gamma P^T r', s = rms(c),
   d = s P (N(c / s) / H_KK), and z += d only if ||r' - S d||_2 < learned_tau ||r'||_2 (FP64):
   otherwise, or when the network output is not finite, z stays the plain cycle's output (counted in
   hyb_info.fallbacks).
   Parameters (FP32, host arrays of hyb_nn_param_count() values): W1 [16][3][45], b1 [16],
   W2 [16][16][45], b2 [16], W3 [1][16][45], b3 [1], tap index = 5*h + (dk+2), h = centre, W, E,
   S, N, SW, SE, NW, NE.  Cell fields x, t, y are DEVICE FP32 arrays [nsamp][nlev][ncol].
   Errors: HYB_ESTATE before hyb_nn_set_weights (or, for the energy calls, before hyb_condense);
   HYB_EINVAL for NULL arrays, nsamp < 1, a wrong parameter count or non-finite weights. */
int hyb_nn_param_count(void);
int hyb_nn_set_weights(hyb_ctx *ctx, const float *weights, int64_t n);
int hyb_nn_get_weights(hyb_ctx *ctx, float *weights, int64_t n);
int hyb_nn_forward(hyb_ctx *ctx, const float *x, float *y, int32_t nsamp);
/* mean squared error of N(x) against t over all cells and samples; gradient (host, may be NULL)
   in the parameter layout above */
int hyb_nn_loss_grad(hyb_ctx *ctx, const float *x, const float *t, int32_t nsamp, float *loss, float *grad);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error; loss (host) may be NULL */
int hyb_nn_train_step(hyb_ctx *ctx, const float *x, const float *t, int32_t nsamp, float lr, float *loss);
/* Error-energy loss of the stage's correction: for pairs x_i = c_i / s_i (FP32) and
   rhat_i = P^T r'_i / s_i (DEVICE FP64 [nsamp][nlev][ncol]), with q_i = N(x_i) / H_KK and
   G = P^T S P, loss = mean_i (q_i^T G q_i - 2 q_i^T rhat_i) * mean(H_KK) / ncell, which is the change
   of (e'^T S e') / s_i^2 when S is symmetric (e' = S^-1 r'), up to that scale.  gradient (host, may be
   NULL) as above; loss (host, may be NULL). */
int hyb_nn_energy_grad(hyb_ctx *ctx, const float *x, const double *rhat, int32_t nsamp, double *loss, float *grad);
/* one Adam step on the energy loss */
int hyb_nn_energy_train_step(hyb_ctx *ctx, const float *x, const double *rhat, int32_t nsamp, float lr,
                             double *loss);
/* The same step on the pairs idx[0..nsamp) (HOST int32, each in [0, npairs)) of a set of pairs X
   [npairs][nlev][ncol] (DEVICE FP32) and R (DEVICE FP64), gathered inside the library.  HYB_EINVAL
   for an index out of range. */
int hyb_nn_energy_train_step_pairs(hyb_ctx *ctx, const float *X, const double *R, int64_t npairs,
                                   const int32_t *idx, int32_t nsamp, float lr, double *loss);
/* Adam state of the training, to resume it in another context or process: the first and second
   moments (host FP32 arrays of hyb_nn_param_count() values, in the parameter layout) and the step
   count.  hyb_nn_set_weights resets the state, so hyb_nn_set_state follows it.  HYB_ESTATE before
   hyb_nn_set_weights; HYB_EINVAL for NULL arrays, a wrong count, a negative step or non-finite or
   (second moment) negative entries. */
int hyb_nn_get_state(hyb_ctx *ctx, float *m, float *v, int64_t n, int64_t *step);
int hyb_nn_set_state(hyb_ctx *ctx, const float *m, const float *v, int64_t n, int64_t step);
/* One training pair from the plain method (the hook of the stage is the coarse correction of
   Alg. 2): the two-level cycle (Alg. 2, without the learned stage, in the context's precision) taken
   as a stationary iteration, z = M(r) and r <- r - S z, then c = Gamma P^T r, s = rms(c) over the
   cells, x = c / s (FP32) and rhat = P^T r / s (FP64).  r: DEVICE FP64 [ntrace], in/out; x, rhat:
   DEVICE [nlev][ncol]; scale (host, may be NULL): s.  Calling it again on the same r gives the next
   pair of the iteration.  Returns HYB_BREAKDOWN (positive) when s is zero or not finite (x and rhat
   are then not usable); HYB_ESTATE before hyb_condense or at order 1. */
int hyb_nn_cycle_pair(hyb_ctx *ctx, double *r, float *x, double *rhat, double *scale);

const char *hyb_last_error(const hyb_ctx *ctx);
void hyb_destroy(hyb_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* HYB_H */
