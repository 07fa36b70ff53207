// Internal declarations of the hybridised trace solver library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hyb.h"

namespace hyb {

// ---------------------------------------------------------------------------------------------
// Device-side mesh description of one multigrid level.
//   col_edge[f][col]: edge of local face f (0..3 = W,E,S,N)
//   nbr[f][col]:      column across local face f
//   nlf[f][col]:      local face index of that edge inside the neighbour column
//   own[j][col]:      edges whose normal enters this column (the column that owns the
//                     trace rows of the edge), -1 padded, j = 0..3
//   est[i][e]:        row neighbours of edge e: columns c0, c1 and the other three edges of each
//   parent[col]:      coarse column (next level) of this column; children[q][ccol] the reverse
// ---------------------------------------------------------------------------------------------
struct LevelDev {
  int ncol = 0, nedge = 0;
  int32_t *col_edge = nullptr, *edge_col = nullptr, *edge_lf = nullptr;
  int32_t *nbr = nullptr, *nlf = nullptr, *own = nullptr;
  int32_t *est = nullptr;       // [8][nedge]: c0, c1, other 3 edges of c0, other 3 edges of c1
  int32_t *parent = nullptr;    // [ncol] -> column of level l+1 (nullptr on the coarsest level)
  int32_t *children = nullptr;  // [4][ncol] -> columns of level l-1 (nullptr on level 0)
  bool child_pairs = false;     // children[1] = children[0] + 1 and children[3] = children[2] + 1, both even
  double *H = nullptr;          // [7][nlev*ncol] pressure stencil: diag, W, E, S, N, below, above
  float *Hf = nullptr;          // FP32 copy
  double *zf = nullptr;         // [3][nlev*ncol] LU factors of the column part H_z: l, 1/u, c/u
  float *zff = nullptr;
  void *b = nullptr, *x = nullptr, *y = nullptr;  // [nlev*ncol] work vectors
  void *w = nullptr;  // coarsest level only: the third iterate of the Chebyshev coarsest solve
};

// The 11-entry trace stencil S (and its FP32 copy) is stored in tiles of 64 rows: entry j of row F
// at ((F / 64) * 11 + j) * 64 + F mod 64, so the entries a wavefront reads for 64 consecutive rows lie
// in one contiguous 5.5 KB block (one stream from HBM instead of eleven).
constexpr int kSTile = 64;
__host__ __device__ __forceinline__ size_t s_idx(size_t F, int j) {
  return ((F / kSTile) * 11 + (size_t)j) * kSTile + F % kSTile;
}
__host__ __device__ __forceinline__ size_t s_entries(size_t ntr) { return 11 * ((ntr + kSTile - 1) / kSTile) * kSTile; }

constexpr int kNNChannels = 16;
// network input channels: the normalised coarse residual, then two static fields of the mesh,
// log(h / dz) (h = sqrt(|K| / dz), the cell's horizontal size) and the cell-centre height over the
// height of the lid
constexpr int kNNInputs = 3;

// Learned coarse-correction network state (device buffers).
struct NNState {
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // FP32 parameters, Adam moments, gradient
  uint16_t *wb = nullptr;                                         // BF16 copy of the weights
  int32_t *isbf = nullptr;                                        // parameter -> BF16 index (-1: bias)
  int32_t *nb9 = nullptr;                                         // [9][ncol] 3x3 horizontal neighbourhood (-1: none)
  int32_t *rv9 = nullptr;                                         // [9][ncol] readers of a column: col * 9 + tap
  int32_t *rvh = nullptr;                                         // [9][ncol] the reader through tap h (-1: none)
  int32_t *lo_off = nullptr, *lo_list = nullptr;                  // further readers per column (CSR)
  float *wpart = nullptr;                                         // matrix-core weight-gradient partials
  float *st = nullptr;                                            // [2][ncell] static input channels
  double *layer = nullptr;                                        // [2][nlev] log(dz), centre height / lid
  bool st_ready = false;
  float *a1 = nullptr, *a2 = nullptr, *y = nullptr;               // activations [nsamp][C][ncell]
  float *d1 = nullptr, *d2 = nullptr, *dy = nullptr;              // their gradients
  float *part = nullptr, *tmpg = nullptr, *lpart = nullptr;       // reduction scratch
  float *cin = nullptr, *cout = nullptr;                          // learned stage input / output [ncell]
  double *scal = nullptr;                                         // learned stage scalars (device)
  uint16_t *a1h = nullptr, *a2h = nullptr;                        // stage activations [ncell][16] BF16
  double *d64 = nullptr, *sd64 = nullptr;                         // correction d and S d [ntrace]
  double *gq = nullptr, *epart = nullptr;                         // energy loss: G q [nsamp][ncell], partials
  size_t gq_cap = 0;
  float *xb = nullptr;                                            // gathered training batch: inputs
  double *rb = nullptr;                                           // and targets [nsamp][ncell]
  size_t batch_cap = 0;                                           // cells x samples they hold
  double dbar = 0.0;                                              // mean of the diagonal of H
  size_t cap = 0;                                                 // cells x samples the activations hold
  long step = 0;
  bool loaded = false;
};

// p = 1 system (p1.hip): cell data per cell (array of structures)
struct P1State {
  double *tbl = nullptr;    // reference tables of the assembly
  double *A = nullptr;      // [ncell][748] the entries of A_K left non-zero by its block structure
  double *cdiag = nullptr;  // [ncell][24] diagonal of C_K on the face dofs
  double *kdiag = nullptr;  // [ncell][24] diagonal of K_K
  double *SK = nullptr;     // [24 x 24][ncell] S_K = C_K [A_K^-1]_ff K_K, entry (r, j) at (r * 24 + j) * ncell
  float *SKf = nullptr;     // [576][ncell] S_K in FP32 (the MFMA modes; the preconditioner's copy when mixed)
  double *bK = nullptr;     // [24][ncell] the cells' shares of B_lambda, or of S x on its way to the rows
  double *fac = nullptr;    // [748][ncell] factors of A_K by its block structure: M^-1, M^-1 G, Dr, Sg^-1
  // two-level preconditioner
  double *dS = nullptr;     // [ntrace] diagonal of S
  double *zf = nullptr;     // [nz][48] block LU factors of the column systems: Dinv, W, U (4x4 each)
  double *gamma = nullptr;  // [ncell] Gamma = H 1 / (P^T S P 1)
  double *den = nullptr;    // [ncell]
  double *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;  // [ntrace] work vectors
};

struct ProfFamily {
  std::string name;
  std::vector<hipEvent_t> ev;  // start/stop pairs
  size_t used = 0;
};

}  // namespace hyb

struct hyb_ctx {
  hipStream_t stream = nullptr;
  hyb_params p{};
  int nlev = 0, ncol = 0, nedge = 0, ncell = 0, nz = 0, ntrace = 0, nlevels = 0;
  double dx = 0, dy = 0;
  std::vector<double> dz;
  double *dz_d = nullptr;
  int geom = HYB_GEOM_BOX;
  double *corners_d = nullptr;  // HYB_GEOM_SHELL: [4][3][ncol] corner unit vectors
  double *radius_d = nullptr;   // HYB_GEOM_SHELL: [nlev + 1]
  std::vector<hyb::LevelDev> lv;

  // cell data
  double *A = nullptr;      // [49][ncell] A_K row-major (i*7+j)
  double *LU = nullptr;     // [49][ncell] LU factors of A_K (unit lower, no pivoting)
  double *kv = nullptr;     // [6][ncell] diagonal of K_K
  double *vol = nullptr;    // [ncell] cell volumes (the Gauss rule of the mass forms)
  double *ck = nullptr;     // [10][ncell] vectors of the Krylov coarse solve (coarse_mode 2)
  double *Scell = nullptr;  // [36][ncell] S_K = [A_K^-1]_uu diag(k)  (setup only)
  double *bcell = nullptr;  // [6][ncell] [A_K^-1 R_K]_u
  double *ec = nullptr;     // [8][ncell] coefficients of the theta' / rho' elimination (assemble.hip)
  // trace operator
  double *S = nullptr;      // 11-entry rows in tiles of 64 rows (s_idx)
  float *Sf = nullptr;      // FP32 copy, same layout
  double *m2l = nullptr;    // [ntrace] lumped velocity mass (interior facets)
  double *zfac = nullptr;   // [3][nz] LU factors of S^zz per column: l, 1/u, c/u
  float *zfacf = nullptr;
  double *zfacp = nullptr;  // [3][nlev+1][ncol of level 1] the same per 2x2 patch (smoother_patch)
  float *zfacpf = nullptr;
  double *gamma = nullptr;  // [ncell]
  float *gammaf = nullptr;
  // preconditioner work vectors (precision of the preconditioner)
  void *tIn = nullptr, *tA = nullptr, *tB = nullptr, *tR = nullptr;  // [ntrace]
  double *t64 = nullptr;    // [ntrace]
  // Krylov workspace
  int m = 0;
  double *V = nullptr;      // [(m+1)][ldv]
  void *Z = nullptr;        // [m][ldv] (double or float)
  size_t ldv = 0;           // leading dimension of V and Z: ntrace plus kBasisPad
  double *Vm = nullptr;     // Configuration 1: [(m+1)][ntrace + ncell]
  double *Zm = nullptr;     // Configuration 1: [m][ntrace + ncell]
  int mm = 0;               // restart length Vm / Zm were allocated for
  double *partial = nullptr;  // [nblk_red][2*(m+2)]
  double *hdev = nullptr;   // [4*(m+2)]
  double *hhost = nullptr;  // pinned [4*(m+2)]
  hipEvent_t ev_coef = nullptr;  // the read-back of a Gram-Schmidt step's coefficients has landed
  int nblk_red = 0;
  long reorth = 0;           // second Gram-Schmidt passes taken (diagnostics)
  // host side of the restart cycle (Hessenberg matrix, Givens rotations, least-squares solution),
  // sized with the basis so that a solve allocates no host memory either
  std::vector<double> kR, kHr, kg, kcs, ksn, ky, kca, kcb;
  // the device current at hyb_create and that device's copy of the library's static reduction
  // scratch (hyb_solve_noalloc); null when its address could not be taken
  int device = -1;
  double *scratch = nullptr;
  std::string scratch_err;

  bool assembled = false, condensed = false;
  std::string err;
  size_t bytes = 0;

  bool prof = false;
  uint64_t prof_mask = ~0ull;  // families recorded while prof is on
  std::vector<hyb::ProfFamily> fam;

  hyb::NNState nn;
  double *cell64 = nullptr;  // [ncell] scratch of the learned stage

  int order = 0;             // 0: RT0 / Q0 / one trace dof per facet; 1: RT1 / DG1 / 4 per facet
  hyb::P1State p1;
  hyb_ctx *coarse = nullptr;  // order 1: order-0 context on the same mesh (the DG0 coarse space)
};

namespace hyb {

constexpr int kBlock = 256;
constexpr int kColBlock = 64;  // one wavefront per workgroup for the column (Thomas) kernels

// profiling helpers (no-ops unless ctx->prof)
int prof_begin(hyb_ctx *c, int fam);
void prof_end(hyb_ctx *c, int fam, int slot);
enum Family {
  F_SMOOTH_ROWS = 0,  // LineSmooth residual rows, sweeps from a nonzero iterate
  F_SMOOTH_ROWS0,     // the first presmoothing sweep (iterate zero): vertical facets only
  F_THOMAS,           // LineSmooth column solves
  F_TRACE_APPLY,
  F_MG_SMOOTH,
  F_RESTRICT,
  F_PROLONG,
  F_KRYLOV,
  F_CELL,
  F_NN,               // learned coarse-correction stage
  F_P1_CONDENSE,      // order 1: S_K on MFMA
  F_P1_FACTOR,        // order 1: FP64 LU of A_K (and S_K in the FP64 mode)
  F_COUNT
};

// ----- setup kernels (assemble.hip) -----
hipError_t launch_assemble_box(hyb_ctx *c, const double *theta_w, const double *exner_hat_w,
                               const double *exner_c, const double *rho_c);
hipError_t launch_factor_cells(hyb_ctx *c);
hipError_t launch_build_stencil(hyb_ctx *c);
hipError_t launch_assemble_shell(hyb_ctx *c, const double *theta_w, const double *exner_hat_w,
                                 const double *exner_c, double *rs);
hipError_t launch_lumped_mass(hyb_ctx *c, const double *rs = nullptr);
hipError_t launch_pressure_stencil(hyb_ctx *c);
hipError_t launch_galerkin(hyb_ctx *c, int coarse_level);
hipError_t launch_gamma(hyb_ctx *c);
hipError_t launch_to_float(hyb_ctx *c, const double *src, float *dst, size_t n);
// elimination of theta' and rho' (Sec. 2.1, 2.2): coefficients at assembly, then the pointwise passes
hipError_t launch_elim_coeffs(hyb_ctx *c, const double *theta_w, const double *exner_hat_w, const double *rho_c);
hipError_t launch_eliminate(hyb_ctx *c, const double *r_ub, const double *r_rho, const double *r_theta,
                            const double *r_pi, double *r_ub_bar, double *r_pi_bar);
hipError_t launch_back_substitute(hyb_ctx *c, const double *r_rho, const double *r_theta, const double *u_b,
                                  double *rho, double *theta);
hipError_t launch_fill(hyb_ctx *c, double *dst, size_t n, double v);

// ----- cell solves (assemble.hip) -----
hipError_t launch_cell_rhs(hyb_ctx *c, const double *r_ub, const double *r_pi, double *b_lambda);
hipError_t launch_recover(hyb_ctx *c, const double *r_ub, const double *r_pi, const double *lambda,
                          double *u_b, double *pi);

// ----- trace operator and preconditioner (solve.hip) -----
// y = S x (mode 0) or y = b - S x (mode 1); Tm matrix, Tx input, Ty output precision
template <typename Tm, typename Tx, typename Ty>
hipError_t launch_trace_apply(hyb_ctx *c, const Tm *S, const Tx *x, const Ty *b, Ty *y, int mode);
template <typename T>
hipError_t precondition(hyb_ctx *c, const T *r, T *z);
hipError_t configure_kernels(int nlev);
hipError_t launch_thomas_factor(hyb_ctx *c);
hipError_t launch_mg_factor(hyb_ctx *c, int level);

// ----- Krylov (krylov.hip) -----
hipError_t launch_convert(hyb_ctx *c, const double *src, float *dst, size_t n);
hipError_t launch_copy_widen(hyb_ctx *c, const float *src, double *dst, size_t n);
// out[i] = sum_k a[k][i] * w[i] for k < nv (rows of a with stride lda), plus ||w||^2 when with_norm
hipError_t launch_multidot(hyb_ctx *c, const double *a, size_t lda, int nv, const double *w, size_t n,
                           double *out_dev, bool with_norm);
// w -= sum_k h[k] a[k]  (h on device)
hipError_t launch_multi_axpy_dev(hyb_ctx *c, const double *a, size_t lda, int nv, const double *h_dev,
                                 double *w, size_t n);
// fused classical Gram-Schmidt with reorthogonalisation (nv <= 32): h1 = V w, w -= V^T h1,
// h2n[0..nv-1] = V w, h2n[nv] = ||w||^2; then w = (w - V^T h2) * s
hipError_t launch_gs_passes(hyb_ctx *c, const double *V, size_t lda, size_t n, int nv, double *w, double *h1,
                            double *h2n);
hipError_t launch_gs_finish(hyb_ctx *c, const double *V, size_t lda, size_t n, int nv, const double *h2, double *w,
                            double s);
// Gram-Schmidt with delayed reorthogonalisation (steps j < kDgsMax): dots of V_j and V_{j+1}
// against V_0..V_j and ||V_{j+1}||^2 (2 j + 3 values into out_dev: [V_k . V_j], [V_k . V_{j+1}],
// ||V_{j+1}||^2); the step's coefficients from them on the device (2 j + 6 values into coef: ca,
// cb, rho, hjj, eta, breakdown flag, 1 / rho, 1 / eta); then V_j <- (V_j - sum_{k<j} ca_k V_k) / rho
// and V_{j+1} <- (V_{j+1} - sum_{k<j} cb_k V_k - hjj V_j) / eta in one pass (and its FP32 copy into
// wf if wf is not null), reading the coefficients from coef, so that no host round trip sits
// between the reduction and the update.
constexpr int kDgsMax = 31;
// the basis vectors of V and Z start kBasisPad entries apart beyond their length, so that entry i
// of the vectors does not fall on the same HBM channel for all of them (a leading dimension of
// 2^16 times an odd number made the reduction pass over 18 vectors 50 % slower than over 17)
constexpr size_t kBasisPad = 256;
// a restart cycle that leaves more than this fraction of the true residual counts as stalled
constexpr double kStagnation = 0.999;
hipError_t launch_dgs_dots(hyb_ctx *c, const double *V, size_t lda, size_t n, int j, double *out_dev);
hipError_t launch_dgs_coef(hyb_ctx *c, const double *dots, int j, double *coef);
hipError_t launch_dgs_update(hyb_ctx *c, double *V, size_t lda, size_t n, int j, const double *coef,
                             float *wf = nullptr);
// w -= sum_k h[k] a[k], then nrm_dev[0] = ||w||^2
hipError_t launch_axpy_norm(hyb_ctx *c, const double *a, size_t lda, int nv, const double *h_dev, double *w,
                            size_t n, double *nrm_dev);
template <typename Tz>
hipError_t launch_update_solution(hyb_ctx *c, const Tz *Z, size_t ldz, int nv, const double *y_dev,
                                  double *x, size_t n);
hipError_t launch_scale(hyb_ctx *c, double *w, size_t n, double s);

// ----- p = 1 (p1.hip) -----
hipError_t p1_setup(hyb_ctx *c);
hipError_t p1_assemble(hyb_ctx *c, const double *theta_w, const double *exner_hat_w, const double *exner_c,
                       const double *rho_c);
hipError_t p1_factor(hyb_ctx *c);
bool p1_sk_fp32(const hyb_ctx *c);
// mode 0: the cells' shares of B_lambda into p1.bK; mode 1: recovery into u [36][ncell], pi [8][ncell]
hipError_t p1_cell_solve(hyb_ctx *c, const double *r_u, const double *r_p, const double *lam, int mode, double *u,
                         double *pi);
// mode 0: y = S x; mode 1: y = gather of p1.bK (B_lambda); mode 2: y = b - S x; mode 3: y = diag(S);
// precond: an application inside the preconditioner (the FP32 copy of S_K in the mixed form)
hipError_t p1_rows(hyb_ctx *c, const double *x, double *y, int mode, const double *b, bool precond = false);
hipError_t p1_precond_setup(hyb_ctx *c);
hipError_t p1_precondition(hyb_ctx *c, const double *r, double *z);
void p1_free(hyb_ctx *c);
// one FP64 pressure multigrid V-cycle on level 0: lv[0].b -> lv[0].x (solve.hip)
hipError_t coarse_vcycle(hyb_ctx *c);

// ----- Configuration 1: the unhybridised mixed system (schur.hip) -----
// mixed vectors: [ntrace] facet velocities (global orientation, 0 on ground and lid), [ncell] Pi
hipError_t launch_mixed_rows(hyb_ctx *c, const double *x, const double *b, double *y);  // y = A x or b - A x
hipError_t launch_mixed_rhs(hyb_ctx *c, const double *r_ub, const double *r_pi, double *y);
hipError_t schur_precondition(hyb_ctx *c, const double *r, double *z);  // Steps 1-3 of Sec. 2.3

// ----- learned coarse correction (nn.hip) -----
int nn_param_count();
hipError_t nn_setup(hyb_ctx *c);
hipError_t nn_set_weights(hyb_ctx *c, const float *host_w);
hipError_t nn_get_weights(hyb_ctx *c, float *host_w);
hipError_t nn_get_state(hyb_ctx *c, float *m, float *v, int64_t *step);
hipError_t nn_set_state(hyb_ctx *c, const float *m, const float *v, int64_t step);
hipError_t nn_forward(hyb_ctx *c, const float *x, float *out, int nsamp);
hipError_t nn_loss_grad(hyb_ctx *c, const float *x, const float *target, int nsamp, float *loss_host);
hipError_t nn_energy_grad(hyb_ctx *c, const float *x, const double *rhat, int nsamp, double *loss_host);
hipError_t nn_adam(hyb_ctx *c, float lr);
hipError_t nn_stage_buffers(hyb_ctx *c);
hipError_t nn_pair_finish(hyb_ctx *c, float *x, double *rhat, double *scale_host);
hipError_t nn_gather_batch(hyb_ctx *c, const float *X, const double *R, const int32_t *idx, int nsamp);
void nn_free(hyb_ctx *c);
// restriction of a trace vector to cells: mode 0 Gamma P^T r, mode 1 P^T r / P^T 1 (cell average),
// mode 2 H_diag times mode 1, mode 3 P^T r
hipError_t launch_restrict_cells(hyb_ctx *c, const double *r, double *cells, int mode);
// learned stage: d = s P (N(c / s) / H_diag), c = Gamma P^T (r - S z), s = rms(c); z += d if it
// lowers ||r - S z||, else counted as a fallback
template <typename Tz>
hipError_t learned_stage(hyb_ctx *c, const double *r, Tz *z, double *Sz = nullptr);

}  // namespace hyb
