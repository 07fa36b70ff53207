// C ABI of the hybridised trace solver: context management, the setup sequence and the flexible
// GMRES outer loop (host-driven; every vector operation runs in the kernels of this library).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "hyb_internal.h"

using namespace hyb;

namespace hyb {
int reduction_blocks();
}

// Reduction scratch of hyb_solve_noalloc: the workgroup partial sums of the Gram-Schmidt dots and
// norms and the summed results, in a fixed array of 2 MiB per device (every device the library
// runs on holds its own copy until the process ends).  Host code never uses the array's name as
// an address: hyb_create looks up the device address once per device and keeps it.
constexpr size_t kScratchDoubles = (size_t(2) << 20) / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// The device address of this device's scratch (the device must be current); nullptr if unknown.
double *scratch_address(int dev, std::string *err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = "device index out of range for the static scratch table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_dev[dev] = (double *)ptr;
  }
  return g_scratch_dev[dev];
}

}  // namespace

namespace {

const char *kFamilyNames[F_COUNT] = {"smooth_rows", "smooth_rows0", "thomas",      "trace_apply", "mg_smooth",
                                     "restrict",    "prolong",      "krylov",      "cell_solve",  "nn",
                                     "p1_condense", "p1_factor"};

int fail(hyb_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hipfail(hyb_ctx *c, hipError_t e, const char *where) {
  return fail(c, HYB_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define CHECK_HIP(expr, where)                  \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hipfail(c, e_, where); \
  } while (0)

template <typename T>
int dalloc(hyb_ctx *c, T **p, size_t count) {
  if (*p) return HYB_OK;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc((void **)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, HYB_ENOMEM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes failed");
  }
  c->bytes += bytes;
  return HYB_OK;
}

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

int upload(hyb_ctx *c, int32_t **dst, const std::vector<int32_t> &v) {
  int rc = dalloc(c, dst, v.size());
  if (rc) return rc;
  CHECK_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice), "upload table");
  return HYB_OK;
}

int check_params(hyb_ctx *c, const hyb_params *p) {
  if (!p) return fail(c, HYB_EINVAL, "params is NULL");
  if (!(p->omega > 0) || !(p->omega_p > 0)) return fail(c, HYB_EINVAL, "omega and omega_p must be positive");
  if (p->n_pre < 0 || p->n_post < 0 || p->mg_pre < 0 || p->mg_post < 0 || p->mg_coarse_sweeps < 1)
    return fail(c, HYB_EINVAL, "sweep counts must be >= 0 (coarse sweeps >= 1)");
  if (p->restart < 1 || p->restart > 200) return fail(c, HYB_EINVAL, "restart must be in [1, 200]");
  if (p->precision != HYB_PREC_FP64 && p->precision != HYB_PREC_MIXED && p->precision != HYB_PREC_MFMA_FP32 &&
      p->precision != HYB_PREC_MFMA_BF16X)
    return fail(c, HYB_EINVAL, "unknown precision mode");
  if (p->learned != 0 && p->learned != 1) return fail(c, HYB_EINVAL, "learned must be 0 or 1");
  if (!(p->learned_tau > 0.0) || !std::isfinite(p->learned_tau)) return fail(c, HYB_EINVAL, "learned_tau must be > 0");
  if (p->mg_coarse_cheb != 0 && p->mg_coarse_cheb != 1) return fail(c, HYB_EINVAL, "mg_coarse_cheb must be 0 or 1");
  if (p->mg_coarse_cheb && !(p->cheb_lo > 0.0 && p->cheb_hi > p->cheb_lo && std::isfinite(p->cheb_hi)))
    return fail(c, HYB_EINVAL, "the Chebyshev interval needs 0 < cheb_lo < cheb_hi");
  if (!std::isfinite(p->omega_rot)) return fail(c, HYB_EINVAL, "omega_rot must be finite");
  if (p->coarse_mode < 0 || p->coarse_mode > 2) return fail(c, HYB_EINVAL, "coarse_mode must be 0, 1 or 2");
  if (p->coarse_mode == 2 && (p->precision != HYB_PREC_FP64 || c->order != 0))
    return fail(c, HYB_EINVAL, "the Krylov coarse solve (coarse_mode 2) is an order-0 FP64 mode");
  if (p->coarse_mode == 2 && !(p->coarse_rtol > 0.0 && p->coarse_rtol < 1.0))
    return fail(c, HYB_EINVAL, "coarse_rtol must be in (0, 1)");
  if (p->smoother_patch != 0 && p->smoother_patch != 1) return fail(c, HYB_EINVAL, "smoother_patch must be 0 or 1");
  if (p->nn_fp32 != 0 && p->nn_fp32 != 1) return fail(c, HYB_EINVAL, "nn_fp32 must be 0 or 1");
  if (p->debug & ~(HYB_DEBUG_ZERO_GAMMA | HYB_DEBUG_NAN_STAGE | HYB_DEBUG_UNPAIRED_RESTRICT))
    return fail(c, HYB_EINVAL, "unknown debug bits");
  if (p->smoother_patch && c->ncol > 0 && (c->order != 0 || c->nlevels < 2))  // (hyb_create checks it itself)
    return fail(c, HYB_EINVAL, "patch-cached column matrices need order 0 and a multigrid level of patches");
  if (p->omega_rot != 0.0 && c->geom != HYB_GEOM_SHELL)
    return fail(c, HYB_EINVAL, "rotation (omega_rot) is defined on HYB_GEOM_SHELL meshes only");
  return HYB_OK;
}

// Host-side checks and derived tables of one level.
int setup_level(hyb_ctx *c, const hyb_mesh *mesh, int l) {
  const hyb_level &hl = mesh->levels[l];
  LevelDev &L = c->lv[l];
  int ncol = hl.ncol, nedge = 2 * hl.ncol;
  if (ncol < 1 || !hl.col_edge || !hl.edge_col || !hl.edge_lf) return fail(c, HYB_EINVAL, "level tables missing");
  L.ncol = ncol;
  L.nedge = nedge;
  std::vector<int32_t> ce(hl.col_edge, hl.col_edge + 4 * (size_t)ncol);
  std::vector<int32_t> ec(hl.edge_col, hl.edge_col + 2 * (size_t)nedge);
  std::vector<int32_t> el(hl.edge_lf, hl.edge_lf + 2 * (size_t)nedge);
  for (int e = 0; e < nedge; ++e) {
    for (int s = 0; s < 2; ++s) {
      int col = ec[(size_t)s * nedge + e], f = el[(size_t)s * nedge + e];
      if (col < 0 || col >= ncol || f < 0 || f > 3) return fail(c, HYB_EINVAL, "edge table out of range");
      if (ce[(size_t)f * ncol + col] != e) return fail(c, HYB_EINVAL, "col_edge / edge_col / edge_lf disagree");
    }
    if (ec[e] == ec[(size_t)nedge + e]) return fail(c, HYB_EINVAL, "an edge joins a column to itself");
  }
  std::vector<int32_t> nbr(4 * (size_t)ncol), nlf(4 * (size_t)ncol), own(4 * (size_t)ncol, -1);
  std::vector<int> nown(ncol, 0);
  for (int col = 0; col < ncol; ++col)
    for (int f = 0; f < 4; ++f) {
      int e = ce[(size_t)f * ncol + col];
      if (e < 0 || e >= nedge) return fail(c, HYB_EINVAL, "col_edge out of range");
      int side = (ec[e] == col && el[e] == f) ? 0 : 1;
      if (ec[(size_t)side * nedge + e] != col || el[(size_t)side * nedge + e] != f)
        return fail(c, HYB_EINVAL, "column face not found on its edge");
      nbr[(size_t)f * ncol + col] = ec[(size_t)(1 - side) * nedge + e];
      nlf[(size_t)f * ncol + col] = el[(size_t)(1 - side) * nedge + e];
    }
  for (int e = 0; e < nedge; ++e) {
    int c1 = ec[(size_t)nedge + e];
    own[(size_t)nown[c1] * ncol + c1] = e;  // at most 4 edges enter a column
    nown[c1]++;
  }
  std::vector<int32_t> est(8 * (size_t)nedge);
  for (int e = 0; e < nedge; ++e) {
    int c0 = ec[e], c1 = ec[(size_t)nedge + e], l0 = el[e], l1 = el[(size_t)nedge + e];
    est[e] = c0;
    est[(size_t)nedge + e] = c1;
    int j0 = 2, j1 = 5;
    for (int f = 0; f < 4; ++f) {
      if (f != l0) est[(size_t)(j0++) * nedge + e] = ce[(size_t)f * ncol + c0];
      if (f != l1) est[(size_t)(j1++) * nedge + e] = ce[(size_t)f * ncol + c1];
    }
  }
  int rc;
  if ((rc = upload(c, &L.col_edge, ce)) || (rc = upload(c, &L.edge_col, ec)) || (rc = upload(c, &L.edge_lf, el)) ||
      (rc = upload(c, &L.nbr, nbr)) || (rc = upload(c, &L.nlf, nlf)))
    return rc;
  if (l == 0) {
    if ((rc = upload(c, &L.own, own)) || (rc = upload(c, &L.est, est))) return rc;
  }
  if (l > 0) {
    const hyb_level &fine = mesh->levels[l - 1];
    if (!hl.parent) return fail(c, HYB_EINVAL, "coarse level without parent map");
    std::vector<int32_t> par(hl.parent, hl.parent + fine.ncol);
    std::vector<int32_t> ch(4 * (size_t)ncol, -1);
    std::vector<int> cnt(ncol, 0);
    for (int fc = 0; fc < fine.ncol; ++fc) {
      int P = par[fc];
      if (P < 0 || P >= ncol || cnt[P] >= 4) return fail(c, HYB_EINVAL, "every coarse column needs 4 children");
      ch[(size_t)cnt[P] * ncol + P] = fc;
      cnt[P]++;
    }
    for (int P = 0; P < ncol; ++P)
      if (cnt[P] != 4) return fail(c, HYB_EINVAL, "every coarse column needs 4 children");
    // children as two pairs of adjacent columns, each starting at an even column of a level with an
    // even column count (the box and the cubed sphere number their children that way): the
    // restriction then loads each pair as one aligned vector
    L.child_pairs = fine.ncol % 2 == 0;
    for (int P = 0; P < ncol && L.child_pairs; ++P) {
      const int32_t a = ch[P], b = ch[(size_t)ncol + P], e = ch[2 * (size_t)ncol + P], f = ch[3 * (size_t)ncol + P];
      L.child_pairs = a % 2 == 0 && b == a + 1 && e % 2 == 0 && f == e + 1;
    }
    if ((rc = upload(c, &L.children, ch)) || (rc = upload(c, &c->lv[l - 1].parent, par))) return rc;
  }
  size_t n = (size_t)ncol * c->nlev;
  if ((rc = dalloc(c, &L.H, 7 * n)) || (rc = dalloc(c, &L.Hf, 7 * n)) || (rc = dalloc(c, &L.zf, 3 * n)) ||
      (rc = dalloc(c, &L.zff, 3 * n)))
    return rc;
  double **vecs[3] = {(double **)&L.b, (double **)&L.x, (double **)&L.y};
  for (auto v : vecs)
    if ((rc = dalloc(c, v, n))) return rc;
  if (l == mesh->nlevels - 1 && (rc = dalloc(c, (double **)&L.w, n))) return rc;  // third Chebyshev iterate
  return HYB_OK;
}

void free_all(hyb_ctx *c) {
  for (auto &L : c->lv) {
    dfree(L.col_edge), dfree(L.edge_col), dfree(L.edge_lf), dfree(L.nbr), dfree(L.nlf), dfree(L.own);
    dfree(L.est), dfree(L.parent), dfree(L.children), dfree(L.H), dfree(L.Hf);
    dfree(L.zf), dfree(L.zff), dfree(L.b), dfree(L.x), dfree(L.y), dfree(L.w);
  }
  dfree(c->dz_d), dfree(c->corners_d), dfree(c->radius_d), dfree(c->vol), dfree(c->ck), dfree(c->A), dfree(c->LU), dfree(c->kv), dfree(c->Scell), dfree(c->bcell);
  dfree(c->ec);
  dfree(c->S), dfree(c->Sf), dfree(c->m2l), dfree(c->gamma), dfree(c->gammaf), dfree(c->zfac), dfree(c->zfacf);
  dfree(c->zfacp), dfree(c->zfacpf);
  dfree(c->tIn), dfree(c->tA), dfree(c->tB), dfree(c->tR), dfree(c->t64);
  dfree(c->V), dfree(c->Z), dfree(c->Vm), dfree(c->Zm), dfree(c->partial), dfree(c->hdev);
  if (c->hhost) (void)hipHostFree(c->hhost);
  c->hhost = nullptr;
  if (c->ev_coef) (void)hipEventDestroy(c->ev_coef);
  c->ev_coef = nullptr;
  for (auto &f : c->fam)
    for (auto ev : f.ev) (void)hipEventDestroy(ev);
  c->fam.clear();
  nn_free(c);
  p1_free(c);
  if (c->coarse) hyb_destroy(c->coarse), c->coarse = nullptr;
}

int alloc_krylov(hyb_ctx *c) {
  int m = c->p.restart;
  if (c->V && c->m == m) return HYB_OK;
  dfree(c->V), dfree(c->Z), dfree(c->partial), dfree(c->hdev);
  if (c->hhost) (void)hipHostFree(c->hhost);
  c->hhost = nullptr;
  c->m = m;
  size_t n = (size_t)c->ntrace;
  c->ldv = n + kBasisPad;
  int rc;
  c->nblk_red = reduction_blocks();
  if ((rc = dalloc(c, &c->V, (size_t)(m + 1) * c->ldv)) || (rc = dalloc(c, (double **)&c->Z, (size_t)m * c->ldv)) ||
      (rc = dalloc(c, &c->partial, (size_t)c->nblk_red * 2 * (m + 2))) || (rc = dalloc(c, &c->hdev, 4 * (size_t)(m + 2))))
    return rc;
  CHECK_HIP(hipHostMalloc((void **)&c->hhost, 4 * (size_t)(m + 2) * sizeof(double), hipHostMallocDefault),
            "hipHostMalloc");
  if (!c->ev_coef) CHECK_HIP(hipEventCreateWithFlags(&c->ev_coef, hipEventDisableTiming), "hipEventCreate");
  const size_t hm = (size_t)(m + 1) * m;
  c->kR.assign(hm, 0.0), c->kHr.assign(hm, 0.0), c->kg.assign(m + 1, 0.0);
  c->kcs.assign(m, 0.0), c->ksn.assign(m, 0.0), c->ky.assign(m, 0.0), c->kca.assign(m, 0.0), c->kcb.assign(m, 0.0);
  return HYB_OK;
}

// Flexible GMRES(m) from x on n-vectors, right preconditioned, FP64 basis V [(m+1)][ldv] and
// preconditioned basis Z [m][ldv] (FP32 when zf32).  resid(V0) writes b - A x into V0 (not called
// while x is zero); apply(j) writes Z_j = M V_j and V_{j+1} = A Z_j.  Returns the status
// (HYB_OK, HYB_NOT_CONVERGED, HYB_BREAKDOWN) or a negative error code.
template <typename Resid, typename Apply>
int fgmres(hyb_ctx *c, size_t n, size_t ldv, double *V, void *Zbuf, bool zf32, const double *b, double *x, double rtol,
           int32_t maxit, hyb_info *info, Resid resid, Apply apply_op) {
  const int m = c->m;
  int rc = 0;
  double *h1 = c->hdev, *h2 = c->hdev + (m + 2), *nrm = c->hdev + 2 * (m + 2);
  double *hh = c->hhost;
  std::vector<double> &R = c->kR, &g = c->kg, &cs = c->kcs, &sn = c->ksn, &y = c->ky;
  if (R.size() < (size_t)(m + 1) * m || g.size() < (size_t)m + 1)
    return fail(c, HYB_ESTATE, "the Krylov workspace does not match the restart length");
  std::fill(R.begin(), R.end(), 0.0);
  if (info) {
    info->iters = 0, info->restarts = 0, info->history_len = 0, info->rel_res = 0, info->status = HYB_OK;
    info->fallbacks = 0;
  }
  // ||b|| and ||lambda_0||^2: from a zero initial guess the first residual is b itself
  CHECK_HIP(launch_multidot(c, b, 0, 0, b, n, nrm, true), "norm b");
  CHECK_HIP(launch_multidot(c, x, 0, 0, x, n, nrm + 1, true), "norm x");
  CHECK_HIP(hipMemcpyAsync(hh, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "d2h");
  CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
  double bnorm = std::sqrt(hh[0]);
  bool x_zero = hh[1] == 0.0;
  if (!std::isfinite(bnorm)) return fail(c, HYB_EINVAL, "right-hand side is not finite");
  if (bnorm == 0.0) {
    CHECK_HIP(launch_fill(c, x, n, 0.0), "zero");
    return HYB_OK;
  }
  int its = 0, restarts = 0, status = HYB_NOT_CONVERGED;
  double rel = 0.0, rel_cycle = 0.0;
  int stalled = 0;  // consecutive restart cycles that left the true residual almost where it was
  for (;;) {
    // true residual r = b - S lam into V_0
    if (x_zero)
      CHECK_HIP(hipMemcpyAsync(V, b, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "residual");
    else if ((rc = resid(V)))
      return rc;
    x_zero = false;
    CHECK_HIP(launch_multidot(c, V, 0, 0, V, n, nrm, true), "norm r");
    CHECK_HIP(hipMemcpyAsync(hh, nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream), "d2h");
    CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
    double beta = std::sqrt(hh[0]);
    rel = beta / bnorm;
    if (!std::isfinite(rel)) {
      status = HYB_BREAKDOWN;
      break;
    }
    if (rel <= rtol) {
      status = HYB_OK;
      break;
    }
    if (its >= maxit) break;
    // a restart cycle that reduced the true residual by less than kStagnation twice in a row (the
    // rounding floor of the residual, or a preconditioned operator the cycle cannot reduce) ends
    // the solve instead of running on to maxit
    if (its > 0) {
      stalled = rel > kStagnation * rel_cycle ? stalled + 1 : 0;
      if (stalled >= 2) {
        status = HYB_STAGNATED;
        break;
      }
    }
    rel_cycle = rel;
    if (its > 0) restarts++;
    CHECK_HIP(launch_scale(c, V, n, 1.0 / beta), "scale");
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    bool breakdown = false;
    if (m <= kDgsMax) {
      // Arnoldi with classical Gram-Schmidt and delayed reorthogonalisation: step j applies the
      // operator to V_j as orthogonalised once in step j - 1 (scaled by the estimated norm eta),
      // then one reduction pass gives the dots that finish V_j (second orthogonalisation, exact
      // norm rho) and orthogonalise w once, and one update pass writes both.  Column j - 1 of the
      // Hessenberg matrix is completed with eta_j a and eta_j rho; the Givens QR of the columns
      // so far is redone every step from the unrotated matrix Hr.
      std::vector<double> &Hr = c->kHr, &ca = c->kca, &cb = c->kcb;
      std::fill(Hr.begin(), Hr.end(), 0.0);
      double eta_prev = 1.0, g0 = beta;
      for (int j = 0; j < m; ++j) {
        if ((rc = apply_op(j))) return rc;
        // dots, then the step's coefficients on the device, whose read-back is queued before the
        // update pass that uses them: the host waits for the read-back only, and its Hessenberg
        // and Givens work below overlaps the update pass
        double *coef = c->hdev + 2 * (size_t)(m + 2);
        const double *hc = hh + 2 * (size_t)(m + 2);
        CHECK_HIP(launch_dgs_dots(c, V, ldv, n, j, c->hdev), "gram-schmidt dots");
        CHECK_HIP(launch_dgs_coef(c, c->hdev, j, coef), "gram-schmidt coefficients");
        CHECK_HIP(hipMemcpyAsync((void *)hc, coef, (2 * (size_t)j + 6) * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream),
                  "d2h");
        CHECK_HIP(hipEventRecord(c->ev_coef, c->stream), "event");
        CHECK_HIP(launch_dgs_update(c, V, ldv, n, j, coef, zf32 ? (float *)c->tIn : nullptr), "gram-schmidt update");
        CHECK_HIP(hipEventSynchronize(c->ev_coef), "event sync");
        if (hc[2 * j + 3] != 0.0) {  // rho^2 not positive: the update pass wrote nothing
          breakdown = true;
          break;
        }
        for (int k = 0; k < j; ++k) ca[k] = hc[k], cb[k] = hc[j + k];
        const double rho = hc[2 * j];
        if (j == 0) {
          g0 = beta * rho;  // r = beta V_0 (as scaled) = beta rho v_0
        } else {
          double *prev = &Hr[(size_t)(j - 1) * (m + 1)];
          for (int k = 0; k < j; ++k) prev[k] += eta_prev * ca[k];
          prev[j] = eta_prev * rho;
        }
        double *col = &Hr[(size_t)j * (m + 1)];
        const double hjj = hc[2 * j + 1];
        for (int k = 0; k < j; ++k) col[k] = cb[k];
        col[j] = hjj;
        const double eta = hc[2 * j + 2];
        col[j + 1] = eta;
        eta_prev = eta;
        // Givens QR of columns 0..j
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = g0;
        bool bad = false;
        for (int q = 0; q <= j; ++q) {
          double *rq = &R[(size_t)q * (m + 1)];
          const double *hq = &Hr[(size_t)q * (m + 1)];
          for (int i = 0; i <= q + 1; ++i) rq[i] = hq[i];
          for (int i = 0; i < q; ++i) {
            const double x = rq[i], z = rq[i + 1];
            rq[i] = cs[i] * x + sn[i] * z;
            rq[i + 1] = -sn[i] * x + cs[i] * z;
          }
          const double rr = std::hypot(rq[q], rq[q + 1]);
          if (!(rr > 0) || !std::isfinite(rr)) {
            bad = true;
            break;
          }
          cs[q] = rq[q] / rr;
          sn[q] = rq[q + 1] / rr;
          rq[q] = rr;
          rq[q + 1] = 0.0;
          g[q + 1] = -sn[q] * g[q];
          g[q] = cs[q] * g[q];
        }
        if (bad) {
          breakdown = true;
          break;
        }
        its++;
        jend = j + 1;
        const double est = std::fabs(g[j + 1]) / bnorm;
        if (info && info->history && info->history_len < info->history_cap) info->history[info->history_len++] = est;
        if (!std::isfinite(est)) {
          breakdown = true;
          break;
        }
        if (est <= rtol || its >= maxit || eta == 0.0) break;
      }
    } else
    for (int j = 0; j < m; ++j) {
      double *w = V + (size_t)(j + 1) * ldv;
      if ((rc = apply_op(j))) return rc;
      double *col = &R[(size_t)j * (m + 1)];
      double hn;
      bool scaled = false;
      if (j + 1 <= 32) {
        // classical Gram-Schmidt with reorthogonalisation in three passes over the basis and one
        // host read: h1 = V^T w; w -= V h1 while h2 = V^T w and ||w||^2 accumulate; the last pass
        // subtracts V h2 and normalises with ||w - V h2||^2 = ||w||^2 - ||h2||^2 (V orthonormal)
        CHECK_HIP(launch_gs_passes(c, V, ldv, n, j + 1, w, h1, h2), "gram-schmidt");
        CHECK_HIP(hipMemcpyAsync(hh, c->hdev, 2 * (size_t)(m + 2) * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream),
                  "d2h");
        CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
        double h2sq = 0.0;
        for (int i = 0; i <= j; ++i) {
          col[i] = hh[i] + hh[(m + 2) + i];
          h2sq += hh[(m + 2) + i] * hh[(m + 2) + i];
        }
        double wp2 = hh[(m + 2) + j + 1];
        hn = std::sqrt(std::max(0.0, wp2 - h2sq));
        if (hn > 0.0 && std::isfinite(hn)) {
          CHECK_HIP(launch_gs_finish(c, V, ldv, n, j + 1, h2, w, 1.0 / hn), "gram-schmidt finish");
          scaled = true;
        }
      } else {
        // long restart cycles: classical Gram-Schmidt, second pass when the first one cancelled
        // more than half of the norm (||w'|| < ||w|| / sqrt(2))
        CHECK_HIP(launch_multidot(c, V, ldv, j + 1, w, n, h1, true), "cgs1");
        CHECK_HIP(launch_axpy_norm(c, V, ldv, j + 1, h1, w, n, nrm), "cgs1 update");
        CHECK_HIP(hipMemcpyAsync(hh, c->hdev, 3 * (size_t)(m + 2) * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream),
                  "d2h");
        CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
        for (int i = 0; i <= j; ++i) col[i] = hh[i];
        double w2 = hh[j + 1], wp2 = hh[2 * (m + 2)];
        if (!(wp2 >= 0.5 * w2)) {
          CHECK_HIP(launch_multidot(c, V, ldv, j + 1, w, n, h2, false), "cgs2");
          CHECK_HIP(launch_axpy_norm(c, V, ldv, j + 1, h2, w, n, nrm), "cgs2 update");
          CHECK_HIP(hipMemcpyAsync(hh, c->hdev, 3 * (size_t)(m + 2) * sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream),
                    "d2h");
          CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
          for (int i = 0; i <= j; ++i) col[i] += hh[(m + 2) + i];
          wp2 = hh[2 * (m + 2)];
          c->reorth++;
        }
        hn = std::sqrt(wp2);
      }
      col[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        double a = col[i], bb = col[i + 1];
        col[i] = cs[i] * a + sn[i] * bb;
        col[i + 1] = -sn[i] * a + cs[i] * bb;
      }
      double a = col[j], bb = col[j + 1];
      double rr = std::hypot(a, bb);
      if (!(rr > 0) || !std::isfinite(rr)) {
        breakdown = true;
        jend = j;
        break;
      }
      cs[j] = a / rr;
      sn[j] = bb / rr;
      col[j] = rr;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      its++;
      jend = j + 1;
      double est = std::fabs(g[j + 1]) / bnorm;
      if (info && info->history && info->history_len < info->history_cap) info->history[info->history_len++] = est;
      if (!std::isfinite(est)) {
        breakdown = true;
        break;
      }
      if (est <= rtol || its >= maxit || hn == 0.0) break;
      if (!scaled) CHECK_HIP(launch_scale(c, w, n, 1.0 / hn), "scale");
    }
    if (jend > 0) {
      for (int i = jend - 1; i >= 0; --i) {
        double s = g[i];
        for (int k = i + 1; k < jend; ++k) s -= R[(size_t)k * (m + 1) + i] * y[k];
        y[i] = s / R[(size_t)i * (m + 1) + i];
      }
      // y goes to the device through the pinned buffer (after the last sync the buffer is free)
      std::copy(y.begin(), y.begin() + jend, hh + 3 * (m + 2));
      double *ydev = c->hdev + 3 * (m + 2);
      CHECK_HIP(hipMemcpyAsync(ydev, hh + 3 * (m + 2), jend * sizeof(double), hipMemcpyHostToDevice, c->stream),
                "h2d");
      if (zf32)
        CHECK_HIP(launch_update_solution<float>(c, (const float *)Zbuf, ldv, jend, ydev, x, n), "update");
      else
        CHECK_HIP(launch_update_solution<double>(c, (const double *)Zbuf, ldv, jend, ydev, x, n), "update");
      CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
    }
    if (breakdown && jend == 0) {
      status = HYB_BREAKDOWN;
      break;
    }
  }
  if (info) {
    info->iters = its;
    info->restarts = restarts;
    info->rel_res = rel;
    info->status = status;
  }
  return status;
}

}  // namespace

namespace hyb {

int prof_begin(hyb_ctx *c, int fam) {
  if (!c->prof || !((c->prof_mask >> fam) & 1)) return -1;
  ProfFamily &f = c->fam[fam];
  if (f.used + 2 > f.ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) return -1;
      f.ev.push_back(ev);
    }
  }
  int slot = (int)f.used;
  f.used += 2;
  (void)hipEventRecord(f.ev[slot], c->stream);
  return slot;
}

void prof_end(hyb_ctx *c, int fam, int slot) {
  if (slot < 0) return;
  (void)hipEventRecord(c->fam[fam].ev[slot + 1], c->stream);
}

}  // namespace hyb

extern "C" {

int hyb_create(const hyb_mesh *mesh, const hyb_params *params, void *stream, hyb_ctx **out) {
  if (!out) return HYB_EINVAL;
  *out = nullptr;
  hyb_ctx *c = new (std::nothrow) hyb_ctx();
  if (!c) return HYB_ENOMEM;
  if (!mesh || mesh->nlev < 1 || mesh->nlevels < 1 || !mesh->levels) {
    delete c;
    return HYB_EINVAL;
  }
  c->geom = mesh->geom;
  int rc = check_params(c, params);
  if (rc) {
    delete c;
    return rc;
  }
  bool geom_ok = false;
  if (mesh->geom == HYB_GEOM_BOX) {
    geom_ok = mesh->dz && mesh->dx > 0 && mesh->dy > 0;
  } else if (mesh->geom == HYB_GEOM_SHELL) {
    geom_ok = mesh->corners && mesh->radius && mesh->order == 0 && mesh->radius[0] > 0;
    for (int k = 0; geom_ok && k < mesh->nlev; ++k) geom_ok = mesh->radius[k + 1] > mesh->radius[k];
    for (size_t i = 0; geom_ok && i < (size_t)12 * mesh->levels[0].ncol; ++i) geom_ok = std::isfinite(mesh->corners[i]);
    // every column frame must turn the same way seen from outside (a positive cell Jacobian):
    // (c1 - c0) x (c2 - c0) points outwards, along the sum of the corners
    const size_t nc = mesh->levels[0].ncol;
    for (size_t col = 0; geom_ok && col < nc; ++col) {
      double q[4][3];
      for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) q[a][d] = mesh->corners[((size_t)a * 3 + d) * nc + col];
      double u[3], v[3], m[3];
      for (int d = 0; d < 3; ++d) u[d] = q[1][d] - q[0][d], v[d] = q[2][d] - q[0][d], m[d] = q[0][d] + q[1][d] + q[2][d] + q[3][d];
      const double nx = u[1] * v[2] - u[2] * v[1], ny = u[2] * v[0] - u[0] * v[2], nz = u[0] * v[1] - u[1] * v[0];
      geom_ok = nx * m[0] + ny * m[1] + nz * m[2] > 0.0;
    }
  }
  if (!geom_ok) {
    delete c;
    return HYB_EINVAL;
  }
  c->p = *params;
  c->stream = (hipStream_t)stream;
  c->nlev = mesh->nlev;
  c->nlevels = mesh->nlevels;
  c->ncol = mesh->levels[0].ncol;
  c->nedge = 2 * c->ncol;
  c->ncell = c->nlev * c->ncol;
  c->nz = (c->nlev + 1) * c->ncol;
  c->ntrace = c->nz + c->nlev * c->nedge;
  if (mesh->order != 0 && mesh->order != 1) {
    delete c;
    return HYB_EINVAL;
  }
  c->order = mesh->order;
  if (params->smoother_patch && (c->order != 0 || c->nlevels < 2)) {
    delete c;
    return HYB_EINVAL;  // patch-cached column matrices: order 0 with a multigrid level of patches
  }
  if (c->order == 1) c->ntrace *= 4;
  if (c->order == 1 && params->coarse_mode == 2) {
    delete c;
    return HYB_EINVAL;  // the Krylov coarse solve is an order-0 FP64 mode
  }
  {
    const bool mfma = params->precision == HYB_PREC_MFMA_FP32 || params->precision == HYB_PREC_MFMA_BF16X;
    // MFMA condensation is an order-1 mode
    if (c->order == 0 && mfma) {
      delete c;
      return HYB_EINVAL;
    }
  }
  c->dx = mesh->dx;
  c->dy = mesh->dy;
  if (c->geom == HYB_GEOM_SHELL) {
    c->dz.resize(c->nlev);
    for (int k = 0; k < c->nlev; ++k) c->dz[k] = mesh->radius[k + 1] - mesh->radius[k];
  } else {
    c->dz.assign(mesh->dz, mesh->dz + c->nlev);
  }
  for (double d : c->dz)
    if (!(d > 0)) {
      delete c;
      return HYB_EINVAL;
    }
  if ((size_t)c->ntrace * 11 > (size_t)INT64_MAX / 8) {
    delete c;
    return HYB_EINVAL;
  }
  if ((size_t)sizeof(double) * (c->nlev + 1) * kColBlock > 160 * 1024) {
    delete c;
    return HYB_EINVAL;  // column coefficients must fit in the 160 KiB LDS of a CU
  }
  if (configure_kernels(c->nlev) != hipSuccess) {
    delete c;
    return HYB_EHIP;
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return HYB_EHIP;
  }
  {
    std::string why;
    c->scratch = scratch_address(c->device, &why);
    if (!c->scratch) c->scratch_err = why;  // reported by hyb_solve_noalloc; no other call needs it
  }
  c->fam.resize(F_COUNT);
  for (int i = 0; i < F_COUNT; ++i) c->fam[i].name = kFamilyNames[i];
  c->lv.resize(c->nlevels);
  for (int l = 0; l < c->nlevels && rc == HYB_OK; ++l) rc = setup_level(c, mesh, l);
  if (rc == HYB_OK) {
    rc = dalloc(c, &c->dz_d, c->nlev);
    if (rc == HYB_OK && hipMemcpy(c->dz_d, c->dz.data(), c->nlev * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      rc = HYB_EHIP;
  }
  if (rc == HYB_OK && c->geom == HYB_GEOM_SHELL) {
    const size_t nco = (size_t)12 * c->ncol;
    rc = dalloc(c, &c->corners_d, nco);
    if (rc == HYB_OK) rc = dalloc(c, &c->radius_d, (size_t)c->nlev + 1);
    if (rc == HYB_OK && (hipMemcpy(c->corners_d, mesh->corners, nco * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
                         hipMemcpy(c->radius_d, mesh->radius, (c->nlev + 1) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess))
      rc = fail(c, HYB_EHIP, "upload of the shell geometry");
  }
  if (rc != HYB_OK) {
    fprintf(stderr, "hyb_create: %s\n", c->err.c_str());
    free_all(c);
    delete c;
    return rc;
  }
  if (c->order == 1) {
    // the DG0 coarse space: an order-0 context on the same mesh (its pressure operator H, the
    // multigrid hierarchy and its V-cycle)
    hyb_mesh m0 = *mesh;
    m0.order = 0;
    hyb_params p0 = *params;
    p0.precision = HYB_PREC_FP64;
    p0.learned = 0;
    rc = hyb_create(&m0, &p0, stream, &c->coarse);
    if (rc != HYB_OK) {
      free_all(c);
      delete c;
      return rc;
    }
  }
  *out = c;
  return HYB_OK;
}

int hyb_set_params(hyb_ctx *c, const hyb_params *params) {
  if (!c) return HYB_EINVAL;
  int rc = check_params(c, params);
  if (rc) return rc;
  bool prec_change = params->precision != c->p.precision;
  if (c->order == 1) {
    if (params->learned) return fail(c, HYB_EINVAL, "order 1 has no learned stage");
    hyb_params p0 = *params;
    p0.precision = HYB_PREC_FP64;
    if ((rc = hyb_set_params(c->coarse, &p0))) return fail(c, rc, std::string("coarse space: ") + hyb_last_error(c->coarse));
    c->p = *params;
    if (prec_change) c->condensed = false;  // condense again in the new arithmetic
    return HYB_OK;
  }
  if (params->precision == HYB_PREC_MFMA_FP32 || params->precision == HYB_PREC_MFMA_BF16X)
    return fail(c, HYB_EINVAL, "MFMA condensation is an order-1 mode");
  c->p = *params;
  if (prec_change && c->condensed && c->p.precision == HYB_PREC_MIXED) {
    // FP32 copies are made at condensation; refresh them for the new mode
    CHECK_HIP(launch_to_float(c, c->S, c->Sf, s_entries(c->ntrace)), "to_float S");
    CHECK_HIP(launch_to_float(c, c->gamma, c->gammaf, (size_t)c->ncell), "to_float gamma");
    CHECK_HIP(launch_to_float(c, c->zfac, c->zfacf, 3 * (size_t)c->nz), "to_float zfac");
    if (c->zfacp)
      CHECK_HIP(launch_to_float(c, c->zfacp, c->zfacpf, 3 * (size_t)(c->nlev + 1) * c->lv[1].ncol), "to_float zfacp");
    for (int l = 0; l < c->nlevels; ++l)
    {
      CHECK_HIP(launch_to_float(c, c->lv[l].H, c->lv[l].Hf, (size_t)7 * c->nlev * c->lv[l].ncol), "to_float H");
      CHECK_HIP(launch_to_float(c, c->lv[l].zf, c->lv[l].zff, (size_t)3 * c->nlev * c->lv[l].ncol), "to_float Hz");
    }
  }
  return alloc_krylov(c);
}

int hyb_assemble_local(hyb_ctx *c, const double *theta_w, const double *exner_hat_w, const double *exner_c,
                       const double *rho_c) {
  if (!c) return HYB_EINVAL;
  if (!theta_w || !exner_hat_w || !exner_c || !rho_c) return fail(c, HYB_EINVAL, "null field");
  int rc;
  if (c->order == 1) {
    hyb::P1State &s = c->p1;
    const size_t nc = (size_t)c->ncell;
    if ((rc = dalloc(c, &s.A, 748 * nc)) || (rc = dalloc(c, &s.cdiag, 24 * nc)) ||
        (rc = dalloc(c, &s.kdiag, 24 * nc)) || (rc = dalloc(c, &s.SK, 24 * 24 * nc)) || (rc = dalloc(c, &s.bK, 24 * nc)) ||
        (rc = dalloc(c, &s.fac, 748 * nc)) || (rc = dalloc(c, &s.SKf, 24 * 24 * nc)))
      return rc;
    CHECK_HIP(p1_setup(c), "p1 tables");
    CHECK_HIP(p1_assemble(c, theta_w, exner_hat_w, exner_c, rho_c), "p1 assemble_local");
    if ((rc = hyb_assemble_local(c->coarse, theta_w, exner_hat_w, exner_c, rho_c)))
      return fail(c, rc, std::string("coarse space: ") + hyb_last_error(c->coarse));
    c->assembled = true;
    c->condensed = false;
    return HYB_OK;
  }
  if ((rc = dalloc(c, &c->A, (size_t)49 * c->ncell)) || (rc = dalloc(c, &c->kv, (size_t)6 * c->ncell)) ||
      (rc = dalloc(c, &c->m2l, (size_t)c->ntrace)) || (rc = dalloc(c, &c->vol, (size_t)c->ncell)) ||
      (rc = dalloc(c, &c->ec, (size_t)8 * c->ncell)))
    return rc;
  c->nn.st_ready = false;  // the network's static inputs follow the cell volumes
  // the lumped velocity mass (Sec. 2.3) leaves the Coriolis term out: on the sphere the assembly
  // writes each cell's share of it (row sums before the term is added) to a temporary array
  if (c->geom == HYB_GEOM_SHELL) {
    double *rs = nullptr;
    if ((rc = dalloc(c, &rs, (size_t)6 * c->ncell))) return rc;
    hipError_t e = launch_assemble_shell(c, theta_w, exner_hat_w, exner_c, rs);
    if (e == hipSuccess) e = launch_lumped_mass(c, rs);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // before the temporary is freed
    c->bytes -= (size_t)6 * c->ncell * sizeof(double);
    dfree(rs);
    CHECK_HIP(e, "assemble_local");
  } else {
    CHECK_HIP(launch_assemble_box(c, theta_w, exner_hat_w, exner_c, rho_c), "assemble_local");
    CHECK_HIP(launch_lumped_mass(c), "lumped_mass");
  }
  // the theta' / rho' elimination needs the reference state after the call returns
  CHECK_HIP(launch_elim_coeffs(c, theta_w, exner_hat_w, rho_c), "elimination coefficients");
  c->assembled = true;
  c->condensed = false;
  return HYB_OK;
}

int hyb_condense(hyb_ctx *c, const double *r_ub, const double *r_pi, double *b_lambda) {
  if (!c) return HYB_EINVAL;
  if (!c->assembled) return fail(c, HYB_ESTATE, "condense before assemble_local");
  int rc;
  if (c->order == 1) {
    if (r_ub == nullptr) {
      if (c->condensed) return HYB_OK;
      if ((rc = hyb_condense(c->coarse, nullptr, nullptr, nullptr)))
        return fail(c, rc, std::string("coarse space: ") + hyb_last_error(c->coarse));
      CHECK_HIP(p1_factor(c), "p1 factor");
      hyb::P1State &s = c->p1;
      const size_t ntr = (size_t)c->ntrace, nc = (size_t)c->ncell;
      if ((rc = dalloc(c, &s.dS, ntr)) || (rc = dalloc(c, &s.zf, 48 * (size_t)c->nz)) ||
          (rc = dalloc(c, &s.gamma, nc)) || (rc = dalloc(c, &s.den, nc)) || (rc = dalloc(c, &s.t1, ntr)) ||
          (rc = dalloc(c, &s.t2, ntr)) || (rc = dalloc(c, &s.t3, ntr)))
        return rc;
      CHECK_HIP(p1_precond_setup(c), "p1 preconditioner setup");
      if ((rc = alloc_krylov(c))) return rc;
      CHECK_HIP(hipStreamSynchronize(c->stream), "condense sync");
      c->condensed = true;
      return HYB_OK;
    }
    if (!c->condensed) return fail(c, HYB_ESTATE, "condense the operator (r_ub = NULL) first");
    if (!r_pi || !b_lambda) return fail(c, HYB_EINVAL, "null argument");
    CHECK_HIP(p1_cell_solve(c, r_ub, r_pi, nullptr, 0, nullptr, nullptr), "p1 condense rhs");
    CHECK_HIP(p1_rows(c, nullptr, b_lambda, 1, nullptr), "p1 gather rhs");
    return HYB_OK;
  }
  if (r_ub == nullptr) {
    size_t ntr = (size_t)c->ntrace, nc = (size_t)c->ncell;
    if ((rc = dalloc(c, &c->LU, 49 * nc)) || (rc = dalloc(c, &c->Scell, 36 * nc)) || (rc = dalloc(c, &c->S, s_entries(ntr))) ||
        (rc = dalloc(c, &c->Sf, s_entries(ntr))) || (rc = dalloc(c, &c->gamma, nc)) ||
        (rc = dalloc(c, &c->zfac, 3 * (size_t)c->nz)) || (rc = dalloc(c, &c->zfacf, 3 * (size_t)c->nz)) ||
        (c->nlevels > 1 && (rc = dalloc(c, &c->zfacp, 3 * (size_t)(c->nlev + 1) * c->lv[1].ncol))) ||
        (c->nlevels > 1 && (rc = dalloc(c, &c->zfacpf, 3 * (size_t)(c->nlev + 1) * c->lv[1].ncol))) ||
        (rc = dalloc(c, &c->gammaf, nc)) || (rc = dalloc(c, &c->bcell, 6 * nc)) ||
        (rc = dalloc(c, (double **)&c->tIn, ntr)) || (rc = dalloc(c, (double **)&c->tA, ntr)) ||
        (rc = dalloc(c, (double **)&c->tB, ntr)) || (rc = dalloc(c, (double **)&c->tR, ntr)) ||
        (rc = dalloc(c, &c->t64, ntr)))
      return rc;
    if ((rc = alloc_krylov(c))) return rc;
    CHECK_HIP(launch_factor_cells(c), "factor_cells");
    CHECK_HIP(launch_build_stencil(c), "build_stencil");
    CHECK_HIP(launch_thomas_factor(c), "thomas_factor");
    CHECK_HIP(launch_pressure_stencil(c), "pressure_stencil");
    for (int l = 1; l < c->nlevels; ++l) CHECK_HIP(launch_galerkin(c, l), "galerkin");
    for (int l = 0; l < c->nlevels; ++l) CHECK_HIP(launch_mg_factor(c, l), "mg_factor");
    CHECK_HIP(launch_gamma(c), "gamma");
    CHECK_HIP(launch_to_float(c, c->S, c->Sf, s_entries(ntr)), "to_float S");
    CHECK_HIP(launch_to_float(c, c->gamma, c->gammaf, nc), "to_float gamma");
    CHECK_HIP(launch_to_float(c, c->zfac, c->zfacf, 3 * (size_t)c->nz), "to_float zfac");
    if (c->zfacp)
      CHECK_HIP(launch_to_float(c, c->zfacp, c->zfacpf, 3 * (size_t)(c->nlev + 1) * c->lv[1].ncol), "to_float zfacp");
    for (int l = 0; l < c->nlevels; ++l)
    {
      CHECK_HIP(launch_to_float(c, c->lv[l].H, c->lv[l].Hf, (size_t)7 * c->nlev * c->lv[l].ncol), "to_float H");
      CHECK_HIP(launch_to_float(c, c->lv[l].zf, c->lv[l].zff, (size_t)3 * c->nlev * c->lv[l].ncol), "to_float Hz");
    }
    CHECK_HIP(hipStreamSynchronize(c->stream), "condense sync");
    dfree(c->Scell);
    c->condensed = true;
    return HYB_OK;
  }
  if (!c->condensed) return fail(c, HYB_ESTATE, "condense the operator (r_ub = NULL) first");
  if (!r_pi || !b_lambda) return fail(c, HYB_EINVAL, "null argument");
  CHECK_HIP(launch_cell_rhs(c, r_ub, r_pi, b_lambda), "condense rhs");
  return HYB_OK;
}

int hyb_trace_apply(hyb_ctx *c, const double *x, double *y) {
  if (!c) return HYB_EINVAL;
  if (!c->condensed) return fail(c, HYB_ESTATE, "trace_apply before condense");
  if (!x || !y || x == y) return fail(c, HYB_EINVAL, "bad vectors");
  if (c->order == 1) {
    CHECK_HIP(p1_rows(c, x, y, 0, nullptr), "p1 trace_apply");
    return HYB_OK;
  }
  CHECK_HIP((launch_trace_apply<double, double, double>(c, c->S, x, nullptr, y, 0)), "trace_apply");
  return HYB_OK;
}

int hyb_precondition(hyb_ctx *c, const double *r, double *z) {
  if (!c) return HYB_EINVAL;
  if (c->order == 1) {
    if (!c->condensed) return fail(c, HYB_ESTATE, "precondition before condense");
    if (!r || !z || r == z) return fail(c, HYB_EINVAL, "bad vectors");
    CHECK_HIP(p1_precondition(c, r, z), "p1 precondition");
    return HYB_OK;
  }
  if (!c->condensed) return fail(c, HYB_ESTATE, "precondition before condense");
  if (!r || !z || r == z) return fail(c, HYB_EINVAL, "bad vectors");
  if (c->p.learned && !c->nn.loaded) return fail(c, HYB_ESTATE, "learned stage requested without weights");
  if (c->p.learned || c->p.precision != HYB_PREC_FP64) {
    // the learned stage reduces into the Krylov scratch; the FP32 path uses the first basis slot of Z
    int rc = alloc_krylov(c);
    if (rc) return rc;
  }
  if (c->p.precision == HYB_PREC_FP64) {
    CHECK_HIP(precondition<double>(c, r, z), "precondition");
    if (c->p.learned) CHECK_HIP(learned_stage<double>(c, r, z), "learned stage");
  } else {
    size_t n = (size_t)c->ntrace;
    float *rf = (float *)c->tIn;
    float *zf = (float *)c->Z;
    CHECK_HIP(launch_convert(c, r, rf, n), "convert");
    CHECK_HIP(precondition<float>(c, rf, zf), "precondition");
    if (c->p.learned) CHECK_HIP(learned_stage<float>(c, r, zf), "learned stage");
    CHECK_HIP(launch_copy_widen(c, zf, z, n), "widen");
  }
  return HYB_OK;
}

namespace {

// FGMRES on the trace system with the context's Krylov basis (allocated) and the reduction
// buffers c->partial / c->hdev (the context's own, or the static scratch).
int solve_impl(hyb_ctx *c, const double *b, double *lam, double rtol, int32_t maxit, hyb_info *info) {
  const size_t n = (size_t)c->ntrace;
  const int m = c->m;
  // the order-0 mixed form keeps the preconditioned basis Z in FP32 (at order 1 the mixed form only
  // changes the preconditioner's copy of S_K, and Z stays FP64)
  const bool mixed = c->p.precision == HYB_PREC_MIXED && c->order == 0;
  double *V = c->V;
  const bool learned = c->p.learned && c->nn.loaded;
  if (c->p.learned && !c->nn.loaded) return fail(c, HYB_ESTATE, "learned stage requested without weights");
  double fb0 = 0.0;
  if (learned && c->nn.scal) {
    CHECK_HIP(hipMemcpyAsync(&fb0, c->nn.scal + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream), "d2h");
    CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
  }
  auto resid = [&](double *V0) -> int {
    if (c->order == 1)
      CHECK_HIP(p1_rows(c, lam, V0, 2, b), "residual");
    else
      CHECK_HIP((launch_trace_apply<double, double, double>(c, c->S, lam, b, V0, 1)), "residual");
    return HYB_OK;
  };
  // z_j = M(V_j) into Z, w = S z_j into V_{j+1}
  auto apply_op = [&](int j) -> int {
    const size_t ldv = c->ldv;
    double *vj = V + (size_t)j * ldv, *w = V + (size_t)(j + 1) * ldv;
    if (mixed) {
      float *zf = (float *)c->Z + (size_t)j * ldv;
      // the two-pass Gram-Schmidt writes the FP32 copy of V_j with V_j itself (steps j > 0)
      if (j == 0 || m > kDgsMax) CHECK_HIP(launch_convert(c, vj, (float *)c->tIn, n), "convert");
      CHECK_HIP(precondition<float>(c, (const float *)c->tIn, zf), "precondition");
      if (learned) CHECK_HIP(learned_stage<float>(c, vj, zf), "learned stage");
      CHECK_HIP((launch_trace_apply<double, float, double>(c, c->S, zf, nullptr, w, 0)), "matvec");
    } else if (c->order == 1) {
      double *zj = (double *)c->Z + (size_t)j * ldv;
      CHECK_HIP(p1_precondition(c, vj, zj), "precondition");
      CHECK_HIP(p1_rows(c, zj, w, 0, nullptr), "matvec");
    } else {
      double *zj = (double *)c->Z + (size_t)j * ldv;
      CHECK_HIP(precondition<double>(c, vj, zj), "precondition");
      if (learned)  // the stage's own applications of S give w = S z (no separate matvec)
        CHECK_HIP(learned_stage<double>(c, vj, zj, w), "learned stage");
      else
        CHECK_HIP((launch_trace_apply<double, double, double>(c, c->S, zj, nullptr, w, 0)), "matvec");
    }
    return HYB_OK;
  };
  const int status = fgmres(c, n, c->ldv, V, c->Z, mixed, b, lam, rtol, maxit, info, resid, apply_op);
  if (status >= 0 && info && learned) {
    double fb = 0.0;
    CHECK_HIP(hipMemcpyAsync(&fb, c->nn.scal + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream), "d2h");
    CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
    info->fallbacks = (int32_t)(fb - fb0);
  }
  (void)m;
  return status;
}

}  // namespace

int hyb_solve(hyb_ctx *c, const double *b, double *lam, double rtol, int32_t maxit, hyb_info *info) {
  if (!c) return HYB_EINVAL;
  if (!c->condensed) return fail(c, HYB_ESTATE, "solve before condense");
  if (!b || !lam || b == lam || !(rtol >= 0) || maxit < 0) return fail(c, HYB_EINVAL, "bad solve arguments");
  int rc = alloc_krylov(c);
  if (rc) return rc;
  return solve_impl(c, b, lam, rtol, maxit, info);
}

int hyb_solve_noalloc(hyb_ctx *c, const double *b, double *lam, double rtol, int32_t maxit, hyb_info *info) {
  if (!c) return HYB_EINVAL;
  if (!c->condensed) return fail(c, HYB_ESTATE, "solve before condense");
  if (!b || !lam || b == lam || !(rtol >= 0) || maxit < 0) return fail(c, HYB_EINVAL, "bad solve arguments");
  if (c->order != 0 || c->p.learned || c->p.coarse_mode == 2)
    return fail(c, HYB_EINVAL,
                "hyb_solve_noalloc covers order 0 without the learned stage or the Krylov coarse solve");
  if (c->prof) return fail(c, HYB_ESTATE, "hyb_solve_noalloc does not record profiling events");
  if (!c->V || !c->Z || !c->hhost || !c->ev_coef || c->m != c->p.restart || c->kR.size() < (size_t)(c->m + 1) * c->m)
    return fail(c, HYB_ESTATE, "the Krylov basis for this restart length is not allocated (condense first)");
  if (!c->scratch) return fail(c, HYB_EHIP, "no static scratch on this device: " + c->scratch_err);
  int dev = -1;
  CHECK_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev != c->device) return fail(c, HYB_ESTATE, "hyb_solve_noalloc called with another device current");
  const size_t npart = (size_t)c->nblk_red * 2 * (c->m + 2), nh = 4 * (size_t)(c->m + 2);
  if (npart + nh > kScratchDoubles)
    return fail(c, HYB_EINVAL, "restart length " + std::to_string(c->m) + " needs " +
                                   std::to_string((npart + nh) * sizeof(double)) +
                                   " bytes of reduction scratch; the static scratch holds " +
                                   std::to_string(kScratchDoubles * sizeof(double)));
  // the reductions of this call write into the static scratch: the workgroup partials first, the
  // summed results after them; every slot a reduction reads is written by the same reduction, so
  // nothing needs clearing
  double *own_partial = c->partial, *own_hdev = c->hdev;
  c->partial = c->scratch;
  c->hdev = c->scratch + npart;
  const int status = solve_impl(c, b, lam, rtol, maxit, info);
  c->partial = own_partial;
  c->hdev = own_hdev;
  return status;
}

// ----- Configuration 1: the unhybridised system with the approximate-Schur preconditioner -----

static int mixed_ready(hyb_ctx *c) {
  if (!c->condensed) return fail(c, HYB_ESTATE, "mixed-system call before condense");
  if (c->order != 0) return fail(c, HYB_EINVAL, "the mixed system is built for order 0 only");
  return HYB_OK;
}

int hyb_mixed_rhs(hyb_ctx *c, const double *r_ub, const double *r_pi, double *b) {
  if (!c) return HYB_EINVAL;
  int rc = mixed_ready(c);
  if (rc) return rc;
  if (!r_ub || !r_pi || !b) return fail(c, HYB_EINVAL, "null argument");
  CHECK_HIP(launch_mixed_rhs(c, r_ub, r_pi, b), "mixed rhs");
  return HYB_OK;
}

int hyb_mixed_apply(hyb_ctx *c, const double *x, double *y) {
  if (!c) return HYB_EINVAL;
  int rc = mixed_ready(c);
  if (rc) return rc;
  if (!x || !y || x == y) return fail(c, HYB_EINVAL, "bad mixed apply arguments");
  CHECK_HIP(launch_mixed_rows(c, x, nullptr, y), "mixed apply");
  return HYB_OK;
}

int hyb_mixed_precondition(hyb_ctx *c, const double *r, double *z) {
  if (!c) return HYB_EINVAL;
  int rc = mixed_ready(c);
  if (rc) return rc;
  if (!r || !z || r == z) return fail(c, HYB_EINVAL, "bad mixed precondition arguments");
  CHECK_HIP(schur_precondition(c, r, z), "approximate Schur");
  return HYB_OK;
}

int hyb_mixed_solve(hyb_ctx *c, const double *b, double *x, double rtol, int32_t maxit, hyb_info *info) {
  if (!c) return HYB_EINVAL;
  int rc = mixed_ready(c);
  if (rc) return rc;
  if (!b || !x || b == x || !(rtol >= 0) || maxit < 0) return fail(c, HYB_EINVAL, "bad mixed solve arguments");
  if ((rc = alloc_krylov(c))) return rc;
  const int m = c->m;
  const size_t n = (size_t)c->ntrace + c->ncell;
  if (!c->Vm || c->mm != m) {
    dfree(c->Vm), dfree(c->Zm);
    c->mm = 0;
    if ((rc = dalloc(c, &c->Vm, (size_t)(m + 1) * n)) || (rc = dalloc(c, &c->Zm, (size_t)m * n))) return rc;
    c->mm = m;
  }
  double *V = c->Vm, *Z = c->Zm;
  auto resid = [&](double *V0) -> int {
    CHECK_HIP(launch_mixed_rows(c, x, b, V0), "residual");
    return HYB_OK;
  };
  auto apply_op = [&](int j) -> int {
    double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n, *w = V + (size_t)(j + 1) * n;
    CHECK_HIP(schur_precondition(c, vj, zj), "approximate Schur");
    CHECK_HIP(launch_mixed_rows(c, zj, nullptr, w), "matvec");
    return HYB_OK;
  };
  return fgmres(c, n, n, V, Z, false, b, x, rtol, maxit, info, resid, apply_op);
}

int hyb_recover(hyb_ctx *c, const double *r_ub, const double *r_pi, const double *lambda, double *u_b, double *pi) {
  if (!c) return HYB_EINVAL;
  if (!c->condensed) return fail(c, HYB_ESTATE, "recover before condense");
  if (!r_ub || !r_pi || !lambda || !u_b || !pi) return fail(c, HYB_EINVAL, "null argument");
  if (c->order == 1) {
    CHECK_HIP(p1_cell_solve(c, r_ub, r_pi, lambda, 1, u_b, pi), "p1 recover");
    return HYB_OK;
  }
  CHECK_HIP(launch_recover(c, r_ub, r_pi, lambda, u_b, pi), "recover");
  return HYB_OK;
}

int hyb_eliminate(hyb_ctx *c, const double *r_ub, const double *r_rho, const double *r_theta, const double *r_pi,
                  double *r_ub_bar, double *r_pi_bar) {
  if (!c) return HYB_EINVAL;
  if (c->order != 0) return fail(c, HYB_EINVAL, "the theta' / rho' elimination is built for order 0");
  if (!c->assembled) return fail(c, HYB_ESTATE, "eliminate before assemble_local");
  if (!r_ub || !r_rho || !r_theta || !r_pi || !r_ub_bar || !r_pi_bar) return fail(c, HYB_EINVAL, "null argument");
  CHECK_HIP(launch_eliminate(c, r_ub, r_rho, r_theta, r_pi, r_ub_bar, r_pi_bar), "eliminate");
  return HYB_OK;
}

int hyb_back_substitute(hyb_ctx *c, const double *r_rho, const double *r_theta, const double *u_b, double *rho,
                        double *theta) {
  if (!c) return HYB_EINVAL;
  if (c->order != 0) return fail(c, HYB_EINVAL, "the theta' / rho' back-substitution is built for order 0");
  if (!c->assembled) return fail(c, HYB_ESTATE, "back_substitute before assemble_local");
  if (!r_rho || !r_theta || !u_b || !rho || !theta) return fail(c, HYB_EINVAL, "null argument");
  if (rho == u_b || theta == u_b || rho == r_rho || theta == r_theta)
    return fail(c, HYB_EINVAL, "outputs must not alias inputs");
  CHECK_HIP(launch_back_substitute(c, r_rho, r_theta, u_b, rho, theta), "back_substitute");
  return HYB_OK;
}

int hyb_sizes(const hyb_ctx *c, int64_t *ntrace, int64_t *ncell, int64_t *bytes) {
  if (!c) return HYB_EINVAL;
  if (ntrace) *ntrace = c->ntrace;
  if (ncell) *ncell = c->ncell;
  if (bytes) *bytes = (int64_t)c->bytes;
  return HYB_OK;
}

int hyb_profile(hyb_ctx *c, int32_t enable) {
  if (!c) return HYB_EINVAL;
  CHECK_HIP(hipStreamSynchronize(c->stream), "profile sync");
  for (auto &f : c->fam) f.used = 0;
  c->prof = enable != 0;
  c->prof_mask = ~0ull;
  return HYB_OK;
}

int hyb_profile_family(hyb_ctx *c, const char *family) {
  if (!c || !family) return HYB_EINVAL;
  for (size_t i = 0; i < c->fam.size(); ++i) {
    if (c->fam[i].name != family) continue;
    CHECK_HIP(hipStreamSynchronize(c->stream), "profile sync");
    for (auto &f : c->fam) f.used = 0;
    c->prof = true;
    c->prof_mask = 1ull << i;
    return HYB_OK;
  }
  return fail(c, HYB_EINVAL, std::string("unknown kernel family ") + family);
}

int hyb_profile_read(hyb_ctx *c, const char *family, int64_t *launches, double *total_ms) {
  if (!c || !family) return HYB_EINVAL;
  CHECK_HIP(hipStreamSynchronize(c->stream), "profile sync");
  for (auto &f : c->fam) {
    if (f.name != family) continue;
    double tot = 0.0;
    for (size_t i = 0; i + 1 < f.used; i += 2) {
      float ms = 0.f;
      CHECK_HIP(hipEventElapsedTime(&ms, f.ev[i], f.ev[i + 1]), "event elapsed");
      tot += ms;
    }
    if (launches) *launches = (int64_t)(f.used / 2);
    if (total_ms) *total_ms = tot;
    return HYB_OK;
  }
  return fail(c, HYB_EINVAL, std::string("unknown kernel family ") + family);
}

int hyb_restrict(hyb_ctx *c, const double *r, double *cells, int32_t mode) {
  if (!c) return HYB_EINVAL;
  if (c->order == 1) return fail(c, HYB_ESTATE, "hyb_restrict is not available at order 1");
  if (!c->condensed) return fail(c, HYB_ESTATE, "restrict before condense");
  if (!r || !cells || mode < 0 || mode > 3) return fail(c, HYB_EINVAL, "bad restrict arguments");
  CHECK_HIP(launch_restrict_cells(c, r, cells, mode), "restrict");
  return HYB_OK;
}

int hyb_nn_param_count(void) { return nn_param_count(); }

int hyb_nn_set_weights(hyb_ctx *c, const float *w, int64_t n) {
  if (!c) return HYB_EINVAL;
  if (c->order == 1) return fail(c, HYB_ESTATE, "hyb_nn_set_weights is not available at order 1");
  if (!w || n != nn_param_count()) return fail(c, HYB_EINVAL, "weights: wrong size");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(w[i])) return fail(c, HYB_EINVAL, "weights: not finite");
  CHECK_HIP(nn_setup(c), "nn setup");
  CHECK_HIP(nn_set_weights(c, w), "nn set weights");
  c->nn.loaded = true;
  return HYB_OK;
}

int hyb_nn_get_weights(hyb_ctx *c, float *w, int64_t n) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!w || n != nn_param_count()) return fail(c, HYB_EINVAL, "weights: wrong size");
  CHECK_HIP(nn_get_weights(c, w), "nn get weights");
  return HYB_OK;
}

int hyb_nn_get_state(hyb_ctx *c, float *m, float *v, int64_t n, int64_t *step) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!m || !v || !step || n != nn_param_count()) return fail(c, HYB_EINVAL, "state: wrong size");
  CHECK_HIP(nn_get_state(c, m, v, step), "nn get state");
  return HYB_OK;
}

int hyb_nn_set_state(hyb_ctx *c, const float *m, const float *v, int64_t n, int64_t step) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!m || !v || n != nn_param_count() || step < 0) return fail(c, HYB_EINVAL, "state: wrong size or step");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(m[i]) || !std::isfinite(v[i]) || v[i] < 0.f) return fail(c, HYB_EINVAL, "state: bad moment");
  CHECK_HIP(nn_set_state(c, m, v, step), "nn set state");
  return HYB_OK;
}

int hyb_nn_forward(hyb_ctx *c, const float *x, float *y, int32_t nsamp) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!x || !y || nsamp < 1) return fail(c, HYB_EINVAL, "bad forward arguments");
  CHECK_HIP(nn_forward(c, x, y, nsamp), "nn forward");
  return HYB_OK;
}

int hyb_nn_loss_grad(hyb_ctx *c, const float *x, const float *t, int32_t nsamp, float *loss, float *grad) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!x || !t || nsamp < 1) return fail(c, HYB_EINVAL, "bad loss arguments");
  CHECK_HIP(nn_loss_grad(c, x, t, nsamp, loss), "nn loss/grad");
  if (grad) {
    CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
    CHECK_HIP(hipMemcpy(grad, c->nn.g, nn_param_count() * sizeof(float), hipMemcpyDeviceToHost), "d2h grad");
  }
  return HYB_OK;
}

int hyb_nn_train_step(hyb_ctx *c, const float *x, const float *t, int32_t nsamp, float lr, float *loss) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!x || !t || nsamp < 1 || !(lr > 0)) return fail(c, HYB_EINVAL, "bad train arguments");
  CHECK_HIP(nn_loss_grad(c, x, t, nsamp, loss), "nn loss/grad");
  CHECK_HIP(nn_adam(c, lr), "nn adam");
  return HYB_OK;
}

int hyb_nn_energy_grad(hyb_ctx *c, const float *x, const double *rhat, int32_t nsamp, double *loss, float *grad) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!c->condensed) return fail(c, HYB_ESTATE, "energy loss before condense");
  if (!x || !rhat || nsamp < 1) return fail(c, HYB_EINVAL, "bad energy arguments");
  CHECK_HIP(nn_energy_grad(c, x, rhat, nsamp, loss), "nn energy grad");
  if (grad) {
    CHECK_HIP(hipStreamSynchronize(c->stream), "sync");
    CHECK_HIP(hipMemcpy(grad, c->nn.g, nn_param_count() * sizeof(float), hipMemcpyDeviceToHost), "d2h grad");
  }
  return HYB_OK;
}

int hyb_nn_energy_train_step(hyb_ctx *c, const float *x, const double *rhat, int32_t nsamp, float lr, double *loss) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!c->condensed) return fail(c, HYB_ESTATE, "energy loss before condense");
  if (!x || !rhat || nsamp < 1 || !(lr > 0)) return fail(c, HYB_EINVAL, "bad train arguments");
  CHECK_HIP(nn_energy_grad(c, x, rhat, nsamp, loss), "nn energy grad");
  CHECK_HIP(nn_adam(c, lr), "nn adam");
  return HYB_OK;
}

int hyb_nn_cycle_pair(hyb_ctx *c, double *r, float *x, double *rhat, double *scale) {
  if (!c) return HYB_EINVAL;
  if (c->order == 1) return fail(c, HYB_ESTATE, "hyb_nn_cycle_pair is not available at order 1");
  if (!c->condensed) return fail(c, HYB_ESTATE, "training pairs before condense");
  if (!r || !x || !rhat) return fail(c, HYB_EINVAL, "bad pair arguments");
  int rc = alloc_krylov(c);  // reduction scratch, and the FP32 slots of the mixed form
  if (rc) return rc;
  CHECK_HIP(nn_stage_buffers(c), "pair buffers");
  const size_t n = (size_t)c->ntrace;
  double *z = c->nn.d64;
  // the plain two-level cycle (never the learned stage)
  if (c->p.precision == HYB_PREC_FP64) {
    CHECK_HIP(precondition<double>(c, r, z), "precondition");
  } else {
    float *rf = (float *)c->tIn, *zf = (float *)c->Z;
    CHECK_HIP(launch_convert(c, r, rf, n), "convert");
    CHECK_HIP(precondition<float>(c, rf, zf), "precondition");
    CHECK_HIP(launch_copy_widen(c, zf, z, n), "widen");
  }
  CHECK_HIP((launch_trace_apply<double, double, double>(c, c->S, z, r, c->t64, 1)), "residual");
  CHECK_HIP(hipMemcpyAsync(r, c->t64, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "copy residual");
  CHECK_HIP(launch_restrict_cells(c, c->t64, c->cell64, 0), "restrict");
  double s = 0.0;
  CHECK_HIP(nn_pair_finish(c, x, rhat, &s), "pair");
  if (scale) *scale = s;
  if (!std::isfinite(s) || s == 0.0) return HYB_BREAKDOWN;
  return HYB_OK;
}

int hyb_nn_energy_train_step_pairs(hyb_ctx *c, const float *X, const double *R, int64_t npairs, const int32_t *idx,
                                   int32_t nsamp, float lr, double *loss) {
  if (!c) return HYB_EINVAL;
  if (!c->nn.loaded) return fail(c, HYB_ESTATE, "no weights");
  if (!c->condensed) return fail(c, HYB_ESTATE, "energy loss before condense");
  if (!X || !R || !idx || nsamp < 1 || npairs < 1 || !(lr > 0)) return fail(c, HYB_EINVAL, "bad train arguments");
  for (int32_t i = 0; i < nsamp; ++i)
    if (idx[i] < 0 || idx[i] >= npairs) return fail(c, HYB_EINVAL, "pair index out of range");
  CHECK_HIP(nn_gather_batch(c, X, R, idx, nsamp), "gather batch");
  CHECK_HIP(nn_energy_grad(c, c->nn.xb, c->nn.rb, nsamp, loss), "nn energy grad");
  CHECK_HIP(nn_adam(c, lr), "nn adam");
  return HYB_OK;
}

const char *hyb_last_error(const hyb_ctx *c) { return c ? c->err.c_str() : "null context"; }

void hyb_destroy(hyb_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

}  // extern "C"
