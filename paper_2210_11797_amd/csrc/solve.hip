// Trace operator, LineSmooth (Alg. 1), intergrid transfers and the pressure multigrid V-cycle,
// assembled into the non-nested two-level cycle (Alg. 2).
//
// Column kernels put one column per lane (64 consecutive columns per wavefront, so every access
// to a [k][col] array is coalesced) and walk up the column: the tridiagonal Thomas solve keeps its
// forward-elimination coefficients in LDS and runs the back substitution from there.
#include "hyb_internal.h"

namespace hyb {

namespace {

inline unsigned nblk(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

template <typename T>
struct Acc {
  using type = T;
};

// Row of S for the horizontal facet (k, col): neighbours below/above and the vertical facets of
// the two cells (layers k-1 and k), with the stencil order of the setup gather.
template <typename A, typename Tm, typename Tx>
__device__ __forceinline__ A row_z(const Tm *__restrict__ S, size_t ntr, const Tx *__restrict__ x, size_t F,
                                   int k, int nlev, int ncol, int nedge, size_t nz, const int ce[4]) {
  A acc = (A)S[F] * (A)x[F];
  if (k > 0) {
    size_t hb = nz + (size_t)(k - 1) * nedge;
    acc += (A)S[ntr + F] * (A)x[F - ncol];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc += (A)S[(3 + f) * ntr + F] * (A)x[hb + ce[f]];
  }
  if (k < nlev) {
    size_t hb = nz + (size_t)k * nedge;
    acc += (A)S[2 * ntr + F] * (A)x[F + ncol];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc += (A)S[(7 + f) * ntr + F] * (A)x[hb + ce[f]];
  }
  return acc;
}

// Edge stencil table: est[0..7][e] = c0, c1, three other edges of c0, three other edges of c1.
template <typename A, typename Tm, typename Tx>
__device__ __forceinline__ A row_h(const Tm *__restrict__ S, size_t ntr, const Tx *__restrict__ x, size_t F,
                                   int k, int ncol, int nedge, size_t nz, const int t[8]) {
  size_t hb = nz + (size_t)k * nedge;
  size_t zb = (size_t)k * ncol;
  A acc = (A)S[F] * (A)x[F];
  acc += (A)S[ntr + F] * (A)x[zb + t[0]];
  acc += (A)S[2 * ntr + F] * (A)x[zb + ncol + t[0]];
  acc += (A)S[3 * ntr + F] * (A)x[hb + t[2]];
  acc += (A)S[4 * ntr + F] * (A)x[hb + t[3]];
  acc += (A)S[5 * ntr + F] * (A)x[hb + t[4]];
  acc += (A)S[6 * ntr + F] * (A)x[zb + t[1]];
  acc += (A)S[7 * ntr + F] * (A)x[zb + ncol + t[1]];
  acc += (A)S[8 * ntr + F] * (A)x[hb + t[5]];
  acc += (A)S[9 * ntr + F] * (A)x[hb + t[6]];
  acc += (A)S[10 * ntr + F] * (A)x[hb + t[7]];
  return acc;
}

// y = S x (MODE 0) or y = b - S x (MODE 1); one thread per trace row.
template <typename Tm, typename Tx, typename Ty, int MODE>
__global__ void k_trace_apply(const Tm *__restrict__ S, const Tx *__restrict__ x, const Ty *__restrict__ b,
                              Ty *__restrict__ y, int nlev, int ncol, int nedge, size_t nz, size_t ntr,
                              const int32_t *__restrict__ col_edge, const int32_t *__restrict__ est) {
  using A = typename Acc<Ty>::type;
  size_t F = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (F >= ntr) return;
  A v;
  if (F < nz) {
    int k = (int)(F / ncol), col = (int)(F - (size_t)k * ncol);
    int ce[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) ce[f] = col_edge[(size_t)f * ncol + col];
    v = row_z<A>(S, ntr, x, F, k, nlev, ncol, nedge, nz, ce);
  } else {
    size_t h = F - nz;
    int k = (int)(h / nedge), e = (int)(h - (size_t)k * nedge);
    int t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = est[(size_t)i * nedge + e];
    v = row_h<A>(S, ntr, x, F, k, ncol, nedge, nz, t);
  }
  if (MODE == 1) v = (A)b[F] - v;
  y[F] = (Ty)v;
}

// One sweep of LineSmooth (Alg. 1, with the update lambda <- lambda + omega delta):
// residual R = B - S lambda_in, tridiagonal solve S^zz_j delta = R^z_j per column (Thomas),
// point Jacobi delta = R^h / diag(S^hh) on the vertical facets owned by the column.
// ZERO: lambda_in = 0 (R = B, the first sweep of Alg. 2).  Writes lambda_out (Jacobi: no in-place).
template <typename T, bool ZERO>
__global__ void __launch_bounds__(kColBlock) k_line_smooth(const T *__restrict__ S, const T *__restrict__ B,
                                                           const T *__restrict__ lin, T *__restrict__ lout,
                                                           int nlev, int ncol, int nedge, size_t nz, size_t ntr,
                                                           const int32_t *__restrict__ col_edge,
                                                           const int32_t *__restrict__ own,
                                                           const int32_t *__restrict__ est, T omega) {
  extern __shared__ unsigned char smem_raw[];
  T *cpv = reinterpret_cast<T *>(smem_raw);
  T *dpv = cpv + (size_t)(nlev + 1) * blockDim.x;
  int tid = threadIdx.x;
  int col = blockIdx.x * blockDim.x + tid;
  if (col >= ncol) return;
  int ce[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) ce[f] = col_edge[(size_t)f * ncol + col];
  int ne = 0, oe[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int e = own[(size_t)j * ncol + col];
    oe[j] = e;
    ne += (e >= 0);
  }
  T cprev = 0, dprev = 0;
  for (int k = 0; k <= nlev; ++k) {
    size_t F = (size_t)k * ncol + col;
    T r = B[F];
    if (!ZERO) r -= row_z<T>(S, ntr, lin, F, k, nlev, ncol, nedge, nz, ce);
    T a = S[ntr + F], bb = S[F], c = S[2 * ntr + F];
    T inv = (T)1 / (bb - a * cprev);
    cprev = c * inv;
    dprev = (r - a * dprev) * inv;
    cpv[(size_t)k * blockDim.x + tid] = cprev;
    dpv[(size_t)k * blockDim.x + tid] = dprev;
    if (k < nlev) {
      for (int j = 0; j < ne; ++j) {
        int e = oe[j];
        size_t hF = nz + (size_t)k * nedge + e;
        T rh = B[hF];
        T base = 0;
        if (!ZERO) {
          int t[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) t[i] = est[(size_t)i * nedge + e];
          rh -= row_h<T>(S, ntr, lin, hF, k, ncol, nedge, nz, t);
          base = lin[hF];
        }
        lout[hF] = base + omega * rh / S[hF];
      }
    }
  }
  T xk = 0;
  for (int k = nlev; k >= 0; --k) {
    size_t F = (size_t)k * ncol + col;
    xk = dpv[(size_t)k * blockDim.x + tid] - cpv[(size_t)k * blockDim.x + tid] * xk;
    T base = ZERO ? (T)0 : lin[F];
    lout[F] = base + omega * xk;
  }
}

// Restriction to the pressure space and scaling: Bbar_K = Gamma_K sum_F w_F R_F over the six
// facets of K, w = 1/2 (1 on ground and lid facets, where prolongation is one sided).
template <typename T>
__global__ void k_restrict(const T *__restrict__ R, const T *__restrict__ gamma, T *__restrict__ out, int nlev,
                           int ncol, int nedge, size_t nz, const int32_t *__restrict__ col_edge) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nlev * ncol) return;
  int k = c / ncol, col = c - k * ncol;
  T s = 0;
  size_t hb = nz + (size_t)k * nedge;
#pragma unroll
  for (int f = 0; f < 4; ++f) s += R[hb + col_edge[(size_t)f * ncol + col]];
  s *= (T)0.5;
  s += (k == 0 ? (T)1 : (T)0.5) * R[(size_t)k * ncol + col];
  s += (k == nlev - 1 ? (T)1 : (T)0.5) * R[(size_t)(k + 1) * ncol + col];
  out[c] = gamma[c] * s;
}

// lambda_F += (P dPi)_F: average of the two cells of the facet (one sided on ground / lid).
template <typename T>
__global__ void k_prolong(const T *__restrict__ dpi, T *__restrict__ lam, int nlev, int ncol, int nedge, size_t nz,
                          size_t ntr, const int32_t *__restrict__ edge_col) {
  size_t F = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (F >= ntr) return;
  T v;
  if (F < nz) {
    int k = (int)(F / ncol), col = (int)(F - (size_t)k * ncol);
    if (k == 0)
      v = dpi[col];
    else if (k == nlev)
      v = dpi[(size_t)(nlev - 1) * ncol + col];
    else
      v = (T)0.5 * (dpi[(size_t)(k - 1) * ncol + col] + dpi[(size_t)k * ncol + col]);
  } else {
    size_t h = F - nz;
    int k = (int)(h / nedge), e = (int)(h - (size_t)k * nedge);
    v = (T)0.5 * (dpi[(size_t)k * ncol + edge_col[e]] + dpi[(size_t)k * ncol + edge_col[nedge + e]]);
  }
  lam[F] += v;
}

// Block-Jacobi sweep of the pressure multigrid (Sec. 2.3):
//   x_out = x_in + omega H_z^-1 (b - H x_in), H_z = the column (tridiagonal) part of H.
// ZERO: x_in = 0.  ADDC: x_in is the fine iterate plus the injected coarse correction
// (prolongation fused into the first post-smoothing sweep).
template <typename T, bool ZERO, bool ADDC>
__global__ void __launch_bounds__(kColBlock) k_mg_smooth(const T *__restrict__ H, const T *__restrict__ b,
                                                         const T *__restrict__ xin, const T *__restrict__ xc,
                                                         T *__restrict__ xout, int nlev, int ncol, int ncolc,
                                                         const int32_t *__restrict__ nbr,
                                                         const int32_t *__restrict__ parent, T omega) {
  extern __shared__ unsigned char smem_raw[];
  T *cpv = reinterpret_cast<T *>(smem_raw);
  T *dpv = cpv + (size_t)nlev * blockDim.x;
  int tid = threadIdx.x;
  int col = blockIdx.x * blockDim.x + tid;
  if (col >= ncol) return;
  size_t n = (size_t)nlev * ncol;
  int nb[4], pc = 0, pn[4] = {0, 0, 0, 0};
#pragma unroll
  for (int f = 0; f < 4; ++f) nb[f] = nbr[(size_t)f * ncol + col];
  if (ADDC) {
    pc = parent[col];
#pragma unroll
    for (int f = 0; f < 4; ++f) pn[f] = parent[nb[f]];
  }
  auto X = [&](int k, int cc, int pcc) -> T {
    T v = xin[(size_t)k * ncol + cc];
    if (ADDC) v += xc[(size_t)k * ncolc + pcc];
    return v;
  };
  T cprev = 0, dprev = 0;
  for (int k = 0; k < nlev; ++k) {
    size_t c = (size_t)k * ncol + col;
    T r = b[c];
    T a = H[5 * n + c], d = H[c], u = H[6 * n + c];
    if (!ZERO) {
      T hx = d * X(k, col, pc);
#pragma unroll
      for (int f = 0; f < 4; ++f) hx += H[(1 + f) * n + c] * X(k, nb[f], pn[f]);
      if (k > 0) hx += a * X(k - 1, col, pc);
      if (k < nlev - 1) hx += u * X(k + 1, col, pc);
      r -= hx;
    }
    T inv = (T)1 / (d - a * cprev);
    cprev = u * inv;
    dprev = (r - a * dprev) * inv;
    cpv[(size_t)k * blockDim.x + tid] = cprev;
    dpv[(size_t)k * blockDim.x + tid] = dprev;
  }
  T xk = 0;
  for (int k = nlev - 1; k >= 0; --k) {
    xk = dpv[(size_t)k * blockDim.x + tid] - cpv[(size_t)k * blockDim.x + tid] * xk;
    T base = ZERO ? (T)0 : X(k, col, pc);
    xout[(size_t)k * ncol + col] = base + omega * xk;
  }
}

// Coarse right-hand side: b_c = R (b - H x), R = sum over the four children.
template <typename T>
__global__ void k_mg_residual_restrict(const T *__restrict__ H, const T *__restrict__ b, const T *__restrict__ x,
                                       T *__restrict__ bc, int nlev, int ncolf, int ncolc,
                                       const int32_t *__restrict__ children, const int32_t *__restrict__ nbrf) {
  int cc = blockIdx.x * blockDim.x + threadIdx.x;
  if (cc >= nlev * ncolc) return;
  int k = cc / ncolc, P = cc - k * ncolc;
  size_t n = (size_t)nlev * ncolf;
  T s = 0;
  for (int q = 0; q < 4; ++q) {
    int col = children[(size_t)q * ncolc + P];
    size_t c = (size_t)k * ncolf + col;
    T hx = H[c] * x[c];
#pragma unroll
    for (int f = 0; f < 4; ++f) hx += H[(1 + f) * n + c] * x[(size_t)k * ncolf + nbrf[(size_t)f * ncolf + col]];
    if (k > 0) hx += H[5 * n + c] * x[c - ncolf];
    if (k < nlev - 1) hx += H[6 * n + c] * x[c + ncolf];
    s += b[c] - hx;
  }
  bc[cc] = s;
}

template <typename T>
__global__ void k_mg_prolong_add(T *__restrict__ x, const T *__restrict__ xc, int nlev, int ncolf, int ncolc,
                                 const int32_t *__restrict__ parent) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nlev * ncolf) return;
  int k = c / ncolf, col = c - k * ncolf;
  x[c] += xc[(size_t)k * ncolc + parent[col]];
}

template <typename T>
__global__ void k_zero(T *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)0;
}

template <typename T>
__global__ void k_copy(const T *__restrict__ s, T *__restrict__ d, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

template <typename T>
const T *pick(const double *d, const float *f);
template <>
const double *pick<double>(const double *d, const float *) {
  return d;
}
template <>
const float *pick<float>(const double *, const float *f) {
  return f;
}

template <typename T>
hipError_t line_smooth(hyb_ctx *c, const T *S, const T *B, const T *lin, T *lout, bool zero) {
  const LevelDev &L0 = c->lv[0];
  size_t shm = 2 * sizeof(T) * (size_t)(c->nlev + 1) * kColBlock;
  int fam = zero ? F_LINE_SMOOTH0 : F_LINE_SMOOTH;
  int slot = prof_begin(c, fam);
  T om = (T)c->p.omega;
  if (zero)
    hipLaunchKernelGGL((k_line_smooth<T, true>), dim3(nblk(c->ncol, kColBlock)), dim3(kColBlock), shm, c->stream,
                       S, B, lin, lout, c->nlev, c->ncol, c->nedge, (size_t)c->nz, (size_t)c->ntrace, L0.col_edge,
                       L0.own, L0.est, om);
  else
    hipLaunchKernelGGL((k_line_smooth<T, false>), dim3(nblk(c->ncol, kColBlock)), dim3(kColBlock), shm,
                       c->stream, S, B, lin, lout, c->nlev, c->ncol, c->nedge, (size_t)c->nz, (size_t)c->ntrace,
                       L0.col_edge, L0.own, L0.est, om);
  prof_end(c, fam, slot);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_smooth(hyb_ctx *c, int l, const T *b, const T *xin, const T *xc, T *xout, int mode) {
  const LevelDev &Lv = c->lv[l];
  const T *H = pick<T>(Lv.H, Lv.Hf);
  size_t shm = 2 * sizeof(T) * (size_t)c->nlev * kColBlock;
  int ncolc = (l + 1 < c->nlevels) ? c->lv[l + 1].ncol : 1;
  T om = (T)c->p.omega_p;
  dim3 g(nblk(Lv.ncol, kColBlock)), bl(kColBlock);
  int slot = prof_begin(c, F_MG_SMOOTH);
  if (mode == 0)
    hipLaunchKernelGGL((k_mg_smooth<T, true, false>), g, bl, shm, c->stream, H, b, xin, xc, xout, c->nlev, Lv.ncol,
                       ncolc, Lv.nbr, Lv.parent, om);
  else if (mode == 1)
    hipLaunchKernelGGL((k_mg_smooth<T, false, false>), g, bl, shm, c->stream, H, b, xin, xc, xout, c->nlev,
                       Lv.ncol, ncolc, Lv.nbr, Lv.parent, om);
  else
    hipLaunchKernelGGL((k_mg_smooth<T, false, true>), g, bl, shm, c->stream, H, b, xin, xc, xout, c->nlev,
                       Lv.ncol, ncolc, Lv.nbr, Lv.parent, om);
  prof_end(c, F_MG_SMOOTH, slot);
  return hipGetLastError();
}

#define HYB_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

// One V-cycle on level l from a zero initial guess: right-hand side lv[l].b, result lv[l].x.
template <typename T>
hipError_t vcycle(hyb_ctx *c, int l) {
  LevelDev &Lv = c->lv[l];
  size_t n = (size_t)c->nlev * Lv.ncol;
  T *b = (T *)Lv.b;
  const hyb_params &p = c->p;
  bool coarsest = (l == c->nlevels - 1);
  int pre = coarsest ? p.mg_coarse_sweeps : p.mg_pre;
  if (pre <= 0) {
    hipLaunchKernelGGL((k_zero<T>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, (T *)Lv.x, n);
    HYB_TRY(hipGetLastError());
  } else {
    HYB_TRY(mg_smooth<T>(c, l, b, nullptr, nullptr, (T *)Lv.x, 0));
    for (int s = 1; s < pre; ++s) {
      HYB_TRY(mg_smooth<T>(c, l, b, (T *)Lv.x, nullptr, (T *)Lv.y, 1));
      std::swap(Lv.x, Lv.y);
    }
  }
  if (coarsest) return hipSuccess;
  LevelDev &Lc = c->lv[l + 1];
  const T *H = pick<T>(Lv.H, Lv.Hf);
  int slot = prof_begin(c, F_RESTRICT);
  hipLaunchKernelGGL((k_mg_residual_restrict<T>), dim3(nblk((size_t)c->nlev * Lc.ncol)), dim3(kBlock), 0, c->stream,
                     H, b, (const T *)Lv.x, (T *)Lc.b, c->nlev, Lv.ncol, Lc.ncol, Lc.children, Lv.nbr);
  prof_end(c, F_RESTRICT, slot);
  HYB_TRY(hipGetLastError());
  HYB_TRY(vcycle<T>(c, l + 1));
  if (p.mg_post <= 0) {
    hipLaunchKernelGGL((k_mg_prolong_add<T>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, (T *)Lv.x,
                       (const T *)Lc.x, c->nlev, Lv.ncol, Lc.ncol, Lv.parent);
    return hipGetLastError();
  }
  HYB_TRY(mg_smooth<T>(c, l, b, (T *)Lv.x, (const T *)Lc.x, (T *)Lv.y, 2));
  std::swap(Lv.x, Lv.y);
  for (int s = 1; s < p.mg_post; ++s) {
    HYB_TRY(mg_smooth<T>(c, l, b, (T *)Lv.x, nullptr, (T *)Lv.y, 1));
    std::swap(Lv.x, Lv.y);
  }
  return hipSuccess;
}

}  // namespace

template <typename Tm, typename Tx, typename Ty>
hipError_t launch_trace_apply(hyb_ctx *c, const Tm *S, const Tx *x, const Ty *b, Ty *y, int mode) {
  const LevelDev &L0 = c->lv[0];
  int slot = prof_begin(c, F_TRACE_APPLY);
  if (mode == 0)
    hipLaunchKernelGGL((k_trace_apply<Tm, Tx, Ty, 0>), dim3(nblk(c->ntrace)), dim3(kBlock), 0, c->stream, S, x, b,
                       y, c->nlev, c->ncol, c->nedge, (size_t)c->nz, (size_t)c->ntrace, L0.col_edge, L0.est);
  else
    hipLaunchKernelGGL((k_trace_apply<Tm, Tx, Ty, 1>), dim3(nblk(c->ntrace)), dim3(kBlock), 0, c->stream, S, x, b,
                       y, c->nlev, c->ncol, c->nedge, (size_t)c->nz, (size_t)c->ntrace, L0.col_edge, L0.est);
  prof_end(c, F_TRACE_APPLY, slot);
  return hipGetLastError();
}

template hipError_t launch_trace_apply<double, double, double>(hyb_ctx *, const double *, const double *,
                                                               const double *, double *, int);
template hipError_t launch_trace_apply<double, float, double>(hyb_ctx *, const double *, const float *,
                                                              const double *, double *, int);
template hipError_t launch_trace_apply<float, float, float>(hyb_ctx *, const float *, const float *, const float *,
                                                            float *, int);

// Alg. 2 from a zero initial guess: z = M(r).
template <typename T>
hipError_t precondition(hyb_ctx *c, const T *r, T *z) {
  const hyb_params &p = c->p;
  const T *S = pick<T>(c->S, c->Sf);
  const T *gam = pick<T>(c->gamma, c->gammaf);
  T *tA = (T *)c->tA, *tB = (T *)c->tB, *tR = (T *)c->tR;
  size_t ntr = (size_t)c->ntrace;
  const LevelDev &L0 = c->lv[0];
  // presmoothing
  if (p.n_pre <= 0) {
    hipLaunchKernelGGL((k_zero<T>), dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, tA, ntr);
    HYB_TRY(hipGetLastError());
  } else {
    HYB_TRY(line_smooth<T>(c, S, r, nullptr, tA, true));
    for (int s = 1; s < p.n_pre; ++s) {
      HYB_TRY(line_smooth<T>(c, S, r, tA, tB, false));
      std::swap(tA, tB);
    }
  }
  // residual, restriction and scaling
  HYB_TRY((launch_trace_apply<T, T, T>(c, S, tA, r, tR, 1)));
  int slot = prof_begin(c, F_RESTRICT);
  hipLaunchKernelGGL((k_restrict<T>), dim3(nblk(c->ncell)), dim3(kBlock), 0, c->stream, tR, gam, (T *)c->lv[0].b,
                     c->nlev, c->ncol, c->nedge, (size_t)c->nz, L0.col_edge);
  prof_end(c, F_RESTRICT, slot);
  HYB_TRY(hipGetLastError());
  // coarse solve: one pressure multigrid V-cycle
  HYB_TRY(vcycle<T>(c, 0));
  // prolongation and update
  slot = prof_begin(c, F_PROLONG);
  hipLaunchKernelGGL((k_prolong<T>), dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, (const T *)c->lv[0].x, tA,
                     c->nlev, c->ncol, c->nedge, (size_t)c->nz, ntr, L0.edge_col);
  prof_end(c, F_PROLONG, slot);
  HYB_TRY(hipGetLastError());
  // postsmoothing, the last sweep writes z
  if (p.n_post <= 0) {
    hipLaunchKernelGGL((k_copy<T>), dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, (const T *)tA, z, ntr);
    return hipGetLastError();
  }
  const T *src = tA;
  for (int s = 0; s < p.n_post; ++s) {
    T *dst = (s == p.n_post - 1) ? z : (src == tA ? tB : tA);
    HYB_TRY(line_smooth<T>(c, S, r, src, dst, false));
    src = dst;
  }
  return hipSuccess;
}

template hipError_t precondition<double>(hyb_ctx *, const double *, double *);
template hipError_t precondition<float>(hyb_ctx *, const float *, float *);

// The column kernels keep two (nlev+1)-long coefficient arrays per lane in LDS; allow the
// dynamic LDS size they need (above the 64 KiB default for tall columns in FP64).
hipError_t configure_kernels(int nlev) {
  int need = (int)(2 * sizeof(double) * (size_t)(nlev + 1) * kColBlock);
  if (need <= 65536) return hipSuccess;
  const void *fns[] = {
      (const void *)k_line_smooth<double, true>, (const void *)k_line_smooth<double, false>,
      (const void *)k_line_smooth<float, true>,  (const void *)k_line_smooth<float, false>,
      (const void *)k_mg_smooth<double, true, false>, (const void *)k_mg_smooth<double, false, false>,
      (const void *)k_mg_smooth<double, false, true>, (const void *)k_mg_smooth<float, true, false>,
      (const void *)k_mg_smooth<float, false, false>, (const void *)k_mg_smooth<float, false, true>};
  for (const void *f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, need);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hyb
