// The paper's Configuration 1 (Sec. 2.3): the unhybridised velocity / Exner-pressure system of
// Sec. 2.2 and its approximate-Schur preconditioner.
//
// Layout of a mixed vector: the velocity on every facet of the trace numbering, in the facet's
// global orientation (the +z normal for horizontal facets, the normal leaving the first column of
// the edge for vertical ones), ground and lid facets held at zero since they carry no velocity
// dof; then one Exner-pressure value per cell.  Every kernel is owner-computes: one thread per
// facet row or per cell row, gathering from the cell matrices A_K (outward-flux orientation,
// [49][ncell]) and the facet coefficients k ([6][ncell]) that the assembly wrote.
//
// The velocity-pressure block G includes the facet term of the form g: on facet F it adds half
// the jump J_F = k_{K0,F} - k_{K1,F} (K0 the cell the normal leaves) to the entries of both cells.

#include "hyb_internal.h"

#define HYB_TRY(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

namespace hyb {

namespace {

__device__ __forceinline__ size_t at(int i, int n, int c) { return (size_t)i * n + c; }

inline unsigned nblk(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

struct Topo {
  int nlev, ncol, nedge, ncell;
  size_t nz, nt;
  const int32_t *col_edge, *edge_col, *edge_lf;
};

// The two cells of interior facet F and their local faces (cell 0: the normal leaves it).
// Returns false on the ground and lid.
__device__ __forceinline__ bool facet_cells(const Topo &t, size_t F, int cells[2], int lfs[2]) {
  if (F < t.nz) {
    int k = (int)(F / t.ncol), col = (int)(F - (size_t)k * t.ncol);
    if (k == 0 || k == t.nlev) return false;
    cells[0] = (k - 1) * t.ncol + col, lfs[0] = 5;
    cells[1] = k * t.ncol + col, lfs[1] = 4;
    return true;
  }
  size_t h = F - t.nz;
  int k = (int)(h / t.nedge), e = (int)(h - (size_t)k * t.nedge);
  cells[0] = k * t.ncol + t.edge_col[e], lfs[0] = t.edge_lf[e];
  cells[1] = k * t.ncol + t.edge_col[t.nedge + e], lfs[1] = t.edge_lf[t.nedge + e];
  return true;
}

// Facet index and orientation sign of local face b of cell c; sign 0 for the ground and lid.
__device__ __forceinline__ size_t cell_facet(const Topo &t, int c, int b, double &s) {
  int k = c / t.ncol, col = c - k * t.ncol;
  if (b < 4) {
    int e = t.col_edge[(size_t)b * t.ncol + col];
    s = (t.edge_col[e] == col && t.edge_lf[e] == b) ? 1.0 : -1.0;
    return t.nz + (size_t)k * t.nedge + e;
  }
  if (b == 4) {
    s = k == 0 ? 0.0 : -1.0;
    return (size_t)k * t.ncol + col;
  }
  s = k == t.nlev - 1 ? 0.0 : 1.0;
  return (size_t)(k + 1) * t.ncol + col;
}

// Row a of A_K applied to the cell's velocity (global facet values) and pressure.
__device__ __forceinline__ double cell_row(const Topo &t, const double *__restrict__ A,
                                           const double *__restrict__ x, int c, int a) {
  double acc = A[at(a * 7 + 6, t.ncell, c)] * x[t.nt + c];
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    double s;
    size_t Fb = cell_facet(t, c, b, s);
    if (s != 0.0) acc += A[at(a * 7 + b, t.ncell, c)] * s * x[Fb];
  }
  return acc;
}

// MODE 0: y = A x; MODE 1: y = b - A x.
template <int MODE>
__global__ void k_mixed_rows(Topo t, const double *__restrict__ A, const double *__restrict__ kv,
                             const double *__restrict__ x, const double *__restrict__ b, double *__restrict__ y) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.nt + t.ncell) return;
  double v;
  if (i < t.nt) {
    int cells[2], lfs[2];
    if (!facet_cells(t, i, cells, lfs)) {
      y[i] = 0.0;
      return;
    }
    const double J = kv[at(lfs[0], t.ncell, cells[0])] - kv[at(lfs[1], t.ncell, cells[1])];
    v = cell_row(t, A, x, cells[0], lfs[0]) - cell_row(t, A, x, cells[1], lfs[1]) +
        0.5 * J * (x[t.nt + cells[0]] + x[t.nt + cells[1]]);
  } else {
    v = cell_row(t, A, x, (int)(i - t.nt), 6);
  }
  y[i] = MODE == 1 ? b[i] - v : v;
}

// The mixed right-hand side from the broken one: R_u(F) = sum over the two cells of F of the
// orientation sign times r^b_{K,F} (Sec. 2.4), zero on the ground and lid; then R_Pi.
__global__ void k_mixed_rhs(Topo t, const double *__restrict__ rub, const double *__restrict__ rpi,
                            double *__restrict__ y) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.nt + t.ncell) return;
  if (i < t.nt) {
    int cells[2], lfs[2];
    y[i] = facet_cells(t, i, cells, lfs)
               ? rub[at(lfs[0], t.ncell, cells[0])] - rub[at(lfs[1], t.ncell, cells[1])]
               : 0.0;
  } else {
    y[i] = rpi[i - t.nt];
  }
}

// Step 1: B = R_Pi - (Q32 + M3rho M3^-1 D) M2lumped^-1 R_u, one thread per cell.
__global__ void k_schur_pressure_rhs(Topo t, const double *__restrict__ A, const double *__restrict__ m2l,
                                     const double *__restrict__ r, double *__restrict__ B) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t.ncell) return;
  double acc = r[t.nt + c];
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    double s;
    size_t Fb = cell_facet(t, c, b, s);
    if (s != 0.0) acc -= A[at(6 * 7 + b, t.ncell, c)] * s * r[Fb] / m2l[Fb];
  }
  B[c] = acc;
}

// Step 3: u = M2lumped^-1 (R_u - G Pi) on the facets (zero on the ground and lid), and the
// pressure of Step 2 copied into the cell part.
__global__ void k_schur_velocity(Topo t, const double *__restrict__ A, const double *__restrict__ kv,
                                 const double *__restrict__ m2l, const double *__restrict__ r,
                                 const double *__restrict__ pi, double *__restrict__ z) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.nt + t.ncell) return;
  if (i >= t.nt) {
    z[i] = pi[i - t.nt];
    return;
  }
  int cells[2], lfs[2];
  if (!facet_cells(t, i, cells, lfs)) {
    z[i] = 0.0;
    return;
  }
  const double J = kv[at(lfs[0], t.ncell, cells[0])] - kv[at(lfs[1], t.ncell, cells[1])];
  const double g0 = A[at(lfs[0] * 7 + 6, t.ncell, cells[0])] + 0.5 * J;
  const double g1 = -A[at(lfs[1] * 7 + 6, t.ncell, cells[1])] + 0.5 * J;
  z[i] = (r[i] - g0 * pi[cells[0]] - g1 * pi[cells[1]]) / m2l[i];
}

Topo topo(const hyb_ctx *c) {
  const LevelDev &L0 = c->lv[0];
  return Topo{c->nlev, c->ncol, c->nedge, c->ncell, (size_t)c->nz, (size_t)c->ntrace,
              L0.col_edge, L0.edge_col, L0.edge_lf};
}

}  // namespace

hipError_t launch_mixed_rows(hyb_ctx *c, const double *x, const double *b, double *y) {
  const Topo t = topo(c);
  const unsigned g = nblk(t.nt + t.ncell);
  if (b)
    hipLaunchKernelGGL(k_mixed_rows<1>, dim3(g), dim3(kBlock), 0, c->stream, t, (const double *)c->A,
                       (const double *)c->kv, x, b, y);
  else
    hipLaunchKernelGGL(k_mixed_rows<0>, dim3(g), dim3(kBlock), 0, c->stream, t, (const double *)c->A,
                       (const double *)c->kv, x, b, y);
  return hipGetLastError();
}

hipError_t launch_mixed_rhs(hyb_ctx *c, const double *r_ub, const double *r_pi, double *y) {
  const Topo t = topo(c);
  hipLaunchKernelGGL(k_mixed_rhs, dim3(nblk(t.nt + t.ncell)), dim3(kBlock), 0, c->stream, t, r_ub, r_pi, y);
  return hipGetLastError();
}

hipError_t schur_precondition(hyb_ctx *c, const double *r, double *z) {
  const Topo t = topo(c);
  LevelDev &L = c->lv[0];
  hipLaunchKernelGGL(k_schur_pressure_rhs, dim3(nblk(t.ncell)), dim3(kBlock), 0, c->stream, t,
                     (const double *)c->A, (const double *)c->m2l, r, (double *)L.b);
  HYB_TRY(hipGetLastError());
  HYB_TRY(coarse_vcycle(c));  // Step 2: one V-cycle from zero on H, L.b -> L.x
  hipLaunchKernelGGL(k_schur_velocity, dim3(nblk(t.nt + t.ncell)), dim3(kBlock), 0, c->stream, t,
                     (const double *)c->A, (const double *)c->kv, (const double *)c->m2l, r,
                     (const double *)L.x, z);
  return hipGetLastError();
}

}  // namespace hyb
