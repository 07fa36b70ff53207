// Trace operator, LineSmooth (Alg. 1), intergrid transfers and the pressure multigrid V-cycle,
// assembled into the non-nested two-level cycle (Alg. 2).
//
// Column kernels put one column per lane (64 consecutive columns per wavefront, so every access
// to a [k][col] array is coalesced) and walk up the column: the tridiagonal Thomas solve keeps its
// forward-elimination coefficients in LDS and runs the back substitution from there.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "hyb_internal.h"

namespace hyb {

namespace {

inline unsigned nblk(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

#define HYB_TRY(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

template <typename T>
struct Acc {
  using type = T;
};

// Row of S for the horizontal facet (k, col): neighbours below/above and the vertical facets of
// the two cells (layers k-1 and k), with the stencil order of the setup gather.  The stencil is
// read once per application, so its loads are non-temporal (they do not displace the gathered
// neighbour values from the caches; measured 2 % faster).
template <typename A, typename Tm, typename Tx>
__device__ __forceinline__ A row_z(const Tm *__restrict__ S, size_t ntr, const Tx *__restrict__ x, size_t F,
                                   int k, int nlev, int ncol, int nedge, size_t nz, const int ce[4]) {
  A acc = (A)__builtin_nontemporal_load(&S[s_idx(F, 0)]) * (A)x[F];
  if (k > 0) {
    size_t hb = nz + (size_t)(k - 1) * nedge;
    acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 1)]) * (A)x[F - ncol];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 3 + f)]) * (A)x[hb + ce[f]];
  }
  if (k < nlev) {
    size_t hb = nz + (size_t)k * nedge;
    acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 2)]) * (A)x[F + ncol];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 7 + f)]) * (A)x[hb + ce[f]];
  }
  return acc;
}

// Edge stencil table: est[0..7][e] = c0, c1, three other edges of c0, three other edges of c1.
template <typename A, typename Tm, typename Tx>
__device__ __forceinline__ A row_h(const Tm *__restrict__ S, size_t ntr, const Tx *__restrict__ x, size_t F,
                                   int k, int ncol, int nedge, size_t nz, const int t[8]) {
  size_t hb = nz + (size_t)k * nedge;
  size_t zb = (size_t)k * ncol;
  A acc = (A)__builtin_nontemporal_load(&S[s_idx(F, 0)]) * (A)x[F];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 1)]) * (A)x[zb + t[0]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 2)]) * (A)x[zb + ncol + t[0]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 3)]) * (A)x[hb + t[2]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 4)]) * (A)x[hb + t[3]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 5)]) * (A)x[hb + t[4]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 6)]) * (A)x[zb + t[1]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 7)]) * (A)x[zb + ncol + t[1]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 8)]) * (A)x[hb + t[5]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 9)]) * (A)x[hb + t[6]];
  acc += (A)__builtin_nontemporal_load(&S[s_idx(F, 10)]) * (A)x[hb + t[7]];
  return acc;
}

// Row operations on the trace operator.
//   OP_APPLY  y = S x
//   OP_RESID  y = b - S x
//   OP_SMOOTH LineSmooth rows: horizontal facets y = b - S x (kept for the column solve), vertical
//             facets lout = x + omega (b - S x) / diag(S^hh) (point Jacobi)
//   OP_SMOOTH0 the same from x = 0 on vertical facets only: lout = omega b / diag(S^hh)
enum { OP_APPLY = 0, OP_RESID = 1, OP_SMOOTH = 2, OP_SMOOTH0 = 3 };
constexpr int kRowBlock = 256;  // threads per workgroup of the row kernels (swept 64-512)
constexpr int kRowChunk = 2;  // layers per thread (swept 1-32 at 256x256x64: 2 is fastest)

template <typename Tm, typename Tx, typename Ty, int OP>
__device__ __forceinline__ void zrow_op(const Tm *__restrict__ S, const Tx *__restrict__ x, const Ty *__restrict__ b,
                                        Ty *__restrict__ y, int k, int col, int nlev, int ncol, int nedge, size_t nz,
                                        size_t ntr, const int ce[4]) {
  using A = typename Acc<Ty>::type;
  size_t F = (size_t)k * ncol + col;
  A v = row_z<A>(S, ntr, x, F, k, nlev, ncol, nedge, nz, ce);
  if (OP != OP_APPLY) v = (A)b[F] - v;
  y[F] = (Ty)v;
}

template <typename Tm, typename Tx, typename Ty, int OP>
__device__ __forceinline__ void hrow_op(const Tm *__restrict__ S, const Tx *__restrict__ x, const Ty *__restrict__ b,
                                        Ty *__restrict__ y, Ty *__restrict__ lout, int k, int e, int ncol, int nedge,
                                        size_t nz, size_t ntr, const int t[8], Ty omega) {
  using A = typename Acc<Ty>::type;
  size_t F = nz + (size_t)k * nedge + e;
  if (OP == OP_SMOOTH0) {
    lout[F] = omega * b[F] / (Ty)S[s_idx(F, 0)];
  } else {
    A v = row_h<A>(S, ntr, x, F, k, ncol, nedge, nz, t);
    if (OP != OP_APPLY) v = (A)b[F] - v;
    if (OP == OP_SMOOTH)
      lout[F] = (Ty)x[F] + omega * (Ty)v / (Ty)S[s_idx(F, 0)];
    else
      y[F] = (Ty)v;
  }
}

// A thread owns one column (its horizontal facets) or one edge (its vertical facets) for kRowChunk
// consecutive layers, so the neighbour tables are read once per chunk; at a fixed layer
// consecutive threads touch consecutive rows (coalesced).  Workgroups keep the hardware's
// round-robin placement over the XCDs: measured, it spreads the streams over the HBM channels
// better than giving each XCD a contiguous range (which would raise L2 reuse of the gathers).
template <typename Tm, typename Tx, typename Ty, int OP>
__global__ void __launch_bounds__(kRowBlock) k_rows(const Tm *__restrict__ S, const Tx *__restrict__ x,
                                                 const Ty *__restrict__ b, Ty *__restrict__ y,
                                                 Ty *__restrict__ lout, int nlev, int ncol, int nedge, size_t nz,
                                                 size_t ntr, int ent0, const int32_t *__restrict__ col_edge,
                                                 const int32_t *__restrict__ est, Ty omega) {
  const int ent = ent0 + blockIdx.x * blockDim.x + threadIdx.x;
  const int k0 = blockIdx.y * kRowChunk;
  if (ent < ncol) {
    if (OP == OP_SMOOTH0) return;
    const int col = ent;
    int ce[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) ce[f] = col_edge[(size_t)f * ncol + col];
#pragma unroll
    for (int q = 0; q < kRowChunk; ++q) {
      const int k = k0 + q;
      if (k <= nlev) zrow_op<Tm, Tx, Ty, OP>(S, x, b, y, k, col, nlev, ncol, nedge, nz, ntr, ce);
    }
  } else if (ent < ncol + nedge) {
    const int e = ent - ncol;
    int t[8];
    if (OP != OP_SMOOTH0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) t[i] = est[(size_t)i * nedge + e];
    }
#pragma unroll
    for (int q = 0; q < kRowChunk; ++q) {
      const int k = k0 + q;
      if (k < nlev) hrow_op<Tm, Tx, Ty, OP>(S, x, b, y, lout, k, e, ncol, nedge, nz, ntr, t, omega);
    }
  }
}

// grid of the row kernels: entities (columns, plus edges unless column-owned) x layer chunks
inline dim3 row_grid(const hyb_ctx *c, bool edges_only) {
  int ents = edges_only ? c->nedge : c->ncol + c->nedge;
  return dim3(nblk(ents, kRowBlock), (c->nlev + kRowChunk) / kRowChunk);
}
inline int row_ent0(const hyb_ctx *c, bool edges_only) { return edges_only ? c->ncol : 0; }

// Tridiagonal column solve with precomputed LU factors, one column per lane:
//   fac[0][i] = l_k (unit lower), fac[1][i] = 1/u_k, fac[2][i] = c_k/u_k, i = k*ncol + col,
//   y_k = R_k - l_k y_{k-1};  x_k = y_k/u_k - (c_k/u_k) x_{k+1};  out_k = base_k + omega x_k,
// base = 0 (ZERO), xin, or xin plus the injected coarse correction (ADDC).  The loads of KC levels
// are issued together before the recurrence runs over them, so a column pays the memory latency
// once per KC levels; y_k/u_k waits in LDS for the back substitution.  The factors of row k are at
// k * fcols + fmap[col] (fmap null: k * ncol + col): with fmap the patch of the column, a patch of
// columns shares one set of factors.
template <typename T, bool ZERO, bool ADDC>
__global__ void __launch_bounds__(kColBlock) k_column_solve(const T *__restrict__ R, const T *__restrict__ fac,
                                                            size_t fstride, const T *__restrict__ xin,
                                                            const T *__restrict__ xc, T *__restrict__ xout,
                                                            int nrows, int ncol, int ncolc,
                                                            const int32_t *__restrict__ parent, T omega,
                                                            const int32_t *__restrict__ fmap, int fcols) {
  constexpr int KC = 8;
  extern __shared__ unsigned char smem_raw[];
  T *wv = reinterpret_cast<T *>(smem_raw);
  const int tid = threadIdx.x, bd = blockDim.x;
  const int col = blockIdx.x * bd + tid;
  if (col >= ncol) return;
  const int fc = fmap ? fmap[col] : col;
  const int fcs = fmap ? fcols : ncol;
  T y = 0;
  for (int k0 = 0; k0 < nrows; k0 += KC) {
    T rv[KC], lv[KC], iv[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      int k = k0 + q;
      if (k < nrows) {
        size_t i = (size_t)k * ncol + col, f = (size_t)k * fcs + fc;
        rv[q] = R[i];
        lv[q] = fac[f];
        iv[q] = fac[fstride + f];
      }
    }
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      int k = k0 + q;
      if (k < nrows) {
        y = rv[q] - lv[q] * y;
        wv[(size_t)k * bd + tid] = y * iv[q];
      }
    }
  }
  const int pc = ADDC ? parent[col] : 0;
  T x = 0;
  for (int k1 = nrows - 1; k1 >= 0; k1 -= KC) {
    T cv[KC], bv[KC], w[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      int k = k1 - q;
      if (k >= 0) {
        size_t i = (size_t)k * ncol + col;
        cv[q] = fac[2 * fstride + (size_t)k * fcs + fc];
        w[q] = wv[(size_t)k * bd + tid];
        bv[q] = 0;
        if (!ZERO) {
          bv[q] = xin[i];
          if (ADDC) bv[q] += xc[(size_t)k * ncolc + pc];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      int k = k1 - q;
      if (k >= 0) {
        x = w[q] - cv[q] * x;
        xout[(size_t)k * ncol + col] = bv[q] + omega * x;
      }
    }
  }
}

// LU factors of the tridiagonal S^zz of every column (setup): row k has a_k (to facet k-1),
// b_k (diagonal), c_k (to facet k+1); l_k = a_k / u_{k-1}, u_k = b_k - l_k c_{k-1}.
__global__ void k_thomas_factor(const double *__restrict__ S, double *__restrict__ fac, int nlev, int ncol,
                                size_t nz, size_t ntr) {
  int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  double up = 1.0, cprev = 0.0;
  for (int k = 0; k <= nlev; ++k) {
    size_t F = (size_t)k * ncol + col;
    double a = S[s_idx(F, 1)], b = S[s_idx(F, 0)], c = S[s_idx(F, 2)];
    double l = (k == 0) ? 0.0 : a / up;
    double u = b - l * cprev;
    fac[F] = l;
    fac[nz + F] = 1.0 / u;
    fac[2 * nz + F] = c / u;
    up = u;
    cprev = c;
  }
}

// LU factors of the patch-cached column matrices (setup): the tridiagonal of each 2x2 patch of
// columns is the mean of its four columns' S^zz (below, diagonal, above per level), factored as in
// k_thomas_factor; one thread per patch, factors at k * npatch + patch.
__global__ void k_thomas_factor_patch(const double *__restrict__ S, double *__restrict__ fac, int nlev, int ncol,
                                      int npatch, const int32_t *__restrict__ children) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= npatch) return;
  int ch[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) ch[q] = children[(size_t)q * npatch + P];
  const size_t nzp = (size_t)(nlev + 1) * npatch;
  double up = 1.0, cprev = 0.0;
  for (int k = 0; k <= nlev; ++k) {
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const size_t F = (size_t)k * ncol + ch[q];
      a += S[s_idx(F, 1)], b += S[s_idx(F, 0)], c += S[s_idx(F, 2)];
    }
    a *= 0.25, b *= 0.25, c *= 0.25;
    const double l = (k == 0) ? 0.0 : a / up;
    const double u = b - l * cprev;
    const size_t f = (size_t)k * npatch + P;
    fac[f] = l;
    fac[nzp + f] = 1.0 / u;
    fac[2 * nzp + f] = c / u;
    up = u;
    cprev = c;
  }
}

// Restriction to the pressure space and scaling: Bbar_K = Gamma_K sum_F w_F R_F over the six
// facets of K, w = 1/2 (1 on ground and lid facets, where prolongation is one sided); gamma null:
// Gamma = 0.
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
  out[c] = gamma ? gamma[c] * s : (T)0;
}

// lambda_F += (P dPi)_F: average of the two cells of the facet (one sided on ground / lid).  Laid
// out like the row kernels: a thread owns one column (its horizontal facets) or one edge (its
// vertical facets) for kRowChunk consecutive layers, so the edge's two columns are read once per
// chunk and no facet index is divided back into (layer, column) (a thread per facet with 64-bit
// divisions ran at 3.9 TB/s).
template <typename T>
__global__ void __launch_bounds__(kRowBlock) k_prolong(const T *__restrict__ dpi, T *__restrict__ lam, int nlev,
                                                    int ncol, int nedge, size_t nz,
                                                    const int32_t *__restrict__ edge_col) {
  const int ent = blockIdx.x * blockDim.x + threadIdx.x;
  const int k0 = blockIdx.y * kRowChunk;
  if (ent < ncol) {
    const int col = ent;
#pragma unroll
    for (int q = 0; q < kRowChunk; ++q) {
      const int k = k0 + q;
      if (k > nlev) break;
      T v;
      if (k == 0)
        v = dpi[col];
      else if (k == nlev)
        v = dpi[(size_t)(nlev - 1) * ncol + col];
      else
        v = (T)0.5 * (dpi[(size_t)(k - 1) * ncol + col] + dpi[(size_t)k * ncol + col]);
      lam[(size_t)k * ncol + col] += v;
    }
  } else if (ent < ncol + nedge) {
    const int e = ent - ncol;
    const int c0 = edge_col[e], c1 = edge_col[nedge + e];
#pragma unroll
    for (int q = 0; q < kRowChunk; ++q) {
      const int k = k0 + q;
      if (k >= nlev) break;
      lam[nz + (size_t)k * nedge + e] += (T)0.5 * (dpi[(size_t)k * ncol + c0] + dpi[(size_t)k * ncol + c1]);
    }
  }
}

// LU factors of H_z per column (setup): a = coupling below, b = diagonal, c = coupling above.
__global__ void k_mg_factor(const double *__restrict__ H, double *__restrict__ fac, int nlev, int ncol) {
  int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  size_t n = (size_t)nlev * ncol;
  double up = 1.0, cprev = 0.0;
  for (int k = 0; k < nlev; ++k) {
    size_t c = (size_t)k * ncol + col;
    double a = H[5 * n + c], d = H[c], u = H[6 * n + c];
    double l = (k == 0) ? 0.0 : a / up;
    double piv = d - l * cprev;
    fac[c] = l;
    fac[n + c] = 1.0 / piv;
    fac[2 * n + c] = u / piv;
    up = piv;
    cprev = u;
  }
}

// Two entries of a [k][col] array at an even column, read as one aligned vector.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T a, b;
};
template <typename T>
__device__ __forceinline__ Pair<T> ld_pair(const T *p) {
  return *reinterpret_cast<const Pair<T> *>(p);
}

// Coarse right-hand side b_c = R (b - H x) (Sec. 2.3): the 7-point residual of the four children of a
// coarse cell, summed without going through memory.  One thread per coarse column and chunk of kl
// levels (consecutive threads take consecutive coarse columns of one chunk): the children's columns
// and their horizontal neighbours are read once per chunk, and x of the children at the levels below
// and above rides along in registers, so only the chunk's first level reloads them.  PAIRED: the
// children are columns c0, c0 + 1, c2, c2 + 1 with c0 and c2 even, and the stencil, b and x of each
// pair are loaded as one vector, so a wavefront's loads cover whole cache lines (with single loads
// every line is fetched by two instructions that each use half of it).  The arithmetic and its order
// per coarse cell do not depend on kl or PAIRED.
template <typename T, bool PAIRED>
__global__ void __launch_bounds__(kBlock) k_mg_restrict_residual(const T *__restrict__ H, const T *__restrict__ b,
                                                                const T *__restrict__ x, T *__restrict__ bc, int nlev,
                                                                int ncolf, int ncolc, int kl,
                                                                const int32_t *__restrict__ children,
                                                                const int32_t *__restrict__ nbr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nchunk = (nlev + kl - 1) / kl;
  if (t >= ncolc * nchunk) return;
  const int ch = t / ncolc, P = t - ch * ncolc;
  const int k0 = ch * kl, k1 = min(nlev, k0 + kl);
  const size_t n = (size_t)nlev * ncolf;
  int col[4], nb[4][4];
  if (PAIRED) {
    col[0] = children[P];
    col[1] = col[0] + 1;
    col[2] = children[(size_t)2 * ncolc + P];
    col[3] = col[2] + 1;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) col[q] = children[(size_t)q * ncolc + P];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int f = 0; f < 4; ++f) nb[q][f] = nbr[(size_t)f * ncolf + col[q]];
  // load the four children's entries of array a at level row `row` into v[0..3]
  auto load4 = [&](const T *a, size_t row, T v[4]) {
    if (PAIRED) {
      const Pair<T> p0 = ld_pair(a + row + col[0]), p1 = ld_pair(a + row + col[2]);
      v[0] = p0.a, v[1] = p0.b, v[2] = p1.a, v[3] = p1.b;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = a[row + col[q]];
    }
  };
  T xd[4], x0[4];  // x of each child at levels k - 1 and k
  if (k0 > 0)
    load4(x, (size_t)(k0 - 1) * ncolf, xd);
  else
#pragma unroll
    for (int q = 0; q < 4; ++q) xd[q] = T(0);
  load4(x, (size_t)k0 * ncolf, x0);
#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    const size_t row = (size_t)k * ncolf;
    T xu[4], h[7][4], bv[4];
    if (k < nlev - 1)
      load4(x, row + ncolf, xu);
    else
#pragma unroll
      for (int q = 0; q < 4; ++q) xu[q] = T(0);
#pragma unroll
    for (int s = 0; s < 7; ++s) load4(H + (size_t)s * n, row, h[s]);
    load4(b, row, bv);
    T s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T hx = h[0][q] * x0[q];
#pragma unroll
      for (int f = 0; f < 4; ++f) hx += h[1 + f][q] * x[row + nb[q][f]];
      if (k > 0) hx += h[5][q] * xd[q];
      if (k < nlev - 1) hx += h[6][q] * xu[q];
      s += bv[q] - hx;
      xd[q] = x0[q];
      x0[q] = xu[q];
    }
    bc[(size_t)k * ncolc + P] = s;
  }
}

// Levels per thread of the restriction: the largest power of two up to 8 that still leaves about
// 2^17 threads (measured on the 256x256x64 box: 77 us with 8 levels on the finest restriction
// against 90 us with one thread per coarse cell, 17.4 us with 2 on the next; one level below that).
inline int restrict_chunk(int nlev, int ncolc) {
  int kl = 1;
  while (kl < 8 && (size_t)ncolc * (size_t)(nlev / (2 * kl)) >= ((size_t)1 << 17)) kl *= 2;
  return kl;
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
  const bool patch = c->p.smoother_patch != 0;
  const T *fac = patch ? pick<T>(c->zfacp, c->zfacpf) : pick<T>(c->zfac, c->zfacf);
  const size_t fstride = patch ? (size_t)(c->nlev + 1) * c->lv[1].ncol : (size_t)c->nz;
  const int32_t *fmap = patch ? L0.parent : nullptr;
  const int fcols = patch ? c->lv[1].ncol : c->ncol;
  T *R = (T *)c->tR;
  T om = (T)c->p.omega;
  size_t ntr = (size_t)c->ntrace, nz = (size_t)c->nz;
  size_t shm = sizeof(T) * (size_t)(c->nlev + 1) * kColBlock;
  int fam = zero ? F_SMOOTH_ROWS0 : F_SMOOTH_ROWS;
  int slot = prof_begin(c, fam);
  dim3 grid = row_grid(c, zero);
  if (zero)
    hipLaunchKernelGGL((k_rows<T, T, T, OP_SMOOTH0>), grid, dim3(kRowBlock), 0, c->stream, S, lin, B, R, lout, c->nlev,
                       c->ncol, c->nedge, nz, ntr, row_ent0(c, true), L0.col_edge, L0.est, om);
  else
    hipLaunchKernelGGL((k_rows<T, T, T, OP_SMOOTH>), grid, dim3(kRowBlock), 0, c->stream, S, lin, B, R, lout, c->nlev,
                       c->ncol, c->nedge, nz, ntr, 0, L0.col_edge, L0.est, om);
  prof_end(c, fam, slot);
  HYB_TRY(hipGetLastError());
  slot = prof_begin(c, F_THOMAS);
  if (zero)
    hipLaunchKernelGGL((k_column_solve<T, true, false>), dim3(nblk(c->ncol, kColBlock)), dim3(kColBlock), shm,
                       c->stream, B, fac, fstride, lin, (const T *)nullptr, lout, c->nlev + 1, c->ncol, 1,
                       (const int32_t *)nullptr, om, fmap, fcols);
  else
    hipLaunchKernelGGL((k_column_solve<T, false, false>), dim3(nblk(c->ncol, kColBlock)), dim3(kColBlock), shm,
                       c->stream, (const T *)R, fac, fstride, lin, (const T *)nullptr, lout, c->nlev + 1, c->ncol, 1,
                       (const int32_t *)nullptr, om, fmap, fcols);
  prof_end(c, F_THOMAS, slot);
  return hipGetLastError();
}

constexpr int kPcrMaxColumns = 16384;
// columns per workgroup of the cyclic-reduction sweep (swept on the 256x256x64 box, multigrid
// smoothing per solve: 2 columns 7.5 ms, 4 columns 7.3, 8 columns 7.4, 16 columns 7.8; the form
// with a lane per level reading its column directly, 7.6)
constexpr int kPcrColumns = 4;

// One block-Jacobi sweep of the pressure multigrid, fused: x_out = base + omega H_z^-1 (b - H X) with
// X = 0 (MODE 0), xin (MODE 1) or xin plus the injected coarse correction xc[parent] (MODE 2), base = X;
// MODE 3 is a step of the Chebyshev semi-iteration, base = X + c1 (X - xprev).  A workgroup takes CPB
// consecutive columns of all levels (nlev <= 64) in three phases:
//  1. thread (k, c) = (t / CPB, t mod CPB) forms the residual of level k of column c and the row's
//     entries below / diagonal / above (H slots 5, 0, 6); a load covers CPB consecutive entries of
//     a level, so the loads are coalesced;
//  2. wavefront c takes column c, lane k = level k, and solves the tridiagonal column system by
//     parallel cyclic reduction: at stride s every row eliminates its couplings to rows k -/+ s, so
//     after ceil(log2 nlev) steps it is diagonal (lanes k >= nlev carry the identity row);
//  3. thread (k, c) stores the result, again coalesced.
// The rows meet in LDS with a stride of CPB + 1 entries.  The workgroups are handed to the 8 XCDs
// (workgroup b runs on XCD b mod 8, each with its own L2) in contiguous ranges of columns, so that
// horizontal neighbours mostly meet in one L2; any bijection of the blocks gives the same result.
template <typename T, int MODE, int CPB>
__global__ void __launch_bounds__(64 * CPB) k_mg_sweep_pcr(const T *__restrict__ H, const T *__restrict__ b,
                                                          const T *__restrict__ xin, const T *__restrict__ xc,
                                                          T *__restrict__ xout, int nlev, int ncol, int ncolc,
                                                          const int32_t *__restrict__ nbr,
                                                          const int32_t *__restrict__ parent, T omega,
                                                          const T *__restrict__ xprev, T c1) {
  constexpr int LS = CPB + 1;
  __shared__ T sa[64 * LS], sb[64 * LS], sc[64 * LS], sd[64 * LS], sx[64 * LS];
  const int nb = gridDim.x;
  const int blk = (nb & 7) == 0 ? (int)(blockIdx.x & 7) * (nb >> 3) + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  const int col0 = blk * CPB;
  const size_t n = (size_t)nlev * ncol;
  auto X = [&](int k, int cc) -> T {
    T v = xin[(size_t)k * ncol + cc];
    if (MODE == 2) v += xc[(size_t)k * ncolc + parent[cc]];
    return v;
  };
  {  // phase 1
    const int k = threadIdx.x / CPB, cc = threadIdx.x - k * CPB, col = col0 + cc;
    T am = 0, bm = 1, cm = 0, dm = 0, base = 0;
    if (k < nlev && col < ncol) {
      const size_t c = (size_t)k * ncol + col;
      am = k > 0 ? H[5 * n + c] : T(0);
      bm = H[c];
      cm = k < nlev - 1 ? H[6 * n + c] : T(0);
      dm = b[c];
      if (MODE != 0) {
        const T xk = X(k, col);
        T hx = bm * xk;
#pragma unroll
        for (int f = 0; f < 4; ++f) hx += H[(1 + f) * n + c] * X(k, nbr[(size_t)f * ncol + col]);
        dm -= hx;
        const T xdn = k > 0 ? X(k - 1, col) : T(0), xup = k < nlev - 1 ? X(k + 1, col) : T(0);
        dm -= am * xdn + cm * xup;  // am = 0 at the ground, cm = 0 at the lid
        base = xk;
        if (MODE == 3) base += c1 * (xk - (xprev ? xprev[c] : T(0)));  // a null xprev is the zero vector
      }
    }
    const int s = k * LS + cc;
    sa[s] = am, sb[s] = bm, sc[s] = cm, sd[s] = dm, sx[s] = base;
  }
  __syncthreads();
  {  // phase 2
    const int k = threadIdx.x & 63, w = threadIdx.x >> 6, s = k * LS + w;
    const bool on = k < nlev;
    T am = sa[s], bm = sb[s], cm = sc[s], dm = sd[s];
    for (int st = 1; st < nlev; st <<= 1) {
      const T a1 = __shfl_up(am, st, 64), b1 = __shfl_up(bm, st, 64), c1u = __shfl_up(cm, st, 64),
              d1 = __shfl_up(dm, st, 64);
      const T a2 = __shfl_down(am, st, 64), b2 = __shfl_down(bm, st, 64), c2 = __shfl_down(cm, st, 64),
              d2 = __shfl_down(dm, st, 64);
      const bool lo = k >= st, hi = k + st < nlev;
      const T al = (on && lo) ? -am / b1 : T(0), ga = (on && hi) ? -cm / b2 : T(0);
      const T an = lo ? al * a1 : T(0), cn = hi ? ga * c2 : T(0);
      const T bn = bm + (lo ? al * c1u : T(0)) + (hi ? ga * a2 : T(0));
      const T dn = dm + (lo ? al * d1 : T(0)) + (hi ? ga * d2 : T(0));
      if (on) am = an, bm = bn, cm = cn, dm = dn;
    }
    if (on) sx[s] = sx[s] + omega * (dm / bm);
  }
  __syncthreads();
  {  // phase 3
    const int k = threadIdx.x / CPB, cc = threadIdx.x - k * CPB, col = col0 + cc;
    if (k < nlev && col < ncol) xout[(size_t)k * ncol + col] = sx[k * LS + cc];
  }
}

// One block-Jacobi sweep of the pressure multigrid on a large level, fused into one pass up and down
// every column (one column per lane, 64 consecutive columns per wavefront, so every [k][col] access
// is coalesced): x_out = base + omega H_z^-1 (b - H X), with X = xin and base = X (MODE 1), or, for a
// Chebyshev step, base = X + c1 (X - xprev) (MODE 3; a null xprev is the zero vector).  On the way up each level's 7-point residual
// is formed from X of the column (kept in registers) and of its four neighbours and fed straight into
// the forward elimination with the LU factors of H_z; y_k / u_k waits in LDS for the back
// substitution on the way down, which reloads X for the base.  The loads of KC levels are issued
// before the recurrence runs over them.  This replaces a residual kernel and a column-solve kernel
// (the residual no longer goes through memory) with the same arithmetic in the same order.
template <typename T, int MODE, int KC>
__global__ void __launch_bounds__(kColBlock) k_mg_sweep_col(const T *__restrict__ H, const T *__restrict__ b,
                                                            const T *__restrict__ xin, const T *__restrict__ fac,
                                                            T *__restrict__ xout, int nlev, int ncol,
                                                            const int32_t *__restrict__ nbr, T omega,
                                                            const T *__restrict__ xprev, T c1) {
  extern __shared__ unsigned char smem_raw[];
  T *wv = reinterpret_cast<T *>(smem_raw);
  const int tid = threadIdx.x, bd = blockDim.x;
  const int col = blockIdx.x * bd + tid;
  if (col >= ncol) return;
  static_assert(MODE == 1 || MODE == 3, "plain and Chebyshev sweeps");
  const size_t n = (size_t)nlev * ncol;
  int nb[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) nb[f] = nbr[(size_t)f * ncol + col];
  auto X = [&](int k, int cc) -> T { return xin[(size_t)k * ncol + cc]; };
  T xdn = 0, x0 = X(0, col), y = 0;
  for (int k0 = 0; k0 < nlev; k0 += KC) {
    T hv[KC][7], bv[KC], xn[KC][4], xu[KC], lv[KC], iv[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      const int k = k0 + q;
      if (k < nlev) {
        const size_t c = (size_t)k * ncol + col;
#pragma unroll
        for (int s = 0; s < 5; ++s) hv[q][s] = H[(size_t)s * n + c];
        hv[q][5] = k > 0 ? H[5 * n + c] : T(0);
        hv[q][6] = k < nlev - 1 ? H[6 * n + c] : T(0);
        bv[q] = b[c];
#pragma unroll
        for (int f = 0; f < 4; ++f) xn[q][f] = X(k, nb[f]);
        xu[q] = k < nlev - 1 ? X(k + 1, col) : T(0);
        lv[q] = fac[c];
        iv[q] = fac[n + c];
      }
    }
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      const int k = k0 + q;
      if (k < nlev) {
        T hx = hv[q][0] * x0;
#pragma unroll
        for (int f = 0; f < 4; ++f) hx += hv[q][1 + f] * xn[q][f];
        if (k > 0) hx += hv[q][5] * xdn;
        if (k < nlev - 1) hx += hv[q][6] * xu[q];
        const T r = bv[q] - hx;
        y = r - lv[q] * y;
        wv[(size_t)k * bd + tid] = y * iv[q];
        xdn = x0;
        x0 = xu[q];
      }
    }
  }
  T x = 0;
  for (int k1 = nlev - 1; k1 >= 0; k1 -= KC) {
    T cv[KC], w[KC], base[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      const int k = k1 - q;
      if (k >= 0) {
        const size_t c = (size_t)k * ncol + col;
        cv[q] = fac[2 * n + c];
        w[q] = wv[(size_t)k * bd + tid];
        base[q] = X(k, col);
        if (MODE == 3) base[q] += c1 * (base[q] - (xprev ? xprev[c] : T(0)));
      }
    }
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      const int k = k1 - q;
      if (k >= 0) {
        x = w[q] - cv[q] * x;
        xout[(size_t)k * ncol + col] = base[q] + omega * x;
      }
    }
  }
}

// levels whose loads a column issues together in the fused sweep: 8 where the level fills at most
// one wavefront per SIMD (65536 columns: 84 us against 87 with 4), 4 beyond, where a second
// resident wavefront (the 8-level form needs all 256 registers) hides more of the latency
constexpr int kMgColKC = 4, kMgColKCWide = 8;
constexpr int kSimds = 1024;

template <typename T>
hipError_t mg_smooth(hyb_ctx *c, int l, const T *b, const T *xin, const T *xc, T *xout, int mode, T om,
                     const T *xprev = nullptr, T c1 = 0) {
  const LevelDev &Lv = c->lv[l];
  const T *H = pick<T>(Lv.H, Lv.Hf);
  const T *fac = pick<T>(Lv.zf, Lv.zff);
  size_t n = (size_t)c->nlev * Lv.ncol;
  size_t shm = sizeof(T) * (size_t)c->nlev * kColBlock;
  int ncolc = (l + 1 < c->nlevels) ? c->lv[l + 1].ncol : 1;
  dim3 gc(nblk(Lv.ncol, kColBlock)), bc(kColBlock);
  int slot = prof_begin(c, F_MG_SMOOTH);
  // the sweep with cyclic reduction (a wavefront per column) pays on levels of up to 16384 columns,
  // where a lane per column leaves the recurrence latency bound (256x256x64 box, multigrid smoothing
  // per solve: 7.36 ms with cyclic reduction up to 4096 columns, 7.30 up to 16384); on larger levels
  // its shuffles and divisions outweigh the latency it hides (up to 65536 columns: 9.34 ms), and the
  // lane-per-column sweep runs there
  if (c->nlev <= 64 && Lv.ncol <= kPcrMaxColumns) {
    constexpr int CPB = kPcrColumns;
    const dim3 gw(nblk(Lv.ncol, CPB)), bw(64 * CPB);
    if (mode == 0)
      hipLaunchKernelGGL((k_mg_sweep_pcr<T, 0, CPB>), gw, bw, 0, c->stream, H, b, xin, xc, xout, c->nlev, Lv.ncol,
                         ncolc, Lv.nbr, Lv.parent, om, xprev, c1);
    else if (mode == 1)
      hipLaunchKernelGGL((k_mg_sweep_pcr<T, 1, CPB>), gw, bw, 0, c->stream, H, b, xin, xc, xout, c->nlev, Lv.ncol,
                         ncolc, Lv.nbr, Lv.parent, om, xprev, c1);
    else if (mode == 2)
      hipLaunchKernelGGL((k_mg_sweep_pcr<T, 2, CPB>), gw, bw, 0, c->stream, H, b, xin, xc, xout, c->nlev, Lv.ncol,
                         ncolc, Lv.nbr, Lv.parent, om, xprev, c1);
    else
      hipLaunchKernelGGL((k_mg_sweep_pcr<T, 3, CPB>), gw, bw, 0, c->stream, H, b, xin, xc, xout, c->nlev, Lv.ncol,
                         ncolc, Lv.nbr, Lv.parent, om, xprev, c1);
  } else if (mode == 0) {
    hipLaunchKernelGGL((k_column_solve<T, true, false>), gc, bc, shm, c->stream, b, fac, n, xin, xc, xout, c->nlev,
                       Lv.ncol, ncolc, Lv.parent, om, (const int32_t *)nullptr, 0);
  } else if (mode == 1 || mode == 3) {
    const bool wide = (size_t)Lv.ncol <= (size_t)64 * kSimds;
    if (mode == 1 && wide)
      hipLaunchKernelGGL((k_mg_sweep_col<T, 1, kMgColKCWide>), gc, bc, shm, c->stream, H, b, xin, fac, xout, c->nlev,
                         Lv.ncol, Lv.nbr, om, xprev, c1);
    else if (mode == 1)
      hipLaunchKernelGGL((k_mg_sweep_col<T, 1, kMgColKC>), gc, bc, shm, c->stream, H, b, xin, fac, xout, c->nlev,
                         Lv.ncol, Lv.nbr, om, xprev, c1);
    else if (wide)
      hipLaunchKernelGGL((k_mg_sweep_col<T, 3, kMgColKCWide>), gc, bc, shm, c->stream, H, b, xin, fac, xout, c->nlev,
                         Lv.ncol, Lv.nbr, om, xprev, c1);
    else
      hipLaunchKernelGGL((k_mg_sweep_col<T, 3, kMgColKC>), gc, bc, shm, c->stream, H, b, xin, fac, xout, c->nlev,
                         Lv.ncol, Lv.nbr, om, xprev, c1);
  } else {
    // the coarse correction is injected into xin in place first (its caller drops xin after this
    // sweep): one streaming pass, then the plain sweep, which is cheaper than gathering the
    // correction for the column and its four neighbours at every level inside the sweep (65536
    // columns: 121 us fused)
    T *xw = const_cast<T *>(xin);
    hipLaunchKernelGGL((k_mg_prolong_add<T>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, xw, xc, c->nlev, Lv.ncol,
                       ncolc, Lv.parent);
    if ((size_t)Lv.ncol <= (size_t)64 * kSimds)
      hipLaunchKernelGGL((k_mg_sweep_col<T, 1, kMgColKCWide>), gc, bc, shm, c->stream, H, b, (const T *)xw, fac, xout,
                         c->nlev, Lv.ncol, Lv.nbr, om, xprev, c1);
    else
      hipLaunchKernelGGL((k_mg_sweep_col<T, 1, kMgColKC>), gc, bc, shm, c->stream, H, b, (const T *)xw, fac, xout,
                         c->nlev, Lv.ncol, Lv.nbr, om, xprev, c1);
  }
  prof_end(c, F_MG_SMOOTH, slot);
  return hipGetLastError();
}

// One V-cycle on level l from a zero initial guess: right-hand side lv[l].b, result lv[l].x.
template <typename T>
hipError_t vcycle(hyb_ctx *c, int l) {
  LevelDev &Lv = c->lv[l];
  size_t n = (size_t)c->nlev * Lv.ncol;
  T *b = (T *)Lv.b;
  const hyb_params &p = c->p;
  bool coarsest = (l == c->nlevels - 1);
  const T om = (T)p.omega_p;
  if (coarsest && p.mg_coarse_cheb) {
    // Chebyshev semi-iteration from x = 0 for H x = b, preconditioned by H_z, tuned to eigenvalues of
    // H_z^-1 H in [lo, hi]: x_1 = H_z^-1 b / theta, then
    // x_{k+1} = x_k + rho_k rho_{k-1} (x_k - x_{k-1}) + (2 rho_k / delta) H_z^-1 (b - H x_k),
    // rho_0 = delta / theta, rho_k = 1 / (2 theta / delta - rho_{k-1})
    const double theta = 0.5 * (p.cheb_hi + p.cheb_lo), delta = 0.5 * (p.cheb_hi - p.cheb_lo);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    void *buf[3] = {Lv.x, Lv.y, Lv.w};
    int cur = 0, prv = -1, nxt = 1;  // x_0 = 0 is passed as a null pointer
    HYB_TRY(mg_smooth<T>(c, l, b, nullptr, nullptr, (T *)buf[cur], 0, (T)(1.0 / theta)));
    for (int s = 1; s < p.mg_coarse_sweeps; ++s) {
      const double rho_next = 1.0 / (2.0 * sigma - rho);
      HYB_TRY(mg_smooth<T>(c, l, b, (const T *)buf[cur], nullptr, (T *)buf[nxt], 3, (T)(2.0 * rho_next / delta),
                           prv < 0 ? (const T *)nullptr : (const T *)buf[prv], (T)(rho_next * rho)));
      rho = rho_next;
      prv = cur, cur = nxt, nxt = 3 - prv - cur;
    }
    Lv.x = buf[cur], Lv.y = buf[(cur + 1) % 3], Lv.w = buf[(cur + 2) % 3];
    return hipSuccess;
  }
  int pre = coarsest ? p.mg_coarse_sweeps : p.mg_pre;
  if (pre <= 0) {
    hipLaunchKernelGGL((k_zero<T>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, (T *)Lv.x, n);
    HYB_TRY(hipGetLastError());
  } else {
    HYB_TRY(mg_smooth<T>(c, l, b, nullptr, nullptr, (T *)Lv.x, 0, om));
    for (int s = 1; s < pre; ++s) {
      HYB_TRY(mg_smooth<T>(c, l, b, (T *)Lv.x, nullptr, (T *)Lv.y, 1, om));
      std::swap(Lv.x, Lv.y);
    }
  }
  if (coarsest) return hipSuccess;
  LevelDev &Lc = c->lv[l + 1];
  const T *H = pick<T>(Lv.H, Lv.Hf);
  int slot = prof_begin(c, F_RESTRICT);
  const int kl = restrict_chunk(c->nlev, Lc.ncol);
  const dim3 rg(nblk((size_t)Lc.ncol * ((c->nlev + kl - 1) / kl)));
  auto al = [](const void *p) { return ((uintptr_t)p % (2 * sizeof(T))) == 0; };
  if (Lc.child_pairs && !(p.debug & HYB_DEBUG_UNPAIRED_RESTRICT) && al(H) && al(b) && al(Lv.x))
    hipLaunchKernelGGL((k_mg_restrict_residual<T, true>), rg, dim3(kBlock), 0, c->stream, H, b, (const T *)Lv.x,
                       (T *)Lc.b, c->nlev, Lv.ncol, Lc.ncol, kl, Lc.children, Lv.nbr);
  else
    hipLaunchKernelGGL((k_mg_restrict_residual<T, false>), rg, dim3(kBlock), 0, c->stream, H, b, (const T *)Lv.x,
                       (T *)Lc.b, c->nlev, Lv.ncol, Lc.ncol, kl, Lc.children, Lv.nbr);
  prof_end(c, F_RESTRICT, slot);
  HYB_TRY(hipGetLastError());
  HYB_TRY(vcycle<T>(c, l + 1));
  if (p.mg_post <= 0) {
    hipLaunchKernelGGL((k_mg_prolong_add<T>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, (T *)Lv.x,
                       (const T *)Lc.x, c->nlev, Lv.ncol, Lc.ncol, Lv.parent);
    return hipGetLastError();
  }
  HYB_TRY(mg_smooth<T>(c, l, b, (T *)Lv.x, (const T *)Lc.x, (T *)Lv.y, 2, om));
  std::swap(Lv.x, Lv.y);
  for (int s = 1; s < p.mg_post; ++s) {
    HYB_TRY(mg_smooth<T>(c, l, b, (T *)Lv.x, nullptr, (T *)Lv.y, 1, om));
    std::swap(Lv.x, Lv.y);
  }
  return hipSuccess;
}

// ---- Krylov coarse solve of the paper's Configurations 3a / 3b (coarse_mode 2, FP64) ----

// y = H x on multigrid level 0 (the 7-point pressure operator)
__global__ void k_h_apply(const double *__restrict__ H, const double *__restrict__ x, double *__restrict__ y,
                          int nlev, int ncol, const int32_t *__restrict__ nbr) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)nlev * ncol;
  if (c >= (int)n) return;
  const int k = c / ncol, col = c - k * ncol;
  double hx = H[c] * x[c];
#pragma unroll
  for (int f = 0; f < 4; ++f) hx += H[(1 + f) * n + c] * x[(size_t)k * ncol + nbr[(size_t)f * ncol + col]];
  if (k > 0) hx += H[5 * n + c] * x[c - ncol];
  if (k < nlev - 1) hx += H[6 * n + c] * x[c + ncol];
  y[c] = hx;
}

// up to three dot products at once: per-workgroup partial sums part[blk][j] (fixed order)
__global__ void __launch_bounds__(kBlock) k_dots3(const double *__restrict__ a0, const double *__restrict__ b0,
                                                  const double *__restrict__ a1, const double *__restrict__ b1,
                                                  const double *__restrict__ a2, const double *__restrict__ b2,
                                                  int k, size_t n, double *__restrict__ part) {
  __shared__ double sm[3][kBlock / 64];
  double v[3] = {0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    v[0] += a0[i] * b0[i];
    if (k > 1) v[1] += a1[i] * b1[i];
    if (k > 2) v[2] += a2[i] * b2[i];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_down(v[j], off, 64);
    if (lane == 0) sm[j][wave] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sm[threadIdx.x][w];
    part[(size_t)blockIdx.x * 3 + threadIdx.x] = t;
  }
}

__global__ void k_reduce3(const double *__restrict__ part, int nb, double *__restrict__ out) {
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[(size_t)b * 3 + threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// p = r + beta (p - omega v)
__global__ void k_bicg_dir(const double *__restrict__ r, const double *__restrict__ v, double *__restrict__ p,
                           double beta, double omega, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// y = x + a z
__global__ void k_axpy_to(const double *__restrict__ x, double a, const double *__restrict__ z, double *__restrict__ y,
                          size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] + a * z[i];
}

// x += a u + w q
__global__ void k_axpy2(double *__restrict__ x, double a, const double *__restrict__ u, double w,
                        const double *__restrict__ q, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += a * u[i] + w * q[i];
}

// (a_j, b_j) for j < k, summed on the device and read by the host
hipError_t dots(hyb_ctx *c, int k, const double *a0, const double *b0, const double *a1, const double *b1,
                const double *a2, const double *b2, size_t n, double *out) {
  const unsigned nb = std::min<unsigned>(1024, nblk(n));
  hipLaunchKernelGGL(k_dots3, dim3(nb), dim3(kBlock), 0, c->stream, a0, b0, a1 ? a1 : a0, b1 ? b1 : b0,
                     a2 ? a2 : a0, b2 ? b2 : b0, k, n, c->partial);
  hipLaunchKernelGGL(k_reduce3, dim3(1), dim3(64), 0, c->stream, (const double *)c->partial, (int)nb, c->hdev);
  HYB_TRY(hipGetLastError());
  HYB_TRY(hipMemcpyAsync(c->hhost, c->hdev, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HYB_TRY(hipStreamSynchronize(c->stream));
  for (int j = 0; j < k; ++j) out[j] = c->hhost[j];
  return hipSuccess;
}

// H x = b on level 0 (b in lv[0].b, x to lv[0].x) by BiCGStab (van der Vorst 1992; the right-preconditioned
// form of Saad, Iterative Methods for Sparse Linear Systems, Sec. 9.3) with one V-cycle as the
// preconditioner, from x = 0 until ||b - H x|| <= coarse_rtol ||b|| (at most kCoarseKrylovMax steps)
constexpr int kCoarseKrylovMax = 200;
hipError_t coarse_bicgstab(hyb_ctx *c) {
  LevelDev &L = c->lv[0];
  const size_t n = (size_t)c->nlev * L.ncol;
  if (!c->ck) {
    HYB_TRY(hipMalloc((void **)&c->ck, 10 * n * sizeof(double)));
    c->bytes += 10 * n * sizeof(double);
  }
  double *b = c->ck, *x = b + n, *r = x + n, *rh = r + n, *p = rh + n, *v = p + n, *sv = v + n, *t = sv + n,
         *ph = t + n, *sh = ph + n;
  double *Lb = (double *)L.b, *Lx = (double *)L.x;
  const dim3 g(nblk(n)), bl(kBlock);
  auto copy = [&](const double *src, double *dst) {
    hipLaunchKernelGGL((k_copy<double>), g, bl, 0, c->stream, src, dst, n);
    return hipGetLastError();
  };
  auto precond = [&](const double *y, double *yh) -> hipError_t {  // yh = V-cycle applied to y
    HYB_TRY(copy(y, Lb));
    HYB_TRY(vcycle<double>(c, 0));
    return copy(Lx, yh);
  };
  auto happly = [&](const double *y, double *Hy) {
    hipLaunchKernelGGL(k_h_apply, g, bl, 0, c->stream, (const double *)L.H, y, Hy, c->nlev, L.ncol, L.nbr);
    return hipGetLastError();
  };
  HYB_TRY(copy(Lb, b));
  HYB_TRY(copy(Lb, r));
  HYB_TRY(copy(Lb, rh));
  hipLaunchKernelGGL((k_zero<double>), g, bl, 0, c->stream, x, n);
  hipLaunchKernelGGL((k_zero<double>), g, bl, 0, c->stream, p, n);
  hipLaunchKernelGGL((k_zero<double>), g, bl, 0, c->stream, v, n);
  HYB_TRY(hipGetLastError());
  double d[3];
  HYB_TRY(dots(c, 1, b, b, nullptr, nullptr, nullptr, nullptr, n, d));
  const double bn = std::sqrt(d[0]), tol = c->p.coarse_rtol * bn;
  double rho = 1.0, alpha = 1.0, omega = 1.0, rho1 = d[0];  // rh = r = b at the start
  for (int it = 0; it < kCoarseKrylovMax && bn > 0.0; ++it) {
    if (rho1 == 0.0 || omega == 0.0) break;  // breakdown: keep the current iterate
    const double beta = (rho1 / rho) * (alpha / omega);
    hipLaunchKernelGGL(k_bicg_dir, g, bl, 0, c->stream, r, v, p, it == 0 ? 0.0 : beta, omega, n);
    HYB_TRY(hipGetLastError());
    HYB_TRY(precond(p, ph));
    HYB_TRY(happly(ph, v));
    HYB_TRY(dots(c, 1, rh, v, nullptr, nullptr, nullptr, nullptr, n, d));
    if (d[0] == 0.0) break;
    alpha = rho1 / d[0];
    hipLaunchKernelGGL(k_axpy_to, g, bl, 0, c->stream, r, -alpha, v, sv, n);
    HYB_TRY(hipGetLastError());
    HYB_TRY(dots(c, 1, sv, sv, nullptr, nullptr, nullptr, nullptr, n, d));
    if (std::sqrt(d[0]) <= tol) {
      hipLaunchKernelGGL(k_axpy2, g, bl, 0, c->stream, x, alpha, ph, 0.0, ph, n);
      HYB_TRY(hipGetLastError());
      break;
    }
    HYB_TRY(precond(sv, sh));
    HYB_TRY(happly(sh, t));
    HYB_TRY(dots(c, 2, t, sv, t, t, nullptr, nullptr, n, d));
    omega = d[1] > 0.0 ? d[0] / d[1] : 0.0;
    hipLaunchKernelGGL(k_axpy2, g, bl, 0, c->stream, x, alpha, ph, omega, sh, n);
    hipLaunchKernelGGL(k_axpy_to, g, bl, 0, c->stream, sv, -omega, t, r, n);
    HYB_TRY(hipGetLastError());
    rho = rho1;
    HYB_TRY(dots(c, 2, r, r, rh, r, nullptr, nullptr, n, d));
    rho1 = d[1];
    if (std::sqrt(d[0]) <= tol) break;
  }
  return copy(x, Lx);
}

}  // namespace

template <typename Tm, typename Tx, typename Ty>
hipError_t launch_trace_apply(hyb_ctx *c, const Tm *S, const Tx *x, const Ty *b, Ty *y, int mode) {
  const LevelDev &L0 = c->lv[0];
  int slot = prof_begin(c, F_TRACE_APPLY);
  dim3 grid = row_grid(c, false);
  if (mode == 0)
    hipLaunchKernelGGL((k_rows<Tm, Tx, Ty, OP_APPLY>), grid, dim3(kRowBlock), 0, c->stream, S, x, b, y, (Ty *)nullptr,
                       c->nlev, c->ncol, c->nedge, (size_t)c->nz, (size_t)c->ntrace, 0, L0.col_edge, L0.est, (Ty)0);
  else
    hipLaunchKernelGGL((k_rows<Tm, Tx, Ty, OP_RESID>), grid, dim3(kRowBlock), 0, c->stream, S, x, b, y, (Ty *)nullptr,
                       c->nlev, c->ncol, c->nedge, (size_t)c->nz, (size_t)c->ntrace, 0, L0.col_edge, L0.est, (Ty)0);
  prof_end(c, F_TRACE_APPLY, slot);
  return hipGetLastError();
}

template hipError_t launch_trace_apply<double, double, double>(hyb_ctx *, const double *, const double *,
                                                               const double *, double *, int);
template hipError_t launch_trace_apply<double, float, double>(hyb_ctx *, const double *, const float *,
                                                              const double *, double *, int);
template hipError_t launch_trace_apply<float, float, float>(hyb_ctx *, const float *, const float *, const float *,
                                                            float *, int);

// Alg. 2 from a zero initial guess: z = M(r) (with coarse_mode 1, the LineSmooth sweeps alone).
template <typename T>
hipError_t precondition(hyb_ctx *c, const T *r, T *z) {
  const hyb_params &p = c->p;
  const T *S = pick<T>(c->S, c->Sf);
  // debug bit 1: Gamma taken as zero, so the coarse correction adds nothing (failure injection)
  const T *gam = (p.debug & HYB_DEBUG_ZERO_GAMMA) ? nullptr : pick<T>(c->gamma, c->gammaf);
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
  if (p.coarse_mode != 1) {
    // residual, restriction and scaling
    HYB_TRY((launch_trace_apply<T, T, T>(c, S, tA, r, tR, 1)));
    int slot = prof_begin(c, F_RESTRICT);
    hipLaunchKernelGGL((k_restrict<T>), dim3(nblk(c->ncell)), dim3(kBlock), 0, c->stream, tR, gam, (T *)c->lv[0].b,
                       c->nlev, c->ncol, c->nedge, (size_t)c->nz, L0.col_edge);
    prof_end(c, F_RESTRICT, slot);
    HYB_TRY(hipGetLastError());
    // coarse solve: one pressure multigrid V-cycle, or (coarse_mode 2, FP64) BiCGStab preconditioned by it
    if (p.coarse_mode == 2) {
      if constexpr (std::is_same<T, double>::value)
        HYB_TRY(coarse_bicgstab(c));
      else
        return hipErrorInvalidValue;  // rejected by the parameter check
    } else {
      HYB_TRY(vcycle<T>(c, 0));
    }
    // prolongation and update
    slot = prof_begin(c, F_PROLONG);
    hipLaunchKernelGGL((k_prolong<T>), row_grid(c, false), dim3(kRowBlock), 0, c->stream, (const T *)c->lv[0].x, tA,
                       c->nlev, c->ncol, c->nedge, (size_t)c->nz, L0.edge_col);
    prof_end(c, F_PROLONG, slot);
    HYB_TRY(hipGetLastError());
  }  // coarse_mode 1: LineSmooth alone (no coarse correction)
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
  int need = (int)(sizeof(double) * (size_t)(nlev + 1) * kColBlock);
  if (need <= 65536) return hipSuccess;
  const void *fns[] = {
      (const void *)k_column_solve<double, true, false>, (const void *)k_column_solve<double, false, false>,
      (const void *)k_column_solve<double, false, true>, (const void *)k_column_solve<float, true, false>,
      (const void *)k_column_solve<float, false, false>, (const void *)k_column_solve<float, false, true>,
      (const void *)k_mg_sweep_col<double, 1, kMgColKC>, (const void *)k_mg_sweep_col<double, 3, kMgColKC>,
      (const void *)k_mg_sweep_col<float, 1, kMgColKC>, (const void *)k_mg_sweep_col<float, 3, kMgColKC>,
      (const void *)k_mg_sweep_col<double, 1, kMgColKCWide>, (const void *)k_mg_sweep_col<double, 3, kMgColKCWide>,
      (const void *)k_mg_sweep_col<float, 1, kMgColKCWide>, (const void *)k_mg_sweep_col<float, 3, kMgColKCWide>};
  for (const void *f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, need);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_mg_factor(hyb_ctx *c, int l) {
  const LevelDev &Lv = c->lv[l];
  hipLaunchKernelGGL(k_mg_factor, dim3(nblk(Lv.ncol, kColBlock)), dim3(kColBlock), 0, c->stream, Lv.H, Lv.zf, c->nlev,
                     Lv.ncol);
  return hipGetLastError();
}

hipError_t launch_thomas_factor(hyb_ctx *c) {
  hipLaunchKernelGGL(k_thomas_factor, dim3(nblk(c->ncol, kColBlock)), dim3(kColBlock), 0, c->stream, c->S, c->zfac,
                     c->nlev, c->ncol, (size_t)c->nz, (size_t)c->ntrace);
  if (c->zfacp) {
    const int np = c->lv[1].ncol;
    hipLaunchKernelGGL(k_thomas_factor_patch, dim3(nblk(np, kColBlock)), dim3(kColBlock), 0, c->stream, c->S, c->zfacp,
                       c->nlev, c->ncol, np, c->lv[1].children);
  }
  return hipGetLastError();
}

// FP64 V-cycle on level 0 (lv[0].b -> lv[0].x), for a context used as another's coarse space
hipError_t coarse_vcycle(hyb_ctx *c) { return vcycle<double>(c, 0); }

}  // namespace hyb
