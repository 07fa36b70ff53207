// Next-to-lowest-order (p = 1) hybridised system on the box: RT1 broken velocity (36 per cell),
// DG1 pressure nodal at the 2x2x2 Gauss points (8), Q1 trace nodal at the 2x2 face Gauss points
// (4 per facet, trace dof 4 F + i).  The paper states the method for general p (Sec. 2.2 forms,
// n = p + 3 point Gauss rules, q32 / m3^rho / m3^Pi at the W3 nodes; Sec. 2.4 hybridisation) and
// the p = 1 sizes in its table of unknowns (44 x 44 cell matrices, 24 x 24 condensed blocks).
//
// Every form is linear in the cell's coefficients (cell sizes, theta* and Pi-hat* at the bottom
// and top facets, the cell values of Pi* and rho*), so the assembly multiplies reference tables --
// integrals of products of the reference basis functions, computed once on the host with exact
// Gauss rules -- by per-cell scalars.  Cell data are stored per cell (array of structures): one
// wavefront owns one cell in the assembly and the condensation, and reads the 748 entries of A_K
// that the block structure leaves non-zero contiguously.  The condensed blocks S_K are stored entry by entry over
// the cells ([24 x 24][ncell]): the trace rows of consecutive cells then read consecutive addresses.
//
// Dof order per cell: velocity face dofs 4 f + i (f = W, E, S, N, B, T; face point i = 2 t1 + t2
// in the face's tangential coordinates (y, z), (x, z) or (x, y)), velocity interior dofs
// 24 + 4 d + (2 t1 + t2), then the 8 pressure dofs 36 + 4 i + 2 j + k.
#include <cmath>
#include <vector>

#include "hyb_internal.h"

namespace hyb {

namespace {

constexpr int NU = 36, NPR = 8, NF = 24, NX = 44, NS = NF * NF;

inline unsigned nblk(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// ---- reference tables (host) ------------------------------------------------------------------
// tbl layout (doubles): Tm2[36][36], Tzz[36][36], TgB[36][8], TgT[36][8], Tgz[36][8], Td[8][36],
// Uz[36][8], dir[36] (direction of each velocity function, as double)
constexpr int OFF_M2 = 0, OFF_ZZ = OFF_M2 + NU * NU, OFF_GB = OFF_ZZ + NU * NU, OFF_GT = OFF_GB + NU * NPR,
              OFF_GZ = OFF_GT + NU * NPR, OFF_TD = OFF_GZ + NU * NPR, OFF_UZ = OFF_TD + NPR * NU,
              OFF_DIR = OFF_UZ + NU * NPR, TBL_LEN = OFF_DIR + NU;

struct Basis1D {
  // Lagrange polynomials on nodes; value and derivative
  std::vector<double> nodes;
  double val(int j, double x) const {
    double v = 1.0;
    for (size_t m = 0; m < nodes.size(); ++m)
      if ((int)m != j) v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
    return v;
  }
  double der(int j, double x) const {
    double d = 0.0;
    for (size_t m = 0; m < nodes.size(); ++m) {
      if ((int)m == j) continue;
      double t = 1.0 / (nodes[j] - nodes[m]);
      for (size_t q = 0; q < nodes.size(); ++q)
        if ((int)q != j && q != m) t *= (x - nodes[q]) / (nodes[j] - nodes[q]);
      d += t;
    }
    return d;
  }
};

struct RT1Fn {
  int d, a, t1, t2;
  double sgn;
};

std::vector<RT1Fn> rt1_functions() {
  const int fdir[6] = {0, 0, 1, 1, 2, 2};
  const double fsgn[6] = {-1, 1, -1, 1, -1, 1};
  std::vector<RT1Fn> out;
  for (int f = 0; f < 6; ++f)
    for (int i = 0; i < 4; ++i) out.push_back({fdir[f], fsgn[f] < 0 ? 0 : 2, i / 2, i % 2, fsgn[f]});
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < 4; ++i) out.push_back({d, 1, i / 2, i % 2, 1.0});
  return out;
}

std::vector<double> build_tables() {
  const double g0 = 0.5 - 0.5 / std::sqrt(3.0), g1 = 0.5 + 0.5 / std::sqrt(3.0);
  Basis1D Lq{{0.0, 0.5, 1.0}}, Lg{{g0, g1}};
  // 4-point Gauss-Legendre on [0, 1] (exact for the products below)
  const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0)),
               b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double xs[4] = {-b, -a, a, b};
  const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
  const double ws[4] = {wb, wa, wa, wb};
  double X[4], W[4];
  for (int i = 0; i < 4; ++i) X[i] = 0.5 * (xs[i] + 1.0), W[i] = 0.5 * ws[i];
  auto fns = rt1_functions();
  const int tang[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  auto uval = [&](const RT1Fn &f, const double p[3]) {
    return f.sgn * Lq.val(f.a, p[f.d]) * Lg.val(f.t1, p[tang[f.d][0]]) * Lg.val(f.t2, p[tang[f.d][1]]);
  };
  auto udiv = [&](const RT1Fn &f, const double p[3]) {  // d/d(own reference coordinate)
    return f.sgn * Lq.der(f.a, p[f.d]) * Lg.val(f.t1, p[tang[f.d][0]]) * Lg.val(f.t2, p[tang[f.d][1]]);
  };
  auto phi = [&](int q, const double p[3]) {
    return Lg.val(q / 4, p[0]) * Lg.val((q / 2) % 2, p[1]) * Lg.val(q % 2, p[2]);
  };
  std::vector<double> T(TBL_LEN, 0.0);
  for (int ix = 0; ix < 4; ++ix)
    for (int iy = 0; iy < 4; ++iy)
      for (int iz = 0; iz < 4; ++iz) {
        const double p[3] = {X[ix], X[iy], X[iz]}, w = W[ix] * W[iy] * W[iz];
        double u[NU], dv[NU], ph[NPR];
        for (int j = 0; j < NU; ++j) u[j] = uval(fns[j], p), dv[j] = udiv(fns[j], p);
        for (int q = 0; q < NPR; ++q) ph[q] = phi(q, p);
        for (int i = 0; i < NU; ++i) {
          for (int j = 0; j < NU; ++j) {
            if (fns[i].d == fns[j].d) T[OFF_M2 + i * NU + j] += w * u[i] * u[j];
            if (fns[i].d == 2 && fns[j].d == 2) T[OFF_ZZ + i * NU + j] += w * u[i] * u[j];
          }
          for (int q = 0; q < NPR; ++q) {
            T[OFF_GB + i * NPR + q] += w * (1.0 - p[2]) * dv[i] * ph[q];
            T[OFF_GT + i * NPR + q] += w * p[2] * dv[i] * ph[q];
            if (fns[i].d == 2) T[OFF_GZ + i * NPR + q] += w * u[i] * ph[q];
            T[OFF_TD + q * NU + i] += w * ph[q] * dv[i];
          }
        }
      }
  const double G[2] = {g0, g1};
  for (int i = 0; i < NU; ++i) {
    for (int q = 0; q < NPR; ++q) {
      const double p[3] = {G[q / 4], G[(q / 2) % 2], G[q % 2]};
      T[OFF_UZ + i * NPR + q] = fns[i].d == 2 ? uval(fns[i], p) : 0.0;
    }
    T[OFF_DIR + i] = fns[i].d;
  }
  return T;
}

// ---- kernels ----------------------------------------------------------------------------------

struct CellCoef {
  double hx, hy, hz, thB, thT, dpi, pic, rhoc;
};

__device__ __forceinline__ CellCoef cell_coef(int c, int ncol, const double *dz, double dx, double dy,
                                              const double *theta_w, const double *exner_hat_w,
                                              const double *exner_c, const double *rho_c) {
  const int k = c / ncol, col = c - k * ncol;
  CellCoef q;
  q.hx = dx, q.hy = dy, q.hz = dz[k];
  q.thB = theta_w[(size_t)k * ncol + col], q.thT = theta_w[(size_t)(k + 1) * ncol + col];
  q.dpi = (exner_hat_w[(size_t)(k + 1) * ncol + col] - exner_hat_w[(size_t)k * ncol + col]) / q.hz;
  q.pic = exner_c[c], q.rhoc = rho_c[c];
  return q;
}

// Workgroups go to the 8 XCDs in turn (workgroup b to XCD b mod 8), each with its own L2.  Kernels
// that write entry by entry over the cells renumber their workgroups so that each XCD owns one
// contiguous range of cells: neighbouring cells, whose values share cache lines, are then written
// through the same L2 and leave it as whole lines.
__device__ __forceinline__ int xcd_block() {
  constexpr int kXcd = 8;
  const int b = blockIdx.x, n = gridDim.x, x = b % kXcd, base = n / kXcd, rem = n % kXcd;
  return x * base + (x < rem ? x : rem) + b / kXcd;
}

// The velocity block M = m2 - q22 of an axis-aligned cell in twelve 3 x 3 blocks: block 4 d + i holds the
// two face functions and the interior function of direction d at tangential point i.
__device__ __forceinline__ int blk_dof(int blk, int r) {  // dof of position r (0: "-" face, 1: "+" face, 2: interior)
  const int d = blk >> 2, i = blk & 3;
  return r == 0 ? 8 * d + i : (r == 1 ? 8 * d + 4 + i : 24 + 4 * d + i);
}
__device__ __forceinline__ void dof_blk(int a, int &blk, int &r) {
  if (a < 24) {
    const int f = a >> 2, i = a & 3;
    blk = 4 * (f >> 1) + i, r = f & 1;
  } else {
    blk = a - 24, r = 2;  // 24 + 4 d + i  ->  block 4 d + i
  }
}

// A_K as the library keeps it: the entries that the block structure of an axis-aligned cell leaves
// non-zero (M block diagonal in the twelve 3 x 3 blocks, the pressure block diagonal), cell by cell
// ([ncell][NAC]: the condensation kernels give each cell a wavefront, whose loads then stay inside
// the cell's 6 KB; laid out entry by entry over the cells they ran 1.2-1.4x slower): block b of M at
// AO_M + 9 b + 3 r + q (rows and columns blk_dof(b, .)), G (velocity row a, pressure column p) at
// AO_G + 8 a + p, the pressure rows Dr = q32 + M3^rho M3^-1 D at AO_DR + 36 p + a, the pressure
// block at AO_P + 8 p + q.  Every other entry of the 44 x 44 matrix is zero.
constexpr int AO_M = 0, AO_G = 108, AO_DR = AO_G + 288, AO_P = AO_DR + 288, NAC = AO_P + 64;

// position of entry (i, j) of A_K in the compact layout, -1 where the structure makes it zero
__device__ __forceinline__ int a_compact(int i, int j) {
  if (i < NU && j < NU) {
    int bi, ri, bj, rj;
    dof_blk(i, bi, ri);
    dof_blk(j, bj, rj);
    return bi == bj ? AO_M + 9 * bi + 3 * ri + rj : -1;
  }
  if (i < NU) return AO_G + NPR * i + (j - NU);
  if (j < NU) return AO_DR + NU * (i - NU) + j;
  return AO_P + NPR * (i - NU) + (j - NU);
}

// entry (i, j) of A_K at position e of the compact layout
__device__ __forceinline__ void a_entry_of(int e, int &i, int &j) {
  if (e < AO_G) {
    const int b = e / 9, r = (e % 9) / 3;
    i = blk_dof(b, r), j = blk_dof(b, e % 3);
  } else if (e < AO_DR) {
    i = (e - AO_G) / NPR, j = NU + (e - AO_G) % NPR;
  } else if (e < AO_P) {
    i = NU + (e - AO_DR) / NU, j = (e - AO_DR) % NU;
  } else {
    i = NU + (e - AO_P) / NPR, j = NU + (e - AO_P) % NPR;
  }
}

// One wavefront per cell writes the compact A_K (its lanes along the entries) and the diagonals of
// C_K and K_K ([ncell][24]).
__global__ void __launch_bounds__(kBlock) k_p1_assemble(int ncell, int ncol, const double *__restrict__ dz, double dx,
                                                        double dy, const double *__restrict__ theta_w,
                                                        const double *__restrict__ exner_hat_w,
                                                        const double *__restrict__ exner_c,
                                                        const double *__restrict__ rho_c,
                                                        const double *__restrict__ T, double dt, double tu,
                                                        double tr, double tt, double cp, double kappa,
                                                        double *__restrict__ A, double *__restrict__ cdiag,
                                                        double *__restrict__ kdiag) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (c >= ncell) return;
  const CellCoef q = cell_coef(c, ncol, dz, dx, dy, theta_w, exner_hat_w, exner_c, rho_c);
  const double vol = q.hx * q.hy * q.hz, dth = (q.thT - q.thB) / q.hz;
  const double h[3] = {q.hx, q.hy, q.hz};
  const double c22 = tu * tt * dt * dt * cp * q.dpi * dth * vol, cg = -tu * dt * cp * vol, cd = tr * dt * vol;
  const double G0 = 0.5 - 0.5 / sqrt(3.0), G1 = 0.5 + 0.5 / sqrt(3.0);
  double *Ac = A + (size_t)c * NAC;
  for (int e = lane; e < NAC; e += 64) {
    int i, j;
    a_entry_of(e, i, j);
    double v;
    if (i < NU && j < NU) {  // m2 - q22
      v = vol * T[OFF_M2 + i * NU + j] - c22 * T[OFF_ZZ + i * NU + j];
    } else if (i < NU) {  // g^b: velocity row i, pressure column
      const int p = j - NU;
      const double hi = h[(int)T[OFF_DIR + i]];
      v = cg * ((q.thB * T[OFF_GB + i * NPR + p] + q.thT * T[OFF_GT + i * NPR + p]) / hi + dth * T[OFF_GZ + i * NPR + p]);
    } else if (j < NU) {  // q32 + M3rho M3^-1 D: pressure row, velocity column
      const int p = i - NU;
      const double hj = h[(int)T[OFF_DIR + j]];
      const double zp = (p % 2) ? G1 : G0;
      const double thp = q.thB * (1.0 - zp) + q.thT * zp;
      v = tt * dt * 0.125 * vol * T[OFF_UZ + j * NPR + p] * dth / thp + cd * T[OFF_TD + p * NU + j] / hj;
    } else {  // m3^Pi, nodal
      v = (i == j) ? (1.0 - kappa) / kappa * 0.125 * vol / q.pic : 0.0;
    }
    Ac[e] = v;
  }
  if (lane < NF) {
    const int f = lane / 4, i = lane % 4;
    const double area = (f < 2) ? q.hy * q.hz : (f < 4) ? q.hx * q.hz : q.hx * q.hy;
    double th;
    if (f < 4)
      th = (i % 2) ? q.thB * (1.0 - G1) + q.thT * G1 : q.thB * (1.0 - G0) + q.thT * G0;
    else
      th = (f == 4) ? q.thB : q.thT;
    cdiag[(size_t)c * NF + lane] = 0.25 * area;
    kdiag[(size_t)c * NF + lane] = tu * dt * cp * 0.25 * area * th;
  }
}

// ---- condensation on MFMA ------------------------------------------------------------------------
// S_K from A_K and K_K with matrix cores: one wavefront per cell; [A_K | [K_K; 0]] padded to 48 rows,
// 48 + 32 columns (identity on the padding), FP32, held in registers as 3 x 5 tiles of 16 x 16 in the
// accumulator layout of the 16x16 MFMA (lane l: rows 4 (l / 16) .. + 3, column l mod 16 of every
// tile).  Blocked right-looking elimination without pivoting, block 16: within a block each pivot
// row and column is shuffled across the lanes and the lanes update their own entries; after the block
// the trailing update A22 -= L21 U12 runs on MFMA straight into the accumulators (L21 and U12
// staged through LDS into the operand layouts).  Then the blocked back substitution: the diagonal
// blocks row by row, the blocks above by MFMA.  SPLIT: each FP32 operand is split into BF16 hi + lo
// and a tile product is hi*lo + lo*hi + hi*hi (FP32 accumulation), else FP32 MFMA.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
constexpr int MP = 48, MW = 80;  // padded size, augmented width
constexpr int TS = 17;           // row stride of a 16 x 16 tile staged in LDS
constexpr int kMW = 4;           // cells (wavefronts) per workgroup

__device__ __forceinline__ short bf16_rne(float f) {
  const unsigned u = __float_as_uint(f);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

// entry q of an accumulator with q known only at run time (no dynamic register indexing)
__device__ __forceinline__ float f4_get(const f32x4 &v, int q) {
  return q == 0 ? v[0] : (q == 1 ? v[1] : (q == 2 ? v[2] : v[3]));
}
__device__ __forceinline__ void f4_set(f32x4 &v, int q, float x) {
  if (q == 0) v[0] = x;
  else if (q == 1) v[1] = x;
  else if (q == 2) v[2] = x;
  else v[3] = x;
}

// acc - L U for 16 x 16 tiles L, U staged row-major in LDS.  Operand layouts: FP32 16x16x4:
// a = A[l%16][l/16], b = B[l/16][l%16]; BF16 16x16x16: a[j] = A[l%16][4(l/16)+j], b[j] = B[4(l/16)+j][l%16];
// result d[j] = D[4(l/16)+j][l%16], the layout of acc.
template <bool SPLIT>
__device__ __forceinline__ f32x4 tile_msub(const float *L, const float *U, f32x4 acc, int lc, int lg) {
  if constexpr (!SPLIT) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(-L[lc * TS + 4 * s + lg], U[(4 * s + lg) * TS + lc], acc, 0, 0, 0);
  } else {
    bf16x4 ah, al, bh, bl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float a = -L[lc * TS + 4 * lg + j], b = U[(4 * lg + j) * TS + lc];
      const short a1 = bf16_rne(a), b1 = bf16_rne(b);
      ah[j] = a1, al[j] = bf16_rne(a - bf16_val(a1));
      bh[j] = b1, bl[j] = bf16_rne(b - bf16_val(b1));
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
  }
  return acc;
}

struct MfmaLds {
  float stg[6][16 * TS];  // tiles staged for MFMA operands; at the end the 24 x 24 result
};

// The 16 pivots of block KB.  Lane l holds column 16 tj + l mod 16 of rows 16 ti + 4 (l / 16) + q,
// so the pivot row's entry of a lane's column comes from lane 16 (kk / 4) + l mod 16 and the pivot
// column's entry of a lane's row from lane 16 (l / 16) + kk: shuffles, no barriers.
template <int KB>
__device__ __forceinline__ void mf_elim_block(f32x4 (&acc)[3][5], int lc, int lg) {
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 16 * KB + kk, qk = kk & 3, src_row = 16 * (kk >> 2) + lc, src_col = 16 * lg + kk;
    float prow[5], pcol[3][4];
#pragma unroll
    for (int tj = KB; tj < 5; ++tj) prow[tj] = __shfl(f4_get(acc[KB][tj], qk), src_row);
    const float inv = 1.f / __shfl(prow[KB], kk);  // lane kk holds column k of the pivot row
#pragma unroll
    for (int ti = KB; ti < 3; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) pcol[ti][q] = __shfl(acc[ti][KB][q], src_col);
    // rows of the block below the pivot: every column right of it (U12 and the right-hand sides)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (16 * KB + 4 * lg + q > k) {
        const float l = pcol[KB][q] * inv;
#pragma unroll
        for (int tj = KB; tj < 5; ++tj)
          if (16 * tj + lc > k) acc[KB][tj][q] -= l * prow[tj];
      }
    }
    // rows below the block: the panel columns right of the pivot; the multiplier into column k
#pragma unroll
    for (int ti = KB + 1; ti < 3; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float l = pcol[ti][q] * inv;
        const int j = 16 * KB + lc;
        if (j > k) acc[ti][KB][q] -= l * prow[KB];
        else if (j == k) acc[ti][KB][q] = l;
      }
  }
}

// A22 -= L21 U12 after block KB (KB < 2); every wavefront of the workgroup reaches the barriers
template <int KB, bool SPLIT>
__device__ __forceinline__ void mf_trailing(f32x4 (&acc)[3][5], MfmaLds &S, bool active, int lc, int lg) {
  if (active) {
#pragma unroll
    for (int ti = KB + 1; ti < 3; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) S.stg[ti - KB - 1][(4 * lg + q) * TS + lc] = acc[ti][KB][q];
#pragma unroll
    for (int tj = KB + 1; tj < 5; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) S.stg[2 + tj - KB - 1][(4 * lg + q) * TS + lc] = acc[KB][tj][q];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int ti = KB + 1; ti < 3; ++ti)
#pragma unroll
      for (int tj = KB + 1; tj < 5; ++tj)
        acc[ti][tj] = tile_msub<SPLIT>(S.stg[ti - KB - 1], S.stg[2 + tj - KB - 1], acc[ti][tj], lc, lg);
  }
  __syncthreads();
}

// Back substitution of block row KB for the right-hand-side tiles 3 and 4 (row by row, the solved
// row and the U column shuffled across the lanes), then their update in the block rows above (MFMA)
template <int KB, bool SPLIT>
__device__ __forceinline__ void mf_back_block(f32x4 (&acc)[3][5], MfmaLds &S, bool active, int lc, int lg) {
  if (active)
#pragma unroll
    for (int ii = 15; ii >= 0; --ii) {
      const int qi = ii & 3, src_row = 16 * (ii >> 2) + lc, src_col = 16 * lg + ii;
      const float d = 1.f / __shfl(f4_get(acc[KB][KB], qi), 16 * (ii >> 2) + ii);
      const float x3 = __shfl(f4_get(acc[KB][3], qi), src_row) * d;
      const float x4 = __shfl(f4_get(acc[KB][4], qi), src_row) * d;
      if (lg == (ii >> 2)) {
        f4_set(acc[KB][3], qi, x3);
        f4_set(acc[KB][4], qi, x4);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float u = __shfl(acc[KB][KB][q], src_col);
        if (4 * lg + q < ii) {
          acc[KB][3][q] -= u * x3;
          acc[KB][4][q] -= u * x4;
        }
      }
    }
  if constexpr (KB > 0) {
    if (active) {
#pragma unroll
      for (int ti = 0; ti < KB; ++ti)
#pragma unroll
        for (int q = 0; q < 4; ++q) S.stg[1 + ti][(4 * lg + q) * TS + lc] = acc[ti][KB][q];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        S.stg[3][(4 * lg + q) * TS + lc] = acc[KB][3][q];
        S.stg[4][(4 * lg + q) * TS + lc] = acc[KB][4][q];
      }
    }
    __syncthreads();
    if (active)
#pragma unroll
      for (int ti = 0; ti < KB; ++ti) {
        acc[ti][3] = tile_msub<SPLIT>(S.stg[1 + ti], S.stg[3], acc[ti][3], lc, lg);
        acc[ti][4] = tile_msub<SPLIT>(S.stg[1 + ti], S.stg[4], acc[ti][4], lc, lg);
      }
    __syncthreads();
  }
}

template <bool SPLIT>
__global__ void __launch_bounds__(64 * kMW) k_p1_condense_mfma(int ncell, const double *__restrict__ A,
                                                              const double *__restrict__ cdiag,
                                                              const double *__restrict__ kdiag,
                                                              float *__restrict__ SK) {
  __shared__ MfmaLds sL[kMW];
  __shared__ double sC[kMW][NF];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lc = lane & 15, lg = lane >> 4;
  const int c = xcd_block() * kMW + wv;
  const bool active = c < ncell;  // uniform within a wavefront
  MfmaLds &S = sL[wv];
  // the cell's compact A_K staged in FP32 through the tile area (coalesced loads), then spread over
  // the accumulator tiles from there
  static_assert(NAC <= 6 * 16 * TS, "the compact A_K fits the staging area");
  float *Ast = &S.stg[0][0];
  if (active) {
    const double *Ac = A + (size_t)c * NAC;
    for (int e = lane; e < NAC; e += 64) Ast[e] = (float)Ac[e];
    if (lane < NF) sC[wv][lane] = cdiag[(size_t)c * NF + lane];
  }
  __syncthreads();
  f32x4 acc[3][5];
  if (active) {
#pragma unroll
    for (int ti = 0; ti < 3; ++ti)
#pragma unroll
      for (int tj = 0; tj < 5; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * ti + 4 * lg + q, j = 16 * tj + lc;
          float v;
          if (r < NX && j < NX) {
            const int e = a_compact(r, j);
            v = e < 0 ? 0.f : Ast[e];
          } else if (j < MP) {
            v = (r == j) ? 1.f : 0.f;
          } else {
            v = (j - MP == r && r < NF) ? (float)kdiag[(size_t)c * NF + r] : 0.f;
          }
          acc[ti][tj][q] = v;
        }
  } else {
#pragma unroll
    for (int ti = 0; ti < 3; ++ti)
#pragma unroll
      for (int tj = 0; tj < 5; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  __syncthreads();  // the staging area is the elimination's from here on
  if (active) mf_elim_block<0>(acc, lc, lg);
  mf_trailing<0, SPLIT>(acc, S, active, lc, lg);
  if (active) mf_elim_block<1>(acc, lc, lg);
  mf_trailing<1, SPLIT>(acc, S, active, lc, lg);
  if (active) mf_elim_block<2>(acc, lc, lg);
  mf_back_block<2, SPLIT>(acc, S, active, lc, lg);
  mf_back_block<1, SPLIT>(acc, S, active, lc, lg);
  mf_back_block<0, SPLIT>(acc, S, active, lc, lg);
  // X = the rows 0..23 of the solution in the right-hand-side columns 0..23 -> LDS, then S_K = C X
  float *X = &S.stg[0][0];
  if (active)
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + 4 * lg + q;
        if (r < NF) {
          X[r * NF + lc] = acc[ti][3][q];
          if (lc < NF - 16) X[r * NF + 16 + lc] = acc[ti][4][q];
        }
      }
  __syncthreads();
  // thread t writes cell t mod kMW of the workgroup: each store covers kMW consecutive cells
  const int w = threadIdx.x % kMW, cw = c - wv + w;
  if (cw < ncell) {
    const float *Xw = &sL[w].stg[0][0];
    for (int e = threadIdx.x / kMW; e < NS; e += 64) {
      const int r = e / NF;
      SK[(size_t)e * ncell + cw] = (float)(sC[w][r] * (double)Xw[e]);
    }
  }
}

// Global trace dof of local face dof j of cell (k, col).
__device__ __forceinline__ size_t p1_dof(int j, int k, int col, int ncol, int nedge, size_t nz,
                                         const int32_t *__restrict__ col_edge) {
  const int f = j >> 2;
  size_t F;
  if (f < 4)
    F = nz + (size_t)k * nedge + col_edge[(size_t)f * ncol + col];
  else
    F = (size_t)(k + (f - 4)) * ncol + col;
  return 4 * F + (j & 3);
}

// For trace row T = 4 F + i: the (up to two) cells of facet F and the facet's local face in each.
__device__ __forceinline__ int p1_row_cells(size_t T, int nlev, int ncol, int nedge, size_t nz,
                                            const int32_t *__restrict__ edge_col, const int32_t *__restrict__ edge_lf,
                                            int cells[2], int faces[2]) {
  const size_t F = T >> 2;
  int n = 0;
  if (F < nz) {
    const int k = (int)(F / ncol), col = (int)(F - (size_t)k * ncol);
    if (k > 0) cells[n] = (k - 1) * ncol + col, faces[n++] = 5;
    if (k < nlev) cells[n] = k * ncol + col, faces[n++] = 4;
  } else {
    const size_t h = F - nz;
    const int k = (int)(h / nedge), e = (int)(h - (size_t)k * nedge);
    cells[0] = k * ncol + edge_col[e], faces[0] = edge_lf[e];
    cells[1] = k * ncol + edge_col[nedge + e], faces[1] = edge_lf[nedge + e];
    n = 2;
  }
  return n;
}

// ---- condensation by the block structure of A_K --------------------------------------------------
// On an axis-aligned cell the velocity block M = m2 - q22 is block diagonal: every RT1 function is a
// Lagrange function on the Gauss points in its two tangential directions, and those are orthogonal,
// so a function couples only to the two others of its direction and tangential point -- twelve 3x3
// blocks {4 (2d) + i, 4 (2d + 1) + i, 24 + 4 d + i} (d direction, i tangential point).  With
// Mi = M^-1 and the pressure Schur complement Sg = P - Dr Mi G (8x8),
//   [A^-1]_uu = Mi + (Mi G) Sg^-1 (Dr Mi),   S_K = C_F ([Mi]_FF + [Mi G]_F Sg^-1 [Dr Mi]_F) K_F,
// and the cell solves X = A^-1 R are y = Mi R_u, x_p = Sg^-1 (R_p - Dr y), x_u = y - (Mi G) x_p.
// Factors kept per cell (entry by entry over the cells): Mi (12 x 9), Mi G (36 x 8), Dr (8 x 36),
// Sg^-1 (8 x 8).
constexpr int FO_MI = 0, FO_MIG = 108, FO_DR = FO_MIG + 288, FO_SGI = FO_DR + 288, NFAC = FO_SGI + 64;


// One wavefront per cell, SW cells per workgroup.  LDS per cell: Mi, Dr, Mi G, Sg, the diagonals of
// C_K and K_K, and T (first the trace-face columns of Dr Mi, then Sg^-1 times them in place): 988
// doubles, each array padded per cell (1008 in all) so that the write-out, where consecutive lanes
// read the same entry of different cells, finds the cells' copies in different LDS banks (unpadded,
// the strides of 288, 192 and 64 doubles put all eight cells on one bank).  G is read from A_K
// where Mi G is formed rather than staged.
constexpr int LP_DR = 292, LP_MIG = 292, LP_SG = 68, LP_T = 196, LP_CK = 2 * NF + 4;
template <int SW>
__global__ void __launch_bounds__(64 * SW) k_p1_condense_struct(int ncell, const double *__restrict__ A,
                                                               const double *__restrict__ cdiag,
                                                               const double *__restrict__ kdiag,
                                                               double *__restrict__ SK, double *__restrict__ fac,
                                                               int write_sk) {
  __shared__ double sMi[SW][108], sDr[SW][LP_DR], sMiG[SW][LP_MIG], sSg[SW][LP_SG], sT[SW][LP_T], sCK[SW][LP_CK];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = xcd_block() * SW + wv;
  const bool active = c < ncell;
  double *Mi = sMi[wv], *Dr = sDr[wv], *MiG = sMiG[wv], *Sg = sSg[wv], *T = sT[wv];
  auto Ae = [&](int e) { return A[(size_t)c * NAC + e]; };  // compact A_K
  if (active) {
#pragma unroll
    for (int e = lane; e < 288; e += 64) {
      const int a = e >> 3, p = e & 7;
      Dr[p * NU + a] = Ae(AO_DR + NU * p + a);  // Dr[p][a]
    }
    if (lane < NF) sCK[wv][lane] = cdiag[(size_t)c * NF + lane];
    else if (lane < 2 * NF) sCK[wv][lane] = kdiag[(size_t)c * NF + lane - NF];
    Sg[lane] = Ae(AO_P + lane);  // P
    if (lane < 12) {  // invert the 3x3 block by cofactors
      double m[3][3];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) m[r][q] = Ae(AO_M + 9 * lane + 3 * r + q);
      const double c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1], c01 = m[1][2] * m[2][0] - m[1][0] * m[2][2],
                   c02 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
      const double inv = 1.0 / (m[0][0] * c00 + m[0][1] * c01 + m[0][2] * c02);
      double *o = Mi + 9 * lane;
      o[0] = c00 * inv, o[3] = c01 * inv, o[6] = c02 * inv;
      o[1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * inv, o[4] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * inv,
      o[7] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * inv;
      o[2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * inv, o[5] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * inv,
      o[8] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * inv;
    }
  }
  __syncthreads();
  if (active) {
    for (int e = lane; e < 288; e += 64) {  // (Mi G)[a][p], G[a][p] = A_K[a][NU + p]
      int blk, r;
      const int a = e >> 3, p = e & 7;
      dof_blk(a, blk, r);
      double s1 = 0.0;
      for (int q = 0; q < 3; ++q) s1 += Mi[9 * blk + 3 * r + q] * Ae(AO_G + NPR * blk_dof(blk, q) + p);
      MiG[e] = s1;
    }
    for (int e = lane; e < 192; e += 64) {  // (Dr Mi)[p][f] for the trace-face dofs f < NF
      int blk, r;
      const int p = e / NF, f = e - p * NF;
      dof_blk(f, blk, r);
      double s2 = 0.0;
      for (int q = 0; q < 3; ++q) s2 += Dr[p * NU + blk_dof(blk, q)] * Mi[9 * blk + 3 * q + r];
      T[e] = s2;
    }
  }
  __syncthreads();
  if (active) {  // Sg = P - Dr (Mi G)
    const int p = lane >> 3, q = lane & 7;
    double s = 0.0;
    for (int a = 0; a < NU; ++a) s += Dr[p * NU + a] * MiG[a * 8 + q];
    Sg[lane] -= s;
  }
  __syncthreads();
  if (active) {
    // Sg^-1 in place by Gauss-Jordan without pivoting (Sg is dominated by its positive diagonal):
    // lane 8 i + j holds entry (i, j); each step reads the pivot row and column across lanes
    const int i = lane >> 3, j = lane & 7;
    double a = Sg[lane];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double akk = __shfl(a, 9 * k), aik = __shfl(a, 8 * i + k), akj = __shfl(a, 8 * k + j);
      const double p = 1.0 / akk;
      if (i == k && j == k) a = p;
      else if (i == k) a = akj * p;
      else if (j == k) a = -aik * p;
      else a -= aik * akj * p;
    }
    Sg[lane] = a;
  }
  __syncthreads();
  double tv[3] = {0.0, 0.0, 0.0};  // T = Sg^-1 [Dr Mi]_F, formed in registers, then written over its input
  if (active)
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = lane + 64 * u, p = e / NF, f = e - p * NF;
      double s = 0.0;
      for (int q = 0; q < 8; ++q) s += Sg[8 * p + q] * T[q * NF + f];
      tv[u] = s;
    }
  __syncthreads();
  if (active)
#pragma unroll
    for (int u = 0; u < 3; ++u) T[lane + 64 * u] = tv[u];
  __syncthreads();
  // Writes: thread t takes cell w = t mod SW of the workgroup, so each store covers SW consecutive
  // cells of 64 / SW entries (8 SW-byte pieces) instead of 64 scattered doubles.
  const int w = threadIdx.x % SW, c0 = c - wv;
  if (c0 + w >= ncell) return;
  const double *wMi = sMi[w], *wMiG = sMiG[w], *wT = sT[w], *wDr = sDr[w], *wSg = sSg[w];
  const size_t cw = (size_t)c0 + w;
  // S_K: the 64 threads of a cell take rows r = j / 8 + 8 i and columns f = j mod 8 + 8 u (i, u < 3),
  // so the eight T entries of a column and the eight Mi G entries of a row are read once per three
  // products (about 5 LDS reads per entry instead of 16).
  static_assert(NF == 24, "three row and three column groups of eight");
  if (write_sk) {
    const int j = threadIdx.x / SW, rg = j >> 3, f0 = j & 7;
    double tc[3][8];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int p = 0; p < 8; ++p) tc[u][p] = wT[p * NF + f0 + 8 * u];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int r = rg + 8 * i;
      double mr[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) mr[p] = wMiG[r * 8 + p];
      int br, pr;
      dof_blk(r, br, pr);
      const double ckr = sCK[w][r];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int f = f0 + 8 * u;
        int bf, pf;
        dof_blk(f, bf, pf);
        double v = (br == bf) ? wMi[9 * br + 3 * pr + pf] : 0.0;
#pragma unroll
        for (int p = 0; p < 8; ++p) v += mr[p] * tc[u][p];
        SK[(size_t)(r * NF + f) * ncell + cw] = ckr * v * sCK[w][NF + f];
      }
    }
  }
  for (int e = threadIdx.x / SW; e < NFAC; e += 64) {
    double v;
    if (e < FO_MIG) v = wMi[e];
    else if (e < FO_DR) v = wMiG[e - FO_MIG];
    else if (e < FO_SGI) v = wDr[e - FO_DR];
    else v = wSg[e - FO_SGI];
    fac[(size_t)e * ncell + cw] = v;
  }
}

// cells (wavefronts) per workgroup of the structured condensation (128^2x32, FP64 call: 4 cells
// 5.6 ms, 8 cells 5.0 ms, 16 cells 9.2 ms with the unpadded LDS arrays; with them padded, 8 cells
// 3.51 ms with S_K and 2.27 ms for the factors alone, 16 cells, one workgroup per CU, 3.46 and 2.54)
constexpr int kSW = 8;

// Thread per cell: X = A_K^-1 (R - [K lambda; 0]) from the structured factors.  mode 0: the cell's
// share C_F [X_u]_F of B_lambda into bK [24][ncell]; mode 1: recovery into u [36][ncell], pi [8][ncell].
__global__ void __launch_bounds__(kBlock) k_p1_cell_struct(int ncell, int ncol, int nedge, size_t nz,
                                                          const int32_t *__restrict__ col_edge,
                                                          const double *__restrict__ fac,
                                                          const double *__restrict__ cdiag,
                                                          const double *__restrict__ kdiag,
                                                          const double *__restrict__ r_u,
                                                          const double *__restrict__ r_p,
                                                          const double *__restrict__ lam, int mode,
                                                          double *__restrict__ bK, double *__restrict__ u,
                                                          double *__restrict__ pi) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int k = c / ncol, col = c - k * ncol;
  auto F = [&](int e) { return fac[(size_t)e * ncell + c]; };
  double R[NU], y[NU], g[NPR], xp[NPR];
#pragma unroll
  for (int a = 0; a < NU; ++a) R[a] = r_u[(size_t)a * ncell + c];
  if (mode == 1)
#pragma unroll
    for (int f = 0; f < NF; ++f) R[f] -= kdiag[(size_t)c * NF + f] * lam[p1_dof(f, k, col, ncol, nedge, nz, col_edge)];
#pragma unroll
  for (int blk = 0; blk < 12; ++blk) {
    const int d0 = blk_dof(blk, 0), d1 = blk_dof(blk, 1), d2 = blk_dof(blk, 2);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      y[blk_dof(blk, r)] = F(FO_MI + 9 * blk + 3 * r) * R[d0] + F(FO_MI + 9 * blk + 3 * r + 1) * R[d1] +
                           F(FO_MI + 9 * blk + 3 * r + 2) * R[d2];
  }
#pragma unroll
  for (int p = 0; p < NPR; ++p) {
    double s = r_p[(size_t)p * ncell + c];
#pragma unroll
    for (int a = 0; a < NU; ++a) s -= F(FO_DR + p * NU + a) * y[a];
    g[p] = s;
  }
#pragma unroll
  for (int p = 0; p < NPR; ++p) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NPR; ++q) s += F(FO_SGI + 8 * p + q) * g[q];
    xp[p] = s;
  }
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    double s = y[a];
#pragma unroll
    for (int p = 0; p < NPR; ++p) s -= F(FO_MIG + 8 * a + p) * xp[p];
    y[a] = s;
  }
  if (mode == 0) {
#pragma unroll
    for (int f = 0; f < NF; ++f) bK[(size_t)f * ncell + c] = cdiag[(size_t)c * NF + f] * y[f];
  } else {
#pragma unroll
    for (int a = 0; a < NU; ++a) u[(size_t)a * ncell + c] = y[a];
#pragma unroll
    for (int p = 0; p < NPR; ++p) pi[(size_t)p * ncell + c] = xp[p];
  }
}

// S x in two passes.  Thread per cell: t_K = S_K x_K into t [24][ncell] (mode 0), or the diagonal of
// S_K (mode 1).  Each cell gathers its 24 trace values once and reads its S_K entry by entry over
// the cells, so both the matrix and t stream coalesced.
template <typename TS>
__global__ void __launch_bounds__(kBlock) k_p1_cell_mv(int ncell, int ncol, int nedge, size_t nz,
                                                      const int32_t *__restrict__ col_edge,
                                                      const TS *__restrict__ SK, const double *__restrict__ x,
                                                      int mode, double *__restrict__ t) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  if (mode == 1) {
#pragma unroll 4
    for (int r = 0; r < NF; ++r) t[(size_t)r * ncell + c] = SK[(size_t)(r * NF + r) * ncell + c];
    return;
  }
  const int k = c / ncol, col = c - k * ncol;
  double xk[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) xk[j] = x[p1_dof(j, k, col, ncol, nedge, nz, col_edge)];
#pragma unroll 2
  for (int r = 0; r < NF; ++r) {
    const TS *row = SK + (size_t)r * NF * ncell + c;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j) s += (double)__builtin_nontemporal_load(&row[(size_t)j * ncell]) * xk[j];
    t[(size_t)r * ncell + c] = s;
  }
}

// The same with FP32 entries and two cells of a layer per thread (ncol even): the entries of the
// adjacent cells 2i and 2i + 1 sit side by side in the [entry][cell] layout, so one 8-byte load
// takes both and a wavefront reads 512 contiguous bytes per entry instead of 256 (0.24 ms against
// 0.33 ms at 128^2x32; with FP64 entries the same pairing was slower, 0.53 ms against 0.48).  Per
// cell the arithmetic and its order are those of k_p1_cell_mv<float>.
typedef float p1_f2 __attribute__((ext_vector_type(2)));
__global__ void __launch_bounds__(kBlock) k_p1_cell_mv_pair(int ncell, int ncol, int nedge, size_t nz,
                                                           const int32_t *__restrict__ col_edge,
                                                           const float *__restrict__ SK,
                                                           const double *__restrict__ x, int mode,
                                                           double *__restrict__ t) {
  using V2 = p1_f2;
  const int c = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= ncell) return;
  auto ld2 = [&](size_t e) { return __builtin_nontemporal_load(reinterpret_cast<const V2 *>(SK + e * ncell + c)); };
  if (mode == 1) {
#pragma unroll 4
    for (int r = 0; r < NF; ++r) {
      const V2 v = ld2((size_t)r * NF + r);
      t[(size_t)r * ncell + c] = v[0];
      t[(size_t)r * ncell + c + 1] = v[1];
    }
    return;
  }
  const int k = c / ncol, col = c - k * ncol;
  double xa[NF], xb[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    xa[j] = x[p1_dof(j, k, col, ncol, nedge, nz, col_edge)];
    xb[j] = x[p1_dof(j, k, col + 1, ncol, nedge, nz, col_edge)];
  }
#pragma unroll 2
  for (int r = 0; r < NF; ++r) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const V2 v = ld2((size_t)r * NF + j);
      sa += (double)v[0] * xa[j];
      sb += (double)v[1] * xb[j];
    }
    t[(size_t)r * ncell + c] = sa;
    t[(size_t)r * ncell + c + 1] = sb;
  }
}

// Thread per trace row T = 4 F + i: the sum of the shares t_K of the (up to two) cells of facet F,
// y = sum (sub = 0) or y = b - sum (sub = 1).  t is [24][ncell] (the cells' shares of S x, of
// diag(S), or of B_lambda).
__global__ void k_p1_gather(size_t ntr, int nlev, int ncol, int nedge, size_t nz, const int32_t *__restrict__ edge_col,
                            const int32_t *__restrict__ edge_lf, const double *__restrict__ t,
                            const double *__restrict__ b, double *__restrict__ y, int sub) {
  const size_t T = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= ntr) return;
  int cells[2], faces[2];
  const int n = p1_row_cells(T, nlev, ncol, nedge, nz, edge_col, edge_lf, cells, faces);
  const size_t ncell = (size_t)nlev * ncol;
  const int i = (int)(T & 3);
  double s = 0.0;
  for (int q = 0; q < n; ++q) s += t[(size_t)(4 * faces[q] + i) * ncell + cells[q]];
  y[T] = sub ? b[T] - s : s;
}

// ---- two-level preconditioner at order 1 ------------------------------------------------------
// Per column, the horizontal-facet dofs (4 per facet, facets k = 0..L) form a block-tridiagonal
// system with 4x4 blocks: facet k couples to itself through the cells below (its T face) and above
// (its B face), and to facets k -/+ 1 through those cells.  Block LU (Thomas) factors per facet:
// Dinv_k = (D_k - W_k U_{k-1})^-1, W_k = Lo_k Dinv_{k-1}, and U_k; 48 doubles per facet.
__device__ __forceinline__ void inv4(const double *a, double *o) {
  // 4x4 inverse by Gauss-Jordan without pivoting (diagonal blocks of an S^zz that is dominant)
  double m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = a[4 * i + j], m[i][4 + j] = (i == j) ? 1.0 : 0.0;
  for (int k = 0; k < 4; ++k) {
    const double p = 1.0 / m[k][k];
    for (int j = 0; j < 8; ++j) m[k][j] *= p;
    for (int i = 0; i < 4; ++i)
      if (i != k) {
        const double f = m[i][k];
        for (int j = 0; j < 8; ++j) m[i][j] -= f * m[k][j];
      }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) o[4 * i + j] = m[i][4 + j];
}

// block of S_K between local faces fa (rows) and fb (columns)
template <typename TS>
__device__ __forceinline__ void sk_block(const TS *SK, size_t ncell, int c, int fa, int fb, double *o) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) o[4 * i + j] = SK[(size_t)((4 * fa + i) * NF + 4 * fb + j) * ncell + c];
}

template <typename TS>
__global__ void k_p1_zfactor(int nlev, int ncol, const TS *__restrict__ SK, double *__restrict__ zf) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  const size_t ncell = (size_t)nlev * ncol;
  double Dinv[16], Up[16];
  for (int k = 0; k <= nlev; ++k) {
    double D[16] = {0}, t[16];
    if (k > 0) {
      sk_block(SK, ncell, (k - 1) * ncol + col, 5, 5, t);
      for (int q = 0; q < 16; ++q) D[q] += t[q];
    }
    if (k < nlev) {
      sk_block(SK, ncell, k * ncol + col, 4, 4, t);
      for (int q = 0; q < 16; ++q) D[q] += t[q];
    }
    double W[16] = {0};
    if (k > 0) {
      double Lo[16];
      sk_block(SK, ncell, (k - 1) * ncol + col, 5, 4, Lo);  // facet k's rows, facet k-1's columns
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          double a = 0.0;
          for (int m = 0; m < 4; ++m) a += Lo[4 * i + m] * Dinv[4 * m + j];
          W[4 * i + j] = a;
        }
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          double a = 0.0;
          for (int m = 0; m < 4; ++m) a += W[4 * i + m] * Up[4 * m + j];
          D[4 * i + j] -= a;
        }
    }
    inv4(D, Dinv);
    if (k < nlev)
      sk_block(SK, ncell, k * ncol + col, 4, 5, Up);  // facet k's rows, facet k+1's columns
    else
      for (int q = 0; q < 16; ++q) Up[q] = 0.0;
    double *o = zf + ((size_t)k * ncol + col) * 48;
    for (int q = 0; q < 16; ++q) o[q] = Dinv[q], o[16 + q] = W[q], o[32 + q] = Up[q];
  }
}

// LineSmooth (Alg. 1) at order 1, given the residual R: horizontal facets by the block-tridiagonal
// column solve, vertical facets by point Jacobi; lambda_out = lambda_in + omega delta.
// Four lanes per column, lane i holding dof row i of every facet's 4-vector; the 4x4 products take
// the other rows of the vector from the group's lanes by shuffles, so the loads of a level do not
// wait on the recurrence and a column's rows are read as one 128-byte piece.
__global__ void __launch_bounds__(kBlock) k_p1_zsolve(int nlev, int ncol, const double *__restrict__ zf,
                                                     const double *__restrict__ R, const double *__restrict__ lin,
                                                     double *__restrict__ lout, double omega) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = t >> 2, i = t & 3, lane = threadIdx.x & 63, g0 = lane & ~3;
  const bool on = col < ncol;  // uniform over a group of four; every lane takes part in the shuffles
  const int cl = on ? col : ncol - 1;  // lanes past the last column read (and discard) the last one's
  double prev = 0.0;
#pragma unroll 4
  for (int k = 0; k <= nlev; ++k) {  // forward: y_k = R_k - W_k y_{k-1}, kept in lout
    const size_t F = (size_t)k * ncol + cl;
    double w[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) w[m] = zf[F * 48 + 16 + 4 * i + m];
    double y = R[4 * F + i];
#pragma unroll
    for (int m = 0; m < 4; ++m) y -= w[m] * __shfl(prev, g0 + m, 64);
    if (on) lout[4 * F + i] = y;
    prev = y;
  }
  double next = 0.0;
#pragma unroll 4
  for (int k = nlev; k >= 0; --k) {  // backward: x_k = Dinv_k (y_k - U_k x_{k+1})
    const size_t F = (size_t)k * ncol + cl;
    double dv[4], up[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) dv[m] = zf[F * 48 + 4 * i + m], up[m] = zf[F * 48 + 32 + 4 * i + m];
    double tt = lout[4 * F + i];
#pragma unroll
    for (int m = 0; m < 4; ++m) tt -= up[m] * __shfl(next, g0 + m, 64);
    double x = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) x += dv[m] * __shfl(tt, g0 + m, 64);
    next = x;
    if (on) lout[4 * F + i] = (lin ? lin[4 * F + i] : 0.0) + omega * x;
  }
}

__global__ void k_p1_hjacobi(size_t nz4, size_t ntr, const double *__restrict__ dS, const double *__restrict__ R,
                             const double *__restrict__ lin, double *__restrict__ lout, double omega) {
  const size_t T = nz4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= ntr) return;
  lout[T] = (lin ? lin[T] : 0.0) + omega * R[T] / dS[T];
}

// Restriction to the DG0 coarse space with scaling: out_c = g_c (P^T r)_c; P sets every dof of a
// facet to the average of its two cells (to the one cell at ground and lid), so P^T weights the 24
// dofs of a cell by 1/2, by 1 on ground and lid facets.  g = NULL: no scaling.
__global__ void k_p1_restrict(int nlev, int ncol, int nedge, size_t nz, const int32_t *__restrict__ col_edge,
                              const double *__restrict__ r, const double *__restrict__ g, double *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nlev * ncol) return;
  const int k = c / ncol, col = c - k * ncol;
  double s = 0.0;
  for (int j = 0; j < NF; ++j) {
    const int f = j >> 2;
    const double w = (f == 4 && k == 0) || (f == 5 && k == nlev - 1) ? 1.0 : 0.5;
    s += w * r[p1_dof(j, k, col, ncol, nedge, nz, col_edge)];
  }
  out[c] = g ? g[c] * s : s;
}

// lambda_T += (P x)_T
__global__ void k_p1_prolong(size_t ntr, int nlev, int ncol, int nedge, size_t nz, const int32_t *__restrict__ edge_col,
                             const int32_t *__restrict__ edge_lf, const double *__restrict__ x, double *__restrict__ lam) {
  const size_t T = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= ntr) return;
  int cells[2], faces[2];
  const int n = p1_row_cells(T, nlev, ncol, nedge, nz, edge_col, edge_lf, cells, faces);
  const double v = n == 1 ? x[cells[0]] : 0.5 * (x[cells[0]] + x[cells[1]]);
  lam[T] += v;
}

// Gamma_c = (H 1)_c / (P^T S P 1)_c with the coarse operator H (7-entry stencil rows)
__global__ void k_p1_gamma(int ncell, const double *__restrict__ H, const double *__restrict__ den,
                           double *__restrict__ g) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  double h1 = 0.0;
  for (int s = 0; s < 7; ++s) h1 += H[(size_t)s * ncell + c];
  g[c] = h1 / den[c];
}

__global__ void k_p1_fill(double *x, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace

// ---- host ---------------------------------------------------------------------------------------

hipError_t p1_setup(hyb_ctx *c) {
  P1State &s = c->p1;
  if (s.tbl) return hipSuccess;
  std::vector<double> T = build_tables();
  hipError_t e = hipMalloc((void **)&s.tbl, T.size() * 8);
  if (e) return e;
  c->bytes += T.size() * 8;
  return hipMemcpy(s.tbl, T.data(), T.size() * 8, hipMemcpyHostToDevice);
}

hipError_t p1_assemble(hyb_ctx *c, const double *theta_w, const double *exner_hat_w, const double *exner_c,
                       const double *rho_c) {
  P1State &s = c->p1;
  const hyb_params &p = c->p;
  const double kappa = p.rd / p.cp;
  hipLaunchKernelGGL(k_p1_assemble, dim3(nblk(c->ncell, kBlock / 64)), dim3(kBlock), 0, c->stream, c->ncell, c->ncol,
                     c->dz_d, c->dx, c->dy, theta_w, exner_hat_w, exner_c, rho_c, s.tbl, p.dt, p.tau_u, p.tau_rho,
                     p.tau_theta, p.cp, kappa, s.A, s.cdiag, s.kdiag);
  return hipGetLastError();
}

// S_K in the arithmetic of params.precision: FP64 from the block structure, or the dense elimination
// of A_K on MFMA (FP32, BF16 split); the per-solve cell factors always in FP64 from the structure.
// S_K is held in FP32 when the matrix cores condensed it (FP32-accurate there), else in FP64; the
// mixed form keeps an FP32 copy of the FP64 S_K for the preconditioner
bool p1_sk_fp32(const hyb_ctx *c) {
  return c->p.precision == HYB_PREC_MFMA_FP32 || c->p.precision == HYB_PREC_MFMA_BF16X;
}

hipError_t p1_factor(hyb_ctx *c) {
  P1State &s = c->p1;
  const int prec = c->p.precision;
  if (prec == HYB_PREC_MFMA_FP32 || prec == HYB_PREC_MFMA_BF16X) {
    const int slot = prof_begin(c, F_P1_CONDENSE);
    if (prec == HYB_PREC_MFMA_FP32)
      hipLaunchKernelGGL((k_p1_condense_mfma<false>), dim3(nblk(c->ncell, kMW)), dim3(64 * kMW), 0, c->stream,
                         c->ncell, s.A, s.cdiag, s.kdiag, s.SKf);
    else
      hipLaunchKernelGGL((k_p1_condense_mfma<true>), dim3(nblk(c->ncell, kMW)), dim3(64 * kMW), 0, c->stream,
                         c->ncell, s.A, s.cdiag, s.kdiag, s.SKf);
    prof_end(c, F_P1_CONDENSE, slot);
    hipError_t e = hipGetLastError();
    if (e) return e;
  }
  const int slot = prof_begin(c, F_P1_FACTOR);
  hipLaunchKernelGGL((k_p1_condense_struct<kSW>), dim3(nblk(c->ncell, kSW)), dim3(64 * kSW), 0, c->stream, c->ncell, s.A,
                     s.cdiag, s.kdiag, s.SK, s.fac, p1_sk_fp32(c) ? 0 : 1);
  prof_end(c, F_P1_FACTOR, slot);
  hipError_t e = hipGetLastError();
  if (e || prec != HYB_PREC_MIXED) return e;
  return launch_to_float(c, s.SK, s.SKf, (size_t)NS * c->ncell);
}

hipError_t p1_cell_solve(hyb_ctx *c, const double *r_u, const double *r_p, const double *lam, int mode, double *u,
                         double *pi) {
  P1State &s = c->p1;
  const LevelDev &L0 = c->lv[0];
  const int slot = prof_begin(c, F_CELL);
  hipLaunchKernelGGL(k_p1_cell_struct, dim3(nblk(c->ncell)), dim3(kBlock), 0, c->stream, c->ncell, c->ncol, c->nedge,
                     (size_t)c->nz, L0.col_edge, s.fac, s.cdiag, s.kdiag, r_u, r_p, lam, mode, s.bK, u, pi);
  prof_end(c, F_CELL, slot);
  return hipGetLastError();
}

hipError_t p1_rows(hyb_ctx *c, const double *x, double *y, int mode, const double *b, bool precond) {
  P1State &s = c->p1;
  const LevelDev &L0 = c->lv[0];
  const size_t ntr = (size_t)c->ntrace;
  int slot = prof_begin(c, F_TRACE_APPLY);
  if (mode != 1) {  // mode 1 gathers the shares already in bK
    const bool f32 = p1_sk_fp32(c) || (precond && c->p.precision == HYB_PREC_MIXED);
    const dim3 g2(nblk((size_t)c->ncell / 2)), g1(nblk(c->ncell));
    if (f32 && c->ncol % 2 == 0)
      hipLaunchKernelGGL(k_p1_cell_mv_pair, g2, dim3(kBlock), 0, c->stream, c->ncell, c->ncol, c->nedge,
                         (size_t)c->nz, L0.col_edge, (const float *)s.SKf, x, mode == 3 ? 1 : 0, s.bK);
    else if (f32)
      hipLaunchKernelGGL(k_p1_cell_mv<float>, g1, dim3(kBlock), 0, c->stream, c->ncell, c->ncol, c->nedge,
                         (size_t)c->nz, L0.col_edge, (const float *)s.SKf, x, mode == 3 ? 1 : 0, s.bK);
    else
      hipLaunchKernelGGL(k_p1_cell_mv<double>, g1, dim3(kBlock), 0, c->stream, c->ncell, c->ncol, c->nedge,
                         (size_t)c->nz, L0.col_edge, (const double *)s.SK, x, mode == 3 ? 1 : 0, s.bK);
  }
  hipLaunchKernelGGL(k_p1_gather, dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, ntr, c->nlev, c->ncol, c->nedge,
                     (size_t)c->nz, L0.edge_col, L0.edge_lf, s.bK, b, y, mode == 2 ? 1 : 0);
  prof_end(c, F_TRACE_APPLY, slot);
  return hipGetLastError();
}

// Setup of the two-level preconditioner at order 1 (after the condensation): diag(S), the block
// factors of the column systems, and Gamma with the coarse context's H.
hipError_t p1_precond_setup(hyb_ctx *c) {
  P1State &s = c->p1;
  hyb_ctx *cc = c->coarse;
  const LevelDev &L0 = c->lv[0];
  const size_t ntr = (size_t)c->ntrace, nc = (size_t)c->ncell;
  hipError_t e;
  if ((e = p1_rows(c, nullptr, s.dS, 3, nullptr))) return e;
  if (p1_sk_fp32(c))
    hipLaunchKernelGGL(k_p1_zfactor<float>, dim3(nblk(c->ncol)), dim3(kBlock), 0, c->stream, c->nlev, c->ncol,
                       (const float *)s.SKf, s.zf);
  else
    hipLaunchKernelGGL(k_p1_zfactor<double>, dim3(nblk(c->ncol)), dim3(kBlock), 0, c->stream, c->nlev, c->ncol,
                       (const double *)s.SK, s.zf);
  if ((e = hipGetLastError())) return e;
  // P 1 = 1 on every dof; den = P^T S 1
  hipLaunchKernelGGL(k_p1_fill, dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, s.t1, ntr, 1.0);
  if ((e = p1_rows(c, s.t1, s.t2, 0, nullptr))) return e;
  hipLaunchKernelGGL(k_p1_restrict, dim3(nblk(nc)), dim3(kBlock), 0, c->stream, c->nlev, c->ncol, c->nedge,
                     (size_t)c->nz, L0.col_edge, s.t2, (const double *)nullptr, s.den);
  hipLaunchKernelGGL(k_p1_gamma, dim3(nblk(nc)), dim3(kBlock), 0, c->stream, c->ncell, cc->lv[0].H, s.den, s.gamma);
  return hipGetLastError();
}

// z = M(r): Alg. 2 at order 1 (LineSmooth n_pre sweeps from zero, residual, restriction to DG0 with
// Gamma, one V-cycle of the coarse context's pressure multigrid, prolongation, n_post sweeps).
hipError_t p1_precondition(hyb_ctx *c, const double *r, double *z) {
  P1State &s = c->p1;
  hyb_ctx *cc = c->coarse;
  const hyb_params &p = c->p;
  const LevelDev &L0 = c->lv[0];
  const size_t ntr = (size_t)c->ntrace, nc = (size_t)c->ncell, nz4 = 4 * (size_t)c->nz;
  double *lam = s.t1, *tmp = s.t2, *R = s.t3;
  hipError_t e;
  auto sweep = [&](const double *lin, double *lout) -> hipError_t {
    hipError_t q;
    if (lin) {
      if ((q = p1_rows(c, lin, R, 2, r, true))) return q;
    }
    const double *res = lin ? R : r;
    int slot = prof_begin(c, F_THOMAS);
    hipLaunchKernelGGL(k_p1_zsolve, dim3(nblk(4 * (size_t)c->ncol)), dim3(kBlock), 0, c->stream, c->nlev, c->ncol, s.zf,
                       res, lin,
                       lout, p.omega);
    hipLaunchKernelGGL(k_p1_hjacobi, dim3(nblk(ntr - nz4)), dim3(kBlock), 0, c->stream, nz4, ntr, s.dS, res, lin, lout,
                       p.omega);
    prof_end(c, F_THOMAS, slot);
    return hipGetLastError();
  };
  bool have = false;
  for (int k = 0; k < p.n_pre; ++k) {
    if ((e = sweep(have ? lam : nullptr, have ? tmp : lam))) return e;
    if (have) std::swap(lam, tmp);
    have = true;
  }
  if (!have) {
    hipLaunchKernelGGL(k_p1_fill, dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, lam, ntr, 0.0);
    if ((e = hipGetLastError())) return e;
  }
  if (p.coarse_mode == 0) {  // the DG0 coarse correction (coarse_mode 1: LineSmooth alone)
    if ((e = p1_rows(c, lam, R, 2, r, true))) return e;
    int slot = prof_begin(c, F_RESTRICT);
    hipLaunchKernelGGL(k_p1_restrict, dim3(nblk(nc)), dim3(kBlock), 0, c->stream, c->nlev, c->ncol, c->nedge,
                       (size_t)c->nz, L0.col_edge, R, s.gamma, (double *)cc->lv[0].b);
    prof_end(c, F_RESTRICT, slot);
    if ((e = hipGetLastError())) return e;
    if ((e = coarse_vcycle(cc))) return e;
    slot = prof_begin(c, F_PROLONG);
    hipLaunchKernelGGL(k_p1_prolong, dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, ntr, c->nlev, c->ncol, c->nedge,
                       (size_t)c->nz, L0.edge_col, L0.edge_lf, (const double *)cc->lv[0].x, lam);
    prof_end(c, F_PROLONG, slot);
    if ((e = hipGetLastError())) return e;
  }
  for (int k = 0; k < p.n_post; ++k) {
    double *dst = (k == p.n_post - 1) ? z : tmp;
    if ((e = sweep(lam, dst))) return e;
    if (dst == tmp) std::swap(lam, tmp);
  }
  if (p.n_post <= 0) return hipMemcpyAsync(z, lam, ntr * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  return hipSuccess;
}

void p1_free(hyb_ctx *c) {
  P1State &s = c->p1;
  if (s.SKf) (void)hipFree(s.SKf);
  s.SKf = nullptr;
  for (double **q : {&s.tbl, &s.A, &s.cdiag, &s.kdiag, &s.SK, &s.bK, &s.fac, &s.dS, &s.zf, &s.gamma, &s.den, &s.t1,
                     &s.t2, &s.t3})
    if (*q) (void)hipFree(*q), *q = nullptr;
}

}  // namespace hyb
