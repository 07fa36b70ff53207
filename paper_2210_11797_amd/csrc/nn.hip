// Learned coarse-correction network: three 3D convolutions on DG0 fields (1 -> C -> C -> 1
// channels, taps = the 3x3 horizontal neighbourhood of a column x 5 vertical offsets, zero padded
// below the ground and above the lid), ReLU after the first two.  Weights are kept in FP32 (master
// copy, Adam state) and used in BF16; activations and accumulation are FP32.
//
// Fields are [sample][channel][k][col].  One thread computes all output channels of one cell, so
// every gathered input value is reused for all of them; the weights of a layer sit in LDS.
// Weight gradients are reduced per workgroup and then summed over workgroups in a fixed order.
#include <hip/hip_bf16.h>

#include "hyb_internal.h"

namespace hyb {

namespace {

constexpr int NHT = 9, NVT = 5, NTAP = NHT * NVT;
constexpr int C1 = 16;  // hidden channels (the inference kernels are written for 16)
// opposite horizontal direction of each tap (centre, W, E, S, N, SW, SE, NW, NE)

inline unsigned nblk(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest, ties to even (finite inputs)
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

// y[s][co][cell] = bias[co] + sum_{ci,t} W[co][ci][t] x[s][ci][k+dk][nb[h][col]]   (RELU: max(.,0));
// the last CS of the CI input channels are static fields xst[CS][cell], the same for every sample
template <int CI, int CO, bool RELU, int CS = 0>
__global__ void __launch_bounds__(kBlock) k_conv_fwd(const float *__restrict__ x, const uint16_t *__restrict__ wb,
                                                     const float *__restrict__ bias, float *__restrict__ y, int nlev,
                                                     int ncol, int nsamp, const int32_t *__restrict__ nb9,
                                                     const float *__restrict__ xst = nullptr) {
  constexpr int CD = CI - CS;  // per-sample channels
  __shared__ float w[CO * CI * NTAP];
  for (int i = threadIdx.x; i < CO * CI * NTAP; i += blockDim.x) w[i] = bf2f(wb[i]);
  __syncthreads();
  const size_t n = (size_t)nlev * ncol;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * nsamp) return;
  const int s = (int)(gid / n);
  const int cell = (int)(gid - (size_t)s * n);
  const int k = cell / ncol, col = cell - k * ncol;
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = bias[co];
  const float *xs = x + (size_t)s * CD * n;
  for (int h = 0; h < NHT; ++h) {
    const int c2 = nb9[(size_t)h * ncol + col];
    if (c2 < 0) continue;  // no corner neighbour at a cube vertex: zero padding
#pragma unroll
    for (int v = 0; v < NVT; ++v) {
      const int kk = k + v - 2;
      if (kk < 0 || kk >= nlev) continue;
      const int t = h * NVT + v;
#pragma unroll
      for (int ci = 0; ci < CI; ++ci) {
        const float *src = ci < CD ? xs + (size_t)ci * n : xst + (size_t)(ci - CD) * n;
        const float xv = src[(size_t)kk * ncol + c2];
#pragma unroll
        for (int co = 0; co < CO; ++co) acc[co] += w[(co * CI + ci) * NTAP + t] * xv;
      }
    }
  }
  float *ys = y + (size_t)s * CO * n;
#pragma unroll
  for (int co = 0; co < CO; ++co) ys[(size_t)co * n + cell] = RELU ? fmaxf(acc[co], 0.f) : acc[co];
}

// dx[s][ci][cell] = (sum over the columns c' and taps h with nb[h][c'] = col of
//                    sum_{co,v} W[co][ci][h,v] dy[s][co][k-dk][c']) * (xin > 0 if MASK);
// rv9[r][col] = c' * 9 + h lists those pairs (at most 9, ordered by h; -1 pads)
template <int CI, int CO, bool MASK>
__global__ void __launch_bounds__(kBlock) k_conv_bwd_data(const float *__restrict__ dy, const uint16_t *__restrict__ wb,
                                                          const float *__restrict__ xin, float *__restrict__ dx,
                                                          int nlev, int ncol, int nsamp,
                                                          const int32_t *__restrict__ rv9) {
  __shared__ float w[CO * CI * NTAP];
  for (int i = threadIdx.x; i < CO * CI * NTAP; i += blockDim.x) w[i] = bf2f(wb[i]);
  __syncthreads();
  const size_t n = (size_t)nlev * ncol;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * nsamp) return;
  const int s = (int)(gid / n);
  const int cell = (int)(gid - (size_t)s * n);
  const int k = cell / ncol, col = cell - k * ncol;
  float acc[CI];
#pragma unroll
  for (int ci = 0; ci < CI; ++ci) acc[ci] = 0.f;
  const float *dys = dy + (size_t)s * CO * n;
  for (int rr = 0; rr < NHT; ++rr) {
    const int pk = rv9[(size_t)rr * ncol + col];
    if (pk < 0) continue;
    const int c2 = pk / NHT, h = pk - c2 * NHT;
#pragma unroll
    for (int v = 0; v < NVT; ++v) {
      const int kk = k - (v - 2);
      if (kk < 0 || kk >= nlev) continue;
      const int t = h * NVT + v;
#pragma unroll
      for (int co = 0; co < CO; ++co) {
        const float g = dys[(size_t)co * n + (size_t)kk * ncol + c2];
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) acc[ci] += w[(co * CI + ci) * NTAP + t] * g;
      }
    }
  }
  float *dxs = dx + (size_t)s * CI * n;
  const float *xs = xin + (size_t)s * CI * n;
#pragma unroll
  for (int ci = 0; ci < CI; ++ci) {
    float v = acc[ci];
    if (MASK && !(xs[(size_t)ci * n + cell] > 0.f)) v = 0.f;
    dxs[(size_t)ci * n + cell] = v;
  }
}

// Per-workgroup partial weight gradients over a tile of cells:
//   part[blk][co][ci][t] = sum_cells dy[co][cell] x[ci][k+dk][nb[h][col]],  part[blk][wsize+co] = sum dy[co]
constexpr int kTile = 512;
template <int CI, int CO, int CS = 0>
__global__ void __launch_bounds__(kBlock) k_conv_bwd_weight(const float *__restrict__ dy, const float *__restrict__ x,
                                                            float *__restrict__ part, int nlev, int ncol, int nsamp,
                                                            const int32_t *__restrict__ nb9,
                                                            const float *__restrict__ xst = nullptr) {
  constexpr int WS = CO * CI * NTAP, CD = CI - CS;
  __shared__ float sdy[kTile][CO];
  __shared__ int scell[kTile];
  const size_t n = (size_t)nlev * ncol, total = n * nsamp;
  const size_t t0 = (size_t)blockIdx.x * kTile;
  const int cnt = (int)min((size_t)kTile, total - t0);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    size_t g = t0 + i;
    int s = (int)(g / n), cell = (int)(g - (size_t)s * n);
#pragma unroll
    for (int co = 0; co < CO; ++co) sdy[i][co] = dy[((size_t)s * CO + co) * n + cell];
    scell[i] = (int)(g - (size_t)s * n);
  }
  __syncthreads();
  float *out = part + (size_t)blockIdx.x * (WS + CO);
  // one thread per (ci, tap) pair accumulates all CO outputs
  for (int p = threadIdx.x; p < CI * NTAP; p += blockDim.x) {
    const int ci = p / NTAP, t = p - ci * NTAP;
    const int h = t / NVT, dk = t - h * NVT - 2;
    float acc[CO];
#pragma unroll
    for (int co = 0; co < CO; ++co) acc[co] = 0.f;
    for (int i = 0; i < cnt; ++i) {
      const size_t g = t0 + i;
      const int s = (int)(g / n), cell = scell[i];
      const int k = cell / ncol, col = cell - k * ncol;
      const int kk = k + dk;
      if (kk < 0 || kk >= nlev) continue;
      const int c2 = nb9[(size_t)h * ncol + col];
      if (c2 < 0) continue;
      const float xv = ci < CD ? x[((size_t)s * CD + ci) * n + (size_t)kk * ncol + c2]
                               : xst[(size_t)(ci - CD) * n + (size_t)kk * ncol + c2];
#pragma unroll
      for (int co = 0; co < CO; ++co) acc[co] += sdy[i][co] * xv;
    }
#pragma unroll
    for (int co = 0; co < CO; ++co) out[(co * CI + ci) * NTAP + t] = acc[co];
  }
  if (threadIdx.x < CO) {
    float sb = 0.f;
    for (int i = 0; i < cnt; ++i) sb += sdy[i][threadIdx.x];
    out[WS + threadIdx.x] = sb;
  }
}

// grad[j] = sum over workgroups of part[blk][j] (fixed order)
__global__ void k_sum_parts(const float *__restrict__ part, int nparts, int len, float *__restrict__ grad) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  float s = 0.f;
  for (int b = 0; b < nparts; ++b) s += part[(size_t)b * len + j];
  grad[j] = s;
}

// dy = 2 (y - t) / N and partial sums of (y - t)^2
__global__ void __launch_bounds__(kBlock) k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                                float *__restrict__ dy, size_t total, float *__restrict__ part) {
  __shared__ float red[kBlock / 64];
  float acc = 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    float d = y[i] - t[i];
    dy[i] = 2.f * d;  // d loss / d y without the 1 / total of the mean (applied to the gradients)
    acc += d * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int q = 0; q < kBlock / 64; ++q) s += red[q];
    part[blockIdx.x] = s;
  }
}

// g *= a (the loss scale, backpropagated as 1 so that the backward passes do not carry it)
__global__ void k_scale_f32(float *__restrict__ g, int n, float a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] *= a;
}

// Adam on the FP32 master weights; refresh the BF16 copy of the weights (not of the biases)
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, uint16_t *__restrict__ wb, const int32_t *__restrict__ isbf,
                       int len, float lr, float b1, float b2, float eps, float c1, float c2) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  float gj = g[j];
  float mj = b1 * m[j] + (1.f - b1) * gj;
  float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  float wj = w[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
  w[j] = wj;
  int q = isbf[j];
  if (q >= 0) wb[q] = f2bf(wj);
}

__global__ void k_weights_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ wb,
                                  const int32_t *__restrict__ isbf, int len) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  int q = isbf[j];
  if (q >= 0) wb[q] = f2bf(w[j]);
}

// cells[c] = mode 0: Gamma_c sum_F w_F r_F;  mode 1: sum_F w_F r_F / sum_F w_F;  mode 2: H_cc times
// mode 1;  mode 3: sum_F w_F r_F, i.e. (P^T r)_c  (w = 1/2, 1 on ground and lid facets: P^T for the
// facet-average prolongation P)
__global__ void k_restrict_cells(const double *__restrict__ r, const double *__restrict__ gamma,
                                 const double *__restrict__ hdiag, double *__restrict__ out, int nlev, int ncol,
                                 int nedge, size_t nz, const int32_t *__restrict__ col_edge, int mode) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nlev * ncol) return;
  int k = c / ncol, col = c - k * ncol;
  size_t hb = nz + (size_t)k * nedge;
  double s = 0.0;
#pragma unroll
  for (int f = 0; f < 4; ++f) s += r[hb + col_edge[(size_t)f * ncol + col]];
  s *= 0.5;
  double wb = (k == 0 ? 1.0 : 0.5), wt = (k == nlev - 1 ? 1.0 : 0.5);
  s += wb * r[(size_t)k * ncol + col] + wt * r[(size_t)(k + 1) * ncol + col];
  double v;
  if (mode == 0)
    v = gamma[c] * s;
  else if (mode == 1)
    v = s / (2.0 + wb + wt);
  else if (mode == 2)
    v = hdiag[c] * s / (2.0 + wb + wt);
  else
    v = s;
  out[c] = v;
}

// sum of squares of a vector into part[blk]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sumsq(const T *__restrict__ x, size_t n, double *__restrict__ part) {
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double v = (double)x[i];
    acc += v * v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t += red[q];
    part[blockIdx.x] = t;
  }
}

__global__ void k_sum_into(const double *__restrict__ part, int nb, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  *out = s;
}

// x = c / s with s = sqrt(scal[0] / n) (0 when s = 0)
__global__ void k_normalise(const double *__restrict__ c, const double *__restrict__ scal, float *__restrict__ x,
                            size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = sqrt(scal[0] / (double)n);
  x[i] = s > 0.0 ? (float)(c[i] / s) : 0.f;
}

// v /= s with s = sqrt(scal[0] / ncell) (0 when s = 0)
__global__ void k_div_rms(double *__restrict__ v, const double *__restrict__ scal, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = sqrt(scal[0] / (double)n);
  v[i] = s > 0.0 ? v[i] / s : 0.0;
}

// d_F = s (P (y / H_diag))_F when the network output is finite (scal[1] = sum y^2), else 0
__global__ void k_prolong_correction(const float *__restrict__ y, const double *__restrict__ scal,
                                     const double *__restrict__ hdiag, double *__restrict__ d, int nlev, int ncol,
                                     int nedge, size_t nz, size_t ntr, const int32_t *__restrict__ edge_col) {
  size_t F = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (F >= ntr) return;
  if (!isfinite(scal[1])) {
    d[F] = 0.0;
    return;
  }
  const double s = sqrt(scal[0] / (double)((size_t)nlev * ncol));
  double v;
  if (F < nz) {
    int k = (int)(F / ncol), col = (int)(F - (size_t)k * ncol);
    size_t lo = (size_t)(k - 1) * ncol + col, hi = (size_t)k * ncol + col;
    if (k == 0)
      v = (double)y[hi] / hdiag[hi];
    else if (k == nlev)
      v = (double)y[lo] / hdiag[lo];
    else
      v = 0.5 * ((double)y[lo] / hdiag[lo] + (double)y[hi] / hdiag[hi]);
  } else {
    size_t h = F - nz;
    int k = (int)(h / nedge), e = (int)(h - (size_t)k * nedge);
    size_t a = (size_t)k * ncol + edge_col[e], b = (size_t)k * ncol + edge_col[nedge + e];
    v = 0.5 * ((double)y[a] / hdiag[a] + (double)y[b] / hdiag[b]);
  }
  d[F] = s * v;
}

// partial sums of ||t - u||^2 (row 0) and ||t||^2 (row 1) per block: part[row * gridDim.x + blk]
__global__ void __launch_bounds__(kBlock) k_judge_sums(const double *__restrict__ t, const double *__restrict__ u,
                                                      size_t n, double *__restrict__ part) {
  __shared__ double red[2][kBlock / 64];
  double a = 0.0, b = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double ti = t[i], di = ti - u[i];
    a += di * di;
    b += ti * ti;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) red[0][threadIdx.x >> 6] = a, red[1][threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x < 2) {
    double t2 = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t2 += red[threadIdx.x][q];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t2;
  }
}

// z += d if the network output was finite (scal[1] = sum y^2) and the corrected residual stays
// below tau times the cycle's (scal[3] = ||r' - S d||^2, scal[4] = ||r'||^2); otherwise z is left as
// the two-level cycle made it and the fallback counter scal[2] grows
template <typename Tz>
__global__ void k_apply_correction(const double *__restrict__ d, double *__restrict__ scal, Tz *__restrict__ z,
                                   size_t n, double tau2) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = isfinite(scal[1]) && scal[3] < tau2 * scal[4];  // false for NaN
  if (!ok) {
    if (i == 0) scal[2] += 1.0;
    return;
  }
  if (i < n) z[i] = (Tz)((double)z[i] + d[i]);
}

// w = S z after the stage from the applications it already made: r - r' + S d if the correction
// was kept (r' = r - S z of the plain z), else r - r'
__global__ void k_stage_matvec(const double *__restrict__ r, const double *__restrict__ rp,
                               const double *__restrict__ sd, const double *__restrict__ scal, double *__restrict__ w,
                               size_t n, double tau2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = isfinite(scal[1]) && scal[3] < tau2 * scal[4];  // the same decision as the apply
  if (i < n) w[i] = r[i] - rp[i] + (ok ? sd[i] : 0.0);
}

// out_F = (P (y / H_diag))_F for one sample of network outputs y [ncell]
__global__ void k_prolong_q(const float *__restrict__ y, const double *__restrict__ hdiag, double *__restrict__ out,
                            int nlev, int ncol, int nedge, size_t nz, size_t ntr, const int32_t *__restrict__ edge_col) {
  size_t F = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (F >= ntr) return;
  double v;
  if (F < nz) {
    int k = (int)(F / ncol), col = (int)(F - (size_t)k * ncol);
    size_t lo = (size_t)(k - 1) * ncol + col, hi = (size_t)k * ncol + col;
    if (k == 0)
      v = (double)y[hi] / hdiag[hi];
    else if (k == nlev)
      v = (double)y[lo] / hdiag[lo];
    else
      v = 0.5 * ((double)y[lo] / hdiag[lo] + (double)y[hi] / hdiag[hi]);
  } else {
    size_t h = F - nz;
    int k = (int)(h / nedge), e = (int)(h - (size_t)k * nedge);
    size_t a = (size_t)k * ncol + edge_col[e], b = (size_t)k * ncol + edge_col[nedge + e];
    v = 0.5 * ((double)y[a] / hdiag[a] + (double)y[b] / hdiag[b]);
  }
  out[F] = v;
}

// Energy loss over a batch: q = y / H_diag per cell (H_diag repeats for every sample), partial sums of
// q (Gq - 2 rhat) per block, and dy = 2 (Gq - rhat) / H_diag (the loss scale is applied to the gradients)
__global__ void __launch_bounds__(kBlock) k_energy(const float *__restrict__ y, const double *__restrict__ gq,
                                                  const double *__restrict__ rhat, const double *__restrict__ hdiag,
                                                  float *__restrict__ dy, size_t ncell, size_t total,
                                                  double *__restrict__ part) {
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    double h = hdiag[i % ncell], q = (double)y[i] / h, g = gq[i], r = rhat[i];
    acc += q * (g - 2.0 * r);
    dy[i] = (float)(2.0 * (g - r) / h);  // without the loss scale (applied to the gradients)
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t += red[q];
    part[blockIdx.x] = t;
  }
}

// ---- inference path of the stage (one sample): BF16 activations on matrix cores -------------------
// a1 = bf16(relu(conv1(x))) by the lanes (FP32 accumulation), a2 = bf16(relu(conv2(a1))) as an implicit
// GEMM on BF16 MFMA (FP32 accumulation): for 16 cells and one tap, A = a1 of the 16 tapped cells x 16
// input channels, B = W2[:, :, tap]^T (16 x 16), 45 taps accumulate into the 16 cells x 16 outputs;
// y = conv3(a2) by the lanes.  Activations are stored per cell, 16 BF16 channels contiguous.
typedef float nn_f32x4 __attribute__((ext_vector_type(4)));
typedef short nn_bf16x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kBlock) k_inf_layer1(const float *__restrict__ x, const uint16_t *__restrict__ wb,
                                                      const float *__restrict__ bias, uint16_t *__restrict__ a1,
                                                      int nlev, int ncol, int nsamp, const int32_t *__restrict__ nb9,
                                                      const float *__restrict__ xst) {
  constexpr int CIN = kNNInputs;  // x, then the static fields xst[CIN - 1][cell]
  // weights in LDS as [tap][ci][co], so that a tap's weights are read as whole vectors
  __shared__ float w[C1 * CIN * NTAP];
  for (int i = threadIdx.x; i < C1 * CIN * NTAP; i += blockDim.x) {
    const int t = i / (CIN * C1), rem = i - t * (CIN * C1), ci = rem / C1, co = rem - ci * C1;
    w[i] = bf2f(wb[(co * CIN + ci) * NTAP + t]);
  }
  __syncthreads();
  // 32-bit row arithmetic (the host keeps rows x samples below 2^32)
  const unsigned n = (unsigned)nlev * (unsigned)ncol;
  const unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * (unsigned)nsamp) return;
  const unsigned smp = gid / n;
  const int cell = (int)(gid - smp * n);
  const int k = cell / ncol, col = cell - k * ncol;
  x += (size_t)smp * n;
  float acc[C1];
#pragma unroll
  for (int co = 0; co < C1; ++co) acc[co] = bias[co];
  for (int h = 0; h < NHT; ++h) {
    const int c2 = nb9[(size_t)h * ncol + col];
    if (c2 < 0) continue;
#pragma unroll
    for (int v = 0; v < NVT; ++v) {
      const int kk = k + v - 2;
      if (kk < 0 || kk >= nlev) continue;
      const size_t at2 = (size_t)kk * ncol + c2;
      float xv[CIN];
      xv[0] = x[at2];
#pragma unroll
      for (int ci = 1; ci < CIN; ++ci) xv[ci] = xst[(size_t)(ci - 1) * nlev * ncol + at2];
#pragma unroll
      for (int co = 0; co < C1; ++co)
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci) acc[co] += w[((h * NVT + v) * CIN + ci) * C1 + co] * xv[ci];
    }
  }
#pragma unroll
  for (int co = 0; co < C1; ++co) a1[(size_t)gid * C1 + co] = f2bf(fmaxf(acc[co], 0.f));
}

// Layer 2 (16 -> 16 channels) as an implicit GEMM on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulation): a wavefront takes tiles of 16 rows (sample, cell); one product covers two taps, the
// A operand holding the 16 rows' tapped activations (lanes of quarter q: tap 2p + q / 2, channels
// 8 (q % 2) .. + 7, one 16-byte load) and B the two taps' weights from LDS.  23 products cover the 45
// taps.  Forward: out = bf16(relu(conv2(in) + b2)) with tap_col = the 3x3 neighbourhood.  Backward
// (BWD): out = bf16(conv2^T(in) * (gate > 0)), the transposed convolution gathered through the readers
// of each column: tap_col[h][col] is the column that reads col through horizontal tap h (its level
// offset reversed); where several columns read col through the same tap (next to cube edges), the
// others are listed in lo_list[lo_off[col] .. lo_off[col + 1]) as reader * 9 + h and added by the
// lanes after the products.  Rows are [sample][cell], 16 BF16 channels contiguous.
typedef __bf16 nn_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int nn_u32x4 __attribute__((ext_vector_type(4)));
typedef short nn_s16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ nn_f32x4 mfma_bf16_32(nn_u32x4 a, nn_u32x4 b, nn_f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(nn_bf16x8, a), __builtin_bit_cast(nn_bf16x8, b), c,
                                                 0, 0, 0);
}

constexpr int kC2Tiles = 8;  // 16-row tiles per wavefront
template <bool BWD>
__global__ void __launch_bounds__(kBlock) k_conv2_mfma(const uint16_t *__restrict__ in, const uint16_t *__restrict__ wb2,
                                                      const float *__restrict__ bias, const uint16_t *__restrict__ gate,
                                                      uint16_t *__restrict__ out, int nlev, int ncol, int nsamp,
                                                      const int32_t *__restrict__ tap_col,
                                                      const int32_t *__restrict__ lo_off,
                                                      const int32_t *__restrict__ lo_list) {
  // weights as [tap][n][k]: forward n = output channel, k = input channel; backward the transpose
  __shared__ nn_u32x4 sW[NTAP][C1][2];
  for (int i = threadIdx.x; i < NTAP * C1 * C1; i += blockDim.x) {
    const int t = i / (C1 * C1), rem = i - t * (C1 * C1), nn = rem / C1, kk = rem - nn * C1;
    const int co = BWD ? kk : nn, ci = BWD ? nn : kk;
    reinterpret_cast<uint16_t *>(&sW[t][nn][0])[kk] = wb2[(co * C1 + ci) * NTAP + t];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4, half = q & 1;
  const bool second = q >= 2;
  const unsigned n = (unsigned)nlev * (unsigned)ncol, total = n * (unsigned)nsamp;
  const unsigned wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const nn_u32x4 zero4 = {0u, 0u, 0u, 0u};
  for (int tile = 0; tile < kC2Tiles; ++tile) {
    const unsigned base = (wave * kC2Tiles + tile) * 16;
    if (base >= total) break;  // uniform over the wavefront
    const unsigned g = base + r;
    const bool live = g < total;
    const unsigned gs = live ? g : base;
    const unsigned smp = gs / n;
    const int cell = (int)(gs - smp * n);
    const int k = cell / ncol, col = cell - k * ncol;
    const uint16_t *ins = in + (size_t)smp * n * C1;
    int cn[NHT];  // the 3x3 neighbourhood first, so that the tap loads do not wait on it
#pragma unroll
    for (int h = 0; h < NHT; ++h) cn[h] = tap_col[(size_t)h * ncol + col];
    nn_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < (NTAP + 1) / 2; ++p) {
      constexpr int kLast = NTAP - 1;
      const int t0 = 2 * p, t1 = (2 * p + 1 <= kLast) ? 2 * p + 1 : kLast;
      const bool has = second ? (2 * p + 1 <= kLast) : true;
      const int t = second ? t1 : t0;
      const int c2 = second ? cn[t1 / NVT] : cn[t0 / NVT];
      const int v = second ? t1 % NVT : t0 % NVT;
      const int kk = BWD ? k - (v - 2) : k + (v - 2);
      const int kc = kk < 0 ? 0 : (kk >= nlev ? nlev - 1 : kk);
      // unconditional load from a clamped place (discarded outside), so the loads issue ahead
      const nn_u32x4 u = *reinterpret_cast<const nn_u32x4 *>(ins + ((size_t)kc * ncol + (c2 >= 0 ? c2 : col)) * C1 +
                                                              8 * half);
      const bool ok = live && has && c2 >= 0 && kk == kc;
      const nn_u32x4 a = ok ? u : zero4;
      const nn_u32x4 b = has ? sW[t][r][half] : zero4;
      acc = mfma_bf16_32(a, b, acc);
    }
    // acc[j] = channel r of row base + 4 q + j
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned go = base + 4 * q + j;
      if (go >= total) continue;
      float val = acc[j];
      if (!BWD) {
        out[(size_t)go * C1 + r] = f2bf(fmaxf(val + bias[r], 0.f));
      } else {
        const unsigned so = go / n;
        const int oc = (int)(go - so * n), ko = oc / ncol, colo = oc - ko * ncol;
        for (int e = lo_off[colo]; e < lo_off[colo + 1]; ++e) {
          const int pk = lo_list[e], cr = pk / NHT, hh = pk - cr * NHT;
          for (int v = 0; v < NVT; ++v) {
            const int kk = ko - (v - 2);
            if (kk < 0 || kk >= nlev) continue;
            const uint16_t *src = in + ((size_t)so * n + (size_t)kk * ncol + cr) * C1;
            const uint16_t *w = reinterpret_cast<const uint16_t *>(&sW[hh * NVT + v][r][0]);
            for (int co = 0; co < C1; ++co) val += bf2f(w[co]) * bf2f(src[co]);
          }
        }
        out[(size_t)go * C1 + r] = bf2f(gate[(size_t)go * C1 + r]) > 0.f ? f2bf(val) : (uint16_t)0;
      }
    }
  }
}

// Weight gradients on BF16 MFMA: for horizontal tap h = blockIdx.y and the five vertical offsets v,
//   part[blk][h][v][co][ci] = sum over this workgroup's rows of dA[row][co] * act[tap(row, h, v)][ci],
// and for h = 0 the bias sums bpart[blk][co] = sum over the rows of dA[row][co].  A wavefront takes
// chunks of 32 rows (sample, cell): D = A B with A = dA^T (16 output channels x 32 rows) and B = the
// tapped activations (32 rows x 16 input channels).  Both operands need 8 rows of one channel per
// lane, so each chunk is loaded with one 16-byte load per lane (lane = row / 2, half the channels)
// and turned over in the wavefront's own LDS tile ([channel][row], rows padded to 40 so that the
// operand reads fall on distinct banks).
// dA: CA = 16 BF16 [sample][cell][16], CA = 1 FP32 [sample][cell] (rounded to BF16 for the product; the
// bias sum takes it unrounded).  act: CB = 16 BF16 [sample][cell][16]; CB = 3 the network's input, x
// FP32 [sample][cell] and the static fields st FP32 [2][cell].  Channels beyond CA / CB are zero.
constexpr int kWgBlocks = 256;
constexpr int kWgPad = 40;

// LDS written by some lanes of a wavefront and then read by others: the wavefront's LDS accesses are
// processed in order, so only the compiler must keep the order
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CA, int CB>
__global__ void __launch_bounds__(kBlock) k_wgrad_mfma(const void *__restrict__ dA_, const void *__restrict__ act_,
                                                      const float *__restrict__ st, float *__restrict__ part,
                                                      float *__restrict__ bpart, int nlev, int ncol, int nsamp,
                                                      const int32_t *__restrict__ nb9) {
  constexpr int NW = kBlock / 64;
  __shared__ uint16_t sA[NW][16][kWgPad], sB[NW][16][kWgPad];
  __shared__ float red[NW][NVT][4][64];
  __shared__ float bred[NW][64][8];
  const int h = blockIdx.y;
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4, wv = threadIdx.x >> 6;
  const int rho = lane >> 1, hf = lane & 1;  // the row this lane loads, and which 8 channels
  const unsigned n = (unsigned)nlev * (unsigned)ncol, total = n * (unsigned)nsamp;
  const unsigned nchunks = (total + 31) / 32;
  const unsigned nwaves = gridDim.x * NW;
  // rows and channels no lane writes stay zero
  for (int i = lane; i < 16 * kWgPad; i += 64) (&sA[wv][0][0])[i] = 0, (&sB[wv][0][0])[i] = 0;
  wave_lds_sync();
  const nn_f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  nn_f32x4 acc[NVT];
#pragma unroll
  for (int v = 0; v < NVT; ++v) acc[v] = zero;
  float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (unsigned ch = blockIdx.x * NW + wv; ch < nchunks; ch += nwaves) {
    const unsigned g = ch * 32 + rho;
    const bool live = g < total;
    const unsigned gs = live ? g : 0;
    const unsigned smp = gs / n, cell = gs - smp * n;
    const int k = (int)(cell / (unsigned)ncol), col = (int)(cell - (unsigned)k * ncol);
    const size_t soff = (size_t)smp * n;
    const int c2 = live ? nb9[(size_t)h * ncol + col] : -1;
    // A: this lane's row, 8 channels, into the tile [co][row]
    if (CA == 16) {
      nn_u32x4 u = {0u, 0u, 0u, 0u};
      if (live) u = *reinterpret_cast<const nn_u32x4 *>(reinterpret_cast<const uint16_t *>(dA_) + (size_t)gs * 16 + 8 * hf);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint16_t hv = (uint16_t)((i & 1) ? (u[i >> 1] >> 16) : (u[i >> 1] & 0xFFFFu));
        sA[wv][8 * hf + i][rho] = hv;
        bsum[i] += bf2f(hv);
      }
    } else if (hf == 0) {
      const float fv = live ? reinterpret_cast<const float *>(dA_)[gs] : 0.f;
      sA[wv][0][rho] = f2bf(fv);
      bsum[0] += fv;
    }
    wave_lds_sync();
    const nn_u32x4 a = *reinterpret_cast<const nn_u32x4 *>(&sA[wv][r][8 * q]);
#pragma unroll
    for (int v = 0; v < NVT; ++v) {
      const int kk = k + v - 2;
      const bool ok = c2 >= 0 && kk >= 0 && kk < nlev;
      const size_t at = soff + (ok ? (size_t)kk * ncol + c2 : 0);
      if (CB == 16) {
        nn_u32x4 u = {0u, 0u, 0u, 0u};
        if (ok) u = *reinterpret_cast<const nn_u32x4 *>(reinterpret_cast<const uint16_t *>(act_) + at * 16 + 8 * hf);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          sB[wv][8 * hf + i][rho] = (uint16_t)((i & 1) ? (u[i >> 1] >> 16) : (u[i >> 1] & 0xFFFFu));
      } else if (hf == 0) {
        const size_t c2n = at - soff;
        sB[wv][0][rho] = f2bf(ok ? reinterpret_cast<const float *>(act_)[at] : 0.f);
        sB[wv][1][rho] = f2bf(ok ? st[c2n] : 0.f);
        sB[wv][2][rho] = f2bf(ok ? st[(size_t)n + c2n] : 0.f);
      }
      wave_lds_sync();
      const nn_u32x4 b = *reinterpret_cast<const nn_u32x4 *>(&sB[wv][r][8 * q]);
      acc[v] = mfma_bf16_32(a, b, acc[v]);
      wave_lds_sync();  // the tile is rewritten by the next offset
    }
  }
  // the block's waves in a fixed order; lane (r, q) holds entry j of output channel 4 q + j, input r
#pragma unroll
  for (int v = 0; v < NVT; ++v)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wv][v][j][lane] = acc[v][j];
#pragma unroll
  for (int i = 0; i < 8; ++i) bred[wv][lane][i] = bsum[i];
  __syncthreads();
  float *out = part + ((size_t)blockIdx.x * NHT + h) * (NVT * 256);
  for (int o = threadIdx.x; o < NVT * 256; o += blockDim.x) {
    const int v = o >> 8, co = (o >> 4) & 15, ci = o & 15;
    const int src = ci + 16 * (co >> 2), j = co & 3;
    float sacc = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) sacc += red[w][v][j][src];
    out[o] = sacc;
  }
  if (h == 0 && threadIdx.x < 16) {  // channel co: half co / 8 of every row, entry co % 8
    const int co = threadIdx.x, hh = co >> 3, e = co & 7;
    float sacc = 0.f;
    for (int w = 0; w < NW; ++w)
      for (int rr = 0; rr < 32; ++rr) sacc += bred[w][2 * rr + hh][e];
    bpart[(size_t)blockIdx.x * 16 + co] = sacc;
  }
}

// grad_w[(co * CI + ci) * 45 + 5 h + v] and grad_b[co] summed over the workgroups' partials in a
// fixed order (co < CO, ci < CI); one thread per partial entry, so consecutive threads read
// consecutive partials.
__global__ void k_wgrad_sum(const float *__restrict__ part, const float *__restrict__ bpart, int nparts, int CO,
                            int CI, float *__restrict__ grad_w, float *__restrict__ grad_b) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int PER = NHT * NVT * 256;
  if (o < PER) {
    const int hv = o >> 8, co = (o >> 4) & 15, ci = o & 15;
    if (co >= CO || ci >= CI) return;
    float sacc = 0.f;
    for (int b = 0; b < nparts; ++b) sacc += part[(size_t)b * PER + o];
    grad_w[(co * CI + ci) * NTAP + hv] = sacc;
  } else if (o < PER + CO) {
    const int co = o - PER;
    float sacc = 0.f;
    for (int b = 0; b < nparts; ++b) sacc += bpart[(size_t)b * 16 + co];
    grad_b[co] = sacc;
  }
}

// Layer 3 backward to its input: dz2[row][ci] = bf16((a2[row][ci] > 0) * sum over the readers (c', h)
// of the column and v of W3[0][ci][5 h + v] dy[sample][k - (v - 2)][c']) (rv9: the readers, any order).
__global__ void __launch_bounds__(kBlock) k_bwd3_bf16(const float *__restrict__ dy, const uint16_t *__restrict__ wb3,
                                                     const uint16_t *__restrict__ a2, uint16_t *__restrict__ dz2,
                                                     int nlev, int ncol, int nsamp, const int32_t *__restrict__ rv9) {
  __shared__ float w[C1 * NTAP];  // [tap][ci]
  for (int i = threadIdx.x; i < C1 * NTAP; i += blockDim.x) w[i] = bf2f(wb3[(i % C1) * NTAP + i / C1]);
  __syncthreads();
  const unsigned n = (unsigned)nlev * (unsigned)ncol;
  const unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * (unsigned)nsamp) return;
  const unsigned smp = gid / n;
  const int cell = (int)(gid - smp * n);
  const int k = cell / ncol, col = cell - k * ncol;
  const float *dys = dy + (size_t)smp * n;
  float acc[C1];
#pragma unroll
  for (int ci = 0; ci < C1; ++ci) acc[ci] = 0.f;
  for (int rr = 0; rr < NHT; ++rr) {
    const int pk = rv9[(size_t)rr * ncol + col];
    if (pk < 0) continue;
    const int c2 = pk / NHT, hh = pk - c2 * NHT;
#pragma unroll
    for (int v = 0; v < NVT; ++v) {
      const int kk = k - (v - 2);
      if (kk < 0 || kk >= nlev) continue;
      const float g = dys[(size_t)kk * ncol + c2];
#pragma unroll
      for (int ci = 0; ci < C1; ++ci) acc[ci] += w[(hh * NVT + v) * C1 + ci] * g;
    }
  }
  const uint16_t *ag = a2 + (size_t)gid * C1;
  uint16_t *o = dz2 + (size_t)gid * C1;
#pragma unroll
  for (int ci = 0; ci < C1; ++ci) o[ci] = bf2f(ag[ci]) > 0.f ? f2bf(acc[ci]) : (uint16_t)0;
}

__global__ void __launch_bounds__(kBlock) k_inf_layer3(const uint16_t *__restrict__ a2, const uint16_t *__restrict__ wb3,
                                                      const float *__restrict__ bias, float *__restrict__ y, int nlev,
                                                      int ncol, int nsamp, const int32_t *__restrict__ nb9) {
  __shared__ float w[C1 * NTAP];  // [tap][ci]
  for (int i = threadIdx.x; i < C1 * NTAP; i += blockDim.x) w[i] = bf2f(wb3[(i % C1) * NTAP + i / C1]);
  __syncthreads();
  const unsigned n = (unsigned)nlev * (unsigned)ncol;
  const unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * (unsigned)nsamp) return;
  const unsigned smp = gid / n;
  const int cell = (int)(gid - smp * n);
  const int k = cell / ncol, col = cell - k * ncol;
  a2 += (size_t)smp * n * C1;
  float acc = bias[0];
  for (int h = 0; h < NHT; ++h) {
    const int c2 = nb9[(size_t)h * ncol + col];
    if (c2 < 0) continue;
#pragma unroll
    for (int v = 0; v < NVT; ++v) {
      const int kk = k + v - 2;
      if (kk < 0 || kk >= nlev) continue;
      const uint4 *src = reinterpret_cast<const uint4 *>(a2 + ((size_t)kk * ncol + c2) * C1);
      const uint4 u0 = src[0], u1 = src[1];
      const uint32_t words[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
      for (int ci = 0; ci < C1; ++ci) {
        const uint16_t hv = (uint16_t)((ci & 1) ? (words[ci >> 1] >> 16) : (words[ci >> 1] & 0xFFFFu));
        acc += w[(h * NVT + v) * C1 + ci] * bf2f(hv);
      }
    }
  }
  y[gid] = acc;
}

// Static input channels of the network: st[0] = log(h / dz) with h = sqrt(|K| / dz) the cell's
// horizontal size (0.5 log |K| - 1.5 log dz), st[1] = height of the cell centre over the lid's;
// layer[0][k] = log dz_k, layer[1][k] = centre height / lid height
__global__ void k_static_inputs(int ncell, int ncol, const double *__restrict__ vol, const double *__restrict__ layer,
                                int nlev, float *__restrict__ st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int k = c / ncol;
  st[c] = (float)(0.5 * log(vol[c]) - 1.5 * layer[k]);
  st[(size_t)ncell + c] = (float)layer[nlev + k];
}

__global__ void k_fill_nan(float *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = __uint_as_float(0x7FC00000u);
}

__global__ void k_zero_scal(double *p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0.0;
}

}  // namespace

hipError_t launch_restrict_cells(hyb_ctx *c, const double *r, double *cells, int mode) {
  const LevelDev &L0 = c->lv[0];
  hipLaunchKernelGGL(k_restrict_cells, dim3(nblk(c->ncell)), dim3(kBlock), 0, c->stream, r, c->gamma, L0.H, cells,
                     c->nlev, c->ncol, c->nedge, (size_t)c->nz, L0.col_edge, mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Host side.  Parameter vector layout (FP32): W1 [C][1][45], b1 [C], W2 [C][C][45], b2 [C],
// W3 [1][C][45], b3 [1].  The BF16 copy holds W1, W2, W3 back to back.
// ---------------------------------------------------------------------------------------------
static constexpr int C = kNNChannels;
static constexpr int CIN = kNNInputs;
static constexpr int W1N = C * CIN * NTAP, W2N = C * C * NTAP, W3N = 1 * C * NTAP;
static constexpr int OFF_W1 = 0, OFF_B1 = W1N, OFF_W2 = OFF_B1 + C, OFF_B2 = OFF_W2 + W2N, OFF_W3 = OFF_B2 + C,
                     OFF_B3 = OFF_W3 + W3N, NPARAM = OFF_B3 + 1;

int nn_param_count() { return NPARAM; }

hipError_t nn_setup(hyb_ctx *c) {
  NNState &s = c->nn;
  if (s.w) return hipSuccess;
  hipError_t e;
  auto A = [&](void **p, size_t b) -> hipError_t {
    hipError_t r = hipMalloc(p, b);
    if (r == hipSuccess) c->bytes += b;
    return r;
  };
  if ((e = A((void **)&s.w, NPARAM * 4)) || (e = A((void **)&s.m, NPARAM * 4)) || (e = A((void **)&s.v, NPARAM * 4)) ||
      (e = A((void **)&s.g, NPARAM * 4)) || (e = A((void **)&s.wb, (W1N + W2N + W3N) * 2)) ||
      (e = A((void **)&s.isbf, NPARAM * 4)) || (e = A((void **)&s.nb9, 9 * (size_t)c->ncol * 4)) ||
      (e = A((void **)&s.rv9, 9 * (size_t)c->ncol * 4)))
    return e;
  std::vector<int32_t> isbf(NPARAM, -1);
  for (int j = 0; j < W1N; ++j) isbf[OFF_W1 + j] = j;
  for (int j = 0; j < W2N; ++j) isbf[OFF_W2 + j] = W1N + j;
  for (int j = 0; j < W3N; ++j) isbf[OFF_W3 + j] = W1N + W2N + j;
  if ((e = hipMemcpy(s.isbf, isbf.data(), NPARAM * 4, hipMemcpyHostToDevice))) return e;
  // 3x3 horizontal neighbourhood in each column's frame: the edge neighbours, and the corner
  // neighbour at (dx, dy) one step along y and then one along x, the x direction turned into the
  // neighbour's frame by the quarter turn between the frames (none on the periodic box); where the
  // two step orders disagree (cube vertices) there is no corner neighbour: -1, read as zeros.
  // rv9 lists, per column, the (column, tap) pairs that read it, for the transposed convolution.
  std::vector<int32_t> nbr(4 * (size_t)c->ncol), nlf(4 * (size_t)c->ncol), nb9(9 * (size_t)c->ncol);
  if ((e = hipMemcpy(nbr.data(), c->lv[0].nbr, nbr.size() * 4, hipMemcpyDeviceToHost)) ||
      (e = hipMemcpy(nlf.data(), c->lv[0].nlf, nlf.size() * 4, hipMemcpyDeviceToHost)))
    return e;
  const size_t n = c->ncol;
  static const int kDirOfFace[4] = {2, 0, 3, 1};  // W, E, S, N -> counter-clockwise direction (E, N, W, S)
  static const int kFaceOfDir[4] = {1, 3, 0, 2};
  auto route = [&](size_t col, int f1, int f2) {
    const int nb = nbr[f1 * n + col];
    const int turn = (kDirOfFace[nlf[f1 * n + col]] + 2 - kDirOfFace[f1]) & 3;
    return nbr[(size_t)kFaceOfDir[(kDirOfFace[f2] + turn) & 3] * n + nb];
  };
  auto corner = [&](size_t col, int fx, int fy) {
    const int a = route(col, fy, fx), b = route(col, fx, fy);
    return a == b ? a : -1;
  };
  for (size_t col = 0; col < n; ++col) {
    int v[9] = {(int)col, nbr[0 * n + col], nbr[1 * n + col], nbr[2 * n + col], nbr[3 * n + col],
                corner(col, 0, 2), corner(col, 1, 2), corner(col, 0, 3), corner(col, 1, 3)};
    for (int h = 0; h < 9; ++h) nb9[h * n + col] = v[h];
  }
  std::vector<int32_t> rv9(9 * n, -1);
  std::vector<int> cnt(n, 0);
  if (n * 9 > (size_t)INT32_MAX) return hipErrorInvalidValue;
  for (int h = 0; h < 9; ++h)
    for (size_t col = 0; col < n; ++col) {
      const int t = nb9[h * n + col];
      if (t < 0) continue;
      if (cnt[t] >= 9) return hipErrorInvalidValue;  // more than 9 readers of one column
      rv9[(size_t)cnt[t]++ * n + t] = (int32_t)(col * 9 + h);
    }
  // the same readers by tap for the transposed convolution on matrix cores: rvh[h][col] = the first
  // column that reads col through tap h (-1: none), the further ones (next to cube edges) listed
  // per column as col' * 9 + h
  std::vector<int32_t> rvh(9 * n, -1), lo_off(n + 1, 0), lo_list;
  std::vector<std::vector<int32_t>> extra(n);
  for (int h = 0; h < 9; ++h)
    for (size_t col = 0; col < n; ++col) {
      const int t = nb9[h * n + col];
      if (t < 0) continue;
      if (rvh[h * n + t] < 0)
        rvh[h * n + t] = (int32_t)col;
      else
        extra[t].push_back((int32_t)(col * 9 + h));
    }
  for (size_t col = 0; col < n; ++col) {
    lo_off[col + 1] = lo_off[col] + (int32_t)extra[col].size();
    lo_list.insert(lo_list.end(), extra[col].begin(), extra[col].end());
  }
  if (lo_list.empty()) lo_list.push_back(0);  // a valid pointer when no column has further readers
  auto A2 = [&](int32_t **p, const std::vector<int32_t> &v) -> hipError_t {
    hipError_t r = hipMalloc((void **)p, v.size() * 4);
    if (r) return r;
    c->bytes += v.size() * 4;
    return hipMemcpy(*p, v.data(), v.size() * 4, hipMemcpyHostToDevice);
  };
  if ((e = hipMemcpy(s.nb9, nb9.data(), nb9.size() * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(s.rv9, rv9.data(), rv9.size() * 4, hipMemcpyHostToDevice)) || (e = A2(&s.rvh, rvh)) ||
      (e = A2(&s.lo_off, lo_off)) || (e = A2(&s.lo_list, lo_list)))
    return e;
  std::vector<float> zero(NPARAM, 0.f);
  if ((e = hipMemcpy(s.m, zero.data(), NPARAM * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(s.v, zero.data(), NPARAM * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(s.w, zero.data(), NPARAM * 4, hipMemcpyHostToDevice)))
    return e;
  s.step = 0;
  return hipSuccess;
}

hipError_t nn_set_weights(hyb_ctx *c, const float *host_w) {
  NNState &s = c->nn;
  hipError_t e = hipMemcpy(s.w, host_w, NPARAM * 4, hipMemcpyHostToDevice);
  if (e) return e;
  std::vector<float> zero(NPARAM, 0.f);
  if ((e = hipMemcpy(s.m, zero.data(), NPARAM * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(s.v, zero.data(), NPARAM * 4, hipMemcpyHostToDevice)))
    return e;
  s.step = 0;
  hipLaunchKernelGGL(k_weights_to_bf16, dim3(nblk(NPARAM)), dim3(kBlock), 0, c->stream, s.w, s.wb, s.isbf, NPARAM);
  e = hipGetLastError();
  if (e) return e;
  return hipStreamSynchronize(c->stream);
}

hipError_t nn_get_state(hyb_ctx *c, float *m, float *v, int64_t *step) {
  NNState &s = c->nn;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e || (e = hipMemcpy(m, s.m, NPARAM * 4, hipMemcpyDeviceToHost)) ||
      (e = hipMemcpy(v, s.v, NPARAM * 4, hipMemcpyDeviceToHost)))
    return e;
  *step = s.step;
  return hipSuccess;
}

hipError_t nn_set_state(hyb_ctx *c, const float *m, const float *v, int64_t step) {
  NNState &s = c->nn;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e || (e = hipMemcpy(s.m, m, NPARAM * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(s.v, v, NPARAM * 4, hipMemcpyHostToDevice)))
    return e;
  s.step = (long)step;
  return hipSuccess;
}

hipError_t nn_get_weights(hyb_ctx *c, float *host_w) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e) return e;
  return hipMemcpy(host_w, c->nn.w, NPARAM * 4, hipMemcpyDeviceToHost);
}

static hipError_t ensure_acts(hyb_ctx *c, int nsamp) {
  NNState &s = c->nn;
  size_t n = (size_t)c->ncell * nsamp;
  if (s.cap >= n) return hipSuccess;
  for (float **p : {&s.a1, &s.a2, &s.y, &s.d1, &s.d2, &s.dy})
    if (*p) (void)hipFree(*p), *p = nullptr;
  if (s.part) (void)hipFree(s.part), s.part = nullptr;
  hipError_t e;
  if ((e = hipMalloc((void **)&s.a1, n * C * 4)) || (e = hipMalloc((void **)&s.a2, n * C * 4)) ||
      (e = hipMalloc((void **)&s.d1, n * C * 4)) || (e = hipMalloc((void **)&s.d2, n * C * 4)) ||
      (e = hipMalloc((void **)&s.y, n * 4)) || (e = hipMalloc((void **)&s.dy, n * 4)))
    return e;
  size_t nparts = (n + kTile - 1) / kTile;
  if ((e = hipMalloc((void **)&s.part, nparts * (size_t)(W2N + C) * 4))) return e;
  c->bytes += n * (4 * C + 2) * 4 + nparts * (size_t)(W2N + C) * 4;
  s.cap = n;
  return hipSuccess;
}

// The static input channels from the cell volumes of the last assembly and the layer thicknesses.
static hipError_t nn_static(hyb_ctx *c) {
  NNState &s = c->nn;
  if (s.st_ready) return hipSuccess;
  if (!c->vol || !c->assembled) return hipErrorInvalidValue;  // the network needs the assembled mesh
  hipError_t e;
  const size_t n = (size_t)c->ncell;
  if (!s.st) {
    if ((e = hipMalloc((void **)&s.st, 2 * n * 4)) || (e = hipMalloc((void **)&s.layer, 2 * (size_t)c->nlev * 8)))
      return e;
    c->bytes += 2 * n * 4 + 2 * (size_t)c->nlev * 8;
  }
  std::vector<double> layer(2 * (size_t)c->nlev);
  double top = 0.0;
  for (double d : c->dz) top += d;
  double z = 0.0;
  for (int k = 0; k < c->nlev; ++k) {
    layer[k] = std::log(c->dz[k]);
    layer[c->nlev + k] = (z + 0.5 * c->dz[k]) / top;
    z += c->dz[k];
  }
  if ((e = hipMemcpyAsync(s.layer, layer.data(), layer.size() * 8, hipMemcpyHostToDevice, c->stream))) return e;
  hipLaunchKernelGGL(k_static_inputs, dim3(nblk(n)), dim3(kBlock), 0, c->stream, c->ncell, c->ncol, c->vol, s.layer,
                     c->nlev, s.st);
  if ((e = hipGetLastError())) return e;
  if ((e = hipStreamSynchronize(c->stream))) return e;  // the host array goes out of scope
  s.st_ready = true;
  return hipSuccess;
}

// The BF16 matrix-core forward pass of nsamp fields: a1, a2 BF16 [nsamp][ncell][16] (in the
// activation buffers), out FP32 [nsamp][ncell].
static hipError_t forward_bf16(hyb_ctx *c, const float *x, uint16_t *a1, uint16_t *a2, float *out, int nsamp) {
  NNState &s = c->nn;
  const size_t n = (size_t)c->ncell * nsamp;
  if (n + 64 > (size_t)UINT32_MAX) return hipErrorInvalidValue;  // the kernels index rows in 32 bits
  const int L = c->nlev, nc = c->ncol;
  hipLaunchKernelGGL(k_inf_layer1, dim3(nblk(n)), dim3(kBlock), 0, c->stream, x, s.wb, s.w + OFF_B1, a1, L, nc, nsamp,
                     s.nb9, (const float *)s.st);
  const size_t waves = (n + 16 * kC2Tiles - 1) / (16 * kC2Tiles);
  hipLaunchKernelGGL((k_conv2_mfma<false>), dim3(nblk(waves, kBlock / 64)), dim3(kBlock), 0, c->stream,
                     (const uint16_t *)a1, s.wb + W1N, s.w + OFF_B2, (const uint16_t *)nullptr, a2, L, nc, nsamp, s.nb9,
                     (const int32_t *)nullptr, (const int32_t *)nullptr);
  hipLaunchKernelGGL(k_inf_layer3, dim3(nblk(n)), dim3(kBlock), 0, c->stream, (const uint16_t *)a2, s.wb + W1N + W2N,
                     s.w + OFF_B3, out, L, nc, nsamp, s.nb9);
  return hipGetLastError();
}

// Forward pass of nsamp fields x [nsamp][ncell] -> out [nsamp][ncell] (activations kept for backward):
// BF16 activations on matrix cores, or with params.nn_fp32 FP32 activations on the vector units.
hipError_t nn_forward(hyb_ctx *c, const float *x, float *out, int nsamp) {
  NNState &s = c->nn;
  hipError_t e = ensure_acts(c, nsamp);
  if (e) return e;
  if ((e = nn_static(c))) return e;
  if (!c->p.nn_fp32) return forward_bf16(c, x, (uint16_t *)s.a1, (uint16_t *)s.a2, out, nsamp);
  size_t n = (size_t)c->ncell * nsamp;
  dim3 g(nblk(n)), b(kBlock);
  int L = c->nlev, nc = c->ncol;
  hipLaunchKernelGGL((k_conv_fwd<CIN, C, true, CIN - 1>), g, b, 0, c->stream, x, s.wb, s.w + OFF_B1, s.a1, L, nc,
                     nsamp, s.nb9, (const float *)s.st);
  hipLaunchKernelGGL((k_conv_fwd<C, C, true>), g, b, 0, c->stream, s.a1, s.wb + W1N, s.w + OFF_B2, s.a2, L, nc, nsamp,
                     s.nb9);
  hipLaunchKernelGGL((k_conv_fwd<C, 1, false>), g, b, 0, c->stream, s.a2, s.wb + W1N + W2N, s.w + OFF_B3, out, L, nc,
                     nsamp, s.nb9);
  return hipGetLastError();
}

// Forward pass of one field for the stage inside the solve: BF16 activations, middle layer on MFMA.
static hipError_t nn_forward_inference(hyb_ctx *c, const float *x, float *out) {
  NNState &s = c->nn;
  static_assert(C == C1, "the inference kernels are written for 16 hidden channels");
  const size_t n = (size_t)c->ncell;
  hipError_t e;
  if (!s.a1h) {
    if ((e = hipMalloc((void **)&s.a1h, n * C * 2)) || (e = hipMalloc((void **)&s.a2h, n * C * 2))) return e;
    c->bytes += 2 * n * C * 2;
  }
  if ((e = nn_static(c))) return e;
  return forward_bf16(c, x, s.a1h, s.a2h, out, 1);
}

// Weight and bias gradients of one layer on matrix cores (k_wgrad_mfma, then the fixed-order sum).
template <int CA, int CB>
static hipError_t wgrad_mfma(hyb_ctx *c, const void *dA, const void *act, int nsamp, int CO, int CI, float *grad_w,
                             float *grad_b) {
  NNState &s = c->nn;
  const size_t nchunks = ((size_t)c->ncell * nsamp + 31) / 32;
  if ((size_t)c->ncell * nsamp + 32 > (size_t)UINT32_MAX) return hipErrorInvalidValue;  // 32-bit row indices
  const int nparts = (int)std::min<size_t>(kWgBlocks, (nchunks + 3) / 4);
  float *bp = s.wpart + (size_t)kWgBlocks * NHT * NVT * 256;
  hipLaunchKernelGGL((k_wgrad_mfma<CA, CB>), dim3(nparts, NHT), dim3(kBlock), 0, c->stream, dA, act,
                     (const float *)s.st, s.wpart, bp, c->nlev, c->ncol, nsamp, s.nb9);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_wgrad_sum, dim3(nblk(NHT * NVT * 256 + 16)), dim3(kBlock), 0, c->stream, (const float *)s.wpart,
                     (const float *)bp, nparts, CO, CI, grad_w, grad_b);
  return hipGetLastError();
}

// Gradients of every parameter into s.g from dL/dy in s.dy, BF16 matrix-core path: activations of
// forward_bf16 in s.a1 / s.a2 (BF16), the backpropagated fields in s.d2 / s.d1 (BF16 [nsamp][ncell][16]).
static hipError_t backward_bf16(hyb_ctx *c, const float *x, int nsamp) {
  NNState &s = c->nn;
  hipError_t e;
  const size_t n = (size_t)c->ncell * nsamp;
  const int L = c->nlev, nc = c->ncol;
  const uint16_t *a1 = (const uint16_t *)s.a1, *a2 = (const uint16_t *)s.a2;
  uint16_t *dz2 = (uint16_t *)s.d2, *dz1 = (uint16_t *)s.d1;
  // layer 3 (16 -> 1): dW3, db3, then dz2 = conv3^T(dy) * (a2 > 0)
  if ((e = wgrad_mfma<1, C1>(c, s.dy, a2, nsamp, 1, C, s.g + OFF_W3, s.g + OFF_B3))) return e;
  hipLaunchKernelGGL(k_bwd3_bf16, dim3(nblk(n)), dim3(kBlock), 0, c->stream, (const float *)s.dy, s.wb + W1N + W2N, a2,
                     dz2, L, nc, nsamp, s.rv9);
  if ((e = hipGetLastError())) return e;
  // layer 2 (16 -> 16): dW2, db2, then dz1 = conv2^T(dz2) * (a1 > 0)
  if ((e = wgrad_mfma<C1, C1>(c, dz2, a1, nsamp, C, C, s.g + OFF_W2, s.g + OFF_B2))) return e;
  const size_t waves = (n + 16 * kC2Tiles - 1) / (16 * kC2Tiles);
  hipLaunchKernelGGL((k_conv2_mfma<true>), dim3(nblk(waves, kBlock / 64)), dim3(kBlock), 0, c->stream,
                     (const uint16_t *)dz2, s.wb + W1N, (const float *)nullptr, a1, dz1, L, nc, nsamp, s.rvh, s.lo_off,
                     s.lo_list);
  if ((e = hipGetLastError())) return e;
  // layer 1 (the input x and the two static fields -> 16)
  return wgrad_mfma<C1, CIN>(c, dz1, x, nsamp, C, CIN, s.g + OFF_W1, s.g + OFF_B1);
}

template <int CI, int CO, int CS = 0>
static hipError_t weight_grad(hyb_ctx *c, const float *dy, const float *x, int nsamp, float *grad_w, float *grad_b) {
  NNState &s = c->nn;
  size_t n = (size_t)c->ncell * nsamp;
  int nparts = (int)((n + kTile - 1) / kTile);
  constexpr int WS = CO * CI * NTAP;
  hipLaunchKernelGGL((k_conv_bwd_weight<CI, CO, CS>), dim3(nparts), dim3(kBlock), 0, c->stream, dy, x, s.part,
                     c->nlev, c->ncol, nsamp, s.nb9, (const float *)s.st);
  hipError_t e = hipGetLastError();
  if (e) return e;
  // sum: weights then biases (contiguous WS + CO per part; the grad layout keeps W and b apart)
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(WS + CO)), dim3(kBlock), 0, c->stream, s.part, nparts, WS + CO, s.tmpg);
  e = hipGetLastError();
  if (e) return e;
  e = hipMemcpyAsync(grad_w, s.tmpg, WS * 4, hipMemcpyDeviceToDevice, c->stream);
  if (e) return e;
  return hipMemcpyAsync(grad_b, s.tmpg + WS, CO * 4, hipMemcpyDeviceToDevice, c->stream);
}

static hipError_t ensure_grad_scratch(NNState &s) {
  hipError_t e = hipSuccess;
  if (!s.tmpg) {
    if ((e = hipMalloc((void **)&s.tmpg, (W2N + C) * 4))) return e;
    if ((e = hipMalloc((void **)&s.lpart, 1024 * 4))) return e;
  }
  if (!s.wpart) {  // partial weight gradients of the matrix-core path, then the bias partials
    if ((e = hipMalloc((void **)&s.wpart, (size_t)kWgBlocks * (NHT * NVT * 256 + 16) * 4))) return e;
  }
  return e;
}

// Gradients of every parameter into s.g from dL/dy in s.dy (activations of the last forward pass).
static hipError_t nn_backward(hyb_ctx *c, const float *x, int nsamp) {
  NNState &s = c->nn;
  hipError_t e;
  if (!c->p.nn_fp32) {
    if ((e = ensure_grad_scratch(s))) return e;
    return backward_bf16(c, x, nsamp);
  }
  size_t n = (size_t)c->ncell * nsamp;
  dim3 g(nblk(n)), b(kBlock);
  int L = c->nlev, nc = c->ncol;
  // layer 3: dy -> dW3, db3, d(a2) masked by a2 > 0
  if ((e = weight_grad<C, 1>(c, s.dy, s.a2, nsamp, s.g + OFF_W3, s.g + OFF_B3))) return e;
  hipLaunchKernelGGL((k_conv_bwd_data<C, 1, true>), g, b, 0, c->stream, s.dy, s.wb + W1N + W2N, s.a2, s.d2, L, nc,
                     nsamp, s.rv9);
  if ((e = hipGetLastError())) return e;
  // layer 2
  if ((e = weight_grad<C, C>(c, s.d2, s.a1, nsamp, s.g + OFF_W2, s.g + OFF_B2))) return e;
  hipLaunchKernelGGL((k_conv_bwd_data<C, C, true>), g, b, 0, c->stream, s.d2, s.wb + W1N, s.a1, s.d1, L, nc, nsamp,
                     s.rv9);
  if ((e = hipGetLastError())) return e;
  // layer 1 (input x and the static fields)
  return weight_grad<CIN, C, CIN - 1>(c, s.d1, x, nsamp, s.g + OFF_W1, s.g + OFF_B1);
}

// Loss (mean squared error over all cells and samples) and gradients into s.g.
hipError_t nn_loss_grad(hyb_ctx *c, const float *x, const float *target, int nsamp, float *loss_host) {
  NNState &s = c->nn;
  // the activation buffers (s.y among them) must exist at this size before s.y is passed on
  hipError_t e = ensure_acts(c, nsamp);
  if (e) return e;
  if ((e = nn_forward(c, x, s.y, nsamp))) return e;
  if ((e = ensure_grad_scratch(s))) return e;
  size_t n = (size_t)c->ncell * nsamp;
  unsigned nb = std::min<unsigned>(1024, nblk(n));
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kBlock), 0, c->stream, s.y, target, s.dy, n, s.lpart);
  if ((e = hipGetLastError())) return e;
  if ((e = nn_backward(c, x, nsamp))) return e;
  hipLaunchKernelGGL(k_scale_f32, dim3(nblk(NPARAM)), dim3(kBlock), 0, c->stream, s.g, NPARAM, (float)(1.0 / (double)n));
  if ((e = hipGetLastError())) return e;
  if (loss_host) {
    std::vector<float> lp(nb);
    if ((e = hipMemcpyAsync(lp.data(), s.lpart, nb * 4, hipMemcpyDeviceToHost, c->stream))) return e;
    if ((e = hipStreamSynchronize(c->stream))) return e;
    double acc = 0.0;
    for (unsigned i = 0; i < nb; ++i) acc += lp[i];
    *loss_host = (float)(acc / (double)n);
  }
  return hipSuccess;
}

// Energy loss of a batch, (1/nsamp) sum_i (q_i^T G q_i - 2 q_i^T rhat_i) mean(H_diag) / ncell with
// q_i = N(x_i) / H_diag and G = P^T S P, and its gradients into s.g.  x [nsamp][ncell] FP32,
// rhat [nsamp][ncell] FP64.
hipError_t nn_energy_grad(hyb_ctx *c, const float *x, const double *rhat, int nsamp, double *loss_host) {
  NNState &s = c->nn;
  hipError_t e = ensure_acts(c, nsamp);
  if (e) return e;
  if ((e = ensure_grad_scratch(s))) return e;
  const size_t ncell = (size_t)c->ncell, ntr = (size_t)c->ntrace, n = ncell * nsamp;
  if (s.gq_cap < n) {
    if (s.gq) (void)hipFree(s.gq), s.gq = nullptr;
    if ((e = hipMalloc((void **)&s.gq, n * 8))) return e;
    s.gq_cap = n;
  }
  if (!s.d64) {
    if ((e = hipMalloc((void **)&s.d64, ntr * 8)) || (e = hipMalloc((void **)&s.sd64, ntr * 8))) return e;
  }
  const LevelDev &L0 = c->lv[0];
  if (!(s.dbar > 0.0)) {  // mean of the diagonal of H (once)
    std::vector<double> h(ncell);
    if ((e = hipMemcpy(h.data(), L0.H, ncell * 8, hipMemcpyDeviceToHost))) return e;
    double acc = 0.0;
    for (double v : h) acc += v;
    s.dbar = acc / (double)ncell;
  }
  if ((e = nn_forward(c, x, s.y, nsamp))) return e;
  for (int i = 0; i < nsamp; ++i) {
    hipLaunchKernelGGL(k_prolong_q, dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, s.y + (size_t)i * ncell, L0.H, s.d64,
                       c->nlev, c->ncol, c->nedge, (size_t)c->nz, ntr, L0.edge_col);
    if ((e = hipGetLastError())) return e;
    if ((e = launch_trace_apply<double, double, double>(c, c->S, s.d64, nullptr, s.sd64, 0))) return e;
    if ((e = launch_restrict_cells(c, s.sd64, s.gq + (size_t)i * ncell, 3))) return e;
  }
  const double scale = s.dbar / (double)ncell / (double)nsamp;
  unsigned nb = std::min<unsigned>(1024, nblk(n));
  double *part = s.epart;
  if (!part) {
    if ((e = hipMalloc((void **)&s.epart, 1024 * 8))) return e;
    part = s.epart;
  }
  hipLaunchKernelGGL(k_energy, dim3(nb), dim3(kBlock), 0, c->stream, s.y, s.gq, rhat, L0.H, s.dy, ncell, n, part);
  if ((e = hipGetLastError())) return e;
  if ((e = nn_backward(c, x, nsamp))) return e;
  hipLaunchKernelGGL(k_scale_f32, dim3(nblk(NPARAM)), dim3(kBlock), 0, c->stream, s.g, NPARAM, (float)scale);
  if ((e = hipGetLastError())) return e;
  if (loss_host) {
    std::vector<double> lp(nb);
    if ((e = hipMemcpyAsync(lp.data(), part, nb * 8, hipMemcpyDeviceToHost, c->stream))) return e;
    if ((e = hipStreamSynchronize(c->stream))) return e;
    double acc = 0.0;
    for (unsigned i = 0; i < nb; ++i) acc += lp[i];
    *loss_host = acc * scale;
  }
  return hipSuccess;
}

hipError_t nn_adam(hyb_ctx *c, float lr) {
  NNState &s = c->nn;
  s.step++;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)s.step), c2 = 1.f - powf(b2, (float)s.step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAM)), dim3(kBlock), 0, c->stream, s.w, s.m, s.v, s.g, s.wb, s.isbf, NPARAM,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// Buffers of the stage and of the training pairs: network input / output [ncell], scalars, the
// correction and its image [ntrace], a cell field in FP64 (allocated on first use).
hipError_t nn_stage_buffers(hyb_ctx *c) {
  NNState &s = c->nn;
  hipError_t e;
  const size_t n = (size_t)c->ncell, ntr = (size_t)c->ntrace;
  if (!s.cin) {
    if ((e = hipMalloc((void **)&s.cin, n * 4)) || (e = hipMalloc((void **)&s.cout, n * 4)) ||
        (e = hipMalloc((void **)&s.scal, 8 * sizeof(double))))
      return e;
    hipLaunchKernelGGL(k_zero_scal, dim3(1), dim3(64), 0, c->stream, s.scal, 8);
    if ((e = hipGetLastError())) return e;
    c->bytes += n * 8 + 64;
  }
  if (!s.d64) {
    if ((e = hipMalloc((void **)&s.d64, ntr * 8)) || (e = hipMalloc((void **)&s.sd64, ntr * 8))) return e;
    c->bytes += 2 * ntr * 8;
  }
  if (!c->cell64) {
    if ((e = hipMalloc((void **)&c->cell64, n * 8))) return e;
    c->bytes += n * 8;
  }
  return hipSuccess;
}

// The training pair of a residual r' (in c->t64) whose Gamma P^T r' is in c->cell64:
// s = rms(Gamma P^T r'), x = Gamma P^T r' / s (FP32), rhat = P^T r' / s; s to the host.
hipError_t nn_pair_finish(hyb_ctx *c, float *x, double *rhat, double *scale_host) {
  NNState &s = c->nn;
  const size_t n = (size_t)c->ncell;
  const unsigned nb = std::min<unsigned>(1024, nblk(n));
  double *part = c->partial;
  hipLaunchKernelGGL((k_sumsq<double>), dim3(nb), dim3(kBlock), 0, c->stream, c->cell64, n, part);
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(64), 0, c->stream, part, (int)nb, s.scal);
  hipLaunchKernelGGL(k_normalise, dim3(nblk(n)), dim3(kBlock), 0, c->stream, c->cell64, s.scal, x, n);
  hipError_t e = hipGetLastError();
  if (e) return e;
  if ((e = launch_restrict_cells(c, c->t64, rhat, 3))) return e;
  hipLaunchKernelGGL(k_div_rms, dim3(nblk(n)), dim3(kBlock), 0, c->stream, rhat, s.scal, n);
  if ((e = hipGetLastError())) return e;
  double ss = 0.0;
  if ((e = hipMemcpyAsync(&ss, s.scal, sizeof(double), hipMemcpyDeviceToHost, c->stream))) return e;
  if ((e = hipStreamSynchronize(c->stream))) return e;
  *scale_host = std::sqrt(ss / (double)n);
  return hipSuccess;
}

// Gathers pairs idx[0..nsamp) of X [npairs][ncell] (FP32) and R (FP64) into the batch buffers.
hipError_t nn_gather_batch(hyb_ctx *c, const float *X, const double *R, const int32_t *idx, int nsamp) {
  NNState &s = c->nn;
  const size_t n = (size_t)c->ncell, need = n * nsamp;
  hipError_t e;
  if (s.batch_cap < need) {
    if (s.xb) (void)hipFree(s.xb), s.xb = nullptr;
    if (s.rb) (void)hipFree(s.rb), s.rb = nullptr;
    s.batch_cap = 0;
    if ((e = hipMalloc((void **)&s.xb, need * 4)) || (e = hipMalloc((void **)&s.rb, need * 8))) return e;
    c->bytes += need * 12;
    s.batch_cap = need;
  }
  for (int i = 0; i < nsamp; ++i) {
    if ((e = hipMemcpyAsync(s.xb + (size_t)i * n, X + (size_t)idx[i] * n, n * 4, hipMemcpyDeviceToDevice,
                            c->stream)) ||
        (e = hipMemcpyAsync(s.rb + (size_t)i * n, R + (size_t)idx[i] * n, n * 8, hipMemcpyDeviceToDevice,
                            c->stream)))
      return e;
  }
  return hipSuccess;
}

// The learned coarse correction applied after the two-level cycle z = M(r):
//   r' = r - S z,  c = Gamma P^T r',  s = rms(c),  d = s P (N(c / s) / H_diag),
//   z += d  if ||r' - S d|| < ||r'||  (the FP64 residual judges every correction),
// otherwise z stays the plain cycle's output and the fallback counter scal[2] grows (also when the
// network output is not finite).  Everything stays on the device; no host synchronisation.
template <typename Tz>
hipError_t learned_stage(hyb_ctx *c, const double *r, Tz *z, double *Sz) {
  NNState &s = c->nn;
  hipError_t e;
  const size_t n = (size_t)c->ncell, ntr = (size_t)c->ntrace;
  if ((e = nn_stage_buffers(c))) return e;
  int slot = prof_begin(c, F_NN);
  const LevelDev &L0 = c->lv[0];
  if ((e = launch_trace_apply<double, Tz, double>(c, c->S, z, r, c->t64, 1))) return e;
  if ((e = launch_restrict_cells(c, c->t64, c->cell64, 0))) return e;
  unsigned nb = std::min<unsigned>(1024, nblk(n));
  double *part = c->partial;  // Krylov reduction scratch (>= 2 x 1024 doubles)
  hipLaunchKernelGGL((k_sumsq<double>), dim3(nb), dim3(kBlock), 0, c->stream, c->cell64, n, part);
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(64), 0, c->stream, part, (int)nb, s.scal);
  hipLaunchKernelGGL(k_normalise, dim3(nblk(n)), dim3(kBlock), 0, c->stream, c->cell64, s.scal, s.cin, n);
  if ((e = hipGetLastError())) return e;
  if ((e = nn_forward_inference(c, s.cin, s.cout))) return e;
  if (c->p.debug & HYB_DEBUG_NAN_STAGE) {
    hipLaunchKernelGGL(k_fill_nan, dim3(nblk(n)), dim3(kBlock), 0, c->stream, s.cout, n);
    if ((e = hipGetLastError())) return e;
  }
  hipLaunchKernelGGL((k_sumsq<float>), dim3(nb), dim3(kBlock), 0, c->stream, s.cout, n, part);
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(64), 0, c->stream, part, (int)nb, s.scal + 1);
  hipLaunchKernelGGL(k_prolong_correction, dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, s.cout, s.scal, L0.H, s.d64,
                     c->nlev, c->ncol, c->nedge, (size_t)c->nz, ntr, L0.edge_col);
  if ((e = hipGetLastError())) return e;
  if ((e = launch_trace_apply<double, double, double>(c, c->S, s.d64, nullptr, s.sd64, 0))) return e;
  unsigned nbt = std::min<unsigned>(1024, nblk(ntr));
  hipLaunchKernelGGL(k_judge_sums, dim3(nbt), dim3(kBlock), 0, c->stream, c->t64, s.sd64, ntr, part);
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(64), 0, c->stream, part, (int)nbt, s.scal + 3);
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(64), 0, c->stream, part + nbt, (int)nbt, s.scal + 4);
  if (Sz)  // before the apply, which counts a rejected correction in scal[2] (not read here)
    hipLaunchKernelGGL(k_stage_matvec, dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, r, c->t64, s.sd64, s.scal, Sz, ntr,
                       c->p.learned_tau * c->p.learned_tau);
  hipLaunchKernelGGL((k_apply_correction<Tz>), dim3(nblk(ntr)), dim3(kBlock), 0, c->stream, s.d64, s.scal, z, ntr,
                     c->p.learned_tau * c->p.learned_tau);
  prof_end(c, F_NN, slot);
  return hipGetLastError();
}
template hipError_t learned_stage<double>(hyb_ctx *, const double *, double *, double *);
template hipError_t learned_stage<float>(hyb_ctx *, const double *, float *, double *);

void nn_free(hyb_ctx *c) {
  NNState &s = c->nn;
  for (float **p : {&s.w, &s.m, &s.v, &s.g, &s.a1, &s.a2, &s.y, &s.d1, &s.d2, &s.dy, &s.part, &s.tmpg, &s.lpart,
                    &s.cin, &s.cout})
    if (*p) (void)hipFree(*p), *p = nullptr;
  if (s.wb) (void)hipFree(s.wb), s.wb = nullptr;
  if (s.isbf) (void)hipFree(s.isbf), s.isbf = nullptr;
  if (s.nb9) (void)hipFree(s.nb9), s.nb9 = nullptr;
  if (s.rv9) (void)hipFree(s.rv9), s.rv9 = nullptr;
  for (int32_t **p : {&s.rvh, &s.lo_off, &s.lo_list})
    if (*p) (void)hipFree(*p), *p = nullptr;
  if (s.wpart) (void)hipFree(s.wpart), s.wpart = nullptr;
  if (s.st) (void)hipFree(s.st), s.st = nullptr;
  if (s.layer) (void)hipFree(s.layer), s.layer = nullptr;
  s.st_ready = false;
  if (s.scal) (void)hipFree(s.scal), s.scal = nullptr;
  if (s.a1h) (void)hipFree(s.a1h), s.a1h = nullptr;
  if (s.a2h) (void)hipFree(s.a2h), s.a2h = nullptr;
  if (s.d64) (void)hipFree(s.d64), s.d64 = nullptr;
  if (s.sd64) (void)hipFree(s.sd64), s.sd64 = nullptr;
  if (s.gq) (void)hipFree(s.gq), s.gq = nullptr;
  if (s.epart) (void)hipFree(s.epart), s.epart = nullptr;
  if (s.xb) (void)hipFree(s.xb), s.xb = nullptr;
  if (s.rb) (void)hipFree(s.rb), s.rb = nullptr;
  s.batch_cap = 0;
  s.gq_cap = 0;
  s.dbar = 0.0;
  if (c->cell64) (void)hipFree(c->cell64), c->cell64 = nullptr;
  s.cap = 0;
}

}  // namespace hyb
