// Vector kernels of the flexible GMRES outer loop: fused multi-vector dot products with a
// deterministic two-stage reduction (wavefront shuffles, then a fixed-order pass over the
// per-block partial sums), multi-vector updates and precision conversions.
#include "hyb_internal.h"

namespace hyb {

namespace {

constexpr int kChunk = 8;  // dot products accumulated per pass over w
constexpr int kRedBlocks = 2048;
constexpr int kDgsStage = 1;  // kBlock-entry chunks staged per reduction step (swept 1, 2, 4 with 1024-8192 blocks)

inline unsigned nblk(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// partial[k][blk] = sum over this block's entries of a_k . w (k < nv), and w . w at k = nv.
__global__ void __launch_bounds__(kBlock) k_multidot_partial(const double *__restrict__ a, size_t lda, int nv,
                                                             const double *__restrict__ w, size_t n, int nout,
                                                             double *__restrict__ partial) {
  __shared__ double red[kBlock / 64][kChunk];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int k0 = 0; k0 < nout; k0 += kChunk) {
    double acc[kChunk];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) acc[j] = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
      double wi = w[i];
#pragma unroll
      for (int j = 0; j < kChunk; ++j) {
        int k = k0 + j;
        if (k < nv)
          acc[j] += a[(size_t)k * lda + i] * wi;
        else if (k < nout)
          acc[j] += wi * wi;
      }
    }
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      double v = wave_sum(acc[j]);
      if (lane == 0) red[wv][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kChunk && k0 + (int)threadIdx.x < nout) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kBlock / 64; ++q) s += red[q][threadIdx.x];
      partial[(size_t)(k0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[k] = sum over blocks of partial[k][*]: one workgroup per output, fixed summation order.
__global__ void __launch_bounds__(kBlock) k_multidot_final(const double *__restrict__ partial, int nb,
                                                           double *__restrict__ out) {
  __shared__ double red[kBlock / 64];
  int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[(size_t)k * nb + b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) t += red[q];
    out[k] = t;
  }
}

__global__ void k_multi_axpy(const double *__restrict__ a, size_t lda, int nv, const double *__restrict__ h,
                             double *__restrict__ w, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = w[i];
  for (int k = 0; k < nv; ++k) v -= h[k] * a[(size_t)k * lda + i];
  w[i] = v;
}

// w -= sum_k h[k] a_k and partial[blk] = sum over the block of the updated w^2.
__global__ void __launch_bounds__(kBlock) k_axpy_norm(const double *__restrict__ a, size_t lda, int nv,
                                                      const double *__restrict__ h, double *__restrict__ w,
                                                      size_t n, double *__restrict__ partial) {
  __shared__ double red[kBlock / 64];
  size_t stride = (size_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v = w[i];
    for (int k = 0; k < nv; ++k) v -= h[k] * a[(size_t)k * lda + i];
    w[i] = v;
    acc += v * v;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) t += red[q];
    partial[blockIdx.x] = t;
  }
}

// Fused Gram-Schmidt passes for up to NV basis vectors (registers hold one value of each).
// Block reductions write partial[k][blk]; k_multidot_final sums them in a fixed order.
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV + 1], int nout, double *partial) {
  __shared__ double red[kBlock / 64][NV + 1];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= NV; ++k) {
    if (k < nout) {
      double v = wave_sum(acc[k]);
      if (lane == 0) red[wv][k] = v;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nout; k += blockDim.x) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) t += red[q][k];
    partial[(size_t)k * gridDim.x + blockIdx.x] = t;
  }
}

// pass 1: h1_k = a_k . w for k < nv (w read once)
template <int NV>
__global__ void __launch_bounds__(kBlock) k_gs_dots(const double *__restrict__ a, size_t lda, int nv,
                                                    const double *__restrict__ w, size_t n,
                                                    double *__restrict__ partial) {
  double acc[NV + 1];
#pragma unroll
  for (int k = 0; k <= NV; ++k) acc[k] = 0.0;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) acc[k] += a[(size_t)k * lda + i] * wi;
  }
  block_reduce_store<NV>(acc, nv, partial);
}

// pass 2: w <- w - sum_k h1_k a_k, then h2_k = a_k . w and ||w||^2 (index nv) of the updated w
template <int NV>
__global__ void __launch_bounds__(kBlock) k_gs_update_dots(const double *__restrict__ a, size_t lda, int nv,
                                                           const double *__restrict__ h1, double *__restrict__ w,
                                                           size_t n, double *__restrict__ partial) {
  double acc[NV + 1], hk[NV];
#pragma unroll
  for (int k = 0; k <= NV; ++k) acc[k] = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) hk[k] = (k < nv) ? h1[k] : 0.0;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double av[NV];
    double v = w[i];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      av[k] = (k < nv) ? a[(size_t)k * lda + i] : 0.0;
      v -= hk[k] * av[k];
    }
    w[i] = v;
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += av[k] * v;
    acc[NV] += v * v;
  }
  // move the norm into slot nv so that the outputs are contiguous
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if (k == nv) acc[k] = acc[NV];
  block_reduce_store<NV>(acc, nv + 1, partial);
}

// pass 3: w <- (w - sum_k h2_k a_k) * s
template <int NV>
__global__ void __launch_bounds__(kBlock) k_gs_update_scale(const double *__restrict__ a, size_t lda, int nv,
                                                            const double *__restrict__ h2, double *__restrict__ w,
                                                            size_t n, double s) {
  double hk[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) hk[k] = (k < nv) ? h2[k] : 0.0;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = w[i];
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if (k < nv) v -= hk[k] * a[(size_t)k * lda + i];
  w[i] = v * s;
}

// Gram-Schmidt with delayed reorthogonalisation: one reduction pass and one update pass over the
// basis per step.  u = a_j was orthogonalised once in the previous step; w = a_{j+1} is the new
// vector.  Outputs (in partial, then summed): a_k . u for k <= j at [k], a_k . w for k <= j at
// [j + 1 + k], and w . w at [2 j + 2].  A workgroup stages kDgsStage x 256 entries of u and w in LDS; its
// waves split the basis vectors (wave q takes k = q, q + 4, ...) and each runs over all of them, so
// every vector entry is loaded once and a thread keeps at most 2 KW accumulators.
template <int KW, int NW>
__global__ void __launch_bounds__(NW * 64) k_dgs_dots(const double *__restrict__ a, size_t lda, int j, size_t n,
                                                      double *__restrict__ partial) {
  constexpr int NT = NW * 64, RS = kDgsStage, NE = RS * NT;  // entries staged per step
  __shared__ double su[NE], sw[NE], red[NW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double au[KW], aw[KW], ww = 0.0;
#pragma unroll
  for (int q = 0; q < KW; ++q) au[q] = aw[q] = 0.0;
  const double *u = a + (size_t)j * lda, *w = a + (size_t)(j + 1) * lda;
  const size_t stride = (size_t)gridDim.x * NE;
  for (size_t base = (size_t)blockIdx.x * NE; base < n; base += stride) {
    double ur[RS], wr[RS];
#pragma unroll
    for (int q = 0; q < RS; ++q) {
      const size_t i = base + q * NT + threadIdx.x;
      ur[q] = i < n ? u[i] : 0.0, wr[q] = i < n ? w[i] : 0.0;
      ww += wr[q] * wr[q];
    }
    __syncthreads();  // the previous entries are no longer read
#pragma unroll
    for (int q = 0; q < RS; ++q) su[q * NT + threadIdx.x] = ur[q], sw[q * NT + threadIdx.x] = wr[q];
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NE / 64; ++g) {
      const size_t ii = base + 64 * g + lane;
      const double us = su[64 * g + lane], ws = sw[64 * g + lane];
#pragma unroll
      for (int q = 0; q < KW; ++q) {
        const int k = wv + NW * q;
        if (k < j) {
          const double v = ii < n ? __builtin_nontemporal_load(&a[(size_t)k * lda + ii]) : 0.0;  // streamed
          au[q] += v * us;
          aw[q] += v * ws;
        } else if (k == j) {
          au[q] += us * us;
          aw[q] += us * ws;
        }
      }
    }
  }
  const size_t nb = gridDim.x;
#pragma unroll
  for (int q = 0; q < KW; ++q) {
    const int k = wv + NW * q;
    if (k <= j) {
      const double x = wave_sum(au[q]), y = wave_sum(aw[q]);
      if (lane == 0) partial[(size_t)k * nb + blockIdx.x] = x, partial[(size_t)(j + 1 + k) * nb + blockIdx.x] = y;
    }
  }
  const double z = wave_sum(ww);
  if (lane == 0) red[wv] = z;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) t += red[q];
    partial[(size_t)(2 * j + 2) * nb + blockIdx.x] = t;
  }
}

// Coefficients of delayed Gram-Schmidt step j from its 2 j + 3 dot products d: with a_k = V_k . V_j
// and b_k = V_k . V_{j+1} (k < j), rho^2 = V_j . V_j - sum a_k^2 is the squared norm of V_j after its
// second orthogonalisation, hjj = (V_j . V_{j+1} - sum a_k b_k) / rho, and
// eta^2 = V_{j+1} . V_{j+1} - sum b_k^2 - hjj^2 that of V_{j+1} after its first.
// out: [0, j) a, [j, 2 j) b, then rho, hjj, eta, a breakdown flag (rho^2 not positive or not
// finite), 1 / rho and 1 / eta (0 where eta is 0).  One wavefront (j < 64): lane k loads a_k and
// b_k, the three sums are fixed-order shuffle trees; the host reads the values back for the
// Hessenberg matrix.
__global__ void __launch_bounds__(64) k_dgs_coef(const double *__restrict__ d, int j, double *__restrict__ out) {
  const int l = threadIdx.x;
  double a = 0.0, b = 0.0;
  if (l < j) {
    a = d[l];
    b = d[j + 1 + l];
    out[l] = a;
    out[j + l] = b;
  }
  const double a2 = wave_sum(a * a), ab = wave_sum(a * b), b2 = wave_sum(b * b);
  if (l != 0) return;
  const double rho2 = d[j] - a2;
  const bool bad = !(rho2 > 0.0) || !isfinite(rho2);
  const double rho = bad ? 0.0 : sqrt(rho2);
  const double hjj = bad ? 0.0 : (d[2 * j + 1] - ab) / rho;
  const double eta2 = d[2 * j + 2] - b2 - hjj * hjj;
  const double eta = (!bad && eta2 > 0.0 && isfinite(eta2)) ? sqrt(eta2) : 0.0;
  out[2 * j] = rho;
  out[2 * j + 1] = hjj;
  out[2 * j + 2] = eta;
  out[2 * j + 3] = bad ? 1.0 : 0.0;
  out[2 * j + 4] = bad ? 0.0 : 1.0 / rho;
  out[2 * j + 5] = eta > 0.0 ? 1.0 / eta : 0.0;
}

// The update pass: a_j <- (u - sum_{k<j} ca_k a_k) / rho (the reorthogonalised, normalised u) and
// a_{j+1} <- (w - sum_{k<j} cb_k a_k - hjj a_j) / eta (w orthogonalised once and scaled), with the
// coefficients cf written by k_dgs_coef; nothing is written after a breakdown.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_dgs_update(double *__restrict__ a, size_t lda, int j,
                                                       const double *__restrict__ cf, size_t n,
                                                       float *__restrict__ wf) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || cf[2 * j + 3] != 0.0) return;
  double su = 0.0, sw = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k)
    if (k < j) {
      const double v = __builtin_nontemporal_load(&a[(size_t)k * lda + i]);  // streamed
      su += cf[k] * v;
      sw += cf[j + k] * v;
    }
  double *u = a + (size_t)j * lda, *w = a + (size_t)(j + 1) * lda;
  const double vj = (u[i] - su) * cf[2 * j + 4];
  u[i] = vj;
  const double wn = (w[i] - sw - cf[2 * j + 1] * vj) * cf[2 * j + 5];
  w[i] = wn;
  if (wf) wf[i] = (float)wn;  // the FP32 input of the next preconditioner application (mixed form)
}

template <typename Tz>
__global__ void k_update_solution(const Tz *__restrict__ Z, size_t ldz, int nv, const double *__restrict__ y,
                                  double *__restrict__ x, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = x[i];
  for (int k = 0; k < nv; ++k) v += y[k] * (double)Z[(size_t)k * ldz + i];
  x[i] = v;
}

__global__ void k_scale(double *w, size_t n, double s) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] *= s;
}

__global__ void k_narrow(const double *__restrict__ s, float *__restrict__ d, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

__global__ void k_widen(const float *__restrict__ s, double *__restrict__ d, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (double)s[i];
}

}  // namespace

int reduction_blocks() { return kRedBlocks; }

hipError_t launch_multidot(hyb_ctx *c, const double *a, size_t lda, int nv, const double *w, size_t n,
                           double *out_dev, bool with_norm) {
  int nout = nv + (with_norm ? 1 : 0);
  if (nout > c->m + 2) return hipErrorInvalidValue;
  int slot = prof_begin(c, F_KRYLOV);
  unsigned nb = std::min<unsigned>(kRedBlocks, nblk(n));
  hipLaunchKernelGGL(k_multidot_partial, dim3(nb), dim3(kBlock), 0, c->stream, a, lda, nv, w, n, nout, c->partial);
  hipLaunchKernelGGL(k_multidot_final, dim3(nout), dim3(kBlock), 0, c->stream, c->partial, (int)nb, out_dev);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

hipError_t launch_multi_axpy_dev(hyb_ctx *c, const double *a, size_t lda, int nv, const double *h_dev, double *w,
                                 size_t n) {
  int slot = prof_begin(c, F_KRYLOV);
  hipLaunchKernelGGL(k_multi_axpy, dim3(nblk(n)), dim3(kBlock), 0, c->stream, a, lda, nv, h_dev, w, n);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

hipError_t launch_axpy_norm(hyb_ctx *c, const double *a, size_t lda, int nv, const double *h_dev, double *w,
                            size_t n, double *nrm_dev) {
  int slot = prof_begin(c, F_KRYLOV);
  unsigned nb = std::min<unsigned>(kRedBlocks, nblk(n));
  hipLaunchKernelGGL(k_axpy_norm, dim3(nb), dim3(kBlock), 0, c->stream, a, lda, nv, h_dev, w, n, c->partial);
  hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(kBlock), 0, c->stream, c->partial, (int)nb, nrm_dev);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

template <int NV>
hipError_t gs_passes_nv(hyb_ctx *c, const double *V, size_t lda, size_t n, int nv, double *w, double *h1,
                        double *h2n) {
  unsigned nb = std::min<unsigned>(kRedBlocks, nblk(n));
  hipLaunchKernelGGL((k_gs_dots<NV>), dim3(nb), dim3(kBlock), 0, c->stream, V, lda, nv, w, n, c->partial);
  hipLaunchKernelGGL(k_multidot_final, dim3(nv), dim3(kBlock), 0, c->stream, c->partial, (int)nb, h1);
  hipLaunchKernelGGL((k_gs_update_dots<NV>), dim3(nb), dim3(kBlock), 0, c->stream, V, lda, nv, (const double *)h1, w,
                     n, c->partial);
  hipLaunchKernelGGL(k_multidot_final, dim3(nv + 1), dim3(kBlock), 0, c->stream, c->partial, (int)nb, h2n);
  return hipGetLastError();
}

// Classical Gram-Schmidt with reorthogonalisation against the nv orthonormal rows of V (stride n):
// h1 = V w; w -= V^T h1; h2 = V w; ||w||^2 -> h2n[nv]; the final update and normalisation is
// launch_gs_finish once the host knows the norm.
hipError_t launch_gs_passes(hyb_ctx *c, const double *V, size_t lda, size_t n, int nv, double *w, double *h1,
                            double *h2n) {
  if (nv < 1 || nv > 32 || nv + 1 > c->m + 2) return hipErrorInvalidValue;
  int slot = prof_begin(c, F_KRYLOV);
  hipError_t e;
  if (nv <= 8)
    e = gs_passes_nv<8>(c, V, lda, n, nv, w, h1, h2n);
  else if (nv <= 16)
    e = gs_passes_nv<16>(c, V, lda, n, nv, w, h1, h2n);
  else
    e = gs_passes_nv<32>(c, V, lda, n, nv, w, h1, h2n);
  prof_end(c, F_KRYLOV, slot);
  return e;
}

hipError_t launch_gs_finish(hyb_ctx *c, const double *V, size_t lda, size_t n, int nv, const double *h2, double *w,
                            double s) {
  if (nv < 1 || nv > 32) return hipErrorInvalidValue;
  int slot = prof_begin(c, F_KRYLOV);
  if (nv <= 8)
    hipLaunchKernelGGL((k_gs_update_scale<8>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, V, lda, nv, h2, w, n, s);
  else if (nv <= 16)
    hipLaunchKernelGGL((k_gs_update_scale<16>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, V, lda, nv, h2, w, n, s);
  else
    hipLaunchKernelGGL((k_gs_update_scale<32>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, V, lda, nv, h2, w, n, s);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

hipError_t launch_dgs_dots(hyb_ctx *c, const double *V, size_t lda, size_t n, int j, double *out_dev) {
  if (j < 0 || j >= kDgsMax || 2 * j + 3 > 2 * (c->m + 2)) return hipErrorInvalidValue;
  int slot = prof_begin(c, F_KRYLOV);
  // the j + 1 vectors a_0..a_j split over the waves of a workgroup, exactly as many accumulator
  // slots as needed (spare slots cost registers and occupancy): four waves up to j = 15, eight
  // beyond (five slots on four waves ran at 3.4 TB/s against 5.3 for four)
  // eight-wave workgroups run best at half as many workgroups (j = 17: 362 us against 375, j = 20:
  // 386 against 458)
  const int nw = j < 16 ? 4 : 8;
  const unsigned nb = std::min<unsigned>(nw == 4 ? kRedBlocks : kRedBlocks / 2, nblk(n, kDgsStage * 64 * nw));
  const int kw = (j + nw) / nw;
  switch (nw * 16 + kw) {
#define HYB_DGS_CASE(W, K)                                                                                   \
  case W * 16 + K:                                                                                           \
    hipLaunchKernelGGL((k_dgs_dots<K, W>), dim3(nb), dim3(64 * W), 0, c->stream, V, lda, j, n, c->partial); \
    break;
    HYB_DGS_CASE(4, 1) HYB_DGS_CASE(4, 2) HYB_DGS_CASE(4, 3) HYB_DGS_CASE(4, 4)
    HYB_DGS_CASE(8, 3) HYB_DGS_CASE(8, 4)
#undef HYB_DGS_CASE
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_multidot_final, dim3(2 * j + 3), dim3(kBlock), 0, c->stream, c->partial, (int)nb, out_dev);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

hipError_t launch_dgs_coef(hyb_ctx *c, const double *dots, int j, double *coef) {
  if (j < 0 || j >= kDgsMax) return hipErrorInvalidValue;
  int slot = prof_begin(c, F_KRYLOV);
  hipLaunchKernelGGL(k_dgs_coef, dim3(1), dim3(64), 0, c->stream, dots, j, coef);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

hipError_t launch_dgs_update(hyb_ctx *c, double *V, size_t lda, size_t n, int j, const double *coef, float *wf) {
  if (j < 0 || j >= kDgsMax) return hipErrorInvalidValue;
  int slot = prof_begin(c, F_KRYLOV);
  if (j < 8)
    hipLaunchKernelGGL((k_dgs_update<8>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, V, lda, j, coef, n, wf);
  else if (j < 16)
    hipLaunchKernelGGL((k_dgs_update<16>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, V, lda, j, coef, n, wf);
  else
    hipLaunchKernelGGL((k_dgs_update<32>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, V, lda, j, coef, n, wf);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

template <typename Tz>
hipError_t launch_update_solution(hyb_ctx *c, const Tz *Z, size_t ldz, int nv, const double *y_dev, double *x,
                                  size_t n) {
  int slot = prof_begin(c, F_KRYLOV);
  hipLaunchKernelGGL((k_update_solution<Tz>), dim3(nblk(n)), dim3(kBlock), 0, c->stream, Z, ldz, nv, y_dev, x, n);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}
template hipError_t launch_update_solution<double>(hyb_ctx *, const double *, size_t, int, const double *, double *,
                                                   size_t);
template hipError_t launch_update_solution<float>(hyb_ctx *, const float *, size_t, int, const double *, double *,
                                                  size_t);

hipError_t launch_scale(hyb_ctx *c, double *w, size_t n, double s) {
  int slot = prof_begin(c, F_KRYLOV);
  hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(kBlock), 0, c->stream, w, n, s);
  prof_end(c, F_KRYLOV, slot);
  return hipGetLastError();
}

hipError_t launch_convert(hyb_ctx *c, const double *src, float *dst, size_t n) {
  hipLaunchKernelGGL(k_narrow, dim3(nblk(n)), dim3(kBlock), 0, c->stream, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_copy_widen(hyb_ctx *c, const float *src, double *dst, size_t n) {
  hipLaunchKernelGGL(k_widen, dim3(nblk(n)), dim3(kBlock), 0, c->stream, src, dst, n);
  return hipGetLastError();
}

}  // namespace hyb
