// Vector kernels of the flexible GMRES outer loop: fused multi-vector dot products with a
// deterministic two-stage reduction (wavefront shuffles, then a fixed-order pass over the
// per-block partial sums), multi-vector updates and precision conversions.
#include "hyb_internal.h"

namespace hyb {

namespace {

constexpr int kChunk = 8;  // dot products accumulated per pass over w
constexpr int kRedBlocks = 1024;

inline unsigned nblk(size_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// partial[blk][k] = sum over this block's entries of a_k . w (k < nv), and w . w at k = nv.
__global__ void __launch_bounds__(kBlock) k_multidot_partial(const double *__restrict__ a, size_t lda, int nv,
                                                             const double *__restrict__ w, size_t n, int nout,
                                                             double *__restrict__ partial, int ldp) {
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
      partial[(size_t)blockIdx.x * ldp + k0 + threadIdx.x] = s;
    }
    __syncthreads();
  }
}

__global__ void k_multidot_final(const double *__restrict__ partial, int ldp, int nb, int nout,
                                 double *__restrict__ out) {
  int k = threadIdx.x;
  if (k >= nout) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(size_t)b * ldp + k];
  out[k] = s;
}

__global__ void k_multi_axpy(const double *__restrict__ a, size_t lda, int nv, const double *__restrict__ h,
                             double *__restrict__ w, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = w[i];
  for (int k = 0; k < nv; ++k) v -= h[k] * a[(size_t)k * lda + i];
  w[i] = v;
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
  int ldp = c->m + 2;
  if (nout > ldp || nout > kBlock) return hipErrorInvalidValue;
  int slot = prof_begin(c, F_KRYLOV);
  unsigned nb = std::min<unsigned>(kRedBlocks, nblk(n));
  hipLaunchKernelGGL(k_multidot_partial, dim3(nb), dim3(kBlock), 0, c->stream, a, lda, nv, w, n, nout, c->partial,
                     ldp);
  hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(kBlock), 0, c->stream, c->partial, ldp, (int)nb, nout, out_dev);
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
