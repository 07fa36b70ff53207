// Test harness only: a CPU stand-in for the part of the HIP runtime the library uses, so that the
// library's own sources (host logic and kernels) can be built with g++ and AddressSanitizer and
// their memory accesses checked on the CPU.  Each thread of a workgroup runs as a fiber; workgroups
// run one after another; __syncthreads and wavefront shuffles are barriers among the fibers of the
// workgroup; device memory is heap memory filled with garbage.  Nothing here is used by the product.
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>
#include <algorithm>
#include <type_traits>

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3() = default;
  dim3(unsigned a, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
typedef enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2,
                          hipErrorIllegalAddress = 700 } hipError_t;
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
                     hipMemcpyDefault };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
#define hipHostMallocDefault 0

namespace emu {
extern dim3 threadIdx_, blockIdx_, blockDim_, gridDim_;
void launch(dim3 g, dim3 b, size_t shm, const std::function<void()> &body);
void barrier();
unsigned char *dyn_smem();
void *xchg_slot();  // 8-byte exchange slot of the current thread
void *xchg_slot_of(unsigned tid);
unsigned cur_tid();
}  // namespace emu
#define threadIdx emu::threadIdx_
#define blockIdx emu::blockIdx_
#define blockDim emu::blockDim_
#define gridDim emu::gridDim_

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __constant__
#define __shared__ static
#define __syncthreads() emu::barrier()

#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) \
  emu::launch(dim3(G), dim3(B), (size_t)(SH), [&]() { K(__VA_ARGS__); })

template <typename T>
inline T __shfl_down(T v, unsigned off, int width = 64) {
  static_assert(sizeof(T) <= 8, "shfl of a large type");
  std::memcpy(emu::xchg_slot(), &v, sizeof(T));
  emu::barrier();
  unsigned tid = emu::cur_tid();
  unsigned lane = tid % (unsigned)width, src = lane + off;
  T r = v;
  if (src < (unsigned)width) std::memcpy(&r, emu::xchg_slot_of(tid - lane + src), sizeof(T));
  emu::barrier();
  return r;
}
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
template <class A, class B> inline auto min(A a, B b) -> typename std::common_type<A, B>::type { return a < b ? a : b; }
template <class A, class B> inline auto max(A a, B b) -> typename std::common_type<A, B>::type { return a < b ? b : a; }
using std::isfinite;
using std::sqrt;
using std::fabs;

hipError_t hipMalloc(void **p, size_t n);
template <class T> inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc((void **)p, n); }
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags = 0);
template <class T> inline hipError_t hipHostMalloc(T **p, size_t n, unsigned flags = 0) { return hipHostMalloc((void **)p, n, flags); }
hipError_t hipHostFree(void *p);
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
template <class F> inline hipError_t hipFuncSetAttribute(F, hipFuncAttribute, int) { return hipSuccess; }
