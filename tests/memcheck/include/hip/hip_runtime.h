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
struct uint2 { uint32_t x, y; };
inline uint2 make_uint2(uint32_t x, uint32_t y) { return uint2{x, y}; }
struct uint4 { uint32_t x, y, z, w; };
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
void wave_barrier();  // barrier among the fibers of the current wavefront (64 threads)
void *xchg(unsigned tid);  // 64-byte exchange slot of a thread of the current workgroup
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
#define __align__(n) __attribute__((aligned(n)))
#define __shared__ static
#define __syncthreads() emu::barrier()
#define __builtin_nontemporal_load(p) (*(p))

#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) \
  emu::launch(dim3(G), dim3(B), (size_t)(SH), [&]() { K(__VA_ARGS__); })

template <typename T>
inline T __shfl_down(T v, unsigned off, int width = 64) {
  static_assert(sizeof(T) <= 8, "shfl of a large type");
  const unsigned tid = emu::cur_tid();
  std::memcpy(emu::xchg(tid), &v, sizeof(T));
  emu::wave_barrier();
  unsigned lane = tid % (unsigned)width, src = lane + off;
  T r = v;
  if (src < (unsigned)width) std::memcpy(&r, emu::xchg(tid - lane + src), sizeof(T));
  emu::wave_barrier();
  return r;
}

template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  static_assert(sizeof(T) <= 8, "shfl of a large type");
  const unsigned tid = emu::cur_tid();
  std::memcpy(emu::xchg(tid), &v, sizeof(T));
  emu::wave_barrier();
  const unsigned lane = tid % 64u, seg = lane - lane % (unsigned)width;
  T r;
  std::memcpy(&r, emu::xchg(tid - lane + seg + ((unsigned)src % (unsigned)width)), sizeof(T));
  emu::wave_barrier();
  return r;
}

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  static_assert(sizeof(T) <= 8, "shfl of a large type");
  const unsigned tid = emu::cur_tid();
  std::memcpy(emu::xchg(tid), &v, sizeof(T));
  emu::wave_barrier();
  const unsigned lane = tid % 64u, seg = lane - lane % (unsigned)width;
  const unsigned src = lane ^ (unsigned)mask;
  T r = v;
  if (src >= seg && src < seg + (unsigned)width) std::memcpy(&r, emu::xchg(tid - lane + src), sizeof(T));
  emu::wave_barrier();
  return r;
}

template <typename T>
inline T __shfl_up(T v, unsigned off, int width = 64) {
  static_assert(sizeof(T) <= 8, "shfl of a large type");
  const unsigned tid = emu::cur_tid();
  std::memcpy(emu::xchg(tid), &v, sizeof(T));
  emu::wave_barrier();
  unsigned lane = tid % (unsigned)width;
  T r = v;
  if (lane >= off) std::memcpy(&r, emu::xchg(tid - off), sizeof(T));
  emu::wave_barrier();
  return r;
}

// Matrix-core instructions used by the library, with their lane layouts (wavefront of 64):
// f32 16x16x4: a = A[l%16][l/16], b = B[l/16][l%16]; bf16 16x16x16: a[j] = A[l%16][4(l/16)+j],
// b[j] = B[4(l/16)+j][l%16]; result d[j] = D[4(l/16)+j][l%16].
struct emu_f32x4 {
  float v[4];
  float &operator[](int i) { return v[i]; }
  float operator[](int i) const { return v[i]; }
};
struct emu_bf16x4 {
  short v[4];
  short &operator[](int i) { return v[i]; }
  short operator[](int i) const { return v[i]; }
};
inline float emu_bf16_to_f32(short h) {
  uint32_t u = ((uint32_t)(uint16_t)h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
inline emu_f32x4 emu_mfma_f32_16x16x4f32(float a, float b, emu_f32x4 c, int, int, int) {
  const unsigned tid = emu::cur_tid(), lane = tid % 64, base = tid - lane;
  float ab[2] = {a, b};
  std::memcpy(emu::xchg(tid), ab, 8);
  emu::wave_barrier();
  for (int j = 0; j < 4; ++j) {
    const unsigned row = 4 * (lane / 16) + j, col = lane % 16;
    float acc = 0.f;
    for (unsigned k = 0; k < 4; ++k) {
      float A[2], B[2];
      std::memcpy(A, emu::xchg(base + k * 16 + row), 8);
      std::memcpy(B, emu::xchg(base + k * 16 + col), 8);
      acc += A[0] * B[1];
    }
    c[j] += acc;
  }
  emu::wave_barrier();
  return c;
}
inline emu_f32x4 emu_mfma_f32_16x16x16bf16_1k(emu_bf16x4 a, emu_bf16x4 b, emu_f32x4 c, int, int, int) {
  const unsigned tid = emu::cur_tid(), lane = tid % 64, base = tid - lane;
  short ab[8];
  for (int j = 0; j < 4; ++j) ab[j] = a[j], ab[4 + j] = b[j];
  std::memcpy(emu::xchg(tid), ab, 16);
  emu::wave_barrier();
  for (int j = 0; j < 4; ++j) {
    const unsigned row = 4 * (lane / 16) + j, col = lane % 16;
    float acc = 0.f;
    for (unsigned k = 0; k < 16; ++k) {
      short A[8], B[8];
      std::memcpy(A, emu::xchg(base + (k / 4) * 16 + row), 16);
      std::memcpy(B, emu::xchg(base + (k / 4) * 16 + col), 16);
      acc += emu_bf16_to_f32(A[k % 4]) * emu_bf16_to_f32(B[4 + k % 4]);
    }
    c[j] += acc;
  }
  emu::wave_barrier();
  return c;
}
struct alignas(8) emu_f32x2 {
  float v[2];
  float operator[](int i) const { return v[i]; }
};
// bf16 16x16x32 (gfx950): a[j] = A[l%16][8(l/16)+j], b[j] = B[8(l/16)+j][l%16]; d as above
struct emu_s16x8 {
  short v[8];
  short &operator[](int i) { return v[i]; }
  short operator[](int i) const { return v[i]; }
};
struct emu_u32x4 {
  uint32_t v[4];
  uint32_t &operator[](int i) { return v[i]; }
  uint32_t operator[](int i) const { return v[i]; }
};
inline emu_f32x4 emu_mfma_f32_16x16x32_bf16(emu_s16x8 a, emu_s16x8 b, emu_f32x4 c, int, int, int) {
  const unsigned tid = emu::cur_tid(), lane = tid % 64, base = tid - lane;
  short ab[16];
  for (int j = 0; j < 8; ++j) ab[j] = a[j], ab[8 + j] = b[j];
  std::memcpy(emu::xchg(tid), ab, 32);
  emu::wave_barrier();
  for (int j = 0; j < 4; ++j) {
    const unsigned row = 4 * (lane / 16) + j, col = lane % 16;
    float acc = 0.f;
    for (unsigned k = 0; k < 32; ++k) {
      short A[16], B[16];
      std::memcpy(A, emu::xchg(base + (k / 8) * 16 + row), 32);
      std::memcpy(B, emu::xchg(base + (k / 8) * 16 + col), 32);
      acc += emu_bf16_to_f32(A[k % 8]) * emu_bf16_to_f32(B[8 + k % 8]);
    }
    c[j] += acc;
  }
  emu::wave_barrier();
  return c;
}
#define __builtin_amdgcn_mfma_f32_16x16x4f32 emu_mfma_f32_16x16x4f32
#define __builtin_amdgcn_mfma_f32_16x16x16bf16_1k emu_mfma_f32_16x16x16bf16_1k
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16 emu_mfma_f32_16x16x32_bf16
// a wavefront's fibers meet at a wave barrier; the fences order nothing further on the CPU
#define __builtin_amdgcn_wave_barrier() emu::wave_barrier()
#define __builtin_amdgcn_fence(order, scope) ((void)0)

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
// one device; a device variable is a host static, so its address is its own
inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
#define HIP_SYMBOL(X) ((const void *)&(X))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
  *p = const_cast<void *>(sym);
  return hipSuccess;
}
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipEventCreate(hipEvent_t *e);
#define hipEventDisableTiming 2u
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
template <class F> inline hipError_t hipFuncSetAttribute(F, hipFuncAttribute, int) { return hipSuccess; }
