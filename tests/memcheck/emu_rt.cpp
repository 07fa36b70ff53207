// Fiber scheduler and host API of the CPU stand-in for the HIP runtime (test harness only).
// Fibers switch with a minimal x86-64 context switch (callee-saved registers, MXCSR and the x87
// control word) and tell AddressSanitizer about every stack switch.
#include "hip/hip_runtime.h"
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" void emu_switch(void **save_sp, void *new_sp);
asm(R"(
.text
.globl emu_switch
.type emu_switch,@function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  subq $8, %rsp
  stmxcsr (%rsp)
  fnstcw 4(%rsp)
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  ldmxcsr (%rsp)
  fldcw 4(%rsp)
  addq $8, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size emu_switch, .-emu_switch
)");

namespace emu {
dim3 threadIdx_, blockIdx_, blockDim_, gridDim_;

namespace {
constexpr size_t kStack = 256 * 1024;
enum State { READY, WAIT, WAVE_WAIT, DONE };
struct Fiber {
  void *sp = nullptr;
  char *stack = nullptr;
  void *fake = nullptr;
  State st = READY;
  unsigned tid = 0;
  alignas(16) unsigned char xchg[64];
};
std::vector<Fiber> fibers;
Fiber *cur = nullptr;
void *main_sp = nullptr;
void *main_fake = nullptr;
const void *main_bottom = nullptr;
size_t main_size = 0;
const std::function<void()> *body = nullptr;
std::vector<unsigned char> dyn;
size_t launches = 0;

void to_main(bool dying) {
  Fiber *f = cur;
  __sanitizer_start_switch_fiber(dying ? nullptr : &f->fake, main_bottom, main_size);
  emu_switch(&f->sp, main_sp);
  __sanitizer_finish_switch_fiber(f->fake, nullptr, nullptr);
}

void entry() {
  __sanitizer_finish_switch_fiber(nullptr, &main_bottom, &main_size);
  (*body)();
  cur->st = DONE;
  to_main(true);
  std::abort();
}

void init_fiber(Fiber &f, unsigned tid) {
  if (!f.stack) {
    f.stack = (char *)mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (f.stack == MAP_FAILED) { std::perror("mmap"); std::abort(); }
  }
  __asan_unpoison_memory_region(f.stack, kStack);
  uintptr_t top = ((uintptr_t)(f.stack + kStack - 64)) & ~(uintptr_t)15;
  // [csr][r15][r14][r13][r12][rbx][rbp][ret = entry][pad]; top is 16-aligned, so p = 8 (mod 16) and
  // after the final ret rsp = 8 (mod 16), as at the entry of any function
  uint64_t *p = (uint64_t *)(top - 8 * 9);
  uint32_t csr[2] = {0x1F80, 0x037F};
  std::memcpy(&p[0], csr, 8);
  for (int i = 1; i <= 6; ++i) p[i] = 0;
  p[7] = (uint64_t)(uintptr_t)&entry;
  p[8] = 0;
  f.sp = p;
  f.st = READY;
  f.tid = tid;
  f.fake = nullptr;
}
}  // namespace

void barrier() {
  if (!cur) { std::fprintf(stderr, "barrier outside a kernel\n"); std::abort(); }
  cur->st = WAIT;
  to_main(false);
}
void wave_barrier() {
  if (!cur) { std::fprintf(stderr, "wavefront barrier outside a kernel\n"); std::abort(); }
  cur->st = WAVE_WAIT;
  to_main(false);
}
unsigned char *dyn_smem() { return dyn.data(); }
void *xchg(unsigned tid) { return fibers[tid].xchg; }
unsigned cur_tid() { return cur->tid; }

void launch(dim3 g, dim3 b, size_t shm, const std::function<void()> &k) {
  ++launches;
  unsigned nt = b.x * b.y * b.z;
  if (nt == 0 || nt > 1024 || g.x == 0 || g.y == 0 || g.z == 0 || g.y > 65535 || g.z > 65535) {
    std::fprintf(stderr, "EMU: bad launch grid (%u,%u,%u) block (%u,%u,%u)\n", g.x, g.y, g.z, b.x, b.y, b.z);
    std::abort();
  }
  if (fibers.size() < nt) fibers.resize(nt);
  dyn.assign(shm + 16, 0xCD);
  body = &k;
  gridDim_ = g;
  blockDim_ = b;
  for (unsigned bz = 0; bz < g.z; ++bz)
    for (unsigned by = 0; by < g.y; ++by)
      for (unsigned bx = 0; bx < g.x; ++bx) {
        blockIdx_ = dim3(bx, by, bz);
        for (unsigned t = 0; t < nt; ++t) init_fiber(fibers[t], t);
        for (;;) {
          for (unsigned t = 0; t < nt; ++t) {
            Fiber &f = fibers[t];
            if (f.st != READY) continue;
            cur = &f;
            threadIdx_ = dim3(t % b.x, (t / b.x) % b.y, t / (b.x * b.y));
            __sanitizer_start_switch_fiber(&main_fake, f.stack, kStack);
            emu_switch(&main_sp, f.sp);
            __sanitizer_finish_switch_fiber(main_fake, nullptr, nullptr);
          }
          cur = nullptr;
          // a wavefront whose live threads all wait at a wavefront barrier goes on first; then a
          // workgroup barrier once every live thread waits at one
          bool released = false;
          for (unsigned w0 = 0; w0 < nt; w0 += 64) {
            unsigned live = 0, wwait = 0;
            for (unsigned t = w0; t < nt && t < w0 + 64; ++t)
              if (fibers[t].st != DONE) ++live, wwait += fibers[t].st == WAVE_WAIT;
            if (live && wwait == live) {
              for (unsigned t = w0; t < nt && t < w0 + 64; ++t) fibers[t].st = READY;
              released = true;
            }
          }
          if (released) continue;
          unsigned live = 0, waiting = 0;
          for (unsigned t = 0; t < nt; ++t)
            if (fibers[t].st != DONE) ++live, waiting += fibers[t].st == WAIT;
          if (!live) break;
          if (waiting != live) {
            std::fprintf(stderr, "EMU: threads of a workgroup wait at different barriers (kernel launch %zu)\n",
                         launches);
            std::abort();
          }
          for (unsigned t = 0; t < nt; ++t) fibers[t].st = READY;
        }
      }
}
}  // namespace emu

hipError_t hipMalloc(void **p, size_t n) {
  *p = std::malloc(n ? n : 1);
  if (!*p) return hipErrorOutOfMemory;
  std::memset(*p, 0xA5, n);  // device memory starts with garbage
  return hipSuccess;
}
hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { *p = std::malloc(n ? n : 1); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void *p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
struct Ev { std::chrono::steady_clock::time_point t; };
hipError_t hipEventCreate(hipEvent_t *e) { *e = new Ev(); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { ((Ev *)e)->t = std::chrono::steady_clock::now(); return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(((Ev *)b)->t - ((Ev *)a)->t).count();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) { delete (Ev *)e; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = new Ev(); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }  // kernels run at launch
extern "C" size_t emu_launch_count() { return emu::launches; }
