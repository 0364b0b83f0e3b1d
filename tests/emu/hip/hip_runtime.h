// CPU emulation of the subset of HIP device code that the library's kernel
// headers use, for host-side tests of the kernels' indexing and
// synchronisation (never part of the library): one std::thread per GPU
// thread, __syncthreads as a barrier of the workgroup, and the wave-local
// barrier (__builtin_amdgcn_wave_barrier) as a barrier of the thread's
// 64-thread wave.  Built with ThreadSanitizer, any LDS access that neither
// kind of barrier orders against another thread's access to the same
// element is reported as a data race.
#pragma once
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <barrier>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(...)
#define SG_WAVES_PER_EU(...)
#define __constant__
#define SG_OPAQUE(v) __asm__ volatile("" : "+r"(v))

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct float2 {
  float x, y;
};
struct double2 {
  double x, y;
};
inline float2 make_float2(float a, float b) { return {a, b}; }
inline double2 make_double2(double a, double b) { return {a, b}; }

namespace emu {
struct Block {
  std::unique_ptr<std::barrier<>> all;
  std::vector<std::unique_ptr<std::barrier<>>> waves;
};
inline thread_local dim3 tid, bid;
inline dim3 bdim, gdim;
inline Block* block = nullptr;
}  // namespace emu

#define threadIdx (emu::tid)
#define blockIdx (emu::bid)
#define blockDim (emu::bdim)
#define gridDim (emu::gdim)

inline void __syncthreads() { emu::block->all->arrive_and_wait(); }
inline void __builtin_amdgcn_wave_barrier() { emu::block->waves[emu::tid.x / 64]->arrive_and_wait(); }
#define __builtin_amdgcn_fence(...) ((void)0)
// the kernels apply it to wave-uniform values only
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }

inline void sincospi(double x, double* s, double* c) {
  const long double pi = 3.141592653589793238462643383279502884L;
  *s = (double)sinl(pi * (long double)x);
  *c = (double)cosl(pi * (long double)x);
}

namespace emu {
// Run fn over a grid: blocks one after another, the threads of a block
// concurrently (blockDim.x threads, a multiple of 64).
inline void launch(dim3 grid, dim3 blk, const std::function<void()>& fn) {
  gdim = grid;
  bdim = blk;
  for (unsigned by = 0; by < grid.y; ++by)
    for (unsigned bx = 0; bx < grid.x; ++bx) {
      Block b;
      b.all = std::make_unique<std::barrier<>>((ptrdiff_t)blk.x);
      for (unsigned w = 0; w < (blk.x + 63) / 64; ++w) b.waves.push_back(std::make_unique<std::barrier<>>(64));
      block = &b;
      std::vector<std::thread> th;
      th.reserve(blk.x);
      for (unsigned t = 0; t < blk.x; ++t)
        th.emplace_back([&, t, bx, by] {
          tid = dim3(t, 0, 0);
          bid = dim3(bx, by, 0);
          fn();
        });
      for (auto& x : th) x.join();
      block = nullptr;
    }
}
}  // namespace emu

typedef int hipError_t;
typedef void* hipStream_t;
