// Device helpers shared by the kernel sources: elements per thread,
// workgroup-to-tile mapping, batch descriptors.
#pragma once
#include <hip/hip_runtime.h>

#include "sg_internal.h"

// Hides a value from the optimiser: loads at an index passed through it are
// issued where they are written instead of being merged with earlier loads
// of the same addresses (which would keep those values live in registers in
// between).
#ifndef SG_OPAQUE
#define SG_OPAQUE(v) __asm__ volatile("" : "+v"(v))
#endif

// Minimum waves per SIMD a kernel's register allocation must allow.
#ifndef SG_WAVES_PER_EU
#define SG_WAVES_PER_EU(...) __attribute__((amdgpu_waves_per_eu(__VA_ARGS__)))
#endif

namespace sg {

__device__ __forceinline__ int opaque(int i) {
  SG_OPAQUE(i);
  return i;
}

// Elements per thread for a transform of length L: E0 (a power of two) for
// L = 2^a, E3 (a multiple of 3) for L = 3 * 2^a, never more than L.
__host__ __device__ constexpr int elems_for(int L, int E0, int E3) {
  return (L % 3 == 0) ? (E3 < L ? E3 : L) : (E0 < L ? E0 : L);
}
// Largest power of two that divides v, capped at cap (a power of two).
__host__ __device__ constexpr int pow2_div(int v, int cap) {
  return (v % 2 == 0 && cap > 1) ? 2 * pow2_div(v / 2, cap / 2) : 1;
}

// Map the launch index to a tile so that consecutive tiles land on the same
// XCD (workgroups are dealt round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

// The batch descriptor of grid blockIdx.y, read through the constant address
// space: pointers loaded from constant memory are taken to be global, so
// accesses through them compile to global instructions rather than flat ones
// (flat accesses also count on the LDS wait counter, so every LDS wait would
// wait for them too).  All of the library's buffers are device memory.
__device__ __forceinline__ sg_bgrid grid_desc(const sg_bgrid* bg) {
  using K = const __attribute__((address_space(4))) sg_bgrid;
  const K* k = (const K*)bg + blockIdx.y;
  sg_bgrid d;
  d.off = k->off;
  d.X = k->X;
  d.V = k->V;
  d.tabx = k->tabx;
  d.taby = k->taby;
  return d;
}

}  // namespace sg
