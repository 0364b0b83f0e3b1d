// Four-step workgroup FFT for long columns (gfx950, wave64), FP32 and FP64.
//
// A length-N transform is spread over T = N / E threads (T a multiple of
// 64), E elements each, as N = B1 * B2 with input index n = n1 + B1 n2 and
// output index k = k2 + B2 k1:
//   step 1: B1 transforms of length B2 over n2 (one per n1),
//   step 2: the twiddle w_N^(n1 k2),
//   step 3: B2 transforms of length B1 over n1 (one per k2).
// Each step-1 or step-3 transform (length B = E * LB) runs on LB lanes of one
// wave: an E-point DFT in registers, a transpose among the LB lanes through
// the wave's own LDS region, the twiddle w_B, and E / LB DFTs of length LB
// in registers.  The transposes inside a wave need no workgroup barrier;
// only the exchange between steps 1 and 3 crosses waves.  Compared with a
// radix-E Stockham transform (log_E N stages, each ending in a workgroup
// barrier) the arithmetic and LDS traffic are the same and the barriers drop
// to one per transform (shared by every array exchanged together).
//
// The inverse runs the same steps backwards and takes its input in the
// forward's output order, so a pointwise product between the two needs no
// data movement.  Twiddles come from tables built in FP64 (long double on
// the host) and rounded once; nothing is accumulated by recurrence.
//
// Layouts (t = thread within the slice, w = t / 64, lane = t % 64):
//  D1 (time order): s = lane % S1, l = lane / S1, n1 = w S1 + s; element e
//     holds n = n1 + B1 (l + LB2 e).
//  D3 (frequency order): s = lane % S3, l = lane / S3, k2 = w S3 + s;
//     register r = i LB1 + b holds k = k2 + B2 ((l E/LB1 + i) + E b).
// LDS: an exchange area holds NA slots of SLOT padded elements (array i at
// slot i); index j of a slot lives at fspad(j) = j + D1 (j >> K1) + D2 (j >> K2).
#pragma once
#include "fft.hpp"
#include "kcommon.hpp"

namespace sg {

// The LDS layout of the exchange slots (compile-time knobs; the default is
// one skew element per 32).  Every shift is far below log2(64 E), so a
// wave's indices [w 64 E, (w+1) 64 E) map to its own part of a slot.
#ifndef SG_FS_K1
#define SG_FS_K1 5
#endif
#ifndef SG_FS_D1
#define SG_FS_D1 1
#endif
#ifndef SG_FS_K2
#define SG_FS_K2 30
#endif
#ifndef SG_FS_D2
#define SG_FS_D2 0
#endif
__host__ __device__ constexpr int fspad(int i) { return i + SG_FS_D1 * (i >> SG_FS_K1) + SG_FS_D2 * (i >> SG_FS_K2); }
// A block of B consecutive indices that starts at a multiple of B lies within
// one padding period (2^SG_FS_K1 indices) or covers whole ones: fspad then
// splits over the block's index arithmetic as the exchanges below assume
// (blocks of 16 occur for N = 1024, 64 x 16).
__host__ __device__ constexpr bool fs_block_ok(int B) {
  return B % (1 << SG_FS_K1) == 0 || (1 << SG_FS_K1) % B == 0;
}
// Shape of the four-step split for length N with E elements per thread:
// step-1 transforms of length B2 = 8 E on 8 lanes, step-3 transforms of
// length B1 = N / B2 on LB1 = B1 / E lanes.
template <int N, int E>
struct fs_shape {
  static constexpr int T = N / E;
  static constexpr int LB2 = 8;
  static constexpr int B2 = E * LB2;
  static constexpr int B1 = N / B2;
  static constexpr int LB1 = B1 / E;
  static constexpr int S1 = 64 / LB2;
  static constexpr int S3 = 64 / LB1;
  static constexpr int Q1 = E / LB2, Q3 = E / LB1;
  static constexpr int WAVE = 64 * E;  // elements of one wave (one array)
  static constexpr int SLOT = fspad(N);
  static_assert(T % 64 == 0, "a slice is whole waves");
  static_assert(LB1 >= 1 && LB1 <= E && (64 % LB1) == 0, "step-3 transforms must fit one wave");
  static_assert(B1 * B2 == N, "N = B1 * B2");
  // twiddle table: step-1 lane sets (B2), step-3 lane sets (B1), outer (N)
  static constexpr int TW1 = 0, TW3 = B2, TWO = B2 + B1, TW_SIZE = B2 + B1 + N;
  // D1 element e of thread t: its index n
  __host__ __device__ static constexpr int d1_index(int t, int e) {
    return ((t >> 6) * S1 + (t & 63) % S1) + B1 * ((t & 63) / S1 + LB2 * e);
  }
  // D3 register r of thread t: its index k
  __host__ __device__ static constexpr int d3_index(int t, int r) {
    return ((t >> 6) * S3 + (t & 63) % S3) + B2 * (((t & 63) / S3) * Q3 + r / LB1 + E * (r % LB1));
  }
  // the same split into a per-thread part in [0, D3_SPAN) and a per-register
  // part (a compile-time constant once the register loop is unrolled)
  static constexpr int D3_SPAN = B2 * (E - Q3 + 1);
  __host__ __device__ static constexpr int d3_base(int t) {
    return ((t >> 6) * S3 + (t & 63) % S3) + B2 * (((t & 63) / S3) * Q3);
  }
  __host__ __device__ static constexpr int d3_off(int r) { return B2 * (r / LB1 + E * (r % LB1)); }
  static constexpr bool d3_split_ok() {
    for (int t = 0; t < T; ++t) {
      if (d3_base(t) < 0 || d3_base(t) >= D3_SPAN) return false;
      for (int r = 0; r < E; ++r)
        if (d3_index(t, r) != d3_base(t) + d3_off(r)) return false;
    }
    return true;
  }
};

// The LDS indices below are written as a per-thread base plus compile-time
// offsets (immediate offsets of the LDS instructions), using
//   fspad(x + y) = fspad(x) + fspad(y)
// whenever adding y to x carries across no multiple of 2^K1 or 2^K2 (y a
// multiple of both, or below 2^K1 with x a multiple of 2^K1, ...), so that
// each access pattern takes one address register.  Every split below is of
// that kind for the shapes in use (for the default layout and the others a
// build may choose; the emulation tests check the results).

// Wave-local barrier: orders this wave's LDS accesses (the LDS operations of
// one wave complete in order) and keeps the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward sub-transform of length B = E * LB on the LB lanes of a group,
// for NA arrays.  In: lane l holds x[l + LB e] in v[i][e].  Out: lane l holds
// X[a + E b], a = l Q + q (Q = E / LB), at register q LB + b.  The transpose
// goes through indices [base, base + B) of each array's slot (array i at
// area + i * SLOT).  tw[r]: w_B^(ll a) for register r = q LB + ll of this
// lane (conjugated for INV); tw[r] is read once per r.
template <bool INV, int E, int LB, int SLOT, int NA, typename R, typename TV>
__device__ __forceinline__ void fs_sub_fwd(cx<R> (&v)[NA][E], cx<R>* area, int base, const TV& tw, int l) {
  constexpr int Q = E / LB;
#pragma unroll
  for (int i = 0; i < NA; ++i) dft<E, INV>(v[i]);
  wave_sync();  // the wave's earlier reads of the region come first
  static_assert((1 << SG_FS_K1) % E == 0 && fs_block_ok(E * LB), "index decomposition");
  // base is a multiple of B = E LB (fs_block_ok)
  cx<R>* wr = area + fspad(base + l * E);     // + i SLOT + a
  cx<R>* rd = area + fspad(base) + l * Q;     // + i SLOT + fspad(ll E) + q
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int a = 0; a < E; ++a) wr[i * SLOT + a] = v[i][a];
  wave_sync();
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int ll = 0; ll < LB; ++ll) {
      const int r = q * LB + ll;
      const cx<R> w = ll == 0 ? cx<R>{(R)1, (R)0} : tw[r];
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const cx<R> u = rd[i * SLOT + fspad(ll * E) + q];
        v[i][r] = (ll == 0) ? u : (INV ? cmulc(u, w) : cmul(u, w));
      }
    }
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int q = 0; q < Q; ++q) dft<LB, INV>(&v[i][q * LB]);
  wave_sync();
}

// The transform of fs_sub_fwd run backwards: input in its output order,
// output in its input order.  With INV it is the (unnormalised) inverse.
template <bool INV, int E, int LB, int SLOT, int NA, typename R, typename TV>
__device__ __forceinline__ void fs_sub_bwd(cx<R> (&v)[NA][E], cx<R>* area, int base, const TV& tw, int l) {
  constexpr int Q = E / LB;
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int q = 0; q < Q; ++q) dft<LB, INV>(&v[i][q * LB]);
  static_assert((1 << SG_FS_K1) % E == 0 && fs_block_ok(E * LB), "index decomposition");
  cx<R>* wr = area + fspad(base) + l * Q;     // + i SLOT + fspad(ll E) + q
  cx<R>* rd = area + fspad(base + l * E);     // + i SLOT + a
  wave_sync();  // the wave's earlier reads of the region come first
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int ll = 0; ll < LB; ++ll) {
      const int r = q * LB + ll;
      const cx<R> w = ll == 0 ? cx<R>{(R)1, (R)0} : tw[r];
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const cx<R> u = v[i][r];
        wr[i * SLOT + fspad(ll * E) + q] = (ll == 0) ? u : (INV ? cmulc(u, w) : cmul(u, w));
      }
    }
  wave_sync();
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int a = 0; a < E; ++a) v[i][a] = rd[i * SLOT + a];
#pragma unroll
  for (int i = 0; i < NA; ++i) dft<E, INV>(v[i]);
  wave_sync();
}

// A set of E twiddles: held in registers (REG), or read from a table with
// each element loaded where it is used (a load merged with an earlier one of
// the same address would keep the value live in a register in between).
template <typename R, bool REG>
struct tw_view {
  const cx<R>* p;  // registers, or the table
  int o;           // offset of the set in the table
  __device__ __forceinline__ cx<R> operator[](int r) const {
    if constexpr (REG) return p[r];
    else return p[(unsigned)opaque(o) + r];
  }
};

// Per-thread twiddles of the four-step transform: the step-1 and step-3 lane
// sets and the outer twiddles w_N^(n1 k2) of this thread's D1 elements after
// step 1.  KEEP: held in registers (loaded once; the two lane sets are one
// when the steps have the same shape); otherwise read from the table at each
// use.
template <int N, int E, typename R, bool KEEP>
struct fs_tw {
  using S = fs_shape<N, E>;
  static constexpr bool SAME = S::B1 == S::B2 && S::LB1 == S::LB2;
  cx<R> t1[KEEP ? E : 1], t3[KEEP && !SAME ? E : 1], to[KEEP ? E : 1];
  const cx<R>* tab;
  int o1, o3, oo;  // offsets of this thread's sets in the table
  __device__ __forceinline__ void init(const cx<R>* __restrict__ table, int t) {
    const int lane = t & 63, w = t >> 6;
    const int l1 = lane / S::S1, n1 = w * S::S1 + lane % S::S1;
    const int l3 = lane / S::S3;
    tab = table;
    o1 = S::TW1 + l1 * E;
    o3 = S::TW3 + l3 * E;
    oo = S::TWO + (n1 * S::LB2 + l1) * E;
    if constexpr (KEEP) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        t1[r] = table[o1 + r];
        if constexpr (!SAME) t3[r] = table[o3 + r];
        to[r] = table[oo + r];
      }
    }
  }
  __device__ __forceinline__ tw_view<R, KEEP> set1() const {
    if constexpr (KEEP) return {t1, 0};
    else return {tab, o1};
  }
  __device__ __forceinline__ tw_view<R, KEEP> set3() const {
    if constexpr (KEEP && SAME) return {t1, 0};
    else if constexpr (KEEP) return {t3, 0};
    else return {tab, o3};
  }
  __device__ __forceinline__ tw_view<R, KEEP> outer() const {
    if constexpr (KEEP) return {to, 0};
    else return {tab, oo};
  }
};

// Host side: the twiddle table of fs_shape<N, E> (TW_SIZE entries), from a
// function giving exp(-2 pi i m / L) for 0 <= m < L (any L dividing 2N).
template <int N, int E, typename F>
void fs_fill_twiddles(F root, double* out_re, double* out_im) {
  using S = fs_shape<N, E>;
  // step-1 and step-3 lane sets: lane l, register r = q LB + ll -> w_B^(ll (l Q + q))
  auto lane_set = [&](int off, int B, int LB, int Q) {
    for (int l = 0; l < LB; ++l)
      for (int r = 0; r < E; ++r) {
        const int q = r / LB, ll = r % LB;
        const int m = (ll * (l * Q + q)) % B;
        root(m, B, out_re + off + l * E + r, out_im + off + l * E + r);
      }
  };
  lane_set(S::TW1, S::B2, S::LB2, S::Q1);
  lane_set(S::TW3, S::B1, S::LB1, S::Q3);
  // outer: thread (n1, l), register r = q LB2 + b -> w_N^(n1 k2), k2 = l Q1 + q + E b
  for (int n1 = 0; n1 < S::B1; ++n1)
    for (int l = 0; l < S::LB2; ++l)
      for (int r = 0; r < E; ++r) {
        const int q = r / S::LB2, b = r % S::LB2;
        const int k2 = l * S::Q1 + q + E * b;
        const int m = (int)(((long long)n1 * k2) % N);
        const int o = S::TWO + (n1 * S::LB2 + l) * E + r;
        root(m, N, out_re + o, out_im + o);
      }
}

// The four-step transform in phases.  Forward: fs_step1_fwd (wave-local),
// fs_cross13 (the one workgroup exchange), fs_step3_fwd (wave-local): D1 ->
// D3.  Inverse: fs_step3_inv, fs_cross31, fs_step1_inv: D3 -> D1.  Each
// wave-local phase transposes in the indices of the area that its wave reads
// in the adjacent exchange (step 1: [n1 B2, (n1+1) B2), n1-major; step 3:
// [k2 B1, (k2+1) B1), k2-major; both lie in [w WAVE, (w+1) WAVE)), which no
// other wave touches between that exchange's barrier and the next exchange's
// writes.  A caller that writes an exchange area which some wave may still
// be using for its transposes passes sync_before = true (a workgroup barrier
// before the writes).

// Step 1 of the forward transform and the outer twiddle (D1 in, step-1
// output order out: register r = q LB2 + b holds k2 = l Q1 + q + E b).
template <int N, int E, int NA, typename R, typename TW>
__device__ __forceinline__ void fs_step1_fwd(cx<R> (&v)[NA][E], cx<R>* area, const TW& tw, int t) {
  using S = fs_shape<N, E>;
  const int lane = t & 63, w = t >> 6;
  const int s = lane % S::S1, l = lane / S::S1;
  fs_sub_fwd<false, E, S::LB2, S::SLOT, NA>(v, area, (w * S::S1 + s) * S::B2, tw.set1(), l);
  const auto to = tw.outer();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const cx<R> w = to[r];
#pragma unroll
    for (int i = 0; i < NA; ++i) v[i][r] = cmul(v[i][r], w);
  }
}

// Exchange after step 1 (k2-major: (n1, k2) at index k2 B1 + n1): step-1
// output order in, step-3 input order out (element e holds n1 = l + LB1 e).
template <int N, int E, int NA, typename R>
__device__ __forceinline__ void fs_cross13(cx<R> (&v)[NA][E], cx<R>* xa, bool sync_before, int t) {
  using S = fs_shape<N, E>;
  const int lane = t & 63, w = t >> 6;
  if (sync_before) __syncthreads();
  {
    const int s = lane % S::S1, l = lane / S::S1;
    const int n1 = w * S::S1 + s;
    static_assert(fs_block_ok(S::B1), "index decomposition");
    cx<R>* wr = xa + fspad(l * S::Q1 * S::B1 + n1);  // + i SLOT + fspad((q + E b) B1)
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int q = 0; q < S::Q1; ++q)
#pragma unroll
        for (int b = 0; b < S::LB2; ++b) wr[i * S::SLOT + fspad((q + E * b) * S::B1)] = v[i][q * S::LB2 + b];
  }
  __syncthreads();
  {
    const int s = lane % S::S3, l = lane / S::S3;
    const int k2 = w * S::S3 + s;
    static_assert(32 % S::LB1 == 0, "index decomposition");
    const cx<R>* rd = xa + fspad(k2 * S::B1) + l;  // + i SLOT + fspad(LB1 e)
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int e = 0; e < E; ++e) v[i][e] = rd[i * S::SLOT + fspad(S::LB1 * e)];
  }
}

// Step 3 of the forward transform (D3 out).
template <int N, int E, int NA, typename R, typename TW>
__device__ __forceinline__ void fs_step3_fwd(cx<R> (&v)[NA][E], cx<R>* area, const TW& tw, int t) {
  using S = fs_shape<N, E>;
  const int lane = t & 63, w = t >> 6;
  fs_sub_fwd<false, E, S::LB1, S::SLOT, NA>(v, area, (w * S::S3 + lane % S::S3) * S::B1, tw.set3(), lane / S::S3);
}

// Step 3 of the inverse transform (D3 in; element e then holds n1 = l + LB1 e).
template <int N, int E, int NA, typename R, typename TW>
__device__ __forceinline__ void fs_step3_inv(cx<R> (&v)[NA][E], cx<R>* area, const TW& tw, int t) {
  using S = fs_shape<N, E>;
  const int lane = t & 63, w = t >> 6;
  fs_sub_bwd<true, E, S::LB1, S::SLOT, NA>(v, area, (w * S::S3 + lane % S::S3) * S::B1, tw.set3(), lane / S::S3);
}

// Exchange of the inverse (n1-major: (n1, k2) at index n1 B2 + k2) with the
// conjugate outer twiddle: step-3 inverse output in, step-1 inverse input out.
template <int N, int E, int NA, typename R, typename TW>
__device__ __forceinline__ void fs_cross31(cx<R> (&v)[NA][E], cx<R>* xa, bool sync_before, const TW& tw, int t) {
  using S = fs_shape<N, E>;
  const int lane = t & 63, w = t >> 6;
  if (sync_before) __syncthreads();
  {
    const int k2 = w * S::S3 + lane % S::S3, l = lane / S::S3;
    static_assert(S::B2 % 32 == 0, "index decomposition");
    cx<R>* wr = xa + fspad(l * S::B2 + k2);  // + i SLOT + fspad(LB1 e B2)
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int e = 0; e < E; ++e) wr[i * S::SLOT + fspad(S::LB1 * e * S::B2)] = v[i][e];
  }
  __syncthreads();
  {
    const int s = lane % S::S1, l = lane / S::S1;
    const int n1 = w * S::S1 + s;
    const auto to = tw.outer();
    const cx<R>* rd = xa + fspad(n1 * S::B2) + l * S::Q1;  // + i SLOT + q + fspad(E b)
#pragma unroll
    for (int q = 0; q < S::Q1; ++q)
#pragma unroll
      for (int b = 0; b < S::LB2; ++b) {
        const int r = q * S::LB2 + b;
        const cx<R> w = to[r];
#pragma unroll
        for (int i = 0; i < NA; ++i) v[i][r] = cmulc(rd[i * S::SLOT + q + fspad(E * b)], w);
      }
  }
}

// Step 1 of the inverse transform (D1 out).
template <int N, int E, int NA, typename R, typename TW>
__device__ __forceinline__ void fs_step1_inv(cx<R> (&v)[NA][E], cx<R>* area, const TW& tw, int t) {
  using S = fs_shape<N, E>;
  const int lane = t & 63, w = t >> 6;
  fs_sub_bwd<true, E, S::LB2, S::SLOT, NA>(v, area, (w * S::S1 + lane % S::S1) * S::B2, tw.set1(), lane / S::S1);
}

}  // namespace sg
