// Batched solve of tridiag(1, 6, 1) x = d (x = 0 outside the line), the
// systems of Eqs. (z_system) and (C_system) (Sec. 2.3), in FP64, one line
// per slice of T threads of a workgroup.
//
// The constant matrix factors exactly: with r = 3 - 2 sqrt(2) (the root of
// r^2 - 6 r + 1 = 0 below 1), L = I + r E and U = I + r E^T (E the lower
// shift) satisfy
//     tridiag(1, 6, 1) = L U / r + r e0 e0^T,
// because (1 + r^2) / r = 6 everywhere on the diagonal except at row 0,
// where L U / r has 1 / r = 6 - r.  So x = y - alpha z with
//     y = r U^-1 L^-1 d                    (two first-order recurrences)
//     z = r U^-1 L^-1 e0,  z_i = r (-r)^i (1 - r^(2(n-i))) / (1 - r^2)
//     alpha = r y_0 / (1 + r z_0)          (Sherman-Morrison).
// Thread t owns the chunk [t*CH, (t+1)*CH) and runs both recurrences on it
// with a zero carry; the true carry into a chunk is a geometric sum of the
// neighbouring chunks' end values with ratio q = (-r)^CH, truncated after S
// terms where |r|^(S*CH) < 1e-18 (|r| = 0.17, so S = 3 for CH = 8).  Three
// workgroup barriers in all (the last one, optional, lets the caller reuse
// the LDS);
// z_i is below 1e-19 of z_0 past i = 24, so the rank-one term touches only
// the first 24 unknowns.
#pragma once
#include <hip/hip_runtime.h>

namespace sg {

template <typename V>
__device__ __forceinline__ V vscale(V a, double s);
template <>
__device__ __forceinline__ double vscale(double a, double s) { return a * s; }
template <>
__device__ __forceinline__ double2 vscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
template <typename V>
__device__ __forceinline__ V vzero();
template <>
__device__ __forceinline__ double vzero() { return 0.0; }
template <>
__device__ __forceinline__ double2 vzero() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// r = 3 - 2 sqrt(2) to double precision
constexpr double kTriR = 0.17157287525380990240;
constexpr int kTriHead = 24;  // unknowns reached by the rank-one correction

template <int CH, int T>
struct tri_consts {
  static constexpr int N = CH * T;
  static constexpr int S0 = (24 + CH - 1) / CH;                 // carry terms
  static constexpr int S = S0 < 1 ? 1 : (S0 > T - 1 ? (T > 1 ? T - 1 : 1) : S0);
  static constexpr int H = kTriHead < N ? kTriHead : N;
  double pw[CH + 1];    // (-r)^e, e = 0..CH
  double qp[4 * 8];     // q^(s-1), s = 1..S, q = (-r)^CH (at most 32 terms used)
  double z[kTriHead];   // z_i, i < H
  double alpha_scale;   // r / (1 + r z_0)
  constexpr tri_consts() : pw(), qp(), z(), alpha_scale(0) {
    const double r = kTriR;
    pw[0] = 1.0;
    for (int e = 1; e <= CH; ++e) pw[e] = pw[e - 1] * (-r);
    qp[0] = 1.0;
    for (int s = 1; s < 32; ++s) qp[s] = qp[s - 1] * pw[CH];
    double rr = r * r;
    for (int i = 0; i < H; ++i) {
      double p = 1.0;  // r^(2(N-i))
      for (int a = 0; a < N - i && p > 1e-300; ++a) p *= rr;
      double ri = 1.0;
      for (int a = 0; a < i; ++a) ri *= -r;
      z[i] = r * ri * (1.0 - p) / (1.0 - rr);
    }
    alpha_scale = r / (1.0 + r * z[0]);
  }
};

// LDS needed by tri_solve for one line of T threads.
template <typename V, int T>
struct tri_smem {
  V fwd[T];
  V bwd[T];
};

// Solve tridiag(1,6,1) x = d on a line of CH*T unknowns; d (this thread's
// CH values, chunk t) is overwritten with x.  Every thread of the workgroup
// must call it (it holds workgroup barriers); each line passes its own LDS.
template <int CH, int T, typename V, bool TAIL = true>
__device__ __forceinline__ void tri_solve(V* d, int t, tri_smem<V, T>& sm) {
  using K = tri_consts<CH, T>;
  constexpr K k{};
  constexpr double r = kTriR;
  // forward recurrence u_i = d_i - r u_(i-1), zero carry into the chunk
#pragma unroll
  for (int e = 1; e < CH; ++e) d[e] = d[e] - vscale(d[e - 1], r);
  sm.fwd[t] = d[CH - 1];
  __syncthreads();
  if (T > 1) {
    V c = vzero<V>();
#pragma unroll
    for (int s = 1; s <= K::S; ++s)
      if (t - s >= 0) c = c + vscale(sm.fwd[t - s], k.qp[s - 1]);
#pragma unroll
    for (int e = 0; e < CH; ++e) d[e] = d[e] + vscale(c, k.pw[e + 1]);
  }
  // backward recurrence v_i = u_i - r v_(i+1), zero carry into the chunk
#pragma unroll
  for (int e = CH - 2; e >= 0; --e) d[e] = d[e] - vscale(d[e + 1], r);
  sm.bwd[t] = d[0];
  __syncthreads();
  if (T > 1) {
    V c = vzero<V>();
#pragma unroll
    for (int s = 1; s <= K::S; ++s)
      if (t + s < T) c = c + vscale(sm.bwd[t + s], k.qp[s - 1]);
#pragma unroll
    for (int e = 0; e < CH; ++e) d[e] = d[e] + vscale(c, k.pw[CH - e]);
  }
#pragma unroll
  for (int e = 0; e < CH; ++e) d[e] = vscale(d[e], r);  // y = r v
  // rank-one correction x = y - alpha z, alpha = r y_0 / (1 + r z_0); y_0 is
  // rebuilt from thread 0's backward start value and its carry, both in LDS
  if (t * CH < K::H) {
    V c = vzero<V>();
#pragma unroll
    for (int s = 1; s <= K::S; ++s)
      if (s < T) c = c + vscale(sm.bwd[s], k.qp[s - 1]);
    const V y0 = vscale(sm.bwd[0] + vscale(c, k.pw[CH]), r);
    const V a = vscale(y0, k.alpha_scale);
#pragma unroll
    for (int i = 0; i < K::H; ++i)  // compile-time indices into z and d
      if (i / CH == t) d[i % CH] = d[i % CH] - vscale(a, k.z[i]);
  }
  // the caller may reuse the LDS after this barrier (TAIL); without it, the
  // caller must pass a barrier of its own before writing over sm
  if constexpr (TAIL) __syncthreads();
}

}  // namespace sg
