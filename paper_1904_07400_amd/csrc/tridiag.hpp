// Batched solve of tridiag(1, 6, 1) x = d (x = 0 outside the line), the
// systems of Eqs. (z_system) and (C_system) (Sec. 2.3), in FP64 on one
// workgroup-slice per line.
//
// Partition method: thread t owns the contiguous chunk [t*CH, (t+1)*CH) of
// the line.  A downward and an upward elimination inside the chunk express
// every interior unknown through the chunk's first and last unknowns; the
// 2T boundary unknowns of all chunks then satisfy a tridiagonal system,
// solved by parallel cyclic reduction in LDS; back-substitution recovers
// the interior.  The matrix is constant, so the elimination multipliers are
// compile-time constants and only the right-hand side is data.
#pragma once
#include <hip/hip_runtime.h>

namespace sg {

template <int CH>
struct tri_consts {
  // row r (1 <= r <= CH-1) after the downward sweep: al[r] x_0 + be[r] x_r + x_{r+1} = dl_r
  // row r (1 <= r <= CH-2) after the upward sweep:   ap[r] x_0 + be[r] x_r + ga[r] x_{CH-1} = du_r
  double be[CH], ibe[CH], al[CH], ap[CH], ga[CH];
  double P, Q, A, B;  // reduced rows: x_prev + P f + Q l = R ; A f + B l + x_next = D
  constexpr tri_consts() : be(), ibe(), al(), ap(), ga(), P(0), Q(0), A(0), B(0) {
    static_assert(CH >= 3, "chunk must hold at least 3 unknowns");
    al[1] = 1.0;
    be[1] = 6.0;
    for (int r = 2; r < CH; ++r) {
      al[r] = -al[r - 1] / be[r - 1];
      be[r] = 6.0 - 1.0 / be[r - 1];
    }
    for (int r = 1; r < CH; ++r) ibe[r] = 1.0 / be[r];
    ap[CH - 2] = al[CH - 2];
    ga[CH - 2] = 1.0;
    for (int r = CH - 3; r >= 1; --r) {
      ap[r] = al[r] - ap[r + 1] / be[r + 1];
      ga[r] = -ga[r + 1] / be[r + 1];
    }
    P = 6.0 - ap[1] / be[1];
    Q = -ga[1] / be[1];
    A = al[CH - 1];
    B = be[CH - 1];
  }
};

template <typename V>
__device__ __forceinline__ V vscale(V a, double s);
template <>
__device__ __forceinline__ double vscale(double a, double s) { return a * s; }
template <>
__device__ __forceinline__ double2 vscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// LDS needed by tri_solve for T threads: coefficient and rhs arrays of the
// reduced system (2T rows).
template <typename V, int T>
struct tri_smem {
  double a[2 * T], b[2 * T], c[2 * T];
  V d[2 * T];
};

// Solve tridiag(1,6,1) x = d on a line of CH*T unknowns; d (CH values in
// this thread's chunk) is overwritten with x.  Every thread of the
// workgroup must call it (it contains workgroup barriers); each slice of T
// threads passes its own LDS area.
template <int CH, int T, typename V>
__device__ __forceinline__ void tri_solve(V* d, int t, tri_smem<V, T>& sm) {
  constexpr tri_consts<CH> K{};
  // downward sweep in place: d_r <- d_r - d_{r-1} / be_{r-1}, r >= 2
#pragma unroll
  for (int r = 2; r < CH; ++r) d[r] = d[r] - vscale(d[r - 1], K.ibe[r - 1]);
  // upward sweep in place: d_r <- d_r - d_{r+1} / be_{r+1}, r = CH-3 .. 1
#pragma unroll
  for (int r = CH - 3; r >= 1; --r) d[r] = d[r] - vscale(d[r + 1], K.ibe[r + 1]);
  // reduced system rows 2t (first unknown f_t) and 2t+1 (last unknown l_t)
  const int i0 = 2 * t, i1 = 2 * t + 1;
  sm.a[i0] = (t == 0) ? 0.0 : 1.0;
  sm.b[i0] = K.P;
  sm.c[i0] = K.Q;
  sm.d[i0] = d[0] - vscale(d[1], K.ibe[1]);
  sm.a[i1] = K.A;
  sm.b[i1] = K.B;
  sm.c[i1] = (t == T - 1) ? 0.0 : 1.0;
  sm.d[i1] = d[CH - 1];
  __syncthreads();
  // parallel cyclic reduction on the 2T reduced rows
#pragma unroll 1
  for (int s = 1; s < 2 * T; s *= 2) {
    double na[2], nb[2], nc[2];
    V nd[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 2 * t + h;
      const double ai = sm.a[i], bi = sm.b[i], ci = sm.c[i];
      const V di = sm.d[i];
      double k1 = 0.0, k2 = 0.0, am = 0.0, cm = 0.0, ap = 0.0, cp = 0.0;
      V dm = vscale(di, 0.0), dp = vscale(di, 0.0);
      if (i - s >= 0) {
        k1 = ai / sm.b[i - s];
        am = sm.a[i - s];
        cm = sm.c[i - s];
        dm = sm.d[i - s];
      }
      if (i + s < 2 * T) {
        k2 = ci / sm.b[i + s];
        ap = sm.a[i + s];
        cp = sm.c[i + s];
        dp = sm.d[i + s];
      }
      na[h] = -am * k1;
      nc[h] = -cp * k2;
      nb[h] = bi - cm * k1 - ap * k2;
      nd[h] = di - vscale(dm, k1) - vscale(dp, k2);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 2 * t + h;
      sm.a[i] = na[h];
      sm.b[i] = nb[h];
      sm.c[i] = nc[h];
      sm.d[i] = nd[h];
    }
    __syncthreads();
  }
  const V f = vscale(sm.d[i0], 1.0 / sm.b[i0]);
  const V l = vscale(sm.d[i1], 1.0 / sm.b[i1]);
  __syncthreads();
#pragma unroll
  for (int r = 1; r <= CH - 2; ++r)
    d[r] = vscale(d[r] - vscale(f, K.ap[r]) - vscale(l, K.ga[r]), K.ibe[r]);
  d[0] = f;
  d[CH - 1] = l;
}

}  // namespace sg
