// Batched solve of tridiag(1, 6, 1) x = d (x = 0 outside the line), the
// systems of Eqs. (z_system) and (C_system) (Sec. 2.3), in FP64, one line
// per slice of T threads of a workgroup; the same for tridiag(1, 4, 1) and
// pentadiag(1, 76, 230, 76, 1), the systems of the cubic and quartic splines
// (k = 4, 5; the extension the end of Sec. 2.3 states), further below.
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

// Roots below 1 of the first-order factors (see each system) to double
// precision, and for each the distance in unknowns over which its powers
// fall below 5e-19 (the reach of a carry or of the boundary correction):
//   0: 3 - 2 sqrt(2)   tridiag(1, 6, 1)   (k = 3)
//   1: 2 - sqrt(3)     tridiag(1, 4, 1)   (k = 4)
//   2, 3: the two roots l of l^2 - w l + 1 = 0, w = 38 -+ sqrt(1216), so that
//         (1 + l1 z)(1 + l1/z)(1 + l2 z)(1 + l2/z) / (l1 l2) is
//         z^-2 + 76 z^-1 + 230 + 76 z + z^2: pentadiag(1, 76, 230, 76, 1) (k = 5)
constexpr double kLam[4] = {0.17157287525380990240, 0.26794919243112270647, 0.36134122590022017709,
                            0.013725429297339121360};
constexpr int kLamReach[4] = {24, 32, 42, 10};

// r = 3 - 2 sqrt(2) to double precision
constexpr double kTriR = kLam[0];
constexpr int kTriHead = 32;  // largest reach of a rank-one correction (k = 3: 24, k = 4: 32)

// SYS: 3 = tridiag(1, 6, 1), 4 = tridiag(1, 4, 1); both are L U / r + r e0 e0^T
// with their own r (since (1 + r^2) / r is the diagonal)
template <int CH, int T, int SYS = 3>
struct tri_consts {
  static constexpr int N = CH * T;
  static constexpr double R = kLam[SYS - 3];
  static constexpr int REACH = kLamReach[SYS - 3];
  static constexpr int S0 = (REACH + CH - 1) / CH;              // carry terms
  static constexpr int S = S0 < 1 ? 1 : (S0 > T - 1 ? (T > 1 ? T - 1 : 1) : S0);
  static constexpr int H = REACH < N ? REACH : N;
  double pw[CH + 1];    // (-r)^e, e = 0..CH
  double qp[4 * 8];     // q^(s-1), s = 1..S, q = (-r)^CH (at most 32 terms used)
  double z[kTriHead];   // z_i, i < H
  double alpha_scale;   // r / (1 + r z_0)
  constexpr tri_consts() : pw(), qp(), z(), alpha_scale(0) {
    const double r = R;
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
template <int CH, int T, typename V, bool TAIL = true, int SYS = 3>
__device__ __forceinline__ void tri_solve(V* d, int t, tri_smem<V, T>& sm) {
  using K = tri_consts<CH, T, SYS>;
  constexpr K k{};
  constexpr double r = K::R;
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

// ------------------------------------------------ pentadiagonal (k = 5) --
// pentadiag(1, 76, 230, 76, 1) x = d, x = 0 outside the line.  With the roots
// l1, l2 above, L = (I + l1 E)(I + l2 E) (lower, bandwidth 2) and
// c = 1 / (l1 l2), c L L^T has the matrix's rows everywhere except in its
// top-left 2 x 2 block, which misses the terms of the rows above the line:
//     A = c L L^T + P K P^T,  P = [e0 e1],
//     K = [[(m1^2 + m2^2) / m2, m1], [m1, m2]],  m1 = l1 + l2, m2 = l1 l2.
// So y = (1/c) L^-T L^-1 d takes four first-order sweeps (two forward, two
// backward, one barrier each), and Woodbury's identity gives
//     x = y - Z a,  Z = (c L L^T)^-1 P,  a = (I + K Z_p)^-1 K y_p,
// with Z_p and y_p the first two rows of Z and y.  Z's entries fall below
// 5e-19 past row 42 (|l1|^42), so the correction touches the first 42
// unknowns only.

// one first-order sweep's constants for root LI on chunks of CH
template <int LI, int CH, int T>
struct sweep_consts {
  static constexpr int S0 = (kLamReach[LI] + CH - 1) / CH;  // carry terms
  static constexpr int S = S0 < 1 ? 1 : (S0 > T - 1 ? (T > 1 ? T - 1 : 1) : S0);
  double pw[CH + 1];  // (-l)^e, e = 0..CH
  double qp[64];      // q^(s-1), q = (-l)^CH
  constexpr sweep_consts() : pw(), qp() {
    pw[0] = 1.0;
    for (int e = 1; e <= CH; ++e) pw[e] = pw[e - 1] * (-kLam[LI]);
    qp[0] = 1.0;
    for (int s = 1; s < 64; ++s) qp[s] = qp[s - 1] * pw[CH];
  }
};

// u_i = d_i - l u_(i-1) along the line; thread t owns chunk t and takes its
// carry from the end values of the S chunks before it (through buf)
template <int LI, int CH, int T, typename V>
__device__ __forceinline__ void sweep_fwd(V* d, int t, V* buf) {
  using K = sweep_consts<LI, CH, T>;
  constexpr K k{};
  constexpr double l = kLam[LI];
#pragma unroll
  for (int e = 1; e < CH; ++e) d[e] = d[e] - vscale(d[e - 1], l);
  buf[t] = d[CH - 1];
  __syncthreads();
  if (T > 1) {
    V c = vzero<V>();
#pragma unroll
    for (int s = 1; s <= K::S; ++s)
      if (t - s >= 0) c = c + vscale(buf[t - s], k.qp[s - 1]);
#pragma unroll
    for (int e = 0; e < CH; ++e) d[e] = d[e] + vscale(c, k.pw[e + 1]);
  }
}

// v_i = u_i - l v_(i+1) along the line, carries from the chunks after; with
// SECOND, thread 0 also leaves its local second value in *second
template <int LI, int CH, int T, typename V, bool SECOND>
__device__ __forceinline__ void sweep_bwd(V* d, int t, V* buf, V* second) {
  using K = sweep_consts<LI, CH, T>;
  constexpr K k{};
  constexpr double l = kLam[LI];
#pragma unroll
  for (int e = CH - 2; e >= 0; --e) d[e] = d[e] - vscale(d[e + 1], l);
  buf[t] = d[0];
  if (SECOND && t == 0) *second = d[1];
  __syncthreads();
  if (T > 1) {
    V c = vzero<V>();
#pragma unroll
    for (int s = 1; s <= K::S; ++s)
      if (t + s < T) c = c + vscale(buf[t + s], k.qp[s - 1]);
#pragma unroll
    for (int e = 0; e < CH; ++e) d[e] = d[e] + vscale(c, k.pw[CH - e]);
  }
}

template <int CH, int T>
struct penta_consts {
  static constexpr int N = CH * T;
  static constexpr int H = kLamReach[2] < N ? kLamReach[2] : N;
  static constexpr int NW = N < H + 80 ? N : H + 80;  // rows of Z computed (the rest is below 1e-40)
  static constexpr double L1 = kLam[2], L2 = kLam[3];
  double z0[kLamReach[2]], z1[kLamReach[2]];  // columns of Z, rows < H
  double q[2][2];                             // (I + K Z_p)^-1 K
  constexpr penta_consts() : z0(), z1(), q() {
    const double m1 = L1 + L2, m2 = L1 * L2;
    for (int j = 0; j < 2; ++j) {
      double u[NW] = {};
      u[j] = 1.0;
      for (int i = 1; i < NW; ++i) u[i] -= L1 * u[i - 1];
      for (int i = 1; i < NW; ++i) u[i] -= L2 * u[i - 1];
      for (int i = NW - 2; i >= 0; --i) u[i] -= L1 * u[i + 1];
      for (int i = NW - 2; i >= 0; --i) u[i] -= L2 * u[i + 1];
      for (int i = 0; i < H; ++i) (j ? z1 : z0)[i] = m2 * u[i];
    }
    const double K00 = (m1 * m1 + m2 * m2) / m2, K01 = m1, K11 = m2;
    // Z_p[i][j] = column j, row i
    const double Z00 = z0[0], Z01 = z1[0], Z10 = z0[1], Z11 = N > 1 ? z1[1] : 0.0;
    // B = I + K Z_p
    const double B00 = 1.0 + K00 * Z00 + K01 * Z10, B01 = K00 * Z01 + K01 * Z11;
    const double B10 = K01 * Z00 + K11 * Z10, B11 = 1.0 + K01 * Z01 + K11 * Z11;
    const double det = B00 * B11 - B01 * B10;
    const double I00 = B11 / det, I01 = -B01 / det, I10 = -B10 / det, I11 = B00 / det;
    q[0][0] = I00 * K00 + I01 * K01;
    q[0][1] = I00 * K01 + I01 * K11;
    q[1][0] = I10 * K00 + I11 * K01;
    q[1][1] = I10 * K01 + I11 * K11;
  }
};

// LDS needed by penta_solve for one line of T threads
template <typename V, int T>
struct penta_smem {
  V f1[T], f2[T], b1[T], b2[T];
  V second;  // thread 0's local second value of the last backward sweep
};

template <int CH, int T, typename V, bool TAIL = true>
__device__ __forceinline__ void penta_solve(V* d, int t, penta_smem<V, T>& sm) {
  static_assert(CH >= 2, "the correction reads y_0 and y_1 from thread 0");
  using K = penta_consts<CH, T>;
  using K2 = sweep_consts<3, CH, T>;
  constexpr K k{};
  constexpr K2 k2{};
  constexpr double m2 = K::L1 * K::L2;
  sweep_fwd<2, CH, T>(d, t, sm.f1);
  sweep_fwd<3, CH, T>(d, t, sm.f2);
  sweep_bwd<2, CH, T, V, false>(d, t, sm.b1, nullptr);
  sweep_bwd<3, CH, T, V, true>(d, t, sm.b2, &sm.second);
#pragma unroll
  for (int e = 0; e < CH; ++e) d[e] = vscale(d[e], m2);  // y = L^-T L^-1 d / c
  if (t * CH < K::H) {
    // y_0, y_1 rebuilt from thread 0's local values and its carry
    V c = vzero<V>();
#pragma unroll
    for (int s = 1; s <= K2::S; ++s)
      if (s < T) c = c + vscale(sm.b2[s], k2.qp[s - 1]);
    const V y0 = vscale(sm.b2[0] + vscale(c, k2.pw[CH]), m2);
    const V y1 = vscale(sm.second + vscale(c, k2.pw[CH - 1]), m2);
    const V a0 = vscale(y0, k.q[0][0]) + vscale(y1, k.q[0][1]);
    const V a1 = vscale(y0, k.q[1][0]) + vscale(y1, k.q[1][1]);
#pragma unroll
    for (int i = 0; i < K::H; ++i)  // compile-time indices into z and d
      if (i / CH == t) d[i % CH] = d[i % CH] - vscale(a0, k.z0[i]) - vscale(a1, k.z1[i]);
  }
  if constexpr (TAIL) __syncthreads();
}

// ------------------------------------------------------------ dispatch --
// Interpolation system of order k (3, 4, 5), scaled to integer stencils:
// the caller multiplies the right-hand side by band_scale(k) per axis
// ((1/8) (1, 6, 1), (1/6) (1, 4, 1), (1/384) (1, 76, 230, 76, 1)).
__host__ __device__ constexpr double band_scale(int k) { return k == 5 ? 384.0 : (k == 4 ? 6.0 : 8.0); }

// LDS for any of the systems (the pentadiagonal one is the largest)
template <typename V, int T>
struct band_smem {
  static constexpr int BYTES = sizeof(penta_smem<V, T>) > sizeof(tri_smem<V, T>) ? (int)sizeof(penta_smem<V, T>)
                                                                                   : (int)sizeof(tri_smem<V, T>);
};

template <int SYS, int CH, int T, typename V, bool TAIL = true>
__device__ __forceinline__ void band_solve(V* d, int t, void* lds) {
  if constexpr (SYS == 5)
    penta_solve<CH, T, V, TAIL>(d, t, *reinterpret_cast<penta_smem<V, T>*>(lds));
  else
    tri_solve<CH, T, V, TAIL, SYS>(d, t, *reinterpret_cast<tri_smem<V, T>*>(lds));
}

}  // namespace sg
