// Workgroup-cooperative Stockham FFT for gfx950 (wave64), FP32 and FP64.
//
// One length-L transform is spread over T = L/E threads, E elements each, in
// the "strided" distribution: thread t holds x[t + e*T], e = 0..E-1.  Each
// Stockham stage of radix r (r | E) lets every thread run E/r butterflies on
// elements it already holds; the stage output goes through LDS and is read
// back in the strided distribution, except after the last stage, whose
// output lands in registers in natural order.  Twiddles are read from a
// table of roots of unity computed in FP64 on the host (rounded once for
// FP32), never accumulated by recurrence.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, R s) { return {a.x * s, a.y * s}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename R>
__device__ __forceinline__ cx<R> rot(cx<R> a) {
  return INV ? cx<R>{-a.y, a.x} : cx<R>{a.y, -a.x};
}

// ------------------------------------------------------------ small DFTs --
template <bool INV, typename R>
__device__ __forceinline__ void dft2(cx<R>* v) {
  cx<R> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <bool INV, typename R>
__device__ __forceinline__ void dft4(cx<R>& a, cx<R>& b, cx<R>& c, cx<R>& d) {
  cx<R> t0 = a + c, t1 = a - c, t2 = b + d, t3 = rot<INV>(b - d);
  a = t0 + t2;
  c = t0 - t2;
  b = t1 + t3;
  d = t1 - t3;
}

template <bool INV, typename R>
__device__ __forceinline__ void dft4(cx<R>* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }

// multiply by w_16^j (forward; conjugate for the inverse), j in 0..9
template <bool INV, int J, typename R>
__device__ __forceinline__ cx<R> w16(cx<R> a) {
  constexpr double C1 = 0.92387953251128675613, S1 = 0.38268343236508977173;
  constexpr double C2 = 0.70710678118654752440;
  constexpr int j = J % 16;
  // exp(-2 pi i j / 16) = (c, -s); inverse (c, +s)
  constexpr double c = j == 0 ? 1 : j == 1 ? C1 : j == 2 ? C2 : j == 3 ? S1 : j == 4 ? 0 : j == 5 ? -S1
                     : j == 6 ? -C2 : j == 7 ? -C1 : j == 8 ? -1 : j == 9 ? -C1 : 0;
  constexpr double s = j == 0 ? 0 : j == 1 ? S1 : j == 2 ? C2 : j == 3 ? C1 : j == 4 ? 1 : j == 5 ? C1
                     : j == 6 ? C2 : j == 7 ? S1 : j == 8 ? 0 : j == 9 ? -S1 : 0;
  if constexpr (j == 0) return a;
  else if constexpr (j == 4) return rot<INV>(a);
  else if constexpr (j == 8) return cx<R>{-a.x, -a.y};
  else {
    const R cc = (R)c, ss = INV ? (R)s : (R)(-s);
    return {a.x * cc - a.y * ss, a.x * ss + a.y * cc};
  }
}

template <bool INV, typename R>
__device__ __forceinline__ void dft8(cx<R>* v) {
  // n = 2 n1 + n2, k = k1 + 4 k2
  cx<R> a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
  cx<R> b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  b1 = w16<INV, 2>(b1);
  b2 = w16<INV, 4>(b2);
  b3 = w16<INV, 6>(b3);
  v[0] = a0 + b0;
  v[4] = a0 - b0;
  v[1] = a1 + b1;
  v[5] = a1 - b1;
  v[2] = a2 + b2;
  v[6] = a2 - b2;
  v[3] = a3 + b3;
  v[7] = a3 - b3;
}

template <bool INV, typename R>
__device__ __forceinline__ void dft16(cx<R>* v) {
  // n = 4 n1 + n2, k = k1 + 4 k2
  cx<R> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = v[n2];
    y[n2][1] = v[4 + n2];
    y[n2][2] = v[8 + n2];
    y[n2][3] = v[12 + n2];
    dft4<INV>(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
  }
  y[1][1] = w16<INV, 1>(y[1][1]);
  y[1][2] = w16<INV, 2>(y[1][2]);
  y[1][3] = w16<INV, 3>(y[1][3]);
  y[2][1] = w16<INV, 2>(y[2][1]);
  y[2][2] = w16<INV, 4>(y[2][2]);
  y[2][3] = w16<INV, 6>(y[2][3]);
  y[3][1] = w16<INV, 3>(y[3][1]);
  y[3][2] = w16<INV, 6>(y[3][2]);
  y[3][3] = w16<INV, 9>(y[3][3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<R> a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
    dft4<INV>(a, b, c, d);
    v[k1] = a;
    v[k1 + 4] = b;
    v[k1 + 8] = c;
    v[k1 + 12] = d;
  }
}

// length 3: X_1,2 = a - (b + c)/2 -/+ i (sqrt(3)/2)(b - c) (forward; the
// inverse swaps the sign of the imaginary term)
template <bool INV, typename R>
__device__ __forceinline__ void dft3(cx<R>* v) {
  constexpr double S3 = 0.86602540378443864676;  // sqrt(3) / 2
  const cx<R> a = v[0], b = v[1], c = v[2];
  const cx<R> s = b + c, d = b - c;
  const cx<R> m{a.x - (R)0.5 * s.x, a.y - (R)0.5 * s.y};
  const cx<R> j = rot<INV>(cx<R>{d.x * (R)S3, d.y * (R)S3});  // -i (sqrt(3)/2) d forward
  v[0] = a + s;
  v[1] = m + j;
  v[2] = m - j;
}

template <int r, bool INV, typename R>
__device__ __forceinline__ void dft(cx<R>* v) {
  if constexpr (r == 1) {
  } else if constexpr (r == 2) dft2<INV>(v);
  else if constexpr (r == 3) dft3<INV>(v);
  else if constexpr (r == 4) dft4<INV>(v);
  else if constexpr (r == 8) dft8<INV>(v);
  else if constexpr (r == 16) dft16<INV>(v);
  else static_assert(r == 2, "unsupported radix");
}

// ----------------------------------------------------------- radix plan --
// Stages for length L = 2^a or 3 * 2^a with E elements per thread: for
// L = 3 * 2^a a radix-3 stage first (E must then be a multiple of 3); then
// radix R0 = the largest power of two dividing E (at most 16) while it fits,
// then the power-of-two remainder.  Each stage of radix r runs E / r
// butterflies per thread.
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
__host__ __device__ constexpr int pow2_part(int v) { return (v & 1) ? 1 : 2 * pow2_part(v / 2); }
template <int L, int E>
struct plan {
  static constexpr int R3 = (L % 3 == 0) ? 1 : 0;  // leading radix-3 stage
  static constexpr int L2 = R3 ? L / 3 : L;        // power-of-two part of L
  static constexpr int R0 = pow2_part(E) < 16 ? pow2_part(E) : 16;
  static constexpr int nfull = R0 > 1 ? ilog2c(L2) / ilog2c(R0) : 0;
  static constexpr int rem = L2 >> (nfull * ilog2c(R0));  // 1 if exact
  static constexpr int nstages = R3 + nfull + (rem > 1 ? 1 : 0);
  static constexpr int radix(int s) { return s < R3 ? 3 : (s < R3 + nfull ? R0 : rem); }
  static constexpr int ns_before(int s) { return s == 0 ? 1 : ns_before(s - 1) * radix(s - 1); }
  // per-stage twiddle tables, stage s >= 1: entry (q-1)*Ns + k holds
  // w_{Ns r}^{k q}, q in [1, r), k in [0, Ns); tables laid end to end
  static constexpr int tw_offset(int s) {
    return s <= 1 ? 0 : tw_offset(s - 1) + (radix(s - 1) - 1) * ns_before(s - 1);
  }
  static constexpr int tw_size = tw_offset(nstages);
  static_assert(L2 == (1 << ilog2c(L2)), "length must be 2^a or 3 * 2^a");
  static_assert(E % (R3 ? 3 : 1) == 0 && (R0 == 1 ? L2 == 1 : true), "elements per thread do not fit the radices");
};

// LDS padding against bank conflicts: one slot every 2^SG_LDS_PAD elements
#ifndef SG_LDS_PAD
#define SG_LDS_PAD 5
#endif
__device__ __forceinline__ int pad(int i) { return i + (i >> SG_LDS_PAD); }
template <int L>
struct lds_len {
  static constexpr int value = L + (L >> SG_LDS_PAD);
};

// roots(i) = exp(-2 pi i * i / L) read from a table of the RB-th roots with
// stride S (RB = L * S).
template <typename R>
struct roots_t {
  const cx<R>* __restrict__ tab;
  int S;
  __device__ __forceinline__ cx<R> operator()(int i) const { return tab[i * S]; }
};

#ifndef SG_TW_EARLY_BYTES
#define SG_TW_EARLY_BYTES 64
#endif

// Stages of radix 8 and 16 load the twiddles of inputs q = 1, 2, 4
// (and 8) only and form the others as products of those, at most two
// products deep (fewer table loads; each product adds about one rounding)
#ifndef SG_TW_DERIVE
#define SG_TW_DERIVE 1
#endif
// the same for the FP64 stages
#ifndef SG_TW_DERIVE64
#define SG_TW_DERIVE64 1
#endif

// Twiddles of stage S of plan<L, L/T> held by one thread: the table entries
// it loads for each butterfly u (nothing for the first stage, Ns = 1).
template <int L, int T, int S, typename R>
struct stage_tw {
  using P = plan<L, L / T>;
  static constexpr bool live = S < P::nstages;
  static constexpr int r = live ? P::radix(S) : 1;
  static constexpr int NB = (L / T) / r;
  static constexpr int Ns = live ? P::ns_before(S) : 1;
  static constexpr bool has = live && Ns > 1;
  static constexpr bool DER = (sizeof(R) == 4 ? SG_TW_DERIVE : SG_TW_DERIVE64) && (r == 8 || r == 16);
  // entries loaded per butterfly: inputs q = 1, 2, 4 (, 8), or every q >= 1
  static constexpr int NL = DER ? (r == 16 ? 4 : 3) : (r > 1 ? r - 1 : 1);
  // loaded one stage ahead when they take few registers, else at the stage
  static constexpr bool early = has && NB * NL * (int)sizeof(cx<R>) <= SG_TW_EARLY_BYTES;
  cx<R> w[early ? NB : 1][early ? NL : 1];
  static __device__ __forceinline__ constexpr int qload(int i) { return DER ? (1 << i) : i + 1; }
  __device__ __forceinline__ cx<R> fetch(const cx<R>* __restrict__ tw, int t, int u, int q) const {
    constexpr int off = P::tw_offset(S);
    const unsigned k = (unsigned)(t + u * T) % (unsigned)Ns;
    return tw[(unsigned)(off + (q - 1) * Ns) + k];
  }
  __device__ __forceinline__ void load(const cx<R>* __restrict__ tw, int t) {
    if constexpr (early) {
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int i = 0; i < NL; ++i) w[u][i] = fetch(tw, t, u, qload(i));
    }
  }
  // loaded entry i of butterfly u: from registers, or loaded now
  __device__ __forceinline__ cx<R> loaded(const cx<R>* __restrict__ tw, int t, int u, int i) const {
    if constexpr (early) return w[u][i];
    else return fetch(tw, t, u, qload(i));
  }
  // all twiddles of butterfly u: o[q] = w_{Ns r}^{k q}, q in [1, r)
  __device__ __forceinline__ void all(const cx<R>* __restrict__ tw, int t, int u, cx<R>* o) const {
    if constexpr (!DER) {
#pragma unroll
      for (int q = 1; q < r; ++q) o[q] = loaded(tw, t, u, q - 1);
    } else {
      o[1] = loaded(tw, t, u, 0);
      o[2] = loaded(tw, t, u, 1);
      o[4] = loaded(tw, t, u, 2);
      o[3] = cmul(o[1], o[2]);
      o[5] = cmul(o[4], o[1]);
      o[6] = cmul(o[4], o[2]);
      if constexpr (r == 16) {
        o[8] = loaded(tw, t, u, 3);
        o[7] = cmulc(o[8], o[1]);  // w^8 conj(w)
        o[9] = cmul(o[8], o[1]);
        o[10] = cmul(o[8], o[2]);
        o[11] = cmul(o[8], o[3]);
        o[12] = cmul(o[8], o[4]);
        o[13] = cmul(o[12], o[1]);
        o[14] = cmul(o[12], o[2]);
        o[15] = cmul(o[8], o[7]);
      } else {
        o[7] = cmul(o[4], o[3]);
      }
    }
  }
};

// One Stockham stage.  v: E registers (strided distribution).  Unless this
// is the last stage, the result is exchanged through lds (L padded slots)
// and v again holds the strided distribution of the stage output.  tw: the
// stage's twiddle table (see plan::tw_offset): consecutive butterflies read
// consecutive entries.
template <bool INV, int L, int T, int r, int Ns, typename R, typename W>
__device__ __forceinline__ void stockham_stage(cx<R>* v, cx<R>* lds, const W& tws, const cx<R>* __restrict__ tw,
                                               int t) {
  constexpr int E = L / T;
  constexpr int NB = E / r;
  constexpr bool last = (Ns * r == L);
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int b = t + u * T;
    cx<R> a[r];
#pragma unroll
    for (int q = 0; q < r; ++q) a[q] = v[u + q * NB];
    if constexpr (Ns > 1) {
      cx<R> w[r];
      tws.all(tw, t, u, w);
#pragma unroll
      for (int q = 1; q < r; ++q) a[q] = INV ? cmulc(a[q], w[q]) : cmul(a[q], w[q]);
    }
    dft<r, INV>(a);
    if constexpr (last) {
      // in place: butterfly u reads and writes the same register slots
#pragma unroll
      for (int q = 0; q < r; ++q) v[u + q * NB] = a[q];
    } else {
      const int base = (b / Ns) * Ns * r + b % Ns;
#pragma unroll
      for (int q = 0; q < r; ++q) lds[pad(base + q * Ns)] = a[q];
    }
  }
  if constexpr (!last) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[pad(t + e * T)];
    __syncthreads();
  }
}

// Stage S onwards; the next stage's twiddles are loaded before this stage's
// butterflies and barriers, so that their latency hides behind them.
template <bool INV, int L, int T, int S, typename R>
__device__ __forceinline__ void fft_stages(cx<R>* v, cx<R>* lds, const cx<R>* __restrict__ tw,
                                           const stage_tw<L, T, S, R>& cur, int t) {
  using P = plan<L, L / T>;
  if constexpr (S < P::nstages) {
    stage_tw<L, T, S + 1, R> nxt;
    nxt.load(tw, t);
    stockham_stage<INV, L, T, P::radix(S), P::ns_before(S)>(v, lds, cur, tw, t);
    fft_stages<INV, L, T, S + 1>(v, lds, tw, nxt, t);
  }
}

// Full length-L transform (unnormalised; INV uses the conjugate twiddles).
// tw: the stage tables of plan<L, L/T>.  All threads of the workgroup must
// call it (it contains barriers).
template <bool INV, int L, int T, typename R>
__device__ __forceinline__ void fft(cx<R>* v, cx<R>* lds, const cx<R>* __restrict__ tw, int t) {
  static_assert(L % T == 0, "L must be a multiple of T");
  stage_tw<L, T, 0, R> s0;  // the first stage has no twiddles
  fft_stages<INV, L, T, 0>(v, lds, tw, s0, t);
}

// Two independent transforms of the same length through the same stages,
// sharing each exchange's barriers (lds0, lds1: separate padded buffers).
template <bool INV, int L, int T, int r, int Ns, typename R, typename W>
__device__ __forceinline__ void stockham_stage2(cx<R>* v0, cx<R>* v1, cx<R>* lds0, cx<R>* lds1, const W& tws,
                                                const cx<R>* __restrict__ tw, int t) {
  constexpr int E = L / T;
  constexpr int NB = E / r;
  constexpr bool last = (Ns * r == L);
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int b = t + u * T;
    cx<R> a0[r], a1[r];
#pragma unroll
    for (int q = 0; q < r; ++q) {
      a0[q] = v0[u + q * NB];
      a1[q] = v1[u + q * NB];
    }
    if constexpr (Ns > 1) {
      cx<R> w[r];
      tws.all(tw, t, u, w);
#pragma unroll
      for (int q = 1; q < r; ++q) {
        a0[q] = INV ? cmulc(a0[q], w[q]) : cmul(a0[q], w[q]);
        a1[q] = INV ? cmulc(a1[q], w[q]) : cmul(a1[q], w[q]);
      }
    }
    dft<r, INV>(a0);
    dft<r, INV>(a1);
    if constexpr (last) {
#pragma unroll
      for (int q = 0; q < r; ++q) {
        v0[u + q * NB] = a0[q];
        v1[u + q * NB] = a1[q];
      }
    } else {
      const int base = (b / Ns) * Ns * r + b % Ns;
#pragma unroll
      for (int q = 0; q < r; ++q) {
        lds0[pad(base + q * Ns)] = a0[q];
        lds1[pad(base + q * Ns)] = a1[q];
      }
    }
  }
  if constexpr (!last) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v0[e] = lds0[pad(t + e * T)];
      v1[e] = lds1[pad(t + e * T)];
    }
    __syncthreads();
  }
}

template <bool INV, int L, int T, int S, typename R>
__device__ __forceinline__ void fft2_stages(cx<R>* v0, cx<R>* v1, cx<R>* lds0, cx<R>* lds1,
                                            const cx<R>* __restrict__ tw, const stage_tw<L, T, S, R>& cur, int t) {
  using P = plan<L, L / T>;
  if constexpr (S < P::nstages) {
    stage_tw<L, T, S + 1, R> nxt;
    nxt.load(tw, t);
    stockham_stage2<INV, L, T, P::radix(S), P::ns_before(S)>(v0, v1, lds0, lds1, cur, tw, t);
    fft2_stages<INV, L, T, S + 1>(v0, v1, lds0, lds1, tw, nxt, t);
  }
}

// fft() on two arrays at once (half the barriers of two calls).
template <bool INV, int L, int T, typename R>
__device__ __forceinline__ void fft2(cx<R>* v0, cx<R>* v1, cx<R>* lds0, cx<R>* lds1, const cx<R>* __restrict__ tw,
                                     int t) {
  static_assert(L % T == 0, "L must be a multiple of T");
  stage_tw<L, T, 0, R> s0;
  fft2_stages<INV, L, T, 0>(v0, v1, lds0, lds1, tw, s0, t);
}

// NA independent transforms of the same length through the same stages,
// sharing each exchange's barriers: v[i] in registers, exchange buffer i at
// lds + i * stride.  W: this stage's twiddles, already loaded.
template <bool INV, int L, int T, int r, int Ns, int NA, typename R, typename W, bool TAIL = true>
__device__ __forceinline__ void stockham_stage_n(cx<R> (&v)[NA][L / T], cx<R>* lds, int stride, const W& tws,
                                                 const cx<R>* __restrict__ tw, int t) {
  constexpr int E = L / T;
  constexpr int NB = E / r;
  constexpr bool last = (Ns * r == L);
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int b = t + u * T;
    cx<R> w[r];
    if constexpr (Ns > 1) tws.all(tw, t, u, w);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      cx<R> a[r];
#pragma unroll
      for (int q = 0; q < r; ++q) a[q] = v[i][u + q * NB];
      if constexpr (Ns > 1) {
#pragma unroll
        for (int q = 1; q < r; ++q) a[q] = INV ? cmulc(a[q], w[q]) : cmul(a[q], w[q]);
      }
      dft<r, INV>(a);
      if constexpr (last) {
#pragma unroll
        for (int q = 0; q < r; ++q) v[i][u + q * NB] = a[q];
      } else {
        const int base = (b / Ns) * Ns * r + b % Ns;
#pragma unroll
        for (int q = 0; q < r; ++q) lds[i * stride + pad(base + q * Ns)] = a[q];
      }
    }
  }
  if constexpr (!last) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int e = 0; e < E; ++e) v[i][e] = lds[i * stride + pad(t + e * T)];
    if constexpr (TAIL) __syncthreads();
  }
}

// Stage S onwards.  The next stage's twiddles are loaded before this
// stage's butterflies and barriers, so that their latency is hidden behind
// them rather than exposed after the barrier.
template <bool INV, int L, int T, int S, int NA, typename R>
__device__ __forceinline__ void fftn_stages(cx<R> (&v)[NA][L / T], cx<R>* lds, int stride,
                                            const cx<R>* __restrict__ tw, const stage_tw<L, T, S, R>& cur, int t) {
  using P = plan<L, L / T>;
  if constexpr (S < P::nstages) {
    stage_tw<L, T, S + 1, R> nxt;
    nxt.load(tw, t);
    stockham_stage_n<INV, L, T, P::radix(S), P::ns_before(S), NA>(v, lds, stride, cur, tw, t);
    fftn_stages<INV, L, T, S + 1, NA>(v, lds, stride, tw, nxt, t);
  }
}

// fft() on NA arrays at once (the barriers of one transform).
template <bool INV, int L, int T, int NA, typename R>
__device__ __forceinline__ void fftn(cx<R> (&v)[NA][L / T], cx<R>* lds, int stride, const cx<R>* __restrict__ tw,
                                     int t) {
  static_assert(L % T == 0, "L must be a multiple of T");
  stage_tw<L, T, 0, R> s0;  // the first stage has no twiddles
  fftn_stages<INV, L, T, 0, NA>(v, lds, stride, tw, s0, t);
}

// fftn() with the exchanges alternating between two sets of NA buffers
// (set s % 2 at lds + (s % 2) * NA * stride): a stage's writes cannot meet a
// slower thread's reads of the previous stage, which used the other set, so
// each exchange needs one barrier instead of two.  One barrier at the end
// lets the caller reuse the buffers.  Needs 2 * NA buffers.
template <bool INV, int L, int T, int S, int NA, typename R>
__device__ __forceinline__ void fftn_pp_stages(cx<R> (&v)[NA][L / T], cx<R>* lds, int stride,
                                               const cx<R>* __restrict__ tw, const stage_tw<L, T, S, R>& cur, int t) {
  using P = plan<L, L / T>;
  if constexpr (S < P::nstages) {
    stage_tw<L, T, S + 1, R> nxt;
    nxt.load(tw, t);
    stockham_stage_n<INV, L, T, P::radix(S), P::ns_before(S), NA, R, stage_tw<L, T, S, R>, false>(
        v, lds + (S % 2) * NA * stride, stride, cur, tw, t);
    fftn_pp_stages<INV, L, T, S + 1, NA>(v, lds, stride, tw, nxt, t);
  }
}
template <bool INV, int L, int T, int NA, typename R>
__device__ __forceinline__ void fftn_pp(cx<R> (&v)[NA][L / T], cx<R>* lds, int stride, const cx<R>* __restrict__ tw,
                                        int t) {
  static_assert(L % T == 0, "L must be a multiple of T");
  stage_tw<L, T, 0, R> s0;
  fftn_pp_stages<INV, L, T, 0, NA>(v, lds, stride, tw, s0, t);
  if constexpr (plan<L, L / T>::nstages > 1) __syncthreads();
}

// Fill the stage tables of plan<L, E> from a table of roots of unity
// (roots(i) = exp(-2 pi i * i / L)); one thread per entry.
template <int L, int E, typename R>
__device__ __forceinline__ void build_stage_twiddles(roots_t<R> roots, cx<R>* out, int idx) {
  using P = plan<L, E>;
#pragma unroll 1
  for (int s = 1; s < P::nstages; ++s) {
    const int r = P::radix(s), Ns = P::ns_before(s), off = P::tw_offset(s);
    if (idx >= off && idx < off + (r - 1) * Ns) {
      const int q = (idx - off) / Ns + 1, k = (idx - off) % Ns;
      out[idx] = roots(k * q * (L / (Ns * r)));
    }
  }
}

}  // namespace sg
