// Column pass for long columns (N = 2048, 4096, 8192) on the four-step transform
// of fft4.hpp: one column of the row spectra per workgroup of N / E threads.
//
// Per column p (a bin of the row transforms; column 0 carries the real bins
// p = 0 and p = M packed as U = C_0 + i C_M):
//   [k >= 3: the y-solve of the interpolation system (Eq. (z_system); its
//    k = 4, 5 counterparts) on the complex row spectra, FP64],
//   forward transform of the column zero-padded to 2N as its even and odd
//   output bins: fe = FFT_N(a), fo = FFT_N(a_j w_2N^j),
//   products with the spectra of w^x and w^y (convolution theorem, Eq. (eqnF)),
//   four inverse transforms cropped to the first N outputs, combined as
//   Y = IFFT_N(G_e) + w_2N^-j IFFT_N(G_o),
//   V(p) = Yx + i Yy and V(2M - p) = conj(Yx) + i conj(Yy), stored in the
//   tiled layout the inverse row pass reads.
// The spectrum tables, their quarter storage and reflection signs, the
// even-k half-cell phases and the packed column are those of the Stockham
// column pass in sg_kernels.hip (same plan-time tables).
//
// LDS: AREAS = 2 gives two exchange areas of two slots each, used in turn,
// so that no exchange needs a barrier before its writes; AREAS = 1 gives one
// area of two slots (FP64, or N = 8192 in FP32), whose exchanges take a
// barrier before their writes as well.
#pragma once
#include "fft4.hpp"
#include "kcommon.hpp"
#include "sg_internal.h"
#include "tridiag.hpp"

namespace sg {

// Stored entry of the real spectrum table for row bin q' of half h (h = 0:
// q = 2q', h = 1: q = 2q'+1) and its sign (+1, or the reflection sign eps
// past q -> 2N - q).
template <typename TO, int N>
__device__ __forceinline__ int fs_tab_index(int qq, int h) {
  return h == 0 ? (qq <= N / 2 ? qq : N - qq) : N / 2 + 1 + (qq < N / 2 ? qq : N - 1 - qq);
}
template <int N>
__device__ __forceinline__ bool fs_tab_direct(int qq, int h) {
  return h == 0 ? qq <= N / 2 : qq < N / 2;
}
// The same two for row bin qq = base + off, base in [0, SPAN) per thread,
// off a compile-time constant per register: where the whole range [off,
// off + SPAN) lies on one side of the reflection, the test and the index
// choice fold at compile time (all but one register of a D3 thread).
template <int N, int SPAN>
__device__ __forceinline__ bool fs_tab_direct_at(int base, int off, int h) {
  const int lim = h == 0 ? N / 2 : N / 2 - 1;  // direct iff qq <= lim
  if (off + SPAN - 1 <= lim) return true;
  if (off > lim) return false;
  return base + off <= lim;
}
template <int N, int SPAN>
__device__ __forceinline__ int fs_tab_index_at(int base, int off, int h) {
  const int lim = h == 0 ? N / 2 : N / 2 - 1;
  const int o = h == 0 ? 0 : N / 2 + 1, m = h == 0 ? N : N - 1;  // reflected entry: o + m - qq
  if (off + SPAN - 1 <= lim) return o + off + base;
  if (off > lim) return o + m - off - base;
  const int qq = base + off;
  return qq <= lim ? o + qq : o + m - qq;
}

// z * i A (A: a double, a float, or a float hi+lo pair), times sgn
__device__ __forceinline__ cx<double> fs_iA(cx<double> z, double a, double sgn) {
  a *= sgn;
  return {-z.y * a, z.x * a};
}
__device__ __forceinline__ cx<float> fs_iA(cx<float> z, float2 a, float sgn) {
  return {-(z.y * a.x + z.y * a.y) * sgn, (z.x * a.x + z.x * a.y) * sgn};
}
__device__ __forceinline__ cx<float> fs_iA(cx<float> z, float a, float sgn) {
  a *= sgn;
  return {-z.y * a, z.x * a};
}

template <typename R>
__device__ __forceinline__ cx<R> fs_half_phase(double frac) {
  double sn, cs;
  sincospi(-frac, &sn, &cs);
  return cx<R>{(R)cs, (R)sn};
}

template <typename R, int N, int E, int SLOTS>
struct colfs_cfg {
  using S = fs_shape<N, E>;
  static constexpr int T = S::T;
  static constexpr int SL = S::SLOT;
  static constexpr int LDS = SLOTS * SL;  // complex elements
  // twiddles and table entries kept in registers when they are cheap (FP32, E = 8)
  static constexpr bool KEEP = sizeof(R) == 4 && E == 8;
};

// MODE: 0 = k 1, 1 = k 2, 2 = k 3, 3 = k 4, 4 = k 5 (as k_col).
// SLOTS: LDS slots of N padded elements.  4: two exchange areas of two slots
// used in turn (no exchange waits before its writes); 2: one area of two
// slots; 1: one slot, every transform exchanged alone.  With fewer than four
// slots, each phase that writes LDS some other wave may still use starts
// with a workgroup barrier.
// COMP: 0 both force components; 1 the x component only, Yx left in V(p);
// 2 the y component, combined with the Yx of a COMP = 1 pass into V(p),
// V(2M - p) (half the registers of COMP 0).  k_colfs_xy runs COMP 1 and 2
// for the same column in one launch, so that the second pass finds the
// column and Yx in L2.
// PF: a workgroup loops over columns b, b + gridDim.x, ... (in the order
// that keeps an XCD's columns together) and loads the next column and its
// table entries while it transforms the current one; the phases w_2N^j stay
// in registers, so that no load in the loop body waits behind the prefetch
// (loads complete in order).  Needs the table entries in registers (KEEP).
// Minimum waves per SIMD the registers of k_colfs must allow: 2 for FP64
// columns of 2048 (two workgroups of four waves per compute unit; left
// alone it takes more than 256 registers, one wave per SIMD), 3 for FP32
// columns of 2048 (three workgroups with two LDS slots each), else no cap.
// SG_FWD_OPQ: see colfs_body
#ifndef SG_FWD_OPQ
#define SG_FWD_OPQ 1
#endif
#ifndef SG_COLFS_WPE_D2048
#define SG_COLFS_WPE_D2048 2
#endif
#ifndef SG_COLFS_WPE_F4096
#define SG_COLFS_WPE_F4096 1
#endif
#ifndef SG_COLFS_WPE_F2048
#define SG_COLFS_WPE_F2048 3
#endif
template <typename R, int N>
struct colfs_wpe {
  static constexpr int value =
      sizeof(R) == 8 ? (N == 2048 ? SG_COLFS_WPE_D2048 : 1)
                     : (N == 4096 ? SG_COLFS_WPE_F4096 : (N == 2048 ? SG_COLFS_WPE_F2048 : 1));
};

// OPQ: the thread index through opaque() (as in the prefetching loop), so
// that a second pass in the same launch recomputes its index arithmetic
// instead of keeping the first pass's live across it.
template <typename R, typename TO, int N, int MODE, int E, int SLOTS, int COMP, bool PF, bool OPQ = false>
__device__ __forceinline__ void colfs_body(const cx<R>* __restrict__ X, cx<R>* __restrict__ V, int M, int tj,
                                           const TO* __restrict__ tox, const TO* __restrict__ toy,
                                           const cx<R>* __restrict__ r2n, const cx<R>* __restrict__ twfs,
                                           const sg_bgrid* __restrict__ bg, cx<R>* smem) {
  constexpr int kind = (MODE == 1 || MODE == 3) ? 1 : 0;
  constexpr bool solve = MODE >= 2;
  constexpr int SYS = MODE == 2 ? 3 : (MODE == 3 ? 4 : 5);
  using C = colfs_cfg<R, N, E, SLOTS>;
  using S = fs_shape<N, E>;
  constexpr int T = C::T, SL = C::SL;
  constexpr int NG = COMP == 0 ? 4 : 2;  // spectra after the products
  static_assert(SLOTS == 4 || SLOTS == 2 || (SLOTS == 1 && COMP != 0), "LDS plan");
  static_assert(S::d3_split_ok(), "D3 index split");
  if (bg) {
    const sg_bgrid d = grid_desc(bg);
    X = reinterpret_cast<const cx<R>*>(d.X);
    V = reinterpret_cast<cx<R>*>(d.V);
    tox = reinterpret_cast<const TO*>(d.tabx);
    toy = reinterpret_cast<const TO*>(d.taby);
  }
  // exchange areas: A0 (slots 0, 1) and A1 (slots 2, 3, or A0 again)
  cx<R>* A0 = smem;
  cx<R>* A1 = SLOTS == 4 ? smem + 2 * SL : smem;
  constexpr bool cautious = SLOTS < 4;
  const int t0 = OPQ ? opaque((int)threadIdx.x) : (int)threadIdx.x;
  constexpr bool pre = C::KEEP;
  static_assert(!PF || (pre && COMP == 0), "the prefetching loop keeps the table entries in registers");
  constexpr int NT = COMP == 0 ? 4 : 2;  // tables used: (x even, y even, x odd, y odd) or one component's halves
  // table of product i: component (COMP 0: i & 1; else COMP - 1), half (COMP 0: i >> 1; else i)
  auto comp_of = [](int i) { return COMP == 0 ? (i & 1) : COMP - 1; };
  auto half_of = [](int i) { return COMP == 0 ? (i >> 1) : i; };
  // ---- loads of a column: the column (chunk of E per thread for the solve,
  // else D1); the spectrum-table entries of this thread's D3 bins
  auto load_col = [&](int t, int cc, cx<R> (&aa)[E]) {
    const cx<R>* col = X + (int64_t)cc * N;
#pragma unroll
    for (int e = 0; e < E; ++e) aa[e] = col[(unsigned)(solve ? t * E + e : S::d1_index(t, e))];
  };
  auto load_tab = [&](int t, int cc, TO (&tt)[pre ? NT : 1][pre ? E : 1]) {
    if constexpr (pre) {
      const TO* rx = tox + (int64_t)cc * (N + 1);
      const TO* ry = toy + (int64_t)cc * (N + 1);
      const int db = S::d3_base(t);
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int r = 0; r < E; ++r)
          tt[i][r] = (comp_of(i) ? ry : rx)[(unsigned)fs_tab_index_at<N, S::D3_SPAN>(db, S::d3_off(r), half_of(i))];
    }
  };
  fs_tw<N, E, R, C::KEEP> tw;
  tw.init(twfs, t0);
  cx<R> w2k[PF ? E : 1];  // w_2N^j of this thread's D1 elements, kept by the loop
  if constexpr (PF) {
#pragma unroll
    for (int e = 0; e < E; ++e) w2k[e] = r2n[(unsigned)S::d1_index(t0, e)];
  }
  cx<R> a[E];
  int it = blockIdx.x;
  load_col(t0, xcd_tile(it, M), a);
  for (;;) {
  // the thread index through opaque(): the per-thread index arithmetic of
  // the loop body stays in the body instead of being hoisted out of the loop
  // and held in registers across it
  const int t = PF ? opaque(t0) : t0;
  // a copy of t per phase (SG_FWD_OPQ), as in the adjoint: the products and
  // the output recompute their indices instead of keeping the load's
  auto fresh_t = [&]() { return SG_FWD_OPQ ? opaque(t) : t; };
  auto w2n_at = [&](int tt, int e) -> cx<R> {
    if constexpr (PF) return w2k[e];
    else return r2n[(unsigned)opaque(S::d1_index(tt, e))];
  };
  const int c = xcd_tile(it, M);
  const bool packed = (c == 0);
  const TO* rowx = tox + (int64_t)c * (N + 1);
  const TO* rowy = toy + (int64_t)c * (N + 1);
  const int itn = it + (int)gridDim.x;
  // this column's table entries first, then (PF) the next column: loads
  // complete in order, so waiting for the entries leaves the prefetch in
  // flight
  TO tv[pre ? NT : 1][pre ? E : 1];
  load_tab(t, c, tv);
  cx<R> an[PF ? E : 1];
  if constexpr (PF) {
    // unconditional (the last column reloads itself), so that the loads
    // issue together without a branch
    load_col(t, xcd_tile(itn < M ? itn : it, M), an);
  }

  // ---- y-solve (FP64, chunks), then into D1 through slot 0
  if constexpr (solve) {
    double2 d[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
      d[e] = make_double2(band_scale(SYS) * (double)a[e].x, band_scale(SYS) * (double)a[e].y);
    // the solve's LDS: the last slot (or the only one, then with its trailing barrier)
    band_solve<SYS, E, T, double2, SLOTS == 1>(d, t, smem + (SLOTS - 1) * SL);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      // chunk element j = t E + e goes to the D1 position of j
      const int j = t * E + e;
      const int n1 = j % S::B1, n2 = j / S::B1;
      const int l = n2 % S::LB2, ep = n2 / S::LB2;
      const int tp = (n1 / S::S1) * 64 + n1 % S::S1 + S::S1 * l;
      smem[fspad(tp * E + ep)] = cx<R>{(R)d[e].x, (R)d[e].y};
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = smem[fspad(t * E + e)];
  }

  // ---- forward: fe = FFT(a), fo = FFT(a w_2N^j) (D1 -> D3)
  cx<R> f[2][E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    f[0][e] = a[e];
    f[1][e] = cmul(a[e], w2n_at(t, e));
  }
  if constexpr (SLOTS == 1) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cx<R> fh[1][E];
#pragma unroll
      for (int e = 0; e < E; ++e) fh[0][e] = f[h][e];
      if (h) __syncthreads();  // the slot's last step-3 transposes
      fs_step1_fwd<N, E, 1>(fh, smem, tw, t);
      fs_cross13<N, E, 1>(fh, smem, true, t);
      fs_step3_fwd<N, E, 1>(fh, smem, tw, t);
#pragma unroll
      for (int e = 0; e < E; ++e) f[h][e] = fh[0][e];
    }
  } else {
    fs_step1_fwd<N, E, 2>(f, A0, tw, t);
    fs_cross13<N, E, 2>(f, A1, cautious, t);
    fs_step3_fwd<N, E, 2>(f, A1, tw, t);
  }

  // ---- products: g = (x even, y even, x odd, y odd), or (even, odd) of
  // one component
  cx<R> g[NG][E];
  constexpr R ex = kind == 1 ? (R)-1 : (R)1;  // reflection sign of the x table (y: -ex)
  cx<R> php{(R)1, (R)0}, rho{(R)1, (R)0};
  if constexpr (kind == 1) {
    php = fs_half_phase<R>((double)c / (2.0 * M));
    rho = fs_half_phase<R>(1.0 / (2.0 * N));
  }
  if (!packed) {
    const int tq = fresh_t();
    if constexpr (kind == 1) {
      // even k: the bin phases exp(-i pi (p/2M + q/2N)), shared by x and y
      const cx<R> pho = cmul(php, rho);
#pragma unroll
      for (int r = 0; r < E; ++r) {
        // exp(-i pi q'/N); without the prefetched tables (long columns, FP64)
        // each load is issued at its use, to bound the registers in flight
        const cx<R> wq = r2n[(unsigned)(pre ? S::d3_index(tq, r) : opaque(S::d3_index(tq, r)))];
        f[0][r] = cmul(f[0][r], cmul(wq, php));
        f[1][r] = cmul(f[1][r], cmul(wq, pho));
      }
    }
    const int db = S::d3_base(tq);
#pragma unroll
    for (int i = 0; i < NG; ++i)
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int h = half_of(i), cy = comp_of(i);
        const R sgn = fs_tab_direct_at<N, S::D3_SPAN>(db, S::d3_off(r), h) ? (R)1 : (cy ? -ex : ex);
        TO ent;
        if constexpr (pre) ent = tv[i][r];
        else ent = (cy ? rowy : rowx)[(unsigned)opaque(fs_tab_index_at<N, S::D3_SPAN>(db, S::d3_off(r), h))];
        g[i][r] = fs_iA(f[h][r], ent, sgn);
      }
  } else {
    // packed column: U(q) holds C_0 + i C_M; C_0 = (U(q) + conj U(-q)) / 2,
    // C_M = (U(q) - conj U(-q)) / (2i); the products re-packed as G_0 + i G_M.
    // U(-q) of half 0 sits at q' -> N - q', of half 1 at q' -> N - 1 - q'.
    const TO* row0x = tox;
    const TO* row0y = toy;
    const TO* rowMx = tox + (int64_t)M * (N + 1);
    const TO* rowMy = toy + (int64_t)M * (N + 1);
    // the partner values through slots 0, 1 (A0, free since the forward
    // exchange when there are four slots; slot 0 for each half in turn when
    // there is one)
    auto product = [&](int h, const cx<R>* part) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int qq = S::d3_index(t, r);
        const int qm = h == 0 ? (qq == 0 ? 0 : N - qq) : N - 1 - qq;
        const cx<R> u = f[h][r], um = conj(part[fspad(qm)]);
        cx<R> c0v{(R)0.5 * (u.x + um.x), (R)0.5 * (u.y + um.y)};
        cx<R> cmv{(R)0.5 * (u.y - um.y), (R)-0.5 * (u.x - um.x)};
        if constexpr (kind == 1) {
          // phases of bins p = 0 (1) and p = M (-i) times that of row bin q
          const cx<R> wq = r2n[(unsigned)qq];
          const cx<R> ph0 = h ? cmul(wq, rho) : wq;
          c0v = cmul(c0v, ph0);
          cmv = cmul(cmv, cx<R>{ph0.y, -ph0.x});
        }
        const bool dir = fs_tab_direct<N>(qq, h);
        const int ti = fs_tab_index<TO, N>(qq, h);
        const R sx = dir ? (R)1 : ex, sy = dir ? (R)1 : -ex;
        if constexpr (COMP != 2) {
          const cx<R> x0 = fs_iA(c0v, row0x[ti], sx), xm = fs_iA(cmv, rowMx[ti], sx);
          g[COMP == 0 ? 2 * h : h][r] = cx<R>{x0.x - xm.y, x0.y + xm.x};
        }
        if constexpr (COMP != 1) {
          const cx<R> y0 = fs_iA(c0v, row0y[ti], sy), ym = fs_iA(cmv, rowMy[ti], sy);
          g[COMP == 0 ? 2 * h + 1 : h][r] = cx<R>{y0.x - ym.y, y0.y + ym.x};
        }
      }
    };
    if constexpr (SLOTS >= 2) {
      if (cautious) __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < E; ++r) smem[h * SL + fspad(S::d3_index(t, r))] = f[h][r];
      __syncthreads();
      product(0, smem);
      product(1, smem + SL);
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < E; ++r) smem[fspad(S::d3_index(t, r))] = f[h][r];
        __syncthreads();
        product(h, smem);
      }
    }
    __syncthreads();
  }

  // ---- inverse (D3 -> D1)
  if constexpr (COMP == 0) {
    // step 3 of all four (two at a time, in this wave's part of A1), then the
    // two exchanges and step 1
    cx<R> g01[2][E], g23[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      g01[0][e] = g[0][e];
      g01[1][e] = g[1][e];
      g23[0][e] = g[2][e];
      g23[1][e] = g[3][e];
    }
    if (cautious) __syncthreads();
    fs_step3_inv<N, E, 2>(g01, A1, tw, t);
    fs_step3_inv<N, E, 2>(g23, A1, tw, t);
    fs_cross31<N, E, 2>(g01, A0, cautious, tw, t);
    fs_step1_inv<N, E, 2>(g01, A0, tw, t);
    fs_cross31<N, E, 2>(g23, A1, cautious, tw, t);
    fs_step1_inv<N, E, 2>(g23, A1, tw, t);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      g[0][e] = g01[0][e];
      g[1][e] = g01[1][e];
      g[2][e] = g23[0][e];
      g[3][e] = g23[1][e];
    }
  } else if constexpr (SLOTS == 2) {
    __syncthreads();
    fs_step3_inv<N, E, 2>(g, A0, tw, t);
    fs_cross31<N, E, 2>(g, A0, true, tw, t);
    fs_step1_inv<N, E, 2>(g, A0, tw, t);
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cx<R> gh[1][E];
#pragma unroll
      for (int e = 0; e < E; ++e) gh[0][e] = g[h][e];
      __syncthreads();
      fs_step3_inv<N, E, 1>(gh, smem, tw, t);
      fs_cross31<N, E, 1>(gh, smem, true, tw, t);
      fs_step1_inv<N, E, 1>(gh, smem, tw, t);
#pragma unroll
      for (int e = 0; e < E; ++e) g[h][e] = gh[0][e];
    }
  }

  // ---- Y = IFFT(G_e) + w_2N^-j IFFT(G_o); V(c) = Yx + i Yy, V(2M - c) =
  // conj(Yx) + i conj(Yy); packed: V(0) = Re Yx + i Re Yy, V(M) = Im Yx + i Im Yy.
  // V(p, j) at ((j/tj*2 + p%2)*M + p/2)*tj + j%tj.
  const int pa = c, pb = packed ? M : 2 * M - c;
  cx<R>* va = V + (int64_t)(pa & 1) * M * tj + (int64_t)(pa >> 1) * tj;
  cx<R>* vb = V + (int64_t)(pb & 1) * M * tj + (int64_t)(pb >> 1) * tj;
  const int64_t jstride = (int64_t)2 * M * tj;
  const int ts = fresh_t();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = S::d1_index(ts, e);
    const cx<R> w = w2n_at(ts, e);
    const int64_t o = (int64_t)(j / tj) * jstride + (j % tj);
    if constexpr (COMP == 1) {
      va[o] = g[0][e] + cmulc(g[1][e], w);  // Yx, kept for the y launch
    } else {
      const cx<R> yx = COMP == 0 ? g[0][e] + cmulc(g[2][e], w) : va[o];
      const cx<R> yy = COMP == 0 ? g[1][e] + cmulc(g[3][e], w) : g[0][e] + cmulc(g[1][e], w);
      cx<R> v1, v2;
      if (packed) {
        v1 = cx<R>{yx.x, yy.x};
        v2 = cx<R>{yx.y, yy.y};
      } else {
        v1 = cx<R>{yx.x - yy.y, yx.y + yy.x};
        v2 = cx<R>{yx.x + yy.y, yy.x - yx.y};
      }
      va[o] = v1;
      vb[o] = v2;
    }
  }
  if constexpr (!PF) {
    break;
  } else {
    if (itn >= M) break;
    it = itn;
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = an[e];
    __syncthreads();  // this column's last LDS reads come before the next column's writes
  }
  }
}

template <typename R, typename TO, int N, int MODE, int E, int SLOTS, int COMP, bool PF = false>
__global__ void __launch_bounds__(N / E) SG_WAVES_PER_EU(colfs_wpe<R, N>::value)
    k_colfs(const cx<R>* __restrict__ X, cx<R>* __restrict__ V, int M, int tj, const TO* __restrict__ tox,
            const TO* __restrict__ toy, const cx<R>* __restrict__ r2n, const cx<R>* __restrict__ twfs,
            const sg_bgrid* __restrict__ bg) {
  __shared__ cx<R> smem[colfs_cfg<R, N, E, SLOTS>::LDS];
  colfs_body<R, TO, N, MODE, E, SLOTS, COMP, PF>(X, V, M, tj, tox, toy, r2n, twfs, bg, smem);
}

// Both force components of a column in one launch: the x pass (Yx into
// V(p)), a barrier (the LDS of the first pass is the second's), then the y
// pass, which rereads the column and reads Yx back, each thread the
// elements it wrote itself, mostly from L2.
template <typename R, typename TO, int N, int MODE, int E, int SLOTS>
__global__ void __launch_bounds__(N / E) SG_WAVES_PER_EU(colfs_wpe<R, N>::value)
    k_colfs_xy(const cx<R>* __restrict__ X, cx<R>* __restrict__ V, int M, int tj, const TO* __restrict__ tox,
               const TO* __restrict__ toy, const cx<R>* __restrict__ r2n, const cx<R>* __restrict__ twfs,
               const sg_bgrid* __restrict__ bg) {
  __shared__ cx<R> smem[colfs_cfg<R, N, E, SLOTS>::LDS];
  colfs_body<R, TO, N, MODE, E, SLOTS, 1, false, true>(X, V, M, tj, tox, toy, r2n, twfs, bg, smem);
  __syncthreads();
  colfs_body<R, TO, N, MODE, E, SLOTS, 2, false, true>(X, V, M, tj, tox, toy, r2n, twfs, bg, smem);
}

// Plan-time spectrum columns of the long columns (FP64): column c of the
// row spectra S of the padded weight table (2N values), its 2N-point
// transform as even bins FFT_N(lo + hi) and odd bins FFT_N((lo - hi) w_2N^j),
// stored in the form the column passes read (see k_spec_col in
// sg_kernels.hip): odd k A = Im W, even k A = Im(W conj(ph)), scaled, on the
// quarter q' <= N/2 (half 0), q' < N/2 (half 1).  One slot of LDS; the two
// halves one after the other.
template <int N, int E>
__global__ void __launch_bounds__(N / E)
    k_specfs(const cx<double>* __restrict__ Sg, int M, void* __restrict__ tab, int kind, int fp32, double scale,
             const cx<double>* __restrict__ r2n, const cx<double>* __restrict__ twfs) {
  using S = fs_shape<N, E>;
  __shared__ cx<double> smem[S::SLOT];
  const int t = threadIdx.x;
  const int c = blockIdx.x;
  fs_tw<N, E, double, false> tw;
  tw.init(twfs, t);
  const cx<double>* col = Sg + (int64_t)c * (2 * N);
  for (int h = 0; h < 2; ++h) {
    cx<double> f[1][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = S::d1_index(t, e);
      const cx<double> lo = col[j], hi = col[j + N];
      f[0][e] = h ? cmul(lo - hi, r2n[(unsigned)j]) : lo + hi;
    }
    __syncthreads();  // the slot's last use (the previous half)
    fs_step1_fwd<N, E, 1>(f, smem, tw, t);
    fs_cross13<N, E, 1>(f, smem, true, t);
    fs_step3_fwd<N, E, 1>(f, smem, tw, t);
    // the packed column 0 needs U(-q): through the slot
    if (c == 0) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < E; ++r) smem[fspad(S::d3_index(t, r))] = f[0][r];
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int qq = S::d3_index(t, r);
      const bool keep = h == 0 ? qq <= N / 2 : qq < N / 2;
      cx<double> vals[2];
      int rows[2];
      int nv = 1;
      if (c == 0) {
        const int qm = h == 0 ? (qq == 0 ? 0 : N - qq) : (N - 1 - qq);
        const cx<double> u = f[0][r], um = conj(smem[fspad(qm)]);
        vals[0] = cx<double>{0.5 * (u.x + um.x), 0.5 * (u.y + um.y)};
        vals[1] = cx<double>{0.5 * (u.y - um.y), -0.5 * (u.x - um.x)};
        rows[0] = 0;
        rows[1] = M;
        nv = 2;
      } else {
        vals[0] = f[0][r];
        rows[0] = c;
      }
      if (!keep) continue;
      for (int v = 0; v < nv; ++v) {
        const cx<double> w = vals[v] * scale;
        double a = w.y;
        if (kind == 1) {
          double sn, cs;
          sincospi((double)rows[v] / (2.0 * M) + (double)(2 * qq + h) / (2.0 * N), &sn, &cs);
          a = w.y * cs + w.x * sn;
        }
        const int64_t idx = (int64_t)rows[v] * (N + 1) + (h == 0 ? qq : N / 2 + 1 + qq);
        if (fp32 == 1) {
          const float hv = (float)a;
          reinterpret_cast<float2*>(tab)[idx] = make_float2(hv, (float)(a - (double)hv));
        } else if (fp32 == 2) {
          reinterpret_cast<float*>(tab)[idx] = (float)a;
        } else {
          reinterpret_cast<double*>(tab)[idx] = a;
        }
      }
    }
  }
}

// Adjoint column pass for the long columns: the transposed convolution of
// the gradients (gx, gy) with the weights (products with the conjugate
// spectra, conj(i A) = -i A, summed over both components), cropped to N,
// then the y-solve of the interpolation system (symmetric, so its own
// transpose).  Xx, Xy: row spectra of gx, gy (column-major like X); Y: the
// packed row spectra of gC in tiles of tj rows, bin p of row j at
// ((j/tj*2 + p%2)*(M/2) + p/2)*tj + j%tj.  SLOTS (1 or 2) arrays go through
// each exchange; every exchange waits for the area to be free.
// SG_ADJ_OPQ: each phase (forward loads, products, output) takes the thread
// index through its own opaque move, so that its per-register indices are
// recomputed there instead of held in registers across the kernel.
#ifndef SG_ADJ_OPQ
#define SG_ADJ_OPQ 1
#endif
template <typename R, typename TO, int N, int MODE, int E, int SLOTS>
__global__ void __launch_bounds__(N / E)
    k_colfs_adj(const cx<R>* __restrict__ Xx, const cx<R>* __restrict__ Xy, cx<R>* __restrict__ Y, int M, int tj,
                const TO* __restrict__ tox, const TO* __restrict__ toy, const cx<R>* __restrict__ r2n,
                const cx<R>* __restrict__ twfs, const sg_bgrid* __restrict__ bg) {
  constexpr int kind = (MODE == 1 || MODE == 3) ? 1 : 0;
  constexpr bool solve = MODE >= 2;
  constexpr int SYS = MODE == 2 ? 3 : (MODE == 3 ? 4 : 5);
  using S = fs_shape<N, E>;
  constexpr int T = S::T, SL = S::SLOT;
  static_assert(SLOTS == 1 || SLOTS == 2, "LDS plan");
  if (bg) {  // batched: gx spectra in X, gy spectra in the first half of V, output in its second half
    const sg_bgrid d = grid_desc(bg);
    Xx = reinterpret_cast<const cx<R>*>(d.X);
    Xy = reinterpret_cast<const cx<R>*>(d.V);
    Y = reinterpret_cast<cx<R>*>(d.V) + (int64_t)M * N;
    tox = reinterpret_cast<const TO*>(d.tabx);
    toy = reinterpret_cast<const TO*>(d.taby);
  }
  __shared__ cx<R> smem[SLOTS * SL];
  const int t = threadIdx.x;
  const int c = xcd_tile(blockIdx.x, gridDim.x);
  const bool packed = (c == 0);
  fs_tw<N, E, R, false> tw;
  tw.init(twfs, t);
  const cx<R>* colx = Xx + (int64_t)c * N;
  const cx<R>* coly = Xy + (int64_t)c * N;
  const TO* rowx = tox + (int64_t)c * (N + 1);
  const TO* rowy = toy + (int64_t)c * (N + 1);
  constexpr R ex = kind == 1 ? (R)-1 : (R)1;  // reflection sign of the x table (y: -ex)
  cx<R> php{(R)1, (R)0}, rho{(R)1, (R)0};
  if constexpr (kind == 1) {
    php = fs_half_phase<R>((double)c / (2.0 * M));
    rho = fs_half_phase<R>(1.0 / (2.0 * N));
  }
  // forward transforms of one half of both components (D1 -> D3)
  auto fresh_t = [&]() { return SG_ADJ_OPQ ? opaque(t) : t; };
  auto forward = [&](int h, cx<R> (&fx)[E], cx<R> (&fy)[E]) {
    const int tl = fresh_t();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = S::d1_index(tl, e);
      const cx<R> w = h ? r2n[(unsigned)opaque(j)] : cx<R>{(R)1, (R)0};
      fx[e] = cmul(colx[(unsigned)j], w);
      fy[e] = cmul(coly[(unsigned)j], w);
    }
    if constexpr (SLOTS == 2) {
      cx<R> f2[2][E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        f2[0][e] = fx[e];
        f2[1][e] = fy[e];
      }
      __syncthreads();
      fs_step1_fwd<N, E, 2>(f2, smem, tw, t);
      fs_cross13<N, E, 2>(f2, smem, true, t);
      fs_step3_fwd<N, E, 2>(f2, smem, tw, t);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        fx[e] = f2[0][e];
        fy[e] = f2[1][e];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        cx<R> f1[1][E];
#pragma unroll
        for (int e = 0; e < E; ++e) f1[0][e] = i ? fy[e] : fx[e];
        __syncthreads();
        fs_step1_fwd<N, E, 1>(f1, smem, tw, t);
        fs_cross13<N, E, 1>(f1, smem, true, t);
        fs_step3_fwd<N, E, 1>(f1, smem, tw, t);
#pragma unroll
        for (int e = 0; e < E; ++e) (i ? fy : fx)[e] = f1[0][e];
      }
    }
  };
  // conjugate-spectrum products of one half, summed over the components
  auto products = [&](int h, const cx<R> (&fx)[E], const cx<R> (&fy)[E], cx<R> (&hh)[E]) {
    if (!packed) {
      const int tl = fresh_t();
      const int db = S::d3_base(tl);
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int qq = S::d3_index(tl, r);
        cx<R> zx = fx[r], zy = fy[r];
        if constexpr (kind == 1) {
          const cx<R> wq = r2n[(unsigned)opaque(qq)];
          const cx<R> ph = cmul(wq, h ? cmul(php, rho) : php);
          zx = cmulc(zx, ph);
          zy = cmulc(zy, ph);
        }
        const bool dir = fs_tab_direct_at<N, S::D3_SPAN>(db, S::d3_off(r), h);
        const int ti = fs_tab_index_at<N, S::D3_SPAN>(db, S::d3_off(r), h);
        const R sx = dir ? (R)-1 : -ex, sy = dir ? (R)-1 : ex;  // conj(i A) = -i A
        hh[r] = fs_iA(zx, rowx[(unsigned)opaque(ti)], sx) + fs_iA(zy, rowy[(unsigned)opaque(ti)], sy);
      }
    } else {
      // each spectrum U carries bins p = 0 and p = M: split both through the
      // two slots (or the one slot twice)
      cx<R> umx[E], umy[E];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (SLOTS == 2 && i == 1) break;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int q = S::d3_index(t, r);
          if (SLOTS == 2) {
            smem[fspad(q)] = fx[r];
            smem[SL + fspad(q)] = fy[r];
          } else {
            smem[fspad(q)] = i ? fy[r] : fx[r];
          }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int qq = S::d3_index(t, r);
          const int qm = h == 0 ? (qq == 0 ? 0 : N - qq) : N - 1 - qq;
          if (SLOTS == 2) {
            umx[r] = conj(smem[fspad(qm)]);
            umy[r] = conj(smem[SL + fspad(qm)]);
          } else if (i == 0) {
            umx[r] = conj(smem[fspad(qm)]);
          } else {
            umy[r] = conj(smem[fspad(qm)]);
          }
        }
      }
      const TO* row0x = tox;
      const TO* row0y = toy;
      const TO* rowMx = tox + (int64_t)M * (N + 1);
      const TO* rowMy = toy + (int64_t)M * (N + 1);
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int qq = S::d3_index(t, r);
        const cx<R> ux = fx[r], uy = fy[r];
        cx<R> x0v{(R)0.5 * (ux.x + umx[r].x), (R)0.5 * (ux.y + umx[r].y)};
        cx<R> xmv{(R)0.5 * (ux.y - umx[r].y), (R)-0.5 * (ux.x - umx[r].x)};
        cx<R> y0v{(R)0.5 * (uy.x + umy[r].x), (R)0.5 * (uy.y + umy[r].y)};
        cx<R> ymv{(R)0.5 * (uy.y - umy[r].y), (R)-0.5 * (uy.x - umy[r].x)};
        if constexpr (kind == 1) {
          const cx<R> wq = r2n[(unsigned)qq];
          const cx<R> ph0 = h ? cmul(wq, rho) : wq;  // bins p = 0 and p = M (-i ph0)
          const cx<R> phm{ph0.y, -ph0.x};
          x0v = cmulc(x0v, ph0);
          y0v = cmulc(y0v, ph0);
          xmv = cmulc(xmv, phm);
          ymv = cmulc(ymv, phm);
        }
        const bool dir = fs_tab_direct<N>(qq, h);
        const int ti = fs_tab_index<TO, N>(qq, h);
        const R sx = dir ? (R)-1 : -ex, sy = dir ? (R)-1 : ex;
        const cx<R> h0 = fs_iA(x0v, row0x[ti], sx) + fs_iA(y0v, row0y[ti], sy);
        const cx<R> hm = fs_iA(xmv, rowMx[ti], sx) + fs_iA(ymv, rowMy[ti], sy);
        hh[r] = cx<R>{h0.x - hm.y, h0.y + hm.x};
      }
    }
  };

  cx<R> hs[2][E];
  {
    cx<R> fx[E], fy[E];
    forward(0, fx, fy);
    products(0, fx, fy, hs[0]);
    forward(1, fx, fy);
    products(1, fx, fy, hs[1]);
  }
  // inverse of both halves (D3 -> D1); acc = IFFT(H_e) + w_2N^-j IFFT(H_o)
  if constexpr (SLOTS == 2) {
    __syncthreads();
    fs_step3_inv<N, E, 2>(hs, smem, tw, t);
    fs_cross31<N, E, 2>(hs, smem, true, tw, t);
    fs_step1_inv<N, E, 2>(hs, smem, tw, t);
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cx<R> g1[1][E];
#pragma unroll
      for (int e = 0; e < E; ++e) g1[0][e] = hs[h][e];
      __syncthreads();
      fs_step3_inv<N, E, 1>(g1, smem, tw, t);
      fs_cross31<N, E, 1>(g1, smem, true, tw, t);
      fs_step1_inv<N, E, 1>(g1, smem, tw, t);
#pragma unroll
      for (int e = 0; e < E; ++e) hs[h][e] = g1[0][e];
    }
  }
  cx<R> acc[E];
  const int to = fresh_t();
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = hs[0][e] + cmulc(hs[1][e], r2n[(unsigned)opaque(S::d1_index(to, e))]);
  cx<R>* out = Y + (int64_t)(c & 1) * (M / 2) * tj + (int64_t)(c >> 1) * tj;
  const int64_t jstride = (int64_t)M * tj;
  if constexpr (solve) {
    // D1 -> chunks of E (thread t: rows [t E, (t+1) E)) through slot 0, then
    // the y-solve (its LDS in the same slot, after the barrier)
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) smem[fspad(S::d1_index(to, e))] = acc[e];
    __syncthreads();
    double2 d[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<R> v = smem[fspad(t * E + e)];
      d[e] = make_double2(band_scale(SYS) * (double)v.x, band_scale(SYS) * (double)v.y);
    }
    __syncthreads();
    band_solve<SYS, E, T, double2, false>(d, t, smem);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = t * E + e;
      out[(int64_t)(j / tj) * jstride + (j % tj)] = cx<R>{(R)d[e].x, (R)d[e].y};
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = S::d1_index(to, e);
      out[(int64_t)(j / tj) * jstride + (j % tj)] = acc[e];
    }
  }
}

}  // namespace sg
