// Column pass for columns of N = 3 L (FP32-split), L = 512 (N = 1536) or 256
// (N = 768), on three waves: a radix-3 step across the waves and, per wave, a
// transform of length L that stays inside the wave: for 512 the four-step
// transform of fft4.hpp (fs_shape<512, 8>: step 1 is eight 64-point
// transforms on 8-lane groups, step 3 one 8-point DFT per lane in registers),
// for 256 four radix-4 Stockham stages.
//
// With w_L = exp(-2 pi i / L), n, k < L, r, q < 3:
//   forward (decimation in frequency): X[3k + q] = DFT_L(y_q)[k],
//     y_q[n] = w_N^(n q) sum_r w_3^(r q) x[n + L r];
//   inverse (decimation in time): x[n + L r] = sum_q w_3^(-r q) u_q[n],
//     u_q[n] = w_N^(-n q) IDFT_L(X[3 . + q])[n].
// Wave q computes y_q / u_q; thread t = 64 q + lane holds element e of the
// sub-transform at n = lane + 64 e (e < E = L / 64) and, after the forward,
// register r at k = lane + 64 r, i.e. bin 3 (lane + 64 r) + q.
//
// The column is otherwise processed as in colfs.hpp (y-solve, forward of the
// zero-padded 2N column as even and odd bins, products with the spectra,
// four inverses cropped to N, V(p) and V(2M - p) in the tiled layout):
//  - the odd-bin input x_j w_2N^j shares the radix-3 reads of x: its radix-3
//    weights are (w_6 w_3^q)^r, its twiddle w_2N^(n (2q + 1));
//  - the crop's w_2N^-j, j = n + L r, splits into w_2N^-n, applied with the
//    inverse's twiddle by the writer, and w_2N^(-L r) = w_6^-r, applied by
//    the reader.
// LDS: four slots of one padded column.  Slot 0 holds x for the forward
// radix-3 step, slots 2 and 3 the y-solve's scratch and then the waves'
// sub-transform areas ([L q, L q + L) of each slot, touched by wave q only),
// all four the inverse radix-3 exchange.  Workgroup barriers: after x is
// written, before and after the inverse exchange, and those of the y-solve.
#pragma once
#include <type_traits>

#include "colfs.hpp"

namespace sg {

// Shape per sub-transform length L (512 for columns of 1536, 256 for 768):
// three waves of 64 lanes, E = L / 64 elements per lane
template <int L>
struct c3_shape {
  static constexpr int N = 3 * L;        // column length
  static constexpr int E = L / 64;       // elements per thread
  static constexpr int T = 3 * 64;       // threads per column
  static constexpr int SL = fspad(N);    // slot (complex elements)
  static_assert(L == 512 || L == 256, "sub-transform lengths");
};
constexpr int kC3T = 3 * 64;

// Minimum waves per SIMD the registers of k_colfs3 must allow (three
// workgroups of three waves per compute unit fit its LDS)
#ifndef SG_COLFS3_WPE
#define SG_COLFS3_WPE 3
#endif
// 1: the spectrum-table entries are loaded with the column (registers); 0:
// at the products
#ifndef SG_COLFS3_PRE
#define SG_COLFS3_PRE 0
#endif

// sum_r c^r x_r for the radix-3 weight c = exp(-2 pi i m / 6), m in [0, 6)
// (m even: the weights w_3^q of the plain input; m odd: those of the
// twisted input)
template <int m, typename R>
__device__ __forceinline__ cx<R> c3_sum(cx<R> x0, cx<R> x1, cx<R> x2) {
  constexpr R h = (R)0.5, s = (R)0.86602540378443864676;  // cos, sin of pi / 3
  if constexpr (m == 0) {
    return x0 + x1 + x2;
  } else if constexpr (m == 3) {  // c = -1
    return x0 - x1 + x2;
  } else {
    // c = a + i b, c^2 = a2 + i b2 (a, b from the table of sixth roots)
    constexpr R a = m == 1 ? h : (m == 2 ? -h : (m == 4 ? -h : h));
    constexpr R b = m == 1 ? -s : (m == 2 ? -s : (m == 4 ? s : s));
    constexpr R a2 = a * a - b * b, b2 = 2 * a * b;
    return cx<R>{x0.x + a * x1.x - b * x1.y + a2 * x2.x - b2 * x2.y,
                 x0.y + a * x1.y + b * x1.x + a2 * x2.y + b2 * x2.x};
  }
}
// f(integral_constant<q>) for the wave-uniform q in [0, 3): each wave runs a
// radix-3 phase compiled for its own q, straight-line code whose loads can
// issue together (a branch per element would split them)
template <typename F>
__device__ __forceinline__ void c3_wave(int q, F f) {
  if (q == 0) f(std::integral_constant<int, 0>{});
  else if (q == 1) f(std::integral_constant<int, 1>{});
  else f(std::integral_constant<int, 2>{});
}

// Forward 512-point transform of NA arrays on one wave: D1 (element e at
// n = lane + 64 e) -> D3 (register r at k = lane + 64 r).  area: this wave's
// part of the first array's slot (array i at area + i * SL).
template <int SL, int NA, typename R, typename TW>
__device__ __forceinline__ void c3_sub_fwd(cx<R> (&v)[NA][8], cx<R>* area, const TW& tw, int lane) {
  constexpr int E = 8;
  const int s = lane % 8, l = lane / 8;
  // step 1: 64-point transforms over n2 for n1 = s, then w_512^(n1 k2)
  fs_sub_fwd<false, E, 8, SL, NA>(v, area, s * 64, tw.set1(), l);
  const auto to = tw.outer();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const cx<R> w = to[r];
#pragma unroll
    for (int i = 0; i < NA; ++i) v[i][r] = cmul(v[i][r], w);
  }
  // exchange within the wave: register b of lane (n1 = s, k2 = l + 8 b) to
  // index k2 * 8 + n1 = lane + 64 b; read back n1 = e of k2 = lane
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int b = 0; b < E; ++b) area[i * SL + fspad(lane) + fspad(64 * b)] = v[i][b];
  wave_sync();
  const cx<R>* rd = area + fspad(8 * lane);
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int e = 0; e < E; ++e) v[i][e] = rd[i * SL + e];
  // step 3: the 8-point DFT over n1 in registers (register r: k1 = r)
#pragma unroll
  for (int i = 0; i < NA; ++i) dft<E, false>(v[i]);
  wave_sync();  // the exchange's reads come before the area's next writes
}

// The inverse (unnormalised) of c3_sub_fwd: D3 in, D1 out.
template <int SL, int NA, typename R, typename TW>
__device__ __forceinline__ void c3_sub_inv(cx<R> (&v)[NA][8], cx<R>* area, const TW& tw, int lane) {
  constexpr int E = 8;
#pragma unroll
  for (int i = 0; i < NA; ++i) dft<E, true>(v[i]);  // element e: n1 = e of k2 = lane
  // n1-major: (n1, k2) at index n1 * 64 + k2
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int e = 0; e < E; ++e) area[i * SL + fspad(lane) + fspad(64 * e)] = v[i][e];
  wave_sync();
  const int s = lane % 8, l = lane / 8;
  const auto to = tw.outer();
  const cx<R>* rd = area + fspad(64 * s) + l;  // + i SL + fspad(8 b)
#pragma unroll
  for (int b = 0; b < E; ++b) {
    const cx<R> w = to[b];
#pragma unroll
    for (int i = 0; i < NA; ++i) v[i][b] = cmulc(rd[i * SL + fspad(8 * b)], w);
  }
  fs_sub_bwd<true, E, 8, SL, NA>(v, area, s * 64, tw.set1(), l);
}

// 256-point transform of NA arrays on one wave (columns of 768): four radix-4
// Stockham stages, 4 elements per lane, element e at index lane + 64 e in and
// out (so the output order is that of c3_sub_fwd: register r at k = lane +
// 64 r), exchanged through this wave's area (array i at area + i * SL) with
// wave barriers only.  Stage twiddles w_(4 Ns)^(k r) = w_2N^((384 / Ns) k r)
// from the 2N-roots table of N = 768; INV: conjugate twiddles and inverse
// DFTs (unnormalised).
template <bool INV, int SL, int NA, typename R>
__device__ __forceinline__ void c3_stockham256(cx<R> (&v)[NA][4], cx<R>* area, const cx<R>* __restrict__ r2n,
                                               int lane) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int Ns = 1 << (2 * st);  // 1, 4, 16, 64
    const int k = lane & (Ns - 1);
    cx<R> w[4];
    if (st > 0) {
#pragma unroll
      for (int r = 1; r < 4; ++r) w[r] = r2n[(unsigned)((384 / Ns) * k * r)];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      cx<R> a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = v[i][r];
      if (st > 0) {
#pragma unroll
        for (int r = 1; r < 4; ++r) a[r] = INV ? cmulc(a[r], w[r]) : cmul(a[r], w[r]);
      }
      dft<4, INV>(a);
      if (st < 3) {
        const int base = (lane / Ns) * Ns * 4 + k;
#pragma unroll
        for (int r = 0; r < 4; ++r) area[i * SL + fspad(base + Ns * r)] = a[r];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[i][r] = a[r];
      }
    }
    if (st < 3) {
      wave_sync();
#pragma unroll
      for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[i][e] = area[i * SL + fspad(lane + 64 * e)];
      wave_sync();  // the reads come before the area's next writes
    }
  }
}

// The sub-transforms by length: the four-step one of 512, the Stockham one
// of 256
template <int L, int SL, int NA, typename R, typename TW>
__device__ __forceinline__ void c3_fwd(cx<R> (&v)[NA][L / 64], cx<R>* area, const TW& tw, const cx<R>* r2n, int lane) {
  if constexpr (L == 512) c3_sub_fwd<SL, NA>(v, area, tw, lane);
  else c3_stockham256<false, SL, NA>(v, area, r2n, lane);
}
template <int L, int SL, int NA, typename R, typename TW>
__device__ __forceinline__ void c3_inv(cx<R> (&v)[NA][L / 64], cx<R>* area, const TW& tw, const cx<R>* r2n, int lane) {
  if constexpr (L == 512) c3_sub_inv<SL, NA>(v, area, tw, lane);
  else c3_stockham256<true, SL, NA>(v, area, r2n, lane);
}

template <typename R, typename TO, int MODE, int L = 512>
__global__ void __launch_bounds__(kC3T) SG_WAVES_PER_EU(SG_COLFS3_WPE)
    k_colfs3(const cx<R>* __restrict__ X, cx<R>* __restrict__ V, int M, int tj, const TO* __restrict__ tox,
             const TO* __restrict__ toy, const cx<R>* __restrict__ r2n, const cx<R>* __restrict__ twfs,
             const sg_bgrid* __restrict__ bg) {
  using S3 = c3_shape<L>;
  constexpr int N = S3::N, E = S3::E, T = S3::T, SL = S3::SL;
  constexpr int kind = (MODE == 1 || MODE == 3) ? 1 : 0;
  constexpr bool solve = MODE >= 2;
  constexpr int SYS = MODE == 2 ? 3 : (MODE == 3 ? 4 : 5);
  constexpr bool pre = SG_COLFS3_PRE;
  static_assert(band_smem<double2, T>::BYTES <= 2 * SL * (int)sizeof(cx<R>), "the solve's LDS fits slots 2, 3");
  __shared__ cx<R> smem[4 * SL];
  if (bg) {
    const sg_bgrid d = grid_desc(bg);
    X = reinterpret_cast<const cx<R>*>(d.X);
    V = reinterpret_cast<cx<R>*>(d.V);
    tox = reinterpret_cast<const TO*>(d.tabx);
    toy = reinterpret_cast<const TO*>(d.taby);
  }
  const int t = threadIdx.x;
  const int q = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  const int c = xcd_tile(blockIdx.x, M);
  const bool packed = (c == 0);
  const TO* rowx = tox + (int64_t)c * (N + 1);
  const TO* rowy = toy + (int64_t)c * (N + 1);
  // bin of register r within each half: 3 (lane + 64 r) + q
  auto bin = [&](int r) { return 3 * (lane + 64 * r) + q; };

  // ---- the column (chunk of E per thread) and this thread's table entries
  cx<R> a[E];
  {
    const cx<R>* col = X + (int64_t)c * N;
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = col[(unsigned)(t * E + e)];
  }
  TO tv[pre ? 4 : 1][pre ? E : 1];
  if constexpr (pre) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < E; ++r) tv[i][r] = ((i & 1) ? rowy : rowx)[(unsigned)fs_tab_index<TO, N>(bin(r), i >> 1)];
  }
  // the four-step twiddles of the 512-point sub-transforms (unused for 256)
  fs_tw<512, 8, R, true> tw;
  if constexpr (L == 512) tw.init(twfs, lane);

  // ---- y-solve (FP64, chunks; its LDS in slots 2, 3), then x to slot 0
  if constexpr (solve) {
    double2 d[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
      d[e] = make_double2(band_scale(SYS) * (double)a[e].x, band_scale(SYS) * (double)a[e].y);
    band_solve<SYS, E, T, double2, false>(d, t, smem + 2 * SL);
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = cx<R>{(R)d[e].x, (R)d[e].y};
  }
#pragma unroll
  for (int e = 0; e < E; ++e) smem[fspad(t * E + e)] = a[e];
  __syncthreads();

  // ---- forward radix-3 step: f[0] for x, f[1] for x_j w_2N^j
  cx<R> f[2][E];
  c3_wave(q, [&](auto Q) {
    constexpr int qc = decltype(Q)::value;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = lane + 64 * e;
      const cx<R> x0 = smem[fspad(n)], x1 = smem[fspad(n + L)], x2 = smem[fspad(n + 2 * L)];
      f[0][e] = c3_sum<2 * qc>(x0, x1, x2);
      f[1][e] = c3_sum<2 * qc + 1>(x0, x1, x2);
      if constexpr (qc != 0) f[0][e] = cmul(f[0][e], r2n[(unsigned)(2 * qc * n)]);  // w_N^(n q) = w_2N^(2 n q)
      f[1][e] = cmul(f[1][e], r2n[(unsigned)((2 * qc + 1) * n)]);
    }
  });
  cx<R>* sub = smem + 2 * SL + fspad(q * L);  // wave q's area in slot 2 (array 1: slot 3)
  c3_fwd<L, SL, 2>(f, sub, tw, r2n, lane);

  // ---- products: g = (x even, y even, x odd, y odd)
  cx<R> g[4][E];
  constexpr R ex = kind == 1 ? (R)-1 : (R)1;  // reflection sign of the x table (y: -ex)
  cx<R> php{(R)1, (R)0}, rho{(R)1, (R)0};
  if constexpr (kind == 1) {
    php = fs_half_phase<R>((double)c / (2.0 * M));
    rho = fs_half_phase<R>(1.0 / (2.0 * N));
  }
  if (!packed) {
    if constexpr (kind == 1) {
      const cx<R> pho = cmul(php, rho);
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const cx<R> wq = r2n[(unsigned)bin(r)];
        f[0][r] = cmul(f[0][r], cmul(wq, php));
        f[1][r] = cmul(f[1][r], cmul(wq, pho));
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int h = i >> 1, cy = i & 1, qq = bin(r);
        const R sgn = fs_tab_direct<N>(qq, h) ? (R)1 : (cy ? -ex : ex);
        TO ent;
        if constexpr (pre) ent = tv[i][r];
        else ent = (cy ? rowy : rowx)[(unsigned)fs_tab_index<TO, N>(qq, h)];
        g[i][r] = fs_iA(f[h][r], ent, sgn);
      }
  } else {
    // packed column: as in colfs.hpp, the partner bins through slots 0, 1
    const TO* row0x = tox;
    const TO* row0y = toy;
    const TO* rowMx = tox + (int64_t)M * (N + 1);
    const TO* rowMy = toy + (int64_t)M * (N + 1);
    __syncthreads();  // every wave's radix-3 reads of slot 0 come first
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < E; ++r) smem[h * SL + fspad(bin(r))] = f[h][r];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int qq = bin(r);
        const int qm = h == 0 ? (qq == 0 ? 0 : N - qq) : N - 1 - qq;
        const cx<R> u = f[h][r], um = conj(smem[h * SL + fspad(qm)]);
        cx<R> c0v{(R)0.5 * (u.x + um.x), (R)0.5 * (u.y + um.y)};
        cx<R> cmv{(R)0.5 * (u.y - um.y), (R)-0.5 * (u.x - um.x)};
        if constexpr (kind == 1) {
          const cx<R> wq = r2n[(unsigned)qq];
          const cx<R> ph0 = h ? cmul(wq, rho) : wq;
          c0v = cmul(c0v, ph0);
          cmv = cmul(cmv, cx<R>{ph0.y, -ph0.x});
        }
        const bool dir = fs_tab_direct<N>(qq, h);
        const int ti = fs_tab_index<TO, N>(qq, h);
        const R sx = dir ? (R)1 : ex, sy = dir ? (R)1 : -ex;
        const cx<R> x0 = fs_iA(c0v, row0x[ti], sx), xm = fs_iA(cmv, rowMx[ti], sx);
        const cx<R> y0 = fs_iA(c0v, row0y[ti], sy), ym = fs_iA(cmv, rowMy[ti], sy);
        g[2 * h][r] = cx<R>{x0.x - xm.y, x0.y + xm.x};
        g[2 * h + 1][r] = cx<R>{y0.x - ym.y, y0.y + ym.x};
      }
  }

  // ---- inverse sub-transforms (each wave in its areas of slots 2, 3), then
  // u_q = w_N^(-n q) (even halves) and w_2N^(-n (2q + 1)) (odd halves)
  {
    cx<R> g01[2][E], g23[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      g01[0][e] = g[0][e];
      g01[1][e] = g[1][e];
      g23[0][e] = g[2][e];
      g23[1][e] = g[3][e];
    }
    c3_inv<L, SL, 2>(g01, sub, tw, r2n, lane);
    c3_inv<L, SL, 2>(g23, sub, tw, r2n, lane);
    // (for q = 0 the even twiddle is the root 1, an exact product)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = lane + 64 * e;
      const cx<R> we = r2n[(unsigned)(2 * n * q)], wo = r2n[(unsigned)(n * (2 * q + 1))];
      g[0][e] = cmulc(g01[0][e], we);
      g[1][e] = cmulc(g01[1][e], we);
      g[2][e] = cmulc(g23[0][e], wo);
      g[3][e] = cmulc(g23[1][e], wo);
    }
  }
  // ---- inverse radix-3 exchange: array i at slot i, u_q[n] at index L q + n
  __syncthreads();  // every wave is done with its areas and with slot 0
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < E; ++e) smem[i * SL + fspad(q * L + lane + 64 * e)] = g[i][e];
  __syncthreads();
  // V(p, j) at ((j/tj*2 + p%2)*M + p/2)*tj + j%tj
  const int pa = c, pb = packed ? M : 2 * M - c;
  cx<R>* va = V + (int64_t)(pa & 1) * M * tj + (int64_t)(pa >> 1) * tj;
  cx<R>* vb = V + (int64_t)(pb & 1) * M * tj + (int64_t)(pb >> 1) * tj;
  const int64_t jstride = (int64_t)2 * M * tj;
  // thread (wave r = q, lane): outputs j = n + L r, n = lane + 64 e
  c3_wave(q, [&](auto Q) {
    constexpr int r3 = decltype(Q)::value;
    // w_3^(-q r) = exp(+2 pi i q r / 3): radix-3 weight c = exp(-2 pi i m / 6),
    // m = (6 - 2 r) mod 6; the odd halves also take w_2N^(-L r) = w_6^(-r)
    constexpr int m3 = (6 - 2 * r3) % 6;
    constexpr R s3 = (R)0.86602540378443864676;
    const cx<R> w6 = r3 == 0 ? cx<R>{(R)1, (R)0} : (r3 == 1 ? cx<R>{(R)0.5, s3} : cx<R>{(R)-0.5, s3});
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = lane + 64 * e, j = n + L * r3;
      cx<R> y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        y[i] = c3_sum<m3>(smem[i * SL + fspad(n)], smem[i * SL + fspad(n + L)], smem[i * SL + fspad(n + 2 * L)]);
      const cx<R> yx = r3 == 0 ? y[0] + y[2] : y[0] + cmul(y[2], w6);
      const cx<R> yy = r3 == 0 ? y[1] + y[3] : y[1] + cmul(y[3], w6);
      cx<R> v1, v2;
      if (packed) {
        v1 = cx<R>{yx.x, yy.x};
        v2 = cx<R>{yx.y, yy.y};
      } else {
        v1 = cx<R>{yx.x - yy.y, yx.y + yy.x};
        v2 = cx<R>{yx.x + yy.y, yy.x - yx.y};
      }
      const int64_t o = (int64_t)(j / tj) * jstride + (j % tj);
      va[o] = v1;
      vb[o] = v2;
    }
  });
}

}  // namespace sg
