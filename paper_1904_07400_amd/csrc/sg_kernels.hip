// Device kernels of the thin-disk self-gravity library (gfx950).
//
// Per-step path for one M x N grid (sigma row-major [N][M], x fastest):
//   pass A (rows):    [k >= 3: x-solve, Eq. (C_system)] + real FFT of the row
//                     zero-padded to 2M, written as M packed complex bins
//                     (bin 0 carries the real bins 0 and M);
//   pass B (columns): [k >= 3: y-solve, Eq. (z_system), on the row spectra] +
//                     FFT of the column zero-padded to 2N, products with the
//                     spectra of w^x and w^y (convolution theorem), two
//                     inverse FFTs cropped to N outputs, written as the
//                     combined spectrum V = Yx + i Yy of length 2M per row;
//   pass C (rows):    inverse FFT of V, cropped to M outputs:
//                     Fx = Re, Fy = Im.
// The y-solve commutes with the x-transform (tensor-product operators), so
// it runs inside pass B at no extra HBM traffic.
//
// Plan time: weights of Eq. (eqnwB) on the padded 2M x 2N lattice (FP64),
// then the same row/column transforms in FP64 to get their spectra.
#include <type_traits>

#include "fft.hpp"
#include "kcommon.hpp"
#include "sg_internal.h"
#include "tridiag.hpp"

// Launch-shape knobs (compile-time; elements per thread E and threads per
// workgroup of each pass).  Defaults are the measured best on MI355X.
#ifndef SG_RF_THREADS32
#define SG_RF_THREADS32 1024
#endif
#ifndef SG_RF_THREADS64
#define SG_RF_THREADS64 512
#endif
#ifndef SG_RI_THREADS32
#define SG_RI_THREADS32 256
#endif
#ifndef SG_RI_THREADS64
#define SG_RI_THREADS64 1024
#endif
#ifndef SG_RI_E32
#define SG_RI_E32 8
#endif
// FP32 inverse rows from this length on: SG_RI_BIG_E elements per thread,
// SG_RI_BIG_NB exchange buffers per row, SG_RI_BIG_WG threads per workgroup
#ifndef SG_RI_BIG32
#define SG_RI_BIG32 2048
#endif
#ifndef SG_RI_BIG_E
#define SG_RI_BIG_E 16
#endif
#ifndef SG_RI_BIG_NB
#define SG_RI_BIG_NB 1
#endif
#ifndef SG_RI_BIG_WG
#define SG_RI_BIG_WG 512
#endif
// 1: those rows load both halves before the transforms
#ifndef SG_RI_PRE
#define SG_RI_PRE 1
#endif
// the inverse row pass takes its thread index through an opaque move for
// its loads and its stores, so that their indices are not held across the
// transforms
#ifndef SG_RI_OPQ
#define SG_RI_OPQ 1
#endif
#ifndef SG_RI_E64
#define SG_RI_E64 16
#endif
#ifndef SG_COL_E32
#define SG_COL_E32 8
#endif
// rows per tile of the column pass's output (its store segments hold
// SG_TJ consecutive rows of one column)
#ifndef SG_TJ32
#define SG_TJ32 8
#endif
#ifndef SG_TJ64
#define SG_TJ64 2
#endif
#ifndef SG_COL_E64
#define SG_COL_E64 8
#endif
#ifndef SG_RF_E32
#define SG_RF_E32 8
#endif
#ifndef SG_COL_PP
#define SG_COL_PP 1
#endif
#ifndef SG_COL_WG32
#define SG_COL_WG32 256
#endif
#ifndef SG_COL_NBUF32
#define SG_COL_NBUF32 4
#endif
// skewed LDS layout of the forward row pass's transposed store (1: one slot
// every 32 elements, 0: plain)
#ifndef SG_RF_SKEW
#define SG_RF_SKEW 1
#endif
// the row passes read entry s + j of their table of roots of unity as
// entry s times entry j, j the same for the whole workgroup (a scalar load),
// so that each thread reads one entry of its own per set (1) or every entry
// (0)
#ifndef SG_ROOT_SPLIT
#define SG_ROOT_SPLIT 1
#endif
// exchange buffers per row of the FP32 row passes (2: both half-length
// transforms share their barriers)
#ifndef SG_RF_NBUF32
#define SG_RF_NBUF32 2
#endif
#ifndef SG_RI_NBUF32
#define SG_RI_NBUF32 2
#endif
#ifndef SG_RF_E64
#define SG_RF_E64 8
#endif
// elements per thread for transform lengths 3 * 2^a (a multiple of 3)
#ifndef SG_E3
#define SG_E3 12
#endif
// minimum waves per SIMD the register allocation must allow (1 = no cap),
// per pass and precision
#ifndef SG_RF_WPE32
#define SG_RF_WPE32 1
#endif
#ifndef SG_RF_WPE64
#define SG_RF_WPE64 1
#endif
#ifndef SG_COL_WPE32
#define SG_COL_WPE32 1
#endif
#ifndef SG_COL_WPE64
#define SG_COL_WPE64 1
#endif
#ifndef SG_RI_WPE32
#define SG_RI_WPE32 1
#endif
#ifndef SG_RI_WPE64
#define SG_RI_WPE64 1
#endif
#define SG_WPE(R, P) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? SG_##P##_WPE32 : SG_##P##_WPE64)))

// The host dispatch is split into parts that can be compiled as separate
// objects in parallel (bit 0: plan-time and helper kernels, 1: row passes,
// 2: column pass, 3: adjoint column and row passes; SG_PART is a mask of
// them); without SG_PART everything is compiled.
#ifndef SG_PART
#define SG_PART 15
#endif
#define SG_IN_PART(n) ((SG_PART >> (n)) & 1)

namespace sg {

// ------------------------------------------------------------- weights --
#if SG_IN_PART(0)
__constant__ double c_glx[4][16];
__constant__ double c_glw[4][16];
__constant__ int c_glq[4] = {4, 6, 10, 16};
// Spline pieces as polynomials c0 + c1 xi + ... + c_{k-1} xi^{k-1} in the
// piece-centred variable xi in [-1/2, 1/2] (Eqs. (Bspline1)-(Bspline3) on
// uniform knots, and the recursion of Eq. (eqnBk) carried to the cubic and
// quartic): order k, piece r (piece r spans [t_r, t_{r+1}]).
__constant__ double c_piece[5][5][5] = {
    {{1.0}},
    {{0.5, 1.0}, {0.5, -1.0}},
    {{0.125, 0.5, 0.5}, {0.75, 0.0, -1.0}, {0.125, -0.5, 0.5}},
    {{1.0 / 48, 1.0 / 8, 1.0 / 4, 1.0 / 6},
     {23.0 / 48, 5.0 / 8, -1.0 / 4, -1.0 / 2},
     {23.0 / 48, -5.0 / 8, -1.0 / 4, 1.0 / 2},
     {1.0 / 48, -1.0 / 8, 1.0 / 4, -1.0 / 6}},
    {{1.0 / 384, 1.0 / 48, 1.0 / 16, 1.0 / 12, 1.0 / 24},
     {19.0 / 96, 11.0 / 24, 1.0 / 4, -1.0 / 6, -1.0 / 6},
     {115.0 / 192, 0.0, -5.0 / 8, 0.0, 1.0 / 4},
     {19.0 / 96, -11.0 / 24, 1.0 / 4, 1.0 / 6, -1.0 / 6},
     {1.0 / 384, -1.0 / 48, 1.0 / 16, -1.0 / 12, 1.0 / 24}}};

// a piece's polynomial at xi (Horner, degree k - 1)
__device__ __forceinline__ double piece_at(const double* p, int k, double xi) {
  double v = p[k - 1];
  for (int d = k - 2; d >= 0; --d) v = p[d] + xi * v;
  return v;
}

// int_0^T t^n (1 + t^2)^(-3/2) dt for even n: the moments of Eq. (intMoment)
// with a = 1, by their recursion from n = 0, 2; below T = 1/2 by the power
// series of (1 + t^2)^(-3/2) instead, where the closed forms cancel.
__device__ double gmoment(int n, double T) {
  if (T < 0.5) {
    const double T2 = T * T;
    double tp = T, c = 1.0, acc = 0.0;
    for (int j = 0; j < n; ++j) tp *= T;
    for (int m = 0; m < 40; ++m) {
      acc += c * tp / (double)(n + 2 * m + 1);
      tp *= T2;
      c *= (-1.5 - m) / (double)(m + 1);
    }
    return acc;
  }
  const double rho = sqrt(1.0 + T * T);
  if (n == 0) return T / rho;
  double g = asinh(T) - T / rho, tp = T;
  for (int j = 4; j <= n; j += 2) {
    tp *= T * T;
    g = tp / ((double)(j - 2) * rho) - (double)(j - 1) / (double)(j - 2) * g;
  }
  return g;
}

// Principal value of x^al y^be / r^3 over [-X, X] x [-Y, Y] (al, be even,
// al + be >= 2): four times the quarter [0, X] x [0, Y], which polar
// coordinates split at the diagonal into two one-dimensional moments (the
// form of Eq. (intF)).
__device__ double pv_moment(int al, int be, double X, double Y) {
  const int s = al + be - 1;
  double xs = 1.0, ys = 1.0;
  for (int j = 0; j < s; ++j) {
    xs *= X;
    ys *= Y;
  }
  return 4.0 * (xs * gmoment(be, Y / X) + ys * gmoment(al, X / Y)) / (double)s;
}

// Both weight components at offset (m, n): the integrals of x~/r^3 and
// y~/r^3 against the tensor spline attached to C_{i-m, j-n} (Eq. (eqnwB)).
// The spline's piece that holds the singular point is integrated in closed
// form (principal value over the centred square [-dx/2,dx/2]x[-dy/2,dy/2]:
// only monomials even in both variables survive, each is 4x its integral
// over [0,dx/2]x[0,dy/2], taken from the antiderivatives of Appendix A for
// (alpha, beta) = (2,0), (0,2), (2,2)); every other piece by tensor
// Gauss-Legendre, whose node count grows as the piece nears the singularity.
__device__ void weight_pair(int k, double hx, double hy, int m, int n, double& wx, double& wy) {
  const int shift = (k - 1) / 2;
  double sx = 0.0, sy = 0.0;
  for (int r = 0; r < k; ++r) {
    const int ox = r - m - shift;  // piece centre in cells
    const double cxp = (double)ox * hx;
    const double* px = c_piece[k - 1][r];
    for (int s = 0; s < k; ++s) {
      const int oy = s - n - shift;
      const double cyp = (double)oy * hy;
      const double* py = c_piece[k - 1][s];
      if (ox == 0 && oy == 0 && k > 3) {
        // cubic and quartic pieces: every monomial pair odd in the force
        // direction and even across it
        const double X = 0.5 * hx, Y = 0.5 * hy;
        double sa = 1.0;
        for (int a = 0; a < k; ++a) {
          double sb = 1.0;
          for (int b = 0; b < k; ++b) {
            const double c = px[a] * py[b] / (sa * sb);
            if ((a & 1) && !(b & 1)) sx += c * pv_moment(a + 1, b, X, Y);
            if (!(a & 1) && (b & 1)) sy += c * pv_moment(a, b + 1, X, Y);
            sb *= hy;
          }
          sa *= hx;
        }
        continue;
      }
      if (ox == 0 && oy == 0) {
        const double X = 0.5 * hx, Y = 0.5 * hy, Rr = sqrt(X * X + Y * Y);
        const double LX = log((X + Rr) / Y), LY = log((Y + Rr) / X);
        const double I20 = 4.0 * Y * LX, I02 = 4.0 * X * LY;
        const double I22 = 4.0 * (-X * Y * Rr + Y * Y * Y * LX + X * X * X * LY) / 3.0;
        const double p0 = px[0], p1 = px[1] / hx, p2 = px[2] / (hx * hx);
        const double q0 = py[0], q1 = py[1] / hy, q2 = py[2] / (hy * hy);
        sx += p1 * (q0 * I20 + q2 * I22);
        sy += q1 * (p0 * I02 + p2 * I22);
        continue;
      }
      // Gauss-Legendre on nsx x nsy equal sub-rectangles of the piece, each no
      // larger than the piece's distance to the singular point, so that the
      // kernel's complex singularities stay >= 2 half-widths from every
      // quadrature interval (pieces next to the singular one, dx != dy)
      const double dxm = fmax(fabs(cxp) - 0.5 * hx, 0.0), dym = fmax(fabs(cyp) - 0.5 * hy, 0.0);
      const double dist = sqrt(dxm * dxm + dym * dym);
      const int nsx = dist >= hx ? 1 : (int)ceil(hx / dist);
      const int nsy = dist >= hy ? 1 : (int)ceil(hy / dist);
      const double sw = hx / nsx, sh = hy / nsy;
      const double ratio = dist / fmax(sw, sh);
      const int qi = ratio < 2.0 ? 3 : ratio < 8.0 ? 2 : ratio < 64.0 ? 1 : 0;
      const int q = c_glq[qi];
      double ax = 0.0, ay = 0.0;
      for (int sa = 0; sa < nsx; ++sa) {
        const double xic = -0.5 + (sa + 0.5) / nsx;  // sub-rectangle centre in xi
        for (int a = 0; a < q; ++a) {
          const double xi = xic + (0.5 / nsx) * c_glx[qi][a];
          const double x = cxp + xi * hx;
          const double bx = piece_at(px, k, xi) * c_glw[qi][a];
          double ix = 0.0, iy = 0.0;
          for (int sb = 0; sb < nsy; ++sb) {
            const double etc = -0.5 + (sb + 0.5) / nsy;
            for (int b = 0; b < q; ++b) {
              const double eta = etc + (0.5 / nsy) * c_glx[qi][b];
              const double y = cyp + eta * hy;
              const double by = piece_at(py, k, eta) * c_glw[qi][b];
              const double r2 = x * x + y * y;
              const double inv = by / (r2 * sqrt(r2));
              ix += x * inv;
              iy += y * inv;
            }
          }
          ax += bx * ix;
          ay += bx * iy;
        }
      }
      sx += ax * (0.25 * sw * sh);
      sy += ay * (0.25 * sw * sh);
    }
  }
  wx = sx;
  wy = sy;
}

// Padded lattice (layout 0): entry (p, q), p in [0,2M), q in [0,2N), row
// q; offset m = p (p < M) or p - 2M (p > M), likewise n.  The slots p = M
// and q = N are never read by cropped outputs; they are filled so that the
// padded table keeps the symmetry of the weights over the whole period
// (odd about the spline centre in the force direction, even across it),
// which makes the spectra purely imaginary for odd k.  Export layout
// (layout 1): (2N-1) x (2M-1), offsets m in [-(M-1), M-1].
__global__ void k_weights(int k, double hx, double hy, int M, int N, double* __restrict__ wx,
                          double* __restrict__ wy, int layout) {
  const int W = layout == 0 ? 2 * M : 2 * M - 1;
  const int H = layout == 0 ? 2 * N : 2 * N - 1;
  const int64_t total = (int64_t)W * H;
  const int s2 = (k % 2 == 0) ? 1 : 0;  // twice the spline-centre offset, in cells
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(idx % W), q = (int)(idx / W);
    double vx, vy;
    if (layout == 1) {
      weight_pair(k, hx, hy, p - (M - 1), q - (N - 1), vx, vy);
    } else {
      const bool sp = (p == M), sq = (q == N);
      const int m = sp ? s2 - M : (p < M ? p : p - 2 * M);
      const int n = sq ? s2 - N : (q < N ? q : q - 2 * N);
      if ((sp || sq) && s2 == 0) {
        vx = 0.0;
        vy = 0.0;
      } else {
        weight_pair(k, hx, hy, m, n, vx, vy);
        if (sp) { vx = -vx; }
        if (sq) { vy = -vy; }
      }
    }
    if (wx) wx[idx] = vx;
    if (wy) wy[idx] = vy;
  }
}

#endif

// entry s + j of a table of roots of unity (entry n = exp(+-2 pi i n / L)),
// given ws = entry s
template <typename R>
__device__ __forceinline__ cx<R> root_at(const cx<R>* __restrict__ tab, cx<R> ws, int s, int j) {
  if constexpr (SG_ROOT_SPLIT) return j == 0 ? ws : cmul(ws, tab[j]);
  else return tab[s + j];
}

// ---------------------------------------------------------------- pass A --
// Real FFT of length 2M of a row whose upper half is zero (or, with full,
// of a row of 2M values), via the complex FFT of length M of
// z[n] = x[2n] + i x[2n+1], itself split into its even and odd output bins
// (two FFTs of length M/2).  Output: M packed bins, bin 0 = (X_0, X_M),
// stored column-major (bin p of row r at X[p*ldx + r]) so that the column
// pass reads whole columns.  G rows per workgroup; the transposed store
// goes through LDS so that each bin's G consecutive rows leave as one
// contiguous segment.
constexpr int kLdsBudget = 144 * 1024;

template <typename R, typename In, int M>
struct rowfwd_cfg {
  static constexpr int L = M / 2;
  static constexpr int E0 = sizeof(R) == 4 ? SG_RF_E32 : SG_RF_E64;
  static constexpr int E = elems_for(L, E0, SG_E3);
  static constexpr int T = L / E;
  static constexpr int LL = lds_len<L>::value;
  // per-row LDS slot (complex elements): FFT exchange buffer, also used
  // for the reduced system of the x-solve
  static constexpr int TRI = band_smem<double, T>::BYTES / (int)sizeof(cx<R>) + 1;
  static constexpr int SLOT = LL > TRI ? LL : TRI;
  static constexpr int NB = (sizeof(R) == 4 && sizeof(In) == 4) ? SG_RF_NBUF32 : 1;  // exchange buffers per row
  // rows per workgroup: more rows make longer segments of the transposed store
  static constexpr int WG = sizeof(R) == 4 ? SG_RF_THREADS32 : SG_RF_THREADS64;
  static constexpr int G0 = WG / T < 1 ? 1 : (WG / T < 16 ? WG / T : 16);
  static constexpr int GL = kLdsBudget / (NB * SLOT * (int)sizeof(cx<R>));
  static constexpr int G = (G0 < GL ? G0 : GL) < 1 ? 1 : (G0 < GL ? G0 : GL);
  // e-values per transposed-store chunk (2T bins per e, G rows)
  static constexpr int EC = (SLOT / (2 * T)) < 1 ? 1 : ((SLOT / (2 * T)) > E ? E : SLOT / (2 * T));
};

// HI: the x-solve of k = 4, 5 (solve = 4, 5); otherwise that of k = 3 (solve
// = 3) or none (solve = 0).  Separate instantiations keep the registers of
// the k <= 3 kernels those of their own solve.
template <typename R, typename In, int M, bool HI = false>
__global__ void __launch_bounds__((rowfwd_cfg<R, In, M>::G * rowfwd_cfg<R, In, M>::T))
    SG_WPE(R, RF)
    k_row_fwd(const In* __restrict__ src, int64_t src_ld, cx<R>* __restrict__ X, int ldx, int nrows,
              const cx<R>* __restrict__ r2m, int solve, int full, const cx<R>* __restrict__ tw,
              const sg_bgrid* __restrict__ bg) {
  if (bg) {  // batched: grid blockIdx.y of the class
    const sg_bgrid d = grid_desc(bg);
    src += d.off;
    X = reinterpret_cast<cx<R>*>(d.X);
  }
  using C = rowfwd_cfg<R, In, M>;
  constexpr int L = C::L, E = C::E, T = C::T, SLOT = C::SLOT, EC = C::EC, NB = C::NB;
  // G * SLOT * NB elements, sized at launch (dyn_lds)
  extern __shared__ __align__(16) unsigned char sg_dyn_lds[];
  cx<R>* const smem = reinterpret_cast<cx<R>*>(sg_dyn_lds);
  const int G = blockDim.x / T;  // rows per workgroup (<= C::G)
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int row0 = xcd_tile(blockIdx.x, gridDim.x) * G, row = row0 + g;
  const bool active = row < nrows;
  cx<R>* lds = smem + g * SLOT * NB;
  cx<R>* lds2 = lds + (NB - 1) * SLOT;
  // loads are unconditional (a row past nrows reads row 0 and is masked
  // afterwards), so that they issue together rather than one at a time
  // behind a branch each
  const In* s = src + (int64_t)(active ? row : 0) * src_ld;
  const double msk = active ? (HI ? band_scale(solve) : band_scale(3)) : 0.0;
  cx<R> ze[E], zo[E];
  if (solve) {
    // chunk of 2E reals per thread: x-solve of Eq. (C_system) (order
    // solve = 3, 4 or 5), FP64
    constexpr int CH = 2 * E;
    double d[CH];
#pragma unroll
    for (int e = 0; e < CH; ++e) d[e] = msk * (double)s[t * CH + e];
    if constexpr (!HI)
      band_solve<3, CH, T>(d, t, lds);
    else if (solve == 4)
      band_solve<4, CH, T>(d, t, lds);
    else
      band_solve<5, CH, T>(d, t, lds);
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t * E + e)] = cx<R>{(R)d[2 * e], (R)d[2 * e + 1]};
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) ze[e] = lds[pad(t + e * T)];
    __syncthreads();
  } else {
    const R m1 = active ? (R)1 : (R)0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = t + e * T;
      ze[e] = cx<R>{m1 * (R)s[2 * n], m1 * (R)s[2 * n + 1]};
    }
  }
  if (full) {  // rows of 2M values (plan time): fold the upper half in
    const R m1 = active ? (R)1 : (R)0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = t + e * T;
      const cx<R> lo = ze[e], hi{m1 * (R)s[2 * (n + L)], m1 * (R)s[2 * (n + L) + 1]};
      ze[e] = lo + hi;
      zo[e] = cmul(lo - hi, r2m[2 * n]);  // w_M^n
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) zo[e] = cmul(ze[e], root_at(r2m, r2m[2 * t], 2 * t, 2 * e * T));  // w_M^n
  }
  cx<R> xe[E];
  if constexpr (NB == 2) {
    // even and odd bins of Z through the same stages
    cx<R> z2[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      z2[0][e] = ze[e];
      z2[1][e] = zo[e];
    }
    fftn<false, L, T, 2>(z2, lds, SLOT, tw, t);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ze[e] = z2[0][e];
      zo[e] = z2[1][e];
      lds[pad(t + e * T)] = ze[e];
      lds2[pad(t + e * T)] = zo[e];
    }
    __syncthreads();
  } else {
    fft<false, L, T>(ze, lds, tw, t);  // even bins of Z
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t + e * T)] = ze[e];
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pp = t + e * T;                         // X bin p = 2 pp
    const cx<R> zp = ze[e], zm = conj(lds[pad(pp == 0 ? 0 : L - pp)]);
    const cx<R> sum = zp + zm, dif = cmul(root_at(r2m, r2m[2 * t], 2 * t, 2 * e * T), zp - zm);
    xe[e] = cx<R>{(R)0.5 * (sum.x + dif.y), (R)0.5 * (sum.y - dif.x)};
    if (pp == 0) xe[e] = cx<R>{zp.x + zp.y, zp.x - zp.y};
  }
  if constexpr (NB != 2) {
    __syncthreads();
    fft<false, L, T>(zo, lds, tw, t);  // odd bins of Z
#pragma unroll
    for (int e = 0; e < E; ++e) lds2[pad(t + e * T)] = zo[e];
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pp = t + e * T;                         // X bin p = 2 pp + 1
    const cx<R> zp = zo[e], zm = conj(lds2[pad(L - 1 - pp)]);
    const cx<R> sum = zp + zm, dif = cmul(root_at(r2m, r2m[2 * t + 1], 2 * t + 1, 2 * e * T), zp - zm);
    zo[e] = cx<R>{(R)0.5 * (sum.x + dif.y), (R)0.5 * (sum.y - dif.x)};
  }
  __syncthreads();
  // transposed store: chunk of EC e-values = bins [2 e0 T, 2 (e0+EC) T) of all G rows.
  // The writes of one wave are 2G elements apart; with the one-per-32 skew
  // (where the LDS holds it) they fall in distinct banks.
  constexpr bool SKW = SG_RF_SKEW && (2 * T * EC + (2 * T * EC + 31) / 32 <= SLOT * NB);
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += EC) {
#pragma unroll
    for (int e = e0; e < e0 + EC && e < E; ++e) {
      const int pl = 2 * (t + (e - e0) * T);
      const int i0 = pl * G + g, i1 = (pl + 1) * G + g;
      smem[SKW ? pad(i0) : i0] = xe[e];
      smem[SKW ? pad(i1) : i1] = zo[e];
    }
    __syncthreads();
    const int nchunk = 2 * T * (E - e0 < EC ? E - e0 : EC) * G;
    for (int idx = threadIdx.x; idx < nchunk; idx += blockDim.x) {
      const int pl = idx / G, gg = idx % G;
      if (row0 + gg < nrows) X[(int64_t)(2 * e0 * T + pl) * ldx + row0 + gg] = smem[SKW ? pad(idx) : idx];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- pass B --
// Lengths with a second launch variant (FP32): the Stockham column pass
// from 64 to 1536 (2048 and up take the four-step pass), the inverse row
// pass from 512 on.
template <int N>
constexpr bool col_variants() {
  return N >= 64 && N <= 1536;
}
template <int M>
constexpr bool rowinv_variants() {
  return M >= 512;
}

// V: launch variant (FP32 only): 0 = SG_COL_NBUF32 exchange buffers per
// column, 1 = two (more columns per workgroup; the same arithmetic)
template <typename R, int N, int V = 0>
struct col_cfg {
  static constexpr int E0 = sizeof(R) == 4 ? SG_COL_E32 : SG_COL_E64;
  static constexpr int E = elems_for(N, E0, SG_E3);
  static constexpr int T = N / E;
  static constexpr int LL = lds_len<N>::value;
  static constexpr int TRI = band_smem<double2, T>::BYTES / (int)sizeof(cx<R>) + 1;
  static constexpr int SLOT = LL > TRI ? LL : TRI;  // per-column LDS slot (complex elements)
  // exchange buffers per column: 2 or 4 let as many transforms share their
  // barriers
  static constexpr int NBUF = sizeof(R) == 4 ? (V == 1 ? 2 : SG_COL_NBUF32) : 1;
  static constexpr int BYTES = NBUF * SLOT * (int)sizeof(cx<R>);
  // columns per workgroup: up to SG_COL_WG threads, within the LDS budget
  static constexpr int WG = sizeof(R) == 4 ? SG_COL_WG32 : 256;
  static constexpr int LB = WG > 256 ? kLdsBudget : 65536;
  static constexpr int P0 = T >= WG ? 1 : WG / T;
  static constexpr int PL = (LB / BYTES) < 1 ? 1 : (LB / BYTES);
  static constexpr int P = P0 < PL ? P0 : PL;
};

// spectrum lookup helpers: real tables A with W = i A (odd k) or W = ph i A
// (even k, ph the bin's half-cell phase)
// z * (i A sgn) with a table entry A (double, or a float hi+lo pair)
__device__ __forceinline__ cx<double> apply_iA(cx<double> z, double a, double sgn) {
  a *= sgn;
  return {-z.y * a, z.x * a};
}
__device__ __forceinline__ cx<float> apply_iA(cx<float> z, float2 a, float sgn) {
  // the sign is applied last (exact either way), so that a prefetched entry
  // is not needed before the product itself
  return {-(z.y * a.x + z.y * a.y) * sgn, (z.x * a.x + z.x * a.y) * sgn};
}
template <typename R, typename TO>
__device__ __forceinline__ cx<R> mul_iA(cx<R> z, const TO* tab, int idx, R sgn) {
  return apply_iA(z, tab[(unsigned)idx], sgn);
}
// Even k: the spline centres sit half a cell off the cell centres in both
// directions.  The padded weight table is then odd (force direction) and
// even (across) about that centre, over the whole period once its slots
// m = M, n = N hold the mirrored values, so W^d = ph(p, q) i A^d with
// ph = exp(-i pi (p / 2M + q / 2N)) and A^d real; the tables store A^d like
// the odd-k tables.
// exp(-i pi frac), from FP64:
template <typename R>
__device__ __forceinline__ cx<R> half_cell_phase(double frac) {
  double sn, cs;
  sincospi(-frac, &sn, &cs);
  return cx<R>{(R)cs, (R)sn};
}

// Product of the column spectrum with W^d (or conj W^d, CJ) at column bin p.
// half 0: bins q = 2q', half 1: q = 2q'+1.  eps: symmetry of the stored
// table across q -> 2N - q for odd k (+1 for x, -1 for y); even k has the
// opposite one.  kind 1 (even k): ph is the phase of the bin.
// Odd k: the stored entry of the real table for column bin p, row bin qq of
// half `half` (row: the table row of bin p), and its sign (+1, or eps past
// the reflection q -> 2N - q).
template <typename TO, int N>
__device__ __forceinline__ TO odd_entry(const TO* row, int qq, int half) {
  if (half == 0) return row[(unsigned)(qq <= N / 2 ? qq : N - qq)];
  return row[(unsigned)(N / 2 + 1 + (qq < N / 2 ? qq : N - 1 - qq))];
}
template <typename R, int N>
__device__ __forceinline__ R odd_sign(int qq, int half, R eps) {
  return (half == 0 ? qq <= N / 2 : qq < N / 2) ? (R)1 : eps;
}

template <typename R, typename TO, int N, bool CJ = false>
__device__ __forceinline__ cx<R> spec_mul(cx<R> z, int kind, const TO* to, int p, int qq, int half, R eps,
                                          cx<R> ph) {
  if (kind == 1) {
    z = CJ ? cmulc(z, ph) : cmul(z, ph);
    eps = -eps;
  }
  const TO* row = to + (int64_t)p * (N + 1);
  const R c = CJ ? (R)-1 : (R)1;  // conj(i A) = -i A
  if (half == 0) {
    const bool lo = qq <= N / 2;
    return mul_iA(z, row, lo ? qq : N - qq, lo ? c : c * eps);
  }
  const bool lo = qq < N / 2;
  return mul_iA(z, row + N / 2 + 1, lo ? qq : N - 1 - qq, lo ? c : c * eps);
}

// Product of one half of the column spectrum with W^d of one component
// (to/tc: that component's table, eps: its reflection sign).  exch: the
// workgroup holds the packed column 0 (uniform over the workgroup); packed:
// this slice is column 0, whose spectrum U carries bins p = 0 and p = M:
// C_0 = (U(q) + conj U(-q))/2, C_M = (U(q) - conj U(-q))/(2i), and the
// products are re-packed as G_0 + i G_M.  Even k: w2n = exp(-i pi q'/N),
// php = exp(-i pi c / 2M), rho = exp(-i pi / 2N) make the bin phases.
template <typename R, typename TO, int N, int E, int T>
__device__ __forceinline__ void col_product(const cx<R>* f, cx<R>* g, int half, bool exch, bool packed, cx<R>* lds,
                                            int kind, const TO* to, R eps, int c, int M, int t, const cx<R>* w2n,
                                            cx<R> php, cx<R> rho) {
  const cx<R> phh = half ? cmul(php, rho) : php;  // column and half part of the phase
  if (!exch) {
    // no packed column in this workgroup: independent loads, no branches
#pragma unroll
    for (int e = 0; e < E; ++e)
      g[e] = spec_mul<R, TO, N>(f[e], kind, to, c, t + e * T, half, eps, cmul(w2n[e], phh));
    return;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) lds[pad(t + e * T)] = f[e];
  __syncthreads();
  // one branch around each loop (uniform per column group), so that the
  // loads of a loop issue together
  if (packed) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int qq = t + e * T;
      const int qm = half == 0 ? (qq == 0 ? 0 : N - qq) : (N - 1 - qq);
      const cx<R> u = f[e], um = conj(lds[pad(qm)]);
      const cx<R> c0v{(R)0.5 * (u.x + um.x), (R)0.5 * (u.y + um.y)};
      const cx<R> cmv{(R)0.5 * (u.y - um.y), (R)-0.5 * (u.x - um.x)};
      // phases of bins p = 0 (1) and p = M (-i) times that of row bin q
      const cx<R> ph0 = half ? cmul(w2n[e], rho) : w2n[e];
      const cx<R> w0 = spec_mul<R, TO, N>(c0v, kind, to, 0, qq, half, eps, ph0);
      const cx<R> wm = spec_mul<R, TO, N>(cmv, kind, to, M, qq, half, eps, cx<R>{ph0.y, -ph0.x});
      g[e] = cx<R>{w0.x - wm.y, w0.y + wm.x};
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e)
      g[e] = spec_mul<R, TO, N>(f[e], kind, to, c, t + e * T, half, eps, cmul(w2n[e], phh));
  }
  __syncthreads();
}

// MODE: 0 = k 1 (no solve), 1 = k 2 (phased tables), 2 = k 3 (y-solve), 3 =
// k 4 (phased tables, y-solve), 4 = k 5 (pentadiagonal y-solve)
template <typename R, typename TO, int N, int MODE, int VA = 0>
__global__ void __launch_bounds__((col_cfg<R, N, VA>::P * col_cfg<R, N, VA>::T))
    SG_WPE(R, COL) k_col(const cx<R>* __restrict__ X, cx<R>* __restrict__ V, int M, int tj, const TO* __restrict__ tox,
          const TO* __restrict__ toy, const cx<R>* __restrict__ r2n, const cx<R>* __restrict__ tw,
          const sg_bgrid* __restrict__ bg) {
  constexpr int kind = (MODE == 1 || MODE == 3) ? 1 : 0;
  constexpr bool solve = MODE >= 2;
  constexpr int SYS = MODE == 2 ? 3 : (MODE == 3 ? 4 : 5);  // order of the y-solve
  if (bg) {  // batched: grid blockIdx.y of the class
    const sg_bgrid d = grid_desc(bg);
    X = reinterpret_cast<const cx<R>*>(d.X);
    V = reinterpret_cast<cx<R>*>(d.V);
    tox = reinterpret_cast<const TO*>(d.tabx);
    toy = reinterpret_cast<const TO*>(d.taby);
  }
  using C = col_cfg<R, N, VA>;
  constexpr int E = C::E, T = C::T, LL = C::SLOT, NBUF = C::NBUF;
  // P * LL * NBUF elements, sized at launch (dyn_lds)
  extern __shared__ __align__(16) unsigned char sg_dyn_lds[];
  cx<R>* const smem = reinterpret_cast<cx<R>*>(sg_dyn_lds);
  const int P = blockDim.x / T;  // columns per workgroup (<= C::P, divides M)
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c0 = tile * P, c = c0 + g;
  cx<R>* lds = smem + g * LL * NBUF;
  cx<R>* lds2 = lds + (NBUF - 1) * LL;
  const cx<R>* col = X + (int64_t)c * N;  // column c, contiguous (column-major X)
  const bool exch = (c0 == 0);            // this workgroup holds the packed column 0
  // the column: chunk of E per thread for the solve, else strided
  cx<R> a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) a[e] = col[(unsigned)(solve ? t * E + e : t + e * T)];
  // With four exchange buffers: every table entry of the four products is
  // loaded here, after the column (loads complete in order), so that their
  // latency overlaps the solve and the forward transforms (in order x even,
  // y even, x odd, y odd).
  constexpr bool pre = NBUF == 4;
  TO tv[pre ? 4 : 1][pre ? E : 1];
  if constexpr (pre) {
    // unconditional (unused by the packed workgroup), so that the waits
    // for the column above can count them
    const TO* rx = tox + (int64_t)c * (N + 1);
    const TO* ry = toy + (int64_t)c * (N + 1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < E; ++e) tv[i][e] = odd_entry<TO, N>((i & 1) ? ry : rx, t + e * T, i >> 1);
  }
  // phases exp(-i pi j / N) of the odd-bin transforms (used twice), loaded
  // now so that their latency hides behind the solve
  cx<R> w2n[E];
#pragma unroll
  for (int e = 0; e < E; ++e) w2n[e] = r2n[(unsigned)(t + e * T)];
  // even k: phase of column bin c and the extra phase of the odd row bins
  cx<R> php{(R)1, (R)0}, rho{(R)1, (R)0};
  if constexpr (kind == 1) {
    php = half_cell_phase<R>((double)c / (2.0 * M));
    rho = half_cell_phase<R>(1.0 / (2.0 * N));
  }
  // with four buffers the forward transforms alternate between buffers
  // {0, 1} and {2, 3} (one barrier per exchange)
  constexpr bool pp = (NBUF == 4) && SG_COL_PP;
  if (solve) {
    // y-solve of Eq. (z_system) on the complex row spectra, FP64, chunk of E per thread
    double2 d[E];
#pragma unroll
    for (int e = 0; e < E; ++e) d[e] = make_double2(band_scale(SYS) * (double)a[e].x, band_scale(SYS) * (double)a[e].y);
    if constexpr (pp) {
      // the solve's LDS lies in buffer 0; the transpose goes through buffer
      // 2, and the forward transform's first exchange (buffers 0 and 1)
      // follows the transpose's barrier, so neither needs a barrier after it
      band_solve<SYS, E, T, double2, false>(d, t, lds);
      cx<R>* tb = lds + 2 * LL;
#pragma unroll
      for (int e = 0; e < E; ++e) tb[pad(t * E + e)] = cx<R>{(R)d[e].x, (R)d[e].y};
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) a[e] = tb[pad(t + e * T)];
    } else {
      band_solve<SYS, E, T, double2>(d, t, lds);
#pragma unroll
      for (int e = 0; e < E; ++e) lds[pad(t * E + e)] = cx<R>{(R)d[e].x, (R)d[e].y};
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) a[e] = lds[pad(t + e * T)];
      __syncthreads();
    }
  }

  const bool packed = (c == 0);
  // forward transform of the column zero-padded to 2N: even bins
  // fe = FFT_N(a), odd bins fo = FFT_N(a_j w_2N^j)
  cx<R> fe[E], fo[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    fo[e] = cmul(a[e], w2n[e]);
    fe[e] = a[e];
  }
  cx<R> accx[E], accy[E];
  if constexpr (NBUF == 4) {
    // both forward transforms together, then all four products (x and y of
    // each half) and their inverses together
    {
      cx<R> f2[2][E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        f2[0][e] = fe[e];
        f2[1][e] = fo[e];
      }
      if constexpr (pp)
        fftn_pp<false, N, T, 2>(f2, lds, LL, tw, t);
      else
        fftn<false, N, T, 2>(f2, lds, LL, tw, t);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        fe[e] = f2[0][e];
        fo[e] = f2[1][e];
      }
    }
    cx<R> g4[4][E];
    bool done = false;
    if constexpr (pre) {
      if (!exch) {
        if constexpr (kind == 1) {
          // even k: the bin phases, shared by both components
          const cx<R> pho = cmul(php, rho);
#pragma unroll
          for (int e = 0; e < E; ++e) {
            fe[e] = cmul(fe[e], cmul(w2n[e], php));
            fo[e] = cmul(fo[e], cmul(w2n[e], pho));
          }
        }
        constexpr R ex = kind == 1 ? (R)-1 : (R)1;  // reflection sign of the x table
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int e = 0; e < E; ++e)
            g4[i][e] = apply_iA((i >> 1) ? fo[e] : fe[e], tv[i][e],
                                odd_sign<R, N>(t + e * T, i >> 1, (i & 1) ? -ex : ex));
        done = true;
      }
    }
    if (!done) {
      col_product<R, TO, N, E, T>(fe, g4[0], 0, exch, packed, lds, kind, tox, (R)1, c, M, t, w2n, php, rho);
      col_product<R, TO, N, E, T>(fe, g4[1], 0, exch, packed, lds, kind, toy, (R)-1, c, M, t, w2n, php, rho);
      col_product<R, TO, N, E, T>(fo, g4[2], 1, exch, packed, lds, kind, tox, (R)1, c, M, t, w2n, php, rho);
      col_product<R, TO, N, E, T>(fo, g4[3], 1, exch, packed, lds, kind, toy, (R)-1, c, M, t, w2n, php, rho);
    }
    fftn<true, N, T, 4>(g4, lds, LL, tw, t);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<R> w = w2n[e];  // conj -> exp(+i pi j / N)
      accx[e] = g4[0][e] + cmulc(g4[2][e], w);
      accy[e] = g4[1][e] + cmulc(g4[3][e], w);
    }
  } else if constexpr (NBUF == 2) {
    // both forward transforms, then per half both components' inverses,
    // two at a time through the two exchange buffers
    fft2<false, N, T>(fe, fo, lds, lds2, tw, t);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const cx<R>* f = half ? fo : fe;
      cx<R> gx[E], gy[E];
      col_product<R, TO, N, E, T>(f, gx, half, exch, packed, lds, kind, tox, (R)1, c, M, t, w2n, php, rho);
      col_product<R, TO, N, E, T>(f, gy, half, exch, packed, lds, kind, toy, (R)-1, c, M, t, w2n, php, rho);
      fft2<true, N, T>(gx, gy, lds, lds2, tw, t);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (half == 0) {
          accx[e] = gx[e];
          accy[e] = gy[e];
        } else {
          const cx<R> w = w2n[e];  // conj -> exp(+i pi j / N)
          accx[e] = accx[e] + cmulc(gx[e], w);
          accy[e] = accy[e] + cmulc(gy[e], w);
        }
      }
    }
  } else {
    fft<false, N, T>(fe, lds, tw, t);
    fft<false, N, T>(fo, lds, tw, t);
    // one half and one component at a time: g = f W^d, inverse, accumulate
    // (the odd half with the phase exp(+i pi j / N))
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const cx<R>* f = half ? fo : fe;
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        cx<R> g[E];
        col_product<R, TO, N, E, T>(f, g, half, exch, packed, lds, kind, comp ? toy : tox, comp ? (R)-1 : (R)1, c,
                                    M, t, w2n, php, rho);
        fft<true, N, T>(g, lds, tw, t);
        cx<R>* acc = comp ? accy : accx;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (half == 0) {
            acc[e] = g[e];
          } else {
            const cx<R> w = w2n[e];  // conj -> exp(+i pi j / N)
            acc[e] = acc[e] + cmulc(g[e], w);
          }
        }
      }
    }
  }
  // V(c) = Yx + i Yy and V(2M - c) = conj(Yx) + i conj(Yy); the packed
  // column gives V(0) = Re Yx + i Re Yy and V(M) = Im Yx + i Im Yy.
  // V is stored in tiles of tj rows: V(p, j) at ((jb*2 + (p&1))*M + p/2)*tj + jj,
  // jb = j / tj, jj = j % tj, which the row pass reads contiguously.
  const int pa = c, pb = packed ? M : 2 * M - c;
  cx<R>* va = V + (int64_t)(pa & 1) * M * tj + (int64_t)(pa >> 1) * tj;
  cx<R>* vb = V + (int64_t)(pb & 1) * M * tj + (int64_t)(pb >> 1) * tj;
  const int64_t jstride = (int64_t)2 * M * tj;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = t + e * T;
    const cx<R> yx = accx[e], yy = accy[e];
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
}

// ---------------------------------------------------------------- pass C --
// Rows j of the combined spectrum V: v = IFFT_2M(V) cropped to n < M via its
// even and odd input bins (two inverse FFTs of length M); Fx = Re, Fy = Im.
// V is stored in tiles of tj rows (element (p, j) at ((j/tj*2 + p%2)*M +
// p/2)*tj + j%tj); each row loads its elements straight from the tile, and
// the rows of one tile go to workgroups on the same XCD so that the tile's
// cache lines are shared in its L2.
// V: launch variant (FP32 only): 0 = SG_RI_E32 elements per thread, both
// half-length inverses through the same stages (SG_RI_NBUF32 buffers); 1 =
// SG_RI_BIG_E elements per thread, the halves one after the other (one
// exchange buffer per row), so that more rows share a workgroup and the
// loads of adjacent tile rows leave together (the default from SG_RI_BIG32
// bins on)
template <typename R, int M, int V = 0>
struct rowinv_cfg {
  static constexpr int L = M;
  static constexpr bool BIG = sizeof(R) == 4 && V == 1;
  static constexpr int E = elems_for(L, sizeof(R) == 4 ? (BIG ? SG_RI_BIG_E : SG_RI_E32) : SG_RI_E64, SG_E3);
  static constexpr int T = L / E;
  static constexpr int LL = lds_len<L>::value;
  static constexpr int NB = sizeof(R) == 4 ? (BIG ? SG_RI_BIG_NB : SG_RI_NBUF32) : 1;  // exchange buffers per row
  // LDS of one row: its buffers plus a shift of 8 elements, so that the
  // rows' buffers start in different banks
  static constexpr int RS = NB * LL + 8;
  static constexpr int WG = sizeof(R) == 4 ? (BIG ? SG_RI_BIG_WG : SG_RI_THREADS32) : SG_RI_THREADS64;
  static constexpr int G0 = WG / T < 1 ? 1 : (WG / T < 16 ? WG / T : 16);
  static constexpr int GL = kLdsBudget / (RS * (int)sizeof(cx<R>));
  static constexpr int G = (G0 < GL ? G0 : GL) < 1 ? 1 : (G0 < GL ? G0 : GL);
};

// Minimum waves per SIMD of the inverse row pass: SG_RI_WPE_BIG for the FP32
// rows of 2048 and 4096 in launch variant 1 (two workgroups of 512 threads
// per compute unit at 128 registers), else SG_RI_WPE32 / SG_RI_WPE64
#ifndef SG_RI_WPE_BIG
#define SG_RI_WPE_BIG 4
#endif
template <typename R, int M, int VA>
struct rowinv_wpe {
  static constexpr int value = (rowinv_cfg<R, M, VA>::BIG && (M == 2048 || M == 4096))
                                   ? SG_RI_WPE_BIG
                                   : (sizeof(R) == 4 ? SG_RI_WPE32 : SG_RI_WPE64);
};

template <typename R, typename Out, int M, int VA = 0>
__global__ void __launch_bounds__((rowinv_cfg<R, M, VA>::G * rowinv_cfg<R, M, VA>::T))
    __attribute__((amdgpu_waves_per_eu(rowinv_wpe<R, M, VA>::value)))
    k_row_inv(const cx<R>* __restrict__ V, Out* __restrict__ fx, Out* __restrict__ fy, int nrows, int tj,
              const cx<R>* __restrict__ r2m, const cx<R>* __restrict__ tw, const sg_bgrid* __restrict__ bg) {
  if (bg) {  // batched: grid blockIdx.y of the class
    const sg_bgrid d = grid_desc(bg);
    V = reinterpret_cast<const cx<R>*>(d.V);
    fx += d.off;
    fy += d.off;
  }
  using C = rowinv_cfg<R, M, VA>;
  constexpr int E = C::E, T = C::T, LL = C::LL, NB = C::NB;
  // static, for the compiled maximum of rows (LDS sized at launch measured
  // slower here: its 128 registers then spill)
  __shared__ cx<R> smem[C::G * C::RS];
  // G rows per workgroup, interleaved lane by lane (thread t of row g is
  // thread t G + g), so that the G rows' elements of one bin, adjacent in a
  // tile, are read by adjacent lanes
  const int G = blockDim.x / T;
  const int g = threadIdx.x % G, t = threadIdx.x / G;
  const int row = xcd_tile(blockIdx.x, gridDim.x) * G + g;
  const bool active = row < nrows;
  cx<R>* lds = smem + g * C::RS;
  const int jb = (active ? row : 0) / tj, jj = (active ? row : 0) % tj;
  // NB == 2 and the FP32 rows of four per workgroup: both halves loaded
  // before any transform, so that all loads are in flight together; other
  // FP64 rows load the odd half after the even half's transform (registers)
  constexpr bool PRE = NB == 2 || (C::BIG && SG_RI_PRE);
  cx<R> v2[2][E], wr[NB == 2 ? E : 1];
  auto load_half = [&](int half) {
    const cx<R>* base = V + ((int64_t)jb * 2 + half) * M * tj + jj;
    const int tl = SG_RI_OPQ ? opaque(t) : t;
#pragma unroll
    for (int e = 0; e < E; ++e) v2[half][e] = base[(int64_t)(tl + e * T) * tj];
  };
  load_half(0);
  if constexpr (PRE) load_half(1);
  if constexpr (NB == 2) {
    // phases of the odd half, loaded now so that their latency hides
    // behind the transforms
#pragma unroll
    for (int e = 0; e < E; ++e) wr[e] = root_at(r2m, r2m[t], t, e * T);
    // both half-length inverses through the same stages
    fftn<true, M, T, 2>(v2, lds, LL, tw, t);
  } else {
    fft<true, M, T>(v2[0], lds, tw, t);
    if constexpr (!PRE) load_half(1);
    fft<true, M, T>(v2[1], lds, tw, t);
  }
  if (active) {
    const int ts = SG_RI_OPQ ? opaque(t) : t;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = ts + e * T;
      const cx<R> r = v2[0][e] + cmulc(v2[1][e], NB == 2 ? wr[e] : root_at(r2m, r2m[ts], ts, e * T));
      fx[(int64_t)row * M + n] = (Out)r.x;
      fy[(int64_t)row * M + n] = (Out)r.y;
    }
  }
}

// -------------------------------------------------------------- adjoint --
// Transposed convolution: gC = crop(IFFT(FFT(pad gx) conj Wx + FFT(pad gy)
// conj Wy)) with the forward pass's spectra and scaling, then the
// transposed coefficient solve (the same symmetric systems).  Row
// transforms of gx, gy reuse k_row_fwd; the column pass below multiplies by
// the conjugate spectra, sums the two components, inverts cropped to N rows,
// applies the y-solve and writes the packed row spectra of gC in tiles of
// tj rows: bin p of row j at ((j/tj*2 + p%2)*(M/2) + p/2)*tj + j%tj.
// Even k: r2n = exp(-i pi q'/N), php and rho as in col_product.
template <typename R, typename TO, int N, int E, int T>
__device__ __forceinline__ void col_products_adj(const cx<R>* fx, const cx<R>* fy, cx<R>* h, int half, bool exch,
                                                 bool packed, cx<R>* lds, int kind, const TO* tox, const TO* toy,
                                                 int c, int M, int t, const cx<R>* r2n, cx<R> php, cx<R> rho) {
  const cx<R> phh = half ? cmul(php, rho) : php;
  if (!exch) {
    // no packed column in this workgroup: independent loads, no branches
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int qq = t + e * T;
      const cx<R> ph = kind == 1 ? cmul(r2n[(unsigned)qq], phh) : cx<R>{(R)1, (R)0};
      h[e] = spec_mul<R, TO, N, true>(fx[e], kind, tox, c, qq, half, (R)1, ph) +
             spec_mul<R, TO, N, true>(fy[e], kind, toy, c, qq, half, (R)-1, ph);
    }
    return;
  }
  // packed column: each spectrum U carries bins p = 0 and p = M; split both
  cx<R> umx[E], umy[E];
  {
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t + e * T)] = fx[e];
    __syncthreads();
    if (packed) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int qq = t + e * T;
        umx[e] = conj(lds[pad(half == 0 ? (qq == 0 ? 0 : N - qq) : (N - 1 - qq))]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t + e * T)] = fy[e];
    __syncthreads();
    if (packed) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int qq = t + e * T;
        umy[e] = conj(lds[pad(half == 0 ? (qq == 0 ? 0 : N - qq) : (N - 1 - qq))]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int qq = t + e * T;
    const cx<R> w = kind == 1 ? r2n[(unsigned)qq] : cx<R>{(R)1, (R)0};
    if (packed) {
      const cx<R> ux = fx[e], uy = fy[e];
      const cx<R> x0v{(R)0.5 * (ux.x + umx[e].x), (R)0.5 * (ux.y + umx[e].y)};
      const cx<R> xmv{(R)0.5 * (ux.y - umx[e].y), (R)-0.5 * (ux.x - umx[e].x)};
      const cx<R> y0v{(R)0.5 * (uy.x + umy[e].x), (R)0.5 * (uy.y + umy[e].y)};
      const cx<R> ymv{(R)0.5 * (uy.y - umy[e].y), (R)-0.5 * (uy.x - umy[e].x)};
      const cx<R> ph0 = half ? cmul(w, rho) : w;  // bins p = 0 and p = M (-i ph0)
      const cx<R> phm{ph0.y, -ph0.x};
      const cx<R> h0 = spec_mul<R, TO, N, true>(x0v, kind, tox, 0, qq, half, (R)1, ph0) +
                       spec_mul<R, TO, N, true>(y0v, kind, toy, 0, qq, half, (R)-1, ph0);
      const cx<R> hm = spec_mul<R, TO, N, true>(xmv, kind, tox, M, qq, half, (R)1, phm) +
                       spec_mul<R, TO, N, true>(ymv, kind, toy, M, qq, half, (R)-1, phm);
      h[e] = cx<R>{h0.x - hm.y, h0.y + hm.x};
    } else {
      const cx<R> ph = cmul(w, phh);
      h[e] = spec_mul<R, TO, N, true>(fx[e], kind, tox, c, qq, half, (R)1, ph) +
             spec_mul<R, TO, N, true>(fy[e], kind, toy, c, qq, half, (R)-1, ph);
    }
  }
}

template <typename R, typename TO, int N, int MODE>
__global__ void __launch_bounds__((col_cfg<R, N>::P * col_cfg<R, N>::T))
    k_col_adj(const cx<R>* __restrict__ Xx, const cx<R>* __restrict__ Xy, cx<R>* __restrict__ Y, int M, int tj,
              const TO* __restrict__ tox, const TO* __restrict__ toy, const cx<R>* __restrict__ r2n,
              const cx<R>* __restrict__ tw, const sg_bgrid* __restrict__ bg) {
  constexpr int kind = (MODE == 1 || MODE == 3) ? 1 : 0;
  constexpr bool solve = MODE >= 2;
  constexpr int SYS = MODE == 2 ? 3 : (MODE == 3 ? 4 : 5);  // order of the y-solve
  if (bg) {  // batched: gx spectra in X, gy spectra in the first half of V, output in its second half
    const sg_bgrid d = grid_desc(bg);
    Xx = reinterpret_cast<const cx<R>*>(d.X);
    Xy = reinterpret_cast<const cx<R>*>(d.V);
    Y = reinterpret_cast<cx<R>*>(d.V) + (int64_t)M * N;
    tox = reinterpret_cast<const TO*>(d.tabx);
    toy = reinterpret_cast<const TO*>(d.taby);
  }
  using C = col_cfg<R, N>;
  constexpr int E = C::E, T = C::T, LL = C::SLOT;
  __shared__ cx<R> smem[C::P * LL];
  const int P = blockDim.x / T;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int c0 = xcd_tile(blockIdx.x, gridDim.x) * P, c = c0 + g;
  cx<R>* lds = smem + g * LL;
  const bool packed = (c == 0);
  cx<R> php{(R)1, (R)0}, rho{(R)1, (R)0};  // even k: as in k_col
  if constexpr (kind == 1) {
    php = half_cell_phase<R>((double)c / (2.0 * M));
    rho = half_cell_phase<R>(1.0 / (2.0 * N));
  }
  cx<R> ax[E], ay[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    ax[e] = Xx[(int64_t)c * N + t + e * T];
    ay[e] = Xy[(int64_t)c * N + t + e * T];
  }
  cx<R> acc[E];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    cx<R> fx[E], fy[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<R> w = r2n[(unsigned)(t + e * T)];
      fx[e] = half ? cmul(ax[e], w) : ax[e];
      fy[e] = half ? cmul(ay[e], w) : ay[e];
    }
    fft<false, N, T>(fx, lds, tw, t);
    fft<false, N, T>(fy, lds, tw, t);
    cx<R> h[E];
    col_products_adj<R, TO, N, E, T>(fx, fy, h, half, c0 == 0, packed, lds, kind, tox, toy, c, M, t, r2n, php, rho);
    fft<true, N, T>(h, lds, tw, t);
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = half ? acc[e] + cmulc(h[e], r2n[(unsigned)(t + e * T)]) : h[e];
  }
  if (solve) {
    // transposed y-solve (Eq. (z_system) is symmetric): chunk of E per thread
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t + e * T)] = acc[e];
    __syncthreads();
    double2 d[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<R> v = lds[pad(t * E + e)];
      d[e] = make_double2(band_scale(SYS) * (double)v.x, band_scale(SYS) * (double)v.y);
    }
    __syncthreads();
    band_solve<SYS, E, T, double2>(d, t, lds);
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t * E + e)] = cx<R>{(R)d[e].x, (R)d[e].y};
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = lds[pad(t + e * T)];
  }
  cx<R>* out = Y + (int64_t)(c & 1) * (M / 2) * tj + (int64_t)(c >> 1) * tj;
  const int64_t jstride = (int64_t)M * tj;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = t + e * T;
    out[(int64_t)(j / tj) * jstride + (j % tj)] = acc[e];
  }
}

// Rows of the packed gC spectra -> real row of length 2M cropped to M via
// the half-length complex inverse FFT (z = x_even + i x_odd, its first M/2
// outputs from the even and odd input bins: two inverse FFTs of length M/2),
// then the transposed x-solve (Eq. (C_system) is symmetric).
// Rows per workgroup: those of the forward row pass, but at most 512
// threads for the banded x-solve of k = 4, 5 (HI), whose registers would
// not fit 1024 threads without spilling.
template <typename R, int M, bool HI>
struct rowc2r_cfg {
  using F = rowfwd_cfg<R, R, M>;
  static constexpr int G = (HI && F::G * F::T > 512) ? (512 / F::T > 0 ? 512 / F::T : 1) : F::G;
};

template <typename R, typename Out, int M, bool HI = false>  // HI: as in k_row_fwd
__global__ void __launch_bounds__((rowc2r_cfg<R, M, HI>::G * rowfwd_cfg<R, R, M>::T))
    k_row_c2r(const cx<R>* __restrict__ Y, Out* __restrict__ out, int nrows, int tj, const cx<R>* __restrict__ r2m,
              int solve, const cx<R>* __restrict__ tw, const sg_bgrid* __restrict__ bg) {
  if (bg) {  // batched: packed spectra in the second half of V
    const sg_bgrid d = grid_desc(bg);
    Y = reinterpret_cast<const cx<R>*>(d.V) + (int64_t)M * nrows;
    out += d.off;
  }
  using C = rowfwd_cfg<R, R, M>;
  constexpr int L = C::L, E = C::E, T = C::T, SLOT = C::SLOT;
  __shared__ cx<R> smem[rowc2r_cfg<R, M, HI>::G * SLOT];
  const int G = blockDim.x / T;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int row = xcd_tile(blockIdx.x, gridDim.x) * G + g;
  const bool active = row < nrows;
  cx<R>* lds = smem + g * SLOT;
  const int jb = (active ? row : 0) / tj, jj = (active ? row : 0) % tj;
  // bin p of this row: tile half p&1, index p>>1
  const cx<R>* b0 = Y + ((int64_t)jb * 2) * L * tj + jj;
  const cx<R>* b1 = Y + ((int64_t)jb * 2 + 1) * L * tj + jj;
  cx<R> ze[E], zo[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pp = t + e * T;
    // Z'[p] = (X[p] + conj X[M-p]) + i conj(w_2M^p) (X[p] - conj X[M-p]), X[M] packed in slot 0
    const cx<R> xe = b0[(int64_t)pp * tj];                       // X[2pp]
    const cx<R> xo = b1[(int64_t)pp * tj];                       // X[2pp+1]
    cx<R> me = conj(b0[(int64_t)(pp == 0 ? 0 : L - pp) * tj]);   // conj X[M - 2pp]
    const cx<R> mo = conj(b1[(int64_t)(L - 1 - pp) * tj]);       // conj X[M - 2pp - 1]
    if (pp == 0) {
      const cx<R> x0 = xe;  // (X_0, X_M)
      ze[e] = cx<R>{x0.x + x0.y, x0.x - x0.y};
    } else {
      const cx<R> sum = xe + me, dif = cmulc(xe - me, root_at(r2m, r2m[2 * t], 2 * t, 2 * e * T));
      ze[e] = cx<R>{sum.x - dif.y, sum.y + dif.x};
    }
    const cx<R> sum = xo + mo, dif = cmulc(xo - mo, root_at(r2m, r2m[2 * t + 1], 2 * t + 1, 2 * e * T));
    zo[e] = cx<R>{sum.x - dif.y, sum.y + dif.x};
  }
  fft<true, L, T>(ze, lds, tw, t);
  fft<true, L, T>(zo, lds, tw, t);
  // z[n'] = ze + exp(2 pi i n'/M) zo, n' < M/2: x[2n'] = Re z, x[2n'+1] = Im z
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = t + e * T;
    ze[e] = ze[e] + cmulc(zo[e], root_at(r2m, r2m[2 * t], 2 * t, 2 * e * T));
  }
  if (solve) {
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t + e * T)] = ze[e];
    __syncthreads();
    constexpr int CH = 2 * E;
    double d[CH];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<R> v = lds[pad(t * E + e)];
      d[2 * e] = (HI ? band_scale(solve) : band_scale(3)) * (double)v.x;
      d[2 * e + 1] = (HI ? band_scale(solve) : band_scale(3)) * (double)v.y;
    }
    __syncthreads();
    if constexpr (!HI)
      band_solve<3, CH, T>(d, t, lds);
    else if (solve == 4)
      band_solve<4, CH, T>(d, t, lds);
    else
      band_solve<5, CH, T>(d, t, lds);
    if (active) {
#pragma unroll
      for (int e = 0; e < CH; ++e) out[(int64_t)row * M + t * CH + e] = (Out)d[e];
    }
  } else if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = t + e * T;
      out[(int64_t)row * M + 2 * n] = (Out)ze[e].x;
      out[(int64_t)row * M + 2 * n + 1] = (Out)ze[e].y;
    }
  }
}

// ------------------------------------------------------ spectrum (plan) --
// Column FFT (FP64, full length 2N: the even/odd output split preceded by
// the first radix-2 butterfly) of the row spectra of the padded weight
// table, then the stored form of W^d(p, q) / (4MN):
//   odd k : A = Im W (W is purely imaginary), q in [0, N], split by parity;
//   even k: A = Im(W conj(ph)), ph = exp(-i pi (p / 2M + q / 2N)) the
//           half-cell phase, on the same quarter.
// Output element type: double (FP64 plans) or a hi+lo float pair.
template <int N>
struct spec_cfg {
  static constexpr int E = elems_for(N, 8, SG_E3);
  static constexpr int T = N / E;
  static constexpr int LL = lds_len<N>::value;
};

// fp32: 0 double, 1 float hi + lo pair, 2 float
__device__ __forceinline__ void put_odd(void* tab, int fp32, int64_t idx, double v) {
  if (fp32 == 1) {
    const float h = (float)v;
    reinterpret_cast<float2*>(tab)[idx] = make_float2(h, (float)(v - (double)h));
  } else if (fp32 == 2) {
    reinterpret_cast<float*>(tab)[idx] = (float)v;
  } else {
    reinterpret_cast<double*>(tab)[idx] = v;
  }
}

template <int N>
__global__ void __launch_bounds__((spec_cfg<N>::T))
    k_spec_col(const cx<double>* __restrict__ S, int M, void* __restrict__ tab, int kind, int fp32,
               double scale, const cx<double>* __restrict__ r2n, const cx<double>* __restrict__ tw) {
  using C = spec_cfg<N>;
  constexpr int E = C::E, T = C::T, LL = C::LL;
  __shared__ cx<double> lds[LL];
  const int t = threadIdx.x;
  const int c = blockIdx.x;
  cx<double> lo[E], hi[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = t + e * T;
    lo[e] = S[(int64_t)c * (2 * N) + j];
    hi[e] = S[(int64_t)c * (2 * N) + j + N];
  }
  for (int half = 0; half < 2; ++half) {
    cx<double> f[E];
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] = half ? cmul(lo[e] - hi[e], r2n[(unsigned)(t + e * T)]) : lo[e] + hi[e];
    fft<false, N, T>(f, lds, tw, t);
#pragma unroll
    for (int e = 0; e < E; ++e) lds[pad(t + e * T)] = f[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int qq = t + e * T;
      cx<double> vals[2];
      int rows[2];
      int nv = 1;
      if (c == 0) {
        const int qm = half == 0 ? (qq == 0 ? 0 : N - qq) : (N - 1 - qq);
        const cx<double> u = f[e], um = conj(lds[pad(qm)]);
        vals[0] = cx<double>{0.5 * (u.x + um.x), 0.5 * (u.y + um.y)};
        vals[1] = cx<double>{0.5 * (u.y - um.y), -0.5 * (u.x - um.x)};
        rows[0] = 0;
        rows[1] = M;
        nv = 2;
      } else {
        vals[0] = f[e];
        rows[0] = c;
      }
      for (int h = 0; h < nv; ++h) {
        const cx<double> w = vals[h] * scale;
        // odd k: W = i A; even k: W = ph i A with the phase of bin (p, q),
        // ph = exp(-i pi (p / 2M + q / 2N)), so A = Im(W conj(ph))
        double a = w.y;
        if (kind == 1) {
          double sn, cs;
          sincospi((double)rows[h] / (2.0 * M) + (double)(2 * qq + half) / (2.0 * N), &sn, &cs);
          a = w.y * cs + w.x * sn;
        }
        if (half == 0 && qq <= N / 2) put_odd(tab, fp32, (int64_t)rows[h] * (N + 1) + qq, a);
        if (half == 1 && qq < N / 2) put_odd(tab, fp32, (int64_t)rows[h] * (N + 1) + N / 2 + 1 + qq, a);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ finite check --
template <typename In>
__global__ void k_check_finite(const In* __restrict__ x, int64_t n, int* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite((double)x[i]);
  if (bad) atomicOr(flag, 1);
}

// ------------------------------------------------- coefficients (C out) --
// sigma -> C for k = 3, 4, 5 written out (sg_bspline_coeffs): the x-solve along
// rows (Eq. (C_system)) then the y-solve along columns (Eq. (z_system));
// the two commute.  The per-step force path fuses them into passes A and B.
template <int M>
struct coeff_cfg {
  static constexpr int CH = elems_for(M, 16, 12);
  static constexpr int T = M / CH;
  static constexpr int G = T >= 256 ? 1 : 256 / T;
  static constexpr int SLOT = band_smem<double, T>::BYTES / 8 + 1;
};

template <typename R, int M>
__global__ void __launch_bounds__((coeff_cfg<M>::G * coeff_cfg<M>::T))
    k_coeff_rows(const R* __restrict__ src, R* __restrict__ dst, int nrows, int sys) {
  using C = coeff_cfg<M>;
  constexpr int CH = C::CH, T = C::T;
  __shared__ double smem[C::G * C::SLOT];
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int row = blockIdx.x * C::G + g;
  const bool active = row < nrows;
  double d[CH];
  // unconditional loads (row 0 stands in for rows past nrows), masked
  const R* s = src + (int64_t)(active ? row : 0) * M + t * CH;
  const double msk = active ? band_scale(sys) : 0.0;
#pragma unroll
  for (int e = 0; e < CH; ++e) d[e] = msk * (double)s[e];
  double* sl = smem + g * C::SLOT;
  if (sys == 3)
    band_solve<3, CH, T>(d, t, sl);
  else if (sys == 4)
    band_solve<4, CH, T>(d, t, sl);
  else
    band_solve<5, CH, T>(d, t, sl);
  if (active) {
#pragma unroll
    for (int e = 0; e < CH; ++e) dst[(int64_t)row * M + t * CH + e] = (R)d[e];
  }
}

template <int N>
struct coeffc_cfg {
  static constexpr int CH = elems_for(N, 16, 12);
  static constexpr int T = N / CH;
  static constexpr int P = T >= 64 ? 1 : 64 / T;
  static constexpr int TRI = band_smem<double, T>::BYTES / 8 + 1;
  static constexpr int SLOT = (N + 1) > TRI ? (N + 1) : TRI;
};

template <typename R, int N>
__global__ void __launch_bounds__((coeffc_cfg<N>::P * coeffc_cfg<N>::T))
    k_coeff_cols(R* __restrict__ data, int M, int sys) {
  using C = coeffc_cfg<N>;
  constexpr int CH = C::CH, T = C::T, SLOT = C::SLOT;
  __shared__ double smem[C::P * SLOT];
  const int P = blockDim.x / T;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int c0 = blockIdx.x * P;
  for (int s = 0; s < CH; ++s) {
    const int l = threadIdx.x + s * P * T;
    smem[(l % P) * SLOT + l / P] = (double)data[(int64_t)(l / P) * M + c0 + l % P];
  }
  __syncthreads();
  double d[CH];
#pragma unroll
  for (int e = 0; e < CH; ++e) d[e] = band_scale(sys) * smem[g * SLOT + t * CH + e];
  __syncthreads();
  if (sys == 3)
    band_solve<3, CH, T>(d, t, smem + g * SLOT);
  else if (sys == 4)
    band_solve<4, CH, T>(d, t, smem + g * SLOT);
  else
    band_solve<5, CH, T>(d, t, smem + g * SLOT);
#pragma unroll
  for (int e = 0; e < CH; ++e) smem[g * SLOT + t * CH + e] = d[e];
  __syncthreads();
  for (int s = 0; s < CH; ++s) {
    const int l = threadIdx.x + s * P * T;
    data[(int64_t)(l / P) * M + c0 + l % P] = (R)smem[(l % P) * SLOT + l / P];
  }
}

// ------------------------------------------------------------ launches --
template <typename R>
struct tabs {
  using odd = typename std::conditional<sizeof(R) == 4, float2, double>::type;
};

// Transform lengths with kernels: SG_SIZES for the column passes of this
// file (the four-step column pass of sg_colfs.hip takes 2048, 4096 and 8192,
// the last only there), SG_ROW_SIZES for the row passes and the coefficient solves.
#ifndef SG_SIZES
#define SG_SIZES(X)                                                                                        \
  X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(12) X(24) X(48) X(96) X(192) X(384) \
      X(768) X(1536)
#endif
#ifndef SG_ROW_SIZES
#define SG_ROW_SIZES(X) SG_SIZES(X) X(8192)
#endif

// rows (or columns) per workgroup: the requested tile if it is in [1, cap],
// else cap, and never more than n
// LDS of the forward row kernel and of the Stockham column kernel: sized at
// launch for the rows (columns) per workgroup actually launched, so that a smaller
// tile than the compiled maximum leaves room for more workgroups per compute
// unit.  The first launch of each kernel allows its largest size (LDS above
// 64 KB per workgroup is opt-in on some runtimes; an error there is cleared,
// and an oversized launch then reports its own).
template <auto K>
static void dyn_lds_optin(int max_bytes) {
  static const bool once = [max_bytes] {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(K), hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes) !=
        hipSuccess)
      (void)hipGetLastError();
    return true;
  }();
  (void)once;
}

static inline int pick_tile(int tile, int cap, int n) {
  int g = (tile > 0 && tile <= cap) ? tile : cap;
  return g < n ? g : n;
}

template <typename R, typename In, int M>
static hipError_t launch_row_fwd_t(const In* src, int64_t src_ld, cx<R>* X, int nrows, const cx<R>* r2m,
                                   int solve, int full, const cx<R>* tw, const sg_bgrid* bg, int ngrids, int tile,
                                   hipStream_t st) {
  using C = rowfwd_cfg<R, In, M>;
  const int G = pick_tile(tile, C::G, nrows);
  const int blocks = (nrows + G - 1) / G;
  constexpr int row_bytes = C::SLOT * C::NB * (int)sizeof(cx<R>);
  if (solve >= 4) {
    dyn_lds_optin<&k_row_fwd<R, In, M, true>>(C::G * row_bytes);
    hipLaunchKernelGGL((k_row_fwd<R, In, M, true>), dim3(blocks, bg ? ngrids : 1), dim3(G * C::T), G * row_bytes,
                       st, src, src_ld, X, nrows, nrows, r2m, solve, full, tw, bg);
  } else {
    dyn_lds_optin<&k_row_fwd<R, In, M>>(C::G * row_bytes);
    hipLaunchKernelGGL((k_row_fwd<R, In, M>), dim3(blocks, bg ? ngrids : 1), dim3(G * C::T), G * row_bytes, st, src,
                       src_ld, X, nrows, nrows, r2m, solve, full, tw, bg);
  }
  return hipGetLastError();
}

template <typename R, int N, int VA = 0>
static hipError_t launch_col_t(const cx<R>* X, cx<R>* V, int M, int tj, const void* tx, const void* ty, int kind,
                               const cx<R>* r2n, int solve, const cx<R>* tw, const sg_bgrid* bg, int ngrids,
                               int tile, hipStream_t st) {
  using C = col_cfg<R, N, VA>;
  using TO = typename tabs<R>::odd;
  const int P = pow2_div(M, (tile > 0 && tile <= C::P) ? tile : C::P);
  const dim3 grid(M / P, bg ? ngrids : 1);
  const TO* tox = (const TO*)tx;
  const TO* toy = (const TO*)ty;
  constexpr int col_bytes = C::SLOT * C::NBUF * (int)sizeof(cx<R>);
  const int lds = P * col_bytes;
  // modes: 0 = k 1, 1 = k 2, 2 = k 3, 3 = k 4, 4 = k 5 (solve = k for k >= 3)
  auto go = [&](auto mode) {
    constexpr int MD = decltype(mode)::value;
    dyn_lds_optin<&k_col<R, TO, N, MD, VA>>(C::P * col_bytes);
    hipLaunchKernelGGL((k_col<R, TO, N, MD, VA>), grid, dim3(P * C::T), lds, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  };
  if (solve == 4)
    go(std::integral_constant<int, 3>{});
  else if (solve == 5)
    go(std::integral_constant<int, 4>{});
  else if (kind == 1)
    go(std::integral_constant<int, 1>{});
  else if (solve)
    go(std::integral_constant<int, 2>{});
  else
    go(std::integral_constant<int, 0>{});
  return hipGetLastError();
}

template <typename R, typename Out, int M, int VA = 0>
static hipError_t launch_row_inv_t(const cx<R>* V, Out* fx, Out* fy, int nrows, int tj, const cx<R>* r2m,
                                   const cx<R>* tw, const sg_bgrid* bg, int ngrids, int tile, hipStream_t st) {
  using C = rowinv_cfg<R, M, VA>;
  const int G = pick_tile(tile, C::G, nrows);
  const int blocks = (nrows + G - 1) / G;
  hipLaunchKernelGGL((k_row_inv<R, Out, M, VA>), dim3(blocks, bg ? ngrids : 1), dim3(G * C::T), 0, st, V, fx, fy, nrows,
                     tj, r2m, tw, bg);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_spec_col_t(const cx<double>* S, int M, void* tab, int kind, int fp32, double scale,
                                    const cx<double>* r2n, const cx<double>* tw, hipStream_t st) {
  using C = spec_cfg<N>;
  hipLaunchKernelGGL((k_spec_col<N>), dim3(M), dim3(C::T), 0, st, S, M, tab, kind, fp32, scale, r2n, tw);
  return hipGetLastError();
}

}  // namespace sg

// ------------------------------------------------- dispatch (host side) --
using namespace sg;

#if SG_IN_PART(0)
hipError_t sg_launch_weights(int k, double hx, double hy, int M, int N, double* wx, double* wy, int layout,
                             hipStream_t st) {
  const int64_t total = (int64_t)(layout == 0 ? 2 * M : 2 * M - 1) * (layout == 0 ? 2 * N : 2 * N - 1);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_weights, dim3((unsigned)blocks), dim3(256), 0, st, k, hx, hy, M, N, wx, wy, layout);
  return hipGetLastError();
}

hipError_t sg_set_gl_tables(const double* x, const double* w) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_glx), x, sizeof(double) * 64);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_glw), w, sizeof(double) * 64);
}

#endif

#if SG_IN_PART(1)
template <typename R, typename In>
static hipError_t row_fwd_dispatch(int M, const In* src, int64_t ld, cx<R>* X, int nrows, const cx<R>* r2m,
                                   int solve, int full, const cx<R>* tw, const sg_bgrid* bg, int ngrids, int tile,
                                   hipStream_t st) {
  switch (M) {
#define CASE(SZ) \
  case SZ:       \
    return launch_row_fwd_t<R, In, SZ>(src, ld, X, nrows, r2m, solve, full, tw, bg, ngrids, tile, st);
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

#endif

#if SG_IN_PART(2)
template <typename R>
static hipError_t col_dispatch(int N, const cx<R>* X, cx<R>* V, int M, int tj, const void* tx, const void* ty,
                               int kind, const cx<R>* r2n, int solve, const cx<R>* tw, const sg_bgrid* bg,
                               int ngrids, int tile, int variant, hipStream_t st) {
  switch (N) {
#define CASE(SZ)                                                                                        \
  case SZ:                                                                                              \
    if (sizeof(R) == 4 && variant == 1 && col_variants<SZ>())                                           \
      return launch_col_t<R, SZ, col_variants<SZ>() ? 1 : 0>(X, V, M, tj, tx, ty, kind, r2n, solve, tw, bg, \
                                                              ngrids, tile, st);                        \
    return launch_col_t<R, SZ>(X, V, M, tj, tx, ty, kind, r2n, solve, tw, bg, ngrids, tile, st);
    SG_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

#endif

#if SG_IN_PART(1)
template <typename R, typename Out>
static hipError_t row_inv_dispatch(int M, const cx<R>* V, Out* fx, Out* fy, int nrows, int tj, const cx<R>* r2m,
                                   const cx<R>* tw, const sg_bgrid* bg, int ngrids, int tile, int variant,
                                   hipStream_t st) {
  switch (M) {
#define CASE(SZ)                                                                                            \
  case SZ:                                                                                                  \
    if (sizeof(R) == 4 && variant == 1 && rowinv_variants<SZ>())                                            \
      return launch_row_inv_t<R, Out, SZ, rowinv_variants<SZ>() ? 1 : 0>(V, fx, fy, nrows, tj, r2m, tw, bg, \
                                                                          ngrids, tile, st);                \
    return launch_row_inv_t<R, Out, SZ>(V, fx, fy, nrows, tj, r2m, tw, bg, ngrids, tile, st);
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

#endif

#if SG_IN_PART(1)
hipError_t sg_launch_row_fwd(int prec, int M, const void* src, int64_t ld, void* X, int nrows, const void* r2m,
                             int solve, int full, const void* tw, const sg_bgrid* bg, int ngrids, int tile,
                             hipStream_t st) {
  if (prec == 0)
    return row_fwd_dispatch<double, double>(M, (const double*)src, ld, (cx<double>*)X, nrows,
                                            (const cx<double>*)r2m, solve, full, (const cx<double>*)tw, bg, ngrids,
                                            tile, st);
  return row_fwd_dispatch<float, float>(M, (const float*)src, ld, (cx<float>*)X, nrows, (const cx<float>*)r2m,
                                        solve, full, (const cx<float>*)tw, bg, ngrids, tile, st);
}

#endif

#if SG_IN_PART(2)
hipError_t sg_launch_col(int prec, int N, const void* X, void* V, int M, int tj, const void* tx, const void* ty,
                         int kind, const void* r2n, int solve, const void* tw, const sg_bgrid* bg, int ngrids,
                         int tile, int variant, hipStream_t st) {
  if (prec == 0)
    return col_dispatch<double>(N, (const cx<double>*)X, (cx<double>*)V, M, tj, tx, ty, kind,
                                (const cx<double>*)r2n, solve, (const cx<double>*)tw, bg, ngrids, tile, 0, st);
  return col_dispatch<float>(N, (const cx<float>*)X, (cx<float>*)V, M, tj, tx, ty, kind, (const cx<float>*)r2n,
                             solve, (const cx<float>*)tw, bg, ngrids, tile, variant, st);
}

int sg_row_tile(int prec, int M, int N) {
  (void)M;
  // a power of two that divides N (tiles never straddle the last row)
  return pow2_div(N, prec == 0 ? SG_TJ64 : SG_TJ32);
}

#endif

#if SG_IN_PART(1)
hipError_t sg_launch_row_inv(int prec, int M, const void* V, void* fx, void* fy, int nrows, int tj, const void* r2m,
                             const void* tw, const sg_bgrid* bg, int ngrids, int tile, int variant, hipStream_t st) {
  if (prec == 0)
    return row_inv_dispatch<double, double>(M, (const cx<double>*)V, (double*)fx, (double*)fy, nrows, tj,
                                            (const cx<double>*)r2m, (const cx<double>*)tw, bg, ngrids, tile, 0, st);
  return row_inv_dispatch<float, float>(M, (const cx<float>*)V, (float*)fx, (float*)fy, nrows, tj,
                                        (const cx<float>*)r2m, (const cx<float>*)tw, bg, ngrids, tile, variant, st);
}

// Largest tile of a pass (0 = A rows, 1 = B columns, 2 = C rows) for a
// transform length (M for A and C, N for B); 0 for an unsupported length.
template <typename R>
static int max_tile_t(int pass, int len, int v) {
  switch (len) {
#define CASE(SZ)                                                                       \
  case SZ:                                                                             \
    if (pass == 0) return rowfwd_cfg<R, R, SZ>::G;                                     \
    if (pass == 1) return SZ > 4096 ? 1 : (v ? col_cfg<R, SZ, 1>::P : col_cfg<R, SZ>::P); \
    return v ? rowinv_cfg<R, SZ, 1>::G : rowinv_cfg<R, SZ>::G;
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return 0;
  }
}

int sg_variants(int prec, int pass, int len) {
  if (prec == 0) return 1;
  switch (len) {
#define CASE(SZ)                                                        \
  case SZ:                                                              \
    if (pass == 1) return (SZ <= 4096 && col_variants<SZ>()) ? 2 : 1; \
    if (pass == 2) return rowinv_variants<SZ>() ? 2 : 1;                \
    return 1;
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return 0;
  }
}

int sg_default_variant(int prec, int pass, int len) {
  return (prec == 1 && pass == 2 && len >= SG_RI_BIG32 && sg_variants(prec, pass, len) > 1) ? 1 : 0;
}

int sg_max_tile(int prec, int pass, int len, int variant) {
  if (variant < 0 || variant >= sg_variants(prec, pass, len)) return 0;
  return prec == 0 ? max_tile_t<double>(pass, len, 0) : max_tile_t<float>(pass, len, variant);
}

#endif

#if SG_IN_PART(0)
hipError_t sg_launch_spec_col(int N, const void* rowspec, int M, void* tab, int kind, int fp32, double scale,
                              const void* r2n, const void* tw, hipStream_t st) {
  switch (N) {
#define CASE(SZ) \
  case SZ:       \
    return launch_spec_col_t<SZ>((const cx<double>*)rowspec, M, tab, kind, fp32, scale, (const cx<double>*)r2n, \
                                (const cx<double>*)tw, st);
    SG_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t sg_launch_check_finite(int prec, const void* x, int64_t n, int* flag, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  if (prec == 0)
    hipLaunchKernelGGL(k_check_finite<double>, dim3((unsigned)blocks), dim3(256), 0, st, (const double*)x, n, flag);
  else
    hipLaunchKernelGGL(k_check_finite<float>, dim3((unsigned)blocks), dim3(256), 0, st, (const float*)x, n, flag);
  return hipGetLastError();
}

template <typename R>
static hipError_t coeff_rows_dispatch(int M, const R* src, R* dst, int nrows, int sys, hipStream_t st) {
  switch (M) {
#define CASE(SZ)                                                                                     \
  case SZ: {                                                                                         \
    using C = coeff_cfg<SZ>;                                                                         \
    hipLaunchKernelGGL((k_coeff_rows<R, SZ>), dim3((nrows + C::G - 1) / C::G), dim3(C::G * C::T), 0, st, src, \
                       dst, nrows, sys);                                                            \
    return hipGetLastError();                                                                       \
  }
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R>
static hipError_t coeff_cols_dispatch(int N, R* data, int M, int sys, hipStream_t st) {
  switch (N) {
#define CASE(SZ)                                                                                      \
  case SZ: {                                                                                          \
    using C = coeffc_cfg<SZ>;                                                                         \
    const int P = pow2_div(M, C::P);                                                               \
    hipLaunchKernelGGL((k_coeff_cols<R, SZ>), dim3(M / P), dim3(P * C::T), 0, st, data, M, sys);      \
    return hipGetLastError();                                                                        \
  }
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t sg_launch_coeff_rows(int prec, int M, const void* src, void* dst, int nrows, int k, hipStream_t st) {
  if (k < 3 || k > 5) return hipErrorInvalidValue;
  if (prec == 0) return coeff_rows_dispatch<double>(M, (const double*)src, (double*)dst, nrows, k, st);
  return coeff_rows_dispatch<float>(M, (const float*)src, (float*)dst, nrows, k, st);
}

hipError_t sg_launch_coeff_cols(int prec, int N, void* data, int M, int k, hipStream_t st) {
  if (k < 3 || k > 5) return hipErrorInvalidValue;
  if (prec == 0) return coeff_cols_dispatch<double>(N, (double*)data, M, k, st);
  return coeff_cols_dispatch<float>(N, (float*)data, M, k, st);
}

// ------------------------------------------------- stage twiddle tables --
template <typename R, int L, int E>
__global__ void k_build_tw(const cx<R>* __restrict__ roots, int stride, cx<R>* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < plan<L, E>::tw_size) build_stage_twiddles<L, E>(roots_t<R>{roots, stride}, out, idx);
}

template <typename R, int L, int E>
static int tw_build(const void* roots, int stride, void* out, hipStream_t st) {
  constexpr int n = plan<L, E>::tw_size;
  if (out && n > 0)
    hipLaunchKernelGGL((k_build_tw<R, L, E>), dim3((n + 255) / 256), dim3(256), 0, st, (const cx<R>*)roots, stride,
                       (cx<R>*)out);
  return n;
}

// pass: 0 = forward rows (length M/2), 1 = columns (N), 2 = inverse rows (M),
// 3 = plan-time spectrum columns (N, FP64), 4 = inverse rows in launch
// variant 1 (FP32).  len = M or N.  roots: the
// table of the 2*len-th roots in the pass precision.  With out == NULL only
// the entry count is returned; otherwise the table is filled on st.
template <typename R>
static int tw_dispatch(int pass, int len, const void* roots, void* out, hipStream_t st) {
  switch (len) {
#define CASE(SZ)                                                                                         \
  case SZ:                                                                                               \
    if (pass == 0) return tw_build<R, SZ / 2, rowfwd_cfg<R, R, SZ>::E>(roots, 4, out, st);               \
    if (pass == 1) return tw_build<R, SZ, col_cfg<R, SZ>::E>(roots, 2, out, st);                         \
    if (pass == 2) return tw_build<R, SZ, rowinv_cfg<R, SZ>::E>(roots, 2, out, st);                      \
    if (pass == 3) return tw_build<R, SZ, spec_cfg<SZ>::E>(roots, 2, out, st);                           \
    if (pass == 4) return tw_build<R, SZ, rowinv_cfg<R, SZ, 1>::E>(roots, 2, out, st);                   \
    return -1;
    SG_SIZES(CASE)
#undef CASE
    case 8192:  // row passes only (the columns of this length take the four-step pass)
      if (pass == 0) return tw_build<R, 4096, rowfwd_cfg<R, R, 8192>::E>(roots, 4, out, st);
      if (pass == 2) return tw_build<R, 8192, rowinv_cfg<R, 8192>::E>(roots, 2, out, st);
      if (pass == 4) return tw_build<R, 8192, rowinv_cfg<R, 8192, 1>::E>(roots, 2, out, st);
      return 0;
    default:
      return -1;
  }
}

int sg_twiddles(int prec, int pass, int len, const void* roots, void* out, hipStream_t st) {
  if (pass == 3 && prec != 0) return -1;
  if (pass == 4 && (prec != 1 || sg_variants(1, 2, len) < 2)) return -1;
  return prec == 0 ? tw_dispatch<double>(pass, len, roots, out, st) : tw_dispatch<float>(pass, len, roots, out, st);
}

#endif

#if SG_IN_PART(3)
// ------------------------------------------------------ adjoint launches --
template <typename R, int N>
static hipError_t launch_col_adj_t(const cx<R>* Xx, const cx<R>* Xy, cx<R>* Y, int M, int tj, const void* tx,
                                   const void* ty, int kind, const cx<R>* r2n, int solve, const cx<R>* tw,
                                   const sg_bgrid* bg, int ngrids, hipStream_t st) {
  using C = col_cfg<R, N>;
  using TO = typename tabs<R>::odd;
  const int P = pow2_div(M, C::P);
  const dim3 grid(M / P, bg ? ngrids : 1);
  const TO* tox = (const TO*)tx;
  const TO* toy = (const TO*)ty;
  // modes: 0 = k 1, 1 = k 2, 2 = k 3, 3 = k 4, 4 = k 5 (solve = k for k >= 3)
  if (solve == 4)
    hipLaunchKernelGGL((k_col_adj<R, TO, N, 3>), grid, dim3(P * C::T), 0, st, Xx, Xy, Y, M, tj, tox, toy,
                       r2n, tw, bg);
  else if (solve == 5)
    hipLaunchKernelGGL((k_col_adj<R, TO, N, 4>), grid, dim3(P * C::T), 0, st, Xx, Xy, Y, M, tj, tox, toy,
                       r2n, tw, bg);
  else if (kind == 1)
    hipLaunchKernelGGL((k_col_adj<R, TO, N, 1>), grid, dim3(P * C::T), 0, st, Xx, Xy, Y, M, tj, tox, toy,
                       r2n, tw, bg);
  else if (solve)
    hipLaunchKernelGGL((k_col_adj<R, TO, N, 2>), grid, dim3(P * C::T), 0, st, Xx, Xy, Y, M, tj, tox, toy,
                       r2n, tw, bg);
  else
    hipLaunchKernelGGL((k_col_adj<R, TO, N, 0>), grid, dim3(P * C::T), 0, st, Xx, Xy, Y, M, tj, tox, toy,
                       r2n, tw, bg);
  return hipGetLastError();
}

template <typename R, int M>
static hipError_t launch_row_c2r_t(const cx<R>* Y, R* out, int nrows, int tj, const cx<R>* r2m, int solve,
                                   const cx<R>* tw, const sg_bgrid* bg, int ngrids, hipStream_t st) {
  using C = rowfwd_cfg<R, R, M>;
  if (solve >= 4) {
    constexpr int GH = rowc2r_cfg<R, M, true>::G;
    const int G = GH < nrows ? GH : nrows;
    hipLaunchKernelGGL((k_row_c2r<R, R, M, true>), dim3((nrows + G - 1) / G, bg ? ngrids : 1), dim3(G * C::T), 0, st,
                       Y, out, nrows, tj, r2m, solve, tw, bg);
  } else {
    const int G = C::G < nrows ? C::G : nrows;
    hipLaunchKernelGGL((k_row_c2r<R, R, M>), dim3((nrows + G - 1) / G, bg ? ngrids : 1), dim3(G * C::T), 0, st, Y,
                       out, nrows, tj, r2m, solve, tw, bg);
  }
  return hipGetLastError();
}

template <typename R>
static hipError_t adj_dispatch(int M, int N, const cx<R>* Xx, const cx<R>* Xy, cx<R>* Y, R* out, int tj,
                               const void* tx, const void* ty, int kind, const cx<R>* r2m, const cx<R>* r2n,
                               int solve, const cx<R>* twB, const cx<R>* twA, const sg_bgrid* bg, int ngrids,
                               hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  switch (N) {
#define CASE(SZ)                                                                                  \
  case SZ:                                                                                        \
    e = launch_col_adj_t<R, SZ>(Xx, Xy, Y, M, tj, tx, ty, kind, r2n, solve, twB, bg, ngrids, st); \
    break;
    SG_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (M) {
#define CASE(SZ) \
  case SZ:       \
    return launch_row_c2r_t<R, SZ>(Y, out, N, tj, r2m, solve, twA, bg, ngrids, st);
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R>
static hipError_t c2r_dispatch(int M, int N, const cx<R>* Y, R* out, int tj, const cx<R>* r2m, int solve,
                               const cx<R>* twA, const sg_bgrid* bg, int ngrids, hipStream_t st) {
  switch (M) {
#define CASE(SZ) \
  case SZ:       \
    return launch_row_c2r_t<R, SZ>(Y, out, N, tj, r2m, solve, twA, bg, ngrids, st);
    SG_ROW_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t sg_launch_row_c2r(int prec, int M, int N, const void* Y, void* gsigma, int tj, const void* r2m, int solve,
                             const void* twA, const sg_bgrid* bg, int ngrids, hipStream_t st) {
  if (prec == 0)
    return c2r_dispatch<double>(M, N, (const cx<double>*)Y, (double*)gsigma, tj, (const cx<double>*)r2m, solve,
                                (const cx<double>*)twA, bg, ngrids, st);
  return c2r_dispatch<float>(M, N, (const cx<float>*)Y, (float*)gsigma, tj, (const cx<float>*)r2m, solve,
                             (const cx<float>*)twA, bg, ngrids, st);
}

hipError_t sg_launch_adjoint_tail(int prec, int M, int N, const void* Xx, const void* Xy, void* Y, void* gsigma,
                                  int tj, const void* tx, const void* ty, int kind, const void* r2m, const void* r2n,
                                  int solve, const void* twB, const void* twA, const sg_bgrid* bg, int ngrids,
                                  hipStream_t st) {
  if (prec == 0)
    return adj_dispatch<double>(M, N, (const cx<double>*)Xx, (const cx<double>*)Xy, (cx<double>*)Y, (double*)gsigma,
                                tj, tx, ty, kind, (const cx<double>*)r2m, (const cx<double>*)r2n, solve,
                                (const cx<double>*)twB, (const cx<double>*)twA, bg, ngrids, st);
  return adj_dispatch<float>(M, N, (const cx<float>*)Xx, (const cx<float>*)Xy, (cx<float>*)Y, (float*)gsigma, tj, tx,
                             ty, kind, (const cx<float>*)r2m, (const cx<float>*)r2n, solve, (const cx<float>*)twB,
                             (const cx<float>*)twA, bg, ngrids, st);
}
#endif
