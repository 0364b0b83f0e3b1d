// Launches of the four-step column pass (colfs.hpp) for the long columns:
// N = 2048, 4096 and 8192 (and 1024 in FP64), one workgroup of N / E threads per
// column; and of the radix-3 form for columns of 1536 and 768, FP32
// (colfs3.hpp, forward only), one workgroup of three waves per column.  For a batch,
// blockIdx.y is the grid of the class.
#include <type_traits>

#include "colfs3.hpp"

#ifndef SG_COLFS_SPLIT_F4096
#define SG_COLFS_SPLIT_F4096 0
#endif
#ifndef SG_COLFS_E_F4096
#define SG_COLFS_E_F4096 8
#endif
#ifndef SG_COLFS_SLOTS_F4096
#define SG_COLFS_SLOTS_F4096 4
#endif
#ifndef SG_COLFS_SPLIT_D4096
#define SG_COLFS_SPLIT_D4096 0
#endif
// the prefetching persistent loop (FP32, 4096, single-float tables)
#ifndef SG_COLFS_PF
#define SG_COLFS_PF 1
#endif
// component split (FP32 columns of 8192): both passes in one launch (1) or two
#ifndef SG_COLFS_XY
#define SG_COLFS_XY 1
#endif
// ... and for columns of 2048 (two workgroups per compute unit)
#ifndef SG_COLFS_PF2048
#define SG_COLFS_PF2048 0
#endif

namespace sg {

// elements per thread, LDS slots and component split per precision and
// length (chosen so that no kernel spills registers)
template <typename R, int N>
struct colfs_sel {
  static constexpr bool ok = false;
};
// FP32 columns of 2048: two slots (34 KB of LDS) and registers capped at
// three waves per SIMD (colfs_wpe), so that three workgroups share a
// compute unit
#ifndef SG_COLFS_SLOTS_F2048
#define SG_COLFS_SLOTS_F2048 2
#endif
template <>
struct colfs_sel<float, 1024> {
  static constexpr bool ok = true;
  static constexpr int E = 8, SLOTS = 4, SPLIT = 0;
};
template <>
struct colfs_sel<double, 1024> {
  static constexpr bool ok = true;
  static constexpr int E = 8, SLOTS = 2, SPLIT = 0;
};
template <>
struct colfs_sel<float, 2048> {
  static constexpr bool ok = true;
  static constexpr int E = 8, SLOTS = SG_COLFS_SLOTS_F2048, SPLIT = 0;
};
template <>
struct colfs_sel<double, 2048> {
  static constexpr bool ok = true;
  static constexpr int E = 8, SLOTS = 2, SPLIT = 0;
};
template <>
struct colfs_sel<float, 4096> {
  static constexpr bool ok = true;
  static constexpr int E = SG_COLFS_E_F4096, SLOTS = SG_COLFS_SLOTS_F4096, SPLIT = SG_COLFS_SPLIT_F4096;
};
template <>
struct colfs_sel<float, 8192> {
  static constexpr bool ok = true;
  static constexpr int E = 16, SLOTS = 2, SPLIT = 1;
};
template <>
struct colfs_sel<double, 4096> {
  static constexpr bool ok = true;
  static constexpr int E = 8, SLOTS = 2, SPLIT = SG_COLFS_SPLIT_D4096;
};
template <>
struct colfs_sel<double, 8192> {
  static constexpr bool ok = true;
  static constexpr int E = 16, SLOTS = 1, SPLIT = 1;
};

// Compute units of the current device (the persistent launches' width).
static int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return n > 0 ? n : 256;
}

// The prefetching loop for FP32 columns of 4096 with single-float tables
// (its registers fit only then): one workgroup per compute unit.
template <typename R, typename TO, int N, int MODE>
struct colfs_pf {
  // odd orders only: the even orders' bin phases leave no registers for it
  static constexpr bool on = sizeof(R) == 4 && sizeof(TO) == 4 && (MODE % 2 == 0) &&
                             ((N == 4096 && SG_COLFS_PF) || (N == 2048 && SG_COLFS_PF2048));
  static constexpr int per_cu = N == 2048 ? 2 : 1;  // resident workgroups per compute unit
};

template <typename R, typename TO, int N, int MODE, int COMP>
static void launch_colfs_k(const cx<R>* X, cx<R>* V, int M, int tj, const TO* tox, const TO* toy, const cx<R>* r2n,
                           const cx<R>* tw, const sg_bgrid* bg, int ngrids, hipStream_t st) {
  using Sel = colfs_sel<R, N>;
  if constexpr (colfs_pf<R, TO, N, MODE>::on && COMP == 0) {
    static const int cus = device_cus();
    const int slots = cus * colfs_pf<R, TO, N, MODE>::per_cu;
    const int nb = M < slots ? M : slots;
    hipLaunchKernelGGL((k_colfs<R, TO, N, MODE, Sel::E, Sel::SLOTS, COMP, true>), dim3(nb, bg ? ngrids : 1),
                       dim3(N / Sel::E), 0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  } else {
    hipLaunchKernelGGL((k_colfs<R, TO, N, MODE, Sel::E, Sel::SLOTS, COMP>), dim3(M, bg ? ngrids : 1),
                       dim3(N / Sel::E), 0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  }
}

template <typename R, typename TO, int N, int MODE>
static hipError_t launch_colfs_m(const cx<R>* X, cx<R>* V, int M, int tj, const TO* tox, const TO* toy,
                                 const cx<R>* r2n, const cx<R>* tw, const sg_bgrid* bg, int ngrids, hipStream_t st) {
  using Sel = colfs_sel<R, N>;
  if constexpr (Sel::SPLIT && SG_COLFS_XY && sizeof(R) == 4) {
    // both component passes of a column in one launch
    hipLaunchKernelGGL((k_colfs_xy<R, TO, N, MODE, Sel::E, Sel::SLOTS>), dim3(M, bg ? ngrids : 1), dim3(N / Sel::E),
                       0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  } else if constexpr (Sel::SPLIT) {
    launch_colfs_k<R, TO, N, MODE, 1>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
    launch_colfs_k<R, TO, N, MODE, 2>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  } else {
    launch_colfs_k<R, TO, N, MODE, 0>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  }
  return hipGetLastError();
}

template <typename R, typename TO, int N>
static hipError_t launch_colfs_t(const cx<R>* X, cx<R>* V, int M, int tj, const void* tx, const void* ty, int kind,
                                 const cx<R>* r2n, int solve, const cx<R>* tw, const sg_bgrid* bg, int ngrids,
                                 hipStream_t st) {
  const TO* tox = (const TO*)tx;
  const TO* toy = (const TO*)ty;
  // modes: 0 = k 1, 1 = k 2, 2 = k 3, 3 = k 4, 4 = k 5 (solve = k for k >= 3)
  if (solve == 4) return launch_colfs_m<R, TO, N, 3>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  if (solve == 5) return launch_colfs_m<R, TO, N, 4>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  if (kind == 1) return launch_colfs_m<R, TO, N, 1>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  if (solve) return launch_colfs_m<R, TO, N, 2>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  return launch_colfs_m<R, TO, N, 0>(X, V, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
}

template <typename R, int N>
static int colfs_twiddles_t(double* re, double* im) {
  using Sel = colfs_sel<R, N>;
  using S = fs_shape<N, Sel::E>;
  if (re && im)
    fs_fill_twiddles<N, Sel::E>(
        [](int m, int L, double* cr, double* ci) {
          // exp(-2 pi i m / L) from long double, rounded once
          const long double a = 6.283185307179586476925286766559005768L * (long double)m / (long double)L;
          *cr = (double)cosl(a);
          *ci = (double)-sinl(a);
        },
        re, im);
  return S::TW_SIZE;
}

}  // namespace sg

using namespace sg;

// 1: forward and adjoint; 2: forward only (the radix-3 columns of 1536 and
// 768).  Columns of 1024 take the
// four-step pass in FP64 only (FP32: the Stockham kernel, at 100-116
// registers, measured faster).
int sg_colfs_supported(int prec, int N) {
  if (N == 2048 || N == 4096 || N == 8192) return 1;
  if (N == 1024) return prec == 0 ? 1 : 0;
  return ((N == 1536 || N == 768) && prec == 1) ? 2 : 0;
}

int sg_colfs_twiddles(int prec, int N, double* re, double* im) {
  if (!sg_colfs_supported(prec, N)) return -1;
  if (N == 1536 || N == 768) {
    // the three waves' 512-point transforms (null re, im: the size only); the
    // 256-point ones of 768 take their twiddles from the 2N-roots table and
    // ignore it
    if (re && im)
      fs_fill_twiddles<512, 8>(
        [](int m, int L, double* cr, double* ci) {
          const long double a = 6.283185307179586476925286766559005768L * (long double)m / (long double)L;
          *cr = (double)cosl(a);
          *ci = (double)-sinl(a);
        },
        re, im);
    return fs_shape<512, 8>::TW_SIZE;
  }
  if (prec == 0)
    return N == 1024 ? colfs_twiddles_t<double, 1024>(re, im)
                     : N == 2048 ? colfs_twiddles_t<double, 2048>(re, im)
                                 : (N == 4096 ? colfs_twiddles_t<double, 4096>(re, im)
                                              : colfs_twiddles_t<double, 8192>(re, im));
  return N == 1024 ? colfs_twiddles_t<float, 1024>(re, im)
                   : N == 2048 ? colfs_twiddles_t<float, 2048>(re, im)
                               : (N == 4096 ? colfs_twiddles_t<float, 4096>(re, im)
                                            : colfs_twiddles_t<float, 8192>(re, im));
}

namespace sg {
// f(integral_constant<N>) for the supported lengths
template <typename F>
static hipError_t colfs_len(int N, F f) {
  if (N == 1024) return f(std::integral_constant<int, 1024>{});
  if (N == 2048) return f(std::integral_constant<int, 2048>{});
  if (N == 4096) return f(std::integral_constant<int, 4096>{});
  if (N == 8192) return f(std::integral_constant<int, 8192>{});
  return hipErrorInvalidValue;
}
}  // namespace sg

namespace sg {
template <typename TO, int L>
static hipError_t launch_colfs3(const cx<float>* X, cx<float>* V, int M, int tj, const void* tx, const void* ty,
                                int kind, const cx<float>* r2n, int solve, const cx<float>* tw, const sg_bgrid* bg,
                                int ngrids, hipStream_t st) {
  const TO* tox = (const TO*)tx;
  const TO* toy = (const TO*)ty;
  const dim3 grid(M, bg ? ngrids : 1), blk(kC3T);
  if (solve == 4)
    hipLaunchKernelGGL((k_colfs3<float, TO, 3, L>), grid, blk, 0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  else if (solve == 5)
    hipLaunchKernelGGL((k_colfs3<float, TO, 4, L>), grid, blk, 0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  else if (kind == 1)
    hipLaunchKernelGGL((k_colfs3<float, TO, 1, L>), grid, blk, 0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  else if (solve)
    hipLaunchKernelGGL((k_colfs3<float, TO, 2, L>), grid, blk, 0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  else
    hipLaunchKernelGGL((k_colfs3<float, TO, 0, L>), grid, blk, 0, st, X, V, M, tj, tox, toy, r2n, tw, bg);
  return hipGetLastError();
}
}  // namespace sg

hipError_t sg_launch_colfs(int prec, int N, const void* X, void* V, int M, int tj, const void* tx, const void* ty,
                           int kind, int tab_bytes, const void* r2n, int solve, const void* tw, const sg_bgrid* bg,
                           int ngrids, hipStream_t st) {
  if (N == 1536 || N == 768) {
    if (prec != 1 || tab_bytes != 8) return hipErrorInvalidValue;
    auto go = [&](auto ll) {
      return launch_colfs3<float2, decltype(ll)::value>((const cx<float>*)X, (cx<float>*)V, M, tj, tx, ty, kind,
                                                        (const cx<float>*)r2n, solve, (const cx<float>*)tw, bg, ngrids,
                                                        st);
    };
    return N == 1536 ? go(std::integral_constant<int, 512>{}) : go(std::integral_constant<int, 256>{});
  }
  if (prec == 0) {
    if (tab_bytes != 8) return hipErrorInvalidValue;
    const cx<double>* Xd = (const cx<double>*)X;
    cx<double>* Vd = (cx<double>*)V;
    const cx<double>* rd = (const cx<double>*)r2n;
    const cx<double>* td = (const cx<double>*)tw;
    return colfs_len(N, [&](auto n) {
      return launch_colfs_t<double, double, decltype(n)::value>(Xd, Vd, M, tj, tx, ty, kind, rd, solve, td, bg, ngrids,
                                                                st);
    });
  }
  const cx<float>* Xf = (const cx<float>*)X;
  cx<float>* Vf = (cx<float>*)V;
  const cx<float>* rf = (const cx<float>*)r2n;
  const cx<float>* tf = (const cx<float>*)tw;
  return colfs_len(N, [&](auto n) {
    constexpr int NN = decltype(n)::value;
    if (tab_bytes == 8)
      return launch_colfs_t<float, float2, NN>(Xf, Vf, M, tj, tx, ty, kind, rf, solve, tf, bg, ngrids, st);
    return launch_colfs_t<float, float, NN>(Xf, Vf, M, tj, tx, ty, kind, rf, solve, tf, bg, ngrids, st);
  });
}

// ---------------------------------------------------------------- adjoint --
namespace sg {
template <typename R, int N>
struct colfs_adj_sel {
  static constexpr int E = N == 8192 ? 16 : 8;
  static constexpr int SLOTS = (sizeof(R) == 8 && N == 8192) ? 1 : 2;
};

template <typename R, typename TO, int N, int MODE>
static hipError_t launch_colfs_adj_m(const cx<R>* Xx, const cx<R>* Xy, cx<R>* Y, int M, int tj, const TO* tox,
                                     const TO* toy, const cx<R>* r2n, const cx<R>* tw, const sg_bgrid* bg,
                                     int ngrids, hipStream_t st) {
  using Sel = colfs_adj_sel<R, N>;
  hipLaunchKernelGGL((k_colfs_adj<R, TO, N, MODE, Sel::E, Sel::SLOTS>), dim3(M, bg ? ngrids : 1), dim3(N / Sel::E), 0,
                     st, Xx, Xy, Y, M, tj, tox, toy, r2n, tw, bg);
  return hipGetLastError();
}

template <typename R, typename TO, int N>
static hipError_t launch_colfs_adj_t(const cx<R>* Xx, const cx<R>* Xy, cx<R>* Y, int M, int tj, const void* tx,
                                     const void* ty, int kind, const cx<R>* r2n, int solve, const cx<R>* tw,
                                     const sg_bgrid* bg, int ngrids, hipStream_t st) {
  const TO* tox = (const TO*)tx;
  const TO* toy = (const TO*)ty;
  if (solve == 4) return launch_colfs_adj_m<R, TO, N, 3>(Xx, Xy, Y, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  if (solve == 5) return launch_colfs_adj_m<R, TO, N, 4>(Xx, Xy, Y, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  if (kind == 1) return launch_colfs_adj_m<R, TO, N, 1>(Xx, Xy, Y, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  if (solve) return launch_colfs_adj_m<R, TO, N, 2>(Xx, Xy, Y, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
  return launch_colfs_adj_m<R, TO, N, 0>(Xx, Xy, Y, M, tj, tox, toy, r2n, tw, bg, ngrids, st);
}
}  // namespace sg

hipError_t sg_launch_colfs_adj(int prec, int N, const void* Xx, const void* Xy, void* Y, int M, int tj, const void* tx,
                               const void* ty, int kind, int tab_bytes, const void* r2n, int solve, const void* tw,
                               const sg_bgrid* bg, int ngrids, hipStream_t st) {
  if (prec == 0) {
    if (tab_bytes != 8) return hipErrorInvalidValue;
    const cx<double>* a = (const cx<double>*)Xx;
    const cx<double>* b = (const cx<double>*)Xy;
    cx<double>* y = (cx<double>*)Y;
    const cx<double>* rd = (const cx<double>*)r2n;
    const cx<double>* td = (const cx<double>*)tw;
    return colfs_len(N, [&](auto n) {
      return launch_colfs_adj_t<double, double, decltype(n)::value>(a, b, y, M, tj, tx, ty, kind, rd, solve, td, bg,
                                                                    ngrids, st);
    });
  }
  const cx<float>* a = (const cx<float>*)Xx;
  const cx<float>* b = (const cx<float>*)Xy;
  cx<float>* y = (cx<float>*)Y;
  const cx<float>* rf = (const cx<float>*)r2n;
  const cx<float>* tf = (const cx<float>*)tw;
  return colfs_len(N, [&](auto n) {
    constexpr int NN = decltype(n)::value;
    if (tab_bytes == 8)
      return launch_colfs_adj_t<float, float2, NN>(a, b, y, M, tj, tx, ty, kind, rf, solve, tf, bg, ngrids, st);
    return launch_colfs_adj_t<float, float, NN>(a, b, y, M, tj, tx, ty, kind, rf, solve, tf, bg, ngrids, st);
  });
}

// ------------------------------------------------------- spectrum (plan) --
hipError_t sg_launch_specfs(int N, const void* rowspec, int M, void* tab, int kind, int fp32, double scale,
                            const void* r2n, const void* tw, hipStream_t st) {
  if (N != 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_specfs<8192, 16>), dim3(M), dim3(512), 0, st, (const cx<double>*)rowspec, M, tab, kind, fp32,
                     scale, (const cx<double>*)r2n, (const cx<double>*)tw);
  return hipGetLastError();
}
