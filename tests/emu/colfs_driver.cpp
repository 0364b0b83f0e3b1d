// Host driver of the CPU emulation of the four-step column kernels: reads
// the kernel's inputs from a file written by the test, runs the kernel over
// every column, writes its output.  Configuration at compile time: EMU_KERNEL
// (0 the column pass k_colfs, 1 the adjoint column pass k_colfs_adj, 2 the
// plan-time spectrum columns k_specfs, 3 the column pass of 1536 or 768, k_colfs3),
// EMU_R (float|double), EMU_N, EMU_E,
// EMU_SLOTS, EMU_MODE, EMU_TO (table element type), EMU_SPLIT (1: the
// component-split pair of column-pass launches, x then y; 2: both in one
// launch, k_colfs_xy).
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#include <cmath>
#include <type_traits>
#include <vector>

#include "colfs3.hpp"

using namespace sg;
using R = EMU_R;
using TO = EMU_TO;
constexpr int N = EMU_N, E = EMU_E, SLOTS = EMU_SLOTS, MODE = EMU_MODE, SPLIT = EMU_SPLIT;

template <typename T>
static void rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  if (fread(v.data(), sizeof(T), n, f) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
}

#ifndef EMU_KERNEL
#define EMU_KERNEL 0
#endif

#ifndef EMU_PF
#define EMU_PF 0
#endif

template <int CP>
static void run_one(int M, int tj, std::vector<cx<R>>& X, std::vector<cx<R>>& V, std::vector<TO>& tx,
                    std::vector<TO>& ty, std::vector<cx<R>>& r2n, std::vector<cx<R>>& tw) {
  // EMU_PF: the prefetching loop with two workgroups, each taking several columns
  emu::launch(dim3(EMU_PF ? 2 : M), dim3(N / E), [&] {
    k_colfs<R, TO, N, MODE, E, SLOTS, CP, (bool)EMU_PF>(X.data(), V.data(), M, tj, tx.data(), ty.data(), r2n.data(),
                                                        tw.data(), nullptr);
  });
}

template <int SP>
static void run_all(int M, int tj, std::vector<cx<R>>& X, std::vector<cx<R>>& V, std::vector<TO>& tx,
                    std::vector<TO>& ty, std::vector<cx<R>>& r2n, std::vector<cx<R>>& tw) {
  if constexpr (SP == 2) {
    emu::launch(dim3(M), dim3(N / E), [&] {
      k_colfs_xy<R, TO, N, MODE, E, SLOTS>(X.data(), V.data(), M, tj, tx.data(), ty.data(), r2n.data(), tw.data(),
                                           nullptr);
    });
  } else if constexpr (SP) {
    run_one<1>(M, tj, X, V, tx, ty, r2n, tw);
    run_one<2>(M, tj, X, V, tx, ty, r2n, tw);
  } else {
    run_one<0>(M, tj, X, V, tx, ty, r2n, tw);
  }
}

template <int K>
static void run_kernel(FILE* f, FILE* o, int M, int tj, std::vector<cx<R>>& tw, std::vector<double>& re,
                       std::vector<double>& im) {
  if constexpr (K == 0 || K == 3) {
    std::vector<cx<R>> X, r2n;
    std::vector<TO> tx, ty;
    rd(f, X, (size_t)M * N);
    rd(f, tx, (size_t)(M + 1) * (N + 1));
    rd(f, ty, (size_t)(M + 1) * (N + 1));
    rd(f, r2n, (size_t)2 * N);
    std::vector<cx<R>> V((size_t)2 * M * N, cx<R>{(R)0, (R)0});
    if constexpr (K == 3) {
      static_assert(K == 3 && (N == 1536 || N == 768) && E == N / 192, "k_colfs3: columns of 1536 or 768");
      emu::launch(dim3(M), dim3(kC3T), [&] {
        k_colfs3<R, TO, MODE, N / 3>(X.data(), V.data(), M, tj, tx.data(), ty.data(), r2n.data(), tw.data(), nullptr);
      });
    } else {
      run_all<SPLIT>(M, tj, X, V, tx, ty, r2n, tw);
    }
    fwrite(V.data(), sizeof(cx<R>), V.size(), o);
  } else if constexpr (K == 1) {
    std::vector<cx<R>> Xx, Xy, r2n;
    std::vector<TO> tx, ty;
    rd(f, Xx, (size_t)M * N);
    rd(f, Xy, (size_t)M * N);
    rd(f, tx, (size_t)(M + 1) * (N + 1));
    rd(f, ty, (size_t)(M + 1) * (N + 1));
    rd(f, r2n, (size_t)2 * N);
    std::vector<cx<R>> Y((size_t)M * N, cx<R>{(R)0, (R)0});
    emu::launch(dim3(M), dim3(N / E), [&] {
      k_colfs_adj<R, TO, N, MODE, E, SLOTS>(Xx.data(), Xy.data(), Y.data(), M, tj, tx.data(), ty.data(), r2n.data(),
                                            tw.data(), nullptr);
    });
    fwrite(Y.data(), sizeof(cx<R>), Y.size(), o);
  } else {
    // spectrum columns: S (M columns of 2N), FP64; tables as TO (the length
    // depends on K, so that other kernels' builds do not instantiate it)
    constexpr int NS = K == 2 ? N : 2048;
    using S = fs_shape<NS, E>;
    std::vector<cx<double>> Sg, r2n;
    rd(f, Sg, (size_t)M * 2 * N);
    rd(f, r2n, (size_t)2 * N);
    std::vector<cx<double>> twd(S::TW_SIZE);
    for (int i = 0; i < S::TW_SIZE; ++i) twd[i] = cx<double>{re[i], im[i]};
    const int fp32 = std::is_same<TO, double>::value ? 0 : (std::is_same<TO, float>::value ? 2 : 1);
    std::vector<TO> tab((size_t)(M + 1) * (N + 1));
    const int kind = (MODE == 1 || MODE == 3) ? 1 : 0;
    emu::launch(dim3(M), dim3(NS / E), [&] {
      k_specfs<NS, E>(Sg.data(), M, tab.data(), kind, fp32, 0.25, r2n.data(), twd.data());
    });
    fwrite(tab.data(), sizeof(TO), tab.size(), o);
  }
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: %s M in.bin out.bin\n", argv[0]);
    return 2;
  }
  const int M = atoi(argv[1]);
  FILE* f = fopen(argv[2], "rb");
  if (!f) return 2;
  // the four-step twiddle table from long double roots, rounded once (for
  // k_colfs3: that of the 512-point sub-transforms, which 768 ignores)
  constexpr int TN = EMU_KERNEL == 3 ? 512 : N, TE = EMU_KERNEL == 3 ? 8 : E;
  using S = fs_shape<TN, TE>;
  std::vector<double> re(S::TW_SIZE), im(S::TW_SIZE);
  fs_fill_twiddles<TN, TE>(
      [](int m, int L, double* cr, double* ci) {
        const long double a = 6.283185307179586476925286766559005768L * m / L;
        *cr = (double)cosl(a);
        *ci = (double)-sinl(a);
      },
      re.data(), im.data());
  std::vector<cx<R>> tw(S::TW_SIZE);
  for (int i = 0; i < S::TW_SIZE; ++i) tw[i] = cx<R>{(R)re[i], (R)im[i]};
  const int tj = pow2_div(N, sizeof(R) == 4 ? 8 : 2);
  FILE* o = fopen(argv[3], "wb");
  fwrite(&tj, sizeof(int), 1, o);
  run_kernel<EMU_KERNEL>(f, o, M, tj, tw, re, im);
  fclose(f);
  fclose(o);
  return 0;
}
