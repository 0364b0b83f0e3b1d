// Launch entry points shared by the host library and the kernel file.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// One grid of a batched launch (device memory, read by the per-step
// kernels): element offset of the grid in the packed sigma / force buffers,
// its workspace and its spectrum tables.
struct sg_bgrid {
  int64_t off;
  void* X;
  void* V;
  const void* tabx;
  const void* taby;
};

// precision code: 0 = FP64, 1 = FP32 (complex arrays are interleaved pairs)
// Per-step launches take an optional batch: bg = NULL runs one grid from the
// pointer arguments; otherwise ngrids grids of the same sizes and order from
// bg (blockIdx.y = grid), with the buffer arguments as bases of the packed
// buffers.  tile: rows (passes A, C) or columns (pass B) per workgroup,
// 0 = the compiled maximum.
hipError_t sg_set_gl_tables(const double* x /*4x16*/, const double* w /*4x16*/);
hipError_t sg_launch_weights(int k, double hx, double hy, int M, int N, double* wx, double* wy, int layout,
                             hipStream_t st);
// tw: stage twiddle tables of the pass (sg_twiddles).  solve: 0 for k = 1, 2,
// else the order k (3, 4, 5) of the interpolation system solved on the way
hipError_t sg_launch_row_fwd(int prec, int M, const void* src, int64_t ld, void* X, int nrows, const void* r2m,
                             int solve, int full, const void* tw, const sg_bgrid* bg, int ngrids, int tile,
                             hipStream_t st);
// Launch variants of a pass (0 = A, 1 = B, 2 = C) for a transform length
// (kernels of the same result with other buffering or elements per
// thread): their number (0 for an unsupported length) and the default.
int sg_variants(int prec, int pass, int len);
int sg_default_variant(int prec, int pass, int len);
// largest tile (rows or columns per workgroup) of a pass in a variant
int sg_max_tile(int prec, int pass, int len, int variant);
// X: column-major row spectra (bin p of row j at X[p*N + j]); V: tiles of
// tj rows (sg_row_tile), the layout the inverse row pass reads.  kind: 0 for
// odd k (tables of A, W = i A), 1 for even k (W = ph i A, ph the bin's
// half-cell phase); tx, ty are the quarter tables of A in either case.
hipError_t sg_launch_col(int prec, int N, const void* X, void* V, int M, int tj, const void* tx, const void* ty,
                         int kind, const void* r2n, int solve, const void* tw, const sg_bgrid* bg, int ngrids,
                         int tile, int variant, hipStream_t st);
int sg_row_tile(int prec, int M, int N);
hipError_t sg_launch_row_inv(int prec, int M, const void* V, void* fx, void* fy, int nrows, int tj, const void* r2m,
                             const void* tw, const sg_bgrid* bg, int ngrids, int tile, int variant, hipStream_t st);
hipError_t sg_launch_spec_col(int N, const void* S, int M, void* tab, int kind, int fp32, double scale,
                              const void* r2n, const void* tw, hipStream_t st);
// Stage twiddle tables of a pass's FFT (pass 0: forward rows, 1: columns,
// 2: inverse rows, 3: spectrum columns, FP64 only, 4: inverse rows in
// launch variant 1, FP32 only); len = M or N; roots =
// the 2*len-th roots in the pass precision.  Returns the entry count (out ==
// NULL) or fills out on st; -1 for an unsupported size.
int sg_twiddles(int prec, int pass, int len, const void* roots, void* out, hipStream_t st);
hipError_t sg_launch_check_finite(int prec, const void* x, int64_t n, int* flag, hipStream_t st);
hipError_t sg_launch_coeff_rows(int prec, int M, const void* src, void* dst, int nrows, int k, hipStream_t st);
hipError_t sg_launch_coeff_cols(int prec, int N, void* data, int M, int k, hipStream_t st);
// Adjoint after the two forward row transforms of gx, gy (Xx, Xy
// column-major like X): conjugate-spectrum column pass into Y (tiles of tj
// rows), then the inverse real row pass with the x-solve into gsigma.
// Batched (bg != NULL): Xx, Xy, Y and gsigma come from the descriptors (X,
// the two halves of V, the offset into the packed gsigma base).
hipError_t sg_launch_adjoint_tail(int prec, int M, int N, const void* Xx, const void* Xy, void* Y, void* gsigma,
                                  int tj, const void* tx, const void* ty, int kind, const void* r2m, const void* r2n,
                                  int solve, const void* twB, const void* twA, const sg_bgrid* bg, int ngrids,
                                  hipStream_t st);
// Four-step column pass for long columns (sg_colfs.hip): supported
// (precision, N); its twiddle table (entry count, and filled from long double
// when re and im are given); the launch (the arguments of sg_launch_col, plus
// tab_bytes: 8 for double or float hi+lo tables, 4 for float tables).
int sg_colfs_supported(int prec, int N);
int sg_colfs_twiddles(int prec, int N, double* re, double* im);
hipError_t sg_launch_colfs(int prec, int N, const void* X, void* V, int M, int tj, const void* tx, const void* ty,
                           int kind, int tab_bytes, const void* r2n, int solve, const void* tw, const sg_bgrid* bg,
                           int ngrids, hipStream_t st);
// Adjoint column pass of the long columns (the arguments of the column
// pass of sg_launch_adjoint_tail, plus tab_bytes).
hipError_t sg_launch_colfs_adj(int prec, int N, const void* Xx, const void* Xy, void* Y, int M, int tj, const void* tx,
                               const void* ty, int kind, int tab_bytes, const void* r2n, int solve, const void* tw,
                               const sg_bgrid* bg, int ngrids, hipStream_t st);
// Plan-time spectrum columns of length 8192 (FP64; tw: the FP64 four-step
// twiddle table of that length; fp32: 0 double, 1 float hi + lo, 2 float).
hipError_t sg_launch_specfs(int N, const void* rowspec, int M, void* tab, int kind, int fp32, double scale,
                            const void* r2n, const void* tw, hipStream_t st);
// The inverse real row pass of the adjoint alone (after a column pass that
// wrote the packed gC spectra Y; batched: Y from the descriptors).
hipError_t sg_launch_row_c2r(int prec, int M, int N, const void* Y, void* gsigma, int tj, const void* r2m, int solve,
                             const void* twA, const sg_bgrid* bg, int ngrids, hipStream_t st);
