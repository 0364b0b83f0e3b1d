// Launch entry points shared by the host library and the kernel file.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// precision code: 0 = FP64, 1 = FP32 (complex arrays are interleaved pairs)
hipError_t sg_set_gl_tables(const double* x /*4x16*/, const double* w /*4x16*/);
hipError_t sg_launch_weights(int k, double hx, double hy, int M, int N, double* wx, double* wy, int layout,
                             hipStream_t st);
hipError_t sg_launch_row_fwd(int prec, int M, const void* src, int64_t ld, void* X, int nrows, const void* r2m,
                             int solve, int full, hipStream_t st);
hipError_t sg_launch_col(int prec, int N, const void* X, void* V, int M, const void* tx, const void* ty, int kind,
                         const void* r2n, int solve, hipStream_t st);
hipError_t sg_launch_row_inv(int prec, int M, const void* V, void* fx, void* fy, int nrows, const void* r2m,
                             hipStream_t st);
hipError_t sg_launch_spec_col(int N, const void* S, int M, void* tab, int kind, int fp32, double scale,
                              const void* r2n, hipStream_t st);
hipError_t sg_launch_check_finite(int prec, const void* x, int64_t n, int* flag, hipStream_t st);
hipError_t sg_launch_coeff_rows(int prec, int M, const void* src, void* dst, int nrows, hipStream_t st);
hipError_t sg_launch_coeff_cols(int prec, int N, void* data, int M, hipStream_t st);
