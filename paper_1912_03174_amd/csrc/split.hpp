// Split-bf16 product and slicing launchers (see gemm_split_bf16.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace td {

enum { SLICE_PLAIN = 0, SLICE_SUM = 1, SLICE_DH = 2, SLICE_RENORM = 3, SLICE_SUM_AND_M1 = 4 };

// Source of the values sliced row by row:
//   SLICE_PLAIN: sign * M0[r][c]
//   SLICE_SUM:   M0[r][c] + M1[r][c]
//   SLICE_DH:    1/2 M0[r][c] (v[r] + v[c])   (M0 = S, v = potential change)
//   SLICE_RENORM: M0[r][c] - cs[0] M1[r][c], also written back to M0
//   SLICE_SUM_AND_M1: M0 + M1 into out / exps and, in the same pass, M1 into
//                     out2 / exps2 (one read of M1 for both); rows of at most
//                     4096 values
struct SliceSrc {
  const double* M0 = nullptr;
  int ld0 = 0;
  const double* M1 = nullptr;
  int ld1 = 0;
  const double* v = nullptr;
  double sign = 1.0;
  const double* cs = nullptr;
  double* M0w = nullptr;   // SLICE_RENORM: writable alias of M0
  __bf16* out2 = nullptr;  // SLICE_SUM_AND_M1: second output (same ldo)
  int* exps2 = nullptr;
};

// C[m x n] = sum over K segments of 2^(eL+fR-16) (sliced L)(sliced R)^T (+ Cin).
// Slices are k-blocked: element (slice s, row r, k) of an operand lives at
// r * ld + (k / 16) * 16 S + s * 16 + k % 16.
// L: [m][ldl] bf16, row exponents eL[seg][m] (stride eL_stride);
// R: [n][ldr] bf16 holding the right operand transposed, column exponents
// fR[seg][n]. Tiles whose first column is < n_split use K = k_hi, the
// others K = k_lo. m, n multiples of 128; seg_len a multiple of 128 and
// each K value seg_len or 2 seg_len; ldl, ldr multiples of 16 S.
struct SplitGemm {
  int m = 0, n = 0;
  const __bf16* L = nullptr;
  int ldl = 0;
  const int* eL = nullptr;
  int eL_stride = 0;
  const __bf16* R = nullptr;
  int ldr = 0;
  const int* fR = nullptr;
  int fR_stride = 0;
  int seg_len = 0;
  int k_lo = 0, k_hi = 0, n_split = 0;
  double* C = nullptr;
  int ldc = 0;
  const double* Cin = nullptr;
  int ldcin = 0;
};

hipError_t split_gemm(hipStream_t st, int n_slices, const SplitGemm& g);

// Slices rows [0, rows) x columns [0, cols) of the source into the k-blocked
// layout out[r * ldo + (c / 16) * 16 S + s * 16 + c % 16], exponents into
// exps[r]; cols multiple of 16.
hipError_t slice_rows(hipStream_t st, int n_slices, int mode, const SliceSrc& src, int rows,
                      int cols, __bf16* out, int ldo, int* exps);

}  // namespace td
