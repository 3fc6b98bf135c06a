// td_util_gemm_noalloc: the product building block of td_util_gemm for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc). Operands are device pointers on
// the caller's stream; the padded staging copies, the bf16 slices and their
// exponents live in one fixed device array, `scratch`, of
// TD_GEMM_NOALLOC_SCRATCH_BYTES. Nothing is allocated on the device or on
// the host, nothing is synchronised, and errors are written into the
// caller's buffer.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>

#include "../../include/tddftb.h"
#include "common.hpp"
#include "split.hpp"

namespace {

constexpr size_t kScratchBytes = TD_GEMM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Each GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: only
// the address from hipGetSymbolAddress (per device) is handed to the device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per
// device with that device current.
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(g_lock);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// dst[rows_p x cols_p] (ld ldd) = src[rows x cols] (ld lds) with zeros
// beyond: every element of dst is written (no separate clearing pass).
__global__ void k_stage_pad(const double* __restrict__ src, int lds, int rows, int cols,
                            double* __restrict__ dst, int ldd, int rows_p, int cols_p) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)rows_p * cols_p) return;
  const int r = (int)(idx / cols_p), c = (int)(idx % cols_p);
  dst[(size_t)r * ldd + c] = (r < rows && c < cols) ? src[(size_t)r * lds + c] : 0.0;
}

// dst[cols_p x rows_p] (ld ldd) = the transpose of src[rows x cols] with
// zeros beyond, through 32 x 32 tiles in LDS (coalesced both ways).
__global__ __launch_bounds__(256) void k_stage_pad_t(const double* __restrict__ src, int lds,
                                                     int rows, int cols,
                                                     double* __restrict__ dst, int ldd,
                                                     int rows_p, int cols_p) {
  __shared__ double tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < rows && c < cols) ? src[(size_t)r * lds + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;                        // dst row c, column r
    if (c < cols_p && r < rows_p) dst[(size_t)c * ldd + r] = tile[tx][k];
  }
}

struct Err {
  char* buf;
  int32_t len;
  td_status fail(td_status st, const char* fmt, ...) {
    if (buf && len > 0) {
      va_list ap;
      va_start(ap, fmt);
      std::vsnprintf(buf, (size_t)len, fmt, ap);
      va_end(ap);
    }
    return st;
  }
  td_status hip(hipError_t e, const char* what) {
    return fail(TD_EHIP, "%s: %s", what, hipGetErrorString(e));
  }
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

td_status td_util_gemm_noalloc(int32_t precision, int32_t n_slices, int32_t m, int32_t n,
                               int32_t k, const double* A, int32_t lda, const double* B,
                               int32_t ldb, double* C, int32_t ldc, void* hip_stream, char* err,
                               int32_t errlen) {
  Err er{err, errlen};
  if (err && errlen > 0) err[0] = '\0';
  if (!A || !B || !C || m <= 0 || n <= 0 || k <= 0 || lda < k || ldb < n || ldc < n)
    return er.fail(TD_EINVAL, "invalid gemm arguments (null pointer, size or leading dimension)");
  if (precision != TD_FP64 && precision != TD_SPLIT_BF16)
    return er.fail(TD_EINVAL, "unknown precision");
  const bool split = precision == TD_SPLIT_BF16;
  if (split && (n_slices < 3 || n_slices > 5))
    return er.fail(TD_EINVAL, "n_slices must be 3, 4 or 5");
  // padding as td_util_gemm: rows, columns and K to the 128-wide tile
  const int mp = td::round_up(m, td::kGemmTile), npd = td::round_up(n, td::kGemmTile);
  const int kp = td::round_up(k, td::kGemmTile);
  const size_t sA = align256(sizeof(double) * mp * (size_t)kp);
  const size_t sB = align256(sizeof(double) * npd * (size_t)kp);
  const size_t sC = align256(sizeof(double) * mp * (size_t)npd);
  size_t need = sA + sB + sC;
  size_t sL = 0, sR = 0, sE = 0, sF = 0;
  if (split) {
    sL = align256(sizeof(__bf16) * (size_t)n_slices * mp * kp);
    sR = align256(sizeof(__bf16) * (size_t)n_slices * npd * kp);
    sE = align256(sizeof(int) * (size_t)mp);
    sF = align256(sizeof(int) * (size_t)npd);
    need += sL + sR + sE + sF;
  }
  if (need > kScratchBytes)
    return er.fail(TD_EINVAL,
                   "product %d x %d x %d needs %zu bytes of scratch; the fixed array holds %zu",
                   m, n, k, need, kScratchBytes);
  hipStream_t st = (hipStream_t)hip_stream;
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return er.hip(e, "scratch address (hipGetSymbolAddress)");
  unsigned char* p = (unsigned char*)base;
  double* Ap = (double*)p;
  double* Bp = (double*)(p + sA);
  double* Cp = (double*)(p + sA + sB);
  if (!split) {
    hipLaunchKernelGGL(k_stage_pad, dim3((unsigned)(((size_t)mp * kp + 255) / 256)), dim3(256), 0,
                       st, A, lda, m, k, Ap, kp, mp, kp);
    hipLaunchKernelGGL(k_stage_pad, dim3((unsigned)(((size_t)kp * npd + 255) / 256)), dim3(256),
                       0, st, B, ldb, k, n, Bp, npd, kp, npd);
    if ((e = hipGetLastError()) != hipSuccess) return er.hip(e, "staging kernels");
    e = td::dgemm(st, 0, mp, npd, kp, 1.0, Ap, kp, Bp, npd, 0.0, nullptr, 0, Cp, npd);
    if (e != hipSuccess) return er.hip(e, "dgemm");
  } else {
    __bf16* Ls = (__bf16*)(p + sA + sB + sC);
    __bf16* Rs = (__bf16*)(p + sA + sB + sC + sL);
    int* eL = (int*)(p + sA + sB + sC + sL + sR);
    int* fR = (int*)(p + sA + sB + sC + sL + sR + sE);
    // A padded (rows sliced), B transposed and padded (its columns sliced as rows)
    hipLaunchKernelGGL(k_stage_pad, dim3((unsigned)(((size_t)mp * kp + 255) / 256)), dim3(256), 0,
                       st, A, lda, m, k, Ap, kp, mp, kp);
    hipLaunchKernelGGL(k_stage_pad_t, dim3(npd / 32, kp / 32), dim3(256), 0, st, B, ldb, k, n, Bp,
                       kp, kp, npd);
    if ((e = hipGetLastError()) != hipSuccess) return er.hip(e, "staging kernels");
    td::SliceSrc sa;
    sa.M0 = Ap;
    sa.ld0 = kp;
    e = td::slice_rows(st, n_slices, td::SLICE_PLAIN, sa, mp, kp, Ls, kp * n_slices, eL);
    if (e != hipSuccess) return er.hip(e, "slicing A");
    td::SliceSrc sb;
    sb.M0 = Bp;
    sb.ld0 = kp;
    e = td::slice_rows(st, n_slices, td::SLICE_PLAIN, sb, npd, kp, Rs, kp * n_slices, fR);
    if (e != hipSuccess) return er.hip(e, "slicing B");
    td::SplitGemm g;
    g.m = mp;
    g.n = npd;
    g.L = Ls;
    g.ldl = kp * n_slices;
    g.eL = eL;
    g.eL_stride = 0;
    g.R = Rs;
    g.ldr = kp * n_slices;
    g.fR = fR;
    g.fR_stride = 0;
    g.seg_len = kp;
    g.k_lo = kp;
    g.k_hi = kp;
    g.n_split = npd;
    g.C = Cp;
    g.ldc = npd;
    e = td::split_gemm(st, n_slices, g);
    if (e != hipSuccess) return er.hip(e, "split product");
  }
  e = hipMemcpy2DAsync(C, sizeof(double) * ldc, Cp, sizeof(double) * npd, sizeof(double) * n, m,
                       hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return er.hip(e, "copy of C");
  return TD_OK;
}

}  // extern "C"
