// FP64 matrix-core product C = alpha A B + beta Cin for the density-matrix
// step (the S^-1 H and (S^-1 H)[Re rho | Im rho] products of Sec. 2.3).
//
// gfx950 design:
//  * 128 x 128 macro tile per 256-thread workgroup, four 64-wide waves in
//    a 2 x 2 grid, each wave owning a 64 x 64 sub-tile = 4 x 4 blocks of
//    v_mfma_f64_16x16x4_f64 (16 double4 accumulators per lane).
//  * K advances 16 per stage. Tiles of A (stored k-major, so one MFMA
//    operand fetch is 16 consecutive doubles per k row) and B are staged
//    in LDS with double buffering: the next stage's global loads are in
//    flight in registers while the matrix cores work on the current one;
//    one barrier per stage. 66.5 KB of LDS per workgroup, two per CU.
//  * Workgroups are dispatched round-robin over the 8 XCDs; the block id
//    is remapped so each XCD owns a contiguous range of tiles, ordered in
//    groups of 8 tile rows, so concurrently running tiles on one XCD share
//    A and B panels in that XCD's L2.
#include <atomic>

#include "common.hpp"

namespace td {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;
constexpr int BN = 128;
constexpr int BK = 16;
constexpr int PAD = 2;
constexpr int LDA_S = BM + PAD;   // As[k][m]
constexpr int LDB_S = BN + PAD;   // Bs[k][n]
constexpr int GROUP_M = 8;

template <int TAG>
__global__ __launch_bounds__(256) void dgemm_nn(const double* __restrict__ A, int lda,
                                                const double* __restrict__ B, int ldb,
                                                double* C, int ldc, const double* Cin,
                                                int ldcin, int K, double alpha, double beta,
                                                int tiles_m, int tiles_n) {
  __shared__ double As[2][BK][LDA_S];
  __shared__ double Bs[2][BK][LDB_S];

  // XCD-aware tile order: blocks w with w % 8 == x run on XCD x.
  const int nt = tiles_m * tiles_n;
  const int w = blockIdx.x;
  const int q = nt >> 3, r = nt & 7;
  const int xcd = w & 7, slot = w >> 3;
  const int lin = xcd * q + (xcd < r ? xcd : r) + slot;
  const int group = GROUP_M * tiles_n;
  const int g = lin / group;
  const int first_m = g * GROUP_M;
  const int gsz = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
  const int in_g = lin - g * group;
  const int tm = first_m + in_g % gsz;
  const int tn = in_g / gsz;
  const int m0 = tm * BM, n0 = tn * BN;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;

  // Global -> register mapping: A rows (t>>1), 8 consecutive k at (t&1)*8;
  // B k row (t>>4), 8 consecutive n at (t&15)*8.
  const int a_row = t >> 1, a_k = (t & 1) * 8;
  const int b_k = t >> 4, b_n = (t & 15) * 8;
  const double* Ag = A + (size_t)(m0 + a_row) * lda + a_k;
  const double* Bg = B + (size_t)b_k * ldb + n0 + b_n;

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // Stage helpers as macros so the staging registers stay in VGPRs.
#define TD_LOAD_GLOBAL(kt)                                                     \
  do {                                                                         \
    const double* an_ = Ag + (size_t)(kt) * BK;                                \
    const double* bn_ = Bg + (size_t)(kt) * BK * ldb;                          \
    ra0 = *reinterpret_cast<const double2*>(an_ + 0);                          \
    ra1 = *reinterpret_cast<const double2*>(an_ + 2);                          \
    ra2 = *reinterpret_cast<const double2*>(an_ + 4);                          \
    ra3 = *reinterpret_cast<const double2*>(an_ + 6);                          \
    rb0 = *reinterpret_cast<const double2*>(bn_ + 0);                          \
    rb1 = *reinterpret_cast<const double2*>(bn_ + 2);                          \
    rb2 = *reinterpret_cast<const double2*>(bn_ + 4);                          \
    rb3 = *reinterpret_cast<const double2*>(bn_ + 6);                          \
  } while (0)
#define TD_STORE_LDS(buf)                                                      \
  do {                                                                         \
    As[buf][a_k + 0][a_row] = ra0.x;                                           \
    As[buf][a_k + 1][a_row] = ra0.y;                                           \
    As[buf][a_k + 2][a_row] = ra1.x;                                           \
    As[buf][a_k + 3][a_row] = ra1.y;                                           \
    As[buf][a_k + 4][a_row] = ra2.x;                                           \
    As[buf][a_k + 5][a_row] = ra2.y;                                           \
    As[buf][a_k + 6][a_row] = ra3.x;                                           \
    As[buf][a_k + 7][a_row] = ra3.y;                                           \
    *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 0]) = rb0;                 \
    *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 2]) = rb1;                 \
    *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 4]) = rb2;                 \
    *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 6]) = rb3;                 \
  } while (0)

  double2 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
  const int nk = K / BK;
  TD_LOAD_GLOBAL(0);
  TD_STORE_LDS(0);
  __syncthreads();
  // Steady state: the loads of stage kt+1 are in flight while stage kt computes.
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) TD_LOAD_GLOBAL(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kl = kk + lk;
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[cur][kl][wm * 64 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[cur][kl][wn * 64 + j * 16 + l16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) TD_STORE_LDS(cur ^ 1);
    __syncthreads();
  }
#undef TD_LOAD_GLOBAL
#undef TD_STORE_LDS

  // Accumulator layout of the 16x16 f64 block: register r of lane l holds
  // row l/16 + 4 r, column l%16.
  if (beta == 0.0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = n0 + wn * 64 + j * 16 + l16;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = m0 + wm * 64 + i * 16 + lk + 4 * rr;
          __builtin_nontemporal_store(alpha * acc[i][j][rr], &C[(size_t)row * ldc + col]);
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = n0 + wn * 64 + j * 16 + l16;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = m0 + wm * 64 + i * 16 + lk + 4 * rr;
          C[(size_t)row * ldc + col] =
              alpha * acc[i][j][rr] + beta * Cin[(size_t)row * ldcin + col];
        }
      }
  }
}

// Grouped form: the block id picks a problem (binary search over tile0)
// and a tile inside it. BT = 128: the same waves, LDS staging and MFMA
// sequence as dgemm_nn (256 threads); BT = 64: eight waves of 32 x 16
// (2 x 1 MFMA blocks each, 512 threads) for small matrices, where 128-wide
// tiles would mostly multiply padding. Each output element sees the same
// MFMA sequence over k in both.
template <int BT>
__device__ __forceinline__ void dgemm_tile_body(const GemmProblem* __restrict__ pp, int local);
__device__ __forceinline__ void dgemm_tile64(const GemmProblem* __restrict__ pp, int local);

template <int BT>
__global__ __launch_bounds__(BT == 64 ? 512 : 256)
__attribute__((amdgpu_waves_per_eu(BT == 64 ? 6 : 1)))
void dgemm_grouped_k(const GemmProblem* __restrict__ probs, int nprob, int ntiles) {
  // XCD-aware order over the launch's tiles (a problem's tiles stay together).
  const int w = blockIdx.x;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int xcd = w & 7, slot = w >> 3;
  const int lin = xcd * q + (xcd < r ? xcd : r) + slot;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile0 <= lin) lo = mid; else hi = mid - 1;
  }
  if constexpr (BT == 64)
    dgemm_tile64(probs + lo, lin - probs[lo].tile0);
  else
    dgemm_tile_body<BT>(probs + lo, lin - probs[lo].tile0);
}

// One problem passed by value (no device table): the 64-tile form for
// products whose 128 x 128 tiles would fill the chip's rounds badly.
template <int BT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6)))
void dgemm_single_k(GemmProblem pr) {
  static_assert(BT == 64, "single-problem launches use the 64-wide tile");
  const int ntiles = pr.upper ? pr.tiles_n * (pr.tiles_n + 1) / 2 : pr.tiles_m * pr.tiles_n;
  const int w = blockIdx.x;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int xcd = w & 7, slot = w >> 3;
  dgemm_tile64(&pr, xcd * q + (xcd < r ? xcd : r) + slot);
}

// 64 x 64 tile over eight waves in 2 x 4, each 32 rows x 16 columns (two
// 16 x 16 MFMA blocks sharing the B operand). Twice the waves of a 4-wave
// layout, for latency hiding at the 2-3 workgroups per CU that products of
// n ~ 1000-3000 give. K stages of 16 are loaded two stages ahead from two
// register sets (one stage is 8 MFMAs per wave, shorter than the load
// latency); prefetch indices are clamped to the last stage (a harmless
// reload) so the loop body is straight-line.
__device__ __forceinline__ void dgemm_tile64(const GemmProblem* __restrict__ pp, int local) {
  constexpr int T = 64;
  __shared__ double As[2][BK][T + PAD];
  __shared__ double Bs[2][BK][T + PAD];
  const int tiles_m = pp->tiles_m, tiles_n = pp->tiles_n;
  const int lda = pp->lda, ldb = pp->ldb, ldc = pp->ldc, Kp = pp->K;
  const double* __restrict__ Ap = pp->A;
  const double* __restrict__ Bp = pp->B;
  double* Cp = pp->C;
  int m0, n0;
  if (pp->upper) {
    // the tiles with tile row <= tile column, row by row
    int r = 0, rem = local;
    while (rem >= tiles_n - r) {
      rem -= tiles_n - r;
      ++r;
    }
    m0 = r * T;
    n0 = (r + rem) * T;
  } else {
    const int group = GROUP_M * tiles_n;
    const int g = local / group;
    const int first_m = g * GROUP_M;
    const int gsz = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
    const int in_g = local - g * group;
    m0 = (first_m + in_g % gsz) * T;
    n0 = (in_g / gsz) * T;
  }

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int l16 = lane & 15, lk = lane >> 4;
  const int a_row = t >> 3, a_k = (t & 7) * 2;      // A: 64 rows x 16 k, one double2 a thread
  const int b_k = t >> 5, b_n = (t & 31) * 2;       // B: 16 k x 64 columns, one double2 a thread
  const double* Ag = Ap + (size_t)(m0 + a_row) * lda + a_k;
  const double* Bg = Bp + (size_t)b_k * ldb + n0 + b_n;

  d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = d4{0.0, 0.0, 0.0, 0.0};
  double2 pa, pb, qa, qb;   // two staging sets (named, so they stay in VGPRs)
#define TD_W_LOAD(P, kt)                                                       \
  do {                                                                         \
    P##a = *reinterpret_cast<const double2*>(Ag + (size_t)(kt) * BK);          \
    P##b = *reinterpret_cast<const double2*>(Bg + (size_t)(kt) * BK * ldb);    \
  } while (0)
#define TD_W_STORE(P, buf)                                                     \
  do {                                                                         \
    As[buf][a_k][a_row] = P##a.x;                                              \
    As[buf][a_k + 1][a_row] = P##a.y;                                          \
    *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n]) = P##b;                    \
  } while (0)
#define TD_W_COMPUTE(cur)                                                      \
  do {                                                                         \
    _Pragma("unroll") for (int kk = 0; kk < BK; kk += 4) {                     \
      const int kl = kk + lk;                                                  \
      const double a0 = As[cur][kl][wm * 32 + l16];                            \
      const double a1 = As[cur][kl][wm * 32 + 16 + l16];                       \
      const double b0 = Bs[cur][kl][wn * 16 + l16];                            \
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);      \
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc1, 0, 0, 0);      \
    }                                                                          \
  } while (0)
  const int nk = Kp / BK, last = nk - 1;
  TD_W_LOAD(p, 0);
  TD_W_LOAD(q, 1 < last ? 1 : last);
  TD_W_STORE(p, 0);
  TD_W_LOAD(p, 2 < last ? 2 : last);
  __syncthreads();
  // Pairs of stages: LDS buffer 0 holds even stages, buffer 1 odd ones; set
  // q carries stage kt + 1, set p stage kt + 2 when a pair starts.
  for (int kt = 0; kt < nk; kt += 2) {
    TD_W_COMPUTE(0);
    TD_W_STORE(q, 1);
    __syncthreads();
    TD_W_LOAD(q, kt + 3 < last ? kt + 3 : last);
    if (kt + 1 >= nk) break;
    TD_W_COMPUTE(1);
    TD_W_STORE(p, 0);
    __syncthreads();
    TD_W_LOAD(p, kt + 4 < last ? kt + 4 : last);
  }
#undef TD_W_LOAD
#undef TD_W_STORE
#undef TD_W_COMPUTE
  // output layout of a 16 x 16 block: register rr of lane l holds row
  // l / 16 + 4 rr, column l % 16
  const int col = n0 + wn * 16 + l16;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int row = m0 + wm * 32 + lk + 4 * rr;
    Cp[(size_t)row * ldc + col] = acc0[rr];
    Cp[(size_t)(row + 16) * ldc + col] = acc1[rr];
  }
}

template <int BT>
__device__ __forceinline__ void dgemm_tile_body(const GemmProblem* __restrict__ pp, int local) {
  constexpr int FR = BT / 32;                 // 16 x 16 blocks per wave dimension
  static_assert(BT == 128, "the 64-wide tile has its own body (dgemm_tile64)");
  constexpr int EA = BT * BK / 256;           // A (and B) elements loaded per thread: 8
  constexpr int EB = EA;
  constexpr int LD = BT + PAD;
  __shared__ double As[2][BK][LD];
  __shared__ double Bs[2][BK][LD];
  const int tiles_m = pp->tiles_m, tiles_n = pp->tiles_n;
  const int lda = pp->lda, ldb = pp->ldb, ldc = pp->ldc, Kp = pp->K;
  const double* __restrict__ Ap = pp->A;
  const double* __restrict__ Bp = pp->B;
  double* Cp = pp->C;
  const int group = GROUP_M * tiles_n;
  const int g = local / group;
  const int first_m = g * GROUP_M;
  const int gsz = (tiles_m - first_m) < GROUP_M ? (tiles_m - first_m) : GROUP_M;
  const int in_g = local - g * group;
  const int m0 = (first_m + in_g % gsz) * BT, n0 = (in_g / gsz) * BT;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;

  constexpr int APR = BK / EA;                // threads per A row
  constexpr int BPR = BT / EB;                // threads per B k row
  const int a_row = t / APR, a_k = (t % APR) * EA;
  const int b_k = t / BPR, b_n = (t % BPR) * EB;
  const double* Ag = Ap + (size_t)(m0 + a_row) * lda + a_k;
  const double* Bg = Bp + (size_t)b_k * ldb + n0 + b_n;

  d4 acc[FR][FR];
#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < FR; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // staging registers (named, so they stay in VGPRs): the next stage's
  // global loads are in flight while the matrix cores work on this one
  double2 pa0, pa1, pa2, pa3, pb0, pb1, pb2, pb3;
#define TD_G_LOAD(P, kt)                                                       \
  do {                                                                         \
    const double* an_ = Ag + (size_t)(kt) * BK;                                \
    const double* bn_ = Bg + (size_t)(kt) * BK * ldb;                          \
    P##a0 = *reinterpret_cast<const double2*>(an_ + 0);                        \
    P##a1 = *reinterpret_cast<const double2*>(an_ + 2);                        \
    P##b0 = *reinterpret_cast<const double2*>(bn_ + 0);                        \
    P##b1 = *reinterpret_cast<const double2*>(bn_ + 2);                        \
    if constexpr (EA == 8) {                                                   \
      P##a2 = *reinterpret_cast<const double2*>(an_ + 4);                      \
      P##a3 = *reinterpret_cast<const double2*>(an_ + 6);                      \
      P##b2 = *reinterpret_cast<const double2*>(bn_ + 4);                      \
      P##b3 = *reinterpret_cast<const double2*>(bn_ + 6);                      \
    }                                                                          \
  } while (0)
#define TD_G_STORE(P, buf)                                                     \
  do {                                                                         \
    As[buf][a_k + 0][a_row] = P##a0.x;                                         \
    As[buf][a_k + 1][a_row] = P##a0.y;                                         \
    As[buf][a_k + 2][a_row] = P##a1.x;                                         \
    As[buf][a_k + 3][a_row] = P##a1.y;                                         \
    *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 0]) = P##b0;               \
    *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 2]) = P##b1;               \
    if constexpr (EA == 8) {                                                   \
      As[buf][a_k + 4][a_row] = P##a2.x;                                       \
      As[buf][a_k + 5][a_row] = P##a2.y;                                       \
      As[buf][a_k + 6][a_row] = P##a3.x;                                       \
      As[buf][a_k + 7][a_row] = P##a3.y;                                       \
      *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 4]) = P##b2;             \
      *reinterpret_cast<double2*>(&Bs[buf][b_k][b_n + 6]) = P##b3;             \
    }                                                                          \
  } while (0)
#define TD_G_COMPUTE(cur)                                                      \
  do {                                                                         \
    _Pragma("unroll") for (int kk = 0; kk < BK; kk += 4) {                     \
      const int kl = kk + lk;                                                  \
      double a[FR], b[FR];                                                     \
      _Pragma("unroll") for (int i = 0; i < FR; ++i)                           \
          a[i] = As[cur][kl][wm * (BT / 2) + i * 16 + l16];                    \
      _Pragma("unroll") for (int j = 0; j < FR; ++j)                           \
          b[j] = Bs[cur][kl][wn * (BT / 2) + j * 16 + l16];                    \
      _Pragma("unroll") for (int i = 0; i < FR; ++i)                           \
          _Pragma("unroll") for (int j = 0; j < FR; ++j) acc[i][j] =           \
              __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0); \
    }                                                                          \
  } while (0)

  const int nk = Kp / BK;
  TD_G_LOAD(p, 0);
  TD_G_STORE(p, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) TD_G_LOAD(p, kt + 1);
    TD_G_COMPUTE(cur);
    if (more) TD_G_STORE(p, cur ^ 1);
    __syncthreads();
  }
#undef TD_G_LOAD
#undef TD_G_STORE
#undef TD_G_COMPUTE

#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < FR; ++j) {
      const int col = n0 + wn * (BT / 2) + j * 16 + l16;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = m0 + wm * (BT / 2) + i * 16 + lk + 4 * rr;
        Cp[(size_t)row * ldc + col] = 1.0 * acc[i][j][rr];
      }
    }
}

}  // namespace

namespace {
// Lower 64-wide tiles of a symmetric C from their transposes: 32 x 32
// blocks (bi, bj) with bi > bj outside the diagonal 64-tiles, staged
// through LDS so both the reads and the writes are row-contiguous.
__global__ __launch_bounds__(256) void k_mirror_lower(double* C, int ldc) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi <= bj || (bi >> 1) == (bj >> 1)) return;
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
#pragma unroll
  for (int r = ty; r < 32; r += 8) t[r][tx] = C[(size_t)(bj * 32 + r) * ldc + bi * 32 + tx];
  __syncthreads();
#pragma unroll
  for (int r = ty; r < 32; r += 8) C[(size_t)(bi * 32 + r) * ldc + bj * 32 + tx] = t[tx][r];
}
}  // namespace

hipError_t dgemm_symmetric(hipStream_t s, int n, int k, const double* A, int lda,
                           const double* B, int ldb, double* C, int ldc) {
  if (n <= 0 || k <= 0 || n % 64 || k % BK) return hipErrorInvalidValue;
  if (lda % 2 || ldb % 2 || lda < k || ldb < n || ldc < n) return hipErrorInvalidValue;
  GemmProblem pr{};
  pr.A = A;
  pr.B = B;
  pr.C = C;
  pr.lda = lda;
  pr.ldb = ldb;
  pr.ldc = ldc;
  pr.K = k;
  pr.tiles_m = n / 64;
  pr.tiles_n = n / 64;
  pr.upper = 1;
  const int t = n / 64;
  hipLaunchKernelGGL(dgemm_single_k<64>, dim3(t * (t + 1) / 2), dim3(512), 0, s, pr);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mirror_lower, dim3(n / 32, n / 32), dim3(256), 0, s, C, ldc);
  return hipGetLastError();
}

hipError_t symmetric_mirror(hipStream_t s, double* C, int ldc, int n) {
  if (n <= 0 || n % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mirror_lower, dim3(n / 32, n / 32), dim3(256), 0, s, C, ldc);
  return hipGetLastError();
}

hipError_t dgemm_grouped(hipStream_t s, int tile, const GemmProblem* probs, int nprob,
                         int ntiles) {
  if (nprob <= 0 || ntiles <= 0 || !probs) return hipErrorInvalidValue;
  if (tile == 128)
    hipLaunchKernelGGL(dgemm_grouped_k<128>, dim3(ntiles), dim3(256), 0, s, probs, nprob, ntiles);
  else if (tile == 64)
    hipLaunchKernelGGL(dgemm_grouped_k<64>, dim3(ntiles), dim3(512), 0, s, probs, nprob, ntiles);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

namespace {
// Compute units of the current device (queried once per device; racing
// first queries store the same value).
int cu_count() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int cu = cache[dev].load(std::memory_order_relaxed);
  if (cu == 0) {
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0)
      cu = 256;
    cache[dev].store(cu, std::memory_order_relaxed);
  }
  return cu;
}
}  // namespace

hipError_t dgemm(hipStream_t s, int tag, int m, int n, int k, double alpha, const double* A,
                 int lda, const double* B, int ldb, double beta, const double* Cin, int ldcin,
                 double* C, int ldc) {
  if (m % BM || n % BN || k % BK || m <= 0 || n <= 0 || k <= 0) return hipErrorInvalidValue;
  if (lda % 2 || ldb % 2 || lda < k || ldb < n || ldc < n) return hipErrorInvalidValue;
  if (beta != 0.0 && (Cin == nullptr || ldcin < n)) return hipErrorInvalidValue;
  const int tm = m / BM, tn = n / BN;
  // 128-wide tiles run two per CU; they pay only when their last round of
  // 2 x (CU count) workgroups is nearly full (at n = 2944, 529 tiles make a
  // second round with 17 tiles in it and the product takes 17% longer than
  // with 64-wide tiles, which fill the CUs more evenly). Otherwise 64-wide
  // tiles: the same sums in the same order, so the result is bit for bit
  // the same.
  const int slots = 2 * cu_count();
  const int t128 = tm * tn;
  const int rounds = (t128 + slots - 1) / slots;
  const bool full_rounds = 10 * (long long)t128 >= 9LL * rounds * slots;
  if (!full_rounds && alpha == 1.0 && beta == 0.0) {
    GemmProblem pr{};
    pr.A = A;
    pr.B = B;
    pr.C = C;
    pr.lda = lda;
    pr.ldb = ldb;
    pr.ldc = ldc;
    pr.K = k;
    pr.tiles_m = m / 64;
    pr.tiles_n = n / 64;
    hipLaunchKernelGGL(dgemm_single_k<64>, dim3(pr.tiles_m * pr.tiles_n), dim3(512), 0, s, pr);
    return hipGetLastError();
  }
  const dim3 grid(tm * tn), block(256);
  switch (tag) {
    case 1:
      hipLaunchKernelGGL(dgemm_nn<1>, grid, block, 0, s, A, lda, B, ldb, C, ldc, Cin, ldcin, k,
                         alpha, beta, tm, tn);
      break;
    case 2:
      hipLaunchKernelGGL(dgemm_nn<2>, grid, block, 0, s, A, lda, B, ldb, C, ldc, Cin, ldcin, k,
                         alpha, beta, tm, tn);
      break;
    default:
      hipLaunchKernelGGL(dgemm_nn<0>, grid, block, 0, s, A, lda, B, ldb, C, ldc, Cin, ldcin, k,
                         alpha, beta, tm, tn);
      break;
  }
  return hipGetLastError();
}

}  // namespace td
