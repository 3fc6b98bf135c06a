// Split-BF16 matrix-core product (error-free splitting in the manner of
// Ozaki, Ogita, Oishi and Rump, Numer. Algorithms 59 (2012)) for the
// density-matrix step's two products (Sec. 2.3) at close to FP64 accuracy.
//
// Operands are cut into S bf16 slices with one power-of-two exponent per
// row (left operand) or per column (right operand, stored transposed so k
// is contiguous). Slices are stored k-blocked: row r holds, for each block
// of 16 values of k, the S slices of that block one after another (32 S
// bytes), so one K step of the product reads whole cache lines per row.
// Row i of M is scaled by 2^-e_i (|M_ik| < 2^e_i) and
// written as an integer series
//     M_ik 2^-e_i 2^8 = sigma_1 + sigma_2 2^-8 + ... + sigma_S 2^-8(S-1) + rest,
// each sigma_t an integer with |sigma_t| <= 256, rounded to nearest, and
// stored as w_t = sigma_t 2^-8(t-1), exact in bf16 (8 significant bits).
// A product of two slices is exact in fp32 (16 bits); so is the sum over
// 256 values of k of the leading pair (1,1), accumulated on its own, and of
// the two pairs (1,2), (2,1). Pairs with t_a + t_b <= S + 1 are kept.
// At every multiple of 256 in k and at the end of each K segment (so a
// chunk is at most 256 long and never spans two segments) the fp32
// accumulators are added into an fp64 accumulator with the row and column
// exponents of the segment: one product may concatenate segments with
// different operand scales along K (used for (S^-1 H) rho_delta +
// (S^-1 dH) rho_ref).
#include <cmath>

#include "common.hpp"
#include "split.hpp"

namespace td {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int CHUNK = 256;       // exact fp32 accumulation length of the leading pairs
constexpr int KUNIT = 128;       // K, segment lengths: multiples of the tile width
constexpr int GROUP_M = 8;

template <int S>
struct SplitArgs {
  const __bf16* L;      // [M][ldl], k-blocked slices
  int ldl;
  const int* eL;        // [nseg][M]
  int eL_stride;
  const __bf16* R;      // [Ncols][ldr] (transposed right operand), k-blocked slices
  int ldr;
  const int* fR;        // [nseg][Ncols]
  int fR_stride;
  int seg_len;          // K length of one segment (multiple of KUNIT)
  int k_lo, k_hi;       // K extent for tiles with n0 >= n_split / n0 < n_split
  int n_split;
  double* C;
  int ldc;
  const double* Cin;    // optional addend (same layout as C), may be null
  int ldcin;
  int tiles_m, tiles_n;
};

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding:
// vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[15:14]).
#define TD_WAIT_VMCNT(n) __builtin_amdgcn_s_waitcnt(((n) & 15) | (7 << 4) | (15 << 8) | (((n) >> 4) << 14))

// LDS stage layout: [mat][row][2S slots of 8 bf16] -- one K step of the
// k-blocked global layout, so each direct-to-LDS instruction moves whole
// 128-byte lines (S = 4) -- with the slots of row r rotated by
// f(r) = 2 r + r/4. A 128-bit fragment read is served for lanes i..i+3
// together with lanes 32+i..32+i+3 (rows r..r+3, both k halves): with this
// rotation those eight 16-byte reads hit eight different bank groups, as
// do eight or sixteen consecutive lanes.
__device__ __forceinline__ int rot(int row) { return 2 * row + (row >> 2); }

typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lds_u32(const __bf16* p) {
  return (uint32_t)(uintptr_t)(lds_void*)p;
}

// All 3 S operand fragments of one K step from LDS in one block that also
// waits for them (lgkmcnt(0) inside the block, so no read is in flight when
// the compiler takes the registers). Reading LDS through the compiler
// would make it wait for every direct-to-LDS load in flight (vmcnt(0)) at
// the top of the unrolled K loop, where it cannot tell the stages apart;
// the stage being read is guarded by the explicit waits and the barrier.
template <int S>
struct Frags {
  i32x4 a[S], b0[S], b1[S];
};

template <int S>
__device__ __forceinline__ void read_frags(Frags<S>& f, uint32_t base, const uint32_t* ao,
                                           const uint32_t* bo0, const uint32_t* bo1) {
  if constexpr (S == 3) {
    asm volatile("ds_read_b128 %0, %9\n"
                 "ds_read_b128 %1, %10\n"
                 "ds_read_b128 %2, %11\n"
                 "ds_read_b128 %3, %12\n"
                 "ds_read_b128 %4, %13\n"
                 "ds_read_b128 %5, %14\n"
                 "ds_read_b128 %6, %15\n"
                 "ds_read_b128 %7, %16\n"
                 "ds_read_b128 %8, %17\n"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(f.a[0]), "=&v"(f.a[1]), "=&v"(f.a[2]), "=&v"(f.b0[0]), "=&v"(f.b0[1]), "=&v"(f.b0[2]), "=&v"(f.b1[0]), "=&v"(f.b1[1]), "=&v"(f.b1[2])
                 : "v"(base + ao[0]), "v"(base + ao[1]), "v"(base + ao[2]), "v"(base + bo0[0]), "v"(base + bo0[1]), "v"(base + bo0[2]), "v"(base + bo1[0]), "v"(base + bo1[1]), "v"(base + bo1[2])
                 : "memory");
  } else if constexpr (S == 4) {
    asm volatile("ds_read_b128 %0, %12\n"
                 "ds_read_b128 %1, %13\n"
                 "ds_read_b128 %2, %14\n"
                 "ds_read_b128 %3, %15\n"
                 "ds_read_b128 %4, %16\n"
                 "ds_read_b128 %5, %17\n"
                 "ds_read_b128 %6, %18\n"
                 "ds_read_b128 %7, %19\n"
                 "ds_read_b128 %8, %20\n"
                 "ds_read_b128 %9, %21\n"
                 "ds_read_b128 %10, %22\n"
                 "ds_read_b128 %11, %23\n"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(f.a[0]), "=&v"(f.a[1]), "=&v"(f.a[2]), "=&v"(f.a[3]), "=&v"(f.b0[0]), "=&v"(f.b0[1]), "=&v"(f.b0[2]), "=&v"(f.b0[3]), "=&v"(f.b1[0]), "=&v"(f.b1[1]), "=&v"(f.b1[2]), "=&v"(f.b1[3])
                 : "v"(base + ao[0]), "v"(base + ao[1]), "v"(base + ao[2]), "v"(base + ao[3]), "v"(base + bo0[0]), "v"(base + bo0[1]), "v"(base + bo0[2]), "v"(base + bo0[3]), "v"(base + bo1[0]), "v"(base + bo1[1]), "v"(base + bo1[2]), "v"(base + bo1[3])
                 : "memory");
  } else {
    static_assert(S == 5, "3, 4 or 5 slices");
    asm volatile("ds_read_b128 %0, %15\n"
                 "ds_read_b128 %1, %16\n"
                 "ds_read_b128 %2, %17\n"
                 "ds_read_b128 %3, %18\n"
                 "ds_read_b128 %4, %19\n"
                 "ds_read_b128 %5, %20\n"
                 "ds_read_b128 %6, %21\n"
                 "ds_read_b128 %7, %22\n"
                 "ds_read_b128 %8, %23\n"
                 "ds_read_b128 %9, %24\n"
                 "ds_read_b128 %10, %25\n"
                 "ds_read_b128 %11, %26\n"
                 "ds_read_b128 %12, %27\n"
                 "ds_read_b128 %13, %28\n"
                 "ds_read_b128 %14, %29\n"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(f.a[0]), "=&v"(f.a[1]), "=&v"(f.a[2]), "=&v"(f.a[3]), "=&v"(f.a[4]), "=&v"(f.b0[0]), "=&v"(f.b0[1]), "=&v"(f.b0[2]), "=&v"(f.b0[3]), "=&v"(f.b0[4]), "=&v"(f.b1[0]), "=&v"(f.b1[1]), "=&v"(f.b1[2]), "=&v"(f.b1[3]), "=&v"(f.b1[4])
                 : "v"(base + ao[0]), "v"(base + ao[1]), "v"(base + ao[2]), "v"(base + ao[3]), "v"(base + ao[4]), "v"(base + bo0[0]), "v"(base + bo0[1]), "v"(base + bo0[2]), "v"(base + bo0[3]), "v"(base + bo0[4]), "v"(base + bo1[0]), "v"(base + bo1[1]), "v"(base + bo1[2]), "v"(base + bo1[3]), "v"(base + bo1[4])
                 : "memory");
  }
}

// SEG256: the segment length is a multiple of CHUNK, so chunks end only at
// multiples of CHUNK and the segment of a chunk follows from its start (the
// N_orb = 4096 case); otherwise a chunk also ends at the segment boundary.
template <int S, bool SEG256>
__global__ __launch_bounds__(512) void sgemm_split(SplitArgs<S> p) {
  // LDS ring of STAGES separate arrays (so the compiler can see that the
  // direct-to-LDS loads into one stage do not alias the fragment reads of
  // another, and does not wait for them); loads run STAGES-1 stages ahead.
  constexpr int STAGES = S <= 4 ? 4 : 2;
  constexpr int SLOTS = 2 * S;                             // 16-byte slots per row per K step
  constexpr int MAT_ELEMS = 128 * SLOTS * 8;               // one operand tile per stage
  constexpr int STAGE_ELEMS = 2 * MAT_ELEMS;
  __shared__ __attribute__((aligned(1024))) __bf16 st0[STAGE_ELEMS];
  __shared__ __attribute__((aligned(1024))) __bf16 st1[STAGE_ELEMS];
  __shared__ __attribute__((aligned(1024))) __bf16 st2[STAGES > 2 ? STAGE_ELEMS : 8];
  __shared__ __attribute__((aligned(1024))) __bf16 st3[STAGES > 2 ? STAGE_ELEMS : 8];
  __shared__ int sh_e[2][BM], sh_f[2][BN];                // segment exponents of the tile

  const int nt = p.tiles_m * p.tiles_n;
  const int w = blockIdx.x;
  const int xcd = w & 7, slot = w >> 3;                    // workgroups go to XCDs round-robin
  // Column tiles below n_split use K = k_hi, the others K = k_lo. When these
  // are two equal halves with a tile count per half divisible by 8, every
  // XCD takes the same share of each half, the long-K tiles first: its CUs
  // then finish together, with no long tile left over at the end.
  const int half = p.tiles_n / 2;
  const int per_half = p.tiles_m * half;
  const bool halves = p.k_lo != p.k_hi && 2 * p.n_split == p.tiles_n * BN && per_half % 8 == 0;
  int idx, cols, col0;
  if (halves) {
    const int share = per_half >> 3;
    const bool second = slot >= share;
    idx = xcd * share + (second ? slot - share : slot);
    cols = half;
    col0 = second ? half : 0;
  } else {
    const int q = nt >> 3, r = nt & 7;
    idx = xcd * q + (xcd < r ? xcd : r) + slot;          // contiguous range per XCD
    cols = p.tiles_n;
    col0 = 0;
  }
  // GROUP_M row tiles side by side share every column tile's K panel in L2
  const int group = GROUP_M * cols;
  const int g = idx / group;
  const int first_m = g * GROUP_M;
  const int gsz = (p.tiles_m - first_m) < GROUP_M ? (p.tiles_m - first_m) : GROUP_M;
  const int in_g = idx - g * group;
  const int m0 = (first_m + in_g % gsz) * BM;
  const int n0 = (col0 + in_g / gsz) * BN;
  const int K = (n0 < p.n_split) ? p.k_hi : p.k_lo;
  const int nk = K / BK;

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;      // 4 x 2 waves: 32 rows x 64 columns each
  const int l32 = lane & 31, lh = lane >> 5;

  // A stage is 8 S direct-to-LDS instructions of 64 x 16 B, S per wave.
  // Instruction gi: operand gi / (4S); its lane covers linear slot
  // qq = (gi % 4S) * 64 + lane = row * 2S + physical slot.
  constexpr int PER_WAVE = S;
  const __bf16* src_base[PER_WAVE];
  int lds_off[PER_WAVE];
#pragma unroll
  for (int c = 0; c < PER_WAVE; ++c) {
    const int gi = wave + 8 * c;
    const int mat = gi / (4 * S);
    const int li = gi % (4 * S);
    const int qq = li * 64 + lane;
    const int row = qq / SLOTS;
    const int ph = qq % SLOTS;
    const int lg = (ph + rot(row)) % SLOTS;               // logical slot fetched
    src_base[c] = mat ? (p.R + (size_t)(n0 + row) * p.ldr + lg * 8)
                      : (p.L + (size_t)(m0 + row) * p.ldl + lg * 8);
    lds_off[c] = mat * MAT_ELEMS + li * 512;
  }
#define TD_ISSUE_STAGE(BUF, kt)                                                            \
  do {                                                                                     \
    _Pragma("unroll") for (int c = 0; c < PER_WAVE; ++c) {                                 \
      __builtin_amdgcn_global_load_lds(                                                    \
          (const void*)(src_base[c] + (size_t)(kt) * (BK * S)),                            \
          (lds_void*)((BUF) + lds_off[c]), 16, 0, 0);                                      \
    }                                                                                      \
  } while (0)

  // acc2: pair (1,1), exact over a chunk; acc3: every other kept pair. Its
  // leading terms (1,2), (2,1) are 2^-8 of acc2 and exact on their own; the
  // smaller pairs added to them round at about 2^-32 of the leading term.
  f32x16 acc2[2], acc3[2];
  double acc64[2][16];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      acc2[j][e] = 0.0f;
      acc3[j][e] = 0.0f;
      acc64[j][e] = 0.0;
    }
  }
  // segment exponents of this tile's rows and columns, staged once in LDS
  const int nseg = (p.k_hi > p.seg_len) ? 2 : 1;
  for (int i = t; i < nseg * BM; i += 512) {
    const int sg = i / BM, rr = i % BM;
    sh_e[sg][rr] = p.eL[sg * p.eL_stride + m0 + rr];
    sh_f[sg][rr] = p.fR[sg * p.fR_stride + n0 + rr];
  }

  // Output layout of the 32x32 fp32 block: register e of lane l holds row
  // 8 (e/4) + 4 (l/32) + e%4, column l%32. `seg`: the K segment of the
  // chunk being flushed (a chunk never spans two segments).
#define TD_SPLIT_FLUSH(seg_of_chunk)                                                       \
  {                                                                                        \
    const int seg = (seg_of_chunk);                                                        \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) {                                        \
      const int fc = sh_f[seg][wn * 64 + j * 32 + l32] - 16;                               \
      _Pragma("unroll") for (int e = 0; e < 16; ++e) {                                     \
        const int sc = sh_e[seg][wm * 32 + 8 * (e >> 2) + 4 * lh + (e & 3)] + fc;          \
        acc64[j][e] += ldexp((double)acc2[j][e] + (double)acc3[j][e], sc);                 \
        acc2[j][e] = 0.0f;                                                                 \
        acc3[j][e] = 0.0f;                                                                 \
      }                                                                                    \
    }                                                                                      \
  }

  __syncthreads();     // exponents visible before any flush; no loads in flight yet
  // prologue: stages 0 .. STAGES-2 in flight
  TD_ISSUE_STAGE(st0, 0);
  if (STAGES > 2) {
    TD_ISSUE_STAGE(st1, 1);
    TD_ISSUE_STAGE(st2, 2);
  }

  // fragment offsets (elements) inside a stage: logical slot 2 s + lh of a row
  int a_off[S], b_off[2][S];
  uint32_t ao[S], bo0[S], bo1[S];   // the same offsets in bytes
  {
    const int arow = wm * 32 + l32;
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
      const int ph = ((2 * sl + lh - rot(arow)) % SLOTS + SLOTS) % SLOTS;
      a_off[sl] = arow * SLOTS * 8 + ph * 8;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int brow = wn * 64 + j * 32 + l32;
#pragma unroll
      for (int sl = 0; sl < S; ++sl) {
        const int ph = ((2 * sl + lh - rot(brow)) % SLOTS + SLOTS) % SLOTS;
        b_off[j][sl] = MAT_ELEMS + brow * SLOTS * 8 + ph * 8;
      }
    }
  }
#pragma unroll
  for (int sl = 0; sl < S; ++sl) {
    ao[sl] = 2u * a_off[sl];
    bo0[sl] = 2u * b_off[0][sl];
    bo1[sl] = 2u * b_off[1][sl];
  }
  // One K step on stage RD: wait for this wave's loads of it, barrier (all
  // waves' loads landed and all waves are past the previous step), refill
  // slot WR (the stage consumed in the previous step) STAGES-1 ahead, then
  // the matrix cores. The plain s_barrier carries no memory fence, so the
  // loads of later stages stay in flight across it.
#define TD_SPLIT_STEP(RD, WR, kt, FLUSH_OK)                                                \
  {                                                                                        \
    const int ahead = (nk - 1 - (kt)) < (STAGES - 2) ? (nk - 1 - (kt)) : (STAGES - 2);    \
    if (ahead >= 2) {                                                                      \
      TD_WAIT_VMCNT(2 * PER_WAVE);                                                         \
    } else if (ahead == 1) {                                                               \
      TD_WAIT_VMCNT(PER_WAVE);                                                             \
    } else {                                                                               \
      TD_WAIT_VMCNT(0);                                                                    \
    }                                                                                      \
    __builtin_amdgcn_s_barrier();                                                          \
    if ((kt) + STAGES - 1 < nk) TD_ISSUE_STAGE(WR, (kt) + STAGES - 1);                     \
    Frags<S> fr;                                                                           \
    read_frags<S>(fr, lds_u32(RD), ao, bo0, bo1);                                          \
    bf16x8 a[S], b[2][S];                                                                  \
    _Pragma("unroll") for (int sl = 0; sl < S; ++sl) {                                     \
      a[sl] = __builtin_bit_cast(bf16x8, fr.a[sl]);                                        \
      b[0][sl] = __builtin_bit_cast(bf16x8, fr.b0[sl]);                                    \
      b[1][sl] = __builtin_bit_cast(bf16x8, fr.b1[sl]);                                    \
    }                                                                                      \
    _Pragma("unroll") for (int j = 0; j < 2; ++j)                                          \
      acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][0], acc2[j], 0, 0, 0);  \
    _Pragma("unroll") for (int j = 0; j < 2; ++j)                                          \
      acc3[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][1], acc3[j], 0, 0, 0);  \
    _Pragma("unroll") for (int j = 0; j < 2; ++j)                                          \
      acc3[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][0], acc3[j], 0, 0, 0);  \
    _Pragma("unroll") for (int sa = 0; sa < S; ++sa)                                       \
      _Pragma("unroll") for (int sb = 0; sb < S; ++sb)                                     \
        if (sa + sb >= 2 && sa + sb <= S - 1)                                              \
          _Pragma("unroll") for (int j = 0; j < 2; ++j)                                    \
            acc3[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[sa], b[j][sb], acc3[j], 0, \
                                                              0, 0);                       \
    if (FLUSH_OK) {                                                                        \
      const int k_next = ((kt) + 1) * BK;                                                  \
      if constexpr (SEG256) {                                                              \
        if (k_next % CHUNK == 0 || (kt) + 1 == nk)                                         \
          TD_SPLIT_FLUSH(((kt) * BK - ((kt) * BK) % CHUNK) / p.seg_len)                    \
      } else {                                                                             \
        if ((k_next & (CHUNK - 1)) == 0 || k_next == p.seg_len || (kt) + 1 == nk)          \
          TD_SPLIT_FLUSH(((kt) * BK >= p.seg_len) ? 1 : 0)   /* at most two segments */     \
      }                                                                                    \
    }                                                                                      \
  }

  // K and the segment length are multiples of KUNIT (8 steps of BK), so nk
  // is a multiple of STAGES and every chunk and segment ends on the last
  // step of an unrolled group, where the flushes fall.
  for (int kt = 0; kt < nk; kt += STAGES) {
    if (STAGES == 4) {
      TD_SPLIT_STEP(st0, st3, kt, false)
      TD_SPLIT_STEP(st1, st0, kt + 1, false)
      TD_SPLIT_STEP(st2, st1, kt + 2, false)
      TD_SPLIT_STEP(st3, st2, kt + 3, true)
    } else {
      TD_SPLIT_STEP(st0, st1, kt, false)
      TD_SPLIT_STEP(st1, st0, kt + 1, true)
    }
  }
#undef TD_SPLIT_STEP
#undef TD_ISSUE_STAGE
#undef TD_SPLIT_FLUSH

#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = n0 + wn * 64 + j * 32 + l32;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = m0 + wm * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
      double v = acc64[j][e];
      if (p.Cin) v += p.Cin[(size_t)row * p.ldcin + col];
      __builtin_nontemporal_store(v, &p.C[(size_t)row * p.ldc + col]);   // streamed out
    }
  }
}

// ------------------------------------------------------------------ slicing
// One wave per row: exponent e with max |x| < 2^e (0 for a zero row), then S
// rounded slices of x 2^-e 2^8, stored pre-scaled as sigma_t 2^-8(t-1).
template <int S, int MODE>
__global__ __launch_bounds__(256) void k_slice_rows(SliceSrc src, int rows, int cols,
                                                    __bf16* out, int ldo, int* exps) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (row >= rows) return;
  auto value = [&](int c) -> double {
    if (MODE == SLICE_PLAIN) return src.sign * src.M0[(size_t)row * src.ld0 + c];
    if (MODE == SLICE_SUM)
      return src.M0[(size_t)row * src.ld0 + c] + src.M1[(size_t)row * src.ld1 + c];
    if (MODE == SLICE_RENORM)
      return src.M0[(size_t)row * src.ld0 + c] - src.cs[0] * src.M1[(size_t)row * src.ld1 + c];
    // SLICE_DH: 1/2 S_uv (dv_u + dv_v)
    return 0.5 * src.M0[(size_t)row * src.ld0 + c] * (src.v[row] + src.v[c]);
  };
  double m = 0.0;
  for (int c = l; c < cols; c += 64) m = fmax(m, fabs(value(c)));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  int e = 0;
  if (m > 0.0) {
    frexp(m, &e);          // m = f 2^e, f in [0.5, 1): max |x| < 2^e
  }
  if (l == 0) exps[row] = e;
  for (int c = l; c < cols; c += 64) {
    const double x = value(c);
    if (MODE == SLICE_RENORM) src.M0w[(size_t)row * src.ld0 + c] = x;
    double rr = ldexp(x, 8 - e);    // |rr| < 256
    __bf16* o = out + (size_t)row * ldo + (size_t)(c >> 4) * (16 * S) + (c & 15);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double sig = rint(rr);
      o[s * 16] = (__bf16)(float)ldexp(sig, -8 * s);
      rr = (rr - sig) * 256.0;
    }
  }
}

template <int S>
hipError_t launch_split(hipStream_t st, const SplitGemm& g) {
  SplitArgs<S> p;
  p.L = g.L;
  p.ldl = g.ldl;
  p.eL = g.eL;
  p.eL_stride = g.eL_stride;
  p.R = g.R;
  p.ldr = g.ldr;
  p.fR = g.fR;
  p.fR_stride = g.fR_stride;
  p.seg_len = g.seg_len;
  p.k_lo = g.k_lo;
  p.k_hi = g.k_hi;
  p.n_split = g.n_split;
  p.C = g.C;
  p.ldc = g.ldc;
  p.Cin = g.Cin;
  p.ldcin = g.ldcin;
  p.tiles_m = g.m / BM;
  p.tiles_n = g.n / BN;
  if (g.seg_len % CHUNK == 0)
    hipLaunchKernelGGL((sgemm_split<S, true>), dim3(p.tiles_m * p.tiles_n), dim3(512), 0, st, p);
  else
    hipLaunchKernelGGL((sgemm_split<S, false>), dim3(p.tiles_m * p.tiles_n), dim3(512), 0, st, p);
  return hipGetLastError();
}

// Same slicing for rows of at most 128 CPL values, two waves per row: each
// lane keeps its CPL values in registers between the row maximum and the
// slicing, so the source is read from memory once instead of twice. A lane
// holds CPL / 8 runs of 8 consecutive columns, read as 16-byte pairs, and
// writes each slice of a run as one 16-byte store (half a k block).
// SLICE_SUM_AND_M1 slices two rows (M0 + M1 and M1) from one read of M1.
template <int S>
__device__ __forceinline__ void slice_store8(const double* x, int e, __bf16* o) {
  double rr[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) rr[i] = ldexp(x[i], 8 - e);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double sig = rint(rr[i]);
      v[i] = (__bf16)(float)ldexp(sig, -8 * s);
      rr[i] = (rr[i] - sig) * 256.0;
    }
    *reinterpret_cast<bf16x8*>(o + s * 16) = v;
  }
}

__device__ __forceinline__ double pair_max(double m, double* wmax) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  return fmax(wmax[(threadIdx.x >> 7) * 2], wmax[(threadIdx.x >> 7) * 2 + 1]);
}

// 8 consecutive doubles from a 16-byte aligned address
__device__ __forceinline__ void load8(const double* p, double* v) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 t = q[i];
    v[2 * i] = t.x;
    v[2 * i + 1] = t.y;
  }
}

template <int S, int MODE, int CPL>
__global__ __launch_bounds__(256) void k_slice_rows_cached(SliceSrc src, int rows, int cols,
                                                           __bf16* out, int ldo, int* exps) {
  static_assert(CPL % 8 == 0, "runs of 8 columns");
  constexpr int RUNS = CPL / 8;
  __shared__ double wmax[4], wmax2[4];
  const int row = blockIdx.x * 2 + (threadIdx.x >> 7);
  const int l = threadIdx.x & 127;
  const bool live = row < rows;
  constexpr bool TWO = MODE == SLICE_SUM_AND_M1;
  double x[CPL], y[TWO ? CPL : 1];
  double m = 0.0, m2 = 0.0;
#pragma unroll
  for (int g = 0; g < RUNS; ++g) {
    const int c = 8 * (l + 128 * g);          // cols is a multiple of 16: runs are whole
    double* xv = x + 8 * g;
    double a[8], b[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = b[i] = 0.0;
    if (live && c < cols) {
      load8(src.M0 + (size_t)row * src.ld0 + c, a);
      if (MODE == SLICE_SUM || MODE == SLICE_SUM_AND_M1 || MODE == SLICE_RENORM)
        load8(src.M1 + (size_t)row * src.ld1 + c, b);
      else if (MODE == SLICE_DH)
        load8(src.v + c, b);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      double val;
      if (MODE == SLICE_PLAIN) {
        val = src.sign * a[i];
      } else if (MODE == SLICE_SUM || MODE == SLICE_SUM_AND_M1) {
        val = a[i] + b[i];
      } else if (MODE == SLICE_RENORM) {
        val = a[i] - src.cs[0] * b[i];
      } else {
        val = 0.5 * a[i] * (src.v[row < rows ? row : 0] + b[i]);
      }
      xv[i] = val;
      m = fmax(m, fabs(val));
      if constexpr (TWO) {
        y[8 * g + i] = b[i];
        m2 = fmax(m2, fabs(b[i]));
      }
    }
  }
  m = pair_max(m, wmax);
  if constexpr (TWO) m2 = pair_max(m2, wmax2);
  if (!live) return;
  int e = 0, e2 = 0;
  if (m > 0.0) frexp(m, &e);
  if (TWO && m2 > 0.0) frexp(m2, &e2);
  if (l == 0) {
    exps[row] = e;
    if (TWO) src.exps2[row] = e2;
  }
#pragma unroll
  for (int g = 0; g < RUNS; ++g) {
    const int c = 8 * (l + 128 * g);
    if (c < cols) {
      if (MODE == SLICE_RENORM) {
        double2* w = reinterpret_cast<double2*>(src.M0w + (size_t)row * src.ld0 + c);
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = make_double2(x[8 * g + 2 * i], x[8 * g + 2 * i + 1]);
      }
      const size_t at = (size_t)row * ldo + (size_t)(c >> 4) * (16 * S) + (c & 15);
      slice_store8<S>(x + 8 * g, e, out + at);
      if constexpr (TWO) slice_store8<S>(y + 8 * g, e2, src.out2 + at);
    }
  }
}

template <int S>
hipError_t launch_slice(hipStream_t st, int mode, const SliceSrc& src, int rows, int cols,
                        __bf16* out, int ldo, int* exps) {
  if (cols <= 128 * 32) {
    const dim3 grid((rows + 1) / 2), block(256);
    switch (mode) {
      case SLICE_PLAIN:
        hipLaunchKernelGGL((k_slice_rows_cached<S, SLICE_PLAIN, 32>), grid, block, 0, st, src,
                           rows, cols, out, ldo, exps);
        break;
      case SLICE_SUM:
        hipLaunchKernelGGL((k_slice_rows_cached<S, SLICE_SUM, 32>), grid, block, 0, st, src, rows,
                           cols, out, ldo, exps);
        break;
      case SLICE_DH:
        hipLaunchKernelGGL((k_slice_rows_cached<S, SLICE_DH, 32>), grid, block, 0, st, src, rows,
                           cols, out, ldo, exps);
        break;
      case SLICE_RENORM:
        hipLaunchKernelGGL((k_slice_rows_cached<S, SLICE_RENORM, 32>), grid, block, 0, st, src,
                           rows, cols, out, ldo, exps);
        break;
      case SLICE_SUM_AND_M1:
        if (!src.out2 || !src.exps2) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_slice_rows_cached<S, SLICE_SUM_AND_M1, 32>), grid, block, 0, st,
                           src, rows, cols, out, ldo, exps);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const dim3 grid((rows + 3) / 4), block(256);
  switch (mode) {
    case SLICE_PLAIN:
      hipLaunchKernelGGL((k_slice_rows<S, SLICE_PLAIN>), grid, block, 0, st, src, rows, cols, out,
                         ldo, exps);
      break;
    case SLICE_SUM:
      hipLaunchKernelGGL((k_slice_rows<S, SLICE_SUM>), grid, block, 0, st, src, rows, cols, out,
                         ldo, exps);
      break;
    case SLICE_DH:
      hipLaunchKernelGGL((k_slice_rows<S, SLICE_DH>), grid, block, 0, st, src, rows, cols, out,
                         ldo, exps);
      break;
    case SLICE_RENORM:
      hipLaunchKernelGGL((k_slice_rows<S, SLICE_RENORM>), grid, block, 0, st, src, rows, cols,
                         out, ldo, exps);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t split_gemm(hipStream_t st, int n_slices, const SplitGemm& g) {
  if (g.m % BM || g.n % BN || g.m <= 0 || g.n <= 0) return hipErrorInvalidValue;
  // one or two K segments of seg_len
  const auto segs_ok = [&](int k) { return k == g.seg_len || k == 2 * g.seg_len; };
  if (g.seg_len <= 0 || g.seg_len % KUNIT || !segs_ok(g.k_lo) || !segs_ok(g.k_hi))
    return hipErrorInvalidValue;
  if (g.ldl % (16 * n_slices) || g.ldr % (16 * n_slices)) return hipErrorInvalidValue;
  switch (n_slices) {
    case 3: return launch_split<3>(st, g);
    case 4: return launch_split<4>(st, g);
    case 5: return launch_split<5>(st, g);
    default: return hipErrorInvalidValue;
  }
}

hipError_t slice_rows(hipStream_t st, int n_slices, int mode, const SliceSrc& src, int rows,
                      int cols, __bf16* out, int ldo, int* exps) {
  if (cols % 16) return hipErrorInvalidValue;
  switch (n_slices) {
    case 3: return launch_slice<3>(st, mode, src, rows, cols, out, ldo, exps);
    case 4: return launch_slice<4>(st, mode, src, rows, cols, out, ldo, exps);
    case 5: return launch_slice<5>(st, mode, src, rows, cols, out, ldo, exps);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace td
