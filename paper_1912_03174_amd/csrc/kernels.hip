// O(n^2) and O(n_atoms^2) kernels of the propagation step and of the
// initialisation: Mulliken charges (Sec. 2.1, Eq. 5), the SCC potential
// and Hamiltonian rebuild (Eqs. 6-7), the leapfrog update (Sec. 2.3,
// Eq. 19) with rhodot = -i (X - X^+), X = S^-1 H rho (Eq. 10), the kick
// phase (Sec. 2.2, Eq. 16), purification and Newton-Schulz helpers, and
// deterministic reductions (fixed-order trees, no floating-point atomics),
// so repeated runs give bitwise identical results.
#include <cmath>

#include "common.hpp"
#include "reduce.hpp"

namespace td {
namespace {

// ------------------------------------------------------------------ rowdot
// One wave per row; 4 rows per 256-thread block; cols even.
__global__ __launch_bounds__(256) void k_rowdot(const double* __restrict__ X, int ldx,
                                                const double* __restrict__ Y, int ldy,
                                                double* __restrict__ out, int rows, int cols) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (row >= rows) return;
  const double2* x = reinterpret_cast<const double2*>(X + (size_t)row * ldx);
  const double2* y = reinterpret_cast<const double2*>(Y + (size_t)row * ldy);
  double acc = 0.0;
  for (int c = l; c < cols / 2; c += WAVE) {
    const double2 a = x[c], b = y[c];
    acc = fma(a.x, b.x, acc);
    acc = fma(a.y, b.y, acc);
  }
  acc = wave_sum(acc);
  if (l == 0) out[row] = acc;
}

// ------------------------------------------------------------------ charges
__global__ __launch_bounds__(1024) void k_charges_dipole(const double* __restrict__ q_orb,
                                                         const int* __restrict__ off,
                                                         const double* __restrict__ q0,
                                                         const double* __restrict__ pos,
                                                         int na, double* __restrict__ dq,
                                                         double* __restrict__ mu_out,
                                                         double* __restrict__ ne_out) {
  __shared__ double sh[17];
  double mx = 0.0, my = 0.0, mz = 0.0, ne = 0.0;
  for (int a = threadIdx.x; a < na; a += 1024) {
    double q = 0.0;
    for (int u = off[a]; u < off[a + 1]; ++u) q += q_orb[u];
    const double d = q - q0[a];
    dq[a] = d;
    ne += q;
    mx -= d * pos[3 * a + 0];
    my -= d * pos[3 * a + 1];
    mz -= d * pos[3 * a + 2];
  }
  mx = block_sum_1024(mx, sh);
  my = block_sum_1024(my, sh);
  mz = block_sum_1024(mz, sh);
  ne = block_sum_1024(ne, sh);
  if (threadIdx.x == 0) {
    mu_out[0] = mx;
    mu_out[1] = my;
    mu_out[2] = mz;
    if (ne_out) ne_out[0] = ne;
  }
}

// ------------------------------------------------------------------ potential
// One wave per atom.
__global__ __launch_bounds__(256) void k_potential(const double* __restrict__ gamma,
                                                   const double* __restrict__ dq,
                                                   const double* __restrict__ pos,
                                                   const double* __restrict__ E,
                                                   const int* __restrict__ off, int na,
                                                   double* __restrict__ v,
                                                   double* __restrict__ vorb,
                                                   const double* __restrict__ v_ref) {
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (a >= na) return;
  const double* g = gamma + (size_t)a * na;
  double acc = 0.0;
  for (int c = l; c < na; c += WAVE) acc = fma(g[c], dq[c], acc);
  acc = wave_sum(acc);
  if (E) acc += pos[3 * a] * E[0] + pos[3 * a + 1] * E[1] + pos[3 * a + 2] * E[2];
  if (l == 0) v[a] = acc;
  const double vo = v_ref ? acc - v_ref[a] : acc;
  for (int u = off[a] + l; u < off[a + 1]; u += WAVE) vorb[u] = vo;
}

// ------------------------------------------------------------------ H assembly
__global__ __launch_bounds__(256) void k_assemble_h(const double* __restrict__ H0,
                                                    const double* __restrict__ S,
                                                    const double* __restrict__ vorb,
                                                    double* __restrict__ H, int n) {
  const size_t idx2 = (size_t)blockIdx.x * 256 + threadIdx.x;   // pair index
  const size_t total2 = (size_t)n * n / 2;
  if (idx2 >= total2) return;
  const size_t e = idx2 * 2;
  const int r = (int)(e / n), c = (int)(e % n);
  const double2 h0 = reinterpret_cast<const double2*>(H0)[idx2];
  const double2 s = reinterpret_cast<const double2*>(S)[idx2];
  const double vr = vorb[r];
  double2 out;
  out.x = h0.x + 0.5 * s.x * (vr + vorb[c]);
  out.y = h0.y + 0.5 * s.y * (vr + vorb[c + 1]);
  reinterpret_cast<double2*>(H)[idx2] = out;
}

// ------------------------------------------------------------------ pair passes
constexpr int TS = 32;
constexpr int TLD = TS + 1;

enum { PAIR_LEAPFROG = 0, PAIR_HERM = 1, PAIR_SYM = 2 };

// Block k of the upper triangle of ntiles x ntiles tiles, row by row, handles
// tiles (bi, bj) and (bj, bi), bi <= bj.
// Thread t: row t/8 of the tile, 4 consecutive columns at 4*(t%8), moved as
// two 16-byte pairs. Every global read of a thread (both tiles, and the
// addend b of the leapfrog) is issued before its first write: the output
// may alias b or x (in-place update), and reads then stores in program order
// keep the loads in flight together instead of one round trip per store.
// For PAIR_LEAPFROG, xref (optional, leading dimension ldr) is a real
// addend of X: Re X = xre + xref.
template <int MODE>
__global__ __launch_bounds__(256) void k_pair(const double* xre, const double* xim, int ldx,
                                              const double* bre, const double* bim, int ldb,
                                              double* ore, double* oim, int ldo, double f,
                                              const double* xref, int ldr, const double* zre,
                                              const double* zim, int ldz, int ntiles) {
  // row bi of the triangle starts at bi T - bi (bi - 1) / 2, T = ntiles
  const int T = ntiles, k = blockIdx.x;
  const double w = 2.0 * T + 1.0;
  int bi = (int)((w - sqrt(w * w - 8.0 * k)) * 0.5);
  bi = bi < 0 ? 0 : (bi >= T ? T - 1 : bi);
  while (bi > 0 && bi * T - bi * (bi - 1) / 2 > k) --bi;
  while (bi + 1 < T && (bi + 1) * T - (bi + 1) * bi / 2 <= k) ++bi;
  const int bj = bi + (k - (bi * T - bi * (bi - 1) / 2));
  __shared__ double sre[2][TS][TLD];   // [0]: tile (bi,bj), [1]: tile (bj,bi)
  __shared__ double sim[2][TS][TLD];
  const int t = threadIdx.x;
  const int tr = t >> 3, tc = (t & 7) * 4;
  const bool diag = (bi == bj);
  const int nt = diag ? 1 : 2;
  double2 xr[2][2], xi[2][2], br[2][2], bm[2][2], xf[2][2], zr[2][2], zi[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p < nt) {
      const int ti = p ? bj : bi, tj = p ? bi : bj;
      const size_t g = (size_t)(ti * TS + tr) * ldx + tj * TS + tc;
      xr[p][0] = *reinterpret_cast<const double2*>(xre + g);
      xr[p][1] = *reinterpret_cast<const double2*>(xre + g + 2);
      if (MODE == PAIR_LEAPFROG && xref) {
        const size_t gr = (size_t)(ti * TS + tr) * ldr + tj * TS + tc;
        xf[p][0] = *reinterpret_cast<const double2*>(xref + gr);
        xf[p][1] = *reinterpret_cast<const double2*>(xref + gr + 2);
      }
      if (MODE != PAIR_SYM) {
        xi[p][0] = *reinterpret_cast<const double2*>(xim + g);
        xi[p][1] = *reinterpret_cast<const double2*>(xim + g + 2);
      }
      if (MODE == PAIR_LEAPFROG && zre) {
        const size_t gz = (size_t)(ti * TS + tr) * ldz + tj * TS + tc;
        zr[p][0] = *reinterpret_cast<const double2*>(zre + gz);
        zr[p][1] = *reinterpret_cast<const double2*>(zre + gz + 2);
        zi[p][0] = *reinterpret_cast<const double2*>(zim + gz);
        zi[p][1] = *reinterpret_cast<const double2*>(zim + gz + 2);
      }
      if (MODE == PAIR_LEAPFROG) {
        const size_t gb = (size_t)(ti * TS + tr) * ldb + tj * TS + tc;
        br[p][0] = *reinterpret_cast<const double2*>(bre + gb);
        br[p][1] = *reinterpret_cast<const double2*>(bre + gb + 2);
        bm[p][0] = *reinterpret_cast<const double2*>(bim + gb);
        bm[p][1] = *reinterpret_cast<const double2*>(bim + gb + 2);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p < nt) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (MODE == PAIR_LEAPFROG && xref) {
          xr[p][h].x = xr[p][h].x + xf[p][h].x;
          xr[p][h].y = xr[p][h].y + xf[p][h].y;
        }
        if (MODE == PAIR_LEAPFROG && zre) {      // X - i Z
          xr[p][h].x = xr[p][h].x + zi[p][h].x;
          xr[p][h].y = xr[p][h].y + zi[p][h].y;
          xi[p][h].x = xi[p][h].x - zr[p][h].x;
          xi[p][h].y = xi[p][h].y - zr[p][h].y;
        }
        sre[p][tr][tc + 2 * h] = xr[p][h].x;
        sre[p][tr][tc + 2 * h + 1] = xr[p][h].y;
        if (MODE != PAIR_SYM) {
          sim[p][tr][tc + 2 * h] = xi[p][h].x;
          sim[p][tr][tc + 2 * h + 1] = xi[p][h].y;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p < nt) {
      const int ti = p ? bj : bi, tj = p ? bi : bj;
      const int q = diag ? 0 : (p ^ 1);   // tile holding the transpose partner
      const size_t go = (size_t)(ti * TS + tr) * ldo + tj * TS + tc;
      double r[4], m[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int cc = tc + c;
        const double are = sre[p][tr][cc], aret = sre[q][cc][tr];
        if (MODE == PAIR_LEAPFROG) {
          const double aim = sim[p][tr][cc], aimt = sim[q][cc][tr];
          const double dre = aim + aimt;     // Re rhodot = Xim + Xim^T
          const double dim = aret - are;     // Im rhodot = Xre^T - Xre
          const double b_re = (c & 1) ? br[p][c >> 1].y : br[p][c >> 1].x;
          const double b_im = (c & 1) ? bm[p][c >> 1].y : bm[p][c >> 1].x;
          r[c] = b_re + f * dre;
          m[c] = b_im + f * dim;
        } else if (MODE == PAIR_HERM) {
          const double aim = sim[p][tr][cc], aimt = sim[q][cc][tr];
          r[c] = 0.5 * (are + aret);
          m[c] = 0.5 * (aim - aimt);
        } else {
          r[c] = 0.5 * (are + aret);
          m[c] = 0.0;
        }
      }
      *reinterpret_cast<double2*>(ore + go) = make_double2(r[0], r[1]);
      *reinterpret_cast<double2*>(ore + go + 2) = make_double2(r[2], r[3]);
      if (MODE != PAIR_SYM || oim) {
        *reinterpret_cast<double2*>(oim + go) = make_double2(m[0], m[1]);
        *reinterpret_cast<double2*>(oim + go + 2) = make_double2(m[2], m[3]);
      }
    }
  }
}

// ------------------------------------------------------------------ elementwise
__global__ void k_kick_phase(double* re, double* im, int ld, const double* __restrict__ x,
                             int np, double kappa) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  const size_t g = (size_t)r * ld + c;
  double sn, cs;
  sincos(-kappa * (x[r] - x[c]), &sn, &cs);
  const double a = re[g], b = im[g];
  re[g] = a * cs - b * sn;
  im[g] = a * sn + b * cs;
}

__global__ void k_scaled_identity(double* X, int np, int n, double c) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), cc = (int)(idx % np);
  X[idx] = (r == cc && r < n) ? c : 0.0;
}

// y <- 2 x - y
__global__ void k_extrapolate(const double* x0, const double* x1, const double* x2, double* out,
                              size_t len) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= len) return;
  if (x2)
    out[idx] = 3.0 * (x0[idx] - x1[idx]) + x2[idx];
  else
    out[idx] = 2.0 * x0[idx] - x1[idx];
}

__global__ void k_two_minus(double* T, int np, int n) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  T[idx] = ((r == c && r < n) ? 2.0 : 0.0) - T[idx];
}

__global__ void k_sp2_init(const double* __restrict__ T, double* __restrict__ X, int np, int n,
                           double emax, double inv_width) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  const double id = (r == c && r < n) ? emax : 0.0;
  X[idx] = (id - T[idx]) * inv_width;
}

__global__ void k_sp2_update(double* X, const double* __restrict__ X2, size_t total, int mode) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  X[idx] = mode ? (2.0 * X[idx] - X2[idx]) : X2[idx];
}

__global__ void k_real_to_wide(const double* __restrict__ R, int ldr, double* __restrict__ W,
                               int np) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  W[(size_t)r * 2 * np + c] = R[(size_t)r * ldr + c];
  W[(size_t)r * 2 * np + np + c] = 0.0;
}

__global__ void k_interleaved_to_wide(const double* __restrict__ Z, int n,
                                      double* __restrict__ W, int np) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  double a = 0.0, b = 0.0;
  if (r < n && c < n) {
    a = Z[2 * ((size_t)r * n + c)];
    b = Z[2 * ((size_t)r * n + c) + 1];
  }
  W[(size_t)r * 2 * np + c] = a;
  W[(size_t)r * 2 * np + np + c] = b;
}

__global__ void k_wide_to_interleaved(const double* __restrict__ W, int np,
                                      double* __restrict__ Z, int n) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int r = (int)(idx / n), c = (int)(idx % n);
  Z[2 * idx] = W[(size_t)r * 2 * np + c];
  Z[2 * idx + 1] = W[(size_t)r * 2 * np + np + c];
}

__global__ void k_pad_copy(const double* __restrict__ src, int n, double* __restrict__ dst,
                           int np) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int r = (int)(idx / n), c = (int)(idx % n);
  dst[(size_t)r * np + c] = src[idx];
}

__global__ void k_unpad_copy(const double* __restrict__ src, int np, double* __restrict__ dst,
                             int n) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int r = (int)(idx / n), c = (int)(idx % n);
  dst[idx] = src[(size_t)r * np + c];
}

// ------------------------------------------------------------------ reductions
__global__ __launch_bounds__(1024) void k_trace(const double* __restrict__ X, int ld, int n,
                                                double* out) {
  __shared__ double sh[17];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += X[(size_t)i * ld + i];
  acc = block_sum_1024(acc, sh);
  if (threadIdx.x == 0) out[0] = acc;
}

__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ x, int n, double* out) {
  __shared__ double sh[17];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += x[i];
  acc = block_sum_1024(acc, sh);
  if (threadIdx.x == 0) out[0] = acc;
}

// per-row max |delta_ij - T_ij|
__global__ __launch_bounds__(256) void k_row_identity_resid(const double* __restrict__ T, int ld,
                                                            int n, double* __restrict__ rowmax) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (row >= n) return;
  double m = 0.0;
  for (int c = l; c < n; c += WAVE) {
    const double d = ((c == row) ? 1.0 : 0.0) - T[(size_t)row * ld + c];
    m = fmax(m, fabs(d));
  }
  m = wave_max(m);
  if (l == 0) rowmax[row] = m;
}

__global__ __launch_bounds__(1024) void k_max(const double* __restrict__ x, int n, double* out) {
  __shared__ double sh[17];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 1024) m = fmax(m, x[i]);
  m = block_max_1024(m, sh);
  if (threadIdx.x == 0) out[0] = m;
}

// Per row: +inf if the row holds a value that is not finite, else the
// largest |M[r, c] - M[c, r]| (symmetric) or 0.
__global__ __launch_bounds__(256) void k_row_check(const double* __restrict__ M, int ld, int rows,
                                                   int cols, int symmetric,
                                                   double* __restrict__ rowmax) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (row >= rows) return;
  double m = 0.0;
  for (int c = l; c < cols; c += WAVE) {
    const double v = M[(size_t)row * ld + c];
    if (!isfinite(v)) m = INFINITY;
    else if (symmetric && c != row) m = fmax(m, fabs(v - M[(size_t)c * ld + row]));
  }
  m = wave_max(m);
  if (l == 0) rowmax[row] = m;
}

__global__ __launch_bounds__(256) void k_row_gershgorin(const double* __restrict__ T, int ld,
                                                        int n, double* __restrict__ lo,
                                                        double* __restrict__ hi) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (row >= n) return;
  double rad = 0.0;
  for (int c = l; c < n; c += WAVE)
    if (c != row) rad += fabs(T[(size_t)row * ld + c]);
  rad = wave_sum(rad);
  if (l == 0) {
    const double d = T[(size_t)row * ld + row];
    lo[row] = d - rad;
    hi[row] = d + rad;
  }
}

__global__ __launch_bounds__(1024) void k_minmax(const double* __restrict__ lo,
                                                 const double* __restrict__ hi, int n,
                                                 double* out) {
  __shared__ double sh[17];
  double a = INFINITY, b = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 1024) {
    a = fmin(a, lo[i]);
    b = fmax(b, hi[i]);
  }
  a = block_min_1024(a, sh);
  b = block_max_1024(b, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// ------------------------------------------------------------------ Anderson mixing
// One 1024-thread block. History ring of m entries (x = dq_in, f = residual).
constexpr int MAXH = 8;
__global__ __launch_bounds__(1024) void k_anderson(double* dq_in, const double* __restrict__ dq_out,
                                                   double* hx, double* hf, int na, int m,
                                                   int count, int slot, double beta,
                                                   double* out_resid) {
  __shared__ double sh[17];
  __shared__ double G[MAXH][MAXH];
  __shared__ double rhs[MAXH];
  __shared__ double gsol[MAXH];
  double rmax = 0.0;
  for (int a = threadIdx.x; a < na; a += 1024) {
    const double r = dq_out[a] - dq_in[a];
    hx[(size_t)slot * na + a] = dq_in[a];
    hf[(size_t)slot * na + a] = r;
    rmax = fmax(rmax, fabs(r));
  }
  rmax = block_max_1024(rmax, sh);
  if (threadIdx.x == 0) out_resid[0] = rmax;
  __syncthreads();
  const int k = count;            // entries valid, newest at slot
  const int p = k - 1;            // difference columns
  if (p <= 0) {
    for (int a = threadIdx.x; a < na; a += 1024)
      dq_in[a] += beta * hf[(size_t)slot * na + a];
    return;
  }
  // entry i (0 = oldest) lives at ring index (slot - k + 1 + i) mod m
  auto idx = [&](int i) { return ((slot - k + 1 + i) % m + m) % m; };
  for (int i = 0; i < p; ++i) {
    for (int j = i; j < p; ++j) {
      double acc = 0.0;
      for (int a = threadIdx.x; a < na; a += 1024) {
        const double fi = hf[(size_t)idx(i + 1) * na + a] - hf[(size_t)idx(i) * na + a];
        const double fj = hf[(size_t)idx(j + 1) * na + a] - hf[(size_t)idx(j) * na + a];
        acc += fi * fj;
      }
      acc = block_sum_1024(acc, sh);
      if (threadIdx.x == 0) {
        G[i][j] = acc;
        G[j][i] = acc;
      }
    }
    double acc = 0.0;
    for (int a = threadIdx.x; a < na; a += 1024) {
      const double fi = hf[(size_t)idx(i + 1) * na + a] - hf[(size_t)idx(i) * na + a];
      acc += fi * hf[(size_t)slot * na + a];
    }
    acc = block_sum_1024(acc, sh);
    if (threadIdx.x == 0) rhs[i] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double M[MAXH][MAXH + 1];
    double dmax = 0.0;
    for (int i = 0; i < p; ++i) dmax = fmax(dmax, G[i][i]);
    for (int i = 0; i < p; ++i) {
      for (int j = 0; j < p; ++j) M[i][j] = G[i][j] + ((i == j) ? 1e-12 * dmax : 0.0);
      M[i][p] = rhs[i];
    }
    for (int c = 0; c < p; ++c) {           // Gaussian elimination, partial pivoting
      int piv = c;
      for (int i = c + 1; i < p; ++i)
        if (fabs(M[i][c]) > fabs(M[piv][c])) piv = i;
      if (piv != c)
        for (int j = 0; j <= p; ++j) {
          const double tmp = M[c][j];
          M[c][j] = M[piv][j];
          M[piv][j] = tmp;
        }
      const double d = M[c][c];
      if (d == 0.0) continue;
      for (int i = c + 1; i < p; ++i) {
        const double fct = M[i][c] / d;
        for (int j = c; j <= p; ++j) M[i][j] -= fct * M[c][j];
      }
    }
    for (int i = p - 1; i >= 0; --i) {
      double acc = M[i][p];
      for (int j = i + 1; j < p; ++j) acc -= M[i][j] * gsol[j];
      gsol[i] = (M[i][i] != 0.0) ? acc / M[i][i] : 0.0;
    }
  }
  __syncthreads();
  for (int a = threadIdx.x; a < na; a += 1024) {
    double x = dq_in[a] + beta * hf[(size_t)slot * na + a];
    for (int i = 0; i < p; ++i) {
      const double dx = hx[(size_t)idx(i + 1) * na + a] - hx[(size_t)idx(i) * na + a];
      const double df = hf[(size_t)idx(i + 1) * na + a] - hf[(size_t)idx(i) * na + a];
      x -= gsol[i] * (dx + beta * df);
    }
    dq_in[a] = x;
  }
}

// ------------------------------------------------------------------ energy
__global__ __launch_bounds__(1024) void k_energy(const double* __restrict__ band_rows, int n,
                                                 const double* __restrict__ dq,
                                                 const double* __restrict__ vg,
                                                 const double* __restrict__ pos,
                                                 const double* __restrict__ E, int na,
                                                 double* out) {
  __shared__ double sh[17];
  double b = 0.0, c = 0.0, e = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) b += band_rows[i];
  for (int a = threadIdx.x; a < na; a += 1024) {
    c += 0.5 * dq[a] * vg[a];
    if (E) e += dq[a] * (pos[3 * a] * E[0] + pos[3 * a + 1] * E[1] + pos[3 * a + 2] * E[2]);
  }
  b = block_sum_1024(b, sh);
  c = block_sum_1024(c, sh);
  e = block_sum_1024(e, sh);
  if (threadIdx.x == 0) {
    out[0] = b;
    out[1] = c;
    out[2] = e;
  }
}

// Split precision: populations q = q_delta + q_ref; the electron count
// N(t) = sum q gives the trace correction c = (N(t) - n_elec) / n_elec,
// applied as rho <- rho - c rho_ref (linear, so q <- q - c q_ref).
__global__ __launch_bounds__(1024) void k_charges_dipole_split(
    const double* __restrict__ q_delta, const double* __restrict__ q_ref,
    const int* __restrict__ off, const double* __restrict__ q0, const double* __restrict__ pos,
    int na, double n_elec, double* __restrict__ dq, double* __restrict__ mu_out,
    double* __restrict__ c_out) {
  __shared__ double sh[17];
  double ne = 0.0;
  for (int a = threadIdx.x; a < na; a += 1024)
    for (int u = off[a]; u < off[a + 1]; ++u) ne += q_delta[u] + q_ref[u];
  ne = block_sum_1024(ne, sh);
  const double c = (ne - n_elec) / n_elec;
  double mx = 0.0, my = 0.0, mz = 0.0;
  for (int a = threadIdx.x; a < na; a += 1024) {
    double q = 0.0;
    for (int u = off[a]; u < off[a + 1]; ++u) q += q_delta[u] + (1.0 - c) * q_ref[u];
    const double d = q - q0[a];
    dq[a] = d;
    mx -= d * pos[3 * a + 0];
    my -= d * pos[3 * a + 1];
    mz -= d * pos[3 * a + 2];
  }
  mx = block_sum_1024(mx, sh);
  my = block_sum_1024(my, sh);
  mz = block_sum_1024(mz, sh);
  if (threadIdx.x == 0) {
    mu_out[0] = mx;
    mu_out[1] = my;
    mu_out[2] = mz;
    c_out[0] = c;
  }
}

__global__ void k_wide_add_real(double* W, const double* __restrict__ R, int np, double sign) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  W[(size_t)r * 2 * np + c] += sign * R[idx];
}

__global__ void k_vec_add(const double* __restrict__ a, const double* __restrict__ b,
                          double* __restrict__ out, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

// ------------------------------------------------------------------ spectral width
// Start block of the power iteration: +-1 from a hash of (row, column) in
// the first n rows, zero in the padding rows.
__global__ void k_power_start(double* __restrict__ V, int ld, int n, int np, int ncols) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * ncols) return;
  const int r = (int)(idx / ncols), j = (int)(idx % ncols);
  unsigned h = (unsigned)r * 2654435761u ^ ((unsigned)j * 40503u + 0x9e3779b9u);
  h ^= h >> 15;
  h *= 0x2c1b3c6du;
  h ^= h >> 12;
  V[(size_t)r * ld + j] = r < n ? ((h & 1u) ? 1.0 : -1.0) : 0.0;
}

// One block per column j: U = W - lo V (j < half) or hi V - W (j >= half),
// then V = U / |U|. Each element is read and rewritten by the same thread,
// after the block's norm is complete.
__global__ __launch_bounds__(1024) void k_power_step(const double* __restrict__ W,
                                                     double* __restrict__ V, int ld, int np,
                                                     int half, double lo, double hi) {
  __shared__ double sh[17];
  const int j = blockIdx.x;
  const bool top = j < half;
  double ss = 0.0;
  for (int r = threadIdx.x; r < np; r += 1024) {
    const size_t o = (size_t)r * ld + j;
    const double u = top ? W[o] - lo * V[o] : hi * V[o] - W[o];
    ss += u * u;
  }
  ss = block_sum_1024(ss, sh);
  const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  for (int r = threadIdx.x; r < np; r += 1024) {
    const size_t o = (size_t)r * ld + j;
    const double u = top ? W[o] - lo * V[o] : hi * V[o] - W[o];
    V[o] = u * inv;
  }
}

// Generalized Rayleigh quotient of each column: W = T V with T = S^-1 H
// and SV = S V give x^T H x / x^T S x = (SV . W) / (SV . V).
__global__ __launch_bounds__(1024) void k_rayleigh(const double* __restrict__ V,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ SV, int ld, int np,
                                                   double* __restrict__ out) {
  __shared__ double sh[17];
  const int j = blockIdx.x;
  double num = 0.0, den = 0.0;
  for (int r = threadIdx.x; r < np; r += 1024) {
    const size_t o = (size_t)r * ld + j;
    num += SV[o] * W[o];
    den += SV[o] * V[o];
  }
  num = block_sum_1024(num, sh);
  den = block_sum_1024(den, sh);
  if (threadIdx.x == 0) out[j] = num / den;
}

inline unsigned blocks_for(size_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t rowdot(hipStream_t s, const double* X, int ldx, const double* Y, int ldy,
                  double* out, int rows, int cols) {
  if (cols % 2 || ldx % 2 || ldy % 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rowdot, dim3((rows + 3) / 4), dim3(256), 0, s, X, ldx, Y, ldy, out, rows,
                     cols);
  return hipGetLastError();
}

hipError_t charges_dipole(hipStream_t s, const double* q_orb, const int* orb_off,
                          const double* q0, const double* pos, int na, double* dq,
                          double* mu_out, double* ne_out) {
  hipLaunchKernelGGL(k_charges_dipole, dim3(1), dim3(1024), 0, s, q_orb, orb_off, q0, pos, na,
                     dq, mu_out, ne_out);
  return hipGetLastError();
}

hipError_t potential(hipStream_t s, const double* gamma, const double* dq, const double* pos,
                     const double* E, const int* orb_off, int na, double* v, double* vorb,
                     const double* v_ref) {
  hipLaunchKernelGGL(k_potential, dim3((na + 3) / 4), dim3(256), 0, s, gamma, dq, pos, E,
                     orb_off, na, v, vorb, v_ref);
  return hipGetLastError();
}

hipError_t charges_dipole_split(hipStream_t s, const double* q_delta, const double* q_ref,
                                const int* orb_off, const double* q0, const double* pos, int na,
                                double n_elec, double* dq, double* mu_out, double* c_out) {
  hipLaunchKernelGGL(k_charges_dipole_split, dim3(1), dim3(1024), 0, s, q_delta, q_ref, orb_off,
                     q0, pos, na, n_elec, dq, mu_out, c_out);
  return hipGetLastError();
}

hipError_t wide_add_real(hipStream_t s, double* W, const double* R, int np, double sign) {
  hipLaunchKernelGGL(k_wide_add_real, dim3(blocks_for((size_t)np * np)), dim3(256), 0, s, W, R,
                     np, sign);
  return hipGetLastError();
}

hipError_t vec_add(hipStream_t s, const double* a, const double* b, double* out, int n) {
  hipLaunchKernelGGL(k_vec_add, dim3(blocks_for((size_t)n)), dim3(256), 0, s, a, b, out, n);
  return hipGetLastError();
}

hipError_t assemble_h(hipStream_t s, const double* H0, const double* S, const double* vorb,
                      double* H, int n) {
  if (n % 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_assemble_h, dim3(blocks_for((size_t)n * n / 2)), dim3(256), 0, s, H0, S,
                     vorb, H, n);
  return hipGetLastError();
}

hipError_t pair_leapfrog(hipStream_t s, const double* xre, const double* xim, int ldx,
                         const double* bre, const double* bim, int ldb, double* ore, double* oim,
                         int ldo, int np, double f, const double* xref, int ldr,
                         const double* zre, const double* zim, int ldz) {
  if (np % TS) return hipErrorInvalidValue;
  if ((zre == nullptr) != (zim == nullptr)) return hipErrorInvalidValue;
  const int nt = np / TS;
  hipLaunchKernelGGL(k_pair<PAIR_LEAPFROG>, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, xre, xim,
                     ldx, bre, bim, ldb, ore, oim, ldo, f, xref, ldr, zre, zim, ldz, nt);
  return hipGetLastError();
}

hipError_t pair_herm(hipStream_t s, const double* tre, const double* tim, int ldt, double* ore,
                     double* oim, int ldo, int np) {
  if (np % TS) return hipErrorInvalidValue;
  const int nt = np / TS;
  hipLaunchKernelGGL(k_pair<PAIR_HERM>, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, tre, tim, ldt,
                     (const double*)nullptr, (const double*)nullptr, 0, ore, oim, ldo, 0.0,
                     (const double*)nullptr, 0, (const double*)nullptr, (const double*)nullptr,
                     0, nt);
  return hipGetLastError();
}

hipError_t pair_sym(hipStream_t s, const double* t, int ldt, double* ore, double* oim, int ldo,
                    int np) {
  if (np % TS) return hipErrorInvalidValue;
  const int nt = np / TS;
  hipLaunchKernelGGL(k_pair<PAIR_SYM>, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, t,
                     (const double*)nullptr, ldt, (const double*)nullptr, (const double*)nullptr,
                     0, ore, oim, ldo, 0.0, (const double*)nullptr, 0, (const double*)nullptr,
                     (const double*)nullptr, 0, nt);
  return hipGetLastError();
}

hipError_t kick_phase(hipStream_t s, double* re, double* im, int ld, const double* x, int np,
                      double kappa) {
  hipLaunchKernelGGL(k_kick_phase, dim3(blocks_for((size_t)np * np)), dim3(256), 0, s, re, im,
                     ld, x, np, kappa);
  return hipGetLastError();
}

hipError_t scaled_identity(hipStream_t s, double* X, int np, int n, double c) {
  hipLaunchKernelGGL(k_scaled_identity, dim3(blocks_for((size_t)np * np)), dim3(256), 0, s, X,
                     np, n, c);
  return hipGetLastError();
}

hipError_t extrapolate(hipStream_t s, const double* x0, const double* x1, const double* x2,
                       double* out, size_t len) {
  if (len == 0) return hipSuccess;
  hipLaunchKernelGGL(k_extrapolate, dim3(blocks_for(len)), dim3(256), 0, s, x0, x1, x2, out, len);
  return hipGetLastError();
}

hipError_t two_minus(hipStream_t s, double* T, int np, int n) {
  hipLaunchKernelGGL(k_two_minus, dim3(blocks_for((size_t)np * np)), dim3(256), 0, s, T, np, n);
  return hipGetLastError();
}

hipError_t sp2_init(hipStream_t s, const double* T, double* X, int np, int n, double emax,
                    double emin) {
  hipLaunchKernelGGL(k_sp2_init, dim3(blocks_for((size_t)np * np)), dim3(256), 0, s, T, X, np,
                     n, emax, 1.0 / (emax - emin));
  return hipGetLastError();
}

hipError_t sp2_update(hipStream_t s, double* X, const double* X2, int np, int mode) {
  const size_t total = (size_t)np * np;
  hipLaunchKernelGGL(k_sp2_update, dim3(blocks_for(total)), dim3(256), 0, s, X, X2, total, mode);
  return hipGetLastError();
}

hipError_t real_to_wide(hipStream_t s, const double* R, int ldr, double* W, int np) {
  hipLaunchKernelGGL(k_real_to_wide, dim3(blocks_for((size_t)np * np)), dim3(256), 0, s, R, ldr,
                     W, np);
  return hipGetLastError();
}

hipError_t interleaved_to_wide(hipStream_t s, const double* Z, int n, double* W, int np) {
  hipLaunchKernelGGL(k_interleaved_to_wide, dim3(blocks_for((size_t)np * np)), dim3(256), 0, s,
                     Z, n, W, np);
  return hipGetLastError();
}

hipError_t wide_to_interleaved(hipStream_t s, const double* W, int np, double* Z, int n) {
  hipLaunchKernelGGL(k_wide_to_interleaved, dim3(blocks_for((size_t)n * n)), dim3(256), 0, s, W,
                     np, Z, n);
  return hipGetLastError();
}

hipError_t pad_copy(hipStream_t s, const double* src, int n, double* dst, int np) {
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks_for((size_t)n * n)), dim3(256), 0, s, src, n, dst,
                     np);
  return hipGetLastError();
}

hipError_t unpad_copy(hipStream_t s, const double* src, int np, double* dst, int n) {
  hipLaunchKernelGGL(k_unpad_copy, dim3(blocks_for((size_t)n * n)), dim3(256), 0, s, src, np,
                     dst, n);
  return hipGetLastError();
}

hipError_t trace(hipStream_t s, const double* X, int ld, int n, double* out) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(1024), 0, s, X, ld, n, out);
  return hipGetLastError();
}

hipError_t identity_residual(hipStream_t s, const double* T, int ld, int n, double* work,
                             double* out) {
  hipLaunchKernelGGL(k_row_identity_resid, dim3((n + 3) / 4), dim3(256), 0, s, T, ld, n, work);
  hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, work, n, out);
  return hipGetLastError();
}

hipError_t check_matrix(hipStream_t s, const double* M, int ld, int rows, int cols,
                        int symmetric, double* work, double* out) {
  if (rows < 1 || cols < 1 || ld < cols || (symmetric && rows != cols))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_row_check, dim3((rows + 3) / 4), dim3(256), 0, s, M, ld, rows, cols,
                     symmetric, work);
  hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, work, rows, out);
  return hipGetLastError();
}

hipError_t gershgorin(hipStream_t s, const double* T, int ld, int n, double* work_lo,
                      double* work_hi, double* out) {
  hipLaunchKernelGGL(k_row_gershgorin, dim3((n + 3) / 4), dim3(256), 0, s, T, ld, n, work_lo,
                     work_hi);
  hipLaunchKernelGGL(k_minmax, dim3(1), dim3(1024), 0, s, work_lo, work_hi, n, out);
  return hipGetLastError();
}

hipError_t sum_vector(hipStream_t s, const double* x, int n, double* out) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t anderson_mix(hipStream_t s, double* dq_in, const double* dq_out, double* hx,
                        double* hf, int na, int m, int count, int slot, double beta,
                        double* out_resid) {
  if (m < 1 || m > MAXH || count < 1 || count > m || slot < 0 || slot >= m)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_anderson, dim3(1), dim3(1024), 0, s, dq_in, dq_out, hx, hf, na, m, count,
                     slot, beta, out_resid);
  return hipGetLastError();
}

hipError_t energy_terms(hipStream_t s, const double* band_rows, int n, const double* dq,
                        const double* v_gamma, const double* pos, const double* E, int na,
                        double* out) {
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, s, band_rows, n, dq, v_gamma, pos, E, na,
                     out);
  return hipGetLastError();
}

hipError_t power_start(hipStream_t s, double* V, int ld, int n, int np, int ncols) {
  hipLaunchKernelGGL(k_power_start, dim3(blocks_for((size_t)np * ncols)), dim3(256), 0, s, V, ld,
                     n, np, ncols);
  return hipGetLastError();
}

hipError_t power_step(hipStream_t s, const double* W, double* V, int ld, int np, int ncols,
                      int half, double lo, double hi) {
  hipLaunchKernelGGL(k_power_step, dim3(ncols), dim3(1024), 0, s, W, V, ld, np, half, lo, hi);
  return hipGetLastError();
}

hipError_t rayleigh(hipStream_t s, const double* V, const double* W, const double* SV, int ld,
                    int np, int ncols, double* out) {
  hipLaunchKernelGGL(k_rayleigh, dim3(ncols), dim3(1024), 0, s, V, W, SV, ld, np, out);
  return hipGetLastError();
}

}  // namespace td
