// Batched step kernels: the O(n^2) and O(n_atoms^2) work of the density
// step (Mulliken charges, Sec. 2.1 Eq. 5; SCC potential and Hamiltonian,
// Eqs. 6-7; leapfrog update, Sec. 2.3 Eq. 19) for many trajectories of
// different sizes in one launch each. A launch walks a table of work items
// (member, row / atom / tile pair); each item is computed exactly as the
// one-trajectory kernel computes it, so a member of a batch follows its
// solo trajectory bit for bit.
#include "common.hpp"
#include "reduce.hpp"

namespace td {
namespace {

constexpr int TS = 32;
constexpr int TLD = TS + 1;

// One wave per row, 4 rows per block (as the one-trajectory row dot).
__global__ __launch_bounds__(256) void k_b_rowdot(const BatchMember* __restrict__ mem,
                                                  const BatchItem* __restrict__ rows, int nrows,
                                                  int cur) {
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (item >= nrows) return;
  const BatchItem it = rows[item];
  const BatchMember& M = mem[it.m];
  const int np = M.np;
  const double2* x = reinterpret_cast<const double2*>(M.R[cur] + (size_t)it.r * 2 * np);
  const double2* y = reinterpret_cast<const double2*>(M.S + (size_t)it.r * np);
  double acc = 0.0;
  // the one-trajectory row dot runs over all np columns; the terms from
  // kw on are products with zero density entries and leave every partial
  // sum unchanged
  for (int c = l; c < M.kw / 2; c += WAVE) {
    const double2 a = x[c], b = y[c];
    acc = fma(a.x, b.x, acc);
    acc = fma(a.y, b.y, acc);
  }
  acc = wave_sum(acc);
  if (l == 0) M.q_orb[it.r] = acc;
}

// One 1024-thread block per member.
__global__ __launch_bounds__(1024) void k_b_charges(const BatchMember* __restrict__ mem,
                                                    const int* __restrict__ kstep,
                                                    double* __restrict__ dip, int cap) {
  __shared__ double sh[17];
  const BatchMember& M = mem[blockIdx.x];
  const int na = M.na;
  const int* off = M.orb_off;
  double mx = 0.0, my = 0.0, mz = 0.0;
  for (int a = threadIdx.x; a < na; a += 1024) {
    double q = 0.0;
    for (int u = off[a]; u < off[a + 1]; ++u) q += M.q_orb[u];
    const double d = q - M.q0[a];
    M.dq[a] = d;
    mx -= d * M.pos[3 * a + 0];
    my -= d * M.pos[3 * a + 1];
    mz -= d * M.pos[3 * a + 2];
  }
  mx = block_sum_1024(mx, sh);
  my = block_sum_1024(my, sh);
  mz = block_sum_1024(mz, sh);
  if (threadIdx.x == 0) {
    double* mu = dip + ((size_t)blockIdx.x * cap + *kstep) * 3;
    mu[0] = mx;
    mu[1] = my;
    mu[2] = mz;
  }
}

// One wave per atom.
__global__ __launch_bounds__(256) void k_b_potential(const BatchMember* __restrict__ mem,
                                                     const BatchItem* __restrict__ atoms,
                                                     int natoms, const double* __restrict__ field,
                                                     const int* __restrict__ kstep) {
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (item >= natoms) return;
  const BatchItem it = atoms[item];
  const BatchMember& M = mem[it.m];
  const int a = it.r, na = M.na;
  const double* g = M.gamma + (size_t)a * na;
  double acc = 0.0;
  for (int c = l; c < na; c += WAVE) acc = fma(g[c], M.dq[c], acc);
  acc = wave_sum(acc);
  const double* E = field + 3 * (size_t)(*kstep);
  acc += M.pos[3 * a] * E[0] + M.pos[3 * a + 1] * E[1] + M.pos[3 * a + 2] * E[2];
  if (l == 0) M.v[a] = acc;
  for (int u = M.orb_off[a] + l; u < M.orb_off[a + 1]; u += WAVE) M.vorb[u] = acc;
}

// One wave per row: H = H0 + 1/2 S o (v_u + v_v), two columns per lane step.
__global__ __launch_bounds__(256) void k_b_assemble(const BatchMember* __restrict__ mem,
                                                    const BatchItem* __restrict__ rows,
                                                    int nrows) {
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (item >= nrows) return;
  const BatchItem it = rows[item];
  const BatchMember& M = mem[it.m];
  const int np = M.np;
  const size_t base2 = (size_t)it.r * np / 2;
  const double* vorb = M.vorb;
  const double vr = vorb[it.r];
  for (int c2 = l; c2 < M.hw / 2; c2 += WAVE) {
    const double2 h0 = reinterpret_cast<const double2*>(M.H0)[base2 + c2];
    const double2 s = reinterpret_cast<const double2*>(M.S)[base2 + c2];
    const int c = 2 * c2;
    double2 out;
    out.x = h0.x + 0.5 * s.x * (vr + vorb[c]);
    out.y = h0.y + 0.5 * s.y * (vr + vorb[c + 1]);
    reinterpret_cast<double2*>(M.H)[base2 + c2] = out;
  }
}

// Leapfrog on the tile pair (bi, bj), (bj, bi): out = base + f rhodot with
// Re rhodot = Xim + Xim^T, Im rhodot = Xre^T - Xre (as the one-trajectory
// pair kernel). base may equal out (in place).
__global__ __launch_bounds__(256) void k_b_leapfrog(const BatchMember* __restrict__ mem,
                                                    const BatchPair* __restrict__ pairs, int base,
                                                    int outb, double f) {
  const BatchPair it = pairs[blockIdx.x];
  const BatchMember& M = mem[it.m];
  const int np = M.np, ld = 2 * np;
  const double* xre = M.X;
  const double* xim = M.X + np;
  const double* bre = M.R[base];
  const double* bim = M.R[base] + np;
  double* ore = M.R[outb];
  double* oim = M.R[outb] + np;
  const int bi = it.bi, bj = it.bj;
  __shared__ double sre[2][TS][TLD];
  __shared__ double sim[2][TS][TLD];
  const int t = threadIdx.x;
  const int tr = t >> 3, tc = (t & 7) * 4;
  const bool diag = (bi == bj);
  const int nt = diag ? 1 : 2;
  // every read (both X tiles and rho_{n-1}) before the first write: the
  // update is in place, so the compiler could not reorder them itself
  double2 xr[2][2], xi[2][2], br[2][2], bm[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p < nt) {
      const int ti = p ? bj : bi, tj = p ? bi : bj;
      const size_t g = (size_t)(ti * TS + tr) * ld + tj * TS + tc;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        xr[p][h] = *reinterpret_cast<const double2*>(xre + g + 2 * h);
        xi[p][h] = *reinterpret_cast<const double2*>(xim + g + 2 * h);
        br[p][h] = *reinterpret_cast<const double2*>(bre + g + 2 * h);
        bm[p][h] = *reinterpret_cast<const double2*>(bim + g + 2 * h);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p < nt) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        sre[p][tr][tc + 2 * h] = xr[p][h].x;
        sre[p][tr][tc + 2 * h + 1] = xr[p][h].y;
        sim[p][tr][tc + 2 * h] = xi[p][h].x;
        sim[p][tr][tc + 2 * h + 1] = xi[p][h].y;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p < nt) {
      const int ti = p ? bj : bi, tj = p ? bi : bj;
      const int q = diag ? 0 : (p ^ 1);
      const size_t go = (size_t)(ti * TS + tr) * ld + tj * TS + tc;
      double r[4], m[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int cc = tc + c;
        const double are = sre[p][tr][cc], aret = sre[q][cc][tr];
        const double aim = sim[p][tr][cc], aimt = sim[q][cc][tr];
        const double dre = aim + aimt;
        const double dim = aret - are;
        const double b_re = (c & 1) ? br[p][c >> 1].y : br[p][c >> 1].x;
        const double b_im = (c & 1) ? bm[p][c >> 1].y : bm[p][c >> 1].x;
        r[c] = b_re + f * dre;
        m[c] = b_im + f * dim;
      }
      *reinterpret_cast<double2*>(ore + go) = make_double2(r[0], r[1]);
      *reinterpret_cast<double2*>(ore + go + 2) = make_double2(r[2], r[3]);
      *reinterpret_cast<double2*>(oim + go) = make_double2(m[0], m[1]);
      *reinterpret_cast<double2*>(oim + go + 2) = make_double2(m[2], m[3]);
    }
  }
}

__global__ void k_b_tick(int* kstep, int reset) {
  if (threadIdx.x == 0) *kstep = reset ? 0 : *kstep + 1;
}

}  // namespace

hipError_t batch_rowdot(hipStream_t s, const BatchMember* mem, const BatchItem* rows, int nrows,
                        int cur) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_rowdot, dim3((nrows + 3) / 4), dim3(256), 0, s, mem, rows, nrows, cur);
  return hipGetLastError();
}

hipError_t batch_charges(hipStream_t s, const BatchMember* mem, int nm, const int* kstep,
                         double* dip, int cap) {
  if (nm <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_charges, dim3(nm), dim3(1024), 0, s, mem, kstep, dip, cap);
  return hipGetLastError();
}

hipError_t batch_potential(hipStream_t s, const BatchMember* mem, const BatchItem* atoms,
                           int natoms, const double* field, const int* kstep) {
  if (natoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_potential, dim3((natoms + 3) / 4), dim3(256), 0, s, mem, atoms, natoms,
                     field, kstep);
  return hipGetLastError();
}

hipError_t batch_assemble(hipStream_t s, const BatchMember* mem, const BatchItem* rows,
                          int nrows) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_assemble, dim3((nrows + 3) / 4), dim3(256), 0, s, mem, rows, nrows);
  return hipGetLastError();
}

hipError_t batch_leapfrog(hipStream_t s, const BatchMember* mem, const BatchPair* pairs,
                          int npairs, int base, int out, double f) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_leapfrog, dim3(npairs), dim3(256), 0, s, mem, pairs, base, out, f);
  return hipGetLastError();
}

hipError_t batch_tick(hipStream_t s, int* kstep, int reset) {
  hipLaunchKernelGGL(k_b_tick, dim3(1), dim3(64), 0, s, kstep, reset);
  return hipGetLastError();
}

}  // namespace td
