// On-site corrections of the SCC Hamiltonian (Sec. 3.2): the
// fully-localised limit of DFTB+U (Eqs. 21-23) and pseudo-SIC
// (Eqs. 24-25) on the dual block populations of each shell.
#include "common.hpp"

namespace td {
namespace {

constexpr int MAXB = kPlusUMaxShell;   // orbitals per shell
constexpr int BS = MAXB * MAXB;        // stride of one shell's block

// One workgroup per shell b of m <= MB orbitals starting at o:
// A_uv = sum_k Re rho[o+u][k] S[o+v][k]; n = (A + A^T) / 2 is the block of
// 1/2 (Re(rho) S + S Re(rho)) (Eq. 23; rho and S symmetric in their real
// parts). Writes n as a MAXB x MAXB block and the shell's correction
// energy (Eq. 21 or 24, spin-summed density).
template <int MB>
__global__ __launch_bounds__(256) void k_block_pop(const double* __restrict__ rho, int ldr,
                                                   const double* __restrict__ S, int lds,
                                                   const int* __restrict__ sh_off,
                                                   const double* __restrict__ sh_u, int mode,
                                                   int ncols, double* __restrict__ n_out,
                                                   double* __restrict__ e_sh) {
  const int b = blockIdx.x;
  const int o = sh_off[b], m = sh_off[b + 1] - o;
  double acc[MB][MB];
#pragma unroll
  for (int u = 0; u < MB; ++u)
#pragma unroll
    for (int v = 0; v < MB; ++v) acc[u][v] = 0.0;
  for (int k = threadIdx.x; k < ncols; k += 256) {
    double r[MB], s[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      r[u] = u < m ? rho[(size_t)(o + u) * ldr + k] : 0.0;
      s[u] = u < m ? S[(size_t)(o + u) * lds + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < MB; ++u)
#pragma unroll
      for (int v = 0; v < MB; ++v) acc[u][v] += r[u] * s[v];
  }
  __shared__ double red[4][MB * MB];
  __shared__ double nb[MB * MB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < MB; ++u)
#pragma unroll
    for (int v = 0; v < MB; ++v) {
      double x = acc[u][v];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0) red[wave][u * MB + v] = x;
    }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < MB * MB) {
    const int u = t / MB, v = t % MB;
    double n = 0.0;
    if (u < m && v < m) {
      const double a_uv = red[0][u * MB + v] + red[1][u * MB + v] + red[2][u * MB + v] +
                          red[3][u * MB + v];
      const double a_vu = red[0][v * MB + u] + red[1][v * MB + u] + red[2][v * MB + u] +
                          red[3][v * MB + u];
      n = 0.5 * (a_uv + a_vu);
    }
    nb[t] = n;
  }
  __syncthreads();
  if (t < BS) {
    const int u = t / MAXB, v = t % MAXB;
    n_out[(size_t)b * BS + t] = (u < MB && v < MB) ? nb[u * MB + v] : 0.0;
  }
  if (t == 0 && e_sh) {
    double sq = 0.0, tr = 0.0;
    for (int u = 0; u < m; ++u) {
      tr += nb[u * MB + u];
      for (int v = 0; v < m; ++v) sq += nb[u * MB + v] * nb[u * MB + v];
    }
    const double U = sh_u[b];
    e_sh[b] = -0.25 * U * sq + (mode == 1 ? 0.5 * U * tr : 0.0);
  }
}

// V_b = d(dE)/d(n_b): -(U/2)(n - 1) (FLL, Eq. 22) or -(U/2) n (pSIC, Eq. 25).
__global__ void k_plus_u_potential(const double* __restrict__ n, const int* __restrict__ sh_off,
                                   const double* __restrict__ sh_u, int nsh, int mode,
                                   double* __restrict__ V) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nsh * BS) return;
  const int b = idx / BS, r = idx % BS, u = r / MAXB, v = r % MAXB;
  const int m = sh_off[b + 1] - sh_off[b];
  double x = 0.0;
  if (u < m && v < m) {
    const double d = (mode == 1 && u == v) ? 1.0 : 0.0;
    x = -0.5 * sh_u[b] * (n[idx] - d);
  }
  V[idx] = x;
}

// Change of the potentials from the reference state (split products): the
// populations are linear in rho, so for rho = rho_ref + delta - c rho_ref
// (delta's populations n, the reference's nref, c the trace correction)
// both modes give dV = -(U/2) (n - c nref).
__global__ void k_plus_u_delta_potential(const double* __restrict__ n,
                                         const double* __restrict__ nref,
                                         const double* __restrict__ cs,
                                         const int* __restrict__ sh_off,
                                         const double* __restrict__ sh_u, int nsh,
                                         double* __restrict__ V) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nsh * BS) return;
  const int b = idx / BS, r = idx % BS, u = r / MAXB, v = r % MAXB;
  const int m = sh_off[b + 1] - sh_off[b];
  V[idx] = (u < m && v < m) ? -0.5 * sh_u[b] * (n[idx] - cs[0] * nref[idx]) : 0.0;
}

// H = H0 + 1/2 S_rc (v_r + v_c) (Eqs. 6-7) + 1/2 (S V + V S)_rc with V the
// block-diagonal shell potentials: (S V)_rc sums over the shell of c,
// (V S)_rc over the shell of r. sh_of[u] = shell of orbital u (-1 in the
// padding). H0 may be null (the change of H for split products).
__global__ void k_assemble_h_u(const double* __restrict__ H0, const double* __restrict__ S,
                               const double* __restrict__ vorb, const int* __restrict__ sh_of,
                               const int* __restrict__ sh_off, const double* __restrict__ V,
                               double* __restrict__ H, int np) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  double h = (H0 ? H0[idx] : 0.0) + 0.5 * S[idx] * (vorb[r] + vorb[c]);
  double corr = 0.0;
  const int bc = sh_of[c];
  if (bc >= 0) {
    const int oc = sh_off[bc], mc = sh_off[bc + 1] - oc;
    const double* Vb = V + (size_t)bc * BS;
    for (int k = 0; k < mc; ++k) corr += S[(size_t)r * np + oc + k] * Vb[k * MAXB + (c - oc)];
  }
  const int br = sh_of[r];
  if (br >= 0) {
    const int orr = sh_off[br], mr = sh_off[br + 1] - orr;
    const double* Vb = V + (size_t)br * BS;
    for (int k = 0; k < mr; ++k) corr += Vb[(r - orr) * MAXB + k] * S[(size_t)(orr + k) * np + c];
  }
  H[idx] = h + 0.5 * corr;
}

inline unsigned blocks_of(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t block_populations(hipStream_t s, const double* rho, int ldr, const double* S, int lds,
                             const int* sh_off, const double* sh_u, int nsh, int max_shell,
                             int mode, int ncols, double* n_out, double* e_sh) {
  if (nsh <= 0) return hipSuccess;
  if (max_shell <= 4) {
    hipLaunchKernelGGL(k_block_pop<4>, dim3(nsh), dim3(256), 0, s, rho, ldr, S, lds, sh_off, sh_u,
                       mode, ncols, n_out, e_sh);
  } else if (max_shell <= MAXB) {
    hipLaunchKernelGGL(k_block_pop<MAXB>, dim3(nsh), dim3(256), 0, s, rho, ldr, S, lds, sh_off,
                       sh_u, mode, ncols, n_out, e_sh);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t plus_u_potential(hipStream_t s, const double* n, const int* sh_off, const double* sh_u,
                            int nsh, int mode, double* V) {
  if (nsh <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plus_u_potential, dim3(blocks_of((size_t)nsh * BS)), dim3(256), 0, s, n,
                     sh_off, sh_u, nsh, mode, V);
  return hipGetLastError();
}

hipError_t plus_u_delta_potential(hipStream_t s, const double* n, const double* nref,
                                  const double* cs, const int* sh_off, const double* sh_u,
                                  int nsh, double* V) {
  if (nsh <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plus_u_delta_potential, dim3(blocks_of((size_t)nsh * BS)), dim3(256), 0, s,
                     n, nref, cs, sh_off, sh_u, nsh, V);
  return hipGetLastError();
}

hipError_t assemble_h_plus_u(hipStream_t s, const double* H0, const double* S, const double* vorb,
                             const int* sh_of, const int* sh_off, const double* V, double* H,
                             int np) {
  hipLaunchKernelGGL(k_assemble_h_u, dim3(blocks_of((size_t)np * np)), dim3(256), 0, s, H0, S,
                     vorb, sh_of, sh_off, V, H, np);
  return hipGetLastError();
}

}  // namespace td
