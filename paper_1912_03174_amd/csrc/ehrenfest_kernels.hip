// Moving-nuclei (Ehrenfest) kernels: the two-centre model rebuild of S and
// H0 with their central-difference gradients (Sec. 2.3, Eq. 20), gamma and
// its analytic gradient, the non-adiabatic coupling D (Sec. 2.1, Eq. 14),
// the Ehrenfest force without velocity terms (Sec. 2.1, Eq. 15) and the
// velocity Verlet updates of the nuclei (Sec. 2.3).
#include "common.hpp"
#include "reduce.hpp"

namespace td {
namespace {

// Element (i, j) of the two-centre block of atoms a (species sa) -> b
// (species sb) with unit vector l from a to b and radial factor f;
// orbital index 0 = s, 1..3 = p_x, p_y, p_z.
__device__ inline double sk_elem(const double* sk, int nsp, int sa, int sb, int i, int j,
                                 const double* l, double f) {
  const double* ab = sk + (sa * nsp + sb) * 4;
  if (i == 0 && j == 0) return ab[0] * f;
  if (i == 0) return l[j - 1] * ab[1] * f;                       // s on a, p on b
  if (j == 0) return -l[i - 1] * sk[(sb * nsp + sa) * 4 + 1] * f; // p on a, s on b
  return (l[i - 1] * l[j - 1] * (ab[2] - ab[3]) + (i == j ? ab[3] : 0.0)) * f;
}

// Block of table `sk` between atoms a -> b displaced by d (bohr) into out[4][4].
__device__ inline void sk_block(const double* sk, const double* scale, int na, int nsp, int a,
                                int b, int sa, int sb, int oa, int ob, double decay,
                                const double* d, double out[4][4]) {
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double l[3] = {d[0] / r, d[1] / r, d[2] / r};
  const double f = exp(-r / decay) * scale[(size_t)a * na + b];
  for (int i = 0; i < oa; ++i)
    for (int j = 0; j < ob; ++j) out[i][j] = sk_elem(sk, nsp, sa, sb, i, j, l, f);
}

// One thread per ordered atom pair (a, b): S, H0 blocks and, for a != b,
// G[k] = (X(d + h e_k) - X(d - h e_k)) / 2h, d = R_b - R_a (the derivative
// with respect to the column atom b).
__global__ void k_model(ModelArgs m, const double* __restrict__ pos, double* __restrict__ S,
                        double* __restrict__ H0, double* __restrict__ GS,
                        double* __restrict__ GH, int np) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int na = m.na;
  if (idx >= (size_t)na * na) return;
  const int a = (int)(idx / na), b = (int)(idx % na);
  const int sa = m.species[a], sb = m.species[b];
  const int oa = m.norb[sa], ob = m.norb[sb];
  const int ra = m.orb_off[a], cb = m.orb_off[b];
  const size_t nn = (size_t)np * np;
  if (a == b) {
    for (int i = 0; i < oa; ++i)
      for (int j = 0; j < ob; ++j) {
        const size_t e = (size_t)(ra + i) * np + cb + j;
        S[e] = i == j ? 1.0 : 0.0;
        H0[e] = i == j ? m.onsite[sa * 2 + (i > 0 ? 1 : 0)] : 0.0;
        for (int k = 0; k < 3; ++k) {
          GS[k * nn + e] = 0.0;
          GH[k * nn + e] = 0.0;
        }
      }
    return;
  }
  const double d[3] = {pos[3 * b] - pos[3 * a], pos[3 * b + 1] - pos[3 * a + 1],
                       pos[3 * b + 2] - pos[3 * a + 2]};
  double blk[4][4], bp[4][4], bm[4][4];
  for (int t = 0; t < 2; ++t) {
    const double* sk = t ? m.sk_h : m.sk_s;
    const double* sc = t ? m.scale_h : m.scale_s;
    double* X = t ? H0 : S;
    double* G = t ? GH : GS;
    sk_block(sk, sc, na, m.nsp, a, b, sa, sb, oa, ob, m.decay, d, blk);
    for (int i = 0; i < oa; ++i)
      for (int j = 0; j < ob; ++j) X[(size_t)(ra + i) * np + cb + j] = blk[i][j];
    for (int k = 0; k < 3; ++k) {
      double dp[3] = {d[0], d[1], d[2]}, dm[3] = {d[0], d[1], d[2]};
      dp[k] += m.fd_step;
      dm[k] -= m.fd_step;
      sk_block(sk, sc, na, m.nsp, a, b, sa, sb, oa, ob, m.decay, dp, bp);
      sk_block(sk, sc, na, m.nsp, a, b, sa, sb, oa, ob, m.decay, dm, bm);
      for (int i = 0; i < oa; ++i)
        for (int j = 0; j < ob; ++j)
          G[k * nn + (size_t)(ra + i) * np + cb + j] = (bp[i][j] - bm[i][j]) / (2.0 * m.fd_step);
    }
  }
}

// gamma_AB = 1 / sqrt(r^2 + U^-2); dgamma[(A na + B) 3 + k] = d gamma_AB / d R_A,k.
__global__ void k_gamma(const double* __restrict__ pos, int na, double u,
                        double* __restrict__ gamma, double* __restrict__ dgamma) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)na * na) return;
  const int a = (int)(idx / na), b = (int)(idx % na);
  const double d[3] = {pos[3 * a] - pos[3 * b], pos[3 * a + 1] - pos[3 * b + 1],
                       pos[3 * a + 2] - pos[3 * b + 2]};
  const double q = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 1.0 / (u * u);
  gamma[idx] = 1.0 / sqrt(q);
  const double c = -1.0 / (q * sqrt(q));
  for (int k = 0; k < 3; ++k) dgamma[idx * 3 + k] = c * d[k];
}

// D[u][v] = sum_k vel[atom(v)][k] GS[k][u][v] on the n x n block (GS is zero
// where u and v share an atom).
__global__ void k_nac(const double* __restrict__ GS, const double* __restrict__ vel,
                      const int* __restrict__ atom_of, int n, int np, double* __restrict__ D) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int u = (int)(idx / n), v = (int)(idx % n);
  const size_t e = (size_t)u * np + v, nn = (size_t)np * np;
  const double* w = vel + 3 * atom_of[v];
  D[e] = w[0] * GS[e] + w[1] * GS[nn + e] + w[2] * GS[2 * nn + e];
}

// Wide X (np x 2np) += -i Z: Re X += Im Z, Im X -= Re Z.
__global__ void k_add_minus_i(double* __restrict__ X, const double* __restrict__ Z, int np) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int r = (int)(idx / np), c = (int)(idx % np);
  const size_t re = (size_t)r * 2 * np + c, im = re + np;
  const double zr = Z[re], zi = Z[im];
  X[re] += zi;
  X[im] -= zr;
}

// One block per atom A:
// F_A = 2 sum_{u in A, v} [Re rho_uv GH_uv + (1/2 Re rho_uv (v_u + v_v) - W_uv) GS_uv]
//       - dq_A sum_B dgamma_AB dq_B - dq_A E.
__global__ __launch_bounds__(1024) void k_forces(const double* __restrict__ rho, int ldr,
                                                 const double* __restrict__ W,
                                                 const double* __restrict__ GS,
                                                 const double* __restrict__ GH,
                                                 const double* __restrict__ vorb,
                                                 const int* __restrict__ orb_off,
                                                 const double* __restrict__ dq,
                                                 const double* __restrict__ dgamma,
                                                 const double* __restrict__ E, int na, int n,
                                                 int np, double* __restrict__ F) {
  __shared__ double sh[17];
  const int A = blockIdx.x;
  const size_t nn = (size_t)np * np;
  double acc[3] = {0.0, 0.0, 0.0};
  const int u0 = orb_off[A], u1 = orb_off[A + 1];
  for (int u = u0; u < u1; ++u) {
    const double vu = vorb[u];
    for (int v = threadIdx.x; v < n; v += 1024) {
      const size_t e = (size_t)u * np + v;
      const double r = rho[(size_t)u * ldr + v];
      const double ms = 0.5 * r * (vu + vorb[v]) - W[e];
      for (int k = 0; k < 3; ++k) acc[k] += r * GH[k * nn + e] + ms * GS[k * nn + e];
    }
  }
  double g[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < na; b += 1024)
    for (int k = 0; k < 3; ++k) g[k] += dgamma[((size_t)A * na + b) * 3 + k] * dq[b];
  for (int k = 0; k < 3; ++k) {
    const double s = block_sum_1024(acc[k], sh);
    const double t = block_sum_1024(g[k], sh);
    if (threadIdx.x == 0)
      F[3 * A + k] = 2.0 * s - dq[A] * t - (E ? dq[A] * E[k] : 0.0);
  }
}

// vel += scale dt F / M (per atom, 3 components).
__global__ void k_kick_nuclei(double* __restrict__ vel, const double* __restrict__ F,
                              const int* __restrict__ species, const double* __restrict__ mass,
                              int na, double h) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= 3 * na) return;
  vel[i] += h * F[i] / mass[species[i / 3]];
}

__global__ void k_drift(double* __restrict__ pos, const double* __restrict__ vel, int na,
                        double dt) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= 3 * na) return;
  pos[i] += dt * vel[i];
}

// out[0] = 1/2 sum M (vel + h F / M)^2 (the kinetic energy of vel advanced by h).
__global__ __launch_bounds__(1024) void k_kinetic(const double* __restrict__ vel,
                                                  const double* __restrict__ F,
                                                  const int* __restrict__ species,
                                                  const double* __restrict__ mass, int na,
                                                  double h, double* __restrict__ out) {
  __shared__ double sh[17];
  double acc = 0.0;
  for (int i = threadIdx.x; i < 3 * na; i += 1024) {
    const double m = mass[species[i / 3]];
    const double v = vel[i] + h * F[i] / m;
    acc += 0.5 * m * v * v;
  }
  acc = block_sum_1024(acc, sh);
  if (threadIdx.x == 0) out[0] = acc;
}

unsigned nblocks(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t model_build(hipStream_t s, const ModelArgs& m, const double* pos, double* S,
                       double* H0, double* GS, double* GH, int np) {
  hipLaunchKernelGGL(k_model, dim3(nblocks((size_t)m.na * m.na)), dim3(256), 0, s, m, pos, S, H0,
                     GS, GH, np);
  return hipGetLastError();
}

hipError_t gamma_build(hipStream_t s, const double* pos, int na, double u, double* gamma,
                       double* dgamma) {
  hipLaunchKernelGGL(k_gamma, dim3(nblocks((size_t)na * na)), dim3(256), 0, s, pos, na, u, gamma,
                     dgamma);
  return hipGetLastError();
}

hipError_t nac_build(hipStream_t s, const double* GS, const double* vel, const int* atom_of, int n,
                     int np, double* D) {
  hipLaunchKernelGGL(k_nac, dim3(nblocks((size_t)n * n)), dim3(256), 0, s, GS, vel, atom_of, n, np,
                     D);
  return hipGetLastError();
}

hipError_t add_minus_i(hipStream_t s, double* X, const double* Z, int np) {
  hipLaunchKernelGGL(k_add_minus_i, dim3(nblocks((size_t)np * np)), dim3(256), 0, s, X, Z, np);
  return hipGetLastError();
}

hipError_t ehrenfest_forces(hipStream_t s, const double* rho, int ldr, const double* W,
                            const double* GS, const double* GH, const double* vorb,
                            const int* orb_off, const double* dq, const double* dgamma,
                            const double* E, int na, int n, int np, double* F) {
  hipLaunchKernelGGL(k_forces, dim3(na), dim3(1024), 0, s, rho, ldr, W, GS, GH, vorb, orb_off, dq,
                     dgamma, E, na, n, np, F);
  return hipGetLastError();
}

hipError_t kick_nuclei(hipStream_t s, double* vel, const double* F, const int* species,
                       const double* mass, int na, double h) {
  hipLaunchKernelGGL(k_kick_nuclei, dim3(nblocks((size_t)3 * na)), dim3(256), 0, s, vel, F,
                     species, mass, na, h);
  return hipGetLastError();
}

hipError_t drift_nuclei(hipStream_t s, double* pos, const double* vel, int na, double dt) {
  hipLaunchKernelGGL(k_drift, dim3(nblocks((size_t)3 * na)), dim3(256), 0, s, pos, vel, na, dt);
  return hipGetLastError();
}

hipError_t kinetic_energy(hipStream_t s, const double* vel, const double* F, const int* species,
                          const double* mass, int na, double h, double* out) {
  hipLaunchKernelGGL(k_kinetic, dim3(1), dim3(1024), 0, s, vel, F, species, mass, na, h, out);
  return hipGetLastError();
}

}  // namespace td
