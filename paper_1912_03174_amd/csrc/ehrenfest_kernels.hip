// Moving-nuclei (Ehrenfest) kernels: the two-centre model rebuild of S and
// H0 with their central-difference gradients (Sec. 2.3, Eq. 20), gamma and
// its analytic gradient, the non-adiabatic coupling D (Sec. 2.1, Eq. 14),
// the Ehrenfest force without velocity terms (Sec. 2.1, Eq. 15) and the
// velocity Verlet updates of the nuclei (Sec. 2.3).
#include "common.hpp"
#include "reduce.hpp"

namespace td {
namespace {

// Component c (1..3) of the unit vector l, chosen by selects (no indexed
// private array).
__device__ inline double lcomp(const double* l, int c) {
  return c == 1 ? l[0] : (c == 2 ? l[1] : l[2]);
}

// Element (i, j) of the two-centre block of atoms a (species sa) -> b
// (species sb) with unit vector l from a to b and radial factor f;
// orbital index 0 = s, 1..3 = p_x, p_y, p_z.
__device__ inline double sk_elem(const double* sk, int nsp, int sa, int sb, int i, int j,
                                 const double* l, double f) {
  const double* ab = sk + (sa * nsp + sb) * 4;
  if (i == 0 && j == 0) return ab[0] * f;
  if (i == 0) return lcomp(l, j) * ab[1] * f;                       // s on a, p on b
  if (j == 0) return -lcomp(l, i) * sk[(sb * nsp + sa) * 4 + 1] * f; // p on a, s on b
  return (lcomp(l, i) * lcomp(l, j) * (ab[2] - ab[3]) + (i == j ? ab[3] : 0.0)) * f;
}

// Geometry of the pair a -> b displaced by d (bohr): unit vector l and the
// radial factors of the S and H0 tables.
struct PairGeom {
  double l[3];
  double fs, fh;
};

__device__ inline PairGeom pair_geom(const ModelArgs& m, size_t ab, const double* d) {
  PairGeom g;
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  g.l[0] = d[0] / r;
  g.l[1] = d[1] / r;
  g.l[2] = d[2] / r;
  const double e = exp(-r / m.decay);
  g.fs = e * m.scale_s[ab];
  g.fh = e * m.scale_h[ab];
  return g;
}

// One thread per (row atom a, column orbital v), consecutive threads along
// v: orbital v is orbital j of atom b; the thread writes column v of the
// a -> b block (rows i < norb(a)) of S, H0 and, for a != b,
// G[k] = (X(d + h e_k) - X(d - h e_k)) / 2h, d = R_b - R_a (the derivative
// with respect to the column atom b). Every row store is coalesced over v,
// and the pair geometry is evaluated once per displacement for the column.
__global__ void k_model(ModelArgs m, const double* __restrict__ pos, double* __restrict__ S,
                        double* __restrict__ H0, double* __restrict__ GS,
                        double* __restrict__ GH, int n, int np) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)m.na * n) return;
  const int a = (int)(idx / n), v = (int)(idx % n);
  const int b = m.atom_of[v];
  const int j = v - m.orb_off[b];
  const int sa = m.species[a], sb = m.species[b];
  const int oa = m.norb[sa], ra = m.orb_off[a];
  const size_t nn = (size_t)np * np;
  const size_t e0 = (size_t)ra * np + v;
  if (a == b) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i >= oa) break;
      const size_t e = e0 + (size_t)i * np;
      S[e] = i == j ? 1.0 : 0.0;
      H0[e] = i == j ? m.onsite[sa * 2 + (i > 0 ? 1 : 0)] : 0.0;
      for (int k = 0; k < 3; ++k) {
        GS[k * nn + e] = 0.0;
        GH[k * nn + e] = 0.0;
      }
    }
    return;
  }
  const size_t ab = (size_t)a * m.na + b;
  const double d[3] = {pos[3 * b] - pos[3 * a], pos[3 * b + 1] - pos[3 * a + 1],
                       pos[3 * b + 2] - pos[3 * a + 2]};
  {
    const PairGeom g = pair_geom(m, ab, d);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i >= oa) break;
      const size_t e = e0 + (size_t)i * np;
      S[e] = sk_elem(m.sk_s, m.nsp, sa, sb, i, j, g.l, g.fs);
      H0[e] = sk_elem(m.sk_h, m.nsp, sa, sb, i, j, g.l, g.fh);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double dp[3] = {d[0], d[1], d[2]}, dm[3] = {d[0], d[1], d[2]};
    dp[k] += m.fd_step;
    dm[k] -= m.fd_step;
    const PairGeom gp = pair_geom(m, ab, dp), gm = pair_geom(m, ab, dm);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i >= oa) break;
      const size_t e = k * nn + e0 + (size_t)i * np;
      const double sp = sk_elem(m.sk_s, m.nsp, sa, sb, i, j, gp.l, gp.fs);
      const double sm = sk_elem(m.sk_s, m.nsp, sa, sb, i, j, gm.l, gm.fs);
      const double hp = sk_elem(m.sk_h, m.nsp, sa, sb, i, j, gp.l, gp.fh);
      const double hm = sk_elem(m.sk_h, m.nsp, sa, sb, i, j, gm.l, gm.fh);
      GS[e] = (sp - sm) / (2.0 * m.fd_step);
      GH[e] = (hp - hm) / (2.0 * m.fd_step);
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
  hipLaunchKernelGGL(k_model, dim3(nblocks((size_t)m.na * m.n)), dim3(256), 0, s, m, pos, S, H0,
                     GS, GH, m.n, np);
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

// One wave per atom A, its lanes over the other atoms B: the pair term
// w = rep_a[s_A, s_B] exp(-r / decay), its force on A
// (w / decay) (R_A - R_B) / r (Sec. 2.1, the -grad_A E_rep of Eq. 15) and
// half of w (each pair is seen from both atoms), summed by a fixed-order
// wave reduction.
__global__ __launch_bounds__(256) void k_repulsion(const double* __restrict__ pos,
                                                   const int* __restrict__ species,
                                                   const double* __restrict__ rep_a, int nsp,
                                                   double decay, int na, double* F,
                                                   double* __restrict__ e_atom) {
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (a >= na) return;
  const double xa = pos[3 * a], ya = pos[3 * a + 1], za = pos[3 * a + 2];
  const double* row = rep_a + (size_t)species[a] * nsp;
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
  for (int b = l; b < na; b += 64) {
    if (b == a) continue;
    const double dx = xa - pos[3 * b], dy = ya - pos[3 * b + 1], dz = za - pos[3 * b + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double w = row[species[b]] * exp(-r / decay);
    const double g = w / (decay * r);
    fx += g * dx;
    fy += g * dy;
    fz += g * dz;
    e += 0.5 * w;
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  e = wave_sum(e);
  if (l == 0) {
    if (F) {
      F[3 * a] += fx;
      F[3 * a + 1] += fy;
      F[3 * a + 2] += fz;
    }
    e_atom[a] = e;
  }
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

hipError_t repulsion(hipStream_t s, const double* pos, const int* species, const double* rep_a,
                     int nsp, double decay, int na, double* F, double* e_atom, double* energy) {
  if (na <= 0 || nsp <= 0 || !(decay > 0.0) || !rep_a || !e_atom || !energy)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_repulsion, dim3((na + 3) / 4), dim3(256), 0, s, pos, species, rep_a, nsp,
                     decay, na, F, e_atom);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return sum_vector(s, e_atom, na, energy);
}

hipError_t kinetic_energy(hipStream_t s, const double* vel, const double* F, const int* species,
                          const double* mass, int na, double h, double* out) {
  hipLaunchKernelGGL(k_kinetic, dim3(1), dim3(1024), 0, s, vel, F, species, mass, na, h, out);
  return hipGetLastError();
}

}  // namespace td
