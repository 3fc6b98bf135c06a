// Shared declarations of the TD-DFTB HIP library (device launchers and
// host helpers). Every launcher enqueues work on the given stream and
// returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace td {

// Macro tile of the FP64 matrix-core product. Matrix dimensions handed to
// the product kernels are multiples of it; the library pads every matrix
// to a multiple of kPad with zeros.
constexpr int kGemmTile = 128;
constexpr int kPad = 128;
constexpr int kPlusUMaxShell = 7;   // orbitals per shell of the on-site corrections

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------- products
// C[m x n] = alpha * A[m x k] B[k x n] + beta * Cin, row-major, leading
// dimensions in elements; m, n multiples of kGemmTile, k multiple of 16.
// `tag` only selects a separately named kernel instance (so profilers
// separate the two products of a step): 0 generic, 1 S^-1 H, 2 A rho.
// C (n x n) = A B for a product known to be symmetric in exact arithmetic:
// the 64-wide tiles on and above the diagonal are computed, the ones below
// are copied from their transposes. n a multiple of 64, k of 16.
hipError_t dgemm_symmetric(hipStream_t s, int n, int k, const double* A, int lda,
                           const double* B, int ldb, double* C, int ldc);
hipError_t dgemm(hipStream_t s, int tag, int m, int n, int k, double alpha,
                 const double* A, int lda, const double* B, int ldb, double beta,
                 const double* Cin, int ldcin, double* C, int ldc);

// One product of a grouped launch: C = A B with A [m x K], B [K x n] and
// m, n multiples of the launch's tile, K a multiple of 16. tile0 is the
// index of the problem's first tile in the launch (problems in ascending
// tile0, tile0 of the first = 0).
struct GemmProblem {
  const double* A;
  const double* B;
  double* C;
  int lda, ldb, ldc, K;
  int tiles_m, tiles_n, tile0;
  int upper;   // 1: only the tiles on or above the diagonal (square, symmetric C)
};

// All problems of `probs` (device array, nprob entries, ntiles tiles in
// total) in one launch with tile x tile macro tiles (tile = 128 or 64).
// Every output element is accumulated in the same order as by dgemm, so
// both give bitwise identical results.
hipError_t dgemm_grouped(hipStream_t s, int tile, const GemmProblem* probs, int nprob,
                         int ntiles);
// The second half of dgemm_symmetric for a C whose 64-wide tiles on and
// above the diagonal are computed (upper problems of a 64-tile grouped
// launch): the tiles below from their transposes.
hipError_t symmetric_mirror(hipStream_t s, double* C, int ldc, int n);

// ---------------------------------------------------------------- batches
// Device buffers of one trajectory of a batch (layouts as for one
// trajectory: np x np real, np x 2np wide planar complex).
struct BatchMember {
  const double* S;
  const double* H0;
  double* H;
  double* A;
  double* X;
  double* R[2];          // the two density buffers
  const double* gamma;
  const double* pos;
  const double* q0;
  const int* orb_off;
  double* q_orb;
  double* dq;
  double* v;
  double* vorb;
  int np, na;
  int kw;   // columns of the Mulliken row dots: round_up(n, 16); beyond, rho is zero
  int hw;   // columns of H assembled: those the S^-1 H product reads (its tile span)
};
struct BatchItem {        // row (or atom) r of member m
  int m, r;
};
struct BatchPair {        // 32 x 32 tiles (bi, bj) and (bj, bi) of member m, bi <= bj
  int m, bi, bj, pad_;
};

// The step kernels of one trajectory applied to every member of a batch in
// one launch each, with the same arithmetic in the same order (bitwise equal
// to the one-trajectory kernels). `cur` / `base` / `out` index R[].
// q_orb[r] = sum_c Re R[cur][r, c] S[r, c] for each listed row.
hipError_t batch_rowdot(hipStream_t s, const BatchMember* mem, const BatchItem* rows, int nrows,
                        int cur);
// dq and the dipole of each member; dipole -> dip[(m * cap + *kstep) * 3].
hipError_t batch_charges(hipStream_t s, const BatchMember* mem, int nm, const int* kstep,
                         double* dip, int cap);
// v and vorb of each listed atom with the field field[3 * *kstep].
hipError_t batch_potential(hipStream_t s, const BatchMember* mem, const BatchItem* atoms,
                           int natoms, const double* field, const int* kstep);
// H rows of each listed row.
hipError_t batch_assemble(hipStream_t s, const BatchMember* mem, const BatchItem* rows, int nrows);
// R[out] = R[base] + f rhodot(X) on each listed tile pair.
hipError_t batch_leapfrog(hipStream_t s, const BatchMember* mem, const BatchPair* pairs, int npairs,
                          int base, int out, double f);
// *kstep += 1, or = 0 (plain kernels, so they can be captured in a graph).
hipError_t batch_tick(hipStream_t s, int* kstep, int reset);

// ---------------------------------------------------------------- moving nuclei
// Two-centre model on the device (species-indexed tables, see td_model).
struct ModelArgs {
  const int* species;      // [na]
  const int* norb;         // [nsp]: 1 or 4
  const int* orb_off;      // [na + 1]
  const int* atom_of;      // [n]: atom of each orbital
  const double* sk_s;      // [nsp * nsp * 4]
  const double* sk_h;
  const double* scale_s;   // [na * na]
  const double* scale_h;
  const double* onsite;    // [nsp * 2]
  int na, nsp, n;
  double decay;            // bohr
  double fd_step;          // central-difference step (bohr)
};
// S, H0 (np x np, n x n block written) and their column-atom gradients
// GS, GH (3 consecutive np x np matrices each) at positions pos [na * 3].
hipError_t model_build(hipStream_t s, const ModelArgs& m, const double* pos, double* S,
                       double* H0, double* GS, double* GH, int np);
// gamma [na x na] and dgamma [na x na x 3] (d gamma_AB / d R_A).
hipError_t gamma_build(hipStream_t s, const double* pos, int na, double u, double* gamma,
                       double* dgamma);
// D = sum_k vel[atom(v)][k] GS[k] on the n x n block of the np x np D.
hipError_t nac_build(hipStream_t s, const double* GS, const double* vel, const int* atom_of,
                     int n, int np, double* D);
// Forces F [na x 3] (Ehrenfest, without velocity terms).
hipError_t ehrenfest_forces(hipStream_t s, const double* rho, int ldr, const double* W,
                            const double* GS, const double* GH, const double* vorb,
                            const int* orb_off, const double* dq, const double* dgamma,
                            const double* E, int na, int n, int np, double* F);
// vel += h F / M; pos += dt vel; out[0] = kinetic energy of vel + h F / M.
hipError_t kick_nuclei(hipStream_t s, double* vel, const double* F, const int* species,
                       const double* mass, int na, double h);
hipError_t drift_nuclei(hipStream_t s, double* pos, const double* vel, int na, double dt);
hipError_t kinetic_energy(hipStream_t s, const double* vel, const double* F, const int* species,
                          const double* mass, int na, double h, double* out);
// Pair repulsion E_rep = sum_{A<B} rep_a[s_A, s_B] exp(-r_AB / decay): adds
// -grad_A E_rep to F (if not null) and writes E_rep to *energy, summed in a
// fixed order from the per-atom halves in e_atom [na].
hipError_t repulsion(hipStream_t s, const double* pos, const int* species, const double* rep_a,
                     int nsp, double decay, int na, double* F, double* e_atom, double* energy);

// ---------------------------------------------------------------- O(n^2) kernels
// out[r] = sum_c X[r, c] * Y[r, c] for r < rows (cols multiple of 2).
hipError_t rowdot(hipStream_t s, const double* X, int ldx, const double* Y, int ldy,
                  double* out, int rows, int cols);

// dq[a] = sum_{u in a} q_orb[u] - q0[a]; mu = -sum_a dq[a] R_a -> mu_out[3];
// electrons (sum of q_orb) -> ne_out (may be null).
hipError_t charges_dipole(hipStream_t s, const double* q_orb, const int* orb_off,
                          const double* q0, const double* pos, int na, double* dq,
                          double* mu_out, double* ne_out);

// v[a] = sum_c gamma[a, c] dq[c] + R_a . E (E may be null);
// vorb[u] = v[atom(u)] - v_ref[atom(u)] (v_ref may be null).
hipError_t potential(hipStream_t s, const double* gamma, const double* dq,
                     const double* pos, const double* E, const int* orb_off, int na,
                     double* v, double* vorb, const double* v_ref = nullptr);

// Split precision charges: q_u = q_delta[u] + (1 - c) q_ref[u] with the trace
// correction c = (sum(q_delta + q_ref) - n_elec) / n_elec -> c_out[0];
// dq, dipole as charges_dipole.
hipError_t charges_dipole_split(hipStream_t s, const double* q_delta, const double* q_ref,
                                const int* orb_off, const double* q0, const double* pos, int na,
                                double n_elec, double* dq, double* mu_out, double* c_out);
// Real block of a wide matrix += sign * R (np x np).
hipError_t wide_add_real(hipStream_t s, double* W, const double* R, int np, double sign);
hipError_t vec_add(hipStream_t s, const double* a, const double* b, double* out, int n);

// H = H0 + 1/2 S o (vorb_u + vorb_v), n x n with leading dimension n.
hipError_t assemble_h(hipStream_t s, const double* H0, const double* S, const double* vorb,
                      double* H, int n);

// Transpose-pair passes over np x np tiles (np multiple of 32):
//  leapfrog:   out = base + f * rhodot with rhodot = -i (X - X^+),
//              X = Xre + i Xim:  Re rhodot = Xim + Xim^T,  Im rhodot = Xre^T - Xre;
//              with xref (leading dimension ldr), Xre = xre + xref; with zre, zim
//              (leading dimension ldz), X = (xre + i xim) - i (zre + i zim)
//  herm:       out = (T + T^+) / 2
//  sym:        out_re = (T + T^T) / 2 (real), out_im = 0 when given
hipError_t pair_leapfrog(hipStream_t s, const double* xre, const double* xim, int ldx,
                         const double* bre, const double* bim, int ldb, double* ore,
                         double* oim, int ldo, int np, double f, const double* xref = nullptr,
                         int ldr = 0, const double* zre = nullptr, const double* zim = nullptr,
                         int ldz = 0);
hipError_t pair_herm(hipStream_t s, const double* tre, const double* tim, int ldt,
                     double* ore, double* oim, int ldo, int np);
hipError_t pair_sym(hipStream_t s, const double* t, int ldt, double* ore, double* oim,
                    int ldo, int np);

// (re, im)[u, v] *= exp(-i kappa (x_u - x_v)).
hipError_t kick_phase(hipStream_t s, double* re, double* im, int ld, const double* x,
                      int np, double kappa);

// X = c * I on the first n diagonal entries, zero elsewhere (np x np, ld np).
hipError_t scaled_identity(hipStream_t s, double* X, int np, int n, double c);
// T = 2 I_n - T (np x np).
hipError_t two_minus(hipStream_t s, double* T, int np, int n);

// On-site corrections (plus_u_kernels.hip). Shell blocks are stored as
// kPlusUMaxShell^2 doubles per shell (row-major, zero beyond the shell).
// n_out: block populations of Re(rho) (rho wide, leading dimension ldr);
// e_sh (optional): each shell's correction energy. mode: 1 FLL, 2 pSIC.
hipError_t block_populations(hipStream_t s, const double* rho, int ldr, const double* S, int lds,
                             const int* sh_off, const double* sh_u, int nsh, int max_shell,
                             int mode, int ncols, double* n_out, double* e_sh);
hipError_t plus_u_potential(hipStream_t s, const double* n, const int* sh_off, const double* sh_u,
                            int nsh, int mode, double* V);
// dV = -(U/2)(n - cs[0] nref) per shell block (change from the reference)
hipError_t plus_u_delta_potential(hipStream_t s, const double* n, const double* nref,
                                  const double* cs, const int* sh_off, const double* sh_u,
                                  int nsh, double* V);
// H0 may be null: the SCC and correction terms alone
hipError_t assemble_h_plus_u(hipStream_t s, const double* H0, const double* S, const double* vorb,
                             const int* sh_of, const int* sh_off, const double* V, double* H,
                             int np);
// y = 2 x - y over len elements
// Extrapolation along a trajectory: out = 2 x0 - x1 (x2 null) or
// 3 x0 - 3 x1 + x2; out may alias x1 or x2.
hipError_t extrapolate(hipStream_t s, const double* x0, const double* x1, const double* x2,
                       double* out, size_t len);
// X = (emax I_n - T) / (emax - emin).
hipError_t sp2_init(hipStream_t s, const double* T, double* X, int np, int n, double emax,
                    double emin);
// mode 0: X = X2; mode 1: X = 2 X - X2.
hipError_t sp2_update(hipStream_t s, double* X, const double* X2, int np, int mode);
// Copy a real np x np matrix (ld ldr) into the real block of a wide matrix, zero imag.
hipError_t real_to_wide(hipStream_t s, const double* R, int ldr, double* W, int np);
// Interleaved complex [n x n] <-> wide planar [np x 2np] (re | im).
hipError_t interleaved_to_wide(hipStream_t s, const double* Z, int n, double* W, int np);
hipError_t wide_to_interleaved(hipStream_t s, const double* W, int np, double* Z, int n);
// Plain real copy with padding: dst[np x np] <- src[n x n] (rest zero beforehand).
hipError_t pad_copy(hipStream_t s, const double* src, int n, double* dst, int np);
hipError_t unpad_copy(hipStream_t s, const double* src, int np, double* dst, int n);

// ---------------------------------------------------------------- reductions
// out[0] = sum_i X[i, i], i < n.
hipError_t trace(hipStream_t s, const double* X, int ld, int n, double* out);
// out[0] = max_{i,j<n} |delta_ij - T_ij| (work: n doubles).
hipError_t identity_residual(hipStream_t s, const double* T, int ld, int n, double* work,
                             double* out);
// out[0] = +inf if M (rows x cols) holds a value that is not finite, else
// max |M_ij - M_ji| when symmetric (rows == cols) or 0 (work: rows doubles).
hipError_t check_matrix(hipStream_t s, const double* M, int ld, int rows, int cols,
                        int symmetric, double* work, double* out);
// Gershgorin bounds of T (n x n): out[0] = min(center - radius), out[1] = max(...).
hipError_t gershgorin(hipStream_t s, const double* T, int ld, int n, double* work_lo,
                      double* work_hi, double* out);
// out[0] = sum_i x[i]
hipError_t sum_vector(hipStream_t s, const double* x, int n, double* out);

// Power iteration on column blocks (V, W, SV: np x ncols, leading dimension
// ld). power_start: +-1 entries in rows < n, zero in the padding rows.
// power_step: columns j < half become (W - lo V) / |W - lo V|, the others
// (hi V - W) / |hi V - W|. rayleigh: out[j] = (SV_j . W_j) / (SV_j . V_j).
hipError_t power_start(hipStream_t s, double* V, int ld, int n, int np, int ncols);
hipError_t power_step(hipStream_t s, const double* W, double* V, int ld, int np, int ncols,
                      int half, double lo, double hi);
hipError_t rayleigh(hipStream_t s, const double* V, const double* W, const double* SV, int ld,
                    int np, int ncols, double* out);

// Anderson mixing of SCC charges: r = dq_out - dq_in, out_resid[0] = max|r|;
// history slot `slot` <- (dq_in, r); `count` valid entries after storing;
// dq_in <- Anderson update with parameter beta.
hipError_t anderson_mix(hipStream_t s, double* dq_in, const double* dq_out, double* hx,
                        double* hf, int na, int m, int count, int slot, double beta,
                        double* out_resid);

// Energy pieces of the current state: out[0] = sum R o H0 (work: rows),
// out[1] = 1/2 dq gamma dq, out[2] = sum dq_a R_a . E (E may be null).
hipError_t energy_terms(hipStream_t s, const double* q_band_rows, int n, const double* dq,
                        const double* v_gamma, const double* pos, const double* E, int na,
                        double* out);

}  // namespace td
