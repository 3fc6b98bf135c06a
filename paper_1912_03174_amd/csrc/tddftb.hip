// C ABI of the TD-DFTB propagation library (declared in tddftb.h).
//
// Device layout (all float64, row-major, dimension padded to np, a
// multiple of 128, with zeros outside the n x n block):
//   S, H0, S^-1, H, A = S^-1 H           np x np
//   rho_cur, rho_prev, X = A rho         np x 2np "wide" planar complex:
//                                        columns [0, np) real part,
//                                        columns [np, 2np) imaginary part
// so that A [Re rho | Im rho] is one real product with 2np columns, and
// the zero padding keeps every product and update exact on the n x n
// block without tail handling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tddftb.h"
#include "common.hpp"
#include "ctx.hpp"
#include "split.hpp"

using td::round_up;

namespace {

// scal[] slots
enum { SC_MU = 0, SC_NE = 3, SC_RES = 4, SC_TR1 = 5, SC_TR2 = 6, SC_BOUNDS = 8, SC_E = 10,
       SC_RENORM = 13, SC_FIELD = 16, SC_EREP = 20, SC_COUNT = 32 };

using tdi::Fail;
using tdi::guarded;
using tdi::set_err;

void dalloc(td_ctx* c, double** p, size_t count) {
  HIPCHK(c, hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(double)));
  HIPCHK(c, hipMemsetAsync(*p, 0, std::max<size_t>(count, 1) * sizeof(double), c->stream));
}

void free_all(td_ctx* c) {
  double** bufs[] = {&c->S,   &c->H0,   &c->Sinv, &c->H,     &c->A,    &c->rho_cur,
                     &c->rho_prev, &c->X, &c->gamma, &c->pos, &c->q0, &c->q_orb,
                     &c->dq,  &c->dq_in, &c->v,   &c->vorb,  &c->xorb, &c->work1,
                     &c->work2, &c->scal, &c->hx, &c->hf,    &c->field, &c->dip};
  for (double** b : bufs) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  double** sbufs[] = {&c->rho_ref, &c->Agsb, &c->Xref, &c->q_ref, &c->v_ref, &c->band_ref,
                      &c->stage};
  for (double** b : sbufs) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  __bf16** slb[] = {&c->sl_sinv, &c->sl_dh, &c->sl_L2, &c->sl_R2};
  for (__bf16** b : slb) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  int** eb[] = {&c->e_sinv, &c->e_dh, &c->e_L2, &c->e_R2};
  for (int** b : eb) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  double** ebufs[] = {&c->sk_s, &c->sk_h, &c->scale_s, &c->scale_h, &c->onsite, &c->mass,
                      &c->rep_a, &c->e_rep_atom,
                      &c->GS, &c->GH, &c->W, &c->Dm, &c->Sinv_prev, &c->Sinv_prev2, &c->Z, &c->dgamma,
                      &c->vel, &c->F,
                      &c->e_kin, &c->e_el, &c->sh_u, &c->sh_n, &c->sh_v, &c->sh_e,
                      &c->sh_nref,
                      &c->mix_in, &c->mix_out, &c->mix_hx, &c->mix_hf};
  for (double** b : ebufs) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  int** eib[] = {&c->species, &c->norb, &c->atom_of, &c->sh_off, &c->sh_of};
  for (int** b : eib) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  if (c->orb_off) (void)hipFree(c->orb_off);
  c->orb_off = nullptr;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  c->stream = nullptr;
}

void sync(td_ctx* c) { HIPCHK(c, hipStreamSynchronize(c->stream)); }

void read_scal(td_ctx* c, int slot, double* out, int count) {
  HIPCHK(c, hipMemcpyAsync(out, c->scal + slot, sizeof(double) * count, hipMemcpyDeviceToHost,
                           c->stream));
  sync(c);
}

void gemm(td_ctx* c, int tag, int m, int n, int k, double alpha, const double* A, int lda,
          const double* B, int ldb, double* C, int ldc) {
  HIPCHK(c, td::dgemm(c->stream, tag, m, n, k, alpha, A, lda, B, ldb, 0.0, nullptr, 0, C, ldc));
}

// Mulliken charges, dipole and electron count of rho_cur; dipole -> `mu`
// (device, 3 doubles).
void mulliken(td_ctx* c, double* mu) {
  HIPCHK(c, td::rowdot(c->stream, c->rho_cur, 2 * c->np, c->S, c->np, c->q_orb, c->np, c->np));
  if (c->split) {
    // rho = rho_ref + delta; trace correction c -> scal[SC_RENORM]
    HIPCHK(c, td::charges_dipole_split(c->stream, c->q_orb, c->q_ref, c->orb_off, c->q0, c->pos,
                                       c->na, (double)c->nelec, c->dq, mu,
                                       c->scal + SC_RENORM));
  } else {
    HIPCHK(c, td::charges_dipole(c->stream, c->q_orb, c->orb_off, c->q0, c->pos, c->na, c->dq,
                                 mu, c->scal + SC_NE));
  }
}

// Observables of the current state, copied to the host; checks finiteness
// and the electron count Tr(rho S), a constant of the leapfrog motion
// (Sec. 2.3). `reference`: the state was just set (creation, kick,
// restore) and its count becomes the one later states are held to.
// Otherwise a count that moved by more than 1e-6 N_e (1e-3 N_e with moving
// nuclei, where S changes and leapfrog keeps the count only to its own
// error) is reported as an unstable run; in split-bf16 precision, where
// every step restores the count, the departure of the last step is checked.
void refresh(td_ctx* c, bool reference = false) {
  mulliken(c, c->scal + SC_MU);
  c->dq_h.resize(c->na);
  HIPCHK(c, hipMemcpyAsync(c->dq_h.data(), c->dq, sizeof(double) * c->na, hipMemcpyDeviceToHost,
                           c->stream));
  double sc[4];                            // dipole, electron count (FP64 path)
  read_scal(c, SC_MU, sc, 4);
  std::memcpy(c->mu_h, sc, sizeof(c->mu_h));
  bool ok = std::isfinite(c->mu_h[0]) && std::isfinite(c->mu_h[1]) && std::isfinite(c->mu_h[2]);
  for (int a = 0; a < c->na && ok; ++a) ok = std::isfinite(c->dq_h[a]);
  REQUIRE(c, ok, TD_EUNSTABLE, "density matrix became non-finite (time step too large?)");
  double ne = sc[3];
  if (c->split) {
    double cr;
    read_scal(c, SC_RENORM, &cr, 1);
    ne = c->nelec * (1.0 + cr);
  }
  REQUIRE(c, std::isfinite(ne), TD_EUNSTABLE, "electron count became non-finite");
  if (reference) {
    c->ne_ref = ne;
    return;
  }
  const double tol = (c->ehr ? 1e-3 : 1e-6) * c->nelec;
  const double drift = c->split ? std::fabs(ne - c->nelec) : std::fabs(ne - c->ne_ref);
  if (!(drift <= tol)) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "electron count Tr(rho S) = %.12g moved by %.3g from %.12g by step %lld "
                  "(unstable run?)",
                  ne, drift, c->split ? (double)c->nelec : c->ne_ref, (long long)c->step);
    REQUIRE(c, false, TD_EUNSTABLE, msg);
  }
}

// S^-1 by the Newton-Schulz iteration X <- X (2 - S X), X_0 = I / g with g
// a Gershgorin bound of the largest eigenvalue of S.
// With `warm`, the iteration starts from the current S^-1 (the inverse of a
// nearby S, as after a nuclear step); when the inverse at the positions
// before is kept too (moving nuclei), from the linear extrapolation
// 2 X_n - X_{n-1} along the trajectory, whose residual is second order in
// the step instead of first.
//
// The iteration is a sequence of decisions on the measured residual
// max |1 - S X| (ns_decide), shared by one trajectory and by batches of
// them: the same decisions in the same order give bitwise the same inverse.
struct NsIter {
  bool warm = false, restarted = false, done = false;
  double prev = INFINITY, res = INFINITY;
  int it = 0;
};
enum NsAction { NS_UPDATE, NS_RESTART, NS_DONE };

// X = I / g, g the Gershgorin bound of the largest eigenvalue of S.
void ns_cold_start(td_ctx* c) {
  HIPCHK(c, td::gershgorin(c->stream, c->S, c->np, c->n, c->work1, c->work2,
                           c->scal + SC_BOUNDS));
  double b[2];
  read_scal(c, SC_BOUNDS, b, 2);
  REQUIRE(c, std::isfinite(b[1]) && b[1] > 0, TD_ENOTPOSDEF, "S has no positive spectrum bound");
  HIPCHK(c, td::scaled_identity(c->stream, c->Sinv, c->np, c->n, 1.0 / b[1]));
}

// The starting inverse. Warm: from the inverses at earlier positions of the
// trajectory, the quadratic extrapolation 3 X_n - 3 X_{n-1} + X_{n-2}
// (residual third order in the step), linear 2 X_n - X_{n-1} while only two
// are known, X_n itself at the first.
void ns_begin(td_ctx* c, bool warm, NsIter& s) {
  s = NsIter{};
  s.warm = warm;
  if (warm && c->Sinv_prev) {
    const size_t len = (size_t)c->np * c->np;
    if (c->sinv_hist == 0) {
      HIPCHK(c, hipMemcpyAsync(c->Sinv_prev, c->Sinv, sizeof(double) * len,
                               hipMemcpyDeviceToDevice, c->stream));
    } else {
      HIPCHK(c, td::extrapolate(c->stream, c->Sinv, c->Sinv_prev,
                                c->sinv_hist >= 2 ? c->Sinv_prev2 : nullptr, c->Sinv_prev2,
                                len));
      double* start = c->Sinv_prev2;         // X_{n-2} is overwritten by the start
      c->Sinv_prev2 = c->Sinv_prev;
      c->Sinv_prev = c->Sinv;
      c->Sinv = start;
    }
    c->sinv_hist = std::min(c->sinv_hist + 1, 2);
  }
  if (!warm) ns_cold_start(c);
}

// The residual of 1 - S X with T = S X in c->A, into c->scal[SC_RES].
void ns_residual(td_ctx* c) {
  HIPCHK(c, td::identity_residual(c->stream, c->A, c->np, c->n, c->work1, c->scal + SC_RES));
}

// What to do with the residual just measured.
NsAction ns_decide(td_ctx* c, NsIter& s, double res) {
  s.it += 1;
  s.res = res;
  REQUIRE(c, s.it <= 200, TD_ENOTPOSDEF, "S is singular or indefinite: inverse did not converge");
  // A warm start converges only while the spectral radius of 1 - S X is
  // below 1, which the element-wise residual does not bound: after a long
  // nuclear step (a start residual above 1/4) or a residual that grows,
  // begin again from the scaled identity, which always converges.
  if (s.warm && !s.restarted && !(res <= 0.25 && res < s.prev)) {
    s.restarted = true;
    s.prev = INFINITY;
    c->info.inverse_restarts += 1;
    return NS_RESTART;
  }
  REQUIRE(c, std::isfinite(res) && res < 1e3, TD_ENOTPOSDEF,
          "S is not positive definite: inverse iteration diverged");
  if (res < 1e-15 || (res < 1e-9 && res >= 0.5 * s.prev)) return NS_DONE;
  s.prev = res;
  return NS_UPDATE;
}

// After the update X (2 - S X) (the new X in c->Sinv): the residual squares
// with each update, so from a warm start below 1e-8 the updated inverse is
// at the rounding floor and the iteration stops without a check.
void ns_updated(td_ctx* c, NsIter& s) {
  std::swap(c->Sinv, c->H);
  c->info.inverse_updates += 1;
  if (s.warm && s.res < 1e-8) s.done = true;
}

void ns_finish(td_ctx* c, const NsIter& s) {
  REQUIRE(c, s.res < 1e-8, TD_ENOTPOSDEF, "S is singular or indefinite: inverse did not converge");
  HIPCHK(c, td::pair_sym(c->stream, c->Sinv, c->np, c->Sinv, nullptr, c->np, c->np));
  c->info.inverse_iterations = s.it;
  c->info.inverse_residual = s.res;
}

void inverse_overlap(td_ctx* c, bool warm = false) {
  const int np = c->np;
  NsIter s;
  ns_begin(c, warm, s);
  while (!s.done) {
    gemm(c, 0, np, np, np, 1.0, c->S, np, c->Sinv, np, c->A, np);     // T = S X
    ns_residual(c);
    double res;
    read_scal(c, SC_RES, &res, 1);
    const NsAction a = ns_decide(c, s, res);
    if (a == NS_RESTART) {
      ns_cold_start(c);
      continue;
    }
    if (a == NS_DONE) break;
    HIPCHK(c, td::two_minus(c->stream, c->A, np, c->n));               // 2 - S X
    // X (2 - S X) = 2 X - X S X is symmetric: the upper tiles and a mirror
    HIPCHK(c, td::dgemm_symmetric(c->stream, np, np, c->Sinv, np, c->A, np, c->H, np));
    ns_updated(c, s);
  }
  ns_finish(c, s);
}

// Zero-temperature density by second-order spectral projection (SP2,
// Niklasson, Phys. Rev. B 66, 155115 (2002)) of T = S^-1 H: X_0 maps the
// spectrum into [0, 1] reversed, X <- X^2 or 2X - X^2 steers Tr X to the
// number of occupied states; rho = 2 X S^-1. Input H in c->H; output the
// real density in the real block of rho_cur.
void purify(td_ctx* c) {
  const int n = c->n, np = c->np;
  const double nocc = 0.5 * c->nelec;
  gemm(c, 0, np, np, np, 1.0, c->Sinv, np, c->H, np, c->A, np);        // T = S^-1 H
  HIPCHK(c, td::gershgorin(c->stream, c->A, np, n, c->work1, c->work2, c->scal + SC_BOUNDS));
  double b[2];
  read_scal(c, SC_BOUNDS, b, 2);
  REQUIRE(c, std::isfinite(b[0]) && std::isfinite(b[1]) && b[1] > b[0], TD_ESCF,
          "invalid spectrum bounds of S^-1 H");
  c->info.spectrum_lo = b[0];
  c->info.spectrum_hi = b[1];
  double* Xm = c->H;          // H is consumed by T
  double* X2 = c->rho_prev;   // scratch (np x np view)
  HIPCHK(c, td::sp2_init(c->stream, c->A, Xm, np, n, b[1], b[0]));
  double prev = INFINITY, err = INFINITY;
  int it;
  for (it = 1; it <= 400; ++it) {
    gemm(c, 0, np, np, np, 1.0, Xm, np, Xm, np, X2, np);
    HIPCHK(c, td::trace(c->stream, Xm, np, n, c->scal + SC_TR1));
    HIPCHK(c, td::trace(c->stream, X2, np, n, c->scal + SC_TR2));
    double tr[2];
    read_scal(c, SC_TR1, tr, 2);
    err = tr[0] - tr[1];
    REQUIRE(c, std::isfinite(err), TD_ESCF, "purification produced non-finite values");
    const int mode = (std::fabs(tr[1] - nocc) < std::fabs(2.0 * tr[0] - tr[1] - nocc)) ? 0 : 1;
    HIPCHK(c, td::sp2_update(c->stream, Xm, X2, np, mode));
    if (std::fabs(err) < 1e-5 && std::fabs(err) >= prev) break;
    prev = std::fabs(err);
  }
  REQUIRE(c, it <= 400 && std::fabs(err) < 1e-6, TD_ESCF,
          "purification did not converge (HOMO-LUMO gap too small?)");
  c->info.purification_iterations = it;
  c->info.purification_error = err;
  gemm(c, 0, np, np, np, 2.0, Xm, np, c->Sinv, np, X2, np);            // rho = 2 X S^-1
  HIPCHK(c, td::pair_sym(c->stream, X2, np, c->rho_cur, c->rho_cur + np, 2 * np, np));
}

void assemble_hamiltonian(td_ctx* c, const double* n_blocks);
void block_pops(td_ctx* c, double* out, const double* rho = nullptr, int ldr = 0);

// With on-site corrections the mixed vector is [dq | block populations]:
// H is built from the mixed charges and populations, and both are
// compared with those of the purified density.
void ground_state(td_ctx* c) {
  const int na = c->na;
  const int m = std::max(1, std::min(8, c->opt.mix_history));
  const bool pu = c->plus_u != TD_PLUS_U_NONE;
  const int len = pu ? c->mix_len : na;
  double* x_in = pu ? c->mix_in : c->dq_in;
  double* x_out = pu ? c->mix_out : c->dq;
  double* hx = pu ? c->mix_hx : c->hx;
  double* hf = pu ? c->mix_hf : c->hf;
  HIPCHK(c, hipMemsetAsync(x_in, 0, sizeof(double) * len, c->stream));
  double res = INFINITY;
  int it;
  for (it = 1; it <= c->opt.scc_maxiter; ++it) {
    HIPCHK(c, td::potential(c->stream, c->gamma, x_in, c->pos, nullptr, c->orb_off, na, c->v,
                            c->vorb));
    assemble_hamiltonian(c, pu ? x_in + na : nullptr);
    purify(c);
    mulliken(c, c->scal + SC_MU);
    if (pu) {
      HIPCHK(c, hipMemcpyAsync(x_out, c->dq, sizeof(double) * na, hipMemcpyDeviceToDevice,
                               c->stream));
      block_pops(c, x_out + na);
    }
    const int count = std::min(it, m), slot = (it - 1) % m;
    HIPCHK(c, td::anderson_mix(c->stream, x_in, x_out, hx, hf, len, m, count, slot,
                               c->opt.mix_beta, c->scal + SC_RES));
    read_scal(c, SC_RES, &res, 1);
    REQUIRE(c, std::isfinite(res), TD_ESCF, "SCC cycle produced non-finite charges");
    if (res < c->opt.scc_tol) break;
  }
  c->info.scc_iterations = std::min(it, c->opt.scc_maxiter);
  c->info.scc_residual = res;
  if (!(res < c->opt.scc_tol)) {
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "SCC ground state did not converge: %d cycles, max |dq_out - dq_in| = %.3e, "
                  "last purification %d iterations",
                  c->info.scc_iterations, res, c->info.purification_iterations);
    c->err = msg;
    throw Fail{TD_ESCF};
  }
}

void ensure_events(td_ctx* c, size_t count) {
  while (c->ev.size() < count) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Shells of the on-site corrections: contiguous, covering all orbitals,
// each of 1..TD_PLUS_U_MAX_SHELL orbitals of one atom, finite U >= 0.
void validate_plus_u(td_ctx* c, const td_system* s) {
  REQUIRE(c, s->plus_u == TD_PLUS_U_NONE || s->plus_u == TD_PLUS_U_FLL ||
                 s->plus_u == TD_PLUS_U_PSIC,
          TD_EINVAL, "unknown plus_u");
  if (s->plus_u == TD_PLUS_U_NONE) return;
  REQUIRE(c, s->n_shells > 0 && s->n_shells <= s->n_orb && s->shell_offset && s->shell_u,
          TD_EINVAL, "plus_u needs n_shells, shell_offset and shell_u");
  REQUIRE(c, s->shell_offset[0] == 0 && s->shell_offset[s->n_shells] == s->n_orb, TD_EINVAL,
          "shell_offset must start at 0 and end at n_orb");
  int a = 0;
  for (int b = 0; b < s->n_shells; ++b) {
    const int lo = s->shell_offset[b], hi = s->shell_offset[b + 1];
    REQUIRE(c, hi > lo && hi - lo <= TD_PLUS_U_MAX_SHELL, TD_EINVAL,
            "every shell needs 1 to TD_PLUS_U_MAX_SHELL orbitals");
    while (a < s->n_atoms && s->orb_offset[a + 1] <= lo) ++a;
    REQUIRE(c, a < s->n_atoms && s->orb_offset[a] <= lo && hi <= s->orb_offset[a + 1], TD_EINVAL,
            "a shell must lie within one atom");
    REQUIRE(c, std::isfinite(s->shell_u[b]) && s->shell_u[b] >= 0.0, TD_EINVAL,
            "shell_u must be finite and >= 0");
  }
}

// Checks of the model and options on the host. With `big_on_host` false the
// n x n and n_atoms x n_atoms arrays (S, H0, gamma, rho0) are device
// pointers, checked on the device after their copy (check_device_arrays).
void validate(td_ctx* c, const td_system* s, const td_options* o, bool big_on_host) {
  REQUIRE(c, s && o, TD_EINVAL, "null system or options");
  REQUIRE(c, s->n_atoms > 0 && s->n_orb > 0, TD_EINVAL, "n_atoms and n_orb must be positive");
  REQUIRE(c, s->n_orb <= 65536, TD_EINVAL, "n_orb too large");
  REQUIRE(c, s->orb_offset && s->positions && s->S && s->H0 && s->gamma && s->q0, TD_EINVAL,
          "null array in td_system");
  REQUIRE(c, s->orb_offset[0] == 0 && s->orb_offset[s->n_atoms] == s->n_orb, TD_EINVAL,
          "orb_offset must start at 0 and end at n_orb");
  for (int a = 0; a < s->n_atoms; ++a)
    REQUIRE(c, s->orb_offset[a + 1] > s->orb_offset[a], TD_EINVAL,
            "orb_offset must be strictly increasing");
  if (s->occ) {
    // closed-shell aufbau only: 2 for the lowest states, then 0
    REQUIRE(c, finite_all(s->occ, (size_t)s->n_orb), TD_EINVAL, "non-finite occ");
    int n2 = 0;
    while (n2 < s->n_orb && s->occ[n2] == 2.0) ++n2;
    bool aufbau = true;
    for (int i = n2; i < s->n_orb; ++i) aufbau = aufbau && s->occ[i] == 0.0;
    REQUIRE(c, aufbau, TD_ENOTSUP,
            "occ must be closed-shell aufbau (2 for the lowest states, then 0): the ground "
            "state is a zero-temperature purification");
    REQUIRE(c, s->n_elec == 0 || s->n_elec == 2 * n2, TD_EINVAL, "n_elec must be 0 or sum(occ)");
    REQUIRE(c, n2 > 0, TD_EINVAL, "occ holds no electrons");
  } else {
    REQUIRE(c, s->n_elec > 0 && s->n_elec % 2 == 0 && s->n_elec <= 2 * s->n_orb, TD_EINVAL,
            "n_elec must be even and in (0, 2 n_orb]");
  }
  REQUIRE(c, o->dt > 0 && std::isfinite(o->dt), TD_EINVAL, "dt must be positive");
  REQUIRE(c, o->precision == TD_FP64 || o->precision == TD_SPLIT_BF16, TD_EINVAL,
          "unknown precision");
  validate_plus_u(c, s);
  REQUIRE(c, o->precision == TD_FP64 || (o->n_slices >= 3 && o->n_slices <= 5), TD_EINVAL,
          "n_slices must be 3, 4 or 5");
  REQUIRE(c, o->precision == TD_FP64 || o->n_slices_dh == 0 ||
                 (o->n_slices_dh >= 3 && o->n_slices_dh <= o->n_slices),
          TD_EINVAL, "n_slices_dh must be 0 or 3 .. n_slices");
  REQUIRE(c, o->scc_tol > 0 && o->scc_maxiter > 0 && o->mix_beta > 0 && o->mix_beta <= 1,
          TD_EINVAL, "invalid SCC options");
  const size_t n = (size_t)s->n_orb, na = (size_t)s->n_atoms;
  REQUIRE(c, finite_all(s->q0, na) && finite_all(s->positions, na * 3), TD_EINVAL,
          "non-finite input values");
  if (!big_on_host) return;
  REQUIRE(c, finite_all(s->S, n * n) && finite_all(s->H0, n * n) &&
                 finite_all(s->gamma, na * na),
          TD_EINVAL, "non-finite input values");
  double asym = 0.0;
  for (size_t i = 0; i < n; ++i)
    for (size_t j = i + 1; j < n; ++j) {
      asym = std::max(asym, std::fabs(s->S[i * n + j] - s->S[j * n + i]));
      asym = std::max(asym, std::fabs(s->H0[i * n + j] - s->H0[j * n + i]));
    }
  REQUIRE(c, asym <= 1e-12, TD_EINVAL, "S and H0 must be symmetric");
  if (s->rho0) REQUIRE(c, finite_all(s->rho0, 2 * n * n), TD_EINVAL, "non-finite rho0");
}

void salloc(td_ctx* c, __bf16** p, size_t count) {
  HIPCHK(c, hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(__bf16)));
  HIPCHK(c, hipMemsetAsync(*p, 0, std::max<size_t>(count, 1) * sizeof(__bf16), c->stream));
}

void ialloc(td_ctx* c, int** p, size_t count) {
  HIPCHK(c, hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(int)));
  HIPCHK(c, hipMemsetAsync(*p, 0, std::max<size_t>(count, 1) * sizeof(int), c->stream));
}

void slice(td_ctx* c, int mode, const td::SliceSrc& src, int rows, int cols, __bf16* out,
           int ldo, int* exps, int ns = 0) {
  HIPCHK(c, td::slice_rows(c->stream, ns ? ns : c->ns, mode, src, rows, cols, out, ldo, exps));
}

// Split precision set-up. The current (full) density becomes the reference
// rho_ref (its real part) and the state holds delta = rho - rho_ref. With
// A_ref = S^-1 H_ref and B = S^-1 dH (dH = H - H_ref, from dv = v - v_ref),
//   X = S^-1 H rho = A_ref rho_ref + (A_ref + B) delta + B rho_ref,
// so the products act on O(signal) operands and the O(1) part A_ref rho_ref
// is formed once in FP64.
void split_init(td_ctx* c) {
  const int n = c->n, np = c->np, na = c->na;
  const size_t m2 = (size_t)np * np;
  dalloc(c, &c->rho_ref, m2);
  dalloc(c, &c->Agsb, m2);
  dalloc(c, &c->Xref, 2 * m2);
  dalloc(c, &c->q_ref, np);
  dalloc(c, &c->v_ref, na);
  dalloc(c, &c->band_ref, np);
  dalloc(c, &c->stage, 2 * m2);
  salloc(c, &c->sl_sinv, (size_t)c->ns * m2);
  salloc(c, &c->sl_dh, (size_t)c->ns * m2);
  salloc(c, &c->sl_L2, (size_t)c->ns * 2 * m2);
  salloc(c, &c->sl_R2, (size_t)c->ns * 4 * m2);
  ialloc(c, &c->e_sinv, np);
  ialloc(c, &c->e_dh, np);
  ialloc(c, &c->e_L2, 2 * (size_t)np);
  ialloc(c, &c->e_R2, 4 * (size_t)np);
  hipStream_t st = c->stream;
  HIPCHK(c, td::pair_sym(st, c->rho_cur, 2 * np, c->rho_ref, nullptr, np, np));
  HIPCHK(c, td::wide_add_real(st, c->rho_cur, c->rho_ref, np, -1.0));
  HIPCHK(c, td::rowdot(st, c->rho_ref, np, c->S, np, c->q_ref, np, np));
  HIPCHK(c, td::rowdot(st, c->rho_ref, np, c->H0, np, c->band_ref, np, np));
  HIPCHK(c, td::charges_dipole(st, c->q_ref, c->orb_off, c->q0, c->pos, na, c->dq,
                               c->scal + SC_MU, c->scal + SC_NE));
  HIPCHK(c, td::potential(st, c->gamma, c->dq, c->pos, nullptr, c->orb_off, na, c->v_ref,
                          c->vorb));
  if (c->plus_u != TD_PLUS_U_NONE) {
    dalloc(c, &c->sh_nref, (size_t)c->nsh * td::kPlusUMaxShell * td::kPlusUMaxShell);
    block_pops(c, c->sh_nref, c->rho_ref, np);
  }
  assemble_hamiltonian(c, c->sh_nref);     // H_ref, with the correction of rho_ref
  gemm(c, 0, np, np, np, 1.0, c->Sinv, np, c->H, np, c->Agsb, np);
  gemm(c, 0, np, np, np, 1.0, c->Agsb, np, c->rho_ref, np, c->Xref, 2 * np);
  td::SliceSrc si;
  si.M0 = c->Sinv;
  si.ld0 = np;
  const int S = c->ns;
  slice(c, td::SLICE_PLAIN, si, np, np, c->sl_sinv, np * c->ns1, c->e_sinv, c->ns1);
  td::SliceSrc sr;
  sr.M0 = c->rho_ref;
  sr.ld0 = np;
  // reference rows become K segment 1 of the second product's right operand
  slice(c, td::SLICE_PLAIN, sr, np, np, c->sl_R2 + (size_t)np * S, 2 * np * S,
        c->e_R2 + 2 * np);
  (void)n;
}

// One split-precision step body (after the dipole of rho_k is recorded):
// sliced [delta_re + renorm | -delta_im], potential change, sliced dH,
// B = S^-1 dH, sliced [A | B], X = A_ref rho_ref + [A | B][delta; rho_ref].
void split_products(td_ctx* c, const double* E, hipEvent_t* ev) {
  const int np = c->np, na = c->na;
  hipStream_t st = c->stream;
  const int S = c->ns, S1 = c->ns1;    // slices of the second and of the first product
  // [delta_re + renorm | -delta_im] (renormalises delta_re in place)
  auto slice_density = [&] {
    td::SliceSrc sdr;
    sdr.M0 = c->rho_cur;
    sdr.M0w = c->rho_cur;
    sdr.ld0 = 2 * np;
    sdr.M1 = c->rho_ref;
    sdr.ld1 = np;
    sdr.cs = c->scal + SC_RENORM;
    slice(c, td::SLICE_RENORM, sdr, np, np, c->sl_R2, 2 * np * S, c->e_R2);
    td::SliceSrc sdi;
    sdi.M0 = c->rho_cur + np;
    sdi.ld0 = 2 * np;
    sdi.sign = -1.0;
    slice(c, td::SLICE_PLAIN, sdi, np, np, c->sl_R2 + (size_t)np * 2 * np * S, 2 * np * S,
          c->e_R2 + np);
  };
  // right after the charges pass has read the density, while its lines are
  // still cached; the on-site correction reads the density first
  if (c->plus_u == TD_PLUS_U_NONE) slice_density();
  HIPCHK(c, td::potential(st, c->gamma, c->dq, c->pos, E, c->orb_off, na, c->v, c->vorb,
                          c->v_ref));
  td::SliceSrc sdh;
  sdh.M0 = c->S;
  sdh.ld0 = np;
  sdh.v = c->vorb;
  if (c->plus_u != TD_PLUS_U_NONE) {
    // dH = 1/2 S o (dv + dv) + 1/2 (S dV + dV S) (Sec. 3.2) formed in A, then sliced
    block_pops(c, c->sh_n);
    HIPCHK(c, td::plus_u_delta_potential(st, c->sh_n, c->sh_nref, c->scal + SC_RENORM,
                                         c->sh_off, c->sh_u, c->nsh, c->sh_v));
    HIPCHK(c, td::assemble_h_plus_u(st, nullptr, c->S, c->vorb, c->sh_of, c->sh_off, c->sh_v,
                                    c->A, np));
    td::SliceSrc sa;
    sa.M0 = c->A;
    sa.ld0 = np;
    slice(c, td::SLICE_PLAIN, sa, np, np, c->sl_dh, np * S1, c->e_dh, S1);
    slice_density();
  } else {
    slice(c, td::SLICE_DH, sdh, np, np, c->sl_dh, np * S1, c->e_dh, S1);
  }
  td::SplitGemm g1;
  g1.m = np;
  g1.n = np;
  g1.L = c->sl_sinv;
  g1.ldl = np * S1;
  g1.eL = c->e_sinv;
  g1.R = c->sl_dh;
  g1.ldr = np * S1;
  g1.fR = c->e_dh;
  g1.seg_len = np;
  g1.k_lo = np;
  g1.k_hi = np;
  g1.n_split = np;
  g1.C = c->H;            // B = S^-1 dH
  g1.ldc = np;
  if (ev) HIPCHK(c, hipEventRecord(ev[1], st));
  HIPCHK(c, td::split_gemm(st, S1, g1));
  if (ev) HIPCHK(c, hipEventRecord(ev[2], st));
  td::SliceSrc sa;
  sa.M0 = c->Agsb;
  sa.ld0 = np;
  sa.M1 = c->H;
  sa.ld1 = np;
  if (np <= 4096) {
    // [A_ref + B | B] from one read of B
    sa.out2 = c->sl_L2 + (size_t)np * S;
    sa.exps2 = c->e_L2 + np;
    slice(c, td::SLICE_SUM_AND_M1, sa, np, np, c->sl_L2, 2 * np * S, c->e_L2);
  } else {
    slice(c, td::SLICE_SUM, sa, np, np, c->sl_L2, 2 * np * S, c->e_L2);
    td::SliceSrc sb;
    sb.M0 = c->H;
    sb.ld0 = np;
    slice(c, td::SLICE_PLAIN, sb, np, np, c->sl_L2 + (size_t)np * S, 2 * np * S, c->e_L2 + np);
  }
  td::SplitGemm g2;
  g2.m = np;
  g2.n = 2 * np;
  g2.L = c->sl_L2;
  g2.ldl = 2 * np * S;
  g2.eL = c->e_L2;
  g2.eL_stride = np;
  g2.R = c->sl_R2;
  g2.ldr = 2 * np * S;
  g2.fR = c->e_R2;
  g2.fR_stride = 2 * np;
  g2.seg_len = np;
  g2.k_hi = 2 * np;     // real columns: A delta_re + B rho_ref
  g2.k_lo = np;         // imaginary columns: A delta_im
  g2.n_split = np;
  g2.C = c->X;            // without X_ref: the update adds it (real part only)
  g2.ldc = 2 * np;
  if (ev) HIPCHK(c, hipEventRecord(ev[3], st));
  HIPCHK(c, td::split_gemm(st, c->ns, g2));
  if (ev) HIPCHK(c, hipEventRecord(ev[4], st));
}

// Full density (rho_ref + delta in split precision) of `src` into the wide `dst`.
void full_density(td_ctx* c, const double* src, double* dst) {
  if (dst != src)
    HIPCHK(c, hipMemcpyAsync(dst, src, sizeof(double) * 2 * (size_t)c->np * c->np,
                             hipMemcpyDeviceToDevice, c->stream));
  if (c->split) HIPCHK(c, td::wide_add_real(c->stream, dst, c->rho_ref, c->np, 1.0));
}

void upload_padded(td_ctx* c, const double* src, int n, double* dev, int np,
                   hipMemcpyKind kind = hipMemcpyHostToDevice) {
  HIPCHK(c, hipMemcpy2DAsync(dev, sizeof(double) * np, src, sizeof(double) * n,
                             sizeof(double) * n, n, kind, c->stream));
}

// Host copies of the per-atom and per-shell arrays of a model given by
// device pointers (the n x n and n_atoms x n_atoms arrays stay on the device).
struct HostModel {
  std::vector<int32_t> orb_offset, shell_offset;
  std::vector<double> positions, q0, occ, shell_u;
};

template <class T>
void fetch(td_ctx* c, hipStream_t st, const T* src, size_t count, std::vector<T>& dst) {
  dst.resize(count);
  if (src)
    HIPCHK(c, hipMemcpyAsync(dst.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost, st));
}

// Reads the small arrays of a device-pointer model into host memory (stream
// order of `st`, which is then drained, so that the device-to-device copies
// of the large arrays on the context's stream follow every earlier write) and
// returns a view with host pointers for them and the caller's device
// pointers for S, H0, gamma and rho0.
td_system host_view(td_ctx* c, const td_system* s, const td_options* o, HostModel& m) {
  REQUIRE(c, s && o, TD_EINVAL, "null system or options");
  REQUIRE(c, s->n_atoms > 0 && s->n_orb > 0 && s->n_orb <= 65536 && s->n_atoms <= s->n_orb,
          TD_EINVAL, "n_atoms and n_orb must be positive, n_atoms <= n_orb <= 65536");
  REQUIRE(c, s->orb_offset && s->positions && s->S && s->H0 && s->gamma && s->q0, TD_EINVAL,
          "null array in td_system");
  hipStream_t st = (hipStream_t)o->hip_stream;
  const size_t n = (size_t)s->n_orb, na = (size_t)s->n_atoms;
  fetch(c, st, s->orb_offset, na + 1, m.orb_offset);
  fetch(c, st, s->positions, 3 * na, m.positions);
  fetch(c, st, s->q0, na, m.q0);
  if (s->occ) fetch(c, st, s->occ, n, m.occ);
  const bool pu = s->plus_u != TD_PLUS_U_NONE && s->n_shells > 0 && s->n_shells <= s->n_orb;
  if (pu && s->shell_offset) fetch(c, st, s->shell_offset, (size_t)s->n_shells + 1, m.shell_offset);
  if (pu && s->shell_u) fetch(c, st, s->shell_u, (size_t)s->n_shells, m.shell_u);
  HIPCHK(c, hipStreamSynchronize(st));
  td_system h = *s;
  h.orb_offset = m.orb_offset.data();
  h.positions = m.positions.data();
  h.q0 = m.q0.data();
  h.occ = s->occ ? m.occ.data() : nullptr;
  h.shell_offset = (pu && s->shell_offset) ? m.shell_offset.data() : nullptr;
  h.shell_u = (pu && s->shell_u) ? m.shell_u.data() : nullptr;
  return h;
}

// The device checks of the arrays copied device to device: S and H0
// symmetric (to 1e-12) and finite, gamma and rho0 finite.
void check_device_arrays(td_ctx* c, bool has_rho0) {
  const int n = c->n, na = c->na, np = c->np;
  HIPCHK(c, td::check_matrix(c->stream, c->S, np, n, n, 1, c->work1, c->scal + SC_TR1));
  HIPCHK(c, td::check_matrix(c->stream, c->H0, np, n, n, 1, c->work1, c->scal + SC_TR2));
  HIPCHK(c, td::check_matrix(c->stream, c->gamma, na, na, na, 0, c->work1, c->scal + SC_RES));
  if (has_rho0)
    HIPCHK(c, td::check_matrix(c->stream, c->X, 2 * n, n, 2 * n, 0, c->work1,
                               c->scal + SC_NE));
  double r[4] = {0, 0, 0, 0};
  read_scal(c, SC_NE, r, 4);                           // SC_NE, SC_RES, SC_TR1, SC_TR2
  REQUIRE(c, std::isfinite(r[1]) && std::isfinite(r[2]) && std::isfinite(r[3]), TD_EINVAL,
          "non-finite input values");
  REQUIRE(c, std::max(r[2], r[3]) <= 1e-12, TD_EINVAL, "S and H0 must be symmetric");
  REQUIRE(c, !has_rho0 || std::isfinite(r[0]), TD_EINVAL, "non-finite rho0");
}

// Device copies of the shells, the shell of every orbital (-1 in the
// padding) and the buffers of the corrections and of their SCC mixing.
void setup_plus_u(td_ctx* c, const td_system* s) {
  const int nsh = s->n_shells, np = c->np;
  constexpr int BS = td::kPlusUMaxShell * td::kPlusUMaxShell;
  c->plus_u = s->plus_u;
  c->nsh = nsh;
  c->max_shell = 0;
  std::vector<int> of(np, -1);
  for (int b = 0; b < nsh; ++b) {
    c->max_shell = std::max(c->max_shell, s->shell_offset[b + 1] - s->shell_offset[b]);
    for (int u = s->shell_offset[b]; u < s->shell_offset[b + 1]; ++u) of[u] = b;
  }
  HIPCHK(c, hipMalloc((void**)&c->sh_off, sizeof(int) * (nsh + 1)));
  HIPCHK(c, hipMalloc((void**)&c->sh_of, sizeof(int) * np));
  HIPCHK(c, hipMemcpyAsync(c->sh_off, s->shell_offset, sizeof(int) * (nsh + 1),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->sh_of, of.data(), sizeof(int) * np, hipMemcpyHostToDevice,
                           c->stream));
  dalloc(c, &c->sh_u, nsh);
  HIPCHK(c, hipMemcpyAsync(c->sh_u, s->shell_u, sizeof(double) * nsh, hipMemcpyHostToDevice,
                           c->stream));
  dalloc(c, &c->sh_n, (size_t)nsh * BS);
  dalloc(c, &c->sh_v, (size_t)nsh * BS);
  dalloc(c, &c->sh_e, nsh);
  c->mix_len = c->na + nsh * BS;
  dalloc(c, &c->mix_in, c->mix_len);
  dalloc(c, &c->mix_out, c->mix_len);
  dalloc(c, &c->mix_hx, (size_t)8 * c->mix_len);
  dalloc(c, &c->mix_hf, (size_t)8 * c->mix_len);
  sync(c);   // `of` is a pageable staging buffer: finish its copy before it goes
}

// H of the current potential (c->vorb) plus, with on-site corrections, the
// term of the block populations n (device, shell blocks): V from n, then
// the assembly.
void assemble_hamiltonian(td_ctx* c, const double* n_blocks) {
  if (c->plus_u == TD_PLUS_U_NONE) {
    HIPCHK(c, td::assemble_h(c->stream, c->H0, c->S, c->vorb, c->H, c->np));
    return;
  }
  HIPCHK(c, td::plus_u_potential(c->stream, n_blocks, c->sh_off, c->sh_u, c->nsh, c->plus_u,
                                 c->sh_v));
  HIPCHK(c, td::assemble_h_plus_u(c->stream, c->H0, c->S, c->vorb, c->sh_of, c->sh_off, c->sh_v,
                                  c->H, c->np));
}

// Block populations of a density (default: the current one, wide) into
// `out`, and the shells' correction energies into sh_e.
void block_pops(td_ctx* c, double* out, const double* rho, int ldr) {
  if (!rho) {
    rho = c->rho_cur;
    ldr = 2 * c->np;
  }
  HIPCHK(c, td::block_populations(c->stream, rho, ldr, c->S, c->np, c->sh_off, c->sh_u, c->nsh,
                                  c->max_shell, c->plus_u, c->np, out, c->sh_e));
}

// Lower bound of the width of the spectrum of S^-1 H (the generalized
// eigenvalues of (H, S)) of the current state at zero field. The leapfrog
// step multiplies the (i, j) element of rho in the generalized eigenbasis
// by the roots of z^2 + 2 i theta z - 1 with theta = dt (eps_i - eps_j),
// which leave the unit circle once |theta| > 1 (Sec. 2.3, Eq. 19). Every
// Rayleigh quotient x^T H x / x^T S x lies between the extreme eigenvalues,
// so the largest quotient of 64 vectors steered to the top of the spectrum
// by power iteration with S^-1 H - lo, minus the smallest of 64 steered to
// its bottom with hi - S^-1 H (lo, hi: Gershgorin bounds), never exceeds
// the width; after 80 steps it is within a few percent of it.
void spectral_width(td_ctx* c) {
  constexpr int kCols = 128, kIters = 80;
  const int n = c->n, np = c->np, na = c->na;
  hipStream_t st = c->stream;
  HIPCHK(c, td::potential(st, c->gamma, c->dq, c->pos, nullptr, c->orb_off, na, c->v, c->vorb));
  if (c->plus_u != TD_PLUS_U_NONE) block_pops(c, c->sh_n);
  assemble_hamiltonian(c, c->sh_n);
  gemm(c, 0, np, np, np, 1.0, c->Sinv, np, c->H, np, c->A, np);        // T = S^-1 H
  HIPCHK(c, td::gershgorin(st, c->A, np, n, c->work1, c->work2, c->scal + SC_BOUNDS));
  double b[2];
  read_scal(c, SC_BOUNDS, b, 2);
  REQUIRE(c, std::isfinite(b[0]) && std::isfinite(b[1]), TD_EUNSTABLE,
          "non-finite Hamiltonian: no spectrum bounds");
  // np x 128 blocks in buffers that hold nothing yet: X (np x 2np) and rho_prev
  double* V = c->X;
  double* Wb = c->X + (size_t)np * kCols;
  double* SV = c->rho_prev;
  HIPCHK(c, td::power_start(st, V, kCols, n, np, kCols));
  for (int k = 0; k < kIters; ++k) {
    gemm(c, 0, np, kCols, np, 1.0, c->A, np, V, kCols, Wb, kCols);
    HIPCHK(c, td::power_step(st, Wb, V, kCols, np, kCols, kCols / 2, b[0], b[1]));
  }
  gemm(c, 0, np, kCols, np, 1.0, c->A, np, V, kCols, Wb, kCols);
  gemm(c, 0, np, kCols, np, 1.0, c->S, np, V, kCols, SV, kCols);
  HIPCHK(c, td::rayleigh(st, V, Wb, SV, kCols, np, kCols, c->work1));
  std::vector<double> r(kCols);
  HIPCHK(c, hipMemcpyAsync(r.data(), c->work1, sizeof(double) * kCols, hipMemcpyDeviceToHost, st));
  sync(c);
  double top = -INFINITY, bottom = INFINITY;
  for (int j = 0; j < kCols / 2; ++j) top = std::max(top, r[j]);
  for (int j = kCols / 2; j < kCols; ++j) bottom = std::min(bottom, r[j]);
  REQUIRE(c, std::isfinite(top) && std::isfinite(bottom), TD_EUNSTABLE,
          "non-finite Rayleigh quotients of S^-1 H");
  c->info.width_estimate = std::max(top - bottom, 0.0);
  c->info.stability = c->opt.dt * c->info.width_estimate;
  // X and rho_prev served as scratch: back to zeros (no leapfrog history
  // exists yet, and kernels that cover only the n x n block rely on the
  // padding being zero)
  HIPCHK(c, hipMemsetAsync(c->rho_prev, 0, sizeof(double) * 2 * (size_t)np * np, st));
  HIPCHK(c, hipMemsetAsync(c->X, 0, sizeof(double) * 2 * (size_t)np * np, st));
}

void create_impl(td_ctx* c, const td_system* s_in, const td_options* o) {
  REQUIRE(c, s_in && o, TD_EINVAL, "null system or options");
  REQUIRE(c, (s_in->flags & ~TD_DEVICE_PTRS) == 0, TD_EINVAL, "unknown td_system flags");
  HostModel staged;
  td_system view;
  const td_system* s = s_in;
  const bool dev = (s_in->flags & TD_DEVICE_PTRS) != 0;
  if (dev) {
    view = host_view(c, s_in, o, staged);
    s = &view;
  }
  validate(c, s, o, !dev);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  REQUIRE(c, e == hipSuccess && ndev > 0, TD_EHIP,
          std::string("no HIP device available: ") + hipGetErrorString(e));
  c->opt = *o;
  c->na = s->n_atoms;
  c->n = s->n_orb;
  // c->split switches on only after split_init: the ground state and the
  // inverse run in FP64 and need the reference buffers not yet allocated.
  const bool want_split = o->precision == TD_SPLIT_BF16;
  c->ns = o->n_slices;
  c->ns1 = o->n_slices_dh ? o->n_slices_dh : o->n_slices;
  // every matrix at the 128-wide tile, in both precisions (the split
  // products' exact chunks also end at K segment boundaries, so K needs no
  // coarser padding)
  c->np = round_up(s->n_orb, td::kPad);
  if (s->occ) {
    int n2 = 0;
    while (n2 < s->n_orb && s->occ[n2] == 2.0) ++n2;
    c->nelec = 2 * n2;
  } else {
    c->nelec = s->n_elec;
  }
  const int na = c->na, n = c->n, np = c->np;
  if (o->hip_stream) {
    c->stream = (hipStream_t)o->hip_stream;
  } else {
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  const size_t m2 = (size_t)np * np;
  dalloc(c, &c->S, m2);
  dalloc(c, &c->H0, m2);
  dalloc(c, &c->Sinv, m2);
  dalloc(c, &c->H, m2);
  dalloc(c, &c->A, m2);
  dalloc(c, &c->rho_cur, 2 * m2);
  dalloc(c, &c->rho_prev, 2 * m2);
  dalloc(c, &c->X, 2 * m2);
  dalloc(c, &c->gamma, (size_t)na * na);
  dalloc(c, &c->pos, (size_t)na * 3);
  dalloc(c, &c->q0, na);
  dalloc(c, &c->q_orb, np);
  dalloc(c, &c->dq, na);
  dalloc(c, &c->dq_in, na);
  dalloc(c, &c->v, na);
  dalloc(c, &c->vorb, np);
  dalloc(c, &c->xorb, np);
  dalloc(c, &c->work1, np);
  dalloc(c, &c->work2, np);
  dalloc(c, &c->scal, SC_COUNT);
  dalloc(c, &c->hx, (size_t)8 * na);
  dalloc(c, &c->hf, (size_t)8 * na);
  HIPCHK(c, hipMalloc((void**)&c->orb_off, sizeof(int) * (na + 1)));
  c->orb_off_h.assign(s->orb_offset, s->orb_offset + na + 1);
  c->pos_h.assign(s->positions, s->positions + 3 * na);
  HIPCHK(c, hipMemcpyAsync(c->orb_off, s->orb_offset, sizeof(int) * (na + 1),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->pos, s->positions, sizeof(double) * 3 * na, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->q0, s->q0, sizeof(double) * na, hipMemcpyHostToDevice, c->stream));
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(c, hipMemcpyAsync(c->gamma, s->gamma, sizeof(double) * na * na, kind, c->stream));
  upload_padded(c, s->S, n, c->S, np, kind);
  upload_padded(c, s->H0, n, c->H0, np, kind);
  if (s->rho0)   // staged in X (interleaved n x n) until the inverse is built
    HIPCHK(c, hipMemcpyAsync(c->X, s->rho0, sizeof(double) * 2 * (size_t)n * n, kind,
                             c->stream));
  if (dev) check_device_arrays(c, s->rho0 != nullptr);
  if (s->plus_u != TD_PLUS_U_NONE) setup_plus_u(c, s);
  c->info.n_atoms = na;
  c->info.n_orb = n;
  c->info.n_pad = np;
  c->info.precision = o->precision;
  if (s->rho0) HIPCHK(c, td::interleaved_to_wide(c->stream, c->X, n, c->rho_cur, np));
  inverse_overlap(c);
  if (!s->rho0) {
    ground_state(c);
  }
  refresh(c, true);                        // charges of the initial state
  spectral_width(c);
  if (want_split && !c->ehr_setup) {
    split_init(c);
    c->split = true;
  }
  c->step = 0;
  c->has_prev = false;
  refresh(c, true);
}

// ---------------------------------------------------------------- moving nuclei
td::ModelArgs model_args(td_ctx* c) {
  td::ModelArgs m;
  m.species = c->species;
  m.norb = c->norb;
  m.orb_off = c->orb_off;
  m.atom_of = c->atom_of;
  m.sk_s = c->sk_s;
  m.sk_h = c->sk_h;
  m.scale_s = c->scale_s;
  m.scale_h = c->scale_h;
  m.onsite = c->onsite;
  m.na = c->na;
  m.nsp = c->nsp;
  m.n = c->n;
  m.decay = c->decay;
  m.fd_step = std::pow(2.220446049250313e-16, 0.25);   // eps^(1/4) (Sec. 2.3, Eq. 20)
  return m;
}

// S, H0, their gradients, gamma and S^-1 at the current positions.
void rebuild_model(td_ctx* c, bool warm) {
  HIPCHK(c, td::model_build(c->stream, model_args(c), c->pos, c->S, c->H0, c->GS, c->GH, c->np));
  HIPCHK(c, td::gamma_build(c->stream, c->pos, c->na, c->hub_u, c->gamma, c->dgamma));
  inverse_overlap(c, warm);
}

// One moving-nuclei step (r18) in phases, shared by one trajectory and by
// batches of them. Between the phases come the step's products: one
// trajectory runs each on its own, a batch runs each over all its members
// in one grouped launch, with the same arithmetic (the same MFMA sequence
// over k for every element).
//   phase_h:       charges (dipole -> mu), energy (-> energy3, optional),
//                  potential with the field E, H
//                     then A = S^-1 H and X = A rho
//   phase_forces:  W = sym Re X and the forces (Sec. 2.1, Eq. 15 without
//                  velocity terms)
//   phase_nac:     v_k (velocity Verlet), kinetic energy, D from v_k
//                     then A = S^-1 D and Z = A rho
//   phase_move:    leapfrog with X - iZ (Sec. 2.1, Eq. 10; Sec. 2.3,
//                  Eq. 19), v_{k+1/2}, drift, S, H0, gradients and gamma at
//                  R_{k+1}
//                     then the Newton-Schulz update of S^-1
// out = A [Re rho | Im rho] (np x 2np) as a split-bf16 product, for moving
// nuclei: there is no fixed reference (S, H0 and S^-1 change every step),
// so rho itself is sliced. rho is Hermitian, so the rows of Re rho and of
// -Im rho are the columns of the two halves of the right operand. With
// `slice_rho` false the slices of rho from the previous call are reused
// (rho unchanged in between).
void ehr_split_product(td_ctx* c, const double* A, double* out, bool slice_rho) {
  const int np = c->np, S = c->ns;
  if (slice_rho) {
    td::SliceSrc re;
    re.M0 = c->rho_cur;
    re.ld0 = 2 * np;
    slice(c, td::SLICE_PLAIN, re, np, np, c->sl_R2, np * S, c->e_R2);
    td::SliceSrc im;
    im.M0 = c->rho_cur + np;
    im.ld0 = 2 * np;
    im.sign = -1.0;
    slice(c, td::SLICE_PLAIN, im, np, np, c->sl_R2 + (size_t)np * np * S, np * S, c->e_R2 + np);
  }
  td::SliceSrc a;
  a.M0 = A;
  a.ld0 = np;
  slice(c, td::SLICE_PLAIN, a, np, np, c->sl_L2, np * S, c->e_L2);
  td::SplitGemm g;
  g.m = np;
  g.n = 2 * np;
  g.L = c->sl_L2;
  g.ldl = np * S;
  g.eL = c->e_L2;
  g.R = c->sl_R2;
  g.ldr = np * S;
  g.fR = c->e_R2;
  g.seg_len = np;
  g.k_lo = np;
  g.k_hi = np;
  g.n_split = 2 * np;
  g.C = out;
  g.ldc = 2 * np;
  HIPCHK(c, td::split_gemm(c->stream, S, g));
}

void ehr_phase_h(td_ctx* c, const double* E, double* mu, double* energy3) {
  hipStream_t st = c->stream;
  const int np = c->np, na = c->na;
  mulliken(c, mu);
  if (energy3) {
    HIPCHK(c, td::potential(st, c->gamma, c->dq, c->pos, nullptr, c->orb_off, na, c->v, c->vorb));
    HIPCHK(c, td::rowdot(st, c->rho_cur, 2 * np, c->H0, np, c->work1, np, np));
    HIPCHK(c, td::energy_terms(st, c->work1, np, c->dq, c->v, c->pos, E, na, energy3));
  }
  HIPCHK(c, td::potential(st, c->gamma, c->dq, c->pos, E, c->orb_off, na, c->v, c->vorb));
  HIPCHK(c, td::assemble_h(st, c->H0, c->S, c->vorb, c->H, np));
}

// energy4: the step's four energy terms (band, Coulomb, field, E_rep), or
// null when no energy is recorded.
void ehr_phase_forces(td_ctx* c, const double* E, double* energy4) {
  hipStream_t st = c->stream;
  const int np = c->np;
  HIPCHK(c, td::pair_sym(st, c->X, 2 * np, c->W, nullptr, np, np));
  HIPCHK(c, td::ehrenfest_forces(st, c->rho_cur, 2 * np, c->W, c->GS, c->GH, c->vorb, c->orb_off,
                                 c->dq, c->dgamma, E, c->na, c->n, np, c->F));
  if (c->rep_a)   // -grad E_rep (Eq. 15) and E_rep itself
    HIPCHK(c, td::repulsion(st, c->pos, c->species, c->rep_a, c->nsp, c->rep_decay, c->na, c->F,
                            c->e_rep_atom, energy4 ? energy4 + 3 : c->scal + SC_EREP));
}

void ehr_phase_nac(td_ctx* c, int k) {
  hipStream_t st = c->stream;
  const int na = c->na;
  if (c->vel_half)
    HIPCHK(c, td::kick_nuclei(st, c->vel, c->F, c->species, c->mass, na, 0.5 * c->opt.dt));  // v_k
  HIPCHK(c, td::kinetic_energy(st, c->vel, c->F, c->species, c->mass, na, 0.0, c->e_kin + k));
  HIPCHK(c, td::nac_build(st, c->GS, c->vel, c->atom_of, c->n, c->np, c->Dm));
}

void ehr_phase_move(td_ctx* c) {
  hipStream_t st = c->stream;
  const int np = c->np, na = c->na;
  const double dt = c->opt.dt;
  // the leapfrog pass stages X - i Z (the coupling term) as it reads X
  if (c->has_prev) {
    HIPCHK(c, td::pair_leapfrog(st, c->X, c->X + np, 2 * np, c->rho_prev, c->rho_prev + np,
                                2 * np, c->rho_prev, c->rho_prev + np, 2 * np, np, 2.0 * dt,
                                nullptr, 0, c->Z, c->Z + np, 2 * np));
  } else {
    HIPCHK(c, td::pair_leapfrog(st, c->X, c->X + np, 2 * np, c->rho_cur, c->rho_cur + np,
                                2 * np, c->rho_prev, c->rho_prev + np, 2 * np, np, dt, nullptr, 0,
                                c->Z, c->Z + np, 2 * np));
    c->has_prev = true;
  }
  std::swap(c->rho_cur, c->rho_prev);
  HIPCHK(c, td::kick_nuclei(st, c->vel, c->F, c->species, c->mass, na, 0.5 * dt));  // v_{k+1/2}
  HIPCHK(c, td::drift_nuclei(st, c->pos, c->vel, na, dt));
  c->vel_half = true;
  HIPCHK(c, td::model_build(st, model_args(c), c->pos, c->S, c->H0, c->GS, c->GH, np));
  HIPCHK(c, td::gamma_build(st, c->pos, na, c->hub_u, c->gamma, c->dgamma));
}

// Charges (dipole -> mu), H with field E, X = (S^-1 H) rho_cur, W = sym Re X and
// the forces F of the current state (Sec. 2.1, Eq. 15 without velocity terms).
void ehr_forces(td_ctx* c, const double* E, double* mu, double* energy4) {
  const int np = c->np;
  ehr_phase_h(c, E, mu, energy4);
  gemm(c, 1, np, np, np, 1.0, c->Sinv, np, c->H, np, c->A, np);
  if (c->ehr_split)
    ehr_split_product(c, c->A, c->X, true);
  else
    gemm(c, 2, np, 2 * np, np, 1.0, c->A, np, c->rho_cur, 2 * np, c->X, 2 * np);
  ehr_phase_forces(c, E, energy4);
}

// One Ehrenfest step k (model matrices current at R_k): forces, velocity
// Verlet around the leapfrog step of rho with the coupling D (Sec. 2.1,
// Eqs. 10, 14, 15; Sec. 2.3, Eq. 19), then the matrices at R_{k+1}.
void ehr_step(td_ctx* c, int k, const double* E) {
  const int np = c->np;
  ehr_forces(c, E, c->dip + 3 * (size_t)k, c->e_el + 4 * (size_t)k);
  ehr_phase_nac(c, k);
  // X += -i S^-1 D rho with D from v_k
  gemm(c, 0, np, np, np, 1.0, c->Sinv, np, c->Dm, np, c->A, np);
  if (c->ehr_split)
    ehr_split_product(c, c->A, c->Z, false);
  else
    gemm(c, 0, np, 2 * np, np, 1.0, c->A, np, c->rho_cur, 2 * np, c->Z, 2 * np);
  ehr_phase_move(c);
  inverse_overlap(c, true);
}

// Device series of the dipole (and, with moving nuclei, the energies) for
// nsteps steps.
void ensure_series(td_ctx* c, int nsteps) {
  if (c->dip_cap >= nsteps) return;
  if (c->dip) (void)hipFree(c->dip);
  c->dip = nullptr;
  c->dip_cap = 0;
  dalloc(c, &c->dip, 3 * (size_t)nsteps);
  if (c->ehr) {
    if (c->e_kin) (void)hipFree(c->e_kin);
    if (c->e_el) (void)hipFree(c->e_el);
    c->e_kin = c->e_el = nullptr;
    dalloc(c, &c->e_kin, (size_t)nsteps);
    dalloc(c, &c->e_el, 4 * (size_t)nsteps);
  }
  c->dip_cap = nsteps;
}

void step_impl(td_ctx* c, int nsteps, const double* field) {
  REQUIRE(c, nsteps >= 0, TD_EINVAL, "n must be >= 0");
  if (!(c->info.stability < 1.0)) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "time step %.4g too large for the leapfrog: the spectrum of S^-1 H is at least "
                  "%.4g wide, and dt times that width is %.3g (must be below 1)",
                  c->opt.dt, c->info.width_estimate, c->info.stability);
    REQUIRE(c, false, TD_EUNSTABLE, msg);
  }
  if (nsteps == 0) {
    c->last_n = 0;     // an empty call records no dipoles (or energies)
    return;
  }
  if (field) {
    REQUIRE(c, finite_all(field, 3 * (size_t)nsteps), TD_EINVAL, "non-finite field");
    // the field's potential R_A . E widens the spectrum of S^-1 H by about
    // its spread over the atoms (Sec. 2.1, Eq. 7)
    const double spread = tdi::field_spread(c, field, nsteps);
    const double st = c->opt.dt * (c->info.width_estimate + spread);
    if (!(st < 1.0)) {
      char msg[300];
      std::snprintf(msg, sizeof(msg),
                    "time step %.4g too large for the leapfrog under this field: the spectrum of "
                    "S^-1 H is at least %.4g wide, the field spreads the atomic potentials R . E "
                    "over up to %.4g, and dt times their sum is %.3g (must be below 1)",
                    c->opt.dt, c->info.width_estimate, spread, st);
      REQUIRE(c, false, TD_EUNSTABLE, msg);
    }
  }
  const int na = c->na, np = c->np;
  if (field && c->field_cap < nsteps) {
    if (c->field) (void)hipFree(c->field);
    c->field = nullptr;
    c->field_cap = 0;
    dalloc(c, &c->field, 3 * (size_t)nsteps);
    c->field_cap = nsteps;
  }
  ensure_series(c, nsteps);
  if (field)
    HIPCHK(c, hipMemcpyAsync(c->field, field, sizeof(double) * 3 * nsteps, hipMemcpyHostToDevice,
                             c->stream));
  const bool prof = c->opt.profile != 0;
  // events per step: start | G1 | G1 end | G2 | G2 end | update end
  if (prof) ensure_events(c, 6 * (size_t)nsteps);
  hipStream_t st = c->stream;
  if (c->ehr) {
    for (int k = 0; k < nsteps; ++k) {
      ehr_step(c, k, field ? c->field + 3 * (size_t)k : nullptr);
      c->step += 1;
    }
    c->last_n = nsteps;
    HIPCHK(c, hipMemcpyAsync(c->pos_h.data(), c->pos, sizeof(double) * 3 * na,
                             hipMemcpyDeviceToHost, st));
    refresh(c);
    return;
  }
  for (int k = 0; k < nsteps; ++k) {
    hipEvent_t* e = prof ? &c->ev[6 * (size_t)k] : nullptr;
    if (prof) HIPCHK(c, hipEventRecord(e[0], st));
    // charges and dipole of rho_k, SCC potential, Hamiltonian (Eqs. 5-7)
    mulliken(c, c->dip + 3 * (size_t)k);
    const double* Ek = field ? c->field + 3 * (size_t)k : nullptr;
    if (c->split) {
      split_products(c, Ek, e);
    } else {
      HIPCHK(c, td::potential(st, c->gamma, c->dq, c->pos, Ek, c->orb_off, na, c->v, c->vorb));
      if (c->plus_u != TD_PLUS_U_NONE) block_pops(c, c->sh_n);
      assemble_hamiltonian(c, c->sh_n);
      if (prof) HIPCHK(c, hipEventRecord(e[1], st));
      // X = S^-1 H rho (Eq. 10), as A = S^-1 H then A [Re rho | Im rho]
      gemm(c, 1, np, np, np, 1.0, c->Sinv, np, c->H, np, c->A, np);
      if (prof) HIPCHK(c, hipEventRecord(e[2], st));
      if (prof) HIPCHK(c, hipEventRecord(e[3], st));
      gemm(c, 2, np, 2 * np, np, 1.0, c->A, np, c->rho_cur, 2 * np, c->X, 2 * np);
      if (prof) HIPCHK(c, hipEventRecord(e[4], st));
    }
    // rho_{k+1} = rho_{k-1} + 2 dt rhodot (Eq. 19); Euler start without history
    // split products leave out X_ref = A_ref rho_ref (real); it is added here
    const double* xref = c->split ? c->Xref : nullptr;
    if (c->has_prev) {
      HIPCHK(c, td::pair_leapfrog(st, c->X, c->X + np, 2 * np, c->rho_prev, c->rho_prev + np,
                                  2 * np, c->rho_prev, c->rho_prev + np, 2 * np, np,
                                  2.0 * c->opt.dt, xref, 2 * np));
    } else {
      HIPCHK(c, td::pair_leapfrog(st, c->X, c->X + np, 2 * np, c->rho_cur, c->rho_cur + np,
                                  2 * np, c->rho_prev, c->rho_prev + np, 2 * np, np, c->opt.dt,
                                  xref, 2 * np));
      c->has_prev = true;
    }
    std::swap(c->rho_cur, c->rho_prev);
    if (prof) HIPCHK(c, hipEventRecord(e[5], st));
    c->step += 1;
  }
  c->last_n = nsteps;
  refresh(c);
  if (prof) {
    for (int k = 0; k < nsteps; ++k) {
      hipEvent_t* e = &c->ev[6 * (size_t)k];
      float ms[5];
      for (int q = 0; q < 5; ++q) HIPCHK(c, hipEventElapsedTime(&ms[q], e[q], e[q + 1]));
      c->kt_ms[TD_KT_OTHER] += ms[0] + ms[2];
      c->kt_ms[TD_KT_GEMM_SH] += ms[1];
      c->kt_ms[TD_KT_GEMM_ARHO] += ms[3];
      c->kt_ms[TD_KT_UPDATE] += ms[4];
      for (int q = 0; q < TD_KT_COUNT; ++q) c->kt_n[q] += 1;
    }
  }
}

void kick_impl(td_ctx* c, double e0, const double* dir) {
  REQUIRE(c, dir && std::isfinite(e0), TD_EINVAL, "invalid kick arguments");
  const double nrm = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  REQUIRE(c, nrm > 0 && std::isfinite(nrm), TD_EINVAL, "kick direction must be non-zero");
  const int np = c->np;
  std::vector<double> x(np, 0.0);
  for (int a = 0; a < c->na; ++a) {
    const double xa = (c->pos_h[3 * a] * dir[0] + c->pos_h[3 * a + 1] * dir[1] +
                       c->pos_h[3 * a + 2] * dir[2]) / nrm;
    for (int u = c->orb_off_h[a]; u < c->orb_off_h[a + 1]; ++u) x[u] = xa;
  }
  HIPCHK(c, hipMemcpyAsync(c->xorb, x.data(), sizeof(double) * np, hipMemcpyHostToDevice,
                           c->stream));
  // rho(0+) = 1/2 (T + T^+), T = S^-1 K S rho K^+ (Sec. 2.2, Eq. 16), in FP64
  const double* full = c->rho_cur;
  if (c->split) {
    full_density(c, c->rho_cur, c->stage);
    full = c->stage;
  }
  gemm(c, 0, np, 2 * np, np, 1.0, c->S, np, full, 2 * np, c->X, 2 * np);
  HIPCHK(c, td::kick_phase(c->stream, c->X, c->X + np, 2 * np, c->xorb, np, e0));
  gemm(c, 0, np, 2 * np, np, 1.0, c->Sinv, np, c->X, 2 * np, c->rho_prev, 2 * np);
  HIPCHK(c, td::pair_herm(c->stream, c->rho_prev, c->rho_prev + np, 2 * np, c->rho_cur,
                          c->rho_cur + np, 2 * np, np));
  if (c->split) HIPCHK(c, td::wide_add_real(c->stream, c->rho_cur, c->rho_ref, np, -1.0));
  c->has_prev = false;
  sync(c);
  refresh(c, true);
}

// Host-pointer split-bf16 product for td_util_gemm: A rows and B columns
// (B transposed on the host) are sliced on the device.
void split_gemm_host(td_ctx* c, int ns, int m, int n, int k, const double* A, const double* B,
                     double* C) {
  const int mp = round_up(m, 128), npd = round_up(n, 128), kp = round_up(k, 128);
  std::vector<double> bt((size_t)n * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < n; ++j) bt[(size_t)j * k + i] = B[(size_t)i * n + j];
  dalloc(c, &c->S, (size_t)mp * kp);
  dalloc(c, &c->H, (size_t)npd * kp);
  dalloc(c, &c->A, (size_t)mp * npd);
  HIPCHK(c, hipMemcpy2DAsync(c->S, sizeof(double) * kp, A, sizeof(double) * k,
                             sizeof(double) * k, m, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpy2DAsync(c->H, sizeof(double) * kp, bt.data(), sizeof(double) * k,
                             sizeof(double) * k, n, hipMemcpyHostToDevice, c->stream));
  __bf16 *ls = nullptr, *rs = nullptr;
  int *el = nullptr, *fr = nullptr;
  const size_t lsz = (size_t)mp * kp, rsz = (size_t)npd * kp;
  HIPCHK(c, hipMalloc((void**)&ls, sizeof(__bf16) * lsz * ns));
  HIPCHK(c, hipMalloc((void**)&rs, sizeof(__bf16) * rsz * ns));
  HIPCHK(c, hipMalloc((void**)&el, sizeof(int) * mp));
  HIPCHK(c, hipMalloc((void**)&fr, sizeof(int) * npd));
  struct Free {
    void* p[4];
    ~Free() {
      for (void* q : p)
        if (q) (void)hipFree(q);
    }
  } guard{{ls, rs, el, fr}};
  td::SliceSrc sa;
  sa.M0 = c->S;
  sa.ld0 = kp;
  HIPCHK(c, td::slice_rows(c->stream, ns, td::SLICE_PLAIN, sa, mp, kp, ls, kp * ns, el));
  td::SliceSrc sb;
  sb.M0 = c->H;
  sb.ld0 = kp;
  HIPCHK(c, td::slice_rows(c->stream, ns, td::SLICE_PLAIN, sb, npd, kp, rs, kp * ns, fr));
  td::SplitGemm g;
  g.m = mp;
  g.n = npd;
  g.L = ls;
  g.ldl = kp * ns;
  g.eL = el;
  g.eL_stride = 0;
  g.R = rs;
  g.ldr = kp * ns;
  g.fR = fr;
  g.fR_stride = 0;
  g.seg_len = kp;
  g.k_lo = kp;
  g.k_hi = kp;
  g.n_split = npd;
  g.C = c->A;
  g.ldc = npd;
  HIPCHK(c, td::split_gemm(c->stream, ns, g));
  HIPCHK(c, hipMemcpy2DAsync(C, sizeof(double) * n, c->A, sizeof(double) * npd,
                             sizeof(double) * n, m, hipMemcpyDeviceToHost, c->stream));
  sync(c);
}

// Host checks of a two-centre model against the system's layout.
void validate_model(td_ctx* c, const td_system* s, const td_model* m) {
  REQUIRE(c, s && m, TD_EINVAL, "null system or model");
  REQUIRE(c, s->n_atoms > 0 && s->n_orb > 0 && s->positions && s->orb_offset && s->q0,
          TD_EINVAL, "null array in td_system");
  REQUIRE(c, m->n_species > 0 && m->species && m->species_norb && m->sk_s && m->sk_h &&
                 m->scale_s && m->scale_h && m->onsite && m->mass,
          TD_EINVAL, "null array in td_model");
  const int na = s->n_atoms, nsp = m->n_species;
  for (int k = 0; k < nsp; ++k) {
    REQUIRE(c, m->species_norb[k] == 1 || m->species_norb[k] == 4, TD_EINVAL,
            "species_norb must be 1 or 4");
    REQUIRE(c, m->mass[k] > 0 && std::isfinite(m->mass[k]), TD_EINVAL, "masses must be positive");
  }
  REQUIRE(c, s->orb_offset[0] == 0, TD_EINVAL, "orb_offset must start at 0");
  for (int a = 0; a < na; ++a) {
    REQUIRE(c, m->species[a] >= 0 && m->species[a] < nsp, TD_EINVAL, "species out of range");
    REQUIRE(c, s->orb_offset[a + 1] - s->orb_offset[a] == m->species_norb[m->species[a]],
            TD_EINVAL, "orb_offset does not match the species' orbital counts");
  }
  REQUIRE(c, s->orb_offset[na] == s->n_orb, TD_EINVAL, "orb_offset must end at n_orb");
  REQUIRE(c, m->decay > 0 && std::isfinite(m->decay) && m->hubbard_u > 0 &&
                 std::isfinite(m->hubbard_u),
          TD_EINVAL, "decay and hubbard_u must be positive");
  REQUIRE(c, finite_all(m->sk_s, (size_t)nsp * nsp * 4) && finite_all(m->sk_h, (size_t)nsp * nsp * 4) &&
                 finite_all(m->onsite, (size_t)nsp * 2) &&
                 finite_all(m->scale_s, (size_t)na * na) && finite_all(m->scale_h, (size_t)na * na) &&
                 finite_all(s->positions, (size_t)na * 3),
          TD_EINVAL, "non-finite model or positions");
  if (m->rep_a) {
    REQUIRE(c, finite_all(m->rep_a, (size_t)nsp * nsp) && m->rep_decay > 0 &&
                   std::isfinite(m->rep_decay),
            TD_EINVAL, "rep_a must be finite and rep_decay positive");
    for (int i = 0; i < nsp; ++i)
      for (int j = 0; j < nsp; ++j)
        REQUIRE(c, m->rep_a[i * nsp + j] >= 0 && m->rep_a[i * nsp + j] == m->rep_a[j * nsp + i],
                TD_EINVAL, "rep_a must be symmetric and non-negative");
  }
  for (int a = 0; a < na; ++a)
    for (int b = a + 1; b < na; ++b) {
      const double* p = s->positions;
      const double d0 = p[3 * b] - p[3 * a], d1 = p[3 * b + 1] - p[3 * a + 1],
                   d2 = p[3 * b + 2] - p[3 * a + 2];
      REQUIRE(c, d0 * d0 + d1 * d1 + d2 * d2 > 1e-6, TD_EINVAL, "two atoms at one position");
    }
}

// Model arrays, gradients and nuclear state on the device of context c.
void upload_model(td_ctx* c, const td_system* s, const td_model* m, const double* vel) {
  const int na = s->n_atoms, nsp = m->n_species, n = s->n_orb;
  c->nsp = nsp;
  c->decay = m->decay;
  c->hub_u = m->hubbard_u;
  ialloc(c, &c->species, na);
  ialloc(c, &c->norb, nsp);
  ialloc(c, &c->atom_of, c->np);
  dalloc(c, &c->sk_s, (size_t)nsp * nsp * 4);
  dalloc(c, &c->sk_h, (size_t)nsp * nsp * 4);
  dalloc(c, &c->scale_s, (size_t)na * na);
  dalloc(c, &c->scale_h, (size_t)na * na);
  dalloc(c, &c->onsite, (size_t)nsp * 2);
  dalloc(c, &c->mass, nsp);
  if (m->rep_a) {
    dalloc(c, &c->rep_a, (size_t)nsp * nsp);
    dalloc(c, &c->e_rep_atom, na);
    c->rep_decay = m->rep_decay;
  }
  dalloc(c, &c->GS, 3 * (size_t)c->np * c->np);
  dalloc(c, &c->GH, 3 * (size_t)c->np * c->np);
  dalloc(c, &c->dgamma, 3 * (size_t)na * na);
  dalloc(c, &c->vel, 3 * (size_t)na);
  dalloc(c, &c->F, 3 * (size_t)na);
  std::vector<int> atom(c->np, 0);
  for (int a = 0; a < na; ++a)
    for (int u = s->orb_offset[a]; u < s->orb_offset[a + 1]; ++u) atom[u] = a;
  (void)n;
  hipStream_t st = c->stream;
  HIPCHK(c, hipMemcpyAsync(c->species, m->species, sizeof(int) * na, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->norb, m->species_norb, sizeof(int) * nsp, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->atom_of, atom.data(), sizeof(int) * c->np, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->sk_s, m->sk_s, sizeof(double) * nsp * nsp * 4, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->sk_h, m->sk_h, sizeof(double) * nsp * nsp * 4, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->scale_s, m->scale_s, sizeof(double) * na * na, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->scale_h, m->scale_h, sizeof(double) * na * na, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->onsite, m->onsite, sizeof(double) * nsp * 2, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->mass, m->mass, sizeof(double) * nsp, hipMemcpyHostToDevice, st));
  if (m->rep_a)
    HIPCHK(c, hipMemcpyAsync(c->rep_a, m->rep_a, sizeof(double) * nsp * nsp,
                             hipMemcpyHostToDevice, st));
  if (vel)
    HIPCHK(c, hipMemcpyAsync(c->vel, vel, sizeof(double) * 3 * na, hipMemcpyHostToDevice, st));
}

void create_ehr_impl(td_ctx* c, const td_system* s, const td_model* m, const double* vel,
                     const td_options* o) {
  REQUIRE(c, o, TD_EINVAL, "null options");
  REQUIRE(c, s && (s->flags & TD_DEVICE_PTRS) == 0, TD_EINVAL,
          "moving-nuclei contexts take host pointers");
  validate_model(c, s, m);
  REQUIRE(c, o->precision == TD_FP64 || o->precision == TD_SPLIT_BF16, TD_EINVAL,
          "unknown precision");
  REQUIRE(c, o->precision == TD_FP64 || (o->n_slices >= 3 && o->n_slices <= 5), TD_EINVAL,
          "n_slices must be 3, 4 or 5");
  REQUIRE(c, s->plus_u == TD_PLUS_U_NONE, TD_ENOTSUP,
          "moving nuclei have no on-site corrections (plus_u)");
  if (vel) REQUIRE(c, finite_all(vel, 3 * (size_t)s->n_atoms), TD_EINVAL, "non-finite velocities");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  REQUIRE(c, e == hipSuccess && ndev > 0, TD_EHIP,
          std::string("no HIP device available: ") + hipGetErrorString(e));
  // S, H0 and gamma at the initial positions, built on the device
  const int na = s->n_atoms, n = s->n_orb;
  std::vector<double> hS((size_t)n * n), hH((size_t)n * n), hG((size_t)na * na);
  {
    td_ctx b;
    b.na = na;
    b.n = n;
    b.np = round_up(n, td::kPad);
    struct Free {
      td_ctx* p;
      ~Free() {
        if (p->stream) (void)hipStreamSynchronize(p->stream);
        free_all(p);
      }
    } guard{&b};
    try {
      HIPCHK(&b, hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
      b.own_stream = true;
      const size_t m2 = (size_t)b.np * b.np;
      dalloc(&b, &b.S, m2);
      dalloc(&b, &b.H0, m2);
      dalloc(&b, &b.gamma, (size_t)na * na);
      dalloc(&b, &b.pos, 3 * (size_t)na);
      HIPCHK(&b, hipMalloc((void**)&b.orb_off, sizeof(int) * (na + 1)));
      HIPCHK(&b, hipMemcpyAsync(b.orb_off, s->orb_offset, sizeof(int) * (na + 1),
                                hipMemcpyHostToDevice, b.stream));
      HIPCHK(&b, hipMemcpyAsync(b.pos, s->positions, sizeof(double) * 3 * na,
                                hipMemcpyHostToDevice, b.stream));
      upload_model(&b, s, m, nullptr);
      HIPCHK(&b, td::model_build(b.stream, model_args(&b), b.pos, b.S, b.H0, b.GS, b.GH, b.np));
      HIPCHK(&b, td::gamma_build(b.stream, b.pos, na, b.hub_u, b.gamma, b.dgamma));
      HIPCHK(&b, hipMemcpy2DAsync(hS.data(), sizeof(double) * n, b.S, sizeof(double) * b.np,
                                  sizeof(double) * n, n, hipMemcpyDeviceToHost, b.stream));
      HIPCHK(&b, hipMemcpy2DAsync(hH.data(), sizeof(double) * n, b.H0, sizeof(double) * b.np,
                                  sizeof(double) * n, n, hipMemcpyDeviceToHost, b.stream));
      HIPCHK(&b, hipMemcpyAsync(hG.data(), b.gamma, sizeof(double) * na * na,
                                hipMemcpyDeviceToHost, b.stream));
      HIPCHK(&b, hipStreamSynchronize(b.stream));
    } catch (const Fail& f) {
      c->err = b.err;
      throw;
    }
  }
  td_system view = *s;
  view.S = hS.data();
  view.H0 = hH.data();
  view.gamma = hG.data();
  c->ehr_setup = true;                     // split precision: no reference form
  create_impl(c, &view, o);
  upload_model(c, s, m, vel);
  const size_t m2 = (size_t)c->np * c->np;
  if (o->precision == TD_SPLIT_BF16) {
    salloc(c, &c->sl_L2, (size_t)c->ns * m2);
    salloc(c, &c->sl_R2, (size_t)c->ns * 2 * m2);
    ialloc(c, &c->e_L2, c->np);
    ialloc(c, &c->e_R2, 2 * (size_t)c->np);
    c->ehr_split = true;
  }
  dalloc(c, &c->W, m2);
  dalloc(c, &c->Dm, m2);
  dalloc(c, &c->Sinv_prev, m2);
  dalloc(c, &c->Sinv_prev2, m2);
  c->sinv_hist = 0;
  dalloc(c, &c->Z, 2 * m2);
  c->ehr = true;
  c->vel_half = false;
  rebuild_model(c, true);
  c->sinv_hist = 0;   // that refinement is at the starting positions: no trajectory yet
  refresh(c, true);
}

}  // namespace

namespace tdi {
void sync_ctx(td_ctx* c) { sync(c); }
void refresh_ctx(td_ctx* c) { refresh(c); }

void ehr_group_alloc(td_ctx* c, EhrGroup& g, int nm) {
  g.per = nm;
  g.slots = 16;
  HIPCHK(c, hipMalloc((void**)&g.dev, sizeof(td::GemmProblem) * (size_t)g.slots * nm));
  HIPCHK(c, hipHostMalloc((void**)&g.host, sizeof(td::GemmProblem) * (size_t)g.slots * nm,
                          hipHostMallocDefault));
  HIPCHK(c, hipHostMalloc((void**)&g.res_host, sizeof(double) * nm, hipHostMallocDefault));
  HIPCHK(c, hipEventCreateWithFlags(&g.fork, hipEventDisableTiming));
  for (int i = 0; i < EhrGroup::kLanes; ++i) {
    HIPCHK(c, hipStreamCreateWithFlags(&g.lane[i], hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&g.join[i], hipEventDisableTiming));
  }
}

void ehr_group_free(EhrGroup& g) {
  for (int i = 0; i < EhrGroup::kLanes; ++i) {
    if (g.lane[i]) {
      (void)hipStreamSynchronize(g.lane[i]);
      (void)hipStreamDestroy(g.lane[i]);
    }
    if (g.join[i]) (void)hipEventDestroy(g.join[i]);
  }
  if (g.fork) (void)hipEventDestroy(g.fork);
  if (g.dev) (void)hipFree(g.dev);
  if (g.host) (void)hipHostFree(g.host);
  if (g.res_host) (void)hipHostFree(g.res_host);
  g = EhrGroup{};
}

namespace {

// One grouped launch of the problems in `pr` through the next table slot;
// slots are reused only after the stream has been synchronised.
void grouped_launch(td_ctx* c0, EhrGroup& g, std::vector<td::GemmProblem>& pr, int tile) {
  if (pr.empty()) return;
  REQUIRE(c0, g.used < g.slots && (int)pr.size() <= g.per, TD_EHIP,
          "internal: grouped product tables exhausted");
  int t = 0;
  for (auto& q : pr) {
    q.tile0 = t;
    t += q.upper ? q.tiles_n * (q.tiles_n + 1) / 2 : q.tiles_m * q.tiles_n;
  }
  td::GemmProblem* h = g.host + (size_t)g.used * g.per;
  td::GemmProblem* d = g.dev + (size_t)g.used * g.per;
  std::copy(pr.begin(), pr.end(), h);
  HIPCHK(c0, hipMemcpyAsync(d, h, sizeof(td::GemmProblem) * pr.size(), hipMemcpyHostToDevice,
                            c0->stream));
  HIPCHK(c0, td::dgemm_grouped(c0->stream, tile, d, (int)pr.size(), t));
  g.used += 1;
  pr.clear();
}

td::GemmProblem problem(const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                        int rows, int cols, int K, int tile, int upper) {
  td::GemmProblem q{};
  q.A = A;
  q.B = B;
  q.C = C;
  q.lda = lda;
  q.ldb = ldb;
  q.ldc = ldc;
  q.K = K;
  q.tiles_m = rows / tile;
  q.tiles_n = cols / tile;
  q.upper = upper;
  return q;
}

}  // namespace

void ehr_batch_steps(std::vector<td_ctx*>& mem, EhrGroup& g, int nsteps, const double* field,
                     std::string& err) {
  const int nm = (int)mem.size();
  td_ctx* c0 = mem[0];
  hipStream_t st = c0->stream;
  const int np = c0->np;
  constexpr int T = 128;       // np is a multiple of 128; 64 and 128 tiles give the same sums
  // The per-member passes between two grouped launches: member m runs on
  // lane m mod kLanes (its context's stream switched for the duration), the
  // lanes start after the work already on the batch stream and the batch
  // stream waits for all of them. Each member's kernels keep their order.
  auto each = [&](auto&& f) {
    HIPCHK(c0, hipEventRecord(g.fork, st));
    for (int i = 0; i < EhrGroup::kLanes; ++i) HIPCHK(c0, hipStreamWaitEvent(g.lane[i], g.fork, 0));
    for (int m = 0; m < nm; ++m) {
      td_ctx* c = mem[m];
      c->stream = g.lane[m % EhrGroup::kLanes];
      try {
        f(c, m);
      } catch (const Fail&) {
        c->stream = st;
        err = "member " + std::to_string(m) + ": " + c->err;
        throw;
      }
      c->stream = st;
    }
    for (int i = 0; i < EhrGroup::kLanes; ++i) {
      HIPCHK(c0, hipEventRecord(g.join[i], g.lane[i]));
      HIPCHK(c0, hipStreamWaitEvent(st, g.join[i], 0));
    }
  };
  std::vector<td::GemmProblem> pr;
  std::vector<NsIter> ns(nm);
  std::vector<char> active(nm);
  std::vector<int> upd;
  g.used = 0;
  for (int k = 0; k < nsteps; ++k) {
    const double* E = field ? field + 3 * (size_t)k : nullptr;
    each([&](td_ctx* c, int) { ehr_phase_h(c, E, c->dip + 3 * (size_t)k, c->e_el + 4 * (size_t)k); });
    for (td_ctx* c : mem) pr.push_back(problem(c->Sinv, np, c->H, np, c->A, np, np, np, np, T, 0));
    grouped_launch(c0, g, pr, T);                                   // A = S^-1 H
    if (c0->ehr_split) {
      each([&](td_ctx* c, int) { ehr_split_product(c, c->A, c->X, true); });
    } else {
      for (td_ctx* c : mem)
        pr.push_back(problem(c->A, np, c->rho_cur, 2 * np, c->X, 2 * np, np, 2 * np, np, T, 0));
      grouped_launch(c0, g, pr, T);                                 // X = A rho
    }
    each([&](td_ctx* c, int) {
      ehr_phase_forces(c, E, c->e_el + 4 * (size_t)k);
      ehr_phase_nac(c, k);
    });
    for (td_ctx* c : mem) pr.push_back(problem(c->Sinv, np, c->Dm, np, c->A, np, np, np, np, T, 0));
    grouped_launch(c0, g, pr, T);                                   // A = S^-1 D
    if (c0->ehr_split) {
      each([&](td_ctx* c, int) { ehr_split_product(c, c->A, c->Z, false); });
    } else {
      for (td_ctx* c : mem)
        pr.push_back(problem(c->A, np, c->rho_cur, 2 * np, c->Z, 2 * np, np, 2 * np, np, T, 0));
      grouped_launch(c0, g, pr, T);                                 // Z = A rho
    }
    each([&](td_ctx* c, int) { ehr_phase_move(c); });
    // S^-1 at R_{k+1}: each member takes the decisions of one trajectory
    // (ns_decide), with one host synchronisation per round for all of them
    each([&](td_ctx* c, int m) {
      ns_begin(c, true, ns[m]);
      active[m] = 1;
    });
    for (;;) {
      for (int m = 0; m < nm; ++m)
        if (active[m]) {
          td_ctx* c = mem[m];
          pr.push_back(problem(c->S, np, c->Sinv, np, c->A, np, np, np, np, T, 0));
        }
      grouped_launch(c0, g, pr, T);                                 // T = S X
      each([&](td_ctx* c, int m) {
        if (!active[m]) return;
        ns_residual(c);
        HIPCHK(c, hipMemcpyAsync(g.res_host + m, c->scal + SC_RES, sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
      });
      HIPCHK(c0, hipStreamSynchronize(st));
      g.used = 0;
      upd.clear();
      each([&](td_ctx* c, int m) {
        if (!active[m]) return;
        const NsAction a = ns_decide(c, ns[m], g.res_host[m]);
        if (a == NS_RESTART) {
          ns_cold_start(c);
        } else if (a == NS_DONE) {
          active[m] = 0;
        } else {
          HIPCHK(c, td::two_minus(c->stream, c->A, np, c->n));     // 2 - S X
          upd.push_back(m);
        }
      });
      if (!upd.empty()) {
        // X (2 - S X): the 64-wide tiles on and above the diagonal, then a mirror
        for (int m : upd) {
          td_ctx* c = mem[m];
          pr.push_back(problem(c->Sinv, np, c->A, np, c->H, np, np, np, np, 64, 1));
        }
        grouped_launch(c0, g, pr, 64);
        each([&](td_ctx* c, int m) {
          if (std::find(upd.begin(), upd.end(), m) == upd.end()) return;
          HIPCHK(c, td::symmetric_mirror(c->stream, c->H, np, np));
          ns_updated(c, ns[m]);
          if (ns[m].done) active[m] = 0;
        });
      }
      bool any = false;
      for (int m = 0; m < nm; ++m) any = any || active[m];
      if (!any) break;
    }
    each([&](td_ctx* c, int m) {
      ns_finish(c, ns[m]);
      c->step += 1;
    });
  }
  for (int m = 0; m < nm; ++m) {
    td_ctx* c = mem[m];
    try {
      c->last_n = nsteps;
      HIPCHK(c, hipMemcpyAsync(c->pos_h.data(), c->pos, sizeof(double) * 3 * c->na,
                               hipMemcpyDeviceToHost, st));
      refresh(c);
    } catch (const Fail&) {
      err = "member " + std::to_string(m) + ": " + c->err;
      throw;
    }
  }
}

void ensure_series_ctx(td_ctx* c, int nsteps) { ensure_series(c, nsteps); }

double field_spread(const td_ctx* c, const double* field, int nsteps) {
  double spread = 0.0;
  const double* p = c->pos_h.data();
  for (int k = 0; k < nsteps; ++k) {
    const double* E = field + 3 * (size_t)k;
    double lo = INFINITY, hi = -INFINITY;
    for (int a = 0; a < c->na; ++a) {
      const double v = p[3 * a] * E[0] + p[3 * a + 1] * E[1] + p[3 * a + 2] * E[2];
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
    spread = std::max(spread, hi - lo);
  }
  return spread;
}
}  // namespace tdi

extern "C" {

void td_default_options(td_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = TD_FP64;
  o->n_slices = 4;
  o->dt = 0.2;
  o->scc_tol = 1e-12;
  o->scc_maxiter = 300;
  o->mix_beta = 0.3;
  o->mix_history = 8;
  o->profile = 0;
  o->hip_stream = nullptr;
}

td_status td_create(const td_system* sys, const td_options* opt, td_ctx** out, char* err,
                    int32_t errlen) {
  if (!out) {
    set_err(err, errlen, "out must not be null");
    return TD_EINVAL;
  }
  *out = nullptr;
  td_ctx* c = new (std::nothrow) td_ctx();
  if (!c) {
    set_err(err, errlen, "host allocation failed");
    return TD_ENOMEM;
  }
  td_status st = guarded(c, [&] { create_impl(c, sys, opt); });
  if (st != TD_OK) {
    set_err(err, errlen, c->err);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return st;
  }
  set_err(err, errlen, "");
  *out = c;
  return TD_OK;
}

td_status td_kick(td_ctx* ctx, double e0, const double dir[3]) {
  return guarded(ctx, [&] { kick_impl(ctx, e0, dir); });
}

td_status td_step(td_ctx* ctx, int32_t n, const double* field) {
  return guarded(ctx, [&] { step_impl(ctx, n, field); });
}

td_status td_get_charges(td_ctx* ctx, double* dq) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, dq, TD_EINVAL, "null output");
    std::memcpy(dq, ctx->dq_h.data(), sizeof(double) * ctx->na);
  });
}

td_status td_get_dipole(td_ctx* ctx, double mu[3]) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, mu, TD_EINVAL, "null output");
    std::memcpy(mu, ctx->mu_h, sizeof(double) * 3);
  });
}

td_status td_get_dipole_series(td_ctx* ctx, double* mu, int32_t cap, int32_t* n_out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, n_out && cap >= 0 && (mu || cap == 0), TD_EINVAL, "invalid output");
    const int k = std::min(cap, ctx->last_n);
    if (k > 0)
      HIPCHK(ctx, hipMemcpyAsync(mu, ctx->dip, sizeof(double) * 3 * k, hipMemcpyDeviceToHost,
                                 ctx->stream));
    sync(ctx);
    *n_out = ctx->last_n;
  });
}

td_status td_get_energy(td_ctx* ctx, const double field[3], double* energy) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, energy, TD_EINVAL, "null output");
    td_ctx* c = ctx;
    if (field)
      HIPCHK(c, hipMemcpyAsync(c->scal + SC_FIELD, field, sizeof(double) * 3,
                               hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, td::rowdot(c->stream, c->rho_cur, 2 * c->np, c->H0, c->np, c->work1, c->np, c->np));
    if (c->split) HIPCHK(c, td::vec_add(c->stream, c->work1, c->band_ref, c->work1, c->np));
    HIPCHK(c, td::potential(c->stream, c->gamma, c->dq, c->pos, nullptr, c->orb_off, c->na, c->v,
                            c->vorb));
    HIPCHK(c, td::energy_terms(c->stream, c->work1, c->np, c->dq, c->v, c->pos,
                               field ? c->scal + SC_FIELD : nullptr, c->na, c->scal + SC_E));
    double e[3];
    read_scal(c, SC_E, e, 3);
    double e_rep = 0.0;
    if (c->ehr && c->rep_a) {   // moving nuclei: the pair repulsion at the current positions
      HIPCHK(c, td::repulsion(c->stream, c->pos, c->species, c->rep_a, c->nsp, c->rep_decay,
                              c->na, nullptr, c->e_rep_atom, c->scal + SC_EREP));
      read_scal(c, SC_EREP, &e_rep, 1);
    }
    double e_u = 0.0;
    if (c->plus_u != TD_PLUS_U_NONE) {
      // correction energy (Sec. 3.2, Eq. 21 or 24) of the current density
      if (c->split) {
        full_density(c, c->rho_cur, c->stage);
        block_pops(c, c->sh_n, c->stage, 2 * c->np);
      } else {
        block_pops(c, c->sh_n);
      }
      std::vector<double> es(c->nsh);
      HIPCHK(c, hipMemcpyAsync(es.data(), c->sh_e, sizeof(double) * c->nsh,
                               hipMemcpyDeviceToHost, c->stream));
      sync(c);
      for (double x : es) e_u += x;
    }
    *energy = e[0] + e[1] + e[2] + e_rep + e_u;
  });
}

td_status td_get_rho(td_ctx* ctx, double* rho, double* rho_prev, int64_t* step,
                     int32_t* has_prev) {
  return guarded(ctx, [&] {
    td_ctx* c = ctx;
    const size_t n2 = (size_t)c->n * c->n;
    const double* cur = c->rho_cur;
    if (c->split) {
      full_density(c, c->rho_cur, c->stage);
      cur = c->stage;
    }
    if (rho) {
      HIPCHK(c, td::wide_to_interleaved(c->stream, cur, c->np, c->X, c->n));
      HIPCHK(c, hipMemcpyAsync(rho, c->X, sizeof(double) * 2 * n2, hipMemcpyDeviceToHost,
                               c->stream));
    }
    if (rho_prev) {
      REQUIRE(c, c->has_prev, TD_ESTATE, "no previous density matrix (next step is Euler)");
      const double* prev = c->rho_prev;
      if (c->split) {
        sync(c);
        full_density(c, c->rho_prev, c->stage);
        prev = c->stage;
      }
      HIPCHK(c, td::wide_to_interleaved(c->stream, prev, c->np, c->X, c->n));
      HIPCHK(c, hipMemcpyAsync(rho_prev, c->X, sizeof(double) * 2 * n2, hipMemcpyDeviceToHost,
                               c->stream));
    }
    sync(c);
    if (step) *step = c->step;
    if (has_prev) *has_prev = c->has_prev ? 1 : 0;
  });
}

td_status td_set_rho(td_ctx* ctx, const double* rho, const double* rho_prev, int64_t step) {
  return guarded(ctx, [&] {
    td_ctx* c = ctx;
    REQUIRE(c, rho, TD_EINVAL, "rho must not be null");
    const size_t n2 = (size_t)c->n * c->n;
    REQUIRE(c, finite_all(rho, 2 * n2) && (!rho_prev || finite_all(rho_prev, 2 * n2)),
            TD_EINVAL, "non-finite density matrix");
    HIPCHK(c, hipMemcpyAsync(c->X, rho, sizeof(double) * 2 * n2, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, td::interleaved_to_wide(c->stream, c->X, c->n, c->rho_cur, c->np));
    if (c->split) HIPCHK(c, td::wide_add_real(c->stream, c->rho_cur, c->rho_ref, c->np, -1.0));
    if (rho_prev) {
      HIPCHK(c, hipMemcpyAsync(c->X, rho_prev, sizeof(double) * 2 * n2, hipMemcpyHostToDevice,
                               c->stream));
      HIPCHK(c, td::interleaved_to_wide(c->stream, c->X, c->n, c->rho_prev, c->np));
      if (c->split)
        HIPCHK(c, td::wide_add_real(c->stream, c->rho_prev, c->rho_ref, c->np, -1.0));
    }
    c->has_prev = rho_prev != nullptr;
    c->step = step;
    sync(c);
    refresh(c, true);
  });
}

td_status td_get_info(td_ctx* ctx, td_info* info) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, info, TD_EINVAL, "null output");
    ctx->info.step = ctx->step;
    ctx->info.has_prev = ctx->has_prev ? 1 : 0;
    *info = ctx->info;
  });
}

td_status td_get_kernel_time(td_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, kind >= 0 && kind < TD_KT_COUNT && total_ms && launches, TD_EINVAL,
            "invalid kernel class or output");
    *total_ms = ctx->kt_ms[kind];
    *launches = ctx->kt_n[kind];
  });
}

td_status td_reset_kernel_time(td_ctx* ctx) {
  return guarded(ctx, [&] {
    for (int q = 0; q < TD_KT_COUNT; ++q) {
      ctx->kt_ms[q] = 0.0;
      ctx->kt_n[q] = 0;
    }
  });
}

td_status td_get_forces(td_ctx* ctx, double* forces) {
  return guarded(ctx, [&] {
    td_ctx* c = ctx;
    REQUIRE(c, c->ehr, TD_ENOTSUP,
            "forces need a model of S(R) and H0(R): create the context with "
            "td_create_ehrenfest");
    REQUIRE(c, forces, TD_EINVAL, "null output");
    ehr_forces(c, nullptr, c->scal + SC_MU, nullptr);
    HIPCHK(c, hipMemcpyAsync(forces, c->F, sizeof(double) * 3 * c->na, hipMemcpyDeviceToHost,
                             c->stream));
    sync(c);
  });
}

td_status td_create_ehrenfest(const td_system* sys, const td_model* model,
                              const double* velocities, const td_options* opt, td_ctx** out,
                              char* err, int32_t errlen) {
  if (!out) {
    set_err(err, errlen, "out must not be null");
    return TD_EINVAL;
  }
  *out = nullptr;
  td_ctx* c = new (std::nothrow) td_ctx();
  if (!c) {
    set_err(err, errlen, "host allocation failed");
    return TD_ENOMEM;
  }
  td_status st = guarded(c, [&] { create_ehr_impl(c, sys, model, velocities, opt); });
  if (st != TD_OK) {
    set_err(err, errlen, c->err);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return st;
  }
  set_err(err, errlen, "");
  *out = c;
  return TD_OK;
}

td_status td_get_nuclei(td_ctx* ctx, double* positions, double* velocities) {
  return guarded(ctx, [&] {
    td_ctx* c = ctx;
    REQUIRE(c, c->ehr, TD_ENOTSUP, "clamped-nuclei context");
    if (positions)
      HIPCHK(c, hipMemcpyAsync(positions, c->pos, sizeof(double) * 3 * c->na,
                               hipMemcpyDeviceToHost, c->stream));
    if (velocities)
      HIPCHK(c, hipMemcpyAsync(velocities, c->vel, sizeof(double) * 3 * c->na,
                               hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

td_status td_get_energy_series(td_ctx* ctx, double* e_el, double* e_kin, int32_t cap,
                               int32_t* n_out) {
  return guarded(ctx, [&] {
    td_ctx* c = ctx;
    REQUIRE(c, c->ehr, TD_ENOTSUP, "clamped-nuclei context");
    REQUIRE(c, n_out && cap >= 0 && ((e_el && e_kin) || cap == 0), TD_EINVAL, "invalid output");
    const int k = std::min(cap, c->last_n);
    std::vector<double> parts(4 * (size_t)std::max(k, 1));
    if (k > 0) {
      HIPCHK(c, hipMemcpyAsync(parts.data(), c->e_el, sizeof(double) * 4 * k,
                               hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(e_kin, c->e_kin, sizeof(double) * k, hipMemcpyDeviceToHost,
                               c->stream));
    }
    sync(c);
    for (int i = 0; i < k; ++i)
      e_el[i] = parts[4 * i] + parts[4 * i + 1] + parts[4 * i + 2] + parts[4 * i + 3];
    *n_out = c->last_n;
  });
}

const char* td_last_error(const td_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

const char* td_status_string(int32_t s) {
  switch (s) {
    case TD_OK: return "TD_OK";
    case TD_EINVAL: return "TD_EINVAL";
    case TD_ENOMEM: return "TD_ENOMEM";
    case TD_EHIP: return "TD_EHIP";
    case TD_ENOTPOSDEF: return "TD_ENOTPOSDEF";
    case TD_ESCF: return "TD_ESCF";
    case TD_EUNSTABLE: return "TD_EUNSTABLE";
    case TD_ENOTSUP: return "TD_ENOTSUP";
    case TD_ESTATE: return "TD_ESTATE";
    default: return "unknown status";
  }
}

void td_destroy(td_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  delete ctx;
}

td_status td_util_gemm(int32_t precision, int32_t n_slices, int32_t m, int32_t n, int32_t k,
                       const double* A, const double* B, double* C, char* err, int32_t errlen) {
  td_ctx tmp;
  td_ctx* c = &tmp;
  td_status st = guarded(c, [&] {
    REQUIRE(c, A && B && C && m > 0 && n > 0 && k > 0, TD_EINVAL, "invalid gemm arguments");
    REQUIRE(c, precision == TD_FP64 || precision == TD_SPLIT_BF16, TD_EINVAL,
            "unknown precision");
    REQUIRE(c, precision == TD_FP64 || (n_slices >= 3 && n_slices <= 5), TD_EINVAL,
            "n_slices must be 3, 4 or 5");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    REQUIRE(c, e == hipSuccess && ndev > 0, TD_EHIP, "no HIP device available");
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
    if (precision == TD_SPLIT_BF16) {
      split_gemm_host(c, n_slices, m, n, k, A, B, C);
      return;
    }
    const int mp = round_up(m, td::kGemmTile), npd = round_up(n, td::kGemmTile),
              kp = round_up(k, td::kGemmTile);
    dalloc(c, &c->S, (size_t)mp * kp);
    dalloc(c, &c->H, (size_t)kp * npd);
    dalloc(c, &c->A, (size_t)mp * npd);
    HIPCHK(c, hipMemcpy2DAsync(c->S, sizeof(double) * kp, A, sizeof(double) * k,
                               sizeof(double) * k, m, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpy2DAsync(c->H, sizeof(double) * npd, B, sizeof(double) * n,
                               sizeof(double) * n, k, hipMemcpyHostToDevice, c->stream));
    gemm(c, 0, mp, npd, kp, 1.0, c->S, kp, c->H, npd, c->A, npd);
    HIPCHK(c, hipMemcpy2DAsync(C, sizeof(double) * n, c->A, sizeof(double) * npd,
                               sizeof(double) * n, m, hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
  set_err(err, errlen, st == TD_OK ? "" : c->err);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c);
  return st;
}

}  // extern "C"
