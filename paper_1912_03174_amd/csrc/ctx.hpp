// Private state of the TD-DFTB library shared by its host sources: the
// per-trajectory context behind the opaque td_ctx handle, and the error
// plumbing of the C entry points (no exception crosses the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "../../include/tddftb.h"
#include "common.hpp"

struct td_ctx {
  int na = 0, n = 0, np = 0, nelec = 0;
  td_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double *S = nullptr, *H0 = nullptr, *Sinv = nullptr, *H = nullptr, *A = nullptr;
  double *rho_cur = nullptr, *rho_prev = nullptr, *X = nullptr;
  double *gamma = nullptr, *pos = nullptr, *q0 = nullptr;
  int* orb_off = nullptr;
  double *q_orb = nullptr, *dq = nullptr, *dq_in = nullptr, *v = nullptr, *vorb = nullptr;
  double *xorb = nullptr, *work1 = nullptr, *work2 = nullptr, *scal = nullptr;
  double *hx = nullptr, *hf = nullptr;
  // on-site corrections (Sec. 3.2): shells, their U, block populations n,
  // potentials V and energies; the SCC mixing vector [dq | n blocks]
  int plus_u = 0, nsh = 0, max_shell = 0, mix_len = 0;
  int *sh_off = nullptr, *sh_of = nullptr;
  double *sh_u = nullptr, *sh_n = nullptr, *sh_v = nullptr, *sh_e = nullptr;
  double* sh_nref = nullptr;   // split products: block populations of rho_ref
  double *mix_in = nullptr, *mix_out = nullptr, *mix_hx = nullptr, *mix_hf = nullptr;
  double* field = nullptr;
  int field_cap = 0;
  double* dip = nullptr;
  int dip_cap = 0;
  std::vector<int> orb_off_h;
  std::vector<double> pos_h;
  std::vector<double> dq_h;
  double mu_h[3] = {0, 0, 0};
  int64_t step = 0;
  bool has_prev = false;
  double ne_ref = 0.0;         // Tr(rho S) when the state was last set (creation, kick, restore)
  int last_n = 0;
  td_info info{};
  std::string err;
  // split-bf16 precision: the state buffers hold rho - rho_ref
  bool split = false;
  int ns = 4;                  // slices of [S^-1 H | S^-1 dH] [rho - rho_ref ; rho_ref]
  int ns1 = 4;                 // slices of S^-1 dH
  double *rho_ref = nullptr;   // np x np real reference density (the initial state)
  double *Agsb = nullptr;      // S^-1 H_ref
  double *Xref = nullptr;      // np x 2np wide: (S^-1 H_ref) rho_ref | 0
  double *q_ref = nullptr;     // np: Mulliken row sums of rho_ref
  double *v_ref = nullptr;     // na: SCC potential of rho_ref
  double *band_ref = nullptr;  // np: row sums of rho_ref o H0
  double *stage = nullptr;     // np x 2np scratch
  __bf16 *sl_sinv = nullptr, *sl_dh = nullptr, *sl_L2 = nullptr, *sl_R2 = nullptr;
  int *e_sinv = nullptr, *e_dh = nullptr, *e_L2 = nullptr, *e_R2 = nullptr;
  // moving nuclei (Ehrenfest); positions live in pos (device) and pos_h
  bool ehr = false;
  bool ehr_setup = false;      // td_create_ehrenfest is building this context
  bool ehr_split = false;      // the products with rho as split-bf16 (no reference
                               // form: sl_L2 holds the left operand, sl_R2 the rows
                               // of Re rho and -Im rho)
  bool vel_half = false;       // vel holds v_{n-1/2} (else v_n, before the first step)
  int nsp = 0;
  double decay = 0.0, hub_u = 0.0;
  int *species = nullptr, *norb = nullptr, *atom_of = nullptr;
  double *sk_s = nullptr, *sk_h = nullptr, *scale_s = nullptr, *scale_h = nullptr;
  double *onsite = nullptr, *mass = nullptr;
  double *rep_a = nullptr;               // nsp x nsp pair repulsion amplitudes (or none)
  double rep_decay = 0.0;
  double *e_rep_atom = nullptr;          // na: per-atom halves of the pair repulsion
  double *GS = nullptr, *GH = nullptr;   // 3 np x np each
  double *W = nullptr, *Dm = nullptr;    // np x np
  double *Sinv_prev = nullptr;           // np x np: S^-1 of the previous positions
  double *Sinv_prev2 = nullptr;          // np x np: S^-1 two positions back
  int sinv_hist = 0;                     // inverses of earlier positions held (0..2)
  double *Z = nullptr;                   // np x 2np
  double *dgamma = nullptr;              // na x na x 3
  double *vel = nullptr, *F = nullptr;   // na x 3
  double *e_kin = nullptr, *e_el = nullptr;   // per-step series (dip_cap); e_el holds
                                              // 4 terms a step: band, Coulomb, field, E_rep
  // profiling
  std::vector<hipEvent_t> ev;
  double kt_ms[TD_KT_COUNT] = {0, 0, 0, 0};
  int64_t kt_n[TD_KT_COUNT] = {0, 0, 0, 0};
};

namespace tdi {

struct Fail {
  td_status st;
};

inline void set_err(char* buf, int len, const std::string& m) {
  if (buf && len > 0) {
    std::snprintf(buf, (size_t)len, "%s", m.c_str());
  }
}

#define HIPCHK(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                       \
      throw tdi::Fail{e_ == hipErrorOutOfMemory ? TD_ENOMEM : TD_EHIP};                     \
    }                                                                                       \
  } while (0)

#define REQUIRE(ctx, cond, status, msg) \
  do {                                  \
    if (!(cond)) {                      \
      (ctx)->err = (msg);               \
      throw tdi::Fail{status};          \
    }                                   \
  } while (0)

// Runs f, mapping failures to a status; C is any context with an `err` string.
template <class C, class F>
td_status guarded(C* ctx, F&& f) {
  if (!ctx) return TD_EINVAL;
  try {
    ctx->err.clear();
    f();
    return TD_OK;
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return TD_ENOMEM;
  } catch (...) {
    ctx->err = "unexpected internal error";
    return TD_EHIP;
  }
}

// Device tables of the grouped products of a batch of moving-nuclei
// trajectories: `slots` tables of `per` problems, filled from a pinned host
// mirror and reused after the stream has been synchronised; res_host holds
// one Newton-Schulz residual per member.
struct EhrGroup {
  td::GemmProblem* dev = nullptr;
  td::GemmProblem* host = nullptr;
  double* res_host = nullptr;
  int slots = 0, per = 0, used = 0;
  // the per-member passes between two grouped launches spread over
  // kLanes streams (default priority), joined by events
  static constexpr int kLanes = 4;
  hipStream_t lane[kLanes] = {};
  hipEvent_t fork = nullptr, join[kLanes] = {};
};
void ehr_group_alloc(td_ctx* c, EhrGroup& g, int nm);
void ehr_group_free(EhrGroup& g);
// n moving-nuclei steps of every member (contexts of one system on one
// stream): the step's products as grouped launches over all members, the
// other passes per member, the arithmetic of one trajectory (each member
// follows its solo trajectory bit for bit). field: device [n * 3] or null.
// On failure err names the member.
void ehr_batch_steps(std::vector<td_ctx*>& mem, EhrGroup& g, int nsteps, const double* field,
                     std::string& err);
// Device series for nsteps dipoles and energies.
void ensure_series_ctx(td_ctx* c, int nsteps);
// Largest spread over the atoms (current host positions) of the field's
// potential R_A . E_k over the steps of `field` [nsteps x 3].
double field_spread(const td_ctx* c, const double* field, int nsteps);

// Waits for the context's stream.
void sync_ctx(td_ctx* c);
// Mulliken charges and dipole of the current density copied to the host
// (what td_get_charges / td_get_dipole return); checks finiteness.
void refresh_ctx(td_ctx* c);

}  // namespace tdi
