/*
 * tddftb.h - C ABI of the MI355X real-time TD-DFTB propagation library.
 *
 * The library propagates the complex one-body density matrix rho of a
 * density-functional tight-binding model with clamped nuclei under the
 * Liouville-von Neumann equation in a non-orthogonal basis,
 *     drho/dt = -i (S^-1 H rho - rho H S^-1)
 * (Bonafe et al., arXiv 1912.03174, Sec. 2.1, Eq. 10 with the
 * non-adiabatic coupling D = 0), with the leapfrog integrator and an Euler
 * start (Sec. 2.3, Eq. 19). At every step the self-consistent-charge
 * Hamiltonian is rebuilt from the Mulliken charge fluctuations and the
 * external field (Sec. 2.1, Eqs. 5-7), and the Mulliken dipole is
 * recorded.
 *
 * Conventions shared by every entry point:
 *  - Atomic units (bohr, hartree, au of time, au of field).
 *  - Matrices are dense, row-major, float64; complex matrices are
 *    interleaved complex128 (re, im) pairs, row-major.
 *  - Orbitals of atom A are contiguous: orbitals orb_offset[A] ..
 *    orb_offset[A+1]-1.
 *  - All pointers passed to the library are host pointers unless stated
 *    otherwise. Input arrays are copied; the caller keeps ownership.
 *    Output arrays are caller-allocated and written only when the call
 *    returns TD_OK.
 *  - Every call returns a td_status. On failure, td_last_error(ctx) holds
 *    a message (for td_create failures, the message is in the err buffer
 *    of td_create). No C++ exception crosses the boundary.
 *  - A context owns one trajectory, its device buffers and one HIP
 *    stream. Calls on one context must not overlap; different contexts
 *    are independent.
 *
 * Readings of the paper fixed by this interface:
 *  - Mulliken dipole mu = -sum_A dq_A R_A with dq_A = q_A - q0_A the
 *    excess electron population (Sec. 2.1, Eq. 5).
 *  - The external potential entering the Hamiltonian is V_A = R_A . E(t)
 *    (dipole approximation, Sec. 2.1, relation after Eq. 15).
 *  - The delta kick multiplies orbital u by exp(-i E0 e . R_A(u))
 *    (Sec. 2.2, Eq. 16).
 */
#ifndef TDDFTB_H
#define TDDFTB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TD_API __attribute__((visibility("default")))

typedef struct td_ctx td_ctx;

typedef enum {
  TD_OK = 0,
  TD_EINVAL = -1,       /* bad argument: null pointer, size, shape, value  */
  TD_ENOMEM = -2,       /* device or host allocation failed                */
  TD_EHIP = -3,         /* HIP runtime error (message has the HIP text)    */
  TD_ENOTPOSDEF = -4,   /* S is not positive definite (inverse diverged)   */
  TD_ESCF = -5,         /* ground state: SCC or purification not converged */
  TD_EUNSTABLE = -6,    /* leapfrog unstable: dt too large for the spectrum
                           of S^-1 H, or the state became non-finite, or
                           its electron count Tr(rho S) drifted            */
  TD_ENOTSUP = -7,      /* feature not available in this library           */
  TD_ESTATE = -8        /* call not valid in the context's current state   */
} td_status;

typedef enum {
  TD_FP64 = 0,          /* all products in float64 on the FP64 matrix cores */
  TD_SPLIT_BF16 = 1     /* products as split-bf16 slices, fp32 accumulation */
} td_precision;

/* td_system.flags: the array fields are device pointers (for example the
 * data of framework tensors) readable on td_options.hip_stream (or the
 * null stream when that is NULL); td_create reads them once, in stream
 * order, and keeps no reference. Without the flag they are host pointers.
 * S, H0, gamma and rho0 are copied device to device into the context's
 * padded buffers and checked there (finite; S and H0 symmetric), with the
 * same errors as host arrays; only the per-atom and per-shell arrays and
 * occ pass through host memory. Batches and moving-nuclei contexts take
 * host pointers only. */
#define TD_DEVICE_PTRS 1u

/* td_system.plus_u: the on-site corrections of Sec. 3.2 added to the SCC
 * Hamiltonian in the ground state and at every step: the fully-localised
 * limit of DFTB+U (Eqs. 21-23) or pseudo-SIC (Eqs. 24-25). Per shell b
 * (a contiguous range of orbitals of one atom) with U_b = shell_u[b], the
 * dual block population n_b = 1/2 (Re(rho) S + S Re(rho)) restricted to the
 * shell (Eq. 23; the density is spin-summed, n_b / 2 per spin), the energy
 *   FLL:  dE = sum_b -(U_b / 4) sum_uv n_uv^2 + (U_b / 2) sum_u n_uu
 *   pSIC: dE = sum_b -(U_b / 4) sum_uv n_uv^2
 * and its derivative V_b = -(U_b / 2) (n_b - 1) (FLL) or -(U_b / 2) n_b
 * (pSIC) enters H as 1/2 (S V + V S), V block diagonal. Batches and
 * moving nuclei return TD_ENOTSUP. */
#define TD_PLUS_U_NONE 0
#define TD_PLUS_U_FLL 1
#define TD_PLUS_U_PSIC 2
#define TD_PLUS_U_MAX_SHELL 7   /* orbitals per shell (up to an f shell) */

/* The model: positions, overlap S, non-SCC Hamiltonian H0 (Sec. 2.1,
 * Eq. 6), charge kernel gamma (Sec. 2.1, Eq. 3), reference populations
 * q0, and the occupations of the ground state (Sec. 2.1): either occ,
 * the occupation of each generalized eigenstate in ascending energy, or,
 * when occ is NULL, the electron count n_elec (closed shell: n_elec / 2
 * doubly occupied states). The ground state is found by zero-temperature
 * purification, so occ must be closed-shell aufbau: 2 for the lowest
 * states, then 0 (anything else returns TD_ENOTSUP); n_elec is then 0 or
 * sum(occ). rho0 is optional: NULL asks td_create for the self-consistent
 * ground state; otherwise it is the initial density matrix,
 * [n_orb * n_orb] interleaved complex128, Hermitian. */
typedef struct {
  int32_t n_atoms;
  int32_t n_orb;
  const int32_t *orb_offset;   /* [n_atoms + 1], orb_offset[0] = 0, increasing */
  const double *positions;     /* [n_atoms * 3] bohr                            */
  const double *S;             /* [n_orb * n_orb] symmetric positive definite   */
  const double *H0;            /* [n_orb * n_orb] symmetric, hartree            */
  const double *gamma;         /* [n_atoms * n_atoms] symmetric, hartree        */
  const double *q0;            /* [n_atoms] electrons                           */
  int32_t n_elec;              /* even, 0 < n_elec <= 2 n_orb (see occ)         */
  const double *rho0;          /* optional, see above                           */
  const double *occ;           /* optional [n_orb], see above                   */
  uint32_t flags;              /* 0 or TD_DEVICE_PTRS                           */
  int32_t plus_u;              /* TD_PLUS_U_NONE / _FLL / _PSIC (see above)     */
  int32_t n_shells;            /* shells when plus_u != TD_PLUS_U_NONE          */
  const int32_t *shell_offset; /* [n_shells + 1]: shell b is orbitals           */
                               /* [shell_offset[b], shell_offset[b + 1]), 1 to  */
                               /* TD_PLUS_U_MAX_SHELL orbitals of one atom;     */
                               /* shell_offset[0] = 0, last = n_orb             */
  const double *shell_u;       /* [n_shells] U_eff, hartree, finite and >= 0    */
} td_system;

typedef struct {
  int32_t precision;           /* td_precision                                  */
  int32_t n_slices;            /* split-bf16 slices per operand (3..5)          */
  double dt;                   /* time step, au (> 0)                           */
  double scc_tol;              /* ground state: max |dq_out - dq_in| to stop    */
  int32_t scc_maxiter;         /* ground state: SCC cycle limit                 */
  double mix_beta;             /* ground state: Anderson mixing parameter       */
  int32_t mix_history;         /* ground state: Anderson history (1..8)         */
  int32_t profile;             /* 1: time kernel classes with HIP events        */
  void *hip_stream;            /* hipStream_t to use, or NULL for an own stream */
  int32_t n_slices_dh;         /* split-bf16: slices of the S^-1 dH product     */
                               /* (3 .. n_slices), 0: n_slices. For accuracy    */
                               /* studies: that product multiplies rho_ref,     */
                               /* so fewer slices there cost accuracy much as   */
                               /* in the other product                           */
} td_options;

/* Statistics of the initialisation. */
typedef struct {
  int32_t n_atoms, n_orb, n_pad;      /* n_pad: padded matrix dimension      */
  int32_t inverse_iterations;         /* Newton-Schulz steps for S^-1        */
  double inverse_residual;            /* max |1 - S S^-1| at exit            */
  int32_t scc_iterations;             /* 0 when rho0 was given               */
  double scc_residual;                /* max |dq_out - dq_in| at exit        */
  int32_t purification_iterations;    /* in the last SCC cycle               */
  double purification_error;          /* Tr(X) - Tr(X^2) at exit             */
  double spectrum_lo, spectrum_hi;    /* bounds of the S^-1 H spectrum       */
  int64_t step;                       /* index of the current rho            */
  int32_t has_prev;                   /* 0: next step is an Euler start      */
  int32_t precision;
  int64_t inverse_updates;            /* Newton-Schulz updates of S^-1 since creation
                                         (moving nuclei: along the trajectory) */
  double width_estimate;              /* lower bound of the width of the spectrum of
                                         S^-1 H of the initial state at zero field
                                         (Rayleigh quotients after power iteration) */
  double stability;                   /* dt * width_estimate; td_step refuses to run
                                         (TD_EUNSTABLE) unless it is below 1, the
                                         leapfrog limit (Sec. 2.3, Eq. 19)           */
  int64_t inverse_restarts;           /* moving nuclei: Newton-Schulz iterations begun
                                         again from the scaled identity after a poor
                                         start along the trajectory                  */
} td_info;

/* Kernel classes timed when td_options.profile = 1. In split-bf16
 * precision the two classes of products are S^-1 dH and
 * [S^-1 H | S^-1 dH] [rho - rho_ref ; rho_ref], and the slicing kernels
 * count as TD_KT_OTHER. */
enum {
  TD_KT_GEMM_SH = 0,      /* S^-1 H product                 (2 n^3 flop) */
  TD_KT_GEMM_ARHO = 1,    /* (S^-1 H) [Re rho | Im rho]     (4 n^3 flop) */
  TD_KT_UPDATE = 2,       /* leapfrog update                             */
  TD_KT_OTHER = 3,        /* charges, potential, H assembly, dipole      */
  TD_KT_COUNT = 4
};

/* Fills *opt with defaults: FP64, 4 slices, dt = 0.2, scc_tol = 1e-12,
 * scc_maxiter = 300, mix_beta = 0.3, mix_history = 8, profile = 0, own
 * stream, n_slices_dh = 0. */
TD_API void td_default_options(td_options *opt);

/* Creates a context (Sec. 2.3): copies the model to the GPU, forms S^-1,
 * and either takes rho0 or solves the SCC ground state (Sec. 2.1) by
 * density-matrix purification (with plus_u, charges and block populations
 * are made self-consistent together). The ground state is the initial
 * density with no leapfrog history. Invalid shells return TD_EINVAL. On
 * failure *out is NULL and err (if not NULL) receives a message of at
 * most errlen bytes. */
TD_API td_status td_create(const td_system *sys, const td_options *opt, td_ctx **out,
                           char *err, int32_t errlen);

/* Applies a delta pulse E(t) = e0 delta(t) dir to the current rho
 * (Sec. 2.2, Eq. 16). dir need not be normalised (non-zero). Clears the
 * leapfrog history: the next step is an Euler start. */
TD_API td_status td_kick(td_ctx *ctx, double e0, const double dir[3]);

/* Advances n >= 0 steps of dt (Sec. 2.3, Eq. 19). field is NULL (no
 * field) or [n * 3]: field[3k..3k+2] = E(t) at the time of the k-th
 * density matrix of this call. The dipole of each density entering a
 * step is recorded (see td_get_dipole_series). Returns TD_EUNSTABLE
 * before any step when dt times the width of the spectrum of S^-1 H (a
 * lower bound taken at creation, td_info.width_estimate), plus with a
 * field the largest spread of the field's potential R_A . E over the atoms
 * (current positions) among this call's steps, is 1 or more, where the
 * leapfrog diverges (Sec. 2.3, Eq. 19); and after the steps if
 * the state became non-finite or its electron count Tr(rho S), which the
 * leapfrog keeps, moved by more than 1e-6 N_e since creation, the last
 * kick or restore (1e-3 N_e with moving nuclei; in split-bf16 precision,
 * which restores the count every step, within the last step). */
TD_API td_status td_step(td_ctx *ctx, int32_t n, const double *field);

/* Mulliken charge fluctuations dq [n_atoms] of the current rho (Eq. 5). */
TD_API td_status td_get_charges(td_ctx *ctx, double *dq);

/* Mulliken dipole mu[3] of the current rho. */
TD_API td_status td_get_dipole(td_ctx *ctx, double mu[3]);

/* Dipoles recorded by the last td_step: mu[3k..3k+2] for the k-th step,
 * k < min(cap, n); *n_out = number recorded by that call. */
TD_API td_status td_get_dipole_series(td_ctx *ctx, double *mu, int32_t cap, int32_t *n_out);

/* Energy of the current rho: Re Tr(rho H0) + 1/2 dq gamma dq
 * + sum_A dq_A R_A . field (field may be NULL for zero) (Sec. 2.1,
 * Eqs. 2-3); with moving nuclei, plus the model's repulsive energy E_rep
 * at the current positions. */
TD_API td_status td_get_energy(td_ctx *ctx, const double field[3], double *energy);

/* Checkpoint: current and previous density matrices as [n_orb * n_orb]
 * interleaved complex128 (rho_prev may be NULL), the step index and
 * whether a previous density exists. */
TD_API td_status td_get_rho(td_ctx *ctx, double *rho, double *rho_prev, int64_t *step,
                            int32_t *has_prev);

/* Restore: rho (required) and rho_prev (NULL: next step is an Euler start),
 * both [n_orb * n_orb] interleaved complex128; step is the index of rho. */
TD_API td_status td_set_rho(td_ctx *ctx, const double *rho, const double *rho_prev,
                            int64_t step);

TD_API td_status td_get_info(td_ctx *ctx, td_info *info);

/* Accumulated HIP-event time (ms) and launch count of a kernel class
 * since creation or the last reset (needs td_options.profile = 1). */
TD_API td_status td_get_kernel_time(td_ctx *ctx, int32_t kind, double *total_ms,
                                    int64_t *launches);
TD_API td_status td_reset_kernel_time(td_ctx *ctx);

/* Ehrenfest forces (Sec. 2.1, Eq. 15) on the nuclei [n_atoms * 3] for the
 * current density and positions at zero field (a moving-nuclei context,
 * see td_create_ehrenfest); TD_ENOTSUP for clamped-nuclei contexts, which
 * carry no model of S(R) and H0(R). */
TD_API td_status td_get_forces(td_ctx *ctx, double *forces);

TD_API const char *td_last_error(const td_ctx *ctx);
TD_API const char *td_status_string(int32_t status);
TD_API void td_destroy(td_ctx *ctx);

/* Dense product C = A B (row-major, A [m x k], B [k x n], C [m x n]) on
 * the GPU with the library's propagation kernels in the given precision:
 * the matrix-product building block of the step (Sec. 2.3). Host
 * pointers; err receives a message on failure. */
TD_API td_status td_util_gemm(int32_t precision, int32_t n_slices, int32_t m, int32_t n,
                              int32_t k, const double *A, const double *B, double *C,
                              char *err, int32_t errlen);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the product of
 * td_util_gemm, C = A B in the given precision, on device pointers and
 * the caller's stream, allocating nothing on the device or the host.
 * A [m x k] (leading dimension lda >= k), B [k x n] (ldb >= n) and
 * C [m x n] (ldc >= n) are row-major float64 device arrays; hip_stream is
 * a hipStream_t (NULL: the null stream). The call only enqueues work: C is
 * complete once the stream reaches this point, and A and B must stay
 * unchanged until then. The result is bit for bit td_util_gemm's.
 * Scratch (padded copies of A, B and C, and in split-bf16 the slices and
 * their exponents) comes from one fixed device array of
 * TD_GEMM_NOALLOC_SCRATCH_BYTES per GPU, kept until the process ends. A
 * product needs 8 (m k + k n + m n) bytes of it in FP64 and
 * (8 + 2 s)(m k + n k) + 8 m n in split-bf16 with s slices (sizes padded
 * to the 128-wide tiles), so up to
 * m = n = k = 1664 in FP64 and 1280 at s = 4; a larger one returns
 * TD_EINVAL before any device work.
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * GPU (other streams, other threads) race, so order them on one stream or
 * with events. The first call on each device resolves the array's address
 * (hipGetSymbolAddress), so under stream capture make one call on that
 * device beforehand. Errors: TD_EINVAL (arguments, size), TD_EHIP (HIP
 * errors); err (if not NULL) receives a message of at most errlen bytes. */
#define TD_GEMM_NOALLOC_SCRATCH_BYTES (64u << 20)
TD_API td_status td_util_gemm_noalloc(int32_t precision, int32_t n_slices, int32_t m, int32_t n,
                                      int32_t k, const double *A, int32_t lda, const double *B,
                                      int32_t ldb, double *C, int32_t ldc, void *hip_stream,
                                      char *err, int32_t errlen);

/* ---------------------------------------------------------------- moving nuclei
 * Ehrenfest dynamics (Sec. 2.1, Eqs. 9-15; Sec. 2.3): S, H0 and gamma are
 * rebuilt every step from a two-centre model at the current positions, the
 * density follows Eq. 10 with the non-adiabatic coupling
 * D_uv = v_B . grad_B S_uv (u on A != B, v on B; Eq. 14; gradients by
 * central differences with step eps^(1/4), Eq. 20), and the nuclei follow
 * velocity Verlet with the Ehrenfest force of Eq. 15 without its velocity
 * terms (as the paper's implementation), the overlap terms taken as
 * +1/2 Re Tr{rho ((grad S) S^-1 H + H S^-1 (grad S))} (the sign that
 * conserves electronic plus nuclear kinetic energy and reduces to the
 * ground-state energy gradient), the SCC term with the Hamiltonian's full
 * atomic potential (gamma dq + R . E), and the repulsive term -grad_A E_rep
 * of the model's pair repulsion (td_model.rep_a). */

/* Two-centre model: every off-site integral between orbital i of atom a
 * and orbital j of atom b at d = R_b - R_a is
 *   prefactor x exp(-|d| / decay) x Slater-Koster angular factor x scale[a, b]
 * with the prefactors of the ordered species pair (sa, sb):
 * (ss sigma, sp sigma for s on a and p on b, pp sigma, pp pi); the p-on-a,
 * s-on-b element uses the (sb, sa) sp prefactor with d reversed. On-site:
 * S = 1, H0 = onsite[s][0] (s) or onsite[s][1] (p), no on-site coupling.
 * gamma_AB = 1 / sqrt(r^2 + hubbard_u^-2). Orbitals per atom: s, or s,
 * p_x, p_y, p_z, in that order, consistent with td_system.orb_offset.
 * Repulsive energy (Sec. 2.1: the pairwise E_rep of the total energy):
 *   E_rep = sum_{A<B} rep_a[s_A, s_B] exp(-r_AB / rep_decay),
 * every pair, no cutoff; rep_a NULL means none. It adds -grad_A E_rep to
 * the forces and E_rep to the energies (td_get_energy, the energy
 * series). */
typedef struct {
  int32_t n_species;
  const int32_t *species;        /* [n_atoms], values in [0, n_species)              */
  const int32_t *species_norb;   /* [n_species]: 1 or 4                              */
  const double *sk_s;            /* [n_species * n_species * 4] overlap prefactors   */
  const double *sk_h;            /* [n_species * n_species * 4] H0 prefactors        */
  double decay;                  /* bohr, > 0                                        */
  const double *scale_s;         /* [n_atoms * n_atoms] symmetric pair factors       */
  const double *scale_h;         /* [n_atoms * n_atoms]                              */
  const double *onsite;          /* [n_species * 2] hartree                          */
  double hubbard_u;              /* hartree, > 0                                     */
  const double *mass;            /* [n_species] electron masses, > 0                 */
  const double *rep_a;           /* [n_species * n_species] hartree, symmetric,      */
                                 /* finite, >= 0; NULL: no repulsion                 */
  double rep_decay;              /* bohr, > 0 when rep_a is given                    */
} td_model;

/* Creates a context with moving nuclei. sys gives positions, orb_offset,
 * q0, the occupations and optionally rho0 as for td_create; its S, H0 and
 * gamma are ignored (built from the model, on the GPU). velocities
 * [n_atoms * 3] bohr per au of time (NULL: at rest). No plus_u
 * (TD_ENOTSUP). In TD_SPLIT_BF16 precision the two products with the
 * density, (S^-1 H) rho and (S^-1 D) rho, run as split-bf16 products of
 * rho itself (S, H0 and S^-1 change every step, so there is no fixed
 * reference); S^-1 H, S^-1 D, the S^-1 update, charges, forces and
 * energies stay FP64. td_step then advances electrons and nuclei with
 * the same dt; td_kick, td_get_rho / td_set_rho act on the electrons and
 * keep the nuclei. */
TD_API td_status td_create_ehrenfest(const td_system *sys, const td_model *model,
                                     const double *velocities, const td_options *opt,
                                     td_ctx **out, char *err, int32_t errlen);

/* Nuclear state of a moving-nuclei context: positions [n_atoms * 3] of
 * the current density; velocities [n_atoms * 3] as velocity Verlet keeps
 * them: the initial velocities before the first step, afterwards half a
 * step behind the positions (v_{n-1/2}). Any pointer may be NULL. */
TD_API td_status td_get_nuclei(td_ctx *ctx, double *positions, double *velocities);

/* Per step of the last td_step on a moving-nuclei context: energy e_el[k]
 * (as td_get_energy, at the step's field: electronic terms plus E_rep) of
 * the density and positions entering step k and the nuclear kinetic energy
 * e_kin[k] of the velocities at that step; k < min(cap, n); *n_out =
 * number recorded. */
TD_API td_status td_get_energy_series(td_ctx *ctx, double *e_el, double *e_kin, int32_t cap,
                                      int32_t *n_out);

/* ---------------------------------------------------------------- batches
 * Many independent trajectories of different sizes stepped together, as in
 * the pump-probe protocol (Sec. 5.1: one probe trajectory per pump delay,
 * phase and kick direction, each a clamped-nuclei propagation of its own
 * density matrix). Every member follows exactly the trajectory a solo
 * context created from the same td_system would follow (bitwise, FP64);
 * each kernel of a step covers all members in one launch, and the steps
 * after the first are replayed from a captured HIP graph. */
typedef struct td_batch td_batch;

#define TD_BATCH_NO_GRAPH 1u   /* launch each step's kernels directly            */
#define TD_BATCH_TILE_128 2u   /* no tuning: 128 x 128 product tiles everywhere  */
#define TD_BATCH_TILE_64 4u    /* no tuning: 64 x 64 product tiles everywhere    */

#define TD_BATCH_BUCKETS 8     /* size buckets: padded n / 128 - 1, capped at 7  */

typedef struct {
  int32_t n_members;
  int64_t step;                          /* index of the current densities       */
  int32_t has_prev;
  int32_t graph;                         /* 1: steps replay a captured graph     */
  int32_t bucket_members[TD_BATCH_BUCKETS];
  int32_t bucket_tile[TD_BATCH_BUCKETS]; /* product tile edge used per bucket    */
  double bucket_ms[TD_BATCH_BUCKETS][2]; /* tuning: ms per launch, 128 and 64    */
} td_batch_info;

/* Creates a batch of n >= 1 trajectories, systems[m] as for td_create
 * (host or device pointers per its flags; rho0 NULL: SCC ground state).
 * opt applies to every member and must ask for TD_FP64 (split-bf16
 * batches, and members with plus_u, return TD_ENOTSUP). flags: TD_BATCH_* bits. Without a TILE flag
 * the library times both product tiles on each size bucket's members and
 * keeps the faster one. The batch owns one stream (opt.hip_stream, or its
 * own); a failure names the member in err. */
TD_API td_status td_batch_create(int32_t n, const td_system *systems, const td_options *opt,
                                 uint32_t flags, td_batch **out, char *err, int32_t errlen);

/* Kicks member m with e0[m] along dir[3m..3m+2] (Sec. 2.2, Eq. 16;
 * e0[m] = 0 leaves it unkicked but still restarts its integrator, as all
 * members share one step counter). Next step is an Euler start. */
TD_API td_status td_batch_kick(td_batch *b, const double *e0, const double *dir);

/* Advances every member n >= 0 steps (Sec. 2.3, Eq. 19); field is NULL or
 * [n * 3], the same field for all members. Records each member's dipole of
 * each density entering a step. TD_EUNSTABLE (as for td_step: the leapfrog
 * limit before any step, then a non-finite state or a drifted electron
 * count) names the first member concerned. */
TD_API td_status td_batch_step(td_batch *b, int32_t n, const double *field);

/* Per-member results, as the td_get_* calls of a solo context. */
TD_API td_status td_batch_get_dipole_series(td_batch *b, int32_t member, double *mu, int32_t cap,
                                            int32_t *n_out);
TD_API td_status td_batch_get_charges(td_batch *b, int32_t member, double *dq);
TD_API td_status td_batch_get_rho(td_batch *b, int32_t member, double *rho, double *rho_prev,
                                  int64_t *step, int32_t *has_prev);
TD_API td_status td_batch_get_info(td_batch *b, td_batch_info *info);

/* A batch of moving-nuclei trajectories of one system (Sec. 2.1, Eqs.
 * 9-15; Sec. 2.3), as in an ensemble of pump trajectories that differ in
 * their nuclear velocities: member m is the context td_create_ehrenfest
 * would make from sys, model and velocities[m * n_atoms * 3 ..] (NULL: all
 * at rest). The initial density is sys->rho0, or the SCC ground state
 * solved once for all members. td_batch_step advances every member; each
 * step's FP64 products (S^-1 H, (S^-1 H) rho, S^-1 D, (S^-1 D) rho, and the
 * Newton-Schulz products of the S^-1 update) run as one grouped launch over
 * all members (in TD_SPLIT_BF16 precision the two products with rho run per
 * member as split-bf16 products, as in a solo context), the other passes per member,
 * spread over four streams of the batch between the grouped launches, and
 * the residual checks of the S^-1 updates of all members share one host
 * synchronisation per round. Every member
 * follows exactly the trajectory of its solo context (bitwise).
 * td_batch_kick, td_batch_get_dipole_series, td_batch_get_charges,
 * td_batch_get_rho and td_batch_destroy work on it as on a probe batch;
 * td_batch_get_info reports the member count and step. */
TD_API td_status td_batch_create_ehrenfest(int32_t n, const td_system *sys,
                                           const td_model *model, const double *velocities,
                                           const td_options *opt, td_batch **out, char *err,
                                           int32_t errlen);

/* Nuclear state of member m of a moving-nuclei batch, as td_get_nuclei;
 * TD_ENOTSUP for a clamped-nuclei batch. */
TD_API td_status td_batch_get_nuclei(td_batch *b, int32_t member, double *positions,
                                     double *velocities);

/* Energy series of member m of a moving-nuclei batch for the last
 * td_batch_step, as td_get_energy_series; TD_ENOTSUP for a clamped-nuclei
 * batch. */
TD_API td_status td_batch_get_energy_series(td_batch *b, int32_t member, double *e_el,
                                            double *e_kin, int32_t cap, int32_t *n_out);

TD_API const char *td_batch_last_error(const td_batch *b);
TD_API void td_batch_destroy(td_batch *b);

/* ---------------------------------------------------------------- spectra
 * Spectra from recorded dipole series, computed on the GPU (host pointers
 * in and out; err receives a message on failure). */

/* Polarizability of kicked runs (Sec. 2.2, Eqs. 17-18), one per series j:
 *   alpha[j, w] = dt / e0[j] sum_{n < n_t} (mu[j, n] - r[j, n])
 *                 exp(i omega[w] t_n) exp(-t_n / tau),   t_n = n dt,
 * with r = ref (a reference run over the same times, e.g. the pump-only
 * dipole of Sec. 5.1) or, when ref is NULL, r[j, n] = mu[j, 0] (the static
 * dipole). tau <= 0: no damping. mu, ref: [n_series * n_t], the dipole
 * component along the kick of each series; e0 [n_series] non-zero; omega
 * [n_omega]. Outputs [n_series * n_omega]: alpha_re, alpha_im, and
 * sigma = 4 pi omega / c Im alpha (the series' share of the cross-section;
 * the isotropic cross-section is the mean over three kick directions). */
TD_API td_status td_spectrum(int32_t n_series, int32_t n_t, const double *mu, const double *ref,
                             const double *e0, double dt, double tau, int32_t n_omega,
                             const double *omega, double *alpha_re, double *alpha_im,
                             double *sigma, char *err, int32_t errlen);

/* Transient absorption from pump-probe runs (Sec. 5.1): series
 * j = d * n_avg + a are the probes of delay d (a runs over kick directions
 * and pump phases), ref[j] the pump-only dipole over the same times (both
 * along the probe's kick). out[d, w] = 4 pi omega_w / c Im(mean_a
 * alpha[j, w]) with alpha as in td_spectrum; then, if filter_width > 0, a
 * Gaussian low-pass along the delays exp(-nu^2 / (2 filter_width^2)) (nu in
 * cycles per unit time, periodic discrete transform over the n_delay delays
 * spaced delay_step); then, if ref_delay >= 0, the change against that
 * delay's spectrum, the end of the pump (Sec. 5.2). out [n_delay * n_omega]. */
TD_API td_status td_transient_absorption(int32_t n_delay, int32_t n_avg, int32_t n_t,
                                         const double *mu, const double *ref, const double *e0,
                                         double dt, double tau, int32_t n_omega,
                                         const double *omega, int32_t ref_delay,
                                         double delay_step, double filter_width, double *out,
                                         char *err, int32_t errlen);

#ifdef __cplusplus
}
#endif

#endif /* TDDFTB_H */
