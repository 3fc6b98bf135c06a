"""Plain CPU oracle: real-time TD-DFTB density-matrix propagation in FP64.

TEST INFRASTRUCTURE. This module is the slow, literal statement of what
the GPU library computes. It is imported only by the tests, the smoke
check and the CPU-baseline leg of the benchmark; the GPU library never
calls it and the two share no code. Every function cites the passage of
Bonafe et al., "A real-time time-dependent density functional
tight-binding implementation for semiclassical excited state
electron-nuclear dynamics and pump-probe spectroscopy simulations"
(arXiv 1912.03174) that it follows. Arithmetic is float64 / complex128
and uses numpy matrix products, inverses and scipy's generalized
symmetric eigensolver as the only library primitives.

Readings of the paper where it is silent or ambiguous:

* External potential in the Hamiltonian (Sec. 2.1, Eq. 7 and the
  dipole-approximation relation after Eq. 15): the paper writes the
  energy -mu_A . E = dq_A R_A . E; the Hamiltonian needs its derivative
  with respect to dq_A, so V_A = R_A . E(t).
* Dipole: mu = -sum_A dq_A R_A, with dq_A = q_A - q0_A the excess electron
  population (electrons carry charge -1).
* Kick (Sec. 2.2, Eq. 16): exp(iV) is read as the diagonal phase
  exp(-i E0 e . R_A(mu)) on each orbital, the impulse an electron takes
  from E(t) = E0 delta(t) e. With the Fourier sign exp(+i w t) this gives
  positive absorption.
* Mulliken populations (Sec. 2.1, Eq. 5) of a complex rho: the real part
  of Tr_A(rho S) (the imaginary part of the full trace vanishes).
* Leapfrog start (Sec. 2.3, Eq. 19): rho_1 = rho_0 + dt * rhodot(rho_0, t_0);
  the field is sampled at t_n = n dt; a kick resets the start.
* Energy: E = Re Tr(rho H0) + 1/2 dq^T gamma dq + sum_A dq_A R_A . E(t)
  (Sec. 2.1 band and Coulomb terms plus the external term); the repulsive
  energy is constant for frozen nuclei and left out.
* Ground state (Sec. 2.1, self-consistent charges): zero-temperature
  aufbau filling of N_e / 2 generalized eigenstates with two electrons
  each, iterated to self-consistency of the Mulliken charges.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.linalg

C_AU = 137.035999084   # speed of light in atomic units

__all__ = [
    "atom_of_orbital", "mulliken_populations", "charge_fluctuations",
    "external_potential", "scc_hamiltonian", "scc_hamiltonian_fast", "inverse_overlap", "rho_dot", "rho_dot_rows",
    "rho_dot_reference_split", "renormalise_delta",
    "euler_step", "leapfrog_step", "kick", "dipole", "energy", "electron_count",
    "GroundState", "ground_state", "Trajectory", "propagate",
    "polarizability", "cross_section", "stationarity_residual",
    "effective_polarizability", "transient_cross_section", "delta_absorbance",
    "gaussian_filter_delay",
]


def atom_of_orbital(orb_offset):
    """Atom index of every orbital; orbitals of atom A are contiguous."""
    off = np.asarray(orb_offset)
    counts = np.diff(off)
    return np.repeat(np.arange(len(counts)), counts)


def mulliken_populations(rho, S, orb_offset):
    """q_A = Tr_A(rho S) (Sec. 2.1, Eq. 5), real part.

    Tr_A sums the diagonal elements (rho S)_vv over the orbitals v of atom A.
    Only the diagonal of the product is formed.
    """
    diag = np.einsum("vu,uv->v", rho, S)
    off = np.asarray(orb_offset)
    return np.array([np.real(diag[off[a]:off[a + 1]].sum()) for a in range(len(off) - 1)])


def charge_fluctuations(rho, S, orb_offset, q0):
    """dq_A = q_A - q0_A (Sec. 2.1, Eqs. 3 and 5)."""
    return mulliken_populations(rho, S, orb_offset) - np.asarray(q0)


def electron_count(rho, S):
    """N_e = Re Tr(rho S), conserved by the leapfrog step (Sec. 2.3)."""
    return float(np.real(np.trace(rho @ S)))


def external_potential(positions, field):
    """V_A = R_A . E(t) (dipole approximation after Eq. 15; reading above)."""
    if field is None:
        return np.zeros(len(positions))
    return np.asarray(positions) @ np.asarray(field, dtype=np.float64)


def scc_hamiltonian(H0, S, gamma, dq, orb_offset, V=None):
    """SCC Hamiltonian with an external potential (Sec. 2.1, Eqs. 6 and 7).

    H_uv = H0_uv + 1/2 S_uv sum_C (gamma_AC + gamma_BC) dq_C
                 + 1/2 S_uv (V_A + V_B),          u on atom A, v on atom B.
    """
    atom = atom_of_orbital(orb_offset)
    shift = np.asarray(gamma) @ np.asarray(dq)      # sum_C gamma_AC dq_C
    H = np.array(H0, dtype=np.float64, copy=True)
    n = H.shape[0]
    for u in range(n):
        A = atom[u]
        for v in range(n):
            B = atom[v]
            total = shift[A] + shift[B]
            if V is not None:
                total = total + V[A] + V[B]
            H[u, v] += 0.5 * S[u, v] * total
    return H


def inverse_overlap(S):
    """S^-1, the inverse overlap in the equations of motion (Sec. 2.1, Eq. 10)."""
    return np.linalg.inv(S)


def rho_dot(rho, H, Sinv):
    """Time derivative of rho for clamped nuclei (Sec. 2.1, Eq. 10 with D = 0).

    rhodot = -i (S^-1 H rho - rho H S^-1), formed with the three matrix
    products the paper names (Sec. 2.3).
    """
    SinvH = Sinv @ H
    HSinv = H @ Sinv
    return -1j * (SinvH @ rho - rho @ HSinv)


def rho_dot_rows(rho, H, Sinv, rows):
    """Selected rows of Eq. 10 (D = 0): rhodot[i, :] for i in ``rows``.

    (S^-1 H)[i, :] = S^-1[i, :] H and (rho H S^-1)[i, :] = (rho[i, :] H) S^-1,
    each O(n^2) per row, so single rows are checkable at any size.
    """
    rows = np.asarray(rows)
    a = Sinv[rows, :] @ H
    b = (rho[rows, :] @ H) @ Sinv
    return -1j * (a @ rho - b)


def rho_dot_reference_split(delta, rho_ref, H_ref, dH, Sinv):
    """Eq. 10 (D = 0) written around a fixed reference density and Hamiltonian.

    With rho = rho_ref + delta and H = H_ref + dH, S^-1 H rho expands into
    S^-1 H_ref rho_ref + (S^-1 H_ref + S^-1 dH) delta + S^-1 dH rho_ref. The
    first term is fixed for a fixed reference; every other term is of the
    size of the departure from it. In exact arithmetic this is Eq. 10 itself;
    it is the form in which reduced-precision products carry only the
    departure. rhodot = -i (X - X^+), X = S^-1 H rho (S and H symmetric, rho
    Hermitian, so rho H S^-1 = X^+).
    """
    A_ref = Sinv @ H_ref
    B = Sinv @ dH
    X = A_ref @ rho_ref + (A_ref + B) @ delta + B @ rho_ref
    return -1j * (X - X.conj().T)


def renormalise_delta(delta, rho_ref, S, n_elec):
    """Restore Tr(rho S) = N_e (Sec. 2.3: the trace is a constant of the
    exact motion) by moving rho = rho_ref + delta along rho_ref:
    delta -= c rho_ref with c = (Tr(rho S) - N_e) / N_e, which needs
    Tr(rho_ref S) = N_e. A no-op for a density with the exact trace."""
    c = (electron_count(rho_ref + delta, S) - n_elec) / n_elec
    return delta - c * rho_ref


def euler_step(rho, rhodot, dt):
    """Single-step start of the two-step integrator (Sec. 2.3)."""
    return rho + dt * rhodot


def leapfrog_step(rho_prev, rhodot, dt):
    """rho_{i+1} = rho_{i-1} + 2 dt rhodot_i (Sec. 2.3, Eq. 19)."""
    return rho_prev + 2.0 * dt * rhodot


def kick(rho0, S, Sinv, positions, orb_offset, e0, direction):
    """Density matrix right after a delta pulse E0 delta(t) e (Sec. 2.2, Eq. 16).

    rho(0+) = 1/2 (K rho0 S K^+ S^-1 + S^-1 K S rho0 K^+),
    with K = exp(iV) the diagonal phase exp(-i E0 e . R_A(u)) (reading above).
    """
    e = np.asarray(direction, dtype=np.float64)
    e = e / np.linalg.norm(e)
    atom = atom_of_orbital(orb_offset)
    x = np.asarray(positions)[atom] @ e
    K = np.diag(np.exp(-1j * e0 * x))
    Kd = K.conj().T
    return 0.5 * (K @ rho0 @ S @ Kd @ Sinv + Sinv @ K @ S @ rho0 @ Kd)


def dipole(dq, positions):
    """mu = -sum_A dq_A R_A (Mulliken dipole; sign reading above)."""
    return -(np.asarray(dq)[:, None] * np.asarray(positions)).sum(axis=0)


def energy(rho, H0, gamma, dq, positions, field=None):
    """E = Re Tr(rho H0) + 1/2 dq gamma dq + sum_A dq_A R_A . E (Sec. 2.1, Eqs. 2-3)."""
    e_band = float(np.real(np.trace(rho @ H0)))
    e_coul = 0.5 * float(dq @ np.asarray(gamma) @ dq)
    e_ext = float(dq @ external_potential(positions, field)) if field is not None else 0.0
    return e_band + e_coul + e_ext


def stationarity_residual(rho, H, Sinv):
    """max |S^-1 H rho - rho H S^-1|, zero for a stationary state."""
    return float(np.abs(Sinv @ H @ rho - rho @ H @ Sinv).max())


# ----------------------------------------------------------------------------
# ground state
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class GroundState:
    rho: np.ndarray          # real symmetric [n_orb, n_orb]
    dq: np.ndarray           # [n_atoms], Mulliken fluctuations of rho
    H: np.ndarray            # SCC Hamiltonian built from dq_in
    eps: np.ndarray          # generalized eigenvalues of (H, S)
    C: np.ndarray            # eigenvectors, C^T S C = 1
    iterations: int
    residual: float          # max |dq_out - dq_in| at exit
    gap: float               # LUMO - HOMO


def _aufbau_density(H, S, n_occ):
    eps, C = scipy.linalg.eigh(H, S)
    f = np.zeros(len(eps))
    f[:n_occ] = 2.0
    rho = (C * f) @ C.T
    return rho, eps, C


def ground_state(system, tol=1e-13, maxiter=400, history=8, beta=0.3,
                 field=None) -> GroundState:
    """Self-consistent-charge ground state (Sec. 2.1).

    Start from dq = 0; each cycle builds H (Eqs. 6-7), solves the
    generalized eigenproblem H C = S C eps, fills the n_elec/2 lowest
    states with two electrons (rho = C f C^T) and recomputes dq (Eq. 5).
    The charge update uses Anderson mixing over the last ``history``
    residuals (Anderson, J. ACM 12, 547 (1965)); only the converged fixed
    point matters. Stops when max |dq_out - dq_in| < tol.
    """
    S, H0, gamma = system.S, system.H0, system.gamma
    off, q0 = system.orb_offset, system.q0
    n_occ = system.n_elec // 2
    V = external_potential(system.positions, field) if field is not None else None
    dq_in = np.zeros(system.n_atoms)
    xs, fs = [], []
    res = np.inf
    for it in range(1, maxiter + 1):
        H = scc_hamiltonian_fast(H0, S, gamma, dq_in, off, V)
        rho, eps, C = _aufbau_density(H, S, n_occ)
        dq_out = charge_fluctuations(rho, S, off, q0)
        r = dq_out - dq_in
        res = float(np.abs(r).max())
        if res < tol:
            break
        xs.append(dq_in.copy())
        fs.append(r.copy())
        xs, fs = xs[-history:], fs[-history:]
        if len(fs) == 1:
            dq_in = dq_in + beta * r
        else:
            dF = np.array([fs[k + 1] - fs[k] for k in range(len(fs) - 1)]).T
            dX = np.array([xs[k + 1] - xs[k] for k in range(len(xs) - 1)]).T
            g, *_ = np.linalg.lstsq(dF, r, rcond=None)
            dq_in = dq_in + beta * r - (dX + beta * dF) @ g
    gap = float(eps[n_occ] - eps[n_occ - 1]) if n_occ < len(eps) else np.inf
    return GroundState(rho=rho, dq=dq_out, H=H, eps=eps, C=C, iterations=it,
                       residual=res, gap=gap)


def scc_hamiltonian_fast(H0, S, gamma, dq, orb_offset, V=None):
    """Eqs. 6-7 in array form; equal to :func:`scc_hamiltonian` term by term."""
    atom = atom_of_orbital(orb_offset)
    shift = np.asarray(gamma) @ np.asarray(dq)
    if V is not None:
        shift = shift + V
    s = shift[atom]
    return np.asarray(H0) + 0.5 * np.asarray(S) * (s[:, None] + s[None, :])


# ----------------------------------------------------------------------------
# propagation
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Trajectory:
    rho: np.ndarray          # current density matrix after the last step
    rho_prev: np.ndarray     # the one before it
    step: int                # index of the current density matrix
    dipoles: np.ndarray      # [n, 3]  mu(t_k) of the density used at step k
    charges: np.ndarray      # [n, n_atoms]
    energies: np.ndarray     # [n]
    electrons: np.ndarray    # [n]  Re Tr(rho_k S)


def propagate(system, rho, n_steps, dt, rho_prev=None, step0=0, field=None,
              Sinv=None, record_energy=True) -> Trajectory:
    """Frozen-nuclei propagation with leapfrog (Sec. 2.3, Eq. 19).

    ``rho`` is the density at t_step0. Without ``rho_prev`` the first step
    is the Euler start; with it, every step is a leapfrog step.
    ``field[k]`` is E(t) at t = (step0 + k) dt, or None for no field.
    Records the dipole, charges, energy and electron count of the density
    matrix entering each step.
    """
    S, H0, gamma = system.S, system.H0, system.gamma
    off, q0, pos = system.orb_offset, system.q0, system.positions
    if Sinv is None:
        Sinv = inverse_overlap(S)
    cur = np.asarray(rho, dtype=np.complex128)
    prev = None if rho_prev is None else np.asarray(rho_prev, dtype=np.complex128)
    mus = np.zeros((n_steps, 3))
    dqs = np.zeros((n_steps, system.n_atoms))
    es = np.zeros(n_steps)
    ns = np.zeros(n_steps)
    for k in range(n_steps):
        E = None if field is None else field[k]
        dq = charge_fluctuations(cur, S, off, q0)
        V = external_potential(pos, E) if E is not None else None
        H = scc_hamiltonian_fast(H0, S, gamma, dq, off, V)
        mus[k] = dipole(dq, pos)
        dqs[k] = dq
        if record_energy:
            es[k] = energy(cur, H0, gamma, dq, pos, E)
            ns[k] = electron_count(cur, S)
        rd = rho_dot(cur, H, Sinv)
        if prev is None:
            nxt = euler_step(cur, rd, dt)
        else:
            nxt = leapfrog_step(prev, rd, dt)
        prev, cur = cur, nxt
    return Trajectory(rho=cur, rho_prev=prev, step=step0 + n_steps, dipoles=mus,
                      charges=dqs, energies=es, electrons=ns)


# ----------------------------------------------------------------------------
# spectra
# ----------------------------------------------------------------------------

def polarizability(t, mu_along, e0, omega, tau=None):
    """alpha(w) = (mu(w) - mu_0) / E0 (Sec. 2.2, Eq. 17) by direct summation.

    mu(w) is the transform sum_n (mu(t_n) - mu(t_0)) exp(i w t_n) dt of the
    dipole along the kick direction, damped by exp(-t/tau) before the
    transform when ``tau`` is given (Sec. 3.1).
    """
    t = np.asarray(t, dtype=np.float64)
    d = np.asarray(mu_along, dtype=np.float64) - float(mu_along[0])
    if tau is not None:
        d = d * np.exp(-t / tau)
    dt = t[1] - t[0]
    w = np.asarray(omega, dtype=np.float64)
    return (np.exp(1j * np.outer(w, t)) @ d) * dt / e0


def cross_section(omega, alpha_avg):
    """sigma(w) = 4 pi w / c Im(alpha_bar(w)) (Sec. 2.2, Eq. 18)."""
    return 4.0 * np.pi * np.asarray(omega) / C_AU * np.imag(alpha_avg)


# ----------------------------------------------------------------------------
# transient absorption (Sec. 5.1)
# ----------------------------------------------------------------------------

def effective_polarizability(t, mu_probe, mu_pump, e0, omega, tau=None):
    """Effective polarizability of one probe (Sec. 5.1): the Fourier transform
    of the probe's dipole minus the pump-only dipole over the same times,
    divided by the kick strength, damped by exp(-t/tau) when ``tau`` is given.

    ``t`` counts from the probe kick; both dipoles are the component along
    the kick direction. Direct summation over the samples, as
    ``polarizability`` but with the pump-only run as the reference.
    """
    t = np.asarray(t, dtype=np.float64)
    d = np.asarray(mu_probe, dtype=np.float64) - np.asarray(mu_pump, dtype=np.float64)
    if tau is not None:
        d = d * np.exp(-t / tau)
    dt = t[1] - t[0]
    w = np.asarray(omega, dtype=np.float64)
    return (np.exp(1j * np.outer(w, t)) @ d) * dt / e0


def transient_cross_section(omega, alphas):
    """sigma(w, tau) = 4 pi w / c Im(alpha_eff(w, tau)) (Sec. 5.1), with
    alpha_eff the mean of the diagonal effective polarizabilities over the
    kick directions and the pump phases: ``alphas`` is
    [n_delay, n_average, n_omega]."""
    a = np.asarray(alphas).mean(axis=1)
    return 4.0 * np.pi * np.asarray(omega)[None, :] / C_AU * np.imag(a)


def delta_absorbance(sigma, ref_index):
    """Absorption change against the spectrum at one delay, the end of the
    pump (Sec. 5.2): Delta A(tau) = A(tau) - A(t_p), rows = delays."""
    sigma = np.asarray(sigma)
    return sigma - sigma[ref_index][None, :]


def gaussian_filter_delay(values, delay_step, width):
    """Low-pass along the delay axis (rows) as described in Sec. 5.1: Fourier
    transform over the delays, multiply by exp(-nu^2 / (2 width^2)) (nu in
    cycles per unit time), transform back. The transform is the discrete
    one over the given delays (periodic)."""
    v = np.asarray(values, dtype=np.float64)
    n = v.shape[0]
    nu = np.fft.fftfreq(n, d=delay_step)
    g = np.exp(-nu ** 2 / (2.0 * width ** 2))
    return np.real(np.fft.ifft(g[:, None] * np.fft.fft(v, axis=0), axis=0))

