"""Pins of the absolute scale of the oracle's spectra (Sec. 2.2, Eqs. 17-18;
Sec. 5.1) against physics that does not go through the spectrum code.

* Eq. 17 (alpha = transform of the dipole change / E0): the zero-frequency
  limit of the damped transform of a kicked SCC run is the static
  polarizability d mu / dE, taken by central differences of SCC ground
  states in a static field. This fixes the transform's time step, the
  division by E0 and the sign convention that ties the kick phase, the
  field potential and the dipole together.
* Eq. 18 (sigma = 4 pi w / c Im alpha): for a damped sum of lines
  chi(t) = sum_I A_I sin(w_I t) exp(-t / tau), int_0^inf w Im chi(w) dw
  = (pi / 2) chi'(0+) = (pi / 2) sum_I A_I w_I for any tau (the inverse
  transform of -i w chi(w) at t = 0 is the mean of chi'(0-) = 0 and
  chi'(0+)). So int sigma dw = (2 pi^2 / c) sum_I A_I w_I, with the lines
  A_I, w_I of a non-SCC system from its exact generalized
  eigendecomposition.
* Sec. 5.1 (sigma(w, tau) of the pump-probe protocol): with the pump
  switched off the pump-only run is the stationary ground state, every
  probe is a ground-state kick, and the transient cross-section at every
  delay must equal the ground-state cross-section of Eq. 18 with
  alpha_bar = Tr(alpha) / 3.

Constants are typed here from their definitions, not taken from the
oracle: c = 137.035999084 au (CODATA 2018).
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W

C_LIGHT = 137.035999084


@pytest.fixture(scope="module")
def benzene():
    return W.benzene()


def _transform(t, mu, e0, omega, tau, chunks=1):
    """Eq. 17 through the oracle, a block of frequencies at a time (memory)."""
    return np.concatenate([O.polarizability(t, mu, e0, w, tau=tau)
                           for w in np.array_split(np.asarray(omega), chunks)])


def test_static_limit_of_the_kick_spectrum_is_the_static_polarizability(benzene):
    """Re alpha(0) of a weakly kicked SCC run, damped by exp(-t / tau), equals
    d mu_x / dE_x of the SCC ground state in a static field. The damping
    leaves sum_I A_I w_I / (w_I^2 + tau^-2) instead of sum_I A_I / w_I, a
    relative error of about (w_min tau)^-2 = 1.4e-3 at the benzene gap; the
    leapfrog frequency shift at dt = 0.05 is smaller still."""
    s = benzene
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    h = 1e-4
    mu_p = O.dipole(O.ground_state(s, tol=1e-13, field=(h, 0.0, 0.0)).dq, s.positions)
    mu_m = O.dipole(O.ground_state(s, tol=1e-13, field=(-h, 0.0, 0.0)).dq, s.positions)
    static = (mu_p[0] - mu_m[0]) / (2 * h)
    assert static > 1.0                                   # electrons follow the field
    kappa, dt, tau = 1e-5, 0.05, 100.0
    n = int(round(10 * tau / dt))
    rk = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, kappa, (1.0, 0.0, 0.0))
    tr = O.propagate(s, rk, n, dt, Sinv=Sinv, record_energy=False)
    t = np.arange(n) * dt
    a0 = O.polarizability(t, tr.dipoles[:, 0], kappa, [0.0], tau=tau)[0]
    assert abs(a0.imag) < 1e-12 * abs(a0)
    assert abs(a0.real / static - 1.0) < 2e-3, (a0.real, static)


def _lines(s):
    """Lines of the x-x linear response of a non-SCC system per unit kick:
    chi(t) = sum_I A_I sin(w_I t), from the generalized eigenbasis
    (A_I = (f_j - f_i) M_ij^2 / 2, M = C^T (S X + X S) C, w_I = eps_i - eps_j)."""
    eps, C = scipy.linalg.eigh(s.H0, s.S)
    n_occ = s.n_elec // 2
    counts = np.diff(np.asarray(s.orb_offset))
    atom = np.repeat(np.arange(len(counts)), counts)
    Xd = np.diag(np.asarray(s.positions)[atom, 0])
    M = C.T @ (s.S @ Xd + Xd @ s.S) @ C
    f = np.zeros(len(eps))
    f[:n_occ] = 2.0
    w, A = [], []
    for i in range(len(eps)):
        for j in range(len(eps)):
            if eps[i] > eps[j] and f[j] != f[i]:
                w.append(eps[i] - eps[j])
                A.append(0.5 * (f[j] - f[i]) * M[i, j] ** 2)
    return np.array(w), np.array(A), eps, C


def test_integrated_cross_section_sum_rule(benzene):
    """int_0^Omega sigma(w) dw of a kicked non-SCC run equals
    (2 pi^2 / c) sum_I A_I w_I. Omitted: the tail beyond Omega, a relative
    2 / (tau Omega) = 1.7e-3, and the leapfrog frequency shift of the upper
    lines, (w dt)^2 / 6, a few 1e-3 at dt = 0.05."""
    s = dataclasses.replace(benzene, gamma=np.zeros_like(benzene.gamma))
    w, A, eps, C = _lines(s)
    exact = 2.0 * np.pi ** 2 / C_LIGHT * float((A * w).sum())
    assert exact > 0
    n_occ = s.n_elec // 2
    rho0 = 2.0 * C[:, :n_occ] @ C[:, :n_occ].T
    Sinv = O.inverse_overlap(s.S)
    kappa, dt, tau = 1e-5, 0.05, 100.0
    n = int(round(8 * tau / dt))
    rk = O.kick(rho0, s.S, Sinv, s.positions, s.orb_offset, kappa, (1.0, 0.0, 0.0))
    tr = O.propagate(s, rk, n, dt, Sinv=Sinv, record_energy=False)
    t = np.arange(n) * dt
    omega = np.linspace(0.0, 12.0, 4801)                # 4 points per line width 1/tau
    sigma = O.cross_section(omega, _transform(t, tr.dipoles[:, 0], kappa, omega, tau, 24))
    got = np.trapezoid(sigma, omega)
    assert abs(got / exact - 1.0) < 1e-2, (got, exact)
    # each well separated line carries its own share, (2 pi^2 / c) A_I w_I
    order = np.argsort(-A * w)
    top = w[order[0]]
    others = np.delete(w, order[0])
    gap = np.abs(others - top).min()
    if gap > 0.3:
        win = np.abs(omega - top) < 0.5 * gap
        share = np.trapezoid(sigma[win], omega[win])
        line = 2.0 * np.pi ** 2 / C_LIGHT * A[order[0]] * top
        assert abs(share / line - 1.0) < 5e-2, (share, line)


def test_transient_spectrum_without_pump_is_the_ground_state_spectrum(benzene):
    """Sec. 5.1 with E_b = 0: probes branched from the (stationary) pump-only
    run at several delays, kicked along x, y and z, each with four pump
    phases, give sigma(w, tau) equal at every delay to the ground-state
    sigma(w) of Eq. 18 with alpha_bar = Tr(alpha) / 3."""
    s = benzene
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    kappa, dt, tau = 1e-4, 0.2, 40.0
    n = 600
    t = np.arange(n) * dt
    omega = np.linspace(0.05, 1.5, 120)
    pump = O.propagate(s, gs.rho.astype(np.complex128), 400, dt, Sinv=Sinv, record_energy=False)
    axes = np.eye(3)

    def probe_alpha(rho_start, mu_ref, e):
        rk = O.kick(rho_start, s.S, Sinv, s.positions, s.orb_offset, kappa, e)
        tr = O.propagate(s, rk, n, dt, Sinv=Sinv, record_energy=False)
        return tr.dipoles @ e, O.effective_polarizability(t, tr.dipoles @ e, mu_ref @ e,
                                                          kappa, omega, tau=tau)

    # ground state spectrum of Eq. 17-18
    diag = []
    for e in axes:
        mu_e, _ = probe_alpha(gs.rho, np.zeros(3), e)
        diag.append(O.polarizability(t, mu_e, kappa, omega, tau=tau))
    sigma_gs = O.cross_section(omega, np.mean(diag, axis=0))
    assert sigma_gs.max() > 0
    # the pump-probe protocol with the pump off: delays 0 and 400 dt
    mu_pump = O.dipole(gs.dq, s.positions)
    rows = []
    for rho_delay in (gs.rho, pump.rho):
        per = []
        for e in axes:
            _, a = probe_alpha(rho_delay, np.tile(mu_pump, (n, 1)), e)
            per.extend([a] * 4)                           # four pump phases, identical without a pump
        rows.append(per)
    sigma_t = O.transient_cross_section(omega, np.array(rows))
    for k in range(2):
        assert np.abs(sigma_t[k] - sigma_gs).max() < 1e-6 * np.abs(sigma_gs).max(), k
