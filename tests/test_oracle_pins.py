"""Pins of the CPU oracle against closed forms, invariants and special cases.

None of these compares the oracle with a retyped copy of itself: each
check is a consequence of the equations that a plausible mistake (a
dropped term, a wrong sign, a swapped index or factor) would break.
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from tests import exact as X


def non_scc(system):
    """The same system with the SCC kernel switched off (gamma = 0)."""
    return dataclasses.replace(system, gamma=np.zeros_like(system.gamma))


def aufbau(H, S, n_occ):
    eps, C = scipy.linalg.eigh(H, S)
    return 2.0 * C[:, :n_occ] @ C[:, :n_occ].T


@pytest.fixture(scope="module")
def benzene():
    return W.benzene()


@pytest.fixture(scope="module")
def flake():
    return W.flake_c24h16()


@pytest.fixture(scope="module")
def flake_gs(flake):
    return O.ground_state(flake)


# ---------------------------------------------------------------- P3 / P1 / P11

def test_leapfrog_matches_discrete_closed_form(benzene):
    """Euler-started leapfrog equals its exact scalar recurrence per eigen-pair."""
    s = non_scc(benzene)
    Sinv = O.inverse_overlap(s.S)
    rho0 = aufbau(s.H0, s.S, s.n_occ)
    rk = O.kick(rho0, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.3, 0.0))
    dt, n = 0.2, 2000
    tr = O.propagate(s, rk, n, dt, Sinv=Sinv, record_energy=False)
    ref = X.exact_leapfrog(rk, s.H0, s.S, dt, n)
    signal = np.abs(rk - rho0).max()
    assert np.abs(tr.rho - ref).max() / signal < 1e-9
    ref_prev = X.exact_leapfrog(rk, s.H0, s.S, dt, n - 1)
    assert np.abs(tr.rho_prev - ref_prev).max() / signal < 1e-9


def test_converges_to_exact_continuous_dynamics(benzene):
    """Error against exp(-i eps t) evolution falls as dt^2 (second order)."""
    s = non_scc(benzene)
    Sinv = O.inverse_overlap(s.S)
    rho0 = aufbau(s.H0, s.S, s.n_occ)
    rk = O.kick(rho0, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (0.0, 1.0, 0.0))
    T = 4.0
    errs = []
    for dt in (0.04, 0.02):
        n = int(round(T / dt))
        tr = O.propagate(s, rk, n, dt, Sinv=Sinv, record_energy=False)
        errs.append(np.abs(tr.rho - X.exact_continuous(rk, s.H0, s.S, T)).max())
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, ratio


def test_orthogonal_basis_reduces_to_unitary_evolution():
    """S = 1: rhodot = -i[H, rho]; compare with expm(-iHt) rho expm(iHt)."""
    rng = np.random.default_rng(3)
    n = 12
    A = rng.standard_normal((n, n)) * 0.1
    H = (A + A.T) / 2.0
    pos = rng.standard_normal((n, 3))
    sysm = W.System(species=["H"] * n, positions=pos,
                    orb_offset=np.arange(n + 1, dtype=np.int32), S=np.eye(n), H0=H,
                    gamma=np.zeros((n, n)), q0=np.ones(n), n_elec=n)
    rho0 = aufbau(H, np.eye(n), n // 2)
    rk = O.kick(rho0, np.eye(n), np.eye(n), pos, sysm.orb_offset, 0.05, (1.0, 0.0, 0.0))
    # orthogonal kick is K rho0 K^+ exactly
    K = np.diag(np.exp(-1j * 0.05 * pos[:, 0]))
    assert np.abs(rk - K @ rho0 @ K.conj().T).max() < 1e-15
    T, dt = 3.0, 0.005
    tr = O.propagate(sysm, rk, int(round(T / dt)), dt, record_energy=False)
    U = scipy.linalg.expm(-1j * H * T)
    ref = U @ rk @ U.conj().T
    assert np.abs(tr.rho - ref).max() < 1e-5


# ---------------------------------------------------------------- P2 / P12

def test_dimer_hand_derived_response():
    """Two-orbital dimer: d mu_x(t) = kappa d^2 / (1 - s^2) sin(w t), w = 2(alpha s - beta)/(1 - s^2).

    Derived by hand from the bonding/antibonding pair (1, +-1)/sqrt(2(1 +- s)).
    Pins the kick sign (positive initial slope), the dipole sign and scale.
    """
    d, s_, a, b = 1.4, 0.3, -0.5, -0.35
    sysm = W.dimer(d=d, s=s_, alpha=a, beta=b)
    Sinv = O.inverse_overlap(sysm.S)
    rho0 = aufbau(sysm.H0, sysm.S, 1)
    kappa = 1e-5
    rk = O.kick(rho0, sysm.S, Sinv, sysm.positions, sysm.orb_offset, kappa, (1.0, 0.0, 0.0))
    w = 2.0 * (a * s_ - b) / (1.0 - s_ ** 2)
    amp = kappa * d ** 2 / (1.0 - s_ ** 2)
    dt, n = 0.005, 4000
    tr = O.propagate(sysm, rk, n, dt, Sinv=Sinv, record_energy=False)
    t = np.arange(n) * dt
    mu0 = O.dipole(O.charge_fluctuations(rho0, sysm.S, sysm.orb_offset, sysm.q0), sysm.positions)
    dmu = tr.dipoles[:, 0] - mu0[0]
    ref = amp * np.sin(w * t)
    assert np.abs(dmu - ref).max() / amp < 2e-3
    assert dmu[40] > 0  # electrons pushed against the field: positive slope


def test_linear_response_closed_form(benzene):
    """Kick along x, measure y and x: sum of sines at eigenvalue differences."""
    s = non_scc(benzene)
    Sinv = O.inverse_overlap(s.S)
    rho0 = aufbau(s.H0, s.S, s.n_occ)
    mu0 = O.dipole(O.charge_fluctuations(rho0, s.S, s.orb_offset, s.q0), s.positions)
    kick_dir = (1.0, 0.0, 0.0)
    T, dt = 6.0, 0.005
    n = int(round(T / dt))
    t = np.arange(n) * dt
    resid = []
    for kappa in (1e-4, 1e-5):
        rk = O.kick(rho0, s.S, Sinv, s.positions, s.orb_offset, kappa, kick_dir)
        tr = O.propagate(s, rk, n, dt, Sinv=Sinv, record_energy=False)
        for m in range(2):
            meas = np.eye(3)[m]
            ref = X.linear_response_dipole(s.H0, s.S, s.positions, s.orb_offset, s.n_occ,
                                           kick_dir, meas, kappa, t)
            got = tr.dipoles[:, m] - mu0[m]
            scale = np.abs(X.linear_response_dipole(s.H0, s.S, s.positions, s.orb_offset,
                                                    s.n_occ, kick_dir, kick_dir, kappa, t)).max()
            resid.append(np.abs(got - ref).max() / scale)
    assert max(resid) < 5e-3, resid


# ---------------------------------------------------------------- invariants

def test_electron_number_and_hermiticity_conserved(flake, flake_gs):
    """Tr(rho S) = N_e and rho = rho^+ along an SCC run with a field (Sec. 2.3)."""
    s = flake
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(flake_gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.0, 0.0))
    assert abs(O.electron_count(rk, s.S) - s.n_elec) < 1e-12
    n = 300
    field = W.sin2_pulse(np.arange(n) * 0.2, 0.005, 0.1, n * 0.2, (0.0, 1.0, 0.0))
    tr = O.propagate(s, rk, n, 0.2, Sinv=Sinv, field=field)
    assert np.abs(tr.electrons - s.n_elec).max() < 1e-11
    assert np.abs(tr.rho - tr.rho.conj().T).max() < 1e-14 * np.abs(tr.rho).max() * 100


def test_ground_state_is_stationary_and_idempotent(flake, flake_gs):
    s, gs = flake, flake_gs
    Sinv = O.inverse_overlap(s.S)
    assert gs.residual < 1e-12
    assert gs.gap > 0.01
    assert np.abs(gs.rho @ s.S @ gs.rho - 2.0 * gs.rho).max() < 1e-12
    assert O.stationarity_residual(gs.rho, gs.H, Sinv) < 1e-12
    tr = O.propagate(s, gs.rho, 200, 0.2, Sinv=Sinv)
    assert np.abs(tr.rho - gs.rho).max() < 1e-11
    assert np.abs(tr.dipoles - tr.dipoles[0]).max() < 1e-11


def test_scc_ground_state_minimises_energy(flake, flake_gs):
    """The SCC fixed point is a stationary minimum of E[rho] over occupied-virtual rotations.

    This pins the 1/2 factors and signs of the SCC Hamiltonian (Eq. 6)
    against the Coulomb energy (Eq. 3): a wrong factor moves the fixed
    point off the energy minimum and leaves a first-order slope.
    """
    s, gs = flake, flake_gs
    n_occ = s.n_occ

    def E(rho):
        dq = O.charge_fluctuations(rho, s.S, s.orb_offset, s.q0)
        return O.energy(rho, s.H0, s.gamma, dq, s.positions)

    rng = np.random.default_rng(5)
    n = s.n_orb
    G = np.zeros((n, n))
    G[n_occ:, :n_occ] = rng.standard_normal((n - n_occ, n_occ))
    G = G - G.T
    e0 = E(gs.rho)
    for h in (1e-3, 5e-4):
        U = scipy.linalg.expm(h * G)
        Cp = gs.C @ U
        rp = 2.0 * Cp[:, :n_occ] @ Cp[:, :n_occ].T
        rm_ = 2.0 * (gs.C @ U.T)[:, :n_occ] @ (gs.C @ U.T)[:, :n_occ].T
        ep, em = E(rp), E(rm_)
        slope = (ep - em) / (2 * h)
        curv = (ep + em - 2 * e0) / h ** 2
        assert curv > 0
        assert abs(slope) < 1e-6 * curv


def test_energy_conservation_and_work(flake, flake_gs):
    """Free propagation: E bounded to O(dt^2), no drift; driven: dE = -int mu . dE/dt."""
    s = flake
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(flake_gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-2, (1.0, 0.0, 0.0))
    spreads = []
    for dt in (0.2, 0.1):
        tr = O.propagate(s, rk, int(round(40 / dt)), dt, Sinv=Sinv)
        spreads.append(tr.energies.max() - tr.energies.min())
    assert 3.0 < spreads[0] / spreads[1] < 5.0
    # driven run from the ground state
    dt, n = 0.05, 2000
    t = np.arange(n) * dt
    omega, e0, tp = 0.3, 0.01, n * dt
    field = W.sin2_pulse(t, e0, omega, tp, (1.0, 0.5, 0.0))
    tr = O.propagate(s, flake_gs.rho, n, dt, Sinv=Sinv, field=field)
    # analytic dE/dt of the pulse
    eps_ = 1e-6
    dfield = (W.sin2_pulse(t + eps_, e0, omega, tp, (1.0, 0.5, 0.0))
              - W.sin2_pulse(t - eps_, e0, omega, tp, (1.0, 0.5, 0.0))) / (2 * eps_)
    power = -(tr.dipoles * dfield).sum(axis=1)
    work = np.concatenate([[0.0], np.cumsum(0.5 * (power[1:] + power[:-1]) * dt)])
    dE = tr.energies - tr.energies[0]
    assert np.abs(dE).max() > 1e-5
    assert np.abs(dE - work).max() < 2e-2 * np.abs(dE).max()


def test_time_reversal(flake, flake_gs):
    """Swap (rho_N, rho_{N-1}) and step with -dt: returns to the start (Sec. 2.3)."""
    s = flake
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(flake_gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 1.0, 0.0))
    n, dt = 150, 0.2
    t = np.arange(n + 1) * dt
    field = W.sin2_pulse(t, 0.003, 0.2, n * dt, (0.0, 1.0, 0.0))
    fw = O.propagate(s, rk, n, dt, Sinv=Sinv, field=field[:n], record_energy=False)
    # backwards: current rho_{N-1}, previous rho_N, fields at t_{N-1} ... t_1
    bw = O.propagate(s, fw.rho_prev, n - 1, -dt, rho_prev=fw.rho, Sinv=Sinv,
                     field=field[n - 1:0:-1], record_energy=False)
    assert np.abs(bw.rho - rk).max() < 1e-11


def test_translation_and_permutation_invariance(flake, flake_gs):
    s = flake
    Sinv = O.inverse_overlap(s.S)
    n = 120
    field = W.sin2_pulse(np.arange(n) * 0.2, 0.005, 0.15, n * 0.2, (1.0, 0.0, 0.0))

    def run(sysm, rho0):
        Si = O.inverse_overlap(sysm.S)
        rk = O.kick(rho0, sysm.S, Si, sysm.positions, sysm.orb_offset, 1e-3, (0.3, 1.0, 0.0))
        return O.propagate(sysm, rk, n, 0.2, Sinv=Si, field=field, record_energy=False)

    base = run(s, flake_gs.rho)
    moved = dataclasses.replace(s, positions=s.positions + np.array([3.0, -2.0, 1.0]))
    tr = run(moved, flake_gs.rho)
    assert np.abs(tr.dipoles - base.dipoles).max() < 1e-10
    # reverse the atom order (orbital blocks move with their atoms)
    perm = np.arange(s.n_atoms)[::-1]
    off = s.orb_offset
    orb = np.concatenate([np.arange(off[a], off[a + 1]) for a in perm])
    counts = np.diff(off)[perm]
    off2 = np.zeros(s.n_atoms + 1, dtype=np.int32)
    off2[1:] = np.cumsum(counts)
    ps = dataclasses.replace(s, species=[s.species[a] for a in perm], positions=s.positions[perm],
                             orb_offset=off2, S=s.S[np.ix_(orb, orb)], H0=s.H0[np.ix_(orb, orb)],
                             gamma=s.gamma[np.ix_(perm, perm)], q0=s.q0[perm])
    tr = run(ps, flake_gs.rho[np.ix_(orb, orb)])
    assert np.abs(tr.dipoles - base.dipoles).max() < 1e-10
    assert np.abs(tr.charges[:, ::-1] - base.charges).max() < 1e-10


def test_kick_properties(flake, flake_gs):
    s = flake
    Sinv = O.inverse_overlap(s.S)
    mu0 = O.dipole(flake_gs.dq, s.positions)
    devs = []
    for kappa in (1e-2, 5e-3):
        rk = O.kick(flake_gs.rho, s.S, Sinv, s.positions, s.orb_offset, kappa, (1.0, 0.0, 0.0))
        assert abs(O.electron_count(rk, s.S) - s.n_elec) < 1e-12
        assert np.abs(rk - rk.conj().T).max() < 1e-14
        # first-order change is purely imaginary for a real rho0
        assert np.abs(rk.real - flake_gs.rho).max() < 20 * kappa ** 2
        dq = O.charge_fluctuations(rk, s.S, s.orb_offset, s.q0)
        devs.append(np.abs(O.dipole(dq, s.positions) - mu0).max())
    assert 3.0 < devs[0] / devs[1] < 5.0  # mu(0+) - mu0 = O(kappa^2)


def test_mulliken_populations_and_special_cases(flake, flake_gs):
    s, gs = flake, flake_gs
    rng = np.random.default_rng(9)
    re, im = W.random_hermitian_pair(s.n_orb, 4, scale=0.1, base=gs.rho)
    rho = re + 1j * im
    q = O.mulliken_populations(rho, s.S, s.orb_offset)
    # the symmetrised definition 1/2 (rho S + S rho) gives the same diagonal
    sym = np.real(np.diag(0.5 * (rho @ s.S + s.S @ rho)))
    off = s.orb_offset
    q_sym = np.array([sym[off[a]:off[a + 1]].sum() for a in range(s.n_atoms)])
    assert np.abs(q - q_sym).max() < 1e-13
    assert abs(q.sum() - np.real(np.trace(rho @ s.S))) < 1e-12
    # orthogonal basis: populations are diagonal sums of rho
    n = 6
    rr = rng.standard_normal((n, n))
    rr = rr + rr.T
    qo = O.mulliken_populations(rr, np.eye(n), np.array([0, 2, 3, 6]))
    assert np.allclose(qo, [rr[0, 0] + rr[1, 1], rr[2, 2], rr[3, 3] + rr[4, 4] + rr[5, 5]])


def test_hamiltonian_forms_agree(flake, flake_gs):
    s = flake
    V = O.external_potential(s.positions, np.array([0.01, -0.02, 0.005]))
    h1 = O.scc_hamiltonian(s.H0, s.S, s.gamma, flake_gs.dq, s.orb_offset, V)
    h2 = O.scc_hamiltonian_fast(s.H0, s.S, s.gamma, flake_gs.dq, s.orb_offset, V)
    assert np.abs(h1 - h2).max() < 1e-15
    # a uniform potential shift c adds c S to H, which commutes out of rhodot
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(flake_gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.0, 0.0))
    c = 0.37
    h3 = O.scc_hamiltonian_fast(s.H0, s.S, s.gamma, flake_gs.dq, s.orb_offset, V + c)
    assert np.abs(h3 - h2 - c * s.S).max() < 1e-14
    assert np.abs(O.rho_dot(rk, h3, Sinv) - O.rho_dot(rk, h2, Sinv)).max() < 1e-13


# ---------------------------------------------------------------- P15 stability

def test_leapfrog_stability_threshold(benzene):
    s = non_scc(benzene)
    eps = scipy.linalg.eigh(s.H0, s.S, eigvals_only=True)
    spread = eps[-1] - eps[0]
    Sinv = O.inverse_overlap(s.S)
    rho0 = aufbau(s.H0, s.S, s.n_occ)
    rk = O.kick(rho0, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.0, 0.0))
    stable = O.propagate(s, rk, 400, 0.9 / spread, Sinv=Sinv, record_energy=False)
    unstable = O.propagate(s, rk, 400, 1.2 / spread, Sinv=Sinv, record_energy=False)
    assert np.abs(stable.rho).max() < 10.0
    assert np.abs(unstable.rho).max() > 1e3


# ---------------------------------------------------------------- spectrum

def test_dimer_spectrum_peak_and_sign():
    """Im alpha > 0 and the peak sits at the dimer transition energy."""
    d, s_, a, b = 1.4, 0.3, -0.5, -0.35
    sysm = W.dimer(d=d, s=s_, alpha=a, beta=b)
    Sinv = O.inverse_overlap(sysm.S)
    rho0 = aufbau(sysm.H0, sysm.S, 1)
    kappa = 1e-4
    rk = O.kick(rho0, sysm.S, Sinv, sysm.positions, sysm.orb_offset, kappa, (1.0, 0.0, 0.0))
    dt, n = 0.05, 8000
    tr = O.propagate(sysm, rk, n, dt, Sinv=Sinv, record_energy=False)
    t = np.arange(n) * dt
    w0 = 2.0 * (a * s_ - b) / (1.0 - s_ ** 2)
    omegas = np.linspace(0.2 * w0, 2.0 * w0, 721)
    alpha = O.polarizability(t, tr.dipoles[:, 0], kappa, omegas, tau=60.0)
    sigma = O.cross_section(omegas, alpha)
    k = int(np.argmax(sigma))
    assert sigma[k] > 0
    assert abs(omegas[k] - w0) < 0.01 * w0
    # static limit: alpha(w -> small) approaches the positive static polarisability
    assert np.real(alpha[0]) > 0


def test_row_sampled_rhodot_equals_full(flake, flake_gs):
    """Row-restricted Eq. 10 equals the rows of the full (pinned) derivative."""
    s = flake
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(flake_gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-2, (1.0, 1.0, 0.0))
    H = O.scc_hamiltonian_fast(s.H0, s.S, s.gamma, flake_gs.dq, s.orb_offset)
    rows = [0, 7, 50, s.n_orb - 1]
    full = O.rho_dot(rk, H, Sinv)
    assert np.abs(O.rho_dot_rows(rk, H, Sinv, rows) - full[rows]).max() < 1e-14


def test_reference_split_form_equals_eq10(flake, flake_gs):
    """The reference-density form of Eq. 10 equals the direct form (pinned above)
    for a kicked SCC state in a field, and its reference part alone vanishes at
    the stationary ground state."""
    s = flake
    Sinv = O.inverse_overlap(s.S)
    rho_ref = flake_gs.rho
    H_ref = O.scc_hamiltonian_fast(s.H0, s.S, s.gamma, flake_gs.dq, s.orb_offset)
    rk = O.kick(rho_ref, s.S, Sinv, s.positions, s.orb_offset, 1e-2, (1.0, 0.5, 0.0))
    tr = O.propagate(s, rk, 30, 0.2, Sinv=Sinv, record_energy=False,
                     field=np.tile([0.0, 0.003, 0.0], (30, 1)))
    rho = tr.rho
    dq = O.charge_fluctuations(rho, s.S, s.orb_offset, s.q0)
    H = O.scc_hamiltonian_fast(s.H0, s.S, s.gamma, dq, s.orb_offset,
                               O.external_potential(s.positions, [0.0, 0.003, 0.0]))
    direct = O.rho_dot(rho, H, Sinv)
    split = O.rho_dot_reference_split(rho - rho_ref, rho_ref, H_ref, H - H_ref, Sinv)
    assert np.abs(split - direct).max() < 1e-13 * np.abs(direct).max() + 1e-15
    assert np.abs(direct).max() > 1e-4
    zero = np.zeros_like(rho)
    still = O.rho_dot_reference_split(zero, rho_ref, H_ref, np.zeros_like(H_ref), Sinv)
    assert np.abs(still).max() < 1e-10


def test_trace_renormalisation(flake, flake_gs):
    """Moving along rho_ref restores Tr(rho S) = N_e exactly and is a no-op on
    a density that already has it (leapfrog keeps the trace, Sec. 2.3)."""
    s = flake
    Sinv = O.inverse_overlap(s.S)
    rho_ref = flake_gs.rho
    rk = O.kick(rho_ref, s.S, Sinv, s.positions, s.orb_offset, 1e-2, (0.0, 1.0, 0.0))
    delta = rk - rho_ref
    same = O.renormalise_delta(delta, rho_ref, s.S, s.n_elec)
    assert np.abs(same - delta).max() < 1e-15
    off = delta + 1e-3 * rho_ref                  # trace off by 1e-3 N_e
    fixed = O.renormalise_delta(off, rho_ref, s.S, s.n_elec)
    assert abs(O.electron_count(rho_ref + fixed, s.S) - s.n_elec) < 1e-12
    assert np.abs(fixed - delta).max() < 1e-14


# ---------------------------------------------------------------- transient absorption

def test_effective_polarizability_closed_form():
    """A damped probe-minus-pump signal A sin(w0 t) transforms to a sum of two
    geometric series: sum_n z^n = (1 - z^N) / (1 - z), z = exp((i w +- i w0 - 1/tau) dt)."""
    dt, n, w0, amp, tau, e0 = 0.2, 3000, 0.37, 2e-4, 150.0, 1e-3
    t = np.arange(n) * dt
    pump = 0.05 * np.cos(0.11 * t) + 0.3             # pump-only signal, cancelled exactly
    probe = pump + amp * np.sin(w0 * t)
    omega = np.linspace(0.05, 1.0, 97)
    alpha = O.effective_polarizability(t, probe, pump, e0, omega, tau=tau)

    def geo(z):
        return (1.0 - z ** n) / (1.0 - z)

    zp = np.exp((1j * (omega + w0) - 1.0 / tau) * dt)
    zm = np.exp((1j * (omega - w0) - 1.0 / tau) * dt)
    exact = amp * (geo(zp) - geo(zm)) / (2j) * dt / e0
    assert np.abs(alpha - exact).max() < 1e-10 * np.abs(exact).max()
    # absorption peak at w0 with Im alpha > 0
    k = int(np.argmax(np.imag(alpha)))
    assert abs(omega[k] - w0) < 0.02 and np.imag(alpha[k]) > 0


def test_phase_average_cancels_pump_probe_beat():
    """Averaging over four pump phases 0, pi/2, pi, 3 pi/2 removes a response
    term that carries the pump phase (Sec. 5.1), keeping the phase-free part."""
    dt, n, e0 = 0.2, 2000, 1e-3
    t = np.arange(n) * dt
    omega = np.linspace(0.1, 0.8, 40)
    zero = np.zeros(n)
    base = 1e-4 * np.sin(0.4 * t)
    alphas = []
    for phi in (0.0, 0.5 * np.pi, np.pi, 1.5 * np.pi):
        beat = 3e-5 * np.sin(0.25 * t + phi)
        alphas.append(O.effective_polarizability(t, base + beat, zero, e0, omega))
    avg = O.transient_cross_section(omega, np.array(alphas)[None, :, :])[0]
    clean = O.transient_cross_section(
        omega, O.effective_polarizability(t, base, zero, e0, omega)[None, None, :])[0]
    assert np.abs(avg - clean).max() < 1e-12 * np.abs(clean).max()
    single = O.transient_cross_section(omega, np.array(alphas[:1])[None, :, :])[0]
    assert np.abs(single - clean).max() > 1e-3 * np.abs(clean).max()


def test_gaussian_delay_filter_and_delta_absorbance():
    n, step, width = 64, 5.0, 0.01
    const = np.full((n, 3), 2.5)
    assert np.abs(O.gaussian_filter_delay(const, step, width) - 2.5).max() < 1e-13
    k = 5                                             # a discrete-transform bin
    nu = k / (n * step)
    wave = np.cos(2 * np.pi * k * np.arange(n) / n)[:, None] * np.ones((1, 2))
    out = O.gaussian_filter_delay(wave, step, width)
    assert np.abs(out - np.exp(-nu ** 2 / (2 * width ** 2)) * wave).max() < 1e-13
    sig = np.random.default_rng(1).standard_normal((7, 4))
    d = O.delta_absorbance(sig, 2)
    assert np.all(d[2] == 0.0) and np.allclose(d[5], sig[5] - sig[2])
