"""Pins of the Ehrenfest oracle (moving nuclei) against closed forms,
numerical derivatives and conservation laws."""
import dataclasses

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import oracle.ehrenfest as OE
import workloads as W


@pytest.fixture(scope="module")
def benzene():
    s = W.benzene()
    return s, W.two_centre_model(s)


def test_model_rebuilds_the_input_matrices(benzene):
    """The oracle's two-centre evaluation reproduces S, H0 and gamma of the input."""
    for s in (benzene[0], W.flake_c24h16()):
        m = W.two_centre_model(s)
        S, H0 = OE.model_matrices(m, s.positions)
        assert np.abs(S - s.S).max() < 1e-14 and np.abs(H0 - s.H0).max() < 1e-14
        assert np.abs(OE.gamma_matrix(s.positions, m["hubbard_u"]) - s.gamma).max() < 1e-14


def test_fd_gradient_matches_analytic_two_centre_derivatives(benzene):
    """Central differences (Eq. 20) against the analytic derivative of the
    s-s integral c f exp(-r/L) (-l / L) and of the s-p integral
    c f exp(-r/L) [(delta_kj - l_k l_j) / r - l_k l_j / L]."""
    s, m = benzene
    GS, GH = OE.fd_gradients(m, s.positions)
    off = OE.orbital_offsets(m)
    L = m["decay"]
    worst = 0.0
    for a, b in [(0, 1), (0, 3), (1, 7), (6, 2)]:          # C-C, C-C, C-H, H-C pairs
        d = s.positions[b] - s.positions[a]
        r = np.linalg.norm(d)
        l = d / r
        sa, sb = m["species"][a], m["species"][b]
        f = m["scale_s"][a, b] * np.exp(-r / L)
        c = m["sk_s"][sa, sb, 0]
        exact_ss = c * f * (-l / L)
        got = GS[:, off[a], off[b]]
        worst = max(worst, np.abs(got - exact_ss).max() / np.abs(exact_ss).max())
        if m["species_norb"][sb] == 4:
            csp = m["sk_s"][sa, sb, 1]
            for k in range(3):
                exact = csp * f * ((np.eye(3)[k] - l[k] * l) / r - l[k] * l / L)
                got = GS[:, off[a], off[b] + 1 + k]
                worst = max(worst, np.abs(got - exact).max() / np.abs(csp * f / L))
    assert worst < 1e-8


def _scc_energy(s, m, positions, field=None):
    S, H0 = OE.model_matrices(m, positions)
    gamma = OE.gamma_matrix(positions, m["hubbard_u"])
    sys2 = dataclasses.replace(s, positions=positions, S=S, H0=H0, gamma=gamma)
    gs = O.ground_state(sys2, tol=1e-13, field=field)
    e = O.energy(gs.rho, H0, gamma, gs.dq, positions, field) + OE.repulsive_energy(m, positions)
    return gs, sys2, e


def test_repulsive_force_is_minus_gradient_of_the_pair_energy(benzene):
    """The -grad E_rep term of Eq. 15: the oracle's repulsive forces against
    central differences of its pair energy, on a geometry with pairs at
    every distance class (bonded C-C and C-H, and H-H across the ring),
    and the pair energy against one pair written out."""
    s, m = benzene
    assert m["rep_a"] is not None and m["rep_a"][0, 0] > 0 and m["rep_a"][1, 1] > 0
    rng = np.random.default_rng(3)
    R = s.positions + rng.normal(scale=0.05, size=s.positions.shape)
    F = OE.repulsive_forces(m, R)
    h = 1e-4
    for a, k in [(0, 0), (3, 1), (6, 2), (11, 0)]:
        p = R.copy()
        p[a, k] += h
        ep = OE.repulsive_energy(m, p)
        p[a, k] -= 2 * h
        em = OE.repulsive_energy(m, p)
        assert abs(F[a, k] + (ep - em) / (2 * h)) < 1e-7 * np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).max()     # pair forces cancel
    two = dict(m, species=np.array([0, 1], dtype=np.int32))
    d = np.array([[0.0, 0.0, 0.0], [1.3, -0.4, 0.2]])
    r = np.linalg.norm(d[1])
    assert OE.repulsive_energy(two, d) == m["rep_a"][0, 1] * np.exp(-r / m["rep_decay"])


def test_ground_state_force_is_minus_energy_gradient(benzene):
    """At the SCC ground state the force of Eq. 15 (velocity terms aside)
    equals -dE/dR of the self-consistent energy, by central differences."""
    s, m = benzene
    gs, sys0, _ = _scc_energy(s, m, s.positions)
    S, H0 = sys0.S, sys0.H0
    Sinv = O.inverse_overlap(S)
    GS, GH = OE.fd_gradients(m, s.positions)
    atom_of, _ = OE.orbital_types(m)
    v_orb = (sys0.gamma @ gs.dq)[atom_of]
    H = H0 + 0.5 * S * (v_orb[:, None] + v_orb[None, :])
    F = OE.forces(gs.rho, H, Sinv, GS, GH, v_orb, gs.dq, s.positions, m["hubbard_u"], None, m)
    h = 1e-3
    for a, k in [(0, 0), (2, 1), (7, 0), (10, 2)]:
        p = s.positions.copy()
        p[a, k] += h
        ep = _scc_energy(s, m, p)[2]
        p[a, k] -= 2 * h
        em = _scc_energy(s, m, p)[2]
        num = -(ep - em) / (2 * h)
        assert abs(F[a, k] - num) < 1e-5 * np.abs(F).max() + 1e-9, (a, k, F[a, k], num)
    assert np.abs(F.sum(axis=0)).max() < 1e-10 * np.abs(F).max()


def test_ground_state_force_in_a_static_field(benzene):
    """In a static uniform field the SCC ground state minimises
    E = E_band + E_coul + sum_A dq_A R_A . E (Eq. 7 and the relation after
    Eq. 15), so the force of Eq. 15 with its field term -dq_A E equals -dE/dR
    by central differences. The field term is 4e-3 to 1.5e-2 here against a
    central-difference error below 1e-7: either sign of it, or leaving it out,
    fails. The forces still sum to -sum_A dq_A E = 0 for a neutral system."""
    s, m = benzene
    field = np.array([0.03, -0.02, 0.0])
    gs, sys0, _ = _scc_energy(s, m, s.positions, field)
    S, H0 = sys0.S, sys0.H0
    Sinv = O.inverse_overlap(S)
    GS, GH = OE.fd_gradients(m, s.positions)
    atom_of, _ = OE.orbital_types(m)
    v_orb = (sys0.gamma @ gs.dq + s.positions @ field)[atom_of]
    H = H0 + 0.5 * S * (v_orb[:, None] + v_orb[None, :])
    F = OE.forces(gs.rho, H, Sinv, GS, GH, v_orb, gs.dq, s.positions, m["hubbard_u"], field, m)
    h = 3e-4                  # the repulsive wall's third derivative sets the difference error
    checked = 0
    for a, k in [(0, 0), (2, 1), (7, 0), (3, 1), (9, 0)]:
        p = s.positions.copy()
        p[a, k] += h
        ep = _scc_energy(s, m, p, field)[2]
        p[a, k] -= 2 * h
        em = _scc_energy(s, m, p, field)[2]
        num = -(ep - em) / (2 * h)
        assert abs(F[a, k] - num) < 1e-6 * np.abs(F).max(), (a, k, F[a, k], num)
        checked += abs(gs.dq[a] * field[k]) > 1e-3
    assert checked >= 3                                   # the field term is visible
    assert np.abs(F.sum(axis=0)).max() < 1e-10 * np.abs(F).max()


def test_total_energy_conserved_in_a_constant_field(benzene):
    """Under a constant field the Hamiltonian does not depend on time, so
    electronic energy (with its sum_A dq_A R_A . E term) plus nuclear kinetic
    energy is conserved. Started from the SCC ground state in the field with
    thermal nuclei (2000 K), the total stays within 1.8e-6 Ha at dt = 0.2 and
    1.5e-6 at 0.1 (the velocity-dependent force terms, dropped as in the
    paper, leave this nearly dt-independent remainder) while 5e-3 Ha of
    kinetic energy swings; the field force on the charges (-dq_A E, Eq. 15)
    with the other sign lets it drift by 1.4e-3."""
    s, m = benzene
    field = np.array([0.03, 0.02, 0.0])
    gs = O.ground_state(s, tol=1e-13, field=field)
    vel = W.thermal_velocities(s, 2000.0, seed=5)
    for dt, n in ((0.2, 200), (0.1, 400)):
        tr = OE.propagate(s, m, gs.rho.astype(np.complex128), vel, n, dt,
                          field=np.tile(field, (n, 1)))
        etot = tr.e_elec + tr.e_kin
        swing = np.abs(tr.e_kin - tr.e_kin[0]).max()
        assert swing > 3e-3
        assert np.abs(etot - etot[0]).max() < 2e-5, dt


def test_total_energy_conserved(benzene):
    """Electronic plus nuclear kinetic energy is conserved (no field) to the
    integrators' second order, while energy flows between them: after a
    strong kick (0.05 au) the total moves by 2.9e-3 Ha at dt = 0.2 and
    7.3e-4 at dt = 0.1 (the electronic leapfrog's error) while 8e-3 Ha of
    kinetic energy swings."""
    s, m = benzene
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    rho = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 0.05, (1.0, 0.3, 0.0))
    vel = W.thermal_velocities(s, 2000.0, seed=5)
    err = []
    for dt, n in ((0.2, 200), (0.1, 400)):
        tr = OE.propagate(s, m, rho, vel, n, dt)
        etot = tr.e_elec + tr.e_kin
        swing = np.abs(tr.e_kin - tr.e_kin[0]).max()
        assert swing > 5e-3                               # real energy exchange
        err.append(np.abs(etot - etot[0]).max())
        assert err[-1] < 4e-3
        # Tr(rho S) with moving S: kept by the D terms up to the integrator's error
        err.append(np.abs(tr.electrons - s.n_elec).max())
        assert err[-1] < 1e-4
    assert err[0] / err[2] > 3.5 and err[1] / err[3] > 3.5   # second order in dt


def test_frozen_nuclei_limit(benzene):
    """Huge masses and no initial velocity: the trajectory is the clamped one."""
    s, m = benzene
    heavy = dict(m, mass=m["mass"] * 1e12)
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    rho = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-2, (0.0, 1.0, 0.0))
    tr = OE.propagate(s, heavy, rho, np.zeros((s.n_atoms, 3)), 200, 0.2)
    ref = O.propagate(s, rho, 200, 0.2, Sinv=Sinv, record_energy=False)
    assert np.abs(tr.dipoles - ref.dipoles).max() < 1e-9 * np.abs(ref.dipoles - ref.dipoles[0]).max()


def test_nac_sums_to_overlap_derivative(benzene):
    """D + D^T = dS/dt along any motion (the two atoms of each pair carry
    the derivative between them), and D is antisymmetric when all atoms move
    with one velocity (Sec. 2.1, remark b: unitary evolution)."""
    s, m = benzene
    GS, _ = OE.fd_gradients(m, s.positions)
    atom_of, _ = OE.orbital_types(m)
    vel = np.random.default_rng(7).standard_normal((s.n_atoms, 3)) * 0.01
    D = OE.nac(GS, vel, atom_of)
    h = 1e-4
    Sp, _ = OE.model_matrices(m, s.positions + h * vel)
    Sm, _ = OE.model_matrices(m, s.positions - h * vel)
    sdot = (Sp - Sm) / (2 * h)
    assert np.abs(D + D.T - sdot).max() < 1e-8 * np.abs(sdot).max()
    assert np.abs(np.diag(D)).max() == 0.0
    Du = OE.nac(GS, np.tile([0.02, -0.01, 0.005], (s.n_atoms, 1)), atom_of)
    assert np.abs(Du + Du.T).max() < 1e-9 * np.abs(Du).max()


def test_nac_moves_the_column_orbital(benzene):
    """D_uv = <phi_u | d/dt phi_v> (Sec. 2.1, Eq. 14): the derivative of S_uv
    when only the atom of v moves along its velocity. This fixes the index
    convention (the transpose also satisfies D + D^T = dS/dt and conserves
    the energy, so only a direct check tells them apart)."""
    s, m = benzene
    GS, _ = OE.fd_gradients(m, s.positions)
    atom_of, _ = OE.orbital_types(m)
    vel = np.random.default_rng(11).standard_normal((s.n_atoms, 3)) * 0.01
    D = OE.nac(GS, vel, atom_of)
    h = 1e-4
    worst = 0.0
    for u, v in [(0, 5), (5, 0), (3, 17), (17, 3), (1, 9), (20, 2)]:
        b = atom_of[v]
        if atom_of[u] == b:
            continue
        p = s.positions.copy()
        p[b] += h * vel[b]
        Sp, _ = OE.model_matrices(m, p)
        p[b] -= 2 * h * vel[b]
        Sm, _ = OE.model_matrices(m, p)
        fd = (Sp[u, v] - Sm[u, v]) / (2 * h)
        worst = max(worst, abs(D[u, v] - fd) / np.abs(D).max())
        assert abs(D[v, u] - D[u, v]) > 1e-6 * np.abs(D).max()   # the pair is not symmetric
    assert worst < 1e-8


def _rho_s_spectrum(rho, S):
    L = np.linalg.cholesky(S)
    return np.linalg.eigvalsh(L.T @ rho @ L)


def test_spectrum_of_rho_s_conserved_along_any_path(benzene):
    """With D + D^dagger = dS/dt the exact motion is d(rho S)/dt = [G, rho S]
    for G = -S^-1 (iH + D): the spectrum of rho S is conserved along any
    nuclear path (uniform translation, the case of Sec. 2.1 remark b,
    included). Leapfrog keeps it to second order in dt. The nuclei follow
    straight lines with unequal velocities (masses 10^12 times larger);
    dropping D (planted in the oracle) leaves an error that does not fall
    with dt."""
    s, m = benzene
    heavy = dict(m, mass=m["mass"] * 1e12)
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    rho = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 5e-2, (1.0, 0.4, 0.0))
    lam0 = _rho_s_spectrum(rho, s.S)
    vel = np.random.default_rng(3).standard_normal((s.n_atoms, 3)) * 0.006

    def deviation(dt):
        n = int(round(10.0 / dt))
        tr = OE.propagate(s, heavy, rho, vel, n, dt)
        S_end, _ = OE.model_matrices(m, tr.positions)
        assert np.abs(tr.positions - s.positions).max() > 0.1   # the atoms moved
        return np.abs(_rho_s_spectrum(tr.rho, S_end) - lam0).max()

    dev = [deviation(dt) for dt in (0.2, 0.1, 0.05)]
    assert dev[0] / dev[1] > 3.0 and dev[1] / dev[2] > 3.0
    assert dev[2] < 5e-4
    good = OE.nac
    try:
        OE.nac = lambda GS, v, a: 0.0 * good(GS, v, a)
        dropped = [deviation(dt) for dt in (0.1, 0.05)]
    finally:
        OE.nac = good
    assert dropped[1] > 0.5 * dropped[0] and dropped[1] > 20 * dev[2]
