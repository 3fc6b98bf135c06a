"""Pins of the on-site correction oracle (DFTB+U FLL and pseudo-SIC,
Sec. 3.2, Eqs. 21-25), checked against what the mathematics fixes:

* U = 0 is the plain SCC model;
* the block potential is the derivative of the correction energy, and the
  whole Hamiltonian is the derivative of the total energy with respect to
  rho (pins the dual assembly 1/2 (S V + V S) and its factors);
* closed form on non-interacting shells with S = 1: FLL shifts the occupied
  orbitals of a corrected shell by -U/2 and the empty ones by +U/2, pSIC
  shifts only the occupied ones, by -U (the actions the paper's text
  describes);
* the corrected ground state is stationary and idempotent;
* with no field the total energy is a constant of the motion: its leapfrog
  oscillation is second order in dt with no drift.
"""
import numpy as np
import pytest

import oracle as O
import oracle.plus_u as U
import workloads as W


@pytest.fixture(scope="module")
def flake():
    return W.flake_c24h16()


def _pu(system, mode, up=0.15, us=0.0):
    off, u = W.atomic_shells(system, {("C", "p"): up, ("C", "s"): us, ("H", "s"): us})
    return U.PlusU(mode=mode, shell_offset=off, shell_u=u)


def test_zero_u_is_the_scc_model(flake):
    s = flake
    pu = _pu(s, U.FLL, up=0.0)
    rng = np.random.default_rng(1)
    gs = O.ground_state(s, tol=1e-13)
    r, i = W.random_hermitian_pair(s.n_orb, seed=3, scale=1e-2, base=gs.rho)
    rho = r + 1j * i
    H, dq, e_u = U.hamiltonian(s, rho, pu)
    ref = O.scc_hamiltonian_fast(s.H0, s.S, s.gamma, dq, s.orb_offset)
    assert np.array_equal(H, ref) and e_u == 0.0
    assert U.energy(s, rho, pu) == O.energy(rho, s.H0, s.gamma, dq, s.positions)
    g0 = U.ground_state(s, pu, tol=1e-12)
    assert np.abs(g0.rho - gs.rho).max() < 1e-10
    del rng


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_block_potential_is_the_energy_derivative(mode):
    rng = np.random.default_rng(7)
    blocks = []
    for m in (1, 3, 3, 1, 5):
        a = rng.standard_normal((m, m))
        blocks.append(a + a.T + np.eye(m))
    us = rng.uniform(0.05, 0.4, size=len(blocks))
    V = U.plus_u_potential(blocks, us, mode)
    eps = 1e-5
    for b in range(len(blocks)):
        d = rng.standard_normal(blocks[b].shape)
        d = d + d.T
        up = [x.copy() for x in blocks]
        dn = [x.copy() for x in blocks]
        up[b] += eps * d
        dn[b] -= eps * d
        fd = (U.plus_u_energy(up, us, mode) - U.plus_u_energy(dn, us, mode)) / (2 * eps)
        assert abs(fd - float((V[b] * d).sum())) < 1e-9 * max(1.0, abs(fd))


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_hamiltonian_is_the_total_energy_derivative(flake, mode):
    s = flake
    pu = _pu(s, mode, up=0.3, us=0.1)
    gs = O.ground_state(s, tol=1e-12)
    r, i = W.random_hermitian_pair(s.n_orb, seed=5, scale=2e-2, base=gs.rho)
    rho = r + 1j * i
    H, _, _ = U.hamiltonian(s, rho, pu)
    dr, di = W.random_hermitian_pair(s.n_orb, seed=6, scale=1.0)
    d = dr + 1j * di
    eps = 1e-5
    fd = (U.energy(s, rho + eps * d, pu) - U.energy(s, rho - eps * d, pu)) / (2 * eps)
    an = float(np.real(np.trace(H @ d)))
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an))
    # a wrong factor in the dual assembly (half the correction term) fails this check
    half = 0.5 * U.plus_u_hamiltonian(s.S, U.plus_u_potential(
        U.block_populations(rho, s.S, pu.shell_offset), pu.shell_u, mode), pu.shell_offset)
    assert abs(fd - float(np.real(np.trace((H - half) @ d)))) > 1e-5


def _isolated_shells():
    """Two far-apart atoms with S = 1, gamma = 0 and diagonal H0: atom A
    with an s and a p shell, atom B with an s shell; six electrons fill A s,
    the lowest A p orbital and B s."""
    h = np.array([-0.9, -0.6, -0.3, -0.1, -0.5])
    sysm = W.System(species=["C", "H"], positions=np.array([[0.0, 0, 0], [50.0, 0, 0]]),
                    orb_offset=np.array([0, 4, 5], dtype=np.int32), S=np.eye(5),
                    H0=np.diag(h), gamma=np.zeros((2, 2)), q0=np.array([4.0, 2.0]), n_elec=6)
    return sysm, h


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_scissor_closed_form(mode):
    s, h = _isolated_shells()
    u = 0.2
    pu = U.PlusU(mode=mode, shell_offset=np.array([0, 1, 4, 5], dtype=np.int32),
                 shell_u=np.array([0.0, u, 0.0]))
    g = U.ground_state(s, pu, tol=1e-13)
    occupied_p, empty_p = -0.6, (-0.3, -0.1)
    if mode == U.FLL:
        expect = {-0.9: -0.9, -0.5: -0.5, occupied_p: occupied_p - u / 2,
                  empty_p[0]: empty_p[0] + u / 2, empty_p[1]: empty_p[1] + u / 2}
    else:
        expect = {-0.9: -0.9, -0.5: -0.5, occupied_p: occupied_p - u,
                  empty_p[0]: empty_p[0], empty_p[1]: empty_p[1]}
    assert np.allclose(np.sort(g.eps), np.sort(list(expect.values())), atol=1e-12)
    n_p = U.block_populations(g.rho, s.S, pu.shell_offset)[1]
    assert np.allclose(n_p, np.diag([2.0, 0.0, 0.0]), atol=1e-12)


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_corrected_ground_state_is_stationary(flake, mode):
    s = flake
    pu = _pu(s, mode)
    g = U.ground_state(s, pu, tol=1e-12)
    H, _, _ = U.hamiltonian(s, g.rho, pu)
    Sinv = O.inverse_overlap(s.S)
    assert O.stationarity_residual(g.rho, H, Sinv) < 1e-9
    assert np.abs(g.rho @ s.S @ g.rho - 2.0 * g.rho).max() < 1e-10
    assert abs(O.electron_count(g.rho, s.S) - s.n_elec) < 1e-10
    # the correction changes the state
    g0 = O.ground_state(s, tol=1e-12)
    assert np.abs(g.rho - g0.rho).max() > 1e-4


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_energy_is_conserved_to_second_order(flake, mode):
    """Free propagation after a kick: the spread of E over 40 au falls 4x when
    dt halves (leapfrog error), which fails if H were not dE/drho (the
    energy would then drift independently of dt)."""
    s = flake
    pu = _pu(s, mode)
    g = U.ground_state(s, pu, tol=1e-12)
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(g.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-2, (1.0, 0.0, 0.0))
    spreads = []
    for dt in (0.2, 0.1):
        _, _, _, es = U.propagate(s, pu, rk, int(round(40 / dt)), dt, Sinv=Sinv)
        spreads.append(es.max() - es.min())
    assert 3.0 < spreads[0] / spreads[1] < 5.0
