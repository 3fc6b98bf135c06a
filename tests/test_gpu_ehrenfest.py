"""Moving nuclei (Ehrenfest) on the GPU against the CPU oracle."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.ehrenfest as OE
import workloads as W

pytestmark = pytest.mark.gpu


def _T():
    from paper_1912_03174_amd import tddftb as T
    return T


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_forces(s, m, rho, field=None):
    S, H0 = OE.model_matrices(m, s.positions)
    gamma = OE.gamma_matrix(s.positions, m["hubbard_u"])
    Sinv = O.inverse_overlap(S)
    GS, GH = OE.fd_gradients(m, s.positions)
    atom_of, _ = OE.orbital_types(m)
    dq = O.charge_fluctuations(rho, S, s.orb_offset, s.q0)
    vx = np.zeros(s.n_atoms) if field is None else O.external_potential(s.positions, field)
    v_orb = (gamma @ dq + vx)[atom_of]
    H = H0 + 0.5 * S * (v_orb[:, None] + v_orb[None, :])
    return OE.forces(rho, H, Sinv, GS, GH, v_orb, dq, s.positions, m["hubbard_u"], field, m)


@pytest.mark.parametrize("which", ["benzene", "flake"])
def test_ground_state_forces_match_oracle(which):
    T = _T()
    s = W.benzene() if which == "benzene" else W.flake_c24h16()
    m = W.two_centre_model(s)
    say(f"forces {which}")
    gs = O.ground_state(s, tol=1e-13)
    e = T.Ehrenfest(s, m, rho0=gs.rho)
    F = e.forces()
    ref = oracle_forces(s, m, gs.rho)
    err = np.abs(F - ref).max() / np.abs(ref).max()
    say(f"force relative difference {err:.2e}")
    assert err < 1e-9
    pos, vel = e.nuclei()
    assert np.array_equal(pos, s.positions) and np.all(vel == 0.0)
    e.close()


def test_trajectory_matches_oracle():
    T = _T()
    s = W.benzene()
    m = W.two_centre_model(s)
    say("ehrenfest trajectory benzene")
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    vel = W.thermal_velocities(s, 1500.0, seed=9)
    n = 150
    field = W.sin2_pulse(np.arange(n) * 0.2, 0.01, 0.4, n * 0.2, (1.0, 0.5, 0.2))
    e = T.Ehrenfest(s, m, velocities=vel, rho0=gs.rho)
    e.kick(1e-3, (0.0, 1.0, 0.0))
    upd0 = e.info()["inverse_updates"]
    mu = e.step(n, field)
    # S^-1 at each new geometry: from the third-order start along the
    # trajectory one Newton-Schulz update per step reaches the rounding floor
    # (two when the start is further off; the first steps have less history)
    upd = e.info()["inverse_updates"] - upd0
    say(f"inverse updates {upd} over {n} steps")
    assert n <= upd <= 2 * n
    ee, ek = e.energy_series(n)
    pos, _ = e.nuclei()
    rho = e.rho()[0]
    rk = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (0.0, 1.0, 0.0))
    ref = OE.propagate(s, m, rk, vel, n, 0.2, field=field)
    d_err = np.abs(mu - ref.dipoles).max() / np.abs(ref.dipoles - ref.dipoles[0]).max()
    say(f"dipole relative difference {d_err:.2e}")
    assert d_err < 1e-10                 # the FP64 bar; measured 9e-14 to 9e-13
    assert np.abs(pos - ref.positions).max() < 1e-10
    assert np.abs(ek - ref.e_kin).max() < 1e-10 * ref.e_kin.max()
    assert np.abs(ee - ref.e_elec).max() < 1e-10 * np.abs(ref.e_elec).max()
    assert np.abs(rho - ref.rho).max() < 1e-10
    e.close()


def test_multi_tile_trajectory_matches_oracle():
    """A 276-orbital strip (93 atoms, every product several tiles) with
    thermal nuclei and a kick: dipoles, positions and rho against the oracle."""
    T = _T()
    s = W.small_strip(8, 4, seed=1)
    m = W.two_centre_model(s)
    say(f"ehrenfest trajectory strip n_orb={s.n_orb}")
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    vel = W.thermal_velocities(s, 600.0, seed=3)
    n = 30
    e = T.Ehrenfest(s, m, velocities=vel, rho0=gs.rho)
    e.kick(1e-3, (1.0, 0.0, 0.0))
    mu = e.step(n)
    pos, _ = e.nuclei()
    rho = e.rho()[0]
    rk = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.0, 0.0))
    ref = OE.propagate(s, m, rk, vel, n, 0.2)
    d_err = np.abs(mu - ref.dipoles).max() / np.abs(ref.dipoles - ref.dipoles[0]).max()
    say(f"dipole relative difference {d_err:.2e}")
    assert d_err < 1e-10                 # the FP64 bar; measured 9e-14 to 9e-13
    assert np.abs(pos - ref.positions).max() < 1e-10
    assert np.abs(rho - ref.rho).max() < 1e-10
    e.close()


def test_spectrum_of_rho_s_conserved_on_a_prescribed_path():
    """Straight-line nuclear paths with unequal velocities (masses 10^12
    times larger): the GPU run follows the oracle and, like it, keeps the
    spectrum of rho S (Sec. 2.1, Eq. 14: D + D^dagger = dS/dt) to the
    leapfrog's second order."""
    T = _T()
    s = W.benzene()
    m = W.two_centre_model(s)
    heavy = dict(m, mass=m["mass"] * 1e12)
    say("ehrenfest prescribed path benzene")
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    vel = np.random.default_rng(3).standard_normal((s.n_atoms, 3)) * 0.006
    n, dt = 100, 0.1
    e = T.Ehrenfest(s, heavy, velocities=vel, dt=dt, rho0=gs.rho)
    e.kick(5e-2, (1.0, 0.4, 0.0))
    e.step(n)
    pos, _ = e.nuclei()
    rho = e.rho()[0]
    rk = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 5e-2, (1.0, 0.4, 0.0))
    ref = OE.propagate(s, heavy, rk, vel, n, dt)
    assert np.abs(pos - ref.positions).max() < 1e-10
    assert np.abs(rho - ref.rho).max() < 1e-10
    S_end, _ = OE.model_matrices(m, pos)

    def spec(r, S):
        L = np.linalg.cholesky(S)
        return np.linalg.eigvalsh(L.T @ r @ L)

    dev = np.abs(spec(rho, S_end) - spec(rk, s.S)).max()
    say(f"spectrum deviation {dev:.3e}")
    assert dev < 2e-3
    e.close()


def test_energy_conserved_on_gpu():
    T = _T()
    s = W.flake_c24h16()
    m = W.two_centre_model(s)
    say("ehrenfest energy conservation flake")
    e = T.Ehrenfest(s, m, velocities=W.thermal_velocities(s, 2000.0, seed=4), scc_tol=1e-12)
    e.kick(5e-3, (1.0, 0.0, 0.0))
    n = 400
    e.step(n)
    ee, ek = e.energy_series(n)
    tot = ee + ek
    swing = np.abs(ek - ek[0]).max()
    say(f"kinetic swing {swing:.3e}, total drift {np.abs(tot - tot[0]).max():.3e}")
    # the oracle's run of the same trajectory: drift 1.4e-4 Ha against a swing of 1.5e-2
    assert swing > 1e-2 and np.abs(tot - tot[0]).max() < 2e-2 * swing
    e.close()


def test_ehrenfest_errors():
    T = _T()
    s = W.benzene()
    m = W.two_centre_model(s)
    o = T.td_default_options()
    o.precision = T.TD_SPLIT_BF16
    o.n_slices = 6
    with pytest.raises(T.TdError) as err:
        T.td_create_ehrenfest(s, m, None, o)
    assert err.value.status == T.TD_EINVAL
    bad = dict(m, species_norb=np.array([4, 4], dtype=np.int32))
    with pytest.raises(T.TdError) as err:
        T.td_create_ehrenfest(s, bad)
    assert err.value.status == T.TD_EINVAL
    p = T.Propagator(s)
    with pytest.raises(T.TdError) as err:
        T.td_get_nuclei(p.ctx, s.n_atoms)
    assert err.value.status == T.TD_ENOTSUP
    p.close()


@pytest.mark.parametrize("which,n", [("benzene", 150), ("strip276", 30)])
def test_split_products_match_oracle(which, n):
    """Split-bf16 products of rho itself for moving nuclei: the FP64 oracle's
    trajectory (kick, laser, thermal nuclei) within the split form's
    admissible 1e-6 of the dipole's change."""
    T = _T()
    s = W.benzene() if which == "benzene" else W.small_strip(8, 4, seed=1)
    m = W.two_centre_model(s)
    say(f"split ehrenfest {which} n_orb={s.n_orb}")
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    vel = W.thermal_velocities(s, 1500.0, seed=9)
    field = W.sin2_pulse(np.arange(n) * 0.2, 0.01, 0.4, n * 0.2, (1.0, 0.5, 0.2))
    e = T.Ehrenfest(s, m, velocities=vel, rho0=gs.rho, precision=T.TD_SPLIT_BF16, n_slices=4)
    e.kick(1e-3, (0.0, 1.0, 0.0))
    mu = e.step(n, field)
    pos, _ = e.nuclei()
    rk = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (0.0, 1.0, 0.0))
    ref = OE.propagate(s, m, rk, vel, n, 0.2, field=field)
    err = np.abs(mu - ref.dipoles).max() / np.abs(ref.dipoles - ref.dipoles[0]).max()
    say(f"dipole relative difference {err:.2e}")
    assert err < 1e-6
    assert np.abs(pos - ref.positions).max() < 1e-6 * np.abs(ref.positions).max()
    e.close()
