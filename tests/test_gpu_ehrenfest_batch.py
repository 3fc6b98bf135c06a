"""Batches of moving-nuclei trajectories of one system (td_batch_create_ehrenfest)
against solo contexts and the CPU oracle.

Every member runs the arithmetic of its solo context (the products as
grouped launches over all members give each element the same MFMA sequence
over k; the Newton-Schulz decisions are those of one trajectory), so each
member must equal its solo trajectory bit for bit; one member is also held
to the oracle (Sec. 2.1, Eqs. 10, 14, 15; Sec. 2.3)."""
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


@pytest.mark.parametrize("which", ["benzene", "strip276"])
def test_members_equal_solo_runs(which):
    T = _T()
    s = W.benzene() if which == "benzene" else W.small_strip(8, 4, seed=1)
    m = W.two_centre_model(s)
    nm, n = 3, 24
    say(f"ehrenfest batch {which} n_orb={s.n_orb}, {nm} members, {n} steps")
    gs = O.ground_state(s, tol=1e-13)
    vel = np.array([W.thermal_velocities(s, 600.0 + 300.0 * j, seed=20 + j) for j in range(nm)])
    field = W.sin2_pulse(np.arange(2 * n) * 0.2, 0.01, 0.3, 2 * n * 0.2, (1.0, 0.4, 0.0))
    e0 = np.array([1e-3, 0.0, 2e-3])
    axes = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.3, 1.0, 0.0]])
    b = T.EhrenfestBatch(s, m, nm, velocities=vel, rho0=gs.rho)
    b.kick(e0, axes)
    b.step(n, field[:n])
    b.step(n, field[n:])
    for j in range(nm):
        e = T.Ehrenfest(s, m, velocities=vel[j], rho0=gs.rho)
        if e0[j] != 0.0:
            e.kick(e0[j], axes[j])
        else:
            e.kick(0.0, axes[j])
        e.step(n, field[:n])
        mu = e.step(n, field[n:])
        assert np.array_equal(b.dipoles(j, n), mu), j
        pos_b, vel_b = b.nuclei(j)
        pos_s, vel_s = e.nuclei()
        assert np.array_equal(pos_b, pos_s) and np.array_equal(vel_b, vel_s), j
        ee_b, ek_b = b.energy_series(j, n)
        ee_s, ek_s = e.energy_series(n)
        assert np.array_equal(ee_b, ee_s) and np.array_equal(ek_b, ek_s), j
        assert np.array_equal(b.rho(j)[0], e.rho()[0]), j
        assert np.array_equal(b.charges(j), e.charges()), j
        e.close()
    info = b.info()
    assert info["n_members"] == nm and info["step"] == 2 * n
    b.close()


def test_member_matches_oracle():
    """A kicked member under a laser against the oracle's trajectory."""
    T = _T()
    s = W.benzene()
    m = W.two_centre_model(s)
    say("ehrenfest batch member against the oracle")
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    vel = np.array([W.thermal_velocities(s, 1500.0, seed=9), W.thermal_velocities(s, 900.0, seed=4)])
    n = 60
    field = W.sin2_pulse(np.arange(n) * 0.2, 0.01, 0.4, n * 0.2, (1.0, 0.5, 0.2))
    b = T.EhrenfestBatch(s, m, 2, velocities=vel, rho0=gs.rho)
    b.kick(np.array([1e-3, 1e-3]), np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0]]))
    b.step(n, field)
    mu = b.dipoles(0, n)
    pos, _ = b.nuclei(0)
    rk = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (0.0, 1.0, 0.0))
    ref = OE.propagate(s, m, rk, vel[0], n, 0.2, field=field)
    err = np.abs(mu - ref.dipoles).max() / np.abs(ref.dipoles - ref.dipoles[0]).max()
    say(f"dipole relative difference {err:.2e}")
    assert err < 1e-10
    assert np.abs(pos - ref.positions).max() < 1e-10
    assert np.abs(b.rho(0)[0] - ref.rho).max() < 1e-10
    b.close()


def test_batch_errors():
    T = _T()
    s = W.benzene()
    m = W.two_centre_model(s)
    say("ehrenfest batch errors")
    o = T.td_default_options()
    o.precision = T.TD_SPLIT_BF16
    o.n_slices = 6
    with pytest.raises(T.TdError) as e:
        T.td_batch_create_ehrenfest(s, m, 2, options=o)
    assert e.value.status == T.TD_EINVAL and "member 0" in str(e.value)
    b = T.Batch([s])
    with pytest.raises(T.TdError) as e:
        T.td_batch_get_nuclei(b.b, 0, s.n_atoms)
    assert e.value.status == T.TD_ENOTSUP
    b.close()
    # the leapfrog limit is checked for every member before any step
    eb = T.EhrenfestBatch(s, m, 2, dt=2.0)
    with pytest.raises(T.TdError) as e:
        eb.step(1)
    assert e.value.status == T.TD_EUNSTABLE and "member 0" in str(e.value)
    eb.close()


def test_split_members_equal_solo_runs():
    """Split-bf16 moving-nuclei batch: each member's products with rho run
    as in its solo context, so members equal solo runs bit for bit."""
    T = _T()
    s = W.benzene()
    m = W.two_centre_model(s)
    say("split ehrenfest batch benzene")
    gs = O.ground_state(s, tol=1e-13)
    vel = np.array([W.thermal_velocities(s, 800.0 + 400.0 * j, seed=30 + j) for j in range(2)])
    n = 20
    b = T.EhrenfestBatch(s, m, 2, velocities=vel, rho0=gs.rho, precision=T.TD_SPLIT_BF16)
    b.kick(np.array([1e-3, 2e-3]), np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]))
    b.step(n)
    for j in range(2):
        e = T.Ehrenfest(s, m, velocities=vel[j], rho0=gs.rho, precision=T.TD_SPLIT_BF16)
        e.kick([1e-3, 2e-3][j], [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]][j])
        mu = e.step(n)
        assert np.array_equal(b.dipoles(j, n), mu), j
        assert np.array_equal(b.nuclei(j)[0], e.nuclei()[0]), j
        e.close()
    b.close()
