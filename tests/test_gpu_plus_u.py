"""On-site corrections (DFTB+U FLL and pseudo-SIC, Sec. 3.2) on the GPU,
through the C ABI, against the CPU oracle (``oracle.plus_u``).

Tolerances as for the SCC path: charges and densities to 1e-9 / 1e-12,
dipole relative error 1e-10 over the run, energies to 1e-10 (FP64);
split-bf16 products: dipole relative error 1e-6.
"""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.plus_u as U
import workloads as W

pytestmark = pytest.mark.gpu


def _T():
    from paper_1912_03174_amd import tddftb as T
    return T


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def flake():
    return W.flake_c24h16()


def _pu(system, mode, up=0.15, us=0.05):
    off, u = W.atomic_shells(system, {("C", "p"): up, ("C", "s"): us})
    return U.PlusU(mode=mode, shell_offset=off, shell_u=u)


@pytest.fixture(scope="module")
def ground(flake):
    out = {}
    for mode in (U.FLL, U.PSIC):
        pu = _pu(flake, mode)
        out[mode] = (pu, U.ground_state(flake, pu, tol=1e-13))
    return out


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_ground_state_matches_oracle(flake, ground, mode):
    T = _T()
    s = flake
    pu, g = ground[mode]
    say(f"plus_u ground state {mode}")
    p = T.Propagator(s, plus_u=pu, scc_tol=1e-12)
    info = p.info()
    say(f"scc iterations {info['scc_iterations']} residual {info['scc_residual']:.2e}")
    assert np.abs(p.charges() - g.dq).max() < 1e-9
    assert np.abs(p.rho()[0] - g.rho).max() < 1e-9
    assert abs(p.energy() - U.energy(s, g.rho, pu)) < 1e-9
    p.close()


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_kicked_run_matches_oracle(flake, ground, mode):
    T = _T()
    s = flake
    pu, g = ground[mode]
    say(f"plus_u kicked run {mode}")
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(g.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.5, 0.0))
    rho, _, mus, es = U.propagate(s, pu, rk, 300, 0.2, Sinv=Sinv)
    p = T.Propagator(s, rho0=g.rho, plus_u=pu)
    p.kick(1e-3, (1.0, 0.5, 0.0))
    mu = p.step(300)
    err = np.abs(mu - mus).max() / np.abs(mus - mus[0]).max()
    say(f"dipole relative error {err:.3e}")
    assert err < 1e-10
    assert np.abs(p.rho()[0] - rho).max() < 1e-12
    assert abs(p.energy() - U.energy(s, rho, pu)) < 1e-10
    p.close()


def test_laser_run_matches_oracle(flake, ground):
    T = _T()
    s = flake
    pu, g = ground[U.FLL]
    say("plus_u laser run")
    n = 200
    t = np.arange(n) * 0.2
    field = W.sin2_pulse(t, 0.01, 0.3, n * 0.2, (0.0, 1.0, 0.0))
    _, _, mus, _ = U.propagate(s, pu, g.rho, n, 0.2, field=field)
    p = T.Propagator(s, rho0=g.rho, plus_u=pu)
    mu = p.step(n, field)
    err = np.abs(mu - mus).max() / np.abs(mus - mus[0]).max()
    say(f"dipole relative error {err:.3e}")
    assert err < 1e-10
    p.close()


@pytest.mark.parametrize("mode", [U.FLL, U.PSIC])
def test_split_bf16_kicked_run(flake, ground, mode):
    """Split-bf16 products with the correction in the change of H from the
    reference: within the split path's 1e-6 dipole bound of the FP64 oracle."""
    T = _T()
    s = flake
    pu, g = ground[mode]
    say(f"plus_u split run {mode}")
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(g.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.0, 0.0))
    rho, _, mus, _ = U.propagate(s, pu, rk, 500, 0.2, Sinv=Sinv)
    p = T.Propagator(s, rho0=g.rho, plus_u=pu, precision=T.TD_SPLIT_BF16, n_slices=4)
    p.kick(1e-3, (1.0, 0.0, 0.0))
    mu = p.step(500)
    err = np.abs(mu - mus).max() / np.abs(mus - mus[0]).max()
    say(f"split dipole relative error {err:.3e}")
    assert err < 1e-6
    assert abs(p.energy() - U.energy(s, rho, pu)) < 1e-6 * abs(U.energy(s, rho, pu))
    # and the split ground state stays put
    q = T.Propagator(s, rho0=g.rho, plus_u=pu, precision=T.TD_SPLIT_BF16, n_slices=4)
    m0 = q.step(100)
    assert np.abs(m0 - m0[0]).max() < 1e-10 * max(1.0, np.abs(m0[0]).max())
    p.close()
    q.close()


def test_zero_u_is_bitwise_the_plain_path(flake, ground):
    T = _T()
    s = flake
    say("plus_u with U = 0")
    _, g = ground[U.FLL]
    pu0 = _pu(s, U.FLL, up=0.0, us=0.0)
    a = T.Propagator(s, rho0=g.rho)
    b = T.Propagator(s, rho0=g.rho, plus_u=pu0)
    for p in (a, b):
        p.kick(1e-3, (0.0, 1.0, 0.0))
    ma, mb = a.step(100), b.step(100)
    assert np.array_equal(ma, mb)
    assert np.array_equal(a.rho()[0], b.rho()[0])
    a.close()
    b.close()


@pytest.fixture(scope="module")
def strip648_fll():
    """A 648-orbital strip with FLL corrections on 358 shells (many tiles of
    every product), its corrected ground state and a 20-step kicked oracle run."""
    s = W.small_strip(20, 10, seed=1)
    pu = _pu(s, U.FLL)
    g = U.ground_state(s, pu, tol=1e-12)
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(g.rho, s.S, Sinv, s.positions, s.orb_offset, 1e-3, (1.0, 0.0, 0.0))
    rho, _, mus, _ = U.propagate(s, pu, rk, 20, 0.2, Sinv=Sinv)
    return s, pu, g, rho, mus


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_multi_tile_corrected_run(strip648_fll, precision):
    T = _T()
    s, pu, g, rho, mus = strip648_fll
    say(f"plus_u strip648 {precision}")
    prec = T.TD_FP64 if precision == "fp64" else T.TD_SPLIT_BF16
    p = T.Propagator(s, rho0=g.rho, plus_u=pu, precision=prec, n_slices=4)
    p.kick(1e-3, (1.0, 0.0, 0.0))
    mu = p.step(20)
    err = np.abs(mu - mus).max() / np.abs(mus - mus[0]).max()
    say(f"dipole relative error {err:.3e}")
    if precision == "fp64":
        assert err < 1e-10
        assert np.abs(p.rho()[0] - rho).max() < 1e-12
    else:
        assert err < 1e-6
    p.close()
