"""Degenerate cases of the step on the GPU (through the C ABI).

* an empty step call is a no-op (solo and batch) and records no dipoles;
* the SCC ground state with no kick and no field is stationary (the exact
  motion leaves it unchanged, Sec. 2.1): ρ and the dipole stay put to the
  level of the SCC residual, in FP64 and in split-bf16 (where the state is
  the zero departure from the reference);
* a kick of strength zero (Sec. 2.2, Eq. 16 with E0 = 0) leaves ρ unchanged
  and restarts the integrator;
* an orthogonal basis, S = 1, where Eq. 10 reduces to the textbook
  -i[H, ρ]: the GPU run follows the oracle.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle as O
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
    s = W.flake_c24h16()
    gs = O.ground_state(s, tol=1e-13)
    return s, gs


def test_step_zero_is_a_no_op(flake):
    T = _T()
    s, gs = flake
    say("step(0)")
    p = T.Propagator(s, rho0=gs.rho)
    p.kick(1e-3, (0.0, 1.0, 0.0))
    p.step(7)
    before, prev_before, step_before, _ = T.td_get_rho(p.ctx, s.n_orb, with_prev=True)
    T.td_step(p.ctx, 0)
    # the series of the last call is empty, whatever the capacity asked for
    assert len(T.td_get_dipole_series(p.ctx, 10)) == 0
    after, prev_after, step_after, has_prev = T.td_get_rho(p.ctx, s.n_orb, with_prev=True)
    assert has_prev and step_after == step_before == 7
    assert np.array_equal(after, before) and np.array_equal(prev_after, prev_before)
    p.close()


def test_batch_step_zero_is_a_no_op(flake):
    T = _T()
    s, gs = flake
    say("batch step(0)")
    b = T.Batch([s, s], rho0s=[gs.rho, gs.rho])
    b.kick(np.array([1e-3, 2e-3]), np.array([(1.0, 0.0, 0.0), (0.0, 0.0, 1.0)]))
    b.step(5)
    before = [b.rho(m, with_prev=True) for m in range(2)]
    b.step(0)
    for m in range(2):
        assert len(T.td_batch_get_dipole_series(b.b, m, 10)) == 0
        after = b.rho(m, with_prev=True)
        assert np.array_equal(after[0], before[m][0]) and np.array_equal(after[1], before[m][1])
        assert after[2] == before[m][2] == 5
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_ground_state_is_stationary(flake, precision):
    T = _T()
    s, gs = flake
    say(f"stationary ground state, {precision}")
    prec = T.TD_FP64 if precision == "fp64" else T.TD_SPLIT_BF16
    p = T.Propagator(s, rho0=gs.rho, precision=prec, n_slices=4)
    mu = p.step(300)
    rho = p.rho()[0]
    # the oracle's ground state is converged to 1e-13 in the charges
    assert np.abs(rho - gs.rho).max() < 1e-10
    assert np.abs(mu - mu[0]).max() < 1e-10 * max(1.0, np.abs(mu[0]).max())
    assert np.abs(p.charges() - gs.dq).max() < 1e-10
    p.close()


def test_zero_kick_leaves_rho_and_restarts(flake):
    T = _T()
    s, gs = flake
    say("zero kick")
    p = T.Propagator(s, rho0=gs.rho)
    p.step(3)
    p.kick(0.0, (1.0, 0.0, 0.0))
    rho = p.rho()[0]
    assert np.abs(rho - gs.rho).max() < 1e-12
    # history cleared: asking for the previous density is a state error
    with pytest.raises(T.TdError) as e:
        p.rho(with_prev=True)
    assert e.value.status == T.TD_ESTATE
    mu = p.step(100)
    assert np.abs(mu - mu[0]).max() < 1e-10 * max(1.0, np.abs(mu[0]).max())
    p.close()


def test_orthogonal_basis_follows_oracle(flake):
    T = _T()
    s, _ = flake
    so = dataclasses.replace(s, S=np.eye(s.n_orb))
    say("orthogonal basis")
    gs = O.ground_state(so, tol=1e-13)
    Sinv = np.eye(s.n_orb)
    rk = O.kick(gs.rho, so.S, Sinv, so.positions, so.orb_offset, 1e-3, (1.0, 1.0, 0.0))
    ref = O.propagate(so, rk, 300, 0.2, Sinv=Sinv, record_energy=False)
    p = T.Propagator(so, rho0=gs.rho)
    p.kick(1e-3, (1.0, 1.0, 0.0))
    mu = p.step(300)
    scale = np.abs(ref.dipoles - ref.dipoles[0]).max()
    err = np.abs(mu - ref.dipoles).max() / scale
    say(f"orthogonal basis dipole relative error {err:.3e}")
    assert err < 1e-10
    assert np.abs(p.rho()[0] - ref.rho).max() < 1e-12
    # with S = 1 the GPU ground state is the same fixed point
    q = T.Propagator(so, scc_tol=1e-12)
    assert np.abs(q.charges() - gs.dq).max() < 1e-9
    p.close()
    q.close()
