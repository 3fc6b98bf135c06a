"""Batches of probe trajectories (through the C ABI).

Each member of a batch must follow the trajectory of a solo context on the
same system bit for bit (same kernels' arithmetic in the same order), for
every product tile choice, with and without graph replay; a pump-excited
batch is checked against the CPU oracle.
"""
import sys

import numpy as np
import pytest
import scipy.linalg

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
def members():
    # sizes across the 128- and 64-tile buckets, plus the smallest and largest
    systems, axes = W.probe_batch(10, seed=4100)
    systems.append(W.probe_molecule(60, 4200))
    systems.append(W.probe_molecule(800, 4201))
    axes = np.vstack([axes, [[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]]])
    return systems, axes


def solo_run(T, s, axis, n, field=None, scc_tol=1e-12):
    p = T.Propagator(s, scc_tol=scc_tol)
    p.kick(1e-3, axis)
    mu = p.step(n, field)
    rho = p.rho()[0]
    p.close()
    return mu, rho


@pytest.mark.parametrize("flags", ["default", "tile128_nograph", "tile64"])
def test_batch_members_equal_solo_runs(members, flags):
    T = _T()
    systems, axes = members
    f = {"default": 0, "tile128_nograph": T.TD_BATCH_TILE_128 | T.TD_BATCH_NO_GRAPH,
         "tile64": T.TD_BATCH_TILE_64}[flags]
    say(f"batch of {len(systems)} ({flags}), sizes {[s.n_orb for s in systems]}")
    b = T.Batch(systems, flags=f)
    info = b.info()
    say(f"tiles per bucket {info['bucket_tile']} ms {info['bucket_ms']}")
    b.kick(np.full(len(systems), 1e-3), axes)
    n = 40
    b.step(n)
    for m, s in enumerate(systems):
        mu, rho = solo_run(T, s, axes[m], n)
        assert np.array_equal(b.dipoles(m, n), mu), f"member {m}"
        assert np.array_equal(b.rho(m)[0], rho), f"member {m}"
    b.close()


def test_batch_field_split_calls_and_state(members):
    T = _T()
    systems, axes = members
    systems, axes = systems[:4], axes[:4]
    say("batch with a field over two calls")
    n = 30
    field = W.sin2_pulse(np.arange(2 * n) * 0.2, 0.01, 0.15, 2 * n * 0.2, (1.0, 1.0, 0.0))
    b = T.Batch(systems)
    b.kick(np.array([1e-3, 0.0, 2e-3, 1e-3]), axes)
    b.step(n, field[:n])
    first = [b.dipoles(m, n) for m in range(4)]
    b.step(n, field[n:])
    info = b.info()
    assert info["step"] == 2 * n and info["has_prev"]
    for m, s in enumerate(systems):
        p = T.Propagator(s)
        p.kick([1e-3, 0.0, 2e-3, 1e-3][m], axes[m])
        mu = p.step(2 * n, field)
        assert np.array_equal(np.vstack([first[m], b.dipoles(m, n)]), mu)
        assert np.array_equal(b.charges(m), p.charges())
        rho, prev, step, has_prev = b.rho(m, with_prev=True)
        rs, ps, steps, _ = p.rho(with_prev=True)
        assert np.array_equal(rho, rs) and np.array_equal(prev, ps) and step == steps
        p.close()
    b.close()


def pump_excited(s, amount=0.1):
    """Ground state with `amount` electrons moved from HOMO to LUMO (oracle)."""
    gs = O.ground_state(s, tol=1e-13)
    H = O.scc_hamiltonian_fast(s.H0, s.S, s.gamma, gs.dq, s.orb_offset)
    _, C = scipy.linalg.eigh(H, s.S)
    h = s.n_elec // 2 - 1
    cH, cL = C[:, h], C[:, h + 1]
    return gs.rho + amount * (np.outer(cL, cL) - np.outer(cH, cH))


@pytest.mark.parametrize("n_lo,n_hi,seed,n", [(60, 200, 4300, 200), (600, 808, 4301, 40)])
def test_pump_excited_batch_matches_oracle(n_lo, n_hi, seed, n):
    """Members drawn from the small and from the large end of the probe
    sizes (several 64- and 128-wide product tiles each), each against the
    oracle directly."""
    T = _T()
    systems, axes = W.probe_batch(3, seed=seed, n_lo=n_lo, n_hi=n_hi)
    say(f"pump-excited batch vs oracle, sizes {[s.n_orb for s in systems]}")
    rho0 = [pump_excited(s) for s in systems]
    b = T.Batch(systems, rho0s=rho0)
    b.kick(np.full(3, 1e-3), axes)
    b.step(n)
    for m, s in enumerate(systems):
        Sinv = O.inverse_overlap(s.S)
        rk = O.kick(rho0[m], s.S, Sinv, s.positions, s.orb_offset, 1e-3, axes[m])
        ref = O.propagate(s, rk, n, 0.2, Sinv=Sinv, record_energy=False)
        mu = b.dipoles(m, n)
        err = np.abs(mu - ref.dipoles).max() / np.abs(ref.dipoles - ref.dipoles[0]).max()
        say(f"member {m} N={s.n_orb} dipole relative error {err:.2e}")
        assert err < 1e-10
    b.close()


def test_batch_errors(members):
    T = _T()
    systems, _ = members
    o = T.td_default_options()
    o.precision = T.TD_SPLIT_BF16
    with pytest.raises(T.TdError) as e:
        T.td_batch_create(systems[:2], o)
    assert e.value.status == T.TD_ENOTSUP
    bad = [systems[0], W.dimer()]
    bad[1].n_elec = 3
    with pytest.raises(T.TdError) as e:
        T.td_batch_create(bad)
    assert e.value.status == T.TD_EINVAL and "member 1" in str(e.value)
    b = T.Batch(systems[:2])
    with pytest.raises(T.TdError) as e:
        T.td_batch_get_charges(b.b, 5, 10)
    assert e.value.status == T.TD_EINVAL
    b.close()
