"""Synthetic input generator: exact counts, symmetry, definiteness, determinism."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W


def _check(s, n_c, n_h):
    assert sum(x == "C" for x in s.species) == n_c
    assert sum(x == "H" for x in s.species) == n_h
    assert s.n_orb == 4 * n_c + n_h
    assert s.n_elec == 4 * n_c + n_h and s.n_elec % 2 == 0
    assert np.array_equal(s.S, s.S.T) and np.array_equal(s.H0, s.H0.T)
    assert np.allclose(np.diag(s.S), 1.0)
    off = s.S - np.eye(s.n_orb)
    assert np.abs(off).max() <= 0.3
    assert np.allclose(np.diag(s.gamma), W.HUBBARD_U)
    # same-atom off-diagonal blocks vanish
    for a in range(0, s.n_atoms, max(1, s.n_atoms // 50)):
        o0, o1 = s.orb_offset[a], s.orb_offset[a + 1]
        blk = s.S[o0:o1, o0:o1]
        assert np.allclose(blk, np.eye(o1 - o0))
        assert np.allclose(s.H0[o0:o1, o0:o1], np.diag(np.diag(s.H0[o0:o1, o0:o1])))


def test_flake_counts_and_spectrum():
    s = W.flake_c24h16()
    _check(s, 24, 16)
    assert np.linalg.eigvalsh(s.S)[0] > 0.05
    eps = scipy.linalg.eigh(s.H0, s.S, eigvals_only=True)
    k = s.n_occ
    assert eps[k] - eps[k - 1] > 0.01            # closed shell with a gap
    assert 0.2 * (eps[-1] - eps[0]) < 0.8         # leapfrog stable at dt = 0.2


def test_deterministic():
    a, b = W.flake_c24h16(), W.flake_c24h16()
    assert np.array_equal(a.S, b.S) and np.array_equal(a.positions, b.positions)
    c = W.flake_c24h16(seed=2001)
    assert not np.array_equal(a.positions, c.positions)


@pytest.mark.slow
def test_large_strip_counts():
    s = W.strip_c640h384()
    _check(s, 640, 384)
    assert s.n_orb == 2944
    s = W.strip_c938h344()
    _check(s, 938, 344)
    assert s.n_orb == 4096


def test_small_strip_closed_shell():
    s = W.small_strip(6, 2, seed=1)
    assert s.n_elec % 2 == 0
    assert np.linalg.eigvalsh(s.S)[0] > 0.05


def test_sin2_pulse_shape():
    t = np.linspace(0.0, 100.0, 1001)
    e = W.sin2_pulse(t, 0.005, 0.1, 100.0, (0.0, 2.0, 0.0))
    assert e.shape == (1001, 3)
    assert np.all(e[:, 0] == 0) and np.all(e[:, 2] == 0)
    assert e[0, 1] == 0 and abs(e[-1, 1]) < 1e-18
    assert np.abs(e[:, 1]).max() <= 0.005
    w = W.workload(3)
    f = w.field(10, 5)
    assert f.shape == (5, 3)
    assert np.allclose(f, W.sin2_pulse(np.arange(10, 15) * 0.2, 0.005, 0.1, 2000.0, (0, 1, 0)))


def test_spectrum_strip_counts_and_gap():
    s = W.strip_c677h236()
    assert s.n_orb == 2944 and s.species.count("C") == 677 and s.species.count("H") == 236
    assert s.n_elec % 2 == 0
