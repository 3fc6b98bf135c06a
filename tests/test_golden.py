"""Regression of the oracle against its stored flake trajectory."""
import os

import numpy as np

from tests.golden.make_golden import compute

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_reproduces_stored_flake_dipole():
    data = np.loadtxt(os.path.join(HERE, "golden", "flake112_dipole.txt"))
    steps, mu = compute()
    assert np.array_equal(steps, data[:, 0].astype(int))
    scale = np.abs(mu - mu[0]).max()
    assert np.abs(mu - data[:, 1:]).max() < 1e-10 * scale


def test_oracle_reproduces_stored_strip4096_start():
    """The first two dipoles (the start and one leapfrog step) of the stored
    500-step N_orb = 4096 run (the GPU parity fixture) from the oracle as it
    stands."""
    from tests.golden import make_strip4096 as M
    data = np.loadtxt(M.DIPOLE)
    mu, _ = M.compute(steps=2)
    scale = np.abs(data[:, 1:] - data[0, 1:]).max()
    assert np.abs(mu - data[:2, 1:]).max() < 1e-12 * scale
