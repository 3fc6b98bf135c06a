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
