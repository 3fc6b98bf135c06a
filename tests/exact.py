"""Closed forms that pin the oracle (test helpers; independent of oracle/).

All of these follow from the clamped-nuclei equation of motion
rhodot = -i (S^-1 H rho - rho H S^-1) (Sec. 2.1, Eq. 10 with D = 0) for a
fixed Hamiltonian (no SCC term, no field), by moving to the generalized
eigenbasis H C = S C eps, C^T S C = 1, where rho = C rt C^T and each element
obeys d rt_ij / dt = -i (eps_i - eps_j) rt_ij.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def eigenbasis(H, S):
    eps, C = scipy.linalg.eigh(H, S)
    return eps, C


def to_eigen(rho, S, C):
    return C.T @ S @ rho @ S @ C


def from_eigen(rt, C):
    return C @ rt @ C.T


def exact_continuous(rho0, H, S, t):
    """rho(t) = C exp(-i eps t) rt(0) exp(+i eps t) C^T."""
    eps, C = eigenbasis(H, S)
    rt = to_eigen(rho0, S, C)
    ph = np.exp(-1j * eps * t)
    return from_eigen(ph[:, None] * rt * ph.conj()[None, :], C)


def exact_leapfrog(rho0, H, S, dt, n):
    """Closed form of n steps of Euler-started leapfrog, element by element.

    y_{k+1} = y_{k-1} - 2 i th y_k, y_1 = (1 - i th) y_0, th = (eps_i - eps_j) dt,
    gives y_n = a l+^n + b l-^n with l+- = -i th +- sqrt(1 - th^2),
    a = y_0 (1 + c) / (2 c), b = y_0 - a, c = sqrt(1 - th^2)  (needs |th| < 1).
    """
    eps, C = eigenbasis(H, S)
    y0 = to_eigen(rho0, S, C)
    th = (eps[:, None] - eps[None, :]) * dt
    c = np.sqrt(1.0 - th ** 2 + 0j)
    lp = -1j * th + c
    lm = -1j * th - c
    a = y0 * (1.0 + c) / (2.0 * c)
    b = y0 - a
    yn = a * lp ** n + b * lm ** n
    return from_eigen(yn, C)


def linear_response_dipole(H, S, positions, orb_offset, n_occ, kick_dir, meas_dir, kappa, t):
    """First-order dipole change after a kick kappa along ``kick_dir``.

    d mu_m(t) = (kappa/2) sum_{eps_i > eps_j} (f_j - f_i) Mk_ij Mm_ij sin((eps_i - eps_j) t),
    M = C^T (S X + X S) C with X = diag(e . R_A(u)), f = 2 for the n_occ lowest states.
    """
    eps, C = eigenbasis(H, S)
    counts = np.diff(np.asarray(orb_offset))
    atom = np.repeat(np.arange(len(counts)), counts)

    def M(e):
        e = np.asarray(e, float) / np.linalg.norm(e)
        X = np.diag(np.asarray(positions)[atom] @ e)
        return C.T @ (S @ X + X @ S) @ C

    Mk, Mm = M(kick_dir), M(meas_dir)
    f = np.zeros(len(eps))
    f[:n_occ] = 2.0
    t = np.asarray(t, float)
    out = np.zeros_like(t)
    n = len(eps)
    for i in range(n):
        for j in range(n):
            if eps[i] > eps[j]:
                w = eps[i] - eps[j]
                out += 0.5 * kappa * (f[j] - f[i]) * Mk[i, j] * Mm[i, j] * np.sin(w * t)
    return out
