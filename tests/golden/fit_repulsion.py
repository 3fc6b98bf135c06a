"""Fit the synthetic model's pair repulsion (the repulsive energy of Sec. 2.1,
Eqs. 1 and 15) and print the constants that workloads/ stores.

Run from the repository root:  python tests/golden/fit_repulsion.py
Calls only oracle/ and workloads/ (about a minute on 8 host cores).

The two-centre model of the synthetic C/H systems has no repulsive energy of
its own, so its band energy falls without bound as atoms approach and
nuclei moving under its forces collapse. The repulsion
V_AB(r) = a[s_A, s_B] exp(-r / decay) (decay 0.5 bohr, a short-range wall)
takes its amplitudes from a non-negative least-squares fit: at the
reference geometry of the 499-atom moving-nuclei strip, in its SCC ground
state, the repulsive forces should cancel the oracle's electronic forces
(Eq. 15 without the repulsive term). One amplitude for C-C pairs and one
shared by C-H and H-H pairs; the seeded pair factors of the model leave
about half of the force (rms) that no species-pair repulsion can cancel.
"""
import os
import sys

import numpy as np
from scipy.optimize import nnls

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O              # noqa: E402
import oracle.ehrenfest as OE   # noqa: E402
import workloads as W           # noqa: E402

DECAY = 0.5                     # bohr


def electronic_forces(s, m):
    """Eq. 15 without the repulsive term, SCC ground state, no field."""
    gs = O.ground_state(s, tol=1e-10)
    Sinv = O.inverse_overlap(s.S)
    atom_of, _ = OE.orbital_types(m)
    v_orb = (s.gamma @ gs.dq)[atom_of]
    H = s.H0 + 0.5 * s.S * (v_orb[:, None] + v_orb[None, :])
    GS, GH = OE.fd_gradients(m, np.asarray(s.positions))
    return OE.forces(gs.rho.astype(np.complex128), H, Sinv, GS, GH, v_orb, gs.dq,
                     np.asarray(s.positions), m["hubbard_u"], None, m)


def fit(F, m, R):
    """Amplitudes (C-C, C-H = H-H) minimising |F + F_rep| over all atoms."""
    cols = []
    for pair in ("CC", "CH"):
        mm = dict(m, rep_decay=DECAY)
        a = np.zeros((2, 2))
        if pair == "CC":
            a[0, 0] = 1.0
        else:
            a[0, 1] = a[1, 0] = a[1, 1] = 1.0
        mm["rep_a"] = a
        cols.append(OE.repulsive_forces(mm, R).reshape(-1))
    G = np.array(cols).T
    amp, _ = nnls(G, -F.reshape(-1))
    res = F.reshape(-1) + G @ amp
    return amp, float(np.sqrt((res ** 2).mean() / (F ** 2).mean()))


def main():
    w = W.ehrenfest_workload()
    s = w.system
    m = W.two_centre_model(s)
    m.pop("rep_a", None)
    m.pop("rep_decay", None)
    R = np.asarray(s.positions)
    F = electronic_forces(s, m)
    amp, ratio = fit(F, m, R)
    print(f"REP_DECAY = {DECAY}")
    print(f"REP_A = {{'CC': {amp[0]:.6f}, 'CH': {amp[1]:.6f}, 'HH': {amp[1]:.6f}}}")
    print(f"# residual force rms / electronic force rms: {ratio:.3f}")


if __name__ == "__main__":
    main()
