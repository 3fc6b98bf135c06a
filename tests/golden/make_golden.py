"""Write the oracle regression fixture for the 112-orbital flake workload.

Run from the repository root:  python tests/golden/make_golden.py
Calls only oracle/ and workloads/. The fixture holds the dipole of the
kicked flake (delta kick 0.001 au along x, dt 0.2 au) every 10 steps
over 500 steps, starting from the oracle's SCC ground state.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O      # noqa: E402
import workloads as W   # noqa: E402


def compute():
    w = W.workload(1)
    s = w.system
    gs = O.ground_state(s)
    Sinv = O.inverse_overlap(s.S)
    rk = O.kick(gs.rho, s.S, Sinv, s.positions, s.orb_offset, *w.kick)
    tr = O.propagate(s, rk, w.n_steps, w.dt, Sinv=Sinv, record_energy=False)
    return np.arange(0, w.n_steps, 10), tr.dipoles[::10]


if __name__ == "__main__":
    steps, mu = compute()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "flake112_dipole.txt")
    with open(out, "w") as f:
        f.write("# oracle dipole (au) of the kicked C24H16 flake, every 10 steps of 0.2 au\n")
        f.write("# written by tests/golden/make_golden.py (oracle/ only)\n")
        f.write("# step mu_x mu_y mu_z\n")
        for k, m in zip(steps, mu):
            f.write(f"{k:d} {m[0]:.17e} {m[1]:.17e} {m[2]:.17e}\n")
    print("wrote", out)
