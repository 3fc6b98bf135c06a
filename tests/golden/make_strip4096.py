"""Write the oracle fixture of a 500-step FP64 run at N_orb = 4096.

Run from the repository root:  python tests/golden/make_strip4096.py
Calls only oracle/ and workloads/ (about 15 minutes on 8 host cores).

The run: the benchmark's C938H344 strip (N_orb = 4096), its sin^2 laser
sampled at steps 5000 .. 5499 (mid pulse), dt = 0.2 au, from the seeded
pair of Hermitian densities around the neutral rho = 1 (seeds 43 and 44,
scale 1e-3, each scaled to Tr(rho S) = N_e) taken as (rho_5000,
rho_4999): 500 leapfrog steps of Eq. 19 with the charges, the SCC
Hamiltonian and the three complex products of Eq. 10 at every step. The
fixture holds the dipole of every step and the charges of the final
density.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O      # noqa: E402
import workloads as W   # noqa: E402

K0, STEPS = 5000, 500
HERE = os.path.dirname(os.path.abspath(__file__))
DIPOLE = os.path.join(HERE, "strip4096_fp64_dipole.txt")
CHARGES = os.path.join(HERE, "strip4096_fp64_charges.txt")


def start_state(s):
    """The seeded (current, previous) densities of the run (inputs only)."""
    n = s.n_orb
    r1, i1 = W.random_hermitian_pair(n, seed=43, scale=1e-3, base=np.eye(n))
    r0, i0 = W.random_hermitian_pair(n, seed=44, scale=1e-3, base=np.eye(n))
    cur, prev = r1 + 1j * i1, r0 + 1j * i0
    cur *= s.n_elec / np.sum(cur.real * s.S)
    prev *= s.n_elec / np.sum(prev.real * s.S)
    return cur, prev


def compute(steps=STEPS):
    w = W.workload(3)
    s = w.system
    cur, prev = start_state(s)
    tr = O.propagate(s, cur, steps, w.dt, rho_prev=prev, step0=K0, field=w.field(K0, steps),
                     record_energy=False)
    dq_end = O.charge_fluctuations(tr.rho, s.S, s.orb_offset, s.q0)
    return tr.dipoles, dq_end


if __name__ == "__main__":
    mu, dq = compute()
    with open(DIPOLE, "w") as f:
        f.write(f"# oracle dipole (au) of {STEPS} FP64 leapfrog steps of the C938H344 strip "
                f"(N_orb = 4096) under its laser from step {K0}\n")
        f.write("# written by tests/golden/make_strip4096.py (oracle/ and workloads/ only)\n")
        f.write("# step mu_x mu_y mu_z\n")
        for k, m in enumerate(mu):
            f.write(f"{K0 + k:d} {m[0]:.17e} {m[1]:.17e} {m[2]:.17e}\n")
    with open(CHARGES, "w") as f:
        f.write(f"# oracle Mulliken charge fluctuations of the density after step {K0 + STEPS - 1}"
                " of the same run\n")
        f.write("# written by tests/golden/make_strip4096.py (oracle/ and workloads/ only)\n")
        for v in dq:
            f.write(f"{v:.17e}\n")
    print("wrote", DIPOLE, CHARGES)
