"""Plain CPU oracle: the DFTB+U (fully-localised limit) and pseudo-SIC
corrections of the Hamiltonian, in FP64.

TEST INFRASTRUCTURE, like ``oracle.tddftb``: imported only by the tests;
shares no code with the GPU library. Follows Bonafe et al., arXiv
1912.03174, Sec. 3.2: the FLL energy and potential (Eqs. 21-22) in the
dual (Mulliken-block) populations of Eq. 23, and the pseudo-SIC energy
and potential (Eqs. 24-25).

Readings:

* Shells. A shell is a contiguous range of orbitals of one atom (s, p, ...)
  with its own U_eff; the corrections act on the on-site block of each
  shell (Eq. 23: mu, nu in the same shell l of atom A).
* Spin. The density matrix is spin-summed (closed shell). The per-spin
  block population is n / 2, and Eqs. 21 and 24 are summed over both spins:
      FLL:  dE = sum_b [ -(U_b / 4) sum_uv n_uv^2 + (U_b / 2) sum_u n_uu ]
      pSIC: dE = sum_b   -(U_b / 4) sum_uv n_uv^2
  The printed FLL energy places n_uu inside the double sum over u, v; the
  printed potential (Eq. 22, -U (n - delta/2) per spin) fixes it as one
  term per diagonal element. With this reading FLL moves an occupied
  orbital of the shell down by U/2 and an empty one up by U/2 (the
  scissor-like action the text describes) and pSIC moves only occupied
  orbitals, down by U (it leaves empty states alone, as the text says).
* Complex rho. During propagation the off-diagonal block populations
  acquire imaginary parts; the paper does not say how they enter. The
  populations are taken from Re(rho), so H stays real symmetric and the
  energy E(rho) has dE = Tr(H drho), which makes it a constant of the
  motion of Eq. 10 with no field.
* Potential to Hamiltonian. With V_b = dE / dn_b on each block (the
  potential of Eq. 22 / 25 per spin), the Hamiltonian term is the
  derivative of dE through Eq. 23: dH = 1/2 (S V + V S), V block diagonal,
  the same dual form as the SCC term 1/2 S_uv (v_u + v_v) of Eq. 6.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import tddftb as T

FLL = "fll"
PSIC = "psic"


@dataclasses.dataclass
class PlusU:
    mode: str                  # FLL or PSIC
    shell_offset: np.ndarray   # [n_shells + 1] orbital ranges, each inside one atom
    shell_u: np.ndarray        # [n_shells] U_eff (Ha); 0 leaves a shell uncorrected


def block_populations(rho, S, shell_offset):
    """Dual populations of each shell's on-site block (Sec. 3.2, Eq. 23):
    n = 1/2 (rho S + S rho) restricted to the shell, from Re(rho)."""
    R = np.real(np.asarray(rho))
    N = 0.5 * (R @ S + S @ R)
    off = np.asarray(shell_offset)
    return [N[a:b, a:b].copy() for a, b in zip(off[:-1], off[1:])]


def plus_u_energy(blocks, shell_u, mode):
    """Correction energy (Sec. 3.2, Eq. 21 for FLL, Eq. 24 for pSIC; spin
    reading in the module header)."""
    e = 0.0
    for n, u in zip(blocks, shell_u):
        e -= 0.25 * u * float((n * n).sum())
        if mode == FLL:
            e += 0.5 * u * float(np.trace(n))
    return e


def plus_u_potential(blocks, shell_u, mode):
    """V_b = d(dE)/d(n_b) (Sec. 3.2, Eq. 22 for FLL, Eq. 25 for pSIC)."""
    out = []
    for n, u in zip(blocks, shell_u):
        if mode == FLL:
            out.append(-0.5 * u * (n - np.eye(len(n))))
        else:
            out.append(-0.5 * u * n)
    return out


def plus_u_hamiltonian(S, potentials, shell_offset):
    """dH = 1/2 (S V + V S) with V the block-diagonal matrix of the shell
    potentials (the derivative of the energy through Eq. 23)."""
    n = len(S)
    V = np.zeros((n, n))
    off = np.asarray(shell_offset)
    for (a, b), vb in zip(zip(off[:-1], off[1:]), potentials):
        V[a:b, a:b] = vb
    return 0.5 * (S @ V + V @ S)


def hamiltonian(system, rho, pu, field=None):
    """SCC Hamiltonian (Eqs. 6-7) plus the correction of rho's block
    populations; also returns the charges and the correction energy."""
    dq = T.charge_fluctuations(rho, system.S, system.orb_offset, system.q0)
    V = T.external_potential(system.positions, field) if field is not None else None
    H = T.scc_hamiltonian_fast(system.H0, system.S, system.gamma, dq, system.orb_offset, V)
    blocks = block_populations(rho, system.S, pu.shell_offset)
    H = H + plus_u_hamiltonian(system.S, plus_u_potential(blocks, pu.shell_u, pu.mode),
                               pu.shell_offset)
    return H, dq, plus_u_energy(blocks, pu.shell_u, pu.mode)


def energy(system, rho, pu, field=None):
    """Total energy: the SCC energy of ``oracle.tddftb.energy`` plus the
    correction (Eq. 21 or 24)."""
    dq = T.charge_fluctuations(rho, system.S, system.orb_offset, system.q0)
    blocks = block_populations(rho, system.S, pu.shell_offset)
    return (T.energy(rho, system.H0, system.gamma, dq, system.positions, field)
            + plus_u_energy(blocks, pu.shell_u, pu.mode))


def ground_state(system, pu, tol=1e-13, maxiter=400, history=8, beta=0.3):
    """Self-consistent ground state with the correction: the charges and the
    shells' block populations are iterated together (Anderson mixing of
    the concatenated vector) to a fixed point of aufbau filling (Sec. 2.1)
    of the corrected Hamiltonian."""
    S, H0, gamma = system.S, system.H0, system.gamma
    off, q0 = system.orb_offset, system.q0
    n_occ = system.n_elec // 2
    soff = np.asarray(pu.shell_offset)
    sizes = [int(b - a) for a, b in zip(soff[:-1], soff[1:])]
    na = system.n_atoms

    def split(x):
        dq = x[:na]
        blocks, p = [], na
        for m in sizes:
            blocks.append(x[p:p + m * m].reshape(m, m))
            p += m * m
        return dq, blocks

    x_in = np.zeros(na + sum(m * m for m in sizes))
    xs, fs = [], []
    res = np.inf
    for it in range(1, maxiter + 1):
        dq_in, n_in = split(x_in)
        H = T.scc_hamiltonian_fast(H0, S, gamma, dq_in, off)
        H = H + plus_u_hamiltonian(S, plus_u_potential(n_in, pu.shell_u, pu.mode), soff)
        rho, eps, C = T._aufbau_density(H, S, n_occ)
        dq_out = T.charge_fluctuations(rho, S, off, q0)
        n_out = block_populations(rho, S, soff)
        x_out = np.concatenate([dq_out] + [b.reshape(-1) for b in n_out])
        r = x_out - x_in
        res = float(np.abs(r).max())
        if res < tol:
            break
        xs.append(x_in.copy())
        fs.append(r.copy())
        xs, fs = xs[-history:], fs[-history:]
        if len(fs) == 1:
            x_in = x_in + beta * r
        else:
            dF = np.array([fs[k + 1] - fs[k] for k in range(len(fs) - 1)]).T
            dX = np.array([xs[k + 1] - xs[k] for k in range(len(xs) - 1)]).T
            g, *_ = np.linalg.lstsq(dF, r, rcond=None)
            x_in = x_in + beta * r - (dX + beta * dF) @ g
    gap = float(eps[n_occ] - eps[n_occ - 1]) if n_occ < len(eps) else np.inf
    return T.GroundState(rho=rho, dq=dq_out, H=H, eps=eps, C=C, iterations=it, residual=res,
                         gap=gap)


def propagate(system, pu, rho, n_steps, dt, field=None, Sinv=None):
    """Clamped-nuclei leapfrog (Sec. 2.3, Eq. 19) with the corrected
    Hamiltonian rebuilt from rho at every step. Returns (rho, rho_prev,
    dipoles [n, 3], energies [n]) of the densities entering each step."""
    S = system.S
    if Sinv is None:
        Sinv = T.inverse_overlap(S)
    cur = np.asarray(rho, dtype=np.complex128)
    prev = None
    mus = np.zeros((n_steps, 3))
    es = np.zeros(n_steps)
    for k in range(n_steps):
        E = None if field is None else field[k]
        H, dq, _ = hamiltonian(system, cur, pu, E)
        mus[k] = T.dipole(dq, system.positions)
        es[k] = energy(system, cur, pu, E)
        rd = T.rho_dot(cur, H, Sinv)
        nxt = T.euler_step(cur, rd, dt) if prev is None else T.leapfrog_step(prev, rd, dt)
        prev, cur = cur, nxt
    return cur, prev, mus, es
