"""Seeded synthetic TD-DFTB inputs (geometry, S, H0, gamma, fields).

This module is shared by the CPU oracle, the tests and the benchmark. It
builds *inputs only*: atom positions, the orbital layout, the overlap S,
the non-SCC Hamiltonian H0, the charge kernel gamma, reference
populations, sampled external fields and seeded random matrices. It
contains none of the propagation arithmetic (charges, Hamiltonian
rebuild, equation of motion, integrator, kick, observables).

Systems are carbon/hydrogen honeycomb flakes and armchair strips, the
shape of the paper's aromatic-molecule and armchair graphene-nanoribbon
workloads (Sec. 3.1, Sec. 5.2). The paper's Slater-Koster parameter files
are not available, so S and H0 are synthetic two-centre tables:

* every two-centre integral (overlap or hopping) of type k between atoms
  at distance r is  c_k * exp(-r / 1.2 Angstrom), times the Slater-Koster
  angular factor of the orbital pair (Slater and Koster 1954, Table I);
  each atom pair carries one seeded scale factor in [0.95, 1.05];
* on-site blocks: S = identity, H0 = diag(s: -0.5 Ha, p: -0.2 Ha);
* gamma_AB = 1 / sqrt(r_AB^2 + U^-2) with U = 0.4 Ha, so gamma_AA = U (the
  on-site Hubbard value of the Coulomb term, Sec. 2.1) and 1/r at range;
* reference populations are the neutral valence counts q0_C = 4,
  q0_H = 1, giving a closed shell with N_e = N_orb.

Carbon atoms carry s, px, py, pz (in that order), hydrogen one s.
Units are atomic (bohr, hartree, au of time and field).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ANGSTROM = 1.8897261246257702  # bohr per Angstrom
FS = 41.341373335              # au of time per femtosecond

CC_BOND_A = 1.42
CH_BOND_A = 1.09
DECAY_A = 1.2

# c_k prefactors (value at r -> 0 of c_k exp(-r / 1.2 A)).
# Overlap: |S| <= 0.28 at the C-C and C-H bond lengths.
S_TABLE = {
    "CC": dict(ss=0.80, sp=-0.80, pps=-0.90, ppp=0.50),
    "CH": dict(ss=0.68, sp=-0.68),
    "HH": dict(ss=0.70),
}
# Hopping: signs and sizes of a carbon tight-binding parameter set.
H_TABLE = {
    "CC": dict(ss=-1.17, sp=1.17, pps=0.99, ppp=-0.675),
    "CH": dict(ss=-1.08, sp=1.08),
    "HH": dict(ss=-1.08),
}
ONSITE = dict(s=-0.5, p=-0.2)
HUBBARD_U = 0.4
Q0 = dict(C=4.0, H=1.0)
N_ORB = dict(C=4, H=1)


@dataclasses.dataclass
class System:
    """Inputs of one trajectory. Arrays are float64, row-major."""

    species: list            # 'C' or 'H' per atom
    positions: np.ndarray    # [n_atoms, 3] bohr
    orb_offset: np.ndarray   # [n_atoms + 1] int32, orbitals of atom A contiguous
    S: np.ndarray            # [n_orb, n_orb]
    H0: np.ndarray           # [n_orb, n_orb]
    gamma: np.ndarray        # [n_atoms, n_atoms]
    q0: np.ndarray           # [n_atoms]
    n_elec: int              # closed shell, even
    name: str = ""
    seed: int = 0            # seed of the two-centre scale factors (see two_centre_model)

    @property
    def n_atoms(self) -> int:
        return len(self.species)

    @property
    def n_orb(self) -> int:
        return int(self.orb_offset[-1])

    @property
    def n_occ(self) -> int:
        return self.n_elec // 2


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def _honeycomb(centres, a, start_deg):
    """Unique vertices and bond matrix of hexagons of side a at ``centres``."""
    verts = {}
    for c in centres:
        for k in range(6):
            ang = math.radians(start_deg + 60.0 * k)
            p = np.asarray(c) + a * np.array([math.cos(ang), math.sin(ang)])
            key = (round(p[0] * 1e4), round(p[1] * 1e4))
            verts.setdefault(key, p)
    pts = np.array([verts[k] for k in sorted(verts)])
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=-1)
    bonds = np.abs(d - a) < 1e-3 * a
    return pts, bonds


def coronene_skeleton(a=CC_BOND_A):
    """C24 coronene: a hexagon and its six neighbours."""
    s3 = math.sqrt(3.0)
    cs = [(0.0, 0.0)] + [(s3 * a * math.cos(math.radians(60 * k)),
                          s3 * a * math.sin(math.radians(60 * k))) for k in range(6)]
    return _honeycomb(cs, a, 30.0)


def armchair_skeleton(width, length, extra=0, a=CC_BOND_A):
    """Armchair strip along x: ``length`` columns of flat-top hexagons.

    Columns alternate ``width`` and ``width - 1`` hexagons (a (2 width + 1)
    dimer-line armchair ribbon); ``extra`` hexagons start one more column.
    """
    s3 = math.sqrt(3.0)
    cells = [(i, j) for i in range(length) for j in range(width - (i % 2))]
    cells += [(length, j) for j in range(extra)]
    cs = [(1.5 * a * i, s3 * a * (j + 0.5 * (i % 2))) for (i, j) in cells]
    return _honeycomb(cs, a, 0.0)


def saturate(pts, bonds, n_pairs, rng):
    """Hydrogen positions (Angstrom) for a planar carbon skeleton.

    Each carbon with two C neighbours gets one H along its open sigma
    direction, except for sp3 CH2 sites, whose carbon gets two H above and
    below the plane at the tetrahedral angle:

    * every isolated edge carbon (two C neighbours, neither of them an
      edge carbon: a zigzag site) is a CH2 site, which removes the
      zigzag end states that would otherwise sit at the Fermi level of a
      finite armchair strip;
    * ``n_pairs`` seeded disjoint pairs of *bonded* edge carbons are CH2
      sites (a hydrogenated edge C=C bond, keeping the pi system
      closed-shell).
    """
    deg = bonds.sum(1)
    if (deg < 2).any():
        raise ValueError("carbon with fewer than two C neighbours")
    n = len(pts)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)
             if bonds[i, j] and deg[i] == 2 and deg[j] == 2]
    in_pair = {x for p in pairs for x in p}
    used = {i for i in range(n) if deg[i] == 2 and i not in in_pair}
    chosen = 0
    if n_pairs:
        for k in rng.permutation(len(pairs)):
            i, j = pairs[k]
            if i in used or j in used:
                continue
            used |= {i, j}
            chosen += 1
            if chosen == n_pairs:
                break
    if chosen != n_pairs:
        raise ValueError("not enough edge C=C pairs for the CH2 count")
    up = np.array([0.0, 0.0, 1.0])
    half = math.radians(109.47 / 2.0)
    h = []
    for c in np.nonzero(deg == 2)[0]:
        u = np.zeros(2)
        for nb in np.nonzero(bonds[c])[0]:
            v = pts[nb] - pts[c]
            u -= v / np.linalg.norm(v)
        u = np.array([u[0], u[1], 0.0]) / np.linalg.norm(u)
        p = np.array([pts[c][0], pts[c][1], 0.0])
        if c in used:
            for s in (1.0, -1.0):
                h.append(p + CH_BOND_A * (math.cos(half) * u + s * math.sin(half) * up))
        else:
            h.append(p + CH_BOND_A * u)
    return np.array(h)


def molecule(pts, bonds, n_pairs, seed, jitter_a=0.01):
    """(species, positions in bohr) of a saturated, jittered, centred C/H system."""
    rng = np.random.default_rng(seed)
    hs = saturate(pts, bonds, n_pairs, rng)
    c3 = np.concatenate([pts, np.zeros((len(pts), 1))], axis=1)
    pos = np.concatenate([c3, hs], axis=0)
    pos = pos - pos.mean(axis=0)
    pos = pos + rng.normal(scale=jitter_a, size=pos.shape)
    return ["C"] * len(pts) + ["H"] * len(hs), pos * ANGSTROM


# ----------------------------------------------------------------------------
# matrices
# ----------------------------------------------------------------------------

def orbital_layout(species):
    counts = np.array([N_ORB[s] for s in species], dtype=np.int32)
    off = np.zeros(len(species) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    return off


def _two_centre(species, positions, table, jit):
    """Dense matrix of two-centre integrals c_k exp(-r/1.2A) x SK angular factor.

    Off-site blocks only; on-site blocks are zero. ``jit`` [n_atoms, n_atoms]
    scales each atom pair.
    """
    off = orbital_layout(species)
    n = int(off[-1])
    is_c = np.array([s == "C" for s in species])
    pos_a = positions / ANGSTROM
    v = pos_a[None, :, :] - pos_a[:, None, :]          # v[a, b] = R_b - R_a
    r = np.linalg.norm(v, axis=-1)
    np.fill_diagonal(r, 1.0)
    d = v / r[..., None]
    f = jit * np.exp(-r / DECAY_A)
    np.fill_diagonal(f, 0.0)
    s_idx = off[:-1]
    c_idx = np.nonzero(is_c)[0]
    cc = is_c[:, None] & is_c[None, :]
    hh = ~is_c[:, None] & ~is_c[None, :]
    M = np.zeros((n, n))
    ss = np.where(cc, table["CC"]["ss"], np.where(hh, table["HH"]["ss"], table["CH"]["ss"]))
    M[np.ix_(s_idx, s_idx)] = ss * f
    # s on atom a, p on carbon b: d_k * c_sp (the reverse pair follows by symmetry)
    sp = np.where(is_c[:, None], table["CC"]["sp"], table["CH"]["sp"]) * f
    for k in range(3):
        blk = (d[:, :, k] * sp)[:, c_idx]
        M[np.ix_(s_idx, off[c_idx] + 1 + k)] = blk
        M[np.ix_(off[c_idx] + 1 + k, s_idx)] = blk.T
    fcc = f[np.ix_(c_idx, c_idx)]
    dcc = d[np.ix_(c_idx, c_idx)]
    pps, ppp = table["CC"]["pps"], table["CC"]["ppp"]
    for k in range(3):
        for l in range(3):
            blk = dcc[:, :, k] * dcc[:, :, l] * (pps - ppp) * fcc
            if k == l:
                blk = blk + ppp * fcc
            M[np.ix_(off[c_idx] + 1 + k, off[c_idx] + 1 + l)] = blk
    return off, M


def build_matrices(species, positions, seed):
    """(orb_offset, S, H0, gamma) for atoms at ``positions`` (bohr)."""
    jit_s, jit_h = pair_scales(len(species), seed)
    off, S = _two_centre(species, positions, S_TABLE, jit_s)
    _, H0 = _two_centre(species, positions, H_TABLE, jit_h)
    n = int(off[-1])
    onsite = np.full(n, ONSITE["s"])
    for a, s in enumerate(species):
        if s == "C":
            onsite[off[a] + 1:off[a] + 4] = ONSITE["p"]
    S[np.diag_indices(n)] = 1.0
    H0[np.diag_indices(n)] = onsite
    rb = np.linalg.norm(positions[:, None, :] - positions[None, :, :], axis=-1)
    gamma = 1.0 / np.sqrt(rb ** 2 + HUBBARD_U ** -2)
    return off, S, H0, gamma


def make_system(species, positions, seed, name="") -> System:
    off, S, H0, gamma = build_matrices(species, positions, seed)
    q0 = np.array([Q0[s] for s in species])
    n_elec = int(round(q0.sum()))
    if n_elec % 2:
        raise ValueError("open-shell electron count")
    return System(species=list(species), positions=np.ascontiguousarray(positions),
                  orb_offset=off, S=S, H0=H0, gamma=gamma, q0=q0, n_elec=n_elec,
                  name=name, seed=seed)


AMU = 1822.888486209           # electron masses per atomic mass unit
MASS_AMU = dict(C=12.0, H=1.0)


def pair_scales(n_atoms, seed):
    """The seeded per-atom-pair factors of the overlap and of H0 (symmetric,
    [0.95, 1.05] off the diagonal, 0 on it), as used by build_matrices."""
    rng = np.random.default_rng(seed + 7919)
    jit_s = np.triu(rng.uniform(0.95, 1.05, size=(n_atoms, n_atoms)), 1)
    jit_s = jit_s + jit_s.T
    jit_h = np.triu(rng.uniform(0.95, 1.05, size=(n_atoms, n_atoms)), 1)
    jit_h = jit_h + jit_h.T
    return jit_s, jit_h


# Pair repulsion of the two-centre model, V_AB(r) = a exp(-r / REP_DECAY)
# (hartree, bohr): the model's repulsive energy (Sec. 2.1), a short-range
# wall whose amplitudes were fitted by tests/golden/fit_repulsion.py (oracle
# forces of the 499-atom strip's ground state; stored here as constants).
REP_DECAY = 0.5
REP_A = {"CC": 18.837233, "CH": 5.910942, "HH": 5.910942}


def two_centre_model(system: System) -> dict:
    """The parameters S and H0 of ``system`` are built from, as plain arrays,
    so S(R) and H0(R) can be rebuilt at other positions (moving nuclei).

    Species index 0 = C (s, px, py, pz), 1 = H (s). ``sk_s`` / ``sk_h``
    [2, 2, 4]: for the ordered species pair (i, j) the prefactors of
    (ss sigma, sp sigma with s on i and p on j, pp sigma, pp pi); each
    integral is prefactor x exp(-r / decay) x the Slater-Koster angular
    factor (direction cosines from the first atom to the second) x the
    pair's scale factor. ``onsite`` [2, 2]: H0 on-site s and p energies.
    ``mass`` in electron masses. ``rep_a`` [2, 2] and ``rep_decay``: the
    pair repulsion a[s_A, s_B] exp(-r / rep_decay)."""
    idx = {"C": 0, "H": 1}
    sk_s = np.zeros((2, 2, 4))
    sk_h = np.zeros((2, 2, 4))
    for tab, out in ((S_TABLE, sk_s), (H_TABLE, sk_h)):
        out[0, 0] = [tab["CC"]["ss"], tab["CC"]["sp"], tab["CC"]["pps"], tab["CC"]["ppp"]]
        out[0, 1, 0] = out[1, 0, 0] = tab["CH"]["ss"]
        out[1, 0, 1] = tab["CH"]["sp"]           # s on H, p on C
        out[1, 1, 0] = tab["HH"]["ss"]
    jit_s, jit_h = pair_scales(system.n_atoms, system.seed)
    return dict(
        species=np.array([idx[x] for x in system.species], dtype=np.int32),
        species_norb=np.array([4, 1], dtype=np.int32),
        sk_s=sk_s, sk_h=sk_h, decay=DECAY_A * ANGSTROM,
        scale_s=jit_s, scale_h=jit_h,
        onsite=np.array([[ONSITE["s"], ONSITE["p"]], [ONSITE["s"], ONSITE["p"]]]),
        hubbard_u=HUBBARD_U,
        mass=np.array([MASS_AMU["C"], MASS_AMU["H"]]) * AMU,
        rep_a=np.array([[REP_A["CC"], REP_A["CH"]], [REP_A["CH"], REP_A["HH"]]]),
        rep_decay=REP_DECAY,
    )


def thermal_velocities(system: System, kelvin, seed):
    """Seeded Maxwell-Boltzmann velocities (bohr / au time) at ``kelvin``,
    with the centre-of-mass motion removed."""
    rng = np.random.default_rng(seed)
    kb = 3.166811563e-6                      # hartree per kelvin
    m = np.array([MASS_AMU[x] for x in system.species]) * AMU
    v = rng.standard_normal((system.n_atoms, 3)) * np.sqrt(kb * kelvin / m)[:, None]
    v -= (m[:, None] * v).sum(axis=0) / m.sum()
    return v


def flake_c24h16(seed=1001) -> System:
    """40-atom hexagonal flake: coronene with two hydrogenated rim C=C bonds."""
    pts, bonds = coronene_skeleton()
    sp, pos = molecule(pts, bonds, n_pairs=2, seed=seed)
    return make_system(sp, pos, seed, name="C24H16 flake")


def strip_c640h384(seed=1002) -> System:
    """5-line armchair strip, 127 columns, 62 hydrogenated edge pairs: N_orb = 2944."""
    pts, bonds = armchair_skeleton(2, 127)
    sp, pos = molecule(pts, bonds, n_pairs=62, seed=seed)
    return make_system(sp, pos, seed, name="C640H384 strip")


def strip_c677h236(seed=1002) -> System:
    """7-line armchair strip, 96 columns, 18 pair CH2 sites: N_orb = 2944 as the
    C640H384 strip, but from the semiconducting ribbon family (non-SCC gap
    0.038 Ha), so its zero-temperature SCC ground state exists."""
    pts, bonds = armchair_skeleton(3, 96)
    sp, pos = molecule(pts, bonds, n_pairs=18, seed=seed)
    return make_system(sp, pos, seed, name="C677H236 strip")


def strip_c938h344(seed=1003) -> System:
    """7-line armchair strip, 133 columns, 2 zigzag + 34 pair CH2 sites: N_orb = 4096."""
    pts, bonds = armchair_skeleton(3, 133)
    sp, pos = molecule(pts, bonds, n_pairs=34, seed=seed)
    return make_system(sp, pos, seed, name="C938H344 strip")


def benzene(seed=11) -> System:
    """C6H6 ring (N_orb = 30), the smallest honeycomb test system."""
    pts, bonds = _honeycomb([(0.0, 0.0)], CC_BOND_A, 30.0)
    sp, pos = molecule(pts, bonds, n_pairs=0, seed=seed)
    return make_system(sp, pos, seed, name="C6H6")


def dimer(d=1.4, s=0.3, alpha=-0.5, beta=-0.35, u=0.0) -> System:
    """Two one-orbital atoms on the x axis at -d/2 and +d/2 (bohr), two electrons.

    S = [[1, s], [s, 1]], H0 = [[alpha, beta], [beta, alpha]]; gamma is
    u times the synthetic kernel (u = 0 switches the SCC term off).
    """
    pos = np.array([[-d / 2.0, 0.0, 0.0], [d / 2.0, 0.0, 0.0]])
    off = np.array([0, 1, 2], dtype=np.int32)
    S = np.array([[1.0, s], [s, 1.0]])
    H0 = np.array([[alpha, beta], [beta, alpha]])
    rb = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=-1)
    gamma = u / np.sqrt(rb ** 2 + HUBBARD_U ** -2)
    return System(species=["H", "H"], positions=pos, orb_offset=off, S=S, H0=H0,
                  gamma=gamma, q0=np.array([1.0, 1.0]), n_elec=2, name="dimer")


def small_strip(columns, n_pairs, seed, width=3) -> System:
    """Armchair strip of about ``columns`` columns (test sizes between the workloads).

    The first partial column (0..width hexagons) that gives a closed shell
    is appended.
    """
    for extra in range(width + 1):
        pts, bonds = armchair_skeleton(width, columns, extra)
        sp, pos = molecule(pts, bonds, n_pairs=n_pairs, seed=seed)
        if sum(Q0[s] for s in sp) % 2 == 0:
            return make_system(sp, pos, seed, name=f"strip w{width} x{columns}+{extra}")
    raise ValueError("no closed-shell strip of this length")


def probe_molecule(target_n, seed) -> System:
    """C/H strip with close to ``target_n`` orbitals (one member of a probe batch).

    Armchair strips one and three hexagons wide (two-wide strips of these
    lengths have near-degenerate frontier levels); the width whose length
    step lands closest to the target is taken. ``seed`` jitters the geometry
    and the two-centre parameters.
    """
    best = None
    for width, base, per in ((1, 30, 14), (3, 88, 30)):
        cols = max(2, int(round((target_n - base) / per)) + 2)
        s = small_strip(cols, 0, seed=seed, width=width)
        if best is None or abs(s.n_orb - target_n) < abs(best.n_orb - target_n):
            best = s
    return best


def probe_batch(count, seed=4000, n_lo=60, n_hi=800):
    """``count`` probe molecules with N_orb ~ uniform in [n_lo, n_hi] and a kick
    axis drawn from {x, y, z} for each: returns (systems, axes [count, 3])."""
    rng = np.random.default_rng(seed)
    targets = rng.integers(n_lo, n_hi + 1, size=count)
    axes = np.eye(3)[rng.integers(0, 3, size=count)]
    return [probe_molecule(int(t), seed + 1 + j) for j, t in enumerate(targets)], axes


# ----------------------------------------------------------------------------
# fields and workloads
# ----------------------------------------------------------------------------

def sin2_pulse(t, e0, omega, t_p, direction, phase=0.0):
    """E(t) = e0 sin(omega t + phase) sin^2(pi t / t_p) e, zero outside [0, t_p].

    The pump-pulse form of Sec. 5.1 with a sin^2 envelope; returns [len(t), 3].
    """
    t = np.asarray(t, dtype=np.float64)
    env = np.where((t >= 0) & (t <= t_p), np.sin(np.pi * t / t_p) ** 2, 0.0)
    amp = e0 * np.sin(omega * t + phase) * env
    e = np.asarray(direction, dtype=np.float64)
    e = e / np.linalg.norm(e)
    return amp[:, None] * e[None, :]


@dataclasses.dataclass
class Workload:
    name: str
    system: System
    dt: float
    n_steps: int
    kick: Optional[tuple]          # (E0, direction[3]) or None
    laser: Optional[dict]          # sin^2 pulse parameters or None
    description: str = ""

    def field(self, step0: int, n: int) -> Optional[np.ndarray]:
        """E(t_k) at t_k = k dt for k = step0 .. step0 + n - 1, shape [n, 3]."""
        if self.laser is None:
            return None
        t = np.arange(step0, step0 + n, dtype=np.float64) * self.dt
        L = self.laser
        return sin2_pulse(t, L["e0"], L["omega"], L["t_p"], L["direction"], L.get("phase", 0.0))


def workload(cfg: int) -> Workload:
    """Workloads by number: 1 flake N=112, 2 strip N=2944, 3 strip N=4096."""
    if cfg == 1:
        return Workload("flake112", flake_c24h16(), dt=0.2, n_steps=500,
                        kick=(1e-3, (1.0, 0.0, 0.0)), laser=None,
                        description="C24H16 flake, N_orb=112, delta kick 0.001 au along x, "
                                    "500 steps of 0.2 au")
    if cfg == 2:
        return Workload("strip2944", strip_c640h384(), dt=0.2, n_steps=20000,
                        kick=(1e-3, (1.0, 0.0, 0.0)), laser=None,
                        description="C640H384 armchair strip, N_orb=2944, delta kick 0.001 au "
                                    "along the strip axis, 20000 steps of 0.2 au")
    if cfg == 3:
        n_steps = 10000
        return Workload("strip4096", strip_c938h344(), dt=0.2, n_steps=n_steps,
                        kick=None,
                        laser=dict(e0=0.005, omega=0.1, t_p=n_steps * 0.2,
                                   direction=(0.0, 1.0, 0.0)),
                        description="C938H344 armchair strip, N_orb=4096, sin^2 laser "
                                    "0.1 Ha, 0.005 au, in-plane transverse, 10000 steps "
                                    "of 0.2 au")
    raise ValueError(f"unknown workload {cfg}")


def ehrenfest_workload() -> Workload:
    """Moving-nuclei pump run: 499-atom 7-line armchair strip (C383H116,
    N_orb = 1648), nuclei at 300 K (thermal_velocities seed 5000), sin^2 pump
    0.15 Ha, 0.01 au, t_p = 10 fs, in-plane across the strip (y), 5000 steps
    of 0.2 au. Across, not along: the strip is 223 bohr long, and a 0.01 au
    field along it would spread the atomic potentials R . E over 2.2 Ha,
    which with the 3.7 Ha wide spectrum of S^-1 H takes dt times the width
    past the leapfrog's limit of 1 at the pump's peak (18 bohr across:
    0.18 Ha)."""
    s = small_strip(54, 0, seed=1005, width=3)
    t_p = 10.0 * FS
    return Workload("strip1648md", s, dt=0.2, n_steps=5000, kick=None,
                    laser=dict(e0=0.01, omega=0.15, t_p=t_p, direction=(0.0, 1.0, 0.0)),
                    description="C383H116 strip, N_orb=1648, moving nuclei at 300 K, sin^2 "
                                "pump 0.15 Ha, 0.01 au, 10 fs across the strip, 5000 steps "
                                "of 0.2 au")


def spectrum_workload() -> Workload:
    """Absorption spectrum of a 2944-orbital ribbon: delta kick 0.001 au along
    the ribbon axis, 20000 steps of 0.2 au (the 2944-orbital workload's
    protocol on the semiconducting strip_c677h236)."""
    return Workload("strip2944s", strip_c677h236(), dt=0.2, n_steps=20000,
                    kick=(1e-3, (1.0, 0.0, 0.0)), laser=None,
                    description="C677H236 7-line armchair strip, N_orb=2944, delta kick "
                                "0.001 au along the strip axis, 20000 steps of 0.2 au")


# ----------------------------------------------------------------------------
# seeded random matrices (no physics)
# ----------------------------------------------------------------------------

def atomic_shells(system: System, u_by_shell=None):
    """Shells of the synthetic basis for the on-site corrections: one s
    shell per atom and one p shell per carbon, as contiguous orbital ranges.
    Returns (shell_offset [n_shells + 1] int32, shell_u [n_shells]) with
    shell_u taken from ``u_by_shell`` keyed by (species, 's' | 'p')
    (missing keys: 0)."""
    u_by_shell = u_by_shell or {}
    off, us = [0], []
    for a, sp in enumerate(system.species):
        lo, hi = int(system.orb_offset[a]), int(system.orb_offset[a + 1])
        off.append(lo + 1)
        us.append(float(u_by_shell.get((sp, "s"), 0.0)))
        if hi - lo == 4:
            off.append(hi)
            us.append(float(u_by_shell.get((sp, "p"), 0.0)))
    return np.array(off, dtype=np.int32), np.array(us)


def random_hermitian_pair(n, seed, scale=1e-3, base=None):
    """Seeded (Re, Im) of a Hermitian matrix: symmetric Re, antisymmetric Im."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) * scale
    b = rng.standard_normal((n, n)) * scale
    re = (a + a.T) / 2.0
    im = (b - b.T) / 2.0
    if base is not None:
        re = re + base
    return re, im


def random_matrix(m, n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) * scale
