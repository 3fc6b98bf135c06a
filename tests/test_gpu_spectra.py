"""Spectra on the GPU (through the C ABI) against the CPU oracle.

The damped Fourier sums run as FP64 matrix-core products, so they match the
oracle's direct sums to FP64 rounding; a pump-probe protocol run end to end
(pump with a laser, probe batch branched from its snapshots, transient
absorption) is checked against the same protocol run by the oracle.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _T():
    from paper_1912_03174_amd import tddftb as T
    return T


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def series(J, T, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(T) * 0.2
    freqs = rng.uniform(0.05, 1.2, size=(J, 6))
    amps = rng.standard_normal((J, 6)) * 1e-4
    mu = (amps[:, :, None] * np.sin(freqs[:, :, None] * t[None, None, :])).sum(axis=1)
    return t, mu + rng.standard_normal((J, 1)) * 0.3


@pytest.mark.parametrize("J,T,Wn,tau", [(1, 2, 1, 0.0), (5, 1001, 137, 0.0), (130, 777, 65, 60.0)])
def test_spectrum_matches_oracle(J, T, Wn, tau):
    Tm = _T()
    say(f"spectrum {J}x{T} at {Wn} frequencies")
    t, mu = series(J, T, seed=J + T)
    e0 = np.linspace(1e-3, 2e-3, J)
    omega = np.linspace(0.02, 1.5, Wn)
    alpha, sigma = Tm.td_spectrum(mu, e0, 0.2, omega, tau=tau)
    for j in range(J):
        ref = O.polarizability(t, mu[j], e0[j], omega, tau=tau if tau > 0 else None)
        scale = np.abs(ref).max() + 1e-300
        assert np.abs(alpha[j] - ref).max() <= 1e-12 * scale + 1e-300
        assert np.abs(sigma[j] - O.cross_section(omega, ref)).max() <= \
            1e-12 * np.abs(O.cross_section(omega, ref)).max() + 1e-300


def test_effective_polarizability_with_reference():
    Tm = _T()
    t, mu = series(7, 900, seed=3)
    _, pump = series(7, 900, seed=4)
    omega = np.linspace(0.05, 1.0, 70)
    alpha, _ = Tm.td_spectrum(mu, 1e-3, 0.2, omega, ref=pump, tau=80.0)
    for j in range(7):
        ref = O.effective_polarizability(t, mu[j], pump[j], 1e-3, omega, tau=80.0)
        assert np.abs(alpha[j] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("width,ref_delay", [(0.0, -1), (0.004, 5)])
def test_transient_absorption_matches_oracle(width, ref_delay):
    Tm = _T()
    D, A, Tn = 40, 12, 700
    t, mu = series(D * A, Tn, seed=11)
    _, pump = series(D * A, Tn, seed=12)
    mu = mu.reshape(D, A, Tn)
    pump = pump.reshape(D, A, Tn)
    e0 = np.full((D, A), 1e-3)
    omega = np.linspace(0.05, 1.2, 90)
    step = 6.0
    out = Tm.td_transient_absorption(mu, pump, e0, 0.2, omega, tau=100.0, ref_delay=ref_delay,
                                     delay_step=step, filter_width=width)
    alphas = np.array([[O.effective_polarizability(t, mu[d, a], pump[d, a], 1e-3, omega,
                                                   tau=100.0) for a in range(A)]
                       for d in range(D)])
    ref = O.transient_cross_section(omega, alphas)
    if width > 0:
        ref = O.gaussian_filter_delay(ref, step, width)
    if ref_delay >= 0:
        ref = O.delta_absorbance(ref, ref_delay)
    assert np.abs(out - ref).max() <= 1e-10 * np.abs(ref).max()


def test_pump_probe_protocol_end_to_end():
    """Pump laser on the flake, probe batch branched at three delays after the
    pump (x, y, z kicks, four pump phases), transient absorption on the GPU;
    the oracle runs the same protocol."""
    Tm = _T()
    s = W.flake_c24h16()
    dt, t_p, e0 = 0.2, 60.0, 1e-3
    n_pump = int(round(t_p / dt))
    delays = [n_pump, n_pump + 25, n_pump + 50]
    n_probe = 150
    n_total = delays[-1] + n_probe
    phases = [0.0, 0.5 * np.pi, np.pi, 1.5 * np.pi]
    axes = np.eye(3)
    omega = np.linspace(0.05, 1.0, 60)
    say("pump-probe end to end")
    gs = O.ground_state(s, tol=1e-13)
    Sinv = O.inverse_overlap(s.S)
    mu_gpu, ref_gpu, mu_cpu, ref_cpu = [], [], [], []
    snaps = []
    for phi in phases:
        field = W.sin2_pulse(np.arange(n_total) * dt, 0.01, 0.3, t_p, (1.0, 1.0, 0.0), phase=phi)
        p = Tm.Propagator(s, rho0=gs.rho)
        pump_mu = []
        done = 0
        snap = {}
        for d in delays:
            pump_mu.append(p.step(d - done, field[done:d]))
            snap[d] = p.rho()[0]
            done = d
        pump_mu.append(p.step(n_total - done, field[done:]))
        pump_mu = np.vstack(pump_mu)
        p.close()
        ref_o = O.propagate(s, gs.rho, n_total, dt, Sinv=Sinv, field=field, record_energy=False)
        snaps.append((phi, snap, pump_mu, ref_o))
    # probes: one batch over delays x phases x axes
    systems, rho0s, kicks = [], [], []
    for phi, snap, _, _ in snaps:
        for d in delays:
            for ax in axes:
                systems.append(s)
                rho0s.append(snap[d])
                kicks.append(ax)
    b = Tm.Batch(systems, rho0s=rho0s)
    b.kick(np.full(len(systems), e0), np.array(kicks))
    b.step(n_probe)
    m = 0
    for phi, snap, pump_mu, ref_o in snaps:
        for d in delays:
            for k, ax in enumerate(axes):
                mu_gpu.append(b.dipoles(m, n_probe) @ ax)
                ref_gpu.append(pump_mu[d:d + n_probe] @ ax)
                m += 1
    b.close()
    # the oracle's probes, branched from its own pump run at the same steps
    for phi, snap, pump_mu, ref_o in snaps:
        field = W.sin2_pulse(np.arange(n_total) * dt, 0.01, 0.3, t_p, (1.0, 1.0, 0.0), phase=phi)
        for d in delays:
            pre = O.propagate(s, gs.rho, d, dt, Sinv=Sinv, field=field[:d], record_energy=False)
            for ax in axes:
                rk = O.kick(pre.rho, s.S, Sinv, s.positions, s.orb_offset, e0, ax)
                pr = O.propagate(s, rk, n_probe, dt, Sinv=Sinv, record_energy=False)
                mu_cpu.append(pr.dipoles @ ax)
                ref_cpu.append(ref_o.dipoles[d:d + n_probe] @ ax)
    shape = (len(phases), len(delays), 3, n_probe)
    to_delay_major = lambda x: np.array(x).reshape(shape).transpose(1, 0, 2, 3).reshape(
        len(delays), len(phases) * 3, n_probe)
    mg, rg, mc, rc = map(to_delay_major, (mu_gpu, ref_gpu, mu_cpu, ref_cpu))
    diff = np.abs((mg - rg) - (mc - rc)).max() / np.abs(mc - rc).max()
    say(f"probe-minus-pump dipole relative difference {diff:.2e}")
    assert diff < 1e-8
    ta = Tm.td_transient_absorption(mg, rg, e0, dt, omega, tau=40.0, ref_delay=0)
    t = np.arange(n_probe) * dt
    alphas = np.array([[O.effective_polarizability(t, mc[d, a], rc[d, a], e0, omega, tau=40.0)
                        for a in range(mc.shape[1])] for d in range(len(delays))])
    ta_ref = O.delta_absorbance(O.transient_cross_section(omega, alphas), 0)
    sig_ref = O.transient_cross_section(omega, alphas)
    err = np.abs(ta - ta_ref).max() / np.abs(sig_ref).max()
    say(f"transient absorption relative difference {err:.2e}")
    assert err < 1e-7
