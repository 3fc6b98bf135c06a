"""The C ABI library loads and exports every declared entry point (CPU only)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tddftb.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"TD_API\s+[\w\s\*]+?\b(td_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def T():
    from paper_1912_03174_amd import tddftb as T
    if not os.path.exists(T.LIB_PATH):
        pytest.fail("libtddftb.so is not built (run __graft_entry__.build())")
    T.load()
    return T


def test_every_declared_symbol_is_exported(T):
    names = declared()
    assert len(names) >= 15
    lib = ctypes.CDLL(T.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (td_\w+)", out))
    assert set(names) == exported
    assert set(T.EXPORTED) == set(names)


def test_defaults_and_status_strings(T):
    o = T.td_default_options()
    assert o.precision == T.TD_FP64 and o.dt == 0.2 and o.n_slices == 4
    assert T.status_string(T.TD_EINVAL) == "TD_EINVAL"
    assert T.status_string(-99) == "unknown status"


def test_invalid_arguments_rejected_before_device(T):
    s = W.flake_c24h16()
    bad = W.flake_c24h16()
    bad.n_elec = 3
    with pytest.raises(T.TdError) as e:
        T.td_create(bad)
    assert e.value.status == T.TD_EINVAL
    bad = W.flake_c24h16()
    bad.orb_offset = bad.orb_offset.copy()
    bad.orb_offset[3] = bad.orb_offset[2]
    with pytest.raises(T.TdError) as e:
        T.td_create(bad)
    assert e.value.status == T.TD_EINVAL
    bad = W.flake_c24h16()
    bad.S = bad.S.copy()
    bad.S[0, 1] += 1e-6
    with pytest.raises(T.TdError) as e:
        T.td_create(bad)
    assert e.value.status == T.TD_EINVAL
    o = T.td_default_options()
    o.dt = -0.1
    with pytest.raises(T.TdError) as e:
        T.td_create(s, o)
    assert e.value.status == T.TD_EINVAL
    occ = np.zeros(s.n_orb)
    occ[: s.n_elec // 2] = 2.0
    frac = occ.copy()
    frac[s.n_elec // 2 - 1 : s.n_elec // 2 + 1] = 1.0      # open shell: not a purification
    with pytest.raises(T.TdError) as e:
        T.td_create(s, occ=frac)
    assert e.value.status == T.TD_ENOTSUP
    holes = occ.copy()
    holes[0], holes[s.n_elec // 2] = 0.0, 2.0               # not aufbau
    with pytest.raises(T.TdError) as e:
        T.td_create(s, occ=holes)
    assert e.value.status == T.TD_ENOTSUP
    lib = T.load()
    sysd = T.TdSystem(n_atoms=1, n_orb=1, flags=2)          # unknown flag
    err = ctypes.create_string_buffer(256)
    ctx = ctypes.c_void_p()
    assert lib.td_create(ctypes.byref(sysd), ctypes.byref(o), ctypes.byref(ctx), err, 256) \
        == T.TD_EINVAL
    assert b"flags" in err.value
    assert lib.td_kick(None, 1e-3, None) == T.TD_EINVAL
    assert lib.td_step(None, 1, None) == T.TD_EINVAL


def test_no_device_is_an_error_not_a_fallback(T):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    with pytest.raises(T.TdError) as e:
        T.td_create(W.flake_c24h16())
    assert e.value.status == T.TD_EHIP
    with pytest.raises(T.TdError) as e:
        T.td_util_gemm(np.eye(4), np.eye(4))
    assert e.value.status == T.TD_EHIP


def test_batch_arguments_rejected_before_device(T):
    s = W.flake_c24h16()
    o = T.td_default_options()
    o.precision = T.TD_SPLIT_BF16
    with pytest.raises(T.TdError) as e:
        T.td_batch_create([s, s], o)
    assert e.value.status == T.TD_ENOTSUP
    with pytest.raises(T.TdError) as e:
        T.td_batch_create([s], flags=T.TD_BATCH_TILE_64 | T.TD_BATCH_TILE_128)
    assert e.value.status == T.TD_EINVAL
    with pytest.raises(T.TdError) as e:
        T.td_batch_create([s], flags=64)
    assert e.value.status == T.TD_EINVAL
    lib = T.load()
    assert lib.td_batch_step(None, 1, None) == T.TD_EINVAL
    assert lib.td_batch_kick(None, None, None) == T.TD_EINVAL
    assert T.load().td_batch_last_error(None) == b"null batch"


def test_spectrum_arguments_rejected_before_device(T):
    mu = np.zeros((2, 10))
    with pytest.raises(T.TdError) as e:
        T.td_spectrum(mu, [1e-3, 0.0], 0.2, [0.1, 0.2])
    assert e.value.status == T.TD_EINVAL
    with pytest.raises(T.TdError) as e:
        T.td_spectrum(np.zeros((2, 1)), 1e-3, 0.2, [0.1])
    assert e.value.status == T.TD_EINVAL
    with pytest.raises(T.TdError) as e:
        T.td_transient_absorption(np.zeros((3, 2, 10)), np.zeros((3, 2, 10)), 1e-3, 0.2, [0.1],
                                  ref_delay=5)
    assert e.value.status == T.TD_EINVAL


def test_ehrenfest_arguments_rejected_before_device(T):
    s = W.benzene()
    m = W.two_centre_model(s)
    o = T.td_default_options()
    o.precision = T.TD_SPLIT_BF16
    o.n_slices = 7
    with pytest.raises(T.TdError) as e:
        T.td_create_ehrenfest(s, m, None, o)
    assert e.value.status == T.TD_EINVAL
    o.precision = 9
    with pytest.raises(T.TdError) as e:
        T.td_create_ehrenfest(s, m, None, o)
    assert e.value.status == T.TD_EINVAL
    with pytest.raises(T.TdError) as e:
        T.td_create_ehrenfest(s, dict(m, decay=-1.0))
    assert e.value.status == T.TD_EINVAL
    with pytest.raises(T.TdError) as e:
        T.td_create_ehrenfest(s, dict(m, species=np.zeros(s.n_atoms, dtype=np.int32)))
    assert e.value.status == T.TD_EINVAL
    # the pair repulsion: negative, asymmetric, non-finite amplitudes; no decay
    bad = [np.array([[1.0, -0.1], [-0.1, 1.0]]), np.array([[1.0, 0.2], [0.3, 1.0]]),
           np.array([[1.0, np.inf], [np.inf, 1.0]])]
    for rep in bad:
        with pytest.raises(T.TdError) as e:
            T.td_create_ehrenfest(s, dict(m, rep_a=rep))
        assert e.value.status == T.TD_EINVAL and "rep" in str(e.value)
    with pytest.raises(T.TdError) as e:
        T.td_create_ehrenfest(s, dict(m, rep_decay=0.0))
    assert e.value.status == T.TD_EINVAL and "rep" in str(e.value)


class _PU:
    def __init__(self, mode, shell_offset, shell_u):
        self.mode, self.shell_offset, self.shell_u = mode, shell_offset, shell_u


def test_plus_u_arguments_rejected_before_device(T):
    s = W.flake_c24h16()
    off, u = W.atomic_shells(s, {("C", "p"): 0.2})

    def status(pu, **kw):
        with pytest.raises(T.TdError) as e:
            T.td_create(s, kw.get("opt"), plus_u=pu)
        return e.value.status

    # a shell spanning two atoms, a shell of 8 orbitals, negative or
    # non-finite U, offsets not ending at n_orb, an unknown mode
    assert list(off[:5]) == [0, 1, 4, 5, 8]      # atom 0: s 0, p 1-3; atom 1: s 4, p 5-7
    cross = np.array([0, 1, 3, 5] + off[4:].tolist(), dtype=np.int32)   # shell [3, 5)
    assert status(_PU("fll", cross, np.zeros(len(cross) - 1))) == T.TD_EINVAL
    big = np.array([0, 8, s.n_orb], dtype=np.int32)
    assert status(_PU("fll", big, np.zeros(2))) == T.TD_EINVAL
    neg = u.copy()
    neg[1] = -0.1
    assert status(_PU("fll", off, neg)) == T.TD_EINVAL
    nan = u.copy()
    nan[1] = np.nan
    assert status(_PU("psic", off, nan)) == T.TD_EINVAL
    assert status(_PU("fll", off[:-1], u[:-1])) == T.TD_EINVAL
    assert status(_PU(7, off, u)) == T.TD_EINVAL
    # not available in batches or with moving nuclei
    with pytest.raises(T.TdError) as e:
        T.td_batch_create([s, s], plus_us=[None, _PU("fll", off, u)])
    assert e.value.status == T.TD_ENOTSUP
    b = W.benzene()
    boff, bu = W.atomic_shells(b, {("C", "p"): 0.2})
    with pytest.raises(T.TdError) as e:
        T.td_create_ehrenfest(b, W.two_centre_model(b), plus_u=_PU("psic", boff, bu))
    assert e.value.status == T.TD_ENOTSUP


def test_missing_library_fails_loudly():
    """Without the built library the binding raises; nothing falls back to
    a CPU path (fresh interpreter, so no library is loaded yet)."""
    import subprocess
    import sys
    code = ("from paper_1912_03174_amd import tddftb as T\n"
            "T.load('/nonexistent/libtddftb.so')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=str(__import__('pathlib').Path(__file__).resolve().parents[1]),
                       timeout=120)
    assert r.returncode != 0
    assert "FileNotFoundError" in r.stderr and "is not built" in r.stderr


def test_noalloc_gemm_rejects_before_device(T):
    """Arguments and sizes beyond the fixed scratch array are rejected before
    any device call (the pointers are never touched)."""
    big = 4096
    with pytest.raises(T.TdError) as e:
        T.td_util_gemm_noalloc(big, big, big, 1, big, 1, big, 1, big,
                               precision=T.TD_SPLIT_BF16, n_slices=4)
    assert e.value.status == T.TD_EINVAL and "scratch" in str(e.value)
    with pytest.raises(T.TdError) as e:
        T.td_util_gemm_noalloc(2048, 2048, 2048, 1, 2048, 1, 2048, 1, 2048)
    assert e.value.status == T.TD_EINVAL and "scratch" in str(e.value)
    for args in ((0, 8, 8, 1, 8, 1, 8, 1, 8), (8, 8, 8, 0, 8, 1, 8, 1, 8),
                 (8, 8, 8, 1, 7, 1, 8, 1, 8), (8, 8, 8, 1, 8, 1, 7, 1, 8),
                 (8, 8, 8, 1, 8, 1, 8, 1, 7)):
        with pytest.raises(T.TdError) as e:
            T.td_util_gemm_noalloc(*args)
        assert e.value.status == T.TD_EINVAL
    with pytest.raises(T.TdError) as e:
        T.td_util_gemm_noalloc(8, 8, 8, 1, 8, 1, 8, 1, 8, precision=T.TD_SPLIT_BF16, n_slices=6)
    assert e.value.status == T.TD_EINVAL
