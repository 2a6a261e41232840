"""C ABI contract checks that need no GPU: symbols, status codes, host-side
argument validation and the host FP64 profile evaluation."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle
import paper_2609_37723_amd as nuc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def _declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(nuc_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = nuc.load()
    names = _declared_functions()
    assert "nuc_run" in names and "nuc_correlator" in names and "nuc_elementals" in names
    assert "nuc_server_submit" in names and "nuc_server_wait" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings_and_version():
    lib = nuc.load()
    for s in range(0, -9, -1):
        assert lib.nuc_status_string(s)
    assert lib.nuc_status_string(-99) == b"unknown status"
    assert b"gfx950" in lib.nuc_version()


def test_create_rejects_null_out():
    lib = nuc.load()
    assert lib.nuc_create(None, 0, 0) == nuc.NUC_ERR_INVALID
    assert b"NULL" in lib.nuc_last_error(None)


def test_compute_calls_reject_null_context():
    lib = nuc.load()
    g = nuc.Geom(4, 8, 8, 0)
    mom = np.zeros(3, np.int32)
    st = lib.nuc_elementals(None, ctypes.byref(g), ctypes.c_void_p(16), 1, mom.ctypes.data, 0,
                            ctypes.c_void_p(16), None)
    assert st == nuc.NUC_ERR_INVALID
    assert b"ctx" in lib.nuc_last_error(None)


@pytest.mark.parametrize("geom,msg", [
    ((0, 8, 8, 0), "L="), ((4, 0, 8, 0), "T="), ((4, 8, 2, 0), "nvec="), ((4, 8, 129, 0), "nvec="),
    ((4, 8, 8, 8), "t0="), ((4, 8, 8, -1), "t0=")])
def test_workspace_query_validates_geometry(geom, msg):
    with pytest.raises(nuc.NucError) as e:
        nuc.workspace_query(*geom[:3], nmom=1, nprof=1, t0=geom[3])
    assert e.value.status == nuc.NUC_ERR_INVALID and msg in str(e.value)


def test_workspace_query_sizes_scale():
    small = nuc.workspace_query(4, 8, 8, 1, 3)
    plain = nuc.workspace_query(16, 32, 32, 7, 4)
    assert 0 < small < plain
    with pytest.raises(nuc.NucError) as e:
        nuc.workspace_query(4, 8, 8, 1, 3, precision=7)
    assert e.value.status == nuc.NUC_ERR_INVALID


def test_profiles_eval_matches_oracle_profiles():
    g = np.random.default_rng(0)
    ev = np.sort(g.random((5, 12)), axis=1)
    prof = [(0, 0.2), (0, 0.5), (1, 0.0)]
    got = nuc.profiles_eval(2, 5, 12, ev, prof)
    ref = oracle.profiles(ev, prof)
    assert np.max(np.abs(got - ref)) <= 1e-15


def test_profiles_eval_one_and_explicit():
    vals = np.arange(5 * 4, dtype=np.float64).reshape(5, 4) / 7.0
    got = nuc.profiles_eval(2, 5, 4, None, [(nuc.PROF_ONE, 0.0), (nuc.PROF_EXPLICIT, 0.0, vals)])
    assert np.all(got[0] == 1.0)
    assert np.array_equal(got[1], vals)


@pytest.mark.parametrize("prof,msg", [([(0, 0.0)], "sigma"), ([(0, -1.0)], "sigma"), ([(9, 1.0)], "kind"),
                                      ([(0, float("nan"))], "sigma")])
def test_profiles_eval_rejects_bad_profiles(prof, msg):
    with pytest.raises(nuc.NucError) as e:
        nuc.profiles_eval(2, 5, 4, np.zeros((5, 4)), prof)
    assert msg in str(e.value)


def test_gaussian_profile_needs_eigenvalues():
    with pytest.raises(nuc.NucError) as e:
        nuc.profiles_eval(2, 5, 4, None, [(0, 0.3)])
    assert "evals" in str(e.value)


def test_no_cpu_fallback_in_binding():
    # the binding's compute entry points insist on device tensors
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        nuc.elementals(torch.zeros((2, 3, 8, 3), dtype=torch.complex64), 2, [(0, 0, 0)])


def test_kernel_name_table_matches_the_header():
    """Every kernel id of the header has a distinct name, and the binding's count matches."""
    text = open(os.path.join(ROOT, "include", "nucleon.h")).read()
    count = int(re.search(r"NUC_K_COUNT\s*=\s*(\d+)", text).group(1))
    assert count == nuc.KERNEL_COUNT
    lib = nuc.load()
    names = [lib.nuc_kernel_name(i).decode() for i in range(count)]
    assert len(set(names)) == count and "?" not in names
    assert lib.nuc_kernel_name(count) == b"?" and lib.nuc_kernel_name(-1) == b"?"
    ids = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"(NUC_K_[A-Z0-9_]+)\s*=\s*(\d+)", text))
    assert sorted(v for k, v in ids.items() if k != "NUC_K_COUNT") == list(range(count))


def test_twomeson_and_glueball_calls_reject_null_context():
    lib = nuc.load()
    g = nuc.Geom(4, 8, 8, 0)
    mom = np.zeros(3, np.int32)
    parr, keep = nuc._profiles([(1, 0.0)])
    w = np.ones(6)
    assert lib.nuc_twomeson_correlator(None, ctypes.byref(g), ctypes.c_void_p(16), None, 1, parr, w.ctypes.data, 1,
                                       mom.ctypes.data, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                       None) == nuc.NUC_ERR_INVALID
    assert lib.nuc_glueball_operators(None, 4, 2, 1, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                      None) == nuc.NUC_ERR_INVALID


def test_nucleon_spin_tensors_from_the_library():
    # nuc_spin_nucleon (host) against the oracle's independently built tensors, both parities
    import oracle.spin as osp
    for parity in (+1, -1):
        np.testing.assert_array_equal(nuc.nucleon_spin(parity), osp.nucleon_spin(parity))
    with pytest.raises(nuc.NucError):
        nuc.nucleon_spin(0)


def test_twomeson_weights_from_the_library():
    rng = np.random.default_rng(5)
    v = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    U = rng.standard_normal((9, 4)) + 1j * rng.standard_normal((9, 4))
    np.testing.assert_array_equal(nuc.twomeson_weights(v), np.conj(v))
    np.testing.assert_allclose(nuc.twomeson_weights(v, U), np.conj(U @ v), rtol=1e-15, atol=1e-15)
    with pytest.raises(nuc.NucError):
        nuc.twomeson_weights(v, U[:2])
