"""FP64 CPU oracle for profiled-distillation nucleon correlators (ctypes wrapper).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use this package. The HIP library and its
Python binding never import it; it imports nothing from them.

The arithmetic lives in ``oracle.c`` (plain double-precision loops written
from the definitions of the paper's Section 2.1); this file only marshals
numpy arrays. See ``oracle.c`` for the definitions and the readings used where
the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2); with sanitize, into
    liboracle_asan.so with AddressSanitizer and UndefinedBehaviorSanitizer (load it by
    naming it in ORACLE_LIBRARY, with gcc's libasan preloaded)."""
    path = os.path.join(_HERE, "liboracle_asan.so") if sanitize else _LIB_PATH
    if force or sanitize or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                 "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
        subprocess.check_call(["gcc"] + flags + ["-fopenmp", "-shared", "-fPIC", "-std=gnu11",
                                                 "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIBRARY")
        if not path:
            path = build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i = ctypes.c_int
        lib.oracle_profiles.argtypes = [i, i, P, i, P, P, P]
        lib.oracle_elementals.argtypes = [i, i, i, P, i, P, P]
        lib.oracle_correlator.argtypes = [i, i, i, i, P, P, P, P, P, P, P, P]
        lib.oracle_cg5.argtypes = [P]
        lib.oracle_elemental_entries.argtypes = [i, i, P, P, i, P, P]
        lib.oracle_elemental_entries.restype = ctypes.c_int
        for f in (lib.oracle_profiles, lib.oracle_elementals, lib.oracle_correlator):
            f.restype = ctypes.c_int
        lib.oracle_cg5.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def cg5() -> np.ndarray:
    out = np.zeros(16)
    _load().oracle_cg5(_ptr(out))
    return out.reshape(4, 4)


def profiles(evals: np.ndarray, prof: Sequence[Tuple[int, float]]) -> np.ndarray:
    """g [nprof][T][N] from eigenvalues [T][N] and (kind, sigma) descriptors."""
    ev = np.ascontiguousarray(evals, dtype=np.float64)
    T, N = ev.shape
    kinds = np.asarray([k for k, _ in prof], dtype=np.int32)
    sig = np.asarray([s for _, s in prof], dtype=np.float64)
    g = np.empty((len(prof), T, N))
    rc = _load().oracle_profiles(T, N, _ptr(ev), len(prof), _ptr(kinds), _ptr(sig), _ptr(g))
    if rc != 0:
        raise ValueError("oracle_profiles failed (%d)" % rc)
    return g


def elementals(L: int, evecs: np.ndarray, mom: np.ndarray) -> np.ndarray:
    """Phi [nt][nmom][N][N][N] (complex128) from eigenvectors [nt][N][V3][3]."""
    ev = np.ascontiguousarray(evecs, dtype=np.complex128)
    nt, N, V3, three = ev.shape
    assert three == 3 and V3 == L ** 3
    m = np.ascontiguousarray(mom, dtype=np.int32).reshape(-1, 3)
    out = np.empty((nt, m.shape[0], N, N, N), np.complex128)
    rc = _load().oracle_elementals(L, N, nt, _ptr(ev), m.shape[0], _ptr(m), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_elementals failed (%d)" % rc)
    return out


def elemental_entries(L: int, evecs_t: np.ndarray, mom: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Phi[p]_{ijk} for the rows (p, i, j, k) of idx, one timeslice [N][V3][3]."""
    ev = np.ascontiguousarray(evecs_t, dtype=np.complex128)
    N = ev.shape[0]
    m = np.ascontiguousarray(mom, dtype=np.int32).reshape(-1, 3)
    ix = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 4)
    out = np.empty(ix.shape[0], np.complex128)
    rc = _load().oracle_elemental_entries(L, N, _ptr(ev), _ptr(m), ix.shape[0], _ptr(ix), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_elemental_entries failed (%d)" % rc)
    return out


def correlator(phi_snk: np.ndarray, phi_src: np.ndarray, tau: np.ndarray,
               g_snk: np.ndarray, g_src: np.ndarray):
    """C, D, E [nmom][nt][nprof][nprof] (complex128).

    phi_snk [nt][nmom][N][N][N], phi_src [nmom][N][N][N], tau [nt][4N][4N],
    g_snk [nprof][nt][N] (sink profiles), g_src [nprof][N] (profiles at t0).
    """
    ps = np.ascontiguousarray(phi_snk, dtype=np.complex128)
    p0 = np.ascontiguousarray(phi_src, dtype=np.complex128)
    tu = np.ascontiguousarray(tau, dtype=np.complex128)
    gs = np.ascontiguousarray(g_snk, dtype=np.float64)
    g0 = np.ascontiguousarray(g_src, dtype=np.float64)
    nt, nmom, N = ps.shape[0], ps.shape[1], ps.shape[2]
    nprof = gs.shape[0]
    assert p0.shape == (nmom, N, N, N) and tu.shape == (nt, 4 * N, 4 * N)
    assert gs.shape == (nprof, nt, N) and g0.shape == (nprof, N)
    shape = (nmom, nt, nprof, nprof)
    c = np.empty(shape, np.complex128)
    d = np.empty(shape, np.complex128)
    e = np.empty(shape, np.complex128)
    rc = _load().oracle_correlator(N, nt, nmom, nprof, _ptr(ps), _ptr(p0), _ptr(tu), _ptr(gs),
                                   _ptr(g0), _ptr(c), _ptr(d), _ptr(e))
    if rc != 0:
        raise ValueError("oracle_correlator failed (%d)" % rc)
    return c, d, e


def run(L: int, evecs: np.ndarray, evals: np.ndarray, tau: np.ndarray, mom: np.ndarray,
        prof: Sequence[Tuple[int, float]], ts: Sequence[int] | None = None, t0: int = 0):
    """Elementals at the sink times ``ts`` (default all) and C_ab(t) there.

    evecs [T][N][V3][3], evals [T][N], tau [T][4N][4N] (tau(t, t0) for every t).
    Returns (phi [len(ts)][nmom][N^3...], corr [nmom][len(ts)][nprof][nprof]).
    """
    T = evecs.shape[0]
    ts = list(range(T)) if ts is None else list(ts)
    g = profiles(evals, prof)
    phi_t = elementals(L, evecs[ts], mom)
    phi_0 = elementals(L, evecs[[t0]], mom)[0]
    corr, _, _ = correlator(phi_t, phi_0, tau[ts], g[:, ts, :], g[:, t0, :])
    return phi_t, corr


def gevp(corr: np.ndarray, t0: int = 0):
    """Generalised eigenproblem C(t) v = lambda C(t0) v of the Hermitised matrices
    (C + C^H)/2 of one momentum's correlation matrix [T][nb][nb] (the GEVP of
    Section 2.1), in FP64 with scipy's generalised Hermitian eigensolver as the
    library step. Returns (lambda [T][nb] descending, vecs [T][nb][nb], columns
    normalised to v^H C(t0) v = 1)."""
    import scipy.linalg
    c = np.asarray(corr, dtype=np.complex128)
    h = 0.5 * (c + np.conj(np.swapaxes(c, -1, -2)))
    T, nb = c.shape[0], c.shape[1]
    lam = np.empty((T, nb))
    vecs = np.empty((T, nb, nb), np.complex128)
    for t in range(T):
        w, v = scipy.linalg.eigh(h[t], h[t0])
        order = np.argsort(-w, kind="stable")
        lam[t] = w[order]
        vecs[t] = v[:, order]
    return lam, vecs


def effective_mass(lam: np.ndarray) -> np.ndarray:
    """log(lambda(t) / lambda(t+1)) per eigenvalue (the effective mass of the GEVP)."""
    lam = np.asarray(lam, dtype=np.float64)
    return np.log(lam[:-1] / lam[1:])
