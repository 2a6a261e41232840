"""Seeded synthetic inputs for the profiled-distillation nucleon correlator.

This module only draws random numbers and lays them out. It holds none of the
method's arithmetic (no elementals, no profile evaluation, no contraction), so
it can feed both the FP64 CPU oracle and the HIP library without either one
depending on the other.

Every stream is ``numpy.random.Generator(PCG64(SeedSequence([0x37723, cfg_id,
conf_id, field, t])))`` with ``field`` 0 = eigenvectors, 1 = eigenvalues,
2 = perambulators, 3 = job stream, 4 = gauge links, 5 = stand-in meson elementals. Complex Gaussians have Re and Im iid
N(0, 1/2), so E|z|^2 = 1.

Layouts (all row-major, complex interleaved):

* eigenvectors  ``[T][N][V3][3]``: vector i, site x = x0 + L*(x1 + L*x2),
  colour a innermost; the vectors of one timeslice are orthonormal under the
  Hermitian product over (x, a).
* eigenvalues   ``[T][N]`` ascending, uniform in [0, 1).
* perambulators ``[T][4N][4N]``: tau(t, t0) with row/column index
  ``spin * N + i`` (sink row, source column).
* momenta       ``[nmom][3]`` integers in units of 2*pi/L.
* profiles      a list of ``(kind, sigma)`` descriptors; kind 0 is a Gaussian
  in the Laplacian eigenvalue, kind 1 is linear in the distillation index.

All floating-point arrays are returned in complex128/float64 but already
rounded through complex64, so the oracle (which works in FP64) and the GPU
(which is fed complex64) see exactly the same numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

SEED_ROOT = 0x37723
FIELD_EVECS, FIELD_EVALS, FIELD_TAU, FIELD_JOBS = 0, 1, 2, 3

PROF_GAUSS = 0
PROF_LINEAR = 1

# Momenta of the 7-momentum set, units of 2*pi/L.
MOMENTA_7 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def rng(cfg_id: int, conf_id: int, field: int, t: int) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg_id, conf_id, field, t])))


@dataclasses.dataclass
class Config:
    name: str
    cfg_id: int
    L: int
    T: int
    nvec: int
    momenta: List[Tuple[int, int, int]]
    profiles: List[Tuple[int, float]]
    tau_kind: str = "gauss"          # gauss | gauss_decay | lognormal | identity
    t0: int = 0

    @property
    def V3(self) -> int:
        return self.L ** 3

    @property
    def nmom(self) -> int:
        return len(self.momenta)

    @property
    def nprof(self) -> int:
        return len(self.profiles)


def tiny() -> Config:
    """4^3 x 8, N=8, p=0, three Gaussian profiles, plain complex Gaussian tau."""
    return Config("tiny", 0, 4, 8, 8, [(0, 0, 0)],
                  [(PROF_GAUSS, 0.2), (PROF_GAUSS, 0.5), (PROF_GAUSS, 1.0)], "gauss")


def plain() -> Config:
    """16^3 x 32, N=32, 7 momenta, 3 Gaussians + linear, tau decaying as exp(-t/2)."""
    return Config("plain", 1, 16, 32, 32, list(MOMENTA_7),
                  [(PROF_GAUSS, 0.2), (PROF_GAUSS, 0.5), (PROF_GAUSS, 1.0), (PROF_LINEAR, 0.0)],
                  "gauss_decay")


def prec() -> Config:
    """24^3 x 48, N=64, 3 momenta, 5 Gaussians + linear, log-normal tau (sigma=2)."""
    return Config("prec", 2, 24, 48, 64, [(0, 0, 0), (1, 0, 0), (1, 1, 0)],
                  [(PROF_GAUSS, s) for s in (0.1, 0.2, 0.35, 0.5, 1.0)] + [(PROF_LINEAR, 0.0)],
                  "lognormal")


def custom(name: str, L: int, T: int, nvec: int, momenta: Sequence[Tuple[int, int, int]],
           profiles: Sequence[Tuple[int, float]], tau_kind: str = "gauss", cfg_id: int = 9) -> Config:
    return Config(name, cfg_id, L, T, nvec, [tuple(m) for m in momenta], list(profiles), tau_kind)


def _round_c64(z: np.ndarray) -> np.ndarray:
    return z.astype(np.complex64).astype(np.complex128)


def _complex_gauss(g: np.random.Generator, shape) -> np.ndarray:
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) * math.sqrt(0.5)


def orthonormalise(m: np.ndarray) -> np.ndarray:
    """Rows of ``m`` ([N][K]) made orthonormal in order (Gram-Schmidt result).

    Computed as a QR factorisation of the columns with the diagonal of R made
    real and positive, which is the same set of vectors classical Gram-Schmidt
    in the order 0..N-1 produces in exact arithmetic.
    """
    q, r = np.linalg.qr(m.T)
    d = np.diag(r)
    ph = d / np.abs(d)
    return (q * ph[None, :]).T


def eigenvectors(cfg: Config, conf_id: int = 0, ts: Sequence[int] | None = None) -> np.ndarray:
    """Complex [len(ts)][N][V3][3], orthonormal per timeslice, rounded through c64."""
    ts = range(cfg.T) if ts is None else ts
    out = np.empty((len(ts), cfg.nvec, cfg.V3, 3), np.complex128)
    for n, t in enumerate(ts):
        g = rng(cfg.cfg_id, conf_id, FIELD_EVECS, t)
        m = _complex_gauss(g, (cfg.nvec, 3 * cfg.V3))
        out[n] = orthonormalise(m).reshape(cfg.nvec, cfg.V3, 3)
    return _round_c64(out)


def eigenvalues(cfg: Config, conf_id: int = 0) -> np.ndarray:
    """float64 [T][N], uniform in [0,1), ascending per timeslice."""
    out = np.empty((cfg.T, cfg.nvec))
    for t in range(cfg.T):
        out[t] = np.sort(rng(cfg.cfg_id, conf_id, FIELD_EVALS, t).random(cfg.nvec))
    return out


def perambulators(cfg: Config, conf_id: int = 0, ts: Sequence[int] | None = None) -> np.ndarray:
    """Complex [len(ts)][4N][4N] tau(t, t0), rounded through c64."""
    ts = range(cfg.T) if ts is None else ts
    n4 = 4 * cfg.nvec
    out = np.empty((len(ts), n4, n4), np.complex128)
    for n, t in enumerate(ts):
        if cfg.tau_kind == "identity":
            out[n] = np.eye(n4)
            continue
        g = rng(cfg.cfg_id, conf_id, FIELD_TAU, t)
        if cfg.tau_kind == "lognormal":
            zeta = g.standard_normal((n4, n4))
            phase = g.random((n4, n4)) * 2.0 * math.pi
            out[n] = np.exp(2.0 * zeta) * np.exp(1j * phase)
        else:
            out[n] = _complex_gauss(g, (n4, n4))
            if cfg.tau_kind == "gauss_decay":
                out[n] *= math.exp(-0.5 * t)
    return _round_c64(out)


def momenta(cfg: Config) -> np.ndarray:
    return np.asarray(cfg.momenta, dtype=np.int32).reshape(-1, 3)


@dataclasses.dataclass
class Inputs:
    cfg: Config
    evecs: np.ndarray
    evals: np.ndarray
    tau: np.ndarray
    mom: np.ndarray


def make_inputs(cfg: Config, conf_id: int = 0) -> Inputs:
    return Inputs(cfg, eigenvectors(cfg, conf_id), eigenvalues(cfg, conf_id),
                  perambulators(cfg, conf_id), momenta(cfg))


def random_su3(g: np.random.Generator, nsites: int) -> np.ndarray:
    """[nsites][3][3] Haar-like SU(3) matrices (QR with phase fix, det divided out)."""
    z = _complex_gauss(g, (nsites, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


FIELD_LINKS = 4


def gauge_links(cfg: Config, conf_id: int = 0) -> np.ndarray:
    """Spatial gauge links U_d(x, t), d = 0, 1, 2 (directions x0, x1, x2), as complex
    [T][V3][3][3][3] (direction, colour row, colour column): Haar-like random SU(3)
    per link, rounded through c64. Stream field 4."""
    out = np.empty((cfg.T, cfg.V3, 3, 3, 3), np.complex128)
    for t in range(cfg.T):
        g = rng(cfg.cfg_id, conf_id, FIELD_LINKS, t)
        out[t] = random_su3(g, cfg.V3 * 3).reshape(cfg.V3, 3, 3, 3)
    return _round_c64(out)


# ------------------------------------------------------------------ large inputs on the GPU
def torch_inputs(cfg: Config, conf_id: int = 0, device: str = "cuda:0", nvec: int | None = None):
    """Seeded inputs generated directly in device memory (for workloads too large
    to build on the host): complex64 eigenvectors [T][N][V3][3] orthonormalised per
    timeslice (Cholesky QR in complex128: the rows of L^-1 M for M = L Q, i.e.
    the Gram-Schmidt vectors), complex64 perambulators [T][4N][4N] with the
    config's tau recipe, and host eigenvalues [T][N]. The streams are torch
    generators seeded from the same SeedSequence keys as the numpy generators,
    so the values differ from eigenvectors()/perambulators() but are
    reproducible. nvec overrides cfg.nvec (store at a larger N and use prefixes).
    """
    import torch
    N = cfg.nvec if nvec is None else nvec
    V3, T = cfg.V3, cfg.T
    ev = torch.empty((T, N, V3, 3), dtype=torch.complex64, device=device)
    tau = torch.empty((T, 4 * N, 4 * N), dtype=torch.complex64, device=device)
    gen = torch.Generator(device=device)
    for t in range(T):
        seed = int(np.random.SeedSequence([SEED_ROOT, cfg.cfg_id, conf_id, FIELD_EVECS, t]).generate_state(1)[0])
        gen.manual_seed(seed)
        m = torch.complex(torch.randn((N, 3 * V3), generator=gen, device=device, dtype=torch.float64),
                          torch.randn((N, 3 * V3), generator=gen, device=device, dtype=torch.float64))
        m *= math.sqrt(0.5)
        gram = m @ m.conj().transpose(0, 1)
        low = torch.linalg.cholesky(gram)
        q = torch.linalg.inv(low) @ m
        ev[t] = q.reshape(N, V3, 3).to(torch.complex64)
        seed = int(np.random.SeedSequence([SEED_ROOT, cfg.cfg_id, conf_id, FIELD_TAU, t]).generate_state(1)[0])
        gen.manual_seed(seed)
        if cfg.tau_kind == "identity":
            tau[t] = torch.eye(4 * N, dtype=torch.complex64, device=device)
            continue
        if cfg.tau_kind == "lognormal":
            zeta = torch.randn((4 * N, 4 * N), generator=gen, device=device, dtype=torch.float64)
            ph = torch.rand((4 * N, 4 * N), generator=gen, device=device, dtype=torch.float64) * 2 * math.pi
            z = torch.polar(torch.exp(2.0 * zeta), ph)
        else:
            z = torch.complex(torch.randn((4 * N, 4 * N), generator=gen, device=device, dtype=torch.float64),
                              torch.randn((4 * N, 4 * N), generator=gen, device=device, dtype=torch.float64))
            z *= math.sqrt(0.5)
            if cfg.tau_kind == "gauss_decay":
                z *= math.exp(-0.5 * t)
        tau[t] = z.to(torch.complex64)
    evals = np.empty((T, N))
    for t in range(T):
        evals[t] = np.sort(rng(cfg.cfg_id, conf_id, FIELD_EVALS, t).random(N))
    return ev, tau, evals


def torch_links(cfg: Config, nconf: int = 1, device: str = "cuda:0"):
    """Seeded random SU(3) links generated in device memory, complex64
    [nconf][T][V3][3][3][3]: per link, rows u1, u2 from Gram-Schmidt of two complex
    Gaussian vectors and u3 = conj(u1 x u2), an SU(3) matrix (det exactly 1 in exact
    arithmetic). A torch generator per (configuration, timeslice) seeded from the links
    stream's SeedSequence key; values differ from gauge_links() but are reproducible."""
    import torch
    V3, T = cfg.V3, cfg.T
    out = torch.empty((nconf, T, V3, 3, 3, 3), dtype=torch.complex64, device=device)
    gen = torch.Generator(device=device)
    for c in range(nconf):
        for t in range(T):
            seed = int(np.random.SeedSequence([SEED_ROOT, cfg.cfg_id, c, FIELD_LINKS, t]).generate_state(1)[0])
            gen.manual_seed(seed)
            z = torch.complex(torch.randn((V3 * 3, 2, 3), generator=gen, device=device, dtype=torch.float64),
                              torch.randn((V3 * 3, 2, 3), generator=gen, device=device, dtype=torch.float64))
            u1 = z[:, 0] / torch.linalg.vector_norm(z[:, 0], dim=1, keepdim=True)
            b = z[:, 1] - (u1.conj() * z[:, 1]).sum(dim=1, keepdim=True) * u1
            u2 = b / torch.linalg.vector_norm(b, dim=1, keepdim=True)
            u3 = torch.stack([u1[:, 1] * u2[:, 2] - u1[:, 2] * u2[:, 1],
                              u1[:, 2] * u2[:, 0] - u1[:, 0] * u2[:, 2],
                              u1[:, 0] * u2[:, 1] - u1[:, 1] * u2[:, 0]], dim=1).conj()
            out[c, t] = torch.stack([u1, u2, u3], dim=1).reshape(V3, 3, 3, 3).to(torch.complex64)
    return out


FIELD_MESON_PHI = 5


def meson_elementals_like(cfg: Config, nmom: int, conf_id: int = 0) -> np.ndarray:
    """Complex Gaussian stand-ins for meson elementals, [T][nmom][7][N][N] with
    E|z|^2 = 1, rounded through c64 (for sizes where elementals from vectors and links
    are too slow for the oracle). Stream field 5, one stream per timeslice."""
    out = np.empty((cfg.T, nmom, 7, cfg.nvec, cfg.nvec), np.complex128)
    for t in range(cfg.T):
        out[t] = _complex_gauss(rng(cfg.cfg_id, conf_id, FIELD_MESON_PHI, t), out.shape[1:])
    return _round_c64(out)
