"""Python binding of the MI355X nucleon-correlator library (libnucleon.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/nucleon.h``. PyTorch supplies
device memory (``Tensor.data_ptr()``) and the HIP stream
(``torch.cuda.current_stream().cuda_stream``). There is no CPU fallback: if the
library is not built, or no GPU is visible, calls raise.

Functions mirror the ABI names without the ``nuc_`` prefix:

* :func:`elementals` -- baryon elementals Phi[t][p][i][j][k] (c64)
* :func:`correlator` -- C_ab(t) (c128 [nmom][T][nprof][nprof]) from elementals
* :func:`run`        -- both in one call
* :func:`profiles_eval` -- host FP64 profile values (no GPU needed)
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NUC_LIBRARY may name another build of the same library (the host-sanitizer builds of
# build.py); by default the in-tree libnucleon.so.
LIB_PATH = os.environ.get("NUC_LIBRARY") or os.path.join(_HERE, "libnucleon.so")

(NUC_OK, NUC_ERR_INVALID, NUC_ERR_NOMEM, NUC_ERR_DEVICE, NUC_ERR_UNSUPPORTED, NUC_ERR_BUSY, NUC_ERR_INTERNAL,
 NUC_ERR_TIMEOUT, NUC_ERR_CANCELLED) = (0, -1, -2, -3, -4, -5, -6, -7, -8)
EXEC_HIP, EXEC_FAKE = 0, 1
FP32, BF16X3, FP16X3, FP64 = 0, 1, 2, 3
PROF_GAUSS, PROF_LINEAR, PROF_ONE, PROF_EXPLICIT = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3, "fp64": FP64}
KERNEL_COUNT = 23


class NucError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("T", ctypes.c_int), ("nvec", ctypes.c_int), ("t0", ctypes.c_int)]


class Spin(ctypes.Structure):
    _fields_ = [("nrow", ctypes.c_int), ("snk", ctypes.c_void_p), ("src", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("sigma", ctypes.c_double), ("values", ctypes.c_void_p)]


class Job(ctypes.Structure):
    _fields_ = [("geom", Geom), ("evecs", ctypes.c_void_p), ("evals", ctypes.c_void_p), ("nprof", ctypes.c_int),
                ("prof", ctypes.c_void_p), ("nmom", ctypes.c_int), ("mom", ctypes.c_void_p),
                ("peramb", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("corr", ctypes.c_void_p),
                ("ld_nvec", ctypes.c_int)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("executor", ctypes.c_int), ("device", ctypes.c_int), ("hbm_budget", ctypes.c_size_t),
                ("job_arena", ctypes.c_size_t), ("slot_workspace", ctypes.c_size_t), ("slots", ctypes.c_int),
                ("max_active", ctypes.c_int), ("quantum_flops", ctypes.c_double), ("start_paused", ctypes.c_int),
                ("fake_flops_per_s", ctypes.c_double), ("fake_fixed_s", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("conf_id", ctypes.c_uint64), ("nvec", ctypes.c_int), ("nmom", ctypes.c_int),
                ("mom", ctypes.c_void_p), ("nprof", ctypes.c_int), ("prof", ctypes.c_void_p),
                ("precision", ctypes.c_int)]


class JobInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double), ("flops", ctypes.c_double),
                ("iterations", ctypes.c_int)]


class ServerMetrics(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("cancelled", ctypes.c_longlong), ("iterations", ctypes.c_longlong), ("queued", ctypes.c_int),
                ("active", ctypes.c_int), ("max_outstanding", ctypes.c_int), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("window_s", ctypes.c_double), ("jobs_per_s", ctypes.c_double), ("flops_per_s", ctypes.c_double),
                ("bytes_resident", ctypes.c_size_t), ("bytes_arena_used", ctypes.c_size_t),
                ("bytes_arena_peak", ctypes.c_size_t), ("bytes_arena", ctypes.c_size_t),
                ("bytes_total", ctypes.c_size_t)]


_lib = None


def load():
    """Load libnucleon.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnucleon.so is not built; run paper_2609_37723_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "nuc_create": ([ctypes.POINTER(P), I, S], st),
        "nuc_destroy": ([P], st),
        "nuc_status_string": ([I], ctypes.c_char_p),
        "nuc_last_error": ([P], ctypes.c_char_p),
        "nuc_version": ([], ctypes.c_char_p),
        "nuc_profiles_eval": ([ctypes.POINTER(Geom), P, I, P, P], st),
        "nuc_workspace_query": ([ctypes.POINTER(Geom), I, I, I, ctypes.POINTER(S)], st),
        "nuc_elementals": ([P, ctypes.POINTER(Geom), P, I, P, I, P, P], st),
        "nuc_correlator": ([P, ctypes.POINTER(Geom), P, P, I, P, I, P, I, P, P], st),
        "nuc_correlator_noalloc": ([P, ctypes.POINTER(Geom), P, P, I, P, I, P, I, P, P], st),
        "nuc_run": ([P, ctypes.POINTER(Geom), P, P, I, P, I, P, P, I, P, P, P], st),
        "nuc_batch_run": ([P, I, P, I, P], st),
        "nuc_batch_graph": ([P, I, P, I, ctypes.POINTER(P)], st),
        "nuc_graph_launch": ([P, P], st),
        "nuc_autotune": ([P, P, I, P, P], st),
        "nuc_graph_destroy": ([P], st),
        "nuc_timing_enable": ([P, I], st),
        "nuc_timing_read": ([P, P, P], st),
        "nuc_kernel_name": ([I], ctypes.c_char_p),
        "nuc_gevp": ([P, I, I, I, P, P], st),
        "nuc_effective_mass": ([P, I, I, P], st),
        "nuc_meson_elementals": ([P, ctypes.POINTER(Geom), P, P, I, P, P, P], st),
        "nuc_meson_correlator": ([P, ctypes.POINTER(Geom), P, P, I, P, I, P, P, P], st),
        "nuc_meson_run": ([P, ctypes.POINTER(Geom), P, P, P, I, P, I, P, P, P, P, P], st),
        "nuc_svd_prune": ([P, I, I, I, I, P, P], st),
        "nuc_glueball_operators": ([P, I, I, I, P, P, P], st),
        "nuc_correlator_spin": ([P, ctypes.POINTER(Geom), P, P, I, P, I, P, ctypes.POINTER(Spin), P, P], st),
        "nuc_spin_nucleon": ([I, P], st),
        "nuc_twomeson_weights": ([P, I, P, I, P], st),
        "nuc_glueball_correlator": ([P, I, I, P], st),
        "nuc_twomeson_correlator": ([P, ctypes.POINTER(Geom), P, P, I, P, P, I, P, P, P, P], st),
        "nuc_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(P)], st),
        "nuc_server_destroy": ([P], st),
        "nuc_server_register": ([P, ctypes.c_uint64, ctypes.POINTER(Geom), P, P, P], st),
        "nuc_server_unregister": ([P, ctypes.c_uint64], st),
        "nuc_server_submit": ([P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], st),
        "nuc_server_wait": ([P, ctypes.c_uint64, I, P, ctypes.POINTER(JobInfo)], st),
        "nuc_server_cancel": ([P, ctypes.c_uint64], st),
        "nuc_server_resume": ([P], st),
        "nuc_server_stats": ([P, ctypes.POINTER(ServerMetrics)], st),
        "nuc_server_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status != NUC_OK:
        lib = load()
        msg = lib.nuc_last_error(ctx).decode() if ctx is not None else lib.nuc_last_error(None).decode()
        raise NucError(status, msg or lib.nuc_status_string(status).decode())


def version() -> str:
    return load().nuc_version().decode()


class Context:
    """Owns a library context (workspace, events) on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.nuc_create(ctypes.byref(h), device, hbm_budget_bytes))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def timing_enable(self, on: bool = True):
        """Bracket every kernel launch of this context with HIP events (see nuc_timing_read)."""
        _check(load().nuc_timing_enable(self._h, 1 if on else 0), self._h)

    def timing_read(self):
        """{kernel name: (summed ms, launches)} since enabling or the last read."""
        lib = load()
        ms = np.zeros(KERNEL_COUNT)
        n = np.zeros(KERNEL_COUNT, np.int32)
        _check(lib.nuc_timing_read(self._h, ms.ctypes.data, n.ctypes.data), self._h)
        return {lib.nuc_kernel_name(k).decode(): (float(ms[k]), int(n[k])) for k in range(KERNEL_COUNT)}

    def close(self):
        if self._h:
            load().nuc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def _geom(L: int, T: int, nvec: int, t0: int = 0) -> Geom:
    return Geom(L, T, nvec, t0)


def _profiles(prof: Sequence[Tuple[int, float]]):
    arr = (Profile * len(prof))()
    keep = []
    for n, item in enumerate(prof):
        kind, sigma = int(item[0]), float(item[1])
        arr[n].kind = kind
        arr[n].sigma = sigma
        arr[n].values = None
        if kind == PROF_EXPLICIT:
            vals = np.ascontiguousarray(item[2], dtype=np.float64)
            keep.append(vals)
            arr[n].values = vals.ctypes.data
    return arr, keep


def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _prec(precision) -> int:
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def profiles_eval(L: int, T: int, nvec: int, evals: np.ndarray | None, prof, t0: int = 0) -> np.ndarray:
    """Host FP64 profile values g[nprof][T][nvec] (no GPU involved)."""
    lib = load()
    g = _geom(L, T, nvec, t0)
    parr, keep = _profiles(prof)
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    out = np.empty((len(prof), T, nvec))
    _check(lib.nuc_profiles_eval(ctypes.byref(g), None if ev is None else ev.ctypes.data, len(prof), parr,
                                 out.ctypes.data))
    return out


def workspace_query(L: int, T: int, nvec: int, nmom: int, nprof: int, precision="fp32", t0: int = 0) -> int:
    lib = load()
    g = _geom(L, T, nvec, t0)
    n = ctypes.c_size_t()
    _check(lib.nuc_workspace_query(ctypes.byref(g), nmom, nprof, _prec(precision), ctypes.byref(n)))
    return n.value


def _require_device_tensor(x, dtype, shape, name):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if x.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, x.dtype))
    if tuple(x.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(x.shape)))
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def elementals(evecs, L: int, mom, precision="fp32", out=None, ctx: Context | None = None, stream=None):
    """Phi [T][nmom][N][N][N] complex64 from eigenvectors [T][N][L^3][3] complex64 (device)."""
    import torch
    T, N = evecs.shape[0], evecs.shape[1]
    _require_device_tensor(evecs, torch.complex64, (T, N, L ** 3, 3), "evecs")
    ctx = ctx or default_context(evecs.device.index or 0)
    m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    nmom = m.shape[0]
    if out is None:
        out = torch.empty((T, nmom, N, N, N), dtype=torch.complex64, device=evecs.device)
    _require_device_tensor(out, torch.complex64, (T, nmom, N, N, N), "out")
    g = _geom(L, T, N, 0)
    _check(load().nuc_elementals(ctx.handle, ctypes.byref(g), ctypes.c_void_p(evecs.data_ptr()), nmom,
                                 m.ctypes.data, _prec(precision), ctypes.c_void_p(out.data_ptr()),
                                 _stream_ptr(stream)), ctx.handle)
    return out


def correlator(phi, evals, prof, tau, L: int, t0: int = 0, precision="fp32", out=None,
               ctx: Context | None = None, stream=None):
    """C [nmom][T][nprof][nprof] complex128 from elementals (device), eigenvalues (host), tau (device)."""
    import torch
    T, nmom, N = phi.shape[0], phi.shape[1], phi.shape[2]
    _require_device_tensor(phi, torch.complex64, (T, nmom, N, N, N), "phi")
    _require_device_tensor(tau, torch.complex64, (T, 4 * N, 4 * N), "tau")
    ctx = ctx or default_context(phi.device.index or 0)
    nprof = len(prof)
    if out is None:
        out = torch.empty((nmom, T, nprof, nprof), dtype=torch.complex128, device=phi.device)
    _require_device_tensor(out, torch.complex128, (nmom, T, nprof, nprof), "out")
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    parr, keep = _profiles(prof)
    g = _geom(L, T, N, t0)
    _check(load().nuc_correlator(ctx.handle, ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()),
                                 None if ev is None else ev.ctypes.data, nprof, parr, nmom,
                                 ctypes.c_void_p(tau.data_ptr()), _prec(precision),
                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return out


def correlator_noalloc(phi, evals, prof, tau, L: int, out, t0: int = 0, precision="fp32",
                       ctx: Context | None = None, stream=None):
    """nuc_correlator_noalloc: as :func:`correlator` into the caller's ``out``
    (c128 [nmom][T][nprof][nprof] on the device); the library allocates nothing."""
    import torch
    T, nmom, N = phi.shape[0], phi.shape[1], phi.shape[2]
    _require_device_tensor(phi, torch.complex64, (T, nmom, N, N, N), "phi")
    _require_device_tensor(tau, torch.complex64, (T, 4 * N, 4 * N), "tau")
    nprof = len(prof)
    _require_device_tensor(out, torch.complex128, (nmom, T, nprof, nprof), "out")
    ctx = ctx or default_context(phi.device.index or 0)
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    parr, keep = _profiles(prof)
    g = _geom(L, T, N, t0)
    _check(load().nuc_correlator_noalloc(ctx.handle, ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()),
                                         None if ev is None else ev.ctypes.data, nprof, parr, nmom,
                                         ctypes.c_void_p(tau.data_ptr()), _prec(precision),
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return out


def run(evecs, evals, prof, mom, tau, L: int, t0: int = 0, precision="fp32", phi_out=None, out=None,
        return_phi: bool = False, ctx: Context | None = None, stream=None):
    """Elementals then C_ab(t) in one library call; returns corr (and phi if asked)."""
    import torch
    T, N = evecs.shape[0], evecs.shape[1]
    _require_device_tensor(evecs, torch.complex64, (T, N, L ** 3, 3), "evecs")
    _require_device_tensor(tau, torch.complex64, (T, 4 * N, 4 * N), "tau")
    ctx = ctx or default_context(evecs.device.index or 0)
    m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    nmom, nprof = m.shape[0], len(prof)
    if return_phi and phi_out is None:
        phi_out = torch.empty((T, nmom, N, N, N), dtype=torch.complex64, device=evecs.device)
    if phi_out is not None:
        _require_device_tensor(phi_out, torch.complex64, (T, nmom, N, N, N), "phi_out")
    if out is None:
        out = torch.empty((nmom, T, nprof, nprof), dtype=torch.complex128, device=evecs.device)
    _require_device_tensor(out, torch.complex128, (nmom, T, nprof, nprof), "out")
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    parr, keep = _profiles(prof)
    g = _geom(L, T, N, t0)
    _check(load().nuc_run(ctx.handle, ctypes.byref(g), ctypes.c_void_p(evecs.data_ptr()),
                          None if ev is None else ev.ctypes.data, nprof, parr, nmom, m.ctypes.data,
                          ctypes.c_void_p(tau.data_ptr()), _prec(precision),
                          None if phi_out is None else ctypes.c_void_p(phi_out.data_ptr()),
                          ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return (out, phi_out) if return_phi else out


# --------------------------------------------------------------------- batching
class BatchJob:
    """One job of a batch: device tensors plus host eigenvalues, profiles and momenta.

    ``corr`` (and ``phi`` if given) are filled by :func:`batch_run`.
    """

    def __init__(self, evecs, evals, prof, mom, tau, L: int, t0: int = 0, phi=None, corr=None, nvec=None):
        """``nvec`` < evecs.shape[1] uses the first nvec vectors of inputs stored at a larger nvec."""
        import torch
        T, ld = evecs.shape[0], evecs.shape[1]
        N = ld if nvec is None else int(nvec)
        _require_device_tensor(evecs, torch.complex64, (T, ld, L ** 3, 3), "evecs")
        _require_device_tensor(tau, torch.complex64, (T, 4 * ld, 4 * ld), "tau")
        self.evecs, self.tau, self.L, self.t0, self.nvec, self.ld = evecs, tau, L, t0, N, ld
        if evals is not None:
            evals = np.asarray(evals)[:, :N]
        self.evals = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
        self.prof = list(prof)
        self.mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
        nmom, nprof = self.mom.shape[0], len(self.prof)
        if phi is not None:
            _require_device_tensor(phi, torch.complex64, (T, nmom, N, N, N), "phi")
        self.phi = phi
        if corr is None:
            corr = torch.empty((nmom, T, nprof, nprof), dtype=torch.complex128, device=evecs.device)
        _require_device_tensor(corr, torch.complex128, (nmom, T, nprof, nprof), "corr")
        self.corr = corr

    def _fill(self, j: "Job", keep: list):
        T, N = self.evecs.shape[0], self.nvec
        parr, k2 = _profiles(self.prof)
        keep.extend([parr, k2, self.evals, self.mom])
        j.geom = Geom(self.L, T, N, self.t0)
        j.evecs = self.evecs.data_ptr()
        j.evals = None if self.evals is None else self.evals.ctypes.data
        j.nprof = len(self.prof)
        j.prof = ctypes.cast(parr, ctypes.c_void_p)
        j.nmom = self.mom.shape[0]
        j.mom = self.mom.ctypes.data
        j.peramb = self.tau.data_ptr()
        j.phi = None if self.phi is None else self.phi.data_ptr()
        j.corr = self.corr.data_ptr()
        j.ld_nvec = 0 if self.ld == N else self.ld


def _job_array(jobs):
    arr = (Job * len(jobs))()
    keep = []
    for n, jb in enumerate(jobs):
        jb._fill(arr[n], keep)
    return arr, keep


def batch_run(jobs, precision="fp32", ctx: Context | None = None, stream=None):
    """Run every job of the batch in shared launches; results land in each job's ``corr``."""
    ctx = ctx or default_context(jobs[0].evecs.device.index or 0)
    arr, keep = _job_array(jobs)
    _check(load().nuc_batch_run(ctx.handle, len(jobs), arr, _prec(precision), _stream_ptr(stream)), ctx.handle)
    return [jb.corr for jb in jobs]


def autotune(job: "BatchJob", precision="fp32", ctx: Context | None = None, stream=None):
    """Tune the launch shapes for this job's shape on ctx; returns (momenta per wave, step-1 target)."""
    ctx = ctx or default_context(job.evecs.device.index or 0)
    arr, keep = _job_array([job])
    best = np.zeros(2, np.int32)
    _check(load().nuc_autotune(ctx.handle, arr, _prec(precision), _stream_ptr(stream), best.ctypes.data),
           ctx.handle)
    return int(best[0]), int(best[1])


class BatchGraph:
    """A captured batch (HIP graph) that can be replayed with :meth:`launch`."""

    def __init__(self, jobs, precision="fp32", ctx: Context | None = None):
        self.ctx = ctx or default_context(jobs[0].evecs.device.index or 0)
        self.jobs = jobs
        arr, keep = _job_array(jobs)
        h = ctypes.c_void_p()
        _check(load().nuc_batch_graph(self.ctx.handle, len(jobs), arr, _prec(precision), ctypes.byref(h)),
               self.ctx.handle)
        self._h = h

    def launch(self, stream=None):
        _check(load().nuc_graph_launch(self._h, _stream_ptr(stream)), self.ctx.handle)

    def close(self):
        if getattr(self, "_h", None):
            load().nuc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------- analysis
def gevp(corr, t0: int = 0, vectors: bool = True):
    """Host FP64 GEVP C(t) v = lambda C(t0) v of one momentum's C [T][nb][nb]
    (complex128, host or device tensor / array). Returns (lambda [T][nb] descending,
    vecs [T][nb][nb] with v_n in column n, or None)."""
    c = corr.cpu().numpy() if hasattr(corr, "cpu") else np.asarray(corr)
    c = np.ascontiguousarray(c, dtype=np.complex128)
    T, nb = c.shape[0], c.shape[1]
    lam = np.empty((T, nb))
    vecs = np.empty((T, nb, nb), np.complex128) if vectors else None
    st = load().nuc_gevp(c.ctypes.data, T, nb, t0, lam.ctypes.data, None if vecs is None else vecs.ctypes.data)
    if st != NUC_OK:
        raise NucError(st, "nuc_gevp failed (C(t0) not positive definite, or bad arguments)")
    return lam, vecs


def effective_mass(lam):
    """m_n(t) = log(lambda_n(t) / lambda_n(t+1)) from gevp's eigenvalues."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    T, nb = lam.shape
    out = np.empty((T - 1, nb))
    st = load().nuc_effective_mass(lam.ctypes.data, T, nb, out.ctypes.data)
    if st != NUC_OK:
        raise NucError(st, "nuc_effective_mass: bad arguments")
    return out


def svd_prune(corr, t_p: int, m: int):
    """Project C(t) [T][n][n] onto the m leading left singular vectors of C(t_p)
    (host FP64). Returns (C' [T][m][m], basis [n][m])."""
    c = corr.cpu().numpy() if hasattr(corr, "cpu") else np.asarray(corr)
    c = np.ascontiguousarray(c, dtype=np.complex128)
    T, n = c.shape[0], c.shape[1]
    out = np.empty((T, m, m), np.complex128)
    basis = np.empty((n, m), np.complex128)
    st = load().nuc_svd_prune(c.ctypes.data, T, n, t_p, m, out.ctypes.data, basis.ctypes.data)
    if st != NUC_OK:
        raise NucError(st, "nuc_svd_prune: bad arguments")
    return out, basis


# ---------------------------------------------------------------- meson operators
MESON_ND = 7          # D = 1, nabla_0..2, B_0..2
MESON_FAMILIES = 3    # g4 g5;  g4 g5 g_k nabla_k;  g_k B_k


def meson_elementals(evecs, links, mom, L: int, out=None, ctx: Context | None = None, stream=None):
    """Meson elementals Phi^D [T][nmom][7][N][N] (complex64, device) from evecs
    [T][N][L^3][3] and links [T][L^3][3][3][3] (complex64, device)."""
    import torch
    T, N = evecs.shape[0], evecs.shape[1]
    _require_device_tensor(evecs, torch.complex64, (T, N, L ** 3, 3), "evecs")
    _require_device_tensor(links, torch.complex64, (T, L ** 3, 3, 3, 3), "links")
    ctx = ctx or default_context(evecs.device.index or 0)
    m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    nmom = m.shape[0]
    if out is None:
        out = torch.empty((T, nmom, MESON_ND, N, N), dtype=torch.complex64, device=evecs.device)
    _require_device_tensor(out, torch.complex64, (T, nmom, MESON_ND, N, N), "out")
    g = _geom(L, T, N, 0)
    _check(load().nuc_meson_elementals(ctx.handle, ctypes.byref(g), ctypes.c_void_p(evecs.data_ptr()),
                                       ctypes.c_void_p(links.data_ptr()), nmom, m.ctypes.data,
                                       ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return out


def meson_correlator(phi, evals, prof, tau, L: int, t0: int = 0, out=None, ctx: Context | None = None,
                     stream=None):
    """C_AB(t) [nmom][T][3 nprof][3 nprof] (complex128, device) of the profiled meson
    operators from elementals phi [T][nmom][7][N][N] and tau [T][4N][4N]."""
    import torch
    T, nmom, N = phi.shape[0], phi.shape[1], phi.shape[3]
    _require_device_tensor(phi, torch.complex64, (T, nmom, MESON_ND, N, N), "phi")
    _require_device_tensor(tau, torch.complex64, (T, 4 * N, 4 * N), "tau")
    ctx = ctx or default_context(phi.device.index or 0)
    nop = MESON_FAMILIES * len(prof)
    if out is None:
        out = torch.empty((nmom, T, nop, nop), dtype=torch.complex128, device=phi.device)
    _require_device_tensor(out, torch.complex128, (nmom, T, nop, nop), "out")
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    parr, keep = _profiles(prof)
    g = _geom(L, T, N, t0)
    _check(load().nuc_meson_correlator(ctx.handle, ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()),
                                       None if ev is None else ev.ctypes.data, len(prof), parr, nmom,
                                       ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       _stream_ptr(stream)), ctx.handle)
    return out


def twomeson_weights(vec, basis=None):
    """nuc_twomeson_weights: coefficients w_A of the optimal one-meson operator from a GEVP
    eigenvector v (w = conj(v)), or from a pruned GEVP's eigenvector with the pruning basis
    U_m (w = conj(U_m v))."""
    v = np.ascontiguousarray(np.asarray(vec, np.complex128).reshape(-1))
    m = v.size
    if basis is None:
        w = np.empty(m, np.complex128)
        _check(load().nuc_twomeson_weights(v.ctypes.data, m, None, 0, w.ctypes.data))
        return w
    U = np.ascontiguousarray(np.asarray(basis, np.complex128))
    w = np.empty(U.shape[0], np.complex128)
    _check(load().nuc_twomeson_weights(v.ctypes.data, m, U.ctypes.data, U.shape[0], w.ctypes.data))
    return w


def twomeson_correlator(phi, evals, prof, weights, mom, tau, L: int, t0: int = 0, out=None,
                        ctx: Context | None = None, stream=None):
    """(C, D, X)(t) [T][3] (complex128, device) of the I=2 two-meson operator
    sum_k pi(p_k) pi(-p_k) built from the optimal one-meson operator with coefficients
    weights [3 nprof], from elementals phi [T][nmom][7][N][N] at the momenta mom
    (closed under negation) and tau [T][4N][4N]."""
    import torch
    T, nmom, N = phi.shape[0], phi.shape[1], phi.shape[3]
    _require_device_tensor(phi, torch.complex64, (T, nmom, MESON_ND, N, N), "phi")
    _require_device_tensor(tau, torch.complex64, (T, 4 * N, 4 * N), "tau")
    m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    if m.shape[0] != nmom:
        raise ValueError("mom has %d momenta, phi %d" % (m.shape[0], nmom))
    w = np.ascontiguousarray(np.asarray(weights, np.complex128).reshape(-1))
    if w.shape[0] != MESON_FAMILIES * len(prof):
        raise ValueError("weights needs %d entries" % (MESON_FAMILIES * len(prof)))
    ctx = ctx or default_context(phi.device.index or 0)
    if out is None:
        out = torch.empty((T, 3), dtype=torch.complex128, device=phi.device)
    _require_device_tensor(out, torch.complex128, (T, 3), "out")
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    parr, keep = _profiles(prof)
    g = _geom(L, T, N, t0)
    _check(load().nuc_twomeson_correlator(ctx.handle, ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()),
                                          None if ev is None else ev.ctypes.data, len(prof), parr,
                                          w.ctypes.data, nmom, m.ctypes.data, ctypes.c_void_p(tau.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return out


def meson_run(evecs, links, evals, prof, mom, tau, L: int, t0: int = 0, phi_out=None, out=None,
              return_phi: bool = False, ctx: Context | None = None, stream=None):
    """Meson elementals then C_AB(t) in one library call; returns corr (and phi if asked)."""
    import torch
    T, N = evecs.shape[0], evecs.shape[1]
    _require_device_tensor(evecs, torch.complex64, (T, N, L ** 3, 3), "evecs")
    _require_device_tensor(links, torch.complex64, (T, L ** 3, 3, 3, 3), "links")
    _require_device_tensor(tau, torch.complex64, (T, 4 * N, 4 * N), "tau")
    ctx = ctx or default_context(evecs.device.index or 0)
    m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    nmom, nop = m.shape[0], MESON_FAMILIES * len(prof)
    if return_phi and phi_out is None:
        phi_out = torch.empty((T, nmom, MESON_ND, N, N), dtype=torch.complex64, device=evecs.device)
    if phi_out is not None:
        _require_device_tensor(phi_out, torch.complex64, (T, nmom, MESON_ND, N, N), "phi_out")
    if out is None:
        out = torch.empty((nmom, T, nop, nop), dtype=torch.complex128, device=evecs.device)
    _require_device_tensor(out, torch.complex128, (nmom, T, nop, nop), "out")
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    parr, keep = _profiles(prof)
    g = _geom(L, T, N, t0)
    _check(load().nuc_meson_run(ctx.handle, ctypes.byref(g), ctypes.c_void_p(evecs.data_ptr()),
                                ctypes.c_void_p(links.data_ptr()), None if ev is None else ev.ctypes.data,
                                len(prof), parr, nmom, m.ctypes.data, ctypes.c_void_p(tau.data_ptr()),
                                None if phi_out is None else ctypes.c_void_p(phi_out.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return (out, phi_out) if return_phi else out


# ------------------------------------------------------------- general spin tensors
def nucleon_spin(parity: int = +1) -> np.ndarray:
    """nuc_spin_nucleon: S [2][4][4][4] of the nucleon, (C gamma5)_{alpha beta} delta_{gamma sigma}
    with the third quark's parity projection (1 + parity gamma4)/2 (rows 0, 1 for +1; 2, 3
    for -1); C = gamma2 gamma4 in the Euclidean Dirac-Pauli basis."""
    S = np.empty((2, 4, 4, 4), np.complex128)
    _check(load().nuc_spin_nucleon(int(parity), S.ctypes.data))
    return S


def correlator_spin(phi, evals, prof, tau, L: int, S, Sp, t0: int = 0, out=None, ctx: Context | None = None,
                    stream=None):
    """C_ab(t) [nmom][T][nprof][nprof] of three-quark operators with sink spin tensor S and
    source tensor Sp (each [nrow][4][4][4], host) from elementals phi [T][nmom][N][N][N]."""
    import torch
    T, nmom, N = phi.shape[0], phi.shape[1], phi.shape[2]
    _require_device_tensor(phi, torch.complex64, (T, nmom, N, N, N), "phi")
    _require_device_tensor(tau, torch.complex64, (T, 4 * N, 4 * N), "tau")
    S = np.ascontiguousarray(S, dtype=np.complex128)
    Sp = np.ascontiguousarray(Sp, dtype=np.complex128)
    if S.shape != Sp.shape or S.shape[1:] != (4, 4, 4):
        raise ValueError("spin tensors must both be [nrow][4][4][4]")
    ctx = ctx or default_context(phi.device.index or 0)
    nprof = len(prof)
    if out is None:
        out = torch.empty((nmom, T, nprof, nprof), dtype=torch.complex128, device=phi.device)
    _require_device_tensor(out, torch.complex128, (nmom, T, nprof, nprof), "out")
    ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
    parr, keep = _profiles(prof)
    spin = Spin(S.shape[0], S.ctypes.data, Sp.ctypes.data)
    g = _geom(L, T, N, t0)
    _check(load().nuc_correlator_spin(ctx.handle, ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()),
                                      None if ev is None else ev.ctypes.data, nprof, parr, nmom,
                                      ctypes.c_void_p(tau.data_ptr()), ctypes.byref(spin),
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return out


# ------------------------------------------------------------ glueball operators
GLUE_NOP = 5


def glueball_operators(links, L: int, out=None, ctx: Context | None = None, stream=None):
    """The five A1-+ glueball operators O [nconf][T][5] (complex128, device) from links
    [nconf][T][L^3][3][3][3] (or [T][L^3][3][3][3] for one configuration; complex64, device)."""
    import torch
    single = links.dim() == 5
    lk = links.unsqueeze(0) if single else links
    nconf, T = lk.shape[0], lk.shape[1]
    _require_device_tensor(lk, torch.complex64, (nconf, T, L ** 3, 3, 3, 3), "links")
    ctx = ctx or default_context(links.device.index or 0)
    if out is None:
        out = torch.empty((nconf, T, GLUE_NOP), dtype=torch.complex128, device=links.device)
    _require_device_tensor(out, torch.complex128, (nconf, T, GLUE_NOP), "out")
    _check(load().nuc_glueball_operators(ctx.handle, L, T, nconf, ctypes.c_void_p(lk.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), ctx.handle)
    return out[0] if single else out


def glueball_correlator(ops):
    """C [T][nop][nop] (host FP64) of one configuration's operators O [T][nop]."""
    o = ops.cpu().numpy() if hasattr(ops, "cpu") else np.asarray(ops)
    o = np.ascontiguousarray(o, dtype=np.complex128)
    T, nop = o.shape
    c = np.empty((T, nop, nop), np.complex128)
    st = load().nuc_glueball_correlator(o.ctypes.data, T, nop, c.ctypes.data)
    if st != NUC_OK:
        raise NucError(st, "nuc_glueball_correlator: bad arguments")
    return c


# ---------------------------------------------------------------------- serving
def _struct_dict(x) -> dict:
    return {name: getattr(x, name) for name, _ in x._fields_}


class Server:
    """Continuous-batching correlator server (nuc_server_* of include/nucleon_server.h).

    ``executor="hip"`` runs on the GPU; ``executor="fake"`` runs the same
    scheduler with a cost model and a virtual clock and no device at all.
    """

    def __init__(self, executor="hip", device: int = 0, hbm_budget: int = 0, job_arena: int = 0,
                 slot_workspace: int = 0, slots: int = 0, max_active: int = 0, quantum_flops: float = 0.0,
                 start_paused: bool = False, fake_flops_per_s: float = 0.0, fake_fixed_s: float = 0.0):
        lib = load()
        cfg = ServerConfig(EXEC_FAKE if executor == "fake" else EXEC_HIP, device, hbm_budget, job_arena,
                           slot_workspace, slots, max_active, quantum_flops, 1 if start_paused else 0,
                           fake_flops_per_s, fake_fixed_s)
        h = ctypes.c_void_p()
        st = lib.nuc_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != NUC_OK:
            raise NucError(st, lib.nuc_server_last_error(None).decode())
        self._h = h
        self._T = {}

    def _check(self, st):
        if st != NUC_OK:
            raise NucError(st, load().nuc_server_last_error(self._h).decode())

    def register(self, conf_id: int, L: int, evecs=None, evals=None, tau=None, t0: int = 0, T=None, nvec=None):
        """Make a configuration resident: evecs [T][nvec_max][L^3][3] c64 and tau
        [T][4 nvec_max][4 nvec_max] c64 device tensors (copied), evals [T][nvec_max]
        host. With the fake executor pass T and nvec instead of tensors."""
        if evecs is not None:
            import torch
            T, nvec = evecs.shape[0], evecs.shape[1]
            _require_device_tensor(evecs, torch.complex64, (T, nvec, L ** 3, 3), "evecs")
            _require_device_tensor(tau, torch.complex64, (T, 4 * nvec, 4 * nvec), "tau")
        ev = None if evals is None else np.ascontiguousarray(evals, dtype=np.float64)
        g = Geom(L, int(T), int(nvec), t0)
        self._check(load().nuc_server_register(
            self._h, conf_id, ctypes.byref(g), None if evecs is None else ctypes.c_void_p(evecs.data_ptr()),
            None if ev is None else ev.ctypes.data, None if tau is None else ctypes.c_void_p(tau.data_ptr())))
        self._T[conf_id] = int(T)

    def unregister(self, conf_id: int):
        self._check(load().nuc_server_unregister(self._h, conf_id))

    def submit(self, conf_id: int, nvec: int, mom, prof, precision="fp32") -> int:
        m = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
        parr, keep = _profiles(prof)
        req = Request(conf_id, nvec, m.shape[0], m.ctypes.data, len(prof), ctypes.cast(parr, ctypes.c_void_p),
                      _prec(precision))
        t = ctypes.c_uint64()
        self._check(load().nuc_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._shape = getattr(self, "_shape", {})
        self._shape[t.value] = (m.shape[0], self._T[conf_id], len(prof))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(corr [nmom][T][nprof][nprof] complex128 or None, info dict). Raises on
        a failed or cancelled job (NucError.status tells which) and on timeout."""
        shape = getattr(self, "_shape", {}).get(ticket)
        out = None if shape is None else np.zeros(shape[:2] + (shape[2], shape[2]), np.complex128)
        info = JobInfo()
        st = load().nuc_server_wait(self._h, ticket, timeout_ms, None if out is None else out.ctypes.data,
                                    ctypes.byref(info))
        if st == NUC_ERR_INVALID:
            raise NucError(st, load().nuc_server_last_error(self._h).decode())
        if st == NUC_ERR_TIMEOUT:
            raise NucError(st, "ticket %d still running" % ticket)
        self._shape.pop(ticket, None)
        d = _struct_dict(info)
        if st != NUC_OK:
            raise NucError(st, "ticket %d ended with %s: %s" % (ticket, load().nuc_status_string(st).decode(),
                                                              load().nuc_server_last_error(self._h).decode()))
        return out, d

    def cancel(self, ticket: int):
        self._check(load().nuc_server_cancel(self._h, ticket))

    def resume(self):
        self._check(load().nuc_server_resume(self._h))

    def stats(self) -> dict:
        m = ServerMetrics()
        self._check(load().nuc_server_stats(self._h, ctypes.byref(m)))
        return _struct_dict(m)

    def close(self):
        if getattr(self, "_h", None):
            load().nuc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
