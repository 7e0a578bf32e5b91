"""Thin ctypes binding of libkaldo.so (argument marshalling only).

Every computation runs in the library's HIP kernels (or, for the Gamma-point
eigenproblem, its host C++); this module only moves arguments: numpy arrays
for host inputs, torch CUDA tensors for device buffers, and the current torch
stream as the HIP stream.  It fails loudly if the library is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkaldo.so")

FP64, FP32, BF16X3 = 0, 1, 2
GAUSS, LORENTZ = 0, 1
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENUMERIC", -5: "EUNSUPPORTED"}


class KaldoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class Broadening(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("adaptive", ctypes.c_int32),
                ("sigma_thz", ctypes.c_double), ("sigma_floor_thz", ctypes.c_double),
                ("nu_min_thz", ctypes.c_double)]

    @classmethod
    def of(cls, b):
        """From any object with shape/adaptive/sigma_thz/sigma_floor_thz/nu_min_thz."""
        return cls(int(b.shape), int(bool(b.adaptive)), float(b.sigma_thz),
                   float(b.sigma_floor_thz), float(b.nu_min_thz))


_lib = None

P = ctypes.c_void_p
I32P = ctypes.POINTER(ctypes.c_int32)
F64P = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2602_23728_amd.build "
                              "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        L.kaldo_last_error.restype = ctypes.c_char_p
        L.kaldo_version.restype = ctypes.c_int
        L.kaldo_crystal_create.argtypes = [ctypes.c_int32, F64P, F64P, ctypes.c_int32, I32P, F64P,
                                           ctypes.c_int64, I32P, I32P, I32P, F64P,
                                           ctypes.POINTER(P)]
        L.kaldo_crystal_destroy.argtypes = [P]
        L.kaldo_phonons.argtypes = [P, I32P, P, P, P, P]
        L.kaldo_phonons_gamma.argtypes = [ctypes.c_int32, F64P, ctypes.c_int32, F64P, F64P, F64P]
        L.kaldo_linewidths_workspace.argtypes = [P, I32P, ctypes.c_int32]
        L.kaldo_linewidths_workspace.restype = ctypes.c_size_t
        L.kaldo_linewidths.argtypes = [P, I32P, P, P, P, ctypes.c_double,
                                       ctypes.POINTER(Broadening), ctypes.c_int32, P,
                                       ctypes.c_int64, P, ctypes.c_size_t, P, P]
        L.kaldo_linewidths_gamma_workspace.argtypes = [P, ctypes.c_int32]
        L.kaldo_linewidths_gamma_workspace.restype = ctypes.c_size_t
        L.kaldo_linewidths_gamma.argtypes = [P, P, P, ctypes.c_double, ctypes.POINTER(Broadening),
                                             ctypes.c_int32, P, ctypes.c_int64, P,
                                             ctypes.c_size_t, P, P]
        L.kaldo_kappa_rta.argtypes = [P, I32P, P, P, P, ctypes.c_double, ctypes.c_double, P, P]
        L.kaldo_mesh_ibz.argtypes = [F64P, ctypes.c_int32, F64P, F64P, I32P, I32P, I32P, I32P, I32P]
        L.kaldo_jdos_workspace.argtypes = [P, I32P]
        L.kaldo_jdos_workspace.restype = ctypes.c_size_t
        L.kaldo_jdos.argtypes = [P, I32P, P, P, ctypes.POINTER(Broadening), P, ctypes.c_int64, P,
                                 ctypes.c_size_t, P, P, P]
        L.kaldo_surrogate_feature_count.argtypes = [P]
        L.kaldo_surrogate_feature_count.restype = ctypes.c_int32
        L.kaldo_surrogate_features.argtypes = [P, I32P, P, P, P, P, P, ctypes.c_int64, P, P]
        L.kaldo_standardize.argtypes = [ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int64, P, P]
        L.kaldo_surrogate_targets.argtypes = [P, P, ctypes.c_int64, P, P, P]
        L.kaldo_mlp_param_count.argtypes = [ctypes.c_int32]
        L.kaldo_mlp_param_count.restype = ctypes.c_int32
        L.kaldo_mlp_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.kaldo_mlp_workspace.restype = ctypes.c_size_t
        L.kaldo_mlp_train.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P, P,
                                      ctypes.c_int32, ctypes.c_float, P, ctypes.c_size_t, P, P, P]
        L.kaldo_mlp_predict.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P, P, P, P, P]
        L.kaldo_gate_calibrate.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, ctypes.c_int32,
                                           ctypes.c_double, ctypes.c_double, P, P]
        L.kaldo_gate_select.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P, P, P, P]
        L.kaldo_surrogate_domain.argtypes = [ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int64, P, P]
        L.kaldo_gate_score.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_int32,
                                       ctypes.c_double, P, P, P]
        L.kaldo_surrogate_fill.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P, P, P]
        L.kaldo_device_status.argtypes = [P, P]
        L.kaldo_linewidths_noalloc.argtypes = [P, I32P, P, P, P, ctypes.c_double,
                                               ctypes.POINTER(Broadening), ctypes.c_int32, P,
                                               ctypes.c_int64, P, P]
        L.kaldo_linewidths_noalloc_max_bytes.argtypes = []
        L.kaldo_bte_workspace.argtypes = [P, I32P]
        L.kaldo_bte_workspace.restype = ctypes.c_size_t
        L.kaldo_scattering_matrix.argtypes = [P, I32P, P, P, P, ctypes.c_double,
                                              ctypes.POINTER(Broadening), P, ctypes.c_size_t, P,
                                              P, P]
        L.kaldo_bte_solve.argtypes = [P, I32P, P, P, P, ctypes.c_double, ctypes.c_double, P, P,
                                      ctypes.c_size_t, P, P, P]
        L.kaldo_bte_iterate.argtypes = [P, I32P, P, P, P, ctypes.c_double, ctypes.c_double, P,
                                        ctypes.c_int32, ctypes.c_double, P, ctypes.c_size_t, P, P,
                                        ctypes.POINTER(ctypes.c_int32), P]
        L.kaldo_linewidths_noalloc_max_bytes.restype = ctypes.c_size_t
        L.kaldo_isotope_workspace.argtypes = [P, I32P]
        L.kaldo_isotope_workspace.restype = ctypes.c_size_t
        L.kaldo_isotope_linewidths.argtypes = [P, I32P, P, P, P, F64P, ctypes.POINTER(Broadening),
                                               ctypes.c_int32, P, ctypes.c_size_t, P, P]
        L.kaldo_qhgk_crystal_workspace.argtypes = [P, I32P]
        L.kaldo_qhgk_crystal_workspace.restype = ctypes.c_size_t
        L.kaldo_qhgk_gamma_workspace.argtypes = [P]
        L.kaldo_qhgk_gamma_workspace.restype = ctypes.c_size_t
        L.kaldo_qhgk_crystal.argtypes = [P, I32P, F64P, P, P, P, ctypes.c_double, ctypes.c_double, P,
                                         ctypes.c_size_t, P, P]
        L.kaldo_qhgk_gamma.argtypes = [P, F64P, P, P, P, ctypes.c_double, ctypes.c_double, P,
                                       ctypes.c_size_t, P, P, P]
        L.kaldo_tcache_workspace.argtypes = [P, I32P, ctypes.c_int32]
        L.kaldo_tcache_workspace.restype = ctypes.c_size_t
        L.kaldo_tcache_build.argtypes = [P, I32P, P, P, P, ctypes.POINTER(Broadening),
                                         ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_size_t, P,
                                         ctypes.c_int64, P, P, ctypes.POINTER(ctypes.c_int64), P]
        L.kaldo_tcache_gamma_workspace.argtypes = [P, I32P]
        L.kaldo_tcache_gamma_workspace.restype = ctypes.c_size_t
        L.kaldo_tcache_gamma.argtypes = [P, I32P, P, ctypes.c_double, P, ctypes.c_int64, P, P,
                                         ctypes.c_int32, F64P, P, ctypes.c_size_t, P, P]
        L.kaldo_star_map.argtypes = [I32P, ctypes.c_int32, P, P, P, P, P]
        L.kaldo_profile_begin.argtypes = []
        L.kaldo_profile_end.argtypes = [ctypes.POINTER(KernelTime), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


EXPORTED = ["kaldo_crystal_create", "kaldo_crystal_destroy", "kaldo_phonons",
            "kaldo_phonons_gamma", "kaldo_linewidths_workspace", "kaldo_linewidths",
            "kaldo_linewidths_gamma_workspace", "kaldo_linewidths_gamma", "kaldo_kappa_rta",
            "kaldo_last_error", "kaldo_version", "kaldo_profile_begin", "kaldo_profile_end",
            "kaldo_mesh_ibz", "kaldo_jdos_workspace", "kaldo_jdos", "kaldo_surrogate_feature_count",
            "kaldo_surrogate_features", "kaldo_standardize", "kaldo_surrogate_targets",
            "kaldo_mlp_param_count", "kaldo_mlp_workspace", "kaldo_mlp_train", "kaldo_mlp_predict",
            "kaldo_gate_calibrate", "kaldo_gate_select", "kaldo_surrogate_fill", "kaldo_star_map",
            "kaldo_surrogate_domain", "kaldo_gate_score", "kaldo_device_status",
            "kaldo_linewidths_noalloc", "kaldo_linewidths_noalloc_max_bytes",
            "kaldo_bte_workspace", "kaldo_scattering_matrix", "kaldo_bte_solve",
            "kaldo_bte_iterate", "kaldo_tcache_workspace", "kaldo_tcache_build",
            "kaldo_tcache_gamma_workspace", "kaldo_tcache_gamma", "kaldo_isotope_workspace",
            "kaldo_isotope_linewidths", "kaldo_qhgk_crystal_workspace", "kaldo_qhgk_gamma_workspace",
            "kaldo_qhgk_crystal", "kaldo_qhgk_gamma"]


def _check(rc):
    if rc != 0:
        raise KaldoError(rc, lib().kaldo_last_error().decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _dev(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensor expected"
    return ctypes.c_void_p(t.data_ptr())


_EMPTY = {}


def _sub(t):
    """Pointer of a modes_subset tensor: NULL only for "no subset" (None); an
    empty subset gets a valid pointer with a count of 0 (an empty tensor's
    data pointer is NULL, which the library reads as "all modes")."""
    if t is None:
        return None
    if t.numel() == 0:
        dev = t.device.index if t.device.index is not None else torch.cuda.current_device()
        if dev not in _EMPTY:
            _EMPTY[dev] = torch.zeros(1, dtype=torch.int32, device=t.device)
        return ctypes.c_void_p(_EMPTY[dev].data_ptr())
    return _dev(t)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mesh(mesh):
    m = _i32(mesh)
    assert m.shape == (3,)
    return m


_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    """Frees every open handle while the HIP runtime is still up: atexit
    handlers run before the interpreter's finalisers and before the C
    runtime's static destructors (which tear the HIP runtime down)."""
    for c in list(_LIVE):
        c.close()


class Crystal:
    """A cell with FC2 / FC3 uploaded to the current device.  close() frees
    the device tables; handles still open at exit are closed by an atexit
    hook, never from a finaliser during interpreter shutdown."""

    def __init__(self, n_basis, lattice, mass, rep, fc2, fc3_i, fc3_j, fc3_k, fc3_val):
        self._keep = [_f64(lattice).reshape(9), _f64(mass), _i32(rep).reshape(-1), _f64(fc2).reshape(-1),
                      _i32(fc3_i), _i32(fc3_j), _i32(fc3_k), _f64(fc3_val)]
        lat, m, r, f2, fi, fj, fk, fv = self._keep
        self.n_basis = int(n_basis)
        self.nb3 = 3 * self.n_basis
        self.volume = float(abs(np.linalg.det(_f64(lattice).reshape(3, 3))))
        h = P()
        _check(lib().kaldo_crystal_create(self.n_basis, _ptr(lat, F64P), _ptr(m, F64P),
                                          int(len(r) // 3), _ptr(r, I32P), _ptr(f2, F64P),
                                          int(len(fv)), _ptr(fi, I32P), _ptr(fj, I32P),
                                          _ptr(fk, I32P), _ptr(fv, F64P), ctypes.byref(h)))
        self.handle = h
        _LIVE.add(self)

    @classmethod
    def from_model(cls, m):
        return cls(m.n_basis, m.lattice, m.mass, m.rep, m.fc2, m.fc3_i, m.fc3_j, m.fc3_k, m.fc3_val)

    def close(self):
        if getattr(self, "handle", None):
            lib().kaldo_crystal_destroy(self.handle)
            self.handle = None

    def device_status(self):
        """Synchronises the current stream and raises KaldoError if a kernel
        found invalid device inputs since the last query (kaldo_device_status)."""
        _check(lib().kaldo_device_status(self.handle, _stream()))

    def __del__(self):
        if not getattr(self, "handle", None):
            return  # closed already
        # during interpreter shutdown module globals may already be None: the
        # atexit hook has closed every handle by then, so do nothing
        _sys = sys
        if _sys is None or _sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def phonons(c: Crystal, mesh, out=None):
    """omega [N_q, nb3], evec [N_q, nb3, nb3] complex128, vel [N_q, nb3, 3] on cuda."""
    m = _mesh(mesh)
    nq = int(np.prod(m))
    if out is None:
        dev = torch.device("cuda")
        out = (torch.empty(nq, c.nb3, dtype=torch.float64, device=dev),
               torch.empty(nq, c.nb3, c.nb3, 2, dtype=torch.float64, device=dev),
               torch.empty(nq, c.nb3, 3, dtype=torch.float64, device=dev))
    om, ev, ve = out
    _check(lib().kaldo_phonons(c.handle, _ptr(m, I32P), _dev(om), _dev(ev), _dev(ve), _stream()))
    return om, torch.view_as_complex(ev), ve


def phonons_gamma(n_basis, mass, fc2):
    """Host FP64 Gamma-point eigenproblem: omega [nb3], E [nb3, nb3] (numpy).
    fc2: [3N_b][n_rep][3N_b]."""
    m = _f64(mass)
    f2 = _f64(fc2)
    nb3 = 3 * int(n_basis)
    n_rep = f2.size // (nb3 * nb3)
    om = np.empty(nb3)
    E = np.empty((nb3, nb3))
    _check(lib().kaldo_phonons_gamma(int(n_basis), _ptr(m, F64P), int(n_rep), _ptr(f2.reshape(-1), F64P),
                                     _ptr(om, F64P), _ptr(E, F64P)))
    return om, E


def linewidths_workspace(c: Crystal, mesh, precision):
    return int(lib().kaldo_linewidths_workspace(c.handle, _ptr(_mesh(mesh), I32P), int(precision)))


def _as_real(evec):
    if evec.is_complex():
        return torch.view_as_real(evec)
    return evec


def linewidths(c: Crystal, mesh, omega, evec, vel, temperature, broadening, precision=FP32,
               subset=None, workspace=None, out=None):
    """Gamma [N_q, nb3] (rad/ps) on cuda."""
    m = _mesh(mesh)
    nq = int(np.prod(m))
    ws_bytes = linewidths_workspace(c, m, precision)
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    if out is None:
        out = torch.zeros(nq, c.nb3, dtype=torch.float64, device="cuda")
    ev = _as_real(evec).contiguous()
    b = Broadening.of(broadening)
    sub = None if subset is None else subset.to(torch.int32).contiguous()
    _check(lib().kaldo_linewidths(c.handle, _ptr(m, I32P), _dev(omega), _dev(ev), _dev(vel),
                                  float(temperature), ctypes.byref(b), int(precision), _sub(sub),
                                  0 if sub is None else int(sub.numel()), _dev(workspace),
                                  int(workspace.numel()), _dev(out), _stream()))
    return out


def linewidths_noalloc(c: Crystal, mesh, omega, evec, vel, temperature, broadening,
                       precision=FP32, subset=None, out=None):
    """Gamma [N_q, nb3] (rad/ps) on cuda, computed on the library's device
    scratch array (kaldo_linewidths_noalloc); `out` must be given to avoid
    any allocation on this side too."""
    m = _mesh(mesh)
    nq = int(np.prod(m))
    if out is None:
        out = torch.zeros(nq, c.nb3, dtype=torch.float64, device="cuda")
    ev = _as_real(evec)
    assert ev.is_contiguous(), "evec must be contiguous"
    b = Broadening.of(broadening)
    sub = None if subset is None else subset
    if sub is not None:
        assert sub.dtype == torch.int32 and sub.is_contiguous()
    _check(lib().kaldo_linewidths_noalloc(c.handle, _ptr(m, I32P), _dev(omega), _dev(ev), _dev(vel),
                                          float(temperature), ctypes.byref(b), int(precision),
                                          _sub(sub), 0 if sub is None else int(sub.numel()),
                                          _dev(out), _stream()))
    return out


def linewidths_gamma(c: Crystal, omega, evec, temperature, broadening, precision=FP32,
                     subset=None, workspace=None, out=None):
    """Gamma [nb3] (rad/ps) of a Gamma-point solid, on cuda."""
    ws_bytes = int(lib().kaldo_linewidths_gamma_workspace(c.handle, int(precision)))
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    if out is None:
        out = torch.zeros(c.nb3, dtype=torch.float64, device="cuda")
    b = Broadening.of(broadening)
    sub = None if subset is None else subset.to(torch.int32).contiguous()
    _check(lib().kaldo_linewidths_gamma(c.handle, _dev(omega), _dev(evec.contiguous()),
                                        float(temperature), ctypes.byref(b), int(precision),
                                        _sub(sub), 0 if sub is None else int(sub.numel()),
                                        _dev(workspace), int(workspace.numel()), _dev(out),
                                        _stream()))
    return out


def kappa_rta(c: Crystal, mesh, omega, vel, gamma, temperature, nu_min_thz, out=None):
    """kappa [3, 3] W/(m K) on cuda."""
    m = _mesh(mesh)
    if out is None:
        out = torch.empty(3, 3, dtype=torch.float64, device="cuda")
    _check(lib().kaldo_kappa_rta(c.handle, _ptr(m, I32P), _dev(omega), _dev(vel), _dev(gamma),
                                 float(temperature), float(nu_min_thz), _dev(out), _stream()))
    return out


# ------------------------------------------------------------------ full BTE

def bte_workspace(c: Crystal, mesh):
    return int(lib().kaldo_bte_workspace(c.handle, _ptr(_mesh(mesh), I32P)))


def scattering_matrix(c: Crystal, mesh, omega, evec, vel, temperature, broadening, workspace=None,
                      out=None):
    """(matrix [n, n], gamma0 [n]) float64 on cuda, n = N_q nb3."""
    m = _mesh(mesh)
    n = int(np.prod(m)) * c.nb3
    if workspace is None:
        workspace = torch.empty(max(bte_workspace(c, m), 1), dtype=torch.uint8, device="cuda")
    if out is None:
        out = (torch.empty(n, n, dtype=torch.float64, device="cuda"),
               torch.empty(n, dtype=torch.float64, device="cuda"))
    ev = _as_real(evec).contiguous()
    b = Broadening.of(broadening)
    _check(lib().kaldo_scattering_matrix(c.handle, _ptr(m, I32P), _dev(omega), _dev(ev), _dev(vel),
                                         float(temperature), ctypes.byref(b), _dev(workspace),
                                         int(workspace.numel()), _dev(out[0]), _dev(out[1]),
                                         _stream()))
    return out


def bte_solve(c: Crystal, mesh, omega, vel, gamma0, temperature, nu_min_thz, matrix,
              workspace=None):
    """Eq. inverse on the GPU (matrix overwritten by its LU factors):
    (lambda [n, 3], kappa [3, 3]) float64 on cuda."""
    m = _mesh(mesh)
    n = int(np.prod(m)) * c.nb3
    if workspace is None:
        workspace = torch.empty(max(bte_workspace(c, m), 1), dtype=torch.uint8, device="cuda")
    lam = torch.empty(n, 3, dtype=torch.float64, device="cuda")
    kap = torch.empty(3, 3, dtype=torch.float64, device="cuda")
    _check(lib().kaldo_bte_solve(c.handle, _ptr(m, I32P), _dev(omega), _dev(vel), _dev(gamma0),
                                 float(temperature), float(nu_min_thz), _dev(matrix),
                                 _dev(workspace), int(workspace.numel()), _dev(lam), _dev(kap),
                                 _stream()))
    return lam, kap


def bte_iterate(c: Crystal, mesh, omega, vel, gamma0, temperature, nu_min_thz, matrix,
                n_iterations=200, tolerance=1e-10, workspace=None, check=True):
    """Eq. sc_iter on the GPU: (lambda [n, 3], kappa [3, 3], iterations, status).
    Raises on non-convergence when check is True."""
    m = _mesh(mesh)
    n = int(np.prod(m)) * c.nb3
    if workspace is None:
        workspace = torch.empty(max(bte_workspace(c, m), 1), dtype=torch.uint8, device="cuda")
    lam = torch.empty(n, 3, dtype=torch.float64, device="cuda")
    kap = torch.empty(3, 3, dtype=torch.float64, device="cuda")
    it = ctypes.c_int32()
    rc = lib().kaldo_bte_iterate(c.handle, _ptr(m, I32P), _dev(omega), _dev(vel), _dev(gamma0),
                                 float(temperature), float(nu_min_thz), _dev(matrix),
                                 int(n_iterations), float(tolerance), _dev(workspace),
                                 int(workspace.numel()), _dev(lam), _dev(kap), ctypes.byref(it),
                                 _stream())
    if check:
        _check(rc)
    return lam, kap, it.value, rc


# ------------------------------------------------------------------ isotope scattering

def isotope_workspace(c: Crystal, mesh):
    return int(lib().kaldo_isotope_workspace(c.handle, _ptr(_mesh(mesh), I32P)))


def isotope_linewidths(c: Crystal, mesh, omega, evec, vel, g_factor, broadening, out=None,
                       accumulate=False, workspace=None):
    """gamma_iso [N_q, nb3] (rad/ps) on cuda (Eq. isotope); with accumulate
    it is added to `out` (e.g. the anharmonic Gamma) instead."""
    m = _mesh(mesh)
    nq = int(np.prod(m))
    g = _f64(g_factor)
    assert g.shape == (c.n_basis,), "one g factor per basis atom"
    if workspace is None:
        workspace = torch.empty(max(isotope_workspace(c, m), 1), dtype=torch.uint8, device="cuda")
    if out is None:
        assert not accumulate, "accumulate needs out"
        out = torch.empty(nq, c.nb3, dtype=torch.float64, device="cuda")
    ev = _as_real(evec).contiguous()
    b = Broadening.of(broadening)
    _check(lib().kaldo_isotope_linewidths(c.handle, _ptr(m, I32P), _dev(omega), _dev(ev), _dev(vel),
                                          _ptr(g, F64P), ctypes.byref(b), int(bool(accumulate)),
                                          _dev(workspace), int(workspace.numel()), _dev(out),
                                          _stream()))
    return out


# ------------------------------------------------------------------ QHGK conductivity

def qhgk_crystal(c: Crystal, mesh, frac, omega, evec, gamma, temperature, nu_min_thz,
                 workspace=None, out=None):
    """Interband term of Eq. qhgk_crystal: kappa [3, 3] float64 on cuda, W/(m K)."""
    m = _mesh(mesh)
    fr = _f64(frac).reshape(-1)
    assert fr.shape == (3 * c.n_basis,)
    if workspace is None:
        workspace = torch.empty(max(int(lib().kaldo_qhgk_crystal_workspace(c.handle, _ptr(m, I32P))),
                                    1), dtype=torch.uint8, device="cuda")
    if out is None:
        out = torch.empty(3, 3, dtype=torch.float64, device="cuda")
    ev = _as_real(evec).contiguous()
    _check(lib().kaldo_qhgk_crystal(c.handle, _ptr(m, I32P), _ptr(fr, F64P), _dev(omega), _dev(ev),
                                    _dev(gamma), float(temperature), float(nu_min_thz),
                                    _dev(workspace), int(workspace.numel()), _dev(out), _stream()))
    return out


def qhgk_gamma(c: Crystal, frac, omega, evec, gamma, temperature, nu_min_thz, diffusivity=True,
               workspace=None):
    """Eq. qhgk for a Gamma-point solid: (kappa [3, 3] W/(m K), mode diffusivity
    [3N] A^2/ps or None) on cuda."""
    fr = _f64(frac).reshape(-1)
    assert fr.shape == (3 * c.n_basis,)
    if workspace is None:
        workspace = torch.empty(max(int(lib().kaldo_qhgk_gamma_workspace(c.handle)), 1),
                                dtype=torch.uint8, device="cuda")
    kap = torch.empty(3, 3, dtype=torch.float64, device="cuda")
    diff = torch.empty(c.nb3, dtype=torch.float64, device="cuda") if diffusivity else None
    _check(lib().kaldo_qhgk_gamma(c.handle, _ptr(fr, F64P), _dev(omega), _dev(evec), _dev(gamma),
                                  float(temperature), float(nu_min_thz), _dev(workspace),
                                  int(workspace.numel()), _dev(kap), _dev(diff), _stream()))
    return kap, diff


# ------------------------------------------------------------------ temperature sweeps

class TempCache:
    """Temperature-independent factors of Eq. gamma on cuda (see
    kaldo_tcache_build): row_ptr int64 [n_modes + 1], pairs int32 [n, 2]
    (partner modes, read as uint32), factors float64 [n, 2] (c, d)."""

    def __init__(self, mesh, row_ptr, pairs, factors):
        self.mesh = tuple(int(x) for x in mesh)
        self.row_ptr = row_ptr
        self.pairs = pairs
        self.factors = factors

    @property
    def n_entries(self):
        return int(self.pairs.shape[0])

    @property
    def nbytes(self):
        return (self.row_ptr.numel() * 8 + self.pairs.numel() * 4 + self.factors.numel() * 8)


def tcache_workspace(c: Crystal, mesh, precision=FP64):
    return int(lib().kaldo_tcache_workspace(c.handle, _ptr(_mesh(mesh), I32P), int(precision)))


def tcache_count(c: Crystal, mesh, omega, evec, vel, broadening, precision=FP64, subset=None,
                 workspace=None, row_ptr=None):
    """Count pass alone: (row_ptr int64 [n_modes + 1] on cuda, entries)."""
    m = _mesh(mesh)
    n_modes = int(np.prod(m)) * c.nb3
    if workspace is None:
        workspace = torch.empty(max(tcache_workspace(c, m, precision), 1), dtype=torch.uint8,
                                device="cuda")
    if row_ptr is None:
        row_ptr = torch.empty(n_modes + 1, dtype=torch.int64, device="cuda")
    ev = _as_real(evec).contiguous()
    b = Broadening.of(broadening)
    sub = None if subset is None else subset.to(torch.int32).contiguous()
    n = ctypes.c_int64()
    _check(lib().kaldo_tcache_build(c.handle, _ptr(m, I32P), _dev(omega), _dev(ev), _dev(vel),
                                    ctypes.byref(b), int(precision), _sub(sub),
                                    0 if sub is None else int(sub.numel()), _dev(workspace),
                                    int(workspace.numel()), _dev(row_ptr), 0, None, None,
                                    ctypes.byref(n), _stream()))
    return row_ptr, n.value


def tcache_build(c: Crystal, mesh, omega, evec, vel, broadening, precision=FP64, subset=None,
                 workspace=None):
    """TempCache of the modes in `subset` (all modes by default): a count
    call for the size, then the filling call."""
    m = _mesh(mesh)
    if workspace is None:
        workspace = torch.empty(max(tcache_workspace(c, m, precision), 1), dtype=torch.uint8,
                                device="cuda")
    row_ptr, n = tcache_count(c, m, omega, evec, vel, broadening, precision, subset, workspace)
    pairs = torch.empty(max(n, 1), 2, dtype=torch.int32, device="cuda")
    factors = torch.empty(max(n, 1), 2, dtype=torch.float64, device="cuda")
    ev = _as_real(evec).contiguous()
    b = Broadening.of(broadening)
    sub = None if subset is None else subset.to(torch.int32).contiguous()
    got = ctypes.c_int64()
    _check(lib().kaldo_tcache_build(c.handle, _ptr(m, I32P), _dev(omega), _dev(ev), _dev(vel),
                                    ctypes.byref(b), int(precision), _sub(sub),
                                    0 if sub is None else int(sub.numel()), _dev(workspace),
                                    int(workspace.numel()), _dev(row_ptr), int(pairs.shape[0]),
                                    _dev(pairs), _dev(factors), ctypes.byref(got), _stream()))
    assert got.value == n
    return TempCache(m, row_ptr, pairs[:n], factors[:n])


def tcache_gamma_workspace(c: Crystal, mesh):
    return int(lib().kaldo_tcache_gamma_workspace(c.handle, _ptr(_mesh(mesh), I32P)))


def tcache_gamma(c: Crystal, cache: TempCache, omega, nu_min_thz, temperatures, workspace=None,
                 out=None):
    """Gamma [n_T, N_q, nb3] (rad/ps) on cuda at each temperature."""
    m = _mesh(cache.mesh)
    nq = int(np.prod(m))
    t = _f64(np.atleast_1d(temperatures))
    if workspace is None:
        workspace = torch.empty(max(tcache_gamma_workspace(c, m), 1), dtype=torch.uint8,
                                device="cuda")
    if out is None:
        out = torch.empty(len(t), nq, c.nb3, dtype=torch.float64, device="cuda")
    n = cache.n_entries
    _check(lib().kaldo_tcache_gamma(c.handle, _ptr(m, I32P), _dev(omega), float(nu_min_thz),
                                    _dev(cache.row_ptr), n, _dev(cache.pairs) if n else None,
                                    _dev(cache.factors) if n else None, len(t), _ptr(t, F64P),
                                    _dev(workspace), int(workspace.numel()), _dev(out), _stream()))
    return out


# ------------------------------------------------------------------ learned form

def mesh_ibz(lattice, frac, mass, mesh):
    """Host: (ir_of_q [N_q], star_size [N_q], n_ops, n_ir) as numpy int32."""
    m = _mesh(mesh)
    nq = int(np.prod(m))
    lat = _f64(lattice).reshape(9)
    fr = _f64(frac).reshape(-1)
    ms = _f64(mass)
    ir = np.empty(nq, np.int32)
    star = np.empty(nq, np.int32)
    n_ops = ctypes.c_int32()
    n_ir = ctypes.c_int32()
    _check(lib().kaldo_mesh_ibz(_ptr(lat, F64P), int(len(ms)), _ptr(fr, F64P), _ptr(ms, F64P),
                                _ptr(m, I32P), _ptr(ir, I32P), _ptr(star, I32P),
                                ctypes.byref(n_ops), ctypes.byref(n_ir)))
    return ir, star, n_ops.value, n_ir.value


def jdos(c: Crystal, mesh, omega, vel, broadening, subset=None, workspace=None, out=None):
    """(D+, D-) [N_q, nb3] ps/rad on cuda; only subset entries are written."""
    m = _mesh(mesh)
    nq = int(np.prod(m))
    ws = int(lib().kaldo_jdos_workspace(c.handle, _ptr(m, I32P)))
    if workspace is None:
        workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device="cuda")
    if out is None:
        out = (torch.zeros(nq, c.nb3, dtype=torch.float64, device="cuda"),
               torch.zeros(nq, c.nb3, dtype=torch.float64, device="cuda"))
    b = Broadening.of(broadening)
    sub = None if subset is None else subset.to(torch.int32).contiguous()
    _check(lib().kaldo_jdos(c.handle, _ptr(m, I32P), _dev(omega), _dev(vel), ctypes.byref(b),
                            _sub(sub), 0 if sub is None else int(sub.numel()), _dev(workspace),
                            int(workspace.numel()), _dev(out[0]), _dev(out[1]), _stream()))
    return out


def surrogate_feature_count(c: Crystal):
    return int(lib().kaldo_surrogate_feature_count(c.handle))


def surrogate_features(c: Crystal, mesh, omega, vel, dplus, dminus, modes, out=None):
    """float32 [n, nb3 + 8] on cuda."""
    m = _mesh(mesh)
    modes = modes.to(torch.int32).contiguous()
    n = int(modes.numel())
    if out is None:
        out = torch.empty(n, surrogate_feature_count(c), dtype=torch.float32, device="cuda")
    _check(lib().kaldo_surrogate_features(c.handle, _ptr(m, I32P), _dev(omega), _dev(vel),
                                          _dev(dplus), _dev(dminus), _dev(modes), n, _dev(out),
                                          _stream()))
    return out


def standardize(X, n_fit, mu_sd=None):
    """Standardises X (float32 [n, n_feat], cuda) in place; returns mu_sd [n_feat, 2]."""
    n, nf = X.shape
    if mu_sd is None:
        mu_sd = torch.empty(nf, 2, dtype=torch.float32, device="cuda")
    _check(lib().kaldo_standardize(int(n), int(nf), _dev(X), int(n_fit), _dev(mu_sd), _stream()))
    return mu_sd


def surrogate_targets(gamma, modes, out=None):
    """(y float32 [n], y_mu_sd float32 [2]) on cuda."""
    modes = modes.to(torch.int32).contiguous()
    n = int(modes.numel())
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device="cuda"),
               torch.empty(2, dtype=torch.float32, device="cuda"))
    _check(lib().kaldo_surrogate_targets(_dev(gamma), _dev(modes), n, _dev(out[0]), _dev(out[1]),
                                         _stream()))
    return out


def mlp_param_count(n_in):
    return int(lib().kaldo_mlp_param_count(int(n_in)))


def mlp_train(X, y, counts, params, steps, lr=1e-3, losses=False, grad=False, workspace=None):
    """Trains params (float32 [M, P], cuda) in place.  Returns (losses [M, steps] or None,
    gradient of the last step [M, P] or None).  Synchronises the stream."""
    n, n_in = X.shape
    M = params.shape[0]
    ws = int(lib().kaldo_mlp_workspace(int(n_in), int(M), int(n)))
    if workspace is None:
        workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device="cuda")
    L = torch.zeros(M, max(int(steps), 1), dtype=torch.float32, device="cuda") if losses else None
    G = torch.zeros_like(params) if grad else None
    _check(lib().kaldo_mlp_train(int(n_in), int(M), int(n), _dev(X.contiguous()), _dev(y.contiguous()),
                                 _dev(counts.contiguous()), _dev(params), int(steps), float(lr),
                                 _dev(workspace), int(workspace.numel()), _dev(L), _dev(G), _stream()))
    return L, G


def mlp_predict(X, params, out=None):
    """(mean, spread) float32 [n] on cuda."""
    n, n_in = X.shape
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device="cuda"),
               torch.empty(n, dtype=torch.float32, device="cuda"))
    _check(lib().kaldo_mlp_predict(int(n_in), int(params.shape[0]), int(n), _dev(X.contiguous()),
                                   _dev(params.contiguous()), _dev(out[0]), _dev(out[1]), _stream()))
    return out


def surrogate_domain(X, n_fit, out=None):
    """uint8 [n] on cuda: 1 where the row lies inside the first n_fit rows' ranges."""
    n, nf = X.shape
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device="cuda")
    _check(lib().kaldo_surrogate_domain(int(n), int(nf), _dev(X), int(n_fit), _dev(out), _stream()))
    return out


def gate_score(modes, mean, spread, y_mu_sd, omega, vel, star_size, nb3, temperature, inside=None,
               out=None):
    """float32 [n] on cuda."""
    modes = modes.to(torch.int32).contiguous()
    n = int(modes.numel())
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
    _check(lib().kaldo_gate_score(n, _dev(modes), _dev(mean), _dev(spread), _dev(y_mu_sd), _dev(omega),
                                  _dev(vel), _dev(star_size), int(nb3), float(temperature),
                                  _dev(inside), _dev(out), _stream()))
    return out


def gate_calibrate(modes, gamma, mean, y_mu_sd, score, omega, vel, star_size, nb3, temperature,
                   tol, out=None):
    """tau: float32 [1] on cuda."""
    modes = modes.to(torch.int32).contiguous()
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().kaldo_gate_calibrate(int(modes.numel()), _dev(modes), _dev(gamma), _dev(mean),
                                      _dev(y_mu_sd), _dev(score), _dev(omega), _dev(vel),
                                      _dev(star_size), int(nb3), float(temperature), float(tol),
                                      _dev(out), _stream()))
    return out


def gate_select(modes, score, tau, computed, out=None):
    """(fallback int32 [n], n_fallback int32 [1]) on cuda; marks computed."""
    modes = modes.to(torch.int32).contiguous()
    n = int(modes.numel())
    if out is None:
        out = (torch.empty(max(n, 1), dtype=torch.int32, device="cuda"),
               torch.empty(1, dtype=torch.int32, device="cuda"))
    _check(lib().kaldo_gate_select(n, int(computed.numel()), _dev(modes), _dev(score), _dev(tau),
                                   _dev(computed), _dev(out[0]), _dev(out[1]), _stream()))
    return out


def surrogate_fill(modes, mean, y_mu_sd, computed, gamma):
    modes = modes.to(torch.int32).contiguous()
    assert gamma.numel() == computed.numel(), "gamma and computed cover the same modes"
    _check(lib().kaldo_surrogate_fill(int(modes.numel()), int(computed.numel()), _dev(modes),
                                      _dev(mean), _dev(y_mu_sd), _dev(computed), _dev(gamma),
                                      _stream()))
    return gamma


def star_map(mesh, nb3, ir_of_q, omega, gamma_ir, out=None):
    m = _mesh(mesh)
    if out is None:
        out = torch.empty_like(gamma_ir)
    _check(lib().kaldo_star_map(_ptr(m, I32P), int(nb3), _dev(ir_of_q), _dev(omega), _dev(gamma_ir),
                                _dev(out), _stream()))
    return out
