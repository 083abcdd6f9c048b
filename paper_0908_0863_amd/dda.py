"""Thin ctypes binding of libdda (include/dda.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libdda.so.  Device memory and streams come from PyTorch (ROCm);
vectors are torch tensors of shape [nrhs, 3, N_d], complex128 (FP64) or
complex64 (FP32), on the library's device.

Functions keep the C names (``dda_open``, ``dda_target_create``, ...);
``Library`` and ``Target`` are small owners of the handles on top of them.
If libdda.so is missing this module raises on load: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime that libdda binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdda.so")

DDA_OK, DDA_EINVAL, DDA_ENOMEM, DDA_EDEVICE, DDA_ENOTCONV, DDA_ESTATE = 0, -1, -2, -3, -4, -5
DDA_FP64, DDA_FP32 = 0, 1
DDA_POL_CM, DDA_POL_RR, DDA_POL_LDR = 0, 1, 2
DDA_BICGSTAB, DDA_QMR_SYM, DDA_BICG_SYM, DDA_CGS, DDA_TFQMR = 0, 1, 2, 3, 4
DDA_BICG, DDA_QMR, DDA_RBICGSTAB, DDA_MLBICGSTAB = 5, 6, 7, 8
DDA_SOLVE_FP64, DDA_SOLVE_MIXED = 0, 1

_PRESC = {"cm": DDA_POL_CM, "rr": DDA_POL_RR, "ldr": DDA_POL_LDR}
# Scheme names as the paper's Table 3 lists them (cocg = bicg_sym).
_SOLVER = {"bicgstab": DDA_BICGSTAB, "qmr_sym": DDA_QMR_SYM, "bicg_sym": DDA_BICG_SYM, "cocg": DDA_BICG_SYM,
           "cgs": DDA_CGS, "tfqmr": DDA_TFQMR, "bicg": DDA_BICG, "qmr": DDA_QMR, "rbicgstab": DDA_RBICGSTAB,
           "mlbicgstab": DDA_MLBICGSTAB}
_SPREC = {"fp64": DDA_SOLVE_FP64, "mixed": DDA_SOLVE_MIXED}


class DDAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdda error {code}: {msg}")
        self.code = code


class NotConverged(DDAError):
    pass


class dda_solve_opts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("precision", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("jacobi", ctypes.c_int), ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("solver_param", ctypes.c_int)]


class dda_solve_info(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int), ("iterations", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("matvecs", ctypes.c_int), ("rel_residual", ctypes.c_double)]


class dda_batch_item(ctypes.Structure):
    _fields_ = [("target", ctypes.c_void_p), ("nrhs", ctypes.c_int), ("khat", ctypes.c_void_p),
                ("ehat", ctypes.c_void_p), ("S", ctypes.c_void_p), ("einc_dev", ctypes.c_void_p),
                ("p_dev", ctypes.c_void_p), ("info", ctypes.c_void_p)]


# Every symbol the header declares (tests check that the library exports them).
EXPORTS = ["dda_open", "dda_close", "dda_target_create", "dda_target_destroy", "dda_set_occupancy",
           "dda_set_permittivity", "dda_set_polarizability", "dda_set_composition", "dda_build_spectrum", "dda_matvec",
           "dda_matvec_noalloc", "dda_solve", "dda_solve_orientation_factors", "dda_batch_solve",
           "dda_incident_field", "dda_cross_sections", "dda_far_field", "dda_csca_quadrature", "dda_mueller",
           "dda_grad_cabs_eps", "dda_target_set_option",
           "dda_target_info", "dda_target_set_padding", "dda_tune_padding",
           "dda_get_spectrum", "dda_profile_enable", "dda_profile_read", "dda_profile_reset",
           "dda_last_error"]

PASS_NAMES = ["y_forward", "x_forward", "z_product", "x_inverse", "y_inverse", "xy_forward", "xy_inverse", "matvec"]
DDA_PROF_SLOTS = len(PASS_NAMES)
DDA_OPT_SCHEDULE, DDA_OPT_INJECT_BREAKDOWN, DDA_OPT_CANARY, DDA_OPT_FUSE_QMR_STEP, DDA_OPT_RHS_PER_BLOCK = 1, 2, 3, 4, 5
DDA_OPT_Y_TILE = 6
DDA_OPT_INJECT_BAD_STEP = 7
DDA_OPT_X_ROWS = 8

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Open libdda.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libdda.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "dda_open": (i, [i, ctypes.c_char_p, P(vp)]),
        "dda_close": (None, [vp]),
        "dda_target_create": (i, [vp, i, i, i, d, P(vp)]),
        "dda_target_destroy": (None, [vp]),
        "dda_set_occupancy": (i, [vp, vp, P(i64)]),
        "dda_set_permittivity": (i, [vp, vp, i]),
        "dda_set_polarizability": (i, [vp, vp]),
        "dda_set_composition": (i, [vp, i, vp, vp, i]),
        "dda_build_spectrum": (i, [vp, vp]),
        "dda_matvec": (i, [vp, i, i, vp, i, vp, vp, vp]),
        "dda_matvec_noalloc": (i, [vp, i, i, vp, i, vp, vp, vp]),
        "dda_solve": (i, [vp, P(dda_solve_opts), i, vp, vp, vp, vp, vp, vp, vp]),
        "dda_solve_orientation_factors": (i, [vp, i, vp]),
        "dda_batch_solve": (i, [vp, P(dda_solve_opts), i, vp, i, vp]),
        "dda_incident_field": (i, [vp, i, vp, vp, vp, vp]),
        "dda_cross_sections": (i, [vp, i, vp, vp, vp, vp, vp, vp, vp]),
        "dda_far_field": (i, [vp, i, vp, i, vp, vp, vp]),
        "dda_csca_quadrature": (i, [vp, i, vp, i, i, vp, vp]),
        "dda_mueller": (i, [vp, vp, i, vp, vp, vp, vp]),
        "dda_grad_cabs_eps": (i, [vp, P(dda_solve_opts), i, vp, vp, vp, vp]),
        "dda_target_set_option": (i, [vp, i, i]),
        "dda_target_info": (i, [vp, vp]),
        "dda_target_set_padding": (i, [vp, i, i, i]),
        "dda_tune_padding": (i, [vp, i, i, vp, vp]),
        "dda_get_spectrum": (i, [vp, i, vp, vp]),
        "dda_profile_enable": (i, [vp, i]),
        "dda_profile_read": (i, [vp, vp, vp]),
        "dda_profile_reset": (i, [vp]),
        "dda_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != DDA_OK:
        msg = load().dda_last_error().decode()
        if rc == DDA_ENOTCONV:
            raise NotConverged(rc, msg)
        raise DDAError(rc, msg)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _opt_np(a, dtype, n):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=dtype).reshape(-1))
    if arr.size != n:
        raise ValueError(f"expected {n} values, got {arr.size}")
    return arr, _np_ptr(arr)


class Library:
    """An opened libdda on one HIP device."""

    def __init__(self, device: int | None = None, tune_cache: str | None = None):
        lib = load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = ctypes.c_void_p()
        _check(lib.dda_open(device, tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            load().dda_close(self.h)
            self.h = None

    def profile(self, enable=True):
        """True/1: time every pass and every whole product; 2: whole products
        only (no events between the passes); False/0: off."""
        _check(load().dda_profile_enable(self.h, int(enable)))

    def profile_reset(self):
        _check(load().dda_profile_reset(self.h))

    def profile_read(self) -> dict:
        """{(pass name, 'fp64'|'fp32'): (total ms, launches)} over the recorded launches."""
        npass = len(PASS_NAMES)
        ms = np.zeros(2 * npass)
        n = np.zeros(2 * npass, np.int64)
        _check(load().dda_profile_read(self.h, _np_ptr(ms), _np_ptr(n)))
        keys = [(p, "fp64") for p in PASS_NAMES] + [(p, "fp32") for p in PASS_NAMES]
        return {k: (float(a), int(b)) for k, a, b in zip(keys, ms, n)}

    def batch_solve(self, items, nworkers: int = 0, raise_on_fail: bool = True, **kw):
        """Solve several targets in one dda_batch_solve call.

        items: list of dicts with key ``target`` and either ``khat``/``ehat``
        (optionally ``S``) or ``einc`` (a device tensor, with ``S``).
        Returns a list of (P, infos) in the order of ``items``."""
        opts = Target.make_opts(**kw)
        arr = (dda_batch_item * len(items))()
        keep, out = [], []
        for k, it in enumerate(items):
            t = it["target"]
            kh = eh = None
            if it.get("einc") is None:
                kh = np.ascontiguousarray(np.asarray(it["khat"], np.float64).reshape(-1, 3))
                eh = np.ascontiguousarray(np.asarray(it["ehat"], np.complex128).reshape(-1, 3))
                nrhs = kh.shape[0]
            else:
                nrhs = it["einc"].shape[0]
            Sa, Sp = _opt_np(it.get("S"), np.float64, nrhs)
            P = torch.empty((nrhs, 3, t.nd), dtype=torch.complex128, device=t.dev)
            info = (dda_solve_info * nrhs)()
            keep += [kh, eh, Sa, info]
            arr[k].target = t.h.value
            arr[k].nrhs = nrhs
            arr[k].khat = kh.ctypes.data if kh is not None else None
            arr[k].ehat = eh.ctypes.data if eh is not None else None
            arr[k].S = Sa.ctypes.data if Sa is not None else None
            arr[k].einc_dev = _dptr(it["einc"]).value if it.get("einc") is not None else None
            arr[k].p_dev = P.data_ptr()
            arr[k].info = ctypes.addressof(info)
            out.append((P, info))
        rc = load().dda_batch_solve(self.h, ctypes.byref(opts), len(items), ctypes.cast(arr, ctypes.c_void_p),
                                    int(nworkers), _stream())
        if rc != DDA_ENOTCONV or raise_on_fail:
            _check(rc)
        return [(P, [dict(converged=i.converged, iterations=i.iterations, outer_iterations=i.outer_iterations,
                          matvecs=i.matvecs, rel_residual=i.rel_residual) for i in info]) for P, info in out]

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Target:
    """A lattice target: occupancy, polarisabilities and the interaction spectrum."""

    def __init__(self, lib: Library, K: int, J: int, P: int, kd: float):
        self.lib = lib
        self.K, self.J, self.P, self.kd = int(K), int(J), int(P), float(kd)
        h = ctypes.c_void_p()
        _check(load().dda_target_create(lib.h, self.K, self.J, self.P, self.kd, ctypes.byref(h)))
        self.h = h
        self.nd = 0

    def close(self):
        if getattr(self, "h", None):
            load().dda_target_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dev(self):
        return torch.device("cuda", self.lib.device)

    def set_occupancy(self, occ) -> int:
        occ = np.ascontiguousarray(np.asarray(occ, dtype=np.uint8).reshape(-1))
        if occ.size != self.K * self.J * self.P:
            raise ValueError("occupancy size")
        nd = ctypes.c_int64()
        _check(load().dda_set_occupancy(self.h, _np_ptr(occ), ctypes.byref(nd)))
        self.nd = int(nd.value)
        return self.nd

    def set_permittivity(self, eps, prescription: str = "ldr"):
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.complex128), (self.nd,)))
        _check(load().dda_set_permittivity(self.h, _np_ptr(e), _PRESC[prescription]))

    def set_polarizability(self, alpha):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha, np.complex128), (self.nd,)))
        _check(load().dda_set_polarizability(self.h, _np_ptr(a)))

    def set_composition(self, eps_materials, flags, prescription: str = "ldr"):
        """Materials eps_materials [nmat] and the material index of every
        component of every dipole, flags [3, N_d] (x, y, z)."""
        e = np.ascontiguousarray(np.asarray(eps_materials, np.complex128).reshape(-1))
        f = np.ascontiguousarray(np.asarray(flags, np.uint8).reshape(3, self.nd))
        _check(load().dda_set_composition(self.h, e.size, _np_ptr(e), _np_ptr(f), _PRESC[prescription]))

    def build_spectrum(self):
        _check(load().dda_build_spectrum(self.h, _stream()))

    def set_option(self, option: int, value: int):
        _check(load().dda_target_set_option(self.h, int(option), int(value)))

    def set_padding(self, Kpp: int = 0, Jpp: int = 0, Ppp: int = 0):
        """Padded FFT lengths (0: the default rule); the spectrum must be
        built again afterwards."""
        _check(load().dda_target_set_padding(self.h, int(Kpp), int(Jpp), int(Ppp)))

    def tune_padding(self, nrhs: int = 1, precision: str = "fp32") -> tuple:
        """Padded lengths chosen by timing products (spectrum built for them)."""
        out = np.zeros(3, np.int32)
        prec = DDA_FP32 if precision == "fp32" else DDA_FP64
        _check(load().dda_tune_padding(self.h, int(nrhs), prec, _np_ptr(out), _stream()))
        return tuple(int(v) for v in out)

    def info(self) -> dict:
        dims = np.zeros(9, np.int64)
        _check(load().dda_target_info(self.h, _np_ptr(dims)))
        keys = ["Kpp", "Jpp", "Ppp", "Kh", "Jh", "Ph", "nd", "lines_matvec", "lines_spectrum"]
        return {k: int(v) for k, v in zip(keys, dims)}

    def spectrum(self, precision: int = DDA_FP64) -> torch.Tensor:
        i = self.info()
        dt = torch.complex128 if precision == DDA_FP64 else torch.complex64
        out = torch.empty((6, i["Ph"], i["Jh"], i["Kh"]), dtype=dt, device=self.dev)
        _check(load().dda_get_spectrum(self.h, precision, _dptr(out), _stream()))
        torch.cuda.current_stream().synchronize()
        return out

    def matvec(self, x: torch.Tensor, S=None, jacobi: bool = False, out: torch.Tensor | None = None):
        if x.dim() != 3 or x.shape[1] != 3 or x.shape[2] != self.nd:
            raise ValueError("x must be [nrhs, 3, N_d]")
        prec = {torch.complex128: DDA_FP64, torch.complex64: DDA_FP32}[x.dtype]
        nrhs = x.shape[0]
        y = torch.empty_like(x) if out is None else out
        Sa, Sp = _opt_np(S, np.float64, nrhs)
        _check(load().dda_matvec(self.h, prec, nrhs, Sp, int(bool(jacobi)), _dptr(x), _dptr(y), _stream()))
        return y

    def matvec_noalloc(self, x: torch.Tensor, out: torch.Tensor, S=None, jacobi: bool = False):
        """dda_matvec_noalloc: y = A x into the caller's ``out`` with the
        library's device scratch for every other buffer (nothing allocated)."""
        if x.dim() != 3 or x.shape[1] != 3 or x.shape[2] != self.nd or out.shape != x.shape or out.dtype != x.dtype:
            raise ValueError("x and out must be [nrhs, 3, N_d] of one dtype")
        prec = {torch.complex128: DDA_FP64, torch.complex64: DDA_FP32}[x.dtype]
        Sa, Sp = _opt_np(S, np.float64, x.shape[0])
        _check(load().dda_matvec_noalloc(self.h, prec, x.shape[0], Sp, int(bool(jacobi)), _dptr(x), _dptr(out),
                                         _stream()))
        return out

    def incident_field(self, khat, ehat) -> torch.Tensor:
        kh = np.ascontiguousarray(np.asarray(khat, np.float64).reshape(-1, 3))
        eh = np.ascontiguousarray(np.asarray(ehat, np.complex128).reshape(-1, 3))
        nrhs = kh.shape[0]
        E = torch.empty((nrhs, 3, self.nd), dtype=torch.complex128, device=self.dev)
        _check(load().dda_incident_field(self.h, nrhs, _np_ptr(kh), _np_ptr(eh), _dptr(E), _stream()))
        return E

    @staticmethod
    def make_opts(solver="qmr_sym", precision="fp64", tol=1e-6, inner_tol=0.0, max_iter=0, max_outer=0,
                  jacobi=True, check_every=0, use_graph=False, solver_param=0) -> dda_solve_opts:
        """solver_param: l of "rbicgstab", n of "mlbicgstab" (1..4; 0 = 2)."""
        return dda_solve_opts(_SOLVER[solver], _SPREC[precision], int(max_iter), int(max_outer), float(tol),
                              float(inner_tol), int(bool(jacobi)), int(check_every), int(bool(use_graph)),
                              int(solver_param))

    def solve(self, khat=None, ehat=None, S=None, einc: torch.Tensor | None = None, raise_on_fail=True, **kw):
        """Solve A P = E_inc.  Returns (P [nrhs,3,N_d] complex128, list of info dicts)."""
        opts = self.make_opts(**kw)
        kh = eh = None
        khp = ehp = None
        if khat is not None:
            kh = np.ascontiguousarray(np.asarray(khat, np.float64).reshape(-1, 3))
            eh = np.ascontiguousarray(np.asarray(ehat, np.complex128).reshape(-1, 3))
            khp, ehp = _np_ptr(kh), _np_ptr(eh)
            nrhs = kh.shape[0]
        else:
            nrhs = einc.shape[0]
        Sa, Sp = _opt_np(S, np.float64, nrhs)
        P = torch.empty((nrhs, 3, self.nd), dtype=torch.complex128, device=self.dev)
        info = (dda_solve_info * nrhs)()
        ep = _dptr(einc) if einc is not None else None
        rc = load().dda_solve(self.h, ctypes.byref(opts), nrhs, khp, ehp, Sp, ep, _dptr(P), info, _stream())
        infos = [dict(converged=i.converged, iterations=i.iterations, outer_iterations=i.outer_iterations,
                      matvecs=i.matvecs, rel_residual=i.rel_residual) for i in info]
        if rc != DDA_ENOTCONV or raise_on_fail:
            _check(rc)
        return P, infos

    def orientation_factors(self, nrhs: int) -> list:
        """The LDR orientation factors S the last solve on this target used."""
        out = np.zeros(int(nrhs))
        _check(load().dda_solve_orientation_factors(self.h, int(nrhs), _np_ptr(out)))
        return [float(v) for v in out]

    def cross_sections(self, einc: torch.Tensor, P: torch.Tensor, S=None):
        nrhs = P.shape[0]
        Sa, Sp = _opt_np(S, np.float64, nrhs)
        ce = np.zeros(nrhs)
        ca = np.zeros(nrhs)
        cs = np.zeros(nrhs)
        _check(load().dda_cross_sections(self.h, nrhs, Sp, _dptr(einc), _dptr(P), _np_ptr(ce), _np_ptr(ca),
                                         _np_ptr(cs), _stream()))
        return ce, ca, cs

    def far_field(self, P: torch.Tensor, dirs) -> torch.Tensor:
        """F(n) [nrhs, ndir, 3] complex128 for unit directions dirs [ndir, 3]."""
        d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
        F = torch.empty((P.shape[0], d.shape[0], 3), dtype=torch.complex128, device=self.dev)
        _check(load().dda_far_field(self.h, P.shape[0], _dptr(P), d.shape[0], _np_ptr(d), _dptr(F), _stream()))
        return F

    def csca_quadrature(self, P: torch.Tensor, ntheta: int = 0, nphi: int = 0) -> np.ndarray:
        """C_sca per right-hand side by far-field quadrature."""
        out = np.zeros(P.shape[0])
        _check(load().dda_csca_quadrature(self.h, P.shape[0], _dptr(P), int(ntheta), int(nphi), _np_ptr(out),
                                          _stream()))
        return out

    def mueller(self, P_xy: torch.Tensor, theta, phi):
        """(S [ndir, 4] complex128 = S1..S4, M [ndir, 4, 4] float64) for incidence
        along +z from the x- and y-polarised solves P_xy [2, 3, N_d]."""
        if P_xy.shape[0] != 2:
            raise ValueError("P_xy must hold the x- and y-polarised solves")
        tp = np.ascontiguousarray(np.stack([np.asarray(theta, np.float64).ravel(),
                                            np.asarray(phi, np.float64).ravel()], 1))
        n = tp.shape[0]
        S = torch.empty((n, 4), dtype=torch.complex128, device=self.dev)
        M = torch.empty((n, 4, 4), dtype=torch.float64, device=self.dev)
        _check(load().dda_mueller(self.h, _dptr(P_xy), n, _np_ptr(tp), _dptr(S), _dptr(M), _stream()))
        return S, M

    def grad_cabs_eps(self, P: torch.Tensor, S=None, **kw) -> torch.Tensor:
        opts = self.make_opts(**kw)
        nrhs = P.shape[0]
        Sa, Sp = _opt_np(S, np.float64, nrhs)
        g = torch.empty((nrhs, self.nd), dtype=torch.complex128, device=self.dev)
        _check(load().dda_grad_cabs_eps(self.h, ctypes.byref(opts), nrhs, Sp, _dptr(P), _dptr(g), _stream()))
        return g
