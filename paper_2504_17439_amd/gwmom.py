"""Thin ctypes binding of libgwmom.so (C ABI in include/gwmom.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream; the
binding allocates output tensors and passes raw device pointers.  If the
library is not built, or no HIP device is visible, construction fails
loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgwmom.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EHIP, GW_ENUMERIC, GW_ENOCONV, GW_ELIB = 0, -1, -2, -3, -4, -5, -6
GW_FP64, GW_MIXED = 0, 1
GW_TDA, GW_RPA = 0, 1

_STATUS = {GW_EINVAL: "GW_EINVAL", GW_ENOMEM: "GW_ENOMEM", GW_EHIP: "GW_EHIP",
           GW_ENUMERIC: "GW_ENUMERIC", GW_ENOCONV: "GW_ENOCONV", GW_ELIB: "GW_ELIB"}

# every symbol declared in include/gwmom.h
EXPORTS = ("gw_create", "gw_set_stream", "gw_synchronize", "gw_destroy", "gw_last_error",
           "gw_moments_tda", "gw_moments_rpa", "gw_sigma_moments", "gw_sigma_from_R", "gw_sigma_moments_noalloc",
           "gw_poles", "gw_eigh",
           "gw_fsgw", "gw_evgw", "gw_naf", "gw_qsgw", "gw_spectral", "gw_aufbau", "gw_zeta_shift", "gw_batch_create", "gw_batch_run", "gw_batch_info", "gw_batch_destroy",
           "gw_mlp_param_count", "gw_mlp_features", "gw_mlp_forward", "gw_mlp_backward",
           "gw_mlp_adam", "gw_mlp_norm", "gw_mlp_target", "gw_mlp_warm_start", "gw_timing_enable",
           "gw_timing_reset", "gw_timing_read")


class GWError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("nquad", ctypes.c_int), ("quad_scale", ctypes.c_double),
                ("pinv_tol", ctypes.c_double), ("neg_tol", ctypes.c_double),
                ("zchunk_bytes", ctypes.c_size_t),
                ("moment_eps", ctypes.c_double)]


class System(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int), ("nvir", ctypes.c_int), ("naux", ctypes.c_int),
                ("eps", ctypes.c_void_p), ("L", ctypes.c_void_p),
                ("sigma_occ", ctypes.c_void_p), ("sigma_vir", ctypes.c_void_p)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("job_bytes", ctypes.c_size_t), ("wave_bytes", ctypes.c_size_t), ("split_target", ctypes.c_int),
                ("autotune", ctypes.c_int), ("no_graph", ctypes.c_int), ("branches", ctypes.c_int),
                ("small_tile_nmo", ctypes.c_int)]


class FsgwOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("max_fock", ctypes.c_int),
                ("fock_tol", ctypes.c_double), ("diis_space", ctypes.c_int), ("zeta_tol", ctypes.c_double),
                ("zeta_lo", ctypes.c_double), ("zeta_hi", ctypes.c_double)]


class FsgwInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("fock_steps", ctypes.c_int), ("eig_calls", ctypes.c_int),
                ("converged", ctypes.c_int), ("zeta", ctypes.c_double), ("last_dqp", ctypes.c_double),
                ("last_dF", ctypes.c_double)]


class QsgwOpts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("srg_s", ctypes.c_double), ("delta", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("max_scf", ctypes.c_int),
                ("scf_tol", ctypes.c_double), ("diis_space", ctypes.c_int), ("outer_diis", ctypes.c_int)]


class QsgwInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("scf_steps", ctypes.c_int), ("converged", ctypes.c_int),
                ("last_change", ctypes.c_double)]


class AufbauInfo(ctypes.Structure):
    _fields_ = [("nfill", ctypes.c_int), ("nelec", ctypes.c_double), ("mu", ctypes.c_double),
                ("homo", ctypes.c_int), ("lumo", ctypes.c_int)]


class ZetaOpts(ctypes.Structure):
    _fields_ = [("zeta_lo", ctypes.c_double), ("zeta_hi", ctypes.c_double), ("zeta_tol", ctypes.c_double)]


class ZetaInfo(ctypes.Structure):
    _fields_ = [("zeta", ctypes.c_double), ("nfill", ctypes.c_int), ("nelec", ctypes.c_double),
                ("eig_calls", ctypes.c_int)]


class EvgwOpts(ctypes.Structure):
    _fields_ = [("g0", ctypes.c_int), ("w0", ctypes.c_int), ("max_iter", ctypes.c_int), ("tol", ctypes.c_double),
                ("diis_space", ctypes.c_int)]


class EvgwInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("last_change", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgwmom.so and declare its prototypes (no device needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2504_17439_amd.build first")
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    H = ctypes.c_void_p
    sig = {
        "gw_create": ([ctypes.POINTER(H), I], I),
        "gw_set_stream": ([H, P], I),
        "gw_synchronize": ([H], I),
        "gw_destroy": ([H], I),
        "gw_last_error": ([H], ctypes.c_char_p),
        "gw_moments_tda": ([H, I, I, I, I, P, P, I, P, P, P], I),
        "gw_moments_rpa": ([H, I, I, I, I, P, P, I, P, P, P], I),
        "gw_sigma_moments": ([H, I, I, I, I, I, P, P, I, P, P, P], I),
        "gw_sigma_from_R": ([H, I, I, I, I, P, P, P, I, P, P, P], I),
        "gw_sigma_moments_noalloc": ([H, I, I, I, I, P, P, P, P], I),
        "gw_poles": ([H, I, I, P, P, P, P, ctypes.POINTER(I), ctypes.POINTER(I), P, P, P, P, P, P], I),
        "gw_eigh": ([H, I, P, P], I),
        "gw_fsgw": ([H, I, I, I, I, I, P, P, P, I, P, P, P, P, P, P], I),
        "gw_evgw": ([H, I, I, I, I, I, P, P, I, P, P, P, P, P], I),
        "gw_naf": ([H, I, I, I, P, D, I, P, ctypes.POINTER(I), P], I),
        "gw_qsgw": ([H, I, I, I, I, I, P, P, I, P, P, P, P, P, P], I),
        "gw_spectral": ([H, I, I, I, P, P, I, P, D, P, P], I),
        "gw_aufbau": ([H, I, I, I, P, P, D, P, P], I),
        "gw_zeta_shift": ([H, I, I, I, I, P, P, P, D, P, P, P, P, P, P], I),
        "gw_batch_create": ([H, I, P, I, I, I, P, P, ctypes.POINTER(ctypes.c_void_p)], I),
        "gw_batch_run": ([P], I),
        "gw_batch_info": ([P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                          ctypes.POINTER(I)], I),
        "gw_batch_destroy": ([P], I),
        "gw_mlp_param_count": ([], ctypes.c_long),
        "gw_mlp_features": ([H, I, I, I, P, P, P], I),
        "gw_mlp_forward": ([H, I, P, P, P, P, P], I),
        "gw_mlp_backward": ([H, I, P, P, P, P, P, P, P, P], I),
        "gw_mlp_adam": ([H, I, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P, P, P, P], I),
        "gw_mlp_norm": ([H, I, P, P, P], I),
        "gw_mlp_target": ([H, I, P, P, P], I),
        "gw_mlp_warm_start": ([H, I, I, I, P, P, P, P, P], I),
        "gw_timing_enable": ([H, I], I),
        "gw_timing_reset": ([H], I),
        "gw_timing_read": ([H, ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_long)], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, Opts):
        return ctypes.byref(opts)
    o = Opts()
    for k, v in dict(opts).items():
        setattr(o, k, v)
    return ctypes.byref(o)


def _prec(p):
    return {"fp64": GW_FP64, "mixed": GW_MIXED}[p] if isinstance(p, str) else int(p)


def _check_dev(t, name, shape=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _check_rows(t, name, rows, cols):
    """float64 device matrix [rows][cols] whose rows may be strided (a column
    slice of a wider array); returns the leading dimension."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.dim() == 2):
        raise ValueError(f"{name} must be a 2-D float64 device tensor")
    if tuple(t.shape) != (rows, cols) or (cols > 1 and t.stride(1) != 1) or (rows > 1 and t.stride(0) < cols):
        raise ValueError(f"{name}: expected [{rows}][{cols}] with unit column stride")
    return max(cols, t.stride(0))


def _check_f32(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")


class Handle:
    """One library handle on one device, running on torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the library has no CPU path")
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.gw_create(ctypes.byref(h), device)
        if st != GW_OK:
            raise GWError(st, self.lib.gw_last_error(None).decode())
        self.h = h
        self._sync_stream()

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.gw_set_stream(self.h, ctypes.c_void_p(s))

    def close(self):
        if getattr(self, "h", None):
            self.lib.gw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        self._sync_stream()
        st = getattr(self.lib, name)(self.h, *args)
        if st != GW_OK:
            raise GWError(st, self.lib.gw_last_error(self.h).decode())

    def _new(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=f"cuda:{self.device}")

    # ------------------------------------------------------------------ timing
    def timing(self, enable: bool):
        self._call("gw_timing_enable", 1 if enable else 0)

    def timing_reset(self):
        self._call("gw_timing_reset")

    def timing_read(self, family: str):
        """(total_ms, launches) of one kernel family since the last reset."""
        ms, n = ctypes.c_double(0.0), ctypes.c_long(0)
        self._call("gw_timing_read", family.encode(), ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    # ------------------------------------------------------------------ moments
    def moments(self, eps, L, nocc, nmom_max, screening="tda", precision="fp64", eta=False, opts=None):
        """R[nmom_max+1][naux][naux] (and eta~[nmom_max+1][naux][ov] if eta)."""
        naux, nmo = L.shape[0], L.shape[1]
        nvir = nmo - nocc
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        R = self._new(nmom_max + 1, naux, naux)
        E = self._new(nmom_max + 1, naux, nocc * nvir) if eta else None
        fn = "gw_moments_tda" if screening == "tda" else "gw_moments_rpa"
        self._call(fn, nocc, nvir, naux, nmom_max, _ptr(eps), _ptr(L), _prec(precision), _opts(opts),
                   _ptr(R), _ptr(E))
        return (R, E) if eta else R

    def sigma_moments(self, eps, L, nocc, nmom_max, screening="tda", precision="fp64", opts=None,
                      out=None):
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        if out is None:
            so, sv = self._new(nmom_max + 1, nmo, nmo), self._new(nmom_max + 1, nmo, nmo)
        else:
            so, sv = out
        scr = GW_TDA if screening == "tda" else GW_RPA
        self._call("gw_sigma_moments", scr, nocc, nmo - nocc, naux, nmom_max, _ptr(eps), _ptr(L),
                   _prec(precision), _opts(opts), _ptr(so), _ptr(sv))
        return so, sv

    def sigma_moments_noalloc(self, eps, L, nocc, nmom_max, out=None):
        """FP64 TDA self-energy moments on the library's static scratch (the
        call allocates no device memory; outputs come from `out` or torch)."""
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        if out is None:
            so, sv = self._new(nmom_max + 1, nmo, nmo), self._new(nmom_max + 1, nmo, nmo)
        else:
            so, sv = out
            _check_dev(so, "sigma_occ", (nmom_max + 1, nmo, nmo))
            _check_dev(sv, "sigma_vir", (nmom_max + 1, nmo, nmo))
        self._call("gw_sigma_moments_noalloc", nocc, nmo - nocc, naux, nmom_max, _ptr(eps), _ptr(L), _ptr(so),
                   _ptr(sv))
        return so, sv

    def sigma_from_R(self, eps, L, R, nocc, precision="fp64", opts=None):
        naux, nmo = L.shape[0], L.shape[1]
        nmom_max = R.shape[0] - 1
        _check_dev(R, "R", (nmom_max + 1, naux, naux))
        so, sv = self._new(nmom_max + 1, nmo, nmo), self._new(nmom_max + 1, nmo, nmo)
        self._call("gw_sigma_from_R", nocc, nmo - nocc, naux, nmom_max, _ptr(eps), _ptr(L), _ptr(R),
                   _prec(precision), _opts(opts), _ptr(so), _ptr(sv))
        return so, sv

    # ------------------------------------------------------------------ fsGW
    def fsgw(self, eps, L, nocc, nmom_max, screening="tda", precision="fp64", F0=None, opts=None,
             fopts=None, allow_noconv=False):
        """Self-consistent loop; returns dict(F, qp, qp_weight, iterations, fock_steps,
        eig_calls, converged, zeta, last_dqp, last_dF)."""
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        if F0 is not None:
            _check_dev(F0, "F0", (nmo, nmo))
        F = self._new(nmo, nmo)
        qe, qw = self._new(nmo), self._new(nmo)
        fo = FsgwOpts()
        for k, v in dict(fopts or {}).items():
            setattr(fo, k, v)
        info = FsgwInfo()
        scr = GW_TDA if screening == "tda" else GW_RPA
        self._sync_stream()
        st = self.lib.gw_fsgw(self.h, scr, nocc, nmo - nocc, naux, nmom_max, _ptr(eps), _ptr(L), _ptr(F0),
                              _prec(precision), _opts(opts), ctypes.byref(fo), _ptr(F), _ptr(qe), _ptr(qw),
                              ctypes.byref(info))
        if st != GW_OK and not (st == GW_ENOCONV and allow_noconv):
            raise GWError(st, self.lib.gw_last_error(self.h).decode())
        return dict(F=F, qp=qe, qp_weight=qw, iterations=info.iterations, fock_steps=info.fock_steps,
                    eig_calls=info.eig_calls, converged=bool(info.converged), zeta=info.zeta,
                    last_dqp=info.last_dqp, last_dF=info.last_dF)

    def naf(self, L, nocc, eps_naf=1e-5, full_space=False):
        """Natural auxiliary functions: returns (L_naf [nnaf][nmo][nmo], all
        eigenvalues of M ascending)."""
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(L, "L", (naux, nmo, nmo))
        out = self._new(naux, nmo, nmo)
        w = self._new(naux)
        n = ctypes.c_int(0)
        self._sync_stream()
        self._call("gw_naf", nocc, nmo - nocc, naux, _ptr(L), ctypes.c_double(eps_naf), int(bool(full_space)),
                   _ptr(out), ctypes.byref(n), _ptr(w))
        return out[: n.value], w

    def evgw(self, eps, L, nocc, nmom_max, screening="tda", precision="fp64", g0=False, w0=False, tol=1e-6,
             max_iter=30, opts=None, allow_noconv=False, diis_space=12):
        """Eigenvalue self-consistent loop (g0 / w0 keep G / W at the reference);
        returns dict(qp, qp_weight, iterations, converged, last_change)."""
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        qe, qw = self._new(nmo), self._new(nmo)
        eo = EvgwOpts(int(bool(g0)), int(bool(w0)), int(max_iter), float(tol), int(diis_space) if diis_space else -1)
        info = EvgwInfo()
        scr = GW_TDA if screening == "tda" else GW_RPA
        self._sync_stream()
        st = self.lib.gw_evgw(self.h, scr, nocc, nmo - nocc, naux, nmom_max, _ptr(eps), _ptr(L), _prec(precision),
                              _opts(opts), ctypes.byref(eo), _ptr(qe), _ptr(qw), ctypes.byref(info))
        if st != GW_OK and not (st == GW_ENOCONV and allow_noconv):
            raise GWError(st, self.lib.gw_last_error(self.h).decode())
        return dict(qp=qe, qp_weight=qw, iterations=info.iterations, converged=bool(info.converged),
                    last_change=info.last_change)

    def qsgw(self, eps, L, nocc, nmom_max, screening="tda", precision="fp64", scheme="srg", s=500.0, delta=1e-3,
             tol=1e-6, max_iter=30, scf_tol=1e-10, max_scf=200, diis_space=12, outer_diis=12, opts=None,
             allow_noconv=False):
        """Quasiparticle self-consistent loop; returns dict(qp, C, F, iterations,
        scf_steps, converged, last_change).  outer_diis <= 0: no DIIS over the
        static potential."""
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        qe, C, F = self._new(nmo), self._new(nmo, nmo), self._new(nmo, nmo)
        qo = QsgwOpts({"srg": 0, "lorentzian": 1}[scheme], float(s), float(delta), float(tol), int(max_iter),
                      int(max_scf), float(scf_tol), int(diis_space), int(outer_diis) if outer_diis > 0 else -1)
        info = QsgwInfo()
        scr = GW_TDA if screening == "tda" else GW_RPA
        self._sync_stream()
        st = self.lib.gw_qsgw(self.h, scr, nocc, nmo - nocc, naux, nmom_max, _ptr(eps), _ptr(L), _prec(precision),
                              _opts(opts), ctypes.byref(qo), _ptr(qe), _ptr(C), _ptr(F), ctypes.byref(info))
        if st != GW_OK and not (st == GW_ENOCONV and allow_noconv):
            raise GWError(st, self.lib.gw_last_error(self.h).decode())
        return dict(qp=qe, C=C, F=F, iterations=info.iterations, scf_steps=info.scf_steps,
                    converged=bool(info.converged), last_change=info.last_change)

    # ------------------------------------------------------------------ batches
    def batch(self, systems, nmom_max, screening="tda", precision="mixed", opts=None, bopts=None):
        """systems: list of (eps, L, nocc) device tensors.  Returns a Batch whose
        .sigma[i] = (sigma_occ, sigma_vir) are filled at creation and by every run()."""
        return Batch(self, systems, nmom_max, screening, precision, opts, bopts)

    # ------------------------------------------------------------------ warm-start MLP
    def _f32(self, *shape):
        return torch.empty(*shape, dtype=torch.float32, device=f"cuda:{self.device}")

    def mlp_features(self, eps, L, nocc):
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        feat = self._f32(nmo, 3)
        self._call("gw_mlp_features", nocc, nmo - nocc, naux, _ptr(eps), _ptr(L), _ptr(feat))
        return feat

    def mlp_forward(self, params, norm, x, act=None):
        rows = x.shape[0]
        for t, n in ((params, "params"), (norm, "norm"), (x, "x")):
            _check_f32(t, n)
        y = self._f32(rows)
        self._call("gw_mlp_forward", rows, _ptr(params), _ptr(norm), _ptr(x), _ptr(act), _ptr(y))
        return y

    def mlp_backward(self, params, norm, x, act, y, target, grad=None, loss=None):
        rows = x.shape[0]
        grad = self._f32(params.shape[0]) if grad is None else grad
        self._call("gw_mlp_backward", rows, _ptr(params), _ptr(norm), _ptr(x), _ptr(act), _ptr(y), _ptr(target),
                   _ptr(grad), _ptr(loss))
        return grad

    def mlp_adam(self, step, params, grad, m, v, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._call("gw_mlp_adam", step, lr, beta1, beta2, eps, _ptr(params), _ptr(grad), _ptr(m), _ptr(v))

    def mlp_norm(self, x, target):
        rows = x.shape[0]
        _check_f32(x, "x")
        _check_f32(target, "target")
        if tuple(x.shape) != (rows, 3) or tuple(target.shape) != (rows,):
            raise ValueError("x must be [rows][3] and target [rows]")
        norm = self._f32(8)
        self._call("gw_mlp_norm", rows, _ptr(x), _ptr(target), _ptr(norm))
        return norm

    def mlp_target(self, F, eps):
        nmo = eps.shape[0]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(F, "F", (nmo, nmo))
        t = self._f32(nmo)
        self._call("gw_mlp_target", nmo, _ptr(F), _ptr(eps), _ptr(t))
        return t

    def mlp_warm_start(self, params, norm, eps, L, nocc):
        naux, nmo = L.shape[0], L.shape[1]
        _check_dev(eps, "eps", (nmo,))
        _check_dev(L, "L", (naux, nmo, nmo))
        _check_f32(params, "params")
        _check_f32(norm, "norm")
        F0 = self._new(nmo, nmo)
        self._call("gw_mlp_warm_start", nocc, nmo - nocc, naux, _ptr(eps), _ptr(L), _ptr(params), _ptr(norm),
                   _ptr(F0))
        return F0

    # ------------------------------------------------------------------ poles
    def poles(self, sigma_occ, sigma_vir, fock, opts=None, want_chi=True):
        nmom_max = sigma_occ.shape[0] - 1
        nmo = sigma_occ.shape[1]
        _check_dev(sigma_occ, "sigma_occ", (nmom_max + 1, nmo, nmo))
        _check_dev(sigma_vir, "sigma_vir", (nmom_max + 1, nmo, nmo))
        _check_dev(fock, "fock", (nmo, nmo))
        cap = nmo * (nmom_max + 1) // 2
        dim_max = nmo * (nmom_max + 2)
        pe, pv = self._new(2 * cap), self._new(nmo, 2 * cap)
        E = self._new(dim_max)
        chi = self._new(nmo, dim_max) if want_chi else None
        qe, qw = self._new(nmo), self._new(nmo)
        no, nv = ctypes.c_int(0), ctypes.c_int(0)
        self._call("gw_poles", nmo, nmom_max, _ptr(sigma_occ), _ptr(sigma_vir), _ptr(fock), _opts(opts),
                   ctypes.byref(no), ctypes.byref(nv), _ptr(pe), _ptr(pv), _ptr(E), _ptr(chi), _ptr(qe),
                   _ptr(qw))
        no, nv = no.value, nv.value
        dim = nmo + no + nv
        return dict(e_occ=pe[:no], v_occ=pv[:, :no], e_vir=pe[no:no + nv], v_vir=pv[:, no:no + nv],
                    E=E[:dim], chi=None if chi is None else chi[:, :dim], qp=qe, qp_weight=qw,
                    packed=(pe, pv, no, nv, nmom_max))

    def eigh(self, A):
        """(w [n] ascending, V [n][n]) of the symmetric A [n][n] (row i of V is
        eigenvector i); A itself is left unchanged."""
        n = A.shape[0]
        _check_dev(A, "A", (n, n))
        V = A.clone()
        w = self._new(n)
        self._call("gw_eigh", n, _ptr(V), _ptr(w))
        return w, V

    # ------------------------------------------------------------------ Green's function
    def spectral(self, E, chi, omega, delta, per_orbital=False):
        """A(omega) (and A_p(omega) [nmo][nomega] if per_orbital) from the
        eigenpairs of H~ (E [dim], chi [nmo][dim], rows may be strided)."""
        dim = E.shape[0]
        nmo = chi.shape[0]
        _check_dev(E, "E", (dim,))
        _check_dev(omega, "omega", (omega.shape[0],))
        ld = _check_rows(chi, "chi", nmo, dim)
        nw = omega.shape[0]
        A = self._new(nw)
        Ap = self._new(nmo, nw) if per_orbital else None
        self._call("gw_spectral", nmo, dim, ld, _ptr(E), _ptr(chi), nw, _ptr(omega), ctypes.c_double(delta),
                   _ptr(A), _ptr(Ap))
        return (A, Ap) if per_orbital else A

    def aufbau(self, E, chi, nelec):
        """Aufbau filling of H~'s eigenstates: dict(rho, nfill, nelec, mu, homo, lumo)."""
        dim = E.shape[0]
        nmo = chi.shape[0]
        _check_dev(E, "E", (dim,))
        ld = _check_rows(chi, "chi", nmo, dim)
        rho = self._new(nmo, nmo)
        info = AufbauInfo()
        self._call("gw_aufbau", nmo, dim, ld, _ptr(E), _ptr(chi), ctypes.c_double(nelec), _ptr(rho),
                   ctypes.byref(info))
        return dict(rho=rho, nfill=info.nfill, nelec=info.nelec, mu=info.mu, homo=info.homo, lumo=info.lumo)

    def zeta_shift(self, poles, fock, nelec, zeta_lo=0.0, zeta_hi=0.0, zeta_tol=0.0):
        """Electron-number conserving one-shot GW from the output of poles():
        dict(E, chi, qp, qp_weight, zeta, nfill, nelec, eig_calls)."""
        pe, pv, no, nv, nmom_max = poles["packed"]
        nmo = pv.shape[0]
        _check_dev(fock, "fock", (nmo, nmo))
        dim_max = nmo * (nmom_max + 2)
        E, chi = self._new(dim_max), self._new(nmo, dim_max)
        qe, qw = self._new(nmo), self._new(nmo)
        zo = ZetaOpts(float(zeta_lo), float(zeta_hi), float(zeta_tol))
        info = ZetaInfo()
        self._call("gw_zeta_shift", nmo, nmom_max, no, nv, _ptr(fock), _ptr(pe), _ptr(pv), ctypes.c_double(nelec),
                   ctypes.byref(zo), _ptr(E), _ptr(chi), _ptr(qe), _ptr(qw), ctypes.byref(info))
        dim = nmo + no + nv
        return dict(E=E[:dim], chi=chi[:, :dim], qp=qe, qp_weight=qw, zeta=info.zeta, nfill=info.nfill,
                    nelec=info.nelec, eig_calls=info.eig_calls)


class Batch:
    """A planned batch (gw_batch): the tensors it reads and writes stay referenced here."""

    def __init__(self, handle, systems, nmom_max, screening, precision, opts, bopts):
        self.handle = handle
        self.inputs = []
        self.sigma = []
        arr = (System * len(systems))()
        for i, (eps, L, nocc) in enumerate(systems):
            naux, nmo = L.shape[0], L.shape[1]
            _check_dev(eps, "eps", (nmo,))
            _check_dev(L, "L", (naux, nmo, nmo))
            so, sv = handle._new(nmom_max + 1, nmo, nmo), handle._new(nmom_max + 1, nmo, nmo)
            self.inputs.append((eps, L))
            self.sigma.append((so, sv))
            arr[i] = System(nocc, nmo - nocc, naux, eps.data_ptr(), L.data_ptr(), so.data_ptr(), sv.data_ptr())
        bo = BatchOpts()
        for k, v in dict(bopts or {}).items():
            setattr(bo, k, v)
        self.b = ctypes.c_void_p()
        scr = GW_TDA if screening == "tda" else GW_RPA
        handle._call("gw_batch_create", len(systems), ctypes.cast(arr, ctypes.c_void_p), scr, nmom_max,
                     _prec(precision), _opts(opts), ctypes.byref(bo), ctypes.byref(self.b))

    def run(self):
        self.handle._sync_stream()
        st = self.handle.lib.gw_batch_run(self.b)
        if st != GW_OK:
            raise GWError(st, self.handle.lib.gw_last_error(self.handle.h).decode())

    def info(self):
        v = [ctypes.c_int(0) for _ in range(5)]
        self.handle.lib.gw_batch_info(self.b, *[ctypes.byref(x) for x in v])
        return dict(jobs=v[0].value, waves=v[1].value, graph=bool(v[2].value), split_target=v[3].value,
                    small_tile_nmo=v[4].value)

    def close(self):
        if getattr(self, "b", None) and self.b.value:
            self.handle.lib.gw_batch_destroy(self.b)
            self.b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
