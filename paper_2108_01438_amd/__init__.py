"""MI355X-native MBIR for spectral-domain OCT: Python binding of liboct.

Every step of the operator, its adjoint, the proximal steps and FISTA runs in
the HIP kernels of liboct.so; this module only marshals arguments.  PyTorch
provides device memory and streams.  There is no CPU fallback: if the
library is missing the import raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboct.so")

OCT_OK, OCT_E_INVALID, OCT_E_NOMEM, OCT_E_DEVICE, OCT_E_UNSUPPORTED = range(5)
PEN_L1, PEN_TV, PEN_HAAR, PEN_DTCWT = 0, 1, 2, 3
PENALTIES = {"l1": PEN_L1, "tv": PEN_TV, "haar": PEN_HAAR, "dtcwt": PEN_DTCWT}
# direct reconstructions of Sec. 3.1 (oct_direct_kind)
DIRECT = {"axial": 0, "dispersion": 1, "isam": 2, "interp_isam": 3}
# oct_solve_flags
SOLVE_PAPER_BACKWARD = 1


class OctError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"liboct status {status}: {msg}")
        self.status = status


class _CGeometry(ctypes.Structure):
    _fields_ = [("lateral_dims", ctypes.c_int32), ("kb_width", ctypes.c_int32),
                ("n_depth", ctypes.c_int64), ("n_x", ctypes.c_int64), ("n_y", ctypes.c_int64),
                ("n_k", ctypes.c_int64), ("batch", ctypes.c_int64),
                ("k_min", ctypes.c_double), ("k_max", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("z_focus", ctypes.c_double), ("beam_waist", ctypes.c_double),
                ("disp_a", ctypes.c_double), ("disp_b", ctypes.c_double),
                ("oversamp", ctypes.c_double), ("kb_beta", ctypes.c_double), ("model", ctypes.c_int32)]


class _CSolveParams(ctypes.Structure):
    _fields_ = [("penalty", ctypes.c_int32), ("iters", ctypes.c_int32), ("tv_inner", ctypes.c_int32),
                ("haar_levels", ctypes.c_int32), ("power_iters", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("seed", ctypes.c_uint64), ("lambda_", ctypes.c_double),
                ("delta", ctypes.c_double), ("bound", ctypes.c_double), ("x0", ctypes.c_void_p),
                ("lambda_item", ctypes.POINTER(ctypes.c_double)), ("z_prev0", ctypes.c_void_p),
                ("z_prev_out", ctypes.c_void_p), ("k0", ctypes.c_int32)]


class _CSolveReport(ctypes.Structure):
    _fields_ = [("delta_used", ctypes.c_double), ("lipschitz_est", ctypes.c_double),
                ("objective", ctypes.POINTER(ctypes.c_double))]


def _load():
    # torch brings its own HIP runtime (soname libamdhip64.so.7); loading it
    # first makes liboct bind to that same runtime instead of a second copy.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2108_01438_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    sig = {
        "oct_plan_create": ([ctypes.POINTER(_CGeometry), P, ctypes.POINTER(P)], ctypes.c_int),
        "oct_plan_destroy": ([P], ctypes.c_int),
        "oct_plan_release": ([P], ctypes.c_int),
        "oct_plan_footprint_bytes": ([ctypes.POINTER(_CGeometry), ctypes.c_int32], ctypes.c_size_t),
        "oct_forward": ([P, P, P, P], ctypes.c_int),
        "oct_adjoint": ([P, P, P, P], ctypes.c_int),
        "oct_adjoint_paper": ([P, P, P, P], ctypes.c_int),
        "oct_dtcwt_filter": ([ctypes.c_int32, P, P], ctypes.c_int),
        "oct_grad": ([P, P, P, P, P, P], ctypes.c_int),
        "oct_prox": ([P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                      ctypes.c_double, P, P, P, P], ctypes.c_int),
        "oct_lipschitz": ([P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), P],
                          ctypes.c_int),
        "oct_mbir_solve": ([P, P, ctypes.POINTER(_CSolveParams), P, ctypes.POINTER(_CSolveReport), P],
                           ctypes.c_int),
        "oct_run_stage": ([P, ctypes.c_int32, ctypes.c_int32, P, P], ctypes.c_int),
        "oct_direct": ([P, ctypes.c_int32, P, P, P], ctypes.c_int),
        "oct_ncc": ([P, P, P, ctypes.POINTER(ctypes.c_double), P], ctypes.c_int),
        "oct_ncc_noalloc": ([P, P, ctypes.c_int64, P, P], ctypes.c_int),
        "oct_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def last_error() -> str:
    return _lib.oct_last_error().decode()


def _check(status: int):
    if status != OCT_OK:
        raise OctError(status, last_error())


@dataclass
class Geometry:
    """Acquisition geometry (field meanings as in include/oct.h)."""
    n_depth: int
    n_x: int
    n_k: int
    n_y: int = 1
    lateral_dims: int = 1
    batch: int = 1
    k_min: float = 2.0 * np.pi / 0.9
    k_max: float = 2.0 * np.pi / 0.75
    dx: float = 2.0
    dy: float = 2.0
    dz: float = 0.0
    z_focus: float = -1.0
    beam_waist: float = 5.0
    disp_a: float = 1e-3
    disp_b: float = 0.0
    kb_width: int = 6
    oversamp: float = 2.0
    kb_beta: float = 0.0
    model: int = 0            # 0: NUFFT at every detector wavenumber; 1: the literal K, Q, D chain (n_k = 2 n_depth)

    @classmethod
    def from_dict(cls, d: dict) -> "Geometry":
        names = {f.name for f in fields(cls)}
        return cls(**{k: v for k, v in d.items() if k in names})

    def to_c(self) -> _CGeometry:
        return _CGeometry(self.lateral_dims, self.kb_width, self.n_depth, self.n_x, self.n_y, self.n_k,
                          self.batch, self.k_min, self.k_max, self.dx, self.dy, self.dz, self.z_focus,
                          self.beam_waist, self.disp_a, self.disp_b, self.oversamp, self.kb_beta, self.model)

    @property
    def img_shape(self):
        return (self.batch, self.n_y, self.n_x, self.n_depth)

    @property
    def meas_shape(self):
        return (self.batch, self.n_y, self.n_x, self.n_k)


def dtcwt_filter(which: int) -> np.ndarray:
    """Lowpass analysis filter of the DT-CWT as the library designed it
    (0/1: first level, tree a/b; 2/3: later levels, tree a/b)."""
    taps = (ctypes.c_float * 16)()
    n = ctypes.c_int32()
    _check(_lib.oct_dtcwt_filter(int(which), taps, ctypes.byref(n)))
    return np.array(taps[:n.value], dtype=np.float64)


def footprint_bytes(geom: Geometry, penalty: int = PEN_L1) -> int:
    g = geom.to_c()
    return int(_lib.oct_plan_footprint_bytes(ctypes.byref(g), int(penalty)))


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def ncc_noalloc(x, z, r_out, stream=None):
    """NCC of magnitudes (eq. (17)) of the device complex64 arrays x and z
    (same number of elements) into the float64 device scalar r_out, without a
    plan and without any allocation in the library (oct_ncc_noalloc).
    Asynchronous; returns r_out."""
    import torch
    if x.shape != z.shape:
        raise ValueError("x and z must have the same shape")
    n = x.numel()
    _check(_lib.oct_ncc_noalloc(_dev(x, torch.complex64, x.shape, "x"), _dev(z, torch.complex64, x.shape, "z"),
                                ctypes.c_int64(n), _dev(r_out, torch.float64, (), "r_out"),
                                ctypes.c_void_p(_stream_ptr(stream))))
    return r_out


class Plan:
    """A liboct plan: tables and workspace for one geometry and mask."""

    def __init__(self, geom: Geometry, mask=None):
        self.geom = geom
        g = geom.to_c()
        h = ctypes.c_void_p()
        if mask is not None:
            m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
            if m.shape != (geom.n_y, geom.n_x, geom.n_k):
                raise ValueError(f"mask must have shape {(geom.n_y, geom.n_x, geom.n_k)}")
            self._mask = m
            mp = m.ctypes.data_as(ctypes.c_void_p)
        else:
            self._mask = None
            mp = None
        _check(_lib.oct_plan_create(ctypes.byref(g), mp, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.oct_plan_destroy(self._h)
            self._h = None

    def release(self):
        """Free the plan without synchronising the device (oct_plan_release):
        only when every call using it has completed."""
        if getattr(self, "_h", None):
            _lib.oct_plan_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- operators -------------------------------------------------------
    def forward(self, x, y=None, stream=None):
        import torch
        g = self.geom
        if y is None:
            y = torch.empty(g.meas_shape, dtype=torch.float32, device=x.device)
        _check(_lib.oct_forward(self._h, _dev(x, torch.complex64, g.img_shape, "x"),
                                _dev(y, torch.float32, g.meas_shape, "y"), ctypes.c_void_p(_stream_ptr(stream))))
        return y

    def adjoint(self, r, x=None, stream=None):
        import torch
        g = self.geom
        if x is None:
            x = torch.empty(g.img_shape, dtype=torch.complex64, device=r.device)
        _check(_lib.oct_adjoint(self._h, _dev(r, torch.float32, g.meas_shape, "r"),
                                _dev(x, torch.complex64, g.img_shape, "x"), ctypes.c_void_p(_stream_ptr(stream))))
        return x

    def adjoint_paper(self, r, x=None, stream=None):
        """x = Phi* r, the backward operator of eq. (10)-(11) (conjugate analytic
        signal along k in place of the real part's adjoint)."""
        import torch
        g = self.geom
        if x is None:
            x = torch.empty(g.img_shape, dtype=torch.complex64, device=r.device)
        _check(_lib.oct_adjoint_paper(self._h, _dev(r, torch.float32, g.meas_shape, "r"),
                                      _dev(x, torch.complex64, g.img_shape, "x"),
                                      ctypes.c_void_p(_stream_ptr(stream))))
        return x

    def direct(self, y, kind: str, x=None, stream=None):
        """Direct reconstruction of the measurement y: "axial" (IFFT),
        "dispersion" (dispersion corrected), "isam" or "interp_isam"."""
        import torch
        g = self.geom
        if kind not in DIRECT:
            raise ValueError(f"unknown direct reconstruction {kind!r}; one of {sorted(DIRECT)}")
        if x is None:
            x = torch.empty(g.img_shape, dtype=torch.complex64, device=y.device)
        _check(_lib.oct_direct(self._h, DIRECT[kind], _dev(y, torch.float32, g.meas_shape, "y"),
                               _dev(x, torch.complex64, g.img_shape, "x"), ctypes.c_void_p(_stream_ptr(stream))))
        return x

    def ncc(self, x, z, stream=None) -> float:
        """Normalised cross-correlation of magnitudes of x against the reference z (eq. (17))."""
        import torch
        g = self.geom
        r = ctypes.c_double(0.0)
        _check(_lib.oct_ncc(self._h, _dev(x, torch.complex64, g.img_shape, "x"),
                            _dev(z, torch.complex64, g.img_shape, "z"), ctypes.byref(r),
                            ctypes.c_void_p(_stream_ptr(stream))))
        return float(r.value)

    def grad(self, x, y, g_out=None, resid=None, stream=None):
        """Returns (g, half_resid_sq) with half_resid_sq a float64 device scalar tensor."""
        import torch
        g = self.geom
        if g_out is None:
            g_out = torch.empty(g.img_shape, dtype=torch.complex64, device=x.device)
        if resid is None:
            resid = torch.empty((), dtype=torch.float64, device=x.device)
        _check(_lib.oct_grad(self._h, _dev(x, torch.complex64, g.img_shape, "x"),
                             _dev(y, torch.float32, g.meas_shape, "y"),
                             _dev(g_out, torch.complex64, g.img_shape, "g"),
                             _dev(resid, torch.float64, (), "resid"), ctypes.c_void_p(_stream_ptr(stream))))
        return g_out, resid

    def prox(self, penalty, lam: float, delta: float, v, z=None, state=None, tv_inner: int = 10,
             haar_levels: int = 3, bound=None, stream=None):
        """z = prox_{lam delta R}(v) over C = {|x_i| <= bound} (bound None: no constraint)."""
        import torch
        g = self.geom
        pen = PENALTIES[penalty] if isinstance(penalty, str) else int(penalty)
        if z is None:
            z = torch.empty(g.img_shape, dtype=torch.complex64, device=v.device)
        sp = None
        if state is not None:
            sp = _dev(state, torch.complex64, (g.lateral_dims + 1,) + g.img_shape, "state")
        _check(_lib.oct_prox(self._h, pen, float(lam), float(delta), int(tv_inner), int(haar_levels),
                             0.0 if bound is None else float(bound), _dev(v, torch.complex64, g.img_shape, "v"), _dev(z, torch.complex64, g.img_shape, "z"),
                             sp, ctypes.c_void_p(_stream_ptr(stream))))
        return z

    STAGES = ("lat_fwd", "nufft_fwd", "normal", "nufft_adj", "lat_update", "prox", "nufft_normal")

    def run_stage(self, stage, penalty="tv", y=None, stream=None):
        """One stage of a FISTA iteration on the plan's workspace (timing only)."""
        import torch
        st = self.STAGES.index(stage) if isinstance(stage, str) else int(stage)
        pen = PENALTIES[penalty] if isinstance(penalty, str) else int(penalty)
        yp = None if y is None else _dev(y, torch.float32, self.geom.meas_shape, "y")
        _check(_lib.oct_run_stage(self._h, st, pen, yp, ctypes.c_void_p(_stream_ptr(stream))))

    def lipschitz(self, iters: int = 50, seed: int = 0, paper_backward: bool = False, stream=None) -> float:
        """Power iteration on Phi^H Phi (on Phi* Phi with paper_backward=True)."""
        out = ctypes.c_double()
        flags = SOLVE_PAPER_BACKWARD if paper_backward else 0
        _check(_lib.oct_lipschitz(self._h, int(iters), ctypes.c_uint64(seed), flags, ctypes.byref(out),
                                  ctypes.c_void_p(_stream_ptr(stream))))
        return out.value

    def mbir_solve(self, y, penalty, lam, iters: int, delta: float = 0.0, tv_inner: int = 10,
                   haar_levels: int = 3, power_iters: int = 50, seed: int = 0, x0=None, x_out=None,
                   objective: bool = False, paper_backward: bool = False, bound=None, stream=None,
                   z_prev0=None, k0: int = 0, z_prev_out=None):
        """FISTA; returns (z^K, info) with info = {delta, lipschitz, objective (np.ndarray or None)}.
        paper_backward=True takes each gradient with the backward operator of
        eq. (10)-(11) (adjoint_paper) instead of the exact adjoint; bound sets the
        constraint set C = {|x_i| <= bound} of the prox (l1, TV; None: none).
        lam: one weight, or a sequence of one weight per batch item.
        Resume: x0 = z^k0, z_prev0 = z^{k0-1}, k0 = iterations already done
        (z_prev_out receives z^{K-1} of this solve)."""
        import torch
        g = self.geom
        pen = PENALTIES[penalty] if isinstance(penalty, str) else int(penalty)
        if x_out is None:
            x_out = torch.empty(g.img_shape, dtype=torch.complex64, device=y.device)
        lam_item = None
        if np.ndim(lam) > 0:
            lam_item = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
            if lam_item.shape != (g.batch,):
                raise ValueError(f"per-item weights must have shape ({g.batch},)")
            lam = 0.0
        prm = _CSolveParams(pen, int(iters), int(tv_inner), int(haar_levels), int(power_iters),
                            SOLVE_PAPER_BACKWARD if paper_backward else 0,
                            int(seed), float(lam), float(delta), 0.0 if bound is None else float(bound),
                            None if x0 is None else _dev(x0, torch.complex64, g.img_shape, "x0").value,
                            None if lam_item is None else lam_item.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            None if z_prev0 is None else _dev(z_prev0, torch.complex64, g.img_shape, "z_prev0").value,
                            None if z_prev_out is None else _dev(z_prev_out, torch.complex64, g.img_shape,
                                                                 "z_prev_out").value,
                            int(k0))
        obj = np.zeros(iters, dtype=np.float64) if objective else None
        rep = _CSolveReport(0.0, 0.0, obj.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if objective else None)
        _check(_lib.oct_mbir_solve(self._h, _dev(y, torch.float32, g.meas_shape, "y"), ctypes.byref(prm),
                                   _dev(x_out, torch.complex64, g.img_shape, "x_out"), ctypes.byref(rep),
                                   ctypes.c_void_p(_stream_ptr(stream))))
        return x_out, dict(delta=rep.delta_used, lipschitz=rep.lipschitz_est, objective=obj)


__all__ = ["Geometry", "Plan", "OctError", "footprint_bytes", "last_error", "LIB_PATH", "ncc_noalloc",
           "PEN_L1", "PEN_TV", "PEN_HAAR", "PEN_DTCWT", "PENALTIES", "dtcwt_filter", "DIRECT", "SOLVE_PAPER_BACKWARD"]
