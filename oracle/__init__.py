"""FP64 CPU oracle of the coupled lattice-Boltzmann ice-growth step (Tan et al., arXiv:2101.07163).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the GPU library never does, and this package imports nothing from the GPU library.

The forward step lives in ``snow_oracle.c`` (plain C, FP64, OpenMP over rows); this module is the
ctypes marshalling around it plus the oracle's own parameter struct.  Population arrays use the
canonical layout ``[q, y, x]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsnow_oracle.so")
_SOURCES = ["snow_oracle.c", "snow_oracle_adj.c", "snow_oracle3d.c"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_SO):
        return _SO
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("flow", ctypes.c_int32),
        ("inout", ctypes.c_int32), ("n_fold", ctypes.c_int32), ("stencil", ctypes.c_int32),
        ("eps", ctypes.c_double), ("W0", ctypes.c_double), ("tau0", ctypes.c_double),
        ("lam", ctypes.c_double), ("L_sat", ctypes.c_double), ("tau_vap", ctypes.c_double),
        ("tau_f", ctypes.c_double), ("h_drag", ctypes.c_double), ("kappa_N", ctypes.c_double),
        ("rho0", ctypes.c_double), ("u_in", ctypes.c_double), ("U_in", ctypes.c_double),
        ("grad_eps2", ctypes.c_double), ("symmetric", ctypes.c_int32), ("pad_", ctypes.c_int32),
    ]


class Orc3Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("flow", ctypes.c_int32), ("inout", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("eps", ctypes.c_double), ("W0", ctypes.c_double), ("tau0", ctypes.c_double),
        ("lam", ctypes.c_double), ("L_sat", ctypes.c_double), ("tau_vap", ctypes.c_double),
        ("tau_f", ctypes.c_double), ("h_drag", ctypes.c_double), ("kappa_N", ctypes.c_double),
        ("rho0", ctypes.c_double), ("u_in", ctypes.c_double), ("U_in", ctypes.c_double),
        ("grad_eps2", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        d = ctypes.c_double
        dp = P(d)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [P(OrcParams)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_init_seed.argtypes = [ctypes.c_void_p, d, d, d, d, d, ctypes.c_void_p]
        L.orc_set_state.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        L.orc_get_state.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc_step_count.restype = ctypes.c_int64
        L.orc_step_count.argtypes = [ctypes.c_void_p]
        L.orc_fields.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
        L.orc_diag.argtypes = [ctypes.c_void_p, dp]
        L.orc_feq.argtypes = [d, d, d, dp]
        L.orc_geq.argtypes = [d, d, d, dp]
        L.orc_guo.argtypes = [P(OrcParams), d, d, d, d, dp]
        L.orc_aniso.argtypes = [P(OrcParams), d, d, dp, dp, dp]
        L.orc_grad.argtypes = [P(OrcParams), dp, dp, dp]
        L.orc_threads.restype = ctypes.c_int32
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_adj_run.restype = d
        L.orc_adj_run.argtypes = [P(OrcParams), d, d, d, d, dp, dp, ctypes.c_int32, ctypes.c_int32, dp, dp,
                                  ctypes.c_void_p]
        L.orc_loss.restype = d
        L.orc_loss.argtypes = [P(OrcParams), d, d, d, d, dp, dp, ctypes.c_int32, ctypes.c_void_p]
        # three dimensions
        L.orc3_create.restype = ctypes.c_void_p
        L.orc3_create.argtypes = [P(Orc3Params)]
        L.orc3_destroy.argtypes = [ctypes.c_void_p]
        L.orc3_init_seed.argtypes = [ctypes.c_void_p, d, d, d, d, d, d, ctypes.c_void_p]
        L.orc3_set_state.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        L.orc3_get_state.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        L.orc3_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc3_step_count.restype = ctypes.c_int64
        L.orc3_step_count.argtypes = [ctypes.c_void_p]
        L.orc3_fields.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
        L.orc3_diag.argtypes = [ctypes.c_void_p, dp]
        L.orc3_feq.argtypes = [d, d, d, d, dp]
        L.orc3_geq.argtypes = [d, d, d, d, dp]
        L.orc3_aniso.argtypes = [P(Orc3Params), d, d, d, dp, dp, dp, dp]
        L.orc3_grad.argtypes = [P(Orc3Params), dp, dp, dp, dp]
        L.orc3_lattice.argtypes = [P(ctypes.c_int32), dp, dp]
        _lib = L
    return _lib


@dataclass
class Params:
    """Oracle parameter set (lattice units).  Field names follow the paper's symbols."""
    nx: int = 128
    ny: int = 128
    flow: int = 0
    inout: int = 0
    n_fold: int = 6
    stencil: int = 4      # isotropic gradient: 2 (central difference), 4, 6, 8 (Table 1)
    symmetric: int = 0    # 1: diffusivity q = 1 in both phases (thermal model of Sec. 3.1.1)
    eps: float = 0.05
    W0: float = 1.0
    tau0: float = 10.0
    lam: float = 3.0
    L_sat: float = 1.6
    tau_vap: float = 0.8
    tau_f: float = 0.6
    h_drag: float = 2.757
    kappa_N: float = 1.0
    rho0: float = 1.0
    u_in: float = 0.0
    U_in: float = 0.0
    grad_eps2: float = 1e-10

    @classmethod
    def from_dict(cls, d: dict) -> "Params":
        names = {f.name for f in fields(cls)}
        return cls(**{k: v for k, v in d.items() if k in names})

    def c_struct(self) -> OrcParams:
        s = OrcParams()
        for f in fields(self):
            setattr(s, f.name, getattr(self, f.name))
        return s


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """One FP64 lattice.  ``Oracle(params).init_seed(...).step(n)`` then ``fields()``."""

    def __init__(self, params: Params):
        self.p = params
        self._cp = params.c_struct()
        self._h = lib().orc_create(ctypes.byref(self._cp))
        if not self._h:
            raise ValueError("oracle: invalid parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().orc_destroy(h)
            except Exception:  # interpreter shutdown: module globals may already be gone
                pass
            self._h = None

    @property
    def shape(self):
        return (self.p.ny, self.p.nx)

    def init_seed(self, xs, ys, R, w_init=1.0, U0=0.5, U_init: np.ndarray | None = None):
        Ui = None if U_init is None else np.ascontiguousarray(U_init, dtype=np.float64)
        if Ui is not None:
            assert Ui.shape == self.shape
        lib().orc_init_seed(self._h, float(xs), float(ys), float(R), float(w_init), float(U0),
                            _ptr(Ui))
        return self

    def set_state(self, f=None, g=None, h=None, phip=None):
        conv = lambda a, q: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(
            (q,) + self.shape if q else self.shape)
        f, g, h, phip = conv(f, 9), conv(g, 5), conv(h, 9), conv(phip, 0)
        lib().orc_set_state(self._h, _ptr(f), _ptr(g), _ptr(h), _ptr(phip))
        return self

    def get_state(self):
        ny, nx = self.shape
        f = np.empty((9, ny, nx)); g = np.empty((5, ny, nx)); h = np.empty((9, ny, nx))
        phip = np.empty((ny, nx))
        lib().orc_get_state(self._h, _ptr(f), _ptr(g), _ptr(h), _ptr(phip))
        return {"f": f, "g": g, "h": h, "phip": phip}

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))
        return self

    @property
    def step_count(self) -> int:
        return int(lib().orc_step_count(self._h))

    def fields(self) -> dict:
        ny, nx = self.shape
        out = {k: np.empty((ny, nx)) for k in ("phi", "U", "rho", "ux", "uy")}
        lib().orc_fields(self._h, *(_ptr(out[k]) for k in ("phi", "U", "rho", "ux", "uy")))
        return out

    def diag(self) -> dict:
        a = np.zeros(8)
        lib().orc_diag(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        keys = ("rho", "jx", "jy", "U", "phi", "phi_prev", "n_solid", "n_nonfinite")
        d = dict(zip(keys, a.tolist()))
        d["species"] = d["U"] + 0.5 * self.p.L_sat * d["phi_prev"]
        return d


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Number of OpenMP threads of the following oracle calls."""
    lib().orc_set_threads(int(n))


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_feq(rho, ux, uy, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def geq(U, ux, uy):
    out = np.zeros(5)
    lib().orc_geq(U, ux, uy, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def guo(params: Params, ux, uy, Fx, Fy):
    out = np.zeros(9)
    cp = params.c_struct()
    lib().orc_guo(ctypes.byref(cp), ux, uy, Fx, Fy, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def aniso(params: Params, gx, gy):
    a, nx_, ny_ = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    cp = params.c_struct()
    lib().orc_aniso(ctypes.byref(cp), gx, gy, ctypes.byref(a), ctypes.byref(nx_), ctypes.byref(ny_))
    return a.value, nx_.value, ny_.value


def grad(params: Params, phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    assert phi.shape == (params.ny, params.nx)
    gx = np.empty_like(phi); gy = np.empty_like(phi)
    cp = params.c_struct()
    P = ctypes.POINTER(ctypes.c_double)
    lib().orc_grad(ctypes.byref(cp), phi.ctypes.data_as(P), gx.ctypes.data_as(P), gy.ctypes.data_as(P))
    return gx, gy


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def adjoint(params: Params, seed, w_init, U_init, phi_target, nsteps, stride=0):
    """Loss L = sum (phi_T - phi_target)^2 after nsteps (no flow, periodic) and its FP64 discrete
    adjoint gradients: returns (L, dL/dU_init [ny, nx], dL/deps, phi_T)."""
    U = np.ascontiguousarray(U_init, dtype=np.float64)
    T = np.ascontiguousarray(phi_target, dtype=np.float64)
    assert U.shape == (params.ny, params.nx) and T.shape == U.shape
    gU = np.zeros_like(U)
    ge = ctypes.c_double()
    phiT = np.zeros_like(U)
    cp = params.c_struct()
    xs, ys, R = seed
    L = lib().orc_adj_run(ctypes.byref(cp), xs, ys, R, w_init, _dp(U), _dp(T), int(nsteps), int(stride),
                          _dp(gU), ctypes.byref(ge), phiT.ctypes.data_as(ctypes.c_void_p))
    return L, gU, ge.value, phiT


def loss(params: Params, seed, w_init, U_init, phi_target, nsteps):
    U = np.ascontiguousarray(U_init, dtype=np.float64)
    T = np.ascontiguousarray(phi_target, dtype=np.float64)
    cp = params.c_struct()
    xs, ys, R = seed
    return lib().orc_loss(ctypes.byref(cp), xs, ys, R, w_init, _dp(U), _dp(T), int(nsteps), None)


def final_phi(params: Params, seed, w_init, U_init, nsteps):
    U = np.ascontiguousarray(U_init, dtype=np.float64)
    T = np.zeros_like(U)
    out = np.zeros_like(U)
    cp = params.c_struct()
    xs, ys, R = seed
    lib().orc_loss(ctypes.byref(cp), xs, ys, R, w_init, _dp(U), _dp(T), int(nsteps),
                   out.ctypes.data_as(ctypes.c_void_p))
    return out


# ----------------------------------------------------------------------------- three dimensions

@dataclass
class Params3D:
    """Parameters of the three-dimensional oracle (lattice units; see snow_oracle3d.c)."""
    nx: int = 32
    ny: int = 32
    nz: int = 32
    flow: int = 0
    inout: int = 0
    eps: float = 0.05
    W0: float = 1.0
    tau0: float = 10.0
    lam: float = 3.0
    L_sat: float = 1.6
    tau_vap: float = 0.8
    tau_f: float = 0.6
    h_drag: float = 2.757
    kappa_N: float = 1.0
    rho0: float = 1.0
    u_in: float = 0.0
    U_in: float = 0.0
    grad_eps2: float = 1e-10

    @classmethod
    def from_dict(cls, d: dict) -> "Params3D":
        names = {f.name for f in fields(cls)}
        return cls(**{k: v for k, v in d.items() if k in names})

    def c_struct(self) -> Orc3Params:
        s = Orc3Params()
        for f in fields(self):
            setattr(s, f.name, getattr(self, f.name))
        return s


class Oracle3D:
    """One FP64 3D lattice: ``Oracle3D(params).init_seed(...).step(n)`` then ``fields()``.  Arrays are
    [z, y, x] fields and [q, z, y, x] populations."""

    def __init__(self, params: Params3D):
        self.p = params
        self._cp = params.c_struct()
        self._h = lib().orc3_create(ctypes.byref(self._cp))
        if not self._h:
            raise ValueError("oracle: invalid parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().orc3_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    @property
    def shape(self):
        return (self.p.nz, self.p.ny, self.p.nx)

    def init_seed(self, xs, ys, zs, R, w_init=1.0, U0=0.5, U_init: np.ndarray | None = None):
        Ui = None if U_init is None else np.ascontiguousarray(U_init, dtype=np.float64)
        if Ui is not None:
            assert Ui.shape == self.shape
        lib().orc3_init_seed(self._h, float(xs), float(ys), float(zs), float(R), float(w_init), float(U0), _ptr(Ui))
        return self

    def set_state(self, f=None, g=None, h=None, phip=None):
        conv = lambda a, q: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(
            (q,) + self.shape if q else self.shape)
        f, g, h, phip = conv(f, 19), conv(g, 7), conv(h, 7), conv(phip, 0)
        lib().orc3_set_state(self._h, _ptr(f), _ptr(g), _ptr(h), _ptr(phip))
        return self

    def get_state(self):
        f = np.empty((19,) + self.shape); g = np.empty((7,) + self.shape); h = np.empty((7,) + self.shape)
        phip = np.empty(self.shape)
        lib().orc3_get_state(self._h, _ptr(f), _ptr(g), _ptr(h), _ptr(phip))
        return {"f": f, "g": g, "h": h, "phip": phip}

    def step(self, n: int = 1):
        lib().orc3_step(self._h, int(n))
        return self

    @property
    def step_count(self) -> int:
        return int(lib().orc3_step_count(self._h))

    def fields(self) -> dict:
        keys = ("phi", "U", "rho", "ux", "uy", "uz")
        out = {k: np.empty(self.shape) for k in keys}
        lib().orc3_fields(self._h, *(_ptr(out[k]) for k in keys))
        return out

    def diag(self) -> dict:
        a = np.zeros(9)
        lib().orc3_diag(self._h, _dp(a))
        keys = ("rho", "jx", "jy", "jz", "U", "phi", "phi_prev", "n_solid", "n_nonfinite")
        d = dict(zip(keys, a.tolist()))
        d["species"] = d["U"] + 0.5 * self.p.L_sat * d["phi_prev"]
        return d


def lattice3():
    """(c [19, 3], w19 [19], w7 [7]) of the 3D oracle."""
    c = (ctypes.c_int32 * 57)()
    w19 = np.zeros(19)
    w7 = np.zeros(7)
    lib().orc3_lattice(c, _dp(w19), _dp(w7))
    return np.array(list(c)).reshape(19, 3), w19, w7


def feq3(rho, ux, uy, uz):
    out = np.zeros(19)
    lib().orc3_feq(rho, ux, uy, uz, _dp(out))
    return out


def geq3(U, ux, uy, uz):
    out = np.zeros(7)
    lib().orc3_geq(U, ux, uy, uz, _dp(out))
    return out


def aniso3(params: Params3D, gx, gy, gz):
    a, nx_, ny_, nz_ = (ctypes.c_double() for _ in range(4))
    cp = params.c_struct()
    lib().orc3_aniso(ctypes.byref(cp), gx, gy, gz, ctypes.byref(a), ctypes.byref(nx_), ctypes.byref(ny_),
                     ctypes.byref(nz_))
    return a.value, nx_.value, ny_.value, nz_.value


def grad3(params: Params3D, phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    assert phi.shape == (params.nz, params.ny, params.nx)
    gx, gy, gz = np.empty_like(phi), np.empty_like(phi), np.empty_like(phi)
    cp = params.c_struct()
    lib().orc3_grad(ctypes.byref(cp), _dp(phi), _dp(gx), _dp(gy), _dp(gz))
    return gx, gy, gz
