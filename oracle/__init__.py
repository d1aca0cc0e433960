"""ctypes binding of the plain FP64 CPU oracle (``oracle/grmhd_oracle.c``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_1102_5202_amd``) never touches it.

Arrays are numpy float64, structure-of-arrays ``[9, nz, ny, nx]`` over interior
cells, variable order P = (rho, p, u~x, u~y, u~z, Bx, By, Bz, Phi) and
U = (D, tau, Sx, Sy, Sz, Bdx, Bdy, Bdz, Phi).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

FLAT, ISO_SCHW, STORED = 0, 1, 2
SOFT_SQRT, SOFT_MAX = 0, 1
PERIODIC, OUTFLOW = 0, 1
FLAG_FAIL, FLAG_ATM, FLAG_PFLOOR = 1, 2, 4
RECON_MC, RECON_PPM = 0, 1


class _Metric(C.Structure):
    _fields_ = [("kind", C.c_int), ("soft", C.c_int), ("M", C.c_double), ("r_min", C.c_double),
                ("alpha_grid", C.POINTER(C.c_double)), ("psi4_grid", C.POINTER(C.c_double))]


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bc", C.c_int * 3)]


class _Problem(C.Structure):
    _fields_ = [("metric", _Metric), ("grid", _Grid), ("gamma", C.c_double),
                ("rk_order", C.c_int), ("c_h", C.c_double), ("kappa", C.c_double),
                ("rho_atm", C.c_double), ("p_atm", C.c_double), ("recon", C.c_int),
                ("ct", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("fail", C.c_longlong), ("atm", C.c_longlong), ("pfloor", C.c_longlong)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_prim2con.argtypes = [C.POINTER(_Problem), dp, dp]
        L.orc_con2prim.argtypes = [C.POINTER(_Problem), dp, dp, dp, C.c_void_p, C.POINTER(_Stats)]
        L.orc_rhs.argtypes = [C.POINTER(_Problem), dp, dp]
        L.orc_step.argtypes = [C.POINTER(_Problem), dp, dp, C.c_double, C.c_int, C.POINTER(_Stats)]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_point_geom.argtypes = [C.POINTER(_Metric), C.c_double, C.c_double, C.c_double, dp]
        L.orc_point_cons.argtypes = [C.POINTER(_Metric), C.c_double, C.c_double, C.c_double,
                                     C.c_double, dp, dp]
        L.orc_point_flux.argtypes = [C.POINTER(_Metric), C.c_double, C.c_double, C.c_int,
                                     C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_point_speeds.argtypes = [C.POINTER(_Metric), C.c_double, C.c_int, C.c_double,
                                       C.c_double, C.c_double, dp, dp, dp]
        L.orc_point_stress.argtypes = [C.POINTER(_Metric), C.c_double, C.c_double, C.c_double,
                                       C.c_double, dp, dp]
        L.orc_point_source.argtypes = [C.POINTER(_Metric), C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_double, dp, dp]
        L.orc_point_c2p.argtypes = [C.POINTER(_Metric), C.c_double, C.c_double, C.c_double,
                                    C.c_double, dp, dp]
        L.orc_point_c2p.restype = C.c_int
        L.orc_point_face_flux.argtypes = [C.POINTER(_Metric), C.c_double, C.c_double, C.c_int,
                                          C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.orc_mc_slope.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_mc_slope.restype = C.c_double
        L.orc_ppm_edges.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_ppm_edges.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


@dataclass
class Problem:
    """Problem description shared by all whole-grid oracle calls."""
    n: tuple = (16, 1, 1)
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    metric: int = FLAT
    M: float = 0.0
    soft: int = SOFT_SQRT
    r_min: float = 1.0
    gamma: float = 5.0 / 3.0
    rk_order: int = 3
    c_h: float = 1.0
    kappa: float = 1.0
    rho_atm: float = 1e-12
    p_atm: float = 1e-12
    recon: int = RECON_MC
    ct: int = 0
    # metric STORED: lapse and psi^4 at the cell centres with 2 ghost layers
    # on every active axis, arrays [z][y][x]
    alpha_grid: np.ndarray = None
    psi4_grid: np.ndarray = None
    _c: _Problem = field(default=None, init=False, repr=False)

    def c(self) -> _Problem:
        p = _Problem()
        p.metric.kind = self.metric
        p.metric.soft = self.soft
        p.metric.M = self.M
        p.metric.r_min = self.r_min
        for d in range(3):
            p.grid.n[d] = int(self.n[d])
            p.grid.lo[d] = float(self.lo[d])
            p.grid.hi[d] = float(self.hi[d])
            p.grid.bc[d] = int(self.bc[d])
        p.gamma = self.gamma
        p.rk_order = self.rk_order
        p.c_h = self.c_h
        p.kappa = self.kappa
        p.rho_atm = self.rho_atm
        p.p_atm = self.p_atm
        p.recon = int(self.recon)
        p.ct = int(self.ct)
        if self.metric == STORED:
            shape = tuple(self.n[d] + (4 if self.n[d] > 1 else 0) for d in (2, 1, 0))
            self._keep = [np.ascontiguousarray(self.alpha_grid, dtype=np.float64),
                          np.ascontiguousarray(self.psi4_grid, dtype=np.float64)]
            for a in self._keep:
                if a.shape != shape:
                    raise ValueError("stored metric arrays must have shape %s" % (shape,))
            p.metric.alpha_grid = _ptr(self._keep[0])
            p.metric.psi4_grid = _ptr(self._keep[1])
        return p

    @property
    def shape(self):
        return (9, self.n[2], self.n[1], self.n[0])

    def metric_c(self) -> _Metric:
        m = _Metric()
        m.kind, m.soft, m.M, m.r_min = self.metric, self.soft, self.M, self.r_min
        return m


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def prim2con(pb: Problem, P: np.ndarray) -> np.ndarray:
    P = _arr(P)
    U = np.empty_like(P)
    c = pb.c()
    lib().orc_prim2con(C.byref(c), _ptr(P), _ptr(U))
    return U


def con2prim(pb: Problem, U: np.ndarray, Pguess: np.ndarray):
    """Recovery + floors. Returns (P, U_adjusted, flags, stats_dict)."""
    U = _arr(U).copy()
    Pg = _arr(Pguess)
    P = np.empty_like(U)
    flags = np.zeros(U.shape[1:], dtype=np.uint8)
    st = _Stats()
    c = pb.c()
    lib().orc_con2prim(C.byref(c), _ptr(U), _ptr(Pg), _ptr(P), flags.ctypes.data_as(C.c_void_p),
                       C.byref(st))
    return P, U, flags, {"fail": st.fail, "atm": st.atm, "pfloor": st.pfloor}


def rhs(pb: Problem, P: np.ndarray) -> np.ndarray:
    P = _arr(P)
    R = np.empty_like(P)
    c = pb.c()
    if lib().orc_rhs(C.byref(c), _ptr(P), _ptr(R)) != 0:
        raise MemoryError("oracle rhs failed")
    return R


def step(pb: Problem, U: np.ndarray, P: np.ndarray, dt: float, nsteps: int = 1):
    """nsteps full RK steps.  Returns (U, P, stats_dict); inputs are not modified."""
    U = _arr(U).copy()
    P = _arr(P).copy()
    st = _Stats()
    c = pb.c()
    if lib().orc_step(C.byref(c), _ptr(U), _ptr(P), float(dt), int(nsteps), C.byref(st)) != 0:
        raise RuntimeError("oracle step failed")
    return U, P, {"fail": st.fail, "atm": st.atm, "pfloor": st.pfloor}


# ---- point functions ---------------------------------------------------------

def _m(metric=FLAT, M=0.0, soft=SOFT_SQRT, r_min=1.0) -> _Metric:
    m = _Metric()
    m.kind, m.soft, m.M, m.r_min = metric, soft, M, r_min
    return m


def point_geom(x, y, z, **mk):
    out = np.zeros(3 + 16 + 16 + 48)
    lib().orc_point_geom(C.byref(_m(**mk)), x, y, z, _ptr(out))
    return {"alpha": out[0], "sqrtgamma": out[1], "sqrtmg": out[2],
            "g": out[3:19].reshape(4, 4), "gi": out[19:35].reshape(4, 4),
            "dg": out[35:83].reshape(3, 4, 4)}


def point_cons(P, gamma, x=0.0, y=0.0, z=0.0, **mk):
    P = _arr(P)
    U = np.zeros(9)
    lib().orc_point_cons(C.byref(_m(**mk)), gamma, x, y, z, _ptr(P), _ptr(U))
    return U


def point_flux(P, gamma, dir, c_h=1.0, x=0.0, y=0.0, z=0.0, **mk):
    P = _arr(P)
    F = np.zeros(9)
    lib().orc_point_flux(C.byref(_m(**mk)), gamma, c_h, dir, x, y, z, _ptr(P), _ptr(F))
    return F


def point_speeds(P, gamma, dir, x=0.0, y=0.0, z=0.0, **mk):
    P = _arr(P)
    lm = np.zeros(1)
    lp = np.zeros(1)
    lib().orc_point_speeds(C.byref(_m(**mk)), gamma, dir, x, y, z, _ptr(P), _ptr(lm), _ptr(lp))
    return lm[0], lp[0]


def point_stress(P, gamma, x=0.0, y=0.0, z=0.0, **mk):
    P = _arr(P)
    T = np.zeros(16)
    lib().orc_point_stress(C.byref(_m(**mk)), gamma, x, y, z, _ptr(P), _ptr(T))
    return T.reshape(4, 4)


def point_source(P, gamma, kappa=1.0, x=0.0, y=0.0, z=0.0, **mk):
    P = _arr(P)
    S = np.zeros(9)
    lib().orc_point_source(C.byref(_m(**mk)), gamma, kappa, x, y, z, _ptr(P), _ptr(S))
    return S


def point_c2p(U, gamma, x=0.0, y=0.0, z=0.0, **mk):
    U = _arr(U)
    P = np.zeros(9)
    ok = lib().orc_point_c2p(C.byref(_m(**mk)), gamma, x, y, z, _ptr(U), _ptr(P))
    return P, bool(ok)


def point_face_flux(qL, qR, gamma, dir, c_h=1.0, x=0.0, y=0.0, z=0.0, **mk):
    qL = _arr(qL)
    qR = _arr(qR)
    F = np.zeros(9)
    lib().orc_point_face_flux(C.byref(_m(**mk)), gamma, c_h, dir, x, y, z, _ptr(qL), _ptr(qR),
                              _ptr(F))
    return F


def ppm_edges(a) -> tuple:
    """PPM edge values (left, right) of the middle cell of five cell values."""
    a = _arr(a)
    assert a.shape == (5,)
    l, r = C.c_double(), C.c_double()
    lib().orc_ppm_edges(_ptr(a), C.byref(l), C.byref(r))
    return l.value, r.value


def mc_slope(qm, q0, qp) -> float:
    return float(lib().orc_mc_slope(qm, q0, qp))


# ---- parity metric (test infrastructure) ----------------------------------------

GROUPS = ((0,), (1,), (2, 3, 4), (5, 6, 7), (8,))


def parity_error(U, U_ref):
    """Relative L1 distance per conserved variable, sum|U - U_ref| / sum|U_ref|
    over all cells.  Components of a vector (momentum S, densitised field Bd)
    are normalised by the L1 norm of the largest component of that vector, so
    that a component which vanishes analytically (rounding noise on both
    sides) is judged against the vector's size.  A variable whose whole group
    is zero in the reference reports the absolute L1 distance."""
    U = np.asarray(U).reshape(9, -1)
    R = np.asarray(U_ref).reshape(9, -1)
    num = np.abs(U - R).sum(axis=1)
    l1 = np.abs(R).sum(axis=1)
    out = np.empty(9)
    for grp in GROUPS:
        den = max(l1[v] for v in grp)
        for v in grp:
            out[v] = num[v] / den if den > 0 else num[v]
    return out
