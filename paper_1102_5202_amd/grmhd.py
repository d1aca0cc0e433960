"""ctypes binding of ``libgrmhd.so`` (the C ABI of ``include/grmhd.h``).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  PyTorch provides the device memory (tensors) and the stream.  The
binding fails loudly when the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgrmhd.so")

FLAT, ISO_SCHW, STORED = 0, 1, 2
SOFT_SQRT, SOFT_MAX = 0, 1
PERIODIC, OUTFLOW = 0, 1
FP64, MIXED = 0, 1
PRECISIONS = {"fp64": FP64, "mixed": MIXED}
RECOVERY = {"2d": 0, "1d": 1}
RECONSTRUCTION = {"mc": 0, "ppm": 1}
DIVERGENCE = {"cleaning": 0, "fluxct": 1}
KERNELS = ("bc", "flux_x", "flux_y", "flux_z", "update", "cons", "prim", "rhs", "adj_rec",
           "adj_face", "adj_gather", "adj_cell", "ct")
NVAR = 9

# exported symbols of include/grmhd.h
SYMBOLS = ("grmhd_workspace_bytes", "grmhd_init", "grmhd_set_stream", "grmhd_cons", "grmhd_step",
           "grmhd_prim", "grmhd_rhs", "grmhd_metric_bytes", "grmhd_set_metric",
           "grmhd_step_adjoint", "grmhd_step_record",
           "grmhd_step_adjoint_recorded", "grmhd_cons_adjoint",
           "grmhd_prim_adjoint", "grmhd_status", "grmhd_timing", "grmhd_free", "grmhd_strerror",
           "grmhd_batch_workspace_bytes", "grmhd_batch_init", "grmhd_batch_set_stream",
           "grmhd_batch_cons", "grmhd_batch_evolve", "grmhd_batch_prim", "grmhd_batch_tune",
           "grmhd_batch_set_shape", "grmhd_batch_status", "grmhd_batch_busy", "grmhd_batch_free",
           "grmhd_rhs_noalloc", "grmhd_device_arith")


class Metric(C.Structure):
    _fields_ = [("kind", C.c_int), ("soft", C.c_int), ("M", C.c_double), ("r_min", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bc", C.c_int * 3)]


class Eos(C.Structure):
    _fields_ = [("kind", C.c_int), ("gamma", C.c_double), ("K", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("rk_order", C.c_int), ("precision", C.c_int), ("c_h", C.c_double),
                ("kappa", C.c_double), ("rho_atm", C.c_double), ("p_atm", C.c_double),
                ("newton_tol", C.c_double), ("newton_maxit", C.c_int), ("recovery", C.c_int),
                ("reconstruction", C.c_int), ("divergence", C.c_int), ("timing", C.c_int),
                ("adjoint", C.c_int), ("tape_steps", C.c_int), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class BatchDesc(C.Structure):
    _fields_ = [("nprob", C.c_int), ("n", C.POINTER(C.c_int)), ("lo", C.POINTER(C.c_double)),
                ("hi", C.POINTER(C.c_double)), ("dt", C.POINTER(C.c_double)),
                ("steps", C.POINTER(C.c_int)), ("bc", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("c2p_fail", C.c_longlong), ("atm_hits", C.c_longlong),
                ("p_floor_hits", C.c_longlong), ("fallback_1d", C.c_longlong),
                ("max_newton_it", C.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libgrmhd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libgrmhd.so is not built (%s); run `python -m paper_1102_5202_amd.build`"
                           " or __graft_entry__.build()" % path)
    L = C.CDLL(path)
    vp = C.c_void_p
    L.grmhd_workspace_bytes.argtypes = [C.POINTER(Grid), C.POINTER(Opts)]
    L.grmhd_workspace_bytes.restype = C.c_size_t
    L.grmhd_init.argtypes = [C.POINTER(vp), C.POINTER(Metric), C.POINTER(Grid), C.POINTER(Eos),
                             C.POINTER(Opts)]
    L.grmhd_set_stream.argtypes = [vp, vp]
    L.grmhd_cons.argtypes = [vp, vp, vp]
    L.grmhd_step.argtypes = [vp, vp, C.c_double]
    L.grmhd_prim.argtypes = [vp, vp, vp]
    L.grmhd_rhs.argtypes = [vp, vp, vp]
    L.grmhd_metric_bytes.argtypes = [C.POINTER(Grid)]
    L.grmhd_metric_bytes.restype = C.c_size_t
    L.grmhd_set_metric.argtypes = [vp, vp, vp, vp, C.c_size_t]
    L.grmhd_step_adjoint.argtypes = [vp, vp, vp, C.c_double]
    L.grmhd_step_record.argtypes = [vp, vp, C.c_double, C.c_int]
    L.grmhd_step_adjoint_recorded.argtypes = [vp, C.c_int, vp]
    L.grmhd_cons_adjoint.argtypes = [vp, vp, vp, vp]
    L.grmhd_prim_adjoint.argtypes = [vp, vp, vp, vp]
    L.grmhd_status.argtypes = [vp, C.POINTER(Stats), C.c_int]
    L.grmhd_batch_workspace_bytes.argtypes = [C.POINTER(BatchDesc), C.POINTER(Opts)]
    L.grmhd_batch_workspace_bytes.restype = C.c_size_t
    L.grmhd_batch_init.argtypes = [C.POINTER(vp), C.POINTER(BatchDesc), C.POINTER(Eos), C.POINTER(Opts)]
    L.grmhd_batch_set_stream.argtypes = [vp, vp]
    L.grmhd_batch_cons.argtypes = [vp, vp, vp]
    L.grmhd_batch_evolve.argtypes = [vp, vp, C.c_int]
    L.grmhd_batch_prim.argtypes = [vp, vp, vp]
    L.grmhd_batch_tune.argtypes = [vp, vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.grmhd_batch_set_shape.argtypes = [vp, C.c_int, C.c_int]
    L.grmhd_batch_status.argtypes = [vp, C.POINTER(Stats), C.c_int]
    L.grmhd_batch_busy.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.grmhd_batch_free.argtypes = [vp]
    L.grmhd_rhs_noalloc.argtypes = [C.POINTER(Metric), C.POINTER(Grid), C.POINTER(Eos), C.POINTER(Opts), vp, vp,
                                    vp]
    L.grmhd_device_arith.argtypes = [vp, vp, vp, C.c_longlong, vp]
    L.grmhd_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.c_int]
    L.grmhd_free.argtypes = [vp]
    L.grmhd_strerror.argtypes = [C.c_int]
    L.grmhd_strerror.restype = C.c_char_p
    for name in SYMBOLS:
        if name not in ("grmhd_workspace_bytes", "grmhd_strerror", "grmhd_batch_workspace_bytes",
                        "grmhd_metric_bytes"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, what: str) -> None:
    if rc != 0:
        msg = load().grmhd_strerror(rc).decode()
        raise RuntimeError("%s failed: %s (%d)" % (what, msg, rc))


def make_grid(n, lo, hi, bc) -> Grid:
    g = Grid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.lo[d] = float(lo[d])
        g.hi[d] = float(hi[d])
        g.bc[d] = int(bc[d])
    return g


def workspace_bytes(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(0, 0, 0), precision="fp64",
                    rk_order=3, adjoint=False, tape_steps=0) -> int:
    o = Opts()
    o.precision = PRECISIONS[precision]
    o.rk_order = int(rk_order)
    o.adjoint = int(bool(adjoint))
    o.tape_steps = int(tape_steps)
    return int(load().grmhd_workspace_bytes(C.byref(make_grid(n, lo, hi, bc)), C.byref(o)))


class Solver:
    """One simulation context: grid, metric, EOS and options, with the
    workspace and stream owned by PyTorch.

    Tensors are float64, contiguous, shape (9, nz, ny, nx), on the solver's
    device: P = (rho, p, u~x, u~y, u~z, Bx, By, Bz, Phi),
    U = (D, tau, Sx, Sy, Sz, Bdx, Bdy, Bdz, Phi).  precision "fp64" or
    "mixed" (float face physics and caches, double accumulation and recovery).
    recovery "2d" (Newton on (Wc, v^2)) or "1d" (Newton on Wc alone);
    reconstruction "mc" or "ppm"; divergence "cleaning" (GLM, Phi) or "fluxct".
    adjoint=True (FP64 only) reserves the workspace of the adjoint calls;
    tape_steps > 0 (with adjoint) adds that many slots of recorded steps."""

    def __init__(self, n, lo, hi, bc, metric=FLAT, M=0.0, soft=SOFT_SQRT, r_min=1.0,
                 gamma=5.0 / 3.0, K=0.0, rk_order=3, c_h=1.0, kappa=1.0, rho_atm=1e-12,
                 p_atm=1e-12, newton_tol=1e-12, newton_maxit=50, timing=False, device="cuda",
                 stream=None, precision="fp64", adjoint=False, tape_steps=0, recovery="2d",
                 reconstruction="mc", divergence="cleaning"):
        L = load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("Solver needs a GPU device; got %s" % self.device)
        self.n = tuple(int(v) for v in n)
        self.shape = (NVAR, self.n[2], self.n[1], self.n[0])
        self._grid = make_grid(n, lo, hi, bc)
        self._metric = Metric(int(metric), int(soft), float(M), float(r_min))
        self._eos = Eos(0, float(gamma), float(K))
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
        if recovery not in RECOVERY:
            raise ValueError("recovery must be one of %s" % sorted(RECOVERY))
        if reconstruction not in RECONSTRUCTION:
            raise ValueError("reconstruction must be one of %s" % sorted(RECONSTRUCTION))
        if divergence not in DIVERGENCE:
            raise ValueError("divergence must be one of %s" % sorted(DIVERGENCE))
        self.precision = precision
        self._opts = Opts(int(rk_order), PRECISIONS[precision], float(c_h), float(kappa),
                          float(rho_atm), float(p_atm), float(newton_tol), int(newton_maxit),
                          RECOVERY[recovery], RECONSTRUCTION[reconstruction], DIVERGENCE[divergence],
                          int(bool(timing)), int(bool(adjoint)), int(tape_steps), None, 0)
        nbytes = int(L.grmhd_workspace_bytes(C.byref(self._grid), C.byref(self._opts)))
        if nbytes == 0:
            raise ValueError("invalid grid")
        # torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._opts.workspace = C.c_void_p(self.workspace.data_ptr())
        self._opts.workspace_bytes = nbytes
        ctx = C.c_void_p()
        _check(L.grmhd_init(C.byref(ctx), C.byref(self._metric), C.byref(self._grid),
                            C.byref(self._eos), C.byref(self._opts)), "grmhd_init")
        self._ctx = ctx
        self.tape_steps = int(tape_steps) if adjoint else 0
        self.tape_owner = None      # the differentiable evolution whose steps the tape holds
        self.set_stream(stream if stream is not None else torch.cuda.current_stream(self.device))

    # -- plumbing ------------------------------------------------------------
    def set_stream(self, stream) -> None:
        self.stream = stream
        _check(load().grmhd_set_stream(self._ctx, C.c_void_p(stream.cuda_stream)),
               "grmhd_set_stream")

    def _t(self, x: torch.Tensor, name: str) -> int:
        if (not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_contiguous()
                or x.device != self.device or tuple(x.shape) != self.shape):
            raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s"
                             % (name, self.shape, self.device))
        return x.data_ptr()

    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    # -- the C ABI -----------------------------------------------------------
    def cons(self, P: torch.Tensor, U: torch.Tensor = None) -> torch.Tensor:
        U = self.empty() if U is None else U
        _check(load().grmhd_cons(self._ctx, C.c_void_p(self._t(P, "P")), C.c_void_p(self._t(U, "U"))),
               "grmhd_cons")
        return U

    def step(self, U: torch.Tensor, dt: float) -> torch.Tensor:
        _check(load().grmhd_step(self._ctx, C.c_void_p(self._t(U, "U")), float(dt)), "grmhd_step")
        return U

    def prim(self, U: torch.Tensor, P: torch.Tensor = None) -> torch.Tensor:
        P = self.empty() if P is None else P
        _check(load().grmhd_prim(self._ctx, C.c_void_p(self._t(U, "U")), C.c_void_p(self._t(P, "P"))),
               "grmhd_prim")
        return P

    def rhs(self, P: torch.Tensor, R: torch.Tensor = None) -> torch.Tensor:
        R = self.empty() if R is None else R
        _check(load().grmhd_rhs(self._ctx, C.c_void_p(self._t(P, "P")), C.c_void_p(self._t(R, "R"))),
               "grmhd_rhs")
        return R

    def set_metric(self, alpha: torch.Tensor, psi4: torch.Tensor) -> None:
        """The metric of a STORED solver: lapse and psi^4 at the cell centres with
        2 ghost layers on every active axis, float64 device tensors of shape
        (nz+2gz, ny+2gy, nx+2gx).  The derived values live in a buffer owned
        by the solver."""
        shape = tuple(self.n[d] + (4 if self.n[d] > 1 else 0) for d in (2, 1, 0))
        for x, name in ((alpha, "alpha"), (psi4, "psi4")):
            if (not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_contiguous()
                    or x.device != self.device or tuple(x.shape) != shape):
                raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s"
                                 % (name, shape, self.device))
        L = load()
        nb = int(L.grmhd_metric_bytes(C.byref(self._grid)))
        # the buffer is used on the solver's stream; the inputs are read there
        # after this call returns, so the allocator must not hand them out
        # again before that stream has passed the read
        with torch.cuda.stream(self.stream):
            self.metric_buffer = torch.empty(nb, dtype=torch.uint8, device=self.device)
        alpha.record_stream(self.stream)
        psi4.record_stream(self.stream)
        _check(L.grmhd_set_metric(self._ctx, C.c_void_p(alpha.data_ptr()), C.c_void_p(psi4.data_ptr()),
                                  C.c_void_p(self.metric_buffer.data_ptr()), nb), "grmhd_set_metric")

    # -- adjoint (vector-Jacobian products) ----------------------------------
    def step_adjoint(self, U: torch.Tensor, Ubar: torch.Tensor, dt: float) -> torch.Tensor:
        """Ubar <- (dU^(n+1)/dU^n)^T Ubar for one step from U (not modified)."""
        _check(load().grmhd_step_adjoint(self._ctx, C.c_void_p(self._t(U, "U")),
                                         C.c_void_p(self._t(Ubar, "Ubar")), float(dt)),
               "grmhd_step_adjoint")
        return Ubar

    def step_record(self, U: torch.Tensor, dt: float, slot: int) -> torch.Tensor:
        """One step of U in place, as step(), keeping its stages in tape slot `slot`."""
        self.tape_owner = None
        _check(load().grmhd_step_record(self._ctx, C.c_void_p(self._t(U, "U")), float(dt), int(slot)),
               "grmhd_step_record")
        return U

    def step_adjoint_recorded(self, slot: int, Ubar: torch.Tensor) -> torch.Tensor:
        """Ubar <- (dU^(n+1)/dU^n)^T Ubar for the step recorded in tape slot `slot`."""
        _check(load().grmhd_step_adjoint_recorded(self._ctx, int(slot), C.c_void_p(self._t(Ubar, "Ubar"))),
               "grmhd_step_adjoint_recorded")
        return Ubar

    def cons_adjoint(self, P: torch.Tensor, Ubar: torch.Tensor, Pbar: torch.Tensor = None) -> torch.Tensor:
        """Pbar = (dU/dP)^T Ubar at P."""
        Pbar = self.empty() if Pbar is None else Pbar
        _check(load().grmhd_cons_adjoint(self._ctx, C.c_void_p(self._t(P, "P")),
                                         C.c_void_p(self._t(Ubar, "Ubar")),
                                         C.c_void_p(self._t(Pbar, "Pbar"))), "grmhd_cons_adjoint")
        return Pbar

    def prim_adjoint(self, U: torch.Tensor, Pbar: torch.Tensor, Ubar: torch.Tensor = None) -> torch.Tensor:
        """Ubar = (dU/dP)^-T Pbar at the primitives of U."""
        Ubar = self.empty() if Ubar is None else Ubar
        _check(load().grmhd_prim_adjoint(self._ctx, C.c_void_p(self._t(U, "U")),
                                         C.c_void_p(self._t(Pbar, "Pbar")),
                                         C.c_void_p(self._t(Ubar, "Ubar"))), "grmhd_prim_adjoint")
        return Ubar

    def status(self, reset: bool = False) -> dict:
        st = Stats()
        _check(load().grmhd_status(self._ctx, C.byref(st), int(bool(reset))), "grmhd_status")
        return {"fail": st.c2p_fail, "atm": st.atm_hits, "pfloor": st.p_floor_hits,
                "fallback_1d": st.fallback_1d, "max_newton_it": st.max_newton_it}

    def timing(self, reset: bool = False) -> dict:
        ms = (C.c_double * len(KERNELS))()
        cnt = (C.c_longlong * len(KERNELS))()
        _check(load().grmhd_timing(self._ctx, ms, cnt, int(bool(reset))), "grmhd_timing")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}

    def close(self) -> None:
        if getattr(self, "_ctx", None):
            load().grmhd_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """An ensemble of independent 1D problems along x (flat metric), advanced
    in one persistent launch per call.  Packed float64 device arrays: problem
    b's (9, n_b) block follows problem b-1's; ``pack``/``unpack`` convert
    from and to per-problem (9, n_b) arrays."""

    def __init__(self, n, lo, hi, dt, steps, bc=OUTFLOW, gamma=5.0 / 3.0, K=0.0, rk_order=3,
                 c_h=1.0, kappa=1.0, rho_atm=1e-12, p_atm=1e-12, newton_tol=1e-12, newton_maxit=50,
                 device="cuda", stream=None, precision="fp64", recovery="2d"):
        L = load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("BatchSolver needs a GPU device; got %s" % self.device)
        self.n = [int(v) for v in n]
        self.nprob = len(self.n)
        self.offsets = [0]
        for v in self.n[:-1]:
            self.offsets.append(self.offsets[-1] + v)
        self.ncell = sum(self.n)
        self._arrays = ((C.c_int * self.nprob)(*self.n), (C.c_double * self.nprob)(*map(float, lo)),
                        (C.c_double * self.nprob)(*map(float, hi)), (C.c_double * self.nprob)(*map(float, dt)),
                        (C.c_int * self.nprob)(*map(int, steps)))
        self._desc = BatchDesc(self.nprob, *self._arrays, int(bc))
        self._eos = Eos(0, float(gamma), float(K))
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
        if recovery not in RECOVERY:
            raise ValueError("recovery must be one of %s" % sorted(RECOVERY))
        self.precision = precision
        self._opts = Opts(int(rk_order), PRECISIONS[precision], float(c_h), float(kappa), float(rho_atm),
                          float(p_atm), float(newton_tol), int(newton_maxit), RECOVERY[recovery], 0, 0, 0, 0,
                          0, None, 0)
        nbytes = int(L.grmhd_batch_workspace_bytes(C.byref(self._desc), C.byref(self._opts)))
        if nbytes == 0:
            raise ValueError("invalid batch description")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._opts.workspace = C.c_void_p(self.workspace.data_ptr())
        self._opts.workspace_bytes = nbytes
        ctx = C.c_void_p()
        _check(L.grmhd_batch_init(C.byref(ctx), C.byref(self._desc), C.byref(self._eos),
                                  C.byref(self._opts)), "grmhd_batch_init")
        self._ctx = ctx
        self.set_stream(stream if stream is not None else torch.cuda.current_stream(self.device))

    def set_stream(self, stream) -> None:
        self.stream = stream
        _check(load().grmhd_batch_set_stream(self._ctx, C.c_void_p(stream.cuda_stream)),
               "grmhd_batch_set_stream")

    def _t(self, x: torch.Tensor, name: str) -> int:
        if (not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_contiguous()
                or x.device != self.device or x.numel() != 9 * self.ncell):
            raise ValueError("%s must be a contiguous float64 tensor of %d values on %s"
                             % (name, 9 * self.ncell, self.device))
        return x.data_ptr()

    def pack(self, arrays) -> torch.Tensor:
        """Per-problem arrays of shape (9, n_b) (or (9, 1, 1, n_b)) to one packed tensor."""
        return torch.cat([torch.as_tensor(a, dtype=torch.float64).reshape(9, -1).reshape(-1)
                          for a in arrays]).to(self.device)

    def unpack(self, x: torch.Tensor):
        return [x[9 * o:9 * (o + n)].reshape(9, n) for o, n in zip(self.offsets, self.n)]

    def empty(self) -> torch.Tensor:
        return torch.empty(9 * self.ncell, dtype=torch.float64, device=self.device)

    def cons(self, P: torch.Tensor, U: torch.Tensor = None) -> torch.Tensor:
        U = self.empty() if U is None else U
        _check(load().grmhd_batch_cons(self._ctx, C.c_void_p(self._t(P, "P")), C.c_void_p(self._t(U, "U"))),
               "grmhd_batch_cons")
        return U

    def evolve(self, U: torch.Tensor, max_steps: int = 2 ** 31 - 1) -> torch.Tensor:
        _check(load().grmhd_batch_evolve(self._ctx, C.c_void_p(self._t(U, "U")), int(max_steps)),
               "grmhd_batch_evolve")
        return U

    def prim(self, U: torch.Tensor, P: torch.Tensor = None) -> torch.Tensor:
        P = self.empty() if P is None else P
        _check(load().grmhd_batch_prim(self._ctx, C.c_void_p(self._t(U, "U")), C.c_void_p(self._t(P, "P"))),
               "grmhd_batch_prim")
        return P

    def tune(self, U: torch.Tensor, trial_steps: int = 20):
        """Pick the fastest launch shape on copies of the state; returns
        (threads per workgroup, placement): placement 0 one workgroup per
        problem with the rows in HBM, 1 the same with the rows in LDS, 2 the
        problems split among workgroups in proportion to their work."""
        th, lds = C.c_int(), C.c_int()
        _check(load().grmhd_batch_tune(self._ctx, C.c_void_p(self._t(U, "U")), int(trial_steps),
                                       C.byref(th), C.byref(lds)), "grmhd_batch_tune")
        return th.value, lds.value

    def set_shape(self, threads: int, lds) -> None:
        """Launch shape of evolve: threads per workgroup (256, 512, 1024) and
        the placement (0 / False: rows in HBM, 1 / True: rows in LDS, 2: split
        problems, with 256 threads)."""
        _check(load().grmhd_batch_set_shape(self._ctx, int(threads), int(lds)), "grmhd_batch_set_shape")

    def status(self, reset: bool = False) -> dict:
        st = Stats()
        _check(load().grmhd_batch_status(self._ctx, C.byref(st), int(bool(reset))), "grmhd_batch_status")
        return {"fail": st.c2p_fail, "atm": st.atm_hits, "pfloor": st.p_floor_hits,
                "fallback_1d": st.fallback_1d, "max_newton_it": st.max_newton_it}

    def busy(self) -> tuple:
        """(busy fraction, workgroup slots) of the last evolve launch: the
        workgroups' summed durations over slots x the launch's span."""
        frac, slots = C.c_double(), C.c_int()
        _check(load().grmhd_batch_busy(self._ctx, C.byref(frac), C.byref(slots)), "grmhd_batch_busy")
        return frac.value, slots.value

    def close(self) -> None:
        if getattr(self, "_ctx", None):
            load().grmhd_batch_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_for(ensemble, **over) -> BatchSolver:
    """A BatchSolver for a :class:`workloads.Ensemble`."""
    kw = dict(n=ensemble.n, lo=[0.0] * len(ensemble.n), hi=[1.0] * len(ensemble.n), dt=ensemble.dt,
              steps=ensemble.steps, bc=ensemble.bc, gamma=ensemble.gamma, rk_order=ensemble.rk_order,
              rho_atm=ensemble.rho_atm, p_atm=ensemble.p_atm)
    kw.update(over)
    return BatchSolver(**kw)


def device_arith(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """grmhd_device_arith: (x / y, sqrt(x), 1 / sqrt(x)) as the kernels compute
    them, for float64 1D tensors on a GPU; returns a (3, n) tensor."""
    if x.dtype != torch.float64 or y.dtype != torch.float64 or x.shape != y.shape or x.dim() != 1:
        raise ValueError("x and y must be float64 1D tensors of one shape")
    x, y = x.contiguous(), y.contiguous()
    out = torch.empty((3, x.numel()), dtype=torch.float64, device=x.device)
    st = torch.cuda.current_stream(x.device)
    _check(load().grmhd_device_arith(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                     C.c_void_p(out.data_ptr()), x.numel(), C.c_void_p(st.cuda_stream)),
           "grmhd_device_arith")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def rhs_noalloc(P: torch.Tensor, n, lo, hi, bc, metric=FLAT, M=0.0, soft=SOFT_SQRT, r_min=1.0,
                gamma=5.0 / 3.0, K=0.0, rk_order=3, c_h=1.0, kappa=1.0, rho_atm=1e-12, p_atm=1e-12,
                newton_tol=1e-12, newton_maxit=50, precision="fp64", recovery="2d", reconstruction="mc",
                divergence="cleaning", R: torch.Tensor = None, stream=None) -> torch.Tensor:
    """grmhd_rhs_noalloc: the right-hand side of the primitives P (float64,
    (9, nz, ny, nx), on a GPU) with the library's static scratch, no context
    and no workspace.  R is written (allocated here by torch if not given)."""
    n = tuple(int(v) for v in n)
    shape = (NVAR, n[2], n[1], n[0])
    if (not isinstance(P, torch.Tensor) or P.dtype != torch.float64 or not P.is_contiguous()
            or P.device.type != "cuda" or tuple(P.shape) != shape):
        raise ValueError("P must be a contiguous float64 GPU tensor of shape %s" % (shape,))
    R = torch.empty_like(P) if R is None else R
    if (R.dtype != torch.float64 or not R.is_contiguous() or R.device != P.device
            or tuple(R.shape) != shape):
        raise ValueError("R must be a contiguous float64 tensor of shape %s on %s" % (shape, P.device))
    opts = Opts(int(rk_order), PRECISIONS[precision], float(c_h), float(kappa), float(rho_atm),
                float(p_atm), float(newton_tol), int(newton_maxit), RECOVERY[recovery],
                RECONSTRUCTION[reconstruction], DIVERGENCE[divergence], 0, 0, 0, None, 0)
    st = stream if stream is not None else torch.cuda.current_stream(P.device)
    with torch.cuda.device(P.device):
        _check(load().grmhd_rhs_noalloc(C.byref(Metric(int(metric), int(soft), float(M), float(r_min))),
                                        C.byref(make_grid(n, lo, hi, bc)), C.byref(Eos(0, float(gamma), float(K))),
                                        C.byref(opts), C.c_void_p(P.data_ptr()), C.c_void_p(R.data_ptr()),
                                        C.c_void_p(st.cuda_stream)), "grmhd_rhs_noalloc")
    return R


def rhs_noalloc_for(workload, P: torch.Tensor, **over) -> torch.Tensor:
    """rhs_noalloc configured for a :class:`workloads.Workload`."""
    kw = dict(n=workload.n, lo=workload.lo, hi=workload.hi, bc=workload.bc, metric=workload.metric,
              M=workload.M, soft=workload.soft, r_min=workload.r_min, gamma=workload.gamma,
              rk_order=workload.rk_order, c_h=workload.c_h, kappa=workload.kappa,
              rho_atm=workload.rho_atm, p_atm=workload.p_atm)
    kw.update(over)
    return rhs_noalloc(P, **kw)


def solver_for(workload, **over) -> Solver:
    """A Solver configured for a :class:`workloads.Workload`."""
    kw = dict(n=workload.n, lo=workload.lo, hi=workload.hi, bc=workload.bc, metric=workload.metric,
              M=workload.M, soft=workload.soft, r_min=workload.r_min, gamma=workload.gamma,
              rk_order=workload.rk_order, c_h=workload.c_h, kappa=workload.kappa,
              rho_atm=workload.rho_atm, p_atm=workload.p_atm)
    kw.update(over)
    return Solver(**kw)
