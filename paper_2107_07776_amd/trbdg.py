"""ctypes binding of libtrbdg (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor device,
dtype, size and contiguity, passes raw device pointers and turns non-zero
status codes into ``TrbdgError``.  PyTorch provides device memory and the
stream.  Loading fails loudly when the library has not been built.
"""
import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrbdg.so")

STATUS = {0: "OK", -1: "EINVAL", -2: "EDEVICE", -3: "ENOMEM", -4: "ENOTCONV",
          -5: "EBREAKDOWN", -6: "ENAN", -7: "EUNSUPPORTED"}

# Symbols declared in include/trbdg.h
EXPORTED = [
    "tbdg_create", "tbdg_destroy", "tbdg_last_error", "tbdg_set_stream", "tbdg_sizes",
    "tbdg_node_coords", "tbdg_extrapolate", "tbdg_apply_momentum", "tbdg_apply_pressure",
    "tbdg_diag_momentum", "tbdg_diag_pressure", "tbdg_rhs_momentum", "tbdg_grad_p",
    "tbdg_add_grad_p", "tbdg_rhs_pressure", "tbdg_solve_momentum", "tbdg_solve_pressure",
    "tbdg_solve_pressure_noalloc",
    "tbdg_step", "tbdg_profile_enable", "tbdg_profile_read", "tbdg_mg_setup",
    "tbdg_mg_levels", "tbdg_mg_apply", "tbdg_mg_apply_momentum", "tbdg_mg_levels_momentum",
    "tbdg_set_mg_graphs", "tbdg_mg_fused",
    "tbdg_net_create", "tbdg_net_destroy",
    "tbdg_net_last_error", "tbdg_net_num_params", "tbdg_net_set_params", "tbdg_net_get_params",
    "tbdg_net_get_grads", "tbdg_net_zero_grad", "tbdg_net_forward", "tbdg_net_backward",
    "tbdg_net_mse", "tbdg_net_quad_loss", "tbdg_net_adam_step", "tbdg_set_guess_net",
    "tbdg_guess_reset", "tbdg_guess_record", "tbdg_guess_recorded", "tbdg_guess_features",
    "tbdg_guess_inject", "tbdg_guess_target",
    "tbdg_guess_last", "tbdg_face_qpoints", "tbdg_set_dirichlet", "tbdg_set_nonlinear",
    "tbdg_set_scheme",
    "tbdg_nonlinear_solves", "tbdg_profile_bytes", "tbdg_precond_momentum",
    "tbdg_amr_create", "tbdg_amr_destroy", "tbdg_amr_last_error", "tbdg_amr_set_stream",
    "tbdg_amr_sizes", "tbdg_amr_leaves", "tbdg_amr_apply_pressure", "tbdg_amr_diag_pressure",
    "tbdg_amr_solve_pressure", "tbdg_amr_indicator", "tbdg_amr_mark", "tbdg_amr_plan",
    "tbdg_amr_transfer", "tbdg_amr_commit", "tbdg_amr_face_qpoints", "tbdg_amr_apply_momentum",
    "tbdg_amr_solve_momentum", "tbdg_amr_set_flow", "tbdg_amr_rhs_momentum", "tbdg_amr_rhs_pressure",
    "tbdg_amr_add_grad_p", "tbdg_amr_step",
]

GUESS = {"given": 0, "previous": 1, "learned": 2, "extrap2": 3, "extrap3": 4}

# channels of the guess network's input and output per cell
GUESS_IN, GUESS_OUT = 6, 2

# largest pressure space of the allocation-free solve (TBDG_NOALLOC_MAX_NP)
NOALLOC_MAX_NP = 1 << 20

PRECOND = {"jacobi": 0, "mg_fp32": 1, "mg_bf16": 2, "line": 3}

# time schemes of step(): TR-BDF2, Bell-Colella-Glaz (Crank-Nicolson), BDF2
SCHEME = {"trbdf2": 0, "bcg": 1, "bdf2": 2}


class AmrDesc(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int * 2), ("lo", ctypes.c_double * 2),
                ("hi", ctypes.c_double * 2), ("periodic", ctypes.c_int * 2), ("k", ctypes.c_int),
                ("max_level", ctypes.c_int), ("pen_p", ctypes.c_double), ("pen_u", ctypes.c_double)]


class AmrStepOpts(ctypes.Structure):
    _fields_ = [("nonlinear", ctypes.c_int), ("mom_tol", ctypes.c_double), ("prs_tol", ctypes.c_double),
                ("mom_maxiter", ctypes.c_int), ("prs_maxiter", ctypes.c_int), ("restart", ctypes.c_int)]


class TrbdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_cells", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int * 3), ("mapping", ctypes.c_int),
                ("map_amp", ctypes.c_double)]


class DiscDesc(ctypes.Structure):
    _fields_ = [("k_u", ctypes.c_int), ("nu", ctypes.c_double), ("c", ctypes.c_double),
                ("dt", ctypes.c_double), ("gamma", ctypes.c_double),
                ("pen_u", ctypes.c_double), ("pen_p", ctypes.c_double)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("restart", ctypes.c_int),
                ("precond", ctypes.c_int), ("guess", ctypes.c_int)]


class MGDesc(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("lanczos_steps", ctypes.c_int), ("range", ctypes.c_double),
                ("safety", ctypes.c_double), ("coarse_cells", ctypes.c_int),
                ("max_coarse_dofs", ctypes.c_int), ("no_fuse", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("guess_used", ctypes.c_int),
                ("precond_fallbacks", ctypes.c_int)]

    def as_dict(self):
        return dict(iters=self.iters, res0=self.res0, res_final=self.res_final,
                    guess_used=self.guess_used, precond_fallbacks=self.precond_fallbacks)


class State(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("u_hist", ctypes.c_void_p), ("p", ctypes.c_void_p),
                ("t", ctypes.c_double), ("n", ctypes.c_int64)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libtrbdg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2107_07776_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "tbdg_create": ([P(MeshDesc), P(DiscDesc), vp, P(vp)], i),
        "tbdg_destroy": ([vp], None),
        "tbdg_last_error": ([vp], ctypes.c_char_p),
        "tbdg_set_stream": ([vp, vp], i),
        "tbdg_sizes": ([vp, P(i64), P(i64), P(i64)], i),
        "tbdg_node_coords": ([vp, i, vp], i),
        "tbdg_extrapolate": ([vp, i, vp, vp, vp], i),
        "tbdg_apply_momentum": ([vp, i, vp, vp, vp], i),
        "tbdg_apply_pressure": ([vp, i, vp, vp], i),
        "tbdg_diag_momentum": ([vp, i, vp, vp], i),
        "tbdg_diag_pressure": ([vp, i, vp], i),
        "tbdg_rhs_momentum": ([vp, i, vp, vp, vp, vp, vp], i),
        "tbdg_grad_p": ([vp, vp, vp], i),
        "tbdg_add_grad_p": ([vp, vp, d, vp, vp], i),
        "tbdg_rhs_pressure": ([vp, i, vp, vp, vp], i),
        "tbdg_solve_momentum": ([vp, i, vp, vp, vp, P(SolverOpts), P(SolveInfo)], i),
        "tbdg_solve_pressure": ([vp, i, vp, vp, P(SolverOpts), P(SolveInfo)], i),
        "tbdg_solve_pressure_noalloc": ([vp, i, vp, vp, P(SolverOpts), P(SolveInfo)], i),
        "tbdg_step": ([vp, P(State), P(SolverOpts), P(SolverOpts), P(SolveInfo)], i),
        "tbdg_profile_enable": ([vp, i], i),
        "tbdg_profile_read": ([vp, i, P(d), P(i64)], i),
        "tbdg_mg_setup": ([vp, P(MGDesc)], i),
        "tbdg_mg_levels": ([vp, i, P(i), P(i64), P(d)], i),
        "tbdg_mg_apply": ([vp, i, i, vp, vp], i),
        "tbdg_mg_apply_momentum": ([vp, i, vp, vp], i),
        "tbdg_mg_levels_momentum": ([vp, i, P(i), P(i64), P(d)], i),
        "tbdg_set_mg_graphs": ([vp, i], i),
        "tbdg_mg_fused": ([vp, i, P(i), P(i64)], i),
        "tbdg_net_create": ([i, ctypes.c_uint64, vp, P(vp)], i),
        "tbdg_net_destroy": ([vp], None),
        "tbdg_net_last_error": ([vp], ctypes.c_char_p),
        "tbdg_net_num_params": ([vp, P(i64)], i),
        "tbdg_net_set_params": ([vp, vp], i),
        "tbdg_net_get_params": ([vp, vp], i),
        "tbdg_net_get_grads": ([vp, vp], i),
        "tbdg_net_zero_grad": ([vp], i),
        "tbdg_net_forward": ([vp, vp, vp, i, i, i, i], i),
        "tbdg_net_backward": ([vp, vp], i),
        "tbdg_net_mse": ([vp, vp, vp, i64, vp, P(d)], i),
        "tbdg_net_quad_loss": ([vp, vp, vp, i64, i, vp, P(d)], i),
        "tbdg_net_adam_step": ([vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float], i),
        "tbdg_set_guess_net": ([vp, vp], i),
        "tbdg_guess_reset": ([vp], i),
        "tbdg_guess_record": ([vp, vp, i], i),
        "tbdg_guess_recorded": ([vp, P(i)], i),
        "tbdg_guess_last": ([vp, P(d), P(d)], i),
        "tbdg_face_qpoints": ([vp, P(i64), vp], i),
        "tbdg_set_dirichlet": ([vp, i, vp], i),
        "tbdg_set_nonlinear": ([vp, i, d], i),
        "tbdg_set_scheme": ([vp, i], i),
        "tbdg_nonlinear_solves": ([vp, P(i)], i),
        "tbdg_profile_bytes": ([vp, i, P(d)], i),
        "tbdg_precond_momentum": ([vp, i, vp, vp, vp], i),
        "tbdg_guess_features": ([vp, i, vp, vp, vp, d, vp, vp, vp, P(d)], i),
        "tbdg_guess_inject": ([vp, vp, vp, vp, vp, vp, vp], i),
        "tbdg_guess_target": ([vp, vp, vp, vp, vp, vp, vp], i),
        "tbdg_amr_create": ([P(AmrDesc), vp, P(vp)], i),
        "tbdg_amr_destroy": ([vp], None),
        "tbdg_amr_last_error": ([vp], ctypes.c_char_p),
        "tbdg_amr_set_stream": ([vp, vp], i),
        "tbdg_amr_sizes": ([vp, P(i64), P(i64), P(i64)], i),
        "tbdg_amr_leaves": ([vp, vp], i),
        "tbdg_amr_apply_pressure": ([vp, d, vp, vp], i),
        "tbdg_amr_diag_pressure": ([vp, d, vp], i),
        "tbdg_amr_solve_pressure": ([vp, d, vp, vp, d, i, P(SolveInfo)], i),
        "tbdg_amr_indicator": ([vp, vp, vp], i),
        "tbdg_amr_mark": ([vp, vp, d, d, d, d, vp], i),
        "tbdg_amr_plan": ([vp, vp, P(i64)], i),
        "tbdg_amr_transfer": ([vp, i, vp, vp], i),
        "tbdg_amr_commit": ([vp], i),
        "tbdg_amr_face_qpoints": ([vp, P(i64), vp], i),
        "tbdg_amr_apply_momentum": ([vp, d, d, d, vp, vp, vp, vp], i),
        "tbdg_amr_solve_momentum": ([vp, d, d, d, vp, vp, vp, vp, d, i, i, P(SolveInfo)], i),
        "tbdg_amr_set_flow": ([vp, d, d, d], i),
        "tbdg_amr_rhs_momentum": ([vp, i, vp, vp, vp, vp, vp, vp, vp], i),
        "tbdg_amr_rhs_pressure": ([vp, i, vp, vp, vp], i),
        "tbdg_amr_add_grad_p": ([vp, vp, d, vp, vp], i),
        "tbdg_amr_step": ([vp, P(AmrStepOpts), vp, vp, vp, vp, P(SolveInfo), P(d)], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def solver_opts(tol=1e-8, maxiter=1000, restart=30, precond="jacobi", guess="given"):
    return SolverOpts(float(tol), int(maxiter), int(restart), PRECOND[precond], GUESS[guess])


class Context:
    """One mesh + discretisation on the current HIP device and stream."""

    def __init__(self, dim, n_cells, lo, hi, k, nu, dt, c=1.0e3, periodic=None,
                 gamma=0.0, pen_u=1.0, pen_p=1.0, stream=None, device="cuda", mapping=0,
                 map_amp=0.0):
        self.lib = load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("trbdg needs a ROCm GPU device")
        periodic = periodic if periodic is not None else (1,) * dim
        m = MeshDesc()
        m.dim = dim
        for a in range(3):
            m.n_cells[a] = int(n_cells[a]) if a < dim else 1
            m.lo[a] = float(lo[a]) if a < dim else 0.0
            m.hi[a] = float(hi[a]) if a < dim else 1.0
            m.periodic[a] = int(bool(periodic[a])) if a < dim else 1
        m.mapping = int(mapping)
        m.map_amp = float(map_amp)
        dd = DiscDesc(int(k), float(nu), float(c), float(dt), float(gamma), float(pen_u), float(pen_p))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self.lib.tbdg_create(ctypes.byref(m), ctypes.byref(dd),
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise TrbdgError(st, "tbdg_create failed (invalid or unsupported descriptor)")
        self.h = h
        nu_, np_, nc_ = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.tbdg_sizes(self.h, ctypes.byref(nu_), ctypes.byref(np_), ctypes.byref(nc_)))
        self.dim, self.k = dim, k
        self.N_u, self.N_p, self.N_c = nu_.value, np_.value, nc_.value
        self.nbu = (k + 1) ** dim
        self.nbp = k ** dim
        self.dt = dt
        self.gamma = float(gamma) if gamma > 0.0 else 2.0 - math.sqrt(2.0)

    # -- plumbing ----------------------------------------------------------
    def _check(self, st):
        if st != 0:
            msg = self.lib.tbdg_last_error(self.h)
            raise TrbdgError(st, msg.decode() if msg else "")

    def _vec(self, t, n, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
        return t

    def empty_u(self):
        return torch.empty(self.N_u, dtype=torch.float64, device=self.device)

    def empty_p(self):
        return torch.empty(self.N_p, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tbdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points ---------------------------------------------------------
    def node_coords(self, field=0):
        nb = self.nbu if field == 0 else self.nbp
        out = torch.empty(self.N_c * nb * self.dim, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_node_coords(self.h, field, _ptr(out)))
        return out.view(-1, self.dim)

    def face_qpoints(self):
        """Boundary face points [n][dim] (float64, device), empty if periodic."""
        n = ctypes.c_int64()
        self._check(self.lib.tbdg_face_qpoints(self.h, ctypes.byref(n), None))
        out = torch.empty((n.value, self.dim), dtype=torch.float64, device=self.device)
        if n.value:
            self._check(self.lib.tbdg_face_qpoints(self.h, ctypes.byref(n), _ptr(out)))
        return out

    def set_dirichlet(self, slot, uD):
        """Dirichlet data [n][dim] at the boundary points; slot 0: stage-1 time
        t^n + gamma dt, slot 1: t^{n+1}."""
        n = self.face_qpoints().shape[0] if not hasattr(self, "_nbp") else self._nbp
        self._nbp = n
        if uD.dtype != torch.float64 or uD.device.type != "cuda" or not uD.is_contiguous() \
                or uD.numel() != n * self.dim:
            raise ValueError(f"uD must be a contiguous float64 CUDA tensor of {n} x {self.dim}")
        self._check(self.lib.tbdg_set_dirichlet(self.h, int(slot), _ptr(uD)))

    def extrapolate(self, stage, u_new, u_old, out=None):
        out = self.empty_u() if out is None else self._vec(out, self.N_u, "out")
        self._check(self.lib.tbdg_extrapolate(self.h, stage, _ptr(self._vec(u_new, self.N_u, "u_new")),
                                              _ptr(self._vec(u_old, self.N_u, "u_old")), _ptr(out)))
        return out

    def apply_momentum(self, stage, w, u, out=None):
        out = self.empty_u() if out is None else self._vec(out, self.N_u, "out")
        self._check(self.lib.tbdg_apply_momentum(self.h, stage, _ptr(self._vec(w, self.N_u, "w")),
                                                 _ptr(self._vec(u, self.N_u, "u")), _ptr(out)))
        return out

    def precond_momentum(self, stage, w, v, out=None):
        """z = P^{-1} v with the line-block preconditioner of V_s(w)."""
        out = self.empty_u() if out is None else self._vec(out, self.N_u, "out")
        self._check(self.lib.tbdg_precond_momentum(self.h, stage, _ptr(self._vec(w, self.N_u, "w")),
                                                   _ptr(self._vec(v, self.N_u, "v")), _ptr(out)))
        return out

    def apply_pressure(self, stage, p, out=None):
        out = self.empty_p() if out is None else self._vec(out, self.N_p, "out")
        self._check(self.lib.tbdg_apply_pressure(self.h, stage, _ptr(self._vec(p, self.N_p, "p")), _ptr(out)))
        return out

    def diag_momentum(self, stage, w):
        out = torch.empty(self.N_u // self.dim, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_diag_momentum(self.h, stage, _ptr(self._vec(w, self.N_u, "w")), _ptr(out)))
        return out

    def diag_pressure(self, stage):
        out = self.empty_p()
        self._check(self.lib.tbdg_diag_pressure(self.h, stage, _ptr(out)))
        return out

    def rhs_momentum(self, stage, u_n, u_g, w, p_prev):
        out = self.empty_u()
        ug = None if u_g is None else self._vec(u_g, self.N_u, "u_g")
        self._check(self.lib.tbdg_rhs_momentum(self.h, stage, _ptr(self._vec(u_n, self.N_u, "u_n")), _ptr(ug),
                                               _ptr(self._vec(w, self.N_u, "w")),
                                               _ptr(self._vec(p_prev, self.N_p, "p_prev")), _ptr(out)))
        return out

    def grad_p(self, p):
        out = self.empty_u()
        self._check(self.lib.tbdg_grad_p(self.h, _ptr(self._vec(p, self.N_p, "p")), _ptr(out)))
        return out

    def add_grad_p(self, x, a, p, out=None):
        out = self.empty_u() if out is None else self._vec(out, self.N_u, "out")
        self._check(self.lib.tbdg_add_grad_p(self.h, _ptr(self._vec(x, self.N_u, "x")), float(a),
                                             _ptr(self._vec(p, self.N_p, "p")), _ptr(out)))
        return out

    def rhs_pressure(self, stage, u_ss, p_prev):
        out = self.empty_p()
        self._check(self.lib.tbdg_rhs_pressure(self.h, stage, _ptr(self._vec(u_ss, self.N_u, "u_ss")),
                                               _ptr(self._vec(p_prev, self.N_p, "p_prev")), _ptr(out)))
        return out

    def solve_momentum(self, stage, w, rhs, u_inout, tol=1e-8, maxiter=1000, restart=30, check=True,
                       precond="jacobi"):
        """GMRES(restart) with the Jacobi or the line-block ("line") preconditioner."""
        o = solver_opts(tol, maxiter, restart, precond)
        info = SolveInfo()
        st = self.lib.tbdg_solve_momentum(self.h, stage, _ptr(self._vec(w, self.N_u, "w")),
                                          _ptr(self._vec(rhs, self.N_u, "rhs")),
                                          _ptr(self._vec(u_inout, self.N_u, "u")), ctypes.byref(o),
                                          ctypes.byref(info))
        if check:
            self._check(st)
        return info.as_dict() | {"status": st}

    def solve_pressure(self, stage, rhs, p_inout, tol=1e-8, maxiter=5000, precond="jacobi",
                       check=True):
        o = solver_opts(tol, maxiter, 0, precond)
        info = SolveInfo()
        st = self.lib.tbdg_solve_pressure(self.h, stage, _ptr(self._vec(rhs, self.N_p, "rhs")),
                                          _ptr(self._vec(p_inout, self.N_p, "p")), ctypes.byref(o),
                                          ctypes.byref(info))
        if check:
            self._check(st)
        return info.as_dict() | {"status": st}

    def solve_pressure_noalloc(self, stage, rhs, p_inout, tol=1e-8, maxiter=5000, check=True):
        """Jacobi-preconditioned CG of ``solve_pressure`` with the library's
        static device scratch in place of the context's workspace (the entry
        point allocates nothing; N_p <= NOALLOC_MAX_NP)."""
        o = solver_opts(tol, maxiter, 0, "jacobi")
        info = SolveInfo()
        st = self.lib.tbdg_solve_pressure_noalloc(self.h, stage, _ptr(self._vec(rhs, self.N_p, "rhs")),
                                                  _ptr(self._vec(p_inout, self.N_p, "p")),
                                                  ctypes.byref(o), ctypes.byref(info))
        if check:
            self._check(st)
        return info.as_dict() | {"status": st}

    def step(self, u, u_hist, p, t=0.0, n=0, mom_tol=1e-8, prs_tol=1e-8, mom_maxiter=1000,
             prs_maxiter=5000, restart=30, precond="jacobi", guess="given", mom_guess="given",
             check=True, mom_precond="jacobi"):
        """One TR-BDF2 step in place on (u, u_hist, p); returns per-solve info.
        ``precond`` selects the pressure preconditioner, ``guess`` the initial
        guess of the pressure solves ("given": previous pressure, "previous":
        rescaled newest increment, "learned": the attached network),
        ``mom_precond`` the momentum preconditioner ("jacobi", "line" or
        "mg_fp32")."""
        S = State(_ptr(self._vec(u, self.N_u, "u")), _ptr(self._vec(u_hist, self.N_u, "u_hist")),
                  _ptr(self._vec(p, self.N_p, "p")), float(t), int(n))
        mo = solver_opts(mom_tol, mom_maxiter, restart, mom_precond, guess=mom_guess)
        po = solver_opts(prs_tol, prs_maxiter, 0, precond, guess)
        infos = (SolveInfo * 4)()
        st = self.lib.tbdg_step(self.h, ctypes.byref(S), ctypes.byref(mo), ctypes.byref(po), infos)
        if check:
            self._check(st)
        out = [infos[i].as_dict() for i in range(4)]
        solves = (ctypes.c_int * 2)()
        self._check(self.lib.tbdg_nonlinear_solves(self.h, solves))
        out[0]["solves"], out[2]["solves"] = solves[0], solves[1]
        return out, st

    def set_nonlinear(self, max_solves=1, tol=0.0):
        """Fully nonlinear momentum predictors in step(): up to ``max_solves``
        fixed-point solves per stage, early stop at relative change ``tol``
        (1 = the linearised scheme with the extrapolated advector)."""
        self._check(self.lib.tbdg_set_nonlinear(self.h, int(max_solves), float(tol)))

    def set_scheme(self, scheme):
        """Time scheme of step(): "trbdf2", "bcg" or "bdf2" (for the
        single-stage schemes u_hist is u^{n-1} and the solves fill info[0]
        and info[1])."""
        self._check(self.lib.tbdg_set_scheme(self.h, SCHEME[scheme]))

    def mg_setup(self, degree=0, lanczos_steps=0, range_=0.0, safety=0.0, coarse_cells=0,
                 max_coarse_dofs=0, fuse="auto"):
        """Build the pressure multigrid hierarchy (0 = library default; fuse:
        the coarse Q1 levels in one single-workgroup launch per V-cycle,
        "auto" in 2D only, True in 2D and 3D, False never)."""
        nf = 0 if fuse == "auto" else (2 if fuse else 1)
        d = MGDesc(int(degree), int(lanczos_steps), float(range_), float(safety), int(coarse_cells),
                   int(max_coarse_dofs), nf)
        self._check(self.lib.tbdg_mg_setup(self.h, ctypes.byref(d)))

    def mg_levels(self, cap=16, field="p"):
        """List of per-level dicts (nodes per direction, cells, DoFs, eigenvalue
        estimates of stages 1 and 2) of the pressure ("p") or the momentum
        ("u") hierarchy."""
        n = ctypes.c_int()
        desc = (ctypes.c_int64 * (5 * cap))()
        lam = (ctypes.c_double * (2 * cap))()
        fn = self.lib.tbdg_mg_levels if field == "p" else self.lib.tbdg_mg_levels_momentum
        self._check(fn(self.h, cap, ctypes.byref(n), desc, lam))
        return [dict(np=desc[5 * l], cells=tuple(desc[5 * l + 1:5 * l + 4]), dofs=desc[5 * l + 4],
                     lam=(lam[l], lam[cap + l])) for l in range(min(n.value, cap))]

    def mg_apply(self, stage, r, precision="fp32"):
        """z = B r, one V-cycle of the stage's hierarchy."""
        z = self.empty_p()
        self._check(self.lib.tbdg_mg_apply(self.h, stage, 1 if precision == "fp32" else 2,
                                           _ptr(self._vec(r, self.N_p, "r")), _ptr(z)))
        return z

    def mg_apply_momentum(self, stage, v):
        """z = P^{-1} v: one FP32 V-cycle of the momentum hierarchy per velocity
        component of v / (theta_s nu)."""
        z = self.empty_u()
        self._check(self.lib.tbdg_mg_apply_momentum(self.h, stage, _ptr(self._vec(v, self.N_u, "v")),
                                                    _ptr(z)))
        return z

    def mg_fused(self, field="p"):
        """(first level of the single-workgroup coarse cycle or -1, its LDS
        bytes) of the pressure ("p") or momentum ("u") hierarchy."""
        first = ctypes.c_int()
        lds = ctypes.c_int64()
        self._check(self.lib.tbdg_mg_fused(self.h, 0 if field == "p" else 1, ctypes.byref(first),
                                           ctypes.byref(lds)))
        return first.value, lds.value

    def set_mg_graphs(self, enable):
        """V-cycles inside the solves as HIP-graph replays (True, the
        default) or launched kernel by kernel (False); same results."""
        self._check(self.lib.tbdg_set_mg_graphs(self.h, 1 if enable else 0))

    def set_guess_net(self, net):
        """Attach a Net (same stream) for guess="learned", or None to detach."""
        self._net = net
        self._check(self.lib.tbdg_set_guess_net(self.h, net.h if net is not None else None))

    def guess_reset(self):
        self._check(self.lib.tbdg_guess_reset(self.h))

    def guess_record(self, buf):
        """Record (input, target) samples of the pressure solves into buf
        (float32 CUDA tensor [capacity][12][N_c]: network input [6][N_c],
        Gram target [6][N_c]); None stops recording."""
        if buf is None:
            self._rec = None
            self._check(self.lib.tbdg_guess_record(self.h, None, 0))
            return
        if buf.dtype != torch.float32 or buf.device.type != "cuda" or not buf.is_contiguous() \
                or buf.dim() != 3 or buf.shape[1:] != (GUESS_IN + 6, self.N_c):
            raise ValueError("buf must be a contiguous float32 CUDA tensor [capacity][12][N_c]")
        self._rec = buf
        self._check(self.lib.tbdg_guess_record(self.h, _ptr(buf), buf.shape[0]))

    def guess_recorded(self):
        n = ctypes.c_int()
        self._check(self.lib.tbdg_guess_recorded(self.h, ctypes.byref(n)))
        return n.value

    def guess_last(self):
        """(||b - H x_learned||, ||b - H x_fallback||) of the last learned decision."""
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.tbdg_guess_last(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def guess_features(self, stage, b, p_prev, d0, beta0, d1, d2):
        """(x [6][N_c] float32, (s_inc, s_div)) of the guess network."""
        x = torch.empty((GUESS_IN, self.N_c), dtype=torch.float32, device=self.device)
        sc = (ctypes.c_double * 2)()
        self._check(self.lib.tbdg_guess_features(
            self.h, stage, _ptr(self._vec(b, self.N_p, "b")), _ptr(self._vec(p_prev, self.N_p, "p_prev")),
            _ptr(self._vec(d0, self.N_p, "d0")), float(beta0), _ptr(self._vec(d1, self.N_p, "d1")),
            _ptr(self._vec(d2, self.N_p, "d2")), _ptr(x), sc))
        return x, (sc[0], sc[1])

    def guess_inject(self, p_prev, d1, d2, d3, y):
        """p_prev + (3 + y0_K) d1 - (3 - y1_K) d2 + d3 for y float32 [2][N_c]."""
        out = self.empty_p()
        if y.dtype != torch.float32 or y.numel() != GUESS_OUT * self.N_c or not y.is_contiguous():
            raise ValueError("y must be a contiguous float32 tensor of 2 N_c entries")
        self._check(self.lib.tbdg_guess_inject(self.h, _ptr(self._vec(p_prev, self.N_p, "p_prev")),
                                               _ptr(self._vec(d1, self.N_p, "d1")),
                                               _ptr(self._vec(d2, self.N_p, "d2")),
                                               _ptr(self._vec(d3, self.N_p, "d3")), _ptr(y), _ptr(out)))
        return out

    def guess_target(self, p_new, p_prev, d1, d2, d3):
        """Gram target [6][N_c] float32 of a solve (training data of the network)."""
        out = torch.empty((6, self.N_c), dtype=torch.float32, device=self.device)
        self._check(self.lib.tbdg_guess_target(self.h, _ptr(self._vec(p_new, self.N_p, "p_new")),
                                               _ptr(self._vec(p_prev, self.N_p, "p_prev")),
                                               _ptr(self._vec(d1, self.N_p, "d1")),
                                               _ptr(self._vec(d2, self.N_p, "d2")),
                                               _ptr(self._vec(d3, self.N_p, "d3")), _ptr(out)))
        return out

    def profile(self, enable):
        """Bracket every operator-kernel launch with HIP events (measurement)."""
        self._check(self.lib.tbdg_profile_enable(self.h, int(bool(enable))))

    def profile_read(self, which):
        """(total kernel ms, launches) since the last read; which 0 = pressure
        operator, 1 = momentum operator."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.tbdg_profile_read(self.h, int(which), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def profile_bytes(self, which):
        """Algorithmic bytes of the timed launches since the last call."""
        b = ctypes.c_double()
        self._check(self.lib.tbdg_profile_bytes(self.h, int(which), ctypes.byref(b)))
        return b.value


class Net:
    """The learned pressure-guess network on the current HIP device and stream."""

    def __init__(self, channels=32, seed=0, stream=None, device="cuda"):
        self.lib = load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("trbdg needs a ROCm GPU device")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self.lib.tbdg_net_create(int(channels), ctypes.c_uint64(seed),
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise TrbdgError(st, "tbdg_net_create failed")
        self.h = h
        n = ctypes.c_int64()
        self._check(self.lib.tbdg_net_num_params(self.h, ctypes.byref(n)))
        self.n_params = n.value
        self.shape = None

    def _check(self, st):
        if st != 0:
            raise TrbdgError(st, self.lib.tbdg_net_last_error(self.h).decode())

    def _f32(self, t, n, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 \
                or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of {n} entries")
        return t

    def set_params(self, theta):
        self._check(self.lib.tbdg_net_set_params(self.h, _ptr(self._f32(theta, self.n_params, "theta"))))

    def params(self):
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        self._check(self.lib.tbdg_net_get_params(self.h, _ptr(out)))
        return out

    def grads(self):
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        self._check(self.lib.tbdg_net_get_grads(self.h, _ptr(out)))
        return out

    def zero_grad(self):
        self._check(self.lib.tbdg_net_zero_grad(self.h))

    def forward(self, x):
        """x: float32 [B][6][nz][ny][nx] -> y: float32 [B][2][nz][ny][nx]."""
        if x.dim() != 5 or x.shape[1] != GUESS_IN:
            raise ValueError(f"x must have shape [B][{GUESS_IN}][nz][ny][nx]")
        B, _, nz, ny, nx = x.shape
        self._f32(x, x.numel(), "x")
        y = torch.empty((B, GUESS_OUT, nz, ny, nx), dtype=torch.float32, device=self.device)
        self._check(self.lib.tbdg_net_forward(self.h, _ptr(x), _ptr(y), B, nx, ny, nz))
        self.shape = (B, GUESS_OUT, nz, ny, nx)
        return y

    def backward(self, dy):
        if self.shape is None or tuple(dy.shape) != self.shape:
            raise ValueError("dy must have the shape of the last forward output")
        self._check(self.lib.tbdg_net_backward(self.h, _ptr(self._f32(dy, dy.numel(), "dy"))))

    def mse(self, yhat, target):
        """(loss, dL/dyhat) with L = mean((yhat - target)^2)."""
        dy = torch.empty_like(yhat)
        loss = ctypes.c_double()
        self._check(self.lib.tbdg_net_mse(self.h, _ptr(self._f32(yhat, yhat.numel(), "yhat")),
                                          _ptr(self._f32(target, yhat.numel(), "target")),
                                          yhat.numel(), _ptr(dy), ctypes.byref(loss)))
        return loss.value, dy

    def quad_loss(self, yhat, gram):
        """(loss, dL/dyhat) of the guess's per-cell quadratic loss; yhat
        [B][2][...], gram [B][6][...] (float32)."""
        B = yhat.shape[0]
        n = yhat.numel() // (GUESS_OUT * B)
        dy = torch.empty_like(yhat)
        loss = ctypes.c_double()
        self._check(self.lib.tbdg_net_quad_loss(self.h, _ptr(self._f32(yhat, yhat.numel(), "yhat")),
                                                _ptr(self._f32(gram, 6 * B * n, "gram")), n, B, _ptr(dy),
                                                ctypes.byref(loss)))
        return loss.value, dy

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.tbdg_net_adam_step(self.h, lr, beta1, beta2, eps))

    def close(self):
        if getattr(self, "h", None):
            self.lib.tbdg_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Adaptive:
    """Adaptive 2D mesh with hanging nodes on the current HIP device and
    stream: the pressure Helmholtz operator and its CG solve, the vorticity
    indicator, marking and remeshing with field transfer."""

    def __init__(self, n_cells, lo, hi, k, max_level, periodic=(0, 0), pen_p=1.0, pen_u=1.0,
                 stream=None, device="cuda"):
        self.lib = load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("trbdg needs a ROCm GPU device")
        d = AmrDesc()
        for a in range(2):
            d.n_cells[a] = int(n_cells[a])
            d.lo[a] = float(lo[a])
            d.hi[a] = float(hi[a])
            d.periodic[a] = int(bool(periodic[a]))
        d.k, d.max_level, d.pen_p, d.pen_u = int(k), int(max_level), float(pen_p), float(pen_u)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self.lib.tbdg_amr_create(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h))
        if st != 0:
            raise TrbdgError(st, "tbdg_amr_create failed (invalid descriptor)")
        self.h = h
        self.k = int(k)
        self._sizes()

    def _check(self, st):
        if st != 0:
            msg = self.lib.tbdg_amr_last_error(self.h)
            raise TrbdgError(st, msg.decode() if msg else "")

    def _sizes(self):
        nc, nu, np_ = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.tbdg_amr_sizes(self.h, ctypes.byref(nc), ctypes.byref(nu), ctypes.byref(np_)))
        self.N_c, self.N_u, self.N_p = nc.value, nu.value, np_.value

    def _vec(self, t, n, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 \
                or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of {n} entries")
        return t

    def leaves(self):
        """(N_c, 3) int32 array of (level, i, j)."""
        out = np.empty((self.N_c, 3), dtype=np.int32)
        self._check(self.lib.tbdg_amr_leaves(self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def apply_pressure(self, alpha, p, out=None):
        y = out if out is not None else torch.empty(self.N_p, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_amr_apply_pressure(self.h, float(alpha), _ptr(self._vec(p, self.N_p, "p")),
                                                     _ptr(self._vec(y, self.N_p, "out"))))
        return y

    def face_qpoints(self):
        """(n, 2) tensor of the wall faces' velocity Gauss points."""
        n = ctypes.c_int64()
        self._check(self.lib.tbdg_amr_face_qpoints(self.h, ctypes.byref(n), None))
        out = torch.empty((n.value, 2), dtype=torch.float64, device=self.device)
        if n.value:
            self._check(self.lib.tbdg_amr_face_qpoints(self.h, ctypes.byref(n), _ptr(out)))
        return out

    def apply_momentum(self, mc, tnu, th, w, u, uD=None, out=None):
        y = out if out is not None else torch.empty(self.N_u, dtype=torch.float64, device=self.device)
        if uD is not None and (uD.dtype != torch.float64 or not uD.is_contiguous()):
            raise ValueError("uD must be a contiguous float64 CUDA tensor")
        self._check(self.lib.tbdg_amr_apply_momentum(
            self.h, float(mc), float(tnu), float(th), _ptr(self._vec(w, self.N_u, "w")),
            _ptr(self._vec(u, self.N_u, "u")), _ptr(uD), _ptr(self._vec(y, self.N_u, "out"))))
        return y

    def solve_momentum(self, mc, tnu, th, w, b, x, uD=None, tol=1e-10, maxiter=5000, restart=30,
                       check=True):
        info = SolveInfo()
        st = self.lib.tbdg_amr_solve_momentum(
            self.h, float(mc), float(tnu), float(th), _ptr(self._vec(w, self.N_u, "w")), _ptr(uD),
            _ptr(self._vec(b, self.N_u, "b")), _ptr(self._vec(x, self.N_u, "x")), float(tol),
            int(maxiter), int(restart), ctypes.byref(info))
        if check:
            self._check(st)
        return info.as_dict() | {"status": st}

    def set_flow(self, nu, dt, c=1.0e3):
        self._check(self.lib.tbdg_amr_set_flow(self.h, float(nu), float(dt), float(c)))

    def rhs_momentum(self, stage, u_n, u_g, w, p_prev, uD=None, w_explicit=None):
        out = torch.empty(self.N_u, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_amr_rhs_momentum(
            self.h, int(stage), _ptr(self._vec(u_n, self.N_u, "u_n")),
            _ptr(self._vec(u_g, self.N_u, "u_g") if u_g is not None else None),
            _ptr(self._vec(w, self.N_u, "w")),
            _ptr(self._vec(w_explicit, self.N_u, "w_explicit") if w_explicit is not None else None),
            _ptr(self._vec(p_prev, self.N_p, "p_prev")), _ptr(uD), _ptr(out)))
        return out

    def rhs_pressure(self, stage, u_ss, p_prev):
        out = torch.empty(self.N_p, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_amr_rhs_pressure(self.h, int(stage), _ptr(self._vec(u_ss, self.N_u, "u_ss")),
                                                   _ptr(self._vec(p_prev, self.N_p, "p_prev")), _ptr(out)))
        return out

    def add_grad_p(self, x, a, p, out=None):
        y = out if out is not None else torch.empty(self.N_u, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_amr_add_grad_p(self.h, _ptr(self._vec(x, self.N_u, "x")), float(a),
                                                 _ptr(self._vec(p, self.N_p, "p")),
                                                 _ptr(self._vec(y, self.N_u, "out"))))
        return y

    def step(self, u, u_hist, p, uD=None, nonlinear=1, mom_tol=1e-10, prs_tol=1e-10, mom_maxiter=5000,
             prs_maxiter=20000, restart=30, check=True):
        o = AmrStepOpts(int(nonlinear), float(mom_tol), float(prs_tol), int(mom_maxiter), int(prs_maxiter),
                        int(restart))
        info = (SolveInfo * 4)()
        mdu = ctypes.c_double(0.0)
        st = self.lib.tbdg_amr_step(self.h, ctypes.byref(o), _ptr(self._vec(u, self.N_u, "u")),
                                    _ptr(self._vec(u_hist, self.N_u, "u_hist")),
                                    _ptr(self._vec(p, self.N_p, "p")), _ptr(uD), info, ctypes.byref(mdu))
        if check:
            self._check(st)
        self.last_max_du = mdu.value
        return [info[q].as_dict() for q in range(4)], st

    def simulate(self, u, u_hist, p, wall_data, steps, remesh_every=1000, check_every=50,
                 check_tol=1e-2, refine_frac=0.1, coarsen_frac=0.3, h_min=0.0, h_max=float("inf"),
                 **step_kw):
        """The adaptive schedule of Sec. 4: TR-BDF2 steps; after every
        ``remesh_every`` steps, and after every ``check_every`` steps while the
        last step changed the velocity by more than ``check_tol`` (max norm),
        the indicator marks ``refine_frac`` / ``coarsen_frac`` of the cells and
        the mesh is adapted with u, u_hist and p transferred.  ``wall_data(x)``
        returns the wall velocity at the (n, 2) host points (None on a fully
        periodic mesh).  Returns the fields and a log of (step, cells)."""
        def walls():
            x = self.face_qpoints()
            if x.shape[0] == 0 or wall_data is None:
                return None
            return torch.tensor(np.asarray(wall_data(x.cpu().numpy()), dtype=np.float64),
                                device=self.device).contiguous()
        uD = walls()
        log = [(0, self.N_c)]
        for n in range(1, steps + 1):
            self.step(u, u_hist, p, uD, **step_kw)
            if n % remesh_every == 0 or (n % check_every == 0 and self.last_max_du > check_tol):
                flags = self.mark(self.indicator(u), refine_frac, coarsen_frac, h_min, h_max)
                u, u_hist, p = self.adapt(flags, [("u", u), ("u", u_hist), ("p", p)])
                uD = walls()
                log.append((n, self.N_c))
        return u, u_hist, p, log

    def diag_pressure(self, alpha):
        y = torch.empty(self.N_p, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_amr_diag_pressure(self.h, float(alpha), _ptr(y)))
        return y

    def solve_pressure(self, alpha, b, x, tol=1e-10, maxiter=5000, check=True):
        info = SolveInfo()
        st = self.lib.tbdg_amr_solve_pressure(self.h, float(alpha), _ptr(self._vec(b, self.N_p, "b")),
                                              _ptr(self._vec(x, self.N_p, "x")), float(tol), int(maxiter),
                                              ctypes.byref(info))
        if check:
            self._check(st)
        return info.as_dict() | {"status": st}

    def indicator(self, u):
        eta = torch.empty(self.N_c, dtype=torch.float64, device=self.device)
        self._check(self.lib.tbdg_amr_indicator(self.h, _ptr(self._vec(u, self.N_u, "u")), _ptr(eta)))
        return eta

    def mark(self, eta, refine_frac=0.1, coarsen_frac=0.3, h_min=0.0, h_max=float("inf")):
        flags = np.zeros(self.N_c, dtype=np.int8)
        self._check(self.lib.tbdg_amr_mark(self.h, _ptr(self._vec(eta, self.N_c, "eta")), float(refine_frac),
                                           float(coarsen_frac), float(h_min), float(h_max),
                                           flags.ctypes.data_as(ctypes.c_void_p)))
        return flags

    def adapt(self, flags, fields=()):
        """Remesh with host flags; ``fields`` = [("u" | "p", tensor), ...] on
        the current mesh; returns the transferred tensors on the new mesh."""
        flags = np.ascontiguousarray(flags, dtype=np.int8)
        if flags.size != self.N_c:
            raise ValueError(f"flags has {flags.size} entries, expected {self.N_c}")
        nn = ctypes.c_int64()
        self._check(self.lib.tbdg_amr_plan(self.h, flags.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nn)))
        nbu, nbp = 2 * (self.k + 1) ** 2, self.k ** 2
        out = []
        for kind, t in fields:
            f = 0 if kind == "u" else 1
            nb = nbu if f == 0 else nbp
            self._vec(t, self.N_c * nb, kind)
            dst = torch.empty(nn.value * nb, dtype=torch.float64, device=self.device)
            self._check(self.lib.tbdg_amr_transfer(self.h, f, _ptr(t), _ptr(dst)))
            out.append(dst)
        self._check(self.lib.tbdg_amr_commit(self.h))
        self._sizes()
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.tbdg_amr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
