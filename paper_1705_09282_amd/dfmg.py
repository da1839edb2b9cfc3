"""Python binding of libdfmg.so (the C-ABI declared in include/dfmg.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace, F and U) and the
stream.  The library must have been built (``python -m
paper_1705_09282_amd.build``); importing this module without it raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfmg.so")

c_int, c_double, c_size_t, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_i32p = ctypes.POINTER(ctypes.c_int32)
c_dblp = ctypes.POINTER(ctypes.c_double)

MAX_HISTORY = 512
MAX_STEPS = 16   # smoothing steps per phase and level (schedule entries per phase)
# Chebyshev schedule defaults: smoothing interval [b / alpha, b] and 30 power
# iterations for b.  alpha None asks the library for the ratio of the
# problem's dimension (10 in 2D, 60 in 3D).
CHEB_ITERS = 30
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTCONV", -5: "EDIVERGED", -6: "ESTATE"}


class Grid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n_elem", c_int), ("n_levels", c_int), ("geometry", c_int),
                ("r_inner", c_double), ("r_outer", c_double), ("depth", c_double)]


# the paper's quarter annulus and hollow cylinder section
ANNULUS = {"r_inner": 0.075, "r_outer": 0.225, "depth": 0.1}


def _grid(dim, n_elem, n_levels, geometry=0, shape=None):
    """dfmg_grid: geometry 0 the unit square / cube, 1 the quarter annulus
    (hollow cylinder section in 3D) with radii and depth from `shape`
    (default ANNULUS)."""
    g = Grid(dim, n_elem, n_levels, int(geometry), 0.0, 0.0, 0.0)
    if geometry:
        sh = dict(ANNULUS, **(shape or {}))
        g.r_inner, g.r_outer, g.depth = sh["r_inner"], sh["r_outer"], sh["depth"]
    return g


class Advection(ctypes.Structure):
    _fields_ = [("kind", c_int), ("c", c_double), ("coeffs", c_dblp)]


class Options(ctypes.Structure):
    _fields_ = [("nu1", c_int), ("nu2", c_int), ("eta", c_double), ("precision", c_int),
                ("smoother", c_int), ("max_cycles", c_int), ("use_graph", c_int),
                ("cycles_per_check", c_int), ("share_inverses", c_int),
                ("inner_cycles", c_int), ("multiplicative", c_int), ("time_stepping", c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("cycles", c_int), ("converged", c_int), ("status", c_int), ("fallback", c_int), ("res0", c_double),
                ("res_final", c_double), ("rho", c_double), ("fnorm", c_double),
                ("solve_seconds", c_double), ("n_history", c_int),
                ("history", c_double * MAX_HISTORY)]

    def as_dict(self):
        return {"cycles": self.cycles, "converged": bool(self.converged), "status": self.status,
                "fallback": bool(self.fallback),
                "res0": self.res0, "res_final": self.res_final, "rho": self.rho, "fnorm": self.fnorm,
                "solve_seconds": self.solve_seconds,
                "history": [self.history[i] for i in range(self.n_history)]}


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("dfmg_default_options", None, [ctypes.POINTER(Options)]),
    ("dfmg_setup", c_int, [ctypes.POINTER(Grid), c_int, c_double, c_double, ctypes.POINTER(Advection),
                           ctypes.POINTER(Options), ctypes.POINTER(c_void_p)]),
    ("dfmg_batch_setup", c_int, [c_int, ctypes.POINTER(Grid), c_int, c_dblp, c_dblp, ctypes.POINTER(Advection),
                                 ctypes.POINTER(Options), ctypes.POINTER(c_void_p)]),
    ("dfmg_batch_size", c_int, [c_void_p, ctypes.POINTER(c_int)]),
    ("dfmg_destroy", None, [c_void_p]),
    ("dfmg_workspace_bytes", c_int, [c_void_p, ctypes.POINTER(c_size_t)]),
    ("dfmg_bind", c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    ("dfmg_sizes", c_int, [c_void_p, c_int, c_i64p, c_i64p, c_i64p, c_i64p]),
    ("dfmg_set_eta", c_int, [c_void_p, c_dblp, c_int]),
    ("dfmg_vcycle", c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    ("dfmg_set_smoothing", c_int, [c_void_p, c_i32p, c_i32p, c_int]),
    ("dfmg_get_smoothing", c_int, [c_void_p, c_i32p, c_i32p]),
    ("dfmg_solve", c_int, [c_void_p, c_void_p, c_void_p, c_double, ctypes.POINTER(Stats)]),
    ("dfmg_cnab_rhs", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("dfmg_cnab_step", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, ctypes.POINTER(Stats)]),
    ("dfmg_go_rhs", c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("dfmg_residual_norm", c_int, [c_void_p, c_void_p, c_void_p, c_dblp]),
    ("dfmg_div_norm", c_int, [c_void_p, c_void_p, c_dblp]),
    ("dfmg_level_residual", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    ("dfmg_level_smooth", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int]),
    ("dfmg_level_restrict", c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    ("dfmg_level_prolong_add", c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    ("dfmg_coarse_solve", c_int, [c_void_p, c_void_p, c_void_p]),
    ("dfmg_time_kernel", c_int, [c_void_p, c_int, c_int, c_int, c_dblp]),
    ("dfmg_get_tuning", c_int, [c_void_p, c_i32p, c_i32p]),
    ("dfmg_set_tuning", c_int, [c_void_p, c_i32p, c_i32p]),
    ("dfmg_get_tile_shape", c_int, [c_void_p, c_i32p, c_i32p, c_i32p]),
    ("dfmg_set_tile_shape", c_int, [c_void_p, c_i32p, c_i32p, c_i32p]),
    ("dfmg_time_cycle", c_int, [c_void_p, c_int, c_dblp]),
    ("dfmg_autotune", c_int, [c_void_p, c_int, c_dblp]),
    ("dfmg_mlp_forward", c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("dfmg_mlp_grad", c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float, c_void_p, c_void_p,
                              c_void_p, c_void_p]),
    ("dfmg_mlp_grad_noalloc", c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float, c_void_p,
                                      c_void_p, c_void_p]),
    ("dfmg_mlp_adam", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float, c_void_p]),
    ("dfmg_set_learned", c_int, [c_void_p, ctypes.POINTER(ctypes.c_float), c_dblp]),
    ("dfmg_get_eta", c_int, [c_void_p, c_dblp]),
    ("dfmg_set_chebyshev", c_int, [c_void_p, c_double, c_int]),
    ("dfmg_get_lmax", c_int, [c_void_p, c_dblp]),
    ("dfmg_set_chebyshev_alpha", c_int, [c_void_p, c_dblp, c_int]),
    ("dfmg_get_alpha", c_int, [c_void_p, c_dblp]),
    ("dfmg_set_learned_chebyshev", c_int, [c_void_p, ctypes.POINTER(ctypes.c_float), c_dblp, c_int]),
    ("dfmg_get_schedule", c_int, [c_void_p, c_dblp]),
    ("dfmg_export_matrix", c_int, [c_void_p, c_int, c_i64p, c_i32p, c_dblp]),
    ("dfmg_patch_total", c_int, [c_void_p, c_int, c_i64p]),
    ("dfmg_export_patches", c_int, [c_void_p, c_int, c_i64p, c_i32p, c_i32p]),
    ("dfmg_export_sweep_colours", c_int, [c_void_p, c_int, c_i32p]),
    ("dfmg_prolongation_nnz", c_int, [c_void_p, c_int, c_i64p]),
    ("dfmg_export_prolongation", c_int, [c_void_p, c_int, c_i64p, c_i32p, c_dblp]),
    ("dfmg_manufactured_rhs", c_int, [c_void_p, c_dblp]),
    ("dfmg_multi_setup", c_int, [c_int, ctypes.POINTER(Grid), c_i32p, c_dblp, c_dblp, ctypes.POINTER(Advection),
                                 ctypes.POINTER(Options), ctypes.POINTER(c_void_p)]),
    ("dfmg_multi_destroy", None, [c_void_p]),
    ("dfmg_multi_layout", c_int, [c_void_p, c_i64p, ctypes.POINTER(c_int)]),
    ("dfmg_multi_workspace_bytes", c_int, [c_void_p, ctypes.POINTER(c_size_t)]),
    ("dfmg_multi_bind", c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    ("dfmg_multi_autotune", c_int, [c_void_p, c_int]),
    ("dfmg_multi_set_learned", c_int, [c_void_p, ctypes.POINTER(ctypes.c_float), c_dblp]),
    ("dfmg_multi_set_chebyshev", c_int, [c_void_p, c_double, c_int]),
    ("dfmg_multi_set_learned_chebyshev", c_int, [c_void_p, ctypes.POINTER(ctypes.c_float), c_dblp, c_int]),
    ("dfmg_multi_manufactured_rhs", c_int, [c_void_p, c_dblp]),
    ("dfmg_multi_solve", c_int, [c_void_p, c_void_p, c_void_p, c_double, ctypes.POINTER(Stats)]),
    ("dfmg_multi_residual_norm", c_int, [c_void_p, c_void_p, c_void_p, c_dblp]),
    ("dfmg_multi_div_norm", c_int, [c_void_p, c_void_p, c_dblp]),
    ("dfmg_last_error", ctypes.c_char_p, []),
]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1705_09282_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _advection(c, kind, coeffs=None, keep=None, n_v=None):
    """dfmg_advection of speed c: kind None takes rotation (1) for c != 0 and
    none (0) otherwise; kind 2 advects with c times the manufactured velocity,
    kind 3 with c times the finest-grid velocity field `coeffs` (the array is
    appended to `keep`, which must outlive the setup call; n_v its expected
    length)."""
    if kind is None:
        kind = 1 if c != 0.0 else 0
    a = Advection(int(kind), float(c), None)
    if kind == 3 and coeffs is not None:  # without a field the library reports the error
        arr = np.ascontiguousarray(coeffs, dtype=np.float64).ravel()
        if n_v is not None and arr.size != n_v:
            raise ValueError(f"advection field needs {n_v} coefficients, got {arr.size}")
        keep.append(arr)
        a.coeffs = _ptr(arr, ctypes.c_double)
    return a


def _per_problem(coeffs, nprob):
    """One coefficient array per problem from a single array or a list."""
    if coeffs is None:
        return [None] * nprob
    if isinstance(coeffs, (list, tuple)):
        if len(coeffs) != nprob:
            raise ValueError("one advection field per problem")
        return list(coeffs)
    return [coeffs] * nprob


def _network_args(W, rho_plain, nprob):
    w = np.ascontiguousarray(W, dtype=np.float32)
    if w.size != MLP_NPARAM:
        raise ValueError(f"expected {MLP_NPARAM} parameters")
    r = None if rho_plain is None else np.ascontiguousarray(rho_plain, dtype=np.float64)
    if r is not None and r.size != nprob:
        raise ValueError("one plain rate per problem")
    return w, r


class DfmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(code):
    if code != 0:
        raise DfmgError(code, lib().dfmg_last_error().decode())
    return code


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dev(t, n):
    """Device pointer of a contiguous FP64 torch tensor of n entries on the GPU."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return c_void_p(t.data_ptr())


MLP_NPARAM = 1546
MLP_NOUT = 10


def _devf(t, n):
    """Device pointer of a contiguous FP32 torch tensor of n entries on the GPU."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return c_void_p(t.data_ptr())


def _stream(t):
    import torch
    return c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_forward(W, X, Z):
    """Z (n x 10) = outputs of the smoothing-parameter network for X (n x 4)."""
    n = X.numel() // 4
    _check(lib().dfmg_mlp_forward(n, _devf(W, MLP_NPARAM), _devf(X, 4 * n), _devf(Z, MLP_NOUT * n), _stream(W)))


def mlp_grad(W, X, Y, M, scale, work, G, loss):
    """G = gradient and loss[0] = value of scale * sum M (Z - Y)^2."""
    n = X.numel() // 4
    _check(lib().dfmg_mlp_grad(n, _devf(W, MLP_NPARAM), _devf(X, 4 * n), _devf(Y, MLP_NOUT * n), _devf(M, MLP_NOUT * n),
                               float(scale), _devf(work, n * (MLP_NPARAM + 1)), _devf(G, MLP_NPARAM),
                               _devf(loss, 1), _stream(W)))


MLP_SCRATCH_SAMPLES = 512


def mlp_grad_noalloc(W, X, Y, M, scale, G, loss):
    """mlp_grad with the library's static scratch instead of a work array
    (at most MLP_SCRATCH_SAMPLES samples; no device allocation)."""
    n = X.numel() // 4
    _check(lib().dfmg_mlp_grad_noalloc(n, _devf(W, MLP_NPARAM), _devf(X, 4 * n), _devf(Y, MLP_NOUT * n),
                                       _devf(M, MLP_NOUT * n), float(scale), _devf(G, MLP_NPARAM),
                                       _devf(loss, 1), _stream(W)))


def mlp_adam(W, m, v, G, t, lr):
    _check(lib().dfmg_mlp_adam(_devf(W, MLP_NPARAM), _devf(m, MLP_NPARAM), _devf(v, MLP_NPARAM),
                               _devf(G, MLP_NPARAM), int(t), float(lr), _stream(W)))


def default_options(**kw):
    o = Options()
    lib().dfmg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Solver:
    """Hierarchy for one problem: unit square (dim 2) or cube (dim 3),
    n_elem elements per direction on the finest of n_levels grids, pressure
    degree k, viscosity nu, reaction sigma, rotation advection speed c.
    A Solver is the batch of one; BatchSolver holds several problems on the
    same mesh and solves them together."""

    def __init__(self, dim, n_elem, n_levels, k, nu=1.0, sigma=1.0, c=0.0, adv_kind=None, adv_coeffs=None,
                 geometry=0, shape=None, **options):
        self._init(dim, n_elem, n_levels, k, [nu], [sigma], [c], options, adv_kind, adv_coeffs, geometry, shape)

    def _init(self, dim, n_elem, n_levels, k, nus, sigmas, cs, options, adv_kind=None, adv_coeffs=None,
              geometry=0, shape=None):
        self.dim, self.n_elem, self.n_levels, self.k = dim, n_elem, n_levels, k
        self.nprob = len(nus)
        self.nus, self.sigmas, self.cs = list(nus), list(sigmas), list(cs)
        if not (len(sigmas) == len(cs) == self.nprob):
            raise ValueError("one nu, sigma and c per problem")
        g = _grid(dim, n_elem, n_levels, geometry, shape)
        self.geometry = int(geometry)
        self.adv_kind = adv_kind
        keep = []
        fields = _per_problem(adv_coeffs, self.nprob)
        n_v = dim * (n_elem + k - 1) * (n_elem + k) ** (dim - 1)
        adv = (Advection * self.nprob)(*[_advection(c, adv_kind, f, keep, n_v) for c, f in zip(cs, fields)])
        nu_a = np.ascontiguousarray(nus, dtype=np.float64)
        sg_a = np.ascontiguousarray(sigmas, dtype=np.float64)
        opt = default_options(**options)
        self._options = dict(options)
        ctx = c_void_p()
        self._ctx = c_void_p()
        _check(lib().dfmg_batch_setup(self.nprob, ctypes.byref(g), k, _ptr(nu_a, ctypes.c_double),
                                      _ptr(sg_a, ctypes.c_double), adv, ctypes.byref(opt), ctypes.byref(ctx)))
        self._ctx = ctx
        self._ws = None
        self._sizes = {}

    # ---------------------------------------------------------------- host
    def sizes(self, level=None):
        level = self.n_levels - 1 if level is None else level
        if level in self._sizes:
            return dict(self._sizes[level])
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().dfmg_sizes(self._ctx, level, *[ctypes.byref(x) for x in v]))
        nv, nq, npatch, nnz = (x.value for x in v)
        self._sizes[level] = {"n_vel": nv, "n_pres": nq, "n": nv + nq, "n_patch": npatch, "nnz": nnz}
        return dict(self._sizes[level])

    @property
    def n(self):
        """finest-level DOFs of one problem"""
        return self.sizes()["n"]

    def _nlev(self, level):
        if not 0 <= level < self.n_levels:
            raise ValueError("level out of range")
        return self.sizes(level)["n"] * self.nprob

    def export_matrix(self, level):
        s = self.sizes(level)
        rp = np.zeros(s["n"] + 1, np.int64)
        col = np.zeros(s["nnz"], np.int32)
        val = np.zeros(s["nnz"], np.float64)
        _check(lib().dfmg_export_matrix(self._ctx, level, _ptr(rp, ctypes.c_int64), _ptr(col, ctypes.c_int32),
                                        _ptr(val, ctypes.c_double)))
        return rp, col, val

    def export_patches(self, level):
        s = self.sizes(level)
        tot = ctypes.c_int64()
        _check(lib().dfmg_patch_total(self._ctx, level, ctypes.byref(tot)))
        ptr = np.zeros(s["n_patch"] + 1, np.int64)
        dofs = np.zeros(tot.value, np.int32)
        color = np.zeros(s["n_patch"], np.int32)
        _check(lib().dfmg_export_patches(self._ctx, level, _ptr(ptr, ctypes.c_int64), _ptr(dofs, ctypes.c_int32),
                                         _ptr(color, ctypes.c_int32)))
        return ptr, dofs, color

    def export_sweep_colours(self, level):
        """Coupling-free colour of every subdomain of `level` (the visiting
        order of the multiplicative sweep)."""
        out = np.zeros(self.sizes(level)["n_patch"], np.int32)
        _check(lib().dfmg_export_sweep_colours(self._ctx, level, _ptr(out, ctypes.c_int32)))
        return out

    def export_prolongation(self, level):
        s = self.sizes(level)
        nnz = ctypes.c_int64()
        _check(lib().dfmg_prolongation_nnz(self._ctx, level, ctypes.byref(nnz)))
        rp = np.zeros(s["n"] + 1, np.int64)
        col = np.zeros(nnz.value, np.int32)
        val = np.zeros(nnz.value, np.float64)
        _check(lib().dfmg_export_prolongation(self._ctx, level, _ptr(rp, ctypes.c_int64),
                                              _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_double)))
        return rp, col, val

    def manufactured_rhs(self):
        F = np.zeros(self.n * self.nprob, np.float64)
        _check(lib().dfmg_manufactured_rhs(self._ctx, _ptr(F, ctypes.c_double)))
        return F

    def workspace_bytes(self):
        b = c_size_t()
        _check(lib().dfmg_workspace_bytes(self._ctx, ctypes.byref(b)))
        return b.value

    # -------------------------------------------------------------- device
    def bind(self, device="cuda"):
        import torch
        nbytes = self.workspace_bytes()
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        stream = torch.cuda.current_stream(self._ws.device).cuda_stream
        _check(lib().dfmg_bind(self._ctx, c_void_p(aligned), nbytes, c_void_p(stream)))
        return self

    def set_eta(self, etas):
        a = np.ascontiguousarray(etas, dtype=np.float64).ravel()
        _check(lib().dfmg_set_eta(self._ctx, _ptr(a, ctypes.c_double), int(a.size)))

    def set_smoothing(self, nu1, nu2):
        """Per-level smoothing steps, finest level first (n_levels - 1 each)."""
        a = np.ascontiguousarray(nu1, dtype=np.int32)
        b = np.ascontiguousarray(nu2, dtype=np.int32)
        if a.size != b.size:
            raise ValueError("nu1 and nu2 need the same length")
        _check(lib().dfmg_set_smoothing(self._ctx, _ptr(a, ctypes.c_int32), _ptr(b, ctypes.c_int32), int(a.size)))

    def get_smoothing(self):
        a = np.zeros(self.n_levels - 1, np.int32)
        b = np.zeros(self.n_levels - 1, np.int32)
        _check(lib().dfmg_get_smoothing(self._ctx, _ptr(a, ctypes.c_int32), _ptr(b, ctypes.c_int32)))
        return a.tolist(), b.tolist()

    def vcycle(self, F, U, ncycles=1):
        n = self.n * self.nprob
        _check(lib().dfmg_vcycle(self._ctx, _dev(F, n), _dev(U, n), int(ncycles)))

    def _solve(self, F, U, tol, raise_on_error):
        n = self.n * self.nprob
        st = (Stats * self.nprob)()
        code = lib().dfmg_solve(self._ctx, _dev(F, n), _dev(U, n), float(tol), st)
        if raise_on_error:
            _check(code)
        return [s.as_dict() for s in st]

    def _residual_norms(self, F, U):
        n = self.n * self.nprob
        out = np.zeros(self.nprob)
        _check(lib().dfmg_residual_norm(self._ctx, _dev(F, n), _dev(U, n), _ptr(out, ctypes.c_double)))
        return out

    def _div_norms(self, U):
        out = np.zeros(self.nprob)
        _check(lib().dfmg_div_norm(self._ctx, _dev(U, self.n * self.nprob), _ptr(out, ctypes.c_double)))
        return out

    def solve(self, F, U, tol=1e-8, raise_on_error=True):
        return self._solve(F, U, tol, raise_on_error)[0]

    def residual_norm(self, F, U):
        return float(self._residual_norms(F, U)[0])

    def cnab_rhs(self, F2, U, Uold, Fout):
        """Load of one Crank-Nicolson / Adams-Bashforth step (Uold None: the
        first step); needs time_stepping=1."""
        n = self.n * self.nprob
        _check(lib().dfmg_cnab_rhs(self._ctx, _dev(F2, n), _dev(U, n), None if Uold is None else _dev(Uold, n),
                                   _dev(Fout, n)))

    def go_rhs(self, F2, U, Fout):
        """Load of Guermond's step (the context's operator advects with
        3/2 u^n - 1/2 u^{n-1}); needs time_stepping=1."""
        n = self.n * self.nprob
        _check(lib().dfmg_go_rhs(self._ctx, _dev(F2, n), _dev(U, n), _dev(Fout, n)))

    def cnab_step(self, F2, Uold, U, Unext, tol=1e-8, raise_on_error=True):
        """One Crank-Nicolson / Adams-Bashforth step: Unext = U^{n+1} from U
        (= U^n) and Uold (= U^{n-1}, None at the first step); per-problem
        stats of its solve."""
        n = self.n * self.nprob
        st = (Stats * self.nprob)()
        code = lib().dfmg_cnab_step(self._ctx, _dev(F2, n), None if Uold is None else _dev(Uold, n), _dev(U, n),
                                    _dev(Unext, n), float(tol), st)
        if raise_on_error:
            _check(code)
        return [x.as_dict() for x in st]

    def div_norm(self, U):
        return float(self._div_norms(U)[0])

    def level_residual(self, level, F, U, r):
        n = self._nlev(level)
        _check(lib().dfmg_level_residual(self._ctx, level, _dev(F, n), _dev(U, n), _dev(r, n)))

    def level_smooth(self, level, F, U, nsteps=1):
        n = self._nlev(level)
        _check(lib().dfmg_level_smooth(self._ctx, level, _dev(F, n), _dev(U, n), int(nsteps)))

    def level_restrict(self, level, r, G):
        _check(lib().dfmg_level_restrict(self._ctx, level, _dev(r, self._nlev(level)), _dev(G, self._nlev(level - 1))))

    def level_prolong_add(self, level, dU, U):
        _check(lib().dfmg_level_prolong_add(self._ctx, level, _dev(dU, self._nlev(level - 1)), _dev(U, self._nlev(level))))

    def time_kernel(self, kernel, level, reps=50):
        """Average milliseconds per launch of kernel 0 (FP64 residual), 1 (FP32
        residual), 2 (FP64 smoothing step) or 3 (FP32 smoothing step) on
        `level`, for the whole batch."""
        out = c_double()
        _check(lib().dfmg_time_kernel(self._ctx, int(kernel), int(level), int(reps), ctypes.byref(out)))
        return out.value

    def get_tuning(self):
        lpr = np.zeros(self.n_levels, np.int32)
        sm = np.zeros(self.n_levels, np.int32)
        _check(lib().dfmg_get_tuning(self._ctx, _ptr(lpr, ctypes.c_int32), _ptr(sm, ctypes.c_int32)))
        out = {"lpr": lpr.tolist(), "smoother": sm.tolist()}
        out["tile"] = self.get_tile_shape()
        return out

    def set_tuning(self, lpr, smoother, tile=None):
        lpr = np.ascontiguousarray(lpr, dtype=np.int32)
        sm = np.ascontiguousarray(smoother, dtype=np.int32)
        if lpr.size != self.n_levels or sm.size != self.n_levels:
            raise ValueError("one entry per level")
        _check(lib().dfmg_set_tuning(self._ctx, _ptr(lpr, ctypes.c_int32), _ptr(sm, ctypes.c_int32)))
        if tile is not None:
            self.set_tile_shape(tile["bs"], tile["ms"], tile["tb"])

    def get_tile_shape(self):
        """Tile shape of the form-4 local solves per level: threads per
        workgroup (bs), reading of shared inverses (ms), threads per boundary
        subdomain (tb)."""
        a = [np.zeros(self.n_levels, np.int32) for _ in range(3)]
        _check(lib().dfmg_get_tile_shape(self._ctx, *[_ptr(x, ctypes.c_int32) for x in a]))
        return {"bs": a[0].tolist(), "ms": a[1].tolist(), "tb": a[2].tolist()}

    def set_tile_shape(self, bs, ms, tb):
        a = [np.ascontiguousarray(x, dtype=np.int32) for x in (bs, ms, tb)]
        if any(x.size != self.n_levels for x in a):
            raise ValueError("one entry per level")
        _check(lib().dfmg_set_tile_shape(self._ctx, *[_ptr(x, ctypes.c_int32) for x in a]))

    def time_cycle(self, reps=20):
        """Milliseconds of one captured V-cycle (best of three rounds)."""
        out = c_double()
        _check(lib().dfmg_time_cycle(self._ctx, int(reps), ctypes.byref(out)))
        return out.value

    def tuning_key(self):
        """Cache key of the tuned variants: dimension, degree, grid, levels,
        precision, smoother and batch size."""
        o = self._options
        return (f"d{self.dim}-k{self.k}-N{self.n_elem}-L{self.n_levels}-p{o.get('precision', 0)}"
                f"-m{o.get('multiplicative', 0)}-b{self.nprob}")

    def autotune(self, reps=20, cache=None, key=None):
        """Pick the fastest kernel variant and tile shape per level by timing
        on the device.  With ``cache`` (a JSON file path) a stored choice
        under ``key`` (default: tuning_key(), the dimension, degree, grid,
        levels, precision, smoother and batch size) is reused instead of
        timing, and a new choice is stored."""
        import json
        if cache and not key:
            key = self.tuning_key()
        if cache and key and os.path.exists(cache):
            try:
                stored = json.load(open(cache)).get(key)
            except ValueError:
                stored = None
            if stored:
                self.set_tuning(stored["lpr"], stored["smoother"], stored.get("tile"))
                return dict(stored, cached=True)
        ms = np.zeros(2 * self.n_levels)
        _check(lib().dfmg_autotune(self._ctx, int(reps), _ptr(ms, ctypes.c_double)))
        out = self.get_tuning()
        out["ms"] = ms.tolist()
        if cache and key:
            data = {}
            if os.path.exists(cache):
                try:
                    data = json.load(open(cache))
                except ValueError:
                    data = {}
            data[key] = {"lpr": out["lpr"], "smoother": out["smoother"], "tile": out["tile"], "ms": out["ms"]}
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        out["cached"] = False
        return out

    def set_learned(self, W, rho_plain=None):
        """Dampings (per problem) and smoothing steps (per batch) from the
        network W (1546 floats); with rho_plain (one per problem) a solve falls
        back to the fixed damping when a cycle contracts worse than
        1.05 * rho_plain.  W None: fixed damping, the options' steps."""
        if W is None:
            _check(lib().dfmg_set_learned(self._ctx, None, None))
            return
        w = np.ascontiguousarray(W, dtype=np.float32)
        if w.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        r = None
        if rho_plain is not None:
            r = np.ascontiguousarray(rho_plain, dtype=np.float64)
            if r.size != self.nprob:
                raise ValueError("one plain rate per problem")
        _check(lib().dfmg_set_learned(self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                      None if r is None else _ptr(r, ctypes.c_double)))

    def get_eta(self):
        """Current dampings, one row per problem, finest level first."""
        out = np.zeros(self.nprob * (self.n_levels - 1))
        _check(lib().dfmg_get_eta(self._ctx, _ptr(out, ctypes.c_double)))
        return out.reshape(self.nprob, self.n_levels - 1)

    def set_chebyshev(self, alpha=None, iters=CHEB_ITERS):
        """Chebyshev damping schedule on [b / alpha, b] per problem and level
        (b from a power-iteration estimate of the largest eigenvalue of the
        undamped smoother's operator); alpha None: the default of the
        dimension; 0 turns it off."""
        _check(lib().dfmg_set_chebyshev(self._ctx, -1.0 if alpha is None else float(alpha), int(iters)))

    def set_chebyshev_alpha(self, alphas):
        """Interval ratios per smoothed level (finest first), one row for all
        problems or one row per problem."""
        a = np.ascontiguousarray(alphas, dtype=np.float64).ravel()
        _check(lib().dfmg_set_chebyshev_alpha(self._ctx, _ptr(a, ctypes.c_double), int(a.size)))

    def get_alpha(self):
        out = np.zeros(self.nprob * (self.n_levels - 1))
        _check(lib().dfmg_get_alpha(self._ctx, _ptr(out, ctypes.c_double)))
        return out.reshape(self.nprob, self.n_levels - 1)

    def set_learned_chebyshev(self, W, rho_plain=None, iters=CHEB_ITERS):
        """Chebyshev schedule with the interval ratio per level and the step
        counts predicted by the network W; W None turns it off."""
        if W is None:
            _check(lib().dfmg_set_learned_chebyshev(self._ctx, None, None, int(iters)))
            return
        w, r = _network_args(W, rho_plain, self.nprob)
        _check(lib().dfmg_set_learned_chebyshev(self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                None if r is None else _ptr(r, ctypes.c_double), int(iters)))

    def get_lmax(self):
        """Eigenvalue estimates of set_chebyshev, one row per problem, finest
        level first."""
        out = np.zeros(self.nprob * (self.n_levels - 1))
        _check(lib().dfmg_get_lmax(self._ctx, _ptr(out, ctypes.c_double)))
        return out.reshape(self.nprob, self.n_levels - 1)

    def get_schedule(self):
        """Per-step dampings in use: array (nprob, n_levels - 1, 2, 16),
        finest level first; [.., 0, j] pre-smoothing step j, [.., 1, j]
        post-smoothing step j."""
        out = np.zeros(self.nprob * (self.n_levels - 1) * 2 * MAX_STEPS)
        _check(lib().dfmg_get_schedule(self._ctx, _ptr(out, ctypes.c_double)))
        return out.reshape(self.nprob, self.n_levels - 1, 2, MAX_STEPS)

    def coarse_solve(self, G, dU):
        n = self._nlev(0)
        _check(lib().dfmg_coarse_solve(self._ctx, _dev(G, n), _dev(dU, n)))

    def close(self):
        if self._ctx:
            lib().dfmg_destroy(self._ctx)
            self._ctx = c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver(Solver):
    """Several independent problems on one mesh (same dim, n_elem, n_levels,
    k) with per-problem nu, sigma and rotation speed c, solved together: every
    kernel launch covers the whole batch.  Vectors are problem-major blocks of
    the finest-level length n."""

    def __init__(self, dim, n_elem, n_levels, k, nus, sigmas, cs=None, adv_kind=None, adv_coeffs=None,
                 geometry=0, shape=None, **options):
        cs = [0.0] * len(nus) if cs is None else list(cs)
        self._init(dim, n_elem, n_levels, k, list(nus), list(sigmas), cs, options, adv_kind, adv_coeffs,
                   geometry, shape)

    def solve(self, F, U, tol=1e-8, raise_on_error=True):
        return self._solve(F, U, tol, raise_on_error)

    def residual_norm(self, F, U):
        return self._residual_norms(F, U)

    def div_norm(self, U):
        return self._div_norms(U)


class MultiSolver:
    """Independent problems on different meshes: problem p is (dim, n_elem,
    n_levels, k)[p] with nu[p], sigma[p] and rotation speed c[p].  Problems
    sharing a mesh and degree run as one batch; the batches run concurrently
    on their own streams inside one captured graph per step.  Vectors: one
    FP64 array, problem p at offsets[p] .. offsets[p + 1]."""

    def __init__(self, meshes, nus, sigmas, cs=None, adv_kind=None, **options):
        self.nprob = len(meshes)
        cs = [0.0] * self.nprob if cs is None else list(cs)
        if not (len(nus) == len(sigmas) == len(cs) == self.nprob):
            raise ValueError("one mesh, nu, sigma and c per problem")
        self.meshes = [tuple(int(x) for x in m) for m in meshes]
        self.nus, self.sigmas, self.cs = list(nus), list(sigmas), list(cs)
        grids = (Grid * self.nprob)(*[_grid(d, N, L) for (d, N, L, _k) in self.meshes])
        ks = np.ascontiguousarray([m[3] for m in self.meshes], dtype=np.int32)
        self.adv_kind = adv_kind
        keep = []
        adv = (Advection * self.nprob)(*[_advection(c, adv_kind, None, keep) for c in cs])
        nu_a = np.ascontiguousarray(nus, dtype=np.float64)
        sg_a = np.ascontiguousarray(sigmas, dtype=np.float64)
        opt = default_options(**options)
        ctx = c_void_p()
        self._ctx = c_void_p()
        _check(lib().dfmg_multi_setup(self.nprob, grids, _ptr(ks, ctypes.c_int32), _ptr(nu_a, ctypes.c_double),
                                      _ptr(sg_a, ctypes.c_double), adv, ctypes.byref(opt), ctypes.byref(ctx)))
        self._ctx = ctx
        self._ws = None
        off = np.zeros(self.nprob + 1, np.int64)
        ng = c_int()
        _check(lib().dfmg_multi_layout(self._ctx, _ptr(off, ctypes.c_int64), ctypes.byref(ng)))
        self.offsets = off
        self.n_groups = ng.value

    @property
    def n_total(self):
        return int(self.offsets[-1])

    def workspace_bytes(self):
        b = c_size_t()
        _check(lib().dfmg_multi_workspace_bytes(self._ctx, ctypes.byref(b)))
        return b.value

    def bind(self, device="cuda"):
        import torch
        nbytes = self.workspace_bytes()
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        aligned = (self._ws.data_ptr() + 255) & ~255
        stream = torch.cuda.current_stream(self._ws.device).cuda_stream
        _check(lib().dfmg_multi_bind(self._ctx, c_void_p(aligned), nbytes, c_void_p(stream)))
        return self

    def autotune(self, reps=10):
        _check(lib().dfmg_multi_autotune(self._ctx, int(reps)))

    def set_learned(self, W, rho_plain=None):
        if W is None:
            _check(lib().dfmg_multi_set_learned(self._ctx, None, None))
            return
        w = np.ascontiguousarray(W, dtype=np.float32)
        if w.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        r = None if rho_plain is None else np.ascontiguousarray(rho_plain, dtype=np.float64)
        if r is not None and r.size != self.nprob:
            raise ValueError("one plain rate per problem")
        _check(lib().dfmg_multi_set_learned(self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            None if r is None else _ptr(r, ctypes.c_double)))

    def set_chebyshev(self, alpha=None, iters=CHEB_ITERS):
        """As Solver.set_chebyshev: one ratio for every group, or with alpha
        None each group's default for its dimension."""
        _check(lib().dfmg_multi_set_chebyshev(self._ctx, -1.0 if alpha is None else float(alpha), int(iters)))

    def set_learned_chebyshev(self, W, rho_plain=None, iters=CHEB_ITERS):
        if W is None:
            _check(lib().dfmg_multi_set_learned_chebyshev(self._ctx, None, None, int(iters)))
            return
        w, r = _network_args(W, rho_plain, self.nprob)
        _check(lib().dfmg_multi_set_learned_chebyshev(self._ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                      None if r is None else _ptr(r, ctypes.c_double), int(iters)))

    def manufactured_rhs(self):
        F = np.zeros(self.n_total, np.float64)
        _check(lib().dfmg_multi_manufactured_rhs(self._ctx, _ptr(F, ctypes.c_double)))
        return F

    def solve(self, F, U, tol=1e-8, raise_on_error=True):
        st = (Stats * self.nprob)()
        code = lib().dfmg_multi_solve(self._ctx, _dev(F, self.n_total), _dev(U, self.n_total), float(tol), st)
        if raise_on_error:
            _check(code)
        return [x.as_dict() for x in st]

    def residual_norm(self, F, U):
        out = np.zeros(self.nprob)
        _check(lib().dfmg_multi_residual_norm(self._ctx, _dev(F, self.n_total), _dev(U, self.n_total),
                                              _ptr(out, ctypes.c_double)))
        return out

    def div_norm(self, U):
        out = np.zeros(self.nprob)
        _check(lib().dfmg_multi_div_norm(self._ctx, _dev(U, self.n_total), _ptr(out, ctypes.c_double)))
        return out

    def close(self):
        if self._ctx:
            lib().dfmg_multi_destroy(self._ctx)
            self._ctx = c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
