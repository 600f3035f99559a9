"""Python binding of the C ABI in include/nfs.h (argument marshalling only).

Every step of the path runs in the HIP kernels of lib/libnfs.so; this module
only checks tensor types, allocates the workspace and the outputs with
PyTorch on the current device, and passes raw pointers and the current HIP
stream.  It raises if the library is missing: there is no fallback.
"""
import ctypes
import os
from dataclasses import dataclass, field

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libnfs.so")

NFS_OK, NFS_EINVAL, NFS_EWEIGHTS, NFS_ENONPOS, NFS_EUNSUPPORTED, NFS_EHIP, NFS_EWORKSPACE = range(7)
NFS_FP64, NFS_FP32, NFS_AUTO = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20   # NFS_NOALLOC_SCRATCH_BYTES of include/nfs.h
FLAG_NO_GRAPH, FLAG_PRIMAL_COST, FLAG_TILE_REDUCE, FLAG_LOG_DOMAIN, FLAG_AUTOTUNE, FLAG_CENTER = 1, 2, 4, 8, 16, 32

EXPORTED = ("nfs_last_error", "nfs_validate", "nfs_workspace_size", "nfs_fastsum_apply",
            "nfs_fastsum_apply_noalloc",
            "nfs_nfft_adjoint", "nfs_nfft_trafo", "nfs_sinkhorn_solve", "nfs_sinkhorn_solve_log",
            "nfs_sinkhorn_grad", "nfs_sinkhorn_grad_targets", "nfs_plan_apply",
            "nfs_solver_create", "nfs_solver_iterate", "nfs_solver_residual", "nfs_solver_finish",
            "nfs_solver_profile", "nfs_solver_grad", "nfs_solver_destroy", "nfs_batch_workspace_size",
            "nfs_batch_solver_create", "nfs_batch_solve", "nfs_divergence_workspace_size",
            "nfs_sinkhorn_divergence")


class NfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nfs error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("r", ctypes.c_int32), ("eps", ctypes.c_double),
                ("N", ctypes.c_int32), ("m", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("precision", ctypes.c_int32), ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("eps_I", ctypes.c_double), ("p_smooth", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rexp", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_double), ("cost_upper", ctypes.c_double),
                ("cost_primal", ctypes.c_double), ("marg_err", ctypes.c_double),
                ("marg_err_row", ctypes.c_double), ("marg_err_col", ctypes.c_double),
                ("scale", ctypes.c_double), ("kernel_err", ctypes.c_double),
                ("iters", ctypes.c_int32), ("precision_used", ctypes.c_int32),
                ("n_nonpos", ctypes.c_int64), ("dyn_range", ctypes.c_double), ("centred", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


@dataclass
class Params:
    """Problem and fast-summation parameters (see include/nfs.h)."""
    d: int
    eps: float
    N: int
    m: int
    r: float = 2  # cost exponent: 1, 2, or a real value in (1, 4] (rexp of the C params)
    sigma: float = 2.0
    precision: str = "fp64"
    tile: int = 0
    chunk: int = 0
    flags: int = 0
    eps_I: float = 0.0
    p_smooth: int = 0

    def to_c(self):
        prec = {"fp64": NFS_FP64, "fp32": NFS_FP32, "auto": NFS_AUTO}[self.precision]
        r, rexp = (int(self.r), 0.0) if float(self.r) in (1.0, 2.0) else (0, float(self.r))
        return _Params(self.d, r, self.eps, self.N, self.m, self.sigma, prec, self.tile,
                       self.chunk, self.flags, self.eps_I, self.p_smooth, 0, rexp)


_lib = None


def load_library():
    """Load lib/libnfs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    PP = ctypes.POINTER(_Params)
    lib.nfs_last_error.restype = ctypes.c_char_p
    lib.nfs_last_error.argtypes = []
    lib.nfs_validate.restype = ctypes.c_int
    lib.nfs_validate.argtypes = [PP, I64, I64]
    lib.nfs_workspace_size.restype = ctypes.c_int
    lib.nfs_workspace_size.argtypes = [PP, I64, I64, ctypes.POINTER(SZ)]
    lib.nfs_fastsum_apply.restype = ctypes.c_int
    lib.nfs_fastsum_apply.argtypes = [PP, P, I64, P, P, I64, P, P, SZ, P]
    lib.nfs_fastsum_apply_noalloc.restype = ctypes.c_int
    lib.nfs_fastsum_apply_noalloc.argtypes = [PP, P, I64, P, P, I64, P, P]
    lib.nfs_nfft_adjoint.restype = ctypes.c_int
    lib.nfs_nfft_adjoint.argtypes = [PP, P, I64, P, P, P, SZ, P]
    lib.nfs_nfft_trafo.restype = ctypes.c_int
    lib.nfs_nfft_trafo.argtypes = [PP, P, P, I64, P, P, SZ, P]
    lib.nfs_sinkhorn_solve.restype = ctypes.c_int
    lib.nfs_sinkhorn_solve.argtypes = [PP, P, I64, P, P, I64, P, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int32, P, P, ctypes.POINTER(_Result), P, SZ, P]
    lib.nfs_sinkhorn_solve_log.restype = ctypes.c_int
    lib.nfs_sinkhorn_solve_log.argtypes = lib.nfs_sinkhorn_solve.argtypes
    lib.nfs_sinkhorn_grad.restype = ctypes.c_int
    lib.nfs_sinkhorn_grad.argtypes = [PP, P, I64, P, P, I64, P, P, P, P, P, P, SZ, P]
    lib.nfs_sinkhorn_grad_targets.restype = ctypes.c_int
    lib.nfs_sinkhorn_grad_targets.argtypes = lib.nfs_sinkhorn_grad.argtypes
    lib.nfs_plan_apply.restype = ctypes.c_int
    lib.nfs_plan_apply.argtypes = [PP, P, I64, P, I64, P, P, P, ctypes.c_int32, P, P, SZ, P]
    lib.nfs_solver_create.restype = ctypes.c_int
    lib.nfs_solver_create.argtypes = [PP, P, I64, P, P, I64, P, P, P, SZ, P, ctypes.POINTER(P)]
    lib.nfs_solver_iterate.restype = ctypes.c_int
    lib.nfs_solver_iterate.argtypes = [P, ctypes.c_int32, P]
    lib.nfs_solver_residual.restype = ctypes.c_int
    lib.nfs_solver_residual.argtypes = [P, ctypes.POINTER(ctypes.c_double), P]
    lib.nfs_solver_finish.restype = ctypes.c_int
    lib.nfs_solver_finish.argtypes = [P, P, P, ctypes.POINTER(_Result), P]
    lib.nfs_solver_profile.restype = ctypes.c_int
    lib.nfs_solver_profile.argtypes = [P, ctypes.c_int32, P, P, P]
    lib.nfs_solver_grad.restype = ctypes.c_int
    lib.nfs_solver_grad.argtypes = [P, P, P, P, P, P]
    lib.nfs_solver_destroy.restype = ctypes.c_int
    lib.nfs_solver_destroy.argtypes = [P]
    PI64, PD = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    lib.nfs_batch_workspace_size.restype = ctypes.c_int
    lib.nfs_batch_workspace_size.argtypes = [PP, ctypes.c_int32, PI64, PI64, ctypes.POINTER(SZ)]
    lib.nfs_batch_solver_create.restype = ctypes.c_int
    lib.nfs_batch_solver_create.argtypes = [PP, ctypes.c_int32, PI64, PI64, PD, P, P, P, P, P, P, SZ, P,
                                            ctypes.POINTER(P)]
    lib.nfs_batch_solve.restype = ctypes.c_int
    lib.nfs_batch_solve.argtypes = [PP, ctypes.c_int32, PI64, PI64, PD, P, P, P, P, ctypes.c_int32,
                                    ctypes.c_double, P, P, ctypes.POINTER(_Result), P, SZ, P]
    lib.nfs_divergence_workspace_size.restype = ctypes.c_int
    lib.nfs_divergence_workspace_size.argtypes = [PP, I64, I64, ctypes.POINTER(SZ)]
    lib.nfs_sinkhorn_divergence.restype = ctypes.c_int
    lib.nfs_sinkhorn_divergence.argtypes = [PP, P, I64, P, P, I64, P, ctypes.c_int32, ctypes.c_double,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_Result), P, SZ, P]
    _lib = lib
    return lib


def _check(rc):
    if rc != NFS_OK:
        raise NfsError(rc, load_library().nfs_last_error().decode())


def validate(params, n, nt):
    """CPU-only argument check; returns the error code (0 = valid)."""
    lib = load_library()
    return lib.nfs_validate(ctypes.byref(params.to_c()), int(n), int(nt))


def workspace_size(params, n, nt):
    lib = load_library()
    out = ctypes.c_size_t(0)
    _check(lib.nfs_workspace_size(ctypes.byref(params.to_c()), int(n), int(nt), ctypes.byref(out)))
    return out.value


def _dev(t, name, shape0=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return t


def _pts(t, d, name):
    _dev(t, name)
    if t.dim() == 1 and d == 1:
        return t
    if t.dim() != 2 or t.shape[1] != d:
        raise ValueError(f"{name} must have shape (n, {d})")
    return t


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(params, n, nt, device):
    nbytes = workspace_size(params, n, nt)
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def fastsum(params, src, w, tgt):
    """out_i = sum_j w_j exp(-|tgt_i - src_j|^r / eps) by NFFT fast summation."""
    lib = load_library()
    src = _pts(src, params.d, "src")
    tgt = _pts(tgt, params.d, "tgt")
    _dev(w, "w")
    ns, nt = src.shape[0], tgt.shape[0]
    out = torch.empty(nt, dtype=torch.float64, device=tgt.device)
    ws, nb = _workspace(params, ns, nt, tgt.device)
    _check(lib.nfs_fastsum_apply(ctypes.byref(params.to_c()), src.data_ptr(), ns, w.data_ptr(),
                                 tgt.data_ptr(), nt, out.data_ptr(), ws.data_ptr(), nb, _stream()))
    return out


def fastsum_noalloc(params, src, w, tgt, out=None):
    """fastsum() through the allocation-free entry point: no workspace, the
    library's static device scratch (NFS_NOALLOC_SCRATCH_BYTES) instead.
    `out` (nt float64 GPU values) may be passed in to keep the call free of
    allocations on the Python side as well."""
    lib = load_library()
    src = _pts(src, params.d, "src")
    tgt = _pts(tgt, params.d, "tgt")
    _dev(w, "w")
    ns, nt = src.shape[0], tgt.shape[0]
    if out is None:
        out = torch.empty(nt, dtype=torch.float64, device=tgt.device)
    else:
        _dev(out, "out")
        if out.numel() != nt:
            raise ValueError("out must hold one value per target")
    _check(lib.nfs_fastsum_apply_noalloc(ctypes.byref(params.to_c()), src.data_ptr(), ns, w.data_ptr(),
                                         tgt.data_ptr(), nt, out.data_ptr(), _stream()))
    return out


def nfft_adjoint(params, pts, w):
    """fhat_k = sum_j w_j exp(-2 pi i k.y_j), k in I_N; returns complex128 of shape (N,)*d."""
    lib = load_library()
    pts = _pts(pts, params.d, "pts")
    _dev(w, "w")
    n = pts.shape[0]
    out = torch.empty(params.N ** params.d * 2, dtype=torch.float64, device=pts.device)
    ws, nb = _workspace(params, n, 1, pts.device)
    _check(lib.nfs_nfft_adjoint(ctypes.byref(params.to_c()), pts.data_ptr(), n, w.data_ptr(),
                                out.data_ptr(), ws.data_ptr(), nb, _stream()))
    return torch.view_as_complex(out.view(-1, 2)).reshape((params.N,) * params.d)


def nfft_trafo(params, fhat, pts):
    """out_i = Re sum_{k in I_N} fhat_k exp(2 pi i k.x_i)."""
    lib = load_library()
    pts = _pts(pts, params.d, "pts")
    if fhat.dtype != torch.complex128 or not fhat.is_cuda:
        raise TypeError("fhat must be a complex128 GPU tensor")
    fr = torch.view_as_real(fhat.contiguous()).contiguous()
    n = pts.shape[0]
    out = torch.empty(n, dtype=torch.float64, device=pts.device)
    ws, nb = _workspace(params, n, 1, pts.device)
    _check(lib.nfs_nfft_trafo(ctypes.byref(params.to_c()), fr.data_ptr(), pts.data_ptr(), n,
                              out.data_ptr(), ws.data_ptr(), nb, _stream()))
    return out


_PREC_NAME = {NFS_FP64: "fp64", NFS_FP32: "fp32"}


@dataclass
class SinkhornResult:
    alpha: torch.Tensor
    alpha_t: torch.Tensor
    cost: float
    cost_upper: float
    cost_primal: float
    marg_err: float
    marg_err_row: float
    marg_err_col: float
    iters: int
    n_nonpos: int
    scale: float
    kernel_err: float
    precision_used: str = ""
    extra: dict = field(default_factory=dict)
    dyn_range: float = float("nan")   # max over half-steps of ||w||_1 / min t (see include/nfs.h)
    centred: bool = False             # solved in the centred form (FLAG_CENTER)


def sinkhorn(params, x, mu, y, nu, iters, tol=0.0, alpha_t0=None, workspace=None, check=True):
    """NFFT-accelerated Sinkhorn (Algorithm 3) on the GPU; returns a SinkhornResult."""
    lib = load_library()
    x = _pts(x, params.d, "x")
    y = _pts(y, params.d, "y")
    _dev(mu, "mu")
    _dev(nu, "nu")
    n, nt = x.shape[0], y.shape[0]
    alpha = torch.empty(n, dtype=torch.float64, device=x.device)
    if alpha_t0 is not None:
        alpha_t = _dev(alpha_t0, "alpha_t0").clone()
    else:
        alpha_t = torch.empty(nt, dtype=torch.float64, device=x.device)
    if workspace is None:
        ws, nb = _workspace(params, n, nt, x.device)
    else:
        ws, nb = workspace, workspace.numel()
    res = _Result()
    rc = lib.nfs_sinkhorn_solve(ctypes.byref(params.to_c()), x.data_ptr(), n, mu.data_ptr(),
                                y.data_ptr(), nt, nu.data_ptr(), int(iters), float(tol),
                                1 if alpha_t0 is not None else 0, alpha.data_ptr(), alpha_t.data_ptr(),
                                ctypes.byref(res), ws.data_ptr(), nb, _stream())
    if rc != NFS_OK and (check or rc != NFS_ENONPOS):
        _check(rc)
    return SinkhornResult(alpha, alpha_t, res.cost, res.cost_upper, res.cost_primal, res.marg_err,
                          res.marg_err_row, res.marg_err_col, res.iters, res.n_nonpos, res.scale,
                          res.kernel_err, _PREC_NAME.get(res.precision_used, ""), dyn_range=res.dyn_range,
                          centred=bool(res.centred))


@dataclass
class LogSinkhornResult:
    """Result of the log-domain solve: potentials beta (n) and gamma (nt),
    alpha = exp(beta/eps - 1/2), alpha_t = exp(gamma/eps - 1/2)."""
    beta: torch.Tensor
    gamma: torch.Tensor
    cost: float
    cost_upper: float
    marg_err: float
    marg_err_row: float
    marg_err_col: float
    iters: int
    n_nonpos: int
    scale: float
    kernel_err: float
    precision_used: str = ""


def sinkhorn_log(params, x, mu, y, nu, iters, tol=0.0, gamma0=None, workspace=None, check=True):
    """NFFT-accelerated log-domain Sinkhorn (Algorithm 4) on the GPU; returns a
    LogSinkhornResult.  gamma0 (nt, finite) is the starting value of gamma
    (zeros when None)."""
    lib = load_library()
    x = _pts(x, params.d, "x")
    y = _pts(y, params.d, "y")
    _dev(mu, "mu")
    _dev(nu, "nu")
    n, nt = x.shape[0], y.shape[0]
    beta = torch.empty(n, dtype=torch.float64, device=x.device)
    if gamma0 is not None:
        gamma = _dev(gamma0, "gamma0").clone()
    else:
        gamma = torch.empty(nt, dtype=torch.float64, device=x.device)
    if workspace is None:
        ws, nb = _workspace(params, n, nt, x.device)
    else:
        ws, nb = workspace, workspace.numel()
    res = _Result()
    rc = lib.nfs_sinkhorn_solve_log(ctypes.byref(params.to_c()), x.data_ptr(), n, mu.data_ptr(),
                                    y.data_ptr(), nt, nu.data_ptr(), int(iters), float(tol),
                                    1 if gamma0 is not None else 0, beta.data_ptr(), gamma.data_ptr(),
                                    ctypes.byref(res), ws.data_ptr(), nb, _stream())
    if rc != NFS_OK and (check or rc != NFS_ENONPOS):
        _check(rc)
    return LogSinkhornResult(beta, gamma, res.cost, res.cost_upper, res.marg_err, res.marg_err_row,
                             res.marg_err_col, res.iters, res.n_nonpos, res.scale, res.kernel_err,
                             _PREC_NAME.get(res.precision_used, ""))


def sinkhorn_grad(params, x, mu, y, nu, alpha, alpha_t, want_x=True, want_mu=True):
    """Envelope gradient of the cost at (alpha, alpha_t): (grad_x (n, d), grad_mu (n,))."""
    lib = load_library()
    x = _pts(x, params.d, "x")
    y = _pts(y, params.d, "y")
    for t, nm in ((mu, "mu"), (nu, "nu"), (alpha, "alpha"), (alpha_t, "alpha_t")):
        _dev(t, nm)
    n, nt = x.shape[0], y.shape[0]
    gx = torch.empty((n, params.d), dtype=torch.float64, device=x.device) if want_x else None
    gm = torch.empty(n, dtype=torch.float64, device=x.device) if want_mu else None
    ws, nb = _workspace(params, n, nt, x.device)
    _check(lib.nfs_sinkhorn_grad(ctypes.byref(params.to_c()), x.data_ptr(), n, mu.data_ptr(),
                                 y.data_ptr(), nt, nu.data_ptr(), alpha.data_ptr(), alpha_t.data_ptr(),
                                 gx.data_ptr() if gx is not None else None,
                                 gm.data_ptr() if gm is not None else None,
                                 ws.data_ptr(), nb, _stream()))
    return gx, gm


def sinkhorn_grad_targets(params, x, mu, y, nu, alpha, alpha_t, want_y=True, want_nu=True):
    """Target side of the envelope gradient: (grad_y (nt, d), grad_nu (nt,))."""
    lib = load_library()
    x = _pts(x, params.d, "x")
    y = _pts(y, params.d, "y")
    for t, nm in ((mu, "mu"), (nu, "nu"), (alpha, "alpha"), (alpha_t, "alpha_t")):
        _dev(t, nm)
    n, nt = x.shape[0], y.shape[0]
    gy = torch.empty((nt, params.d), dtype=torch.float64, device=x.device) if want_y else None
    gn = torch.empty(nt, dtype=torch.float64, device=x.device) if want_nu else None
    ws, nb = _workspace(params, n, nt, x.device)
    _check(lib.nfs_sinkhorn_grad_targets(ctypes.byref(params.to_c()), x.data_ptr(), n, mu.data_ptr(),
                                         y.data_ptr(), nt, nu.data_ptr(), alpha.data_ptr(), alpha_t.data_ptr(),
                                         gy.data_ptr() if gy is not None else None,
                                         gn.data_ptr() if gn is not None else None,
                                         ws.data_ptr(), nb, _stream()))
    return gy, gn


def plan_apply(params, x, y, alpha, alpha_t, v, transpose=False):
    """pi v (n values) or, with transpose, pi^T v (nt values), pi = diag(alpha) K diag(alpha_t)."""
    lib = load_library()
    x = _pts(x, params.d, "x")
    y = _pts(y, params.d, "y")
    for t, nm in ((alpha, "alpha"), (alpha_t, "alpha_t"), (v, "v")):
        _dev(t, nm)
    n, nt = x.shape[0], y.shape[0]
    if v.shape[0] != (n if transpose else nt):
        raise ValueError("v has the wrong length")
    out = torch.empty(nt if transpose else n, dtype=torch.float64, device=x.device)
    ws, nb = _workspace(params, n, nt, x.device)
    _check(lib.nfs_plan_apply(ctypes.byref(params.to_c()), x.data_ptr(), n, y.data_ptr(), nt, alpha.data_ptr(),
                              alpha_t.data_ptr(), v.data_ptr(), 1 if transpose else 0, out.data_ptr(),
                              ws.data_ptr(), nb, _stream()))
    return out


class Solver:
    """Persistent Sinkhorn state on the GPU (nfs_solver_* entry points).

    The plan runs once in the constructor; ``iterate(k)`` replays the captured
    iteration k times; ``finish()`` returns a SinkhornResult without ending
    the solver; ``profile(k)`` times the stages with events.
    """

    def __init__(self, params, x, mu, y, nu, alpha_t0=None):
        lib = load_library()
        self.params = params
        self.x = _pts(x, params.d, "x")
        self.y = _pts(y, params.d, "y")
        self.mu = _dev(mu, "mu")
        self.nu = _dev(nu, "nu")
        self.n, self.nt = self.x.shape[0], self.y.shape[0]
        self.ws, self.nb = _workspace(params, self.n, self.nt, self.x.device)
        a0 = None if alpha_t0 is None else _dev(alpha_t0, "alpha_t0")
        h = ctypes.c_void_p()
        _check(lib.nfs_solver_create(ctypes.byref(params.to_c()), self.x.data_ptr(), self.n,
                                     self.mu.data_ptr(), self.y.data_ptr(), self.nt, self.nu.data_ptr(),
                                     a0.data_ptr() if a0 is not None else None, self.ws.data_ptr(),
                                     self.nb, _stream(), ctypes.byref(h)))
        self.h = h

    def iterate(self, k):
        _check(load_library().nfs_solver_iterate(self.h, int(k), _stream()))

    def residual(self):
        e = ctypes.c_double(0.0)
        _check(load_library().nfs_solver_residual(self.h, ctypes.byref(e), _stream()))
        return e.value

    def finish(self, check=True):
        lib = load_library()
        alpha = torch.empty(self.n, dtype=torch.float64, device=self.x.device)
        alpha_t = torch.empty(self.nt, dtype=torch.float64, device=self.x.device)
        res = _Result()
        rc = lib.nfs_solver_finish(self.h, alpha.data_ptr(), alpha_t.data_ptr(), ctypes.byref(res), _stream())
        if rc != NFS_OK and (check or rc != NFS_ENONPOS):
            _check(rc)
        return SinkhornResult(alpha, alpha_t, res.cost, res.cost_upper, res.cost_primal, res.marg_err,
                              res.marg_err_row, res.marg_err_col, res.iters, res.n_nonpos, res.scale,
                              res.kernel_err, dyn_range=res.dyn_range, centred=bool(res.centred))

    def grad(self, want_x=True, want_mu=True, want_y=False, want_nu=False):
        """Envelope gradient at the current scalings on the solver's own plan
        (nfs_solver_grad): (grad_x (n, d), grad_mu (n,), grad_y (nt, d),
        grad_nu (nt,)), None where not wanted; batch solvers return the packed
        arrays."""
        dev, d = self.x.device, self.params.d
        gx = torch.empty((self.n, d), dtype=torch.float64, device=dev) if want_x else None
        gm = torch.empty(self.n, dtype=torch.float64, device=dev) if want_mu else None
        gy = torch.empty((self.nt, d), dtype=torch.float64, device=dev) if want_y else None
        gn = torch.empty(self.nt, dtype=torch.float64, device=dev) if want_nu else None
        ptr = lambda t: t.data_ptr() if t is not None else None
        _check(load_library().nfs_solver_grad(self.h, ptr(gx), ptr(gm), ptr(gy), ptr(gn), _stream()))
        return gx, gm, gy, gn

    def profile(self, k):
        """Average device ms per launch of (spread, fft chain, interp+update, iteration, near field)
        and sizes."""
        st = (ctypes.c_double * 5)()
        info = (ctypes.c_double * 9)()
        _check(load_library().nfs_solver_profile(self.h, int(k), st, info, _stream()))
        keys = ("n", "nt", "d", "grid_cells", "grid_value_bytes", "chunks_x", "chunks_y", "taps_per_point", "tile")
        return list(st), dict(zip(keys, list(info)))

    def close(self):
        if self.h is not None and self.h.value:
            load_library().nfs_solver_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _results(arr, alpha, alpha_t, offs_x, offs_y):
    out = []
    for b, r in enumerate(arr):
        out.append(SinkhornResult(alpha[offs_x[b]:offs_x[b + 1]], alpha_t[offs_y[b]:offs_y[b + 1]], r.cost,
                                  r.cost_upper, r.cost_primal, r.marg_err, r.marg_err_row, r.marg_err_col,
                                  r.iters, r.n_nonpos, r.scale, r.kernel_err, _PREC_NAME.get(r.precision_used, ""),
                                  dyn_range=r.dyn_range, centred=bool(r.centred)))
    return out


class BatchSolver(Solver):
    """Many independent problems (same d, N, m, sigma) in one solver.

    ``xs, mus, ys, nus`` are lists of GPU float64 tensors, ``eps`` a list of
    floats.  ``finish()`` returns one SinkhornResult per problem.
    """

    def __init__(self, params, xs, mus, ys, nus, eps):
        lib = load_library()
        self.params = params
        self.nprob = len(xs)
        self.ns = [int(x.shape[0]) for x in xs]
        self.nts = [int(y.shape[0]) for y in ys]
        self.offs_x = [0]
        self.offs_y = [0]
        for a, b in zip(self.ns, self.nts):
            self.offs_x.append(self.offs_x[-1] + a)
            self.offs_y.append(self.offs_y[-1] + b)
        self.x = torch.cat([_pts(x, params.d, "x").reshape(-1, params.d) for x in xs]).contiguous()
        self.y = torch.cat([_pts(y, params.d, "y").reshape(-1, params.d) for y in ys]).contiguous()
        self.mu = torch.cat([_dev(m, "mu") for m in mus]).contiguous()
        self.nu = torch.cat([_dev(m, "nu") for m in nus]).contiguous()
        self.n, self.nt = self.x.shape[0], self.y.shape[0]
        n_arr = (ctypes.c_int64 * self.nprob)(*self.ns)
        nt_arr = (ctypes.c_int64 * self.nprob)(*self.nts)
        self.eps = (ctypes.c_double * self.nprob)(*[float(e) for e in eps])
        nb = ctypes.c_size_t(0)
        _check(lib.nfs_batch_workspace_size(ctypes.byref(params.to_c()), self.nprob, n_arr, nt_arr,
                                            ctypes.byref(nb)))
        self.nb = nb.value
        self.ws = torch.empty(self.nb, dtype=torch.uint8, device=self.x.device)
        h = ctypes.c_void_p()
        _check(lib.nfs_batch_solver_create(ctypes.byref(params.to_c()), self.nprob, n_arr, nt_arr, self.eps,
                                           self.x.data_ptr(), self.mu.data_ptr(), self.y.data_ptr(),
                                           self.nu.data_ptr(), None, self.ws.data_ptr(), self.nb, _stream(),
                                           ctypes.byref(h)))
        self.h = h

    def finish(self, check=True):
        lib = load_library()
        alpha = torch.empty(self.n, dtype=torch.float64, device=self.x.device)
        alpha_t = torch.empty(self.nt, dtype=torch.float64, device=self.x.device)
        res = (_Result * self.nprob)()
        rc = lib.nfs_solver_finish(self.h, alpha.data_ptr(), alpha_t.data_ptr(), res, _stream())
        if rc != NFS_OK and (check or rc != NFS_ENONPOS):
            _check(rc)
        return _results(res, alpha, alpha_t, self.offs_x, self.offs_y)


def batch_sinkhorn(params, xs, mus, ys, nus, eps, iters, tol=0.0, check=True):
    """Solve many problems at once (nfs_batch_solve; precision "auto" promotes
    the problems whose FP32 sums hit t <= 0 to FP64 grids); returns a list of
    SinkhornResult."""
    lib = load_library()
    nprob = len(xs)
    ns = [int(x.shape[0]) for x in xs]
    nts = [int(y.shape[0]) for y in ys]
    offs_x, offs_y = [0], [0]
    for a, b in zip(ns, nts):
        offs_x.append(offs_x[-1] + a)
        offs_y.append(offs_y[-1] + b)
    x = torch.cat([_pts(v, params.d, "x").reshape(-1, params.d) for v in xs]).contiguous()
    y = torch.cat([_pts(v, params.d, "y").reshape(-1, params.d) for v in ys]).contiguous()
    mu = torch.cat([_dev(v, "mu") for v in mus]).contiguous()
    nu = torch.cat([_dev(v, "nu") for v in nus]).contiguous()
    n_arr = (ctypes.c_int64 * nprob)(*ns)
    nt_arr = (ctypes.c_int64 * nprob)(*nts)
    eps_arr = (ctypes.c_double * nprob)(*[float(e) for e in eps])
    prm = params.to_c()
    nb = ctypes.c_size_t(0)
    _check(lib.nfs_batch_workspace_size(ctypes.byref(prm), nprob, n_arr, nt_arr, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
    alpha = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    alpha_t = torch.empty(y.shape[0], dtype=torch.float64, device=x.device)
    res = (_Result * nprob)()
    rc = lib.nfs_batch_solve(ctypes.byref(prm), nprob, n_arr, nt_arr, eps_arr, x.data_ptr(), mu.data_ptr(),
                             y.data_ptr(), nu.data_ptr(), int(iters), float(tol), alpha.data_ptr(),
                             alpha_t.data_ptr(), res, ws.data_ptr(), nb.value, _stream())
    if rc != NFS_OK and (check or rc != NFS_ENONPOS):
        _check(rc)
    return _results(res, alpha, alpha_t, offs_x, offs_y)


def sinkhorn_divergence(params, x, mu, y, nu, iters, tol=0.0, check=True):
    """Sinkhorn divergence s(P, Pt) - s(P, P)/2 - s(Pt, Pt)/2 (nfs_sinkhorn_divergence);
    returns (sd, [cost(P, Pt), cost(P, P), cost(Pt, Pt)], [n_nonpos of each])."""
    lib = load_library()
    x = _pts(x, params.d, "x")
    y = _pts(y, params.d, "y")
    _dev(mu, "mu")
    _dev(nu, "nu")
    n, nt = x.shape[0], y.shape[0]
    prm = params.to_c()
    nb = ctypes.c_size_t(0)
    _check(lib.nfs_divergence_workspace_size(ctypes.byref(prm), n, nt, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
    out = ctypes.c_double(0.0)
    res = (_Result * 3)()
    rc = lib.nfs_sinkhorn_divergence(ctypes.byref(prm), x.data_ptr(), n, mu.data_ptr(), y.data_ptr(), nt,
                                     nu.data_ptr(), int(iters), float(tol), ctypes.byref(out), res,
                                     ws.data_ptr(), nb.value, _stream())
    if rc != NFS_OK and (check or rc != NFS_ENONPOS):
        _check(rc)
    return out.value, [r.cost for r in res], [r.n_nonpos for r in res]


class SinkhornCost(torch.autograd.Function):
    """Sinkhorn cost s(x, mu; y, nu) with gradients w.r.t. x, mu, y and nu.

    Forward runs the NFFT-accelerated Sinkhorn solve; backward evaluates the
    envelope gradient with the adjoint fast summation.  With a fixed
    iteration count and FP32 or FP64 grids the solve runs on a solver handle
    that backward reuses (its plan, tables and scalings: no re-sort); with a
    tolerance or NFS_AUTO the one-shot solve runs and backward plans again,
    at the grid precision the solve ended with.
    """

    @staticmethod
    def forward(ctx, x, mu, y, nu, params, iters, tol=0.0):
        ctx.params = params
        ctx.solver = None
        if tol <= 0.0 and params.precision != "auto":
            s = Solver(params, x.detach(), mu.detach(), y.detach(), nu.detach())
            s.iterate(iters)
            res = s.finish()
            ctx.solver = s
            ctx.save_for_backward(x.detach(), mu.detach(), y.detach(), nu.detach())
        else:
            res = sinkhorn(params, x.detach(), mu.detach(), y.detach(), nu.detach(), iters, tol)
            ctx.save_for_backward(x.detach(), mu.detach(), y.detach(), nu.detach(), res.alpha, res.alpha_t)
            if params.precision == "auto":
                from dataclasses import replace
                ctx.params = replace(params, precision=res.precision_used or "fp64")
        return torch.tensor(res.cost, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, grad_out):
        need = ctx.needs_input_grad
        gx = gm = gy = gn = None
        if ctx.solver is not None:
            gx, gm, gy, gn = ctx.solver.grad(need[0], need[1], need[2], need[3])
            ctx.solver.close()
            ctx.solver = None
        else:
            x, mu, y, nu, a, at = ctx.saved_tensors
            if need[0] or need[1]:
                gx, gm = sinkhorn_grad(ctx.params, x, mu, y, nu, a, at, want_x=need[0], want_mu=need[1])
            if need[2] or need[3]:
                gy, gn = sinkhorn_grad_targets(ctx.params, x, mu, y, nu, a, at, want_y=need[2], want_nu=need[3])
        g = grad_out.to(torch.float64)
        scale = lambda t: t * g if t is not None else None
        return scale(gx), scale(gm), scale(gy), scale(gn), None, None, None
