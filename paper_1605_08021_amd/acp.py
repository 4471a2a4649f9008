"""Python binding of libacp.so (argument marshalling only).

Every numerical step runs in the HIP library; this module converts torch
tensors (device memory, column-major views) and numpy arrays (host memory) to
the plain pointers of the C ABI declared in include/acp.h, and turns status
codes into exceptions.  There is no fallback: if the library is missing or the
device is not a GPU, calls fail loudly.

Column-major convention: a matrix with m rows and n columns is a torch tensor
of shape (m, n) and strides (1, m).  ``colmajor(t)`` produces one.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libacp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "acp.h")

ACP_OK, ACP_EINVAL, ACP_ENOMEM, ACP_EDEVICE, ACP_ENOCONV, ACP_ENOTSPD, ACP_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "ACP_OK", -1: "ACP_EINVAL", -2: "ACP_ENOMEM", -3: "ACP_EDEVICE",
                -4: "ACP_ENOCONV", -5: "ACP_ENOTSPD", -6: "ACP_ESTATE"}
PREC_FP64, PREC_FP32_REFINE, PREC_BF16_PROJ = 0, 1, 2
SOLVER_CG, SOLVER_MINRES, SOLVER_CG_SINGLE = 0, 1, 2
NODES_CHEBYSHEV, NODES_OCCUPIED = 0, 1


class ACPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class AcpGrid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 2), ("h", C.c_double), ("kappa", C.c_double),
                ("eps0", C.c_double), ("occ", C.c_double)]


class AcpOpts(C.Structure):
    _fields_ = [("n_cheb", C.c_int), ("n_mu", C.c_int), ("sketch_r", C.c_int),
                ("isdf_tol", C.c_double), ("node_mode", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("solver", C.c_int), ("precision", C.c_int),
                ("dyson_max_iter", C.c_int), ("dyson_tol", C.c_double),
                ("inner_tol", C.c_double), ("use_learned_precond", C.c_int), ("reorthonormalize", C.c_int), ("deterministic", C.c_int)]


class AcpStats(C.Structure):
    _fields_ = [("systems_solved", C.c_int64), ("system_iterations", C.c_int64),
                ("tile_iterations", C.c_int64), ("iters_min", C.c_int), ("iters_max", C.c_int),
                ("max_rel_residual", C.c_double), ("dyson_iters", C.c_int),
                ("refinements", C.c_int), ("ms_isdf", C.c_double), ("ms_rhs", C.c_double),
                ("ms_solve", C.c_double), ("ms_w", C.c_double), ("ms_dyson_small", C.c_double),
                ("ms_dynmat", C.c_double), ("ms_solve_kernel", C.c_double),
                ("solve_kernel_launches", C.c_int64), ("d_asymmetry", C.c_double),
                ("krylov_bytes", C.c_double), ("krylov_flops", C.c_double),
                ("krylov_group", C.c_int), ("n_mu", C.c_int), ("vector_bytes", C.c_double),
                ("ms_vectors", C.c_double), ("ms_residual", C.c_double)]


class AcpEigOpts(C.Structure):
    _fields_ = [("n_want", C.c_int), ("n_guard", C.c_int), ("degree", C.c_int), ("max_pass", C.c_int),
                ("tol", C.c_double), ("seed", C.c_ulonglong)]


class AcpScfOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tol", C.c_double), ("beta", C.c_double), ("history", C.c_int),
                ("kerker_q0", C.c_double), ("eig", AcpEigOpts)]


class AcpBatchInfo(C.Structure):
    _fields_ = [("n_systems", C.c_int), ("n_tiles", C.c_int), ("grid", C.c_int), ("order", C.c_int),
                ("tuned", C.c_int), ("graph_replays", C.c_longlong), ("ms_last", C.c_double),
                ("tune_ms", C.c_double * 6)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libacp.so (torch is imported first so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.c_void_p
    I = C.c_int
    sig = {
        "acp_default_opts": (None, [C.POINTER(AcpOpts)]),
        "acp_version": (C.c_char_p, []),
        "acp_setup": (I, [C.POINTER(P), C.POINTER(AcpGrid), C.POINTER(AcpOpts), P, P, I, P, P]),
        "acp_set_opts": (I, [P, C.POINTER(AcpOpts)]),
        "acp_apply_h": (I, [P, P, I, P, P]),
        "acp_apply_vc": (I, [P, I, P, P]),
        "acp_apply_vc_inv": (I, [P, I, P, P]),
        "acp_sternheimer": (I, [P, P, I, P, P, P]),
        "acp_compress": (I, [P, P, I, P, P, P]),
        "acp_compress_get": (I, [P, I, P, P]),
        "acp_apply_chi0": (I, [P, P, I, P]),
        "acp_dyson": (I, [P, P, I, P, P, P, P, P]),
        "acp_dynmat": (I, [P, P, P, I, P, P, P, P]),
        "acp_residual": (I, [P, P, I, P, P, P]),
        "acp_residual_noalloc": (I, [P, P, I, P, P, P]),
        "acp_dfpt": (I, [P, P, I, I, C.c_double, I, C.c_double, P, P, P]),
        "acp_precond_n_params": (I, [I]),
        "acp_precond_init": (I, [P, C.c_ulonglong]),
        "acp_precond_set": (I, [P, P, I]),
        "acp_precond_get": (I, [P, P, I]),
        "acp_precond_forward": (I, [P, P, I, P, P]),
        "acp_precond_apply": (I, [P, P, I, P, P]),
        "acp_precond_train_step": (I, [P, P, I, P, P, C.c_double, P, P]),
        "acp_precond_trajectory": (I, [P, P, I, P, P, I, P, P]),
        "acp_batch_create": (I, [C.POINTER(P), P, I, I]),
        "acp_batch_compress": (I, [P, P, P, P, P]),
        "acp_batch_info": (I, [P, C.POINTER(AcpBatchInfo)]),
        "acp_batch_last_error": (C.c_char_p, [P]),
        "acp_batch_destroy": (None, [P]),
        "acp_get_stats": (I, [P, C.POINTER(AcpStats)]),
        "acp_syev": (I, [I, P, I, P, P, I, P]),
        "acp_gesv": (I, [I, I, P, I, P, I, P]),
        "acp_scf": (I, [C.POINTER(AcpGrid), P, P, I, C.POINTER(AcpScfOpts), P, P, P, P, P, P, P]),
        "acp_lowest_eigenpairs": (I, [C.POINTER(AcpGrid), P, C.POINTER(AcpEigOpts), P, P, P, P, P, P]),
        "acp_phonon_dos": (I, [P, I, I, C.c_double, P, I, P, P]),
        "acp_reset_stats": (None, [P]),
        "acp_last_error": (C.c_char_p, [P]),
        "acp_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_symbols(path: str = HEADER) -> list:
    """Entry points declared in include/acp.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(acp_[a-z0-9_]+)\s*\(", text)))


def colmajor(t):
    """Same values, column-major storage (strides (1, m)) for a 2-D tensor."""
    if t.dim() == 1:
        return t.contiguous()
    if t.stride(0) == 1 and t.stride(1) == t.shape[0]:
        return t
    return t.t().contiguous().t()


def _dptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ACPError(ACP_EINVAL, "device argument must be a torch tensor on a GPU")
    if t.dtype != torch.float64:
        raise ACPError(ACP_EINVAL, "device argument must be float64")
    return t.data_ptr()


def _hostd(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _hptr(a: np.ndarray) -> int:
    return a.ctypes.data


def phonon_dos(omega2, n_modes: int, sigma: float, w, stream=None):
    """The smeared phonon spectrum on the frequencies w (acp_phonon_dos): omega2
    and w host arrays or device tensors; the result is a device tensor."""
    import torch
    lib = load_library()
    dev = torch.device("cuda", torch.cuda.current_device())
    om = torch.as_tensor(omega2, dtype=torch.float64).to(dev).contiguous()
    wd = torch.as_tensor(w, dtype=torch.float64).to(dev).contiguous()
    out = torch.empty_like(wd)
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib.acp_phonon_dos(_dptr(om), om.numel(), n_modes, float(sigma), _dptr(wd), wd.numel(), _dptr(out),
                            C.c_void_p(stream.cuda_stream))
    if st != ACP_OK:
        raise ACPError(st, lib.acp_last_error(None).decode())
    return out


def syev(A, want_vectors: bool = True, stream=None):
    """Eigenvalues (numpy, ascending) and eigenvectors (device, column-major) of
    the symmetric device matrix A (not modified: a copy is passed)."""
    import torch
    lib = load_library()
    A = colmajor(A).clone()
    A = colmajor(A)
    n = A.shape[0]
    w = np.zeros(n)
    V = None
    if want_vectors:
        V = torch.empty((n, n), dtype=torch.float64, device=A.device).t()
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib.acp_syev(n, _dptr(A), n, _hptr(w), None if V is None else _dptr(V), n,
                      C.c_void_p(stream.cuda_stream))
    if st != ACP_OK:
        raise ACPError(st, "acp_syev")
    return w, V


def gesv(A, B, stream=None):
    """X = A^{-1} B (device, column-major); A and B are copied first."""
    import torch
    lib = load_library()
    A = colmajor(colmajor(A).clone())
    X = colmajor(colmajor(B).clone())
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib.acp_gesv(A.shape[0], X.shape[1], _dptr(A), A.shape[0], _dptr(X), X.shape[0],
                      C.c_void_p(stream.cuda_stream))
    if st != ACP_OK:
        raise ACPError(st, "acp_gesv")
    return X


def _grid_struct(grid: dict) -> AcpGrid:
    g = AcpGrid()
    g.dim = int(grid["dim"])
    n = list(grid["n"]) + [1]
    g.n[0], g.n[1] = int(n[0]), int(n[1])
    g.h = float(grid["h"])
    g.kappa, g.eps0, g.occ = (float(grid.get("kappa", 1.0)), float(grid.get("eps0", 1.0)),
                              float(grid.get("occ", 2.0)))
    return g


def lowest_eigenpairs(grid: dict, veff, n_want: int, n_guard: int = 0, degree: int = 0,
                      max_pass: int = 0, tol: float = 0.0, seed: int = 1, stream=None):
    """acp_lowest_eigenpairs: (psi dev N_g x n_want, eps numpy n_want, next Ritz value,
    passes, largest residual)."""
    import torch
    lib = load_library()
    veff = veff.contiguous()
    g = _grid_struct(grid)
    o = AcpEigOpts(n_want, n_guard, degree, max_pass, tol, seed)
    psi = torch.empty((n_want, veff.shape[0]), dtype=torch.float64, device=veff.device).t()
    lam = np.zeros(n_want)
    nxt = C.c_double(0.0)
    passes = C.c_int(0)
    res = C.c_double(0.0)
    if stream is None:
        stream = torch.cuda.current_stream()
    st = lib.acp_lowest_eigenpairs(C.byref(g), _dptr(veff), C.byref(o), _dptr(psi), _hptr(lam),
                                   C.byref(nxt), C.byref(passes), C.byref(res),
                                   C.c_void_p(stream.cuda_stream))
    if st != ACP_OK:
        raise ACPError(st, lib.acp_last_error(None).decode())
    return psi, lam, nxt.value, passes.value, res.value


def scf(grid: dict, m, n_e: int, rho0=None, max_iter: int = 0, tol: float = 0.0, beta: float = 0.0,
        history: int = 0, kerker_q0: float = 0.0, eig_tol: float = 0.0, seed: int = 1, stream=None):
    """acp_scf: (psi dev N_g x n_e, eps numpy n_e + 1, veff dev, rho dev, iterations, residual)."""
    import torch
    lib = load_library()
    m = m.contiguous()
    g = _grid_struct(grid)
    o = AcpScfOpts(max_iter, tol, beta, history, kerker_q0, AcpEigOpts(n_e, 0, 0, 0, eig_tol, seed))
    ng = m.shape[0]
    psi = torch.empty((n_e, ng), dtype=torch.float64, device=m.device).t()
    eps = np.zeros(n_e + 1)
    veff = torch.empty(ng, dtype=torch.float64, device=m.device)
    rho = torch.empty(ng, dtype=torch.float64, device=m.device)
    it = C.c_int(0)
    res = C.c_double(0.0)
    if stream is None:
        stream = torch.cuda.current_stream()
    r0 = None if rho0 is None else rho0.contiguous()
    st = lib.acp_scf(C.byref(g), _dptr(m), None if r0 is None else _dptr(r0), n_e, C.byref(o), _dptr(psi),
                     _hptr(eps), _dptr(veff), _dptr(rho), C.byref(it), C.byref(res),
                     C.c_void_p(stream.cuda_stream))
    if st != ACP_OK:
        raise ACPError(st, lib.acp_last_error(None).decode())
    return psi, eps, veff, rho, it.value, res.value


class Context:
    """One acp_ctx: the occupied space of H[V_eff] on a grid, on one stream."""

    def __init__(self, grid: dict, opts: dict, psi, eps, veff, stream=None):
        import torch
        self.lib = load_library()
        self._ctx = C.c_void_p()
        g = AcpGrid()
        g.dim = int(grid["dim"])
        n = list(grid["n"]) + [1]
        g.n[0], g.n[1] = int(n[0]), int(n[1])
        g.h, g.kappa, g.eps0, g.occ = (float(grid["h"]), float(grid["kappa"]),
                                       float(grid["eps0"]), float(grid["occ"]))
        self.grid = g
        self.opts = self.make_opts(**opts)
        self.psi = colmajor(psi)
        self.veff = veff.contiguous()
        self.eps = _hostd(eps)
        self.n_g = self.psi.shape[0]
        self.n_e = self.psi.shape[1]
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        st = self.lib.acp_setup(C.byref(self._ctx), C.byref(g), C.byref(self.opts),
                                _dptr(self.psi), _hptr(self.eps), self.n_e, _dptr(self.veff),
                                C.c_void_p(stream.cuda_stream))
        if st != ACP_OK:
            msg = self.lib.acp_last_error(self._ctx).decode() if self._ctx else ""
            self.lib.acp_destroy(self._ctx)
            self._ctx = C.c_void_p()
            raise ACPError(st, msg)

    # -- helpers --------------------------------------------------------------
    def make_opts(self, **kw) -> AcpOpts:
        o = AcpOpts()
        self.lib.acp_default_opts(C.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        return o

    def _check(self, st: int, allow=(ACP_OK,)):
        if st not in allow:
            raise ACPError(st, self.lib.acp_last_error(self._ctx).decode())
        return st

    def _empty(self, m, n):
        import torch
        return torch.empty((n, m), dtype=torch.float64, device=self.psi.device).t()

    def set_opts(self, **kw):
        self.opts = self.make_opts(**{**{f: getattr(self.opts, f) for f, _ in AcpOpts._fields_}, **kw})
        self._check(self.lib.acp_set_opts(self._ctx, C.byref(self.opts)))

    # -- entry points -----------------------------------------------------------
    def apply_h(self, X, shifts: Optional[Sequence[float]] = None):
        X = colmajor(X)
        Y = self._empty(*X.shape)
        sh = None if shifts is None else _hostd(shifts)
        self._check(self.lib.acp_apply_h(self._ctx, None if sh is None else _hptr(sh), X.shape[1],
                                         _dptr(X), _dptr(Y)))
        return Y

    def apply_vc(self, X):
        X = colmajor(X)
        Y = self._empty(*X.shape)
        self._check(self.lib.acp_apply_vc(self._ctx, X.shape[1], _dptr(X), _dptr(Y)))
        return Y

    def apply_vc_inv(self, X):
        X = colmajor(X)
        Y = self._empty(*X.shape)
        self._check(self.lib.acp_apply_vc_inv(self._ctx, X.shape[1], _dptr(X), _dptr(Y)))
        return Y

    def sternheimer(self, shifts, B, allow_noconv=False):
        B = colmajor(B)
        n = B.shape[1]
        sh = _hostd(shifts)
        assert sh.shape == (n,)
        X = self._empty(*B.shape)
        iters = np.zeros(n, dtype=np.int32)
        allow = (ACP_OK, ACP_ENOCONV) if allow_noconv else (ACP_OK,)
        st = self._check(self.lib.acp_sternheimer(self._ctx, _hptr(sh), n, _dptr(B), _dptr(X),
                                                  iters.ctypes.data), allow)
        return X, iters, st

    def compress(self, G, omega, sel_in=None):
        G = colmajor(G)
        omega = colmajor(omega)
        n_mu = self.opts.n_mu
        sel = np.zeros(n_mu, dtype=np.int32)
        si = None
        if sel_in is not None:
            si = np.ascontiguousarray(np.asarray(sel_in, dtype=np.int32))
        self._check(self.lib.acp_compress(self._ctx, _dptr(G), G.shape[1], _dptr(omega),
                                          None if si is None else si.ctypes.data, sel.ctypes.data))
        return sel[: self.stats()["n_mu"]]

    def compress_get(self, what: str):
        idx = {"xi": 0, "rhs": 1, "w": 2, "z": 3}[what]
        n_mu = self.stats()["n_mu"]
        nc = self.n_shifts()
        cols = n_mu * nc if what == "z" else n_mu
        out = self._empty(self.n_g, cols)
        shifts = np.zeros(max(nc, 1))
        self._check(self.lib.acp_compress_get(self._ctx, idx, _dptr(out), _hptr(shifts)))
        return out

    def shifts(self) -> np.ndarray:
        nc = self.n_shifts()
        out = np.zeros(nc)
        self._check(self.lib.acp_compress_get(self._ctx, 0, None, _hptr(out)), (ACP_OK,))
        return out

    def n_shifts(self) -> int:
        if self.opts.node_mode == NODES_OCCUPIED:
            return len(np.unique(self.eps))
        lo, hi = self.eps[0], self.eps[-1]
        if self.opts.n_cheb == 1 or hi - lo <= 1e-14 * max(1.0, abs(lo)):
            return 1
        return self.opts.n_cheb

    def apply_chi0(self, X):
        X = colmajor(X)
        Y = self._empty(*X.shape)
        self._check(self.lib.acp_apply_chi0(self._ctx, _dptr(X), X.shape[1], _dptr(Y)))
        return Y

    def dyson(self, G, omega, sel_hist_in=None):
        G = colmajor(G)
        omega = colmajor(omega)
        kmax, n_mu = self.opts.dyson_max_iter, self.opts.n_mu
        hist = np.zeros((kmax, n_mu), dtype=np.int32)
        hin = None
        if sel_hist_in is not None:
            hin = np.ascontiguousarray(np.asarray(sel_hist_in, dtype=np.int32).reshape(kmax, n_mu))
        U = self._empty(*G.shape)
        iters = C.c_int(0)
        self._check(self.lib.acp_dyson(self._ctx, _dptr(G), G.shape[1], _dptr(omega),
                                       None if hin is None else hin.ctypes.data,
                                       hist.ctypes.data, _dptr(U), C.byref(iters)))
        return U, iters.value, hist[: iters.value]

    def dynmat(self, G, U=None, K_local=None, mass=None):
        G = colmajor(G)
        n_p = G.shape[1]
        K = None if K_local is None else np.asfortranarray(np.asarray(K_local, dtype=np.float64))
        m = None if mass is None else _hostd(mass)
        D = np.zeros((n_p, n_p), order="F")
        w2 = np.zeros(n_p)
        Up = None if U is None else _dptr(colmajor(U))
        self._check(self.lib.acp_dynmat(self._ctx, _dptr(G), Up, n_p,
                                        None if K is None else K.ctypes.data,
                                        None if m is None else _hptr(m), D.ctypes.data,
                                        _hptr(w2)))
        return D, w2

    def residual(self, shifts, B, X):
        B, X = colmajor(B), colmajor(X)
        sh = _hostd(shifts)
        R = self._empty(*B.shape)
        self._check(self.lib.acp_residual(self._ctx, _hptr(sh), B.shape[1], _dptr(B), _dptr(X),
                                          _dptr(R)))
        return R

    def dfpt(self, G, max_iter=60, tol=1e-10, history=8, beta=0.5):
        """acp_dfpt: (U = chi G on the device, chi0 applications, last relative change)."""
        G = colmajor(G)
        U = self._empty(*G.shape)
        it = C.c_int(0)
        ch = C.c_double(0.0)
        self._check(self.lib.acp_dfpt(self._ctx, _dptr(G), G.shape[1], int(max_iter), float(tol), int(history),
                                      float(beta), _dptr(U), C.byref(it), C.byref(ch)))
        return U, it.value, ch.value

    def residual_noalloc(self, shifts, B, X, R=None):
        """acp_residual_noalloc into R (allocated here when None: the library
        call itself allocates nothing)."""
        B, X = colmajor(B), colmajor(X)
        sh = _hostd(shifts)
        if R is None:
            R = self._empty(*B.shape)
        self._check(self.lib.acp_residual_noalloc(self._ctx, _hptr(sh), B.shape[1], _dptr(B),
                                                  _dptr(X), _dptr(R)))
        return R

    # -- learned preconditioner (marshalling only) ----------------------------
    def precond_n_params(self) -> int:
        return self.lib.acp_precond_n_params(self.grid.dim)

    def precond_init(self, seed: int):
        self._check(self.lib.acp_precond_init(self._ctx, C.c_ulonglong(seed)))

    def precond_set(self, theta):
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        self._check(self.lib.acp_precond_set(self._ctx, t.ctypes.data, t.size))

    def precond_get(self) -> np.ndarray:
        t = np.zeros(self.precond_n_params(), dtype=np.float32)
        self._check(self.lib.acp_precond_get(self._ctx, t.ctypes.data, t.size))
        return t

    def precond_forward(self, shifts, R):
        import torch
        R = colmajor(R)
        sh = _hostd(shifts)
        out = torch.empty((R.shape[1], R.shape[0]), dtype=torch.float32, device=R.device)
        self._check(self.lib.acp_precond_forward(self._ctx, _hptr(sh), R.shape[1], _dptr(R),
                                                 out.data_ptr()))
        return out

    def precond_apply(self, shifts, R):
        R = colmajor(R)
        sh = _hostd(shifts)
        D = self._empty(*R.shape)
        self._check(self.lib.acp_precond_apply(self._ctx, _hptr(sh), R.shape[1], _dptr(R), _dptr(D)))
        return D

    def precond_trajectory(self, shifts, B, Xstar, steps: int):
        """(R, E): residuals and errors along `steps` steps of steepest descent
        with the current network (N_g x steps n each, step-major)."""
        B, Xstar = colmajor(B), colmajor(Xstar)
        sh = _hostd(shifts)
        n = B.shape[1]
        R = self._empty(B.shape[0], steps * n)
        E = self._empty(B.shape[0], steps * n)
        self._check(self.lib.acp_precond_trajectory(self._ctx, _hptr(sh), n, _dptr(B), _dptr(Xstar), steps,
                                                    _dptr(R), _dptr(E)))
        return R, E

    def precond_train_step(self, shifts, R, E, lr: float, want_grad: bool = False):
        R, E = colmajor(R), colmajor(E)
        sh = _hostd(shifts)
        loss = C.c_double(0.0)
        g = np.zeros(self.precond_n_params(), dtype=np.float32) if want_grad else None
        self._check(self.lib.acp_precond_train_step(self._ctx, _hptr(sh), R.shape[1], _dptr(R),
                                                    _dptr(E), float(lr), C.byref(loss),
                                                    None if g is None else g.ctypes.data))
        return (loss.value, g) if want_grad else loss.value

    def stats(self) -> dict:
        s = AcpStats()
        self._check(self.lib.acp_get_stats(self._ctx, C.byref(s)))
        return {f: getattr(s, f) for f, _ in AcpStats._fields_}

    def reset_stats(self):
        self.lib.acp_reset_stats(self._ctx)

    def close(self):
        if self._ctx:
            self.lib.acp_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """acp_batch: the shifted solves of several contexts in one persistent launch."""

    def __init__(self, contexts, use_graph: bool = False):
        self.lib = load_library()
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c._ctx.value for c in self.contexts])
        self._b = C.c_void_p()
        st = self.lib.acp_batch_create(C.byref(self._b), arr, len(self.contexts), int(use_graph))
        if st != ACP_OK:
            msg = self.lib.acp_batch_last_error(self._b).decode() if self._b else ""
            self.lib.acp_batch_destroy(self._b)
            self._b = C.c_void_p()
            raise ACPError(st, msg)

    def compress(self, Gs, omegas, sel_in=None):
        Gs = [colmajor(g) for g in Gs]
        oms = [colmajor(o) for o in omegas]
        n = len(self.contexts)
        gp = (C.c_void_p * n)(*[_dptr(g) for g in Gs])
        op = (C.c_void_p * n)(*[_dptr(o) for o in oms])
        npv = (C.c_int * n)(*[g.shape[1] for g in Gs])
        keep = []
        sp = None
        if sel_in is not None:
            ptrs = []
            for sel in sel_in:
                if sel is None:
                    ptrs.append(None)
                else:
                    a = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
                    keep.append(a)
                    ptrs.append(a.ctypes.data)
            sp = (C.c_void_p * n)(*ptrs)
        st = self.lib.acp_batch_compress(self._b, gp, npv, op, sp)
        if st != ACP_OK:
            raise ACPError(st, self.lib.acp_batch_last_error(self._b).decode())

    def info(self) -> dict:
        i = AcpBatchInfo()
        st = self.lib.acp_batch_info(self._b, C.byref(i))
        if st != ACP_OK:
            raise ACPError(st, "acp_batch_info")
        d = {f: getattr(i, f) for f, _ in AcpBatchInfo._fields_ if f != "tune_ms"}
        d["tune_ms"] = list(i.tune_ms)
        return d

    def close(self):
        if self._b:
            self.lib.acp_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
