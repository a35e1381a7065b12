"""ctypes binding of the gfx950 block CG library (include/bcg.h).

Argument marshalling only: every step of the operator, the solvers and the
link force runs in the HIP kernels of libbcg.so.  Vectors are complex128 torch
tensors of shape [N, V/2, 3] on the GPU; links are complex128 [4, V, 3, 3]
tensors (GPU or CPU) or numpy arrays.  There is no CPU fallback: without the
built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcg.so")

OK = 0
ERR_ARG = -1
ERR_HIP = -2
ERR_NOMEM = -3
ERR_NOT_CONVERGED = -4
ERR_BREAKDOWN = -5
ERR_STATE = -6
STATUS_NAMES = {OK: "ok", ERR_ARG: "bad argument", ERR_HIP: "HIP error", ERR_NOMEM: "out of memory",
                ERR_NOT_CONVERGED: "not converged", ERR_BREAKDOWN: "breakdown",
                ERR_STATE: "bad state"}

PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fix16": 4}
OPTIONS = {"hop_tr": 0, "hop_tpb": 1, "hop_pipeline": 2, "pass_cpt": 3, "fuse_gram": 4, "hop_kernel": 5, "gram_kernel": 6,
           "small_threads": 7, "site_order": 8,
           "pass_kernel": 9, "graph": 10, "hop_sched": 11}
KERNELS = ["hop_oe", "hop_eo", "gram", "reduce", "small", "pass_a", "pass_b", "cg_vec",
           "convert", "other"]
MAX_RHS = 64


class BcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class NotConverged(BcgError):
    pass


class Breakdown(BcgError):
    pass


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("status", ctypes.c_int), ("restarts", ctypes.c_int),
                ("seconds", ctypes.c_double), ("max_true_rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.POINTER(ctypes.c_double))]


_LIB = None
MONITOR_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double)


def load_library():
    """Load libbcg.so (built in-tree by paper_1710_09745_amd/build.py)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    sig = {
        "bcg_create": ([ctypes.POINTER(P), ctypes.POINTER(I), I, P], I),
        "bcg_destroy": ([P], I),
        "bcg_load_links": ([P, P, P, I], I),
        "bcg_set_mass": ([P, D], I),
        "bcg_set_solver": ([P, D, I, I, D], I),
        "bcg_apply": ([P, P, P, I], I),
        "bcg_hop": ([P, I, P, P, I], I),
        "bcg_apply_prec": ([P, I, P, P, I], I),
        "bcg_apply_noalloc": ([P, P, P, I], I),
        "bcg_solve": ([P, P, P, I, I, ctypes.POINTER(Stats)], I),
        "bcg_solve_cg": ([P, P, P, I, ctypes.POINTER(Stats)], I),
        "bcg_solve_pseudo": ([P, P, P, I, ctypes.POINTER(Stats)], I),
        "bcg_solve_sstep": ([P, P, P, I, I, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Stats)], I),
        "bcg_link_force": ([P, P, P, I, P, P], I),
        "bcg_set_profiling": ([P, U], I),
        "bcg_set_option": ([P, I, I], I),
        "bcg_set_stability": ([P, I, I, I], I),
        "bcg_set_monitor": ([P, MONITOR_FN, P], I),
        "bcg_profile_reset": ([P], I),
        "bcg_kernel_time": ([P, I, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(D)], I),
        "bcg_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _LIB = lib
    return lib


def _vec(t, name, nrhs=None, vh=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() != 3 or t.shape[2] != 3 or (vh is not None and t.shape[1] != vh):
        raise ValueError(f"{name} must have shape [N, V/2={vh}, 3], got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """One lattice, its links, mass and solver settings (a bcg_ctx)."""

    def __init__(self, dims, improved=True, device=None, stream=None):
        self.lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.V = 1
        for d in self.dims:
            self.V *= d
        self.Vh = self.V // 2
        self.improved = bool(improved)
        self.device = torch.device(device if device is not None else "cuda")
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        d4 = (ctypes.c_int * 4)(*self.dims)
        with torch.cuda.device(self.device):
            rc = self.lib.bcg_create(ctypes.byref(h), d4, int(self.improved),
                                     ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise BcgError(rc, self.lib.bcg_last_error(None).decode())
        self.h = h
        self._links = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.bcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc == OK:
            return
        msg = self.lib.bcg_last_error(self.h).decode()
        if rc == ERR_NOT_CONVERGED:
            raise NotConverged(rc, msg)
        if rc == ERR_BREAKDOWN:
            raise Breakdown(rc, msg)
        raise BcgError(rc, msg)

    # -- setup -------------------------------------------------------------------------------
    def load_links(self, fat, lng=None):
        """Links [4, V, 3, 3] complex128 (torch CPU/GPU tensor or numpy array)."""
        def prep(u):
            if u is None:
                return None, None
            if not isinstance(u, torch.Tensor):
                u = torch.from_numpy(u)
            if u.dtype != torch.complex128 or tuple(u.shape) != (4, self.V, 3, 3):
                raise ValueError(f"links must be complex128 [4, {self.V}, 3, 3]")
            u = u.contiguous()
            return u, u.is_cuda
        f, fd = prep(fat)
        l, ld = prep(lng)
        if l is not None and fd != ld:
            l = l.to(f.device)
        on_dev = 1 if fd else 0
        rc = self.lib.bcg_load_links(self.h, ctypes.c_void_p(f.data_ptr()),
                                     ctypes.c_void_p(l.data_ptr()) if l is not None else None, on_dev)
        self._check(rc)
        self._links = (f, l)

    def set_mass(self, m):
        self._check(self.lib.bcg_set_mass(self.h, float(m)))
        self.mass = float(m)

    def set_solver(self, tol=1e-10, max_iter=100000, prec="fp64", ru_delta=0.1):
        self._check(self.lib.bcg_set_solver(self.h, float(tol), int(max_iter), PREC[prec],
                                            float(ru_delta)))

    def set_monitor(self, fn):
        """fn(iters, reliable_updates, max_rel_res) on every state read of a solve; None = off."""
        if fn is None:
            self._monitor = None
            self._check(self.lib.bcg_set_monitor(self.h, MONITOR_FN(), None))
            return
        self._monitor = MONITOR_FN(lambda user, it, ru, r: fn(it, ru, r))   # kept alive here
        self._check(self.lib.bcg_set_monitor(self.h, self._monitor, None))

    def set_stability(self, ru_window=100, stall_limit=3, qr_passes=1):
        """Adaptive reliable updates, stagnation exit and CholQR2 (bcg_set_stability)."""
        self._check(self.lib.bcg_set_stability(self.h, int(ru_window), int(stall_limit), int(qr_passes)))

    # -- operator ----------------------------------------------------------------------------
    def apply(self, x, out=None):
        """A x with A = 4 m^2 - D_eo D_oe (FP64), x [N, V/2, 3]."""
        _vec(x, "x", vh=self.Vh)
        out = torch.empty_like(x) if out is None else _vec(out, "out", vh=self.Vh)
        self._check(self.lib.bcg_apply(self.h, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), x.shape[0]))
        return out

    def apply_noalloc(self, x, out):
        """A x without any device allocation in the library (bcg_apply_noalloc); out given."""
        _vec(x, "x", vh=self.Vh)
        _vec(out, "out", vh=self.Vh)
        self._check(self.lib.bcg_apply_noalloc(self.h, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), x.shape[0]))
        return out

    def apply_prec(self, prec, x, out=None):
        """A x as the iteration evaluates it in storage precision prec (bcg_apply_prec)."""
        _vec(x, "x", vh=self.Vh)
        out = torch.empty_like(x) if out is None else _vec(out, "out", vh=self.Vh)
        self._check(self.lib.bcg_apply_prec(self.h, PREC[prec], ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), x.shape[0]))
        return out

    def hop(self, out_parity, x, out=None):
        """D_{p,1-p} x (p = out_parity), FP64."""
        _vec(x, "x", vh=self.Vh)
        out = torch.empty_like(x) if out is None else _vec(out, "out", vh=self.Vh)
        self._check(self.lib.bcg_hop(self.h, int(out_parity), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), x.shape[0]))
        return out

    # -- solvers -----------------------------------------------------------------------------
    def _solve(self, fn, B, X, *extra):
        n = B.shape[0]
        tr = (ctypes.c_double * n)()
        st = Stats()
        st.true_rel_res = ctypes.cast(tr, ctypes.POINTER(ctypes.c_double))
        rc = fn(self.h, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()), n, *extra,
                ctypes.byref(st))
        info = dict(iters=st.iters, reliable_updates=st.reliable_updates, status=st.status,
                    restarts=st.restarts, seconds=st.seconds, max_true_rel_res=st.max_true_rel_res,
                    true_rel_res=[tr[i] for i in range(n)])
        return rc, info

    def solve(self, B, X0=None, raise_on_error=True):
        """blockCGrQ: X = A^{-1} B for all N columns at once.  Returns (X, info)."""
        _vec(B, "B", vh=self.Vh)
        if X0 is not None:
            X = _vec(X0, "X0", vh=self.Vh).clone()
        else:
            X = torch.empty_like(B)
        rc, info = self._solve(self.lib.bcg_solve, B, X, 1 if X0 is not None else 0)
        if raise_on_error:
            self._check(rc)
        info["rc"] = rc
        return X, info

    def solve_cg(self, B, raise_on_error=True):
        """N independent CG solves, one after the other (the baseline).  Returns (X, info)."""
        _vec(B, "B", vh=self.Vh)
        X = torch.empty_like(B)
        rc, info = self._solve(self.lib.bcg_solve_cg, B, X)
        if raise_on_error:
            self._check(rc)
        info["rc"] = rc
        return X, info

    def solve_pseudo(self, B, raise_on_error=True):
        """Pseudo-block CG: N independent CG recurrences sharing each stencil
        application.  Returns (X, info)."""
        _vec(B, "B", vh=self.Vh)
        X = torch.empty_like(B)
        rc, info = self._solve(self.lib.bcg_solve_pseudo, B, X)
        if raise_on_error:
            self._check(rc)
        info["rc"] = rc
        return X, info

    def solve_sstep(self, B, s, lmin=0.0, lmax=0.0, raise_on_error=True):
        """s-step block CG with s block directions per outer iteration (s * N <= 64)
        and a Chebyshev basis on [lmin, lmax] (<= 0: 4 m^2, and 1.1 times a
        power-iteration estimate), in the storage precision set by set_solver (fp64 or
        fp32; fp32 adds reliable updates).  Returns (X, info); info["iters"] counts
        s-steps."""
        _vec(B, "B", vh=self.Vh)
        X = torch.empty_like(B)
        rc, info = self._solve(self.lib.bcg_solve_sstep, B, X, int(s), float(lmin), float(lmax))
        if raise_on_error:
            self._check(rc)
        info["rc"] = rc
        return X, info

    def link_force(self, X, Lam):
        """Gradients w.r.t. (fat, long) for dL = -Re sum_i Lam_i^H dA X_i."""
        _vec(X, "X", vh=self.Vh)
        _vec(Lam, "Lam", vh=self.Vh)
        if X.shape != Lam.shape:
            raise ValueError("X and Lam must have the same shape")
        gf = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device=X.device)
        gl = torch.empty_like(gf) if self.improved else None
        self._check(self.lib.bcg_link_force(self.h, ctypes.c_void_p(X.data_ptr()),
                                            ctypes.c_void_p(Lam.data_ptr()), X.shape[0],
                                            ctypes.c_void_p(gf.data_ptr()),
                                            ctypes.c_void_p(gl.data_ptr()) if gl is not None else None))
        return gf, gl

    # -- tuning ------------------------------------------------------------------------------
    def set_option(self, name, value):
        """Launch-shape / kernel-variant option (see OPTIONS); 0 restores the default."""
        if name not in OPTIONS:
            raise ValueError(f"unknown option {name!r}; known: {sorted(OPTIONS)}")
        self._check(self.lib.bcg_set_option(self.h, OPTIONS[name], int(value)))

    # -- profiling ---------------------------------------------------------------------------
    def set_profiling(self, kernels):
        mask = 0
        for k in kernels:
            mask |= 1 << KERNELS.index(k)
        self._check(self.lib.bcg_set_profiling(self.h, mask))

    def profile_reset(self):
        self._check(self.lib.bcg_profile_reset(self.h))

    def kernel_time(self, kernel):
        n = ctypes.c_long()
        ms = ctypes.c_double()
        self._check(self.lib.bcg_kernel_time(self.h, KERNELS.index(kernel), ctypes.byref(n),
                                             ctypes.byref(ms)))
        return n.value, ms.value


class BlockSolve(torch.autograd.Function):
    """X = A(fat, long)^{-1} B with a hand-written backward.

    Forward: blockCGrQ.  Backward: the adjoint solve Lam = A^{-1} dL/dX (A is
    Hermitian, so it is the same block solve) gives dL/dB = Lam, and the link
    force of (X, Lam) gives dL/dfat and dL/dlong.  X is kept; no Krylov basis is.
    """

    @staticmethod
    def forward(ctx, B, fat, lng, solver):
        solver.load_links(fat.detach(), None if lng is None else lng.detach())
        X, info = solver.solve(B.detach().contiguous())
        ctx.solver = solver
        ctx.save_for_backward(X)
        ctx.has_long = lng is not None
        return X

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors
        solver = ctx.solver
        gX = gX.contiguous()
        n = gX.shape[0]
        # columns the loss does not depend on have Lam_i = 0 and add nothing to the
        # link force (it is a sum over columns of products with Lam_i); only the
        # others are solved (the solver rejects a zero right-hand side)
        live = torch.nonzero(gX.reshape(n, -1).abs().amax(dim=1) > 0).flatten()
        if live.numel() == n:
            Lam, _ = solver.solve(gX)
            gf, gl = solver.link_force(X, Lam)
        else:
            Lam = torch.zeros_like(gX)
            if live.numel() == 0:
                V = solver.V
                gf = torch.zeros((4, V, 3, 3), dtype=gX.dtype, device=gX.device)
                gl = torch.zeros_like(gf) if ctx.has_long else None
            else:
                Ls, _ = solver.solve(gX[live].contiguous())
                Lam[live] = Ls
                gf, gl = solver.link_force(X[live].contiguous(), Ls)
        return Lam, gf, (gl if ctx.has_long else None), None
