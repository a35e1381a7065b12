"""CPU FP64 oracle for block CG (blockCGrQ) on the even-odd staggered normal operator.

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the bench's CPU-baseline
leg may import or call this package; the solver library and its Python
binding never do, and the two share no code.  It is written to be read
against the paper, not to be fast:

* the stencil, the normal operator A = 4 m^2 - D_eo D_oe and the link force are
  plain C99 (``stencil.c``, FP64, one OpenMP loop over sites);
* the Krylov algorithms below are NumPy in the paper's order and notation, with
  library matmul / Cholesky / triangular solves as the only building blocks.

Block vectors are [N][V/2][3] complex128 arrays (N right-hand sides on the even
checkerboard).  The algorithms view them as L x N matrices with L = 3 V/2,
columns = right-hand sides, as in Alg. 1.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
from scipy.linalg import solve_triangular

from . import build as _build

_LIB = None
_HERE = os.path.dirname(os.path.abspath(__file__))


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if (not os.path.exists(path)
                or os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L = ctypes.c_long
        lib.oracle_dslash_full.argtypes = [P, I, P, P, P, P]
        lib.oracle_hop.argtypes = [P, I, P, P, I, I, P, P]
        lib.oracle_apply.argtypes = [P, I, P, P, D, I, P, P, P]
        lib.oracle_apply_sites.argtypes = [P, I, P, P, D, I, P, L, P, P]
        lib.oracle_link_force.argtypes = [P, I, I, P, P, P, P, P, P]
        lib.oracle_num_threads.restype = I
        _LIB = lib
    return _LIB


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    if d.shape != (4,) or np.any(d < 2) or np.any(d % 2):
        raise ValueError(f"dims must be four even extents >= 2, got {dims}")
    return d


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


class Operator:
    """The staggered stencil and A = 4 m^2 - D_eo D_oe for one set of links."""

    def __init__(self, dims, fat, lng=None, mass=0.0):
        self.dims = _dims(dims)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.improved = lng is not None
        self.fat = _c128(fat).reshape(4, self.V, 3, 3)
        self.lng = _c128(lng).reshape(4, self.V, 3, 3) if self.improved else None
        self.mass = float(mass)

    # -- stencil ---------------------------------------------------------------------------
    def dslash_full(self, psi):
        """D on the whole lattice, psi [V][3] in lex order (Sec. 3.2, Eq. 2)."""
        psi = _c128(psi).reshape(self.V, 3)
        out = np.empty_like(psi)
        _lib().oracle_dslash_full(_ptr(self.dims), int(self.improved), _ptr(self.fat),
                                  _ptr(self.lng), _ptr(psi), _ptr(out))
        return out

    def hop(self, out_parity, v):
        """D_{p,1-p}: [N][V/2][3] on parity 1-p -> [N][V/2][3] on parity p."""
        v = _c128(v)
        n = v.shape[0]
        v = v.reshape(n, self.Vh, 3)
        out = np.empty_like(v)
        _lib().oracle_hop(_ptr(self.dims), int(self.improved), _ptr(self.fat), _ptr(self.lng),
                          int(out_parity), n, _ptr(v), _ptr(out))
        return out

    def apply(self, v):
        """A v = 4 m^2 v - D_eo D_oe v on even fields [N][V/2][3] (Sec. 3.2)."""
        v = _c128(v)
        n = v.shape[0]
        v = v.reshape(n, self.Vh, 3)
        out = np.empty_like(v)
        work = np.empty_like(v)
        _lib().oracle_apply(_ptr(self.dims), int(self.improved), _ptr(self.fat), _ptr(self.lng),
                            self.mass, n, _ptr(v), _ptr(out), _ptr(work))
        return out

    def apply_sites(self, v, cb_sites):
        """(A v)(x) only at the given even checkerboard sites -> [N][nsites][3]."""
        v = _c128(v)
        n = v.shape[0]
        v = v.reshape(n, self.Vh, 3)
        cb = np.ascontiguousarray(cb_sites, dtype=np.int64)
        if cb.size and (cb.min() < 0 or cb.max() >= self.Vh):
            raise ValueError("site index out of range")
        out = np.empty((n, cb.size, 3), dtype=np.complex128)
        _lib().oracle_apply_sites(_ptr(self.dims), int(self.improved), _ptr(self.fat),
                                  _ptr(self.lng), self.mass, n, _ptr(v), int(cb.size), _ptr(cb),
                                  _ptr(out))
        return out

    def link_force(self, X, Lam):
        """Gradients w.r.t. (fat, long) of L with dL = -Re sum_i Lam_i^H dA X_i.

        Y_X = D_oe X and Y_Lam = D_oe Lam are formed with the oracle's own hop.
        Returns (grad_fat, grad_long or None), each [4][V][3][3].
        """
        X = _c128(X)
        Lam = _c128(Lam)
        n = X.shape[0]
        YX = self.hop(1, X)
        YL = self.hop(1, Lam)
        gf = np.empty((4, self.V, 3, 3), dtype=np.complex128)
        gl = np.empty((4, self.V, 3, 3), dtype=np.complex128) if self.improved else None
        _lib().oracle_link_force(_ptr(self.dims), int(self.improved), n, _ptr(X), _ptr(Lam),
                                 _ptr(YX), _ptr(YL), _ptr(gf), _ptr(gl))
        return gf, gl


# ---------------------------------------------------------------------------------------------
# Block vectors as L x N matrices
# ---------------------------------------------------------------------------------------------
def to_mat(v) -> np.ndarray:
    """[N][V/2][3] -> L x N (column i = right-hand side i)."""
    v = np.asarray(v)
    return v.reshape(v.shape[0], -1).T


def from_mat(m, vh) -> np.ndarray:
    return np.ascontiguousarray(m.T).reshape(m.shape[1], vh, 3)


class Breakdown(RuntimeError):
    """A Cholesky factorisation met a non-positive pivot (R^H R singular, Sec. 4)."""


def cholesky_upper(H) -> np.ndarray:
    """H = R^H R with R upper triangular and positive real diagonal."""
    try:
        Lo = np.linalg.cholesky(H)
    except np.linalg.LinAlgError as e:
        raise Breakdown(str(e)) from None
    return Lo.conj().T


def thin_qr(M):
    """Alg. 2 (CholQR): H = M^H M, H = R^H R, Q = M R^{-1}.  Returns (Q, R)."""
    H = M.conj().T @ M
    R = cholesky_upper(H)
    Q = solve_triangular(R, M.T, trans="T", lower=False).T
    return Q, R


def thin_qr2(M):
    """CholQR2: Alg. 2 applied twice, the second time to the Q of the first.
    Q1 C1 = M, Q C2 = Q1, so M = Q (C2 C1).  Returns (Q, C2 C1)."""
    Q1, C1 = thin_qr(M)
    Q, C2 = thin_qr(Q1)
    return Q, C2 @ C1


def hpd_inverse(G) -> np.ndarray:
    """G^{-1} for Hermitian positive-definite G via its Cholesky factor."""
    R = cholesky_upper(G)
    Rinv = solve_triangular(R, np.eye(R.shape[0], dtype=R.dtype), lower=False)
    return Rinv @ Rinv.conj().T


class SolveInfo(dict):
    __getattr__ = dict.__getitem__


def block_cg_rq(apply_A, B, tol, max_iter=100000, X0=None, ru_delta=0.0, sloppy=None,
                trace=None, apply_sloppy=None, ru_window=0, stall_limit=0, qr_passes=1):
    """blockCGrQ (Alg. 1) with CholQR (Alg. 2) and block reliable updates (Alg. 3).

    apply_A: maps [N][V/2][3] -> [N][V/2][3].
    B: [N][V/2][3] right-hand sides (no zero column).
    tol: stop when every relative residual ||b_i - A x_i|| / ||b_i|| <= tol.  The
      test runs on the iterated residual, R_{k+1} = Qt C_k, whose column norms are
      sqrt((C_k^H H C_k)_ii) with H = Qt^H Qt (Sec. 6, residual-norm identity);
      the result is then checked against the true residual B - A Y and, if a
      column misses tol, a reliable update is made and the iteration continues.
    ru_delta: reliable update when the maximum relative iterated residual has
      dropped by this factor since the last one (0 disables; 0.1 in Sec. 7.1).
    sloppy: rounding applied to the low-precision block vectors P, Q, AP (None:
      all FP64).  Y (solution) and X (update since the last reliable update)
      stay FP64 (Sec. 6, mixed precision).
    apply_sloppy: the operator of the iteration's A P (Sec. 6: the iteration
      runs on low-precision links); None = apply_A.  The initial and the
      reliable-update residuals B - A Y always use apply_A (Alg. 3).
    ru_window: adaptive reliable updates: also update when the maximum relative
      iterated residual has not reached a new minimum since the last reliable
      update for this many iterations (0 disables).  In exact arithmetic an
      update changes nothing (S = C^ C_k^{-1} continues the recurrence), so
      this only decides how often the true residual replaces the iterated one
      -- one form of the better reliable-update schemes that Sec. 8 leaves
      open for low storage precision.
    stall_limit: stop without convergence after this many reliable updates in
      a row whose true residual fails to halve the smallest maximum true
      relative residual seen so far (0 disables); info.stalled is then True
      and the solution returned is the iterate with the smallest true residual
      among those checked.
    qr_passes: 1 = the initial and reliable-update thin QR is CholQR (Alg. 2),
      2 = CholQR2 (thin_qr2).  The QR inside the iteration is always Alg. 2.
    trace: optional list; per iteration a dict with beta, C (before the update),
      S and the relative iterated residuals is appended (and the true relative
      residuals at a reliable update).

    Returns (solution [N][V/2][3], SolveInfo).
    Raises Breakdown when a Cholesky factorisation fails before convergence.
    """
    B = np.asarray(B, dtype=np.complex128)
    n, vh = B.shape[0], B.shape[1]
    rnd = sloppy if sloppy is not None else (lambda a: a)

    def A(M):
        return to_mat(apply_A(from_mat(M, vh)))

    As = A if apply_sloppy is None else (lambda M: to_mat(apply_sloppy(from_mat(M, vh))))

    Bm = to_mat(B)
    bnorm = np.linalg.norm(Bm, axis=0)
    if np.any(bnorm == 0):
        raise ValueError("zero right-hand side column")
    Y = to_mat(X0).astype(np.complex128) if X0 is not None else np.zeros_like(Bm)
    X = np.zeros_like(Bm)
    R = Bm - A(Y) if X0 is not None else Bm.copy()
    qr = thin_qr2 if qr_passes == 2 else thin_qr
    Q, C = qr(R)                                # Q C = R
    Q = rnd(Q)
    S = np.eye(n, dtype=np.complex128)
    P = np.zeros_like(Bm)
    rho_ru = float(np.max(np.linalg.norm(R, axis=0) / bnorm))
    it = 0
    n_ru = 0
    history = []
    converged = False
    stalled = False
    best_it, best_res = 0, rho_ru               # newest minimum of the iterated residual
    best_true, n_stall = rho_ru, 0              # smallest true residual, updates without progress
    Y_best = Y.copy()                           # the iterate of best_true
    true_rel = np.linalg.norm(R, axis=0) / bnorm
    if rho_ru <= tol:
        converged = True
    while not converged and it < max_iter:
        P = rnd(Q + P @ S.conj().T)             # P = Q + P S^H
        AP = rnd(As(P))
        G = P.conj().T @ AP                     # P^H A P
        beta = hpd_inverse(G)                   # beta = (P^H A P)^{-1}
        X = X + P @ (beta @ C)                  # X = X + P beta C
        Qt = rnd(Q - AP @ beta)                 # Q S = Q - A P beta  (before the QR)
        H = Qt.conj().T @ Qt
        it += 1
        relres = np.sqrt(np.maximum(np.real(np.diag(C.conj().T @ H @ C)), 0.0)) / bnorm
        history.append(float(relres.max()))
        rec = dict(beta=beta, C=C.copy(), relres=relres)
        conv = bool(relres.max() <= tol)
        if relres.max() < best_res:
            best_it, best_res = it, float(relres.max())
        stuck = ru_window > 0 and it - best_it >= ru_window
        if conv or stuck or (ru_delta > 0 and relres.max() <= ru_delta * rho_ru):
            # reliable update (Alg. 3): fold X into Y, recompute the true residual
            Y = Y + X
            X = np.zeros_like(X)
            R = Bm - A(Y)
            true_rel = np.linalg.norm(R, axis=0) / bnorm
            rec["true_rel"] = true_rel
            if conv and true_rel.max() <= tol:
                converged = True
                rec["S"] = None
                if trace is not None:
                    trace.append(rec)
                break
            n_stall = 0 if true_rel.max() <= 0.5 * best_true else n_stall + 1
            if true_rel.max() < best_true:
                best_true, Y_best = float(true_rel.max()), Y.copy()
            if stall_limit > 0 and n_stall >= stall_limit:
                stalled = True
                rec["S"] = None
                if trace is not None:
                    trace.append(rec)
                break
            Qh, Ch = qr(R)                      # Q^ C^ = R
            S = Ch @ np.linalg.inv(C)           # S = C^ C_k^{-1}, C_k the C before this step
            C = Ch
            Q = rnd(Qh)
            rho_ru = float(true_rel.max())
            best_it, best_res = it, rho_ru
            n_ru += 1
            rec["ru"] = True
        else:
            S = cholesky_upper(H)               # H = S^H S
            Q = rnd(solve_triangular(S, Qt.T, trans="T", lower=False).T)   # Q = Qt S^{-1}
            C = S @ C                           # C = S C
        rec["S"] = S
        if trace is not None:
            trace.append(rec)
    if not converged:
        Y = Y + X
        true_rel = np.linalg.norm(Bm - A(Y), axis=0) / bnorm
        if stalled and not true_rel.max() <= best_true:
            # a stalled solve returns the iterate with the smallest true residual seen
            Y = Y_best
            true_rel = np.linalg.norm(Bm - A(Y), axis=0) / bnorm
    info = SolveInfo(iters=it, reliable_updates=n_ru, converged=converged, stalled=stalled,
                     true_rel_res=true_rel, history=history)
    return from_mat(Y, vh), info


def sstep_block_cg(apply_A, B, s, tol, lam, max_outer=100000, basis="chebyshev", trace=None,
                   sloppy=None, apply_sloppy=None, ru_delta=0.0):
    """s-step block CG: every outer iteration extends the search space by s block
    Krylov directions at once, so that all of its inner products form one
    reduction phase per s steps instead of two per step -- the s-step methods that
    Sec. 8 proposes for block solvers (Chronopoulos and Gear's s-step CG, with N
    columns per direction).

    Outer iteration k, with R_k the L x N block residual and K = s N columns:
      basis       V = [V_0 ... V_{s-1}], V_0 = R_k, each V_j = p_j(A) R_k with p_j of
                  degree j: the Chebyshev polynomials of the interval
                  lam = (lmin, lmax) (c = (lmax + lmin) / 2, h = (lmax - lmin) / 2;
                  V_1 = (A V_0 - c V_0) / h, V_{j+1} = 2 (A V_j - c V_j) / h - V_{j-1}),
                  or the monomials V_{j+1} = A V_j (basis="monomial");  AV = A V
      reduction   Gv = V^H AV and Gr = V^H R_k; after the first outer iteration also
                  Ga = (A P_{k-1})^H V, Wp = P_{k-1}^H A P_{k-1} and Pr = P_{k-1}^H R_k
      directions  first outer iteration (and after a restart): P = V, AP = AV,
                  W = Gv, g = Gr;  otherwise Bk = -Wp^{-1} Ga (P A-orthogonal to
                  P_{k-1}), P = V + P_{k-1} Bk, AP = AV + AP_{k-1} Bk,
                  W = Gv + Ga^H Bk (= P^H A P) and g = Gr + Bk^H Pr (= P^H R_k)
      step        alpha = W^{-1} g, X = X + P alpha, R = R_k - AP alpha.
    In exact arithmetic Pr = 0, Wp is the previous W and X after k outer
    iterations is the Galerkin solution over X0 + K_{ks}(A, R_0), i.e. blockCGrQ's
    X after k s iterations, whatever the basis polynomials.  In floating point the
    recurrence needs the freshly reduced Wp and Pr: carrying W over, or dropping Pr,
    breaks down for s >= 3 on the 4^4 test operators (the instability of s-step
    methods that Sec. 8 anticipates).

    The stopping test runs on the iterated residual at the top of each outer
    iteration (max_i ||r_i|| / ||b_i|| <= tol), then on the true residual
    B - A X; if that misses tol, the recurrence restarts from it (P discarded).
    max_outer bounds the outer iterations.
    trace: optional list; per outer iteration a dict with Bk, W and alpha.

    Low-precision storage (Sec. 6's mixed precision carried over): sloppy rounds
    the stored block vectors V, AV, P and AP (each as formed, V_0 = R rounded) and
    apply_sloppy is the operator of the basis; X, R, the Grams and all N x N work
    stay FP64.  ru_delta > 0 adds reliable updates (Alg. 3's role): when the
    maximum relative iterated residual has dropped by ru_delta since the last one,
    R is replaced by the FP64 true residual B - A X and the directions P, AP are
    kept (the reduced Pr = P^H R absorbs the change).

    Returns (X [N][V/2][3], SolveInfo(iters = outer iterations * s, outer,
    restarts, reliable_updates, converged, true_rel_res)).
    Raises Breakdown when Wp or W is not positive definite.
    """
    B = np.asarray(B, dtype=np.complex128)
    n, vh = B.shape[0], B.shape[1]
    if s < 1:
        raise ValueError("s must be at least 1")

    def A(M):
        return to_mat(apply_A(from_mat(M, vh)))

    rnd = sloppy if sloppy is not None else (lambda a: a)
    As = A if apply_sloppy is None else (lambda M: to_mat(apply_sloppy(from_mat(M, vh))))
    lmin, lmax = float(lam[0]), float(lam[1])
    c, h = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    Bm = to_mat(B)
    bnorm = np.linalg.norm(Bm, axis=0)
    if np.any(bnorm == 0):
        raise ValueError("zero right-hand side column")
    X = np.zeros_like(Bm)
    R = Bm.copy()
    P = AP = None
    outer = restarts = n_ru = 0
    converged = False
    true_rel = np.linalg.norm(R, axis=0) / bnorm
    rho_ru = float(true_rel.max())
    while True:
        relres = np.max(np.linalg.norm(R, axis=0) / bnorm)
        if relres <= tol:
            Rt = Bm - A(X)
            true_rel = np.linalg.norm(Rt, axis=0) / bnorm
            if true_rel.max() <= tol:
                converged = True
                break
            R, P, AP = Rt, None, None
            restarts += 1
            rho_ru = float(true_rel.max())
        elif ru_delta > 0 and relres <= ru_delta * rho_ru:
            R = Bm - A(X)
            rho_ru = float(np.max(np.linalg.norm(R, axis=0) / bnorm))
            n_ru += 1
        if outer >= max_outer:
            break
        # the s basis blocks and their images under A
        Vb, AVb = [rnd(R)], []
        for j in range(s):
            AVb.append(rnd(As(Vb[j])))
            if j + 1 < s:
                if basis == "monomial":
                    Vb.append(AVb[j])
                elif j == 0:
                    Vb.append(rnd((AVb[0] - c * Vb[0]) / h))
                else:
                    Vb.append(rnd(2.0 * (AVb[j] - c * Vb[j]) / h - Vb[j - 1]))
        V, AV = np.hstack(Vb), np.hstack(AVb)
        Gv = V.conj().T @ AV
        Gr = V.conj().T @ Vb[0]
        if P is None:
            Bk = np.zeros((s * n, s * n), dtype=np.complex128)
            P, AP, W, g = V, AV, Gv, Gr
        else:
            Ga = AP.conj().T @ V
            Wp = P.conj().T @ AP
            Pr = P.conj().T @ Vb[0]
            Bk = -hpd_inverse(0.5 * (Wp + Wp.conj().T)) @ Ga
            P = rnd(V + P @ Bk)
            AP = rnd(AV + AP @ Bk)
            W = Gv + Ga.conj().T @ Bk
            g = Gr + Bk.conj().T @ Pr
        W = 0.5 * (W + W.conj().T)
        alpha = hpd_inverse(W) @ g
        X = X + P @ alpha
        R = R - AP @ alpha
        outer += 1
        if trace is not None:
            trace.append(dict(Bk=Bk, W=W, alpha=alpha))
    if not converged:
        true_rel = np.linalg.norm(Bm - A(X), axis=0) / bnorm
    info = SolveInfo(iters=outer * s, outer=outer, restarts=restarts, reliable_updates=n_ru,
                     converged=converged, true_rel_res=true_rel)
    return from_mat(X, vh), info


def cg(apply_A, b, tol, max_iter=100000):
    """Textbook Hestenes-Stiefel CG for one right-hand side b [V/2][3] (the baseline, Sec. 7.1).

    Stops on the iterated residual, then checks the true residual; if it misses
    tol the recurrence restarts from r = b - A x.
    Returns (x, SolveInfo).
    """
    b = np.asarray(b, dtype=np.complex128)
    shape = b.shape

    def A(v):
        return apply_A(v.reshape((1,) + shape)).reshape(shape)

    bn = np.sqrt(np.vdot(b, b).real)
    if bn == 0:
        raise ValueError("zero right-hand side")
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    it = 0
    restarts = 0
    converged = False
    while it < max_iter:
        if np.sqrt(rr) / bn <= tol:
            r = b - A(x)
            rr = np.vdot(r, r).real
            if np.sqrt(rr) / bn <= tol:
                converged = True
                break
            p = r.copy()
            restarts += 1
        Ap = A(p)
        alpha = rr / np.vdot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    true = np.sqrt(np.vdot(b - A(x), b - A(x)).real) / bn
    return x, SolveInfo(iters=it, restarts=restarts, converged=converged, true_rel_res=true)


def solve_with_grads(op: Operator, B, G_up, tol=1e-12, max_iter=100000):
    """X = A^{-1} B and the backward for an upstream gradient G_up = dL/dX.

    Lam = A^{-1} G_up (A is Hermitian, so the adjoint solve uses the same operator);
    grad_B = Lam; link gradients from the link force of (X, Lam).
    Returns (X, grad_B, grad_fat, grad_long).
    """
    X, _ = block_cg_rq(op.apply, B, tol, max_iter)
    Lam, _ = block_cg_rq(op.apply, G_up, tol, max_iter)
    gf, gl = op.link_force(X, Lam)
    return X, Lam, gf, gl
