"""Right-preconditioned restarted GMRES and the block-triangular
preconditioner of the transformed system.  Test infrastructure.

The paper remarks (Section 2.2, the remark on block-triangular
preconditioners) that the upper block-triangular preconditioner built from
the (1,1) block and the Schur complement leaves the preconditioned operator
with the single eigenvalue 1 and a minimal polynomial of degree two, so that
GMRES converges in at most two iterations when both blocks are exact; in
practice the blocks are replaced by M~ and the AMG cycle on S~, and GMRES
replaces MINRES because the preconditioner is not symmetric.

For A = [[M, D^T], [D, -C]] (essential RT dofs: identity rows and columns)
the triangular factor is P = [[M~, D_f^T], [0, -S^]] with D_f^T the coupling
restricted to the free RT dofs, so that A P^{-1} = [[I + ..., 0], [D M~^{-1},
I]] is unit lower triangular when M~ = M and S^ = C + D M^{-1} D^T.  Applying
P^{-1} to r = [r_u; r_q]:

    z_q = -S^{-1} r_q,    z_u = M~^{-1} (r_u - D_f^T z_q)   (free dofs),
    z_u = r_u on the essential dofs.

GMRES (Saad and Schultz): Arnoldi on A P^{-1} with modified Gram-Schmidt,
Givens rotations on the Hessenberg matrix, |g_{j+1}| the residual norm of
the current iterate; stop when it is <= tol ||r_0||, restart after `restart`
Arnoldi steps.  x = x_0 + P^{-1} V y.  The iteration count is the number of
operator applications after the initial residual.
"""
import numpy as np
import scipy.sparse as sp

from . import precond


class TriangularPreconditioner:
    """z = P^{-1} r for the upper block-triangular P = [[tau M~, D_f^T],
    [0, -S^]].  schur = 'amg' (one V-cycle on S~, the block-diagonal
    preconditioner's) or 'exact_blocks': M~ = M and S^ = C + D_f M^{-1} D_f^T
    both exact (dense solves; tiny problems only)."""

    def __init__(self, prob, tau=1.0, schur='amg', amg_kwargs=None):
        self.prob = prob
        self.nu = prob.mesh.n_u
        self.free = ~prob.ess
        D = prob.D.tocsr()
        self.Df = (D @ sp.diags(self.free.astype(np.float64))).tocsr()
        if schur == 'exact_blocks':
            fi = np.nonzero(self.free)[0]
            Mff = prob.M.toarray()[np.ix_(fi, fi)]
            Dff = prob.D.toarray()[:, fi]
            Sx = prob.C.toarray() + Dff @ np.linalg.solve(Mff, Dff.T)
            self._fi = fi
            self._Mff = Mff
            self._mu = lambda v: np.linalg.solve(Mff, v)
            self.schur = lambda r: np.linalg.solve(Sx, r)
            self.exact = True
        else:
            self.Md = precond.diag_M(prob)
            bp = precond.BlockPreconditioner(prob, tau=tau, schur=schur, amg_kwargs=amg_kwargs)
            self.schur = bp.schur
            self.tau = tau
            self.exact = False

    def __call__(self, r):
        r = np.asarray(r, dtype=np.float64)
        ru, rq = r[:self.nu], r[self.nu:]
        zq = -self.schur(rq)
        t = ru - self.Df.T @ zq
        if self.exact:
            zu = ru.copy()
            zu[self._fi] = self._mu(t[self._fi])
        else:
            zu = t / (self.tau * self.Md)
            zu[self.prob.ess] = ru[self.prob.ess]
        return np.concatenate([zu, zq])


def gmres(apply_A, apply_Pinv, b, x0=None, tol=1e-10, restart=30, maxiter=10000, history=None):
    """Return (x, iterations, info) with info = {'res': [...], 'converged'}."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r = b - apply_A(x)
    beta0 = np.linalg.norm(r)
    res = [1.0]
    if beta0 == 0.0:
        return x, 0, dict(res=res, converged=True)
    it = 0
    converged = False
    while it < maxiter and not converged:
        beta = np.linalg.norm(r)
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        for j in range(restart):
            it += 1
            w = apply_A(apply_Pinv(V[j]))
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):              # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            res.append(abs(g[j + 1]) / beta0)
            if abs(g[j + 1]) <= tol * beta0 or it >= maxiter or hn == 0.0:
                converged = abs(g[j + 1]) <= tol * beta0 or hn == 0.0
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + apply_Pinv(sum(y[i] * V[i] for i in range(k)))
        r = b - apply_A(x)
        if history is not None:
            history.append(np.linalg.norm(r) / beta0)
    return x, it, dict(res=res, converged=converged)
