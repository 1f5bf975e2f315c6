"""Preconditioned MINRES.  Test infrastructure.

The paper solves the symmetric indefinite transformed system with MINRES and
the symmetric positive definite block-diagonal preconditioner (Sections 2, 2.2
and 3).  This is the preconditioned Lanczos process with Givens rotations of
Paige and Saunders, in the form given by Elman, Silvester and Wathen: the
Lanczos vectors are orthonormal in the B^{-1} inner product, and the quantity
|eta| carried by the recurrence equals the B^{-1}-norm of the current
residual, ||r_k||_{B^{-1}}.

Stopping: |eta_k| <= tol * |eta_0|.  The iteration count is the number of
operator applications after the initial residual.
"""
import numpy as np


def minres(apply_A, apply_Binv, b, x0=None, tol=1e-10, maxiter=10000, history=None):
    """Return (x, iterations, info) with info = {'eta': [...], 'converged': bool}."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    v_old = np.zeros(n)
    w_old = np.zeros(n)
    w = np.zeros(n)
    v = b - apply_A(x)
    z = apply_Binv(v)
    gamma = np.sqrt(np.dot(z, v))
    gamma_old = 1.0
    eta = gamma
    eta0 = gamma
    s_old = s = 0.0
    c_old = c = 1.0
    etas = [abs(eta)]
    if eta0 == 0.0:
        return x, 0, dict(eta=etas, converged=True)
    it = 0
    converged = False
    while it < maxiter:
        it += 1
        z = z / gamma
        Az = apply_A(z)
        delta = np.dot(Az, z)
        v_new = Az - (delta / gamma) * v - (gamma / gamma_old) * v_old
        z_new = apply_Binv(v_new)
        g2 = np.dot(z_new, v_new)
        if g2 < 0:
            raise FloatingPointError("preconditioner is not positive definite")
        gamma_new = np.sqrt(g2)
        a0 = c * delta - c_old * s * gamma
        a1 = np.sqrt(a0 * a0 + gamma_new * gamma_new)
        a2 = s * delta + c_old * c * gamma
        a3 = s_old * gamma
        c_new = a0 / a1
        s_new = gamma_new / a1
        w_new = (z - a3 * w_old - a2 * w) / a1
        x = x + c_new * eta * w_new
        eta = -s_new * eta
        etas.append(abs(eta))
        # shift
        v_old, v = v, v_new
        z = z_new
        w_old, w = w, w_new
        gamma_old, gamma = gamma, gamma_new
        c_old, c = c, c_new
        s_old, s = s, s_new
        if abs(eta) <= tol * eta0:
            converged = True
            break
        if gamma == 0.0:
            converged = True
            break
    return x, it, dict(eta=etas, converged=converged)
