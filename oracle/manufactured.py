"""Manufactured Darcy solution and discretisation errors.  Test infrastructure.

Darcy problem (eq. darcy) with eps = 1, gamma = 0 on the unit cube:
    u + grad p = 0,   div u = g,   p = sin(pi x) sin(pi y) sin(pi z)
so u = -grad p and g = 3 pi^2 p; p = 0 on the boundary, so the natural
condition adds no boundary term.

Sign reading: with the block form of eq. (darcy-nonzero),
[[M, B^T], [B, -W_gamma]] [u; p_sys] = [f^; g^], the pressure unknown is
p_sys = -p (integrating (grad p, v) by parts gives -(p, div v)).  The
transformed unknown of eq. (transformed-system-darcy) is p~ = W p_sys and the
transformed right-hand side is [f^; W^{-1} g^].
"""
import numpy as np

from .element import tensor_points, tensor_weights, trilinear, rt_reference, l2_reference
from .basis import gauss_legendre


def p_exact(x):
    return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) * np.sin(np.pi * x[..., 2])


def u_exact(x):
    s = np.sin(np.pi * x)
    c = np.cos(np.pi * x)
    return -np.pi * np.stack([c[..., 0] * s[..., 1] * s[..., 2],
                              s[..., 0] * c[..., 1] * s[..., 2],
                              s[..., 0] * s[..., 1] * c[..., 2]], axis=-1)


def g_exact(x):
    return 3.0 * np.pi ** 2 * p_exact(x)


def _quad(prob, nq):
    xq, wq = gauss_legendre(nq)
    X = tensor_points(xq)
    w = tensor_weights(wq)
    V = prob.mesh.element_vertices()
    x, J = trilinear(V, X)
    det = np.linalg.det(J)
    return X, w, x, J, det


def l2_load(prob, fun, nq=None):
    """Vector of (f, psi_a) over all L2 dofs (element-major)."""
    p = prob.mesh.p
    nq = p + 1 if nq is None else nq
    X, w, x, J, det = _quad(prob, nq)
    psi = l2_reference(p, X)                       # [Q, nl]
    f = fun(x)                                      # [E, Q]
    # psi_phys = psi_hat / det, dx = det dxi
    return np.einsum('q,eq,qa->ea', w, f, psi).ravel()


def darcy_rhs(prob):
    """[f^; W^{-1} g^] of the transformed system for the manufactured case."""
    import scipy.sparse.linalg as spla
    gh = l2_load(prob, g_exact)
    bq = spla.spsolve(prob.W.tocsc(), gh)
    return np.concatenate([np.zeros(prob.mesh.n_u), bq])


def darcy_errors(prob, sol, nq_err=None):
    """Errors of the transformed solution sol = [u; p~]:
    ||u - u_h||, ||p - p_h||, ||Pi_W p - p_h|| (Pi_W the L2 projection)."""
    import scipy.sparse.linalg as spla
    mesh = prob.mesh
    p = mesh.p
    nq = p + 3 if nq_err is None else nq_err
    u = sol[:mesh.n_u]
    ptil = sol[mesh.n_u:]
    p_sys = spla.spsolve(prob.W.tocsc(), ptil)
    ph = -p_sys
    X, w, x, J, det = _quad(prob, nq)
    phi, _ = rt_reference(p, X)                    # [Q, nrt, 3]
    psi = l2_reference(p, X)                       # [Q, nl]
    ue = u[prob.l2g]                               # [E, nrt]
    uh_ref = np.einsum('qar,ea->eqr', phi, ue)
    uh = np.einsum('eqrc,eqc->eqr', J, uh_ref) / det[..., None]
    err_u = np.sqrt(np.einsum('q,eq,eq->', w, det, ((uh - u_exact(x)) ** 2).sum(-1)))
    phe = ph.reshape(mesh.ne, -1)
    ph_x = np.einsum('qa,ea->eq', psi, phe) / det
    err_p = np.sqrt(np.einsum('q,eq,eq->', w, det, (ph_x - p_exact(x)) ** 2))
    # L2 projection of p onto W_h (coefficients W^{-1} (p, psi))
    pi = spla.spsolve(prob.W.tocsc(), l2_load(prob, p_exact, nq))
    d = pi - ph
    err_pp = np.sqrt(d @ (prob.W @ d))
    return dict(u=err_u, p=err_p, proj_p=err_pp)
