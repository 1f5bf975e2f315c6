"""Reference element, geometry and element matrices.  Test infrastructure.

Section 2 and eq. (matrices).  Reference element [0,1]^3.

* RT_p (H(div)) reference space Q_{p,p-1,p-1} x Q_{p-1,p,p-1} x Q_{p-1,p-1,p}.
  In the IH basis the x-component functions are  l_i(x) h_j(y) h_k(z) e_x
  (i = 0..p, j, k = 0..p-1), and y, z by permutation.  3 p^2 (p+1) in total.
  Local numbering: component-major (x, then y, then z); inside a component
  lexicographic with the first index fastest over its own shape
  ((p+1, p, p) for x, (p, p+1, p) for y, (p, p, p+1) for z).
* L2 space Q_{p-1}: h_a(x) h_b(y) h_c(z), a fastest.  p^3 functions.
* Element map: trilinear in the 8 vertices, J = dX/dxi.  RT functions use the
  contravariant Piola map  u = J u_hat / det J  (div u = div_hat u_hat / det J),
  L2 functions the integral-preserving map  q = q_hat / det J.
* Quadrature: tensor Gauss-Legendre rule with n_q = p + 1 points per direction
  for every matrix.  The paper does not fix the rule; this reading makes the
  rule exact on affine elements and is shared by the GPU path.
"""
import numpy as np

from .basis import Tables1D, lagrange, lagrange_deriv, histopolation, gauss_lobatto_points, gauss_legendre


def n_rt(p):
    return 3 * p * p * (p + 1)


def n_l2(p):
    return p ** 3


def rt_shapes(p):
    """Per-component index shapes (n_x, n_y, n_z) with the interpolation
    direction equal to the component."""
    return [(p + 1, p, p), (p, p + 1, p), (p, p, p + 1)]


def rt_reference(p, X):
    """Evaluate the reference RT_p IH basis at points X [n, 3].

    Returns (phi [n, n_rt, 3], div [n, n_rt]).
    """
    X = np.atleast_2d(X)
    xi = gauss_lobatto_points(p)
    l = [lagrange(xi, X[:, d]) for d in range(3)]          # [n, p+1]
    dl = [lagrange_deriv(xi, X[:, d]) for d in range(3)]
    h = [histopolation(xi, X[:, d]) for d in range(3)]      # [n, p]
    n = X.shape[0]
    phis, divs = [], []
    for c in range(3):
        f = [h[0], h[1], h[2]]
        f[c] = l[c]
        g = [h[0], h[1], h[2]]
        g[c] = dl[c]
        # array indexed [n, k, j, i] so that a C-order reshape gives i fastest
        v = np.einsum('ni,nj,nk->nkji', f[0], f[1], f[2]).reshape(n, -1)
        dv = np.einsum('ni,nj,nk->nkji', g[0], g[1], g[2]).reshape(n, -1)
        ph = np.zeros((n, v.shape[1], 3))
        ph[:, :, c] = v
        phis.append(ph)
        divs.append(dv)
    return np.concatenate(phis, axis=1), np.concatenate(divs, axis=1)


def l2_reference(p, X):
    """Evaluate the reference Q_{p-1} IH basis at points X [n, 3] -> [n, p^3]."""
    X = np.atleast_2d(X)
    xi = gauss_lobatto_points(p)
    h = [histopolation(xi, X[:, d]) for d in range(3)]
    n = X.shape[0]
    return np.einsum('na,nb,nc->ncba', h[0], h[1], h[2]).reshape(n, -1)


def tensor_points(x1d):
    """All points of the tensor grid x1d^3, first coordinate fastest."""
    z, y, x = np.meshgrid(x1d, x1d, x1d, indexing='ij')
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def tensor_weights(w1d):
    wz, wy, wx = np.meshgrid(w1d, w1d, w1d, indexing='ij')
    return (wx * wy * wz).ravel()


def trilinear(V, X):
    """Trilinear element map.

    V : vertices [..., 2, 2, 2, 3] indexed [dz, dy, dx, coord].
    X : reference points [n, 3].
    Returns (x [..., n, 3], J [..., n, 3, 3]) with J[r, c] = d x_r / d xi_c.
    """
    X = np.atleast_2d(X)
    N = [np.stack([1.0 - X[:, d], X[:, d]], axis=1) for d in range(3)]   # [n, 2]
    dN = np.array([-1.0, 1.0])
    x = np.einsum('na,nb,nc,...cbar->...nr', N[0], N[1], N[2], V)
    J0 = np.einsum('a,nb,nc,...cbar->...nr', dN, N[1], N[2], V)
    J1 = np.einsum('na,b,nc,...cbar->...nr', N[0], dN, N[2], V)
    J2 = np.einsum('na,nb,c,...cbar->...nr', N[0], N[1], dN, V)
    J = np.stack([J0, J1, J2], axis=-1)
    return x, J


class RefElement:
    """Reference basis values at the tensor Gauss-Legendre points."""

    def __init__(self, p, nq=None):
        self.p = p
        self.t = Tables1D(p, nq)
        self.nq = self.t.nq
        self.Xq = tensor_points(self.t.xq)
        self.wq = tensor_weights(self.t.wq)
        self.phi, self.div = rt_reference(p, self.Xq)   # [Q, nrt, 3], [Q, nrt]
        self.psi = l2_reference(p, self.Xq)             # [Q, nl2]


def element_matrices(p, V, c_mass=None, ref=None):
    """Element matrices of eq. (matrices) for a batch of elements.

    V : vertices [E, 2, 2, 2, 3].  c_mass : per-element weight of M (or None).
    Returns dict with
      M [E, nrt, nrt]  : sum_q w_q c (J phi_a).(J phi_b) / det J
      W [E, nl2, nl2]  : sum_q w_q psi_a psi_b / det J     (unweighted)
      B [E, nl2, nrt]  : sum_q w_q psi_a div_hat phi_b / det J
      detJ [E, Q]
    """
    if ref is None:
        ref = RefElement(p)
    V = np.asarray(V, dtype=np.float64)
    _, J = trilinear(V, ref.Xq)                       # [E, Q, 3, 3]
    det = np.linalg.det(J)                            # [E, Q]
    if np.any(det <= 0):
        raise ValueError("non-positive Jacobian determinant")
    Jphi = np.einsum('eqrc,qac->eqar', J, ref.phi)    # [E, Q, nrt, 3]
    wd = ref.wq[None, :] / det                        # [E, Q]
    M = np.einsum('eq,eqar,eqbr->eab', wd, Jphi, Jphi)
    if c_mass is not None:
        M = M * np.asarray(c_mass, dtype=np.float64)[:, None, None]
    W = np.einsum('eq,qa,qb->eab', wd, ref.psi, ref.psi)
    B = np.einsum('eq,qa,qb->eab', wd, ref.psi, ref.div)
    return dict(M=M, W=W, B=B, detJ=det)


def reference_divergence(p):
    """The local +-1 incidence D_e: rows = sub-volumes (a,b,c), columns = RT
    dofs.  From div_hat of l_i h_j h_k = l_i' h_j h_k and l_i' = h_{i-1} - h_i:
    the face at i = a+1 (upper face of volume a) enters with +1 and the face at
    i = a with -1 (Section 2.1, third basis property)."""
    nl = n_l2(p)
    D = np.zeros((nl, n_rt(p)))
    shapes = rt_shapes(p)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in shapes])
    for c in range(p):
        for b in range(p):
            for a in range(p):
                row = a + p * (b + p * c)
                loc = [a, b, c]
                for comp in range(3):
                    s = shapes[comp]
                    for shift, sign in ((1, +1.0), (0, -1.0)):
                        idx = list(loc)
                        idx[comp] += shift
                        col = offs[comp] + idx[0] + s[0] * (idx[1] + s[1] * idx[2])
                        D[row, col] = sign
    return D
