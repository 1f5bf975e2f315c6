"""Structured global assembly and the transformed block operator.  Test infrastructure.

Mesh: nx x ny x nz hexahedra, vertices [(nx+1)(ny+1)(nz+1), 3] with x fastest,
element e = ex + nx (ey + ny ez), element vertex (dx, dy, dz) at vertex index
(ex+dx) + (nx+1) ((ey+dy) + (ny+1)(ez+dz)).

Global RT numbering (one global dof per sub-element face of the refined grid):
direction-major (all x-normal faces, then y, then z); inside a direction
lexicographic over the refined face grid, first index fastest.  The global
face normal is the +axis direction, which coincides with the reference
orientation of every element on a structured mesh (sigma_glob = +1).

Global L2 numbering is element-major: e, then the local (a, b, c), a fastest.

Operator (eq. transformed-system and eq. transformed-system-darcy):
    A = [[M, D^T], [D, -C]]
  grad-div:  M = M_beta, C = W_alpha^{-1}, kappa_e = 1/alpha_e
  Darcy:     M = M_{1/eps}, C = W^{-1} W_gamma W^{-1} = W_{1/gamma}^{-1}
             for piecewise-constant gamma, kappa_e = gamma_e (0 allowed)
  so in both cases C is block diagonal with blocks kappa_e W_e^{-1}, W_e the
  unweighted element L2 mass matrix.  Darcy with gamma varying inside the
  elements (a continuous piecewise-trilinear field given at the vertices,
  `gamma_vertices`): C_e = W_e^{-1} W_gamma,e W_e^{-1} in full (Section 2.4,
  the general case of eq. transformed-system-darcy).
Essential flux dofs (faces on the selected sides of the box) get identity rows
and columns.
"""
import numpy as np
import scipy.sparse as sp

from .element import RefElement, element_matrices, n_rt, n_l2, rt_shapes

GRADDIV = 0
DARCY = 1

# bit masks of the six sides of the box
SIDE_XMIN, SIDE_XMAX, SIDE_YMIN, SIDE_YMAX, SIDE_ZMIN, SIDE_ZMAX = 1, 2, 4, 8, 16, 32


class Mesh:
    def __init__(self, nx, ny, nz, p, vertices):
        self.nx, self.ny, self.nz, self.p = int(nx), int(ny), int(nz), int(p)
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        assert self.vertices.shape[0] == (nx + 1) * (ny + 1) * (nz + 1)
        self.ne = nx * ny * nz
        P = p
        self.nface = [(nx * P + 1) * (ny * P) * (nz * P),
                      (nx * P) * (ny * P + 1) * (nz * P),
                      (nx * P) * (ny * P) * (nz * P + 1)]
        self.n_u = sum(self.nface)
        self.n_q = self.ne * P ** 3
        self.n = self.n_u + self.n_q

    def element_index(self, ex, ey, ez):
        return ex + self.nx * (ey + self.ny * ez)

    def element_coords(self, e):
        e = np.asarray(e)
        return e % self.nx, (e // self.nx) % self.ny, e // (self.nx * self.ny)

    def element_vertices(self, elems=None):
        """[E, 2, 2, 2, 3] vertex coordinates indexed [dz, dy, dx, :]."""
        if elems is None:
            elems = np.arange(self.ne)
        ex, ey, ez = self.element_coords(np.asarray(elems))
        V = np.zeros((len(ex), 2, 2, 2, 3))
        nx1, ny1 = self.nx + 1, self.ny + 1
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    vid = (ex + dx) + nx1 * ((ey + dy) + ny1 * (ez + dz))
                    V[:, dz, dy, dx, :] = self.vertices[vid]
        return V

    def rt_local_to_global(self, elems=None):
        """[E, n_rt] global RT dof of each local dof (rt_local_to_global of
        Algorithm 1, here by index arithmetic on the structured grid)."""
        if elems is None:
            elems = np.arange(self.ne)
        P = self.p
        ex, ey, ez = self.element_coords(np.asarray(elems))
        base = [ex * P, ey * P, ez * P]
        out = []
        off = 0
        dims = [(self.nx * P, self.ny * P, self.nz * P)] * 3
        for c, shp in enumerate(rt_shapes(P)):
            gdim = list(dims[c])
            gdim[c] += 1
            kk, jj, ii = np.meshgrid(np.arange(shp[2]), np.arange(shp[1]), np.arange(shp[0]), indexing='ij')
            ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
            gi = base[0][:, None] + ii[None, :]
            gj = base[1][:, None] + jj[None, :]
            gk = base[2][:, None] + kk[None, :]
            out.append(off + gi + gdim[0] * (gj + gdim[1] * gk))
            off += self.nface[c]
        return np.concatenate(out, axis=1)

    def essential_mask(self, sides):
        """Boolean mask over RT dofs on the selected sides of the box."""
        P = self.p
        mask = np.zeros(self.n_u, dtype=bool)
        off = 0
        for c in range(3):
            gdim = [self.nx * P, self.ny * P, self.nz * P]
            gdim[c] += 1
            idx = np.arange(self.nface[c])
            coord = [idx % gdim[0], (idx // gdim[0]) % gdim[1], idx // (gdim[0] * gdim[1])]
            lo_bit = 1 << (2 * c)
            hi_bit = 1 << (2 * c + 1)
            m = np.zeros(self.nface[c], dtype=bool)
            if sides & lo_bit:
                m |= coord[c] == 0
            if sides & hi_bit:
                m |= coord[c] == gdim[c] - 1
            mask[off:off + self.nface[c]] = m
            off += self.nface[c]
        return mask


def constant_field_fluxes(mesh, u):
    """RT degrees of freedom of a constant vector field u on a box mesh whose
    vertices form a tensor grid (Cartesian, possibly non-uniform spacing).

    In the interpolation-histopolation basis a face dof is the flux of the
    field through its sub-element face (the histopolation conditions in the
    two tangential directions, Section 2.1), oriented along +axis.  On an
    axis-aligned cell of widths (hx, hy, hz) the x-normal sub-face
    (i, j, k) has area hy (xi_{j+1} - xi_j) hz (xi_{k+1} - xi_k), with xi
    the Gauss-Lobatto sub-element vertices on [0, 1]."""
    from .basis import gauss_lobatto_points
    P = mesh.p
    V = mesh.vertices.reshape(mesh.nz + 1, mesh.ny + 1, mesh.nx + 1, 3)
    xs, ys, zs = V[0, 0, :, 0], V[0, :, 0, 1], V[:, 0, 0, 2]
    grid = np.stack(np.meshgrid(zs, ys, xs, indexing='ij')[::-1], axis=-1)
    assert np.allclose(V, grid, rtol=0, atol=1e-12 * max(1.0, np.abs(V).max())), "tensor grid required"
    dxi = np.diff(gauss_lobatto_points(P))

    def sub_widths(coord):
        # widths of the refined intervals along one axis: cell width x dxi
        return (np.diff(coord)[:, None] * dxi[None, :]).ravel()

    w = [sub_widths(xs), sub_widths(ys), sub_widths(zs)]
    out = []
    for c in range(3):
        t = [d for d in range(3) if d != c]
        # refined face grid: extent n_c P + 1 along c, n_d P along the others
        area = np.outer(w[t[1]], w[t[0]])   # [k-like, j-like] for first index fastest
        n_c = len(w[c]) + 1
        if c == 0:
            blk = np.broadcast_to(area[:, :, None], (len(w[2]), len(w[1]), n_c))
        elif c == 1:
            blk = np.broadcast_to(area[:, None, :], (len(w[2]), n_c, len(w[0])))
        else:
            blk = np.broadcast_to(area[None, :, :], (n_c, len(w[1]), len(w[0])))
        out.append(u[c] * blk.ravel())
    return np.concatenate(out)


def divergence_algorithm1(mesh):
    """The discrete divergence D in CSR form following Algorithm 1.

    One row per L2 dof i (sub-element volume), 2d = 6 nonzeros per row, row
    pointer I[i] = 2 d i.  For each of the 6 faces k of the volume the local RT
    dof comes from a volume-to-face table, its global index from the
    element's local-to-global map, and the value is the product of the local
    orientation and the global orientation.

    Reading: the printed listing indexes the local orientation by the local
    face dof alone; the sign of a face relative to a volume depends on whether
    it is the volume's lower or upper face, so here the table is indexed by
    (face slot k, volume) -- -1 for the lower and +1 for the upper face in
    each direction, which is the sign of l_i' = h_{i-1} - h_i.
    """
    P = mesh.p
    d = 3
    N = mesh.n_q
    nl = P ** 3
    shapes = rt_shapes(P)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in shapes])
    # volume_to_face[k, i_loc] and local_orientation[k, i_loc]
    volume_to_face = np.zeros((2 * d, nl), dtype=np.int64)
    local_orientation = np.zeros((2 * d, nl))
    for i_loc in range(nl):
        loc = [i_loc % P, (i_loc // P) % P, i_loc // (P * P)]
        for comp in range(3):
            s = shapes[comp]
            for t, (shift, sign) in enumerate(((0, -1.0), (1, +1.0))):
                idx = list(loc)
                idx[comp] += shift
                k = 2 * comp + t
                volume_to_face[k, i_loc] = offs[comp] + idx[0] + s[0] * (idx[1] + s[1] * idx[2])
                local_orientation[k, i_loc] = sign
    rt_l2g = mesh.rt_local_to_global()
    global_orientation = np.ones(mesh.n_u)
    element_map = np.arange(N) // nl
    l2_global_to_local = np.arange(N) % nl
    I = 2 * d * np.arange(N + 1)
    J = np.zeros(2 * d * N, dtype=np.int64)
    A = np.zeros(2 * d * N)
    for k in range(2 * d):
        j_loc = volume_to_face[k, l2_global_to_local]
        s_loc = local_orientation[k, l2_global_to_local]
        j = rt_l2g[element_map, j_loc]
        J[2 * d * np.arange(N) + k] = j
        A[2 * d * np.arange(N) + k] = s_loc * global_orientation[j]
    return sp.csr_matrix((A, J, I), shape=(N, mesh.n_u))


def gamma_at_quadrature(mesh, gamma_vertices, Xq):
    """gamma at the reference points Xq [Q, 3] of every element, by trilinear
    interpolation of the element's 8 vertex values (the reference map's own
    shape functions).  Returns [E, Q]."""
    g = np.asarray(gamma_vertices, dtype=np.float64).reshape(-1)
    assert g.size == (mesh.nx + 1) * (mesh.ny + 1) * (mesh.nz + 1)
    ex, ey, ez = mesh.element_coords(np.arange(mesh.ne))
    out = np.zeros((mesh.ne, Xq.shape[0]))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                v = (ex + dx) + (mesh.nx + 1) * ((ey + dy) + (mesh.ny + 1) * (ez + dz))
                N = ((Xq[:, 0] if dx else 1.0 - Xq[:, 0]) * (Xq[:, 1] if dy else 1.0 - Xq[:, 1]) *
                     (Xq[:, 2] if dz else 1.0 - Xq[:, 2]))
                out += g[v][:, None] * N[None, :]
    return out


class Problem:
    """Assembled matrices of one problem instance (dense per element, sparse
    globally).  Intended for the small meshes the oracle handles."""

    def __init__(self, mesh, problem, c_mass, c_22=None, ess_sides=0, ref=None, gamma_vertices=None):
        self.mesh = mesh
        self.problem = problem
        ne = mesh.ne
        self.c_mass = np.asarray(c_mass, dtype=np.float64).reshape(ne)
        if c_22 is None:
            c_22 = np.zeros(ne)
        self.c_22 = np.asarray(c_22, dtype=np.float64).reshape(ne)
        if problem == GRADDIV:
            self.kappa = 1.0 / self.c_22
        else:
            self.kappa = self.c_22.copy()
        self.ref = RefElement(mesh.p) if ref is None else ref
        self.ess = mesh.essential_mask(ess_sides)
        V = mesh.element_vertices()
        em = element_matrices(mesh.p, V, self.c_mass, self.ref)
        self.Me, self.We, self.Be = em['M'], em['W'], em['B']
        self.detJ = em['detJ']
        self.gamma_field = gamma_vertices is not None
        if self.gamma_field:
            if problem != DARCY:
                raise ValueError("a gamma field is a Darcy coefficient")
            self.gamma_q = gamma_at_quadrature(mesh, gamma_vertices, self.ref.Xq)
            wd = self.ref.wq[None, :] / self.detJ
            psi = self.ref.psi
            self.Wge = np.einsum('eq,qa,qb->eab', self.gamma_q * wd, psi, psi)
            self.kappa = np.ones(ne)
        self.l2g = mesh.rt_local_to_global()
        self._assemble()

    def _assemble(self):
        mesh = self.mesh
        ne, nrt, nl = mesh.ne, n_rt(mesh.p), n_l2(mesh.p)
        rows = np.repeat(self.l2g, nrt, axis=1).ravel()
        cols = np.tile(self.l2g, (1, nrt)).ravel()
        self.M = sp.csr_matrix((self.Me.reshape(ne, -1).ravel(), (rows, cols)), shape=(mesh.n_u, mesh.n_u))
        qrow = (np.arange(ne)[:, None] * nl + np.arange(nl)[None, :])
        r2 = np.repeat(qrow, nl, axis=1).ravel()
        c2 = np.tile(qrow, (1, nl)).ravel()
        self.W = sp.csr_matrix((self.We.reshape(ne, -1).ravel(), (r2, c2)), shape=(mesh.n_q, mesh.n_q))
        rb = np.repeat(qrow, nrt, axis=1).ravel()
        cb = np.tile(self.l2g, (1, nl)).ravel()
        self.B = sp.csr_matrix((self.Be.reshape(ne, -1).ravel(), (rb, cb)), shape=(mesh.n_q, mesh.n_u))
        self.D = divergence_algorithm1(mesh)
        # C = blockdiag(kappa_e W_e^{-1}) via per-element inverses (dense, small);
        # with a gamma field blockdiag(W_e^{-1} W_gamma,e W_e^{-1})
        Winv = np.linalg.inv(self.We)
        if self.gamma_field:
            Cblocks = Winv @ self.Wge @ Winv
            self.Wg = sp.csr_matrix((self.Wge.reshape(ne, -1).ravel(), (r2, c2)), shape=(mesh.n_q, mesh.n_q))
        else:
            Cblocks = self.kappa[:, None, None] * Winv
        self.C = sp.csr_matrix((Cblocks.reshape(ne, -1).ravel(), (r2, c2)), shape=(mesh.n_q, mesh.n_q))

    # ---- operator ------------------------------------------------------
    def block_matrix(self, with_essential=True):
        """The transformed saddle-point matrix [[M, D^T], [D, -C]] as CSR; with
        essential rows/columns replaced by identity when requested."""
        A = sp.bmat([[self.M, self.D.T], [self.D, -self.C]], format='csr')
        if with_essential and self.ess.any():
            n = self.mesh.n
            keep = np.ones(n)
            keep[:self.mesh.n_u][self.ess] = 0.0
            K = sp.diags(keep)
            A = (K @ A @ K + sp.diags(1.0 - keep)).tocsr()
        return A

    def apply(self, x):
        """y = A x with the essential convention of the library: essential
        inputs are ignored and essential outputs copy the input."""
        x = np.asarray(x, dtype=np.float64)
        nu = self.mesh.n_u
        xu = x[:nu].copy()
        xu[self.ess] = 0.0
        xq = x[nu:]
        yu = self.M @ xu + self.D.T @ xq
        yq = self.D @ xu - self.C @ xq
        yu[self.ess] = x[:nu][self.ess]
        return np.concatenate([yu, yq])

    def mass_inverse(self, xq):
        """C xq = kappa_e W_e^{-1} xq (the (2,2) block without the sign)."""
        return self.C @ xq

    def lift_essential(self, b, u_bc):
        """Right-hand side of the system with identity essential rows:
        b_f - (A [u_bc; 0])_f on free rows, u_bc on essential rows."""
        nu = self.mesh.n_u
        ub = np.zeros(self.mesh.n)
        ub[:nu][self.ess] = u_bc[self.ess]
        A = self.block_matrix(with_essential=False)
        out = b - A @ ub
        out[:nu][self.ess] = u_bc[self.ess]
        return out


def apply_element_rows(mesh, problem, c_mass, c_22, ess_sides, x, elems):
    """Rows of y = A x at the dofs of the listed elements, computed from
    element matrices only (for sampled checks on meshes too large to
    assemble): every L2 row of the elements and every RT row of theirs.

    An RT dof on a face shared with a neighbour is a sum over both elements
    (M = sum_e E_e^T M_e E_e and D^T likewise, Section 3 eq.
    transformed-saddle-point), so the face neighbours' matrices are formed
    too.  Essential rows copy the input, as in `Problem.apply`.  Returns
    (q_rows, y_q, u_rows, y_u), rows in increasing order."""
    from .element import element_matrices, reference_divergence
    elems = np.unique(np.asarray(elems, dtype=np.int64))
    p = mesh.p
    nl = p ** 3
    nu = mesh.n_u
    # the sampled elements and their face neighbours
    ex, ey, ez = mesh.element_coords(elems)
    work = [elems]
    for coord, n, stride in ((ex, mesh.nx, 1), (ey, mesh.ny, mesh.nx), (ez, mesh.nz, mesh.nx * mesh.ny)):
        work.append(elems[coord > 0] - stride)
        work.append(elems[coord < n - 1] + stride)
    work = np.unique(np.concatenate(work))
    V = mesh.element_vertices(work)
    em = element_matrices(p, V, np.asarray(c_mass)[work])
    if problem == GRADDIV:
        kap = 1.0 / np.asarray(c_22)[work]
    else:
        kap = np.zeros(len(work)) if c_22 is None else np.asarray(c_22)[work]
    l2g = mesh.rt_local_to_global(work)
    ess = mesh.essential_mask(ess_sides)
    D = reference_divergence(p)
    yu_e = np.zeros((len(work), l2g.shape[1]))
    q_rows, y_q = [], []
    sampled = np.isin(work, elems)
    for n, e in enumerate(work):
        xu = x[l2g[n]].copy()
        xu[ess[l2g[n]]] = 0.0
        xq = x[nu + e * nl: nu + (e + 1) * nl]
        yu_e[n] = em['M'][n] @ xu + D.T @ xq
        if sampled[n]:
            q_rows.append(nu + e * nl + np.arange(nl))
            y_q.append(D @ xu - kap[n] * np.linalg.solve(em['W'][n], xq))
    # sum the element contributions per global RT dof
    rows_all, inv = np.unique(l2g.ravel(), return_inverse=True)
    acc = np.zeros(len(rows_all))
    np.add.at(acc, inv, yu_e.ravel())
    u_rows = np.unique(l2g[sampled].ravel())
    y_u = acc[np.searchsorted(rows_all, u_rows)]
    y_u[ess[u_rows]] = x[u_rows][ess[u_rows]]
    return np.concatenate(q_rows), np.concatenate(y_q), u_rows, y_u
