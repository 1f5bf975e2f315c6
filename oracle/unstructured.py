"""Unstructured hexahedral meshes: face orientation, RT/L2 numbering,
Algorithm 1 with real index arrays, and the transformed operator.  Test
infrastructure.

Section 3.2 builds the discrete divergence D from element-to-dof index arrays
and the product of a local and a global orientation sign (Algorithm 1);
Section 4.1 runs on an unstructured hexahedral mesh.  This module is the
plain CPU form of that general case.

Mesh: vertex coordinates [nv, 3] and, per element, its 8 vertex numbers in the
reference order v = dx + 2 dy + 4 dz (the trilinear map of `element.trilinear`
with V[dz, dy, dx]).  Every element must map with det J > 0.

Faces are identified by their 4 vertex numbers.  Local face (d, s) of an
element is its side x_d = s of the reference cube, with tangential axes
(t0, t1) = the other two axes in increasing order.  A global face carries a
canonical frame fixed by the global vertex numbers alone, so both elements
of an interior face agree on it:
  origin  the face vertex with the smallest number,
  a1      towards the smaller-numbered of the origin's two face neighbours,
  a2      towards the other neighbour,
  normal  a1 x a2.
The global RT dof of a sub-face is the flux through it along the global
normal (sigma_glob); an element's local face dof is the flux along its
reference +e_d, so local = sigma(e, f) * global with sigma(e, f) = +1 when
a1 x a2 (taken in the element's reference coordinates, where the map is
orientation preserving) points along +e_d, and -1 otherwise.  Sub-face
(j, k) of the element (indices along t0, t1 over the Gauss-Lobatto
sub-intervals) is sub-face (j', k') of the canonical frame, j' along a1 and
k' along a2, an index reversed when its axis runs against the element's
(the Gauss-Lobatto points are symmetric about 1/2, so the sub-face grids of
the two elements coincide).

Global RT numbering: all face dofs, face by face (p^2 each, j' fastest),
then the interior dofs element by element (3 (p-1) p^2 each: component-major,
the normal index 1..p-1 fastest, then t0, then t1), sign +1.  Global L2
numbering: element-major as on structured meshes.
"""
import numpy as np
import scipy.sparse as sp

from .basis import gauss_lobatto_points
from .element import RefElement, element_matrices, n_l2, n_rt, rt_shapes, trilinear

GRADDIV = 0
DARCY = 1

# reference coordinates of the 8 element vertices, v = dx + 2 dy + 4 dz
REF_VERTS = np.array([[v & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], dtype=np.int64)


def _tangential(d):
    return [a for a in range(3) if a != d]


class HexMesh:
    def __init__(self, vertices, elements, p):
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        self.elements = np.asarray(elements, dtype=np.int64).reshape(-1, 8)
        self.p = int(p)
        self.ne = self.elements.shape[0]
        self._faces()
        self._numbering()

    def element_vertices(self, elems=None):
        """[E, 2, 2, 2, 3] indexed [dz, dy, dx, :]."""
        if elems is None:
            elems = np.arange(self.ne)
        V = self.vertices[self.elements[np.asarray(elems)]]          # [E, 8, 3], v = dx + 2dy + 4dz
        return V.reshape(-1, 2, 2, 2, 3)

    # ---- faces and their canonical frames ---------------------------------
    def _faces(self):
        """Global faces, and per element and local face (d, s): the global
        face, sigma, and the map of local sub-face indices to canonical ones."""
        keys = {}
        self.face_verts = []        # global vertex numbers of each face (4)
        self.face_elems = []        # [(element, d, s)]
        self.ef = np.zeros((self.ne, 3, 2), dtype=np.int64)
        self.esig = np.zeros((self.ne, 3, 2), dtype=np.int64)
        # how (j_loc, k_loc) map to (j', k'): for each canonical axis, which
        # local index feeds it (0: j along t0, 1: k along t1) and whether it
        # is reversed
        self.emap = np.zeros((self.ne, 3, 2, 2, 2), dtype=np.int64)
        for e in range(self.ne):
            gv = self.elements[e]
            for d in range(3):
                t0, t1 = _tangential(d)
                for s in (0, 1):
                    loc = [v for v in range(8) if REF_VERTS[v, d] == s]
                    key = tuple(sorted(gv[loc]))
                    if key not in keys:
                        keys[key] = len(self.face_verts)
                        self.face_verts.append(key)
                        self.face_elems.append([])
                    f = keys[key]
                    self.face_elems[f].append((e, d, s))
                    self.ef[e, d, s] = f
                    # canonical frame in the element's reference coordinates
                    o = min(loc, key=lambda v: gv[v])
                    nbrs = [v for v in loc if np.abs(REF_VERTS[v] - REF_VERTS[o]).sum() == 1]
                    v1, v2 = sorted(nbrs, key=lambda v: gv[v])
                    a1 = REF_VERTS[v1] - REF_VERTS[o]
                    a2 = REF_VERTS[v2] - REF_VERTS[o]
                    n = np.cross(a1, a2)
                    self.esig[e, d, s] = 1 if n[d] > 0 else -1
                    for ax, a in enumerate((a1, a2)):
                        src = 0 if a[t0] != 0 else 1
                        tt = t0 if src == 0 else t1
                        self.emap[e, d, s, ax] = (src, 1 if a[tt] < 0 else 0)
        self.nfaces = len(self.face_verts)
        self.boundary_face = np.array([len(x) == 1 for x in self.face_elems])
        for f, el in enumerate(self.face_elems):
            if len(el) > 2:
                raise ValueError("a face shared by more than two elements")

    # ---- dof numbering -------------------------------------------------------
    def _numbering(self):
        P = self.p
        self.n_face_dofs = self.nfaces * P * P
        self.n_int_per_elem = 3 * (P - 1) * P * P
        self.n_u = self.n_face_dofs + self.ne * self.n_int_per_elem
        self.n_q = self.ne * P ** 3
        self.n = self.n_u + self.n_q
        nrt = n_rt(P)
        self.l2g = np.zeros((self.ne, nrt), dtype=np.int64)
        self.sgn = np.ones((self.ne, nrt))
        shapes = rt_shapes(P)
        for e in range(self.ne):
            off = 0
            for c, shp in enumerate(shapes):
                t0, t1 = _tangential(c)
                for i2 in range(shp[2]):
                    for i1 in range(shp[1]):
                        for i0 in range(shp[0]):
                            idx = (i0, i1, i2)
                            li = off + i0 + shp[0] * (i1 + shp[1] * i2)
                            ic, j, k = idx[c], idx[t0], idx[t1]
                            if ic == 0 or ic == P:
                                s = 0 if ic == 0 else 1
                                f = self.ef[e, c, s]
                                jk = (j, k)
                                canon = []
                                for ax in range(2):
                                    src, rev = self.emap[e, c, s, ax]
                                    v = jk[src]
                                    canon.append(P - 1 - v if rev else v)
                                self.l2g[e, li] = f * P * P + canon[0] + P * canon[1]
                                self.sgn[e, li] = self.esig[e, c, s]
                            else:
                                self.l2g[e, li] = (self.n_face_dofs + e * self.n_int_per_elem +
                                                   c * (P - 1) * P * P + (ic - 1) + (P - 1) * (j + P * k))
                off += int(np.prod(shp))

    def boundary_dof_mask(self, select=None):
        """Boolean mask over RT dofs on boundary faces; `select(centroid)`
        (optional) picks the boundary faces by their vertex centroid."""
        P = self.p
        mask = np.zeros(self.n_u, dtype=bool)
        for f in np.nonzero(self.boundary_face)[0]:
            if select is not None and not select(self.vertices[list(self.face_verts[f])].mean(axis=0)):
                continue
            mask[f * P * P:(f + 1) * P * P] = True
        return mask


def divergence_algorithm1(mesh):
    """D in CSR form by Algorithm 1: one row per sub-volume, 2d = 6 entries;
    the local RT dof of face slot k of the volume from a volume-to-face table,
    its global index from the element's index array, the value the product
    of the local orientation (-1 lower, +1 upper face of the volume; the
    reading of the listing's sign table taken on structured meshes too) and
    the global orientation sigma of that dof in the element."""
    P = mesh.p
    nl = P ** 3
    shapes = rt_shapes(P)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in shapes])
    vol2face = np.zeros((6, nl), dtype=np.int64)
    loc_or = np.zeros((6, nl))
    for il in range(nl):
        loc = [il % P, (il // P) % P, il // (P * P)]
        for comp in range(3):
            s = shapes[comp]
            for t, (shift, sign) in enumerate(((0, -1.0), (1, +1.0))):
                idx = list(loc)
                idx[comp] += shift
                k = 2 * comp + t
                vol2face[k, il] = offs[comp] + idx[0] + s[0] * (idx[1] + s[1] * idx[2])
                loc_or[k, il] = sign
    N = mesh.n_q
    element_map = np.arange(N) // nl
    g2l = np.arange(N) % nl
    I = 6 * np.arange(N + 1)
    J = np.zeros(6 * N, dtype=np.int64)
    A = np.zeros(6 * N)
    for k in range(6):
        jl = vol2face[k, g2l]
        J[6 * np.arange(N) + k] = mesh.l2g[element_map, jl]
        A[6 * np.arange(N) + k] = loc_or[k, g2l] * mesh.sgn[element_map, jl]
    return sp.csr_matrix((A, J, I), shape=(N, mesh.n_u))


class UnstructuredProblem:
    """Assembled transformed operator [[M, D^T], [D, -C]] on an unstructured
    mesh (grad-div: M = M_beta, C = W_alpha^{-1}; Darcy with piecewise-constant
    gamma: M = M_{1/eps}, C = gamma W^{-1}), essential dofs with identity rows
    and columns."""

    def __init__(self, mesh, problem, c_mass, c_22=None, ess=None):
        self.mesh = mesh
        P = mesh.p
        ne = mesh.ne
        self.c_mass = np.asarray(c_mass, dtype=np.float64).reshape(ne)
        c22 = np.zeros(ne) if c_22 is None else np.asarray(c_22, dtype=np.float64).reshape(ne)
        self.kappa = 1.0 / c22 if problem == GRADDIV else c22
        self.ess = np.zeros(mesh.n_u, dtype=bool) if ess is None else np.asarray(ess, dtype=bool)
        self.ref = RefElement(P)
        em = element_matrices(P, mesh.element_vertices(), self.c_mass, self.ref)
        self.Me, self.We, self.Be, self.detJ = em['M'], em['W'], em['B'], em['detJ']
        nrt, nl = n_rt(P), n_l2(P)
        l2g, sg = mesh.l2g, mesh.sgn
        Ms = self.Me * sg[:, :, None] * sg[:, None, :]
        rows = np.repeat(l2g, nrt, axis=1).ravel()
        cols = np.tile(l2g, (1, nrt)).ravel()
        self.M = sp.csr_matrix((Ms.reshape(ne, -1).ravel(), (rows, cols)), shape=(mesh.n_u, mesh.n_u))
        qrow = np.arange(ne)[:, None] * nl + np.arange(nl)[None, :]
        r2 = np.repeat(qrow, nl, axis=1).ravel()
        c2 = np.tile(qrow, (1, nl)).ravel()
        self.W = sp.csr_matrix((self.We.reshape(ne, -1).ravel(), (r2, c2)), shape=(mesh.n_q, mesh.n_q))
        Bs = self.Be * sg[:, None, :]
        rb = np.repeat(qrow, nrt, axis=1).ravel()
        cb = np.tile(l2g, (1, nl)).ravel()
        self.B = sp.csr_matrix((Bs.reshape(ne, -1).ravel(), (rb, cb)), shape=(mesh.n_q, mesh.n_u))
        self.D = divergence_algorithm1(mesh)
        Cb = self.kappa[:, None, None] * np.linalg.inv(self.We)
        self.C = sp.csr_matrix((Cb.reshape(ne, -1).ravel(), (r2, c2)), shape=(mesh.n_q, mesh.n_q))

    def block_matrix(self, with_essential=True):
        A = sp.bmat([[self.M, self.D.T], [self.D, -self.C]], format='csr')
        if with_essential and self.ess.any():
            keep = np.ones(self.mesh.n)
            keep[:self.mesh.n_u][self.ess] = 0.0
            K = sp.diags(keep)
            A = (K @ A @ K + sp.diags(1.0 - keep)).tocsr()
        return A

    def apply(self, x):
        x = np.asarray(x, dtype=np.float64)
        nu = self.mesh.n_u
        xu = x[:nu].copy()
        xu[self.ess] = 0.0
        xq = x[nu:]
        yu = self.M @ xu + self.D.T @ xq
        yq = self.D @ xu - self.C @ xq
        yu[self.ess] = x[:nu][self.ess]
        return np.concatenate([yu, yq])


# ---- geometric signatures (for checks) -----------------------------------------

def flux_normal(J, comps):
    """The normal a reference flux along +e_c has in physical space,
    J_{c+1} x J_{c+2} (cyclic), for J [n, 3, 3] and c = comps [n]: the same
    line from both elements of a face, since it only involves the face's
    tangent vectors."""
    a = J[np.arange(len(comps)), :, (comps + 1) % 3]
    b = J[np.arange(len(comps)), :, (comps + 2) % 3]
    return np.cross(a, b)


def rt_dof_signatures(mesh):
    """Per global RT dof: the physical centre of its sub-face and the
    physical normal along which it measures flux (the element's reference
    +e_c direction mapped as a normal, times its sign), from any element that
    holds it."""
    P = mesh.p
    xi = gauss_lobatto_points(P)
    mid = 0.5 * (xi[:-1] + xi[1:])
    shapes = rt_shapes(P)
    centre = np.zeros((mesh.n_u, 3))
    direc = np.zeros((mesh.n_u, 3))
    V = mesh.element_vertices()
    pts, comps = [], []
    for c, shp in enumerate(shapes):
        for i2 in range(shp[2]):
            for i1 in range(shp[1]):
                for i0 in range(shp[0]):
                    idx = (i0, i1, i2)
                    X = [mid[idx[d]] if d != c else xi[idx[d]] for d in range(3)]
                    pts.append(X)
                    comps.append(c)
    pts = np.array(pts)
    comps = np.array(comps)
    x, J = trilinear(V, pts)                          # [E, n, 3], [E, n, 3, 3]
    for e in range(mesh.ne):
        dirs = flux_normal(J[e], comps) * mesh.sgn[e][:, None]
        centre[mesh.l2g[e]] = x[e]
        direc[mesh.l2g[e]] = dirs
    return centre, direc


def l2_dof_centres(mesh):
    P = mesh.p
    xi = gauss_lobatto_points(P)
    mid = 0.5 * (xi[:-1] + xi[1:])
    c, b, a = np.meshgrid(mid, mid, mid, indexing='ij')
    X = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
    x, _ = trilinear(mesh.element_vertices(), X)
    return x.reshape(-1, 3)
