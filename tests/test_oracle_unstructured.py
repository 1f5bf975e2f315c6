"""Pins of the unstructured-mesh oracle (Section 3.2, Algorithm 1 with real
index arrays and orientation signs; Section 2.1 for the +-1 divergence):

* a structured mesh whose vertices and elements are renumbered and whose
  elements are turned by random rotations of the reference cube is the same
  discrete problem: its operator equals the structured oracle's up to a
  signed permutation, found here by matching sub-face centres and flux
  directions in physical space (independent of either numbering);
* W^{-1} B is the signed +-1 incidence D of Algorithm 1, also on an O-grid
  mesh with vertices of valence 3 in the cross section;
* the divergence theorem per element and over the domain;
* the Schur identity M + D^T W_alpha D = the grad-div matrix assembled from
  element quadrature, and the saddle-point solution equal to the primal one.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assemble, element, unstructured as un
from oracle.basis import gauss_lobatto_points
from paper_2304_12387_amd import inputs


def _structured_signatures(sm):
    """Centre and flux normal of every RT dof of the structured oracle (global
    normal +axis: the element's J_{c+1} x J_{c+2}), and the L2 sub-volume
    centres."""
    P = sm.p
    xi = gauss_lobatto_points(P)
    mid = 0.5 * (xi[:-1] + xi[1:])
    pts, comps = [], []
    for c, shp in enumerate(element.rt_shapes(P)):
        for i2 in range(shp[2]):
            for i1 in range(shp[1]):
                for i0 in range(shp[0]):
                    idx = (i0, i1, i2)
                    pts.append([mid[idx[d]] if d != c else xi[idx[d]] for d in range(3)])
                    comps.append(c)
    pts, comps = np.array(pts), np.array(comps)
    V = sm.element_vertices()
    x, J = element.trilinear(V, pts)
    l2g = sm.rt_local_to_global()
    cen = np.zeros((sm.n_u, 3))
    dirs = np.zeros((sm.n_u, 3))
    for e in range(sm.ne):
        cen[l2g[e]] = x[e]
        a_, b_ = J[e, np.arange(len(comps)), :, (comps + 1) % 3], J[e, np.arange(len(comps)), :, (comps + 2) % 3]
        dirs[l2g[e]] = np.cross(a_, b_)
    c, b, a = np.meshgrid(mid, mid, mid, indexing='ij')
    xq, _ = element.trilinear(V, np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1))
    return cen, dirs, xq.reshape(-1, 3)


def _match(ca, cb, scale):
    """Index map a -> b of equal points (rounded coordinates)."""
    key = lambda c: tuple(np.round(c / scale, 8))
    lookup = {key(c): i for i, c in enumerate(cb)}
    assert len(lookup) == len(cb)
    return np.array([lookup[key(c)] for c in ca])


def _signed_permutation(m, sm):
    cu, du = un.rt_dof_signatures(m)
    cs, ds, qs = _structured_signatures(sm)
    qu = un.l2_dof_centres(m)
    pu = _match(cu, cs, 1.0)
    s = np.sign(np.einsum('ij,ij->i', du, ds[pu]))
    assert np.all(s != 0)
    # flux directions agree up to sign (parallel)
    cosang = np.abs(np.einsum('ij,ij->i', du, ds[pu])) / (np.linalg.norm(du, axis=1) * np.linalg.norm(ds[pu], axis=1))
    assert cosang.min() > 1 - 1e-12
    pq = _match(qu, qs, 1.0)
    perm = np.concatenate([pu, sm.n_u + pq])
    sign = np.concatenate([s, np.ones(len(pq))])
    n = sm.n
    return sp.csr_matrix((sign, (np.arange(n), perm)), shape=(n, n))


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("problem", [un.GRADDIV, un.DARCY])
def test_scrambled_structured_mesh_is_the_same_problem(p, problem):
    nx, ny, nz = 3, 2, 2
    seed = 10 * p + problem
    rng = np.random.default_rng(seed)
    V = inputs.jittered_vertices(nx, ny, nz, 0.1, seed)
    ne = nx * ny * nz
    c_mass = inputs.loguniform(ne, 1e-2, 1e2, rng)
    c_22 = inputs.loguniform(ne, 1e-2, 1e2, rng) if problem == un.GRADDIV else rng.uniform(0.5, 2.0, ne)
    sm = assemble.Mesh(nx, ny, nz, p, V)
    sprob = assemble.Problem(sm, problem, c_mass, c_22, 0)
    Vv, el = inputs.from_structured(nx, ny, nz, V)
    V2, el2, eperm = inputs.scramble(Vv, el, seed + 1)
    m = un.HexMesh(V2, el2, p)
    assert (m.sgn < 0).any(), "the rotations must flip some orientations"
    uprob = un.UnstructuredProblem(m, problem, c_mass[eperm], c_22[eperm])
    S = _signed_permutation(m, sm)
    A_s = sprob.block_matrix(with_essential=False)
    A_u = uprob.block_matrix(with_essential=False)
    diff = (A_u - S @ A_s @ S.T)
    assert abs(diff).max() <= 1e-12 * abs(A_s).max()


def _o_grid_problem(p, problem=un.GRADDIV, seed=3):
    V, el = inputs.o_grid(2, 1, 2, seed=seed)
    m = un.HexMesh(V, el, p)
    rng = np.random.default_rng(seed)
    c_mass = inputs.loguniform(m.ne, 1e-1, 1e1, rng)
    c_22 = inputs.loguniform(m.ne, 1e-1, 1e1, rng)
    return m, un.UnstructuredProblem(m, problem, c_mass, c_22), c_mass, c_22


def test_o_grid_is_unstructured():
    V, el = inputs.o_grid(2, 1, 2)
    m = un.HexMesh(V, el, 1)
    # vertices of the cross section with 3 (not 4) edges at the central block's corners
    counts = np.bincount(el[:, :4].ravel(), minlength=V.shape[0])
    assert (counts[counts > 0] == 3).any()
    assert m.boundary_face.sum() > 0 and (~m.boundary_face).sum() > 0


@pytest.mark.parametrize("p", [1, 2, 3])
def test_divergence_is_signed_incidence(p):
    for mesh_kind in ('o_grid', 'scrambled'):
        if mesh_kind == 'o_grid':
            m, prob, _, _ = _o_grid_problem(p)
        else:
            V = inputs.jittered_vertices(2, 2, 2, 0.1, 5)
            Vv, el = inputs.from_structured(2, 2, 2, V)
            V2, el2, _ = inputs.scramble(Vv, el, 9)
            m = un.HexMesh(V2, el2, p)
            prob = un.UnstructuredProblem(m, un.GRADDIV, np.ones(m.ne), np.ones(m.ne))
        Dq = np.linalg.solve(prob.W.toarray(), prob.B.toarray())
        D = prob.D.toarray()
        assert np.abs(Dq - D).max() <= 1e-11
        assert set(np.unique(D)) <= {-1.0, 0.0, 1.0}
        assert np.all((D != 0).sum(axis=1) == 6)
        # an interior face dof couples to exactly two sub-volumes, with opposite signs
        col_nnz = (D != 0).sum(axis=0)
        assert col_nnz.max() == 2 and np.all(D.sum(axis=0)[col_nnz == 2] == 0.0)


def test_divergence_theorem_per_element_and_globally():
    m, prob, _, _ = _o_grid_problem(2)
    P = m.p
    u = np.random.default_rng(1).uniform(-1, 1, m.n_u)
    Du = prob.D @ u
    per_elem = Du.reshape(m.ne, P ** 3).sum(axis=1)
    for e in range(m.ne):
        flux = 0.0
        for d in range(3):
            for s in (0, 1):
                f = m.ef[e, d, s]
                # outward flux: the element's local flux (+e_d) is sigma * global,
                # outward on side s = 1, inward on side s = 0
                flux += (2 * s - 1) * m.esig[e, d, s] * u[f * P * P:(f + 1) * P * P].sum()
        assert abs(per_elem[e] - flux) <= 1e-12 * max(1.0, abs(flux))
    # globally only the boundary faces remain
    total = 0.0
    for f in np.nonzero(m.boundary_face)[0]:
        (e, d, s), = m.face_elems[f]
        total += (2 * s - 1) * m.esig[e, d, s] * u[f * P * P:(f + 1) * P * P].sum()
    assert abs(Du.sum() - total) <= 1e-11


@pytest.mark.parametrize("p", [1, 2])
def test_schur_identity_and_primal_solution_on_o_grid(p):
    m, prob, c_mass, alpha = _o_grid_problem(p)
    ref = element.RefElement(p)
    V = m.element_vertices()
    _, J = element.trilinear(V, ref.Xq)
    det = np.linalg.det(J)
    # (alpha div u, div v) from element quadrature: div u = div_hat / det J
    G_e = np.einsum('eq,qa,qb->eab', ref.wq[None, :] / det, ref.div, ref.div) * alpha[:, None, None]
    sg = m.sgn
    Gs = G_e * sg[:, :, None] * sg[:, None, :]
    nrt = element.n_rt(p)
    rows = np.repeat(m.l2g, nrt, axis=1).ravel()
    cols = np.tile(m.l2g, (1, nrt)).ravel()
    G = sp.csr_matrix((Gs.reshape(m.ne, -1).ravel(), (rows, cols)), shape=(m.n_u, m.n_u))
    Walpha = sp.block_diag([alpha[e] * prob.We[e] for e in range(m.ne)], format='csr')
    lhs = prob.M + prob.D.T @ Walpha @ prob.D
    K = prob.M + G
    assert abs(lhs - K).max() <= 1e-11 * abs(K).max()
    # the saddle point system gives the primal solution
    f = np.random.default_rng(2).uniform(-1, 1, m.n_u)
    b = np.concatenate([f, np.zeros(m.n_q)])
    x = spla.spsolve(prob.block_matrix().tocsc(), b)
    u = spla.spsolve(K.tocsc(), f)
    assert np.linalg.norm(x[:m.n_u] - u) <= 1e-9 * np.linalg.norm(u)
