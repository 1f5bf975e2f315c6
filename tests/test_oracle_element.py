"""Pins of element matrices, assembly and the divergence (Sections 2 and 2.1,
eq. matrices, eq. transformed-system, Algorithm 1)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.integrate import quad

from oracle import basis, element, assemble
from paper_2304_12387_amd import inputs


def distorted_element(rng, amp=0.15):
    V = np.zeros((1, 2, 2, 2, 3))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                V[0, dz, dy, dx] = [dx, dy, dz]
    return V + rng.uniform(-amp, amp, size=V.shape)


@pytest.mark.parametrize("p", range(1, 5))
def test_divergence_is_pm1_incidence_on_distorted_elements(p):
    """W_e^{-1} B_e is the geometry-free +-1 incidence, two nonzeros per
    column inside the element, 2d = 6 per row (Section 2.1)."""
    rng = np.random.default_rng(100 + p)
    for _ in range(3):
        em = element.element_matrices(p, distorted_element(rng))
        D = np.linalg.solve(em['W'][0], em['B'][0])
        R = np.round(D)
        assert abs(D - R).max() < 1e-12
        assert set(np.unique(R)) <= {-1.0, 0.0, 1.0}
        assert np.all((R != 0).sum(1) == 6)
        assert np.all((R != 0).sum(0) <= 2)
        assert np.array_equal(R, element.reference_divergence(p))


def one_d_mass(f, g, n):
    return np.array([[quad(lambda t: f(t)[0, i] * g(t)[0, j], 0, 1, epsabs=1e-14)[0]
                      for j in range(n)] for i in range(n)])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_kronecker_structure_on_a_box(p):
    hx, hy, hz = 0.7, 1.3, 0.4
    V = np.zeros((1, 2, 2, 2, 3))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                V[0, dz, dy, dx] = [dx * hx, dy * hy, dz * hz]
    em = element.element_matrices(p, V)
    xi = basis.gauss_lobatto_points(p)
    Ml = one_d_mass(lambda t: basis.lagrange(xi, t), lambda t: basis.lagrange(xi, t), p + 1)
    Mh = one_d_mass(lambda t: basis.histopolation(xi, t), lambda t: basis.histopolation(xi, t), p)
    n1 = p * p * (p + 1)
    M = em['M'][0]
    Mxx = (hx / (hy * hz)) * np.kron(np.kron(Mh, Mh), Ml)
    Myy = (hy / (hx * hz)) * np.kron(np.kron(Mh, Ml), Mh)
    Mzz = (hz / (hx * hy)) * np.kron(np.kron(Ml, Mh), Mh)
    assert np.allclose(M[:n1, :n1], Mxx, atol=1e-12)
    assert np.allclose(M[n1:2 * n1, n1:2 * n1], Myy, atol=1e-12)
    assert np.allclose(M[2 * n1:, 2 * n1:], Mzz, atol=1e-12)
    assert abs(M[:n1, n1:]).max() < 1e-13 and abs(M[n1:2 * n1, 2 * n1:]).max() < 1e-13
    W = em['W'][0]
    assert np.allclose(W, np.kron(np.kron(Mh, Mh), Mh) / (hx * hy * hz), atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_element_mass_spd(p):
    em = element.element_matrices(p, distorted_element(np.random.default_rng(7)))
    M = em['M'][0]
    assert np.allclose(M, M.T, atol=1e-14)
    assert np.linalg.eigvalsh(M).min() > 0


def test_divergence_of_subvolumes_by_quadrature():
    """D u equals the integrals of div u_h over the physical sub-volumes
    (W_h = div V_h), computed by quadrature of the Piola-mapped field."""
    p = 3
    rng = np.random.default_rng(3)
    V = distorted_element(rng, 0.1)
    u = rng.standard_normal(element.n_rt(p))
    D = element.reference_divergence(p)
    xi = basis.gauss_lobatto_points(p)
    xg, wg = basis.gauss_legendre(p + 2)
    got = np.zeros(p ** 3)
    for c in range(p):
        for b in range(p):
            for a in range(p):
                lo = np.array([xi[a], xi[b], xi[c]])
                hi = np.array([xi[a + 1], xi[b + 1], xi[c + 1]])
                X = lo + element.tensor_points(xg) * (hi - lo)
                w = element.tensor_weights(wg) * np.prod(hi - lo)
                _, J = element.trilinear(V, X)
                det = np.linalg.det(J)[0]
                _, dv = element.rt_reference(p, X)
                div_phys = (dv @ u) / det            # div u = div_hat u_hat / det J
                got[a + p * (b + p * c)] = np.sum(w * det * div_phys)
    assert np.allclose(got, D @ u, atol=1e-12)


def small_problem(n=3, p=2, problem=0, ess=0, seed=1):
    cfg = inputs.graddiv_jittered(n, p, seed_mesh=seed, seed_coef=seed + 10)
    m = assemble.Mesh(n, n, n, p, cfg['vertices'])
    c22 = cfg['c_22'] if problem == 0 else None
    return assemble.Problem(m, problem, cfg['c_mass'], c22, ess_sides=ess)


def test_algorithm1_matches_assembled_w_inverse_b():
    prob = small_problem()
    Winv = sp.csr_matrix(np.linalg.inv(prob.W.toarray()))
    assert abs((Winv @ prob.B - prob.D).toarray()).max() < 1e-12
    D = prob.D.tocsc()
    colnnz = np.diff(D.indptr)
    assert colnnz.max() == 2 and colnnz.min() == 1
    inner = colnnz == 2
    sums = np.asarray(D.sum(axis=0)).ravel()
    assert np.all(sums[inner] == 0)


def test_global_divergence_theorem():
    """1^T D u over all sub-volumes equals the net outward flux through the
    boundary faces (interior faces cancel)."""
    prob = small_problem(n=3, p=3)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(prob.mesh.n_u)
    mesh = prob.mesh
    flux = 0.0
    off = 0
    for c in range(3):
        gdim = [mesh.nx * mesh.p, mesh.ny * mesh.p, mesh.nz * mesh.p]
        gdim[c] += 1
        idx = np.arange(mesh.nface[c])
        coord = [idx % gdim[0], (idx // gdim[0]) % gdim[1], idx // (gdim[0] * gdim[1])]
        uc = u[off:off + mesh.nface[c]]
        flux += uc[coord[c] == gdim[c] - 1].sum() - uc[coord[c] == 0].sum()
        off += mesh.nface[c]
    assert abs((prob.D @ u).sum() - flux) < 1e-10


def test_schur_wrt_22_block_is_graddiv_matrix():
    """M_beta + D^T W_alpha D equals the grad-div matrix (alpha div u, div v) +
    (beta u, v) assembled independently (Section 2, remark after eq. matrices)."""
    prob = small_problem(n=2, p=3)
    mesh, ref = prob.mesh, prob.ref
    V = mesh.element_vertices()
    _, J = element.trilinear(V, ref.Xq)
    det = np.linalg.det(J)
    alpha = prob.c_22
    K = np.einsum('eq,qa,qb->eab', ref.wq[None] / det * alpha[:, None], ref.div, ref.div)
    nrt = element.n_rt(mesh.p)
    rows = np.repeat(prob.l2g, nrt, axis=1).ravel()
    cols = np.tile(prob.l2g, (1, nrt)).ravel()
    A = sp.csr_matrix((K.reshape(mesh.ne, -1).ravel(), (rows, cols)), shape=(mesh.n_u, mesh.n_u)) + prob.M
    Wa = sp.diags(np.repeat(alpha, mesh.p ** 3)) @ prob.W
    S = prob.M + prob.D.T @ Wa @ prob.D
    assert abs((S - A).toarray()).max() < 1e-13 * abs(A).max()
    # and the transformed system is congruent to the untransformed one
    Wainv = np.linalg.inv(Wa.toarray())
    Bal = Wa @ prob.D
    top = np.hstack([prob.M.toarray(), Bal.T.toarray()])
    bot = np.hstack([Bal.toarray(), -Wa.toarray()])
    Aun = np.vstack([top, bot])
    T = np.eye(mesh.n)
    T[mesh.n_u:, mesh.n_u:] = Wainv
    assert np.allclose(T @ Aun @ T, prob.block_matrix().toarray(), atol=1e-10 * abs(Aun).max())


def test_piecewise_constant_gamma_block():
    """W^{-1} W_gamma W^{-1} = W_{1/gamma}^{-1} for element-wise constant gamma
    (Section 2.4), with W_gamma assembled by quadrature of gamma psi psi."""
    prob = small_problem(n=2, p=2, problem=1)
    mesh, ref = prob.mesh, prob.ref
    gam = np.random.default_rng(9).uniform(0.5, 3.0, mesh.ne)
    _, J = element.trilinear(mesh.element_vertices(), ref.Xq)
    det = np.linalg.det(J)
    Wg = np.einsum('eq,qa,qb->eab', ref.wq[None] / det * gam[:, None], ref.psi, ref.psi)
    Wi = np.linalg.inv(prob.We)
    lhs = Wi @ Wg @ Wi
    rhs = np.linalg.inv(prob.We / gam[:, None, None])
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-11 * abs(rhs).max())


@pytest.mark.parametrize("p", [2, 3, 4])
def test_gauss_legendre_mass_is_diagonal_on_parallelepipeds(p):
    """In the nodal basis at the p Gauss-Legendre points the L2 mass matrix of
    an affine (parallelepiped) element is diagonal (Section 2.5)."""
    rng = np.random.default_rng(p)
    A = np.eye(3) + rng.uniform(-0.3, 0.3, (3, 3))
    V = np.zeros((1, 2, 2, 2, 3))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                V[0, dz, dy, dx] = A @ np.array([dx, dy, dz], float)
    ref = element.RefElement(p)
    g, _ = basis.gauss_legendre(p)
    Lg = basis.lagrange(g, ref.t.xq)
    Bg = np.einsum('ai,bj,ck->cbakji', Lg, Lg, Lg).reshape(ref.nq ** 3, p ** 3)
    _, J = element.trilinear(V, ref.Xq)
    det = np.linalg.det(J)[0]
    Wgl = np.einsum('q,qa,qb->ab', ref.wq / det, Bg, Bg)
    off = Wgl - np.diag(np.diag(Wgl))
    assert abs(off).max() < 1e-14 * abs(Wgl).max()


def test_essential_mask_counts():
    m = assemble.Mesh(3, 4, 5, 2, inputs.box_vertices(3, 4, 5))
    mask = m.essential_mask(63)
    P = 2
    expected = 2 * (4 * P) * (5 * P) + 2 * (3 * P) * (5 * P) + 2 * (3 * P) * (4 * P)
    assert mask.sum() == expected
    assert m.essential_mask(1).sum() == (4 * P) * (5 * P)
