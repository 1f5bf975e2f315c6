"""Pins of the oracle preconditioner: Schur approximation, M-matrix property,
Propositions 1 and 2, and the aggregation AMG (Sections 2.2-2.4)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assemble, precond
from paper_2304_12387_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'propositions.json')))


def make(n=3, p=2, problem=0, ess=0, seed=1, cartesian=False):
    cfg = inputs.graddiv_jittered(n, p, seed_mesh=seed, seed_coef=seed + 10)
    V = inputs.box_vertices(n, n, n) if cartesian else cfg['vertices']
    m = assemble.Mesh(n, n, n, p, V)
    c22 = cfg['c_22'] if problem == 0 else None
    return assemble.Problem(m, problem, cfg['c_mass'], c22, ess_sides=ess)


@pytest.mark.parametrize("problem,ess", [(0, 0), (1, 0), (1, 63), (0, 5)])
def test_schur_formula_equals_triple_product(problem, ess):
    prob = make(problem=problem, ess=ess)
    S1 = precond.schur_by_formula(prob)
    S2 = precond.schur_by_product(prob)
    assert abs((S1 - S2).toarray()).max() <= 1e-15 * abs(S1).max()
    assert (S1 != S1.T).nnz == 0


@pytest.mark.parametrize("problem,ess", [(0, 0), (1, 0), (1, 63)])
def test_schur_is_m_matrix_and_graph_laplacian(problem, ess):
    """Prop. 4 and eq. (graph-laplacian): non-positive off-diagonal, positive
    diagonal, and S~ - C~ has row sums equal to the weights of the row's free
    boundary faces (zero for interior sub-volumes)."""
    prob = make(problem=problem, ess=ess)
    S = precond.schur_by_formula(prob).toarray()
    off = S - np.diag(np.diag(S))
    assert off.max() <= 0 and np.diag(S).min() > 0
    rs = S.sum(1) - precond.c_tilde(prob)
    Md = precond.diag_M(prob)
    D = prob.D.tocsr()
    bnd = prob.mesh.essential_mask(63) & ~prob.ess
    expect = np.array([sum(1.0 / Md[k] for k in D.indices[D.indptr[i]:D.indptr[i + 1]] if bnd[k])
                       for i in range(S.shape[0])])
    assert np.allclose(rs, expect, atol=1e-12 * abs(S).max())
    # at most 2d + 1 = 7 entries per row
    assert (np.count_nonzero(S, axis=1) <= 7).all()


def _prec_spectrum(prob, tau):
    A = prob.block_matrix().toarray()
    nu = prob.mesh.n_u
    M = A[:nu, :nu]
    Dm = A[nu:, :nu]
    C = -A[nu:, nu:]
    S = C + Dm @ np.linalg.solve(M, Dm.T)
    B = np.zeros_like(A)
    B[:nu, :nu] = tau * M
    B[nu:, nu:] = S
    return np.sort(np.linalg.eigvals(np.linalg.solve(B, A)).real)


@pytest.mark.parametrize("problem", [0, 1])
def test_prop1_interval(problem):
    g = GOLD['prop_diag_precond']
    prob = make(n=2, p=2, problem=problem)
    lam = _prec_spectrum(prob, 1.0)
    lo = (1 - np.sqrt(5)) / 2
    hi = (1 + np.sqrt(5)) / 2
    tol = 1e-9
    neg, pos = lam[lam < 0], lam[lam > 0]
    assert neg.min() >= -1 - tol and neg.max() <= lo + tol
    assert pos.min() >= 1 - tol and pos.max() <= hi + tol
    assert pos.max() / abs(lam).min() <= g['kappa_bound'] + 1e-3
    if problem == 1:   # C = 0: exactly three distinct eigenvalues
        for v in lam:
            assert min(abs(v - 1), abs(v - lo), abs(v - hi)) < 1e-8


@pytest.mark.parametrize("problem", [0, 1])
def test_prop2_interval(problem):
    g = GOLD['prop_scaled_precond']
    prob = make(n=2, p=2, problem=problem)
    lam = _prec_spectrum(prob, g['tau'])
    tol = 1e-9
    neg, pos = lam[lam < 0], lam[lam > 0]
    assert neg.min() >= -1 - tol and neg.max() <= -0.5 + tol
    assert pos.min() >= 0.5 - tol and pos.max() <= 1 + tol
    assert abs(lam).max() / abs(lam).min() <= g['kappa_bound'] + 1e-9


def test_splitmix64_reference_values():
    # published test vector of splitmix64 with seed 0: the first outputs of
    # the generator state advanced by the golden gamma
    assert precond.splitmix64(0) == 0xE220A8397B1DCDAF
    assert precond.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def _greedy_mis2(G, keys):
    """Brute force: visit nodes by decreasing key, keep a node when no kept
    node lies within graph distance 2 (breadth-first search)."""
    n = G.shape[0]
    G = G.tocsr()
    kept = np.zeros(n, dtype=bool)
    for v in np.argsort(-keys.astype(np.float64), kind='stable'):
        frontier, seen = {int(v)}, {int(v)}
        for _ in range(2):
            nxt = set()
            for u in frontier:
                nxt.update(int(w) for w in G.indices[G.indptr[u]:G.indptr[u + 1]])
            frontier = nxt - seen
            seen |= nxt
        if not any(kept[u] for u in seen):
            kept[v] = True
    return kept


def _check_aggregates(G, agg, nagg, roots):
    assert agg.min() == 0 and agg.max() == nagg - 1
    assert len(np.unique(agg)) == nagg == roots.sum()
    # each aggregate holds exactly one root and is connected by strong edges
    assert np.array_equal(np.sort(agg[roots]), np.arange(nagg))
    for a in range(nagg):
        members = np.nonzero(agg == a)[0]
        sub = G[members][:, members]
        ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
        assert ncomp == 1


@pytest.mark.parametrize("problem,ess", [(0, 0), (1, 63)])
def test_mis2_matches_greedy_and_aggregates_are_valid(problem, ess):
    prob = make(n=3, p=2, problem=problem, ess=ess)
    S = precond.schur_by_formula(prob)
    G = precond.strength_graph(S, 0.25)
    assert (G != G.T).nnz == 0
    roots = precond.mis2_roots(G)
    n = S.shape[0]
    h = precond.node_hash(n)
    keys = h * np.uint64(1 << 32) + np.arange(n, dtype=np.uint64)
    # exact ordering: sort on the two fields instead of a float cast
    order = np.lexsort((np.arange(n), h))[::-1]
    rank = np.empty(n)
    rank[order] = np.arange(n)[::-1]
    assert np.array_equal(roots, _greedy_mis2(G, rank))
    agg, nagg = precond.mis2_aggregate(G)
    _check_aggregates(G, agg, nagg, roots)


def test_mis2_on_a_path_graph():
    n = 40
    rows = np.arange(n - 1)
    G = sp.csr_matrix((np.ones(2 * (n - 1)), (np.r_[rows, rows + 1], np.r_[rows + 1, rows])), shape=(n, n))
    roots = precond.mis2_roots(G)
    r = np.nonzero(roots)[0]
    assert np.diff(r).min() >= 3                    # independent at distance 2
    gaps = np.diff(np.r_[-3, r, n + 2])
    assert gaps.max() <= 5 + 1                      # maximal: no 5 uncovered in a row
    agg, nagg = precond.mis2_aggregate(G)
    _check_aggregates(G, agg, nagg, roots)


@pytest.mark.parametrize("problem,ess,singular", [(0, 0, False), (1, 0, False), (1, 63, True)])
def test_vcycle_symmetric_positive(problem, ess, singular):
    prob = make(n=3, p=2, problem=problem, ess=ess)
    S = precond.schur_by_formula(prob)
    assert precond.schur_is_singular(prob) == singular
    amg = precond.AMG(S, max_coarse=20, singular=singular)
    assert amg.nlevels >= 3
    n = S.shape[0]
    # in the singular case the cycle acts on the complement of the constant
    Pi = np.eye(n) - np.ones((n, n)) / n if singular else np.eye(n)
    V = np.stack([amg.apply(e) for e in Pi], axis=1)
    assert abs(V - V.T).max() <= 1e-13 * abs(V).max()
    if singular:
        ev = np.linalg.eigvalsh(V)
        assert np.sum(ev < 1e-10 * ev.max()) == 1       # only the constant
        evs = np.linalg.eigvals(V @ S.toarray()).real
        evs = np.sort(evs)[1:]
        assert evs.min() > 0 and evs.max() <= 1 + 1e-10
    else:
        assert np.linalg.eigvalsh(V).min() > 0
        evs = np.linalg.eigvals(V @ S.toarray()).real
        assert evs.min() > 0 and evs.max() <= 1 + 1e-10


def test_prolongator_keeps_constants_for_zero_row_sums():
    prob = make(n=3, p=2, problem=1, ess=63)
    S = precond.schur_by_formula(prob)
    assert abs(S @ np.ones(S.shape[0])).max() < 1e-12 * abs(S).max()
    amg = precond.AMG(S, max_coarse=20, singular=True)
    for P in amg.P:
        assert np.allclose(P @ np.ones(P.shape[1]), 1.0, atol=1e-13)
    for A in amg.A:
        assert abs(A @ np.ones(A.shape[0])).max() < 1e-10 * abs(A).max()
