"""Block-diagonal preconditioner: diagonals, approximate Schur complement,
aggregation AMG.  Test infrastructure.

Section 2.3 (eq. approx-schur, eq. approx-schur-entries, Prop. 4 and 5),
Section 2.4 (Darcy: C~ = diag(W)^{-1} diag(W_gamma) diag(W)^{-1}), the remark
after Prop. 3 (relative block scaling tau), and Section 4.2 (singular Schur
complement under pure flux boundary conditions: remove the constant after
every Schur preconditioner application).

    B = diag(tau M~, S^)    M~ = diag(M)    S~ = C~ + D M~^{-1} D^T
    S^{-1} = one V-cycle of an aggregation AMG on S~.

The paper uses BoomerAMG for S^{-1}; here it is replaced by a smoothed
aggregation V(1,1)-cycle whose every choice is fixed here (and reproduced by
the GPU library), so that the two can be compared number by number:

* strength: an off-diagonal a_ij < 0 is strong when
  -a_ij >= theta * min(m_i, m_j), m_i = max_{k != i}(-a_ik)  (the classical
  row-relative test of either endpoint, theta = 0.25);
* aggregation: distance-2 maximal independent set on the strength graph with
  node keys (state, h(i), i), h = low 30 bits of splitmix64(i); roots seed
  aggregates numbered in index order; neighbours of roots join the root of
  largest key; the remaining nodes join the first-pass neighbour of largest
  key;
* tentative prolongator T = aggregate indicator (entries 1);
  P = (I - omega D_F^{-1} A_F) T with omega = 2/3 and A_F the strength-filtered
  matrix (weak entries added to the diagonal, so row sums are kept);
* Galerkin A_c = P^T A P, then symmetrised (A_c + A_c^T) / 2;
* stop at <= max_coarse rows or when a level no longer shrinks; the coarsest
  matrix is inverted densely (with s e e^T added when singular,
  s = trace/n_c^2);
* smoother: l1-Jacobi, D_l1 = sum_j |a_ij|, one sweep before (from zero) and
  one after the coarse correction, which keeps the cycle symmetric.
"""
import numpy as np
import scipy.sparse as sp

MASK64 = (1 << 64) - 1


def diag_M(prob):
    """M~ = diag(M) (free dofs); 1 on essential dofs (unused there)."""
    d = prob.M.diagonal().copy()
    d[prob.ess] = 1.0
    return d


def diag_W(prob):
    """diag of the unweighted L2 mass matrix, element by element."""
    return prob.W.diagonal().copy()


def c_tilde(prob):
    """C~_ii = kappa_e / W_ii (grad-div: diag(W_alpha)^{-1}; Darcy with
    piecewise-constant gamma: diag(W)^{-1} diag(W_gamma) diag(W)^{-1}); with a
    gamma field that product of diagonals itself (Section 2.4)."""
    if getattr(prob, 'gamma_field', False):
        w = diag_W(prob)
        return prob.Wg.diagonal() / (w * w)
    nl = prob.mesh.p ** 3
    kap = np.repeat(prob.kappa, nl)
    return kap / diag_W(prob)


def schur_by_formula(prob, Md=None):
    """S~ entry by entry from eq. (approx-schur-entries).  Md replaces
    diag(M) as M~ when given (the learned diagonal).

    Row i (sub-volume): diagonal C~_ii + sum over its free faces k of 1/M~_kk;
    off-diagonal -1/M~_kk for each neighbour j sharing the free face k.
    Faces are read from the rows of D (its columns list the sub-volumes that
    share a face)."""
    D = prob.D.tocsr()
    Dt = D.T.tocsr()
    Mt = diag_M(prob) if Md is None else Md
    Ct = c_tilde(prob)
    free = ~prob.ess
    n = D.shape[0]
    rows, cols, vals = [], [], []
    diag = Ct.copy()
    for i in range(n):
        for k in D.indices[D.indptr[i]:D.indptr[i + 1]]:
            if not free[k]:
                continue
            w = 1.0 / Mt[k]
            diag[i] += w
            for j in Dt.indices[Dt.indptr[k]:Dt.indptr[k + 1]]:
                if j != i:
                    rows.append(i)
                    cols.append(j)
                    vals.append(-w)
    rows.extend(range(n))
    cols.extend(range(n))
    vals.extend(diag)
    S = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    S.sum_duplicates()
    S.sort_indices()
    return S


def schur_by_product(prob):
    """S~ = C~ + D_f M~^{-1} D_f^T with D_f the divergence restricted to free
    RT dofs (sparse triple product, the paper's construction)."""
    Df = prob.D.tocsc().copy()
    Df = Df @ sp.diags((~prob.ess).astype(np.float64))
    S = sp.diags(c_tilde(prob)) + Df @ sp.diags(1.0 / diag_M(prob)) @ Df.T
    S = S.tocsr()
    S.sort_indices()
    return S


def schur_is_singular(prob):
    """S~ has the constant null vector when C~ = 0 and no boundary face is
    free (pure flux boundary conditions, Section 4.2)."""
    if getattr(prob, 'gamma_field', False):
        return not np.any(prob.gamma_q != 0)
    if np.any(prob.kappa != 0):
        return False
    return bool(prob.mesh.essential_mask(63).sum() == (prob.ess & prob.mesh.essential_mask(63)).sum())


# ------------------------------------------------------------------------
# aggregation AMG
# ------------------------------------------------------------------------

def splitmix64(x):
    x = (int(x) + 0x9E3779B97F4A7C15) & MASK64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def node_hash(n):
    return np.array([splitmix64(i) & 0x3FFFFFFF for i in range(n)], dtype=np.uint64)


def strength_graph(A, theta):
    """Symmetric strength pattern (CSR, no diagonal) of the matrix A."""
    A = A.tocsr()
    n = A.shape[0]
    r = np.repeat(np.arange(n), np.diff(A.indptr))
    c = A.indices
    v = A.data
    off = r != c
    # m_i = max(0, max_{k != i} -a_ik)
    m = np.zeros(n)
    np.maximum.at(m, r[off], -v[off])
    strong = off & (-v > 0) & (-v >= theta * np.minimum(m[r], m[c]))
    G = sp.csr_matrix((np.ones(strong.sum()), (r[strong], c[strong])), shape=(n, n))
    G.sort_indices()
    return G


def _rowmax(indptr, indices, key, self_key):
    out = self_key.copy()
    for i in range(len(indptr) - 1):
        seg = indices[indptr[i]:indptr[i + 1]]
        if seg.size:
            mx = key[seg].max()
            if mx > out[i]:
                out[i] = mx
    return out


def mis2_roots(G):
    """Distance-2 maximal independent set on the strength graph G (CSR,
    symmetric, no diagonal).  Node keys are (state, h(i), i) with the states
    OUT < UNDECIDED < IN; each round an undecided node whose key is the
    largest within distance 2 joins the set, and an undecided node with a set
    member within distance 2 leaves.  Returns a boolean mask of the roots."""
    n = G.shape[0]
    h = node_hash(n)
    idx = np.arange(n, dtype=np.uint64)
    OUT, UND, IN = 0, 1, 2
    state = np.full(n, UND, dtype=np.uint64)
    ip, ind = G.indptr, G.indices
    while True:
        und = state == UND
        if not und.any():
            break
        key = (state << np.uint64(62)) | (h << np.uint64(32)) | idx
        m1 = _rowmax(ip, ind, key, key)
        m2 = _rowmax(ip, ind, m1, m1)
        becomes_in = und & (m2 == key)
        becomes_out = und & ~becomes_in & ((m2 >> np.uint64(62)) == IN)
        state[becomes_in] = IN
        state[becomes_out] = OUT
    return state == IN


def mis2_aggregate(G):
    """Aggregates seeded by the distance-2 MIS roots.
    Returns agg[n] (aggregate id per node) and the number of aggregates."""
    n = G.shape[0]
    h = node_hash(n)
    idx = np.arange(n, dtype=np.uint64)
    ip, ind = G.indptr, G.indices
    is_root = mis2_roots(G)
    roots = np.nonzero(is_root)[0]
    agg = np.full(n, -1, dtype=np.int64)
    agg[roots] = np.arange(len(roots))
    nk = (h << np.uint64(32)) | idx
    # pass 1: neighbours of roots join the root of largest key
    first = agg.copy()
    for i in range(n):
        if agg[i] >= 0:
            continue
        best = None
        for j in ind[ip[i]:ip[i + 1]]:
            if is_root[j] and (best is None or nk[j] > nk[best]):
                best = j
        if best is not None:
            first[i] = agg[best]
    # pass 2: the rest join the first-pass neighbour of largest key
    final = first.copy()
    for i in range(n):
        if first[i] >= 0:
            continue
        best = None
        for j in ind[ip[i]:ip[i + 1]]:
            if first[j] >= 0 and not is_root[j] and (best is None or nk[j] > nk[best]):
                best = j
        if best is None:
            raise RuntimeError("aggregation left a node unassigned")
        final[i] = first[best]
    return final, len(roots)


def smoothed_prolongator(A, G, agg, nagg, omega=2.0 / 3.0):
    """P = (I - omega D_F^{-1} A_F) T, A_F = A with weak off-diagonals lumped
    into the diagonal."""
    A = A.tocsr()
    n = A.shape[0]
    r = np.repeat(np.arange(n), np.diff(A.indptr))
    c = A.indices
    v = A.data
    Gs = set(zip(*G.nonzero()))
    strong = np.array([(ri, ci) in Gs for ri, ci in zip(r, c)], dtype=bool)
    diag = r == c
    weak_off = ~diag & ~strong
    dF = np.zeros(n)
    np.add.at(dF, r[diag], v[diag])
    np.add.at(dF, r[weak_off], v[weak_off])
    keep = diag | strong
    vals = np.where(diag, dF[r], v)
    AF = sp.csr_matrix((vals[keep], (r[keep], c[keep])), shape=(n, n))
    T = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nagg))
    P = T - omega * (sp.diags(1.0 / dF) @ AF @ T)
    P = P.tocsr()
    P.eliminate_zeros()
    P.sort_indices()
    return P


class AMG:
    """Hierarchy and V(1,1)-cycle as described in the module docstring."""

    def __init__(self, S, theta=0.25, max_coarse=1024, max_levels=25, singular=False, omega=2.0 / 3.0):
        self.singular = singular
        self.A = [S.tocsr()]
        self.P = []
        self.aggs = []
        A = self.A[0]
        while A.shape[0] > max_coarse and len(self.A) < max_levels:
            G = strength_graph(A, theta)
            agg, nagg = mis2_aggregate(G)
            if nagg >= A.shape[0]:
                break
            P = smoothed_prolongator(A, G, agg, nagg, omega)
            Ac = (P.T @ A @ P).tocsr()
            Ac = ((Ac + Ac.T) * 0.5).tocsr()
            Ac.sort_indices()
            self.P.append(P)
            self.aggs.append(agg)
            self.A.append(Ac)
            A = Ac
        self.dl1 = [np.asarray(abs(L).sum(axis=1)).ravel() for L in self.A]
        Ac = self.A[-1].toarray()
        if singular:
            nc = Ac.shape[0]
            s = np.trace(Ac) / nc / nc
            Ac = Ac + s * np.ones((nc, nc))
        self.coarse_inv = np.linalg.inv(Ac)

    @property
    def nlevels(self):
        return len(self.A)

    def vcycle(self, b, level=0):
        if level == self.nlevels - 1:
            return self.coarse_inv @ b
        A, d = self.A[level], self.dl1[level]
        x = b / d
        r = b - A @ x
        xc = self.vcycle(self.P[level].T @ r, level + 1)
        x = x + self.P[level] @ xc
        x = x + (b - A @ x) / d
        return x

    def apply(self, b):
        z = self.vcycle(np.asarray(b, dtype=np.float64))
        if self.singular:
            z = z - z.mean()
        return z


class BlockPreconditioner:
    """z = B^{-1} r = [ (tau M~)^{-1} r_u ; S^{-1} r_q ], identity on the
    essential RT dofs.  schur = 'amg' (one V-cycle), 'exact' (sparse direct
    solve with S~) or a callable.  Md: M~ to use instead of diag(M) (the
    learned diagonal); S~ and the AMG are then built from it."""

    def __init__(self, prob, tau=1.0, schur='amg', amg_kwargs=None, Md=None):
        self.prob = prob
        self.tau = tau
        self.Md = diag_M(prob) if Md is None else np.asarray(Md, dtype=np.float64)
        self.S = schur_by_formula(prob, self.Md)
        self.singular = schur_is_singular(prob)
        self.nu = prob.mesh.n_u
        if schur == 'amg':
            self.amg = AMG(self.S, singular=self.singular, **(amg_kwargs or {}))
            self.schur = self.amg.apply
        elif schur == 'exact':
            import scipy.sparse.linalg as spla
            if self.singular:
                n = self.S.shape[0]
                Sreg = (self.S + sp.csr_matrix(np.full((n, n), 1.0 / n))).tocsc()
                lu = spla.splu(Sreg)
                self.schur = lambda r: (lambda z: z - z.mean())(lu.solve(r))
            else:
                lu = spla.splu(self.S.tocsc())
                self.schur = lu.solve
        else:
            self.schur = schur

    def __call__(self, r):
        r = np.asarray(r, dtype=np.float64)
        zu = r[:self.nu] / (self.tau * self.Md)
        zu[self.prob.ess] = r[:self.nu][self.prob.ess]
        zq = self.schur(r[self.nu:])
        return np.concatenate([zu, zq])
