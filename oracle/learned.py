"""Learned per-element correction of the (1,1)-block diagonal.  Test
infrastructure: plain FP64 reference of every step of the learned path.

The paper preconditions the (1,1) block with M~ = diag(M) (Section 2.3).  The
learned form rescales each element's contribution to that diagonal before it
is summed into M~; S~ and the AMG are then built from the corrected M~.
Nothing of this is in the paper; the definitions below are the readings this
library uses, written out once here and once in the HIP code.

Scalings.  Six per element, theta = log s ordered (x-, x+, y-, y+, z-, z+).
An RT dof of component c whose index along direction c is i (Gauss-Lobatto
sub-element vertex xi_i in [0, 1]) is scaled by
    s_dof = exp((1 - xi_i) theta_{2c} + xi_i theta_{2c+1}),
i.e. geometrically between the two faces normal to c.

Target (per element, independent of the coefficients).  With m = diag(M_e)
for unit coefficient and D(theta) = diag(s_dof * m),
    f(theta) = log lambda_max - log lambda_min  of the pencil (M_e, D(theta)),
minimised over theta with sum(theta) = 0 by projected gradient descent from
theta = 0 with Armijo backtracking (at most MAX_STEPS accepted steps).  The
gradient uses the eigenvectors: with w the unit eigenvector of
D^{-1/2} M_e D^{-1/2}, d log(lambda)/d theta_j = -sum_dof w_dof^2 a_dof,j,
a_dof,j the weight of theta_j in log s_dof.

Network.  x in R^27 = 24 vertex offsets from the centroid divided by the
mean edge length (vertex order (dz, dy, dx), coordinate fastest), ln alpha,
ln beta, p / 6.  Linear(27, 64) - GELU - Linear(64, 64) - GELU - Linear(64, 6)
with the exact GELU x Phi(x); the scalings are exp(clip(o, -ln 4, ln 4)).
Loss: mean squared error against the targets clipped to the same range.
Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.
"""
import math

import numpy as np
from scipy.special import erf

from .basis import gauss_lobatto_points
from .element import element_matrices, rt_shapes

LN4 = math.log(4.0)
N_IN, N_HID, N_OUT = 27, 64, 6
MAX_STEPS = 30
ARMIJO = 1e-4


# ---------------------------------------------------------------------------
# per-dof scaling weights
# ---------------------------------------------------------------------------
def dof_weights(p):
    """A [nrt, 6]: log s_dof = A @ theta, local RT numbering
    (component-major, first index fastest)."""
    xi = gauss_lobatto_points(p)
    rows = []
    for c, shape in enumerate(rt_shapes(p)):
        # shape is (n0, n1, n2) with extent p + 1 along c
        n0, n1, n2 = shape
        for k in range(n2):
            for j in range(n1):
                for i in range(n0):
                    idx = (i, j, k)[c]
                    a = np.zeros(6)
                    a[2 * c] = 1.0 - xi[idx]
                    a[2 * c + 1] = xi[idx]
                    rows.append(a)
    return np.array(rows)


# ---------------------------------------------------------------------------
# target: minimise the spread of the pencil (M_e, D(theta))
# ---------------------------------------------------------------------------
def pencil_extremes(Me, m, A, theta, vectors=True):
    """(lambda_min, lambda_max) of (M_e, diag(m exp(A theta))) and, when
    asked, the unit eigenvectors of the symmetrically scaled matrix."""
    d = m * np.exp(A @ theta)
    r = 1.0 / np.sqrt(d)
    S = Me * r[:, None] * r[None, :]
    lam, V = np.linalg.eigh(S)
    if vectors:
        return lam[0], lam[-1], V[:, 0], V[:, -1]
    return lam[0], lam[-1]


def spread(Me, m, A, theta):
    lo, hi = pencil_extremes(Me, m, A, theta, vectors=False)
    return math.log(hi) - math.log(lo)


def spread_gradient(Me, m, A, theta):
    """f(theta) and its gradient."""
    lo, hi, wlo, whi = pencil_extremes(Me, m, A, theta)
    f = math.log(hi) - math.log(lo)
    g = A.T @ (wlo ** 2 - whi ** 2)
    return f, g


def element_target(Me, p, max_steps=MAX_STEPS):
    """Projected-gradient minimiser theta* of f on sum(theta) = 0, with the
    spread at theta = 0 and at theta*.  Step rule: start with eta = 1; a
    trial theta - eta P g is accepted when f drops by at least
    ARMIJO eta |P g|^2 (then eta doubles, at most 4), otherwise eta halves
    (at most 20 times per step, after which the descent ends)."""
    A = dof_weights(p)
    m = np.diag(Me).copy()
    theta = np.zeros(6)
    f, g = spread_gradient(Me, m, A, theta)
    f0 = f
    eta = 1.0
    for _ in range(max_steps):
        pg = g - g.mean()
        gg = float(pg @ pg)
        if gg <= 1e-24:
            break
        accepted = False
        for _ in range(20):
            trial = theta - eta * pg
            ft = spread(Me, m, A, trial)
            if ft <= f - ARMIJO * eta * gg:
                accepted = True
                break
            eta *= 0.5
        if not accepted:
            break
        theta = trial
        f, g = spread_gradient(Me, m, A, theta)
        eta = min(2.0 * eta, 4.0)
    return theta, f0, f


def element_targets(V, p):
    """theta* [E, 6] and (lambda_min, lambda_max) [E, 2] at theta* for
    elements V [E, 2, 2, 2, 3] of order p (unit coefficient)."""
    mats = element_matrices(p, V)
    A = dof_weights(p)
    th = np.zeros((len(V), 6))
    lam = np.zeros((len(V), 2))
    for e, Me in enumerate(mats['M']):
        th[e], _, _ = element_target(Me, p)
        lo, hi = pencil_extremes(Me, np.diag(Me), A, th[e], vectors=False)
        lam[e] = lo, hi
    return th, lam


# ---------------------------------------------------------------------------
# second target: the element's saddle-point pencil, which sees alpha and beta
# ---------------------------------------------------------------------------
# For one element in isolation (all of its RT dofs free), the transformed
# grad-div block (Section 3, eq. transformed-saddle-point)
#     A_e = [[beta M1, D^T], [D, -(1/alpha) W^{-1}]]
# (M1 the unit-coefficient RT mass matrix, D the +-1 incidence, W the L2 mass
# matrix) and the block-diagonal preconditioner of Section 2.3 with the
# scaled diagonal
#     B_e(theta) = diag(Md, C~ + D Md^{-1} D^T),  Md = s_dof beta diag(M1),
#     C~ = (1/alpha) diag(W)^{-1}.
# The target minimises f2 = log max|lambda| - log min|lambda| over the
# eigenvalues of A_e v = lambda B_e v, over all of theta (a common factor of
# the six scalings is not neutral here: it moves weight between the (1,1)
# block and the Schur block).  For B-normalised v = (v_u, v_q),
#     d lambda / d theta_j = -lambda v^T (dB / d theta_j) v,
#     v^T (dB/dtheta_j) v = sum a_dj Md_d v_u,d^2 - sum a_dj (D^T v_q)_d^2 / Md_d,
# with a_dj the weight of theta_j in log s_dof.

def saddle_blocks(M1, W, D, alpha, beta):
    """A_e and the pieces of B_e that do not depend on theta."""
    Winv = np.linalg.inv(W)
    A = np.block([[beta * M1, D.T], [D, -(1.0 / alpha) * Winv]])
    m = beta * np.diag(M1)
    ct = (1.0 / alpha) / np.diag(W)
    return A, m, ct


def saddle_pencil(A, m, ct, D, Aw, theta, exact=None):
    """Eigenvalues and B-normalised eigenvectors of A v = lambda B(theta) v.
    exact = (M, S): use the exact blocks M and S = C + D M^{-1} D^T instead
    (the setting of Prop. 1)."""
    import scipy.linalg as sla
    nu = D.shape[1]
    if exact is not None:
        Bm = sla.block_diag(exact[0], exact[1])
        md = None
    else:
        md = m * np.exp(Aw @ theta)
        S = np.diag(ct) + (D / md[None, :]) @ D.T
        Bm = sla.block_diag(np.diag(md), S)
    lam, V = sla.eigh(A, Bm)
    return lam, V, md, nu


def saddle_spread_gradient(A, m, ct, D, Aw, theta):
    """f2(theta) and its gradient."""
    lam, V, md, nu = saddle_pencil(A, m, ct, D, Aw, theta)
    a = np.abs(lam)
    i_hi, i_lo = int(np.argmax(a)), int(np.argmin(a))
    f = math.log(a[i_hi]) - math.log(a[i_lo])

    def vdb(v):
        vu, vq = v[:nu], v[nu:]
        dq = D.T @ vq
        return Aw.T @ (md * vu ** 2) - Aw.T @ (dq ** 2 / md)

    # d log|lambda| / d theta = -v^T dB v
    g = -vdb(V[:, i_hi]) + vdb(V[:, i_lo])
    return f, g


def saddle_target(A, m, ct, D, p, max_steps=MAX_STEPS):
    """Gradient-descent minimiser of f2 from theta = 0 (Armijo rule as in
    element_target, without the projection), with f2 at 0 and at the end."""
    Aw = dof_weights(p)
    theta = np.zeros(6)
    f, g = saddle_spread_gradient(A, m, ct, D, Aw, theta)
    f0 = f
    eta = 1.0
    for _ in range(max_steps):
        gg = float(g @ g)
        if gg <= 1e-24:
            break
        accepted = False
        for _ in range(20):
            trial = theta - eta * g
            ft, gt = saddle_spread_gradient(A, m, ct, D, Aw, trial)
            if ft <= f - ARMIJO * eta * gg:
                accepted = True
                break
            eta *= 0.5
        if not accepted:
            break
        theta, f, g = trial, ft, gt
        eta = min(2.0 * eta, 4.0)
    return theta, f0, f


def saddle_targets(V, p, alpha, beta, max_steps=MAX_STEPS):
    """theta* [E, 6] and f2 at 0 and at theta* [E, 2] for elements
    V [E, 2, 2, 2, 3] with coefficients alpha, beta [E]."""
    from .element import reference_divergence
    mats = element_matrices(p, V)
    D = reference_divergence(p)
    th = np.zeros((len(V), 6))
    fs = np.zeros((len(V), 2))
    for e in range(len(V)):
        A, m, ct = saddle_blocks(mats['M'][e], mats['W'][e], D, alpha[e], beta[e])
        th[e], fs[e, 0], fs[e, 1] = saddle_target(A, m, ct, D, p, max_steps)
    return th, fs


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
_EDGES = [((0, 0, 0), (0, 0, 1)), ((0, 1, 0), (0, 1, 1)), ((1, 0, 0), (1, 0, 1)), ((1, 1, 0), (1, 1, 1)),
          ((0, 0, 0), (0, 1, 0)), ((0, 0, 1), (0, 1, 1)), ((1, 0, 0), (1, 1, 0)), ((1, 0, 1), (1, 1, 1)),
          ((0, 0, 0), (1, 0, 0)), ((0, 0, 1), (1, 0, 1)), ((0, 1, 0), (1, 1, 0)), ((0, 1, 1), (1, 1, 1))]


def features(V, alpha, beta, p):
    """x [E, 27] for elements V [E, 2, 2, 2, 3] (indexed [dz, dy, dx, :])."""
    V = np.asarray(V, dtype=np.float64)
    E = V.shape[0]
    c = V.reshape(E, 8, 3).mean(axis=1)
    h = np.zeros(E)
    for a, b in _EDGES:
        h += np.linalg.norm(V[:, a[0], a[1], a[2]] - V[:, b[0], b[1], b[2]], axis=1)
    h /= 12.0
    off = (V.reshape(E, 8, 3) - c[:, None, :]) / h[:, None, None]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), (E,))
    return np.concatenate([off.reshape(E, 24), np.log(alpha)[:, None], np.log(beta)[:, None],
                           (p / 6.0)[:, None]], axis=1)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_deriv(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def init_params(seed=0):
    """W_l [out, in] ~ U(-1/sqrt(in), 1/sqrt(in)), b_l = 0."""
    rng = np.random.default_rng(seed)
    sizes = [(N_HID, N_IN), (N_HID, N_HID), (N_OUT, N_HID)]
    params = []
    for o, i in sizes:
        bound = 1.0 / math.sqrt(i)
        params.append(rng.uniform(-bound, bound, (o, i)))
        params.append(np.zeros(o))
    return params


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    a1 = gelu(z1)
    z2 = a1 @ W2.T + b2
    a2 = gelu(z2)
    o = a2 @ W3.T + b3
    return o, (X, z1, a1, z2, a2)


def loss_and_grad(params, X, Y):
    """Mean squared error over all outputs of the batch and its gradient."""
    W1, b1, W2, b2, W3, b3 = params
    o, (X, z1, a1, z2, a2) = forward(params, X)
    T = np.clip(Y, -LN4, LN4)
    n = o.size
    diff = o - T
    loss = float((diff ** 2).sum() / n)
    do = 2.0 * diff / n
    gW3 = do.T @ a2
    gb3 = do.sum(axis=0)
    dz2 = (do @ W3) * gelu_deriv(z2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_deriv(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = dict(t, m, v)."""
    state['t'] += 1
    t = state['t']
    for k, (p_, g) in enumerate(zip(params, grads)):
        state['m'][k] = b1 * state['m'][k] + (1 - b1) * g
        state['v'][k] = b2 * state['v'][k] + (1 - b2) * g * g
        mh = state['m'][k] / (1 - b1 ** t)
        vh = state['v'][k] / (1 - b2 ** t)
        p_ -= lr * mh / (np.sqrt(vh) + eps)


def adam_state(params):
    return dict(t=0, m=[np.zeros_like(p_) for p_ in params], v=[np.zeros_like(p_) for p_ in params])


def scalings(params, X):
    """theta used by the preconditioner: clip(o, -ln 4, ln 4)."""
    o, _ = forward(params, X)
    return np.clip(o, -LN4, LN4)


# ---------------------------------------------------------------------------
# corrected diagonal
# ---------------------------------------------------------------------------
def learned_diag(prob, theta):
    """M~ = sum_e E_e^T (diag(M_e) * s_e) with s_e from theta [ne, 6]
    (1 on essential dofs, as for the plain diagonal)."""
    mesh = prob.mesh
    A = dof_weights(mesh.p)
    d = np.zeros(mesh.n_u)
    for e in range(mesh.ne):
        local = np.diag(prob.Me[e]) * np.exp(A @ theta[e])
        np.add.at(d, prob.l2g[e], local)
    d[prob.ess] = 1.0
    return d
