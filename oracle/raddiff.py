"""Grey nonlinear radiation diffusion (Section 4.3): the time-stepping driver
around the Darcy-type saddle-point solves.  Test infrastructure: a plain FP64
CPU version of what hd_rd_step computes.

Equations (Section 4.3, eq. rad-diff-e, rad-diff-E, rad-diff-F):
    rho de/dt = -c sigma (a T^4 - E) + Q,     T = e / C_v,
    dE/dt + div F = c sigma (a T^4 - E) + S,
    F = -(c / (3 sigma)) grad E,
with e, E in the L2 space and F in RT_p, F . n = 0 on the boundary (every
boundary RT dof essential and zero), Q = S = 0, sigma constant.

Readings (the paper does not write out the discrete equations):
* The energies live in the L2 space of the transformed system, whose basis
  functions are mapped with 1 / det J (so that D = W^{-1} B is the +-1
  incidence, Section 2.1): a dof is the integral of the function over its
  sub-cell K_j.  The unknowns are therefore energy amounts per sub-cell,
  e_j = integral of rho e and E_j = integral of E over K_j, and the sum over
  the dofs of e_j + E_j is the total energy.
* The nonlinear exchange term is taken sub-cell by sub-cell with the
  sub-cell mean temperature T_j = e_j / (rho C_v |K_j|):
      de_j/dt = -c sigma (a T_j^4 |K_j| - E_j),
      dE_j/dt + (D F)_j = c sigma (a T_j^4 |K_j| - E_j),
  with |K_j| the physical volume of the sub-cell.
* The flux equation in weak form is M_{3 sigma / c} F - B^T E = 0, i.e.
  M F + D^T q~ = 0 with q~ = -W E.
* Time stepping: the three-stage L-stable SDIRK method of Alexander (1977),
  diagonal gamma, stiffly accurate (the last stage is the new state).
* Each stage value X_i = (e, E, F) solves (X_i - Xhat_i) / (gamma dt) = f(X_i)
  with Xhat_i = X_n + sum_{j<i} (a_ij / gamma) (X_j - Xhat_j).  The stage
  equations are solved by the outer iteration of Section 4.3: (1) F fixed,
  the 2 x 2 system of each L2 dof for (e_j, E_j) by Newton's method; (2) e
  fixed, the linear Darcy-type system for (E, F):
      kappa E + D F = r,  kappa = 1 / (gamma dt) + c sigma,
      r = Ehat / (gamma dt) + c sigma a T^4 |K|,
  which is the library's transformed Darcy system [[M, D^T], [D, -kappa W^{-1}]]
  with c_mass = 3 sigma / c, gamma = kappa, unknowns (F, q~ = -W E) and
  right-hand side [0; r]; repeated until the relative residual of the
  e-equation with the new E is below the outer tolerance.
"""
import math

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import DARCY, Mesh, Problem
from .basis import gauss_legendre, gauss_lobatto_points
from .element import trilinear

# Alexander (1977): gamma the root in (1/6, 1/2) of x^3 - 3 x^2 + 3 x / 2 - 1/6
SDIRK_GAMMA = 0.43586652150845899942


def sdirk3_tableau():
    g = SDIRK_GAMMA
    b1 = -(6 * g * g - 16 * g + 1) / 4
    b2 = (6 * g * g - 20 * g + 5) / 4
    A = np.array([[g, 0.0, 0.0], [(1 - g) / 2, g, 0.0], [b1, b2, g]])
    return A


def subcell_volumes(mesh):
    """|K_j| for every L2 dof (element-major, then a, b, c): the integral of
    det J over the sub-cell [xi_a, xi_a+1] x [xi_b, xi_b+1] x [xi_c, xi_c+1]
    of the Gauss-Lobatto points, by 2 x 2 x 2 Gauss-Legendre points per
    sub-cell (det J of the trilinear map has degree 2 in each variable)."""
    p = mesh.p
    xi = gauss_lobatto_points(p)
    g, w = gauss_legendre(2)
    pts, wts = [], []
    for c in range(p):
        for b in range(p):
            for a in range(p):
                for k in range(2):
                    for j in range(2):
                        for i in range(2):
                            lo = np.array([xi[a], xi[b], xi[c]])
                            h = np.array([xi[a + 1] - xi[a], xi[b + 1] - xi[b], xi[c + 1] - xi[c]])
                            pts.append(lo + h * np.array([g[i], g[j], g[k]]))
                            wts.append(np.prod(h) * w[i] * w[j] * w[k])
    pts = np.array(pts)
    wts = np.array(wts)
    _, J = trilinear(mesh.element_vertices(), pts)
    det = np.linalg.det(J)                                   # [E, p^3 * 8]
    vol = (det * wts[None, :]).reshape(mesh.ne, p ** 3, 8).sum(axis=2)
    return vol.reshape(-1)


class RadDiff:
    """The radiation-diffusion system on a structured mesh of order p; the
    state is (e, E) per L2 dof (energy amounts per sub-cell) and F."""

    def __init__(self, nx, ny, nz, p, vertices, rho=1.0, cv=1.0, c=1.0, a=1.0, sigma=1.0):
        self.mesh = Mesh(nx, ny, nz, p, vertices)
        self.rho, self.cv, self.c, self.a, self.sigma = rho, cv, c, a, sigma
        self.ne = nx * ny * nz
        self.vol = subcell_volumes(self.mesh)
        self._prob = {}

    def problem(self, kappa):
        if kappa not in self._prob:
            self._prob[kappa] = Problem(self.mesh, DARCY, np.full(self.ne, 3 * self.sigma / self.c),
                                        np.full(self.ne, kappa), ess_sides=63)
        return self._prob[kappa]

    def energy(self, e, E):
        """Total energy: the sum of the sub-cell amounts."""
        return float(np.sum(e) + np.sum(E))

    def emission(self, e):
        """a T^4 |K| with T = e / (rho C_v |K|)."""
        T = e / (self.rho * self.cv * self.vol)
        return self.a * T ** 4 * self.vol

    def newton(self, ehat, Ehat, dF, gdt, tol=1e-12, max_it=50):
        """The 2 x 2 system of every dof for (e, E) with D F fixed."""
        c, s = self.c, self.sigma
        e, E = ehat.copy(), Ehat.copy()
        its = 0
        for it in range(max_it):
            B = self.emission(e)
            dB = 4.0 * B / e
            R1 = (e - ehat) / gdt + c * s * (B - E)
            R2 = (E - Ehat) / gdt + dF - c * s * (B - E)
            J11 = 1.0 / gdt + c * s * dB
            J12 = -c * s
            J21 = -c * s * dB
            J22 = 1.0 / gdt + c * s
            det = J11 * J22 - J12 * J21
            de = (J22 * R1 - J12 * R2) / det
            dE = (-J21 * R1 + J11 * R2) / det
            e = e - de
            E = E - dE
            its = it + 1
            if np.all(np.abs(de) <= tol * np.abs(e)) and np.all(np.abs(dE) <= tol * np.maximum(np.abs(E), 1e-300)):
                break
        return e, E, its

    def darcy_solve(self, e, Ehat, gdt):
        """(E, F) with e fixed: the transformed Darcy system, direct solve."""
        kappa = 1.0 / gdt + self.c * self.sigma
        P = self.problem(kappa)
        nu = self.mesh.n_u
        r = Ehat / gdt + self.c * self.sigma * self.emission(e)
        b = np.concatenate([np.zeros(nu), r])
        x = spla.spsolve(P.block_matrix().tocsc(), b)
        F = x[:nu]
        E = -spla.spsolve(P.W.tocsc(), x[nu:])
        return E, F

    def div(self, F):
        return np.asarray(self.problem(1.0).D @ F)

    def e_residual(self, e, E, ehat, gdt):
        """Relative residual of the e-equation (the E-equation holds after
        the Darcy solve)."""
        R1 = (e - ehat) / gdt + self.c * self.sigma * (self.emission(e) - E)
        scale = np.linalg.norm(e - ehat) / gdt + self.c * self.sigma * np.linalg.norm(E) + 1e-300
        return np.linalg.norm(R1) / scale

    def stage(self, ehat, Ehat, e0, E0, F0, gdt, tol_outer=1e-12, max_outer=20):
        """One SDIRK stage: outer iterations from (e0, E0, F0)."""
        e, E, F = e0.copy(), E0.copy(), F0.copy()
        outer = 0
        for k in range(max_outer):
            e, _, _ = self.newton(ehat, Ehat, self.div(F), gdt)
            E, F = self.darcy_solve(e, Ehat, gdt)
            outer = k + 1
            if self.e_residual(e, E, ehat, gdt) <= tol_outer:
                break
        return e, E, F, outer

    def step(self, e, E, F, dt, tol_outer=1e-12):
        """One SDIRK3 step; returns (e, E, F) at t + dt and the outer
        iteration counts of the stages."""
        A = sdirk3_tableau()
        g = SDIRK_GAMMA
        gdt = g * dt
        X = []      # stage values (e, E)
        H = []      # their Xhat
        Fi = F.copy()
        ei, Ei = e.copy(), E.copy()
        outers = []
        for i in range(3):
            eh, Eh = e.copy(), E.copy()
            for j in range(i):
                eh += (A[i, j] / g) * (X[j][0] - H[j][0])
                Eh += (A[i, j] / g) * (X[j][1] - H[j][1])
            ei, Ei, Fi, k = self.stage(eh, Eh, ei, Ei, Fi, gdt, tol_outer)
            X.append((ei, Ei))
            H.append((eh, Eh))
            outers.append(k)
        return ei, Ei, Fi, outers


def uniform_exchange_reference(e0, E0, t, vol=1.0, rho=1.0, cv=1.0, c=1.0, a=1.0, sigma=1.0):
    """The exchange ODE of one sub-cell of volume vol with D F = 0,
    integrated accurately by scipy's Radau method: the exact solution the
    time steps of a uniform state converge to."""
    from scipy.integrate import solve_ivp

    def f(_, y):
        T = y[0] / (rho * cv * vol)
        ex = c * sigma * (a * T ** 4 * vol - y[1])
        return [-ex, ex]

    sol = solve_ivp(f, (0.0, t), [e0, E0], method='Radau', rtol=1e-13, atol=1e-15)
    return sol.y[0, -1], sol.y[1, -1]
