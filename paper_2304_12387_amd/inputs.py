"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws meshes, coefficient fields and right-hand sides from
numpy's seeded generators.  It holds none of the method's arithmetic and is
shared by the tests (GPU library and CPU oracle alike) and the benchmark.

Workloads
---------
darcy_cube_4     Darcy (eps = 1, gamma = 0) on the unit cube, 4^3 Cartesian
                 hexahedra, RT p = 2, manufactured p = sin(pi x) sin(pi y) sin(pi z).
graddiv_32       grad-div on the unit cube, 32^3 hexahedra with vertices
                 jittered by +-10% h, p = 4, alpha and beta per element
                 log-uniform in [1e-2, 1e2].
darcy_layered    Darcy on a 60 x 220 x 85 Cartesian grid of 20 x 10 x 2 cells,
                 p = 2, per-element permeability k = exp(z), z a smoothed
                 Gaussian field (sigma 2.5, correlation 3 cells horizontally
                 and 1 vertically), eps = 1/k, gamma = 0, flux condition
                 u.n = (1,0,0).n on the whole boundary (a stand-in for the SPE10
                 data, which is not available here).
"""
import numpy as np

SIDES_ALL = 63


def box_vertices(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    """Cartesian vertices [(nx+1)(ny+1)(nz+1), 3], x fastest."""
    x = np.linspace(0.0, lx, nx + 1)
    y = np.linspace(0.0, ly, ny + 1)
    z = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing='ij')
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def jittered_vertices(nx, ny, nz, frac, seed, lx=1.0, ly=1.0, lz=1.0):
    """Cartesian vertices moved by U[-frac h, frac h] per coordinate.  A
    coordinate is only moved when the vertex is interior in that direction,
    so boundary vertices slide along the boundary and corners stay fixed."""
    V = box_vertices(nx, ny, nz, lx, ly, lz)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, size=V.shape)
    h = np.array([lx / nx, ly / ny, lz / nz])
    n = np.array([nx, ny, nz])
    idx = np.arange(V.shape[0])
    ijk = np.stack([idx % (nx + 1), (idx // (nx + 1)) % (ny + 1), idx // ((nx + 1) * (ny + 1))], axis=1)
    interior = (ijk > 0) & (ijk < n[None, :])
    return V + d * frac * h[None, :] * interior


def loguniform(n, lo, hi, rng):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def uniform_vector(n, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def gaussian_field(shape, corr_cells, sigma, seed):
    """Unit-std Gaussian field: i.i.d. N(0,1) on the grid, separable Gaussian
    smoothing with standard deviation corr/sqrt(2) cells per axis (reflecting
    boundaries), re-normalised to zero mean and unit empirical std, times
    sigma.  ``shape`` and ``corr_cells`` are in (z, y, x) order."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(size=shape)
    g = gaussian_filter(g, sigma=[c / np.sqrt(2.0) for c in corr_cells], mode='reflect')
    g = (g - g.mean()) / g.std()
    return sigma * g


def darcy_cube_4():
    n, p = 4, 2
    return dict(name='darcy_cube_4', nx=n, ny=n, nz=n, p=p, problem=1,
                vertices=box_vertices(n, n, n), c_mass=np.ones(n ** 3), c_22=None,
                ess_sides=0, tol=1e-10)


def graddiv_jittered(n, p, seed_mesh=2, seed_coef=12, jitter=0.1):
    rng = np.random.default_rng(seed_coef)
    ne = n ** 3
    alpha = loguniform(ne, 1e-2, 1e2, rng)
    beta = loguniform(ne, 1e-2, 1e2, rng)
    return dict(name=f'graddiv_{n}_p{p}', nx=n, ny=n, nz=n, p=p, problem=0,
                vertices=jittered_vertices(n, n, n, jitter, seed_mesh),
                c_mass=beta, c_22=alpha, ess_sides=0, tol=1e-8)


def graddiv_32():
    return graddiv_jittered(32, 4)


def darcy_layered(nx=60, ny=220, nz=85, p=2, seed=3):
    hx, hy, hz = 20.0, 10.0, 2.0
    z = gaussian_field((nz, ny, nx), (1.0, 3.0, 3.0), 2.5, seed)
    k = np.exp(z).ravel()          # element-major order e = ex + nx (ey + ny ez)
    return dict(name=f'darcy_layered_{nx}x{ny}x{nz}_p{p}', nx=nx, ny=ny, nz=nz, p=p, problem=1,
                vertices=box_vertices(nx, ny, nz, nx * hx, ny * hy, nz * hz),
                c_mass=k, c_22=None, ess_sides=SIDES_ALL, tol=1e-8, cell=(hx, hy, hz))


def graddiv_rhs(n_u, n_q, seed=22):
    """b_u ~ U[-1, 1] on the RT dofs, b_q = 0."""
    return np.concatenate([uniform_vector(n_u, seed), np.zeros(n_q)])
