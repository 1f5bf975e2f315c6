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
graddiv_distorted
                 grad-div on the unit cube, 48^3 hexahedra, p = 4: z-layers
                 graded so that their thickness varies 8x, shear
                 x' = x + tan(t(z)) y with t rising smoothly from 0 to 30 deg,
                 interior vertices jittered by +-10% of the local spacing,
                 alpha and beta per element log-uniform in [1e-2, 1e2].
batch_instances  independent grad-div problems for batching: n^3 unit-cube
                 meshes (n uniform in [nmin, nmax]) jittered by +-10% h, p
                 uniform in 1..6, alpha = T^3 / 3 and sigma = T^-3 with
                 T = 2^clip(G, -1, 1), G a unit-std Gaussian field with
                 correlation length a quarter of the domain, beta per instance
                 log-uniform in [0.1, 10].
training_elements
                 single distorted hexahedra for the learned diagonal: axis
                 stretches log-uniform with max/min <= 8, shears in U[-30, 30]
                 deg on the three coordinate planes, vertex jitter +-10% of the
                 shortest edge, p uniform in 1..6, ln alpha and ln beta uniform
                 in [ln 1e-2, ln 1e2].
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


def gamma_vertex_field(nx, ny, nz, seed, sigma=1.0, corr=2.0):
    """Positive vertex values [(nx+1)(ny+1)(nz+1)] (x fastest) of a Darcy
    coefficient gamma that varies inside the elements: exp of a smooth
    Gaussian field with correlation `corr` vertex spacings."""
    z = gaussian_field((nz + 1, ny + 1, nx + 1), (corr, corr, corr), sigma, seed)
    return np.exp(z).ravel()


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


def raddiff_hotspot(n, seed=9, jitter=0.1, centre=(0.5, 0.5, 0.5), width=0.1, amp=1.0, rad_frac=0.5):
    """Grey radiation-diffusion test state on the jittered unit cube n^3:
    the mesh vertices, and per element the material temperature of a
    Gaussian hot spot T_e = 1 + amp exp(-|x_e - centre|^2 / width^2) at the
    element's vertex centroid x_e, and the radiation temperature rad_frac T_e
    (radiation out of equilibrium with the material).  The energies per
    sub-cell follow as e_j = rho C_v T_e |K_j| and E_j = a T_r^4 |K_j|."""
    V = jittered_vertices(n, n, n, jitter, seed)
    G = V.reshape(n + 1, n + 1, n + 1, 3)
    xc = sum(G[dz:dz + n, dy:dy + n, dx:dx + n] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)) / 8.0
    r2 = ((xc - np.asarray(centre)) ** 2).sum(axis=-1).reshape(-1)
    T = 1.0 + amp * np.exp(-r2 / width ** 2)
    return dict(vertices=V, T_mat=T, T_rad=rad_frac * T)


def graddiv_rhs(n_u, n_q, seed=22):
    """b_u ~ U[-1, 1] on the RT dofs, b_q = 0."""
    return np.concatenate([uniform_vector(n_u, seed), np.zeros(n_q)])


def graddiv_distorted(n=48, p=4, seed=5, jitter=0.1):
    """Graded, sheared and jittered unit-cube mesh with high-contrast
    coefficients (seeds: mesh `seed`, coefficients `seed` + 10)."""
    r = 8.0 ** (1.0 / (n - 1))
    t = r ** np.arange(n)
    zc = np.concatenate([[0.0], np.cumsum(t / t.sum())])
    xc = np.linspace(0.0, 1.0, n + 1)
    Z, Y, X = np.meshgrid(zc, xc, xc, indexing='ij')
    idx = np.arange(X.size)
    ijk = np.stack([idx % (n + 1), (idx // (n + 1)) % (n + 1), idx // ((n + 1) ** 2)], axis=1)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, size=(X.size, 3))
    # local spacing: the smaller of the two adjacent intervals per axis
    hz_cell = np.diff(zc)
    hz = np.minimum(hz_cell[np.clip(ijk[:, 2] - 1, 0, n - 1)], hz_cell[np.clip(ijk[:, 2], 0, n - 1)])
    h = np.stack([np.full(X.size, 1.0 / n), np.full(X.size, 1.0 / n), hz], axis=1)
    interior = np.all((ijk > 0) & (ijk < n), axis=1)[:, None]
    V = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + jitter * d * h * interior
    ang = np.radians(30.0) * 0.5 * (1.0 - np.cos(np.pi * V[:, 2]))
    V[:, 0] = V[:, 0] + np.tan(ang) * V[:, 1]
    crng = np.random.default_rng(seed + 10)
    ne = n ** 3
    alpha = loguniform(ne, 1e-2, 1e2, crng)
    beta = loguniform(ne, 1e-2, 1e2, crng)
    return dict(name=f'graddiv_distorted_{n}_p{p}', nx=n, ny=n, nz=n, p=p, problem=0, vertices=V,
                c_mass=beta, c_22=alpha, ess_sides=0, tol=1e-8)


def training_elements(n, seed=50):
    """n single hexahedra: vertices [n, 2, 2, 2, 3] (indexed [dz, dy, dx, :]),
    p [n], alpha [n], beta [n].  Unit cube -> axis stretches (ln s_i uniform
    in [0, ln 8], so max/min <= 8) -> shears tan(t) with t ~ U[-30, 30] deg
    on the xy, yz and zx planes -> independent vertex jitter of +-10% of the
    shortest edge.  Elements whose corner frames lose orientation are drawn
    again."""
    rng = np.random.default_rng(seed)
    cube = np.array([[dx, dy, dz] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)], dtype=np.float64)
    out = np.zeros((n, 8, 3))
    filled = 0
    while filled < n:
        m = n - filled
        s = np.exp(rng.uniform(0.0, np.log(8.0), size=(m, 3)))
        sh = np.tan(np.radians(rng.uniform(-30.0, 30.0, size=(m, 3))))
        V = cube[None, :, :] * s[:, None, :]
        V[:, :, 0] += sh[:, 0:1] * V[:, :, 1]
        V[:, :, 1] += sh[:, 1:2] * V[:, :, 2]
        V[:, :, 2] += sh[:, 2:3] * V[:, :, 0]
        edges = [(0, 1), (2, 3), (4, 5), (6, 7), (0, 2), (1, 3), (4, 6), (5, 7), (0, 4), (1, 5), (2, 6), (3, 7)]
        emin = np.min([np.linalg.norm(V[:, a] - V[:, b], axis=1) for a, b in edges], axis=0)
        V = V + 0.1 * emin[:, None, None] * rng.uniform(-1.0, 1.0, size=V.shape)
        # keep elements whose eight corner frames are right-handed
        ok = np.ones(m, dtype=bool)
        for v in range(8):
            dx, dy, dz = v & 1, (v >> 1) & 1, (v >> 2) & 1
            a = V[:, v ^ 1] - V[:, v]
            b = V[:, v ^ 2] - V[:, v]
            c = V[:, v ^ 4] - V[:, v]
            sgn = (1 - 2 * dx) * (1 - 2 * dy) * (1 - 2 * dz)
            ok &= sgn * np.einsum('ni,ni->n', a, np.cross(b, c)) > 0
        k = int(ok.sum())
        out[filled:filled + k] = V[ok][:k]
        filled += k
    p = rng.integers(1, 7, size=n)
    alpha = np.exp(rng.uniform(np.log(1e-2), np.log(1e2), size=n))
    beta = np.exp(rng.uniform(np.log(1e-2), np.log(1e2), size=n))
    return out.reshape(n, 2, 2, 2, 3), p, alpha, beta


def batch_instances(n_inst=32, seed=4, nmin=8, nmax=40, pmin=1, pmax=6):
    """A list of instance dicts (seeds: sizes and degrees `seed`, mesh of
    instance i `seed` + 10 + i, its field `seed` + 20 + i)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=n_inst)
    ps = rng.integers(pmin, pmax + 1, size=n_inst)
    betas = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=n_inst))
    out = []
    for i in range(n_inst):
        n, p = int(ns[i]), int(ps[i])
        G = gaussian_field((n, n, n), (0.25 * n,) * 3, 1.0, seed + 20 + i)
        T = 2.0 ** np.clip(G, -1.0, 1.0)
        alpha = (T ** 3 / 3.0).ravel()
        out.append(dict(name=f'batch_{i}_{n}^3_p{p}', nx=n, ny=n, nz=n, p=p, problem=0,
                        vertices=jittered_vertices(n, n, n, 0.1, seed + 10 + i),
                        c_mass=np.full(n ** 3, betas[i]), c_22=alpha, ess_sides=0))
    return out


# ---- unstructured hexahedral meshes --------------------------------------------
# Element vertices in the reference order v = dx + 2 dy + 4 dz.

REF_VERTS = np.array([[v & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], dtype=np.int64)


def from_structured(nx, ny, nz, vertices):
    """Element-to-vertex array of a structured nx x ny x nz box mesh (vertex
    (ix, iy, iz) numbered ix + (nx+1)(iy + (ny+1) iz), elements x fastest)."""
    el = []
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                el.append([(ex + (v & 1)) + (nx + 1) * ((ey + ((v >> 1) & 1)) + (ny + 1) * (ez + (v >> 2)))
                           for v in range(8)])
    return np.asarray(vertices, dtype=np.float64).reshape(-1, 3), np.asarray(el, dtype=np.int64)


def cube_rotations():
    """The 24 orientation-preserving symmetries of the reference cube as
    permutations of its 8 vertices: new_local[v] = old_local[perm[v]]."""
    mats = []
    for perm in ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]):
        for signs in np.ndindex(2, 2, 2):
            R = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                R[r, perm[r]] = 1 if signs[r] == 0 else -1
            if round(np.linalg.det(R)) == 1:
                mats.append(R)
    out = []
    for R in mats:
        # vertex at reference point x goes to R (x - 1/2) + 1/2
        p = []
        for v in range(8):
            x = REF_VERTS[v] * 2 - 1
            y = (R @ x + 1) // 2
            p.append(int(y[0] + 2 * y[1] + 4 * y[2]))
        out.append(np.array(p))
    return out


def scramble(vertices, elements, seed):
    """The same mesh with the vertices and the elements renumbered at random
    and every element's vertex list turned by a random rotation of the
    reference cube (orientation preserving, so det J stays positive)."""
    rng = np.random.default_rng(seed)
    nv = vertices.shape[0]
    vperm = rng.permutation(nv)            # old vertex v -> new number vperm[v]
    newV = np.empty_like(vertices)
    newV[vperm] = vertices
    rots = cube_rotations()
    el = vperm[elements]
    out = np.empty_like(el)
    for e in range(el.shape[0]):
        r = rots[rng.integers(len(rots))]
        # local vertex v of the turned element is the old local vertex r^-1[v]
        inv = np.empty(8, dtype=np.int64)
        inv[r] = np.arange(8)
        out[e] = el[e][inv]
    eperm = rng.permutation(el.shape[0])
    return newV, out[eperm], eperm


def o_grid(n, m, nz, seed=0, jitter=0.05):
    """An O-grid hexahedral mesh of a cylinder-like domain: a central n x n
    block and four n x m blocks around it, extruded over nz layers.  The four
    corners of the central block have 3 neighbouring vertices in the cross
    section instead of 4 (an unstructured mesh).  Interior vertices are
    jittered by +-jitter of the spacing (seeded)."""
    rng = np.random.default_rng(seed)
    pts = {}
    coords = []

    def vid(key, xy):
        if key not in pts:
            pts[key] = len(coords)
            coords.append(xy)
        return pts[key]

    # cross-section vertices: central square [-a, a]^2, outer ring radius R
    a, R = 0.5, 1.5
    quads = []
    # central block
    g = np.linspace(-a, a, n + 1)
    for j in range(n):
        for i in range(n):
            q = [('c', i + di, j + dj) for (di, dj) in ((0, 0), (1, 0), (0, 1), (1, 1))]
            quads.append(q)
    # boundary of the central block, counter-clockwise, 4n points
    def square_pt(t):
        # t in [0, 4n): side 0 bottom (left->right), 1 right (bottom->top), 2 top (right->left), 3 left
        s, r = divmod(t, n)
        if s == 0:
            return ('c', r, 0)
        if s == 1:
            return ('c', n, r)
        if s == 2:
            return ('c', n - r, n)
        return ('c', 0, n - r)

    def square_xy(t):
        key = square_pt(t)
        return np.array([g[key[1]], g[key[2]]])

    for t in range(4 * n):
        for k in range(m):
            q = []
            for (dt, dk) in ((0, 0), (1, 0), (0, 1), (1, 1)):
                tt = (t + dt) % (4 * n)
                kk = k + dk
                q.append(square_pt(tt) if kk == 0 else ('r', tt, kk))
            quads.append(q)
    # coordinates
    cross = {}
    for j in range(n + 1):
        for i in range(n + 1):
            cross[('c', i, j)] = np.array([g[i], g[j]])
    for t in range(4 * n):
        inner = square_xy(t)
        ang = np.arctan2(inner[1], inner[0])
        outer = R * np.array([np.cos(ang), np.sin(ang)])
        for kk in range(1, m + 1):
            s = kk / m
            cross[('r', t, kk)] = (1 - s) * inner + s * outer
    keys2 = list(cross.keys())
    idx2 = {k: i for i, k in enumerate(keys2)}
    xy = np.array([cross[k] for k in keys2])
    # jitter cross-section vertices that are not on the outer circle and not
    # on the central block's corners
    interior = np.array([not (k[0] == 'r' and k[2] == m) for k in keys2])
    h = 2 * a / n
    xy = xy + interior[:, None] * rng.uniform(-jitter * h, jitter * h, xy.shape)
    zs = np.linspace(0.0, 1.0, nz + 1)
    nv2 = len(keys2)
    V = np.zeros(((nz + 1) * nv2, 3))
    for kz in range(nz + 1):
        V[kz * nv2:(kz + 1) * nv2, :2] = xy
        V[kz * nv2:(kz + 1) * nv2, 2] = zs[kz]
    el = []
    for kz in range(nz):
        for q in quads:
            v = [idx2[k] for k in q]      # (0,0), (1,0), (0,1), (1,1) in the quad's own frame
            x0 = xy[v[0]]
            d1, d2 = xy[v[1]] - x0, xy[v[2]] - x0
            cr = d1[0] * d2[1] - d1[1] * d2[0]
            if cr < 0:                    # keep the cross-section quad counter-clockwise
                v = [v[0], v[2], v[1], v[3]]
            bot = [kz * nv2 + w for w in v]
            top = [(kz + 1) * nv2 + w for w in v]
            el.append(bot + top)
    return V, np.asarray(el, dtype=np.int64)
