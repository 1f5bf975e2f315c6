// Grey nonlinear radiation diffusion (Section 4.3): one time step of the
// three-stage L-stable SDIRK method of Alexander (1977), each stage solved by
// the outer iteration the paper describes:
//   (1) the flux F lagged, the 2 x 2 system of every L2 dof for (e_j, E_j)
//       by Newton's method (element by element, here dof by dof);
//   (2) e fixed, the Darcy-type system for (E, F), which is the library's
//       transformed Darcy system [[M, D^T], [D, -kappa W^{-1}]] with
//       c_mass = 3 sigma / c and gamma = kappa = 1 / (gamma_rk dt) + c sigma,
//       unknowns (F, q~ = -W E), solved by block-preconditioned MINRES;
// repeated until the relative residual of the material-energy equation with
// the new E falls below the outer tolerance.
//
// The energies are L2 dofs of the transformed space, whose basis functions
// are mapped with 1 / det J (D = W^{-1} B is the +-1 incidence, Section 2.1):
// a dof is the integral of the function over its sub-cell K_j, so e_j and
// E_j are energy amounts per sub-cell, the sub-cell temperature is
// T_j = e_j / (rho C_v |K_j|) and the emission term a T_j^4 |K_j|.
//
// Device work: the sub-cell volumes (2 x 2 x 2 Gauss-Legendre points of
// det J per sub-cell), D F, the stage combinations, the per-dof Newton
// solves, the Darcy right-hand side, E = -W^{-1} q~ and the residual norms
// are kernels of this file; the Darcy solves are the library's MINRES.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "hd_internal.hpp"
#include "kernels_common.hpp"

namespace hd {

// Alexander (1977): gamma is the root in (1/6, 1/2) of
// x^3 - 3 x^2 + 3 x / 2 - 1/6; stiffly accurate (the last row of A is b).
constexpr double SDIRK_G = 0.43586652150845899942;

struct RadDiffState {
    hd_rd_params prm;
    double* ws = nullptr;      // one allocation for everything below
    double* vol = nullptr;     // [n_q] sub-cell volumes |K_j|
    double* xe[3] = {nullptr, nullptr, nullptr};   // stage values e_i
    double* xE[3] = {nullptr, nullptr, nullptr};   // stage values E_i
    double* he[3] = {nullptr, nullptr, nullptr};   // their e^_i
    double* hE[3] = {nullptr, nullptr, nullptr};   // their E^_i
    double* df = nullptr;      // [n_q] D F
    double* b = nullptr;       // [n_u + n_q] Darcy right-hand side
    double* sol = nullptr;     // [n_u + n_q] Darcy solution (F, q~), the warm start
    double* q = nullptr;       // [n_u + n_q] A sol (the warm start's residual, HD_MODE_MIXED)
    double* part = nullptr;    // [3][RD_BLOCKS] residual partial sums, then 3 totals
    int* flags = nullptr;      // [0] largest Newton count, [1] Newton failure, then RD_BLOCKS per-workgroup counts
};

namespace {

constexpr int RD_BLOCKS = 1024;
constexpr int RD_T = 256;

struct Gll {
    double x[HD_MAXQ];
};

// |K_j| of every L2 dof (element-major, then a, b, c with a fastest): det J
// of the trilinear map integrated over the sub-cell by 2 x 2 x 2
// Gauss-Legendre points (det J has degree 2 in each variable).
__global__ void subcell_volume_kernel(int nx, int ny, int nz, int P, const double* __restrict__ vert,
                                      const double* __restrict__ evx, Gll gll, double* __restrict__ vol) {
    const int NL = P * P * P;
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ne * NL) return;
    const int64_t e = t / NL;
    const int l = (int)(t % NL);
    const int a = l % P, b = (l / P) % P, c = l / (P * P);
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
    double X[8][3];
    for (int v = 0; v < 8; ++v) {
        const int dx = v & 1, dy = (v >> 1) & 1, dz = v >> 2;
        if (evx) {
            for (int r = 0; r < 3; ++r) X[v][r] = evx[24 * e + 3 * v + r];
        } else {
            const int64_t g = (ex + dx) + (int64_t)(nx + 1) * ((ey + dy) + (int64_t)(ny + 1) * (ez + dz));
            for (int r = 0; r < 3; ++r) X[v][r] = vert[3 * g + r];
        }
    }
    const double g0 = 0.5 - 0.5 / sqrt(3.0), g1 = 0.5 + 0.5 / sqrt(3.0);
    const double lo[3] = {gll.x[a], gll.x[b], gll.x[c]};
    const double h[3] = {gll.x[a + 1] - gll.x[a], gll.x[b + 1] - gll.x[b], gll.x[c + 1] - gll.x[c]};
    double s = 0.0;
    for (int q = 0; q < 8; ++q) {
        double xi[3];
        for (int d = 0; d < 3; ++d) xi[d] = lo[d] + h[d] * (((q >> d) & 1) ? g1 : g0);
        double J[3][3];
        for (int r = 0; r < 3; ++r) {
            double s0 = 0, s1 = 0, s2 = 0;
            for (int v = 0; v < 8; ++v) {
                const int dx = v & 1, dy = (v >> 1) & 1, dz = v >> 2;
                const double Nx = dx ? xi[0] : 1.0 - xi[0], Ny = dy ? xi[1] : 1.0 - xi[1],
                             Nz = dz ? xi[2] : 1.0 - xi[2];
                const double gx = dx ? 1.0 : -1.0, gy = dy ? 1.0 : -1.0, gz = dz ? 1.0 : -1.0;
                s0 += gx * Ny * Nz * X[v][r];
                s1 += Nx * gy * Nz * X[v][r];
                s2 += Nx * Ny * gz * X[v][r];
            }
            J[r][0] = s0;
            J[r][1] = s1;
            J[r][2] = s2;
        }
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        s += det;
    }
    // the eight Gauss weights are 1/8 of the sub-cell's reference volume each
    vol[t] = s * (h[0] * h[1] * h[2] * 0.125);
}

// (D F)_j on a structured mesh: the flux through the upper minus the flux
// through the lower face of sub-cell j along each axis (RT dofs oriented
// along +axis).
__global__ void div_structured_kernel(Geo g, int P, const double* __restrict__ F, double* __restrict__ q,
                                      int64_t nq) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nq) return;
    const int NL = P * P * P;
    const int64_t e = j / NL;
    const int l = (int)(j % NL);
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    const int64_t gi = (int64_t)ex * P + l % P, gj = (int64_t)ey * P + (l / P) % P, gk = (int64_t)ez * P + l / (P * P);
    const int64_t Nx = (int64_t)g.nx * P, Ny = (int64_t)g.ny * P;
    const int64_t ix = g.off[0] + gi + (Nx + 1) * (gj + Ny * gk);
    const int64_t iy = g.off[1] + gi + Nx * (gj + (Ny + 1) * gk);
    const int64_t iz = g.off[2] + gi + Nx * (gj + Ny * gk);
    q[j] = (F[ix + 1] - F[ix]) + (F[iy + Nx] - F[iy]) + (F[iz + Nx * Ny] - F[iz]);
}

// (D F)_j on an unstructured mesh: the six signed face dofs of sub-cell j
// (~g where D's entry is -1).
__global__ void div_uns_kernel(const int32_t* __restrict__ rdof, const double* __restrict__ F,
                               double* __restrict__ q, int64_t nq) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nq) return;
    double s = 0.0;
    for (int k = 0; k < 6; ++k) {
        const int32_t v = rdof[6 * j + k];
        s += v < 0 ? -F[~v] : F[v];
    }
    q[j] = s;
}

// X^_i = X_n + sum_{j < i} (a_ij / gamma) (X_j - X^_j), for e and E at once
struct Combine {
    const double* xe[2];
    const double* he[2];
    const double* xE[2];
    const double* hE[2];
    double w[2];
    int nprev;
};

__global__ void combine_kernel(int64_t n, const double* __restrict__ e0, const double* __restrict__ E0, Combine cb,
                               double* __restrict__ eh, double* __restrict__ Eh) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    double se = e0[j], sE = E0[j];
    for (int k = 0; k < cb.nprev; ++k) {
        se += cb.w[k] * (cb.xe[k][j] - cb.he[k][j]);
        sE += cb.w[k] * (cb.xE[k][j] - cb.hE[k][j]);
    }
    eh[j] = se;
    Eh[j] = sE;
}

struct Phys {
    double rho_cv, c_sigma, a, gdt;
};

__device__ __forceinline__ double emission(double e, double vol, const Phys& ph) {
    const double T = e / (ph.rho_cv * vol);
    const double T2 = T * T;
    return ph.a * T2 * T2 * vol;
}

// Newton's method on the 2 x 2 system of dof j with D F fixed:
//   (e - e^) / (g dt) + c sigma (B(e) - E) = 0,
//   (E - E^) / (g dt) + (D F)_j - c sigma (B(e) - E) = 0,
// from (e^, E^), until both updates are below tol relative to the iterate.
// Only e is kept (E comes from the Darcy solve).  Grid-stride over RD_BLOCKS
// workgroups; each stores the largest iteration count it saw in nit[block]
// (no atomics on one address), a failed dof sets flags[1].
__global__ void newton_kernel(int64_t n, const double* __restrict__ eh, const double* __restrict__ Eh,
                              const double* __restrict__ df, const double* __restrict__ vol, Phys ph, double tol,
                              int max_it, double* __restrict__ e_out, int* __restrict__ nit, int* __restrict__ flags) {
    int mx = 0;
    bool bad = false;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double e0 = eh[j], E0 = Eh[j], d = df[j], v = vol[j];
        const double inv = 1.0 / ph.gdt, cs = ph.c_sigma;
        double e = e0, E = E0;
        bool conv = false;
        int its = 0;
        while (its < max_it) {
            const double B = emission(e, v, ph);
            const double dB = 4.0 * B / e;
            const double R1 = (e - e0) * inv + cs * (B - E);
            const double R2 = (E - E0) * inv + d - cs * (B - E);
            const double J11 = inv + cs * dB, J12 = -cs, J21 = -cs * dB, J22 = inv + cs;
            const double det = J11 * J22 - J12 * J21;
            const double de = (J22 * R1 - J12 * R2) / det;
            const double dE = (-J21 * R1 + J11 * R2) / det;
            e -= de;
            E -= dE;
            ++its;
            if (fabs(de) <= tol * fabs(e) && fabs(dE) <= tol * fmax(fabs(E), 1e-300)) {
                conv = true;
                break;
            }
        }
        e_out[j] = e;
        mx = max(mx, its);
        if (!conv || !(e > 0.0) || !isfinite(e)) bad = true;
    }
    if (bad) atomicOr(flags + 1, 1);
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
    __shared__ int red[RD_T / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int w = 0; w < RD_T / 64; ++w) m = max(m, red[w]);
        nit[blockIdx.x] = m;
    }
}

// flags[0] = max(flags[0], max of the RD_BLOCKS per-workgroup Newton counts)
__global__ void newton_finish_kernel(const int* __restrict__ nit, int* __restrict__ flags) {
    int m = 0;
    for (int b = threadIdx.x; b < RD_BLOCKS; b += 64) m = max(m, nit[b]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if (threadIdx.x == 0) flags[0] = max(flags[0], m);
}

// b = [0; E^ / (g dt) + c sigma B(e)]
__global__ void darcy_rhs_kernel(int64_t nu, int64_t nq, const double* __restrict__ e, const double* __restrict__ Eh,
                                 const double* __restrict__ vol, Phys ph, double* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nu) {
        b[i] = 0.0;
    } else if (i < nu + nq) {
        const int64_t j = i - nu;
        b[i] = Eh[j] / ph.gdt + ph.c_sigma * emission(e[j], vol[j], ph);
    }
}

__global__ void negate_kernel(double* __restrict__ x, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = -x[i];
}

__global__ void copy_kernel(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

// Per-workgroup partial sums over a grid-stride range of ||R1||^2,
// ||e - e^||^2 and ||E||^2 with R1 = (e - e^) / (g dt) + c sigma (B(e) - E)
__global__ void resid_kernel(int64_t n, const double* __restrict__ e, const double* __restrict__ E,
                             const double* __restrict__ eh, const double* __restrict__ vol, Phys ph,
                             double* __restrict__ part) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double d = e[j] - eh[j];
        const double R = d / ph.gdt + ph.c_sigma * (emission(e[j], vol[j], ph) - E[j]);
        s[0] += R * R;
        s[1] += d * d;
        s[2] += E[j] * E[j];
    }
    __shared__ double red[3][RD_T / 64];
    for (int k = 0; k < 3; ++k) {
        const double w = wave_sum(s[k]);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < RD_T / 64; ++w) t += red[threadIdx.x][w];
        part[threadIdx.x * RD_BLOCKS + blockIdx.x] = t;
    }
}

// Per-workgroup partial sums of ||b - q||^2 and ||b||^2 (slots 0 and 1 of
// the residual layout; slot 2 zeroed)
__global__ void res0_kernel(int64_t n, const double* __restrict__ b, const double* __restrict__ q,
                            double* __restrict__ part) {
    double s0 = 0.0, s1 = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double d = b[j] - q[j];
        s0 += d * d;
        s1 += b[j] * b[j];
    }
    __shared__ double red[2][RD_T / 64];
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double t = 0.0;
        for (int w = 0; w < RD_T / 64; ++w) t += red[threadIdx.x][w];
        part[threadIdx.x * RD_BLOCKS + blockIdx.x] = t;
    }
    if (threadIdx.x == 2) part[2 * RD_BLOCKS + blockIdx.x] = 0.0;
}

// the three totals, each over the RD_BLOCKS partials in a fixed order
__global__ void resid_finish_kernel(double* __restrict__ part) {
    const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double t = 0.0;
    if (k < 3)
        for (int b = lane; b < RD_BLOCKS; b += 64) t += part[k * RD_BLOCKS + b];
    t = wave_sum(t);
    if (k < 3 && lane == 0) part[3 * RD_BLOCKS + k] = t;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + RD_T - 1) / RD_T); }

}  // namespace

void rd_free(hd_ctx* c) {
    if (!c->rd) return;
    dfree(c->rd->ws);
    dfree(c->rd->flags);
    delete c->rd;
    c->rd = nullptr;
}

int launch_divergence(hd_ctx* c, const double* F, double* q) {
    if (c->n_q == 0) return HD_OK;
    if (c->unstructured)
        hipLaunchKernelGGL(div_uns_kernel, dim3(nblk(c->n_q)), dim3(RD_T), 0, c->stream, c->d_rdof, F, q, c->n_q);
    else
        hipLaunchKernelGGL(div_structured_kernel, dim3(nblk(c->n_q)), dim3(RD_T), 0, c->stream, geo_of(c), c->p, F, q,
                           c->n_q);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int launch_subcell_volumes(hd_ctx* c, double* vol) {
    Gll g;
    std::memset(&g, 0, sizeof(g));
    for (int i = 0; i <= c->p; ++i) g.x[i] = c->tab64_host.gll[i];
    if (c->n_q == 0) return HD_OK;
    hipLaunchKernelGGL(subcell_volume_kernel, dim3(nblk(c->n_q)), dim3(RD_T), 0, c->stream, c->nx, c->ny, c->nz,
                       c->p, c->d_vert, c->unstructured ? c->d_evx : nullptr, g, vol);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int rd_setup(hd_ctx* c, const hd_rd_params& prm, const hd_precond_params* pp) {
    rd_free(c);
    const int64_t ne = c->ne, nu = c->n_u, nq = c->n_q;
    const double kappa = 1.0 / (SDIRK_G * prm.dt) + prm.c * prm.sigma;
    std::vector<double> cm(ne, 3.0 * prm.sigma / prm.c), kap(ne, kappa);
    int rc = hd_setup_coeffs(c, HD_DARCY, cm.data(), kap.data(), HD_SIDE_ALL);
    if (rc) return rc;
    rc = hd_build_precond(c, pp);
    if (rc < 0) return rc;
    RadDiffState* s = new (std::nothrow) RadDiffState;
    if (!s) return set_err(c, HD_ERR_OOM, "radiation-diffusion state");
    s->prm = prm;
    const int64_t n = 14 * nq + 3 * (nu + nq) + 4 * RD_BLOCKS;
    s->ws = dalloc<double>(n);
    s->flags = dalloc<int>(4 + RD_BLOCKS);
    if (!s->ws || !s->flags) {
        dfree(s->ws);
        dfree(s->flags);
        delete s;
        return set_err(c, HD_ERR_OOM, "radiation-diffusion work space");
    }
    double* p = s->ws;
    s->vol = p;
    p += nq;
    for (int i = 0; i < 3; ++i) {
        s->xe[i] = p;
        p += nq;
        s->xE[i] = p;
        p += nq;
        s->he[i] = p;
        p += nq;
        s->hE[i] = p;
        p += nq;
    }
    s->df = p;
    p += nq;
    s->b = p;
    p += nu + nq;
    s->sol = p;
    p += nu + nq;
    s->q = p;
    p += nu + nq;
    s->part = p;
    c->rd = s;
    HD_HIP(c, hipMemsetAsync(s->flags, 0, 4 * sizeof(int), c->stream));
    HD_HIP(c, hipMemsetAsync(s->part, 0, 4 * RD_BLOCKS * sizeof(double), c->stream));
    if ((rc = launch_subcell_volumes(c, s->vol))) return rc;
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return rc;
}

int rd_step(hd_ctx* c, double* e, double* E, double* F, hd_rd_info* info) {
    RadDiffState& s = *c->rd;
    const hd_rd_params& P = s.prm;
    const int64_t nu = c->n_u, nq = c->n_q;
    const double g = SDIRK_G, gdt = g * P.dt;
    // the Butcher tableau of Alexander's method (stiffly accurate)
    const double b1 = -(6 * g * g - 16 * g + 1) / 4, b2 = (6 * g * g - 20 * g + 5) / 4;
    const double A[3][3] = {{g, 0, 0}, {(1 - g) / 2, g, 0}, {b1, b2, g}};
    const Phys ph{P.rho * P.cv, P.c * P.sigma, P.a, gdt};
    hd_rd_info inf;
    std::memset(&inf, 0, sizeof(inf));
    const auto t0 = std::chrono::steady_clock::now();
    HD_HIP(c, hipMemsetAsync(s.flags, 0, 4 * sizeof(int), c->stream));
    // warm start of the first Darcy solve: (F_n, 0)
    hipLaunchKernelGGL(copy_kernel, dim3(nblk(nu)), dim3(RD_T), 0, c->stream, F, s.sol, nu);
    HD_HIP(c, hipMemsetAsync(s.sol + nu, 0, sizeof(double) * nq, c->stream));
    hd_solve_params lp;
    lp.tol = P.lin_tol;
    lp.max_it = P.lin_max_it;
    lp.mode = P.lin_mode;
    lp.use_x0 = 1;
    lp.inner_tol = 1e-5;
    lp.max_outer = 20;
    lp.check_every = 8;
    lp.stop_true = 0;
    lp.use_graph = 1;
    int status = HD_OK;
    for (int i = 0; i < 3; ++i) {
        Combine cb;
        std::memset(&cb, 0, sizeof(cb));
        cb.nprev = i;
        for (int j = 0; j < i; ++j) {
            cb.xe[j] = s.xe[j];
            cb.he[j] = s.he[j];
            cb.xE[j] = s.xE[j];
            cb.hE[j] = s.hE[j];
            cb.w[j] = A[i][j] / g;
        }
        hipLaunchKernelGGL(combine_kernel, dim3(nblk(nq)), dim3(RD_T), 0, c->stream, nq, e, E, cb, s.he[i], s.hE[i]);
        HD_HIP(c, hipGetLastError());
        int k = 0;
        double res = 0.0;
        for (; k < P.max_outer;) {
            int rc = launch_divergence(c, s.sol, s.df);
            if (rc) return rc;
            hipLaunchKernelGGL(newton_kernel, dim3(RD_BLOCKS), dim3(RD_T), 0, c->stream, nq, s.he[i], s.hE[i], s.df,
                               s.vol, ph, P.newton_tol, P.newton_max_it, s.xe[i], s.flags + 4, s.flags);
            hipLaunchKernelGGL(newton_finish_kernel, dim3(1), dim3(64), 0, c->stream, (const int*)(s.flags + 4),
                               s.flags);
            hipLaunchKernelGGL(darcy_rhs_kernel, dim3(nblk(nu + nq)), dim3(RD_T), 0, c->stream, nu, nq, s.xe[i],
                               s.hE[i], s.vol, ph, s.b);
            HD_HIP(c, hipGetLastError());
            if (P.lin_mode == HD_MODE_MIXED) {
                // the mixed solve stops on the true residual relative to
                // ||b||: ask for lin_tol times the warm start's own
                if ((rc = launch_apply(c, HD_F64, 1, s.sol, s.q, nullptr, 0, nullptr, 0, ESS_IDENTITY, nullptr, 0)))
                    return rc;
                hipLaunchKernelGGL(res0_kernel, dim3(RD_BLOCKS), dim3(RD_T), 0, c->stream, nu + nq, s.b, s.q, s.part);
                hipLaunchKernelGGL(resid_finish_kernel, dim3(1), dim3(256), 0, c->stream, s.part);
                HD_HIP(c, hipGetLastError());
                double h0[2];
                HD_HIP(c, hipMemcpyAsync(h0, s.part + 3 * RD_BLOCKS, sizeof(h0), hipMemcpyDeviceToHost, c->stream));
                HD_HIP(c, hipStreamSynchronize(c->stream));
                const double rel0 = h0[1] > 0.0 ? std::sqrt(h0[0] / h0[1]) : 0.0;
                lp.tol = std::max(P.lin_tol * rel0, 1e-13);   // above the FP64 round-off of r
            }
            hd_solve_info si;
            rc = minres_solve(c, lp, 1, s.b, s.sol, &si);
            if (rc < 0) return rc;
            if (rc == HD_NOT_CONVERGED) status = HD_NOT_CONVERGED;
            inf.linear_solves += 1;
            inf.linear_iterations += si.iterations;
            inf.linear_time_s += si.time_s;
            // E = -W^{-1} q~
            if ((rc = launch_mass_inverse(c, HD_F64, s.sol + nu, s.xE[i], false))) return rc;
            hipLaunchKernelGGL(negate_kernel, dim3(nblk(nq)), dim3(RD_T), 0, c->stream, s.xE[i], nq);
            hipLaunchKernelGGL(resid_kernel, dim3(RD_BLOCKS), dim3(RD_T), 0, c->stream, nq, s.xe[i], s.xE[i],
                               s.he[i], s.vol, ph, s.part);
            hipLaunchKernelGGL(resid_finish_kernel, dim3(1), dim3(256), 0, c->stream, s.part);
            HD_HIP(c, hipGetLastError());
            double h[3];
            HD_HIP(c, hipMemcpyAsync(h, s.part + 3 * RD_BLOCKS, sizeof(h), hipMemcpyDeviceToHost, c->stream));
            HD_HIP(c, hipStreamSynchronize(c->stream));
            const double scale = std::sqrt(h[1]) / gdt + P.c * P.sigma * std::sqrt(h[2]) + 1e-300;
            res = std::sqrt(h[0]) / scale;
            ++k;
            if (!std::isfinite(res)) return set_err(c, HD_ERR_NONFINITE, "non-finite residual in a stage");
            if (res <= P.tol_outer) break;
        }
        inf.outer[i] = k;
        inf.e_residual[i] = res;
        if (res > P.tol_outer) status = HD_NOT_CONVERGED;
    }
    int fl[2];
    HD_HIP(c, hipMemcpyAsync(fl, s.flags, sizeof(fl), hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    inf.newton_max_it = fl[0];
    if (fl[1]) {
        // the caller's state stays as it was
        if (info) *info = inf;
        return set_err(c, HD_ERR_NONFINITE, "Newton did not converge to a positive energy in some dof");
    }
    // the new state is the last stage (stiffly accurate)
    hipLaunchKernelGGL(copy_kernel, dim3(nblk(nq)), dim3(RD_T), 0, c->stream, s.xe[2], e, nq);
    hipLaunchKernelGGL(copy_kernel, dim3(nblk(nq)), dim3(RD_T), 0, c->stream, s.xE[2], E, nq);
    hipLaunchKernelGGL(copy_kernel, dim3(nblk(nu)), dim3(RD_T), 0, c->stream, s.sol, F, nu);
    HD_HIP(c, hipGetLastError());
    HD_HIP(c, hipStreamSynchronize(c->stream));
    inf.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    inf.status = status;
    if (info) *info = inf;
    if (status == HD_NOT_CONVERGED) c->err = "an outer iteration or a Darcy solve reached its limit";
    return status;
}

}  // namespace hd
