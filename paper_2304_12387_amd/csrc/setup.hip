// Setup kernels: geometric factors at quadrature points (partial assembly),
// the diagonals diag(M) and diag(W) by squared-basis sum factorisation
// (Section 3.2), the approximate Schur complement S~ assembled row by row from
// eq. (approx-schur-entries), and deterministic reductions and scans.
#include "kernels_common.hpp"

#include <type_traits>

namespace hd {

namespace {

// ---------------------------------------------------------------------------
// geometry: one thread per (element, point); points are the q^3 quadrature
// points followed by the 8 vertices.  Writes w J^T J / det J (6 entries) and
// w / det J per quadrature point, flags det J <= 0 (or non-finite).
// ---------------------------------------------------------------------------
// With evx (unstructured meshes) the element's vertices are read from
// evx[e][v][r], v = dx + 2 dy + 4 dz, instead of the structured grid.
__global__ void geometry_kernel(int nx, int ny, int nz, int P, const double* __restrict__ vert,
                                const double* __restrict__ evx, const Tables<double>* __restrict__ tab,
                                double* __restrict__ pa, float* __restrict__ pa32, int* __restrict__ bad) {
    const int Q = P + 1, Q3 = Q * Q * Q, NP = Q3 + 8;
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ne * NP) return;
    const int64_t e = t / NP;
    const int pt = (int)(t % NP);
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
    double X[2][2][2][3];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                if (evx) {
                    for (int r = 0; r < 3; ++r) X[dz][dy][dx][r] = evx[24 * e + 3 * (dx + 2 * dy + 4 * dz) + r];
                    continue;
                }
                const int64_t v = (ex + dx) + (int64_t)(nx + 1) * ((ey + dy) + (int64_t)(ny + 1) * (ez + dz));
                for (int r = 0; r < 3; ++r) X[dz][dy][dx][r] = vert[3 * v + r];
            }
    double xi[3], w = 1.0;
    if (pt < Q3) {
        const int a = pt % Q, b = (pt / Q) % Q, c = pt / (Q * Q);
        xi[0] = tab->xq[a];
        xi[1] = tab->xq[b];
        xi[2] = tab->xq[c];
        w = tab->wq[a] * tab->wq[b] * tab->wq[c];
    } else {
        const int v = pt - Q3;
        xi[0] = v & 1;
        xi[1] = (v >> 1) & 1;
        xi[2] = (v >> 2) & 1;
    }
    // J[r][d] = d x_r / d xi_d of the trilinear map
    double J[3][3];
    for (int r = 0; r < 3; ++r) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const double Nx = dx ? xi[0] : 1.0 - xi[0], Ny = dy ? xi[1] : 1.0 - xi[1],
                                 Nz = dz ? xi[2] : 1.0 - xi[2];
                    const double gx = dx ? 1.0 : -1.0, gy = dy ? 1.0 : -1.0, gz = dz ? 1.0 : -1.0;
                    const double Xv = X[dz][dy][dx][r];
                    s0 += gx * Ny * Nz * Xv;
                    s1 += Nx * gy * Nz * Xv;
                    s2 += Nx * Ny * gz * Xv;
                }
        J[r][0] = s0;
        J[r][1] = s1;
        J[r][2] = s2;
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0) || !isfinite(det)) *bad = 1;
    if (pt >= Q3) return;
    double G[6];
    const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
    for (int m = 0; m < 6; ++m) {
        double s = 0;
        for (int r = 0; r < 3; ++r) s += J[r][rr[m]] * J[r][cc[m]];
        G[m] = w * s / det;
    }
    double* pe = pa + (size_t)e * NPA * Q3;
    float* pe32 = pa32 + (size_t)e * NPA * Q3;
    for (int m = 0; m < 6; ++m) {
        pe[m * Q3 + pt] = G[m];
        pe32[m * Q3 + pt] = (float)G[m];
    }
    pe[6 * Q3 + pt] = w / det;
    pe32[6 * Q3 + pt] = (float)(w / det);
}

// ---------------------------------------------------------------------------
// diagonals: one wavefront per element.  diag(M_e) for the x-component dof
// (i, j, k) is c_mass sum_{abc} G00 L(a,i)^2 H(b,j)^2 H(c,k)^2 (y, z by
// permutation with G11, G22); diag(W_e) is sum gw H^2 H^2 H^2.  RT entries
// are added into the zero-initialised global diagonal (at most two
// contributions per dof, so the result does not depend on their order).
// ---------------------------------------------------------------------------
// With theta (per element (x-, x+, y-, y+, z-, z+) log-scalings) each local
// diagonal entry is multiplied by exp((1 - xi_i) theta_{2c} + xi_i theta_{2c+1})
// before it is added (the learned correction of the (1,1) block).
// On unstructured meshes (l2g given) the entries are added through the
// element-to-dof map instead.
template <int P>
__global__ __launch_bounds__(64) void diag_kernel(Geo g, const double* __restrict__ pa,
                                                  const Tables<double>* __restrict__ tab,
                                                  const double* __restrict__ cm, const double* __restrict__ theta,
                                                  const int32_t* __restrict__ l2g, double* __restrict__ mdiag,
                                                  double* __restrict__ wdiag) {
    using D = Dim<P>;
    constexpr int Q = D::Q, Q3 = D::Q3, NL = D::NL, NC = D::NC;
    __shared__ double sL2[Q * (P + 1)], sH2[Q * P], in[Q3], b1[Q3], b2[Q3], loc[NC];
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    for (int i = tid; i < Q * (P + 1); i += 64) sL2[i] = tab->L2[i / (P + 1)][i % (P + 1)];
    for (int i = tid; i < Q * P; i += 64) sH2[i] = tab->H2[i / P][i % P];
    const double* pe = pa + (size_t)e * NPA * Q3;
    const double c = cm[e];
    const int gidx_comp[3] = {0, 3, 5};
    for (int comp = 0; comp < 3; ++comp) {
        __syncthreads();
        for (int qd = tid; qd < Q3; qd += 64) in[qd] = pe[gidx_comp[comp] * Q3 + qd];
        __syncthreads();
        if (comp == 0) {
            contract<double, Q, Q, Q, 2, P, true, P>(in, b1, sH2, tid, 64);
            __syncthreads();
            contract<double, Q, Q, P, 1, P, true, P>(b1, b2, sH2, tid, 64);
            __syncthreads();
            contract<double, Q, P, P, 0, P + 1, true, P + 1>(b2, loc, sL2, tid, 64);
        } else if (comp == 1) {
            contract<double, Q, Q, Q, 2, P, true, P>(in, b1, sH2, tid, 64);
            __syncthreads();
            contract<double, Q, Q, P, 1, P + 1, true, P + 1>(b1, b2, sL2, tid, 64);
            __syncthreads();
            contract<double, Q, P + 1, P, 0, P, true, P>(b2, loc, sH2, tid, 64);
        } else {
            contract<double, Q, Q, Q, 2, P + 1, true, P + 1>(in, b1, sL2, tid, 64);
            __syncthreads();
            contract<double, Q, Q, P + 1, 1, P, true, P>(b1, b2, sH2, tid, 64);
            __syncthreads();
            contract<double, Q, P, P + 1, 0, P, true, P>(b2, loc, sH2, tid, 64);
        }
        __syncthreads();
        for (int l = tid; l < NC; l += 64) {
            int i, j, k, onf, bs;
            local_ijk<P>(comp, l, i, j, k);
            if (l2g) {
                const int32_t m = l2g[e * D::NRT + comp * NC + l];
                atomicAdd(&mdiag[m < 0 ? ~m : m], c * loc[l]);
                continue;
            }
            const int64_t gi = rt_global<P>(g, comp, ex, ey, ez, i, j, k, onf, bs);
            double v = c * loc[l];
            if (theta) {
                const double xi = tab->gll[comp == 0 ? i : (comp == 1 ? j : k)];
                v *= exp((1.0 - xi) * theta[e * 6 + 2 * comp] + xi * theta[e * 6 + 2 * comp + 1]);
            }
            if (!onf || bs >= 0) mdiag[gi] = v;
            else atomicAdd(&mdiag[gi], v);
        }
    }
    // diag(W_e)
    __syncthreads();
    for (int qd = tid; qd < Q3; qd += 64) in[qd] = pe[6 * Q3 + qd];
    __syncthreads();
    contract<double, Q, Q, Q, 2, P, true, P>(in, b1, sH2, tid, 64);
    __syncthreads();
    contract<double, Q, Q, P, 1, P, true, P>(b1, b2, sH2, tid, 64);
    __syncthreads();
    contract<double, Q, P, P, 0, P, true, P>(b2, in, sH2, tid, 64);
    __syncthreads();
    for (int l = tid; l < NL; l += 64) wdiag[e * NL + l] = in[l];
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ y, T v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

// essential dofs of diag(M) -> 1; inverse of tau diag(M) in FP64 and FP32;
// coupling weight 1/M~_kk of every free face shared by two sub-volumes (0 on
// essential and domain-boundary faces), the off-diagonal magnitude of S~
__global__ void mdiag_finish_kernel(Geo g, int P, uint32_t ess, double tau, double* __restrict__ mdiag,
                                    double* __restrict__ mdinv, float* __restrict__ mdinv32,
                                    double* __restrict__ wface, int64_t n_u) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_u) return;
    const int c = t >= g.off[2] ? 2 : (t >= g.off[1] ? 1 : 0);
    const int64_t r = t - g.off[c];
    const int64_t d0 = (int64_t)g.nx * P + (c == 0), d1 = (int64_t)g.ny * P + (c == 1);
    const int64_t coord = c == 0 ? r % d0 : (c == 1 ? (r / d0) % d1 : r / (d0 * d1));
    const int64_t nal = c == 0 ? (int64_t)g.nx * P : (c == 1 ? (int64_t)g.ny * P : (int64_t)g.nz * P);
    const bool boundary = coord == 0 || coord == nal;
    if (rt_is_essential(g, P, ess, t)) {
        mdiag[t] = 1.0;
        mdinv[t] = 1.0;
        mdinv32[t] = 1.0f;
        wface[t] = 0.0;
    } else {
        const double m = mdiag[t];
        mdinv[t] = 1.0 / (tau * m);
        mdinv32[t] = (float)(1.0 / (tau * m));
        wface[t] = boundary ? 0.0 : 1.0 / m;
    }
}

// the same on an unstructured mesh: essential dofs from the mask; the face
// weights are not used there (level 0 of the V-cycle is a CSR level)
__global__ void mdiag_finish_uns_kernel(const uint8_t* __restrict__ essm, double tau, double* __restrict__ mdiag,
                                        double* __restrict__ mdinv, float* __restrict__ mdinv32,
                                        double* __restrict__ wface, int64_t n_u) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_u) return;
    wface[t] = 0.0;
    if (essm[t]) {
        mdiag[t] = 1.0;
        mdinv[t] = 1.0;
        mdinv32[t] = 1.0f;
    } else {
        const double m = mdiag[t];
        mdinv[t] = 1.0 / (tau * m);
        mdinv32[t] = (float)(1.0 / (tau * m));
    }
}

// ---------------------------------------------------------------------------
// S~ rows.  Row i = sub-volume (a, b, c) of element e.  For each of its six
// faces k: if k is free, the diagonal gains 1/M~_kk and the neighbour volume
// across k (if any) gets the off-diagonal -1/M~_kk; C~_ii = kappa_e / W_ii, or
// ctil[i] when given (Darcy with a gamma field).
// ---------------------------------------------------------------------------
struct RowEnt {
    int32_t col;
    double val;
};

__device__ int schur_row(Geo g, int P, uint32_t ess, int64_t i, const double* __restrict__ mdiag,
                         const double* __restrict__ wdiag, const double* __restrict__ kap,
                         const double* __restrict__ ctil, RowEnt* ent) {
    const int NL = P * P * P;
    const int64_t e = i / NL;
    const int l = (int)(i % NL);
    const int loc[3] = {l % P, (l / P) % P, l / (P * P)};
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    const int eidx[3] = {ex, ey, ez};
    const int ndim[3] = {g.nx, g.ny, g.nz};
    const int64_t estride[3] = {1, g.nx, (int64_t)g.nx * g.ny};
    const int lstride[3] = {1, P, P * P};
    double diag = ctil ? ctil[i] : kap[e] / wdiag[i];
    int n = 0;
    for (int c = 0; c < 3; ++c) {
        for (int side = 0; side < 2; ++side) {
            // face index along c: loc[c] (lower) or loc[c] + 1 (upper)
            const int t = loc[c] + side;
            const int64_t gcoord = (int64_t)eidx[c] * P + t;
            const int64_t nal = (int64_t)ndim[c] * P;
            const bool on_bnd = gcoord == 0 || gcoord == nal;
            const int bside = gcoord == 0 ? 0 : 1;
            if (on_bnd && ((ess >> (2 * c + bside)) & 1u)) continue;   // essential face
            // global RT index of the face
            int ii = loc[0], jj = loc[1], kk = loc[2];
            if (c == 0) ii = t; else if (c == 1) jj = t; else kk = t;
            const int gi = ex * P + ii, gj = ey * P + jj, gkk = ez * P + kk;
            const int64_t d0 = (int64_t)g.nx * P + (c == 0), d1 = (int64_t)g.ny * P + (c == 1);
            const int64_t gk = g.off[c] + gi + d0 * (gj + d1 * gkk);
            const double wk = 1.0 / mdiag[gk];
            diag += wk;
            if (on_bnd) continue;
            int64_t nb;
            if (side == 0) {
                nb = loc[c] > 0 ? i - lstride[c] : (e - estride[c]) * NL + (l + (P - 1) * lstride[c]);
            } else {
                nb = loc[c] < P - 1 ? i + lstride[c] : (e + estride[c]) * NL + (l - (P - 1) * lstride[c]);
            }
            ent[n].col = (int32_t)nb;
            ent[n].val = -wk;
            ++n;
        }
    }
    ent[n].col = (int32_t)i;
    ent[n].val = diag;
    ++n;
    // insertion sort by column
    for (int a = 1; a < n; ++a) {
        RowEnt x = ent[a];
        int b = a - 1;
        while (b >= 0 && ent[b].col > x.col) {
            ent[b + 1] = ent[b];
            --b;
        }
        ent[b + 1] = x;
    }
    return n;
}

// Row i of S~ on an unstructured mesh, from its six (signed RT dof,
// neighbour) slots: S~_ij = sum over the free dofs k shared by i and j of
// D_ik D_jk / M~_kk (the product is -1 for the two sub-volumes of a face),
// C~_ii on the diagonal.  Columns sorted; repeated columns summed.
__device__ int schur_row_uns(int64_t i, const int32_t* __restrict__ rdof, const int32_t* __restrict__ rnbr,
                             const uint8_t* __restrict__ essm, int NL, const double* __restrict__ mdiag,
                             const double* __restrict__ wdiag, const double* __restrict__ kap,
                             const double* __restrict__ ctil, RowEnt* ent) {
    double diag = ctil ? ctil[i] : kap[i / NL] / wdiag[i];
    int n = 0;
    for (int sl = 0; sl < 6; ++sl) {
        const int32_t v = rdof[6 * i + sl];
        const int32_t k = v < 0 ? ~v : v;
        if (essm[k]) continue;
        const double wk = 1.0 / mdiag[k];
        diag += wk;
        const int32_t j = rnbr[6 * i + sl];
        if (j < 0) continue;
        // sign of D_jk: the slot of j that holds k
        double sj = 0.0;
        for (int s2 = 0; s2 < 6; ++s2) {
            const int32_t w = rdof[6 * (int64_t)j + s2];
            if ((w < 0 ? ~w : w) == k) sj = w < 0 ? -1.0 : 1.0;
        }
        const double si = v < 0 ? -1.0 : 1.0;
        ent[n].col = j;
        ent[n].val = si * sj * wk;
        ++n;
    }
    ent[n].col = (int32_t)i;
    ent[n].val = diag;
    ++n;
    for (int a = 1; a < n; ++a) {
        RowEnt x = ent[a];
        int b = a - 1;
        while (b >= 0 && ent[b].col > x.col) {
            ent[b + 1] = ent[b];
            --b;
        }
        ent[b + 1] = x;
    }
    int m = 0;
    for (int a = 0; a < n; ++a) {
        if (m > 0 && ent[m - 1].col == ent[a].col) ent[m - 1].val += ent[a].val;
        else ent[m++] = ent[a];
    }
    return m;
}

__global__ void schur_uns_kernel(int64_t nq, int NL, const int32_t* __restrict__ rdof,
                                 const int32_t* __restrict__ rnbr, const uint8_t* __restrict__ essm,
                                 const double* __restrict__ mdiag, const double* __restrict__ wdiag,
                                 const double* __restrict__ kap, const double* __restrict__ ctil,
                                 int32_t* __restrict__ cnt, const int32_t* __restrict__ rp, int32_t* __restrict__ ci,
                                 double* __restrict__ v, float* __restrict__ v32, double* __restrict__ sdiag,
                                 float* __restrict__ sdiag32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    RowEnt ent[7];
    const int n = schur_row_uns(i, rdof, rnbr, essm, NL, mdiag, wdiag, kap, ctil, ent);
    if (cnt) {
        cnt[i] = n;
        return;
    }
    const int32_t o = rp[i];
    for (int k = 0; k < n; ++k) {
        ci[o + k] = ent[k].col;
        v[o + k] = ent[k].val;
        v32[o + k] = (float)ent[k].val;
        if (ent[k].col == (int32_t)i) {
            sdiag[i] = ent[k].val;
            sdiag32[i] = (float)ent[k].val;
        }
    }
}

__global__ void schur_count_kernel(Geo g, int P, uint32_t ess, int64_t nq, const double* __restrict__ mdiag,
                                   const double* __restrict__ wdiag, const double* __restrict__ kap,
                                   const double* __restrict__ ctil, int32_t* __restrict__ cnt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    RowEnt ent[7];
    cnt[i] = schur_row(g, P, ess, i, mdiag, wdiag, kap, ctil, ent);
}

__global__ void schur_fill_kernel(Geo g, int P, uint32_t ess, int64_t nq, const double* __restrict__ mdiag,
                                  const double* __restrict__ wdiag, const double* __restrict__ kap,
                                  const double* __restrict__ ctil, const int32_t* __restrict__ rp, int32_t* __restrict__ ci, double* __restrict__ v,
                                  float* __restrict__ v32, double* __restrict__ sdiag, float* __restrict__ sdiag32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    RowEnt ent[7];
    const int n = schur_row(g, P, ess, i, mdiag, wdiag, kap, ctil, ent);
    const int32_t o = rp[i];
    for (int k = 0; k < n; ++k) {
        ci[o + k] = ent[k].col;
        v[o + k] = ent[k].val;
        v32[o + k] = (float)ent[k].val;
        if (ent[k].col == (int32_t)i) {
            sdiag[i] = ent[k].val;
            sdiag32[i] = (float)ent[k].val;
        }
    }
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts into an int32 row pointer (n + 1 entries)
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_PER = 8, SCAN_CH = SCAN_T * SCAN_PER;

__global__ void scan_sums_kernel(const int32_t* __restrict__ cnt, int64_t n, int64_t* __restrict__ bsum) {
    __shared__ int64_t s[SCAN_T];
    const int64_t base = blockIdx.x * (int64_t)SCAN_CH + threadIdx.x * SCAN_PER;
    int64_t acc = 0;
    for (int k = 0; k < SCAN_PER; ++k)
        if (base + k < n) acc += cnt[base + k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = SCAN_T / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

// exclusive scan of nb block sums in place, single block of 1024 threads
__global__ void scan_bsums_kernel(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ total) {
    __shared__ int64_t s[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = t * per, hi = lo + per < nb ? lo + per : nb;
    int64_t acc = 0;
    for (int64_t k = lo; k < hi; ++k) acc += bsum[k];
    s[t] = acc;
    __syncthreads();
    // Hillis-Steele inclusive scan
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? s[t - 1] : 0;
    for (int64_t k = lo; k < hi; ++k) {
        int64_t v = bsum[k];
        bsum[k] = run;
        run += v;
    }
    if (t == 1023) *total = s[1023];
}

__global__ void scan_final_kernel(const int32_t* __restrict__ cnt, int64_t n, const int64_t* __restrict__ bsum,
                                  const int64_t* __restrict__ total, int32_t* __restrict__ out) {
    __shared__ int64_t s[SCAN_T];
    const int t = threadIdx.x;
    const int64_t base = blockIdx.x * (int64_t)SCAN_CH + t * SCAN_PER;
    int64_t v[SCAN_PER];
    int64_t acc = 0;
    for (int k = 0; k < SCAN_PER; ++k) {
        v[k] = base + k < n ? cnt[base + k] : 0;
        acc += v[k];
    }
    s[t] = acc;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int64_t w = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += w;
        __syncthreads();
    }
    int64_t run = bsum[blockIdx.x] + (t > 0 ? s[t - 1] : 0);
    for (int k = 0; k < SCAN_PER; ++k) {
        if (base + k < n) out[base + k] = (int32_t)run;
        run += v[k];
    }
    if (blockIdx.x == 0 && t == 0) out[n] = (int32_t)*total;
}

// deterministic sum of n partials into out[0] (one block, fixed order)
__global__ void reduce_kernel(const double* __restrict__ part, int64_t n, double* __restrict__ out) {
    __shared__ double s[1024];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int64_t k = t; k < n; k += 1024) acc += part[k];
    s[t] = acc;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (t < off) s[t] += s[t + off];
        __syncthreads();
    }
    if (t == 0) *out = s[0];
}

template <int P>
void launch_diag_p(hd_ctx* c, Geo g, const double* theta) {
    hipLaunchKernelGGL((diag_kernel<P>), dim3((unsigned)c->ne), dim3(64), 0, c->stream, g, c->d_pa, c->d_tab64,
                       c->d_cm, theta, c->unstructured ? c->d_l2g : nullptr, c->d_mdiag, c->d_wdiag);
}

// ---------------------------------------------------------------------------
// RT interpolant of a constant field u: every dof is the flux of u through
// its sub-element face (the face dofs of the interpolation-histopolation
// basis, Section 2.1), oriented along +axis.  A sub-face is a bilinear patch
// of its element's trilinear map, whose vector area is half the cross product
// of its diagonals, so the flux u . area is exact on any mesh of the class.
// ---------------------------------------------------------------------------
__device__ void map_point(const double (&X)[8][3], double a, double b, double cc, double (&out)[3]) {
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int v = 0; v < 8; ++v) {
            const int dx = v & 1, dy = (v >> 1) & 1, dz = (v >> 2) & 1;
            s += (dx ? a : 1.0 - a) * (dy ? b : 1.0 - b) * (dz ? cc : 1.0 - cc) * X[v][r];
        }
        out[r] = s;
    }
}

__global__ void constant_flux_kernel(Geo g, int P, const double* __restrict__ vert,
                                     const Tables<double>* __restrict__ tab, double u0, double u1, double u2,
                                     int64_t n_u, double* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_u) return;
    const int c = t >= g.off[2] ? 2 : (t >= g.off[1] ? 1 : 0);
    const int64_t r = t - g.off[c];
    const int ne[3] = {g.nx, g.ny, g.nz};
    int64_t dim[3] = {(int64_t)g.nx * P, (int64_t)g.ny * P, (int64_t)g.nz * P};
    dim[c] += 1;
    const int64_t I[3] = {r % dim[0], (r / dim[0]) % dim[1], r / (dim[0] * dim[1])};
    int e[3], loc[3];
    for (int d = 0; d < 3; ++d) {
        e[d] = (int)(I[d] / P);
        if (e[d] >= ne[d]) e[d] = ne[d] - 1;   // the last face belongs to the last element
        loc[d] = (int)(I[d] - (int64_t)e[d] * P);
    }
    double X[8][3];
    for (int v = 0; v < 8; ++v) {
        const int dx = v & 1, dy = (v >> 1) & 1, dz = (v >> 2) & 1;
        const int64_t gv = (e[0] + dx) + (int64_t)(g.nx + 1) * ((e[1] + dy) + (int64_t)(g.ny + 1) * (e[2] + dz));
        for (int q = 0; q < 3; ++q) X[v][q] = vert[3 * gv + q];
    }
    // tangential directions (a, b) with (c, a, b) cyclic, so a x b is +c
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = tab->gll[loc[d]];
        hi[d] = d == c ? lo[d] : tab->gll[loc[d] + 1];
    }
    double x00[3], x11[3], x01[3], x10[3], p[3];
    p[c] = lo[c];
    p[a] = lo[a]; p[b] = lo[b]; map_point(X, p[0], p[1], p[2], x00);
    p[a] = hi[a]; p[b] = hi[b]; map_point(X, p[0], p[1], p[2], x11);
    p[a] = lo[a]; p[b] = hi[b]; map_point(X, p[0], p[1], p[2], x01);
    p[a] = hi[a]; p[b] = lo[b]; map_point(X, p[0], p[1], p[2], x10);
    double d1[3], d2[3];
    for (int q = 0; q < 3; ++q) {
        d1[q] = x11[q] - x00[q];
        d2[q] = x01[q] - x10[q];
    }
    const double A0 = 0.5 * (d1[1] * d2[2] - d1[2] * d2[1]);
    const double A1 = 0.5 * (d1[2] * d2[0] - d1[0] * d2[2]);
    const double A2 = 0.5 * (d1[0] * d2[1] - d1[1] * d2[0]);
    out[t] = u0 * A0 + u1 * A1 + u2 * A2;
}

}  // namespace

int launch_constant_flux(hd_ctx* c, const double* u, double* out) {
    if (!c->d_vert) return set_err(c, HD_ERR_STATE, "mesh vertices not available");
    Geo g = geo_of(c);
    const int bs = 256;
    hipLaunchKernelGGL(constant_flux_kernel, dim3((unsigned)((c->n_u + bs - 1) / bs)), dim3(bs), 0, c->stream, g,
                       c->p, c->d_vert, c->d_tab64, u[0], u[1], u[2], c->n_u, out);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

Geo geo_of(const hd_ctx* c) {
    Geo g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.off[0] = 0;
    g.off[1] = c->nface[0];
    g.off[2] = c->nface[0] + c->nface[1];
    return g;
}

int launch_geometry(hd_ctx* c, const double* d_vert, int* d_bad) {
    const int Q = c->p + 1;
    const int64_t nt = c->ne * (Q * Q * Q + 8);
    const int bs = 256;
    hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)((nt + bs - 1) / bs)), dim3(bs), 0, c->stream, c->nx, c->ny,
                       c->nz, c->p, d_vert, c->unstructured ? c->d_evx : nullptr, c->d_tab64, c->d_pa, c->d_pa32,
                       d_bad);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int launch_diagonals(hd_ctx* c, const double* theta) {
    Geo g = geo_of(c);
    const int bs = 256;
    // zero diag(M) (shared faces are accumulated)
    hipLaunchKernelGGL(fill_kernel<double>, dim3((unsigned)((c->n_u + bs - 1) / bs)), dim3(bs), 0, c->stream,
                       c->d_mdiag, 0.0, c->n_u);
    switch (c->p) {
        case 1: launch_diag_p<1>(c, g, theta); break;
        case 2: launch_diag_p<2>(c, g, theta); break;
        case 3: launch_diag_p<3>(c, g, theta); break;
        case 4: launch_diag_p<4>(c, g, theta); break;
        case 5: launch_diag_p<5>(c, g, theta); break;
        case 6: launch_diag_p<6>(c, g, theta); break;
        default: return set_err(c, HD_ERR_ARG, "p out of range");
    }
    if (c->unstructured)
        hipLaunchKernelGGL(mdiag_finish_uns_kernel, dim3((unsigned)((c->n_u + bs - 1) / bs)), dim3(bs), 0, c->stream,
                           c->d_essm, c->tau, c->d_mdiag, c->d_mdinv, c->d_mdinv32, c->d_wface, c->n_u);
    else
        hipLaunchKernelGGL(mdiag_finish_kernel, dim3((unsigned)((c->n_u + bs - 1) / bs)), dim3(bs), 0, c->stream, g,
                           c->p, c->ess, c->tau, c->d_mdiag, c->d_mdinv, c->d_mdinv32, c->d_wface, c->n_u);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int scan_counts(hd_ctx* c, const int32_t* cnt, int64_t n, int32_t* rp, int64_t* total_host) {
    const int64_t nb = (n + SCAN_CH - 1) / SCAN_CH;
    int64_t* bsum = dalloc<int64_t>(nb + 1);
    if (!bsum) return set_err(c, HD_ERR_OOM, "scan buffer");
    int64_t* tot = bsum + nb;
    hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(SCAN_T), 0, c->stream, cnt, n, bsum);
    hipLaunchKernelGGL(scan_bsums_kernel, dim3(1), dim3(1024), 0, c->stream, bsum, nb, tot);
    hipLaunchKernelGGL(scan_final_kernel, dim3((unsigned)nb), dim3(SCAN_T), 0, c->stream, cnt, n, bsum, tot, rp);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(total_host, tot, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    dfree(bsum);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return set_err(c, HD_ERR_HIP, "scan failed");
    return HD_OK;
}

// Darcy with a gamma field: C~_ii = diag(W_gamma)_ii / W_ii^2 (the product of
// the diagonals of W^{-1} W_gamma W^{-1}, Section 2.4), one thread per L2 dof;
// gamma at the quadrature points is the trilinear interpolant of the element's
// vertex values, w / det J the stored seventh factor.
template <int P>
__global__ void gamma_ctil_kernel(Geo g, int64_t nq, const double* __restrict__ pa,
                                  const Tables<double>* __restrict__ tab, const double* __restrict__ gv,
                                  const double* __restrict__ wdiag, double* __restrict__ ctil) {
    constexpr int Q = P + 1, Q3 = Q * Q * Q, NL = P * P * P;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int64_t e = i / NL;
    const int l = (int)(i % NL);
    const int i0 = l % P, i1 = (l / P) % P, i2 = l / (P * P);
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    double gvx[8];
    for (int v = 0; v < 8; ++v) {
        const int dx = v & 1, dy = (v >> 1) & 1, dz = v >> 2;
        gvx[v] = gv[(ex + dx) + (int64_t)(g.nx + 1) * ((ey + dy) + (int64_t)(g.ny + 1) * (ez + dz))];
    }
    const double* gw = pa + (size_t)e * NPA * Q3 + 6 * Q3;
    double s = 0.0;
    for (int q = 0; q < Q3; ++q) {
        const int a = q % Q, b = (q / Q) % Q, c = q / (Q * Q);
        const double x = tab->xq[a], y = tab->xq[b], z = tab->xq[c];
        double gam = 0.0;
        for (int v = 0; v < 8; ++v)
            gam += gvx[v] * ((v & 1) ? x : 1.0 - x) * (((v >> 1) & 1) ? y : 1.0 - y) * ((v >> 2) ? z : 1.0 - z);
        const double h = tab->H[a][i0] * tab->H[b][i1] * tab->H[c][i2];
        s += gam * gw[q] * h * h;
    }
    ctil[i] = s / (wdiag[i] * wdiag[i]);
}

int launch_schur(hd_ctx* c) {
    Geo g = geo_of(c);
    const int bs = 256;
    const int64_t n = c->n_q;
    const double* ctil = nullptr;
    if (c->gamma_field) {
        const unsigned nbk = (unsigned)((n + bs - 1) / bs);
#define GCT(PP)                                                                                                    \
    hipLaunchKernelGGL(gamma_ctil_kernel<PP>, dim3(nbk), dim3(bs), 0, c->stream, g, n, c->d_pa, c->d_tab64, c->d_gv, \
                       c->d_wdiag, c->d_ctil)
        switch (c->p) {
            case 1: GCT(1); break;
            case 2: GCT(2); break;
            case 3: GCT(3); break;
            case 4: GCT(4); break;
            case 5: GCT(5); break;
            default: GCT(6); break;
        }
#undef GCT
        HD_HIP(c, hipGetLastError());
        ctil = c->d_ctil;
    }
    int32_t* cnt = dalloc<int32_t>(n);
    int32_t* rp = dalloc<int32_t>(n + 1);
    if (!cnt || !rp) {
        dfree(cnt);
        dfree(rp);
        return set_err(c, HD_ERR_OOM, "schur row counts");
    }
    const int NL = c->p * c->p * c->p;
    if (c->unstructured)
        hipLaunchKernelGGL(schur_uns_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, c->stream, n, NL,
                           c->d_rdof, c->d_rnbr, c->d_essm, c->d_mdiag, c->d_wdiag, c->d_kap, ctil, cnt,
                           (const int32_t*)nullptr, (int32_t*)nullptr, (double*)nullptr, (float*)nullptr,
                           (double*)nullptr, (float*)nullptr);
    else
        hipLaunchKernelGGL(schur_count_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, c->stream, g, c->p,
                           c->ess, n, c->d_mdiag, c->d_wdiag, c->d_kap, ctil, cnt);
    int64_t nnz = 0;
    int rc = scan_counts(c, cnt, n, rp, &nnz);
    dfree(cnt);
    if (rc) return rc;
    if (nnz > INT32_MAX) return set_err(c, HD_ERR_ARG, "S~ has more than 2^31 nonzeros");
    DevCSR& S = c->S;
    dfree(S.rp);
    dfree(S.ci);
    dfree(S.v);
    dfree(S.v32);
    S.nrows = S.ncols = n;
    S.nnz = nnz;
    S.rp = rp;
    S.ci = dalloc<int32_t>(nnz);
    S.v = dalloc<double>(nnz);
    S.v32 = dalloc<float>(nnz);
    if (!S.ci || !S.v || !S.v32) return set_err(c, HD_ERR_OOM, "S~ storage");
    if (c->unstructured)
        hipLaunchKernelGGL(schur_uns_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, c->stream, n, NL,
                           c->d_rdof, c->d_rnbr, c->d_essm, c->d_mdiag, c->d_wdiag, c->d_kap, ctil, (int32_t*)nullptr,
                           (const int32_t*)S.rp, S.ci, S.v, S.v32, c->d_sdiag, c->d_sdiag32);
    else
        hipLaunchKernelGGL(schur_fill_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, c->stream, g, c->p,
                           c->ess, n, c->d_mdiag, c->d_wdiag, c->d_kap, ctil, S.rp, S.ci, S.v, S.v32, c->d_sdiag,
                           c->d_sdiag32);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int launch_ensure_partial(hd_ctx* c, int64_t n) {
    if (n <= c->partial_cap) return HD_OK;
    dfree(c->d_partial);
    c->d_partial = dalloc<double>(n);
    if (!c->d_partial) {
        c->partial_cap = 0;
        return set_err(c, HD_ERR_OOM, "partial sums");
    }
    c->partial_cap = n;
    return HD_OK;
}

int reduce_sum_partials(hd_ctx* c, const double* partial, int64_t n, double* out_dev) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, c->stream, partial, n, out_dev);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

}  // namespace hd
