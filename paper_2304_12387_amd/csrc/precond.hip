// Block-diagonal preconditioner B^{-1} = diag((tau M~)^{-1}, S^{-1}) with
// S^{-1} one V(1,1)-cycle of the aggregation AMG on S~ (Section 2.3, Prop. 5;
// the remark after Prop. 3 for tau).  When S~ is singular (pure flux
// boundary conditions and C~ = 0) the constant is removed from the cycle's
// output (Section 4.2).
//
// V-cycle on level l with input b and output z:
//   x = D_l1^{-1} b,  r = b - A x          (pre-smoothing from zero, fused)
//   b_c = P^T r,  x_c = cycle(l+1, b_c)    (coarsest: dense inverse, FP64)
//   x += P x_c,   z = x + D_l1^{-1} (b - A x)
// l1-Jacobi: D_l1 = sum_j |a_ij|.  Level matrices are CSR; SpMV uses one
// thread per row.  FP32 variants read FP32 copies of the level matrices and
// keep the coarse solve in FP64.
#include "kernels_common.hpp"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace hd {

namespace {

constexpr int BS = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

// Kernels that emit per-block partial sums use at most RED_BLOCKS blocks with
// a grid-stride loop, so that the one-block final reductions stay short.
constexpr unsigned RED_BLOCKS = 1024;
inline unsigned red_grid(int64_t n) { return nblk(n) < RED_BLOCKS ? nblk(n) : RED_BLOCKS; }

// ---------------------------------------------------------------------------
// Level 0 of the hierarchy is S~ itself, the 7-point sub-volume operator of
// eq. (approx-schur-entries): S~ x = diag(S~) x - sum over the free interior
// faces k of w_k x_{neighbour(k)}, w_k = 1/M~_kk.  It is applied matrix-free
// from diag(S~) and the face weights, walking the structured neighbours.
// ---------------------------------------------------------------------------
template <int P, typename F>
__device__ __forceinline__ void for_each_coupling(const Geo& g, int64_t i, F&& f) {
    constexpr int NL = P * P * P;
    const int64_t e = i / NL;
    const int l = (int)(i % NL);
    const int a = l % P, b = (l / P) % P, c = l / (P * P);
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    const int64_t nxp = (int64_t)g.nx * P, nyp = (int64_t)g.ny * P;
    const int64_t gx = (int64_t)ex * P + a, gy = (int64_t)ey * P + b, gz = (int64_t)ez * P + c;
    const int64_t eNL = NL, rowNL = (int64_t)g.nx * NL, planeNL = (int64_t)g.nx * g.ny * NL;
    // x-normal faces
    {
        const int64_t k = g.off[0] + gx + (nxp + 1) * (gy + nyp * gz);
        if (a > 0) f(k, i - 1);
        else if (ex > 0) f(k, i - eNL + (P - 1));
        if (a < P - 1) f(k + 1, i + 1);
        else if (ex < g.nx - 1) f(k + 1, i + eNL - (P - 1));
    }
    // y-normal faces
    {
        const int64_t k = g.off[1] + gx + nxp * (gy + (nyp + 1) * gz);
        if (b > 0) f(k, i - P);
        else if (ey > 0) f(k, i - rowNL + (P - 1) * P);
        if (b < P - 1) f(k + nxp, i + P);
        else if (ey < g.ny - 1) f(k + nxp, i + rowNL - (P - 1) * P);
    }
    // z-normal faces
    {
        const int64_t k = g.off[2] + gx + nxp * (gy + nyp * gz);
        if (c > 0) f(k, i - P * P);
        else if (ez > 0) f(k, i - planeNL + (P - 1) * P * P);
        if (c < P - 1) f(k + nxp * nyp, i + P * P);
        else if (ez < g.nz - 1) f(k + nxp * nyp, i + planeNL - (P - 1) * P * P);
    }
}

// Lower and upper neighbours of sub-volume i in direction d (-1 at the
// domain boundary), in the element-major L2 numbering.
template <int P>
__device__ __forceinline__ void s0_neighbours(const Geo& g, int64_t i, int64_t (&lo)[3], int64_t (&up)[3]) {
    constexpr int NL = P * P * P;
    const int64_t e = i / NL;
    const int l = (int)(i % NL);
    const int a = l % P, b = (l / P) % P, c = l / (P * P);
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    const int64_t eNL = NL, rowNL = (int64_t)g.nx * NL, planeNL = (int64_t)g.nx * g.ny * NL;
    lo[0] = a > 0 ? i - 1 : (ex > 0 ? i - eNL + (P - 1) : -1);
    up[0] = a < P - 1 ? i + 1 : (ex < g.nx - 1 ? i + eNL - (P - 1) : -1);
    lo[1] = b > 0 ? i - P : (ey > 0 ? i - rowNL + (P - 1) * P : -1);
    up[1] = b < P - 1 ? i + P : (ey < g.ny - 1 ? i + rowNL - (P - 1) * P : -1);
    lo[2] = c > 0 ? i - P * P : (ez > 0 ? i - planeNL + (P - 1) * P * P : -1);
    up[2] = c < P - 1 ? i + P * P : (ez < g.nz - 1 ? i + planeNL - (P - 1) * P * P : -1);
}

// Face weights by sub-volume: wlo[d * n + i] = weight of the face between i
// and its lower neighbour in direction d (the same face as for_each_coupling
// visits), 0 where there is none.  The upper face of i is the lower face of
// its upper neighbour, so the level-0 kernels read both from this array in
// the L2 numbering instead of gathering from the RT face layout.
template <int P, typename T>
__global__ __launch_bounds__(BS) void s0_wlo_kernel(Geo g, int64_t n, const double* __restrict__ wf,
                                                    T* __restrict__ wlo) {
    const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (i >= n) return;
    T w[3] = {T(0), T(0), T(0)};
    for_each_coupling<P>(g, i, [&](int64_t k, int64_t j) {
        // the face's direction from its RT-layout block; lower faces couple
        // to a smaller index
        const int d = k >= g.off[2] ? 2 : (k >= g.off[1] ? 1 : 0);
        if (j < i) w[d] = (T)wf[k];
    });
    for (int dd = 0; dd < 3; ++dd) wlo[dd * n + i] = w[dd];
}

// off-diagonal part of row i of S~ applied to xval: sum over the free
// couplings of w_k xval(j), in for_each_coupling's order (x lower, x upper,
// y lower, ...)
template <int P, typename T, typename F>
__device__ __forceinline__ T s0_offdiag(const Geo& g, int64_t n, int64_t i, const T* __restrict__ wlo, F&& xval) {
    int64_t lo[3], up[3];
    s0_neighbours<P>(g, i, lo, up);
    T off = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (lo[d] >= 0) off += wlo[d * n + i] * xval(lo[d]);
        if (up[d] >= 0) off += wlo[d * n + up[d]] * xval(up[d]);
    }
    return off;
}

// x = dinv b;  r = b - S~ (dinv b)
template <int P, typename T>
__global__ __launch_bounds__(BS) void s0_pre_kernel(Geo g, int64_t n, const T* __restrict__ sdiag,
                                                    const T* __restrict__ wlo, const T* __restrict__ dinv,
                                                    const T* __restrict__ b, T* __restrict__ x, T* __restrict__ r,
                                                    const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t i = xcd_chunk(blockIdx.x, gridDim.x) * (int64_t)BS + threadIdx.x;
    if (i >= n) return;
    const T off = s0_offdiag<P, T>(g, n, i, wlo, [&](int64_t j) { return dinv[j] * b[j]; });
    const T xi = dinv[i] * b[i];
    x[i] = xi;
    r[i] = b[i] - (sdiag[i] * xi - off);
}

// z = x + dinv (b - S~ x), per-block partials of z (kind 1) or z b (kind 2)
template <int P, typename T>
__global__ __launch_bounds__(BS) void s0_post_kernel(Geo g, int64_t n, const T* __restrict__ sdiag,
                                                     const T* __restrict__ wlo, const T* __restrict__ dinv,
                                                     const T* __restrict__ b, const T* __restrict__ x,
                                                     T* __restrict__ z, double* __restrict__ part, int part_kind,
                                                     const int* __restrict__ done) {
    if (done && *done) return;
    double contrib = 0.0;
    const unsigned lb = xcd_chunk(blockIdx.x, gridDim.x);
    const int64_t i = lb * (int64_t)BS + threadIdx.x;
    if (i < n) {
        const T off = s0_offdiag<P, T>(g, n, i, wlo, [&](int64_t j) { return x[j]; });
        const T zi = x[i] + dinv[i] * (b[i] - (sdiag[i] * x[i] - off));
        z[i] = zi;
        contrib = part_kind == 1 ? (double)zi : (double)zi * (double)b[i];
    }
    if (part) {
        __shared__ double s[BS];
        s[threadIdx.x] = contrib;
        __syncthreads();
        for (int off = BS / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[lb] = s[0];
    }
}

// out[t] = sum of in[t q .. (t+1) q) (fixed order), t < nout: folds the
// post-smoother's per-block partials to the RED_BLOCKS-sized set the solver
// reduces.
__global__ void fold_partials_kernel(int64_t nin, int64_t q, int64_t nout, const double* __restrict__ in,
                                     double* __restrict__ out, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nout) return;
    double s = 0.0;
    const int64_t e = (t + 1) * q < nin ? (t + 1) * q : nin;
    for (int64_t k = t * q; k < e; ++k) s += in[k];
    out[t] = s;
}

// Sub-wave CSR row products: a group of G lanes (G a power of two <= 64)
// handles one row, each lane RU entries per pass, with all of a pass's index
// and value loads issued before its gathers and products; the group sum is
// formed with cross-lane shuffles.  Per lane the entries are summed in index
// order.
constexpr int RU = 4;

template <int G, typename T, typename F>
__device__ __forceinline__ T group_row(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                       const T* __restrict__ av, int64_t row, int lane, F&& xval) {
    T s = 0;
    const int32_t e = rp[row + 1];
    for (int32_t k0 = rp[row] + lane; k0 < e; k0 += G * RU) {
        int32_t cc[RU];
        T vv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int32_t k = k0 + u * G;
            cc[u] = k < e ? ci[k] : -1;
            vv[u] = k < e ? av[k] : T(0);
        }
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (cc[u] >= 0) s += vv[u] * xval(cc[u]);
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    return s;
}

// block-wide sum of one value per row (lane 0 of each group contributes),
// stored in part[slot]
__device__ __forceinline__ void block_partial(double v, double* __restrict__ part, unsigned slot) {
    __shared__ double s[BS];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[slot] = s[0];
}

// x = dinv b;  r = b - A (dinv b).  With XPRE the restriction that produced
// b has already written x = dinv b, and only x is gathered.
template <int G, typename T, bool XPRE>
__global__ __launch_bounds__(BS) void vc_pre_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const T* __restrict__ av,
                                                    const T* __restrict__ dinv, const T* __restrict__ b,
                                                    T* __restrict__ x, T* __restrict__ r, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t row = (xcd_chunk(blockIdx.x, gridDim.x) * (int64_t)BS + threadIdx.x) / G;
    const int lane = threadIdx.x % G;
    if (row >= n) return;
    T s;
    if (XPRE) s = group_row<G, T>(rp, ci, av, row, lane, [&](int32_t j) { return x[j]; });
    else s = group_row<G, T>(rp, ci, av, row, lane, [&](int32_t j) { return dinv[j] * b[j]; });
    if (lane == 0) {
        if (!XPRE) x[row] = dinv[row] * b[row];
        r[row] = b[row] - s;
    }
}

// y = M x (restriction with R = P^T) or y += M x (prolongation); with XN
// (restriction) also xn = dn y, the next level's pre-smoothed x
template <int G, typename T, bool ADD, bool XN = false>
__global__ __launch_bounds__(BS) void vc_spmv_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const T* __restrict__ mv,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     const T* __restrict__ dn, T* __restrict__ xn,
                                                     const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t row = (xcd_chunk(blockIdx.x, gridDim.x) * (int64_t)BS + threadIdx.x) / G;
    const int lane = threadIdx.x % G;
    if (row >= n) return;
    const T s = group_row<G, T>(rp, ci, mv, row, lane, [&](int32_t j) { return x[j]; });
    if (lane == 0) {
        if (ADD) y[row] += s;
        else y[row] = s;
        if (XN) xn[row] = dn[row] * s;
    }
}

// z = x + dinv (b - A x); optional per-block partial sums of z (kind 1, for
// the mean) or of z * b (kind 2, the preconditioned norm)
template <int G, typename T>
__global__ __launch_bounds__(BS) void vc_post_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const T* __restrict__ av,
                                                     const T* __restrict__ dinv, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ z,
                                                     double* __restrict__ part, int part_kind,
                                                     const int* __restrict__ done) {
    if (done && *done) return;
    const unsigned lb = xcd_chunk(blockIdx.x, gridDim.x);
    const int64_t row = (lb * (int64_t)BS + threadIdx.x) / G;
    const int lane = threadIdx.x % G;
    double contrib = 0.0;
    if (row < n) {
        const T acc = group_row<G, T>(rp, ci, av, row, lane, [&](int32_t j) { return x[j]; });
        if (lane == 0) {
            const T zi = x[row] + dinv[row] * (b[row] - acc);
            z[row] = zi;
            contrib = part_kind == 1 ? (double)zi : (double)zi * (double)b[row];
        }
    }
    if (part) block_partial(contrib, part, lb);
}

// z -= mean (mean = sum / n from a device scalar), partial sums of z * b
template <typename T>
__global__ void vc_sub_mean_kernel(int64_t n, const double* __restrict__ sum, const T* __restrict__ b,
                                   T* __restrict__ z, double* __restrict__ part, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double s[BS];
    const double mean = *sum / (double)n;
    double contrib = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const T zi = (T)((double)z[i] - mean);
        z[i] = zi;
        contrib += (double)zi * (double)b[i];
    }
    if (part) {
        s[threadIdx.x] = contrib;
        __syncthreads();
        for (int off = BS / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = s[0];
    }
}

// x = Cinv b, dense row-major FP64, one wavefront per row
template <typename T>
__global__ void vc_coarse_kernel(int64_t n, const double* __restrict__ cinv, const T* __restrict__ b,
                                 T* __restrict__ x, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t row = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (row >= n) return;
    double s = 0.0;
    for (int64_t k = lane; k < n; k += 64) s += cinv[row * n + k] * (double)b[k];
    s = wave_sum(s);
    if (lane == 0) x[row] = (T)s;
}

// z_u = mdinv * r_u (1 on essential dofs), partial sums of z_u * r_u
template <typename T>
__global__ void diag_prec_kernel(int64_t n, const T* __restrict__ mdinv, const T* __restrict__ r, T* __restrict__ z,
                                 double* __restrict__ part) {
    __shared__ double s[BS];
    double contrib = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const T zi = mdinv[i] * r[i];
        z[i] = zi;
        contrib += (double)zi * (double)r[i];
    }
    if (part) {
        s[threadIdx.x] = contrib;
        __syncthreads();
        for (int off = BS / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = s[0];
    }
}

template <typename T>
const T* pick(const double* d, const float* f) {
    if constexpr (std::is_same<T, double>::value) return d;
    else return f;
}
template <typename T>
T* pickw(double* d, float* f) {
    if constexpr (std::is_same<T, double>::value) return d;
    else return f;
}

// lanes per row for a CSR matrix: the power of two for which one pass of RU
// entries per lane covers at least three quarters of the mean row length
inline int group_of(const DevCSR& m) {
    const double avg = m.nrows ? (double)m.nnz / (double)m.nrows : 1.0;
    int g = 1;
    while (g < 64 && g * RU < 0.75 * avg) g *= 2;
    return g;
}

inline unsigned gblk(int64_t rows, int g) { return (unsigned)((rows * g + BS - 1) / BS); }

#define HD_GROUP_DISPATCH(g, KERNEL, ...)                                  \
    switch (g) {                                                           \
        case 1: KERNEL(1, __VA_ARGS__); break;                             \
        case 2: KERNEL(2, __VA_ARGS__); break;                             \
        case 4: KERNEL(4, __VA_ARGS__); break;                             \
        case 8: KERNEL(8, __VA_ARGS__); break;                             \
        case 16: KERNEL(16, __VA_ARGS__); break;                           \
        case 32: KERNEL(32, __VA_ARGS__); break;                           \
        default: KERNEL(64, __VA_ARGS__); break;                           \
    }

template <typename T>
int cycle(hd_ctx* c, int l, const T* b, T* z, double* part, int part_kind, const int* done) {
    const int L = (int)c->lev.size();
    DevLevel& lv = c->lev[l];
    const int64_t n = lv.A.nrows;
    if (l == L - 1) {
        hipLaunchKernelGGL(vc_coarse_kernel<T>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, c->stream, n, c->d_cinv,
                           b, z, done);
        return HD_OK;
    }
    const T* av = pick<T>(lv.A.v, lv.A.v32);
    const T* dinv = pick<T>(lv.dinv, lv.dinv32);
    T* x = pickw<T>(lv.x, lv.x32);
    T* r = pickw<T>(lv.r, lv.r32);
    DevLevel& nx = c->lev[l + 1];
    T* bc = pickw<T>(nx.b, nx.b32);
    T* zc = pickw<T>(nx.z, nx.z32);
    const int gA = group_of(lv.A), gR = group_of(lv.R), gP = group_of(lv.P);
#define PRE(G, ...) hipLaunchKernelGGL((vc_pre_kernel<G, T, false>), dim3(gblk(n, G)), dim3(BS), 0, c->stream, __VA_ARGS__)
#define PREX(G, ...) hipLaunchKernelGGL((vc_pre_kernel<G, T, true>), dim3(gblk(n, G)), dim3(BS), 0, c->stream, __VA_ARGS__)
#define RES(G, ...) hipLaunchKernelGGL((vc_spmv_kernel<G, T, false>), dim3(gblk(lv.R.nrows, G)), dim3(BS), 0, c->stream, __VA_ARGS__)
#define RESX(G, ...) hipLaunchKernelGGL((vc_spmv_kernel<G, T, false, true>), dim3(gblk(lv.R.nrows, G)), dim3(BS), 0, c->stream, __VA_ARGS__)
#define PRO(G, ...) hipLaunchKernelGGL((vc_spmv_kernel<G, T, true>), dim3(gblk(n, G)), dim3(BS), 0, c->stream, __VA_ARGS__)
#define POST(G, ...) hipLaunchKernelGGL((vc_post_kernel<G, T>), dim3(gblk(n, G)), dim3(BS), 0, c->stream, __VA_ARGS__)
    if (l == 0 && !c->unstructured) {
        const T* sd = pick<T>(c->d_sdiag, c->d_sdiag32);
        const T* wl = pick<T>(c->d_wlo, c->d_wlo32);
        const Geo g = geo_of(c);
#define S0PRE(PP) hipLaunchKernelGGL((s0_pre_kernel<PP, T>), dim3(nblk(n)), dim3(BS), 0, c->stream, g, n, sd, wl, dinv, b, x, r, done)
        switch (c->p) {
            case 1: S0PRE(1); break;
            case 2: S0PRE(2); break;
            case 3: S0PRE(3); break;
            case 4: S0PRE(4); break;
            case 5: S0PRE(5); break;
            default: S0PRE(6); break;
        }
#undef S0PRE
    } else if (l > 0) {
        // x = dinv b was written with b by the restriction from level l - 1
        HD_GROUP_DISPATCH(gA, PREX, n, lv.A.rp, lv.A.ci, av, dinv, b, x, r, done)
    } else {
        HD_GROUP_DISPATCH(gA, PRE, n, lv.A.rp, lv.A.ci, av, dinv, b, x, r, done)
    }
    // restriction; above the coarsest level it also writes the next level's
    // x = dinv b (the pre-smoother's first half)
    if (l + 2 < L) {
        const T* dn = pick<T>(nx.dinv, nx.dinv32);
        T* xn = pickw<T>(nx.x, nx.x32);
        HD_GROUP_DISPATCH(gR, RESX, lv.R.nrows, lv.R.rp, lv.R.ci, pick<T>(lv.R.v, lv.R.v32), (const T*)r, bc, dn, xn,
                          done)
    } else {
        HD_GROUP_DISPATCH(gR, RES, lv.R.nrows, lv.R.rp, lv.R.ci, pick<T>(lv.R.v, lv.R.v32), (const T*)r, bc,
                          (const T*)nullptr, (T*)nullptr, done)
    }
    int rc = cycle<T>(c, l + 1, bc, zc, nullptr, 0, done);
    if (rc) return rc;
    HD_GROUP_DISPATCH(gP, PRO, n, lv.P.rp, lv.P.ci, pick<T>(lv.P.v, lv.P.v32), (const T*)zc, x, (const T*)nullptr,
                      (T*)nullptr, done)
    if (l == 0 && !c->unstructured) {
        const T* sd = pick<T>(c->d_sdiag, c->d_sdiag32);
        const T* wl = pick<T>(c->d_wlo, c->d_wlo32);
        const Geo g = geo_of(c);
        // one thread per row over the full grid; with more blocks than the
        // solver's partial count, the block partials are folded afterwards
        const bool fold = part && (int64_t)nblk(n) > (int64_t)red_grid(n);
        double* bp = fold ? c->d_s0part : part;
#define S0POST(PP) hipLaunchKernelGGL((s0_post_kernel<PP, T>), dim3(nblk(n)), dim3(BS), 0, c->stream, g, n, sd, wl, dinv, b, (const T*)x, z, bp, part_kind, done)
        switch (c->p) {
            case 1: S0POST(1); break;
            case 2: S0POST(2); break;
            case 3: S0POST(3); break;
            case 4: S0POST(4); break;
            case 5: S0POST(5); break;
            default: S0POST(6); break;
        }
#undef S0POST
        if (fold) {
            const int64_t nin = nblk(n), nout = red_grid(n), q = (nin + nout - 1) / nout;
            hipLaunchKernelGGL(fold_partials_kernel, dim3((unsigned)((nout + BS - 1) / BS)), dim3(BS), 0, c->stream,
                               nin, q, nout, (const double*)c->d_s0part, part, done);
        }
    } else {
        // a CSR level (level 0 of an unstructured mesh too): with more blocks
        // than the solver's partial count, the block partials are folded
        const bool fold = part && (int64_t)gblk(n, gA) > (int64_t)red_grid(n);
        double* bp = fold ? c->d_s0part : part;
        HD_GROUP_DISPATCH(gA, POST, n, lv.A.rp, lv.A.ci, av, dinv, b, (const T*)x, z, bp, part_kind, done)
        if (fold) {
            const int64_t nin = gblk(n, gA), nout = red_grid(n), q = (nin + nout - 1) / nout;
            hipLaunchKernelGGL(fold_partials_kernel, dim3((unsigned)((nout + BS - 1) / BS)), dim3(BS), 0, c->stream,
                               nin, q, nout, (const double*)c->d_s0part, part, done);
        }
    }
#undef PRE
#undef PREX
#undef RES
#undef RESX
#undef PRO
#undef POST
    return HD_OK;
}

template <typename T>
__global__ void sum_partial_kernel(int64_t n, const T* __restrict__ a, const T* __restrict__ b,
                                   double* __restrict__ part, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double s[BS];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        acc += b ? (double)a[i] * (double)b[i] : (double)a[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Number of per-block partial sums of every kernel that reduces over the L2 dofs.
int64_t post_partials(const hd_ctx* c) { return red_grid(c->n_q); }

// z = S^{-1} b on the L2 dofs; `part` (optional) receives per-block partial
// sums of z * b (after the constant has been removed in the singular case);
// their number is schur_partial_count().
template <typename T>
int schur_apply(hd_ctx* c, const T* b, T* z, double* part, const int* done) {
    const int64_t n = c->n_q;
    const bool one_level = c->lev.size() == 1;
    if (!c->singular) {
        int rc = cycle<T>(c, 0, b, z, one_level ? nullptr : part, 2, done);
        if (rc) return rc;
        if (one_level && part)
            hipLaunchKernelGGL(sum_partial_kernel<T>, dim3(red_grid(n)), dim3(BS), 0, c->stream, n, z, b, part, done);
        return HD_OK;
    }
    const int64_t np = post_partials(c);
    // sized by hd_build_precond
    if (np > c->partial_cap) return set_err(c, HD_ERR_STATE, "partial-sum buffer smaller than the V-cycle needs");
    double* zs = c->d_partial;
    int rc;
    rc = cycle<T>(c, 0, b, z, one_level ? nullptr : zs, 1, done);
    if (rc) return rc;
    if (one_level)
        hipLaunchKernelGGL(sum_partial_kernel<T>, dim3(red_grid(n)), dim3(BS), 0, c->stream, n, z, (const T*)nullptr,
                           zs, done);
    rc = reduce_sum_partials(c, zs, np, c->d_scal + 6);
    if (rc) return rc;
    hipLaunchKernelGGL(vc_sub_mean_kernel<T>, dim3(red_grid(n)), dim3(BS), 0, c->stream, n, c->d_scal + 6, b, z,
                       part, done);
    return HD_OK;
}

// ---- batches: levels >= 1 of every instance's V-cycle in shared launches --
// One descriptor per (instance, operation) of a level; a workgroup finds its
// descriptor from the first-block offsets and runs the same row computation,
// with the same lanes per row, as the single-instance kernels, so the results
// are those of the instances' own V-cycles bit for bit.
enum { U_PRE = 0, U_RES = 1, U_PRO = 2, U_POST = 3, U_COARSE = 4 };

template <int G, int OP, typename T>
__device__ __forceinline__ void ubody(const UDesc<T>& D, unsigned lb) {
    if constexpr (OP == U_COARSE) {
        // x = Cinv b, one wavefront per row (as vc_coarse_kernel)
        const int64_t row = lb * (int64_t)(BS / 64) + threadIdx.x / 64;
        const int lane = threadIdx.x % 64;
        if (row >= D.n) return;
        double acc = 0.0;
        for (int64_t k = lane; k < D.n; k += 64) acc += D.cinv[row * D.n + k] * (double)D.in[k];
        acc = wave_sum(acc);
        if (lane == 0) D.out[row] = (T)acc;
    } else {
        const int64_t row = (lb * (int64_t)BS + threadIdx.x) / G;
        const int lane = threadIdx.x % G;
        if (row >= D.n) return;
        const T* in = D.in;
        const T acc = group_row<G, T>(D.rp, D.ci, D.mv, row, lane, [&](int32_t j) { return in[j]; });
        if (lane != 0) return;
        if constexpr (OP == U_PRE) {
            D.out[row] = D.b[row] - acc;
        } else if constexpr (OP == U_RES) {
            D.out[row] = acc;
            if (D.out2) D.out2[row] = D.dinv[row] * acc;
        } else if constexpr (OP == U_PRO) {
            D.out[row] += acc;
        } else {
            D.out[row] = in[row] + D.dinv[row] * (D.b[row] - acc);
        }
    }
}

template <int OP, typename T>
__global__ __launch_bounds__(BS) void uvc_kernel(const UDesc<T>* __restrict__ d, int nd, const int* __restrict__ stop,
                                                 int stop_stride) {
    __shared__ int di;
    if (threadIdx.x == 0) {
        int k = 0;
        while (k + 1 < nd && d[k + 1].blk0 <= blockIdx.x) ++k;
        di = k;
    }
    __syncthreads();
    const UDesc<T> D = d[di];
    if (stop && stop[(int64_t)D.inst * stop_stride]) return;
    const unsigned lb = blockIdx.x - D.blk0;
    switch (D.g) {
        case 1: ubody<1, OP, T>(D, lb); break;
        case 2: ubody<2, OP, T>(D, lb); break;
        case 4: ubody<4, OP, T>(D, lb); break;
        case 8: ubody<8, OP, T>(D, lb); break;
        case 16: ubody<16, OP, T>(D, lb); break;
        case 32: ubody<32, OP, T>(D, lb); break;
        default: ubody<64, OP, T>(D, lb); break;
    }
}

// level 0 of one instance's cycle (matrix-free on structured meshes):
// x = dinv b, r = b - S~ x
template <typename T>
void s0_pre_launch(hd_ctx* c, const T* b, const int* done) {
    DevLevel& lv = c->lev[0];
    const int64_t n = lv.A.nrows;
    const T* sd = pick<T>(c->d_sdiag, c->d_sdiag32);
    const T* wl = pick<T>(c->d_wlo, c->d_wlo32);
    const T* dinv = pick<T>(lv.dinv, lv.dinv32);
    T* x = pickw<T>(lv.x, lv.x32);
    T* r = pickw<T>(lv.r, lv.r32);
    const Geo g = geo_of(c);
#define S0PRE_U(PP) hipLaunchKernelGGL((s0_pre_kernel<PP, T>), dim3(nblk(n)), dim3(BS), 0, c->stream, g, n, sd, wl, dinv, b, x, r, done)
    switch (c->p) {
        case 1: S0PRE_U(1); break;
        case 2: S0PRE_U(2); break;
        case 3: S0PRE_U(3); break;
        case 4: S0PRE_U(4); break;
        case 5: S0PRE_U(5); break;
        default: S0PRE_U(6); break;
    }
#undef S0PRE_U
}

// z = x + dinv (b - S~ x) at level 0 with the partial sums of z * b (the
// solver's count, folded as in the single-instance cycle)
template <typename T>
void s0_post_launch(hd_ctx* c, const T* b, T* z, double* part, const int* done) {
    DevLevel& lv = c->lev[0];
    const int64_t n = lv.A.nrows;
    const T* sd = pick<T>(c->d_sdiag, c->d_sdiag32);
    const T* wl = pick<T>(c->d_wlo, c->d_wlo32);
    const T* dinv = pick<T>(lv.dinv, lv.dinv32);
    const T* x = pickw<T>(lv.x, lv.x32);
    const Geo g = geo_of(c);
    const bool fold = part && (int64_t)nblk(n) > (int64_t)red_grid(n);
    double* bp = fold ? c->d_s0part : part;
#define S0POST_U(PP) hipLaunchKernelGGL((s0_post_kernel<PP, T>), dim3(nblk(n)), dim3(BS), 0, c->stream, g, n, sd, wl, dinv, b, x, z, bp, 2, done)
    switch (c->p) {
        case 1: S0POST_U(1); break;
        case 2: S0POST_U(2); break;
        case 3: S0POST_U(3); break;
        case 4: S0POST_U(4); break;
        case 5: S0POST_U(5); break;
        default: S0POST_U(6); break;
    }
#undef S0POST_U
    if (fold) {
        const int64_t nin = nblk(n), nout = red_grid(n), q = (nin + nout - 1) / nout;
        hipLaunchKernelGGL(fold_partials_kernel, dim3((unsigned)((nout + BS - 1) / BS)), dim3(BS), 0, c->stream, nin,
                           q, nout, (const double*)c->d_s0part, part, done);
    }
}

template <typename T>
void launch_union(hd_ctx* c, const UnionLaunch<T>& u, const int* stop, int stop_stride) {
    if (u.nd == 0 || u.nblocks == 0) return;
    switch (u.op) {
        case U_PRE: hipLaunchKernelGGL((uvc_kernel<U_PRE, T>), dim3(u.nblocks), dim3(BS), 0, c->stream, u.d, u.nd, stop, stop_stride); break;
        case U_RES: hipLaunchKernelGGL((uvc_kernel<U_RES, T>), dim3(u.nblocks), dim3(BS), 0, c->stream, u.d, u.nd, stop, stop_stride); break;
        case U_PRO: hipLaunchKernelGGL((uvc_kernel<U_PRO, T>), dim3(u.nblocks), dim3(BS), 0, c->stream, u.d, u.nd, stop, stop_stride); break;
        case U_POST: hipLaunchKernelGGL((uvc_kernel<U_POST, T>), dim3(u.nblocks), dim3(BS), 0, c->stream, u.d, u.nd, stop, stop_stride); break;
        default: hipLaunchKernelGGL((uvc_kernel<U_COARSE, T>), dim3(u.nblocks), dim3(BS), 0, c->stream, u.d, u.nd, stop, stop_stride); break;
    }
}

}  // namespace

int launch_diag_prec(hd_ctx* c, int prec, const void* r, void* z, double* part) {
    const int64_t n = c->n_u;
    if (prec == HD_F64)
        hipLaunchKernelGGL(diag_prec_kernel<double>, dim3(red_grid(n)), dim3(BS), 0, c->stream, n, c->d_mdinv,
                           (const double*)r, (double*)z, part);
    else
        hipLaunchKernelGGL(diag_prec_kernel<float>, dim3(red_grid(n)), dim3(BS), 0, c->stream, n, c->d_mdinv32,
                           (const float*)r, (float*)z, part);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int launch_schur_prec(hd_ctx* c, int prec, const void* b, void* z, double* part, const int* done) {
    int rc = prec == HD_F64 ? schur_apply<double>(c, (const double*)b, (double*)z, part, done)
                            : schur_apply<float>(c, (const float*)b, (float*)z, part, done);
    if (rc) return rc;
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int64_t schur_partial_count(const hd_ctx* c) { return red_grid(c->n_q); }

namespace {

// The shared launches of one precision for the instances' levels >= 1
// (their order is the cycle's: restrictions and pre-smoothing down, the
// coarse solves, prolongations and post-smoothing up).
template <typename T>
int build_union_t(hd_ctx* c, std::vector<UnionLaunch<T>>& out) {
    BatchState& B = *c->batch;
    const int ni = (int)B.inst.size();
    int lmax = 0;
    for (int i = 0; i < ni; ++i)
        if (B.in_union[i]) lmax = std::max(lmax, (int)B.inst[i]->lev.size());
    auto make = [&](int op, auto&& pickdesc) -> int {
        std::vector<UDesc<T>> ds;
        unsigned blk = 0;
        for (int i = 0; i < ni; ++i) {
            UDesc<T> d = {};
            if (!B.in_union[i] || !pickdesc(i, d)) continue;
            d.inst = i;
            d.blk0 = blk;
            const int64_t nb = op == U_COARSE ? (d.n + 3) / 4 : (int64_t)gblk(d.n, d.g);
            if (nb <= 0) continue;
            blk += (unsigned)nb;
            ds.push_back(d);
        }
        UnionLaunch<T> u;
        u.op = op;
        u.nd = (int)ds.size();
        u.nblocks = blk;
        if (u.nd) {
            u.d = dalloc<UDesc<T>>(ds.size());
            if (!u.d) return set_err(c, HD_ERR_OOM, "batched V-cycle tables");
            HD_HIP(c, hipMemcpy(u.d, ds.data(), ds.size() * sizeof(UDesc<T>), hipMemcpyHostToDevice));
        }
        out.push_back(u);
        return HD_OK;
    };
    int rc;
    for (int l = 0; l + 1 < lmax; ++l) {
        if (l >= 1 && (rc = make(U_PRE, [&](int i, UDesc<T>& d) {
                hd_ctx* s = B.inst[i];
                if ((int)s->lev.size() <= l + 1) return false;
                DevLevel& lv = s->lev[l];
                d.rp = lv.A.rp; d.ci = lv.A.ci; d.mv = pick<T>(lv.A.v, lv.A.v32);
                d.in = pickw<T>(lv.x, lv.x32); d.b = pickw<T>(lv.b, lv.b32); d.out = pickw<T>(lv.r, lv.r32);
                d.n = lv.A.nrows; d.g = group_of(lv.A);
                return true;
            })))
            return rc;
        if ((rc = make(U_RES, [&](int i, UDesc<T>& d) {
                hd_ctx* s = B.inst[i];
                const int L = (int)s->lev.size();
                if (L <= l + 1) return false;
                DevLevel& lv = s->lev[l];
                DevLevel& nx = s->lev[l + 1];
                d.rp = lv.R.rp; d.ci = lv.R.ci; d.mv = pick<T>(lv.R.v, lv.R.v32);
                d.in = pickw<T>(lv.r, lv.r32); d.out = pickw<T>(nx.b, nx.b32);
                if (l + 2 < L) {
                    d.out2 = pickw<T>(nx.x, nx.x32);
                    d.dinv = pick<T>(nx.dinv, nx.dinv32);
                }
                d.n = lv.R.nrows; d.g = group_of(lv.R);
                return true;
            })))
            return rc;
    }
    if ((rc = make(U_COARSE, [&](int i, UDesc<T>& d) {
            hd_ctx* s = B.inst[i];
            DevLevel& lv = s->lev.back();
            d.cinv = s->d_cinv;
            d.in = pickw<T>(lv.b, lv.b32); d.out = pickw<T>(lv.z, lv.z32);
            d.n = lv.A.nrows;
            return true;
        })))
        return rc;
    for (int l = lmax - 2; l >= 0; --l) {
        if ((rc = make(U_PRO, [&](int i, UDesc<T>& d) {
                hd_ctx* s = B.inst[i];
                if ((int)s->lev.size() <= l + 1) return false;
                DevLevel& lv = s->lev[l];
                DevLevel& nx = s->lev[l + 1];
                d.rp = lv.P.rp; d.ci = lv.P.ci; d.mv = pick<T>(lv.P.v, lv.P.v32);
                d.in = pickw<T>(nx.z, nx.z32); d.out = pickw<T>(lv.x, lv.x32);
                d.n = lv.P.nrows; d.g = group_of(lv.P);
                return true;
            })))
            return rc;
        if (l >= 1 && (rc = make(U_POST, [&](int i, UDesc<T>& d) {
                hd_ctx* s = B.inst[i];
                if ((int)s->lev.size() <= l + 1) return false;
                DevLevel& lv = s->lev[l];
                d.rp = lv.A.rp; d.ci = lv.A.ci; d.mv = pick<T>(lv.A.v, lv.A.v32);
                d.dinv = pick<T>(lv.dinv, lv.dinv32);
                d.in = pickw<T>(lv.x, lv.x32); d.b = pickw<T>(lv.b, lv.b32); d.out = pickw<T>(lv.z, lv.z32);
                d.n = lv.A.nrows; d.g = group_of(lv.A);
                return true;
            })))
            return rc;
    }
    return HD_OK;
}

}  // namespace

int batch_union_build(hd_ctx* c) {
    BatchState& B = *c->batch;
    batch_union_free(c);
    // instances with a structured, non-singular hierarchy of at least two
    // levels take part; the others keep their own V-cycle launches
    B.in_union.assign(B.inst.size(), 0);
    bool any = false;
    for (size_t i = 0; i < B.inst.size(); ++i) {
        hd_ctx* s = B.inst[i];
        B.in_union[i] = !s->unstructured && !s->singular && s->lev.size() >= 2;
        any = any || B.in_union[i];
    }
    if (!any) return HD_OK;
    int rc = build_union_t<double>(c, B.un64);
    if (!rc) rc = build_union_t<float>(c, B.un32);
    if (rc) {
        batch_union_free(c);
        return rc;
    }
    B.union_ok = true;
    return HD_OK;
}

void batch_union_free(hd_ctx* c) {
    BatchState& B = *c->batch;
    for (auto& u : B.un64) dfree(u.d);
    for (auto& u : B.un32) dfree(u.d);
    B.un64.clear();
    B.un32.clear();
    B.in_union.clear();
    B.union_ok = false;
}

template <typename T>
int batch_union_cycle(hd_ctx* c, const T* const* vq, T* const* zq, double* const* part, const int* stop,
                      int stop_stride) {
    BatchState& B = *c->batch;
    const int ni = (int)B.inst.size();
    const std::vector<UnionLaunch<T>>* U;
    if constexpr (std::is_same<T, double>::value) U = &B.un64;
    else U = &B.un32;
    for (int i = 0; i < ni; ++i)
        if (B.in_union[i]) s0_pre_launch<T>(B.inst[i], vq[i], stop + (int64_t)i * stop_stride);
    for (const auto& u : *U) launch_union<T>(c, u, stop, stop_stride);
    for (int i = 0; i < ni; ++i)
        if (B.in_union[i]) s0_post_launch<T>(B.inst[i], vq[i], zq[i], part[i], stop + (int64_t)i * stop_stride);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

template int batch_union_cycle<double>(hd_ctx*, const double* const*, double* const*, double* const*, const int*, int);
template int batch_union_cycle<float>(hd_ctx*, const float* const*, float* const*, double* const*, const int*, int);

int launch_precond(hd_ctx* c, int prec, const void* r, void* z, double* dot_partial_u, double* dot_partial_q,
                   const int* done) {
    int rc = launch_diag_prec(c, prec, r, z, dot_partial_u);
    if (rc) return rc;
    const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
    return launch_schur_prec(c, prec, (const char*)r + es * c->n_u, (char*)z + es * c->n_u, dot_partial_q, done);
}

// ---- upload of the host hierarchy ------------------------------------------

namespace {

void free_csr(DevCSR& d) {
    dfree(d.rp);
    dfree(d.ci);
    dfree(d.v);
    dfree(d.v32);
    d = DevCSR();
}

}  // namespace

void free_levels(hd_ctx* c) {
    for (auto& lv : c->lev) {
        // level 0's A aliases S~, owned by the context
        if (&lv != &c->lev[0]) free_csr(lv.A);
        free_csr(lv.P);
        free_csr(lv.R);
        dfree(lv.dinv);
        dfree(lv.dinv32);
        dfree(lv.b);
        dfree(lv.x);
        dfree(lv.r);
        dfree(lv.z);
        dfree(lv.b32);
        dfree(lv.x32);
        dfree(lv.r32);
        dfree(lv.z32);
    }
    c->lev.clear();
    dfree(c->d_cinv);
    c->d_cinv = nullptr;
    dfree(c->d_wlo);
    dfree(c->d_wlo32);
    dfree(c->d_s0part);
    c->d_wlo = nullptr;
    c->d_wlo32 = nullptr;
    c->d_s0part = nullptr;
}

__global__ void l1_diag_kernel(int64_t n, const int32_t* __restrict__ rp, const double* __restrict__ v,
                               double* __restrict__ d, float* __restrict__ d32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s = __dadd_rn(s, fabs(v[k]));
    const double r = __ddiv_rn(1.0, s);
    d[i] = r;
    d32[i] = (float)r;
}

// Work vectors and l1 diagonals of every level of c->lev, the level-0 face
// weights by sub-volume and the post-smoother's partials; FP32 copies of the
// coarse inverse.  The level matrices and c->d_cinv are already on the device.
int finish_levels(hd_ctx* c) {
    for (auto& lv : c->lev) {
        const int64_t n = lv.A.nrows;
        lv.dinv = dalloc<double>(n);
        lv.dinv32 = dalloc<float>(n);
        lv.b = dalloc<double>(n);
        lv.x = dalloc<double>(n);
        lv.r = dalloc<double>(n);
        lv.z = dalloc<double>(n);
        lv.b32 = dalloc<float>(n);
        lv.x32 = dalloc<float>(n);
        lv.r32 = dalloc<float>(n);
        lv.z32 = dalloc<float>(n);
        if (!lv.dinv || !lv.dinv32 || !lv.b || !lv.x || !lv.r || !lv.z || !lv.b32 || !lv.x32 || !lv.r32 || !lv.z32)
            return set_err(c, HD_ERR_OOM, "AMG work vectors");
        hipLaunchKernelGGL(l1_diag_kernel, dim3(nblk(n)), dim3(BS), 0, c->stream, n, lv.A.rp, lv.A.v, lv.dinv,
                           lv.dinv32);
        HD_HIP(c, hipGetLastError());
    }
    if (c->unstructured) {
        // level 0 is a CSR level: only the post-smoother's partials
        const int64_t n = c->n_q;
        c->d_s0part = dalloc<double>(std::max<int64_t>(nblk(n), gblk(n, group_of(c->lev[0].A))));
        if (!c->d_s0part) return set_err(c, HD_ERR_OOM, "level-0 partials");
    } else {
        // level-0 face weights by sub-volume, and the post-smoother's partials
        const int64_t n = c->n_q;
        c->d_wlo = dalloc<double>(3 * n);
        c->d_wlo32 = dalloc<float>(3 * n);
        c->d_s0part = dalloc<double>(nblk(n));
        if (!c->d_wlo || !c->d_wlo32 || !c->d_s0part) return set_err(c, HD_ERR_OOM, "level-0 face weights");
        const Geo g = geo_of(c);
#define WLO(PP)                                                                                                   \
    do {                                                                                                          \
        hipLaunchKernelGGL((s0_wlo_kernel<PP, double>), dim3(nblk(n)), dim3(BS), 0, c->stream, g, n, c->d_wface, \
                           c->d_wlo);                                                                             \
        hipLaunchKernelGGL((s0_wlo_kernel<PP, float>), dim3(nblk(n)), dim3(BS), 0, c->stream, g, n, c->d_wface,  \
                           c->d_wlo32);                                                                           \
    } while (0)
        switch (c->p) {
            case 1: WLO(1); break;
            case 2: WLO(2); break;
            case 3: WLO(3); break;
            case 4: WLO(4); break;
            case 5: WLO(5); break;
            default: WLO(6); break;
        }
#undef WLO
        HD_HIP(c, hipGetLastError());
    }
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

}  // namespace hd
