// Matrix-free action of the transformed block operator (eq. transformed-
// saddle-point, Section 3):
//
//   y_u = M u + D^T q~            M by sum factorisation at the (p+1)^3
//   y_q = D u - kappa_e W_e^{-1} q~   Gauss-Legendre points (partial assembly)
//
// D is the +-1 sub-element incidence of the interpolation-histopolation basis
// (Section 2.1), applied element by element as signed neighbour differences.
// W_e^{-1} is applied by a preconditioned CG that runs entirely inside the
// element's wavefront in the Gauss-Legendre nodal basis, after the change of
// basis T^{-T} of the right-hand side and followed by T^{-1} (Section 2.5,
// Section 3.1).  The Jacobi preconditioner of that CG is the diagonal of the
// Gauss-Legendre mass matrix, formed on the fly by squared-basis sum
// factorisation.
//
// Launch: one 64-lane workgroup (one wavefront) per element.  The element's
// RT and L2 coefficients, its quadrature-point values and the 1D tables live
// in LDS.  Element-interior RT dofs are written with plain stores; dofs on a
// face shared with a neighbour element receive exactly two atomic additions
// onto a zero-initialised value, which is order-independent (a + b = b + a).
#include "kernels_common.hpp"

#include <type_traits>

namespace hd {

namespace {

constexpr int TEAM = 64;

// Load the tables of degree P compactly into LDS.
template <int P, typename T>
__device__ void load_tables(const Tables<T>* __restrict__ tab, T* sL, T* sH, T* sBg, T* sBg2, T* sTi, int tid) {
    constexpr int Q = P + 1;
    for (int i = tid; i < Q * (P + 1); i += TEAM) sL[i] = tab->L[i / (P + 1)][i % (P + 1)];
    for (int i = tid; i < Q * P; i += TEAM) {
        sH[i] = tab->H[i / P][i % P];
        sBg[i] = tab->Bg[i / P][i % P];
        sBg2[i] = tab->Bg2[i / P][i % P];
    }
    for (int i = tid; i < P * P; i += TEAM) sTi[i] = tab->Tinv[i / P][i % P];
}

// y = M u for one component on the element: interpolate to the quadrature
// points (3 stages), the caller applies G, then transpose back (3 stages).
template <int P, typename T, int C>
__device__ void interp_to_quad(const T* u, T* U, T* b1, T* b2, const T* sL, const T* sH, int tid) {
    constexpr int Q = P + 1;
    constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
    const T* B0 = C == 0 ? sL : sH;
    const T* B1 = C == 1 ? sL : sH;
    const T* B2 = C == 2 ? sL : sH;
    constexpr int L0 = C == 0 ? P + 1 : P, L1 = C == 1 ? P + 1 : P, L2 = C == 2 ? P + 1 : P;
    contract<T, N0, N1, N2, 0, Q, false, L0>(u, b1, B0, tid, TEAM);
    team_sync();
    contract<T, Q, N1, N2, 1, Q, false, L1>(b1, b2, B1, tid, TEAM);
    team_sync();
    contract<T, Q, Q, N2, 2, Q, false, L2>(b2, U, B2, tid, TEAM);
}

template <int P, typename T, int C>
__device__ void quad_to_dofs(const T* U, T* y, T* b1, T* b2, const T* sL, const T* sH, int tid) {
    constexpr int Q = P + 1;
    constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
    const T* B0 = C == 0 ? sL : sH;
    const T* B1 = C == 1 ? sL : sH;
    const T* B2 = C == 2 ? sL : sH;
    constexpr int L0 = C == 0 ? P + 1 : P, L1 = C == 1 ? P + 1 : P, L2 = C == 2 ? P + 1 : P;
    contract<T, Q, Q, Q, 2, N2, true, L2>(U, b1, B2, tid, TEAM);
    team_sync();
    contract<T, Q, Q, N2, 1, N1, true, L1>(b1, b2, B1, tid, TEAM);
    team_sync();
    contract<T, Q, N1, N2, 0, N0, true, L0>(b2, y, B0, tid, TEAM);
}

// Solve W_e x = rhs (unweighted element L2 mass, IH basis) in place in
// `sol`, given the quadrature weights gw = w/detJ at the Q^3 points (LDS).
// Returns nothing; `sol` receives the solution in the IH basis.
template <int P, typename T>
__device__ void local_cg(const T* rhs, T* sol, const T* gw, T* r, T* z, T* pv, T* dW, T* b1, T* b2, T* b3,
                         const T* sBg, const T* sBg2, const T* sTi, int tid, T tol, int maxit) {
    constexpr int Q = P + 1;
    constexpr int NL = P * P * P;
    constexpr int PER = (NL + TEAM - 1) / TEAM;
    // r = T^{-T} rhs  (Bm(o=m, k=j) = Ti[j][m])
    contract<T, P, P, P, 0, P, true, P>(rhs, b1, sTi, tid, TEAM);
    team_sync();
    contract<T, P, P, P, 1, P, true, P>(b1, b2, sTi, tid, TEAM);
    team_sync();
    contract<T, P, P, P, 2, P, true, P>(b2, r, sTi, tid, TEAM);
    // Jacobi diagonal of the Gauss-Legendre mass: (Bg^2)^T (x) (Bg^2)^T (x) (Bg^2)^T gw
    contract<T, Q, Q, Q, 0, P, true, P>(gw, b3, sBg2, tid, TEAM);
    team_sync();
    contract<T, P, Q, Q, 1, P, true, P>(b3, b1, sBg2, tid, TEAM);
    team_sync();
    contract<T, P, P, Q, 2, P, true, P>(b1, dW, sBg2, tid, TEAM);
    team_sync();
    // x = 0, z = r / d, p = z
    T rz = 0, rr0 = 0;
    for (int l = tid; l < NL; l += TEAM) {
        T zz = r[l] / dW[l];
        z[l] = zz;
        pv[l] = zz;
        sol[l] = 0;
        rz += r[l] * zz;
    }
    rz = wave_sum(rz);
    rr0 = rz;
    (void)PER;
    if (rr0 == T(0)) {
        team_sync();
    } else {
        for (int it = 0; it < maxit; ++it) {
            team_sync();
            // Ap = Bg^T diag(gw) Bg p
            contract<T, P, P, P, 0, Q, false, P>(pv, b1, sBg, tid, TEAM);
            team_sync();
            contract<T, Q, P, P, 1, Q, false, P>(b1, b2, sBg, tid, TEAM);
            team_sync();
            contract<T, Q, Q, P, 2, Q, false, P>(b2, b3, sBg, tid, TEAM);
            team_sync();
            for (int qd = tid; qd < Q * Q * Q; qd += TEAM) b3[qd] *= gw[qd];
            team_sync();
            contract<T, Q, Q, Q, 2, P, true, P>(b3, b1, sBg, tid, TEAM);
            team_sync();
            contract<T, Q, Q, P, 1, P, true, P>(b1, b2, sBg, tid, TEAM);
            team_sync();
            contract<T, Q, P, P, 0, P, true, P>(b2, b1, sBg, tid, TEAM);   // b1 = A p
            team_sync();
            T pAp = 0;
            for (int l = tid; l < NL; l += TEAM) pAp += pv[l] * b1[l];
            pAp = wave_sum(pAp);
            const T alpha = rz / pAp;
            T rz_new = 0;
            for (int l = tid; l < NL; l += TEAM) {
                sol[l] += alpha * pv[l];
                T rl = r[l] - alpha * b1[l];
                r[l] = rl;
                T zl = rl / dW[l];
                z[l] = zl;
                rz_new += rl * zl;
            }
            rz_new = wave_sum(rz_new);
            if (rz_new <= tol * tol * rr0) break;
            const T beta = rz_new / rz;
            rz = rz_new;
            for (int l = tid; l < NL; l += TEAM) pv[l] = z[l] + beta * pv[l];
        }
        team_sync();
    }
    // sol <- T^{-1} sol  (Bm(o=j, k=m) = Ti[j][m])
    contract<T, P, P, P, 0, P, false, P>(sol, b1, sTi, tid, TEAM);
    team_sync();
    contract<T, P, P, P, 1, P, false, P>(b1, b2, sTi, tid, TEAM);
    team_sync();
    contract<T, P, P, P, 2, P, false, P>(b2, sol, sTi, tid, TEAM);
    team_sync();
}

template <typename T>
struct CGParams {
    T tol;
    int maxit;
};

template <int P, typename T>
__global__ __launch_bounds__(TEAM) void block_apply_kernel(
    Geo g, const T* __restrict__ pa, const Tables<T>* __restrict__ tab, const T* __restrict__ cm,
    const T* __restrict__ kap, uint32_t ess, int ess_mode, int64_t n_u, const T* __restrict__ x,
    T* __restrict__ y, const double* __restrict__ in_scale, double* __restrict__ dot_partial,
    const int* __restrict__ done, CGParams<T> cgp, int with_c) {
    if (done && *done) return;
    using D = Dim<P>;
    constexpr int Q = D::Q, Q3 = D::Q3, NL = D::NL, NC = D::NC, NRT = D::NRT;
    __shared__ T sL[Q * (P + 1)], sH[Q * P], sBg[Q * P], sBg2[Q * P], sTi[P * P];
    __shared__ T su[NRT], sq[NL], syu[NRT], syq[NL];
    __shared__ T sU[3 * Q3], b1[Q3], b2[Q3], b3[Q3], gw[Q3];
    __shared__ T cr[NL], cz[NL], cp[NL], cd[NL], csol[NL];
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int ex = (int)(e % g.nx), ey = (int)((e / g.nx) % g.ny), ez = (int)(e / ((int64_t)g.nx * g.ny));
    load_tables<P, T>(tab, sL, sH, sBg, sBg2, sTi, tid);
    const T s_in = in_scale ? (T)(*in_scale) : T(1);
    const T cM = cm[e];
    const T kE = kap[e];
    // gather u (essential dofs read as zero), q~
    for (int l = tid; l < NRT; l += TEAM) {
        int c = l / NC, ll = l % NC, i, j, k, onf, bs;
        local_ijk<P>(c, ll, i, j, k);
        int64_t gidx = rt_global<P>(g, c, ex, ey, ez, i, j, k, onf, bs);
        bool is_ess = ess_mode == ESS_IDENTITY && bs >= 0 && (ess >> (2 * c + bs)) & 1u;
        su[l] = is_ess ? T(0) : s_in * x[gidx];
    }
    for (int l = tid; l < NL; l += TEAM) sq[l] = s_in * x[n_u + e * NL + l];
    const T* pe = pa + (size_t)e * NPA * Q3;
    for (int qd = tid; qd < Q3; qd += TEAM) gw[qd] = pe[6 * Q3 + qd];
    team_sync();

    // ---- M u: interpolate the three components to the quadrature points
    interp_to_quad<P, T, 0>(su, sU, b1, b2, sL, sH, tid);
    team_sync();
    interp_to_quad<P, T, 1>(su + NC, sU + Q3, b1, b2, sL, sH, tid);
    team_sync();
    interp_to_quad<P, T, 2>(su + 2 * NC, sU + 2 * Q3, b1, b2, sL, sH, tid);
    team_sync();
    for (int qd = tid; qd < Q3; qd += TEAM) {
        const T g00 = pe[0 * Q3 + qd], g01 = pe[1 * Q3 + qd], g02 = pe[2 * Q3 + qd];
        const T g11 = pe[3 * Q3 + qd], g12 = pe[4 * Q3 + qd], g22 = pe[5 * Q3 + qd];
        const T a = sU[qd], b = sU[Q3 + qd], c = sU[2 * Q3 + qd];
        sU[qd] = cM * (g00 * a + g01 * b + g02 * c);
        sU[Q3 + qd] = cM * (g01 * a + g11 * b + g12 * c);
        sU[2 * Q3 + qd] = cM * (g02 * a + g12 * b + g22 * c);
    }
    team_sync();
    quad_to_dofs<P, T, 0>(sU, syu, b1, b2, sL, sH, tid);
    team_sync();
    quad_to_dofs<P, T, 1>(sU + Q3, syu + NC, b1, b2, sL, sH, tid);
    team_sync();
    quad_to_dofs<P, T, 2>(sU + 2 * Q3, syu + 2 * NC, b1, b2, sL, sH, tid);
    team_sync();

    // ---- D^T q~ into y_u and D u into y_q
    for (int l = tid; l < NRT; l += TEAM) {
        int c = l / NC, ll = l % NC, i, j, k;
        local_ijk<P>(c, ll, i, j, k);
        int t = c == 0 ? i : (c == 1 ? j : k);
        int a = i, b = j, cc = k;
        T add = 0;
        // volume below the face (index t-1 along c) sees it as its upper face: +1
        if (t >= 1) {
            if (c == 0) a = i - 1; else if (c == 1) b = j - 1; else cc = k - 1;
            add += sq[a + P * (b + P * cc)];
            a = i; b = j; cc = k;
        }
        if (t <= P - 1) add -= sq[a + P * (b + P * cc)];
        syu[l] += add;
    }
    for (int l = tid; l < NL; l += TEAM) {
        int a = l % P, b = (l / P) % P, c = l / (P * P);
        // x-face (i, b, c) has local index i + (P+1)(b + P c)
        T v = su[(a + 1) + (P + 1) * (b + P * c)] - su[a + (P + 1) * (b + P * c)];
        // y-face (a, j, c): a + P (j + (P+1) c)
        v += su[NC + a + P * ((b + 1) + (P + 1) * c)] - su[NC + a + P * (b + (P + 1) * c)];
        // z-face (a, b, k): a + P (b + P k)
        v += su[2 * NC + a + P * (b + P * (c + 1))] - su[2 * NC + a + P * (b + P * c)];
        syq[l] = v;
    }
    team_sync();

    // ---- -kappa_e W_e^{-1} q~
    if (with_c && kE != T(0)) {
        local_cg<P, T>(sq, csol, gw, cr, cz, cp, cd, b1, b2, b3, sBg, sBg2, sTi, tid, cgp.tol, cgp.maxit);
        for (int l = tid; l < NL; l += TEAM) syq[l] -= kE * csol[l];
        team_sync();
    }

    // ---- scatter, and the local contribution to <y, x_scaled>
    double dot = 0.0;
    for (int l = tid; l < NRT; l += TEAM) {
        int c = l / NC, ll = l % NC, i, j, k, onf, bs;
        local_ijk<P>(c, ll, i, j, k);
        int64_t gidx = rt_global<P>(g, c, ex, ey, ez, i, j, k, onf, bs);
        bool is_ess = ess_mode == ESS_IDENTITY && bs >= 0 && (ess >> (2 * c + bs)) & 1u;
        if (is_ess) {
            T xv = s_in * x[gidx];
            y[gidx] = xv;
            dot += (double)xv * (double)xv;
        } else {
            T v = syu[l];
            if (!onf || bs >= 0) y[gidx] = v;
            else atomicAdd(&y[gidx], v);
            dot += (double)v * (double)su[l];
        }
    }
    for (int l = tid; l < NL; l += TEAM) {
        T v = syq[l];
        y[n_u + e * NL + l] = v;
        dot += (double)v * (double)sq[l];
    }
    if (dot_partial) {
        dot = wave_sum(dot);
        if (tid == 0) dot_partial[e] = dot;
    }
}

// Zero the RT dofs on faces shared by two elements (the only ones updated
// with atomics).  One thread per shared face dof.
template <typename T>
__global__ void zero_shared_faces(Geo g, int P, T* __restrict__ y, int64_t n_x, int64_t n_y, int64_t n_z) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nxp = (int64_t)g.nx * P, nyp = (int64_t)g.ny * P, nzp = (int64_t)g.nz * P;
    if (t < n_x) {
        // planes f = 1..nx-1 at gi = f P; (gj, gk) over nyp x nzp
        int64_t f = t / (nyp * nzp) + 1, r = t % (nyp * nzp);
        int64_t gj = r % nyp, gk = r / nyp;
        y[g.off[0] + f * P + (nxp + 1) * (gj + nyp * gk)] = T(0);
        return;
    }
    t -= n_x;
    if (t < n_y) {
        int64_t f = t / (nxp * nzp) + 1, r = t % (nxp * nzp);
        int64_t gi = r % nxp, gk = r / nxp;
        y[g.off[1] + gi + nxp * (f * P + (nyp + 1) * gk)] = T(0);
        return;
    }
    t -= n_y;
    if (t < n_z) {
        int64_t f = t / (nxp * nyp) + 1, r = t % (nxp * nyp);
        int64_t gi = r % nxp, gj = r / nxp;
        y[g.off[2] + gi + nxp * (gj + nyp * (f * P))] = T(0);
    }
}

// y_q = (weighted ? kappa_e : 1) W_e^{-1} x_q, one wavefront per element.
template <int P, typename T>
__global__ __launch_bounds__(TEAM) void mass_inverse_kernel(const T* __restrict__ pa, const Tables<T>* __restrict__ tab,
                                                            const T* __restrict__ kap, int weighted,
                                                            const T* __restrict__ x, T* __restrict__ y,
                                                            CGParams<T> cgp) {
    using D = Dim<P>;
    constexpr int Q = D::Q, Q3 = D::Q3, NL = D::NL;
    __shared__ T sL[Q * (P + 1)], sH[Q * P], sBg[Q * P], sBg2[Q * P], sTi[P * P];
    __shared__ T sq[NL], b1[Q3], b2[Q3], b3[Q3], gw[Q3];
    __shared__ T cr[NL], cz[NL], cp[NL], cd[NL], csol[NL];
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    load_tables<P, T>(tab, sL, sH, sBg, sBg2, sTi, tid);
    const T* pe = pa + (size_t)e * NPA * Q3;
    for (int qd = tid; qd < Q3; qd += TEAM) gw[qd] = pe[6 * Q3 + qd];
    for (int l = tid; l < NL; l += TEAM) sq[l] = x[e * NL + l];
    team_sync();
    local_cg<P, T>(sq, csol, gw, cr, cz, cp, cd, b1, b2, b3, sBg, sBg2, sTi, tid, cgp.tol, cgp.maxit);
    const T s = weighted ? kap[e] : T(1);
    for (int l = tid; l < NL; l += TEAM) y[e * NL + l] = s * csol[l];
}

template <typename T>
CGParams<T> cg_params();
template <>
CGParams<double> cg_params<double>() { return {1e-14, 64}; }
template <>
CGParams<float> cg_params<float>() { return {1e-6f, 32}; }

template <int P, typename T>
void launch_apply_p(hd_ctx* c, const T* x, T* y, const double* in_scale, double* dot_partial, int ess_mode,
                    const int* done) {
    Geo g = geo_of(c);
    const int64_t nsx = (int64_t)(c->nx - 1) * c->ny * P * c->nz * P;
    const int64_t nsy = (int64_t)(c->ny - 1) * c->nx * P * c->nz * P;
    const int64_t nsz = (int64_t)(c->nz - 1) * c->nx * P * c->ny * P;
    const int64_t ns = nsx + nsy + nsz;
    if (ns > 0) {
        const int bs = 256;
        hipLaunchKernelGGL(zero_shared_faces<T>, dim3((unsigned)((ns + bs - 1) / bs)), dim3(bs), 0, c->stream, g, P,
                           y, nsx, nsy, nsz);
    }
    const T* pa = std::is_same<T, double>::value ? (const T*)c->d_pa : (const T*)c->d_pa32;
    const Tables<T>* tab = std::is_same<T, double>::value ? (const Tables<T>*)c->d_tab64 : (const Tables<T>*)c->d_tab32;
    const T* cm = std::is_same<T, double>::value ? (const T*)c->d_cm : (const T*)c->d_cm32;
    const T* kap = std::is_same<T, double>::value ? (const T*)c->d_kap : (const T*)c->d_kap32;
    hipLaunchKernelGGL((block_apply_kernel<P, T>), dim3((unsigned)c->ne), dim3(TEAM), 0, c->stream, g, pa, tab, cm,
                       kap, c->ess, ess_mode, c->n_u, x, y, in_scale, dot_partial, done, cg_params<T>(),
                       c->kappa_zero ? 0 : 1);
}

template <int P, typename T>
void launch_minv_p(hd_ctx* c, const T* x, T* y, bool weighted) {
    const T* pa = std::is_same<T, double>::value ? (const T*)c->d_pa : (const T*)c->d_pa32;
    const Tables<T>* tab = std::is_same<T, double>::value ? (const Tables<T>*)c->d_tab64 : (const Tables<T>*)c->d_tab32;
    const T* kap = std::is_same<T, double>::value ? (const T*)c->d_kap : (const T*)c->d_kap32;
    hipLaunchKernelGGL((mass_inverse_kernel<P, T>), dim3((unsigned)c->ne), dim3(TEAM), 0, c->stream, pa, tab, kap,
                       weighted ? 1 : 0, x, y, cg_params<T>());
}

template <typename T>
void dispatch_apply(hd_ctx* c, const T* x, T* y, const double* s, double* dp, int em, const int* done) {
    switch (c->p) {
        case 1: launch_apply_p<1, T>(c, x, y, s, dp, em, done); break;
        case 2: launch_apply_p<2, T>(c, x, y, s, dp, em, done); break;
        case 3: launch_apply_p<3, T>(c, x, y, s, dp, em, done); break;
        case 4: launch_apply_p<4, T>(c, x, y, s, dp, em, done); break;
        case 5: launch_apply_p<5, T>(c, x, y, s, dp, em, done); break;
        case 6: launch_apply_p<6, T>(c, x, y, s, dp, em, done); break;
    }
}

template <typename T>
void dispatch_minv(hd_ctx* c, const T* x, T* y, bool w) {
    switch (c->p) {
        case 1: launch_minv_p<1, T>(c, x, y, w); break;
        case 2: launch_minv_p<2, T>(c, x, y, w); break;
        case 3: launch_minv_p<3, T>(c, x, y, w); break;
        case 4: launch_minv_p<4, T>(c, x, y, w); break;
        case 5: launch_minv_p<5, T>(c, x, y, w); break;
        case 6: launch_minv_p<6, T>(c, x, y, w); break;
    }
}

// t = [u_bc on essential dofs, 0 elsewhere]
__global__ void lift_prepare_kernel(Geo g, int P, uint32_t ess, int64_t n_u, int64_t N, const double* __restrict__ ubc,
                                    double* __restrict__ t) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    t[i] = (i < n_u && rt_is_essential(g, P, ess, i)) ? ubc[i] : 0.0;
}

// b_f -= y_f, b_e = u_bc
__global__ void lift_finish_kernel(Geo g, int P, uint32_t ess, int64_t n_u, int64_t N, const double* __restrict__ ubc,
                                   const double* __restrict__ y, double* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (i < n_u && rt_is_essential(g, P, ess, i)) b[i] = ubc[i];
    else b[i] -= y[i];
}

}  // namespace

int launch_lift(hd_ctx* c, const double* ubc, double* b) {
    const int64_t N = c->n_u + c->n_q;
    double* t = dalloc<double>(N);
    double* y = dalloc<double>(N);
    if (!t || !y) {
        dfree(t);
        dfree(y);
        return set_err(c, HD_ERR_OOM, "lift buffers");
    }
    Geo g = geo_of(c);
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(lift_prepare_kernel, dim3(nb), dim3(256), 0, c->stream, g, c->p, c->ess, c->n_u, N, ubc, t);
    dispatch_apply<double>(c, t, y, nullptr, nullptr, ESS_NONE, nullptr);
    hipLaunchKernelGGL(lift_finish_kernel, dim3(nb), dim3(256), 0, c->stream, g, c->p, c->ess, c->n_u, N, ubc, y, b);
    hipError_t e = hipStreamSynchronize(c->stream);
    dfree(t);
    dfree(y);
    if (e != hipSuccess) return set_err(c, HD_ERR_HIP, hipGetErrorString(e));
    return HD_OK;
}

int launch_apply(hd_ctx* c, int prec, const void* x, void* y, const double* in_scale, double* dot_partial,
                 int ess_mode, const int* done) {
    if (c->time_apply) HD_HIP(c, hipEventRecord(c->ev0, c->stream));
    if (prec == HD_F64)
        dispatch_apply<double>(c, (const double*)x, (double*)y, in_scale, dot_partial, ess_mode, done);
    else
        dispatch_apply<float>(c, (const float*)x, (float*)y, in_scale, dot_partial, ess_mode, done);
    HD_HIP(c, hipGetLastError());
    if (c->time_apply) {
        HD_HIP(c, hipEventRecord(c->ev1, c->stream));
        HD_HIP(c, hipEventSynchronize(c->ev1));
        float ms = 0.f;
        HD_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
        c->apply_ms_sum += ms;
        c->apply_count += 1;
    }
    return HD_OK;
}

int launch_mass_inverse(hd_ctx* c, int prec, const void* x, void* y, bool weighted) {
    if (prec == HD_F64)
        dispatch_minv<double>(c, (const double*)x, (double*)y, weighted);
    else
        dispatch_minv<float>(c, (const float*)x, (float*)y, weighted);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

}  // namespace hd
