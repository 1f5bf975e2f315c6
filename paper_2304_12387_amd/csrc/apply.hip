// Matrix-free action of the transformed block operator (eq. transformed-
// saddle-point, Section 3):
//
//   y_u = M u + D^T q~            M by sum factorisation at the (p+1)^3
//   y_q = D u - kappa_e W_e^{-1} q~   Gauss-Legendre points
//
// The geometric factors w J^T J / det J and w / det J at the quadrature points
// are computed in the kernel from the element's 8 vertices (the map is
// trilinear, so along a lane's quadrature column J is linear in zeta): the
// apply streams x, y and the vertices instead of 7 (p+1)^3 stored factors
// per element, and holds no factors in registers across the sum
// factorisation.
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
// Launch: one 64-lane wavefront per workgroup, holding 64 / W elements (W
// lanes per element, see Slot).  Each lane owns register pencils; LDS
// only re-orients pencils between contraction directions.  RT dofs are
// shared only by the two elements across a face, and face neighbours always
// differ in the parity of ex + ey + ez, so the operator runs as two launches
// (two colours): the first stores every dof it touches, the second stores
// its own dofs and adds its contribution to the faces it shares with the
// first.  No atomics, no zero fill, and a fixed summation order.
#include "pencil.hpp"

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

namespace hd {

namespace {

template <typename T>
struct CGParams {
    T tol;
    int maxit;
};

// Lanes per element slot W (a power of two dividing 64; a wavefront holds
// EPW = 64 / W elements).  A stage with more pencils than W takes them in
// passes of W; in particular the (p+1)^2 quadrature columns are held QC per
// lane (column t + W c on lane t).  The vectors of the local CG live in the
// p^2 x-pencils, so W >= p^2.  W is the smallest power of two >= (p+1)^2, so
// that one pass covers every stage (4 at p = 1, 16 at p = 3, 32 at p = 4, 64
// at p = 5 and 6), except at p = 2: 8-lane slots, eight elements per
// wavefront, the ninth quadrature column in a second pass.  There the
// 16-lane slot leaves 7 of its lanes idle in the column stages and most of
// them in the line stages, and the 8-lane one measured 10-18% faster in FP64
// and 10-34% in FP32 (jittered and box grids, with and without the (2,2)
// block).  At p = 4, 16-lane slots with two passes (four elements per
// wavefront) measured 7% slower: they need twice the LDS and registers per
// wavefront, which halves the wavefronts per SIMD.
template <int P>
struct Slot {
    static constexpr int Q = P + 1;
    static constexpr int W = P == 2 ? 8 : (Q * Q <= 4 ? 4 : (Q * Q <= 16 ? 16 : (Q * Q <= 32 ? 32 : 64)));
    static constexpr int EPW = 64 / W;
    static constexpr int QC = (Q * Q + W - 1) / W;
    static_assert(P * P <= W && 64 % W == 0, "slot width");
};

template <int P, typename T>
using tkp = const __attribute__((address_space(4))) TabK<P, T>*;

// A fresh view of the table pointer for each stage (see stage_tab).
template <int P, typename T>
__device__ __forceinline__ tkp<P, T> tfence(tkp<P, T> p) {
    uint64_t v = (uint64_t)p;
    asm volatile("" : "+s"(v));
    return (tkp<P, T>)v;
}

template <int P, typename T>
struct ElemLDS {
    T su[Dim<P>::NRT];   // gathered RT coefficients (scaled, essential dofs zeroed)
    T sq[Dim<P>::NL];    // gathered L2 coefficients
    T A1[Dim<P>::Q3];    // stage buffers
    T A2[Dim<P>::Q3];
    T vx[24];            // element vertices X[dz][dy][dx][coordinate]
    T gv[8];             // gamma at the element vertices (Darcy with a gamma field)
};

// ---------------------------------------------------------------------------
// Local preconditioned CG for W_e x = rhs (Section 2.5): runs in the
// Gauss-Legendre nodal basis; vectors live in x-pencil registers of the slot
// (lane t < P^2 holds the x-line (., j, k), t = j + P k).  The right-hand
// side enters as sq (IH basis) in LDS; the IH-basis solution times kappa is
// left in A1 (L2 numbering).  gw: w / det J at the quadrature points held as
// z-pencils
// (lane t < Q^2 holds (a, b, .), t = a + Q b).  Every slot iterates until its
// own residual meets the tolerance; the wavefront loops while any slot has
// not converged.
// ---------------------------------------------------------------------------
template <int P, typename T>
__device__ void local_cg(ElemLDS<P, T>& L, tkp<P, T> tk, const T (&gw)[Slot<P>::QC][P + 1], int t, bool active, T kE,
                         const CGParams<T>& cgp) {
    constexpr int Q = P + 1;
    constexpr int W = Slot<P>::W, QC = Slot<P>::QC;
#define Ti (&tfence<P, T>(tk)->Ti[0][0])
#define Bg (&tfence<P, T>(tk)->Bg[0][0])
#define Bg2 (&tfence<P, T>(tk)->Bg2[0][0])
    T r[P], z[P], pv[P], x[P], dW[P], Ap[P];
    // rhs in the GL nodal basis: T^{-T} sq, contracted z, y, then x
    stage_lds<T, P, P, P, 2, P, P, true, W>(L.sq, L.A1, Ti, t);
    __syncthreads();
    stage_lds<T, P, P, P, 1, P, P, true, W>(L.A1, L.A2, Ti, t);
    __syncthreads();
    if (t < P * P) {
        T in[P];
        pencil_load<T, P, P, P, 0>(L.A2, t, in);
        pencil_mul<T, P, P, P, true>(in, r, Ti);
    }
    __syncthreads();
    // Jacobi diagonal of the GL mass: (Bg^2)^T applied to gw in z, y, x
#pragma unroll
    for (int cc = 0; cc < QC; ++cc) {
        const int col = t + cc * W;
        if (col < Q * Q) {
            T o[P];
            pencil_mul<T, Q, P, P, true>(gw[cc], o, Bg2);
            pencil_store<T, Q, Q, Q, 2, P>(L.A1, col, o);
        }
    }
    __syncthreads();
    stage_lds<T, Q, Q, P, 1, P, P, true, W>(L.A1, L.A2, Bg2, t);
    __syncthreads();
    T rz = 0;
    if (t < P * P) {
        T in[Q];
        pencil_load<T, Q, P, P, 0>(L.A2, t, in);
        pencil_mul<T, Q, P, P, true>(in, dW, Bg2);
#pragma unroll
        for (int s = 0; s < P; ++s) {
            dW[s] = T(1) / dW[s];   // keep the reciprocal of the Jacobi diagonal
            z[s] = r[s] * dW[s];
            pv[s] = z[s];
            x[s] = 0;
            rz += r[s] * z[s];
        }
    } else {
#pragma unroll
        for (int s = 0; s < P; ++s) r[s] = z[s] = pv[s] = x[s] = dW[s] = T(0);
    }
    rz = slot_sum<T, W>(rz);
    const T rr0 = rz;
    bool done = !active || !(rr0 > T(0));
    // the loop's only table, read once (wavefront-uniform: scalar registers)
    T bgr[Q * P];
#pragma unroll
    for (int k = 0; k < Q * P; ++k) bgr[k] = Bg[k];
    for (int it = 0; it < cgp.maxit; ++it) {
        if (__all(done)) break;
        __syncthreads();
        // Ap = Bg^T diag(gw) Bg p : x (regs) -> y (LDS) -> z (regs), scale,
        // z^T (regs) -> y^T (LDS) -> x^T (regs)
        if (t < P * P) {
            T o[Q];
            pencil_mul<T, P, Q, P, false>(pv, o, bgr);
            pencil_store<T, P, P, P, 0, Q>(L.A1, t, o);
        }
        __syncthreads();
        stage_lds<T, Q, P, P, 1, Q, P, false, W>(L.A1, L.A2, bgr, t);
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < QC; ++cc) {
            const int col = t + cc * W;
            if (col < Q * Q) {
                T in[P], w[Q], o[P];
                pencil_load<T, Q, Q, P, 2>(L.A2, col, in);
                pencil_mul<T, P, Q, P, false>(in, w, bgr);
#pragma unroll
                for (int c = 0; c < Q; ++c) w[c] *= gw[cc][c];
                pencil_mul<T, Q, P, P, true>(w, o, bgr);
                pencil_store<T, Q, Q, Q, 2, P>(L.A1, col, o);
            }
        }
        __syncthreads();
        stage_lds<T, Q, Q, P, 1, P, P, true, W>(L.A1, L.A2, bgr, t);
        __syncthreads();
        T pAp = 0;
        if (t < P * P) {
            T in[Q];
            pencil_load<T, Q, P, P, 0>(L.A2, t, in);
            pencil_mul<T, Q, P, P, true>(in, Ap, bgr);
#pragma unroll
            for (int s = 0; s < P; ++s) pAp += pv[s] * Ap[s];
        }
        pAp = slot_sum<T, W>(pAp);
        T rzn = 0;
        const T alpha = rz / pAp;
        if (!done && t < P * P) {
#pragma unroll
            for (int s = 0; s < P; ++s) {
                x[s] += alpha * pv[s];
                r[s] -= alpha * Ap[s];
                z[s] = r[s] * dW[s];
                rzn += r[s] * z[s];
            }
        }
        rzn = slot_sum<T, W>(rzn);
        if (!done) {
            if (rzn <= cgp.tol * cgp.tol * rr0) {
                done = true;
            } else {
                const T beta = rzn / rz;
                rz = rzn;
#pragma unroll
                for (int s = 0; s < P; ++s) pv[s] = z[s] + beta * pv[s];
            }
        }
    }
    __syncthreads();
    // IH-basis solution T^{-1} x: x (regs) -> y (LDS) -> z, A1 = kappa * sol
    if (t < P * P) {
        T o[P];
        pencil_mul<T, P, P, P, false>(x, o, Ti);
        pencil_store<T, P, P, P, 0, P>(L.A1, t, o);
    }
    __syncthreads();
    stage_lds<T, P, P, P, 1, P, P, false, W>(L.A1, L.A2, Ti, t);
    __syncthreads();
    if (t < P * P && active) {
        T in[P], o[P];
        pencil_load<T, P, P, P, 2>(L.A2, t, in);
        pencil_mul<T, P, P, P, false>(in, o, Ti);
        using G = PencilGeom<P, P, P, 2>;
        const int b = G::base(t);
#pragma unroll
        for (int s = 0; s < P; ++s) L.A1[b + s * G::STRIDE] = kE * o[s];
    }
    __syncthreads();
#undef Ti
#undef Bg
#undef Bg2
}

// sq = W_gamma A1 for one element (Darcy with gamma varying inside the
// element, Section 2.4): the L2 coefficients in A1 to the quadrature points
// with the histopolation table in x, y (LDS) and z (registers), times
// gamma w / det J there (gamma the trilinear interpolant of the vertex values
// in gv, w / det J in gw as z-pencils), and back with the transposed table.
template <int P, typename T>
__device__ void w_gamma(ElemLDS<P, T>& L, tkp<P, T> tk, const T (&gw)[Slot<P>::QC][P + 1], int t) {
    constexpr int Q = P + 1;
    constexpr int W = Slot<P>::W, QC = Slot<P>::QC;
#define Hm (&tfence<P, T>(tk)->H[0][0])
    stage_lds<T, P, P, P, 0, Q, P, false, W>(L.A1, L.A2, Hm, t);
    __syncthreads();
    stage_lds<T, Q, P, P, 1, Q, P, false, W>(L.A2, L.A1, Hm, t);
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < QC; ++cc) {
        const int col = t + cc * W;
        if (col < Q * Q) {
            const int qa = col % Q, qb = col / Q;
            T in[P], w[Q], o[P];
            pencil_load<T, Q, Q, P, 2>(L.A1, col, in);
            pencil_mul<T, P, Q, P, false>(in, w, Hm);
            const T xa = tk->xq[qa], xb = tk->xq[qb];
            const T nx[2] = {T(1) - xa, xa}, ny[2] = {T(1) - xb, xb};
            T gz[2];
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
                gz[dz] = (L.gv[(dz * 2 + 0) * 2 + 0] * nx[0] + L.gv[(dz * 2 + 0) * 2 + 1] * nx[1]) * ny[0] +
                         (L.gv[(dz * 2 + 1) * 2 + 0] * nx[0] + L.gv[(dz * 2 + 1) * 2 + 1] * nx[1]) * ny[1];
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const T z1 = tk->xq[c];
                w[c] *= (gz[0] * (T(1) - z1) + gz[1] * z1) * gw[cc][c];
            }
            pencil_mul<T, Q, P, P, true>(w, o, Hm);
            pencil_store<T, Q, Q, Q, 2, P>(L.A2, col, o);
        }
    }
    __syncthreads();
    stage_lds<T, Q, Q, P, 1, P, P, true, W>(L.A2, L.A1, Hm, t);
    __syncthreads();
    stage_lds<T, Q, P, P, 0, P, P, true, W>(L.A1, L.sq, Hm, t);
    __syncthreads();
#undef Hm
}

// A1 = kappa W_e^{-1} sq: the explicit element inverse when given (p <= 2,
// row l per lane), otherwise the local CG.
template <int P, typename T>
__device__ __forceinline__ void local_solve(ElemLDS<P, T>& L, tkp<P, T> tk, const T (&gw)[Slot<P>::QC][P + 1], int t, bool active,
                                            T kE, const CGParams<T>& cgp, const T* __restrict__ winv, int64_t ee) {
    constexpr int NL = Dim<P>::NL, W = Slot<P>::W;
    if constexpr (P <= 2) {
        if (winv) {
            __syncthreads();
            if (active)
                for (int l = t; l < NL; l += W) {
                    const T* wr = winv + ((size_t)ee * NL + l) * NL;
                    T s = 0;
#pragma unroll
                    for (int k = 0; k < NL; ++k) s += wr[k] * L.sq[k];
                    L.A1[l] = kE * s;
                }
            __syncthreads();
            return;
        }
    }
    local_cg<P, T>(L, tk, gw, t, active, kE, cgp);
}

// Forward sum factorisation of RT component C (shape N0,N1,N2) to the
// quadrature points: x and y through LDS, z into registers (z-pencil of the
// quadrature point column (a, b, .), column t + W c in U[c] of lane t).
template <int P, typename T, int C>
__device__ __forceinline__ void rt_to_quad(ElemLDS<P, T>& L, tkp<P, T> tk, int t, T (&U)[Slot<P>::QC][P + 1]) {
    constexpr int Q = P + 1, NC = Dim<P>::NC, W = Slot<P>::W, QC = Slot<P>::QC;
    constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
#define B0 (C == 0 ? &tfence<P, T>(tk)->L[0][0] : &tfence<P, T>(tk)->H[0][0])
#define B1 (C == 1 ? &tfence<P, T>(tk)->L[0][0] : &tfence<P, T>(tk)->H[0][0])
#define B2 (C == 2 ? &tfence<P, T>(tk)->L[0][0] : &tfence<P, T>(tk)->H[0][0])
    stage_lds<T, N0, N1, N2, 0, Q, N0, false, W>(L.su + C * NC, L.A1, B0, t);
    __syncthreads();
    stage_lds<T, Q, N1, N2, 1, Q, N1, false, W>(L.A1, L.A2, B1, t);
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < QC; ++cc) {
        const int col = t + cc * W;
        if (col < Q * Q) {
            T in[N2];
            pencil_load<T, Q, Q, N2, 2>(L.A2, col, in);
            pencil_mul<T, N2, Q, N2, false>(in, U[cc], B2);
        }
    }
    __syncthreads();
#undef B0
#undef B1
#undef B2
}

// Transpose of the z and y stages of rt_to_quad for component C: from the
// z-pencil registers V to the (Q, N1, N2) array in A1, whose x-lines
// finish_rt contracts.
template <int P, typename T, int C>
__device__ __forceinline__ void quad_to_rt(ElemLDS<P, T>& L, tkp<P, T> tk, int t, const T (&V)[Slot<P>::QC][P + 1]) {
    constexpr int Q = P + 1, W = Slot<P>::W, QC = Slot<P>::QC;
    constexpr int N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
#define B1 (C == 1 ? &tfence<P, T>(tk)->L[0][0] : &tfence<P, T>(tk)->H[0][0])
#define B2 (C == 2 ? &tfence<P, T>(tk)->L[0][0] : &tfence<P, T>(tk)->H[0][0])
#pragma unroll
    for (int cc = 0; cc < QC; ++cc) {
        const int col = t + cc * W;
        if (col < Q * Q) {
            T o[N2];
            pencil_mul<T, Q, N2, N2, true>(V[cc], o, B2);
            pencil_store<T, Q, Q, Q, 2, N2>(L.A2, col, o);
        }
    }
    __syncthreads();
    stage_lds<T, Q, Q, N2, 1, N1, N1, true, W>(L.A2, L.A1, B1, t);
    __syncthreads();
#undef B1
#undef B2
}

// At each quadrature column (a, b, .) of lane t: U = c_mass (w J^T J / det J) U
// for the three components, and gw = w / det J (1 without a (2,2) block).
// The factors come from the trilinear map of the element vertices in L.vx:
// dx/dxi and dx/deta are linear in zeta and dx/dzeta is constant along the
// column.  AFF: every element of the mesh is a parallelepiped (the map is
// affine), so J is the same at every point and J^T J / det J is formed once
// per lane; the points differ only in their weights.
template <int P, typename T, bool HAS_C, bool AFF = false>
__device__ __forceinline__ void quad_factors(ElemLDS<P, T>& L, tkp<P, T> tb, int t, T cM, T (&U0)[Slot<P>::QC][P + 1],
                                             T (&U1)[Slot<P>::QC][P + 1], T (&U2)[Slot<P>::QC][P + 1],
                                             T (&gw)[Slot<P>::QC][P + 1]) {
    constexpr int Q = P + 1, W = Slot<P>::W, QC = Slot<P>::QC;
    if constexpr (AFF) {
        // columns of J: the edges from vertex 0 to vertices 1 (dx), 2 (dy), 4 (dz)
        const T* X = L.vx;
        T J0[3], J1[3], C[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            J0[r] = X[3 + r] - X[r];
            J1[r] = X[6 + r] - X[r];
            C[r] = X[12 + r] - X[r];
        }
        const T det = J0[0] * (J1[1] * C[2] - J1[2] * C[1]) - J0[1] * (J1[0] * C[2] - J1[2] * C[0]) +
                      J0[2] * (J1[0] * C[1] - J1[1] * C[0]);
        const T id = T(1) / det;
        const T h = cM * id;
        const T g00 = h * (J0[0] * J0[0] + J0[1] * J0[1] + J0[2] * J0[2]);
        const T g01 = h * (J0[0] * J1[0] + J0[1] * J1[1] + J0[2] * J1[2]);
        const T g02 = h * (J0[0] * C[0] + J0[1] * C[1] + J0[2] * C[2]);
        const T g11 = h * (J1[0] * J1[0] + J1[1] * J1[1] + J1[2] * J1[2]);
        const T g12 = h * (J1[0] * C[0] + J1[1] * C[1] + J1[2] * C[2]);
        const T g22 = h * (C[0] * C[0] + C[1] * C[1] + C[2] * C[2]);
#pragma unroll
        for (int cc = 0; cc < QC; ++cc) {
            const int col = t + cc * W;
            if (col < Q * Q) {
                const T wab = tb->wq[col % Q] * tb->wq[col / Q];
#pragma unroll
                for (int c = 0; c < Q; ++c) {
                    const T w = wab * tb->wq[c];
                    const T a0 = U0[cc][c], a1 = U1[cc][c], a2 = U2[cc][c];
                    U0[cc][c] = w * (g00 * a0 + g01 * a1 + g02 * a2);
                    U1[cc][c] = w * (g01 * a0 + g11 * a1 + g12 * a2);
                    U2[cc][c] = w * (g02 * a0 + g12 * a1 + g22 * a2);
                    gw[cc][c] = HAS_C ? w * id : T(1);
                }
            } else {
#pragma unroll
                for (int c = 0; c < Q; ++c) gw[cc][c] = T(1);
            }
        }
        return;
    }
#pragma unroll
    for (int cc = 0; cc < QC; ++cc) {
        const int col = t + cc * W;
        if (col < Q * Q) {
            const int qa = col % Q, qb = col / Q;
            const T xa = tb->xq[qa], xb = tb->xq[qb];
            const T nx[2] = {T(1) - xa, xa}, ny[2] = {T(1) - xb, xb};
            const T* X = L.vx;
            T A[2][3], B[2][3], C[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
#pragma unroll
                for (int dz = 0; dz < 2; ++dz) {
                    A[dz][r] = (X[((dz * 2 + 0) * 2 + 1) * 3 + r] - X[((dz * 2 + 0) * 2 + 0) * 3 + r]) * ny[0] +
                               (X[((dz * 2 + 1) * 2 + 1) * 3 + r] - X[((dz * 2 + 1) * 2 + 0) * 3 + r]) * ny[1];
                    B[dz][r] = (X[((dz * 2 + 1) * 2 + 0) * 3 + r] - X[((dz * 2 + 0) * 2 + 0) * 3 + r]) * nx[0] +
                               (X[((dz * 2 + 1) * 2 + 1) * 3 + r] - X[((dz * 2 + 0) * 2 + 1) * 3 + r]) * nx[1];
                }
                T cz = 0;
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx)
                        cz += (X[((2 + dy) * 2 + dx) * 3 + r] - X[(dy * 2 + dx) * 3 + r]) * nx[dx] * ny[dy];
                C[r] = cz;
                __builtin_amdgcn_sched_barrier(0);   // one coordinate's 8 vertex values live at a time
            }
            const T wab = tb->wq[qa] * tb->wq[qb];
            // one quadrature point at a time: keeps the scheduler from
            // computing every point's factors at once (register pressure)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const T z1 = tb->xq[c], z0 = T(1) - z1;
                T J0[3], J1[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    J0[r] = A[0][r] * z0 + A[1][r] * z1;
                    J1[r] = B[0][r] * z0 + B[1][r] * z1;
                }
                // det J = J0 . (J1 x C), columns of J = d x / d (xi, eta, zeta)
                const T det = J0[0] * (J1[1] * C[2] - J1[2] * C[1]) - J0[1] * (J1[0] * C[2] - J1[2] * C[0]) +
                              J0[2] * (J1[0] * C[1] - J1[1] * C[0]);
                const T s = wab * tb->wq[c] / det;
                const T g00 = s * (J0[0] * J0[0] + J0[1] * J0[1] + J0[2] * J0[2]);
                const T g01 = s * (J0[0] * J1[0] + J0[1] * J1[1] + J0[2] * J1[2]);
                const T g02 = s * (J0[0] * C[0] + J0[1] * C[1] + J0[2] * C[2]);
                const T g11 = s * (J1[0] * J1[0] + J1[1] * J1[1] + J1[2] * J1[2]);
                const T g12 = s * (J1[0] * C[0] + J1[1] * C[1] + J1[2] * C[2]);
                const T g22 = s * (C[0] * C[0] + C[1] * C[1] + C[2] * C[2]);
                const T a0 = U0[cc][c], a1 = U1[cc][c], a2 = U2[cc][c];
                U0[cc][c] = cM * (g00 * a0 + g01 * a1 + g02 * a2);
                U1[cc][c] = cM * (g01 * a0 + g11 * a1 + g12 * a2);
                U2[cc][c] = cM * (g02 * a0 + g12 * a1 + g22 * a2);
                gw[cc][c] = HAS_C ? s : T(1);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < Q; ++c) gw[cc][c] = T(1);
        }
    }
}

// Global position of the x-line (., j, k) of RT component C in element
// (ex, ey, ez): index of its first dof, whether the whole line lies on an
// element face normal to y or z (C = 1, 2), and its domain-boundary side.
// Index arithmetic of the structured element kernels: 32-bit at p <= 3 (a
// context holds fewer than 2^31 unknowns, checked when the mesh is set up),
// where the per-element index work is a visible share of the kernel (layered
// Darcy grid, p = 2: 14% less time per apply); 64-bit at p >= 4, where the
// 32-bit form measured 3-7% slower (a different register allocation).
template <int P>
using Idx = typename std::conditional<(P <= 3), uint32_t, int64_t>::type;

template <typename I>
struct RtLine {
    I base;            // global index of local i = 0
    int tan_face;      // C = 1 (j in {0,P}) or C = 2 (k in {0,P}): the line lies on an element face
    int tan_bnd;       // ... and that face is on the domain boundary: side 0 / 1, else -1
};

template <int P, int C>
__device__ __forceinline__ RtLine<Idx<P>> rt_line(const Geo& g, int ex, int ey, int ez, int j, int k) {
    using I = Idx<P>;
    const I d0 = (I)g.nx * P + (C == 0), d1 = (I)g.ny * P + (C == 1);
    const I gj = (I)ey * P + j, gk = (I)ez * P + k;
    RtLine<I> r;
    r.base = (I)g.off[C] + (I)ex * P + d0 * (gj + d1 * gk);
    r.tan_face = 0;
    r.tan_bnd = -1;
    if (C == 1) {
        r.tan_face = j == 0 || j == P;
        r.tan_bnd = gj == 0 ? 0 : (gj == (I)g.ny * P ? 1 : -1);
    } else if (C == 2) {
        r.tan_face = k == 0 || k == P;
        r.tan_bnd = gk == 0 ? 0 : (gk == (I)g.nz * P ? 1 : -1);
    }
    return r;
}

// Classify dof i of an x-line of component C: on an element face, and on
// which domain-boundary side (-1: interior).
template <int P, int C>
__device__ __forceinline__ void rt_line_dof(const Geo& g, int ex, const RtLine<Idx<P>>& r, int i, int& onf, int& bs) {
    if (C == 0) {
        onf = i == 0 || i == P;
        const int gi = ex * P + i;
        bs = gi == 0 ? 0 : (gi == g.nx * P ? 1 : -1);
    } else {
        onf = r.tan_face;
        bs = r.tan_bnd;
    }
}

// Gather the RT coefficients of component C line by line into LDS.
template <int P, typename T, int C>
__device__ __forceinline__ void gather_rt(ElemLDS<P, T>& L, const Geo& g, int ex, int ey, int ez, int t, uint32_t ess,
                                          int ess_mode, T s_in, const T* __restrict__ x) {
    constexpr int NC = Dim<P>::NC;
    constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
    constexpr int W = Slot<P>::W;
    for (int tt = t; tt < N1 * N2; tt += W) {
        const int j = tt % N1, k = tt / N1;
        const auto r = rt_line<P, C>(g, ex, ey, ez, j, k);
        T v[N0];
#pragma unroll
        for (int i = 0; i < N0; ++i) v[i] = x[r.base + i];
#pragma unroll
        for (int i = 0; i < N0; ++i) {
            int onf, bs;
            rt_line_dof<P, C>(g, ex, r, i, onf, bs);
            const bool is_ess = ess_mode == ESS_IDENTITY && bs >= 0 && ((ess >> (2 * C + bs)) & 1u);
            L.su[C * NC + N0 * tt + i] = is_ess ? T(0) : s_in * v[i];
        }
    }
}

// Values the first colour left in y on the dofs of this lane's x-line of
// component C (the second colour adds to them on shared faces).  Issued
// before the transposed sum factorisation of C, so that the loads are in
// flight while it runs; one batch of loads per line instead of a load, wait
// and store per dof.
template <int P, typename T, int C>
__device__ __forceinline__ void prefetch_line(const Geo& g, int ex, int ey, int ez, int t, const T* __restrict__ y,
                                              T (&old)[P + 1]) {
    constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
    if (t < N1 * N2) {
        const auto r = rt_line<P, C>(g, ex, ey, ez, t % N1, t / N1);
        if (C == 0) {
            // only the two end dofs of an x-line lie on element faces
            old[0] = y[r.base];
            old[P] = y[r.base + P];
        } else if (r.tan_face) {
#pragma unroll
            for (int i = 0; i < N0; ++i) old[i] = y[r.base + i];
        }
    }
}

// x-line t of component C: the last stage of the transposed sum
// factorisation (from the (Q, N1, N2) array in A1), D^T q~ added, scatter
// to y and the local contribution to <y, x_scaled>.  Essential dofs
// (identity rows) take the scaled input value.  Straight-line stores: every
// dof of the line is written once, with the first colour's value (`old`)
// added on shared faces.
template <int P, typename T, int C>
__device__ __forceinline__ double finish_rt(ElemLDS<P, T>& L, tkp<P, T> tk, const Geo& g, int ex, int ey, int ez,
                                            int t, const T (&old)[P + 1], uint32_t ess, int ess_mode, T s_in,
                                            const T* __restrict__ x, T* __restrict__ y, int colour) {
    constexpr int NC = Dim<P>::NC, Q = P + 1;
    constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
    double dot = 0.0;
    if (t >= N1 * N2) return dot;
    T yv[N0];
    {
        T in[Q];
        pencil_load<T, Q, N1, N2, 0>(L.A1, t, in);
        pencil_mul<T, Q, N0, N0, true>(in, yv, C == 0 ? &tfence<P, T>(tk)->L[0][0] : &tfence<P, T>(tk)->H[0][0]);
    }
    const int j = t % N1, k = t / N1;
    const auto r = rt_line<P, C>(g, ex, ey, ez, j, k);
    unsigned ess_mask = 0, add_mask = 0;
#pragma unroll
    for (int i = 0; i < N0; ++i) {
        int onf, bs;
        rt_line_dof<P, C>(g, ex, r, i, onf, bs);
        if (ess_mode == ESS_IDENTITY && bs >= 0 && ((ess >> (2 * C + bs)) & 1u)) ess_mask |= 1u << i;
        // faces shared with a neighbour: the first colour stores, the
        // second adds (face neighbours always have opposite colours)
        if (colour == 1 && onf && bs < 0) add_mask |= 1u << i;
    }
    T xe[N0];
    if (ess_mask) {
#pragma unroll
        for (int i = 0; i < N0; ++i) xe[i] = s_in * x[r.base + i];
    }
#pragma unroll
    for (int i = 0; i < N0; ++i) {
        const int tn = C == 0 ? i : (C == 1 ? j : k);   // index along the normal
        int a = i, b = j, c = k;
        T add = 0;
        if (tn >= 1) {
            if (C == 0) a = i - 1; else if (C == 1) b = j - 1; else c = k - 1;
            add += L.sq[a + P * (b + P * c)];
        }
        if (tn <= P - 1) add -= L.sq[i + P * (j + P * k)];
        T v = yv[i] + add;
        const T ref = L.su[C * NC + i + N0 * t];
        double d = (double)v * (double)ref;
        if ((ess_mask >> i) & 1u) {
            v = xe[i];
            d = (double)v * (double)v;
        } else if ((add_mask >> i) & 1u) {
            v = old[i] + v;
        }
        y[r.base + i] = v;
        dot += d;
    }
    return dot;
}

// Per-right-hand-side arguments of the apply: nrhs vectors stored one after
// the other (stride ldv); optional per-RHS input scale and skip flag (strided
// views into caller state) and per-RHS partial sums of <A x, x>.
struct RhsArgs {
    int nrhs;
    int64_t ldv;
    const double* scale;
    int scale_stride;
    const int* done;
    int done_stride;
    double* partial;
    int64_t part_stride;
};

// One element group (EPW elements of one colour) of y = A x: gather, D u,
// M u by sum factorisation, the local CG for -kappa W^{-1} q~, scatter.
// x and y point at one right-hand side's vector; the return value is the
// group's <A x, x> contribution summed over the wavefront (all lanes).
template <int P, typename T, bool HAS_C = true, bool VARG = false, bool AFF = false>
__device__ __forceinline__ double apply_group(ElemLDS<P, T>* sm, const Geo& g, const double* __restrict__ vert,
                                              tkp<P, T> tb,
                                              const T* __restrict__ cm, const T* __restrict__ kap, uint32_t ess,
                                              int ess_mode, int64_t n_u, const T* __restrict__ x, T* __restrict__ y,
                                              T s_in, const CGParams<T>& cgp, int with_c, int colour, unsigned grp,
                                              unsigned nb, const T* __restrict__ winv,
                                              const double* __restrict__ gvert = nullptr) {
    using D = Dim<P>;
    using S = Slot<P>;
    constexpr int Q = D::Q, Q3 = D::Q3, NL = D::NL, NC = D::NC, W = S::W;
    const int lane = threadIdx.x;
    const int slot = lane / W, t = lane % W;
    // elements of one colour ((ex + ey + ez) mod 2 == colour), half-row by half-row
    using I = Idx<P>;
    const I hx = (I)((g.nx + 1) / 2);
    const I idx = (I)grp * S::EPW + slot;
    const I row = idx / hx;
    const int m = (int)(idx % hx);
    const int ey0 = (int)(row % (I)g.ny), ez0 = (int)(row / (I)g.ny);
    const int ex0 = 2 * m + ((colour + ey0 + ez0) & 1);
    const bool valid = grp < nb && row < (I)g.ny * (I)g.nz && ex0 < g.nx;
    const int ex = valid ? ex0 : 0, ey = valid ? ey0 : 0, ez = valid ? ez0 : 0;
    const I ee = ex + (I)g.nx * (ey + (I)g.ny * ez);   // clamped for address arithmetic
    const I qoff = (I)n_u + ee * NL;                   // first L2 dof of the element
    ElemLDS<P, T>& L = sm[slot];
    const T cM = cm[ee];
    const T kE = kap[ee];
    __syncthreads();
    // gather u (essential dofs read as zero), q~ and the element's vertices
    if (valid) {
        for (int l = t; l < 24; l += W) {
            const int v = l / 3, r = l % 3;
            const int dx = v & 1, dy = (v >> 1) & 1, dz = v >> 2;
            L.vx[l] = (T)vert[3 * ((ex + dx) + (int64_t)(g.nx + 1) * ((ey + dy) + (int64_t)(g.ny + 1) * (ez + dz))) + r];
        }
        if constexpr (VARG) {
            for (int l = t; l < 8; l += W) {
                const int dx = l & 1, dy = (l >> 1) & 1, dz = l >> 2;
                L.gv[l] = (T)gvert[(ex + dx) + (int64_t)(g.nx + 1) * ((ey + dy) + (int64_t)(g.ny + 1) * (ez + dz))];
            }
        }
        gather_rt<P, T, 0>(L, g, ex, ey, ez, t, ess, ess_mode, s_in, x);
        gather_rt<P, T, 1>(L, g, ex, ey, ez, t, ess, ess_mode, s_in, x);
        gather_rt<P, T, 2>(L, g, ex, ey, ez, t, ess, ess_mode, s_in, x);
        for (int l = t; l < NL; l += W) L.sq[l] = s_in * x[qoff + l];
    }
    __syncthreads();
    // M u: the three components to the quadrature points
    constexpr int QC = S::QC;
    T U0[QC][Q], U1[QC][Q], U2[QC][Q];
    rt_to_quad<P, T, 0>(L, tb, t, U0);
    rt_to_quad<P, T, 1>(L, tb, t, U1);
    rt_to_quad<P, T, 2>(L, tb, t, U2);
    T gw[QC][Q];
    quad_factors<P, T, HAS_C, AFF>(L, tb, t, cM, U0, U1, U2, gw);
    double dot = 0.0;
    {
        // the first colour's values on this lane's lines, loaded before the
        // transposed sum factorisation so that they arrive while it runs
        const bool pre = valid && colour == 1;
        constexpr int LC0 = (P * P + W - 1) / W, LC12 = ((P + 1) * P + W - 1) / W;
        T old0[LC0][Q], old1[LC12][Q], old2[LC12][Q];
        if (pre) {
#pragma unroll
            for (int lc = 0; lc < LC0; ++lc) prefetch_line<P, T, 0>(g, ex, ey, ez, t + lc * W, y, old0[lc]);
        }
        quad_to_rt<P, T, 0>(L, tb, t, U0);
        if (valid) {
#pragma unroll
            for (int lc = 0; lc < LC0; ++lc)
                dot += finish_rt<P, T, 0>(L, tb, g, ex, ey, ez, t + lc * W, old0[lc], ess, ess_mode, s_in, x, y, colour);
        }
        if (pre) {
#pragma unroll
            for (int lc = 0; lc < LC12; ++lc) prefetch_line<P, T, 1>(g, ex, ey, ez, t + lc * W, y, old1[lc]);
        }
        quad_to_rt<P, T, 1>(L, tb, t, U1);
        if (valid) {
#pragma unroll
            for (int lc = 0; lc < LC12; ++lc)
                dot += finish_rt<P, T, 1>(L, tb, g, ex, ey, ez, t + lc * W, old1[lc], ess, ess_mode, s_in, x, y, colour);
        }
        if (pre) {
#pragma unroll
            for (int lc = 0; lc < LC12; ++lc) prefetch_line<P, T, 2>(g, ex, ey, ez, t + lc * W, y, old2[lc]);
        }
        quad_to_rt<P, T, 2>(L, tb, t, U2);
        if (valid) {
#pragma unroll
            for (int lc = 0; lc < LC12; ++lc)
                dot += finish_rt<P, T, 2>(L, tb, g, ex, ey, ez, t + lc * W, old2[lc], ess, ess_mode, s_in, x, y, colour);
        }
    }
    // finish_rt read A1, which the local solve overwrites
    __syncthreads();
    // -kappa_e W_e^{-1} q~ (compiled out of the variant for a zero (2,2) block,
    // which then needs fewer registers and runs more wavefronts per SIMD)
    if constexpr (HAS_C) {
        if (with_c) {
            const bool act = valid && kE != T(0);
            if constexpr (VARG) {
                // W^{-1} W_gamma W^{-1} q~ (kappa = 1); q~ kept in registers
                // for the inner product of the final store
                constexpr int NS = (NL + W - 1) / W;
                T sqs[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k) sqs[k] = t + k * W < NL ? L.sq[t + k * W] : T(0);
                local_solve<P, T>(L, tb, gw, t, act, T(1), cgp, winv, ee);
                w_gamma<P, T>(L, tb, gw, t);
                local_solve<P, T>(L, tb, gw, t, act, kE, cgp, winv, ee);
#pragma unroll
                for (int k = 0; k < NS; ++k)
                    if (t + k * W < NL) L.sq[t + k * W] = sqs[k];
            } else {
                local_solve<P, T>(L, tb, gw, t, act, kE, cgp, winv, ee);
            }
        }
    }
    __syncthreads();
    // y_q = D u (element-local, +1 upper face, -1 lower face) - kappa W^{-1} q~
    if (valid) {
        const bool cg = HAS_C && with_c && kE != T(0);
        for (int l = t; l < NL; l += W) {
            const int a = l % P, b = (l / P) % P, c = l / (P * P);
            T v = L.su[(a + 1) + (P + 1) * (b + P * c)] - L.su[a + (P + 1) * (b + P * c)];
            v += L.su[NC + a + P * ((b + 1) + (P + 1) * c)] - L.su[NC + a + P * (b + (P + 1) * c)];
            v += L.su[2 * NC + a + P * (b + P * (c + 1))] - L.su[2 * NC + a + P * (b + P * c)];
            if (cg) v -= L.A1[l];
            y[qoff + l] = v;
            dot += (double)v * (double)L.sq[l];
        }
    }
    return slot_sum<double, 64>(dot);
}

// At p = 3 the register budget is held to 4 wavefronts per SIMD (the LDS
// allows 4): without it the FP64 kernels take 145-148 VGPRs and run 3; with
// it they spill 32-40 bytes per lane and run 5% faster (FP32 1%).
template <int P, typename T, bool HAS_C, bool VARG = false, bool AFF = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P == 3 && !VARG ? 4 : 1))) void block_apply_kernel(
    Geo g, const double* __restrict__ vert, tkp<P, T> tb, const T* __restrict__ cm, const T* __restrict__ kap,
    uint32_t ess, int ess_mode, int64_t ne, int64_t n_u, const T* __restrict__ xall, T* __restrict__ yall, RhsArgs ra,
    CGParams<T> cgp, int with_c, int colour, int64_t part_offset, unsigned nb, const T* __restrict__ winv,
    const double* __restrict__ gvert) {
    // Block -> (element group, right-hand side).  Each XCD (block b runs on
    // XCD b mod 8) owns a contiguous chunk of element groups and walks it once
    // per right-hand side, so that neighbouring groups, which share cache
    // lines of x and y, meet in its L2 as they do with one right-hand side.
    unsigned grp;
    int r = 0;
    if (ra.nrhs > 1) {
        const unsigned gpx = (nb + 7) / 8, k = blockIdx.x / 8;
        r = (int)(k / gpx);
        grp = (blockIdx.x % 8) * gpx + k % gpx;
    } else {
        // element groups dealt to the XCDs in contiguous chunks: neighbouring
        // groups share cache lines of x and y and meet in one L2
        grp = xcd_chunk(blockIdx.x, nb);
    }
    if (ra.done && ra.done[(int64_t)r * ra.done_stride]) return;   // uniform over the block
    __shared__ ElemLDS<P, T> sm[Slot<P>::EPW];
    const T s_in = ra.scale ? (T)ra.scale[(int64_t)r * ra.scale_stride] : T(1);
    const double dot = apply_group<P, T, HAS_C, VARG, AFF>(sm, g, vert, tb, cm, kap, ess, ess_mode, n_u, xall + r * ra.ldv,
                                                yall + r * ra.ldv, s_in, cgp, with_c, colour, grp, nb, winv,
                                                      gvert);
    if (ra.partial && grp < nb && threadIdx.x == 0) ra.partial[r * ra.part_stride + part_offset + grp] = dot;
}

// ---- unstructured hexahedral meshes --------------------------------------
// Element-to-dof index arrays instead of structured index arithmetic
// (Section 3.2, Algorithm 1): the local RT dof l of element e is
// sign * u[g] with l2g[e][l] = g (sign +1) or ~g (sign -1).  There is no
// two-colouring on a general mesh, so one launch covers all elements and
// shared faces are summed with FP64 atomic adds into y_u, which
// uns_init_kernel has set to 0 (and to the scaled input on essential dofs,
// whose identity rows the element kernel skips).  At most two elements add
// to a dof, and two-term sums do not depend on the order.
struct UnsArgs {
    const int32_t* l2g;    // [ne][NRT]
    const double* evx;     // [ne][8][3] element vertex coordinates
    const uint8_t* essm;   // [n_u] essential RT dofs
};

// D^T q~ added to x-line t of component C (from the (Q, N1, N2) array in A1),
// then added to y through the index array.
template <int P, typename T, int C>
__device__ __forceinline__ void finish_uns(ElemLDS<P, T>& L, tkp<P, T> tk, const UnsArgs& ua, int64_t ee, int t,
                                           T* __restrict__ y) {
    constexpr int NC = Dim<P>::NC, NRT = Dim<P>::NRT, Q = P + 1;
    constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
    if (t >= N1 * N2) return;
    T yv[N0];
    {
        T in[Q];
        pencil_load<T, Q, N1, N2, 0>(L.A1, t, in);
        pencil_mul<T, Q, N0, N0, true>(in, yv, C == 0 ? &tfence<P, T>(tk)->L[0][0] : &tfence<P, T>(tk)->H[0][0]);
    }
    const int j = t % N1, k = t / N1;
#pragma unroll
    for (int i = 0; i < N0; ++i) {
        const int tn = C == 0 ? i : (C == 1 ? j : k);   // index along the normal
        int a = i, b = j, c = k;
        T add = 0;
        if (tn >= 1) {
            if (C == 0) a = i - 1; else if (C == 1) b = j - 1; else c = k - 1;
            add += L.sq[a + P * (b + P * c)];
        }
        if (tn <= P - 1) add -= L.sq[i + P * (j + P * k)];
        const int32_t m = ua.l2g[ee * NRT + C * NC + i + N0 * t];
        const int32_t g = m < 0 ? ~m : m;
        if (ua.essm[g]) continue;
        const T v = m < 0 ? -(yv[i] + add) : yv[i] + add;
        if (tn == 0 || tn == P) atomicAdd(&y[g], v);   // a face dof: shared with the neighbour
        else y[g] = v;                                  // interior: this element's own
    }
}

template <int P, typename T, bool HAS_C>
__global__ __launch_bounds__(64) void block_apply_uns_kernel(UnsArgs ua, int64_t ne, tkp<P, T> tb,
                                                             const T* __restrict__ cm, const T* __restrict__ kap,
                                                             int64_t n_u, const T* __restrict__ xall,
                                                             T* __restrict__ yall, RhsArgs ra, CGParams<T> cgp,
                                                             int with_c, const T* __restrict__ winv) {
    using D = Dim<P>;
    using S = Slot<P>;
    constexpr int Q = D::Q, NL = D::NL, NC = D::NC, NRT = D::NRT, W = S::W, QC = S::QC;
    const int r = blockIdx.y;
    if (ra.done && ra.done[(int64_t)r * ra.done_stride]) return;   // uniform over the block
    __shared__ ElemLDS<P, T> sm[S::EPW];
    const T* __restrict__ x = xall + r * ra.ldv;
    T* __restrict__ y = yall + r * ra.ldv;
    const T s_in = ra.scale ? (T)ra.scale[(int64_t)r * ra.scale_stride] : T(1);
    const int lane = threadIdx.x;
    const int slot = lane / W, t = lane % W;
    const int64_t e0 = (int64_t)xcd_chunk(blockIdx.x, gridDim.x) * S::EPW + slot;
    const bool valid = e0 < ne;
    const int64_t ee = valid ? e0 : 0;
    ElemLDS<P, T>& L = sm[slot];
    const T cM = cm[ee];
    const T kE = kap[ee];
    if (valid) {
        for (int l = t; l < 24; l += W) L.vx[l] = (T)ua.evx[24 * ee + l];
        const int32_t* m = ua.l2g + ee * NRT;
        for (int l = t; l < NRT; l += W) {
            const int32_t v = m[l];
            const int32_t g = v < 0 ? ~v : v;
            const T xv = s_in * x[g];
            L.su[l] = ua.essm[g] ? T(0) : (v < 0 ? -xv : xv);
        }
        for (int l = t; l < NL; l += W) L.sq[l] = s_in * x[n_u + ee * NL + l];
    }
    __syncthreads();
    T U0[QC][Q], U1[QC][Q], U2[QC][Q];
    rt_to_quad<P, T, 0>(L, tb, t, U0);
    rt_to_quad<P, T, 1>(L, tb, t, U1);
    rt_to_quad<P, T, 2>(L, tb, t, U2);
    T gw[QC][Q];
    quad_factors<P, T, HAS_C>(L, tb, t, cM, U0, U1, U2, gw);
    constexpr int LC0 = (P * P + W - 1) / W, LC12 = ((P + 1) * P + W - 1) / W;
    quad_to_rt<P, T, 0>(L, tb, t, U0);
    if (valid) {
#pragma unroll
        for (int lc = 0; lc < LC0; ++lc) finish_uns<P, T, 0>(L, tb, ua, ee, t + lc * W, y);
    }
    quad_to_rt<P, T, 1>(L, tb, t, U1);
    if (valid) {
#pragma unroll
        for (int lc = 0; lc < LC12; ++lc) finish_uns<P, T, 1>(L, tb, ua, ee, t + lc * W, y);
    }
    quad_to_rt<P, T, 2>(L, tb, t, U2);
    if (valid) {
#pragma unroll
        for (int lc = 0; lc < LC12; ++lc) finish_uns<P, T, 2>(L, tb, ua, ee, t + lc * W, y);
    }
    __syncthreads();
    if constexpr (HAS_C) {
        if (with_c) local_solve<P, T>(L, tb, gw, t, valid && kE != T(0), kE, cgp, winv, ee);
    }
    __syncthreads();
    if (valid) {
        const bool cg = HAS_C && with_c && kE != T(0);
        for (int l = t; l < NL; l += W) {
            const int a = l % P, b = (l / P) % P, c = l / (P * P);
            T v = L.su[(a + 1) + (P + 1) * (b + P * c)] - L.su[a + (P + 1) * (b + P * c)];
            v += L.su[NC + a + P * ((b + 1) + (P + 1) * c)] - L.su[NC + a + P * (b + (P + 1) * c)];
            v += L.su[2 * NC + a + P * (b + P * (c + 1))] - L.su[2 * NC + a + P * (b + P * c)];
            if (cg) v -= L.A1[l];
            y[n_u + ee * NL + l] = v;
        }
    }
}

// y_u = 0 on free dofs and the scaled input on essential ones (identity
// rows), for each right-hand side (blockIdx.y)
template <typename T>
__global__ void uns_init_kernel(int64_t n_u, const uint8_t* __restrict__ essm, const T* __restrict__ xall,
                                T* __restrict__ yall, RhsArgs ra) {
    const int r = blockIdx.y;
    if (ra.done && ra.done[(int64_t)r * ra.done_stride]) return;
    const T s_in = ra.scale ? (T)ra.scale[(int64_t)r * ra.scale_stride] : T(1);
    const T* x = xall + r * ra.ldv;
    T* y = yall + r * ra.ldv;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_u; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = essm[i] ? s_in * x[i] : T(0);
}

constexpr unsigned UNS_DOT_BLOCKS = 1024;

// per-block partial sums of <y, s_in x> over the whole vector, for each
// right-hand side (blockIdx.y); the apply's fused inner product on
// structured meshes
template <typename T>
__global__ void uns_dot_kernel(int64_t N, const T* __restrict__ xall, const T* __restrict__ yall, RhsArgs ra) {
    const int r = blockIdx.y;
    if (ra.done && ra.done[(int64_t)r * ra.done_stride]) return;
    const double s_in = ra.scale ? ra.scale[(int64_t)r * ra.scale_stride] : 1.0;
    const T* x = xall + r * ra.ldv;
    const T* y = yall + r * ra.ldv;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        acc += (double)y[i] * (s_in * (double)x[i]);
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) ra.partial[r * ra.part_stride + blockIdx.x] = sh[0];
}

// ---- several right-hand sides interleaved ([dof][nrhs]) --------------------
// y[d nrhs + r] = (A x_r)[d]: the RT_p and L2 dofs with their right-hand sides
// next to each other (the layout the element kernels read with whole cache
// lines).  One element per workgroup of 256 threads; thread t works on
// right-hand side r0 + t % NR of pencil slot t / NR (PS = 256 / NR slots), so
// the NR lanes of a slot read and write consecutive LDS words (every LDS
// tensor keeps the NR right-hand sides of a value together).  The geometric
// factors of the element are computed once, into LDS, and shared by the NR
// right-hand sides; each right-hand side runs its own local CG.
constexpr int IL_T = 256;

template <int P, typename T, int NR>
struct IlLDS {
    T su[Dim<P>::NRT * NR];   // gathered RT coefficients (scaled, essential dofs zeroed)
    T sq[Dim<P>::NL * NR];    // gathered L2 coefficients
    T A1[Dim<P>::Q3 * NR];    // stage buffers
    T A2[Dim<P>::Q3 * NR];
    T G[7][Dim<P>::Q3];       // c_mass w J^T J / det J (6) and w / det J at the quadrature points
    T dW[Dim<P>::NL];         // reciprocal Jacobi diagonal of the local CG
    T vx[24];
    double red[IL_T];         // per-slot partial sums of the CG's inner products
};

// stage over the NR right-hand sides: pencils of (N0, N1, N2) along DIM
// contracted to extent M, slot ps taking pencils ps, ps + PS, ...
template <typename T, int NR, int N0, int N1, int N2, int DIM, int M, int LDB, bool TR, typename BP>
__device__ __forceinline__ void stage_il(const T* src, T* dst, BP Bm, int ps, int r) {
    constexpr int PS = IL_T / NR;
    using G = PencilGeom<N0, N1, N2, DIM>;
    constexpr int O0 = DIM == 0 ? M : N0, O1 = DIM == 1 ? M : N1, O2 = DIM == 2 ? M : N2;
    using GO = PencilGeom<O0, O1, O2, DIM>;
#pragma unroll
    for (int pass = 0; pass < (G::NP + PS - 1) / PS; ++pass) {
        const int pp = ps + pass * PS;
        if (pp < G::NP) {
            T in[G::K], out[M];
            const int b = G::base(pp);
#pragma unroll
            for (int k = 0; k < G::K; ++k) in[k] = src[(b + k * G::STRIDE) * NR + r];
            pencil_mul<T, G::K, M, LDB, TR>(in, out, Bm);
            const int bo = GO::base(pp);
#pragma unroll
            for (int o = 0; o < M; ++o) dst[(bo + o * GO::STRIDE) * NR + r] = out[o];
        }
    }
}

// sum over the pencil slots ps < NS of v, per right-hand side (all lanes of a
// right-hand side get the same sum, in a fixed order)
template <int NR, int NS>
__device__ __forceinline__ double il_sum(double* red, double v, int ps, int r) {
    __syncthreads();
    red[ps * NR + r] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) s += red[k * NR + r];
    return s;
}

template <int P, typename T, int NR, bool HAS_C>
__global__ __launch_bounds__(IL_T) void block_apply_il_kernel(
    Geo g, const double* __restrict__ vert, tkp<P, T> tb, const T* __restrict__ cm, const T* __restrict__ kap,
    uint32_t ess, int64_t n_u, const T* __restrict__ x, T* __restrict__ y, int ldr, CGParams<T> cgp, int with_c,
    int colour, unsigned nb) {
    // ldr right-hand sides; lanes past the last one (a partial chunk) read
    // the last one and store nothing
    using D = Dim<P>;
    constexpr int Q = D::Q, Q3 = D::Q3, NL = D::NL, NC = D::NC, PS = IL_T / NR;
    static_assert(P * P <= PS && Q * Q <= PS, "pencil slots");
    __shared__ IlLDS<P, T, NR> L;
    const int t = threadIdx.x, ps = t / NR, r = t % NR;
    const bool live = (int)blockIdx.y * NR + r < ldr;
    const int rx = live ? (int)blockIdx.y * NR + r : ldr - 1;   // this lane's right-hand side
    // element of this colour: half-row by half-row, XCD-contiguous chunks
    const unsigned idx = xcd_chunk(blockIdx.x, nb);
    const int hx = (g.nx + 1) / 2;
    const int64_t row = idx / hx;
    const int m = (int)(idx % hx);
    const int ey = (int)(row % g.ny), ez = (int)(row / g.ny);
    const int ex = 2 * m + ((colour + ey + ez) & 1);
    if (ex >= g.nx) return;   // uniform over the workgroup
    const int64_t ee = ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez);
    const T cM = cm[ee];
    const T kE = kap[ee];
    // gather: vertices, u (essential dofs read as zero) line by line, q~
    if (t < 24) {
        const int v = t / 3, c = t % 3;
        const int dx = v & 1, dy = (v >> 1) & 1, dz = v >> 2;
        L.vx[t] = (T)vert[3 * ((ex + dx) + (int64_t)(g.nx + 1) * ((ey + dy) + (int64_t)(g.ny + 1) * (ez + dz))) + c];
    }
    {
        auto body = [&](auto cc) {
            constexpr int C = decltype(cc)::value;
            constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
            for (int tt = ps; tt < N1 * N2; tt += PS) {
                const int j = tt % N1, k = tt / N1;
                const auto rl = rt_line<P, C>(g, ex, ey, ez, j, k);
#pragma unroll
                for (int i = 0; i < N0; ++i) {
                    int onf, bs;
                    rt_line_dof<P, C>(g, ex, rl, i, onf, bs);
                    const bool is_ess = bs >= 0 && ((ess >> (2 * C + bs)) & 1u);
                    const T v = x[((int64_t)rl.base + i) * ldr + rx];
                    L.su[(C * NC + N0 * tt + i) * NR + r] = is_ess ? T(0) : v;
                }
            }
        };
        body(std::integral_constant<int, 0>{});
        body(std::integral_constant<int, 1>{});
        body(std::integral_constant<int, 2>{});
    }
    for (int l = ps; l < NL; l += PS) L.sq[l * NR + r] = x[(n_u + ee * NL + l) * ldr + rx];
    __syncthreads();
    // geometric factors at the quadrature points, once for all right-hand sides
    for (int pt = t; pt < Q3; pt += IL_T) {
        const int a = pt % Q, b = (pt / Q) % Q, c = pt / (Q * Q);
        const T xi[3] = {tb->xq[a], tb->xq[b], tb->xq[c]};
        T J[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int dx = v & 1, dy = (v >> 1) & 1, dz = v >> 2;
                const T Nx = dx ? xi[0] : T(1) - xi[0], Ny = dy ? xi[1] : T(1) - xi[1], Nz = dz ? xi[2] : T(1) - xi[2];
                const T gx = dx ? T(1) : T(-1), gy = dy ? T(1) : T(-1), gz = dz ? T(1) : T(-1);
                const T X = L.vx[3 * v + q];
                s0 += gx * Ny * Nz * X;
                s1 += Nx * gy * Nz * X;
                s2 += Nx * Ny * gz * X;
            }
            J[q][0] = s0;
            J[q][1] = s1;
            J[q][2] = s2;
        }
        const T det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        const T sw = tb->wq[a] * tb->wq[b] * tb->wq[c] / det;
        const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int mm = 0; mm < 6; ++mm) {
            T sj = 0;
#pragma unroll
            for (int q = 0; q < 3; ++q) sj += J[q][rr[mm]] * J[q][cc[mm]];
            L.G[mm][pt] = cM * sw * sj;
        }
        L.G[6][pt] = sw;
    }
    // M u: each component to the quadrature points (z-pencils in registers:
    // slot ps < Q^2 holds the column (a, b) = (ps % Q, ps / Q))
    T U[3][Q];
    {
        auto body = [&](auto cc) {
            constexpr int C = decltype(cc)::value;
            constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
            const auto B0 = C == 0 ? &tfence<P, T>(tb)->L[0][0] : &tfence<P, T>(tb)->H[0][0];
            stage_il<T, NR, N0, N1, N2, 0, Q, N0, false>(L.su + C * NC * NR, L.A1, B0, ps, r);
            __syncthreads();
            const auto B1 = C == 1 ? &tfence<P, T>(tb)->L[0][0] : &tfence<P, T>(tb)->H[0][0];
            stage_il<T, NR, Q, N1, N2, 1, Q, N1, false>(L.A1, L.A2, B1, ps, r);
            __syncthreads();
            if (ps < Q * Q) {
                const auto B2 = C == 2 ? &tfence<P, T>(tb)->L[0][0] : &tfence<P, T>(tb)->H[0][0];
                T in[N2];
#pragma unroll
                for (int k = 0; k < N2; ++k) in[k] = L.A2[(ps + Q * Q * k) * NR + r];
                pencil_mul<T, N2, Q, N2, false>(in, U[C], B2);
            }
            __syncthreads();
        };
        body(std::integral_constant<int, 0>{});
        body(std::integral_constant<int, 1>{});
        body(std::integral_constant<int, 2>{});
    }
    if (ps < Q * Q) {
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const int pt = ps + Q * Q * c;
            const T a0 = U[0][c], a1 = U[1][c], a2 = U[2][c];
            U[0][c] = L.G[0][pt] * a0 + L.G[1][pt] * a1 + L.G[2][pt] * a2;
            U[1][c] = L.G[1][pt] * a0 + L.G[3][pt] * a1 + L.G[4][pt] * a2;
            U[2][c] = L.G[2][pt] * a0 + L.G[4][pt] * a1 + L.G[5][pt] * a2;
        }
    }
    // back to the RT dofs, D^T q~ added, scatter (colour 1 adds on shared faces)
    {
        auto body = [&](auto cc) {
            constexpr int C = decltype(cc)::value;
            constexpr int N0 = C == 0 ? P + 1 : P, N1 = C == 1 ? P + 1 : P, N2 = C == 2 ? P + 1 : P;
            const auto B1 = C == 1 ? &tfence<P, T>(tb)->L[0][0] : &tfence<P, T>(tb)->H[0][0];
            if (ps < Q * Q) {
                const auto B2 = C == 2 ? &tfence<P, T>(tb)->L[0][0] : &tfence<P, T>(tb)->H[0][0];
                T o[N2];
                pencil_mul<T, Q, N2, N2, true>(U[C], o, B2);
#pragma unroll
                for (int k = 0; k < N2; ++k) L.A2[(ps + Q * Q * k) * NR + r] = o[k];
            }
            __syncthreads();
            stage_il<T, NR, Q, Q, N2, 1, N1, N1, true>(L.A2, L.A1, B1, ps, r);
            __syncthreads();
            const auto B0 = C == 0 ? &tfence<P, T>(tb)->L[0][0] : &tfence<P, T>(tb)->H[0][0];
            for (int tt = ps; tt < N1 * N2; tt += PS) {
                const int j = tt % N1, k = tt / N1;
                T in[Q], yv[N0];
                using GQ = PencilGeom<Q, N1, N2, 0>;
#pragma unroll
                for (int q = 0; q < Q; ++q) in[q] = L.A1[(GQ::base(tt) + q) * NR + r];
                pencil_mul<T, Q, N0, N0, true>(in, yv, B0);
                const auto rl = rt_line<P, C>(g, ex, ey, ez, j, k);
#pragma unroll
                for (int i = 0; i < N0; ++i) {
                    int onf, bs;
                    rt_line_dof<P, C>(g, ex, rl, i, onf, bs);
                    const int64_t gi = ((int64_t)rl.base + i) * ldr + rx;
                    if (!live) continue;
                    if (bs >= 0 && ((ess >> (2 * C + bs)) & 1u)) {
                        y[gi] = x[gi];   // identity row
                        continue;
                    }
                    const int tn = C == 0 ? i : (C == 1 ? j : k);
                    int a = i, b = j, c = k;
                    T add = 0;
                    if (tn >= 1) {
                        if (C == 0) a = i - 1; else if (C == 1) b = j - 1; else c = k - 1;
                        add += L.sq[(a + P * (b + P * c)) * NR + r];
                    }
                    if (tn <= P - 1) add -= L.sq[(i + P * (j + P * k)) * NR + r];
                    const T v = yv[i] + add;
                    y[gi] = (colour == 1 && onf && bs < 0) ? y[gi] + v : v;
                }
            }
            __syncthreads();
        };
        body(std::integral_constant<int, 0>{});
        body(std::integral_constant<int, 1>{});
        body(std::integral_constant<int, 2>{});
    }
    // -kappa_e W_e^{-1} q~ by a local CG per right-hand side (Section 2.5)
    if constexpr (HAS_C) {
        if (with_c && kE != T(0)) {
            const auto Ti = &tfence<P, T>(tb)->Ti[0][0];
            const auto Bg = &tfence<P, T>(tb)->Bg[0][0];
            const auto Bg2 = &tfence<P, T>(tb)->Bg2[0][0];
            // Jacobi diagonal (Bg^2)^T gw, shared by the right-hand sides: the
            // threads of right-hand side 0 form it through the stage buffers
            if (ps < Q * Q && r == 0) {
                T gw[Q], o[P];
#pragma unroll
                for (int c = 0; c < Q; ++c) gw[c] = L.G[6][ps + Q * Q * c];
                pencil_mul<T, Q, P, P, true>(gw, o, Bg2);
#pragma unroll
                for (int k = 0; k < P; ++k) L.A1[(ps + Q * Q * k) * NR] = o[k];
            }
            __syncthreads();
            if (r == 0) stage_il<T, NR, Q, Q, P, 1, P, P, true>(L.A1, L.A2, Bg2, ps, 0);
            __syncthreads();
            if (ps < P * P && r == 0) {
                T in[Q], o[P];
#pragma unroll
                for (int q = 0; q < Q; ++q) in[q] = L.A2[(ps * Q + q) * NR];
                pencil_mul<T, Q, P, P, true>(in, o, Bg2);
#pragma unroll
                for (int k = 0; k < P; ++k) L.dW[ps * P + k] = T(1) / o[k];
            }
            // right-hand side T^{-T} q~: z, y, x
            stage_il<T, NR, P, P, P, 2, P, P, true>(L.sq, L.A1, Ti, ps, r);
            __syncthreads();
            stage_il<T, NR, P, P, P, 1, P, P, true>(L.A1, L.A2, Ti, ps, r);
            __syncthreads();
            T rv[P], zv[P], pv[P], xv[P], dW[P], Ap[P];
            double rz = 0.0;
            if (ps < P * P) {
                T in[P];
#pragma unroll
                for (int k = 0; k < P; ++k) in[k] = L.A2[(ps * P + k) * NR + r];
                pencil_mul<T, P, P, P, true>(in, rv, Ti);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    dW[k] = L.dW[ps * P + k];
                    zv[k] = rv[k] * dW[k];
                    pv[k] = zv[k];
                    xv[k] = 0;
                    rz += (double)(rv[k] * zv[k]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < P; ++k) rv[k] = zv[k] = pv[k] = xv[k] = dW[k] = Ap[k] = T(0);
            }
            T rzt = (T)il_sum<NR, P * P>(L.red, rz, ps, r);
            const T rr0 = rzt;
            bool done = !(rr0 > T(0));
            for (int it = 0; it < cgp.maxit; ++it) {
                if (!__syncthreads_or(!done)) break;
                if (ps < P * P) {
                    T o[Q];
                    pencil_mul<T, P, Q, P, false>(pv, o, Bg);
#pragma unroll
                    for (int q = 0; q < Q; ++q) L.A1[(ps * Q + q) * NR + r] = o[q];
                }
                __syncthreads();
                stage_il<T, NR, Q, P, P, 1, Q, P, false>(L.A1, L.A2, Bg, ps, r);
                __syncthreads();
                if (ps < Q * Q) {
                    T in[P], w[Q], o[P];
#pragma unroll
                    for (int k = 0; k < P; ++k) in[k] = L.A2[(ps + Q * Q * k) * NR + r];
                    pencil_mul<T, P, Q, P, false>(in, w, Bg);
#pragma unroll
                    for (int c = 0; c < Q; ++c) w[c] *= L.G[6][ps + Q * Q * c];
                    pencil_mul<T, Q, P, P, true>(w, o, Bg);
#pragma unroll
                    for (int k = 0; k < P; ++k) L.A1[(ps + Q * Q * k) * NR + r] = o[k];
                }
                __syncthreads();
                stage_il<T, NR, Q, Q, P, 1, P, P, true>(L.A1, L.A2, Bg, ps, r);
                __syncthreads();
                double pAp = 0.0;
                if (ps < P * P) {
                    T in[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) in[q] = L.A2[(ps * Q + q) * NR + r];
                    pencil_mul<T, Q, P, P, true>(in, Ap, Bg);
#pragma unroll
                    for (int k = 0; k < P; ++k) pAp += (double)(pv[k] * Ap[k]);
                }
                const T pApt = (T)il_sum<NR, P * P>(L.red, pAp, ps, r);
                const T alpha = rzt / pApt;
                double rzn = 0.0;
                if (!done && ps < P * P) {
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        xv[k] += alpha * pv[k];
                        rv[k] -= alpha * Ap[k];
                        zv[k] = rv[k] * dW[k];
                        rzn += (double)(rv[k] * zv[k]);
                    }
                }
                const T rznt = (T)il_sum<NR, P * P>(L.red, rzn, ps, r);
                if (!done) {
                    if (rznt <= cgp.tol * cgp.tol * rr0) {
                        done = true;
                    } else {
                        const T beta = rznt / rzt;
                        rzt = rznt;
#pragma unroll
                        for (int k = 0; k < P; ++k) pv[k] = zv[k] + beta * pv[k];
                    }
                }
            }
            __syncthreads();
            // IH-basis solution T^{-1} x: x (regs) -> y -> z, A1 = kappa sol
            if (ps < P * P) {
                T o[P];
                pencil_mul<T, P, P, P, false>(xv, o, Ti);
#pragma unroll
                for (int k = 0; k < P; ++k) L.A1[(ps * P + k) * NR + r] = o[k];
            }
            __syncthreads();
            stage_il<T, NR, P, P, P, 1, P, P, false>(L.A1, L.A2, Ti, ps, r);
            __syncthreads();
            stage_il<T, NR, P, P, P, 2, P, P, false>(L.A2, L.A1, Ti, ps, r);
            __syncthreads();
        }
    }
    // y_q = D u - kappa W^{-1} q~
    const bool cg = HAS_C && with_c && kE != T(0);
    for (int l = ps; l < NL; l += PS) {
        const int a = l % P, b = (l / P) % P, c = l / (P * P);
        T v = L.su[((a + 1) + (P + 1) * (b + P * c)) * NR + r] - L.su[(a + (P + 1) * (b + P * c)) * NR + r];
        v += L.su[(NC + a + P * ((b + 1) + (P + 1) * c)) * NR + r] - L.su[(NC + a + P * (b + (P + 1) * c)) * NR + r];
        v += L.su[(2 * NC + a + P * (b + P * (c + 1))) * NR + r] - L.su[(2 * NC + a + P * (b + P * c)) * NR + r];
        if (cg) v -= kE * L.A1[l * NR + r];
        if (live) y[(n_u + ee * NL + l) * ldr + rx] = v;
    }
}

// ---- batches of independent instances ------------------------------------
// LDS of one workgroup: the largest element-slot set over the degrees.
template <typename T>
constexpr size_t batch_lds_bytes() {
    size_t m = 0;
    const size_t s[6] = {sizeof(ElemLDS<1, T>) * Slot<1>::EPW, sizeof(ElemLDS<2, T>) * Slot<2>::EPW,
                         sizeof(ElemLDS<3, T>) * Slot<3>::EPW, sizeof(ElemLDS<4, T>) * Slot<4>::EPW,
                         sizeof(ElemLDS<5, T>) * Slot<5>::EPW, sizeof(ElemLDS<6, T>) * Slot<6>::EPW};
    for (size_t v : s) m = v > m ? v : m;
    return m;
}

// Not inlined: each degree's body keeps its own register allocation, so the
// persistent kernel needs the largest of them rather than their union.
template <int P, typename T>
__device__ __attribute__((noinline)) double batch_group(void* smem, const BatchInstDev& I, const T* x, T* y, T s_in,
                                                        const CGParams<T>& cgp, int ess_mode, int colour,
                                                        unsigned grp) {
    // arguments of a call arrive in vector registers; the table pointer is
    // uniform and must live in scalar registers for the scalar table loads
    const uint64_t tv = (uint64_t)I.tabk;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)tv);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(tv >> 32));
    const tkp<P, T> tb = (tkp<P, T>)(lo | (hi << 32));
    return apply_group<P, T>((ElemLDS<P, T>*)smem, I.g, I.vert, tb, (const T*)I.cm, (const T*)I.kap, I.ess,
                             ess_mode, I.n_u, x, y, s_in, cgp, I.with_c, colour, grp, I.nb, (const T*)I.winv);
}

// Persistent apply over all instances: each workgroup (one wavefront) takes
// the next tile from the work queue (tiles are sorted by decreasing cost) and
// runs its element groups with the element body of the tile's degree.  Every
// wavefront leaves once the queue is empty.
template <typename T>
__global__ __launch_bounds__(64) void batch_apply_kernel(const BatchInstDev* __restrict__ inst,
                                                         const BatchTile* __restrict__ tiles, int ntiles,
                                                         int* __restrict__ counter, const T* __restrict__ x,
                                                         T* __restrict__ y, const double* __restrict__ scale,
                                                         int scale_stride, const int* __restrict__ done,
                                                         int done_stride, int partials, int colour,
                                                         CGParams<T> cgp, int ess_mode) {
    __shared__ __align__(16) unsigned char smem[batch_lds_bytes<T>()];
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = atomicAdd(counter, 1);
        // the tile index is uniform over the wavefront: keep it (and the
        // instance data loaded through it) in scalar registers
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntiles) break;
        const BatchTile tl = tiles[t];
        if (done && done[(int64_t)tl.inst * done_stride]) continue;
        const BatchInstDev I = inst[tl.inst];
        const T s_in = scale ? (T)scale[(int64_t)tl.inst * scale_stride] : T(1);
        const T* xi = x + I.off;
        T* yi = y + I.off;
        for (unsigned k = 0; k < tl.ngrp; ++k) {
            const unsigned grp = tl.grp0 + k;
            double dot = 0.0;
            switch (I.p) {
                case 1: dot = batch_group<1, T>(smem, I, xi, yi, s_in, cgp, ess_mode, colour, grp); break;
                case 2: dot = batch_group<2, T>(smem, I, xi, yi, s_in, cgp, ess_mode, colour, grp); break;
                case 3: dot = batch_group<3, T>(smem, I, xi, yi, s_in, cgp, ess_mode, colour, grp); break;
                case 4: dot = batch_group<4, T>(smem, I, xi, yi, s_in, cgp, ess_mode, colour, grp); break;
                case 5: dot = batch_group<5, T>(smem, I, xi, yi, s_in, cgp, ess_mode, colour, grp); break;
                default: dot = batch_group<6, T>(smem, I, xi, yi, s_in, cgp, ess_mode, colour, grp); break;
            }
            if (partials && threadIdx.x == 0 && grp < I.nb) I.part[(int64_t)colour * I.nb + grp] = dot;
        }
    }
}

// The same work queue, one persistent launch per degree (the tiles of degree
// P form a contiguous range), with the body of that degree inlined.
template <int P, typename T>
__global__ __launch_bounds__(64) void batch_apply_deg_kernel(const BatchInstDev* __restrict__ inst,
                                                             const BatchTile* __restrict__ tiles, int ntiles,
                                                             int* __restrict__ counter, const T* __restrict__ x,
                                                             T* __restrict__ y, const double* __restrict__ scale,
                                                             int scale_stride, const int* __restrict__ done,
                                                             int done_stride, int partials, int colour,
                                                             CGParams<T> cgp, int ess_mode) {
    __shared__ ElemLDS<P, T> sm[Slot<P>::EPW];
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = atomicAdd(counter, 1);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntiles) break;
        const BatchTile tl = tiles[t];
        if (done && done[(int64_t)tl.inst * done_stride]) continue;
        const BatchInstDev I = inst[tl.inst];
        const T s_in = scale ? (T)scale[(int64_t)tl.inst * scale_stride] : T(1);
        for (unsigned k = 0; k < tl.ngrp; ++k) {
            const unsigned grp = tl.grp0 + k;
            const double dot = apply_group<P, T>(sm, I.g, I.vert, (tkp<P, T>)I.tabk, (const T*)I.cm,
                                                 (const T*)I.kap, I.ess, ess_mode, I.n_u, x + I.off, y + I.off, s_in,
                                                 cgp, I.with_c, colour, grp, I.nb, (const T*)I.winv);
            if (partials && threadIdx.x == 0 && grp < I.nb) I.part[(int64_t)colour * I.nb + grp] = dot;
        }
    }
}

constexpr int BATCH_COUNTERS = 16;

__global__ void reset_counters_kernel(int* c) {
    if (threadIdx.x < BATCH_COUNTERS) c[threadIdx.x] = 0;
}


// y_q = (weighted ? kappa_e : 1) W_e^{-1} x_q (same local CG).
template <int P, typename T>
__global__ __launch_bounds__(64) void mass_inverse_kernel(const T* __restrict__ pa, tkp<P, T> tb,
                                                          const T* __restrict__ kap, int weighted, int64_t ne,
                                                          const T* __restrict__ x, T* __restrict__ y,
                                                          CGParams<T> cgp) {
    using D = Dim<P>;
    using S = Slot<P>;
    constexpr int Q = D::Q, Q3 = D::Q3, NL = D::NL, W = S::W;
    __shared__ ElemLDS<P, T> sm[S::EPW];
    const int lane = threadIdx.x;
    const int slot = lane / W, t = lane % W;
    const int64_t e = (int64_t)blockIdx.x * S::EPW + slot;
    const bool valid = e < ne;
    const int64_t ee = valid ? e : ne - 1;
    ElemLDS<P, T>& L = sm[slot];
    if (valid)
        for (int l = t; l < NL; l += W) L.sq[l] = x[ee * NL + l];
    T gw[S::QC][Q];
    const T* pe = pa + (size_t)ee * NPA * Q3;
#pragma unroll
    for (int cc = 0; cc < S::QC; ++cc) {
        const int col = t + cc * W;
#pragma unroll
        for (int c = 0; c < Q; ++c) gw[cc][c] = col < Q * Q ? pe[6 * Q3 + col + Q * Q * c] : T(1);
    }
    __syncthreads();
    // A1 = W^{-1} sq
    local_cg<P, T>(L, tb, gw, t, valid, T(1), cgp);
    const T s = weighted ? kap[ee] : T(1);
    if (valid)
        for (int l = t; l < NL; l += W) y[ee * NL + l] = s * L.A1[l];
}

// W_e in the interpolation-histopolation basis and its inverse, one thread
// per element (p <= 2: at most 8 x 8):
//   W_e[i][j] = sum_q (w / det J)_q psi_i(x_q) psi_j(x_q),
// psi_(i0 i1 i2) = h_i0 h_i1 h_i2 at the (p+1)^3 Gauss-Legendre points, the
// quadrature the local CG and the stored factors use; inverted in place by
// Gauss-Jordan elimination (symmetric positive definite, no pivoting).
template <int P>
__global__ void local_inverse_kernel(int64_t ne, const double* __restrict__ pa, const Tables<double>* __restrict__ tab,
                                     double* __restrict__ winv, float* __restrict__ winv32) {
    constexpr int Q = P + 1, Q3 = Q * Q * Q, NL = P * P * P;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const double* gw = pa + (size_t)e * NPA * Q3 + 6 * Q3;
    double A[NL][NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
#pragma unroll
        for (int j = 0; j < NL; ++j) A[i][j] = 0.0;
    for (int q = 0; q < Q3; ++q) {
        const int a = q % Q, b = (q / Q) % Q, c = q / (Q * Q);
        double psi[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) psi[i] = tab->H[a][i % P] * tab->H[b][(i / P) % P] * tab->H[c][i / (P * P)];
        const double g = gw[q];
#pragma unroll
        for (int i = 0; i < NL; ++i)
#pragma unroll
            for (int j = 0; j < NL; ++j) A[i][j] += g * psi[i] * psi[j];
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const double pk = 1.0 / A[k][k];
        A[k][k] = 1.0;
#pragma unroll
        for (int j = 0; j < NL; ++j) A[k][j] *= pk;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            if (i == k) continue;
            const double f = A[i][k];
            A[i][k] = 0.0;
#pragma unroll
            for (int j = 0; j < NL; ++j) A[i][j] -= f * A[k][j];
        }
    }
    double* o = winv + (size_t)e * NL * NL;
    float* o32 = winv32 + (size_t)e * NL * NL;
#pragma unroll
    for (int i = 0; i < NL; ++i)
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            o[i * NL + j] = A[i][j];
            o32[i * NL + j] = (float)A[i][j];
        }
}

// blocks per colour: half-rows of ceil(nx / 2) elements, EPW elements per block
inline unsigned apply_blocks_per_colour(int nx, int ny, int nz, int epw) {
    const int64_t slots = (int64_t)((nx + 1) / 2) * ny * nz;
    return (unsigned)((slots + epw - 1) / epw);
}

inline int epw_of(int p) {
    switch (p) {
        case 1: return Slot<1>::EPW;
        case 2: return Slot<2>::EPW;
        case 3: return Slot<3>::EPW;
        case 4: return Slot<4>::EPW;
        case 5: return Slot<5>::EPW;
        default: return Slot<6>::EPW;
    }
}

template <typename T>
const Tables<T>& host_tables(const hd_ctx* c);
template <>
const Tables<double>& host_tables<double>(const hd_ctx* c) { return c->tab64_host; }
template <>
const Tables<float>& host_tables<float>(const hd_ctx* c) { return c->tab32_host; }

template <typename T>
CGParams<T> cg_params();
template <>
CGParams<double> cg_params<double>() { return {1e-14, 64}; }
template <>
CGParams<float> cg_params<float>() { return {1e-6f, 32}; }

template <int P, typename T>
void launch_apply_p(hd_ctx* c, const T* x, T* y, const RhsArgs& ra, int ess_mode) {
    Geo g = geo_of(c);
    const T* cm = std::is_same<T, double>::value ? (const T*)c->d_cm : (const T*)c->d_cm32;
    const T* kap = std::is_same<T, double>::value ? (const T*)c->d_kap : (const T*)c->d_kap32;
    const tkp<P, T> tb = (tkp<P, T>)(std::is_same<T, double>::value ? c->d_tabk64 : c->d_tabk32);
    const unsigned nb = apply_blocks_per_colour(c->nx, c->ny, c->nz, Slot<P>::EPW);
    // several right-hand sides: element groups rounded up to a multiple of 8
    // (the XCD count), one block per (group, right-hand side)
    const unsigned grid = ra.nrhs > 1 ? (unsigned)(((nb + 7) / 8) * 8 * (uint64_t)ra.nrhs) : nb;
    const T* winv = std::is_same<T, double>::value ? (const T*)c->d_winv : (const T*)c->d_winv32;
    for (int colour = 0; colour < 2; ++colour) {
        if (c->gamma_field)
            hipLaunchKernelGGL((block_apply_kernel<P, T, true, true>), dim3(grid), dim3(64), 0, c->stream, g,
                               c->d_vert, tb, cm, kap, c->ess, ess_mode, c->ne, c->n_u, x, y, ra, cg_params<T>(), 1,
                               colour, (int64_t)colour * nb, nb, winv, (const double*)c->d_gv);
        else if (!c->kappa_zero && c->affine)
            hipLaunchKernelGGL((block_apply_kernel<P, T, true, false, true>), dim3(grid), dim3(64), 0, c->stream, g,
                               c->d_vert, tb, cm, kap, c->ess, ess_mode, c->ne, c->n_u, x, y, ra, cg_params<T>(), 1,
                               colour, (int64_t)colour * nb, nb, winv, (const double*)nullptr);
        else if (!c->kappa_zero)
            hipLaunchKernelGGL((block_apply_kernel<P, T, true>), dim3(grid), dim3(64), 0, c->stream, g, c->d_vert, tb,
                               cm,
                               kap, c->ess, ess_mode, c->ne, c->n_u, x, y, ra, cg_params<T>(), 1, colour,
                               (int64_t)colour * nb, nb, winv, (const double*)nullptr);
        else if (c->affine)
            hipLaunchKernelGGL((block_apply_kernel<P, T, false, false, true>), dim3(grid), dim3(64), 0, c->stream, g,
                               c->d_vert, tb, cm, kap, c->ess, ess_mode, c->ne, c->n_u, x, y, ra, cg_params<T>(), 0,
                               colour, (int64_t)colour * nb, nb, (const T*)nullptr, (const double*)nullptr);
        else
            hipLaunchKernelGGL((block_apply_kernel<P, T, false>), dim3(grid), dim3(64), 0, c->stream, g, c->d_vert, tb,
                               cm,
                               kap, c->ess, ess_mode, c->ne, c->n_u, x, y, ra, cg_params<T>(), 0, colour,
                               (int64_t)colour * nb, nb, (const T*)nullptr, (const double*)nullptr);
    }
}

template <int P, typename T>
void launch_apply_uns_p(hd_ctx* c, const T* x, T* y, const RhsArgs& ra) {
    const T* cm = std::is_same<T, double>::value ? (const T*)c->d_cm : (const T*)c->d_cm32;
    const T* kap = std::is_same<T, double>::value ? (const T*)c->d_kap : (const T*)c->d_kap32;
    const tkp<P, T> tb = (tkp<P, T>)(std::is_same<T, double>::value ? c->d_tabk64 : c->d_tabk32);
    const T* winv = std::is_same<T, double>::value ? (const T*)c->d_winv : (const T*)c->d_winv32;
    const UnsArgs ua = {c->d_l2g, c->d_evx, c->d_essm};
    const unsigned nb = (unsigned)((c->ne + Slot<P>::EPW - 1) / Slot<P>::EPW);
    const int64_t N = c->n_u + c->n_q;
    hipLaunchKernelGGL(uns_init_kernel<T>, dim3((unsigned)std::min<int64_t>((c->n_u + 255) / 256, 4096), ra.nrhs),
                       dim3(256), 0, c->stream, c->n_u, (const uint8_t*)c->d_essm, x, y, ra);
    if (!c->kappa_zero)
        hipLaunchKernelGGL((block_apply_uns_kernel<P, T, true>), dim3(nb, ra.nrhs), dim3(64), 0, c->stream, ua, c->ne,
                           tb, cm, kap, c->n_u, x, y, ra, cg_params<T>(), 1, winv);
    else
        hipLaunchKernelGGL((block_apply_uns_kernel<P, T, false>), dim3(nb, ra.nrhs), dim3(64), 0, c->stream, ua,
                           c->ne, tb, cm, kap, c->n_u, x, y, ra, cg_params<T>(), 0, (const T*)nullptr);
    if (ra.partial)
        hipLaunchKernelGGL(uns_dot_kernel<T>, dim3(UNS_DOT_BLOCKS, ra.nrhs), dim3(256), 0, c->stream, N, x,
                           (const T*)y, ra);
}

// Right-hand sides per workgroup of the interleaved apply: the largest of
// 16, 8, 4, 2, 1 whose pencil slots hold the (p+1)^2 quadrature columns and
// whose LDS stays within 48 KB.
template <int P, typename T>
constexpr int il_nr() {
    constexpr int Q = P + 1;
    int nr = 16;
    while (nr > 1 && (Q * Q > IL_T / nr || sizeof(T) * (size_t)((Dim<P>::NRT + Dim<P>::NL + 2 * Dim<P>::Q3) * nr +
                                                                 8 * Dim<P>::Q3 + 24) + 8 * IL_T > 48 * 1024))
        nr /= 2;
    return nr;
}

template <int P, typename T>
void launch_apply_il_p(hd_ctx* c, const T* x, T* y, int nrhs) {
    constexpr int NR = il_nr<P, T>();
    Geo g = geo_of(c);
    const T* cm = std::is_same<T, double>::value ? (const T*)c->d_cm : (const T*)c->d_cm32;
    const T* kap = std::is_same<T, double>::value ? (const T*)c->d_kap : (const T*)c->d_kap32;
    const tkp<P, T> tb = (tkp<P, T>)(std::is_same<T, double>::value ? c->d_tabk64 : c->d_tabk32);
    const unsigned nb = apply_blocks_per_colour(c->nx, c->ny, c->nz, 1);
    const dim3 grid(nb, (unsigned)((nrhs + NR - 1) / NR));
    for (int colour = 0; colour < 2; ++colour) {
        if (!c->kappa_zero)
            hipLaunchKernelGGL((block_apply_il_kernel<P, T, NR, true>), grid, dim3(IL_T), 0, c->stream, g, c->d_vert,
                               tb, cm, kap, c->ess, c->n_u, x, y, nrhs, cg_params<T>(), 1, colour, nb);
        else
            hipLaunchKernelGGL((block_apply_il_kernel<P, T, NR, false>), grid, dim3(IL_T), 0, c->stream, g,
                               c->d_vert, tb, cm, kap, c->ess, c->n_u, x, y, nrhs, cg_params<T>(), 0, colour, nb);
    }
}

template <int P, typename T>
void launch_minv_p(hd_ctx* c, const T* x, T* y, bool weighted) {
    const T* pa = std::is_same<T, double>::value ? (const T*)c->d_pa : (const T*)c->d_pa32;
    const T* kap = std::is_same<T, double>::value ? (const T*)c->d_kap : (const T*)c->d_kap32;
    const tkp<P, T> tb = (tkp<P, T>)(std::is_same<T, double>::value ? c->d_tabk64 : c->d_tabk32);
    const unsigned nb = (unsigned)((c->ne + Slot<P>::EPW - 1) / Slot<P>::EPW);
    hipLaunchKernelGGL((mass_inverse_kernel<P, T>), dim3(nb), dim3(64), 0, c->stream, pa, tb, kap, weighted ? 1 : 0,
                       c->ne, x, y, cg_params<T>());
}

template <typename T>
void dispatch_apply(hd_ctx* c, const T* x, T* y, const RhsArgs& ra, int em) {
    if (c->unstructured) {
        switch (c->p) {
            case 1: launch_apply_uns_p<1, T>(c, x, y, ra); break;
            case 2: launch_apply_uns_p<2, T>(c, x, y, ra); break;
            case 3: launch_apply_uns_p<3, T>(c, x, y, ra); break;
            case 4: launch_apply_uns_p<4, T>(c, x, y, ra); break;
            case 5: launch_apply_uns_p<5, T>(c, x, y, ra); break;
            case 6: launch_apply_uns_p<6, T>(c, x, y, ra); break;
        }
        return;
    }
    switch (c->p) {
        case 1: launch_apply_p<1, T>(c, x, y, ra, em); break;
        case 2: launch_apply_p<2, T>(c, x, y, ra, em); break;
        case 3: launch_apply_p<3, T>(c, x, y, ra, em); break;
        case 4: launch_apply_p<4, T>(c, x, y, ra, em); break;
        case 5: launch_apply_p<5, T>(c, x, y, ra, em); break;
        case 6: launch_apply_p<6, T>(c, x, y, ra, em); break;
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

template <int P>
int upload_tabk_p(hd_ctx* c) {
    const TabK<P, double> t64 = make_tabk<P, double>(c->tab64_host);
    const TabK<P, float> t32 = make_tabk<P, float>(c->tab32_host);
    dfree(c->d_tabk64);
    dfree(c->d_tabk32);
    c->d_tabk64 = dalloc<TabK<P, double>>(1);
    c->d_tabk32 = dalloc<TabK<P, float>>(1);
    if (!c->d_tabk64 || !c->d_tabk32) return set_err(c, HD_ERR_OOM, "kernel tables");
    HD_HIP(c, hipMemcpyAsync(c->d_tabk64, &t64, sizeof(t64), hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemcpyAsync(c->d_tabk32, &t32, sizeof(t32), hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

int upload_kernel_tables(hd_ctx* c) {
    switch (c->p) {
        case 1: return upload_tabk_p<1>(c);
        case 2: return upload_tabk_p<2>(c);
        case 3: return upload_tabk_p<3>(c);
        case 4: return upload_tabk_p<4>(c);
        case 5: return upload_tabk_p<5>(c);
        case 6: return upload_tabk_p<6>(c);
    }
    return set_err(c, HD_ERR_ARG, "p out of range");
}

int64_t apply_partial_count(const hd_ctx* c) {
    if (c->unstructured) return UNS_DOT_BLOCKS;
    return 2 * (int64_t)apply_blocks_per_colour(c->nx, c->ny, c->nz, epw_of(c->p));
}

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
    RhsArgs ra = {1, N, nullptr, 0, nullptr, 0, nullptr, 0};
    dispatch_apply<double>(c, t, y, ra, ESS_NONE);
    hipLaunchKernelGGL(lift_finish_kernel, dim3(nb), dim3(256), 0, c->stream, g, c->p, c->ess, c->n_u, N, ubc, y, b);
    hipError_t e = hipStreamSynchronize(c->stream);
    dfree(t);
    dfree(y);
    if (e != hipSuccess) return set_err(c, HD_ERR_HIP, hipGetErrorString(e));
    return HD_OK;
}

int launch_apply(hd_ctx* c, int prec, int nrhs, const void* x, void* y, const double* in_scale, int scale_stride,
                 double* dot_partial, int64_t part_stride, int ess_mode, const int* done, int done_stride) {
    if (c->time_apply) HD_HIP(c, hipEventRecord(c->ev0, c->stream));
    const RhsArgs ra = {nrhs, c->n_u + c->n_q, in_scale, scale_stride, done, done_stride, dot_partial, part_stride};
    if (prec == HD_F64)
        dispatch_apply<double>(c, (const double*)x, (double*)y, ra, ess_mode);
    else
        dispatch_apply<float>(c, (const float*)x, (float*)y, ra, ess_mode);
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

int launch_apply_interleaved(hd_ctx* c, int prec, int nrhs, const void* x, void* y) {
    const bool f64 = prec == HD_F64;
    switch (c->p) {
#define IL(PP)                                                                                               \
    case PP:                                                                                                 \
        if (f64) launch_apply_il_p<PP, double>(c, (const double*)x, (double*)y, nrhs);                     \
        else launch_apply_il_p<PP, float>(c, (const float*)x, (float*)y, nrhs);                            \
        break;
        IL(1) IL(2) IL(3) IL(4) IL(5) IL(6)
#undef IL
        default: return set_err(c, HD_ERR_ARG, "p out of range");
    }
    HD_HIP(c, hipGetLastError());
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


namespace {

template <int P, typename T>
void launch_deg(hd_ctx* c, const BatchState& B, const BatchInstDev* di, int colour, const T* x, T* y,
                const double* scale, int scale_stride, const int* done, int done_stride, bool partials) {
    if (B.deg_nt[P] == 0) return;
    hipLaunchKernelGGL((batch_apply_deg_kernel<P, T>), dim3(B.grid), dim3(64), 0, c->stream, di,
                       B.d_tiles + B.deg_t0[P], B.deg_nt[P], B.d_counter + 2 + 2 * (P - 1) + colour, x, y, scale,
                       scale_stride, done, done_stride, partials ? 1 : 0, colour, cg_params<T>(), (int)ESS_IDENTITY);
}

template <typename T>
void launch_batch_t(hd_ctx* c, const BatchInstDev* di, const T* x, T* y, const double* scale, int scale_stride,
                    const int* done, int done_stride, bool partials) {
    const BatchState& B = *c->batch;
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, c->stream, B.d_counter);
    for (int colour = 0; colour < 2; ++colour) {
        if (B.mode == 0) {
            hipLaunchKernelGGL(batch_apply_kernel<T>, dim3(B.grid), dim3(64), 0, c->stream, di, B.d_tiles, B.ntiles,
                               B.d_counter + colour, x, y, scale, scale_stride, done, done_stride, partials ? 1 : 0,
                               colour, cg_params<T>(), (int)ESS_IDENTITY);
        } else {
            launch_deg<6, T>(c, B, di, colour, x, y, scale, scale_stride, done, done_stride, partials);
            launch_deg<5, T>(c, B, di, colour, x, y, scale, scale_stride, done, done_stride, partials);
            launch_deg<4, T>(c, B, di, colour, x, y, scale, scale_stride, done, done_stride, partials);
            launch_deg<3, T>(c, B, di, colour, x, y, scale, scale_stride, done, done_stride, partials);
            launch_deg<2, T>(c, B, di, colour, x, y, scale, scale_stride, done, done_stride, partials);
            launch_deg<1, T>(c, B, di, colour, x, y, scale, scale_stride, done, done_stride, partials);
        }
    }
}

}  // namespace

int launch_batch_apply(hd_ctx* c, int prec, const void* x, void* y, const double* scale, int scale_stride,
                       const int* done, int done_stride, bool partials) {
    BatchState& B = *c->batch;
    if (B.mode == 2) {
        // each instance's own full-grid apply on its segment (the per-instance
        // partial sums have the layout of a single apply)
        const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
        for (size_t i = 0; i < B.inst.size(); ++i) {
            hd_ctx* s = B.inst[i];
            const size_t o = es * (size_t)B.off[i];
            const int rc = launch_apply(s, prec, 1, (const char*)x + o, (char*)y + o,
                                        scale ? scale + (size_t)scale_stride * i : nullptr, scale_stride,
                                        partials ? B.d_part + B.part_off[i] : nullptr, apply_partial_count(s),
                                        ESS_IDENTITY, done ? done + (size_t)done_stride * i : nullptr, done_stride);
            if (rc) return set_err(c, rc, "instance " + std::to_string(i) + ": " + s->err);
        }
        return HD_OK;
    }
    if (prec == HD_F64)
        launch_batch_t<double>(c, B.d_inst64, (const double*)x, (double*)y, scale, scale_stride, done, done_stride,
                               partials);
    else
        launch_batch_t<float>(c, B.d_inst32, (const float*)x, (float*)y, scale, scale_stride, done, done_stride,
                              partials);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int batch_build_tiles(hd_ctx* c, int tile_groups) {
    BatchState& B = *c->batch;
    const int ninst = (int)B.inst.size();
    std::vector<BatchTile> tiles;
    std::vector<BatchInstDev> d64(ninst), d32(ninst);
    std::vector<std::pair<int, int>> order;   // (-cost rank, instance)
    for (int i = 0; i < ninst; ++i) {
        hd_ctx* s = B.inst[i];
        BatchInstDev a;
        a.g = geo_of(s);
        a.p = s->p;
        a.with_c = s->kappa_zero ? 0 : 1;
        a.ess = s->ess;
        a.nb = apply_blocks_per_colour(s->nx, s->ny, s->nz, epw_of(s->p));
        a.n_u = s->n_u;
        a.off = B.off[i];
        a.part = B.d_part + B.part_off[i];
        BatchInstDev b = a;
        a.vert = s->d_vert;
        a.winv = s->d_winv;
        a.cm = s->d_cm;
        a.kap = s->d_kap;
        a.tabk = s->d_tabk64;
        b.vert = s->d_vert;
        b.winv = s->d_winv32;
        b.cm = s->d_cm32;
        b.kap = s->d_kap32;
        b.tabk = s->d_tabk32;
        d64[i] = a;
        d32[i] = b;
        order.push_back({s->p, i});
    }
    // most expensive degree first, so that the long tiles start early
    std::stable_sort(order.begin(), order.end(), [](const std::pair<int, int>& u, const std::pair<int, int>& v) {
        return u.first > v.first;
    });
    for (int q = 0; q < 7; ++q) B.deg_t0[q] = B.deg_nt[q] = 0;
    for (auto& pr : order) {
        const int i = pr.second;
        const unsigned nb = d64[i].nb;
        const int p = d64[i].p;
        if (B.deg_nt[p] == 0) B.deg_t0[p] = (int)tiles.size();
        for (unsigned g0 = 0; g0 < nb; g0 += (unsigned)tile_groups) {
            tiles.push_back({i, g0, std::min<unsigned>((unsigned)tile_groups, nb - g0)});
            ++B.deg_nt[p];
        }
    }
    dfree(B.d_tiles);
    if (!B.d_inst64) B.d_inst64 = dalloc<BatchInstDev>(ninst);
    if (!B.d_inst32) B.d_inst32 = dalloc<BatchInstDev>(ninst);
    B.d_tiles = dalloc<BatchTile>(tiles.size());
    if (!B.d_inst64 || !B.d_inst32 || !B.d_tiles) return set_err(c, HD_ERR_OOM, "batch tiles");
    HD_HIP(c, hipMemcpyAsync(B.d_inst64, d64.data(), sizeof(BatchInstDev) * ninst, hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemcpyAsync(B.d_inst32, d32.data(), sizeof(BatchInstDev) * ninst, hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemcpyAsync(B.d_tiles, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice,
                             c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    B.ntiles = (int)tiles.size();
    B.tile_groups = tile_groups;
    return HD_OK;
}

void free_local_inverse(hd_ctx* c) {
    dfree(c->d_winv);
    dfree(c->d_winv32);
    c->d_winv = nullptr;
    c->d_winv32 = nullptr;
}

int build_local_inverse(hd_ctx* c) {
    free_local_inverse(c);
    const bool want = c->p <= 2 && !c->kappa_zero && c->local_solver != HD_LOCAL_CG;
    if (!want) return HD_OK;
    const int64_t nl = (int64_t)c->p * c->p * c->p;
    c->d_winv = dalloc<double>(c->ne * nl * nl);
    c->d_winv32 = dalloc<float>(c->ne * nl * nl);
    if (!c->d_winv || !c->d_winv32) {
        free_local_inverse(c);
        return set_err(c, HD_ERR_OOM, "explicit element inverses");
    }
    const unsigned nbk = (unsigned)((c->ne + 127) / 128);
    if (c->p == 1)
        hipLaunchKernelGGL(local_inverse_kernel<1>, dim3(nbk), dim3(128), 0, c->stream, c->ne, c->d_pa, c->d_tab64,
                           c->d_winv, c->d_winv32);
    else
        hipLaunchKernelGGL(local_inverse_kernel<2>, dim3(nbk), dim3(128), 0, c->stream, c->ne, c->d_pa, c->d_tab64,
                           c->d_winv, c->d_winv32);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

}  // namespace hd
