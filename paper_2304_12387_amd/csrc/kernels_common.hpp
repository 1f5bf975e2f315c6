// Device helpers shared by the HIP kernels: element dimensions, LDS tensor
// contractions (sum factorisation) and wave-level reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "hd_internal.hpp"

namespace hd {

template <int P>
struct Dim {
    static constexpr int Q = P + 1;          // quadrature points per direction
    static constexpr int Q3 = Q * Q * Q;
    static constexpr int NL = P * P * P;     // L2 dofs per element
    static constexpr int NC = P * P * (P + 1);   // RT dofs per component
    static constexpr int NRT = 3 * NC;
};

// Contract the 3D array `in` of shape (I0, I1, I2) (I0 fastest) along
// dimension DIM with the matrix B: the output has extent M along DIM and
//   out[.., o, ..] = sum_k Bm(o, k) in[.., k, ..],
//   Bm(o, k) = TR ? B[k * LDB + o] : B[o * LDB + k].
// All threads of the team [tid, nt) share the outputs.
template <typename T, int I0, int I1, int I2, int DIM, int M, bool TR, int LDB>
__device__ __forceinline__ void contract(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ B,
                                         int tid, int nt) {
    constexpr int K = DIM == 0 ? I0 : (DIM == 1 ? I1 : I2);
    constexpr int O0 = DIM == 0 ? M : I0;
    constexpr int O1 = DIM == 1 ? M : I1;
    constexpr int O2 = DIM == 2 ? M : I2;
    constexpr int NO = O0 * O1 * O2;
    for (int idx = tid; idx < NO; idx += nt) {
        const int o0 = idx % O0;
        const int o1 = (idx / O0) % O1;
        const int o2 = idx / (O0 * O1);
        const int o = DIM == 0 ? o0 : (DIM == 1 ? o1 : o2);
        T s = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i0 = DIM == 0 ? k : o0;
            const int i1 = DIM == 1 ? k : o1;
            const int i2 = DIM == 2 ? k : o2;
            const T b = TR ? B[k * LDB + o] : B[o * LDB + k];
            s += b * in[i0 + I0 * (i1 + I1 * i2)];
        }
        out[idx] = s;
    }
}

// Global index of the RT dof (component c, local (i, j, k)) of element
// (ex, ey, ez); also reports whether it lies on the domain boundary and on
// which side (0 = min, 1 = max).
template <int P>
__device__ __forceinline__ int64_t rt_global(const Geo& g, int c, int ex, int ey, int ez, int i, int j, int k,
                                             int& on_elem_face, int& bnd_side) {
    int gi = ex * P + i, gj = ey * P + j, gk = ez * P + k;
    int d0 = g.nx * P, d1 = g.ny * P, d2 = g.nz * P;
    int n_along, gcoord, lcoord;
    if (c == 0) { d0 += 1; n_along = g.nx * P; gcoord = gi; lcoord = i; }
    else if (c == 1) { d1 += 1; n_along = g.ny * P; gcoord = gj; lcoord = j; }
    else { d2 += 1; n_along = g.nz * P; gcoord = gk; lcoord = k; }
    on_elem_face = (lcoord == 0 || lcoord == P);
    bnd_side = gcoord == 0 ? 0 : (gcoord == n_along ? 1 : -1);
    return g.off[c] + gi + (int64_t)d0 * (gj + (int64_t)d1 * gk);
}

template <int P>
__device__ __forceinline__ void local_ijk(int c, int l, int& i, int& j, int& k) {
    // component shape: (P+1) along c, P along the others, first index fastest
    const int n0 = c == 0 ? P + 1 : P;
    const int n1 = c == 1 ? P + 1 : P;
    i = l % n0;
    j = (l / n0) % n1;
    k = l / (n0 * n1);
}

// Is the global RT dof t essential (on a selected side of the box)?
__device__ __forceinline__ bool rt_is_essential(const Geo& g, int P, uint32_t ess, int64_t t) {
    const int c = t >= g.off[2] ? 2 : (t >= g.off[1] ? 1 : 0);
    const int64_t r = t - g.off[c];
    const int64_t d0 = (int64_t)g.nx * P + (c == 0), d1 = (int64_t)g.ny * P + (c == 1);
    const int64_t gi = r % d0, gj = (r / d0) % d1, gk = r / (d0 * d1);
    const int64_t coord = c == 0 ? gi : (c == 1 ? gj : gk);
    const int64_t nal = c == 0 ? (int64_t)g.nx * P : (c == 1 ? (int64_t)g.ny * P : (int64_t)g.nz * P);
    return (coord == 0 && ((ess >> (2 * c)) & 1u)) || (coord == nal && ((ess >> (2 * c + 1)) & 1u));
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b mod 8), each with its own L2.  xcd_chunk maps block b to a logical
// block so that each XCD takes a contiguous chunk of [0, n): work that
// shares cache lines with its neighbours (elements sharing faces, matrix
// rows reading nearby columns) meets in one L2 instead of each XCD fetching
// the line.  A bijection of [0, n).
__device__ __forceinline__ unsigned xcd_chunk(unsigned b, unsigned n) {
    const unsigned x = b % 8, k = b / 8;
    return x * (n / 8) + (x < n % 8 ? x : n % 8) + k;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void team_sync() { __syncthreads(); }

}  // namespace hd
