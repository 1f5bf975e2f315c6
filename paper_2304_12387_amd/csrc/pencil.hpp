// Register-pencil tensor contractions for the element kernels.
//
// An element tensor of shape (N0, N1, N2) (N0 fastest) is processed by a team
// of lanes; for a contraction along one direction each active lane owns one
// 1D line ("pencil") of the tensor along that direction, reads it into
// registers, multiplies it by a small dense 1D matrix whose entries are
// uniform across the wavefront (kernel arguments, held in scalar registers)
// and writes the resulting pencil.  LDS is used only to change the pencil
// direction between stages, so the multiply-adds read no LDS at all.
#pragma once

#include "kernels_common.hpp"

namespace hd {

// 1D tables of degree P passed by value (kernel-argument constant buffer).
template <int P, typename T>
struct TabK {
    static constexpr int Q = P + 1;
    T L[Q][P + 1];     // l_i(x_a)
    T H[Q][P];         // h_j(x_a)
    T Bg[Q][P];        // Gauss-Legendre nodal basis at x_a
    T Bg2[Q][P];       // Bg^2
    T Ti[P][P];        // inverse change of basis IH -> GL nodal
    T xq[Q];           // Gauss-Legendre points on [0, 1]
    T wq[Q];           // and weights
};

template <int P, typename T>
TabK<P, T> make_tabk(const Tables<T>& t) {
    TabK<P, T> k;
    for (int a = 0; a <= P; ++a) {
        for (int i = 0; i <= P; ++i) k.L[a][i] = t.L[a][i];
        for (int j = 0; j < P; ++j) {
            k.H[a][j] = t.H[a][j];
            k.Bg[a][j] = t.Bg[a][j];
            k.Bg2[a][j] = t.Bg2[a][j];
        }
    }
    for (int r = 0; r < P; ++r)
        for (int c = 0; c < P; ++c) k.Ti[r][c] = t.Tinv[r][c];
    for (int a = 0; a <= P; ++a) {
        k.xq[a] = t.xq[a];
        k.wq[a] = t.wq[a];
    }
    return k;
}

// Tables live in device memory in the constant address space, so that loads
// with wavefront-uniform addresses become scalar loads.  `stage_tab` hides
// the table pointer from loop-invariant code motion: each stage re-reads its
// 1D matrix (a few scalar-cache hits) instead of the compiler hoisting every
// table into scalar registers up front, which would exceed the scalar
// register file and spill into vector-register lanes.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> stage_tab(cptr<T> p) {
    uint64_t v = (uint64_t)p;
    asm volatile("" : "+s"(v));
    return (cptr<T>)v;
}

// Pencil index helpers for a (N0, N1, N2) array, contraction along DIM.
template <int N0, int N1, int N2, int DIM>
struct PencilGeom {
    static constexpr int K = DIM == 0 ? N0 : (DIM == 1 ? N1 : N2);
    static constexpr int NP = N0 * N1 * N2 / K;
    static constexpr int STRIDE = DIM == 0 ? 1 : (DIM == 1 ? N0 : N0 * N1);
    // base offset of pencil t in an array with this shape
    __device__ static __forceinline__ int base(int t) {
        if (DIM == 0) return N0 * t;                    // t = j + N1 k
        if (DIM == 1) return (t % N0) + N0 * N1 * (t / N0);   // t = i + N0 k
        return t;                                       // t = i + N0 j
    }
};

// out-pencil = B * in-pencil, B(o, s) = TR ? Bm[s][o] : Bm[o][s].
template <typename T, int K, int M, int LDB, bool TR, typename BP>
__device__ __forceinline__ void pencil_mul(const T (&in)[K], T (&out)[M], BP Bm) {
#pragma unroll
    for (int o = 0; o < M; ++o) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) s += (TR ? Bm[k * LDB + o] : Bm[o * LDB + k]) * in[k];
        out[o] = s;
    }
}

// Read pencil t of `src` (shape N0,N1,N2, along DIM) into registers.
template <typename T, int N0, int N1, int N2, int DIM>
__device__ __forceinline__ void pencil_load(const T* src, int t, T (&v)[PencilGeom<N0, N1, N2, DIM>::K]) {
    using G = PencilGeom<N0, N1, N2, DIM>;
    const int b = G::base(t);
#pragma unroll
    for (int s = 0; s < G::K; ++s) v[s] = src[b + s * G::STRIDE];
}

// Write pencil t (length M along DIM) into `dst` of shape (N0,N1,N2) with
// extent M along DIM.
template <typename T, int N0, int N1, int N2, int DIM, int M>
__device__ __forceinline__ void pencil_store(T* dst, int t, const T (&v)[M]) {
    constexpr int O0 = DIM == 0 ? M : N0, O1 = DIM == 1 ? M : N1, O2 = DIM == 2 ? M : N2;
    using G = PencilGeom<O0, O1, O2, DIM>;
    const int b = G::base(t);
#pragma unroll
    for (int s = 0; s < M; ++s) dst[b + s * G::STRIDE] = v[s];
}

// Full LDS -> LDS stage: contract `src` (N0,N1,N2) along DIM to extent M.
// A team of W lanes (t in [0, W)) takes the pencils in passes of W.
template <typename T, int N0, int N1, int N2, int DIM, int M, int LDB, bool TR, int W, typename BP>
__device__ __forceinline__ void stage_lds(const T* src, T* dst, BP Bm, int t) {
    using G = PencilGeom<N0, N1, N2, DIM>;
#pragma unroll
    for (int pass = 0; pass < (G::NP + W - 1) / W; ++pass) {
        const int tt = t + pass * W;
        if (tt < G::NP) {
            T in[G::K], out[M];
            pencil_load<T, N0, N1, N2, DIM>(src, tt, in);
            pencil_mul<T, G::K, M, LDB, TR>(in, out, Bm);
            pencil_store<T, N0, N1, N2, DIM, M>(dst, tt, out);
        }
    }
}

// Lane exchanges for the slot reductions, on the 32-bit halves of a value:
// DPP moves inside rows of 16 lanes (no LDS access) and ds_swizzle across
// the two rows of a 32-lane group.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_x(double v) {
    return __hiloint2double(dpp_i<CTRL>(__double2hiint(v)), dpp_i<CTRL>(__double2loint(v)));
}
template <int CTRL>
__device__ __forceinline__ float dpp_x(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
// lane l <- lane l ^ XOR inside each group of 32 lanes (swizzle bit mode)
template <int XOR>
__device__ __forceinline__ double swz_x(double v) {
    constexpr int pat = 0x1F | (XOR << 10);
    return __hiloint2double(__builtin_amdgcn_ds_swizzle(__double2hiint(v), pat),
                            __builtin_amdgcn_ds_swizzle(__double2loint(v), pat));
}
template <int XOR>
__device__ __forceinline__ float swz_x(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (XOR << 10)));
}

// Sum over the aligned group of W lanes (W = 4, 8, 16, 32 or 64), returned
// to every lane of the group; a fixed order, so it is reproducible.
template <typename T, int W>
__device__ __forceinline__ T slot_sum(T v) {
    static_assert(W == 4 || W == 8 || W == 16 || W == 32 || W == 64, "slot width");
    v += dpp_x<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_x<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (W == 8) v += swz_x<4>(v);
    if constexpr (W >= 16) {
        v += dpp_x<0x124>(v);   // row_ror:4
        v += dpp_x<0x128>(v);   // row_ror:8
    }
    if constexpr (W >= 32) v += swz_x<16>(v);
    if constexpr (W == 64) {
        if constexpr (sizeof(T) == 8) {
            const double a = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                              __builtin_amdgcn_readlane(__double2loint(v), 0));
            const double b = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                                              __builtin_amdgcn_readlane(__double2loint(v), 32));
            v = a + b;
        } else {
            v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)) +
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
        }
    }
    return v;
}

}  // namespace hd
