// Block-preconditioned MINRES for the transformed saddle-point system
// (Sections 2 and 3: the system is symmetric indefinite, the preconditioner
// symmetric positive definite, so MINRES with its short recurrences applies).
// Preconditioned Lanczos with Givens rotations (Paige-Saunders); |eta| is the
// B^{-1}-norm of the residual and the iteration stops when
// |eta| <= tol |eta_0|.
//
// Several right-hand sides are solved together: vectors are stored one after
// the other, every right-hand side has its own FP64 recurrence state on the
// device (one reduction block per right-hand side) and its own stop flag,
// and the kernels of one iteration serve all of them (the block apply loads
// each element's geometric factors once for all right-hand sides).  No host
// round trip is needed between iterations; the host polls the flags every
// few iterations.  Inner products are two-stage deterministic reductions in
// FP64.  Per iteration:
//   1. q = A (z_j / gamma_j)          block apply, fused partials of <q, z_j/gamma_j>
//   2. delta = sum of partials
//   3. v_{j+1} = q - (delta/gamma_j) v_j - (gamma_j/gamma_{j-1}) v_{j-1}
//      z_{j+1,u} = (tau M~)^{-1} v_{j+1,u}, partials of <z, v> (fused)
//   4. z_{j+1,q} = V-cycle(v_{j+1,q}), partials of <z, v> (fused)
//   5. Givens update, stop test
//   6. w_{j+1} = (z_j/gamma_j - a3 w_{j-1} - a2 w_j) / a1,
//      x += c_{j+1} eta w_{j+1}
// Mixed precision: FP64 residual refinement around an FP32 inner MINRES
// (FP32 vectors, operator and preconditioner, FP64 inner products and
// scalars, FP64 coarse solve).  FP32 preconditioner: the FP64 recurrence and
// operator with the Schur-block V-cycle in FP32 (the diagonal (1,1) block
// stays FP64; it costs one vector pass either way).
#include "kernels_common.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <type_traits>
#include <vector>

namespace hd {

namespace {

constexpr int BS = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + BS - 1) / BS); }
// kernels emitting per-block partial sums use at most RED_BLOCKS blocks
constexpr unsigned RED_BLOCKS = 1024;
inline unsigned red_grid(int64_t n) { return nblk(n) < RED_BLOCKS ? nblk(n) : RED_BLOCKS; }

struct MinresState {
    double gamma, gamma_old, delta;
    double c, c_old, s, s_old;
    double eta, eta0;
    double inv_gamma;     // 1 / gamma_j: scale of the next apply
    double cv1, cv2;      // delta / gamma_j, gamma_j / gamma_{j-1}
    double a1inv, a2, a3, zscale, xcoef;
    double tol;
    int iter, stop, skipped, status;
};
constexpr int ST_STRIDE_D = sizeof(MinresState) / sizeof(double);
constexpr int ST_STRIDE_I = sizeof(MinresState) / sizeof(int);
static_assert(sizeof(MinresState) % sizeof(double) == 0, "state layout");

__device__ double block_sum(double v) {
    __shared__ double s[1024];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

// First stage for long partial-sum arrays: block b of right-hand side r
// (blockIdx.y) sums entries [b chunk, (b + 1) chunk) into out[r gridDim.x + b]
// (fixed order, so the total stays deterministic).
__global__ void k_sum_stage(const double* __restrict__ part, int64_t n, int64_t stride, int64_t chunk,
                            double* __restrict__ out, const MinresState* __restrict__ st) {
    if (st && st[blockIdx.y].stop) return;
    const double* p = part + blockIdx.y * stride;
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double acc = 0.0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) acc += p[k];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// one block per right-hand side r: delta = sum of its apply partials
__device__ void delta_body(MinresState* S, const double* __restrict__ p, int64_t n) {
    if (S->stop) return;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) acc += p[k];
    const double d = block_sum(acc);
    if (threadIdx.x == 0) {
        S->delta = d;
        S->cv1 = d / S->gamma;
        S->cv2 = S->gamma / S->gamma_old;
    }
}

__global__ void k_delta(MinresState* st, const double* __restrict__ part, int64_t n, int64_t stride) {
    delta_body(st + blockIdx.x, part + blockIdx.x * stride, n);
}

__device__ void givens_body(MinresState* S, const double* __restrict__ a, int64_t nu, const double* __restrict__ b,
                            int64_t nq, int maxit) {
    if (S->stop) {
        if (threadIdx.x == 0) S->skipped = 1;
        return;
    }
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nu; k += blockDim.x) acc += a[k];
    double acc2 = 0.0;
    for (int64_t k = threadIdx.x; k < nq; k += blockDim.x) acc2 += b[k];
    const double s1 = block_sum(acc);
    const double s2 = block_sum(acc2);
    if (threadIdx.x != 0) return;
    const double g2 = s1 + s2;
    S->skipped = 0;
    if (!(g2 >= 0.0) || !isfinite(g2)) {
        S->status = isfinite(g2) ? HD_ERR_BREAKDOWN : HD_ERR_NONFINITE;
        S->stop = 1;
        S->skipped = 1;
        return;
    }
    const double gamma = S->gamma, delta = S->delta;
    const double gnew = sqrt(g2);
    const double a0 = S->c * delta - S->c_old * S->s * gamma;
    const double a1 = sqrt(a0 * a0 + gnew * gnew);
    const double a2 = S->s * delta + S->c_old * S->c * gamma;
    const double a3 = S->s_old * gamma;
    const double cn = a0 / a1, sn = gnew / a1;
    S->a1inv = 1.0 / a1;
    S->a2 = a2;
    S->a3 = a3;
    S->zscale = 1.0 / gamma;
    S->xcoef = cn * S->eta;
    S->eta = -sn * S->eta;
    S->gamma_old = gamma;
    S->gamma = gnew;
    S->inv_gamma = gnew > 0.0 ? 1.0 / gnew : 0.0;
    S->c_old = S->c;
    S->c = cn;
    S->s_old = S->s;
    S->s = sn;
    S->iter += 1;
    if (fabs(S->eta) <= S->tol * S->eta0 || gnew == 0.0) {
        S->stop = 1;
        S->status = 0;
    } else if (S->iter >= maxit) {
        S->stop = 1;
        S->status = HD_NOT_CONVERGED;
    }
}

__global__ void k_givens(MinresState* st, const double* __restrict__ pu, int64_t nu, int64_t su,
                         const double* __restrict__ pq, int64_t nq, int64_t sq, int maxit) {
    givens_body(st + blockIdx.x, pu + blockIdx.x * su, nu, pq + blockIdx.x * sq, nq, maxit);
}

__global__ void k_start(MinresState* st, const double* __restrict__ pu, int64_t nu, int64_t su,
                        const double* __restrict__ pq, int64_t nq, int64_t sq, double tol) {
    const double* a = pu + blockIdx.x * su;
    const double* b = pq + blockIdx.x * sq;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nu; k += blockDim.x) acc += a[k];
    double acc2 = 0.0;
    for (int64_t k = threadIdx.x; k < nq; k += blockDim.x) acc2 += b[k];
    const double s1 = block_sum(acc);
    const double s2 = block_sum(acc2);
    if (threadIdx.x != 0) return;
    const double g2 = s1 + s2;
    MinresState s = {};
    s.tol = tol;
    s.c = s.c_old = 1.0;
    s.s = s.s_old = 0.0;
    s.gamma_old = 1.0;
    if (!(g2 >= 0.0) || !isfinite(g2)) {
        s.status = isfinite(g2) ? HD_ERR_BREAKDOWN : HD_ERR_NONFINITE;
        s.stop = 1;
    } else {
        s.gamma = sqrt(g2);
        s.eta = s.eta0 = s.gamma;
        s.inv_gamma = s.gamma > 0.0 ? 1.0 / s.gamma : 0.0;
        s.stop = s.gamma == 0.0;
    }
    st[blockIdx.x] = s;
}

// the stop tolerance of one recurrence (set after k_start)
__global__ void k_set_tol(MinresState* st, double tol) { st->tol = tol; }

// v_old <- q - cv1 v - cv2 v_old  (= v_{j+1});  z_u = mdinv * v_{j+1,u}
// (blockIdx.y = right-hand side)
template <typename T>
__device__ __forceinline__ void vupd_body(int64_t N, int64_t nu, const T* __restrict__ q, const T* __restrict__ v,
                                          T* __restrict__ vo, const T* __restrict__ mdinv, T* __restrict__ z,
                                          const MinresState& st, double* __restrict__ part, unsigned lb, unsigned nb) {
    if (st.stop) return;
    __shared__ double s[BS];
    const T cv1 = (T)st.cv1, cv2 = (T)st.cv2;
    double contrib = 0.0;
    const int64_t stride = (int64_t)nb * BS;
    int64_t i = lb * (int64_t)blockDim.x + threadIdx.x;
    // four strides at a time, all loads first (more bytes in flight per
    // thread, which the 4-byte FP32 loads need); the same per-thread order of
    // the elements and of the partial sum as one at a time
    constexpr int U = 4;
    for (; i + (U - 1) * stride < N; i += U * stride) {
        T qv[U], vv[U], ov[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = i + u * stride;
            qv[u] = q[k];
            vv[u] = v[k];
            ov[u] = vo[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = i + u * stride;
            const T vn = qv[u] - cv1 * vv[u] - cv2 * ov[u];
            vo[k] = vn;
            if (k < nu) {
                const T zi = mdinv[k] * vn;
                z[k] = zi;
                contrib += (double)zi * (double)vn;
            }
        }
    }
    for (; i < N; i += stride) {
        const T vn = q[i] - cv1 * v[i] - cv2 * vo[i];
        vo[i] = vn;
        if (i < nu) {
            const T zi = mdinv[i] * vn;
            z[i] = zi;
            contrib += (double)zi * (double)vn;
        }
    }
    s[threadIdx.x] = contrib;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[lb] = s[0];
}

// v_old <- q - cv1 v - cv2 v_old  (= v_{j+1});  z_u = mdinv * v_{j+1,u}
// (blockIdx.y = right-hand side)
template <typename T>
__global__ void k_vupd(int64_t N, int64_t nu, const T* __restrict__ q, const T* __restrict__ v, T* __restrict__ vo,
                       const T* __restrict__ mdinv, T* __restrict__ z, const MinresState* __restrict__ st,
                       double* __restrict__ part) {
    const int r = blockIdx.y;
    const int64_t o = (int64_t)r * N;
    vupd_body<T>(N, nu, q + o, v + o, vo + o, mdinv, z + o, st[r], part + (int64_t)r * RED_BLOCKS, blockIdx.x,
                 gridDim.x);
}

// w_old <- (z zscale - a3 w_old - a2 w) a1inv  (= w_{j+1});  x += xcoef w_{j+1}
template <typename T, typename X>
__device__ __forceinline__ void wupd_body(int64_t N, const T* __restrict__ z, T* __restrict__ wo,
                                          const T* __restrict__ w, X* __restrict__ x, const MinresState& st,
                                          unsigned lb) {
    if (st.skipped) return;
    const int64_t k = lb * (int64_t)blockDim.x + threadIdx.x;
    if (k >= N) return;
    const T zs = (T)st.zscale, a3 = (T)st.a3, a2 = (T)st.a2, a1i = (T)st.a1inv;
    const T wn = (z[k] * zs - a3 * wo[k] - a2 * w[k]) * a1i;
    wo[k] = wn;
    x[k] += (X)st.xcoef * (X)wn;
}

// w_old <- (z zscale - a3 w_old - a2 w) a1inv  (= w_{j+1});  x += xcoef w_{j+1}
template <typename T, typename X>
__global__ void k_wupd(int64_t N, const T* __restrict__ z, T* __restrict__ wo, const T* __restrict__ w,
                       X* __restrict__ x, const MinresState* __restrict__ st) {
    const int r = blockIdx.y;
    const int64_t o = (int64_t)r * N;
    wupd_body<T, X>(N, z + o, wo + o, w + o, x + o, st[r], blockIdx.x);
}

// ---- the recurrence kernels of a batch in shared launches ----------------
// One descriptor per instance; the bodies are those of the kernels above, so
// every instance computes what its own launches compute, bit for bit.
struct BVec {
    int64_t o, N, nu;          // offset in the concatenated vectors, length, RT part
    const void* mdinv;         // 1 / (tau diag M) of the working precision
    const double* apart;       // the apply's partial sums of <A v, v>
    int64_t napart;
    const double* pq;          // the V-cycle's partial sums of <z_q, v_q>
    int64_t npq;
    unsigned blk_v, nb_v;      // first block and blocks of the vector update (red_grid(N))
    unsigned blk_w;            // first block of the direction update (nblk(N))
};

__device__ __forceinline__ int bvec_find(const BVec* __restrict__ t, int ni, bool w) {
    __shared__ int fi;
    if (threadIdx.x == 0) {
        int k = 0;
        while (k + 1 < ni && (w ? t[k + 1].blk_w : t[k + 1].blk_v) <= blockIdx.x) ++k;
        fi = k;
    }
    __syncthreads();
    return fi;
}

__global__ void kb_delta(MinresState* st, const BVec* __restrict__ t) {
    const BVec& d = t[blockIdx.x];
    delta_body(st + blockIdx.x, d.apart, d.napart);
}

template <typename T>
__global__ void kb_vupd(const BVec* __restrict__ t, int ni, const T* __restrict__ q, const T* __restrict__ v,
                        T* __restrict__ vo, T* __restrict__ z, const MinresState* __restrict__ st,
                        double* __restrict__ pu) {
    const int i = bvec_find(t, ni, false);
    const BVec d = t[i];
    vupd_body<T>(d.N, d.nu, q + d.o, v + d.o, vo + d.o, (const T*)d.mdinv, z + d.o, st[i],
                 pu + (int64_t)i * RED_BLOCKS, blockIdx.x - d.blk_v, d.nb_v);
}

__global__ void kb_givens(MinresState* st, const double* __restrict__ pu, const BVec* __restrict__ t, int maxit) {
    const BVec& d = t[blockIdx.x];
    givens_body(st + blockIdx.x, pu + (int64_t)blockIdx.x * RED_BLOCKS, d.nb_v, d.pq, d.npq, maxit);
}

template <typename T>
__global__ void kb_wupd(const BVec* __restrict__ t, int ni, const T* __restrict__ z, T* __restrict__ wo,
                        const T* __restrict__ w, T* __restrict__ x, const MinresState* __restrict__ st) {
    const int i = bvec_find(t, ni, true);
    const BVec d = t[i];
    wupd_body<T, T>(d.N, z + d.o, wo + d.o, w + d.o, x + d.o, st[i], blockIdx.x - d.blk_w);
}

// v = b - q (or b when q == nullptr), v_old = w = w_old = 0 (all RHS)
template <typename T, typename B>
__global__ void k_init(int64_t n, const B* __restrict__ b, const T* __restrict__ q, T* __restrict__ v,
                       T* __restrict__ vo, T* __restrict__ w, T* __restrict__ wo) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    v[i] = q ? (T)((T)b[i] - q[i]) : (T)b[i];
    vo[i] = 0;
    w[i] = 0;
    wo[i] = 0;
}

template <typename T>
__global__ void k_zero(int64_t n, T* __restrict__ x) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

// swap the contents of two buffers (realigns a recurrence whose executed
// iteration count has the other parity than the host's buffer rotation)
template <typename T>
__global__ void k_swap(int64_t N, T* __restrict__ a, T* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T t = a[i];
    a[i] = b[i];
    b[i] = t;
}

// r = b - q (FP64), per-RHS partial sums of r^2 and b^2 (blockIdx.y = RHS)
__global__ void k_residual(int64_t N, const double* __restrict__ b, const double* __restrict__ q,
                           double* __restrict__ r, double* __restrict__ pr, double* __restrict__ pb) {
    __shared__ double s[BS];
    const int64_t o = (int64_t)blockIdx.y * N;
    double rr = 0.0, bb = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
        const double ri = b[o + i] - q[o + i];
        if (r) r[o + i] = ri;
        rr += ri * ri;
        bb += b[o + i] * b[o + i];
    }
    s[threadIdx.x] = rr;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) pr[(int64_t)blockIdx.y * RED_BLOCKS + blockIdx.x] = s[0];
    __syncthreads();
    s[threadIdx.x] = bb;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) pb[(int64_t)blockIdx.y * RED_BLOCKS + blockIdx.x] = s[0];
}

// out[2r] = ||r||, out[2r+1] = ||b|| (one block per RHS)
__global__ void k_norms(const double* __restrict__ pr, const double* __restrict__ pb, int64_t n,
                        double* __restrict__ out) {
    const double* a = pr + (int64_t)blockIdx.x * RED_BLOCKS;
    const double* b = pb + (int64_t)blockIdx.x * RED_BLOCKS;
    double x = 0.0, y = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
        x += a[k];
        y += b[k];
    }
    const double sx = block_sum(x);
    const double sy = block_sum(y);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = sqrt(sx);
        out[2 * blockIdx.x + 1] = sqrt(sy);
    }
}

// r32 = r / ||r|| (FP64 -> FP32), and x += ||r|| d32 (blockIdx.y = RHS; the
// norm of RHS r is nrm[2r]; a zero norm gives a zero right-hand side)
__global__ void k_to32(int64_t N, const double* __restrict__ r, const double* __restrict__ nrm,
                       float* __restrict__ o) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double s = nrm[2 * blockIdx.y];
    const int64_t k = (int64_t)blockIdx.y * N + i;
    o[k] = s > 0.0 ? (float)(r[k] / s) : 0.0f;
}
__global__ void k_addscaled(int64_t N, const float* __restrict__ d, const double* __restrict__ nrm,
                            double* __restrict__ x) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t k = (int64_t)blockIdx.y * N + i;
    x[k] += nrm[2 * blockIdx.y] * (double)d[k];
}

// FP32 Schur block inside an FP64 recurrence: v_q rounded to FP32 for the
// V-cycle; the FP32 z_q widened back to FP64 with the partial sums of
// <z_q, v_q> taken against the FP64 v_q the recurrence holds.
__global__ void k_down(int64_t n, const double* __restrict__ v, float* __restrict__ o, const int* done) {
    if (done && *done) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) o[i] = (float)v[i];
}
__global__ void k_up_dot(int64_t n, const float* __restrict__ z32, const double* __restrict__ v,
                         double* __restrict__ z, double* __restrict__ part, const int* done) {
    if (done && *done) return;
    __shared__ double s[BS];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const double zi = (double)z32[i];
        z[i] = zi;
        acc += zi * v[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// tighten the stop threshold of one RHS and resume its converged recurrence
__global__ void k_retarget(MinresState* st, double tol) {
    if (st->status == 0) {
        st->tol = tol;
        st->stop = 0;
    }
}

struct Work {
    int64_t N = 0;
    int nrhs = 1;
    int prec = HD_F64;
    void *v = nullptr, *vo = nullptr, *z = nullptr, *zn = nullptr, *w = nullptr, *wo = nullptr, *q = nullptr;
    double *pd = nullptr, *pu = nullptr, *pq = nullptr, *nrm = nullptr;
    int64_t nd_part = 0, nq_part = 0;
    double* pd2 = nullptr;       // first-stage sums of pd when it is long
    int64_t nd_blocks = 0;       // number of first-stage blocks (0: single stage)
    MinresState* st = nullptr;
    MinresState* st_host = nullptr;
    double* nrm_host = nullptr;
    // FP32 Schur block of an FP64 recurrence: v_q and z_q in FP32, partials
    float *t32 = nullptr, *z32 = nullptr;
    double* p32 = nullptr;
};

void free_work(Work& w) {
    for (void* p : {w.v, w.vo, w.z, w.zn, w.w, w.wo, w.q}) dfree(p);
    dfree(w.pd);
    dfree(w.pd2);
    dfree(w.pu);
    dfree(w.pq);
    dfree(w.nrm);
    dfree(w.st);
    dfree(w.t32);
    dfree(w.z32);
    dfree(w.p32);
    if (w.st_host) (void)hipHostFree(w.st_host);
    if (w.nrm_host) (void)hipHostFree(w.nrm_host);
    w = Work();
}

int alloc_work(hd_ctx* c, Work& w, int prec, int nrhs, bool schur32 = false) {
    w.N = c->n_u + c->n_q;
    w.nrhs = nrhs;
    w.prec = prec;
    const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
    void** vs[] = {&w.v, &w.vo, &w.z, &w.zn, &w.w, &w.wo, &w.q};
    for (void** p : vs) {
        if (hipMalloc(p, es * w.N * nrhs) != hipSuccess) return set_err(c, HD_ERR_OOM, "MINRES vectors");
    }
    w.nd_part = apply_partial_count(c);
    w.nq_part = std::max<int64_t>(schur_partial_count(c), RED_BLOCKS);
    w.pd = dalloc<double>(w.nd_part * nrhs);
    // one workgroup reduces up to a few thousand partials quickly; longer
    // arrays (fine meshes of low degree) get a first stage of 2048 per block
    constexpr int64_t STAGE = 2048;
    w.nd_blocks = w.nd_part > 4 * STAGE ? std::min<int64_t>((w.nd_part + STAGE - 1) / STAGE, 1024) : 0;
    if (w.nd_blocks) {
        w.pd2 = dalloc<double>(w.nd_blocks * nrhs);
        if (!w.pd2) return set_err(c, HD_ERR_OOM, "MINRES partials");
    }
    w.pu = dalloc<double>((int64_t)RED_BLOCKS * nrhs);
    w.pq = dalloc<double>(w.nq_part * nrhs);
    w.nrm = dalloc<double>(2 * nrhs);
    w.st = dalloc<MinresState>(nrhs);
    if (!w.pd || !w.pu || !w.pq || !w.st || !w.nrm) return set_err(c, HD_ERR_OOM, "MINRES partials");
    if (hipHostMalloc((void**)&w.st_host, sizeof(MinresState) * nrhs) != hipSuccess ||
        hipHostMalloc((void**)&w.nrm_host, sizeof(double) * 2 * nrhs) != hipSuccess)
        return set_err(c, HD_ERR_OOM, "MINRES host state");
    if (schur32) {
        w.t32 = dalloc<float>(c->n_q);
        w.z32 = dalloc<float>(c->n_q);
        w.p32 = dalloc<double>(w.nq_part);
        if (!w.t32 || !w.z32 || !w.p32) return set_err(c, HD_ERR_OOM, "FP32 Schur buffers");
    }
    return HD_OK;
}

// z_q = S^{-1} v_q with the V-cycle in precision PT, partial sums of
// <z_q, v_q> into part (schur_parts(c) of them)
template <typename T, typename PT>
int schur_step(hd_ctx* c, Work& wk, const T* vq, T* zq, double* part, const int* done) {
    if constexpr (std::is_same<T, PT>::value) {
        return launch_schur_prec(c, std::is_same<T, double>::value ? HD_F64 : HD_F32, vq, zq, part, done);
    } else {
        static_assert(std::is_same<T, double>::value && std::is_same<PT, float>::value, "FP32 V-cycle in FP64");
        const int64_t nq = c->n_q;
        hipLaunchKernelGGL(k_down, dim3(nblk(nq)), dim3(BS), 0, c->stream, nq, vq, wk.t32, done);
        int rc = launch_schur_prec(c, HD_F32, wk.t32, wk.z32, wk.p32, done);
        if (rc) return rc;
        hipLaunchKernelGGL(k_up_dot, dim3(red_grid(nq)), dim3(BS), 0, c->stream, nq, wk.z32, vq, zq, part, done);
        return HD_OK;
    }
}

template <typename T, typename PT>
int64_t schur_parts(const hd_ctx* c) {
    return std::is_same<T, PT>::value ? schur_partial_count(c) : (int64_t)red_grid(c->n_q);
}

// ||b_r - A x_r|| and ||b_r|| for every RHS into wk.nrm_host (and the device
// copy wk.nrm); r (optional) receives b - A x.
int true_residual(hd_ctx* c, Work& wk64, const double* b, const double* x, double* r) {
    const int64_t N = wk64.N;
    const int nr = wk64.nrhs;
    int rc;
    if ((rc = launch_apply(c, HD_F64, nr, x, wk64.q, nullptr, 0, nullptr, 0, ESS_IDENTITY, nullptr, 0))) return rc;
    hipLaunchKernelGGL(k_residual, dim3(red_grid(N), nr), dim3(BS), 0, c->stream, N, b, (const double*)wk64.q, r,
                       wk64.pu, wk64.pq);
    hipLaunchKernelGGL(k_norms, dim3(nr), dim3(1024), 0, c->stream, wk64.pu, wk64.pq, (int64_t)red_grid(N), wk64.nrm);
    HD_HIP(c, hipMemcpyAsync(wk64.nrm_host, wk64.nrm, 2 * nr * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

inline double rel_of(const double* nrm, int r) {
    return nrm[2 * r + 1] > 0 ? nrm[2 * r] / nrm[2 * r + 1] : nrm[2 * r];
}

// Preconditioned MINRES in precision T on A x_r = b_r for wk.nrhs right-hand
// sides (b of precision B, x of precision T, x0 = 0 unless use_x0).
// true_tol > 0 (FP64 only): after the |eta| stop, require the true FP64
// residual and continue the recurrence with a tighter threshold if needed.
// One poll period of iterations as a replayable HIP graph: the vector
// buffers rotate with period 2 and the period is even, so every replay sees
// the same pointers; the recurrence state, the stop flags and the scales live
// in device memory.  The capture is always ended, also on an error, so the
// caller's stream never stays in capture mode.
struct PeriodGraph {
    hipGraphExec_t exec = nullptr;
    ~PeriodGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

template <typename T, typename B, typename PT = T>
int minres_core(hd_ctx* c, Work& wk, const B* b, T* x, bool use_x0, double tol, int maxit, int check_every,
                std::vector<hd_solve_info>& out, double true_tol = 0.0, bool use_graph = false,
                const double* tols = nullptr) {
    const int prec = std::is_same<T, double>::value ? HD_F64 : HD_F32;
    const int64_t N = wk.N, nu = c->n_u;
    const int nr = wk.nrhs;
    T* v = (T*)wk.v;
    T* vo = (T*)wk.vo;
    T* z = (T*)wk.z;
    T* zn = (T*)wk.zn;
    T* w = (T*)wk.w;
    T* wo = (T*)wk.wo;
    T* q = (T*)wk.q;
    const T* mdinv = std::is_same<T, double>::value ? (const T*)c->d_mdinv : (const T*)c->d_mdinv32;
    const int64_t nqp = schur_parts<T, PT>(c);
    int rc;
    const int64_t Nt = N * nr;
    if (use_x0) {
        if ((rc = launch_apply(c, prec, nr, x, q, nullptr, 0, nullptr, 0, ESS_IDENTITY, nullptr, 0))) return rc;
        hipLaunchKernelGGL((k_init<T, B>), dim3(nblk(Nt)), dim3(BS), 0, c->stream, Nt, b, (const T*)q, v, vo, w, wo);
    } else {
        hipLaunchKernelGGL(k_zero<T>, dim3(nblk(Nt)), dim3(BS), 0, c->stream, Nt, x);
        hipLaunchKernelGGL((k_init<T, B>), dim3(nblk(Nt)), dim3(BS), 0, c->stream, Nt, b, (const T*)nullptr, v, vo,
                           w, wo);
    }
    // z_1 = B^{-1} v_1
    for (int r = 0; r < nr; ++r) {
        if ((rc = launch_diag_prec(c, prec, v + r * N, z + r * N, wk.pu + (int64_t)r * RED_BLOCKS))) return rc;
        if ((rc = schur_step<T, PT>(c, wk, v + r * N + nu, z + r * N + nu, wk.pq + r * wk.nq_part, nullptr)))
            return rc;
    }
    hipLaunchKernelGGL(k_start, dim3(nr), dim3(1024), 0, c->stream, wk.st, wk.pu, (int64_t)red_grid(nu),
                       (int64_t)RED_BLOCKS, wk.pq, nqp, wk.nq_part, tol);
    // per right-hand side tolerances (the refinement's inner solves)
    if (tols)
        for (int r = 0; r < nr; ++r) hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(1), 0, c->stream, wk.st + r, tols[r]);
    HD_HIP(c, hipGetLastError());
    const int* stop = &wk.st->stop;
    int launched = 0, retargets = 0;
    // one MINRES iteration for every right-hand side (kernels only)
    auto iteration = [&]() -> int {
        int rc2;
        {
            if ((rc2 = launch_apply(c, prec, nr, z, q, &wk.st->inv_gamma, ST_STRIDE_D, wk.pd, wk.nd_part,
                                    ESS_IDENTITY, stop, ST_STRIDE_I)))
                return rc2;
            if (wk.nd_blocks) {
                const int64_t chunk = (wk.nd_part + wk.nd_blocks - 1) / wk.nd_blocks;
                hipLaunchKernelGGL(k_sum_stage, dim3((unsigned)wk.nd_blocks, nr), dim3(256), 0, c->stream, wk.pd,
                                   wk.nd_part, wk.nd_part, chunk, wk.pd2, (const MinresState*)wk.st);
                hipLaunchKernelGGL(k_delta, dim3(nr), dim3(1024), 0, c->stream, wk.st, wk.pd2, wk.nd_blocks,
                                   wk.nd_blocks);
            } else {
                hipLaunchKernelGGL(k_delta, dim3(nr), dim3(1024), 0, c->stream, wk.st, wk.pd, wk.nd_part,
                                   wk.nd_part);
            }
            hipLaunchKernelGGL(k_vupd<T>, dim3(red_grid(N), nr), dim3(BS), 0, c->stream, N, nu, q, v, vo, mdinv, zn,
                               wk.st, wk.pu);
            for (int r = 0; r < nr; ++r)
                if ((rc2 = schur_step<T, PT>(c, wk, vo + r * N + nu, zn + r * N + nu, wk.pq + r * wk.nq_part,
                                             stop + r * ST_STRIDE_I)))
                    return rc2;
            hipLaunchKernelGGL(k_givens, dim3(nr), dim3(1024), 0, c->stream, wk.st, wk.pu, (int64_t)red_grid(N),
                               (int64_t)RED_BLOCKS, wk.pq, nqp, wk.nq_part, maxit);
            hipLaunchKernelGGL((k_wupd<T, T>), dim3(nblk(N), nr), dim3(BS), 0, c->stream, N, z, wo, w, x, wk.st);
            std::swap(v, vo);
            std::swap(z, zn);
            std::swap(w, wo);
        }
        return HD_OK;
    };
    PeriodGraph graph;
    // (per-apply event timing synchronises inside the apply: no capture then)
    const bool graphs = use_graph && check_every % 2 == 0 && !c->time_apply;
    for (;;) {
        if (graphs && maxit - launched >= check_every) {
            if (!graph.exec) {
                // the caller's stream may be the legacy default stream, which
                // cannot be captured: record on a private stream of the same
                // (default) priority, replay on the caller's
                if (!c->cap_stream) HD_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                HD_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                hipStream_t user = c->stream;
                c->stream = c->cap_stream;
                int crc = HD_OK;
                for (int k = 0; k < check_every && !crc; ++k) crc = iteration();
                c->stream = user;
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
                if (!crc && e != hipSuccess) crc = set_err(c, HD_ERR_HIP, "MINRES graph capture");
                if (!crc && hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0) != hipSuccess)
                    crc = set_err(c, HD_ERR_HIP, "MINRES graph instantiation");
                if (g) (void)hipGraphDestroy(g);
                if (crc) return crc;
            }
            HD_HIP(c, hipGraphLaunch(graph.exec, c->stream));
            launched += check_every;
        } else {
            for (int k = 0; k < check_every && launched < maxit; ++k, ++launched)
                if ((rc = iteration())) return rc;
        }
        HD_HIP(c, hipGetLastError());
        HD_HIP(c, hipMemcpyAsync(wk.st_host, wk.st, nr * sizeof(MinresState), hipMemcpyDeviceToHost, c->stream));
        HD_HIP(c, hipStreamSynchronize(c->stream));
        bool all_stop = true;
        for (int r = 0; r < nr; ++r) all_stop = all_stop && wk.st_host[r].stop;
        if (all_stop && true_tol > 0.0 && retargets < 8) {
            // the recurrence stops on the preconditioned residual norm; when the
            // caller asks for a true FP64 residual, check it and continue the
            // recurrences that have not met it with a tighter threshold
            if constexpr (std::is_same<T, double>::value && std::is_same<B, double>::value) {
                if ((rc = true_residual(c, wk, b, x, nullptr))) return rc;
                // iterations launched after a stop were no-ops for that RHS while
                // the host kept rotating the buffers: realign each RHS to the
                // parity of the launched count before resuming it
                bool resumed = false;
                for (int r = 0; r < nr; ++r) {
                    const MinresState& s = wk.st_host[r];
                    const double rel = rel_of(wk.nrm_host, r);
                    if (s.status != 0 || rel <= true_tol) continue;
                    if ((s.iter % 2) != (launched % 2)) {
                        T* pairs[3][2] = {{v, vo}, {z, zn}, {w, wo}};
                        for (auto& pr : pairs)
                            hipLaunchKernelGGL(k_swap<T>, dim3(nblk(N)), dim3(BS), 0, c->stream, N, pr[0] + r * N,
                                               pr[1] + r * N);
                    }
                    const double nt = s.tol * (true_tol / rel) * 0.7;
                    hipLaunchKernelGGL(k_retarget, dim3(1), dim3(1), 0, c->stream, wk.st + r, nt);
                    resumed = true;
                }
                if (resumed) {
                    ++retargets;
                    if (launched < maxit) continue;
                }
            }
        }
        if (all_stop || launched >= maxit) break;
    }
    out.resize(nr);
    for (int r = 0; r < nr; ++r) {
        const MinresState& s = wk.st_host[r];
        out[r] = hd_solve_info();
        out[r].iterations = s.iter;
        out[r].status = s.stop ? s.status : HD_NOT_CONVERGED;
        out[r].eta_rel = s.eta0 > 0 ? std::fabs(s.eta) / s.eta0 : 0.0;
        out[r].outer = 1;
    }
    return HD_OK;
}

// ---- batches of independent instances ------------------------------------
// One MINRES recurrence per instance on the concatenated vectors: the block
// apply of all instances is one batched (persistent) launch per colour with
// per-instance scales, stop flags and partial sums; the vector updates, the
// reductions and the preconditioner (each instance's own diagonal and
// V-cycle, i.e. the AMG of the block-diagonal union) run per instance.
struct BatchWork {
    int64_t total = 0;
    // the recurrence vectors, of the solve's working precision
    void *v = nullptr, *vo = nullptr, *z = nullptr, *zn = nullptr, *w = nullptr, *wo = nullptr, *q = nullptr;
    double *pu = nullptr, *pr = nullptr, *pq = nullptr, *nrm = nullptr;
    std::vector<int64_t> pq_off, nq_part;
    MinresState* st = nullptr;
    MinresState* st_host = nullptr;
    double* nrm_host = nullptr;
    Work schur32;   // FP32 Schur buffers (sized for the largest instance)
    // FP32 V-cycle input and output of every instance (the shared V-cycle
    // launches with an FP64 recurrence), at q32_off
    float *t32all = nullptr, *z32all = nullptr;
    std::vector<int64_t> q32_off;
    BVec* bvec = nullptr;      // the shared recurrence kernels' descriptors
    int bvec_n = 0;
    ~BatchWork() {
        dfree(t32all);
        dfree(z32all);
        dfree(bvec);
        for (void* p : {v, vo, z, zn, w, wo, q}) dfree(p);
        for (double* p : {pu, pr, pq, nrm}) dfree(p);
        dfree(st);
        if (st_host) (void)hipHostFree(st_host);
        if (nrm_host) (void)hipHostFree(nrm_host);
        dfree(schur32.t32);
        dfree(schur32.z32);
        dfree(schur32.p32);
    }
};

// ||b_i - A_i x_i|| and ||b_i|| of every instance into W.nrm_host (and the
// device copy W.nrm); r (optional) receives b - A x.  W holds FP64 vectors.
int batch_true_residual(hd_ctx* c, BatchWork& W, const double* b, const double* x, double* r = nullptr) {
    const BatchState& B = *c->batch;
    const int ni = (int)B.inst.size();
    const double* q = (const double*)W.q;
    int rc;
    if ((rc = launch_batch_apply(c, HD_F64, x, W.q, nullptr, 0, nullptr, 0, false))) return rc;
    for (int i = 0; i < ni; ++i) {
        const int64_t o = B.off[i], N = B.off[i + 1] - B.off[i];
        hipLaunchKernelGGL(k_residual, dim3(red_grid(N), 1), dim3(BS), 0, c->stream, N, b + o, q + o,
                           r ? r + o : (double*)nullptr, W.pu + (int64_t)i * RED_BLOCKS,
                           W.pr + (int64_t)i * RED_BLOCKS);
        hipLaunchKernelGGL(k_norms, dim3(1), dim3(1024), 0, c->stream, W.pu + (int64_t)i * RED_BLOCKS,
                           W.pr + (int64_t)i * RED_BLOCKS, (int64_t)red_grid(N), W.nrm + 2 * i);
    }
    HD_HIP(c, hipMemcpyAsync(W.nrm_host, W.nrm, 2 * ni * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

// One MINRES recurrence per instance in precision T (vectors and operator;
// the recurrence scalars and reductions are FP64), b of precision Bv, x of
// precision T, Schur block in precision PT.  true_tol > 0 (FP64 only): after
// the |eta| stop, require the true FP64 residual as in the single solve.
template <typename T, typename Bv, typename PT>
int batch_minres_core(hd_ctx* c, BatchWork& W, const Bv* b, T* x, bool use_x0, double tol, int maxit,
                      int check_every, double true_tol, std::vector<hd_solve_info>& out, bool use_graph,
                      const double* tols = nullptr) {
    constexpr bool F64 = std::is_same<T, double>::value;
    const int prec = F64 ? HD_F64 : HD_F32;
    const BatchState& B = *c->batch;
    const int ni = (int)B.inst.size();
    const int64_t tot = B.total;
    T *v = (T*)W.v, *vo = (T*)W.vo, *z = (T*)W.z, *zn = (T*)W.zn, *w = (T*)W.w, *wo = (T*)W.wo, *q = (T*)W.q;
    int rc;
    if (use_x0) {
        if ((rc = launch_batch_apply(c, prec, x, q, nullptr, 0, nullptr, 0, false))) return rc;
        hipLaunchKernelGGL((k_init<T, Bv>), dim3(nblk(tot)), dim3(BS), 0, c->stream, tot, b, (const T*)q, v, vo, w,
                           wo);
    } else {
        hipLaunchKernelGGL(k_zero<T>, dim3(nblk(tot)), dim3(BS), 0, c->stream, tot, x);
        hipLaunchKernelGGL((k_init<T, Bv>), dim3(nblk(tot)), dim3(BS), 0, c->stream, tot, b, (const T*)nullptr, v,
                           vo, w, wo);
    }
    for (int i = 0; i < ni; ++i) {
        hd_ctx* s = B.inst[i];
        const int64_t o = B.off[i];
        if ((rc = launch_diag_prec(s, prec, v + o, z + o, W.pu + (int64_t)i * RED_BLOCKS))) return rc;
        if ((rc = schur_step<T, PT>(s, W.schur32, v + o + s->n_u, z + o + s->n_u, W.pq + W.pq_off[i], nullptr)))
            return rc;
        hipLaunchKernelGGL(k_start, dim3(1), dim3(1024), 0, c->stream, W.st + i, W.pu + (int64_t)i * RED_BLOCKS,
                           (int64_t)red_grid(s->n_u), (int64_t)RED_BLOCKS, W.pq + W.pq_off[i],
                           schur_parts<T, PT>(s), W.nq_part[i], tols ? tols[i] : tol);
    }
    HD_HIP(c, hipGetLastError());
    // the recurrence kernels of all instances in shared launches
    const bool vshared = B.vcycle_shared != 0;
    BVec* d_bvec = nullptr;
    unsigned nbv = 0, nbw = 0;
    if (vshared) {
        std::vector<BVec> tb(ni);
        for (int i = 0; i < ni; ++i) {
            hd_ctx* s = B.inst[i];
            BVec& d = tb[i];
            d.o = B.off[i];
            d.N = s->n_u + s->n_q;
            d.nu = s->n_u;
            d.mdinv = F64 ? (const void*)s->d_mdinv : (const void*)s->d_mdinv32;
            d.apart = c->batch->d_part + c->batch->part_off[i];
            d.napart = apply_partial_count(s);
            d.pq = W.pq + W.pq_off[i];
            d.npq = schur_parts<T, PT>(s);
            d.blk_v = nbv;
            d.nb_v = red_grid(d.N);
            d.blk_w = nbw;
            nbv += d.nb_v;
            nbw += nblk(d.N);
        }
        if (!W.bvec || W.bvec_n < ni) {
            dfree(W.bvec);
            W.bvec = dalloc<BVec>(ni);
            W.bvec_n = W.bvec ? ni : 0;
            if (!W.bvec) return set_err(c, HD_ERR_OOM, "batched MINRES tables");
        }
        d_bvec = W.bvec;
        HD_HIP(c, hipMemcpyAsync(d_bvec, tb.data(), sizeof(BVec) * ni, hipMemcpyHostToDevice, c->stream));
    }
    int launched = 0, retargets = 0;
    // one MINRES iteration for every instance (kernels only; those of a
    // stopped instance return at once on its stop flag)
    auto iteration = [&]() -> int {
        int rc2;
        if ((rc2 = launch_batch_apply(c, prec, z, q, &W.st->inv_gamma, ST_STRIDE_D, &W.st->stop, ST_STRIDE_I, true)))
            return rc2;
        // levels >= 1 of every instance's V-cycle in shared launches (same
        // results as the instances' own cycles); otherwise one cycle each
        const bool shared = B.union_ok && B.vcycle_shared && (std::is_same<T, PT>::value || W.t32all);
        if (vshared) {
            hipLaunchKernelGGL(kb_delta, dim3(ni), dim3(1024), 0, c->stream, W.st, (const BVec*)d_bvec);
            hipLaunchKernelGGL(kb_vupd<T>, dim3(nbv), dim3(BS), 0, c->stream, (const BVec*)d_bvec, ni, (const T*)q,
                               (const T*)v, vo, zn, (const MinresState*)W.st, W.pu);
        }
        for (int i = 0; i < ni; ++i) {
            hd_ctx* s = B.inst[i];
            const int64_t o = B.off[i], N = s->n_u + s->n_q, np = apply_partial_count(s);
            const int* stop_i = &W.st[i].stop;
            const T* mdinv = F64 ? (const T*)s->d_mdinv : (const T*)s->d_mdinv32;
            if (!vshared) {
                hipLaunchKernelGGL(k_delta, dim3(1), dim3(1024), 0, c->stream, W.st + i,
                                   (const double*)(c->batch->d_part + c->batch->part_off[i]), np, np);
                hipLaunchKernelGGL(k_vupd<T>, dim3(red_grid(N), 1), dim3(BS), 0, c->stream, N, s->n_u,
                                   (const T*)q + o, (const T*)v + o, vo + o, mdinv, zn + o,
                                   (const MinresState*)(W.st + i), W.pu + (int64_t)i * RED_BLOCKS);
            }
            if (!shared || !B.in_union[i]) {
                if ((rc2 = schur_step<T, PT>(s, W.schur32, vo + o + s->n_u, zn + o + s->n_u, W.pq + W.pq_off[i],
                                             stop_i)))
                    return rc2;
            } else if constexpr (!std::is_same<T, PT>::value) {
                // the FP32 cycle's input (as schur_step does, per instance)
                hipLaunchKernelGGL(k_down, dim3(nblk(s->n_q)), dim3(BS), 0, c->stream, s->n_q,
                                   (const double*)(vo + o + s->n_u), W.t32all + W.q32_off[i], stop_i);
            }
        }
        if (shared) {
            if constexpr (std::is_same<T, PT>::value) {
                std::vector<const T*> vq(ni);
                std::vector<T*> zq(ni);
                std::vector<double*> pp(ni);
                for (int i = 0; i < ni; ++i) {
                    const int64_t o = B.off[i] + B.inst[i]->n_u;
                    vq[i] = vo + o;
                    zq[i] = zn + o;
                    pp[i] = W.pq + W.pq_off[i];
                }
                if ((rc2 = batch_union_cycle<T>(c, vq.data(), zq.data(), pp.data(), &W.st->stop, ST_STRIDE_I)))
                    return rc2;
            } else {
                std::vector<const float*> vq(ni);
                std::vector<float*> zq(ni);
                std::vector<double*> pp(ni, nullptr);
                for (int i = 0; i < ni; ++i) {
                    vq[i] = W.t32all + W.q32_off[i];
                    zq[i] = W.z32all + W.q32_off[i];
                }
                if ((rc2 = batch_union_cycle<float>(c, vq.data(), zq.data(), pp.data(), &W.st->stop, ST_STRIDE_I)))
                    return rc2;
                // back to FP64 with the partial sums of <z_q, v_q> (as schur_step)
                for (int i = 0; i < ni; ++i) {
                    if (!B.in_union[i]) continue;
                    hd_ctx* s = B.inst[i];
                    const int64_t o = B.off[i] + s->n_u;
                    hipLaunchKernelGGL(k_up_dot, dim3(red_grid(s->n_q)), dim3(BS), 0, c->stream, s->n_q,
                                       (const float*)(W.z32all + W.q32_off[i]), (const double*)(vo + o),
                                       (double*)(zn + o), W.pq + W.pq_off[i], &W.st[i].stop);
                }
            }
        }
        if (vshared) {
            hipLaunchKernelGGL(kb_givens, dim3(ni), dim3(1024), 0, c->stream, W.st, (const double*)W.pu,
                               (const BVec*)d_bvec, maxit);
            hipLaunchKernelGGL(kb_wupd<T>, dim3(nbw), dim3(BS), 0, c->stream, (const BVec*)d_bvec, ni, (const T*)z,
                               wo, (const T*)w, x, (const MinresState*)W.st);
        } else {
            for (int i = 0; i < ni; ++i) {
                hd_ctx* s = B.inst[i];
                const int64_t o = B.off[i], N = s->n_u + s->n_q;
                hipLaunchKernelGGL(k_givens, dim3(1), dim3(1024), 0, c->stream, W.st + i,
                                   (const double*)(W.pu + (int64_t)i * RED_BLOCKS), (int64_t)red_grid(N),
                                   (int64_t)RED_BLOCKS, (const double*)(W.pq + W.pq_off[i]),
                                   schur_parts<T, PT>(s), W.nq_part[i], maxit);
                hipLaunchKernelGGL((k_wupd<T, T>), dim3(nblk(N), 1), dim3(BS), 0, c->stream, N, (const T*)z + o,
                                   wo + o, (const T*)w + o, x + o, (const MinresState*)(W.st + i));
            }
        }
        std::swap(v, vo);
        std::swap(z, zn);
        std::swap(w, wo);
        return HD_OK;
    };
    PeriodGraph graph;
    const bool graphs = use_graph && check_every % 2 == 0 && !c->time_apply;
    for (;;) {
        if (graphs && maxit - launched >= check_every) {
            if (!graph.exec) {
                // record on a private stream of the default priority (the
                // caller's may be the legacy default stream), with every
                // instance context pointed at it, then replay on the caller's
                if (!c->cap_stream) HD_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                HD_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                const hipStream_t user = c->stream;
                c->stream = c->cap_stream;
                for (hd_ctx* s : B.inst) s->stream = c->cap_stream;
                int crc = HD_OK;
                for (int k = 0; k < check_every && !crc; ++k) crc = iteration();
                c->stream = user;
                for (hd_ctx* s : B.inst) s->stream = user;
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
                if (!crc && e != hipSuccess) crc = set_err(c, HD_ERR_HIP, "batched MINRES graph capture");
                if (!crc && hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0) != hipSuccess)
                    crc = set_err(c, HD_ERR_HIP, "batched MINRES graph instantiation");
                if (g) (void)hipGraphDestroy(g);
                if (crc) return crc;
            }
            HD_HIP(c, hipGraphLaunch(graph.exec, c->stream));
            launched += check_every;
        } else {
            for (int k = 0; k < check_every && launched < maxit; ++k, ++launched)
                if ((rc = iteration())) return rc;
        }
        HD_HIP(c, hipGetLastError());
        HD_HIP(c, hipMemcpyAsync(W.st_host, W.st, ni * sizeof(MinresState), hipMemcpyDeviceToHost, c->stream));
        HD_HIP(c, hipStreamSynchronize(c->stream));
        bool all_stop = true;
        for (int i = 0; i < ni; ++i) all_stop = all_stop && W.st_host[i].stop;
        if constexpr (F64 && std::is_same<Bv, double>::value) {
            if (all_stop && true_tol > 0.0 && retargets < 8) {
                if ((rc = batch_true_residual(c, W, b, x))) return rc;
                bool resumed = false;
                for (int i = 0; i < ni; ++i) {
                    const MinresState& st = W.st_host[i];
                    const double rel = rel_of(W.nrm_host, i);
                    if (st.status != 0 || rel <= true_tol) continue;
                    hd_ctx* s = B.inst[i];
                    const int64_t o = B.off[i], N = s->n_u + s->n_q;
                    if ((st.iter % 2) != (launched % 2)) {
                        T* pairs[3][2] = {{v, vo}, {z, zn}, {w, wo}};
                        for (auto& pr : pairs)
                            hipLaunchKernelGGL(k_swap<T>, dim3(nblk(N)), dim3(BS), 0, c->stream, N, pr[0] + o,
                                               pr[1] + o);
                    }
                    hipLaunchKernelGGL(k_retarget, dim3(1), dim3(1), 0, c->stream, W.st + i,
                                       st.tol * (true_tol / rel) * 0.7);
                    resumed = true;
                }
                if (resumed) {
                    ++retargets;
                    if (launched < maxit) continue;
                }
            }
        }
        if (all_stop || launched >= maxit) break;
    }
    out.resize(ni);
    for (int i = 0; i < ni; ++i) {
        const MinresState& st = W.st_host[i];
        out[i] = hd_solve_info();
        out[i].iterations = st.iter;
        out[i].status = st.stop ? st.status : HD_NOT_CONVERGED;
        out[i].eta_rel = st.eta0 > 0 ? std::fabs(st.eta) / st.eta0 : 0.0;
        out[i].outer = 1;
    }
    return HD_OK;
}

}  // namespace

namespace {

// Work space of the solves, kept in the context between calls (vectors,
// partial sums, pinned state) and rebuilt when the sizes change.
struct SolveCache {
    Work w64, w32;
    double* r = nullptr;
    float *r32 = nullptr, *d32 = nullptr;
    int64_t nr = 0;
};

void free_cache(void* p) {
    SolveCache* s = (SolveCache*)p;
    free_work(s->w64);
    free_work(s->w32);
    dfree(s->r);
    dfree(s->r32);
    dfree(s->d32);
    delete s;
}

SolveCache* cache_of(hd_ctx* c) {
    if (!c->solve_cache) {
        c->solve_cache = new SolveCache;
        c->solve_cache_free = free_cache;
    }
    return (SolveCache*)c->solve_cache;
}

bool work_fits(const hd_ctx* c, const Work& w, int prec, int nrhs, bool schur32) {
    return w.st && w.prec == prec && w.nrhs == nrhs && w.N == c->n_u + c->n_q && w.nd_part == apply_partial_count(c) &&
           w.nq_part == std::max<int64_t>(schur_partial_count(c), RED_BLOCKS) && (!schur32 || w.t32);
}

int ensure_work(hd_ctx* c, Work& w, int prec, int nrhs, bool schur32) {
    if (work_fits(c, w, prec, nrhs, schur32)) return HD_OK;
    free_work(w);
    int rc = alloc_work(c, w, prec, nrhs, schur32);
    if (rc) free_work(w);
    return rc;
}

}  // namespace

int minres_solve(hd_ctx* c, const hd_solve_params& prm, int nrhs, const double* b, double* x, hd_solve_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    SolveCache* cache = cache_of(c);
    Work& w64 = cache->w64;
    int rc = ensure_work(c, w64, HD_F64, nrhs, prm.mode == HD_MODE_PREC32);
    if (rc) return rc;
    const int check = prm.check_every > 0 ? prm.check_every : 8;
    std::vector<hd_solve_info> res(nrhs);
    if (prm.mode == HD_MODE_PLAIN64) {
        rc = minres_core<double, double>(c, w64, b, x, prm.use_x0 != 0, prm.tol, prm.max_it, check, res,
                                         prm.stop_true ? prm.tol : 0.0, prm.use_graph != 0);
    } else if (prm.mode == HD_MODE_PREC32) {
        rc = minres_core<double, double, float>(c, w64, b, x, prm.use_x0 != 0, prm.tol, prm.max_it, check, res,
                                                prm.stop_true ? prm.tol : 0.0, prm.use_graph != 0);
    } else if (prm.mode == HD_MODE_MIXED) {
        Work& w32 = cache->w32;
        rc = ensure_work(c, w32, HD_F32, nrhs, false);
        const int64_t Nt = w64.N * nrhs;
        if (!rc && cache->nr != Nt) {
            dfree(cache->r);
            dfree(cache->r32);
            dfree(cache->d32);
            cache->r = dalloc<double>(Nt);
            cache->r32 = dalloc<float>(Nt);
            cache->d32 = dalloc<float>(Nt);
            cache->nr = Nt;
            if (!cache->r || !cache->r32 || !cache->d32) {
                cache->nr = 0;
                rc = set_err(c, HD_ERR_OOM, "refinement vectors");
            }
        }
        double* r = cache->r;
        float *r32 = cache->r32, *d32 = cache->d32;
        if (!rc && !prm.use_x0) hipLaunchKernelGGL(k_zero<double>, dim3(nblk(Nt)), dim3(BS), 0, c->stream, Nt, x);
        std::vector<int> total(nrhs, 0), status(nrhs, HD_NOT_CONVERGED);
        std::vector<double> er(nrhs, 0.0);
        int outer = 0;
        std::vector<hd_solve_info> inner;
        while (!rc) {
            rc = true_residual(c, w64, b, x, r);
            if (rc) break;
            bool all = true;
            for (int k = 0; k < nrhs; ++k) {
                if (status[k] < 0) continue;
                if (rel_of(w64.nrm_host, k) <= prm.tol) {
                    status[k] = 0;
                    w64.nrm_host[2 * k] = 0.0;   // converged: zero right-hand side for the inner solve
                } else {
                    status[k] = HD_NOT_CONVERGED;
                    all = false;
                }
            }
            if (all || outer >= prm.max_outer) break;
            // each inner solve reduces its residual by inner_tol, but no
            // further than the target needs (with a factor 10 of margin for
            // the preconditioned norm it stops on)
            std::vector<double> itol(nrhs, prm.inner_tol);
            for (int k = 0; k < nrhs; ++k)
                if (status[k] == HD_NOT_CONVERGED)
                    itol[k] = std::max(prm.inner_tol, 0.1 * prm.tol / rel_of(w64.nrm_host, k));
            HD_HIP(c, hipMemcpyAsync(w64.nrm, w64.nrm_host, 2 * nrhs * sizeof(double), hipMemcpyHostToDevice,
                                     c->stream));
            hipLaunchKernelGGL(k_to32, dim3(nblk(w64.N), nrhs), dim3(BS), 0, c->stream, w64.N, r, w64.nrm, r32);
            rc = minres_core<float, float>(c, w32, r32, d32, false, prm.inner_tol, prm.max_it, check, inner, 0.0,
                                           prm.use_graph != 0, itol.data());
            if (rc) break;
            ++outer;
            bool brk = false;
            for (int k = 0; k < nrhs; ++k) {
                total[k] += inner[k].iterations;
                er[k] = inner[k].eta_rel;
                if (inner[k].status < 0) {
                    status[k] = inner[k].status;
                    brk = true;
                }
            }
            if (brk) break;
            hipLaunchKernelGGL(k_addscaled, dim3(nblk(w64.N), nrhs), dim3(BS), 0, c->stream, w64.N, d32, w64.nrm, x);
        }
        for (int k = 0; k < nrhs; ++k) {
            res[k].iterations = total[k];
            res[k].outer = outer;
            res[k].eta_rel = er[k];
            res[k].status = status[k];
        }
    } else {
        return set_err(c, HD_ERR_ARG, "solve mode not supported");
    }
    if (!rc) {
        rc = true_residual(c, w64, b, x, nullptr);
        for (int k = 0; k < nrhs && !rc; ++k) res[k].true_rel_res = rel_of(w64.nrm_host, k);
    }
    if (rc) return rc;
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = 0;
    for (int k = 0; k < nrhs; ++k) {
        res[k].time_s = dt;
        if (info) info[k] = res[k];
        if (res[k].status < 0) worst = res[k].status;
        else if (res[k].status > 0 && worst == 0) worst = res[k].status;
    }
    return worst;
}

// Vectors (element size es), partial sums and pinned state of a batched
// solve; schur32 adds the FP32 Schur buffers of an FP64 recurrence.
int alloc_batch_work(hd_ctx* c, BatchWork& W, size_t es, bool schur32) {
    const BatchState& B = *c->batch;
    const int ni = (int)B.inst.size();
    W.total = B.total;
    for (void** p : {&W.v, &W.vo, &W.z, &W.zn, &W.w, &W.wo, &W.q})
        if (hipMalloc(p, es * (size_t)B.total) != hipSuccess) {
            *p = nullptr;
            return set_err(c, HD_ERR_OOM, "batched MINRES vectors");
        }
    int64_t pq_tot = 0, nq_max = 0;
    for (int i = 0; i < ni; ++i) {
        const int64_t np = std::max<int64_t>(schur_partial_count(B.inst[i]), RED_BLOCKS);
        W.pq_off.push_back(pq_tot);
        W.nq_part.push_back(np);
        pq_tot += np;
        nq_max = std::max<int64_t>(nq_max, B.inst[i]->n_q);
    }
    W.pu = dalloc<double>((int64_t)RED_BLOCKS * ni);
    W.pr = dalloc<double>((int64_t)RED_BLOCKS * ni);
    W.pq = dalloc<double>(pq_tot);
    W.nrm = dalloc<double>(2 * ni);
    W.st = dalloc<MinresState>(ni);
    if (!W.pu || !W.pr || !W.pq || !W.nrm || !W.st) return set_err(c, HD_ERR_OOM, "batched MINRES partials");
    if (hipHostMalloc((void**)&W.st_host, sizeof(MinresState) * ni) != hipSuccess ||
        hipHostMalloc((void**)&W.nrm_host, sizeof(double) * 2 * ni) != hipSuccess)
        return set_err(c, HD_ERR_OOM, "batched MINRES host state");
    if (schur32) {
        int64_t npm = 0;
        for (int i = 0; i < ni; ++i) npm = std::max(npm, W.nq_part[i]);
        W.schur32.t32 = dalloc<float>(nq_max);
        W.schur32.z32 = dalloc<float>(nq_max);
        W.schur32.p32 = dalloc<double>(npm);
        if (!W.schur32.t32 || !W.schur32.z32 || !W.schur32.p32) return set_err(c, HD_ERR_OOM, "FP32 Schur buffers");
        if (B.union_ok) {
            int64_t tot = 0;
            for (int i = 0; i < ni; ++i) {
                W.q32_off.push_back(tot);
                tot += B.inst[i]->n_q;
            }
            W.t32all = dalloc<float>(tot);
            W.z32all = dalloc<float>(tot);
            if (!W.t32all || !W.z32all) return set_err(c, HD_ERR_OOM, "FP32 Schur buffers");
        }
    }
    return HD_OK;
}

// Device buffers released on every return path.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    ~DevBuf() { dfree(p); }
};

// HD_MODE_MIXED for a batch: FP64 residual of every instance, FP32 batched
// MINRES on the normalised residuals to inner_tol, FP64 update of x, until
// each instance meets tol on its true residual (instances that have, get a
// zero right-hand side, on which their inner recurrence stops at once).
int batch_mixed(hd_ctx* c, BatchWork& W, const hd_solve_params& prm, const double* b, double* x, int check,
                std::vector<hd_solve_info>& res) {
    const BatchState& B = *c->batch;
    const int ni = (int)B.inst.size();
    BatchWork W32;
    int rc = alloc_batch_work(c, W32, sizeof(float), false);
    if (rc) return rc;
    DevBuf<double> r;
    DevBuf<float> r32, d32;
    r.p = dalloc<double>(B.total);
    r32.p = dalloc<float>(B.total);
    d32.p = dalloc<float>(B.total);
    if (!r.p || !r32.p || !d32.p) return set_err(c, HD_ERR_OOM, "refinement vectors");
    if (!prm.use_x0) hipLaunchKernelGGL(k_zero<double>, dim3(nblk(B.total)), dim3(BS), 0, c->stream, B.total, x);
    std::vector<int> total(ni, 0), status(ni, HD_NOT_CONVERGED);
    std::vector<double> er(ni, 0.0);
    std::vector<hd_solve_info> inner;
    int outer = 0;
    for (;;) {
        if ((rc = batch_true_residual(c, W, b, x, r.p))) return rc;
        bool all = true;
        for (int i = 0; i < ni; ++i) {
            if (status[i] < 0) continue;
            if (rel_of(W.nrm_host, i) <= prm.tol) {
                status[i] = 0;
                W.nrm_host[2 * i] = 0.0;
            } else {
                status[i] = HD_NOT_CONVERGED;
                all = false;
            }
        }
        if (all || outer >= prm.max_outer) break;
        // per-instance inner tolerances, as in the single solve
        std::vector<double> itol(ni, prm.inner_tol);
        for (int i = 0; i < ni; ++i)
            if (status[i] == HD_NOT_CONVERGED) itol[i] = std::max(prm.inner_tol, 0.1 * prm.tol / rel_of(W.nrm_host, i));
        HD_HIP(c, hipMemcpyAsync(W.nrm, W.nrm_host, 2 * ni * sizeof(double), hipMemcpyHostToDevice, c->stream));
        for (int i = 0; i < ni; ++i) {
            const int64_t o = B.off[i], N = B.off[i + 1] - B.off[i];
            hipLaunchKernelGGL(k_to32, dim3(nblk(N), 1), dim3(BS), 0, c->stream, N, (const double*)r.p + o,
                               (const double*)W.nrm + 2 * i, r32.p + o);
        }
        if ((rc = batch_minres_core<float, float, float>(c, W32, r32.p, d32.p, false, prm.inner_tol, prm.max_it,
                                                          check, 0.0, inner, prm.use_graph != 0, itol.data())))
            return rc;
        ++outer;
        bool brk = false;
        for (int i = 0; i < ni; ++i) {
            total[i] += inner[i].iterations;
            er[i] = inner[i].eta_rel;
            if (inner[i].status < 0) {
                status[i] = inner[i].status;
                brk = true;
            }
        }
        if (brk) break;
        for (int i = 0; i < ni; ++i) {
            const int64_t o = B.off[i], N = B.off[i + 1] - B.off[i];
            hipLaunchKernelGGL(k_addscaled, dim3(nblk(N), 1), dim3(BS), 0, c->stream, N, (const float*)d32.p + o,
                               (const double*)W.nrm + 2 * i, x + o);
        }
    }
    HD_HIP(c, hipGetLastError());
    res.resize(ni);
    for (int i = 0; i < ni; ++i) {
        res[i] = hd_solve_info();
        res[i].iterations = total[i];
        res[i].outer = outer;
        res[i].eta_rel = er[i];
        res[i].status = status[i];
    }
    return HD_OK;
}

int batch_minres_solve(hd_ctx* c, const hd_solve_params& prm, const double* b, double* x, hd_solve_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    const BatchState& B = *c->batch;
    const int ni = (int)B.inst.size();
    if (prm.mode != HD_MODE_PLAIN64 && prm.mode != HD_MODE_PREC32 && prm.mode != HD_MODE_MIXED)
        return set_err(c, HD_ERR_ARG, "solve mode not supported");
    BatchWork W;
    int rc = alloc_batch_work(c, W, sizeof(double), prm.mode == HD_MODE_PREC32);
    if (rc) return rc;
    const int check = prm.check_every > 0 ? prm.check_every : 8;
    std::vector<hd_solve_info> res;
    const double tt = prm.stop_true ? prm.tol : 0.0;
    if (prm.mode == HD_MODE_PLAIN64)
        rc = batch_minres_core<double, double, double>(c, W, b, x, prm.use_x0 != 0, prm.tol, prm.max_it, check, tt,
                                                       res, prm.use_graph != 0);
    else if (prm.mode == HD_MODE_PREC32)
        rc = batch_minres_core<double, double, float>(c, W, b, x, prm.use_x0 != 0, prm.tol, prm.max_it, check, tt,
                                                      res, prm.use_graph != 0);
    else
        rc = batch_mixed(c, W, prm, b, x, check, res);
    if (rc) return rc;
    if ((rc = batch_true_residual(c, W, b, x))) return rc;
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = 0;
    for (int i = 0; i < ni; ++i) {
        res[i].true_rel_res = rel_of(W.nrm_host, i);
        res[i].time_s = dt;
        if (info) info[i] = res[i];
        if (res[i].status < 0) worst = res[i].status;
        else if (res[i].status > 0 && worst == 0) worst = res[i].status;
    }
    return worst;
}

}  // namespace hd
