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

#include <cmath>
#include <type_traits>

namespace hd {

namespace {

constexpr int BS = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

template <typename T>
__global__ void vc_pre_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const T* __restrict__ av, const T* __restrict__ dinv, const T* __restrict__ b,
                              T* __restrict__ x, T* __restrict__ r, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    T s = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = ci[k];
        s += av[k] * (dinv[j] * b[j]);
    }
    x[i] = dinv[i] * b[i];
    r[i] = b[i] - s;
}

// y_i = sum_k M_ik x_k  (restriction with R = P^T) or y_i += ... (prolongation)
template <typename T, bool ADD>
__global__ void vc_spmv_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const T* __restrict__ mv, const T* __restrict__ x, T* __restrict__ y,
                               const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    T s = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += mv[k] * x[ci[k]];
    if (ADD) y[i] += s;
    else y[i] = s;
}

// z = x + dinv (b - A x); optional partial sums of z (for the mean) or of
// z * b (the preconditioned norm), one per block
template <typename T>
__global__ void vc_post_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const T* __restrict__ av, const T* __restrict__ dinv, const T* __restrict__ b,
                               const T* __restrict__ x, T* __restrict__ z, double* __restrict__ part, int part_kind,
                               const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double s[BS];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double contrib = 0.0;
    if (i < n) {
        T acc = 0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc += av[k] * x[ci[k]];
        const T zi = x[i] + dinv[i] * (b[i] - acc);
        z[i] = zi;
        contrib = part_kind == 1 ? (double)zi : (double)zi * (double)b[i];
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

// z -= mean (mean = sum / n from a device scalar), partial sums of z * b
template <typename T>
__global__ void vc_sub_mean_kernel(int64_t n, const double* __restrict__ sum, const T* __restrict__ b,
                                   T* __restrict__ z, double* __restrict__ part, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double s[BS];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const double mean = *sum / (double)n;
    double contrib = 0.0;
    if (i < n) {
        const T zi = (T)((double)z[i] - mean);
        z[i] = zi;
        contrib = (double)zi * (double)b[i];
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
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double contrib = 0.0;
    if (i < n) {
        const T zi = mdinv[i] * r[i];
        z[i] = zi;
        contrib = (double)zi * (double)r[i];
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
    hipLaunchKernelGGL(vc_pre_kernel<T>, dim3(nblk(n)), dim3(BS), 0, c->stream, n, lv.A.rp, lv.A.ci, av, dinv, b, x,
                       r, done);
    hipLaunchKernelGGL((vc_spmv_kernel<T, false>), dim3(nblk(lv.R.nrows)), dim3(BS), 0, c->stream, lv.R.nrows,
                       lv.R.rp, lv.R.ci, pick<T>(lv.R.v, lv.R.v32), r, bc, done);
    int rc = cycle<T>(c, l + 1, bc, zc, nullptr, 0, done);
    if (rc) return rc;
    hipLaunchKernelGGL((vc_spmv_kernel<T, true>), dim3(nblk(n)), dim3(BS), 0, c->stream, n, lv.P.rp, lv.P.ci,
                       pick<T>(lv.P.v, lv.P.v32), zc, x, done);
    hipLaunchKernelGGL(vc_post_kernel<T>, dim3(nblk(n)), dim3(BS), 0, c->stream, n, lv.A.rp, lv.A.ci, av, dinv, b, x,
                       z, part, part_kind, done);
    return HD_OK;
}

template <typename T>
__global__ void sum_partial_kernel(int64_t n, const T* __restrict__ a, const T* __restrict__ b,
                                   double* __restrict__ part, const int* __restrict__ done) {
    if (done && *done) return;
    __shared__ double s[BS];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    s[threadIdx.x] = i < n ? (b ? (double)a[i] * (double)b[i] : (double)a[i]) : 0.0;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// z = S^{-1} b on the L2 dofs; `part` (optional) receives per-block partial
// sums of z * b after the constant has been removed (singular case).
template <typename T>
int schur_apply(hd_ctx* c, const T* b, T* z, double* part, const int* done) {
    const int64_t n = c->n_q;
    const bool one_level = c->lev.size() == 1;
    if (!c->singular) {
        int rc = cycle<T>(c, 0, b, z, one_level ? nullptr : part, 2, done);
        if (rc) return rc;
        if (one_level && part)
            hipLaunchKernelGGL(sum_partial_kernel<T>, dim3(nblk(n)), dim3(BS), 0, c->stream, n, z, b, part, done);
        return HD_OK;
    }
    int rc = launch_ensure_partial(c, (int64_t)nblk(n));
    if (rc) return rc;
    double* zs = c->d_partial;
    rc = cycle<T>(c, 0, b, z, one_level ? nullptr : zs, 1, done);
    if (rc) return rc;
    if (one_level)
        hipLaunchKernelGGL(sum_partial_kernel<T>, dim3(nblk(n)), dim3(BS), 0, c->stream, n, z, (const T*)nullptr, zs,
                           done);
    rc = reduce_sum_partials(c, zs, nblk(n), c->d_scal + 6);
    if (rc) return rc;
    hipLaunchKernelGGL(vc_sub_mean_kernel<T>, dim3(nblk(n)), dim3(BS), 0, c->stream, n, c->d_scal + 6, b, z, part,
                       done);
    return HD_OK;
}

}  // namespace

int launch_diag_prec(hd_ctx* c, int prec, const void* r, void* z, double* part) {
    const int64_t n = c->n_u;
    if (prec == HD_F64)
        hipLaunchKernelGGL(diag_prec_kernel<double>, dim3(nblk(n)), dim3(BS), 0, c->stream, n, c->d_mdinv,
                           (const double*)r, (double*)z, part);
    else
        hipLaunchKernelGGL(diag_prec_kernel<float>, dim3(nblk(n)), dim3(BS), 0, c->stream, n, c->d_mdinv32,
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

int precond_partials(const hd_ctx* c) { return (int)nblk(c->n_q > c->n_u ? c->n_q : c->n_u); }

int launch_precond(hd_ctx* c, int prec, const void* r, void* z, double* dot_partial_u, double* dot_partial_q,
                   const int* done) {
    int rc = launch_diag_prec(c, prec, r, z, dot_partial_u);
    if (rc) return rc;
    const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
    return launch_schur_prec(c, prec, (const char*)r + es * c->n_u, (char*)z + es * c->n_u, dot_partial_q, done);
}

// ---- upload of the host hierarchy ------------------------------------------

namespace {

template <typename F>
__global__ void to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

int upload_csr(hd_ctx* c, const HostCSR& h, DevCSR& d) {
    d.nrows = h.nrows;
    d.ncols = h.ncols;
    d.nnz = h.nnz();
    d.rp = dalloc<int32_t>(h.nrows + 1);
    d.ci = dalloc<int32_t>(d.nnz);
    d.v = dalloc<double>(d.nnz);
    d.v32 = dalloc<float>(d.nnz);
    if (!d.rp || !d.ci || !d.v || !d.v32) return set_err(c, HD_ERR_OOM, "AMG level storage");
    HD_HIP(c, hipMemcpyAsync(d.rp, h.rp.data(), sizeof(int32_t) * (h.nrows + 1), hipMemcpyHostToDevice, c->stream));
    if (d.nnz) {
        HD_HIP(c, hipMemcpyAsync(d.ci, h.ci.data(), sizeof(int32_t) * d.nnz, hipMemcpyHostToDevice, c->stream));
        HD_HIP(c, hipMemcpyAsync(d.v, h.v.data(), sizeof(double) * d.nnz, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(to_f32_kernel<float>, dim3(nblk(d.nnz)), dim3(BS), 0, c->stream, d.v, d.v32, d.nnz);
    }
    return HD_OK;
}

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
}

int upload_amg(hd_ctx* c) {
    free_levels(c);
    const HostAMG& H = c->host_amg;
    const int L = (int)H.A.size();
    c->lev.resize(L);
    for (int l = 0; l < L; ++l) {
        DevLevel& lv = c->lev[l];
        const HostCSR& A = H.A[l];
        int rc;
        if (l == 0) lv.A = c->S;
        else if ((rc = upload_csr(c, A, lv.A))) return rc;
        if (l < L - 1) {
            if ((rc = upload_csr(c, H.P[l], lv.P))) return rc;
            HostCSR R;
            // transpose on the host
            R.nrows = H.P[l].ncols;
            R.ncols = H.P[l].nrows;
            R.rp.assign(R.nrows + 1, 0);
            for (int32_t j : H.P[l].ci) R.rp[j + 1]++;
            for (int64_t i = 0; i < R.nrows; ++i) R.rp[i + 1] += R.rp[i];
            R.ci.resize(H.P[l].ci.size());
            R.v.resize(H.P[l].v.size());
            std::vector<int32_t> pos(R.rp.begin(), R.rp.end() - 1);
            for (int64_t i = 0; i < H.P[l].nrows; ++i)
                for (int32_t k = H.P[l].rp[i]; k < H.P[l].rp[i + 1]; ++k) {
                    const int32_t j = H.P[l].ci[k];
                    R.ci[pos[j]] = (int32_t)i;
                    R.v[pos[j]] = H.P[l].v[k];
                    pos[j]++;
                }
            if ((rc = upload_csr(c, R, lv.R))) return rc;
        }
        // l1 diagonal
        std::vector<double> d(A.nrows);
        std::vector<float> d32(A.nrows);
        for (int64_t i = 0; i < A.nrows; ++i) {
            double s = 0.0;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.v[k]);
            d[i] = 1.0 / s;
            d32[i] = (float)(1.0 / s);
        }
        lv.dinv = dalloc<double>(A.nrows);
        lv.dinv32 = dalloc<float>(A.nrows);
        lv.b = dalloc<double>(A.nrows);
        lv.x = dalloc<double>(A.nrows);
        lv.r = dalloc<double>(A.nrows);
        lv.z = dalloc<double>(A.nrows);
        lv.b32 = dalloc<float>(A.nrows);
        lv.x32 = dalloc<float>(A.nrows);
        lv.r32 = dalloc<float>(A.nrows);
        lv.z32 = dalloc<float>(A.nrows);
        if (!lv.dinv || !lv.dinv32 || !lv.b || !lv.x || !lv.r || !lv.z || !lv.b32 || !lv.x32 || !lv.r32 || !lv.z32)
            return set_err(c, HD_ERR_OOM, "AMG work vectors");
        HD_HIP(c, hipMemcpyAsync(lv.dinv, d.data(), sizeof(double) * A.nrows, hipMemcpyHostToDevice, c->stream));
        HD_HIP(c, hipMemcpyAsync(lv.dinv32, d32.data(), sizeof(float) * A.nrows, hipMemcpyHostToDevice, c->stream));
        HD_HIP(c, hipStreamSynchronize(c->stream));
    }
    const int64_t nc = H.A.back().nrows;
    c->n_coarse = nc;
    c->d_cinv = dalloc<double>(nc * nc);
    if (!c->d_cinv) return set_err(c, HD_ERR_OOM, "coarse inverse");
    HD_HIP(c, hipMemcpyAsync(c->d_cinv, H.coarse_inv.data(), sizeof(double) * nc * nc, hipMemcpyHostToDevice,
                             c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

}  // namespace hd
