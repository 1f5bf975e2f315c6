// Right-preconditioned restarted GMRES with the upper block-triangular
// preconditioner of the transformed system (Section 2.2, the remark on
// block-triangular preconditioners: with exact blocks the preconditioned
// operator has the single eigenvalue 1 and GMRES needs at most two steps; the
// blocks are replaced by M~ and the AMG cycle on S~ of the block-diagonal
// preconditioner).
//
//   P = [[tau M~, D_f^T], [0, -S^]]:   s = S^{-1} r_q (the V-cycle),
//   z_q = -s,   z_u = (tau M~)^{-1} (r_u + D_f^T s) on free RT dofs,
//   z_u = r_u on essential ones.
//
// GMRES keeps the Arnoldi basis in device memory ((restart + 1) vectors of
// n_u + n_q doubles); each step orthogonalises by classical Gram-Schmidt with
// one reorthogonalisation (two passes of all inner products at once, then
// the combined update), with deterministic two-stage reductions; the small
// Hessenberg least-squares problem (Givens rotations) is solved on the host.
// Each restart cycle ends with x += P^{-1} V y and a true FP64 residual.
#include "hd_internal.hpp"
#include "kernels_common.hpp"

#include <chrono>
#include <cmath>
#include <vector>

namespace hd {

namespace {

constexpr int BS = 256;
constexpr unsigned RED = 1024;   // first-stage blocks of every reduction

inline unsigned nblk(int64_t n) { return (unsigned)((n + BS - 1) / BS); }
inline unsigned red_grid(int64_t n) { return nblk(n) < RED ? nblk(n) : RED; }

// (D_f^T s)_k for RT dof k: s of the sub-volume below the face minus s of
// the one above (missing at the domain boundary); the face-centric form of
// the element-local incidence the block apply uses.
template <int P>
__global__ void tri_u_kernel(Geo g, uint32_t ess, int64_t n_u, const double* __restrict__ ru,
                             const double* __restrict__ s, const double* __restrict__ mdinv,
                             double* __restrict__ zu) {
    const int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (k >= n_u) return;
    if (rt_is_essential(g, P, ess, k)) {
        zu[k] = ru[k];
        return;
    }
    const int c = k >= g.off[2] ? 2 : (k >= g.off[1] ? 1 : 0);
    const int64_t r = k - g.off[c];
    const int64_t d0 = (int64_t)g.nx * P + (c == 0), d1 = (int64_t)g.ny * P + (c == 1);
    int64_t gc[3] = {r % d0, (r / d0) % d1, r / (d0 * d1)};
    const int64_t nal = c == 0 ? (int64_t)g.nx * P : (c == 1 ? (int64_t)g.ny * P : (int64_t)g.nz * P);
    auto l2 = [&](const int64_t (&v)[3]) {
        const int64_t e = v[0] / P + (int64_t)g.nx * (v[1] / P + (int64_t)g.ny * (v[2] / P));
        return e * (P * P * P) + v[0] % P + P * (v[1] % P + P * (v[2] % P));
    };
    double dt = 0.0;
    if (gc[c] >= 1) {
        int64_t v[3] = {gc[0], gc[1], gc[2]};
        v[c] -= 1;
        dt += s[l2(v)];
    }
    if (gc[c] < nal) dt -= s[l2(gc)];
    zu[k] = mdinv[k] * (ru[k] + dt);
}

// out = -a
__global__ void negate_kernel(int64_t n, const double* __restrict__ a, double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (i < n) out[i] = -a[i];
}

// out = a - b
__global__ void sub_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

// part[j * RED + block] = block's share of <V_j, w> for j < m (blockIdx.y = j)
__global__ void mdot_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, const double* __restrict__ w,
                            double* __restrict__ part) {
    __shared__ double sh[BS];
    const double* v = V + (int64_t)blockIdx.y * ldv;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) s += v[i] * w[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = BS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * RED + blockIdx.x] = sh[0];
}

// h[j] = sum of part[j * RED + 0 .. nb) in a fixed order (one block per j)
__global__ void mdot_final_kernel(const double* __restrict__ part, int nb, double* __restrict__ h) {
    __shared__ double sh[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[(int64_t)blockIdx.x * RED + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[blockIdx.x] = sh[0];
}

// w -= sum_{j < m} h[j] V_j
__global__ void mupdate_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, const double* __restrict__ h,
                               int m, double* __restrict__ w) {
    const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int j = 0; j < m; ++j) s -= h[j] * V[(int64_t)j * ldv + i];
    w[i] = s;
}

// u = sum_{j < m} y[j] V_j
__global__ void combine_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, const double* __restrict__ y,
                               int m, double* __restrict__ u) {
    const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += y[j] * V[(int64_t)j * ldv + i];
    u[i] = s;
}

__global__ void scale_kernel(int64_t n, const double* __restrict__ a, double f, double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (i < n) out[i] = a[i] * f;
}

__global__ void axpy_kernel(int64_t n, const double* __restrict__ a, double* __restrict__ x) {
    const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
    if (i < n) x[i] += a[i];
}

// Device work space of one solve, released on every return path.
struct GWork {
    double* V = nullptr;     // (m + 1) x N basis
    double *w = nullptr, *z = nullptr, *s = nullptr;
    double *part = nullptr, *h = nullptr;
    std::vector<double*> all() const { return {V, w, z, s, part, h}; }
    GWork() = default;
    GWork(const GWork&) = delete;
    GWork& operator=(const GWork&) = delete;
    ~GWork() {
        for (double* p : all()) dfree(p);
    }
};

}  // namespace

// z = P^{-1} r (FP64): the triangular preconditioner
int launch_tri_precond(hd_ctx* c, const double* r, double* z, double* s_scratch) {
    const int64_t nu = c->n_u, nq = c->n_q;
    int rc = launch_schur_prec(c, HD_F64, r + nu, s_scratch, nullptr, nullptr);
    if (rc) return rc;
    const Geo g = geo_of(c);
#define TRIU(PP)                                                                                                     \
    hipLaunchKernelGGL(tri_u_kernel<PP>, dim3(nblk(nu)), dim3(BS), 0, c->stream, g, c->ess, nu, r,                   \
                       (const double*)s_scratch, (const double*)c->d_mdinv, z)
    switch (c->p) {
        case 1: TRIU(1); break;
        case 2: TRIU(2); break;
        case 3: TRIU(3); break;
        case 4: TRIU(4); break;
        case 5: TRIU(5); break;
        default: TRIU(6); break;
    }
#undef TRIU
    hipLaunchKernelGGL(negate_kernel, dim3(nblk(nq)), dim3(BS), 0, c->stream, nq, (const double*)s_scratch, z + nu);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

namespace {

// h[0..m) = V^T w on the device and a host copy
int mdot(hd_ctx* c, const GWork& W, int64_t N, int m, const double* w, double* h_host) {
    const unsigned nb = red_grid(N);
    hipLaunchKernelGGL(mdot_kernel, dim3(nb, m), dim3(BS), 0, c->stream, N, (const double*)W.V, N, w, W.part);
    hipLaunchKernelGGL(mdot_final_kernel, dim3(m), dim3(1024), 0, c->stream, (const double*)W.part, (int)nb, W.h);
    HD_HIP(c, hipGetLastError());
    HD_HIP(c, hipMemcpyAsync(h_host, W.h, sizeof(double) * m, hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

int norm2(hd_ctx* c, GWork& W, int64_t N, const double* v, double* out) {
    const unsigned nb = red_grid(N);
    hipLaunchKernelGGL(mdot_kernel, dim3(nb, 1), dim3(BS), 0, c->stream, N, v, N, v, W.part);
    hipLaunchKernelGGL(mdot_final_kernel, dim3(1), dim3(1024), 0, c->stream, (const double*)W.part, (int)nb, W.h);
    HD_HIP(c, hipGetLastError());
    double s = 0.0;
    HD_HIP(c, hipMemcpyAsync(&s, W.h, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    *out = std::sqrt(s);
    return HD_OK;
}

}  // namespace

int gmres_solve(hd_ctx* c, double tol, int max_it, int restart, const double* b, double* x, hd_solve_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t N = c->n_u + c->n_q;
    const int m = restart;
    GWork W;
    W.V = dalloc<double>((int64_t)(m + 1) * N);
    W.w = dalloc<double>(N);
    W.z = dalloc<double>(N);
    W.s = dalloc<double>(c->n_q);
    W.part = dalloc<double>((int64_t)RED * (m + 1));
    W.h = dalloc<double>(m + 1);
    for (double* p : W.all())
        if (!p) return set_err(c, HD_ERR_OOM, "GMRES basis");
    int rc = HD_OK;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), h(m + 1), h2(m + 1), y(m);
    double bnorm = 0.0, rnorm = 0.0;
    int it = 0, cycles = 0;
    bool converged = false;
    double est = 1.0;
    // r = b - A x into V_0
    auto residual = [&](double* out) -> int {
        int r2 = launch_apply(c, HD_F64, 1, x, W.w, nullptr, 0, nullptr, 0, ESS_IDENTITY, nullptr, 0);
        if (r2) return r2;
        hipLaunchKernelGGL(sub_kernel, dim3(nblk(N)), dim3(BS), 0, c->stream, N, b, (const double*)W.w, out);
        HD_HIP(c, hipGetLastError());
        return HD_OK;
    };
    if ((rc = norm2(c, W, N, b, &bnorm))) goto done;
    if ((rc = residual(W.V))) goto done;
    if ((rc = norm2(c, W, N, W.V, &rnorm))) goto done;
    if (bnorm == 0.0) bnorm = 1.0;
    est = rnorm / bnorm;
    converged = est <= tol;
    while (!converged && it < max_it) {
        ++cycles;
        const double beta = rnorm;
        hipLaunchKernelGGL(scale_kernel, dim3(nblk(N)), dim3(BS), 0, c->stream, N, (const double*)W.V, 1.0 / beta,
                           W.V);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int k = 0;
        for (int j = 0; j < m && it < max_it; ++j) {
            ++it;
            double* vj = W.V + (int64_t)j * N;
            double* vn = W.V + (int64_t)(j + 1) * N;
            if ((rc = launch_tri_precond(c, vj, W.z, W.s))) goto done;
            if ((rc = launch_apply(c, HD_F64, 1, W.z, vn, nullptr, 0, nullptr, 0, ESS_IDENTITY, nullptr, 0)))
                goto done;
            // classical Gram-Schmidt, twice
            if ((rc = mdot(c, W, N, j + 1, vn, h.data()))) goto done;
            hipLaunchKernelGGL(mupdate_kernel, dim3(nblk(N)), dim3(BS), 0, c->stream, N, (const double*)W.V, N,
                               (const double*)W.h, j + 1, vn);
            if ((rc = mdot(c, W, N, j + 1, vn, h2.data()))) goto done;
            hipLaunchKernelGGL(mupdate_kernel, dim3(nblk(N)), dim3(BS), 0, c->stream, N, (const double*)W.V, N,
                               (const double*)W.h, j + 1, vn);
            double hn = 0.0;
            if ((rc = norm2(c, W, N, vn, &hn))) goto done;
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            const double d = std::hypot(a, bb);
            cs[j] = a / d;
            sn[j] = bb / d;
            H[(size_t)j * m + j] = d;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            k = j + 1;
            est = std::fabs(gv[j + 1]) / bnorm;
            if (!std::isfinite(est)) {
                rc = set_err(c, HD_ERR_NONFINITE, "GMRES: non-finite residual estimate");
                goto done;
            }
            if (est <= tol || hn == 0.0) break;
            hipLaunchKernelGGL(scale_kernel, dim3(nblk(N)), dim3(BS), 0, c->stream, N, (const double*)vn, 1.0 / hn,
                               vn);
        }
        // y = R^{-1} g, x += P^{-1} V y
        for (int i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
            y[i] = s / H[(size_t)i * m + i];
        }
        HD_HIP(c, hipMemcpyAsync(W.h, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(combine_kernel, dim3(nblk(N)), dim3(BS), 0, c->stream, N, (const double*)W.V, N,
                           (const double*)W.h, k, W.w);
        HD_HIP(c, hipStreamSynchronize(c->stream));
        if ((rc = launch_tri_precond(c, W.w, W.z, W.s))) goto done;
        hipLaunchKernelGGL(axpy_kernel, dim3(nblk(N)), dim3(BS), 0, c->stream, N, (const double*)W.z, x);
        if ((rc = residual(W.V))) goto done;
        if ((rc = norm2(c, W, N, W.V, &rnorm))) goto done;
        converged = rnorm / bnorm <= tol;
    }
done:
    if (rc) return rc;
    if (info) {
        info->status = converged ? 0 : HD_NOT_CONVERGED;
        info->iterations = it;
        info->outer = cycles;
        info->eta_rel = est;
        info->true_rel_res = rnorm / bnorm;
        info->time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return converged ? HD_OK : HD_NOT_CONVERGED;
}

}  // namespace hd
