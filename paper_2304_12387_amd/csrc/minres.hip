// Block-preconditioned MINRES for the transformed saddle-point system
// (Sections 2 and 3: the system is symmetric indefinite, the preconditioner
// symmetric positive definite, so MINRES with its short recurrences applies).
// Preconditioned Lanczos with Givens rotations (Paige-Saunders); |eta| is the
// B^{-1}-norm of the residual and the iteration stops when
// |eta| <= tol |eta_0|.
//
// The Lanczos/Givens scalars live on the device in FP64 and are updated by a
// one-block kernel per iteration, so no host round trip is needed between
// iterations; the host polls the stop flag every few iterations.  Inner
// products are two-stage deterministic reductions in FP64 (per-block
// partials, then one block in fixed order).  Per iteration:
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
// scalars, FP64 coarse solve).
#include "kernels_common.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <type_traits>

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

__device__ double block_sum(double v) {
    __shared__ double s[1024];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    return s[0];
}

__global__ void k_delta(MinresState* st, const double* __restrict__ part, int64_t n) {
    if (st->stop) return;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) acc += part[k];
    const double d = block_sum(acc);
    if (threadIdx.x == 0) {
        st->delta = d;
        st->cv1 = d / st->gamma;
        st->cv2 = st->gamma / st->gamma_old;
    }
}

__global__ void k_givens(MinresState* st, const double* __restrict__ pu, int64_t nu, const double* __restrict__ pq,
                         int64_t nq, int maxit) {
    if (st->stop) {
        if (threadIdx.x == 0) st->skipped = 1;
        return;
    }
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nu; k += blockDim.x) acc += pu[k];
    double acc2 = 0.0;
    for (int64_t k = threadIdx.x; k < nq; k += blockDim.x) acc2 += pq[k];
    const double g2 = block_sum(acc) + block_sum(acc2);
    if (threadIdx.x != 0) return;
    st->skipped = 0;
    if (!(g2 >= 0.0) || !isfinite(g2)) {
        st->status = isfinite(g2) ? HD_ERR_BREAKDOWN : HD_ERR_NONFINITE;
        st->stop = 1;
        st->skipped = 1;
        return;
    }
    const double gamma = st->gamma, delta = st->delta;
    const double gnew = sqrt(g2);
    const double a0 = st->c * delta - st->c_old * st->s * gamma;
    const double a1 = sqrt(a0 * a0 + gnew * gnew);
    const double a2 = st->s * delta + st->c_old * st->c * gamma;
    const double a3 = st->s_old * gamma;
    const double cn = a0 / a1, sn = gnew / a1;
    st->a1inv = 1.0 / a1;
    st->a2 = a2;
    st->a3 = a3;
    st->zscale = 1.0 / gamma;
    st->xcoef = cn * st->eta;
    st->eta = -sn * st->eta;
    st->gamma_old = gamma;
    st->gamma = gnew;
    st->inv_gamma = gnew > 0.0 ? 1.0 / gnew : 0.0;
    st->c_old = st->c;
    st->c = cn;
    st->s_old = st->s;
    st->s = sn;
    st->iter += 1;
    if (fabs(st->eta) <= st->tol * st->eta0 || gnew == 0.0) {
        st->stop = 1;
        st->status = 0;
    } else if (st->iter >= maxit) {
        st->stop = 1;
        st->status = HD_NOT_CONVERGED;
    }
}

__global__ void k_start(MinresState* st, const double* __restrict__ pu, int64_t nu, const double* __restrict__ pq,
                        int64_t nq, double tol) {
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nu; k += blockDim.x) acc += pu[k];
    double acc2 = 0.0;
    for (int64_t k = threadIdx.x; k < nq; k += blockDim.x) acc2 += pq[k];
    const double g2 = block_sum(acc) + block_sum(acc2);
    if (threadIdx.x != 0) return;
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
    *st = s;
}

// v_old <- q - cv1 v - cv2 v_old  (= v_{j+1});  z_u = mdinv * v_{j+1,u}
template <typename T>
__global__ void k_vupd(int64_t N, int64_t nu, const T* __restrict__ q, const T* __restrict__ v, T* __restrict__ vo,
                       const T* __restrict__ mdinv, T* __restrict__ z, const MinresState* __restrict__ st,
                       double* __restrict__ part) {
    if (st->stop) return;
    __shared__ double s[BS];
    const T cv1 = (T)st->cv1, cv2 = (T)st->cv2;
    double contrib = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
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
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// w_old <- (z zscale - a3 w_old - a2 w) a1inv  (= w_{j+1});  x += xcoef w_{j+1}
template <typename T, typename X>
__global__ void k_wupd(int64_t N, const T* __restrict__ z, T* __restrict__ wo, const T* __restrict__ w,
                       X* __restrict__ x, const MinresState* __restrict__ st) {
    if (st->skipped) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T zs = (T)st->zscale, a3 = (T)st->a3, a2 = (T)st->a2, a1i = (T)st->a1inv;
    const T wn = (z[i] * zs - a3 * wo[i] - a2 * w[i]) * a1i;
    wo[i] = wn;
    x[i] += (X)st->xcoef * (X)wn;
}

// v = b - q (or b when q == nullptr), v_old = w = w_old = 0
template <typename T, typename B>
__global__ void k_init(int64_t N, const B* __restrict__ b, const T* __restrict__ q, T* __restrict__ v,
                       T* __restrict__ vo, T* __restrict__ w, T* __restrict__ wo) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    v[i] = q ? (T)((T)b[i] - q[i]) : (T)b[i];
    vo[i] = 0;
    w[i] = 0;
    wo[i] = 0;
}

template <typename T>
__global__ void k_zero(int64_t N, T* __restrict__ x) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) x[i] = 0;
}

// r = b - q (FP64), partial sums of r^2 and b^2
__global__ void k_residual(int64_t N, const double* __restrict__ b, const double* __restrict__ q,
                           double* __restrict__ r, double* __restrict__ pr, double* __restrict__ pb) {
    __shared__ double s[BS];
    double rr = 0.0, bb = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
        const double ri = b[i] - q[i];
        if (r) r[i] = ri;
        rr += ri * ri;
        bb += b[i] * b[i];
    }
    s[threadIdx.x] = rr;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) pr[blockIdx.x] = s[0];
    __syncthreads();
    s[threadIdx.x] = bb;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) pb[blockIdx.x] = s[0];
}

// r32 = r * inv (FP64 -> FP32) and x += scale * d32
__global__ void k_to32(int64_t N, const double* __restrict__ r, const double* __restrict__ scal, float* __restrict__ o) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) o[i] = (float)(r[i] / scal[0]);
}
__global__ void k_addscaled(int64_t N, const float* __restrict__ d, const double* __restrict__ scal,
                            double* __restrict__ x) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) x[i] += scal[0] * (double)d[i];
}
__global__ void k_sqrt(double* v, int n) {
    if (threadIdx.x < n) v[threadIdx.x] = sqrt(v[threadIdx.x]);
}

struct Work {
    int64_t N = 0;
    int prec = HD_F64;
    void *v = nullptr, *vo = nullptr, *z = nullptr, *zn = nullptr, *w = nullptr, *wo = nullptr, *q = nullptr;
    double *pd = nullptr, *pu = nullptr, *pq = nullptr;
    int64_t nq_part = 0;
    MinresState* st = nullptr;
    MinresState* st_host = nullptr;
};

void free_work(Work& w) {
    dfree(w.v);
    dfree(w.vo);
    dfree(w.z);
    dfree(w.zn);
    dfree(w.w);
    dfree(w.wo);
    dfree(w.q);
    dfree(w.pd);
    dfree(w.pu);
    dfree(w.pq);
    dfree(w.st);
    if (w.st_host) (void)hipHostFree(w.st_host);
    w = Work();
}

int alloc_work(hd_ctx* c, Work& w, int prec) {
    w.N = c->n_u + c->n_q;
    w.prec = prec;
    const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
    void** vs[] = {&w.v, &w.vo, &w.z, &w.zn, &w.w, &w.wo, &w.q};
    for (void** p : vs) {
        if (hipMalloc(p, es * w.N) != hipSuccess) return set_err(c, HD_ERR_OOM, "MINRES vectors");
    }
    w.pd = dalloc<double>(std::max<int64_t>(c->ne, apply_partial_count(c)));
    w.pu = dalloc<double>(nblk(w.N));
    w.nq_part = schur_partial_count(c);
    w.pq = dalloc<double>(std::max<int64_t>(w.nq_part, nblk(w.N)));
    w.st = dalloc<MinresState>(1);
    if (!w.pd || !w.pu || !w.pq || !w.st) return set_err(c, HD_ERR_OOM, "MINRES partials");
    if (hipHostMalloc((void**)&w.st_host, sizeof(MinresState)) != hipSuccess)
        return set_err(c, HD_ERR_OOM, "MINRES host state");
    return HD_OK;
}

int true_residual(hd_ctx* c, Work& wk64, const double* b, const double* x, double* r, double& rel,
                  double* rnorm_dev);

// tighten the stop threshold and resume a converged recurrence
__global__ void k_retarget(MinresState* st, double tol) {
    if (st->status == 0) {
        st->tol = tol;
        st->stop = 0;
    }
}

// Preconditioned MINRES in precision T on A x = b (b of precision B, x of
// precision T, x0 = 0 unless use_x0).  Returns iterations and status.
template <typename T, typename B>
int minres_core(hd_ctx* c, Work& wk, const B* b, T* x, bool use_x0, double tol, int maxit, int check_every,
                int& iters, int& status, double& eta_rel, double true_tol = 0.0) {
    const int prec = std::is_same<T, double>::value ? HD_F64 : HD_F32;
    const int64_t N = wk.N, nu = c->n_u, nq = c->n_q;
    T* v = (T*)wk.v;
    T* vo = (T*)wk.vo;
    T* z = (T*)wk.z;
    T* zn = (T*)wk.zn;
    T* w = (T*)wk.w;
    T* wo = (T*)wk.wo;
    T* q = (T*)wk.q;
    const T* mdinv = std::is_same<T, double>::value ? (const T*)c->d_mdinv : (const T*)c->d_mdinv32;
    int rc;
    if (use_x0) {
        if ((rc = launch_apply(c, prec, x, q, nullptr, nullptr, ESS_IDENTITY, nullptr))) return rc;
        hipLaunchKernelGGL((k_init<T, B>), dim3(nblk(N)), dim3(BS), 0, c->stream, N, b, q, v, vo, w, wo);
    } else {
        hipLaunchKernelGGL(k_zero<T>, dim3(nblk(N)), dim3(BS), 0, c->stream, N, x);
        hipLaunchKernelGGL((k_init<T, B>), dim3(nblk(N)), dim3(BS), 0, c->stream, N, b, (const T*)nullptr, v, vo, w,
                           wo);
    }
    // z_1 = B^{-1} v_1
    if ((rc = launch_diag_prec(c, prec, v, z, wk.pu))) return rc;
    // the diag kernel covers n_u rows; its partial count is nblk(n_u) <= nblk(N)
    if ((rc = launch_schur_prec(c, prec, v + nu, z + nu, wk.pq, nullptr))) return rc;
    hipLaunchKernelGGL(k_start, dim3(1), dim3(1024), 0, c->stream, wk.st, wk.pu, (int64_t)red_grid(nu), wk.pq,
                       wk.nq_part, tol);
    HD_HIP(c, hipGetLastError());
    const int* stop = &wk.st->stop;
    int it_launched = 0, retargets = 0;
    for (;;) {
        for (int k = 0; k < check_every && it_launched < maxit; ++k, ++it_launched) {
            if ((rc = launch_apply(c, prec, z, q, &wk.st->inv_gamma, wk.pd, ESS_IDENTITY, stop))) return rc;
            hipLaunchKernelGGL(k_delta, dim3(1), dim3(1024), 0, c->stream, wk.st, wk.pd, apply_partial_count(c));
            hipLaunchKernelGGL(k_vupd<T>, dim3(red_grid(N)), dim3(BS), 0, c->stream, N, nu, q, v, vo, mdinv, zn,
                               wk.st, wk.pu);
            if ((rc = launch_schur_prec(c, prec, vo + nu, zn + nu, wk.pq, stop))) return rc;
            hipLaunchKernelGGL(k_givens, dim3(1), dim3(1024), 0, c->stream, wk.st, wk.pu, (int64_t)red_grid(N),
                               wk.pq, wk.nq_part, maxit);
            hipLaunchKernelGGL((k_wupd<T, T>), dim3(nblk(N)), dim3(BS), 0, c->stream, N, z, wo, w, x, wk.st);
            std::swap(v, vo);
            std::swap(z, zn);
            std::swap(w, wo);
        }
        HD_HIP(c, hipGetLastError());
        HD_HIP(c, hipMemcpyAsync(wk.st_host, wk.st, sizeof(MinresState), hipMemcpyDeviceToHost, c->stream));
        HD_HIP(c, hipStreamSynchronize(c->stream));
        // iterations launched after the stop flag was raised were no-ops on
        // the device; every executed iteration swapped each buffer pair once,
        // so the parity of the executed count fixes the live arrangement
        {
            const bool odd = wk.st_host->iter % 2 != 0;
            v = (T*)(odd ? wk.vo : wk.v);
            vo = (T*)(odd ? wk.v : wk.vo);
            z = (T*)(odd ? wk.zn : wk.z);
            zn = (T*)(odd ? wk.z : wk.zn);
            w = (T*)(odd ? wk.wo : wk.w);
            wo = (T*)(odd ? wk.w : wk.wo);
        }
        if (wk.st_host->stop && wk.st_host->status == 0 && true_tol > 0.0 && retargets < 8) {
            // the recurrence stops on the preconditioned residual norm; when the
            // caller asks for a true FP64 residual, check it and, if it is not
            // yet met, continue the same recurrence with a tighter threshold
            if constexpr (std::is_same<T, double>::value && std::is_same<B, double>::value) {
                double rel = 0.0;
                if ((rc = true_residual(c, wk, b, x, nullptr, rel, nullptr))) return rc;
                if (rel > true_tol) {
                    const double nt = wk.st_host->tol * (true_tol / rel) * 0.7;
                    hipLaunchKernelGGL(k_retarget, dim3(1), dim3(1), 0, c->stream, wk.st, nt);
                    ++retargets;
                    if (it_launched < maxit) continue;
                }
            }
        }
        if (wk.st_host->stop || it_launched >= maxit) break;
    }
    const MinresState& s = *wk.st_host;
    iters = s.iter;
    status = s.stop ? s.status : HD_NOT_CONVERGED;
    eta_rel = s.eta0 > 0 ? std::fabs(s.eta) / s.eta0 : 0.0;
    return HD_OK;
}

// ||b - A x|| / ||b|| in FP64; r (optional) receives b - A x; rnorm_dev gets
// ||r|| (device scalar) when non-null
int true_residual(hd_ctx* c, Work& wk64, const double* b, const double* x, double* r, double& rel,
                  double* rnorm_dev) {
    const int64_t N = c->n_u + c->n_q;
    int rc;
    if ((rc = launch_apply(c, HD_F64, x, wk64.q, nullptr, nullptr, ESS_IDENTITY, nullptr))) return rc;
    hipLaunchKernelGGL(k_residual, dim3(red_grid(N)), dim3(BS), 0, c->stream, N, b, (const double*)wk64.q, r,
                       wk64.pu, wk64.pq);
    if ((rc = reduce_sum_partials(c, wk64.pu, red_grid(N), c->d_scal + 0))) return rc;
    if ((rc = reduce_sum_partials(c, wk64.pq, red_grid(N), c->d_scal + 1))) return rc;
    hipLaunchKernelGGL(k_sqrt, dim3(1), dim3(64), 0, c->stream, c->d_scal, 2);
    double h[2];
    HD_HIP(c, hipMemcpyAsync(h, c->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    if (rnorm_dev) HD_HIP(c, hipMemcpyAsync(rnorm_dev, c->d_scal, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    rel = h[1] > 0 ? h[0] / h[1] : h[0];
    return HD_OK;
}

}  // namespace

int minres_solve(hd_ctx* c, const hd_solve_params& prm, const double* b, double* x, hd_solve_info& info) {
    info = hd_solve_info();
    auto t0 = std::chrono::steady_clock::now();
    Work w64;
    int rc = alloc_work(c, w64, HD_F64);
    if (rc) {
        free_work(w64);
        return rc;
    }
    const int check = prm.check_every > 0 ? prm.check_every : 8;
    int status = 0;
    if (prm.mode == HD_MODE_PLAIN64) {
        int it = 0;
        double er = 0;
        rc = minres_core<double, double>(c, w64, b, x, prm.use_x0 != 0, prm.tol, prm.max_it, check, it, status, er,
                                         prm.stop_true ? prm.tol : 0.0);
        info.iterations = it;
        info.outer = 1;
        info.eta_rel = er;
    } else if (prm.mode == HD_MODE_MIXED) {
        Work w32;
        rc = alloc_work(c, w32, HD_F32);
        double* r = nullptr;
        float *r32 = nullptr, *d32 = nullptr;
        if (!rc) {
            r = dalloc<double>(w64.N);
            r32 = dalloc<float>(w64.N);
            d32 = dalloc<float>(w64.N);
            if (!r || !r32 || !d32) rc = set_err(c, HD_ERR_OOM, "refinement vectors");
        }
        if (!rc && !prm.use_x0) {
            hipLaunchKernelGGL(k_zero<double>, dim3(nblk(w64.N)), dim3(BS), 0, c->stream, w64.N, x);
        }
        int total = 0, outer = 0;
        double rel = 1.0, er = 0.0;
        status = HD_NOT_CONVERGED;
        while (!rc) {
            rc = true_residual(c, w64, b, x, r, rel, c->d_scal + 2);
            if (rc) break;
            if (rel <= prm.tol) {
                status = 0;
                break;
            }
            if (outer >= prm.max_outer) break;
            hipLaunchKernelGGL(k_to32, dim3(nblk(w64.N)), dim3(BS), 0, c->stream, w64.N, r, c->d_scal + 2, r32);
            int it = 0, st = 0;
            rc = minres_core<float, float>(c, w32, r32, d32, false, prm.inner_tol, prm.max_it, check, it, st, er);
            if (rc) break;
            total += it;
            ++outer;
            if (st < 0) {
                status = st;
                break;
            }
            hipLaunchKernelGGL(k_addscaled, dim3(nblk(w64.N)), dim3(BS), 0, c->stream, w64.N, d32, c->d_scal + 2, x);
        }
        dfree(r);
        dfree(r32);
        dfree(d32);
        free_work(w32);
        info.iterations = total;
        info.outer = outer;
        info.eta_rel = er;
    } else {
        free_work(w64);
        return set_err(c, HD_ERR_ARG, "solve mode not supported");
    }
    if (!rc) {
        double rel = 0;
        rc = true_residual(c, w64, b, x, nullptr, rel, nullptr);
        info.true_rel_res = rel;
    }
    free_work(w64);
    if (rc) return rc;
    auto t1 = std::chrono::steady_clock::now();
    info.time_s = std::chrono::duration<double>(t1 - t0).count();
    info.status = status;
    return status;
}

}  // namespace hd
