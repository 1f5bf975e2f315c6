// Learned per-element correction of the (1,1)-block diagonal M~ = diag(M)
// (Section 2.3 gives the plain diagonal; the correction is an extension).
//
// Six log-scalings theta = (x-, x+, y-, y+, z-, z+) per element rescale the
// element's contribution to the diagonal before it is summed:
//   s_dof = exp((1 - xi_i) theta_{2c} + xi_i theta_{2c+1})
// for an RT dof of component c with index i along c (xi the Gauss-Lobatto
// sub-element vertices).  S~ and the AMG are then built from the result.
//
// Training data: per element, theta* minimises the spread
// log lambda_max - log lambda_min of the pencil (M_e, diag(s * diag M_e)) on
// sum(theta) = 0, by projected gradient descent with Armijo backtracking from
// theta = 0.  The extreme eigenpairs come from a Lanczos run on the
// symmetrically scaled element matrix, applied matrix-free by sum
// factorisation at the Gauss points (one workgroup per element, everything
// in LDS); the Ritz vectors are formed by repeating the run, which
// regenerates the same Lanczos vectors bit for bit.
//
// Network: x in R^27 (24 vertex offsets from the centroid over the mean edge
// length, ln alpha, ln beta, p / 6) -> Linear(27, 64) - GELU -
// Linear(64, 64) - GELU - Linear(64, 6) -> theta = clip(o, +-ln 4), with the
// exact GELU x Phi(x).  Training in FP32 (mean squared error against the
// clipped targets, Adam); inference in BF16 on the matrix cores
// (16 x 16 x 16 BF16 MFMA with FP32 accumulation), or in FP32.
#include "kernels_common.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

namespace hd {

namespace {

constexpr int NIN = 27, NHID = 64, NOUT = 6;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NHID * NIN, OFF_W2 = OFF_B1 + NHID, OFF_B2 = OFF_W2 + NHID * NHID,
              OFF_W3 = OFF_B2 + NHID, OFF_B3 = OFF_W3 + NOUT * NHID, NPARAM = OFF_B3 + NOUT;
constexpr double LN4 = 1.38629436111989061883;

// ---------------------------------------------------------------------------
// target generation
// ---------------------------------------------------------------------------
constexpr int TNT = 256;    // threads per element
constexpr int KLAN = 160;   // Lanczos step limit (fewer when the element has fewer dofs)
constexpr int KCHECK = 16;  // steps between convergence checks
// a Ritz pair is accepted when its residual bound beta_k |z_k| is below this
// fraction of lambda_min (the eigenvalue error is at most the residual)
constexpr double RITZ_TOL = 1e-9;

template <int P>
struct TgtLDS {
    static constexpr int Q = P + 1, Q3 = Q * Q * Q, NC = P * P * (P + 1), NRT = 3 * NC;
    double L[Q * (P + 1)], H[Q * P], L2[Q * (P + 1)], H2[Q * P], gll[P + 1];
    double X[24];
    double G[6][Q3];
    double m[NRT], dh[NRT];
    double v[NRT], vprev[NRT], w[NRT], ylo[NRT], yhi[NRT];
    double u[3][Q3], t1[Q3], t2[Q3];
    double alpha[KLAN], beta[KLAN + 1], zlo[KLAN], zhi[KLAN];
    double red[TNT / 64][8];
    double theta[6], trial[6], g[6], sc[8];
    int flag[4];
    // elements with at most KLAN dofs keep the whole Lanczos basis and
    // re-orthogonalise fully (the run then spans the whole space)
    static constexpr bool FULL = NRT <= KLAN;
    double basis[FULL ? NRT * NRT : 1];
    double hred[TNT / 64][FULL ? NRT : 1];
};

__device__ double block_sum(double v, double (*red)[8], int slot) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[wv][slot] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < TNT / 64; ++k) s += red[k][slot];
    __syncthreads();
    return s;
}

// weight of theta_j in log s of dof d (component c, index i along c)
template <int P>
__device__ __forceinline__ void dof_weight(const TgtLDS<P>& S, int d, int& c, double& a_lo, double& a_hi) {
    constexpr int NC = TgtLDS<P>::NC;
    c = d / NC;
    int i, j, k;
    local_ijk<P>(c, d % NC, i, j, k);
    const int idx = c == 0 ? i : (c == 1 ? j : k);
    a_hi = S.gll[idx];
    a_lo = 1.0 - a_hi;
}

// y = D^{-1/2} M_e D^{-1/2} x (x, y in LDS; y must not alias x)
template <int P>
__device__ void scaled_mass(TgtLDS<P>& S, const double* x, double* y, int tid) {
    constexpr int Q = P + 1, Q3 = Q * Q * Q, NC = TgtLDS<P>::NC, NRT = TgtLDS<P>::NRT;
    for (int d = tid; d < NRT; d += TNT) y[d] = S.dh[d] * x[d];
    __syncthreads();
    // component 0: (P+1, P, P) -> quadrature points
    contract<double, P + 1, P, P, 0, Q, false, P + 1>(y, S.t1, S.L, tid, TNT);
    __syncthreads();
    contract<double, Q, P, P, 1, Q, false, P>(S.t1, S.t2, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, P, 2, Q, false, P>(S.t2, S.u[0], S.H, tid, TNT);
    __syncthreads();
    // component 1: (P, P+1, P)
    contract<double, P, P + 1, P, 0, Q, false, P>(y + NC, S.t1, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, P + 1, P, 1, Q, false, P + 1>(S.t1, S.t2, S.L, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, P, 2, Q, false, P>(S.t2, S.u[1], S.H, tid, TNT);
    __syncthreads();
    // component 2: (P, P, P+1)
    contract<double, P, P, P + 1, 0, Q, false, P>(y + 2 * NC, S.t1, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, P, P + 1, 1, Q, false, P>(S.t1, S.t2, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, P + 1, 2, Q, false, P + 1>(S.t2, S.u[2], S.L, tid, TNT);
    __syncthreads();
    for (int q = tid; q < Q3; q += TNT) {
        const double a0 = S.u[0][q], a1 = S.u[1][q], a2 = S.u[2][q];
        S.u[0][q] = S.G[0][q] * a0 + S.G[1][q] * a1 + S.G[2][q] * a2;
        S.u[1][q] = S.G[1][q] * a0 + S.G[3][q] * a1 + S.G[4][q] * a2;
        S.u[2][q] = S.G[2][q] * a0 + S.G[4][q] * a1 + S.G[5][q] * a2;
    }
    __syncthreads();
    contract<double, Q, Q, Q, 2, P, true, P>(S.u[0], S.t1, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, P, 1, P, true, P>(S.t1, S.t2, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, P, P, 0, P + 1, true, P + 1>(S.t2, y, S.L, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, Q, 2, P, true, P>(S.u[1], S.t1, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, P, 1, P + 1, true, P + 1>(S.t1, S.t2, S.L, tid, TNT);
    __syncthreads();
    contract<double, Q, P + 1, P, 0, P, true, P>(S.t2, y + NC, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, Q, 2, P + 1, true, P + 1>(S.u[2], S.t1, S.L, tid, TNT);
    __syncthreads();
    contract<double, Q, Q, P + 1, 1, P, true, P>(S.t1, S.t2, S.H, tid, TNT);
    __syncthreads();
    contract<double, Q, P, P + 1, 0, P, true, P>(S.t2, y + 2 * NC, S.H, tid, TNT);
    __syncthreads();
    for (int d = tid; d < NRT; d += TNT) y[d] *= S.dh[d];
    __syncthreads();
}

// deterministic start vector entry in [0.5, 1.5]
__device__ __forceinline__ double start_entry(int d) {
    uint64_t z = (uint64_t)(d + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return 1.0 + ((double)(z >> 11) * 0x1.0p-53 - 0.5);
}

// number of eigenvalues of the tridiagonal (a, b) below x (Sturm sequence)
__device__ int sturm_count(const double* a, const double* b, int k, double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < k; ++i) {
        if (q == 0.0) q = 1e-300;
        q = a[i] - x - b[i] * b[i] / q;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// eigenvalue number `which` (0 = smallest, k-1 = largest) by bisection
__device__ double tri_eig(const double* a, const double* b, int k, int which) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < k ? fabs(b[i + 1]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, k, mid) > which) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// unit eigenvector z of the tridiagonal at eigenvalue lam (inverse iteration)
__device__ void tri_vec(const double* a, const double* b, int k, double lam, double* z) {
    double scale = 0.0;
    for (int i = 0; i < k; ++i) scale = fmax(scale, fabs(a[i]) + fabs(b[i]) + (i + 1 < k ? fabs(b[i + 1]) : 0.0));
    const double tiny = 1e-14 * scale;
    double dpiv[KLAN], rhs[KLAN];
    for (int i = 0; i < k; ++i) z[i] = 1.0;
    for (int rep = 0; rep < 3; ++rep) {
        // LDL^T-style elimination of (T - lam I) z_new = z
        for (int i = 0; i < k; ++i) rhs[i] = z[i];
        double dprev = 0.0;
        for (int i = 0; i < k; ++i) {
            double d = a[i] - lam;
            if (i > 0) {
                const double l = b[i] / dprev;
                d -= l * b[i];
                rhs[i] -= l * rhs[i - 1];
            }
            if (fabs(d) < tiny) d = d < 0 ? -tiny : tiny;
            dpiv[i] = d;
            dprev = d;
        }
        z[k - 1] = rhs[k - 1] / dpiv[k - 1];
        for (int i = k - 2; i >= 0; --i) z[i] = (rhs[i] - b[i + 1] * z[i + 1]) / dpiv[i];
        double n2 = 0.0;
        for (int i = 0; i < k; ++i) n2 += z[i] * z[i];
        const double inv = 1.0 / sqrt(n2);
        for (int i = 0; i < k; ++i) z[i] *= inv;
    }
}

// Lanczos on D^{-1/2} M_e D^{-1/2}.  accumulate = false: fills alpha, beta,
// the step count sc[0] and the extreme eigenvalues sc[1], sc[2] and, when
// vectors, the eigenvectors zlo, zhi of the tridiagonal.  accumulate = true:
// repeats the same run and forms the Ritz vectors ylo, yhi.
template <int P>
__device__ void lanczos(TgtLDS<P>& S, bool accumulate, bool vectors, int tid) {
    constexpr int NRT = TgtLDS<P>::NRT;
    constexpr int KMAX = NRT < KLAN ? NRT : KLAN;
    double acc = 0.0;
    for (int d = tid; d < NRT; d += TNT) {
        const double s = start_entry(d);
        S.v[d] = s;
        S.vprev[d] = 0.0;
        acc += s * s;
        if (accumulate) S.ylo[d] = S.yhi[d] = 0.0;
    }
    const double inv0 = 1.0 / sqrt(block_sum(acc, S.red, 0));
    for (int d = tid; d < NRT; d += TNT) S.v[d] *= inv0;
    const int kstop = accumulate ? (int)S.sc[0] : KMAX;
    double bj = 0.0;
    int k = kstop;
    for (int j = 0; j < kstop; ++j) {
        if (accumulate) {
            const double cl = S.zlo[j], ch = S.zhi[j];
            for (int d = tid; d < NRT; d += TNT) {
                S.ylo[d] += cl * S.v[d];
                S.yhi[d] += ch * S.v[d];
            }
            if (j + 1 == kstop) break;
        }
        if constexpr (TgtLDS<P>::FULL) {
            for (int d = tid; d < NRT; d += TNT) S.basis[j * NRT + d] = S.v[d];
        }
        __syncthreads();
        scaled_mass<P>(S, S.v, S.w, tid);
        double pa = 0.0;
        for (int d = tid; d < NRT; d += TNT) pa += S.w[d] * S.v[d];
        const double aj = block_sum(pa, S.red, 1);
        double pc = 0.0;
        for (int d = tid; d < NRT; d += TNT) {
            const double wd = S.w[d] - aj * S.v[d] - bj * S.vprev[d];
            S.w[d] = wd;
            pc += wd * S.v[d];
        }
        // one local re-orthogonalisation against v_j
        const double cj = block_sum(pc, S.red, 2);
        for (int d = tid; d < NRT; d += TNT) S.w[d] -= cj * S.v[d];
        if constexpr (TgtLDS<P>::FULL) {
            // classical Gram-Schmidt against v_0 .. v_j, twice
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) {
                    double h = 0.0;
                    for (int d = tid; d < NRT; d += TNT) h += S.w[d] * S.basis[i * NRT + d];
                    for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
                    if ((tid & 63) == 0) S.hred[tid / 64][i] = h;
                }
                __syncthreads();
                for (int d = tid; d < NRT; d += TNT) {
                    double corr = 0.0;
                    for (int i = 0; i <= j; ++i) {
                        double h = 0.0;
#pragma unroll
                        for (int wv = 0; wv < TNT / 64; ++wv) h += S.hred[wv][i];
                        corr += h * S.basis[i * NRT + d];
                    }
                    S.w[d] -= corr;
                }
                __syncthreads();
            }
        }
        double pn = 0.0;
        for (int d = tid; d < NRT; d += TNT) pn += S.w[d] * S.w[d];
        const double bn = sqrt(block_sum(pn, S.red, 3));
        if (!accumulate && tid == 0) {
            S.alpha[j] = aj + cj;
            S.beta[j + 1] = bn;
        }
        bool last = j + 1 == KMAX || !(bn > 1e-12 * (fabs(aj) + bj));
        if (!accumulate && !last && (j + 1) % KCHECK == 0) {
            // residual bounds of the extreme Ritz pairs of the current tridiagonal
            if (tid == 0) {
                const int kk = j + 1;
                S.beta[0] = 0.0;
                const double lo = tri_eig(S.alpha, S.beta, kk, 0);
                const double hi = tri_eig(S.alpha, S.beta, kk, kk - 1);
                tri_vec(S.alpha, S.beta, kk, lo, S.zlo);
                tri_vec(S.alpha, S.beta, kk, hi, S.zhi);
                const double rl = bn * fabs(S.zlo[kk - 1]), rh = bn * fabs(S.zhi[kk - 1]);
                S.flag[1] = (rl <= RITZ_TOL * lo && rh <= RITZ_TOL * lo) ? 1 : 0;
            }
            __syncthreads();
            last = S.flag[1] != 0;
            __syncthreads();
        }
        if (!accumulate && last) {
            k = j + 1;
            break;
        }
        const double ib = 1.0 / bn;
        for (int d = tid; d < NRT; d += TNT) {
            S.vprev[d] = S.v[d];
            S.v[d] = S.w[d] * ib;
        }
        bj = bn;
    }
    __syncthreads();
    if (!accumulate) {
        if (tid == 0) {
            S.beta[0] = 0.0;
            S.sc[0] = k;
            S.sc[1] = tri_eig(S.alpha, S.beta, k, 0);
            S.sc[2] = tri_eig(S.alpha, S.beta, k, k - 1);
            if (vectors) {
                tri_vec(S.alpha, S.beta, k, S.sc[1], S.zlo);
                tri_vec(S.alpha, S.beta, k, S.sc[2], S.zhi);
            }
        }
        __syncthreads();
    } else {
        // normalise the Ritz vectors
        double a = 0.0, b = 0.0;
        for (int d = tid; d < NRT; d += TNT) {
            a += S.ylo[d] * S.ylo[d];
            b += S.yhi[d] * S.yhi[d];
        }
        const double ia = 1.0 / sqrt(block_sum(a, S.red, 4));
        const double ib = 1.0 / sqrt(block_sum(b, S.red, 5));
        for (int d = tid; d < NRT; d += TNT) {
            S.ylo[d] *= ia;
            S.yhi[d] *= ib;
        }
        __syncthreads();
    }
}

// spread f(theta) (sc[3]) and, when grad, its gradient g; theta in LDS
template <int P>
__device__ void spread_eval(TgtLDS<P>& S, const double* theta, bool grad, int tid) {
    constexpr int NRT = TgtLDS<P>::NRT;
    for (int d = tid; d < NRT; d += TNT) {
        int c;
        double alo, ahi;
        dof_weight<P>(S, d, c, alo, ahi);
        S.dh[d] = 1.0 / sqrt(S.m[d] * exp(alo * theta[2 * c] + ahi * theta[2 * c + 1]));
    }
    __syncthreads();
    lanczos<P>(S, false, grad, tid);
    if (tid == 0) S.sc[3] = log(S.sc[2]) - log(S.sc[1]);
    if (!grad) {
        __syncthreads();
        return;
    }
    if constexpr (TgtLDS<P>::FULL) {
        // Ritz vectors from the stored basis
        const int k = (int)S.sc[0];
        double a = 0.0, b = 0.0;
        for (int d = tid; d < NRT; d += TNT) {
            double yl = 0.0, yh = 0.0;
            for (int j = 0; j < k; ++j) {
                yl += S.zlo[j] * S.basis[j * NRT + d];
                yh += S.zhi[j] * S.basis[j * NRT + d];
            }
            S.ylo[d] = yl;
            S.yhi[d] = yh;
            a += yl * yl;
            b += yh * yh;
        }
        const double ia = 1.0 / sqrt(block_sum(a, S.red, 4));
        const double ib = 1.0 / sqrt(block_sum(b, S.red, 5));
        for (int d = tid; d < NRT; d += TNT) {
            S.ylo[d] *= ia;
            S.yhi[d] *= ib;
        }
        __syncthreads();
    } else {
        lanczos<P>(S, true, true, tid);
    }
    double gl[6] = {0, 0, 0, 0, 0, 0};
    for (int d = tid; d < NRT; d += TNT) {
        int c;
        double alo, ahi;
        dof_weight<P>(S, d, c, alo, ahi);
        const double r = S.ylo[d] * S.ylo[d] - S.yhi[d] * S.yhi[d];
        gl[2 * c] += r * alo;
        gl[2 * c + 1] += r * ahi;
    }
    for (int j = 0; j < 6; ++j) {
        const double s = block_sum(gl[j], S.red, j);
        if (tid == 0) S.g[j] = s;
    }
    __syncthreads();
}

template <int P>
__global__ __launch_bounds__(TNT) void target_kernel(int64_t n, const double* __restrict__ verts,
                                                     const Tables<double>* __restrict__ tab, int max_steps,
                                                     double* __restrict__ theta_out, double* __restrict__ lam_out,
                                                     double* __restrict__ spread_out) {
    constexpr int Q = P + 1, Q3 = Q * Q * Q, NC = TgtLDS<P>::NC;
    __shared__ TgtLDS<P> S;
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    if (e >= n) return;
    for (int i = tid; i < Q * (P + 1); i += TNT) {
        S.L[i] = tab->L[i / (P + 1)][i % (P + 1)];
        S.L2[i] = tab->L2[i / (P + 1)][i % (P + 1)];
    }
    for (int i = tid; i < Q * P; i += TNT) {
        S.H[i] = tab->H[i / P][i % P];
        S.H2[i] = tab->H2[i / P][i % P];
    }
    for (int i = tid; i <= P; i += TNT) S.gll[i] = tab->gll[i];
    for (int i = tid; i < 24; i += TNT) S.X[i] = verts[e * 24 + i];
    if (tid == 0) S.flag[0] = 0;
    __syncthreads();
    // geometric factors w J^T J / det J (unit coefficient) at the Gauss points
    for (int pt = tid; pt < Q3; pt += TNT) {
        const int a = pt % Q, b = (pt / Q) % Q, cq = pt / (Q * Q);
        const double xi0 = tab->xq[a], xi1 = tab->xq[b], xi2 = tab->xq[cq];
        const double wgt = tab->wq[a] * tab->wq[b] * tab->wq[cq];
        double J[3][3];
        for (int r = 0; r < 3; ++r) {
            double s0 = 0, s1 = 0, s2 = 0;
            for (int v = 0; v < 8; ++v) {
                const int dx = v & 1, dy = (v >> 1) & 1, dz = (v >> 2) & 1;
                const double Nx = dx ? xi0 : 1.0 - xi0, Ny = dy ? xi1 : 1.0 - xi1, Nz = dz ? xi2 : 1.0 - xi2;
                const double Xv = S.X[(dz * 4 + dy * 2 + dx) * 3 + r];
                s0 += (dx ? 1.0 : -1.0) * Ny * Nz * Xv;
                s1 += Nx * (dy ? 1.0 : -1.0) * Nz * Xv;
                s2 += Nx * Ny * (dz ? 1.0 : -1.0) * Xv;
            }
            J[r][0] = s0;
            J[r][1] = s1;
            J[r][2] = s2;
        }
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det > 0.0)) S.flag[0] = 1;
        const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
        for (int m = 0; m < 6; ++m) {
            double s = 0;
            for (int r = 0; r < 3; ++r) s += J[r][rr[m]] * J[r][cc[m]];
            S.G[m][pt] = wgt * s / det;
        }
    }
    __syncthreads();
    if (S.flag[0]) {
        if (tid < 6) theta_out[e * 6 + tid] = NAN;
        if (lam_out && tid < 2) lam_out[e * 2 + tid] = NAN;
        if (spread_out && tid < 2) spread_out[e * 2 + tid] = NAN;
        return;
    }
    // diag(M_e): squared-basis contractions of G_cc
    const int gc[3] = {0, 3, 5};
    for (int c = 0; c < 3; ++c) {
        double* out = S.m + c * NC;
        if (c == 0) {
            contract<double, Q, Q, Q, 2, P, true, P>(S.G[gc[c]], S.t1, S.H2, tid, TNT);
            __syncthreads();
            contract<double, Q, Q, P, 1, P, true, P>(S.t1, S.t2, S.H2, tid, TNT);
            __syncthreads();
            contract<double, Q, P, P, 0, P + 1, true, P + 1>(S.t2, out, S.L2, tid, TNT);
        } else if (c == 1) {
            contract<double, Q, Q, Q, 2, P, true, P>(S.G[gc[c]], S.t1, S.H2, tid, TNT);
            __syncthreads();
            contract<double, Q, Q, P, 1, P + 1, true, P + 1>(S.t1, S.t2, S.L2, tid, TNT);
            __syncthreads();
            contract<double, Q, P + 1, P, 0, P, true, P>(S.t2, out, S.H2, tid, TNT);
        } else {
            contract<double, Q, Q, Q, 2, P + 1, true, P + 1>(S.G[gc[c]], S.t1, S.L2, tid, TNT);
            __syncthreads();
            contract<double, Q, Q, P + 1, 1, P, true, P>(S.t1, S.t2, S.H2, tid, TNT);
            __syncthreads();
            contract<double, Q, P, P + 1, 0, P, true, P>(S.t2, out, S.H2, tid, TNT);
        }
        __syncthreads();
    }
    // projected gradient descent on sum(theta) = 0
    if (tid < 6) S.theta[tid] = 0.0;
    __syncthreads();
    spread_eval<P>(S, S.theta, true, tid);
    double f = S.sc[3];
    const double f0 = f;
    double lo = S.sc[1], hi = S.sc[2];
    double eta = 1.0;
    for (int step = 0; step < max_steps; ++step) {
        double pg[6], mean = 0.0, gg = 0.0;
        for (int j = 0; j < 6; ++j) mean += S.g[j];
        mean /= 6.0;
        for (int j = 0; j < 6; ++j) {
            pg[j] = S.g[j] - mean;
            gg += pg[j] * pg[j];
        }
        if (gg <= 1e-24) break;
        bool accepted = false;
        for (int h = 0; h < 20; ++h) {
            __syncthreads();
            if (tid < 6) S.trial[tid] = S.theta[tid] - eta * pg[tid];
            __syncthreads();
            spread_eval<P>(S, S.trial, false, tid);
            if (S.sc[3] <= f - 1e-4 * eta * gg) {
                accepted = true;
                break;
            }
            eta *= 0.5;
        }
        if (!accepted) break;
        __syncthreads();
        if (tid < 6) S.theta[tid] = S.trial[tid];
        __syncthreads();
        spread_eval<P>(S, S.theta, true, tid);
        f = S.sc[3];
        lo = S.sc[1];
        hi = S.sc[2];
        eta = fmin(2.0 * eta, 4.0);
    }
    if (tid < 6) theta_out[e * 6 + tid] = S.theta[tid];
    if (lam_out && tid == 0) {
        lam_out[e * 2] = lo;
        lam_out[e * 2 + 1] = hi;
    }
    if (spread_out && tid == 0) {
        spread_out[e * 2] = f0;
        spread_out[e * 2 + 1] = f;
    }
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
// x[e] from the element's vertices [24] (vertex (dx, dy, dz) at
// (dz * 4 + dy * 2 + dx) * 3), alpha, beta and p
__device__ void element_features(const double* V, double alpha, double beta, int p, float* x) {
    double c[3] = {0, 0, 0};
    for (int v = 0; v < 8; ++v)
        for (int r = 0; r < 3; ++r) c[r] += 0.125 * V[v * 3 + r];
    double h = 0.0;
    for (int v = 0; v < 8; ++v)
        for (int bit = 1; bit < 8; bit <<= 1) {
            const int u = v | bit;
            if (u == v) continue;
            double d2 = 0.0;
            for (int r = 0; r < 3; ++r) {
                const double d = V[u * 3 + r] - V[v * 3 + r];
                d2 += d * d;
            }
            h += sqrt(d2);
        }
    h /= 12.0;
    for (int v = 0; v < 8; ++v)
        for (int r = 0; r < 3; ++r) x[v * 3 + r] = (float)((V[v * 3 + r] - c[r]) / h);
    x[24] = (float)log(alpha);
    x[25] = (float)log(beta);
    x[26] = (float)(p / 6.0);
}

__global__ void features_kernel(int64_t n, const double* __restrict__ verts, const double* __restrict__ alpha,
                                const double* __restrict__ beta, const int* __restrict__ parr, int pconst,
                                float* __restrict__ X) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    element_features(verts + e * 24, alpha[e], beta[e], parr ? parr[e] : pconst, X + e * NIN);
}

// features of the elements of the structured mesh: vertices gathered from
// the grid, alpha = 1 / kappa (1 where kappa = 0), beta = c_mass
__global__ void mesh_features_kernel(int nx, int ny, int nz, int p, const double* __restrict__ vert,
                                     const double* __restrict__ cm, const double* __restrict__ kap,
                                     float* __restrict__ X) {
    const int64_t ne = (int64_t)nx * ny * nz;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((int64_t)nx * ny));
    double V[24];
    for (int v = 0; v < 8; ++v) {
        const int dx = v & 1, dy = (v >> 1) & 1, dz = (v >> 2) & 1;
        const int64_t g = (ex + dx) + (int64_t)(nx + 1) * ((ey + dy) + (int64_t)(ny + 1) * (ez + dz));
        for (int r = 0; r < 3; ++r) V[v * 3 + r] = vert[3 * g + r];
    }
    const double k = kap[e];
    element_features(V, k > 0.0 ? 1.0 / k : 1.0, cm[e], p, X + e * NIN);
}

// ---------------------------------------------------------------------------
// network, FP32
// ---------------------------------------------------------------------------
// clip to +-ln 4; a NaN stays NaN (fminf / fmaxf would replace it by a
// bound), so that a broken network is detected and the plain diagonal used
__device__ __forceinline__ float clip_ln4(float o) {
    return o != o ? o : fminf(fmaxf(o, -(float)LN4), (float)LN4);
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_df(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// one 64-thread block per row: z1, a1, z2, a2, o (stores optional)
__global__ __launch_bounds__(64) void mlp_forward_kernel(int64_t n, const float* __restrict__ X,
                                                         const int* __restrict__ idx, const float* __restrict__ prm,
                                                         float* __restrict__ Z1, float* __restrict__ A1,
                                                         float* __restrict__ Z2, float* __restrict__ A2,
                                                         float* __restrict__ O, int clip) {
    __shared__ float x[NIN], a1[NHID], a2[NHID];
    const int j = threadIdx.x;
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        const int64_t src = idx ? idx[r] : r;
        __syncthreads();
        if (j < NIN) x[j] = X[src * NIN + j];
        __syncthreads();
        float z = prm[OFF_B1 + j];
        for (int k = 0; k < NIN; ++k) z += prm[OFF_W1 + j * NIN + k] * x[k];
        const float h1 = gelu_f(z);
        a1[j] = h1;
        if (Z1) {
            Z1[r * NHID + j] = z;
            A1[r * NHID + j] = h1;
        }
        __syncthreads();
        z = prm[OFF_B2 + j];
        for (int k = 0; k < NHID; ++k) z += prm[OFF_W2 + j * NHID + k] * a1[k];
        const float h2 = gelu_f(z);
        a2[j] = h2;
        if (Z2) {
            Z2[r * NHID + j] = z;
            A2[r * NHID + j] = h2;
        }
        __syncthreads();
        if (j < NOUT) {
            float o = prm[OFF_B3 + j];
            for (int k = 0; k < NHID; ++k) o += prm[OFF_W3 + j * NHID + k] * a2[k];
            if (clip) o = clip_ln4(o);
            O[r * NOUT + j] = o;
        }
    }
}

// dO = 2 (o - clip(y)) / (n * 6); per-block partial sums of the squared error
__global__ void mlp_loss_kernel(int64_t n, const float* __restrict__ O, const float* __restrict__ Y,
                                const int* __restrict__ idx, float* __restrict__ dO, double* __restrict__ part) {
    __shared__ double s[256];
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (r < n) {
        const int64_t src = idx ? idx[r] : r;
        for (int j = 0; j < NOUT; ++j) {
            const float t = fminf(fmaxf(Y[src * NOUT + j], -(float)LN4), (float)LN4);
            const float d = O[r * NOUT + j] - t;
            acc += (double)d * d;
            dO[r * NOUT + j] = 2.0f * d / (float)(n * NOUT);
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// per row: dZ2 = (W3^T dO) * gelu'(Z2), dZ1 = (W2^T dZ2) * gelu'(Z1)
__global__ __launch_bounds__(64) void mlp_backward_rows_kernel(int64_t n, const float* __restrict__ dO,
                                                               const float* __restrict__ Z1,
                                                               const float* __restrict__ Z2,
                                                               const float* __restrict__ prm, float* __restrict__ dZ1,
                                                               float* __restrict__ dZ2) {
    __shared__ float go[NOUT], g2[NHID];
    const int j = threadIdx.x;
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        __syncthreads();
        if (j < NOUT) go[j] = dO[r * NOUT + j];
        __syncthreads();
        float s = 0.0f;
        for (int i = 0; i < NOUT; ++i) s += prm[OFF_W3 + i * NHID + j] * go[i];
        const float d2 = s * gelu_df(Z2[r * NHID + j]);
        dZ2[r * NHID + j] = d2;
        g2[j] = d2;
        __syncthreads();
        s = 0.0f;
        for (int i = 0; i < NHID; ++i) s += prm[OFF_W2 + i * NHID + j] * g2[i];
        dZ1[r * NHID + j] = s * gelu_df(Z1[r * NHID + j]);
    }
}

// one thread per parameter: sums over the rows of the batch (fixed order)
__global__ void mlp_grad_kernel(int64_t n, const float* __restrict__ X, const int* __restrict__ idx,
                                const float* __restrict__ A1, const float* __restrict__ A2,
                                const float* __restrict__ dZ1, const float* __restrict__ dZ2,
                                const float* __restrict__ dO, float* __restrict__ grad) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NPARAM) return;
    double s = 0.0;
    if (t < OFF_B1) {
        const int i = t / NIN, k = t % NIN;
        for (int64_t r = 0; r < n; ++r) s += (double)dZ1[r * NHID + i] * X[(idx ? idx[r] : r) * NIN + k];
    } else if (t < OFF_W2) {
        const int i = t - OFF_B1;
        for (int64_t r = 0; r < n; ++r) s += dZ1[r * NHID + i];
    } else if (t < OFF_B2) {
        const int i = (t - OFF_W2) / NHID, k = (t - OFF_W2) % NHID;
        for (int64_t r = 0; r < n; ++r) s += (double)dZ2[r * NHID + i] * A1[r * NHID + k];
    } else if (t < OFF_W3) {
        const int i = t - OFF_B2;
        for (int64_t r = 0; r < n; ++r) s += dZ2[r * NHID + i];
    } else if (t < OFF_B3) {
        const int i = (t - OFF_W3) / NHID, k = (t - OFF_W3) % NHID;
        for (int64_t r = 0; r < n; ++r) s += (double)dO[r * NOUT + i] * A2[r * NHID + k];
    } else {
        const int i = t - OFF_B3;
        for (int64_t r = 0; r < n; ++r) s += dO[r * NOUT + i];
    }
    grad[t] = (float)s;
}

__global__ void adam_kernel(float* __restrict__ prm, const float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, float lr, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NPARAM) return;
    const float g = grad[t];
    const float mt = 0.9f * m[t] + 0.1f * g;
    const float vt = 0.999f * v[t] + 0.001f * g * g;
    m[t] = mt;
    v[t] = vt;
    prm[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + 1e-8f);
}

// ---------------------------------------------------------------------------
// network, BF16 inference on the matrix cores
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(u >> 16);
}

// One wavefront per workgroup, 16 rows per tile.  A (activations, M x K) and
// B (weights, K x N) fragments of v_mfma_f32_16x16x16_bf16: lane l holds
// row / column l % 16 and k = 4 (l / 16) .. + 3; the accumulator holds column
// l % 16 and rows 4 (l / 16) .. + 3.
__global__ __launch_bounds__(64) void mlp_infer_bf16_kernel(int64_t n, const float* __restrict__ X,
                                                            const float* __restrict__ prm,
                                                            float* __restrict__ theta) {
    __shared__ unsigned short W1b[NHID][32], W2b[NHID][NHID], W3b[16][NHID];
    __shared__ float b1[NHID], b2[NHID], b3[16];
    __shared__ unsigned short Xb[16][32], H1[16][NHID], H2[16][NHID];
    const int lane = threadIdx.x;
    for (int i = lane; i < NHID * 32; i += 64) {
        const int j = i / 32, k = i % 32;
        W1b[j][k] = k < NIN ? to_bf16(prm[OFF_W1 + j * NIN + k]) : 0;
    }
    for (int i = lane; i < NHID * NHID; i += 64) W2b[i / NHID][i % NHID] = to_bf16(prm[OFF_W2 + i]);
    for (int i = lane; i < 16 * NHID; i += 64) {
        const int j = i / NHID, k = i % NHID;
        W3b[j][k] = j < NOUT ? to_bf16(prm[OFF_W3 + j * NHID + k]) : 0;
    }
    b1[lane] = prm[OFF_B1 + lane];
    b2[lane] = prm[OFF_B2 + lane];
    if (lane < 16) b3[lane] = lane < NOUT ? prm[OFF_B3 + lane] : 0.0f;
    const int col = lane % 16, kq = lane / 16;
    for (int64_t tile = blockIdx.x; tile * 16 < n; tile += gridDim.x) {
        const int64_t r0 = tile * 16;
        __syncthreads();
        for (int i = lane; i < 16 * 32; i += 64) {
            const int r = i / 32, k = i % 32;
            Xb[r][k] = (k < NIN && r0 + r < n) ? to_bf16(X[(r0 + r) * NIN + k]) : 0;
        }
        __syncthreads();
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int ks = 0; ks < 2; ++ks) {
                bf16x4 a, b;
                for (int i = 0; i < 4; ++i) {
                    a[i] = (short)Xb[col][ks * 16 + kq * 4 + i];
                    b[i] = (short)W1b[nt * 16 + col][ks * 16 + kq * 4 + i];
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
            }
            for (int i = 0; i < 4; ++i) H1[kq * 4 + i][nt * 16 + col] = to_bf16(gelu_f(acc[i] + b1[nt * 16 + col]));
        }
        __syncthreads();
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int ks = 0; ks < 4; ++ks) {
                bf16x4 a, b;
                for (int i = 0; i < 4; ++i) {
                    a[i] = (short)H1[col][ks * 16 + kq * 4 + i];
                    b[i] = (short)W2b[nt * 16 + col][ks * 16 + kq * 4 + i];
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
            }
            for (int i = 0; i < 4; ++i) H2[kq * 4 + i][nt * 16 + col] = to_bf16(gelu_f(acc[i] + b2[nt * 16 + col]));
        }
        __syncthreads();
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int ks = 0; ks < 4; ++ks) {
            bf16x4 a, b;
            for (int i = 0; i < 4; ++i) {
                a[i] = (short)H2[col][ks * 16 + kq * 4 + i];
                b[i] = (short)W3b[col][ks * 16 + kq * 4 + i];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + kq * 4 + i;
            if (col < NOUT && r < n) {
                const float o = acc[i] + b3[col];
                theta[r * NOUT + col] = clip_ln4(o);
            }
        }
    }
}

__global__ void theta_widen_kernel(int64_t n, const float* __restrict__ t32, double* __restrict__ t64,
                                   int* __restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = t32[i];
    if (!isfinite(v) || fabsf(v) > (float)LN4 * 1.0001f) *bad = 1;
    t64[i] = (double)v;
}

template <int P>
void launch_targets_p(hd_ctx* c, int64_t n, const double* verts, const Tables<double>* tab, int steps, double* th,
                      double* lam, double* spr) {
    hipLaunchKernelGGL((target_kernel<P>), dim3((unsigned)n), dim3(TNT), 0, c->stream, n, verts, tab, steps, th, lam,
                       spr);
}

unsigned grid_rows(int64_t n) { return (unsigned)std::min<int64_t>(n, 65536); }

struct MlpWork {
    int64_t cap = 0;
    float *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *O = nullptr, *dO = nullptr, *dZ1 = nullptr,
          *dZ2 = nullptr, *grad = nullptr;
    double* part = nullptr;
    int* idx = nullptr;
    ~MlpWork() {
        for (float* p : {Z1, A1, Z2, A2, O, dO, dZ1, dZ2, grad}) dfree(p);
        dfree(part);
        dfree(idx);
    }
    bool alloc(int64_t n) {
        cap = n;
        Z1 = dalloc<float>(n * NHID);
        A1 = dalloc<float>(n * NHID);
        Z2 = dalloc<float>(n * NHID);
        A2 = dalloc<float>(n * NHID);
        O = dalloc<float>(n * NOUT);
        dO = dalloc<float>(n * NOUT);
        dZ1 = dalloc<float>(n * NHID);
        dZ2 = dalloc<float>(n * NHID);
        grad = dalloc<float>(NPARAM);
        part = dalloc<double>((n + 255) / 256);
        idx = dalloc<int>(n);
        return Z1 && A1 && Z2 && A2 && O && dO && dZ1 && dZ2 && grad && part && idx;
    }
};

// loss of the rows (idx or all) and the gradient in w.grad; returns the
// partial-sum count in *nparts (loss = sum of part / (n * 6))
int loss_grad(hd_ctx* c, MlpWork& w, int64_t n, const float* X, const float* Y, const int* idx, int64_t* nparts) {
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid_rows(n)), dim3(64), 0, c->stream, n, X, idx, c->d_mlp, w.Z1,
                       w.A1, w.Z2, w.A2, w.O, 0);
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(nb), dim3(256), 0, c->stream, n, w.O, Y, idx, w.dO, w.part);
    hipLaunchKernelGGL(mlp_backward_rows_kernel, dim3(grid_rows(n)), dim3(64), 0, c->stream, n, w.dO, w.Z1, w.Z2,
                       c->d_mlp, w.dZ1, w.dZ2);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, c->stream, n, X, idx, w.A1, w.A2,
                       w.dZ1, w.dZ2, w.dO, w.grad);
    HD_HIP(c, hipGetLastError());
    *nparts = nb;
    return HD_OK;
}

int ensure_mlp(hd_ctx* c) {
    if (!c->d_mlp) c->d_mlp = dalloc<float>(NPARAM);
    if (!c->d_adam_m) c->d_adam_m = dalloc<float>(NPARAM);
    if (!c->d_adam_v) c->d_adam_v = dalloc<float>(NPARAM);
    if (!c->d_mlp || !c->d_adam_m || !c->d_adam_v) return set_err(c, HD_ERR_OOM, "network parameters");
    return HD_OK;
}

int reset_adam(hd_ctx* c) {
    std::vector<float> z(NPARAM, 0.0f);
    HD_HIP(c, hipMemcpyAsync(c->d_adam_m, z.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemcpyAsync(c->d_adam_v, z.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    c->adam_t = 0;
    return HD_OK;
}

double sum_host(const std::vector<double>& v) {
    double s = 0.0;
    for (double x : v) s += x;
    return s;
}

}  // namespace

int mlp_param_count() { return NPARAM; }

int launch_targets(hd_ctx* c, int p, int64_t n, const double* verts, int steps, double* th, double* lam,
                   double* spr) {
    Tables<double> t64;
    Tables<float> t32;
    build_tables(p, t64, t32);
    Tables<double>* dt = dalloc<Tables<double>>(1);
    if (!dt) return set_err(c, HD_ERR_OOM, "tables");
    int rc = HD_OK;
    if (hipMemcpyAsync(dt, &t64, sizeof(t64), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        rc = set_err(c, HD_ERR_HIP, "table upload");
    // bounded launches keep the grid within limits for any n
    const int64_t chunk = 1 << 20;
    for (int64_t s = 0; s < n && !rc; s += chunk) {
        const int64_t m = std::min(chunk, n - s);
        switch (p) {
            case 1: launch_targets_p<1>(c, m, verts + s * 24, dt, steps, th + s * 6, lam ? lam + s * 2 : nullptr, spr ? spr + s * 2 : nullptr); break;
            case 2: launch_targets_p<2>(c, m, verts + s * 24, dt, steps, th + s * 6, lam ? lam + s * 2 : nullptr, spr ? spr + s * 2 : nullptr); break;
            case 3: launch_targets_p<3>(c, m, verts + s * 24, dt, steps, th + s * 6, lam ? lam + s * 2 : nullptr, spr ? spr + s * 2 : nullptr); break;
            case 4: launch_targets_p<4>(c, m, verts + s * 24, dt, steps, th + s * 6, lam ? lam + s * 2 : nullptr, spr ? spr + s * 2 : nullptr); break;
            case 5: launch_targets_p<5>(c, m, verts + s * 24, dt, steps, th + s * 6, lam ? lam + s * 2 : nullptr, spr ? spr + s * 2 : nullptr); break;
            case 6: launch_targets_p<6>(c, m, verts + s * 24, dt, steps, th + s * 6, lam ? lam + s * 2 : nullptr, spr ? spr + s * 2 : nullptr); break;
            default: rc = set_err(c, HD_ERR_ARG, "p out of range");
        }
        if (!rc && hipGetLastError() != hipSuccess) rc = set_err(c, HD_ERR_HIP, "target kernel launch");
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && !rc) rc = set_err(c, HD_ERR_HIP, "target kernel");
    dfree(dt);
    return rc;
}

int launch_features(hd_ctx* c, int64_t n, const double* verts, const double* alpha, const double* beta,
                    const int* parr, int p, float* X) {
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, verts, alpha,
                       beta, parr, p, X);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int mlp_init(hd_ctx* c, uint64_t seed) {
    int rc = ensure_mlp(c);
    if (rc) return rc;
    // W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b = 0
    std::mt19937_64 gen(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    std::vector<float> h(NPARAM, 0.0f);
    const float s1 = 1.0f / std::sqrt((float)NIN), s2 = 1.0f / std::sqrt((float)NHID);
    for (int i = 0; i < NHID * NIN; ++i) h[OFF_W1 + i] = (float)(s1 * U(gen));
    for (int i = 0; i < NHID * NHID; ++i) h[OFF_W2 + i] = (float)(s2 * U(gen));
    for (int i = 0; i < NOUT * NHID; ++i) h[OFF_W3 + i] = (float)(s2 * U(gen));
    HD_HIP(c, hipMemcpyAsync(c->d_mlp, h.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream));
    if ((rc = reset_adam(c))) return rc;
    c->mlp_ready = true;
    return HD_OK;
}

int mlp_set(hd_ctx* c, const float* host) {
    int rc = ensure_mlp(c);
    if (rc) return rc;
    HD_HIP(c, hipMemcpyAsync(c->d_mlp, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream));
    if ((rc = reset_adam(c))) return rc;
    c->mlp_ready = true;
    return HD_OK;
}

int mlp_get(hd_ctx* c, float* host) {
    if (!c->mlp_ready) return set_err(c, HD_ERR_STATE, "no network parameters");
    HD_HIP(c, hipMemcpyAsync(host, c->d_mlp, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

int mlp_loss_grad(hd_ctx* c, int64_t n, const float* X, const float* Y, float* loss, float* grad) {
    if (!c->mlp_ready) return set_err(c, HD_ERR_STATE, "no network parameters");
    MlpWork w;
    if (!w.alloc(n)) return set_err(c, HD_ERR_OOM, "network work space");
    int64_t np = 0;
    int rc = loss_grad(c, w, n, X, Y, nullptr, &np);
    if (rc) return rc;
    std::vector<double> part(np);
    HD_HIP(c, hipMemcpyAsync(part.data(), w.part, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream));
    if (grad) HD_HIP(c, hipMemcpyAsync(grad, w.grad, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    if (loss) *loss = (float)(sum_host(part) / (double)(n * NOUT));
    return HD_OK;
}

int mlp_train(hd_ctx* c, int64_t n, const float* X, const float* Y, int64_t nval, const float* Xv, const float* Yv,
              int epochs, int batch, float lr, uint64_t seed, float* train_loss, float* val_loss) {
    if (!c->mlp_ready) return set_err(c, HD_ERR_STATE, "no network parameters");
    MlpWork w;
    if (!w.alloc(std::max<int64_t>(batch, 1))) return set_err(c, HD_ERR_OOM, "network work space");
    MlpWork wv;
    if (nval > 0 && !wv.alloc(nval)) return set_err(c, HD_ERR_OOM, "network work space");
    std::mt19937_64 gen(seed);
    std::vector<int> perm(n);
    int* d_perm = dalloc<int>(n);
    if (!d_perm) return set_err(c, HD_ERR_OOM, "permutation");
    int rc = HD_OK;
    for (int ep = 0; ep < epochs && !rc; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(gen() % (uint64_t)(i + 1))]);
        if (hipMemcpyAsync(d_perm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            rc = set_err(c, HD_ERR_HIP, "permutation upload");
            break;
        }
        std::vector<std::vector<double>> parts;
        for (int64_t s = 0; s + batch <= n && !rc; s += batch) {
            int64_t np = 0;
            if ((rc = loss_grad(c, w, batch, X, Y, d_perm + s, &np))) break;
            c->adam_t += 1;
            const float c1 = 1.0f - std::pow(0.9f, (float)c->adam_t);
            const float c2 = 1.0f - std::pow(0.999f, (float)c->adam_t);
            hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, c->stream, c->d_mlp, w.grad,
                               c->d_adam_m, c->d_adam_v, lr, c1, c2);
            if (train_loss) {
                std::vector<double> part(np);
                if (hipMemcpyAsync(part.data(), w.part, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream) !=
                        hipSuccess ||
                    hipStreamSynchronize(c->stream) != hipSuccess) {
                    rc = set_err(c, HD_ERR_HIP, "loss readback");
                    break;
                }
                parts.push_back(part);
            }
        }
        if (rc) break;
        if (train_loss) {
            double s = 0.0;
            for (auto& pv : parts) s += sum_host(pv) / (double)(batch * NOUT);
            train_loss[ep] = parts.empty() ? 0.0f : (float)(s / parts.size());
        }
        if (val_loss && nval > 0) {
            int64_t np = 0;
            if ((rc = loss_grad(c, wv, nval, Xv, Yv, nullptr, &np))) break;
            std::vector<double> part(np);
            if (hipMemcpyAsync(part.data(), wv.part, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess) {
                rc = set_err(c, HD_ERR_HIP, "validation loss readback");
                break;
            }
            val_loss[ep] = (float)(sum_host(part) / (double)(nval * NOUT));
        }
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && !rc) rc = set_err(c, HD_ERR_HIP, "training");
    dfree(d_perm);
    return rc;
}

int mlp_infer(hd_ctx* c, int64_t n, const float* X, float* theta, int bf16) {
    if (!c->mlp_ready) return set_err(c, HD_ERR_STATE, "no network parameters");
    if (bf16) {
        const unsigned tiles = (unsigned)std::min<int64_t>((n + 15) / 16, 16384);
        hipLaunchKernelGGL(mlp_infer_bf16_kernel, dim3(tiles), dim3(64), 0, c->stream, n, X, c->d_mlp, theta);
    } else {
        hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid_rows(n)), dim3(64), 0, c->stream, n, X, (const int*)nullptr,
                           c->d_mlp, (float*)nullptr, (float*)nullptr, (float*)nullptr, (float*)nullptr, theta, 1);
    }
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

// theta for every mesh element from the network (BF16); *fallback = 1 when
// an output is not finite (the caller then uses the plain diagonal)
int learned_mesh_theta(hd_ctx* c, int* fallback) {
    const int64_t ne = c->ne;
    float* X = dalloc<float>(ne * NIN);
    float* t32 = dalloc<float>(ne * NOUT);
    if (!c->d_theta_net) c->d_theta_net = dalloc<double>(ne * 6);
    if (!X || !t32 || !c->d_theta_net) {
        dfree(X);
        dfree(t32);
        return set_err(c, HD_ERR_OOM, "learned features");
    }
    hipLaunchKernelGGL(mesh_features_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, c->stream, c->nx, c->ny,
                       c->nz, c->p, c->d_vert, c->d_cm, c->d_kap, X);
    int rc = mlp_infer(c, ne, X, t32, 1);
    int bad = 0;
    if (!rc) {
        if (hipMemcpyAsync(c->d_flag, &bad, sizeof(int), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            rc = set_err(c, HD_ERR_HIP, "flag");
    }
    if (!rc) {
        const int64_t nt = ne * 6;
        hipLaunchKernelGGL(theta_widen_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream, nt, t32,
                           c->d_theta_net, c->d_flag);
        if (hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            rc = set_err(c, HD_ERR_HIP, "learned scalings");
    }
    dfree(X);
    dfree(t32);
    *fallback = bad;
    return rc;
}

}  // namespace hd
