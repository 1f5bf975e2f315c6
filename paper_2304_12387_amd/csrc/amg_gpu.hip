// Smoothed-aggregation AMG set-up on the GPU for the approximate Schur
// complement S~ (an M-matrix graph Laplacian plus a diagonal, Section 2.3,
// Prop. 4 and 5; the paper sets up its AMG on the device, Section 3.2).
//
// The hierarchy is the one amg_host.cpp defines, built here with the same
// arithmetic in the same order, so that both give the same matrices bit for
// bit (floating-point contraction is off in this file: no fused multiply-add,
// since the host code has none):
//
//   strength   a_ij < 0 strong iff -a_ij >= theta min(m_i, m_j),
//              m_i = max(0, max_{k != i} -a_ik)                     (1 kernel + count/scan/fill)
//   MIS-2      keys (state, h(i), i), h = low 30 bits of splitmix64(i);
//              rounds of distance-2 maxima (3 kernels per round)
//   aggregates roots numbered in index order (scan); pass 1: neighbours of
//              roots join the root of largest (h, index); pass 2: the rest
//              join the pass-1 neighbour of largest (h, index)
//   P          (I - omega D_F^{-1} A_F) T, weak entries lumped to the
//              diagonal; one wavefront per row
//   A P, P^T (A P)
//              row-wise products, one wavefront per output row: the
//              candidate columns (the rows of the right factor selected by
//              the row of the left factor) are sorted in LDS, duplicates
//              dropped, then every distinct column sums its products in the
//              order of the left row (the order of Gustavson's algorithm)
//   A_c        (P^T A P + (P^T A P)^T) / 2
//   coarsest   Gauss-Jordan inverse with partial pivoting, one kernel per
//              pivot step
//
// Every step is deterministic: no floating-point atomics, transposes sort
// their rows.
#include <algorithm>
#include <vector>

#include "hd_internal.hpp"

// products and sums stay separately rounded in this file (no fused
// multiply-add), like the host code it must match
#pragma clang fp contract(off)

namespace hd {

namespace {

constexpr int BSA = 256;
inline unsigned nbk(int64_t n, int bs = BSA) { return (unsigned)((n + bs - 1) / bs); }

constexpr uint32_t ST_OUT = 0, ST_UND = 1, ST_IN = 2;

__device__ __forceinline__ uint64_t splitmix64_dev(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t node_h(int64_t i) { return splitmix64_dev((uint64_t)i) & 0x3FFFFFFFull; }
// (h(j), j): the order in which aggregation passes prefer neighbours
__device__ __forceinline__ uint64_t node_key(int64_t j) { return (node_h(j) << 32) | (uint64_t)j; }

// ---- strength ---------------------------------------------------------------

__global__ void strength_m_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const double* __restrict__ v, double* __restrict__ m) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double mx = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] != i) mx = fmax(mx, -v[k]);
    m[i] = mx;
}

__device__ __forceinline__ bool is_strong(int64_t i, int32_t j, double a, const double* m, double theta) {
    const double s = -a;
    return j != i && s > 0.0 && s >= theta * fmin(m[i], m[j]);
}

// FILL = false: strong count per row; true: strong columns (in row order)
template <bool FILL>
__global__ void strength_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const double* __restrict__ v, const double* __restrict__ m, double theta,
                                int32_t* __restrict__ cnt, const int32_t* __restrict__ grp, int32_t* __restrict__ gci) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t o = FILL ? grp[i] : 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = ci[k];
        if (is_strong(i, j, v[k], m, theta)) {
            if (FILL) gci[o] = j;
            ++o;
        }
    }
    if (!FILL) cnt[i] = o;
}

// ---- distance-2 maximal independent set ----------------------------------

__device__ __forceinline__ uint64_t mis_key(const uint8_t* state, int64_t i) {
    return ((uint64_t)state[i] << 62) | (node_h(i) << 32) | (uint64_t)i;
}

__global__ void mis_m1_kernel(int64_t n, const int32_t* __restrict__ grp, const int32_t* __restrict__ gci,
                              const uint8_t* __restrict__ state, uint64_t* __restrict__ m1) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t mx = mis_key(state, i);
    for (int32_t k = grp[i]; k < grp[i + 1]; ++k) {
        const uint64_t kj = mis_key(state, gci[k]);
        mx = kj > mx ? kj : mx;
    }
    m1[i] = mx;
}

__global__ void mis_m2_kernel(int64_t n, const int32_t* __restrict__ grp, const int32_t* __restrict__ gci,
                              const uint64_t* __restrict__ m1, uint64_t* __restrict__ m2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t mx = m1[i];
    for (int32_t k = grp[i]; k < grp[i + 1]; ++k) mx = m1[gci[k]] > mx ? m1[gci[k]] : mx;
    m2[i] = mx;
}

__global__ void mis_update_kernel(int64_t n, uint8_t* __restrict__ state, const uint64_t* __restrict__ m2,
                                  int* __restrict__ undecided) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool und = false;
    if (i < n && state[i] == ST_UND) {
        const uint64_t key = mis_key(state, i);
        if (m2[i] == key) state[i] = ST_IN;
        else if ((m2[i] >> 62) == ST_IN) state[i] = ST_OUT;
        else und = true;
    }
    // one atomic per wavefront that still has undecided nodes
    if (__any(und) && (threadIdx.x % 64) == 0) atomicAdd(undecided, 1);
}

// ---- aggregation ----------------------------------------------------------

__global__ void root_count_kernel(int64_t n, const uint8_t* __restrict__ state, int32_t* __restrict__ cnt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) cnt[i] = state[i] == ST_IN ? 1 : 0;
}

// pass 1: roots keep their number (the exclusive scan of the root flags);
// a neighbour of roots joins the root of largest key; others stay -1
__global__ void agg_pass1_kernel(int64_t n, const int32_t* __restrict__ grp, const int32_t* __restrict__ gci,
                                 const uint8_t* __restrict__ state, const int32_t* __restrict__ rootnum,
                                 int32_t* __restrict__ first) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (state[i] == ST_IN) {
        first[i] = rootnum[i];
        return;
    }
    int64_t best = -1;
    uint64_t bk = 0;
    for (int32_t k = grp[i]; k < grp[i + 1]; ++k) {
        const int32_t j = gci[k];
        if (state[j] != ST_IN) continue;
        const uint64_t kj = node_key(j);
        if (best < 0 || kj > bk) {
            best = j;
            bk = kj;
        }
    }
    first[i] = best >= 0 ? rootnum[best] : -1;
}

// pass 2: the rest join the pass-1 (non-root) neighbour of largest key
__global__ void agg_pass2_kernel(int64_t n, const int32_t* __restrict__ grp, const int32_t* __restrict__ gci,
                                 const uint8_t* __restrict__ state, const int32_t* __restrict__ first,
                                 int32_t* __restrict__ agg, int* __restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (first[i] >= 0) {
        agg[i] = first[i];
        return;
    }
    int64_t best = -1;
    uint64_t bk = 0;
    for (int32_t k = grp[i]; k < grp[i + 1]; ++k) {
        const int32_t j = gci[k];
        if (first[j] < 0 || state[j] == ST_IN) continue;
        const uint64_t kj = node_key(j);
        if (best < 0 || kj > bk) {
            best = j;
            bk = kj;
        }
    }
    if (best < 0) {
        atomicExch(bad, 1);
        agg[i] = 0;
    } else {
        agg[i] = first[best];
    }
}

// ---- smoothed prolongator -------------------------------------------------
// One wavefront per row i of A.  Kept entries: the diagonal (value dF, the
// diagonal plus the weak off-diagonals, summed in row order) and the strong
// off-diagonals; entry k contributes aF_k / dF to column agg(j_k).  Row i of
// P: for each distinct column J in increasing order, (agg(i) == J) -
// omega * sum of its contributions in row order, dropped when exactly 0.
constexpr int PROL_MAXLEN = 1024;

template <bool FILL>
__global__ __launch_bounds__(64) void prolong_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                     const double* __restrict__ m, double theta,
                                                     const int32_t* __restrict__ agg, double omega,
                                                     int32_t* __restrict__ cnt, const int32_t* __restrict__ prp,
                                                     int32_t* __restrict__ pci, double* __restrict__ pv,
                                                     int* __restrict__ bad) {
    __shared__ int32_t J[PROL_MAXLEN];
    __shared__ double w[PROL_MAXLEN];
    __shared__ double val[PROL_MAXLEN];
    __shared__ int32_t keep[PROL_MAXLEN];   // 1: first occurrence of its column with a nonzero value
    __shared__ double s_dF;
    const int64_t i = blockIdx.x;
    const int t = threadIdx.x;
    const int32_t r0 = rp[i], len = rp[i + 1] - r0;
    if (len > PROL_MAXLEN) {
        if (t == 0) atomicExch(bad, 2);
        if (!FILL && t == 0) cnt[i] = 0;
        return;
    }
    // kept entries and their columns; dF in row order (one lane)
    for (int k = t; k < len; k += 64) {
        const int32_t j = ci[r0 + k];
        const bool strong = is_strong(i, j, v[r0 + k], m, theta);
        J[k] = (j == i || strong) ? agg[j] : -1;
    }
    if (t == 0) {
        double dF = 0.0;
        for (int k = 0; k < len; ++k) {
            const int32_t j = ci[r0 + k];
            if (j == i || !is_strong(i, j, v[r0 + k], m, theta)) dF = dF + v[r0 + k];
        }
        s_dF = dF;
    }
    __syncthreads();
    const double dF = s_dF;
    for (int k = t; k < len; k += 64) {
        const int32_t j = ci[r0 + k];
        const double aF = j == i ? dF : v[r0 + k];
        w[k] = J[k] >= 0 ? aF / dF : 0.0;
    }
    __syncthreads();
    const int32_t Ji = agg[i];
    for (int k = t; k < len; k += 64) {
        int kp = 0;
        double acc = 0.0;
        if (J[k] >= 0) {
            bool firstocc = true;
            for (int q = 0; q < k; ++q)
                if (J[q] == J[k]) {
                    firstocc = false;
                    break;
                }
            if (firstocc) {
                for (int q = k; q < len; ++q)
                    if (J[q] == J[k]) acc = acc + w[q];
                const double vv = (Ji == J[k] ? 1.0 : 0.0) - omega * acc;
                val[k] = vv;
                kp = vv != 0.0;
            }
        }
        keep[k] = kp;
    }
    __syncthreads();
    if (!FILL) {
        int c = 0;
        for (int k = t; k < len; k += 64) c += keep[k];
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if (t == 0) cnt[i] = c;
        return;
    }
    for (int k = t; k < len; k += 64) {
        if (!keep[k]) continue;
        int pos = 0;
        for (int q = 0; q < len; ++q) pos += keep[q] && J[q] < J[k];
        pci[prp[i] + pos] = J[k];
        pv[prp[i] + pos] = val[k];
    }
}

// ---- row-wise sparse product C = A B --------------------------------------
// One wavefront per row of C.  The candidate columns (the columns of the
// rows of B selected by row i of A) go to a buffer, are sorted (bitonic,
// padded with INT32_MAX) and made unique; then each distinct column c sums
// A_ik B_kc over the entries of row i of A in order (binary search in row k
// of B, whose columns are sorted).  Rows whose candidates exceed the LDS
// capacity use a slice of a global buffer instead.
constexpr int SPG_LDS = 2048;

__device__ __forceinline__ void bitonic_sort(int32_t* a, int n2, int t, int nt) {
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int x = t; x < n2; x += nt) {
                const int y = x ^ j;
                if (y > x) {
                    const int32_t ax = a[x], ay = a[y];
                    const bool up = (x & k) == 0;
                    if ((ax > ay) == up) {
                        a[x] = ay;
                        a[y] = ax;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int32_t find_col(const int32_t* __restrict__ ci, int32_t lo, int32_t hi, int32_t c) {
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (ci[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// candidates of row i: total count (the sum of the selected B row lengths)
__global__ void spgemm_cand_kernel(int64_t n, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                   const int32_t* __restrict__ brp, int64_t* __restrict__ ncand) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t s = 0;
    for (int32_t k = arp[i]; k < arp[i + 1]; ++k) s += brp[aci[k] + 1] - brp[aci[k]];
    ncand[i] = s;
}

// FILL = false: number of distinct columns of each row; true: the row of C.
// big: rows handled by this launch (null: all rows, LDS buffer); with a
// global buffer, gbuf + goff[r] holds the candidates of the r-th listed row.
template <bool FILL, bool GLOBAL>
__global__ __launch_bounds__(64) void spgemm_row_kernel(
    int64_t nrows_launch, const int32_t* __restrict__ rows, const int32_t* __restrict__ arp,
    const int32_t* __restrict__ aci, const double* __restrict__ av, const int32_t* __restrict__ brp,
    const int32_t* __restrict__ bci, const double* __restrict__ bv, const int64_t* __restrict__ ncand,
    int32_t* __restrict__ gbuf, const int64_t* __restrict__ goff, int32_t* __restrict__ cnt,
    const int32_t* __restrict__ crp, int32_t* __restrict__ cci, double* __restrict__ cv) {
    __shared__ int32_t lbuf[GLOBAL ? 1 : SPG_LDS];
    __shared__ int32_t s_pref[65];
    const int64_t r = blockIdx.x;
    if (r >= nrows_launch) return;
    const int64_t i = rows ? rows[r] : r;
    const int t = threadIdx.x;
    const int64_t nc = ncand[i];
    if (!GLOBAL && nc > SPG_LDS) return;   // handled by the global-buffer launch
    int n2 = 1;
    while (n2 < nc) n2 <<= 1;
    int32_t* buf = GLOBAL ? gbuf + goff[r] : lbuf;
    const int32_t a0 = arp[i], a1 = arp[i + 1];
    // candidates: the rows of B in the order of row i of A, in chunks of 64
    // entries of A with an exclusive scan of their lengths
    int64_t base = 0;
    for (int32_t k0 = a0; k0 < a1; k0 += 64) {
        const int32_t k = k0 + t;
        int32_t len = 0, j = 0;
        if (k < a1) {
            j = aci[k];
            len = brp[j + 1] - brp[j];
        }
        // inclusive scan over the wavefront
        int32_t inc = len;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_up(inc, off, 64);
            if (t >= off) inc += o;
        }
        if (k < a1) {
            const int64_t o = base + inc - len;
            for (int32_t l = 0; l < len; ++l) buf[o + l] = bci[brp[j] + l];
        }
        base += __shfl(inc, 63, 64);
    }
    for (int64_t x = nc + t; x < n2; x += 64) buf[x] = INT32_MAX;
    __syncthreads();
    bitonic_sort(buf, n2, t, 64);
    // distinct columns: first of each run; their rank by a block scan
    int32_t mine = 0;
    const int64_t per = (nc + 63) / 64;
    const int64_t lo = t * per, hi = lo + per < nc ? lo + per : nc;
    for (int64_t x = lo; x < hi; ++x) mine += (x == 0 || buf[x] != buf[x - 1]);
    int32_t inc = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(inc, off, 64);
        if (t >= off) inc += o;
    }
    if (!FILL) {
        if (t == 63) cnt[i] = inc;
        return;
    }
    s_pref[t] = inc - mine;
    __syncthreads();
    int32_t pos = crp[i] + s_pref[t];
    for (int64_t x = lo; x < hi; ++x) {
        if (!(x == 0 || buf[x] != buf[x - 1])) continue;
        const int32_t c = buf[x];
        double acc = 0.0;
        for (int32_t k = a0; k < a1; ++k) {
            const int32_t j = aci[k];
            const int32_t b0 = brp[j], b1 = brp[j + 1];
            const int32_t l = find_col(bci, b0, b1, c);
            if (l < b1 && bci[l] == c) acc = acc + av[k] * bv[l];
        }
        cci[pos] = c;
        cv[pos] = acc;
        ++pos;
    }
}

// ---- transpose (rows of the result sorted) ---------------------------------
__global__ void col_count_kernel(int64_t nnz, const int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < nnz) atomicAdd(&cnt[ci[k]], 1);
}

__global__ void transpose_scatter_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                         const double* __restrict__ v, int32_t* __restrict__ cursor,
                                         int32_t* __restrict__ tci, double* __restrict__ tv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t o = atomicAdd(&cursor[ci[k]], 1);
        tci[o] = (int32_t)i;
        tv[o] = v[k];
    }
}

// sort each row of the transpose by column (the row index of the source,
// unique within the row): insertion sort, one thread per row
__global__ void row_sort_kernel(int64_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ ci,
                                double* __restrict__ v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t a = rp[i], b = rp[i + 1];
    for (int32_t k = a + 1; k < b; ++k) {
        const int32_t c = ci[k];
        const double x = v[k];
        int32_t q = k - 1;
        while (q >= a && ci[q] > c) {
            ci[q + 1] = ci[q];
            v[q + 1] = v[q];
            --q;
        }
        ci[q + 1] = c;
        v[q + 1] = x;
    }
}

// ---- (A + A^T) / 2 by merging row i of A and of A^T ------------------------
template <bool FILL>
__global__ void symm_kernel(int64_t n, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                            const double* __restrict__ av, const int32_t* __restrict__ trp,
                            const int32_t* __restrict__ tci, const double* __restrict__ tv, int32_t* __restrict__ cnt,
                            const int32_t* __restrict__ srp, int32_t* __restrict__ sci, double* __restrict__ sv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t a = arp[i], b = trp[i];
    const int32_t ae = arp[i + 1], be = trp[i + 1];
    int32_t o = FILL ? srp[i] : 0;
    while (a < ae || b < be) {
        const int32_t ca = a < ae ? aci[a] : INT32_MAX;
        const int32_t cb = b < be ? tci[b] : INT32_MAX;
        if (FILL) {
            double x;
            int32_t c;
            if (ca == cb) {
                x = (av[a] + tv[b]) * 0.5;
                c = ca;
            } else if (ca < cb) {
                x = av[a] * 0.5;
                c = ca;
            } else {
                x = tv[b] * 0.5;
                c = cb;
            }
            sci[o] = c;
            sv[o] = x;
        }
        if (ca == cb) {
            ++a;
            ++b;
        } else if (ca < cb) {
            ++a;
        } else {
            ++b;
        }
        ++o;
    }
    if (!FILL) cnt[i] = o;
}

// ---- dense coarse inverse: Gauss-Jordan with partial pivoting ---------------
__global__ void dense_from_csr_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                      const double* __restrict__ v, double* __restrict__ A, double* __restrict__ I,
                                      double* __restrict__ trace_part) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double tr = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        A[i * n + k] = 0.0;
        I[i * n + k] = k == i ? 1.0 : 0.0;
    }
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        A[i * n + ci[k]] = v[k];
        if (ci[k] == i) tr = v[k];
    }
    trace_part[i] = tr;
}

// trace in row order (the host adds the diagonal entries row by row), then
// A += s e e^T with s = trace / n / n (singular S~)
__global__ void dense_regularise_kernel(int64_t n, const double* __restrict__ trace_part, double* __restrict__ A) {
    __shared__ double s_s;
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int64_t i = 0; i < n; ++i) tr = tr + trace_part[i];
        s_s = tr / (double)n / (double)n;
    }
    __syncthreads();
    for (int64_t x = threadIdx.x; x < n * n; x += blockDim.x) A[x] = A[x] + s_s;
}

// pivot row of column c: first row r >= c of largest |A_rc|; swap it with
// row c, scale row c by 1 / A_cc and keep column c of the other rows
__global__ void gj_pivot_kernel(int64_t n, int64_t c, double* __restrict__ A, double* __restrict__ I,
                                double* __restrict__ fcol, int* __restrict__ bad) {
    __shared__ double sv[1024];
    __shared__ int64_t si[1024];
    const int t = threadIdx.x;
    double best = -1.0;
    int64_t bi = -1;
    for (int64_t r = c + t; r < n; r += blockDim.x) {
        const double a = fabs(A[r * n + c]);
        if (a > best) {
            best = a;
            bi = r;
        }
    }
    sv[t] = best;
    si[t] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) {
            const double a = sv[t + s];
            const int64_t ai = si[t + s];
            if (ai >= 0 && (si[t] < 0 || a > sv[t] || (a == sv[t] && ai < si[t]))) {
                sv[t] = a;
                si[t] = ai;
            }
        }
        __syncthreads();
    }
    const int64_t piv = si[0];
    if (piv < 0 || A[piv * n + c] == 0.0) {
        if (t == 0) *bad = 1;
        return;
    }
    if (piv != c)
        for (int64_t k = t; k < n; k += blockDim.x) {
            const double a = A[c * n + k], b = I[c * n + k];
            A[c * n + k] = A[piv * n + k];
            I[c * n + k] = I[piv * n + k];
            A[piv * n + k] = a;
            I[piv * n + k] = b;
        }
    __syncthreads();
    const double d = 1.0 / A[c * n + c];
    __syncthreads();
    for (int64_t k = t; k < n; k += blockDim.x) {
        A[c * n + k] = A[c * n + k] * d;
        I[c * n + k] = I[c * n + k] * d;
    }
    __syncthreads();
    for (int64_t r = t; r < n; r += blockDim.x) fcol[r] = A[r * n + c];
}

__global__ void gj_eliminate_kernel(int64_t n, int64_t c, double* __restrict__ A, double* __restrict__ I,
                                    const double* __restrict__ fcol, const int* __restrict__ bad) {
    if (*bad) return;
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (x >= 2 * n * n) return;
    const bool inv = x >= n * n;
    const int64_t y = inv ? x - n * n : x;
    const int64_t r = y / n, k = y % n;
    if (r == c) return;
    const double f = fcol[r];
    if (f == 0.0) return;
    double* M = inv ? I : A;
    M[r * n + k] = M[r * n + k] - f * M[c * n + k];
}

// ---- device CSR helpers ---------------------------------------------------

int alloc_csr(hd_ctx* c, DevCSR& d, int64_t nrows, int64_t ncols, int64_t nnz, int32_t* rp) {
    d.nrows = nrows;
    d.ncols = ncols;
    d.nnz = nnz;
    d.rp = rp;
    d.ci = dalloc<int32_t>(nnz);
    d.v = dalloc<double>(nnz);
    if (!d.ci || !d.v) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    return HD_OK;
}

struct Tmp {
    std::vector<void*> p;
    template <typename T>
    T* get(int64_t n) {
        T* q = dalloc<T>(n);
        p.push_back(q);
        return q;
    }
    ~Tmp() {
        for (void* q : p) dfree(q);
    }
};

// C = A B (values FP64 only; C.v32 left null)
int spgemm(hd_ctx* c, const DevCSR& A, const DevCSR& B, DevCSR& C) {
    Tmp tmp;
    const int64_t n = A.nrows;
    int64_t* ncand = tmp.get<int64_t>(n);
    int32_t* cnt = tmp.get<int32_t>(n);
    if (!ncand || !cnt) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    hipLaunchKernelGGL(spgemm_cand_kernel, dim3(nbk(n)), dim3(BSA), 0, c->stream, n, A.rp, A.ci, B.rp, ncand);
    // rows with more candidates than the LDS buffer: a global buffer
    std::vector<int64_t> hc(n);
    HD_HIP(c, hipMemcpyAsync(hc.data(), ncand, sizeof(int64_t) * n, hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> big;
    std::vector<int64_t> boff(1, 0);
    for (int64_t i = 0; i < n; ++i)
        if (hc[i] > SPG_LDS) {
            int64_t n2 = 1;
            while (n2 < hc[i]) n2 <<= 1;
            big.push_back((int32_t)i);
            boff.push_back(boff.back() + n2);
        }
    int32_t* d_big = nullptr;
    int64_t* d_boff = nullptr;
    int32_t* gbuf = nullptr;
    if (!big.empty()) {
        d_big = tmp.get<int32_t>((int64_t)big.size());
        d_boff = tmp.get<int64_t>((int64_t)boff.size());
        gbuf = tmp.get<int32_t>(boff.back());
        if (!d_big || !d_boff || !gbuf) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
        HD_HIP(c, hipMemcpyAsync(d_big, big.data(), sizeof(int32_t) * big.size(), hipMemcpyHostToDevice, c->stream));
        HD_HIP(c, hipMemcpyAsync(d_boff, boff.data(), sizeof(int64_t) * boff.size(), hipMemcpyHostToDevice, c->stream));
    }
    // small rows are all launched through the LDS kernel; the big ones return
    // at once there (their count is written by the global-buffer launch)
    auto launch = [&](bool fill, int32_t* crp, int32_t* cci, double* cv) {
        if (fill)
            hipLaunchKernelGGL((spgemm_row_kernel<true, false>), dim3((unsigned)n), dim3(64), 0, c->stream, n,
                               (const int32_t*)nullptr, A.rp, A.ci, A.v, B.rp, B.ci, B.v, ncand, (int32_t*)nullptr,
                               (const int64_t*)nullptr, cnt, crp, cci, cv);
        else
            hipLaunchKernelGGL((spgemm_row_kernel<false, false>), dim3((unsigned)n), dim3(64), 0, c->stream, n,
                               (const int32_t*)nullptr, A.rp, A.ci, A.v, B.rp, B.ci, B.v, ncand, (int32_t*)nullptr,
                               (const int64_t*)nullptr, cnt, crp, cci, cv);
        if (!big.empty()) {
            if (fill)
                hipLaunchKernelGGL((spgemm_row_kernel<true, true>), dim3((unsigned)big.size()), dim3(64), 0,
                                   c->stream, (int64_t)big.size(), (const int32_t*)d_big, A.rp, A.ci, A.v, B.rp, B.ci,
                                   B.v, ncand, gbuf, (const int64_t*)d_boff, cnt, crp, cci, cv);
            else
                hipLaunchKernelGGL((spgemm_row_kernel<false, true>), dim3((unsigned)big.size()), dim3(64), 0,
                                   c->stream, (int64_t)big.size(), (const int32_t*)d_big, A.rp, A.ci, A.v, B.rp, B.ci,
                                   B.v, ncand, gbuf, (const int64_t*)d_boff, cnt, crp, cci, cv);
        }
    };
    launch(false, nullptr, nullptr, nullptr);
    HD_HIP(c, hipGetLastError());
    int32_t* rp = dalloc<int32_t>(n + 1);
    if (!rp) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    int64_t nnz = 0;
    int rc = scan_counts(c, cnt, n, rp, &nnz);
    if (rc || nnz > INT32_MAX) {
        dfree(rp);
        return rc ? rc : set_err(c, HD_ERR_AMG, "Galerkin product has more than 2^31 nonzeros");
    }
    if ((rc = alloc_csr(c, C, n, B.ncols, nnz, rp))) return rc;
    launch(true, C.rp, C.ci, C.v);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

int transpose_dev(hd_ctx* c, const DevCSR& A, DevCSR& T) {
    Tmp tmp;
    const int64_t n = A.nrows, m = A.ncols;
    int32_t* cnt = tmp.get<int32_t>(m);
    if (!cnt) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    HD_HIP(c, hipMemsetAsync(cnt, 0, sizeof(int32_t) * m, c->stream));
    if (A.nnz) hipLaunchKernelGGL(col_count_kernel, dim3(nbk(A.nnz)), dim3(BSA), 0, c->stream, A.nnz, A.ci, cnt);
    int32_t* rp = dalloc<int32_t>(m + 1);
    if (!rp) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    int64_t nnz = 0;
    int rc = scan_counts(c, cnt, m, rp, &nnz);
    if (rc) {
        dfree(rp);
        return rc;
    }
    if ((rc = alloc_csr(c, T, m, n, nnz, rp))) return rc;
    HD_HIP(c, hipMemcpyAsync(cnt, rp, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(transpose_scatter_kernel, dim3(nbk(n)), dim3(BSA), 0, c->stream, n, A.rp, A.ci, A.v, cnt, T.ci,
                       T.v);
    hipLaunchKernelGGL(row_sort_kernel, dim3(nbk(m)), dim3(BSA), 0, c->stream, m, T.rp, T.ci, T.v);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

void free_dev_csr(DevCSR& d) {
    dfree(d.rp);
    dfree(d.ci);
    dfree(d.v);
    dfree(d.v32);
    d = DevCSR();
}

// one level: G, aggregates, P, A_c
int coarsen(hd_ctx* c, const DevCSR& A, const hd_precond_params& prm, DevCSR& P, DevCSR& R, DevCSR& Ac,
            int64_t& na_out) {
    Tmp tmp;
    const int64_t n = A.nrows;
    double* m = tmp.get<double>(n);
    int32_t* cnt = tmp.get<int32_t>(n + 1);
    int32_t* grp = tmp.get<int32_t>(n + 1);
    uint8_t* state = tmp.get<uint8_t>(n);
    uint64_t* m1 = tmp.get<uint64_t>(n);
    uint64_t* m2 = tmp.get<uint64_t>(n);
    int32_t* rootnum = tmp.get<int32_t>(n + 1);
    int32_t* first = tmp.get<int32_t>(n);
    int32_t* agg = tmp.get<int32_t>(n);
    int* flag = tmp.get<int>(4);
    if (!m || !cnt || !grp || !state || !m1 || !m2 || !rootnum || !first || !agg || !flag)
        return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    const unsigned nb = nbk(n);
    // strength graph
    hipLaunchKernelGGL(strength_m_kernel, dim3(nb), dim3(BSA), 0, c->stream, n, A.rp, A.ci, A.v, m);
    hipLaunchKernelGGL((strength_kernel<false>), dim3(nb), dim3(BSA), 0, c->stream, n, A.rp, A.ci, A.v,
                       (const double*)m, prm.theta, cnt, (const int32_t*)nullptr, (int32_t*)nullptr);
    int64_t gnnz = 0;
    int rc = scan_counts(c, cnt, n, grp, &gnnz);
    if (rc) return rc;
    int32_t* gci = tmp.get<int32_t>(gnnz);
    if (!gci) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    hipLaunchKernelGGL((strength_kernel<true>), dim3(nb), dim3(BSA), 0, c->stream, n, A.rp, A.ci, A.v,
                       (const double*)m, prm.theta, (int32_t*)nullptr, (const int32_t*)grp, gci);
    // MIS-2 rounds until no node is undecided
    HD_HIP(c, hipMemsetAsync(state, ST_UND, n, c->stream));
    int undecided = n > 0 ? 1 : 0;
    int rounds = 0;
    while (undecided) {
        HD_HIP(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream));
        hipLaunchKernelGGL(mis_m1_kernel, dim3(nb), dim3(BSA), 0, c->stream, n, grp, gci, state, m1);
        hipLaunchKernelGGL(mis_m2_kernel, dim3(nb), dim3(BSA), 0, c->stream, n, grp, gci, m1, m2);
        hipLaunchKernelGGL(mis_update_kernel, dim3(nb), dim3(BSA), 0, c->stream, n, state, m2, flag);
        HD_HIP(c, hipGetLastError());
        HD_HIP(c, hipMemcpyAsync(&undecided, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HD_HIP(c, hipStreamSynchronize(c->stream));
        if (++rounds > 100000) return set_err(c, HD_ERR_AMG, "MIS-2 did not terminate");
    }
    // aggregates
    hipLaunchKernelGGL(root_count_kernel, dim3(nb), dim3(BSA), 0, c->stream, n, state, cnt);
    int64_t na = 0;
    if ((rc = scan_counts(c, cnt, n, rootnum, &na))) return rc;
    na_out = na;
    if (na >= n) return HD_OK;   // no reduction: the caller stops here
    HD_HIP(c, hipMemsetAsync(flag, 0, 4 * sizeof(int), c->stream));
    hipLaunchKernelGGL(agg_pass1_kernel, dim3(nb), dim3(BSA), 0, c->stream, n, grp, gci, state, rootnum, first);
    hipLaunchKernelGGL(agg_pass2_kernel, dim3(nb), dim3(BSA), 0, c->stream, n, grp, gci, state, first, agg, flag);
    // smoothed prolongator
    hipLaunchKernelGGL((prolong_kernel<false>), dim3((unsigned)n), dim3(64), 0, c->stream, n, A.rp, A.ci, A.v,
                       (const double*)m, prm.theta, (const int32_t*)agg, prm.omega, cnt, (const int32_t*)nullptr,
                       (int32_t*)nullptr, (double*)nullptr, flag + 1);
    HD_HIP(c, hipGetLastError());
    int hflag[2] = {0, 0};
    HD_HIP(c, hipMemcpyAsync(hflag, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    if (hflag[0]) return set_err(c, HD_ERR_AMG, "aggregation left a node unassigned");
    if (hflag[1]) return set_err(c, HD_ERR_AMG, "AMG row longer than the prolongator kernel handles");
    int32_t* prp = dalloc<int32_t>(n + 1);
    if (!prp) return set_err(c, HD_ERR_OOM, "AMG set-up storage");
    int64_t pnnz = 0;
    if ((rc = scan_counts(c, cnt, n, prp, &pnnz))) {
        dfree(prp);
        return rc;
    }
    if ((rc = alloc_csr(c, P, n, na, pnnz, prp))) return rc;
    hipLaunchKernelGGL((prolong_kernel<true>), dim3((unsigned)n), dim3(64), 0, c->stream, n, A.rp, A.ci, A.v,
                       (const double*)m, prm.theta, (const int32_t*)agg, prm.omega, (int32_t*)nullptr,
                       (const int32_t*)P.rp, P.ci, P.v, flag + 1);
    HD_HIP(c, hipGetLastError());
    // A_c = sym(P^T (A P))
    DevCSR AP, Pt, PtAP, T;
    rc = spgemm(c, A, P, AP);
    if (!rc) rc = transpose_dev(c, P, Pt);
    if (!rc) rc = spgemm(c, Pt, AP, PtAP);
    if (!rc) rc = transpose_dev(c, PtAP, T);
    if (!rc) {
        const int64_t nc = PtAP.nrows;
        int32_t* scnt = tmp.get<int32_t>(nc);
        int32_t* srp = dalloc<int32_t>(nc + 1);
        if (!scnt || !srp) {
            dfree(srp);
            rc = set_err(c, HD_ERR_OOM, "AMG set-up storage");
        } else {
            hipLaunchKernelGGL((symm_kernel<false>), dim3(nbk(nc)), dim3(BSA), 0, c->stream, nc, PtAP.rp, PtAP.ci,
                               PtAP.v, T.rp, T.ci, T.v, scnt, (const int32_t*)nullptr, (int32_t*)nullptr,
                               (double*)nullptr);
            int64_t snnz = 0;
            rc = scan_counts(c, scnt, nc, srp, &snnz);
            if (rc) dfree(srp);
            if (!rc) rc = alloc_csr(c, Ac, nc, nc, snnz, srp);
            if (!rc) {
                hipLaunchKernelGGL((symm_kernel<true>), dim3(nbk(nc)), dim3(BSA), 0, c->stream, nc, PtAP.rp,
                                   PtAP.ci, PtAP.v, T.rp, T.ci, T.v, (int32_t*)nullptr, (const int32_t*)Ac.rp, Ac.ci,
                                   Ac.v);
                if (hipGetLastError() != hipSuccess) rc = set_err(c, HD_ERR_HIP, "symmetrise launch");
            }
        }
    }
    // the transpose of P is the restriction of the V-cycle: keep it
    free_dev_csr(AP);
    free_dev_csr(PtAP);
    free_dev_csr(T);
    if (rc) {
        free_dev_csr(Pt);
        return rc;
    }
    R = Pt;
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

__global__ void f32_copy_kernel(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

int add_f32(hd_ctx* c, DevCSR& d) {
    if (d.v32) return HD_OK;
    d.v32 = dalloc<float>(d.nnz);
    if (!d.v32) return set_err(c, HD_ERR_OOM, "AMG level storage");
    if (d.nnz) hipLaunchKernelGGL(f32_copy_kernel, dim3(nbk(d.nnz)), dim3(BSA), 0, c->stream, d.nnz, d.v, d.v32);
    HD_HIP(c, hipGetLastError());
    return HD_OK;
}

}  // namespace

// Builds c->lev (matrices A, P, R of every level, FP64 and FP32 values) and
// the dense coarse inverse c->d_cinv from S~ on the device.
int build_amg_gpu(hd_ctx* c, const hd_precond_params& prm) {
    free_levels(c);
    c->lev.emplace_back();
    c->lev[0].A = c->S;   // level 0 aliases S~
    while (c->lev.back().A.nrows > prm.max_coarse && (int)c->lev.size() < prm.max_levels) {
        DevCSR P, R, Ac;
        int64_t na = 0;
        const DevCSR A = c->lev.back().A;
        int rc = coarsen(c, A, prm, P, R, Ac, na);
        if (rc) {
            free_dev_csr(P);
            free_dev_csr(R);
            free_dev_csr(Ac);
            return rc;
        }
        if (na >= A.nrows) break;
        c->lev.back().P = P;
        c->lev.back().R = R;
        if ((rc = add_f32(c, c->lev.back().P)) || (rc = add_f32(c, c->lev.back().R))) return rc;
        c->lev.emplace_back();
        c->lev.back().A = Ac;
        if ((rc = add_f32(c, c->lev.back().A))) return rc;
    }
    // dense inverse of the coarsest matrix (+ s e e^T when S~ is singular)
    const DevCSR& Ac = c->lev.back().A;
    const int64_t nc = Ac.nrows;
    if (nc > 8192) return set_err(c, HD_ERR_AMG, "coarsest AMG level too large for a dense inverse");
    Tmp tmp;
    double* A = tmp.get<double>(nc * nc);
    double* tr = tmp.get<double>(nc);
    double* fcol = tmp.get<double>(nc);
    int* bad = tmp.get<int>(1);
    c->d_cinv = dalloc<double>(nc * nc);
    if (!A || !tr || !fcol || !bad || !c->d_cinv) return set_err(c, HD_ERR_OOM, "coarse inverse");
    HD_HIP(c, hipMemsetAsync(bad, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(dense_from_csr_kernel, dim3(nbk(nc)), dim3(BSA), 0, c->stream, nc, Ac.rp, Ac.ci, Ac.v, A,
                       c->d_cinv, tr);
    if (c->singular) hipLaunchKernelGGL(dense_regularise_kernel, dim3(1), dim3(1024), 0, c->stream, nc, tr, A);
    for (int64_t col = 0; col < nc; ++col) {
        hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(1024), 0, c->stream, nc, col, A, c->d_cinv, fcol, bad);
        hipLaunchKernelGGL(gj_eliminate_kernel, dim3(nbk(2 * nc * nc)), dim3(BSA), 0, c->stream, nc, col, A,
                           c->d_cinv, (const double*)fcol, (const int*)bad);
    }
    HD_HIP(c, hipGetLastError());
    int hbad = 0;
    HD_HIP(c, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    if (hbad) return set_err(c, HD_ERR_AMG, "coarsest AMG matrix is singular");
    c->n_coarse = nc;
    return HD_OK;
}

}  // namespace hd
