// Smoothed-aggregation AMG setup for the approximate Schur complement S~
// (an M-matrix weighted graph Laplacian plus a diagonal, Section 2.3,
// Prop. 4 and 5).  One V-cycle of this hierarchy stands in for the paper's
// BoomerAMG; every choice is deterministic so that the hierarchy can be
// compared entry by entry with an independent implementation:
//
//   strength   a_ij < 0 strong iff -a_ij >= theta * min(m_i, m_j),
//              m_i = max(0, max_{k != i} -a_ik)
//   MIS-2      keys (state, h(i), i), h = low 30 bits of splitmix64(i);
//              rounds of distance-2 maxima until no node is undecided
//   aggregates roots numbered in index order; pass 1: neighbours of roots
//              join the root of largest (h, index); pass 2: the rest join
//              the pass-1 neighbour of largest (h, index)
//   P          (I - omega D_F^{-1} A_F) T, weak entries lumped to the diagonal
//   A_c        P^T A P, symmetrised as (A_c + A_c^T) / 2
//   coarsest   <= max_coarse rows or no further reduction; dense inverse of
//              A_c (+ s e e^T, s = trace / n^2, when S~ is singular)
//
// Host code (setup only).  Sparse products use Gustavson's row-by-row
// algorithm with a dense marker array.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "hd_internal.hpp"

namespace hd {

namespace {

inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Graph {
    std::vector<int32_t> rp, ci;
};

Graph strength(const HostCSR& A, double theta) {
    const int64_t n = A.nrows;
    std::vector<double> m(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (A.ci[k] != i) m[i] = std::max(m[i], -A.v[k]);
    Graph G;
    G.rp.assign(n + 1, 0);
    G.ci.reserve(A.ci.size());
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.ci[k];
            if (j == i) continue;
            const double v = -A.v[k];
            if (v > 0.0 && v >= theta * std::min(m[i], m[j])) G.ci.push_back(j);
        }
        G.rp[i + 1] = (int32_t)G.ci.size();
    }
    return G;
}

// distance-2 maximal independent set; returns the root mask
std::vector<char> mis2(const Graph& G, const std::vector<uint64_t>& h) {
    const int64_t n = (int64_t)G.rp.size() - 1;
    enum : uint64_t { OUT = 0, UND = 1, IN = 2 };
    std::vector<uint64_t> state(n, UND), key(n), m1(n), m2(n);
    for (;;) {
        bool any = false;
        for (int64_t i = 0; i < n; ++i) any |= state[i] == UND;
        if (!any) break;
        for (int64_t i = 0; i < n; ++i) key[i] = (state[i] << 62) | (h[i] << 32) | (uint64_t)i;
        for (int64_t i = 0; i < n; ++i) {
            uint64_t mx = key[i];
            for (int32_t k = G.rp[i]; k < G.rp[i + 1]; ++k) mx = std::max(mx, key[G.ci[k]]);
            m1[i] = mx;
        }
        for (int64_t i = 0; i < n; ++i) {
            uint64_t mx = m1[i];
            for (int32_t k = G.rp[i]; k < G.rp[i + 1]; ++k) mx = std::max(mx, m1[G.ci[k]]);
            m2[i] = mx;
        }
        for (int64_t i = 0; i < n; ++i) {
            if (state[i] != UND) continue;
            if (m2[i] == key[i]) state[i] = IN;
            else if ((m2[i] >> 62) == IN) state[i] = OUT;
        }
    }
    std::vector<char> root(n);
    for (int64_t i = 0; i < n; ++i) root[i] = state[i] == IN;
    return root;
}

int64_t aggregate(const Graph& G, const std::vector<uint64_t>& h, const std::vector<char>& root,
                  std::vector<int64_t>& agg, std::string& err) {
    const int64_t n = (int64_t)root.size();
    agg.assign(n, -1);
    int64_t na = 0;
    for (int64_t i = 0; i < n; ++i)
        if (root[i]) agg[i] = na++;
    auto nk = [&](int64_t j) { return (h[j] << 32) | (uint64_t)j; };
    std::vector<int64_t> first(agg);
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        int64_t best = -1;
        for (int32_t k = G.rp[i]; k < G.rp[i + 1]; ++k) {
            const int32_t j = G.ci[k];
            if (root[j] && (best < 0 || nk(j) > nk(best))) best = j;
        }
        if (best >= 0) first[i] = agg[best];
    }
    for (int64_t i = 0; i < n; ++i) {
        if (first[i] >= 0) {
            agg[i] = first[i];
            continue;
        }
        int64_t best = -1;
        for (int32_t k = G.rp[i]; k < G.rp[i + 1]; ++k) {
            const int32_t j = G.ci[k];
            if (first[j] >= 0 && !root[j] && (best < 0 || nk(j) > nk(best))) best = j;
        }
        if (best < 0) {
            err = "aggregation left a node unassigned";
            return -1;
        }
        agg[i] = first[best];
    }
    return na;
}

HostCSR prolongator(const HostCSR& A, const Graph& G, const std::vector<int64_t>& agg, int64_t na, double omega) {
    const int64_t n = A.nrows;
    HostCSR P;
    P.nrows = n;
    P.ncols = na;
    P.rp.assign(n + 1, 0);
    std::vector<double> acc(na, 0.0);
    std::vector<char> used(na, 0);
    std::vector<int64_t> cols;
    for (int64_t i = 0; i < n; ++i) {
        // strong flags of row i (both sorted by column)
        double dF = 0.0;
        int32_t gk = G.rp[i];
        cols.clear();
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.ci[k];
            while (gk < G.rp[i + 1] && G.ci[gk] < j) ++gk;
            const bool strong = gk < G.rp[i + 1] && G.ci[gk] == j;
            if (j == i || !strong) dF += A.v[k];
        }
        gk = G.rp[i];
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.ci[k];
            while (gk < G.rp[i + 1] && G.ci[gk] < j) ++gk;
            const bool strong = gk < G.rp[i + 1] && G.ci[gk] == j;
            double aF;
            if (j == i) aF = dF;
            else if (strong) aF = A.v[k];
            else continue;
            const int64_t J = agg[j];
            if (!used[J]) {
                used[J] = 1;
                acc[J] = 0.0;
                cols.push_back(J);
            }
            acc[J] += aF / dF;
        }
        std::sort(cols.begin(), cols.end());
        for (int64_t J : cols) {
            const double val = (agg[i] == J ? 1.0 : 0.0) - omega * acc[J];
            used[J] = 0;
            if (val == 0.0) continue;
            P.ci.push_back((int32_t)J);
            P.v.push_back(val);
        }
        P.rp[i + 1] = (int32_t)P.ci.size();
    }
    return P;
}

HostCSR transpose(const HostCSR& A) {
    HostCSR T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    T.rp.assign(T.nrows + 1, 0);
    for (int32_t j : A.ci) T.rp[j + 1]++;
    for (int64_t i = 0; i < T.nrows; ++i) T.rp[i + 1] += T.rp[i];
    T.ci.resize(A.ci.size());
    T.v.resize(A.v.size());
    std::vector<int32_t> pos(T.rp.begin(), T.rp.end() - 1);
    for (int64_t i = 0; i < A.nrows; ++i)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.ci[k];
            T.ci[pos[j]] = (int32_t)i;
            T.v[pos[j]] = A.v[k];
            pos[j]++;
        }
    return T;   // rows come out with sorted columns
}

HostCSR multiply(const HostCSR& A, const HostCSR& B) {
    HostCSR C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    C.rp.assign(C.nrows + 1, 0);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> mark(B.ncols, -1);
    std::vector<int32_t> cols;
    for (int64_t i = 0; i < A.nrows; ++i) {
        cols.clear();
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.ci[k];
            const double a = A.v[k];
            for (int32_t l = B.rp[j]; l < B.rp[j + 1]; ++l) {
                const int32_t c = B.ci[l];
                if (mark[c] != (int32_t)i) {
                    mark[c] = (int32_t)i;
                    acc[c] = 0.0;
                    cols.push_back(c);
                }
                acc[c] += a * B.v[l];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t c : cols) {
            C.ci.push_back(c);
            C.v.push_back(acc[c]);
        }
        C.rp[i + 1] = (int32_t)C.ci.size();
    }
    return C;
}

// (A + A^T) / 2 for a matrix with symmetric sparsity
HostCSR symmetrise(const HostCSR& A) {
    HostCSR T = transpose(A);
    HostCSR S;
    S.nrows = A.nrows;
    S.ncols = A.ncols;
    S.rp.assign(S.nrows + 1, 0);
    for (int64_t i = 0; i < A.nrows; ++i) {
        int32_t a = A.rp[i], b = T.rp[i];
        while (a < A.rp[i + 1] || b < T.rp[i + 1]) {
            int32_t ca = a < A.rp[i + 1] ? A.ci[a] : INT32_MAX;
            int32_t cb = b < T.rp[i + 1] ? T.ci[b] : INT32_MAX;
            double v;
            int32_t c;
            if (ca == cb) { v = (A.v[a] + T.v[b]) * 0.5; c = ca; ++a; ++b; }
            else if (ca < cb) { v = A.v[a] * 0.5; c = ca; ++a; }
            else { v = T.v[b] * 0.5; c = cb; ++b; }
            S.ci.push_back(c);
            S.v.push_back(v);
        }
        S.rp[i + 1] = (int32_t)S.ci.size();
    }
    return S;
}

bool dense_inverse(int64_t n, std::vector<double>& A, std::vector<double>& inv) {
    // Gauss-Jordan with partial pivoting, row-major
    inv.assign(n * n, 0.0);
    for (int64_t i = 0; i < n; ++i) inv[i * n + i] = 1.0;
    for (int64_t c = 0; c < n; ++c) {
        int64_t piv = c;
        for (int64_t r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return false;
        if (piv != c) {
            for (int64_t k = 0; k < n; ++k) {
                std::swap(A[c * n + k], A[piv * n + k]);
                std::swap(inv[c * n + k], inv[piv * n + k]);
            }
        }
        const double d = 1.0 / A[c * n + c];
        for (int64_t k = 0; k < n; ++k) {
            A[c * n + k] *= d;
            inv[c * n + k] *= d;
        }
        for (int64_t r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[r * n + c];
            if (f == 0.0) continue;
            double* ar = &A[r * n];
            double* ir = &inv[r * n];
            const double* ac = &A[c * n];
            const double* ic = &inv[c * n];
            for (int64_t k = 0; k < n; ++k) {
                ar[k] -= f * ac[k];
                ir[k] -= f * ic[k];
            }
        }
    }
    return true;
}

}  // namespace

int build_amg_host(const HostCSR& S, const hd_precond_params& prm, bool singular, HostAMG& out, std::string& err) {
    out = HostAMG();
    out.singular = singular;
    out.A.push_back(S);
    while (out.A.back().nrows > prm.max_coarse && (int)out.A.size() < prm.max_levels) {
        const HostCSR& A = out.A.back();
        const int64_t n = A.nrows;
        std::vector<uint64_t> h(n);
        for (int64_t i = 0; i < n; ++i) h[i] = splitmix64((uint64_t)i) & 0x3FFFFFFFull;
        Graph G = strength(A, prm.theta);
        std::vector<char> root = mis2(G, h);
        std::vector<int64_t> agg;
        const int64_t na = aggregate(G, h, root, agg, err);
        if (na < 0) return HD_ERR_AMG;
        if (na >= n) break;
        HostCSR P = prolongator(A, G, agg, na, prm.omega);
        HostCSR AP = multiply(A, P);
        HostCSR Pt = transpose(P);
        HostCSR Ac = symmetrise(multiply(Pt, AP));
        out.P.push_back(std::move(P));
        out.A.push_back(std::move(Ac));
    }
    const HostCSR& Ac = out.A.back();
    const int64_t nc = Ac.nrows;
    if (nc > 8192) {
        err = "coarsest AMG level too large for a dense inverse";
        return HD_ERR_AMG;
    }
    std::vector<double> dense(nc * nc, 0.0);
    double tr = 0.0;
    for (int64_t i = 0; i < nc; ++i)
        for (int32_t k = Ac.rp[i]; k < Ac.rp[i + 1]; ++k) {
            dense[i * nc + Ac.ci[k]] = Ac.v[k];
            if (Ac.ci[k] == i) tr += Ac.v[k];
        }
    if (singular) {
        const double s = tr / (double)nc / (double)nc;
        for (auto& v : dense) v += s;
    }
    if (!dense_inverse(nc, dense, out.coarse_inv)) {
        err = "coarsest AMG matrix is singular";
        return HD_ERR_AMG;
    }
    return HD_OK;
}

}  // namespace hd

// ---- host-only C ABI ------------------------------------------------------

struct hd_host_amg {
    hd::HostAMG amg;
};

static void fill_defaults(hd_precond_params& p) {
    p.tau = 1.0;
    p.theta = 0.25;
    p.max_coarse = 1024;
    p.max_levels = 25;
    p.omega = 2.0 / 3.0;
}

extern "C" int hd_host_amg_build(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                                 const hd_precond_params* params, int singular, hd_host_amg** out) {
    if (!out || n <= 0 || !rowptr || !col || !val) return HD_ERR_ARG;
    hd_precond_params prm;
    fill_defaults(prm);
    if (params) prm = *params;
    hd::HostCSR S;
    S.nrows = S.ncols = n;
    S.rp.assign(rowptr, rowptr + n + 1);
    S.ci.assign(col, col + rowptr[n]);
    S.v.assign(val, val + rowptr[n]);
    hd_host_amg* h = new hd_host_amg;
    std::string err;
    int rc = hd::build_amg_host(S, prm, singular != 0, h->amg, err);
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return HD_OK;
}

extern "C" int hd_host_amg_nlevels(const hd_host_amg* h) { return h ? (int)h->amg.A.size() : 0; }

static int copy_csr(const hd::HostCSR& M, int64_t* nr, int64_t* nc, int64_t* nnz, int32_t* rp, int32_t* ci,
                    double* v) {
    if (nr) *nr = M.nrows;
    if (nc) *nc = M.ncols;
    if (nnz) *nnz = M.nnz();
    if (rp) std::memcpy(rp, M.rp.data(), sizeof(int32_t) * (M.nrows + 1));
    if (ci) std::memcpy(ci, M.ci.data(), sizeof(int32_t) * M.ci.size());
    if (v) std::memcpy(v, M.v.data(), sizeof(double) * M.v.size());
    return HD_OK;
}

extern "C" int hd_host_amg_level(const hd_host_amg* h, int level, int64_t* n, int64_t* nnz, int32_t* rowptr,
                                 int32_t* col, double* val) {
    if (!h || level < 0 || level >= (int)h->amg.A.size()) return HD_ERR_ARG;
    return copy_csr(h->amg.A[level], n, nullptr, nnz, rowptr, col, val);
}

extern "C" int hd_host_amg_prolongator(const hd_host_amg* h, int level, int64_t* nrows, int64_t* ncols,
                                       int64_t* nnz, int32_t* rowptr, int32_t* col, double* val) {
    if (!h || level < 0 || level >= (int)h->amg.P.size()) return HD_ERR_ARG;
    return copy_csr(h->amg.P[level], nrows, ncols, nnz, rowptr, col, val);
}

extern "C" int hd_host_amg_free(hd_host_amg* h) {
    delete h;
    return HD_OK;
}
