// Host set-up of unstructured hexahedral meshes (Section 3.2, Algorithm 1;
// Section 4.1 runs on such a mesh): faces, their orientation, the global
// RT and L2 numbering and the element-to-dof index arrays that the element
// kernels gather and scatter through.
//
// Element vertices are given in the reference order v = dx + 2 dy + 4 dz.
// Local face (d, s) of an element is its side x_d = s, with tangential axes
// (t0, t1) = the other two axes in increasing order.  A face is identified
// by its four vertex numbers, and carries a canonical frame fixed by the
// global vertex numbers alone, so both elements of an interior face agree on
// it: origin = the face vertex with the smallest number, a1 = towards the
// smaller-numbered of the origin's two face neighbours, a2 = towards the
// other one, normal a1 x a2.  A global face dof is the flux through its
// sub-face along that normal; the element's local dof is the flux along its
// reference +e_d, so local = sigma * global with sigma = +1 when a1 x a2 (in
// the element's reference coordinates) points along +e_d.  Sub-face (j, k)
// (indices along t0, t1) is sub-face (j', k') of the canonical frame, j'
// along a1 and k' along a2, an index reversed where its axis runs against the
// element's (the Gauss-Lobatto sub-face grid is symmetric about 1/2).
//
// Numbering: face dofs first, face by face in the order of the faces' first
// appearance (element, then d, then s), p^2 per face with j' fastest; then
// the interior dofs element by element, 3 (p-1) p^2 each (component-major,
// the normal index 1..p-1 fastest, then t0, then t1).  L2 dofs are
// element-major as on structured meshes.
#include <algorithm>
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "hd_internal.hpp"

namespace hd {

namespace {

inline int refc(int v, int d) { return (v >> d) & 1; }

}  // namespace

int build_unstructured_numbering(int64_t nv, int64_t ne, const int64_t* elem, int P, UnstructuredMap& out,
                                 std::string& err) {
    out = UnstructuredMap();
    if (ne < 1 || nv < 8) {
        err = "an unstructured mesh needs at least one element and eight vertices";
        return HD_ERR_ARG;
    }
    for (int64_t i = 0; i < 8 * ne; ++i)
        if (elem[i] < 0 || elem[i] >= nv) {
            err = "element vertex number out of range";
            return HD_ERR_ARG;
        }
    // faces: sort the 6 ne (sorted vertex quadruple, occurrence) pairs, then
    // number the distinct quadruples by their first occurrence
    struct Occ {
        std::array<int64_t, 4> key;
        int64_t occ;   // 6 e + 2 d + s
    };
    std::vector<Occ> occ((size_t)(6 * ne));
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t* gv = elem + 8 * e;
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < 2; ++s) {
                std::array<int64_t, 4> k;
                int n = 0;
                for (int v = 0; v < 8; ++v)
                    if (refc(v, d) == s) k[n++] = gv[v];
                std::sort(k.begin(), k.end());
                if (k[0] == k[1] || k[1] == k[2] || k[2] == k[3]) {
                    err = "an element has a face with a repeated vertex";
                    return HD_ERR_MESH;
                }
                occ[(size_t)(6 * e + 2 * d + s)] = {k, 6 * e + 2 * d + s};
            }
    }
    std::vector<int64_t> order((size_t)(6 * ne));
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        if (occ[a].key != occ[b].key) return occ[a].key < occ[b].key;
        return a < b;
    });
    // groups of equal keys; group id -> first occurrence
    std::vector<int64_t> grp_of((size_t)(6 * ne));
    std::vector<int64_t> grp_first;
    std::vector<int> grp_size;
    for (size_t i = 0; i < order.size(); ++i) {
        if (i == 0 || occ[order[i]].key != occ[order[i - 1]].key) {
            grp_first.push_back(order[i]);
            grp_size.push_back(0);
        }
        grp_of[order[i]] = (int64_t)grp_first.size() - 1;
        grp_size.back() += 1;
    }
    const int64_t nf = (int64_t)grp_first.size();
    for (int64_t g = 0; g < nf; ++g)
        if (grp_size[g] > 2) {
            err = "a face is shared by more than two elements";
            return HD_ERR_MESH;
        }
    // face ids in order of first appearance
    std::vector<int64_t> gorder((size_t)nf);
    for (int64_t g = 0; g < nf; ++g) gorder[g] = g;
    std::sort(gorder.begin(), gorder.end(), [&](int64_t a, int64_t b) { return grp_first[a] < grp_first[b]; });
    std::vector<int64_t> face_id((size_t)nf);
    for (int64_t r = 0; r < nf; ++r) face_id[gorder[r]] = r;
    out.nfaces = nf;
    out.boundary_face.assign((size_t)nf, 0);
    for (int64_t g = 0; g < nf; ++g)
        if (grp_size[g] == 1) out.boundary_face[face_id[g]] = 1;

    const int64_t nfd = nf * P * P, nint = 3 * (int64_t)(P - 1) * P * P;
    out.n_face_dofs = nfd;
    out.n_u = nfd + ne * nint;
    out.n_q = ne * (int64_t)P * P * P;
    if (out.n_u + out.n_q > (int64_t)INT32_MAX) {
        err = "problem too large for 32-bit indices";
        return HD_ERR_ARG;
    }
    const int NRT = 3 * P * P * (P + 1);
    out.l2g.assign((size_t)(ne * NRT), 0);
    out.elem_face.assign((size_t)(ne * 6), 0);
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t* gv = elem + 8 * e;
        // per local face: global face, sigma, and how (j, k) map to (j', k')
        int64_t fid[3][2];
        int sig[3][2];
        int src[3][2][2], rev[3][2][2];
        for (int d = 0; d < 3; ++d) {
            const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
            for (int s = 0; s < 2; ++s) {
                fid[d][s] = face_id[grp_of[6 * e + 2 * d + s]];
                out.elem_face[6 * e + 2 * d + s] = (int32_t)fid[d][s];
                int loc[4], n = 0;
                for (int v = 0; v < 8; ++v)
                    if (refc(v, d) == s) loc[n++] = v;
                int o = loc[0];
                for (int m = 1; m < 4; ++m)
                    if (gv[loc[m]] < gv[o]) o = loc[m];
                int nb[2], nn = 0;
                for (int m = 0; m < 4; ++m) {
                    const int v = loc[m];
                    int diff = 0;
                    for (int a = 0; a < 3; ++a) diff += refc(v, a) != refc(o, a);
                    if (diff == 1) nb[nn++] = v;
                }
                if (gv[nb[1]] < gv[nb[0]]) std::swap(nb[0], nb[1]);
                int a1[3], a2[3];
                for (int a = 0; a < 3; ++a) {
                    a1[a] = refc(nb[0], a) - refc(o, a);
                    a2[a] = refc(nb[1], a) - refc(o, a);
                }
                const int nrm[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                                    a1[0] * a2[1] - a1[1] * a2[0]};
                sig[d][s] = nrm[d] > 0 ? 1 : -1;
                const int* ax[2] = {a1, a2};
                for (int m = 0; m < 2; ++m) {
                    const int sr = ax[m][t0] != 0 ? 0 : 1;
                    const int tt = sr == 0 ? t0 : t1;
                    src[d][s][m] = sr;
                    rev[d][s][m] = ax[m][tt] < 0 ? 1 : 0;
                }
            }
        }
        int off = 0;
        for (int c = 0; c < 3; ++c) {
            const int t0 = c == 0 ? 1 : 0, t1 = c == 2 ? 1 : 2;
            const int shp[3] = {c == 0 ? P + 1 : P, c == 1 ? P + 1 : P, c == 2 ? P + 1 : P};
            for (int i2 = 0; i2 < shp[2]; ++i2)
                for (int i1 = 0; i1 < shp[1]; ++i1)
                    for (int i0 = 0; i0 < shp[0]; ++i0) {
                        const int idx[3] = {i0, i1, i2};
                        const int li = off + i0 + shp[0] * (i1 + shp[1] * i2);
                        const int ic = idx[c], j = idx[t0], k = idx[t1];
                        int32_t v;
                        if (ic == 0 || ic == P) {
                            const int s = ic == 0 ? 0 : 1;
                            const int jk[2] = {j, k};
                            int cn[2];
                            for (int m = 0; m < 2; ++m) {
                                const int w = jk[src[c][s][m]];
                                cn[m] = rev[c][s][m] ? P - 1 - w : w;
                            }
                            const int64_t gidx = fid[c][s] * P * P + cn[0] + (int64_t)P * cn[1];
                            v = sig[c][s] > 0 ? (int32_t)gidx : ~(int32_t)gidx;
                        } else {
                            v = (int32_t)(nfd + e * nint + (int64_t)c * (P - 1) * P * P + (ic - 1) +
                                          (int64_t)(P - 1) * (j + (int64_t)P * k));
                        }
                        out.l2g[(size_t)(e * NRT + li)] = v;
                    }
            off += shp[0] * shp[1] * shp[2];
        }
    }
    return HD_OK;
}

// For each L2 row (element e, sub-volume (a, b, c)) and each of its six face
// slots (2 d + side): the global RT dof and its sign in D (the local
// orientation, -1 on the lower and +1 on the upper face of the sub-volume,
// times the dof's sign in the element, Algorithm 1), and the sub-volume
// across that dof (-1 if none).
int build_unstructured_rows(const UnstructuredMap& m, int64_t ne, int P, std::vector<int32_t>& row_dof,
                            std::vector<int32_t>& row_nbr) {
    const int NL = P * P * P, NRT = 3 * P * P * (P + 1);
    const int64_t nq = ne * NL;
    row_dof.assign((size_t)(nq * 6), 0);
    row_nbr.assign((size_t)(nq * 6), -1);
    // the (at most two) sub-volumes of every RT dof
    std::vector<int32_t> vol0((size_t)m.n_u, -1), vol1((size_t)m.n_u, -1);
    const int offs[3] = {0, P * P * (P + 1), 2 * P * P * (P + 1)};
    for (int64_t e = 0; e < ne; ++e) {
        for (int l = 0; l < NL; ++l) {
            const int loc[3] = {l % P, (l / P) % P, l / (P * P)};
            const int64_t i = e * NL + l;
            for (int d = 0; d < 3; ++d) {
                const int shp0 = d == 0 ? P + 1 : P, shp1 = d == 1 ? P + 1 : P;
                for (int side = 0; side < 2; ++side) {
                    int idx[3] = {loc[0], loc[1], loc[2]};
                    idx[d] += side;
                    const int li = offs[d] + idx[0] + shp0 * (idx[1] + shp1 * idx[2]);
                    const int32_t v = m.l2g[(size_t)(e * NRT + li)];
                    const int32_t g = v < 0 ? ~v : v;
                    const int sgn = (v < 0 ? -1 : 1) * (side ? 1 : -1);
                    row_dof[(size_t)(6 * i + 2 * d + side)] = sgn > 0 ? g : ~g;
                    if (vol0[g] < 0) vol0[g] = (int32_t)i;
                    else vol1[g] = (int32_t)i;
                }
            }
        }
    }
    for (int64_t i = 0; i < nq; ++i)
        for (int s = 0; s < 6; ++s) {
            const int32_t v = row_dof[(size_t)(6 * i + s)];
            const int32_t g = v < 0 ? ~v : v;
            const int32_t o = vol0[g] == (int32_t)i ? vol1[g] : vol0[g];
            row_nbr[(size_t)(6 * i + s)] = o;
        }
    return HD_OK;
}

}  // namespace hd

// Host-only view of the numbering (no device): n_u and, if l2g is given,
// the element-to-dof map [ne][3 p^2 (p+1)] of hd_get_dof_map.
extern "C" int hd_host_unstructured_map(int64_t nv, int64_t ne, const int64_t* elements, int p, int64_t* n_u,
                                        int32_t* l2g) {
    if (!elements || p < 1 || p > 6) return HD_ERR_ARG;
    hd::UnstructuredMap m;
    std::string err;
    const int rc = hd::build_unstructured_numbering(nv, ne, elements, p, m, err);
    if (rc) return rc;
    if (n_u) *n_u = m.n_u;
    if (l2g) std::copy(m.l2g.begin(), m.l2g.end(), l2g);
    return HD_OK;
}
