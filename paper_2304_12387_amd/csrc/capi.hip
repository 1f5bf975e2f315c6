// extern "C" entry points of libhdivsp (declared in include/hdivsp.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "hd_internal.hpp"

// Fixed device storage of hd_apply_tri_precond_noalloc: the V-cycle output
// s = S^{-1} r_q (n_q values) that hd_apply_tri_precond allocates per call.
// Each device the library runs on holds its own copy for the life of the
// process.  In host code `scratch` is only a host-side stand-in for the
// symbol: its device address is looked up once per device, with that device
// current, in hd_create, and only that address is passed to kernels.
static constexpr int64_t NOALLOC_MAX_NQ = int64_t(1) << 24;
static __device__ __align__(256) double scratch[NOALLOC_MAX_NQ];

namespace {

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;   // per device ordinal; nullptr until looked up

// Device address of `scratch` on the current device `device` (looked up on
// the first call for that device).
int scratch_lookup(int device, double** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
    if (!g_scratch_dev[device]) {
        double* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HD_ERR_HIP;
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return HD_OK;
}

}  // namespace

namespace hd {

int set_err(hd_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

}  // namespace hd

using namespace hd;

namespace {

void free_mesh(hd_ctx* c) {
    dfree(c->d_pa);
    dfree(c->d_pa32);
    dfree(c->d_vert);
    dfree(c->d_evx);
    dfree(c->d_l2g);
    dfree(c->d_rdof);
    dfree(c->d_rnbr);
    dfree(c->d_essm);
    c->d_evx = nullptr;
    c->d_l2g = c->d_rdof = c->d_rnbr = nullptr;
    c->d_essm = nullptr;
    c->unstructured = false;
    c->u_boundary_dof.clear();
    dfree(c->d_theta);
    dfree(c->d_theta_net);
    c->d_theta_net = nullptr;
    c->d_pa = nullptr;
    c->d_pa32 = nullptr;
    c->d_vert = nullptr;
    c->d_theta = nullptr;
    c->theta_set = false;
    c->affine = false;
    c->have_mesh = false;
}

void free_coeffs(hd_ctx* c) {
    free_local_inverse(c);
    dfree(c->d_gv);
    dfree(c->d_gv32);
    dfree(c->d_ctil);
    c->d_gv = c->d_ctil = nullptr;
    c->d_gv32 = nullptr;
    c->gamma_field = false;
    dfree(c->d_cm);
    dfree(c->d_kap);
    dfree(c->d_cm32);
    dfree(c->d_kap32);
    c->d_cm = c->d_kap = nullptr;
    c->d_cm32 = c->d_kap32 = nullptr;
    c->have_coeffs = false;
}

void free_prec(hd_ctx* c) {
    free_levels(c);
    dfree(c->S.rp);
    dfree(c->S.ci);
    dfree(c->S.v);
    dfree(c->S.v32);
    c->S = DevCSR();
    dfree(c->d_mdiag);
    dfree(c->d_wdiag);
    dfree(c->d_mdinv);
    dfree(c->d_mdinv32);
    dfree(c->d_wface);
    dfree(c->d_sdiag);
    dfree(c->d_sdiag32);
    c->d_mdiag = c->d_wdiag = c->d_mdinv = c->d_wface = c->d_sdiag = nullptr;
    c->d_mdinv32 = c->d_sdiag32 = nullptr;
    c->have_prec = false;
}

int use_device(hd_ctx* c) {
    HD_HIP(c, hipSetDevice(c->device));
    return HD_OK;
}

// the essential-dof mask of an unstructured mesh (n_u bytes, host) to the
// device, and whether every boundary dof is essential (a singular S~ when
// C~ = 0, as with HD_SIDE_ALL on a box)
int upload_essential_mask(hd_ctx* c, const uint8_t* m) {
    if (!c->d_essm) c->d_essm = dalloc<uint8_t>(c->n_u);
    if (!c->d_essm) return set_err(c, HD_ERR_OOM, "essential mask");
    HD_HIP(c, hipMemcpy(c->d_essm, m, (size_t)c->n_u, hipMemcpyHostToDevice));
    bool all = true;
    for (int64_t i = 0; i < c->n_u; ++i)
        if (c->u_boundary_dof[i] && !m[i]) {
            all = false;
            break;
        }
    c->ess = all ? HD_SIDE_ALL : 0;
    return HD_OK;
}

__global__ void f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

int upload_f64_f32(hd_ctx* c, const double* host, int64_t n, double*& d64, float*& d32) {
    d64 = dalloc<double>(n);
    d32 = dalloc<float>(n);
    if (!d64 || !d32) return set_err(c, HD_ERR_OOM, "coefficient storage");
    HD_HIP(c, hipMemcpyAsync(d64, host, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(f64_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, d64, d32, n);
    HD_HIP(c, hipGetLastError());
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

hd_precond_params default_precond();

}  // namespace

void hd::batch_free(hd_ctx* c) {
    if (!c->batch) return;
    batch_union_free(c);
    BatchState* B = c->batch;
    for (hd_ctx* s : B->inst) hd_destroy(s);
    dfree(B->d_inst64);
    dfree(B->d_inst32);
    dfree(B->d_tiles);
    dfree(B->d_counter);
    dfree(B->d_part);
    delete B;
    c->batch = nullptr;
}

namespace {

hd_precond_params default_precond() {
    hd_precond_params p;
    p.tau = 1.0;
    p.theta = 0.25;
    p.max_coarse = 1024;
    p.max_levels = 25;
    p.omega = 2.0 / 3.0;
    p.learned = 0;
    return p;
}

}  // namespace

namespace hd {
namespace {
// Deterministic input in [-1, 1) for the tuner's timing applies (a zero
// input would end every local CG at once and time the mass part only).
template <typename T>
__global__ void tune_pattern_kernel(T* __restrict__ x, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = (T)((double)((uint32_t)(i * 2654435761u) >> 8) * (1.0 / 8388608.0) - 1.0);
}
}  // namespace
}  // namespace hd

namespace {

// Whether every element of the structured mesh is a parallelepiped: the
// bilinear and trilinear terms of its trilinear map (the twist vectors of
// its vertex cube) vanish to 1e-14 of its longest edge from vertex 0.
bool mesh_is_affine(int nx, int ny, int nz, const double* V) {
    auto X = [&](int64_t i, int64_t j, int64_t k, int r) {
        return V[3 * (i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k)) + r];
    };
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double scale = 0.0, twist = 0.0;
                for (int r = 0; r < 3; ++r) {
                    const double x000 = X(i, j, k, r), x100 = X(i + 1, j, k, r), x010 = X(i, j + 1, k, r),
                                 x001 = X(i, j, k + 1, r), x110 = X(i + 1, j + 1, k, r),
                                 x101 = X(i + 1, j, k + 1, r), x011 = X(i, j + 1, k + 1, r),
                                 x111 = X(i + 1, j + 1, k + 1, r);
                    scale = std::max({scale, std::fabs(x100 - x000), std::fabs(x010 - x000), std::fabs(x001 - x000)});
                    twist = std::max({twist, std::fabs(x110 - x100 - x010 + x000),
                                      std::fabs(x101 - x100 - x001 + x000), std::fabs(x011 - x010 - x001 + x000),
                                      std::fabs(x111 - x110 - x101 - x011 + x100 + x010 + x001 - x000)});
                }
                if (!(twist <= 1e-14 * scale)) return false;
            }
    return true;
}

}  // namespace

extern "C" {

int hd_create(hd_ctx** out, int device, void* stream) {
    if (!out) return HD_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HD_ERR_HIP;
    hd_ctx* c = new (std::nothrow) hd_ctx;
    if (!c) return HD_ERR_OOM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return HD_ERR_HIP;
    }
    c->d_scal = dalloc<double>(16);
    c->d_flag = dalloc<int>(4);
    if (!c->d_scal || !c->d_flag || hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return HD_ERR_HIP;
    }
    (void)hipMemset(c->d_scal, 0, 16 * sizeof(double));
    if (scratch_lookup(device, &c->d_noalloc) != HD_OK) {
        hd_destroy(c);
        return HD_ERR_HIP;
    }
    *out = c;
    return HD_OK;
}

int hd_destroy(hd_ctx* c) {
    if (!c) return HD_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->solve_cache) c->solve_cache_free(c->solve_cache);
    batch_free(c);
    rd_free(c);
    free_prec(c);
    free_coeffs(c);
    free_mesh(c);
    dfree(c->d_tab64);
    dfree(c->d_tab32);
    dfree(c->d_tabk64);
    dfree(c->d_tabk32);
    dfree(c->d_partial);
    dfree(c->d_scal);
    dfree(c->d_flag);
    dfree(c->d_mlp);
    dfree(c->d_adam_m);
    dfree(c->d_adam_v);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return HD_OK;
}

const char* hd_last_error(const hd_ctx* c) { return c ? c->err.c_str() : "null context"; }

int hd_setup_mesh(hd_ctx* c, int nx, int ny, int nz, int p, const double* vertices) {
    if (!c) return HD_ERR_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || !vertices) return set_err(c, HD_ERR_ARG, "bad mesh sizes");
    if (p < 1 || p > 6) return set_err(c, HD_ERR_ARG, "p must be in [1, 6]");
    int rc = use_device(c);
    if (rc) return rc;
    // everything built on the previous mesh goes (coefficients included: a
    // failed call below must not leave an apply-able state behind)
    rd_free(c);
    free_prec(c);
    free_coeffs(c);
    free_mesh(c);
    const int64_t nv = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(vertices[i])) return set_err(c, HD_ERR_NONFINITE, "non-finite vertex coordinate");
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->p = p;
    c->ne = (int64_t)nx * ny * nz;
    c->nface[0] = (int64_t)(nx * p + 1) * (ny * p) * (nz * p);
    c->nface[1] = (int64_t)(nx * p) * (ny * p + 1) * (nz * p);
    c->nface[2] = (int64_t)(nx * p) * (ny * p) * (nz * p + 1);
    c->n_u = c->nface[0] + c->nface[1] + c->nface[2];
    c->n_q = c->ne * p * p * p;
    if (c->n_u + c->n_q > (int64_t)INT32_MAX) return set_err(c, HD_ERR_ARG, "problem too large for 32-bit indices");
    Tables<double>& t64 = c->tab64_host;
    Tables<float>& t32 = c->tab32_host;
    build_tables(p, t64, t32);
    if (!c->d_tab64) c->d_tab64 = dalloc<Tables<double>>(1);
    if (!c->d_tab32) c->d_tab32 = dalloc<Tables<float>>(1);
    if (!c->d_tab64 || !c->d_tab32) return set_err(c, HD_ERR_OOM, "tables");
    HD_HIP(c, hipMemcpyAsync(c->d_tab64, &t64, sizeof(t64), hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemcpyAsync(c->d_tab32, &t32, sizeof(t32), hipMemcpyHostToDevice, c->stream));
    if ((rc = upload_kernel_tables(c))) return rc;
    const int64_t q3 = (int64_t)(p + 1) * (p + 1) * (p + 1);
    c->d_pa = dalloc<double>(c->ne * NPA * q3);
    c->d_pa32 = dalloc<float>(c->ne * NPA * q3);
    double* dv = dalloc<double>(3 * nv);
    if (!c->d_pa || !c->d_pa32 || !dv) {
        dfree(dv);
        return set_err(c, HD_ERR_OOM, "geometric factors");
    }
    HD_HIP(c, hipMemcpyAsync(dv, vertices, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    rc = launch_geometry(c, dv, c->d_flag);
    int bad = 0;
    if (!rc) {
        HD_HIP(c, hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HD_HIP(c, hipStreamSynchronize(c->stream));
    }
    c->d_vert = dv;
    if (rc) return rc;
    if (bad) {
        free_mesh(c);
        return set_err(c, HD_ERR_MESH, "Jacobian determinant <= 0 in some element");
    }
    rc = launch_ensure_partial(c, c->ne);
    if (rc) return rc;
    c->affine = mesh_is_affine(nx, ny, nz, vertices);
    c->have_mesh = true;
    c->have_coeffs = false;
    return HD_OK;
}

int hd_setup_coeffs(hd_ctx* c, int problem, const double* c_mass, const double* c_22, uint32_t ess_sides) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_mesh) return set_err(c, HD_ERR_STATE, "hd_setup_mesh first");
    if (problem != HD_GRADDIV && problem != HD_DARCY) return set_err(c, HD_ERR_ARG, "unknown problem");
    if (!c_mass) return set_err(c, HD_ERR_ARG, "c_mass required");
    if (problem == HD_GRADDIV && !c_22) return set_err(c, HD_ERR_ARG, "grad-div needs alpha (c_22)");
    if (ess_sides > 63) return set_err(c, HD_ERR_ARG, "ess_sides must be a 6-bit mask");
    if (c->unstructured && ess_sides != 0 && ess_sides != HD_SIDE_ALL)
        return set_err(c, HD_ERR_ARG, "on an unstructured mesh ess_sides is 0 or HD_SIDE_ALL (every boundary face)");
    int rc = use_device(c);
    if (rc) return rc;
    const int64_t ne = c->ne;
    std::vector<double> kap(ne, 0.0);
    for (int64_t e = 0; e < ne; ++e) {
        if (!std::isfinite(c_mass[e]) || (c_22 && !std::isfinite(c_22[e])))
            return set_err(c, HD_ERR_NONFINITE, "non-finite coefficient");
        if (!(c_mass[e] > 0)) return set_err(c, HD_ERR_ARG, "c_mass must be positive");
        if (problem == HD_GRADDIV) {
            if (!(c_22[e] > 0)) return set_err(c, HD_ERR_ARG, "alpha must be positive");
            kap[e] = 1.0 / c_22[e];
        } else if (c_22) {
            if (c_22[e] < 0) return set_err(c, HD_ERR_ARG, "gamma must be non-negative");
            kap[e] = c_22[e];
        }
    }
    rd_free(c);
    free_prec(c);
    free_coeffs(c);
    c->problem = problem;
    c->ess = ess_sides;
    c->kappa_zero = true;
    for (double k : kap)
        if (k != 0.0) c->kappa_zero = false;
    if ((rc = upload_f64_f32(c, c_mass, ne, c->d_cm, c->d_cm32))) return rc;
    if ((rc = upload_f64_f32(c, kap.data(), ne, c->d_kap, c->d_kap32))) return rc;
    if ((rc = build_local_inverse(c))) return rc;
    if (c->unstructured) {
        std::vector<uint8_t> m(c->n_u, 0);
        if (ess_sides == HD_SIDE_ALL) m = c->u_boundary_dof;
        if ((rc = upload_essential_mask(c, m.data()))) return rc;
    }
    c->have_coeffs = true;
    return HD_OK;
}

int hd_setup_mesh_unstructured(hd_ctx* c, int64_t nv, const double* vertices, int64_t ne, const int64_t* elements,
                               int p) {
    if (!c) return HD_ERR_ARG;
    if (nv < 8 || ne < 1 || !vertices || !elements) return set_err(c, HD_ERR_ARG, "bad mesh sizes");
    if (p < 1 || p > 6) return set_err(c, HD_ERR_ARG, "p must be in [1, 6]");
    if (ne > (int64_t)INT32_MAX / 8) return set_err(c, HD_ERR_ARG, "too many elements");
    int rc = use_device(c);
    if (rc) return rc;
    rd_free(c);
    free_prec(c);
    free_coeffs(c);
    free_mesh(c);
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(vertices[i])) return set_err(c, HD_ERR_NONFINITE, "non-finite vertex coordinate");
    UnstructuredMap m;
    std::string err;
    if ((rc = build_unstructured_numbering(nv, ne, elements, p, m, err))) return set_err(c, rc, err);
    std::vector<int32_t> rdof, rnbr;
    build_unstructured_rows(m, ne, p, rdof, rnbr);
    // element vertex coordinates [ne][8][3]
    std::vector<double> evx((size_t)(24 * ne));
    for (int64_t e = 0; e < ne; ++e)
        for (int v = 0; v < 8; ++v)
            for (int r = 0; r < 3; ++r) evx[(size_t)(24 * e + 3 * v + r)] = vertices[3 * elements[8 * e + v] + r];
    c->unstructured = true;
    c->nx = (int)ne;   // the element count as an nx x 1 x 1 grid for the element-local kernels
    c->ny = c->nz = 1;
    c->p = p;
    c->ne = ne;
    c->n_u = m.n_u;
    c->n_q = m.n_q;
    c->n_face_dofs = m.n_face_dofs;
    c->nface[0] = m.n_u;
    c->nface[1] = c->nface[2] = 0;
    c->u_boundary_dof.assign((size_t)m.n_u, 0);
    for (int64_t f = 0; f < m.nfaces; ++f)
        if (m.boundary_face[f])
            for (int k = 0; k < p * p; ++k) c->u_boundary_dof[(size_t)(f * p * p + k)] = 1;
    Tables<double>& t64 = c->tab64_host;
    Tables<float>& t32 = c->tab32_host;
    build_tables(p, t64, t32);
    if (!c->d_tab64) c->d_tab64 = dalloc<Tables<double>>(1);
    if (!c->d_tab32) c->d_tab32 = dalloc<Tables<float>>(1);
    if (!c->d_tab64 || !c->d_tab32) return set_err(c, HD_ERR_OOM, "tables");
    HD_HIP(c, hipMemcpyAsync(c->d_tab64, &t64, sizeof(t64), hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemcpyAsync(c->d_tab32, &t32, sizeof(t32), hipMemcpyHostToDevice, c->stream));
    if ((rc = upload_kernel_tables(c))) return rc;
    const int64_t q3 = (int64_t)(p + 1) * (p + 1) * (p + 1);
    c->d_pa = dalloc<double>(ne * NPA * q3);
    c->d_pa32 = dalloc<float>(ne * NPA * q3);
    c->d_evx = dalloc<double>(24 * ne);
    c->d_l2g = dalloc<int32_t>(m.l2g.size());
    c->d_rdof = dalloc<int32_t>(rdof.size());
    c->d_rnbr = dalloc<int32_t>(rnbr.size());
    if (!c->d_pa || !c->d_pa32 || !c->d_evx || !c->d_l2g || !c->d_rdof || !c->d_rnbr) {
        free_mesh(c);
        return set_err(c, HD_ERR_OOM, "unstructured mesh arrays");
    }
    HD_HIP(c, hipMemcpyAsync(c->d_evx, evx.data(), sizeof(double) * evx.size(), hipMemcpyHostToDevice, c->stream));
    HD_HIP(c, hipMemcpyAsync(c->d_l2g, m.l2g.data(), sizeof(int32_t) * m.l2g.size(), hipMemcpyHostToDevice,
                             c->stream));
    HD_HIP(c, hipMemcpyAsync(c->d_rdof, rdof.data(), sizeof(int32_t) * rdof.size(), hipMemcpyHostToDevice,
                             c->stream));
    HD_HIP(c, hipMemcpyAsync(c->d_rnbr, rnbr.data(), sizeof(int32_t) * rnbr.size(), hipMemcpyHostToDevice,
                             c->stream));
    HD_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    rc = launch_geometry(c, nullptr, c->d_flag);
    int bad = 0;
    if (!rc) {
        HD_HIP(c, hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HD_HIP(c, hipStreamSynchronize(c->stream));
    }
    if (rc) {
        free_mesh(c);
        return rc;
    }
    if (bad) {
        free_mesh(c);
        return set_err(c, HD_ERR_MESH, "Jacobian determinant <= 0 in some element");
    }
    if ((rc = launch_ensure_partial(c, std::max<int64_t>(c->ne, apply_partial_count(c))))) return rc;
    c->have_mesh = true;
    c->have_coeffs = false;
    return HD_OK;
}

int hd_set_essential_dofs(hd_ctx* c, const uint8_t* mask) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_coeffs || !c->unstructured)
        return set_err(c, HD_ERR_STATE, "hd_setup_mesh_unstructured and hd_setup_coeffs first");
    if (!mask) return set_err(c, HD_ERR_ARG, "mask required");
    int rc = use_device(c);
    if (rc) return rc;
    free_prec(c);
    std::vector<uint8_t> m(mask, mask + c->n_u);
    for (auto& b : m) b = b ? 1 : 0;
    return upload_essential_mask(c, m.data());
}

int hd_get_dof_map(hd_ctx* c, int32_t* l2g) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_mesh || !c->unstructured) return set_err(c, HD_ERR_STATE, "hd_setup_mesh_unstructured first");
    if (!l2g) return set_err(c, HD_ERR_ARG, "l2g required");
    int rc = use_device(c);
    if (rc) return rc;
    const int64_t nrt = 3LL * c->p * c->p * (c->p + 1);
    HD_HIP(c, hipMemcpy(l2g, c->d_l2g, sizeof(int32_t) * nrt * c->ne, hipMemcpyDeviceToHost));
    return HD_OK;
}

int hd_set_gamma_field(hd_ctx* c, const double* gv) {
    if (!c) return HD_ERR_ARG;
    if (c->unstructured) return set_err(c, HD_ERR_STATE, "gamma fields need a structured mesh");
    if (!c->have_coeffs || c->problem != HD_DARCY) return set_err(c, HD_ERR_STATE, "hd_setup_coeffs(HD_DARCY, ...) first");
    if (!gv) return set_err(c, HD_ERR_ARG, "gamma_vertices required");
    const int64_t nv = (int64_t)(c->nx + 1) * (c->ny + 1) * (c->nz + 1);
    bool any = false;
    for (int64_t i = 0; i < nv; ++i) {
        if (!std::isfinite(gv[i])) return set_err(c, HD_ERR_NONFINITE, "non-finite gamma value");
        if (gv[i] < 0) return set_err(c, HD_ERR_ARG, "gamma must be non-negative");
        if (gv[i] > 0) any = true;
    }
    if (!any) return set_err(c, HD_ERR_ARG, "an all-zero gamma field: use hd_setup_coeffs with gamma = 0");
    int rc = use_device(c);
    if (rc) return rc;
    // new arrays first; the context changes only once all of them exist
    double *gv64 = nullptr, *kap64 = nullptr, *ctil = nullptr;
    float *gv32 = nullptr, *kap32 = nullptr;
    std::vector<double> ones(c->ne, 1.0);
    rc = upload_f64_f32(c, gv, nv, gv64, gv32);
    if (!rc) rc = upload_f64_f32(c, ones.data(), c->ne, kap64, kap32);
    if (!rc) {
        ctil = dalloc<double>(c->n_q);
        if (!ctil) rc = set_err(c, HD_ERR_OOM, "C~ of the gamma field");
    }
    if (rc) {
        for (double* p : {gv64, kap64, ctil}) dfree(p);
        for (float* p : {gv32, kap32}) dfree(p);
        return rc;
    }
    free_prec(c);
    dfree(c->d_gv);
    dfree(c->d_gv32);
    dfree(c->d_ctil);
    dfree(c->d_kap);
    dfree(c->d_kap32);
    c->d_gv = gv64;
    c->d_gv32 = gv32;
    c->d_ctil = ctil;
    // kappa = 1: the (2,2) block is W^{-1} W_gamma W^{-1} itself
    c->d_kap = kap64;
    c->d_kap32 = kap32;
    c->kappa_zero = false;
    c->gamma_field = true;
    return build_local_inverse(c);
}

int hd_set_local_solver(hd_ctx* c, int mode) {
    if (!c) return HD_ERR_ARG;
    if (mode != HD_LOCAL_AUTO && mode != HD_LOCAL_CG && mode != HD_LOCAL_EXPLICIT)
        return set_err(c, HD_ERR_ARG, "unknown local solver mode");
    if (mode == HD_LOCAL_EXPLICIT && c->have_mesh && c->p > 2)
        return set_err(c, HD_ERR_ARG, "explicit element inverses are for p <= 2");
    int rc = use_device(c);
    if (rc) return rc;
    c->local_solver = mode;
    if (c->have_coeffs) return build_local_inverse(c);
    return HD_OK;
}

int hd_sizes(const hd_ctx* c, int64_t* n_u, int64_t* n_q) {
    if (!c || !c->have_mesh) return HD_ERR_STATE;
    if (n_u) *n_u = c->n_u;
    if (n_q) *n_q = c->n_q;
    return HD_OK;
}

int hd_mesh_affine(const hd_ctx* c, int* affine) {
    if (!c || !affine) return HD_ERR_ARG;
    if (!c->have_mesh) return HD_ERR_STATE;
    *affine = c->affine ? 1 : 0;
    return HD_OK;
}

int hd_apply_block_op(hd_ctx* c, int prec, int nrhs, const void* x, void* y) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_coeffs) return set_err(c, HD_ERR_STATE, "mesh and coefficients first");
    if (nrhs < 1) return set_err(c, HD_ERR_ARG, "nrhs must be >= 1");
    if (prec != HD_F64 && prec != HD_F32) return set_err(c, HD_ERR_ARG, "prec");
    if (!x || !y || x == y) return set_err(c, HD_ERR_ARG, "x, y must be distinct device pointers");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_apply(c, prec, nrhs, x, y, nullptr, 0, nullptr, 0, ESS_IDENTITY, nullptr, 0);
}

int hd_apply_block_op_interleaved(hd_ctx* c, int prec, int nrhs, const void* x, void* y) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_coeffs) return set_err(c, HD_ERR_STATE, "mesh and coefficients first");
    if (c->unstructured || c->gamma_field)
        return set_err(c, HD_ERR_STATE, "the interleaved layout needs a structured mesh without a gamma field");
    if (nrhs < 1) return set_err(c, HD_ERR_ARG, "nrhs must be >= 1");
    if ((int64_t)nrhs * (c->n_u + c->n_q) > (int64_t)INT32_MAX * 4)
        return set_err(c, HD_ERR_ARG, "nrhs too large");
    if (prec != HD_F64 && prec != HD_F32) return set_err(c, HD_ERR_ARG, "prec");
    if (!x || !y || x == y) return set_err(c, HD_ERR_ARG, "x, y must be distinct device pointers");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_apply_interleaved(c, prec, nrhs, x, y);
}

int hd_apply_mass_inverse(hd_ctx* c, int prec, int nrhs, const void* x, void* y) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_coeffs) return set_err(c, HD_ERR_STATE, "mesh and coefficients first");
    if (c->gamma_field) return set_err(c, HD_ERR_STATE, "not defined for a gamma field");
    if (nrhs < 1) return set_err(c, HD_ERR_ARG, "nrhs must be >= 1");
    if (prec != HD_F64 && prec != HD_F32) return set_err(c, HD_ERR_ARG, "prec");
    if (!x || !y) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
    for (int r = 0; r < nrhs; ++r) {
        const size_t off = es * (size_t)c->n_q * r;
        if ((rc = launch_mass_inverse(c, prec, (const char*)x + off, (char*)y + off, true))) return rc;
    }
    return HD_OK;
}

int hd_apply_l2_mass_inverse(hd_ctx* c, int prec, const void* x, void* y) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_mesh || !c->d_kap) return set_err(c, HD_ERR_STATE, "mesh and coefficients first");
    if (!x || !y) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_mass_inverse(c, prec, x, y, false);
}

int hd_lift_essential(hd_ctx* c, const double* u_bc, double* b) {
    if (!c) return HD_ERR_ARG;
    if (c->unstructured) return set_err(c, HD_ERR_STATE, "hd_lift_essential works on structured box meshes");
    if (!c->have_coeffs) return set_err(c, HD_ERR_STATE, "mesh and coefficients first");
    if (!u_bc || !b) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_lift(c, u_bc, b);
}

int hd_constant_flux(hd_ctx* c, const double* u, double* dofs) {
    if (!c) return HD_ERR_ARG;
    if (c->unstructured) return set_err(c, HD_ERR_STATE, "hd_constant_flux works on structured box meshes");
    if (!c->have_mesh) return set_err(c, HD_ERR_STATE, "hd_setup_mesh first");
    if (!u || !dofs) return set_err(c, HD_ERR_ARG, "null pointer");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(u[d])) return set_err(c, HD_ERR_NONFINITE, "non-finite field");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_constant_flux(c, u, dofs);
}

int hd_build_precond(hd_ctx* c, const hd_precond_params* params) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_coeffs) return set_err(c, HD_ERR_STATE, "mesh and coefficients first");
    hd_precond_params prm = params ? *params : default_precond();
    if (!(prm.tau > 0) || !(prm.theta >= 0) || prm.max_coarse < 1 || prm.max_levels < 1 || !(prm.omega > 0) ||
        prm.learned < 0 || prm.learned > 2)
        return set_err(c, HD_ERR_ARG, "bad preconditioner parameters");
    if (prm.learned != 0 && c->unstructured) return set_err(c, HD_ERR_STATE, "the learned diagonal needs a structured mesh");
    if (prm.learned == 1 && !c->mlp_ready) return set_err(c, HD_ERR_STATE, "learned diagonal needs a network");
    if (prm.learned == 2 && !c->theta_set) return set_err(c, HD_ERR_STATE, "hd_set_diag_scalings first");
    int rc = use_device(c);
    if (rc) return rc;
    free_prec(c);
    c->fallback_used = false;
    const double* theta = nullptr;
    if (prm.learned == 1) {
        int fb = 0;
        if ((rc = learned_mesh_theta(c, &fb))) return rc;
        if (fb) c->fallback_used = true;
        else theta = c->d_theta_net;
    } else if (prm.learned == 2) {
        theta = c->d_theta;
    }
    c->tau = prm.tau;
    c->d_mdiag = dalloc<double>(c->n_u);
    c->d_mdinv = dalloc<double>(c->n_u);
    c->d_mdinv32 = dalloc<float>(c->n_u);
    c->d_wdiag = dalloc<double>(c->n_q);
    c->d_wface = dalloc<double>(c->n_u);
    c->d_sdiag = dalloc<double>(c->n_q);
    c->d_sdiag32 = dalloc<float>(c->n_q);
    if (!c->d_mdiag || !c->d_mdinv || !c->d_mdinv32 || !c->d_wdiag || !c->d_wface || !c->d_sdiag ||
        !c->d_sdiag32)
        return set_err(c, HD_ERR_OOM, "diagonals");
    if ((rc = launch_diagonals(c, theta))) return rc;
    if ((rc = launch_schur(c))) return rc;
    // S~ is singular when C~ = 0 and every boundary face is essential
    c->singular = c->kappa_zero && c->ess == HD_SIDE_ALL;
    // the AMG hierarchy of S~, built on the device
    if ((rc = build_amg_gpu(c, prm))) return rc;
    if ((rc = finish_levels(c))) return rc;
    // the V-cycle's partial sums (singular S~): sized here so that applying
    // the preconditioner never allocates
    if ((rc = launch_ensure_partial(c, schur_partial_count(c)))) return rc;
    c->have_prec = true;
    if (c->fallback_used) {
        c->err = "learned scalings not finite: plain diagonal used";
        return HD_FALLBACK_USED;
    }
    return HD_OK;
}

int hd_apply_precond(hd_ctx* c, int prec, int nrhs, const void* r, void* z) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (nrhs < 1) return set_err(c, HD_ERR_ARG, "nrhs must be >= 1");
    if (prec != HD_F64 && prec != HD_F32) return set_err(c, HD_ERR_ARG, "prec");
    if (!r || !z || r == z) return set_err(c, HD_ERR_ARG, "r, z must be distinct device pointers");
    int rc = use_device(c);
    if (rc) return rc;
    const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
    for (int k = 0; k < nrhs; ++k) {
        const size_t off = es * (size_t)(c->n_u + c->n_q) * k;
        if ((rc = launch_precond(c, prec, (const char*)r + off, (char*)z + off, nullptr, nullptr, nullptr))) return rc;
    }
    return HD_OK;
}

int hd_apply_tri_precond_noalloc(hd_ctx* c, const double* r, double* z) {
    if (!c) return HD_ERR_ARG;
    if (c->unstructured) return set_err(c, HD_ERR_STATE, "the block-triangular preconditioner needs a structured mesh");
    if (!c->have_mesh) return set_err(c, HD_ERR_STATE, "hd_setup_mesh first");
    if (c->n_q > NOALLOC_MAX_NQ)
        return set_err(c, HD_ERR_ARG, "n_q = " + std::to_string(c->n_q) + " exceeds the fixed scratch of " +
                                          std::to_string(NOALLOC_MAX_NQ) + " values");
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (!r || !z || r == z) return set_err(c, HD_ERR_ARG, "r, z must be distinct device pointers");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_tri_precond(c, r, z, c->d_noalloc);
}

int hd_gmres_solve(hd_ctx* c, double tol, int max_it, int restart, const double* b, double* x,
                   hd_solve_info* info) {
    if (!c) return HD_ERR_ARG;
    if (c->unstructured) return set_err(c, HD_ERR_STATE, "the block-triangular preconditioner needs a structured mesh");
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (!b || !x || b == x) return set_err(c, HD_ERR_ARG, "b, x must be distinct device pointers");
    if (!(tol > 0) || max_it < 1 || restart < 1 || restart > 500) return set_err(c, HD_ERR_ARG, "bad GMRES parameters");
    int rc = use_device(c);
    if (rc) return rc;
    return gmres_solve(c, tol, max_it, restart, b, x, info);
}

int hd_apply_tri_precond(hd_ctx* c, const double* r, double* z) {
    if (!c) return HD_ERR_ARG;
    if (c->unstructured) return set_err(c, HD_ERR_STATE, "the block-triangular preconditioner needs a structured mesh");
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (!r || !z || r == z) return set_err(c, HD_ERR_ARG, "r, z must be distinct device pointers");
    int rc = use_device(c);
    if (rc) return rc;
    double* s = dalloc<double>(c->n_q);
    if (!s) return set_err(c, HD_ERR_OOM, "scratch");
    rc = launch_tri_precond(c, r, z, s);
    (void)hipStreamSynchronize(c->stream);
    dfree(s);
    return rc;
}

int hd_minres_solve(hd_ctx* c, const hd_solve_params* params, int nrhs, const double* b, double* x,
                    hd_solve_info* info) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (nrhs < 1) return set_err(c, HD_ERR_ARG, "nrhs must be >= 1");
    if (!b || !x || b == x) return set_err(c, HD_ERR_ARG, "b, x must be distinct device pointers");
    hd_solve_params prm;
    if (params) prm = *params;
    else {
        prm.tol = 1e-8;
        prm.max_it = 10000;
        prm.mode = HD_MODE_PLAIN64;
        prm.use_x0 = 0;
        prm.inner_tol = 1e-5;
        prm.max_outer = 20;
        prm.check_every = 8;
        prm.stop_true = 0;
        prm.use_graph = 1;
    }
    if (!(prm.tol > 0) || prm.max_it < 1) return set_err(c, HD_ERR_ARG, "bad solve parameters");
    if (prm.mode == HD_MODE_MIXED && (!(prm.inner_tol > 0) || prm.max_outer < 1))
        return set_err(c, HD_ERR_ARG, "bad refinement parameters");
    int rc = use_device(c);
    if (rc) return rc;
    rc = minres_solve(c, prm, nrhs, b, x, info);
    if (rc == HD_NOT_CONVERGED) c->err = "MINRES did not reach the tolerance";
    return rc;
}

int hd_apply_divergence(hd_ctx* c, const double* F, double* q) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_mesh) return set_err(c, HD_ERR_STATE, "a mesh first");
    if (!F || !q) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_divergence(c, F, q);
}

int hd_subcell_volumes(hd_ctx* c, double* vol) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_mesh) return set_err(c, HD_ERR_STATE, "a mesh first");
    if (!vol) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_subcell_volumes(c, vol);
}

int hd_rd_default_params(hd_rd_params* p) {
    if (!p) return HD_ERR_ARG;
    p->rho = p->cv = p->c = p->a = p->sigma = p->dt = 1.0;
    p->tol_outer = 1e-10;
    p->max_outer = 20;
    p->newton_tol = 1e-12;
    p->newton_max_it = 50;
    p->lin_tol = 1e-8;
    p->lin_max_it = 10000;
    p->lin_mode = HD_MODE_PLAIN64;
    return HD_OK;
}

int hd_rd_setup(hd_ctx* c, const hd_rd_params* prm, const hd_precond_params* pp) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_mesh) return set_err(c, HD_ERR_STATE, "a mesh first");
    if (!prm) return set_err(c, HD_ERR_ARG, "null parameters");
    const double pos[] = {prm->rho, prm->cv, prm->c, prm->a, prm->sigma, prm->dt, prm->tol_outer, prm->newton_tol,
                          prm->lin_tol};
    for (double v : pos)
        if (!(v > 0) || !std::isfinite(v)) return set_err(c, HD_ERR_ARG, "parameters must be positive and finite");
    if (prm->max_outer < 1 || prm->newton_max_it < 1 || prm->lin_max_it < 1 || prm->lin_mode < HD_MODE_PLAIN64 ||
        prm->lin_mode > HD_MODE_PREC32)
        return set_err(c, HD_ERR_ARG, "bad iteration limits or mode");
    int rc = use_device(c);
    if (rc) return rc;
    return rd_setup(c, *prm, pp);
}

int hd_rd_step(hd_ctx* c, double* e, double* E, double* F, hd_rd_info* info) {
    if (!c) return HD_ERR_ARG;
    if (!c->rd || !c->have_prec) return set_err(c, HD_ERR_STATE, "hd_rd_setup first");
    if (!e || !E || !F || e == E || (void*)e == (void*)F || (void*)E == (void*)F)
        return set_err(c, HD_ERR_ARG, "e, E, F must be distinct device pointers");
    int rc = use_device(c);
    if (rc) return rc;
    return rd_step(c, e, E, F, info);
}

int hd_learned_targets(hd_ctx* c, int p, int64_t n, const double* vertices, int max_steps, double* theta,
                       double* lam, double* spread) {
    if (!c) return HD_ERR_ARG;
    if (p < 1 || p > 6) return set_err(c, HD_ERR_ARG, "p must be in 1..6");
    if (n < 0 || max_steps < 0) return set_err(c, HD_ERR_ARG, "bad sizes");
    if (n == 0) return HD_OK;
    if (!vertices || !theta) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_targets(c, p, n, vertices, max_steps, theta, lam, spread);
}

int hd_learned_features(hd_ctx* c, int64_t n, const double* vertices, const double* alpha, const double* beta,
                        const int* p_per_elem, int p, float* x) {
    if (!c) return HD_ERR_ARG;
    if (n < 0) return set_err(c, HD_ERR_ARG, "bad size");
    if (n == 0) return HD_OK;
    if (!vertices || !alpha || !beta || !x) return set_err(c, HD_ERR_ARG, "null pointer");
    if (!p_per_elem && (p < 1 || p > 6)) return set_err(c, HD_ERR_ARG, "p must be in 1..6");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_features(c, n, vertices, alpha, beta, p_per_elem, p, x);
}

int hd_mlp_param_count(void) { return mlp_param_count(); }

int hd_mlp_init(hd_ctx* c, uint64_t seed) {
    if (!c) return HD_ERR_ARG;
    int rc = use_device(c);
    if (rc) return rc;
    return mlp_init(c, seed);
}

int hd_mlp_set_params(hd_ctx* c, const float* params) {
    if (!c) return HD_ERR_ARG;
    if (!params) return set_err(c, HD_ERR_ARG, "null pointer");
    for (int i = 0; i < mlp_param_count(); ++i)
        if (!std::isfinite(params[i])) return set_err(c, HD_ERR_NONFINITE, "non-finite network parameter");
    int rc = use_device(c);
    if (rc) return rc;
    return mlp_set(c, params);
}

int hd_mlp_get_params(hd_ctx* c, float* params) {
    if (!c) return HD_ERR_ARG;
    if (!params) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    return mlp_get(c, params);
}

int hd_mlp_loss_grad(hd_ctx* c, int64_t n, const float* x, const float* y, float* loss, float* grad) {
    if (!c) return HD_ERR_ARG;
    if (n < 1 || !x || !y) return set_err(c, HD_ERR_ARG, "bad arguments");
    int rc = use_device(c);
    if (rc) return rc;
    return mlp_loss_grad(c, n, x, y, loss, grad);
}

int hd_mlp_train(hd_ctx* c, int64_t n, const float* x, const float* y, int64_t n_val, const float* x_val,
                 const float* y_val, int epochs, int batch, float lr, uint64_t seed, float* train_loss,
                 float* val_loss) {
    if (!c) return HD_ERR_ARG;
    if (n < 1 || !x || !y || epochs < 0 || batch < 1 || batch > n || !(lr > 0) || n > INT32_MAX)
        return set_err(c, HD_ERR_ARG, "bad training arguments");
    if (n_val < 0 || (n_val > 0 && (!x_val || !y_val))) return set_err(c, HD_ERR_ARG, "bad validation arguments");
    int rc = use_device(c);
    if (rc) return rc;
    return mlp_train(c, n, x, y, n_val, x_val, y_val, epochs, batch, lr, seed, train_loss, val_loss);
}

int hd_mlp_infer(hd_ctx* c, int64_t n, const float* x, float* theta, int bf16) {
    if (!c) return HD_ERR_ARG;
    if (n < 0) return set_err(c, HD_ERR_ARG, "bad size");
    if (n == 0) return HD_OK;
    if (!x || !theta) return set_err(c, HD_ERR_ARG, "null pointer");
    int rc = use_device(c);
    if (rc) return rc;
    return mlp_infer(c, n, x, theta, bf16);
}

int hd_set_diag_scalings(hd_ctx* c, const double* theta) {
    if (!c) return HD_ERR_ARG;
    if (c->unstructured) return set_err(c, HD_ERR_STATE, "the learned diagonal needs a structured mesh");
    if (!c->have_mesh) return set_err(c, HD_ERR_STATE, "hd_setup_mesh first");
    int rc = use_device(c);
    if (rc) return rc;
    if (!theta) {
        c->theta_set = false;
        return HD_OK;
    }
    if (!c->d_theta) c->d_theta = dalloc<double>(c->ne * 6);
    if (!c->d_theta) return set_err(c, HD_ERR_OOM, "scalings");
    HD_HIP(c, hipMemcpyAsync(c->d_theta, theta, sizeof(double) * c->ne * 6, hipMemcpyDeviceToDevice, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    c->theta_set = true;
    return HD_OK;
}

int hd_setup_batch(hd_ctx* c, int problem, int ninst, const hd_instance_desc* d) {
    if (!c) return HD_ERR_ARG;
    if (ninst < 1 || !d) return set_err(c, HD_ERR_ARG, "at least one instance required");
    int rc = use_device(c);
    if (rc) return rc;
    batch_free(c);
    BatchState* B = new (std::nothrow) BatchState;
    if (!B) return set_err(c, HD_ERR_OOM, "batch");
    c->batch = B;
    B->off.push_back(0);
    for (int i = 0; i < ninst && !rc; ++i) {
        hd_ctx* s = nullptr;
        if ((rc = hd_create(&s, c->device, (void*)c->stream))) {
            rc = set_err(c, rc, "instance context");
            break;
        }
        B->inst.push_back(s);
        if (d[i].p < 1 || d[i].p > 6) rc = set_err(c, HD_ERR_ARG, "instance " + std::to_string(i) + ": p must be in 1..6");
        else if ((rc = hd_setup_mesh(s, d[i].nx, d[i].ny, d[i].nz, d[i].p, d[i].vertices)) ||
                 (rc = hd_setup_coeffs(s, problem, d[i].c_mass, d[i].c_22, d[i].ess_sides)))
            rc = set_err(c, rc, "instance " + std::to_string(i) + ": " + s->err);
        else {
            // the work-queue launches form the factors point by point; the
            // instance's own launches do the same, so that every launch mode
            // gives the same result bit for bit
            s->affine = false;
            B->off.push_back(B->off.back() + s->n_u + s->n_q);
        }
    }
    if (!rc) {
        B->total = B->off.back();
        int64_t np = 0;
        for (hd_ctx* s : B->inst) {
            B->part_off.push_back(np);
            np += apply_partial_count(s);
        }
        B->d_part = dalloc<double>(np);
        B->d_counter = dalloc<int>(16);
        if (!B->d_part || !B->d_counter) rc = set_err(c, HD_ERR_OOM, "batch work queue");
    }
    if (!rc) {
        B->grid = 2048;
        B->mode = 0;
        rc = batch_build_tiles(c, 1);
    }
    if (rc) batch_free(c);
    return rc;
}

int hd_batch_sizes(hd_ctx* c, int64_t* offsets, int64_t* n_u) {
    if (!c) return HD_ERR_ARG;
    if (!c->batch) return set_err(c, HD_ERR_STATE, "hd_setup_batch first");
    const BatchState& B = *c->batch;
    for (size_t i = 0; i < B.inst.size(); ++i) {
        if (offsets) offsets[i] = B.off[i];
        if (n_u) n_u[i] = B.inst[i]->n_u;
    }
    if (offsets) offsets[B.inst.size()] = B.total;
    return HD_OK;
}

int hd_batch_apply(hd_ctx* c, int prec, const void* x, void* y) {
    if (!c) return HD_ERR_ARG;
    if (!c->batch) return set_err(c, HD_ERR_STATE, "hd_setup_batch first");
    if (prec != HD_F64 && prec != HD_F32) return set_err(c, HD_ERR_ARG, "prec");
    if (!x || !y || x == y) return set_err(c, HD_ERR_ARG, "x, y must be distinct device pointers");
    int rc = use_device(c);
    if (rc) return rc;
    return launch_batch_apply(c, prec, x, y, nullptr, 0, nullptr, 0, false);
}

int hd_batch_tune(hd_ctx* c, int prec, int* mode, int* grid, int* tile_groups, double* ms) {
    if (!c) return HD_ERR_ARG;
    if (!c->batch) return set_err(c, HD_ERR_STATE, "hd_setup_batch first");
    if (prec != HD_F64 && prec != HD_F32) return set_err(c, HD_ERR_ARG, "prec");
    int rc = use_device(c);
    if (rc) return rc;
    BatchState& B = *c->batch;
    const size_t es = prec == HD_F64 ? sizeof(double) : sizeof(float);
    // tuning vectors, freed on every return path
    struct Vecs {
        void* x = nullptr;
        void* y = nullptr;
        ~Vecs() {
            dfree(x);
            dfree(y);
        }
    } v;
    if (hipMalloc(&v.x, es * B.total) != hipSuccess || hipMalloc(&v.y, es * B.total) != hipSuccess)
        return set_err(c, HD_ERR_OOM, "tuning vectors");
    {
        const unsigned nbk = (unsigned)((B.total + 255) / 256);
        if (prec == HD_F64)
            hipLaunchKernelGGL(hd::tune_pattern_kernel<double>, dim3(nbk), dim3(256), 0, c->stream, (double*)v.x,
                               B.total);
        else
            hipLaunchKernelGGL(hd::tune_pattern_kernel<float>, dim3(nbk), dim3(256), 0, c->stream, (float*)v.x,
                               B.total);
        HD_HIP(c, hipGetLastError());
    }
    const int modes[3] = {0, 1, 2}, groups[4] = {1, 2, 4, 8}, grids[4] = {512, 1024, 2048, 4096};
    double best = 1e300;
    int bm = 0, bg = 1, bgrid = 2048;
    // average time of 3 applies after one warm-up in the current launch
    // configuration; the first failing launch ends the whole search
    auto time_one = [&](float& t) -> int {
        int r = launch_batch_apply(c, prec, v.x, v.y, nullptr, 0, nullptr, 0, false);
        if (r) return r;
        HD_HIP(c, hipEventRecord(c->ev0, c->stream));
        for (int k = 0; k < 3; ++k)
            if ((r = launch_batch_apply(c, prec, v.x, v.y, nullptr, 0, nullptr, 0, false))) return r;
        HD_HIP(c, hipEventRecord(c->ev1, c->stream));
        HD_HIP(c, hipEventSynchronize(c->ev1));
        HD_HIP(c, hipEventElapsedTime(&t, c->ev0, c->ev1));
        t /= 3.0f;
        return HD_OK;
    };
    for (int tg : groups) {
        if ((rc = batch_build_tiles(c, tg))) return rc;
        for (int md : modes)
            for (int gr : grids) {
                // one launch per instance: no grid or tile to choose
                if (md == 2 && (tg != groups[0] || gr != grids[0])) continue;
                B.mode = md;
                B.grid = gr;
                float t = 0.0f;
                if ((rc = time_one(t))) return rc;
                if (t < best) {
                    best = t;
                    bm = md;
                    bg = tg;
                    bgrid = gr;
                }
            }
    }
    B.mode = bm;
    B.grid = bgrid;
    if ((rc = batch_build_tiles(c, bg))) return rc;
    if (mode) *mode = bm;
    if (grid) *grid = bgrid;
    if (tile_groups) *tile_groups = bg;
    if (ms) *ms = best;
    return HD_OK;
}

int hd_batch_set_launch(hd_ctx* c, int mode, int grid, int tile_groups) {
    if (!c) return HD_ERR_ARG;
    if (!c->batch) return set_err(c, HD_ERR_STATE, "hd_setup_batch first");
    if (mode < 0 || mode > 2 || grid < 1 || grid > (1 << 20) || tile_groups < 1 || tile_groups > 4096)
        return set_err(c, HD_ERR_ARG, "bad launch configuration");
    int rc = use_device(c);
    if (rc) return rc;
    c->batch->mode = mode;
    c->batch->grid = grid;
    return batch_build_tiles(c, tile_groups);
}

int hd_batch_build_precond(hd_ctx* c, const hd_precond_params* params) {
    if (!c) return HD_ERR_ARG;
    if (!c->batch) return set_err(c, HD_ERR_STATE, "hd_setup_batch first");
    if (params && params->learned != 0) return set_err(c, HD_ERR_ARG, "batched preconditioners use the plain diagonal");
    BatchState& B = *c->batch;
    for (size_t i = 0; i < B.inst.size(); ++i) {
        const int rc = hd_build_precond(B.inst[i], params);
        if (rc) return set_err(c, rc, "instance " + std::to_string(i) + ": " + B.inst[i]->err);
    }
    const int rc = batch_union_build(c);
    if (rc) return rc;
    B.have_prec = true;
    return HD_OK;
}

int hd_batch_set_vcycle(hd_ctx* c, int shared) {
    if (!c) return HD_ERR_ARG;
    if (!c->batch) return set_err(c, HD_ERR_STATE, "hd_setup_batch first");
    if (shared != 0 && shared != 1) return set_err(c, HD_ERR_ARG, "shared must be 0 or 1");
    c->batch->vcycle_shared = shared;
    return HD_OK;
}

int hd_batch_minres_solve(hd_ctx* c, const hd_solve_params* params, const double* b, double* x,
                          hd_solve_info* info) {
    if (!c) return HD_ERR_ARG;
    if (!c->batch || !c->batch->have_prec) return set_err(c, HD_ERR_STATE, "hd_batch_build_precond first");
    if (!b || !x || b == x) return set_err(c, HD_ERR_ARG, "b, x must be distinct device pointers");
    hd_solve_params prm;
    if (params) prm = *params;
    else {
        prm.tol = 1e-8;
        prm.max_it = 10000;
        prm.mode = HD_MODE_PLAIN64;
        prm.use_x0 = 0;
        prm.inner_tol = 1e-5;
        prm.max_outer = 20;
        prm.check_every = 8;
        prm.stop_true = 0;
        prm.use_graph = 1;
    }
    if (!(prm.tol > 0) || prm.max_it < 1) return set_err(c, HD_ERR_ARG, "bad solve parameters");
    if (prm.mode == HD_MODE_MIXED && (!(prm.inner_tol > 0) || prm.max_outer < 1))
        return set_err(c, HD_ERR_ARG, "HD_MODE_MIXED needs inner_tol > 0 and max_outer >= 1");
    int rc = use_device(c);
    if (rc) return rc;
    rc = batch_minres_solve(c, prm, b, x, info);
    if (rc == HD_NOT_CONVERGED) c->err = "MINRES did not reach the tolerance for every instance";
    return rc;
}

int hd_get_diagonals(hd_ctx* c, double* m_diag, double* w_diag) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (m_diag)
        HD_HIP(c, hipMemcpyAsync(m_diag, c->d_mdiag, sizeof(double) * c->n_u, hipMemcpyDeviceToDevice, c->stream));
    if (w_diag)
        HD_HIP(c, hipMemcpyAsync(w_diag, c->d_wdiag, sizeof(double) * c->n_q, hipMemcpyDeviceToDevice, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

int hd_get_schur(hd_ctx* c, int64_t* nnz, int32_t* rowptr, int32_t* col, double* val) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (nnz) *nnz = c->S.nnz;
    if (!rowptr) return HD_OK;
    HD_HIP(c, hipMemcpyAsync(rowptr, c->S.rp, sizeof(int32_t) * (c->n_q + 1), hipMemcpyDeviceToHost, c->stream));
    if (col) HD_HIP(c, hipMemcpyAsync(col, c->S.ci, sizeof(int32_t) * c->S.nnz, hipMemcpyDeviceToHost, c->stream));
    if (val) HD_HIP(c, hipMemcpyAsync(val, c->S.v, sizeof(double) * c->S.nnz, hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

int hd_get_amg_nlevels(hd_ctx* c, int* nlevels) {
    if (!c || !nlevels) return HD_ERR_ARG;
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    *nlevels = (int)c->lev.size();
    return HD_OK;
}

}  // extern "C"

namespace {

// a device CSR matrix to caller-owned host arrays (each may be NULL)
int copy_dev_csr(hd_ctx* c, const DevCSR& M, int64_t* nrows, int64_t* ncols, int64_t* nnz, int32_t* rowptr,
                 int32_t* col, double* val) {
    if (nrows) *nrows = M.nrows;
    if (ncols) *ncols = M.ncols;
    if (nnz) *nnz = M.nnz;
    if (rowptr)
        HD_HIP(c, hipMemcpyAsync(rowptr, M.rp, sizeof(int32_t) * (M.nrows + 1), hipMemcpyDeviceToHost, c->stream));
    if (col && M.nnz)
        HD_HIP(c, hipMemcpyAsync(col, M.ci, sizeof(int32_t) * M.nnz, hipMemcpyDeviceToHost, c->stream));
    if (val && M.nnz) HD_HIP(c, hipMemcpyAsync(val, M.v, sizeof(double) * M.nnz, hipMemcpyDeviceToHost, c->stream));
    HD_HIP(c, hipStreamSynchronize(c->stream));
    return HD_OK;
}

}  // namespace

extern "C" {

int hd_get_amg_level(hd_ctx* c, int level, int64_t* n, int64_t* nnz, int32_t* rowptr, int32_t* col, double* val) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (level < 0 || level >= (int)c->lev.size()) return set_err(c, HD_ERR_ARG, "level");
    int rc = use_device(c);
    if (rc) return rc;
    return copy_dev_csr(c, c->lev[level].A, n, nullptr, nnz, rowptr, col, val);
}

int hd_get_amg_prolongator(hd_ctx* c, int level, int64_t* nrows, int64_t* ncols, int64_t* nnz, int32_t* rowptr,
                           int32_t* col, double* val) {
    if (!c) return HD_ERR_ARG;
    if (!c->have_prec) return set_err(c, HD_ERR_STATE, "hd_build_precond first");
    if (level < 0 || level + 1 >= (int)c->lev.size()) return set_err(c, HD_ERR_ARG, "level");
    int rc = use_device(c);
    if (rc) return rc;
    return copy_dev_csr(c, c->lev[level].P, nrows, ncols, nnz, rowptr, col, val);
}

int hd_apply_timing(hd_ctx* c, int reset, double* avg_ms, int64_t* count) {
    if (!c) return HD_ERR_ARG;
    if (avg_ms) *avg_ms = c->apply_count ? c->apply_ms_sum / (double)c->apply_count : 0.0;
    if (count) *count = c->apply_count;
    if (reset) {
        c->apply_ms_sum = 0.0;
        c->apply_count = 0;
    }
    c->time_apply = true;
    return HD_OK;
}

}  // extern "C"
