// Internal declarations of the hdivsp library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hdivsp.h"

#define HD_MAXP 8
#define HD_MAXQ (HD_MAXP + 1)

namespace hd {

// 1D tables of degree p with q = p + 1 Gauss-Legendre quadrature points.
//   L[a][i]  = l_i(x_a)       interpolation at the Gauss-Lobatto nodes (i <= p)
//   H[a][j]  = h_j(x_a)       histopolation on the Gauss-Lobatto sub-intervals
//   Bg[a][m] = L^g_m(x_a)     Lagrange basis at the p Gauss-Legendre nodes
//   L2, H2, Bg2               squares (diagonal assembly by sum factorisation)
//   Tinv                      inverse of Tm[m][j] = h_j(g_m) (IH -> GL nodal)
//   wq, xq                    quadrature weights and points on [0, 1]
template <typename T>
struct Tables {
    T L[HD_MAXQ][HD_MAXQ];
    T H[HD_MAXQ][HD_MAXP];
    T Bg[HD_MAXQ][HD_MAXP];
    T L2[HD_MAXQ][HD_MAXQ];
    T H2[HD_MAXQ][HD_MAXP];
    T Bg2[HD_MAXQ][HD_MAXP];
    T Tinv[HD_MAXP][HD_MAXP];
    T wq[HD_MAXQ];
    T xq[HD_MAXQ];
    T gll[HD_MAXQ];   // Gauss-Lobatto sub-element vertices on [0, 1]
};

void gauss_legendre01(int n, double* x, double* w);
void gauss_lobatto01(int p, double* xi);
void build_tables(int p, Tables<double>& t64, Tables<float>& t32);

// Number of geometric factors stored per quadrature point: the 6 entries of
// the symmetric w J^T J / det J and w / det J.
constexpr int NPA = 7;

// Host-side CSR (AMG setup works on the host).
struct HostCSR {
    int64_t nrows = 0, ncols = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    int64_t nnz() const { return (int64_t)ci.size(); }
};

struct HostAMG {
    std::vector<HostCSR> A;   // level matrices
    std::vector<HostCSR> P;   // prolongators level l -> l+1 (rows of l)
    std::vector<double> coarse_inv;   // dense, row-major
    bool singular = false;
};

int build_amg_host(const HostCSR& S, const hd_precond_params& prm, bool singular, HostAMG& out,
                   std::string& err);

// Unstructured hexahedral mesh: faces and the element-to-dof index arrays
// (unstructured.cpp).  l2g[e][NRT] holds the global RT dof of each local dof,
// bitwise complemented (~g, a negative value) where the element's local dof
// is minus the global one.
struct UnstructuredMap {
    int64_t nfaces = 0, n_face_dofs = 0, n_u = 0, n_q = 0;
    std::vector<uint8_t> boundary_face;    // [nfaces]
    std::vector<int32_t> elem_face;        // [ne][6] global face of local face (d, s), slot 2 d + s
    std::vector<int32_t> l2g;              // [ne][NRT]
};
int build_unstructured_numbering(int64_t nv, int64_t ne, const int64_t* elem, int P, UnstructuredMap& out,
                                 std::string& err);
// per L2 row and face slot 2 d + side: the signed RT dof of D's entry and
// the sub-volume across it (-1: none)
int build_unstructured_rows(const UnstructuredMap& m, int64_t ne, int P, std::vector<int32_t>& row_dof,
                            std::vector<int32_t>& row_nbr);

// Structured-mesh geometry passed to kernels: element counts and the offsets
// of the x-, y- and z-normal RT dof blocks.
struct Geo {
    int nx, ny, nz;
    int64_t off[3];
};

// Device CSR with FP64 and FP32 values.
struct DevCSR {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    double* v = nullptr;
    float* v32 = nullptr;
};

struct DevLevel {
    DevCSR A, P, R;           // R = P^T
    double* dinv = nullptr;   // 1 / sum_j |a_ij|
    float* dinv32 = nullptr;
    // work vectors (FP64 and FP32)
    double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr;
    float *b32 = nullptr, *x32 = nullptr, *r32 = nullptr, *z32 = nullptr;
};

// ---- batches of independent instances ----------------------------------
// Per-instance view for the persistent batched apply (device array).
struct BatchInstDev {
    Geo g;
    int p = 0;
    int with_c = 0;
    uint32_t ess = 0;
    unsigned nb = 0;          // element groups per colour
    int64_t n_u = 0;
    int64_t off = 0;          // offset of the instance's [u; q] in the concatenated vector
    const double* vert = nullptr; // mesh vertices (the apply computes the geometry from them)
    const void* winv = nullptr;   // explicit element inverses W_e^{-1} (kernel precision) or null
    const void* cm = nullptr;
    const void* kap = nullptr;
    const void* tabk = nullptr;
    double* part = nullptr;   // per-group partial sums of <A x, x> (2 nb)
};
// A work-queue entry: ngrp consecutive element groups of one instance.
struct BatchTile {
    int inst;
    unsigned grp0, ngrp;
};

// One (instance, operation) of a level in the batch's shared V-cycle
// launches: the operation's CSR matrix, its vectors and its first workgroup.
template <typename T>
struct UDesc {
    const int32_t* rp;
    const int32_t* ci;
    const T* mv;
    const T* dinv;       // post: this level's; restriction: the next level's (with out2)
    const double* cinv;  // coarse solve: the dense inverse
    const T* in;         // the vector the matrix multiplies (coarse: b)
    const T* b;          // pre- and post-smoothing: the level's right-hand side
    T* out;
    T* out2;             // restriction: the next level's x = dinv b, or null
    int64_t n;           // rows
    int g;               // lanes per row
    int inst;
    unsigned blk0;       // first workgroup of this descriptor
};
template <typename T>
struct UnionLaunch {
    int op = 0;
    int nd = 0;
    unsigned nblocks = 0;
    UDesc<T>* d = nullptr;
};

struct BatchState {
    std::vector<hd_ctx*> inst;                // one context per instance (shares device and stream)
    std::vector<int64_t> off;                 // ninst + 1 offsets of the concatenated vector
    int64_t total = 0;
    BatchInstDev* d_inst64 = nullptr;
    BatchInstDev* d_inst32 = nullptr;
    BatchTile* d_tiles = nullptr;
    int ntiles = 0;
    int* d_counter = nullptr;                 // work-queue heads: [mode 0: 2 colours][mode 1: 6 degrees x 2]
    int deg_t0[7] = {0, 0, 0, 0, 0, 0, 0};    // tiles of degree p: [deg_t0[p], deg_t0[p] + deg_nt[p])
    int deg_nt[7] = {0, 0, 0, 0, 0, 0, 0};
    int mode = 0;                             // 0: one persistent launch for all degrees; 1: one per degree
    double* d_part = nullptr;                 // all instances' apply partial sums
    std::vector<int64_t> part_off;            // per-instance offsets into d_part (2 nb each)
    int grid = 0;                             // persistent grid (workgroups)
    int tile_groups = 1;                      // element groups per tile
    bool have_prec = false;
    // V-cycle levels >= 1 of all instances in shared launches (built with
    // the preconditioners when every instance qualifies)
    std::vector<UnionLaunch<double>> un64;
    std::vector<UnionLaunch<float>> un32;
    std::vector<char> in_union;               // per instance: takes part in them
    bool union_ok = false;
    int vcycle_shared = 1;                    // 0: each instance's own V-cycle launches
};

struct RadDiffState;

}  // namespace hd

struct hd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // mesh
    bool have_mesh = false;
    int nx = 0, ny = 0, nz = 0, p = 0;
    int64_t ne = 0, n_u = 0, n_q = 0, nface[3] = {0, 0, 0};
    double* d_pa = nullptr;   // [ne][NPA][q^3]
    float* d_pa32 = nullptr;
    hd::Tables<double>* d_tab64 = nullptr;
    hd::Tables<float>* d_tab32 = nullptr;
    void* d_tabk64 = nullptr;       // compact per-degree tables for the element kernels
    void* d_tabk32 = nullptr;
    hd::Tables<double> tab64_host;
    hd::Tables<float> tab32_host;
    double* d_vert = nullptr;   // [(nx+1)(ny+1)(nz+1)][3], kept for the learned features
    bool affine = false;        // every element a parallelepiped (structured meshes): the apply
                                // forms J^T J / det J once per element

    // unstructured hexahedral mesh (hd_setup_mesh_unstructured); nx = ne,
    // ny = nz = 1 then, and the structured index arithmetic is not used
    bool unstructured = false;
    int64_t n_face_dofs = 0;
    double* d_evx = nullptr;        // [ne][8][3] element vertex coordinates
    int32_t* d_l2g = nullptr;       // [ne][NRT] signed element-to-dof map
    int32_t* d_rdof = nullptr;      // [n_q][6] signed RT dof of each sub-volume face slot
    int32_t* d_rnbr = nullptr;      // [n_q][6] sub-volume across it, -1 if none
    uint8_t* d_essm = nullptr;      // [n_u] essential RT dofs (identity rows)
    std::vector<uint8_t> u_boundary_dof;   // [n_u] dofs on boundary faces (host)

    // coefficients
    bool have_coeffs = false;
    int problem = 0;
    uint32_t ess = 0;
    double* d_cm = nullptr;      // c_mass per element
    double* d_kap = nullptr;     // kappa per element
    float* d_cm32 = nullptr;
    float* d_kap32 = nullptr;
    bool kappa_zero = true;

    // preconditioner
    bool have_prec = false;
    double tau = 1.0;
    double* d_mdiag = nullptr;   // diag(M), 1 on essential dofs
    double* d_wdiag = nullptr;   // diag(W) unweighted
    double* d_mdinv = nullptr;   // 1 / (tau diag(M)), 1 on essential dofs
    float* d_mdinv32 = nullptr;
    double* d_wface = nullptr;   // 1 / M~_kk on free interior faces, 0 elsewhere (n_u)
    double* d_sdiag = nullptr;   // diagonal of S~ (n_q)
    float* d_sdiag32 = nullptr;
    hd::DevCSR S;                // S~
    std::vector<hd::DevLevel> lev;
    int64_t n_coarse = 0;
    // level 0 of the V-cycle: for each sub-volume i and direction d, the
    // weight of the face to its lower neighbour (0 if none), [3][n_q] in the
    // element-major L2 numbering; per-block partials of the post-smoother
    double* d_wlo = nullptr;
    float* d_wlo32 = nullptr;
    double* d_s0part = nullptr;
    double* d_cinv = nullptr;
    float* d_cinv32 = nullptr;
    bool singular = false;

    // learned (1,1)-diagonal correction
    float* d_mlp = nullptr;          // network parameters (FP32, flat)
    float* d_adam_m = nullptr;
    float* d_adam_v = nullptr;
    int adam_t = 0;
    bool mlp_ready = false;
    double* d_theta = nullptr;       // [ne][6] log-scalings set by hd_set_diag_scalings
    bool theta_set = false;
    double* d_theta_net = nullptr;   // [ne][6] the network's scalings of the mesh
    bool fallback_used = false;

    // private stream on which MINRES records its graphs (default priority)
    hipStream_t cap_stream = nullptr;

    // explicit element inverses W_e^{-1} for p <= 2 ([N_e][p^3][p^3]), null
    // when the local CG is used; local_solver is an HD_LOCAL_* mode
    int local_solver = 0;
    double* d_winv = nullptr;
    float* d_winv32 = nullptr;

    // Darcy with gamma varying inside the elements (hd_set_gamma_field): the
    // vertex values (FP64 / FP32) and C~ of S~ ([n_q]); kappa is 1 then
    bool gamma_field = false;
    double* d_gv = nullptr;
    float* d_gv32 = nullptr;
    double* d_ctil = nullptr;

    // MINRES work space kept between solves (owned by the solver, released
    // through solve_cache_free)
    void* solve_cache = nullptr;
    void (*solve_cache_free)(void*) = nullptr;

    // batch of independent instances (hd_setup_batch)
    hd::BatchState* batch = nullptr;

    // radiation-diffusion time stepping (hd_rd_setup): work space and parameters
    hd::RadDiffState* rd = nullptr;

    // scratch
    double* d_partial = nullptr;     // per-block partial sums (>= ne and >= reduce grid)
    int64_t partial_cap = 0;
    double* d_noalloc = nullptr;     // device address of the library's fixed scratch on this device (not owned)
    double* d_scal = nullptr;        // small device scalar block
    int* d_flag = nullptr;

    // timing of the block apply
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double apply_ms_sum = 0.0;
    int64_t apply_count = 0;
    bool time_apply = false;
};

namespace hd {

// error helpers
int set_err(hd_ctx* c, int code, const std::string& msg);
#define HD_HIP(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return hd::set_err((ctx), HD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
inline T* dalloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) return nullptr;
    return (T*)p;
}
inline void dfree(void* p) {
    if (p) (void)hipFree(p);
}

// kernels and launchers (setup.hip)
int launch_geometry(hd_ctx* c, const double* d_vert, int* d_bad);
// diag(M) (with optional per-element log-scalings theta [ne][6]) and diag(W)
int launch_diagonals(hd_ctx* c, const double* theta);
int launch_schur(hd_ctx* c);
int launch_ensure_partial(hd_ctx* c, int64_t n);

// apply.hip
enum { ESS_NONE = 0, ESS_IDENTITY = 1 };
// y = A x for nrhs vectors (stride n_u + n_q).  in_scale[r * scale_stride]
// scales the input of RHS r, done[r * done_stride] != 0 skips it, and the
// per-block partial sums of <A x, x> of RHS r start at dot_partial + r * part_stride.
int launch_apply(hd_ctx* c, int prec, int nrhs, const void* x, void* y, const double* in_scale, int scale_stride,
                 double* dot_partial, int64_t part_stride, int ess_mode, const int* done, int done_stride);
int launch_mass_inverse(hd_ctx* c, int prec, const void* x, void* y, bool weighted);
// y = A x for nrhs right-hand sides interleaved ([dof][nrhs])
int launch_apply_interleaved(hd_ctx* c, int prec, int nrhs, const void* x, void* y);
int launch_lift(hd_ctx* c, const double* ubc, double* b);
int launch_constant_flux(hd_ctx* c, const double* u, double* out);
int64_t apply_partial_count(const hd_ctx* c);
int upload_kernel_tables(hd_ctx* c);

// precond.hip: work vectors and l1 diagonals of the levels in c->lev
int finish_levels(hd_ctx* c);
// amg_gpu.hip: the smoothed-aggregation hierarchy of S~ built on the device
int build_amg_gpu(hd_ctx* c, const hd_precond_params& prm);
int launch_precond(hd_ctx* c, int prec, const void* r, void* z, double* dot_partial_u, double* dot_partial_q,
                   const int* done);
int launch_diag_prec(hd_ctx* c, int prec, const void* r, void* z, double* part);
int launch_schur_prec(hd_ctx* c, int prec, const void* b, void* z, double* part, const int* done);
// upper block-triangular preconditioner z = P^{-1} r (FP64; s_scratch: n_q)
int launch_tri_precond(hd_ctx* c, const double* r, double* z, double* s_scratch);
// right-preconditioned restarted GMRES with the block-triangular preconditioner
int gmres_solve(hd_ctx* c, double tol, int max_it, int restart, const double* b, double* x, hd_solve_info* info);
// explicit element inverses of W_e for p <= 2 (built from the stored
// factors w / det J); freed with the coefficients
int build_local_inverse(hd_ctx* c);
void free_local_inverse(hd_ctx* c);
int64_t schur_partial_count(const hd_ctx* c);
void free_levels(hd_ctx* c);
Geo geo_of(const hd_ctx* c);
int scan_counts(hd_ctx* c, const int32_t* cnt, int64_t n, int32_t* rp, int64_t* total_host);

// learned.hip: the learned (1,1)-diagonal correction
int mlp_param_count();
int launch_targets(hd_ctx* c, int p, int64_t n, const double* verts, int steps, double* theta, double* lam,
                   double* spread);
int launch_features(hd_ctx* c, int64_t n, const double* verts, const double* alpha, const double* beta,
                    const int* parr, int p, float* X);
int mlp_init(hd_ctx* c, uint64_t seed);
int mlp_set(hd_ctx* c, const float* host);
int mlp_get(hd_ctx* c, float* host);
int mlp_loss_grad(hd_ctx* c, int64_t n, const float* X, const float* Y, float* loss, float* grad);
int mlp_train(hd_ctx* c, int64_t n, const float* X, const float* Y, int64_t nval, const float* Xv, const float* Yv,
              int epochs, int batch, float lr, uint64_t seed, float* train_loss, float* val_loss);
int mlp_infer(hd_ctx* c, int64_t n, const float* X, float* theta, int bf16);
int learned_mesh_theta(hd_ctx* c, int* fallback);

// batched instances (apply.hip, minres.hip, batch.cpp)
int launch_batch_apply(hd_ctx* c, int prec, const void* x, void* y, const double* scale, int scale_stride,
                       const int* done, int done_stride, bool partials);
int batch_build_tiles(hd_ctx* c, int tile_groups);
int batch_minres_solve(hd_ctx* c, const hd_solve_params& prm, const double* b, double* x, hd_solve_info* info);
void batch_free(hd_ctx* c);

// minres.hip
// nrhs right-hand sides stored one after the other; info: nrhs entries
int minres_solve(hd_ctx* c, const hd_solve_params& prm, int nrhs, const double* b, double* x, hd_solve_info* info);

// precond.hip: the batch's shared V-cycle launches
int batch_union_build(hd_ctx* c);
void batch_union_free(hd_ctx* c);
template <typename T>
int batch_union_cycle(hd_ctx* c, const T* const* vq, T* const* zq, double* const* part, const int* stop,
                      int stop_stride);

// raddiff.hip: the radiation-diffusion time step and its helpers
int launch_divergence(hd_ctx* c, const double* F, double* q);
int launch_subcell_volumes(hd_ctx* c, double* vol);
int rd_setup(hd_ctx* c, const hd_rd_params& prm, const hd_precond_params* pp);
int rd_step(hd_ctx* c, double* e, double* E, double* F, hd_rd_info* info);
void rd_free(hd_ctx* c);

// reductions (setup.hip)
int reduce_sum_partials(hd_ctx* c, const double* partial, int64_t n, double* out_dev);

}  // namespace hd
