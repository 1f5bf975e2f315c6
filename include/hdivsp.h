/*
 * hdivsp.h - C ABI of the MI355X library for the transformed H(div)
 * saddle-point system and its block-preconditioned MINRES solver.
 *
 * Method: Pazner, Kolev, Vassilevski, "Matrix-free GPU-accelerated
 * saddle-point solvers for high-order problems in H(div)".
 *
 *   A = [ M   D^T ]      M  : RT_p mass matrix weighted by c_mass per element
 *       [ D   -C  ]      D  : +-1 sub-element incidence (interpolation-
 *                             histopolation basis, Section 2.1)
 *                        C  : block diagonal, C_e = kappa_e W_e^{-1}, W_e the
 *                             element L2 mass matrix
 *   grad-div (eq. transformed-system):          c_mass = beta, kappa = 1/alpha
 *   Darcy    (eq. transformed-system-darcy,
 *             piecewise-constant gamma):         c_mass = 1/eps, kappa = gamma
 *
 *   B^{-1} = diag( (tau diag(M))^{-1}, one AMG V-cycle on
 *                  S~ = C~ + D diag(M)^{-1} D^T )      (eq. approx-schur,
 *                  eq. approx-schur-entries, Prop. 5)
 *
 * Mesh: structured nx x ny x nz hexahedra with arbitrary (trilinear) vertex
 * positions.  Vertices: host array [(nx+1)(ny+1)(nz+1)][3], x fastest.
 * Element e = ex + nx (ey + ny ez).
 *
 * Vector layout (length n_u + n_q, one right-hand side):
 *   [0, n_u)   RT dofs, one per sub-element face of the refined grid,
 *              direction-major (x-normal faces, then y, then z), each block
 *              lexicographic over the refined face grid, first index fastest;
 *              orientation +axis.
 *   [n_u, n)   L2 dofs, element-major: e, then (a, b, c), a fastest.
 * Multi-RHS buffers (nrhs > 1) are RHS-major: nrhs consecutive vectors.
 *
 * Essential flux dofs (faces on the box sides selected by ess_sides) have
 * identity rows and columns: apply() ignores their input values in every
 * other row and copies the input to their output.
 *
 * Conventions
 *   - Device pointers are caller-owned, allocated on the context's device,
 *     of the precision named by `prec` (HD_F64: double, HD_F32: float).
 *   - Host pointers passed to setup calls are copied before return.
 *   - All work is enqueued on the context stream; calls that return data to
 *     the host (sizes, info, hierarchy queries) synchronise that stream.
 *   - Return value: 0 on success, < 0 on error (see HD_ERR_*), > 0 warning.
 *     The message of the last non-zero status is kept in the context.
 *   - A context is used by one host thread at a time.
 */
#ifndef HDIVSP_H
#define HDIVSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hd_ctx hd_ctx;

enum {
    HD_OK = 0,
    HD_ERR_ARG = -1,        /* invalid argument or size */
    HD_ERR_MESH = -2,       /* non-positive Jacobian determinant */
    HD_ERR_HIP = -3,        /* HIP runtime error */
    HD_ERR_OOM = -4,        /* device allocation failed */
    HD_ERR_AMG = -5,        /* AMG setup failed */
    HD_ERR_BREAKDOWN = -6,  /* MINRES: preconditioner not positive definite */
    HD_ERR_NONFINITE = -7,  /* non-finite value in input or iteration */
    HD_ERR_STATE = -8,      /* call order violated (e.g. solve before setup) */
    HD_NOT_CONVERGED = 1,   /* max iterations reached, info filled */
    HD_FALLBACK_USED = 2
};

enum { HD_GRADDIV = 0, HD_DARCY = 1 };
enum { HD_F64 = 0, HD_F32 = 1 };

/* ess_sides bits */
enum { HD_SIDE_XMIN = 1, HD_SIDE_XMAX = 2, HD_SIDE_YMIN = 4, HD_SIDE_YMAX = 8,
       HD_SIDE_ZMIN = 16, HD_SIDE_ZMAX = 32, HD_SIDE_ALL = 63 };

/* MINRES modes */
enum {
    HD_MODE_PLAIN64 = 0,   /* everything in FP64 */
    HD_MODE_MIXED = 1,     /* FP64 residual refinement around FP32 MINRES
                              (FP32 vectors, operator and preconditioner;
                              FP64 dot products, recurrences and coarse solve) */
    HD_MODE_PREC32 = 2     /* FP64 MINRES and operator with the Schur-block
                              V-cycle in FP32 (FP32 level matrices, FP64
                              coarse solve); the (1,1) diagonal stays FP64 */
};

typedef struct hd_precond_params {
    double tau;          /* (1,1)-block scaling (remark after Prop. 3); default 1 */
    double theta;        /* AMG strength threshold; default 0.25 */
    int max_coarse;      /* AMG coarsest size; default 1024 */
    int max_levels;      /* default 25 */
    double omega;        /* prolongator smoothing weight; default 2/3 */
    int learned;         /* (1,1) diagonal: 0 plain diag(M) (Section 2.3); 1 diag(M)
                            with per-element scalings from the network held by
                            the context (hd_mlp_*), falling back to the plain
                            diagonal with HD_FALLBACK_USED when an output is not
                            finite; 2 with the scalings set by
                            hd_set_diag_scalings.  Default 0 */
} hd_precond_params;

typedef struct hd_solve_params {
    double tol;          /* relative tolerance (see mode and stop_true); default 1e-8.
                            HD_MODE_MIXED always stops on the true FP64 residual */
    int max_it;          /* max MINRES iterations (inner, per refinement); default 10000 */
    int mode;            /* HD_MODE_* */
    int use_x0;          /* 1: x holds the initial guess; 0: start from zero */
    double inner_tol;    /* HD_MODE_MIXED: inner FP32 tolerance; default 1e-5.
                            Each refinement's inner MINRES stops at
                            max(inner_tol, 0.1 tol / rho) relative to its start,
                            rho the current true relative residual, so that the
                            last refinement does not solve past the target */
    int max_outer;       /* HD_MODE_MIXED: max refinement steps; default 20 */
    int check_every;     /* iterations between host polls of the flag; default 8 */
    int stop_true;       /* HD_MODE_PLAIN64, HD_MODE_PREC32: 0 stops when |eta| <= tol |eta_0| (the
                            preconditioned residual norm carried by the
                            recurrence); 1 also requires the true FP64
                            ||b - A x||_2 <= tol ||b||_2, tightening the
                            threshold and continuing the same recurrence */
    int use_graph;       /* 1: each poll period of iterations (check_every, if
                            even) is captured once as a HIP graph and replayed;
                            0: kernels are launched one by one.  Same results.
                            Default 1 */
} hd_solve_params;

typedef struct hd_solve_info {
    int status;          /* 0 converged, HD_NOT_CONVERGED, HD_ERR_BREAKDOWN */
    int iterations;      /* total operator applications (all precisions) */
    int outer;           /* refinement steps (HD_MODE_MIXED), else 1 */
    double eta_rel;      /* last |eta| / |eta_0| of the (last) MINRES */
    double true_rel_res; /* ||b - A x||_2 / ||b||_2 in FP64 */
    double time_s;       /* wall time of the solve on the device stream */
} hd_solve_info;

/* Context bound to `device` and to `stream` (a hipStream_t, may be NULL for
 * the default stream).  Section 3 (solver overview). */
int hd_create(hd_ctx** out, int device, void* stream);
int hd_destroy(hd_ctx* ctx);
const char* hd_last_error(const hd_ctx* ctx);

/* Structured mesh and RT order p (1 <= p <= 8).  Computes the geometric
 * factors at the (p+1)^3 Gauss-Legendre points of every element
 * (w J^T J / det J and w / det J; partial assembly, Section 3) and rejects
 * det J <= 0 at quadrature points and vertices with HD_ERR_MESH. */
int hd_setup_mesh(hd_ctx* ctx, int nx, int ny, int nz, int p, const double* vertices);

/* Coefficients per element and the problem type, which fix the blocks of
 * the transformed system (Section 2.3, eq. transformed-system, grad-div;
 * Section 2.4, eq. transformed-system-darcy, Darcy with piecewise-constant
 * gamma): M = M_beta or M_{1/eps}, and the (2,2) block C = kappa_e W_e^{-1}
 * with kappa = 1/alpha (grad-div) or gamma (Darcy).
 * problem = HD_GRADDIV: c_mass = beta > 0, c_22 = alpha > 0 (required).
 * problem = HD_DARCY:   c_mass = 1/eps > 0, c_22 = gamma >= 0 or NULL (0).
 * c_mass, c_22: host arrays of nx*ny*nz finite values in element order
 * (e = ex + nx (ey + ny ez)), copied; the caller keeps ownership.
 * ess_sides: bit mask of box sides (HD_SIDE_*) whose RT dofs are essential
 * (identity rows and columns of the operator).
 * Errors: HD_ERR_STATE before hd_setup_mesh; HD_ERR_ARG for an unknown
 * problem, a NULL c_mass (or c_22 for grad-div), ess_sides > 63 or an
 * out-of-range value; HD_ERR_NONFINITE for a non-finite value.  Drops any
 * preconditioner (build it again). */
int hd_setup_coeffs(hd_ctx* ctx, int problem, const double* c_mass, const double* c_22,
                    uint32_t ess_sides);

/* Unstructured hexahedral mesh (Section 3.2, Algorithm 1: D from element-to-
 * dof index arrays and orientation signs; Section 4.1 solves on such a mesh)
 * instead of hd_setup_mesh.  vertices: host array [nv][3]; elements: host
 * array [ne][8] of vertex numbers in the reference order v = dx + 2 dy + 4 dz
 * (the trilinear map must keep det J > 0); both copied.  Faces are matched
 * by their four vertex numbers (a face shared by more than two elements, or
 * with a repeated vertex, is HD_ERR_MESH).  Each face carries a canonical
 * frame fixed by its vertex numbers: origin at its smallest-numbered vertex,
 * first axis towards the smaller-numbered of the origin's two neighbours on
 * the face, second axis towards the other, normal = first x second; its RT
 * dofs are the sub-face fluxes along that normal.
 * Numbering of the RT block: the face dofs face by face (faces in the order
 * of their first appearance over (element, local face 2 d + s), local face
 * (d, s) the side x_d = s), p^2 per face, first frame index fastest; then
 * the interior dofs element by element, 3 (p-1) p^2 each: component c, the
 * index along c from 1 to p-1 fastest, then the two others in increasing
 * axis order.  The L2 block is element-major as on structured meshes.  The
 * operator, the preconditioner and MINRES then work as on structured
 * meshes (the L2 rows of S~ through the same index arrays; level 0 of the
 * V-cycle as a CSR level).  hd_setup_coeffs takes per-element arrays in
 * element order and ess_sides 0 or HD_SIDE_ALL (every boundary face
 * essential); hd_set_essential_dofs selects any other set.  Structured-only
 * calls (gamma fields, the learned diagonal, the block-triangular
 * preconditioner and GMRES, hd_constant_flux, hd_lift_essential, batches)
 * return HD_ERR_STATE.  Errors: HD_ERR_ARG for bad sizes, p outside [1, 6]
 * or vertex numbers out of range; HD_ERR_NONFINITE; HD_ERR_MESH. */
int hd_setup_mesh_unstructured(hd_ctx* ctx, int64_t nv, const double* vertices, int64_t ne,
                               const int64_t* elements, int p);

/* Essential RT dofs of an unstructured mesh (identity rows and columns):
 * host array of n_u bytes, nonzero = essential, copied.  Call after
 * hd_setup_coeffs (HD_ERR_STATE otherwise, or on a structured mesh); drops the
 * preconditioner.  The Schur approximation is taken as singular (constants
 * removed, Section 4.2) when the (2,2) block is zero and every dof on a
 * boundary face is essential. */
int hd_set_essential_dofs(hd_ctx* ctx, const uint8_t* mask);

/* The element-to-dof map of an unstructured mesh (Section 3.2, Algorithm 1:
 * the index arrays and orientation signs D is built from): host array [ne][3 p^2 (p+1)]
 * (local RT dofs component-major, each component's tensor index with its
 * first index fastest), entry g where the element's local dof equals global
 * dof g and ~g (bitwise complement, negative) where it equals -g.
 * HD_ERR_STATE before hd_setup_mesh_unstructured. */
int hd_get_dof_map(hd_ctx* ctx, int32_t* l2g);

/* Darcy with gamma varying inside the elements (Section 2.4, the general case
 * of eq. transformed-system-darcy): gamma becomes the continuous
 * piecewise-trilinear field with the given values at the mesh vertices
 * (host array of (nx+1)(ny+1)(nz+1) finite values >= 0, not all zero,
 * numbered like the vertices of hd_setup_mesh), and the (2,2) block of the
 * operator becomes the full W^{-1} W_gamma W^{-1} (W_gamma the gamma-weighted
 * L2 mass matrix, integrated with the (p+1)^3-point rule; two local solves
 * per element and apply), approximated in S~ by
 * diag(W)^{-1} diag(W_gamma) diag(W)^{-1}.  Call after
 * hd_setup_coeffs(HD_DARCY, ...) (HD_ERR_STATE otherwise); it replaces that
 * call's gamma, drops the preconditioner (build it again), and lasts until the
 * next hd_setup_coeffs.  hd_apply_mass_inverse is not defined for a field
 * (HD_ERR_STATE). */
int hd_set_gamma_field(hd_ctx* ctx, const double* gamma_vertices);

/* Global sizes of the two blocks of the unknown (Section 2: RT_p velocity
 * dofs, one per sub-element face of the refined grid, and L2 dofs, p^3 per
 * element): n_u and n_q written to the host pointers (either may be NULL).
 * A vector of the system is [u; q~], n_u + n_q long.  HD_ERR_STATE before
 * hd_setup_mesh. */
int hd_sizes(const hd_ctx* ctx, int64_t* n_u, int64_t* n_q);

/* Whether hd_setup_mesh found every element to be a parallelepiped (the
 * trilinear map of Section 3 affine: the twist vectors of each vertex cube
 * below 1e-14 of its edges), written to *affine as 1 or 0.  Then J, and
 * J^T J / det J, are the same at all quadrature points of an element, and
 * hd_apply_block_op forms them once per element (same operator; unstructured
 * meshes, a gamma field and the instances of a batch always take the general
 * path).  HD_ERR_ARG for a NULL pointer, HD_ERR_STATE before hd_setup_mesh. */
int hd_mesh_affine(const hd_ctx* ctx, int* affine);

/* y = A x (eq. transformed-saddle-point, Section 3).  x != y, device
 * pointers of length nrhs*(n_u+n_q).  Essential convention as above.
 * Matrix-free: M by sum factorisation at the quadrature points, D and D^T
 * by the +-1 sub-element incidence, C by a per-element preconditioned CG in
 * the Gauss-Legendre basis (Section 2.5, Section 3.1) or, for p <= 2, by
 * stored explicit element inverses (hd_set_local_solver). */
int hd_apply_block_op(hd_ctx* ctx, int prec, int nrhs, const void* x, void* y);

/* y = A x for nrhs right-hand sides stored interleaved: entry (dof d, right-
 * hand side r) at d * nrhs + r, for x and y alike (device pointers of
 * nrhs * (n_u + n_q) values of the given precision, x != y, caller-owned;
 * asynchronous on the context's stream).  The same operator as
 * hd_apply_block_op (eq. transformed-saddle-point, Section 3; the (2,2) block
 * always by the local CG of Section 2.5), computed with the right-hand sides
 * side by side: the element's geometric factors are formed once for all of
 * them and every LDS and global access reads the right-hand sides of a dof
 * together.  Structured meshes with piecewise-constant coefficients only
 * (HD_ERR_STATE on an unstructured mesh or with a gamma field); HD_ERR_ARG for
 * nrhs < 1, a bad precision or bad pointers. */
int hd_apply_block_op_interleaved(hd_ctx* ctx, int prec, int nrhs, const void* x, void* y);

/* How the block apply, and everything built on it, applies W_e^{-1} in the
 * (2,2) block (Section 3.1, GPU acceleration of the DG mass inverse: explicit
 * inverses applied by a batched matrix-vector product for small degrees,
 * matrix-free local CG otherwise).
 *   HD_LOCAL_AUTO      explicit inverses for p <= 2, local CG for p >= 3
 *                      (the default);
 *   HD_LOCAL_CG        local CG for every degree;
 *   HD_LOCAL_EXPLICIT  explicit inverses (p <= 2 only, HD_ERR_ARG otherwise).
 * The inverses (p^3 x p^3 per element, FP64 with an FP32 copy, inverted in
 * FP64 by Gauss-Jordan elimination on the SPD element matrix) are built when
 * coefficients with a nonzero (2,2) block are set, or by this call if they
 * already are; the stand-alone hd_apply_mass_inverse keeps the local CG.
 * May be called before or after hd_setup_coeffs; HD_ERR_OOM if the inverses
 * do not fit. */
enum { HD_LOCAL_AUTO = 0, HD_LOCAL_CG = 1, HD_LOCAL_EXPLICIT = 2 };
int hd_set_local_solver(hd_ctx* ctx, int mode);

/* y_q = C x_q = kappa_e W_e^{-1} x_q per element (the (2,2) block without
 * its sign), for nrhs L2 vectors of length n_q stored one after the other.  For HD_DARCY with gamma = 0 use
 * hd_apply_l2_mass_inverse.  Section 2.5. */
int hd_apply_mass_inverse(hd_ctx* ctx, int prec, int nrhs, const void* x, void* y);

/* y_q = W^{-1} x_q (unweighted), e.g. to form W^{-1} g^ for Darcy
 * right-hand sides or p = W^{-1} p~ in post-processing (Section 3). */
int hd_apply_l2_mass_inverse(hd_ctx* ctx, int prec, const void* x, void* y);

/* Essential flux boundary conditions in the block system (Section 2:
 * u.n prescribed on part of the boundary; Section 4.2 uses it for the
 * layered Darcy problem): b <- lifted right-hand side for the essential
 * values u_bc, b_f -= (A_full [u_bc; 0])_f on free rows and b_e = u_bc on
 * essential rows, so that the solution of the system with identity
 * essential rows takes the prescribed values.  u_bc: FP64 device array of
 * length n_u (only essential entries are read); b: FP64 device array of
 * length n_u + n_q, updated in place; both caller-owned.  Asynchronous on
 * the context's stream.  HD_ERR_STATE before hd_setup_coeffs, HD_ERR_ARG
 * for NULL pointers. */
int hd_lift_essential(hd_ctx* ctx, const double* u_bc, double* b);

/* RT interpolant of the constant vector field u[3] (host): every dof (device,
 * length n_u) receives the flux of u through its sub-element face, oriented
 * along +axis (the face dofs of the interpolation-histopolation basis,
 * Section 2.1; exact on trilinear meshes).  Flux boundary data such as
 * u.n = (1,0,0).n then come from hd_lift_essential. */
int hd_constant_flux(hd_ctx* ctx, const double* u, double* dofs);

/* Diagonal M~ = diag(M), the approximate Schur complement S~ in CSR form
 * (eq. approx-schur-entries, assembled row by row; 1 on essential
 * dofs of M~) and the AMG hierarchy on S~.  params may be NULL (defaults). */
int hd_build_precond(hd_ctx* ctx, const hd_precond_params* params);

/* z = B^{-1} r with the block-diagonal preconditioner
 * B = diag(tau M~, S^) (Section 2.2, Prop. 1 and the remark on tau;
 * Section 2.3, eq. approx-schur): z_u = (tau M~)^{-1} r_u and
 * z_q = one AMG V-cycle on S~ applied to r_q (constants removed when S~ is
 * singular).  r, z: distinct caller-owned device arrays of nrhs*(n_u+n_q)
 * values of precision prec (HD_F64 or HD_F32), right-hand sides stored one
 * after the other.  Asynchronous on the context's stream.  HD_ERR_STATE
 * before hd_build_precond, HD_ERR_ARG for bad pointers, prec or nrhs. */
int hd_apply_precond(hd_ctx* ctx, int prec, int nrhs, const void* r, void* z);

/* Block-preconditioned MINRES on A x = b (Section 2.2: MINRES for the
 * symmetric indefinite saddle-point system with the block-diagonal
 * preconditioner of hd_apply_precond; Section 3: one operator apply and one
 * preconditioner apply per iteration).  Stops when the preconditioned
 * residual norm the recurrence carries falls below tol times its initial
 * value, and with stop_true also checks the true FP64 relative residual.
 * params may be NULL (defaults of hd_solve_params); mode selects FP64,
 * mixed-precision refinement or the FP32 Schur V-cycle.
 * b, x: distinct caller-owned FP64 device arrays of nrhs*(n_u+n_q) values,
 * right-hand sides one after the other; x is read as the initial guess when
 * use_x0 is set.  info: host array of nrhs entries (may be NULL).
 * Synchronises the stream before returning.  Returns 0 when every
 * right-hand side converged, HD_NOT_CONVERGED (> 0) when one reached
 * max_it, HD_ERR_BREAKDOWN on a Lanczos breakdown, HD_ERR_STATE before
 * hd_build_precond, HD_ERR_ARG for bad arguments. */
int hd_minres_solve(hd_ctx* ctx, const hd_solve_params* params, int nrhs,
                    const double* b, double* x, hd_solve_info* info);

/* GMRES(restart), right-preconditioned with the upper block-triangular
 * preconditioner P = [[tau M~, D^T], [0, -S^]] (Section 2.2, the remark on
 * block-triangular preconditioners; M~ and the V-cycle S^ of
 * hd_build_precond, which must have been called).  FP64, one right-hand side:
 * b, x FP64 device pointers of length n_u + n_q; x holds the initial guess
 * on entry (zeros for none) and the solution on return.  Stops when the
 * Arnoldi residual estimate, and then the true residual, satisfy
 * ||b - A x||_2 <= tol ||b||_2, or after max_it operator applications.  The
 * Krylov basis ((restart + 1) vectors of n_u + n_q doubles) is allocated for
 * the call (HD_ERR_OOM if it does not fit).  info (optional): iterations =
 * operator applications, outer = restart cycles, eta_rel = last estimate,
 * true_rel_res, time_s.  Returns 0, HD_NOT_CONVERGED or an error code. */
int hd_gmres_solve(hd_ctx* ctx, double tol, int max_it, int restart, const double* b, double* x,
                   hd_solve_info* info);

/* z = P^{-1} r for the block-triangular preconditioner of hd_gmres_solve
 * (Section 2.2, the remark on block-triangular preconditioners):
 * z_q = -S^{-1} r_q (one V-cycle), z_u = (tau M~)^{-1} (r_u - D^T z_q) on free
 * RT dofs and z_u = r_u on essential ones.  FP64 device pointers of length
 * n_u + n_q, r != z.  HD_ERR_STATE before hd_build_precond. */
int hd_apply_tri_precond(hd_ctx* ctx, const double* r, double* z);

/* hd_apply_tri_precond without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, result and kernels, but
 * the V-cycle output it needs (n_q values) lives in a fixed device array of
 * the library of 2^24 FP64 values (128 MiB), which every device the library
 * runs on holds until the process ends.  Calls no hipMalloc, hipFree or
 * allocating routine and does not synchronise (asynchronous on the
 * context's stream).  All calls on one device share that array and leave
 * the last call's contents in it; nothing in it needs to start at zero.
 * Calls that overlap in time on one device (other streams, other contexts
 * or threads) race on it and must be serialised by the caller.
 * HD_ERR_ARG if n_q > 2^24 or for bad pointers (r != z, both FP64 device
 * arrays of n_u + n_q values, caller-owned); HD_ERR_STATE before
 * hd_setup_mesh or hd_build_precond. */
int hd_apply_tri_precond_noalloc(hd_ctx* ctx, const double* r, double* z);
/* The solver's work space (Krylov vectors, partial sums, pinned state) stays
 * allocated in the context between calls and is rebuilt when the sizes,
 * the precision mode or nrhs change; hd_destroy releases it. */

/* ---- batches of independent instances ----------------------------------
 * Many independent problems of different sizes and degrees handled together
 * (not in the paper, which solves one mesh at a time).  Vectors are the
 * instances' [u; q~] blocks concatenated in instance order (offsets from
 * hd_batch_sizes).  The block apply of all instances runs as persistent
 * launches that take (instance, element-group) tiles from a work queue, most
 * expensive degree first; MINRES keeps one recurrence per instance (its own
 * scalars, stop test and preconditioner). */
typedef struct hd_instance_desc {
    int nx, ny, nz, p;          /* mesh and RT order (1..6) */
    const double* vertices;     /* host, (nx+1)(ny+1)(nz+1) x 3 */
    const double* c_mass;       /* host, nx ny nz */
    const double* c_22;         /* host, nx ny nz, or NULL (Darcy with gamma = 0) */
    uint32_t ess_sides;
} hd_instance_desc;

/* Set up ninst instances of one problem type (host arrays are copied); each
 * instance is the system of hd_setup_mesh / hd_setup_coeffs (Section 3).
 * Replaces a previous batch of the context; independent of hd_setup_mesh. */
int hd_setup_batch(hd_ctx* ctx, int problem, int ninst, const hd_instance_desc* inst);
/* offsets [ninst + 1]: start of each instance's block and the total length;
 * n_u [ninst]: its RT dof count (either may be NULL). */
int hd_batch_sizes(hd_ctx* ctx, int64_t* offsets, int64_t* n_u);
/* y = A x for every instance (eq. transformed-saddle-point per instance;
 * device pointers of the total length, x != y). */
int hd_batch_apply(hd_ctx* ctx, int prec, const void* x, void* y);
/* Autotuner: times the batched apply over the launch variants (mode 0: one
 * persistent launch for all degrees; 1: one persistent launch per degree;
 * 2: each instance's own full-grid launch, one per instance), persistent
 * grid sizes and element groups per tile, keeps the fastest and reports it
 * (any output may be NULL). */
int hd_batch_tune(hd_ctx* ctx, int prec, int* mode, int* grid, int* tile_groups, double* ms);
/* Set the launch configuration explicitly (mode 0, 1 or 2, grid >= 1
 * workgroups, tile_groups >= 1; mode 2 uses neither). */
int hd_batch_set_launch(hd_ctx* ctx, int mode, int grid, int tile_groups);
/* Each instance's diagonal, S~ and AMG (Section 2.3, eq. approx-schur;
 * learned must be 0).  The batched MINRES runs the levels >= 1 of the
 * V-cycles (Section 3: one scalar AMG V-cycle per iteration and instance) of
 * all instances whose hierarchy has at least two levels and a non-singular
 * S~ in shared launches, one per operation and level, with the same results
 * as the instances' own cycles; the other instances keep their own. */
int hd_batch_build_precond(hd_ctx* ctx, const hd_precond_params* params);
/* shared = 1 (the default): the shared V-cycle launches above where they
 * apply, and the recurrence's vector updates and scalar steps of all
 * instances in one launch each (same results); 0: every instance's V-cycle
 * and recurrence kernels launched on their own.  HD_ERR_STATE before
 * hd_setup_batch, HD_ERR_ARG for another value. */
int hd_batch_set_vcycle(hd_ctx* ctx, int shared);
/* One MINRES recurrence per instance (Section 2.2), in any HD_MODE_*.  HD_MODE_MIXED
 * refines every instance on its own FP64 residual around one batched FP32
 * MINRES per refinement step (instances already converged get a zero
 * right-hand side); info: host array of ninst entries (may be NULL). */
int hd_batch_minres_solve(hd_ctx* ctx, const hd_solve_params* params, const double* b, double* x,
                          hd_solve_info* info);

/* ---- learned (1,1)-diagonal correction ---------------------------------
 * Not in the paper: an extension of its diagonal (1,1) block (Section 2.3).
 * Six log-scalings theta = (x-, x+, y-, y+, z-, z+) per element multiply the
 * element's contribution to diag(M): an RT dof of component c with index i
 * along c (Gauss-Lobatto sub-element vertex xi_i on [0, 1]) is scaled by
 * exp((1 - xi_i) theta_{2c} + xi_i theta_{2c+1}).  The network maps
 * x in R^27 (24 vertex offsets from the centroid divided by the mean edge
 * length, vertex order (dz, dy, dx) with the coordinate fastest; ln alpha;
 * ln beta; p / 6) through Linear(27,64)-GELU-Linear(64,64)-GELU-Linear(64,6)
 * (exact GELU) to theta = clip(o, -ln 4, ln 4).  Parameters (FP32, flat):
 * W1[64][27], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]. */

/* Training targets: for n single elements of order p (vertices: device
 * [n][2][2][2][3], indexed (dz, dy, dx, coord)), theta* minimising
 * log lambda_max - log lambda_min of the pencil (M_e, diag(s * diag M_e))
 * for unit coefficient on sum(theta) = 0, by at most max_steps projected
 * gradient steps with Armijo backtracking from theta = 0 (eigenpairs by
 * Lanczos, matrix-free).  Outputs (device, caller-owned): theta [n][6];
 * lam [n][2] = (lambda_min, lambda_max) at theta* (may be NULL); spread
 * [n][2] = (value at 0, value at theta*) (may be NULL).  An element with a
 * non-positive Jacobian gets NaN.  Synchronises. */
int hd_learned_targets(hd_ctx* ctx, int p, int64_t n, const double* vertices, int max_steps,
                       double* theta, double* lam, double* spread);

/* Features x [n][27] (device, FP32) of n elements: vertices as above,
 * alpha, beta [n] (device FP64), p_per_elem [n] (device int) or NULL with
 * the constant p. */
int hd_learned_features(hd_ctx* ctx, int64_t n, const double* vertices, const double* alpha,
                        const double* beta, const int* p_per_elem, int p, float* x);

/* Number of network parameters (6342). */
int hd_mlp_param_count(void);
/* Initialise the parameters (W ~ U(+-1/sqrt(fan_in)), b = 0) from seed, or
 * set / get them from / to a host array; both reset the Adam state. */
int hd_mlp_init(hd_ctx* ctx, uint64_t seed);
int hd_mlp_set_params(hd_ctx* ctx, const float* params);
int hd_mlp_get_params(hd_ctx* ctx, float* params);
/* Mean squared error (over the n x 6 outputs, targets clipped to +-ln 4) of
 * the rows x [n][27], y [n][6] (device FP32) and its gradient (host, 6342
 * entries, may be NULL). */
int hd_mlp_loss_grad(hd_ctx* ctx, int64_t n, const float* x, const float* y, float* loss, float* grad);
/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) over
 * `epochs` passes of shuffled mini-batches of `batch` rows; per-epoch mean
 * training loss and validation loss (n_val rows, may be 0) into host arrays
 * of `epochs` entries (may be NULL).  Synchronises. */
int hd_mlp_train(hd_ctx* ctx, int64_t n, const float* x, const float* y, int64_t n_val, const float* x_val,
                 const float* y_val, int epochs, int batch, float lr, uint64_t seed, float* train_loss,
                 float* val_loss);
/* theta [n][6] = clip(o, +-ln 4) for rows x [n][27] (device FP32); bf16 = 1
 * runs the network in BF16 on the matrix cores (FP32 accumulation). */
int hd_mlp_infer(hd_ctx* ctx, int64_t n, const float* x, float* theta, int bf16);
/* Per-element log-scalings [ne][6] (device FP64, copied) used by
 * hd_build_precond with learned = 2; NULL clears them. */
int hd_set_diag_scalings(hd_ctx* ctx, const double* theta);

/* ---- inspection (parity checks) ---------------------------------------- */

/* Copy diag(M) (n_u; M~ of Section 2.3, 1 on essential dofs) and diag(W)
 * (unweighted, n_q; the diagonal behind C~ of eq. approx-schur) into device
 * buffers. */
int hd_get_diagonals(hd_ctx* ctx, double* m_diag, double* w_diag);

/* S~ (eq. approx-schur-entries) in CSR: query nnz with rowptr == NULL, then pass host buffers of n_q+1,
 * nnz, nnz entries. */
int hd_get_schur(hd_ctx* ctx, int64_t* nnz, int32_t* rowptr, int32_t* col, double* val);

/* The AMG hierarchy of S~ (Section 3.2, Schur complement preconditioning; a
 * smoothed-aggregation hierarchy in place of the paper's BoomerAMG).
 * Number of AMG levels and the size/nnz of level `level` (A), and, when the
 * buffers are non-NULL, its CSR arrays (host).  For level < nlevels-1 the
 * prolongator P (rows of level, cols of level+1) is returned by
 * hd_get_amg_prolongator. */
int hd_get_amg_nlevels(hd_ctx* ctx, int* nlevels);
int hd_get_amg_level(hd_ctx* ctx, int level, int64_t* n, int64_t* nnz,
                     int32_t* rowptr, int32_t* col, double* val);
int hd_get_amg_prolongator(hd_ctx* ctx, int level, int64_t* nrows, int64_t* ncols, int64_t* nnz,
                           int32_t* rowptr, int32_t* col, double* val);

/* Measurement helper (no passage of the method): average device duration
 * (ms) of the block-apply kernel over the calls since
 * the last reset, measured with events on the context stream (reset = 1
 * clears the accumulators). */
int hd_apply_timing(hd_ctx* ctx, int reset, double* avg_ms, int64_t* count);

/* ---- grey nonlinear radiation diffusion (Section 4.3) ------------------- */

/* (D F)_j for an RT vector F: the signed sum of the fluxes through the six
 * faces of sub-cell j (D = W^{-1} B, the +-1 incidence of the interpolation-
 * histopolation basis, Section 2.1, Algorithm 1), i.e. the q-part of the block
 * operator applied to [F; 0].  F: FP64 device array of n_u values; q: FP64
 * device array of n_q values; caller-owned.  Asynchronous on the context's
 * stream.  HD_ERR_STATE before a mesh, HD_ERR_ARG for NULL pointers. */
int hd_apply_divergence(hd_ctx* ctx, const double* F, double* q);

/* |K_j| for every L2 dof: the physical volume of its sub-cell (the mapped
 * Gauss-Lobatto sub-cell of Section 2.1), det J integrated by 2 x 2 x 2
 * Gauss-Legendre points per sub-cell (exact for the trilinear map).  An L2
 * dof of the transformed space is the integral of the function over its
 * sub-cell, so a density f is represented by f |K_j|.  vol: FP64 device
 * array of n_q values, caller-owned.  Asynchronous.  HD_ERR_STATE before a
 * mesh. */
int hd_subcell_volumes(hd_ctx* ctx, double* vol);

/* Parameters of the radiation-diffusion time step (Section 4.3, eqs. rad-diff-e,
 * rad-diff-E, rad-diff-F with Q = S = 0 and constant coefficients). */
typedef struct hd_rd_params {
    double rho, cv, c, a, sigma;  /* density, specific heat, speed of light,
                                     radiation constant, opacity; all > 0 */
    double dt;                    /* time step > 0 */
    double tol_outer;             /* stop of a stage's outer iteration:
                                     ||R_e|| / (||e - e^|| / (g dt) + c sigma ||E||)
                                     with R_e the material-energy residual after
                                     the Darcy solve; default 1e-10 */
    int max_outer;                /* default 20 */
    double newton_tol;            /* per-dof Newton: both updates below
                                     newton_tol times the iterate; default 1e-12 */
    int newton_max_it;            /* default 50 */
    double lin_tol;               /* each Darcy MINRES: |eta| <= lin_tol |eta_0|
                                     from the previous solution as initial guess;
                                     default 1e-8 */
    int lin_max_it;               /* default 10000 */
    int lin_mode;                 /* HD_MODE_* of the Darcy solves; default
                                     HD_MODE_PLAIN64.  With HD_MODE_MIXED a
                                     solve stops when its true FP64 residual
                                     has fallen by lin_tol from that of its
                                     initial guess */
} hd_rd_params;

typedef struct hd_rd_info {
    int status;                   /* 0, or HD_NOT_CONVERGED when a stage's
                                     outer iteration or a Darcy solve hit its limit */
    int outer[3];                 /* outer iterations of each stage */
    int newton_max_it;            /* largest Newton count of any dof in the step */
    int linear_solves;            /* Darcy solves in the step */
    int linear_iterations;        /* MINRES iterations summed over them */
    double e_residual[3];         /* the last outer residual of each stage */
    double time_s;                /* wall time of the step */
    double linear_time_s;         /* of which in the Darcy solves (MINRES) */
} hd_rd_info;

/* Fill *p with the defaults above (rho = cv = c = a = sigma = dt = 1). */
int hd_rd_default_params(hd_rd_params* p);

/* Prepare the context for hd_rd_step on its mesh (structured, or
 * unstructured): the coefficients of the Darcy system of a stage
 * (HD_DARCY, c_mass = 3 sigma / c, gamma = kappa = 1 / (g dt) + c sigma with
 * g the SDIRK diagonal, every boundary RT dof essential: F . n = 0), the
 * preconditioner (precond may be NULL for the defaults of hd_build_precond),
 * the sub-cell volumes and the work space (14 n_q + 3 (n_u + n_q) doubles).
 * Replaces any coefficients and preconditioner the context held.  Errors:
 * HD_ERR_STATE before a mesh, HD_ERR_ARG for a parameter out of range, and
 * those of hd_setup_coeffs and hd_build_precond. */
int hd_rd_setup(hd_ctx* ctx, const hd_rd_params* params, const hd_precond_params* precond);

/* One step of length dt of the three-stage L-stable SDIRK method of
 * Alexander (1977, Section 4.3), stiffly accurate, each stage solved by the
 * outer iteration of Section 4.3: (1) F lagged, the 2 x 2 nonlinear system
 * of every L2 dof for (e_j, E_j) by Newton's method from the stage's
 * e^, E^; (2) e fixed, the Darcy system kappa E + D F = E^ / (g dt) +
 * c sigma a T^4 |K|, M_{3 sigma / c} F - B^T E = 0 in the transformed form
 * with unknowns (F, -W E), by block-preconditioned MINRES from the previous
 * solution; repeated until tol_outer.  e_j, E_j are energy amounts per
 * sub-cell (the integrals of rho e and E over K_j), T_j = e_j / (rho C_v |K_j|).
 * e, E: FP64 device arrays of n_q values; F: FP64 device array of n_u values
 * (zero on the boundary); all caller-owned, updated in place to t + dt.
 * Synchronises the stream.  info may be NULL.  Returns 0, HD_NOT_CONVERGED
 * when a stage's outer iteration or a Darcy solve reached its limit (state
 * still updated), HD_ERR_NONFINITE when the Newton iteration of some dof
 * does not meet newton_tol within newton_max_it or ends at a non-positive
 * or non-finite energy, or a residual is not finite (state not updated),
 * HD_ERR_STATE before hd_rd_setup, HD_ERR_ARG for NULL or aliased
 * pointers. */
int hd_rd_step(hd_ctx* ctx, double* e, double* E, double* F, hd_rd_info* info);

/* ---- host-only entry (no device needed) -------------------------------- */

/* Build the aggregation AMG hierarchy (the set-up of Section 3.2's Schur
 * complement preconditioner, as the device builds it) of a host CSR matrix
 * with the library's host code and return level sizes; the hierarchy is kept in a
 * host handle for hd_host_amg_level / hd_host_amg_free.  For checks on
 * machines without a GPU. */
typedef struct hd_host_amg hd_host_amg;
int hd_host_amg_build(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                      const hd_precond_params* params, int singular, hd_host_amg** out);
int hd_host_amg_nlevels(const hd_host_amg* h);
int hd_host_amg_level(const hd_host_amg* h, int level, int64_t* n, int64_t* nnz,
                      int32_t* rowptr, int32_t* col, double* val);
int hd_host_amg_prolongator(const hd_host_amg* h, int level, int64_t* nrows, int64_t* ncols,
                            int64_t* nnz, int32_t* rowptr, int32_t* col, double* val);
int hd_host_amg_free(hd_host_amg* h);

/* The RT numbering of an unstructured mesh as hd_setup_mesh_unstructured
 * builds it, on the host only (no device, no context): n_u and, when l2g is
 * not NULL, the element-to-dof map of hd_get_dof_map ([ne][3 p^2 (p+1)]).
 * Errors as hd_setup_mesh_unstructured for the element array. */
int hd_host_unstructured_map(int64_t nv, int64_t ne, const int64_t* elements, int p, int64_t* n_u,
                             int32_t* l2g);

/* 1D tables of degree p as computed by the library (host, no device):
 * Gauss-Lobatto points (p+1), Gauss-Legendre points and weights (p+1). */
int hd_host_tables(int p, double* gll, double* gl_x, double* gl_w);

#ifdef __cplusplus
}
#endif
#endif
