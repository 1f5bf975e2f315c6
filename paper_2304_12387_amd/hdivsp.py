"""Thin ctypes binding of libhdivsp (include/hdivsp.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers are torch tensors on the context's device; the context is
bound to torch's current HIP stream unless another stream is given.  If the
library is missing or cannot be loaded this module raises, it never falls
back to another implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libhdivsp.so')

HD_OK = 0
HD_ERR_ARG, HD_ERR_MESH, HD_ERR_HIP, HD_ERR_OOM, HD_ERR_AMG = -1, -2, -3, -4, -5
HD_ERR_BREAKDOWN, HD_ERR_NONFINITE, HD_ERR_STATE = -6, -7, -8
HD_NOT_CONVERGED, HD_FALLBACK_USED = 1, 2
HD_GRADDIV, HD_DARCY = 0, 1
HD_F64, HD_F32 = 0, 1
HD_MODE_PLAIN64, HD_MODE_MIXED, HD_MODE_PREC32 = 0, 1, 2
HD_SIDE_ALL = 63
HD_LOCAL_AUTO, HD_LOCAL_CG, HD_LOCAL_EXPLICIT = 0, 1, 2

EXPORTED = [
    'hd_create', 'hd_destroy', 'hd_last_error', 'hd_setup_mesh', 'hd_setup_coeffs', 'hd_sizes', 'hd_mesh_affine',
    'hd_apply_block_op', 'hd_apply_mass_inverse', 'hd_apply_l2_mass_inverse', 'hd_lift_essential',
    'hd_build_precond', 'hd_apply_precond', 'hd_minres_solve', 'hd_get_diagonals', 'hd_get_schur',
    'hd_get_amg_nlevels', 'hd_get_amg_level', 'hd_get_amg_prolongator', 'hd_apply_timing',
    'hd_host_amg_build', 'hd_host_amg_nlevels', 'hd_host_amg_level', 'hd_host_amg_prolongator',
    'hd_host_amg_free', 'hd_host_tables', 'hd_learned_targets', 'hd_learned_features', 'hd_mlp_param_count',
    'hd_mlp_init', 'hd_mlp_set_params', 'hd_mlp_get_params', 'hd_mlp_loss_grad', 'hd_mlp_train', 'hd_mlp_infer',
    'hd_set_diag_scalings', 'hd_setup_batch', 'hd_batch_sizes', 'hd_batch_apply', 'hd_batch_tune',
    'hd_batch_set_launch', 'hd_batch_build_precond', 'hd_batch_minres_solve', 'hd_constant_flux',
    'hd_set_local_solver', 'hd_set_gamma_field', 'hd_gmres_solve', 'hd_apply_tri_precond',
    'hd_apply_tri_precond_noalloc', 'hd_setup_mesh_unstructured', 'hd_set_essential_dofs', 'hd_get_dof_map',
    'hd_host_unstructured_map', 'hd_apply_block_op_interleaved', 'hd_apply_divergence', 'hd_subcell_volumes',
    'hd_rd_default_params', 'hd_rd_setup', 'hd_rd_step', 'hd_batch_set_vcycle',
]


class HdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'hdivsp error {code}: {msg}')
        self.code = code


class PrecondParams(ctypes.Structure):
    _fields_ = [('tau', ctypes.c_double), ('theta', ctypes.c_double), ('max_coarse', ctypes.c_int),
                ('max_levels', ctypes.c_int), ('omega', ctypes.c_double), ('learned', ctypes.c_int)]


class SolveParams(ctypes.Structure):
    _fields_ = [('tol', ctypes.c_double), ('max_it', ctypes.c_int), ('mode', ctypes.c_int),
                ('use_x0', ctypes.c_int), ('inner_tol', ctypes.c_double), ('max_outer', ctypes.c_int),
                ('check_every', ctypes.c_int), ('stop_true', ctypes.c_int), ('use_graph', ctypes.c_int)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [('nx', ctypes.c_int), ('ny', ctypes.c_int), ('nz', ctypes.c_int), ('p', ctypes.c_int),
                ('vertices', ctypes.c_void_p), ('c_mass', ctypes.c_void_p), ('c_22', ctypes.c_void_p),
                ('ess_sides', ctypes.c_uint32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [('status', ctypes.c_int), ('iterations', ctypes.c_int), ('outer', ctypes.c_int),
                ('eta_rel', ctypes.c_double), ('true_rel_res', ctypes.c_double), ('time_s', ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RdParams(ctypes.Structure):
    _fields_ = [('rho', ctypes.c_double), ('cv', ctypes.c_double), ('c', ctypes.c_double), ('a', ctypes.c_double),
                ('sigma', ctypes.c_double), ('dt', ctypes.c_double), ('tol_outer', ctypes.c_double),
                ('max_outer', ctypes.c_int), ('newton_tol', ctypes.c_double), ('newton_max_it', ctypes.c_int),
                ('lin_tol', ctypes.c_double), ('lin_max_it', ctypes.c_int), ('lin_mode', ctypes.c_int)]


class RdInfo(ctypes.Structure):
    _fields_ = [('status', ctypes.c_int), ('outer', ctypes.c_int * 3), ('newton_max_it', ctypes.c_int),
                ('linear_solves', ctypes.c_int), ('linear_iterations', ctypes.c_int),
                ('e_residual', ctypes.c_double * 3), ('time_s', ctypes.c_double), ('linear_time_s', ctypes.c_double)]

    def as_dict(self):
        return {'status': self.status, 'outer': list(self.outer), 'newton_max_it': self.newton_max_it,
                'linear_solves': self.linear_solves, 'linear_iterations': self.linear_iterations,
                'e_residual': list(self.e_residual), 'time_s': self.time_s, 'linear_time_s': self.linear_time_s}


_lib = None


def load():
    """Load libhdivsp.so (torch is imported first so that the library binds
    to the HIP runtime torch already loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f'{LIB_PATH} is missing: build it with `python -m paper_2304_12387_amd.build`')
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    D = ctypes.c_double
    pI64 = ctypes.POINTER(I64)
    sigs = {
        'hd_create': (I, [ctypes.POINTER(P), I, P]),
        'hd_destroy': (I, [P]),
        'hd_last_error': (ctypes.c_char_p, [P]),
        'hd_setup_mesh': (I, [P, I, I, I, I, P]),
        'hd_setup_coeffs': (I, [P, I, P, P, ctypes.c_uint32]),
        'hd_setup_mesh_unstructured': (I, [P, I64, P, I64, P, I]),
        'hd_set_essential_dofs': (I, [P, P]),
        'hd_get_dof_map': (I, [P, P]),
        'hd_sizes': (I, [P, pI64, pI64]),
        'hd_mesh_affine': (I, [P, ctypes.POINTER(ctypes.c_int)]),
        'hd_apply_block_op': (I, [P, I, I, P, P]),
        'hd_apply_block_op_interleaved': (I, [P, I, I, P, P]),
        'hd_apply_mass_inverse': (I, [P, I, I, P, P]),
        'hd_set_local_solver': (I, [P, I]),
        'hd_set_gamma_field': (I, [P, P]),
        'hd_gmres_solve': (I, [P, D, I, I, P, P, ctypes.POINTER(SolveInfo)]),
        'hd_apply_tri_precond': (I, [P, P, P]),
        'hd_apply_tri_precond_noalloc': (I, [P, P, P]),
        'hd_apply_l2_mass_inverse': (I, [P, I, P, P]),
        'hd_lift_essential': (I, [P, P, P]),
        'hd_build_precond': (I, [P, ctypes.POINTER(PrecondParams)]),
        'hd_apply_precond': (I, [P, I, I, P, P]),
        'hd_minres_solve': (I, [P, ctypes.POINTER(SolveParams), I, P, P, ctypes.POINTER(SolveInfo)]),
        'hd_get_diagonals': (I, [P, P, P]),
        'hd_get_schur': (I, [P, pI64, P, P, P]),
        'hd_get_amg_nlevels': (I, [P, ctypes.POINTER(I)]),
        'hd_get_amg_level': (I, [P, I, pI64, pI64, P, P, P]),
        'hd_get_amg_prolongator': (I, [P, I, pI64, pI64, pI64, P, P, P]),
        'hd_apply_timing': (I, [P, I, ctypes.POINTER(D), pI64]),
        'hd_host_amg_build': (I, [I64, P, P, P, ctypes.POINTER(PrecondParams), I, ctypes.POINTER(P)]),
        'hd_host_amg_nlevels': (I, [P]),
        'hd_host_amg_level': (I, [P, I, pI64, pI64, P, P, P]),
        'hd_host_amg_prolongator': (I, [P, I, pI64, pI64, pI64, P, P, P]),
        'hd_host_amg_free': (I, [P]),
        'hd_host_tables': (I, [I, P, P, P]),
        'hd_host_unstructured_map': (I, [I64, I64, P, I, pI64, P]),
        'hd_learned_targets': (I, [P, I, I64, P, I, P, P, P]),
        'hd_learned_features': (I, [P, I64, P, P, P, P, I, P]),
        'hd_mlp_param_count': (I, []),
        'hd_mlp_init': (I, [P, ctypes.c_uint64]),
        'hd_mlp_set_params': (I, [P, P]),
        'hd_mlp_get_params': (I, [P, P]),
        'hd_mlp_loss_grad': (I, [P, I64, P, P, ctypes.POINTER(ctypes.c_float), P]),
        'hd_mlp_train': (I, [P, I64, P, P, I64, P, P, I, I, ctypes.c_float, ctypes.c_uint64, P, P]),
        'hd_mlp_infer': (I, [P, I64, P, P, I]),
        'hd_set_diag_scalings': (I, [P, P]),
        'hd_constant_flux': (I, [P, P, P]),
        'hd_setup_batch': (I, [P, I, I, ctypes.POINTER(InstanceDesc)]),
        'hd_batch_sizes': (I, [P, P, P]),
        'hd_batch_apply': (I, [P, I, P, P]),
        'hd_batch_tune': (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D)]),
        'hd_batch_set_launch': (I, [P, I, I, I]),
        'hd_batch_set_vcycle': (I, [P, I]),
        'hd_batch_build_precond': (I, [P, ctypes.POINTER(PrecondParams)]),
        'hd_batch_minres_solve': (I, [P, ctypes.POINTER(SolveParams), P, P, ctypes.POINTER(SolveInfo)]),
        'hd_apply_divergence': (I, [P, P, P]),
        'hd_subcell_volumes': (I, [P, P]),
        'hd_rd_default_params': (I, [ctypes.POINTER(RdParams)]),
        'hd_rd_setup': (I, [P, ctypes.POINTER(RdParams), ctypes.POINTER(PrecondParams)]),
        'hd_rd_step': (I, [P, P, P, P, ctypes.POINTER(RdInfo)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    """Device pointer of a torch tensor or host pointer of a numpy array."""
    if a is None:
        return None
    if hasattr(a, 'data_ptr'):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def rd_params(**kw):
    """hd_rd_params with the library's defaults, overridden by keyword."""
    p = RdParams()
    load().hd_rd_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise ValueError(f'unknown radiation-diffusion parameter {k}')
        setattr(p, k, v)
    return p


def precond_params(tau=1.0, theta=0.25, max_coarse=1024, max_levels=25, omega=2.0 / 3.0, learned=0):
    return PrecondParams(tau, theta, max_coarse, max_levels, omega, learned)


def solve_params(tol=1e-8, max_it=10000, mode=HD_MODE_PLAIN64, use_x0=0, inner_tol=1e-5, max_outer=20,
                 check_every=8, stop_true=0, use_graph=1):
    return SolveParams(tol, max_it, mode, use_x0, inner_tol, max_outer, check_every, stop_true, use_graph)


class Context:
    """An hd_ctx bound to one device and one HIP stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.lib = load()
        self.torch = torch
        self.device = torch.device('cuda', device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.hd_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise HdError(rc, 'hd_create failed')
        self.h = h

    def close(self):
        if self.h:
            self.lib.hd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise HdError(rc, self.lib.hd_last_error(self.h).decode())
        return rc

    # ---- setup ------------------------------------------------------------
    def setup_mesh(self, nx, ny, nz, p, vertices):
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        if v.size != 3 * (nx + 1) * (ny + 1) * (nz + 1):
            raise ValueError('vertices: (nx+1)(ny+1)(nz+1) x 3 entries required')
        rc = self._check(self.lib.hd_setup_mesh(self.h, nx, ny, nz, p, _ptr(v)))
        self.ne = nx * ny * nz
        return rc

    def setup_mesh_unstructured(self, vertices, elements, p):
        v = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1, 3)
        el = np.ascontiguousarray(elements, dtype=np.int64).reshape(-1, 8)
        rc = self._check(self.lib.hd_setup_mesh_unstructured(self.h, v.shape[0], _ptr(v), el.shape[0], _ptr(el), p))
        self.ne = el.shape[0]
        self.p_uns = p
        return rc

    def set_essential_dofs(self, mask):
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if m.size != self.sizes()[0]:
            raise ValueError('mask: n_u entries required')
        return self._check(self.lib.hd_set_essential_dofs(self.h, _ptr(m)))

    def get_dof_map(self):
        p = self.p_uns
        out = np.empty((self.ne, 3 * p * p * (p + 1)), dtype=np.int32)
        self._check(self.lib.hd_get_dof_map(self.h, _ptr(out)))
        return out

    def setup_coeffs(self, problem, c_mass, c_22=None, ess_sides=0):
        cm = np.ascontiguousarray(c_mass, dtype=np.float64)
        c2 = None if c_22 is None else np.ascontiguousarray(c_22, dtype=np.float64)
        return self._check(self.lib.hd_setup_coeffs(self.h, problem, _ptr(cm), _ptr(c2), ess_sides))

    def sizes(self):
        nu, nq = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.hd_sizes(self.h, ctypes.byref(nu), ctypes.byref(nq)))
        return nu.value, nq.value

    def mesh_affine(self):
        """True when every element of the structured mesh is a parallelepiped."""
        a = ctypes.c_int()
        self._check(self.lib.hd_mesh_affine(self.h, ctypes.byref(a)))
        return bool(a.value)

    def _dev(self, a, n, prec, name):
        """Refuse a buffer the kernels would read or write out of bounds."""
        torch = self.torch
        want = torch.float64 if prec == HD_F64 else torch.float32
        if not (hasattr(a, 'is_cuda') and a.is_cuda and a.is_contiguous()):
            raise ValueError(f"{name}: a contiguous device tensor is required")
        if a.dtype != want:
            raise ValueError(f"{name}: dtype {a.dtype}, expected {want}")
        if a.numel() < n:
            raise ValueError(f"{name}: {a.numel()} entries, at least {n} required")

    # ---- operator ---------------------------------------------------------
    def apply_block_op(self, x, y, prec=HD_F64, nrhs=1):
        nu, nq = self.sizes()
        self._dev(x, nrhs * (nu + nq), prec, 'x')
        self._dev(y, nrhs * (nu + nq), prec, 'y')
        return self._check(self.lib.hd_apply_block_op(self.h, prec, nrhs, _ptr(x), _ptr(y)))

    def apply_block_op_interleaved(self, x, y, nrhs, prec=HD_F64):
        """y = A x for nrhs right-hand sides interleaved ([dof][nrhs])."""
        nu, nq = self.sizes()
        self._dev(x, nrhs * (nu + nq), prec, 'x')
        self._dev(y, nrhs * (nu + nq), prec, 'y')
        return self._check(self.lib.hd_apply_block_op_interleaved(self.h, prec, nrhs, _ptr(x), _ptr(y)))

    def set_gamma_field(self, gamma_vertices):
        """Darcy: gamma as the trilinear field of these vertex values (host
        array, (nx+1)(ny+1)(nz+1)); the (2,2) block becomes W^-1 W_gamma W^-1."""
        g = np.ascontiguousarray(gamma_vertices, dtype=np.float64).reshape(-1)
        return self._check(self.lib.hd_set_gamma_field(self.h, _ptr(g)))

    def set_local_solver(self, mode):
        """HD_LOCAL_AUTO (explicit W_e^{-1} for p <= 2, local CG otherwise),
        HD_LOCAL_CG or HD_LOCAL_EXPLICIT (p <= 2)."""
        return self._check(self.lib.hd_set_local_solver(self.h, mode))

    def apply_mass_inverse(self, x, y, prec=HD_F64, nrhs=1):
        nu, nq = self.sizes()
        self._dev(x, nrhs * nq, prec, 'x')
        self._dev(y, nrhs * nq, prec, 'y')
        return self._check(self.lib.hd_apply_mass_inverse(self.h, prec, nrhs, _ptr(x), _ptr(y)))

    def apply_l2_mass_inverse(self, x, y, prec=HD_F64):
        nu, nq = self.sizes()
        self._dev(x, nq, prec, 'x')
        self._dev(y, nq, prec, 'y')
        return self._check(self.lib.hd_apply_l2_mass_inverse(self.h, prec, _ptr(x), _ptr(y)))

    def constant_flux(self, u):
        """RT dofs (device tensor of n_u) of the constant field u (3 floats)."""
        nu, _ = self.sizes()
        uu = np.ascontiguousarray(u, dtype=np.float64)
        if uu.size != 3:
            raise ValueError('u: three components required')
        out = self.torch.empty(nu, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.hd_constant_flux(self.h, _ptr(uu), _ptr(out)))
        return out

    def lift_essential(self, u_bc, b):
        nu, nq = self.sizes()
        self._dev(u_bc, nu, HD_F64, 'u_bc')
        self._dev(b, nu + nq, HD_F64, 'b')
        return self._check(self.lib.hd_lift_essential(self.h, _ptr(u_bc), _ptr(b)))

    # ---- preconditioner and solver -----------------------------------------
    def build_precond(self, params=None):
        """Returns 0, or HD_FALLBACK_USED when the learned scalings were not
        finite and the plain diagonal was used."""
        pp = ctypes.byref(params) if params is not None else None
        return self._check(self.lib.hd_build_precond(self.h, pp), allow=(HD_FALLBACK_USED,))

    # ---- batches of independent instances ---------------------------------
    def setup_batch(self, problem, instances):
        """instances: dicts with nx, ny, nz, p, vertices, c_mass, c_22, ess_sides."""
        keep = []
        arr = (InstanceDesc * len(instances))()
        for i, d in enumerate(instances):
            v = np.ascontiguousarray(d['vertices'], dtype=np.float64)
            cm = np.ascontiguousarray(d['c_mass'], dtype=np.float64)
            c2 = None if d.get('c_22') is None else np.ascontiguousarray(d['c_22'], dtype=np.float64)
            nx, ny, nz = d['nx'], d['ny'], d['nz']
            if v.size != 3 * (nx + 1) * (ny + 1) * (nz + 1) or cm.size != nx * ny * nz or \
                    (c2 is not None and c2.size != nx * ny * nz):
                raise ValueError(f'instance {i}: array sizes do not match the mesh')
            keep += [v, cm, c2]
            arr[i] = InstanceDesc(nx, ny, nz, d['p'], v.ctypes.data, cm.ctypes.data,
                                  None if c2 is None else c2.ctypes.data, d.get('ess_sides', 0))
        rc = self._check(self.lib.hd_setup_batch(self.h, problem, len(instances), arr))
        self.ninst = len(instances)
        off = np.zeros(self.ninst + 1, dtype=np.int64)
        nu = np.zeros(self.ninst, dtype=np.int64)
        self._check(self.lib.hd_batch_sizes(self.h, _ptr(off), _ptr(nu)))
        self.batch_offsets, self.batch_nu = off, nu
        return rc

    def batch_apply(self, x, y, prec=HD_F64):
        n = int(self.batch_offsets[-1])
        self._dev(x, n, prec, 'x')
        self._dev(y, n, prec, 'y')
        return self._check(self.lib.hd_batch_apply(self.h, prec, _ptr(x), _ptr(y)))

    def batch_tune(self, prec=HD_F64):
        m, g, t, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(self.lib.hd_batch_tune(self.h, prec, ctypes.byref(m), ctypes.byref(g), ctypes.byref(t),
                                           ctypes.byref(ms)))
        return dict(mode=m.value, grid=g.value, tile_groups=t.value, ms=ms.value)

    def batch_set_launch(self, mode, grid, tile_groups):
        return self._check(self.lib.hd_batch_set_launch(self.h, mode, grid, tile_groups))

    def batch_set_vcycle(self, shared):
        """1: the instances' V-cycle levels >= 1 in shared launches; 0: each
        instance's own launches."""
        return self._check(self.lib.hd_batch_set_vcycle(self.h, int(shared)))

    def batch_build_precond(self, params=None):
        pp = ctypes.byref(params) if params is not None else None
        return self._check(self.lib.hd_batch_build_precond(self.h, pp))

    def batch_minres_solve(self, b, x, params=None):
        n = int(self.batch_offsets[-1])
        self._dev(b, n, HD_F64, 'b')
        self._dev(x, n, HD_F64, 'x')
        info = (SolveInfo * self.ninst)()
        pp = ctypes.byref(params) if params is not None else None
        rc = self.lib.hd_batch_minres_solve(self.h, pp, _ptr(b), _ptr(x), info)
        self._check(rc, allow=(HD_NOT_CONVERGED,))
        return [i.as_dict() for i in info]

    # ---- learned (1,1)-diagonal correction ----------------------------------
    def learned_targets(self, p, vertices, max_steps=30):
        """theta* [n, 6], (lambda_min, lambda_max) [n, 2] and the spread at 0
        and at theta* [n, 2] for elements vertices [n, 2, 2, 2, 3] (device
        float64 tensor)."""
        torch = self.torch
        n = vertices.shape[0]
        self._dev(vertices, n * 24, HD_F64, 'vertices')
        th = torch.empty((n, 6), dtype=torch.float64, device=self.device)
        lam = torch.empty((n, 2), dtype=torch.float64, device=self.device)
        spr = torch.empty((n, 2), dtype=torch.float64, device=self.device)
        self._check(self.lib.hd_learned_targets(self.h, p, n, _ptr(vertices), max_steps, _ptr(th), _ptr(lam),
                                                _ptr(spr)))
        return th, lam, spr

    def learned_features(self, vertices, alpha, beta, p):
        """x [n, 27] (float32) for elements vertices [n, 2, 2, 2, 3]; p an int
        or an int32 device tensor [n]."""
        torch = self.torch
        n = vertices.shape[0]
        self._dev(vertices, n * 24, HD_F64, 'vertices')
        self._dev(alpha, n, HD_F64, 'alpha')
        self._dev(beta, n, HD_F64, 'beta')
        parr = None
        if hasattr(p, 'data_ptr'):
            if p.dtype != torch.int32 or not p.is_cuda or p.numel() < n:
                raise ValueError('p: an int32 device tensor with one entry per element is required')
            parr, p = p, 0
        x = torch.empty((n, 27), dtype=torch.float32, device=self.device)
        self._check(self.lib.hd_learned_features(self.h, n, _ptr(vertices), _ptr(alpha), _ptr(beta), _ptr(parr),
                                                 int(p), _ptr(x)))
        return x

    def mlp_init(self, seed=0):
        return self._check(self.lib.hd_mlp_init(self.h, seed))

    def mlp_set_params(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.lib.hd_mlp_param_count():
            raise ValueError('wrong parameter count')
        return self._check(self.lib.hd_mlp_set_params(self.h, _ptr(a)))

    def mlp_get_params(self):
        a = np.empty(self.lib.hd_mlp_param_count(), dtype=np.float32)
        self._check(self.lib.hd_mlp_get_params(self.h, _ptr(a)))
        return a

    def mlp_loss_grad(self, x, y):
        n = x.shape[0]
        self._dev(x, n * 27, HD_F32, 'x')
        self._dev(y, n * 6, HD_F32, 'y')
        loss = ctypes.c_float()
        g = np.empty(self.lib.hd_mlp_param_count(), dtype=np.float32)
        self._check(self.lib.hd_mlp_loss_grad(self.h, n, _ptr(x), _ptr(y), ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def mlp_train(self, x, y, x_val=None, y_val=None, epochs=10, batch=512, lr=1e-3, seed=0):
        n = x.shape[0]
        self._dev(x, n * 27, HD_F32, 'x')
        self._dev(y, n * 6, HD_F32, 'y')
        nv = 0 if x_val is None else x_val.shape[0]
        if nv:
            self._dev(x_val, nv * 27, HD_F32, 'x_val')
            self._dev(y_val, nv * 6, HD_F32, 'y_val')
        tl = np.zeros(epochs, dtype=np.float32)
        vl = np.zeros(epochs, dtype=np.float32)
        self._check(self.lib.hd_mlp_train(self.h, n, _ptr(x), _ptr(y), nv, _ptr(x_val), _ptr(y_val), epochs, batch,
                                          lr, seed, _ptr(tl), _ptr(vl)))
        return tl, vl

    def mlp_infer(self, x, bf16=True):
        torch = self.torch
        n = x.shape[0]
        self._dev(x, n * 27, HD_F32, 'x')
        th = torch.empty((n, 6), dtype=torch.float32, device=self.device)
        self._check(self.lib.hd_mlp_infer(self.h, n, _ptr(x), _ptr(th), 1 if bf16 else 0))
        return th

    def set_diag_scalings(self, theta):
        if theta is not None:
            self._dev(theta, self.ne * 6, HD_F64, 'theta')
        return self._check(self.lib.hd_set_diag_scalings(self.h, _ptr(theta)))

    def apply_precond(self, r, z, prec=HD_F64, nrhs=1):
        nu, nq = self.sizes()
        self._dev(r, nrhs * (nu + nq), prec, 'r')
        self._dev(z, nrhs * (nu + nq), prec, 'z')
        return self._check(self.lib.hd_apply_precond(self.h, prec, nrhs, _ptr(r), _ptr(z)))

    def minres_solve(self, b, x, params=None, nrhs=1):
        """Solve A x_r = b_r for nrhs right-hand sides stored one after the
        other; returns one info dict (nrhs = 1) or a list of them."""
        nu, nq = self.sizes()
        self._dev(b, nrhs * (nu + nq), HD_F64, 'b')
        self._dev(x, nrhs * (nu + nq), HD_F64, 'x')
        info = (SolveInfo * nrhs)()
        pp = ctypes.byref(params) if params is not None else None
        rc = self.lib.hd_minres_solve(self.h, pp, nrhs, _ptr(b), _ptr(x), info)
        self._check(rc, allow=(HD_NOT_CONVERGED,))
        out = [i.as_dict() for i in info]
        return out[0] if nrhs == 1 else out

    def apply_tri_precond(self, r, z):
        """z = P^{-1} r, the block-triangular preconditioner (FP64)."""
        nu, nq = self.sizes()
        self._dev(r, nu + nq, HD_F64, 'r')
        self._dev(z, nu + nq, HD_F64, 'z')
        return self._check(self.lib.hd_apply_tri_precond(self.h, _ptr(r), _ptr(z)))

    def apply_tri_precond_noalloc(self, r, z):
        """hd_apply_tri_precond_noalloc: the same z = P^{-1} r with the V-cycle
        output in the library's fixed device array (no allocation)."""
        nu, nq = self.sizes()
        self._dev(r, nu + nq, HD_F64, 'r')
        self._dev(z, nu + nq, HD_F64, 'z')
        return self._check(self.lib.hd_apply_tri_precond_noalloc(self.h, _ptr(r), _ptr(z)))

    def gmres_solve(self, b, x, tol=1e-8, max_it=2000, restart=30):
        """GMRES(restart) with the block-triangular preconditioner; x is the
        initial guess on entry.  Returns the info dict."""
        nu, nq = self.sizes()
        self._dev(b, nu + nq, HD_F64, 'b')
        self._dev(x, nu + nq, HD_F64, 'x')
        info = SolveInfo()
        rc = self.lib.hd_gmres_solve(self.h, float(tol), int(max_it), int(restart), _ptr(b), _ptr(x),
                                     ctypes.byref(info))
        self._check(rc, allow=(HD_NOT_CONVERGED,))
        return info.as_dict()

    # ---- inspection ---------------------------------------------------------
    def get_diagonals(self):
        torch = self.torch
        nu, nq = self.sizes()
        m = torch.empty(nu, dtype=torch.float64, device=self.device)
        w = torch.empty(nq, dtype=torch.float64, device=self.device)
        self._check(self.lib.hd_get_diagonals(self.h, _ptr(m), _ptr(w)))
        return m, w

    def get_schur(self):
        nnz = ctypes.c_int64()
        self._check(self.lib.hd_get_schur(self.h, ctypes.byref(nnz), None, None, None))
        _, nq = self.sizes()
        rp = np.empty(nq + 1, np.int32)
        ci = np.empty(nnz.value, np.int32)
        v = np.empty(nnz.value, np.float64)
        self._check(self.lib.hd_get_schur(self.h, ctypes.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v)))
        return rp, ci, v

    def amg_nlevels(self):
        n = ctypes.c_int()
        self._check(self.lib.hd_get_amg_nlevels(self.h, ctypes.byref(n)))
        return n.value

    def get_amg_level(self, level):
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.hd_get_amg_level(self.h, level, ctypes.byref(n), ctypes.byref(nnz), None, None, None))
        rp = np.empty(n.value + 1, np.int32)
        ci = np.empty(nnz.value, np.int32)
        v = np.empty(nnz.value, np.float64)
        self._check(self.lib.hd_get_amg_level(self.h, level, ctypes.byref(n), ctypes.byref(nnz), _ptr(rp), _ptr(ci),
                                              _ptr(v)))
        return rp, ci, v

    def get_amg_prolongator(self, level):
        nr, nc, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.hd_get_amg_prolongator(self.h, level, ctypes.byref(nr), ctypes.byref(nc),
                                                    ctypes.byref(nnz), None, None, None))
        rp = np.empty(nr.value + 1, np.int32)
        ci = np.empty(nnz.value, np.int32)
        v = np.empty(nnz.value, np.float64)
        self._check(self.lib.hd_get_amg_prolongator(self.h, level, ctypes.byref(nr), ctypes.byref(nc),
                                                    ctypes.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v)))
        return (nr.value, nc.value), rp, ci, v

    # ---- radiation diffusion (Section 4.3) -----------------------------------
    def apply_divergence(self, F, q):
        """q = D F (n_u -> n_q, FP64 device tensors)."""
        nu, nq = self.sizes()
        self._dev(F, nu, HD_F64, 'F')
        self._dev(q, nq, HD_F64, 'q')
        return self._check(self.lib.hd_apply_divergence(self.h, _ptr(F), _ptr(q)))

    def subcell_volumes(self):
        """|K_j| of every L2 dof (FP64 device tensor of n_q)."""
        _, nq = self.sizes()
        out = self.torch.empty(nq, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.hd_subcell_volumes(self.h, _ptr(out)))
        return out

    def rd_setup(self, params, precond=None):
        pp = ctypes.byref(precond) if precond is not None else None
        return self._check(self.lib.hd_rd_setup(self.h, ctypes.byref(params), pp), allow=(HD_FALLBACK_USED,))

    def rd_step(self, e, E, F):
        """One SDIRK3 step in place; returns the step's RdInfo as a dict
        (HD_NOT_CONVERGED is reported in it, not raised)."""
        nu, nq = self.sizes()
        self._dev(e, nq, HD_F64, 'e')
        self._dev(E, nq, HD_F64, 'E')
        self._dev(F, nu, HD_F64, 'F')
        info = RdInfo()
        self._check(self.lib.hd_rd_step(self.h, _ptr(e), _ptr(E), _ptr(F), ctypes.byref(info)),
                    allow=(HD_NOT_CONVERGED,))
        return info.as_dict()

    def apply_timing(self, reset=False):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.hd_apply_timing(self.h, 1 if reset else 0, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


# ---- host-only helpers (no device needed) -----------------------------------

def host_tables(p):
    lib = load()
    gll = np.empty(p + 1)
    x = np.empty(p + 1)
    w = np.empty(p + 1)
    rc = lib.hd_host_tables(p, _ptr(gll), _ptr(x), _ptr(w))
    if rc:
        raise HdError(rc, 'hd_host_tables')
    return gll, x, w


def host_unstructured_map(nv, elements, p):
    """The library's RT numbering of an unstructured mesh, computed on the
    host: (n_u, element-to-dof map [ne][3 p^2 (p+1)], ~g for sign -1)."""
    lib = load()
    el = np.ascontiguousarray(elements, dtype=np.int64).reshape(-1, 8)
    nu = ctypes.c_int64()
    out = np.empty((el.shape[0], 3 * p * p * (p + 1)), dtype=np.int32)
    rc = lib.hd_host_unstructured_map(nv, el.shape[0], _ptr(el), p, ctypes.byref(nu), _ptr(out))
    if rc:
        raise HdError(rc, 'hd_host_unstructured_map')
    return nu.value, out


def host_amg(rowptr, col, val, singular=False, params=None):
    """Build the library's AMG hierarchy on the host from a CSR matrix.
    Returns (levels, prolongators) as lists of (shape, rowptr, col, val)."""
    lib = load()
    rp = np.ascontiguousarray(rowptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    n = len(rp) - 1
    h = ctypes.c_void_p()
    pp = ctypes.byref(params) if params is not None else None
    rc = lib.hd_host_amg_build(n, _ptr(rp), _ptr(ci), _ptr(v), pp, 1 if singular else 0, ctypes.byref(h))
    if rc:
        raise HdError(rc, 'hd_host_amg_build')
    try:
        levels, prolongs = [], []
        for l in range(lib.hd_host_amg_nlevels(h)):
            nn, nnz = ctypes.c_int64(), ctypes.c_int64()
            lib.hd_host_amg_level(h, l, ctypes.byref(nn), ctypes.byref(nnz), None, None, None)
            a = np.empty(nn.value + 1, np.int32)
            b = np.empty(nnz.value, np.int32)
            c = np.empty(nnz.value, np.float64)
            lib.hd_host_amg_level(h, l, ctypes.byref(nn), ctypes.byref(nnz), _ptr(a), _ptr(b), _ptr(c))
            levels.append(((nn.value, nn.value), a, b, c))
        for l in range(len(levels) - 1):
            nr, nc, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            lib.hd_host_amg_prolongator(h, l, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nnz), None, None, None)
            a = np.empty(nr.value + 1, np.int32)
            b = np.empty(nnz.value, np.int32)
            c = np.empty(nnz.value, np.float64)
            lib.hd_host_amg_prolongator(h, l, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nnz), _ptr(a), _ptr(b),
                                        _ptr(c))
            prolongs.append(((nr.value, nc.value), a, b, c))
        return levels, prolongs
    finally:
        lib.hd_host_amg_free(h)
