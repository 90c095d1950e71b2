"""Python binding of the C ABI in ``include/pf.h`` (argument marshalling only).

Every numerical step runs in ``libpf.so``'s HIP kernels; this module loads the
library, mirrors its structs with ctypes and uses PyTorch only to allocate the
device workspace and to name the stream.  There is no fallback: if the library
is missing, importing the binding's functions raises.  PF_LIBRARY, if set,
names another build of the same library to load (an instrumented one, say).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PF_LIBRARY") or os.path.join(HERE, "libpf.so")

PF_OK, PF_ERR_INVALID_ARG, PF_ERR_HIP, PF_ERR_OOM, PF_ERR_CG_NOT_CONVERGED = 0, 1, 2, 3, 4
PF_ERR_NONFINITE, PF_ERR_LEDGER, PF_ERR_BAD_STATE, PF_ERR_UNSUPPORTED = 5, 6, 7, 8
PF_FP64, PF_MIXED = 0, 1
PF_WARM_ZERO, PF_WARM_PREV, PF_WARM_LEARNED = 0, 1, 2
WARM = {"zero": PF_WARM_ZERO, "prev": PF_WARM_PREV, "learned": PF_WARM_LEARNED}
PF_NN_OP_FORWARD, PF_NN_OP_BACKWARD_DATA, PF_NN_OP_BACKWARD_WEIGHT = 0, 1, 2
PF_NN_BUF_INPUT, PF_NN_BUF_OUTPUT, PF_NN_BUF_TARGET, PF_NN_BUF_LOSS_GRAD = 0, 1, 2, 3
FIELDS = {"phi_f": 0, "phi_w": 1, "xO": 2, "xH": 3, "xW": 4, "ux": 5, "uy": 6, "uz": 7, "epsp": 8, "epsP": 9}


class pf_config(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("h", C.c_double), ("dt", C.c_double),
                ("precision", C.c_int), ("mechanics", C.c_int), ("plasticity", C.c_int),
                ("dirichlet", C.c_int), ("chem_phase", C.c_int),
                ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int), ("warm", C.c_int),
                ("ledger_tol", C.c_double), ("species_implicit", C.c_int), ("species_max_iter", C.c_int),
                ("species_rtol", C.c_double), ("cg_precond", C.c_int)]


class pf_params(C.Structure):
    _fields_ = [("R", C.c_double), ("theta", C.c_double), ("Vmol", C.c_double),
                ("w", C.c_double * 3), ("eps", C.c_double * 3), ("L", C.c_double * 3),
                ("kappaO", C.c_double), ("K", C.c_double * 3), ("G", C.c_double * 3),
                ("sigY", C.c_double), ("Hhard", C.c_double),
                ("DO", C.c_double * 3), ("DH", C.c_double * 3), ("DW", C.c_double * 3),
                ("kfor", C.c_double), ("Omega_f", C.c_double), ("xH_bc", C.c_double), ("xW_bc", C.c_double),
                ("m_form", C.c_int), ("pad_", C.c_int)]


class pf_extent(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int)]


class pf_batch_tiles(C.Structure):
    _fields_ = [("apply_rows", C.c_int), ("update_chunk", C.c_int), ("blocks_per_cu", C.c_int), ("pad_", C.c_int),
                ("spin_limit", C.c_longlong)]


class pf_nn_config(C.Structure):
    _fields_ = [("max_voxels", C.c_longlong), ("training", C.c_int), ("pad_", C.c_int), ("seed", C.c_ulonglong)]


class pf_step_stats(C.Structure):
    _fields_ = [("cg_iters", C.c_int), ("warm_used", C.c_int), ("cg_rel_resid", C.c_double),
                ("O_tot", C.c_double), ("O_out", C.c_double), ("O_drift", C.c_double),
                ("H_tot", C.c_double), ("H_out", C.c_double), ("H_drift", C.c_double),
                ("red_degree", C.c_double), ("max_vm", C.c_double), ("max_epsP", C.c_double),
                ("step", C.c_longlong), ("nonfinite", C.c_int), ("pad_", C.c_int),
                ("cg_iters_total", C.c_longlong), ("r0_learned", C.c_double), ("r0_prev", C.c_double),
                ("species_iters", C.c_int), ("pad2_", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("pad")}


class pf_fs_config(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double),
                ("plasticity", C.c_int), ("newton_max_iter", C.c_int), ("newton_rtol", C.c_double),
                ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int), ("pad_", C.c_int)]


class pf_fs_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int), ("cg_iters", C.c_int), ("rel_resid", C.c_double), ("max_vm", C.c_double),
                ("max_epsP", C.c_double), ("yielded", C.c_int), ("line_search_cuts", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


FS_FIELDS = {"phi_f": 0, "phi_w": 1, "u": 2, "Fp": 3, "epsP": 4, "drive": 5}
FS_KERNEL_KINDS = ("tangent", "gather", "residual", "vector", "return", "post")


EXPORTS = ("pf_workspace_bytes", "pf_init", "pf_step", "pf_mech_solve", "pf_cg_chunk", "pf_fields", "pf_ledger_reset",
           "pf_timing", "pf_timing_every", "pf_timing_get", "pf_last_error", "pf_destroy",
           "pf_batch_workspace_bytes", "pf_batch_init", "pf_batch_set_tiles", "pf_batch_get_tiles",
           "pf_batch_fields", "pf_batch_step", "pf_batch_last_error", "pf_batch_destroy",
           "pf_nn_param_count", "pf_nn_workspace_bytes", "pf_nn_init", "pf_nn_destroy", "pf_nn_last_error", "pf_nn_weights", "pf_nn_copy",
           "pf_nn_forward", "pf_nn_loss", "pf_nn_backward", "pf_nn_adam", "pf_nn_layer", "pf_nn_increment_scale",
           "pf_nn_pack", "pf_nn_attach", "pf_increment_scale_static",
           "pf_fs_workspace_bytes", "pf_fs_init", "pf_fs_fields", "pf_fs_solve", "pf_fs_timing", "pf_fs_timing_get", "pf_fs_attach",
           "pf_fs_last_error", "pf_fs_destroy")
PRECOND = {"jacobi": 0, "mg": 1}
KERNEL_KINDS = ("apply", "update", "solve_setup", "step", "mu", "other", "nn", "species", "precond", "smooth")

_lib = None


def lib():
    """Load ``libpf.so`` (built in-tree by ``build.py``); raises if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2111_11538_amd/build.py (or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.pf_workspace_bytes.argtypes = [C.POINTER(pf_config)]
        L.pf_workspace_bytes.restype = C.c_size_t
        L.pf_init.argtypes = [C.POINTER(pf_config), C.POINTER(pf_params), C.c_void_p, C.c_size_t, C.c_void_p,
                              C.POINTER(C.c_void_p)]
        L.pf_init.restype = C.c_int
        L.pf_step.argtypes = [C.c_void_p, C.c_int, C.POINTER(pf_step_stats)]
        L.pf_step.restype = C.c_int
        L.pf_mech_solve.argtypes = [C.c_void_p, C.c_int, C.POINTER(pf_step_stats)]
        L.pf_mech_solve.restype = C.c_int
        L.pf_fields.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_int]
        L.pf_fields.restype = C.c_int
        L.pf_ledger_reset.argtypes = [C.c_void_p]
        L.pf_ledger_reset.restype = C.c_int
        L.pf_timing.argtypes = [C.c_void_p, C.c_int]
        L.pf_timing.restype = C.c_int
        L.pf_timing_every.argtypes = [C.c_void_p, C.c_int]
        L.pf_timing_every.restype = C.c_int
        L.pf_cg_chunk.argtypes = [C.c_void_p, C.c_int]
        L.pf_cg_chunk.restype = C.c_int
        L.pf_timing_get.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
        L.pf_timing_get.restype = C.c_int
        L.pf_batch_workspace_bytes.argtypes = [C.POINTER(pf_config), C.POINTER(pf_extent), C.c_int]
        L.pf_batch_workspace_bytes.restype = C.c_size_t
        L.pf_batch_init.argtypes = [C.POINTER(pf_config), C.POINTER(pf_params), C.POINTER(pf_extent), C.c_int,
                                    C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.pf_batch_init.restype = C.c_int
        L.pf_batch_set_tiles.argtypes = [C.c_void_p, C.POINTER(pf_batch_tiles)]
        L.pf_batch_set_tiles.restype = C.c_int
        L.pf_batch_get_tiles.argtypes = [C.c_void_p, C.POINTER(pf_batch_tiles)]
        L.pf_batch_get_tiles.restype = C.c_int
        L.pf_batch_fields.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_int]
        L.pf_batch_fields.restype = C.c_int
        L.pf_batch_step.argtypes = [C.c_void_p, C.c_int, C.POINTER(pf_step_stats)]
        L.pf_batch_step.restype = C.c_int
        L.pf_batch_last_error.argtypes = [C.c_void_p]
        L.pf_batch_last_error.restype = C.c_char_p
        L.pf_batch_destroy.argtypes = [C.c_void_p]
        L.pf_batch_destroy.restype = None
        L.pf_last_error.argtypes = [C.c_void_p]
        L.pf_last_error.restype = C.c_char_p
        L.pf_destroy.argtypes = [C.c_void_p]
        L.pf_destroy.restype = None
        P3 = C.POINTER(C.c_void_p)
        L.pf_nn_param_count.argtypes = []
        L.pf_nn_param_count.restype = C.c_size_t
        L.pf_nn_workspace_bytes.argtypes = [C.POINTER(pf_nn_config)]
        L.pf_nn_workspace_bytes.restype = C.c_size_t
        L.pf_nn_init.argtypes = [C.POINTER(pf_nn_config), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.pf_nn_destroy.argtypes = [C.c_void_p]
        L.pf_nn_destroy.restype = None
        L.pf_nn_last_error.argtypes = [C.c_void_p]
        L.pf_nn_last_error.restype = C.c_char_p
        L.pf_nn_weights.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_float), C.c_size_t]
        L.pf_nn_copy.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_size_t]
        L.pf_nn_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_int] * 4
        L.pf_nn_loss.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
        L.pf_nn_backward.argtypes = [C.c_void_p, C.c_void_p]
        L.pf_nn_adam.argtypes = [C.c_void_p] + [C.c_double] * 4
        L.pf_nn_layer.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_int] * 4
        L.pf_nn_increment_scale.argtypes = [C.c_void_p, P3, P3] + [C.c_int] * 3 + [C.POINTER(C.c_double)]
        L.pf_nn_pack.argtypes = [C.c_void_p] + [C.c_void_p] * 3 + [P3] * 3 + [C.c_int] * 10 + [C.c_double] * 2
        L.pf_nn_attach.argtypes = [C.c_void_p, C.c_void_p]
        L.pf_increment_scale_static.argtypes = [P3, P3] + [C.c_int] * 3 + [C.c_void_p, C.c_void_p]
        L.pf_increment_scale_static.restype = C.c_int
        for f in ("pf_nn_init", "pf_nn_weights", "pf_nn_copy", "pf_nn_forward", "pf_nn_loss", "pf_nn_backward",
                  "pf_nn_adam", "pf_nn_layer", "pf_nn_increment_scale", "pf_nn_pack", "pf_nn_attach"):
            getattr(L, f).restype = C.c_int
        L.pf_fs_workspace_bytes.argtypes = [C.POINTER(pf_fs_config)]
        L.pf_fs_workspace_bytes.restype = C.c_size_t
        L.pf_fs_init.argtypes = [C.POINTER(pf_fs_config), C.POINTER(pf_params), C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.POINTER(C.c_void_p)]
        L.pf_fs_init.restype = C.c_int
        L.pf_fs_fields.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_int]
        L.pf_fs_fields.restype = C.c_int
        L.pf_fs_solve.argtypes = [C.c_void_p, C.POINTER(pf_fs_stats)]
        L.pf_fs_solve.restype = C.c_int
        L.pf_fs_timing.argtypes = [C.c_void_p, C.c_int]
        L.pf_fs_timing.restype = C.c_int
        L.pf_fs_timing_get.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
        L.pf_fs_timing_get.restype = C.c_int
        L.pf_fs_attach.argtypes = [C.c_void_p, C.c_void_p]
        L.pf_fs_attach.restype = C.c_int
        L.pf_fs_last_error.argtypes = [C.c_void_p]
        L.pf_fs_last_error.restype = C.c_char_p
        L.pf_fs_destroy.argtypes = [C.c_void_p]
        L.pf_fs_destroy.restype = None
        _lib = L
    return _lib


class PFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pf status {status}: {msg}")
        self.status = status


def make_params(p) -> pf_params:
    o = pf_params()
    for name in ("R", "theta", "Vmol", "kappaO", "sigY", "Hhard", "kfor", "Omega_f", "xH_bc", "xW_bc"):
        setattr(o, name, float(getattr(p, name)))
    for name in ("w", "eps", "L", "K", "G", "DO", "DH", "DW"):
        arr = getattr(o, name)
        for a, v in enumerate(getattr(p, name)):
            arr[a] = float(v)
    o.m_form = int(p.m_form)
    return o


def make_config(dim, shape, h, dt, precision="fp64", mechanics=True, plasticity=False, dirichlet=True,
                chem_phase=True, cg_rtol=1e-10, cg_max_iter=200000, warm="prev", ledger_tol=0.0,
                species_implicit=False, species_rtol=None, species_max_iter=100000,
                cg_precond="jacobi") -> pf_config:
    c = pf_config()
    c.dim = dim
    if dim == 2:
        c.ny, c.nx = shape
        c.nz = 1
    else:
        c.nz, c.ny, c.nx = shape
    c.h, c.dt = h, dt
    c.precision = {"fp64": PF_FP64, "mixed": PF_MIXED}[precision]
    c.mechanics, c.plasticity, c.dirichlet, c.chem_phase = int(mechanics), int(plasticity), int(dirichlet), int(chem_phase)
    c.cg_rtol, c.cg_max_iter = cg_rtol, cg_max_iter
    c.warm = WARM[warm]
    c.ledger_tol = ledger_tol
    c.species_implicit = int(species_implicit)        # 0, 1 (or True) or 2
    c.species_max_iter = int(species_max_iter)
    c.species_rtol = species_rtol if species_rtol is not None else (1e-12 if precision == "fp64" else 1e-6)
    c.cg_precond = PRECOND[cg_precond]
    return c


def field_shape(name, dim, shape):
    if dim == 2:
        ny, nx = shape
        nz = None
    else:
        nz, ny, nx = shape
    nc = 4 if dim == 2 else 6
    cell = tuple(shape)
    if name == "ux":
        return (ny, nx + 1) if dim == 2 else (nz, ny, nx + 1)
    if name == "uy":
        return (ny + 1, nx) if dim == 2 else (nz, ny + 1, nx)
    if name == "uz":
        return (nz + 1, ny, nx)
    if name == "epsp":
        return (nc,) + cell
    return cell


class Context:
    """One simulation on one GPU: a thin owner of a ``pf_ctx`` and of the
    torch-allocated device workspace it lives in."""

    def __init__(self, dim, shape, h, dt, params, device=0, stream=None, **cfg_kw):
        import torch
        self.dim, self.shape = dim, tuple(shape)
        self.cfg = make_config(dim, shape, h, dt, **cfg_kw)
        self.params = make_params(params)
        L = lib()
        nbytes = L.pf_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise PFError(PF_ERR_INVALID_ARG, "invalid configuration")
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        rc = L.pf_init(C.byref(self.cfg), C.byref(self.params), C.c_void_p(self.workspace.data_ptr()), nbytes,
                       C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx))
        if rc != PF_OK:
            raise PFError(rc, L.pf_last_error(None).decode())

    # -- helpers -------------------------------------------------------------
    def _check(self, rc):
        if rc != PF_OK:
            raise PFError(rc, lib().pf_last_error(self.ctx).decode())

    def set(self, name, value):
        """Set one field from a numpy array or a torch tensor (any device)."""
        import torch
        shp = field_shape(name, self.dim, self.shape)
        if isinstance(value, torch.Tensor):
            t = value.detach().to(dtype=torch.float64)
            if t.device.type == "cuda":
                t = t.contiguous()
                assert tuple(t.shape) == shp, (name, t.shape, shp)
                self._check(lib().pf_fields(self.ctx, FIELDS[name], 1, C.c_void_p(t.data_ptr()), t.numel() * 8, 1))
                return
            value = t.numpy()
        a = np.ascontiguousarray(value, dtype=np.float64)
        assert a.shape == shp, (name, a.shape, shp)
        self._check(lib().pf_fields(self.ctx, FIELDS[name], 1, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))

    def get(self, name):
        a = np.zeros(field_shape(name, self.dim, self.shape), dtype=np.float64)
        self._check(lib().pf_fields(self.ctx, FIELDS[name], 0, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))
        return a

    def get_device(self, name):
        """Field as an FP64 torch tensor on the context's device."""
        import torch
        t = torch.empty(field_shape(name, self.dim, self.shape), dtype=torch.float64, device=self.device)
        self._check(lib().pf_fields(self.ctx, FIELDS[name], 0, C.c_void_p(t.data_ptr()), t.numel() * 8, 1))
        return t

    def set_fields(self, fields: dict):
        for k, v in fields.items():
            if k in FIELDS:
                self.set(k, v)

    def fields(self, names=None):
        names = names or [n for n in FIELDS if not (n == "uz" and self.dim == 2)]
        return {n: self.get(n) for n in names}

    def step(self, n=1):
        st = pf_step_stats()
        self._check(lib().pf_step(self.ctx, int(n), C.byref(st)))
        return st.as_dict()

    def attach_fs(self, fs):
        """Drive this context's steps with the finite-strain mechanics of a
        ``FiniteStrain`` on the same grid and stream (None detaches); the
        context must have been created with mechanics=False."""
        self._fs = fs
        self._check(lib().pf_fs_attach(self.ctx, fs.ctx if fs is not None else None))

    def mech_solve(self, warm="zero"):
        st = pf_step_stats()
        self._check(lib().pf_mech_solve(self.ctx, WARM[warm], C.byref(st)))
        return st.as_dict()

    def cg_chunk(self, n=0):
        """CG launches between convergence checks (0: adaptive)."""
        self._check(lib().pf_cg_chunk(self.ctx, int(n)))

    def timing(self, enable=True, kinds=None, every=1):
        """Start (or with enable False stop) event timing of the named kernel
        kinds (all of them by default); the CG kernels only on every
        `every`-th iteration."""
        self._check(lib().pf_timing_every(self.ctx, int(every)))
        mask = 0
        if enable:
            names = KERNEL_KINDS if kinds is None else kinds
            for n in names:
                mask |= 1 << KERNEL_KINDS.index(n)
        self._check(lib().pf_timing(self.ctx, mask))

    def timing_report(self):
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            ms, n = C.c_double(), C.c_longlong()
            self._check(lib().pf_timing_get(self.ctx, k, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def ledger_reset(self):
        self._check(lib().pf_ledger_reset(self.ctx))

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().pf_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many uneven 2D instances advanced together (one persistent graph launch
    per step).  `shapes` is a list of (ny, nx)."""

    def __init__(self, shapes, h, dt, params, device=0, stream=None, **cfg_kw):
        import torch
        self.shapes = [tuple(s) for s in shapes]
        self.count = len(self.shapes)
        self.cfg = make_config(2, self.shapes[0], h, dt, **cfg_kw)
        self.params = make_params(params)
        self.ext = (pf_extent * self.count)()
        for k, (ny, nx) in enumerate(self.shapes):
            self.ext[k].nx, self.ext[k].ny, self.ext[k].nz = nx, ny, 1
        L = lib()
        nbytes = L.pf_batch_workspace_bytes(C.byref(self.cfg), self.ext, self.count)
        if nbytes == 0:
            raise PFError(PF_ERR_INVALID_ARG, "invalid batch configuration")
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        rc = L.pf_batch_init(C.byref(self.cfg), C.byref(self.params), self.ext, self.count,
                             C.c_void_p(self.workspace.data_ptr()), nbytes, C.c_void_p(self.stream.cuda_stream),
                             C.byref(self.ctx))
        if rc != PF_OK:
            raise PFError(rc, L.pf_batch_last_error(None).decode())

    def _check(self, rc):
        if rc != PF_OK:
            raise PFError(rc, lib().pf_batch_last_error(self.ctx).decode())

    def set(self, k, name, value):
        a = np.ascontiguousarray(value, dtype=np.float64)
        assert a.shape == field_shape(name, 2, self.shapes[k]), (name, a.shape)
        self._check(lib().pf_batch_fields(self.ctx, k, FIELDS[name], 1, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))

    def get(self, k, name):
        a = np.zeros(field_shape(name, 2, self.shapes[k]), dtype=np.float64)
        self._check(lib().pf_batch_fields(self.ctx, k, FIELDS[name], 0, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))
        return a

    def set_fields(self, k, fields):
        for name, v in fields.items():
            if name in FIELDS and name != "uz":
                self.set(k, name, v)

    def fields(self, k):
        return {n: self.get(k, n) for n in FIELDS if n != "uz"}

    def step(self, n=1):
        st = (pf_step_stats * self.count)()
        self._check(lib().pf_batch_step(self.ctx, int(n), st))
        return [s.as_dict() for s in st]

    def tiles(self):
        t = pf_batch_tiles()
        self._check(lib().pf_batch_get_tiles(self.ctx, C.byref(t)))
        return {"apply_rows": t.apply_rows, "update_chunk": t.update_chunk, "blocks_per_cu": t.blocks_per_cu,
                "spin_limit": t.spin_limit}

    def set_tiles(self, apply_rows=None, update_chunk=None, blocks_per_cu=None, spin_limit=None):
        cur = self.tiles()
        t = pf_batch_tiles()
        t.apply_rows = apply_rows if apply_rows is not None else cur["apply_rows"]
        t.update_chunk = update_chunk if update_chunk is not None else cur["update_chunk"]
        t.blocks_per_cu = blocks_per_cu if blocks_per_cu is not None else cur["blocks_per_cu"]
        t.spin_limit = spin_limit if spin_limit is not None else cur["spin_limit"]
        self._check(lib().pf_batch_set_tiles(self.ctx, C.byref(t)))

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().pf_batch_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr3(arrs):
    """Three device tensors (or None) as a C array of pointers."""
    if arrs is None:
        return None
    a = (C.c_void_p * 3)(*[C.c_void_p(t.data_ptr()) for t in arrs])
    return C.cast(a, C.POINTER(C.c_void_p))


def increment_scale_static(u1, u0, s_dev, stream=None):
    """``pf_increment_scale_static``: RMS of u1 - u0 over the low faces into the
    one-element FP64 device tensor ``s_dev``, without any allocation.  u1, u0:
    three FP64 device tensors each (u0 may be None)."""
    import torch
    nz, ny, nx = u1[2].shape[0] - 1, u1[2].shape[1], u1[2].shape[2]
    st = stream if stream is not None else torch.cuda.current_stream(s_dev.device)
    rc = lib().pf_increment_scale_static(_ptr3(u1), _ptr3(u0), nx, ny, nz, C.c_void_p(s_dev.data_ptr()),
                                         C.c_void_p(st.cuda_stream))
    if rc != PF_OK:
        raise PFError(rc, lib().pf_nn_last_error(None).decode())


class Net:
    """The learned warm start's network (``pf_nn``): parameters, training
    buffers and the MFMA convolution kernels live in the library."""

    N_PARAMS = None

    def __init__(self, max_voxels, training=False, seed=2111_11538, device=0, stream=None):
        import torch
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg = pf_nn_config()
        cfg.max_voxels, cfg.training, cfg.seed = int(max_voxels), int(training), int(seed)
        self.nn = C.c_void_p()
        L = lib()
        nbytes = L.pf_nn_workspace_bytes(C.byref(cfg))
        if nbytes == 0:
            raise PFError(PF_ERR_INVALID_ARG, "invalid network configuration")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        rc = L.pf_nn_init(C.byref(cfg), C.c_void_p(self.workspace.data_ptr()), nbytes,
                          C.c_void_p(self.stream.cuda_stream), C.byref(self.nn))
        if rc != PF_OK:
            raise PFError(rc, L.pf_nn_last_error(None).decode())
        self.n_params = L.pf_nn_param_count()

    def _check(self, rc):
        if rc != PF_OK:
            raise PFError(rc, lib().pf_nn_last_error(self.nn).decode())

    @staticmethod
    def _p(t):
        return None if t is None else C.c_void_p(t.data_ptr())

    def params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(lib().pf_nn_weights(self.nn, 0, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        self._check(lib().pf_nn_weights(self.nn, 1, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))

    def grads(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(lib().pf_nn_weights(self.nn, 2, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def copy(self, which, t, to_buffer=False):
        """Copy an internal buffer (``PF_NN_BUF_*``) into the device tensor t,
        or t into the buffer; the first t.nbytes bytes."""
        self._check(lib().pf_nn_copy(self.nn, which, int(to_buffer), C.c_void_p(t.data_ptr()), t.numel() * t.element_size()))

    def forward(self, x=None, y=None, n=1, D=1, H=1, W=1):
        self._check(lib().pf_nn_forward(self.nn, self._p(x), self._p(y), n, D, H, W))

    def loss(self, target=None):
        out = C.c_double()
        self._check(lib().pf_nn_loss(self.nn, self._p(target), C.byref(out)))
        return out.value

    def backward(self, dy=None):
        self._check(lib().pf_nn_backward(self.nn, self._p(dy)))

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self._check(lib().pf_nn_adam(self.nn, lr, b1, b2, eps))

    def layer(self, op, layer, x, aux, out, n, D, H, W):
        self._check(lib().pf_nn_layer(self.nn, op, layer, self._p(x), self._p(aux), self._p(out), n, D, H, W))

    def increment_scale(self, u1, u0=None):
        nz, ny, nx = u1[2].shape[0] - 1, u1[2].shape[1], u1[2].shape[2]
        s = C.c_double()
        self._check(lib().pf_nn_increment_scale(self.nn, _ptr3(u1), _ptr3(u0), nx, ny, nz, C.byref(s)))
        return s.value

    def pack(self, phi_f, phi_w, phi_prev, u1, u0=None, u2=None, origin=(0, 0, 0), size=None, slot=0, Omega=0.4, h=1.0):
        nz, ny, nx = phi_f.shape
        cz, cy, cx = size if size is not None else (nz, ny, nx)
        z0, y0, x0 = origin
        self._check(lib().pf_nn_pack(self.nn, self._p(phi_f), self._p(phi_w), self._p(phi_prev), _ptr3(u1), _ptr3(u0),
                                     _ptr3(u2), nx, ny, nz, x0, y0, z0, cx, cy, cz, slot, float(Omega), float(h)))

    def attach(self, ctx):
        rc = lib().pf_nn_attach(ctx.ctx, self.nn)
        if rc != PF_OK:
            raise PFError(rc, lib().pf_last_error(ctx.ctx).decode())

    def close(self):
        if getattr(self, "nn", None) and self.nn.value:
            lib().pf_nn_destroy(self.nn)
            self.nn = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_fs_config(dim, shape, h, plasticity=False, newton_rtol=1e-10, newton_max_iter=50, cg_rtol=1e-3,
                   cg_max_iter=20000) -> pf_fs_config:
    c = pf_fs_config()
    c.dim = dim
    if dim == 2:
        c.ny, c.nx = shape
        c.nz = 1
    else:
        c.nz, c.ny, c.nx = shape
    c.h = h
    c.plasticity = int(plasticity)
    c.newton_rtol, c.newton_max_iter = newton_rtol, newton_max_iter
    c.cg_rtol, c.cg_max_iter = cg_rtol, cg_max_iter
    return c


class FiniteStrain:
    """Finite-strain mechanics on one GPU: owner of a ``pf_fs`` and of the
    torch-allocated device workspace it lives in.  Arrays use the exchange
    layouts of ``include/pf.h`` (cells ``shape``; nodal displacement
    ``(dim,) + nodes``; F_P ``shape + (2^dim, 3, 3)``; eps_P ``shape +
    (2^dim,)``; driving forces ``(2,) + shape``)."""

    def __init__(self, dim, shape, h, params, device=0, stream=None, **cfg_kw):
        import torch
        self.dim, self.shape = dim, tuple(shape)
        self.nodes = tuple(n + 1 for n in self.shape)
        self.cfg = make_fs_config(dim, shape, h, **cfg_kw)
        self.params = make_params(params)
        L = lib()
        nbytes = L.pf_fs_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise PFError(PF_ERR_INVALID_ARG, "invalid finite-strain configuration")
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        rc = L.pf_fs_init(C.byref(self.cfg), C.byref(self.params), C.c_void_p(self.workspace.data_ptr()), nbytes,
                          C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx))
        if rc != PF_OK:
            raise PFError(rc, L.pf_fs_last_error(None).decode())

    def _check(self, rc):
        if rc != PF_OK:
            raise PFError(rc, lib().pf_fs_last_error(self.ctx).decode())

    def field_shape(self, name):
        ngp = 1 << self.dim
        return {"phi_f": self.shape, "phi_w": self.shape, "u": (self.dim,) + self.nodes,
                "Fp": self.shape + (ngp, 3, 3), "epsP": self.shape + (ngp,), "drive": (2,) + self.shape}[name]

    def set(self, name, value):
        a = np.ascontiguousarray(value, dtype=np.float64)
        assert a.shape == self.field_shape(name), (name, a.shape, self.field_shape(name))
        self._check(lib().pf_fs_fields(self.ctx, FS_FIELDS[name], 1, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))

    def get(self, name):
        a = np.zeros(self.field_shape(name), dtype=np.float64)
        self._check(lib().pf_fs_fields(self.ctx, FS_FIELDS[name], 0, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))
        return a

    def solve(self):
        st = pf_fs_stats()
        self._check(lib().pf_fs_solve(self.ctx, C.byref(st)))
        return st.as_dict()

    def timing(self, on=True):
        self._check(lib().pf_fs_timing(self.ctx, int(on)))

    def timing_report(self):
        """{kind: (total ms, launches)} since timing was switched on."""
        out = {}
        for k, name in enumerate(FS_KERNEL_KINDS):
            ms, n = C.c_double(), C.c_longlong()
            self._check(lib().pf_fs_timing_get(self.ctx, k, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if self.ctx:
            lib().pf_fs_destroy(self.ctx)
            self.ctx = C.c_void_p()
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
