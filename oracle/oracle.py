"""ctypes front end of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PF_ORACLE_LIBRARY, if set, names another build of the oracle to load (the
# sanitizer test's instrumented one)
LIB_PATH = os.environ.get("PF_ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")
CFLAGS = ["-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall"]


def build(force: bool = True, out: str | None = None, extra: tuple = ("-O2",)) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over independent cell loops);
    `out` and `extra` give another output path and flags (sanitizers)."""
    path = out or LIB_PATH
    if force or not os.path.exists(path):
        cmd = ["gcc"] + list(extra) + CFLAGS + ["-o", path + ".tmp", os.path.join(HERE, "pf_oracle.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(path + ".tmp", path)
    return path


class OrParams(C.Structure):
    _fields_ = [("R", C.c_double), ("theta", C.c_double), ("Vmol", C.c_double),
                ("w", C.c_double * 3), ("eps", C.c_double * 3), ("L", C.c_double * 3),
                ("kappaO", C.c_double), ("K", C.c_double * 3), ("G", C.c_double * 3),
                ("sigY", C.c_double), ("Hhard", C.c_double),
                ("DO", C.c_double * 3), ("DH", C.c_double * 3), ("DW", C.c_double * 3),
                ("kfor", C.c_double), ("Omega_f", C.c_double), ("xH_bc", C.c_double), ("xW_bc", C.c_double),
                ("m_form", C.c_int), ("pad_", C.c_int)]


class OrConfig(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("h", C.c_double), ("dt", C.c_double),
                ("mechanics", C.c_int), ("plasticity", C.c_int), ("dirichlet", C.c_int), ("chem_phase", C.c_int),
                ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int), ("species_implicit", C.c_int),
                ("gext", C.POINTER(C.c_double))]


_P = C.POINTER(C.c_double)


class OrState(C.Structure):
    _fields_ = [(n, _P) for n in ("phi_f", "phi_w", "xO", "xH", "xW", "ux", "uy", "uz", "epsp", "epsP")]


class OrLedger(C.Structure):
    _fields_ = [("O_tot0", C.c_double), ("O_out", C.c_double), ("H_tot0", C.c_double), ("H_out", C.c_double),
                ("xO_sum0", C.c_double), ("step", C.c_long)]


class OrStats(C.Structure):
    _fields_ = [("cg_iters", C.c_int), ("pad_", C.c_int), ("cg_rel_resid", C.c_double),
                ("O_tot", C.c_double), ("O_out", C.c_double), ("O_drift", C.c_double),
                ("H_tot", C.c_double), ("H_out", C.c_double), ("H_drift", C.c_double),
                ("red_degree", C.c_double), ("max_vm", C.c_double), ("max_epsP", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.or_step.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.POINTER(OrState), C.POINTER(OrLedger),
                              C.POINTER(OrStats)]
        L.or_ledger_init.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.POINTER(OrState), C.POINTER(OrLedger)]
        L.or_mech_solve.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.POINTER(OrState), C.POINTER(OrStats)]
        L.or_moduli.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), _P, _P, _P, _P]
        L.or_apply.argtypes = [C.POINTER(OrConfig), _P, _P, _P, _P, _P, _P, _P, _P]
        L.or_rhs.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.POINTER(OrState), _P, _P, _P]
        L.or_diag.argtypes = [C.POINTER(OrConfig), _P, _P, _P, _P, _P]
        L.or_cell_strain.argtypes = [C.POINTER(OrConfig), _P, _P, _P, C.c_int, C.c_int, C.c_int, _P]
        L.or_local.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double, C.c_double, _P]
        L.or_return_map.argtypes = [C.POINTER(OrParams), C.c_double, _P, C.c_double, _P, _P]
        L.or_driving_force.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.c_double, C.c_double, C.c_double,
                                       _P, _P, _P]
        L.or_point_energy.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.c_double, C.c_double, C.c_double,
                                      _P, _P, _P]
        L.or_energy.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.POINTER(OrState)]
        L.or_energy.restype = C.c_double
        L.or_elastic_energy.argtypes = [C.POINTER(OrConfig), C.POINTER(OrParams), C.POINTER(OrState)]
        L.or_elastic_energy.restype = C.c_double
        L.or_common_tangent.argtypes = [_P, _P, _P]
        L.or_fe.argtypes = [C.c_int, C.c_double, _P]
        L.or_simplex_project.argtypes = [_P, _P]
        L.or_reaction_exact.argtypes = [C.POINTER(OrParams)] + [C.c_double] * 5
        L.or_reaction_exact.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_P)


def make_params(p) -> OrParams:
    """Convert an ``inputs.Params`` (or any object with the same fields)."""
    o = OrParams()
    for name in ("R", "theta", "Vmol", "kappaO", "sigY", "Hhard", "kfor", "Omega_f", "xH_bc", "xW_bc"):
        setattr(o, name, float(getattr(p, name)))
    for name in ("w", "eps", "L", "K", "G", "DO", "DH", "DW"):
        arr = getattr(o, name)
        for a, v in enumerate(getattr(p, name)):
            arr[a] = float(v)
    o.m_form = int(p.m_form)
    return o


def face_shapes(dim, shape):
    if dim == 2:
        ny, nx = shape
        return (ny, nx + 1), (ny + 1, nx), None
    nz, ny, nx = shape
    return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)


def ncomp(dim):
    return 4 if dim == 2 else 6


class OracleSim:
    """One simulation held in numpy FP64 arrays and advanced by the C oracle."""

    def __init__(self, dim, shape, h, dt, params, fields, mechanics=True, plasticity=False, dirichlet=True,
                 chem_phase=True, cg_rtol=1e-10, cg_max_iter=200000, u=None, epsp=None, epsP=None,
                 implicit=False, finite_strain=False, fs_rtol=1e-13):
        """finite_strain: the mechanics of each step is the finite-strain
        solve of `fs_fe_oracle` (Newton to fs_rtol, then the return map when
        `plasticity`), whose cell-mean driving forces enter the phase-field
        update; the small-strain mechanics is then off."""
        self.dim = dim
        self.shape = tuple(shape)
        cfg = OrConfig()
        cfg.dim = dim
        if dim == 2:
            cfg.ny, cfg.nx = shape
            cfg.nz = 1
        else:
            cfg.nz, cfg.ny, cfg.nx = shape
        cfg.h, cfg.dt = h, dt
        if finite_strain:
            mechanics = False
        cfg.mechanics, cfg.plasticity, cfg.dirichlet, cfg.chem_phase = int(mechanics), int(plasticity), int(dirichlet), int(chem_phase)
        cfg.cg_rtol, cfg.cg_max_iter = cg_rtol, cg_max_iter
        cfg.species_implicit = int(implicit)
        self.cfg = cfg
        self.params = params
        self.cp = make_params(params)
        self.f = {k: np.ascontiguousarray(fields[k], dtype=np.float64).copy() for k in ("phi_f", "phi_w", "xO", "xH", "xW")}
        fx, fy, fz = face_shapes(dim, shape)
        self.ux = np.zeros(fx)
        self.uy = np.zeros(fy)
        self.uz = np.zeros(fz) if fz else None
        if u is not None:
            self.ux[...] = u[0]
            self.uy[...] = u[1]
            if fz:
                self.uz[...] = u[2]
        self.epsp = np.zeros((ncomp(dim),) + self.shape) if epsp is None else np.array(epsp, dtype=np.float64)
        self.epsP = np.zeros(self.shape) if epsP is None else np.array(epsP, dtype=np.float64)
        self.fs = finite_strain
        if finite_strain:
            from oracle import fs_fe_oracle as FE
            self.FE = FE
            self.h = h
            self.fs_rtol = fs_rtol
            self.fs_plastic = plasticity
            self.fs_u = np.zeros((dim,) + tuple(n + 1 for n in self.shape))
            self.fs_Fp, self.fs_eP = FE.identity_plastic(self.shape, dim)
            self.gext = np.zeros(2 * int(np.prod(self.shape)))
            cfg.gext = self.gext.ctypes.data_as(C.POINTER(C.c_double))
        self._state()
        self.ledger = OrLedger()
        lib().or_ledger_init(C.byref(self.cfg), C.byref(self.cp), C.byref(self.st), C.byref(self.ledger))

    def _state(self):
        st = OrState()
        for k in ("phi_f", "phi_w", "xO", "xH", "xW"):
            setattr(st, k, _ptr(self.f[k]))
        st.ux, st.uy, st.uz = _ptr(self.ux), _ptr(self.uy), _ptr(self.uz)
        st.epsp, st.epsP = _ptr(self.epsp), _ptr(self.epsP)
        self.st = st

    def fs_solve(self):
        """The finite-strain mechanics of the current phases: equilibrium from
        the previous displacement, the return map, the driving forces (into the
        array the C step adds); returns (newton iterations, max vm, max eps_P)."""
        g = self.FE.FEGrid(self.dim, self.shape, self.h, self.params, self.f["phi_f"], self.f["phi_w"])
        u, it, rr = g.solve(self.fs_u, self.fs_Fp, rtol=self.fs_rtol)
        if rr > self.fs_rtol:
            raise RuntimeError(f"oracle finite-strain solve stopped at {rr:.3e}")
        self.fs_u = u
        if self.fs_plastic:
            self.fs_Fp, self.fs_eP, _ = g.return_map(u, self.fs_Fp, self.fs_eP)
        gf, gw = g.driving_forces(u, self.fs_Fp)
        n = gf.size
        self.gext[:n] = gf.ravel()
        self.gext[n:] = gw.ravel()
        return it, g.max_von_mises(u, self.fs_Fp), float(self.fs_eP.max())

    def fs_energy(self):
        """Elastic energy of the finite-strain state (displacement and F_P as they are)."""
        g = self.FE.FEGrid(self.dim, self.shape, self.h, self.params, self.f["phi_f"], self.f["phi_w"])
        return g.energy(self.fs_u, self.fs_Fp)

    def step(self, n=1):
        stats = OrStats()
        for _ in range(n):
            if self.fs:
                _, vm, ep = self.fs_solve()
            rc = lib().or_step(C.byref(self.cfg), C.byref(self.cp), C.byref(self.st), C.byref(self.ledger), C.byref(stats))
            if rc != 0:
                raise RuntimeError(f"oracle step failed with status {rc}")
        out = stats.as_dict()
        if self.fs:
            out["max_vm"], out["max_epsP"] = vm, ep
        return out

    def mech_solve(self):
        stats = OrStats()
        rc = lib().or_mech_solve(C.byref(self.cfg), C.byref(self.cp), C.byref(self.st), C.byref(stats))
        if rc != 0:
            raise RuntimeError(f"oracle mechanics solve failed with status {rc}")
        return stats.as_dict()

    def energy(self):
        return lib().or_energy(C.byref(self.cfg), C.byref(self.cp), C.byref(self.st))

    def elastic_energy(self):
        return lib().or_elastic_energy(C.byref(self.cfg), C.byref(self.cp), C.byref(self.st))

    def fields(self):
        out = dict(self.f)
        out["ux"], out["uy"] = self.ux, self.uy
        if self.uz is not None:
            out["uz"] = self.uz
        out["epsp"], out["epsP"] = self.epsp, self.epsP
        return out

    # pieces for the pins -------------------------------------------------
    def moduli(self):
        K = np.zeros(self.shape)
        G = np.zeros(self.shape)
        lib().or_moduli(C.byref(self.cfg), C.byref(self.cp), _ptr(self.f["phi_f"]), _ptr(self.f["phi_w"]), _ptr(K), _ptr(G))
        return K, G

    def apply(self, K, G, u):
        fx, fy, fz = face_shapes(self.dim, self.shape)
        q = [np.zeros(fx), np.zeros(fy), np.zeros(fz) if fz else None]
        ux, uy = np.ascontiguousarray(u[0]), np.ascontiguousarray(u[1])
        uz = np.ascontiguousarray(u[2]) if fz else None
        lib().or_apply(C.byref(self.cfg), _ptr(K), _ptr(G), _ptr(ux), _ptr(uy), _ptr(uz), _ptr(q[0]), _ptr(q[1]), _ptr(q[2]))
        return q if fz else q[:2]

    def rhs(self):
        fx, fy, fz = face_shapes(self.dim, self.shape)
        b = [np.zeros(fx), np.zeros(fy), np.zeros(fz) if fz else None]
        lib().or_rhs(C.byref(self.cfg), C.byref(self.cp), C.byref(self.st), _ptr(b[0]), _ptr(b[1]), _ptr(b[2]))
        return b if fz else b[:2]

    def diag(self, K, G):
        fx, fy, fz = face_shapes(self.dim, self.shape)
        d = [np.zeros(fx), np.zeros(fy), np.zeros(fz) if fz else None]
        lib().or_diag(C.byref(self.cfg), _ptr(K), _ptr(G), _ptr(d[0]), _ptr(d[1]), _ptr(d[2]))
        return d if fz else d[:2]

    def cell_strain(self, i, j, k=0):
        e = np.zeros(6)
        lib().or_cell_strain(C.byref(self.cfg), _ptr(self.ux), _ptr(self.uy), _ptr(self.uz), i, j, k, _ptr(e))
        return e


# ---------------------------------------------------------------------------
# point functions
# ---------------------------------------------------------------------------
def fe(phase: int, x: float):
    out = np.zeros(3)
    lib().or_fe(phase, x, _ptr(out))
    return out


def simplex_project(phi_f, phi_w):
    a, b = np.array([float(phi_f)]), np.array([float(phi_w)])
    lib().or_simplex_project(_ptr(a), _ptr(b))
    return a[0], b[0]


def reaction_exact(params, m, xO, xH, xW, t):
    return lib().or_reaction_exact(C.byref(make_params(params)), m, xO, xH, xW, t)


def common_tangent():
    a, b, r = C.c_double(), C.c_double(), C.c_double()
    lib().or_common_tangent(C.byref(a), C.byref(b), C.byref(r))
    return a.value, b.value, r.value


LOCAL_KEYS = ("phi_g", "h_f", "h_g", "h_w", "dT", "eT", "K", "G", "mu_loc", "psi_xx", "M_O", "D_O", "D_H", "D_W",
              "g_f_chem", "g_w_chem")


def local(params, phi_f, phi_w, xO):
    out = np.zeros(16)
    lib().or_local(C.byref(make_params(params)), phi_f, phi_w, xO, _ptr(out))
    return dict(zip(LOCAL_KEYS, out))


def return_map(params, G, e_tr, epsP_n):
    dl = np.zeros(1)
    nn = np.zeros(6)
    lib().or_return_map(C.byref(make_params(params)), G, _ptr(np.ascontiguousarray(e_tr, dtype=np.float64)), epsP_n,
                        _ptr(dl), _ptr(nn))
    return dl[0], nn


def _cfg(dim=3, mechanics=True, chem_phase=True):
    c = OrConfig()
    c.dim, c.nx, c.ny, c.nz = dim, 1, 1, 1
    c.h, c.dt = 1.0, 1.0
    c.mechanics, c.chem_phase = int(mechanics), int(chem_phase)
    return c


def driving_force(params, phi_f, phi_w, xO, ebar, epsp, mechanics=True, chem_phase=True):
    g = np.zeros(2)
    lib().or_driving_force(C.byref(_cfg(3, mechanics, chem_phase)), C.byref(make_params(params)), phi_f, phi_w, xO,
                           _ptr(np.ascontiguousarray(ebar, dtype=np.float64)),
                           _ptr(np.ascontiguousarray(epsp, dtype=np.float64)), _ptr(g))
    return g


def point_energy(params, phi_f, phi_w, xO, ebar, epsp, mechanics=True, chem_phase=True):
    e = np.zeros(2)
    lib().or_point_energy(C.byref(_cfg(3, mechanics, chem_phase)), C.byref(make_params(params)), phi_f, phi_w, xO,
                          _ptr(np.ascontiguousarray(ebar, dtype=np.float64)),
                          _ptr(np.ascontiguousarray(epsp, dtype=np.float64)), _ptr(e))
    return e
