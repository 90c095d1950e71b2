"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module holds *inputs only*: the material parameters of the paper's
Table 1 (plus the gas constant, which the paper does not print), the time-step
choice, a counter-based random generator and the initial-condition builders
for the core-shell and porous workloads.  It contains none of the model's
arithmetic (no free energy, no fluxes, no mechanics); both the GPU path and the
CPU oracle receive these arrays and numbers as plain inputs.

Layouts are compact, x fastest: 2D cell fields are ``[ny][nx]``, 3D are
``[nz][ny][nx]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

# ---------------------------------------------------------------------------
# Parameters (Table 1 of the paper, SI units).  Phase order everywhere:
# index 0 = ferrite (f), 1 = gas (g), 2 = wuestite (w).
# ---------------------------------------------------------------------------

#: Molar gas constant (CODATA 2018); the paper uses R without printing it.
R_GAS = 8.314462618
#: Temperature of the calibration and of all simulations (Section 3.1).
THETA = 973.15
#: Molar volume of wuestite (Table 1).
V_MOL = 1.224e-5

#: Equilibrium oxygen fractions used for initial conditions: the common
#: tangent of the two calibrated polynomials of Eq. 35 (the test-suite checks
#: these digits against an independent tangent solve).  The caption of Fig. 1
#: prints 0.01 and 0.571 instead.
X_F_EQ = 0.010065296752744644
X_W_EQ = 0.5171256575723897
#: The values printed in the caption of Fig. 1.
X_F_PRINTED = 0.01
X_W_PRINTED = 0.571


@dataclass
class Params:
    """Material and model parameters (Table 1; Sections 2 and 3)."""
    R: float = R_GAS
    theta: float = THETA
    Vmol: float = V_MOL
    w: tuple = (1.0e3 / V_MOL, 1.0e3 / V_MOL, 1.0e3 / V_MOL)   # barrier heights
    eps: tuple = (4.0e-5, 4.0e-5, 4.0e-5)                      # phase gradient energy
    L: tuple = (1.5e-10, 1.5e-10, 1.5e-10)                     # phase mobilities
    kappaO: float = 5.0e-10                                    # chemical gradient energy
    K: tuple = (85e9, 0.17e9, 88e9)                            # bulk moduli f, g, w
    G: tuple = (41e9, 0.082e9, 24e9)                           # shear moduli f, g, w
    sigY: float = 0.3e9                                        # yield stress
    Hhard: float = 1.29e9                                      # hardening modulus (table value)
    DO: tuple = (2.16e-11, 1.0e-8, 2.16e-11)                   # oxygen diffusivity f, g, w
    DH: tuple = (2.5e-11, 1.0e-8, 2.5e-11)                     # hydrogen diffusivity
    DW: tuple = (2.5e-20, 1.0e-8, 2.5e-20)                     # water diffusivity
    kfor: float = 4.5e4                                        # reaction constant
    Omega_f: float = 0.4                                       # relative volume change
    xH_bc: float = 0.01                                        # hydrogen at gas boundaries
    xW_bc: float = 0.0                                         # water at gas boundaries
    m_form: int = 0    # 0: m(x)=16x^2(1-x)^2, 1: m(x)=x^2(1-x)^2

    def replace(self, **kw) -> "Params":
        d = asdict(self)
        d.update(kw)
        return Params(**d)


#: Grid spacing used by every workload: the paper's 5 um core-shell box over
#: 64 cells (the paper never states its mesh size).
H_DEFAULT = 5.0e-6 / 64


def stable_dt(p: Params, h: float, dim: int, safety: float = 0.2) -> float:
    """Explicit time step: ``safety`` times the tightest second-order
    diffusion-type bound of the scheme (species diffusion and the phase-field
    gradient term).  At the paper's parameters the gas diffusivities bind by
    many orders of magnitude; the reaction and fourth-order oxygen bounds are
    looser still and are documented rather than evaluated here."""
    dmax = max(max(p.DO), max(p.DH), max(p.DW))
    b_diff = h * h / (2.0 * dim * dmax)
    b_ac = min(h * h / (2.0 * dim * p.L[a] * (p.eps[a] + p.eps[1])) for a in (0, 2))
    return safety * min(b_diff, b_ac)


# ---------------------------------------------------------------------------
# Counter-based generator: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).
# Value k of stream ``seed`` is the SplitMix64 finaliser applied to
# seed + (k + 1) * golden-gamma, so any element can be drawn independently.
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, idx) -> np.ndarray:
    """Vectorised SplitMix64 outputs for counters ``idx`` of stream ``seed``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, idx) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Stream:
    """Sequential draws from one SplitMix64 stream."""

    def __init__(self, seed: int):
        self.seed = seed
        self.k = 0

    def uniform(self, n: int | None = None):
        m = 1 if n is None else n
        v = uniform01(self.seed, np.arange(self.k, self.k + m, dtype=np.uint64))
        self.k += m
        return float(v[0]) if n is None else v


# ---------------------------------------------------------------------------
# Initial conditions.  Each returns a dict of compact float64 arrays
# phi_f, phi_w, xO, xH, xW (gas phase is 1 - phi_f - phi_w).
# ---------------------------------------------------------------------------

def _empty(shape):
    return {k: np.zeros(shape, dtype=np.float64) for k in ("phi_f", "phi_w", "xO", "xH", "xW")}


def _noise(fields, seed: int, amp: float = 0.01):
    """phi_f += eta, phi_w -= eta with eta ~ U[-amp, amp) per cell index."""
    n = fields["phi_f"].size
    eta = (-amp + 2.0 * amp * uniform01(seed, np.arange(n, dtype=np.uint64))).reshape(fields["phi_f"].shape)
    fields["phi_f"] += eta
    fields["phi_w"] -= eta


def _centres(shape):
    """Cell-centre coordinates in cell units, one array per axis (x first)."""
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) + 0.5 for s in shape], indexing="ij")
    return list(reversed(grids))   # shape is (…, ny, nx); return x, y(, z)


def ic_core_shell(shape, r_core: float, r_shell: float | None = None, frame: int = 0,
                  noise_seed: int | None = None, x_w: float = X_W_EQ, x_f: float = X_F_EQ,
                  xH_gas: float = 0.01):
    """Core-shell workload (Section 4.2 geometry on a voxel grid).

    * ``r_shell is None`` (2D config style): wuestite disk of radius ``r_core``
      centred, ferrite everywhere else, and a gas frame ``frame`` cells wide
      along every edge.
    * ``r_shell`` given (3D config style): wuestite for r <= r_core, ferrite
      for r_core < r <= r_shell, gas outside.
    Solids start with x_O at their equilibrium value, gas with x_O = 0 and
    x_H = ``xH_gas``; x_H2O = 0 everywhere.
    """
    f = _empty(shape)
    coords = _centres(shape)
    centre = [s / 2.0 for s in reversed(shape)]
    r = np.sqrt(sum((c - m) ** 2 for c, m in zip(coords, centre)))
    core = r <= r_core
    if r_shell is None:
        gas = np.zeros(shape, dtype=bool)
        if frame > 0:
            for ax in range(len(shape)):
                idx = [slice(None)] * len(shape)
                idx[ax] = slice(0, frame)
                gas[tuple(idx)] = True
                idx[ax] = slice(shape[ax] - frame, shape[ax])
                gas[tuple(idx)] = True
        shell = ~core & ~gas
    else:
        shell = (~core) & (r <= r_shell)
        gas = ~(core | shell)
    f["phi_w"][core] = 1.0
    f["xO"][core] = x_w
    f["phi_f"][shell] = 1.0
    f["xO"][shell] = x_f
    f["xH"][gas] = xH_gas
    if noise_seed is not None:
        _noise(f, noise_seed)
    return f


def ic_porous(shape, porosity: float, n_grains: int, seed: int, semi_min: float = 4.0,
              semi_max: float = 20.0, x_w: float = X_W_EQ, xH_gas: float = 0.01, rim: float = 0.0,
              x_f: float = X_F_EQ):
    """Porous wuestite microstructure (stand-in for the SEM-derived section of
    Section 4.3, whose image is not available).

    Voronoi grain seeds are drawn (grain ids are returned but the model has a
    single isotropic wuestite field, so they do not enter the step); gas pores
    are ellipses (2D) or ellipsoids (3D) with semi-axes U(semi_min, semi_max)
    cells and random orientation, added until the gas fraction reaches
    ``porosity``.  With ``rim`` > 0 the solid within that distance (in cells,
    centre to centre) of a pore is already reduced: ferrite at x_O = x_f.
    """
    dim = len(shape)
    st = Stream(seed)
    nxyz = list(reversed(shape))
    seeds = np.stack([st.uniform(n_grains) * s for s in nxyz], axis=1)
    gas = np.zeros(shape, dtype=bool)
    target = porosity * gas.size
    count = 0
    while count < target:
        c = [st.uniform() * s for s in nxyz]
        a = [semi_min + (semi_max - semi_min) * st.uniform() for _ in range(dim)]
        if dim == 2:
            th = math.pi * st.uniform()
            rot = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        else:
            # random rotation from a unit quaternion (Shoemake's method)
            u1, u2, u3 = st.uniform(), st.uniform(), st.uniform()
            q = (math.sqrt(1 - u1) * math.sin(2 * math.pi * u2), math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
                 math.sqrt(u1) * math.sin(2 * math.pi * u3), math.sqrt(u1) * math.cos(2 * math.pi * u3))
            x, y, z, w = q
            rot = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
        rmax = max(a)
        lo = [max(0, int(math.floor(c[d] - rmax))) for d in range(dim)]
        hi = [min(nxyz[d], int(math.ceil(c[d] + rmax)) + 1) for d in range(dim)]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        axes = [np.arange(lo[d], hi[d], dtype=np.float64) + 0.5 - c[d] for d in range(dim)]
        mesh = np.meshgrid(*axes, indexing="ij")          # x, y(, z) order
        local = np.stack([m.ravel() for m in mesh], axis=0)
        body = rot.T @ local                                # coordinates in the ellipse frame
        inside = (sum((body[d] / a[d]) ** 2 for d in range(dim)) <= 1.0).reshape(mesh[0].shape)
        sl = tuple(slice(lo[d], hi[d]) for d in reversed(range(dim)))
        sub = gas[sl]
        add = np.transpose(inside)                          # to (z,) y, x order
        newly = add & ~sub
        count += int(newly.sum())
        sub |= add
    f = _empty(shape)
    solid = ~gas
    f["phi_w"][solid] = 1.0
    f["xO"][solid] = x_w
    f["xH"][gas] = xH_gas
    if rim > 0.0:
        from scipy.ndimage import distance_transform_edt
        ferrite = solid & (distance_transform_edt(solid) <= rim)
        f["phi_w"][ferrite] = 0.0
        f["phi_f"][ferrite] = 1.0
        f["xO"][ferrite] = x_f
    f["grain"] = _voronoi_ids(shape, seeds)
    return f


def ic_pores(shape=(32, 48), radius: float = 3.0, iso_x: float = 6.0, open_x: float = 34.0,
             channel_half: float = 1.0, prefill=None, prefill_rings: float = 1.0, x_w: float = X_W_EQ,
             xH_gas: float = 0.01):
    """Two pores in wuestite (the isolated and open pores of Sec. 4.3 on a
    synthetic section): gas disks of `radius` cells centred at mid-height and
    x = iso_x and x = open_x; the open one is joined to the right edge by a gas
    channel of half-width `channel_half` cells (every outer face carries the
    H-rich gas of the Dirichlet boundary), the isolated one is closed.  With
    `prefill` = value, the isolated pore and `prefill_rings` rings of solid
    around it start with x_H2O = value.  Returns the fields and the masks
    "iso", "open" and "wet" (the prefilled cells)."""
    ny, nx = shape
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    yc = ny / 2
    iso = (xx - iso_x) ** 2 + (yy - yc) ** 2 <= radius ** 2
    opn = ((xx - open_x) ** 2 + (yy - yc) ** 2 <= radius ** 2) | ((xx >= open_x) & (np.abs(yy - yc) <= channel_half))
    gas = iso | opn
    f = _empty(shape)
    f["phi_w"][~gas] = 1.0
    f["xO"][~gas] = x_w
    f["xH"][gas] = xH_gas
    wet = (xx - iso_x) ** 2 + (yy - yc) ** 2 <= (radius + prefill_rings) ** 2
    if prefill is not None:
        f["xW"][wet] = prefill
    return f, {"iso": iso, "open": opn, "wet": wet}


def _voronoi_ids(shape, seeds):
    from scipy.spatial import cKDTree
    coords = _centres(shape)
    pts = np.stack([c.ravel() for c in coords], axis=1)
    _, idx = cKDTree(seeds).query(pts)
    return idx.reshape(shape).astype(np.int32)


# ---------------------------------------------------------------------------
# The five workloads (seed 2111_11538 + config number).
# ---------------------------------------------------------------------------
SEED_BASE = 2111_11538


@dataclass
class Workload:
    name: str
    dim: int
    shape: tuple            # (ny, nx) or (nz, ny, nx)
    fields: dict
    params: Params
    h: float
    dt: float
    steps: int
    precision: str          # "fp64" or "mixed"
    plasticity: bool
    cg_rtol: float
    extra: dict = field(default_factory=dict)


def workload(name: str, n: int | None = None, steps: int | None = None) -> Workload:
    """Build one of the named workloads.  ``n`` overrides the grid side for a
    reduced-size variant of the same recipe (used by parity tests)."""
    p = Params()
    h = H_DEFAULT
    if name == "core_shell_2d":          # 64^2 core-shell, FP64, elastic
        n = n or 64
        f = ic_core_shell((n, n), r_core=20.0 * n / 64, frame=2, noise_seed=SEED_BASE + 1)
        return Workload(name, 2, (n, n), f, p, h, stable_dt(p, h, 2), steps or 200, "fp64", False, 1e-10)
    if name == "core_shell_3d":          # 128^3 core-shell, mixed, plastic
        n = n or 128
        f = ic_core_shell((n, n, n), r_core=48.0 * n / 128, r_shell=52.0 * n / 128, noise_seed=SEED_BASE + 2)
        return Workload(name, 3, (n, n, n), f, p, h, stable_dt(p, h, 3), steps or 1000, "mixed", True, 1e-6)
    if name == "porous_2d":              # 2048^2 porous, plastic, Omega_f 0.2, iron rims on the pores
        n = n or 2048
        ng = max(4, int(round(400 * (n / 2048) ** 2)))
        f = ic_porous((n, n), 0.15, ng, SEED_BASE + 3, rim=2.0)
        pp = p.replace(Omega_f=0.2)
        return Workload(name, 2, (n, n), f, pp, h, stable_dt(pp, h, 2), steps or 5000, "mixed", True, 1e-6)
    if name == "porous_3d":              # 256^3 porous, plastic, Omega_f 0.2, iron rims on the pores
        n = n or 256
        ng = max(4, int(round(64 * (n / 256) ** 3)))
        f = ic_porous((n, n, n), 0.20, ng, SEED_BASE + 5, rim=2.0)
        pp = p.replace(Omega_f=0.2)
        return Workload(name, 3, (n, n, n), f, pp, h, stable_dt(pp, h, 3), steps or 500, "mixed", True, 1e-6)
    raise ValueError(f"unknown workload {name}")


def batch_instances(count: int = 64, side_lo: int = 64, side_hi: int = 512, seed: int = SEED_BASE + 4):
    """Uneven batch of 2D core-shell instances: side ~ U{side_lo..side_hi},
    disk radius ~ U(0.2, 0.45) * side, same template as the 64^2 workload."""
    st = Stream(seed)
    out = []
    for b in range(count):
        side = side_lo + int(st.uniform() * (side_hi - side_lo + 1))
        side = min(side, side_hi)
        rfrac = 0.2 + 0.25 * st.uniform()
        f = ic_core_shell((side, side), r_core=rfrac * side, frame=2, noise_seed=seed * 1000 + b)
        out.append(((side, side), f))
    return out
