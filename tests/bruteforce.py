"""Brute-force reference for tiny grids, written independently of the C oracle.

Mechanics: the displacement solve is done by assembling the quadratic elastic
energy explicitly -- a strain-displacement matrix B for the cell normal strains
and the interior-edge shear strains, a per-cell 3x3 stiffness and a per-edge
shear stiffness -- and solving the dense system with numpy.linalg.solve.
Chemistry and phase fields: whole-array numpy on ghost-padded grids.  The free
energy polynomials are differentiated with numpy.polyder.
"""
import math

import numpy as np

# Eq. 35 / 36 coefficients, highest power first (numpy.polyval convention)
POLY = {0: [163.708, -182.510, 90.573, -36.031, -4.372],
        2: [173.263, -213.460, 41.953],
        1: [1.0e3, 0.0, 0.0]}


def _h(x):
    return x ** 3 * (6 * x ** 2 - 15 * x + 10)


def _dh(x):
    return 30 * x ** 2 * (1 - x) ** 2


def _m(x, form):
    v = x ** 2 * (1 - x) ** 2
    return 16 * v if form == 0 else v


def _dm(x, form):
    v = 2 * x * (1 - x) * (1 - 2 * x)
    return 16 * v if form == 0 else v


def simplex(pf, pw):
    """Order parameters bounded to [0, 1] with phi_g = 1 - phi_f - phi_w: the
    nearest point of {phi >= 0, sum = 1} is max(u - theta, 0), with theta the
    root of sum_a max(u_a - theta, 0) = 1 (found here by bisection; cells
    already inside are returned unchanged)."""
    u = np.stack([pf, 1 - pf - pw, pw])
    inside = np.all(u >= 0, axis=0)
    lo = u.min(0) - 1.0                       # sum_a max(u_a - lo, 0) >= 1
    hi = u.max(0)                             # sum_a max(u_a - hi, 0) = 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        big = np.maximum(u - mid[None], 0).sum(0) > 1
        lo = np.where(big, mid, lo)
        hi = np.where(big, hi, mid)
    v = np.maximum(u - (0.5 * (lo + hi))[None], 0)
    return np.where(inside, pf, v[0]), np.where(inside, pw, v[2])


# ---------------------------------------------------------------------------
# Mechanics by explicit energy assembly
# ---------------------------------------------------------------------------
class Mech:
    def __init__(self, dim, shape, h):
        self.dim, self.h = dim, h
        if dim == 2:
            self.ny, self.nx = shape
            self.nz = 1
        else:
            self.nz, self.ny, self.nx = shape
        self.dof = {}
        nx, ny, nz = self.nx, self.ny, self.nz
        for k in range(nz):
            for j in range(ny):
                for i in range(1, nx):
                    self.dof[(0, i, j, k)] = len(self.dof)
        for k in range(nz):
            for j in range(1, ny):
                for i in range(nx):
                    self.dof[(1, i, j, k)] = len(self.dof)
        if dim == 3:
            for k in range(1, nz):
                for j in range(ny):
                    for i in range(nx):
                        self.dof[(2, i, j, k)] = len(self.dof)
        self.n = len(self.dof)

    def _row(self, terms):
        r = np.zeros(self.n)
        for (key, coef) in terms:
            if key in self.dof:
                r[self.dof[key]] += coef
        return r

    def cells(self):
        for k in range(self.nz):
            for j in range(self.ny):
                for i in range(self.nx):
                    yield i, j, k

    def normal_B(self, i, j, k):
        """3 x n rows: eps_xx, eps_yy, eps_zz of cell (i, j, k)."""
        ih = 1.0 / self.h
        B = np.zeros((3, self.n))
        B[0] = self._row([((0, i + 1, j, k), ih), ((0, i, j, k), -ih)])
        B[1] = self._row([((1, i, j + 1, k), ih), ((1, i, j, k), -ih)])
        if self.dim == 3:
            B[2] = self._row([((2, i, j, k + 1), ih), ((2, i, j, k), -ih)])
        return B

    def edges(self):
        """Interior edges: (kind, i, j, k, strain row, the 4 adjacent cells)."""
        ih = 0.5 / self.h
        nx, ny, nz = self.nx, self.ny, self.nz
        for k in range(nz):
            for j in range(1, ny):
                for i in range(1, nx):
                    row = self._row([((0, i, j, k), ih), ((0, i, j - 1, k), -ih), ((1, i, j, k), ih), ((1, i - 1, j, k), -ih)])
                    yield 3, row, [(i - 1, j - 1, k), (i, j - 1, k), (i - 1, j, k), (i, j, k)]
        if self.dim == 3:
            for k in range(1, nz):
                for j in range(ny):
                    for i in range(1, nx):
                        row = self._row([((0, i, j, k), ih), ((0, i, j, k - 1), -ih), ((2, i, j, k), ih), ((2, i - 1, j, k), -ih)])
                        yield 4, row, [(i - 1, j, k - 1), (i, j, k - 1), (i - 1, j, k), (i, j, k)]
            for k in range(1, nz):
                for j in range(1, ny):
                    for i in range(nx):
                        row = self._row([((1, i, j, k), ih), ((1, i, j, k - 1), -ih), ((2, i, j, k), ih), ((2, i, j - 1, k), -ih)])
                        yield 5, row, [(i, j - 1, k - 1), (i, j, k - 1), (i, j - 1, k), (i, j, k)]

    def solve(self, K, G, eT, epsp):
        """K, G, eT: cell arrays [nz][ny][nx]; epsp: (6, nz, ny, nx).  Minimise
        h^d sum_cells 1/2 (e - e*)^T C (e - e*) + h^d sum_edges 2 G_e (g - g*)^2."""
        A = np.zeros((self.n, self.n))
        b = np.zeros(self.n)
        one = np.ones(3)
        for (i, j, k) in self.cells():
            B = self.normal_B(i, j, k)
            C = K[k, j, i] * np.outer(one, one) + 2 * G[k, j, i] * (np.eye(3) - np.outer(one, one) / 3)
            es = eT[k, j, i] * one + epsp[:3, k, j, i]
            A += B.T @ C @ B
            b += B.T @ C @ es
        for kind, row, cells in self.edges():
            Ge = np.mean([G[c[2], c[1], c[0]] for c in cells])
            gs = np.mean([epsp[kind, c[2], c[1], c[0]] for c in cells])
            A += 4 * Ge * np.outer(row, row)
            b += 4 * Ge * row * gs
        u = np.linalg.solve(A, b)
        return self.unpack(u)

    def unpack(self, u):
        nx, ny, nz = self.nx, self.ny, self.nz
        ux = np.zeros((nz, ny, nx + 1))
        uy = np.zeros((nz, ny + 1, nx))
        uz = np.zeros((nz + 1, ny, nx)) if self.dim == 3 else None
        for (c, i, j, k), q in self.dof.items():
            (ux, uy, uz)[c][(k, j, i)] = u[q]
        return ux, uy, uz

    def cell_strains(self, ux, uy, uz):
        """(6, nz, ny, nx): normal strains at cells, shear = mean of the 4
        surrounding edges (boundary edges contribute zero)."""
        h = self.h
        nx, ny, nz = self.nx, self.ny, self.nz
        e = np.zeros((6, nz, ny, nx))
        e[0] = np.diff(ux, axis=2) / h
        e[1] = np.diff(uy, axis=1) / h
        if self.dim == 3:
            e[2] = np.diff(uz, axis=0) / h
        exy = np.zeros((nz, ny + 1, nx + 1))
        exy[:, 1:ny, 1:nx] = 0.5 * (np.diff(ux[:, :, 1:nx], axis=1) + np.diff(uy[:, 1:ny, :], axis=2)) / h
        e[3] = 0.25 * (exy[:, :-1, :-1] + exy[:, :-1, 1:] + exy[:, 1:, :-1] + exy[:, 1:, 1:])
        if self.dim == 3:
            exz = np.zeros((nz + 1, ny, nx + 1))
            exz[1:nz, :, 1:nx] = 0.5 * (np.diff(ux[:, :, 1:nx], axis=0) + np.diff(uz[1:nz, :, :], axis=2)) / h
            e[4] = 0.25 * (exz[:-1, :, :-1] + exz[:-1, :, 1:] + exz[1:, :, :-1] + exz[1:, :, 1:])
            eyz = np.zeros((nz + 1, ny + 1, nx))
            eyz[1:nz, 1:ny, :] = 0.5 * (np.diff(uy[:, 1:ny, :], axis=0) + np.diff(uz[1:nz, :, :], axis=1)) / h
            e[5] = 0.25 * (eyz[:-1, :-1, :] + eyz[:-1, 1:, :] + eyz[1:, :-1, :] + eyz[1:, 1:, :])
        return e


# ---------------------------------------------------------------------------
# One full step (2D or 3D) on whole arrays
# ---------------------------------------------------------------------------
def implicit_matrix(coef, dt, h, dirichlet):
    """Dense I + dt A for one species on the (nz, ny, nx) grid, assembled face
    by face: every interior face between cells a and b with the mean
    diffusivity couples them with weight D_face / h^2; a Dirichlet boundary
    face adds 2 D_cell / h^2 to its cell."""
    shp = coef.shape
    n = coef.size
    A = np.zeros((n, n))
    idx = np.arange(n).reshape(shp)
    for ax in range(3):
        m = shp[ax]
        if m == 1:
            continue
        for c in np.ndindex(*shp):
            a = idx[c]
            if c[ax] + 1 < m:
                nb = list(c)
                nb[ax] += 1
                b = idx[tuple(nb)]
                w = 0.5 * (coef[c] + coef[tuple(nb)]) / h ** 2
                A[a, a] += w
                A[b, b] += w
                A[a, b] -= w
                A[b, a] -= w
            if dirichlet and (c[ax] == 0 or c[ax] == m - 1):
                A[a, a] += 2 * coef[c] / h ** 2 * ((c[ax] == 0) + (c[ax] == m - 1))
    return np.eye(n) + dt * A


def reacted(a0, b0, xw, m, k, t):
    """Amount of O reacted in time t by a' = -k m a b, b' = -2 k m a b (the
    textbook solution a(t) = c a0 / ((2 a0 + c) e^(c k m t) - 2 a0),
    c = b0 - 2 a0; a0 / (1 + 2 a0 k m t) when c = 0), zero where a0 or b0 is
    not positive or the cell is full of water."""
    ok = (a0 > 0) & (b0 > 0) & (xw < 1) & (m > 0)
    a0s, b0s, ms = np.where(ok, a0, 1.0), np.where(ok, b0, 3.0), np.where(ok, m, 1.0)
    c = b0s - 2 * a0s
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        e = np.exp(c * k * ms * t)
        a = np.where(np.abs(c) > 1e-13, c * a0s / ((2 * a0s + c) * e - 2 * a0s), a0s / (1 + 2 * a0s * k * ms * t))
    a = np.where(np.isfinite(a), a, 0.0)
    return np.where(ok, a0s - a, 0.0)


def step(dim, shape, h, dt, p, f, u, epsp, epsP, plasticity=True, dirichlet=True, implicit=False):
    """Returns new (fields, u, epsp, epsP).  Arrays use (nz, ny, nx) shapes
    (2D: nz = 1); epsp is (6, nz, ny, nx)."""
    pf, pw, xO, xH, xW = (f[k] for k in ("phi_f", "phi_w", "xO", "xH", "xW"))
    pg = 1 - pf - pw
    H = [_h(pf), _h(pg), _h(pw)]
    dH = [_dh(pf), _dh(pg), _dh(pw)]
    Mm = [_m(pf, p.m_form), _m(pg, p.m_form), _m(pw, p.m_form)]
    dM = [_dm(pf, p.m_form), _dm(pg, p.m_form), _dm(pw, p.m_form)]
    dT = 1 - p.Omega_f * H[0]
    dTp = -p.Omega_f * dH[0]
    eT = np.cbrt(dT) - 1
    eTp = dTp / (3 * np.cbrt(dT) ** 2)
    K = dT * sum(H[a] * p.K[a] for a in range(3))
    G = dT * sum(H[a] * p.G[a] for a in range(3))
    # mechanics
    mech = Mech(dim, shape, h)
    ux, uy, uz = mech.solve(K, G, eT, epsp)
    ebar = mech.cell_strains(ux, uy, uz)
    one = np.array([1, 1, 1, 0, 0, 0], dtype=float)[:, None, None, None]
    etr = ebar - eT[None] * one - epsp
    tr = etr[0] + etr[1] + etr[2]
    dev = etr - tr[None] / 3 * one
    wts = np.array([1, 1, 1, 2, 2, 2], dtype=float)[:, None, None, None]
    ndev = np.sqrt((wts * dev ** 2).sum(0))
    s_norm = 2 * G * ndev
    ftr = s_norm - math.sqrt(2 / 3) * (p.sigY + p.Hhard * epsP)
    new_epsp, new_epsP = epsp.copy(), epsP.copy()
    if plasticity:
        yl = ftr > 0
        dl = np.where(yl, ftr / (2 * G + math.sqrt(2 / 3) * p.Hhard), 0.0)
        nrm = np.where(yl[None], dev / np.where(ndev > 0, ndev, 1)[None], 0.0)
        new_epsp = epsp + dl[None] * nrm
        new_epsP = epsP + dl
    ee = ebar - eT[None] * one - new_epsp
    tr = ee[0] + ee[1] + ee[2]
    dev = ee - tr[None] / 3 * one
    nd2 = (wts * dev ** 2).sum(0)
    pel = [0.5 * p.K[a] * tr ** 2 + p.G[a] * nd2 for a in range(3)]
    phi_el = sum(H[a] * pel[a] for a in range(3))
    gmf = dTp * phi_el + dT * (dH[0] * pel[0] - dH[1] * pel[1]) - eTp * 3 * K * tr
    gmw = dT * (dH[2] * pel[2] - dH[1] * pel[1])
    # chemistry
    scale = p.R * p.theta / p.Vmol
    psi = [scale * np.polyval(POLY[a], xO) for a in range(3)]
    mu_loc = scale * sum(H[a] * np.polyval(np.polyder(POLY[a]), xO) for a in range(3))
    pxx = scale * sum(H[a] * np.polyval(np.polyder(POLY[a], 2), xO) for a in range(3))
    hs = H[0] + H[1] + H[2]
    DO = sum(H[a] * p.DO[a] for a in range(3)) / hs
    DHh = sum(H[a] * p.DH[a] for a in range(3)) / hs
    DWw = sum(H[a] * p.DW[a] for a in range(3)) / hs
    MO = DO / pxx
    gf = dH[0] * psi[0] - dH[1] * psi[1] + p.w[0] * dM[0] - p.w[1] * dM[1] + gmf
    gw = dH[2] * psi[2] - dH[1] * psi[1] + p.w[2] * dM[2] - p.w[1] * dM[1] + gmw
    axes = [2, 1, 0][:dim]

    def lap(a):
        out = np.zeros_like(a)
        for ax in axes:
            pad = [(0, 0)] * 3
            pad[ax] = (1, 1)
            b = np.pad(a, pad, mode="edge")
            sl = lambda s, e: tuple(slice(s, e if e != 0 else None) if d == ax else slice(None) for d in range(3))
            out += b[sl(2, 0)] + b[sl(0, -2)] - 2 * a
        return out / h ** 2

    mu = mu_loc - p.kappaO * lap(xO)

    def div_flux(coef, val, bc):
        out = np.zeros_like(val)
        for ax in axes:
            n = val.shape[ax]
            J = np.zeros(tuple(s + 1 if d == ax else s for d, s in enumerate(val.shape)))
            lo = lambda a: np.take(a, range(0, n - 1), axis=ax)
            hi = lambda a: np.take(a, range(1, n), axis=ax)
            inner = -0.5 * (lo(coef) + hi(coef)) * (hi(val) - lo(val)) / h
            idx = [slice(None)] * 3
            idx[ax] = slice(1, n)
            J[tuple(idx)] = inner
            if bc is not None:
                idx[ax] = 0
                J[tuple(idx)] = -np.take(coef, 0, axis=ax) * (np.take(val, 0, axis=ax) - bc) / (h / 2)
                idx[ax] = n
                J[tuple(idx)] = -np.take(coef, n - 1, axis=ax) * (bc - np.take(val, n - 1, axis=ax)) / (h / 2)
            out += (np.take(J, range(1, n + 1), axis=ax) - np.take(J, range(0, n), axis=ax)) / h
        return out

    divO = div_flux(MO, mu, None)
    divH = div_flux(DHh, xH, p.xH_bc if dirichlet else None)
    divW = div_flux(DWw, xW, p.xW_bc if dirichlet else None)
    r = np.where(xW < 1, Mm[1] * p.kfor * np.clip(xO, 0, None) * np.clip(xH, 0, None), 0.0)
    if implicit == 2:
        r = np.zeros_like(r)                  # the reaction follows the transport, exactly
    lf, lw = lap(pf), lap(pw)
    nf, nw = simplex(pf + dt * p.L[0] * ((p.eps[0] + p.eps[1]) * lf + p.eps[1] * lw - gf),
                     pw + dt * p.L[2] * ((p.eps[2] + p.eps[1]) * lw + p.eps[1] * lf - gw))
    inc = {"xO": dt * (-divO - r), "xH": dt * (-divH - 2 * r), "xW": dt * (-divW + r)}
    if implicit:
        # linearly implicit Euler: (I + dt A) d = dt T(x^n), A the species' diffusion
        for key, coef, bc in (("xO", DO, False), ("xH", DHh, dirichlet), ("xW", DWw, dirichlet)):
            M = implicit_matrix(coef, dt, h, bc)
            inc[key] = np.linalg.solve(M, inc[key].ravel()).reshape(inc[key].shape)
    out = {
        "phi_f": nf,
        "phi_w": nw,
        "xO": xO + inc["xO"],
        "xH": xH + inc["xH"],
        "xW": xW + inc["xW"],
    }
    if implicit == 2:
        R = reacted(out["xO"], out["xH"], out["xW"], Mm[1], p.kfor, dt)
        out["xO"] = out["xO"] - R
        out["xH"] = out["xH"] - 2 * R
        out["xW"] = out["xW"] + R
    return out, (ux, uy, uz), new_epsp, new_epsP
