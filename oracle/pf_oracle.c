/* FP64 CPU oracle of one explicit time step of the chemo-mechanical
 * phase-field model of wuestite reduction by hydrogen (arXiv:2111.11538).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark to check the HIP path.  It shares no code
 * with that path.  Plain loops, no blocking or fusion beyond what the
 * discrete definitions below state; every sum runs in one fixed
 * (lexicographic) order so the oracle is bitwise reproducible.
 *
 * Discrete model (paper section / equation in brackets):
 *  - cell-centred phi_f, phi_w, x_O, x_H, x_H2O; phi_g = 1 - phi_f - phi_w [Eq. 15]
 *  - chemical energy psi_che = sum_a h(phi_a) (R theta / V_mol) f_a(x_O)
 *    [Eq. 6, Eq. 35, Eq. 36]; h(x) = x^3 (6x^2 - 15x + 10) [Sec. 3.1];
 *    m(x) is never written out in the paper; the reading used here is
 *    m = 16 x^2 (1-x)^2, so that w_a is the barrier height [Eq. 7]
 *  - Allen-Cahn for phi_f, phi_w [Eq. 29 (5,6), Eq. 33]
 *  - O flux j_O = -M_O grad mu_O, mu_O = d psi_che / d x_O - kappa_O lap x_O,
 *    M_O = D_O / (d^2 psi_che / d x_O^2) [Eq. 19, Eq. 24, Eq. 30, Sec. 3.2]
 *  - H and H2O: Fick with phase-interpolated D [Eq. 29 (1,2)]
 *  - reaction r = m(phi_g) k_for x_O x_H, zero where x_H2O >= 1 [Eq. 27, 28;
 *    Sec. 4.3]
 *  - small-strain reading of the kinematics: eps_e = eps(u) - eps_T I - eps_p,
 *    eps_T = d_T^(1/3) - 1, d_T = 1 - h(phi_f) Omega_f [Eq. 9];
 *    K = d_T sum h K_a, G = d_T sum h G_a [Eq. 32]
 *  - J2 plasticity with linear hardening, backward-Euler radial return
 *    [Eq. 25, Eq. 34]
 *  - quasi-static equilibrium div sigma = 0 [Eq. 29 (4)] on a staggered grid
 *    (normal strains at cells, shear strains at edges, rollers on the outer
 *    faces), solved by Jacobi-preconditioned CG.
 */
#include "pf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define XX 0
#define YY 1
#define ZZ 2
#define XY 3
#define XZ 4
#define YZ 5

static int ncomp(const or_config *c) { return c->dim == 2 ? 4 : 6; }
static long ncell(const or_config *c) { return (long)c->nx * c->ny * c->nz; }
static long nfx(const or_config *c) { return (long)(c->nx + 1) * c->ny * c->nz; }
static long nfy(const or_config *c) { return (long)c->nx * (c->ny + 1) * c->nz; }
static long nfz(const or_config *c) { return c->dim == 3 ? (long)c->nx * c->ny * (c->nz + 1) : 0; }

static long CI(const or_config *c, int i, int j, int k) { return ((long)k * c->ny + j) * c->nx + i; }
static long XI(const or_config *c, int i, int j, int k) { return ((long)k * c->ny + j) * (c->nx + 1) + i; }
static long YI(const or_config *c, int i, int j, int k) { return ((long)k * (c->ny + 1) + j) * c->nx + i; }
static long ZI(const or_config *c, int i, int j, int k) { return ((long)k * c->ny + j) * c->nx + i; }
/* edges: xy on z-edges (x = i h, y = j h), xz on y-edges (x = i h, z = k h),
 * yz on x-edges (y = j h, z = k h) */
static long EXY(const or_config *c, int i, int j, int k) { return ((long)k * (c->ny + 1) + j) * (c->nx + 1) + i; }
static long EXZ(const or_config *c, int i, int j, int k) { return ((long)k * c->ny + j) * (c->nx + 1) + i; }
static long EYZ(const or_config *c, int i, int j, int k) { return ((long)k * (c->ny + 1) + j) * c->nx + i; }
static long nexy(const or_config *c) { return (long)(c->nx + 1) * (c->ny + 1) * c->nz; }
static long nexz(const or_config *c) { return (long)(c->nx + 1) * c->ny * (c->nz + 1); }
static long neyz(const or_config *c) { return (long)c->nx * (c->ny + 1) * (c->nz + 1); }

/* ------------------------------------------------------------------------ */
/* Interpolation functions                                                   */
/* ------------------------------------------------------------------------ */
static double hfun(double x) { return x * x * x * (6.0 * x * x - 15.0 * x + 10.0); }
static double dhfun(double x) { return 30.0 * x * x * (1.0 - x) * (1.0 - x); }
static double mfun(const or_params *p, double x) {
  double v = x * x * (1.0 - x) * (1.0 - x);
  return p->m_form == 0 ? 16.0 * v : v;
}
static double dmfun(const or_params *p, double x) {
  double v = 2.0 * x * (1.0 - x) * (1.0 - 2.0 * x);
  return p->m_form == 0 ? 16.0 * v : v;
}

/* ------------------------------------------------------------------------ */
/* Scaled chemical free energies f_a(x) = (V_mol / R theta) psi_a [Eq. 35,36] */
/* out[0] = f, out[1] = f', out[2] = f''                                     */
/* ------------------------------------------------------------------------ */
void or_fe(int phase, double x, double out[3]) {
  if (phase == 0) {        /* ferrite, Eq. 35 first line */
    out[0] = 163.708 * x * x * x * x - 182.510 * x * x * x + 90.573 * x * x - 36.031 * x - 4.372;
    out[1] = 4.0 * 163.708 * x * x * x - 3.0 * 182.510 * x * x + 2.0 * 90.573 * x - 36.031;
    out[2] = 12.0 * 163.708 * x * x - 6.0 * 182.510 * x + 2.0 * 90.573;
  } else if (phase == 2) { /* wuestite, Eq. 35 second line */
    out[0] = 173.263 * x * x - 213.460 * x + 41.953;
    out[1] = 2.0 * 173.263 * x - 213.460;
    out[2] = 2.0 * 173.263;
  } else {                 /* gas, Eq. 36 */
    out[0] = 1.0e3 * x * x;
    out[1] = 2.0e3 * x;
    out[2] = 2.0e3;
  }
}

/* Common tangent of f_f and f_w [Eq. 37]: f_f'(a) = f_w'(b) = (f_w(b) - f_f(a)) / (b - a). */
int or_common_tangent(double *xf, double *xw, double *resid) {
  double a = 0.01, b = 0.52;
  for (int it = 0; it < 100; ++it) {
    double fa[3], fb[3];
    or_fe(0, a, fa);
    or_fe(2, b, fb);
    double F1 = fa[1] - fb[1];
    double F2 = fa[0] + fa[1] * (b - a) - fb[0];
    double J11 = fa[2], J12 = -fb[2];
    double J21 = fa[2] * (b - a), J22 = fa[1] - fb[1];
    double det = J11 * J22 - J12 * J21;
    double da = (F1 * J22 - J12 * F2) / det;
    double db = (J11 * F2 - J21 * F1) / det;
    a -= da;
    b -= db;
    if (fabs(da) + fabs(db) < 1e-16) break;
  }
  double fa[3], fb[3];
  or_fe(0, a, fa);
  or_fe(2, b, fb);
  *xf = a;
  *xw = b;
  *resid = fabs(fa[1] - fb[1]) + fabs(fa[1] - (fb[0] - fa[0]) / (b - a));
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Local constitutive quantities of one cell                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  double pf, pg, pw;            /* phase fields */
  double h[3], dh[3], m[3], dm[3];
  double dT, dTp, eT, eTp;      /* d_T, d d_T/d phi_f, eps_T, d eps_T / d phi_f */
  double K, G;                  /* effective moduli [Eq. 32] */
  double psi[3];                /* psi_a = (R theta / V_mol) f_a(x_O) */
  double mu_loc, psi_xx, MO;    /* d psi_che/dx, d2 psi_che/dx2, M_O = D_O/psi_xx */
  double DO, DH, DW;            /* phase-interpolated diffusivities */
} local_t;

static void local_eval(const or_params *p, double pf, double pw, double xO, local_t *q) {
  double ph[3];
  q->pf = pf;
  q->pw = pw;
  q->pg = 1.0 - pf - pw;                                  /* Eq. 15 */
  ph[0] = q->pf; ph[1] = q->pg; ph[2] = q->pw;
  for (int a = 0; a < 3; ++a) {
    q->h[a] = hfun(ph[a]);
    q->dh[a] = dhfun(ph[a]);
    q->m[a] = mfun(p, ph[a]);
    q->dm[a] = dmfun(p, ph[a]);
  }
  q->dT = 1.0 - q->h[0] * p->Omega_f;                     /* Eq. 9 */
  q->dTp = -q->dh[0] * p->Omega_f;
  q->eT = cbrt(q->dT) - 1.0;                              /* small-strain F_T - I */
  q->eTp = q->dTp / (3.0 * cbrt(q->dT) * cbrt(q->dT));
  q->K = q->dT * (q->h[0] * p->K[0] + q->h[1] * p->K[1] + q->h[2] * p->K[2]);   /* Eq. 32 */
  q->G = q->dT * (q->h[0] * p->G[0] + q->h[1] * p->G[1] + q->h[2] * p->G[2]);
  double scale = p->R * p->theta / p->Vmol;
  double mu = 0.0, pxx = 0.0;
  for (int a = 0; a < 3; ++a) {
    double f[3];
    or_fe(a, xO, f);
    q->psi[a] = scale * f[0];
    mu += q->h[a] * f[1];
    pxx += q->h[a] * f[2];
  }
  q->mu_loc = scale * mu;
  q->psi_xx = scale * pxx;
  double hs = q->h[0] + q->h[1] + q->h[2];
  q->DO = (q->h[0] * p->DO[0] + q->h[1] * p->DO[1] + q->h[2] * p->DO[2]) / hs;
  q->DH = (q->h[0] * p->DH[0] + q->h[1] * p->DH[1] + q->h[2] * p->DH[2]) / hs;
  q->DW = (q->h[0] * p->DW[0] + q->h[1] * p->DW[1] + q->h[2] * p->DW[2]) / hs;
  q->MO = q->DO / q->psi_xx;                              /* Sec. 3.2 */
}

void or_local(const or_params *p, double phi_f, double phi_w, double xO, double out[16]) {
  local_t q;
  local_eval(p, phi_f, phi_w, xO, &q);
  out[0] = q.pg; out[1] = q.h[0]; out[2] = q.h[1]; out[3] = q.h[2];
  out[4] = q.dT; out[5] = q.eT; out[6] = q.K; out[7] = q.G;
  out[8] = q.mu_loc; out[9] = q.psi_xx; out[10] = q.MO; out[11] = q.DO;
  out[12] = q.DH; out[13] = q.DW;
  /* chemical + barrier part of d psi / d phi_f and d psi / d phi_w [Eq. 33] */
  out[14] = q.dh[0] * q.psi[0] - q.dh[1] * q.psi[1] + p->w[0] * q.dm[0] - p->w[1] * q.dm[1];
  out[15] = q.dh[2] * q.psi[2] - q.dh[1] * q.psi[1] + p->w[2] * q.dm[2] - p->w[1] * q.dm[1];
}

/* ------------------------------------------------------------------------ */
/* Small-strain elasticity on the staggered grid                              */
/* ------------------------------------------------------------------------ */
void or_moduli(const or_config *c, const or_params *p, const double *phi_f, const double *phi_w,
               double *K, double *G) {
  long n = ncell(c);
#pragma omp parallel for
  for (long q = 0; q < n; ++q) {
    local_t L;
    local_eval(p, phi_f[q], phi_w[q], 0.0, &L);
    K[q] = L.K;
    G[q] = L.G;
  }
}

/* total shear strains at interior edges; zero on boundary edges (mirror
 * symmetry of the roller faces) */
static double exy_u(const or_config *c, const double *ux, const double *uy, int i, int j, int k) {
  if (i <= 0 || i >= c->nx || j <= 0 || j >= c->ny) return 0.0;
  return 0.5 * ((ux[XI(c, i, j, k)] - ux[XI(c, i, j - 1, k)]) + (uy[YI(c, i, j, k)] - uy[YI(c, i - 1, j, k)])) / c->h;
}
static double exz_u(const or_config *c, const double *ux, const double *uz, int i, int j, int k) {
  if (i <= 0 || i >= c->nx || k <= 0 || k >= c->nz) return 0.0;
  return 0.5 * ((ux[XI(c, i, j, k)] - ux[XI(c, i, j, k - 1)]) + (uz[ZI(c, i, j, k)] - uz[ZI(c, i - 1, j, k)])) / c->h;
}
static double eyz_u(const or_config *c, const double *uy, const double *uz, int i, int j, int k) {
  if (j <= 0 || j >= c->ny || k <= 0 || k >= c->nz) return 0.0;
  return 0.5 * ((uy[YI(c, i, j, k)] - uy[YI(c, i, j, k - 1)]) + (uz[ZI(c, i, j, k)] - uz[ZI(c, i, j - 1, k)])) / c->h;
}

/* Cell strain: normal components from the face differences, shear components
 * as the mean of the four surrounding edges. */
void or_cell_strain(const or_config *c, const double *ux, const double *uy, const double *uz,
                    int i, int j, int k, double e[6]) {
  double ih = 1.0 / c->h;
  e[XX] = (ux[XI(c, i + 1, j, k)] - ux[XI(c, i, j, k)]) * ih;
  e[YY] = (uy[YI(c, i, j + 1, k)] - uy[YI(c, i, j, k)]) * ih;
  e[ZZ] = c->dim == 3 ? (uz[ZI(c, i, j, k + 1)] - uz[ZI(c, i, j, k)]) * ih : 0.0;   /* plane strain */
  e[XY] = 0.25 * (exy_u(c, ux, uy, i, j, k) + exy_u(c, ux, uy, i + 1, j, k) +
                  exy_u(c, ux, uy, i, j + 1, k) + exy_u(c, ux, uy, i + 1, j + 1, k));
  if (c->dim == 3) {
    e[XZ] = 0.25 * (exz_u(c, ux, uz, i, j, k) + exz_u(c, ux, uz, i + 1, j, k) +
                    exz_u(c, ux, uz, i, j, k + 1) + exz_u(c, ux, uz, i + 1, j, k + 1));
    e[YZ] = 0.25 * (eyz_u(c, uy, uz, i, j, k) + eyz_u(c, uy, uz, i, j + 1, k) +
                    eyz_u(c, uy, uz, i, j, k + 1) + eyz_u(c, uy, uz, i, j + 1, k + 1));
  } else {
    e[XZ] = 0.0;
    e[YZ] = 0.0;
  }
}

typedef struct {
  double *sxx, *syy, *szz, *sxy, *sxz, *syz;
} stress_t;

static void stress_alloc(const or_config *c, stress_t *s) {
  long n = ncell(c);
  s->sxx = calloc(n, sizeof(double));
  s->syy = calloc(n, sizeof(double));
  s->szz = calloc(n, sizeof(double));
  s->sxy = calloc(nexy(c), sizeof(double));
  s->sxz = c->dim == 3 ? calloc(nexz(c), sizeof(double)) : NULL;
  s->syz = c->dim == 3 ? calloc(neyz(c), sizeof(double)) : NULL;
}
static void stress_free(stress_t *s) {
  free(s->sxx); free(s->syy); free(s->szz); free(s->sxy); free(s->sxz); free(s->syz);
}

/* mean over the 4 cells around an edge */
static double edge_mean_xy(const or_config *c, const double *a, int i, int j, int k) {
  return 0.25 * (a[CI(c, i - 1, j - 1, k)] + a[CI(c, i, j - 1, k)] + a[CI(c, i - 1, j, k)] + a[CI(c, i, j, k)]);
}
static double edge_mean_xz(const or_config *c, const double *a, int i, int j, int k) {
  return 0.25 * (a[CI(c, i - 1, j, k - 1)] + a[CI(c, i, j, k - 1)] + a[CI(c, i - 1, j, k)] + a[CI(c, i, j, k)]);
}
static double edge_mean_yz(const or_config *c, const double *a, int i, int j, int k) {
  return 0.25 * (a[CI(c, i, j - 1, k - 1)] + a[CI(c, i, j, k - 1)] + a[CI(c, i, j - 1, k)] + a[CI(c, i, j, k)]);
}

/* Stresses of (eps(u) - eps*) with eps* = eT I + eps_p (both may be NULL = 0).
 * Cell normal stresses: sigma_ii = K tr + 2G (e_ii - tr/3).  Interior-edge
 * shear stresses: 2 G_e (eps_ij(u) - mean eps_p,ij), boundary edges carry 0. */
static void stresses(const or_config *c, const double *K, const double *G, const double *eT,
                     const double *epsp, const double *ux, const double *uy, const double *uz,
                     stress_t *s) {
  long n = ncell(c);
  double ih = 1.0 / c->h;
  int nx = c->nx, ny = c->ny, nz = c->nz;
#pragma omp parallel for collapse(2)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long q = CI(c, i, j, k);
        double e[3];
        e[0] = (ux[XI(c, i + 1, j, k)] - ux[XI(c, i, j, k)]) * ih;
        e[1] = (uy[YI(c, i, j + 1, k)] - uy[YI(c, i, j, k)]) * ih;
        e[2] = c->dim == 3 ? (uz[ZI(c, i, j, k + 1)] - uz[ZI(c, i, j, k)]) * ih : 0.0;
        for (int d = 0; d < 3; ++d) {
          if (eT) e[d] -= eT[q];
          if (epsp) e[d] -= epsp[d * n + q];
        }
        double tr = e[0] + e[1] + e[2];
        s->sxx[q] = K[q] * tr + 2.0 * G[q] * (e[0] - tr / 3.0);
        s->syy[q] = K[q] * tr + 2.0 * G[q] * (e[1] - tr / 3.0);
        s->szz[q] = K[q] * tr + 2.0 * G[q] * (e[2] - tr / 3.0);
      }
#pragma omp parallel for collapse(2)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        double v = 0.0;
        if (i > 0 && i < nx && j > 0 && j < ny) {
          double ep = epsp ? edge_mean_xy(c, epsp + XY * n, i, j, k) : 0.0;
          v = 2.0 * edge_mean_xy(c, G, i, j, k) * (exy_u(c, ux, uy, i, j, k) - ep);
        }
        s->sxy[EXY(c, i, j, k)] = v;
      }
  if (c->dim == 3) {
#pragma omp parallel for collapse(2)
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
          double v = 0.0;
          if (i > 0 && i < nx && k > 0 && k < nz) {
            double ep = epsp ? edge_mean_xz(c, epsp + XZ * n, i, j, k) : 0.0;
            v = 2.0 * edge_mean_xz(c, G, i, j, k) * (exz_u(c, ux, uz, i, j, k) - ep);
          }
          s->sxz[EXZ(c, i, j, k)] = v;
        }
#pragma omp parallel for collapse(2)
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double v = 0.0;
          if (j > 0 && j < ny && k > 0 && k < nz) {
            double ep = epsp ? edge_mean_yz(c, epsp + YZ * n, i, j, k) : 0.0;
            v = 2.0 * edge_mean_yz(c, G, i, j, k) * (eyz_u(c, uy, uz, i, j, k) - ep);
          }
          s->syz[EYZ(c, i, j, k)] = v;
        }
  }
}

/* g = (gradient of the discrete elastic energy) / h^(d-1) on every face;
 * boundary (roller) faces are fixed and get 0. */
static void divergence(const or_config *c, const stress_t *s, double *gx, double *gy, double *gz) {
  int nx = c->nx, ny = c->ny, nz = c->nz, d3 = c->dim == 3;
#pragma omp parallel for collapse(2)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        double v = 0.0;
        if (i > 0 && i < nx) {
          v = s->sxx[CI(c, i - 1, j, k)] - s->sxx[CI(c, i, j, k)] +
              s->sxy[EXY(c, i, j, k)] - s->sxy[EXY(c, i, j + 1, k)];
          if (d3) v += s->sxz[EXZ(c, i, j, k)] - s->sxz[EXZ(c, i, j, k + 1)];
        }
        gx[XI(c, i, j, k)] = v;
      }
#pragma omp parallel for collapse(2)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double v = 0.0;
        if (j > 0 && j < ny) {
          v = s->syy[CI(c, i, j - 1, k)] - s->syy[CI(c, i, j, k)] +
              s->sxy[EXY(c, i, j, k)] - s->sxy[EXY(c, i + 1, j, k)];
          if (d3) v += s->syz[EYZ(c, i, j, k)] - s->syz[EYZ(c, i, j, k + 1)];
        }
        gy[YI(c, i, j, k)] = v;
      }
  if (d3) {
#pragma omp parallel for collapse(2)
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double v = 0.0;
          if (k > 0 && k < nz) {
            v = s->szz[CI(c, i, j, k - 1)] - s->szz[CI(c, i, j, k)] +
                s->sxz[EXZ(c, i, j, k)] - s->sxz[EXZ(c, i + 1, j, k)] +
                s->syz[EYZ(c, i, j, k)] - s->syz[EYZ(c, i, j + 1, k)];
          }
          gz[ZI(c, i, j, k)] = v;
        }
  }
}

void or_apply(const or_config *c, const double *K, const double *G,
              const double *ux, const double *uy, const double *uz,
              double *qx, double *qy, double *qz) {
  stress_t s;
  stress_alloc(c, &s);
  stresses(c, K, G, NULL, NULL, ux, uy, uz, &s);
  divergence(c, &s, qx, qy, qz);
  stress_free(&s);
}

static void eigen_arrays(const or_config *c, const or_params *p, const double *phi_f, const double *phi_w,
                         double *eT, double *K, double *G) {
  long n = ncell(c);
#pragma omp parallel for
  for (long q = 0; q < n; ++q) {
    local_t L;
    local_eval(p, phi_f[q], phi_w[q], 0.0, &L);
    eT[q] = L.eT;
    K[q] = L.K;
    G[q] = L.G;
  }
}

/* b = -g(0): right-hand side of A u = b */
void or_rhs(const or_config *c, const or_params *p, const or_state *st, double *bx, double *by, double *bz) {
  long n = ncell(c);
  double *eT = malloc(n * sizeof(double)), *K = malloc(n * sizeof(double)), *G = malloc(n * sizeof(double));
  double *zx = calloc(nfx(c), sizeof(double)), *zy = calloc(nfy(c), sizeof(double));
  double *zz = c->dim == 3 ? calloc(nfz(c), sizeof(double)) : NULL;
  eigen_arrays(c, p, st->phi_f, st->phi_w, eT, K, G);
  stress_t s;
  stress_alloc(c, &s);
  stresses(c, K, G, eT, st->epsp, zx, zy, zz, &s);
  divergence(c, &s, bx, by, bz);
  for (long q = 0; q < nfx(c); ++q) bx[q] = -bx[q];
  for (long q = 0; q < nfy(c); ++q) by[q] = -by[q];
  for (long q = 0; q < nfz(c); ++q) bz[q] = -bz[q];
  stress_free(&s);
  free(eT); free(K); free(G); free(zx); free(zy); free(zz);
}

/* Diagonal of A: (M_left + M_right + sum of G_e over adjacent interior edges) / h,
 * M = K + 4G/3; zero on the fixed boundary faces. */
void or_diag(const or_config *c, const double *K, const double *G, double *dx, double *dy, double *dz) {
  int nx = c->nx, ny = c->ny, nz = c->nz, d3 = c->dim == 3;
  double ih = 1.0 / c->h;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        double v = 0.0;
        if (i > 0 && i < nx) {
          long a = CI(c, i - 1, j, k), b = CI(c, i, j, k);
          v = K[a] + 4.0 * G[a] / 3.0 + K[b] + 4.0 * G[b] / 3.0;
          if (j > 0) v += edge_mean_xy(c, G, i, j, k);
          if (j + 1 < ny) v += edge_mean_xy(c, G, i, j + 1, k);
          if (d3 && k > 0) v += edge_mean_xz(c, G, i, j, k);
          if (d3 && k + 1 < nz) v += edge_mean_xz(c, G, i, j, k + 1);
        }
        dx[XI(c, i, j, k)] = v * ih;
      }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double v = 0.0;
        if (j > 0 && j < ny) {
          long a = CI(c, i, j - 1, k), b = CI(c, i, j, k);
          v = K[a] + 4.0 * G[a] / 3.0 + K[b] + 4.0 * G[b] / 3.0;
          if (i > 0) v += edge_mean_xy(c, G, i, j, k);
          if (i + 1 < nx) v += edge_mean_xy(c, G, i + 1, j, k);
          if (d3 && k > 0) v += edge_mean_yz(c, G, i, j, k);
          if (d3 && k + 1 < nz) v += edge_mean_yz(c, G, i, j, k + 1);
        }
        dy[YI(c, i, j, k)] = v * ih;
      }
  if (d3) {
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double v = 0.0;
          if (k > 0 && k < nz) {
            long a = CI(c, i, j, k - 1), b = CI(c, i, j, k);
            v = K[a] + 4.0 * G[a] / 3.0 + K[b] + 4.0 * G[b] / 3.0;
            if (i > 0) v += edge_mean_xz(c, G, i, j, k);
            if (i + 1 < nx) v += edge_mean_xz(c, G, i + 1, j, k);
            if (j > 0) v += edge_mean_yz(c, G, i, j, k);
            if (j + 1 < ny) v += edge_mean_yz(c, G, i, j + 1, k);
          }
          dz[ZI(c, i, j, k)] = v * ih;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned CG on A u = b (warm start from the state's u)        */
/* ------------------------------------------------------------------------ */
static double dot3(const double *a, const double *b, long n) {
  double s = 0.0;
  for (long q = 0; q < n; ++q) s += a[q] * b[q];
  return s;
}

int or_mech_solve(const or_config *c, const or_params *p, or_state *st, or_stats *stats) {
  long n = ncell(c);
  long nf = nfx(c) + nfy(c) + nfz(c);
  long ox = 0, oy = nfx(c), oz = nfx(c) + nfy(c);
  double *eT = malloc(n * sizeof(double)), *K = malloc(n * sizeof(double)), *G = malloc(n * sizeof(double));
  double *u = malloc(nf * sizeof(double)), *r = malloc(nf * sizeof(double)), *z = malloc(nf * sizeof(double));
  double *pp = malloc(nf * sizeof(double)), *qq = malloc(nf * sizeof(double)), *dg = malloc(nf * sizeof(double));
  double *b = malloc(nf * sizeof(double)), *zero = calloc(nf, sizeof(double));
  eigen_arrays(c, p, st->phi_f, st->phi_w, eT, K, G);
  memcpy(u + ox, st->ux, nfx(c) * sizeof(double));
  memcpy(u + oy, st->uy, nfy(c) * sizeof(double));
  if (c->dim == 3) memcpy(u + oz, st->uz, nfz(c) * sizeof(double));
  /* roller faces are fixed at zero */
  or_diag(c, K, G, dg + ox, dg + oy, c->dim == 3 ? dg + oz : NULL);
  for (long q = 0; q < nf; ++q)
    if (dg[q] == 0.0) u[q] = 0.0;
  stress_t s;
  stress_alloc(c, &s);
#define GRAD(vec, eig, out)                                                                     \
  do {                                                                                        \
    stresses(c, K, G, (eig) ? eT : NULL, (eig) ? st->epsp : NULL, (vec) + ox, (vec) + oy,     \
             c->dim == 3 ? (vec) + oz : NULL, &s);                                             \
    divergence(c, &s, (out) + ox, (out) + oy, c->dim == 3 ? (out) + oz : NULL);               \
  } while (0)
  GRAD(zero, 1, b);
  for (long q = 0; q < nf; ++q) b[q] = -b[q];
  GRAD(u, 1, r);
  for (long q = 0; q < nf; ++q) r[q] = -r[q];
  double bnorm = sqrt(dot3(b, b, nf));
  int it = 0, status = OR_OK;
  double rel = 0.0;
  if (bnorm == 0.0) {
    for (long q = 0; q < nf; ++q) u[q] = 0.0;
  } else {
    double rnorm = sqrt(dot3(r, r, nf));
    if (rnorm > c->cg_rtol * bnorm) {
      for (long q = 0; q < nf; ++q) z[q] = dg[q] > 0.0 ? r[q] / dg[q] : 0.0;
      memcpy(pp, z, nf * sizeof(double));
      double rz = dot3(r, z, nf);
      int conv = 0;
      while (it < c->cg_max_iter) {
        GRAD(pp, 0, qq);
        double pq = dot3(pp, qq, nf);
        double alpha = rz / pq;
        for (long q = 0; q < nf; ++q) {
          u[q] += alpha * pp[q];
          r[q] -= alpha * qq[q];
        }
        ++it;
        rnorm = sqrt(dot3(r, r, nf));
        if (rnorm <= c->cg_rtol * bnorm) { conv = 1; break; }
        for (long q = 0; q < nf; ++q) z[q] = dg[q] > 0.0 ? r[q] / dg[q] : 0.0;
        double rz_new = dot3(r, z, nf);
        double beta = rz_new / rz;
        rz = rz_new;
        for (long q = 0; q < nf; ++q) pp[q] = z[q] + beta * pp[q];
      }
      if (!conv) status = OR_CG_NOT_CONVERGED;
    }
    GRAD(u, 1, r);   /* true residual on exit */
    rel = sqrt(dot3(r, r, nf)) / bnorm;
  }
#undef GRAD
  memcpy(st->ux, u + ox, nfx(c) * sizeof(double));
  memcpy(st->uy, u + oy, nfy(c) * sizeof(double));
  if (c->dim == 3) memcpy(st->uz, u + oz, nfz(c) * sizeof(double));
  if (stats) {
    stats->cg_iters = it;
    stats->cg_rel_resid = rel;
  }
  stress_free(&s);
  free(eT); free(K); free(G); free(u); free(r); free(z); free(pp); free(qq); free(dg); free(b); free(zero);
  return status;
}

/* ------------------------------------------------------------------------ */
/* J2 return map [Eq. 25, Eq. 34], backward Euler, linear hardening           */
/* ------------------------------------------------------------------------ */
static double tnorm(const double a[6]) {
  return sqrt(a[XX] * a[XX] + a[YY] * a[YY] + a[ZZ] * a[ZZ] +
              2.0 * (a[XY] * a[XY] + a[XZ] * a[XZ] + a[YZ] * a[YZ]));
}

/* e_tr: trial elastic strain (6 comps).  Returns the plastic multiplier
 * increment (0 if elastic) and the flow direction n = dev / |dev|. */
void or_return_map(const or_params *p, double G, const double e_tr[6], double epsP_n,
                   double dl_out[1], double n_out[6]) {
  double tr = e_tr[XX] + e_tr[YY] + e_tr[ZZ];
  double s[6];
  for (int a = 0; a < 6; ++a) s[a] = 2.0 * G * e_tr[a];
  for (int a = 0; a < 3; ++a) s[a] -= 2.0 * G * tr / 3.0;
  double ns = tnorm(s);
  double ftr = ns - sqrt(2.0 / 3.0) * (p->sigY + p->Hhard * epsP_n);
  dl_out[0] = 0.0;
  for (int a = 0; a < 6; ++a) n_out[a] = 0.0;
  if (ftr > 0.0) {
    dl_out[0] = ftr / (2.0 * G + sqrt(2.0 / 3.0) * p->Hhard);
    for (int a = 0; a < 6; ++a) n_out[a] = s[a] / ns;
  }
}

/* ------------------------------------------------------------------------ */
/* Local driving forces d psi / d phi_f and d psi / d phi_w [Eq. 33] with the */
/* elastic part obtained by differentiating the small-strain energy           */
/* d_T sum_a h(phi_a) (K_a tr^2 / 2 + G_a |dev|^2), eps_e = ebar - eT I - eps_p */
/* ------------------------------------------------------------------------ */
static void elastic_strain(const local_t *L, const double ebar[6], const double epsp[6], double e[6]) {
  for (int a = 0; a < 6; ++a) e[a] = ebar[a] - epsp[a];
  for (int a = 0; a < 3; ++a) e[a] -= L->eT;
}

static void mech_force(const or_params *p, const local_t *L, const double e[6], double *gf, double *gw,
                       double *vm) {
  double tr = e[XX] + e[YY] + e[ZZ];
  double dv[6];
  for (int a = 0; a < 6; ++a) dv[a] = e[a];
  for (int a = 0; a < 3; ++a) dv[a] -= tr / 3.0;
  double nd = tnorm(dv);
  double pel[3];
  for (int a = 0; a < 3; ++a) pel[a] = 0.5 * p->K[a] * tr * tr + p->G[a] * nd * nd;
  double phi_el = L->h[0] * pel[0] + L->h[1] * pel[1] + L->h[2] * pel[2];
  double trs = 3.0 * L->K * tr;
  *gf = L->dTp * phi_el + L->dT * (L->dh[0] * pel[0] - L->dh[1] * pel[1]) - L->eTp * trs;
  *gw = L->dT * (L->dh[2] * pel[2] - L->dh[1] * pel[1]);
  if (vm) *vm = sqrt(1.5) * 2.0 * L->G * nd;
}

void or_driving_force(const or_config *c, const or_params *p, double phi_f, double phi_w, double xO,
                      const double ebar[6], const double epsp[6], double g_out[2]) {
  local_t L;
  local_eval(p, phi_f, phi_w, xO, &L);
  double gf = p->w[0] * L.dm[0] - p->w[1] * L.dm[1];
  double gw = p->w[2] * L.dm[2] - p->w[1] * L.dm[1];
  if (c->chem_phase) {
    gf += L.dh[0] * L.psi[0] - L.dh[1] * L.psi[1];
    gw += L.dh[2] * L.psi[2] - L.dh[1] * L.psi[1];
  }
  if (c->mechanics) {
    double e[6], mf, mw;
    elastic_strain(&L, ebar, epsp, e);
    mech_force(p, &L, e, &mf, &mw, NULL);
    gf += mf;
    gw += mw;
  }
  g_out[0] = gf;
  g_out[1] = gw;
}

/* Local energy density: out[0] = chemical + barrier [Eq. 6, Eq. 7 first sum],
 * out[1] = elastic d_T sum h (K_a tr^2/2 + G_a |dev|^2) at a point. */
void or_point_energy(const or_config *c, const or_params *p, double phi_f, double phi_w, double xO,
                     const double ebar[6], const double epsp[6], double out[2]) {
  local_t L;
  local_eval(p, phi_f, phi_w, xO, &L);
  double e0 = 0.0;
  for (int a = 0; a < 3; ++a) e0 += (c->chem_phase ? L.h[a] * L.psi[a] : 0.0) + L.m[a] * p->w[a];
  out[0] = e0;
  out[1] = 0.0;
  if (c->mechanics) {
    double e[6];
    elastic_strain(&L, ebar, epsp, e);
    double tr = e[XX] + e[YY] + e[ZZ];
    double dv[6];
    for (int a = 0; a < 6; ++a) dv[a] = e[a];
    for (int a = 0; a < 3; ++a) dv[a] -= tr / 3.0;
    double nd = tnorm(dv);
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += L.h[a] * (0.5 * p->K[a] * tr * tr + p->G[a] * nd * nd);
    out[1] = L.dT * s;
  }
}

/* ------------------------------------------------------------------------ */
/* Discrete energies                                                          */
/* ------------------------------------------------------------------------ */
double or_elastic_energy(const or_config *c, const or_params *p, const or_state *st) {
  long n = ncell(c);
  double *eT = malloc(n * sizeof(double)), *K = malloc(n * sizeof(double)), *G = malloc(n * sizeof(double));
  eigen_arrays(c, p, st->phi_f, st->phi_w, eT, K, G);
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double ih = 1.0 / c->h, E = 0.0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long q = CI(c, i, j, k);
        double e[3];
        e[0] = (st->ux[XI(c, i + 1, j, k)] - st->ux[XI(c, i, j, k)]) * ih;
        e[1] = (st->uy[YI(c, i, j + 1, k)] - st->uy[YI(c, i, j, k)]) * ih;
        e[2] = c->dim == 3 ? (st->uz[ZI(c, i, j, k + 1)] - st->uz[ZI(c, i, j, k)]) * ih : 0.0;
        for (int d = 0; d < 3; ++d) e[d] -= eT[q] + st->epsp[d * n + q];
        double tr = e[0] + e[1] + e[2];
        double dd = 0.0;
        for (int d = 0; d < 3; ++d) dd += (e[d] - tr / 3.0) * (e[d] - tr / 3.0);
        E += 0.5 * K[q] * tr * tr + G[q] * dd;
      }
  for (int k = 0; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) {
        double v = exy_u(c, st->ux, st->uy, i, j, k) - edge_mean_xy(c, st->epsp + XY * n, i, j, k);
        E += 2.0 * edge_mean_xy(c, G, i, j, k) * v * v;
      }
  if (c->dim == 3) {
    for (int k = 1; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
          double v = exz_u(c, st->ux, st->uz, i, j, k) - edge_mean_xz(c, st->epsp + XZ * n, i, j, k);
          E += 2.0 * edge_mean_xz(c, G, i, j, k) * v * v;
        }
    for (int k = 1; k < nz; ++k)
      for (int j = 1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double v = eyz_u(c, st->uy, st->uz, i, j, k) - edge_mean_yz(c, st->epsp + YZ * n, i, j, k);
          E += 2.0 * edge_mean_yz(c, G, i, j, k) * v * v;
        }
  }
  free(eT); free(K); free(G);
  return E * pow(c->h, c->dim);
}

/* Total free energy: bulk chemical + barrier per cell, gradient energies on
 * interior faces [Eq. 7], plus the elastic energy when mechanics is on. */
double or_energy(const or_config *c, const or_params *p, const or_state *st) {
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double E = 0.0, ih = 1.0 / c->h;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long q = CI(c, i, j, k);
        local_t L;
        local_eval(p, st->phi_f[q], st->phi_w[q], st->xO[q], &L);
        double e0 = 0.0;
        for (int a = 0; a < 3; ++a) e0 += (c->chem_phase ? L.h[a] * L.psi[a] : 0.0) + L.m[a] * p->w[a];
        E += e0;
        int nb[3][3] = {{i + 1, j, k}, {i, j + 1, k}, {i, j, k + 1}};
        int lim[3] = {nx, ny, nz};
        int cc[3] = {i, j, k};
        for (int d = 0; d < c->dim; ++d) {
          if (cc[d] + 1 >= lim[d]) continue;
          long r = CI(c, nb[d][0], nb[d][1], nb[d][2]);
          double df = (st->phi_f[r] - st->phi_f[q]) * ih;
          double dw = (st->phi_w[r] - st->phi_w[q]) * ih;
          double dg = -df - dw;
          double dx = (st->xO[r] - st->xO[q]) * ih;
          E += 0.5 * (p->eps[0] * df * df + p->eps[1] * dg * dg + p->eps[2] * dw * dw) + 0.5 * p->kappaO * dx * dx;
        }
      }
  E *= pow(c->h, c->dim);
  if (c->mechanics) E += or_elastic_energy(c, p, st);
  return E;
}

/* ------------------------------------------------------------------------ */
/* Ledger                                                                     */
/* ------------------------------------------------------------------------ */
static void totals(const or_config *c, const or_state *s, double *O, double *H, double *xs) {
  long n = ncell(c);
  double o = 0.0, hh = 0.0, x = 0.0;
  for (long q = 0; q < n; ++q) {
    o += s->xO[q] + s->xW[q];
    hh += s->xH[q] + 2.0 * s->xW[q];
    x += s->xO[q];
  }
  double v = pow(c->h, c->dim);
  *O = o * v;
  *H = hh * v;
  *xs = x;
}

int or_ledger_init(const or_config *c, const or_params *p, const or_state *s, or_ledger *lg) {
  (void)p;
  totals(c, s, &lg->O_tot0, &lg->H_tot0, &lg->xO_sum0);
  lg->O_out = 0.0;
  lg->H_out = 0.0;
  lg->step = 0;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One explicit time step                                                     */
/* ------------------------------------------------------------------------ */
/* Flux through the face between cell "a" (lower coordinate) and "b": positive
 * along the axis.  Called with the same argument order from both sides so
 * that the face flux is bitwise identical for the two cells it couples. */
static double face_flux(double ca, double cb, double va, double vb, double h) {
  return -0.5 * (ca + cb) * (vb - va) / h;
}

/* The order parameters lie in [0, 1] (Sec. 2.2) and phi_g = 1 - phi_f - phi_w.
 * After the explicit update the triple (phi_f, phi_g, phi_w) is replaced by its
 * Euclidean projection onto {phi_a >= 0, sum_a phi_a = 1}, by the sort-based
 * algorithm of Held, Wolfe and Crowder (1974): sort descending, find the
 * largest rho with s_rho > (s_1 + ... + s_rho - 1) / rho, shift every entry by
 * that threshold and clip at zero.  A triple already inside is left as is. */
void or_simplex_project(double *phi_f, double *phi_w) {
  double u[3] = {*phi_f, 1.0 - *phi_f - *phi_w, *phi_w};
  if (u[0] >= 0.0 && u[1] >= 0.0 && u[2] >= 0.0) return;
  double srt[3] = {u[0], u[1], u[2]};
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (srt[b] > srt[a]) {
        double t = srt[a];
        srt[a] = srt[b];
        srt[b] = t;
      }
  double cum = 0.0, theta = 0.0;
  for (int j = 0; j < 3; ++j) {
    cum += srt[j];
    double t = (cum - 1.0) / (double)(j + 1);
    if (srt[j] - t > 0.0) theta = t;
  }
  *phi_f = fmax(u[0] - theta, 0.0);
  *phi_w = fmax(u[2] - theta, 0.0);
}

/* Linearly implicit Euler for one species.  The increment d of a step
 * solves (I + dt A) d = t, where t = dt T(x^n) is the explicit increment (the
 * full fluxes and reaction at x^n) and A = -div(D grad .) is the linear part
 * of the species' diffusion with the two-cell mean D at interior faces and,
 * where `dirichlet` is set, the half-cell boundary faces (D of the cell,
 * distance h/2).  Backward Euler for the stiff diffusion (Sec. 2.4 uses
 * backward Euler for the species), explicit for the rest.  Plain
 * Jacobi-preconditioned CG from d = 0 to ||t - (I + dt A) d|| <= 1e-13 ||t||,
 * sums in lexicographic order. */
static void species_op(const or_config *c, const double *D, int dirichlet, const double *v, double *out) {
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double ih2 = 1.0 / (c->h * c->h), dt = c->dt;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long q = CI(c, i, j, k);
        int cc[3] = {i, j, k}, lim[3] = {nx, ny, nz};
        double a = 0.0;
        for (int d = 0; d < c->dim; ++d)
          for (int side = -1; side <= 1; side += 2) {
            int nb[3] = {i, j, k};
            nb[d] += side;
            if (nb[d] < 0 || nb[d] >= lim[d]) {
              if (dirichlet) a += 2.0 * D[q] * v[q] * ih2;
              continue;
            }
            long r = CI(c, nb[0], nb[1], nb[2]);
            a -= 0.5 * (D[q] + D[r]) * (v[r] - v[q]) * ih2;
          }
        (void)cc;
        out[q] = v[q] + dt * a;
      }
}

static int species_solve(const or_config *c, const double *D, int dirichlet, const double *t, double *d) {
  long n = ncell(c);
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double ih2 = 1.0 / (c->h * c->h), dt = c->dt;
  double *dg = malloc(n * sizeof(double)), *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
  double *pv = malloc(n * sizeof(double)), *qv = malloc(n * sizeof(double));
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long q = CI(c, i, j, k);
        int lim[3] = {nx, ny, nz};
        double a = 0.0;
        for (int dd = 0; dd < c->dim; ++dd)
          for (int side = -1; side <= 1; side += 2) {
            int nb[3] = {i, j, k};
            nb[dd] += side;
            if (nb[dd] < 0 || nb[dd] >= lim[dd]) {
              if (dirichlet) a += 2.0 * D[q] * ih2;
              continue;
            }
            a += 0.5 * (D[q] + D[CI(c, nb[0], nb[1], nb[2])]) * ih2;
          }
        dg[q] = 1.0 / (1.0 + dt * a);
      }
  double tt = dot3(t, t, n);
  for (long q = 0; q < n; ++q) {
    d[q] = 0.0;
    r[q] = t[q];
    z[q] = dg[q] * r[q];
    pv[q] = z[q];
  }
  int status = OR_OK;
  if (tt > 0.0) {
    double rz = dot3(r, z, n);
    int it = 0;
    while (dot3(r, r, n) > 1e-26 * tt) {
      if (++it > 100000) { status = OR_CG_NOT_CONVERGED; break; }
      species_op(c, D, dirichlet, pv, qv);
      double alpha = rz / dot3(pv, qv, n);
      for (long q = 0; q < n; ++q) {
        d[q] += alpha * pv[q];
        r[q] -= alpha * qv[q];
        z[q] = dg[q] * r[q];
      }
      double rz1 = dot3(r, z, n);
      double beta = rz1 / rz;
      rz = rz1;
      for (long q = 0; q < n; ++q) pv[q] = z[q] + beta * pv[q];
    }
  }
  free(dg); free(r); free(z); free(pv); free(qv);
  return status;
}

/* The reaction of Eq. 27, 28 alone over a time t in one cell, with m(phi_g)
 * frozen: a = x_O obeys a' = -k m a (2a + c) with c = x_H - 2 x_O constant,
 * solved exactly:  a(t) = c a0 / ((2 a0 + c) e^(c k m t) - 2 a0) = a0 / D with
 * D = e^x + 2 a0 k m t g(x), x = c k m t, g(x) = (e^x - 1)/x, which holds for
 * every sign of c (and c = 0).  Since D - 1 = k m t x_H g(x), the amount
 * reacted is a0 - a = a0 k m t x_H g(x) / D, formed without cancellation.
 * None when x_O or x_H is not positive or the cell is full of water. */
double or_reaction_exact(const or_params *p, double m, double xO, double xH, double xW, double t) {
  if (!(xW < 1.0) || !(xO > 0.0) || !(xH > 0.0) || !(m > 0.0)) return 0.0;
  double kmt = p->kfor * m * t;
  double c = xH - 2.0 * xO;
  double x = c * kmt;
  double g = fabs(x) < 1e-8 ? 1.0 + x * (0.5 + x / 6.0) : expm1(x) / x;
  if (x > 700.0) return xO;                       /* e^x overflows: everything reacted to double precision */
  double dm1 = kmt * xH * g;
  return xO * dm1 / (1.0 + dm1);
}

int or_step(const or_config *c, const or_params *p, or_state *s, or_ledger *lg, or_stats *st) {
  if (c->dim != 2 && c->dim != 3) return OR_INVALID;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1 || (c->dim == 2 && c->nz != 1)) return OR_INVALID;
  long n = ncell(c);
  int nc = ncomp(c);
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double h = c->h, dt = c->dt, ih2 = 1.0 / (h * h);
  int status = OR_OK;
  or_stats loc;
  memset(&loc, 0, sizeof(loc));

  /* (1) mechanical equilibrium with phi^n, eps_p^n */
  if (c->mechanics) status = or_mech_solve(c, p, s, &loc);

  double *mu = malloc(n * sizeof(double)), *MO = malloc(n * sizeof(double));
  double *DH = malloc(n * sizeof(double)), *DW = malloc(n * sizeof(double));
  double *gf = malloc(n * sizeof(double)), *gw = malloc(n * sizeof(double));
  double *vm = calloc(n, sizeof(double));
  double *epsp_new = malloc((long)nc * n * sizeof(double)), *epsP_new = malloc(n * sizeof(double));
  memcpy(epsp_new, s->epsp, (long)nc * n * sizeof(double));
  memcpy(epsP_new, s->epsP, n * sizeof(double));

  /* (2) per cell: return map, elastic driving force, local chemistry */
#pragma omp parallel for collapse(2)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long q = CI(c, i, j, k);
        local_t L;
        local_eval(p, s->phi_f[q], s->phi_w[q], s->xO[q], &L);
        double g_f = p->w[0] * L.dm[0] - p->w[1] * L.dm[1];
        double g_w = p->w[2] * L.dm[2] - p->w[1] * L.dm[1];
        if (c->chem_phase) {
          g_f += L.dh[0] * L.psi[0] - L.dh[1] * L.psi[1];
          g_w += L.dh[2] * L.psi[2] - L.dh[1] * L.psi[1];
        }
        if (c->mechanics) {
          double ebar[6], ep[6] = {0, 0, 0, 0, 0, 0}, e[6];
          or_cell_strain(c, s->ux, s->uy, s->uz, i, j, k, ebar);
          for (int a = 0; a < nc; ++a) ep[a] = s->epsp[(long)a * n + q];
          if (c->plasticity) {
            double etr[6], dl, nn[6];
            elastic_strain(&L, ebar, ep, etr);
            or_return_map(p, L.G, etr, s->epsP[q], &dl, nn);
            if (dl > 0.0) {
              for (int a = 0; a < nc; ++a) {
                ep[a] += dl * nn[a];
                epsp_new[(long)a * n + q] = ep[a];
              }
              epsP_new[q] = s->epsP[q] + dl;
            }
          }
          double mf, mw;
          elastic_strain(&L, ebar, ep, e);
          mech_force(p, &L, e, &mf, &mw, &vm[q]);
          g_f += mf;
          g_w += mw;
        }
        if (c->gext) {
          g_f += c->gext[q];
          g_w += c->gext[n + q];
        }
        gf[q] = g_f;
        gw[q] = g_w;
        MO[q] = L.MO;
        DH[q] = L.DH;
        DW[q] = L.DW;
        /* mu_O = d psi_che / d x_O - kappa_O lap x_O, mirror (no-flux) ghosts */
        double lap = 0.0;
        int cc[3] = {i, j, k}, lim[3] = {nx, ny, nz};
        for (int d = 0; d < c->dim; ++d) {
          int lo[3] = {i, j, k}, hi[3] = {i, j, k};
          lo[d] = cc[d] > 0 ? cc[d] - 1 : cc[d];
          hi[d] = cc[d] + 1 < lim[d] ? cc[d] + 1 : cc[d];
          lap += (s->xO[CI(c, hi[0], hi[1], hi[2])] - s->xO[q]) - (s->xO[q] - s->xO[CI(c, lo[0], lo[1], lo[2])]);
        }
        mu[q] = L.mu_loc - p->kappaO * lap * ih2;
      }

  /* (3) explicit update of the five fields */
  double *nf_ = malloc(n * sizeof(double)), *nw_ = malloc(n * sizeof(double));
  double *nO = malloc(n * sizeof(double)), *nH = malloc(n * sizeof(double)), *nW = malloc(n * sizeof(double));
#pragma omp parallel for collapse(2)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long q = CI(c, i, j, k);
        int cc[3] = {i, j, k}, lim[3] = {nx, ny, nz};
        double lf = 0.0, lw = 0.0, divO = 0.0, divH = 0.0, divW = 0.0;
        for (int d = 0; d < c->dim; ++d) {
          int lo[3] = {i, j, k}, hi[3] = {i, j, k};
          int has_lo = cc[d] > 0, has_hi = cc[d] + 1 < lim[d];
          lo[d] = has_lo ? cc[d] - 1 : cc[d];
          hi[d] = has_hi ? cc[d] + 1 : cc[d];
          long ql = CI(c, lo[0], lo[1], lo[2]), qh = CI(c, hi[0], hi[1], hi[2]);
          lf += (s->phi_f[qh] - s->phi_f[q]) - (s->phi_f[q] - s->phi_f[ql]);
          lw += (s->phi_w[qh] - s->phi_w[q]) - (s->phi_w[q] - s->phi_w[ql]);
          double JOm, JOp, JHm, JHp, JWm, JWp;
          if (has_lo) {
            JOm = face_flux(MO[ql], MO[q], mu[ql], mu[q], h);
            JHm = face_flux(DH[ql], DH[q], s->xH[ql], s->xH[q], h);
            JWm = face_flux(DW[ql], DW[q], s->xW[ql], s->xW[q], h);
          } else {
            JOm = 0.0;
            JHm = c->dirichlet ? -DH[q] * (s->xH[q] - p->xH_bc) / (0.5 * h) : 0.0;
            JWm = c->dirichlet ? -DW[q] * (s->xW[q] - p->xW_bc) / (0.5 * h) : 0.0;
          }
          if (has_hi) {
            JOp = face_flux(MO[q], MO[qh], mu[q], mu[qh], h);
            JHp = face_flux(DH[q], DH[qh], s->xH[q], s->xH[qh], h);
            JWp = face_flux(DW[q], DW[qh], s->xW[q], s->xW[qh], h);
          } else {
            JOp = 0.0;
            JHp = c->dirichlet ? -DH[q] * (p->xH_bc - s->xH[q]) / (0.5 * h) : 0.0;
            JWp = c->dirichlet ? -DW[q] * (p->xW_bc - s->xW[q]) / (0.5 * h) : 0.0;
          }
          divO += (JOp - JOm) / h;
          divH += (JHp - JHm) / h;
          divW += (JWp - JWm) / h;
        }
        lf *= ih2;
        lw *= ih2;
        local_t L;
        local_eval(p, s->phi_f[q], s->phi_w[q], s->xO[q], &L);
        /* Eq. 27, 28: forward rate k_for m(phi_g) x_O x_H, zero where the cell
         * is full of water; mole fractions below zero (the variational O flux
         * leaves the gas slightly below x_O = 0) take no part in it */
        double r = s->xW[q] < 1.0 ? L.m[1] * p->kfor * fmax(s->xO[q], 0.0) * fmax(s->xH[q], 0.0) : 0.0;
        if (c->species_implicit == 2) r = 0.0;        /* the reaction follows the transport below */
        nf_[q] = s->phi_f[q] + dt * p->L[0] * ((p->eps[0] + p->eps[1]) * lf + p->eps[1] * lw - gf[q]);
        nw_[q] = s->phi_w[q] + dt * p->L[2] * ((p->eps[2] + p->eps[1]) * lw + p->eps[1] * lf - gw[q]);
        or_simplex_project(&nf_[q], &nw_[q]);
        /* the explicit increments of the species; added below (explicit) or
         * taken as the right-hand sides of the implicit solves */
        nO[q] = dt * (-divO - r);
        nH[q] = dt * (-divH - 2.0 * r);
        nW[q] = dt * (-divW + r);
      }

  if (c->species_implicit) {
    double *DO = malloc(n * sizeof(double)), *dx = malloc(n * sizeof(double));
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          long q = CI(c, i, j, k);
          local_t L;
          local_eval(p, s->phi_f[q], s->phi_w[q], s->xO[q], &L);
          DO[q] = L.DO;
        }
    double *tx[3] = {nO, nH, nW};
    const double *Dc[3] = {DO, DH, DW};
    for (int sp = 0; sp < 3; ++sp) {
      int rc = species_solve(c, Dc[sp], sp > 0 && c->dirichlet, tx[sp], dx);
      if (rc != OR_OK) status = rc;
      memcpy(tx[sp], dx, n * sizeof(double));
    }
    free(DO); free(dx);
  }
  for (long q = 0; q < n; ++q) {
    nO[q] += s->xO[q];
    nH[q] += s->xH[q];
    nW[q] += s->xW[q];
  }
  if (c->species_implicit == 2) {
    /* the reaction over dt after the transport, exactly per cell, m at phi^n */
    for (long q = 0; q < n; ++q) {
      double g = 1.0 - s->phi_f[q] - s->phi_w[q];
      double R = or_reaction_exact(p, mfun(p, g), nO[q], nH[q], nW[q], dt);
      nO[q] -= R;
      nH[q] -= 2.0 * R;
      nW[q] += R;
    }
  }

  /* (4) boundary outflux for the ledger (lexicographic over faces) */
  double outO = 0.0, outH = 0.0;
  if (c->dirichlet) {
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          long q = CI(c, i, j, k);
          int cc[3] = {i, j, k}, lim[3] = {nx, ny, nz};
          for (int d = 0; d < c->dim; ++d) {
            int nb = (cc[d] == 0) + (cc[d] == lim[d] - 1);   /* boundary faces of this cell on axis d */
            if (!nb) continue;
            /* outward flux, with the values the update used at the face: x^n
             * (explicit) or x^(n+1) (implicit) */
            double xw = c->species_implicit ? nW[q] : s->xW[q], xh = c->species_implicit ? nH[q] : s->xH[q];
            double jw = 2.0 * DW[q] * (xw - p->xW_bc) / h;
            double jh = 2.0 * DH[q] * (xh - p->xH_bc) / h;
            outO += nb * jw;
            outH += nb * (jh + 2.0 * jw);
          }
        }
  }
  double area = pow(h, c->dim - 1);
  lg->O_out += dt * area * outO;
  lg->H_out += dt * area * outH;
  lg->step += 1;

  memcpy(s->phi_f, nf_, n * sizeof(double));
  memcpy(s->phi_w, nw_, n * sizeof(double));
  memcpy(s->xO, nO, n * sizeof(double));
  memcpy(s->xH, nH, n * sizeof(double));
  memcpy(s->xW, nW, n * sizeof(double));
  memcpy(s->epsp, epsp_new, (long)nc * n * sizeof(double));
  memcpy(s->epsP, epsP_new, n * sizeof(double));

  if (st) {
    double O, H, xs;
    totals(c, s, &O, &H, &xs);
    *st = loc;
    st->O_tot = O;
    st->O_out = lg->O_out;
    st->O_drift = (O + lg->O_out - lg->O_tot0) / lg->O_tot0;
    st->H_tot = H;
    st->H_out = lg->H_out;
    st->H_drift = (H + lg->H_out - lg->H_tot0) / lg->H_tot0;
    st->red_degree = lg->xO_sum0 != 0.0 ? 1.0 - xs / lg->xO_sum0 : 0.0;
    double mv = 0.0, me = 0.0;
    for (long q = 0; q < n; ++q) {
      if (vm[q] > mv) mv = vm[q];
      if (s->epsP[q] > me) me = s->epsP[q];
    }
    st->max_vm = mv;
    st->max_epsP = me;
  }
  free(mu); free(MO); free(DH); free(DW); free(gf); free(gw); free(vm);
  free(epsp_new); free(epsP_new); free(nf_); free(nw_); free(nO); free(nH); free(nW);
  return status;
}
