/* FP64 CPU oracle of the chemo-mechanical phase-field step (Bai et al.,
 * "Chemo-Mechanical Phase-Field Modeling of Iron Oxide Reduction with
 * Hydrogen", arXiv:2111.11538).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path; only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * Layouts are compact and x fastest.  Cells: [nz][ny][nx].  Staggered
 * displacement faces: ux [nz][ny][nx+1], uy [nz][ny+1][nx], uz [nz+1][ny][nx]
 * (2D: nz = 1 and uz unused).  Plastic strain: component-major, components
 * xx, yy, zz, xy (2D, plane strain) or xx, yy, zz, xy, xz, yz (3D).
 */
#ifndef PF_ORACLE_H
#define PF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Phase order everywhere: 0 ferrite (f), 1 gas (g), 2 wuestite (w). */
typedef struct {
  double R, theta, Vmol;
  double w[3], eps[3], L[3];
  double kappaO;
  double K[3], G[3];
  double sigY, Hhard;
  double DO[3], DH[3], DW[3];
  double kfor;
  double Omega_f;
  double xH_bc, xW_bc;
  int m_form;          /* 0: m = 16 x^2 (1-x)^2 ; 1: m = x^2 (1-x)^2 */
  int pad_;
} or_params;

typedef struct {
  int dim, nx, ny, nz;
  double h, dt;
  int mechanics;       /* elastic energy on (1) or off (0) */
  int plasticity;      /* J2 return map on (1) or off (0) */
  int dirichlet;       /* species Dirichlet faces (x_H, x_H2O) on all outer faces */
  int chem_phase;      /* chemical energy drives the phase fields (1, the model) */
  double cg_rtol;
  int cg_max_iter;
  int species_implicit; /* 0: explicit Euler for the species; 1: linearly implicit Euler (or_step);
                           2: as 1 for the transport, then the reaction over dt solved exactly per cell */
  const double *gext;   /* nullable: [2][ncell] mechanical driving forces d psi / d phi_f, d psi / d phi_w
                           from outside (the finite-strain mechanics), added to those of the phase fields */
} or_config;

typedef struct {
  double *phi_f, *phi_w, *xO, *xH, *xW;
  double *ux, *uy, *uz;
  double *epsp;        /* NC * ncell, component-major */
  double *epsP;        /* accumulated plastic strain */
} or_state;

typedef struct {
  double O_tot0, O_out, H_tot0, H_out, xO_sum0;
  long step;
} or_ledger;

typedef struct {
  int cg_iters, pad_;
  double cg_rel_resid;
  double O_tot, O_out, O_drift, H_tot, H_out, H_drift;
  double red_degree, max_vm, max_epsP;
} or_stats;

/* status codes */
#define OR_OK 0
#define OR_CG_NOT_CONVERGED 1
#define OR_INVALID 2

int  or_ledger_init(const or_config *c, const or_params *p, const or_state *s, or_ledger *lg);
int  or_step(const or_config *c, const or_params *p, or_state *s, or_ledger *lg, or_stats *st);
int  or_mech_solve(const or_config *c, const or_params *p, or_state *s, or_stats *st);

/* pieces exported for the pins */
void or_moduli(const or_config *c, const or_params *p, const double *phi_f, const double *phi_w,
               double *K, double *G);
void or_apply(const or_config *c, const double *K, const double *G,
              const double *ux, const double *uy, const double *uz,
              double *qx, double *qy, double *qz);
void or_rhs(const or_config *c, const or_params *p, const or_state *s,
            double *bx, double *by, double *bz);
void or_diag(const or_config *c, const double *K, const double *G,
             double *dx, double *dy, double *dz);
void or_cell_strain(const or_config *c, const double *ux, const double *uy, const double *uz,
                    int i, int j, int k, double e[6]);
void or_local(const or_params *p, double phi_f, double phi_w, double xO, double out[16]);
void or_return_map(const or_params *p, double G, const double e_tr[6], double epsP_n,
                   double dl_out[1], double n_out[6]);
void or_driving_force(const or_config *c, const or_params *p, double phi_f, double phi_w, double xO,
                      const double ebar[6], const double epsp[6], double g_out[2]);
void or_point_energy(const or_config *c, const or_params *p, double phi_f, double phi_w, double xO,
                     const double ebar[6], const double epsp[6], double out[2]);
double or_energy(const or_config *c, const or_params *p, const or_state *s);
double or_elastic_energy(const or_config *c, const or_params *p, const or_state *s);
int  or_common_tangent(double *xf, double *xw, double *resid);
void or_simplex_project(double *phi_f, double *phi_w);
double or_reaction_exact(const or_params *p, double m, double xO, double xH, double xW, double t);
void or_fe(int phase, double x, double out[3]);

#ifdef __cplusplus
}
#endif
#endif
