/* pf.h -- C ABI of the MI355X (gfx950) library that advances the
 * chemo-mechanically coupled phase-field model of wuestite-to-iron reduction
 * by hydrogen (Bai, Mianroodi, Ma, Kwiatkowski da Silva, Svendsen, Raabe,
 * arXiv:2111.11538) on a regular 2D/3D voxel grid.
 *
 * One call of pf_step advances the unknowns of the model's field relations
 * (Section 2.4, Eq. 29): the phase fields phi_f, phi_w (Allen-Cahn, Eq. 29
 * rows 5-6 with Eq. 33), the species x_O, x_H, x_H2O (Eq. 29 rows 1-3 with
 * the variational O flux of Eq. 24, Eq. 30 and Section 3.2), the plastic
 * strain (J2 with linear hardening, Eq. 25 and Eq. 34) and the displacement
 * of the quasi-static momentum balance (Eq. 29 row 4), in a small-strain
 * reading of the kinematics (eigenstrain d_T^(1/3) - 1 from Eq. 9, moduli of
 * Eq. 32).  All arithmetic runs in the library's HIP kernels.
 *
 * Conventions shared by every entry point
 *  - Every function returns pf_status and never throws.  pf_last_error()
 *    gives a human-readable message for the last failure on a context.
 *  - Device memory is owned by the caller: pf_init receives one device
 *    workspace of pf_workspace_bytes() bytes (e.g. a torch uint8 tensor) and
 *    a HIP stream; the library carves all state out of it and never frees it.
 *    pf_destroy frees only host-side objects.
 *  - Calls on one context are stream-ordered on that stream and are not
 *    thread-safe; different contexts are independent.
 *  - Field exchange (pf_fields) always uses FP64, compact, x-fastest arrays:
 *    cells [nz][ny][nx] (2D: [ny][nx]); staggered displacement faces
 *    u_x [nz][ny][nx+1], u_y [nz][ny+1][nx], u_z [nz+1][ny][nx]; plastic
 *    strain component-major with components xx, yy, zz, xy (2D, plane strain)
 *    or xx, yy, zz, xy, xz, yz (3D).  Internally the library may hold the
 *    state in FP32 (PF_MIXED) and in a padded layout.
 *  - SI units throughout.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_ctx pf_ctx;

typedef enum {
  PF_OK = 0,
  PF_ERR_INVALID_ARG = 1,       /* bad pointer, size or configuration */
  PF_ERR_HIP = 2,               /* a HIP runtime call failed */
  PF_ERR_OOM = 3,               /* workspace smaller than pf_workspace_bytes() */
  PF_ERR_CG_NOT_CONVERGED = 4,  /* mechanics solve hit cg_max_iter */
  PF_ERR_NONFINITE = 5,         /* a NaN/Inf appeared in the fields */
  PF_ERR_LEDGER = 6,            /* oxygen ledger drift above ledger_tol */
  PF_ERR_BAD_STATE = 7,         /* context failed earlier; restore fields first */
  PF_ERR_UNSUPPORTED = 8
} pf_status;

typedef enum { PF_FP64 = 0, PF_MIXED = 1 } pf_precision;   /* MIXED: FP32 state and stencils, FP64 reductions */
typedef enum {
  PF_WARM_ZERO = 0,       /* each solve starts from u = 0 */
  PF_WARM_PREV = 1,       /* from the displacement of the previous solve */
  PF_WARM_LEARNED = 2     /* from the previous displacement plus the increment an attached
                             network predicts, when its residual is the smaller (3D only) */
} pf_warm;

typedef enum {
  PF_FIELD_PHI_F = 0, PF_FIELD_PHI_W = 1, PF_FIELD_XO = 2, PF_FIELD_XH = 3, PF_FIELD_XW = 4,
  PF_FIELD_UX = 5, PF_FIELD_UY = 6, PF_FIELD_UZ = 7,
  PF_FIELD_EPSP = 8,            /* plastic strain tensor, 4 (2D) or 6 (3D) components */
  PF_FIELD_EPSP_ACC = 9         /* accumulated plastic strain epsilon_P */
} pf_field;

typedef struct {
  int dim;                /* 2 (plane strain) or 3 */
  int nx, ny, nz;         /* cells; nz must be 1 when dim == 2; each >= 1 */
  double h;               /* cell size (m) */
  double dt;              /* explicit time step (s) */
  int precision;          /* pf_precision */
  int mechanics;          /* 1: elastic energy, eigenstrain and the equilibrium solve are on */
  int plasticity;         /* 1: J2 return map after each solve */
  int dirichlet;          /* 1: x_H = xH_bc and x_H2O = xW_bc on every outer face; 0: closed box */
  int chem_phase;         /* 1 (the model): chemical energy drives the phase fields */
  double cg_rtol;         /* stop when ||b - A u|| <= cg_rtol ||b|| */
  int cg_max_iter;        /* reaching it is an error */
  int warm;               /* pf_warm: start of each step's solve */
  double ledger_tol;      /* |O drift| above this raises PF_ERR_LEDGER; <= 0 disables */
  int species_implicit;   /* 0: explicit Euler for x_O, x_H, x_H2O; 1: linearly implicit Euler (see pf_step);
                             2: as 1 without the reaction, then the reaction over dt solved exactly per cell */
  int species_max_iter;   /* implicit species: CG iteration limit per step (reaching it is an error) */
  double species_rtol;    /* implicit species: stop each species' CG at ||r|| <= species_rtol ||b|| */
  int cg_precond;         /* preconditioner of the equilibrium CG: 0 Jacobi; 1 a geometric multigrid V-cycle
                             (levels halve the cells, an odd side n to (n + 1) / 2, while every side is above 8;
                             Jacobi smoothing with Chebyshev steps; see pf_step).  Batches take 0 only. */
} pf_config;

/* Material and model parameters, Table 1 of the paper; phase index 0 ferrite,
 * 1 gas, 2 wuestite. */
typedef struct {
  double R, theta, Vmol;  /* gas constant, temperature, molar volume */
  double w[3];            /* barrier heights w_a (J/m^3) */
  double eps[3];          /* phase gradient energy coefficients (J/m) */
  double L[3];            /* phase mobilities (m^3/(J s)) */
  double kappaO;          /* oxygen gradient energy coefficient (J/m) */
  double K[3], G[3];      /* bulk and shear moduli (Pa) */
  double sigY, Hhard;     /* yield stress and linear hardening modulus (Pa) */
  double DO[3], DH[3], DW[3];   /* diffusivities of O, H, H2O per phase (m^2/s) */
  double kfor;            /* forward reaction constant (1/s) */
  double Omega_f;         /* relative volume decrease of the transformation */
  double xH_bc, xW_bc;    /* boundary values of x_H and x_H2O */
  int m_form;             /* 0: m(x) = 16 x^2 (1-x)^2 ; 1: m(x) = x^2 (1-x)^2 */
  int pad_;
} pf_params;

typedef struct {
  int cg_iters;           /* CG iterations of the last solve */
  int warm_used;          /* pf_warm used by the last solve */
  double cg_rel_resid;    /* true ||b - A u|| / ||b|| after the last solve */
  double O_tot, O_out, O_drift;   /* h^d sum (x_O + x_H2O); cumulative outflux; relative drift */
  double H_tot, H_out, H_drift;   /* same for hydrogen, h^d sum (x_H + 2 x_H2O) */
  double red_degree;      /* reduction degree f = 1 - sum x_O / sum x_O(ledger reset), Eq. 39 */
  double max_vm;          /* largest cell von Mises stress after the return map (Pa) */
  double max_epsP;        /* largest accumulated plastic strain */
  long long step;         /* steps taken since pf_init */
  int nonfinite;          /* number of cells with a non-finite field value in the last step */
  int pad_;
  long long cg_iters_total;   /* CG iterations summed over every solve since pf_init */
  double r0_learned;      /* learned start: ||b - A u0|| / ||b|| of the network's start, 0 if not evaluated */
  double r0_prev;         /* learned start: the same for the previous displacement, 0 if not evaluated */
  int species_iters;      /* implicit species: the most CG iterations any species took in the last step */
  int pad2_;
} pf_step_stats;

/* Bytes of device workspace pf_init needs for this configuration (0 if the
 * configuration is invalid). */
size_t pf_workspace_bytes(const pf_config *cfg);

/* Create a context.  `workspace` is a device pointer (256-byte aligned) to at
 * least pf_workspace_bytes(cfg) bytes, owned by the caller and kept alive
 * until pf_destroy; `hip_stream` is a hipStream_t (NULL = default stream).
 * All fields start at zero; set them with pf_fields, then step.  The ledger
 * reference (initial O, H and x_O totals) is taken at the first pf_step after
 * any field was set, or by pf_ledger_reset. */
pf_status pf_init(const pf_config *cfg, const pf_params *params, void *workspace, size_t workspace_bytes,
                  void *hip_stream, pf_ctx **out);

/* Advance `nsteps` steps (Section 2.4 field relations; each step:
 * equilibrium solve with phi^n and eps_p^n, return map, driving forces,
 * fluxes and reaction, explicit Euler update, FP64 ledger).  With
 * species_implicit the species take a linearly implicit Euler step instead
 * (Sec. 2.4 uses backward Euler for them): the increment d of x_O, x_H and
 * x_H2O solves (I + dt A) d = dt T(x^n), T the explicit tendency (every flux
 * and the reaction at x^n), A = -div(D grad .) the species' diffusion with
 * the two-cell mean D at interior faces and, for x_H and x_H2O, the half-cell
 * Dirichlet faces; each species is solved by Jacobi-PCG to species_rtol.
 * This removes the gas-diffusion limit on dt; the phase fields stay
 * explicit.  With species_implicit == 2 the tendency leaves the reaction out
 * and, after the solve, each cell's reaction over dt (Eq. 27, 28 with
 * m(phi_g^n) frozen) is applied from the exact solution of its rate law,
 * which removes the reaction's limit on dt as well and keeps x_O + x_H2O and
 * x_H + 2 x_H2O of every cell unchanged.  With cg_precond == 1 the
 * equilibrium CG is preconditioned by one multigrid V-cycle per iteration:
 * coarse levels of half the cells (the same staggered operator at 2h with
 * the moduli averaged over the 8 (2D: 4) children), face transfers that are
 * full weighting along the normal and linear across it (restriction =
 * transposed prolongation / 4, in 2D / 2), two Jacobi sweeps with Chebyshev
 * steps before and after
 * each coarse correction and eight on the coarsest level (in 3D PF_MIXED the
 * sweeps read bf16 copies of each level's moduli and diagonal, which keeps
 * the cycle a fixed symmetric positive definite operator; CG itself keeps
 * the FP32 moduli); the solution is the same to cg_rtol, in far fewer
 * iterations.  The CG
 * recurrence scalars and the convergence test live on the device; the host
 * reads the convergence flag once per chunk of queued CG launches (a stream
 * synchronisation per chunk, see pf_cg_chunk: launches queued past
 * convergence exit at entry) and once at the end; `last` (nullable)
 * receives the stats of the last step.  In PF_MIXED the solve stops when the
 * recursive residual reaches cg_rtol; cg_rel_resid reports the true residual
 * recomputed afterwards, which for an FP32 iterate levels off near 1e-5.
 * After an error the context is in BAD_STATE until fields are set. */
pf_status pf_step(pf_ctx *ctx, int nsteps, pf_step_stats *last);

/* Solve only the mechanical equilibrium (Eq. 29 row 4) for the current phase
 * fields and plastic strain, starting from zero (PF_WARM_ZERO), from the
 * current displacement (PF_WARM_PREV) or from the learned start
 * (PF_WARM_LEARNED, contexts created with it only).  Fills cg_iters, warm_used and
 * cg_rel_resid of `stats` (nullable). */
pf_status pf_mech_solve(pf_ctx *ctx, int warm, pf_step_stats *stats);

/* CG launches queued between two convergence checks (each check synchronises
 * the stream).  n = 0 (the default) adapts the chunk to the iteration counts
 * of the last two solves; n >= 1 fixes it.  The results do not depend on it:
 * iterations queued past convergence exit at entry.  Errors: n < 0. */
pf_status pf_cg_chunk(pf_ctx *ctx, int n);

/* Copy one field between the context and caller memory.  dir 0: get (context
 * -> ptr), 1: set (ptr -> context).  ptr holds FP64 compact data (layouts
 * above) of exactly nbytes; ptr_is_device selects a device or host pointer.
 * Displacement values on the roller faces are forced to zero on set.
 * Stream-ordered; a get on a host pointer synchronises the stream. */
pf_status pf_fields(pf_ctx *ctx, int field_id, int dir, void *ptr, size_t nbytes, int ptr_is_device);

/* Take the current fields as the ledger reference (O, H and x_O totals) and
 * zero the cumulative boundary fluxes. */
pf_status pf_ledger_reset(pf_ctx *ctx);

/* Message of the last error on this context ("" if none); ctx may be NULL for
 * errors raised before a context existed. */
const char *pf_last_error(const pf_ctx *ctx);

/* Kernel classes reported by the timing interface. */
typedef enum {
  PF_K_APPLY = 0,     /* q = A p with the fused direction update (one per CG iteration) */
  PF_K_UPDATE = 1,    /* u, r, z update with FP64 partial dots (one per CG iteration) */
  PF_K_SOLVE_SETUP = 2, /* ||b||, initial residual / diagonal, true residual (three per solve) */
  PF_K_STEP = 3,      /* fused chemistry, phase-field and plasticity update (one per step) */
  PF_K_MU = 4,        /* oxygen chemical potential (one per step) */
  PF_K_OTHER = 5,     /* moduli, convergence checks, ledger (small kernels), and the
                         CG launches queued past convergence, which exit at once */
  PF_K_NN = 6,        /* the four convolutions of a learned-start inference (one group per solve) */
  PF_K_SPECIES = 7,   /* implicit species: set-up, apply, update and final update of their CG */
  PF_K_PRECOND = 8,   /* multigrid preconditioner: coarse-level smoothing, transfers, coarse moduli and
                         diagonals */
  PF_K_SMOOTH = 9,    /* multigrid preconditioner: the smoothing and residual sweeps on the solve's own grid
                         (four per cycle) */
  PF_K_COUNT = 10
} pf_kernel_kind;

/* Per-kernel timing with HIP events recorded on the context's stream around
 * the launches of the selected kinds.  kinds is a bit mask of
 * (1 << pf_kernel_kind) values (PF_TIMING_ALL selects every kind); a nonzero
 * mask clears the accumulators and starts recording, 0 stops.  Each recorded
 * launch costs a few microseconds of stream time and the stream is
 * synchronised once per solve while recording; leave it off, or restrict it
 * to one kind, for throughput runs.  The events are created without the
 * system-scope fence (hipEventDisableSystemFence), so that recording them
 * does not write back and invalidate the caches between kernels. */
#define PF_TIMING_ALL ((1 << PF_K_COUNT) - 1)
pf_status pf_timing(pf_ctx *ctx, int kinds);

/* Sampling of the CG kernels (PF_K_APPLY, PF_K_UPDATE and, with the
 * multigrid preconditioner, PF_K_PRECOND and PF_K_SMOOTH) while timing: only
 * the launches of every `every`-th CG iteration are timed, with the phase
 * advancing by one per solve (solve s times iterations i with (i + s) a
 * multiple of every), so that over many solves every iteration index is
 * sampled alike; the reported totals and launch counts cover that sample.
 * every >= 1 (1, the default, times all).  Other kinds are always timed in
 * full. */
pf_status pf_timing_every(pf_ctx *ctx, int every);

/* Accumulated device time (ms) and launch count of one pf_kernel_kind since
 * timing was enabled.  Synchronises the stream. */
pf_status pf_timing_get(pf_ctx *ctx, int kind, double *total_ms, long long *launches);

/* ------------------------------------------------------------------------ */
/* Batches: many uneven 2D instances advanced together.                      */
/* Each instance has its own grid, fields, CG recurrence (and convergence)   */
/* and ledger; one step of the whole batch is ONE persistent kernel launch   */
/* (moduli, right-hand side, the data-dependent CG loop of every instance,   */
/* return map, chemistry and ledger, separated by bounded grid barriers),    */
/* replayed from a hipGraph.  The caller's workspace holds every array and   */
/* the tile tables.                                                          */
/* ------------------------------------------------------------------------ */
typedef struct pf_batch pf_batch;

typedef struct { int nx, ny, nz; } pf_extent;   /* one instance's cells (2D: nz = 1) */

/* Work decomposition of a batch step (chosen by an autotuner):
 *  apply_rows     rows per CG apply strip (62 columns, one wave each) (4..256)
 *  update_chunk   16-byte vectors per CG-update work item (256..65536)
 *  blocks_per_cu  persistent blocks per compute unit (1..occupancy limit)
 *  spin_limit     polls before a grid barrier gives up and reports an error */
typedef struct {
  int apply_rows;
  int update_chunk;
  int blocks_per_cu;
  int pad_;
  long long spin_limit;
} pf_batch_tiles;

/* Workspace bytes for `count` instances (1..256) with the shared settings of
 * `cfg` (dim must be 2; cfg->nx/ny/nz are ignored); 0 if invalid. */
size_t pf_batch_workspace_bytes(const pf_config *cfg, const pf_extent *ext, int count);

/* Create a batch.  Same ownership rules as pf_init; every instance starts at
 * zero.  Requires dim == 2, mechanics == 1, warm == PF_WARM_PREV (the
 * first step of an instance starts its solve from u = 0) and explicit
 * species (species_implicit == 0; PF_ERR_UNSUPPORTED otherwise). */
pf_status pf_batch_init(const pf_config *cfg, const pf_params *params, const pf_extent *ext, int count,
                        void *workspace, size_t workspace_bytes, void *hip_stream, pf_batch **out);

/* Replace the work decomposition (rebuilds the tile tables and the graphs). */
pf_status pf_batch_set_tiles(pf_batch *b, const pf_batch_tiles *tiles);
pf_status pf_batch_get_tiles(const pf_batch *b, pf_batch_tiles *tiles);

/* pf_fields for instance `instance` of the batch (same layouts and rules). */
pf_status pf_batch_fields(pf_batch *b, int instance, int field_id, int dir, void *ptr, size_t nbytes,
                          int ptr_is_device);

/* Advance every instance `nsteps` steps, one graph launch per step; `stats`
 * (nullable) receives `count` entries for the last step.  Returns
 * PF_ERR_CG_NOT_CONVERGED if an instance's solve reached cg_max_iter (the
 * step is still taken with the last iterate), PF_ERR_NONFINITE /
 * PF_ERR_LEDGER as pf_step, PF_ERR_HIP if a grid barrier timed out. */
pf_status pf_batch_step(pf_batch *b, int nsteps, pf_step_stats *stats);

const char *pf_batch_last_error(const pf_batch *b);
void pf_batch_destroy(pf_batch *b);

/* ---------------------------------------------------------------------------
 * Learned warm start.  An extension of the method: the paper solves the
 * mechanical equilibrium (Eq. 29, last line) without any learned component.
 * A network of four 3x3x3 'same' convolutions (zero padding) with 6 -> 32 ->
 * 32 -> 32 -> 3 channels, ReLU between layers and a linear output, predicts
 * the displacement increment of the next solve; the CG residual decides
 * whether the solve starts from it or from the previous displacement.
 *
 * Tensors are device arrays, channel-last: voxel v of n volumes of D x H x W
 * voxels (x fastest), channel c at v * C + c.  Activations and inputs are
 * bfloat16 (uint16 bit patterns); the network output is FP32 with 4
 * channels (the 4th is zero).  The arithmetic is bf16 x bf16 products with
 * FP32 accumulation on the matrix cores.
 *
 * Inputs per voxel (8 channels, the last 2 zero): phi_f, phi_w,
 * (eps_T(phi_f) - eps_T(phi_f of the previous solve)) * 32 h / s and the
 * previous increment of u_x, u_y, u_z on the cell's low faces divided by s,
 * where eps_T = cbrt(1 - Omega_f h(phi_f)) - 1 (Eq. 9, small strain) and s is
 * the root mean square of the previous increment over the low faces of all
 * cells.  Output channel c times s is the predicted increment of the low
 * face of direction c (zero on the low boundary faces, fixed by the rollers).
 *
 * Parameters are one FP32 vector: per layer W[27][cout][cin] (tap
 * t = 9 (dz+1) + 3 (dy+1) + (dx+1) reads voxel (z+dz, y+dy, x+dx)) then
 * b[cout].  All calls are ordered on the stream given at creation and
 * return without waiting unless stated.
 * ------------------------------------------------------------------------- */
typedef struct pf_nn pf_nn;

typedef struct {
  long long max_voxels;   /* capacity: the largest n * D * H * W of any call (and the grid of an attached context) */
  int training;           /* 1: also allocate targets, loss gradient and backward buffers */
  int pad_;
  unsigned long long seed;  /* He-uniform initial weights from SplitMix64(seed); biases 0 */
} pf_nn_config;

typedef enum { PF_NN_OP_FORWARD = 0, PF_NN_OP_BACKWARD_DATA = 1, PF_NN_OP_BACKWARD_WEIGHT = 2 } pf_nn_op;
typedef enum { PF_NN_BUF_INPUT = 0, PF_NN_BUF_OUTPUT = 1, PF_NN_BUF_TARGET = 2, PF_NN_BUF_LOSS_GRAD = 3 } pf_nn_buffer_id;

/* Number of FP32 parameters (63 171). */
size_t pf_nn_param_count(void);

/* Bytes of device workspace a network with this configuration needs (about
 * 224 bytes per voxel of capacity, 384 with training buffers, plus the
 * parameters, their gradients, Adam moments and operand images); 0 if the
 * configuration is invalid. */
size_t pf_nn_workspace_bytes(const pf_nn_config *cfg);

/* Create a network.  `workspace` is a caller-owned device pointer (256-byte
 * aligned) to at least pf_nn_workspace_bytes(cfg) bytes, kept alive until
 * pf_nn_destroy; the library carves every device buffer of the network out of
 * it and allocates no device memory.  `hip_stream` is a hipStream_t (NULL =
 * default stream).  Errors: PF_ERR_INVALID_ARG (NULL or misaligned pointers,
 * max_voxels < 1), PF_ERR_OOM (workspace too small), PF_ERR_HIP. */
pf_status pf_nn_init(const pf_nn_config *cfg, void *workspace, size_t workspace_bytes, void *hip_stream,
                     pf_nn **out);
void pf_nn_destroy(pf_nn *nn);            /* frees the host object only, never the workspace */
const char *pf_nn_last_error(const pf_nn *nn);

/* Parameters to (dir 0) or from (dir 1) the host, or the gradients of the
 * last pf_nn_backward to the host (dir 2); `count` must equal
 * pf_nn_param_count().  Synchronises. */
pf_status pf_nn_weights(pf_nn *nn, int dir, float *host, size_t count);

/* Copy the first `bytes` bytes of an internal buffer (pf_nn_buffer_id: the
 * packed input [cap][8] bf16, the output [cap][4] FP32, the packed target
 * [cap][4] FP32, the loss gradient [cap][8] bf16) to the device array `dev`
 * (dir 0), or from it into the buffer (dir 1). */
pf_status pf_nn_copy(pf_nn *nn, int which, int dir, void *dev, size_t bytes);

/* Forward pass over n volumes of D x H x W voxels: x (8 channels; NULL: the
 * packed input buffer) -> y (4 channels FP32; NULL: the output buffer).  The
 * activations are kept for pf_nn_loss and pf_nn_backward. */
pf_status pf_nn_forward(pf_nn *nn, const void *x, float *y, int n, int D, int H, int W);

/* Relative mean-square loss of the last forward pass against `target`
 * (4 channels FP32 per voxel, the first 3 count; NULL: the packed targets):
 * L = (1/n) sum_s |p_s - q_s|^2 / |q_s|^2 (denominator 1 if q_s = 0).  Writes
 * dL/dp into the loss-gradient buffer; `mean_loss` (nullable, synchronises)
 * receives L. */
pf_status pf_nn_loss(pf_nn *nn, const float *target, double *mean_loss);

/* Gradients of the last forward pass for the output gradient dy (8 channels
 * bf16; NULL: the loss-gradient buffer), into the gradient vector. */
pf_status pf_nn_backward(pf_nn *nn, const void *dy);

/* One Adam step (bias-corrected, Kingma and Ba 2015) on the gradient vector. */
pf_status pf_nn_adam(pf_nn *nn, double lr, double b1, double b2, double eps);

/* One convolution kernel alone (pf_nn_op), for layer 0..3 over n volumes:
 *  FORWARD:          in = layer input (8 channels for layer 0, else 32) ->
 *                    out = max(conv + b, 0) as 32 bf16 channels (layers 0-2)
 *                    or conv + b as 4 FP32 channels (layer 3);
 *  BACKWARD_DATA:    (layers 1-3) in = output gradient (8 channels for layer 3,
 *                    else 32), aux = the layer's input (32 channels) ->
 *                    out = input gradient where aux > 0, else 0 (32 bf16);
 *  BACKWARD_WEIGHT:  in = layer input, aux = output gradient ->
 *                    out = FP32 dW[27][cout][cin] followed by db[cout]
 *                    (needs training buffers).
 * in, aux and out are device pointers aligned to 16 bytes
 * (PF_ERR_INVALID_ARG otherwise). */
pf_status pf_nn_layer(pf_nn *nn, int op, int layer, const void *in, const void *aux, void *out, int n, int D, int H,
                      int W);

/* s = root mean square of u1 - u0 over the low faces of every cell (u0 may be
 * NULL: zero).  u1, u0 are 3 device FP64 arrays in the exchange layout of
 * pf_fields.  Kept for pf_nn_pack; `s_out` (nullable, synchronises). */
pf_status pf_nn_increment_scale(pf_nn *nn, const double *const *u1, const double *const *u0, int nx, int ny, int nz,
                                double *s_out);

/* The increment scale of pf_nn_increment_scale for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): no network, no allocation of any kind.
 * s = root mean square of u1 - u0 over the low faces of every cell (u0 may be
 * NULL: zero), written to the caller's device scalar `s_dev` on `hip_stream`
 * (NULL = default stream); u1, u0 are 3 device FP64 arrays in the exchange
 * layout of pf_fields.  Stream-ordered, returns without waiting.  The result
 * is bitwise that of pf_nn_increment_scale (same kernels, same reduction
 * order).
 * Scratch: the 1024 FP64 block partials live in a static device array of the
 * library (8 KiB per GPU, held until the process ends); each call overwrites
 * all of it before reading it.  Calls that overlap on one GPU (other streams
 * or threads) share that array and race: serialise them.
 * Errors: PF_ERR_INVALID_ARG for NULL arrays or s_dev, sizes < 1, or
 * (nx+1)(ny+1)(nz+1) above 2^31 - 1; PF_ERR_HIP if there is no current device
 * or a launch fails.  Messages via pf_nn_last_error(NULL). */
pf_status pf_increment_scale_static(const double *const *u1, const double *const *u0, int nx, int ny, int nz,
                                    double *s_dev, void *hip_stream);

/* Pack the crop [x0, x0+cx) x [y0, y0+cy) x [z0, z0+cz) of a state into volume
 * `slot` of the input buffer (voxels outside the grid get zero), with the
 * scale of the last pf_nn_increment_scale: previous increment u1 - u0; when u2
 * is given also the target (u2 - u1) / s into the target buffer.  Device FP64
 * arrays in the exchange layout of pf_fields. */
pf_status pf_nn_pack(pf_nn *nn, const double *phi_f, const double *phi_w, const double *phi_prev,
                     const double *const *u1, const double *const *u0, const double *const *u2, int nx, int ny, int nz,
                     int x0, int y0, int z0, int cx, int cy, int cz, int slot, double Omega, double h);

/* Attach a network to a context created with warm == PF_WARM_LEARNED (3D,
 * grid within the network's capacity); NULL detaches.  The context does not
 * own the network.  From the second solve on, each solve packs the state,
 * runs the network, evaluates ||b - A u0|| for the learned and the previous
 * start and starts CG from the smaller; stats report both. */
pf_status pf_nn_attach(pf_ctx *ctx, pf_nn *nn);

/* Free the host-side context (never the caller's workspace). */
void pf_destroy(pf_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Finite-strain mechanics (Sec. 2.2, Eq. 9-14, 19, 25, 31, 34)
 *
 * The paper's kinematics F = F_E F_T F_P with F_T = d_T^(1/3) I (Eq. 9-12),
 * the phase-weighted neo-Hooke energy psi = d_T sum_a h(phi_a) phi_a(F_E)
 * (Eq. 13, 14) and the first Piola-Kirchhoff stress taken as its derivative
 * d psi / d F (Eq. 31; the printed form is twice that derivative), on a voxel
 * grid of bilinear (2D, plane strain) or trilinear (3D) cells with the
 * displacement at the cell corners and 2^d Gauss points per cell, each with
 * its own plastic deformation gradient F_P and accumulated plastic strain.
 * One solve: equilibrium Div P = 0 (Eq. 29, momentum line) under rollers on
 * every outer face (u . n = 0 there) by Newton's method, each Newton step
 * solved by Jacobi-preconditioned CG with the Jacobian applied matrix-free
 * (exact directional derivatives of the nodal forces), with a halving line
 * search on ||R||; then, with plasticity, the J2 return in the Mandel stress
 * at every Gauss point (Eq. 25, 34: backward Euler along the trial direction,
 * F_P = exp(dl N) F_P^n); then the cell means of d psi / d phi_f and
 * d psi / d phi_w at fixed F, F_P (the elastic driving forces of Eq. 33 in
 * this kinematics) and the largest von Mises stress of the Cauchy stress.
 * FP64 throughout.
 *
 * Exchange layouts (FP64, compact, x fastest): cells [nz][ny][nx]; nodal
 * displacement [d][nz+1][ny+1][nx+1] (2D: [2][ny+1][nx+1]); plastic
 * deformation gradient [nz][ny][nx][2^d][3][3] (Gauss point g: bit 0 the x
 * side, bit 1 y, bit 2 z of the cell, at 1/2 -+ 1/(2 sqrt 3)); accumulated
 * plastic strain [nz][ny][nx][2^d]; driving forces [2][nz][ny][nx].
 * ------------------------------------------------------------------------- */
typedef struct pf_fs pf_fs;

typedef struct {
  int dim;                /* 2 (plane strain) or 3 */
  int nx, ny, nz;         /* cells; nz == 1 when dim == 2; each >= 1 */
  double h;               /* cell size (m) */
  int plasticity;         /* 1: return map after the equilibrium solve */
  int newton_max_iter;    /* reaching it without convergence is an error */
  double newton_rtol;     /* stop when ||R(u)|| <= newton_rtol ||R(0)|| (free components) */
  double cg_rtol;         /* each Newton step: stop CG at ||J d + R|| <= cg_rtol ||R|| */
  int cg_max_iter;        /* per Newton step; reaching it ends that step's CG (not an error) */
  int pad_;
} pf_fs_config;

typedef struct {
  int newton_iters;       /* Newton steps of the last solve */
  int cg_iters;           /* CG iterations summed over its Newton steps */
  double rel_resid;       /* ||R(u)|| / ||R(0)|| at its end (0 when R(0) = 0) */
  double max_vm;          /* largest von Mises stress over the Gauss points (Pa) */
  double max_epsP;        /* largest accumulated plastic strain */
  int yielded;            /* Gauss points the return map moved */
  int line_search_cuts;   /* halvings of Newton steps */
} pf_fs_stats;

typedef enum {
  PF_FS_PHI_F = 0, PF_FS_PHI_W = 1,   /* cells, set/get */
  PF_FS_U = 2,                        /* nodes, d components, set/get (roller components forced to 0 on set) */
  PF_FS_FP = 3,                       /* Gauss points, 9 components, set/get */
  PF_FS_EPSP = 4,                     /* Gauss points, set/get */
  PF_FS_DRIVE = 5                     /* cells, 2 components, get only (from the last solve) */
} pf_fs_field;

/* Bytes of device workspace for this configuration (about 9 d + 2^d (d + 10)
 * + 4 doubles per cell); 0 if the configuration is invalid. */
size_t pf_fs_workspace_bytes(const pf_fs_config *cfg);

/* Create a finite-strain mechanics context on the caller's device workspace
 * (256-byte aligned, at least pf_fs_workspace_bytes bytes, kept alive until
 * pf_fs_destroy) and HIP stream (NULL = default).  Material parameters from
 * `params` (K, G, Omega_f, sigY, Hhard).  Starts with phi_f = phi_w = 0 (gas),
 * u = 0, F_P = I, eps_P = 0.  Allocates no device memory.  Errors:
 * PF_ERR_INVALID_ARG (bad configuration, NULL or misaligned pointers),
 * PF_ERR_OOM (workspace too small), PF_ERR_HIP. */
pf_status pf_fs_init(const pf_fs_config *cfg, const pf_params *params, void *workspace, size_t workspace_bytes,
                     void *hip_stream, pf_fs **out);

/* Copy one field (pf_fs_field) between the context and caller memory; dir 0
 * get, 1 set; ptr holds exactly nbytes of FP64 in the exchange layout;
 * ptr_is_device selects a device or host pointer.  Stream-ordered; a get to
 * host memory synchronises the stream.  Errors: PF_ERR_INVALID_ARG (unknown
 * field, wrong size, set of PF_FS_DRIVE), PF_ERR_HIP. */
pf_status pf_fs_fields(pf_fs *fs, int field, int dir, void *ptr, size_t nbytes, int ptr_is_device);

/* Solve for the displacement from the current one, then (plasticity) update
 * F_P and eps_P, then the driving forces and max_vm; `stats` nullable.
 * Synchronises the stream once per Newton step (for ||R||) and once per chunk
 * of CG launches.  Errors: PF_ERR_CG_NOT_CONVERGED when Newton reaches
 * newton_max_iter above newton_rtol or the tangent is not positive along a CG
 * direction; PF_ERR_NONFINITE when no step of the line search keeps the
 * residual finite (a cell turned inside out); PF_ERR_HIP. */
pf_status pf_fs_solve(pf_fs *fs, pf_fs_stats *stats);

/* Kernel classes of the finite-strain timing interface. */
typedef enum {
  PF_FS_K_TANGENT = 0,    /* element kernel on dual numbers: J v (one per CG iteration) */
  PF_FS_K_GATHER = 1,     /* nodal gather of element forces, with a dot-product partial */
  PF_FS_K_RESIDUAL = 2,   /* element kernel on FP64: nodal forces R(u) */
  PF_FS_K_VECTOR = 3,     /* CG vector updates and reductions */
  PF_FS_K_RETURN = 4,     /* return map at the Gauss points */
  PF_FS_K_POST = 5,       /* driving forces and von Mises stress */
  PF_FS_K_COUNT = 6
} pf_fs_kernel;

/* Switch per-kernel timing on (1) or off (0): HIP events around every launch
 * of the classes above, read back at the solve's synchronisations; turning it
 * on clears the accumulators.  Errors: PF_ERR_INVALID_ARG, PF_ERR_HIP. */
pf_status pf_fs_timing(pf_fs *fs, int on);

/* Accumulated device time (ms) and launch count of one kernel class since
 * timing was switched on.  Errors: PF_ERR_INVALID_ARG (NULL, unknown kind). */
pf_status pf_fs_timing_get(pf_fs *fs, int kind, double *ms, long long *launches);

/* Drive a context's phase-field step with the finite-strain mechanics (NULL
 * detaches).  Each pf_step then imports the current phases into `fs`, runs
 * pf_fs_solve (from the previous displacement and plastic state of `fs`) and
 * adds its cell driving forces d psi / d phi_f, d psi / d phi_w (Eq. 33) to
 * the Allen-Cahn update of that step; the step's stats report the solve's CG
 * iterations, residual, largest von Mises stress and plastic strain.  The
 * context must have been created with mechanics = 0 (its small-strain
 * mechanics off), on the same grid, h and stream; it does not own `fs`.
 * Errors: PF_ERR_INVALID_ARG (mismatch; message on the context). */
pf_status pf_fs_attach(pf_ctx *ctx, pf_fs *fs);

/* Message of the last error on this context (fs NULL: errors raised before a
 * context existed). */
const char *pf_fs_last_error(const pf_fs *fs);

/* Free the host side (never the caller's workspace). */
void pf_fs_destroy(pf_fs *fs);

#ifdef __cplusplus
}
#endif
#endif
