// Host side of the C ABI declared in include/pf.h: context, workspace layout,
// device-side CG control and field exchange.  Every numerical step runs in the
// kernels of pf_kernels.h.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/pf.h"
#include "pf_kernels.h"
#include "pf_species.h"
#include "pf_step3.h"
#include "pf_mg.h"

using namespace pfk;

namespace {

constexpr size_t kAlign = 256;
constexpr int kUpdBlocksMax = 512;
constexpr int kApplyBY = 8;          // tile height of the 3D apply kernel (block = 64 x 8 threads)
constexpr int kCgBY = 8;             // tile height of its CG instance
// deepest z slab per block of the 3D apply kernels (halved while the grid
// has fewer than 512 blocks): the slab re-reads one plane at each end
constexpr int kSlabMax = 32;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kStagger = 17 * kAlign;

constexpr int kAfterBlocks = 2048;   // blocks of the learned start's after-solve pass
constexpr int kFoldBlocks = 128;     // blocks folding the field update's partials before the ledger

struct Layout {
  Grid g;
  int nc;                  // plastic strain components
  size_t es;               // element size (4 or 8)
  int kz;
  dim3 gel, gcell;
  int kz_ap;               // z planes per block of the 3D apply kernel
  dim3 gap;                // its grid (64 x kApplyBY tiles)
  int kz_cg;               // the same for the CG instance (64 x kCgBY tiles); 2D: the apply grid
  dim3 gcg;
  int nb_cg;
  int nb_el, nb_cell, nb_upd;
  int nb_res;              // blocks (partial pairs) of the residual pass CG starts from: the apply grid (3D), the elast grid (2D)
  size_t stage_elems;
  // byte offsets into the workspace
  size_t o_fld[2][5], o_u[3], o_epsp, o_epsP, o_mu, o_K, o_G;
  size_t o_lo[2][5];       // FP32 state: low parts of the five fields (0 in FP64)
  size_t o_r[3], o_z[3], o_pa[3], o_pb[3], o_q[3], o_di[3];
  size_t o_scal, o_part_u, o_part_a, o_part_b, o_part_c, o_part_f, o_stage;
  size_t o_uo[3], o_du[3], o_phiprev;   // learned start only
  size_t o_phiprev_lo;                  // learned start, FP32 state: low part of phi_prev
  size_t o_dsq;                          // learned start: partials of the increment's sum of squares
  size_t o_b[3];                        // 3D: right-hand side b of the equilibrium solve
  // implicit species: per species D, D^-1, r, z, two directions, q and the increment
  size_t o_sp[8][3];
  size_t o_sp_part, o_sp_scal;
  int nb_sp;
  // multigrid preconditioner (cg_precond == 1): level 0 is the grid of
  // the solve (its K, G, D^-1; b is the CG residual, x the preconditioned z);
  // levels 1 .. mg_n - 1 own their moduli, diagonal, b, x, a second x and r
  struct MGLevel {
    Grid g;
    int kz;
    dim3 grid;             // apply-kernel grid of the level
    double h;
    size_t oK, oG, odi[3], ob[3], ox[3], oxt[3], orr[3];
    size_t olo[5];         // 3D FP32: bf16 copies of K, G, D^-1 (x, y, z) for the sweeps
  };
  static constexpr int kMGMax = 10;
  int mg_n;
  MGLevel mg[kMGMax];
  size_t o_mg_part;
  size_t o_mg_tail;        // 2D: the tail kernel's level table (written once per solve)
  int nb_mg;               // partials of the level-0 smoothing (its apply grid)
  int mg_tail;             // 2D: first level (>= 1) the single-block tail kernel runs from, or -1
  size_t total;
};

bool valid_cfg(const pf_config* c, char* msg, size_t len) {
  if (!c) { snprintf(msg, len, "config is NULL"); return false; }
  if (c->dim != 2 && c->dim != 3) { snprintf(msg, len, "dim must be 2 or 3 (got %d)", c->dim); return false; }
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) { snprintf(msg, len, "grid sizes must be >= 1"); return false; }
  if (c->dim == 2 && c->nz != 1) { snprintf(msg, len, "nz must be 1 when dim == 2"); return false; }
  if (!(c->h > 0.0) || !(c->dt > 0.0)) { snprintf(msg, len, "h and dt must be positive"); return false; }
  if (c->precision != PF_FP64 && c->precision != PF_MIXED) { snprintf(msg, len, "unknown precision %d", c->precision); return false; }
  if (c->mechanics && (!(c->cg_rtol > 0.0) || c->cg_max_iter < 1)) { snprintf(msg, len, "cg_rtol > 0 and cg_max_iter >= 1 required"); return false; }
  if (c->warm != PF_WARM_ZERO && c->warm != PF_WARM_PREV && c->warm != PF_WARM_LEARNED) { snprintf(msg, len, "unknown warm start %d", c->warm); return false; }
  if (c->warm == PF_WARM_LEARNED && (c->dim != 3 || !c->mechanics)) { snprintf(msg, len, "the learned warm start needs dim 3 and mechanics"); return false; }
  if (c->species_implicit < 0 || c->species_implicit > 2) { snprintf(msg, len, "species_implicit must be 0, 1 or 2"); return false; }
  if (c->cg_precond != 0 && c->cg_precond != 1) { snprintf(msg, len, "cg_precond must be 0 or 1"); return false; }
  if (c->species_implicit && (!(c->species_rtol > 0.0) || c->species_max_iter < 1)) { snprintf(msg, len, "species_rtol > 0 and species_max_iter >= 1 required"); return false; }
  long long px = (c->nx + 15) / 16 * 16;
  if (px * c->ny * (long long)c->nz >= (1LL << 31) / 8) { snprintf(msg, len, "grid too large for 32-bit indexing"); return false; }
  return true;
}

Layout make_layout(const pf_config* c) {
  Layout L{};
  Grid& g = L.g;
  g.nx = c->nx; g.ny = c->ny; g.nz = c->nz;
  g.px = (c->nx + 15) / 16 * 16;
  g.n = g.px * g.ny * g.nz;
  g.ns = g.n;
  L.nc = c->dim == 2 ? 4 : 6;
  L.es = c->precision == PF_FP64 ? 8 : 4;
  int nbx = (g.nx + TX - 1) / TX, nby = (g.ny + TY - 1) / TY;
  L.kz = 1;
  if (c->dim == 3) {
    L.kz = 8;
    while (L.kz > 1 && (long long)nbx * nby * ((g.nz + L.kz - 1) / L.kz) < 2048) L.kz /= 2;
  }
  L.gel = dim3(nbx, nby, c->dim == 3 ? (g.nz + L.kz - 1) / L.kz : 1);
  if (c->dim == 3) {
    // deeper z chunks and taller tiles cut the re-fetched halo; keep >= 512 blocks
    int nby8 = (g.ny + kApplyBY - 1) / kApplyBY;
    L.kz_ap = kSlabMax;
    while (L.kz_ap > 1 && (long long)nbx * nby8 * ((g.nz + L.kz_ap - 1) / L.kz_ap) < 512) L.kz_ap /= 2;
    L.gap = dim3(nbx, nby8, (g.nz + L.kz_ap - 1) / L.kz_ap);
    int nbyc = (g.ny + kCgBY - 1) / kCgBY;
    L.kz_cg = kSlabMax;
    while (L.kz_cg > 1 && (long long)nbx * nbyc * ((g.nz + L.kz_cg - 1) / L.kz_cg) < 512) L.kz_cg /= 2;
    L.gcg = dim3(nbx, nbyc, (g.nz + L.kz_cg - 1) / L.kz_cg);
  } else {
    // rows of A2W columns marching along y over kz_ap rows; keep >= 2048
    // blocks (a block is 4 waves: at 2048^2, 512 blocks left the apply and
    // the multigrid sweeps latency-bound, 47 and 62 us against 39 and 31 us
    // with 2048; 4096 and 8192 were slower again)
    int nbx2 = (g.nx + A2W - 1) / A2W;
    L.kz_ap = 32;
    while (L.kz_ap > 1 && (long long)nbx2 * ((g.ny + L.kz_ap - 1) / L.kz_ap) < 2048) L.kz_ap /= 2;
    L.gap = dim3(nbx2, (g.ny + L.kz_ap - 1) / L.kz_ap, 1);
    L.kz_cg = L.kz_ap;
    L.gcg = L.gap;
  }
  L.nb_cg = (int)(L.gcg.x * L.gcg.y * L.gcg.z);
  L.nb_el = nbx * nby * (int)L.gel.z;
  L.gcell = dim3(nbx, nby, g.nz);
  L.nb_cell = nbx * nby * g.nz;
  int vn = (int)(16 / L.es);
  L.nb_upd = std::max(1, std::min(kUpdBlocksMax, (g.n / vn + NT - 1) / NT));
  size_t fx = (size_t)(g.nx + 1) * g.ny * g.nz, fy = (size_t)g.nx * (g.ny + 1) * g.nz;
  size_t fz = (size_t)g.nx * g.ny * (g.nz + 1);
  L.stage_elems = std::max(fx, std::max(fy, fz));
  size_t off = 0;
  size_t arr = align_up((size_t)g.n * L.es);
  // consecutive arrays start 17 x 256 bytes apart beyond their size (with
  // power-of-two sizes, the arrays a kernel streams together would otherwise
  // start at the same offset of the memory channel interleave)
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes) + kStagger; return o; };
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 5; ++f) L.o_fld[s][f] = take(arr);
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 5; ++f) L.o_lo[s][f] = L.es == 4 ? take(arr) : 0;
  for (int d = 0; d < 3; ++d) L.o_u[d] = d < c->dim ? take(arr) : 0;
  L.o_epsp = take(arr * L.nc);
  L.o_epsP = take(arr);
  L.o_mu = take(arr);
  L.o_K = take(arr);
  L.o_G = take(arr);
  for (int d = 0; d < c->dim; ++d) {
    L.o_r[d] = take(arr); L.o_z[d] = take(arr); L.o_pa[d] = take(arr);
    L.o_pb[d] = take(arr); L.o_q[d] = take(arr); L.o_di[d] = take(arr);
  }
  if (c->dim == 3)
    for (int d = 0; d < 3; ++d) L.o_b[d] = take(arr);
  L.o_scal = take(S_COUNT * sizeof(double));
  L.nb_res = c->dim == 3 ? (int)(L.gap.x * L.gap.y * L.gap.z) : L.nb_el;
  int nbmax = std::max(std::max(L.nb_el, (int)(L.gap.x * L.gap.y * L.gap.z)), std::max(L.nb_cell, L.nb_upd));
  nbmax = std::max(nbmax, L.nb_cg);
  L.o_part_u = take(2 * (size_t)nbmax * sizeof(double));
  L.o_part_a = take(2 * (size_t)nbmax * sizeof(double));
  L.o_part_b = take(2 * (size_t)nbmax * sizeof(double));
  L.o_part_c = take(NQ_STEP * (size_t)nbmax * sizeof(double));
  L.o_part_f = take(NQ_STEP * (size_t)kFoldBlocks * sizeof(double));
  L.o_stage = take(L.stage_elems * sizeof(double));
  L.nb_sp = std::max(1, std::min(kSpBlocksMax, (g.n + NT - 1) / NT));
  if (c->species_implicit) {
    for (int a = 0; a < 8; ++a)
      for (int q = 0; q < 3; ++q) L.o_sp[a][q] = take(arr);
    L.o_sp_part = take(9 * (size_t)L.nb_sp * sizeof(double));
    L.o_sp_scal = take(SP_COUNT * sizeof(double));
  }
  L.mg_n = 0;
  L.mg_tail = -1;
  if (c->cg_precond == 1) {
    const int dim = c->dim;
    // apply-kernel grid of a level: 3D 64 x kApplyBY column tiles over slabs
    // of kz planes, 2D rows of A2W cells over runs of kz rows; kz halved
    // until the level has 512 (2D: 2048) blocks or kz is 1
    auto apply_geom = [dim](Layout::MGLevel& m) {
      if (dim == 3) {
        const int nbx = (m.g.nx + TX - 1) / TX, nby8 = (m.g.ny + kApplyBY - 1) / kApplyBY;
        m.kz = kSlabMax;
        while (m.kz > 1 && (long long)nbx * nby8 * ((m.g.nz + m.kz - 1) / m.kz) < 512) m.kz /= 2;
        m.grid = dim3(nbx, nby8, (m.g.nz + m.kz - 1) / m.kz);
      } else {
        const int nbx = (m.g.nx + A2W - 1) / A2W;
        m.kz = 32;
        while (m.kz > 1 && (long long)nbx * ((m.g.ny + m.kz - 1) / m.kz) < 2048) m.kz /= 2;
        m.grid = dim3(nbx, (m.g.ny + m.kz - 1) / m.kz, 1);
      }
    };
    const bool lo = dim == 3 && L.es == 4;
    auto take_lo = [&](Layout::MGLevel& m) {
      for (int a = 0; a < 5; ++a) m.olo[a] = lo ? take(align_up((size_t)m.g.n * 2)) : 0;
    };
    Layout::MGLevel& m0 = L.mg[0];
    m0.g = g;
    m0.h = c->h;
    apply_geom(m0);
    take_lo(m0);
    m0.oK = L.o_K;
    m0.oG = L.o_G;
    for (int d = 0; d < 3; ++d) {
      m0.odi[d] = d < dim ? L.o_di[d] : 0;
      m0.ob[d] = d < dim ? L.o_r[d] : 0;
      m0.ox[d] = d < dim ? L.o_z[d] : 0;
      m0.oxt[d] = d < dim ? take(arr) : 0;
      m0.orr[d] = d < dim ? take(arr) : 0;
    }
    L.mg_n = 1;
    while (L.mg_n < Layout::kMGMax) {
      const Grid& f = L.mg[L.mg_n - 1].g;
      const int lo = dim == 3 ? std::min(f.nx, std::min(f.ny, f.nz)) : std::min(f.nx, f.ny);
      if (lo <= 8) break;
      Layout::MGLevel& m = L.mg[L.mg_n];
      m.g.nx = (f.nx + 1) / 2; m.g.ny = (f.ny + 1) / 2; m.g.nz = dim == 3 ? (f.nz + 1) / 2 : 1;
      m.g.px = (m.g.nx + 15) / 16 * 16;
      m.g.n = m.g.px * m.g.ny * m.g.nz;
      m.g.ns = m.g.n;
      m.h = 2.0 * L.mg[L.mg_n - 1].h;
      apply_geom(m);
      take_lo(m);
      const size_t la = align_up((size_t)m.g.n * L.es);
      m.oK = take(la);
      m.oG = take(la);
      for (int d = 0; d < 3; ++d) {
        if (d < dim) {
          m.odi[d] = take(la); m.ob[d] = take(la); m.ox[d] = take(la); m.oxt[d] = take(la); m.orr[d] = take(la);
        } else {
          m.odi[d] = m.ob[d] = m.ox[d] = m.oxt[d] = m.orr[d] = 0;
        }
      }
      ++L.mg_n;
    }
    L.mg_tail = -1;
    if (dim == 2)
      for (int l = 1; l < L.mg_n; ++l)
        if ((long long)L.mg[l].g.nx * L.mg[l].g.ny <= kTailCells && L.mg_n - l <= kTailMax) {
          L.mg_tail = l;
          break;
        }
    L.nb_mg = (int)(m0.grid.x * m0.grid.y * m0.grid.z);
    int nb_mg_max = 0;
    for (int l = 0; l < L.mg_n; ++l) nb_mg_max = std::max(nb_mg_max, (int)(L.mg[l].grid.x * L.mg[l].grid.y * L.mg[l].grid.z));
    L.o_mg_part = take((size_t)nb_mg_max * sizeof(double));
    L.o_mg_tail = L.mg_tail > 0 ? take(sizeof(MGTailArgs<double>)) : 0;
  }
  if (c->warm == PF_WARM_LEARNED) {
    for (int d = 0; d < 3; ++d) { L.o_uo[d] = take(arr); L.o_du[d] = take(arr); }
    L.o_phiprev = take(arr);
    L.o_phiprev_lo = L.es == 4 ? take(arr) : 0;
    L.o_dsq = take(kAfterBlocks * sizeof(double));
  }
  L.total = off;
  return L;
}

template <typename T>
KP<T> make_kp(const pf_config* c, const pf_params* p) {
  KP<T> k{};
  k.scale = (T)(p->R * p->theta / p->Vmol);
  for (int a = 0; a < 3; ++a) {
    k.w[a] = (T)p->w[a]; k.eps[a] = (T)p->eps[a]; k.L[a] = (T)p->L[a];
    k.K[a] = (T)p->K[a]; k.G[a] = (T)p->G[a];
    k.DO[a] = (T)p->DO[a]; k.DH[a] = (T)p->DH[a]; k.DW[a] = (T)p->DW[a];
  }
  k.kappaO = (T)p->kappaO;
  k.sigY = (T)p->sigY; k.Hh = (T)p->Hhard;
  k.kfor = (T)p->kfor; k.Omega = (T)p->Omega_f;
  k.xHbc = (T)p->xH_bc; k.xWbc = (T)p->xW_bc;
  k.h = (T)c->h; k.ih = (T)(1.0 / c->h); k.ih2 = (T)(1.0 / (c->h * c->h)); k.dt = (T)c->dt;
  k.mform = p->m_form; k.dirichlet = c->dirichlet; k.chem = c->chem_phase;
  k.plastic = c->plasticity; k.mech = c->mechanics;
  k.rsplit = c->species_implicit == 2;
  return k;
}

}  // namespace

struct pf_ctx {
  pf_config cfg;
  pf_params prm;
  hipStream_t stream;
  Layout L;
  char* ws;
  double* host_scal;       // pinned copy of the device scalars
  char err[512];
  bool bad;
  bool ledger_valid;
  bool mg_tail_ready;      // the 2D multigrid tail kernel's level table is in the workspace
  int cur;                 // which field buffer holds the current state
  long long steps;
  int last_iters;
  int prev_iters;          // iteration count of the solve before the last one
  int cg_chunk;            // CG launches between convergence checks (0: adaptive)
  int warm_used;
  // per-kernel event timing
  unsigned timing;         // bit mask of the kernel kinds being recorded (0: off)
  int timing_every;        // CG kernels: record every n-th iteration only
  long long solves;        // solves started (rotates the sampled iterations)
  std::vector<hipEvent_t> ev_pool;
  struct Rec { int kind, ev, launch; bool count; };
  std::vector<Rec> pending;   // start event index ev, stop ev + 1; launch = CG launch index or -1
  long long iters_total;
  int ev_next;
  long long n_flush;       // timing flushes so far (a flush empties `pending`)
  double t_ms[PF_K_COUNT];
  long long t_n[PF_K_COUNT];
  // learned start
  pf_nn* net;
  bool have_prev_incr;
  bool judged;             // the last solve evaluated the learned start
  double r0_learned, r0_prev;
  int sp_last_iters;       // implicit species: the most CG iterations of a species in the last step
  double* host_sp;         // pinned copy of the species scalars
  // attached finite-strain mechanics (pf_fs_attach): solved for the phases
  // of each step, its cell driving forces enter the phase-field update
  pf_fs* fs;
  pf_fs_stats fs_last;
  template <typename T> T* arr(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  double* scal() const { return arr<double>(L.o_scal); }
};

static char g_err[512] = "";

static pf_status fail(pf_ctx* c, pf_status s, const char* fmt, ...) {
  char* dst = c ? c->err : g_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return s;
}

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail((ctx), PF_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(ctx)                                                                               \
  do {                                                                                               \
    hipError_t e_ = hipGetLastError();                                                               \
    if (e_ != hipSuccess) return fail((ctx), PF_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
  } while (0)

// Resolve recorded event pairs into the per-kind accumulators (after a sync).
static void timing_flush(pf_ctx* c) {
  for (auto& pr : c->pending) {
    float ms = 0.f;
    if (pr.count && hipEventElapsedTime(&ms, c->ev_pool[pr.ev], c->ev_pool[pr.ev + 1]) == hipSuccess) {
      c->t_ms[pr.kind] += ms;
      c->t_n[pr.kind] += 1;
    }
  }
  c->pending.clear();
  c->ev_next = 0;
  ++c->n_flush;
}

// Launch helper: brackets the launch with events when timing is on.
template <typename F>
static void timed(pf_ctx* c, int kind, F&& launch, int cg_launch = -1) {
  if (!((c->timing >> kind) & 1u) || (cg_launch >= 0 && (cg_launch + c->solves) % c->timing_every != 0)) {
    launch();
    return;
  }
  if (c->ev_next + 2 > (int)c->ev_pool.size()) {
    (void)hipStreamSynchronize(c->stream);
    timing_flush(c);
  }
  int i = c->ev_next;
  c->ev_next += 2;
  (void)hipEventRecord(c->ev_pool[i], c->stream);
  launch();
  (void)hipEventRecord(c->ev_pool[i + 1], c->stream);
  c->pending.push_back({kind, i, cg_launch, true});
}

// Launch of one kernel, timed when its kind is being recorded: the events
// are attached to the dispatch itself (hipExtLaunchKernel).  A dispatch
// with events that follows one without them reads a few microseconds long,
// so in a sampled CG iteration every launch carries events, and so does the
// update before it; only the selected kinds of the sampled iteration count.
template <typename K, typename... Args>
static void timed_launch(pf_ctx* c, int kind, int cg_launch, K kernel, dim3 grid, dim3 block, uint32_t smem,
                         hipStream_t st, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool rec = false, count = false;
  if (c->timing) {
    const bool on = (c->timing >> kind) & 1u;
    if (cg_launch < 0) {
      rec = count = on;
    } else {
      const bool sampled = (cg_launch + c->solves) % c->timing_every == 0;
      const bool guard = kind == PF_K_UPDATE && (cg_launch + 1 + c->solves) % c->timing_every == 0;
      const bool cg_on = ((c->timing >> PF_K_APPLY) & 1u) || ((c->timing >> PF_K_UPDATE) & 1u) ||
                         ((c->timing >> PF_K_PRECOND) & 1u) || ((c->timing >> PF_K_SMOOTH) & 1u);
      rec = cg_on && (sampled || guard);
      count = on && sampled;
    }
  }
  if (rec) {
    if (c->ev_next + 2 > (int)c->ev_pool.size()) {
      (void)hipStreamSynchronize(c->stream);
      timing_flush(c);
    }
    const int i = c->ev_next;
    c->ev_next += 2;
    e0 = c->ev_pool[i];
    e1 = c->ev_pool[i + 1];
    c->pending.push_back({kind, i, cg_launch, count});
  }
  hipExtLaunchKernelGGL(kernel, grid, block, smem, st, e0, e1, 0u, args...);
}

// finite-strain mechanics of a step (defined with the finite-strain code at the
// end of this file): imports the current phases (padded, element size es,
// FP32 pairs when lo is given) into the attached solver, solves, and returns
// its cell driving forces
static pf_status fs_couple(pf_ctx* c, const Grid& g, const void* pf_hi, const void* pw_hi, const void* pf_lo,
                           const void* pw_lo, int es, const double** drive);

// learned start (defined with the network code at the end of this file)
template <typename T, int DIM> static pf_status learned_start(pf_ctx* c, ElastArgs<T> e, double* part);
template <typename T, int DIM> static pf_status learned_after_solve(pf_ctx* c);

// ---------------------------------------------------------------------------
// typed implementation
// ---------------------------------------------------------------------------
template <typename T, int DIM>
struct Impl {
  static CellArgs<T> cell_args(pf_ctx* c) {
    const Layout& L = c->L;
    CellArgs<T> a{};
    a.g = L.g;
    a.p = make_kp<T>(&c->cfg, &c->prm);
    int s = c->cur;
    a.pf = c->arr<T>(L.o_fld[s][0]); a.pw = c->arr<T>(L.o_fld[s][1]); a.xO = c->arr<T>(L.o_fld[s][2]);
    a.xH = c->arr<T>(L.o_fld[s][3]); a.xW = c->arr<T>(L.o_fld[s][4]);
    a.npf = c->arr<T>(L.o_fld[s ^ 1][0]); a.npw = c->arr<T>(L.o_fld[s ^ 1][1]); a.nxO = c->arr<T>(L.o_fld[s ^ 1][2]);
    a.nxH = c->arr<T>(L.o_fld[s ^ 1][3]); a.nxW = c->arr<T>(L.o_fld[s ^ 1][4]);
    if (L.es == 4)
      for (int f = 0; f < 5; ++f) {
        a.lo[f] = c->arr<T>(L.o_lo[s][f]);
        a.nlo[f] = c->arr<T>(L.o_lo[s ^ 1][f]);
      }
    if (c->cfg.species_implicit)
      for (int q = 0; q < 3; ++q) {
        a.sp_r[q] = c->arr<T>(L.o_sp[2][q]);
        a.sp_D[q] = c->arr<T>(L.o_sp[0][q]);
      }
    a.mu = c->arr<T>(L.o_mu);
    a.mu_out = c->arr<T>(L.o_mu);
    for (int d = 0; d < DIM; ++d) a.u[d] = c->arr<T>(L.o_u[d]);
    a.epsp = c->arr<T>(L.o_epsp);
    a.epsP = c->arr<T>(L.o_epsP);
    a.K = c->arr<T>(L.o_K);
    a.G = c->arr<T>(L.o_G);
    return a;
  }

  static ElastArgs<T> elast_args(pf_ctx* c) {
    const Layout& L = c->L;
    ElastArgs<T> a{};
    a.g = L.g;
    a.p = make_kp<T>(&c->cfg, &c->prm);
    a.K = c->arr<T>(L.o_K);
    a.G = c->arr<T>(L.o_G);
    a.phi_f = c->arr<T>(L.o_fld[c->cur][0]);
    a.epsp = c->arr<T>(L.o_epsp);
    a.scal = c->scal();
    a.tol2 = c->cfg.cg_rtol * c->cfg.cg_rtol;
    a.kz = L.kz;
    return a;
  }

  static pf_status ledger_reset(pf_ctx* c) {
    const Layout& L = c->L;
    CellArgs<T> a = cell_args(c);
    a.part = c->arr<double>(L.o_part_c);
    timed_launch(c, PF_K_OTHER, -1, k_totals<T, DIM>, L.gcell, dim3(NT), 0, c->stream, a);
    double vol = std::pow(c->cfg.h, DIM);
    hipLaunchKernelGGL(k_ledger, dim3(1), dim3(NT), 0, c->stream, (const double*)a.part, L.nb_cell, c->scal(), vol, 0.0, 0);
    LAUNCHCHK(c);
    c->ledger_valid = true;
    return PF_OK;
  }

  // q = A x on the 3D apply kernel outside the CG recurrence (x into z's
  // place; the direction buffer pa receives a copy of x).
  // q = A x on the apply kernel; with jr set, the block partials are
  // ||jr - q||^2 instead of x.q
  static void apply_plain(pf_ctx* c, const ElastArgs<T>& e, T* x0, T* x1, T* x2, double* part,
                          const T* const* jr = nullptr) {
    if constexpr (DIM == 3) {
      const Layout& L = c->L;
      ElastArgs<T> ap = e;
      ap.kz = L.kz_ap;
      ap.part = part;
      T* x[3] = {x0, x1, x2};
      for (int d = 0; d < 3; ++d) {
        ap.z[d] = x[d];
        ap.u[d] = c->arr<T>(L.o_pa[d]);
        ap.o1[d] = c->arr<T>(L.o_pa[d]);
        ap.o2[d] = c->arr<T>(L.o_q[d]);
        ap.jr[d] = jr ? jr[d] : nullptr;
      }
      timed_launch(c, PF_K_SOLVE_SETUP, -1, k_apply3<T, kApplyBY, APPLY_PLAIN>, L.gap, dim3(ApplyTile<kApplyBY>::NTB), 0, c->stream, ap);
    }
  }

  // Multigrid preconditioner (3D).  Grid-stride launches over a level.
  static dim3 mg_blocks(const Grid& g) {
    const long n = (long)g.nx * g.ny * g.nz;
    return dim3((unsigned)std::max(1L, std::min(4096L, (n + NT - 1) / NT)));
  }
  // one thread per cell of the level (the transfers)
  static dim3 mg_cell_blocks(const Grid& g) {
    const long n = (long)g.nx * g.ny * g.nz;
    return dim3((unsigned)((n + NT - 1) / NT));
  }
  // the 3D prolongation: one thread per fine x pair
  static dim3 mg_pair_blocks(const Grid& g) {
    const long n = (long)((g.nx + 1) / 2) * g.ny * g.nz;
    return dim3((unsigned)((n + NT - 1) / NT));
  }
  static Vec3<T> mg_vec(pf_ctx* c, const size_t (&o)[3]) {
    Vec3<T> v;
    for (int d = 0; d < 3; ++d) v.a[d] = c->arr<T>(o[d]);
    return v;
  }
  static CVec3<T> mg_cvec(pf_ctx* c, const size_t (&o)[3]) {
    CVec3<T> v;
    for (int d = 0; d < 3; ++d) v.a[d] = c->arr<T>(o[d]);
    return v;
  }
  // coarse moduli and Jacobi diagonals of every level from the moduli the
  // set-up pass wrote (once per solve)
  static void mg_setup(pf_ctx* c) {
    const Layout& L = c->L;
    if constexpr (DIM == 2)
      if (L.mg_tail > 0 && !c->mg_tail_ready) {
        // the tail kernel's level table, passed by pointer (as a kernel
        // argument, about 1 KB, it cost a device copy per launch); the
        // workspace addresses it holds are fixed for the context's life
        MGTailArgs<T> ta = mg_tail_args(c);
        if (hipMemcpyAsync(c->ws + L.o_mg_tail, &ta, sizeof(ta), hipMemcpyHostToDevice, c->stream) == hipSuccess)
          c->mg_tail_ready = true;
      }
    for (int l = 1; l < L.mg_n; ++l) {
      const Layout::MGLevel& f = L.mg[l - 1];
      const Layout::MGLevel& m = L.mg[l];
      timed_launch(c, PF_K_PRECOND, -1, DIM == 3 ? k_mg_coarsen<T> : k_mg_coarsen2<T>, mg_blocks(m.g), dim3(NT), 0,
                   c->stream, f.g, m.g, (const T*)c->arr<T>(f.oK), (const T*)c->arr<T>(f.oG), c->arr<T>(m.oK),
                   c->arr<T>(m.oG));
      timed_launch(c, PF_K_PRECOND, -1, DIM == 3 ? k_mg_diag<T> : k_mg_diag2<T>, mg_blocks(m.g), dim3(NT), 0,
                   c->stream, m.g, (T)(1.0 / m.h), (const T*)c->arr<T>(m.oK), (const T*)c->arr<T>(m.oG),
                   mg_vec(c, m.odi));
    }
    if constexpr (DIM == 3 && sizeof(T) == 4)    // the sweeps' bf16 K, G, D^-1 of the coarse levels
      for (int l = 1; l < L.mg_n; ++l) {
        const Layout::MGLevel& m = L.mg[l];
        MGLoCopy cp;
        const size_t src[5] = {m.oK, m.oG, m.odi[0], m.odi[1], m.odi[2]};
        for (int a = 0; a < 5; ++a) {
          cp.src[a] = (const float*)c->arr<T>(src[a]);
          cp.dst[a] = c->arr<unsigned short>(m.olo[a]);
        }
        timed_launch(c, PF_K_PRECOND, -1, k_mg_lo, mg_blocks(m.g), dim3(NT), 0, c->stream, cp, m.g.n);
      }
  }
  // a level's bf16 copies in the sweep arguments
  static void mg_lo_args(pf_ctx* c, const Layout::MGLevel& m, ElastArgs<T>& a) {
    if constexpr (DIM == 3 && sizeof(T) == 4) {
      a.lo_K = c->arr<unsigned short>(m.olo[0]);
      a.lo_G = c->arr<unsigned short>(m.olo[1]);
      for (int d = 0; d < 3; ++d) a.lo_d[d] = c->arr<unsigned short>(m.olo[2 + d]);
    }
  }
  // z = M^-1 r: one V-cycle from zero on the CG residual (level 0: b = r,
  // x = z), then r.z into the r.z partials CG reads (n_rz slots of part_u).
  // j: the CG launch index the cycle follows (-1: before the first).
  // Jacobi steps: each pair of sweeps applies (I - s0 D^-1 A)(I - s1 D^-1 A),
  // the degree-2 Chebyshev polynomial smallest on [lmax / 6, lmax] (its
  // roots 1 / s at the Chebyshev nodes of that interval).  Power iteration
  // on the 32^3 porous and core-shell recipes puts the largest eigenvalue
  // of D^-1 A near 4.26 (the phases' Poisson ratios fix it); lmax = 4.5,
  // and the pair amplifies only eigenvalues above (s0 + s1) / (s0 s1) = 5.25.
  static constexpr double kLmax = 4.5, kLmin = kLmax / 6.0;
  static constexpr double kMid = 0.5 * (kLmax + kLmin), kHalf = 0.5 * (kLmax - kLmin) * 0.70710678118654752;
  static constexpr double kStep[2] = {1.0 / (kMid + kHalf), 1.0 / (kMid - kHalf)};
  static constexpr int kCoarseSweeps = 8;

  // 2D: the level table of the single-block tail kernel (levels mg_tail ..)
  static MGTailArgs<T> mg_tail_args(pf_ctx* c) {
    const Layout& L = c->L;
    MGTailArgs<T> ta{};
    ta.n = L.mg_n - L.mg_tail;
    for (int t = 0; t < ta.n; ++t) {
      const Layout::MGLevel& m = L.mg[L.mg_tail + t];
      MGTailLevel<T>& v = ta.lv[t];
      v.g = m.g;
      v.ih = (T)(1.0 / m.h);
      v.K = c->arr<T>(m.oK);
      v.G = c->arr<T>(m.oG);
      for (int d = 0; d < 2; ++d) {
        v.dinv[d] = c->arr<T>(m.odi[d]);
        v.b[d] = c->arr<T>(m.ob[d]);
        v.bw[d] = c->arr<T>(m.ob[d]);
        v.x[d] = c->arr<T>(m.ox[d]);
        v.xt[d] = c->arr<T>(m.oxt[d]);
        v.r[d] = c->arr<T>(m.orr[d]);
      }
    }
    ta.s0 = (T)kStep[0];
    ta.s1 = (T)kStep[1];
    ta.coarse_sweeps = kCoarseSweeps;
    ta.scal = c->scal();
    return ta;
  }

  static void mg_vcycle(pf_ctx* c, const ElastArgs<T>& e, int j, int n_rz) {
    constexpr int kNu = 2;
    static_assert(kNu == 2, "the pre-smoothing is the two-sweep pass from zero; two post-smoothing sweeps");
    const Layout& L = c->L;
    hipStream_t st = c->stream;
    double* part = c->arr<double>(L.o_mg_part);
    const double* scal = c->scal();
    const int last = L.mg_n - 1;
    // one Jacobi sweep xout = xin + omega D^-1 (b - A xin) of level l, or
    // with omega = 0 the residual xout = b - A xin
    auto sweep = [&](int l, const size_t (&xin)[3], const size_t (&xout)[3], double omega) {
      const Layout::MGLevel& m = L.mg[l];
      ElastArgs<T> a = e;
      a.g = m.g;
      a.p.ih = (T)(1.0 / m.h);
      a.K = c->arr<T>(m.oK);
      a.G = c->arr<T>(m.oG);
      for (int d = 0; d < 3; ++d) {
        a.z[d] = c->arr<T>(xin[d]);
        a.u[d] = c->arr<T>(xin[d]);      // not read
        a.jr[d] = c->arr<T>(m.ob[d]);
        a.dinv[d] = c->arr<T>(m.odi[d]);
        a.o1[d] = c->arr<T>(xout[d]);
      }
      a.part = part;
      a.kz = m.kz;
      a.omega = omega;
      a.scal = c->scal();
      mg_lo_args(c, m, a);
      if constexpr (DIM == 3)
        timed_launch(c, l == 0 ? PF_K_SMOOTH : PF_K_PRECOND, j, k_apply3<T, kApplyBY, APPLY_SMOOTH>, m.grid,
                     dim3(ApplyTile<kApplyBY>::NTB), 0, st, a);
      else
        timed_launch(c, l == 0 ? PF_K_SMOOTH : PF_K_PRECOND, j, k_apply2s<T, APPLY_SMOOTH>, m.grid, dim3(A2W), 0, st,
                     a);
    };
    // the first two sweeps from zero in one pass
    auto sweep0 = [&](int l, const size_t (&xout)[3]) {
      const Layout::MGLevel& m = L.mg[l];
      ElastArgs<T> a = e;
      a.g = m.g;
      a.p.ih = (T)(1.0 / m.h);
      a.K = c->arr<T>(m.oK);
      a.G = c->arr<T>(m.oG);
      for (int d = 0; d < 3; ++d) {
        a.z[d] = c->arr<T>(m.ob[d]);        // not read
        a.u[d] = c->arr<T>(m.odi[d]);       // not read
        a.jr[d] = c->arr<T>(m.ob[d]);
        a.dinv[d] = c->arr<T>(m.odi[d]);
        a.o1[d] = c->arr<T>(xout[d]);
      }
      a.part = part;
      a.kz = m.kz;
      a.omega0 = kStep[0];
      a.omega = kStep[1];
      a.scal = c->scal();
      mg_lo_args(c, m, a);
      if constexpr (DIM == 3)
        timed_launch(c, l == 0 ? PF_K_SMOOTH : PF_K_PRECOND, j, k_apply3<T, kApplyBY, APPLY_SMOOTH0>, m.grid,
                     dim3(ApplyTile<kApplyBY>::NTB), 0, st, a);
      else
        timed_launch(c, l == 0 ? PF_K_SMOOTH : PF_K_PRECOND, j, k_apply2s<T, APPLY_SMOOTH0>, m.grid, dim3(A2W), 0, st,
                     a);
    };
    // 2D: the levels from mg_tail on run in one single-block launch
    const int tail = DIM == 2 ? L.mg_tail : -1;
    const int down_end = tail > 0 ? tail : last;
    for (int l = 0; l < down_end; ++l) {         // pre-smoothing and restriction, down to the coarsest
      const Layout::MGLevel& m = L.mg[l];
      sweep0(l, m.ox);
      sweep(l, m.ox, m.orr, 0.0);
      const Layout::MGLevel& mc = L.mg[l + 1];
      timed_launch(c, PF_K_PRECOND, j, DIM == 3 ? k_mg_restrict<T> : k_mg_restrict2<T>, mg_cell_blocks(mc.g), dim3(NT),
                   0, st, m.g, mc.g, mg_cvec(c, m.orr), mg_vec(c, mc.ob), scal);
    }
    static_assert(kCoarseSweeps % 2 == 0, "the coarsest sweeps end in x");
    if (tail > 0) {                              // the small levels' whole cycle in one launch
      timed_launch(c, PF_K_PRECOND, j, k_mg_tail2<T>, dim3(1), dim3(kTailNT), 0, st,
                   (const MGTailArgs<T>*)c->arr<MGTailArgs<T>>(L.o_mg_tail));
    } else if (DIM == 3 && last >= 1 &&
               (long)L.mg[last].g.nx * L.mg[last].g.ny * L.mg[last].g.nz <= kCoarseLdsCells * 4 / (long)sizeof(T)) {
      // a small coarsest level (not the solve's own grid, whose last sweep
      // forms the r.z partials): its sweeps in one block, in LDS
      const Layout::MGLevel& m = L.mg[last];
      CoarseArgs<T> ca{};
      ca.g = m.g;
      ca.ih = (T)(1.0 / m.h);
      ca.K = c->arr<T>(m.oK);
      ca.G = c->arr<T>(m.oG);
      for (int d = 0; d < 3; ++d) {
        ca.b[d] = c->arr<T>(m.ob[d]);
        ca.dinv[d] = c->arr<T>(m.odi[d]);
        ca.x[d] = c->arr<T>(m.ox[d]);
      }
      ca.s0 = (T)kStep[0];
      ca.s1 = (T)kStep[1];
      ca.sweeps = kCoarseSweeps;
      ca.scal = scal;
      timed_launch(c, PF_K_PRECOND, j, k_mg_coarse3<T>, dim3(1), dim3(kCoarseNT), 0, st, ca);
    } else {                                     // coarsest level: a fixed number of sweeps from zero
      const Layout::MGLevel& m = L.mg[last];
      sweep0(last, m.ox);
      for (int s = 2; s < kCoarseSweeps; ++s) {
        if (s & 1) sweep(last, m.oxt, m.ox, kStep[1]);
        else sweep(last, m.ox, m.oxt, kStep[0]);
      }
    }
    for (int l = down_end - 1; l >= 0; --l) {    // prolongation and post-smoothing, up to the solve's grid
      const Layout::MGLevel& m = L.mg[l];
      const Layout::MGLevel& mc = L.mg[l + 1];
      timed_launch(c, PF_K_PRECOND, j, DIM == 3 ? k_mg_prolong<T> : k_mg_prolong2<T>,
                   DIM == 3 ? mg_pair_blocks(m.g) : mg_cell_blocks(m.g), dim3(NT), 0,
                   st, m.g, mc.g, mg_cvec(c, mc.ox), mg_vec(c, m.ox), scal);
      sweep(l, m.ox, m.oxt, kStep[0]);
      sweep(l, m.oxt, m.ox, kStep[1]);           // level 0: z, with the partials of r.z
    }
    timed_launch(c, PF_K_PRECOND, j, k_mg_rz, dim3(1), dim3(NT), 0, st, (const double*)part, L.nb_mg,
                 c->arr<double>(L.o_part_u), n_rz, scal);
  }

  // Solve A u = b for the current phase fields and plastic strain.
  static pf_status solve(pf_ctx* c, int warm) {
    const Layout& L = c->L;
    hipStream_t st = c->stream;
    // Every launch of this solve stays in the pending list until it is
    // retagged below: flush (which waits for the stream) when the event pool
    // might not hold a solve of twice the recent iteration counts (a longer
    // one flushes when the pool is full; only its launches still pending are
    // then retagged).
    if (c->timing) {
      const long long expect = 2LL * std::max(c->last_iters, c->prev_iters) + 64;
      const long long need = 4LL * (2LL * std::min<long long>(c->cfg.cg_max_iter, expect) + 256);
      if (c->ev_next + need > (long long)c->ev_pool.size()) {
        HIPCHK(c, hipStreamSynchronize(st));
        timing_flush(c);
      }
    }
    ++c->solves;
    const size_t pend0 = c->pending.size();
    const long long flush0 = c->n_flush;
    if (warm == PF_WARM_ZERO)
      for (int d = 0; d < DIM; ++d) HIPCHK(c, hipMemsetAsync(c->ws + L.o_u[d], 0, (size_t)L.g.n * sizeof(T), st));
    c->warm_used = warm;
    CellArgs<T> ca = cell_args(c);
    if constexpr (DIM != 3)           // 3D: the set-up pass evaluates the moduli itself
      timed_launch(c, PF_K_OTHER, -1, k_moduli<T, DIM>, L.gcell, dim3(NT), 0, st, ca);

    ElastArgs<T> e = elast_args(c);
    double* part_u = c->arr<double>(L.o_part_u);
    double* part_a = c->arr<double>(L.o_part_a);
    double* part_b = c->arr<double>(L.o_part_b);
    if constexpr (DIM == 3) {
      // b, D^-1 and the partials of ||b||^2 in one pass; then, on the apply
      // kernel, q = A u with r = b - q, z = D^-1 r and the partials CG starts
      // from formed in its epilogue (q itself is not stored)
      ElastArgs<T> sa = e;
      sa.part = part_b;
      sa.phi_w = c->arr<T>(L.o_fld[c->cur][1]);
      sa.Kw = c->arr<T>(L.o_K);
      sa.Gw = c->arr<T>(L.o_G);
      for (int d = 0; d < 3; ++d) {
        sa.o1[d] = c->arr<T>(L.o_b[d]);
        sa.dinv[d] = c->arr<T>(L.o_di[d]);
      }
      sa.kz = L.kz_ap;
      if (sizeof(T) == 4 && L.mg_n > 0)          // the multigrid sweeps' bf16 copies of level 0
        for (int a = 0; a < 5; ++a) sa.lo_w[a] = c->arr<unsigned short>(L.mg[0].olo[a]);
      timed_launch(c, PF_K_SOLVE_SETUP, -1, k_setup3<T, kApplyBY>, L.gap, dim3(ApplyTile<kApplyBY>::NTB), 0, st, sa);
      ElastArgs<T> ra = e;
      ra.kz = L.kz_ap;
      for (int d = 0; d < 3; ++d) {
        ra.z[d] = c->arr<T>(L.o_u[d]);      // the vector applied
        ra.u[d] = c->arr<T>(L.o_u[d]);      // not read; zeroed when b = 0
        ra.jr[d] = c->arr<T>(L.o_b[d]);
        ra.dinv[d] = c->arr<T>(L.o_di[d]);
        ra.o1[d] = c->arr<T>(L.o_r[d]);
        ra.o2[d] = c->arr<T>(L.o_z[d]);
      }
      ra.part_in = part_b;
      ra.n_in = L.nb_res;                   // the set-up pass's ||b||^2 partials
      ra.part = part_u;
      ra.scal = c->scal();
      timed_launch(c, PF_K_SOLVE_SETUP, -1, k_apply3<T, kApplyBY, APPLY_RESID>, L.gap, dim3(ApplyTile<kApplyBY>::NTB), 0, st, ra);
      LAUNCHCHK(c);
    } else {
      // ||b||^2
      e.part = part_b;
      timed_launch(c, PF_K_SOLVE_SETUP, -1, k_elast<T, DIM, M_BNORM>, L.gel, dim3(NT), 0, st, e);
      // r = b - A u, D^-1, z, and the partials of r.z and r.r
      ElastArgs<T> r = e;
      for (int d = 0; d < DIM; ++d) {
        r.u[d] = c->arr<T>(L.o_u[d]);
        r.o1[d] = c->arr<T>(L.o_r[d]);
        r.o2[d] = c->arr<T>(L.o_z[d]);
        r.dinv[d] = c->arr<T>(L.o_di[d]);
      }
      r.part_in = part_b;
      r.n_in = L.nb_el;
      r.part = part_u;
      timed_launch(c, PF_K_SOLVE_SETUP, -1, k_elast<T, DIM, M_RESID>, L.gel, dim3(NT), 0, st, r);
      LAUNCHCHK(c);
    }
    c->warm_used = warm == PF_WARM_LEARNED ? PF_WARM_PREV : warm;
    if (warm == PF_WARM_LEARNED) {
      pf_status s = learned_start<T, DIM>(c, e, part_a);
      if (s != PF_OK) return s;
    }
    const bool mg = L.mg_n > 0;
    if (mg) {                       // z = M^-1 r of the starting residual
      mg_setup(c);
      mg_vcycle(c, e, -1, L.nb_res);
      LAUNCHCHK(c);
    }

    ElastArgs<T> ap = elast_args(c);
    UpdArgs<T> up{};
    up.n = L.g.n;
    up.scal = c->scal();
    up.part = part_u;
    up.part_in = part_a;
    up.n_in = L.nb_cg;
    for (int d = 0; d < DIM; ++d) {
      ap.z[d] = c->arr<T>(L.o_z[d]);
      ap.o2[d] = c->arr<T>(L.o_q[d]);
      up.u[d] = c->arr<T>(L.o_u[d]);
      up.r[d] = c->arr<T>(L.o_r[d]);
      up.q[d] = c->arr<T>(L.o_q[d]);
      up.dinv[d] = c->arr<T>(L.o_di[d]);
      up.z[d] = c->arr<T>(L.o_z[d]);
    }
    ap.part = part_a;
    ap.part_in = part_u;
    ap.kz = L.kz_cg;
    if constexpr (DIM == 3)   // the apply launch that stops the solve completes u
      for (int d = 0; d < 3; ++d) ap.xs[d] = c->arr<T>(L.o_u[d]);

    const int maxit = c->cfg.cg_max_iter;
    int launched = 0;
    bool conv = false;
    // Launches queued past convergence cost a few microseconds each, a check
    // (with its host synchronisation) some tens: the first chunk covers the
    // smaller of the last two counts, the second reaches the larger one, and
    // later chunks grow with what has been launched.  With the multigrid an
    // iteration queued past convergence is some 45 launches and a check is
    // cheap beside an iteration: the first chunk stops at the smaller count
    // (a solve that needs exactly that many ends there without a queued
    // iteration), the second at the larger, and later ones go one by one.
    const int p2 = c->prev_iters > 0 ? c->prev_iters : c->last_iters;
    const int lo = std::min(c->last_iters, p2), hi = std::max(c->last_iters, p2);
    const bool mg_chunks = L.mg_n > 0;
    int chunk = c->cg_chunk > 0 ? c->cg_chunk : mg_chunks ? std::max(1, lo) : std::max(2, lo + 2);
    int nchunk = 0;
    auto apply_cg = [&](int j) {       // the apply launch of CG iteration j
      const int par = j & 1;
      const size_t* pold = par ? L.o_pb : L.o_pa;
      const size_t* pnew = par ? L.o_pa : L.o_pb;
      for (int d = 0; d < DIM; ++d) {
        ap.u[d] = c->arr<T>(pold[d]);
        ap.o1[d] = c->arr<T>(pnew[d]);
        up.p[d] = c->arr<T>(pnew[d]);
        up.pp[d] = c->arr<T>(pold[d]);
      }
      ap.parity = par;
      ap.it = j;
      ap.n_in = j == 0 ? L.nb_res : L.nb_upd;
      up.parity = par;
      if constexpr (DIM == 3)
        timed_launch(c, PF_K_APPLY, j, k_apply3<T, kCgBY, APPLY_CG>, L.gcg, dim3(ApplyTile<kCgBY>::NTB), 0, st, ap);
      else
        timed_launch(c, PF_K_APPLY, j, k_apply2<T>, L.gap, dim3(A2W), 0, st, ap);
    };
    while (true) {
      int n = std::min(chunk, maxit - launched);
      for (int q = 0; q < n; ++q) {
        apply_cg(launched);
        if (mg) {
          timed_launch(c, PF_K_UPDATE, launched, k_cg_update<T, DIM, true>, dim3(L.nb_upd), dim3(NT), 0, st, up);
          mg_vcycle(c, e, launched, L.nb_upd);
        } else {
          timed_launch(c, PF_K_UPDATE, launched, k_cg_update<T, DIM>, dim3(L.nb_upd), dim3(NT), 0, st, up);
        }
        ++launched;
      }
      timed_launch(c, PF_K_OTHER, -1, k_cg_check, dim3(1), dim3(NT), 0, st, (const double*)part_u,
                   launched == 0 ? L.nb_res : L.nb_upd, c->scal(), c->cfg.cg_rtol * c->cfg.cg_rtol,
                   DIM == 3 ? (double)(launched + 1) : 1.0);
      LAUNCHCHK(c);
      HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal(), S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipStreamSynchronize(st));
      if (c->host_scal[S_CONV] != 0.0) {
        conv = true;
        // 3D: the check found the last update converged; the apply launch
        // it marked adds that update's alpha p to u and stops
        if (DIM == 3 && c->host_scal[S_CONV] == (double)(launched + 1)) {
          apply_cg(launched);
          LAUNCHCHK(c);
        }
        break;
      }
      if (launched >= maxit) {
        if constexpr (DIM == 3) {   // not converged: u still gets the last update's alpha p
          timed_launch(c, PF_K_OTHER, -1, k_cg_check, dim3(1), dim3(NT), 0, st, (const double*)part_u, L.nb_upd,
                       c->scal(), -1.0, (double)(launched + 1));
          apply_cg(launched);
          LAUNCHCHK(c);
        }
        break;
      }
      ++nchunk;
      if (c->cg_chunk > 0) continue;
      if (mg_chunks)
        chunk = nchunk == 1 && hi > launched ? hi - launched : 1;
      else
        chunk = nchunk == 1 && hi + 2 > launched ? hi + 2 - launched : std::max(4, std::min(64, launched / 4));
    }
    c->prev_iters = c->last_iters;
    c->last_iters = (int)c->host_scal[S_ITERS];
    c->iters_total += c->last_iters;
    if (c->judged) {
      const double* hs = c->host_scal;
      c->r0_learned = hs[S_BB] > 0.0 ? std::sqrt(hs[S_JL] / hs[S_BB]) : 0.0;
      c->r0_prev = hs[S_BB] > 0.0 ? std::sqrt(hs[S_JP] / hs[S_BB]) : 0.0;
      if (hs[S_JB] != 0.0) c->warm_used = PF_WARM_LEARNED;
    } else {
      c->r0_learned = 0.0;
      c->r0_prev = 0.0;
    }
    // launches queued past convergence exit at entry: account them as small
    // kernels (only this solve's entries; after a flush inside a very long
    // solve, the ones still pending)
    for (size_t q = c->n_flush == flush0 ? pend0 : 0; q < c->pending.size(); ++q) {
      auto& pr = c->pending[q];
      if (pr.launch >= c->last_iters && (pr.kind == PF_K_APPLY || pr.kind == PF_K_UPDATE || pr.kind == PF_K_PRECOND ||
                                         pr.kind == PF_K_SMOOTH))
        pr.kind = PF_K_OTHER;
    }
    // true residual ||b - A u|| (3D: the apply kernel's ||b - q||^2 partials)
    int n_true = L.nb_el;
    if constexpr (DIM == 3) {
      const T* bvec[3] = {c->arr<T>(L.o_b[0]), c->arr<T>(L.o_b[1]), c->arr<T>(L.o_b[2])};
      apply_plain(c, e, c->arr<T>(L.o_u[0]), c->arr<T>(L.o_u[1]), c->arr<T>(L.o_u[2]), part_b, bvec);
      n_true = (int)(L.gap.x * L.gap.y * L.gap.z);
    } else {
      ElastArgs<T> t = e;
      for (int d = 0; d < DIM; ++d) t.u[d] = c->arr<T>(L.o_u[d]);
      t.part = part_b;
      timed_launch(c, PF_K_SOLVE_SETUP, -1, k_elast<T, DIM, M_TRUE>, L.gel, dim3(NT), 0, st, t);
    }
    timed_launch(c, PF_K_OTHER, -1, k_sum_to, dim3(1), dim3(NT), 0, st, (const double*)part_b, n_true, c->scal(), (int)S_TRUE);
    LAUNCHCHK(c);
    if (!conv)
      return fail(c, PF_ERR_CG_NOT_CONVERGED, "CG did not reach rtol %.3g in %d iterations", c->cfg.cg_rtol, maxit);
    if (warm == PF_WARM_LEARNED) return learned_after_solve<T, DIM>(c);
    return PF_OK;
  }

  static SpArgs<T> sp_args(pf_ctx* c) {
    const Layout& L = c->L;
    SpArgs<T> a{};
    a.g = L.g;
    a.dt_ih2 = (T)(c->cfg.dt / (c->cfg.h * c->cfg.h));
    a.dirichlet = c->cfg.dirichlet;
    for (int q = 0; q < 3; ++q) {
      a.D[q] = c->arr<T>(L.o_sp[0][q]);
      a.dinv[q] = c->arr<T>(L.o_sp[1][q]);
      a.r[q] = c->arr<T>(L.o_sp[2][q]);
      a.z[q] = c->arr<T>(L.o_sp[3][q]);
      a.pa[q] = c->arr<T>(L.o_sp[4][q]);
      a.pb[q] = c->arr<T>(L.o_sp[5][q]);
      a.q[q] = c->arr<T>(L.o_sp[6][q]);
      a.d[q] = c->arr<T>(L.o_sp[7][q]);
    }
    a.nb = L.nb_sp;
    a.part_rr = c->arr<double>(L.o_sp_part);
    a.part_pq = a.part_rr + 6 * (size_t)L.nb_sp;
    a.sc = c->arr<double>(L.o_sp_scal);
    a.tol2 = c->cfg.species_rtol * c->cfg.species_rtol;
    return a;
  }

  // The three species' CG solves (I + dt A_s) d_s = b_s, side by side: every
  // chunk of apply / update launches is followed by a convergence test the
  // host reads (a synchronisation per chunk).
  static pf_status species_solve(pf_ctx* c) {
    const Layout& L = c->L;
    hipStream_t st = c->stream;
    SpArgs<T> a = sp_args(c);
    timed_launch(c, PF_K_SPECIES, -1, k_sp_init<T, DIM>, dim3(L.nb_sp), dim3(NT), 0, st, a);
    const int maxit = c->cfg.species_max_iter;
    int it = 0;
    int chunk = std::max(4, c->sp_last_iters + 1);
    while (true) {
      const int n = std::min(chunk, maxit - it);
      for (int q = 0; q < n; ++q, ++it) {
        a.it = it;
        timed_launch(c, PF_K_SPECIES, -1, k_sp_apply<T, DIM>, dim3(L.nb_sp), dim3(NT), 0, st, a);
        timed_launch(c, PF_K_SPECIES, -1, k_sp_update<T, DIM>, dim3(L.nb_sp), dim3(NT), 0, st, a);
      }
      hipLaunchKernelGGL(k_sp_check, dim3(1), dim3(NT), 0, st, (const double*)a.part_rr, L.nb_sp, a.sc, a.tol2, 0);
      LAUNCHCHK(c);
      HIPCHK(c, hipMemcpyAsync(c->host_sp, a.sc, SP_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipStreamSynchronize(st));
      const double* h = c->host_sp;
      if (h[SP_CONV] != 0.0 && h[SP_CONV + 1] != 0.0 && h[SP_CONV + 2] != 0.0) break;
      if (it >= maxit)
        return fail(c, PF_ERR_CG_NOT_CONVERGED, "implicit species CG did not reach rtol %.3g in %d iterations",
                    c->cfg.species_rtol, maxit);
      chunk = std::max(4, std::min(64, it / 4));
    }
    const double* h = c->host_sp;
    c->sp_last_iters = (int)std::max(h[SP_ITERS], std::max(h[SP_ITERS + 1], h[SP_ITERS + 2]));
    return PF_OK;
  }

  static pf_status step_once(pf_ctx* c) {
    const Layout& L = c->L;
    if (!c->ledger_valid) {
      pf_status s = ledger_reset(c);
      if (s != PF_OK) return s;
    }
    if (c->cfg.mechanics) {
      pf_status s = solve(c, c->cfg.warm);
      if (s != PF_OK) return s;
    }
    CellArgs<T> a = cell_args(c);
    a.part = c->arr<double>(L.o_part_c);
    if (c->fs) {
      pf_status s = fs_couple(c, L.g, a.pf, a.pw, L.es == 4 ? (const void*)a.lo[0] : nullptr,
                              L.es == 4 ? (const void*)a.lo[1] : nullptr, (int)sizeof(T), &a.gext);
      if (s != PF_OK) return s;
    }
    timed_launch(c, PF_K_MU, -1, k_mu<T, DIM>, L.gcell, dim3(NT), 0, c->stream, a);
    int ln = L.nb_cell;                // partials of the field update
    if (DIM == 3 && !c->cfg.species_implicit) {
      // 3D: the LDS plane-tile kernel (64 x 8 tiles)
      const dim3 g3((L.g.nx + TX - 1) / TX, (L.g.ny + S3_BY - 1) / S3_BY, L.g.nz);
      ln = (int)(g3.x * g3.y * g3.z);
      timed_launch(c, PF_K_STEP, -1, k_step3<T>, g3, dim3(S3_NT), 0, c->stream, a);
    } else {
      timed_launch(c, PF_K_STEP, -1, k_step<T, DIM>, L.gcell, dim3(NT), 0, c->stream, a);
    }
    if (c->cfg.species_implicit) {
      pf_status s = species_solve(c);
      if (s != PF_OK) return s;
      timed_launch(c, PF_K_SPECIES, -1, k_sp_finish<T, DIM>, L.gcell, dim3(NT), 0, c->stream, a, sp_args(c));
    }
    double vol = std::pow(c->cfg.h, DIM), area = std::pow(c->cfg.h, DIM - 1);
    const double* lp = a.part;
    if (ln > 8 * kFoldBlocks) {         // many partials: fold them on kFoldBlocks blocks first
      double* fold = c->arr<double>(L.o_part_f);
      timed_launch(c, PF_K_OTHER, -1, k_fold_step, dim3(kFoldBlocks), dim3(NT), 0, c->stream, (const double*)a.part, ln,
                   fold, kFoldBlocks);
      lp = fold;
      ln = kFoldBlocks;
    }
    timed_launch(c, PF_K_OTHER, -1, k_ledger, dim3(1), dim3(NT), 0, c->stream, lp, ln, c->scal(), vol,
                 area * c->cfg.dt, 1);
    LAUNCHCHK(c);
    c->cur ^= 1;
    c->steps += 1;
    return PF_OK;
  }
};

template <typename F>
static pf_status dispatch(pf_ctx* c, F&& f) {
  if (c->cfg.precision == PF_FP64) {
    if (c->cfg.dim == 2) return f(Impl<double, 2>());
    return f(Impl<double, 3>());
  }
  if (c->cfg.dim == 2) return f(Impl<float, 2>());
  return f(Impl<float, 3>());
}

static void fill_stats(pf_ctx* c, pf_step_stats* s) {
  const double* h = c->host_scal;
  memset(s, 0, sizeof(*s));
  s->cg_iters = (int)h[S_ITERS];
  s->warm_used = c->warm_used;
  s->cg_rel_resid = h[S_BB] > 0.0 ? std::sqrt(h[S_TRUE] / h[S_BB]) : 0.0;
  s->O_tot = h[S_OTOT];
  s->O_out = h[S_OOUT];
  s->O_drift = h[S_O0] != 0.0 ? (h[S_OTOT] + h[S_OOUT] - h[S_O0]) / h[S_O0] : 0.0;
  s->H_tot = h[S_HTOT];
  s->H_out = h[S_HOUT];
  s->H_drift = h[S_H0] != 0.0 ? (h[S_HTOT] + h[S_HOUT] - h[S_H0]) / h[S_H0] : 0.0;
  s->red_degree = h[S_XO0] != 0.0 ? 1.0 - h[S_XOSUM] / h[S_XO0] : 0.0;
  s->max_vm = h[S_MAXVM];
  s->max_epsP = h[S_MAXEP];
  s->step = c->steps;
  s->nonfinite = (int)h[S_NONFIN];
  s->cg_iters_total = c->iters_total;
  s->r0_learned = c->r0_learned;
  s->r0_prev = c->r0_prev;
  s->species_iters = c->sp_last_iters;
  if (c->fs) {                         // the mechanics of the step was the finite-strain solve
    s->cg_iters = c->fs_last.cg_iters;
    s->cg_rel_resid = c->fs_last.rel_resid;
    s->max_vm = c->fs_last.max_vm;
    s->max_epsP = c->fs_last.max_epsP;
  }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t pf_workspace_bytes(const pf_config* cfg) {
  char msg[256];
  if (!valid_cfg(cfg, msg, sizeof msg)) return 0;
  return make_layout(cfg).total;
}

pf_status pf_init(const pf_config* cfg, const pf_params* params, void* workspace, size_t workspace_bytes,
                  void* hip_stream, pf_ctx** out) {
  if (!out) return fail(nullptr, PF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  char msg[256];
  if (!valid_cfg(cfg, msg, sizeof msg)) return fail(nullptr, PF_ERR_INVALID_ARG, "%s", msg);
  if (!params) return fail(nullptr, PF_ERR_INVALID_ARG, "params is NULL");
  if (params->m_form != 0 && params->m_form != 1) return fail(nullptr, PF_ERR_INVALID_ARG, "m_form must be 0 or 1");
  if (!workspace) return fail(nullptr, PF_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(nullptr, PF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Layout L = make_layout(cfg);
  if (workspace_bytes < L.total)
    return fail(nullptr, PF_ERR_OOM, "workspace has %zu bytes, %zu needed", workspace_bytes, L.total);
  pf_ctx* c = new (std::nothrow) pf_ctx();
  if (!c) return fail(nullptr, PF_ERR_OOM, "host allocation failed");
  c->cfg = *cfg;
  c->prm = *params;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->L = L;
  c->ws = reinterpret_cast<char*>(workspace);
  c->err[0] = 0;
  c->bad = false;
  c->ledger_valid = false;
  c->mg_tail_ready = false;
  c->cur = 0;
  c->steps = 0;
  c->last_iters = 0;
  c->prev_iters = 0;
  c->cg_chunk = 0;
  c->warm_used = cfg->warm;
  c->timing = 0u;
  c->timing_every = 1;
  c->solves = 0;
  c->ev_next = 0;
  c->n_flush = 0;
  c->iters_total = 0;
  c->net = nullptr;
  c->have_prev_incr = false;
  c->judged = false;
  c->r0_learned = 0.0;
  c->r0_prev = 0.0;
  c->sp_last_iters = 0;
  for (int k = 0; k < PF_K_COUNT; ++k) { c->t_ms[k] = 0.0; c->t_n[k] = 0; }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_scal), (S_COUNT + SP_COUNT) * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return fail(nullptr, PF_ERR_HIP, "hipHostMalloc of the stats block failed");
  }
  memset(c->host_scal, 0, (S_COUNT + SP_COUNT) * sizeof(double));
  c->host_sp = c->host_scal + S_COUNT;
  hipError_t e = hipMemsetAsync(c->ws, 0, L.total, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    (void)hipHostFree(c->host_scal);
    delete c;
    return fail(nullptr, PF_ERR_HIP, "clearing the workspace failed: %s", hipGetErrorString(e));
  }
  *out = c;
  return PF_OK;
}

pf_status pf_step(pf_ctx* c, int nsteps, pf_step_stats* last) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (c->bad) return fail(c, PF_ERR_BAD_STATE, "context failed earlier; set the fields to restore it");
  if (nsteps < 0) return fail(c, PF_ERR_INVALID_ARG, "nsteps < 0");
  for (int s = 0; s < nsteps; ++s) {
    pf_status st = dispatch(c, [&](auto impl) { return decltype(impl)::step_once(c); });
    if (st != PF_OK) { c->bad = true; return st; }
  }
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal(), S_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  pf_step_stats s;
  fill_stats(c, &s);
  if (last) *last = s;
  if (nsteps > 0 && s.nonfinite > 0) {
    c->bad = true;
    return fail(c, PF_ERR_NONFINITE, "%d cells hold non-finite values after step %lld", s.nonfinite, c->steps);
  }
  if (nsteps > 0 && c->cfg.ledger_tol > 0.0 && std::fabs(s.O_drift) > c->cfg.ledger_tol) {
    c->bad = true;
    return fail(c, PF_ERR_LEDGER, "oxygen ledger drift %.3e exceeds %.3e", s.O_drift, c->cfg.ledger_tol);
  }
  return PF_OK;
}

pf_status pf_mech_solve(pf_ctx* c, int warm, pf_step_stats* stats) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (c->bad) return fail(c, PF_ERR_BAD_STATE, "context failed earlier; set the fields to restore it");
  if (warm != PF_WARM_ZERO && warm != PF_WARM_PREV && warm != PF_WARM_LEARNED)
    return fail(c, PF_ERR_INVALID_ARG, "unknown warm start %d", warm);
  if (warm == PF_WARM_LEARNED && c->cfg.warm != PF_WARM_LEARNED)
    return fail(c, PF_ERR_INVALID_ARG, "the context was not created with the learned warm start");
  if (!c->cfg.mechanics) return fail(c, PF_ERR_INVALID_ARG, "mechanics is off in this context");
  pf_status st = dispatch(c, [&](auto impl) { return decltype(impl)::solve(c, warm); });
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal(), S_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (stats) fill_stats(c, stats);
  return st;
}

pf_status pf_ledger_reset(pf_ctx* c) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  pf_status st = dispatch(c, [&](auto impl) { return decltype(impl)::ledger_reset(c); });
  if (st != PF_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PF_OK;
}

pf_status pf_fields(pf_ctx* c, int field_id, int dir, void* ptr, size_t nbytes, int ptr_is_device) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (!ptr) return fail(c, PF_ERR_INVALID_ARG, "ptr is NULL");
  if (dir != 0 && dir != 1) return fail(c, PF_ERR_INVALID_ARG, "dir must be 0 (get) or 1 (set)");
  const Layout& L = c->L;
  const Grid& g = L.g;
  const int dim = c->cfg.dim;
  int cx = g.nx, cy = g.ny, cz = g.nz, zaxis = -1, ncomp = 1;
  size_t base = 0, base_lo = 0;
  switch (field_id) {
    case PF_FIELD_PHI_F: case PF_FIELD_PHI_W: case PF_FIELD_XO: case PF_FIELD_XH: case PF_FIELD_XW:
      base = L.o_fld[c->cur][field_id];
      base_lo = L.o_lo[c->cur][field_id];
      break;
    case PF_FIELD_UX: base = L.o_u[0]; cx += 1; zaxis = 0; break;
    case PF_FIELD_UY: base = L.o_u[1]; cy += 1; zaxis = 1; break;
    case PF_FIELD_UZ:
      if (dim != 3) return fail(c, PF_ERR_INVALID_ARG, "u_z exists only in 3D");
      base = L.o_u[2]; cz += 1; zaxis = 2; break;
    case PF_FIELD_EPSP: base = L.o_epsp; ncomp = L.nc; break;
    case PF_FIELD_EPSP_ACC: base = L.o_epsP; break;
    default: return fail(c, PF_ERR_INVALID_ARG, "unknown field id %d", field_id);
  }
  size_t per = (size_t)cx * cy * cz;
  if (nbytes != per * ncomp * sizeof(double))
    return fail(c, PF_ERR_INVALID_ARG, "field %d needs %zu bytes, got %zu", field_id, per * ncomp * sizeof(double), nbytes);
  double* stage = c->arr<double>(L.o_stage);
  const int nthr = 256;
  const int nblk = (int)((per + nthr - 1) / nthr);
  for (int comp = 0; comp < ncomp; ++comp) {
    size_t dev_off = base + (size_t)comp * g.n * L.es;   // plastic strain components are g.n elements apart
    char* user = reinterpret_cast<char*>(ptr) + comp * per * sizeof(double);
    double* buf = ptr_is_device ? reinterpret_cast<double*>(user) : stage;
    if (dir == 1) {
      if (!ptr_is_device) HIPCHK(c, hipMemcpyAsync(stage, user, per * sizeof(double), hipMemcpyHostToDevice, c->stream));
      if (L.es == 8)
        hipLaunchKernelGGL(k_unpack<double>, dim3(nblk), dim3(nthr), 0, c->stream, (const double*)buf, c->arr<double>(dev_off), g, cx, cy, cz, zaxis);
      else if (base_lo)
        hipLaunchKernelGGL(k_unpack_pair, dim3(nblk), dim3(nthr), 0, c->stream, (const double*)buf, c->arr<float>(dev_off),
                           c->arr<float>(base_lo), g, cx, cy, cz);
      else
        hipLaunchKernelGGL(k_unpack<float>, dim3(nblk), dim3(nthr), 0, c->stream, (const double*)buf, c->arr<float>(dev_off), g, cx, cy, cz, zaxis);
      LAUNCHCHK(c);
    } else {
      if (L.es == 8)
        hipLaunchKernelGGL(k_pack<double>, dim3(nblk), dim3(nthr), 0, c->stream, (const double*)c->arr<double>(dev_off), buf, g, cx, cy, cz);
      else if (base_lo)
        hipLaunchKernelGGL(k_pack_pair, dim3(nblk), dim3(nthr), 0, c->stream, (const float*)c->arr<float>(dev_off),
                           (const float*)c->arr<float>(base_lo), buf, g, cx, cy, cz);
      else
        hipLaunchKernelGGL(k_pack<float>, dim3(nblk), dim3(nthr), 0, c->stream, (const float*)c->arr<float>(dev_off), buf, g, cx, cy, cz);
      LAUNCHCHK(c);
      if (!ptr_is_device) HIPCHK(c, hipMemcpyAsync(user, stage, per * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
  }
  if (dir == 1) {
    c->bad = false;
    c->have_prev_incr = false;
    if (field_id <= PF_FIELD_XW) c->ledger_valid = false;
  }
  if (dir == 0 || !ptr_is_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  return PF_OK;
}

pf_status pf_timing(pf_ctx* c, int kinds) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (kinds & ~PF_TIMING_ALL) return fail(c, PF_ERR_INVALID_ARG, "timing mask 0x%x has bits beyond the kernel kinds", kinds);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  timing_flush(c);
  if (kinds) {
    if (c->ev_pool.empty()) {
      c->ev_pool.resize(32768);
      // timing-only events: no system-scope fence (cache write-back and
      // invalidation) at each record, which would slow the next kernel; every
      // read of them follows a stream synchronisation
      for (auto& e : c->ev_pool) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    for (int k = 0; k < PF_K_COUNT; ++k) { c->t_ms[k] = 0.0; c->t_n[k] = 0; }
  }
  c->timing = (unsigned)kinds;
  return PF_OK;
}

pf_status pf_timing_every(pf_ctx* c, int every) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (every < 1) return fail(c, PF_ERR_INVALID_ARG, "every must be >= 1");
  c->timing_every = every;
  return PF_OK;
}

pf_status pf_cg_chunk(pf_ctx* c, int n) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 0) return fail(c, PF_ERR_INVALID_ARG, "chunk must be >= 0");
  c->cg_chunk = n;
  return PF_OK;
}

pf_status pf_timing_get(pf_ctx* c, int kind, double* total_ms, long long* launches) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (kind < 0 || kind >= PF_K_COUNT) return fail(c, PF_ERR_INVALID_ARG, "unknown kernel kind %d", kind);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  timing_flush(c);
  if (total_ms) *total_ms = c->t_ms[kind];
  if (launches) *launches = c->t_n[kind];
  return PF_OK;
}

const char* pf_last_error(const pf_ctx* c) { return c ? c->err : g_err; }

void pf_destroy(pf_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  delete c;
}

}  // extern "C"

#include "pf_batch_api.h"
#include "pf_nn_api.h"
#include "pf_fs_api.h"
