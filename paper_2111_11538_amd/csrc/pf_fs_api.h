// Host side of the finite-strain mechanics (pf_fs_* in include/pf.h).
// Included at the end of pf_api.hip.
#pragma once

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "pf_fs.h"

using pfs::FSGrid;

struct pf_fs {
  pf_fs_config cfg;
  pfs::FSP p;
  FSGrid g;
  hipStream_t stream;
  int nb;                  // blocks of the grid-stride kernels (partials per quantity)
  long long nd;            // d * nodes
  double *pf, *pw, *u, *uold, *R, *x, *r, *z, *pd, *q, *dinv, *Fp, *epsP, *drive, *ef, *part, *sc;
  double* host;            // pinned copy of the scalars
  bool fp_identity;        // every F_P is the identity (the element kernels skip loading it)
  // timing: event pairs around launches, resolved at the next synchronisation
  bool timing;
  std::vector<hipEvent_t> ev;
  std::vector<std::pair<int, int>> pend;   // (kind, first event)
  int ev_used;
  double t_ms[PF_FS_K_COUNT];
  long long t_n[PF_FS_K_COUNT];
  char err[512];
};

static void fs_flush(pf_fs* f) {
  for (auto& pr : f->pend) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, f->ev[pr.second], f->ev[pr.second + 1]) == hipSuccess) {
      f->t_ms[pr.first] += ms;
      f->t_n[pr.first] += 1;
    }
  }
  f->pend.clear();
  f->ev_used = 0;
}

// Launch through `launch`, bracketed by events of class `kind` when timing is on.
template <typename L>
static void fs_timed(pf_fs* f, int kind, L&& launch) {
  if (!f->timing) {
    launch();
    return;
  }
  if (f->ev_used + 2 > (int)f->ev.size()) {
    (void)hipStreamSynchronize(f->stream);
    fs_flush(f);
  }
  const int i = f->ev_used;
  (void)hipEventRecord(f->ev[i], f->stream);
  launch();
  (void)hipEventRecord(f->ev[i + 1], f->stream);
  f->pend.emplace_back(kind, i);
  f->ev_used += 2;
}

static char g_fs_err[512] = "";

static pf_status fs_fail(pf_fs* f, pf_status s, const char* fmt, ...) {
  char* dst = f ? f->err : g_fs_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return s;
}

#define FSCHK(f, call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fs_fail((f), PF_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define FSLAUNCH(f)                                                                                        \
  do {                                                                                                     \
    hipError_t e_ = hipGetLastError();                                                                     \
    if (e_ != hipSuccess) return fs_fail((f), PF_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_));     \
  } while (0)

static bool fs_valid(const pf_fs_config* c) {
  if (!c || (c->dim != 2 && c->dim != 3)) return false;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1 || (c->dim == 2 && c->nz != 1)) return false;
  if (!(c->h > 0.0) || !(c->newton_rtol > 0.0) || !(c->cg_rtol > 0.0)) return false;
  if (c->newton_max_iter < 1 || c->cg_max_iter < 1) return false;
  const double cells = (double)c->nx * c->ny * c->nz;
  return cells * 8.0 * (1 << c->dim) < 9.0e18 && (double)(c->nx + 1) * (c->ny + 1) * (c->nz + 1) < 4.0e9;
}

static FSGrid fs_grid(const pf_fs_config* c) {
  FSGrid g;
  g.nx = c->nx;
  g.ny = c->ny;
  g.nz = c->nz;
  g.mx = c->nx + 1;
  g.my = c->ny + 1;
  g.mz = c->dim == 3 ? c->nz + 1 : 1;
  g.ne = (long long)c->nx * c->ny * c->nz;
  g.nn = (long long)g.mx * g.my * g.mz;
  g.h = c->h;
  g.w = std::pow(c->h, c->dim) / (double)(1 << c->dim);
  return g;
}

static int fs_blocks(long long n) {
  long long b = (n + pfs::kFsThreads - 1) / pfs::kFsThreads;
  return (int)std::max(1LL, std::min<long long>(b, pfs::kFsBlocksMax));
}

// Carve the device arrays out of the workspace (256-byte aligned pieces);
// with base == nullptr only the size is computed.
static size_t fs_layout(pf_fs* f, const pf_fs_config* c, char* base) {
  const FSGrid g = fs_grid(c);
  const long long ngp = 1LL << c->dim;
  const long long nd = (long long)c->dim * g.nn;
  size_t off = 0;
  auto take = [&](double*& p, long long n) {
    if (base) p = reinterpret_cast<double*>(base + off);
    off += (std::max<size_t>((size_t)n * 8, 256) + 255) / 256 * 256;
  };
  pf_fs tmp{};
  pf_fs* t = f ? f : &tmp;
  take(t->pf, g.ne);
  take(t->pw, g.ne);
  take(t->u, nd);
  take(t->uold, nd);
  take(t->R, nd);
  take(t->x, nd);
  take(t->r, nd);
  take(t->z, nd);
  take(t->pd, nd);
  take(t->q, nd);
  take(t->dinv, nd);
  take(t->Fp, g.ne * ngp * 9);
  take(t->epsP, g.ne * ngp);
  take(t->drive, 2 * g.ne);
  take(t->ef, g.ne * ngp * c->dim);
  take(t->part, 3 * pfs::kFsBlocksMax);
  take(t->sc, pfs::FS_COUNT);
  return off;
}

template <int DIM>
static pfs::FSElemArgs fs_elem_args(pf_fs* f, const double* u, const double* v) {
  pfs::FSElemArgs a;
  a.g = f->g;
  a.p = f->p;
  a.pf = f->pf;
  a.pw = f->pw;
  a.u = u;
  a.v = v;
  a.Fp = f->fp_identity ? nullptr : f->Fp;
  a.ef = f->ef;
  a.sc = f->sc;
  return a;
}

// R = nodal forces of the displacement `u`; ||R||^2 into sc[FS_NORM]
template <int DIM>
static pf_status fs_residual(pf_fs* f, const double* u, double* R) {
  const int nbe = fs_blocks(f->g.ne);
  const pfs::FSElemArgs ea = fs_elem_args<DIM>(f, u, nullptr);
  fs_timed(f, PF_FS_K_RESIDUAL, [&] {
    hipLaunchKernelGGL((pfs::k_fs_elem<DIM, false>), dim3(nbe), dim3(pfs::kFsThreads), 0, f->stream, ea);
  });
  pfs::FSGatherArgs ga{f->g, f->ef, R, nullptr, f->part, nullptr};
  fs_timed(f, PF_FS_K_GATHER, [&] {
    hipLaunchKernelGGL((pfs::k_fs_gather<DIM>), dim3(f->nb), dim3(pfs::kFsThreads), 0, f->stream, ga);
  });
  hipLaunchKernelGGL(pfs::k_fs_reduce, dim3(1), dim3(pfs::kFsThreads), 0, f->stream, (const double*)f->part, f->nb, f->sc,
                     (int)pfs::FSR_NORM, 0);
  FSLAUNCH(f);
  return PF_OK;
}

static pf_status fs_read_scalars(pf_fs* f) {
  FSCHK(f, hipMemcpyAsync(f->host, f->sc, pfs::FS_COUNT * sizeof(double), hipMemcpyDeviceToHost, f->stream));
  FSCHK(f, hipStreamSynchronize(f->stream));
  if (f->timing) fs_flush(f);
  return PF_OK;
}

// CG on J x = -R at the displacement u (Jacobi preconditioner f->dinv).
template <int DIM>
static pf_status fs_cg(pf_fs* f, int* iters) {
  pfs::FSVec v{f->nd, f->dinv, f->x, f->r, f->z, f->pd, f->q, f->part, f->sc};
  const double tol2 = f->cfg.cg_rtol * f->cfg.cg_rtol;
  FSCHK(f, hipMemcpyAsync(f->sc + pfs::FS_TOL2, &tol2, sizeof(double), hipMemcpyHostToDevice, f->stream));
  const int nbv = f->nb;
  hipLaunchKernelGGL(pfs::k_fs_cg_init, dim3(nbv), dim3(pfs::kFsThreads), 0, f->stream, v, (const double*)f->R);
  hipLaunchKernelGGL(pfs::k_fs_reduce, dim3(1), dim3(pfs::kFsThreads), 0, f->stream, (const double*)f->part, nbv, f->sc,
                     (int)pfs::FSR_INIT, f->cfg.cg_max_iter);
  FSLAUNCH(f);
  const int nbe = fs_blocks(f->g.ne);
  pfs::FSElemArgs ea = fs_elem_args<DIM>(f, f->u, f->pd);
  pfs::FSGatherArgs ga{f->g, f->ef, f->q, f->pd, f->part, f->sc};
  int launched = 0, chunk = 16;
  for (;;) {
    for (int t = 0; t < chunk; ++t) {
      if (launched > 0)
        fs_timed(f, PF_FS_K_VECTOR, [&] {
          hipLaunchKernelGGL(pfs::k_fs_cg_dir, dim3(nbv), dim3(pfs::kFsThreads), 0, f->stream, v);
        });
      fs_timed(f, PF_FS_K_TANGENT, [&] {
        hipLaunchKernelGGL((pfs::k_fs_elem<DIM, true>), dim3(nbe), dim3(pfs::kFsThreads), 0, f->stream, ea);
      });
      fs_timed(f, PF_FS_K_GATHER, [&] {
        hipLaunchKernelGGL((pfs::k_fs_gather<DIM>), dim3(nbv), dim3(pfs::kFsThreads), 0, f->stream, ga);
      });
      fs_timed(f, PF_FS_K_VECTOR, [&] {
        hipLaunchKernelGGL(pfs::k_fs_reduce, dim3(1), dim3(pfs::kFsThreads), 0, f->stream, (const double*)f->part, nbv, f->sc,
                           (int)pfs::FSR_ALPHA, f->cfg.cg_max_iter);
        hipLaunchKernelGGL(pfs::k_fs_cg_update, dim3(nbv), dim3(pfs::kFsThreads), 0, f->stream, v);
        hipLaunchKernelGGL(pfs::k_fs_reduce, dim3(1), dim3(pfs::kFsThreads), 0, f->stream, (const double*)f->part, nbv, f->sc,
                           (int)pfs::FSR_BETA, f->cfg.cg_max_iter);
      });
      ++launched;
    }
    FSLAUNCH(f);
    pf_status s = fs_read_scalars(f);
    if (s != PF_OK) return s;
    if (f->host[pfs::FS_CONV] != 0.0) break;
    if (launched >= f->cfg.cg_max_iter) break;
    chunk = std::min(2 * chunk, 64);
  }
  *iters = (int)f->host[pfs::FS_ITERS];
  if (f->host[pfs::FS_BAD] != 0.0)
    return fs_fail(f, PF_ERR_CG_NOT_CONVERGED, "finite strain: the tangent is not positive along a CG direction");
  return PF_OK;
}

template <int DIM>
static pf_status fs_solve_dim(pf_fs* f, pf_fs_stats* out) {
  pf_fs_stats st{};
  hipStream_t s = f->stream;
  pf_status rc;
  // load scale: ||R(0)||
  hipLaunchKernelGGL(pfs::k_fs_axpy, dim3(f->nb), dim3(pfs::kFsThreads), 0, s, f->nd, (const double*)f->u, -1.0,
                     (const double*)f->u, f->x);   // x = 0
  if ((rc = fs_residual<DIM>(f, f->x, f->R)) != PF_OK) return rc;
  if ((rc = fs_read_scalars(f)) != PF_OK) return rc;
  const double r0 = std::sqrt(f->host[pfs::FS_NORM]);
  hipLaunchKernelGGL((pfs::k_fs_diag<DIM>), dim3(f->nb), dim3(pfs::kFsThreads), 0, s, f->g, f->p,
                     (const double*)f->pf, (const double*)f->pw, f->dinv);
  FSLAUNCH(f);
  // a load at the rounding level of the stress evaluation (no transformation
  // misfit: P(I) is zero only up to rounding) is no load: u = 0
  double mod = 0.0;
  for (int a = 0; a < 3; ++a) mod = std::max(mod, f->p.K[a] + f->p.G[a]);
  const double zero_load = 1e-12 * mod * std::pow(f->cfg.h, DIM - 1) * std::sqrt((double)f->nd);
  if (!(r0 > zero_load)) {
    if (!std::isfinite(r0)) return fs_fail(f, PF_ERR_NONFINITE, "finite strain: non-finite load");
    FSCHK(f, hipMemcpyAsync(f->u, f->x, f->nd * sizeof(double), hipMemcpyDeviceToDevice, s));   // u = 0
  } else {
    if ((rc = fs_residual<DIM>(f, f->u, f->R)) != PF_OK) return rc;
    if ((rc = fs_read_scalars(f)) != PF_OK) return rc;
    double nr = std::sqrt(f->host[pfs::FS_NORM]);
    if (!std::isfinite(nr)) return fs_fail(f, PF_ERR_NONFINITE, "finite strain: the start is outside the domain");
    const double tol = f->cfg.newton_rtol * r0;
    while (nr > tol) {
      if (st.newton_iters >= f->cfg.newton_max_iter)
        return fs_fail(f, PF_ERR_CG_NOT_CONVERGED, "finite strain: Newton at %d steps, ||R||/||R0|| = %.3e",
                       st.newton_iters, nr / r0);
      int it = 0;
      if ((rc = fs_cg<DIM>(f, &it)) != PF_OK) return rc;
      st.cg_iters += it;
      FSCHK(f, hipMemcpyAsync(f->uold, f->u, f->nd * sizeof(double), hipMemcpyDeviceToDevice, s));
      double step = 1.0, nn = 0.0;
      bool ok = false;
      for (int cut = 0; cut < 30; ++cut) {
        hipLaunchKernelGGL(pfs::k_fs_axpy, dim3(f->nb), dim3(pfs::kFsThreads), 0, s, f->nd, (const double*)f->uold,
                           step, (const double*)f->x, f->u);
        if ((rc = fs_residual<DIM>(f, f->u, f->R)) != PF_OK) return rc;
        if ((rc = fs_read_scalars(f)) != PF_OK) return rc;
        nn = std::sqrt(f->host[pfs::FS_NORM]);
        if (std::isfinite(nn) && nn < nr) {
          ok = true;
          break;
        }
        step *= 0.5;
        ++st.line_search_cuts;
      }
      if (!ok) return fs_fail(f, PF_ERR_NONFINITE, "finite strain: no Newton step lowers ||R|| (||R||/||R0|| = %.3e)",
                              nr / r0);
      nr = nn;
      ++st.newton_iters;
    }
    st.rel_resid = nr / r0;
  }
  if (f->cfg.plasticity) {
    pfs::FSRetArgs ra{f->g, f->p, f->pf, f->pw, f->u, f->Fp, f->epsP, f->part, 1e-13};
    fs_timed(f, PF_FS_K_RETURN, [&] {
      hipLaunchKernelGGL((pfs::k_fs_return<DIM>), dim3(f->nb), dim3(pfs::kFsThreads), 0, s, ra);
    });
    hipLaunchKernelGGL(pfs::k_fs_reduce, dim3(1), dim3(pfs::kFsThreads), 0, s, (const double*)f->part, f->nb, f->sc,
                       (int)pfs::FSR_MAX2_SUM, 0);
    FSLAUNCH(f);
    if ((rc = fs_read_scalars(f)) != PF_OK) return rc;
    st.max_epsP = f->host[pfs::FS_MAX0];
    st.yielded = (int)f->host[pfs::FS_SUM0];
    if (st.yielded > 0) f->fp_identity = false;
  }
  pfs::FSPostArgs pa{f->g, f->p, f->pf, f->pw, f->u, f->fp_identity ? nullptr : f->Fp, f->drive, f->part};
  fs_timed(f, PF_FS_K_POST, [&] {
    hipLaunchKernelGGL((pfs::k_fs_post<DIM>), dim3(f->nb), dim3(pfs::kFsThreads), 0, s, pa);
  });
  hipLaunchKernelGGL(pfs::k_fs_reduce, dim3(1), dim3(pfs::kFsThreads), 0, s, (const double*)f->part, f->nb, f->sc,
                     (int)pfs::FSR_MAX2_SUM, 0);
  FSLAUNCH(f);
  if ((rc = fs_read_scalars(f)) != PF_OK) return rc;
  st.max_vm = f->host[pfs::FS_MAX1];
  if (!f->cfg.plasticity) st.max_epsP = 0.0;
  if (out) *out = st;
  return PF_OK;
}

// phases of a context (padded layout, T, optional FP32 low parts) -> the
// solver's compact FP64 cell arrays
template <typename T>
__global__ __launch_bounds__(pfs::kFsThreads) void k_fs_import(pfk::Grid g, const T* pfh, const T* pwh, const T* pfl,
                                                               const T* pwl, double* pf, double* pw) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
    const long long r = c / g.nx;
    const long long e = r * g.px + (c - r * g.nx);
    pf[c] = (double)pfh[e] + (pfl ? (double)pfl[e] : 0.0);
    pw[c] = (double)pwh[e] + (pwl ? (double)pwl[e] : 0.0);
  }
}

static pf_status fs_couple(pf_ctx* c, const Grid& g, const void* pf_hi, const void* pw_hi, const void* pf_lo,
                           const void* pw_lo, int es, const double** drive) {
  pf_fs* f = c->fs;
  const int nb = fs_blocks(f->g.ne);
  if (es == 8)
    hipLaunchKernelGGL((k_fs_import<double>), dim3(nb), dim3(pfs::kFsThreads), 0, c->stream, g,
                       (const double*)pf_hi, (const double*)pw_hi, (const double*)pf_lo, (const double*)pw_lo, f->pf,
                       f->pw);
  else
    hipLaunchKernelGGL((k_fs_import<float>), dim3(nb), dim3(pfs::kFsThreads), 0, c->stream, g, (const float*)pf_hi,
                       (const float*)pw_hi, (const float*)pf_lo, (const float*)pw_lo, f->pf, f->pw);
  HIPCHK(c, hipGetLastError());
  const pf_status s = pf_fs_solve(f, &c->fs_last);
  if (s != PF_OK) return fail(c, s, "finite-strain mechanics: %s", f->err);
  *drive = f->drive;
  return PF_OK;
}

extern "C" {

pf_status pf_fs_attach(pf_ctx* ctx, pf_fs* fs) {
  if (!ctx) return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_attach: NULL context");
  if (fs) {
    const pf_config& a = ctx->cfg;
    const pf_fs_config& b = fs->cfg;
    if (a.dim != b.dim || a.nx != b.nx || a.ny != b.ny || a.nz != b.nz || a.h != b.h)
      return fail(ctx, PF_ERR_INVALID_ARG, "pf_fs_attach: the grids differ");
    if (a.mechanics) return fail(ctx, PF_ERR_INVALID_ARG, "pf_fs_attach: the context's small-strain mechanics must be off");
    if (ctx->stream != fs->stream) return fail(ctx, PF_ERR_INVALID_ARG, "pf_fs_attach: the streams differ");
  }
  ctx->fs = fs;
  ctx->fs_last = pf_fs_stats{};
  return PF_OK;
}

size_t pf_fs_workspace_bytes(const pf_fs_config* cfg) {
  if (!fs_valid(cfg)) return 0;
  return fs_layout(nullptr, cfg, nullptr);
}

pf_status pf_fs_init(const pf_fs_config* cfg, const pf_params* params, void* workspace, size_t workspace_bytes,
                     void* hip_stream, pf_fs** out) {
  if (!out) return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_init: out is NULL");
  *out = nullptr;
  if (!fs_valid(cfg)) return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_init: invalid configuration");
  if (!params) return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_init: params is NULL");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_init: workspace NULL or not 256-byte aligned");
  const size_t need = fs_layout(nullptr, cfg, nullptr);
  if (workspace_bytes < need)
    return fs_fail(nullptr, PF_ERR_OOM, "pf_fs_init: workspace of %zu bytes, %zu needed", workspace_bytes, need);
  pf_fs* f = new (std::nothrow) pf_fs{};
  if (!f) return fs_fail(nullptr, PF_ERR_OOM, "pf_fs_init: host allocation failed");
  f->cfg = *cfg;
  for (int a = 0; a < 3; ++a) {
    f->p.K[a] = params->K[a];
    f->p.G[a] = params->G[a];
  }
  f->p.Omega = params->Omega_f;
  f->p.sigY = params->sigY;
  f->p.Hh = params->Hhard;
  f->g = fs_grid(cfg);
  f->stream = reinterpret_cast<hipStream_t>(hip_stream);
  f->nd = (long long)cfg->dim * f->g.nn;
  f->nb = fs_blocks(std::max(f->nd, f->g.ne));
  fs_layout(f, cfg, reinterpret_cast<char*>(workspace));
  hipError_t e = hipHostMalloc((void**)&f->host, pfs::FS_COUNT * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete f;
    return fs_fail(nullptr, PF_ERR_HIP, "pf_fs_init: hipHostMalloc: %s", hipGetErrorString(e));
  }
  e = hipMemsetAsync(workspace, 0, need, f->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pfs::k_fs_plastic_reset, dim3(fs_blocks(f->g.ne * (1LL << cfg->dim))), dim3(pfs::kFsThreads),
                       0, f->stream, f->g.ne * (1LL << cfg->dim), f->Fp, f->epsP);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  f->fp_identity = true;
  if (e != hipSuccess) {
    (void)hipHostFree(f->host);
    delete f;
    return fs_fail(nullptr, PF_ERR_HIP, "pf_fs_init: %s", hipGetErrorString(e));
  }
  *out = f;
  return PF_OK;
}

pf_status pf_fs_fields(pf_fs* f, int field, int dir, void* ptr, size_t nbytes, int ptr_is_device) {
  if (!f) return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_fields: NULL context");
  if (!ptr || (dir != 0 && dir != 1)) return fs_fail(f, PF_ERR_INVALID_ARG, "pf_fs_fields: NULL pointer or bad dir");
  const long long ngp = 1LL << f->cfg.dim;
  double* arr = nullptr;
  long long n = 0;
  switch (field) {
    case PF_FS_PHI_F: arr = f->pf; n = f->g.ne; break;
    case PF_FS_PHI_W: arr = f->pw; n = f->g.ne; break;
    case PF_FS_U: arr = f->u; n = f->nd; break;
    case PF_FS_FP: arr = f->Fp; n = f->g.ne * ngp * 9; break;
    case PF_FS_EPSP: arr = f->epsP; n = f->g.ne * ngp; break;
    case PF_FS_DRIVE: arr = f->drive; n = 2 * f->g.ne; break;
    default: return fs_fail(f, PF_ERR_INVALID_ARG, "pf_fs_fields: unknown field %d", field);
  }
  if (field == PF_FS_DRIVE && dir == 1) return fs_fail(f, PF_ERR_INVALID_ARG, "pf_fs_fields: driving forces are read-only");
  if (nbytes != (size_t)n * sizeof(double))
    return fs_fail(f, PF_ERR_INVALID_ARG, "pf_fs_fields: %zu bytes given, %lld expected", nbytes, n * 8);
  const hipMemcpyKind kind = dir == 1 ? (ptr_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice)
                                      : (ptr_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
  if (dir == 1)
    FSCHK(f, hipMemcpyAsync(arr, ptr, nbytes, kind, f->stream));
  else
    FSCHK(f, hipMemcpyAsync(ptr, arr, nbytes, kind, f->stream));
  if (dir == 1 && field == PF_FS_FP) f->fp_identity = false;
  if (dir == 1 && field == PF_FS_U) {
    if (f->cfg.dim == 2)
      hipLaunchKernelGGL((pfs::k_fs_fix<2>), dim3(f->nb), dim3(pfs::kFsThreads), 0, f->stream, f->g, f->u);
    else
      hipLaunchKernelGGL((pfs::k_fs_fix<3>), dim3(f->nb), dim3(pfs::kFsThreads), 0, f->stream, f->g, f->u);
    FSLAUNCH(f);
  }
  if (dir == 0 && !ptr_is_device) FSCHK(f, hipStreamSynchronize(f->stream));
  return PF_OK;
}

pf_status pf_fs_solve(pf_fs* f, pf_fs_stats* stats) {
  if (!f) return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_solve: NULL context");
  return f->cfg.dim == 2 ? fs_solve_dim<2>(f, stats) : fs_solve_dim<3>(f, stats);
}

pf_status pf_fs_timing(pf_fs* f, int on) {
  if (!f) return fs_fail(nullptr, PF_ERR_INVALID_ARG, "pf_fs_timing: NULL context");
  FSCHK(f, hipStreamSynchronize(f->stream));
  fs_flush(f);
  if (on && f->ev.empty()) {
    f->ev.resize(4096);
    // timing-only events without the system-scope fence (every read follows a stream synchronisation)
    for (auto& e : f->ev) FSCHK(f, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  for (int k = 0; k < PF_FS_K_COUNT; ++k) {
    f->t_ms[k] = 0.0;
    f->t_n[k] = 0;
  }
  f->timing = on != 0;
  return PF_OK;
}

pf_status pf_fs_timing_get(pf_fs* f, int kind, double* ms, long long* launches) {
  if (!f || !ms || !launches || kind < 0 || kind >= PF_FS_K_COUNT)
    return fs_fail(f, PF_ERR_INVALID_ARG, "pf_fs_timing_get: bad arguments");
  *ms = f->t_ms[kind];
  *launches = f->t_n[kind];
  return PF_OK;
}

const char* pf_fs_last_error(const pf_fs* f) { return f ? f->err : g_fs_err; }

void pf_fs_destroy(pf_fs* f) {
  if (!f) return;
  if (!f->ev.empty()) (void)hipStreamSynchronize(f->stream);
  for (auto& e : f->ev) (void)hipEventDestroy(e);
  (void)hipHostFree(f->host);
  delete f;
}

}  // extern "C"
