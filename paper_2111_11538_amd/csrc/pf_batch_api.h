// Host side of the batch entry points declared in include/pf.h (included once,
// at the end of pf_api.hip).
#pragma once

#include "pf_batch.h"

namespace {

constexpr int kMinApplyRows = 4;       // smallest tuning choices bound the table sizes
constexpr int kMinChunk = 256;
inline int fine_rows(int rows) { return std::max(kMinApplyRows, rows / 4); }
inline int fine_chunk(int chunk) { return std::max(kMinChunk, chunk / 4); }

struct BatchLayout {
  int count;
  size_t es;
  int N;                               // packed elements per array
  std::vector<InstDesc> inst;          // host copy (tile ranges filled by build_tables)
  int n_el, n_ce;
  int max_ap, max_up;                  // table capacities
  size_t o_fld[2][5], o_u[2], o_epsp, o_epsP, o_mu, o_K, o_G;
  size_t o_lo[2][5];       // FP32 state: low parts of the five fields (0 in FP64)
  size_t o_r[2], o_z[2], o_pa[2], o_pb[2], o_q[2], o_di[2];
  size_t o_inst, o_el, o_ap, o_ce, o_up;
  size_t o_bn, o_pr, o_pa_part, o_pu, o_pt, o_pc, o_iscal, o_bar, o_stage;
  size_t stage_elems;
  size_t total;
};

bool valid_batch(const pf_config* c, const pf_extent* ext, int count, char* msg, size_t len) {
  if (!c || !ext) { snprintf(msg, len, "config or extents NULL"); return false; }
  if (count < 1 || count > kMaxBatch) { snprintf(msg, len, "count must be 1..%d", kMaxBatch); return false; }
  if (c->dim != 2) { snprintf(msg, len, "batches are 2D (dim == 2)"); return false; }
  if (!c->mechanics) { snprintf(msg, len, "batches need mechanics == 1"); return false; }
  if (c->warm != PF_WARM_PREV) { snprintf(msg, len, "batches use warm == PF_WARM_PREV"); return false; }
  if (c->cg_precond != 0) { snprintf(msg, len, "batches use the Jacobi preconditioner (cg_precond == 0)"); return false; }
  if (!(c->h > 0.0) || !(c->dt > 0.0)) { snprintf(msg, len, "h and dt must be positive"); return false; }
  if (c->precision != PF_FP64 && c->precision != PF_MIXED) { snprintf(msg, len, "unknown precision"); return false; }
  if (!(c->cg_rtol > 0.0) || c->cg_max_iter < 1) { snprintf(msg, len, "cg_rtol > 0 and cg_max_iter >= 1 required"); return false; }
  long long tot = 0;
  for (int b = 0; b < count; ++b) {
    if (ext[b].nx < 1 || ext[b].ny < 1 || ext[b].nz != 1) { snprintf(msg, len, "instance %d: bad extent", b); return false; }
    tot += (long long)((ext[b].nx + 15) / 16 * 16) * ext[b].ny + 64;
  }
  if (tot * 8 >= (1LL << 31)) { snprintf(msg, len, "batch too large for 32-bit indexing"); return false; }
  return true;
}

BatchLayout make_batch_layout(const pf_config* c, const pf_extent* ext, int count) {
  BatchLayout L{};
  L.count = count;
  L.es = c->precision == PF_FP64 ? 8 : 4;
  int off = 0;
  L.n_el = 0;
  L.max_ap = 0;
  L.max_up = 0;
  const int vn = (int)(16 / L.es);
  L.stage_elems = 0;
  for (int b = 0; b < count; ++b) {
    InstDesc d{};
    d.g.nx = ext[b].nx; d.g.ny = ext[b].ny; d.g.nz = 1;
    d.g.px = (ext[b].nx + 15) / 16 * 16;
    d.g.n = d.g.px * d.g.ny;
    d.off = off;
    off += (d.g.n + 63) / 64 * 64;
    L.n_el += ((d.g.nx + TX - 1) / TX) * ((d.g.ny + TY - 1) / TY);
    // coarse and fine tables together, each at most the finest tiling
    L.max_ap += 2 * ((d.g.nx + A2S - 1) / A2S) * ((d.g.ny + kMinApplyRows - 1) / kMinApplyRows);
    L.max_up += 2 * ((d.g.n / vn + kMinChunk - 1) / kMinChunk);
    L.stage_elems = std::max(L.stage_elems, (size_t)(d.g.nx + 1) * (d.g.ny + 1));
    L.inst.push_back(d);
  }
  L.N = off;
  for (auto& d : L.inst) d.g.ns = L.N;
  L.n_ce = L.n_el;
  size_t pos = 0;
  auto take = [&](size_t bytes) { size_t o = pos; pos += align_up(bytes); return o; };
  const size_t arr = align_up((size_t)L.N * L.es);
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 5; ++f) L.o_fld[s][f] = take(arr);
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 5; ++f) L.o_lo[s][f] = L.es == 4 ? take(arr) : 0;
  for (int d = 0; d < 2; ++d) L.o_u[d] = take(arr);
  L.o_epsp = take((size_t)L.N * L.es * 4);
  L.o_epsP = take(arr);
  L.o_mu = take(arr);
  L.o_K = take(arr);
  L.o_G = take(arr);
  for (int d = 0; d < 2; ++d) {
    L.o_r[d] = take(arr); L.o_z[d] = take(arr); L.o_pa[d] = take(arr);
    L.o_pb[d] = take(arr); L.o_q[d] = take(arr); L.o_di[d] = take(arr);
  }
  L.o_inst = take(count * sizeof(InstDesc));
  L.o_el = take(L.n_el * sizeof(TileRef));
  L.o_ap = take(L.max_ap * sizeof(TileRef));
  L.o_ce = take(L.n_ce * sizeof(TileRef));
  L.o_up = take(L.max_up * sizeof(ChunkRef));
  L.o_bn = take(L.n_el * sizeof(double));
  L.o_pr = take(2 * L.n_el * sizeof(double));
  L.o_pa_part = take(L.max_ap * sizeof(double));
  L.o_pu = take(4 * (size_t)L.max_up * sizeof(double));
  L.o_pt = take(L.n_el * sizeof(double));
  L.o_pc = take(NQ_STEP * (size_t)L.n_ce * sizeof(double));
  L.o_iscal = take((size_t)count * S_COUNT * sizeof(double));
  L.o_bar = take(kBarWords * sizeof(unsigned));
  L.o_stage = take(L.stage_elems * sizeof(double));
  L.total = pos;
  return L;
}

}  // namespace

struct pf_batch {
  pf_config cfg;
  pf_params prm;
  hipStream_t stream;
  BatchLayout L;
  char* ws;
  char err[512];
  bool bad;
  bool ledger_valid;
  int cur;
  long long steps;
  pf_batch_tiles tiles;
  int n_ap, n_up;
  int occupancy, ncu;
  hipGraph_t graph[2];
  hipGraphExec_t exec[2];
  bool have_graph;
  double* host_iscal;      // pinned copy of the per-instance scalars + barrier words
  template <typename T> T* arr(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

static pf_status bfail(pf_batch* b, pf_status s, const char* fmt, ...) {
  char* dst = b ? b->err : g_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return s;
}

#define BHIP(b, call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return bfail((b), PF_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

template <typename T>
static BatchArgs<T> batch_args(pf_batch* bt, int cur) {
  const BatchLayout& L = bt->L;
  BatchArgs<T> B{};
  B.count = L.count;
  B.inst = bt->arr<InstDesc>(L.o_inst);
  B.el = bt->arr<TileRef>(L.o_el);
  B.n_el = L.n_el;
  B.ap = bt->arr<TileRef>(L.o_ap);
  B.n_ap = bt->n_ap;
  B.ce = bt->arr<TileRef>(L.o_ce);
  B.n_ce = L.n_ce;
  B.up = bt->arr<ChunkRef>(L.o_up);
  B.n_up = bt->n_up;
  pf_config c1 = bt->cfg;
  B.p = make_kp<T>(&c1, &bt->prm);
  for (int f = 0; f < 5; ++f) {
    B.f_old[f] = bt->arr<T>(L.o_fld[cur][f]);
    B.f_new[f] = bt->arr<T>(L.o_fld[cur ^ 1][f]);
    B.lo_old[f] = L.es == 4 ? bt->arr<T>(L.o_lo[cur][f]) : nullptr;
    B.lo_new[f] = L.es == 4 ? bt->arr<T>(L.o_lo[cur ^ 1][f]) : nullptr;
  }
  for (int d = 0; d < 2; ++d) {
    B.u[d] = bt->arr<T>(L.o_u[d]);
    B.r[d] = bt->arr<T>(L.o_r[d]);
    B.z[d] = bt->arr<T>(L.o_z[d]);
    B.pa[d] = bt->arr<T>(L.o_pa[d]);
    B.pb[d] = bt->arr<T>(L.o_pb[d]);
    B.q[d] = bt->arr<T>(L.o_q[d]);
    B.dinv[d] = bt->arr<T>(L.o_di[d]);
  }
  B.epsp = bt->arr<T>(L.o_epsp);
  B.epsP = bt->arr<T>(L.o_epsP);
  B.mu = bt->arr<T>(L.o_mu);
  B.K = bt->arr<T>(L.o_K);
  B.G = bt->arr<T>(L.o_G);
  B.part_bn = bt->arr<double>(L.o_bn);
  B.part_r = bt->arr<double>(L.o_pr);
  B.part_a = bt->arr<double>(L.o_pa_part);
  B.part_u = bt->arr<double>(L.o_pu);
  B.part_t = bt->arr<double>(L.o_pt);
  B.part_c = bt->arr<double>(L.o_pc);
  B.iscal = bt->arr<double>(L.o_iscal);
  B.bar = bt->arr<unsigned>(L.o_bar);
  B.tol2 = bt->cfg.cg_rtol * bt->cfg.cg_rtol;
  B.max_iter = bt->cfg.cg_max_iter;
  B.kz_ap = bt->tiles.apply_rows;
  B.kz_apf = fine_rows(bt->tiles.apply_rows);
  B.vol = bt->cfg.h * bt->cfg.h;
  B.area_dt = bt->cfg.h * bt->cfg.dt;
  B.spin_limit = bt->tiles.spin_limit;
  return B;
}

// Tile tables for the current decomposition, uploaded into the workspace.
static pf_status build_tables(pf_batch* bt) {
  BatchLayout& L = bt->L;
  std::vector<TileRef> el, ap;
  std::vector<ChunkRef> up;
  const int vn = (int)(16 / L.es);
  const int rows = bt->tiles.apply_rows, chunk = bt->tiles.update_chunk;
  const int rows_f = fine_rows(rows), chunk_f = fine_chunk(chunk);
  for (int b = 0; b < L.count; ++b) {
    InstDesc& d = L.inst[b];
    d.el0 = (int)el.size();
    for (int by = 0; by < (d.g.ny + TY - 1) / TY; ++by)
      for (int bx = 0; bx < (d.g.nx + TX - 1) / TX; ++bx) el.push_back({b, bx, by, 0});
    d.eln = (int)el.size() - d.el0;
    d.ce0 = d.el0;
    d.cen = d.eln;
    d.ap0 = (int)ap.size();
    for (int by = 0; by < (d.g.ny + rows - 1) / rows; ++by)
      for (int bx = 0; bx < (d.g.nx + A2S - 1) / A2S; ++bx) ap.push_back({b, bx, by, 0});
    d.apn = (int)ap.size() - d.ap0;
    d.up0 = (int)up.size();
    const int nv = d.g.n / vn;
    for (int v = 0; v < nv; v += chunk) up.push_back({b, v, std::min(nv, v + chunk), 0});
    d.upn = (int)up.size() - d.up0;
  }
  // the fine tables, used in passes where the coarse work of the instances
  // still iterating would leave blocks idle
  for (int b = 0; b < L.count; ++b) {
    InstDesc& d = L.inst[b];
    d.apf0 = (int)ap.size();
    for (int by = 0; by < (d.g.ny + rows_f - 1) / rows_f; ++by)
      for (int bx = 0; bx < (d.g.nx + A2S - 1) / A2S; ++bx) ap.push_back({b, bx, by, 0});
    d.apfn = (int)ap.size() - d.apf0;
    d.upf0 = (int)up.size();
    const int nv = d.g.n / vn;
    for (int v = 0; v < nv; v += chunk_f) up.push_back({b, v, std::min(nv, v + chunk_f), 0});
    d.upfn = (int)up.size() - d.upf0;
  }
  if ((int)ap.size() > L.max_ap || (int)up.size() > L.max_up)
    return bfail(bt, PF_ERR_INVALID_ARG, "tile tables exceed their capacity");
  bt->n_ap = (int)ap.size();
  bt->n_up = (int)up.size();
  BHIP(bt, hipMemcpyAsync(bt->ws + L.o_inst, L.inst.data(), L.count * sizeof(InstDesc), hipMemcpyHostToDevice, bt->stream));
  BHIP(bt, hipMemcpyAsync(bt->ws + L.o_el, el.data(), el.size() * sizeof(TileRef), hipMemcpyHostToDevice, bt->stream));
  BHIP(bt, hipMemcpyAsync(bt->ws + L.o_ce, el.data(), el.size() * sizeof(TileRef), hipMemcpyHostToDevice, bt->stream));
  BHIP(bt, hipMemcpyAsync(bt->ws + L.o_ap, ap.data(), ap.size() * sizeof(TileRef), hipMemcpyHostToDevice, bt->stream));
  BHIP(bt, hipMemcpyAsync(bt->ws + L.o_up, up.data(), up.size() * sizeof(ChunkRef), hipMemcpyHostToDevice, bt->stream));
  BHIP(bt, hipStreamSynchronize(bt->stream));
  return PF_OK;
}

template <typename T>
static pf_status build_graphs(pf_batch* bt) {
  if (bt->have_graph) {
    for (int s = 0; s < 2; ++s) {
      (void)hipGraphExecDestroy(bt->exec[s]);
      (void)hipGraphDestroy(bt->graph[s]);
    }
    bt->have_graph = false;
  }
  const int nblk = bt->ncu * bt->tiles.blocks_per_cu;
  for (int s = 0; s < 2; ++s) {
    BatchArgs<T> B = batch_args<T>(bt, s);
    void* args[] = {&B};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(&k_batch_step<T>);
    kp.gridDim = dim3(nblk);
    kp.blockDim = dim3(NT);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    BHIP(bt, hipGraphCreate(&bt->graph[s], 0));
    BHIP(bt, hipGraphAddKernelNode(&node, bt->graph[s], nullptr, 0, &kp));
    BHIP(bt, hipGraphInstantiate(&bt->exec[s], bt->graph[s], nullptr, nullptr, 0));
  }
  bt->have_graph = true;
  return PF_OK;
}

template <typename T>
static pf_status batch_occupancy(pf_batch* bt) {
  int dev = 0, occ = 0, ncu = 0;
  BHIP(bt, hipGetDevice(&dev));
  BHIP(bt, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  BHIP(bt, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_step<T>, NT, 0));
  if (occ < 1) return bfail(bt, PF_ERR_UNSUPPORTED, "the batch kernel cannot be resident");
  bt->occupancy = occ;
  bt->ncu = ncu;
  return PF_OK;
}

template <typename F>
static pf_status bdispatch(pf_batch* b, F&& f) {
  if (b->cfg.precision == PF_FP64) return f((double)0);
  return f((float)0);
}

extern "C" {

size_t pf_batch_workspace_bytes(const pf_config* cfg, const pf_extent* ext, int count) {
  char msg[256];
  if (!valid_batch(cfg, ext, count, msg, sizeof msg)) return 0;
  return make_batch_layout(cfg, ext, count).total;
}

pf_status pf_batch_init(const pf_config* cfg, const pf_params* params, const pf_extent* ext, int count,
                        void* workspace, size_t workspace_bytes, void* hip_stream, pf_batch** out) {
  if (!out) return bfail(nullptr, PF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  char msg[256];
  if (!valid_batch(cfg, ext, count, msg, sizeof msg)) return bfail(nullptr, PF_ERR_INVALID_ARG, "%s", msg);
  if (cfg->species_implicit) return bfail(nullptr, PF_ERR_UNSUPPORTED, "batches step the species explicitly");
  if (!params) return bfail(nullptr, PF_ERR_INVALID_ARG, "params is NULL");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return bfail(nullptr, PF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
  BatchLayout L = make_batch_layout(cfg, ext, count);
  if (workspace_bytes < L.total)
    return bfail(nullptr, PF_ERR_OOM, "workspace has %zu bytes, %zu needed", workspace_bytes, L.total);
  pf_batch* bt = new (std::nothrow) pf_batch();
  if (!bt) return bfail(nullptr, PF_ERR_OOM, "host allocation failed");
  bt->cfg = *cfg;
  bt->prm = *params;
  bt->stream = reinterpret_cast<hipStream_t>(hip_stream);
  bt->L = L;
  bt->ws = reinterpret_cast<char*>(workspace);
  bt->err[0] = 0;
  bt->bad = false;
  bt->ledger_valid = false;
  bt->cur = 0;
  bt->steps = 0;
  bt->have_graph = false;
  bt->tiles.apply_rows = 32;
  bt->tiles.update_chunk = 1024;
  bt->tiles.blocks_per_cu = 2;
  bt->tiles.spin_limit = 20000000LL;
  pf_status st = bdispatch(bt, [&](auto t) { return batch_occupancy<decltype(t)>(bt); });
  if (st == PF_OK && hipHostMalloc(reinterpret_cast<void**>(&bt->host_iscal),
                                   ((size_t)count * S_COUNT + 4) * sizeof(double), hipHostMallocDefault) != hipSuccess)
    st = bfail(nullptr, PF_ERR_HIP, "hipHostMalloc failed");
  if (st == PF_OK) {
    bt->tiles.blocks_per_cu = std::min(bt->tiles.blocks_per_cu, bt->occupancy);
    hipError_t e = hipMemsetAsync(bt->ws, 0, L.total, bt->stream);
    if (e != hipSuccess) st = bfail(nullptr, PF_ERR_HIP, "clearing the workspace: %s", hipGetErrorString(e));
  }
  if (st == PF_OK) st = build_tables(bt);
  if (st == PF_OK) st = bdispatch(bt, [&](auto t) { return build_graphs<decltype(t)>(bt); });
  if (st != PF_OK) {
    if (bt->err[0]) snprintf(g_err, sizeof g_err, "%s", bt->err);
    pf_batch_destroy(bt);
    return st;
  }
  *out = bt;
  return PF_OK;
}

pf_status pf_batch_set_tiles(pf_batch* bt, const pf_batch_tiles* t) {
  if (!bt || !t) return bfail(bt, PF_ERR_INVALID_ARG, "NULL argument");
  if (t->apply_rows < kMinApplyRows || t->apply_rows > 256 || t->update_chunk < kMinChunk || t->update_chunk > 65536 ||
      t->blocks_per_cu < 1 || t->blocks_per_cu > bt->occupancy || t->spin_limit < 0)
    return bfail(bt, PF_ERR_INVALID_ARG, "tile parameters out of range (blocks_per_cu <= %d)", bt->occupancy);
  BHIP(bt, hipStreamSynchronize(bt->stream));
  bt->tiles = *t;
  pf_status st = build_tables(bt);
  if (st == PF_OK) st = bdispatch(bt, [&](auto x) { return build_graphs<decltype(x)>(bt); });
  return st;
}

pf_status pf_batch_get_tiles(const pf_batch* bt, pf_batch_tiles* t) {
  if (!bt || !t) return PF_ERR_INVALID_ARG;
  *t = bt->tiles;
  return PF_OK;
}

pf_status pf_batch_fields(pf_batch* bt, int instance, int field_id, int dir, void* ptr, size_t nbytes, int ptr_is_device) {
  if (!bt) return bfail(nullptr, PF_ERR_INVALID_ARG, "batch is NULL");
  if (!ptr) return bfail(bt, PF_ERR_INVALID_ARG, "ptr is NULL");
  if (instance < 0 || instance >= bt->L.count) return bfail(bt, PF_ERR_INVALID_ARG, "instance out of range");
  if (dir != 0 && dir != 1) return bfail(bt, PF_ERR_INVALID_ARG, "dir must be 0 or 1");
  const BatchLayout& L = bt->L;
  const InstDesc& d = L.inst[instance];
  Grid g = d.g;
  int cx = g.nx, cy = g.ny, cz = 1, zaxis = -1, ncomp = 1;
  size_t base, base_lo = 0;
  switch (field_id) {
    case PF_FIELD_PHI_F: case PF_FIELD_PHI_W: case PF_FIELD_XO: case PF_FIELD_XH: case PF_FIELD_XW:
      base = L.o_fld[bt->cur][field_id];
      base_lo = L.o_lo[bt->cur][field_id];
      break;
    case PF_FIELD_UX: base = L.o_u[0]; cx += 1; zaxis = 0; break;
    case PF_FIELD_UY: base = L.o_u[1]; cy += 1; zaxis = 1; break;
    case PF_FIELD_EPSP: base = L.o_epsp; ncomp = 4; break;
    case PF_FIELD_EPSP_ACC: base = L.o_epsP; break;
    default: return bfail(bt, PF_ERR_INVALID_ARG, "unknown or unsupported field id %d", field_id);
  }
  const size_t per = (size_t)cx * cy * cz;
  if (nbytes != per * ncomp * sizeof(double))
    return bfail(bt, PF_ERR_INVALID_ARG, "field %d needs %zu bytes, got %zu", field_id, per * ncomp * sizeof(double), nbytes);
  double* stage = bt->arr<double>(L.o_stage);
  const int nthr = 256, nblk = (int)((per + nthr - 1) / nthr);
  for (int comp = 0; comp < ncomp; ++comp) {
    const size_t dev_off = base + ((size_t)comp * L.N + d.off) * L.es;
    const size_t lo_off = base_lo ? base_lo + (size_t)d.off * L.es : 0;
    char* user = reinterpret_cast<char*>(ptr) + comp * per * sizeof(double);
    double* buf = ptr_is_device ? reinterpret_cast<double*>(user) : stage;
    if (dir == 1) {
      if (!ptr_is_device) BHIP(bt, hipMemcpyAsync(stage, user, per * sizeof(double), hipMemcpyHostToDevice, bt->stream));
      if (L.es == 8)
        hipLaunchKernelGGL(k_unpack<double>, dim3(nblk), dim3(nthr), 0, bt->stream, (const double*)buf, bt->arr<double>(dev_off), g, cx, cy, cz, zaxis);
      else if (lo_off)
        hipLaunchKernelGGL(k_unpack_pair, dim3(nblk), dim3(nthr), 0, bt->stream, (const double*)buf, bt->arr<float>(dev_off),
                           bt->arr<float>(lo_off), g, cx, cy, cz);
      else
        hipLaunchKernelGGL(k_unpack<float>, dim3(nblk), dim3(nthr), 0, bt->stream, (const double*)buf, bt->arr<float>(dev_off), g, cx, cy, cz, zaxis);
    } else {
      if (L.es == 8)
        hipLaunchKernelGGL(k_pack<double>, dim3(nblk), dim3(nthr), 0, bt->stream, (const double*)bt->arr<double>(dev_off), buf, g, cx, cy, cz);
      else if (lo_off)
        hipLaunchKernelGGL(k_pack_pair, dim3(nblk), dim3(nthr), 0, bt->stream, (const float*)bt->arr<float>(dev_off),
                           (const float*)bt->arr<float>(lo_off), buf, g, cx, cy, cz);
      else
        hipLaunchKernelGGL(k_pack<float>, dim3(nblk), dim3(nthr), 0, bt->stream, (const float*)bt->arr<float>(dev_off), buf, g, cx, cy, cz);
      if (!ptr_is_device) BHIP(bt, hipMemcpyAsync(user, stage, per * sizeof(double), hipMemcpyDeviceToHost, bt->stream));
    }
    BHIP(bt, hipGetLastError());
    if (!ptr_is_device) BHIP(bt, hipStreamSynchronize(bt->stream));   // the staging buffer is reused
  }
  if (dir == 1 && field_id <= PF_FIELD_XW) bt->ledger_valid = false;
  BHIP(bt, hipStreamSynchronize(bt->stream));
  return PF_OK;
}

pf_status pf_batch_step(pf_batch* bt, int nsteps, pf_step_stats* stats) {
  if (!bt) return bfail(nullptr, PF_ERR_INVALID_ARG, "batch is NULL");
  if (bt->bad) return bfail(bt, PF_ERR_BAD_STATE, "batch failed earlier; create a new one");
  if (nsteps < 0) return bfail(bt, PF_ERR_INVALID_ARG, "nsteps < 0");
  const BatchLayout& L = bt->L;
  if (!bt->ledger_valid) {
    pf_status st = bdispatch(bt, [&](auto t) -> pf_status {
      using T = decltype(t);
      BatchArgs<T> B = batch_args<T>(bt, bt->cur);
      hipLaunchKernelGGL(k_batch_totals<T>, dim3(L.n_ce), dim3(NT), 0, bt->stream, B);
      hipLaunchKernelGGL(k_batch_ledger_init<T>, dim3(L.count), dim3(NT), 0, bt->stream, B);
      BHIP(bt, hipGetLastError());
      return PF_OK;
    });
    if (st != PF_OK) return st;
    bt->ledger_valid = true;
  }
  for (int s = 0; s < nsteps; ++s) {
    BHIP(bt, hipGraphLaunch(bt->exec[bt->cur], bt->stream));
    bt->cur ^= 1;
    bt->steps += 1;
  }
  BHIP(bt, hipMemcpyAsync(bt->host_iscal, bt->ws + L.o_iscal, (size_t)L.count * S_COUNT * sizeof(double),
                          hipMemcpyDeviceToHost, bt->stream));
  unsigned barerr = 0u;
  BHIP(bt, hipMemcpyAsync(&barerr, bt->ws + L.o_bar + W_ERR * sizeof(unsigned), sizeof barerr, hipMemcpyDeviceToHost,
                          bt->stream));
  BHIP(bt, hipStreamSynchronize(bt->stream));
  if (barerr != 0u) {
    bt->bad = true;
    return bfail(bt, PF_ERR_HIP, "a grid barrier of the batch kernel timed out (blocks not co-resident?)");
  }
  pf_status result = PF_OK;
  for (int b = 0; b < L.count; ++b) {
    const double* h = bt->host_iscal + (size_t)b * S_COUNT;
    pf_step_stats s;
    memset(&s, 0, sizeof s);
    s.cg_iters = (int)h[S_ITERS];
    s.warm_used = PF_WARM_PREV;
    s.cg_rel_resid = h[S_BB] > 0.0 ? std::sqrt(h[S_TRUE] / h[S_BB]) : 0.0;
    s.O_tot = h[S_OTOT];
    s.O_out = h[S_OOUT];
    s.O_drift = h[S_O0] != 0.0 ? (h[S_OTOT] + h[S_OOUT] - h[S_O0]) / h[S_O0] : 0.0;
    s.H_tot = h[S_HTOT];
    s.H_out = h[S_HOUT];
    s.H_drift = h[S_H0] != 0.0 ? (h[S_HTOT] + h[S_HOUT] - h[S_H0]) / h[S_H0] : 0.0;
    s.red_degree = h[S_XO0] != 0.0 ? 1.0 - h[S_XOSUM] / h[S_XO0] : 0.0;
    s.max_vm = h[S_MAXVM];
    s.max_epsP = h[S_MAXEP];
    s.step = bt->steps;
    s.nonfinite = (int)h[S_NONFIN];
    if (stats) stats[b] = s;
    if (nsteps > 0 && result == PF_OK) {
      if (h[S_CONV] == 0.0)
        result = bfail(bt, PF_ERR_CG_NOT_CONVERGED, "instance %d: CG did not reach rtol in %d iterations", b, bt->cfg.cg_max_iter);
      else if (s.nonfinite > 0)
        result = bfail(bt, PF_ERR_NONFINITE, "instance %d: %d non-finite cells", b, s.nonfinite);
      else if (bt->cfg.ledger_tol > 0.0 && std::fabs(s.O_drift) > bt->cfg.ledger_tol)
        result = bfail(bt, PF_ERR_LEDGER, "instance %d: oxygen ledger drift %.3e", b, s.O_drift);
    }
  }
  if (result != PF_OK) bt->bad = true;
  return result;
}

const char* pf_batch_last_error(const pf_batch* bt) { return bt ? bt->err : g_err; }

void pf_batch_destroy(pf_batch* bt) {
  if (!bt) return;
  (void)hipStreamSynchronize(bt->stream);
  if (bt->have_graph)
    for (int s = 0; s < 2; ++s) {
      (void)hipGraphExecDestroy(bt->exec[s]);
      (void)hipGraphDestroy(bt->graph[s]);
    }
  if (bt->host_iscal) (void)hipHostFree(bt->host_iscal);
  delete bt;
}

}  // extern "C"
