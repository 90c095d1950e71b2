// Batched 2D stepping of many uneven instances in one persistent launch.
//
// Every instance keeps its own grid, CG recurrence and ledger; their arrays
// are packed one after another in shared buffers.  Work is described by tile
// tables (elasticity 64x4 tiles, CG apply strips of 62 columns taken one per
// wave, cell tiles, CG update chunks) that the persistent blocks walk with a
// fixed stride; phases are
// separated by a grid barrier whose wait is bounded (a timeout raises an error
// flag and every block leaves), so the launch always drains.
#pragma once

#include "pf_kernels.h"

namespace pfk {

constexpr int kMaxBatch = 256;

struct InstDesc {
  Grid g;          // the instance's own grid; g.ns = packed component stride of eps_p
  int off;         // element offset of the instance in every packed array (multiple of 64)
  int el0, eln;    // range in the elasticity tile table
  int ap0, apn;    // range in the apply strip table (A2S columns x kz_ap rows, one per wave)
  int ce0, cen;    // range in the cell tile table
  int up0, upn;    // range in the update chunk table
  int apf0, apfn;  // range of the fine apply strips (fewer rows per strip)
  int upf0, upfn;  // range of the fine update chunks
};
struct TileRef {
  int inst, bx, by, bz;
};
struct ChunkRef {
  int inst, v0, v1, pad;   // 16-byte vector range relative to the instance
};

template <typename T>
struct BatchArgs {
  int count;
  const InstDesc* inst;
  const TileRef* el;
  int n_el;
  const TileRef* ap;
  int n_ap;
  const TileRef* ce;
  int n_ce;
  const ChunkRef* up;
  int n_up;
  KP<T> p;
  T* f_old[5];             // current fields phi_f, phi_w, x_O, x_H, x_H2O
  T* f_new[5];             // where the step writes the next ones
  T* lo_old[5];            // FP32 state: low parts of the current fields (null in FP64)
  T* lo_new[5];
  T* u[2];
  T* epsp;
  T* epsP;
  T* mu;
  T* K;
  T* G;
  T* r[2];
  T* z[2];
  T* pa[2];
  T* pb[2];
  T* q[2];
  T* dinv[2];
  double* part_bn;         // [n_el]
  double* part_r;          // [2][n_el]
  double* part_a;          // [n_ap]
  double* part_u;          // [2 parity][2][n_up]
  double* part_t;          // [n_el]
  double* part_c;          // [NQ_STEP][n_ce]
  double* iscal;           // [count][S_COUNT]
  unsigned* bar;           // {arrivals, generation, error}
  double tol2;
  int max_iter;
  int kz_ap;                  // rows per coarse apply strip
  int kz_apf;                 // rows per fine apply strip
  double area_dt;
  double vol;
  long long spin_limit;
};

// Barrier words (unsigned, 64 apart so that no two share a cache line).
constexpr int W_ARR = 0;          // arrivals (blocks, or groups in the grouped barrier)
constexpr int W_GEN = 64;         // generation, published by the last arrival
constexpr int W_ERR = 128;        // set when a bounded wait gave up
constexpr int W_MIS = 192;        // set when a block did not run on the XCD its index predicts
constexpr int W_GARR = 256;       // + 64 x: arrivals within XCD group x
constexpr int W_GREL = 768;       // + 64 x: release of XCD group x
constexpr int kBarWords = 1280;

// Bounded wait until *w == target; false (and the error word set) on timeout
// or when another block already gave up.
__device__ __forceinline__ bool bar_wait(unsigned* bar, const unsigned* w, unsigned target, long long spin_limit,
                                         int sleep) {
  long long spins = 0;
  while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
    if (__hip_atomic_load(&bar[W_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
    if (++spins > spin_limit) {
      __hip_atomic_store(&bar[W_ERR], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    if (sleep) __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// Grid-wide barrier for a launch whose blocks are all resident.
//
// Flat form: every block makes its writes visible device-wide (release fence
// at agent scope: write-back of its XCD's L2), arrives on one counter; the
// last arrival publishes the next generation; every block then invalidates
// its caches (acquire at agent scope).
//
// Grouped form (when every block runs on XCD blockIdx % 8, checked at launch):
// the blocks of one XCD share an L2, so only the last arrival of each XCD
// group writes that L2 back (release at agent scope) before arriving on the
// global counter, on behalf of the group whose stores it has observed through
// the group counter; the group leaders wait for the generation and release
// their groups, and every block then acquires at agent scope.  This replaces
// one L2 write-back per block by one per XCD and keeps the global counter to
// eight arrivals.
//
// Waits are bounded (spin_limit polls): a block that gives up sets the error
// word, and every block that sees it leaves, so the grid always drains.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, unsigned& gen, long long spin_limit,
                                             int grouped, int* flag_sh) {
  __syncthreads();
  if (threadIdx.x == 0) {
    bool ok = true;
    const unsigned target = gen + 1u;
    if (!grouped) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned prev = __hip_atomic_fetch_add(&bar[W_ARR], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == nblocks - 1u) {
        __hip_atomic_store(&bar[W_ARR], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);        // the reset lands before anyone can arrive again
        __hip_atomic_store(&bar[W_GEN], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ok = bar_wait(bar, &bar[W_GEN], target, spin_limit, 1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    } else {
      const unsigned x = blockIdx.x % kXCD;
      const unsigned ngroups = nblocks < (unsigned)kXCD ? nblocks : (unsigned)kXCD;
      const unsigned gsize = nblocks / kXCD + (x < nblocks % kXCD ? 1u : 0u);
      const unsigned prev = __hip_atomic_fetch_add(&bar[W_GARR + 64 * x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == gsize - 1u) {
        __hip_atomic_store(&bar[W_GARR + 64 * x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // also completes the reset above
        const unsigned gp = __hip_atomic_fetch_add(&bar[W_ARR], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gp == ngroups - 1u) {
          __hip_atomic_store(&bar[W_ARR], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __builtin_amdgcn_s_waitcnt(0);      // the reset lands before anyone can arrive again
          __hip_atomic_store(&bar[W_GEN], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          ok = bar_wait(bar, &bar[W_GEN], target, spin_limit, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __builtin_amdgcn_s_waitcnt(0);          // the invalidate has completed before the group is released
        __hip_atomic_store(&bar[W_GREL + 64 * x], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ok = bar_wait(bar, &bar[W_GREL + 64 * x], target, spin_limit, 1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    gen = target;
    *flag_sh = ok ? 1 : 0;
  }
  __syncthreads();
  return *flag_sh != 0;
}

// Sum of part[r0 .. r0+n) in a fixed order, eight independent loads in flight.
__device__ __forceinline__ double range_sum(const double* part, int r0, int n) {
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int q = 0;
  for (; q + 8 <= n; q += 8)
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] += part[r0 + q + k];
  for (; q < n; ++q) s[0] += part[r0 + q];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Inclusive prefix sums over the instances of two per-instance counts (zero
// for converged instances) into shared memory; count <= NT.  Wave-level
// shuffle scans, then the wave totals; two block synchronisations.
__device__ __forceinline__ void active_scan2(int* sha, int* shb, int va, int vb, int count) {
  __shared__ int tot[2][NT / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t >= count) va = vb = 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int xa = __shfl_up(va, o, 64), xb = __shfl_up(vb, o, 64);
    if (lane >= o) { va += xa; vb += xb; }
  }
  if (lane == 63) { tot[0][w] = va; tot[1][w] = vb; }
  __syncthreads();
  for (int q = 0; q < w; ++q) { va += tot[0][q]; vb += tot[1][q]; }
  if (t < count) { sha[t] = va; shb[t] = vb; }
  __syncthreads();
}

// Per-instance sums of the partial ranges [r0(b), r0(b) + rn(b)) of two
// partial arrays, eight lanes per instance with a fixed split and combination
// order, so every block obtains the same values.  Instances with skip[b] set
// are not summed and keep their outputs.  Ends with a block synchronisation.
template <typename R0, typename RN>
__device__ __forceinline__ void instance_sums2(const double* pa, const double* pb, int count, R0 r0, RN rn,
                                               const int* skip, double* oa, double* ob) {
  constexpr int kL = 8;
  const int t = threadIdx.x, q = t & (kL - 1);
  for (int base = 0; base < count; base += NT / kL) {
    const int b = base + t / kL;
    const bool on = b < count && !(skip && skip[b]);
    double sa = 0.0, sb = 0.0;
    if (on) {
      const int a0 = r0(b), n = rn(b);
      for (int k = q; k < n; k += kL) {
        sa += pa[a0 + k];
        if (pb) sb += pb[a0 + k];
      }
    }
#pragma unroll
    for (int o = 1; o < kL; o <<= 1) {
      sa += __shfl_xor(sa, o, 64);
      sb += __shfl_xor(sb, o, 64);
    }
    if (on && q == 0) {
      oa[b] = sa;
      if (ob) ob[b] = sb;
    }
  }
  __syncthreads();
}

// Instance b holding active work item w: incl[b-1] <= w < incl[b].
__device__ __forceinline__ int active_owner(const int* incl, int count, int w) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (incl[mid] > w) hi = mid; else lo = mid + 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ ElastArgs<T> elast_view(const BatchArgs<T>& B, const InstDesc& d) {
  ElastArgs<T> a{};
  a.g = d.g;
  a.p = B.p;
  a.K = B.K + d.off;
  a.G = B.G + d.off;
  a.phi_f = B.f_old[0] + d.off;
  a.epsp = B.epsp + d.off;
  a.kz = B.kz_ap;
  return a;
}

template <typename T>
__device__ __forceinline__ CellArgs<T> cell_view(const BatchArgs<T>& B, const InstDesc& d) {
  CellArgs<T> a{};
  a.g = d.g;
  a.p = B.p;
  a.pf = B.f_old[0] + d.off; a.pw = B.f_old[1] + d.off; a.xO = B.f_old[2] + d.off;
  a.xH = B.f_old[3] + d.off; a.xW = B.f_old[4] + d.off;
  a.npf = B.f_new[0] + d.off; a.npw = B.f_new[1] + d.off; a.nxO = B.f_new[2] + d.off;
  a.nxH = B.f_new[3] + d.off; a.nxW = B.f_new[4] + d.off;
  if constexpr (sizeof(T) == 4)
    for (int f = 0; f < 5; ++f) {
      a.lo[f] = B.lo_old[f] + d.off;
      a.nlo[f] = B.lo_new[f] + d.off;
    }
  a.mu = B.mu + d.off;
  a.mu_out = B.mu + d.off;
  a.u[0] = B.u[0] + d.off;
  a.u[1] = B.u[1] + d.off;
  a.epsp = B.epsp + d.off;
  a.epsP = B.epsP + d.off;
  a.K = B.K + d.off;
  a.G = B.G + d.off;
  a.part = B.part_c;
  return a;
}

template <typename T>
constexpr size_t batch_smem() {
  return sizeof(ElastSmem<T, 2, M_RESID>);
}

#define PF_BARRIER()                                                                   \
  do {                                                                                 \
    if (!grid_barrier(B.bar, nbk, gen, B.spin_limit, grouped, &flag_sh)) return;       \
  } while (0)

// One explicit step of every instance (2D): moduli, ||b||, initial residual,
// the CG loop until every instance has converged, true residual, mu, the
// fused field update and the per-instance ledger.
template <typename T>
__global__ __launch_bounds__(NT) void k_batch_step(BatchArgs<T> B) {
  __shared__ __align__(16) char smem[batch_smem<T>()];
  __shared__ double shA[kMaxBatch], shB[kMaxBatch], shBB[kMaxBatch];
  __shared__ int shC[kMaxBatch];
  __shared__ int shAp[kMaxBatch], shUp[kMaxBatch];   // inclusive prefix sums of active apply tiles / update chunks
  __shared__ double shRzPrev[kMaxBatch];              // r.z of the previous pass
  __shared__ double shRR[kMaxBatch], shPQ[kMaxBatch];  // r.r of this pass, p.q
  __shared__ int up_fine_sh;                          // the last update pass used the fine chunks
  __shared__ int flag_sh, all_sh;
  __shared__ double red[2 * (NT / 64)];
  __shared__ int grouped_sh;
  unsigned gen = 0u;
  int grouped = 0;                 // the first barrier is flat; it publishes the XCD check
  if (threadIdx.x == 0) {
    gen = __hip_atomic_load(&B.bar[W_GEN], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // XCC_ID hardware register (bits 3:0): the XCD this block runs on
    const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 0xFu;
    if (xcc != blockIdx.x % kXCD) __hip_atomic_fetch_or(&B.bar[W_MIS], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const unsigned nbk = gridDim.x;
  const int tid = threadIdx.x;
  const int S = S_COUNT;

  // (1) effective moduli
  for (int w = blockIdx.x; w < B.n_ce; w += nbk) {
    const TileRef tr = B.ce[w];
    const CellArgs<T> a = cell_view(B, B.inst[tr.inst]);
    moduli_tile<T, 2>(a, tr.bx, tr.by, tr.bz);
  }
  PF_BARRIER();
  if (tid == 0) grouped_sh = __hip_atomic_load(&B.bar[W_MIS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
  __syncthreads();
  grouped = grouped_sh;
  // (2) ||b||^2 partials
  for (int w = blockIdx.x; w < B.n_el; w += nbk) {
    const TileRef tr = B.el[w];
    ElastArgs<T> a = elast_view(B, B.inst[tr.inst]);
    a.part = B.part_bn;
    elast_tile<T, 2, M_BNORM>(a, tr.bx, tr.by, tr.bz, false, w, B.n_el, smem);
  }
  PF_BARRIER();
  instance_sums2(B.part_bn, nullptr, B.count, [&](int b) { return B.inst[b].el0; },
                 [&](int b) { return B.inst[b].eln; }, nullptr, shBB, nullptr);
  // (3) initial residual r = b - A u, D^-1, z
  for (int w = blockIdx.x; w < B.n_el; w += nbk) {
    const TileRef tr = B.el[w];
    const InstDesc& d = B.inst[tr.inst];
    ElastArgs<T> a = elast_view(B, d);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      a.u[c] = B.u[c] + d.off;
      a.o1[c] = B.r[c] + d.off;
      a.o2[c] = B.z[c] + d.off;
      a.dinv[c] = B.dinv[c] + d.off;
    }
    a.part = B.part_r;
    elast_tile<T, 2, M_RESID>(a, tr.bx, tr.by, tr.bz, shBB[tr.inst] == 0.0, w, B.n_el, smem);
  }
  if (tid == 0)
    for (int b = blockIdx.x; b < B.count; b += nbk) {
      B.iscal[b * S + S_BB] = shBB[b];
      B.iscal[b * S + S_ITERS] = 0.0;
      B.iscal[b * S + S_CONV] = 0.0;
    }
  PF_BARRIER();

  // (4) CG, one recurrence per instance
  if (tid == 0) up_fine_sh = 0;
  for (int L = 0;; ++L) {
    // r.z and r.r of every instance from the residual / last update partials;
    // an instance that has converged keeps its flag and its last values
    if (L == 0) {
      instance_sums2(B.part_r, B.part_r + B.n_el, B.count, [&](int b) { return B.inst[b].el0; },
                     [&](int b) { return B.inst[b].eln; }, nullptr, shA, shRR);
    } else {
      const double* pu = B.part_u + ((L - 1) & 1) * 2 * B.n_up;
      if (up_fine_sh)
        instance_sums2(pu, pu + B.n_up, B.count, [&](int b) { return B.inst[b].upf0; },
                       [&](int b) { return B.inst[b].upfn; }, shC, shA, shRR);
      else
        instance_sums2(pu, pu + B.n_up, B.count, [&](int b) { return B.inst[b].up0; },
                       [&](int b) { return B.inst[b].upn; }, shC, shA, shRR);
    }
    for (int b = tid; b < B.count; b += NT) {
      const double rz = shA[b];
      const int conv = (L > 0 && shC[b]) || (shRR[b] <= B.tol2 * shBB[b]);
      shB[b] = (L == 0 || conv) ? 0.0 : rz / shRzPrev[b];
      if (!conv || L == 0) shRzPrev[b] = rz;
      shC[b] = conv;
    }
    __syncthreads();
    if (tid == 0) {
      int all = 1;
      for (int b = 0; b < B.count; ++b) all &= shC[b];
      all_sh = all;
      for (int b = blockIdx.x; b < B.count; b += nbk) {
        B.iscal[b * S + S_CONV] = (double)shC[b];
        B.iscal[b * S + S_RR] = shRR[b];
      }
    }
    __syncthreads();
    if (all_sh || L >= B.max_iter) break;
    // the work items of the instances still iterating, dealt out evenly; when
    // the coarse tiles or chunks of those instances would leave blocks idle,
    // the fine ones (a quarter of the size) are dealt instead
    bool ap_fine, up_fine;
    {
      const bool act = tid < B.count && !shC[tid];
      int ca = 0, cu = 0, fa = 0, fu = 0;
      if (act) {
        const InstDesc& d = B.inst[tid];
        ca = d.apn; cu = d.upn; fa = d.apfn; fu = d.upfn;
      }
      active_scan2(shAp, shUp, ca, cu, B.count);
      ap_fine = shAp[B.count - 1] < (int)nbk * (NT / 64);   // apply strips go one per wave
      up_fine = shUp[B.count - 1] < (int)nbk;
      if (ap_fine || up_fine) active_scan2(shAp, shUp, ap_fine ? fa : ca, up_fine ? fu : cu, B.count);
    }
    const int n_ap_act = shAp[B.count - 1], n_up_act = shUp[B.count - 1];
    // apply: q = A p with p = z + beta p, one strip per wave
    T* const pold[2] = {(L & 1) ? B.pb[0] : B.pa[0], (L & 1) ? B.pb[1] : B.pa[1]};
    T* const pnew[2] = {(L & 1) ? B.pa[0] : B.pb[0], (L & 1) ? B.pa[1] : B.pb[1]};
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int wa = blockIdx.x * (NT / 64) + wv; wa < n_ap_act; wa += nbk * (NT / 64)) {
      const int ib = active_owner(shAp, B.count, wa);
      const InstDesc& d = B.inst[ib];
      const int w = (ap_fine ? d.apf0 : d.ap0) + wa - (ib > 0 ? shAp[ib - 1] : 0);
      const TileRef tr = B.ap[w];
      ElastArgs<T> a = elast_view(B, d);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        a.u[c] = pold[c] + d.off;
        a.z[c] = B.z[c] + d.off;
        a.o1[c] = pnew[c] + d.off;
        a.o2[c] = B.q[c] + d.off;
      }
      const int kz = ap_fine ? B.kz_apf : B.kz_ap;
      const int j0 = tr.by * kz, j1 = min(j0 + kz, d.g.ny);
      const double s = wave_sum(apply2_strip(a, tr.bx, j0, j1, shB[tr.inst], L == 0));
      if ((tid & 63) == 0) B.part_a[w] = s;
    }
    PF_BARRIER();
    // alpha = r.z / p.q of every instance still iterating
    if (ap_fine)
      instance_sums2(B.part_a, nullptr, B.count, [&](int b) { return B.inst[b].apf0; },
                     [&](int b) { return B.inst[b].apfn; }, shC, shPQ, nullptr);
    else
      instance_sums2(B.part_a, nullptr, B.count, [&](int b) { return B.inst[b].ap0; },
                     [&](int b) { return B.inst[b].apn; }, shC, shPQ, nullptr);
    for (int b = tid; b < B.count; b += NT)
      if (!shC[b]) shB[b] = shA[b] / shPQ[b];
    __syncthreads();
    // update: u += alpha p, r -= alpha q, z = D^-1 r
    double* pu = B.part_u + (L & 1) * 2 * B.n_up;
    for (int wu = blockIdx.x; wu < n_up_act; wu += nbk) {
      const int ib = active_owner(shUp, B.count, wu);
      const InstDesc& d = B.inst[ib];
      const int w = (up_fine ? d.upf0 : d.up0) + wu - (ib > 0 ? shUp[ib - 1] : 0);
      const ChunkRef cr = B.up[w];
      UpdArgs<T> a{};
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        a.u[c] = B.u[c] + d.off;
        a.p[c] = pnew[c] + d.off;
        a.r[c] = B.r[c] + d.off;
        a.q[c] = B.q[c] + d.off;
        a.dinv[c] = B.dinv[c] + d.off;
        a.z[c] = B.z[c] + d.off;
      }
      double rz = 0.0, rr = 0.0;
      cg_update_range<T, 2>(a, cr.v0 + tid, cr.v1, NT, shB[cr.inst], rz, rr);
      block_sum2(rz, rr, red);
      if (tid == 0) {
        pu[w] = rz;
        pu[B.n_up + w] = rr;
      }
    }
    if (tid == 0)
      for (int b = blockIdx.x; b < B.count; b += nbk)
        if (!shC[b]) B.iscal[b * S + S_ITERS] += 1.0;
    if (tid == 0) up_fine_sh = up_fine ? 1 : 0;       // read by the next pass after the barrier's block sync
    PF_BARRIER();
  }

  // (5) true residual
  for (int w = blockIdx.x; w < B.n_el; w += nbk) {
    const TileRef tr = B.el[w];
    const InstDesc& d = B.inst[tr.inst];
    ElastArgs<T> a = elast_view(B, d);
    a.u[0] = B.u[0] + d.off;
    a.u[1] = B.u[1] + d.off;
    a.part = B.part_t;
    elast_tile<T, 2, M_TRUE>(a, tr.bx, tr.by, tr.bz, false, w, B.n_el, smem);
  }
  // (6) oxygen chemical potential
  for (int w = blockIdx.x; w < B.n_ce; w += nbk) {
    const TileRef tr = B.ce[w];
    const CellArgs<T> a = cell_view(B, B.inst[tr.inst]);
    mu_tile<T, 2>(a, tr.bx, tr.by, tr.bz);
  }
  PF_BARRIER();
  if (tid == 0)
    for (int b = blockIdx.x; b < B.count; b += nbk) B.iscal[b * S + S_TRUE] = range_sum(B.part_t, B.inst[b].el0, B.inst[b].eln);
  // (7) fused chemistry / phase-field / plasticity update
  for (int w = blockIdx.x; w < B.n_ce; w += nbk) {
    const TileRef tr = B.ce[w];
    const CellArgs<T> a = cell_view(B, B.inst[tr.inst]);
    step_tile<T, 2>(a, tr.bx, tr.by, tr.bz, w, B.n_ce);
  }
  PF_BARRIER();
  // (8) per-instance ledger and statistics
  for (int b = blockIdx.x; b < B.count; b += nbk) {
    const InstDesc& d = B.inst[b];
    const double* P = B.part_c;
    double v[5], mx[2], nf = 0.0;
    for (int qn = 0; qn < 5; ++qn) {
      double s = 0.0;
      for (int q = tid; q < d.cen; q += NT) s += P[qn * B.n_ce + d.ce0 + q];
      v[qn] = block_sum(s, red);
    }
    for (int qn = 0; qn < 2; ++qn) {
      double m = 0.0;
      for (int q = tid; q < d.cen; q += NT) m = fmax(m, P[(5 + qn) * B.n_ce + d.ce0 + q]);
      mx[qn] = block_max(m, red);
    }
    {
      double s = 0.0;
      for (int q = tid; q < d.cen; q += NT) s += P[7 * B.n_ce + d.ce0 + q];
      nf = block_sum(s, red);
    }
    if (tid == 0) {
      double* sc = B.iscal + b * S;
      sc[S_OOUT] += B.area_dt * v[3];
      sc[S_HOUT] += B.area_dt * v[4];
      sc[S_OTOT] = v[0] * B.vol;
      sc[S_HTOT] = v[1] * B.vol;
      sc[S_XOSUM] = v[2];
      sc[S_MAXVM] = mx[0];
      sc[S_MAXEP] = mx[1];
      sc[S_NONFIN] = nf;
    }
  }
}

// Ledger reset of every instance: totals of the current fields.
template <typename T>
__global__ __launch_bounds__(NT) void k_batch_totals(BatchArgs<T> B) {
  const int w = blockIdx.x;
  if (w >= B.n_ce) return;
  const TileRef tr = B.ce[w];
  const CellArgs<T> a = cell_view(B, B.inst[tr.inst]);
  totals_tile<T, 2>(a, tr.bx, tr.by, tr.bz, w, B.n_ce);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_batch_ledger_init(BatchArgs<T> B) {
  __shared__ double red[NT / 64];
  const int b = blockIdx.x;
  if (b >= B.count) return;
  const InstDesc& d = B.inst[b];
  double v[3];
  for (int qn = 0; qn < 3; ++qn) {
    double s = 0.0;
    for (int q = threadIdx.x; q < d.cen; q += NT) s += B.part_c[qn * B.n_ce + d.ce0 + q];
    v[qn] = block_sum(s, red);
  }
  if (threadIdx.x == 0) {
    double* sc = B.iscal + b * S_COUNT;
    sc[S_O0] = v[0] * B.vol;
    sc[S_H0] = v[1] * B.vol;
    sc[S_XO0] = v[2];
    sc[S_OOUT] = 0.0;
    sc[S_HOUT] = 0.0;
    sc[S_OTOT] = v[0] * B.vol;
    sc[S_HTOT] = v[1] * B.vol;
    sc[S_XOSUM] = v[2];
  }
}

}  // namespace pfk
