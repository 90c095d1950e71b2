// HIP kernels (gfx950) of the phase-field step.
//
//  k_elast      staggered-grid small-strain elasticity (quasi-static momentum
//               balance, Eq. 29 row 4): q = A p with the CG direction update
//               fused in, the initial residual with the eigenstrain, norms.
//               LDS-staged 64x4 tiles marching along z (2.5D blocking).
//  k_cg_update  x += alpha p, r -= alpha q, z = D^-1 r with FP64 partial dots.
//  k_mu, k_step fused chemistry / phase-field / plasticity update.
//  small kernels for moduli, ledger, checks and field packing.
//
// Every dot product and ledger sum is FP64 and deterministic: each block
// writes one partial, and consumers reduce the partials in a fixed order.
#pragma once

#include <type_traits>

#include "pf_device.h"

namespace pfk {

enum ElastMode { M_APPLY = 0, M_RESID = 1, M_BNORM = 2, M_TRUE = 3 };

template <typename T>
struct ElastArgs {
  Grid g;
  KP<T> p;
  const T* K;
  const T* G;
  const T* phi_f;          // eigenstrain source (modes other than APPLY)
  const T* epsp;           // plastic strain, component-major with stride g.ns
  T* u[3];                 // APPLY: previous direction p; RESID/TRUE: displacement
  const T* z[3];           // APPLY: preconditioned residual
  T* o1[3];                // APPLY: new direction; RESID: residual r
  T* o2[3];                // APPLY: q = A p; RESID: z = D^-1 r
  T* dinv[3];              // RESID: inverse diagonal of A
  double* part;            // partial sums out, [quantity][block]
  const double* part_in;   // partial sums to reduce at entry
  int n_in;
  double* scal;
  double tol2;             // cg_rtol^2
  int parity;              // launch position parity inside the CG loop
  int kz;                  // z planes per block
  const T* jr[3];          // APPLY_PLAIN (3D): if set, the partials are ||jr - q||^2 instead of z.q;
                           // APPLY_RESID: b.  The residual pass writes r = b - q into o1, z = D^-1 r
                           // into o2 (q not stored) and partials r.z, r.r; it opens the solve's scalars
                           // from the ||b||^2 partials part_in[0..n_in), and with b = 0 sets the
                           // vector (u[]) and r, z to zero
  const T* phi_w;          // k_setup3: water phase (with phi_f, the moduli it computes)
  T* Kw;                   // k_setup3: the moduli K, G it writes for the apply kernels
  T* Gw;
  T* xs[3];                // APPLY_CG (3D): the solution (completed by the launch that stops the solve)
  int it;                  // APPLY_CG (3D): index of this launch in the solve
  double omega;            // APPLY_SMOOTH(0): step of the Jacobi sweep (0: write the residual instead)
  double omega0;           // APPLY_SMOOTH0: step of the first sweep from zero
  // APPLY_SMOOTH(0) in FP32: bf16 copies of K, G and D^-1 of the level, which
  // the multigrid sweeps read instead of K, G and dinv (the residual sweep of
  // the cycle uses the same copies, so every sweep of a level applies one
  // operator; CG itself keeps the FP32 moduli)
  const unsigned short* lo_K;
  const unsigned short* lo_G;
  const unsigned short* lo_d[3];
  unsigned short* lo_w[5]; // k_setup3 (FP32): if set, also writes those copies of K, G, D^-1 (x, y, z)
};

// Local tile coordinates: lx = i - i0 + 1 in [0, TX+1], ly = j - j0 + 1 in [0, TY+1].
constexpr int LW = TX + 2, LH = TY + 2, LS = LW * LH;
__device__ __forceinline__ int L(int ly, int lx) { return ly * LW + lx; }

// One 64 x 4 tile (marching over kz planes in 3D) of the elasticity operator
// in the modes RESID (r = b - A u, z = D^-1 r, D^-1; partials r.z, r.r),
// BNORM (||b||^2 partial) and TRUE (||b - A u||^2 partial).  Partials go to
// a.part[pidx] and a.part[pstride + pidx].
// LDS layout of elast_tile (carved from a caller-provided shared buffer so that
// several tile functions in one kernel share the same LDS).
template <typename T, int DIM, int MODE>
struct ElastSmem {
  static constexpr int D3 = (DIM == 3) ? LS : 1;
  static constexpr int R3 = (MODE == M_RESID && DIM == 3) ? LS : 1;
  double red[NT / 64];
  T sP[2][DIM][LS];
  T sK[LS];
  T sG[2][LS];
  T sSxx[LS], sSyy[LS], sSzz[LS], sSxy[LS];
  T sSxz[2][D3], sSyz[2][D3];
  T sEt[LS], sEn[3][LS], sExy[LS];
  T sExz[2][D3], sEyz[2][D3];
  T sGxz[2][R3], sGyz[2][R3];
};

template <typename T, int DIM, int MODE>
__device__ __forceinline__ void elast_tile(const ElastArgs<T>& a, int bx, int by, int bz, bool zero_u, int pidx,
                                           int pstride, char* smem) {
  static_assert(MODE != M_APPLY, "the apply has its own kernels");
  constexpr bool EIG = true;
  ElastSmem<T, DIM, MODE>& SM = *reinterpret_cast<ElastSmem<T, DIM, MODE>*>(smem);
  auto& sP = SM.sP;
  auto& sK = SM.sK;
  auto& sG = SM.sG;
  auto& sSxx = SM.sSxx;
  auto& sSyy = SM.sSyy;
  auto& sSzz = SM.sSzz;
  auto& sSxy = SM.sSxy;
  auto& sSxz = SM.sSxz;
  auto& sSyz = SM.sSyz;
  auto& sEt = SM.sEt;
  auto& sEn = SM.sEn;
  auto& sExy = SM.sExy;
  auto& sExz = SM.sExz;
  auto& sEyz = SM.sEyz;
  auto& sGxz = SM.sGxz;
  auto& sGyz = SM.sGyz;
  double* red = SM.red;
  (void)sGxz; (void)sGyz; (void)sExz; (void)sEyz; (void)sSxz; (void)sSyz;

  const Grid& g = a.g;
  const KP<T>& p = a.p;
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int i0 = bx * TX, j0 = by * TY;
  const int i = i0 + tx, j = j0 + ty;
  const int lx = tx + 1, ly = ty + 1;
  const bool own = (i < g.nx) && (j < g.ny);
  const T ih = p.ih;

  // ---- plane loaders ------------------------------------------------------
  auto in_dom = [&](int ii, int jj, int kk) {
    return ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
  };
  auto load_vec = [&](int kk, int slot) {
    for (int t = threadIdx.x; t < LS; t += NT) {
      int yy = t / LW, xx = t - yy * LW;
      int ii = i0 + xx - 1, jj = j0 + yy - 1;
      bool in = in_dom(ii, jj, kk);
      int e = in ? gidx(g, ii, jj, kk) : 0;
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        T v = T(0);
        if (in) {
          if (MODE == M_BNORM) v = T(0);
          else v = zero_u ? T(0) : a.u[c][e];
        }
        sP[slot][c][t] = v;
      }
    }
  };
  auto load_cell = [&](const T* src, T* dst, int kk) {
    for (int t = threadIdx.x; t < LS; t += NT) {
      int yy = t / LW, xx = t - yy * LW;
      int ii = i0 + xx - 1, jj = j0 + yy - 1;
      dst[t] = in_dom(ii, jj, kk) ? src[gidx(g, ii, jj, kk)] : T(0);
    }
  };
  auto load_eig = [&](int kk) {   // eigenstrain eT and plastic strain of plane kk
    for (int t = threadIdx.x; t < LS; t += NT) {
      int yy = t / LW, xx = t - yy * LW;
      int ii = i0 + xx - 1, jj = j0 + yy - 1;
      bool in = in_dom(ii, jj, kk);
      int e = in ? gidx(g, ii, jj, kk) : 0;
      sEt[t] = in ? eigen_strain(p, a.phi_f[e]) : T(0);
      sEn[0][t] = in ? a.epsp[e] : T(0);
      sEn[1][t] = in ? a.epsp[g.ns + e] : T(0);
      sEn[2][t] = in ? a.epsp[2 * g.ns + e] : T(0);
      sExy[t] = in ? a.epsp[3 * g.ns + e] : T(0);
    }
  };
  auto load_eig_shear3 = [&](int kk, int slot) {   // xz, yz plastic strain of plane kk
    if constexpr (EIG && DIM == 3) {
      for (int t = threadIdx.x; t < LS; t += NT) {
        int yy = t / LW, xx = t - yy * LW;
        int ii = i0 + xx - 1, jj = j0 + yy - 1;
        bool in = in_dom(ii, jj, kk);
        int e = in ? gidx(g, ii, jj, kk) : 0;
        sExz[slot][t] = in ? a.epsp[4 * g.ns + e] : T(0);
        sEyz[slot][t] = in ? a.epsp[5 * g.ns + e] : T(0);
      }
    }
  };

  // ---- stress evaluations ---------------------------------------------------
  // cell normal stresses of plane k on cells lx in [0, TX], ly in [0, TY]
  auto cell_stress = [&](int sk, int sk1) {
    for (int t = threadIdx.x; t < (TX + 1) * (TY + 1); t += NT) {
      int yy = t / (TX + 1), xx = t - yy * (TX + 1);
      int c = L(yy, xx);
      T exx = (sP[sk][0][c + 1] - sP[sk][0][c]) * ih;
      T eyy = (sP[sk][1][c + LW] - sP[sk][1][c]) * ih;
      T ezz = T(0);
      if constexpr (DIM == 3) ezz = (sP[sk1][2][c] - sP[sk][2][c]) * ih;
      if constexpr (EIG) {
        exx -= sEt[c] + sEn[0][c];
        eyy -= sEt[c] + sEn[1][c];
        ezz -= sEt[c] + sEn[2][c];
      }
      T tr = exx + eyy + ezz;
      T Kc = sK[c], G2 = T(2) * sG[sk][c];
      T lam = Kc * tr - G2 * tr * T(1.0 / 3.0);
      sSxx[c] = lam + G2 * exx;
      sSyy[c] = lam + G2 * eyy;
      sSzz[c] = lam + G2 * ezz;
    }
  };
  // xy edge stresses of plane k on edges lx in [1, TX+1], ly in [1, TY+1]
  auto edge_xy = [&](int sk, int kk) {
    for (int t = threadIdx.x; t < (TX + 1) * (TY + 1); t += NT) {
      int yy = t / (TX + 1) + 1, xx = t - (yy - 1) * (TX + 1) + 1;
      int c = L(yy, xx);
      int ii = i0 + xx - 1, jj = j0 + yy - 1;
      T s = T(0);
      if (ii > 0 && ii < g.nx && jj > 0 && jj < g.ny) {
        T ge = T(0.25) * (sG[sk][c - LW - 1] + sG[sk][c - LW] + sG[sk][c - 1] + sG[sk][c]);
        T e = T(0.5) * ((sP[sk][0][c] - sP[sk][0][c - LW]) + (sP[sk][1][c] - sP[sk][1][c - 1])) * ih;
        if constexpr (EIG) e -= T(0.25) * (sExy[c - LW - 1] + sExy[c - LW] + sExy[c - 1] + sExy[c]);
        s = T(2) * ge * e;
      }
      sSxy[c] = s;
    }
    (void)kk;
  };
  // xz / yz edge stresses at level kk (between planes kk-1 in slot s0 and kk in slot s1)
  auto edge_z = [&](int kk, int s0, int s1, int out) {
    if constexpr (DIM == 3) {
      bool zin = kk > 0 && kk < g.nz;
      for (int t = threadIdx.x; t < (TX + 1) * (TY + 1); t += NT) {
        int yy = t / (TX + 1) + 1, xx = t - (yy - 1) * (TX + 1) + 1;
        int c = L(yy, xx);
        int ii = i0 + xx - 1, jj = j0 + yy - 1;
        T sxz = T(0), syz = T(0), gxz = T(0), gyz = T(0);
        if (zin && ii > 0 && ii < g.nx && jj < g.ny && yy <= TY) {
          gxz = T(0.25) * (sG[s0][c - 1] + sG[s0][c] + sG[s1][c - 1] + sG[s1][c]);
          T e = T(0.5) * ((sP[s1][0][c] - sP[s0][0][c]) + (sP[s1][2][c] - sP[s1][2][c - 1])) * ih;
          if constexpr (EIG) e -= T(0.25) * (sExz[s0][c - 1] + sExz[s0][c] + sExz[s1][c - 1] + sExz[s1][c]);
          sxz = T(2) * gxz * e;
        }
        if (zin && jj > 0 && jj < g.ny && ii < g.nx && xx <= TX) {
          gyz = T(0.25) * (sG[s0][c - LW] + sG[s0][c] + sG[s1][c - LW] + sG[s1][c]);
          T e = T(0.5) * ((sP[s1][1][c] - sP[s0][1][c]) + (sP[s1][2][c] - sP[s1][2][c - LW])) * ih;
          if constexpr (EIG) e -= T(0.25) * (sEyz[s0][c - LW] + sEyz[s0][c] + sEyz[s1][c - LW] + sEyz[s1][c]);
          syz = T(2) * gyz * e;
        }
        sSxz[out][c] = sxz;
        sSyz[out][c] = syz;
        if constexpr (MODE == M_RESID) {
          sGxz[out][c] = gxz;
          sGyz[out][c] = gyz;
        }
      }
    }
    (void)kk; (void)s0; (void)s1; (void)out;
  };

  // ---- z march --------------------------------------------------------------
  const int k0 = (DIM == 3) ? bz * a.kz : 0;
  const int k1 = (DIM == 3) ? min(k0 + a.kz, g.nz) : 1;
  double acc0 = 0.0, acc1 = 0.0;
  T szz_prev = T(0), m_prev = T(0);

  if constexpr (DIM == 3) {
    // prologue: planes k0-1 and k0, sigma_zz of the own cell below, edges at level k0
    int sa = (k0 - 1) & 1, sb = k0 & 1;
    load_vec(k0, sb);
    load_cell(a.G, sG[sb], k0);
    load_eig_shear3(k0, sb);
    if (k0 > 0) {
      load_vec(k0 - 1, sa);
      load_cell(a.G, sG[sa], k0 - 1);
      load_cell(a.K, sK, k0 - 1);
      if constexpr (EIG) load_eig(k0 - 1);
      load_eig_shear3(k0 - 1, sa);
    }
    __syncthreads();
    if (k0 > 0) {
      int c = L(ly, lx);
      T exx = (sP[sa][0][c + 1] - sP[sa][0][c]) * ih;
      T eyy = (sP[sa][1][c + LW] - sP[sa][1][c]) * ih;
      T ezz = (sP[sb][2][c] - sP[sa][2][c]) * ih;
      if constexpr (EIG) {
        exx -= sEt[c] + sEn[0][c];
        eyy -= sEt[c] + sEn[1][c];
        ezz -= sEt[c] + sEn[2][c];
      }
      T tr = exx + eyy + ezz;
      T G2 = T(2) * sG[sa][c];
      szz_prev = sK[c] * tr - G2 * tr * T(1.0 / 3.0) + G2 * ezz;
      m_prev = sK[c] + T(2.0 / 3.0) * G2;
    }
    edge_z(k0, sa, sb, sb);
  }

  for (int k = k0; k < k1; ++k) {
    const int sk = k & 1, sk1 = (k + 1) & 1;
    __syncthreads();
    if constexpr (DIM == 3) {
      load_vec(k + 1, sk1);
      load_cell(a.G, sG[sk1], k + 1);
      load_eig_shear3(k + 1, sk1);
    } else {
      load_vec(k, sk);
      load_cell(a.G, sG[sk], k);
    }
    load_cell(a.K, sK, k);
    if constexpr (EIG) load_eig(k);
    __syncthreads();
    cell_stress(sk, sk1);
    edge_xy(sk, k);
    if constexpr (DIM == 3) edge_z(k + 1, sk, sk1, sk1);
    __syncthreads();
    if (own) {
      const int c = L(ly, lx);
      const int e = gidx(g, i, j, k);
      T q[3] = {T(0), T(0), T(0)};
      if (i > 0) {
        q[0] = sSxx[c - 1] - sSxx[c] + sSxy[c] - sSxy[c + LW];
        if constexpr (DIM == 3) q[0] += sSxz[sk][c] - sSxz[sk1][c];
      }
      if (j > 0) {
        q[1] = sSyy[c - LW] - sSyy[c] + sSxy[c] - sSxy[c + 1];
        if constexpr (DIM == 3) q[1] += sSyz[sk][c] - sSyz[sk1][c];
      }
      if constexpr (DIM == 3) {
        if (k > 0) q[2] = szz_prev - sSzz[c] + sSxz[sk][c] - sSxz[sk][c + 1] + sSyz[sk][c] - sSyz[sk][c + LW];
      }
      if constexpr (MODE == M_RESID) {
        // inverse diagonal: (M_left + M_right + adjacent interior edge G_e) / h
        T Mc = sK[c] + T(4.0 / 3.0) * sG[sk][c];
        T d[3] = {T(0), T(0), T(0)};
        auto gxy = [&](int cc2, int ii, int jj) -> T {
          if (ii > 0 && ii < g.nx && jj > 0 && jj < g.ny)
            return T(0.25) * (sG[sk][cc2 - LW - 1] + sG[sk][cc2 - LW] + sG[sk][cc2 - 1] + sG[sk][cc2]);
          return T(0);
        };
        if (i > 0) {
          d[0] = sK[c - 1] + T(4.0 / 3.0) * sG[sk][c - 1] + Mc + gxy(c, i, j) + gxy(c + LW, i, j + 1);
          if constexpr (DIM == 3) d[0] += sGxz[sk][c] + sGxz[sk1][c];
        }
        if (j > 0) {
          d[1] = sK[c - LW] + T(4.0 / 3.0) * sG[sk][c - LW] + Mc + gxy(c, i, j) + gxy(c + 1, i + 1, j);
          if constexpr (DIM == 3) d[1] += sGyz[sk][c] + sGyz[sk1][c];
        }
        if constexpr (DIM == 3) {
          if (k > 0) d[2] = m_prev + Mc + sGxz[sk][c] + sGxz[sk][c + 1] + sGyz[sk][c] + sGyz[sk][c + LW];
          m_prev = Mc;
        }
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) {
          T di = d[cc] > T(0) ? T(1) / (d[cc] * ih) : T(0);
          T r = -q[cc];
          a.dinv[cc][e] = di;
          T zz = di * r;
          a.o1[cc][e] = r;
          a.o2[cc][e] = zz;
          if (zero_u) a.u[cc][e] = T(0);
          acc0 += (double)r * (double)zz;
          acc1 += (double)r * (double)r;
        }
      } else {
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) acc0 += (double)q[cc] * (double)q[cc];
      }
      if constexpr (DIM == 3) szz_prev = sSzz[c];
    }
  }
  double s0 = block_sum(acc0, red);
  if (threadIdx.x == 0) a.part[pidx] = s0;
  if (MODE == M_RESID) {
    double s1 = block_sum(acc1, red);
    if (threadIdx.x == 0) a.part[pstride + pidx] = s1;
  }
}

template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(NT) void k_elast(ElastArgs<T> a) {
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int nblk = gridDim.x * gridDim.y * gridDim.z;
  bool zero_u = false;
  if (MODE == M_RESID) {
    __shared__ double red0[NT / 64];
    const double bb = sum_partials(a.part_in, a.n_in, red0);
    zero_u = (bb == 0.0);
    if (bid == 0 && threadIdx.x == 0) {
      a.scal[S_BB] = bb;
      a.scal[S_FIRST] = 1.0;
      a.scal[S_CONV] = 0.0;
      a.scal[S_ITERS] = 0.0;
    }
  }
  __shared__ __align__(16) char smem[sizeof(ElastSmem<T, DIM, MODE>)];
  elast_tile<T, DIM, MODE>(a, blockIdx.x, blockIdx.y, blockIdx.z, zero_u, bid, nblk, smem);
}



// ---------------------------------------------------------------------------
// 3D q = A p with the direction update p = z + beta p fused in.
//
// Block = 64 x BY threads over a 64 x BY column tile, marching along z.  Each
// thread keeps its own column's displacement, moduli and stresses in
// registers (so the z neighbours never touch LDS); the x / y neighbours come
// from an LDS plane tile with a one-cell ring.  The stresses the tile needs on
// the ring (cell stresses below / left of it, edge stresses above / right of
// it) are a separate short work list.  Global loads run two planes ahead:
// two register sets hold raw values in flight (plane k+3 and k+4 while plane
// k is computed), combined only when stored.  A block reads exactly the
// planes k0-1 .. k1 its slab needs.
// ---------------------------------------------------------------------------
template <int BY>
struct ApplyTile {
  static constexpr int NTB = TX * BY;
  static constexpr int W = TX + 2, H = BY + 2, S = W * H;
  static constexpr int NRING = 2 * W + 2 * BY;       // ring positions of the plane tile
  static constexpr int NHALO = 3 * (TX + BY);        // ring stress items per plane
};

// Modes (compile time, so that the CG instance carries no other code):
// APPLY_CG inside the CG recurrence; APPLY_PLAIN q = A z outside it (the
// previous direction not read, the new one not written; with ElastArgs::jr
// set, ||jr - q||^2 partials); APPLY_RESID the residual pass r = b - A z
// (ElastArgs::resid); APPLY_SMOOTH one damped Jacobi sweep of a multigrid
// level, o1 = z + omega D^-1 (b - A z), or with omega = 0 its residual
// o1 = b - A z (b in jr), with the partials of b . o1; APPLY_SMOOTH0 the
// first two sweeps from zero in one pass: z = omega0 D^-1 b formed from b
// and D^-1 as the tile is loaded (z not read), then o1 as in APPLY_SMOOTH.
enum ApplyMode { APPLY_CG = 0, APPLY_PLAIN = 1, APPLY_RESID = 2, APPLY_SMOOTH = 3, APPLY_SMOOTH0 = 4 };

template <typename T, int BY, int AM>
__global__ __launch_bounds__(ApplyTile<BY>::NTB, sizeof(T) == 4 && AM != APPLY_RESID && AM != APPLY_SMOOTH ? 4 : 1) void k_apply3(ElastArgs<T> a) {
  constexpr bool kPlain = AM != APPLY_CG, kResid = AM == APPLY_RESID, kCG = AM == APPLY_CG;
  constexpr bool kSmooth0 = AM == APPLY_SMOOTH0;
  constexpr bool kSmooth = AM == APPLY_SMOOTH || kSmooth0, kRB = kResid || kSmooth;   // kRB: reads b and D^-1
  constexpr bool kLo = kSmooth && sizeof(T) == 4;   // K, G and D^-1 from their bf16 copies
  using TL = ApplyTile<BY>;
  constexpr int W = TL::W, S = TL::S, NTB = TL::NTB;
  __shared__ T sP[2][3][S];
  __shared__ T sG[2][S];
  __shared__ T sK[2][S];
  __shared__ T sSxx[S], sSyy[S], sSxy[S];
  __shared__ T sSxz[2][S], sSyz[2][S];
  __shared__ double red[NTB / 64];

  const Grid& g = a.g;
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  // Consecutive hardware block ids go to different XCDs (round robin over 8);
  // give each XCD a contiguous run of tiles so that tile halos are re-read
  // from that XCD's own L2.
  const int tile = xcd_tile(bid, gridDim.x * gridDim.y * gridDim.z);
  const int bx = tile % gridDim.x, by = (tile / gridDim.x) % gridDim.y, bz = tile / (gridDim.x * gridDim.y);
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int i0 = bx * TX, j0 = by * BY;
  const int i = i0 + tx, j = j0 + ty;
  const int c = (ty + 1) * W + tx + 1;              // own position in the plane tile
  const bool own = (i < g.nx) && (j < g.ny);
  const T ih = a.p.ih;
  const int pl = g.px * g.ny;

  const int k0 = bz * a.kz;
  const int k1 = min(k0 + a.kz, g.nz);
  const int own_e = own ? j * g.px + i : 0;

  if constexpr (kSmooth)             // a multigrid sweep queued past the solve's convergence
    if (a.scal[S_CONV] != 0.0) return;
  // CG scalars (identical in every block)
  double beta = 0.0;
  bool first = true;                 // plain: p_new = z
  if constexpr (kCG) {
    const double cv = a.scal[S_CONV];
    const double mine = (double)(a.it + 1);
    if (cv != 0.0 && cv != mine) return;
    double rzv = 0.0, rrv = 0.0;
    {
      double v0 = 0.0, v1 = 0.0;
      for (int q = threadIdx.x; q < a.n_in; q += NTB) { v0 += a.part_in[q]; v1 += a.part_in[a.n_in + q]; }
      v0 = wave_sum(v0);
      v1 = wave_sum(v1);
      __shared__ double sh2[2][NTB / 64];
      if ((threadIdx.x & 63) == 0) { sh2[0][threadIdx.x >> 6] = v0; sh2[1][threadIdx.x >> 6] = v1; }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < NTB / 64; ++w) { rzv += sh2[0][w]; rrv += sh2[1][w]; }
    }
    first = a.scal[S_FIRST] != 0.0;
    // converged by the last update (found here, or by the check after a
    // chunk of launches, which marks this launch): stop, after adding the
    // last update's alpha p to x if that update left it pending (the updates
    // add the steps of two iterations at a time, after odd iterations)
    if (cv == mine || rrv <= a.tol2 * a.scal[S_BB]) {
      if (bid == 0 && threadIdx.x == 0) a.scal[S_CONV] = mine;
      if ((a.it & 1) && own) {
        const T al = (T)a.scal[S_ALPHA];
        for (int kk = k0; kk < k1; ++kk) {
          const int e = own_e + kk * pl;
#pragma unroll
          for (int d = 0; d < 3; ++d) a.xs[d][e] += al * a.u[d][e];
        }
      }
      return;
    }
    beta = first ? 0.0 : rzv / a.scal[S_RZ + (a.parity ^ 1)];
    if (bid == 0 && threadIdx.x == 0) {
      a.scal[S_RZ + a.parity] = rzv;
      a.scal[S_RR] = rrv;
    }
  }
  const T tb = (T)beta;
  bool zero_u = false;
  if constexpr (kResid) {            // residual of the set-up: ||b||^2 from the set-up partials
    double v = 0.0;
    for (int q = threadIdx.x; q < a.n_in; q += NTB) v += a.part_in[q];
    v = wave_sum(v);
    __shared__ double shb[NTB / 64];
    if ((threadIdx.x & 63) == 0) shb[threadIdx.x >> 6] = v;
    __syncthreads();
    double bb = 0.0;
#pragma unroll
    for (int w = 0; w < NTB / 64; ++w) bb += shb[w];
    zero_u = bb == 0.0;
    if (bid == 0 && threadIdx.x == 0) {
      a.scal[S_BB] = bb;
      a.scal[S_FIRST] = 1.0;
      a.scal[S_CONV] = 0.0;
      a.scal[S_ITERS] = 0.0;
    }
  }

  // ring position handled by this thread (threads >= NRING have none)
  int rg_t = S, rg_e = 0;
  bool rg_in = false;
  if (threadIdx.x < TL::NRING) {
    int t = threadIdx.x, yy, xx;
    if (t < W) { yy = 0; xx = t; }
    else if (t < 2 * W) { yy = BY + 1; xx = t - W; }
    else { t -= 2 * W; yy = 1 + (t >> 1); xx = (t & 1) ? TX + 1 : 0; }
    const int ii = i0 + xx - 1, jj = j0 + yy - 1;
    rg_t = yy * W + xx;
    rg_in = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny;
    rg_e = rg_in ? jj * g.px + ii : 0;
  }

  // raw (in-flight) loads of one plane: own column and ring position
  struct Raw {
    T oz[3], op[3], og, ok, hz[3], hp[3], hg, hk;
    bool oin, hin;
  };
  Raw ra, rb;
  // loads of cells outside the grid, and of planes the slab does not need
  // (want == false), are range-checked to zero and fetch nothing
  const int nbytes = g.n * (int)sizeof(T);
  __amdgpu_buffer_rsrc_t rz_[3], ru_[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    rz_[d] = buf_rsrc(a.z[d], nbytes);
    ru_[d] = buf_rsrc(a.u[d], nbytes);
  }
  // K, G and D^-1 of a sweep in FP32 are bf16 (half the byte offset of an FP32
  // element; the out-of-range offset halved is still past the array)
  const int nb_lo = g.n * 2;
  auto ld_lo = [&](__amdgpu_buffer_rsrc_t r, int off) __attribute__((always_inline)) -> T {
    if constexpr (kLo) return (T)buf_ld_bf16(r, off >> 1);
    else return buf_ld<T>(r, off);
  };
  const __amdgpu_buffer_rsrc_t rG = kLo ? buf_rsrc(a.lo_G, nb_lo) : buf_rsrc(a.G, nbytes);
  const __amdgpu_buffer_rsrc_t rK = kLo ? buf_rsrc(a.lo_K, nb_lo) : buf_rsrc(a.K, nbytes);
  if constexpr (kPlain)        // p = z: the previous direction is never read
#pragma unroll
    for (int d = 0; d < 3; ++d) ru_[d] = buf_rsrc(a.u[d], 0);
  if constexpr (kSmooth0)      // z = omega D^-1 b: b in the z slots, D^-1 in the direction slots
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      rz_[d] = buf_rsrc(a.jr[d], nbytes);
      ru_[d] = kLo ? buf_rsrc(a.lo_d[d], nb_lo) : buf_rsrc(a.dinv[d], nbytes);
    }
  const T om0 = (T)a.omega0;
  __amdgpu_buffer_rsrc_t rjb_[3], rjd_[3];
  if constexpr (kRB)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      rjb_[d] = buf_rsrc(a.jr[d], nbytes);
      rjd_[d] = kLo ? buf_rsrc(a.lo_d[d], nb_lo) : buf_rsrc(a.dinv[d], nbytes);
    }
  // only the first waves hold ring positions (threads < NRING); the others
  // run a copy of the plane loop without ring loads and stores (RW = false),
  // so that in both copies every load's wait count is exact
  const bool ring_wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) < (TL::NRING + 63) / 64;
  auto fetch = [&](Raw& R, int kk, bool want, auto RW) __attribute__((always_inline)) {
    const bool zin = want && kk >= 0 && kk < g.nz;
    R.oin = own && zin;
    R.hin = rg_in && zin;
    const int eo = R.oin ? (own_e + kk * pl) * (int)sizeof(T) : kOutOfRange;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      R.oz[d] = buf_ld<T>(rz_[d], eo);
      if constexpr (kSmooth0) R.op[d] = ld_lo(ru_[d], eo);
      else R.op[d] = buf_ld<T>(ru_[d], eo);
    }
    R.og = ld_lo(rG, eo); R.ok = ld_lo(rK, eo);
    if constexpr (decltype(RW)::value) {
      const int eh = R.hin ? (rg_e + kk * pl) * (int)sizeof(T) : kOutOfRange;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        R.hz[d] = buf_ld<T>(rz_[d], eh);
        if constexpr (kSmooth0) R.hp[d] = ld_lo(ru_[d], eh);
        else R.hp[d] = buf_ld<T>(ru_[d], eh);
      }
      R.hg = ld_lo(rG, eh); R.hk = ld_lo(rK, eh);
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) R.hz[d] = R.hp[d] = T(0);
      R.hg = R.hk = T(0);
    }
  };
  // combine, store the plane into LDS slot `slot`, and return the own values
  // the vector applied from the raw loads: z, the new direction z + beta p,
  // or (APPLY_SMOOTH0) omega D^-1 b
  auto comb = [&](T z, T p) -> T {
    if constexpr (kSmooth0) return om0 * p * z;
    else return first ? z : z + tb * p;
  };
  // own column's values of one plane (APPLY_SMOOTH0 also keeps b and D^-1,
  // which its epilogue needs again)
  struct Own { T p[3], g, k, b[3], d[3]; };
  auto stash = [&](const Raw& R, int slot, Own& O, auto RW) __attribute__((always_inline)) {
    T (&vp)[3] = O.p;
    T& vg = O.g;
    T& vk = O.k;
    if constexpr (kSmooth0)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        O.b[d] = R.oin ? R.oz[d] : T(0);
        O.d[d] = R.oin ? R.op[d] : T(0);
      }
#pragma unroll
    for (int d = 0; d < 3; ++d) vp[d] = R.oin ? comb(R.oz[d], R.op[d]) : T(0);
    vg = R.oin ? R.og : T(0);
    vk = R.oin ? R.ok : T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) sP[slot][d][c] = vp[d];
    sG[slot][c] = vg;
    sK[slot][c] = vk;
    if (decltype(RW)::value && rg_t < S) {
#pragma unroll
      for (int d = 0; d < 3; ++d) sP[slot][d][rg_t] = R.hin ? comb(R.hz[d], R.hp[d]) : T(0);
      sG[slot][rg_t] = R.hin ? R.hg : T(0);
      sK[slot][rg_t] = R.hin ? R.hk : T(0);
    }
  };
  // stresses from LDS at tile position q (all neighbours from LDS)
  auto cell_lds = [&](int q, int sk, int sk1, T& sxx, T& syy) {
    const T exx = (sP[sk][0][q + 1] - sP[sk][0][q]) * ih;
    const T eyy = (sP[sk][1][q + W] - sP[sk][1][q]) * ih;
    const T ezz = (sP[sk1][2][q] - sP[sk][2][q]) * ih;
    const T tr = exx + eyy + ezz;
    const T G2 = T(2) * sG[sk][q];
    const T lam = sK[sk][q] * tr - G2 * tr * T(1.0 / 3.0);
    sxx = lam + G2 * exx;
    syy = lam + G2 * eyy;
  };
  auto xy_lds = [&](int q, int ii, int jj, int sk) -> T {
    if (!(ii > 0 && ii < g.nx && jj > 0 && jj < g.ny)) return T(0);
    const T ge = T(0.25) * (sG[sk][q - W - 1] + sG[sk][q - W] + sG[sk][q - 1] + sG[sk][q]);
    return ge * ((sP[sk][0][q] - sP[sk][0][q - W]) + (sP[sk][1][q] - sP[sk][1][q - 1])) * ih;
  };
  auto xz_lds = [&](int q, int ii, int jj, int kk, int s0, int s1) -> T {
    if (!(kk > 0 && kk < g.nz && ii > 0 && ii < g.nx && jj < g.ny)) return T(0);
    const T ge = T(0.25) * (sG[s0][q - 1] + sG[s0][q] + sG[s1][q - 1] + sG[s1][q]);
    return ge * ((sP[s1][0][q] - sP[s0][0][q]) + (sP[s1][2][q] - sP[s1][2][q - 1])) * ih;
  };
  auto yz_lds = [&](int q, int ii, int jj, int kk, int s0, int s1) -> T {
    if (!(kk > 0 && kk < g.nz && jj > 0 && jj < g.ny && ii < g.nx)) return T(0);
    const T ge = T(0.25) * (sG[s0][q - W] + sG[s0][q] + sG[s1][q - W] + sG[s1][q]);
    return ge * ((sP[s1][1][q] - sP[s0][1][q]) + (sP[s1][2][q] - sP[s1][2][q - W])) * ih;
  };
  // ring stress items: cells left / below the tile, xy edges above / right,
  // z edges right (xz) / above (yz) at level kk
  // With at least 3 x 128 threads each group starts on a wave boundary
  // (group g on threads 128 g ..), so no wave runs two groups' code.
  constexpr bool kAligned = NTB >= 3 * 128 && TX + BY <= 128;
  auto ring_items = [&](int sk, int sk1, int kk_edge, int s0, int s1, int zout, bool cells_and_xy) __attribute__((always_inline)) {
    for (int w = threadIdx.x; kAligned ? (w < 3 * 128) : (w < TL::NHALO); w += NTB) {
      const int grp = kAligned ? (w >> 7) : w / (TX + BY);
      const int r = kAligned ? (w & 127) : w - grp * (TX + BY);
      if (kAligned && r >= TX + BY) continue;
      if (grp == 0) {
        if (!cells_and_xy) continue;
        const int yy = r < TX ? 0 : 1 + (r - TX), xx = r < TX ? 1 + r : 0;
        const int q = yy * W + xx;
        T sxx, syy;
        cell_lds(q, sk, sk1, sxx, syy);
        sSxx[q] = sxx;
        sSyy[q] = syy;
      } else if (grp == 1) {
        if (!cells_and_xy) continue;
        const int yy = r < TX ? BY + 1 : 1 + (r - TX), xx = r < TX ? 1 + r : TX + 1;
        const int q = yy * W + xx;
        sSxy[q] = xy_lds(q, i0 + xx - 1, j0 + yy - 1, sk);
      } else {
        if (r < TX) {    // yz edge above the tile
          const int q = (BY + 1) * W + 1 + r;
          sSyz[zout][q] = yz_lds(q, i0 + r, j0 + BY, kk_edge, s0, s1);
        } else {         // xz edge right of the tile
          const int yy = 1 + (r - TX);
          const int q = yy * W + TX + 1;
          sSxz[zout][q] = xz_lds(q, i0 + TX, j0 + yy - 1, kk_edge, s0, s1);
        }
      }
    }
  };

  // LDS slots are numbered relative to k0 (plane m in slot (m - k0) & 1), so
  // inside the plane pairs below every slot index is a constant.  The
  // lambdas are forced inline: a call left out of line keeps the register
  // sets it takes by reference in scratch memory.
  Own oA, oB;                         // planes k (current) and k+1, roles alternating
  T szz_prev = T(0), sxz_c = T(0), syz_c = T(0);
  // boundary factors (0 / 1) of the own column: edges on the domain boundary
  // carry no shear stress, the low boundary faces no force; all the LDS
  // values they multiply are finite (zeros outside the domain)
  // (interior in x, interior in y; for the own column, whose q is stored,
  // these are also the low boundary faces)
  const T f_xz = (i > 0 && i < g.nx) ? T(1) : T(0);
  const T f_yz = (j > 0 && j < g.ny) ? T(1) : T(0);

  double acc = 0.0, acc1 = 0.0;
  // prologue: planes k0-1 (slot 1), k0 (slot 0); sigma_zz of the own cell
  // below; z edges at level k0.  Plane m travels in register set ra when
  // m - k0 is odd.
  auto prologue = [&](auto RW) __attribute__((always_inline)) {
    Own ob;
    fetch(ra, k0 - 1, true, RW);
    fetch(rb, k0, true, RW);
    stash(ra, 1, ob, RW);
    stash(rb, 0, oA, RW);
    fetch(ra, k0 + 1, true, RW);
    fetch(rb, k0 + 2, k0 + 1 < k1, RW);
    __syncthreads();
    if (k0 > 0) {
      const T exx = (sP[1][0][c + 1] - ob.p[0]) * ih;
      const T eyy = (sP[1][1][c + W] - ob.p[1]) * ih;
      const T ezz = (oA.p[2] - ob.p[2]) * ih;
      const T tr = exx + eyy + ezz;
      const T G2 = T(2) * ob.g;
      szz_prev = ob.k * tr - G2 * tr * T(1.0 / 3.0) + G2 * ezz;
    }
    sxz_c = xz_lds(c, i, j, k0, 1, 0);
    syz_c = yz_lds(c, i, j, k0, 1, 0);
    sSxz[0][c] = sxz_c;
    sSyz[0][c] = syz_c;
    ring_items(1, 0, k0, 1, 0, 0, false);
    __syncthreads();
    stash(ra, 1, oB, RW);
    fetch(ra, k0 + 3, k0 + 2 < k1, RW);
    __syncthreads();
  };

  // one plane k in slot sk (plane k+1 in slot sk1); C holds its own values,
  // N those of plane k+1.  R carries plane k+2 in (stashed into slot sk and
  // into C, which then holds the plane after N) and is refilled with plane k+4.
  auto plane = [&](int k, Raw& R, const int sk, Own& C, const Own& N, auto RW) __attribute__((always_inline)) {
    const int sk1 = sk ^ 1;
    // residual pass: b and D^-1 of the own cell, issued before the stencil so
    // that their latency hides behind it
    T jb[3], jd[3];
    if constexpr (kSmooth0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        jb[d] = C.b[d];
        jd[d] = C.d[d];
      }
    } else if constexpr (kRB) {
      const int eo = own ? (own_e + k * pl) * (int)sizeof(T) : kOutOfRange;
      // the residual sweep (omega = 0) does not use D^-1: its loads are
      // range-checked to zero and fetch nothing
      const int eod = (kSmooth && a.omega == 0.0) ? kOutOfRange : eo;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        jb[d] = buf_ld<T>(rjb_[d], eo);
        jd[d] = ld_lo(rjd_[d], eod);
      }
    }
    // (A) own stresses of plane k and own z edges at level k+1
    const T exx = (sP[sk][0][c + 1] - C.p[0]) * ih;
    const T eyy = (sP[sk][1][c + W] - C.p[1]) * ih;
    const T ezz = (N.p[2] - C.p[2]) * ih;
    const T tr = exx + eyy + ezz;
    const T G2 = T(2) * C.g;
    const T lam = C.k * tr - G2 * tr * T(1.0 / 3.0);
    const T sxx = lam + G2 * exx, syy = lam + G2 * eyy, szz = lam + G2 * ezz;
    const T gxy = T(0.25) * (sG[sk][c - W - 1] + sG[sk][c - W] + sG[sk][c - 1] + C.g);
    const T sxy = f_xz * f_yz * gxy * ((C.p[0] - sP[sk][0][c - W]) + (C.p[1] - sP[sk][1][c - 1])) * ih;
    const int kn1 = k + 1;
    T sxz_n = T(0), syz_n = T(0);
    if (kn1 < g.nz) {                 // block-uniform
      const T gxz = T(0.25) * (sG[sk][c - 1] + C.g + sG[sk1][c - 1] + N.g);
      sxz_n = f_xz * gxz * ((N.p[0] - C.p[0]) + (N.p[2] - sP[sk1][2][c - 1])) * ih;
      const T gyz = T(0.25) * (sG[sk][c - W] + C.g + sG[sk1][c - W] + N.g);
      syz_n = f_yz * gyz * ((N.p[1] - C.p[1]) + (N.p[2] - sP[sk1][2][c - W])) * ih;
    }
    sSxx[c] = sxx;
    sSyy[c] = syy;
    sSxy[c] = sxy;
    sSxz[sk1][c] = sxz_n;
    sSyz[sk1][c] = syz_n;
    ring_items(sk, sk1, kn1, sk, sk1, sk1, true);
    __syncthreads();
    // (C) divergence onto the own faces of plane k
    if (own) {
      const int e = own_e + k * pl;
      const T q0 = f_xz * (sSxx[c - 1] - sxx + sxy - sSxy[c + W] + sxz_c - sxz_n);
      const T q1 = f_yz * (sSyy[c - W] - syy + sxy - sSxy[c + 1] + syz_c - syz_n);
      const T q2 = k > 0 ? szz_prev - szz + sxz_c - sSxz[sk][c + 1] + syz_c - sSyz[sk][c + W] : T(0);
      if constexpr (kResid) {
        const T qv[3] = {q0, q1, q2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const T r = zero_u ? T(0) : jb[d] - qv[d];
          const T z = jd[d] * r;
          a.o1[d][e] = r;
          a.o2[d][e] = z;
          if (zero_u) a.u[d][e] = T(0);
          acc += (double)r * (double)z;
          acc1 += (double)r * (double)r;
        }
      } else if constexpr (kSmooth) {
        const T qv[3] = {q0, q1, q2};
        const T om = (T)a.omega;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const T r = jb[d] - qv[d];
          const T o = a.omega != 0.0 ? C.p[d] + om * jd[d] * r : r;
          a.o1[d][e] = o;
          acc += (double)jb[d] * (double)o;
        }
      } else {
      if constexpr (!kPlain) { a.o1[0][e] = C.p[0]; a.o1[1][e] = C.p[1]; a.o1[2][e] = C.p[2]; }
      a.o2[0][e] = q0; a.o2[1][e] = q1; a.o2[2][e] = q2;
      if (kPlain && a.jr[0]) {
        const double d0 = (double)a.jr[0][e] - (double)q0, d1 = (double)a.jr[1][e] - (double)q1,
                     d2 = (double)a.jr[2][e] - (double)q2;
        acc += d0 * d0 + d1 * d1 + d2 * d2;
      } else {
        acc += (double)C.p[0] * (double)q0 + (double)C.p[1] * (double)q1 + (double)C.p[2] * (double)q2;
      }
      }
    }
    szz_prev = szz;
    sxz_c = sxz_n;
    syz_c = syz_n;
    if (k + 1 < k1) stash(R, sk, C, RW);   // plane k+2 into the slot of plane k
    fetch(R, k + 4, k + 3 < k1, RW);
    __syncthreads();
  };
  // pairs of planes, so that every path into a plane has the same loads in
  // flight (the wait counts then let the newer set stay outstanding)
  auto march = [&](auto RW) __attribute__((always_inline)) {
    prologue(RW);
    int k = k0;
    for (; k + 1 < k1; k += 2) {
      plane(k, rb, 0, oA, oB, RW);
      plane(k + 1, ra, 1, oB, oA, RW);
    }
    if (k < k1) plane(k, rb, 0, oA, oB, RW);
  };
  if (ring_wave) march(std::true_type{}); else march(std::false_type{});
  const double s0 = block_sum_n<NTB>(acc, red);
  if (threadIdx.x == 0) a.part[bid] = s0;
  if constexpr (kResid) {
    const double s1 = block_sum_n<NTB>(acc1, red);
    if (threadIdx.x == 0) a.part[gridDim.x * gridDim.y * gridDim.z + bid] = s1;
  }
}

// ---------------------------------------------------------------------------
// 3D solve set-up: b = div(C : eps*) of the eigenstrain and plastic strain
// (the right-hand side; u = 0), the Jacobi inverse diagonal D^-1 and the
// block partials of ||b||^2, in the 2.5D layout of k_apply3: block = 64 x BY
// threads over a column tile marching along z, own column values in
// registers, x / y neighbours from a one-cell-ring LDS plane tile, ring
// stresses from a short work list, loads two planes ahead.  Per plane it
// reads phi_f, phi_w and the six plastic strain components, evaluates the
// moduli (Eq. 32) and the eigenstrain from the phases, and writes b, D^-1 and
// the moduli of the cells it owns (the apply kernels read them).
// ---------------------------------------------------------------------------
template <typename T, int BY>
__global__ __launch_bounds__(ApplyTile<BY>::NTB) void k_setup3(ElastArgs<T> a) {
  using TL = ApplyTile<BY>;
  constexpr int W = TL::W, S = TL::S, NTB = TL::NTB;
  __shared__ T sK[2][S], sG[2][S], sN[2][3][S], sExy[2][S], sExz[2][S], sEyz[2][S];
  __shared__ T sSxx[S], sSyy[S], sSxy[S], sGxy[S];
  __shared__ T sSxz[2][S], sSyz[2][S], sGxz[2][S], sGyz[2][S];
  __shared__ double red[NTB / 64];

  const Grid& g = a.g;
  const KP<T>& p = a.p;
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int tile = xcd_tile(bid, gridDim.x * gridDim.y * gridDim.z);
  const int bx = tile % gridDim.x, by = (tile / gridDim.x) % gridDim.y, bz = tile / (gridDim.x * gridDim.y);
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int i0 = bx * TX, j0 = by * BY;
  const int i = i0 + tx, j = j0 + ty;
  const int c = (ty + 1) * W + tx + 1;
  const bool own = (i < g.nx) && (j < g.ny);
  const T ih = p.ih;
  const int pl = g.px * g.ny;

  int rg_t = S, rg_e = 0;
  bool rg_in = false;
  if (threadIdx.x < TL::NRING) {
    int t = threadIdx.x, yy, xx;
    if (t < W) { yy = 0; xx = t; }
    else if (t < 2 * W) { yy = BY + 1; xx = t - W; }
    else { t -= 2 * W; yy = 1 + (t >> 1); xx = (t & 1) ? TX + 1 : 0; }
    const int ii = i0 + xx - 1, jj = j0 + yy - 1;
    rg_t = yy * W + xx;
    rg_in = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny;
    rg_e = rg_in ? jj * g.px + ii : 0;
  }
  const int own_e = own ? j * g.px + i : 0;
  const int k0 = bz * a.kz;
  const int k1 = min(k0 + a.kz, g.nz);

  // raw loads of one plane (own column and ring position), two sets in flight
  struct Raw {
    T ow, of, op[6], hw, hf, hp[6];
    bool oin, hin;
  };
  struct Own { T K, G, n[3], xy, xz, yz; };    // own cell: moduli, eps*_nn (eigen + plastic), plastic shears
  Raw ra, rb;
  const int nbytes = g.n * (int)sizeof(T);
  const __amdgpu_buffer_rsrc_t rW = buf_rsrc(a.phi_w, nbytes), rF = buf_rsrc(a.phi_f, nbytes);
  const __amdgpu_buffer_rsrc_t rE = buf_rsrc(a.epsp, 6 * g.ns * (int)sizeof(T));
  const int cstride = g.ns * (int)sizeof(T);
  auto fetch = [&](Raw& R, int kk, bool want) {
    const bool zin = want && kk >= 0 && kk < g.nz;
    R.oin = own && zin;
    R.hin = rg_in && zin;
    const int eo = R.oin ? (own_e + kk * pl) * (int)sizeof(T) : kOutOfRange;
    const int eh = R.hin ? (rg_e + kk * pl) * (int)sizeof(T) : kOutOfRange;
    R.ow = buf_ld<T>(rW, eo); R.of = buf_ld<T>(rF, eo);
    R.hw = buf_ld<T>(rW, eh); R.hf = buf_ld<T>(rF, eh);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      R.op[q] = buf_ld<T>(rE, R.oin ? eo + q * cstride : kOutOfRange);
      R.hp[q] = buf_ld<T>(rE, R.hin ? eh + q * cstride : kOutOfRange);
    }
  };
  // combine plane kk into LDS slot `slot`: the moduli from the phases (written
  // out for the planes the block owns), the eigenstrain, the plastic strain
  auto stash = [&](const Raw& R, int kk, int slot, Own& O) {
    const T et = R.oin ? eigen_strain(p, R.of) : T(0);
    T mK, mG;
    moduli(p, R.of, R.ow, mK, mG);
    O.K = R.oin ? mK : T(0);
    O.G = R.oin ? mG : T(0);
    if (R.oin && kk >= k0 && kk < k1) {
      const int e = own_e + kk * pl;
      a.Kw[e] = mK;
      a.Gw[e] = mG;
      if (a.lo_w[0]) {
        a.lo_w[0][e] = bf16_rne((float)mK);
        a.lo_w[1][e] = bf16_rne((float)mG);
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) O.n[q] = R.oin ? et + R.op[q] : T(0);
    O.xy = R.oin ? R.op[3] : T(0);
    O.xz = R.oin ? R.op[4] : T(0);
    O.yz = R.oin ? R.op[5] : T(0);
    sK[slot][c] = O.K;
    sG[slot][c] = O.G;
#pragma unroll
    for (int q = 0; q < 3; ++q) sN[slot][q][c] = O.n[q];
    sExy[slot][c] = O.xy;
    sExz[slot][c] = O.xz;
    sEyz[slot][c] = O.yz;
    if (rg_t < S) {
      const T hu = R.hin ? eigen_strain(p, R.hf) : T(0);
      T hK, hG;
      moduli(p, R.hf, R.hw, hK, hG);
      sK[slot][rg_t] = R.hin ? hK : T(0);
      sG[slot][rg_t] = R.hin ? hG : T(0);
#pragma unroll
      for (int q = 0; q < 3; ++q) sN[slot][q][rg_t] = R.hin ? hu + R.hp[q] : T(0);
      sExy[slot][rg_t] = R.hin ? R.hp[3] : T(0);
      sExz[slot][rg_t] = R.hin ? R.hp[4] : T(0);
      sEyz[slot][rg_t] = R.hin ? R.hp[5] : T(0);
    }
  };
  // normal stresses of the cell at tile position q (slot sk), u = 0
  auto cell_sn = [&](int q, int sk, T& sxx, T& syy) {
    const T n0 = sN[sk][0][q], n1 = sN[sk][1][q], n2 = sN[sk][2][q];
    const T tr = -(n0 + n1 + n2);
    const T G2 = T(2) * sG[sk][q];
    const T lam = sK[sk][q] * tr - G2 * tr * T(1.0 / 3.0);
    sxx = lam - G2 * n0;
    syy = lam - G2 * n1;
  };
  // xz / yz edge stresses and moduli at level kk (planes in slots s0 below, s1 above)
  auto xz_edge = [&](int q, int ii, int jj, int kk, int s0, int s1, T& gv) -> T {
    gv = T(0);
    if (!(kk > 0 && kk < g.nz && ii > 0 && ii < g.nx && jj < g.ny)) return T(0);
    gv = T(0.25) * (sG[s0][q - 1] + sG[s0][q] + sG[s1][q - 1] + sG[s1][q]);
    return T(-0.5) * gv * (sExz[s0][q - 1] + sExz[s0][q] + sExz[s1][q - 1] + sExz[s1][q]);
  };
  auto yz_edge = [&](int q, int ii, int jj, int kk, int s0, int s1, T& gv) -> T {
    gv = T(0);
    if (!(kk > 0 && kk < g.nz && jj > 0 && jj < g.ny && ii < g.nx)) return T(0);
    gv = T(0.25) * (sG[s0][q - W] + sG[s0][q] + sG[s1][q - W] + sG[s1][q]);
    return T(-0.5) * gv * (sEyz[s0][q - W] + sEyz[s0][q] + sEyz[s1][q - W] + sEyz[s1][q]);
  };
  // ring work: cells left / below the tile (normal stresses), xy nodes above /
  // right, z edges at level kk above (yz) and right (xz); group g on threads
  // 128 g .. so that no wave runs two groups' code
  constexpr bool kAligned = NTB >= 3 * 128 && TX + BY <= 128;
  auto ring_items = [&](int sk, int kk_edge, int s0, int s1, int zout, bool cells_and_xy) {
    for (int w = threadIdx.x; kAligned ? (w < 3 * 128) : (w < TL::NHALO); w += NTB) {
      const int grp = kAligned ? (w >> 7) : w / (TX + BY);
      const int r = kAligned ? (w & 127) : w - grp * (TX + BY);
      if (kAligned && r >= TX + BY) continue;
      if (grp == 0) {
        if (!cells_and_xy) continue;
        const int yy = r < TX ? 0 : 1 + (r - TX), xx = r < TX ? 1 + r : 0;
        const int q = yy * W + xx;
        T sxx, syy;
        cell_sn(q, sk, sxx, syy);
        sSxx[q] = sxx;
        sSyy[q] = syy;
      } else if (grp == 1) {
        if (!cells_and_xy) continue;
        const int yy = r < TX ? BY + 1 : 1 + (r - TX), xx = r < TX ? 1 + r : TX + 1;
        const int q = yy * W + xx;
        const int ii = i0 + xx - 1, jj = j0 + yy - 1;
        T sxy = T(0), gv = T(0);
        if (ii > 0 && ii < g.nx && jj > 0 && jj < g.ny) {
          gv = T(0.25) * (sG[sk][q - W - 1] + sG[sk][q - W] + sG[sk][q - 1] + sG[sk][q]);
          sxy = T(-0.5) * gv * (sExy[sk][q - W - 1] + sExy[sk][q - W] + sExy[sk][q - 1] + sExy[sk][q]);
        }
        sSxy[q] = sxy;
        sGxy[q] = gv;
      } else {
        T gv;
        if (r < TX) {    // yz edge above the tile
          const int q = (BY + 1) * W + 1 + r;
          sSyz[zout][q] = yz_edge(q, i0 + r, j0 + BY, kk_edge, s0, s1, gv);
          sGyz[zout][q] = gv;
        } else {         // xz edge right of the tile
          const int yy = 1 + (r - TX);
          const int q = yy * W + TX + 1;
          sSxz[zout][q] = xz_edge(q, i0 + TX, j0 + yy - 1, kk_edge, s0, s1, gv);
          sGxz[zout][q] = gv;
        }
      }
    }
  };

  Own oA, oB;                         // own values of planes k and k+1, roles alternating
  T szz_prev = T(0), m_prev = T(0);
  T sxz_c = T(0), syz_c = T(0), gxz_c = T(0), gyz_c = T(0);   // own z edges at level k
  const T f_xy = (i > 0 && i < g.nx && j > 0 && j < g.ny) ? T(1) : T(0);
  const T f_xz = (i > 0 && i < g.nx && j < g.ny) ? T(1) : T(0);
  const T f_yz = (j > 0 && j < g.ny && i < g.nx) ? T(1) : T(0);
  const T f_i = i > 0 ? T(1) : T(0), f_j = j > 0 ? T(1) : T(0);

  // prologue: planes k0-1 (slot 1) and k0 (slot 0); the own cell below; z edges at level k0
  {
    Own ob;
    fetch(ra, k0 - 1, true);
    fetch(rb, k0, true);
    stash(ra, k0 - 1, 1, ob);
    stash(rb, k0, 0, oA);
    fetch(ra, k0 + 1, true);
    fetch(rb, k0 + 2, k0 + 1 < k1);
    __syncthreads();
    if (k0 > 0) {
      const T tr = -(ob.n[0] + ob.n[1] + ob.n[2]);
      const T G2 = T(2) * ob.G;
      szz_prev = ob.K * tr - G2 * tr * T(1.0 / 3.0) - G2 * ob.n[2];
      m_prev = ob.K + T(4.0 / 3.0) * ob.G;
    }
    sxz_c = xz_edge(c, i, j, k0, 1, 0, gxz_c);
    syz_c = yz_edge(c, i, j, k0, 1, 0, gyz_c);
    sSxz[0][c] = sxz_c;
    sSyz[0][c] = syz_c;
    sGxz[0][c] = gxz_c;
    sGyz[0][c] = gyz_c;
    ring_items(1, k0, 1, 0, 0, false);
    __syncthreads();
    stash(ra, k0 + 1, 1, oB);
    fetch(ra, k0 + 3, k0 + 2 < k1);
    __syncthreads();
  }

  double acc = 0.0;
  auto plane = [&](int k, Raw& R, const int sk, Own& C, const Own& N) {
    const int sk1 = sk ^ 1;
    // own cell normal stresses and diagonal term
    const T tr = -(C.n[0] + C.n[1] + C.n[2]);
    const T G2 = T(2) * C.G;
    const T lam = C.K * tr - G2 * tr * T(1.0 / 3.0);
    const T sxx = lam - G2 * C.n[0], syy = lam - G2 * C.n[1], szz = lam - G2 * C.n[2];
    const T Mc = C.K + T(4.0 / 3.0) * C.G;
    // own xy node (i, j)
    const T gxy = f_xy * T(0.25) * (sG[sk][c - W - 1] + sG[sk][c - W] + sG[sk][c - 1] + C.G);
    const T sxy = T(-0.5) * gxy * (sExy[sk][c - W - 1] + sExy[sk][c - W] + sExy[sk][c - 1] + C.xy);
    // own z edges at level k+1
    const int kn1 = k + 1;
    T sxz_n = T(0), syz_n = T(0), gxz_n = T(0), gyz_n = T(0);
    if (kn1 < g.nz) {                 // block-uniform
      gxz_n = f_xz * T(0.25) * (sG[sk][c - 1] + C.G + sG[sk1][c - 1] + N.G);
      sxz_n = T(-0.5) * gxz_n * (sExz[sk][c - 1] + C.xz + sExz[sk1][c - 1] + N.xz);
      gyz_n = f_yz * T(0.25) * (sG[sk][c - W] + C.G + sG[sk1][c - W] + N.G);
      syz_n = T(-0.5) * gyz_n * (sEyz[sk][c - W] + C.yz + sEyz[sk1][c - W] + N.yz);
    }
    sSxx[c] = sxx;
    sSyy[c] = syy;
    sSxy[c] = sxy;
    sGxy[c] = gxy;
    sSxz[sk1][c] = sxz_n;
    sSyz[sk1][c] = syz_n;
    sGxz[sk1][c] = gxz_n;
    sGyz[sk1][c] = gyz_n;
    // the moduli of the cells left of and below the own cell, read before the
    // barrier: after it, other waves stash plane k+2 into slot sk
    const T m_l = sK[sk][c - 1] + T(4.0 / 3.0) * sG[sk][c - 1];
    const T m_b = sK[sk][c - W] + T(4.0 / 3.0) * sG[sk][c - W];
    ring_items(sk, kn1, sk, sk1, sk1, true);
    __syncthreads();
    if (own) {
      const int e = own_e + k * pl;
      const T q0 = f_xz * (sSxx[c - 1] - sxx + sxy - sSxy[c + W] + sxz_c - sxz_n);
      const T q1 = f_yz * (sSyy[c - W] - syy + sxy - sSxy[c + 1] + syz_c - syz_n);
      const T q2 = k > 0 ? szz_prev - szz + sxz_c - sSxz[sk][c + 1] + syz_c - sSyz[sk][c + W] : T(0);
      const T d0 = f_i * (m_l + Mc + gxy + sGxy[c + W] + gxz_c + gxz_n);
      const T d1 = f_j * (m_b + Mc + gxy + sGxy[c + 1] + gyz_c + gyz_n);
      const T d2 = k > 0 ? m_prev + Mc + gxz_c + sGxz[sk][c + 1] + gyz_c + sGyz[sk][c + W] : T(0);
      const T q[3] = {q0, q1, q2}, d[3] = {d0, d1, d2};
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const T r = -q[cc];
        const T di = d[cc] > T(0) ? T(1) / (d[cc] * ih) : T(0);
        a.o1[cc][e] = r;
        a.dinv[cc][e] = di;
        if (a.lo_w[2 + cc]) a.lo_w[2 + cc][e] = bf16_rne((float)di);
        acc += (double)r * (double)r;
      }
    }
    szz_prev = szz;
    m_prev = Mc;
    sxz_c = sxz_n;
    syz_c = syz_n;
    gxz_c = gxz_n;
    gyz_c = gyz_n;
    if (k + 1 < k1) stash(R, k + 2, sk, C);   // plane k+2 into the slot of plane k
    fetch(R, k + 4, k + 3 < k1);
    __syncthreads();
  };
  int k = k0;
  for (; k + 1 < k1; k += 2) {
    plane(k, rb, 0, oA, oB);
    plane(k + 1, ra, 1, oB, oA);
  }
  if (k < k1) plane(k, rb, 0, oA, oB);
  const double s0 = block_sum_n<NTB>(acc, red);
  if (threadIdx.x == 0) a.part[bid] = s0;
}

// ---------------------------------------------------------------------------
// 2D (plane strain) q = A p with the direction update fused in.
//
// Block = 256 threads over 256 consecutive x columns, marching along y over
// `kz` rows.  Each thread keeps its own column's values of rows j and j+1 in
// registers; only the x neighbours go through a one-row LDS tile (width 258).
// The two stresses the tile needs outside it (sigma_xx of the cell left of
// the tile, the xy edge right of it) are computed by two threads.
// ---------------------------------------------------------------------------
constexpr int A2W = 256;                 // columns per block
template <typename T>
struct Apply2Smem {
  static constexpr int W = A2W + 2;
  double red[A2W / 64];
  T sP[2][2][W];                         // [row slot][component][x]
  T sG[2][W];
  T sK[2];                               // K of the ring cell left of the tile, per row slot
  T sSxx[W];
  T sSxy[2][W];                          // xy edge stresses at two y levels
};

// AM (the 3D kernel's modes): APPLY_CG inside the CG recurrence; APPLY_SMOOTH
// one Jacobi sweep of a multigrid level, o1 = z + omega D^-1 (b - A z), or
// with omega = 0 the residual b - A z (b in jr), with partials of b . o1;
// APPLY_SMOOTH0 the first two sweeps from zero, z = omega0 D^-1 b formed as
// the rows are loaded.
template <typename T, int AM = APPLY_CG>
__device__ __forceinline__ void apply2_tile(const ElastArgs<T>& a, int bx, int by, double beta, bool first, int pidx,
                                            char* smem) {
  constexpr bool kSmooth0 = AM == APPLY_SMOOTH0, kSmooth = AM == APPLY_SMOOTH || kSmooth0;
  constexpr int W = A2W + 2;
  Apply2Smem<T>& SM = *reinterpret_cast<Apply2Smem<T>*>(smem);
  auto& sP = SM.sP;
  auto& sG = SM.sG;
  auto& sK = SM.sK;
  auto& sSxx = SM.sSxx;
  auto& sSxy = SM.sSxy;
  double* red = SM.red;

  const Grid& g = a.g;
  const int i0 = bx * A2W;
  const int i = i0 + threadIdx.x;
  const int c = threadIdx.x + 1;         // own x position in the row tile
  const bool own = i < g.nx;
  const T ih = a.p.ih;
  const T tb = (T)beta;

  // ring positions: thread 0 -> x = i0 - 1 (tile slot 0), thread 1 -> x = i0 + A2W (slot W - 1)
  const int rg_x = threadIdx.x == 0 ? i0 - 1 : i0 + A2W;
  const int rg_t = threadIdx.x == 0 ? 0 : (threadIdx.x == 1 ? W - 1 : -1);
  const bool rg_ok = rg_t >= 0 && rg_x >= 0 && rg_x < g.nx;

  // the vector applied: z, or z + beta p (CG), or omega0 D^-1 b (APPLY_SMOOTH0:
  // b in the z slots, D^-1 in the direction slots)
  const T* const* zs = kSmooth0 ? a.jr : a.z;
  const T* const* us = kSmooth0 ? a.dinv : a.u;
  const T om0 = (T)a.omega0;
  auto comb = [&](T z, T p) -> T {
    if constexpr (kSmooth0) return om0 * p * z;
    else return first ? z : z + tb * p;
  };
  T oz[2], op[2] = {T(0), T(0)}, og, ok, hz[2], hp[2] = {T(0), T(0)}, hg, hk;
  bool oin = false, hin = false;
  auto fetch = [&](int jj) {
    const bool yin = jj >= 0 && jj < g.ny;
    oin = own && yin;
    hin = rg_ok && yin;
    const int eo = oin ? jj * g.px + i : 0;
    const int eh = hin ? jj * g.px + rg_x : 0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      oz[d] = zs[d][eo];
      hz[d] = zs[d][eh];
      if constexpr (!kSmooth || kSmooth0) {     // a sweep applies z itself
        op[d] = us[d][eo];
        hp[d] = us[d][eh];
      }
    }
    og = a.G[eo]; ok = a.K[eo];
    hg = a.G[eh]; hk = a.K[eh];
  };
  auto stash = [&](int slot, T (&vp)[2], T& vg, T& vk) {
#pragma unroll
    for (int d = 0; d < 2; ++d) vp[d] = oin ? comb(oz[d], op[d]) : T(0);
    vg = oin ? og : T(0);
    vk = oin ? ok : T(0);
    sP[slot][0][c] = vp[0];
    sP[slot][1][c] = vp[1];
    sG[slot][c] = vg;
    if (rg_t >= 0) {
#pragma unroll
      for (int d = 0; d < 2; ++d) sP[slot][d][rg_t] = hin ? comb(hz[d], hp[d]) : T(0);
      sG[slot][rg_t] = hin ? hg : T(0);
      if (rg_t == 0) sK[slot] = hin ? hk : T(0);
    }
  };
  // xy edge stress at node (ii, jn) between rows jn-1 (slot s0) and jn (slot s1),
  // tile position q (x = ii)
  auto xy_edge = [&](int q, int ii, int jn, int s0, int s1) -> T {
    if (!(ii > 0 && ii < g.nx && jn > 0 && jn < g.ny)) return T(0);
    const T ge = T(0.25) * (sG[s0][q - 1] + sG[s0][q] + sG[s1][q - 1] + sG[s1][q]);
    return ge * ((sP[s1][0][q] - sP[s0][0][q]) + (sP[s1][1][q] - sP[s1][1][q - 1])) * ih;
  };

  const int j0 = by * a.kz;
  const int j1 = min(j0 + a.kz, g.ny);
  T pc[2], gc, kc, pn[2], gn, kn;
  T syy_prev = T(0), sxy_c = T(0);

  // prologue: rows j0-1 and j0; sigma_yy of the own cell below; xy edges at level j0
  {
    T pb[2], gb, kb;
    fetch(j0 - 1);
    stash((j0 - 1) & 1, pb, gb, kb);
    fetch(j0);
    stash(j0 & 1, pc, gc, kc);
    __syncthreads();
    const int sa = (j0 - 1) & 1, sb = j0 & 1;
    if (j0 > 0) {
      const T exx = (sP[sa][0][c + 1] - pb[0]) * ih;
      const T eyy = (pc[1] - pb[1]) * ih;
      const T tr = exx + eyy;
      const T G2 = T(2) * gb;
      syy_prev = kb * tr - G2 * tr * T(1.0 / 3.0) + G2 * eyy;
    }
    sxy_c = xy_edge(c, i, j0, sa, sb);
    sSxy[sb][c] = sxy_c;
    if (threadIdx.x == 1) sSxy[sb][W - 1] = xy_edge(W - 1, i0 + A2W, j0, sa, sb);
    __syncthreads();
    fetch(j0 + 1);
    stash((j0 + 1) & 1, pn, gn, kn);
    fetch(j0 + 2);
    __syncthreads();
  }

  double acc = 0.0;
  for (int j = j0; j < j1; ++j) {
    const int sj = j & 1, sj1 = (j + 1) & 1;
    // own cell stresses of row j (plane strain: eps_zz = 0) and own xy edge at level j+1
    const T exx = (sP[sj][0][c + 1] - pc[0]) * ih;
    const T eyy = (pn[1] - pc[1]) * ih;
    const T tr = exx + eyy;
    const T G2 = T(2) * gc;
    const T lam = kc * tr - G2 * tr * T(1.0 / 3.0);
    const T sxx = lam + G2 * exx, syy = lam + G2 * eyy;
    T sxy_n = T(0);
    if (i > 0 && i < g.nx && j + 1 < g.ny) {
      const T ge = T(0.25) * (sG[sj][c - 1] + gc + sG[sj1][c - 1] + gn);
      sxy_n = ge * ((pn[0] - pc[0]) + (pn[1] - sP[sj1][1][c - 1])) * ih;
    }
    sSxx[c] = sxx;
    sSxy[sj1][c] = sxy_n;
    if (threadIdx.x == 0) {              // sigma_xx of the cell left of the tile
      const T hexx = (sP[sj][0][1] - sP[sj][0][0]) * ih;
      const T heyy = (sP[sj1][1][0] - sP[sj][1][0]) * ih;
      const T htr = hexx + heyy;
      const T hG2 = T(2) * sG[sj][0];
      sSxx[0] = sK[sj] * htr - hG2 * htr * T(1.0 / 3.0) + hG2 * hexx;
    }
    if (threadIdx.x == 1) sSxy[sj1][W - 1] = xy_edge(W - 1, i0 + A2W, j + 1, sj, sj1);
    __syncthreads();
    if (own) {
      const int e = j * g.px + i;
      T q0 = T(0), q1 = T(0);
      if (i > 0) q0 = sSxx[c - 1] - sxx + sxy_c - sxy_n;
      if (j > 0) q1 = syy_prev - syy + sxy_c - sSxy[sj][c + 1];
      if constexpr (kSmooth) {
        const T qv[2] = {q0, q1};
        const T om = (T)a.omega;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const T jb = a.jr[d][e];
          const T r = jb - qv[d];
          T o = r;                                   // the residual sweep (omega = 0) reads no D^-1
          if (a.omega != 0.0) o = pc[d] + om * a.dinv[d][e] * r;
          a.o1[d][e] = o;
          acc += (double)jb * (double)o;
        }
      } else {
        a.o1[0][e] = pc[0]; a.o1[1][e] = pc[1];
        a.o2[0][e] = q0; a.o2[1][e] = q1;
        acc += (double)pc[0] * (double)q0 + (double)pc[1] * (double)q1;
      }
    }
    syy_prev = syy;
    sxy_c = sxy_n;
    if (j + 1 < j1) {
      pc[0] = pn[0]; pc[1] = pn[1];
      gc = gn;
      kc = kn;
      stash(sj, pn, gn, kn);   // row j+2 into the slot of row j
      fetch(j + 3);
    }
    __syncthreads();
  }
  const double s0 = block_sum_n<A2W>(acc, red);
  if (threadIdx.x == 0) a.part[pidx] = s0;
}

// ---------------------------------------------------------------------------
// 2D q = A p with p = z + beta p, by one wave over a strip of A2S columns,
// marching along y over rows [j0, j1).  Lane l holds column sx*A2S - 1 + l:
// lanes 1..A2S are the strip's own columns, lanes 0 and A2S+1 its left and
// right neighbour columns, so every x neighbour a stencil term needs is one
// lane away (shuffles: no LDS tile and no block barrier).  The two edge lanes
// only supply what their inner neighbours read from them (the cell stress
// left of the strip, the xy edge stress right of it) and store nothing.  The
// arithmetic is the same, term by term, as the block tile's above.  Returns
// the lane's share of p.q.
// ---------------------------------------------------------------------------
constexpr int A2S = 62;                  // columns per strip
constexpr int A2PF = 8;                  // rows of loads in flight per strip

template <typename T>
__device__ __forceinline__ double apply2_strip(const ElastArgs<T>& a, int sx, int j0, int j1, double beta,
                                               bool first) {
  const Grid& g = a.g;
  const int lane = threadIdx.x & 63;
  const int i = sx * A2S - 1 + lane;
  const bool col = i >= 0 && i < g.nx;
  const bool store = col && lane >= 1 && lane <= A2S;
  const T ih = a.p.ih;
  const T tb = (T)beta;

  // raw loads of A2PF rows in flight: row j0 + 2 + m travels in set m % A2PF
  // (every set index below is a compile-time constant, so the sets stay in
  // registers and each wait leaves the newer sets outstanding)
  struct Raw { T z[2], p[2], g, k; bool in; };
  Raw rw[A2PF];
  // rows past j1 (the last one the strip reads) load element 0 instead
  auto fetch = [&](Raw& R, int jj) {
    R.in = col && jj >= 0 && jj <= j1 && jj < g.ny;
    const int e = R.in ? jj * g.px + i : 0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      R.z[d] = a.z[d][e];
      R.p[d] = a.u[d][e];
    }
    R.g = a.G[e];
    R.k = a.K[e];
  };
  auto take = [&](const Raw& R, T (&vp)[2], T& vg, T& vk) {
#pragma unroll
    for (int d = 0; d < 2; ++d) vp[d] = R.in ? (first ? R.z[d] : R.z[d] + tb * R.p[d]) : T(0);
    vg = R.in ? R.g : T(0);
    vk = R.in ? R.k : T(0);
  };
  auto left = [](T v) { return __shfl_up(v, 1, 64); };      // value of column i - 1
  auto right = [](T v) { return __shfl_down(v, 1, 64); };   // value of column i + 1

  T pc[2], gc, kc, pn[2], gn, kn;
  T syy_prev = T(0), sxy_c = T(0);
  // prologue: rows j0-1 .. j0+1; sigma_yy of the own cell below; xy edge at level j0
  {
    T pb[2], gb, kb;
    fetch(rw[0], j0 - 1);
    fetch(rw[1], j0);
    fetch(rw[2], j0 + 1);
    take(rw[0], pb, gb, kb);
    take(rw[1], pc, gc, kc);
    take(rw[2], pn, gn, kn);
#pragma unroll
    for (int m = 0; m < A2PF; ++m) fetch(rw[m], j0 + 2 + m);
    const T pb0r = right(pb[0]);
    const T gbl = left(gb), gcl = left(gc), pc1l = left(pc[1]);
    if (j0 > 0) {
      const T exx = (pb0r - pb[0]) * ih;
      const T eyy = (pc[1] - pb[1]) * ih;
      const T tr = exx + eyy;
      const T G2 = T(2) * gb;
      syy_prev = kb * tr - G2 * tr * T(1.0 / 3.0) + G2 * eyy;
    }
    if (i > 0 && i < g.nx && j0 > 0 && j0 < g.ny) {
      const T ge = T(0.25) * (gbl + gb + gcl + gc);
      sxy_c = ge * ((pc[0] - pb[0]) + (pc[1] - pc1l)) * ih;
    }
  }

  double acc = 0.0;
  // row j (m = j - j0): own cell stresses of row j (plane strain), own xy edge
  // at level j+1, the forces of row j; then row j+2 moves in from set m % A2PF
  // and row j+2+A2PF is fetched into it
  auto row = [&](int j, Raw& R) {
    const T pc0r = right(pc[0]);
    const T gcl = left(gc), gnl = left(gn), pn1l = left(pn[1]);
    const T exx = (pc0r - pc[0]) * ih;
    const T eyy = (pn[1] - pc[1]) * ih;
    const T tr = exx + eyy;
    const T G2 = T(2) * gc;
    const T lam = kc * tr - G2 * tr * T(1.0 / 3.0);
    const T sxx = lam + G2 * exx, syy = lam + G2 * eyy;
    T sxy_n = T(0);
    if (i > 0 && i < g.nx && j + 1 < g.ny) {
      const T ge = T(0.25) * (gcl + gc + gnl + gn);
      sxy_n = ge * ((pn[0] - pc[0]) + (pn[1] - pn1l)) * ih;
    }
    const T sxx_l = left(sxx);           // cell stress of column i - 1
    const T sxy_r = right(sxy_c);        // xy edge of node (i + 1, j)
    if (store) {
      const int e = j * g.px + i;
      T q0 = T(0), q1 = T(0);
      if (i > 0) q0 = sxx_l - sxx + sxy_c - sxy_n;
      if (j > 0) q1 = syy_prev - syy + sxy_c - sxy_r;
      a.o1[0][e] = pc[0]; a.o1[1][e] = pc[1];
      a.o2[0][e] = q0; a.o2[1][e] = q1;
      acc += (double)pc[0] * (double)q0 + (double)pc[1] * (double)q1;
    }
    syy_prev = syy;
    sxy_c = sxy_n;
    pc[0] = pn[0]; pc[1] = pn[1];
    gc = gn;
    kc = kn;
    take(R, pn, gn, kn);                 // row j+2
    fetch(R, j + 2 + A2PF);
  };
  for (int j = j0; j < j1; j += A2PF) {
#pragma unroll
    for (int m = 0; m < A2PF; ++m)
      if (j + m < j1) row(j + m, rw[m]);
  }
  return acc;
}

// CG scalars at the start of an apply: r.z and r.r of the latest residual
// (partials part_in[0..n) and part_in[n..2n)); identical in every block.
template <int NTB>
__device__ __forceinline__ void cg_entry_sums(const double* part_in, int n, double& rz, double& rr) {
  __shared__ double sh2[2][NTB / 64];
  double v0 = 0.0, v1 = 0.0;
  for (int q = threadIdx.x; q < n; q += NTB) { v0 += part_in[q]; v1 += part_in[n + q]; }
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { sh2[0][threadIdx.x >> 6] = v0; sh2[1][threadIdx.x >> 6] = v1; }
  __syncthreads();
  rz = 0.0;
  rr = 0.0;
#pragma unroll
  for (int w = 0; w < NTB / 64; ++w) { rz += sh2[0][w]; rr += sh2[1][w]; }
}

template <typename T>
__global__ __launch_bounds__(A2W) void k_apply2(ElastArgs<T> a) {
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  const int tile = xcd_tile(bid, gridDim.x * gridDim.y);
  if (a.scal[S_CONV] != 0.0) return;
  double rzv, rrv;
  cg_entry_sums<A2W>(a.part_in, a.n_in, rzv, rrv);
  if (rrv <= a.tol2 * a.scal[S_BB]) {
    if (bid == 0 && threadIdx.x == 0) a.scal[S_CONV] = 1.0;
    return;
  }
  const bool first = a.scal[S_FIRST] != 0.0;
  const double beta = first ? 0.0 : rzv / a.scal[S_RZ + (a.parity ^ 1)];
  if (bid == 0 && threadIdx.x == 0) {
    a.scal[S_RZ + a.parity] = rzv;
    a.scal[S_RR] = rrv;
  }
  __shared__ __align__(16) char smem[sizeof(Apply2Smem<T>)];
  apply2_tile(a, tile % gridDim.x, tile / gridDim.x, beta, first, bid, smem);
}

// 2D multigrid sweep (AM = APPLY_SMOOTH or APPLY_SMOOTH0) of one level on the
// row tiles of k_apply2; exits at entry once the solve has converged
template <typename T, int AM>
__global__ __launch_bounds__(A2W) void k_apply2s(ElastArgs<T> a) {
  if (a.scal[S_CONV] != 0.0) return;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  const int tile = xcd_tile(bid, gridDim.x * gridDim.y);
  __shared__ __align__(16) char smem[sizeof(Apply2Smem<T>)];
  apply2_tile<T, AM>(a, tile % gridDim.x, tile / gridDim.x, 0.0, true, bid, smem);
}

// ---------------------------------------------------------------------------
// CG update: u += alpha p, r -= alpha q, z = D^-1 r; partials of r.z and r.r
// ---------------------------------------------------------------------------
template <typename T>
struct UpdArgs {
  int n;                   // elements per component array (multiple of 16)
  T* u[3];
  const T* p[3];
  const T* pp[3];          // 3D: the previous direction (read after odd iterations)
  T* r[3];
  const T* q[3];
  const T* dinv[3];
  T* z[3];
  double* part;            // [2][nblocks]
  const double* part_in;   // APPLY partials (p.q)
  int n_in;
  double* scal;
  int parity;
};

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double2; };

// u += alpha p, r -= alpha q, z = D^-1 r over the vector range [v0, v1) of
// every component (vectors of 16 bytes); accumulates r.z and r.r.  Without
// XU, u is updated only when xstep is set, with the steps of this iteration
// and the previous one (alpha_prev along pp), in the order of two single
// updates.  With NZ (another preconditioner forms z) neither D^-1 nor z is
// touched and r.z is left at zero.
template <typename T, int DIM, bool XU = true, bool NZ = false>
__device__ __forceinline__ void cg_update_range(const UpdArgs<T>& a, int v0, int v1, int vstride, double alpha,
                                                double& rz, double& rr, bool xstep = false,
                                                double alpha_prev = 0.0) {
  const T al = (T)alpha, alp = (T)alpha_prev;
  using V = typename Vec4<T>::type;
  constexpr int VN = sizeof(V) / sizeof(T);
  // XM: 0 u untouched, 1 u += alpha p, 2 u += alpha_prev pp + alpha p
  auto run = [&](auto xm_tag) {
    constexpr int XM = decltype(xm_tag)::value;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      V* uu = reinterpret_cast<V*>(a.u[c]);
      const V* pp = reinterpret_cast<const V*>(a.p[c]);
      const V* ppp = reinterpret_cast<const V*>(XM == 2 ? a.pp[c] : a.p[c]);
      V* rrp = reinterpret_cast<V*>(a.r[c]);
      const V* qq = reinterpret_cast<const V*>(a.q[c]);
      const V* dd = reinterpret_cast<const V*>(a.dinv[c]);
      V* zz = reinterpret_cast<V*>(a.z[c]);
      for (int v = v0; v < v1; v += vstride) {
        V uv, pv, ppv, rv = rrp[v], qv = qq[v], dv, zv;
        if constexpr (!NZ) dv = dd[v];
        if constexpr (XM >= 1) {
          uv = uu[v];
          pv = pp[v];
        }
        if constexpr (XM == 2) ppv = ppp[v];
        T* ue = reinterpret_cast<T*>(&uv);
        const T* pe = reinterpret_cast<const T*>(&pv);
        const T* ppe = reinterpret_cast<const T*>(&ppv);
        T* re = reinterpret_cast<T*>(&rv);
        const T* qe = reinterpret_cast<const T*>(&qv);
        const T* de = reinterpret_cast<const T*>(&dv);
        T* ze = reinterpret_cast<T*>(&zv);
#pragma unroll
        for (int l = 0; l < VN; ++l) {
          if constexpr (XM == 1) {
            ue[l] += al * pe[l];
          } else if constexpr (XM == 2) {
            const T t = ue[l] + alp * ppe[l];
            ue[l] = t + al * pe[l];
          }
          re[l] -= al * qe[l];
          if constexpr (!NZ) {
            ze[l] = de[l] * re[l];
            rz += (double)re[l] * (double)ze[l];
          }
          rr += (double)re[l] * (double)re[l];
        }
        if constexpr (XM >= 1) uu[v] = uv;
        rrp[v] = rv;
        if constexpr (!NZ) zz[v] = zv;
      }
    }
  };
  if constexpr (XU) run(std::integral_constant<int, 1>());
  else if (xstep) run(std::integral_constant<int, 2>());
  else run(std::integral_constant<int, 0>());
}

// 3D: u is updated after odd iterations only, with the steps of the last two
// (the previous direction is still held in the other direction buffer); the
// alpha of every update goes to the device scalars (slot S_ALPHA + parity),
// and the apply launch that stops the solve after an even iteration adds its
// step.  NZ: z comes from another preconditioner (not formed here).
template <typename T, int DIM, bool NZ = false>
__global__ __launch_bounds__(NT) void k_cg_update(UpdArgs<T> a) {
  constexpr bool XU = DIM != 3;
  __shared__ double red[2 * (NT / 64)];
  if (a.scal[S_CONV] != 0.0) return;
  const double pq = sum_partials(a.part_in, a.n_in, red);
  const double alpha = a.scal[S_RZ + a.parity] / pq;
  using V = typename Vec4<T>::type;
  constexpr int VN = sizeof(V) / sizeof(T);
  double rz = 0.0, rr = 0.0;
  const bool xstep = !XU && a.parity == 1;
  const double alpha_prev = xstep ? a.scal[S_ALPHA] : 0.0;
  cg_update_range<T, DIM, XU, NZ>(a, blockIdx.x * NT + threadIdx.x, a.n / VN, gridDim.x * NT, alpha, rz, rr, xstep,
                                  alpha_prev);
  double s0 = rz, s1 = rr;
  block_sum2(s0, s1, red);
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = s0;
    a.part[gridDim.x + blockIdx.x] = s1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal[S_FIRST] = 0.0;
    a.scal[S_ITERS] += 1.0;
    a.scal[S_ALPHA + a.parity] = alpha;
  }
}

// After a chunk of CG launches: mark convergence from the latest residual
// with `mark` (3D: the index + 1 of the apply launch that completes u);
// tol2 < 0 marks without testing (3D, iteration limit reached: u is still
// completed).
__global__ __launch_bounds__(NT) void k_cg_check(const double* part_in, int n_in, double* scal, double tol2,
                                                 double mark) {
  __shared__ double red[NT / 64];
  if (scal[S_CONV] != 0.0) return;
  double rr = sum_partials(part_in + n_in, n_in, red);
  if (threadIdx.x == 0) {
    scal[S_RR] = rr;
    if (tol2 < 0.0 || rr <= tol2 * scal[S_BB]) scal[S_CONV] = mark;
  }
}

// Sum of partials into one scalar slot.
__global__ __launch_bounds__(NT) void k_sum_to(const double* part, int n, double* scal, int slot) {
  __shared__ double red[NT / 64];
  double s = sum_partials(part, n, red);
  if (threadIdx.x == 0) scal[slot] = s;
}

// ---------------------------------------------------------------------------
// Step kernels
// ---------------------------------------------------------------------------
template <typename T>
struct CellArgs {
  Grid g;
  KP<T> p;
  const T *pf, *pw, *xO, *xH, *xW, *mu;
  T *npf, *npw, *nxO, *nxH, *nxW;
  // FP32 state only: low parts of the five fields (value = hi + lo, the hi
  // arrays above), read and written by the field update; null in FP64
  const T* lo[5];
  T* nlo[5];
  // linearly implicit species (null: explicit): the step writes the explicit
  // increments dt T of x_O, x_H, x_H2O into sp_r and the cell diffusivities
  // D_O, D_H, D_H2O of the implicit operator into sp_D; the species
  // themselves are updated after the solve
  T* sp_r[3];
  T* sp_D[3];
  const T* u[3];
  T* epsp;
  T* epsP;
  T* K;
  T* G;
  T* mu_out;
  // finite-strain mechanics: [2][nx ny nz] compact FP64 cell driving forces
  // d psi / d phi_f, d psi / d phi_w added to those of the phase fields (null: none)
  const double* gext;
  double* part;            // [NQ][nblocks]
};

constexpr int NQ_STEP = 8;   // O total, H total, x_O sum, O outflux, H outflux, max vm, max epsP, nonfinite

template <typename T, int DIM>
__device__ __forceinline__ void moduli_tile(const CellArgs<T>& a, int bx, int by, int bz) {
  const int i = bx * TX + (threadIdx.x & (TX - 1));
  const int j = by * TY + threadIdx.x / TX;
  const int k = bz;
  if (i >= a.g.nx || j >= a.g.ny) return;
  const int e = gidx(a.g, i, j, k);
  T K, G;
  moduli(a.p, a.pf[e], a.pw[e], K, G);
  a.K[e] = K;
  a.G[e] = G;
}

template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_moduli(CellArgs<T> a) {
  moduli_tile<T, DIM>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// mu_O = d psi_che / d x_O - kappa_O lap(x_O), mirror (no-flux) ghosts
template <typename T, int DIM>
__device__ __forceinline__ void mu_tile(const CellArgs<T>& a, int bx, int by, int bz) {
  const Grid& g = a.g;
  const int i = bx * TX + (threadIdx.x & (TX - 1));
  const int j = by * TY + threadIdx.x / TX;
  const int k = bz;
  if (i >= g.nx || j >= g.ny) return;
  const int e = gidx(g, i, j, k);
  const T xc = a.xO[e];
  T lap = (a.xO[i + 1 < g.nx ? e + 1 : e] - xc) - (xc - a.xO[i > 0 ? e - 1 : e]);
  lap += (a.xO[j + 1 < g.ny ? e + g.px : e] - xc) - (xc - a.xO[j > 0 ? e - g.px : e]);
  if constexpr (DIM == 3) {
    const int pl = g.px * g.ny;
    lap += (a.xO[k + 1 < g.nz ? e + pl : e] - xc) - (xc - a.xO[k > 0 ? e - pl : e]);
  }
  T mu, MO, DH, DW;
  transport(a.p, a.pf[e], a.pw[e], xc, mu, MO, DH, DW);
  a.mu_out[e] = mu - a.p.kappaO * lap * a.p.ih2;
}

template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_mu(CellArgs<T> a) {
  mu_tile<T, DIM>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T>
__device__ __forceinline__ T face_flux(T ca, T cb, T va, T vb, T ih) {
  return T(-0.5) * (ca + cb) * (vb - va) * ih;
}

template <typename T, int DIM>
__device__ __forceinline__ T shear_xy(const Grid& g, const T* ux, const T* uy, int i, int j, int k, T ih) {
  if (i <= 0 || i >= g.nx || j <= 0 || j >= g.ny) return T(0);
  const int e = gidx(g, i, j, k);
  return T(0.5) * ((ux[e] - ux[e - g.px]) + (uy[e] - uy[e - 1])) * ih;
}
template <typename T>
__device__ __forceinline__ T shear_xz(const Grid& g, const T* ux, const T* uz, int i, int j, int k, T ih) {
  if (i <= 0 || i >= g.nx || k <= 0 || k >= g.nz) return T(0);
  const int e = gidx(g, i, j, k), pl = g.px * g.ny;
  return T(0.5) * ((ux[e] - ux[e - pl]) + (uz[e] - uz[e - 1])) * ih;
}
template <typename T>
__device__ __forceinline__ T shear_yz(const Grid& g, const T* uy, const T* uz, int i, int j, int k, T ih) {
  if (j <= 0 || j >= g.ny || k <= 0 || k >= g.nz) return T(0);
  const int e = gidx(g, i, j, k), pl = g.px * g.ny;
  return T(0.5) * ((uy[e] - uy[e - pl]) + (uz[e] - uz[e - g.px])) * ih;
}

// The explicit update of one cell given its transport terms (Laplacians of
// the phases, flux divergences, outward boundary fluxes) and its total
// strain: phase quantities and driving forces (Eq. 33), return map (Eq. 25,
// 34), reaction (Eq. 27, 28), explicit Euler update, and the cell's
// contributions to the step's partial sums.
// New value of a field given its old value and increment d.  FP64 state:
// old + d.  FP32 state: the value is the pair (hi, lo) with value hi + lo; the
// FP32 increment is added in FP64 (and the sum later split again into an FP32
// pair, about 48 significant bits), so that increments far below half an
// FP32 ulp of the field accumulate instead of being rounded away.
template <typename T>
__device__ __forceinline__ double field_new(T hi, T lo, T d) {
  if constexpr (sizeof(T) == 4)
    return ((double)hi + (double)lo) + (double)d;   // hi + lo is exact in FP64
  else
    return hi + d;
}
template <typename T>
__device__ __forceinline__ void field_store(double v, T* out_hi, T* out_lo, int e) {
  if constexpr (sizeof(T) == 4) {
    const float h = (float)v;
    out_hi[e] = h;
    out_lo[e] = (float)(v - (double)h);
  } else {
    (void)out_lo;
    out_hi[e] = v;
  }
}

// The order parameters lie in [0, 1] with phi_g = 1 - phi_f - phi_w (Sec.
// 2.2): after the explicit update (phi_f, phi_g, phi_w) is replaced by its
// Euclidean projection onto {phi_a >= 0, sum = 1}.  Michelot's active-set
// iteration (1986): shift the active entries by (sum - 1) / count, drop the
// ones that become negative, repeat; with three entries two passes suffice.
// A triple already inside is left unchanged.
__device__ __forceinline__ void phase_bound(double& pf, double& pw) {
  double a0 = pf, a1 = 1.0 - pf - pw, a2 = pw;
  if (a0 >= 0.0 && a1 >= 0.0 && a2 >= 0.0) return;
  bool k0 = true, k1 = true, k2 = true;
  double th = 0.0;
#pragma unroll
  for (int pass = 0; pass < 3; ++pass) {
    const double sum = (k0 ? a0 : 0.0) + (k1 ? a1 : 0.0) + (k2 ? a2 : 0.0);
    const int cnt = (int)k0 + (int)k1 + (int)k2;
    th = (sum - 1.0) / (double)cnt;
    const bool d0 = k0 && a0 - th < 0.0, d1 = k1 && a1 - th < 0.0, d2 = k2 && a2 - th < 0.0;
    if (!(d0 || d1 || d2)) break;
    k0 = k0 && !d0;
    k1 = k1 && !d1;
    k2 = k2 && !d2;
  }
  pf = k0 ? a0 - th : 0.0;
  pw = k2 ? a2 - th : 0.0;
}

template <typename T, int DIM>
__device__ __forceinline__ void cell_update(const CellArgs<T>& a, int e, T pf, T pw, T xO, T xH, T xW, T lf, T lw,
                                            T divO, T divH, T divW, T bO, T bH, const T (&eb)[6],
                                            const T (&lo)[5], T DHc, T DWc, double (&acc)[NQ_STEP]) {
  const Grid& g = a.g;
  const KP<T>& p = a.p;
  lf *= p.ih2;
  lw *= p.ih2;

  // phase quantities and the chemical / barrier driving forces (Eq. 33)
  Phase<T> q;
  phase_eval(p, pf, pw, q);
  const T pg = T(1) - pf - pw;
  T gf = p.w[0] * interp_dm(pf, p.mform) - p.w[1] * interp_dm(pg, p.mform);
  T gw = p.w[2] * interp_dm(pw, p.mform) - p.w[1] * interp_dm(pg, p.mform);
  if (p.chem) {
    T f0, f1, f2, g0, g1, g2, w0, w1, w2;
    fe_ferrite(xO, f0, f1, f2);
    fe_gas(xO, g0, g1, g2);
    fe_wuestite(xO, w0, w1, w2);
    gf += p.scale * (q.dhf * f0 - q.dhg * g0);
    gw += p.scale * (q.dhw * w0 - q.dhg * g0);
  }
  T vm = T(0), epsPn = T(0);
  if (p.mech) {
    constexpr int NC = (DIM == 2) ? 4 : 6;
    T ep[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < NC; ++c) ep[c] = a.epsp[c * g.ns + e];
    const T epsP0 = a.epsP[e];
    epsPn = epsP0;
    // elastic strain and its deviator
    T ee[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) ee[c] = eb[c] - ep[c];
    ee[0] -= q.eT; ee[1] -= q.eT; ee[2] -= q.eT;
    T tr = ee[0] + ee[1] + ee[2];
    T dv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) dv[c] = ee[c];
    dv[0] -= tr * T(1.0 / 3.0); dv[1] -= tr * T(1.0 / 3.0); dv[2] -= tr * T(1.0 / 3.0);
    T nd2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2] + T(2) * (dv[3] * dv[3] + dv[4] * dv[4] + dv[5] * dv[5]);
    T nd = tsqrt(nd2);
    if (p.plastic) {
      // J2 radial return, backward Euler (Eq. 25, Eq. 34)
      const T r23 = T(0.816496580927726032732428024902);   // sqrt(2/3)
      T ftr = T(2) * q.G * nd - r23 * (p.sigY + p.Hh * epsP0);
      if (ftr > T(0)) {
        T dl = ftr / (T(2) * q.G + r23 * p.Hh);
        T sc = dl / nd;
#pragma unroll
        for (int c = 0; c < 6; ++c) ep[c] += sc * dv[c];
        epsPn = epsP0 + dl;
#pragma unroll
        for (int c = 0; c < NC; ++c) a.epsp[c * g.ns + e] = ep[c];
        a.epsP[e] = epsPn;
        // the return keeps tr and scales the deviator
        T f = T(1) - T(2) * q.G * dl / (T(2) * q.G * nd);
#pragma unroll
        for (int c = 0; c < 6; ++c) dv[c] *= f;
        nd2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2] + T(2) * (dv[3] * dv[3] + dv[4] * dv[4] + dv[5] * dv[5]);
        nd = tsqrt(nd2);
      }
    }
    // elastic driving force: derivative of d_T sum h(phi_a) (K_a tr^2/2 + G_a |dev|^2)
    T pe_f = T(0.5) * p.K[0] * tr * tr + p.G[0] * nd2;
    T pe_g = T(0.5) * p.K[1] * tr * tr + p.G[1] * nd2;
    T pe_w = T(0.5) * p.K[2] * tr * tr + p.G[2] * nd2;
    T phi_el = q.hf * pe_f + q.hg * pe_g + q.hw * pe_w;
    gf += q.dTp * phi_el + q.dT * (q.dhf * pe_f - q.dhg * pe_g) - q.eTp * T(3) * q.K * tr;
    gw += q.dT * (q.dhw * pe_w - q.dhg * pe_g);
    vm = T(1.2247448713915890491) * T(2) * q.G * nd;   // sqrt(3/2) |dev sigma|
  }
  if (a.gext) {
    const int ci = e % g.px, cr = e / g.px;
    const long c = (long)cr * g.nx + ci;      // compact index of (i, j, k): rows of nx cells
    gf += (T)a.gext[c];
    gw += (T)a.gext[(long)g.nx * g.ny * g.nz + c];
  }
  // reaction (Eq. 27, 28): forward rate, zero once the cell is full of water;
  // mole fractions below zero take no part in it
  const T r = !p.rsplit && (double)xW + (double)lo[4] < 1.0 ? interp_m(pg, p.mform) * p.kfor * fmax(xO, T(0)) * fmax(xH, T(0)) : T(0);
  const T df = p.dt * p.L[0] * ((p.eps[0] + p.eps[1]) * lf + p.eps[1] * lw - gf);
  const T dw = p.dt * p.L[2] * ((p.eps[2] + p.eps[1]) * lw + p.eps[1] * lf - gw);
  const T dO = p.dt * (-divO - r);
  const T dH = p.dt * (-divH - T(2) * r);
  const T dW = p.dt * (-divW + r);
  double nf = field_new(pf, lo[0], df), nw = field_new(pw, lo[1], dw);
  phase_bound(nf, nw);
  field_store(nf, a.npf, a.nlo[0], e);
  field_store(nw, a.npw, a.nlo[1], e);
  acc[5] = (double)vm;
  acc[6] = (double)epsPn;
  if (a.sp_r[0]) {
    // implicit species: right-hand sides and coefficients of the solve; the
    // species' ledger terms come from the update that follows it
    a.sp_r[0][e] = dO;
    a.sp_r[1][e] = dH;
    a.sp_r[2][e] = dW;
    a.sp_D[0][e] = diffusivity_O(p, pf, pw);
    a.sp_D[1][e] = DHc;
    a.sp_D[2][e] = DWc;
    acc[0] = acc[1] = acc[2] = acc[3] = acc[4] = 0.0;
    const bool fin = isfinite(nf) && isfinite(nw) && isfinite(dO) && isfinite(dH) && isfinite(dW) && isfinite(vm);
    acc[7] = fin ? 0.0 : 1.0;
    return;
  }
  const double nO = field_new(xO, lo[2], dO), nH = field_new(xH, lo[3], dH), nW = field_new(xW, lo[4], dW);
  field_store(nO, a.nxO, a.nlo[2], e);
  field_store(nH, a.nxH, a.nlo[3], e);
  field_store(nW, a.nxW, a.nlo[4], e);
  acc[0] = nO + nW;
  acc[1] = nH + 2.0 * nW;
  acc[2] = nO;
  acc[3] = (double)bO;
  acc[4] = (double)bH + 2.0 * (double)bO;
  bool fin = isfinite(nf) && isfinite(nw) && isfinite(nO) && isfinite(nH) && isfinite(nW) && isfinite(vm);
  acc[7] = fin ? 0.0 : 1.0;
}

template <typename T, int DIM>
__device__ __forceinline__ void step_tile(const CellArgs<T>& a, int bx, int by, int bz, int pidx, int pstride) {
  const Grid& g = a.g;
  const KP<T>& p = a.p;
  const int i = bx * TX + (threadIdx.x & (TX - 1));
  const int j = by * TY + threadIdx.x / TX;
  const int k = bz;
  double acc[NQ_STEP] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < g.nx && j < g.ny) {
    const int e = gidx(g, i, j, k);
    const int pl = g.px * g.ny;
    const T ih = p.ih;
    const T pf = a.pf[e], pw = a.pw[e], xO = a.xO[e], xH = a.xH[e], xW = a.xW[e], muc = a.mu[e];
    T lo[5] = {T(0), T(0), T(0), T(0), T(0)};
    if constexpr (sizeof(T) == 4)
#pragma unroll
      for (int f = 0; f < 5; ++f) lo[f] = a.lo[f][e];
    T mu_l, MOc, DHc, DWc;
    transport(p, pf, pw, xO, mu_l, MOc, DHc, DWc);
    (void)mu_l;
    T lf = T(0), lw = T(0), divO = T(0), divH = T(0), divW = T(0);
    T bO = T(0), bH = T(0);   // outward boundary fluxes (J_H2O and J_H) summed over this cell's outer faces
    const int coord[3] = {i, j, k};
    const int lim[3] = {g.nx, g.ny, g.nz};
    const int step[3] = {1, g.px, pl};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool has_lo = coord[d] > 0, has_hi = coord[d] + 1 < lim[d];
      const int el = has_lo ? e - step[d] : e, eh = has_hi ? e + step[d] : e;
      const T pfl = a.pf[el], pfh = a.pf[eh], pwl = a.pw[el], pwh = a.pw[eh];
      lf += (pfh - pf) - (pf - pfl);
      lw += (pwh - pw) - (pw - pwl);
      T JOm = T(0), JOp = T(0), JHm, JHp, JWm, JWp;
      if (has_lo) {
        T m_, M, DHn, DWn;
        transport(p, pfl, pwl, a.xO[el], m_, M, DHn, DWn);
        JOm = face_flux(M, MOc, a.mu[el], muc, ih);
        JHm = face_flux(DHn, DHc, a.xH[el], xH, ih);
        JWm = face_flux(DWn, DWc, a.xW[el], xW, ih);
      } else if (p.dirichlet) {
        JHm = -DHc * (xH - p.xHbc) * (T(2) * ih);
        JWm = -DWc * (xW - p.xWbc) * (T(2) * ih);
        bH -= JHm;
        bO -= JWm;
      } else {
        JHm = T(0);
        JWm = T(0);
      }
      if (has_hi) {
        T m_, M, DHn, DWn;
        transport(p, pfh, pwh, a.xO[eh], m_, M, DHn, DWn);
        JOp = face_flux(MOc, M, muc, a.mu[eh], ih);
        JHp = face_flux(DHc, DHn, xH, a.xH[eh], ih);
        JWp = face_flux(DWc, DWn, xW, a.xW[eh], ih);
      } else if (p.dirichlet) {
        JHp = -DHc * (p.xHbc - xH) * (T(2) * ih);
        JWp = -DWc * (p.xWbc - xW) * (T(2) * ih);
        bH += JHp;
        bO += JWp;
      } else {
        JHp = T(0);
        JWp = T(0);
      }
      divO += (JOp - JOm) * ih;
      divH += (JHp - JHm) * ih;
      divW += (JWp - JWm) * ih;
    }
    T eb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (p.mech) {
      // cell strain: normal from faces, shear as the mean of four edges
      const T* ux = a.u[0];
      const T* uy = a.u[1];
      eb[0] = ((i + 1 < g.nx ? ux[e + 1] : T(0)) - ux[e]) * ih;
      eb[1] = ((j + 1 < g.ny ? uy[e + g.px] : T(0)) - uy[e]) * ih;
      eb[2] = T(0);
      eb[3] = T(0.25) * (shear_xy<T, DIM>(g, ux, uy, i, j, k, ih) + shear_xy<T, DIM>(g, ux, uy, i + 1, j, k, ih) +
                         shear_xy<T, DIM>(g, ux, uy, i, j + 1, k, ih) + shear_xy<T, DIM>(g, ux, uy, i + 1, j + 1, k, ih));
      eb[4] = T(0);
      eb[5] = T(0);
      if constexpr (DIM == 3) {
        const T* uz = a.u[2];
        eb[2] = ((k + 1 < g.nz ? uz[e + pl] : T(0)) - uz[e]) * ih;
        eb[4] = T(0.25) * (shear_xz(g, ux, uz, i, j, k, ih) + shear_xz(g, ux, uz, i + 1, j, k, ih) +
                           shear_xz(g, ux, uz, i, j, k + 1, ih) + shear_xz(g, ux, uz, i + 1, j, k + 1, ih));
        eb[5] = T(0.25) * (shear_yz(g, uy, uz, i, j, k, ih) + shear_yz(g, uy, uz, i, j + 1, k, ih) +
                           shear_yz(g, uy, uz, i, j, k + 1, ih) + shear_yz(g, uy, uz, i, j + 1, k + 1, ih));
      }
    }
    cell_update<T, DIM>(a, e, pf, pw, xO, xH, xW, lf, lw, divO, divH, divW, bO, bH, eb, lo, DHc, DWc, acc);
  }
  // the eight partials together: the wave trees of all quantities interleaved,
  // then one exchange across the waves (the same operations in the same
  // order as eight separate block reductions, with two barriers instead of 16)
  __shared__ double red8[NQ_STEP][NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int qn = 0; qn < NQ_STEP; ++qn) {
      const double v = __shfl_xor(acc[qn], o, 64);
      acc[qn] = (qn == 5 || qn == 6) ? fmax(acc[qn], v) : acc[qn] + v;
    }
  __syncthreads();                  // the previous tile's exchange has been read
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int qn = 0; qn < NQ_STEP; ++qn) red8[qn][threadIdx.x >> 6] = acc[qn];
  __syncthreads();
  if (threadIdx.x < NQ_STEP) {
    const int qn = threadIdx.x;
    const bool mx = qn == 5 || qn == 6;
    double s = mx ? red8[qn][0] : 0.0 + red8[qn][0];
#pragma unroll
    for (int q = 1; q < NT / 64; ++q) s = mx ? fmax(s, red8[qn][q]) : s + red8[qn][q];
    a.part[qn * pstride + pidx] = s;
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_step(CellArgs<T> a) {
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  step_tile<T, DIM>(a, blockIdx.x, blockIdx.y, blockIdx.z, bid, gridDim.x * gridDim.y * gridDim.z);
}

// Totals for a ledger reset: sum (x_O + x_W), sum (x_H + 2 x_W), sum x_O.
template <typename T, int DIM>
__device__ __forceinline__ void totals_tile(const CellArgs<T>& a, int bx, int by, int bz, int pidx, int pstride) {
  __shared__ double red[NT / 64];
  const int i = bx * TX + (threadIdx.x & (TX - 1));
  const int j = by * TY + threadIdx.x / TX;
  const int k = bz;
  double s0 = 0, s1 = 0, s2 = 0;
  if (i < a.g.nx && j < a.g.ny) {
    const int e = gidx(a.g, i, j, k);
    double O = (double)a.xO[e], H = (double)a.xH[e], W = (double)a.xW[e];
    if constexpr (sizeof(T) == 4) {
      O += (double)a.lo[2][e];
      H += (double)a.lo[3][e];
      W += (double)a.lo[4][e];
    }
    s0 = O + W;
    s1 = H + 2.0 * W;
    s2 = O;
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    a.part[pidx] = s0;
    a.part[pstride + pidx] = s1;
    a.part[2 * pstride + pidx] = s2;
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_totals(CellArgs<T> a) {
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  totals_tile<T, DIM>(a, blockIdx.x, blockIdx.y, blockIdx.z, bid, gridDim.x * gridDim.y * gridDim.z);
}

// Fold the eight partial arrays of k_step ([NQ_STEP][n]) into [NQ_STEP][m]:
// block b reduces entries [b len, (b+1) len) of each, in a fixed order (sums,
// and maxima for the two maximum slots), so that the one-block ledger pass
// reads m instead of n partials per quantity.
__global__ __launch_bounds__(NT) void k_fold_step(const double* part, int n, double* out, int m) {
  const int len = (n + m - 1) / m, lo = blockIdx.x * len, hi = min(n, lo + len);
  double acc[NQ_STEP];
#pragma unroll
  for (int qn = 0; qn < NQ_STEP; ++qn) acc[qn] = 0.0;
  for (int t = lo + threadIdx.x; t < hi; t += NT)
#pragma unroll
    for (int qn = 0; qn < NQ_STEP; ++qn) {
      const double v = part[qn * n + t];
      acc[qn] = (qn == 5 || qn == 6) ? fmax(acc[qn], v) : acc[qn] + v;
    }
  __shared__ double red8[NQ_STEP][NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int qn = 0; qn < NQ_STEP; ++qn) {
      const double v = __shfl_xor(acc[qn], o, 64);
      acc[qn] = (qn == 5 || qn == 6) ? fmax(acc[qn], v) : acc[qn] + v;
    }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int qn = 0; qn < NQ_STEP; ++qn) red8[qn][threadIdx.x >> 6] = acc[qn];
  __syncthreads();
  if (threadIdx.x < NQ_STEP) {
    const int qn = threadIdx.x;
    const bool mx = qn == 5 || qn == 6;
    double s = red8[qn][0];
#pragma unroll
    for (int q = 1; q < NT / 64; ++q) s = mx ? fmax(s, red8[qn][q]) : s + red8[qn][q];
    out[qn * m + blockIdx.x] = s;
  }
}

// mode 0: ledger reset from k_totals partials; mode 1: end of step from k_step partials
__global__ __launch_bounds__(NT) void k_ledger(const double* part, int n, double* scal, double vol, double area_dt,
                                               int mode) {
  __shared__ double red[NT / 64];
  if (mode == 0) {
    double O = sum_partials(part, n, red), H = sum_partials(part + n, n, red), X = sum_partials(part + 2 * n, n, red);
    if (threadIdx.x == 0) {
      scal[S_O0] = O * vol;
      scal[S_H0] = H * vol;
      scal[S_XO0] = X;
      scal[S_OOUT] = 0.0;
      scal[S_HOUT] = 0.0;
      scal[S_OTOT] = O * vol;
      scal[S_HTOT] = H * vol;
      scal[S_XOSUM] = X;
    }
    return;
  }
  // one pass over the eight partial arrays (the same per-thread order as
  // sum_partials, so the sums are unchanged), all loads of an index in flight together
  double O = 0.0, H = 0.0, X = 0.0, bo = 0.0, bh = 0.0, vm = 0.0, ep = 0.0, nf = 0.0;
#pragma unroll 8
  for (int q = threadIdx.x; q < n; q += NT) {
    O += part[q];
    H += part[n + q];
    X += part[2 * n + q];
    bo += part[3 * n + q];
    bh += part[4 * n + q];
    vm = fmax(vm, part[5 * n + q]);
    ep = fmax(ep, part[6 * n + q]);
    nf += part[7 * n + q];
  }
  O = block_sum(O, red);
  H = block_sum(H, red);
  X = block_sum(X, red);
  bo = block_sum(bo, red);
  bh = block_sum(bh, red);
  vm = block_max(vm, red);
  ep = block_max(ep, red);
  nf = block_sum(nf, red);
  if (threadIdx.x == 0) {
    scal[S_OOUT] += area_dt * bo;
    scal[S_HOUT] += area_dt * bh;
    scal[S_OTOT] = O * vol;
    scal[S_HTOT] = H * vol;
    scal[S_XOSUM] = X;
    scal[S_MAXVM] = vm;
    scal[S_MAXEP] = ep;
    scal[S_NONFIN] = nf;
  }
}

// ---------------------------------------------------------------------------
// Field exchange: FP64 compact <-> internal padded layout.
// The compact array has dims (cx, cy, cz); entries beyond the stored range
// (the high roller faces) are dropped on set and read as zero on get.
// `zero_axis` (0, 1, 2 or -1) forces the low roller face to zero on set.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_unpack(const double* src, T* dst, Grid g, int cx, int cy, int cz, int zero_axis) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = (long long)cx * cy * cz;
  if (t >= total) return;
  int ii = (int)(t % cx);
  long long rest = t / cx;
  int jj = (int)(rest % cy);
  int kk = (int)(rest / cy);
  if (ii >= g.nx || jj >= g.ny || kk >= g.nz) return;
  double v = src[t];
  if ((zero_axis == 0 && ii == 0) || (zero_axis == 1 && jj == 0) || (zero_axis == 2 && kk == 0)) v = 0.0;
  dst[gidx(g, ii, jj, kk)] = (T)v;
}

// FP32 pair form of the five fields: hi = the FP32 rounding of the value,
// lo = the FP32 rounding of the remainder (set), value = hi + lo (get).
__global__ void k_unpack_pair(const double* src, float* hi, float* lo, Grid g, int cx, int cy, int cz) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = (long long)cx * cy * cz;
  if (t >= total) return;
  int ii = (int)(t % cx);
  long long rest = t / cx;
  int jj = (int)(rest % cy);
  int kk = (int)(rest / cy);
  if (ii >= g.nx || jj >= g.ny || kk >= g.nz) return;
  const double v = src[t];
  const float h = (float)v;
  const int e = gidx(g, ii, jj, kk);
  hi[e] = h;
  lo[e] = (float)(v - (double)h);
}

__global__ void k_pack_pair(const float* hi, const float* lo, double* dst, Grid g, int cx, int cy, int cz) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = (long long)cx * cy * cz;
  if (t >= total) return;
  int ii = (int)(t % cx);
  long long rest = t / cx;
  int jj = (int)(rest % cy);
  int kk = (int)(rest / cy);
  double v = 0.0;
  if (ii < g.nx && jj < g.ny && kk < g.nz) {
    const int e = gidx(g, ii, jj, kk);
    v = (double)hi[e] + (double)lo[e];
  }
  dst[t] = v;
}

template <typename T>
__global__ void k_pack(const T* src, double* dst, Grid g, int cx, int cy, int cz) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = (long long)cx * cy * cz;
  if (t >= total) return;
  int ii = (int)(t % cx);
  long long rest = t / cx;
  int jj = (int)(rest % cy);
  int kk = (int)(rest / cy);
  double v = 0.0;
  if (ii < g.nx && jj < g.ny && kk < g.nz) v = (double)src[gidx(g, ii, jj, kk)];
  dst[t] = v;
}

}  // namespace pfk
