// Geometric multigrid V-cycle as the preconditioner of the equilibrium CG
// (the staggered small-strain operator of Eq. 29, momentum line, and Eq. 32).
//
// Level l + 1 has half the cells of level l along every axis (cell size 2h;
// an odd side of n cells gets (n + 1) / 2, the last covering one fine cell);
// its operator is the same staggered operator with the moduli K, G averaged
// over the children and its own Jacobi diagonal.  Transfers act on the
// face components: the prolongation takes, along the face normal, the
// coincident coarse face (weight 1) or the mean of the two coarse faces
// around a midway fine face, and across the normal interpolates linearly
// between coarse face centres (3/4, 1/4; constant at the walls); the
// restriction is its transpose divided by 4, which makes the coarse problem
// the Galerkin one up to the discretisation (the operator carries a factor
// 1/h, the energy h^(d-1)).  Smoothing is Jacobi with Chebyshev steps
// (k_apply3 in its APPLY_SMOOTH0 mode for the two sweeps from zero,
// APPLY_SMOOTH for the others); every sweep pair is the same polynomial in
// D^-1 A, pre- and post-smoothing take the same sweeps and the coarsest
// level a fixed number of sweeps from zero, so the V-cycle is a fixed
// symmetric positive definite operator, as CG needs.
#pragma once

#include <type_traits>

#include "pf_kernels.h"

namespace pfk {

template <typename T>
struct Vec3 {
  T* a[3];
};
template <typename T>
struct CVec3 {
  const T* a[3];
};

// bf16 copies (round to nearest even) of a coarse level's K, G and D^-1 for
// the FP32 sweeps, once per solve after the levels are set up (the set-up
// pass writes those of the solve's grid itself; the sweeps are
// bound by the bytes they move; the preconditioner only has to be a fixed
// symmetric positive definite operator, which these copies keep it)
struct MGLoCopy {
  const float* src[5];
  unsigned short* dst[5];
};
__global__ __launch_bounds__(NT) void k_mg_lo(MGLoCopy cp, int n) {
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT)
#pragma unroll
    for (int a = 0; a < 5; ++a) cp.dst[a][q] = bf16_rne(cp.src[a][q]);
}

// moduli of the coarse cells: the mean of their children (8; fewer in the
// last coarse cell along an odd side, which covers one fine cell there)
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_coarsen(Grid gf, Grid gc, const T* Kf, const T* Gf, T* Kc, T* Gc) {
  const long n = (long)gc.nx * gc.ny * gc.nz;
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT) {
    const int I = (int)(q % gc.nx);
    const long r = q / gc.nx;
    const int J = (int)(r % gc.ny), K = (int)(r / gc.ny);
    T sk = T(0), sg = T(0);
    int cnt = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int fi = 2 * I + (c & 1), fj = 2 * J + ((c >> 1) & 1), fk = 2 * K + (c >> 2);
      if (fi >= gf.nx || fj >= gf.ny || fk >= gf.nz) continue;
      const int e = gidx(gf, fi, fj, fk);
      sk += Kf[e];
      sg += Gf[e];
      ++cnt;
    }
    const int ec = gidx(gc, I, J, K);
    const T inv = cnt == 8 ? T(0.125) : T(1) / T(cnt);
    Kc[ec] = inv * sk;
    Gc[ec] = inv * sg;
  }
}

// transverse fine rows whose interpolation takes coarse row c (the transpose
// of the prolongation's rows f >> 1 at 3/4 and the neighbour on the side of
// f at 1/4, clamped at the walls): fine rows 2c - 1 .. 2c + 2 with weights
// 1/4, 3/4, 3/4, 1/4; at the low wall row 0 takes the full weight 1; at the
// high wall, the last row 2N - 1 of an even side likewise, and along an odd
// side (the last coarse cell covering one fine cell) rows beyond the fine
// grid get weight zero.  Indices are clamped into the grid.  Edge = false is
// for cells whose row 2c + 1 exists (every cell but the last one along an
// odd side): the rows 2c, 2c + 1 stay affine in c, which lets the compiler
// pair their loads along x.
template <typename T, bool Edge>
__device__ __forceinline__ void restrict_rows(int c, int N, int nf, int (&r)[4], T (&w)[4]) {
  r[0] = max(2 * c - 1, 0);
  r[1] = 2 * c;
  r[2] = Edge ? min(2 * c + 1, nf - 1) : 2 * c + 1;
  r[3] = min(2 * c + 2, nf - 1);
  w[0] = c > 0 ? T(0.25) : T(0);
  w[1] = c > 0 ? T(0.75) : T(1);
  w[2] = (!Edge || 2 * c + 1 < nf) ? (c < N - 1 ? T(0.75) : T(1)) : T(0);
  w[3] = 2 * c + 2 < nf ? T(0.25) : T(0);
}

// Jacobi inverse diagonal of a level from its moduli: per face, the
// M = K + 4G/3 of the two cells it separates and the edge moduli (mean of
// the 4 cells around an interior edge; boundary edges carry none) of the 4
// edges along it, times 1/h; zero on the roller faces.
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_diag(Grid g, T ih, const T* K, const T* G, Vec3<T> dinv) {
  const long n = (long)g.nx * g.ny * g.nz;
  auto Gc = [&](int i, int j, int k) { return G[gidx(g, i, j, k)]; };
  auto M = [&](int i, int j, int k) { const int e = gidx(g, i, j, k); return K[e] + T(4.0 / 3.0) * G[e]; };
  // edge moduli: the edge between cells (i-1, i) and (j-1, j) of plane k, etc.
  auto gxy = [&](int i, int j, int k) -> T {
    return (i > 0 && i < g.nx && j > 0 && j < g.ny)
               ? T(0.25) * (Gc(i - 1, j - 1, k) + Gc(i, j - 1, k) + Gc(i - 1, j, k) + Gc(i, j, k)) : T(0);
  };
  auto gxz = [&](int i, int j, int k) -> T {
    return (i > 0 && i < g.nx && k > 0 && k < g.nz)
               ? T(0.25) * (Gc(i - 1, j, k - 1) + Gc(i, j, k - 1) + Gc(i - 1, j, k) + Gc(i, j, k)) : T(0);
  };
  auto gyz = [&](int i, int j, int k) -> T {
    return (j > 0 && j < g.ny && k > 0 && k < g.nz)
               ? T(0.25) * (Gc(i, j - 1, k - 1) + Gc(i, j, k - 1) + Gc(i, j - 1, k) + Gc(i, j, k)) : T(0);
  };
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT) {
    const int i = (int)(q % g.nx);
    const long r = q / g.nx;
    const int j = (int)(r % g.ny), k = (int)(r / g.ny);
    const int e = gidx(g, i, j, k);
    const T d0 = i > 0 ? M(i - 1, j, k) + M(i, j, k) + gxy(i, j, k) + gxy(i, j + 1, k) + gxz(i, j, k) + gxz(i, j, k + 1) : T(0);
    const T d1 = j > 0 ? M(i, j - 1, k) + M(i, j, k) + gxy(i, j, k) + gxy(i + 1, j, k) + gyz(i, j, k) + gyz(i, j, k + 1) : T(0);
    const T d2 = k > 0 ? M(i, j, k - 1) + M(i, j, k) + gxz(i, j, k) + gxz(i + 1, j, k) + gyz(i, j, k) + gyz(i, j + 1, k) : T(0);
    dinv.a[0][e] = d0 > T(0) ? T(1) / (d0 * ih) : T(0);
    dinv.a[1][e] = d1 > T(0) ? T(1) / (d1 * ih) : T(0);
    dinv.a[2][e] = d2 > T(0) ? T(1) / (d2 * ih) : T(0);
  }
}

// The kernels applied per CG iteration take the solve's scalars and exit at
// entry once the solve has converged (launches queued past convergence).

// The transfers run one thread per cell (its three faces), in the
// precision of the level's vectors, with no branch around a load (indices
// clamped or range-checked, weights zero where a term does not exist) so
// that a thread's loads issue together.  (Staging a block's tile in LDS was
// tried: with the little work per cell, the block-wide wait between the
// loads and the sums made both transfers slower.)

// fine += P coarse.  Per face component d: along the normal the coincident
// coarse face (weight 1) or the two coarse faces around a midway fine face
// (1/2 each; the high wall holds zero and the low roller face is zero);
// across it, per transverse axis, coarse rows f >> 1 (3/4) and its
// neighbour on the side of f (1/4; clamped at the walls).  One thread takes
// the fine x pair 2i, 2i + 1 (the last alone along an odd side): both lie
// over coarse column i and share their y and z rows, so the pair needs the
// coarse columns i - 1, i, i + 1 once (32 coarse loads instead of 48), and
// its fine values are read and written as pairs.  All sums are formed
// before the stores, so no coarse load waits behind a fine store it might
// alias.
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_prolong(Grid gf, Grid gc, CVec3<T> xc, Vec3<T> xf, const double* scal) {
  if (scal[S_CONV] != 0.0) return;
  const int hx = (gf.nx + 1) >> 1;
  const long q = (long)blockIdx.x * NT + threadIdx.x;
  if (q >= (long)hx * gf.ny * gf.nz) return;
  const int i = (int)(q % hx);
  const int f[3] = {2 * i, (int)((q / hx) % gf.ny), (int)(q / ((long)hx * gf.ny))};
  const bool two = 2 * i + 1 < gf.nx;            // the pair's second cell exists
  const int nc[3] = {gc.nx, gc.ny, gc.nz};
  const int cx[3] = {max(i - 1, 0), i, min(i + 1, nc[0] - 1)};
  int t0[3], t1[3];                              // y and z transverse rows
#pragma unroll
  for (int a = 1; a < 3; ++a) {
    t0[a] = f[a] >> 1;
    t1[a] = (f[a] & 1) ? min(t0[a] + 1, nc[a] - 1) : max(t0[a] - 1, 0);
  }
  const T tw[2] = {T(0.75), T(0.25)};
  // normal weights of the coarse faces a0 = f >> 1 and a0 + 1 (y and z)
  auto normal = [&](int a, T (&wn)[2], int (&an)[2]) {
    const int a0 = f[a] >> 1;
    const bool odd = f[a] & 1;
    wn[0] = a0 > 0 ? (odd ? T(0.5) : T(1)) : T(0);
    wn[1] = (odd && a0 + 1 < nc[a]) ? T(0.5) : T(0);
    an[0] = a0;
    an[1] = min(a0 + 1, nc[a] - 1);
  };
  T s0[3], s1[3];                                // sums of the cells 2i and 2i + 1
  {                                              // d = 0: x is the normal
    T v0 = T(0), v1 = T(0);                      // columns i and i + 1 over the y, z rows
    const int ry[2] = {t0[1], t1[1]}, rz[2] = {t0[2], t1[2]};
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int ic = 0; ic < 2; ++ic) {
        const T w = tw[ib] * tw[ic];
        v0 += w * xc.a[0][gidx(gc, cx[1], ry[ib], rz[ic])];
        v1 += w * xc.a[0][gidx(gc, cx[2], ry[ib], rz[ic])];
      }
    s0[0] = i > 0 ? v0 : T(0);                   // coincident face i (face 0 is the roller)
    s1[0] = (i > 0 ? T(0.5) * v0 : T(0)) + (i + 1 < nc[0] ? T(0.5) * v1 : T(0));
  }
#pragma unroll
  for (int d = 1; d < 3; ++d) {                  // x transverse: 2i takes i, i - 1; 2i + 1 takes i, i + 1
    const int o = 3 - d;                         // the other transverse axis
    T wn[2];
    int an[2];
    normal(d, wn, an);
    const int ro[2] = {t0[o], t1[o]};
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
      for (int ic = 0; ic < 2; ++ic) {
        int idx[3];
        idx[d] = an[ia];
        idx[o] = ro[ic];
        const T w = wn[ia] * tw[ic];
        idx[0] = cx[0];
        const T xm = xc.a[d][gidx(gc, idx[0], idx[1], idx[2])];
        idx[0] = cx[1];
        const T x0 = xc.a[d][gidx(gc, idx[0], idx[1], idx[2])];
        idx[0] = cx[2];
        const T xp = xc.a[d][gidx(gc, idx[0], idx[1], idx[2])];
        a0 += w * (tw[0] * x0 + tw[1] * xm);
        a1 += w * (tw[0] * x0 + tw[1] * xp);
      }
    s0[d] = a0;
    s1[d] = a1;
  }
  // fine values; the second of a lone last cell reads the row's padding
  // (the pitch exceeds an odd side) and is not written back
  const int e = gidx(gf, f[0], f[1], f[2]);
  using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
  T o0[3], o1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    o0[d] = xf.a[d][e];
    o1[d] = xf.a[d][e + 1];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d > 0 && f[d] == 0) continue;            // roller face: left as it is (d = 0 sums to zero there)
    if (two) {                                   // one paired store (e is even, rows start aligned)
      V2 v;
      v.x = o0[d] + s0[d];
      v.y = o1[d] + s1[d];
      *reinterpret_cast<V2*>(xf.a[d] + e) = v;
    } else {
      xf.a[d][e] = o0[d] + s0[d];
    }
  }
}

// coarse b = R fine r = P^T r / 4, one coarse cell per thread.  Per face
// component d (the roller face C = 0 gets zero): along the normal fine
// faces 2C - 1, 2C, 2C + 1 (1/2, 1, 1/2; the last is the fine high wall,
// not stored and zero, at the end of an odd side); per transverse axis the
// fine rows whose interpolation takes coarse row C, 2C - 1 .. 2C + 2 with
// weights 1/4, 3/4, 3/4, 1/4 (at a wall the row beyond is absent and the
// clamped interpolation gives the row at the wall the full weight 1; along an
// odd side the rows past the fine grid of the last coarse cell weigh zero).
// A zero weight marks exactly the rows outside the fine grid.  The 48 fine
// values per component are raw buffer loads (one 32-bit offset register
// each, so the compiler keeps them all in flight): a (y, z) row outside the
// grid gets an out-of-range offset and reads zero without touching memory,
// and the x neighbours are immediate offsets from the row's first value, the
// ones outside the grid zeroed by their weight's select.
template <typename T>
__device__ __forceinline__ void restrict3_cell(const Grid& gf, const Grid& gc, const CVec3<T>& rf, const Vec3<T>& bc,
                                               const int (&C)[3]) {
  const int nc[3] = {gc.nx, gc.ny, gc.nz};
  const int nf[3] = {gf.nx, gf.ny, gf.nz};
  const int st[3] = {(int)sizeof(T), gf.px * (int)sizeof(T), gf.px * gf.ny * (int)sizeof(T)};
  const int nbytes = gf.n * (int)sizeof(T);
  T w[3][4];                                     // transverse weights of rows 2C - 1 .. 2C + 2 per axis
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int c = C[a], N = nc[a], n = nf[a];
    w[a][0] = c > 0 ? T(0.25) : T(0);
    w[a][1] = c > 0 ? T(0.75) : T(1);
    w[a][2] = 2 * c + 1 < n ? (c < N - 1 ? T(0.75) : T(1)) : T(0);
    w[a][3] = 2 * c + 2 < n ? T(0.25) : T(0);
  }
  const int ec = gidx(gc, C[0], C[1], C[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (C[d] == 0) {                             // roller face
      bc.a[d][ec] = T(0);
      continue;
    }
    T wt[3][4];                                  // weights per axis from fine index 2C - 1 on
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o < 4; ++o)
        wt[a][o] = a != d ? w[a][o]
                          : (o == 0 ? T(0.5) : o == 1 ? T(1) : o == 2 && 2 * C[d] + 1 < nf[d] ? T(0.5) : T(0));
    const int cnt[3] = {d == 0 ? 3 : 4, d == 1 ? 3 : 4, d == 2 ? 3 : 4};
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(rf.a[d], nbytes);
    const int x0 = (2 * C[0] - 1) * st[0];
    T s = T(0);
#pragma unroll
    for (int oc = 0; oc < cnt[2]; ++oc)
#pragma unroll
      for (int ob = 0; ob < cnt[1]; ++ob) {
        const int ro = wt[1][ob] != T(0) && wt[2][oc] != T(0)
                           ? x0 + (2 * C[1] - 1 + ob) * st[1] + (2 * C[2] - 1 + oc) * st[2]
                           : kOutOfRange;
        T sx = T(0);
#pragma unroll
        for (int oa = 0; oa < cnt[0]; ++oa) {
          const T v = buf_ld<T>(rs, ro + oa * st[0]);
          sx += wt[0][oa] != T(0) ? wt[0][oa] * v : T(0);
        }
        s += wt[1][ob] * wt[2][oc] * sx;
      }
    bc.a[d][ec] = T(0.25) * s;
  }
}

// one coarse cell per thread; the occupancy target of at most 6 waves per
// SIMD lets the scheduler keep a component's loads in flight together (at
// the default target of 8 it issues them one at a time)
template <typename T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, sizeof(T) == 4 ? 6 : 4))) void k_mg_restrict(Grid gf, Grid gc, CVec3<T> rf, Vec3<T> bc, const double* scal) {
  if (scal[S_CONV] != 0.0) return;
  const long q = (long)blockIdx.x * NT + threadIdx.x;
  if (q >= (long)gc.nx * gc.ny * gc.nz) return;
  const int C[3] = {(int)(q % gc.nx), (int)((q / gc.nx) % gc.ny), (int)(q / ((long)gc.nx * gc.ny))};
  restrict3_cell<T>(gf, gc, rf, bc, C);
}

// ---------------------------------------------------------------------------
// The coarsest 3D level's sweeps in one block: at 8^3 each of its 7 launches
// (the pass from zero and 6 sweeps) costs about 5 us whatever its work, so a
// level of at most kCoarseLdsCells cells (FP32; half as many in FP64) is
// staged in LDS (b, K, G, D^-1 and two iterates, compact x-fastest) and
// swept there, a block barrier between sweeps.  The steps are those of the
// launch path (s0 D^-1 b, then alternately s1 and s0); the operator is the
// apply kernel's staggered one, from the level's FP32 moduli (every sweep of
// the level is here, so the level applies one operator): per sweep the cell
// and edge stresses once, then the forces on the faces, a barrier between.
// ---------------------------------------------------------------------------
constexpr int kCoarseNT = 1024;
constexpr int kCoarseLdsCells = 1536;

template <typename T>
struct CoarseArgs {
  Grid g;
  T ih;
  const T* K;
  const T* G;
  const T* b[3];
  const T* dinv[3];
  T* x[3];                 // out: the level's iterate after the sweeps
  T s0, s1;
  int sweeps;              // even, at least 2
  const double* scal;
};

template <typename T>
__global__ __launch_bounds__(kCoarseNT) void k_mg_coarse3(CoarseArgs<T> a) {
  if (a.scal[S_CONV] != 0.0) return;
  constexpr int NMAX = kCoarseLdsCells * 4 / (int)sizeof(T);
  // moduli, b, D^-1, two iterates; per sweep the cell normal stresses and the
  // shear stresses of the edges at each cell's low corner
  __shared__ T sK[NMAX], sG[NMAX], sb[3][NMAX], sd[3][NMAX], sx[2][3][NMAX], sn[3][NMAX], se[3][NMAX];
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz, n = nx * ny * nz;
  const T ih = a.ih;
  for (int q = threadIdx.x; q < n; q += kCoarseNT) {
    const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
    const int e = gidx(a.g, i, j, k);
    sK[q] = a.K[e];
    sG[q] = a.G[e];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sb[d][q] = a.b[d][e];
      sd[d][q] = a.dinv[d][e];
      sx[0][d][q] = a.s0 * a.dinv[d][e] * a.b[d][e];   // the first sweep from zero
    }
  }
  __syncthreads();
  const int sy = nx, sz = nx * ny;                 // compact strides
  // one sweep src -> dst: x + omega D^-1 (b - A x) at every face
  auto sweep = [&](int src, int dst, T om) {
    const T* X0 = sx[src][0];
    const T* X1 = sx[src][1];
    const T* X2 = sx[src][2];
    // (a) per cell: its normal stresses, and the shear stresses of the three
    // edges at its low corner (zero on the boundary); x beyond a high wall is 0
    for (int q = threadIdx.x; q < n; q += kCoarseNT) {
      const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
      const T x0 = X0[q], x1 = X1[q], x2 = X2[q];
      const T exx = ((i + 1 < nx ? X0[q + 1] : T(0)) - x0) * ih;
      const T eyy = ((j + 1 < ny ? X1[q + sy] : T(0)) - x1) * ih;
      const T ezz = ((k + 1 < nz ? X2[q + sz] : T(0)) - x2) * ih;
      const T tr = exx + eyy + ezz;
      const T G2 = T(2) * sG[q];
      const T lam = sK[q] * tr - G2 * tr * T(1.0 / 3.0);
      sn[0][q] = lam + G2 * exx;
      sn[1][q] = lam + G2 * eyy;
      sn[2][q] = lam + G2 * ezz;
      T exy = T(0), exz = T(0), eyz = T(0);
      if (i > 0 && j > 0) {
        const T ge = T(0.25) * (sG[q - 1 - sy] + sG[q - sy] + sG[q - 1] + sG[q]);
        exy = ge * ((x0 - X0[q - sy]) + (x1 - X1[q - 1])) * ih;
      }
      if (i > 0 && k > 0) {
        const T ge = T(0.25) * (sG[q - 1 - sz] + sG[q - sz] + sG[q - 1] + sG[q]);
        exz = ge * ((x0 - X0[q - sz]) + (x2 - X2[q - 1])) * ih;
      }
      if (j > 0 && k > 0) {
        const T ge = T(0.25) * (sG[q - sy - sz] + sG[q - sz] + sG[q - sy] + sG[q]);
        eyz = ge * ((x1 - X1[q - sz]) + (x2 - X2[q - sy])) * ih;
      }
      se[0][q] = exy;
      se[1][q] = exz;
      se[2][q] = eyz;
    }
    __syncthreads();
    // (b) per face: the divergence of the stresses (roller faces i, j, k = 0
    // get zero; the edges past the high walls carry none)
    for (int q = threadIdx.x; q < n; q += kCoarseNT) {
      const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
      const T exy = se[0][q], exz = se[1][q], eyz = se[2][q];
      T qv[3] = {T(0), T(0), T(0)};
      if (i > 0)
        qv[0] = sn[0][q - 1] - sn[0][q] + exy - (j + 1 < ny ? se[0][q + sy] : T(0)) + exz -
                (k + 1 < nz ? se[1][q + sz] : T(0));
      if (j > 0)
        qv[1] = sn[1][q - sy] - sn[1][q] + exy - (i + 1 < nx ? se[0][q + 1] : T(0)) + eyz -
                (k + 1 < nz ? se[2][q + sz] : T(0));
      if (k > 0)
        qv[2] = sn[2][q - sz] - sn[2][q] + exz - (i + 1 < nx ? se[1][q + 1] : T(0)) + eyz -
                (j + 1 < ny ? se[2][q + sy] : T(0));
#pragma unroll
      for (int d = 0; d < 3; ++d) sx[dst][d][q] = sx[src][d][q] + om * sd[d][q] * (sb[d][q] - qv[d]);
    }
    __syncthreads();
  };
  // sweep 0 (from zero) was formed while staging; sweeps 1 .. n - 1
  // alternate the steps s1, s0, s1, ...
  int cur = 0;
  for (int s = 1; s < a.sweeps; ++s) {
    sweep(cur, cur ^ 1, (s & 1) ? a.s1 : a.s0);
    cur ^= 1;
  }
  for (int q = threadIdx.x; q < n; q += kCoarseNT) {
    const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
    const int e = gidx(a.g, i, j, k);
#pragma unroll
    for (int d = 0; d < 3; ++d) a.x[d][e] = sx[cur][d][q];
  }
}

// ---------------------------------------------------------------------------
// 2D (plane strain) levels: the same construction with two face components,
// one transverse axis per component, and the restriction the transposed
// prolongation divided by 2 (the operator carries 1/h, the energy h).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_coarsen2(Grid gf, Grid gc, const T* Kf, const T* Gf, T* Kc, T* Gc) {
  const long n = (long)gc.nx * gc.ny;
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT) {
    const int I = (int)(q % gc.nx), J = (int)(q / gc.nx);
    T sk = T(0), sg = T(0);
    int cnt = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int fi = 2 * I + (c & 1), fj = 2 * J + (c >> 1);
      if (fi >= gf.nx || fj >= gf.ny) continue;
      const int e = gidx(gf, fi, fj, 0);
      sk += Kf[e];
      sg += Gf[e];
      ++cnt;
    }
    const int ec = gidx(gc, I, J, 0);
    const T inv = cnt == 4 ? T(0.25) : T(1) / T(cnt);
    Kc[ec] = inv * sk;
    Gc[ec] = inv * sg;
  }
}

// Jacobi inverse diagonal of a 2D level: per face, the M of the two cells it
// separates and the moduli of the 2 interior nodes at its ends, times 1/h
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_diag2(Grid g, T ih, const T* K, const T* G, Vec3<T> dinv) {
  const long n = (long)g.nx * g.ny;
  auto Gc = [&](int i, int j) { return G[gidx(g, i, j, 0)]; };
  auto M = [&](int i, int j) { const int e = gidx(g, i, j, 0); return K[e] + T(4.0 / 3.0) * G[e]; };
  auto gxy = [&](int i, int j) -> T {
    return (i > 0 && i < g.nx && j > 0 && j < g.ny)
               ? T(0.25) * (Gc(i - 1, j - 1) + Gc(i, j - 1) + Gc(i - 1, j) + Gc(i, j)) : T(0);
  };
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT) {
    const int i = (int)(q % g.nx), j = (int)(q / g.nx);
    const int e = gidx(g, i, j, 0);
    const T d0 = i > 0 ? M(i - 1, j) + M(i, j) + gxy(i, j) + gxy(i, j + 1) : T(0);
    const T d1 = j > 0 ? M(i, j - 1) + M(i, j) + gxy(i, j) + gxy(i + 1, j) : T(0);
    dinv.a[0][e] = d0 > T(0) ? T(1) / (d0 * ih) : T(0);
    dinv.a[1][e] = d1 > T(0) ? T(1) / (d1 * ih) : T(0);
  }
}

// fine += P coarse at fine cell (f0, f1) (2D)
template <typename T>
__device__ __forceinline__ void prolong2_cell(const Grid& gf, const Grid& gc, const T* const* xc, T* const* xf, int f0,
                                              int f1) {
  const int f[2] = {f0, f1};
  const int nc[2] = {gc.nx, gc.ny};
  int t0[2], t1[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    t0[a] = f[a] >> 1;
    t1[a] = (f[a] & 1) ? min(t0[a] + 1, nc[a] - 1) : max(t0[a] - 1, 0);
  }
  const T tw[2] = {T(0.75), T(0.25)};
  const int e = gidx(gf, f[0], f[1], 0);
  T s[2];                                        // both sums before the stores, as in 3D
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const int a0 = f[d] >> 1;
    const bool odd = f[d] & 1;
    const int a1 = min(a0 + 1, nc[d] - 1);
    const T wn[2] = {a0 > 0 ? (odd ? T(0.5) : T(1)) : T(0), (odd && a0 + 1 < nc[d]) ? T(0.5) : T(0)};
    const int an[2] = {a0, a1};
    const int u = 1 - d;
    const int ru[2] = {t0[u], t1[u]};
    s[d] = T(0);
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) {
        int idx[2];
        idx[d] = an[ia];
        idx[u] = ru[ib];
        s[d] += wn[ia] * tw[ib] * xc[d][gidx(gc, idx[0], idx[1], 0)];
      }
  }
  T o[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) o[d] = xf[d][e];
#pragma unroll
  for (int d = 0; d < 2; ++d)
    if (f[d] != 0) xf[d][e] = o[d] + s[d];     // the roller face f = 0 is left as it is
}

// coarse b = P^T r / 2 at coarse cell (c0, c1) (2D)
template <typename T, bool Edge>
__device__ __forceinline__ void restrict2_cell(const Grid& gf, const Grid& gc, const T* const* rf, T* const* bc, int c0,
                                               int c1) {
  const int C[2] = {c0, c1};
  const int nc[2] = {gc.nx, gc.ny};
  const int nf[2] = {gf.nx, gf.ny};
  int rows[2][4];
  T w[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a) restrict_rows<T, Edge>(C[a], nc[a], nf[a], rows[a], w[a]);
  const T wn[3] = {T(0.5), T(1), T(0.5)};
  const int ec = gidx(gc, C[0], C[1], 0);
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    if (C[d] == 0) {                             // roller face
      bc[d][ec] = T(0);
      continue;
    }
    const int u = 1 - d;
    // along the normal: the last is the fine high wall at the end of an odd side
    const int fn[3] = {2 * C[d] - 1, 2 * C[d], Edge ? min(2 * C[d] + 1, nf[d] - 1) : 2 * C[d] + 1};
    const T wa[3] = {wn[0], wn[1], (!Edge || 2 * C[d] + 1 < nf[d]) ? wn[2] : T(0)};
    T s = T(0);
#pragma unroll
    for (int sa = 0; sa < 3; ++sa)
#pragma unroll
      for (int ob = 0; ob < 4; ++ob) {
        int idx[2];
        idx[d] = fn[sa];
        idx[u] = rows[u][ob];
        s += wa[sa] * w[u][ob] * rf[d][gidx(gf, idx[0], idx[1], 0)];
      }
    bc[d][ec] = T(0.5) * s;
  }
}

// the 2D cell with the clamped rows only where they are needed
template <typename T>
__device__ __forceinline__ void restrict2_at(const Grid& gf, const Grid& gc, const T* const* rf, T* const* bc, int c0,
                                             int c1) {
  if (2 * c0 + 1 >= gf.nx || 2 * c1 + 1 >= gf.ny)
    restrict2_cell<T, true>(gf, gc, rf, bc, c0, c1);
  else
    restrict2_cell<T, false>(gf, gc, rf, bc, c0, c1);
}

// fine += P coarse, one fine cell per thread (2D)
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_prolong2(Grid gf, Grid gc, CVec3<T> xc, Vec3<T> xf, const double* scal) {
  if (scal[S_CONV] != 0.0) return;
  const long q = (long)blockIdx.x * NT + threadIdx.x;
  if (q >= (long)gf.nx * gf.ny) return;
  prolong2_cell<T>(gf, gc, xc.a, xf.a, (int)(q % gf.nx), (int)(q / gf.nx));
}

// coarse b = P^T r / 2, one coarse cell per thread (2D)
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_restrict2(Grid gf, Grid gc, CVec3<T> rf, Vec3<T> bc, const double* scal) {
  if (scal[S_CONV] != 0.0) return;
  const long q = (long)blockIdx.x * NT + threadIdx.x;
  if (q >= (long)gc.nx * gc.ny) return;
  restrict2_at<T>(gf, gc, rf.a, bc.a, (int)(q % gc.nx), (int)(q / gc.nx));
}

// ---------------------------------------------------------------------------
// The small 2D levels in one launch: below about a thousand cells a level's
// kernels are launch-bound (about 6 us each, some 20 of them per cycle at
// 2048^2), so one block of 1024 threads runs the whole V-cycle from the
// first such level down and back, each step a loop over the level's cells
// and a block barrier.  The steps, their order and the Chebyshev steps are
// those of the launch-per-step cycle; the operator is the staggered one of
// the apply kernels evaluated per face from global memory (the level's
// vectors stay in the caches).
// ---------------------------------------------------------------------------
constexpr int kTailNT = 1024;
constexpr int kTailMax = 6;
constexpr int kTailCells = 1024;            // levels with at most this many cells go into the tail

template <typename T>
struct MGTailLevel {
  Grid g;
  T ih;
  const T* K;
  const T* G;
  const T* dinv[2];
  const T* b[2];
  T* bw[2];                                      // b of levels after the first (written by the restriction)
  T* x[2];
  T* xt[2];
  T* r[2];
};

template <typename T>
struct MGTailArgs {
  MGTailLevel<T> lv[kTailMax];
  int n;                                         // levels (the last one is the coarsest)
  T s0, s1;                                      // the Chebyshev steps of a sweep pair
  int coarse_sweeps;                             // even
  const double* scal;
};

// q = A u at the two faces of cell (i, j) of a 2D level (the stencil of
// k_apply2: sigma from the face displacements, q0 = sxx(i-1) - sxx(i) +
// sxy(i, j) - sxy(i, j+1), q1 = syy(j-1) - syy(j) + sxy(i, j) - sxy(i+1, j);
// roller faces (i = 0, j = 0) get zero; the high walls hold zero)
template <typename T>
__device__ __forceinline__ void cell_apply2(const MGTailLevel<T>& L, const T* ux, const T* uy, int i, int j, T& q0,
                                            T& q1) {
  const Grid& g = L.g;
  const T ih = L.ih;
  auto X = [&](int ii, int jj) -> T { return (ii < g.nx && jj < g.ny) ? ux[jj * g.px + ii] : T(0); };
  auto Y = [&](int ii, int jj) -> T { return (ii < g.nx && jj < g.ny) ? uy[jj * g.px + ii] : T(0); };
  auto Gc = [&](int ii, int jj) -> T { return L.G[jj * g.px + ii]; };
  auto snn = [&](int ii, int jj, T& sxx, T& syy) {
    const T exx = (X(ii + 1, jj) - X(ii, jj)) * ih;
    const T eyy = (Y(ii, jj + 1) - Y(ii, jj)) * ih;
    const T tr = exx + eyy;
    const T G2 = T(2) * Gc(ii, jj);
    const T lam = L.K[jj * g.px + ii] * tr - G2 * tr * T(1.0 / 3.0);
    sxx = lam + G2 * exx;
    syy = lam + G2 * eyy;
  };
  auto sxy = [&](int ii, int jj) -> T {
    if (!(ii > 0 && ii < g.nx && jj > 0 && jj < g.ny)) return T(0);
    const T ge = T(0.25) * (Gc(ii - 1, jj - 1) + Gc(ii, jj - 1) + Gc(ii - 1, jj) + Gc(ii, jj));
    return ge * ((X(ii, jj) - X(ii, jj - 1)) + (Y(ii, jj) - Y(ii - 1, jj))) * ih;
  };
  T sxx, syy;
  snn(i, j, sxx, syy);
  const T sxy0 = sxy(i, j);
  q0 = T(0);
  q1 = T(0);
  if (i > 0) {
    T lxx, lyy;
    snn(i - 1, j, lxx, lyy);
    q0 = lxx - sxx + sxy0 - sxy(i, j + 1);
  }
  if (j > 0) {
    T bxx, byy;
    snn(i, j - 1, bxx, byy);
    q1 = byy - syy + sxy0 - sxy(i + 1, j);
  }
}

template <typename T>
__global__ __launch_bounds__(kTailNT) void k_mg_tail2(const MGTailArgs<T>* ap) {
  const MGTailArgs<T>& a = *ap;
  if (a.scal[S_CONV] != 0.0) return;
  // writes of one step become visible to the whole block at the barrier
  auto sync = [] {
    __threadfence_block();
    __syncthreads();
  };
  // xt = s0 D^-1 b (the first sweep from zero)
  auto jac0 = [&](const MGTailLevel<T>& L) {
    const int n = L.g.nx * L.g.ny;
    for (int q = threadIdx.x; q < n; q += kTailNT) {
      const int e = (q / L.g.nx) * L.g.px + q % L.g.nx;
#pragma unroll
      for (int d = 0; d < 2; ++d) L.xt[d][e] = a.s0 * L.dinv[d][e] * L.b[d][e];
    }
    sync();
  };
  // out = in + step D^-1 (b - A in), or with resid the residual b - A in
  auto sweep = [&](const MGTailLevel<T>& L, T* const* in, T* const* out, T step, bool resid) {
    const int n = L.g.nx * L.g.ny;
    for (int q = threadIdx.x; q < n; q += kTailNT) {
      const int i = q % L.g.nx, j = q / L.g.nx;
      T q0, q1;
      cell_apply2(L, in[0], in[1], i, j, q0, q1);
      const int e = j * L.g.px + i;
      const T qv[2] = {q0, q1};
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const T r = L.b[d][e] - qv[d];
        out[d][e] = resid ? r : in[d][e] + step * L.dinv[d][e] * r;
      }
    }
    sync();
  };
  const int last = a.n - 1;
  for (int l = 0; l < last; ++l) {               // down: two sweeps from zero, residual, restriction
    const MGTailLevel<T>& L = a.lv[l];
    jac0(L);
    sweep(L, L.xt, L.x, a.s1, false);
    sweep(L, L.x, L.r, T(0), true);
    const MGTailLevel<T>& C = a.lv[l + 1];
    const int nc = C.g.nx * C.g.ny;
    for (int q = threadIdx.x; q < nc; q += kTailNT)
      restrict2_at<T>(L.g, C.g, (const T* const*)L.r, C.bw, q % C.g.nx, q / C.g.nx);
    sync();
  }
  {                                              // the coarsest level: sweeps from zero
    const MGTailLevel<T>& L = a.lv[last];
    jac0(L);
    sweep(L, L.xt, L.x, a.s1, false);
    for (int s = 2; s < a.coarse_sweeps; ++s) {
      if (s & 1) sweep(L, L.xt, L.x, a.s1, false);
      else sweep(L, L.x, L.xt, a.s0, false);
    }
  }
  for (int l = last - 1; l >= 0; --l) {          // up: prolongation, two sweeps
    const MGTailLevel<T>& L = a.lv[l];
    const MGTailLevel<T>& C = a.lv[l + 1];
    const int nf = L.g.nx * L.g.ny;
    for (int q = threadIdx.x; q < nf; q += kTailNT)
      prolong2_cell<T>(L.g, C.g, (const T* const*)C.x, L.x, q % L.g.nx, q / L.g.nx);
    sync();
    sweep(L, L.x, L.xt, a.s0, false);
    sweep(L, L.xt, L.x, a.s1, false);
  }
}

// r.z of the preconditioned residual for the next CG apply: the fixed-order
// sum of the V-cycle's partials into slot 0 of the r.z section, zeros in the
// other n_rz - 1 slots (the r.r section after them is left alone)
__global__ __launch_bounds__(NT) void k_mg_rz(const double* part, int n, double* out, int n_rz, const double* scal) {
  if (scal[S_CONV] != 0.0) return;
  __shared__ double red[NT / 64];
  const double s = sum_partials(part, n, red);
  for (int q = threadIdx.x; q < n_rz; q += NT) out[q] = q == 0 ? s : 0.0;
}

}  // namespace pfk
