// Geometric multigrid V-cycle as the preconditioner of the 3D equilibrium CG
// (the staggered small-strain operator of Eq. 29, momentum line, and Eq. 32).
//
// Level l + 1 has half the cells of level l along every axis (cell size 2h);
// its operator is the same staggered operator with the moduli K, G averaged
// over the 8 children and its own Jacobi diagonal.  Transfers act on the
// face components: the prolongation takes, along the face normal, the
// coincident coarse face (weight 1) or the mean of the two coarse faces
// around a midway fine face, and across the normal interpolates linearly
// between coarse face centres (3/4, 1/4; constant at the walls); the
// restriction is its transpose divided by 4, which makes the coarse problem
// the Galerkin one up to the discretisation (the operator carries a factor
// 1/h, the energy h^(d-1)).  Smoothing is damped Jacobi (k_apply3 in its
// APPLY_SMOOTH0 mode for the two sweeps from zero, APPLY_SMOOTH for the
// others); pre- and post-smoothing take the same sweeps and the coarsest
// level a fixed number of sweeps from zero, so the V-cycle is a fixed
// symmetric positive definite operator, as CG needs.
#pragma once

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

// moduli of the coarse cells: the mean of their 8 children
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_coarsen(Grid gf, Grid gc, const T* Kf, const T* Gf, T* Kc, T* Gc) {
  const long n = (long)gc.nx * gc.ny * gc.nz;
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT) {
    const int I = (int)(q % gc.nx);
    const long r = q / gc.nx;
    const int J = (int)(r % gc.ny), K = (int)(r / gc.ny);
    T sk = T(0), sg = T(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int e = gidx(gf, 2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2));
      sk += Kf[e];
      sg += Gf[e];
    }
    const int ec = gidx(gc, I, J, K);
    Kc[ec] = T(0.125) * sk;
    Gc[ec] = T(0.125) * sg;
  }
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

// weights of the transverse interpolation (fine index f of a coarse row of
// N faces): fine 2J = 3/4 c[J] + 1/4 c[J-1], fine 2J+1 = 3/4 c[J] + 1/4 c[J+1],
// with c[-1] = c[0] and c[N] = c[N-1]
__device__ __forceinline__ void lin_up(int f, int N, int& J0, int& J1, float& w0, float& w1) {
  const int J = f >> 1;
  J0 = J;
  w0 = 0.75f;
  J1 = (f & 1) ? (J + 1 < N ? J + 1 : J) : (J > 0 ? J - 1 : J);
  w1 = 0.25f;
}

// fine += P coarse, one fine cell (its three faces) per thread
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_prolong(Grid gf, Grid gc, CVec3<T> xc, Vec3<T> xf, const double* scal) {
  if (scal[S_CONV] != 0.0) return;
  const long n = (long)gf.nx * gf.ny * gf.nz;
  const int nc[3] = {gc.nx, gc.ny, gc.nz};
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT) {
    const int f[3] = {(int)(q % gf.nx), (int)((q / gf.nx) % gf.ny), (int)(q / ((long)gf.nx * gf.ny))};
    const int e = gidx(gf, f[0], f[1], f[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (f[d] == 0) continue;                 // roller face
      // along the normal d
      int a0 = f[d] >> 1, a1 = a0;
      float wa0 = 1.f, wa1 = 0.f;
      if (f[d] & 1) { a1 = a0 + 1; wa0 = 0.5f; wa1 = 0.5f; }
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      int b0, b1, c0, c1;
      float wb0, wb1, wc0, wc1;
      lin_up(f[t1], nc[t1], b0, b1, wb0, wb1);
      lin_up(f[t2], nc[t2], c0, c1, wc0, wc1);
      double s = 0.0;
      const int an[2] = {a0, a1};
      const float wan[2] = {wa0, wa1};
#pragma unroll
      for (int ia = 0; ia < 2; ++ia) {
        const int A = an[ia];
        if (wan[ia] == 0.f || A <= 0 || A >= nc[d]) continue;   // roller faces of the coarse level
        const int bb[2] = {b0, b1}, cc[2] = {c0, c1};
        const float wb[2] = {wb0, wb1}, wc[2] = {wc0, wc1};
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int ic = 0; ic < 2; ++ic) {
            int idx[3];
            idx[d] = A;
            idx[t1] = bb[ib];
            idx[t2] = cc[ic];
            s += (double)(wan[ia] * wb[ib] * wc[ic]) * (double)xc.a[d][gidx(gc, idx[0], idx[1], idx[2])];
          }
      }
      xf.a[d][e] += (T)s;
    }
  }
}

// coarse b = R fine r = P^T r / 4, one coarse cell (its three faces) per thread
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_restrict(Grid gf, Grid gc, CVec3<T> rf, Vec3<T> bc, const double* scal) {
  if (scal[S_CONV] != 0.0) return;
  const long n = (long)gc.nx * gc.ny * gc.nz;
  const int nf[3] = {gf.nx, gf.ny, gf.nz};
  const int nc[3] = {gc.nx, gc.ny, gc.nz};
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < n; q += (long)gridDim.x * NT) {
    const int C[3] = {(int)(q % gc.nx), (int)((q / gc.nx) % gc.ny), (int)(q / ((long)gc.nx * gc.ny))};
    const int ec = gidx(gc, C[0], C[1], C[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (C[d] == 0) {                          // roller face
        bc.a[d][ec] = T(0);
        continue;
      }
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      // transverse: the fine rows whose interpolation uses coarse row C[t]
      // (the transpose of lin_up), fine indices 2C-1 .. 2C+2
      auto tw = [&](int t, int off, float& w) -> int {   // off in 0..3 -> fine 2C-1+off
        const int fi = 2 * C[t] - 1 + off;
        const int N = nc[t];
        w = 0.f;
        if (off == 1) w = 0.75f + (C[t] == 0 ? 0.25f : 0.f);
        else if (off == 2) w = 0.75f + (C[t] == N - 1 ? 0.25f : 0.f);
        else if (off == 0) w = C[t] > 0 ? 0.25f : 0.f;
        else w = C[t] < N - 1 ? 0.25f : 0.f;
        return fi;
      };
      double s = 0.0;
#pragma unroll
      for (int sa = -1; sa <= 1; ++sa) {        // along the normal: faces 2C-1, 2C, 2C+1
        const int fa = 2 * C[d] + sa;
        if (fa <= 0 || fa >= nf[d]) continue;   // fine roller faces hold nothing
        const float wa = sa == 0 ? 1.f : 0.5f;
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
          float wb;
          const int fb = tw(t1, ob, wb);
          if (wb == 0.f) continue;
#pragma unroll
          for (int oc = 0; oc < 4; ++oc) {
            float wc;
            const int fc = tw(t2, oc, wc);
            if (wc == 0.f) continue;
            int idx[3];
            idx[d] = fa;
            idx[t1] = fb;
            idx[t2] = fc;
            s += (double)(wa * wb * wc) * (double)rf.a[d][gidx(gf, idx[0], idx[1], idx[2])];
          }
        }
      }
      bc.a[d][ec] = (T)(0.25 * s);
    }
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
