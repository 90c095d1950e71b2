// Finite-strain mechanics on the voxel grid (Sec. 2.2, Eq. 9-14, 19, 25,
// 31, 34): bilinear (2D, plane strain) or trilinear (3D) elements on the
// cells, nodal displacements, 2^d Gauss points per cell with a plastic
// deformation gradient F_P and accumulated plastic strain at each.
//
//  * k_fs_elem: per cell, the deformation gradient F = I + sum_a u_a (x) grad N_a
//    at each Gauss point, the first Piola-Kirchhoff stress P = d psi / d F of
//    the phase-weighted neo-Hooke energy with F = F_E F_T F_P, and the cell's
//    nodal forces sum_g w P grad N_a.  Its tangent mode runs the same code on
//    dual numbers seeded with the gradient of a direction v, which yields the
//    exact directional derivative J v of the nodal forces (the Jacobian of
//    Newton's method applied without forming it).
//  * k_fs_gather: per node, the fixed-order sum of the forces its cells
//    computed for it (no atomics), rollers on the outer faces, and the FP64
//    block partial of a dot product.
//  * PCG kernels on the nodal vectors with device-side scalars.
//  * k_fs_return: the J2 return in the Mandel stress at each Gauss point
//    (backward Euler with the exponential map and the flow direction of the
//    end state, solved in the principal frame of the trial elastic stretch).
//  * k_fs_post: the cell-mean driving forces d psi / d phi_f, d psi / d phi_w
//    at fixed F, F_P (dual numbers in phi), and the largest von Mises stress.
#pragma once

#include <hip/hip_runtime.h>

namespace pfs {

// ---------------------------------------------------------------------------
// dual numbers: value and derivative along one direction
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual mkd(double v, double d = 0.0) { return Dual{v, d}; }
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dual dlog(Dual a) { return {log(a.v), a.d / a.v}; }
__device__ __forceinline__ Dual dexp(Dual a) {
  const double e = exp(a.v);
  return {e, a.d * e};
}
__device__ __forceinline__ double dlog(double a) { return log(a); }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(Dual a) { return a.v; }
__device__ __forceinline__ double der(Dual a) { return a.d; }

// ---------------------------------------------------------------------------
// 3x3 matrices, row-major
// ---------------------------------------------------------------------------
template <typename S>
struct M3 {
  S a[9];
};

template <typename S>
__device__ __forceinline__ S det3(const M3<S>& m) {
  const S* a = m.a;
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) + a[2] * (a[3] * a[7] - a[4] * a[6]);
}

// inverse transposed, from the cofactors: (m^-1)^T = cof(m) / det m
template <typename S>
__device__ __forceinline__ M3<S> inv_t3(const M3<S>& m, S det) {
  const S* a = m.a;
  M3<S> r;
  r.a[0] = (a[4] * a[8] - a[5] * a[7]) / det;
  r.a[1] = (a[5] * a[6] - a[3] * a[8]) / det;
  r.a[2] = (a[3] * a[7] - a[4] * a[6]) / det;
  r.a[3] = (a[2] * a[7] - a[1] * a[8]) / det;
  r.a[4] = (a[0] * a[8] - a[2] * a[6]) / det;
  r.a[5] = (a[1] * a[6] - a[0] * a[7]) / det;
  r.a[6] = (a[1] * a[5] - a[2] * a[4]) / det;
  r.a[7] = (a[2] * a[3] - a[0] * a[5]) / det;
  r.a[8] = (a[0] * a[4] - a[1] * a[3]) / det;
  return r;
}

__device__ __forceinline__ M3<double> inv3(const M3<double>& m) {
  const M3<double> t = inv_t3(m, det3(m));
  M3<double> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[3 * i + j] = t.a[3 * j + i];
  return r;
}

template <typename S, typename U>
__device__ __forceinline__ M3<S> mul3(const M3<S>& x, const M3<U>& y) {
  M3<S> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[3 * i + j] = x.a[3 * i] * y.a[j] + x.a[3 * i + 1] * y.a[3 + j] + x.a[3 * i + 2] * y.a[6 + j];
  return r;
}

__device__ __forceinline__ M3<double> mul3t(const M3<double>& x, const M3<double>& y) {   // x^T y
  M3<double> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[3 * i + j] = x.a[i] * y.a[j] + x.a[3 + i] * y.a[3 + j] + x.a[6 + i] * y.a[6 + j];
  return r;
}

__device__ __forceinline__ M3<double> eye3() {
  M3<double> r;
#pragma unroll
  for (int q = 0; q < 9; ++q) r.a[q] = (q % 4 == 0) ? 1.0 : 0.0;
  return r;
}

__device__ __forceinline__ void dev3(M3<double>& m) {
  const double t = (m.a[0] + m.a[4] + m.a[8]) / 3.0;
  m.a[0] -= t;
  m.a[4] -= t;
  m.a[8] -= t;
}

__device__ __forceinline__ double dot3(const M3<double>& x, const M3<double>& y) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 9; ++q) s += x.a[q] * y.a[q];
  return s;
}

// ---------------------------------------------------------------------------
// constitutive law
// ---------------------------------------------------------------------------
struct FSP {
  double K[3], G[3];      // ferrite, gas, wuestite
  double Omega, sigY, Hh;
};

template <typename S>
__device__ __forceinline__ S hpoly(S x) {
  return x * x * x * (x * (x * 6.0 - 15.0) + 10.0);
}

// P = d psi / d F and psi of Eq. 14 with F_E = d_T^(-1/3) F F_P^-1:
//   psi = d_T [Kb/4 (J^2 - 1 - 2 ln J) + Gb/2 (J^(-2/3) tr C_E - 3)],
//   P = d_T d_T^(-1/3) [Kb/2 (J^2 - 1) F_E^-T + Gb J^(-2/3) (F_E - tr C_E / 3 F_E^-T)] F_P^-T,
// Kb, Gb the h-weighted moduli of the three phases.
template <typename S, bool WANT_P>
__device__ __forceinline__ void neo_hooke(const M3<S>& F, S pf, S pw, const M3<double>& Fpi, const FSP& p, M3<S>* P,
                                          S* psi) {
  const S hf = hpoly(pf), hg = hpoly(1.0 - pf - pw), hw = hpoly(pw);
  const S Kb = hf * p.K[0] + hg * p.K[1] + hw * p.K[2];
  const S Gb = hf * p.G[0] + hg * p.G[1] + hw * p.G[2];
  const S dT = 1.0 - hf * p.Omega;
  const S c = dexp(dlog(dT) * (-1.0 / 3.0));
  M3<S> FE = mul3(F, Fpi);
#pragma unroll
  for (int q = 0; q < 9; ++q) FE.a[q] = c * FE.a[q];
  const S J = det3(FE);
  const S lJ = dlog(J);
  S trC = FE.a[0] * FE.a[0];
#pragma unroll
  for (int q = 1; q < 9; ++q) trC = trC + FE.a[q] * FE.a[q];
  const S Ju = dexp(lJ * (-2.0 / 3.0));
  if (psi) *psi = dT * (0.25 * Kb * (J * J - 1.0 - 2.0 * lJ) + 0.5 * Gb * (Ju * trC - 3.0));
  if constexpr (WANT_P) {
    const M3<S> FEiT = inv_t3(FE, J);
    const S a = 0.5 * Kb * (J * J - 1.0);
    const S b = Gb * Ju;
    const S bc = b * trC * (1.0 / 3.0);
    M3<S> Sm;
#pragma unroll
    for (int q = 0; q < 9; ++q) Sm.a[q] = (a - bc) * FEiT.a[q] + b * FE.a[q];
    const S sc = dT * c;
    // P = sc * Sm * Fpi^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        P->a[3 * i + j] = sc * (Sm.a[3 * i] * Fpi.a[3 * j] + Sm.a[3 * i + 1] * Fpi.a[3 * j + 1] + Sm.a[3 * i + 2] * Fpi.a[3 * j + 2]);
  }
}

// ---------------------------------------------------------------------------
// grid, shape functions
// ---------------------------------------------------------------------------
struct FSGrid {
  int nx, ny, nz;          // cells (nz = 1 in 2D)
  int mx, my, mz;          // nodes: nx + 1, ny + 1, nz + 1 (mz = 1 in 2D)
  long long ne, nn;        // cells, nodes
  double h, w;             // cell size, Gauss weight h^d / 2^d
};

constexpr double kG1 = 0.21132486540518711775;   // 1/2 - 1/(2 sqrt 3)
constexpr double kG2 = 0.78867513459481288225;   // 1/2 + 1/(2 sqrt 3)

// d N_a / d X_c at Gauss point g (local node a and Gauss point g: bit 0 the x
// side, bit 1 y, bit 2 z)
template <int DIM>
__device__ __forceinline__ double dshape(int g, int a, int c, double ih) {
  double v = ((a >> c) & 1) ? ih : -ih;
#pragma unroll
  for (int c2 = 0; c2 < DIM; ++c2) {
    if (c2 == c) continue;
    const double xi = ((g >> c2) & 1) ? kG2 : kG1;
    v *= ((a >> c2) & 1) ? xi : 1.0 - xi;
  }
  return v;
}

template <int DIM>
__device__ __forceinline__ long long node_of(const FSGrid& g, int i, int j, int k, int a) {
  const int bi = a & 1, bj = (a >> 1) & 1, bk = DIM == 3 ? (a >> 2) & 1 : 0;
  return ((long long)(k + bk) * g.my + (j + bj)) * g.mx + (i + bi);
}

__device__ __forceinline__ void cell_ijk(const FSGrid& g, long long e, int& i, int& j, int& k) {
  i = (int)(e % g.nx);
  const long long r = e / g.nx;
  j = (int)(r % g.ny);
  k = (int)(r / g.ny);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
constexpr int kFsThreads = 256;
constexpr int kFsBlocksMax = 1024;

enum FsScal {
  FS_RZ = 0,      // r.z of the current residual
  FS_PQ = 1,      // p.q
  FS_RR = 2,      // r.r
  FS_RR0 = 3,     // r.r at the start of the solve
  FS_ALPHA = 4,
  FS_BETA = 5,
  FS_CONV = 6,    // nonzero: the CG solve has stopped
  FS_ITERS = 7,   // CG iterations of the current solve
  FS_TOL2 = 8,    // cg_rtol^2
  FS_BAD = 9,     // nonzero: p.q <= 0 (the tangent was not positive along p)
  FS_NORM = 10,   // the last plain dot product (||R||^2 and the like)
  FS_MAX0 = 11,   // reduced maxima (plastic strain, von Mises stress)
  FS_MAX1 = 12,
  FS_SUM0 = 13,   // reduced count (yielded Gauss points)
  FS_COUNT = 16
};

struct FSElemArgs {
  FSGrid g;
  FSP p;
  const double* pf;
  const double* pw;
  const double* u;         // [DIM][nn]
  const double* v;         // direction of the tangent mode [DIM][nn]
  const double* Fp;        // [ne][ngp][9]; nullptr when every F_P is the identity
  double* ef;              // [2^DIM * DIM][ne] element forces
  const double* sc;        // device scalars (the tangent mode exits once CG has stopped)
};

// F_P^-1 at Gauss point gq of cell e (Fp == nullptr: every F_P is the identity)
__device__ __forceinline__ M3<double> load_Fpi(const double* Fp, long long e, int gq, int ngp) {
  if (!Fp) return eye3();
  M3<double> m;
  const double* s = Fp + (e * ngp + gq) * 9;
#pragma unroll
  for (int q = 0; q < 9; ++q) m.a[q] = s[q];
  return inv3(m);
}

template <int DIM, bool TAN>
__global__ __launch_bounds__(kFsThreads) void k_fs_elem(FSElemArgs a) {
  constexpr int NA = 1 << DIM;
  if (TAN && a.sc[FS_CONV] != 0.0) return;
  const FSGrid& g = a.g;
  const double ih = 1.0 / g.h;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.ne; e += (long long)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(g, e, i, j, k);
    double un[NA][DIM], vn[NA][DIM];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const long long nid = node_of<DIM>(g, i, j, k, n);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        un[n][c] = a.u[c * g.nn + nid];
        vn[n][c] = TAN ? a.v[c * g.nn + nid] : 0.0;
      }
    }
    const double pf = a.pf[e], pw = a.pw[e];
    double f[NA][DIM];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
      for (int c = 0; c < DIM; ++c) f[n][c] = 0.0;
    for (int gq = 0; gq < NA; ++gq) {
      double dN[NA][DIM];
#pragma unroll
      for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int c = 0; c < DIM; ++c) dN[n][c] = dshape<DIM>(gq, n, c, ih);
      const M3<double> Fpi = load_Fpi(a.Fp, e, gq, NA);
      if constexpr (TAN) {
        M3<Dual> F;
#pragma unroll
        for (int q = 0; q < 9; ++q) F.a[q] = mkd((q % 4 == 0) ? 1.0 : 0.0, 0.0);
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
          for (int c = 0; c < DIM; ++c) {
            double fv = 0.0, fd = 0.0;
#pragma unroll
            for (int n = 0; n < NA; ++n) {
              fv += un[n][r] * dN[n][c];
              fd += vn[n][r] * dN[n][c];
            }
            F.a[3 * r + c].v += fv;
            F.a[3 * r + c].d = fd;
          }
        M3<Dual> P;
        neo_hooke<Dual, true>(F, mkd(pf), mkd(pw), Fpi, a.p, &P, (Dual*)nullptr);
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
          for (int r = 0; r < DIM; ++r) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += der(P.a[3 * r + c]) * dN[n][c];
            f[n][r] += g.w * s;
          }
      } else {
        M3<double> F = eye3();
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
          for (int c = 0; c < DIM; ++c) {
            double fv = 0.0;
#pragma unroll
            for (int n = 0; n < NA; ++n) fv += un[n][r] * dN[n][c];
            F.a[3 * r + c] += fv;
          }
        M3<double> P;
        neo_hooke<double, true>(F, pf, pw, Fpi, a.p, &P, (double*)nullptr);
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
          for (int r = 0; r < DIM; ++r) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += P.a[3 * r + c] * dN[n][c];
            f[n][r] += g.w * s;
          }
      }
    }
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
      for (int c = 0; c < DIM; ++c) a.ef[(long long)(n * DIM + c) * g.ne + e] = f[n][c];
  }
}

// FP64 block sum of `v` (every thread contributes), written to part[blockIdx.x].
__device__ __forceinline__ void block_sum(double v, double* part) {
  __shared__ double red[kFsThreads / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = red[0];
#pragma unroll
    for (int q = 1; q < kFsThreads / 64; ++q) s += red[q];
    part[blockIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void block_max(double v, double* part) {
  __shared__ double red[kFsThreads / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = red[0];
#pragma unroll
    for (int q = 1; q < kFsThreads / 64; ++q) s = fmax(s, red[q]);
    part[blockIdx.x] = s;
  }
  __syncthreads();
}

// true when nodal component c of node (i, j, k) is a roller component
template <int DIM>
__device__ __forceinline__ bool fixed_dof(const FSGrid& g, int c, int i, int j, int k) {
  if (c == 0) return i == 0 || i == g.nx;
  if (c == 1) return j == 0 || j == g.ny;
  return k == 0 || k == g.nz;
}

struct FSGatherArgs {
  FSGrid g;
  const double* ef;
  double* out;             // [DIM][nn]
  const double* y;         // nullable: partials of out . y (else of out . out)
  double* part;
  const double* sc;        // nullable: exit once CG has stopped
};

template <int DIM>
__global__ __launch_bounds__(kFsThreads) void k_fs_gather(FSGatherArgs a) {
  constexpr int NA = 1 << DIM;
  if (a.sc && a.sc[FS_CONV] != 0.0) return;
  const FSGrid& g = a.g;
  double acc = 0.0;
  for (long long nid = (long long)blockIdx.x * blockDim.x + threadIdx.x; nid < g.nn;
       nid += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(nid % g.mx);
    const long long r = nid / g.mx;
    const int j = (int)(r % g.my);
    const int k = (int)(r / g.my);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      double s = 0.0;
#pragma unroll
      for (int n = 0; n < NA; ++n) {       // the cell that holds this node as its local node n
        const int ci = i - (n & 1), cj = j - ((n >> 1) & 1), ck = DIM == 3 ? k - ((n >> 2) & 1) : 0;
        if (ci < 0 || ci >= g.nx || cj < 0 || cj >= g.ny || ck < 0 || ck >= g.nz) continue;
        const long long e = ((long long)ck * g.ny + cj) * g.nx + ci;
        s += a.ef[(long long)(n * DIM + c) * g.ne + e];
      }
      if (fixed_dof<DIM>(g, c, i, j, k)) s = 0.0;
      a.out[c * g.nn + nid] = s;
      acc += s * (a.y ? a.y[c * g.nn + nid] : s);
    }
  }
  block_sum(acc, a.part);
}

// Jacobi diagonal of the small-strain stiffness with the cell moduli
// K = d_T sum h K_a, G = d_T sum h G_a: sum over the node's cells and Gauss
// points of w [(K + 4G/3) (dN/dX_c)^2 + G sum_{c' != c} (dN/dX_c')^2];
// stored inverted, zero on the roller components.
template <int DIM>
__global__ __launch_bounds__(kFsThreads) void k_fs_diag(FSGrid g, FSP p, const double* pf, const double* pw,
                                                        double* dinv) {
  constexpr int NA = 1 << DIM;
  const double ih = 1.0 / g.h;
  for (long long nid = (long long)blockIdx.x * blockDim.x + threadIdx.x; nid < g.nn;
       nid += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(nid % g.mx);
    const long long r = nid / g.mx;
    const int j = (int)(r % g.my);
    const int k = (int)(r / g.my);
    double d[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) d[c] = 0.0;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const int ci = i - (n & 1), cj = j - ((n >> 1) & 1), ck = DIM == 3 ? k - ((n >> 2) & 1) : 0;
      if (ci < 0 || ci >= g.nx || cj < 0 || cj >= g.ny || ck < 0 || ck >= g.nz) continue;
      const long long e = ((long long)ck * g.ny + cj) * g.nx + ci;
      const double f = pf[e], w_ = pw[e];
      const double hf = hpoly(f), hg = hpoly(1.0 - f - w_), hw = hpoly(w_);
      const double dT = 1.0 - hf * p.Omega;
      const double K = dT * (hf * p.K[0] + hg * p.K[1] + hw * p.K[2]);
      const double G = dT * (hf * p.G[0] + hg * p.G[1] + hw * p.G[2]);
      for (int gq = 0; gq < NA; ++gq) {
        double q2[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          const double v = dshape<DIM>(gq, n, c, ih);
          q2[c] = v * v;
        }
        double tot = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) tot += q2[c];
#pragma unroll
        for (int c = 0; c < DIM; ++c) d[c] += g.w * ((K + 4.0 * G / 3.0) * q2[c] + G * (tot - q2[c]));
      }
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) dinv[c * g.nn + nid] = fixed_dof<DIM>(g, c, i, j, k) || d[c] <= 0.0 ? 0.0 : 1.0 / d[c];
  }
}

struct FSVec {
  long long nd;            // DIM * nn
  const double* dinv;
  double* x;
  double* r;
  double* z;
  double* p;
  double* q;
  double* part;            // [2][nb]
  double* sc;
};

// start of a CG solve of J x = -R: x = 0, r = -R, z = D^-1 r, p = z; partials r.z, r.r
__global__ __launch_bounds__(kFsThreads) void k_fs_cg_init(FSVec v, const double* R) {
  double rz = 0.0, rr = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < v.nd; q += (long long)gridDim.x * blockDim.x) {
    const double r = -R[q];
    const double z = v.dinv[q] * r;
    v.x[q] = 0.0;
    v.r[q] = r;
    v.z[q] = z;
    v.p[q] = z;
    rz += r * z;
    rr += r * r;
  }
  block_sum(rz, v.part);
  block_sum(rr, v.part + gridDim.x);
}

// x += alpha p, r -= alpha q, z = D^-1 r; partials r.z, r.r
__global__ __launch_bounds__(kFsThreads) void k_fs_cg_update(FSVec v) {
  if (v.sc[FS_CONV] != 0.0) return;
  const double al = v.sc[FS_ALPHA];
  double rz = 0.0, rr = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < v.nd; q += (long long)gridDim.x * blockDim.x) {
    v.x[q] += al * v.p[q];
    const double r = v.r[q] - al * v.q[q];
    const double z = v.dinv[q] * r;
    v.r[q] = r;
    v.z[q] = z;
    rz += r * z;
    rr += r * r;
  }
  block_sum(rz, v.part);
  block_sum(rr, v.part + gridDim.x);
}

// p = z + beta p
__global__ __launch_bounds__(kFsThreads) void k_fs_cg_dir(FSVec v) {
  if (v.sc[FS_CONV] != 0.0) return;
  const double be = v.sc[FS_BETA];
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < v.nd; q += (long long)gridDim.x * blockDim.x)
    v.p[q] = v.z[q] + be * v.p[q];
}

enum FsReduce { FSR_INIT = 0, FSR_ALPHA = 1, FSR_BETA = 2, FSR_NORM = 3, FSR_MAX2_SUM = 4 };

// One block of kFsThreads threads: fixed-order sums (and maxima) of the
// block partials -- thread t takes partials t, t + 256, ... in order, then a
// fixed tree over the threads -- and the CG scalars from them.
__device__ __forceinline__ double fs_block_reduce(const double* a, int nb, bool mx) {
  __shared__ double red[kFsThreads];
  double v = mx ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nb; b += kFsThreads) v = mx ? fmax(v, a[b]) : v + a[b];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kFsThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = mx ? fmax(red[threadIdx.x], red[threadIdx.x + w]) : red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kFsThreads) void k_fs_reduce(const double* part, int nb, double* sc, int mode, int max_iter) {
  const bool conv = sc[FS_CONV] != 0.0;
  if (mode == FSR_INIT) {
    const double rz = fs_block_reduce(part, nb, false), rr = fs_block_reduce(part + nb, nb, false);
    if (threadIdx.x == 0) {
      sc[FS_RZ] = rz;
      sc[FS_RR] = rr;
      sc[FS_RR0] = rr;
      sc[FS_ITERS] = 0.0;
      sc[FS_BAD] = 0.0;
      sc[FS_CONV] = (rr == 0.0) ? 1.0 : 0.0;
    }
  } else if (mode == FSR_ALPHA) {
    if (conv) return;
    const double pq = fs_block_reduce(part, nb, false);
    if (threadIdx.x == 0) {
      sc[FS_PQ] = pq;
      if (!(pq > 0.0)) {
        sc[FS_BAD] = 1.0;
        sc[FS_CONV] = 1.0;
      } else {
        sc[FS_ALPHA] = sc[FS_RZ] / pq;
      }
    }
  } else if (mode == FSR_BETA) {
    if (conv) return;
    const double rz = fs_block_reduce(part, nb, false), rr = fs_block_reduce(part + nb, nb, false);
    if (threadIdx.x == 0) {
      sc[FS_BETA] = rz / sc[FS_RZ];
      sc[FS_RZ] = rz;
      sc[FS_RR] = rr;
      sc[FS_ITERS] += 1.0;
      if (rr <= sc[FS_TOL2] * sc[FS_RR0] || sc[FS_ITERS] >= (double)max_iter) sc[FS_CONV] = 1.0;
    }
  } else if (mode == FSR_NORM) {
    const double v = fs_block_reduce(part, nb, false);
    if (threadIdx.x == 0) sc[FS_NORM] = v;
  } else {
    const double m0 = fs_block_reduce(part, nb, true), m1 = fs_block_reduce(part + nb, nb, true);
    const double s2 = fs_block_reduce(part + 2 * nb, nb, false);
    if (threadIdx.x == 0) {
      sc[FS_MAX0] = m0;
      sc[FS_MAX1] = m1;
      sc[FS_SUM0] = s2;
    }
  }
}

// y = x + s d (line search trial) and the like
__global__ __launch_bounds__(kFsThreads) void k_fs_axpy(long long n, const double* x, double s, const double* d,
                                                        double* y) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
    y[q] = x[q] + s * d[q];
}

// F_P = I and eps_P = 0 at every Gauss point
__global__ __launch_bounds__(kFsThreads) void k_fs_plastic_reset(long long npts, double* Fp, double* epsP) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < npts; q += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 9; ++c) Fp[q * 9 + c] = (c % 4 == 0) ? 1.0 : 0.0;
    epsP[q] = 0.0;
  }
}

// zero the roller components of a nodal vector (after the caller set it)
template <int DIM>
__global__ __launch_bounds__(kFsThreads) void k_fs_fix(FSGrid g, double* u) {
  for (long long nid = (long long)blockIdx.x * blockDim.x + threadIdx.x; nid < g.nn;
       nid += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(nid % g.mx);
    const long long r = nid / g.mx;
    const int j = (int)(r % g.my);
    const int k = (int)(r / g.my);
#pragma unroll
    for (int c = 0; c < DIM; ++c)
      if (fixed_dof<DIM>(g, c, i, j, k)) u[c * g.nn + nid] = 0.0;
  }
}

template <int DIM>
__device__ __forceinline__ M3<double> grad_F(const FSGrid& g, const double* u, int i, int j, int k, int gq) {
  constexpr int NA = 1 << DIM;
  const double ih = 1.0 / g.h;
  M3<double> F = eye3();
#pragma unroll
  for (int n = 0; n < NA; ++n) {
    const long long nid = node_of<DIM>(g, i, j, k, n);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const double dn = dshape<DIM>(gq, n, c, ih);
#pragma unroll
      for (int r = 0; r < DIM; ++r) F.a[3 * r + c] += u[r * g.nn + nid] * dn;
    }
  }
  return F;
}

struct FSRetArgs {
  FSGrid g;
  FSP p;
  const double* pf;
  const double* pw;
  const double* u;
  double* Fp;
  double* epsP;
  double* part;            // [3][nb]: max eps_P, (unused), yielded count
  double tol;
};

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations:
// A = Q diag(c) Q^T (columns of Q are the eigenvectors).
__device__ __forceinline__ void eig_sym3(M3<double> A, double c[3], M3<double>& Q) {
  Q = eye3();
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = A.a[1] * A.a[1] + A.a[2] * A.a[2] + A.a[5] * A.a[5];
    const double dia = A.a[0] * A.a[0] + A.a[4] * A.a[4] + A.a[8] * A.a[8];
    if (off <= 1e-36 * dia || off == 0.0) break;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int pi = r == 2 ? 1 : 0, qi = r == 0 ? 1 : 2;
      const double apq = A.a[3 * pi + qi];
      if (apq == 0.0) continue;
      const double th = (A.a[3 * qi + qi] - A.a[3 * pi + pi]) / (2.0 * apq);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
      const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
      // A <- R^T A R with the rotation in the (pi, qi) plane
#pragma unroll
      for (int k = 0; k < 3; ++k) {           // columns pi, qi
        const double akp = A.a[3 * k + pi], akq = A.a[3 * k + qi];
        A.a[3 * k + pi] = cs * akp - sn * akq;
        A.a[3 * k + qi] = sn * akp + cs * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {           // rows pi, qi
        const double apk = A.a[3 * pi + k], aqk = A.a[3 * qi + k];
        A.a[3 * pi + k] = cs * apk - sn * aqk;
        A.a[3 * qi + k] = sn * apk + cs * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double qkp = Q.a[3 * k + pi], qkq = Q.a[3 * k + qi];
        Q.a[3 * k + pi] = cs * qkp - sn * qkq;
        Q.a[3 * k + qi] = sn * qkp + cs * qkq;
      }
    }
  }
  c[0] = A.a[0];
  c[1] = A.a[4];
  c[2] = A.a[8];
}

// J2 return in the Mandel stress at each Gauss point (Eq. 25, 34), backward
// Euler with the exponential map and the flow direction of the end state:
// in the principal frame Q of the trial elastic stretch C_tr (F_P = F_P^n),
// with the deviatoric log stretches e_tr = ln(c)/2 - ln(J)/3, the neo-Hooke
// energy gives dev M = k dev(exp(2 e)), k = d_T sum h_a G_a; the return
// solves e + dl s(e) / Y(dl) = e_tr (Newton in e) with |s(e(dl))| = Y(dl) =
// sqrt(2/3)(sigma_Y + H (eps_P^n + dl)) (bracket doubled from 1e-3, then
// Illinois regula falsi to hi - lo <= tol hi: the root the oracle's
// bisection reaches, in fewer evaluations) and sets F_P = Q diag(exp(dl n))
// Q^T F_P^n, n = s / |s|.
template <int DIM>
__global__ __launch_bounds__(kFsThreads) void k_fs_return(FSRetArgs a) {
  constexpr int NA = 1 << DIM;
  const FSGrid& g = a.g;
  const double r23 = 0.81649658092772603273;     // sqrt(2/3)
  double mx = 0.0, cnt = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.ne; e += (long long)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(g, e, i, j, k);
    const double pf = a.pf[e], pw = a.pw[e];
    const double hf = hpoly(pf), hg = hpoly(1.0 - pf - pw), hw = hpoly(pw);
    const double dT = 1.0 - hf * a.p.Omega;
    const double kk = dT * (hf * a.p.G[0] + hg * a.p.G[1] + hw * a.p.G[2]);
    const double cT = exp(log(dT) * (-1.0 / 3.0));
    for (int gq = 0; gq < NA; ++gq) {
      const long long pt = e * NA + gq;
      M3<double> Fpn;
#pragma unroll
      for (int q = 0; q < 9; ++q) Fpn.a[q] = a.Fp[pt * 9 + q];
      const double e0 = a.epsP[pt];
      const M3<double> F = grad_F<DIM>(g, a.u, i, j, k, gq);
      M3<double> FE = mul3(F, inv3(Fpn));
#pragma unroll
      for (int q = 0; q < 9; ++q) FE.a[q] *= cT;
      double c[3];
      M3<double> Q;
      eig_sym3(mul3t(FE, FE), c, Q);
      const double lnJ = 0.5 * (log(c[0]) + log(c[1]) + log(c[2]));
      double et[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) et[q] = 0.5 * log(c[q]) - lnJ / 3.0;
      auto s_of = [&](const double* ev, double* sv) {
        const double x0 = exp(2.0 * ev[0]), x1 = exp(2.0 * ev[1]), x2 = exp(2.0 * ev[2]);
        const double m = (x0 + x1 + x2) / 3.0;
        sv[0] = kk * (x0 - m);
        sv[1] = kk * (x1 - m);
        sv[2] = kk * (x2 - m);
      };
      auto Yf = [&](double dl) { return r23 * (a.p.sigY + a.p.Hh * (e0 + dl)); };
      double st[3];
      s_of(et, st);
      const double ytr = sqrt(st[0] * st[0] + st[1] * st[1] + st[2] * st[2]) - Yf(0.0);
      if (ytr > 0.0) {
        // e(dl): Newton on G(e) = e + (dl / Y) s(e) - e_tr from e_tr
        auto e_of = [&](double dl, double* ev) {
          const double al = dl / Yf(dl) * kk;
          ev[0] = et[0];
          ev[1] = et[1];
          ev[2] = et[2];
          for (int t = 0; t < 60; ++t) {
            const double x[3] = {exp(2.0 * ev[0]), exp(2.0 * ev[1]), exp(2.0 * ev[2])};
            const double m = (x[0] + x[1] + x[2]) / 3.0;
            double G[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) G[q] = ev[q] + al * (x[q] - m) - et[q];
            if (fmax(fabs(G[0]), fmax(fabs(G[1]), fabs(G[2]))) <= 1e-15) break;
            M3<double> Jm;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int q = 0; q < 3; ++q)
                Jm.a[3 * r + q] = (r == q ? 1.0 + 2.0 * al * x[q] : 0.0) - al * (2.0 / 3.0) * x[q];
            const M3<double> Ji = inv3(Jm);
#pragma unroll
            for (int r = 0; r < 3; ++r) ev[r] -= Ji.a[3 * r] * G[0] + Ji.a[3 * r + 1] * G[1] + Ji.a[3 * r + 2] * G[2];
          }
        };
        auto phi = [&](double dl) {
          double ev[3], sv[3];
          e_of(dl, ev);
          s_of(ev, sv);
          return sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]) - Yf(dl);
        };
        // bracket [lo, hi] with phi(lo) > 0 >= phi(hi), then the Illinois
        // variant of regula falsi (the retained end's value halved when the
        // same end is kept twice), down to hi - lo <= tol hi or |phi| <= 1e-14 Y
        double lo = 0.0, hi = 1e-3, flo = ytr, fhi = phi(hi);
        for (int t = 0; t < 64 && fhi > 0.0; ++t) {
          lo = hi;
          flo = fhi;
          hi *= 2.0;
          fhi = phi(hi);
        }
        double dl = hi;
        int side = 0;
        for (int t = 0; t < 200; ++t) {
          if (hi - lo <= a.tol * fmax(hi, 1e-300)) {
            dl = 0.5 * (lo + hi);
            break;
          }
          double x = hi - fhi * (hi - lo) / (fhi - flo);
          if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
          const double fx = phi(x);
          dl = x;
          if (fabs(fx) <= 1e-14 * Yf(x)) break;     // |dl - root| ~ 1e-14 Y / (2 G): far below tol dl
          if (fx > 0.0) {
            lo = x;
            flo = fx;
            if (side == 1) fhi *= 0.5;
            side = 1;
          } else {
            hi = x;
            fhi = fx;
            if (side == -1) flo *= 0.5;
            side = -1;
          }
        }
        double ev[3], sv[3];
        e_of(dl, ev);
        s_of(ev, sv);
        const double ns = sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
        double ex[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) ex[q] = exp(dl * sv[q] / ns);
        M3<double> Ex;                          // Q diag(ex) Q^T
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int q = 0; q < 3; ++q)
            Ex.a[3 * r + q] = Q.a[3 * r] * ex[0] * Q.a[3 * q] + Q.a[3 * r + 1] * ex[1] * Q.a[3 * q + 1] +
                              Q.a[3 * r + 2] * ex[2] * Q.a[3 * q + 2];
        const M3<double> Fpnew = mul3(Ex, Fpn);
#pragma unroll
        for (int q = 0; q < 9; ++q) a.Fp[pt * 9 + q] = Fpnew.a[q];
        a.epsP[pt] = e0 + dl;
        cnt += 1.0;
      }
      mx = fmax(mx, a.epsP[pt]);
    }
  }
  block_max(mx, a.part);
  block_max(0.0, a.part + gridDim.x);
  block_sum(cnt, a.part + 2 * gridDim.x);
}

struct FSPostArgs {
  FSGrid g;
  FSP p;
  const double* pf;
  const double* pw;
  const double* u;
  const double* Fp;        // nullptr when every F_P is the identity
  double* drive;           // [2][ne]: cell means of d psi / d phi_f, d psi / d phi_w
  double* part;            // [3][nb]: (unused), max von Mises, (unused)
};

// driving forces at fixed F and F_P (dual numbers in phi) and the largest
// von Mises stress sqrt(3/2) |dev sigma|, sigma = P F^T / det F
template <int DIM>
__global__ __launch_bounds__(kFsThreads) void k_fs_post(FSPostArgs a) {
  constexpr int NA = 1 << DIM;
  const FSGrid& g = a.g;
  double vmax = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.ne; e += (long long)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(g, e, i, j, k);
    const double pf = a.pf[e], pw = a.pw[e];
    double gf = 0.0, gw = 0.0;
    for (int gq = 0; gq < NA; ++gq) {
      const M3<double> F = grad_F<DIM>(g, a.u, i, j, k, gq);
      const M3<double> Fpi = load_Fpi(a.Fp, e, gq, NA);
      M3<Dual> Fd;
#pragma unroll
      for (int q = 0; q < 9; ++q) Fd.a[q] = mkd(F.a[q]);
      Dual psi;
      neo_hooke<Dual, false>(Fd, mkd(pf, 1.0), mkd(pw), Fpi, a.p, (M3<Dual>*)nullptr, &psi);
      gf += der(psi);
      neo_hooke<Dual, false>(Fd, mkd(pf), mkd(pw, 1.0), Fpi, a.p, (M3<Dual>*)nullptr, &psi);
      gw += der(psi);
      M3<double> P;
      neo_hooke<double, true>(F, pf, pw, Fpi, a.p, &P, (double*)nullptr);
      M3<double> sg;
      const double J = det3(F);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          sg.a[3 * r + c] = (P.a[3 * r] * F.a[3 * c] + P.a[3 * r + 1] * F.a[3 * c + 1] + P.a[3 * r + 2] * F.a[3 * c + 2]) / J;
      dev3(sg);
      vmax = fmax(vmax, sqrt(1.5 * dot3(sg, sg)));
    }
    a.drive[e] = gf / NA;
    a.drive[g.ne + e] = gw / NA;
  }
  block_max(0.0, a.part);
  block_max(vmax, a.part + gridDim.x);
  block_sum(0.0, a.part + 2 * gridDim.x);
}

}  // namespace pfs
