// Linearly implicit Euler for the three species (x_O, x_H, x_H2O).
//
// The field update writes, per species s, the explicit increment
// b_s = dt T_s(x^n) (every flux, and the reaction at x^n unless the reaction
// is split off and solved exactly afterwards, see k_sp_finish) and the cell
// diffusivity D_s of the species.  The increment d_s of the step then solves
//   (I + dt A_s) d_s = b_s,   A_s v = -div(D_s grad v),
// with the two-cell mean of D_s at interior faces and, for x_H and x_H2O when
// the outer faces are Dirichlet faces, 2 D_s(cell) / h^2 per outer face on
// the diagonal: backward Euler for the stiff diffusion (Sec. 2.4 integrates
// the species with backward Euler), explicit for the rest.  The three
// systems are solved side by side by Jacobi-preconditioned CG, each with its
// own recurrence scalars and convergence test (a converged species is left
// alone), with fixed-order FP64 dot products; the species are then updated
// and their ledger terms formed from the new values.
#pragma once

#include "pf_kernels.h"

namespace pfk {

constexpr int kSpBlocksMax = 512;

// species scalars (FP64 slots)
enum SpScal {
  SP_BB = 0,       // ||b_s||^2 (3)
  SP_RZ = 3,       // r.z of the current residual, ring of two iterations (2 x 3)
  SP_CONV = 9,     // nonzero once species s has converged (3)
  SP_ITERS = 12,   // CG iterations of species s (3)
  SP_RR = 15,      // ||r_s||^2 at the last test (3)
  SP_COUNT = 32
};

template <typename T>
struct SpArgs {
  Grid g;
  T dt_ih2;                // dt / h^2
  int dirichlet;           // x_H and x_H2O have Dirichlet outer faces
  const T* D[3];
  T* dinv[3];
  T* r[3];
  T* z[3];
  T* pa[3];                // directions, ping-pong by iteration parity
  T* pb[3];
  T* q[3];
  T* d[3];                 // the increments being solved for
  double* part_rr;         // [2 (r.z, r.r)][3][nb] from the set-up and update passes
  double* part_pq;         // [3][nb] from the apply pass
  int nb;                  // blocks of these kernels (and partials per quantity)
  double* sc;              // SP_COUNT scalars
  double tol2;
  int it;                  // CG iteration of an apply / update launch
};

// Cell e -> (i, j, k); false for padding columns.
__device__ __forceinline__ bool sp_cell(const Grid& g, int e, int& i, int& j, int& k) {
  i = e % g.px;
  const int r = e / g.px;
  j = r % g.ny;
  k = r / g.ny;
  return i < g.nx;
}

// Sum of D_face over the faces of cell (i, j, k) and, for the outer faces,
// their count (every face contributes D_face / h^2 to A's diagonal; an outer
// Dirichlet face 2 D_cell / h^2).
template <typename T, int DIM>
__device__ __forceinline__ T sp_diag(const Grid& g, const T* D, int e, int i, int j, int k, bool dir) {
  const int pl = g.px * g.ny;
  const T dc = D[e];
  T s = T(0);
  const int c[3] = {i, j, k}, lim[3] = {g.nx, g.ny, g.nz}, st[3] = {1, g.px, pl};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (c[d] > 0) s += T(0.5) * (dc + D[e - st[d]]); else if (dir) s += T(2) * dc;
    if (c[d] + 1 < lim[d]) s += T(0.5) * (dc + D[e + st[d]]); else if (dir) s += T(2) * dc;
  }
  return s;
}

// (A v)_cell * h^2 for one species, with v_nb given by `at` (so that the apply
// pass can form the new direction of a neighbour on the fly).
template <typename T, int DIM, typename F>
__device__ __forceinline__ T sp_lap(const Grid& g, const T* D, int e, int i, int j, int k, bool dir, T vc, F at) {
  const int pl = g.px * g.ny;
  const T dc = D[e];
  T s = T(0);
  const int c[3] = {i, j, k}, lim[3] = {g.nx, g.ny, g.nz}, st[3] = {1, g.px, pl};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (c[d] > 0) s += T(0.5) * (dc + D[e - st[d]]) * (vc - at(e - st[d])); else if (dir) s += T(2) * dc * vc;
    if (c[d] + 1 < lim[d]) s += T(0.5) * (dc + D[e + st[d]]) * (vc - at(e + st[d])); else if (dir) s += T(2) * dc * vc;
  }
  return s;
}

// Block partials of six (or three) quantities, written at [q][nb] + block.
template <int NQ>
__device__ __forceinline__ void sp_partials(double (&v)[NQ], double* out, int nb) {
  __shared__ double red[NQ][NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += __shfl_xor(v[q], o, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[threadIdx.x][w];
    out[threadIdx.x * nb + blockIdx.x] = s;
  }
}

// Fixed-order sums of NQ partial arrays of length nb (identical in every block).
template <int NQ>
__device__ __forceinline__ void sp_sums(const double* part, int nb, double (&s)[NQ]) {
  __shared__ double red[NQ][NT / 64];
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int t = threadIdx.x; t < nb; t += NT)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += part[q * nb + t];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += __shfl_xor(v[q], o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += red[q][w];
    s[q] = t;
  }
}

// Set-up: d = 0, r = b (already in r), z = D^-1 r; partials r.z and r.r.
template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_sp_init(SpArgs<T> a) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int e = blockIdx.x * NT + threadIdx.x; e < a.g.n; e += a.nb * NT) {
    int i, j, k;
    if (!sp_cell(a.g, e, i, j, k)) continue;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const T di = T(1) / (T(1) + a.dt_ih2 * sp_diag<T, DIM>(a.g, a.D[s], e, i, j, k, s > 0 && a.dirichlet));
      const T r = a.r[s][e];
      const T z = di * r;
      a.dinv[s][e] = di;
      a.z[s][e] = z;
      a.d[s][e] = T(0);
      v[s] += (double)r * (double)z;
      v[3 + s] += (double)r * (double)r;
    }
  }
  sp_partials<6>(v, a.part_rr, a.nb);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int q = 0; q < SP_COUNT; ++q) a.sc[q] = 0.0;
}

// Convergence of every species from the latest r.r partials (every block of
// the apply pass takes the same decision; this one is for the host's test).
__global__ __launch_bounds__(NT) void k_sp_check(const double* part_rr, int nb, double* sc, double tol2, int first) {
  double s[6];
  sp_sums<6>(part_rr, nb, s);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) {
      const double bb = first ? s[3 + q] : sc[SP_BB + q];
      if (first) sc[SP_BB + q] = bb;
      sc[SP_RR + q] = s[3 + q];
      if (s[3 + q] <= tol2 * bb) sc[SP_CONV + q] = 1.0;
    }
}

// Apply pass of iteration it: beta from the latest r.z, p = z + beta p_old
// (p = z at it = 0), q = (I + dt A) p; partials p.q.  Species whose residual
// has met the tolerance are marked converged and left alone.
template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_sp_apply(SpArgs<T> a) {
  double s[6];
  sp_sums<6>(a.part_rr, a.nb, s);
  bool conv[3];
  double beta[3];
  bool all = true;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double bb = a.it == 0 ? s[3 + q] : a.sc[SP_BB + q];
    conv[q] = a.sc[SP_CONV + q] != 0.0 || s[3 + q] <= a.tol2 * bb;
    beta[q] = a.it == 0 ? 0.0 : s[q] / a.sc[SP_RZ + ((a.it - 1) & 1) * 3 + q];
    all = all && conv[q];
  }
  __syncthreads();            // every thread has read the scalars before block 0 writes them
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) {
      if (a.it == 0) a.sc[SP_BB + q] = s[3 + q];
      a.sc[SP_RZ + (a.it & 1) * 3 + q] = s[q];
      a.sc[SP_RR + q] = s[3 + q];
      if (conv[q]) a.sc[SP_CONV + q] = 1.0; else a.sc[SP_ITERS + q] += 1.0;
    }
  if (all) return;
  T** pn = (a.it & 1) ? a.pb : a.pa;
  T** po = (a.it & 1) ? a.pa : a.pb;
  double v[3] = {0, 0, 0};
  for (int e = blockIdx.x * NT + threadIdx.x; e < a.g.n; e += a.nb * NT) {
    int i, j, k;
    if (!sp_cell(a.g, e, i, j, k)) continue;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (conv[q]) continue;
      const T* z = a.z[q];
      const T* p0 = po[q];
      const T b = (T)beta[q];
      auto at = [&](int f) { return a.it == 0 ? z[f] : z[f] + b * p0[f]; };
      const T pc = at(e);
      const T qc = pc + a.dt_ih2 * sp_lap<T, DIM>(a.g, a.D[q], e, i, j, k, q > 0 && a.dirichlet, pc, at);
      pn[q][e] = pc;
      a.q[q][e] = qc;
      v[q] += (double)pc * (double)qc;
    }
  }
  sp_partials<3>(v, a.part_pq, a.nb);
}

// Update pass of iteration it: alpha = r.z / p.q, d += alpha p, r -= alpha q,
// z = D^-1 r; partials r.z and r.r (zero for converged species).
template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_sp_update(SpArgs<T> a) {
  double s[3];
  sp_sums<3>(a.part_pq, a.nb, s);
  bool conv[3];
  double alpha[3];
  bool all = true;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    conv[q] = a.sc[SP_CONV + q] != 0.0;
    alpha[q] = conv[q] ? 0.0 : a.sc[SP_RZ + (a.it & 1) * 3 + q] / s[q];
    all = all && conv[q];
  }
  if (all) return;
  T** pn = (a.it & 1) ? a.pb : a.pa;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int e = blockIdx.x * NT + threadIdx.x; e < a.g.n; e += a.nb * NT) {
    int i, j, k;
    if (!sp_cell(a.g, e, i, j, k)) continue;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (conv[q]) continue;
      const T al = (T)alpha[q];
      a.d[q][e] += al * pn[q][e];
      const T r = a.r[q][e] - al * a.q[q][e];
      const T z = a.dinv[q][e] * r;
      a.r[q][e] = r;
      a.z[q][e] = z;
      v[q] += (double)r * (double)z;
      v[3 + q] += (double)r * (double)r;
    }
  }
  sp_partials<6>(v, a.part_rr, a.nb);
}

// The reaction of Eq. 27, 28 alone over a time t in one cell (m(phi_g)
// frozen), from its exact solution: with b = x_H, c = b - 2a constant and
// x = c k m t, the amount of O reacted is
//   R = a b k m t E / (1 + s k m t E),  E = (1 - e^-|x|) / |x|,
// s = 2a when c >= 0 (hydrogen in excess) and s = b when c < 0 (E -> 1 as
// x -> 0; every term non-negative, no cancellation).  Zero where a or b is not
// positive or the cell is full of water.  FP64.
__device__ __forceinline__ double reaction_exact(double a, double b, double w, double m, double k, double t) {
  if (!(w < 1.0) || !(a > 0.0) || !(b > 0.0) || !(m > 0.0)) return 0.0;
  const double kmt = k * m * t;
  const double c = b - 2.0 * a;
  const double ax = fabs(c) * kmt;
  const double E = ax < 1e-8 ? 1.0 - 0.5 * ax : -expm1(-ax) / ax;
  const double s = c >= 0.0 ? 2.0 * a : b;
  return a * b * kmt * E / (1.0 + s * kmt * E);
}

// After the solve: x^(n+1) = x^n + d for the three species (FP32 state: the
// pair sum in FP64, split again), and the ledger partials of the step (the
// same tiles and slots as the field update, whose slots for the species it
// fills; its non-finite count is added to the update's).
template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_sp_finish(CellArgs<T> a, SpArgs<T> s) {
  const Grid& g = a.g;
  const int i = blockIdx.x * TX + (threadIdx.x & (TX - 1));
  const int j = blockIdx.y * TY + threadIdx.x / TX;
  const int k = blockIdx.z;
  const int pidx = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int pstride = gridDim.x * gridDim.y * gridDim.z;
  double v[6] = {0, 0, 0, 0, 0, 0};
  if (i < g.nx && j < g.ny) {
    const int e = gidx(g, i, j, k);
    const T* old[3] = {a.xO, a.xH, a.xW};
    T* nhi[3] = {a.nxO, a.nxH, a.nxW};
    double x[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      T lo = T(0);
      if constexpr (sizeof(T) == 4) lo = a.lo[2 + q][e];
      x[q] = field_new(old[q][e], lo, s.d[q][e]);
    }
    if (a.p.rsplit) {
      // the reaction over dt after the transport, with m(phi_g) of phi^n
      double pf = (double)a.pf[e], pw = (double)a.pw[e];
      if constexpr (sizeof(T) == 4) {
        pf += (double)a.lo[0][e];
        pw += (double)a.lo[1][e];
      }
      const double g = 1.0 - pf - pw, y = g * (1.0 - g);
      const double m = (a.p.mform == 0 ? 16.0 : 1.0) * y * y;
      const double R = reaction_exact(x[0], x[1], x[2], m, (double)a.p.kfor, (double)a.p.dt);
      x[0] -= R;
      x[1] -= 2.0 * R;
      x[2] += R;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) field_store(x[q], nhi[q], a.nlo[2 + q], e);
    v[0] = x[0] + x[2];
    v[1] = x[1] + 2.0 * x[2];
    v[2] = x[0];
    if (a.p.dirichlet) {
      // outward boundary fluxes with the new values, 2 D_c (x - x_bc) / h per outer face
      const int c[3] = {i, j, k}, lim[3] = {g.nx, g.ny, g.nz};
      int nf = 0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) nf += (c[d] == 0) + (c[d] + 1 == lim[d]);
      const double f = 2.0 * (double)a.p.ih * nf;
      const double bO = f * (double)s.D[2][e] * (x[2] - (double)a.p.xWbc);
      const double bH = f * (double)s.D[1][e] * (x[1] - (double)a.p.xHbc);
      v[3] = bO;
      v[4] = bH + 2.0 * bO;
    }
    v[5] = (isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2])) ? 0.0 : 1.0;
  }
  __shared__ double red[6][NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] += __shfl_xor(v[q], o, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += red[threadIdx.x][w];
    if (threadIdx.x < 5) a.part[threadIdx.x * pstride + pidx] = t;
    else a.part[7 * pstride + pidx] += t;
  }
}

}  // namespace pfk
