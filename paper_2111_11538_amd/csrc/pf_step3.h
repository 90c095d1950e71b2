// Fused 3D field update on an LDS plane tile.
//
// One block owns a 64 x 8 tile of one z plane.  The tile and its one-cell
// ring of that plane are staged once in LDS: the phase fields, x_H, x_H2O,
// mu_O, the three displacement components and the transport coefficients
// M_O, D_H, D_H2O evaluated once per staged cell.  The x and y neighbours of
// every flux, Laplacian and shear then come from LDS; the z neighbours
// (planes k - 1, k + 1) come from global memory, with their transport
// coefficients evaluated in registers.  The arithmetic of each cell is the
// same as the one-plane kernel's (cell_update): fluxes of Eq. 24, 29, the
// cell strain of the staggered grid, return map, driving forces, reaction,
// explicit update and the ledger partials.
#pragma once

#include "pf_kernels.h"

namespace pfk {

constexpr int S3_BY = 8;                       // tile rows
constexpr int S3_NT = TX * S3_BY;              // 512 threads
constexpr int S3_LX = TX + 2;                  // staged row (with the ring)
constexpr int S3_LN = S3_LX * (S3_BY + 2);     // staged cells

template <typename T>
struct Step3Smem {
  T pf[S3_LN], pw[S3_LN], xH[S3_LN], xW[S3_LN], mu[S3_LN];
  T M[S3_LN], DH[S3_LN], DW[S3_LN];
  T ux[S3_LN], uy[S3_LN], uz[S3_LN];
};

template <typename T>
__global__ __launch_bounds__(S3_NT) void k_step3(CellArgs<T> a) {
  __shared__ Step3Smem<T> s;
  __shared__ double red8[NQ_STEP][S3_NT / 64];
  const Grid& g = a.g;
  const KP<T>& p = a.p;
  const int pl = g.px * g.ny;
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * S3_BY, k = blockIdx.z;
  const T* ux = a.u[0];
  const T* uy = a.u[1];
  const T* uz = a.u[2];
  // stage plane k of the tile and its ring
  for (int q = threadIdx.x; q < S3_LN; q += S3_NT) {
    const int li = q % S3_LX, lj = q / S3_LX;
    const int gi = i0 + li - 1, gj = j0 + lj - 1;
    T vpf = T(0), vpw = T(0), vxO = T(0), vxH = T(0), vxW = T(0), vmu = T(0), vux = T(0), vuy = T(0), vuz = T(0);
    if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny) {
      const int e = gidx(g, gi, gj, k);
      vpf = a.pf[e]; vpw = a.pw[e]; vxO = a.xO[e]; vxH = a.xH[e]; vxW = a.xW[e]; vmu = a.mu[e];
      if (p.mech) { vux = ux[e]; vuy = uy[e]; vuz = uz[e]; }
    }
    T m_, M, DH, DW;
    transport(p, vpf, vpw, vxO, m_, M, DH, DW);
    s.pf[q] = vpf; s.pw[q] = vpw; s.xH[q] = vxH; s.xW[q] = vxW; s.mu[q] = vmu;
    s.M[q] = M; s.DH[q] = DH; s.DW[q] = DW;
    s.ux[q] = vux; s.uy[q] = vuy; s.uz[q] = vuz;
  }
  __syncthreads();
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int i = i0 + tx, j = j0 + ty;
  double acc[NQ_STEP] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < g.nx && j < g.ny) {
    const int e = gidx(g, i, j, k);
    const int c = (ty + 1) * S3_LX + (tx + 1);
    const T ih = p.ih;
    const T pf = s.pf[c], pw = s.pw[c], xH = s.xH[c], xW = s.xW[c], muc = s.mu[c];
    const T xO = a.xO[e];
    const T MOc = s.M[c], DHc = s.DH[c], DWc = s.DW[c];
    T lo[5] = {T(0), T(0), T(0), T(0), T(0)};
    if constexpr (sizeof(T) == 4)
#pragma unroll
      for (int f = 0; f < 5; ++f) lo[f] = a.lo[f][e];
    T lf = T(0), lw = T(0), divO = T(0), divH = T(0), divW = T(0);
    T bO = T(0), bH = T(0);
    // faces on the low and high side of direction d: neighbour values
    // (from LDS for x, y; from global memory with its transport for z)
    auto faces = [&](bool has_lo, bool has_hi, T pfl, T pwl, T mul, T Ml, T DHl, T DWl, T xHl, T xWl, T pfh, T pwh,
                     T muh, T Mh, T DHh, T DWh, T xHh, T xWh) {
      lf += (has_hi ? pfh - pf : T(0)) - (has_lo ? pf - pfl : T(0));
      lw += (has_hi ? pwh - pw : T(0)) - (has_lo ? pw - pwl : T(0));
      T JOm = T(0), JOp = T(0), JHm, JHp, JWm, JWp;
      if (has_lo) {
        JOm = face_flux(Ml, MOc, mul, muc, ih);
        JHm = face_flux(DHl, DHc, xHl, xH, ih);
        JWm = face_flux(DWl, DWc, xWl, xW, ih);
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
        JOp = face_flux(MOc, Mh, muc, muh, ih);
        JHp = face_flux(DHc, DHh, xH, xHh, ih);
        JWp = face_flux(DWc, DWh, xW, xWh, ih);
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
    };
    {
      const int l = c - 1, r = c + 1;
      faces(i > 0, i + 1 < g.nx, s.pf[l], s.pw[l], s.mu[l], s.M[l], s.DH[l], s.DW[l], s.xH[l], s.xW[l], s.pf[r],
            s.pw[r], s.mu[r], s.M[r], s.DH[r], s.DW[r], s.xH[r], s.xW[r]);
    }
    {
      const int l = c - S3_LX, r = c + S3_LX;
      faces(j > 0, j + 1 < g.ny, s.pf[l], s.pw[l], s.mu[l], s.M[l], s.DH[l], s.DW[l], s.xH[l], s.xW[l], s.pf[r],
            s.pw[r], s.mu[r], s.M[r], s.DH[r], s.DW[r], s.xH[r], s.xW[r]);
    }
    {
      const bool hl = k > 0, hh = k + 1 < g.nz;
      const int el = hl ? e - pl : e, eh = hh ? e + pl : e;
      const T pfl = a.pf[el], pwl = a.pw[el], pfh = a.pf[eh], pwh = a.pw[eh];
      T m_, Ml, DHl, DWl, Mh, DHh, DWh;
      transport(p, pfl, pwl, a.xO[el], m_, Ml, DHl, DWl);
      transport(p, pfh, pwh, a.xO[eh], m_, Mh, DHh, DWh);
      faces(hl, hh, pfl, pwl, a.mu[el], Ml, DHl, DWl, a.xH[el], a.xW[el], pfh, pwh, a.mu[eh], Mh, DHh, DWh, a.xH[eh],
            a.xW[eh]);
    }
    T eb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (p.mech) {
      eb[0] = ((i + 1 < g.nx ? s.ux[c + 1] : T(0)) - s.ux[c]) * ih;
      eb[1] = ((j + 1 < g.ny ? s.uy[c + S3_LX] : T(0)) - s.uy[c]) * ih;
      eb[2] = ((k + 1 < g.nz ? uz[e + pl] : T(0)) - s.uz[c]) * ih;
      // shear at the four xy edges of the cell (plane k, all in LDS)
      T sxy = T(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ai = i + (q & 1), bj = j + (q >> 1);
        if (ai > 0 && ai < g.nx && bj > 0 && bj < g.ny) {
          const int ca = c + (q & 1) + (q >> 1) * S3_LX;
          sxy += T(0.5) * ((s.ux[ca] - s.ux[ca - S3_LX]) + (s.uy[ca] - s.uy[ca - 1])) * ih;
        }
      }
      eb[3] = T(0.25) * sxy;
      // xz and yz edges: planes k and k + 1
      T sxz = T(0), syz = T(0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int da = q & 1, dk = q >> 1;
        const int ck = k + dk;
        if (ck > 0 && ck < g.nz) {
          {
            const int ai = i + da;
            if (ai > 0 && ai < g.nx) {
              const int ca = c + da;
              const T ux_c = dk ? ux[e + da + pl] : s.ux[ca];
              const T ux_m = dk ? s.ux[ca] : ux[e + da - pl];
              const T uz_c = dk ? uz[e + da + pl] : s.uz[ca];
              const T uz_m = dk ? uz[e + da - 1 + pl] : s.uz[ca - 1];
              sxz += T(0.5) * ((ux_c - ux_m) + (uz_c - uz_m)) * ih;
            }
          }
          {
            const int bj = j + da;
            if (bj > 0 && bj < g.ny) {
              const int ca = c + da * S3_LX;
              const int eo = e + da * g.px;
              const T uy_c = dk ? uy[eo + pl] : s.uy[ca];
              const T uy_m = dk ? s.uy[ca] : uy[eo - pl];
              const T uz_c = dk ? uz[eo + pl] : s.uz[ca];
              const T uz_m = dk ? uz[eo - g.px + pl] : s.uz[ca - S3_LX];
              syz += T(0.5) * ((uy_c - uy_m) + (uz_c - uz_m)) * ih;
            }
          }
        }
      }
      eb[4] = T(0.25) * sxz;
      eb[5] = T(0.25) * syz;
    }
    cell_update<T, 3>(a, e, pf, pw, xO, xH, xW, lf, lw, divO, divH, divW, bO, bH, eb, lo, DHc, DWc, acc);
  }
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
    double sum = red8[qn][0];
#pragma unroll
    for (int q = 1; q < S3_NT / 64; ++q) sum = mx ? fmax(sum, red8[qn][q]) : sum + red8[qn][q];
    const int pidx = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    a.part[qn * (gridDim.x * gridDim.y * gridDim.z) + pidx] = sum;
  }
}

}  // namespace pfk
