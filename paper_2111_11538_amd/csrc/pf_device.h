// Device-side building blocks of the gfx950 phase-field step: parameter block,
// grid layout, interpolation functions, the calibrated chemical energies and
// deterministic FP64 block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

constexpr int TX = 64;   // tile width (one wave64 per row)
constexpr int TY = 4;    // tile height; block = TX * TY = 256 threads
constexpr int NT = TX * TY;

// Device scalars shared by the solver kernels (FP64 slots).
enum Scal {
  S_CONV = 0,      // nonzero once the current solve has converged (3D CG: the index + 1
                   // of the apply launch that completes the solution)
  S_FIRST = 1,     // 1 before the first CG update of a solve
  S_ITERS = 2,     // CG updates performed in the current solve
  S_BB = 3,        // ||b||^2
  S_RZ = 4,        // r.z of the two most recent iterations (slots 4, 5)
  S_RR = 6,        // ||r||^2 of the last check
  S_TRUE = 7,      // true ||b - A u||^2 after the solve
  S_ALPHA = 8,     // alpha of the last CG update of even (slot 8) and odd (slot 9) index
  // ledger (persistent across steps)
  S_O0 = 10, S_H0 = 11, S_XO0 = 12, S_OOUT = 13, S_HOUT = 14,
  // last-step statistics
  S_OTOT = 16, S_HTOT = 17, S_XOSUM = 18, S_MAXVM = 19, S_MAXEP = 20, S_NONFIN = 21,
  // learned start: ||b - A u0||^2 of the learned and of the previous start
  S_JL = 22, S_JP = 23, S_JB = 24,
  S_COUNT = 32
};

template <typename T>
struct KP {
  T scale;                 // R theta / V_mol
  T w[3], eps[3], L[3];
  T kappaO;
  T K[3], G[3];
  T sigY, Hh;
  T DO[3], DH[3], DW[3];
  T kfor, Omega;
  T xHbc, xWbc;
  T h, ih, ih2, dt;
  int mform, dirichlet, chem, plastic, mech;
  int rsplit;              // 1: the reaction is left out of the tendencies and solved exactly after the transport
};

// Padded SoA layout shared by every cell and face array: element (i, j, k) at
// (k * ny + j) * px + i, with px >= nx a multiple of 16.  A face array stores
// the face on the low side of cell (i, j, k); the faces on the high outer
// boundary (index nx, ny or nz) are roller faces, fixed at zero and not stored.
struct Grid {
  int nx, ny, nz, px;
  int n;                   // px * ny * nz elements per array
  int ns;                  // element stride between the components of the plastic strain
};

__device__ __forceinline__ int gidx(const Grid& g, int i, int j, int k) { return (k * g.ny + j) * g.px + i; }

// Raw buffer resources: a load whose byte offset lies past num_records
// returns zero without touching memory, so a load that may or may not be
// needed can be issued unconditionally (no branch, so the compiler's wait
// counts stay exact across it).
constexpr int kBufferFlags = 0x00020000;     // raw buffer, 32-bit data format (gfx9 family)
constexpr int kOutOfRange = 0x7FFFFFF0;      // byte offset past any tensor here: the load returns zero

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const T* p, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), 0, nbytes, kBufferFlags);
}
template <typename T> __device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// FP32 to bf16, round to nearest even (finite values)
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
// a bf16 element (the upper half of an FP32 word) of a raw buffer, as FP32
__device__ __forceinline__ float buf_ld_bf16(__amdgpu_buffer_rsrc_t r, int off) {
  return __uint_as_float((unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0) << 16);
}

// MI355X has 8 XCDs, each with its own L2; workgroups are dispatched to them
// round robin by linear block id.  Map block id b to tile id so that XCD
// (b mod 8) owns the contiguous tile range [x * nb/8, (x+1) * nb/8).  Identity
// when nb is not a multiple of 8.
constexpr int kXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if (nb % kXCD) return b;
  return (b % kXCD) * (nb / kXCD) + b / kXCD;
}

template <typename T> __device__ __forceinline__ T tcbrt(T x);
template <> __device__ __forceinline__ float tcbrt<float>(float x) { return cbrtf(x); }
template <> __device__ __forceinline__ double tcbrt<double>(double x) { return cbrt(x); }
template <typename T> __device__ __forceinline__ T tsqrt(T x);
template <> __device__ __forceinline__ float tsqrt<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double tsqrt<double>(double x) { return sqrt(x); }

// ---------------------------------------------------------------------------
// Interpolation functions: h(x) = x^3 (6x^2 - 15x + 10) and the barrier
// function m, read as 16 x^2 (1-x)^2 (form 0) or x^2 (1-x)^2 (form 1).
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T interp_h(T x) { return x * x * x * (x * (T(6) * x - T(15)) + T(10)); }
template <typename T> __device__ __forceinline__ T interp_dh(T x) { T y = x * (T(1) - x); return T(30) * y * y; }
template <typename T> __device__ __forceinline__ T interp_m(T x, int form) {
  T y = x * (T(1) - x);
  return (form == 0 ? T(16) : T(1)) * y * y;
}
template <typename T> __device__ __forceinline__ T interp_dm(T x, int form) {
  return (form == 0 ? T(32) : T(2)) * x * (T(1) - x) * (T(1) - T(2) * x);
}

// Calibrated scaled chemical energies (Eq. 35 ferrite / wuestite, Eq. 36 gas)
// in Horner form: value, first and second derivative in x_O.
template <typename T> __device__ __forceinline__ void fe_ferrite(T x, T& f, T& d1, T& d2) {
  f = (((T(163.708) * x - T(182.510)) * x + T(90.573)) * x - T(36.031)) * x - T(4.372);
  d1 = ((T(654.832) * x - T(547.530)) * x + T(181.146)) * x - T(36.031);
  d2 = (T(1964.496) * x - T(1095.060)) * x + T(181.146);
}
template <typename T> __device__ __forceinline__ void fe_wuestite(T x, T& f, T& d1, T& d2) {
  f = (T(173.263) * x - T(213.460)) * x + T(41.953);
  d1 = T(346.526) * x - T(213.460);
  d2 = T(346.526);
}
template <typename T> __device__ __forceinline__ void fe_gas(T x, T& f, T& d1, T& d2) {
  f = T(1000) * x * x;
  d1 = T(2000) * x;
  d2 = T(2000);
}

// Phase-dependent quantities of one cell (phi_g = 1 - phi_f - phi_w).
template <typename T>
struct Phase {
  T hf, hg, hw, dhf, dhg, dhw;
  T dT, dTp, eT, eTp, K, G;
};

template <typename T>
__device__ __forceinline__ void phase_eval(const KP<T>& p, T pf, T pw, Phase<T>& q) {
  T pg = T(1) - pf - pw;
  q.hf = interp_h(pf); q.hg = interp_h(pg); q.hw = interp_h(pw);
  q.dhf = interp_dh(pf); q.dhg = interp_dh(pg); q.dhw = interp_dh(pw);
  q.dT = T(1) - p.Omega * q.hf;                      // Eq. 9
  q.dTp = -p.Omega * q.dhf;
  T c = tcbrt(q.dT);
  q.eT = c - T(1);                                  // small-strain eigenstrain
  q.eTp = q.dTp / (T(3) * c * c);
  q.K = q.dT * (q.hf * p.K[0] + q.hg * p.K[1] + q.hw * p.K[2]);   // Eq. 32
  q.G = q.dT * (q.hf * p.G[0] + q.hg * p.G[1] + q.hw * p.G[2]);
}

// eigenstrain only (K, G not needed)
template <typename T>
__device__ __forceinline__ T eigen_strain(const KP<T>& p, T pf) {
  return tcbrt(T(1) - p.Omega * interp_h(pf)) - T(1);
}

template <typename T>
__device__ __forceinline__ void moduli(const KP<T>& p, T pf, T pw, T& K, T& G) {
  T pg = T(1) - pf - pw;
  T hf = interp_h(pf), hg = interp_h(pg), hw = interp_h(pw);
  T dT = T(1) - p.Omega * hf;
  K = dT * (hf * p.K[0] + hg * p.K[1] + hw * p.K[2]);
  G = dT * (hf * p.G[0] + hg * p.G[1] + hw * p.G[2]);
}

// Oxygen chemistry of one cell: local chemical potential, curvature of
// psi_che, mobility M_O = D_O / psi_xx, and the phase-weighted D_H, D_H2O.
template <typename T>
__device__ __forceinline__ void transport(const KP<T>& p, T pf, T pw, T x, T& mu_loc, T& MO, T& DH, T& DW) {
  T pg = T(1) - pf - pw;
  T hf = interp_h(pf), hg = interp_h(pg), hw = interp_h(pw);
  T f0, f1, f2, g0, g1, g2, w0, w1, w2;
  fe_ferrite(x, f0, f1, f2);
  fe_gas(x, g0, g1, g2);
  fe_wuestite(x, w0, w1, w2);
  mu_loc = p.scale * (hf * f1 + hg * g1 + hw * w1);
  T pxx = p.scale * (hf * f2 + hg * g2 + hw * w2);
  T ihs = T(1) / (hf + hg + hw);
  T DO = (hf * p.DO[0] + hg * p.DO[1] + hw * p.DO[2]) * ihs;
  MO = DO / pxx;
  DH = (hf * p.DH[0] + hg * p.DH[1] + hw * p.DH[2]) * ihs;
  DW = (hf * p.DW[0] + hg * p.DW[1] + hw * p.DW[2]) * ihs;
}

// Phase-weighted oxygen diffusivity (the D_O inside M_O = D_O / psi_xx).
template <typename T>
__device__ __forceinline__ T diffusivity_O(const KP<T>& p, T pf, T pw) {
  T pg = T(1) - pf - pw;
  T hf = interp_h(pf), hg = interp_h(pg), hw = interp_h(pw);
  return (hf * p.DO[0] + hg * p.DO[1] + hw * p.DO[2]) / (hf + hg + hw);
}

template <typename T>
__device__ __forceinline__ void transport_D(const KP<T>& p, T pf, T pw, T& DH, T& DW) {
  T pg = T(1) - pf - pw;
  T hf = interp_h(pf), hg = interp_h(pg), hw = interp_h(pw);
  T ihs = T(1) / (hf + hg + hw);
  DH = (hf * p.DH[0] + hg * p.DH[1] + hw * p.DH[2]) * ihs;
  DW = (hf * p.DW[0] + hg * p.DW[1] + hw * p.DW[2]) * ihs;
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions (fixed lane / wave / thread order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the block (blockDim.x == NT); every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) s += sh[q];
  return s;
}
// Two sums over the block at once (the same operations and order as two
// block_sum calls, with two barriers instead of four); sh holds 2 * NT / 64.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) { sh[w] = a; sh[NT / 64 + w] = b; }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) { sa += sh[q]; sb += sh[NT / 64 + q]; }
  a = sa;
  b = sb;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
  v = wave_max(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = sh[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) s = fmax(s, sh[q]);
  return s;
}

// Sum over a block of NTB threads (a multiple of 64); every thread gets the result.
template <int NTB>
__device__ __forceinline__ double block_sum_n(double v, double* sh) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NTB / 64; ++q) s += sh[q];
  return s;
}

// Sum of part[0..n) in a fixed order; identical in every block.
__device__ __forceinline__ double sum_partials(const double* part, int n, double* sh) {
  double v = 0.0;
#pragma unroll 8
  for (int q = threadIdx.x; q < n; q += NT) v += part[q];
  return block_sum(v, sh);
}

}  // namespace pfk
