// Device kernels of the learned warm start: a stack of 3x3x3 'same'
// convolutions (zero padding, ReLU between layers, linear output) on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: bf16 operands, fp32
// accumulation), its backward passes, the relative mean-square loss, Adam,
// and the packing between the simulation state and the network.
//
// Tensors are channel-last bf16: voxel v of n volumes of D x H x W voxels,
// channel c at v * C + c.  Layer l maps C_in to C_out channels with weights
// W[t][co][ci], t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) reading voxel
// (z + dz, y + dy, x + dx).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_device.h"

namespace pfn {

using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using f32x4 = float __attribute__((ext_vector_type(4)));

constexpr int CNT = 256;       // threads per block (4 waves)
constexpr int SEG = 64;        // voxels per wave along x in the convolutions (4 column blocks of 16)
constexpr int NBW = SEG / 16;
constexpr int kTaps = 27;

struct Vol {
  int n, D, H, W;              // n volumes of D x H x W voxels
};

__device__ __forceinline__ uint16_t f2bf(float f) {     // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bool bf_pos(uint32_t h) { return (h & 0x8000u) == 0u && (h & 0x7FFFu) != 0u; }
__device__ __forceinline__ bf16x8 as_bf8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}
__device__ __forceinline__ uint32_t pack2(float a, float b) { return (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16); }

__device__ __forceinline__ void tap_offset(int t, int& dz, int& dy, int& dx) {
  dz = t / 9 - 1;
  dy = (t / 3) % 3 - 1;
  dx = t % 3 - 1;
}

// ---------------------------------------------------------------------------
// Convolution as an implicit GEMM: out^T (co x voxels) = W (co x k) * in (k x voxels),
// k = t * CIN + ci.  The weights arrive as an image in MFMA operand order: for
// output block mb and 32-wide k chunk kc, lane l holds the 8 values
// W(co = 16 mb + l % 16, k = 32 kc + 8 (l / 16) + j), j = 0..7; entries past
// the real channel counts or past tap 26 are zero.  One wave computes 64
// consecutive voxels of one row for all output channels; a block of 8 waves
// takes 8 consecutive rows and shares one LDS copy of the weight image.
//   EPI_RELU:   out (bf16, 16 MB channels) = max(acc + bias, 0)
//   EPI_LINEAR: out (fp32, 4 channels)     = acc + bias, channels 0..3 of block 0
//   EPI_MASK:   out (bf16, 16 MB channels) = acc where mask > 0, else 0
// ---------------------------------------------------------------------------
enum Epi { EPI_RELU = 0, EPI_LINEAR = 1, EPI_MASK = 2 };

template <int CIN>
constexpr int k_chunks() { return (kTaps * CIN + 31) / 32; }

constexpr int CONV_WAVES = 8;              // waves (rows of a tile) per convolution block
constexpr int CONV_NT = CONV_WAVES * 64;


// Input fragment of one 16-voxel column block for k chunk kc: lane (lr, lg)
// holds the 8 channels ci0..ci0+7 of voxel (x + lr + dx, y + dy, z + dz),
// loaded through a buffer resource over the whole input so that voxels
// outside the volume read as zero without branches.
template <int CIN>
__device__ __forceinline__ void conv_load_b(__amdgpu_buffer_rsrc_t rs, const Vol& v, int n, int z, int y, int x0,
                                            int kc, int lr, int lg, uint4 (&b)[NBW]) {
  const int k0 = kc * 32 + lg * 8;
  const int tap = k0 / CIN, ci0 = k0 % CIN;
  int dz, dy, dx;
  tap_offset(tap, dz, dy, dx);
  const int zz = z + dz, yy = y + dy;
  const bool rok = tap < kTaps && zz >= 0 && zz < v.D && yy >= 0 && yy < v.H;
  const int rowv = ((n * v.D + zz) * v.H + yy) * v.W;
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    const int xx = x0 + nb * 16 + lr + dx;
    const int off = (rok && xx >= 0 && xx < v.W) ? ((rowv + xx) * CIN + ci0) * 2 : kOutOfRange;
    const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    b[nb] = uint4{q[0], q[1], q[2], q[3]};
  }
}

template <int CIN, int MB, int EPI>
__global__ __launch_bounds__(CONV_NT) void k_conv(const uint4* __restrict__ wimg, const float* __restrict__ bias,
                                                  const uint16_t* __restrict__ x, void* __restrict__ out,
                                                  const uint16_t* __restrict__ mask, Vol v) {
  constexpr int KC = k_chunks<CIN>();
  constexpr int COUT = MB * 16;
  extern __shared__ uint4 sW[];
  for (int i = threadIdx.x; i < MB * KC * 64; i += CONV_NT) sW[i] = wimg[i];
  __syncthreads();
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint16_t*>(x), 0, (int)((long)v.n * v.D * v.H * v.W * CIN * 2), kBufferFlags);
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lr = lane & 15, lg = lane >> 4;
  const int nseg = (v.W + SEG - 1) / SEG, nyt = (v.H + CONV_WAVES - 1) / CONV_WAVES;
  const long ntiles = (long)nseg * nyt * v.D * v.n;
  for (long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int xs = (int)(t % nseg);
    long r = t / nseg;
    const int y = (int)(r % nyt) * CONV_WAVES + wv;
    r /= nyt;
    const int z = (int)(r % v.D);
    const int n = (int)(r / v.D);
    if (y >= v.H) continue;                     // whole wave; no block barrier follows
    const int x0 = xs * SEG;
    f32x4 acc[MB][NBW];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the fragments of chunk kc + 1 are in flight while chunk kc is
    // multiplied; the two fragment sets alternate roles, and the scheduling
    // barriers keep the compiler from sinking the loads below the multiplies
    auto mul = [&](int kc, const uint4 (&bc)[NBW]) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const bf16x8 a = as_bf8(sW[(mb * KC + kc) * 64 + lane]);
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_bf8(bc[nb]), acc[mb][nb], 0, 0, 0);
      }
    };
    uint4 fa[NBW], fb[NBW];
    conv_load_b<CIN>(rs, v, n, z, y, x0, 0, lr, lg, fa);
    int kc = 0;
    for (; kc + 2 < KC; kc += 2) {
      conv_load_b<CIN>(rs, v, n, z, y, x0, kc + 1, lr, lg, fb);
      __builtin_amdgcn_sched_barrier(0);
      mul(kc, fa);
      conv_load_b<CIN>(rs, v, n, z, y, x0, kc + 2, lr, lg, fa);
      __builtin_amdgcn_sched_barrier(0);
      mul(kc + 1, fb);
    }
    if (kc + 1 < KC) {
      conv_load_b<CIN>(rs, v, n, z, y, x0, kc + 1, lr, lg, fb);
      __builtin_amdgcn_sched_barrier(0);
      mul(kc, fa);
      mul(kc + 1, fb);
    } else {
      mul(kc, fa);
    }
    // lane holds out(co = 16 mb + 4 lg + i, voxel = 16 nb + lr)
    const long vrow = (((long)n * v.D + z) * v.H + y) * v.W;
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      const int xx = x0 + nb * 16 + lr;
      if (xx >= v.W) continue;
      const long vox = vrow + xx;
      if constexpr (EPI == EPI_LINEAR) {
        if (lg == 0) {
          float4 o;
          o.x = acc[0][nb][0] + bias[0];
          o.y = acc[0][nb][1] + bias[1];
          o.z = acc[0][nb][2] + bias[2];
          o.w = acc[0][nb][3] + bias[3];
          reinterpret_cast<float4*>(out)[vox] = o;
        }
      } else {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int co0 = mb * 16 + lg * 4;
          float o[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) o[i] = acc[mb][nb][i];
          if constexpr (EPI == EPI_RELU) {
#pragma unroll
            for (int i = 0; i < 4; ++i) o[i] = fmaxf(o[i] + bias[co0 + i], 0.f);
          } else {
            const uint2 mk = *reinterpret_cast<const uint2*>(mask + vox * COUT + co0);
            if (!bf_pos(mk.x & 0xFFFFu)) o[0] = 0.f;
            if (!bf_pos(mk.x >> 16)) o[1] = 0.f;
            if (!bf_pos(mk.y & 0xFFFFu)) o[2] = 0.f;
            if (!bf_pos(mk.y >> 16)) o[3] = 0.f;
          }
          uint2 st;
          st.x = pack2(o[0], o[1]);
          st.y = pack2(o[2], o[3]);
          *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(out) + vox * COUT + co0) = st;
        }
      }
    }
  }
}

// Convolution with 32 input channels, reusing each input fragment for the three
// x taps.  For a fixed (dz, dy) a wave loads the 64 input voxels x0..x0+63 of
// its output row once (four 16-voxel fragments, one per 16-lane row of the
// wave: lane (lr, lg) holds channels 8 lg..8 lg+7 of voxel lr) plus one halo
// fragment (lanes lr = 0 / 1: voxels x0 - 1 / x0 + 64).  The fragments of the
// dx = -1 and dx = +1 taps are the same data moved by one lane within each
// 16-lane row (DPP row shifts), the lane that leaves the row being filled from
// the neighbouring fragment; all three taps accumulate into one accumulator.

// Move of one 32-bit lane value within 16-lane rows (DPP).  Lanes whose
// source lies outside the row keep `old`.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xF, 0xF, false);
}
constexpr int kRowShl1 = 0x101;   // lane i <- lane i + 1 (lane 15 keeps old)
constexpr int kRowShr1 = 0x111;   // lane i <- lane i - 1 (lane 0 keeps old)
constexpr int kRowRor1 = 0x121;   // lane i <- lane (i - 1) mod 16
constexpr int kRowRor14 = 0x12E;  // lane i <- lane (i + 2) mod 16
constexpr int kRowRor15 = 0x12F;  // lane i <- lane (i + 1) mod 16

template <int CTRL>
__device__ __forceinline__ uint4 dpp4(uint4 old, uint4 src) {
  return uint4{dpp_mov<CTRL>(old.x, src.x), dpp_mov<CTRL>(old.y, src.y), dpp_mov<CTRL>(old.z, src.z),
               dpp_mov<CTRL>(old.w, src.w)};
}
template <int CTRL>
__device__ __forceinline__ uint4 dpp4(uint4 src) {
  return dpp4<CTRL>(src, src);
}

template <int MB, int EPI>
__global__ __launch_bounds__(CONV_NT) void k_conv32(const uint4* __restrict__ wimg, const float* __restrict__ bias,
                                                    const uint16_t* __restrict__ x, void* __restrict__ out,
                                                    const uint16_t* __restrict__ mask, Vol v) {
  constexpr int CIN = 32;
  constexpr int KC = kTaps;                    // one k chunk per tap
  constexpr int COUT = MB * 16;
  extern __shared__ uint4 sW[];
  for (int i = threadIdx.x; i < MB * KC * 64; i += CONV_NT) sW[i] = wimg[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lr = lane & 15, lg = lane >> 4;
  const int nseg = (v.W + SEG - 1) / SEG, nyt = (v.H + CONV_WAVES - 1) / CONV_WAVES;
  const long ntiles = (long)nseg * nyt * v.D * v.n;
  // each block walks a contiguous run of tiles, z fastest, so the input planes
  // shared by consecutive tiles are reused from its XCD's L2
  const long t0 = ntiles * blockIdx.x / gridDim.x, t1 = ntiles * (blockIdx.x + 1) / gridDim.x;
  for (long t = t0; t < t1; ++t) {
    const int z = (int)(t % v.D);
    long r = t / v.D;
    const int xs = (int)(r % nseg);
    r /= nseg;
    const int y = (int)(r % nyt) * CONV_WAVES + wv;
    const int n = (int)(r / nyt);
    if (y >= v.H) continue;                     // whole wave; no block barrier follows
    const int x0 = xs * SEG;
    f32x4 acc[MB][NBW];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Branch-free loads through a buffer resource spanning one input row: the
    // hardware range check returns zero for voxels outside the row (offset
    // pushed past the end) and for rows outside the volume (empty range).
    // b[NBW] is the halo fragment: lane 0 voxel x0 - 1, lane 1 voxel x0 + 64.
    const int xh = lr == 0 ? x0 - 1 : (lr == 1 ? x0 + SEG : -1);
    auto load = [&](int c, uint4 (&b)[NBW + 1]) {   // c = 3 (dz + 1) + (dy + 1)
      const int zz = z + c / 3 - 1, yy = y + c % 3 - 1;
      const bool rok = zz >= 0 && zz < v.D && yy >= 0 && yy < v.H;
      const uint16_t* row = rok ? x + ((((long)n * v.D + zz) * v.H + yy) * v.W) * CIN : x;
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(row), 0, rok ? v.W * CIN * 2 : 0, kBufferFlags);
#pragma unroll
      for (int nb = 0; nb <= NBW; ++nb) {
        const int xx = nb < NBW ? x0 + nb * 16 + lr : xh;
        const int off = (xx >= 0 && xx < v.W) ? (xx * CIN + lg * 8) * 2 : kOutOfRange;
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        b[nb] = uint4{q[0], q[1], q[2], q[3]};
      }
    };
    // the fragments of the next (dz, dy) pair are in flight while one is
    // multiplied; the two fragment sets alternate roles (no copies, so the
    // wait before a multiply leaves the newer loads outstanding)
    auto pair = [&](int c, const uint4 (&bc)[NBW + 1]) {
      bf16x8 wm[MB], w0[MB], wp[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        wm[mb] = as_bf8(sW[(mb * KC + 3 * c + 0) * 64 + lane]);
        w0[mb] = as_bf8(sW[(mb * KC + 3 * c + 1) * 64 + lane]);
        wp[mb] = as_bf8(sW[(mb * KC + 3 * c + 2) * 64 + lane]);
      }
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        // dx = -1: voxel lr - 1; lane 0 takes lane 15 of the previous fragment
        // (for the first, the halo's lane 0, voxel x0 - 1)
        const uint4 bm = dpp4<kRowShr1>(nb > 0 ? dpp4<kRowRor1>(bc[nb - 1]) : bc[NBW], bc[nb]);
        // dx = +1: voxel lr + 1; lane 15 takes lane 0 of the next fragment
        // (for the last, the halo's lane 1, voxel x0 + 64)
        const uint4 bp = dpp4<kRowShl1>(nb + 1 < NBW ? dpp4<kRowRor15>(bc[nb + 1]) : dpp4<kRowRor14>(bc[NBW]), bc[nb]);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wm[mb], as_bf8(bm), acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0[mb], as_bf8(bc[nb]), acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wp[mb], as_bf8(bp), acc[mb][nb], 0, 0, 0);
        }
      }
    };
    // (the scheduling barriers keep the compiler from sinking the loads of
    // the next pair below the multiplies of this one)
    uint4 fa[NBW + 1], fb[NBW + 1];
    load(0, fa);
    for (int c = 0; c < 8; c += 2) {
      load(c + 1, fb);
      __builtin_amdgcn_sched_barrier(0);
      pair(c, fa);
      load(c + 2, fa);
      __builtin_amdgcn_sched_barrier(0);
      pair(c + 1, fb);
    }
    pair(8, fa);
    // lane holds out(co = 16 mb + 4 lg + i, voxel = 16 nb + lr)
    const long vrow = (((long)n * v.D + z) * v.H + y) * v.W;
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      f32x4 o[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) o[mb] = acc[mb][nb];
      const int xx = x0 + nb * 16 + lr;
      if (xx >= v.W) continue;
      const long vox = vrow + xx;
      if constexpr (EPI == EPI_LINEAR) {
        if (lg == 0)
          reinterpret_cast<float4*>(out)[vox] =
              make_float4(o[0][0] + bias[0], o[0][1] + bias[1], o[0][2] + bias[2], o[0][3] + bias[3]);
      } else {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int co0 = mb * 16 + lg * 4;
          float q[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) q[i] = o[mb][i];
          if constexpr (EPI == EPI_RELU) {
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = fmaxf(q[i] + bias[co0 + i], 0.f);
          } else {
            const uint2 mk = *reinterpret_cast<const uint2*>(mask + vox * COUT + co0);
            if (!bf_pos(mk.x & 0xFFFFu)) q[0] = 0.f;
            if (!bf_pos(mk.x >> 16)) q[1] = 0.f;
            if (!bf_pos(mk.y & 0xFFFFu)) q[2] = 0.f;
            if (!bf_pos(mk.y >> 16)) q[3] = 0.f;
          }
          uint2 st;
          st.x = pack2(q[0], q[1]);
          st.y = pack2(q[2], q[3]);
          *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(out) + vox * COUT + co0) = st;
        }
      }
    }
  }
}

// The output layer (32 -> 3 channels, one 16-channel block) moves far more
// bytes than it multiplies, so it marches along z instead: a wave owns one
// output row (64 voxels of row y) through a run of up to kOutZ planes, and
// each input plane p it loads (its rows y - 1, y, y + 1) feeds the three
// output planes p + 1, p and p - 1 it touches (taps dz = -1, 0, +1), kept
// in three accumulator sets that rotate as the march goes on; output plane
// p - 1 is complete after plane p and is stored then.  An input row is thus
// loaded once per plane by the wave instead of three times, and the 8 waves
// of a block (8 consecutive rows) share their rows through the caches.
// The x taps are the DPP row shifts of the 32-channel kernel.
constexpr int kOutZ = 32;

template <int EPI>
__global__ __launch_bounds__(CONV_NT) void k_conv32_out(const uint4* __restrict__ wimg, const float* __restrict__ bias,
                                                        const uint16_t* __restrict__ x, float* __restrict__ out,
                                                        Vol v) {
  static_assert(EPI == EPI_LINEAR, "the z march serves the linear output layer");
  constexpr int CIN = 32;
  constexpr int KC = kTaps;
  extern __shared__ uint4 sW[];
  for (int i = threadIdx.x; i < KC * 64; i += CONV_NT) sW[i] = wimg[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int lr = lane & 15, lg = lane >> 4;
  const int nseg = (v.W + SEG - 1) / SEG, nyt = (v.H + CONV_WAVES - 1) / CONV_WAVES, nzc = (v.D + kOutZ - 1) / kOutZ;
  const long nitems = (long)nseg * nyt * nzc * v.n;
  for (long t = blockIdx.x; t < nitems; t += gridDim.x) {
    const int xs = (int)(t % nseg);
    long r = t / nseg;
    const int y = (int)(r % nyt) * CONV_WAVES + wv;
    r /= nyt;
    const int zc = (int)(r % nzc);
    const int n = (int)(r / nzc);
    if (y >= v.H) continue;                     // whole wave; no block barrier follows
    const int x0 = xs * SEG;
    const int z0 = zc * kOutZ, z1 = min(z0 + kOutZ, v.D);
    const int xh = lr == 0 ? x0 - 1 : (lr == 1 ? x0 + SEG : -1);
    // fragments of input row (p, yy): four 16-voxel blocks and the halo
    // (lane 0: voxel x0 - 1, lane 1: voxel x0 + 64); zero outside the volume
    auto load = [&](int p, int yy, uint4 (&b)[NBW + 1]) __attribute__((always_inline)) {
      const bool rok = p >= 0 && p < v.D && yy >= 0 && yy < v.H;
      const uint16_t* row = rok ? x + ((((long)n * v.D + p) * v.H + yy) * v.W) * CIN : x;
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(row), 0, rok ? v.W * CIN * 2 : 0, kBufferFlags);
#pragma unroll
      for (int nb = 0; nb <= NBW; ++nb) {
        const int xx = nb < NBW ? x0 + nb * 16 + lr : xh;
        const int off = (xx >= 0 && xx < v.W) ? (xx * CIN + lg * 8) * 2 : kOutOfRange;
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        b[nb] = uint4{q[0], q[1], q[2], q[3]};
      }
    };
    // acc[0]: output plane p - 1 (tap dz = +1), acc[1]: p (dz = 0), acc[2]: p + 1 (dz = -1)
    f32x4 acc[3][NBW];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) acc[s][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // one input row (p, y + dyo): its three x shifts times the weights of the
    // three output planes it reaches
    auto row_mul = [&](int dy, const uint4 (&bc)[NBW + 1]) __attribute__((always_inline)) {
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const uint4 bm = dpp4<kRowShr1>(nb > 0 ? dpp4<kRowRor1>(bc[nb - 1]) : bc[NBW], bc[nb]);
        const uint4 bp = dpp4<kRowShl1>(nb + 1 < NBW ? dpp4<kRowRor15>(bc[nb + 1]) : dpp4<kRowRor14>(bc[NBW]), bc[nb]);
#pragma unroll
        for (int s = 0; s < 3; ++s) {            // s = 0: dz = +1, 1: dz = 0, 2: dz = -1
          const int c = 3 * (2 - s) + dy;        // tap row c = 3 (dz + 1) + (dy + 1)
          const bf16x8 wm = as_bf8(sW[(3 * c + 0) * 64 + lane]);
          const bf16x8 w0 = as_bf8(sW[(3 * c + 1) * 64 + lane]);
          const bf16x8 wp = as_bf8(sW[(3 * c + 2) * 64 + lane]);
          acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wm, as_bf8(bm), acc[s][nb], 0, 0, 0);
          acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, as_bf8(bc[nb]), acc[s][nb], 0, 0, 0);
          acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wp, as_bf8(bp), acc[s][nb], 0, 0, 0);
        }
      }
    };
    // rows in march order: (p, y - 1), (p, y), (p, y + 1), (p + 1, y - 1), ...
    // for p = z0 - 1 .. z1; the next row's fragments load while one multiplies
    uint4 bc[NBW + 1], bn[NBW + 1];
    load(z0 - 1, y - 1, bc);
    for (int p = z0 - 1; p <= z1; ++p) {
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int pn = dy < 2 ? p : p + 1, yn = dy < 2 ? y + dy : y - 1;
        if (pn <= z1) load(pn, yn, bn);
        row_mul(dy, bc);
#pragma unroll
        for (int nb = 0; nb <= NBW; ++nb) bc[nb] = bn[nb];
      }
      // output plane p - 1 is complete; lane holds out(co = 4 lg + i, voxel = 16 nb + lr)
      if (p - 1 >= z0 && lg == 0) {
        const long vrow = (((long)n * v.D + (p - 1)) * v.H + y) * v.W;
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) {
          const int xx = x0 + nb * 16 + lr;
          if (xx < v.W)
            reinterpret_cast<float4*>(out)[vrow + xx] =
                make_float4(acc[0][nb][0] + bias[0], acc[0][nb][1] + bias[1], acc[0][nb][2] + bias[2],
                            acc[0][nb][3] + bias[3]);
        }
      }
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        acc[0][nb] = acc[1][nb];
        acc[1][nb] = acc[2][nb];
        acc[2][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[t][co][ci] = sum_v dy(v, co) x(v + d(t), ci).  Grid
// (nsplit, 27): block (s, t) contracts its share of voxel rows for tap t on
// MFMA with M = output channel, N = input channel and K = 32 voxels along x,
// then reduces its 4 waves in a fixed order and writes one partial
// part[s][t][COUTP][CINP].  dy holds CG channels (CG <= COUTP), x holds CIN.
// ---------------------------------------------------------------------------
template <int CIN, int CG, int MB>
__global__ __launch_bounds__(CNT) void k_conv_wgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy,
                                                    float* __restrict__ part, Vol v) {
  constexpr int NB = (CIN + 15) / 16;
  constexpr int COUTP = MB * 16, CINP = NB * 16;
  constexpr int NACC = MB * NB * 4;
  __shared__ float red[4][NACC][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int tap = blockIdx.y;
  int dz, dyo, dx;
  tap_offset(tap, dz, dyo, dx);
  const long rows = (long)v.n * v.D * v.H;
  const long r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  f32x4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long r = r0 + wv; r < r1; r += 4) {
    const int y = (int)(r % v.H);
    const long q = r / v.H;
    const int z = (int)(q % v.D);
    const int n = (int)(q / v.D);
    const int zz = z + dz, yy = y + dyo;
    const bool rok = zz >= 0 && zz < v.D && yy >= 0 && yy < v.H;
    const uint16_t* grow = dy + r * v.W * CG;
    const uint16_t* xrow = x + ((((long)n * v.D + zz) * v.H + yy) * v.W) * CIN;
    for (int xs = 0; xs < v.W; xs += 32) {
      bf16x8 a[MB], b[NB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int co = mb * 16 + lr;
        uint16_t h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int xv = xs + 8 * lg + j;
          h[j] = (co < CG && xv < v.W) ? grow[(long)xv * CG + co] : (uint16_t)0;
        }
        __builtin_memcpy(&a[mb], h, 16);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int ci = nb * 16 + lr;
        uint16_t h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int xv = xs + 8 * lg + j + dx;
          h[j] = (rok && ci < CIN && xv >= 0 && xv < v.W && xs + 8 * lg + j < v.W) ? xrow[(long)xv * CIN + ci] : (uint16_t)0;
        }
        __builtin_memcpy(&b[nb], h, 16);
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wv][(mb * NB + nb) * 4 + i][lane] = acc[mb][nb][i];
  __syncthreads();
  float* dst = part + ((long)blockIdx.x * kTaps + tap) * COUTP * CINP;
  for (int e = threadIdx.x; e < NACC * 64; e += CNT) {
    const int slot = e / 64, l = e % 64;
    const float s = ((red[0][slot][l] + red[1][slot][l]) + red[2][slot][l]) + red[3][slot][l];
    const int mb = slot / (NB * 4), nb = (slot / 4) % NB, i = slot % 4;
    const int co = mb * 16 + 4 * (l >> 4) + i, ci = nb * 16 + (l & 15);
    dst[co * CINP + ci] = s;
  }
}

// Sum of the weight-gradient partials over splits in a fixed order (FP64),
// written in the canonical layout W[t][co][ci] of the real channel counts.
__global__ __launch_bounds__(CNT) void k_wgrad_reduce(const float* __restrict__ part, int nsplit, int coutp, int cinp,
                                                      int cout, int cin, float* __restrict__ grad) {
  const int n = kTaps * cout * cin;
  for (int e = blockIdx.x * CNT + threadIdx.x; e < n; e += gridDim.x * CNT) {
    const int t = e / (cout * cin), co = (e / cin) % cout, ci = e % cin;
    const long off = ((long)t * coutp + co) * cinp + ci;
    // four interleaved partial sums (four loads in flight), combined in a fixed order
    const long st = (long)kTaps * coutp * cinp;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = 0;
    for (; q + 3 < nsplit; q += 4) {
      s0 += (double)part[(long)q * st + off];
      s1 += (double)part[(long)(q + 1) * st + off];
      s2 += (double)part[(long)(q + 2) * st + off];
      s3 += (double)part[(long)(q + 3) * st + off];
    }
    for (; q < nsplit; ++q) s0 += (double)part[(long)q * st + off];
    grad[e] = (float)((s0 + s1) + (s2 + s3));
  }
}

// Bias gradient: db[c] = sum_v dy(v, c), dy holding cg bf16 channels per voxel
// (cg = 8 or 32).  Block s sums its voxel range: a thread reads 8 channels of
// a voxel at once (16 bytes), keeps their FP64 sums and has four such loads
// in flight; the block's threads are then combined per channel in a fixed
// order.  k_bgrad_reduce sums over the blocks.
__device__ __forceinline__ void bgrad_add8(double (&s)[8], const uint4 w) {
  const uint32_t x[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    s[2 * m] += (double)bf2f((uint16_t)(x[m] & 0xFFFFu));
    s[2 * m + 1] += (double)bf2f((uint16_t)(x[m] >> 16));
  }
}
__global__ __launch_bounds__(CNT) void k_bgrad_part(const uint16_t* __restrict__ dy, int cg, long nvox, double* __restrict__ part) {
  __shared__ double sh[8][CNT];
  const long v0 = nvox * blockIdx.x / gridDim.x, v1 = nvox * (blockIdx.x + 1) / gridDim.x;
  const int tpv = cg / 8;                      // threads per voxel
  const int vpb = CNT / tpv;                   // voxels per pass of the block
  const int q = threadIdx.x % tpv, sub = threadIdx.x / tpv;
  const uint4* rows = reinterpret_cast<const uint4*>(dy);
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  long vv = v0 + sub;
  for (; vv + 3L * vpb < v1; vv += 4L * vpb) {
    uint4 w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = rows[(vv + (long)k * vpb) * tpv + q];
#pragma unroll
    for (int k = 0; k < 4; ++k) bgrad_add8(s, w[k]);
  }
  for (; vv < v1; vv += vpb) bgrad_add8(s, rows[vv * tpv + q]);
#pragma unroll
  for (int i = 0; i < 8; ++i) sh[i][threadIdx.x] = s[i];
  __syncthreads();
  if (threadIdx.x < cg) {
    const int qq = threadIdx.x / 8, i = threadIdx.x % 8;   // channel 8 qq + i
    double t = 0.0;
    for (int u = 0; u < vpb; ++u) t += sh[i][u * tpv + qq];
    part[(long)blockIdx.x * cg + threadIdx.x] = t;
  }
}
// Sum over the blocks' partials: one block, channel c = t % cg taken by
// CNT / cg interleaved splits of the partials (four loads in flight each),
// the splits combined in a fixed order.
__global__ __launch_bounds__(CNT) void k_bgrad_reduce(const double* __restrict__ part, int nblk, int cg, int cout,
                                                      float* __restrict__ grad) {
  __shared__ double sh[CNT];
  const int c = threadIdx.x % cg, sp = threadIdx.x / cg, nsp = CNT / cg;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int q = sp;
  for (; q + 3 * nsp < nblk; q += 4 * nsp) {
    a0 += part[(long)q * cg + c];
    a1 += part[(long)(q + nsp) * cg + c];
    a2 += part[(long)(q + 2 * nsp) * cg + c];
    a3 += part[(long)(q + 3 * nsp) * cg + c];
  }
  for (; q < nblk; q += nsp) a0 += part[(long)q * cg + c];
  sh[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (threadIdx.x < cout) {
    double t = 0.0;
    for (int u = 0; u < nsp; ++u) t += sh[u * cg + threadIdx.x];
    grad[threadIdx.x] = (float)t;
  }
}

// ---------------------------------------------------------------------------
// Parameters: one FP32 vector, per layer W[t][co][ci] then b[co].  Adam with
// bias correction; c1 = lr / (1 - b1^t), c2 = 1 / (1 - b2^t).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CNT) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ vv, int n, float b1, float b2, float eps, float c1,
                                              float c2) {
  for (int e = blockIdx.x * CNT + threadIdx.x; e < n; e += gridDim.x * CNT) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * vv[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    vv[e] = vi;
    p[e] -= c1 * mi / (sqrtf(vi * c2) + eps);
  }
}

// Operand images of one layer from the parameter vector.
//   fwd: out channel co = 16 mb + l%16, k = t * cinp + ci            (MB = coutp/16 blocks, cinp in {8, 32})
//   bwd: out channel ci = 16 mb + l%16, k = t' * coutq + co, weight W[26 - t'][co][ci]
//        (the transposed, flipped kernel that maps output gradients to input gradients)
__global__ __launch_bounds__(CNT) void k_pack_image(const float* __restrict__ W, int cout, int cin, int mblocks,
                                                    int kin, int backward, uint16_t* __restrict__ img) {
  const int kc_n = (kTaps * kin + 31) / 32;
  const int n = mblocks * kc_n * 64 * 8;
  for (int e = blockIdx.x * CNT + threadIdx.x; e < n; e += gridDim.x * CNT) {
    const int j = e % 8, l = (e / 8) % 64, kc = (e / 512) % kc_n, mb = e / (512 * kc_n);
    const int row = mb * 16 + (l & 15);
    const int k = kc * 32 + 8 * (l >> 4) + j;
    const int t = k / kin, col = k % kin;
    float w = 0.f;
    if (t < kTaps) {
      if (!backward) {
        if (row < cout && col < cin) w = W[((long)t * cout + row) * cin + col];
      } else {
        if (row < cin && col < cout) w = W[((long)(kTaps - 1 - t) * cout + col) * cin + row];
      }
    }
    img[e] = f2bf(w);
  }
}
__global__ void k_pack_bias(const float* __restrict__ b, int cout, int coutp, float* __restrict__ out) {
  const int c = threadIdx.x;
  if (c < coutp) out[c] = c < cout ? b[c] : 0.f;
}

// ---------------------------------------------------------------------------
// Relative mean-square loss over samples of V voxels: L = (1/n) sum_s
// |p_s - q_s|^2 / |q_s|^2 (denominator 1 if q_s = 0); prediction and target
// hold 4 channels per voxel of which the first 3 count.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CNT) void k_loss_part(const float* __restrict__ p, const float* __restrict__ q, long V,
                                                   double* __restrict__ part) {
  __shared__ double red[CNT / 64];
  const int s = blockIdx.y;
  const long v0 = V * blockIdx.x / gridDim.x, v1 = V * (blockIdx.x + 1) / gridDim.x;
  double a = 0.0, b = 0.0;
  for (long v = v0 + threadIdx.x; v < v1; v += CNT) {
    const float4 pv = reinterpret_cast<const float4*>(p)[s * V + v];
    const float4 qv = reinterpret_cast<const float4*>(q)[s * V + v];
    const double d0 = (double)pv.x - qv.x, d1 = (double)pv.y - qv.y, d2 = (double)pv.z - qv.z;
    a += d0 * d0 + d1 * d1 + d2 * d2;
    b += (double)qv.x * qv.x + (double)qv.y * qv.y + (double)qv.z * qv.z;
  }
  a = pfk::block_sum(a, red);
  b = pfk::block_sum(b, red);
  if (threadIdx.x == 0) {
    part[((long)s * gridDim.x + blockIdx.x) * 2] = a;
    part[((long)s * gridDim.x + blockIdx.x) * 2 + 1] = b;
  }
}
// dL/dp as bf16 with 8 channels (3 used); sample losses to loss[s].
__global__ __launch_bounds__(CNT) void k_loss_grad(const float* __restrict__ p, const float* __restrict__ q, long V,
                                                   const double* __restrict__ part, int nblk, int nsamp,
                                                   uint16_t* __restrict__ g, double* __restrict__ loss) {
  __shared__ double red[CNT / 64];
  const int s = blockIdx.y;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += CNT) {
    a += part[((long)s * nblk + k) * 2];
    b += part[((long)s * nblk + k) * 2 + 1];
  }
  a = pfk::block_sum(a, red);
  b = pfk::block_sum(b, red);
  const double den = b > 0.0 ? b : 1.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) loss[s] = a / den;
  const float sc = (float)(2.0 / (den * nsamp));
  const long v0 = V * blockIdx.x / gridDim.x, v1 = V * (blockIdx.x + 1) / gridDim.x;
  for (long v = v0 + threadIdx.x; v < v1; v += CNT) {
    const float4 pv = reinterpret_cast<const float4*>(p)[s * V + v];
    const float4 qv = reinterpret_cast<const float4*>(q)[s * V + v];
    uint4 o;
    o.x = pack2(sc * (pv.x - qv.x), sc * (pv.y - qv.y));
    o.y = pack2(sc * (pv.z - qv.z), 0.f);
    o.z = 0u;
    o.w = 0u;
    reinterpret_cast<uint4*>(g)[s * V + v] = o;
  }
}

// ---------------------------------------------------------------------------
// Packing between the simulation state and the network (3D).
// A strided view of a cell or face array: element (i, j, k) at k*ps + j*rs + i.
// ---------------------------------------------------------------------------
template <typename T>
struct View {
  const T* p;
  long rs, ps;
  __device__ __forceinline__ double at(int i, int j, int k) const { return (double)p[(long)k * ps + (long)j * rs + i]; }
};

template <typename T>
struct PackArgs {
  View<T> phi_f, phi_w, phi_prev;
  const T* phi_f_lo;           // FP32 state: low parts of phi_f and of phi_prev (null: none)
  const T* phi_prev_lo;
  View<T> u1[3], u0[3];        // previous increment = u1 - u0 (u0 may be null: zero)
  View<T> u2[3];               // current state for targets (u2 - u1), null when no target is wanted
  int nx, ny, nz;              // full grid
  int x0, y0, z0;              // crop origin
  int cx, cy, cz;              // crop size
  double Omega, h;
  const double* s;             // device scalar: increment scale
  uint16_t* x;                 // out: [cz][cy][cx][8] bf16
  float* target;               // out (nullable): [cz][cy][cx][4] fp32
};

__device__ __forceinline__ double eigen_strain_d(double pf, double Omega) {
  const double hf = pf * pf * pf * (pf * (6.0 * pf - 15.0) + 10.0);
  return cbrt(1.0 - Omega * hf) - 1.0;
}

// FP32 difference of the small-strain eigenstrain of two ferrite phases,
// eps_T(x) - eps_T(y) with eps_T = cbrt(1 - Omega h) - 1, accurate to about
// 1e-6 relative everywhere (the difference of the two cube roots in FP64
// loses all digits near x = y = 1, where h' vanishes):
//   h(x) - h(y) = (x - y) * mean of h'(t) = 30 t^2 (1 - t)^2 over [y, x],
// the mean by 3-point Gauss-Legendre (exact for this quartic; a sum of
// non-negative terms, with 1 - t formed from 1 - x and 1 - y), and
//   cbrt(a) - cbrt(b) = (a - b) / (ca^2 + ca cb + cb^2).
// dxy is x - y, passed separately so that a state held as FP32 pairs can give
// it from both parts.
__device__ __forceinline__ float eigen_strain_diff_f(float x, float y, float dxy, float Omega) {
  const float m = 0.5f * (x + y), mc = 0.5f * ((1.f - x) + (1.f - y));
  const float r = 0.7745966692414834f * (0.5f * dxy);         // sqrt(3/5) times the half width
  const float u0 = m * mc, u1 = (m - r) * (mc + r), u2 = (m + r) * (mc - r);
  const float mean = (5.f * (u1 * u1 + u2 * u2) + 8.f * (u0 * u0)) * (1.f / 18.f);
  const float dh = dxy * 30.f * mean;
  const float hx = x * x * x * (x * (6.f * x - 15.f) + 10.f), hy = y * y * y * (y * (6.f * y - 15.f) + 10.f);
  const float ca = cbrtf(1.f - Omega * hx), cb = cbrtf(1.f - Omega * hy);
  return -Omega * dh / (ca * ca + ca * cb + cb * cb);
}

template <typename T>
__global__ __launch_bounds__(CNT) void k_pack_inputs(PackArgs<T> a) {
  const double s = *a.s;
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  if constexpr (sizeof(T) == 4) {
    // FP32 state: FP32 arithmetic (the inputs are rounded to bf16), 32-bit
    // indices (a crop of a grid with fewer than 2^31 cells)
    const float invf = (float)inv, es = (float)(32.0 * a.h * inv), Om = (float)a.Omega;
    const int nv = a.cx * a.cy * a.cz, cxy = a.cx * a.cy;
    for (int v = blockIdx.x * CNT + threadIdx.x; v < nv; v += gridDim.x * CNT) {
      const int lk = v / cxy, r = v - lk * cxy, lj = r / a.cx, li = r - lj * a.cx;
      const int i = a.x0 + li, j = a.y0 + lj, k = a.z0 + lk;
      float c[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float tg[4] = {0.f, 0.f, 0.f, 0.f};
      if (i < a.nx && j < a.ny && k < a.nz) {
        const int e = k * (int)a.phi_f.ps + j * (int)a.phi_f.rs + i;   // every view shares the cell layout
        const float pf = a.phi_f.p[e];
        c[0] = pf;
        c[1] = a.phi_w.p[e];
        const float pp = a.phi_prev.p[e];
        float dxy = pf - pp;
        if (a.phi_f_lo) dxy += a.phi_f_lo[e] - a.phi_prev_lo[e];
        c[2] = eigen_strain_diff_f(pf, pp, dxy, Om) * es;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float u1 = a.u1[d].p[e];
          const float u0 = a.u0[d].p ? a.u0[d].p[e] : 0.f;
          c[3 + d] = (u1 - u0) * invf;
          if (a.target) tg[d] = (a.u2[d].p[e] - u1) * invf;
        }
      }
      uint4 o;
      o.x = pack2(c[0], c[1]);
      o.y = pack2(c[2], c[3]);
      o.z = pack2(c[4], c[5]);
      o.w = pack2(c[6], c[7]);
      reinterpret_cast<uint4*>(a.x)[v] = o;
      if (a.target) reinterpret_cast<float4*>(a.target)[v] = make_float4(tg[0], tg[1], tg[2], 0.f);
    }
    return;
  }
  const long nv = (long)a.cx * a.cy * a.cz;
  for (long v = blockIdx.x * (long)CNT + threadIdx.x; v < nv; v += (long)gridDim.x * CNT) {
    const int li = (int)(v % a.cx), lj = (int)((v / a.cx) % a.cy), lk = (int)(v / ((long)a.cx * a.cy));
    const int i = a.x0 + li, j = a.y0 + lj, k = a.z0 + lk;
    float c[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float tg[4] = {0.f, 0.f, 0.f, 0.f};
    if (i < a.nx && j < a.ny && k < a.nz) {
      const double pf = a.phi_f.at(i, j, k);
      c[0] = (float)pf;
      c[1] = (float)a.phi_w.at(i, j, k);
      c[2] = (float)((eigen_strain_d(pf, a.Omega) - eigen_strain_d(a.phi_prev.at(i, j, k), a.Omega)) *
                     (32.0 * a.h * inv));
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double u1 = a.u1[d].at(i, j, k);
        const double u0 = a.u0[d].p ? a.u0[d].at(i, j, k) : 0.0;
        c[3 + d] = (float)((u1 - u0) * inv);
        if (a.target) tg[d] = (float)((a.u2[d].at(i, j, k) - u1) * inv);
      }
    }
    uint4 o;
    o.x = pack2(c[0], c[1]);
    o.y = pack2(c[2], c[3]);
    o.z = pack2(c[4], c[5]);
    o.w = pack2(c[6], c[7]);
    reinterpret_cast<uint4*>(a.x)[v] = o;
    if (a.target) reinterpret_cast<float4*>(a.target)[v] = make_float4(tg[0], tg[1], tg[2], 0.f);
  }
}

// Partials of sum over all stored faces of (u1 - u0)^2 (FP64) and the count.
template <typename T>
__global__ __launch_bounds__(CNT) void k_incr_sumsq(PackArgs<T> a, double* __restrict__ part) {
  __shared__ double red[CNT / 64];
  const long nv = (long)a.nx * a.ny * a.nz;
  double s = 0.0;
  for (long v = blockIdx.x * (long)CNT + threadIdx.x; v < nv; v += (long)gridDim.x * CNT) {
    const int i = (int)(v % a.nx), j = (int)((v / a.nx) % a.ny), k = (int)(v / ((long)a.nx * a.ny));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double du = a.u1[d].at(i, j, k) - (a.u0[d].p ? a.u0[d].at(i, j, k) : 0.0);
      s += du * du;
    }
  }
  s = pfk::block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
// s = sqrt(sum / count), count = 3 * cells (the low faces of every cell).
__global__ __launch_bounds__(CNT) void k_incr_scale(const double* __restrict__ part, int n, double count, double* __restrict__ s) {
  __shared__ double red[CNT / 64];
  double v = 0.0;
  for (int q = threadIdx.x; q < n; q += CNT) v += part[q];
  v = pfk::block_sum(v, red);
  if (threadIdx.x == 0) *s = sqrt(v / count);
}

}  // namespace pfn
