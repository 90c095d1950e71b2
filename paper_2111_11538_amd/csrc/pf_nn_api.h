// Host side of the learned warm start (pf_nn_* in include/pf.h) and its use
// inside a context's solve.  Included at the end of pf_api.hip.
#pragma once

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "pf_nn.h"

using pfn::Vol;

namespace {

// The network: 6 -> 32 -> 32 -> 32 -> 3 channels, 3x3x3 kernels.
struct LayerDef {
  int cin, cout;
  int cinp;     // input channels as stored (8 or 32)
  int mb;       // 16-row blocks of output channels in the forward image
  int kinb;     // input channels of the backward-data convolution (8 or 32; 0: not needed)
};
constexpr int kLayers = 4;
constexpr LayerDef kDef[kLayers] = {{6, 32, 8, 2, 0}, {32, 32, 32, 2, 32}, {32, 32, 32, 2, 32}, {32, 3, 32, 1, 8}};
constexpr int kWgradSplitMax = 96;
constexpr int kBgradBlocks = 256;

inline int kchunks(int cin) { return (pfn::kTaps * cin + 31) / 32; }

size_t nn_param_count() {
  size_t n = 0;
  for (int l = 0; l < kLayers; ++l) n += (size_t)pfn::kTaps * kDef[l].cout * kDef[l].cin + kDef[l].cout;
  return n;
}

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

}  // namespace

struct pf_nn {
  pf_nn_config cfg;
  hipStream_t stream;
  long long cap;                 // voxels
  size_t np;
  size_t off_w[kLayers], off_b[kLayers];
  float *P, *G, *M, *V;          // parameters, gradients, Adam moments (FP32)
  uint16_t* img_f[kLayers];
  uint16_t* img_b[kLayers];
  float* bias_p[kLayers];        // bias padded to 32
  uint16_t* x0;                  // packed input [cap][8]
  uint16_t* act[3];              // outputs of layers 0..2 [cap][32]
  float* out;                    // network output [cap][4]
  float* target;                 // packed targets [cap][4]
  uint16_t* dpred;               // loss gradient [cap][8]
  uint16_t* g[2];                // backward ping-pong [cap][32]
  float* wpart;                  // weight-gradient partials
  double* dpart;                 // FP64 partials (bias gradient, loss, scale)
  double* dscal;                 // [0] increment scale, [1..] sample losses
  int adam_t;
  // last forward, for backward and loss
  Vol last_v;
  const uint16_t* last_x;
  float* last_y;
  bool have_fwd;
  char err[512];
};

static char g_nn_err[512] = "";

static pf_status nn_fail(pf_nn* n, pf_status s, const char* fmt, ...) {
  char* dst = n ? n->err : g_nn_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return s;
}

#define NNCHK(nn, call)                                                                           \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return nn_fail((nn), PF_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define NNLAUNCH(nn)                                                                                      \
  do {                                                                                                    \
    hipError_t e_ = hipGetLastError();                                                                    \
    if (e_ != hipSuccess) return nn_fail((nn), PF_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_));   \
  } while (0)

static long long vol_voxels(const Vol& v) { return (long long)v.n * v.D * v.H * v.W; }

static pf_status nn_check_vol(pf_nn* nn, const Vol& v) {
  if (v.n < 1 || v.D < 1 || v.H < 1 || v.W < 1) return nn_fail(nn, PF_ERR_INVALID_ARG, "volume sizes must be >= 1");
  // the convolutions address a 32-channel bf16 tensor with 32-bit byte offsets
  if (vol_voxels(v) * 64 >= (1LL << 31)) return nn_fail(nn, PF_ERR_INVALID_ARG, "at most 2^25 voxels per call");
  if (vol_voxels(v) > nn->cap)
    return nn_fail(nn, PF_ERR_INVALID_ARG, "%lld voxels exceed the capacity %lld", vol_voxels(v), nn->cap);
  return PF_OK;
}

static int conv32_grid(const Vol& v, int cap) {
  long long nt = (long long)((v.W + pfn::SEG - 1) / pfn::SEG) * ((v.H + pfn::CONV_WAVES - 1) / pfn::CONV_WAVES) * v.D * v.n;
  return (int)std::max(1LL, std::min(nt, (long long)cap));
}

// the output layer's z march: one block per (volume, row tile, x segment, z run)
static int conv_out_grid(const Vol& v, int cap) {
  long long nt = (long long)((v.W + pfn::SEG - 1) / pfn::SEG) * ((v.H + pfn::CONV_WAVES - 1) / pfn::CONV_WAVES) *
                 ((v.D + pfn::kOutZ - 1) / pfn::kOutZ) * v.n;
  return (int)std::max(1LL, std::min(nt, (long long)cap));
}

static int conv_grid(const Vol& v, int cap) {
  long long nt = (long long)((v.W + pfn::SEG - 1) / pfn::SEG) * ((v.H + pfn::CONV_WAVES - 1) / pfn::CONV_WAVES) * v.D * v.n;
  return (int)std::max(1LL, std::min(nt, (long long)cap));
}

// Forward convolution of layer l: x (cinp channels) -> y.
static pf_status nn_conv_fwd(pf_nn* nn, int l, const uint16_t* x, void* y, const Vol& v, hipStream_t st) {
  const LayerDef& d = kDef[l];
  const size_t smem = (size_t)d.mb * kchunks(d.cinp) * 64 * 16;
  const uint4* w = reinterpret_cast<const uint4*>(nn->img_f[l]);
  if (l == 0)
    hipLaunchKernelGGL((pfn::k_conv<8, 2, pfn::EPI_RELU>), dim3(conv_grid(v, 4096)), dim3(pfn::CONV_NT), smem, st, w,
                       (const float*)nn->bias_p[l], x, y, (const uint16_t*)nullptr, v);
  else if (l < 3)
    hipLaunchKernelGGL((pfn::k_conv32<2, pfn::EPI_RELU>), dim3(conv32_grid(v, 512)), dim3(pfn::CONV_NT), smem, st, w,
                       (const float*)nn->bias_p[l], x, y, (const uint16_t*)nullptr, v);
  else
    hipLaunchKernelGGL((pfn::k_conv32_out<pfn::EPI_LINEAR>), dim3(conv_out_grid(v, 2048)), dim3(pfn::CONV_NT), smem, st,
                       w, (const float*)nn->bias_p[l], x, (float*)y, v);
  NNLAUNCH(nn);
  return PF_OK;
}

// Backward-data convolution of layer l (1..3): dy -> dx masked by (mask > 0).
static pf_status nn_conv_bwd(pf_nn* nn, int l, const uint16_t* dy, const uint16_t* mask, uint16_t* dx, const Vol& v,
                             hipStream_t st) {
  const LayerDef& d = kDef[l];
  const size_t smem = (size_t)2 * kchunks(d.kinb) * 64 * 16;
  const uint4* w = reinterpret_cast<const uint4*>(nn->img_b[l]);
  if (d.kinb == 8)
    hipLaunchKernelGGL((pfn::k_conv<8, 2, pfn::EPI_MASK>), dim3(conv_grid(v, 4096)), dim3(pfn::CONV_NT), smem, st, w,
                       (const float*)nullptr, dy, (void*)dx, mask, v);
  else
    hipLaunchKernelGGL((pfn::k_conv32<2, pfn::EPI_MASK>), dim3(conv32_grid(v, 512)), dim3(pfn::CONV_NT), smem, st, w,
                       (const float*)nullptr, dy, (void*)dx, mask, v);
  NNLAUNCH(nn);
  return PF_OK;
}

// Weight and bias gradients of layer l from its input x and output gradient dy,
// written to gw (27 * cout * cin) and gb (cout) in FP32.
static pf_status nn_conv_wgrad(pf_nn* nn, int l, const uint16_t* x, const uint16_t* dy, float* gw, float* gb, const Vol& v,
                               hipStream_t st) {
  const LayerDef& d = kDef[l];
  const long long rows = (long long)v.n * v.D * v.H;
  const int nsplit = (int)std::max(1LL, std::min(rows, (long long)kWgradSplitMax));
  const dim3 grid(nsplit, pfn::kTaps);
  const int cg = l == 3 ? 8 : 32;
  const int coutp = l == 3 ? 16 : 32;
  if (l == 0)
    hipLaunchKernelGGL((pfn::k_conv_wgrad<8, 32, 2>), grid, dim3(pfn::CNT), 0, st, x, dy, nn->wpart, v);
  else if (l < 3)
    hipLaunchKernelGGL((pfn::k_conv_wgrad<32, 32, 2>), grid, dim3(pfn::CNT), 0, st, x, dy, nn->wpart, v);
  else
    hipLaunchKernelGGL((pfn::k_conv_wgrad<32, 8, 1>), grid, dim3(pfn::CNT), 0, st, x, dy, nn->wpart, v);
  NNLAUNCH(nn);
  const int cinp = d.cinp == 8 ? 16 : 32;
  const int nw = pfn::kTaps * d.cout * d.cin;
  hipLaunchKernelGGL(pfn::k_wgrad_reduce, dim3((nw + pfn::CNT - 1) / pfn::CNT), dim3(pfn::CNT), 0, st,
                     (const float*)nn->wpart, nsplit, coutp, cinp, d.cout, d.cin, gw);
  const long long nvox = vol_voxels(v);
  hipLaunchKernelGGL(pfn::k_bgrad_part, dim3(kBgradBlocks), dim3(pfn::CNT), 0, st, dy, cg, (long)nvox, nn->dpart);
  hipLaunchKernelGGL(pfn::k_bgrad_reduce, dim3(1), dim3(pfn::CNT), 0, st, (const double*)nn->dpart, kBgradBlocks, cg, d.cout, gb);
  NNLAUNCH(nn);
  return PF_OK;
}

static pf_status nn_repack(pf_nn* nn, hipStream_t st) {
  for (int l = 0; l < kLayers; ++l) {
    const LayerDef& d = kDef[l];
    const float* W = nn->P + nn->off_w[l];
    int n = d.mb * kchunks(d.cinp) * 512;
    hipLaunchKernelGGL(pfn::k_pack_image, dim3((n + pfn::CNT - 1) / pfn::CNT), dim3(pfn::CNT), 0, st, W, d.cout, d.cin,
                       d.mb, d.cinp, 0, nn->img_f[l]);
    if (d.kinb) {
      n = 2 * kchunks(d.kinb) * 512;
      hipLaunchKernelGGL(pfn::k_pack_image, dim3((n + pfn::CNT - 1) / pfn::CNT), dim3(pfn::CNT), 0, st, W, d.cout,
                         d.cin, 2, d.kinb, 1, nn->img_b[l]);
    }
    hipLaunchKernelGGL(pfn::k_pack_bias, dim3(1), dim3(32), 0, st, (const float*)(nn->P + nn->off_b[l]), d.cout, 32,
                       nn->bias_p[l]);
  }
  NNLAUNCH(nn);
  return PF_OK;
}

static pf_status nn_forward(pf_nn* nn, const uint16_t* x, float* y, const Vol& v, hipStream_t st) {
  pf_status s;
  if ((s = nn_check_vol(nn, v)) != PF_OK) return s;
  if ((s = nn_conv_fwd(nn, 0, x, nn->act[0], v, st)) != PF_OK) return s;
  if ((s = nn_conv_fwd(nn, 1, nn->act[0], nn->act[1], v, st)) != PF_OK) return s;
  if ((s = nn_conv_fwd(nn, 2, nn->act[1], nn->act[2], v, st)) != PF_OK) return s;
  if ((s = nn_conv_fwd(nn, 3, nn->act[2], y, v, st)) != PF_OK) return s;
  nn->last_v = v;
  nn->last_x = x;
  nn->last_y = y;
  nn->have_fwd = true;
  return PF_OK;
}

// Views of the exchange-format arrays (compact FP64, x fastest): cells
// [nz][ny][nx], faces u_x [nz][ny][nx+1], u_y [nz][ny+1][nx], u_z [nz+1][ny][nx].
static pfn::View<double> xview_cell(const double* p, int nx, int ny) { return {p, nx, (long)nx * ny}; }
static pfn::View<double> xview_face(const double* p, int c, int nx, int ny) {
  if (c == 0) return {p, nx + 1, (long)(nx + 1) * ny};
  if (c == 1) return {p, nx, (long)nx * (ny + 1)};
  return {p, nx, (long)nx * ny};
}

// ---------------------------------------------------------------------------
// Learned start inside a context's solve (3D).  The context holds, when its
// warm start is PF_WARM_LEARNED, the displacement before the solve (uo), the
// increment of the previous solve (du) and the ferrite phase of the previous
// solve (phi_prev).
// ---------------------------------------------------------------------------
// Learned increment on the low faces of every cell: d = s * y, zero on the
// low boundary faces (fixed by the rollers) and in the padding.
template <typename T>
__global__ __launch_bounds__(pfn::CNT) void k_learned_delta(T* __restrict__ d0, T* __restrict__ d1, T* __restrict__ d2,
                                                           const float* __restrict__ y, const double* __restrict__ s,
                                                           Grid g) {
  const double sc = *s;
  for (int e = blockIdx.x * pfn::CNT + threadIdx.x; e < g.n; e += gridDim.x * pfn::CNT) {
    const int row = e / g.px, i = e - row * g.px, k = row / g.ny, j = row - k * g.ny;
    T a = T(0), b = T(0), c = T(0);
    if (i < g.nx) {
      const float4 o = reinterpret_cast<const float4*>(y)[row * g.nx + i];
      if (i > 0) a = (T)(sc * o.x);
      if (j > 0) b = (T)(sc * o.y);
      if (k > 0) c = (T)(sc * o.z);
    }
    d0[e] = a;
    d1[e] = b;
    d2[e] = c;
  }
}

// Judge (one block): compare the residual norm of the learned start, whose
// partials the apply kernel computed with q = A d (||r - q||^2, r = b - A u_prev
// from the residual pass), with that of the previous displacement; the
// decision and both norms go to the device scalars.  Nothing is decided when
// the solve has already converged (b = 0).
__global__ __launch_bounds__(NT) void k_judge_decide(const double* __restrict__ part_l, int nl,
                                                    const double* __restrict__ part_p, int np, double* __restrict__ scal) {
  __shared__ double red[NT / 64];
  const double rl = sum_partials(part_l, nl, red);
  const double rp = sum_partials(part_p, np, red);
  if (threadIdx.x == 0) {
    scal[S_JL] = rl;
    scal[S_JP] = rp;
    scal[S_JB] = (scal[S_CONV] == 0.0 && rl < rp) ? 1.0 : 0.0;
  }
}

// Judge, second step: if the learned start won, move to it: u += d, r -= q,
// z = D^-1 r, and replace the partials of r.z and r.r that CG starts from.
template <typename T>
__global__ __launch_bounds__(NT) void k_judge_apply(T* __restrict__ u0, T* __restrict__ u1, T* __restrict__ u2,
                                                   const T* __restrict__ d0, const T* __restrict__ d1,
                                                   const T* __restrict__ d2, T* __restrict__ r0, T* __restrict__ r1,
                                                   T* __restrict__ r2, const T* __restrict__ q0, const T* __restrict__ q1,
                                                   const T* __restrict__ q2, const T* __restrict__ di0,
                                                   const T* __restrict__ di1, const T* __restrict__ di2,
                                                   T* __restrict__ z0, T* __restrict__ z1, T* __restrict__ z2, long n,
                                                   const double* __restrict__ scal, double* __restrict__ part) {
  __shared__ double red[2 * (NT / 64)];
  if (scal[S_JB] == 0.0) return;
  double rz = 0.0, rr = 0.0;
  for (long e = blockIdx.x * (long)NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) {
    u0[e] += d0[e];
    u1[e] += d1[e];
    u2[e] += d2[e];
    const T a = r0[e] - q0[e], b = r1[e] - q1[e], c = r2[e] - q2[e];
    const T za = di0[e] * a, zb = di1[e] * b, zc = di2[e] * c;
    r0[e] = a; r1[e] = b; r2[e] = c;
    z0[e] = za; z1[e] = zb; z2[e] = zc;
    rz += (double)a * (double)za + (double)b * (double)zb + (double)c * (double)zc;
    rr += (double)a * (double)a + (double)b * (double)b + (double)c * (double)c;
  }
  block_sum2(rz, rr, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[gridDim.x + blockIdx.x] = rr;
  }
}

// After a solve: the increment d = u - u_o of this step (the network's input
// at the next), u_o = u (the next solve's previous displacement), the phase
// field it was taken at, and partials of sum d^2 (the increment's scale; the
// padding holds zeros in u and u_o).
template <typename T>
__global__ __launch_bounds__(pfn::CNT) void k_after_solve(const T* __restrict__ u0, const T* __restrict__ u1,
                                                         const T* __restrict__ u2, T* __restrict__ o0,
                                                         T* __restrict__ o1, T* __restrict__ o2,
                                                         T* __restrict__ d0, T* __restrict__ d1, T* __restrict__ d2,
                                                         const T* __restrict__ phi, T* __restrict__ phi_prev,
                                                         const T* __restrict__ phi_lo, T* __restrict__ phi_prev_lo,
                                                         long n, double* __restrict__ part) {
  __shared__ double red[pfn::CNT / 64];
  double s = 0.0;
  for (long e = blockIdx.x * (long)pfn::CNT + threadIdx.x; e < n; e += (long)gridDim.x * pfn::CNT) {
    const T a = u0[e], b = u1[e], c = u2[e];
    const T da = a - o0[e], db = b - o1[e], dc = c - o2[e];
    d0[e] = da;
    d1[e] = db;
    d2[e] = dc;
    o0[e] = a;
    o1[e] = b;
    o2[e] = c;
    phi_prev[e] = phi[e];
    if (phi_lo) phi_prev_lo[e] = phi_lo[e];
    s += (double)da * (double)da + (double)db * (double)db + (double)dc * (double)dc;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
static pfn::PackArgs<T> ctx_pack_args(pf_ctx* c) {
  const Layout& L = c->L;
  const Grid& g = L.g;
  pfn::PackArgs<T> a{};
  const long rs = g.px, ps = (long)g.px * g.ny;
  a.phi_f = {c->arr<T>(L.o_fld[c->cur][0]), rs, ps};
  a.phi_w = {c->arr<T>(L.o_fld[c->cur][1]), rs, ps};
  a.phi_prev = {c->arr<T>(L.o_phiprev), rs, ps};
  if (L.es == 4) {
    a.phi_f_lo = c->arr<T>(L.o_lo[c->cur][0]);
    a.phi_prev_lo = c->arr<T>(L.o_phiprev_lo);
  }
  for (int d = 0; d < 3; ++d) {
    a.u1[d] = {c->arr<T>(L.o_du[d]), rs, ps};
    a.u0[d] = {nullptr, rs, ps};
    a.u2[d] = {nullptr, rs, ps};
  }
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz;
  a.cx = g.nx; a.cy = g.ny; a.cz = g.nz;
  a.Omega = c->prm.Omega_f;
  a.h = c->cfg.h;
  return a;
}

// Offer the learned start after the residual pass of the previous
// displacement: d = s * NN(state), q = A d on the apply kernel, and the
// residual of u_prev + d is r - q.  The comparison and the switch happen on
// the device (no host synchronisation); the solve reports the choice.
// `part` holds 2 * nb_el doubles of scratch; r, z, D^-1 and their partials
// come from the residual pass.
template <typename T, int DIM>
static pf_status learned_start(pf_ctx* c, ElastArgs<T> e, double* part) {
  const Layout& L = c->L;
  hipStream_t st = c->stream;
  c->judged = false;
  // u_o (the displacement this solve starts from) was left equal to u by the
  // previous solve's after-solve pass, unless there was none since the state
  // was set
  if (!c->have_prev_incr)
    for (int d = 0; d < DIM; ++d)
      HIPCHK(c, hipMemcpyAsync(c->ws + L.o_uo[d], c->ws + L.o_u[d], (size_t)L.g.n * sizeof(T), hipMemcpyDeviceToDevice, st));
  if constexpr (DIM == 3) {
    pf_nn* nn = c->net;
    if (!nn || !c->have_prev_incr) return PF_OK;
    const Vol v{1, L.g.nz, L.g.ny, L.g.nx};
    if (vol_voxels(v) > nn->cap) return fail(c, PF_ERR_INVALID_ARG, "the grid exceeds the network's capacity");
    pfn::PackArgs<T> a = ctx_pack_args<T>(c);
    a.s = nn->dscal;
    a.x = nn->x0;
    a.target = nullptr;
    // the increment's scale from the partials the previous after-solve pass left
    hipLaunchKernelGGL(pfn::k_incr_scale, dim3(1), dim3(pfn::CNT), 0, st, (const double*)c->arr<double>(L.o_dsq),
                       kAfterBlocks, 3.0 * (double)vol_voxels(v), nn->dscal);
    hipLaunchKernelGGL((pfn::k_pack_inputs<T>), dim3(2048), dim3(pfn::CNT), 0, st, a);
    LAUNCHCHK(c);
    pf_status fs = PF_OK;
    timed(c, PF_K_NN, [&] { fs = nn_forward(nn, nn->x0, nn->out, v, st); });
    if (fs != PF_OK) return fail(c, PF_ERR_HIP, "network: %s", nn->err);
    nn->have_fwd = false;    // the activations now belong to this inference, not to a training step
    // d into the second direction buffer, q = A d into q (both free before CG starts)
    T* dl[3] = {c->arr<T>(L.o_pb[0]), c->arr<T>(L.o_pb[1]), c->arr<T>(L.o_pb[2])};
    T* q[3] = {c->arr<T>(L.o_q[0]), c->arr<T>(L.o_q[1]), c->arr<T>(L.o_q[2])};
    T* r[3] = {c->arr<T>(L.o_r[0]), c->arr<T>(L.o_r[1]), c->arr<T>(L.o_r[2])};
    T* z[3] = {c->arr<T>(L.o_z[0]), c->arr<T>(L.o_z[1]), c->arr<T>(L.o_z[2])};
    T* di[3] = {c->arr<T>(L.o_di[0]), c->arr<T>(L.o_di[1]), c->arr<T>(L.o_di[2])};
    T* u[3] = {c->arr<T>(L.o_u[0]), c->arr<T>(L.o_u[1]), c->arr<T>(L.o_u[2])};
    hipLaunchKernelGGL((k_learned_delta<T>), dim3(2048), dim3(pfn::CNT), 0, st, dl[0], dl[1], dl[2],
                       (const float*)nn->out, (const double*)nn->dscal, L.g);
    ElastArgs<T> ap = e;
    ap.kz = L.kz_ap;
    ap.part = part;
    // q = A d, with the partials of ||r - q||^2 (the learned start's residual)
    for (int d = 0; d < 3; ++d) {
      ap.z[d] = dl[d];
      ap.u[d] = c->arr<T>(L.o_pa[d]);      // not read (plain)
      ap.o1[d] = c->arr<T>(L.o_pa[d]);     // not written (plain)
      ap.o2[d] = q[d];
      ap.jr[d] = r[d];
    }
    timed_launch(c, PF_K_OTHER, -1, k_apply3<T, kApplyBY, APPLY_PLAIN>, L.gap, dim3(ApplyTile<kApplyBY>::NTB), 0, st, ap);
    const long n = L.g.n;
    double* part_u = c->arr<double>(L.o_part_u);
    hipLaunchKernelGGL(k_judge_decide, dim3(1), dim3(NT), 0, st, (const double*)part, (int)(L.gap.x * L.gap.y * L.gap.z),
                       (const double*)(part_u + L.nb_res), L.nb_res, c->scal());
    // (its grid is the residual pass's, so CG reads the same number of partials either way)
    hipLaunchKernelGGL((k_judge_apply<T>), dim3(L.nb_res), dim3(NT), 0, st, u[0], u[1], u[2], (const T*)dl[0],
                       (const T*)dl[1], (const T*)dl[2], r[0], r[1], r[2], (const T*)q[0], (const T*)q[1],
                       (const T*)q[2], (const T*)di[0], (const T*)di[1], (const T*)di[2], z[0], z[1], z[2], n,
                       (const double*)c->scal(), part_u);
    LAUNCHCHK(c);
    c->judged = true;
  }
  return PF_OK;
}

template <typename T, int DIM>
static pf_status learned_after_solve(pf_ctx* c) {
  const Layout& L = c->L;
  if constexpr (DIM == 3) {
    hipLaunchKernelGGL((k_after_solve<T>), dim3(kAfterBlocks), dim3(pfn::CNT), 0, c->stream,
                       (const T*)c->arr<T>(L.o_u[0]), (const T*)c->arr<T>(L.o_u[1]), (const T*)c->arr<T>(L.o_u[2]),
                       c->arr<T>(L.o_uo[0]), c->arr<T>(L.o_uo[1]), c->arr<T>(L.o_uo[2]), c->arr<T>(L.o_du[0]),
                       c->arr<T>(L.o_du[1]), c->arr<T>(L.o_du[2]), (const T*)c->arr<T>(L.o_fld[c->cur][0]),
                       c->arr<T>(L.o_phiprev), L.es == 4 ? (const T*)c->arr<T>(L.o_lo[c->cur][0]) : nullptr,
                       L.es == 4 ? c->arr<T>(L.o_phiprev_lo) : nullptr, (long)L.g.n, c->arr<double>(L.o_dsq));
    LAUNCHCHK(c);
    c->have_prev_incr = true;
  }
  return PF_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t pf_nn_param_count(void) { return nn_param_count(); }

// Carve every device buffer of a network out of one caller-owned workspace
// (256-byte aligned pieces).  With base == nullptr only the size is computed.
static size_t nn_layout(pf_nn* nn, const pf_nn_config* cfg, char* base) {
  const size_t cap = (size_t)cfg->max_voxels;
  size_t off = 0;
  auto take = [&](auto*& p, size_t bytes) {
    using P = std::remove_reference_t<decltype(p)>;
    if (base) p = reinterpret_cast<P>(base + off);
    off += (std::max<size_t>(bytes, 256) + 255) / 256 * 256;
  };
  const size_t np = nn_param_count();
  pf_nn tmp{};
  pf_nn* t = nn ? nn : &tmp;
  take(t->P, np * 4);
  take(t->G, np * 4);
  take(t->M, np * 4);
  take(t->V, np * 4);
  for (int l = 0; l < kLayers; ++l) {
    take(t->img_f[l], (size_t)kDef[l].mb * kchunks(kDef[l].cinp) * 1024);
    if (kDef[l].kinb) take(t->img_b[l], (size_t)2 * kchunks(kDef[l].kinb) * 1024);
    take(t->bias_p[l], 32 * 4);
  }
  take(t->x0, cap * 8 * 2);
  for (int q = 0; q < 3; ++q) take(t->act[q], cap * 32 * 2);
  take(t->out, cap * 4 * 4);
  take(t->dscal, 1024 * 8);
  take(t->dpart, (size_t)std::max(kBgradBlocks * 32, 4096) * 8 * 2);
  if (cfg->training) {
    take(t->target, cap * 4 * 4);
    take(t->dpred, cap * 8 * 2);
    take(t->g[0], cap * 32 * 2);
    take(t->g[1], cap * 32 * 2);
    take(t->wpart, (size_t)kWgradSplitMax * pfn::kTaps * 32 * 32 * 4);
  }
  return off;
}

static bool nn_carve(pf_nn* nn, const pf_nn_config* cfg, char* base, size_t bytes) {
  if (!base || nn_layout(nullptr, cfg, nullptr) > bytes) return false;
  nn_layout(nn, cfg, base);
  return true;
}

size_t pf_nn_workspace_bytes(const pf_nn_config* cfg) {
  if (!cfg || cfg->max_voxels < 1) return 0;
  return nn_layout(nullptr, cfg, nullptr);
}

pf_status pf_nn_init(const pf_nn_config* cfg, void* workspace, size_t workspace_bytes, void* hip_stream, pf_nn** out) {
  if (!out) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "config is NULL");
  if (cfg->max_voxels < 1) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "max_voxels must be >= 1");
  if (!workspace) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  pf_nn* nn = new (std::nothrow) pf_nn();
  if (!nn) return nn_fail(nullptr, PF_ERR_OOM, "host allocation failed");
  nn->cfg = *cfg;
  nn->stream = reinterpret_cast<hipStream_t>(hip_stream);
  nn->cap = cfg->max_voxels;
  nn->np = nn_param_count();
  size_t off = 0;
  for (int l = 0; l < kLayers; ++l) {
    nn->off_w[l] = off;
    off += (size_t)pfn::kTaps * kDef[l].cout * kDef[l].cin;
    nn->off_b[l] = off;
    off += kDef[l].cout;
  }
  if (!nn_carve(nn, cfg, reinterpret_cast<char*>(workspace), workspace_bytes)) {
    const size_t need = pf_nn_workspace_bytes(cfg);
    delete nn;
    return nn_fail(nullptr, PF_ERR_OOM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
  }

  // He-uniform initialisation from SplitMix64; the output layer is scaled by 0.1
  std::vector<float> P(nn->np, 0.f);
  uint64_t s = cfg->seed;
  for (int l = 0; l < kLayers; ++l) {
    const double bound = std::sqrt(6.0 / (pfn::kTaps * kDef[l].cin)) * (l == kLayers - 1 ? 0.1 : 1.0);
    const size_t nw = (size_t)pfn::kTaps * kDef[l].cout * kDef[l].cin;
    for (size_t q = 0; q < nw; ++q) {
      const double u = (double)(splitmix64(s) >> 11) * 0x1.0p-53;
      P[nn->off_w[l] + q] = (float)((2.0 * u - 1.0) * bound);
    }
  }
  hipError_t e = hipMemcpyAsync(nn->P, P.data(), nn->np * 4, hipMemcpyHostToDevice, nn->stream);
  if (e == hipSuccess) e = hipMemsetAsync(nn->M, 0, nn->np * 4, nn->stream);
  if (e == hipSuccess) e = hipMemsetAsync(nn->V, 0, nn->np * 4, nn->stream);
  if (e == hipSuccess) e = hipMemsetAsync(nn->G, 0, nn->np * 4, nn->stream);
  if (e == hipSuccess && nn_repack(nn, nn->stream) != PF_OK) e = hipErrorUnknown;
  if (e == hipSuccess) e = hipStreamSynchronize(nn->stream);
  if (e != hipSuccess) {
    pf_nn_destroy(nn);
    return nn_fail(nullptr, PF_ERR_HIP, "initialisation failed: %s", hipGetErrorString(e));
  }
  nn->adam_t = 0;
  nn->have_fwd = false;
  nn->err[0] = 0;
  *out = nn;
  return PF_OK;
}

void pf_nn_destroy(pf_nn* nn) {
  if (!nn) return;
  (void)hipStreamSynchronize(nn->stream);
  delete nn;                       // the device workspace belongs to the caller
}

const char* pf_nn_last_error(const pf_nn* nn) { return nn ? nn->err : g_nn_err; }

pf_status pf_nn_weights(pf_nn* nn, int dir, float* host, size_t count) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (!host) return nn_fail(nn, PF_ERR_INVALID_ARG, "host is NULL");
  if (count != nn->np) return nn_fail(nn, PF_ERR_INVALID_ARG, "%zu parameters expected, got %zu", nn->np, count);
  if (dir == 1) {
    NNCHK(nn, hipMemcpyAsync(nn->P, host, nn->np * 4, hipMemcpyHostToDevice, nn->stream));
    pf_status s = nn_repack(nn, nn->stream);
    if (s != PF_OK) return s;
  } else if (dir == 0) {
    NNCHK(nn, hipMemcpyAsync(host, nn->P, nn->np * 4, hipMemcpyDeviceToHost, nn->stream));
  } else if (dir == 2) {
    NNCHK(nn, hipMemcpyAsync(host, nn->G, nn->np * 4, hipMemcpyDeviceToHost, nn->stream));
  } else {
    return nn_fail(nn, PF_ERR_INVALID_ARG, "dir must be 0 (get), 1 (set) or 2 (get gradients)");
  }
  NNCHK(nn, hipStreamSynchronize(nn->stream));
  return PF_OK;
}

pf_status pf_nn_copy(pf_nn* nn, int which, int dir, void* dev, size_t bytes) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (!dev) return nn_fail(nn, PF_ERR_INVALID_ARG, "dev is NULL");
  if (dir != 0 && dir != 1) return nn_fail(nn, PF_ERR_INVALID_ARG, "dir must be 0 or 1");
  const size_t cap = (size_t)nn->cap;
  void* buf = nullptr;
  size_t size = cap * 16;
  switch (which) {
    case PF_NN_BUF_INPUT: buf = nn->x0; break;
    case PF_NN_BUF_OUTPUT: buf = nn->out; break;
    case PF_NN_BUF_TARGET: buf = nn->target; break;
    case PF_NN_BUF_LOSS_GRAD: buf = nn->dpred; break;
    default: return nn_fail(nn, PF_ERR_INVALID_ARG, "unknown buffer %d", which);
  }
  if (!buf) return nn_fail(nn, PF_ERR_INVALID_ARG, "buffer %d needs a network created for training", which);
  if (bytes > size) return nn_fail(nn, PF_ERR_INVALID_ARG, "%zu bytes exceed the buffer's %zu", bytes, size);
  NNCHK(nn, hipMemcpyAsync(dir == 0 ? dev : buf, dir == 0 ? buf : dev, bytes, hipMemcpyDeviceToDevice, nn->stream));
  return PF_OK;
}

pf_status pf_nn_forward(pf_nn* nn, const void* x, float* y, int n, int D, int H, int W) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  const Vol v{n, D, H, W};
  return nn_forward(nn, x ? reinterpret_cast<const uint16_t*>(x) : nn->x0, y ? y : nn->out, v, nn->stream);
}

pf_status pf_nn_loss(pf_nn* nn, const float* target, double* mean_loss) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (!nn->cfg.training) return nn_fail(nn, PF_ERR_INVALID_ARG, "created without training buffers");
  if (!nn->have_fwd) return nn_fail(nn, PF_ERR_INVALID_ARG, "no forward pass to take the loss of");
  const Vol& v = nn->last_v;
  const long V = (long)v.D * v.H * v.W;
  if (v.n > 1000) return nn_fail(nn, PF_ERR_INVALID_ARG, "at most 1000 samples per loss");
  const int nblk = (int)std::max(1L, std::min(64L, (V + pfn::CNT - 1) / pfn::CNT));
  const float* q = target ? target : nn->target;
  hipLaunchKernelGGL(pfn::k_loss_part, dim3(nblk, v.n), dim3(pfn::CNT), 0, nn->stream, (const float*)nn->last_y, q, V,
                     nn->dpart);
  hipLaunchKernelGGL(pfn::k_loss_grad, dim3(nblk, v.n), dim3(pfn::CNT), 0, nn->stream, (const float*)nn->last_y, q, V,
                     (const double*)nn->dpart, nblk, v.n, nn->dpred, nn->dscal + 1);
  NNLAUNCH(nn);
  if (mean_loss) {
    std::vector<double> ls(v.n);
    NNCHK(nn, hipMemcpyAsync(ls.data(), nn->dscal + 1, v.n * sizeof(double), hipMemcpyDeviceToHost, nn->stream));
    NNCHK(nn, hipStreamSynchronize(nn->stream));
    double s = 0.0;
    for (double q2 : ls) s += q2;
    *mean_loss = s / v.n;
  }
  return PF_OK;
}

pf_status pf_nn_backward(pf_nn* nn, const void* dy) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (!nn->cfg.training) return nn_fail(nn, PF_ERR_INVALID_ARG, "created without training buffers");
  if (!nn->have_fwd) return nn_fail(nn, PF_ERR_INVALID_ARG, "backward needs the activations of a forward pass");
  const Vol& v = nn->last_v;
  hipStream_t st = nn->stream;
  const uint16_t* gout = dy ? reinterpret_cast<const uint16_t*>(dy) : nn->dpred;
  pf_status s;
  if ((s = nn_conv_wgrad(nn, 3, nn->act[2], gout, nn->G + nn->off_w[3], nn->G + nn->off_b[3], v, st)) != PF_OK) return s;
  if ((s = nn_conv_bwd(nn, 3, gout, nn->act[2], nn->g[0], v, st)) != PF_OK) return s;
  if ((s = nn_conv_wgrad(nn, 2, nn->act[1], nn->g[0], nn->G + nn->off_w[2], nn->G + nn->off_b[2], v, st)) != PF_OK) return s;
  if ((s = nn_conv_bwd(nn, 2, nn->g[0], nn->act[1], nn->g[1], v, st)) != PF_OK) return s;
  if ((s = nn_conv_wgrad(nn, 1, nn->act[0], nn->g[1], nn->G + nn->off_w[1], nn->G + nn->off_b[1], v, st)) != PF_OK) return s;
  if ((s = nn_conv_bwd(nn, 1, nn->g[1], nn->act[0], nn->g[0], v, st)) != PF_OK) return s;
  if ((s = nn_conv_wgrad(nn, 0, nn->last_x, nn->g[0], nn->G + nn->off_w[0], nn->G + nn->off_b[0], v, st)) != PF_OK) return s;
  return PF_OK;
}

pf_status pf_nn_adam(pf_nn* nn, double lr, double b1, double b2, double eps) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (!(lr > 0.0) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) || !(eps >= 0.0))
    return nn_fail(nn, PF_ERR_INVALID_ARG, "need lr > 0, 0 <= b1, b2 < 1 and eps >= 0");
  nn->adam_t += 1;
  const double c1 = lr / (1.0 - std::pow(b1, nn->adam_t));
  const double c2 = 1.0 / (1.0 - std::pow(b2, nn->adam_t));
  const int n = (int)nn->np;
  hipLaunchKernelGGL(pfn::k_adam, dim3((n + pfn::CNT - 1) / pfn::CNT), dim3(pfn::CNT), 0, nn->stream, nn->P,
                     (const float*)nn->G, nn->M, nn->V, n, (float)b1, (float)b2, (float)eps, (float)c1, (float)c2);
  NNLAUNCH(nn);
  return nn_repack(nn, nn->stream);
}

pf_status pf_nn_layer(pf_nn* nn, int op, int layer, const void* in, const void* aux, void* out, int n, int D, int H, int W) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (layer < 0 || layer >= kLayers) return nn_fail(nn, PF_ERR_INVALID_ARG, "layer must be 0..3");
  if (!in || !out) return nn_fail(nn, PF_ERR_INVALID_ARG, "in and out are required");
  // the kernels read and write 16-byte channel groups
  if (((uintptr_t)in | (uintptr_t)aux | (uintptr_t)out) & 15u)
    return nn_fail(nn, PF_ERR_INVALID_ARG, "in, aux and out must be 16-byte aligned");
  const Vol v{n, D, H, W};
  pf_status s = nn_check_vol(nn, v);
  if (s != PF_OK) return s;
  const uint16_t* x = reinterpret_cast<const uint16_t*>(in);
  switch (op) {
    case PF_NN_OP_FORWARD:
      return nn_conv_fwd(nn, layer, x, out, v, nn->stream);
    case PF_NN_OP_BACKWARD_DATA:
      if (layer == 0) return nn_fail(nn, PF_ERR_INVALID_ARG, "the input gradient of layer 0 is not computed");
      if (!aux) return nn_fail(nn, PF_ERR_INVALID_ARG, "backward-data needs the layer input as mask");
      return nn_conv_bwd(nn, layer, x, reinterpret_cast<const uint16_t*>(aux), reinterpret_cast<uint16_t*>(out), v, nn->stream);
    case PF_NN_OP_BACKWARD_WEIGHT: {
      if (!nn->cfg.training) return nn_fail(nn, PF_ERR_INVALID_ARG, "created without training buffers");
      if (!aux) return nn_fail(nn, PF_ERR_INVALID_ARG, "backward-weight needs the output gradient");
      float* gw = reinterpret_cast<float*>(out);
      return nn_conv_wgrad(nn, layer, x, reinterpret_cast<const uint16_t*>(aux), gw,
                           gw + (size_t)pfn::kTaps * kDef[layer].cout * kDef[layer].cin, v, nn->stream);
    }
    default:
      return nn_fail(nn, PF_ERR_INVALID_ARG, "unknown op %d", op);
  }
}

// The increment scale's reduction: kStaticScaleBlocks FP64 partials, then one block.
constexpr int kStaticScaleBlocks = 1024;
constexpr long long kStaticScaleMaxCells = (1LL << 31) - 1;   // largest (nx+1)(ny+1)(nz+1) of the static variant

pf_status pf_nn_increment_scale(pf_nn* nn, const double* const* u1, const double* const* u0, int nx, int ny, int nz,
                                double* s_out) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (!u1 || !u1[0] || !u1[1] || !u1[2]) return nn_fail(nn, PF_ERR_INVALID_ARG, "u1 needs three device arrays");
  if (nx < 1 || ny < 1 || nz < 1) return nn_fail(nn, PF_ERR_INVALID_ARG, "grid sizes must be >= 1");
  pfn::PackArgs<double> a{};
  for (int d = 0; d < 3; ++d) {
    a.u1[d] = xview_face(u1[d], d, nx, ny);
    a.u0[d] = xview_face(u0 ? u0[d] : nullptr, d, nx, ny);
  }
  a.nx = nx; a.ny = ny; a.nz = nz;
  const int nblk = kStaticScaleBlocks;
  hipLaunchKernelGGL((pfn::k_incr_sumsq<double>), dim3(nblk), dim3(pfn::CNT), 0, nn->stream, a, nn->dpart);
  hipLaunchKernelGGL(pfn::k_incr_scale, dim3(1), dim3(pfn::CNT), 0, nn->stream, (const double*)nn->dpart, nblk,
                     3.0 * nx * (double)ny * nz, nn->dscal);
  NNLAUNCH(nn);
  if (s_out) {
    NNCHK(nn, hipMemcpyAsync(s_out, nn->dscal, sizeof(double), hipMemcpyDeviceToHost, nn->stream));
    NNCHK(nn, hipStreamSynchronize(nn->stream));
  }
  return PF_OK;
}

// ---------------------------------------------------------------------------
// Increment scale without any allocation: the block partials and nothing else
// live in this file-scope device array (one copy per GPU, held until the
// process ends).  Host code never passes the array's name to a kernel: the
// device address of each GPU's copy is looked up once, with that GPU
// current, and kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kStaticScaleBlocks];
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

static pf_status static_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return nn_fail(nullptr, PF_ERR_HIP, "no current HIP device (or device index >= %d)", kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return nn_fail(nullptr, PF_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = reinterpret_cast<double*>(g_scratch_ptr[dev]);
  return PF_OK;
}

pf_status pf_increment_scale_static(const double* const* u1, const double* const* u0, int nx, int ny, int nz,
                                    double* s_dev, void* hip_stream) {
  if (!u1 || !u1[0] || !u1[1] || !u1[2]) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "u1 needs three device arrays");
  if (u0 && (!u0[0] || !u0[1] || !u0[2])) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "u0 needs three device arrays or NULL");
  if (!s_dev) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "s_dev is NULL");
  if (nx < 1 || ny < 1 || nz < 1) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "grid sizes must be >= 1");
  if (((long long)nx + 1) * ((long long)ny + 1) * ((long long)nz + 1) > kStaticScaleMaxCells)
    return nn_fail(nullptr, PF_ERR_INVALID_ARG, "grid %dx%dx%d exceeds the %lld cells this entry point takes", nx, ny, nz,
                   (long long)kStaticScaleMaxCells);
  double* part = nullptr;
  pf_status st = static_scratch(&part);
  if (st != PF_OK) return st;
  pfn::PackArgs<double> a{};
  for (int d = 0; d < 3; ++d) {
    a.u1[d] = xview_face(u1[d], d, nx, ny);
    a.u0[d] = xview_face(u0 ? u0[d] : nullptr, d, nx, ny);
  }
  a.nx = nx; a.ny = ny; a.nz = nz;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  // every block writes its partial, so nothing left by an earlier call is read
  hipLaunchKernelGGL((pfn::k_incr_sumsq<double>), dim3(kStaticScaleBlocks), dim3(pfn::CNT), 0, stream, a, part);
  hipLaunchKernelGGL(pfn::k_incr_scale, dim3(1), dim3(pfn::CNT), 0, stream, (const double*)part, kStaticScaleBlocks,
                     3.0 * nx * (double)ny * nz, s_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return nn_fail(nullptr, PF_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
  return PF_OK;
}

pf_status pf_nn_pack(pf_nn* nn, const double* phi_f, const double* phi_w, const double* phi_prev,
                     const double* const* u1, const double* const* u0, const double* const* u2, int nx, int ny, int nz,
                     int x0, int y0, int z0, int cx, int cy, int cz, int slot, double Omega, double h) {
  if (!nn) return nn_fail(nullptr, PF_ERR_INVALID_ARG, "nn is NULL");
  if (!phi_f || !phi_w || !phi_prev || !u1 || !u1[0] || !u1[1] || !u1[2])
    return nn_fail(nn, PF_ERR_INVALID_ARG, "phi_f, phi_w, phi_prev and u1 are required");
  if (u2 && (!u2[0] || !u2[1] || !u2[2])) return nn_fail(nn, PF_ERR_INVALID_ARG, "u2 needs three arrays");
  if (u2 && !nn->target) return nn_fail(nn, PF_ERR_INVALID_ARG, "targets need a network created for training");
  if (nx < 1 || ny < 1 || nz < 1 || cx < 1 || cy < 1 || cz < 1 || x0 < 0 || y0 < 0 || z0 < 0 || slot < 0)
    return nn_fail(nn, PF_ERR_INVALID_ARG, "bad grid, crop or slot");
  const long long cv = (long long)cx * cy * cz;
  if ((long long)(slot + 1) * cv > nn->cap) return nn_fail(nn, PF_ERR_INVALID_ARG, "slot %d exceeds the capacity", slot);
  pfn::PackArgs<double> a{};
  a.phi_f = xview_cell(phi_f, nx, ny);
  a.phi_w = xview_cell(phi_w, nx, ny);
  a.phi_prev = xview_cell(phi_prev, nx, ny);
  for (int d = 0; d < 3; ++d) {
    a.u1[d] = xview_face(u1[d], d, nx, ny);
    a.u0[d] = xview_face(u0 ? u0[d] : nullptr, d, nx, ny);
    a.u2[d] = xview_face(u2 ? u2[d] : nullptr, d, nx, ny);
  }
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.x0 = x0; a.y0 = y0; a.z0 = z0;
  a.cx = cx; a.cy = cy; a.cz = cz;
  a.Omega = Omega;
  a.h = h;
  a.s = nn->dscal;
  a.x = nn->x0 + (size_t)slot * cv * 8;
  a.target = u2 ? nn->target + (size_t)slot * cv * 4 : nullptr;
  const int nblk = (int)std::max(1LL, std::min(4096LL, (cv + pfn::CNT - 1) / pfn::CNT));
  hipLaunchKernelGGL((pfn::k_pack_inputs<double>), dim3(nblk), dim3(pfn::CNT), 0, nn->stream, a);
  NNLAUNCH(nn);
  return PF_OK;
}

pf_status pf_nn_attach(pf_ctx* c, pf_nn* nn) {
  if (!c) return fail(nullptr, PF_ERR_INVALID_ARG, "ctx is NULL");
  if (nn && c->cfg.dim != 3) return fail(c, PF_ERR_UNSUPPORTED, "the learned warm start is 3D only");
  if (nn && c->cfg.warm != PF_WARM_LEARNED)
    return fail(c, PF_ERR_INVALID_ARG, "the context was not created with the learned warm start");
  if (nn && (long long)c->cfg.nx * c->cfg.ny * c->cfg.nz > nn->cap)
    return fail(c, PF_ERR_INVALID_ARG, "the grid exceeds the network's capacity");
  c->net = nn;
  return PF_OK;
}

}  // extern "C"
