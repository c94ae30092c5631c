// Field fitting: forward with saved pre-activations and a hand-written backward of one
// field MLP (weights and per-point latents), for minimising squared error against
// snapshots (paper Sec. 4.5; supplementary "Training Details").
//
// Network: a_1 = W_1 [X; z] + b_1, h_k = ELU(a_k), a_{k+1} = W_{k+1} h_k + b_{k+1}
// (k = 1..4), out = W_6 h_5 + b_6. Given dout = dLoss/dout per point:
//   delta_6 = dout,  delta_k = (W_{k+1}^T delta_{k+1}) * ELU'(a_k)   (k = 5 .. 1)
//   dW_k += sum_p delta_k h_{k-1}^T, db_k += sum_p delta_k          (h_0 = [X; z])
//   dz = W_1[:, 3:]^T delta_1, dX = W_1[:, :3]^T delta_1.
//
// Kernels. The forward is the field kernel of the latent step (per-point latents, raw
// output, pre-activations stored point-major: FP32, or BF16 for BF16 training). The
// backward-data kernel carries the deltas through the W^T products on MFMA (the same
// accumulator-layout chaining as the forward, with the transposed weights packed on the
// device): FP32 training takes 32 points per wave on FP32 products with dz and dX on the
// VALU; BF16 training takes 16-point tiles on BF16 products against transposed layers
// resident in LDS, stores its deltas in BF16 and forms dz and dX on FP32 MFMA. The weight
// gradients are reductions over points on MFMA: each workgroup sums a chunk of points for
// one layer into a partial, and the partials are added in a fixed order (deterministic)
// into dW.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "nsf.h"
#include "nsf_dev.h"
#include "pack.h"

namespace nsf {
namespace {

typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int acc_n(int mb, int i, int h) { return 32 * mb + 8 * (i >> 2) + 4 * h + (i & 3); }

// The forward kernels carry scaled pre-activations a' = log2(e) a (see pack.cpp): layer 1
// and the hidden biases are packed times log2(e), the output layer times ln 2.
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
__device__ __forceinline__ float scaled(float w, double f) { return (float)((double)w * f); }

// ---- device packing (same orders as pack.cpp, plus transposed hidden layers) --------
struct Packed {
  float* whp; uint16_t* whb; float* b6; float* w1q; float* bhq; float* w6q;  // forward
  float* w6p; float* whtp;                                                     // backward, FP32
  uint16_t* whbt; float* w1t; float* w6t;                                      // backward, BF16
};

// Fragment counts of the BF16 backward's FP32 operands: W1^T (in = 3 + r rows in blocks
// of 16, K-step pairs over the width) and W6^T (width rows, output components in K-steps
// of 4).
__host__ __device__ inline int w1t_blocks(int r) { return (3 + r + 15) / 16; }
__host__ __device__ inline int w6t_ksteps(int d) { return (d + 3) / 4; }

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void pack_kernel(const float* __restrict__ master, int r, int W, int d, Packed P) {
  const int in1 = 3 + r, MB = W / 32, MQ = W / 16, K1q = (r + 7) / 4;
  const float* W1 = master;
  const float* b1 = W1 + (size_t)W * in1;
  const float* hid = b1 + W;   // W2 b2 W3 b3 W4 b4 W5 b5
  const float* W6 = hid + 4 * ((size_t)W * W + W);
  const float* b6 = W6 + (size_t)d * W;
  const int64_t n1q = (int64_t)MQ * K1q * 64, nh = (int64_t)4 * W * W, nb = 4 * W, n6 = (int64_t)d * W;
  const int MB1 = w1t_blocks(r), K6 = w6t_ksteps(d);
  const int64_t n1t = (int64_t)MB1 * (W / 8) * 128, n6t = (int64_t)MQ * K6 * 64;
  const int64_t total = n1q + 3 * nh + nb + 2 * n6 + d + nh + n1t + n6t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = e;
    if (t < n1q) {   // layer 1, 16x16x4 A operands
      const int l = t % 64, s4 = (t / 64) % K1q, mb = t / (64 * K1q);
      const int m = 16 * mb + (l & 15), k = 4 * s4 + (l >> 4);
      P.w1q[t] = k < in1 ? scaled(W1[(size_t)m * in1 + k], kLog2e) : (k == in1 ? scaled(b1[m], kLog2e) : 0.f);
      continue;
    }
    t -= n1q;
    if (t < nh) {   // FP32 forward: [4][W/16][W/8][64][2]
      const int j = t % 2, l = (t / 2) % 64, hs = (t / 128) % (W / 8), mb = (t / (128 * (W / 8))) % MQ;
      const int kk = t / ((int64_t)W * W);
      const int m = 16 * mb + (l & 15), nn = 16 * (hs >> 1) + 4 * (l >> 4) + 2 * (hs & 1) + j;
      P.whp[t] = hid[kk * ((size_t)W * W + W) + (size_t)m * W + nn];
      continue;
    }
    t -= nh;
    if (t < nh) {   // BF16 forward: [4][W/16][W/32][64][8]
      const int j = t % 8, l = (t / 8) % 64, s = (t / 512) % (W / 32), mb = (t / (512 * (W / 32))) % MQ;
      const int kk = t / ((int64_t)W * W);
      const int m = 16 * mb + (l & 15), nn = 16 * (2 * s + (j >> 2)) + 4 * (l >> 4) + (j & 3);
      P.whb[t] = to_bf16(hid[kk * ((size_t)W * W + W) + (size_t)m * W + nn]);
      continue;
    }
    t -= nh;
    if (t < nh) {   // FP32 transposed (backward): A[m][s] = W[nn(s)][m]
      const int j = t % 4, l = (t / 4) % 64, sg = (t / 256) % (W / 8), mb = (t / (256 * (W / 8))) % MB;
      const int kk = t / ((int64_t)W * W);
      const int s = 4 * sg + j, m = 32 * mb + (l & 31), nn = acc_n(s / 16, s % 16, l >> 5);
      P.whtp[t] = hid[kk * ((size_t)W * W + W) + (size_t)nn * W + m];
      continue;
    }
    t -= nh;
    if (t < nb) {   // hidden biases, plain order
      const int n = t % W, kk = t / W;
      P.bhq[t] = scaled(hid[kk * ((size_t)W * W + W) + (size_t)W * W + n], kLog2e);
      continue;
    }
    t -= nb;
    if (t < n6) {   // output weights, plain order (forward)
      const int n = t % W, o = t / W;
      P.w6q[t] = scaled(W6[(size_t)o * W + n], kLn2);
      continue;
    }
    t -= n6;
    if (t < n6) {   // output weights in 32x32 accumulator order (backward)
      const int s = t % (W / 2), h = (t / (W / 2)) % 2, o = t / W;
      P.w6p[t] = scaled(W6[(size_t)o * W + acc_n(s / 16, s % 16, h)], kLn2);
      continue;
    }
    t -= n6;
    if (t < d) {
      P.b6[t] = b6[t];
      continue;
    }
    t -= d;
    if (t < nh) {   // BF16 transposed (backward): [4][W/16][W/32][64][8], A[m][nn] = W[nn][m]
      const int j = t % 8, l = (t / 8) % 64, s = (t / 512) % (W / 32), mb = (t / (512 * (W / 32))) % MQ;
      const int kk = t / ((int64_t)W * W);
      const int m = 16 * mb + (l & 15), nn = 16 * (2 * s + (j >> 2)) + 4 * (l >> 4) + (j & 3);
      P.whbt[t] = to_bf16(hid[kk * ((size_t)W * W + W) + (size_t)nn * W + m]);
      continue;
    }
    t -= nh;
    if (t < n1t) {   // W1^T (16x16x4, K-step pairs): [MB1][W/8][64][2], rows past 3 + r zero
      const int j = t % 2, l = (t / 2) % 64, hs = (t / 128) % (W / 8), mb = t / (128 * (W / 8));
      const int m = 16 * mb + (l & 15), nn = 16 * (hs >> 1) + 4 * (l >> 4) + 2 * (hs & 1) + j;
      P.w1t[t] = m < in1 ? W1[(size_t)nn * in1 + m] : 0.f;
      continue;
    }
    t -= n1t;
    {   // W6^T (16x16x4): [W/16][K6][64], components past d zero
      const int l = t % 64, s = (t / 64) % K6, mb = t / (64 * K6);
      const int m = 16 * mb + (l & 15), k = 4 * s + (l >> 4);
      P.w6t[t] = k < d ? W6[(size_t)k * W + m] : 0.f;
    }
  }
}

// ELU'(a) and ELU(a) from a saved scaled pre-activation a' = log2(e) a.
__device__ __forceinline__ float elu_prime(float as) { return as > 0.f ? 1.f : __builtin_amdgcn_exp2f(as); }
__device__ __forceinline__ float elu(float as) {
  return as > 0.f ? as * (float)kLn2 : __builtin_amdgcn_exp2f(as) - 1.f;
}

// ---- backward through the network, 32 points per wave --------------------------------
template <int W>
__global__ __launch_bounds__(256) void backward_data_kernel(const float* __restrict__ master,
                                                            const float* __restrict__ whtp,
                                                            const float* __restrict__ w6p,
                                                            const float* __restrict__ saved,
                                                            const float* __restrict__ dout,
                                                            float* __restrict__ delta,
                                                            float* __restrict__ dz,
                                                            float* __restrict__ dX,
                                                            int n, int r, int d) {
  constexpr int MB = W / 32, KH = W / 2;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nw = (gridDim.x * blockDim.x) >> 6;
  const int in1 = 3 + r;
  for (int t = wave; t * 32 < n; t += nw) {
    const int p = t * 32 + (lane & 31);
    const bool valid = p < n;
    const int pc = valid ? p : n - 1;
    float d6[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) d6[o] = (o < d && valid) ? dout[(int64_t)o * n + p] : 0.f;
    // delta_5 = (W6^T delta_6) * ELU'(a_5), in accumulator order
    float D[KH];
    const float* a5 = saved + ((int64_t)4 * n + pc) * W;
#pragma unroll
    for (int s = 0; s < KH; ++s) {
      float g = 0.f;
#pragma unroll
      for (int o = 0; o < 9; ++o)
        if (o < d) g += w6p[(o * 2 + h) * KH + s] * d6[o];
      // w6p holds ln 2 W6: undo the scale
      D[s] = g * (float)kLog2e * elu_prime(a5[acc_n(s / 16, s % 16, h)]);
    }
    for (int L = 4; L >= 0; --L) {
      // store delta_{L+1} point-major
      if (valid) {
        float* row = delta + ((int64_t)L * n + p) * W;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            *reinterpret_cast<f32x4*>(row + 32 * mb + 8 * q + 4 * h) =
                f32x4{D[16 * mb + 4 * q], D[16 * mb + 4 * q + 1], D[16 * mb + 4 * q + 2], D[16 * mb + 4 * q + 3]};
      }
      if (L == 0) break;
      // g_L = W_{L+1}^T delta_{L+1} on MFMA (hidden pack L - 1 maps h_L -> a_{L+1})
      f32x16_t acc[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x16_t{};
      const f32x4* A = reinterpret_cast<const f32x4*>(whtp + (size_t)(L - 1) * W * W);
#pragma unroll
      for (int sg = 0; sg < W / 8; ++sg) {
        f32x4 a4[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) a4[mb] = A[(mb * (W / 8) + sg) * 64 + lane];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[mb][j], D[4 * sg + j], acc[mb], 0, 0, 0);
      }
      const float* aL = saved + ((int64_t)(L - 1) * n + pc) * W;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 16; ++i) D[16 * mb + i] = acc[mb][i] * elu_prime(aL[acc_n(mb, i, h)]);
    }
    // dz_j = sum_n W1[n][3 + j] delta_1[n]
    for (int j = 0; j < r; ++j) {
      float s = 0.f;
#pragma unroll
      for (int s_ = 0; s_ < KH; ++s_) s += master[(size_t)acc_n(s_ / 16, s_ % 16, h) * in1 + 3 + j] * D[s_];
      s += __shfl_xor(s, 32);
      if (valid && h == (j & 1) && dz != nullptr) dz[(int64_t)p * r + j] = s;
    }
    // dX_c = sum_n W1[n][c] delta_1[n], SoA like X
    if (dX != nullptr)
      for (int c = 0; c < 3; ++c) {
        float s = 0.f;
#pragma unroll
        for (int s_ = 0; s_ < KH; ++s_) s += master[(size_t)acc_n(s_ / 16, s_ % 16, h) * in1 + c] * D[s_];
        s += __shfl_xor(s, 32);
        if (valid && h == (c & 1)) dX[(int64_t)c * n + p] = s;
      }
  }
}

// ---- BF16 backward through the network, 16 points per wave --------------------------------
// The tile layout of the BF16 field kernels: lane l holds point p0 + l % 16 and, of every
// 16-neuron block mb, neurons 16 mb + 4 (l / 16) + v in accumulator register v. The four
// transposed hidden layers (BF16 A fragments, 32 KB each at width 128) and W1^T (FP32) stay
// in LDS for the workgroup's life; W6^T is read through the caches.
//   delta_5 = (W6^T dout) * ELU'(a_5): FP32 16x16x4 products over the output components;
//   delta_k = (W_{k+1}^T delta_{k+1}) * ELU'(a_k): the delta rounded to BF16 once as the
//     B operand (its registers are already in the order the packed A expects, as in the
//     forward), 16x16x32 BF16 products with FP32 accumulation;
//   [dX; dz] = W1^T delta_1: FP32 16x16x4 products on the unrounded delta_1.
// ELU' comes from the saved BF16 pre-activations; every delta is stored in BF16 for the
// weight gradients, point-major [5][n][W].
constexpr int kBwdWaves = 8;

typedef __attribute__((address_space(3))) void lds_void;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

struct BwdArgs {
  const uint16_t* whbt;   // [4][W/16][W/32][64][8]
  const float* w1t;       // [MB1][W/8][64][2]
  const float* w6t;       // [W/16][K6][64]
  const __bf16* saved;    // scaled pre-activations [5][n][W]
  const float* dout;      // [d][n]
  __bf16* delta;          // [5][n][W]
  float* dz;              // [n][r] or NULL
  float* dX;              // [3][n] or NULL
  int n, r, d;
};

template <int W>
constexpr int bwd_lds_bytes() { return 4 * W * W * 2 + 3 * (W / 8) * 128 * 4; }

__device__ __forceinline__ f32x4 mfma16f(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int W>
__global__ __launch_bounds__(64 * kBwdWaves) void backward_bf16_kernel(BwdArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int MB = W / 16, S = W / 32, HS = W / 8;
  constexpr int kLayerBytes = W * W * 2;
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = a.n, tiles = (n + 15) / 16;
  const int MB1 = w1t_blocks(a.r), K6 = w6t_ksteps(a.d);
  // the transposed hidden layers by direct global -> LDS loads, W1^T by the threads
  {
    const char* src = reinterpret_cast<const char*>(a.whbt);
    for (int c = wave; c < 4 * kLayerBytes / 1024; c += kBwdWaves)
      __builtin_amdgcn_global_load_lds(src + c * 1024 + lane * 16, (lds_void*)(lds + c * 1024), 16, 0, 0);
    float* w1 = reinterpret_cast<float*>(lds + 4 * kLayerBytes);
    for (int i = threadIdx.x; i < MB1 * HS * 128; i += 64 * kBwdWaves) w1[i] = a.w1t[i];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  const bf16x8* At = reinterpret_cast<const bf16x8*>(lds);
  const f32x2* W1t = reinterpret_cast<const f32x2*>(lds + 4 * kLayerBytes);
  // All of a tile's inputs (its output gradients and the saved values of its five layers)
  // are loaded at the tile's start: one memory latency per tile instead of one per layer.
  // (Loading the next tile's during the current one needs more than the 256 registers.)
  const int stride = gridDim.x * kBwdWaves;
  bf16x4 hi[3][MB];   // layers 5, 4, 3
  bf16x4 lo[2][MB];   // layers 2, 1
  float nb[3];
  auto load_rows = [&](int tt, int i, bf16x4 (&dst)[MB]) {   // layer i (1..5) of tile tt
    const int pp = tt * 16 + (lane & 15);
    const int pcc = pp < n ? pp : n - 1;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      dst[mb] = *reinterpret_cast<const bf16x4*>(a.saved + ((int64_t)(i - 1) * n + pcc) * W + 4 * g + 16 * mb);
  };
  auto load_hi = [&](int tt) {
    const int pp = tt * 16 + (lane & 15);
#pragma unroll
    for (int i = 5; i >= 3; --i) load_rows(tt, i, hi[5 - i]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int o = 4 * k + g;
      nb[k] = (k < K6 && o < a.d && pp < n) ? a.dout[(int64_t)o * n + pp] : 0.f;
    }
  };
  int t = blockIdx.x * kBwdWaves + wave;
  for (; t < tiles; t += stride) {
    const int p = t * 16 + (lane & 15);
    const bool valid = p < n;
    load_hi(t);
    load_rows(t, 2, lo[0]);
    load_rows(t, 1, lo[1]);
    f32x4 D[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) D[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k >= K6) break;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) D[mb] = mfma16f(a.w6t[(mb * K6 + k) * 64 + lane], nb[k], D[mb]);
    }
    // layer i = 5 .. 1: D = W_{i+1}^T delta_{i+1} (W6^T dout for i = 5) at layer i's neurons
#pragma unroll
    for (int i = 5; i >= 1; --i) {
      const bf16x4 (&av)[MB] = i >= 3 ? hi[5 - i] : lo[2 - i];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float as = (float)av[mb][v];
          D[mb][v] *= as > 0.f ? 1.f : __builtin_amdgcn_exp2f(as);
        }
      if (valid) {
        __bf16* drow = a.delta + ((int64_t)(i - 1) * n + p) * W + 4 * g;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          *reinterpret_cast<bf16x4*>(drow + 16 * mb) =
              bf16x4{(__bf16)D[mb][0], (__bf16)D[mb][1], (__bf16)D[mb][2], (__bf16)D[mb][3]};
      }
      if (i == 1) break;
      bf16x8 B[S];
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) B[s][e] = (__bf16)D[2 * s + (e >> 2)][e & 3];
      // hidden pack i - 2 maps h_{i-1} to a_i; its transpose maps delta_i back
      const bf16x8* A = At + (size_t)(i - 2) * (kLayerBytes / 16);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) D[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
      // A fragments read four products ahead; the scheduling barriers keep the compiler
      // from hoisting the whole layer's reads (registers)
      constexpr int NS = S * MB, PF = 4, RING = PF + 1;
      auto at = [&](int st) { return A[((st % MB) * S + st / MB) * 64 + lane]; };
      bf16x8 ring[RING];
#pragma unroll
      for (int u = 0; u < PF; ++u) ring[u] = at(u);
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        if (st + PF < NS) ring[(st + PF) % RING] = at(st + PF);
        __builtin_amdgcn_sched_barrier(0);
        D[st % MB] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ring[st % RING], B[st / MB], D[st % MB], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (a.dz == nullptr && a.dX == nullptr) continue;
    // [dX; dz] = W1^T delta_1: K-step pair hs reads registers 2 (hs % 2) + j of block hs / 2
    f32x4 Z[3];
#pragma unroll
    for (int m1 = 0; m1 < 3; ++m1) Z[m1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m1 = 0; m1 < 3; ++m1) {
      if (m1 >= MB1) break;
      constexpr int PF = 4, RING = PF + 1;
      f32x2 ring[RING];
#pragma unroll
      for (int u = 0; u < PF; ++u) ring[u] = W1t[(m1 * HS + u) * 64 + lane];
#pragma unroll
      for (int hs = 0; hs < HS; ++hs) {
        if (hs + PF < HS) ring[(hs + PF) % RING] = W1t[(m1 * HS + hs + PF) * 64 + lane];
        __builtin_amdgcn_sched_barrier(0);
        Z[m1] = mfma16f(ring[hs % RING][0], D[hs >> 1][2 * (hs & 1)], Z[m1]);
        Z[m1] = mfma16f(ring[hs % RING][1], D[hs >> 1][2 * (hs & 1) + 1], Z[m1]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (!valid) continue;
#pragma unroll
    for (int m1 = 0; m1 < 3; ++m1) {
      if (m1 >= MB1) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * m1 + 4 * g + v;   // input row: X for m < 3, then z
        if (m < 3) {
          if (a.dX) a.dX[(int64_t)m * n + p] = Z[m1][v];
        } else if (m < 3 + a.r && a.dz) {
          a.dz[(int64_t)p * a.r + (m - 3)] = Z[m1][v];
        }
      }
    }
  }
}

// One workgroup per CU (the resident layers take most of its LDS), each wave looping over
// 16-point tiles.
template <int W>
hipError_t launch_backward_bf16_w(const BwdArgs& a, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)backward_bf16_kernel<W>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, bwd_lds_bytes<W>());
    if (e != hipSuccess) return e;
    attr = true;
  }
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  const int tiles = (a.n + 15) / 16;
  const int grid = std::max(1, std::min(cus, (tiles + kBwdWaves - 1) / kBwdWaves));
  hipLaunchKernelGGL(backward_bf16_kernel<W>, dim3(grid), dim3(64 * kBwdWaves), bwd_lds_bytes<W>(), s, a);
  return hipGetLastError();
}

hipError_t launch_backward_bf16(int W, const BwdArgs& a, hipStream_t s) {
  if (a.r < 1 || a.r > 32 || a.d < 1 || a.d > 9) return hipErrorInvalidValue;   // MB1 <= 3, K6 <= 3
  return W == 64 ? launch_backward_bf16_w<64>(a, s) : launch_backward_bf16_w<128>(a, s);
}

constexpr int kChunk = 1024;   // points per weight-gradient workgroup (FP32)
// BF16: half the chunk, so that two workgroups share each CU and twice the loads are in
// flight (the kernel streams its operands; the products are a small part of its time)
constexpr int kChunk16 = 512;

// ---- weight gradients on MFMA -------------------------------------------------------------
// dW[m][j] = sum_p A(p, m) B(p, j) and db[m] = sum_p A(p, m) over one chunk of kChunk points,
// for every layer: A is the layer's delta (point-major [n][W], or the SoA dout [d][n] for
// the output layer), B its input (ELU of the saved pre-activations [n][W], or [X; z] for
// layer 1). The points are the K dimension. Each stage brings kGStage points of A and B
// into LDS as FP32, transposed to [neuron][point]; for the point-major operands the next
// stage's global loads (16 B per lane) are issued before the current stage's products. The
// four waves accumulate 32 x 32 tiles of the M x N output (M, N <= 128, padded to
// multiples of 32) on MFMA: FP32 products on v_mfma_f32_32x32x2_f32, or, for BF16
// training, operands rounded to BF16 on v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
// db is summed in FP32 from the staged A. The chunk's result goes to
// partial[chunk][m][N + 1], bias in the last column.
constexpr int kGStage = 64;        // points per stage
constexpr int kGLd = kGStage + 4;  // LDS row stride (floats): 16-byte aligned rows

enum GradKind { kGradFirst = 0, kGradHidden = 1, kGradOutput = 2 };

struct GradIn {
  const float* A;         // delta [n][W] (first, hidden) or dout [M][n] (output)
  const float* Bsaved;    // pre-activations [n][W] (hidden, output)
  const float* X;         // [3][n] (first)
  const float* zrows;     // [n][r] (first)
  int M, N, r;            // M rows (W, or d), N input columns (W, or 3 + r)
  float* partial;
};

template <int W, bool BF, int KIND>
__global__ __launch_bounds__(256) void grad_mfma_kernel(GradIn g, int n) {
  __shared__ __attribute__((aligned(16))) float sA[128][kGLd];
  __shared__ __attribute__((aligned(16))) float sB[128][kGLd];
  constexpr int V4 = kGStage * W / 4 / 256;   // float4 per thread per point-major stage
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
  const int p0 = blockIdx.x * kChunk, p1 = min(n, p0 + kChunk);
  const int M = g.M, N = g.N;
  const int MB = (M + 31) / 32, NB = (N + 31) / 32, tiles = MB * NB;
  for (int e = tid; e < (32 * MB - M) * kGLd; e += 256) sA[M + e / kGLd][e % kGLd] = 0.f;
  for (int e = tid; e < (32 * NB - N) * kGLd; e += 256) sB[N + e / kGLd][e % kGLd] = 0.f;
  f32x16_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x16_t{};
  float db = 0.f;   // thread tid < M: bias gradient of row tid
  f32x4 ra[V4], rb[V4];
  // point-major [n][W] rows of the stage starting at ps into registers (zero past p1)
  auto load_pm = [&](const float* src, f32x4 (&r)[V4], int ps) {
#pragma unroll
    for (int i = 0; i < V4; ++i) {
      const int e = tid + 256 * i, pt = e / (W / 4), c4 = (e % (W / 4)) * 4;
      r[i] = ps + pt < p1 ? *reinterpret_cast<const f32x4*>(src + (int64_t)(ps + pt) * W + c4)
                          : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto store_pm = [&](float (*dst)[kGLd], const f32x4 (&r)[V4], bool act) {
#pragma unroll
    for (int i = 0; i < V4; ++i) {
      const int e = tid + 256 * i, pt = e / (W / 4), c4 = (e % (W / 4)) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[c4 + q][pt] = act ? elu(r[i][q]) : r[i][q];
    }
  };
  auto load_next = [&](int ps) {
    if constexpr (KIND != kGradOutput) load_pm(g.A, ra, ps);
    if constexpr (KIND != kGradFirst) load_pm(g.Bsaved, rb, ps);
  };
  load_next(p0);
  for (int ps = p0; ps < p1; ps += kGStage) {
    const int cnt = min(kGStage, p1 - ps);
    if constexpr (KIND != kGradOutput) {
      store_pm(sA, ra, false);
    } else {   // dout [M][n], M <= 9
      for (int e = tid; e < M * kGStage; e += 256) {
        const int m = e / kGStage, pt = e % kGStage;
        sA[m][pt] = pt < cnt ? g.A[(int64_t)m * n + ps + pt] : 0.f;
      }
    }
    if constexpr (KIND != kGradFirst) {
      // the saved values are rows of pre-activations; padded points stay exactly zero
      store_pm(sB, rb, true);
      if (cnt < kGStage)
        for (int e = tid; e < W * (kGStage - cnt); e += 256) sB[e / (kGStage - cnt)][cnt + e % (kGStage - cnt)] = 0.f;
    } else {   // [X; z], N = 3 + r
      for (int e = tid; e < N * kGStage; e += 256) {
        const int j = e / kGStage, pt = e % kGStage;
        float v = 0.f;
        if (pt < cnt)
          v = j < 3 ? g.X[(int64_t)j * n + ps + pt] : g.zrows[(int64_t)(ps + pt) * g.r + (j - 3)];
        sB[j][pt] = v;
      }
    }
    __syncthreads();
    if (ps + kGStage < p1) load_next(ps + kGStage);   // in flight during the products below
    if (tid < M)
      for (int pt = 0; pt < cnt; ++pt) db += sA[tid][pt];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int tile = wave + 4 * t;
      if (tile >= tiles) break;
      const int mb = tile / NB, nb = tile % NB;
      const float* arow = sA[32 * mb + (lane & 31)];
      const float* brow = sB[32 * nb + (lane & 31)];
      if constexpr (BF) {
#pragma unroll
        for (int k0 = 0; k0 < kGStage; k0 += 16) {
          const int kk = k0 + 8 * h;
          const f32x4 a0 = *reinterpret_cast<const f32x4*>(arow + kk);
          const f32x4 a1 = *reinterpret_cast<const f32x4*>(arow + kk + 4);
          const f32x4 b0 = *reinterpret_cast<const f32x4*>(brow + kk);
          const f32x4 b1 = *reinterpret_cast<const f32x4*>(brow + kk + 4);
          bf16x8 a, b;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a[q] = (__bf16)a0[q];
            a[4 + q] = (__bf16)a1[q];
            b[q] = (__bf16)b0[q];
            b[4 + q] = (__bf16)b1[q];
          }
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int k0 = 0; k0 < kGStage; k0 += 2)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(arow[k0 + h], brow[k0 + h], acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* out = g.partial + (int64_t)blockIdx.x * M * (N + 1);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= tiles) break;
    const int mb = tile / NB, nb = tile % NB;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int m = 32 * mb + 8 * (e >> 2) + 4 * h + (e & 3);
      const int j = 32 * nb + (lane & 31);
      if (m < M && j < N) out[m * (N + 1) + j] = acc[t][e];
    }
  }
  if (tid < M) out[tid * (N + 1) + N] = db;
}

// BF16 training: the deltas and saved pre-activations arrive in BF16 ([n][W], point-major)
// and are staged in LDS as BF16, [neuron][point], so that each 32x32x16 product reads its
// operands with one 16-byte LDS read per lane and converts nothing. B of the hidden and
// output layers is ELU of the saved value, rounded to BF16 as it is staged.
constexpr int kGLd16 = kGStage + 8;   // LDS row stride (BF16 elements): 16-byte aligned rows

struct GradIn16 {
  const __bf16* A;        // delta [n][W] (first, hidden)
  const float* dout;      // [M][n] (output)
  const __bf16* Bsaved;   // pre-activations [n][W] (hidden, output)
  const float* X;         // [3][n] (first)
  const float* zrows;     // [n][r] (first)
  int M, N, r;
  float* partial;
};

template <int W, int KIND>
__global__ __launch_bounds__(256) void grad_bf16_kernel(GradIn16 g, int n) {
  __shared__ __attribute__((aligned(16))) __bf16 sA[128][kGLd16];
  __shared__ __attribute__((aligned(16))) __bf16 sB[128][kGLd16];
  constexpr int V8 = kGStage * W / 8 / 256;   // 16-byte loads per thread per point-major stage
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
  const int p0 = blockIdx.x * kChunk16, p1 = min(n, p0 + kChunk16);
  const int M = g.M, N = g.N;
  const int MB = (M + 31) / 32, NB = (N + 31) / 32, tiles = MB * NB;
  const __bf16 zero = (__bf16)0.f;
  for (int e = tid; e < (32 * MB - M) * kGLd16; e += 256) sA[M + e / kGLd16][e % kGLd16] = zero;
  for (int e = tid; e < (32 * NB - N) * kGLd16; e += 256) sB[N + e / kGLd16][e % kGLd16] = zero;
  f32x16_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x16_t{};
  float db = 0.f;
  bf16x8 ra[V8], rb[V8];
  // lane = point of the stage, wave w = the 16-byte chunks w V8 .. w V8 + V8 - 1 of the
  // rows: each LDS store then writes one neuron row's 64 consecutive points (no bank
  // conflicts), and each cache line a load touches is read whole by the wave's next loads
  static_assert(kGStage == 64 && W / 8 == 4 * V8, "one point per lane, the chunks split over 4 waves");
  auto load_pm = [&](const __bf16* src, bf16x8 (&r)[V8], int ps) {
#pragma unroll
    for (int i = 0; i < V8; ++i) {
      const int c8 = 8 * (wave * V8 + i);
      if (ps + lane < p1) r[i] = *reinterpret_cast<const bf16x8*>(src + (int64_t)(ps + lane) * W + c8);
      else
#pragma unroll
        for (int q = 0; q < 8; ++q) r[i][q] = zero;
    }
  };
  auto store_pm = [&](__bf16 (*dst)[kGLd16], const bf16x8 (&r)[V8], bool act) {
#pragma unroll
    for (int i = 0; i < V8; ++i) {
      const int c8 = 8 * (wave * V8 + i);
#pragma unroll
      for (int q = 0; q < 8; ++q) dst[c8 + q][lane] = act ? (__bf16)elu((float)r[i][q]) : r[i][q];
    }
  };
  auto load_next = [&](int ps) {
    if constexpr (KIND != kGradOutput) load_pm(g.A, ra, ps);
    if constexpr (KIND != kGradFirst) load_pm(g.Bsaved, rb, ps);
  };
  load_next(p0);
  for (int ps = p0; ps < p1; ps += kGStage) {
    const int cnt = min(kGStage, p1 - ps);
    if constexpr (KIND != kGradOutput) {
      store_pm(sA, ra, false);
    } else {   // dout [M][n], M <= 9
      for (int e = tid; e < M * kGStage; e += 256) {
        const int m = e / kGStage, pt = e % kGStage;
        sA[m][pt] = (__bf16)(pt < cnt ? g.dout[(int64_t)m * n + ps + pt] : 0.f);
      }
    }
    if constexpr (KIND != kGradFirst) {
      // padded points: ELU of the zero pre-activation is zero
      store_pm(sB, rb, true);
    } else {   // [X; z], N = 3 + r
      for (int e = tid; e < N * kGStage; e += 256) {
        const int j = e / kGStage, pt = e % kGStage;
        float v = 0.f;
        if (pt < cnt) v = j < 3 ? g.X[(int64_t)j * n + ps + pt] : g.zrows[(int64_t)(ps + pt) * g.r + (j - 3)];
        sB[j][pt] = (__bf16)v;
      }
    }
    __syncthreads();
    if (ps + kGStage < p1) load_next(ps + kGStage);   // in flight during the products below
    // bias gradient of row tid: the stage's points, eight per LDS read (padding is zero)
    if (tid < M)
#pragma unroll
      for (int pt = 0; pt < kGStage; pt += 8) {
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(&sA[tid][pt]);
#pragma unroll
        for (int q = 0; q < 8; ++q) db += (float)v[q];
      }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int tile = wave + 4 * t;
      if (tile >= tiles) break;
      const int mb = tile / NB, nb = tile % NB;
      const __bf16* arow = sA[32 * mb + (lane & 31)];
      const __bf16* brow = sB[32 * nb + (lane & 31)];
#pragma unroll
      for (int k0 = 0; k0 < kGStage; k0 += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + k0 + 8 * h);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(brow + k0 + 8 * h);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* out = g.partial + (int64_t)blockIdx.x * M * (N + 1);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= tiles) break;
    const int mb = tile / NB, nb = tile % NB;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int m = 32 * mb + 8 * (e >> 2) + 4 * h + (e & 3);
      const int j = 32 * nb + (lane & 31);
      if (m < M && j < N) out[m * (N + 1) + j] = acc[t][e];
    }
  }
  if (tid < M) out[tid * (N + 1) + N] = db;
}

template <int W>
void launch_grad16(const GradIn16& g, int kind, int chunks, int n, hipStream_t s) {
  if (kind == kGradFirst) hipLaunchKernelGGL((grad_bf16_kernel<W, kGradFirst>), dim3(chunks), dim3(256), 0, s, g, n);
  else if (kind == kGradHidden) hipLaunchKernelGGL((grad_bf16_kernel<W, kGradHidden>), dim3(chunks), dim3(256), 0, s, g, n);
  else hipLaunchKernelGGL((grad_bf16_kernel<W, kGradOutput>), dim3(chunks), dim3(256), 0, s, g, n);
}

template <int W, bool BF>
void launch_grad(const GradIn& g, int kind, int chunks, int n, hipStream_t s) {
  if (kind == kGradFirst) hipLaunchKernelGGL((grad_mfma_kernel<W, BF, kGradFirst>), dim3(chunks), dim3(256), 0, s, g, n);
  else if (kind == kGradHidden) hipLaunchKernelGGL((grad_mfma_kernel<W, BF, kGradHidden>), dim3(chunks), dim3(256), 0, s, g, n);
  else hipLaunchKernelGGL((grad_mfma_kernel<W, BF, kGradOutput>), dim3(chunks), dim3(256), 0, s, g, n);
}

// dW[m][j] += sum over the chunks' partials; column N-1 goes to the bias db[m]. Wave w of
// a workgroup adds chunks w, w + G, w + 2G, ... (G waves; four running sums, four loads in
// flight) for 64 consecutive entries, and the G sums are added in wave order: the result
// does not depend on timing.
constexpr int kRedWaves = 8;

__global__ __launch_bounds__(64 * kRedWaves) void grad_reduce_kernel(const float* __restrict__ partial, int n_chunks,
                                                                     int M, int N, float* __restrict__ dW,
                                                                     float* __restrict__ db) {
  __shared__ float part[kRedWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int64_t stride = (int64_t)M * N;
  float a[4] = {0.f, 0.f, 0.f, 0.f};
  if (e < M * N) {
    int c = w;
    for (; c + 3 * kRedWaves < n_chunks; c += 4 * kRedWaves) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = partial[(int64_t)(c + u * kRedWaves) * stride + e];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += v[u];
    }
    for (int u = 0; c < n_chunks; c += kRedWaves, ++u) a[u] += partial[(int64_t)c * stride + e];
  }
  part[w][lane] = (a[0] + a[1]) + (a[2] + a[3]);
  __syncthreads();
  if (w != 0 || e >= M * N) return;
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kRedWaves; ++k) s += part[k][lane];
  const int m = e / N, j = e % N;
  if (j == N - 1) db[m] += s;
  else dW[(int64_t)m * (N - 1) + j] += s;
}

// One Adam step over n parameters (FP32, no weight decay), in PyTorch's arithmetic order:
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   w -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   float b1, float b2, float eps, float step_size,
                                                   float inv_bc2_sqrt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    w[i] -= step_size * (mi / (sqrtf(vi) * inv_bc2_sqrt + eps));
  }
}

// Per-snapshot latent rows of a minibatch whose pairs are grouped by snapshot: segment s
// covers rows [off[s], off[s + 1]). One workgroup per segment.
__global__ __launch_bounds__(256) void rows_expand_kernel(const float* __restrict__ table,
                                                          const int64_t* __restrict__ off, int width,
                                                          float* __restrict__ out) {
  const int s = blockIdx.x;
  const int64_t a = off[s] * width, b = off[s + 1] * width;
  const float* src = table + (int64_t)s * width;
  for (int64_t e = a + threadIdx.x; e < b; e += blockDim.x) out[e] = src[(e - a) % width];
}

// out[s][j] = sum of rows[i][j] over segment s: thread (j, g) adds rows g, g + G, ... of
// column j (G = 256 / width groups), then thread j adds the G sums in order.
__global__ __launch_bounds__(256) void rows_segment_sum_kernel(const float* __restrict__ rows,
                                                               const int64_t* __restrict__ off, int width,
                                                               float* __restrict__ out) {
  __shared__ float part[256];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int G = 256 / width;
  const int j = tid % width, g = tid / width;
  const int64_t a = off[s], b = off[s + 1];
  float acc = 0.f;
  if (g < G)
    for (int64_t i = a + g; i < b; i += G) acc += rows[i * width + j];
  part[tid] = acc;
  __syncthreads();
  if (tid < width) {
    float t = 0.f;
    for (int gg = 0; gg < G; ++gg) t += part[gg * width + tid];
    out[(int64_t)s * width + tid] = t;
  }
}

struct TrainWs {
  Packed pk;
  float* delta;     // [5][n][W]
  float* partial;   // [n_chunks][max M][max N]
  size_t bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

TrainWs carve(char* base, int r, int W, int d, int64_t n, bool backward) {
  TrainWs w{};
  const PackSizes ps = pack_sizes(r, W, d);
  size_t off = 0;
  auto take = [&](size_t bytes) { char* p = base ? base + off : nullptr; off += align256(bytes); return p; };
  w.pk.whp = (float*)take(ps.whp * 4);
  w.pk.whb = (uint16_t*)take(ps.whb * 2);
  w.pk.b6 = (float*)take(ps.b6 * 4);
  w.pk.w1q = (float*)take(ps.w1q * 4);
  w.pk.bhq = (float*)take(ps.bhq * 4);
  w.pk.w6q = (float*)take(ps.w6q * 4);
  w.pk.w6p = (float*)take(ps.w6p * 4);
  w.pk.whtp = (float*)take(ps.whp * 4);
  w.pk.whbt = (uint16_t*)take(ps.whb * 2);
  w.pk.w1t = (float*)take((size_t)w1t_blocks(r) * (W / 8) * 128 * 4);
  w.pk.w6t = (float*)take((size_t)(W / 16) * w6t_ksteps(d) * 64 * 4);
  if (backward) {
    w.delta = (float*)take((size_t)5 * n * W * 4);
    const int64_t chunks = (n + kChunk16 - 1) / kChunk16;   // the larger count of the two
    w.partial = (float*)take((size_t)chunks * W * (W + 1) * 4);
  }
  w.bytes = off;
  return w;
}

thread_local char g_train_err[256];

nsf_status check_mlp(const nsf_mlp* m, int64_t n) {
  if (!m || !m->weights) return NSF_EINVAL;
  if (m->width != 64 && m->width != 128) return NSF_EINVAL;
  if (m->r < 1 || m->r > kMaxR || m->d < 1 || m->d > 9) return NSF_EINVAL;
  if (n < 1 || n > (int64_t)INT32_MAX / 8) return NSF_EINVAL;
  return NSF_OK;
}

nsf_status mlp_forward(const nsf_mlp* m, const float* X, const float* z_rows, int64_t n, float* out,
                       float* saved, char* workspace, size_t workspace_bytes, hipStream_t s) {
  if (check_mlp(m, n) != NSF_OK || !X || !z_rows || !out || !workspace) return NSF_EINVAL;
  const TrainWs ws = carve(workspace, m->r, m->width, m->d, n, false);
  if (workspace_bytes < ws.bytes) return NSF_ENOMEM;
  hipLaunchKernelGGL(pack_kernel, dim3(256), dim3(256), 0, s, m->weights, m->r, m->width, m->d, ws.pk);
  if (hipGetLastError() != hipSuccess) return NSF_EHIP;
  FieldJob j{};
  j.w.whp = ws.pk.whp;
  j.w.whb = reinterpret_cast<const bf16x8*>(ws.pk.whb);
  j.w.b6 = ws.pk.b6;
  j.w.w1q = ws.pk.w1q;
  j.w.bhq = ws.pk.bhq;
  j.w.w6q = ws.pk.w6q;
  j.X = X;
  j.ldx = n;
  j.zrows = z_rows;
  j.saved = saved;
  j.saved_bf16 = m->precision == NSF_BF16;
  j.n = (int)n;
  j.r = m->r;
  j.d = m->d;
  j.out = out;
  j.ldo = n;
  for (int c = 0; c < 9; ++c) { j.scale[c] = 1.f; j.shift[c] = 0.f; }
  if (launch_fields_dense(m->width, m->precision == NSF_BF16, j, (int)n, s) != hipSuccess) return NSF_EHIP;
  return NSF_OK;
}

// The allocation-free forward's workspace: the packed weights of one field, at most
// ~0.7 MB (width 128, r = 32, d = 9). Each device holds its own copy for the life of the
// process; host code uses it only through the address hipGetSymbolAddress returns for the
// current device, never through the symbol itself.
constexpr size_t kScratchBytes = (size_t)1 << 20;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

nsf_status scratch_address(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NSF_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NSF_EHIP;
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return NSF_OK;
}

// The fitting objective: blocks of kSqErrThreads threads take pairs in a grid-stride loop,
// write the gradient and sum the squares in FP64 (per thread in pair order, then over the
// block in a fixed tree); one thread then adds the block sums in block order.
constexpr int kSqErrThreads = 256, kSqErrBlocks = NSF_SQERR_WORKSPACE_BYTES / sizeof(double);

__global__ __launch_bounds__(kSqErrThreads) void sq_err_kernel(const float* __restrict__ out, int d, int64_t n,
                                                               const float* __restrict__ Y, int64_t ldy,
                                                               const int64_t* __restrict__ rows,
                                                               const int64_t* __restrict__ cols, int64_t P,
                                                               float scale, float* grad, double* part) {
  __shared__ double red[kSqErrThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kSqErrThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSqErrThreads) {
    const int64_t q = rows[i] * P + cols[i];
    for (int c = 0; c < d; ++c) {
      const float e = out[c * n + i] - Y[c * ldy + q];
      acc += (double)e * (double)e;
      grad[c * n + i] = e * scale;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kSqErrThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sq_err_total_kernel(const double* __restrict__ part, int blocks, double inv_count, float* loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += part[b];
  loss[0] = (float)(s * inv_count);
}

}  // namespace
}  // namespace nsf

using namespace nsf;

extern "C" {

size_t nsf_mlp_param_count(int32_t r, int32_t width, int32_t d) { return mlp_param_count(r, width, d); }

size_t nsf_mlp_saved_floats(int32_t width, int64_t n) { return (size_t)5 * width * n; }

size_t nsf_mlp_workspace_bytes(const nsf_mlp* m, int64_t n) {
  if (check_mlp(m, n) != NSF_OK) return 0;
  return carve(nullptr, m->r, m->width, m->d, n, true).bytes;
}

nsf_status nsf_mlp_forward(const nsf_mlp* m, const float* X, const float* z_rows, int64_t n,
                           float* out, float* saved, void* workspace, size_t workspace_bytes,
                           void* stream) {
  return mlp_forward(m, X, z_rows, n, out, saved, static_cast<char*>(workspace), workspace_bytes,
                     static_cast<hipStream_t>(stream));
}

nsf_status nsf_mlp_forward_noalloc(const nsf_mlp* m, const float* X, const float* z_rows, int64_t n,
                                   float* out, float* saved, void* stream) {
  if (check_mlp(m, n) != NSF_OK || !X || !z_rows || !out) return NSF_EINVAL;
  const size_t need = carve(nullptr, m->r, m->width, m->d, n, false).bytes;
  if (need > kScratchBytes) return NSF_ENOMEM;
  char* base = nullptr;
  const nsf_status e = scratch_address(&base);
  if (e != NSF_OK) return e;
  return mlp_forward(m, X, z_rows, n, out, saved, base, kScratchBytes, static_cast<hipStream_t>(stream));
}

nsf_status nsf_adam_step(float* w, const float* grad, float* m, float* v, int64_t n, double lr, double beta1,
                         double beta2, double eps, int64_t step, void* stream) {
  if (!w || !grad || !m || !v || n < 1 || step < 1 || !(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return NSF_EINVAL;
  const double bc1 = 1.0 - std::pow(beta1, (double)step), bc2 = 1.0 - std::pow(beta2, (double)step);
  const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(adam_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), w, grad, m, v, n,
                     (float)beta1, (float)beta2, (float)eps, (float)(lr / bc1), (float)(1.0 / std::sqrt(bc2)));
  return hipGetLastError() == hipSuccess ? NSF_OK : NSF_EHIP;
}

nsf_status nsf_rows_expand(const float* table, const int64_t* offsets, int32_t segments, int32_t width,
                           float* out, void* stream) {
  if (!table || !offsets || !out || segments < 0 || width < 1 || width > 256) return NSF_EINVAL;
  if (segments == 0) return NSF_OK;
  hipLaunchKernelGGL(rows_expand_kernel, dim3(segments), dim3(256), 0, static_cast<hipStream_t>(stream), table,
                     offsets, width, out);
  return hipGetLastError() == hipSuccess ? NSF_OK : NSF_EHIP;
}

nsf_status nsf_rows_segment_sum(const float* rows, const int64_t* offsets, int32_t segments, int32_t width,
                                float* out, void* stream) {
  if (!rows || !offsets || !out || segments < 0 || width < 1 || width > 256) return NSF_EINVAL;
  if (segments == 0) return NSF_OK;
  hipLaunchKernelGGL(rows_segment_sum_kernel, dim3(segments), dim3(256), 0, static_cast<hipStream_t>(stream), rows,
                     offsets, width, out);
  return hipGetLastError() == hipSuccess ? NSF_OK : NSF_EHIP;
}

nsf_status nsf_squared_error(const float* out, int32_t d, int64_t n, const float* Y, int64_t ldy,
                             const int64_t* rows, const int64_t* cols, int64_t P, float* loss, float* grad,
                             void* workspace, void* stream) {
  if (!out || !Y || !rows || !cols || !loss || !grad || !workspace || d < 1 || n < 1 || P < 1 || ldy < 1)
    return NSF_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int blocks = (int)std::min<int64_t>(kSqErrBlocks, (n + kSqErrThreads - 1) / kSqErrThreads);
  const double count = (double)d * (double)n;
  double* part = static_cast<double*>(workspace);
  hipLaunchKernelGGL(sq_err_kernel, dim3(blocks), dim3(kSqErrThreads), 0, s, out, (int)d, n, Y, ldy, rows, cols, P,
                     (float)(2.0 / count), grad, part);
  if (hipGetLastError() != hipSuccess) return NSF_EHIP;
  hipLaunchKernelGGL(sq_err_total_kernel, dim3(1), dim3(64), 0, s, part, blocks, 1.0 / count, loss);
  return hipGetLastError() == hipSuccess ? NSF_OK : NSF_EHIP;
}

nsf_status nsf_mlp_backward(const nsf_mlp* m, const float* X, const float* z_rows, int64_t n,
                            const float* saved, const float* dout, float* dW, float* dz, float* dX,
                            void* workspace, size_t workspace_bytes, void* stream) {
  if (check_mlp(m, n) != NSF_OK || !X || !z_rows || !saved || !dout || !dW || !workspace)
    return NSF_EINVAL;
  const int r = m->r, W = m->width, d = m->d;
  const TrainWs ws = carve(static_cast<char*>(workspace), r, W, d, n, true);
  if (workspace_bytes < ws.bytes) return NSF_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(pack_kernel, dim3(256), dim3(256), 0, s, m->weights, r, W, d, ws.pk);
  const bool bf = m->precision == NSF_BF16;
  if (bf) {
    BwdArgs a{};
    a.whbt = ws.pk.whbt; a.w1t = ws.pk.w1t; a.w6t = ws.pk.w6t;
    a.saved = reinterpret_cast<const __bf16*>(saved);
    a.dout = dout;
    a.delta = reinterpret_cast<__bf16*>(ws.delta);
    a.dz = dz; a.dX = dX;
    a.n = (int)n; a.r = r; a.d = d;
    if (launch_backward_bf16(W, a, s) != hipSuccess) return NSF_EHIP;
  } else {
    const int waves = (int)((n + 31) / 32);
    const int grid = (waves + 3) / 4;
    if (W == 64)
      hipLaunchKernelGGL(backward_data_kernel<64>, dim3(grid), dim3(256), 0, s, m->weights, ws.pk.whtp,
                         ws.pk.w6p, saved, dout, ws.delta, dz, dX, (int)n, r, d);
    else
      hipLaunchKernelGGL(backward_data_kernel<128>, dim3(grid), dim3(256), 0, s, m->weights, ws.pk.whtp,
                         ws.pk.w6p, saved, dout, ws.delta, dz, dX, (int)n, r, d);
  }
  if (hipGetLastError() != hipSuccess) return NSF_EHIP;
  // parameter offsets in the master layout
  const size_t in1 = 3 + r;
  float* gW1 = dW;
  float* gb1 = gW1 + (size_t)W * in1;
  float* gh = gb1 + W;
  float* gW6 = gh + 4 * ((size_t)W * W + W);
  float* gb6 = gW6 + (size_t)d * W;
  const int chunks = (int)((n + (bf ? kChunk16 : kChunk) - 1) / (bf ? kChunk16 : kChunk));
  for (int layer = 1; layer <= 6; ++layer) {
    GradIn g{};
    g.partial = ws.partial;
    g.r = r;
    float *tW, *tb;
    int kind;
    if (layer == 6) {
      kind = kGradOutput;
      g.A = dout; g.M = d;
      g.Bsaved = saved + (size_t)4 * n * W; g.N = W;
      tW = gW6; tb = gb6;
    } else {
      g.A = ws.delta + (size_t)(layer - 1) * n * W; g.M = W;
      if (layer == 1) {
        kind = kGradFirst;
        g.X = X; g.zrows = z_rows; g.N = (int)in1;
        tW = gW1; tb = gb1;
      } else {
        kind = kGradHidden;
        g.Bsaved = saved + (size_t)(layer - 2) * n * W; g.N = W;
        tW = gh + (size_t)(layer - 2) * ((size_t)W * W + W);
        tb = tW + (size_t)W * W;
      }
    }
    if (bf) {
      // the same operands in BF16: the deltas of the BF16 backward and the saved values
      GradIn16 g16{};
      g16.A = reinterpret_cast<const __bf16*>(g.A);
      g16.dout = layer == 6 ? dout : nullptr;
      g16.Bsaved = reinterpret_cast<const __bf16*>(saved) + (g.Bsaved ? g.Bsaved - saved : 0);
      g16.X = g.X; g16.zrows = g.zrows;
      g16.M = g.M; g16.N = g.N; g16.r = g.r; g16.partial = g.partial;
      if (layer < 6) g16.A = reinterpret_cast<const __bf16*>(ws.delta) + (size_t)(layer - 1) * n * W;
      if (W == 64) launch_grad16<64>(g16, kind, chunks, (int)n, s);
      else launch_grad16<128>(g16, kind, chunks, (int)n, s);
    } else {
      if (W == 64) launch_grad<64, false>(g, kind, chunks, (int)n, s);
      else launch_grad<128, false>(g, kind, chunks, (int)n, s);
    }
    const int e = g.M * (g.N + 1);
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((e + 63) / 64), dim3(64 * kRedWaves), 0, s, ws.partial, chunks,
                       g.M, g.N + 1, tW, tb);
    if (hipGetLastError() != hipSuccess) return NSF_EHIP;
  }
  return NSF_OK;
}

}  // extern "C"
