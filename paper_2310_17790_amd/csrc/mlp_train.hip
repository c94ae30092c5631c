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
// output, pre-activations stored point-major). The backward-data kernel carries 32 points
// per wave through the five W^T products on MFMA (the same accumulator-layout chaining as
// the forward, with the transposed weights packed on the device) and computes dz and dX
// on the VALU. The weight gradients are reductions over points on MFMA: each workgroup sums a
// chunk of points for one layer into a partial, and the partials are added in chunk order
// (deterministic) into dW.
#include <hip/hip_runtime.h>

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
  float* w6p; float* whtp;                                                     // backward
};

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
  const int64_t total = n1q + 3 * nh + nb + 2 * n6 + d;
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
    P.b6[t] = b6[t];
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

constexpr int kChunk = 1024;   // points per weight-gradient workgroup

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

template <int W, bool BF>
void launch_grad(const GradIn& g, int kind, int chunks, int n, hipStream_t s) {
  if (kind == kGradFirst) hipLaunchKernelGGL((grad_mfma_kernel<W, BF, kGradFirst>), dim3(chunks), dim3(256), 0, s, g, n);
  else if (kind == kGradHidden) hipLaunchKernelGGL((grad_mfma_kernel<W, BF, kGradHidden>), dim3(chunks), dim3(256), 0, s, g, n);
  else hipLaunchKernelGGL((grad_mfma_kernel<W, BF, kGradOutput>), dim3(chunks), dim3(256), 0, s, g, n);
}

// dW[m][j] += sum over chunks (in order); column N-1 goes to the bias db[m].
__global__ void grad_reduce_kernel(const float* __restrict__ partial, int n_chunks, int M, int N,
                                   float* __restrict__ dW, float* __restrict__ db) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  // eight running sums (chunk c goes to sum c mod 8) keep eight loads in flight; they are
  // combined in a fixed order, so the result does not depend on timing
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int64_t stride = (int64_t)M * N;
  int c = 0;
  for (; c + 8 <= n_chunks; c += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(c + u) * stride + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  for (; c < n_chunks; ++c) a[c & 7] += partial[(int64_t)c * stride + e];
  const float s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  const int m = e / N, j = e % N;
  if (j == N - 1) db[m] += s;
  else dW[(int64_t)m * (N - 1) + j] += s;
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
  if (backward) {
    w.delta = (float*)take((size_t)5 * n * W * 4);
    const int64_t chunks = (n + kChunk - 1) / kChunk;
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
  const int waves = (int)((n + 31) / 32);
  const int grid = (waves + 3) / 4;
  if (W == 64)
    hipLaunchKernelGGL(backward_data_kernel<64>, dim3(grid), dim3(256), 0, s, m->weights, ws.pk.whtp,
                       ws.pk.w6p, saved, dout, ws.delta, dz, dX, (int)n, r, d);
  else
    hipLaunchKernelGGL(backward_data_kernel<128>, dim3(grid), dim3(256), 0, s, m->weights, ws.pk.whtp,
                       ws.pk.w6p, saved, dout, ws.delta, dz, dX, (int)n, r, d);
  if (hipGetLastError() != hipSuccess) return NSF_EHIP;
  // parameter offsets in the master layout
  const size_t in1 = 3 + r;
  float* gW1 = dW;
  float* gb1 = gW1 + (size_t)W * in1;
  float* gh = gb1 + W;
  float* gW6 = gh + 4 * ((size_t)W * W + W);
  float* gb6 = gW6 + (size_t)d * W;
  const int chunks = (int)((n + kChunk - 1) / kChunk);
  const bool bf = m->precision == NSF_BF16;
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
    if (W == 64) bf ? launch_grad<64, true>(g, kind, chunks, (int)n, s) : launch_grad<64, false>(g, kind, chunks, (int)n, s);
    else bf ? launch_grad<128, true>(g, kind, chunks, (int)n, s) : launch_grad<128, false>(g, kind, chunks, (int)n, s);
    const int e = g.M * (g.N + 1);
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((e + 255) / 256), dim3(256), 0, s, ws.partial, chunks,
                       g.M, g.N + 1, tW, tb);
    if (hipGetLastError() != hipSuccess) return NSF_EHIP;
  }
  return NSF_OK;
}

}  // extern "C"
