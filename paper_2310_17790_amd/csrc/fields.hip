// Neural field evaluation on MFMA: primal MLP and forward-mode latent Jacobian.
//
// The three fields g, h, l of the paper (Sec. 4.2-4.4) are MLPs with input [X; z]
// (3 + r), five hidden ELU layers of width W and a linear output of d = 3, 6 or 9
// (supplementary "Network architecture"). The inversion (Sec. 5.3) needs du/dz at the
// sample points; it is pushed forward with the primal: the tangent of layer 1 is
// phi'(a1) * W1[:, 3 + j], each hidden layer maps T -> phi'(a_k) * (W_k T), and the output
// is W6 T.
//
// Mapping to the hardware. One wave owns 32 points (the MFMA N dimension) and carries
// them through all six layers in registers. A layer is Y = W H with W the A operand
// (M = output neurons, 32 per block) and H the B operand. The 32x32 accumulator layout
// gives each lane one point (column) and 16 neurons per M-block; instead of re-laying
// the activations out between layers, the host permutes the columns of every weight
// matrix so that K-step s of the next layer consumes exactly the registers each lane
// already holds (see acc_neuron and pack.cpp). Tangent columns of the same 32 points
// ride in extra N-tiles of the same wave, so phi'(a) of the primal is available
// in-lane. A wave processes the primal plus up to TC tangents; a Jacobian with more
// tangents is split over several waves, each recomputing the primal.
//
// Layer 1 also runs on FP32 MFMA, with the bias folded in as an input row equal to 1
// and the tangent seeds as one-hot input columns. FP32 precision: hidden layers on
// v_mfma_f32_32x32x2_f32. BF16 precision: hidden layers on v_mfma_f32_32x32x16_bf16
// with FP32 accumulation; layer 1 and the output layer stay FP32. The output layer
// (d <= 9 rows) is a per-lane dot product plus one cross-half lane exchange.
#include "nsf_dev.h"

namespace nsf {
namespace {

__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// ELU (alpha = 1) and its derivative from one exponential.
__device__ __forceinline__ void elu_pair(float a, float& y, float& dy) {
  const float e = __expf(fminf(a, 0.f));
  y = a > 0.f ? a : e - 1.f;
  dy = a > 0.f ? 1.f : e;
}

template <int W, int T>
__device__ __forceinline__ void activate_f32(const f32x16 (&acc)[T][W / 32], float (&H)[T][W / 2],
                                             int nt) {
#pragma unroll
  for (int mb = 0; mb < W / 32; ++mb)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float y, dy;
      elu_pair(acc[0][mb][i], y, dy);
      H[0][16 * mb + i] = y;
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) H[t][16 * mb + i] = dy * acc[t][mb][i];
    }
}

// K-step s = 2 mb + q of a BF16 layer reads registers 8q .. 8q + 7 of M-block mb.
template <int W, int T>
__device__ __forceinline__ void activate_bf16(const f32x16 (&acc)[T][W / 32],
                                              bf16x8 (&Hb)[T][W / 16], int nt) {
#pragma unroll
  for (int mb = 0; mb < W / 32; ++mb)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bf16x8 p0;
      float dys[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float y;
        elu_pair(acc[0][mb][8 * q + j], y, dys[j]);
        p0[j] = (__bf16)y;
      }
      Hb[0][2 * mb + q] = p0;
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) {
          bf16x8 pt;
#pragma unroll
          for (int j = 0; j < 8; ++j) pt[j] = (__bf16)(dys[j] * acc[t][mb][8 * q + j]);
          Hb[t][2 * mb + q] = pt;
        }
    }
}

// Accumulators of a hidden layer start from the bias (primal) or zero (tangents).
template <int W, int T>
__device__ __forceinline__ void init_hidden(f32x16 (&acc)[T][W / 32], const float* bhp_layer,
                                            int h) {
  const f32x4* bias = reinterpret_cast<const f32x4*>(bhp_layer + h * (W / 2));
#pragma unroll
  for (int mb = 0; mb < W / 32; ++mb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 b4 = bias[mb * 4 + q];
      acc[0][mb][4 * q + 0] = b4[0];
      acc[0][mb][4 * q + 1] = b4[1];
      acc[0][mb][4 * q + 2] = b4[2];
      acc[0][mb][4 * q + 3] = b4[3];
    }
#pragma unroll
    for (int t = 1; t < T; ++t) acc[t][mb] = f32x16{};
  }
}

template <int W, int T>
__device__ __forceinline__ void hidden_f32(f32x16 (&acc)[T][W / 32], const float (&H)[T][W / 2],
                                           const float* whp_layer, int lane, int nt) {
  constexpr int MB = W / 32;
  const f32x4* A = reinterpret_cast<const f32x4*>(whp_layer);
#pragma unroll
  for (int sg = 0; sg < W / 8; ++sg) {
    f32x4 a4[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) a4[mb] = A[(mb * (W / 8) + sg) * 64 + lane];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        acc[0][mb] = mfma_f32(a4[mb][j], H[0][4 * sg + j], acc[0][mb]);
#pragma unroll
        for (int t = 1; t < T; ++t)
          if (t <= nt) acc[t][mb] = mfma_f32(a4[mb][j], H[t][4 * sg + j], acc[t][mb]);
      }
  }
}

template <int W, int T>
__device__ __forceinline__ void hidden_bf16(f32x16 (&acc)[T][W / 32],
                                            const bf16x8 (&Hb)[T][W / 16],
                                            const bf16x8* whb_layer, int lane, int nt) {
  constexpr int MB = W / 32;
#pragma unroll
  for (int s = 0; s < W / 16; ++s) {
    bf16x8 a[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) a[mb] = whb_layer[(mb * (W / 16) + s) * 64 + lane];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      acc[0][mb] = mfma_bf16(a[mb], Hb[0][s], acc[0][mb]);
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) acc[t][mb] = mfma_bf16(a[mb], Hb[t][s], acc[t][mb]);
    }
  }
}

// out_o = sum_n W6[o][n] H[n] over this lane's half of the neurons, then both halves.
template <int W>
__device__ __forceinline__ float output_dot(const float* w6p, int o, int h, const float (&Hrow)[W / 2]) {
  const f32x4* w6 = reinterpret_cast<const f32x4*>(w6p + (o * 2 + h) * (W / 2));
  float s = 0.f;
#pragma unroll
  for (int sg = 0; sg < W / 8; ++sg) {
    const f32x4 w = w6[sg];
    s += w[0] * Hrow[4 * sg + 0];
    s += w[1] * Hrow[4 * sg + 1];
    s += w[2] * Hrow[4 * sg + 2];
    s += w[3] * Hrow[4 * sg + 3];
  }
  return s + __shfl_xor(s, 32);
}

template <int W, int TC, bool BF>
__device__ __forceinline__ void run_tile(const FieldJob& jb, int p0, int t0, int nt, int lane) {
  constexpr int MB = W / 32;
  constexpr int T = 1 + TC;
  constexpr int KH = W / 2;
  const int h = lane >> 5;
  const int p = p0 + (lane & 31);
  const bool valid = p < jb.n;
  int gi = jb.p_off + (valid ? p : jb.n - 1);
  if (jb.idx != nullptr) {
    const int32_t* row = jb.idx;
    if (jb.step != nullptr) row += (*jb.step % jb.plan_steps) * (int64_t)jb.plan_ld;
    gi = row[gi];
  }
  const float X0 = jb.X[gi];
  const float X1 = jb.X[jb.ldx + gi];
  const float X2 = jb.X[2 * jb.ldx + gi];
  const int r = jb.r;

  f32x16 acc[T][MB];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[t][mb] = f32x16{};

  // Layer 1: input rows 0..2 = X, 3..2+r = z, 3+r = 1 (bias column of the packed W1).
  const int K1s = (r + 5) >> 1;
  for (int s2 = 0; s2 < K1s; ++s2) {
    const int k = 2 * s2 + h;
    float b0 = 0.f;
    if (k == 0) b0 = X0;
    else if (k == 1) b0 = X1;
    else if (k == 2) b0 = X2;
    else if (k < 3 + r) b0 = (float)jb.z[k - 3];
    else if (k == 3 + r) b0 = 1.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const float a = jb.w.w1p[(mb * K1s + s2) * 64 + lane];
      acc[0][mb] = mfma_f32(a, b0, acc[0][mb]);
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) acc[t][mb] = mfma_f32(a, (k == 3 + t0 + t - 1) ? 1.f : 0.f, acc[t][mb]);
    }
  }

  float H[T][KH];
  if constexpr (!BF) {
    activate_f32<W, T>(acc, H, nt);
    for (int k = 0; k < 4; ++k) {
      init_hidden<W, T>(acc, jb.w.bhp + k * W, h);
      hidden_f32<W, T>(acc, H, jb.w.whp + (size_t)k * W * W, lane, nt);
      activate_f32<W, T>(acc, H, nt);
    }
  } else {
    bf16x8 Hb[T][W / 16];
    activate_bf16<W, T>(acc, Hb, nt);
    for (int k = 0; k < 3; ++k) {
      init_hidden<W, T>(acc, jb.w.bhp + k * W, h);
      hidden_bf16<W, T>(acc, Hb, jb.w.whb + (size_t)k * MB * (W / 16) * 64, lane, nt);
      activate_bf16<W, T>(acc, Hb, nt);
    }
    init_hidden<W, T>(acc, jb.w.bhp + 3 * W, h);
    hidden_bf16<W, T>(acc, Hb, jb.w.whb + (size_t)3 * MB * (W / 16) * 64, lane, nt);
    activate_f32<W, T>(acc, H, nt);
  }

  // Output layer, primal.
  const int d = jb.d;
  if (t0 == 0) {
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      if (o < d) {
        const float y = output_dot<W>(jb.w.w6p, o, h, H[0]) + jb.w.b6[o];
        float v = jb.scale[o] * y + jb.shift[o];
        if (jb.mode == 1) v += (o == 0) ? X0 : (o == 1) ? X1 : X2;
        if (valid && h == (o & 1)) jb.out[o * jb.ldo + p] = v;
      }
    }
  }
  // Output layer, tangents (deformation field only: d = 3).
#pragma unroll
  for (int t = 1; t < T; ++t) {
    if (t <= nt) {
      const int j = t0 + t - 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float y = output_dot<W>(jb.w.w6p, c, h, H[t]);
        if (valid && h == (c & 1)) jb.jac[(c * r + j) * jb.ldj + p] = jb.scale[c] * y;
      }
    }
  }
}

template <int W, int TC, bool BF>
__global__ __launch_bounds__(256) void fields_table_kernel(const FieldJob* __restrict__ jobs,
                                                           const FieldTile* __restrict__ tiles,
                                                           const int32_t* __restrict__ n_tiles) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nw = (gridDim.x * blockDim.x) >> 6;
  const int total = *n_tiles;
  for (int t = wave; t < total; t += nw) {
    const FieldTile tl = tiles[t];
    run_tile<W, TC, BF>(jobs[tl.job], tl.p0, tl.t0, tl.nt, lane);
  }
}

template <int W, bool BF>
__global__ __launch_bounds__(256) void fields_dense_kernel(FieldJob job, int n_tiles) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int t = wave; t < n_tiles; t += nw) run_tile<W, 0, BF>(job, t * kTile, 0, 0, lane);
}

// Tangents one wave carries next to the primal, by register budget (512 per lane).
constexpr int kTcF32W64 = 3, kTcF32W128 = 2, kTcBf16W64 = 4, kTcBf16W128 = 2;

}  // namespace

int fields_max_tangents(int width, bool bf16) {
  if (width == 64) return bf16 ? kTcBf16W64 : kTcF32W64;
  return bf16 ? kTcBf16W128 : kTcF32W128;
}

hipError_t launch_fields_table(int width, bool bf16, int tc, const FieldJob* jobs,
                               const FieldTile* tiles, const int32_t* n_tiles, int grid,
                               hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  dim3 g(grid), b(256);
  const bool full = tc > 0;
#define NSF_LAUNCH(WW, TT, BB) \
  hipLaunchKernelGGL((fields_table_kernel<WW, TT, BB>), g, b, 0, s, jobs, tiles, n_tiles)
  if (width == 64) {
    if (!bf16) { if (full) NSF_LAUNCH(64, kTcF32W64, false); else NSF_LAUNCH(64, 0, false); }
    else { if (full) NSF_LAUNCH(64, kTcBf16W64, true); else NSF_LAUNCH(64, 0, true); }
  } else if (width == 128) {
    if (!bf16) { if (full) NSF_LAUNCH(128, kTcF32W128, false); else NSF_LAUNCH(128, 0, false); }
    else { if (full) NSF_LAUNCH(128, kTcBf16W128, true); else NSF_LAUNCH(128, 0, true); }
  } else {
    return hipErrorInvalidValue;
  }
#undef NSF_LAUNCH
  return hipGetLastError();
}

hipError_t launch_fields_dense(int width, bool bf16, const FieldJob& job, int n_tiles,
                               hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const int grid = (n_tiles + 3) / 4;
  dim3 g(grid), b(256);
  if (width == 64) {
    if (bf16) hipLaunchKernelGGL((fields_dense_kernel<64, true>), g, b, 0, s, job, n_tiles);
    else hipLaunchKernelGGL((fields_dense_kernel<64, false>), g, b, 0, s, job, n_tiles);
  } else if (width == 128) {
    if (bf16) hipLaunchKernelGGL((fields_dense_kernel<128, true>), g, b, 0, s, job, n_tiles);
    else hipLaunchKernelGGL((fields_dense_kernel<128, false>), g, b, 0, s, job, n_tiles);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nsf
