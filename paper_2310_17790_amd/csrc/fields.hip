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
// Pre-activations are carried scaled by log2(e) (see elu_pair and pack.cpp).
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

// ELU (alpha = 1) on scaled pre-activations. The kernels carry a' = log2(e) a and
// h' = ELU(a) / ln 2 (pack.cpp folds the scales into the weights), so one exp2 of a'
// itself gives e = exp(a), with no multiply (for large a' it may overflow to +inf, which
// the selects discard):
//   exact: h' = a' > 0 ? a' : (e - 1) / ln 2,  dh'/da' = a' > 0 ? 1 : e.
//   fast (values about to be rounded to BF16): since (e - 1) / ln 2 >= a' everywhere and
//     <= 0 for a' <= 0, h' is the median of ((e - 1) / ln 2, a', 0), and dh'/da' =
//     min(e, 1): one op fewer. For 0 < a' < ~3e-4 the FP32 rounding of e can put
//     (e - 1) / ln 2 below a', and the median then returns it, off by at most 1.7e-7 -
//     far below BF16 resolution, so only the BF16 hidden layers use it.
constexpr float kInvLn2 = 1.44269504088896340736f;
template <bool FAST>
__device__ __forceinline__ void elu_pair(float a, float& y, float& dy) {
  const float e = __builtin_amdgcn_exp2f(a);
  const float em1 = fmaf(e, kInvLn2, -kInvLn2);
  if constexpr (FAST) {
    y = __builtin_amdgcn_fmed3f(em1, a, 0.f);
    dy = fminf(e, 1.f);
  } else {
    y = a > 0.f ? a : em1;
    dy = a > 0.f ? 1.f : e;
  }
}

template <int W, int T>
__device__ __forceinline__ void activate_f32(const f32x16 (&acc)[T][W / 32], float (&H)[T][W / 2],
                                             int nt) {
#pragma unroll
  for (int mb = 0; mb < W / 32; ++mb)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float y, dy;
      elu_pair<false>(acc[0][mb][i], y, dy);
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
        elu_pair<true>(acc[0][mb][8 * q + j], y, dys[j]);
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

template <int W, int T, class APtr>
__device__ __forceinline__ void hidden_bf16(f32x16 (&acc)[T][W / 32],
                                            const bf16x8 (&Hb)[T][W / 16],
                                            APtr whb_layer, int lane, int nt) {
  constexpr int MB = W / 32, S = W / 16;
  // A fragments come from LDS two K-steps ahead of their use (a ring of three steps), so
  // each matrix product does not wait on its own LDS read; scheduling barriers keep the
  // compiler from sinking the reads back next to their uses.
  constexpr int D = 2;
  bf16x8 a[D + 1][MB];
#pragma unroll
  for (int s = 0; s < D; ++s)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) a[s][mb] = whb_layer[(mb * S + s) * 64 + lane];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (s + D < S) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a[(s + D) % (D + 1)][mb] = whb_layer[(mb * S + s + D) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      acc[0][mb] = mfma_bf16(a[s % (D + 1)][mb], Hb[0][s], acc[0][mb]);
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) acc[t][mb] = mfma_bf16(a[s % (D + 1)][mb], Hb[t][s], acc[t][mb]);
    }
    __builtin_amdgcn_sched_barrier(0);
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

// Training: store the (scaled) pre-activations of one layer, point-major saved[layer][p][W]. The
// 16 registers of M-block mb hold neurons 32 mb + 8 q + 4 h + (0..3), q = 0..3.
template <int W, int T>
__device__ __forceinline__ void save_preact(const FieldJob& jb, const f32x16 (&acc)[T][W / 32],
                                            int layer, int p, bool valid, int h) {
  if (jb.saved == nullptr || !valid) return;
  float* row = jb.saved + ((int64_t)layer * jb.n + p) * W;
#pragma unroll
  for (int mb = 0; mb < W / 32; ++mb)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<f32x4*>(row + 32 * mb + 8 * q + 4 * h) =
          f32x4{acc[0][mb][4 * q], acc[0][mb][4 * q + 1], acc[0][mb][4 * q + 2], acc[0][mb][4 * q + 3]};
}

// ---- FP32 precision: 16-point tiles on v_mfma_f32_16x16x4_f32 ------------------------
// Lane l holds point l % 16 of the tile and lane group g = l / 16. The 16x16 accumulator
// gives lane (point, g) neurons 16 mb + 4 g + v (v = 0..3) of M-block mb, and K-step
// s = 4 mb + v of the next layer consumes exactly those registers: the host stores, for
// output row m and K-group sg, the inputs 16 sg + 4 g + 0..3 of row m as lane (m % 16 + 16 g)'s
// four floats. Biases and output weights are then read in plain neuron order. A tile
// holds a quarter of the registers of a 32-point tile, so twice as many waves fit on a
// SIMD (two with two tangents, four for the primal), which is what hides the activations
// of one wave behind the matrix products of another.
constexpr int kTile16 = 16;

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int W, int T>
__device__ __forceinline__ void activate16(const f32x4 (&acc)[T][W / 16], float (&H)[T][W / 4], int nt) {
#pragma unroll
  for (int mb = 0; mb < W / 16; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float y, dy;
      elu_pair<false>(acc[0][mb][v], y, dy);
      H[0][4 * mb + v] = y;
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) H[t][4 * mb + v] = dy * acc[t][mb][v];
    }
}

// Accumulators start from the layer's bias (plain order) or zero (tangents).
template <int W, int T>
__device__ __forceinline__ void init16(f32x4 (&acc)[T][W / 16], const float* bias, int g) {
#pragma unroll
  for (int mb = 0; mb < W / 16; ++mb) {
    acc[0][mb] = *reinterpret_cast<const f32x4*>(bias + 16 * mb + 4 * g);
#pragma unroll
    for (int t = 1; t < T; ++t) acc[t][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
}

// One hidden layer from LDS: A is [W/16 output blocks][W/16 K-groups][64 lanes] f32x4,
// read in halves (two K-steps) one half ahead of its use.
template <int W, int T>
__device__ __forceinline__ void hidden16(f32x4 (&acc)[T][W / 16], const float (&H)[T][W / 4],
                                         const f32x4* A, int lane, int nt) {
  constexpr int MB = W / 16, SG = W / 16, HS = 2 * SG;
  const f32x2* A2 = reinterpret_cast<const f32x2*>(A);
  auto at = [&](int mb, int hs) { return A2[2 * ((mb * SG + (hs >> 1)) * 64 + lane) + (hs & 1)]; };
  f32x2 a2[2][MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) a2[0][mb] = at(mb, 0);
#pragma unroll
  for (int hs = 0; hs < HS; ++hs) {
    if (hs + 1 < HS) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a2[(hs + 1) & 1][mb] = at(mb, hs + 1);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        acc[0][mb] = mfma16(a2[hs & 1][mb][j], H[0][2 * hs + j], acc[0][mb]);
#pragma unroll
        for (int t = 1; t < T; ++t)
          if (t <= nt) acc[t][mb] = mfma16(a2[hs & 1][mb][j], H[t][2 * hs + j], acc[t][mb]);
      }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// out_o = sum_n W6[o][n] H[n] over the lane group's neurons, then over the four groups
// (every lane ends with the same sum: the pairwise additions commute).
template <int W>
__device__ __forceinline__ float output_dot16(const float* w6q, int o, int g, const float (&Hrow)[W / 4]) {
  const float* w = w6q + o * W + 4 * g;
  float s = 0.f;
#pragma unroll
  for (int mb = 0; mb < W / 16; ++mb) {
    const f32x4 w4 = *reinterpret_cast<const f32x4*>(w + 16 * mb);
    s += w4[0] * Hrow[4 * mb + 0];
    s += w4[1] * Hrow[4 * mb + 1];
    s += w4[2] * Hrow[4 * mb + 2];
    s += w4[3] * Hrow[4 * mb + 3];
  }
  s += __shfl_xor(s, 16);
  return s + __shfl_xor(s, 32);
}

template <int W, int T>
__device__ __forceinline__ void save_preact16(const FieldJob& jb, const f32x4 (&acc)[T][W / 16],
                                              int layer, int p, bool valid, int g) {
  if (jb.saved == nullptr || !valid) return;
  float* row = jb.saved + ((int64_t)layer * jb.n + p) * W;
#pragma unroll
  for (int mb = 0; mb < W / 16; ++mb) *reinterpret_cast<f32x4*>(row + 16 * mb + 4 * g) = acc[0][mb];
}

// Bytes of one packed hidden layer and of one LDS DMA instruction per wave (64 lanes x 16 B).
template <int W, bool BF>
struct HiddenLayer {
  static constexpr int kBytes = BF ? W * W * 2 : W * W * 4;
  static constexpr int kChunks = kBytes / 1024;
};

typedef __attribute__((address_space(3))) void lds_void;

// Copy hidden layer k of `w` into LDS buffer dst with direct global->LDS loads; the 1 KB
// chunks are dealt to the waves of the workgroup round-robin.
template <int W, bool BF, int WPG>
__device__ __forceinline__ void dma_layer(const FieldPack& w, int k, char* dst, int wave, int lane) {
  const char* src = (BF ? reinterpret_cast<const char*>(w.whb) : reinterpret_cast<const char*>(w.whp)) +
                    (size_t)k * HiddenLayer<W, BF>::kBytes;
#pragma unroll
  for (int chunk = wave; chunk < HiddenLayer<W, BF>::kChunks; chunk += WPG)
    __builtin_amdgcn_global_load_lds(src + chunk * 1024 + lane * 16,
                                      (lds_void*)(dst + chunk * 1024), 16, 0, 0);
}

// Copy all four hidden layers of `w` (contiguous in the pack) into LDS; chunks are dealt
// to the waves round-robin.
template <int W, bool BF, int WPG>
__device__ __forceinline__ void dma_all_layers(const FieldPack& w, char* dst, int wave, int lane) {
  constexpr int kTotal = 4 * HiddenLayer<W, BF>::kChunks;
  const char* src = BF ? reinterpret_cast<const char*>(w.whb) : reinterpret_cast<const char*>(w.whp);
  for (int chunk = wave; chunk < kTotal; chunk += WPG)
    __builtin_amdgcn_global_load_lds(src + chunk * 1024 + lane * 16, (lds_void*)(dst + chunk * 1024), 16, 0, 0);
}

__device__ __forceinline__ void wait_dma_and_sync() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// One wave evaluates a tile of 32 points of a job, starting at point p0: the primal plus
// tangents [t0, t0 + nt). Two ways to hold the hidden-layer weights:
//  - streamed (RES = false): the WPG waves of a workgroup run tiles of the same job in
//    step; layers stream through two LDS buffers, layer k + 1 (or the next group's first
//    hidden layer) fetched while layer k computes, with a workgroup barrier per layer;
//  - resident (RES = true): all four hidden layers sit in LDS for the whole kernel, and
//    waves run their tiles independently, without barriers, so one wave's activations
//    overlap another's matrix products on the same SIMD.
// Returns after the output layer.
template <int W, int NT, bool BF, int WPG, bool RES = false, class NextFn>
__device__ __forceinline__ void run_group(const FieldJob& jb, int p0, int t0, NextFn&& next,
                                          char* lds, int wave, int lane) {
  static_assert(BF, "FP32 tiles run in run_group16");
  constexpr int MB = W / 32;
  constexpr int T = 1 + NT;
  constexpr int nt = NT;  // compile-time: no per-MFMA guards
  constexpr int KH = W / 2;
  constexpr int LB = HiddenLayer<W, BF>::kBytes;
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
  // Tangent columns are one-hot in z (Jacobian) or the direction z - z2 (JVP job).
  const int K1s = (r + 5) >> 1;
  const bool jvp = jb.jvp != 0;
  for (int s2 = 0; s2 < K1s; ++s2) {
    const int k = 2 * s2 + h;
    float b0 = 0.f, bt = 0.f;
    if (k == 0) b0 = X0;
    else if (k == 1) b0 = X1;
    else if (k == 2) b0 = X2;
    else if (k < 3 + r && jb.zrows != nullptr) {
      b0 = jb.zrows[(int64_t)(valid ? p : jb.n - 1) * r + (k - 3)];
    } else if (k < 3 + r) {
      const double zk = jb.z[k - 3];
      if (jvp) {
        const double z2k = jb.z2[k - 3];
        b0 = (float)(0.5 * (zk + z2k));
        bt = (float)(zk - z2k);
      } else {
        b0 = (float)zk;
      }
    } else if (k == 3 + r) b0 = 1.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const float a = jb.w.w1p[(mb * K1s + s2) * 64 + lane];
      acc[0][mb] = mfma_f32(a, b0, acc[0][mb]);
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) acc[t][mb] = mfma_f32(a, jvp ? bt : ((k == 3 + t0 + t - 1) ? 1.f : 0.f), acc[t][mb]);
    }
  }

  if constexpr (NT == 0) save_preact<W, T>(jb, acc, 0, p, valid, h);
  float H[T][KH];
  bf16x8 Hb[T][W / 16];
  activate_bf16<W, T>(acc, Hb, nt);
  // Hidden layers 2..5 (k = 0..3): wait for layer k in LDS, start fetching layer k + 1
  // (after the last layer: the next group's first layer), multiply, activate.
#pragma unroll 1
  for (int k = 0; k < 3; ++k) {
    char* cur = lds + (RES ? k : (k & 1)) * LB;
    if constexpr (!RES) {
      wait_dma_and_sync();
      dma_layer<W, BF, WPG>(jb.w, k + 1, lds + ((k + 1) & 1) * LB, wave, lane);
    }
    init_hidden<W, T>(acc, jb.w.bhp + k * W, h);
    hidden_bf16<W, T>(acc, Hb, reinterpret_cast<const bf16x8*>(cur), lane, nt);
    if constexpr (NT == 0) save_preact<W, T>(jb, acc, k + 1, p, valid, h);
    activate_bf16<W, T>(acc, Hb, nt);
  }
  if constexpr (!RES) {
    wait_dma_and_sync();
    // decide the workgroup's next group now and start fetching its first hidden layer
    if (const FieldPack* next_w = next()) dma_layer<W, BF, WPG>(*next_w, 0, lds, wave, lane);
  }
  char* last = lds + (RES ? 3 : 1) * LB;
  init_hidden<W, T>(acc, jb.w.bhp + 3 * W, h);
  hidden_bf16<W, T>(acc, Hb, reinterpret_cast<const bf16x8*>(last), lane, nt);
  if constexpr (NT == 0) save_preact<W, T>(jb, acc, 4, p, valid, h);
  activate_f32<W, T>(acc, H, nt);

  const int d = jb.d;
  if constexpr (NT >= 1) {
    if (jvp) {  // directional derivative only: out = scale * (W6 T) * jvp_scale
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float y = output_dot<W>(jb.w.w6p, c, h, H[1]);
        if (valid && h == (c & 1)) jb.out[c * jb.ldo + p] = jb.scale[c] * y * jb.jvp_scale;
      }
      return;
    }
  }
  // Output layer, primal.
  if (t0 == 0) {
    // one output at a time: unrolled, the weight loads of all nine would be hoisted
#pragma unroll 1
    for (int o = 0; o < d; ++o) {
      {
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

// FP32 precision: one wave evaluates a 16-point tile (see kTile16) with streamed weights,
// in the same barrier sequence as run_group.
template <int W, int NT, int WPG, class NextFn>
__device__ __forceinline__ void run_group16(const FieldJob& jb, int p0, int t0, NextFn&& next,
                                            char* lds, int wave, int lane) {
  constexpr int MB = W / 16;
  constexpr int T = 1 + NT;
  constexpr int nt = NT;
  constexpr int LB = HiddenLayer<W, false>::kBytes;
  const int g = lane >> 4;
  const int p = p0 + (lane & 15);
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

  f32x4 acc[T][MB];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[t][mb] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Layer 1: input rows 0..2 = X, 3..2+r = z, 3+r = 1 (bias column), four per K-step.
  const int K1q = (r + 7) >> 2;
  const bool jvp = jb.jvp != 0;
  for (int s4 = 0; s4 < K1q; ++s4) {
    const int k = 4 * s4 + g;
    float b0 = 0.f, bt = 0.f;
    if (k == 0) b0 = X0;
    else if (k == 1) b0 = X1;
    else if (k == 2) b0 = X2;
    else if (k < 3 + r && jb.zrows != nullptr) {
      b0 = jb.zrows[(int64_t)(valid ? p : jb.n - 1) * r + (k - 3)];
    } else if (k < 3 + r) {
      const double zk = jb.z[k - 3];
      if (jvp) {
        const double z2k = jb.z2[k - 3];
        b0 = (float)(0.5 * (zk + z2k));
        bt = (float)(zk - z2k);
      } else {
        b0 = (float)zk;
      }
    } else if (k == 3 + r) b0 = 1.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const float a = jb.w.w1q[(mb * K1q + s4) * 64 + lane];
      acc[0][mb] = mfma16(a, b0, acc[0][mb]);
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) acc[t][mb] = mfma16(a, jvp ? bt : ((k == 3 + t0 + t - 1) ? 1.f : 0.f), acc[t][mb]);
    }
  }
  if constexpr (NT == 0) save_preact16<W, T>(jb, acc, 0, p, valid, g);
  float H[T][W / 4];
  activate16<W, T>(acc, H, nt);
  // Hidden layers 2..5 (k = 0..3), as in run_group.
#pragma unroll 1
  for (int k = 0; k < 4; ++k) {
    char* cur = lds + (k & 1) * LB;
    wait_dma_and_sync();
    if (k < 3) dma_layer<W, false, WPG>(jb.w, k + 1, lds + ((k + 1) & 1) * LB, wave, lane);
    else if (const FieldPack* next_w = next()) dma_layer<W, false, WPG>(*next_w, 0, lds, wave, lane);
    init16<W, T>(acc, jb.w.bhq + k * W, g);
    hidden16<W, T>(acc, H, reinterpret_cast<const f32x4*>(cur), lane, nt);
    if constexpr (NT == 0) save_preact16<W, T>(jb, acc, k + 1, p, valid, g);
    activate16<W, T>(acc, H, nt);
  }

  const int d = jb.d;
  if constexpr (NT >= 1) {
    if (jvp) {  // directional derivative only: out = scale * (W6 T) * jvp_scale
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float y = output_dot16<W>(jb.w.w6q, c, g, H[1]);
        if (valid && g == c) jb.out[c * jb.ldo + p] = jb.scale[c] * y * jb.jvp_scale;
      }
      return;
    }
  }
  if (t0 == 0) {
    // one output at a time: unrolled, the weight loads of all nine would be hoisted
#pragma unroll 1
    for (int o = 0; o < d; ++o) {
      {
        const float y = output_dot16<W>(jb.w.w6q, o, g, H[0]) + jb.w.b6[o];
        float v = jb.scale[o] * y + jb.shift[o];
        if (jb.mode == 1) v += (o == 0) ? X0 : (o == 1) ? X1 : X2;
        if (valid && g == (o & 3)) jb.out[o * jb.ldo + p] = v;
      }
    }
  }
#pragma unroll
  for (int t = 1; t < T; ++t) {
    if (t <= nt) {
      const int j = t0 + t - 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float y = output_dot16<W>(jb.w.w6q, c, g, H[t]);
        if (valid && g == c) jb.jac[(c * r + j) * jb.ldj + p] = jb.scale[c] * y;
      }
    }
  }
}

// Run a group with its tangent count as a template argument (0 .. TC).
template <int W, int TC, bool BF, int WPG, class NextFn>
__device__ __forceinline__ void dispatch_nt(const FieldJob& jb, int p0, int t0, int nt,
                                            NextFn&& next, char* lds, int wave, int lane) {
  if constexpr (TC > 0) {
    if (nt == TC) {
      if constexpr (BF) run_group<W, TC, true, WPG>(jb, p0 + kTile * wave, t0, next, lds, wave, lane);
      else run_group16<W, TC, WPG>(jb, p0 + kTile16 * wave, t0, next, lds, wave, lane);
      return;
    }
    dispatch_nt<W, TC - 1, BF, WPG>(jb, p0, t0, nt, next, lds, wave, lane);
  } else {
    if constexpr (BF) run_group<W, 0, true, WPG>(jb, p0 + kTile * wave, t0, next, lds, wave, lane);
    else run_group16<W, 0, WPG>(jb, p0 + kTile16 * wave, t0, next, lds, wave, lane);
  }
}

// Work groups from a table (several jobs; a group is WPG tiles of one job). Workgroups
// claim groups dynamically from a counter (zero at launch), one group ahead so the next
// group's first hidden layer can be fetched while the current group finishes; groups
// are ordered longest first, so the claims balance the load.
template <int W, int TC, bool BF, int WPG>
__global__ __launch_bounds__(64 * WPG) void fields_table_kernel(const FieldJob* __restrict__ jobs,
                                                                const FieldTile* __restrict__ groups,
                                                                const int32_t* __restrict__ n_groups,
                                                                int32_t* __restrict__ claim) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  __shared__ int s_claim;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int total = *n_groups;
  if (threadIdx.x == 0) s_claim = atomicAdd(claim, 1);
  __syncthreads();
  int g = s_claim;
  if (g >= total) return;
  dma_layer<W, BF, WPG>(jobs[groups[g].job].w, 0, lds, wave, lane);
  int gn = total;
  // called by every thread at the same point of run_group (after a barrier)
  auto next = [&]() -> const FieldPack* {
    if (threadIdx.x == 0) s_claim = atomicAdd(claim, 1);
    __syncthreads();
    gn = s_claim;
    return gn < total ? &jobs[groups[gn].job].w : nullptr;
  };
  while (true) {
    const FieldTile tl = groups[g];
    dispatch_nt<W, TC, BF, WPG>(jobs[tl.job], tl.p0, tl.t0, tl.nt, next, lds, wave, lane);
    if (gn >= total) break;
    g = gn;
  }
}

// The barrier and DMA sequence of run_group (streamed weights) for a wave with no tile in
// this round: it keeps the workgroup's per-layer barriers and weight copies in step.
template <int W, bool BF, int WPG, class NextFn>
__device__ __forceinline__ void idle_group(const FieldJob& jb, NextFn&& next, char* lds, int wave,
                                           int lane) {
  constexpr int LB = HiddenLayer<W, BF>::kBytes;
#pragma unroll 1
  for (int k = 0; k < 3; ++k) {
    wait_dma_and_sync();
    dma_layer<W, BF, WPG>(jb.w, k + 1, lds + ((k + 1) & 1) * LB, wave, lane);
  }
  wait_dma_and_sync();
  if (const FieldPack* next_w = next()) dma_layer<W, BF, WPG>(*next_w, 0, lds, wave, lane);
}

// One job over n points (FP32 decode), weights streamed, persistent workgroups, 16-point
// tiles. Tiles are dealt
// so that every round but the last fills all waves of all workgroups, and the last round's
// tiles go to wave 0 of distinct workgroups, which then run alone on their SIMDs:
// tile t = round * gridDim.x * WPG + wave * gridDim.x + blockIdx.x.
template <int W, int WPG>
__global__ __launch_bounds__(64 * WPG) void fields_dense_kernel(FieldJob job, int n_tiles) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int G = gridDim.x, b = blockIdx.x, per_round = G * WPG;
  if (b >= n_tiles) return;
  dma_layer<W, false, WPG>(job.w, 0, lds, wave, lane);
#pragma unroll 1
  for (int base = 0; base + b < n_tiles; base += per_round) {
    const bool more = base + per_round + b < n_tiles;
    auto next = [&]() -> const FieldPack* { return more ? &job.w : nullptr; };
    const int t = base + wave * G + b;
    if (t < n_tiles) run_group16<W, 0, WPG>(job, t * kTile16, 0, next, lds, wave, lane);
    else idle_group<W, false, WPG>(job, next, lds, wave, lane);
  }
}

// One job over n points (BF16 decode), weights resident: every workgroup loads the four
// hidden layers once, then each wave runs its tiles independently.
template <int W, bool BF, int WPG>
__global__ __launch_bounds__(64 * WPG) void fields_dense_res_kernel(FieldJob job, int n_tiles) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  dma_all_layers<W, BF, WPG>(job.w, lds, wave, lane);
  wait_dma_and_sync();
  auto none = []() -> const FieldPack* { return nullptr; };
  // tile t = round * gridDim.x * WPG + wave * gridDim.x + blockIdx.x: the last, partial
  // round's tiles go to distinct workgroups
#pragma unroll 1
  for (int t = wave * (int)gridDim.x + blockIdx.x; t < n_tiles; t += gridDim.x * WPG) {
    // keep the weight reads inside the tile: the LDS contents never change, and hoisting
    // them out of the loop would only exhaust registers
    __asm__ volatile("" ::: "memory");
    run_group<W, 0, BF, WPG, true>(job, t * kTile, 0, none, lds, wave, lane);
  }
}

// Tangents one wave carries next to the primal, by register budget (512 per lane).
constexpr int kTcF32W64 = 3, kTcF32W128 = 2, kTcBf16W64 = 4, kTcBf16W128 = 2;

// Waves per workgroup (one workgroup per CU: its two LDS layer buffers take 128 KB at
// width 128). BF16, 32-point tiles: with tangents ~500 registers (one wave per SIMD),
// primal only two waves per SIMD. FP32, 16-point tiles: two waves per SIMD with tangents,
// four for the primal. Either way a group spans the same points.
template <int TC, bool BF> struct Wpg {
  static constexpr int value = BF ? (TC > 0 ? 4 : 8) : (TC > 0 ? 8 : 16);
};
static_assert(kTile * Wpg<1, true>::value == kTile16 * Wpg<1, false>::value &&
                  kTile * Wpg<0, true>::value == kTile16 * Wpg<0, false>::value,
              "a group spans the same points in both precisions");

template <int W, int TC, bool BF>
hipError_t launch_table(const FieldJob* jobs, const FieldTile* groups, const int32_t* n_groups,
                        int32_t* claim, int grid, hipStream_t s) {
  constexpr int WPG = Wpg<TC, BF>::value;
  constexpr int lds = 2 * HiddenLayer<W, BF>::kBytes;
  auto k = fields_table_kernel<W, TC, BF, WPG>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WPG), lds, s, jobs, groups, n_groups, claim);
  return hipGetLastError();
}

// Streamed-weight decode: as many persistent workgroups as fit on the device at once.
// FP32 decode: eight waves per workgroup (two per SIMD) hold a 16-point tile each without
// spilling; sixteen spill and measured slower.
constexpr int kDenseWpg16 = 8;

template <int W>
hipError_t launch_dense(const FieldJob& job, int n_tiles, int cus, hipStream_t s) {
  constexpr int WPG = kDenseWpg16;
  constexpr int lds = 2 * HiddenLayer<W, false>::kBytes;
  auto k = fields_dense_kernel<W, WPG>;
  static int per_cu = 0;
  if (per_cu == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * WPG, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
  }
  int grid = cus * per_cu;
  if (grid > n_tiles) grid = n_tiles;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WPG), lds, s, job, n_tiles);
  return hipGetLastError();
}

// BF16 decode: twelve waves per workgroup (three per SIMD) measured fastest.
constexpr int kDenseResWpg = 12;

// Resident-weight decode: one workgroup per CU at width 128 (the four hidden layers take
// 4 W^2 x 2 B = 128 KB of LDS in BF16).
template <int W, bool BF>
hipError_t launch_dense_res(const FieldJob& job, int n_tiles, int cus, hipStream_t s) {
  constexpr int WPG = kDenseResWpg;
  constexpr int lds = 4 * HiddenLayer<W, BF>::kBytes;
  static_assert(lds <= 160 * 1024, "resident weights must fit in LDS");
  auto k = fields_dense_res_kernel<W, BF, WPG>;
  static int per_cu = 0;
  if (per_cu == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * WPG, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
  }
  int grid = cus * per_cu;
  const int need = (n_tiles + WPG - 1) / WPG;
  if (grid > need) grid = need;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WPG), lds, s, job, n_tiles);
  return hipGetLastError();
}

}  // namespace

int fields_max_tangents(int width, bool bf16) {
  if (width == 64) return bf16 ? kTcBf16W64 : kTcF32W64;
  return bf16 ? kTcBf16W128 : kTcF32W128;
}

int fields_group_points(int tc) { return kTile * (tc > 0 ? Wpg<1, true>::value : Wpg<0, true>::value); }

hipError_t launch_fields_table(int width, bool bf16, int tc, const FieldJob* jobs,
                               const FieldTile* groups, const int32_t* n_groups, int32_t* claim,
                               int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  const bool full = tc > 0;
#define NSF_TABLE(WW, TT, BB) launch_table<WW, TT, BB>(jobs, groups, n_groups, claim, grid, s)
  if (width == 64) {
    if (!bf16) return full ? NSF_TABLE(64, kTcF32W64, false) : NSF_TABLE(64, 0, false);
    return full ? NSF_TABLE(64, kTcBf16W64, true) : NSF_TABLE(64, 0, true);
  }
  if (width == 128) {
    if (!bf16) return full ? NSF_TABLE(128, kTcF32W128, false) : NSF_TABLE(128, 0, false);
    return full ? NSF_TABLE(128, kTcBf16W128, true) : NSF_TABLE(128, 0, true);
  }
#undef NSF_TABLE
  return hipErrorInvalidValue;
}

int fields_table_blocks_per_cu(int width, bool bf16, int tc) {
  // dynamic LDS (two hidden layers) bounds residency: 160 KB per CU
  const int lds = 2 * (bf16 ? width * width * 2 : width * width * 4);
  int by_lds = (160 * 1024) / (lds + 1024);
  if (by_lds < 1) by_lds = 1;
  // registers: the tangent kernels run one wave per SIMD, the primal ones two
  const int by_regs = tc > 0 ? 1 : 1;
  return by_lds < by_regs ? by_lds : by_regs;
}

__global__ void reset_counters_kernel(int32_t* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

hipError_t launch_reset_counters(int32_t* c, int n, hipStream_t s) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, c, n);
  return hipGetLastError();
}

hipError_t launch_fields_dense(int width, bool bf16, const FieldJob& job, int n_points,
                               hipStream_t s, int max_cus) {
  if (n_points <= 0) return hipSuccess;
  static int dev_cus = 0;
  if (dev_cus == 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  const int cus = max_cus > 0 && max_cus < dev_cus ? max_cus : dev_cus;
  if (bf16) {
    const int tiles = (n_points + kTile - 1) / kTile;
    if (width == 64) return launch_dense_res<64, true>(job, tiles, cus, s);
    if (width == 128) return launch_dense_res<128, true>(job, tiles, cus, s);
    return hipErrorInvalidValue;
  }
  const int tiles = (n_points + kTile16 - 1) / kTile16;
  if (width == 64) return launch_dense<64>(job, tiles, cus, s);
  if (width == 128) return launch_dense<128>(job, tiles, cus, s);
  return hipErrorInvalidValue;
}

}  // namespace nsf
