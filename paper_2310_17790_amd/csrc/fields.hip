// Neural field evaluation on MFMA: primal MLP and forward-mode latent Jacobian.
//
// The three fields g, h, l of the paper (Sec. 4.2-4.4) are MLPs with input [X; z]
// (3 + r), five hidden ELU layers of width W and a linear output of d = 3, 6 or 9
// (supplementary "Network architecture"). The inversion (Sec. 5.3) needs du/dz at the
// sample points; it is pushed forward with the primal: the tangent of layer 1 is
// phi'(a1) * W1[:, 3 + j], each hidden layer maps T -> phi'(a_k) * (W_k T), and the output
// is W6 T.
//
// Mapping to the hardware. One wave owns a tile of 16 points (the MFMA N dimension) and
// carries it through all six layers in registers. A layer is Y = W H with W the A operand
// (M = output neurons, 16 per block) and H the B operand. In the 16x16 accumulator lane l
// holds point l % 16 and, of M-block mb, the four neurons 16 mb + 4 g + v (v = 0..3) of its
// lane group g = l / 16. Instead of re-laying the activations out between layers, the host
// permutes the columns of every weight matrix so that the next layer's K-steps consume
// exactly the registers each lane already holds (pack.cpp):
//  - FP32 (v_mfma_f32_16x16x4_f32): K-step 4 mb + v takes register v of M-block mb, i.e.
//    lane group g supplies input 16 mb + 4 g + v;
//  - BF16 (v_mfma_f32_16x16x32_bf16): K-step s takes M-blocks 2s and 2s + 1, eight BF16
//    values per lane: lane group g supplies inputs 16 (2s + e / 4) + 4 g + e % 4, e = 0..7.
// Biases and output weights are then read in plain neuron order. Tangent columns of the
// same points ride in extra N-tiles of the same wave, so phi'(a) of the primal is
// available in-lane. A wave processes the primal plus up to TC tangents; a Jacobian with
// more tangents is split over several waves, each recomputing the primal. A 16-point tile
// needs a quarter of the registers of a 32-point one, so two waves fit per SIMD with two
// tangents and three or four for the primal: the activations of one wave then overlap
// the matrix products of another.
//
// Pre-activations are carried scaled by log2(e) (see elu_pair and pack.cpp). Layer 1 runs
// on FP32 MFMA in both precisions, with the bias folded in as an input row equal to 1 and
// the tangent seeds as one-hot input columns; so does the output layer's dot product. BF16
// precision rounds the hidden layers' weights and input activations to BF16 and
// accumulates in FP32.
#include "nsf_dev.h"

namespace nsf {
namespace {

constexpr int kTile16 = 16;   // points per wave tile

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma16_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ELU (alpha = 1) on scaled pre-activations. The kernels carry a' = log2(e) a and
// h' = ELU(a) / ln 2 (pack.cpp folds the scales into the weights), so one exp2 of a'
// itself gives e = exp(a), with no multiply (for large a' it may overflow to +inf, which
// the selects discard):
//   exact: h' = a' > 0 ? a' : (e - 1) / ln 2,  dh'/da' = a' > 0 ? 1 : e.
//   fast: since (e - 1) / ln 2 >= a' everywhere and <= 0 for a' <= 0, h' is the median of
//     ((e - 1) / ln 2, a', 0), and dh'/da' = min(e, 1) (the same values): one op fewer.
//     For 0 < a' < ~3e-4 the FP32 rounding of e can put (e - 1) / ln 2 below a', and the
//     median then returns it, off by at most 1.7e-7 absolute - below the FP32 rounding of
//     a width-128 layer's sum of products, so every layer uses it (the decode's ELU work
//     is a sixth of its SIMD cycles, and this took it from 0.759 to 0.768 of the peak).
//     A non-finite latent is still flagged: the solve checks the latent itself.
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

// FP32 activations: H[t][4 mb + v] from register v of M-block mb.
template <int W, int T>
__device__ __forceinline__ void activate16(const f32x4 (&acc)[T][W / 16], float (&H)[T][W / 4], int nt) {
#pragma unroll
  for (int mb = 0; mb < W / 16; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float y, dy;
      elu_pair<true>(acc[0][mb][v], y, dy);
      H[0][4 * mb + v] = y;
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) H[t][4 * mb + v] = dy * acc[t][mb][v];
    }
}

// BF16 activations: K-step s of the next layer packs M-blocks 2s and 2s + 1.
template <int W, int T>
__device__ __forceinline__ void activate16_bf16(const f32x4 (&acc)[T][W / 16], bf16x8 (&Hb)[T][W / 32],
                                                int nt) {
#pragma unroll
  for (int s = 0; s < W / 32; ++s) {
    bf16x8 p0;
    float dys[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float y;
      elu_pair<true>(acc[0][2 * s + (e >> 2)][e & 3], y, dys[e]);
      p0[e] = (__bf16)y;
    }
    Hb[0][s] = p0;
#pragma unroll
    for (int t = 1; t < T; ++t)
      if (t <= nt) {
        bf16x8 pt;
#pragma unroll
        for (int e = 0; e < 8; ++e) pt[e] = (__bf16)(dys[e] * acc[t][2 * s + (e >> 2)][e & 3]);
        Hb[t][s] = pt;
      }
  }
}

// Weight-pack pointers taken from a job table in memory are generic; read through the
// global address space, their loads are counted by the vector-memory counter alone, so a
// product waits for the loads it needs and not for the LDS copies issued after them.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Accumulators start from the layer's bias (plain order; none: zero) or zero (tangents).
// LDS: the bias is in LDS (a generic pointer into it would be read with flat loads too).
template <int W, int T, bool LDS = false>
__device__ __forceinline__ void init16(f32x4 (&acc)[T][W / 16], const float* bias, int g) {
#pragma unroll
  for (int mb = 0; mb < W / 16; ++mb) {
    if (!bias) acc[0][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    else if constexpr (LDS) acc[0][mb] = *reinterpret_cast<const f32x4*>(bias + 16 * mb + 4 * g);
    else acc[0][mb] = *global_ptr(reinterpret_cast<const f32x4*>(bias + 16 * mb + 4 * g));
#pragma unroll
    for (int t = 1; t < T; ++t) acc[t][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
}

// The A fragments of a hidden layer are consumed in a fixed sequence of steps (K-step
// outer, output block inner) and read from LDS kPrefetch steps ahead of their use into a
// small ring; scheduling barriers keep the compiler from sinking the reads back next to
// their uses or hoisting more of them (which only costs registers).
constexpr int kPrefetch = 4;
constexpr int kPrefetchBf16Primal = 8;

// One FP32 hidden layer from LDS: A is [W/16 output blocks][W/8 K-step pairs][64 lanes]
// f32x2 (K-steps 2 hs, 2 hs + 1; lane-contiguous, so the reads are free of bank
// conflicts), one pair per step.
template <int W, int T>
__device__ __forceinline__ void hidden16(f32x4 (&acc)[T][W / 16], const float (&H)[T][W / 4],
                                         const f32x2* A2, int lane, int nt) {
  constexpr int MB = W / 16, HS = W / 8, N = HS * MB, RING = kPrefetch + 1;
  // step i: K-step pair hs = i / MB of output block mb = i % MB
  auto at = [&](int i) { return A2[((i % MB) * HS + i / MB) * 64 + lane]; };
  f32x2 ring[RING];
#pragma unroll
  for (int i = 0; i < kPrefetch; ++i) ring[i] = at(i);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i + kPrefetch < N) ring[(i + kPrefetch) % RING] = at(i + kPrefetch);
    __builtin_amdgcn_sched_barrier(0);
    const int hs = i / MB, mb = i % MB;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[0][mb] = mfma16(ring[i % RING][j], H[0][2 * hs + j], acc[0][mb]);
#pragma unroll
      for (int t = 1; t < T; ++t)
        if (t <= nt) acc[t][mb] = mfma16(ring[i % RING][j], H[t][2 * hs + j], acc[t][mb]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One BF16 hidden layer from LDS: A is [W/16 output blocks][W/32 K-steps][64 lanes] bf16x8.
template <int W, int T>
__device__ __forceinline__ void hidden16_bf16(f32x4 (&acc)[T][W / 16], const bf16x8 (&Hb)[T][W / 32],
                                              const bf16x8* A, int lane, int nt) {
  // a primal tile has registers for a deeper ring: its products are 16 cycles apart, so
  // four steps ahead is shorter than an LDS read's latency
  constexpr int kPrefetch = T == 1 ? kPrefetchBf16Primal : nsf::kPrefetch;
  constexpr int MB = W / 16, S = W / 32, N = S * MB, RING = kPrefetch + 1;
  // step i: K-step s = i / MB of output block mb = i % MB
  auto at = [&](int i) { return A[((i % MB) * S + i / MB) * 64 + lane]; };
  bf16x8 ring[RING];
#pragma unroll
  for (int i = 0; i < kPrefetch; ++i) ring[i] = at(i);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i + kPrefetch < N) ring[(i + kPrefetch) % RING] = at(i + kPrefetch);
    __builtin_amdgcn_sched_barrier(0);
    const int s = i / MB, mb = i % MB;
    acc[0][mb] = mfma16_bf16(ring[i % RING], Hb[0][s], acc[0][mb]);
#pragma unroll
    for (int t = 1; t < T; ++t)
      if (t <= nt) acc[t][mb] = mfma16_bf16(ring[i % RING], Hb[t][s], acc[t][mb]);
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

// Training: store the (scaled) pre-activations of one layer, point-major saved[layer][p][W],
// as FP32 or rounded to BF16 (BF16 training).
template <int W, int T>
__device__ __forceinline__ void save_preact16(const FieldJob& jb, const f32x4 (&acc)[T][W / 16],
                                              int layer, int p, bool valid, int g) {
  if (jb.saved == nullptr || !valid) return;
  if (jb.saved_bf16) {
    __bf16* row = reinterpret_cast<__bf16*>(jb.saved) + ((int64_t)layer * jb.n + p) * W;
#pragma unroll
    for (int mb = 0; mb < W / 16; ++mb) {
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      const bf16x4 v = {(__bf16)acc[0][mb][0], (__bf16)acc[0][mb][1], (__bf16)acc[0][mb][2], (__bf16)acc[0][mb][3]};
      *reinterpret_cast<bf16x4*>(row + 16 * mb + 4 * g) = v;
    }
    return;
  }
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

template <bool BF>
__device__ __forceinline__ const char* hidden_src(const FieldPack& w, bool tr = false) {
  if (tr) return BF ? reinterpret_cast<const char*>(w.whbt) : reinterpret_cast<const char*>(w.whpt);
  return BF ? reinterpret_cast<const char*>(w.whb) : reinterpret_cast<const char*>(w.whp);
}

// Copy hidden layer k of `w` (tr: its transpose) into LDS buffer dst with direct
// global->LDS loads; the 1 KB chunks are dealt to the waves of the workgroup round-robin.
template <int W, bool BF, int WPG>
__device__ __forceinline__ void dma_layer(const FieldPack& w, int k, char* dst, int wave, int lane,
                                          bool tr = false) {
  const char* src = hidden_src<BF>(w, tr) + (size_t)k * HiddenLayer<W, BF>::kBytes;
#pragma unroll
  for (int chunk = wave; chunk < HiddenLayer<W, BF>::kChunks; chunk += WPG)
    __builtin_amdgcn_global_load_lds(src + chunk * 1024 + lane * 16,
                                      (lds_void*)(dst + chunk * 1024), 16, 0, 0);
}

// Copy all four hidden layers of `w` (contiguous in the pack) into LDS, round-robin.
template <int W, bool BF, int WPG>
__device__ __forceinline__ void dma_all_layers(const FieldPack& w, char* dst, int wave, int lane) {
  constexpr int kTotal = 4 * HiddenLayer<W, BF>::kChunks;
  const char* src = hidden_src<BF>(w);
  for (int chunk = wave; chunk < kTotal; chunk += WPG)
    __builtin_amdgcn_global_load_lds(src + chunk * 1024 + lane * 16, (lds_void*)(dst + chunk * 1024), 16, 0, 0);
}

__device__ __forceinline__ void wait_dma_and_sync() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Workgroup barrier that orders LDS accesses only: it waits for the wave's LDS operations
// but not for its global loads, so a weight copy in flight keeps going across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The point of lane l in a 16-point tile starting at p0 (clamped for the ragged tail) and
// its reference position.
struct TilePoint {
  int p;
  bool valid;
  float X[3];
  float xg;   // X[lane / 16] for the lanes of groups 0..2 (layer 1's position rows)
};

__device__ __forceinline__ TilePoint tile_point(const FieldJob& jb, int p0, int lane) {
  TilePoint tp;
  tp.p = p0 + (lane & 15);
  tp.valid = tp.p < jb.n;
  int gi = jb.p_off + (tp.valid ? tp.p : jb.n - 1);
  if (jb.idx != nullptr) {
    const int32_t* row = jb.idx;
    if (jb.step != nullptr) row += ((*jb.step + jb.step_off) % jb.plan_steps) * (int64_t)jb.plan_ld;
    gi = row[gi];
  }
  tp.X[0] = jb.X[gi];
  tp.X[1] = jb.X[jb.ldx + gi];
  tp.X[2] = jb.X[2 * jb.ldx + gi];
  // layer 1's input row k = lane group g < 3 (chosen here from the loaded values: a
  // choice among X[] by a lane-varying index later can become an indexed load from memory)
  const int g = lane >> 4;
  tp.xg = g == 0 ? tp.X[0] : g == 1 ? tp.X[1] : tp.X[2];
  return tp;
}

// Layer 1: input rows 0..2 = X, 3..2+r = z, 3+r = 1 (bias column), four per K-step, into
// zeroed accumulators. Tangent columns (t = 1..NT) are one-hot in z at t0 + t - 1
// (Jacobian) or the direction z - z2 (JVP job).
// f(0) .. f(n - 1) for the K-step counts of layer 1 (2 .. 9): with the count fixed at
// compile time the steps are straight-line code, so all their loads are issued before the
// first product instead of one step's loads per round trip (for a single output block:
// a whole tile's steps would hold too many loads in flight).
template <int N, class F>
__device__ __forceinline__ void unroll_n(F&& f) {
#pragma unroll
  for (int i = 0; i < N; ++i) f(i);
}
template <class F>
__device__ __forceinline__ void for_k1_steps(int n, F&& f) {
  switch (n) {
    case 2: unroll_n<2>(f); break;
    case 3: unroll_n<3>(f); break;
    case 4: unroll_n<4>(f); break;
    case 5: unroll_n<5>(f); break;
    case 6: unroll_n<6>(f); break;
    case 7: unroll_n<7>(f); break;
    case 8: unroll_n<8>(f); break;
    case 9: unroll_n<9>(f); break;
    default:
      for (int i = 0; i < n; ++i) f(i);
  }
}

template <int W, int T, int NT>
__device__ __forceinline__ void layer1_16(const FieldJob& jb, const TilePoint& tp, int t0, int lane,
                                          f32x4 (&acc)[T][W / 16]) {
  constexpr int MB = W / 16;
  const int g = lane >> 4, r = jb.r;
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[t][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int K1q = (r + 7) >> 2;
  const bool jvp = jb.jvp != 0;
  for (int s4 = 0; s4 < K1q; ++s4) {
    const int k = 4 * s4 + g;
    float b0 = 0.f, bt = 0.f;
    if (k < 3) b0 = tp.xg;
    else if (k < 3 + r && jb.zrows != nullptr) {
      b0 = jb.zrows[(int64_t)(tp.valid ? tp.p : jb.n - 1) * r + (k - 3)];
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
        if (t <= NT) acc[t][mb] = mfma16(a, jvp ? bt : ((k == 3 + t0 + t - 1) ? 1.f : 0.f), acc[t][mb]);
    }
  }
}

// One wave evaluates a 16-point tile of a job, starting at point p0: the primal plus
// tangents [t0, t0 + nt). Two ways to hold the hidden-layer weights:
//  - streamed (RES = false): the WPG waves of a workgroup run tiles of the same job in
//    step; layers stream through two LDS buffers, layer k + 1 (or the next group's first
//    hidden layer) fetched while layer k computes, with a workgroup barrier per layer;
//  - resident (RES = true, BF16 decode): all four hidden layers sit in LDS for the whole
//    kernel, and waves run their tiles independently, without barriers.
// Returns after the output layer.
// A kernel that evaluates one weight set (the decode) keeps its small parameters in LDS
// after the two layer buffers, copied once per launch (floats): the four hidden biases
// (4 W), the output rows (up to 9 W), layer 1's B-operand rows k >= 3 (the latent, the
// bias row 1, zeros: 64) and layer 1's A fragments (W / 16 x up to 9 K-steps x 64 lanes).
// Tiles then start and end without waiting for global memory.
template <int W>
struct ParamsLds {
  static constexpr int kBias = 0, kOut = 4 * W, kZ = 13 * W, kW1 = 13 * W + 64;
  static constexpr int kFloats = kW1 + (W / 16) * ((kMaxR + 7) / 4) * 64;
};

// Layer 1 of a primal tile with its A fragments and latent rows in LDS (see ParamsLds).
template <int W>
__device__ __forceinline__ void layer1_16_lds(const FieldJob& jb, const TilePoint& tp, int lane,
                                              f32x4 (&acc)[1][W / 16], const float* prm) {
  constexpr int MB = W / 16;
  const int g = lane >> 4;
  const int K1q = (jb.r + 7) >> 2;
  const float* zrow = prm + ParamsLds<W>::kZ;
  const float* w1 = prm + ParamsLds<W>::kW1;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[0][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int s4 = 0; s4 < K1q; ++s4) {
    const int k = 4 * s4 + g;
    const float b0 = k < 3 ? tp.xg : zrow[k];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[0][mb] = mfma16(w1[(mb * K1q + s4) * 64 + lane], b0, acc[0][mb]);
  }
}

// PARAMS_LDS: the weight set's small parameters are in LDS (ParamsLds; primal groups
// only); otherwise they are read from the pack in global memory.
template <int W, int NT, bool BF, int WPG, bool RES = false, bool PARAMS_LDS = false, class NextFn>
__device__ __forceinline__ void run_group16(const FieldJob& jb, int p0, int t0, NextFn&& next,
                                            char* lds, int wave, int lane) {
  constexpr int MB = W / 16;
  constexpr int T = 1 + NT;
  constexpr int nt = NT;  // compile-time: no per-MFMA guards
  constexpr int LB = HiddenLayer<W, BF>::kBytes;
  const int g = lane >> 4;
  const TilePoint tp = tile_point(jb, p0, lane);
  const int p = tp.p;
  const bool valid = tp.valid;
  const int r = jb.r;
  const bool jvp = jb.jvp != 0;
  f32x4 acc[T][MB];
  // PARAMS_LDS only: after the two streamed layer buffers, or after the four resident layers
  const float* prm = reinterpret_cast<const float*>(lds + (RES ? 4 : 2) * LB);
  if constexpr (PARAMS_LDS) {
    static_assert(NT == 0 && BF == RES, "LDS parameters serve the FP32 primal and the resident BF16 decode");
    layer1_16_lds<W>(jb, tp, lane, acc, prm);
  } else {
    layer1_16<W, T, NT>(jb, tp, t0, lane, acc);
  }
  if constexpr (NT == 0) save_preact16<W, T>(jb, acc, 0, p, valid, g);

  // Hidden layers 2..5 (k = 0..3). Streamed: wait for layer k in LDS, then start fetching
  // layer k + 1 (after the last layer: the next group's first layer) while k computes.
  // The last layer's activations stay FP32 for the FP32 output layer.
  // Layer k's products (after its weights are in LDS) into acc. The bias loads go out
  // before the next layer's copy: loads complete in order, so the first product then
  // waits for the bias alone and the copy overlaps the products.
  auto layer = [&](int k, auto&& hidden) {
    char* cur = lds + (RES ? k : (k & 1)) * LB;
    if constexpr (!RES) wait_dma_and_sync();
    if constexpr (PARAMS_LDS) init16<W, T, true>(acc, prm + ParamsLds<W>::kBias + k * W, g);
    else init16<W, T>(acc, jb.w.bhq + k * W, g);
    if constexpr (!RES) {
      if (k < 3) dma_layer<W, BF, WPG>(jb.w, k + 1, lds + ((k + 1) & 1) * LB, wave, lane);
      else if (const FieldPack* next_w = next()) dma_layer<W, BF, WPG>(*next_w, 0, lds, wave, lane);
    }
    hidden(cur);
    if constexpr (NT == 0) save_preact16<W, T>(jb, acc, k + 1, p, valid, g);
  };
  float H[T][W / 4];
  if constexpr (BF) {
    // BF16 activations between layers; the last layer's are FP32, for the output layer
    // (peeled off the loop, so H and Hb are never live together)
    bf16x8 Hb[T][W / 32];
    activate16_bf16<W, T>(acc, Hb, nt);
    auto hb = [&](char* cur) { hidden16_bf16<W, T>(acc, Hb, reinterpret_cast<const bf16x8*>(cur), lane, nt); };
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
      layer(k, hb);
      activate16_bf16<W, T>(acc, Hb, nt);
    }
    layer(3, hb);
  } else {
    activate16<W, T>(acc, H, nt);
    auto hf = [&](char* cur) { hidden16<W, T>(acc, H, reinterpret_cast<const f32x2*>(cur), lane, nt); };
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
      layer(k, hf);
      activate16<W, T>(acc, H, nt);
    }
    layer(3, hf);
  }
  activate16<W, T>(acc, H, nt);

  const int d = jb.d;
  if constexpr (NT >= 1) {
    if (jvp) {  // directional derivative only: out = scale * (W6 T) * jvp_scale
#pragma unroll 1
      for (int c = 0; c < 3; ++c) {
        const float y = output_dot16<W>(jb.w.w6q, c, g, H[1]);
        if (valid && g == c) jb.out[c * jb.ldo + p] = jb.scale[c] * y * jb.jvp_scale;
      }
      return;
    }
  }
  // Output layer, primal (one output at a time: unrolled, the weight loads of all nine
  // would be hoisted).
  if (t0 == 0) {
#pragma unroll 1
    for (int o = 0; o < d; ++o) {
      const float* w6 = PARAMS_LDS ? prm + ParamsLds<W>::kOut : jb.w.w6q;
      const float y = output_dot16<W>(w6, o, g, H[0]) + jb.w.b6[o];
      float v = jb.scale[o] * y + jb.shift[o];
      if (jb.mode == 1) v += ((o == 0) ? tp.X[0] : (o == 1) ? tp.X[1] : tp.X[2]);
      if (valid && g == (o & 3)) jb.out[o * jb.ldo + p] = v;
    }
  }
  // Output layer, tangents (deformation field only: d = 3), one output row at a time:
  // unrolled, the weight loads of all three rows would be hoisted.
  if constexpr (NT >= 1) {
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int t = 1; t < T; ++t) {
        const float y = output_dot16<W>(jb.w.w6q, c, g, H[t]);
        if (valid && g == c) jb.jac[(c * r + t0 + t - 1) * jb.ldj + p] = jb.scale[c] * y;
      }
    }
  }
}

// ---- reverse-mode Jacobian ----------------------------------------------------------
// For a Jacobian with many latent columns the tangent groups above recompute the primal
// once per TC columns. Reverse mode instead runs the primal once and pulls one output
// component c back through the layers: delta_5 = W6[c, :] . phi'(a_5),
// delta_{k-1} = (W_k^T delta_k) . phi'(a_{k-1}), du_c/dz = W1_z^T delta_1, where W1_z are
// layer 1's latent columns. Each matrix product is the same MFMA pattern as the forward
// one with the transposed weights (packed in the same operand order), so the cotangent
// stays in the accumulator layout and phi' of every layer is applied in-lane. A wave keeps
// phi'(a_1..a_4) of its tile in registers (4 x W/4 floats). One group per output component:
// a 16-point tile costs two matrix passes per wave instead of 1 + TC per TC latent
// columns.

// Activation that also keeps phi': FP32 into H, BF16 into Hb (the next layer's operands).
template <int W, bool BF>
__device__ __forceinline__ void activate_keep(const f32x4 (&acc)[1][W / 16], float (&H)[1][W / 4],
                                              bf16x8 (&Hb)[1][BF ? W / 32 : 1], float (&D)[W / 4]) {
  if constexpr (BF) {
#pragma unroll
    for (int s = 0; s < W / 32; ++s) {
      bf16x8 p0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float y;
        elu_pair<true>(acc[0][2 * s + (e >> 2)][e & 3], y, D[4 * (2 * s + (e >> 2)) + (e & 3)]);
        p0[e] = (__bf16)y;
      }
      Hb[0][s] = p0;
    }
  } else {
#pragma unroll
    for (int mb = 0; mb < W / 16; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) elu_pair<true>(acc[0][mb][v], H[0][4 * mb + v], D[4 * mb + v]);
  }
}

// Cotangent acc . D into the next product's operands (FP32 H, or BF16 Hb).
template <int W, bool BF>
__device__ __forceinline__ void cotangent_operand(const f32x4 (&acc)[1][W / 16], const float (&D)[W / 4],
                                                  float (&H)[1][W / 4], bf16x8 (&Hb)[1][BF ? W / 32 : 1]) {
  if constexpr (BF) {
#pragma unroll
    for (int s = 0; s < W / 32; ++s) {
      bf16x8 p0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int mb = 2 * s + (e >> 2), v = e & 3;
        p0[e] = (__bf16)(acc[0][mb][v] * D[4 * mb + v]);
      }
      Hb[0][s] = p0;
    }
  } else {
#pragma unroll
    for (int mb = 0; mb < W / 16; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) H[0][4 * mb + v] = acc[0][mb][v] * D[4 * mb + v];
  }
}

// One wave: the primal of a 16-point tile (written by the c = 0 group) and row c of its
// Jacobian, with streamed weights: the four hidden layers, then their transposes in
// reverse order, through the two LDS buffers with one workgroup barrier per layer.
template <int W, bool BF, int WPG, class NextFn>
__device__ __forceinline__ void run_rev16(const FieldJob& jb, int p0, int c, NextFn&& next, char* lds,
                                          int wave, int lane) {
  constexpr int MB = W / 16;
  constexpr int LB = HiddenLayer<W, BF>::kBytes;
  const int g = lane >> 4;
  const TilePoint tp = tile_point(jb, p0, lane);
  const int p = tp.p, r = jb.r;
  const bool valid = tp.valid;
  f32x4 acc[1][MB];
  layer1_16<W, 1, 0>(jb, tp, 0, lane, acc);
  float D[4][W / 4];   // phi'(a_1) .. phi'(a_4)
  float H[1][W / 4];
  bf16x8 Hb[1][BF ? W / 32 : 1];
  activate_keep<W, BF>(acc, H, Hb, D[0]);
  // stage i = 0..3: hidden layer i; i = 4..7: the transpose of hidden layer 7 - i. A
  // forward stage loads its bias into acc between the barrier and the next copy (loads
  // complete in order: the products then wait for the bias, not for the copy).
  auto stage = [&](int i) -> const char* {
    wait_dma_and_sync();
    if (i < 4) init16<W, 1>(acc, jb.w.bhq + i * W, g);
    if (i < 7) {
      const int kn = i + 1;
      dma_layer<W, BF, WPG>(jb.w, kn < 4 ? kn : 7 - kn, lds + (kn & 1) * LB, wave, lane, kn >= 4);
    } else if (const FieldPack* next_w = next()) {
      dma_layer<W, BF, WPG>(*next_w, 0, lds, wave, lane);
    }
    return lds + (i & 1) * LB;
  };
  auto product = [&](const char* cur) {
    if constexpr (BF) hidden16_bf16<W, 1>(acc, Hb, reinterpret_cast<const bf16x8*>(cur), lane, 0);
    else hidden16<W, 1>(acc, H, reinterpret_cast<const f32x2*>(cur), lane, 0);
  };
  // unrolled: D is indexed by the layer, and registers cannot be indexed at run time
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const char* cur = stage(k);
    product(cur);
    activate_keep<W, BF>(acc, H, Hb, D[k + 1]);
  }
  {
    const char* cur = stage(3);
    product(cur);
  }
  // layer 5: the primal output from FP32 activations, then delta_5 = W6[c, :] . phi'(a_5)
  // (phi'(a_5) recomputed from a_5, which acc still holds, rather than kept)
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float dy;
      elu_pair<true>(acc[0][mb][v], H[0][4 * mb + v], dy);
    }
  if (c == 0) {
#pragma unroll 1
    for (int o = 0; o < 3; ++o) {
      const float y = output_dot16<W>(jb.w.w6q, o, g, H[0]) + jb.w.b6[o];
      if (valid && g == o) jb.out[o * jb.ldo + p] = jb.scale[o] * y + jb.shift[o];
    }
  }
  {
    const float* w6 = jb.w.w6q + c * W + 4 * g;
    float ones[W / 4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const f32x4 w4 = *reinterpret_cast<const f32x4*>(w6 + 16 * mb);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float y, dy;
        elu_pair<true>(acc[0][mb][v], y, dy);
        acc[0][mb][v] = w4[v] * dy;
        ones[4 * mb + v] = 1.f;
      }
    }
    cotangent_operand<W, BF>(acc, ones, H, Hb);
  }
  // back through W5^T .. W2^T; delta_1 stays FP32 for the latent columns of layer 1
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const char* cur = stage(4 + j);
    init16<W, 1>(acc, nullptr, g);
    product(cur);
    cotangent_operand<W, BF>(acc, D[3 - j], H, Hb);
  }
  {
    const char* cur = stage(7);
    init16<W, 1>(acc, nullptr, g);
    product(cur);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) H[0][4 * mb + v] = acc[0][mb][v] * D[0][4 * mb + v];
  }
  // du_c/dz_j = sum_m W1[m][3 + j] delta_1[m], rows j in blocks of 16 (at most two)
  const int MZ = (r + 15) >> 4;
  const f32x2* Z = reinterpret_cast<const f32x2*>(jb.w.w1zt);
  f32x4 jz[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
  for (int mz = 0; mz < 2; ++mz) {
    if (mz < MZ) {
#pragma unroll
      for (int hs = 0; hs < W / 8; ++hs) {
        const f32x2 a = Z[((size_t)mz * (W / 8) + hs) * 64 + lane];
        jz[mz] = mfma16(a[0], H[0][2 * hs], jz[mz]);
        jz[mz] = mfma16(a[1], H[0][2 * hs + 1], jz[mz]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = 16 * mz + 4 * g + v;
        if (valid && jj < r) jb.jac[(c * r + jj) * jb.ldj + p] = jb.scale[c] * jz[mz][v];
      }
    }
  }
}

// ---- team groups: reverse-mode Jacobian over one or two tiles per workgroup (FP32, W 128)
// The W / 16 waves of a workgroup share NT 16-point tiles (two, FieldTile.nt = -2, or one,
// nt = -3, for tables too short to fill the device with pairs): wave q owns output block
// q (16 neurons) of every layer for all of them. A layer's product needs the whole previous
// layer as the MFMA B operand, so each wave publishes its block through LDS (K-steps
// 4q .. 4q + 3 of each tile's operand, lane-major, conflict-free) and reads back all of
// them. The forward pass runs once, phi'(a_1..a_4) of the wave's block stays in its
// registers, and the three output components are pulled back together: three cotangent
// operands per tile share each weight fragment. du_c/dz = W1_z^T delta_1 is summed over
// the waves' blocks through LDS in a fixed order.
//
// A wave reads only block q of a layer (W / 8 fragments, 8 KB at width 128), so the
// layers need no workgroup-wide copy: each wave copies its block of the next stage's layer
// into its own slot of the first LDS buffer while the current stage computes (block q at
// q x 8 KB, which is also where a whole-layer copy puts it), and reads it into registers
// at the start of that stage. The exchanged operands live in the second buffer. With two
// tiles per group, a stage's products are twice those of one tile between the same
// barriers.
//
// After the Jacobian job, a group can evaluate up to three more jobs over the same point
// range, forward only, in the same way (FieldTile.t0: their job offsets from the group's
// job, one signed byte each, 0 = none): the step's stress and affine fields, or the
// velocity's deformation field at the next step's points. A pass then holds one group per
// CU of equal length instead of Jacobian groups beside longer primal groups.

// Tiles of a team group from its FieldTile.nt (-2: two, -3: one).
__host__ __device__ constexpr int team_tiles(int nt) { return nt == -2 ? 2 : 1; }
constexpr int kTeamW6 = 3;   // output rows per thread (9 rows of W floats over W / 16 waves)

template <int W>
struct TeamFrag {
  f32x2 f[W / 8];
};

template <int W>
constexpr int team_block_bytes() { return (W / 8) * 64 * 8; }

// The layer a team stage copies for the next one: hidden layer k of pk (tr: its
// transpose), or none.
struct TeamNext {
  const FieldPack* pk;
  int k;
  bool tr;
};

// Copy block q of nx's layer into the wave's slot (wave-private: no barrier orders it).
template <int W>
__device__ __forceinline__ void team_stage_copy(const TeamNext& nx, char* lds, int q, int lane) {
  if (nx.pk == nullptr) return;
  constexpr int BB = team_block_bytes<W>();
  const char* src = hidden_src<false>(*nx.pk, nx.tr) + (size_t)nx.k * HiddenLayer<W, false>::kBytes + q * BB;
#pragma unroll
  for (int c = 0; c < BB / 1024; ++c)
    __builtin_amdgcn_global_load_lds(src + c * 1024 + lane * 16, (lds_void*)(lds + q * BB + c * 1024), 16, 0, 0);
}

// The stage's fragments from the wave's slot, once the wave's copy has landed.
template <int W>
__device__ __forceinline__ void team_stage_read(TeamFrag<W>& w, const char* lds, int q, int lane) {
  __builtin_amdgcn_s_waitcnt(0);
  const f32x2* blk = reinterpret_cast<const f32x2*>(lds + q * team_block_bytes<W>());
#pragma unroll
  for (int hs = 0; hs < W / 8; ++hs) w.f[hs] = blk[hs * 64 + lane];
}

// s_waitcnt lgkmcnt(0) alone: the wave's LDS reads have returned (its slot may be
// overwritten by the next copy).
__device__ __forceinline__ void wait_lds_reads() { __builtin_amdgcn_s_waitcnt(0xC07F); }

template <int W>
__device__ __forceinline__ f32x4 layer1_block(const FieldJob& jb, const TilePoint& tp, int lane, int mb) {
  const int g = lane >> 4, r = jb.r;
  const int K1q = (r + 7) >> 2;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for_k1_steps(K1q, [&](int s4) __attribute__((always_inline)) {
    const int k = 4 * s4 + g;
    float b0 = 0.f;
    if (k < 3) b0 = tp.xg;
    else if (k < 3 + r) b0 = (float)jb.z[k - 3];
    else if (k == 3 + r) b0 = 1.f;
    acc = mfma16(jb.w.w1q[(mb * K1q + s4) * 64 + lane], b0, acc);
  });
  return acc;
}

// Forward pass of a team job over NT tiles: layer 1 and the four hidden layers of block
// q (hidden layer 0 already in the wave's slot; the last stage copies `after`). KEEP:
// phi'(a_1 .. a_4) of the block into D. Returns a_5's activation h5 and derivative dphi5,
// and this thread's share of the output rows in w6.
template <int W, int NT, bool KEEP>
__device__ __forceinline__ void team_forward(const FieldJob& jb, const TilePoint (&tp)[NT], const TeamNext& after,
                                             float* X, char* lds, int q, int lane, float (&D)[NT][4][4],
                                             float (&h5)[NT][4], float (&dphi5)[NT][4], float (&w6)[kTeamW6]) {
  constexpr int KS = W / 4, HS = W / 8;
  const int g = lane >> 4;
  auto bias = [&](int k) { return *global_ptr(reinterpret_cast<const f32x4*>(jb.w.bhq + k * W + 16 * q + 4 * g)); };
  f32x4 bnext = bias(0);
  f32x4 a[NT];
  float h[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    a[t] = layer1_block<W>(jb, tp[t], lane, q);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float dy;
      elu_pair<true>(a[t][v], h[t][v], dy);
      if constexpr (KEEP) D[t][0][v] = dy;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // two exchange buffers by layer parity: a stage's writes never meet the previous
    // stage's reads, so one barrier per stage
    float* Xk = X + (k & 1) * NT * KS * 64;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) Xk[(t * KS + 4 * q + v) * 64 + lane] = h[t][v];
    lds_barrier();   // publish the blocks
    TeamFrag<W> wc;
    team_stage_read<W>(wc, lds, q, lane);
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = bnext;
    if (k < 3) {
      bnext = bias(k + 1);
    } else {
      // this thread's share of the output rows, for the output layer
#pragma unroll
      for (int i = 0; i < kTeamW6; ++i) {
        const int e = (int)threadIdx.x + i * 4 * W;   // 4 W = 64 lanes x W / 16 waves
        w6[i] = e < jb.d * W ? jb.w.w6q[e] : 0.f;
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float Hf[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) Hf[s] = Xk[(t * KS + s) * 64 + lane];
      if (t == 0) {
        wait_lds_reads();
        team_stage_copy<W>(k < 3 ? TeamNext{&jb.w, k + 1, false} : after, lds, q, lane);
      }
      __builtin_amdgcn_sched_barrier(0);   // the operand's reads all go out before its products
#pragma unroll
      for (int hs = 0; hs < HS; ++hs) {
        a[t] = mfma16(wc.f[hs][0], Hf[2 * hs], a[t]);
        a[t] = mfma16(wc.f[hs][1], Hf[2 * hs + 1], a[t]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (k < 3) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float dy;
          elu_pair<true>(a[t][v], h[t][v], dy);
          if constexpr (KEEP) D[t][k + 1][v] = dy;
        }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) elu_pair<true>(a[t][v], h5[t][v], dphi5[t][v]);
}

// Output layer of a team job. The blocks of h5 are published like a layer's operand, with
// the job's output rows (w6: this thread's share), and output row o of tile t is then
// formed by one wave over the whole row, with the primal groups' own operation order
// (output_dot16): a job gives the same bits in a team group and in a primal group. Wave
// q takes tile q % NT and outputs q / NT + i WPG / NT.
template <int W, int WPG, int NT>
__device__ __forceinline__ void team_output(const FieldJob& jb, int p0, const float (&h5)[NT][4],
                                            const float (&w6)[kTeamW6], float* X, int q, int lane) {
  constexpr int KS = W / 4, OPW = (9 * NT + WPG - 1) / WPG;   // outputs per wave at most
  static_assert(WPG % NT == 0, "waves split evenly over the tiles");
  const int d = jb.d, g = lane >> 4, t = q % NT, o0 = q / NT;
  // the output rows, [d][W], past both forward exchange buffers: a slower wave may still
  // read the last hidden layer's operand from the second one
  float* Xw = X + 2 * NT * KS * 64;
#pragma unroll
  for (int i = 0; i < kTeamW6; ++i) {
    const int e = (int)threadIdx.x + i * 64 * WPG;   // as loaded in team_forward
    if (e < d * W) Xw[e] = w6[i];
  }
#pragma unroll
  for (int tt = 0; tt < NT; ++tt)
#pragma unroll
    for (int v = 0; v < 4; ++v) X[(tt * KS + 4 * q + v) * 64 + lane] = h5[tt][v];
  lds_barrier();
  float Hrow[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) Hrow[s] = X[(t * KS + s) * 64 + lane];
  const int p = p0 + 16 * t + (lane & 15);
#pragma unroll
  for (int i = 0; i < OPW; ++i) {
    const int o = o0 + i * (WPG / NT);
    if (o < d) {
      const float y = output_dot16<W>(Xw, o, g, Hrow) + jb.w.b6[o];
      if (p < jb.n && g == (o & 3)) jb.out[o * jb.ldo + p] = jb.scale[o] * y + jb.shift[o];
    }
  }
  lds_barrier();   // X may be rewritten
}

// Reverse pass of the Jacobian job: delta_5 of the three components, back through
// W5^T .. W2^T (the transpose of hidden layer 3 already in the wave's slot; the last stage
// copies `after`), then du_c/dz = W1_z^T delta_1 summed over the blocks.
template <int W, int WPG, int NT>
__device__ __forceinline__ void team_reverse(const FieldJob& jb, int p0, const TeamNext& after, float* X,
                                             char* lds, int q, int lane, const float (&D)[NT][4][4],
                                             const float (&dphi5)[NT][4]) {
  constexpr int KS = W / 4, HS = W / 8;
  const int g = lane >> 4, r = jb.r;
  f32x4 w6v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) w6v[c] = *global_ptr(reinterpret_cast<const f32x4*>(jb.w.w6q + c * W + 16 * q + 4 * g));
  const int MZ = (r + 15) >> 4;
  const auto* Z = global_ptr(reinterpret_cast<const f32x2*>(jb.w.w1zt));
  f32x2 zf[2][2];
#pragma unroll
  for (int mz = 0; mz < 2; ++mz)
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
      zf[mz][hh] = mz < MZ ? Z[((size_t)mz * HS + 2 * q + hh) * 64 + lane] : f32x2{0.f, 0.f};
  float d[NT][3][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) d[t][c][v] = w6v[c][v] * dphi5[t][v];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) X[((t * 3 + c) * KS + 4 * q + v) * 64 + lane] = d[t][c][v];
    lds_barrier();   // publish the blocks
    TeamFrag<W> wc;
    team_stage_read<W>(wc, lds, q, lane);
    // one (tile, component) operand at a time: its 32 reads, then its 32 products
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        __builtin_amdgcn_sched_barrier(0);
        float Hc[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) Hc[s] = X[((t * 3 + c) * KS + s) * 64 + lane];
        if (t == 0 && c == 0) {
          wait_lds_reads();
          team_stage_copy<W>(j < 3 ? TeamNext{&jb.w, 2 - j, true} : after, lds, q, lane);
        }
        __builtin_amdgcn_sched_barrier(0);   // the operand's reads all go out before its products
        f32x4 ac = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int hs = 0; hs < HS; ++hs) {
          ac = mfma16(wc.f[hs][0], Hc[2 * hs], ac);
          ac = mfma16(wc.f[hs][1], Hc[2 * hs + 1], ac);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) d[t][c][v] = ac[v] * D[t][3 - j][v];
      }
    lds_barrier();   // every wave has read the operands: X may be rewritten
  }
  // d = delta_1 of block q (K-steps 4q + v of W1_z^T's product): partial du_c/dz over the
  // block, rows in blocks of 16 (at most two), summed over the waves
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      f32x4 jz[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int mz = 0; mz < 2; ++mz) {
        if (mz < MZ) {
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            jz[mz] = mfma16(zf[mz][hh][0], d[t][c][2 * hh], jz[mz]);
            jz[mz] = mfma16(zf[mz][hh][1], d[t][c][2 * hh + 1], jz[mz]);
          }
        }
      }
#pragma unroll
      for (int mz = 0; mz < 2; ++mz)
#pragma unroll
        for (int v = 0; v < 4; ++v) X[(((t * WPG + q) * 2 + mz) * 4 + v) * 64 + lane] = jz[mz][v];
    }
    lds_barrier();
    if (q < NT) {
      const int t = q, p = p0 + 16 * t + (lane & 15);
#pragma unroll
      for (int mz = 0; mz < 2; ++mz) {
        if (mz < MZ) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float sum = 0.f;
#pragma unroll
            for (int qq = 0; qq < WPG; ++qq) sum += X[(((t * WPG + qq) * 2 + mz) * 4 + v) * 64 + lane];
            const int jj = 16 * mz + 4 * g + v;
            if (p < jb.n && jj < r) jb.jac[(c * r + jj) * jb.ldj + p] = jb.scale[c] * sum;
          }
        }
      }
    }
    lds_barrier();
  }
}

// Extra job e of a team group (see above): the group's job plus t0's signed byte e (e < 3;
// 0: no such job).
__device__ __forceinline__ int team_extra(const FieldTile& tl, int e) {
  return (int)(int8_t)((tl.t0 >> (8 * e)) & 0xff);
}

// One team group; hidden layer 0 of its job is in the first LDS buffer on entry (copied by
// the previous group, or at the kernel's start). `claim` claims the following group (every
// thread calls it at the same point) and returns its index; a following team group's
// first layer is then copied by the last stage, a primal group's after the last barrier.
template <int W, int WPG, int NT, class ClaimFn>
__device__ __forceinline__ void run_team(const FieldJob* __restrict__ jobs, const FieldTile& tl, ClaimFn&& claim,
                                         const FieldTile* __restrict__ groups, int total, char* lds, int wave,
                                         int lane) {
  static_assert(W / 16 == WPG, "one output block per wave");
  constexpr int LB = HiddenLayer<W, false>::kBytes;
  static_assert(NT * 3 * (W / 4) * 64 * 4 <= LB && NT * WPG * 2 * 4 * 64 * 4 <= LB &&
                    (2 * NT * (W / 4) * 64 + 9 * W) * 4 <= LB &&
                    kTeamW6 * 64 * WPG >= 9 * W && 64 * WPG == 4 * W && WPG * team_block_bytes<W>() == LB,
                "the exchanged operands fit in the second buffer; the blocks tile the first");
  const int q = wave;
  float* X = reinterpret_cast<float*>(lds + LB);
  const FieldJob& jb = jobs[tl.job];
  const int nx = team_extra(tl, 2) != 0 ? 3 : team_extra(tl, 1) != 0 ? 2 : team_extra(tl, 0) != 0 ? 1 : 0;
  // the previous group's LDS reads and copies are complete
  wait_dma_and_sync();
  TilePoint tp[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) tp[t] = tile_point(jb, tl.p0 + 16 * t, lane);
  float D[NT][4][4], h5[NT][4], dphi5[NT][4], w6[kTeamW6];
  team_forward<W, NT, true>(jb, tp, TeamNext{&jb.w, 3, true}, X, lds, q, lane, D, h5, dphi5, w6);
  team_output<W, WPG, NT>(jb, tl.p0, h5, w6, X, q, lane);
  const int gn = claim();
  const bool next_team = gn < total && groups[gn].nt <= -2;
  const TeamNext next_first{next_team ? &jobs[groups[gn].job].w : nullptr, 0, false};
  team_reverse<W, WPG, NT>(jb, tl.p0, nx > 0 ? TeamNext{&jobs[tl.job + team_extra(tl, 0)].w, 0, false} : next_first,
                           X, lds, q, lane, D, dphi5);
#pragma unroll 1
  for (int e = 0; e < nx; ++e) {
    const FieldJob& xb = jobs[tl.job + team_extra(tl, e)];
    // the same points as the Jacobian job's (the inference's h and l): its tile points
    // again, without the dependent loads of the point list and the positions
    const bool same_points = xb.idx == jb.idx && xb.step == jb.step && xb.step_off == jb.step_off &&
                             xb.plan_steps == jb.plan_steps && xb.plan_ld == jb.plan_ld && xb.p_off == jb.p_off &&
                             xb.X == jb.X && xb.ldx == jb.ldx && xb.n == jb.n;
    TilePoint xp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) xp[t] = same_points ? tp[t] : tile_point(xb, tl.p0 + 16 * t, lane);
    const TeamNext xn = e + 1 < nx ? TeamNext{&jobs[tl.job + team_extra(tl, e + 1)].w, 0, false} : next_first;
    team_forward<W, NT, false>(xb, xp, xn, X, lds, q, lane, D, h5, dphi5, w6);
    team_output<W, WPG, NT>(xb, tl.p0, h5, w6, X, q, lane);
  }
  // a primal group copies its layers over the whole buffer: after every wave's last read
  if (gn < total && !next_team) dma_layer<W, false, WPG>(jobs[groups[gn].job].w, 0, lds, wave, lane);
}

// Run a group with its tangent count as a template argument (0 .. TC).
template <int W, int TC, bool BF, int WPG, class NextFn>
__device__ __forceinline__ void dispatch_nt(const FieldJob& jb, int p0, int t0, int nt,
                                            NextFn&& next, char* lds, int wave, int lane) {
  if constexpr (TC > 0) {
    if (nt == TC) {
      run_group16<W, TC, BF, WPG>(jb, p0 + kTile16 * wave, t0, next, lds, wave, lane);
      return;
    }
    dispatch_nt<W, TC - 1, BF, WPG>(jb, p0, t0, nt, next, lds, wave, lane);
  } else {
    run_group16<W, 0, BF, WPG>(jb, p0 + kTile16 * wave, t0, next, lds, wave, lane);
  }
}

// Work groups from a table (several jobs; a group is WPG tiles of one job). Workgroups
// claim groups dynamically from a counter (zero at launch), one group ahead so the next
// group's first hidden layer can be fetched while the current group finishes; groups
// are ordered longest first, so the claims balance the load. KINDS: the group kinds
// besides primal ones the kernel is built for (kTableTangents, kTableTeam): the tangent
// groups and the team groups each need nearly all registers, and a kernel built for both
// spills.
template <int W, int TC, bool BF, int WPG, int KINDS>
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
  // called by every thread at the same point of a group (after a barrier)
  auto claim_next = [&]() -> int {
    if (threadIdx.x == 0) s_claim = atomicAdd(claim, 1);
    __syncthreads();
    gn = s_claim;
    return gn;
  };
  auto next = [&]() -> const FieldPack* { return claim_next() < total ? &jobs[groups[gn].job].w : nullptr; };
  while (true) {
    const FieldTile tl = groups[g];
    if (tl.p0 >= jobs[tl.job].n) {
      // past the job's points this step (a closure sim's list is shorter than its
      // capacity): keep the weight pipeline going for the next group
      wait_dma_and_sync();
      if (const FieldPack* next_w = next()) dma_layer<W, BF, WPG>(*next_w, 0, lds, wave, lane);
      if (gn >= total) break;
      g = gn;
      continue;
    }
    if constexpr (TC > 0 && !BF && W / 16 == WPG && (KINDS & kTableTeam)) {   // team groups (nt -2, -3)
      if (tl.nt <= -2) {
        run_team<W, WPG, (KINDS & kTableTeamOne) ? 1 : 2>(jobs, tl, claim_next, groups, total, lds, wave, lane);
        if (gn >= total) break;
        g = gn;
        continue;
      }
    }
    if constexpr (TC > 0 && !(!BF && W / 16 == WPG)) {   // one wave per tile and component
      if (tl.nt < 0) {
        run_rev16<W, BF, WPG>(jobs[tl.job], tl.p0 + kTile16 * wave, tl.t0, next, lds, wave, lane);
        if (gn >= total) break;
        g = gn;
        continue;
      }
    }
    if constexpr ((KINDS & kTableTangents) != 0) dispatch_nt<W, TC, BF, WPG>(jobs[tl.job], tl.p0, tl.t0, tl.nt, next, lds, wave, lane);
    else run_group16<W, 0, BF, WPG>(jobs[tl.job], tl.p0 + kTile16 * wave, tl.t0, next, lds, wave, lane);
    if (gn >= total) break;
    g = gn;
  }
}

// The barrier and DMA sequence of run_group16 (streamed weights) for a wave with no tile
// in this round: it keeps the workgroup's per-layer barriers and weight copies in step.
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

// Decode tile t of a persistent workgroup's waves: every round but the last fills all
// waves of all workgroups, and the last round's tiles go to waves 0 and 1 of distinct
// workgroups, which then run alone on their SIMDs. Waves 2q and 2q + 1 take adjacent
// tiles, so each 128-byte line of the point arrays is read by one workgroup:
// t = round * gridDim.x * WPG + q * 2 gridDim.x + 2 blockIdx.x + (wave & 1), q = wave / 2.
__device__ __forceinline__ int dense_tile(int base, int wave, int G, int b) {
  return base + (wave >> 1) * 2 * G + 2 * b + (wave & 1);
}

// One job over n points (FP32 decode), weights streamed, persistent workgroups. PL: the
// job's small parameters are copied to LDS once (ParamsLds; a job with one latent for all
// points), else read from global memory (per-point latents of the training forward).
// Copy one weight set's small parameters into LDS (ParamsLds layout), every thread of the
// workgroup taking part; the caller publishes them with a barrier.
template <int W, int WPG>
__device__ __forceinline__ void copy_params(const FieldJob& job, float* prm) {
  const int K1q = (job.r + 7) >> 2, n1 = (W / 16) * K1q * 64;
  for (int i = threadIdx.x; i < 4 * W; i += 64 * WPG) prm[ParamsLds<W>::kBias + i] = job.w.bhq[i];
  for (int i = threadIdx.x; i < job.d * W; i += 64 * WPG) prm[ParamsLds<W>::kOut + i] = job.w.w6q[i];
  for (int i = threadIdx.x; i < n1; i += 64 * WPG) prm[ParamsLds<W>::kW1 + i] = job.w.w1q[i];
  if (threadIdx.x < 64) {
    const int k = threadIdx.x;
    prm[ParamsLds<W>::kZ + k] = (k >= 3 && k < 3 + job.r) ? (float)job.z[k - 3] : (k == 3 + job.r ? 1.f : 0.f);
  }
}

template <int W, int WPG, bool PL>
__global__ __launch_bounds__(64 * WPG) void fields_dense_kernel(FieldJob job, int n_tiles) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  static_assert(WPG % 2 == 0, "waves take tiles in pairs");
  const int G = gridDim.x, b = blockIdx.x, per_round = G * WPG;
  if (2 * b >= n_tiles) return;
  dma_layer<W, false, WPG>(job.w, 0, lds, wave, lane);
  // the weight set's small parameters, once, after the two layer buffers (the first
  // tile's layer 1 reads them before any layer barrier: published by their own)
  if constexpr (PL) {
    copy_params<W, WPG>(job, reinterpret_cast<float*>(lds + 2 * HiddenLayer<W, false>::kBytes));
    lds_barrier();
  }
#pragma unroll 1
  for (int base = 0; base + 2 * b < n_tiles; base += per_round) {
    const bool more = base + per_round + 2 * b < n_tiles;
    auto next = [&]() -> const FieldPack* { return more ? &job.w : nullptr; };
    const int t = dense_tile(base, wave, G, b);
    if (t < n_tiles) run_group16<W, 0, false, WPG, false, PL>(job, t * kTile16, 0, next, lds, wave, lane);
    else idle_group<W, false, WPG>(job, next, lds, wave, lane);
  }
}

// One job over n points (BF16 decode), weights resident: every workgroup loads the four
// hidden layers once, then each wave runs its tiles independently.
template <int W, int WPG, bool PL>
__global__ __launch_bounds__(64 * WPG) void fields_dense_res_kernel(FieldJob job, int n_tiles) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  static_assert(WPG % 2 == 0, "waves take tiles in pairs");
  const int G = gridDim.x, b = blockIdx.x;
  if (2 * b >= n_tiles) return;
  dma_all_layers<W, true, WPG>(job.w, lds, wave, lane);
  // the small parameters after the four layers (layer 1 and the output layer then read
  // LDS instead of global memory in every tile)
  if constexpr (PL) copy_params<W, WPG>(job, reinterpret_cast<float*>(lds + 4 * HiddenLayer<W, true>::kBytes));
  wait_dma_and_sync();
  auto none = []() -> const FieldPack* { return nullptr; };
#pragma unroll 1
  for (int base = 0; base + 2 * b < n_tiles; base += G * WPG) {
    const int t = dense_tile(base, wave, G, b);
    if (t >= n_tiles) break;
    // keep the weight reads inside the tile: the LDS contents never change, and hoisting
    // them out of the loop would only exhaust registers
    __asm__ volatile("" ::: "memory");
    run_group16<W, 0, true, WPG, true, PL>(job, t * kTile16, 0, none, lds, wave, lane);
  }
}

// Tangents one wave carries next to the primal, by register budget (256 per lane at two
// waves per SIMD).
constexpr int kTcF32W64 = 3, kTcF32W128 = 2, kTcBf16W64 = 4, kTcBf16W128 = 2;

// Waves per workgroup of the table kernels (one workgroup per CU at width 128: its two
// LDS layer buffers take 128 KB in FP32): two waves per SIMD with tangents, four for the
// primal. A group spans WPG tiles of 16 points.
template <int TC> struct Wpg { static constexpr int value = TC > 0 ? 8 : 16; };

// Decode of several jobs (a batch's sims, each with its own weight set) in BF16 with the
// weights resident: each workgroup takes a contiguous range of the table's primal groups
// (one tile per wave), loads a job's four hidden layers and small parameters into LDS when
// its range reaches that job, and runs the groups' tiles as the single-job decode does (the
// same operations, so the same bits). A range spans one or a few jobs, so a workgroup loads
// a weight set once or twice per launch instead of streaming the layers for every group.
template <int W, int WPG>
__global__ __launch_bounds__(64 * WPG) void fields_decode_table_res_kernel(const FieldJob* __restrict__ jobs,
                                                                           const FieldTile* __restrict__ groups,
                                                                           const int32_t* __restrict__ n_groups) {
  static_assert(WPG == Wpg<0>::value, "a primal group holds one tile per wave");
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int total = *n_groups;
  const int g0 = (int)((int64_t)total * blockIdx.x / gridDim.x);
  const int g1 = (int)((int64_t)total * (blockIdx.x + 1) / gridDim.x);
  float* prm = reinterpret_cast<float*>(lds + 4 * HiddenLayer<W, true>::kBytes);
  auto none = []() -> const FieldPack* { return nullptr; };
  int cur = -1;
#pragma unroll 1
  for (int gi = g0; gi < g1; ++gi) {
    const int j = __builtin_amdgcn_readfirstlane(groups[gi].job);
    const int p0 = groups[gi].p0 + kTile16 * wave;
    if (j != cur) {
      if (cur >= 0) __syncthreads();   // every wave is done with the resident weight set
      dma_all_layers<W, true, WPG>(jobs[j].w, lds, wave, lane);
      copy_params<W, WPG>(jobs[j], prm);
      wait_dma_and_sync();
      cur = j;
    }
    // (as in the single-job decode: the weight reads stay inside the tile)
    __asm__ volatile("" ::: "memory");
    if (p0 < jobs[cur].n) run_group16<W, 0, true, WPG, true, true>(jobs[cur], p0, 0, none, lds, wave, lane);
  }
}

template <int W, int TC, bool BF, int KINDS = kTableTangents>
hipError_t launch_table(const FieldJob* jobs, const FieldTile* groups, const int32_t* n_groups,
                        int32_t* claim, int grid, hipStream_t s) {
  constexpr int WPG = Wpg<TC>::value;
  constexpr int lds = 2 * HiddenLayer<W, BF>::kBytes;   // team groups exchange in the second buffer
  auto k = fields_table_kernel<W, TC, BF, WPG, KINDS>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WPG), lds, s, jobs, groups, n_groups, claim);
  return hipGetLastError();
}

// Persistent decode grid: as many workgroups as fit on `cus` CUs at once.
template <class K>
hipError_t decode_grid(K k, int wpg, int lds, int cus, int* per_cu, int* grid) {
  if (*per_cu == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, 64 * wpg, lds);
    if (e != hipSuccess) return e;
    if (*per_cu < 1) *per_cu = 1;
  }
  *grid = cus * *per_cu;
  return hipSuccess;
}

// Waves per decode workgroup: FP32 three per SIMD (137 registers), BF16 four (106), the
// fastest measured.
constexpr int kDenseWpg = 12, kDenseResWpg = 16;

template <int W, int WPG, bool PL>
hipError_t launch_dense_pl(const FieldJob& job, int n_tiles, int cus, hipStream_t s) {
  constexpr int lds = 2 * HiddenLayer<W, false>::kBytes + (PL ? ParamsLds<W>::kFloats * 4 : 0);
  static_assert(lds <= 160 * 1024, "layer buffers and parameters must fit in LDS");
  auto k = fields_dense_kernel<W, WPG, PL>;
  static int per_cu = 0;
  int grid = 0;
  const hipError_t e = decode_grid(k, WPG, lds, cus, &per_cu, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WPG), lds, s, job, n_tiles);
  return hipGetLastError();
}

template <int W, int WPG>
hipError_t launch_dense(const FieldJob& job, int n_tiles, int cus, hipStream_t s) {
  const bool pl = job.zrows == nullptr && job.jvp == 0 && job.r <= kMaxR && job.d <= 9;
  return pl ? launch_dense_pl<W, WPG, true>(job, n_tiles, cus, s) : launch_dense_pl<W, WPG, false>(job, n_tiles, cus, s);
}

// BF16: all four hidden layers resident (4 W^2 x 2 B = 128 KB at width 128), and with PL
// the weight set's small parameters after them (25 KB at width 128).
template <int W, int WPG, bool PL>
hipError_t launch_dense_res_pl(const FieldJob& job, int n_tiles, int cus, hipStream_t s) {
  constexpr int lds = 4 * HiddenLayer<W, true>::kBytes + (PL ? ParamsLds<W>::kFloats * 4 : 0);
  static_assert(lds <= 160 * 1024, "resident weights must fit in LDS");
  auto k = fields_dense_res_kernel<W, WPG, PL>;
  static int per_cu = 0;
  int grid = 0;
  const hipError_t e = decode_grid(k, WPG, lds, cus, &per_cu, &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WPG), lds, s, job, n_tiles);
  return hipGetLastError();
}

template <int W, int WPG>
hipError_t launch_dense_res(const FieldJob& job, int n_tiles, int cus, hipStream_t s) {
  const bool pl = job.zrows == nullptr && job.jvp == 0 && job.r <= kMaxR && job.d <= 9;
  return pl ? launch_dense_res_pl<W, WPG, true>(job, n_tiles, cus, s)
            : launch_dense_res_pl<W, WPG, false>(job, n_tiles, cus, s);
}

template <int W>
hipError_t launch_decode_width(bool bf16, const FieldJob& job, int n_tiles, int cus, hipStream_t s) {
  if (bf16) return launch_dense_res<W, kDenseResWpg>(job, n_tiles, cus, s);
  return launch_dense<W, kDenseWpg>(job, n_tiles, cus, s);
}

}  // namespace

int fields_max_tangents(int width, bool bf16) {
  if (width == 64) return bf16 ? kTcBf16W64 : kTcF32W64;
  return bf16 ? kTcBf16W128 : kTcF32W128;
}

int fields_group_points(int tc) { return kTile16 * (tc > 0 ? Wpg<1>::value : Wpg<0>::value); }

int fields_team_points(int nt) { return kTile16 * team_tiles(nt); }

bool fields_team_jacobian(int width, bool bf16) { return !bf16 && width / 16 == Wpg<1>::value; }

hipError_t launch_fields_table(int width, bool bf16, int tc, int kinds, const FieldJob* jobs,
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
    if (!bf16 && full && (kinds & kTableTeam)) {
#define NSF_TEAM(K) launch_table<128, kTcF32W128, false, K>(jobs, groups, n_groups, claim, grid, s)
      switch (kinds & (kTableTangents | kTableTeamOne)) {
        case 0: return NSF_TEAM(kTableTeam);
        case kTableTangents: return NSF_TEAM(kTableTeam | kTableTangents);
        case kTableTeamOne: return NSF_TEAM(kTableTeam | kTableTeamOne);
        default: return NSF_TEAM(kTableTeam | kTableTeamOne | kTableTangents);
      }
#undef NSF_TEAM
    }
    if (!bf16) return full ? NSF_TABLE(128, kTcF32W128, false) : NSF_TABLE(128, 0, false);
    return full ? NSF_TABLE(128, kTcBf16W128, true) : NSF_TABLE(128, 0, true);
  }
#undef NSF_TABLE
  return hipErrorInvalidValue;
}

int fields_table_blocks_per_cu(int width, bool bf16, int tc) {
  // registers bound residency to one workgroup per CU (two waves per SIMD with tangents,
  // four for the primal), before LDS (two hidden layers, at most 128 KB) does
  (void)width;
  (void)bf16;
  (void)tc;
  return 1;
}

__global__ void reset_counters_kernel(int32_t* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

hipError_t launch_reset_counters(int32_t* c, int n, hipStream_t s) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, c, n);
  return hipGetLastError();
}

hipError_t launch_fields_dense(int width, bool bf16, const FieldJob& job, int n_points,
                               hipStream_t s, bool beside) {
  if (n_points <= 0) return hipSuccess;
  static int dev_cus = 0;
  if (dev_cus == 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  // beside the step's own kernels: three eighths of the CUs stay free for them (sharing a
  // CU with a decode workgroup, they measured no faster than waiting). Of the shares
  // measured (from 1/8 to 1/2 of the CUs free), 3/8 gave the fastest pipelined steps in
  // both precisions taken together.
  const int cus = beside ? dev_cus - dev_cus * 3 / 8 : dev_cus;
  const int tiles = (n_points + kTile16 - 1) / kTile16;
  if (width == 64) return launch_decode_width<64>(bf16, job, tiles, cus, s);
  if (width == 128) return launch_decode_width<128>(bf16, job, tiles, cus, s);
  return hipErrorInvalidValue;
}

template <int W>
hipError_t launch_decode_table_res(const FieldJob* jobs, const FieldTile* groups, const int32_t* n_groups, int grid,
                                   hipStream_t s) {
  constexpr int lds = 4 * HiddenLayer<W, true>::kBytes + ParamsLds<W>::kFloats * 4;
  static_assert(lds <= 160 * 1024, "four BF16 layers and the parameters must fit in LDS");
  auto k = fields_decode_table_res_kernel<W, kDenseResWpg>;
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * kDenseResWpg), lds, s, jobs, groups, n_groups);
  return hipGetLastError();
}

hipError_t launch_fields_decode_table(int width, const FieldJob* jobs, const FieldTile* groups,
                                      const int32_t* n_groups, int cus, hipStream_t s) {
  if (cus <= 0) return hipSuccess;
  if (width == 64) return launch_decode_table_res<64>(jobs, groups, n_groups, cus, s);
  if (width == 128) return launch_decode_table_res<128>(jobs, groups, n_groups, cus, s);
  return hipErrorInvalidValue;
}

}  // namespace nsf
