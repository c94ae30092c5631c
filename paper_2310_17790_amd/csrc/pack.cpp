// Host-side packing of one field's row-major FP32 parameters into the operand orders the
// MFMA field kernels read (see fields.hip for the register mapping).
//
// Scaled pre-activations. The kernels carry a' = log2(e) a instead of a, so that ELU needs
// exp2 (one hardware instruction) with no multiply: layer 1's weights and bias and the
// hidden biases are packed times log2(e); the hidden layers then see h' = ELU(a) / ln 2,
// which their unscaled weights map to log2(e) (W h + b) again, and the output layer's
// weights are packed times ln 2. Each scaled value is rounded to FP32 once.
#include "pack.h"

#include <cstring>

namespace nsf {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
static inline float scaled(float w, double f) { return (float)((double)w * f); }

uint16_t float_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

size_t mlp_param_count(int r, int width, int d) {
  const size_t w = width;
  return w * (3 + r) + w + 4 * (w * w + w) + (size_t)d * w + d;
}

MlpView view_master(const float* p, int r, int width, int d) {
  MlpView v;
  const size_t w = width;
  v.W1 = p;
  v.b1 = v.W1 + w * (3 + r);
  const float* q = v.b1 + w;
  for (int k = 0; k < 4; ++k) {
    v.Wh[k] = q;
    v.bh[k] = q + w * w;
    q = v.bh[k] + w;
  }
  v.W6 = q;
  v.b6 = q + (size_t)d * w;
  return v;
}

PackSizes pack_sizes(int r, int width, int d) {
  PackSizes s;
  const int MB = width / 32;
  const int K1s = (r + 5) / 2;
  s.w1p = (size_t)MB * K1s * 64;
  s.whp = (size_t)4 * width * width;
  s.whb = (size_t)4 * width * width;  // bf16 elements
  s.bhp = (size_t)4 * width;
  s.w6p = (size_t)d * width;
  s.b6 = (size_t)d;
  s.w1q = (size_t)(width / 16) * ((r + 7) / 4) * 64;
  s.bhq = (size_t)4 * width;
  s.w6q = (size_t)d * width;
  s.w1zt = (size_t)((r + 15) / 16) * 16 * width;
  return s;
}

// A operands of an M x K FP32 matrix A(m, k) for v_mfma_f32_16x16x4_f32, read by the
// kernels one K-step pair at a time: [ceil(M/16)][K/8][64][2]. Output block mb, pair hs,
// lane l hold row 16 mb + l % 16 and inputs 16 (hs / 2) + 4 (l / 16) + 2 (hs % 2) + j, i.e.
// K-steps 2 hs + j read the accumulator registers 2 (hs % 2) + j of M-block hs / 2 that lane
// group l / 16 holds in the layer before. Rows past M are zero.
template <class F>
static void pack_a_f32(F A, int M, int K, float* dst) {
  const int MB = (M + 15) / 16;
  for (int mb = 0; mb < MB; ++mb)
    for (int hs = 0; hs < K / 8; ++hs)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 2; ++j) {
          const int m = 16 * mb + (l & 15), n = 16 * (hs >> 1) + 4 * (l >> 4) + 2 * (hs & 1) + j;
          dst[(((size_t)mb * (K / 8) + hs) * 64 + l) * 2 + j] = m < M ? A(m, n) : 0.f;
        }
}

// The same for v_mfma_f32_16x16x32_bf16: [M/16][K/32][64][8]; K-step s, lane l hold row
// 16 mb + l % 16 and inputs 16 (2s + e / 4) + 4 (l / 16) + e % 4 (M-blocks 2s and 2s + 1 of
// the layer before).
template <class F>
static void pack_a_bf16(F A, int M, int K, uint16_t* dst) {
  for (int mb = 0; mb < M / 16; ++mb)
    for (int s = 0; s < K / 32; ++s)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          const int m = 16 * mb + (l & 15), n = 16 * (2 * s + (e >> 2)) + 4 * (l >> 4) + (e & 3);
          dst[(((size_t)mb * (K / 32) + s) * 64 + l) * 8 + e] = float_to_bf16(A(m, n));
        }
}

void pack_field(const float* master, int r, int width, int d, const PackOut& o) {
  const MlpView v = view_master(master, r, width, d);
  const int W = width, MQ = W / 16, K1q = (r + 7) / 4, in1 = 3 + r;
  // layer 1 (16x16x4 A operands) with the bias as input row 3 + r: lane l holds row
  // 16 mb + l % 16, input 4 s4 + l / 16
  for (int mb = 0; mb < MQ; ++mb)
    for (int s4 = 0; s4 < K1q; ++s4)
      for (int l = 0; l < 64; ++l) {
        const int m = 16 * mb + (l & 15), k = 4 * s4 + (l >> 4);
        float val = 0.f;
        if (k < in1) val = scaled(v.W1[(size_t)m * in1 + k], kLog2e);
        else if (k == in1) val = scaled(v.b1[m], kLog2e);
        o.w1q[((size_t)mb * K1q + s4) * 64 + l] = val;
      }
  // reverse mode: dJ/dz = W1_z^T delta_1, the latent columns of layer 1 as an r x W matrix
  if (o.w1zt)
    pack_a_f32([&](int j, int m) { return scaled(v.W1[(size_t)m * in1 + 3 + j], kLog2e); }, r, W, o.w1zt);
  for (int kk = 0; kk < 4; ++kk) {
    const float* Wk = v.Wh[kk];
    auto fwd = [&](int m, int n) { return Wk[(size_t)m * W + n]; };
    auto tr = [&](int m, int n) { return Wk[(size_t)n * W + m]; };
    pack_a_f32(fwd, W, W, o.whp + (size_t)kk * W * W);
    pack_a_bf16(fwd, W, W, o.whb + (size_t)kk * W * W);
    if (o.whpt) pack_a_f32(tr, W, W, o.whpt + (size_t)kk * W * W);
    if (o.whbt) pack_a_bf16(tr, W, W, o.whbt + (size_t)kk * W * W);
    for (int n = 0; n < W; ++n) o.bhq[(size_t)kk * W + n] = scaled(v.bh[kk][n], kLog2e);
  }
  for (int oo = 0; oo < d; ++oo) {
    for (int n = 0; n < W; ++n) o.w6q[(size_t)oo * W + n] = scaled(v.W6[(size_t)oo * W + n], kLn2);
    o.b6[oo] = v.b6[oo];
  }
}

}  // namespace nsf
