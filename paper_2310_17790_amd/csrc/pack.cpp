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

static inline int acc_neuron_h(int mb, int i, int h) { return 32 * mb + 8 * (i >> 2) + 4 * h + (i & 3); }

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
  return s;
}

void pack_field(const float* master, int r, int width, int d, const PackOut& o) {
  const MlpView v = view_master(master, r, width, d);
  const int W = width, MB = W / 32, K1s = (r + 5) / 2, in1 = 3 + r;
  auto layer1 = [&](int m, int k) -> float {   // with the bias as input row 3 + r
    if (k < in1) return scaled(v.W1[(size_t)m * in1 + k], kLog2e);
    if (k == in1) return scaled(v.b1[m], kLog2e);
    return 0.f;
  };
  // BF16 precision, 32x32x2 layer 1: lane l holds row 32 mb + l % 32, input 2 s2 + l / 32
  for (int mb = 0; mb < MB; ++mb)
    for (int s2 = 0; s2 < K1s; ++s2)
      for (int l = 0; l < 64; ++l)
        o.w1p[((size_t)mb * K1s + s2) * 64 + l] = layer1(32 * mb + (l & 31), 2 * s2 + (l >> 5));
  // FP32 precision, 16x16x4 layer 1: lane l holds row 16 mb + l % 16, input 4 s4 + l / 16
  const int MQ = W / 16, K1q = (r + 7) / 4;
  for (int mb = 0; mb < MQ; ++mb)
    for (int s4 = 0; s4 < K1q; ++s4)
      for (int l = 0; l < 64; ++l)
        o.w1q[((size_t)mb * K1q + s4) * 64 + l] = layer1(16 * mb + (l & 15), 4 * s4 + (l >> 4));
  for (int kk = 0; kk < 4; ++kk) {
    const float* Wk = v.Wh[kk];
    // FP32 A operands [W/16][W/16][64][4]: output block mb, K-group sg, lane l: row
    // 16 mb + l % 16, inputs 16 sg + 4 (l / 16) + j (the accumulator registers of lane group
    // l / 16 in the previous layer).
    float* dst = o.whp + (size_t)kk * W * W;
    for (int mb = 0; mb < MQ; ++mb)
      for (int sg = 0; sg < W / 16; ++sg)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 4; ++j) {
            const int m = 16 * mb + (l & 15), n = 16 * sg + 4 * (l >> 4) + j;
            dst[(((size_t)mb * (W / 16) + sg) * 64 + l) * 4 + j] = Wk[(size_t)m * W + n];
          }
    // BF16 A operands: [MB][W/16][64][8], K-step s = 2 mb_in + q holds the lane half's
    // registers 8q .. 8q + 7 of M-block mb_in.
    uint16_t* dstb = o.whb + (size_t)kk * W * W;
    for (int mb = 0; mb < MB; ++mb)
      for (int s = 0; s < W / 16; ++s)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 8; ++j) {
            const int mb_in = s / 2, q = s % 2, m = 32 * mb + (l & 31);
            const int n = acc_neuron_h(mb_in, 8 * q + j, l >> 5);
            dstb[(((size_t)mb * (W / 16) + s) * 64 + l) * 8 + j] = float_to_bf16(Wk[(size_t)m * W + n]);
          }
    // biases: in 32x32 accumulator order [2][W/2] (BF16), plain (FP32)
    for (int h = 0; h < 2; ++h)
      for (int s = 0; s < W / 2; ++s)
        o.bhp[(size_t)kk * W + h * (W / 2) + s] = scaled(v.bh[kk][acc_neuron_h(s / 16, s % 16, h)], kLog2e);
    for (int n = 0; n < W; ++n) o.bhq[(size_t)kk * W + n] = scaled(v.bh[kk][n], kLog2e);
  }
  for (int oo = 0; oo < d; ++oo) {
    for (int h = 0; h < 2; ++h)
      for (int s = 0; s < W / 2; ++s)
        o.w6p[((size_t)oo * 2 + h) * (W / 2) + s] = scaled(v.W6[(size_t)oo * W + acc_neuron_h(s / 16, s % 16, h)], kLn2);
    for (int n = 0; n < W; ++n) o.w6q[(size_t)oo * W + n] = scaled(v.W6[(size_t)oo * W + n], kLn2);
    o.b6[oo] = v.b6[oo];
  }
}

}  // namespace nsf
