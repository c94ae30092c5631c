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
  return s;
}

void pack_field(const float* master, int r, int width, int d, float* w1p, float* whp,
                uint16_t* whb, float* bhp, float* w6p, float* b6) {
  const MlpView v = view_master(master, r, width, d);
  const int W = width, MB = W / 32, K1s = (r + 5) / 2, in1 = 3 + r;
  // layer 1 with the bias as input row 3 + r
  for (int mb = 0; mb < MB; ++mb)
    for (int s2 = 0; s2 < K1s; ++s2)
      for (int l = 0; l < 64; ++l) {
        const int m = 32 * mb + (l & 31), k = 2 * s2 + (l >> 5);
        float val = 0.f;
        if (k < in1) val = scaled(v.W1[(size_t)m * in1 + k], kLog2e);
        else if (k == in1) val = scaled(v.b1[m], kLog2e);
        w1p[((size_t)mb * K1s + s2) * 64 + l] = val;
      }
  for (int kk = 0; kk < 4; ++kk) {
    const float* Wk = v.Wh[kk];
    // FP32 A operands: [MB][W/8][64][4], K-step s = 4 sg + j consumes neuron
    // acc_neuron(s / 16, s % 16, lane half) of the previous layer.
    float* dst = whp + (size_t)kk * W * W;
    for (int mb = 0; mb < MB; ++mb)
      for (int sg = 0; sg < W / 8; ++sg)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 4; ++j) {
            const int s = 4 * sg + j, m = 32 * mb + (l & 31);
            const int n = acc_neuron_h(s / 16, s % 16, l >> 5);
            dst[(((size_t)mb * (W / 8) + sg) * 64 + l) * 4 + j] = Wk[(size_t)m * W + n];
          }
    // BF16 A operands: [MB][W/16][64][8], K-step s = 2 mb_in + q holds the lane half's
    // registers 8q .. 8q + 7 of M-block mb_in.
    uint16_t* dstb = whb + (size_t)kk * W * W;
    for (int mb = 0; mb < MB; ++mb)
      for (int s = 0; s < W / 16; ++s)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 8; ++j) {
            const int mb_in = s / 2, q = s % 2, m = 32 * mb + (l & 31);
            const int n = acc_neuron_h(mb_in, 8 * q + j, l >> 5);
            dstb[(((size_t)mb * (W / 16) + s) * 64 + l) * 8 + j] = float_to_bf16(Wk[(size_t)m * W + n]);
          }
    // biases in accumulator order [2][W/2]
    for (int h = 0; h < 2; ++h)
      for (int s = 0; s < W / 2; ++s)
        bhp[(size_t)kk * W + h * (W / 2) + s] = scaled(v.bh[kk][acc_neuron_h(s / 16, s % 16, h)], kLog2e);
  }
  for (int o = 0; o < d; ++o) {
    for (int h = 0; h < 2; ++h)
      for (int s = 0; s < W / 2; ++s)
        w6p[((size_t)o * 2 + h) * (W / 2) + s] = scaled(v.W6[(size_t)o * W + acc_neuron_h(s / 16, s % 16, h)], kLn2);
    b6[o] = v.b6[o];
  }
}

}  // namespace nsf
