// Host-side weight packing for the MFMA field kernels.
#pragma once

#include <cstddef>
#include <cstdint>

namespace nsf {

// Pointers into one field's row-major parameter block (layout of nsf_sim_desc.weights).
struct MlpView {
  const float* W1;
  const float* b1;
  const float* Wh[4];
  const float* bh[4];
  const float* W6;
  const float* b6;
};

struct PackSizes {
  size_t w1p, whp, whb, bhp, w6p, b6;  // element counts (whb in bf16 elements)
  size_t w1q, bhq, w6q;
  size_t w1zt;                         // layer 1's latent columns, transposed (reverse mode)
};

// The packed arrays of one field (host or device buffers of PackSizes elements). whpt and
// whbt are the transposed hidden layers (sizes whp, whb) of the reverse-mode Jacobian.
struct PackOut {
  float* whp; uint16_t* whb; float* b6; float* w1q; float* bhq; float* w6q;
  float* whpt; uint16_t* whbt; float* w1zt;
};

size_t mlp_param_count(int r, int width, int d);
MlpView view_master(const float* p, int r, int width, int d);
PackSizes pack_sizes(int r, int width, int d);
uint16_t float_to_bf16(float f);
void pack_field(const float* master, int r, int width, int d, const PackOut& out);

}  // namespace nsf
