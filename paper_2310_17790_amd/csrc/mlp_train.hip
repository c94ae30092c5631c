// Field fitting entry points (forward with saved activations, hand-written backward).
#include <hip/hip_runtime.h>

#include "nsf.h"
#include "nsf_dev.h"
#include "pack.h"

extern "C" {

size_t nsf_mlp_param_count(int32_t r, int32_t width, int32_t d) {
  return nsf::mlp_param_count(r, width, d);
}

size_t nsf_mlp_saved_floats(int32_t width, int64_t n) { return (size_t)5 * width * n; }

size_t nsf_mlp_workspace_bytes(const nsf_mlp*, int64_t) { return 0; }

nsf_status nsf_mlp_forward(const nsf_mlp*, const float*, const float*, int64_t, float*, float*,
                           void*, size_t, void*) {
  return NSF_EINVAL;
}

nsf_status nsf_mlp_backward(const nsf_mlp*, const float*, const float*, int64_t, const float*,
                            const float*, float*, float*, void*, size_t, void*) {
  return NSF_EINVAL;
}

}  // extern "C"
