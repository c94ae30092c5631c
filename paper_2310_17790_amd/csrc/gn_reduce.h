// Per-chunk reduction of the Gauss-Newton normal equations (paper Sec. 5.3), shared by the
// fused G2P kernel (iteration 0) and the reduction kernel of later iterations.
//
// A chunk is kGnChunk consecutive sample points. With its Jacobian rows J (3 r x chunk)
// and residuals R (3 x chunk) staged in LDS, entry e of the packed system is
//   e <  r(r+1)/2: H[j][k] = sum_{c, p} J[c r + j][p] J[c r + k][p]   (j <= k)
//   e >= r(r+1)/2: b[j]    = sum_{c, p} J[c r + j][p] R[c][p]
// Thread (e, g) of the block sums entry e over the columns g, g + G, ... (G = threads / E
// column groups), in FP64 from the FP32 Jacobian; the G groups are then added in a fixed
// order and the chunk's partial is stored at gn_part[chunk][e].
#pragma once

#include "nsf_dev.h"

namespace nsf {

// The chunk's LDS, carved from the kernel's dynamic LDS: R [3][kGnChunk] and the group
// sums part[NT] (FP64), then the Jacobian rows Jl [3 r_cap][kGnChunk + 1] (FP32), where
// r_cap bounds the latent size of every sim the launch serves.
template <int NT>
struct GnChunkLds {
  double* R;
  double* part;
  float* Jl;
  __device__ explicit GnChunkLds(char* lds)
      : R(reinterpret_cast<double*>(lds)),
        part(reinterpret_cast<double*>(lds) + 3 * kGnChunk),
        Jl(reinterpret_cast<float*>(lds + (3 * kGnChunk + NT) * sizeof(double))) {}
  __device__ float* row(int i) const { return Jl + i * (kGnChunk + 1); }
  __device__ double& res(int c, int col) const { return R[c * kGnChunk + col]; }
};

// Dynamic LDS bytes of a chunk kernel with NT threads serving latents up to r_cap.
constexpr int gn_chunk_lds_bytes(int nt, int r_cap) {
  return (3 * kGnChunk + nt) * (int)sizeof(double) + 3 * r_cap * (kGnChunk + 1) * (int)sizeof(float);
}

__device__ __forceinline__ int gn_entries_dev(int r) { return r * (r + 1) / 2 + r; }

// Entry e of the packed system: e < r(r+1)/2 -> H[j][k], j <= k (row-major upper
// triangle); else b[e - r(r+1)/2].
__device__ __forceinline__ void gn_decode_entry(int e, int r, int& j, int& k, bool& is_b) {
  const int nh = r * (r + 1) / 2;
  if (e >= nh) { is_b = true; j = e - nh; k = 0; return; }
  is_b = false;
  int row = 0, start = 0;
  while (e >= start + (r - row)) { start += r - row; ++row; }
  j = row;
  k = row + (e - start);
}

// Stage the chunk's Jacobian rows (zero beyond the last sample point). Loads are issued
// in batches of U per thread before any is stored, so their latencies overlap.
template <int NT, int U = 8>
__device__ __forceinline__ void gn_stage_jacobian(const SimDev& S, const float* J, int p0, int cnt,
                                                  const GnChunkLds<NT>& sh) {
  const int r = S.r, ns = S.n_samp;
  const int total = 3 * r * kGnChunk;
  for (int e0 = threadIdx.x; e0 < total; e0 += NT * U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT;
      const int row = e / kGnChunk, col = e % kGnChunk;
      v[u] = (e < total && col < cnt) ? J[(int64_t)row * ns + p0 + col] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT;
      if (e < total) sh.row(e / kGnChunk)[e % kGnChunk] = v[u];
    }
  }
}

// Reduce the staged chunk into gn_part (Jl and R must be staged and visible).
template <int NT>
__device__ __forceinline__ void gn_reduce_chunk(const SimDev& S, int p0, const GnChunkLds<NT>& sh) {
  const int r = S.r, tid = threadIdx.x;
  const int E = gn_entries_dev(r);
  const int G = E >= NT ? 1 : NT / E;   // column groups per entry
  double* out = S.gn_part + (int64_t)(p0 / kGnChunk) * E;
  for (int e0 = 0; e0 < E; e0 += NT / G) {
    const int e = e0 + tid % (NT / G);
    const int g = tid / (NT / G);
    double acc = 0.0;
    if (e < E && g < G) {
      int j, k;
      bool is_b;
      gn_decode_entry(e, r, j, k, is_b);
      for (int c = 0; c < 3; ++c) {
        const float* a = sh.row(c * r + j);
        if (is_b) {
          for (int col = g; col < kGnChunk; col += G) acc += (double)a[col] * sh.res(c, col);
        } else {
          const float* bb = sh.row(c * r + k);
          for (int col = g; col < kGnChunk; col += G) acc += (double)a[col] * (double)bb[col];
        }
      }
    }
    sh.part[tid] = acc;
    __syncthreads();
    if (tid < NT / G && e0 + tid < E) {
      double s = 0.0;
      for (int gg = 0; gg < G; ++gg) s += sh.part[gg * (NT / G) + tid];
      out[e0 + tid] = s;
    }
    __syncthreads();
  }
}

}  // namespace nsf
