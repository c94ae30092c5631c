// Gauss-Newton network inversion (paper Sec. 5.3): z_{n+1} = argmin_z sum_{p in S}
// || g(X_p, z) - x_p^{n+1} ||^2, iterated from z_n.
//
// Iterate k has residual r_p = u(X_p, z^(k)) - u^n_p - dt v^{n+1}_p (3 |S| entries; at
// k = 0 the first two terms are the same value, so r = -dt v) and Jacobian J (3|S| x r)
// from the field kernel. The step solves (J^T J) delta = -J^T r by Cholesky and sets
// z^(k+1) = z^(k) + delta. Everything from the residual on is FP64: J and u enter as the
// FP32 values the field kernel stored, widened.
//
// gn_reduce: one block per 128 sample points stages J and r in LDS and writes its
//   partial H (upper triangle, r(r+1)/2 entries) and b (r entries) in FP64.
// gn_solve: one 64-thread block per simulation sums the partials in a fixed order
//   (deterministic), factors H with a column-parallel Cholesky in LDS, solves, and
//   updates the latent; the last iteration also shifts z_{n-1} <- z_n <- z_{n+1} and
//   advances the step counter. A pivot <= 0 raises the SINGULAR flag and a non-finite
//   system or latent the NONFINITE flag; the latent is then left unchanged.
#include "nsf_dev.h"

namespace nsf {
namespace {

// Entry e of the packed system: e < r(r+1)/2 -> H[j][k], j <= k (row-major upper
// triangle); else b[e - r(r+1)/2].
__device__ __forceinline__ void decode_entry(int e, int r, int& j, int& k, bool& is_b) {
  const int nh = r * (r + 1) / 2;
  if (e >= nh) { is_b = true; j = e - nh; k = 0; return; }
  is_b = false;
  int row = 0, start = 0;
  while (e >= start + (r - row)) { start += r - row; ++row; }
  j = row;
  k = row + (e - start);
}

__global__ __launch_bounds__(256) void gn_reduce_kernel(const SimDev* __restrict__ sims,
                                                        const BlockWork* __restrict__ work,
                                                        const int32_t* __restrict__ n_work,
                                                        int iter) {
  __shared__ float Jl[3 * kMaxR][kGnChunk + 1];
  __shared__ double R[3][kGnChunk];
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    if (iter >= S.gn_iters) continue;
    const int r = S.r, ns = S.n_samp, p0 = wk.p0;
    const int cnt = min(kGnChunk, ns - p0);
    const float* J = iter == 0 ? S.J : S.J2;
    for (int e = threadIdx.x; e < 3 * r * kGnChunk; e += blockDim.x) {
      const int row = e / kGnChunk, col = e % kGnChunk;
      Jl[row][col] = col < cnt ? J[(int64_t)row * ns + p0 + col] : 0.f;
    }
    for (int e = threadIdx.x; e < 3 * kGnChunk; e += blockDim.x) {
      const int c = e / kGnChunk, col = e % kGnChunk;
      double rv = 0.0;
      if (col < cnt) {
        const int p = p0 + col;
        rv = -S.dt_d * (double)S.vnew[c * ns + p];
        if (iter > 0) rv += (double)S.u_gn[c * ns + p] - (double)S.u_n[c * S.n_int + p];
      }
      R[c][col] = rv;
    }
    __syncthreads();
    const int E = r * (r + 1) / 2 + r;
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
      int j, k;
      bool is_b;
      decode_entry(e, r, j, k, is_b);
      double acc = 0.0;
      for (int c = 0; c < 3; ++c) {
        const float* a = Jl[c * r + j];
        if (is_b) {
          for (int col = 0; col < cnt; ++col) acc += (double)a[col] * R[c][col];
        } else {
          const float* bb = Jl[c * r + k];
          for (int col = 0; col < cnt; ++col) acc += (double)a[col] * (double)bb[col];
        }
      }
      S.gn_part[(int64_t)(p0 / kGnChunk) * E + e] = acc;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void gn_solve_kernel(const SimDev* __restrict__ sims,
                                                      const int32_t* __restrict__ n_sims,
                                                      int iter) {
  __shared__ double H[kMaxR][kMaxR + 1];
  __shared__ double y[kMaxR];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int total = *n_sims;
  for (int s = blockIdx.x; s < total; s += gridDim.x) {
    const SimDev& S = sims[s];
    if (iter >= S.gn_iters) continue;
    const int r = S.r;
    const int E = r * (r + 1) / 2 + r;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int e = tid; e < E; e += blockDim.x) {
      double acc = 0.0;
      for (int c = 0; c < S.n_gn_chunks; ++c) acc += S.gn_part[(int64_t)c * E + e];
      int j, k;
      bool is_b;
      decode_entry(e, r, j, k, is_b);
      if (!isfinite(acc)) atomicOr(&bad, 2);
      if (is_b) {
        y[j] = -acc;  // right-hand side -J^T r
      } else {
        H[j][k] = acc;
        H[k][j] = acc;
      }
    }
    __syncthreads();
    // Cholesky H = L L^T, right-looking, L overwrites the lower triangle.
    for (int j = 0; j < r && bad == 0; ++j) {
      if (tid == 0) {
        const double dj = H[j][j];
        if (!(dj > 0.0)) bad = 1;
        else H[j][j] = sqrt(dj);
      }
      __syncthreads();
      if (bad) break;
      const double ljj = H[j][j];
      for (int i = j + 1 + tid; i < r; i += blockDim.x) H[i][j] /= ljj;
      __syncthreads();
      const int m = r - j - 1;
      for (int e = tid; e < m * m; e += blockDim.x) {
        const int i = j + 1 + e / m, k = j + 1 + e % m;
        if (k <= i) H[i][k] -= H[i][j] * H[k][j];
      }
      __syncthreads();
    }
    __syncthreads();
    if (bad == 0) {
      // forward substitution L w = -b, then back substitution L^T delta = w (in y)
      for (int j = 0; j < r; ++j) {
        if (tid == 0) y[j] /= H[j][j];
        __syncthreads();
        for (int i = j + 1 + tid; i < r; i += blockDim.x) y[i] -= H[i][j] * y[j];
        __syncthreads();
      }
      for (int j = r - 1; j >= 0; --j) {
        if (tid == 0) y[j] /= H[j][j];
        __syncthreads();
        for (int i = tid; i < j; i += blockDim.x) y[i] -= H[j][i] * y[j];
        __syncthreads();
      }
    }
    const bool final_iter = (iter == S.gn_iters - 1);
    double* zp = S.z;
    double* zc = S.z + r;
    double* zi = S.z + 2 * r;
    if (tid == 0 && bad) atomicOr(S.flags, (bad & 2) ? FLAG_NONFINITE : FLAG_SINGULAR);
    for (int j = tid; j < r; j += blockDim.x) {
      const double base = (iter == 0) ? zc[j] : zi[j];
      double zn = bad ? base : base + y[j];
      if (!isfinite(zn)) atomicOr(S.flags, FLAG_NONFINITE);
      if (final_iter) {
        zp[j] = zc[j];
        zc[j] = zn;
      } else {
        zi[j] = zn;
      }
    }
    if (final_iter && tid == 0) *S.step += 1;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_gn_reduce(const SimDev* sims, const BlockWork* work, const int32_t* n_work,
                            int iter, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(gn_reduce_kernel, dim3(grid), dim3(256), 0, s, sims, work, n_work, iter);
  return hipGetLastError();
}

hipError_t launch_gn_solve(const SimDev* sims, const int32_t* n_sims, int iter, int grid,
                           hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(gn_solve_kernel, dim3(grid), dim3(64), 0, s, sims, n_sims, iter);
  return hipGetLastError();
}

}  // namespace nsf
