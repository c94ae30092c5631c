// Gauss-Newton network inversion (paper Sec. 5.3): z_{n+1} = argmin_z sum_{p in S}
// || g(X_p, z) - x_p^{n+1} ||^2, iterated from z_n.
//
// Iterate k has residual r_p = u(X_p, z^(k)) - u^n_p - dt v^{n+1}_p (3 |S| entries; at
// k = 0 the first two terms are the same value, so r = -dt v) and Jacobian J (3|S| x r)
// from the field kernel. The step solves (J^T J) delta = -J^T r by Cholesky and sets
// z^(k+1) = z^(k) + delta. Optional damping lambda (Levenberg-Marquardt with Marquardt's
// scaling) solves (J^T J + lambda diag(J^T J)) delta = -J^T r instead. Everything from
// the residual on is FP64: J and u enter as the FP32 values the field kernel stored,
// widened (a product of two FP32 values is exact in FP64).
//
// Two launches per iteration.
//  - the chunk reduction (gn_reduce.h): each block stages 128 sample points of J and r in
//    LDS and stores its partial H (upper triangle) and b. Iteration 0 runs it inside the
//    G2P kernel (mpm.hip), where r = -dt v is at hand; later iterations in
//    gn_partial_kernel, after the field kernel evaluated u and J at the iterate.
//  - gn_solve_kernel: one workgroup per simulation adds the partials in a fixed order
//    (deterministic); up to kSerialR latents one lane factors H by Cholesky and solves in
//    its registers, above that the first wave runs a column-parallel Cholesky in LDS; then
//    it updates the latent; the last iteration also shifts z_{n-1} <- z_n <- z_{n+1} and
//    advances the step counter.
// The kernel boundary publishes the partials to the solving block on whichever XCD it
// runs (a device-scope release inside one kernel would write back every block's L2).
// A pivot <= 0 raises the SINGULAR flag and a non-finite system or latent the NONFINITE
// flag; the latent is then left unchanged.
#include "gn_reduce.h"

namespace nsf {
namespace {

// The chunk partials are summed by the whole workgroup (more loads in flight); the solve
// itself runs in wave 0 (in lane 0's registers up to kSerialR latents, else over the wave,
// synchronised at wave scope).
constexpr int kSolveThreads = 1024;
constexpr int kSerialR = 6;

// Lane l's value of v in every lane (l wave-uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The latent values the update needs, loaded by lane j < r of the solving wave before
// the partials are summed, so their latency overlaps that of the sums: the value the update
// starts from (z_n at iteration 0, else the iterate) and z_n.
struct GnLatent {
  double base, zc;
};

__device__ __forceinline__ GnLatent load_latent(const SimDev& S, int iter) {
  GnLatent L{0.0, 0.0};
  const int j = threadIdx.x, r = S.r;
  if (j < r) {
    L.zc = S.z[r + j];
    L.base = iter == 0 ? L.zc : S.z[2 * r + j];
  }
  return L;
}

// Factor and solve in one wave (lane = threadIdx.x < 64), then update the latent.
// Cholesky H = L L^T is right-looking, one column per round: every lane reads the pivot
// d and forms sqrt(d) and its reciprocal itself; each lane scales its row's entry of the
// column and, once the column is visible, subtracts L[i][j] L[k][j] from its row of the
// trailing matrix (two wave synchronisations per column, no index arithmetic per entry).
// The substitutions multiply by the stored reciprocal pivots idg. H, y and idg live in
// LDS; *bad (LDS) is 2 if the summed system is not finite.
// Small systems (r <= kSerialR): one lane factors H = L L^T column by column
// (left-looking: L[i][j] = (H[i][j] - sum_{k<j} L[i][k] L[j][k]) / L[j][j]) and runs both
// substitutions in its registers, with no synchronisation; the solution goes to y.
// Returns 1 for a pivot <= 0.
__device__ __forceinline__ int solve_serial(const double (*H)[kMaxR + 1], double* y, int r) {
  double L[kSerialR][kSerialR];
  double il[kSerialR], w[kSerialR];
#pragma unroll
  for (int i = 0; i < kSerialR; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) L[i][j] = i < r ? H[i][j] : 0.0;
#pragma unroll
  for (int j = 0; j < kSerialR; ++j) {
    if (j >= r) break;
    double d = L[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) return 1;
    const double l = sqrt(d);
    il[j] = 1.0 / l;
    L[j][j] = l;
#pragma unroll
    for (int i = j + 1; i < kSerialR; ++i) {
      if (i >= r) break;
      double t = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t * il[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kSerialR; ++j) {   // L w = -b
    if (j >= r) break;
    double t = y[j];
#pragma unroll
    for (int k = 0; k < j; ++k) t -= L[j][k] * w[k];
    w[j] = t * il[j];
  }
#pragma unroll
  for (int j = kSerialR - 1; j >= 0; --j) {   // L^T delta = w
    if (j >= r) continue;
    double t = w[j];
#pragma unroll
    for (int k = j + 1; k < kSerialR; ++k)
      if (k < r) t -= L[k][j] * w[k];
    w[j] = t * il[j];
  }
#pragma unroll
  for (int j = 0; j < kSerialR; ++j)
    if (j < r) y[j] = w[j];
  return 0;
}

__device__ void solve_and_update(const SimDev& S, int iter, double (*H)[kMaxR + 1], double* y,
                                 double* idg, const int* bad, const GnLatent& zl) {
  const int r = S.r, tid = threadIdx.x;
  int b = *bad;
  if (b == 0 && r <= kSerialR) {
    int bs = 0;
    if (tid == 0) {
      bs = solve_serial(H, y, r);
      idg[0] = (double)bs;   // hand the pivot test to the wave through LDS
    }
    wave_sync();
    b = idg[0] != 0.0 ? 1 : 0;
  } else if (b == 0) {
    // lane t owns row j + 1 + t of the trailing matrix (r <= kMaxR <= 64): it scales its
    // entry of column j, then (after the column is visible) updates its row
    for (int j = 0; j < r; ++j) {
      const double d = H[j][j];
      if (!(d > 0.0)) {   // every lane read the same pivot
        b = 1;
        break;
      }
      const double l = sqrt(d), il = 1.0 / l;
      const int i = j + 1 + tid;
      double lij = 0.0;
      if (i < r) {
        lij = H[i][j] * il;
        H[i][j] = lij;
      }
      if (tid == 0) {
        H[j][j] = l;
        idg[j] = il;
      }
      wave_sync();
      // the row in chunks of eight: all sixteen reads issued before the writes
      if (i < r)
        for (int k0 = j + 1; k0 <= i; k0 += 8) {
          double c[8], h[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int k = min(k0 + u, i);
            c[u] = H[k][j];
            h[u] = H[i][k];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (k0 + u <= i) H[i][k0 + u] = h[u] - lij * c[u];
        }
      wave_sync();
    }
  }
  if (b == 0 && r > kSerialR) {
    // lane i keeps y_i in a register; round j broadcasts the finished y_j with readlane, so
    // the substitutions need no synchronisation
    // (each round's matrix entry and pivot are read one round ahead)
    const int ti = min(tid, r - 1);
    double yi = tid < r ? y[tid] : 0.0;
    double hn = H[ti][0], gn = idg[0];
    for (int j = 0; j < r; ++j) {            // L w = -b
      const double hj = hn, gj = gn;
      if (j + 1 < r) {
        hn = H[ti][j + 1];
        gn = idg[j + 1];
      }
      const double t = readlane_f64(yi, j) * gj;
      if (tid == j) yi = t;
      else if (tid > j && tid < r) yi -= hj * t;
    }
    hn = H[r - 1][ti];
    gn = idg[r - 1];
    for (int j = r - 1; j >= 0; --j) {       // L^T delta = w
      const double hj = hn, gj = gn;
      if (j > 0) {
        hn = H[j - 1][ti];
        gn = idg[j - 1];
      }
      const double t = readlane_f64(yi, j) * gj;
      if (tid == j) yi = t;
      else if (tid < j) yi -= hj * t;
    }
    if (tid < r) y[tid] = yi;
    wave_sync();
  }
  const bool final_iter = (iter == S.gn_iters - 1);
  if (tid == 0 && b) atomicOr(S.flags, (b & 2) ? FLAG_NONFINITE : FLAG_SINGULAR);
  if (tid < r) {
    const double zn = b ? zl.base : zl.base + y[tid];
    if (!isfinite(zn)) atomicOr(S.flags, FLAG_NONFINITE);
    if (final_iter) {
      S.z[tid] = zl.zc;
      S.z[r + tid] = zn;
      if (S.zh) S.zh[tid] = zn;   // the stress field's latent input
    } else {
      S.z[2 * r + tid] = zn;
    }
  }
  if (final_iter && tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(S.step), 1ull);
}

// Iterations k >= 1: residual r = u(z^(k)) - u^n - dt v^{n+1}, from the field kernel's
// values at the iterate (or, with tangent forms, the trapezoid rule along z^(k) - z_n).
__global__ __launch_bounds__(kGnThreads) void gn_partial_kernel(const SimDev* __restrict__ sims,
                                                                const BlockWork* __restrict__ work,
                                                                const int32_t* __restrict__ n_work,
                                                                int iter) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const GnChunkLds<kGnThreads> sh(lds);
  const int tid = threadIdx.x;
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    if (iter >= S.gn_iters) continue;
    const int r = S.r, ns = S.n_samp, p0 = wk.p0;
    const int cnt = min(kGnChunk, ns - p0);
    const int p = p0 + tid;
    // the residual's values are loaded first, so their latency passes under the
    // Jacobian's (twelve loads per thread: one batch up to r = 8)
    float vn[3] = {0.f, 0.f, 0.f}, ug[3] = {0.f, 0.f, 0.f}, un[3] = {0.f, 0.f, 0.f};
    if (tid < cnt) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vn[c] = S.vnew[c * ns + p];
        if (!S.tangent_forms) {
          ug[c] = S.u_gn[c * ns + p];
          un[c] = S.u_n[c * S.n_int + p];
        }
      }
    }
    gn_stage_jacobian<kGnThreads, 12>(S, S.J2, p0, cnt, sh);
#pragma unroll
    for (int c = 0; c < 3 && tid < kGnChunk; ++c) {
      double rv = 0.0;
      if (tid < cnt) {
        rv = -S.dt_d * (double)vn[c];
        if (S.tangent_forms) {
          // u(z^(k)) - u(z_n) by the trapezoid rule along z^(k) - z_n from the two
          // Jacobians (error O(|dz|^3)), avoiding the difference of two BF16 values
          const double* zc = S.z + r;
          const double* zi = S.z + 2 * r;
          double du = 0.0;
          for (int j = 0; j < r; ++j) {
            const int64_t o = (int64_t)(c * r + j) * ns + p;
            du += 0.5 * ((double)S.J[o] + (double)S.J2[o]) * (zi[j] - zc[j]);
          }
          rv += du;
        } else {
          rv += (double)ug[c] - (double)un[c];
        }
      }
      sh.res(c, tid) = rv;
    }
    __syncthreads();
    gn_reduce_chunk(S, p0, sh);
  }
}

__global__ __launch_bounds__(kSolveThreads) void gn_solve_kernel(const SimDev* __restrict__ sims,
                                                                 const int32_t* __restrict__ n_sims,
                                                                 int iter) {
  __shared__ double part[kSolveThreads];
  __shared__ double H[kMaxR][kMaxR + 1];
  __shared__ double y[kMaxR];
  __shared__ double idg[kMaxR];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int si = blockIdx.x; si < *n_sims; si += gridDim.x) {
    const SimDev& S = sims[si];
    if (iter >= S.gn_iters) continue;
    const int r = S.r;
    const int E = gn_entries_dev(r);
    const int G = E >= kSolveThreads ? 1 : kSolveThreads / E;
    if (tid == 0) bad = 0;
    const GnLatent zl = load_latent(S, iter);
    __syncthreads();
    // Sum the chunk partials: thread (e, g) adds chunks g, g + G, ... (16 loads in flight
    // per batch, four running sums), then the G groups are added in a fixed order.
    const int nch = S.n_gn_chunks;
    for (int e0 = 0; e0 < E; e0 += kSolveThreads / G) {
      const int e = e0 + tid % (kSolveThreads / G);
      const int g = tid / (kSolveThreads / G);
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      if (e < E && g < G) {
        const double* src = S.gn_part + e;
        for (int c0 = g; c0 < nch; c0 += 16 * G) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int c = c0 + u * G;
            v[u] = c < nch ? src[(int64_t)c * E] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) a[u & 3] += v[u];
        }
      }
      part[tid] = (a[0] + a[1]) + (a[2] + a[3]);
      __syncthreads();
      if (tid < kSolveThreads / G && e0 + tid < E) {
        double acc = 0.0;
        for (int gg = 0; gg < G; ++gg) acc += part[gg * (kSolveThreads / G) + tid];
        int j, k;
        bool is_b;
        gn_decode_entry(e0 + tid, r, j, k, is_b);
        if (!isfinite(acc)) atomicOr(&bad, 2);
        if (is_b) {
          y[j] = -acc;  // right-hand side -J^T r
        } else {
          if (j == k) acc += S.gn_damping * acc;  // Marquardt: H + lambda diag(H)
          H[j][k] = acc;
          H[k][j] = acc;
        }
      }
      __syncthreads();
    }
    if (tid < 64) solve_and_update(S, iter, H, y, idg, &bad, zl);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_gn_partial(const SimDev* sims, const BlockWork* work, const int32_t* n_work,
                             int iter, int r_cap, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (r_cap < 1 || r_cap > kMaxR) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)gn_partial_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             gn_chunk_lds_bytes(kGnThreads, kMaxR));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(gn_partial_kernel, dim3(grid), dim3(kGnThreads), gn_chunk_lds_bytes(kGnThreads, r_cap), s,
                     sims, work, n_work, iter);
  return hipGetLastError();
}

hipError_t launch_gn_solve(const SimDev* sims, const int32_t* n_sims, int iter, int grid_sims,
                           hipStream_t s) {
  if (grid_sims <= 0) return hipSuccess;
  hipLaunchKernelGGL(gn_solve_kernel, dim3(grid_sims), dim3(kSolveThreads), 0, s, sims, n_sims, iter);
  return hipGetLastError();
}

}  // namespace nsf
