// MLS-MPM transfers of the reduced step (paper Sec. 3.3 on the integration particles,
// Sec. 5.2).
//
// P2G (Sec. 3.3 step 1 with APIC, plus the node force balance of Sec. 3.2 in MLS form):
// for every integration particle, x = X + u(z_n), v = (u(z_n) - u(z_{n-1})) / dt and
//   A = m_p C - dt V_p (4 / dx^2) tau      (D^-1 = 4 / dx^2 for quadratic B-splines)
// scatter m_i += w m_p and p_i += w (m_p v + A (x_i - x_p)) over the 27 stencil nodes.
//
// Grid update (Sec. 3.3 step 2) is fused into the gather: G2P evaluates each stencil
// node's new velocity v_i = p_i / m_i + dt g, applies the sticky walls and the moving
// knife, and accumulates w v_i (Sec. 3.3 step 3) for the sample particles. The node
// value is a pure function of (m_i, p_i, node index, time), so every reader computes
// the same v_i the separate grid pass would have stored, and no dense grid sweep is
// needed.
//
// The grid is a dense array of float4 (m, p) per node that is zero between steps: after
// G2P the clean kernel zeroes the stencils the integration particles wrote, so a step
// touches only the nodes it uses.
#include "nsf_dev.h"

namespace nsf {
namespace {

struct Stencil {
  int base[3];
  float f[3];
  float w[3][3];
  bool ok;
};

__device__ __forceinline__ Stencil make_stencil(const float x[3], float inv_dx, int n) {
  Stencil st;
  st.ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float xs = x[c] * inv_dx;
    const float b = floorf(xs - 0.5f);
    const float f = xs - b;
    st.base[c] = (int)b;
    st.f[c] = f;
    st.w[c][0] = 0.5f * (1.5f - f) * (1.5f - f);
    st.w[c][1] = 0.75f - (f - 1.f) * (f - 1.f);
    st.w[c][2] = 0.5f * (f - 0.5f) * (f - 0.5f);
    st.ok = st.ok && (b >= 0.f) && (b + 2.f <= (float)(n - 1));
  }
  return st;
}

__device__ __forceinline__ const int32_t* plan_row(const SimDev& S) {
  return S.plan + (*S.step % S.plan_steps) * (int64_t)S.n_int;
}

__device__ __forceinline__ void flag(const SimDev& S, uint32_t bit) { atomicOr(S.flags, bit); }

__global__ __launch_bounds__(kMpmBlock) void p2g_kernel(const SimDev* __restrict__ sims,
                                                        const BlockWork* __restrict__ work,
                                                        const int32_t* __restrict__ n_work) {
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    const int p = wk.p0 + threadIdx.x;
    if (p >= S.n_int) continue;
    const int n_int = S.n_int;
    const int gi = plan_row(S)[p];
    float x[3], v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float u = S.u_n[c * n_int + p];
      const float up = S.u_prev[c * n_int + p];
      x[c] = S.X[(int64_t)c * S.n_part + gi] + u;
      v[c] = (u - up) / S.dt;
    }
    float t6[6], C[9];
#pragma unroll
    for (int c = 0; c < 6; ++c) t6[c] = S.tau[c * n_int + p];
#pragma unroll
    for (int c = 0; c < 9; ++c) C[c] = S.C[c * n_int + p];
    // Voigt (xx, yy, zz, yz, xz, xy) -> symmetric tau
    const float tau[9] = {t6[0], t6[5], t6[4], t6[5], t6[1], t6[3], t6[4], t6[3], t6[2]};
    float A[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) A[e] = S.mp * C[e] - S.stress_k * tau[e];
    const Stencil st = make_stencil(x, S.inv_dx, S.grid_n);
    if (!st.ok) { flag(S, FLAG_DOMAIN); continue; }
    const float mv[3] = {S.mp * v[0], S.mp * v[1], S.mp * v[2]};
    const int n = S.grid_n;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float dx0 = ((float)i - st.f[0]) * S.dx;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float dx1 = ((float)j - st.f[1]) * S.dx;
        const float wij = st.w[0][i] * st.w[1][j];
        const int64_t row = ((int64_t)(st.base[0] + i) * n + (st.base[1] + j)) * n + st.base[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float dx2 = ((float)k - st.f[2]) * S.dx;
          const float w = wij * st.w[2][k];
          float* node = reinterpret_cast<float*>(S.grid + row + k);
          const float px = w * (mv[0] + A[0] * dx0 + A[1] * dx1 + A[2] * dx2);
          const float py = w * (mv[1] + A[3] * dx0 + A[4] * dx1 + A[5] * dx2);
          const float pz = w * (mv[2] + A[6] * dx0 + A[7] * dx1 + A[8] * dx2);
          unsafeAtomicAdd(node + 0, w * S.mp);
          unsafeAtomicAdd(node + 1, px);
          unsafeAtomicAdd(node + 2, py);
          unsafeAtomicAdd(node + 3, pz);
        }
      }
    }
  }
}

// New velocity of node (i, j, k) from its mass and momentum (grid update + boundaries).
__device__ __forceinline__ void node_velocity(const SimDev& S, float4 g, int i, int j, int k,
                                              double t_new, float out[3]) {
  if (!(g.x > 0.f)) { out[0] = out[1] = out[2] = 0.f; return; }
  out[0] = g.y / g.x + S.dt * S.grav[0];
  out[1] = g.z / g.x + S.dt * S.grav[1];
  out[2] = g.w / g.x + S.dt * S.grav[2];
  const int n = S.grid_n, b = S.wall;
  if (i < b || j < b || k < b || i >= n - b || j >= n - b || k >= n - b) {
    out[0] = out[1] = out[2] = 0.f;
  }
  if (S.knife_on) {
    const double xi = i * S.dx_d, yi = j * S.dx_d, zi = k * S.dx_d;
    const double dist = S.kn[0] * xi + S.kn[1] * yi + S.kn[2] * zi - S.koff;
    if (fabs(dist) <= S.khalf && zi >= S.kz0 - S.kspeed * t_new) {
      out[0] = (float)S.kv[0];
      out[1] = (float)S.kv[1];
      out[2] = (float)S.kv[2];
    }
  }
}

__global__ __launch_bounds__(kMpmBlock) void g2p_kernel(const SimDev* __restrict__ sims,
                                                        const BlockWork* __restrict__ work,
                                                        const int32_t* __restrict__ n_work) {
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    const int p = wk.p0 + threadIdx.x;
    if (p >= S.n_samp) continue;
    const int n_int = S.n_int;
    const int gi = plan_row(S)[p];
    float x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = S.X[(int64_t)c * S.n_part + gi] + S.u_n[c * n_int + p];
    const Stencil st = make_stencil(x, S.inv_dx, S.grid_n);
    float v[3] = {0.f, 0.f, 0.f};
    if (st.ok) {
      const double t_new = (double)(*S.step + 1) * S.dt_d;
      const int n = S.grid_n;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const float wij = st.w[0][i] * st.w[1][j];
          const int64_t row = ((int64_t)(st.base[0] + i) * n + (st.base[1] + j)) * n + st.base[2];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const float w = wij * st.w[2][k];
            float vi[3];
            node_velocity(S, S.grid[row + k], st.base[0] + i, st.base[1] + j, st.base[2] + k,
                          t_new, vi);
            v[0] += w * vi[0];
            v[1] += w * vi[1];
            v[2] += w * vi[2];
          }
        }
    } else {
      flag(S, FLAG_DOMAIN);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) S.vnew[c * S.n_samp + p] = v[c];
  }
}

__global__ __launch_bounds__(kMpmBlock) void grid_clean_kernel(const SimDev* __restrict__ sims,
                                                               const BlockWork* __restrict__ work,
                                                               const int32_t* __restrict__ n_work) {
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    const int p = wk.p0 + threadIdx.x;
    if (p >= S.n_int) continue;
    const int gi = plan_row(S)[p];
    float x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      x[c] = S.X[(int64_t)c * S.n_part + gi] + S.u_n[c * S.n_int + p];
    const Stencil st = make_stencil(x, S.inv_dx, S.grid_n);
    if (!st.ok) continue;
    const int n = S.grid_n;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int64_t row = ((int64_t)(st.base[0] + i) * n + (st.base[1] + j)) * n + st.base[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) S.grid[row + k] = z;
      }
  }
}

}  // namespace

hipError_t launch_p2g(const SimDev* sims, const BlockWork* work, const int32_t* n_work, int grid,
                      hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(p2g_kernel, dim3(grid), dim3(kMpmBlock), 0, s, sims, work, n_work);
  return hipGetLastError();
}

hipError_t launch_g2p(const SimDev* sims, const BlockWork* work, const int32_t* n_work, int grid,
                      hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(g2p_kernel, dim3(grid), dim3(kMpmBlock), 0, s, sims, work, n_work);
  return hipGetLastError();
}

hipError_t launch_grid_clean(const SimDev* sims, const BlockWork* work, const int32_t* n_work,
                             int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(grid_clean_kernel, dim3(grid), dim3(kMpmBlock), 0, s, sims, work, n_work);
  return hipGetLastError();
}

}  // namespace nsf
