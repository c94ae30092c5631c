// MLS-MPM transfers of the reduced step (paper Sec. 3.3 on the integration particles,
// Sec. 5.2), written as a gather so that no float atomics are needed.
//
// P2G (Sec. 3.3 step 1 with APIC, plus the node force balance of Sec. 3.2 in MLS form):
// every integration particle has x = X + u(z_n), a velocity v and
//   A = m_p C - dt V_p (4 / dx^2) tau      (D^-1 = 4 / dx^2 for quadratic B-splines)
// and node i receives m_i = sum_p w_ip m_p and p_i = sum_p w_ip (m_p v + A (x_i - x_p)).
// The grid update (Sec. 3.3 step 2: v_i = p_i / m_i + dt g, sticky walls, moving knife)
// runs once per node right after its sums, and G2P (Sec. 3.3 step 3) gathers the new node
// velocities for the sample particles.
//
// Kernels of one step:
//   bin      each integration particle finds its stencil base cell and its bin (a cube
//            of bin_edge^3 cells), counts itself in the bin and remembers its rank;
//   alloc    one workgroup per simulation: a block-wide prefix sum of the bin counts (over
//            the first particle of each bin, or over the bins for large sets) gives each
//            non-empty bin its record slots, the bin is listed as non-empty and the node
//            blocks its particles reach are marked in an LDS bitmap, which is then
//            compacted into the list of active node blocks;
//   place    every particle writes its index at its bin's slot + rank (for small sets the
//            allocation does it itself);
//   sort     one workgroup per non-empty bin sorts the bin's indices and writes the P2G
//            records (x, m v, A, index) in that order;
//   gather   one workgroup per active node block stages, window by window, the records of
//            the 2 x 2 x 2 bins whose particles can reach it whose stencil does reach it,
//            in LDS, sums every node's mass and momentum in that order (deterministic:
//            where each bin's slots lie does not matter, only the sorted order inside a
//            bin and the fixed order of the bins), applies the grid update and stores the
//            node's new velocity;
//   g2p      each sample particle sums w_ip v_i over its 27 stencil nodes, and the block
//            reduces its chunk of the first Gauss-Newton system (gn_reduce.h).
// A node block only holds values written this step; nodes outside active blocks are never
// read because every particle's stencil lies in active blocks. A bin's slot range and
// count are valid only in the epoch that set them, so no per-step clearing of the bin
// tables is needed.
#include "gn_reduce.h"
#include "nsf_dev.h"

namespace nsf {
namespace {

struct Stencil {
  int base[3];
  float f[3];
  float w[3][3];
  bool ok;
};

// Every operation rounds to FP32 on its own (no contraction into FMAs), so the stencil
// base, which decides membership in the integration set, is a reproducible function of
// the FP32 position.
__device__ __forceinline__ Stencil make_stencil(const float x[3], float inv_dx, int n) {
#pragma clang fp contract(off)
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

// Workgroups of a per-sim kernel are dealt to the sims in equal shares: `per` workgroups
// work on each sim (all of them when there is one sim), each taking items q, q + per, ...
struct SimShare {
  int per, groups, q, first;
  __device__ SimShare(int n_sims) {
    per = max(1, (int)gridDim.x / max(n_sims, 1));
    groups = gridDim.x / per;
    q = blockIdx.x % per;
    first = blockIdx.x < groups * per ? blockIdx.x / per : n_sims;
  }
};

__device__ __forceinline__ void particle_x(const SimDev& S, int p, int gi, float x[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] = S.X[(int64_t)c * S.n_part + gi] + S.u_n[c * S.n_int + p];
}

// P2G record of an integration particle, kRec floats (128 bytes), in one of two layouts.
// Workgroup layout (solo plans, dense sets and grids above 128^3; the gather recomputes
// the stencil from x):
//   [0..2] x, [3..5] m_p v, [6..14] A = m_p C - dt V_p (4/dx^2) tau (row-major),
//   [15] the stencil base cell packed 10 bits per axis (x << 20 | y << 10 | z).
// Wave layout (sparse sims on grids up to 128^3 in a batch), everything a node needs to add
// the particle's contribution with a few FMAs: with node offset o = (a, b, c) in {0,1,2}^3
// from the base, the contribution to mass is m_p w and to momentum w (q + dx A o), where
// q = m_p v - dx A f (f = x / dx - base), and each axis weight is a quadratic in o through
// the three B-spline weights (w(o) = alpha + o (beta + gamma o)):
//   [0..2] q, [3..11] dx A (row-major), [12..20] (alpha, beta, gamma) per axis,
//   [21] the packed base, [22..31] unused.
// The binning writes the record in particle order (every field array is read coalesced),
// the sort copies it into bin order.
constexpr int kRec = 32;

__device__ __forceinline__ void write_record(const SimDev& S, int p, const float x[3], const Stencil& st,
                                             bool wave_layout, float* r) {
  const int n_int = S.n_int;
  float v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float u = S.u_n[c * n_int + p];
    const float up = S.u_prev[c * n_int + p];
    v[c] = S.tangent_forms ? up : (u - up) / S.dt;  // u_prev holds v itself in tangent form
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
  const int pb = (st.base[0] << 20) | (st.base[1] << 10) | st.base[2];
  float4* r4 = reinterpret_cast<float4*>(r);
  if (!wave_layout) {
    r4[0] = make_float4(x[0], x[1], x[2], S.mp * v[0]);
    r4[1] = make_float4(S.mp * v[1], S.mp * v[2], A[0], A[1]);
    r4[2] = make_float4(A[2], A[3], A[4], A[5]);
    r4[3] = make_float4(A[6], A[7], A[8], __int_as_float(pb));
    return;
  }
  const float dx = S.dx;
  float dA[9], q[3], poly[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) dA[e] = dx * A[e];
#pragma unroll
  for (int c = 0; c < 3; ++c) q[c] = S.mp * v[c] - (dA[3 * c] * st.f[0] + dA[3 * c + 1] * st.f[1] + dA[3 * c + 2] * st.f[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float w0 = st.w[c][0], w1 = st.w[c][1], w2 = st.w[c][2];
    const float g = 0.5f * (w0 - 2.f * w1 + w2);
    poly[3 * c] = w0;
    poly[3 * c + 1] = w1 - w0 - g;
    poly[3 * c + 2] = g;
  }
  r4[0] = make_float4(q[0], q[1], q[2], dA[0]);
  r4[1] = make_float4(dA[1], dA[2], dA[3], dA[4]);
  r4[2] = make_float4(dA[5], dA[6], dA[7], dA[8]);
  r4[3] = make_float4(poly[0], poly[1], poly[2], poly[3]);
  r4[4] = make_float4(poly[4], poly[5], poly[6], poly[7]);
  r4[5] = make_float4(poly[8], __int_as_float(pb), 0.f, 0.f);
}

// ---- bin ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMpmBlock) void bin_kernel(const SimDev* __restrict__ sims,
                                                        const BlockWork* __restrict__ work,
                                                        const int32_t* __restrict__ n_work,
                                                        int32_t* __restrict__ claims, int full) {
  // the field kernels' claim counters of this step start from zero
  if (blockIdx.x == 0 && threadIdx.x < kClaimCounters) claims[threadIdx.x] = 0;
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    if (wk.p0 == 0) {
      if (threadIdx.x == 0) *S.epoch += 1;   // this step's binning epoch
      // the latent a pipelined decode of this step reads (z_n; the step overwrites z)
      if (S.pipelined_decode && (int)threadIdx.x < S.r) S.zdec[threadIdx.x] = S.z[S.r + threadIdx.x];
    }
    const int p = wk.p0 + threadIdx.x;
    if (p >= live_count(S)) continue;
    float x[3];
    particle_x(S, p, plan_row(S)[p], x);
    const Stencil st = make_stencil(x, S.inv_dx, S.grid_n);
    if (!st.ok) {
      flag(S, FLAG_DOMAIN);
      S.pbin[p] = -1;
      continue;
    }
    const int B = S.bin_edge, nbs = S.nbs;
    const int bin = ((st.base[0] / B) * nbs + st.base[1] / B) * nbs + st.base[2] / B;
    S.pbin[p] = bin;
    S.prank[p] = atomicAdd(&S.bin_cnt[bin], 1);
    write_record(S, p, x, st, full != 0 && S.bin_edge == 4, S.rec_p + (int64_t)p * kRec);
  }
}

// ---- allocate + place ---------------------------------------------------------------
constexpr int kAllocThreads = 1024;
constexpr int kMaxBins = 32768;   // 32 bins per axis at most
constexpr int kBinsPerThread = kMaxBins / kAllocThreads;   // contiguous bins per alloc thread

// Exclusive scan of one value per thread over a workgroup of T threads; returns the prefix
// and the workgroup total in *total. wave_sums holds T / 64 ints.
template <int T>
__device__ __forceinline__ int block_scan(int v, int* wave_sums, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wave_sums[wave] = incl;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int w = threadIdx.x;
    int x = w < T / 64 ? wave_sums[w] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(x, o);
      if (w >= o) x += t;
    }
    if (w < T / 64) wave_sums[w] = x;   // inclusive over waves
  }
  __syncthreads();
  const int excl = (wave > 0 ? wave_sums[wave - 1] : 0) + incl - v;
  *total = wave_sums[T / 64 - 1];
  __syncthreads();
  return excl;
}

__device__ __forceinline__ int block_exclusive_scan(int v, int* wave_sums, int* total) {
  return block_scan<kAllocThreads>(v, wave_sums, total);
}

// Work items spread over the sims of a launch, one item per wave: count(S) items in sim S.
// Every thread of the workgroup computes the exclusive prefix s_pre[s] (items of the sims
// before s; s_pre[nsims] = the total, returned) in LDS; find_sim maps an item to its sim.
// nsims <= kMaxBatchSims.
template <int T, class Count>
__device__ __forceinline__ int sims_prefix(const SimDev* __restrict__ sims, int nsims, int* s_pre,
                                           int* wave_sums, Count count) {
  const int per = (nsims + T - 1) / T;
  const int lo = min(nsims, (int)threadIdx.x * per), hi = min(nsims, lo + per);
  int local = 0;
  for (int s = lo; s < hi; ++s) {
    const int c = count(sims[s]);
    s_pre[s] = c;
    local += c;
  }
  int total;
  int run = block_scan<T>(local, wave_sums, &total);
  for (int s = lo; s < hi; ++s) {
    const int c = s_pre[s];
    s_pre[s] = run;
    run += c;
  }
  if (threadIdx.x == 0) s_pre[nsims] = total;
  __syncthreads();
  return total;
}

// The sim whose items [s_pre[s], s_pre[s + 1]) hold item v (0 <= v < s_pre[nsims]).
__device__ __forceinline__ int find_sim(const int* s_pre, int nsims, int v) {
  int lo = 0, hi = nsims;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_pre[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Orders this wave's earlier LDS accesses before its later ones (the wave owns the region:
// no workgroup barrier is involved).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Slot allocation, one workgroup per sim, in one of two ways (both deterministic; where a
// bin's slots lie does not change any sum):
//  - up to kAllocByParticles particles it walks the particles: the first particle of each
//    bin (rank 0) allocates the bin's slots from a workgroup prefix sum in particle order,
//    and every particle is placed at its bin's slot + rank right away;
//  - above that it walks the bins (a cost that does not grow with the particle count):
//    thread t owns kBinsPerThread consecutive bins, the prefix sum runs in bin order, and
//    place_kernel places the particles afterwards.
// Either way the bin is listed as non-empty and its node blocks (bin + {0, 1}^3: the
// stencils of its particles reach at most one block further on each axis) are marked in
// an LDS bitmap, which is then compacted into the active-block list.
constexpr int kAllocBatch = 8;               // particles per thread per batch of loads

// Record non-empty bin b (count c, first slot start) and mark its node blocks.
__device__ __forceinline__ void describe_bin(const SimDev& S, int b, int c, int start, int ep, uint32_t* mark) {
  S.bin_cnt[b] = 0;   // counts start from zero next step
  S.bin_meta[b] = make_int4(ep, start, c, 0);
  const int nbs = S.nbs;
  const int bx = b / (nbs * nbs), by = (b / nbs) % nbs, bz = b % nbs;
  for (int d = 0; d < 8; ++d) {
    const int x = bx + (d >> 2), y = by + ((d >> 1) & 1), z = bz + (d & 1);
    if (x < nbs && y < nbs && z < nbs) {
      const int k = (x * nbs + y) * nbs + z;
      atomicOr(&mark[k >> 5], 1u << (k & 31));
    }
  }
}

__device__ __forceinline__ void list_bin(const SimDev& S, int b, int c, int start, int ep, int& ne_pos,
                                         uint32_t* mark) {
  S.nonempty[ne_pos++] = b;
  describe_bin(S, b, c, start, ep, mark);
}

// s_start[b] packs the bin's first slot (high 16 bits) and its count (low 16 bits): both
// are at most kAllocByParticles.
static_assert(kAllocByParticles <= 32768, "slot and count packed in 16 bits each");

__device__ __forceinline__ int alloc_by_particles(const SimDev& S, int n, uint32_t* mark, int* wave_sums,
                                                  int* s_start) {
  const int tid = threadIdx.x;
  // thread t owns particles t, t + T, t + 2T, ... (coalesced); loads go kAllocBatch at a
  // time, and with one round (at most T kAllocBatch particles) they stay in registers
  const int round = kAllocThreads * kAllocBatch;
  const bool one = n <= round;
  int pb[kAllocBatch], rk[kAllocBatch], cnt[kAllocBatch];
  auto load = [&](int p0) {
#pragma unroll
    for (int u = 0; u < kAllocBatch; ++u) {
      const int p = p0 + u * kAllocThreads + tid;
      pb[u] = p < n ? S.pbin[p] : -1;
      rk[u] = p < n ? S.prank[p] : 1;
    }
#pragma unroll
    for (int u = 0; u < kAllocBatch; ++u) cnt[u] = (pb[u] >= 0 && rk[u] == 0) ? S.bin_cnt[pb[u]] : 0;
  };
  int local = 0, ne = 0;
  for (int p0 = 0; p0 < n; p0 += round) {
    load(p0);
#pragma unroll
    for (int u = 0; u < kAllocBatch; ++u) {
      local += cnt[u];
      ne += (pb[u] >= 0 && rk[u] == 0);
    }
  }
  int used, n_ne;
  int run = block_exclusive_scan(local, wave_sums, &used);
  int ne_pos = block_exclusive_scan(ne, wave_sums, &n_ne);
  // the first particle of each bin takes the bin's slots and list position (particle order)
  for (int p0 = 0; p0 < n; p0 += round) {
    if (!one) load(p0);
#pragma unroll
    for (int u = 0; u < kAllocBatch; ++u) {
      const int b = pb[u];
      if (b < 0 || rk[u] != 0) continue;
      s_start[b] = (run << 16) | cnt[u];
      S.nonempty[ne_pos++] = b;
      run += cnt[u];
    }
  }
  __syncthreads();
  // then every thread takes part in describing the listed bins and placing the particles
  const int ep = *S.epoch;
  for (int i = tid; i < n_ne; i += kAllocThreads) {
    const int b = S.nonempty[i];
    const int v = s_start[b];
    describe_bin(S, b, v & 0xffff, v >> 16, ep, mark);
  }
  for (int p0 = 0; p0 < n; p0 += round) {
    if (!one) load(p0);
#pragma unroll
    for (int u = 0; u < kAllocBatch; ++u)
      if (pb[u] >= 0) S.sorted[(s_start[pb[u]] >> 16) + rk[u]] = p0 + u * kAllocThreads + tid;
  }
  return n_ne;
}

__device__ __forceinline__ int alloc_by_bins(const SimDev& S, uint32_t* mark, int* wave_sums) {
  const int tid = threadIdx.x, nb = S.n_bins;
  // the thread's bin counts, loaded together (all in flight at once) and kept
  const int blo = tid * kBinsPerThread;
  int cnt[kBinsPerThread];
#pragma unroll
  for (int u = 0; u < kBinsPerThread; ++u) cnt[u] = blo + u < nb ? S.bin_cnt[blo + u] : 0;
  int local = 0, ne = 0;
#pragma unroll
  for (int u = 0; u < kBinsPerThread; ++u) {
    local += cnt[u];
    ne += cnt[u] > 0;
  }
  int used, n_ne;
  int run = block_exclusive_scan(local, wave_sums, &used);
  int ne_pos = block_exclusive_scan(ne, wave_sums, &n_ne);
  const int ep = *S.epoch;
#pragma unroll
  for (int u = 0; u < kBinsPerThread; ++u) {
    if (cnt[u] == 0) continue;
    list_bin(S, blo + u, cnt[u], run, ep, ne_pos, mark);
    run += cnt[u];
  }
  return n_ne;
}

__global__ __launch_bounds__(kAllocThreads) void alloc_kernel(const SimDev* __restrict__ sims,
                                                              const int32_t* __restrict__ n_sims) {
  extern __shared__ int s_start[];              // [n_bins] first slot of each non-empty bin
  __shared__ uint32_t mark[kMaxBins / 32];      // node blocks reached this step
  __shared__ int wave_sums[kAllocThreads / 64];
  const int tid = threadIdx.x;
  for (int s = blockIdx.x; s < *n_sims; s += gridDim.x) {
    const SimDev& S = sims[s];
    const int n = live_count(S);
    const int nwords = (S.n_bins + 31) / 32;
    for (int wd = tid; wd < nwords; wd += kAllocThreads) mark[wd] = 0u;
    __syncthreads();
    const int n_ne = n <= kAllocByParticles ? alloc_by_particles(S, n, mark, wave_sums, s_start)
                                            : alloc_by_bins(S, mark, wave_sums);
    __syncthreads();
    // compact the marked node blocks in index order
    const int wper = (nwords + kAllocThreads - 1) / kAllocThreads;
    const int wlo = min(nwords, tid * wper), whi = min(nwords, wlo + wper);
    int n_marked = 0;
    for (int wd = wlo; wd < whi; ++wd) n_marked += __popc(mark[wd]);
    int n_act;
    int pos = block_exclusive_scan(n_marked, wave_sums, &n_act);
    for (int wd = wlo; wd < whi; ++wd) {
      uint32_t m = mark[wd];
      while (m) {
        const int bit = __ffs(m) - 1;
        m &= m - 1;
        S.active[pos++] = wd * 32 + bit;
      }
    }
    if (tid == 0) {
      S.n_active[0] = n_act;
      S.n_active[1] = n_ne;
    }
    __syncthreads();
  }
}

// Every integration particle's index at its bin's first slot + its rank.
__global__ __launch_bounds__(kMpmBlock) void place_kernel(const SimDev* __restrict__ sims,
                                                          const BlockWork* __restrict__ work,
                                                          const int32_t* __restrict__ n_work) {
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    const int n = live_count(S);
    if (n <= kAllocByParticles) continue;   // placed by the allocation itself
    const int p = wk.p0 + threadIdx.x;
    if (p >= n) continue;
    const int pb = S.pbin[p];
    if (pb >= 0) S.sorted[S.bin_meta[pb].y + S.prank[p]] = p;
  }
}

// One wave per non-empty bin (bins spread over the launch's sims): sort the bin's particle
// indices (in registers up to 64, in the wave's LDS up to kSegMax; a larger bin keeps its
// arrival order) and copy the records into bin order.
constexpr int kSortWaves = 4, kSortThreads = 64 * kSortWaves;

// (native 4-float vectors: an array of HIP's float4 structs is not promoted to registers
// and would live in scratch memory)
template <int NQ>
__device__ __forceinline__ void copy_record(const SimDev& S, int p, int slot) {
  const f32x4* src = reinterpret_cast<const f32x4*>(S.rec_p + (int64_t)p * kRec);
  f32x4* dst = reinterpret_cast<f32x4*>(S.rec + (int64_t)slot * kRec);
  f32x4 q[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) q[k] = src[k];
#pragma unroll
  for (int k = 0; k < NQ; ++k) dst[k] = q[k];
}

// the first NQ float4 of the record: 6 for the wave layout, 4 for the workgroup layout;
// four records per lane are loaded before any is stored, so their latencies overlap
template <int NQ>
__device__ __forceinline__ void copy_records(const SimDev& S, const int* idx, int start, int cnt, int lane) {
  constexpr int U = 4;
  for (int i0 = lane; i0 < cnt; i0 += 64 * U) {
    f32x4 q[U][NQ];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 64 * u;
      if (i < cnt) {
        const f32x4* src = reinterpret_cast<const f32x4*>(S.rec_p + (int64_t)idx[i] * kRec);
#pragma unroll
        for (int k = 0; k < NQ; ++k) q[u][k] = src[k];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 64 * u;
      if (i < cnt) {
        f32x4* dst = reinterpret_cast<f32x4*>(S.rec + (int64_t)(start + i) * kRec);
#pragma unroll
        for (int k = 0; k < NQ; ++k) dst[k] = q[u][k];
      }
    }
  }
}

template <int NQ>
__global__ __launch_bounds__(kSortThreads) void bin_sort_kernel(const SimDev* __restrict__ sims,
                                                                const int32_t* __restrict__ n_sims) {
  __shared__ int s_pre[kMaxBatchSims + 1];
  __shared__ int wave_sums[kSortWaves];
  __shared__ int s_buf[kSortWaves][kSegMax];
  const int nsims = *n_sims;
  const int total = sims_prefix<kSortThreads>(sims, nsims, s_pre, wave_sums,
                                              [](const SimDev& S) { return S.n_active[1]; });
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  int* buf = s_buf[wv];
  for (int v = blockIdx.x * kSortWaves + wv; v < total; v += gridDim.x * kSortWaves) {
    // wave-uniform, so the sim's constants and the bin's slot range come through scalar loads
    const int s = __builtin_amdgcn_readfirstlane(find_sim(s_pre, nsims, v));
    const SimDev& S = sims[s];
    const int b = __builtin_amdgcn_readfirstlane(S.nonempty[v - s_pre[s]]);
    const int4 meta = S.bin_meta[b];
    const int start = meta.y;
    const int cnt = meta.z;
    const int32_t* seg = S.sorted + start;
    if (cnt <= 64) {
      int x = lane < cnt ? seg[lane] : 0x7fffffff;
      for (int kk = 2; kk <= 64; kk <<= 1)
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
          const int o = __shfl_xor(x, jj);
          const bool lower = (lane & jj) == 0, up = (lane & kk) == 0;
          x = (lower == up) ? min(x, o) : max(x, o);
        }
      if (lane < cnt) copy_record<NQ>(S, x, start + lane);
    } else if (cnt <= kSegMax) {
      int p2 = 128;
      while (p2 < cnt) p2 <<= 1;
      for (int i = lane; i < p2; i += 64) buf[i] = i < cnt ? seg[i] : 0x7fffffff;
      wave_lds_sync();
      // each pass touches every element once, from one lane (the lane of the pair's lower
      // index), so a lane reads its pairs eight at a time before writing any of them
      for (int kk = 2; kk <= p2; kk <<= 1)
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
          for (int i0 = lane; i0 < p2; i0 += 64 * 8) {
            int a[8], c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int i = i0 + 64 * u, l = i ^ jj;
              if (i < p2 && l > i) {
                a[u] = buf[i];
                c[u] = buf[l];
              }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int i = i0 + 64 * u, l = i ^ jj;
              if (i < p2 && l > i && (a[u] > c[u]) == ((i & kk) == 0)) {
                buf[i] = c[u];
                buf[l] = a[u];
              }
            }
          }
          wave_lds_sync();
        }
      copy_records<NQ>(S, buf, start, cnt, lane);
      wave_lds_sync();
    } else {
      copy_records<NQ>(S, seg, start, cnt, lane);
    }
  }
}

// ---- gather + grid update ----------------------------------------------------------
// T threads (T / 64 groups of 64 lanes) per workgroup, and a window of T records staged
// in LDS at a time (~30 KB at T = 256: 5 workgroups per CU). A plan sim's sparse blocks
// use T = 256; a closure sim's dense blocks (hundreds of records per bin) T = 512.
constexpr int kGatherThreads = 256, kGatherThreadsDense = 512;
constexpr int kMaxNodesPerLane = 8;   // bin_edge <= 8

// New velocity of node (i, j, k) from its mass and momentum (grid update + boundaries).
__device__ __forceinline__ void node_velocity(const SimDev& S, float m, const float pm[3], int i,
                                              int j, int k, double t_new, float out[3]) {
  if (!(m > 0.f)) { out[0] = out[1] = out[2] = 0.f; return; }
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = pm[c] / m + S.dt * S.grav[c];
  const int n = S.grid_n, b = S.wall;
  const bool side = i < b || j < b || i >= n - b || j >= n - b || k >= n - b;
  if (side || (k < b && !S.ground)) out[0] = out[1] = out[2] = 0.f;
  else if (k < b) out[2] = fmaxf(out[2], 0.f);   // separating ground
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

// NPL: nodes per lane the kernel provides for (1 for 4^3-node blocks, grids up to 128^3;
// kMaxNodesPerLane for any grid); the accumulators of unused nodes cost registers.
template <int T, int NPL>
__global__ __launch_bounds__(T) void gather_kernel(const SimDev* __restrict__ sims,
                                                  const int32_t* __restrict__ n_sims, int edge_only) {
  constexpr int NG = T / 64;   // lane groups
  // staged records, structure of arrays
  __shared__ float s_mv[3][T];
  __shared__ float s_A[9][T];
  __shared__ float s_w[9][T];
  __shared__ float s_f[3][T];
  __shared__ int s_base[T];   // packed base cell (10 bits per axis)
  __shared__ float s_red[NG][64][4];
  __shared__ int s_seg[9];            // the source bins' record ranges, concatenated
  __shared__ int s_from[8];
  __shared__ int s_cnt[8];
  __shared__ int s_wkeep[NG];
  const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
  const int total_sims = *n_sims;
  const SimShare share(total_sims);
  for (int s = share.first; s < total_sims; s += share.groups) {
    const SimDev& S = sims[s];
    if (edge_only && S.bin_edge != edge_only) continue;   // served by gather_wave_kernel
    const int nact = S.n_active[0];
    const int B = S.bin_edge, nbs = S.nbs, n = S.grid_n;
    const int nodes = B * B * B;
    const int npl = (nodes + 63) / 64;   // nodes per lane
    const double t_new = (double)(*S.step + 1) * S.dt_d;
    const int ep = *S.epoch;
    for (int k = share.q; k < nact; k += share.per) {
      const int blk = S.active[k];
      const int bx = blk / (nbs * nbs), by = (blk / nbs) % nbs, bz = blk % nbs;
      // source bins in a fixed order: the block itself and its lower neighbours (looked up
      // by 8 threads at once, then prefix-summed)
      if (tid < 8) {
        const int d = tid;
        const int sx = bx - (d >> 2), sy = by - ((d >> 1) & 1), sz = bz - (d & 1);
        int c = 0, from = 0;
        if (sx >= 0 && sy >= 0 && sz >= 0) {
          const int sb = (sx * nbs + sy) * nbs + sz;
          const int4 meta = S.bin_meta[sb];
          const int e = meta.x, f = meta.y, cc = meta.z;
          if (e == ep) {
            from = f;
            c = cc;
          }
        }
        s_from[d] = from;
        s_cnt[d] = c;
      }
      __syncthreads();
      if (tid == 0) {
        int run = 0;
        for (int d = 0; d < 8; ++d) {
          s_seg[d] = run;
          run += s_cnt[d];
        }
        s_seg[8] = run;
      }
      __syncthreads();
      const int total = s_seg[8];
      float acc[NPL][4];
#pragma unroll
      for (int q = 0; q < NPL; ++q) acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.f;
      // records in concatenated order (bin order, each bin sorted by particle index), a
      // window of T at a time. A block with more than one window stages only the records
      // whose stencil reaches it (base + 2 >= the block's first node on every axis: the
      // source bins lie at or below it), compacted in order.
      const bool dense = total > T;
      for (int c0 = 0; c0 < total; c0 += T) {
        const int g = c0 + tid;
        bool keep = false;
        const float4* r4 = nullptr;
        if (g < total) {
          int d = 0;
          while (g >= s_seg[d + 1]) ++d;
          r4 = reinterpret_cast<const float4*>(S.rec + (int64_t)(s_from[d] + g - s_seg[d]) * kRec);
          keep = true;
          if (dense) {
            const float4 a = r4[0];
            const float x[3] = {a.x, a.y, a.z};
            const Stencil st = make_stencil(x, S.inv_dx, n);
            keep = st.base[0] + 2 >= bx * B && st.base[1] + 2 >= by * B && st.base[2] + 2 >= bz * B;
          }
        }
        int i = tid, cnt = total;
        if (dense) {
          const uint64_t kept = __ballot(keep);
          if (lane == 0) s_wkeep[grp] = __popcll(kept);
          __syncthreads();
          i = __popcll(kept & ((1ull << lane) - 1));
          cnt = 0;
#pragma unroll
          for (int w = 0; w < NG; ++w) {
            if (w < grp) i += s_wkeep[w];
            cnt += s_wkeep[w];
          }
        }
        if (keep) {
          const float4 a = r4[0], b4 = r4[1], c4 = r4[2], e4 = r4[3];
          const float x[3] = {a.x, a.y, a.z};
          const Stencil st = make_stencil(x, S.inv_dx, n);
          s_mv[0][i] = a.w; s_mv[1][i] = b4.x; s_mv[2][i] = b4.y;
          s_A[0][i] = b4.z; s_A[1][i] = b4.w; s_A[2][i] = c4.x; s_A[3][i] = c4.y;
          s_A[4][i] = c4.z; s_A[5][i] = c4.w; s_A[6][i] = e4.x; s_A[7][i] = e4.y;
          s_A[8][i] = e4.z;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            s_f[c][i] = st.f[c];
            s_w[3 * c + 0][i] = st.w[c][0];
            s_w[3 * c + 1][i] = st.w[c][1];
            s_w[3 * c + 2][i] = st.w[c][2];
          }
          s_base[i] = (st.base[0] << 20) | (st.base[1] << 10) | st.base[2];
        }
        __syncthreads();
        // group g adds records g, g + 4, ... of this stage
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
          const int node = lane + 64 * q;
          if (q >= npl || node >= nodes) continue;
          const int ni = bx * B + node / (B * B), nj = by * B + (node / B) % B, nk = bz * B + node % B;
          for (int i = grp; i < cnt; i += NG) {
            const int pb = s_base[i];
            const int di = ni - (pb >> 20), dj = nj - ((pb >> 10) & 1023), dk = nk - (pb & 1023);
            if ((unsigned)di > 2u || (unsigned)dj > 2u || (unsigned)dk > 2u) continue;
            const float w = s_w[di][i] * s_w[3 + dj][i] * s_w[6 + dk][i];
            const float d0 = ((float)di - s_f[0][i]) * S.dx;
            const float d1 = ((float)dj - s_f[1][i]) * S.dx;
            const float d2 = ((float)dk - s_f[2][i]) * S.dx;
            acc[q][0] += w * S.mp;
            acc[q][1] += w * (s_mv[0][i] + s_A[0][i] * d0 + s_A[1][i] * d1 + s_A[2][i] * d2);
            acc[q][2] += w * (s_mv[1][i] + s_A[3][i] * d0 + s_A[4][i] * d1 + s_A[5][i] * d2);
            acc[q][3] += w * (s_mv[2][i] + s_A[6][i] * d0 + s_A[7][i] * d1 + s_A[8][i] * d2);
          }
        }
        __syncthreads();
      }
      // add the four groups in order, grid update, store
#pragma unroll
      for (int q = 0; q < NPL; ++q) {
        if (q >= npl) break;
        const int node = lane + 64 * q;
        s_red[grp][lane][0] = acc[q][0];
        s_red[grp][lane][1] = acc[q][1];
        s_red[grp][lane][2] = acc[q][2];
        s_red[grp][lane][3] = acc[q][3];
        __syncthreads();
        if (grp == 0 && node < nodes) {
          float m = 0.f, pm[3] = {0.f, 0.f, 0.f};
          for (int g = 0; g < NG; ++g) {
            m += s_red[g][lane][0];
            pm[0] += s_red[g][lane][1];
            pm[1] += s_red[g][lane][2];
            pm[2] += s_red[g][lane][3];
          }
          const int ni = bx * B + node / (B * B), nj = by * B + (node / B) % B, nk = bz * B + node % B;
          if (ni < n && nj < n && nk < n) {
            float v[3];
            node_velocity(S, m, pm, ni, nj, nk, t_new, v);
            S.grid[((int64_t)ni * n + nj) * n + nk] = make_float4(v[0], v[1], v[2], m);
          }
        }
        __syncthreads();
      }
    }
  }
}

// Gather with one wave per active node block, for sims whose bins are 4^3 cells (grids up
// to 128^3) and whose integration particles are sparse (under one particle per cell on
// average, as a uniform sample of a few percent is). Node blocks of every sim of the launch
// form one list, dealt to waves in order. Lane q of the wave owns node q of the block and
// keeps its mass and momentum sums in registers. The records of the block's 2 x 2 x 2
// source bins are taken 64 at a time in the fixed order (bin order, each bin sorted by
// particle index): lane j loads record j's stencil base, and the wave walks the records
// whose stencil reaches the block in lane order, reading each through scalar loads into
// scalar registers (a vector load of one address would return a copy to every lane), the
// lanes whose node lies in its stencil adding its contribution. No LDS, no barrier: the sums
// depend only on the sim's own records, so a sim stepped alone or in any batch gives the
// same bits.
// global-address-space views (vector loads that complete in order, not flat loads)
typedef const __attribute__((address_space(1))) float* GlobalF;
typedef const __attribute__((address_space(1))) int* GlobalI;
// constant-address-space view: uniform loads through it are scalar loads
typedef const __attribute__((address_space(4))) float* ConstRec;
constexpr int kGsWaves = 4, kGsThreads = 64 * kGsWaves;
// A kept record's first 22 floats as six 4-float vectors (the last two floats past the
// record's fields are padding); LDS rows of kGsRow floats.
constexpr int kRecVec = 6, kGsRow = 4 * kRecVec;

__global__ __launch_bounds__(kGsThreads) void gather_lanes_kernel(const SimDev* __restrict__ sims,
                                                                  const int32_t* __restrict__ n_sims) {
  __shared__ int s_pre[kMaxBatchSims + 1];
  __shared__ int wave_sums[kGsWaves];
  // each wave's kept records of a chunk, one row each (22 floats, rows 16-byte aligned)
  __shared__ __attribute__((aligned(16))) float s_rec[kGsWaves][64][kGsRow];
  const int nsims = *n_sims;
  const int total = sims_prefix<kGsThreads>(sims, nsims, s_pre, wave_sums,
                                            [](const SimDev& S) { return S.bin_edge == 4 ? S.n_active[0] : 0; });
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lx = lane >> 4, ly = (lane >> 2) & 3, lz = lane & 3;   // node of the lane in its block
  const int stride = gridDim.x * kGsWaves;
  int v = blockIdx.x * kGsWaves + wave;
  int s = 0, blk = 0;
  if (v < total) {
    s = __builtin_amdgcn_readfirstlane(find_sim(s_pre, nsims, v));
    blk = __builtin_amdgcn_readfirstlane(sims[s].active[v - s_pre[s]]);
  }
  for (; v < total; v += stride) {
    const SimDev& S = sims[s];
    // the next block's sim and index, loaded while this one is summed
    const int vn = v + stride;
    int sn = s, bn = 0;
    if (vn < total) {
      sn = __builtin_amdgcn_readfirstlane(find_sim(s_pre, nsims, vn));
      bn = __builtin_amdgcn_readfirstlane(sims[sn].active[vn - s_pre[sn]]);
    }
    const int nbs = S.nbs, n = S.grid_n;
    const int bx = blk / (nbs * nbs), by = (blk / nbs) % nbs, bz = blk % nbs;
    const int ox = 4 * bx, oy = 4 * by, oz = 4 * bz;
    const int ep = *S.epoch;
    const float mp = S.mp;
    // source bins d = 0..7 (the block's own bin and its lower neighbours) on lanes 0..7
    int from = 0, cnt = 0;
    if (lane < 8) {
      const int sx = bx - (lane >> 2), sy = by - ((lane >> 1) & 1), sz = bz - (lane & 1);
      if (sx >= 0 && sy >= 0 && sz >= 0) {
        const GlobalI meta = (GlobalI)S.bin_meta + 4 * ((sx * nbs + sy) * nbs + sz);
        if (meta[0] == ep) {
          from = meta[1];
          cnt = meta[2];
        }
      }
    }
    int incl = cnt;
#pragma unroll
    for (int k = 1; k < 8; k <<= 1) {
      const int t = __shfl_up(incl, k);
      if (lane >= k) incl += t;
    }
    const int excl = incl - cnt;
    int seg_lo[8], seg_off[8];   // wave-uniform: first concatenated index, slot - index
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      seg_lo[d] = __builtin_amdgcn_readlane(excl, d);
      seg_off[d] = __builtin_amdgcn_readlane(from, d) - seg_lo[d];
    }
    const int total_rec = __builtin_amdgcn_readlane(incl, 7);
    const GlobalF recs = (GlobalF)S.rec;
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
    for (int c0 = 0; c0 < total_rec; c0 += 64) {
      // lane j tests record c0 + j: does its stencil reach the block?
      const int g = min(c0 + lane, total_rec - 1);
      int off = seg_off[0];
#pragma unroll
      for (int d = 1; d < 8; ++d)
        if (g >= seg_lo[d]) off = seg_off[d];
      const int slot = off + g;
      const int pb = __float_as_int(recs[(int64_t)slot * kRec + 21]);
      const bool keep = c0 + lane < total_rec && (pb >> 20) + 2 >= ox && ((pb >> 10) & 1023) + 2 >= oy &&
                        (pb & 1023) + 2 >= oz;
      const uint64_t ball = __ballot(keep);
      // contribution of one record to the lane's node, or zero (branch-free)
      auto add = [&](const float (&rr)[22], bool use) {
        const int pbj = __float_as_int(rr[21]);
        const int di = lx - ((pbj >> 20) - ox), dj = ly - (((pbj >> 10) & 1023) - oy), dk = lz - ((pbj & 1023) - oz);
        const bool in = use && (unsigned)di <= 2u && (unsigned)dj <= 2u && (unsigned)dk <= 2u;
        const float a = (float)di, b = (float)dj, c = (float)dk;
        // q = rr[0..2], dx A = rr[3..11], weight polynomials rr[12..20]
        const float wp = (rr[12] + a * (rr[13] + rr[14] * a)) * (rr[15] + b * (rr[16] + rr[17] * b)) *
                         (rr[18] + c * (rr[19] + rr[20] * c));
        const float w = in ? wp : 0.f;
        acc0 += w * mp;
        acc1 += w * (rr[0] + rr[3] * a + rr[4] * b + rr[5] * c);
        acc2 += w * (rr[1] + rr[6] * a + rr[7] * b + rr[8] * c);
        acc3 += w * (rr[2] + rr[9] * a + rr[10] * b + rr[11] * c);
      };
      // the kept records, in lane order, into the wave's rows of LDS: each kept lane loads
      // its own record (all of them in flight together), then every lane reads them back
      // one by one (the same address for all lanes) and adds its node's contribution
      float* rows = &s_rec[wave][0][0];
      if (keep) {
        const int k = __builtin_amdgcn_mbcnt_hi((uint32_t)(ball >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0));
        const auto* src = (const __attribute__((address_space(1))) f32x4*)(S.rec + (int64_t)slot * kRec);
        f32x4 q[kRecVec];
#pragma unroll
        for (int i = 0; i < kRecVec; ++i) q[i] = src[i];
        f32x4* dst = reinterpret_cast<f32x4*>(rows + k * kGsRow);
#pragma unroll
        for (int i = 0; i < kRecVec; ++i) dst[i] = q[i];
      }
      wave_lds_sync();
      const int n_kept = __popcll(ball);
      for (int k = 0; k < n_kept; ++k) {
        const f32x4* row = reinterpret_cast<const f32x4*>(rows + k * kGsRow);
        float rr[22];
#pragma unroll
        for (int i = 0; i < 22; ++i) rr[i] = row[i >> 2][i & 3];
        add(rr, true);
      }
      wave_lds_sync();   // every lane has read the rows: the next chunk may rewrite them
    }
    const int ni = ox + lx, nj = oy + ly, nk = oz + lz;
    if (ni < n && nj < n && nk < n) {
      const double t_new = (double)(*S.step + 1) * S.dt_d;
      const float pm[3] = {acc1, acc2, acc3};
      float vel[3];
      node_velocity(S, acc0, pm, ni, nj, nk, t_new, vel);
      S.grid[((int64_t)ni * n + nj) * n + nk] = make_float4(vel[0], vel[1], vel[2], acc0);
    }
    s = sn;
    blk = bn;
  }
}

// ---- G2P + first Gauss-Newton chunk -------------------------------------------------
__global__ __launch_bounds__(kGnThreads) void g2p_gn_kernel(const SimDev* __restrict__ sims,
                                                            const BlockWork* __restrict__ work,
                                                            const int32_t* __restrict__ n_work) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const GnChunkLds<kGnThreads> sh(lds);
  const int tid = threadIdx.x;
  const int total = *n_work;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const BlockWork wk = work[b];
    const SimDev& S = sims[wk.sim];
    const int ns = S.n_samp;
    const int p = wk.p0 + tid;
    const int cnt = min(kGnChunk, ns - wk.p0);
    gn_stage_jacobian(S, S.J, wk.p0, cnt, sh);
    float v[3] = {0.f, 0.f, 0.f};
    if (tid < kGnChunk && p < ns) {
      float x[3];
      particle_x(S, p, plan_row(S)[p], x);
      const Stencil st = make_stencil(x, S.inv_dx, S.grid_n);
      if (st.ok) {
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
              const float4 g = S.grid[row + k];
              v[0] += w * g.x;
              v[1] += w * g.y;
              v[2] += w * g.z;
            }
          }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) S.vnew[c * ns + p] = v[c];
    }
    // iteration 0: u(z_n) - u^n vanishes, r = -dt v^{n+1}
    if (tid < kGnChunk) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sh.res(c, tid) = p < ns ? -S.dt_d * (double)v[c] : 0.0;
    }
    __syncthreads();
    gn_reduce_chunk(S, wk.p0, sh);
  }
}

// ---- full-order G2P, deformation update, return map, stress -------------------------
// Every particle (identity integration list) after P2G and the grid update: v and the
// APIC matrix C from the 27 stencil nodes, x += dt v (kept as the displacement u = x - X),
// F_trial = (I + dt C) F^E, then the return map of the sim's model and the stress of the
// new F^E for the next step's P2G (supplementary "Elasticity and plasticity details"):
// von Mises in log strain with fixed corotated stress, Drucker-Prager with the StVK
// stress in log strain, or Herschel-Bulkley (h = 1) with its own stress.
//
// The SVD F_trial = U S V^T comes from the symmetric eigen-decomposition
// F_trial^T F_trial = V S^2 V^T (cyclic Jacobi rotations, FP64). U is never formed: with
// G(h) = V diag(h) V^T, F^E = U diag(e^eps') V^T = F_trial G(e^eps' / S) and the polar
// rotation R = U V^T = F_trial G(1 / S), whatever basis Jacobi picks inside a repeated
// singular value.

// A = V diag(A_ii) V^T in place (A symmetric 3 x 3; on return A is diagonal to rounding).
__device__ void jacobi_eig3(double (&a)[3][3], double (&V)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 10; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-32 * dia)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      // rotation J in the (p, q) plane that zeroes a_pq: t = tan, the smaller root of
      // t^2 + 2 theta t - 1 = 0 with theta = (a_qq - a_pp) / (2 a_pq)
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double akp = a[k][p], akq = a[k][q];
        a[k][p] = c * akp - sn * akq;
        a[k][q] = sn * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double apk = a[p][k], aqk = a[q][k];
        a[p][k] = c * apk - sn * aqk;
        a[q][k] = sn * apk + c * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - sn * vkq;
        V[k][q] = sn * vkp + c * vkq;
      }
    }
  }
}

constexpr int kFoThreads = 256;

__global__ __launch_bounds__(kFoThreads) void fo_g2p_kernel(const SimDev* __restrict__ sim) {
  const SimDev& S = *sim;
  const int p = blockIdx.x * kFoThreads + threadIdx.x;
  if (p >= S.n_part) return;
  if (p == 0) *S.step += 1;
  const int n = S.grid_n;
  const int64_t P = S.n_part;
  float u[3], x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u[c] = S.u_n[c * P + p];
    x[c] = S.X[c * P + p] + u[c];
  }
  const Stencil st = make_stencil(x, S.inv_dx, n);
  if (!st.ok) {
    flag(S, FLAG_DOMAIN);
    return;
  }
  float v[3] = {0.f, 0.f, 0.f}, Cm[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float w = st.w[0][a] * st.w[1][b] * st.w[2][c];
        const float4 g = S.grid[((int64_t)(st.base[0] + a) * n + st.base[1] + b) * n + st.base[2] + c];
        const float vi[3] = {g.x, g.y, g.z};
        const float d[3] = {((float)a - st.f[0]) * S.dx, ((float)b - st.f[1]) * S.dx, ((float)c - st.f[2]) * S.dx};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          v[r] += w * vi[r];
#pragma unroll
          for (int k = 0; k < 3; ++k) Cm[3 * r + k] += w * vi[r] * d[k];
        }
      }
  const float k4 = 4.f * S.inv_dx * S.inv_dx;
#pragma unroll
  for (int e = 0; e < 9; ++e) Cm[e] *= k4;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    S.u_n[c * P + p] = u[c] + S.dt * v[c];
    S.u_prev[c * P + p] = v[c];
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) S.C[e * P + p] = Cm[e];
  // F_trial = (I + dt C) F^E
  double F[3][3], Ft[3][3];
#pragma unroll
  for (int e = 0; e < 9; ++e) F[e / 3][e % 3] = S.F[e * P + p];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double acc = F[r][c];
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += S.dt_d * (double)Cm[3 * r + k] * F[k][c];
      Ft[r][c] = acc;
    }
  double A[3][3], V[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) A[r][c] = Ft[0][r] * Ft[0][c] + Ft[1][r] * Ft[1][c] + Ft[2][r] * Ft[2][c];
  jacobi_eig3(A, V);
  double sig[3], eps[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    sig[i] = sqrt(fmax(A[i][i], 0.0));
    eps[i] = log(fmax(sig[i], 1e-12));
  }
  // return map: new log singular values eps (von Mises, Drucker-Prager) or the new
  // isochoric stretch bbar (Herschel-Bulkley), then F^E = U diag(sig_new) V^T
  const double mean = (eps[0] + eps[1] + eps[2]) / 3.0;
  const double eh[3] = {eps[0] - mean, eps[1] - mean, eps[2] - mean};
  const double norm = sqrt(eh[0] * eh[0] + eh[1] * eh[1] + eh[2] * eh[2]);
  double sn[3];      // singular values of the new F^E
  double tp[3];      // principal Kirchhoff stresses (log-strain and Herschel-Bulkley stresses)
  if (S.fo_model == 1) {
    // Drucker-Prager: expansion returns to Sigma = 1, outside the cone onto it
    const double tr = 3.0 * mean;
    const double dgamma = norm + S.fo_dp_k * tr;
    if (tr > 0.0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) eps[i] = 0.0;
    } else if (dgamma > 0.0 && norm > 0.0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) eps[i] -= dgamma * eh[i] / norm;
    }
    const double tre = eps[0] + eps[1] + eps[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sn[i] = exp(eps[i]);
      tp[i] = 2.0 * S.fo_mu * eps[i] + S.fo_lambda * tre;
    }
  } else if (S.fo_model == 2) {
    // Herschel-Bulkley: scale the deviator of bbar = J^(-2/3) S^2, keep det(bbar) = 1
    const double Jt = exp(3.0 * mean);
    const double j23 = exp(-2.0 * mean);
    double bb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) bb[i] = j23 * sig[i] * sig[i];
    const double bm = (bb[0] + bb[1] + bb[2]) / 3.0;
    double a[3] = {bb[0] - bm, bb[1] - bm, bb[2] - bm};
    const double st = S.fo_mu * sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (st > S.fo_hb_lim) {
      const double sc = (st - (st - S.fo_hb_lim) * S.fo_hb_relax) / st;
#pragma unroll
      for (int i = 0; i < 3; ++i) a[i] *= sc;
      // Newton on f(c) = prod(a_i + c) - 1, convex and increasing where every a_i + c > 0
      // (bm is there: a_i shrank towards 0); converges from either side of the root
      double c = bm;
      for (int it = 0; it < 40; ++it) {
        const double p0 = a[0] + c, p1 = a[1] + c, p2 = a[2] + c;
        const double f = p0 * p1 * p2 - 1.0;
        const double df = p1 * p2 + p0 * p2 + p0 * p1;
        const double dc = f / df;
        c -= dc;
        if (fabs(dc) <= 1e-15 * fabs(c)) break;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) bb[i] = a[i] + c;
    }
    const double bmn = (bb[0] + bb[1] + bb[2]) / 3.0;
    const double j13 = exp(mean);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sn[i] = j13 * sqrt(fmax(bb[i], 0.0));
      tp[i] = 0.5 * S.fo_kappa * (Jt * Jt - 1.0) + S.fo_mu * (bb[i] - bmn);
    }
  } else {
    // von Mises in log strain, yield test on the plastic multiplier
    const double dgamma = norm - S.fo_tau_y / (2.0 * S.fo_mu);
    if (dgamma > 0.0 && norm > 0.0)
#pragma unroll
      for (int i = 0; i < 3; ++i) eps[i] -= dgamma * eh[i] / norm;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sn[i] = exp(eps[i]);
      tp[i] = 0.0;
    }
  }
  double ge[3], gr[3], gt[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double si = fmax(sig[i], 1e-300);
    ge[i] = sn[i] / si;
    gr[i] = 1.0 / si;
    gt[i] = tp[i] / (si * si);
  }
  // F^E = Ft V diag(ge) V^T, R = Ft V diag(gr) V^T; for the principal-stress models
  // tau = U diag(tp) U^T = (Ft V) diag(tp / S^2) (Ft V)^T
  double FE[3][3], R[3][3], FV[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) FV[r][k] = Ft[r][0] * V[0][k] + Ft[r][1] * V[1][k] + Ft[r][2] * V[2][k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double me = 0.0, mr = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        me += FV[r][k] * ge[k] * V[c][k];
        mr += FV[r][k] * gr[k] * V[c][k];
      }
      FE[r][c] = me;
      R[r][c] = mr;
    }
  double tau[3][3];
  if (S.fo_model == 0) {
    // fixed corotated: tau = 2 mu (F^E - R) F^E^T + lambda (J - 1) J I
    const double J = sn[0] * sn[1] * sn[2];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += (FE[r][k] - R[r][k]) * FE[c][k];
        tau[r][c] = 2.0 * S.fo_mu * acc + (r == c ? S.fo_lambda * (J - 1.0) * J : 0.0);
      }
  } else {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        tau[r][c] = FV[r][0] * gt[0] * FV[c][0] + FV[r][1] * gt[1] * FV[c][1] + FV[r][2] * gt[2] * FV[c][2];
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) S.F[e * P + p] = FE[e / 3][e % 3];
  const double t6[6] = {tau[0][0], tau[1][1], tau[2][2], tau[1][2], tau[0][2], tau[0][1]};
#pragma unroll
  for (int c = 0; c < 6; ++c) S.tau[c * P + p] = (float)t6[c];
}

// ---- integration set: closure of the sample stencils (Sec. 5.4) ----------------------
// One closure sim per launch. Its integration list holds the samples in its first n_samp
// entries (they never move) and the other members after them, by ascending particle
// index. Positions are the decoded x = X + u(X, z_n) of every particle.

__device__ __forceinline__ void decoded_x(const SimDev& S, int p, float x[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] = S.xdec[(int64_t)c * S.n_part + p];
}

// a. I = the stencil nodes of the sample particles (a stencil that leaves the grid marks
// nothing; the MPM step flags that particle). One thread per stencil row (sample q, row
// 3a + b): its three nodes are consecutive bits, set with one or two atomic ORs.
__global__ __launch_bounds__(kAllocThreads) void closure_mark_kernel(const SimDev* __restrict__ sim) {
  const SimDev& S = *sim;
  const int n = S.grid_n;
  for (int t = blockIdx.x * kAllocThreads + threadIdx.x; t < 9 * S.n_samp; t += gridDim.x * kAllocThreads) {
    const int q = t / 9, row = t % 9;
    float x[3];
    decoded_x(S, S.nlist[q], x);
    const Stencil st = make_stencil(x, S.inv_dx, n);
    if (!st.ok) continue;
    const int node = ((st.base[0] + row / 3) * n + st.base[1] + row % 3) * n + st.base[2];
    const int w = node >> 5, sh = node & 31;
    atomicOr(&S.node_mask[w], 7u << sh);
    if (sh > 29) atomicOr(&S.node_mask[w + 1], 7u >> (32 - sh));
  }
}

// b. The particles other than the samples whose in-grid stencil meets I: a flag per
// particle and a count per workgroup. The three nodes of a stencil row are consecutive
// bits, read as one 64-bit window (the mask has a pad word at its end).
__global__ __launch_bounds__(kAllocThreads) void closure_member_kernel(const SimDev* __restrict__ sim) {
  const SimDev& S = *sim;
  const int n = S.grid_n;
  const int p = blockIdx.x * kAllocThreads + threadIdx.x;
  int m = 0;
  if (p < S.n_part && !S.is_sample[p]) {
    float x[3];
    decoded_x(S, p, x);
    const Stencil st = make_stencil(x, S.inv_dx, n);
    if (st.ok) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const int node = ((st.base[0] + a) * n + st.base[1] + b) * n + st.base[2];
          const uint64_t win = (uint64_t)S.node_mask[node >> 5] | ((uint64_t)S.node_mask[(node >> 5) + 1] << 32);
          m |= ((win >> (node & 31)) & 7u) != 0;
        }
    }
  }
  if (p < S.n_part) S.member[p] = (uint8_t)m;
  const int cnt = __syncthreads_count(m);
  if (threadIdx.x == 0) S.cl_block[blockIdx.x] = cnt;
}

// c. The members go after the samples in ascending index (workgroup offsets from the
// counts of the workgroups before it, then a workgroup scan); entries beyond the list's
// capacity are dropped and flagged. The last workgroup writes the live length; the mask
// is cleared for the next step.
__global__ __launch_bounds__(kAllocThreads) void closure_write_kernel(const SimDev* __restrict__ sim) {
  __shared__ int wave_sums[kAllocThreads / 64];
  const SimDev& S = *sim;
  const int tid = threadIdx.x;
  int before = 0;
  for (int b = tid; b < (int)blockIdx.x; b += kAllocThreads) before += S.cl_block[b];
  int base;
  (void)block_exclusive_scan(before, wave_sums, &base);
  const int p = blockIdx.x * kAllocThreads + tid;
  const int m = p < S.n_part ? S.member[p] : 0;
  int here;
  const int pos = block_exclusive_scan(m, wave_sums, &here);
  const int slot = S.n_samp + base + pos;
  if (m) {
    if (slot < S.n_int) S.nlist[slot] = p;
    else flag(S, FLAG_CAPACITY);
  }
  if (blockIdx.x == gridDim.x - 1 && tid == 0) *S.n_live = min(S.n_samp + base + here, S.n_int);
  for (int w = blockIdx.x * kAllocThreads + tid; w < S.mask_words; w += gridDim.x * kAllocThreads)
    S.node_mask[w] = 0u;
}

// d. The field jobs over the list evaluate its live part.
__global__ void closure_job_counts_kernel(const SimDev* __restrict__ sim, FieldJob* __restrict__ jobs,
                                          ListJobs lj) {
  const int k = threadIdx.x;
  if (k < lj.n) {
    FieldJob& j = jobs[lj.idx[k]];
    j.n = max(*sim->n_live - j.p_off, 0);
  }
}

}  // namespace

hipError_t launch_fo_g2p(const SimDev* sim, int64_t n_part, hipStream_t s) {
  if (n_part < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fo_g2p_kernel, dim3((unsigned)((n_part + kFoThreads - 1) / kFoThreads)), dim3(kFoThreads), 0, s,
                     sim);
  return hipGetLastError();
}

hipError_t launch_closure(const SimDev* sim, int n_samp, int64_t n_part, FieldJob* jobs,
                          ListJobs list_jobs, hipStream_t s) {
  if (n_samp < 1 || n_part < 1 || list_jobs.n < 0 || list_jobs.n > 4) return hipErrorInvalidValue;
  const int blocks = (int)((n_part + kAllocThreads - 1) / kAllocThreads);
  const int rows = 9 * n_samp;
  hipLaunchKernelGGL(closure_mark_kernel, dim3((rows + kAllocThreads - 1) / kAllocThreads), dim3(kAllocThreads), 0,
                     s, sim);
  hipLaunchKernelGGL(closure_member_kernel, dim3(blocks), dim3(kAllocThreads), 0, s, sim);
  hipLaunchKernelGGL(closure_write_kernel, dim3(blocks), dim3(kAllocThreads), 0, s, sim);
  hipLaunchKernelGGL(closure_job_counts_kernel, dim3(1), dim3(64), 0, s, sim, jobs, list_jobs);
  return hipGetLastError();
}

hipError_t launch_bin(const SimDev* sims, const BlockWork* work_int, const int32_t* n_work_int,
                      int32_t* claims, int grid_particles, bool batch, hipStream_t s) {
  if (grid_particles <= 0) return hipSuccess;
  hipLaunchKernelGGL(bin_kernel, dim3(grid_particles), dim3(kMpmBlock), 0, s, sims, work_int, n_work_int, claims,
                     batch ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_p2g_after_bin(const SimDev* sims, const int32_t* n_sims, int grid_sims,
                                const BlockWork* work_int, const int32_t* n_work_int, int grid_particles,
                                int grid_blocks, bool dense, int max_grid_n, bool place, bool batch,
                                hipStream_t s) {
  constexpr int alloc_lds = kMaxBins * 4;
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)alloc_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             alloc_lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(alloc_kernel, dim3(grid_sims), dim3(kAllocThreads), alloc_lds, s, sims, n_sims);
  if (place)
    hipLaunchKernelGGL(place_kernel, dim3(grid_particles), dim3(kMpmBlock), 0, s, sims, work_int, n_work_int);
  const bool full = batch && !dense;   // the records the wave-per-block gather reads
  if (full) hipLaunchKernelGGL(bin_sort_kernel<6>, dim3(grid_blocks), dim3(kSortThreads), 0, s, sims, n_sims);
  else hipLaunchKernelGGL(bin_sort_kernel<4>, dim3(grid_blocks), dim3(kSortThreads), 0, s, sims, n_sims);
  // Dense sets (closure, full order) and a single sparse sim: one workgroup per node block
  // (4^3-node blocks, one node per lane, up to 128^3 grids, 8^3 above). Batches of sparse
  // sims: one wave per 4^3-node block over a list of every sim's blocks, with the
  // workgroup variant for the sims on grids above 128^3.
  const bool small = max_grid_n <= 128;
  if (dense && small)
    hipLaunchKernelGGL((gather_kernel<kGatherThreadsDense, 1>), dim3(grid_blocks), dim3(kGatherThreadsDense), 0, s,
                       sims, n_sims, 0);
  else if (dense)
    hipLaunchKernelGGL((gather_kernel<kGatherThreadsDense, kMaxNodesPerLane>), dim3(grid_blocks),
                       dim3(kGatherThreadsDense), 0, s, sims, n_sims, 0);
  else if (!batch && small)
    hipLaunchKernelGGL((gather_kernel<kGatherThreads, 1>), dim3(grid_blocks), dim3(kGatherThreads), 0, s, sims,
                       n_sims, 0);
  else {
    hipLaunchKernelGGL(gather_lanes_kernel, dim3(2 * grid_blocks), dim3(kGsThreads), 0, s, sims, n_sims);
    if (!small)
      hipLaunchKernelGGL((gather_kernel<kGatherThreads, kMaxNodesPerLane>), dim3(grid_blocks), dim3(kGatherThreads),
                         0, s, sims, n_sims, 8);
  }
  return hipGetLastError();
}

hipError_t launch_g2p_gn(const SimDev* sims, const BlockWork* work_gn, const int32_t* n_work_gn,
                         int r_cap, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (r_cap < 1 || r_cap > kMaxR) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)g2p_gn_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             gn_chunk_lds_bytes(kGnThreads, kMaxR));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(g2p_gn_kernel, dim3(grid), dim3(kGnThreads), gn_chunk_lds_bytes(kGnThreads, r_cap), s,
                     sims, work_gn, n_work_gn);
  return hipGetLastError();
}

}  // namespace nsf
