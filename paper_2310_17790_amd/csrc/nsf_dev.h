// Device-side data structures shared by the library's kernels and host orchestration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsf {

constexpr int kMaxR = 32;          // largest latent dimension
constexpr int kGnChunk = 128;      // sample points per Gauss-Newton reduction block
constexpr int kGnThreads = 256;    // threads of a Gauss-Newton reduction block
constexpr int kClaimCounters = 8;  // work-claim counters of the field kernels, zeroed per step
constexpr int kMpmBlock = 256;     // particles per P2G / G2P block
// up to this many integration particles the slot allocation places them itself; above
// it a separate pass does (launch_p2g_after_bin's `place`)
constexpr int kAllocByParticles = 32768;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Packed parameters of one field (one MLP), all in device memory. See pack.cpp for how
// the host builds each array from the row-major masters.
struct FieldPack {
  const float* w1q;      // layer 1 incl. bias column: [W/16][K1q][64] 16x16x4 A operands
  const float* whp;      // FP32 hidden layers 2..5: [4][W/16][W/8][64][2]
  const bf16x8* whb;     // BF16 hidden layers 2..5: [4][W/16][W/32][64]
  const float* bhq;      // hidden biases, plain order: [4][W]
  const float* w6q;      // output weights, plain order: [d][W]
  const float* b6;       // output bias [d]
  // reverse-mode Jacobian (deformation field): transposed hidden layers in the layouts of
  // whp / whb, and layer 1's latent columns as an r x W matrix [ceil(r/16)][W/8][64][2]
  const float* whpt;
  const bf16x8* whbt;
  const float* w1zt;
};

// One batch of MLP evaluations: a field at one latent over a list of points.
struct FieldJob {
  FieldPack w;
  const double* z;           // device latent (r)
  const float* X;            // reference positions SoA, leading dimension ldx
  const int32_t* idx;        // gather list (NULL: point index is the row of X)
  const int64_t* step;       // if non-NULL, idx += ((step + step_off) mod plan_steps) * plan_ld
  int64_t ldx;
  int32_t plan_steps, plan_ld;
  int32_t p_off;             // point p of this job reads list entry p_off + p
  int32_t n;                 // number of points (a closure sim's jobs over N: rewritten on
                             // the device each step from the list's live length)
  int32_t r, d;
  int32_t mode;              // 0: out = field; 1: out = X + field (decode)
  int32_t jvp;               // 1: directional derivative job (see z2)
  const double* z2;          // jvp: evaluate at (z + z2) / 2 with the one tangent along
                             // z - z2, and write scale * (tangent output) * jvp_scale
  float jvp_scale;
  int32_t step_off;          // 1: the points of the step after the counter's (see step)
  int32_t saved_bf16;        // training: saved holds BF16 values (else FP32)
  const float* zrows;        // training: per-point latents [n][r] instead of z (NULL in the step)
  float* saved;              // training: pre-activations of layers 1..5, [5][n][W] (or NULL)
  float* out; int64_t ldo;   // SoA [d][ldo], already offset to this job's first point
  float* jac; int64_t ldj;   // SoA [3 r][ldj] (row c*r + j), only for d = 3
  float scale[9], shift[9];
};

// One workgroup's work: WPG consecutive 16-point tiles of a job starting at point p0
// (wave w takes p0 + 16 w), the primal plus tangents [t0, t0 + nt) (only groups with
// t0 == 0 write the primal output), or with nt < 0 the primal and Jacobian row t0 in
// reverse mode (the t0 == 0 group writes the primal output).
struct FieldTile {
  int32_t job, p0, t0, nt;
};

// Per-simulation constants and device pointers (lives in the sim's arena and is copied
// into batch tables).
struct SimDev {
  int32_t r, n_part, n_int, n_samp;
  int32_t plan_steps, grid_n, wall, gn_iters;
  int32_t knife_on, n_gn_chunks, width;
  int32_t pipelined_decode;          // 1: the step's first kernel snapshots z_n into zdec
  int32_t tangent_forms;             // 1 (BF16): velocity stored directly in u_prev (a JVP)
                                     // and trapezoid Gauss-Newton residuals from Jacobians
  float dx, inv_dx, dt, mp;          // mp = particle mass rho V_p
  float stress_k;                    // dt V_p 4 / dx^2
  float grav[3];
  double dt_d, dx_d;
  double gn_damping;                 // lambda: Gauss-Newton solves use H + lambda diag(H)
  double grav_d[3];
  double kn[3], koff, khalf, kz0, kspeed, kv[3];
  const float* X;                    // [3][n_part]
  const int32_t* plan;               // [plan_steps][n_int]
  float* u_n;                        // [3][n_int]
  float* u_prev;                     // [3][n_int]
  float* tau;                        // [6][n_int]
  float* C;                          // [9][n_int]
  float* J;                          // [3r][n_samp]  at z_n
  float* vnew;                       // [3][n_samp]
  float* u_gn;                       // [3][n_samp]   at the Gauss-Newton iterate
  float* J2;                         // [3r][n_samp]  at the Gauss-Newton iterate
  float* xdec;                       // [3][n_part]
  float4* grid;                      // [grid_n^3] (m, p_x, p_y, p_z)
  double* z;                         // [3][r]: z_{n-1}, z_n, iterate
  double* zdec;                      // [r]: the latent a pipelined decode reads
  double* zh;                        // [r + n_mu]: (z_n, mu), the stress field's input
                                     // after X (NULL without problem parameters)
  int64_t* step;
  uint32_t* flags;
  double* gn_part;                   // [n_gn_chunks][E], E = r(r+1)/2 + r
  // particle binning for the gather-form P2G: bins of bin_edge^3 cells, nbs per axis
  int32_t bin_edge, nbs, n_bins, pad2;
  int32_t* bin_cnt;                  // [n_bins] particles per bin (zero between steps)
  int4* bin_meta;                    // [n_bins] (epoch in which it was set, first record slot,
                                     // record count, unused) of each bin
  int32_t* epoch;                    // binning epoch, +1 every step
  int32_t* pbin;                     // [n_int] bin of each integration particle, -1 if off-grid
  int32_t* prank;                    // [n_int] slot of the particle inside its bin
  float* rec;                        // [n_int][16] P2G records, each bin contiguous
  float* rec_p;                      // [n_int][16] P2G records in particle order (binning)
  int32_t* sorted;                   // [n_int] particle indices, each bin contiguous
  int32_t* active;                   // [n_bins] node blocks that receive mass this step
  int32_t* nonempty;                 // [n_bins] bins holding particles this step
  int32_t* n_active;                 // [2]: active node blocks, non-empty bins
  // closure integration set (closure = 1): the integration list `nlist` (the plan's single
  // row, samples first) is rebuilt every step from the decoded positions
  int32_t closure, mask_words;
  int32_t* nlist;                    // [n_int] writable alias of plan
  int32_t* n_live;                   // [1] live length of nlist (NULL: n_int, fixed)
  uint32_t* node_mask;               // [mask_words] grid nodes in a sample stencil (+1 pad word)
  uint8_t* is_sample;                // [n_part]
  uint8_t* member;                   // [n_part] member of N \ S this step
  int32_t* cl_block;                 // [ceil(n_part / 1024)] members per workgroup
  // full-order sims (every particle integrated; the reduced buffers hold the state:
  // u_n = x - X, u_prev = v with tangent_forms = 1, tau, C)
  int32_t ground, pad3;              // 1: the bottom wall layers only keep v_z >= 0
  double* F;                         // [9][n_part] elastic deformation gradient
  double fo_mu, fo_lambda, fo_tau_y;  // Lame parameters and yield stress
  int32_t fo_model, pad4;            // return map: 0 von Mises, 1 Drucker-Prager, 2 Herschel-Bulkley
  double fo_kappa;                   // bulk modulus (Herschel-Bulkley stress)
  double fo_dp_k;                    // Drucker-Prager: alpha (3 lambda + 2 mu) / (2 mu)
  double fo_hb_lim, fo_hb_relax;     // Herschel-Bulkley: sqrt(2/3) tau_y, 1 / (1 + eta / (2 mu dt))
};

// Integration particles this step: the live length of a closure list, else n_int.
__device__ __forceinline__ int live_count(const SimDev& S) { return S.n_live ? *S.n_live : S.n_int; }

enum : uint32_t { FLAG_DOMAIN = 1u, FLAG_NONFINITE = 2u, FLAG_SINGULAR = 4u, FLAG_CAPACITY = 8u };

// Work item of a per-particle MPM kernel or a Gauss-Newton reduction block.
struct BlockWork {
  int32_t sim, p0;
};

// ---- launchers (defined in the .hip files) ----
// Group kinds a table holds besides primal groups (launch_fields_table's `kinds`, for
// tc > 0): tangent or one-wave reverse groups (nt > 0, nt == -1), team groups (nt -2, -3;
// kTableTeamOne: the team groups take one tile, nt = -3; a table holds one kind of them).
enum : int { kTableTangents = 1, kTableTeam = 2, kTableTeamOne = 4 };
hipError_t launch_fields_table(int width, bool bf16, int tc, int kinds, const FieldJob* jobs,
                               const FieldTile* groups, const int32_t* n_groups, int32_t* claim,
                               int grid, hipStream_t s);
int fields_table_blocks_per_cu(int width, bool bf16, int tc);
hipError_t launch_reset_counters(int32_t* c, int n, hipStream_t s);   // n <= 64
// One job over n points with persistent workgroups; `beside` = the launch runs next to the
// step's own kernels (a pipelined decode) and leaves them three eighths of the CUs.
hipError_t launch_fields_dense(int width, bool bf16, const FieldJob& job, int n_points,
                               hipStream_t s, bool beside = false);
// BF16 decode over a table of primal groups (one tile per wave of a 16-wave workgroup) whose
// jobs each have their own weight set, one workgroup per CU over `cus` CUs, weights resident
// in LDS: every job must take the single-job decode's LDS-parameter form (no per-point
// latents, no tangent direction, no saved pre-activations, d <= 9).
hipError_t launch_fields_decode_table(int width, const FieldJob* jobs, const FieldTile* groups,
                                      const int32_t* n_groups, int cus, hipStream_t s);
int fields_max_tangents(int width, bool bf16);
int fields_group_points(int tc);  // points one work group (table entry) spans
// Jacobians with more latent columns than forward mode carries take one workgroup per
// fields_team_points(nt) points (FieldTile.nt = -2: two 16-point tiles, -3: one) in this
// configuration; such a group also evaluates up to three more jobs over the same points,
// forward only (FieldTile.t0: their job offsets from FieldTile.job, one signed byte each,
// 0 = none)
bool fields_team_jacobian(int width, bool bf16);
int fields_team_points(int nt);

// MPM transfers: bin (per integration particle; also zeroes the step's claim counters and,
// for pipelined decodes, snapshots z_n), then allocate and place (per sim), sort and write
// records (per non-empty bin), gather + grid update (per active node block).
hipError_t launch_bin(const SimDev* sims, const BlockWork* work_int, const int32_t* n_work_int,
                      int32_t* claims, int grid_particles, bool batch, hipStream_t s);
// dense: the integration particles fill their cells (closure sims): wider gather
// workgroups. max_grid_n bounds grid_n of every sim the launch can see; place: some sim
// may have more than kAllocByParticles integration particles; batch: the launch may serve
// more than one sim (a batch plan).
hipError_t launch_p2g_after_bin(const SimDev* sims, const int32_t* n_sims, int grid_sims,
                                const BlockWork* work_int, const int32_t* n_work_int, int grid_particles,
                                int grid_blocks, bool dense, int max_grid_n, bool place, bool batch,
                                hipStream_t s);
// G2P at the sample particles fused with the first Gauss-Newton reduction: work items are
// Gauss-Newton chunks (kGnChunk sample particles). r_cap (<= kMaxR) bounds the latent size
// of every sim in the launch and sizes the chunk's LDS.
hipError_t launch_g2p_gn(const SimDev* sims, const BlockWork* work_gn, const int32_t* n_work_gn,
                         int r_cap, int grid, hipStream_t s);
constexpr int kSegMax = 2048;  // bin segments up to this size are summed in index order
constexpr int kMaxBatchSims = 1024;  // sims one batched launch serves
// Gauss-Newton: chunk reduction of iteration iter >= 1, and the per-sim solve of any iteration.
hipError_t launch_gn_partial(const SimDev* sims, const BlockWork* work, const int32_t* n_work,
                             int iter, int r_cap, int grid, hipStream_t s);
hipError_t launch_gn_solve(const SimDev* sims, const int32_t* n_sims, int iter, int grid_sims,
                           hipStream_t s);
// Full-order step after P2G: G2P of v and C for every particle, x += dt v, F update,
// return map and the stress of the next step.
hipError_t launch_fo_g2p(const SimDev* sim, int64_t n_part, hipStream_t s);

// Integration set of one closure sim from its decoded positions: mark the samples' stencil
// nodes, flag and count the members, write the list and its live length, and set the
// point count of the field jobs over the list (jobs[idx[k]].n = live - p_off).
struct ListJobs {
  int32_t idx[4];
  int32_t n;
};
hipError_t launch_closure(const SimDev* sim, int n_samp, int64_t n_part, FieldJob* jobs,
                          ListJobs list_jobs, hipStream_t s);

}  // namespace nsf
