// C ABI of the latent-step library: descriptor validation, arena layout, weight packing,
// work tables and step orchestration (one HIP graph per stepped set of simulations).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cassert>
#include <initializer_list>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "nsf.h"
#include "nsf_dev.h"
#include "pack.h"

using namespace nsf;

namespace {

thread_local std::string g_err;

nsf_status fail(nsf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define NSF_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(NSF_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
const int kFieldOut[3] = {3, 6, 9};

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

// Byte offsets of every buffer of a sim inside its arena.
struct Layout {
  size_t simdev;
  size_t whp[3], whb[3], b6[3], w1q[3], bhq[3], w6q[3], whpt[3], whbt[3], w1zt[3];
  size_t X, plan, u_n, u_prev, tau, C, J, vnew, u_gn, J2, xdec, grid, z, zdec, zh, step, flags, gn_part;
  size_t bin_cnt, bin_meta, epoch, pbin, prank, rec, rec_p, sorted, active,
      nonempty, n_active;
  size_t node_mask, is_sample, member, cl_block, n_live;   // closure integration only
  size_t total;
};

int gn_entries(int r) { return r * (r + 1) / 2 + r; }
// inputs after X of field f: the latent, and for the stress field the problem parameters
int field_r(const nsf_sim_desc* d, int f) { return d->r + (f == NSF_FIELD_H ? d->n_mu : 0); }
// node bitmask of a closure sim: one bit per node plus a pad word (the membership test
// reads two consecutive words)
size_t mask_words(int grid_n) { return ((size_t)grid_n * grid_n * grid_n + 31) / 32 + 1; }
// P2G bins: cubes of bin_edge^3 cells, at most 32 per axis
int bin_edge(int grid_n) { return grid_n <= 128 ? 4 : 8; }
int bins_per_axis(int grid_n) { return (grid_n + bin_edge(grid_n) - 1) / bin_edge(grid_n); }

Layout make_layout(const nsf_sim_desc* d) {
  Layout L{};
  Carver c;
  const int r = d->r, W = d->width;
  const int64_t P = d->n_particles, N = d->n_integration, S = d->n_sample;
  L.simdev = c.take(sizeof(SimDev));
  for (int f = 0; f < 3; ++f) {
    const PackSizes ps = pack_sizes(field_r(d, f), W, kFieldOut[f]);
    L.whp[f] = c.take(ps.whp * 4);
    L.whb[f] = c.take(ps.whb * 2);
    L.b6[f] = c.take(ps.b6 * 4);
    L.w1q[f] = c.take(ps.w1q * 4);
    L.bhq[f] = c.take(ps.bhq * 4);
    L.w6q[f] = c.take(ps.w6q * 4);
    L.whpt[f] = c.take(ps.whp * 4);
    L.whbt[f] = c.take(ps.whb * 2);
    L.w1zt[f] = c.take(ps.w1zt * 4);
  }
  L.X = c.take((size_t)3 * P * 4);
  L.plan = c.take((size_t)d->plan_steps * N * 4);
  L.u_n = c.take((size_t)3 * N * 4);
  L.u_prev = c.take((size_t)3 * N * 4);
  L.tau = c.take((size_t)6 * N * 4);
  L.C = c.take((size_t)9 * N * 4);
  L.J = c.take((size_t)3 * r * S * 4);
  L.vnew = c.take((size_t)3 * S * 4);
  L.u_gn = c.take((size_t)3 * S * 4);
  L.J2 = c.take((size_t)3 * r * S * 4);
  L.xdec = c.take((size_t)3 * P * 4);
  const size_t n3 = (size_t)d->grid_n * d->grid_n * d->grid_n;
  L.grid = c.take(n3 * 16);
  L.z = c.take((size_t)3 * r * 8);
  L.zdec = c.take((size_t)r * 8);
  if (d->n_mu > 0) L.zh = c.take((size_t)(r + d->n_mu) * 8);
  L.step = c.take(8);
  L.flags = c.take(4);
  L.gn_part = c.take((size_t)ceil_div(S, kGnChunk) * gn_entries(r) * 8);
  const int nbs = bins_per_axis(d->grid_n);
  const size_t nb = (size_t)nbs * nbs * nbs;
  L.bin_cnt = c.take(nb * 4);
  L.bin_meta = c.take(nb * 16);
  L.epoch = c.take(4);
  L.pbin = c.take((size_t)N * 4);
  L.prank = c.take((size_t)N * 4);
  L.rec = c.take((size_t)N * 128);
  L.rec_p = c.take((size_t)N * 128);
  L.sorted = c.take((size_t)N * 4);
  L.active = c.take(nb * 4);
  L.nonempty = c.take(nb * 4);
  L.n_active = c.take(8);
  if (d->integration == NSF_INTEGRATION_CLOSURE) {
    L.node_mask = c.take((mask_words(d->grid_n)) * 4);
    L.is_sample = c.take((size_t)P);
    L.member = c.take((size_t)P);
    L.cl_block = c.take((size_t)ceil_div(P, 1024) * 4);
    L.n_live = c.take(4);
  }
  L.total = c.off;
  return L;
}

nsf_status validate(const nsf_sim_desc* d) {
  if (!d) return fail(NSF_EINVAL, "descriptor is NULL");
  if (d->r < 1 || d->r > kMaxR) return fail(NSF_EINVAL, "r = %d outside 1..%d", d->r, kMaxR);
  if (d->width != 64 && d->width != 128) return fail(NSF_EINVAL, "width = %d (64 or 128)", d->width);
  if (d->n_hidden != 5) return fail(NSF_EINVAL, "n_hidden = %d (the fields have 5 hidden layers)", d->n_hidden);
  if (d->precision != NSF_FP32 && d->precision != NSF_BF16 && d->precision != NSF_BF16_MIXED)
    return fail(NSF_EINVAL, "unknown precision");
  for (int f = 0; f < 3; ++f)
    if (!d->weights[f]) return fail(NSF_EINVAL, "weights[%d] is NULL", f);
  if (d->n_particles < 1 || d->n_particles > (int64_t)INT32_MAX / 4)
    return fail(NSF_EINVAL, "n_particles = %lld", (long long)d->n_particles);
  if (!d->X) return fail(NSF_EINVAL, "X is NULL");
  if (d->n_integration < 1 || d->n_integration > d->n_particles)
    return fail(NSF_EINVAL, "n_integration = %d must be in 1..n_particles", d->n_integration);
  if (d->n_sample < 1 || d->n_sample > d->n_integration)
    return fail(NSF_EINVAL, "n_sample = %d must be in 1..n_integration", d->n_sample);
  if (3 * (int64_t)d->n_sample < d->r)
    return fail(NSF_EINVAL, "n_sample = %d < r / 3: the inversion is under-determined", d->n_sample);
  if (d->plan_steps < 1 || !d->sample_plan) return fail(NSF_EINVAL, "sample_plan missing");
  if (d->grid_n < 8 || d->grid_n > 256) return fail(NSF_EINVAL, "grid_n = %d outside 8..256", d->grid_n);
  if (!(d->dx > 0) || !(d->dt > 0)) return fail(NSF_EINVAL, "dx and dt must be positive");
  if (!(d->rho > 0) || !(d->body_volume > 0)) return fail(NSF_EINVAL, "rho and body_volume must be positive");
  if (d->wall_nodes < 0 || 2 * d->wall_nodes >= d->grid_n) return fail(NSF_EINVAL, "wall_nodes = %d", d->wall_nodes);
  if (d->gn_iters < 1 || d->gn_iters > 4) return fail(NSF_EINVAL, "gn_iters = %d outside 1..4", d->gn_iters);
  if (!(d->gn_damping >= 0.0 && d->gn_damping <= 1e6))
    return fail(NSF_EINVAL, "gn_damping = %g outside [0, 1e6]", d->gn_damping);
  if (d->decode_every_step < 0 || d->decode_every_step > 2)
    return fail(NSF_EINVAL, "decode_every_step = %d (0, 1 or 2)", d->decode_every_step);
  if (d->n_mu < 0 || d->n_mu > 4 || d->r + d->n_mu > kMaxR)
    return fail(NSF_EINVAL, "n_mu = %d (0..4, r + n_mu <= %d)", d->n_mu, kMaxR);
  for (int i = 0; i < d->n_mu; ++i)
    if (!std::isfinite(d->mu[i])) return fail(NSF_EINVAL, "mu[%d] is not finite", i);
  if (d->integration != NSF_INTEGRATION_PLAN && d->integration != NSF_INTEGRATION_CLOSURE)
    return fail(NSF_EINVAL, "integration = %d (0 plan, 1 closure)", d->integration);
  const bool closure = d->integration == NSF_INTEGRATION_CLOSURE;
  if (closure && d->precision == NSF_BF16_MIXED)
    return fail(NSF_EINVAL, "closure integration runs in FP32 or BF16, not BF16_MIXED");
  if (closure) {
    if (d->plan_steps != 1) return fail(NSF_EINVAL, "closure integration takes one sample row (plan_steps = 1)");
    if (d->decode_every_step != 1)
      return fail(NSF_EINVAL, "closure integration needs decode_every_step = 1 (it reads the decoded positions)");
  }
  if (!d->z0) return fail(NSF_EINVAL, "z0 is NULL");
  for (int j = 0; j < d->r; ++j)
    if (!std::isfinite(d->z0[j]) || (d->z_prev && !std::isfinite(d->z_prev[j])))
      return fail(NSF_EINVAL, "initial latent is not finite");
  const int64_t cnt = closure ? d->n_sample : (int64_t)d->plan_steps * d->n_integration;
  for (int64_t i = 0; i < cnt; ++i)
    if (d->sample_plan[i] < 0 || d->sample_plan[i] >= d->n_particles)
      return fail(NSF_EINVAL, "sample_plan[%lld] = %d out of range", (long long)i, d->sample_plan[i]);
  // a particle listed twice in one step's list would be integrated twice (its mass and
  // momentum counted twice in P2G, its residual twice in the inversion)
  std::vector<int32_t> seen((size_t)d->n_particles, -1);   // last row that listed the particle
  const int64_t row_len = closure ? d->n_sample : d->n_integration;
  for (int64_t i = 0; i < cnt; ++i) {
    const int32_t row = (int32_t)(i / row_len), p = d->sample_plan[i];
    if (seen[p] == row)
      return closure ? fail(NSF_EINVAL, "sample particle %d listed twice", p)
                     : fail(NSF_EINVAL, "particle %d listed twice in sample_plan row %d", p, row);
    seen[p] = row;
  }
  return NSF_OK;
}

bool device_ok(std::string* why) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
    if (why) *why = "no HIP device visible";
    return false;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    if (why) *why = "cannot query the current HIP device";
    return false;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    if (why) *why = std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950";
    return false;
  }
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------------------
struct Plan;

struct nsf_sim {
  int device = 0;
  int r = 0, width = 0;
  bool bf16 = false;       // deformation field where the inversion reads it (BF16 precision)
  bool bf16_hl = false;    // stress and affine fields and the decode (BF16 and BF16_MIXED)
  int64_t n_part = 0;
  int n_int = 0, n_samp = 0, gn_iters = 2;
  int decode_mode = 0;    // decode_every_step: 0, 1 or 2 (pipelined)
  bool closure = false;   // integration set = closure of the sample stencils
  int n_mu = 0;           // problem parameters of the stress field
  std::vector<int32_t> samples;   // closure: the sample list given at creation
  char* arena = nullptr;
  size_t arena_bytes = 0;
  Layout L{};
  SimDev hd{};            // host copy of the device constants
  SimDev* dd = nullptr;   // device copy in the arena
  FieldPack pack[3]{};
  float scale[3][9]{}, shift[3][9]{};
  std::unique_ptr<Plan> solo;
  // The step's field inference for the current latent is in the sim's buffers (the
  // previous step computed it at its end); false after create and set_latent.
  bool inference_ready = false;
};

// Work tables and the captured step graph for one ordered set of sims. A batch plan
// (persistent=true) launches every kernel with a fixed grid that loops over device-side
// work counts, so when the set of sims changes only the tables are rewritten in place
// and the captured graph is replayed unchanged.
struct Plan {
  std::vector<nsf_sim*> members;
  int width = 0, gn_iters = 0, tc = 0;
  int r_cap = kMaxR;             // largest latent the Gauss-Newton chunk kernels serve
  int grid_cap = 256;            // largest grid_n the P2G kernels serve
  bool place = true;             // some member may exceed kAllocByParticles integration particles
  bool bf16 = false, decode = false, pipelined = false, persistent = false;
  bool bf16_hl = false;           // precision of the h and l jobs and of the decode
  bool mixed = false;             // bf16_hl != bf16: h and l run in a table of their own
  int nH = 0;                     // groups of that table
  bool closure = false;           // its one member rebuilds its integration set every step
  ListJobs list_jobs{};           // closure: the jobs over the integration list
  void* dbuf = nullptr;
  size_t dcap = 0;
  void* staging = nullptr;        // pinned host copy of the tables (persistent plans)
  std::vector<size_t> caps;       // byte capacity of each table region
  int32_t* d_counts = nullptr;    // [0..7] work counts, [8..15] claim counters
  SimDev* d_sims = nullptr;
  FieldJob* d_jobs = nullptr;
  FieldTile *d_tA = nullptr, *d_tG = nullptr, *d_tD = nullptr, *d_tH = nullptr;
  BlockWork *d_bP = nullptr, *d_bGN = nullptr;
  int nA = 0, nG = 0, nD = 0, nP = 0, nGN = 0, nsims = 0;
  int nAstep = 0, nGnext = 0;     // see build_plan (velocity job moved into the first G pass)
  int nGvel = 0;                  // velocity groups at the start of the G table
  int kindsA = kTableTangents, kindsG = kTableTangents;   // group kinds of the A and G tables
  // launch grids (fixed for persistent plans)
  int gF = 0, gF0 = 0, gP = 0, gGN = 0, gSims = 0, gBlk = 0, gH = 0;
  FieldJob decode_job{};          // single-sim plans decode with the dense kernel
  // Decode runs on a side stream, concurrently with the next step's inference.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // graphs of one step and of kGraphSteps steps (long runs launch the latter: each graph
  // launch costs some microseconds between the last kernel of one and the first of the next)
  hipGraph_t graph = nullptr, graph_n = nullptr;
  hipGraphExec_t exec = nullptr, exec_n = nullptr;
  void drop_graphs() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (exec_n) (void)hipGraphExecDestroy(exec_n);
    if (graph_n) (void)hipGraphDestroy(graph_n);
    exec = exec_n = nullptr;
    graph = graph_n = nullptr;
  }
  ~Plan() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    drop_graphs();
    if (dbuf) (void)hipFree(dbuf);
    if (staging) (void)hipHostFree(staging);
  }
};

namespace {

std::mutex g_plans_mu;
// One persistent batch plan per (width, precision, Gauss-Newton iterations, decode mode);
// its tables are rewritten when the set of stepped sims changes.
std::map<int, std::unique_ptr<Plan>> g_batch_plans;

int batch_signature(const nsf_sim* s) {
  return s->width * 256 + (s->bf16 ? 32 : 0) + (s->bf16_hl ? 128 : 0) + s->gn_iters * 4 + s->decode_mode;
}

FieldJob base_job(const nsf_sim* s, int field, const double* z) {
  FieldJob j{};
  j.w = s->pack[field];
  j.z = z;
  j.X = s->hd.X;
  j.ldx = s->n_part;
  j.idx = s->hd.plan;
  j.step = s->hd.step;
  j.plan_steps = s->hd.plan_steps;
  j.plan_ld = s->n_int;
  j.r = s->r;
  j.d = kFieldOut[field];
  for (int c = 0; c < 9; ++c) {
    j.scale[c] = s->scale[field][c];
    j.shift[c] = s->shift[field][c];
  }
  return j;
}

// Groups of one job over n points: primal only (ntan = 0), or with the Jacobian's ntan
// latent columns. Forward mode takes ceil(ntan / tc) groups per span of points, each
// recomputing the primal; reverse mode (FieldTile.nt < 0, t0 = output component) takes
// one group per output component and pays off once forward mode needs more than two.
bool reverse_jacobian(int ntan, int tc) { return ntan > 2 * tc; }

// A team group's extra jobs (at most three, forward only over the group's points) as
// FieldTile.t0: signed byte offsets from the group's job.
int32_t team_extras(int job, std::initializer_list<int> extra) {
  uint32_t code = 0;
  int i = 0;
  for (int x : extra) {
    const int dj = x - job;
    assert(i < 3 && dj != 0 && dj >= -128 && dj <= 127);
    code |= (uint32_t)(uint8_t)(int8_t)dj << (8 * i++);
  }
  return (int32_t)code;
}

void add_tiles(std::vector<FieldTile>& out, int job, int n, int ntan, int tc, bool team = false,
               int32_t extras = 0, int team_nt = -2) {
  if (team && reverse_jacobian(ntan, tc)) {   // one workgroup per fields_team_points() points
    for (int p0 = 0; p0 < n; p0 += fields_team_points(team_nt)) out.push_back({job, p0, extras, team_nt});
    return;
  }
  const int span = fields_group_points(ntan > 0 ? tc : 0);
  for (int p0 = 0; p0 < n; p0 += span) {
    if (ntan == 0) {
      out.push_back({job, p0, 0, 0});
    } else if (reverse_jacobian(ntan, tc)) {
      for (int c = 0; c < 3; ++c) out.push_back({job, p0, c, -1});
    } else {
      for (int t0 = 0; t0 < ntan; t0 += tc) out.push_back({job, p0, t0, std::min(tc, ntan - t0)});
    }
  }
}

// Primal-only groups that run in the tangent kernel (same workgroup shape as its
// Jacobian groups).
void add_prim_tiles(std::vector<FieldTile>& out, int job, int n, int tc) {
  const int span = fields_group_points(tc);
  for (int p0 = 0; p0 < n; p0 += span) out.push_back({job, p0, 0, 0});
}

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// Build the work tables of P.members into one blob and install it in P's device buffer.
nsf_status build_plan(Plan& P, hipStream_t stream) {
  nsf_sim* s0 = P.members[0];
  P.width = s0->width;
  P.bf16 = s0->bf16;
  P.bf16_hl = s0->bf16_hl;
  P.mixed = P.bf16 != P.bf16_hl;
  P.gn_iters = s0->gn_iters;
  P.decode = s0->decode_mode != 0;
  P.pipelined = s0->decode_mode == 2;
  P.closure = s0->closure;
  P.tc = fields_max_tangents(P.width, P.bf16);
  // a persistent plan's graph outlives its members: its chunk kernels take the largest size
  P.r_cap = 1;
  for (nsf_sim* m : P.members) P.r_cap = std::max(P.r_cap, m->r);
  if (P.persistent) P.r_cap = kMaxR;
  P.grid_cap = 8;
  for (nsf_sim* m : P.members) P.grid_cap = std::max(P.grid_cap, m->hd.grid_n);
  if (P.persistent) P.grid_cap = 256;
  P.place = P.persistent;
  for (nsf_sim* m : P.members) P.place = P.place || m->n_int > kAllocByParticles;
  std::vector<SimDev> sims;
  std::vector<FieldJob> jobs;
  std::vector<FieldTile> tA_jac, tA_prim, tA_team, tA_vel, tG, tG_vel, tD;  // tD: decode groups
  std::vector<FieldTile> tH;   // mixed precision: the h and l groups (BF16, primal table)
  // team Jacobian groups (half a primal group's time each) go after the primal groups
  std::vector<BlockWork> bP, bGN;
  // The FP32 velocity takes g at z_{n-1} on the step's points. Inside a step with at least
  // one iterate pass, the latent it needs (z_n) is known from the first Gauss-Newton solve
  // on, so that pass (which leaves part of the device idle) evaluates it for the next
  // step's points, after this step's P2G has read the buffer. The end-of-step inference
  // then skips it; a refresh outside a step still runs it at z_{n-1}.
  // (solo plans: the first pass's groups then start at an offset its graph keeps)
  const bool vel_in_g = !s0->bf16 && P.gn_iters >= 2 && !s0->closure && !P.persistent;
  const bool team = fields_team_jacobian(P.width, P.bf16);
  // Team groups carry the jobs over the same points when the sample set is the integration
  // set: the inference's h and l (and the velocity's g at z_{n-1} when it stays in the
  // inference) with its Jacobian job, and the velocity's g at the next step's points with
  // the first Gauss-Newton pass's. Every member must qualify, so that each table holds one
  // kind of team group (not in persistent plans, whose members change under one graph).
  // (nor beside a pipelined decode, which holds most CUs while the step's passes run: there
  // shorter groups share the rest better). Team groups take two tiles when the pairs of
  // one pass still fill the device, else one.
  bool fuse = team && !P.mixed && !P.closure && !P.persistent && !P.pipelined;
  int team_pairs = 0;
  for (nsf_sim* m : P.members) {
    fuse = fuse && m->n_int == m->n_samp && reverse_jacobian(m->r, P.tc) && !m->hd.tangent_forms;
    team_pairs += (m->n_samp + fields_team_points(-2) - 1) / fields_team_points(-2);
  }
  const bool fuse_g = fuse && vel_in_g;
  // (a persistent plan keeps one tiles per group for any set of members: its graph's kernels)
  const int team_nt = !P.pipelined && !P.persistent && team_pairs >= device_cus() ? -2 : -3;
  for (size_t si = 0; si < P.members.size(); ++si) {
    nsf_sim* s = P.members[si];
    const SimDev& H = s->hd;
    sims.push_back(H);
    const double* zp = H.z;
    const double* zc = H.z + s->r;
    const double* zi = H.z + 2 * s->r;
    const int N = s->n_int, S = s->n_samp, r = s->r;
    const int j0 = (int)jobs.size();
    // closure sims: the jobs over N take their point counts from the list each step
    ListJobs lj{};
    auto over_list = [&](int job) { if (s->closure) lj.idx[lj.n++] = job; };
    // inference: g with its Jacobian on S, g on N \ S, velocity, h, l
    FieldJob a = base_job(s, NSF_FIELD_G, zc);
    a.n = S; a.out = H.u_n; a.ldo = N; a.jac = H.J; a.ldj = S;
    jobs.push_back(a);
    if (!fuse) {
      if (team && reverse_jacobian(r, P.tc)) add_tiles(tA_team, j0, S, r, P.tc, true, 0, team_nt);
      else add_tiles(tA_jac, j0, S, r, P.tc);
    }
    if (N > S) {
      FieldJob b = base_job(s, NSF_FIELD_G, zc);
      b.n = N - S; b.p_off = S; b.out = H.u_n + S; b.ldo = N;
      add_prim_tiles(tA_prim, (int)jobs.size(), N - S, P.tc);
      over_list((int)jobs.size());
      jobs.push_back(b);
    }
    FieldJob c = base_job(s, NSF_FIELD_G, zp);
    c.n = N; c.out = H.u_prev; c.ldo = N;
    over_list((int)jobs.size() + (vel_in_g ? 1 : 0));
    if (H.tangent_forms) {
      // velocity as the directional derivative at the midpoint:
      // v = J((z_n + z_{n-1}) / 2) (z_n - z_{n-1}) / dt
      c.z = zc; c.z2 = zp; c.jvp = 1; c.jvp_scale = (float)(1.0 / H.dt_d);
      for (int p0 = 0; p0 < N; p0 += fields_group_points(P.tc))
        tA_jac.push_back({(int)jobs.size(), p0, 0, 1});
    } else {
      const int jc = (int)jobs.size();
      if (!fuse || vel_in_g) add_prim_tiles(tA_vel, jc, N, P.tc);
      if (vel_in_g) {
        FieldJob c1 = c;
        c1.z = zc; c1.step_off = 1;
        if (!fuse_g) add_prim_tiles(tG_vel, jc + 1, N, P.tc);
        jobs.push_back(c);
        c = c1;
      }
    }
    const int jvel = (int)jobs.size();   // the velocity job the step's first G pass (or inference) runs
    jobs.push_back(c);
    FieldJob h = base_job(s, NSF_FIELD_H, zc);
    h.n = N; h.out = H.tau; h.ldo = N;
    if (s->n_mu > 0) {   // h(X, z_n, mu): the solve keeps zh's latent part current
      h.z = H.zh;
      h.r = s->r + s->n_mu;
    }
    const int jh = (int)jobs.size();
    if (P.mixed) add_prim_tiles(tH, jh, N, 0);
    else if (!fuse) add_prim_tiles(tA_prim, jh, N, P.tc);
    over_list((int)jobs.size());
    jobs.push_back(h);
    FieldJob l = base_job(s, NSF_FIELD_L, zc);
    l.n = N; l.out = H.C; l.ldo = N;
    const int jl = (int)jobs.size();
    if (P.mixed) add_prim_tiles(tH, jl, N, 0);
    else if (!fuse) add_prim_tiles(tA_prim, jl, N, P.tc);
    over_list((int)jobs.size());
    if (s->closure) P.list_jobs = lj;
    jobs.push_back(l);
    if (fuse)
      add_tiles(tA_team, j0, S, r, P.tc, true, vel_in_g ? team_extras(j0, {jh, jl}) : team_extras(j0, {jh, jl, jvel}),
                team_nt);
    // Gauss-Newton iterate: g and its Jacobian on S
    FieldJob g = base_job(s, NSF_FIELD_G, zi);
    g.n = S; g.out = H.u_gn; g.ldo = S; g.jac = H.J2; g.ldj = S;
    const int jg = (int)jobs.size();
    add_tiles(tG, jg, S, r, P.tc, team, 0, team_nt);
    if (fuse_g) add_tiles(tG_vel, jg, S, r, P.tc, true, team_extras(jg, {jvel}), team_nt);
    jobs.push_back(g);
    // decode all particles at the new latent
    // (a pipelined decode reads the snapshot of z_n the step's first kernel takes)
    FieldJob dj = base_job(s, NSF_FIELD_G, s->decode_mode == 2 ? H.zdec : zc);
    dj.idx = nullptr; dj.step = nullptr; dj.n = (int)s->n_part; dj.mode = 1;
    dj.out = H.xdec; dj.ldo = s->n_part;
    add_tiles(tD, (int)jobs.size(), (int)s->n_part, 0, 0);
    jobs.push_back(dj);
    P.decode_job = dj;
    for (int p0 = 0; p0 < N; p0 += kMpmBlock) bP.push_back({(int)si, p0});
    for (int p0 = 0; p0 < S; p0 += kGnChunk) bGN.push_back({(int)si, p0});
  }
  // Longest groups first: Jacobian groups, then the primal-only groups; the velocity
  // groups that a step moves into its first G pass come last in both tables, so the
  // step's inference and the other G passes run a prefix of them.
  std::vector<FieldTile> tA(tA_jac);
  tA.insert(tA.end(), tA_prim.begin(), tA_prim.end());
  tA.insert(tA.end(), tA_team.begin(), tA_team.end());
  tA.insert(tA.end(), tA_vel.begin(), tA_vel.end());
  // the first Gauss-Newton pass starts with the velocity groups (longer than team groups)
  // and later passes start after them; with team groups that carry the velocity, the first
  // pass runs those alone and later passes the plain ones
  tG.insert(tG.begin(), tG_vel.begin(), tG_vel.end());
  P.nGvel = (int)tG_vel.size();
  P.nA = (int)tA.size(); P.nG = (int)tG.size(); P.nD = (int)tD.size();
  P.nAstep = P.nA - (vel_in_g ? (int)tA_vel.size() : 0);
  P.nGnext = fuse_g ? P.nGvel : P.nG;
  P.nG -= P.nGvel;
  auto kinds = [](const std::vector<FieldTile>& t) {
    int k = 0;
    for (const FieldTile& f : t)
      k |= f.nt == -2 ? kTableTeam : f.nt == -3 ? kTableTeam | kTableTeamOne : (f.nt != 0 ? kTableTangents : 0);
    return k ? k : kTableTangents;
  };
  // a persistent plan's graph outlives its tables: its kernels take every kind
  P.kindsA = P.persistent ? kTableTangents | kTableTeam | kTableTeamOne : kinds(tA);
  P.kindsG = P.persistent ? kTableTangents | kTableTeam | kTableTeamOne : kinds(tG);
  P.nP = (int)bP.size(); P.nGN = (int)bGN.size();
  P.nsims = (int)sims.size();
  P.nH = (int)tH.size();
  // work counts: [0] step inference, [1] G pass, [2] full inference, [3] MPM blocks,
  // [4] first G pass, [5] Gauss-Newton chunks, [6] sims, [7] decode groups; [8..15] claim
  // counters; [16] the h and l groups of a mixed-precision plan
  std::vector<int32_t> counts = {P.nAstep, P.nG, P.nA, P.nP, P.nGnext, P.nGN, P.nsims, P.nD,
                                 0, 0, 0, 0, 0, 0, 0, 0, P.nH, 0, 0, 0, 0, 0, 0, 0};
  // Regions of the device buffer. A persistent plan keeps fixed region capacities (grown
  // by half when exceeded), so its captured graph stays valid while tables are rewritten.
  struct Region { const void* data; size_t bytes; };
  constexpr int kRegions = 9;
  const Region reg[kRegions] = {
      {counts.data(), counts.size() * 4}, {sims.data(), sims.size() * sizeof(SimDev)},
      {jobs.data(), jobs.size() * sizeof(FieldJob)}, {tA.data(), tA.size() * sizeof(FieldTile)},
      {tG.data(), tG.size() * sizeof(FieldTile)}, {tD.data(), tD.size() * sizeof(FieldTile)},
      {bP.data(), bP.size() * sizeof(BlockWork)}, {bGN.data(), bGN.size() * sizeof(BlockWork)},
      {tH.data(), tH.size() * sizeof(FieldTile)}};
  bool relayout = P.caps.empty();
  for (int i = 0; i < kRegions && !relayout; ++i) relayout = reg[i].bytes > P.caps[i];
  if (relayout) {
    P.caps.assign(kRegions, 0);
    for (int i = 0; i < kRegions; ++i)
      P.caps[i] = align_up(P.persistent ? reg[i].bytes + reg[i].bytes / 2 + 4096 : std::max<size_t>(reg[i].bytes, 1));
  }
  size_t off[kRegions], total = 0;
  for (int i = 0; i < kRegions; ++i) { off[i] = total; total += P.caps[i]; }
  if (relayout || total > P.dcap) {
    P.drop_graphs();
    if (P.dbuf) { NSF_HIP(hipStreamSynchronize(stream)); NSF_HIP(hipFree(P.dbuf)); P.dbuf = nullptr; }
    P.dcap = total;
    NSF_HIP(hipMalloc(&P.dbuf, P.dcap));
    if (P.persistent) {
      if (P.staging) NSF_HIP(hipHostFree(P.staging));
      P.staging = nullptr;
      NSF_HIP(hipHostMalloc(&P.staging, P.dcap, hipHostMallocDefault));
    }
  }
  char* b = static_cast<char*>(P.dbuf);
  P.d_counts = reinterpret_cast<int32_t*>(b + off[0]);
  P.d_sims = reinterpret_cast<SimDev*>(b + off[1]);
  P.d_jobs = reinterpret_cast<FieldJob*>(b + off[2]);
  P.d_tA = reinterpret_cast<FieldTile*>(b + off[3]);
  P.d_tG = reinterpret_cast<FieldTile*>(b + off[4]);
  P.d_tD = reinterpret_cast<FieldTile*>(b + off[5]);
  P.d_bP = reinterpret_cast<BlockWork*>(b + off[6]);
  P.d_bGN = reinterpret_cast<BlockWork*>(b + off[7]);
  P.d_tH = reinterpret_cast<FieldTile*>(b + off[8]);
  if (P.persistent) {
    NSF_HIP(hipStreamSynchronize(stream));  // the previous upload has been consumed
    char* st = static_cast<char*>(P.staging);
    for (int i = 0; i < kRegions; ++i)
      if (reg[i].bytes) std::memcpy(st + off[i], reg[i].data, reg[i].bytes);
    // only the used part of each region is copied (regions are independent)
    for (int i = 0; i < kRegions; ++i)
      if (reg[i].bytes)
        NSF_HIP(hipMemcpyAsync(b + off[i], st + off[i], reg[i].bytes, hipMemcpyHostToDevice, stream));
  } else {
    std::vector<char> blob(total, 0);
    for (int i = 0; i < kRegions; ++i)
      if (reg[i].bytes) std::memcpy(blob.data() + off[i], reg[i].data, reg[i].bytes);
    NSF_HIP(hipMemcpyAsync(P.dbuf, blob.data(), total, hipMemcpyHostToDevice, stream));
    NSF_HIP(hipStreamSynchronize(stream));
  }
  // grids
  const int cus = device_cus();
  const int fcap = cus * fields_table_blocks_per_cu(P.width, P.bf16, P.tc);
  const int fcap0 = cus * fields_table_blocks_per_cu(P.width, P.bf16, 0);
  auto mn = [](int a, int b) { return a < b ? a : b; };
  P.gF = P.persistent ? fcap : mn(fcap, std::max(P.nA, P.nGnext));
  P.gF0 = P.persistent ? fcap0 : mn(fcap0, P.nD);
  P.gH = P.persistent ? cus * fields_table_blocks_per_cu(P.width, true, 0) : mn(cus, P.nH);
  P.gP = P.persistent ? 4 * cus : P.nP;
  P.gGN = P.persistent ? 4 * cus : P.nGN;
  P.gSims = P.persistent ? cus : P.nsims;
  P.gBlk = 5 * cus;   // gather workgroups (5 fit per CU) loop over each sim's active node blocks
  if (P.pipelined && !P.side) {
    NSF_HIP(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
    NSF_HIP(hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming));
    NSF_HIP(hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming));
  }
  return NSF_OK;
}

// Claim counters (zeroed at the start of every launch sequence): 8 inference, 9 + k the
// Gauss-Newton iterate pass k, 13 refresh (inference + decode), 14 decode alone.
constexpr int kClaimA = 8, kClaimG = 9, kClaimD = 14, kClaimH = 15;

// Mixed precision: the h and l groups of the inference, in a BF16 primal table after the
// FP32 table of the deformation field's jobs.
nsf_status launch_hl(Plan& P, hipStream_t s) {
  if (!P.mixed || P.gH <= 0) return NSF_OK;
  NSF_HIP(launch_fields_table(P.width, true, 0, kTableTangents, P.d_jobs, P.d_tH, P.d_counts + 16, P.d_counts + kClaimH, P.gH, s));
  return NSF_OK;
}

nsf_status launch_decode(Plan& P, hipStream_t s, bool beside);

// Closure sims: the integration set from the decoded positions (the decode runs first).
nsf_status enqueue_closure(Plan& P, hipStream_t s) {
  for (nsf_sim* m : P.members)
    if (m->closure) NSF_HIP(launch_closure(m->dd, m->n_samp, m->n_part, P.d_jobs, P.list_jobs, s));
  return NSF_OK;
}

// Field inference of the step for the current latent, alone (prologue after create or
// set_latent; a closure sim decodes and builds its integration set first).
nsf_status enqueue_inference(Plan& P, hipStream_t s) {
  NSF_HIP(launch_reset_counters(P.d_counts + 8, 8, s));
  if (P.closure) {
    nsf_status st = launch_decode(P, s, false);
    if (st == NSF_OK) st = enqueue_closure(P, s);
    if (st != NSF_OK) return st;
  }
  NSF_HIP(launch_fields_table(P.width, P.bf16, P.tc, P.kindsA, P.d_jobs, P.d_tA, P.d_counts + 2,
                              P.d_counts + kClaimA, std::min(P.gF, std::max(P.nA, 1)), s));
  return launch_hl(P, s);
}

// Decode of all particles on stream s: the dense kernel for one sim, else over every sim's
// decode groups: in BF16 with each workgroup's weight sets resident in LDS (one workgroup
// per CU; beside the step, on the CUs a pipelined decode takes), in FP32 the primal table
// kernel, which streams the layers (four FP32 layers do not fit in LDS).
nsf_status launch_decode(Plan& P, hipStream_t s, bool beside) {
  if (P.nsims == 1 && !P.persistent)
    NSF_HIP(launch_fields_dense(P.width, P.bf16_hl, P.decode_job, P.decode_job.n, s, beside));
  else if (P.bf16_hl)
    NSF_HIP(launch_fields_decode_table(P.width, P.d_jobs, P.d_tD, P.d_counts + 7,
                                       beside ? device_cus() - device_cus() * 3 / 8 : device_cus(), s));
  else
    NSF_HIP(launch_fields_table(P.width, P.bf16_hl, 0, kTableTangents, P.d_jobs, P.d_tD, P.d_counts + 7,
                                P.d_counts + kClaimD, P.gF0, s));
  return NSF_OK;
}

// Pipelined decode: on the side stream between a fork and a join recorded on s (inline on
// s when there is no side stream), on five eighths of the CUs: the step's MPM, Gauss-Newton
// and field kernels run on the rest meanwhile (and on all of them once it ends).
nsf_status fork_decode(Plan& P, hipStream_t s) {
  if (s == nullptr || !P.side) return launch_decode(P, s, false);
  NSF_HIP(hipEventRecord(P.ev_fork, s));
  NSF_HIP(hipStreamWaitEvent(P.side, P.ev_fork, 0));
  const nsf_status st = launch_decode(P, P.side, true);
  if (st != NSF_OK) return st;
  NSF_HIP(hipEventRecord(P.ev_join, P.side));
  return NSF_OK;
}

nsf_status join_decode(Plan& P, hipStream_t s) {
  if (s != nullptr && P.side) NSF_HIP(hipStreamWaitEvent(s, P.ev_join, 0));
  return NSF_OK;
}

// The next step's field inference at the current latent (in_step: without the groups the
// step's first G pass ran), then (decode = true) the decode of all particles at the same
// latent, on the same stream: the two persistent kernels fill the device one after the
// other (run side by side they only contend for the same CUs). Counters must have been
// reset in this sequence.
nsf_status enqueue_refresh_body(Plan& P, hipStream_t s, bool decode, bool in_step) {
  if (P.closure) {   // decode, then the integration set at the new positions, then the inference
    nsf_status st = launch_decode(P, s, false);
    if (st == NSF_OK) st = enqueue_closure(P, s);
    if (st != NSF_OK) return st;
    NSF_HIP(launch_fields_table(P.width, P.bf16, P.tc, P.kindsA, P.d_jobs, P.d_tA, P.d_counts + (in_step ? 0 : 2),
                                P.d_counts + kClaimA, P.gF, s));
    return NSF_OK;
  }
  NSF_HIP(launch_fields_table(P.width, P.bf16, P.tc, P.kindsA, P.d_jobs, P.d_tA, P.d_counts + (in_step ? 0 : 2),
                              P.d_counts + kClaimA, P.gF, s));
  const nsf_status hl = launch_hl(P, s);
  if (hl != NSF_OK) return hl;
  return decode ? launch_decode(P, s, false) : NSF_OK;
}

// Refresh outside a step (nsf_refresh): a pipelined sim first points its decode at the
// current latent.
nsf_status enqueue_refresh(Plan& P, hipStream_t s) {
  NSF_HIP(launch_reset_counters(P.d_counts + 8, 8, s));
  if (P.pipelined)
    for (nsf_sim* m : P.members)
      NSF_HIP(hipMemcpyAsync(m->hd.zdec, m->hd.z + m->r, (size_t)m->r * 8, hipMemcpyDeviceToDevice, s));
  return enqueue_refresh_body(P, s, P.decode, false);
}

// One latent step, given its field inference in the buffers: MPM step, Gauss-Newton
// iterations, then the inference of step n + 1. The decode of all particles runs at
// z_{n+1} together with that inference, or (pipelined) at z_n alongside the whole step,
// forked right after the first kernel has taken its latent snapshot.
// The MPM stage of a step (Sec. 5.2): binning (which also zeroes the step's claim
// counters), P2G with the grid update, and G2P at the samples fused with the first
// Gauss-Newton chunk sums. A pipelined decode forks after the binning kernel, which takes
// its latent snapshot.
nsf_status enqueue_mpm(Plan& P, hipStream_t s, bool fork) {
  // every sparse (plan-mode) sim takes the wave-per-block gather, alone or in a batch, so a
  // sim's sums are the same bits either way
  const bool batch = !P.closure;
  NSF_HIP(launch_bin(P.d_sims, P.d_bP, P.d_counts + 3, P.d_counts + 8, P.gP, batch, s));
  if (fork) {
    const nsf_status st = fork_decode(P, s);
    if (st != NSF_OK) return st;
  }
  NSF_HIP(launch_p2g_after_bin(P.d_sims, P.d_counts + 6, P.gSims, P.d_bP, P.d_counts + 3, P.gP, P.gBlk, P.closure,
                               P.grid_cap, P.place, batch, s));
  NSF_HIP(launch_g2p_gn(P.d_sims, P.d_bGN, P.d_counts + 5, P.r_cap, P.gGN, s));
  return NSF_OK;
}

nsf_status enqueue_step(Plan& P, hipStream_t s) {
  const nsf_status sm = enqueue_mpm(P, s, P.decode && P.pipelined);
  if (sm != NSF_OK) return sm;
  NSF_HIP(launch_gn_solve(P.d_sims, P.d_counts + 6, 0, P.gSims, s));
  for (int k = 1; k < P.gn_iters; ++k) {
    NSF_HIP(launch_fields_table(P.width, P.bf16, P.tc, P.kindsG, P.d_jobs, P.d_tG + (k == 1 ? 0 : P.nGvel),
                                P.d_counts + (k == 1 ? 4 : 1),
                                P.d_counts + kClaimG + (k - 1), P.gF, s));
    NSF_HIP(launch_gn_partial(P.d_sims, P.d_bGN, P.d_counts + 5, k, P.r_cap, P.gGN, s));
    NSF_HIP(launch_gn_solve(P.d_sims, P.d_counts + 6, k, P.gSims, s));
  }
  if (P.decode && P.pipelined) {
    const nsf_status st = enqueue_refresh_body(P, s, false, true);
    if (st != NSF_OK) return st;
    return join_decode(P, s);
  }
  return enqueue_refresh_body(P, s, P.decode, true);
}

constexpr int kGraphSteps = 8;

// Capture `steps` consecutive steps on s into a graph and instantiate it.
nsf_status capture_steps(Plan& P, int steps, hipStream_t s, hipGraph_t* graph, hipGraphExec_t* exec) {
  NSF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  nsf_status st = NSF_OK;
  for (int i = 0; i < steps && st == NSF_OK; ++i) st = enqueue_step(P, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != NSF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(NSF_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  *graph = g;
  NSF_HIP(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  return NSF_OK;
}

nsf_status run_plan(Plan& P, int32_t n_steps, hipStream_t s) {
  bool ready = true;
  for (nsf_sim* m : P.members) ready = ready && m->inference_ready;
  if (!ready) {
    const nsf_status st = enqueue_inference(P, s);
    if (st != NSF_OK) return st;
  }
  if (s == nullptr) {
    for (int i = 0; i < n_steps; ++i) {
      const nsf_status st = enqueue_step(P, s);
      if (st != NSF_OK) return st;
    }
  } else {
    if (n_steps >= kGraphSteps && !P.exec_n) {
      const nsf_status st = capture_steps(P, kGraphSteps, s, &P.graph_n, &P.exec_n);
      if (st != NSF_OK) return st;
    }
    if (n_steps % kGraphSteps != 0 && !P.exec) {
      const nsf_status st = capture_steps(P, 1, s, &P.graph, &P.exec);
      if (st != NSF_OK) return st;
    }
    for (int i = 0; i < n_steps / kGraphSteps; ++i) NSF_HIP(hipGraphLaunch(P.exec_n, s));
    for (int i = 0; i < n_steps % kGraphSteps; ++i) NSF_HIP(hipGraphLaunch(P.exec, s));
  }
  for (nsf_sim* m : P.members) m->inference_ready = true;
  return NSF_OK;
}

nsf_status check_batch(nsf_sim* const* sims, int32_t n) {
  if (!sims || n < 1) return fail(NSF_EINVAL, "empty batch");
  if (n > kMaxBatchSims) return fail(NSF_EINVAL, "batch of %d sims exceeds %d", n, kMaxBatchSims);
  for (int i = 0; i < n; ++i) {
    if (!sims[i]) return fail(NSF_EINVAL, "sims[%d] is NULL", i);
    if (n > 1 && sims[i]->closure)
      return fail(NSF_EINVAL, "sims[%d] uses closure integration, which steps alone", i);
    if (sims[i]->width != sims[0]->width || sims[i]->bf16 != sims[0]->bf16 || sims[i]->bf16_hl != sims[0]->bf16_hl ||
        sims[i]->gn_iters != sims[0]->gn_iters || sims[i]->decode_mode != sims[0]->decode_mode)
      return fail(NSF_EINVAL, "sims[%d] differs in width, precision, gn_iters or decode mode", i);
    for (int j = 0; j < i; ++j)
      if (sims[j] == sims[i]) return fail(NSF_EINVAL, "sim listed twice in a batch");
  }
  return NSF_OK;
}

// The persistent batch plan of this set of sims (caller holds g_plans_mu); its tables are
// rewritten when the set differs from the one it last stepped.
nsf_status batch_plan(nsf_sim* const* sims, int32_t n, hipStream_t st, Plan** out) {
  std::vector<nsf_sim*> key(sims, sims + n);
  std::unique_ptr<Plan>& slot = g_batch_plans[batch_signature(key[0])];
  if (!slot) {
    slot.reset(new Plan());
    slot->persistent = true;
  }
  Plan& P = *slot;
  if (P.members != key) {
    P.members = key;
    const nsf_status e = build_plan(P, st);
    if (e != NSF_OK) {
      P.members.clear();
      return e;
    }
  }
  *out = &P;
  return NSF_OK;
}

nsf_status solo_plan(nsf_sim* s, hipStream_t st) {
  if (s->solo) return NSF_OK;
  std::unique_ptr<Plan> p(new Plan());
  p->members.push_back(s);
  const nsf_status e = build_plan(*p, st);
  if (e != NSF_OK) return e;
  s->solo = std::move(p);
  return NSF_OK;
}

void drop_batch_plans_with(nsf_sim* s) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  for (auto& kv : g_batch_plans) {
    Plan& P = *kv.second;
    if (std::find(P.members.begin(), P.members.end(), s) != P.members.end())
      P.members.clear();  // tables reference the sim: rebuild before the next replay
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------
extern "C" {

const char* nsf_last_error(void) { return g_err.c_str(); }

int32_t nsf_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

size_t nsf_sim_bytes(const nsf_sim_desc* d) {
  if (validate(d) != NSF_OK) return 0;
  return make_layout(d).total;
}

nsf_status nsf_create_sim(const nsf_sim_desc* d, void* arena, size_t arena_bytes, void* stream,
                          nsf_sim** out) {
  if (!out) return fail(NSF_EINVAL, "out is NULL");
  *out = nullptr;
  nsf_status st = validate(d);
  if (st != NSF_OK) return st;
  std::string why;
  if (!device_ok(&why)) return fail(NSF_ENODEV, "%s", why.c_str());
  const Layout L = make_layout(d);
  if (!arena) return fail(NSF_EINVAL, "arena is NULL");
  if ((reinterpret_cast<uintptr_t>(arena) & (kAlign - 1)) != 0) return fail(NSF_EINVAL, "arena must be 256-byte aligned");
  if (arena_bytes < L.total) return fail(NSF_ENOMEM, "arena has %zu bytes, needs %zu", arena_bytes, L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::unique_ptr<nsf_sim> sim(new nsf_sim());
  NSF_HIP(hipGetDevice(&sim->device));
  sim->r = d->r;
  sim->width = d->width;
  sim->bf16 = d->precision == NSF_BF16;
  sim->bf16_hl = d->precision != NSF_FP32;
  sim->n_part = d->n_particles;
  sim->n_int = d->n_integration;
  sim->n_samp = d->n_sample;
  sim->gn_iters = d->gn_iters;
  sim->decode_mode = d->decode_every_step;
  sim->closure = d->integration == NSF_INTEGRATION_CLOSURE;
  if (sim->closure) sim->samples.assign(d->sample_plan, d->sample_plan + d->n_sample);
  sim->arena = static_cast<char*>(arena);
  sim->arena_bytes = arena_bytes;
  sim->L = L;
  char* A = sim->arena;
  const int r = d->r, W = d->width;
  for (int f = 0; f < 3; ++f)
    for (int c = 0; c < 9; ++c) {
      sim->scale[f][c] = c < kFieldOut[f] ? (float)d->out_scale[f][c] : 0.f;
      sim->shift[f][c] = c < kFieldOut[f] ? (float)d->out_shift[f][c] : 0.f;
    }
  // pack weights on the host, one upload per field
  std::vector<char> staging;
  for (int f = 0; f < 3; ++f) {
    const int dd = kFieldOut[f], rf = field_r(d, f);
    const PackSizes ps = pack_sizes(rf, W, dd);
    std::vector<float> whp(ps.whp), b6(ps.b6), w1q(ps.w1q), bhq(ps.bhq), w6q(ps.w6q), whpt(ps.whp),
        w1zt(ps.w1zt);
    std::vector<uint16_t> whb(ps.whb), whbt(ps.whb);
    pack_field(d->weights[f], rf, W, dd,
               PackOut{whp.data(), whb.data(), b6.data(), w1q.data(), bhq.data(), w6q.data(), whpt.data(),
                       whbt.data(), w1zt.data()});
    auto up = [&](size_t off, const void* src, size_t bytes) {
      return hipMemcpyAsync(A + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    NSF_HIP(up(L.whp[f], whp.data(), whp.size() * 4));
    NSF_HIP(up(L.whb[f], whb.data(), whb.size() * 2));
    NSF_HIP(up(L.b6[f], b6.data(), b6.size() * 4));
    NSF_HIP(up(L.w1q[f], w1q.data(), w1q.size() * 4));
    NSF_HIP(up(L.bhq[f], bhq.data(), bhq.size() * 4));
    NSF_HIP(up(L.w6q[f], w6q.data(), w6q.size() * 4));
    NSF_HIP(up(L.whpt[f], whpt.data(), whpt.size() * 4));
    NSF_HIP(up(L.whbt[f], whbt.data(), whbt.size() * 2));
    NSF_HIP(up(L.w1zt[f], w1zt.data(), w1zt.size() * 4));
    NSF_HIP(hipStreamSynchronize(s));  // host staging vectors die at the end of this scope
    FieldPack& fp = sim->pack[f];
    fp.whp = reinterpret_cast<const float*>(A + L.whp[f]);
    fp.whb = reinterpret_cast<const bf16x8*>(A + L.whb[f]);
    fp.b6 = reinterpret_cast<const float*>(A + L.b6[f]);
    fp.w1q = reinterpret_cast<const float*>(A + L.w1q[f]);
    fp.bhq = reinterpret_cast<const float*>(A + L.bhq[f]);
    fp.w6q = reinterpret_cast<const float*>(A + L.w6q[f]);
    fp.whpt = reinterpret_cast<const float*>(A + L.whpt[f]);
    fp.whbt = reinterpret_cast<const bf16x8*>(A + L.whbt[f]);
    fp.w1zt = reinterpret_cast<const float*>(A + L.w1zt[f]);
  }
  const int64_t P = d->n_particles;
  NSF_HIP(hipMemcpyAsync(A + L.X, d->X, (size_t)3 * P * 4, hipMemcpyHostToDevice, s));
  std::vector<int32_t> list0;
  std::vector<uint8_t> is_s;
  if (sim->closure) {
    // the list starts as S; entries past its live length only ever hold valid indices
    list0.assign((size_t)d->n_integration, d->sample_plan[0]);
    std::copy(d->sample_plan, d->sample_plan + d->n_sample, list0.begin());
    NSF_HIP(hipMemcpyAsync(A + L.plan, list0.data(), list0.size() * 4, hipMemcpyHostToDevice, s));
    is_s.assign((size_t)P, 0);
    for (int i = 0; i < d->n_sample; ++i) is_s[d->sample_plan[i]] = 1;
    NSF_HIP(hipMemcpyAsync(A + L.is_sample, is_s.data(), is_s.size(), hipMemcpyHostToDevice, s));
    NSF_HIP(hipMemsetAsync(A + L.node_mask, 0, mask_words(d->grid_n) * 4, s));
    NSF_HIP(hipMemcpyAsync(A + L.n_live, &d->n_sample, 4, hipMemcpyHostToDevice, s));
  } else {
    NSF_HIP(hipMemcpyAsync(A + L.plan, d->sample_plan, (size_t)d->plan_steps * d->n_integration * 4,
                           hipMemcpyHostToDevice, s));
  }
  std::vector<double> z(3 * r);
  for (int j = 0; j < r; ++j) {
    z[j] = d->z_prev ? d->z_prev[j] : d->z0[j];
    z[r + j] = d->z0[j];
    z[2 * r + j] = d->z0[j];
  }
  NSF_HIP(hipMemcpyAsync(A + L.z, z.data(), z.size() * 8, hipMemcpyHostToDevice, s));
  NSF_HIP(hipMemcpyAsync(A + L.zdec, z.data() + r, (size_t)r * 8, hipMemcpyHostToDevice, s));
  std::vector<double> zh0;
  if (d->n_mu > 0) {
    zh0.assign(z.begin() + r, z.begin() + 2 * r);
    zh0.insert(zh0.end(), d->mu, d->mu + d->n_mu);
    NSF_HIP(hipMemcpyAsync(A + L.zh, zh0.data(), zh0.size() * 8, hipMemcpyHostToDevice, s));
  }
  const size_t n3 = (size_t)d->grid_n * d->grid_n * d->grid_n;
  NSF_HIP(hipMemsetAsync(A + L.grid, 0, n3 * 16, s));
  NSF_HIP(hipMemsetAsync(A + L.step, 0, 8, s));
  NSF_HIP(hipMemsetAsync(A + L.flags, 0, 4, s));
  NSF_HIP(hipMemsetAsync(A + L.bin_cnt, 0, L.bin_meta - L.bin_cnt, s));
  NSF_HIP(hipMemsetAsync(A + L.bin_meta, 0xff, L.epoch - L.bin_meta, s));   // epoch -1: never set
  NSF_HIP(hipMemsetAsync(A + L.epoch, 0, 4, s));
  NSF_HIP(hipMemsetAsync(A + L.xdec, 0, (size_t)3 * P * 4, s));

  SimDev& H = sim->hd;
  H.r = r;
  H.n_part = (int32_t)P;
  H.n_int = d->n_integration;
  H.n_samp = d->n_sample;
  H.plan_steps = d->plan_steps;
  H.grid_n = d->grid_n;
  H.wall = d->wall_nodes;
  H.gn_iters = d->gn_iters;
  H.gn_damping = d->gn_damping;
  H.knife_on = d->knife.enabled ? 1 : 0;
  H.n_gn_chunks = ceil_div(d->n_sample, kGnChunk);
  H.width = W;
  H.tangent_forms = sim->bf16 ? 1 : 0;
  H.pipelined_decode = sim->decode_mode == 2 ? 1 : 0;
  // each integration particle stands for an equal share of the body (plan), or for its
  // own share, as in the full-order step the closure reproduces
  const double Vp = d->body_volume / (sim->closure ? (double)d->n_particles : (double)d->n_integration);
  H.dx = (float)d->dx;
  H.inv_dx = (float)(1.0 / d->dx);
  H.dt = (float)d->dt;
  H.mp = (float)(d->rho * Vp);
  H.stress_k = (float)(d->dt * Vp * 4.0 / (d->dx * d->dx));
  for (int c = 0; c < 3; ++c) {
    H.grav[c] = (float)d->gravity[c];
    H.grav_d[c] = d->gravity[c];
    H.kn[c] = d->knife.normal[c];
    H.kv[c] = d->knife.velocity[c];
  }
  H.dt_d = d->dt;
  H.dx_d = d->dx;
  H.koff = d->knife.offset;
  H.khalf = d->knife.half_thickness;
  H.kz0 = d->knife.edge_z0;
  H.kspeed = d->knife.edge_speed;
  H.X = reinterpret_cast<const float*>(A + L.X);
  H.plan = reinterpret_cast<const int32_t*>(A + L.plan);
  H.u_n = reinterpret_cast<float*>(A + L.u_n);
  H.u_prev = reinterpret_cast<float*>(A + L.u_prev);
  H.tau = reinterpret_cast<float*>(A + L.tau);
  H.C = reinterpret_cast<float*>(A + L.C);
  H.J = reinterpret_cast<float*>(A + L.J);
  H.vnew = reinterpret_cast<float*>(A + L.vnew);
  H.u_gn = reinterpret_cast<float*>(A + L.u_gn);
  H.J2 = reinterpret_cast<float*>(A + L.J2);
  H.xdec = reinterpret_cast<float*>(A + L.xdec);
  H.grid = reinterpret_cast<float4*>(A + L.grid);
  H.z = reinterpret_cast<double*>(A + L.z);
  H.zdec = reinterpret_cast<double*>(A + L.zdec);
  H.zh = d->n_mu > 0 ? reinterpret_cast<double*>(A + L.zh) : nullptr;
  sim->n_mu = d->n_mu;
  H.step = reinterpret_cast<int64_t*>(A + L.step);
  H.flags = reinterpret_cast<uint32_t*>(A + L.flags);
  H.gn_part = reinterpret_cast<double*>(A + L.gn_part);
  H.bin_edge = bin_edge(d->grid_n);
  H.nbs = bins_per_axis(d->grid_n);
  H.n_bins = H.nbs * H.nbs * H.nbs;
  H.bin_cnt = reinterpret_cast<int32_t*>(A + L.bin_cnt);
  H.bin_meta = reinterpret_cast<int4*>(A + L.bin_meta);
  H.epoch = reinterpret_cast<int32_t*>(A + L.epoch);
  H.pbin = reinterpret_cast<int32_t*>(A + L.pbin);
  H.prank = reinterpret_cast<int32_t*>(A + L.prank);
  H.rec = reinterpret_cast<float*>(A + L.rec);
  H.rec_p = reinterpret_cast<float*>(A + L.rec_p);
  H.sorted = reinterpret_cast<int32_t*>(A + L.sorted);
  H.active = reinterpret_cast<int32_t*>(A + L.active);
  H.nonempty = reinterpret_cast<int32_t*>(A + L.nonempty);
  H.n_active = reinterpret_cast<int32_t*>(A + L.n_active);
  if (sim->closure) {
    H.closure = 1;
    H.mask_words = (int32_t)mask_words(d->grid_n);
    H.nlist = reinterpret_cast<int32_t*>(A + L.plan);
    H.n_live = reinterpret_cast<int32_t*>(A + L.n_live);
    H.node_mask = reinterpret_cast<uint32_t*>(A + L.node_mask);
    H.is_sample = reinterpret_cast<uint8_t*>(A + L.is_sample);
    H.member = reinterpret_cast<uint8_t*>(A + L.member);
    H.cl_block = reinterpret_cast<int32_t*>(A + L.cl_block);
  }
  sim->dd = reinterpret_cast<SimDev*>(A + L.simdev);
  NSF_HIP(hipMemcpyAsync(sim->dd, &H, sizeof(SimDev), hipMemcpyHostToDevice, s));
  NSF_HIP(hipStreamSynchronize(s));
  *out = sim.release();
  return NSF_OK;
}

nsf_status nsf_step(nsf_sim* s, int32_t n_steps, void* stream) {
  if (!s) return fail(NSF_EINVAL, "sim is NULL");
  if (n_steps < 0) return fail(NSF_EINVAL, "n_steps < 0");
  if (n_steps == 0) return NSF_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const nsf_status e = solo_plan(s, st);
  if (e != NSF_OK) return e;
  return run_plan(*s->solo, n_steps, st);
}

nsf_status nsf_step_batch(nsf_sim* const* sims, int32_t n, int32_t n_steps, void* stream) {
  if (!sims || n < 1) return fail(NSF_EINVAL, "empty batch");
  if (n > kMaxBatchSims) return fail(NSF_EINVAL, "batch of %d sims exceeds %d", n, kMaxBatchSims);
  if (n_steps < 0) return fail(NSF_EINVAL, "n_steps < 0");
  if (n == 1) return nsf_step(sims[0], n_steps, stream);
  const nsf_status chk = check_batch(sims, n);
  if (chk != NSF_OK) return chk;
  if (n_steps == 0) return NSF_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_plans_mu);
  Plan* P = nullptr;
  const nsf_status e = batch_plan(sims, n, st, &P);
  if (e != NSF_OK) return e;
  return run_plan(*P, n_steps, st);
}

nsf_status nsf_mpm_stage(nsf_sim* const* sims, int32_t n, void* stream) {
  const nsf_status chk = check_batch(sims, n);
  if (chk != NSF_OK) return chk;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Plan* P = nullptr;
  std::unique_lock<std::mutex> lk(g_plans_mu, std::defer_lock);
  if (n == 1) {
    const nsf_status e = solo_plan(sims[0], st);
    if (e != NSF_OK) return e;
    P = sims[0]->solo.get();
  } else {
    lk.lock();
    const nsf_status e = batch_plan(sims, n, st, &P);
    if (e != NSF_OK) return e;
  }
  bool ready = true;
  for (nsf_sim* m : P->members) ready = ready && m->inference_ready;
  if (!ready) {
    const nsf_status e = enqueue_inference(*P, st);
    if (e != NSF_OK) return e;
    for (nsf_sim* m : P->members) m->inference_ready = true;
  }
  return enqueue_mpm(*P, st, false);
}

nsf_status nsf_decode(nsf_sim* s, const float* X, int64_t n, float* x_out, void* stream) {
  if (!s) return fail(NSF_EINVAL, "sim is NULL");
  if (!x_out) return fail(NSF_EINVAL, "x_out is NULL");
  if (n < 0 || n > (int64_t)INT32_MAX / 4) return fail(NSF_EINVAL, "n = %lld", (long long)n);
  if (!X && n != s->n_part) return fail(NSF_EINVAL, "own X has %lld points, n = %lld", (long long)s->n_part, (long long)n);
  if (n == 0) return NSF_OK;
  FieldJob j = base_job(s, NSF_FIELD_G, s->hd.z + s->r);
  j.idx = nullptr;
  j.step = nullptr;
  j.X = X ? X : s->hd.X;
  j.ldx = n;
  j.n = (int)n;
  j.mode = 1;
  j.out = x_out;
  j.ldo = n;
  NSF_HIP(launch_fields_dense(s->width, s->bf16_hl, j, (int)n, static_cast<hipStream_t>(stream)));
  return NSF_OK;
}

nsf_status nsf_get_latent(nsf_sim* s, double* z, double* z_prev, int64_t* step, void* stream) {
  if (!s) return fail(NSF_EINVAL, "sim is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (z) NSF_HIP(hipMemcpyAsync(z, s->hd.z + s->r, s->r * 8, hipMemcpyDeviceToHost, st));
  if (z_prev) NSF_HIP(hipMemcpyAsync(z_prev, s->hd.z, s->r * 8, hipMemcpyDeviceToHost, st));
  if (step) NSF_HIP(hipMemcpyAsync(step, s->hd.step, 8, hipMemcpyDeviceToHost, st));
  NSF_HIP(hipStreamSynchronize(st));
  return NSF_OK;
}

nsf_status nsf_set_latent(nsf_sim* s, const double* z, const double* z_prev, int64_t step, void* stream) {
  if (!s || !z) return fail(NSF_EINVAL, "sim or z is NULL");
  if (step < 0) return fail(NSF_EINVAL, "step < 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<double> buf(3 * s->r);
  for (int j = 0; j < s->r; ++j) {
    buf[j] = z_prev ? z_prev[j] : z[j];
    buf[s->r + j] = z[j];
    buf[2 * s->r + j] = z[j];
  }
  const uint32_t zero = 0;
  NSF_HIP(hipMemcpyAsync(s->hd.z, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, st));
  if (s->hd.zh) NSF_HIP(hipMemcpyAsync(s->hd.zh, z, s->r * 8, hipMemcpyHostToDevice, st));
  NSF_HIP(hipMemcpyAsync(s->hd.step, &step, 8, hipMemcpyHostToDevice, st));
  NSF_HIP(hipMemcpyAsync(s->hd.flags, &zero, 4, hipMemcpyHostToDevice, st));
  NSF_HIP(hipStreamSynchronize(st));
  s->inference_ready = false;
  return NSF_OK;
}

nsf_status nsf_refresh(nsf_sim* s, void* stream) {
  if (!s) return fail(NSF_EINVAL, "sim is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const nsf_status sp = solo_plan(s, st);
  if (sp != NSF_OK) return sp;
  const nsf_status e = enqueue_refresh(*s->solo, st);
  if (e == NSF_OK) s->inference_ready = true;
  return e;
}

nsf_status nsf_set_sample_count(nsf_sim* s, int32_t n_sample, void* stream) {
  if (!s) return fail(NSF_EINVAL, "sim is NULL");
  if (!s->closure) return fail(NSF_EINVAL, "the sample count changes only with closure integration");
  if (n_sample < 1 || n_sample > (int32_t)s->samples.size())
    return fail(NSF_EINVAL, "n_sample = %d outside 1..%zu", n_sample, s->samples.size());
  if (3 * n_sample < s->r) return fail(NSF_EINVAL, "n_sample = %d < r / 3: the inversion is under-determined", n_sample);
  hipStream_t st = static_cast<hipStream_t>(stream);
  NSF_HIP(hipStreamSynchronize(st));   // no step of the old plan is in flight
  drop_batch_plans_with(s);
  s->solo.reset();
  s->n_samp = n_sample;
  s->hd.n_samp = n_sample;
  s->hd.n_gn_chunks = ceil_div(n_sample, kGnChunk);
  std::vector<uint8_t> is_s((size_t)s->n_part, 0);
  for (int i = 0; i < n_sample; ++i) is_s[s->samples[i]] = 1;
  NSF_HIP(hipMemcpyAsync(s->hd.is_sample, is_s.data(), is_s.size(), hipMemcpyHostToDevice, st));
  NSF_HIP(hipMemcpyAsync(s->dd, &s->hd, sizeof(SimDev), hipMemcpyHostToDevice, st));
  NSF_HIP(hipStreamSynchronize(st));
  s->inference_ready = false;
  return NSF_OK;
}

nsf_status nsf_set_parameters(nsf_sim* s, const double* mu, int32_t n_mu, void* stream) {
  if (!s) return fail(NSF_EINVAL, "sim is NULL");
  if (n_mu != s->n_mu) return fail(NSF_EINVAL, "n_mu = %d, the sim has %d problem parameters", n_mu, s->n_mu);
  if (n_mu == 0) return NSF_OK;
  if (!mu) return fail(NSF_EINVAL, "mu is NULL");
  for (int i = 0; i < n_mu; ++i)
    if (!std::isfinite(mu[i])) return fail(NSF_EINVAL, "mu[%d] is not finite", i);
  hipStream_t st = static_cast<hipStream_t>(stream);
  NSF_HIP(hipMemcpyAsync(s->hd.zh + s->r, mu, (size_t)n_mu * 8, hipMemcpyHostToDevice, st));
  NSF_HIP(hipStreamSynchronize(st));   // mu is a host array read during the call only
  s->inference_ready = false;
  return NSF_OK;
}

nsf_status nsf_status_flags(nsf_sim* s, uint32_t* flags, void* stream) {
  if (!s || !flags) return fail(NSF_EINVAL, "sim or flags is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t f = 0;
  NSF_HIP(hipMemcpyAsync(&f, s->hd.flags, 4, hipMemcpyDeviceToHost, st));
  NSF_HIP(hipStreamSynchronize(st));
  *flags = f;
  if (f & FLAG_NONFINITE) return fail(NSF_ENONFINITE, "the latent or the residual became non-finite");
  if (f & FLAG_SINGULAR) return fail(NSF_ESINGULAR, "Gauss-Newton normal matrix is not positive definite");
  if (f & FLAG_DOMAIN) return fail(NSF_EDOMAIN, "a particle stencil left the grid");
  if (f & FLAG_CAPACITY) return fail(NSF_ECAPACITY, "the integration set outgrew n_integration and was truncated");
  return NSF_OK;
}

nsf_status nsf_sim_buffer(nsf_sim* s, int32_t which, void** ptr, int64_t* count) {
  if (!s || !ptr || !count) return fail(NSF_EINVAL, "NULL argument");
  const SimDev& H = s->hd;
  const int64_t N = s->n_int, S = s->n_samp, P = s->n_part, r = s->r;
  switch (which) {
    case NSF_BUF_U: *ptr = H.u_n; *count = 3 * N; break;
    case NSF_BUF_UPREV: *ptr = H.u_prev; *count = 3 * N; break;
    case NSF_BUF_TAU: *ptr = H.tau; *count = 6 * N; break;
    case NSF_BUF_C: *ptr = H.C; *count = 9 * N; break;
    case NSF_BUF_JAC: *ptr = H.J; *count = 3 * r * S; break;
    case NSF_BUF_VNEW: *ptr = H.vnew; *count = 3 * S; break;
    case NSF_BUF_XDEC: *ptr = H.xdec; *count = 3 * P; break;
    case NSF_BUF_GRID: *ptr = H.grid; *count = (int64_t)4 * H.grid_n * H.grid_n * H.grid_n; break;
    case NSF_BUF_Z: *ptr = H.z; *count = 3 * r; break;
    case NSF_BUF_NLIST:
      *ptr = const_cast<int32_t*>(H.plan);
      *count = (int64_t)H.plan_steps * N;
      break;
    case NSF_BUF_NLIVE:
      if (!s->closure) return fail(NSF_EINVAL, "NSF_BUF_NLIVE needs closure integration");
      *ptr = H.n_live;
      *count = 1;
      break;
    default: return fail(NSF_EINVAL, "unknown buffer %d", which);
  }
  return NSF_OK;
}

nsf_status nsf_destroy_sim(nsf_sim* s) {
  if (!s) return NSF_OK;
  drop_batch_plans_with(s);
  delete s;
  return NSF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Full-order MLS-MPM: every particle integrated, state in the reduced step's buffers
// (u_n = x - X, u_prev = v with tangent forms, tau, C) plus F^E, so the reduced step's
// P2G kernels run unchanged over the identity list, followed by the full-order G2P.
struct nsf_fo {
  int64_t n_part = 0;
  int grid_n = 0;
  char* arena = nullptr;
  SimDev hd{};
  SimDev* dd = nullptr;
  int32_t* d_counts = nullptr;    // [0..7] work counts ([3] P2G blocks, [6] sims), [8..15] claims
  BlockWork* d_bP = nullptr;
  int nP = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~nsf_fo() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

struct FoLayout {
  size_t simdev, counts, bP, X, plan, u, v, tau, C, F, grid, step, flags;
  size_t bin_cnt, bin_meta, epoch, pbin, prank, rec, rec_p, sorted, active, nonempty, n_active;
  size_t z;
  size_t total;
};

nsf_status fo_validate(const nsf_fo_desc* d) {
  if (!d) return fail(NSF_EINVAL, "descriptor is NULL");
  if (d->n_particles < 1 || d->n_particles > (int64_t)INT32_MAX / 16)
    return fail(NSF_EINVAL, "n_particles = %lld", (long long)d->n_particles);
  if (!d->X) return fail(NSF_EINVAL, "X is NULL");
  if (d->grid_n < 8 || d->grid_n > 256) return fail(NSF_EINVAL, "grid_n = %d outside 8..256", d->grid_n);
  if (!(d->dt > 0) || !(d->rho > 0) || !(d->body_volume > 0)) return fail(NSF_EINVAL, "dt, rho and body_volume must be positive");
  if (!(d->youngs > 0) || !(d->poisson > -1.0 && d->poisson < 0.5)) return fail(NSF_EINVAL, "need E > 0 and -1 < nu < 0.5");
  if (d->plasticity != NSF_FO_VON_MISES && d->plasticity != NSF_FO_DRUCKER_PRAGER &&
      d->plasticity != NSF_FO_HERSCHEL_BULKLEY)
    return fail(NSF_EINVAL, "plasticity = %d (0 von Mises, 1 Drucker-Prager, 2 Herschel-Bulkley)", d->plasticity);
  if (d->plasticity != NSF_FO_DRUCKER_PRAGER && !(d->yield_stress > 0))
    return fail(NSF_EINVAL, "yield_stress must be positive");
  if (d->plasticity == NSF_FO_DRUCKER_PRAGER && !(d->friction_angle >= 0.0 && d->friction_angle < 90.0))
    return fail(NSF_EINVAL, "friction_angle = %g outside [0, 90)", d->friction_angle);
  if (d->plasticity == NSF_FO_HERSCHEL_BULKLEY && !(d->viscosity >= 0.0 && std::isfinite(d->viscosity)))
    return fail(NSF_EINVAL, "viscosity = %g must be finite and >= 0", d->viscosity);
  if (d->wall_nodes < 0 || 2 * d->wall_nodes >= d->grid_n) return fail(NSF_EINVAL, "wall_nodes = %d", d->wall_nodes);
  return NSF_OK;
}

FoLayout fo_layout(const nsf_fo_desc* d) {
  FoLayout L{};
  Carver c;
  const int64_t P = d->n_particles;
  const size_t n3 = (size_t)d->grid_n * d->grid_n * d->grid_n;
  const int nbs = bins_per_axis(d->grid_n);
  const size_t nb = (size_t)nbs * nbs * nbs;
  L.simdev = c.take(sizeof(SimDev));
  L.counts = c.take(16 * 4);
  L.bP = c.take((size_t)ceil_div(P, kMpmBlock) * sizeof(BlockWork));
  L.X = c.take((size_t)3 * P * 4);
  L.plan = c.take((size_t)P * 4);
  L.u = c.take((size_t)3 * P * 4);
  L.v = c.take((size_t)3 * P * 4);
  L.tau = c.take((size_t)6 * P * 4);
  L.C = c.take((size_t)9 * P * 4);
  L.F = c.take((size_t)9 * P * 8);
  L.grid = c.take(n3 * 16);
  L.step = c.take(8);
  L.flags = c.take(4);
  L.bin_cnt = c.take(nb * 4);
  L.bin_meta = c.take(nb * 16);
  L.epoch = c.take(4);
  L.pbin = c.take((size_t)P * 4);
  L.prank = c.take((size_t)P * 4);
  L.rec = c.take((size_t)P * 128);
  L.rec_p = c.take((size_t)P * 128);
  L.sorted = c.take((size_t)P * 4);
  L.active = c.take(nb * 4);
  L.nonempty = c.take(nb * 4);
  L.n_active = c.take(8);
  L.z = c.take(3 * 8);
  L.total = c.off;
  return L;
}

nsf_status fo_enqueue_step(nsf_fo& f, hipStream_t s) {
  NSF_HIP(launch_bin(f.dd, f.d_bP, f.d_counts + 3, f.d_counts + 8, f.nP, false, s));
  NSF_HIP(launch_p2g_after_bin(f.dd, f.d_counts + 6, 1, f.d_bP, f.d_counts + 3, f.nP, 5 * device_cus(), true,
                               f.grid_n, f.n_part > kAllocByParticles, false, s));
  NSF_HIP(launch_fo_g2p(f.dd, f.n_part, s));
  return NSF_OK;
}

}  // namespace

extern "C" {

size_t nsf_fo_bytes(const nsf_fo_desc* d) {
  if (fo_validate(d) != NSF_OK) return 0;
  return fo_layout(d).total;
}

nsf_status nsf_fo_create(const nsf_fo_desc* d, void* arena, size_t arena_bytes, void* stream, nsf_fo** out) {
  if (!out) return fail(NSF_EINVAL, "out is NULL");
  *out = nullptr;
  nsf_status st = fo_validate(d);
  if (st != NSF_OK) return st;
  std::string why;
  if (!device_ok(&why)) return fail(NSF_ENODEV, "%s", why.c_str());
  const FoLayout L = fo_layout(d);
  if (!arena) return fail(NSF_EINVAL, "arena is NULL");
  if ((reinterpret_cast<uintptr_t>(arena) & (kAlign - 1)) != 0) return fail(NSF_EINVAL, "arena must be 256-byte aligned");
  if (arena_bytes < L.total) return fail(NSF_ENOMEM, "arena has %zu bytes, needs %zu", arena_bytes, L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::unique_ptr<nsf_fo> f(new nsf_fo());
  char* A = static_cast<char*>(arena);
  const int64_t P = d->n_particles;
  f->n_part = P;
  f->grid_n = d->grid_n;
  f->arena = A;
  // initial state: x = X, v = v0, C = 0, F^E = I, tau = 0 (the stress of F = I)
  std::vector<int32_t> ident((size_t)P);
  for (int64_t i = 0; i < P; ++i) ident[i] = (int32_t)i;
  std::vector<float> v0((size_t)3 * P);
  for (int c = 0; c < 3; ++c) std::fill(v0.begin() + c * P, v0.begin() + (c + 1) * P, (float)d->v0[c]);
  std::vector<double> F0((size_t)9 * P, 0.0);
  for (int c = 0; c < 3; ++c) std::fill(F0.begin() + (4 * c) * P, F0.begin() + (4 * c + 1) * P, 1.0);
  std::vector<BlockWork> bP;
  for (int64_t p0 = 0; p0 < P; p0 += kMpmBlock) bP.push_back({0, (int32_t)p0});
  f->nP = (int)bP.size();
  std::vector<int32_t> counts(16, 0);
  counts[3] = f->nP;
  counts[6] = 1;
  NSF_HIP(hipMemcpyAsync(A + L.X, d->X, (size_t)3 * P * 4, hipMemcpyHostToDevice, s));
  NSF_HIP(hipMemcpyAsync(A + L.plan, ident.data(), ident.size() * 4, hipMemcpyHostToDevice, s));
  NSF_HIP(hipMemsetAsync(A + L.u, 0, (size_t)3 * P * 4, s));
  NSF_HIP(hipMemcpyAsync(A + L.v, v0.data(), v0.size() * 4, hipMemcpyHostToDevice, s));
  NSF_HIP(hipMemsetAsync(A + L.tau, 0, (size_t)6 * P * 4, s));
  NSF_HIP(hipMemsetAsync(A + L.C, 0, (size_t)9 * P * 4, s));
  NSF_HIP(hipMemcpyAsync(A + L.F, F0.data(), F0.size() * 8, hipMemcpyHostToDevice, s));
  const size_t n3 = (size_t)d->grid_n * d->grid_n * d->grid_n;
  NSF_HIP(hipMemsetAsync(A + L.grid, 0, n3 * 16, s));
  NSF_HIP(hipMemsetAsync(A + L.step, 0, 8, s));
  NSF_HIP(hipMemsetAsync(A + L.flags, 0, 4, s));
  NSF_HIP(hipMemsetAsync(A + L.bin_cnt, 0, L.bin_meta - L.bin_cnt, s));
  NSF_HIP(hipMemsetAsync(A + L.bin_meta, 0, L.epoch + 4 - L.bin_meta, s));
  NSF_HIP(hipMemcpyAsync(A + L.counts, counts.data(), counts.size() * 4, hipMemcpyHostToDevice, s));
  NSF_HIP(hipMemcpyAsync(A + L.bP, bP.data(), bP.size() * sizeof(BlockWork), hipMemcpyHostToDevice, s));
  SimDev& H = f->hd;
  H.r = 1;
  H.n_part = (int32_t)P;
  H.n_int = (int32_t)P;
  H.n_samp = 0;
  H.plan_steps = 1;
  H.grid_n = d->grid_n;
  H.wall = d->wall_nodes;
  H.gn_iters = 1;
  H.tangent_forms = 1;   // u_prev holds the velocity itself
  H.ground = 1;
  const double dx = 1.0 / d->grid_n, Vp = d->body_volume / (double)P;
  H.dx = (float)dx;
  H.inv_dx = (float)d->grid_n;
  H.dt = (float)d->dt;
  H.mp = (float)(d->rho * Vp);
  H.stress_k = (float)(d->dt * Vp * 4.0 / (dx * dx));
  for (int c = 0; c < 3; ++c) {
    H.grav[c] = (float)d->gravity[c];
    H.grav_d[c] = d->gravity[c];
  }
  H.dt_d = d->dt;
  H.dx_d = dx;
  H.fo_mu = d->youngs / (2.0 * (1.0 + d->poisson));
  H.fo_lambda = d->youngs * d->poisson / ((1.0 + d->poisson) * (1.0 - 2.0 * d->poisson));
  H.fo_tau_y = d->yield_stress;
  H.fo_model = d->plasticity;
  H.fo_kappa = d->youngs / (3.0 * (1.0 - 2.0 * d->poisson));
  {
    const double sphi = std::sin(d->friction_angle * M_PI / 180.0);
    const double alpha = std::sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi);
    H.fo_dp_k = alpha * (3.0 * H.fo_lambda + 2.0 * H.fo_mu) / (2.0 * H.fo_mu);
  }
  H.fo_hb_lim = std::sqrt(2.0 / 3.0) * d->yield_stress;
  H.fo_hb_relax = 1.0 / (1.0 + d->viscosity / (2.0 * H.fo_mu * d->dt));
  H.X = reinterpret_cast<const float*>(A + L.X);
  H.plan = reinterpret_cast<const int32_t*>(A + L.plan);
  H.u_n = reinterpret_cast<float*>(A + L.u);
  H.u_prev = reinterpret_cast<float*>(A + L.v);
  H.tau = reinterpret_cast<float*>(A + L.tau);
  H.C = reinterpret_cast<float*>(A + L.C);
  H.F = reinterpret_cast<double*>(A + L.F);
  H.grid = reinterpret_cast<float4*>(A + L.grid);
  H.z = reinterpret_cast<double*>(A + L.z);
  H.step = reinterpret_cast<int64_t*>(A + L.step);
  H.flags = reinterpret_cast<uint32_t*>(A + L.flags);
  H.bin_edge = bin_edge(d->grid_n);
  H.nbs = bins_per_axis(d->grid_n);
  H.n_bins = H.nbs * H.nbs * H.nbs;
  H.bin_cnt = reinterpret_cast<int32_t*>(A + L.bin_cnt);
  H.bin_meta = reinterpret_cast<int4*>(A + L.bin_meta);
  H.epoch = reinterpret_cast<int32_t*>(A + L.epoch);
  H.pbin = reinterpret_cast<int32_t*>(A + L.pbin);
  H.prank = reinterpret_cast<int32_t*>(A + L.prank);
  H.rec = reinterpret_cast<float*>(A + L.rec);
  H.rec_p = reinterpret_cast<float*>(A + L.rec_p);
  H.sorted = reinterpret_cast<int32_t*>(A + L.sorted);
  H.active = reinterpret_cast<int32_t*>(A + L.active);
  H.nonempty = reinterpret_cast<int32_t*>(A + L.nonempty);
  H.n_active = reinterpret_cast<int32_t*>(A + L.n_active);
  f->dd = reinterpret_cast<SimDev*>(A + L.simdev);
  f->d_counts = reinterpret_cast<int32_t*>(A + L.counts);
  f->d_bP = reinterpret_cast<BlockWork*>(A + L.bP);
  NSF_HIP(hipMemcpyAsync(f->dd, &H, sizeof(SimDev), hipMemcpyHostToDevice, s));
  NSF_HIP(hipStreamSynchronize(s));
  *out = f.release();
  return NSF_OK;
}

nsf_status nsf_fo_step(nsf_fo* f, int32_t n_steps, void* stream) {
  if (!f) return fail(NSF_EINVAL, "full-order sim is NULL");
  if (n_steps < 0) return fail(NSF_EINVAL, "n_steps < 0");
  if (n_steps == 0) return NSF_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (s == nullptr) {
    for (int i = 0; i < n_steps; ++i) {
      const nsf_status st = fo_enqueue_step(*f, s);
      if (st != NSF_OK) return st;
    }
    return NSF_OK;
  }
  if (!f->exec) {
    NSF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const nsf_status st = fo_enqueue_step(*f, s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != NSF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(NSF_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    f->graph = g;
    NSF_HIP(hipGraphInstantiate(&f->exec, g, nullptr, nullptr, 0));
  }
  for (int i = 0; i < n_steps; ++i) NSF_HIP(hipGraphLaunch(f->exec, s));
  return NSF_OK;
}

nsf_status nsf_fo_buffer(nsf_fo* f, int32_t which, void** ptr, int64_t* count) {
  if (!f || !ptr || !count) return fail(NSF_EINVAL, "NULL argument");
  const SimDev& H = f->hd;
  const int64_t P = f->n_part;
  switch (which) {
    case NSF_FO_U: *ptr = H.u_n; *count = 3 * P; break;
    case NSF_FO_V: *ptr = H.u_prev; *count = 3 * P; break;
    case NSF_FO_C: *ptr = H.C; *count = 9 * P; break;
    case NSF_FO_TAU: *ptr = H.tau; *count = 6 * P; break;
    case NSF_FO_F: *ptr = H.F; *count = 9 * P; break;
    default: return fail(NSF_EINVAL, "unknown full-order buffer %d", which);
  }
  return NSF_OK;
}

nsf_status nsf_fo_flags(nsf_fo* f, uint32_t* flags, void* stream) {
  if (!f || !flags) return fail(NSF_EINVAL, "full-order sim or flags is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t v = 0;
  NSF_HIP(hipMemcpyAsync(&v, f->hd.flags, 4, hipMemcpyDeviceToHost, st));
  NSF_HIP(hipStreamSynchronize(st));
  *flags = v;
  if (v & FLAG_DOMAIN) return fail(NSF_EDOMAIN, "a particle stencil left the grid");
  return NSF_OK;
}

nsf_status nsf_fo_destroy(nsf_fo* f) {
  delete f;
  return NSF_OK;
}

}  // extern "C"
