// Host side of the C ABI: context, workspaces, job lists, and the MD step
// schedule.  Every computation is done by the kernels of scc_kernel.hip and
// md_kernels.hip on the context stream; the host only sequences launches.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <utility>
#include <mutex>
#include <vector>

#include "internal.h"

using namespace cavdftb;

namespace {

__global__ void ws_identity_kernel(double* ws, const int64_t* ws_off, const int32_t* unit_off,
                                   const int8_t* species, int n_units, int nmax_of_unit_stride_dummy) {
  (void)nmax_of_unit_stride_dummy;
  const int u = blockIdx.x;
  if (u >= n_units) return;
  int n = 0;
  for (int a = unit_off[u]; a < unit_off[u + 1]; ++a) n += species[a] == 0 ? 4 : 1;
  const int nmax = n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : n <= 48 ? 48 : n <= 64 ? 64 : n <= 96 ? 96
                 : n <= 128 ? 128 : 192;
  double* w = ws + ws_off[u];
  for (int e = threadIdx.x; e < nmax * nmax; e += blockDim.x) w[e] = (e / nmax == e % nmax) ? 1.0 : 0.0;
}

// orbital buckets: LDS-resident kernels up to 64, global-scratch kernels above
constexpr int kNumBuckets = 8;
constexpr int kBucketNmax[kNumBuckets] = {8, 16, 32, 48, 64, 96, 128, 192};
int bucket_of(int n) {
  for (int k = 0; k < kNumBuckets; ++k)
    if (n <= kBucketNmax[k]) return kBucketNmax[k];
  return -1;
}

struct Bucket {
  int idx = 0;          // position in the context's bucket list (its job counter)
  double cost = 0.0;    // estimated work of one evaluation: sum of (orbitals / 48)^3 over its units
  int nmax = 0;
  int n_units = 0;
  int n_wg = 0;         // workgroups of a launch (<= n_cu * per_cu_max)
  int per_cu_max = 1;   // resident workgroups per CU the scratch was sized for
  int eig_mode = -1;    // CAVDFTB_EIG_* of this bucket's units, -1: the context's
  int job_queue = -1;   // 1 / 0: device job queue or fixed stride for this bucket, -1: the context's
  int64_t scratch_per_wg = 0;
  int32_t* d_units = nullptr;  // center jobs: unit list
  int32_t* d_order = nullptr;  // center jobs of MD evaluations: the units by the cost of their last evaluation
  int32_t* d_order_tmp = nullptr;
  int cjob0 = 0;               // offset of this bucket's center jobs in the center job arrays
  // finite-difference Born jobs
  int n_fd_jobs = 0;
  int fjob0 = 0;               // offset in the fd job arrays
  int32_t* d_fd_job_unit = nullptr;
  int32_t* d_fd_job_disp = nullptr;
  int32_t* d_fd_unit = nullptr;  // [n_units] unit of each fd block
  int32_t* d_fd_job0 = nullptr;  // [n_units] first fd job (relative to this bucket's mu_job base)
  // forward differences: 3 jobs per atom (+h only), in the same job slots
  int n_fw_jobs = 0;
  int32_t* d_fw_job_unit = nullptr;
  int32_t* d_fw_job_disp = nullptr;
  int32_t* d_fw_job0 = nullptr;
  // field jobs of the Maxwell-relation Born charges: six per unit, -2 - (dir*2 + sign)
  int32_t* d_ff_job_unit = nullptr;
  int32_t* d_ff_job_disp = nullptr;
  // compacted displaced (or field) jobs of the units the surrogate hands back (fallback)
  int32_t* d_fb_job_unit = nullptr;
  int32_t* d_fb_job_disp = nullptr;
  int32_t* d_fb_job0 = nullptr;
  int32_t* d_fb_n = nullptr;
  double* d_scratch = nullptr;
};

}  // namespace

struct cavdftb_ctx {
  hipStream_t stream = nullptr;
  DevParams prm{};
  double mass[2] = {0, 0};
  int U = 0, NA = 0, M = 0;
  double pol[3] = {0, 0, 1};
  std::vector<int32_t> h_unit_off;
  int32_t* d_unit_off = nullptr;
  int8_t* d_species = nullptr;
  float* d_cost_scale = nullptr;  // [U] (orbitals / bucket nmax)^3: relative cost of one SCC iteration
  double *d_unit_x = nullptr, *d_omega = nullptr, *d_k = nullptr, *d_theta = nullptr, *d_lam = nullptr;
  int32_t* d_atom_unit = nullptr;
  double *d_mass = nullptr, *d_inv_mass = nullptr;
  int64_t* d_ws_off = nullptr;
  double* d_ws_C = nullptr;
  double* d_ws_dq = nullptr;
  double* d_ws_dq_hist = nullptr;
  double* d_fd_dq = nullptr;        // charge responses of the + jobs (3 n_a^2 + 3 n_a per unit)
  int64_t fd_dq_count = 0;
  int64_t* d_fd_dq_off = nullptr;   // [U] offsets into d_fd_dq
  int md_hist = 0;  // consecutive MD evaluations whose charges are stored
  int64_t* d_hist_off = nullptr;
  double* d_hist = nullptr;
  std::vector<Bucket> buckets;
  int n_fd_total = 0;
  // work arrays
  double *d_energy = nullptr, *d_forces = nullptr, *d_charges = nullptr, *d_dipole = nullptr;
  double *d_mu_pol = nullptr, *d_F = nullptr, *d_fq = nullptr, *d_field = nullptr, *d_zpol = nullptr;
  double* d_mu_job = nullptr;
  double* d_f_job = nullptr;      // [6][NA][3] forces of the field jobs
  int32_t* d_f_status = nullptr;  // [U][6] status of the field jobs
  int32_t *d_status = nullptr, *d_cjob_status = nullptr, *d_cjob_iters = nullptr;
  int32_t* d_unit_fail = nullptr;  // [U] last undisplaced SCC of the unit did not converge
  int32_t *d_fjob_status = nullptr, *d_fjob_iters = nullptr;
  unsigned long long* d_counters = nullptr;
  unsigned int* d_job_counter = nullptr;  // job queues of the SCC launches, one per bucket
  // concurrent bucket launches of the undisplaced evaluations: up to 4 streams
  // of default priority (the context stream and three side streams), forked
  // and joined with events on the context stream
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[3] = {nullptr, nullptr, nullptr};
  int n_streams = 4;
  bool capturing = false;  // inside replay_step's stream capture
  int dynamic_jobs = 1;
  int n_cu = 256;
  // learned Born-charge surrogate
  float* d_sg_params = nullptr;  // [2][members][N_PARAM]
  float* d_sg_norm = nullptr;    // [2][N_NORM]
  double sg_thr = 0.05;
  bool sg_ready = false;
  int32_t fallback_mode = CAVDFTB_BORN_FD;  // exact route for the units the surrogate hands back
  double* d_sg_feat = nullptr;    // [NA][32]
  double* d_sg_frames = nullptr;  // [NA][9]
  float* d_sg_x = nullptr;        // [NA][32], rows of species O then H
  float* d_sg_y = nullptr;        // [members][NA][9]
  double* d_sg_std = nullptr;     // [NA]
  double* d_born = nullptr;       // [NA][9]
  int32_t* d_unit_flag = nullptr; // [U]
  int32_t* d_sp_idx = nullptr;    // [NA] atoms of species O, then of species H
  int32_t* d_pos_in_sp = nullptr; // [NA]
  int32_t* d_n_sp = nullptr;      // [2]
  int n_sp[2] = {0, 0};
  std::vector<void*> allocs;
  // controls
  double tol = 1e-8;
  int32_t max_iter = 200;
  double alpha = 0.6;
  double w0 = 0.01;
  double jac_factor = 1.0e-3;
  int32_t eig_mode = CAVDFTB_EIG_AUTO;
  int keep_hist = 1;
  int warm_enabled = 1;
  bool warm_valid = false;
  bool primed = false;
  int born_every = 1;   // MD: exact Born charges on every born_every-th matter evaluation
  int64_t born_count = 0;
  // MD steps as replays of one captured hipGraph
  bool use_graph = false;
  uint64_t gen = 1;                // bumped by every call that changes what a step launches
  uint64_t graph_gen = 0;          // gen the graph was captured at
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const void* graph_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // r, p, qm, pm, obs
  double graph_dt = 0.0, graph_h = 0.0;
  int32_t graph_born = -1;
  int64_t graph_scc_launches = 0;  // SCC launches inside the graph
  int64_t graph_replays = 0, graph_captures = 0;
  unsigned int* d_obs_row = nullptr;  // row of obs the next observables launch writes
  double* d_obs_part = nullptr;       // [obs_part_rows][8] partial sums of the observables
  int obs_part_rows = 0;
  // real-space cavity: one photon pair per cell (U cells)
  bool rs_ready = false, rs_primed = false;
  double rs_eta = 0.0, rs_w0 = 0.0;
  double* d_rs_wk = nullptr;      // [U] omega_k by DFT index
  double* d_rs_qk = nullptr;      // [U] q_k after the last step
  double* d_rs_pk = nullptr;      // [U] p_k after the last step
  double2* d_rs_buf0 = nullptr;   // [U] transform buffers
  double2* d_rs_buf1 = nullptr;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending, ev_free;
  double t_ms = 0.0;
  int64_t launches = 0;
  std::string err;
};

namespace {

int fail(cavdftb_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(cavdftb_ctx* c, hipError_t e, const char* where) {
  return fail(c, CAVDFTB_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

template <typename T>
hipError_t dalloc(cavdftb_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e == hipSuccess) c->allocs.push_back((void*)*p);
  return e;
}

void drop_graph(cavdftb_ctx* c) {
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  if (c->graph) hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

void release(cavdftb_ctx* c) {
  if (c->stream) hipStreamSynchronize(c->stream);
  drop_graph(c);  // before the streams and events its capture used
  for (int j = 0; j < 3; ++j)
    if (c->side[j]) {
      hipStreamSynchronize(c->side[j]);
      hipStreamDestroy(c->side[j]);
      c->side[j] = nullptr;
    }
  for (int j = 0; j < 3; ++j)
    if (c->ev_join[j]) {
      hipEventDestroy(c->ev_join[j]);
      c->ev_join[j] = nullptr;
    }
  if (c->ev_fork) {
    hipEventDestroy(c->ev_fork);
    c->ev_fork = nullptr;
  }
  for (void* p : c->allocs) hipFree(p);
  c->allocs.clear();
  for (auto& pr : c->ev_pending) {
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  for (auto& pr : c->ev_free) {
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  c->ev_pending.clear();
  c->ev_free.clear();
}

void harvest_events(cavdftb_ctx* c) {
  for (auto& pr : c->ev_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess)
      c->t_ms += ms;
    c->ev_free.push_back(pr);
  }
  c->ev_pending.clear();
}

std::pair<hipEvent_t, hipEvent_t> get_events(cavdftb_ctx* c) {
  if (c->ev_free.empty()) {
    hipEvent_t a = nullptr, b = nullptr;
    hipEventCreate(&a);
    hipEventCreate(&b);
    return {a, b};
  }
  auto pr = c->ev_free.back();
  c->ev_free.pop_back();
  return pr;
}

SccArgs base_args(cavdftb_ctx* c, const double* pos) {
  SccArgs a{};
  a.prm = c->prm;
  a.pos = pos;
  a.unit_off = c->d_unit_off;
  a.species = c->d_species;
  a.ws_off = c->d_ws_off;
  a.ws_C = c->d_ws_C;
  a.ws_dq = c->d_ws_dq;
  a.n_atoms = c->NA;
  a.hist = c->d_hist;
  a.hist_off = c->d_hist_off;
  a.jac_factor = c->jac_factor;
  a.eig_mode = c->eig_mode;
  a.counters = c->d_counters;
  a.unit_fail = c->d_unit_fail;
  a.job_counter = nullptr;  // set per bucket by run_scc
  a.tol = c->tol;
  a.max_iter = c->max_iter;
  a.alpha = c->alpha;
  a.w0 = c->w0;
  return a;
}

bool bucket_queue(const cavdftb_ctx* c, const Bucket& b) { return b.job_queue >= 0 ? b.job_queue != 0 : c->dynamic_jobs != 0; }

int run_scc(cavdftb_ctx* c, const Bucket& b, SccArgs& a, hipStream_t stream) {
  if (a.n_jobs <= 0) return CAVDFTB_OK;
  a.scratch = b.d_scratch;
  a.scratch_per_wg = b.scratch_per_wg;
  a.eig_mode = b.eig_mode >= 0 ? b.eig_mode : c->eig_mode;
  a.job_counter = bucket_queue(c, b) ? c->d_job_counter + b.idx : nullptr;
  const int n_wg = a.n_jobs < b.n_wg ? a.n_jobs : b.n_wg;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (c->timing) {
    if (c->ev_pending.size() > 4096) harvest_events(c);
    ev = get_events(c);
    hipEventRecord(ev.first, stream);
  }
  hipError_t e = launch_scc(b.nmax, n_wg, a, stream);
  if (e != hipSuccess) return hip_fail(c, e, "scc kernel launch");
  if (c->timing) {
    hipEventRecord(ev.second, stream);
    c->ev_pending.push_back(ev);
  }
  c->launches += 1;
  return CAVDFTB_OK;
}

// SCC of every unit at pos (center jobs); writes the context work arrays
int32_t center_flags(cavdftb_ctx* c, bool forces) {
  int32_t flags = JF_STORE | JF_STORE_HIST | (forces ? JF_FORCES : 0);
  if (c->warm_enabled && c->warm_valid) flags |= JF_WARM_C | JF_WARM_DQ | (c->keep_hist ? JF_WARM_HIST : 0);
  return flags;
}

// The bucket launches of one undisplaced evaluation spread over up to
// n_streams streams: buckets by estimated cost, largest first, each to the
// stream with the least work so far (stream 0 is the context stream).  The
// side streams wait for the context stream's earlier work (fork) and the
// context stream waits for theirs (join).
struct BucketFan {
  cavdftb_ctx* c;
  int ns;
  double load[4] = {0.0, 0.0, 0.0, 0.0};
  std::vector<int> order;

  // a step captured into a graph keeps its launches on the context stream: the
  // graph then holds no cross-stream event dependencies, and a recapture reuses
  // no event of a destroyed graph
  explicit BucketFan(cavdftb_ctx* ctx)
      : c(ctx), ns(ctx->capturing ? 1 : std::min(ctx->n_streams, (int)ctx->buckets.size())) {
    order.resize(c->buckets.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return c->buckets[x].cost > c->buckets[y].cost; });
  }
  int fork() {
    if (ns <= 1) return CAVDFTB_OK;
    hipError_t e = hipEventRecord(c->ev_fork, c->stream);
    for (int j = 1; j < ns && e == hipSuccess; ++j) e = hipStreamWaitEvent(c->side[j - 1], c->ev_fork, 0);
    return e == hipSuccess ? CAVDFTB_OK : hip_fail(c, e, "bucket streams fork");
  }
  hipStream_t stream_for(const Bucket& b) {
    int slot = 0;
    for (int j = 1; j < ns; ++j)
      if (load[j] < load[slot]) slot = j;
    load[slot] += b.cost;
    return slot == 0 ? c->stream : c->side[slot - 1];
  }
  int join() {
    if (ns <= 1) return CAVDFTB_OK;
    hipError_t e = hipSuccess;
    for (int j = 1; j < ns && e == hipSuccess; ++j) {
      e = hipEventRecord(c->ev_join[j - 1], c->side[j - 1]);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->ev_join[j - 1], 0);
    }
    return e == hipSuccess ? CAVDFTB_OK : hip_fail(c, e, "bucket streams join");
  }
};

int eval_center(cavdftb_ctx* c, const double* pos, bool forces, bool md = false) {
  const int32_t flags = center_flags(c, forces);
  const bool extrap = md && c->warm_enabled && c->warm_valid;
  BucketFan fan(c);
  if (int rc = fan.fork()) return rc;
  for (int bi : fan.order) {
    const Bucket& b = c->buckets[bi];
    hipStream_t bs = fan.stream_for(b);
    SccArgs a = base_args(c, pos);
    if (md) {
      a.ws_dq_hist = c->d_ws_dq_hist;
      a.n_extrap = extrap ? (c->md_hist < 3 ? c->md_hist : 3) : 0;
    }
    // MD evaluations take the units in the order of their last cost (largest
    // first); the job arrays then follow that order
    a.job_unit = md ? b.d_order : b.d_units;
    a.job_disp = nullptr;
    a.n_jobs = b.n_units;
    a.energy = c->d_energy;
    a.forces = c->d_forces;
    a.charges = c->d_charges;
    a.dipole = c->d_dipole;
    a.status = c->d_status;
    a.job_status = c->d_cjob_status + b.cjob0;
    a.job_iters = c->d_cjob_iters + b.cjob0;
    a.flags = flags;
    int rc = run_scc(c, b, a, bs);
    if (rc) return rc;
    if (md && bucket_queue(c, b)) {
      hipError_t e = launch_order_by_cost(b.n_units, b.d_order, a.job_iters, c->d_cost_scale, b.d_order_tmp, bs);
      if (e != hipSuccess) return hip_fail(c, e, "job order");
    }
  }
  if (int rc = fan.join()) return rc;
  c->md_hist = (md && extrap) ? c->md_hist + 1 : (md && c->warm_enabled ? 1 : 0);
  c->warm_valid = c->warm_enabled != 0;
  return CAVDFTB_OK;
}

// displaced SCCs for the central-difference Born charges; needs eval_center
// first.  With unit_flag, only the flagged units (compacted on the device).
int eval_fd(cavdftb_ctx* c, const double* pos, double h, double* born, const int32_t* unit_flag = nullptr) {
  for (const Bucket& b : c->buckets) {
    SccArgs a = base_args(c, pos);
    const int32_t* job0 = b.d_fd_job0;
    if (unit_flag) {
      hipError_t e = launch_fd_compact(b.n_units, b.d_units, c->d_unit_off, unit_flag, 0, b.d_fb_job_unit,
                                       b.d_fb_job_disp, b.d_fb_job0, b.d_fb_n, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "fallback compaction");
      a.job_unit = b.d_fb_job_unit;
      a.job_disp = b.d_fb_job_disp;
      a.n_jobs_dev = b.d_fb_n;
      job0 = b.d_fb_job0;
    } else {
      a.job_unit = b.d_fd_job_unit;
      a.job_disp = b.d_fd_job_disp;
    }
    a.n_jobs = b.n_fd_jobs;  // capacity; the device count bounds the compacted list
    a.fd_h = h;
    a.mu_job = c->d_mu_job + (int64_t)b.fjob0 * 3;
    a.job_status = c->d_fjob_status + b.fjob0;
    a.job_iters = c->d_fjob_iters + b.fjob0;
    a.flags = JF_WARM_C | JF_WARM_DQ;  // fresh mixer: the stored history belongs to undisplaced SCCs
    // +h jobs first; the -h jobs then start from the +h charges reflected
    // through the centre, second order in h instead of first (fallback lists
    // too, so that their results equal the full route's bit for bit)
    a.fd_dq = c->d_fd_dq;
    a.fd_dq_off = c->d_fd_dq_off;
    for (int pass = 1; pass <= 2; ++pass) {
      a.fd_pass = pass;
      int rc = run_scc(c, b, a, c->stream);
      if (rc) return rc;
    }
    hipError_t e = launch_born_fd_assemble(c->d_unit_off, b.d_fd_unit, job0, b.n_units,
                                           c->d_mu_job + (int64_t)b.fjob0 * 3, h, c->pol,
                                           c->d_fjob_status + b.fjob0, unit_flag, born, c->d_zpol, c->d_status,
                                           c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "born fd assemble");
  }
  return CAVDFTB_OK;
}

// field-perturbed SCCs (six per unit) for the Born charges from the Maxwell
// relation; needs eval_center first.  With unit_flag, only the flagged units.
int eval_field(cavdftb_ctx* c, const double* pos, double e_field, double* born, const int32_t* unit_flag = nullptr) {
  for (const Bucket& b : c->buckets) {
    SccArgs a = base_args(c, pos);
    if (unit_flag) {
      hipError_t e = launch_fd_compact(b.n_units, b.d_units, c->d_unit_off, unit_flag, 1, b.d_fb_job_unit,
                                       b.d_fb_job_disp, b.d_fb_job0, b.d_fb_n, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "fallback compaction");
      a.job_unit = b.d_fb_job_unit;
      a.job_disp = b.d_fb_job_disp;
      a.n_jobs_dev = b.d_fb_n;
    } else {
      a.job_unit = b.d_ff_job_unit;
      a.job_disp = b.d_ff_job_disp;
    }
    a.n_jobs = 6 * b.n_units;  // capacity; the device count bounds the compacted list
    a.fd_h = e_field;
    a.f_job = c->d_f_job;
    a.f_status = c->d_f_status;
    a.job_status = c->d_fjob_status + b.fjob0;  // 6 n_units <= the bucket's displaced-job slots
    a.job_iters = c->d_fjob_iters + b.fjob0;
    a.flags = JF_FORCES | JF_WARM_C | JF_WARM_DQ;  // fresh mixer, as for displaced jobs
    a.fd_dq = c->d_fd_dq;  // -field jobs start from the +field charges reflected through the centre
    a.fd_dq_off = c->d_fd_dq_off;
    for (int pass = 1; pass <= 2; ++pass) {  // also for fallback lists: their results equal the full route's
      a.fd_pass = pass;
      int rc = run_scc(c, b, a, c->stream);
      if (rc) return rc;
    }
  }
  hipError_t e = launch_born_field_assemble(c->NA, c->d_atom_unit, c->d_unit_off, c->d_f_job, e_field, c->pol,
                                            c->d_f_status, unit_flag, born, c->d_zpol, c->d_status, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "born field assemble");
  return CAVDFTB_OK;
}

// forward-difference displaced SCCs (3 per atom) against the undisplaced
// dipoles of eval_center, which must run first
int eval_fd_forward(cavdftb_ctx* c, const double* pos, double h, double* born) {
  for (const Bucket& b : c->buckets) {
    SccArgs a = base_args(c, pos);
    a.job_unit = b.d_fw_job_unit;
    a.job_disp = b.d_fw_job_disp;
    a.n_jobs = b.n_fw_jobs;
    a.fd_h = h;
    a.mu_job = c->d_mu_job + (int64_t)b.fjob0 * 3;
    a.job_status = c->d_fjob_status + b.fjob0;
    a.job_iters = c->d_fjob_iters + b.fjob0;
    a.flags = JF_WARM_C | JF_WARM_DQ;  // fresh mixer, as for central differences
    int rc = run_scc(c, b, a, c->stream);
    if (rc) return rc;
    hipError_t e = launch_born_fd_forward_assemble(c->d_unit_off, b.d_fd_unit, b.d_fw_job0, b.n_units,
                                                   c->d_mu_job + (int64_t)b.fjob0 * 3, c->d_dipole, h, c->pol,
                                                   c->d_fjob_status + b.fjob0, born, c->d_zpol, c->d_status,
                                                   c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "born fd forward assemble");
  }
  return CAVDFTB_OK;
}

// exact Born charges by the route of mode (displacements, central or forward, or field)
int eval_exact(cavdftb_ctx* c, int mode, const double* pos, double h, double* born, const int32_t* unit_flag = nullptr) {
  if (mode == CAVDFTB_BORN_FIELD) return eval_field(c, pos, h, born, unit_flag);
  if (mode == CAVDFTB_BORN_FD_FORWARD) return eval_fd_forward(c, pos, h, born);
  return eval_fd(c, pos, h, born, unit_flag);
}

bool exact_mode(int mode) {
  return mode == CAVDFTB_BORN_FD || mode == CAVDFTB_BORN_FD_FORWARD || mode == CAVDFTB_BORN_FIELD;
}

bool born_mode_ok(int mode) {
  return mode == CAVDFTB_BORN_MULLIKEN || mode == CAVDFTB_BORN_FD || mode == CAVDFTB_BORN_SURROGATE ||
         mode == CAVDFTB_BORN_FIELD || mode == CAVDFTB_BORN_FD_FORWARD;
}

// surrogate Born charges at pos into born (ensemble mean, acoustic sum imposed),
// ensemble spread into d_sg_std and the fallback flags into d_unit_flag
int sg_infer(cavdftb_ctx* c, const double* pos, double* born) {
  hipStream_t st = c->stream;
  hipError_t e = launch_sg_features(c->NA, c->d_atom_unit, c->d_unit_off, c->d_species, pos, c->d_sg_feat,
                                    c->d_sg_frames, st);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate features");
  int64_t off = 0, ybase = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = c->n_sp[sp];
    if (n > 0) {
      e = launch_sg_prep(n, CAVDFTB_SG_N_IN, c->d_sp_idx + off, c->d_sg_feat, c->d_sg_norm + sp * CAVDFTB_SG_N_NORM,
                         c->d_sg_x + off * CAVDFTB_SG_N_IN, st);
      for (int m = 0; m < CAVDFTB_SG_MEMBERS && e == hipSuccess; ++m)
        e = launch_sg_forward(c->d_sg_params + ((int64_t)sp * CAVDFTB_SG_MEMBERS + m) * CAVDFTB_SG_N_PARAM,
                              c->d_sg_x + off * CAVDFTB_SG_N_IN, n,
                              c->d_sg_y + ybase + (int64_t)m * n * CAVDFTB_SG_N_OUT, nullptr, st);
      if (e != hipSuccess) return hip_fail(c, e, "surrogate forward");
    }
    off += n;
    ybase += (int64_t)CAVDFTB_SG_MEMBERS * n * CAVDFTB_SG_N_OUT;
  }
  e = launch_sg_combine(c->NA, c->d_species, c->d_pos_in_sp, c->d_n_sp, c->d_sg_y, c->d_sg_norm, c->d_sg_frames,
                        c->d_charges, born, c->d_sg_std, st);
  if (e == hipSuccess)
    e = launch_sg_asr_flag(c->U, c->d_unit_off, born, c->d_sg_std, c->sg_thr, c->d_unit_flag, c->d_counters + 4, st);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate combine");
  return CAVDFTB_OK;
}

CavArgs cav_args(cavdftb_ctx* c) {
  CavArgs a{};
  a.n_units = c->U;
  a.n_atoms = c->NA;
  a.n_modes = c->M;
  a.unit_x = c->d_unit_x;
  a.k = c->d_k;
  a.theta = c->d_theta;
  a.omega = c->d_omega;
  a.lam = c->d_lam;
  for (int g = 0; g < 3; ++g) a.pol[g] = c->pol[g];
  return a;
}

// matter + Born stage at r: forces, energy, dipole, e.Z into the work arrays
int matter_stage(cavdftb_ctx* c, const double* r, int born_mode, double h) {
  int rc = eval_center(c, r, true, true);
  if (rc) return rc;
  hipError_t e;
  if (exact_mode(born_mode)) {
    // refreshed on every born_every-th evaluation since priming; e.Z kept in between
    const bool refresh = c->born_count % c->born_every == 0;
    c->born_count += 1;
    if (refresh) {
      rc = eval_exact(c, born_mode, r, h, nullptr);
      if (rc) return rc;
    }
  } else if (born_mode == CAVDFTB_BORN_SURROGATE) {
    rc = sg_infer(c, r, c->d_born);
    if (rc == CAVDFTB_OK) rc = eval_exact(c, c->fallback_mode, r, h, c->d_born, c->d_unit_flag);
    if (rc) return rc;
    e = launch_zpol_from_born(c->NA, c->d_born, c->pol, c->d_zpol, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "zpol");
  } else {
    e = launch_zpol_mulliken(c->d_charges, c->pol, c->NA, c->d_zpol, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "zpol");
  }
  e = launch_mu_pol(c->d_dipole, c->pol, c->U, c->d_status, c->d_mu_pol, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "mu_pol");
  return CAVDFTB_OK;
}

// the launches of one MD step (velocity Verlet with the cavity field; the
// matter stage and the cavity force at the new positions in between)
int issue_step(cavdftb_ctx* c, double* r, double* p, double* qm, double* pm, double dt, int32_t born_mode,
               double h_fd, double* obs) {
  hipStream_t s = c->stream;
  CavArgs ca = cav_args(c);
  hipError_t e = launch_photon_kick(c->M, c->d_omega, c->d_lam, c->d_F, dt, pm, 0, qm, s);
  if (e == hipSuccess)
    e = launch_kick_drift(c->NA, c->d_atom_unit, c->d_inv_mass, c->d_forces, c->d_zpol, c->d_field, dt, r, p, 1,
                          c->d_status, s);
  if (e != hipSuccess) return hip_fail(c, e, "step kick/drift");
  int rc = matter_stage(c, r, born_mode, h_fd);
  if (rc) return rc;
  e = launch_cav_scatter(ca, c->d_mu_pol, c->d_F, nullptr, s);
  if (e == hipSuccess) e = launch_cav_gather(ca, qm, c->d_F, c->d_field, s);  // old q
  if (e == hipSuccess)
    e = launch_kick_drift(c->NA, c->d_atom_unit, c->d_inv_mass, c->d_forces, c->d_zpol, c->d_field, dt, r, p, 0,
                          c->d_status, s);
  if (e == hipSuccess) e = launch_photon_kick(c->M, c->d_omega, c->d_lam, c->d_F, dt, pm, 1, qm, s);
  if (e == hipSuccess) e = launch_cav_gather(ca, qm, c->d_F, c->d_field, s);  // rotated q
  if (e == hipSuccess && obs)
    e = launch_observables(c->U, c->NA, c->M, c->d_unit_off, c->d_mass, p, c->d_energy, qm, pm, c->d_omega, c->d_lam,
                           c->d_F, c->d_mu_pol, c->d_status, c->d_cjob_iters, c->U, c->d_obs_part, c->obs_part_rows,
                           obs, c->d_obs_row, s);
  if (e != hipSuccess) return hip_fail(c, e, "step cavity/kick");
  return CAVDFTB_OK;
}

// true when the launches of the next MD step are those of the step after it:
// primed, no per-launch timing events, a capturable stream, and the warm-start
// extrapolation at its full depth (or warm starts off)
bool graph_steady(const cavdftb_ctx* c) {
  return c->use_graph && c->primed && !c->timing && c->stream != nullptr &&
         (!c->warm_enabled || (c->warm_valid && c->md_hist >= 3));
}

// one MD step as a replay of the captured graph; captured (again) when the
// arguments or a setting changed since the last capture
int replay_step(cavdftb_ctx* c, double* r, double* p, double* qm, double* pm, double dt, int32_t born_mode,
                double h_fd, double* obs) {
  const void* key[5] = {r, p, qm, pm, obs};
  bool same = c->graph_exec && c->graph_gen == c->gen && c->graph_dt == dt && c->graph_h == h_fd &&
              c->graph_born == born_mode;
  for (int k = 0; k < 5 && same; ++k) same = c->graph_key[k] == key[k];
  if (!same) {
    drop_graph(c);
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(c, e, "graph capture begin");
    const int64_t l0 = c->launches;
    c->capturing = true;
    const int rc = issue_step(c, r, p, qm, pm, dt, born_mode, h_fd, obs);
    c->capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "graph capture end");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(g);
      return hip_fail(c, e, "graph instantiate");
    }
    c->graph = g;
    c->graph_exec = x;
    c->graph_gen = c->gen;
    c->graph_dt = dt;
    c->graph_h = h_fd;
    c->graph_born = born_mode;
    for (int k = 0; k < 5; ++k) c->graph_key[k] = key[k];
    c->graph_scc_launches = c->launches - l0;
    c->launches = l0;
    c->graph_captures += 1;
  }
  const hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "graph launch");
  c->launches += c->graph_scc_launches;
  c->graph_replays += 1;
  return CAVDFTB_OK;
}

}  // namespace

extern "C" {

const char* cavdftb_version(void) { return "cavdftb 0.1 (gfx950)"; }

const char* cavdftb_last_error(const cavdftb_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int cavdftb_create(const cavdftb_params* params, const cavdftb_layout* L, void* hip_stream, cavdftb_ctx** out) {
  if (!params || !L || !out) return CAVDFTB_EINVAL;
  *out = nullptr;
  if (L->n_units <= 0 || L->n_atoms <= 0 || L->n_modes < 0 || !L->unit_atom_off || !L->species || !L->unit_x)
    return CAVDFTB_EINVAL;
  if (L->n_modes > 0 && (!L->omega || !L->k || !L->theta || !L->lam)) return CAVDFTB_EINVAL;
  cavdftb_ctx* c = new (std::nothrow) cavdftb_ctx();
  if (!c) return CAVDFTB_ENOMEM;
  c->stream = (hipStream_t)hip_stream;
  c->U = L->n_units;
  c->NA = L->n_atoms;
  c->M = L->n_modes;
  for (int g = 0; g < 3; ++g) c->pol[g] = L->pol[g];
  memcpy(c->prm.sk, params->sk, sizeof(c->prm.sk));
  memcpy(c->prm.onsite, params->onsite, sizeof(c->prm.onsite));
  memcpy(c->prm.U, params->hubbard_u, sizeof(c->prm.U));
  if (!(params->q0[0] >= 0.0 && params->q0[0] <= 8.0 && params->q0[1] >= 0.0 && params->q0[1] <= 2.0)) {
    delete c;  // neutral valence populations must fit the minimal basis (O: 4 orbitals, H: 1)
    return CAVDFTB_EINVAL;
  }
  memcpy(c->prm.q0, params->q0, sizeof(c->prm.q0));
  memcpy(c->prm.rep_a, params->rep_a, sizeof(c->prm.rep_a));
  memcpy(c->prm.rep_alpha, params->rep_alpha, sizeof(c->prm.rep_alpha));
  c->mass[0] = params->mass[0];
  c->mass[1] = params->mass[1];

  // ---- validate the layout and size buckets (host)
  const int U = c->U, NA = c->NA;
  c->h_unit_off.assign(L->unit_atom_off, L->unit_atom_off + U + 1);
  if (c->h_unit_off[0] != 0 || c->h_unit_off[U] != NA) {
    delete c;
    return CAVDFTB_EINVAL;
  }
  std::vector<int> n_orb(U);
  std::vector<int32_t> atom_unit(NA);
  std::vector<double> mass(NA), inv_mass(NA);
  for (int u = 0; u < U; ++u) {
    const int a0 = c->h_unit_off[u], a1 = c->h_unit_off[u + 1];
    if (a1 <= a0) {
      delete c;
      return CAVDFTB_EINVAL;
    }
    int n = 0;
    for (int a = a0; a < a1; ++a) {
      const int s = L->species[a];
      if (s != 0 && s != 1) {
        delete c;
        return CAVDFTB_EINVAL;
      }
      n += s == 0 ? 4 : 1;
      atom_unit[a] = u;
      mass[a] = params->mass[s];
      inv_mass[a] = 1.0 / params->mass[s];
    }
    if (n > CAVDFTB_MAX_ORBITALS || (n & 1)) {
      delete c;
      return CAVDFTB_EINVAL;
    }
    n_orb[u] = n;
  }
  int dev = 0, n_cu = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (n_cu <= 0) n_cu = 256;
  c->n_cu = n_cu;

  const int* nmaxs = kBucketNmax;
  std::vector<int64_t> ws_off(U), hist_off(U);
  int64_t ws_total = 0, hist_total = 0;
  std::vector<std::vector<int32_t>> bunits(kNumBuckets);
  for (int u = 0; u < U; ++u) {
    const int nm = bucket_of(n_orb[u]);
    for (int k = 0; k < kNumBuckets; ++k)
      if (nmaxs[k] == nm) bunits[k].push_back(u);
    ws_off[u] = ws_total;
    ws_total += (int64_t)nm * nm;
    hist_off[u] = hist_total;
    hist_total += hist_doubles(nm);
  }
  // largest units first in every bucket (longest-processing-time order for the job queue)
  for (auto& v : bunits)
    std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return n_orb[x] > n_orb[y]; });
  hipError_t e = hipSuccess;
#define CK(x)                                  \
  do {                                         \
    e = (x);                                   \
    if (e != hipSuccess) {                     \
      release(c);                              \
      delete c;                                \
      return e == hipErrorOutOfMemory ? CAVDFTB_ENOMEM : CAVDFTB_EHIP; \
    }                                          \
  } while (0)
  const int M = c->M > 0 ? c->M : 1;
  CK(dalloc(c, &c->d_unit_off, U + 1));
  CK(dalloc(c, &c->d_species, NA));
  CK(dalloc(c, &c->d_unit_x, U));
  CK(dalloc(c, &c->d_omega, M));
  CK(dalloc(c, &c->d_k, M));
  CK(dalloc(c, &c->d_theta, M));
  CK(dalloc(c, &c->d_lam, M));
  CK(dalloc(c, &c->d_atom_unit, NA));
  CK(dalloc(c, &c->d_mass, NA));
  CK(dalloc(c, &c->d_inv_mass, NA));
  CK(dalloc(c, &c->d_ws_off, U));
  CK(dalloc(c, &c->d_ws_C, ws_total));
  CK(dalloc(c, &c->d_ws_dq, NA));
  CK(dalloc(c, &c->d_ws_dq_hist, 2 * (size_t)NA));
  {
    std::vector<int64_t> off(U);
    int64_t tot = 0;
    for (int u = 0; u < U; ++u) {
      const int64_t na = c->h_unit_off[u + 1] - c->h_unit_off[u];
      off[u] = tot;
      tot += 3 * na * na + 3 * na;  // displaced slots, then field slots
    }
    CK(dalloc(c, &c->d_fd_dq_off, (size_t)U));
    CK(dalloc(c, &c->d_fd_dq, (size_t)tot));
    CK(hipMemset(c->d_fd_dq, 0, (size_t)tot * sizeof(double)));
    c->fd_dq_count = tot;
    CK(hipMemcpy(c->d_fd_dq_off, off.data(), U * sizeof(int64_t), hipMemcpyHostToDevice));
  }
  CK(dalloc(c, &c->d_hist_off, U));
  CK(dalloc(c, &c->d_hist, hist_total));
  CK(dalloc(c, &c->d_energy, U));
  CK(dalloc(c, &c->d_forces, (size_t)NA * 3));
  CK(dalloc(c, &c->d_charges, NA));
  CK(dalloc(c, &c->d_dipole, (size_t)U * 3));
  CK(dalloc(c, &c->d_mu_pol, U));
  CK(dalloc(c, &c->d_F, M));
  CK(dalloc(c, &c->d_fq, M));
  CK(dalloc(c, &c->d_field, U));
  CK(dalloc(c, &c->d_zpol, (size_t)NA * 3));
  CK(dalloc(c, &c->d_status, U));
  CK(dalloc(c, &c->d_unit_fail, U));
  CK(hipMemset(c->d_unit_fail, 0, (size_t)U * sizeof(int32_t)));
  CK(dalloc(c, &c->d_cjob_status, U));
  CK(dalloc(c, &c->d_cjob_iters, U));
  CK(dalloc(c, &c->d_sg_params, 2 * (size_t)CAVDFTB_SG_MEMBERS * CAVDFTB_SG_N_PARAM));
  CK(dalloc(c, &c->d_sg_norm, 2 * (size_t)CAVDFTB_SG_N_NORM));
  CK(dalloc(c, &c->d_sg_feat, (size_t)NA * CAVDFTB_SG_N_IN));
  CK(dalloc(c, &c->d_sg_frames, (size_t)NA * 9));
  CK(dalloc(c, &c->d_sg_x, (size_t)NA * CAVDFTB_SG_N_IN));
  CK(dalloc(c, &c->d_sg_y, (size_t)CAVDFTB_SG_MEMBERS * NA * CAVDFTB_SG_N_OUT));
  CK(dalloc(c, &c->d_sg_std, NA));
  CK(dalloc(c, &c->d_born, (size_t)NA * 9));
  CK(dalloc(c, &c->d_unit_flag, U));
  CK(dalloc(c, &c->d_sp_idx, NA));
  CK(dalloc(c, &c->d_pos_in_sp, NA));
  CK(dalloc(c, &c->d_n_sp, 2));
  {
    std::vector<int32_t> idx, pos_in(NA);
    for (int sp = 0; sp < 2; ++sp) {
      int k = 0;
      for (int a2 = 0; a2 < NA; ++a2)
        if (L->species[a2] == sp) {
          idx.push_back(a2);
          pos_in[a2] = k++;
        }
      c->n_sp[sp] = k;
    }
    CK(hipMemcpy(c->d_sp_idx, idx.data(), NA * sizeof(int32_t), hipMemcpyHostToDevice));
    CK(hipMemcpy(c->d_pos_in_sp, pos_in.data(), NA * sizeof(int32_t), hipMemcpyHostToDevice));
    CK(hipMemcpy(c->d_n_sp, c->n_sp, 2 * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  CK(dalloc(c, &c->d_counters, 8));
  CK(dalloc(c, &c->d_job_counter, kNumBuckets));
  for (int j = 0; j < 3; ++j) {
    CK(hipStreamCreateWithFlags(&c->side[j], hipStreamNonBlocking));
    CK(hipEventCreateWithFlags(&c->ev_join[j], hipEventDisableTiming));
  }
  CK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  CK(dalloc(c, &c->d_obs_row, 1));
  c->obs_part_rows = observables_part_rows(std::max(U, c->M));
  CK(dalloc(c, &c->d_obs_part, (size_t)c->obs_part_rows * 8));
  CK(dalloc(c, &c->d_rs_wk, U));
  CK(dalloc(c, &c->d_rs_qk, U));
  CK(dalloc(c, &c->d_rs_pk, U));
  CK(dalloc(c, &c->d_rs_buf0, U));
  CK(dalloc(c, &c->d_rs_buf1, U));
  CK(hipMemcpy(c->d_unit_off, c->h_unit_off.data(), (U + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  CK(hipMemcpy(c->d_species, L->species, NA, hipMemcpyHostToDevice));
  CK(hipMemcpy(c->d_unit_x, L->unit_x, U * sizeof(double), hipMemcpyHostToDevice));
  if (c->M > 0) {
    CK(hipMemcpy(c->d_omega, L->omega, c->M * sizeof(double), hipMemcpyHostToDevice));
    CK(hipMemcpy(c->d_k, L->k, c->M * sizeof(double), hipMemcpyHostToDevice));
    CK(hipMemcpy(c->d_theta, L->theta, c->M * sizeof(double), hipMemcpyHostToDevice));
    CK(hipMemcpy(c->d_lam, L->lam, c->M * sizeof(double), hipMemcpyHostToDevice));
  }
  CK(hipMemcpy(c->d_atom_unit, atom_unit.data(), NA * sizeof(int32_t), hipMemcpyHostToDevice));
  CK(hipMemcpy(c->d_mass, mass.data(), NA * sizeof(double), hipMemcpyHostToDevice));
  CK(hipMemcpy(c->d_inv_mass, inv_mass.data(), NA * sizeof(double), hipMemcpyHostToDevice));
  CK(hipMemcpy(c->d_ws_off, ws_off.data(), U * sizeof(int64_t), hipMemcpyHostToDevice));
  CK(hipMemset(c->d_ws_dq, 0, NA * sizeof(double)));
  CK(hipMemcpy(c->d_hist_off, hist_off.data(), U * sizeof(int64_t), hipMemcpyHostToDevice));
  CK(hipMemset(c->d_hist, 0, hist_total * sizeof(double)));
  CK(hipMemset(c->d_counters, 0, 8 * sizeof(unsigned long long)));
  CK(hipMemset(c->d_status, 0, U * sizeof(int32_t)));
  CK(hipMemset(c->d_cjob_iters, 0, U * sizeof(int32_t)));
  CK(hipMemset(c->d_energy, 0, U * sizeof(double)));

  // ---- buckets: unit lists, scratch, finite-difference job lists
  int cj = 0, fj = 0;
  std::vector<float> cost_scale(U, 0.0f);
  for (int k = 0; k < kNumBuckets; ++k) {
    if (bunits[k].empty()) continue;
    Bucket b;
    b.idx = (int)c->buckets.size();
    b.nmax = nmaxs[k];
    b.n_units = (int)bunits[k].size();
    b.cjob0 = cj;
    cj += b.n_units;
    b.scratch_per_wg = scc_scratch_per_wg(b.nmax);
    int per_cu = scc_blocks_per_cu(b.nmax);
    if (b.nmax > 64 && per_cu > 2) per_cu = 2;  // global-scratch buckets: bound the cache footprint
    b.per_cu_max = per_cu;
    b.n_wg = n_cu * per_cu;
    CK(dalloc(c, &b.d_units, b.n_units));
    CK(hipMemcpy(b.d_units, bunits[k].data(), b.n_units * sizeof(int32_t), hipMemcpyHostToDevice));
    for (int u : bunits[k]) {
      int norb = 0;
      for (int a = c->h_unit_off[u]; a < c->h_unit_off[u + 1]; ++a) norb += L->species[a] == 0 ? 4 : 1;
      const double f = (double)norb / b.nmax;
      cost_scale[u] = (float)(f * f * f);
      const double g = (double)norb / 48.0;
      b.cost += g * g * g;
    }
    CK(dalloc(c, &b.d_order, b.n_units));
    CK(dalloc(c, &b.d_order_tmp, b.n_units));
    CK(hipMemcpy(b.d_order, bunits[k].data(), b.n_units * sizeof(int32_t), hipMemcpyHostToDevice));
    CK(dalloc(c, &b.d_scratch, (size_t)b.n_wg * b.scratch_per_wg));
    std::vector<int32_t> jun, jdisp, fdu, fdj0;
    for (int u : bunits[k]) {
      const int na = c->h_unit_off[u + 1] - c->h_unit_off[u];
      fdu.push_back(u);
      fdj0.push_back((int32_t)jun.size());
      for (int a = 0; a < na; ++a)
        for (int dir = 0; dir < 3; ++dir)
          for (int sg = 0; sg < 2; ++sg) {
            jun.push_back(u);
            jdisp.push_back((a * 3 + dir) * 2 + sg);
          }
    }
    b.n_fd_jobs = (int)jun.size();
    b.fjob0 = fj;
    fj += b.n_fd_jobs;
    CK(dalloc(c, &b.d_fd_job_unit, b.n_fd_jobs));
    CK(dalloc(c, &b.d_fd_job_disp, b.n_fd_jobs));
    CK(dalloc(c, &b.d_fd_unit, b.n_units));
    CK(dalloc(c, &b.d_fd_job0, b.n_units));
    CK(dalloc(c, &b.d_ff_job_unit, 6 * (size_t)b.n_units));
    CK(dalloc(c, &b.d_ff_job_disp, 6 * (size_t)b.n_units));
    CK(dalloc(c, &b.d_fb_job_unit, b.n_fd_jobs));
    CK(dalloc(c, &b.d_fb_job_disp, b.n_fd_jobs));
    CK(dalloc(c, &b.d_fb_job0, b.n_units));
    CK(dalloc(c, &b.d_fb_n, 1));
    CK(hipMemcpy(b.d_fd_job_unit, jun.data(), jun.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    CK(hipMemcpy(b.d_fd_job_disp, jdisp.data(), jdisp.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    CK(hipMemcpy(b.d_fd_unit, fdu.data(), fdu.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    CK(hipMemcpy(b.d_fd_job0, fdj0.data(), fdj0.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    {
      std::vector<int32_t> wu, wd, w0;
      for (int u : bunits[k]) {
        const int na = c->h_unit_off[u + 1] - c->h_unit_off[u];
        w0.push_back((int32_t)wu.size());
        for (int a = 0; a < na; ++a)
          for (int dir = 0; dir < 3; ++dir) {
            wu.push_back(u);
            wd.push_back((a * 3 + dir) * 2);  // + h
          }
      }
      b.n_fw_jobs = (int)wu.size();
      CK(dalloc(c, &b.d_fw_job_unit, b.n_fw_jobs));
      CK(dalloc(c, &b.d_fw_job_disp, b.n_fw_jobs));
      CK(dalloc(c, &b.d_fw_job0, b.n_units));
      CK(hipMemcpy(b.d_fw_job_unit, wu.data(), wu.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      CK(hipMemcpy(b.d_fw_job_disp, wd.data(), wd.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      CK(hipMemcpy(b.d_fw_job0, w0.data(), w0.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    {
      std::vector<int32_t> fu, fd;
      for (int u : bunits[k])
        for (int code = 0; code < 6; ++code) {
          fu.push_back(u);
          fd.push_back(-2 - code);
        }
      CK(hipMemcpy(b.d_ff_job_unit, fu.data(), fu.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      CK(hipMemcpy(b.d_ff_job_disp, fd.data(), fd.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    c->buckets.push_back(b);
  }
  CK(dalloc(c, &c->d_cost_scale, (size_t)U));
  CK(hipMemcpy(c->d_cost_scale, cost_scale.data(), U * sizeof(float), hipMemcpyHostToDevice));
  c->n_fd_total = fj;
  CK(dalloc(c, &c->d_mu_job, (size_t)fj * 3));
  CK(dalloc(c, &c->d_fjob_status, fj));
  CK(dalloc(c, &c->d_fjob_iters, fj));
  CK(dalloc(c, &c->d_f_job, 18 * (size_t)NA));
  CK(dalloc(c, &c->d_f_status, 6 * (size_t)U));
  hipLaunchKernelGGL(ws_identity_kernel, dim3(U), dim3(256), 0, c->stream, c->d_ws_C, c->d_ws_off, c->d_unit_off,
                     c->d_species, U, 0);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(c->stream));
#undef CK
  *out = c;
  return CAVDFTB_OK;
}

int cavdftb_destroy(cavdftb_ctx* ctx) {
  if (!ctx) return CAVDFTB_EINVAL;
  release(ctx);
  delete ctx;
  return CAVDFTB_OK;
}

int cavdftb_set_scc(cavdftb_ctx* ctx, double tol, int32_t max_iter, double mix_alpha) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  if (!(tol > 0.0) || max_iter < 1 || !(mix_alpha > 0.0) || mix_alpha > 1.0)
    return fail(ctx, CAVDFTB_EINVAL, "set_scc: need tol > 0, max_iter >= 1, 0 < alpha <= 1");
  ctx->tol = tol;
  ctx->max_iter = max_iter;
  ctx->alpha = mix_alpha;
  return CAVDFTB_OK;
}

int cavdftb_set_tuning(cavdftb_ctx* ctx, double jacobi_res_factor, int32_t keep_mixer_history) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  if (!(jacobi_res_factor >= 0.0) || jacobi_res_factor > 1.0)
    return fail(ctx, CAVDFTB_EINVAL, "set_tuning: need 0 <= jacobi_res_factor <= 1");
  ctx->jac_factor = jacobi_res_factor;
  ctx->keep_hist = keep_mixer_history ? 1 : 0;
  return CAVDFTB_OK;
}

int cavdftb_set_eigensolver(cavdftb_ctx* ctx, int32_t mode) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (mode != CAVDFTB_EIG_AUTO && mode != CAVDFTB_EIG_FULL && mode != CAVDFTB_EIG_JACOBI)
    return fail(ctx, CAVDFTB_EINVAL, "set_eigensolver: unknown mode");
  ctx->eig_mode = mode;
  ctx->gen += 1;
  return CAVDFTB_OK;
}

int cavdftb_set_schedule(cavdftb_ctx* ctx, int32_t job_queue, int32_t max_wg_per_cu) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  if (max_wg_per_cu < 0) return fail(ctx, CAVDFTB_EINVAL, "set_schedule: need max_wg_per_cu >= 0");
  ctx->dynamic_jobs = job_queue ? 1 : 0;
  for (Bucket& b : ctx->buckets) {
    const int per = max_wg_per_cu > 0 && max_wg_per_cu < b.per_cu_max ? max_wg_per_cu : b.per_cu_max;
    b.n_wg = ctx->n_cu * per;
  }
  return CAVDFTB_OK;
}

int cavdftb_set_bucket_schedule(cavdftb_ctx* ctx, int32_t bucket_orbitals, int32_t wg_per_cu, int32_t eig_mode,
                                int32_t job_queue) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (bucket_of(bucket_orbitals) != bucket_orbitals || wg_per_cu < 0 || eig_mode < -1 ||
      eig_mode > CAVDFTB_EIG_JACOBI || job_queue < -1 || job_queue > 1)
    return fail(ctx, CAVDFTB_EINVAL, "set_bucket_schedule: bad bucket or setting");
  ctx->gen += 1;
  for (Bucket& b : ctx->buckets) {
    if (b.nmax != bucket_orbitals) continue;
    const int per = wg_per_cu > 0 && wg_per_cu < b.per_cu_max ? wg_per_cu : b.per_cu_max;
    b.n_wg = ctx->n_cu * per;
    b.eig_mode = eig_mode;
    b.job_queue = job_queue;
  }
  return CAVDFTB_OK;
}

int cavdftb_set_bucket_streams(cavdftb_ctx* ctx, int32_t n_streams) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (n_streams < 1 || n_streams > 4) return fail(ctx, CAVDFTB_EINVAL, "set_bucket_streams: need 1 <= n <= 4");
  ctx->n_streams = n_streams;
  ctx->gen += 1;
  return CAVDFTB_OK;
}

int cavdftb_bucket_info(cavdftb_ctx* ctx, int32_t bucket_orbitals, int32_t* n_units, int32_t* wg_per_cu_max,
                        int32_t* wg_per_cu) {
  if (!ctx || bucket_of(bucket_orbitals) != bucket_orbitals) return CAVDFTB_EINVAL;
  int32_t nu = 0, mx = 0, cur = 0;
  for (const Bucket& b : ctx->buckets)
    if (b.nmax == bucket_orbitals) {
      nu = b.n_units;
      mx = b.per_cu_max;
      cur = b.n_wg / ctx->n_cu;
    }
  if (n_units) *n_units = nu;
  if (wg_per_cu_max) *wg_per_cu_max = mx;
  if (wg_per_cu) *wg_per_cu = cur;
  return CAVDFTB_OK;
}

// value of "key": in [p, q) as an integer or a string (no escapes); false when absent
static bool json_field(const std::string& t, size_t p, size_t q, const char* key, long* iv, std::string* sv) {
  const std::string k = std::string("\"") + key + "\"";
  size_t at = t.find(k, p);
  if (at == std::string::npos || at >= q) return false;
  at = t.find(':', at + k.size());
  if (at == std::string::npos || at >= q) return false;
  ++at;
  while (at < q && (t[at] == ' ' || t[at] == '\t' || t[at] == '\n' || t[at] == '\r')) ++at;
  if (at >= q) return false;
  if (t[at] == '"') {
    const size_t e = t.find('"', at + 1);
    if (e == std::string::npos || e >= q || !sv) return false;
    *sv = t.substr(at + 1, e - at - 1);
    return true;
  }
  if (!iv) return false;
  char* end = nullptr;
  const long v = strtol(t.c_str() + at, &end, 10);
  if (end == t.c_str() + at) return false;
  *iv = v;
  return true;
}

int cavdftb_load_launch_table(cavdftb_ctx* ctx, const char* path) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!path) return fail(ctx, CAVDFTB_EINVAL, "load_launch_table: null path");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(ctx, CAVDFTB_EINVAL, "load_launch_table: cannot open the file");
  std::string t;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) t.append(buf, got);
  fclose(f);
  std::string arch = "gfx950";
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      arch = prop.gcnArchName;
      const size_t colon = arch.find(':');
      if (colon != std::string::npos) arch.resize(colon);
    }
  }
  // every flat object holding a "bucket" key is one entry
  int applied = 0;
  for (size_t at = t.find("\"bucket\""); at != std::string::npos; at = t.find("\"bucket\"", at + 1)) {
    const size_t p = t.rfind('{', at), q = t.find('}', at);
    if (p == std::string::npos || q == std::string::npos)
      return fail(ctx, CAVDFTB_EINVAL, "load_launch_table: malformed entry");
    long bucket = 0, wg = 0, eig = -1, queue = -1;
    std::string a;
    if (!json_field(t, p, q, "bucket", &bucket, nullptr) || !json_field(t, p, q, "arch", nullptr, &a))
      return fail(ctx, CAVDFTB_EINVAL, "load_launch_table: entry without bucket or arch");
    json_field(t, p, q, "wg_per_cu", &wg, nullptr);
    json_field(t, p, q, "eig_mode", &eig, nullptr);
    json_field(t, p, q, "job_queue", &queue, nullptr);
    if (a != arch) continue;
    const int rc = cavdftb_set_bucket_schedule(ctx, (int32_t)bucket, (int32_t)wg, (int32_t)eig, (int32_t)queue);
    if (rc) return rc;
    ++applied;
  }
  return applied;
}

int cavdftb_set_warm_start(cavdftb_ctx* ctx, int32_t enable) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  ctx->warm_enabled = enable ? 1 : 0;
  if (!enable) ctx->warm_valid = false;
  return CAVDFTB_OK;
}

int cavdftb_reset_warm_start(cavdftb_ctx* ctx) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  ctx->warm_valid = false;
  ctx->md_hist = 0;
  // the charge responses of the finite-difference jobs start over too
  const hipError_t e = hipMemsetAsync(ctx->d_fd_dq, 0, (size_t)ctx->fd_dq_count * sizeof(double), ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "reset_warm_start");
  return CAVDFTB_OK;
}

int cavdftb_eval_units(cavdftb_ctx* ctx, const double* pos, double* energy, double* forces, double* charges,
                       double* dipole, int32_t* unit_status) {
  if (!ctx || !pos || !unit_status) return ctx ? fail(ctx, CAVDFTB_EINVAL, "eval_units: null pointer")
                                               : CAVDFTB_EINVAL;
  ctx->gen += 1;
  const bool want_f = energy || forces;
  const int32_t flags = center_flags(ctx, want_f);
  BucketFan fan(ctx);
  if (int rc = fan.fork()) return rc;
  for (int bi : fan.order) {
    const Bucket& b = ctx->buckets[bi];
    hipStream_t bs = fan.stream_for(b);
    SccArgs a = base_args(ctx, pos);
    a.job_unit = b.d_units;
    a.n_jobs = b.n_units;
    a.energy = energy;
    a.forces = forces;
    a.charges = charges;
    a.dipole = dipole;
    a.status = unit_status;
    a.job_status = ctx->d_cjob_status + b.cjob0;
    a.job_iters = ctx->d_cjob_iters + b.cjob0;
    a.flags = flags;
    int rc = run_scc(ctx, b, a, bs);
    if (rc) return rc;
  }
  if (int rc = fan.join()) return rc;
  ctx->warm_valid = ctx->warm_enabled != 0;
  ctx->primed = false;
  ctx->rs_primed = false;
  ctx->md_hist = 0;
  return CAVDFTB_OK;
}

int cavdftb_born_charges(cavdftb_ctx* ctx, const double* pos, int32_t mode, double h, double* born,
                         double* ens_std, int32_t* unit_status) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!pos || !born || (ens_std && mode != CAVDFTB_BORN_SURROGATE))
    return fail(ctx, CAVDFTB_EINVAL, "born_charges: bad pointer arguments");
  if (!born_mode_ok(mode)) return fail(ctx, CAVDFTB_EINVAL, "born_charges: unknown mode");
  if (mode != CAVDFTB_BORN_MULLIKEN && !(h > 0.0)) return fail(ctx, CAVDFTB_EINVAL, "born_charges: need h > 0");
  if (mode == CAVDFTB_BORN_SURROGATE && !ctx->sg_ready)
    return fail(ctx, CAVDFTB_EINVAL, "born_charges: no surrogate set (cavdftb_set_surrogate)");
  ctx->gen += 1;
  int rc = eval_center(ctx, pos, false);
  if (rc) return rc;
  ctx->primed = false;
  ctx->rs_primed = false;
  if (mode == CAVDFTB_BORN_MULLIKEN) {
    hipError_t e = launch_born_mulliken(ctx->d_charges, ctx->NA, born, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "born mulliken");
  } else if (exact_mode(mode)) {
    rc = eval_exact(ctx, mode, pos, h, born);
    if (rc) return rc;
  } else {
    rc = sg_infer(ctx, pos, born);
    if (rc == CAVDFTB_OK) rc = eval_exact(ctx, ctx->fallback_mode, pos, h, born, ctx->d_unit_flag);
    if (rc) return rc;
    if (ens_std) {
      hipError_t e = hipMemcpyAsync(ens_std, ctx->d_sg_std, ctx->NA * sizeof(double), hipMemcpyDeviceToDevice,
                                    ctx->stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "ens_std copy");
    }
  }
  if (unit_status) {
    hipError_t e = hipMemcpyAsync(unit_status, ctx->d_status, ctx->U * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                  ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "status copy");
  }
  return CAVDFTB_OK;
}

int cavdftb_read_work(cavdftb_ctx* ctx, int32_t which, double* dst) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!dst) return fail(ctx, CAVDFTB_EINVAL, "read_work: null destination");
  const double* src = nullptr;
  size_t count = 0;
  switch (which) {
    case CAVDFTB_WORK_MU_POL: src = ctx->d_mu_pol; count = ctx->U; break;
    case CAVDFTB_WORK_DIPOLE: src = ctx->d_dipole; count = 3 * (size_t)ctx->U; break;
    case CAVDFTB_WORK_ENERGY: src = ctx->d_energy; count = ctx->U; break;
    case CAVDFTB_WORK_CHARGES: src = ctx->d_charges; count = ctx->NA; break;
    case CAVDFTB_WORK_FORCES: src = ctx->d_forces; count = 3 * (size_t)ctx->NA; break;
    case CAVDFTB_WORK_FIELD: src = ctx->d_field; count = ctx->U; break;
    default: return fail(ctx, CAVDFTB_EINVAL, "read_work: unknown array");
  }
  const hipError_t e = hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
  return e == hipSuccess ? CAVDFTB_OK : hip_fail(ctx, e, "read_work copy");
}

int cavdftb_cavity_forces(cavdftb_ctx* ctx, const double* mu_pol, const double* q, double* F, double* field,
                          double* fq) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!mu_pol || (field && !q)) return fail(ctx, CAVDFTB_EINVAL, "cavity_forces: null input");
  CavArgs ca = cav_args(ctx);
  double* Fd = F ? F : ctx->d_F;
  hipError_t e = launch_cav_scatter(ca, mu_pol, Fd, fq, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cavity scatter");
  if (field) {
    e = launch_cav_gather(ca, q, Fd, field, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cavity gather");
  }
  return CAVDFTB_OK;
}

int cavdftb_set_surrogate(cavdftb_ctx* ctx, const float* params, const float* norm, double std_threshold) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  if (!params || !norm || !(std_threshold >= 0.0))
    return fail(ctx, CAVDFTB_EINVAL, "set_surrogate: need params, norm and a threshold >= 0");
  hipError_t e = hipMemcpyAsync(ctx->d_sg_params, params,
                                2 * (size_t)CAVDFTB_SG_MEMBERS * CAVDFTB_SG_N_PARAM * sizeof(float),
                                hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->d_sg_norm, norm, 2 * (size_t)CAVDFTB_SG_N_NORM * sizeof(float), hipMemcpyDeviceToDevice,
                       ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "set_surrogate copy");
  ctx->sg_thr = std_threshold;
  ctx->sg_ready = true;
  return CAVDFTB_OK;
}

int cavdftb_set_fallback(cavdftb_ctx* ctx, int32_t mode) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  if (mode != CAVDFTB_BORN_FD && mode != CAVDFTB_BORN_FIELD)
    return fail(ctx, CAVDFTB_EINVAL, "set_fallback: mode must be CAVDFTB_BORN_FD or CAVDFTB_BORN_FIELD");
  ctx->fallback_mode = mode;
  return CAVDFTB_OK;
}

int cavdftb_sg_features(cavdftb_ctx* ctx, const double* pos, double* feat, double* frames) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!pos || (!feat && !frames)) return fail(ctx, CAVDFTB_EINVAL, "sg_features: null pointer");
  hipError_t e = launch_sg_features(ctx->NA, ctx->d_atom_unit, ctx->d_unit_off, ctx->d_species, pos, feat, frames,
                                    ctx->stream);
  return e == hipSuccess ? CAVDFTB_OK : hip_fail(ctx, e, "sg_features");
}

int cavdftb_sg_prep(const double* v, const int32_t* idx, int32_t n, int32_t width, const float* norm, float* x,
                    void* hip_stream) {
  if (!v || !norm || !x || n < 0 || width <= 0) return CAVDFTB_EINVAL;
  return launch_sg_prep(n, width, idx, v, norm, x, (hipStream_t)hip_stream) == hipSuccess ? CAVDFTB_OK
                                                                                        : CAVDFTB_EHIP;
}

int cavdftb_sg_forward(const float* params, const float* x, int32_t n, float* y, float* act, void* hip_stream) {
  if (!params || !x || !y || n < 0) return CAVDFTB_EINVAL;
  return launch_sg_forward(params, x, n, y, act, (hipStream_t)hip_stream) == hipSuccess ? CAVDFTB_OK : CAVDFTB_EHIP;
}

int cavdftb_sg_backward(const float* params, const float* x, const float* act, const float* dy, int32_t n,
                        float* grad, float* work, void* hip_stream) {
  if (!params || !x || !act || !dy || !grad || !work || n <= 0) return CAVDFTB_EINVAL;
  return launch_sg_backward(params, x, act, dy, n, grad, work, (hipStream_t)hip_stream) == hipSuccess ? CAVDFTB_OK
                                                                                                    : CAVDFTB_EHIP;
}

// ---------------------------------------------------------------- allocation-free backward pass
// Per-tile partial gradients of cavdftb_sg_backward_noalloc: a file-scope
// device array (one copy per GPU).  Host code never passes the array's name
// to a kernel: its device address on the current device is looked up once per
// device with hipGetSymbolAddress and kept in g_noalloc_ptr.
constexpr int kNoallocTiles = (CAVDFTB_SG_NOALLOC_MAX_ROWS + 63) / 64;
static __device__ __align__(256) float scratch[(size_t)kNoallocTiles * CAVDFTB_SG_N_PARAM];
constexpr int kMaxDevices = 64;
static float* g_noalloc_ptr[kMaxDevices] = {};
static std::mutex g_noalloc_mu;

static hipError_t noalloc_scratch(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return hipSuccess;
}

int cavdftb_sg_backward_noalloc(const float* params, const float* x, const float* act, const float* dy, int32_t n,
                                float* grad, void* hip_stream) {
  if (!params || !x || !act || !dy || !grad || n <= 0 || n > CAVDFTB_SG_NOALLOC_MAX_ROWS) return CAVDFTB_EINVAL;
  float* work = nullptr;
  if (noalloc_scratch(&work) != hipSuccess) return CAVDFTB_EHIP;
  return launch_sg_backward(params, x, act, dy, n, grad, work, (hipStream_t)hip_stream) == hipSuccess ? CAVDFTB_OK
                                                                                                    : CAVDFTB_EHIP;
}

int cavdftb_sg_mse(const float* y, const float* t, int32_t count, float* dy, float* loss, float* work,
                   void* hip_stream) {
  if (!y || !t || !dy || !loss || !work || count <= 0) return CAVDFTB_EINVAL;
  return launch_sg_mse(y, t, count, dy, loss, work, (hipStream_t)hip_stream) == hipSuccess ? CAVDFTB_OK
                                                                                          : CAVDFTB_EHIP;
}

int cavdftb_sg_adam(float* params, const float* grad, float* m, float* v, int32_t count, float lr, float beta1,
                    float beta2, float eps, int32_t step, void* hip_stream) {
  if (!params || !grad || !m || !v || count <= 0 || step < 1) return CAVDFTB_EINVAL;
  return launch_sg_adam(params, grad, m, v, count, lr, beta1, beta2, eps, step, (hipStream_t)hip_stream) ==
                 hipSuccess
             ? CAVDFTB_OK
             : CAVDFTB_EHIP;
}

int cavdftb_sg_gather(const float* src, const int32_t* idx, int32_t n, int32_t width, float* dst, void* hip_stream) {
  if (!src || !idx || !dst || n < 0 || width <= 0) return CAVDFTB_EINVAL;
  return launch_sg_gather(src, idx, n, width, dst, (hipStream_t)hip_stream) == hipSuccess ? CAVDFTB_OK
                                                                                         : CAVDFTB_EHIP;
}

int cavdftb_sg_moments(const double* x, const int32_t* idx, int32_t n, int32_t width, float* out, void* hip_stream) {
  if (!x || !out || n <= 0 || width <= 0) return CAVDFTB_EINVAL;
  return launch_sg_moments(x, idx, n, width, out, (hipStream_t)hip_stream) == hipSuccess ? CAVDFTB_OK
                                                                                        : CAVDFTB_EHIP;
}

int cavdftb_sg_to_local(const double* frames, const double* born, const double* charges, const int32_t* idx,
                        int32_t n, double* out, void* hip_stream) {
  if (!frames || !born || !out || n < 0) return CAVDFTB_EINVAL;
  return launch_sg_to_local(n, idx, frames, born, charges, out, (hipStream_t)hip_stream) == hipSuccess
             ? CAVDFTB_OK
             : CAVDFTB_EHIP;
}

int cavdftb_init_photons(cavdftb_ctx* ctx, const double* r, double* qm, double* pm) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  if (!r || !qm || !pm) return fail(ctx, CAVDFTB_EINVAL, "init_photons: null pointer");
  int rc = eval_center(ctx, r, false);
  if (rc) return rc;
  ctx->primed = false;
  ctx->rs_primed = false;
  CavArgs ca = cav_args(ctx);
  hipError_t e = launch_mu_pol(ctx->d_dipole, ctx->pol, ctx->U, ctx->d_status, ctx->d_mu_pol, ctx->stream);
  if (e == hipSuccess) e = launch_cav_scatter(ca, ctx->d_mu_pol, ctx->d_F, nullptr, ctx->stream);
  if (e == hipSuccess) e = launch_init_photons(ca, ctx->d_F, qm, pm, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "init_photons");
  return CAVDFTB_OK;
}

int cavdftb_init_photons_thermal(cavdftb_ctx* ctx, const double* r, double* qm, double* pm, double kT,
                                 const double* xi) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!(kT >= 0.0) || !std::isfinite(kT) || (ctx->M > 0 && !xi))
    return fail(ctx, CAVDFTB_EINVAL, "init_photons_thermal: need finite kT >= 0 and xi");
  const int rc = cavdftb_init_photons(ctx, r, qm, pm);
  if (rc) return rc;
  const hipError_t e = launch_photon_thermal(cav_args(ctx), kT, xi, qm, pm, ctx->stream);
  return e == hipSuccess ? CAVDFTB_OK : hip_fail(ctx, e, "init_photons_thermal");
}

int cavdftb_invalidate(cavdftb_ctx* ctx) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  ctx->primed = false;
  ctx->rs_primed = false;
  return CAVDFTB_OK;
}

int cavdftb_step(cavdftb_ctx* ctx, double* r, double* p, double* qm, double* pm, int32_t n_steps, double dt,
                 int32_t born_mode, double h_fd, double* obs) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!r || !p || (ctx->M > 0 && (!qm || !pm)) || n_steps < 0 || !(dt > 0.0))
    return fail(ctx, CAVDFTB_EINVAL, "step: bad arguments");
  if (!born_mode_ok(born_mode)) return fail(ctx, CAVDFTB_EINVAL, "step: unknown born mode");
  if (born_mode != CAVDFTB_BORN_MULLIKEN && !(h_fd > 0.0)) return fail(ctx, CAVDFTB_EINVAL, "step: need h_fd > 0");
  if (born_mode == CAVDFTB_BORN_SURROGATE && !ctx->sg_ready)
    return fail(ctx, CAVDFTB_EINVAL, "step: no surrogate set (cavdftb_set_surrogate)");
  ctx->rs_primed = false;
  hipStream_t s = ctx->stream;
  CavArgs ca = cav_args(ctx);
  hipError_t e;
  int rc;
  if (!ctx->primed) {
    ctx->born_count = 0;
    rc = matter_stage(ctx, r, born_mode, h_fd);
    if (rc) return rc;
    e = launch_cav_scatter(ca, ctx->d_mu_pol, ctx->d_F, nullptr, s);
    if (e == hipSuccess) e = launch_cav_gather(ca, qm, ctx->d_F, ctx->d_field, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "step prime");
    ctx->primed = true;
  }
  if (obs) {
    e = launch_set_u32(ctx->d_obs_row, 0u, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "step obs row");
  }
  for (int st = 0; st < n_steps; ++st) {
    const bool periodic = ctx->born_every > 1 && exact_mode(born_mode);  // launches differ step to step
    rc = graph_steady(ctx) && !periodic ? replay_step(ctx, r, p, qm, pm, dt, born_mode, h_fd, obs)
                                        : issue_step(ctx, r, p, qm, pm, dt, born_mode, h_fd, obs);
    if (rc) return rc;
  }
  return CAVDFTB_OK;
}

int cavdftb_set_realspace_cavity(cavdftb_ctx* ctx, double eta, double omega0, double c_medium, double cell_a) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!(eta >= 0.0) || !(omega0 > 0.0) || !(c_medium > 0.0) || !(cell_a > 0.0))
    return fail(ctx, CAVDFTB_EINVAL, "set_realspace_cavity: need eta >= 0 and omega0, c, cell_a > 0");
  const int n = ctx->U;
  if ((n & (n - 1)) != 0 && n > CAVDFTB_RS_MAX_DIRECT)
    return fail(ctx, CAVDFTB_EINVAL, "set_realspace_cavity: n_units must be a power of two above 4096");
  std::vector<double> wk(n);
  for (int i = 0; i < n; ++i) {
    const int j = i <= n / 2 ? i : i - n;  // symmetric grid by DFT index
    const double k = 2.0 * M_PI * j / (n * cell_a);
    wk[i] = std::sqrt(omega0 * omega0 + c_medium * c_medium * k * k);
  }
  hipError_t e = hipMemcpyAsync(ctx->d_rs_wk, wk.data(), n * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "set_realspace_cavity copy");
  ctx->rs_eta = eta;
  ctx->rs_w0 = omega0;
  ctx->rs_ready = true;
  ctx->rs_primed = false;
  ctx->gen += 1;
  return CAVDFTB_OK;
}

int cavdftb_init_photons_realspace(cavdftb_ctx* ctx, const double* r, double* qn, double* pn) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!r || !qn || !pn) return fail(ctx, CAVDFTB_EINVAL, "init_photons_realspace: null pointer");
  if (!ctx->rs_ready) return fail(ctx, CAVDFTB_EINVAL, "init_photons_realspace: no real-space cavity set");
  ctx->gen += 1;
  int rc = eval_center(ctx, r, false);
  if (rc) return rc;
  ctx->primed = false;
  ctx->rs_primed = false;
  hipError_t e = launch_mu_pol(ctx->d_dipole, ctx->pol, ctx->U, ctx->d_status, ctx->d_mu_pol, ctx->stream);
  if (e == hipSuccess) e = launch_rs_init(ctx->U, ctx->d_mu_pol, ctx->rs_eta, ctx->rs_w0, qn, pn, ctx->stream);
  return e == hipSuccess ? CAVDFTB_OK : hip_fail(ctx, e, "init_photons_realspace");
}

int cavdftb_init_photons_realspace_thermal(cavdftb_ctx* ctx, const double* r, double* qn, double* pn, double kT,
                                           const double* xi) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!(kT >= 0.0) || !std::isfinite(kT) || !xi)
    return fail(ctx, CAVDFTB_EINVAL, "init_photons_realspace_thermal: need finite kT >= 0 and xi");
  const int rc = cavdftb_init_photons_realspace(ctx, r, qn, pn);
  if (rc) return rc;
  const hipError_t e = launch_rs_thermal(ctx->U, ctx->d_rs_wk, ctx->rs_w0, kT, xi, qn, pn, ctx->d_rs_buf0,
                                         ctx->d_rs_buf1, ctx->stream);
  return e == hipSuccess ? CAVDFTB_OK : hip_fail(ctx, e, "init_photons_realspace_thermal");
}

int cavdftb_step_realspace(cavdftb_ctx* ctx, double* r, double* p, double* qn, double* pn, int32_t n_steps,
                           double dt, int32_t born_mode, double h_fd, double* obs, double* qk_record) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (!r || !p || !qn || !pn || n_steps < 0 || !(dt > 0.0))
    return fail(ctx, CAVDFTB_EINVAL, "step_realspace: bad arguments");
  if (!ctx->rs_ready) return fail(ctx, CAVDFTB_EINVAL, "step_realspace: no real-space cavity set");
  if (!born_mode_ok(born_mode)) return fail(ctx, CAVDFTB_EINVAL, "step_realspace: unknown born mode");
  if (born_mode != CAVDFTB_BORN_MULLIKEN && !(h_fd > 0.0))
    return fail(ctx, CAVDFTB_EINVAL, "step_realspace: need h_fd > 0");
  if (born_mode == CAVDFTB_BORN_SURROGATE && !ctx->sg_ready)
    return fail(ctx, CAVDFTB_EINVAL, "step_realspace: no surrogate set (cavdftb_set_surrogate)");
  hipStream_t s = ctx->stream;
  const int n = ctx->U;
  const double eta = ctx->rs_eta, w0 = ctx->rs_w0;
  hipError_t e;
  int rc;
  ctx->gen += 1;  // the mode-space graph (if any) does not describe these launches
  ctx->primed = false;
  if (!ctx->rs_primed) {
    ctx->born_count = 0;
    rc = matter_stage(ctx, r, born_mode, h_fd);
    if (rc) return rc;
    ctx->rs_primed = true;
  }
  if (obs) {
    e = launch_set_u32(ctx->d_obs_row, 0u, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "step_realspace obs row");
  }
  for (int st = 0; st < n_steps; ++st) {
    // Step 1: local photon half-kick and nuclear velocity Verlet with q(t) held
    e = launch_rs_photon_kick(n, ctx->d_mu_pol, eta, dt, pn, s);
    if (e == hipSuccess) e = launch_rs_field(n, qn, ctx->d_mu_pol, eta, w0, ctx->d_field, s);
    if (e == hipSuccess)
      e = launch_kick_drift(ctx->NA, ctx->d_atom_unit, ctx->d_inv_mass, ctx->d_forces, ctx->d_zpol, ctx->d_field,
                            dt, r, p, 1, ctx->d_status, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "step_realspace kick/drift");
    rc = matter_stage(ctx, r, born_mode, h_fd);
    if (rc) return rc;
    e = launch_rs_field(n, qn, ctx->d_mu_pol, eta, w0, ctx->d_field, s);
    if (e == hipSuccess)
      e = launch_kick_drift(ctx->NA, ctx->d_atom_unit, ctx->d_inv_mass, ctx->d_forces, ctx->d_zpol, ctx->d_field,
                            dt, r, p, 0, ctx->d_status, s);
    if (e == hipSuccess) e = launch_rs_photon_kick(n, ctx->d_mu_pol, eta, dt, pn, s);
    // Steps 2-4: to k-space, exact rotation, back to real space
    if (e == hipSuccess)
      e = launch_rs_photon_step(n, ctx->d_rs_wk, w0, dt, qn, pn, ctx->d_rs_buf0, ctx->d_rs_buf1, ctx->d_rs_qk,
                                ctx->d_rs_pk, qk_record ? qk_record + (int64_t)st * n : nullptr, s);
    if (e == hipSuccess && obs)
      e = launch_rs_observables(ctx->U, ctx->d_unit_off, ctx->d_mass, p, ctx->d_energy, qn, ctx->d_mu_pol,
                                ctx->d_rs_qk, ctx->d_rs_pk, ctx->d_rs_wk, eta, w0, ctx->d_status, ctx->d_cjob_iters,
                                ctx->d_obs_part, ctx->obs_part_rows, obs, ctx->d_obs_row, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "step_realspace photons");
  }
  return CAVDFTB_OK;
}

int cavdftb_sync(cavdftb_ctx* ctx, int32_t* n_bad_units) {
  if (!ctx) return CAVDFTB_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "sync");
  if (n_bad_units) {
    std::vector<int32_t> st(ctx->U);
    e = hipMemcpy(st.data(), ctx->d_status, ctx->U * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "sync status");
    int32_t nb = 0;
    for (int32_t v : st) nb += v != 0;
    *n_bad_units = nb;
  }
  return CAVDFTB_OK;
}

int cavdftb_set_born_interval(cavdftb_ctx* ctx, int32_t every) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (every < 1) return fail(ctx, CAVDFTB_EINVAL, "set_born_interval: need every >= 1");
  ctx->gen += 1;
  ctx->born_every = every;
  return CAVDFTB_OK;
}

int cavdftb_set_graph(cavdftb_ctx* ctx, int32_t enable) {
  if (!ctx) return CAVDFTB_EINVAL;
  if (enable && !ctx->stream) return fail(ctx, CAVDFTB_EINVAL, "set_graph: the null stream cannot be captured");
  ctx->gen += 1;
  ctx->use_graph = enable != 0;
  if (!ctx->use_graph) {
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
  }
  return CAVDFTB_OK;
}

int cavdftb_enable_timing(cavdftb_ctx* ctx, int32_t enable) {
  if (!ctx) return CAVDFTB_EINVAL;
  ctx->gen += 1;
  ctx->timing = enable != 0;
  return CAVDFTB_OK;
}

int cavdftb_read_counters(cavdftb_ctx* ctx, cavdftb_counters* out) {
  if (!ctx || !out) return CAVDFTB_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "counters sync");
  harvest_events(ctx);
  unsigned long long h[4] = {0, 0, 0, 0};
  e = hipMemcpy(h, ctx->d_counters, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "counters copy");
  out->scc_jobs = (int64_t)h[0];
  out->scc_iterations = (int64_t)h[1];
  out->scc_flops = (double)h[2];
  out->scc_kernel_ms = ctx->t_ms;
  out->scc_launches = ctx->launches;
  out->jacobi_sweeps = (int64_t)h[3];
  unsigned long long h47[4] = {0, 0, 0, 0};
  e = hipMemcpy(h47, ctx->d_counters + 4, sizeof(h47), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "counters copy");
  out->surrogate_fallback_units = (int64_t)h47[0];
  out->jacobi_iterations = (int64_t)h47[1];
  out->tridiagonal_solves = (int64_t)h47[2];
  out->tridiagonal_fallbacks = (int64_t)h47[3];
  out->graph_replays = ctx->graph_replays;
  out->graph_captures = ctx->graph_captures;
  return CAVDFTB_OK;
}

int cavdftb_reset_counters(cavdftb_ctx* ctx) {
  if (!ctx) return CAVDFTB_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->d_counters, 0, 8 * sizeof(unsigned long long), ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "reset counters");
  harvest_events(ctx);
  ctx->t_ms = 0.0;
  ctx->launches = 0;
  ctx->graph_replays = 0;
  ctx->graph_captures = 0;
  return CAVDFTB_OK;
}

}  // extern "C"
