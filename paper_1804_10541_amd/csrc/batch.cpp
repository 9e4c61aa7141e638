// Batched registration of independent image pairs (include/mfr.h,
// mfr_batch_*): the multilevel Gauss-Newton / CG driver of Sec. 2.3 run for
// up to kMaxBatch pairs in lockstep, with one launch per phase for all pairs
// and the CG iterations captured into HIP graphs.  Each pair's arithmetic is
// exactly that of the single-pair path, so results agree bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx_internal.h"

using namespace mfr;

struct mfr_batch {
  int n = 0, levels = 0;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  std::vector<std::vector<Level>> lv;   // per pair, coarsest .. finest
  std::vector<size_t> base;             // per pair: offset of its region
  std::vector<size_t> ctx_bytes;        // per pair: context workspace (largest level)
  std::vector<size_t> off_ptab;         // per pair: prolongation tables
  size_t off_ctrl = 0;                  // counter, active flags, CG state, scalars
  int* counter = nullptr;
  int* active = nullptr;                // per pair: CG active flag (written by the CG kernels)
  int* mask = nullptr;                  // per pair: host-set mask for Gauss-Newton phases
  int* state = nullptr;                 // per pair: ST_COUNT ints
  double* sc = nullptr;                 // per pair: SC_COUNT doubles
  int groups = 0;                       // persistent work-groups of a voxel-tile launch (0: resident capacity)
  int cur = -1;                         // level the contexts are built for
  mfr_ctx* ctx[kMaxBatch] = {};
  bool images = false;
  hipGraphExec_t graph = nullptr;
  int graph_level = -1, graph_K = 0, graph_precond = -1;
  ~mfr_batch() {
    for (int k = 0; k < kMaxBatch; ++k) mfr_destroy(ctx[k]);
    if (graph) (void)hipGraphExecDestroy(graph);
  }
};

namespace {

constexpr int kGraphIters = 8;   // CG iterations per captured graph

mfr_status batch_layout(int n, const mfr_grid* grids, int levels, mfr_batch* b, size_t* total) {
  if (n < 1 || n > kMaxBatch) return fail(MFR_EINVAL, "batch size must be in 1..%d", kMaxBatch);
  if (!grids) return fail(MFR_EINVAL, "grids is NULL");
  b->n = n;
  b->levels = levels;
  b->lv.assign(n, {});
  b->base.assign(n, 0);
  b->ctx_bytes.assign(n, 0);
  b->off_ptab.assign(n, 0);
  size_t o = 0;
  for (int k = 0; k < n; ++k) {
    if (grids[k].distance != MFR_DIST_NGF)
      return fail(MFR_EINVAL, "pair %d: the batched path evaluates the NGF distance only", k);
    if (grids[k].regulariser != MFR_REG_CURVATURE)
      return fail(MFR_EINVAL, "pair %d: the batched path evaluates the curvature regulariser only", k);
    if (grids[k].m[2] == 1 && grids[k].my[2] == 1)
      return fail(MFR_EINVAL, "pair %d: the batched path takes three-dimensional problems only", k);
    size_t per = 0;
    MFR_TRY(ml_levels(&grids[k], levels, &b->lv[k], &per));
    size_t cb = 0;
    for (int l = 0; l < levels; ++l) {
      size_t x = 0;
      MFR_TRY(mfr_workspace_size(&b->lv[k][l].grid, &x));
      cb = std::max(cb, x);
    }
    b->ctx_bytes[k] = cb;
    b->base[k] = o;
    const Geo& gf = b->lv[k][levels - 1].geo;
    b->off_ptab[k] = align_up(b->lv[k][levels - 1].off_u + sizeof(float) * 3 * gf.nbar);
    o = align_up(o + per);
  }
  b->off_ctrl = o;
  o = align_up(o + sizeof(int) * (1 + 2 * kMaxBatch + ST_COUNT * kMaxBatch));
  o = align_up(o + sizeof(double) * SC_COUNT * kMaxBatch);
  *total = o;
  return MFR_OK;
}

template <class T>
T* at_pair(mfr_batch* b, int k, size_t off) {
  return reinterpret_cast<T*>(b->ws + b->base[k] + off);
}

float* level_u(mfr_batch* b, int k, int l) { return at_pair<float>(b, k, b->lv[k][l].off_u); }

// (Re)creates the per-pair contexts of level l over their workspace regions.
mfr_status enter_level(mfr_batch* b, int l) {
  if (b->cur == l) return MFR_OK;
  for (int k = 0; k < b->n; ++k) {
    mfr_destroy(b->ctx[k]);
    b->ctx[k] = nullptr;
  }
  b->cur = -1;
  TileShape shape{0, 0};
  for (int k = 0; k < b->n; ++k) {
    MFR_TRY(mfr_create(&b->lv[k][l].grid, b->st, b->ws + b->base[k], b->ctx_bytes[k], &b->ctx[k]));
    MFR_TRY(mfr_set_images(b->ctx[k], at_pair<float>(b, k, b->lv[k][l].off_R),
                           at_pair<float>(b, k, b->lv[k][l].off_T)));
    if (k == 0) shape = b->ctx[k]->tiling.shape;
    if (b->ctx[k]->tiling.shape.bx != shape.bx || b->ctx[k]->tiling.shape.by != shape.by)
      return fail(MFR_EINVAL, "all pairs of a batch must use one tile shape");
  }
  b->cur = l;
  return MFR_OK;
}

// Small device-to-host read after the batch stream has drained (a blocking copy
// into pageable host memory).
mfr_status read_back(mfr_batch* b, void* dst, const void* src, size_t bytes) {
  HIP_TRY(hipStreamSynchronize(b->st));
  HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return MFR_OK;
}

// Fills the persistent work list of a voxel-tile launch.
BatchJobs tile_jobs(mfr_batch* b, const float* const* u, const float* const* p, const int* active) {
  BatchJobs J{};
  J.n = b->n;
  J.prefix[0] = 0;
  for (int k = 0; k < b->n; ++k) {
    J.jobs[k].t = b->ctx[k]->tp;
    J.jobs[k].u = u[k];
    J.jobs[k].p = p ? p[k] : nullptr;
    J.prefix[k + 1] = J.prefix[k] + b->ctx[k]->tiling.grid();
  }
  J.total = J.prefix[b->n];
  J.counter = b->counter;
  J.active = active;
  return J;
}

NodeJobs node_jobs(mfr_batch* b, float s_ngf_scale, const float* const* f, float* const* out, const int* active) {
  NodeJobs J{};
  J.n = b->n;
  J.prefix[0] = 0;
  for (int k = 0; k < b->n; ++k) {
    mfr_ctx* c = b->ctx[k];
    J.jobs[k].q = c->np;
    J.jobs[k].q.s_ngf = (float)(s_ngf_scale * c->geo.hbar());
    J.jobs[k].f = f[k];
    J.jobs[k].out = out ? out[k] : nullptr;
    J.prefix[k + 1] = J.prefix[k] + node_blocks(c);
  }
  J.active = active;
  return J;
}

mfr_status launch_tiles(mfr_batch* b, int mode, const BatchJobs& J) {
  HIP_TRY(launch_zero_ints(b->counter, 1, b->st));   // a kernel, not a memset: capturable
  HIP_TRY(launch_tile_batch(b->ctx[0]->tiling.shape, mode, J, b->groups, b->st));
  return MFR_OK;
}

// Sums the voxel-tile partials of every masked pair into its slot SC_D.
mfr_status sum_tile_parts(mfr_batch* b, const int* mask) {
  SumJobs D{};
  D.n = b->n;
  D.active = mask;
  for (int k = 0; k < b->n; ++k) {
    mfr_ctx* c = b->ctx[k];
    D.jobs[k] = SumJob{c->red_tile, c->tiling.grid(), 1, c->sc + SC_D};
  }
  HIP_TRY(launch_sum_batch(D, b->st));
  return MFR_OK;
}

// Sums the node-pass partials of every masked pair into its slot SC_S: one per
// node group after the regulariser pass (objective), one per group and
// component after the gradient pass.
mfr_status sum_node_parts(mfr_batch* b, const int* mask, bool per_component) {
  SumJobs S{};
  S.n = b->n;
  S.active = mask;
  for (int k = 0; k < b->n; ++k) {
    mfr_ctx* c = b->ctx[k];
    S.jobs[k] = SumJob{c->red_node, per_component ? node_parts(c) : node_blocks(c), 1, c->sc + SC_S};
  }
  HIP_TRY(launch_sum_batch(S, b->st));
  return MFR_OK;
}

// J of every masked pair from its context's scalars (synchronises); a
// non-finite value is an error only where `strict` is set.
mfr_status read_J(mfr_batch* b, const int* mask, bool strict, double* J) {
  HIP_TRY(hipStreamSynchronize(b->st));
  for (int k = 0; k < b->n; ++k) {
    if (!mask[k]) continue;
    mfr_ctx* c = b->ctx[k];
    double h[SC_COUNT];
    HIP_TRY(hipMemcpy(h, c->sc, sizeof(h), hipMemcpyDeviceToHost));
    const double Dv = c->geo.hbar() * h[SC_D];
    const double Sv = c->geo.hybar() * h[SC_S];
    J[k] = Dv + c->geo.alpha * Sv;
    if (strict && !std::isfinite(J[k]))
      return fail(MFR_ENONFINITE, "objective of pair %d is not finite (D = %g, S = %g)", k, Dv, Sv);
  }
  return MFR_OK;
}

// Objective of every masked pair at u (voxel tiles, node pass S, sums).
mfr_status batch_objective(mfr_batch* b, const float* const* u, const int* mask) {
  BatchJobs J = tile_jobs(b, u, nullptr, mask);
  MFR_TRY(launch_tiles(b, MODE_OBJ, J));
  MFR_TRY(sum_tile_parts(b, mask));
  NodeJobs N = node_jobs(b, 0.0f, u, nullptr, mask);
  HIP_TRY(launch_node_pass_batch(NP_S, N, b->st));
  return sum_node_parts(b, mask, false);
}

// Gradient of every masked pair into out[k]; the objective parts in the scalars.
mfr_status batch_gradient(mfr_batch* b, const float* const* u, float* const* out, const int* mask) {
  BatchJobs J = tile_jobs(b, u, nullptr, mask);
  MFR_TRY(launch_tiles(b, MODE_GRAD, J));
  MFR_TRY(sum_tile_parts(b, mask));
  NodeJobs N = node_jobs(b, -2.0f, u, out, mask);
  HIP_TRY(launch_node_pass_batch(NP_GRAD, N, b->st));
  return sum_node_parts(b, mask, true);
}

// q_k = A_k p_k for CG-active pairs; p.q partials in each context's red_node.
mfr_status batch_hv(mfr_batch* b, const float* const* u, const float* const* p, float* const* q, const int* active) {
  BatchJobs J = tile_jobs(b, u, p, active);
  MFR_TRY(launch_tiles(b, MODE_HV, J));
  NodeJobs N = node_jobs(b, 2.0f, p, q, active);
  HIP_TRY(launch_node_pass_batch(NP_HV, N, b->st));
  return MFR_OK;
}

VecJobs vec_jobs(mfr_batch* b, const int* max_iter, double rtol, bool precond) {
  VecJobs V{};
  V.n = b->n;
  V.prefix[0] = 0;
  for (int k = 0; k < b->n; ++k) {
    mfr_ctx* c = b->ctx[k];
    VecJob& v = V.jobs[k];
    v.r = c->vec[0];
    v.z = c->vec[1];
    v.p = c->vec[2];
    v.q = c->vec[3];
    v.s = c->vec[7];
    v.b = c->vec[5];
    v.diag = precond ? c->vec[4] : nullptr;
    v.sc = b->sc + SC_COUNT * k;
    v.state = b->state + ST_COUNT * k;
    v.red = c->red_node;
    v.red_pq = c->red_node;
    v.n_pq = node_parts(c);
    v.n3 = (int)(3 * c->geo.nbar);
    v.max_iter = max_iter[k];
    v.rtol = rtol;
    V.prefix[k + 1] = V.prefix[k] + c->vec_blocks;
  }
  V.active_out = b->active;
  return V;
}

// One CG iteration for all pairs (launches only: capturable).
mfr_status cg_iteration(mfr_batch* b, const VecJobs& V, const float* const* u) {
  const float* p[kMaxBatch];
  float* q[kMaxBatch];
  for (int k = 0; k < b->n; ++k) {
    p[k] = V.jobs[k].p;
    q[k] = V.jobs[k].q;
  }
  MFR_TRY(batch_hv(b, u, p, q, b->active));
  HIP_TRY(launch_pcg_alpha_batch(V, b->st));
  HIP_TRY(launch_pcg_update_batch(V, b->st));
  HIP_TRY(launch_pcg_beta_batch(V, b->st));
  HIP_TRY(launch_pcg_direction_batch(V, b->st));
  return MFR_OK;
}

// Solves A_k s_k = b_k (b_k in vec[5], s_k in vec[7]) for the pairs with
// live[k] set; the others start inactive (iteration limit 0).
mfr_status batch_pcg(mfr_batch* b, const float* const* u, const mfr_ml_opts* o, const int* live, bool use_graph,
                     int* iters, int* replays) {
  int maxit[kMaxBatch];
  for (int k = 0; k < b->n; ++k) maxit[k] = live[k] ? o->pcg_max : 0;
  const bool pre = o->precond == 1;
  if (pre)
    for (int k = 0; k < b->n; ++k)
      if (live[k]) HIP_TRY(enqueue_pcg_diag(b->ctx[k], u[k], b->ctx[k]->vec[4]));
  VecJobs V = vec_jobs(b, maxit, o->pcg_rtol, pre);
  HIP_TRY(launch_pcg_init_batch(V, b->st));
  if (use_graph && (!b->graph || b->graph_level != b->cur || b->graph_precond != (int)pre)) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_level = -1;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    mfr_status s = MFR_OK;
    for (int it = 0; it < kGraphIters && s == MFR_OK; ++it) s = cg_iteration(b, V, u);
    hipError_t e = hipStreamEndCapture(b->st, &g);
    if (s != MFR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    HIP_TRY(e);
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(e);
    b->graph_level = b->cur;
    b->graph_precond = (int)pre;
    b->graph_K = kGraphIters;
  }
  int done = 0;
  int act[kMaxBatch];
  while (done < o->pcg_max) {
    if (use_graph) {
      HIP_TRY(hipGraphLaunch(b->graph, b->st));
      done += b->graph_K;
      ++*replays;
    } else {
      MFR_TRY(cg_iteration(b, V, u));
      done += 1;
    }
    MFR_TRY(read_back(b, act, b->active, sizeof(int) * b->n));
    bool any = false;
    for (int k = 0; k < b->n; ++k) any = any || act[k] != 0;
    if (!any) break;
  }
  int stt[ST_COUNT * kMaxBatch];
  MFR_TRY(read_back(b, stt, b->state, sizeof(int) * ST_COUNT * b->n));
  for (int k = 0; k < b->n; ++k) iters[k] = stt[ST_COUNT * k + ST_ITERS];
  return MFR_OK;
}

mfr_status set_mask(mfr_batch* b, const int* m) {
  HIP_TRY(hipMemcpyAsync(b->mask, m, sizeof(int) * b->n, hipMemcpyHostToDevice, b->st));
  HIP_TRY(hipStreamSynchronize(b->st));   // the host array may change right after
  return MFR_OK;
}

}  // namespace

extern "C" {

mfr_status mfr_batch_workspace_size(int32_t n, const mfr_grid* grids, int32_t levels, size_t* bytes) {
  if (!bytes) return fail(MFR_EINVAL, "bytes is NULL");
  mfr_batch tmp;
  return batch_layout(n, grids, levels, &tmp, bytes);
}

mfr_status mfr_batch_create(int32_t n, const mfr_grid* grids, int32_t levels, void* hip_stream, void* workspace,
                            size_t ws_bytes, mfr_batch** out) {
  if (!out) return fail(MFR_EINVAL, "out is NULL");
  *out = nullptr;
  mfr_batch* b = new (std::nothrow) mfr_batch();
  if (!b) return fail(MFR_EINVAL, "host allocation failed");
  size_t need = 0;
  mfr_status s = batch_layout(n, grids, levels, b, &need);
  if (s == MFR_OK && (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0))
    s = fail(MFR_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (s == MFR_OK && ws_bytes < need)
    s = fail(MFR_ENOMEM, "workspace of %zu bytes is smaller than the required %zu", ws_bytes, need);
  if (s != MFR_OK) {
    delete b;
    return s;
  }
  b->st = reinterpret_cast<hipStream_t>(hip_stream);
  b->ws = reinterpret_cast<char*>(workspace);
  int* ip = reinterpret_cast<int*>(b->ws + b->off_ctrl);
  b->counter = ip;
  b->active = ip + 1;
  b->mask = ip + 1 + kMaxBatch;
  b->state = ip + 1 + 2 * kMaxBatch;
  b->sc = reinterpret_cast<double*>(b->ws + align_up(b->off_ctrl + sizeof(int) * (1 + 2 * kMaxBatch + ST_COUNT * kMaxBatch)));
  b->groups = 0;   // persistent launches: as many work-groups as are resident at once
  *out = b;
  return MFR_OK;
}

void mfr_batch_destroy(mfr_batch* b) { delete b; }

mfr_status mfr_batch_set_images(mfr_batch* b, const float* const* R, const float* const* T) {
  if (!b) return fail(MFR_EINVAL, "batch is NULL");
  if (!R || !T) return fail(MFR_EINVAL, "image arrays are NULL");
  const int nl = b->levels;
  for (int k = 0; k < b->n; ++k) {
    MFR_TRY(check_ptr(R[k], "R[k]"));
    MFR_TRY(check_ptr(T[k], "T[k]"));
    auto& L = b->lv[k];
    const Geo& gf = L[nl - 1].geo;
    HIP_TRY(hipMemcpyAsync(at_pair<float>(b, k, L[nl - 1].off_R), R[k], sizeof(float) * gf.mbar,
                           hipMemcpyDeviceToDevice, b->st));
    HIP_TRY(hipMemcpyAsync(at_pair<float>(b, k, L[nl - 1].off_T), T[k],
                           sizeof(float) * (size_t)gf.mT[0] * gf.mT[1] * gf.mT[2], hipMemcpyDeviceToDevice, b->st));
    for (int l = nl - 2; l >= 0; --l) {
      const Geo& f = L[l + 1].geo;
      HIP_TRY(launch_restrict(at_pair<float>(b, k, L[l + 1].off_R), f.m[0], f.m[1], f.m[2],
                              at_pair<float>(b, k, L[l].off_R), b->st));
      HIP_TRY(launch_restrict(at_pair<float>(b, k, L[l + 1].off_T), f.mT[0], f.mT[1], f.mT[2],
                              at_pair<float>(b, k, L[l].off_T), b->st));
    }
  }
  b->cur = -1;   // contexts bind images when a level is entered
  b->graph_level = -1;
  b->images = true;
  return MFR_OK;
}

mfr_status mfr_batch_hess_vec(mfr_batch* b, const float* const* u, const float* const* p, float* const* q) {
  if (!b || !b->images) return fail(MFR_EINVAL, "batch is NULL or has no images");
  if (!u || !p || !q) return fail(MFR_EINVAL, "vector arrays are NULL");
  for (int k = 0; k < b->n; ++k) {
    MFR_TRY(check_ptr(u[k], "u[k]"));
    MFR_TRY(check_ptr(p[k], "p[k]"));
    MFR_TRY(check_ptr(q[k], "q[k]"));
    if (q[k] == u[k] || q[k] == p[k]) return fail(MFR_EINVAL, "q must not alias u or p");
  }
  MFR_TRY(enter_level(b, b->levels - 1));
  return batch_hv(b, u, p, q, nullptr);
}

mfr_status mfr_batch_register(mfr_batch* b, const mfr_ml_opts* o, int32_t use_graph, float* const* u,
                              mfr_batch_report* report) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!b || !b->images) return fail(MFR_EINVAL, "batch is NULL or has no images");
  if (!o) return fail(MFR_EINVAL, "opts is NULL");
  if (o->levels != b->levels) return fail(MFR_EINVAL, "opts->levels differs from the batch's levels");
  if (o->gn_iters < 0 || o->pcg_max < 0 || !(o->pcg_rtol >= 0) || !(o->armijo_c1 >= 0 && o->armijo_c1 < 1) ||
      o->armijo_max < 1 || o->precond < 0 || o->precond > 1)
    return fail(MFR_EINVAL, "invalid multilevel options");
  if (!u) return fail(MFR_EINVAL, "u is NULL");
  if (o->u_init) return fail(MFR_EINVAL, "the batched path starts every pair at u = 0 (opts->u_init must be NULL)");
  if (use_graph && !b->st) return fail(MFR_EINVAL, "graph replay needs a stream other than the null stream");
  for (int k = 0; k < b->n; ++k) MFR_TRY(check_ptr(u[k], "u[k]"));
  const int n = b->n, nl = b->levels;
  mfr_batch_report rep{};
  double Jcur[kMaxBatch] = {};
  int live[kMaxBatch];   // pair still iterating on this level

  for (int l = 0; l < nl; ++l) {
    // initial displacement of the level
    for (int k = 0; k < n; ++k) {
      const Geo& g = b->lv[k][l].geo;
      float* ul = level_u(b, k, l);
      if (l == 0) {
        if (nl == 1)
          HIP_TRY(hipMemcpyAsync(ul, u[k], sizeof(float) * 3 * g.nbar, hipMemcpyDeviceToDevice, b->st));
        else
          HIP_TRY(hipMemsetAsync(ul, 0, sizeof(float) * 3 * g.nbar, b->st));
      } else {
        const Geo& gc = b->lv[k][l - 1].geo;
        auto px = prolong_table(g.n[0], g.hy[0], gc.n[0], gc.hy[0]);
        auto py = prolong_table(g.n[1], g.hy[1], gc.n[1], gc.hy[1]);
        auto pz = prolong_table(g.n[2], g.hy[2], gc.n[2], gc.hy[2]);
        Conv1* dt = at_pair<Conv1>(b, k, b->off_ptab[k]);
        HIP_TRY(hipMemcpyAsync(dt, px.data(), sizeof(Conv1) * px.size(), hipMemcpyHostToDevice, b->st));
        HIP_TRY(hipMemcpyAsync(dt + g.n[0], py.data(), sizeof(Conv1) * py.size(), hipMemcpyHostToDevice, b->st));
        HIP_TRY(hipMemcpyAsync(dt + g.n[0] + g.n[1], pz.data(), sizeof(Conv1) * pz.size(), hipMemcpyHostToDevice,
                               b->st));
        HIP_TRY(launch_prolong(level_u(b, k, l - 1), gc.n[0], gc.n[1], gc.n[2], ul, g.n[0], g.n[1], g.n[2], dt,
                               dt + g.n[0], dt + g.n[0] + g.n[1], 3, b->st));
        HIP_TRY(hipStreamSynchronize(b->st));
      }
    }
    MFR_TRY(enter_level(b, l));
    const float* ucp[kMaxBatch];
    float* up[kMaxBatch];
    float* grad[kMaxBatch];
    float* trial[kMaxBatch];
    const float* ctrial[kMaxBatch];
    for (int k = 0; k < n; ++k) {
      up[k] = level_u(b, k, l);
      ucp[k] = up[k];
      grad[k] = b->ctx[k]->vec[5];
      trial[k] = b->ctx[k]->vec[6];
      ctrial[k] = trial[k];
      live[k] = 1;
    }
    MFR_TRY(set_mask(b, live));
    MFR_TRY(batch_objective(b, ucp, b->mask));
    MFR_TRY(read_J(b, live, true, Jcur));
    for (int it = 0; it < o->gn_iters; ++it) {
      bool any = false;
      for (int k = 0; k < n; ++k) any = any || live[k];
      if (!any) break;
      // gradient and J (b = -grad J in vec[5])
      MFR_TRY(set_mask(b, live));
      MFR_TRY(batch_gradient(b, ucp, grad, b->mask));
      double Jv[kMaxBatch];
      MFR_TRY(read_J(b, live, true, Jv));
      AxpyJobs neg{};
      neg.n = n;
      neg.prefix[0] = 0;
      for (int k = 0; k < n; ++k) {
        neg.jobs[k] = AxpyJob{grad[k], grad[k], grad[k], -2.0f, (int)(3 * b->ctx[k]->geo.nbar)};
        neg.prefix[k + 1] = neg.prefix[k] + std::min((neg.jobs[k].n + 255) / 256, 4096);
      }
      neg.active = b->mask;
      HIP_TRY(launch_axpy_batch(neg, b->st));
      // CG (only live pairs start: dead pairs get max_iter 0)
      int iters[kMaxBatch];
      MFR_TRY(batch_pcg(b, ucp, o, live, use_graph != 0, iters, &rep.graph_launches));
      // slope = -(b . s)
      VecJobs D{};
      D.n = n;
      D.prefix[0] = 0;
      SumJobs S{};
      S.n = n;
      for (int k = 0; k < n; ++k) {
        mfr_ctx* c = b->ctx[k];
        D.jobs[k].r = c->vec[5];
        D.jobs[k].z = c->vec[7];
        D.jobs[k].red = c->red_node;
        D.jobs[k].n3 = (int)(3 * c->geo.nbar);
        D.prefix[k + 1] = D.prefix[k] + c->vec_blocks;
        S.jobs[k] = SumJob{c->red_node, c->vec_blocks, 1, c->sc + SC_DOT};
      }
      HIP_TRY(launch_dot_batch(D, b->st));
      HIP_TRY(launch_sum_batch(S, b->st));
      HIP_TRY(hipStreamSynchronize(b->st));
      double slope[kMaxBatch];
      for (int k = 0; k < n; ++k) {
        double h[SC_COUNT];
        HIP_TRY(hipMemcpy(h, b->ctx[k]->sc, sizeof(h), hipMemcpyDeviceToHost));
        slope[k] = -h[SC_DOT];
        if (live[k]) rep.pcg_total[k] += iters[k];
      }
      // Armijo line search, all searching pairs per trial
      double eta[kMaxBatch];
      int searching[kMaxBatch], accepted[kMaxBatch];
      for (int k = 0; k < n; ++k) {
        eta[k] = 1.0;
        searching[k] = live[k];
        accepted[k] = 0;
      }
      for (int ls = 0; ls < o->armijo_max; ++ls) {
        bool anys = false;
        for (int k = 0; k < n; ++k) anys = anys || searching[k];
        if (!anys) break;
        MFR_TRY(set_mask(b, searching));
        AxpyJobs tr{};
        tr.n = n;
        tr.prefix[0] = 0;
        for (int k = 0; k < n; ++k) {
          tr.jobs[k] = AxpyJob{up[k], b->ctx[k]->vec[7], trial[k], (float)eta[k], (int)(3 * b->ctx[k]->geo.nbar)};
          tr.prefix[k + 1] = tr.prefix[k] + std::min((tr.jobs[k].n + 255) / 256, 4096);
        }
        tr.active = b->mask;
        HIP_TRY(launch_axpy_batch(tr, b->st));
        MFR_TRY(batch_objective(b, ctrial, b->mask));
        double Jn[kMaxBatch];
        MFR_TRY(read_J(b, searching, false, Jn));
        for (int k = 0; k < n; ++k) {
          if (!searching[k]) continue;
          if (std::isfinite(Jn[k]) && Jn[k] <= Jv[k] + o->armijo_c1 * eta[k] * slope[k]) {
            accepted[k] = 1;
            searching[k] = 0;
            Jcur[k] = Jn[k];
          } else {
            eta[k] *= 0.5;
          }
        }
      }
      for (int k = 0; k < n; ++k) {
        if (!live[k]) continue;
        if (accepted[k]) {
          HIP_TRY(hipMemcpyAsync(up[k], trial[k], sizeof(float) * 3 * b->ctx[k]->geo.nbar, hipMemcpyDeviceToDevice,
                                 b->st));
          rep.gn_done[k] += 1;
        } else {
          live[k] = 0;   // this pair's level ends; J stays at the last accepted point
          rep.status[k] = MFR_ELINESEARCH;
        }
      }
    }
  }
  for (int k = 0; k < n; ++k) {
    HIP_TRY(hipMemcpyAsync(u[k], level_u(b, k, nl - 1), sizeof(float) * 3 * b->lv[k][nl - 1].geo.nbar,
                           hipMemcpyDeviceToDevice, b->st));
    rep.J_final[k] = Jcur[k];
  }
  HIP_TRY(hipStreamSynchronize(b->st));
  rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (report) *report = rep;
  return MFR_OK;
}

}  // extern "C"
