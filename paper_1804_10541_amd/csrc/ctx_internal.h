// Host-side internals of libmfr shared by the single-problem API (api.cpp)
// and the batched path (batch.cpp): validated geometry, tiling, workspace
// layout, the context structure and the enqueue helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <utility>
#include <vector>

#include "../../include/mfr.h"
#include "mfr_internal.h"

namespace mfr {

mfr_status fail(mfr_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(MFR_EHIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

#define MFR_TRY(expr)                \
  do {                               \
    mfr_status s_ = (expr);          \
    if (s_ != MFR_OK) return s_;     \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Derived, validated problem description.
// A two-dimensional problem (dim 2) has m[2] = n[2] = mT[2] = 1 and
// h[2] = hT[2] = hy[2] = 1, so the products below are the 2D cell areas; its
// node vectors have two components.
struct Geo {
  int dim;   // 3, or 2 for a two-dimensional problem (m[2] = my[2] = 1 in the mfr_grid)
  int nc() const { return dim; }   // components of a node vector
  int m[3], n[3], mT[3];
  double h[3], hT[3], hy[3];
  double tau, rho, alpha;
  int dist;   // MFR_DIST_NGF or MFR_DIST_SSD
  int reg;    // MFR_REG_CURVATURE, MFR_REG_DIFFUSIVE or MFR_REG_ELASTIC
  double lame_mu, lame_lambda;   // elastic only
  size_t mbar, nbar;
  double hbar() const { return h[0] * h[1] * h[2]; }
  double hybar() const { return hy[0] * hy[1] * hy[2]; }
  // Scales of the gathered voxel contributions P^T(...) in the gradient and in
  // the Gauss-Newton product.  NGF, psi = hbar sum (1 - r^2): grad = -2 hbar J^T r,
  // H = 2 hbar J^T J (eq. dPsi, eq. NGF_discretized_hessian).  SSD,
  // psi = hbar/2 r^T r: grad = hbar J^T r, H = hbar J^T J.
  double grad_scale() const { return dist == MFR_DIST_SSD ? hbar() : -2.0 * hbar(); }
  double hess_scale() const { return dist == MFR_DIST_SSD ? hbar() : 2.0 * hbar(); }
  // Regulariser: curvature S = hbar^y sum (L u)^2, grad = 2 alpha hbar^y L^T L u;
  // diffusive S = hbar^y/2 sum of squared edge differences (= -hbar^y/2 u.L u),
  // grad = -alpha hbar^y L u.  reg_scale() is the factor of the node pass's
  // stencil term, s_value() the one of its sum.
  // Elastic: both scaled by lame_mu, the divergence part carries kappa() inside the kernels.
  double reg_scale() const {
    return reg == MFR_REG_CURVATURE ? 2.0 * alpha * hybar() : alpha * hybar() * (reg == MFR_REG_ELASTIC ? lame_mu : 1.0);
  }
  double s_mul() const { return reg == MFR_REG_CURVATURE ? hybar() : 0.5 * hybar(); }
  double s_k() const { return reg == MFR_REG_ELASTIC ? lame_mu : 1.0; }
  double s_value(double sum) const { return s_mul() * sum * s_k(); }
  double kappa() const { return reg == MFR_REG_ELASTIC ? (lame_lambda + lame_mu) / lame_mu : 0.0; }
};

mfr_status make_geo(const mfr_grid* g, Geo* o);
std::vector<Conv1> conv_table(int m, int n);
std::vector<Samp1> samp_table(int m, double h, double hT);
std::vector<Range1> node_cols(const std::vector<Conv1>& c, int n);
std::vector<Conv1> prolong_table(int nf, double hyf, int nc, double hyc);

// Tiling of the voxel-tiled Jacobi diagonal (kDiagBX x kDiagBY groups, its own
// chunks); `on` when the node grid fits its per-group tables (at most one node
// per voxel along each axis, at most half a group's threads of node columns).
struct DiagTiling {
  bool on;
  int tiles_x, tiles_y, chunks, chunk_len;
  int nxt, nyt, nzt;
  int grid() const { return tiles_x * tiles_y * chunks; }
};

struct Tiling {
  TileShape shape;
  int tiles_x, tiles_y, chunks, chunk_len;
  int nxt, nyt, nzt;
  int smx, smy, smz;   // partial slots per axis: the most groups overlapping one node along it
  DiagTiling dg;
  int grid() const { return tiles_x * tiles_y * chunks; }
};

Tiling make_tiling(const Geo& g, const std::vector<Conv1>& cx, const std::vector<Conv1>& cy,
                   const std::vector<Conv1>& cz);
bool valid_shape(const TileShape& s);
mfr_tile_config current_tile_config();
void set_tile_config(const mfr_tile_config& c);

struct Layout {
  size_t Tp, cx, cy, cz, sx, sy, sz, ntx, nty, ntz, orgx, orgy, orgz, rx, ry, rz;
  size_t part, red_tile, red_node, sc, vec, jbx, jby, jbz, lap, ctrl, div;
  size_t dntx, dnty, dntz, dorgx, dorgy, dorgz, dpart;   // voxel-tiled diagonal
  size_t n_red_node;
  size_t total;
};

Layout make_layout(const Geo& g, const Tiling& t);

template <class T>
T* at(char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

struct Level {
  mfr_grid grid;
  Geo geo;
  size_t off_R, off_T, off_u;   // coarse images / displacement (finest: caller buffers)
};

mfr_status ml_levels(const mfr_grid* finest, int levels, std::vector<Level>* out, size_t* total);

}  // namespace mfr

// The opaque context of include/mfr.h.
struct mfr_ctx {
  mfr::Geo geo;
  mfr::Tiling tiling;
  mfr::Layout lay;
  hipStream_t stream;
  char* ws;
  const float* R;
  bool have_images;
  mfr::TileParams tp;
  mfr::NodeParams np;
  mfr::DiagParams dp;
  mfr::JacParams jp;
  mfr::DiagTileParams dtp;
  bool jac_tiled;
  double* sc;
  double* red_tile;
  double* red_node;
  float* vec[8];
  int vec_blocks;
  int* ctrl;                     // device-steered CG: [0] active flag, [1..] PcgState
  mfr_pc* pc = nullptr;          // learned preconditioner used by precond = 2
  std::vector<mfr_pc*> bound_pcs;   // preconditioners bound to this context (unbound when it is destroyed)
  unsigned image_version = 0;    // bumped by mfr_set_images
  // host copies of the L-BFGS initial-matrix tables (cosine matrices, their
  // transposes, eigenvalues); kept here so uploads need no synchronisation
  std::vector<float> h0_C[3], h0_Ct[3], h0_lam;
  // kernel timing (mfr_profile_*)
  bool prof_on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  int prof_launches[6] = {0, 0, 0, 0, 0, 0};
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  ~mfr_ctx() {
    for (auto& p : prof_pending) {
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    for (auto e : prof_pool) (void)hipEventDestroy(e);
  }
};

namespace mfr {

mfr_status ctx_init(mfr_ctx* c, const mfr_grid* grid, void* stream, void* ws, size_t ws_bytes);
// Runs `launch` between two event records when timing is on (slot: kernel id).
// out = {J, D, S} (count 3) or {J} (count 1) from the sums at sums[0] (distance)
// and sums[1] (regulariser): D = dmul sums[0], S = (smul sums[1]) sk, J = D + alpha S,
// rounded as Geo::s_value and the host evaluate them (node_kernels.hip)
hipError_t launch_objective_out(const double* sums, double dmul, double smul, double sk, double alpha, double* out,
                                int count, hipStream_t st);
// out = {iterations, relative residual, flag} of a device-steered solve, from its
// state array and scalars (batch_kernels.hip)
hipError_t launch_pcg_info_out(const int* state, const double* sc, double* out, hipStream_t st);
// The line search of the capturable Gauss-Newton step (node_kernels.hip):
// info = {J_before, J_after, eta, slope, pcg iterations, pcg relative residual,
// pcg flag, accepted, trials}; *search is 1 until a step length is accepted.
hipError_t launch_ls_begin(const double* sums, double dmul, double smul, double sk, double alpha, int* search,
                           double* info, hipStream_t st);
hipError_t launch_ls_slope(const double* dot, double* info, hipStream_t st);
hipError_t launch_ls_trial(int n, const float* u, float eta, const float* s, float* trial, const int* search,
                           hipStream_t st);
hipError_t launch_ls_check(const double* sums, double dmul, double smul, double sk, double alpha, double c1, double eta,
                           int k, int* search, double* info, hipStream_t st);
hipError_t launch_ls_commit(int n, const float* trial, float* u, const double* info, hipStream_t st);
hipEvent_t prof_event(mfr_ctx* c);   // a timing event from the context's pool
template <class F>
hipError_t timed(mfr_ctx* c, int slot, F&& launch) {
  if (!c->prof_on) return launch();
  hipEvent_t a = prof_event(c), b = prof_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, c->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, c->stream);
  if (e != hipSuccess) return e;
  c->prof_pending.push_back({slot, {a, b}});
  return hipSuccess;
}

hipError_t enqueue_diag(mfr_ctx* c, const float* u, float* diag);
hipError_t enqueue_pcg_diag(mfr_ctx* c, const float* u, float* diag);   // zero entries -> 1
int node_blocks(const mfr_ctx* c);   // work-groups (per component) of a node pass
int node_parts(const mfr_ctx* c);    // float64 partials of a gradient / Hv node pass (3 per group)
mfr_status check_ptr(const void* p, const char* name);
mfr_status enqueue_objective(mfr_ctx* c, const float* u);
mfr_status read_objective(mfr_ctx* c, double* J, double* D, double* S);
mfr_status enqueue_gradient(mfr_ctx* c, const float* u, float* g);
mfr_status enqueue_hess_vec(mfr_ctx* c, const float* u, const float* p, float* q);
mfr_status pcg_run(mfr_ctx* c, const float* u, const float* b, float* s_out, const mfr_pcg_opts* o,
                   mfr_pcg_info* info);
mfr_status gn_step(mfr_ctx* c, float* u, const mfr_gn_opts* o, mfr_gn_info* out);

// learned preconditioner (pc.cpp) as used by the flexible CG of pcg_run
mfr_status pc_begin_solve(mfr_pc* pc, const float* diag);
// live (nullable): every kernel of the application does nothing while *live == 0.
// keep_input: store the network input in h0 (a separate feature pass; training
// needs it for the first layer's weight gradient).
mfr_status pc_forward(mfr_pc* pc, const float* r, const float* diag, float* z, bool scales_ready = false,
                      const float* rprev = nullptr, double* zred = nullptr, const int* live = nullptr,
                      bool keep_input = false);
float* pc_scratch_vec(mfr_pc* pc);
// The context of pc is being destroyed: pc is left unbound (mfr_pc_bind again before use).
void pc_release_context(mfr_pc* pc);
// Take pc off its context (detached too); mfr_pc_bind before its next use.
void pc_unbind(mfr_pc* pc);
// MFR_EINVAL / MFR_ENOMEM unless pc can be bound to a context of geometry g.
mfr_status pc_check_grid(const mfr_pc* pc, const Geo& g);
double* pc_red(mfr_pc* pc);
double* pc_scalars(mfr_pc* pc);
int pc_conv_blocks(const mfr_pc* pc);

}  // namespace mfr
