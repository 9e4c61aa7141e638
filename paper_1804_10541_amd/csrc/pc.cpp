// Learned preconditioner (include/mfr.h, mfr_pc_*, mfr_cnn_*): workspace
// layout, forward pass, training on Gauss-Newton systems, and the C ABI of the
// convolution kernels.  An extension of the method: the paper solves the
// Newton equation of Sec. 2.3.1 with plain CG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "ctx_internal.h"

using namespace mfr;

struct mfr_pc {
  mfr_ctx* c = nullptr;
  bool train = false;
  int nx = 0, ny = 0, nz = 0, n = 0, n3 = 0;
  float* params = nullptr;    // fp32 master copy, kCnnParams
  uint16_t* w16 = nullptr;    // bf16 weights, both layouts (2 x kCnnLayers x kCnnWeights)
  float* grad = nullptr;      // train: kCnnParams
  float* am = nullptr;        // train: Adam first / second moments
  float* av = nullptr;
  uint16_t* h[kCnnLayers] = {};   // activations h0 (features) .. h3, [n][16] bf16
  uint16_t* gA = nullptr;     // train: gradient activations (ping-pong)
  uint16_t* gB = nullptr;
  float* gR = nullptr;        // |grad R| on the nodes, n
  float* diag = nullptr;      // Jacobi diagonal for mfr_pc_apply / training, 3n
  float* vtmp = nullptr;      // 3n scratch (previous residual of flexible CG)
  float* y = nullptr;         // train: 3n each
  float* Ay = nullptr;
  float* z = nullptr;
  float* Az = nullptr;
  float* s = nullptr;
  float* wpart = nullptr;     // train: weight-gradient partials
  float* gm1 = nullptr;       // |grad R| restriction passes
  float* gm2 = nullptr;
  Range1 *rx = nullptr, *ry = nullptr, *rz = nullptr;
  float *wsx = nullptr, *wsy = nullptr, *wsz = nullptr;
  double* sc = nullptr;       // PC_COUNT scalars
  double* red = nullptr;      // 4 x pc_dots_blocks partials, or 2 per convolution group
  int adam_t = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  const float* gR_src = nullptr;
  unsigned gR_version = ~0u;
};

namespace {

struct PcLayout {
  size_t params, w16, grad, am, av, h[kCnnLayers], gA, gB, gR, diag, vtmp, y, Ay, z, Az, s, wpart, gm1, gm2;
  size_t rx, ry, rz, wsx, wsy, wsz, sc, red, total;
};

PcLayout pc_layout(const Geo& g, bool train) {
  PcLayout L{};
  const size_t n = g.nbar, n3 = 3 * n;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  // parameter state first: its offsets do not depend on the grid (mfr_pc_bind)
  L.params = take(sizeof(float) * kCnnParams);
  L.w16 = take(sizeof(uint16_t) * 2 * kCnnLayers * kCnnWeights);
  L.grad = take(sizeof(float) * kCnnParams);
  L.am = take(sizeof(float) * kCnnParams);
  L.av = take(sizeof(float) * kCnnParams);
  for (int l = 0; l < kCnnLayers; ++l) L.h[l] = take(sizeof(uint16_t) * 16 * n);
  L.gR = take(sizeof(float) * n);
  L.diag = take(sizeof(float) * n3);
  L.vtmp = take(sizeof(float) * n3);
  L.gm1 = take(sizeof(float) * (size_t)g.m[2] * g.m[1] * g.n[0]);
  L.gm2 = take(sizeof(float) * (size_t)g.m[2] * g.n[1] * g.n[0]);
  L.rx = take(sizeof(Range1) * g.n[0]);
  L.ry = take(sizeof(Range1) * g.n[1]);
  L.rz = take(sizeof(Range1) * g.n[2]);
  L.wsx = take(sizeof(float) * g.n[0]);
  L.wsy = take(sizeof(float) * g.n[1]);
  L.wsz = take(sizeof(float) * g.n[2]);
  L.sc = take(sizeof(double) * PC_COUNT);
  L.red = take(sizeof(double) * std::max(4 * pc_dots_blocks(n3), 2 * cnn_conv_blocks(g.n[0], g.n[1], g.n[2])));
  if (train) {
    L.gA = take(sizeof(uint16_t) * 16 * n);
    L.gB = take(sizeof(uint16_t) * 16 * n);
    L.y = take(sizeof(float) * n3);
    L.Ay = take(sizeof(float) * n3);
    L.z = take(sizeof(float) * n3);
    L.Az = take(sizeof(float) * n3);
    L.s = take(sizeof(float) * n3);
    L.wpart = take(sizeof(float) * (size_t)cnn_wgrad_groups(g.n[0], g.n[1], g.n[2]) * kCnnLayerParams);
  }
  L.total = o;
  return L;
}

hipStream_t st_of(const mfr_pc* pc) { return pc->c->stream; }

// |grad R| on the nodes, recomputed when the context's images change.
mfr_status refresh_gR(mfr_pc* pc) {
  mfr_ctx* c = pc->c;
  if (!c->have_images) return fail(MFR_EINVAL, "the context has no images");
  if (pc->gR_src == c->R && pc->gR_version == c->image_version) return MFR_OK;
  const Geo& g = c->geo;
  GmArgs a{};
  a.mx = g.m[0];
  a.my = g.m[1];
  a.mz = g.m[2];
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.R = c->R;
  a.cx = c->tp.cx;
  a.cy = c->tp.cy;
  a.cz = c->tp.cz;
  a.rx = pc->rx;
  a.ry = pc->ry;
  a.rz = pc->rz;
  a.wsx = pc->wsx;
  a.wsy = pc->wsy;
  a.wsz = pc->wsz;
  a.ih2x = (float)(1.0 / (g.h[0] * g.h[0]));
  a.ih2y = (float)(1.0 / (g.h[1] * g.h[1]));
  a.ih2z = (float)(1.0 / (g.h[2] * g.h[2]));
  HIP_TRY(launch_pc_gradmag(a, pc->gm1, pc->gm2, pc->gR, st_of(pc)));
  DotsArgs d{};
  DotsOut o{};
  d.n = (size_t)pc->n;
  d.count = 1;
  d.a[0] = pc->gR;
  o.out[0] = pc->sc + PC_RMS_G;
  o.rms_scale[0] = 1.0 / pc->n;
  HIP_TRY(launch_pc_dots(d, o, pc->red, st_of(pc)));
  pc->gR_src = c->R;
  pc->gR_version = c->image_version;
  return MFR_OK;
}

mfr_status train_step(mfr_pc* pc, const float* u, const float* r, const mfr_pc_train_opts* o) {
  mfr_ctx* c = pc->c;
  hipStream_t st = st_of(pc);
  const int n3 = pc->n3;
  // Jacobi direction and its curvature (the reference energy)
  HIP_TRY(launch_pc_jacobi(n3, r, pc->diag, pc->y, st));
  MFR_TRY(enqueue_hess_vec(c, u, pc->y, pc->Ay));
  // forward pass and A z
  MFR_TRY(pc_forward(pc, r, pc->diag, pc->z, false, nullptr, nullptr, nullptr, true));
  MFR_TRY(enqueue_hess_vec(c, u, pc->z, pc->Az));
  DotsArgs d{};
  DotsOut out{};
  d.n = (size_t)n3;
  d.count = 4;
  d.a[0] = pc->z;
  d.b[0] = r;
  d.a[1] = pc->z;
  d.b[1] = pc->Az;
  d.a[2] = pc->y;
  d.b[2] = r;
  d.a[3] = pc->y;
  d.b[3] = pc->Ay;
  out.out[0] = pc->sc + PC_ZR;
  out.out[1] = pc->sc + PC_ZAZ;
  out.out[2] = pc->sc + PC_YR;
  out.out[3] = pc->sc + PC_YAY;
  HIP_TRY(launch_pc_dots(d, out, pc->red, st));
  HIP_TRY(launch_pc_loss(pc->sc, st));
  // backward: gradient at the output, then layer by layer (ReLU masks from the
  // stored activations), weight gradients per layer
  HIP_TRY(launch_pc_grad_out(pc->n, pc->Az, r, pc->sc, pc->gA, st));
  uint16_t* g = pc->gA;
  uint16_t* gn = pc->gB;
  for (int l = kCnnLayers - 1; l >= 0; --l) {
    HIP_TRY(launch_cnn_wgrad(pc->nx, pc->ny, pc->nz, pc->h[l], g, pc->wpart, pc->grad + (size_t)l * kCnnLayerParams,
                             st));
    if (l > 0) {
      ConvArgs a{};
      a.nx = pc->nx;
      a.ny = pc->ny;
      a.nz = pc->nz;
      a.x = g;
      a.w = pc->w16 + (size_t)l * kCnnWeights;
      a.transpose = 1;
      a.mask = pc->h[l];
      a.y16 = gn;
      HIP_TRY(launch_cnn_conv(a, st));
      std::swap(g, gn);
    }
  }
  ++pc->adam_t;
  AdamArgs h{};
  h.lr = (float)o->lr;
  h.beta1 = (float)o->beta1;
  h.beta2 = (float)o->beta2;
  h.eps = (float)o->eps;
  h.bc1 = (float)(1.0 - std::pow(o->beta1, pc->adam_t));
  h.bc2 = (float)(1.0 - std::pow(o->beta2, pc->adam_t));
  HIP_TRY(launch_cnn_adam(pc->params, pc->grad, pc->am, pc->av, pc->w16, h, st));
  return MFR_OK;
}

mfr_status check_pc(const mfr_pc* pc) {
  if (!pc) return fail(MFR_EINVAL, "preconditioner is NULL");
  return MFR_OK;
}

// A preconditioner whose context was destroyed has none until it is bound again.
mfr_status check_bound(const mfr_pc* pc) {
  MFR_TRY(check_pc(pc));
  if (!pc->c) return fail(MFR_EINVAL, "the preconditioner's context was destroyed; bind it with mfr_pc_bind first");
  return MFR_OK;
}

// Take pc off the context it is bound to (and attached to, if it is).
void unlink_pc(mfr_pc* pc) {
  mfr_ctx* c = pc->c;
  if (!c) return;
  if (c->pc == pc) c->pc = nullptr;
  auto& v = c->bound_pcs;
  v.erase(std::remove(v.begin(), v.end(), pc), v.end());
  pc->c = nullptr;
}

mfr_status check_grid_dims(int nx, int ny, int nz) {
  if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz >= (1LL << 26))
    return fail(MFR_EINVAL, "node grid %d x %d x %d out of range", nx, ny, nz);
  return MFR_OK;
}

mfr_status check_aligned(const void* p, size_t a, const char* name) {
  if (!p) return fail(MFR_EINVAL, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % a != 0) return fail(MFR_EINVAL, "%s is not %zu-byte aligned", name, a);
  return MFR_OK;
}

}  // namespace

namespace mfr {

// Scales of the solve: RMS of the Jacobi diagonal (and |grad R| if the images changed).
mfr_status pc_begin_solve(mfr_pc* pc, const float* diag) {
  MFR_TRY(refresh_gR(pc));
  DotsArgs d{};
  DotsOut o{};
  d.n = (size_t)pc->n3;
  d.count = 1;
  d.a[0] = diag;
  o.out[0] = pc->sc + PC_RMS_D;
  o.rms_scale[0] = 1.0 / pc->n3;
  HIP_TRY(launch_pc_dots(d, o, pc->red, st_of(pc)));
  return MFR_OK;
}

// z = r / diag + rms(r / diag) * CNN(features)[0..2].  scales_ready: the RMS of
// r and r/diag are already in the scalars (the flexible-CG update computes them).
// zred: the final layer also leaves per-group partials of z.r and z.rprev there.
mfr_status pc_forward(mfr_pc* pc, const float* r, const float* diag, float* z, bool scales_ready,
                      const float* rprev, double* zred, const int* live, bool keep_input) {
  hipStream_t st = st_of(pc);
  if (!scales_ready) {
    DotsArgs d{};
    DotsOut o{};
    d.n = (size_t)pc->n3;
    d.count = 2;
    d.a[0] = r;
    d.den[0] = diag;
    d.a[1] = r;
    d.live = live;
    o.out[0] = pc->sc + PC_RMS_Y;
    o.out[1] = pc->sc + PC_RMS_R;
    o.rms_scale[0] = o.rms_scale[1] = 1.0 / pc->n3;
    HIP_TRY(launch_pc_dots(d, o, pc->red, st));
  }
  // the network (timed as one record when the context's timing is on)
  HIP_TRY(timed(pc->c, 5, [&]() -> hipError_t {
    // the network input: stored for the first layer's weight gradient in
    // training, else computed by the first layer itself while it stages a tile
    if (keep_input) {
      const hipError_t e = launch_pc_features(pc->n, r, diag, pc->gR, pc->sc, pc->h[0], st, live);
      if (e != hipSuccess) return e;
    }
    for (int l = 0; l < kCnnLayers; ++l) {
      ConvArgs a{};
      a.nx = pc->nx;
      a.ny = pc->ny;
      a.nz = pc->nz;
      if (l > 0 || keep_input) {
        a.x = pc->h[l];
      } else {
        a.fr = r;
        a.fdiag = diag;
        a.fgR = pc->gR;
        a.fsc = pc->sc;
      }
      a.live = live;
      a.w = pc->w16 + (size_t)(kCnnLayers + l) * kCnnWeights;
      a.w_out_major = 1;
      a.bias = pc->params + (size_t)l * kCnnLayerParams + kCnnWeights;
      if (l < kCnnLayers - 1) {
        a.relu = 1;
        a.y16 = pc->h[l + 1];
      } else {
        a.z = z;
        a.r = r;
        a.diag = diag;
        a.scale = pc->sc + PC_RMS_Y;
        a.rprev = rprev;
        a.zred = zred;
      }
      const hipError_t e = launch_cnn_conv(a, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }));
  return MFR_OK;
}

float* pc_scratch_vec(mfr_pc* pc) { return pc->vtmp; }
void pc_release_context(mfr_pc* pc) { pc->c = nullptr; }
void pc_unbind(mfr_pc* pc) { unlink_pc(pc); }

mfr_status pc_check_grid(const mfr_pc* pc, const Geo& g) {
  MFR_TRY(check_pc(pc));
  if (g.dim == 2) return fail(MFR_EINVAL, "the learned preconditioner takes three-dimensional problems only");
  const size_t need = pc_layout(g, pc->train).total;
  if (pc->ws_bytes < need)
    return fail(MFR_ENOMEM, "preconditioner workspace of %zu bytes is smaller than the %zu the grid needs", pc->ws_bytes,
                need);
  return MFR_OK;
}
double* pc_scalars(mfr_pc* pc) { return pc->sc; }
int pc_conv_blocks(const mfr_pc* pc) { return cnn_conv_blocks(pc->nx, pc->ny, pc->nz); }
double* pc_red(mfr_pc* pc) { return pc->red; }

}  // namespace mfr

extern "C" {

mfr_status mfr_pc_workspace_size(const mfr_grid* grid, int32_t train, size_t* bytes) {
  if (!bytes) return fail(MFR_EINVAL, "bytes is NULL");
  Geo g;
  MFR_TRY(make_geo(grid, &g));
  if (g.dim == 2) return fail(MFR_EINVAL, "the learned preconditioner takes three-dimensional problems only");
  *bytes = pc_layout(g, train != 0).total;
  return MFR_OK;
}

}  // extern "C"

namespace {

// Points the grid-dependent buffers of pc at context c's grid and uploads the
// per-axis tables; the parameter state (front of the workspace) is kept.
mfr_status bind_pc(mfr_pc* pc, mfr_ctx* c) {
  if (!c->have_images) return fail(MFR_EINVAL, "the context has no images");
  const Geo& g = c->geo;
  const PcLayout L = pc_layout(g, pc->train);
  if (pc->ws_bytes < L.total)
    return fail(MFR_ENOMEM, "workspace of %zu bytes is smaller than the required %zu", pc->ws_bytes, L.total);
  if (pc->c != c) {
    unlink_pc(pc);
    c->bound_pcs.push_back(pc);
    pc->c = c;
  }
  char* ws = pc->ws;
  pc->nx = g.n[0];
  pc->ny = g.n[1];
  pc->nz = g.n[2];
  pc->n = (int)g.nbar;
  pc->n3 = (int)(3 * g.nbar);
  for (int l = 0; l < kCnnLayers; ++l) pc->h[l] = at<uint16_t>(ws, L.h[l]);
  pc->gR = at<float>(ws, L.gR);
  pc->diag = at<float>(ws, L.diag);
  pc->vtmp = at<float>(ws, L.vtmp);
  pc->gm1 = at<float>(ws, L.gm1);
  pc->gm2 = at<float>(ws, L.gm2);
  pc->rx = at<Range1>(ws, L.rx);
  pc->ry = at<Range1>(ws, L.ry);
  pc->rz = at<Range1>(ws, L.rz);
  pc->wsx = at<float>(ws, L.wsx);
  pc->wsy = at<float>(ws, L.wsy);
  pc->wsz = at<float>(ws, L.wsz);
  pc->sc = at<double>(ws, L.sc);
  pc->red = at<double>(ws, L.red);
  if (pc->train) {
    pc->gA = at<uint16_t>(ws, L.gA);
    pc->gB = at<uint16_t>(ws, L.gB);
    pc->y = at<float>(ws, L.y);
    pc->Ay = at<float>(ws, L.Ay);
    pc->z = at<float>(ws, L.z);
    pc->Az = at<float>(ws, L.Az);
    pc->s = at<float>(ws, L.s);
    pc->wpart = at<float>(ws, L.wpart);
  }
  pc->gR_src = nullptr;   // |grad R| is recomputed for the new images
  // per-axis node ranges of the conversion and their weight sums (host tables)
  std::vector<Range1> rr[3];
  std::vector<float> wsum[3];
  for (int k = 0; k < 3; ++k) {
    const auto cv = conv_table(g.m[k], g.n[k]);
    rr[k] = node_cols(cv, g.n[k]);
    wsum[k].assign(g.n[k], 0.f);
    for (int a = 0; a < g.m[k]; ++a) {
      wsum[k][cv[a].n0] += 1.0f - cv[a].f;
      wsum[k][cv[a].n0 + 1] += cv[a].f;
    }
  }
  hipStream_t st = c->stream;
  HIP_TRY(hipMemcpyAsync(pc->rx, rr[0].data(), sizeof(Range1) * g.n[0], hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(pc->ry, rr[1].data(), sizeof(Range1) * g.n[1], hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(pc->rz, rr[2].data(), sizeof(Range1) * g.n[2], hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(pc->wsx, wsum[0].data(), sizeof(float) * g.n[0], hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(pc->wsy, wsum[1].data(), sizeof(float) * g.n[1], hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(pc->wsz, wsum[2].data(), sizeof(float) * g.n[2], hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));   // the host tables go out of scope
  return MFR_OK;
}

}  // namespace

extern "C" {

mfr_status mfr_pc_create(mfr_ctx* c, int32_t train, void* workspace, size_t ws_bytes, mfr_pc** out) {
  if (!out) return fail(MFR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  if (c->geo.dim == 2) return fail(MFR_EINVAL, "the learned preconditioner takes three-dimensional problems only");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(MFR_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  mfr_pc* pc = new (std::nothrow) mfr_pc();
  if (!pc) return fail(MFR_EINVAL, "host allocation failed");
  char* ws = reinterpret_cast<char*>(workspace);
  pc->train = train != 0;
  pc->ws = ws;
  pc->ws_bytes = ws_bytes;
  const PcLayout L = pc_layout(c->geo, pc->train);
  pc->params = at<float>(ws, L.params);
  pc->w16 = at<uint16_t>(ws, L.w16);
  pc->grad = at<float>(ws, L.grad);
  pc->am = at<float>(ws, L.am);
  pc->av = at<float>(ws, L.av);
  mfr_status s = bind_pc(pc, c);
  hipStream_t st = c->stream;
  if (s == MFR_OK && (hipMemsetAsync(pc->params, 0, sizeof(float) * kCnnParams, st) != hipSuccess ||
                      hipMemsetAsync(pc->am, 0, sizeof(float) * kCnnParams, st) != hipSuccess ||
                      hipMemsetAsync(pc->av, 0, sizeof(float) * kCnnParams, st) != hipSuccess))
    s = fail(MFR_EHIP, "parameter initialisation failed");
  if (s == MFR_OK && launch_cnn_cast(pc->params, pc->w16, st) != hipSuccess) s = fail(MFR_EHIP, "cast failed");
  if (s == MFR_OK && hipStreamSynchronize(st) != hipSuccess) s = fail(MFR_EHIP, "synchronisation failed");
  if (s != MFR_OK) {
    delete pc;
    return s;
  }
  *out = pc;
  return MFR_OK;
}

mfr_status mfr_pc_bind(mfr_pc* pc, mfr_ctx* c) {
  MFR_TRY(check_pc(pc));
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  if (c->geo.dim == 2) return fail(MFR_EINVAL, "the learned preconditioner takes three-dimensional problems only");
  return bind_pc(pc, c);
}

void mfr_pc_destroy(mfr_pc* pc) {
  if (pc) unlink_pc(pc);
  delete pc;
}

mfr_status mfr_pc_set_params(mfr_pc* pc, const float* params) {
  MFR_TRY(check_bound(pc));
  if (!params) return fail(MFR_EINVAL, "params is NULL");
  for (int i = 0; i < kCnnParams; ++i)
    if (!std::isfinite(params[i])) return fail(MFR_ENONFINITE, "parameter %d is not finite", i);
  hipStream_t st = st_of(pc);
  HIP_TRY(hipMemcpyAsync(pc->params, params, sizeof(float) * kCnnParams, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_cnn_cast(pc->params, pc->w16, st));
  if (pc->train) {
    HIP_TRY(hipMemsetAsync(pc->am, 0, sizeof(float) * kCnnParams, st));
    HIP_TRY(hipMemsetAsync(pc->av, 0, sizeof(float) * kCnnParams, st));
    pc->adam_t = 0;
  }
  HIP_TRY(hipStreamSynchronize(st));
  return MFR_OK;
}

mfr_status mfr_pc_get_params(mfr_pc* pc, float* params) {
  MFR_TRY(check_bound(pc));
  if (!params) return fail(MFR_EINVAL, "params is NULL");
  HIP_TRY(hipMemcpyAsync(params, pc->params, sizeof(float) * kCnnParams, hipMemcpyDeviceToHost, st_of(pc)));
  HIP_TRY(hipStreamSynchronize(st_of(pc)));
  return MFR_OK;
}

mfr_status mfr_pc_apply(mfr_pc* pc, const float* u, const float* r, float* z) {
  MFR_TRY(check_bound(pc));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(r, "r"));
  MFR_TRY(check_ptr(z, "z"));
  if (z == r || z == u) return fail(MFR_EINVAL, "z must not alias u or r");
  HIP_TRY(enqueue_diag(pc->c, u, pc->diag));
  MFR_TRY(pc_begin_solve(pc, pc->diag));
  return pc_forward(pc, r, pc->diag, z);
}

mfr_status mfr_pc_train_system(mfr_pc* pc, const float* u, const float* b, const mfr_pc_train_opts* o,
                               mfr_pc_train_info* info) {
  MFR_TRY(check_bound(pc));
  if (!pc->train) return fail(MFR_EINVAL, "preconditioner was created without training buffers");
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(b, "b"));
  if (!o) return fail(MFR_EINVAL, "opts is NULL");
  if (!(o->lr > 0) || !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1) || !(o->eps > 0) ||
      o->pcg_iters < 0 || o->sample_every < 1)
    return fail(MFR_EINVAL, "invalid training options");
  mfr_ctx* c = pc->c;
  hipStream_t st = c->stream;
  const int n3 = pc->n3, vb = c->vec_blocks;
  float* r = c->vec[0];
  float* z = c->vec[1];
  float* p = c->vec[2];
  float* q = c->vec[3];
  HIP_TRY(enqueue_diag(c, u, pc->diag));
  MFR_TRY(pc_begin_solve(pc, pc->diag));
  HIP_TRY(launch_pcg_init(n3, b, pc->diag, pc->s, r, z, p, c->red_node, vb, st));
  HIP_TRY(launch_pcg_init_finish(c->red_node, vb, c->sc, st));
  mfr_pc_train_info inf{0, 0.0, 0.0, 0.0};
  double sum = 0.0;
  double h[SC_COUNT];
  HIP_TRY(hipMemcpyAsync(h, c->sc, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double bb = h[SC_BB];
  if (!(bb > 0.0) || !std::isfinite(bb)) return fail(MFR_EINVAL, "right-hand side is zero or not finite");
  for (int it = 0; it <= o->pcg_iters; ++it) {
    if (it % o->sample_every == 0) {
      MFR_TRY(train_step(pc, u, r, o));
      double loss = 0.0;
      HIP_TRY(hipMemcpyAsync(&loss, pc->sc + PC_LOSS, sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (!std::isfinite(loss)) return fail(MFR_ENONFINITE, "training loss is not finite");
      if (inf.steps == 0) inf.loss_first = loss;
      inf.loss_last = loss;
      sum += loss;
      ++inf.steps;
    }
    if (it == o->pcg_iters) break;
    // one Jacobi-PCG iteration to move to the next residual
    MFR_TRY(enqueue_hess_vec(c, u, p, q));
    HIP_TRY(launch_pcg_alpha(c->red_node, node_parts(c), c->sc, st));
    HIP_TRY(launch_pcg_update(n3, pc->diag, p, q, pc->s, r, z, c->sc, c->red_node, vb, st));
    HIP_TRY(launch_pcg_beta(c->red_node, vb, c->sc, st));
    HIP_TRY(hipMemcpyAsync(h, c->sc, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!(h[SC_PQ] > 0.0) || !std::isfinite(h[SC_PQ]) || h[SC_RR] <= 1e-24 * bb) break;
    HIP_TRY(launch_pcg_direction(n3, z, p, c->sc, vb, st));
  }
  inf.loss_mean = inf.steps ? sum / inf.steps : 0.0;
  if (info) *info = inf;
  return MFR_OK;
}

mfr_status mfr_attach_pc(mfr_ctx* c, mfr_pc* pc) {
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  if (pc && pc->c != c) return fail(MFR_EINVAL, "the preconditioner belongs to another context");
  c->pc = pc;
  return MFR_OK;
}

mfr_status mfr_cnn_conv(int32_t nx, int32_t ny, int32_t nz, const uint16_t* x, const uint16_t* w, const float* bias,
                        int32_t relu, float* y32, uint16_t* y16, void* hip_stream) {
  MFR_TRY(check_grid_dims(nx, ny, nz));
  MFR_TRY(check_aligned(x, 16, "x"));
  MFR_TRY(check_aligned(w, 16, "w"));
  if (bias) MFR_TRY(check_aligned(bias, 16, "bias"));
  if (y32) MFR_TRY(check_aligned(y32, 16, "y32"));
  if (y16) MFR_TRY(check_aligned(y16, 8, "y16"));
  if (!y32 && !y16) return fail(MFR_EINVAL, "no output");
  ConvArgs a{};
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.x = x;
  a.w = w;
  a.bias = bias;
  a.relu = relu != 0;
  a.y16 = y16;
  a.y32 = y32;
  HIP_TRY(launch_cnn_conv(a, reinterpret_cast<hipStream_t>(hip_stream)));
  return MFR_OK;
}

mfr_status mfr_cnn_conv_bwd_data(int32_t nx, int32_t ny, int32_t nz, const uint16_t* g, const uint16_t* w,
                                 const uint16_t* mask, float* dx32, uint16_t* dx16, void* hip_stream) {
  MFR_TRY(check_grid_dims(nx, ny, nz));
  MFR_TRY(check_aligned(g, 16, "g"));
  MFR_TRY(check_aligned(w, 16, "w"));
  if (mask) MFR_TRY(check_aligned(mask, 8, "mask"));
  if (dx32) MFR_TRY(check_aligned(dx32, 16, "dx32"));
  if (dx16) MFR_TRY(check_aligned(dx16, 8, "dx16"));
  if (!dx32 && !dx16) return fail(MFR_EINVAL, "no output");
  ConvArgs a{};
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.x = g;
  a.w = w;
  a.transpose = 1;
  a.mask = mask;
  a.y16 = dx16;
  a.y32 = dx32;
  HIP_TRY(launch_cnn_conv(a, reinterpret_cast<hipStream_t>(hip_stream)));
  return MFR_OK;
}

mfr_status mfr_cnn_wgrad_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t* bytes) {
  MFR_TRY(check_grid_dims(nx, ny, nz));
  if (!bytes) return fail(MFR_EINVAL, "bytes is NULL");
  *bytes = sizeof(float) * (size_t)cnn_wgrad_groups(nx, ny, nz) * kCnnLayerParams;
  return MFR_OK;
}

mfr_status mfr_cnn_conv_bwd_weight(int32_t nx, int32_t ny, int32_t nz, const uint16_t* x, const uint16_t* g,
                                   float* dwb, void* workspace, size_t ws_bytes, void* hip_stream) {
  MFR_TRY(check_grid_dims(nx, ny, nz));
  MFR_TRY(check_aligned(x, 16, "x"));
  MFR_TRY(check_aligned(g, 16, "g"));
  MFR_TRY(check_aligned(dwb, 4, "dwb"));
  MFR_TRY(check_aligned(workspace, 4, "workspace"));
  size_t need = 0;
  MFR_TRY(mfr_cnn_wgrad_workspace_size(nx, ny, nz, &need));
  if (ws_bytes < need) return fail(MFR_ENOMEM, "workspace of %zu bytes is smaller than the required %zu", ws_bytes, need);
  HIP_TRY(launch_cnn_wgrad(nx, ny, nz, x, g, reinterpret_cast<float*>(workspace), dwb,
                           reinterpret_cast<hipStream_t>(hip_stream)));
  return MFR_OK;
}

}  // extern "C"
