// L-BFGS on J = D + alpha S (Sec. 2.3.2) with the regulariser's Hessian in
// the initial matrix, H_0 = alpha nabla^2 S + gamma I (2 alpha hbar^y L^T L +
// gamma I for curvature, -alpha hbar^y L + gamma I for the diffusive one), solved exactly in the cosine basis of the Neumann Laplacian
// (lbfgs_kernels.hip).  The host runs the two-loop recursion over device
// vectors with float64 dot products, an Armijo line search from eta = 1, and
// keeps a pair (s, y) only when s^T y > 1e-12 |s| |y|.  A direction that is
// not a descent direction clears the memory and restarts from -H_0^{-1} g.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/mfr.h"
#include "ctx_internal.h"

namespace mfr {

mfr_status fail(mfr_status s, const char* fmt, ...);

namespace {

constexpr int kMaxAxis = 4096;   // the cosine matrices hold n^2 floats per axis

struct LbLayout {
  size_t C[3], Ct[3], lam;
  size_t vec;        // first node vector
  size_t vbytes;     // bytes per node vector (aligned)
  int nvec;
  size_t total;
};

LbLayout lb_layout(const Geo& g, int mem) {
  LbLayout L{};
  size_t o = 0;
  for (int d = 0; d < 3; ++d) {
    L.C[d] = o;
    o = align_up(o + sizeof(float) * (size_t)g.n[d] * g.n[d]);
    L.Ct[d] = o;
    o = align_up(o + sizeof(float) * (size_t)g.n[d] * g.n[d]);
  }
  L.lam = o;
  o = align_up(o + sizeof(float) * (size_t)(g.n[0] + g.n[1] + g.n[2]));
  L.vec = o;
  L.vbytes = align_up(sizeof(float) * g.nc() * g.nbar);
  // ta, tb (transform scratch), g, gn, d, trial, and mem + 1 slots of (s, y)
  L.nvec = 6 + 2 * (mem + 1);
  L.total = o + L.vbytes * (size_t)L.nvec;
  return L;
}

mfr_status check_geo(const Geo& g) {
  if (g.reg == MFR_REG_ELASTIC)
    return fail(MFR_EINVAL, "the H_0 solve needs a regulariser that acts on each component alone (not elastic)");
  for (int d = 0; d < 3; ++d)
    if (g.n[d] > kMaxAxis) return fail(MFR_EINVAL, "my[%d] = %d: the H_0 solve supports at most %d nodes per axis", d,
                                      g.n[d], kMaxAxis);
  return MFR_OK;
}

// Orthonormal DCT-II matrices, their transposes and the eigenvalues
// -4 sin^2(pi k / 2n) / hy^2 of the Neumann second difference, built once per
// context on the host and copied into work (the work buffer is the caller's,
// so every call copies them again; the host copies outlive the copies).
mfr_status upload_tables(mfr_ctx* c, const LbLayout& L, char* work, H0Tables* t) {
  const Geo& g = c->geo;
  if (c->h0_lam.empty()) {
    for (int d = 0; d < 3; ++d) {
      const int n = g.n[d];
      std::vector<float>& C = c->h0_C[d];
      std::vector<float>& Ct = c->h0_Ct[d];
      C.assign((size_t)n * n, 0.0f);
      Ct.assign((size_t)n * n, 0.0f);
      for (int k = 0; k < n; ++k) {
        const double w = std::sqrt((k == 0 ? 1.0 : 2.0) / n);
        for (int i = 0; i < n; ++i) {
          const float v = (float)(w * std::cos(M_PI * k * (2.0 * i + 1.0) / (2.0 * n)));
          C[(size_t)k * n + i] = v;
          Ct[(size_t)i * n + k] = v;
        }
        const double sn = std::sin(M_PI * k / (2.0 * n));
        c->h0_lam.push_back((float)(-4.0 * sn * sn / (g.hy[d] * g.hy[d])));
      }
    }
  }
  for (int d = 0; d < 3; ++d) {
    HIP_TRY(hipMemcpyAsync(work + L.C[d], c->h0_C[d].data(), sizeof(float) * c->h0_C[d].size(),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(work + L.Ct[d], c->h0_Ct[d].data(), sizeof(float) * c->h0_Ct[d].size(),
                           hipMemcpyHostToDevice, c->stream));
    t->n[d] = g.n[d];
    t->C[d] = reinterpret_cast<const float*>(work + L.C[d]);
    t->Ct[d] = reinterpret_cast<const float*>(work + L.Ct[d]);
  }
  HIP_TRY(hipMemcpyAsync(work + L.lam, c->h0_lam.data(), sizeof(float) * c->h0_lam.size(), hipMemcpyHostToDevice,
                         c->stream));
  t->lam = reinterpret_cast<const float*>(work + L.lam);
  t->nc = g.nc();
  return MFR_OK;
}

mfr_status check_work(const mfr_ctx* c, const LbLayout& L, const void* work, size_t bytes) {
  (void)c;
  if (!work || reinterpret_cast<uintptr_t>(work) % 256 != 0)
    return fail(MFR_EINVAL, "work must be non-NULL and 256-byte aligned");
  if (bytes < L.total) return fail(MFR_ENOMEM, "work holds %zu bytes, %zu needed", bytes, L.total);
  return MFR_OK;
}

// float64 dot product of two node vectors (synchronises the stream)
mfr_status dot(mfr_ctx* c, const float* a, const float* b, double* out) {
  const int n3 = (int)(c->geo.nc() * c->geo.nbar);
  HIP_TRY(launch_dot(n3, a, b, c->red_node, c->vec_blocks, c->stream));
  HIP_TRY(launch_sum(c->red_node, c->vec_blocks, c->sc + SC_DOT, c->stream));
  HIP_TRY(hipMemcpyAsync(out, c->sc + SC_DOT, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MFR_OK;
}

// H_0 = c2 L^T L + c1 L + gamma I: (2 alpha hbar^y, 0) for curvature, (0, -alpha hbar^y) diffusive
void h0_coeffs(const Geo& g, float* c2, float* c1) {
  *c2 = g.reg == MFR_REG_DIFFUSIVE ? 0.0f : (float)(2.0 * g.alpha * g.hybar());
  *c1 = g.reg == MFR_REG_DIFFUSIVE ? (float)(-g.alpha * g.hybar()) : 0.0f;
}

mfr_status lbfgs_run(mfr_ctx* c, float* u, const mfr_lbfgs_opts* o, char* work, const LbLayout& L,
                     mfr_lbfgs_report* rep) {
  const auto t0 = std::chrono::steady_clock::now();
  const int n3 = (int)(c->geo.nc() * c->geo.nbar);
  H0Tables tab{};
  MFR_TRY(upload_tables(c, L, work, &tab));
  auto vec = [&](int k) { return reinterpret_cast<float*>(work + L.vec + (size_t)k * L.vbytes); };
  float* ta = vec(0);
  float* tb = vec(1);
  float* g = vec(2);
  float* gn = vec(3);
  float* d = vec(4);
  float* trial = vec(5);
  const int slots = o->mem + 1;
  std::vector<float*> S(slots), Y(slots);
  for (int k = 0; k < slots; ++k) {
    S[k] = vec(6 + 2 * k);
    Y[k] = vec(7 + 2 * k);
  }
  std::vector<double> rho(slots, 0.0), a(slots, 0.0);
  std::vector<int> hist;   // slots of the stored pairs, oldest first
  float c2 = 0.0f, c1 = 0.0f;
  h0_coeffs(c->geo, &c2, &c1);
  const float gam = (float)o->gamma;

  mfr_lbfgs_report R{};
  double J = 0.0;
  MFR_TRY(enqueue_gradient(c, u, g));
  MFR_TRY(read_objective(c, &J, nullptr, nullptr));
  R.J_initial = R.J_final = J;
  R.evals = 1;
  for (int it = 0; it < o->iters; ++it) {
    // two-loop recursion: d = -H g
    HIP_TRY(launch_axpy(n3, g, -2.0f, g, d, c->stream));
    for (int h = (int)hist.size() - 1; h >= 0; --h) {
      const int k = hist[h];
      double sq = 0.0;
      MFR_TRY(dot(c, S[k], d, &sq));
      a[k] = rho[k] * sq;
      HIP_TRY(launch_axpy(n3, d, (float)-a[k], Y[k], d, c->stream));
    }
    HIP_TRY(launch_h0_solve(tab, d, d, ta, tb, c2, c1, gam, c->stream));
    for (int k : hist) {
      double yr = 0.0;
      MFR_TRY(dot(c, Y[k], d, &yr));
      HIP_TRY(launch_axpy(n3, d, (float)(a[k] - rho[k] * yr), S[k], d, c->stream));
    }
    double slope = 0.0;
    MFR_TRY(dot(c, g, d, &slope));
    if (!(slope < 0.0)) {
      // not a descent direction: forget the pairs and take -H_0^{-1} g
      hist.clear();
      ++R.restarts;
      HIP_TRY(launch_axpy(n3, g, -2.0f, g, d, c->stream));
      HIP_TRY(launch_h0_solve(tab, d, d, ta, tb, c2, c1, gam, c->stream));
      MFR_TRY(dot(c, g, d, &slope));
      if (!(slope < 0.0)) break;   // zero (or non-finite) gradient: nothing to do
    }
    double eta = 1.0, Jn = 0.0;
    bool accepted = false;
    for (int ls = 0; ls < o->armijo_max; ++ls) {
      HIP_TRY(launch_axpy(n3, u, (float)eta, d, trial, c->stream));
      MFR_TRY(enqueue_objective(c, trial));
      const mfr_status st = read_objective(c, &Jn, nullptr, nullptr);
      ++R.evals;
      if (st == MFR_OK && Jn <= J + o->armijo_c1 * eta * slope) {
        accepted = true;
        break;
      }
      eta *= 0.5;
    }
    if (!accepted) {
      R.status = MFR_ELINESEARCH;
      break;
    }
    // the new pair goes to a free slot (there is always one: mem + 1 slots)
    int slot = 0;
    while (std::find(hist.begin(), hist.end(), slot) != hist.end()) ++slot;
    HIP_TRY(launch_axpy(n3, trial, -1.0f, u, S[slot], c->stream));   // s = u_new - u (the step taken)
    HIP_TRY(hipMemcpyAsync(u, trial, sizeof(float) * n3, hipMemcpyDeviceToDevice, c->stream));
    MFR_TRY(enqueue_gradient(c, u, gn));
    MFR_TRY(read_objective(c, &J, nullptr, nullptr));
    ++R.evals;
    HIP_TRY(launch_axpy(n3, gn, -1.0f, g, Y[slot], c->stream));     // y = g_new - g
    double sy = 0.0, ss = 0.0, yy = 0.0;
    MFR_TRY(dot(c, S[slot], Y[slot], &sy));
    MFR_TRY(dot(c, S[slot], S[slot], &ss));
    MFR_TRY(dot(c, Y[slot], Y[slot], &yy));
    if (sy > 1e-12 * std::sqrt(ss * yy)) {
      rho[slot] = 1.0 / sy;
      hist.push_back(slot);
      if ((int)hist.size() > o->mem) hist.erase(hist.begin());
    } else {
      ++R.pairs_skipped;
    }
    std::swap(g, gn);
    R.iters = it + 1;
    R.J_final = J;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = R;
  return MFR_OK;
}

}  // namespace

}  // namespace mfr

using namespace mfr;

extern "C" {

mfr_status mfr_lbfgs_workspace_size(const mfr_grid* grid, int32_t mem, size_t* bytes) {
  Geo g;
  MFR_TRY(make_geo(grid, &g));
  MFR_TRY(check_geo(g));
  if (!bytes) return fail(MFR_EINVAL, "bytes is NULL");
  if (mem < 1 || mem > MFR_LBFGS_MAX_MEM) return fail(MFR_EINVAL, "mem = %d: need 1..%d", mem, MFR_LBFGS_MAX_MEM);
  *bytes = lb_layout(g, mem).total;
  return MFR_OK;
}

mfr_status mfr_h0_solve(mfr_ctx* c, double gamma, const float* v, float* x, void* work, size_t work_bytes) {
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  MFR_TRY(check_geo(c->geo));
  MFR_TRY(check_ptr(v, "v"));
  MFR_TRY(check_ptr(x, "x"));
  if (!(gamma > 0) || !std::isfinite(gamma)) return fail(MFR_EINVAL, "gamma must be > 0");
  const LbLayout L = lb_layout(c->geo, 1);
  MFR_TRY(check_work(c, L, work, work_bytes));
  char* w = static_cast<char*>(work);
  H0Tables tab{};
  MFR_TRY(upload_tables(c, L, w, &tab));
  float* ta = reinterpret_cast<float*>(w + L.vec);
  float* tb = reinterpret_cast<float*>(w + L.vec + L.vbytes);
  float c2 = 0.0f, c1 = 0.0f;
  h0_coeffs(c->geo, &c2, &c1);
  HIP_TRY(launch_h0_solve(tab, v, x, ta, tb, c2, c1, (float)gamma, c->stream));
  return MFR_OK;
}

mfr_status mfr_lbfgs(mfr_ctx* c, float* u, const mfr_lbfgs_opts* o, void* work, size_t work_bytes,
                     mfr_lbfgs_report* rep) {
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  if (!c->have_images) return fail(MFR_EINVAL, "mfr_set_images has not been called");
  MFR_TRY(check_geo(c->geo));
  MFR_TRY(check_ptr(u, "u"));
  if (!o) return fail(MFR_EINVAL, "opts is NULL");
  if (o->iters < 0 || o->mem < 1 || o->mem > MFR_LBFGS_MAX_MEM || !(o->gamma > 0) || !std::isfinite(o->gamma) ||
      !(o->armijo_c1 >= 0 && o->armijo_c1 < 1) || o->armijo_max < 1)
    return fail(MFR_EINVAL, "invalid L-BFGS options");
  const LbLayout L = lb_layout(c->geo, o->mem);
  MFR_TRY(check_work(c, L, work, work_bytes));
  const char* w = static_cast<const char*>(work);
  const char* ub = reinterpret_cast<const char*>(u);
  if (ub + sizeof(float) * c->geo.nc() * c->geo.nbar > w && ub < w + L.total)
    return fail(MFR_EINVAL, "u must not point into the work buffer");
  return lbfgs_run(c, u, o, static_cast<char*>(work), L, rep);
}

}  // extern "C"
