// libmfr host side: argument validation, workspace layout, lookup tables, the
// C ABI of include/mfr.h, the conjugate-gradient solver and the multilevel
// Gauss-Newton driver (Sec. 2.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mfr.h"
#include "ctx_internal.h"

using namespace mfr;

namespace mfr {

thread_local std::string g_err;

mfr_status fail(mfr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}




mfr_status make_geo(const mfr_grid* g, Geo* o) {
  if (!g) return fail(MFR_EINVAL, "grid is NULL");
  const bool tdef = g->mT[0] == 0 && g->mT[1] == 0 && g->mT[2] == 0;
  const bool hdef = g->hT[0] == 0 && g->hT[1] == 0 && g->hT[2] == 0;
  // one cell and one node along z: the two-dimensional problem (d = 2 in Sec. 2.2)
  const bool plane = g->m[2] == 1 && g->my[2] == 1;
  o->dim = plane ? 2 : 3;
  if (plane && !(g->mT[2] == 0 || g->mT[2] == 1))
    return fail(MFR_EINVAL, "a two-dimensional problem (m[2] = my[2] = 1) needs mT[2] = 0 or 1");
  for (int k = 0; k < 3; ++k) {
    if (plane && k == 2) {
      o->m[2] = o->n[2] = o->mT[2] = 1;
      o->h[2] = o->hT[2] = o->hy[2] = 1.0;
      continue;
    }
    o->m[k] = g->m[k];
    o->n[k] = g->my[k];
    o->h[k] = g->h[k];
    o->mT[k] = tdef ? g->m[k] : g->mT[k];
    o->hT[k] = hdef ? g->h[k] : g->hT[k];
    if (o->m[k] < 2 || o->m[k] > (1 << 20)) return fail(MFR_EINVAL, "m[%d] = %d out of range [2, 2^20]", k, o->m[k]);
    if (o->n[k] < 2 || o->n[k] - 1 > o->m[k])
      return fail(MFR_EINVAL, "my[%d] = %d: need 2 <= my <= m + 1", k, o->n[k]);
    if (o->mT[k] < 1 || o->mT[k] > (1 << 20)) return fail(MFR_EINVAL, "mT[%d] = %d out of range", k, o->mT[k]);
    if (!(o->h[k] > 0) || !std::isfinite(o->h[k])) return fail(MFR_EINVAL, "h[%d] must be > 0", k);
    if (!(o->hT[k] > 0) || !std::isfinite(o->hT[k])) return fail(MFR_EINVAL, "hT[%d] must be > 0", k);
    o->hy[k] = o->m[k] * o->h[k] / (o->n[k] - 1);
  }
  if (g->distance != MFR_DIST_NGF && g->distance != MFR_DIST_SSD)
    return fail(MFR_EINVAL, "distance = %d: need MFR_DIST_NGF (0) or MFR_DIST_SSD (1)", (int)g->distance);
  o->dist = g->distance;
  if (g->regulariser != MFR_REG_CURVATURE && g->regulariser != MFR_REG_DIFFUSIVE && g->regulariser != MFR_REG_ELASTIC)
    return fail(MFR_EINVAL, "regulariser = %d: need MFR_REG_CURVATURE (0), MFR_REG_DIFFUSIVE (1) or MFR_REG_ELASTIC (2)",
                (int)g->regulariser);
  o->reg = g->regulariser;
  o->lame_mu = g->lame_mu;
  o->lame_lambda = g->lame_lambda;
  if (o->reg == MFR_REG_ELASTIC &&
      (!(g->lame_mu > 0) || !std::isfinite(g->lame_mu) || !std::isfinite(g->lame_lambda) ||
       !(g->lame_lambda + g->lame_mu >= 0)))
    return fail(MFR_EINVAL, "elastic regulariser: need lame_mu > 0 and lame_lambda + lame_mu >= 0");
  if (o->dist == MFR_DIST_NGF &&
      (!(g->tau > 0) || !(g->rho > 0) || !std::isfinite(g->tau) || !std::isfinite(g->rho)))
    return fail(MFR_EINVAL, "tau and rho must be > 0");
  if (!(g->alpha >= 0) || !std::isfinite(g->alpha)) return fail(MFR_EINVAL, "alpha must be >= 0");
  o->tau = g->tau;
  o->rho = g->rho;
  o->alpha = g->alpha;
  if (plane && (o->dist != MFR_DIST_NGF || o->reg != MFR_REG_CURVATURE))
    return fail(MFR_EINVAL, "two-dimensional problems take the NGF distance and the curvature regulariser");
  o->mbar = (size_t)o->m[0] * o->m[1] * o->m[2];
  o->nbar = (size_t)o->n[0] * o->n[1] * o->n[2];
  const size_t tpad = (size_t)(o->mT[0] + 4) * (o->mT[1] + 4) * (plane ? 1 : o->mT[2] + 4);
  // kernels address images, the padded template and node vectors with 32-bit byte offsets
  if (o->mbar >= (size_t)1 << 30 || 3 * o->nbar >= (size_t)1 << 30 || tpad >= (size_t)1 << 30)
    return fail(MFR_EINVAL, "problem too large: images, padded template and node vectors must stay below 2^30 elements");
  return MFR_OK;
}

// ---- lookup tables -----------------------------------------------------------
// Grid conversion along one axis: c = (a + 1/2)(n - 1)/m in exact integer
// arithmetic, lower node min(floor(c), n - 2), fraction c - lower.
std::vector<Conv1> conv_table(int m, int n) {
  std::vector<Conv1> t(m);
  const long long den = 2LL * m;
  for (int a = 0; a < m; ++a) {
    const long long num = (2LL * a + 1) * (n - 1);
    long long n0 = std::min<long long>(num / den, n - 2);
    t[a].n0 = (int)n0;
    t[a].f = (float)((double)(num - n0 * den) / (double)den);
  }
  return t;
}

// Template coordinate of voxel centres: (a + 1/2) h / hT - 1/2 = base + frac.
std::vector<Samp1> samp_table(int m, double h, double hT) {
  std::vector<Samp1> t(m);
  for (int a = 0; a < m; ++a) {
    const double q = (a + 0.5) * h / hT - 0.5;
    const double b = std::floor(q);
    t[a].base = (int)b;
    t[a].frac = (float)(q - b);
  }
  return t;
}

// Voxel range contributing to each node (lower node n-1 or n).
std::vector<Range1> node_cols(const std::vector<Conv1>& c, int n) {
  std::vector<Range1> r(n, Range1{1 << 30, -1});
  for (int a = 0; a < (int)c.size(); ++a) {
    for (int j = c[a].n0; j <= c[a].n0 + 1; ++j) {
      r[j].lo = std::min(r[j].lo, a);
      r[j].hi = std::max(r[j].hi, a);
    }
  }
  return r;
}

// Prolongation: coarse node values at the positions of the fine nodes.
std::vector<Conv1> prolong_table(int nf, double hyf, int nc, double hyc) {
  std::vector<Conv1> t(nf);
  for (int j = 0; j < nf; ++j) {
    double s = std::min(std::max(j * hyf / hyc, 0.0), (double)(nc - 1));
    int k0 = std::min((int)std::floor(s), nc - 2);
    t[j].n0 = k0;
    t[j].f = (float)(s - k0);
  }
  return t;
}

// Node blocks along x or y for the Jacobi kernel: consecutive nodes whose voxel
// rows (plus a one-voxel halo) fit into `width` columns.  Returns false if a
// single node does not fit.
bool node_blocks_xy(const std::vector<Range1>& rows, int width, std::vector<NodeBlock>* out) {
  out->clear();
  const int n = (int)rows.size();
  int lo = 0;
  while (lo < n) {
    if (rows[lo].hi - rows[lo].lo + 3 > width) return false;
    int hi = lo;
    while (hi + 1 < n && rows[hi + 1].hi - rows[lo].lo + 3 <= width) ++hi;
    out->push_back(NodeBlock{lo, hi, rows[lo].lo - 1, 0});
    lo = hi + 1;
  }
  return true;
}

// Node-plane chunks along z: `per` planes each; a0 = first voxel plane - 1,
// pad = last voxel plane of the rows touching the chunk.
std::vector<NodeBlock> node_blocks_z(const std::vector<Range1>& rows, int per) {
  std::vector<NodeBlock> out;
  const int n = (int)rows.size();
  for (int lo = 0; lo < n; lo += per) {
    const int hi = std::min(lo + per, n) - 1;
    out.push_back(NodeBlock{lo, hi, rows[lo].lo - 1, rows[hi].hi});
  }
  return out;
}

// ---- tiling -----------------------------------------------------------------

// Process-wide tile configuration (mfr_set_tile_config); initialised from the
// environment variables MFR_TILE ("BXxBY"), MFR_CHUNK and MFR_GROUPS if present.
static mfr_tile_config g_tile_cfg = [] {
  mfr_tile_config c{32, 16, 0, 0};
  if (const char* e = std::getenv("MFR_TILE")) {
    int bx = 0, by = 0;
    if (sscanf(e, "%dx%d", &bx, &by) == 2) {
      c.bx = bx;
      c.by = by;
    }
  }
  if (const char* e = std::getenv("MFR_CHUNK")) c.chunk_len = std::max(0, atoi(e));
  if (const char* e = std::getenv("MFR_GROUPS")) c.target_groups = std::max(0, atoi(e));
  return c;
}();

mfr_tile_config current_tile_config() { return g_tile_cfg; }
void set_tile_config(const mfr_tile_config& c) { g_tile_cfg = c; }

// Two-dimensional problems: work-groups of kPlaneNT pixel columns (one-column
// ring), rows marched in chunks; the node pass sees x tiles, one tile row and
// the row chunks as z chunks.
// Groups whose columns [i T - 1, i T + T] meet the columns [lo, hi] of a node's support.
static Range1 groups_touching(const Range1& cols, int T, int tiles) {
  const int lo = cols.lo < T ? 0 : (cols.lo - 1) / T;
  return Range1{lo, std::min(tiles - 1, (cols.hi + 1) / T)};
}

// The most groups (columns of width T with a one-column ring) overlapping one node's
// support, and the most chunks of `len` planes holding one node plane.
static int most_groups(const std::vector<Conv1>& c, int n, int T, int tiles) {
  int most = 1;
  for (const Range1& r : node_cols(c, n)) {
    const Range1 t = groups_touching(r, T, tiles);
    most = std::max(most, t.hi - t.lo + 1);
  }
  return most;
}
static int most_chunks(const std::vector<Conv1>& c, int n, int len) {
  int most = 1;
  for (const Range1& r : node_cols(c, n)) most = std::max(most, r.hi / len - r.lo / len + 1);
  return most;
}

static Tiling make_tiling_plane(const Geo& g, const std::vector<Conv1>& cx, const std::vector<Conv1>& cy) {
  Tiling t;
  const mfr_tile_config cfg = current_tile_config();
  t.shape = TileShape{kPlaneNT, 1};
  const int TX = kPlaneNT - 2;
  t.tiles_x = (g.m[0] + TX - 1) / TX;
  t.tiles_y = 1;
  const int target = cfg.target_groups > 0 ? cfg.target_groups : 2048;
  int chunks = std::max(1, (target + t.tiles_x - 1) / t.tiles_x);
  chunks = std::min(chunks, std::max(1, g.m[1] / 16));
  int clen = (g.m[1] + chunks - 1) / chunks;
  if (cfg.chunk_len > 0) clen = cfg.chunk_len;
  t.chunk_len = std::min(std::min(clen, g.m[1]), kMaxChunk);
  t.chunks = (g.m[1] + t.chunk_len - 1) / t.chunk_len;
  t.nxt = 0;
  t.nyt = 1;
  t.nzt = 0;
  for (int i = 0; i < t.tiles_x; ++i) {
    const int a0 = std::max(i * TX - 1, 0), a1 = std::min(i * TX + TX, g.m[0] - 1);
    t.nxt = std::max(t.nxt, cx[a1].n0 + 2 - cx[a0].n0);
  }
  for (int i = 0; i < t.chunks; ++i) {
    const int a0 = i * t.chunk_len, a1 = std::min(a0 + t.chunk_len, g.m[1]) - 1;
    t.nzt = std::max(t.nzt, cy[a1].n0 + 2 - cy[a0].n0);
  }
  t.smx = most_groups(cx, g.n[0], TX, t.tiles_x);
  t.smy = 1;
  t.smz = most_chunks(cy, g.n[1], t.chunk_len);
  // the diagonal: the same x tiles and row chunks, seen as x tiles and y tiles of
  // one plane; a chunk's node rows span the rows its dr rows' y stencils reach
  DiagTiling& d = t.dg;
  d.tiles_x = t.tiles_x;
  d.tiles_y = t.chunks;
  d.chunks = 1;
  d.chunk_len = t.chunk_len;
  d.nxt = t.nxt;
  d.nzt = 1;
  d.nyt = 0;
  for (int i = 0; i < t.chunks; ++i) {
    const int yb = i * t.chunk_len, ye = std::min(yb + t.chunk_len, g.m[1]);
    d.nyt = std::max(d.nyt, cy[std::min(ye, g.m[1] - 1)].n0 + 2 - cy[std::max(yb - 1, 0)].n0);
  }
  d.on = g.n[0] <= g.m[0] + 1 && g.n[1] <= g.m[1] + 1 && d.nxt <= kPlaneNT - 32;
  return t;
}

Tiling make_tiling(const Geo& g, const std::vector<Conv1>& cx, const std::vector<Conv1>& cy,
                   const std::vector<Conv1>& cz) {
  if (g.dim == 2) return make_tiling_plane(g, cx, cy);
  Tiling t;
  const mfr_tile_config cfg = current_tile_config();
  t.shape = TileShape{cfg.bx, cfg.by};
  const int TX = t.shape.bx - 2, TY = t.shape.by - 2;   // own columns; one-column ring
  t.tiles_x = (g.m[0] + TX - 1) / TX;
  t.tiles_y = (g.m[1] + TY - 1) / TY;
  const int xy = t.tiles_x * t.tiles_y;
  const int target = cfg.target_groups > 0 ? cfg.target_groups : 2048;
  int chunks = std::max(1, (target + xy - 1) / xy);
  chunks = std::min(chunks, std::max(1, g.m[2] / 16));
  int clen = (g.m[2] + chunks - 1) / chunks;
  if (cfg.chunk_len > 0) clen = cfg.chunk_len;
  t.chunk_len = std::min(std::min(clen, g.m[2]), kMaxChunk);
  t.chunks = (g.m[2] + t.chunk_len - 1) / t.chunk_len;
  t.nxt = t.nyt = t.nzt = 0;
  // node extent of a group's columns inside the image (own columns and ring)
  for (int i = 0; i < t.tiles_x; ++i) {
    const int a0 = std::max(i * TX - 1, 0), a1 = std::min(i * TX + TX, g.m[0] - 1);
    t.nxt = std::max(t.nxt, cx[a1].n0 + 2 - cx[a0].n0);
  }
  for (int i = 0; i < t.tiles_y; ++i) {
    const int a0 = std::max(i * TY - 1, 0), a1 = std::min(i * TY + TY, g.m[1] - 1);
    t.nyt = std::max(t.nyt, cy[a1].n0 + 2 - cy[a0].n0);
  }
  for (int i = 0; i < t.chunks; ++i) {
    const int a0 = i * t.chunk_len, a1 = std::min(a0 + t.chunk_len, g.m[2]) - 1;
    t.nzt = std::max(t.nzt, cz[a1].n0 + 2 - cz[a0].n0);
  }
  t.smx = most_groups(cx, g.n[0], TX, t.tiles_x);
  t.smy = most_groups(cy, g.n[1], TY, t.tiles_y);
  t.smz = most_chunks(cz, g.n[2], t.chunk_len);
  // the diagonal's own tiling: 2048 groups (two per CU resident, eight rounds);
  // a group's z node block spans the planes its rows' z stencils reach
  DiagTiling& d = t.dg;
  const int DX = kDiagBX - 2, DY = kDiagBY - 2;
  d.tiles_x = (g.m[0] + DX - 1) / DX;
  d.tiles_y = (g.m[1] + DY - 1) / DY;
  const int dxy = d.tiles_x * d.tiles_y;
  int dch = std::min(std::max(1, (4096 + dxy - 1) / dxy), std::max(1, g.m[2] / 16));
  d.chunk_len = std::min(std::min((g.m[2] + dch - 1) / dch, g.m[2]), kMaxChunk);
  d.chunks = (g.m[2] + d.chunk_len - 1) / d.chunk_len;
  d.nxt = d.nyt = d.nzt = 0;
  for (int i = 0; i < d.tiles_x; ++i) {
    const int a0 = std::max(i * DX - 1, 0), a1 = std::min(i * DX + DX, g.m[0] - 1);
    d.nxt = std::max(d.nxt, cx[a1].n0 + 2 - cx[a0].n0);
  }
  for (int i = 0; i < d.tiles_y; ++i) {
    const int a0 = std::max(i * DY - 1, 0), a1 = std::min(i * DY + DY, g.m[1] - 1);
    d.nyt = std::max(d.nyt, cy[a1].n0 + 2 - cy[a0].n0);
  }
  for (int i = 0; i < d.chunks; ++i) {
    const int zb = i * d.chunk_len, ze = std::min(zb + d.chunk_len, g.m[2]);
    d.nzt = std::max(d.nzt, cz[std::min(ze, g.m[2] - 1)].n0 + 2 - cz[std::max(zb - 1, 0)].n0);
  }
  d.on = g.n[0] <= g.m[0] + 1 && g.n[1] <= g.m[1] + 1 && g.n[2] <= g.m[2] + 1 &&
         d.nxt <= kDiagBX + 1 && d.nyt <= kDiagBY + 1 && d.nxt * d.nyt <= kDiagBX * kDiagBY / 2;
  return t;
}

bool valid_shape(const TileShape& s) {
  return (s.bx == 32 && s.by == 16) || (s.bx == 64 && s.by == 8) || (s.bx == 32 && s.by == 32) ||
         (s.bx == 64 && s.by == 16);
}

// ---- workspace layout ---------------------------------------------------------

Layout make_layout(const Geo& g, const Tiling& t) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const bool plane = g.dim == 2;
  const int nc = g.nc();
  L.Tp = take(sizeof(float) * (size_t)(g.mT[0] + 4) * (g.mT[1] + 4) * (plane ? 1 : g.mT[2] + 4));
  L.cx = take(sizeof(Conv1) * g.m[0]);
  L.cy = take(sizeof(Conv1) * g.m[1]);
  L.cz = take(sizeof(Conv1) * g.m[2]);
  L.sx = take(sizeof(Samp1) * g.m[0]);
  L.sy = take(sizeof(Samp1) * g.m[1]);
  L.sz = take(sizeof(Samp1) * g.m[2]);
  // node-pass tile ranges; a two-dimensional problem is seen as n[0] x 1 x n[1] nodes
  L.ntx = take(sizeof(Range1) * g.n[0]);
  L.nty = take(sizeof(Range1) * (plane ? 1 : g.n[1]));
  L.ntz = take(sizeof(Range1) * (plane ? g.n[1] : g.n[2]));
  L.orgx = take(sizeof(int) * t.tiles_x);
  L.orgy = take(sizeof(int) * t.tiles_y);
  L.orgz = take(sizeof(int) * t.chunks);
  L.rx = take(sizeof(Range1) * g.n[0]);
  L.ry = take(sizeof(Range1) * g.n[1]);
  L.rz = take(sizeof(Range1) * g.n[2]);
  L.jbx = take(sizeof(NodeBlock) * g.n[0]);
  L.jby = take(sizeof(NodeBlock) * g.n[1]);
  L.jbz = take(sizeof(NodeBlock) * g.n[2]);
  L.part = take(sizeof(float) * (size_t)t.smx * t.smy * t.smz * 3 * g.nbar);
  const DiagTiling& dg = t.dg;
  L.dntx = take(dg.on ? sizeof(Range1) * g.n[0] : 0);
  L.dnty = take(dg.on ? sizeof(Range1) * g.n[1] : 0);
  L.dntz = take(dg.on ? sizeof(Range1) * g.n[2] : 0);
  L.dorgx = take(dg.on ? sizeof(int) * dg.tiles_x : 0);
  L.dorgy = take(dg.on ? sizeof(int) * dg.tiles_y : 0);
  L.dorgz = take(dg.on ? sizeof(int) * dg.chunks : 0);
  L.dpart = take(dg.on ? sizeof(float) * (size_t)dg.grid() * 3 * dg.nzt * dg.nyt * dg.nxt : 0);
  L.red_tile = take(sizeof(double) * (size_t)t.grid());
  const size_t node_blocks = (g.nbar + kNodeBlock - 1) / kNodeBlock;
  L.n_red_node = std::max<size_t>(3 * node_blocks, 2 * 1024);   // node-pass partials (one per block) and others
  L.red_node = take(sizeof(double) * L.n_red_node);
  L.sc = take(sizeof(double) * SC_COUNT);
  L.vec = take(sizeof(float) * nc * g.nbar * 8);   // PCG r z p q diag; GN rhs, trial, direction
  L.lap = take(sizeof(float) * nc * g.nbar);       // curvature Laplacian (node pass, first half)
  L.div = take(sizeof(float) * g.nbar);           // elastic: divergence per cell of the nodal grid
  L.ctrl = take(sizeof(int) * (2 + ST_COUNT));    // device-steered CG: active flag, state; line-search flag
  L.total = o;
  return L;
}

}  // namespace mfr


namespace mfr {



// Context of a two-dimensional problem: tables, the tile kernel's parameters
// (TileParams with mz = nz = 1), the node pass's view of the n[0] x n[1] node
// grid as n[0] x 1 x n[1] (x tiles, one tile row, row chunks as z chunks; the
// clamped 7-point Laplacian with a single node along y is the 5-point one) and
// the one-thread-per-node Jacobi kernel.
static mfr_status ctx_init_plane(mfr_ctx* c, void* stream, void* ws, size_t ws_bytes) {
  const Geo& g = c->geo;
  auto cx = conv_table(g.m[0], g.n[0]);
  auto cy = conv_table(g.m[1], g.n[1]);
  c->tiling = make_tiling(g, cx, cy, cy);
  c->lay = make_layout(g, c->tiling);
  if (!ws) return fail(MFR_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(MFR_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < c->lay.total)
    return fail(MFR_ENOMEM, "workspace of %zu bytes is smaller than the required %zu", ws_bytes, c->lay.total);
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char*>(ws);
  c->R = nullptr;
  c->have_images = false;
  const Tiling& t = c->tiling;
  const int TX = kPlaneNT - 2;
  auto sx = samp_table(g.m[0], g.h[0], g.hT[0]);
  auto sy = samp_table(g.m[1], g.h[1], g.hT[1]);
  auto colx = node_cols(cx, g.n[0]), coly = node_cols(cy, g.n[1]);
  std::vector<Range1> ntx(g.n[0]), nty(1, Range1{0, 0}), ntz(g.n[1]), rx(g.n[0]), ry(g.n[1]);
  for (int i = 0; i < g.n[0]; ++i) {
    ntx[i] = groups_touching(colx[i], TX, t.tiles_x);
    rx[i] = Range1{std::max(colx[i].lo - 1, 0), std::min(colx[i].hi + 1, g.m[0] - 1)};
  }
  for (int i = 0; i < g.n[1]; ++i) {
    ntz[i] = Range1{coly[i].lo / t.chunk_len, coly[i].hi / t.chunk_len};
    ry[i] = Range1{std::max(coly[i].lo - 1, 0), std::min(coly[i].hi + 1, g.m[1] - 1)};
  }
  std::vector<int> orgx(t.tiles_x), orgy(1, 0), orgz(t.chunks);
  for (int i = 0; i < t.tiles_x; ++i) orgx[i] = cx[std::max(i * TX - 1, 0)].n0;
  for (int i = 0; i < t.chunks; ++i) orgz[i] = cy[i * t.chunk_len].n0;
  const Layout& L = c->lay;
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    return hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  HIP_TRY(up(L.cx, cx.data(), sizeof(Conv1) * cx.size()));
  HIP_TRY(up(L.cy, cy.data(), sizeof(Conv1) * cy.size()));
  HIP_TRY(up(L.sx, sx.data(), sizeof(Samp1) * sx.size()));
  HIP_TRY(up(L.sy, sy.data(), sizeof(Samp1) * sy.size()));
  HIP_TRY(up(L.ntx, ntx.data(), sizeof(Range1) * ntx.size()));
  HIP_TRY(up(L.nty, nty.data(), sizeof(Range1) * nty.size()));
  HIP_TRY(up(L.ntz, ntz.data(), sizeof(Range1) * ntz.size()));
  HIP_TRY(up(L.orgx, orgx.data(), sizeof(int) * orgx.size()));
  HIP_TRY(up(L.orgy, orgy.data(), sizeof(int) * orgy.size()));
  HIP_TRY(up(L.orgz, orgz.data(), sizeof(int) * orgz.size()));
  HIP_TRY(up(L.rx, rx.data(), sizeof(Range1) * rx.size()));
  HIP_TRY(up(L.ry, ry.data(), sizeof(Range1) * ry.size()));
  // tiled diagonal: x tiles as for the tile kernel, row chunks whose blocks hold
  // each node row, the first node row of each chunk's block
  const DiagTiling& dg = t.dg;
  std::vector<Range1> dnty, dntz(1, Range1{0, 0});
  std::vector<int> dorgy, dorgz(1, 0);
  if (dg.on) {
    dnty.resize(g.n[1]);
    dorgy.resize(t.chunks);
    std::vector<int> dyend(t.chunks);
    for (int i = 0; i < t.chunks; ++i) {
      const int yb = i * t.chunk_len, ye = std::min(yb + t.chunk_len, g.m[1]);
      dorgy[i] = cy[std::max(yb - 1, 0)].n0;
      dyend[i] = cy[std::min(ye, g.m[1] - 1)].n0 + 2;
    }
    for (int k = 0; k < g.n[1]; ++k) {
      int lo = t.chunks, hi = -1;
      for (int i = 0; i < t.chunks; ++i)
        if (dorgy[i] <= k && k < dyend[i]) {
          lo = std::min(lo, i);
          hi = std::max(hi, i);
        }
      dnty[k] = Range1{lo, hi};
    }
    HIP_TRY(up(L.dntx, ntx.data(), sizeof(Range1) * ntx.size()));
    HIP_TRY(up(L.dnty, dnty.data(), sizeof(Range1) * dnty.size()));
    HIP_TRY(up(L.dntz, dntz.data(), sizeof(Range1)));
    HIP_TRY(up(L.dorgx, orgx.data(), sizeof(int) * orgx.size()));
    HIP_TRY(up(L.dorgy, dorgy.data(), sizeof(int) * dorgy.size()));
    HIP_TRY(up(L.dorgz, dorgz.data(), sizeof(int)));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));

  TileParams& p = c->tp;
  p = TileParams{};
  p.live = nullptr;
  p.mx = g.m[0];
  p.my = g.m[1];
  p.mz = 1;
  p.nx = g.n[0];
  p.ny = g.n[1];
  p.nz = 1;
  p.nbar = (int)g.nbar;
  p.mTx = g.mT[0];
  p.mTy = g.mT[1];
  p.mTz = 1;
  p.PX = g.mT[0] + 4;
  p.PY = g.mT[1] + 4;
  p.PXY = (long long)p.PX * p.PY;
  p.ih2x = (float)(1.0 / (g.h[0] * g.h[0]));
  p.ih2y = (float)(1.0 / (g.h[1] * g.h[1]));
  p.hhx = (float)(0.5 / (g.h[0] * g.h[0]));
  p.hhy = (float)(0.5 / (g.h[1] * g.h[1]));
  p.ihTx = (float)(1.0 / g.hT[0]);
  p.ihTy = (float)(1.0 / g.hT[1]);
  p.tau2 = std::max((float)(g.tau * g.tau), FLT_MIN);
  p.rho2 = std::max((float)(g.rho * g.rho), FLT_MIN);
  p.taurho = (float)(g.tau * g.rho);
  p.Tp = at<float>(c->ws, L.Tp);
  p.Rbytes = (unsigned)(sizeof(float) * g.mbar);
  p.Tbytes = (unsigned)(sizeof(float) * (size_t)(g.mT[0] + 4) * (g.mT[1] + 4));
  p.cx = at<Conv1>(c->ws, L.cx);
  p.cy = at<Conv1>(c->ws, L.cy);
  p.sx = at<Samp1>(c->ws, L.sx);
  p.sy = at<Samp1>(c->ws, L.sy);
  p.tiles_x = t.tiles_x;
  p.tiles_y = 1;
  p.chunks = t.chunks;
  p.chunk_len = t.chunk_len;
  p.nxt = t.nxt;
  p.nyt = 1;
  p.nzt = t.nzt;
  p.part = at<float>(c->ws, L.part);
  p.smx = t.smx;
  p.smy = t.smy;
  p.smz = t.smz;
  p.red = at<double>(c->ws, L.red_tile);

  NodeParams& q = c->np;
  q = NodeParams{};
  q.nx = g.n[0];
  q.ny = 1;
  q.nz = g.n[1];
  q.nbar = (int)g.nbar;
  q.nc = 2;
  q.ihy2x = (float)(1.0 / (g.hy[0] * g.hy[0]));
  q.ihy2y = 0.0f;
  q.ihy2z = (float)(1.0 / (g.hy[1] * g.hy[1]));
  q.s_ngf = 0.0f;
  q.s_curv = (float)g.reg_scale();
  q.reg = MFR_REG_CURVATURE;
  q.div = at<float>(c->ws, L.div);
  q.tiles_x = t.tiles_x;
  q.tiles_y = 1;
  q.nxt = t.nxt;
  q.nyt = 1;
  q.nzt = t.nzt;
  q.part = p.part;
  q.smx = t.smx;
  q.smy = t.smy;
  q.smz = t.smz;
  q.ntx = at<Range1>(c->ws, L.ntx);
  q.nty = at<Range1>(c->ws, L.nty);
  q.ntz = at<Range1>(c->ws, L.ntz);
  q.orgx = at<int>(c->ws, L.orgx);
  q.orgy = at<int>(c->ws, L.orgy);
  q.orgz = at<int>(c->ws, L.orgz);
  q.red = at<double>(c->ws, L.red_node);
  q.lap = at<float>(c->ws, L.lap);
  q.live = nullptr;
  c->ctrl = at<int>(c->ws, L.ctrl);

  DiagParams& d = c->dp;
  d = DiagParams{};
  d.t = p;
  d.rx = at<Range1>(c->ws, L.rx);
  d.ry = at<Range1>(c->ws, L.ry);
  d.rz = nullptr;
  d.s_ngf = (float)g.hess_scale();
  d.s_curv = q.s_curv;
  d.ihy2x = q.ihy2x;
  d.ihy2y = q.ihy2z;
  d.ihy2z = 0.0f;
  c->jac_tiled = false;

  DiagTileParams& dt = c->dtp;
  dt = DiagTileParams{};
  dt.t = p;
  dt.t.tiles_x = dg.tiles_x;
  dt.t.tiles_y = dg.tiles_y;
  dt.t.chunks = 1;
  dt.t.chunk_len = dg.chunk_len;
  dt.t.nxt = dg.nxt;
  dt.t.nyt = dg.nyt;
  dt.t.nzt = 1;
  dt.t.part = at<float>(c->ws, L.dpart);
  dt.t.red = nullptr;
  dt.rx = d.rx;
  dt.ry = d.ry;
  dt.ntx = at<Range1>(c->ws, L.dntx);
  dt.nty = at<Range1>(c->ws, L.dnty);
  dt.ntz = at<Range1>(c->ws, L.dntz);
  dt.orgx = at<int>(c->ws, L.dorgx);
  dt.orgy = at<int>(c->ws, L.dorgy);
  dt.orgz = at<int>(c->ws, L.dorgz);
  dt.s_ngf = d.s_ngf;
  dt.s_curv = d.s_curv;
  dt.ihy2x = d.ihy2x;
  dt.ihy2y = d.ihy2y;
  dt.ihy2z = 0.0f;
  dt.plane = 1;

  c->sc = at<double>(c->ws, L.sc);
  c->red_tile = p.red;
  c->red_node = q.red;
  for (int k = 0; k < 8; ++k) c->vec[k] = at<float>(c->ws, L.vec) + (size_t)k * 2 * g.nbar;
  c->vec_blocks = (int)std::min<size_t>((2 * g.nbar + kVecBlock - 1) / kVecBlock, 1024);
  return MFR_OK;
}

mfr_status ctx_init(mfr_ctx* c, const mfr_grid* grid, void* stream, void* ws, size_t ws_bytes) {
  MFR_TRY(make_geo(grid, &c->geo));
  if (c->geo.dim == 2) return ctx_init_plane(c, stream, ws, ws_bytes);
  const Geo& g = c->geo;
  auto cx = conv_table(g.m[0], g.n[0]);
  auto cy = conv_table(g.m[1], g.n[1]);
  auto cz = conv_table(g.m[2], g.n[2]);
  c->tiling = make_tiling(g, cx, cy, cz);
  if (!valid_shape(c->tiling.shape)) return fail(MFR_EINVAL, "unsupported tile shape %dx%d", c->tiling.shape.bx, c->tiling.shape.by);
  c->lay = make_layout(g, c->tiling);
  if (!ws) return fail(MFR_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(MFR_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < c->lay.total)
    return fail(MFR_ENOMEM, "workspace of %zu bytes is smaller than the required %zu", ws_bytes, c->lay.total);
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char*>(ws);
  c->R = nullptr;
  c->have_images = false;
  const Tiling& t = c->tiling;
  const int TX = t.shape.bx - 2, TY = t.shape.by - 2;

  auto sx = samp_table(g.m[0], g.h[0], g.hT[0]);
  auto sy = samp_table(g.m[1], g.h[1], g.hT[1]);
  auto sz = samp_table(g.m[2], g.h[2], g.hT[2]);
  auto colx = node_cols(cx, g.n[0]), coly = node_cols(cy, g.n[1]), colz = node_cols(cz, g.n[2]);
  std::vector<Range1> ntx(g.n[0]), nty(g.n[1]), ntz(g.n[2]), rx(g.n[0]), ry(g.n[1]), rz(g.n[2]);
  for (int i = 0; i < g.n[0]; ++i) {
    ntx[i] = groups_touching(colx[i], TX, t.tiles_x);
    rx[i] = Range1{std::max(colx[i].lo - 1, 0), std::min(colx[i].hi + 1, g.m[0] - 1)};
  }
  for (int i = 0; i < g.n[1]; ++i) {
    nty[i] = groups_touching(coly[i], TY, t.tiles_y);
    ry[i] = Range1{std::max(coly[i].lo - 1, 0), std::min(coly[i].hi + 1, g.m[1] - 1)};
  }
  for (int i = 0; i < g.n[2]; ++i) {
    ntz[i] = Range1{colz[i].lo / t.chunk_len, colz[i].hi / t.chunk_len};
    rz[i] = Range1{std::max(colz[i].lo - 1, 0), std::min(colz[i].hi + 1, g.m[2] - 1)};
  }
  std::vector<NodeBlock> jbx, jby;
  c->jac_tiled = node_blocks_xy(rx, kJacAX, &jbx) && node_blocks_xy(ry, kJacAY, &jby);
  std::vector<NodeBlock> jbz;
  if (c->jac_tiled) {
    const int nxy = (int)(jbx.size() * jby.size());
    const int nbz = std::max(1, std::min(g.n[2], (2048 + nxy - 1) / nxy));
    jbz = node_blocks_z(rz, (g.n[2] + nbz - 1) / nbz);
  }
  std::vector<int> orgx(t.tiles_x), orgy(t.tiles_y), orgz(t.chunks);
  for (int i = 0; i < t.tiles_x; ++i) orgx[i] = cx[std::max(i * TX - 1, 0)].n0;
  for (int i = 0; i < t.tiles_y; ++i) orgy[i] = cy[std::max(i * TY - 1, 0)].n0;
  for (int i = 0; i < t.chunks; ++i) orgz[i] = cz[i * t.chunk_len].n0;

  const Layout& L = c->lay;
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    return hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  HIP_TRY(up(L.cx, cx.data(), sizeof(Conv1) * cx.size()));
  HIP_TRY(up(L.cy, cy.data(), sizeof(Conv1) * cy.size()));
  HIP_TRY(up(L.cz, cz.data(), sizeof(Conv1) * cz.size()));
  HIP_TRY(up(L.sx, sx.data(), sizeof(Samp1) * sx.size()));
  HIP_TRY(up(L.sy, sy.data(), sizeof(Samp1) * sy.size()));
  HIP_TRY(up(L.sz, sz.data(), sizeof(Samp1) * sz.size()));
  HIP_TRY(up(L.ntx, ntx.data(), sizeof(Range1) * ntx.size()));
  HIP_TRY(up(L.nty, nty.data(), sizeof(Range1) * nty.size()));
  HIP_TRY(up(L.ntz, ntz.data(), sizeof(Range1) * ntz.size()));
  HIP_TRY(up(L.orgx, orgx.data(), sizeof(int) * orgx.size()));
  HIP_TRY(up(L.orgy, orgy.data(), sizeof(int) * orgy.size()));
  HIP_TRY(up(L.orgz, orgz.data(), sizeof(int) * orgz.size()));
  HIP_TRY(up(L.rx, rx.data(), sizeof(Range1) * rx.size()));
  HIP_TRY(up(L.ry, ry.data(), sizeof(Range1) * ry.size()));
  HIP_TRY(up(L.rz, rz.data(), sizeof(Range1) * rz.size()));
  if (c->jac_tiled) {
    HIP_TRY(up(L.jbx, jbx.data(), sizeof(NodeBlock) * jbx.size()));
    HIP_TRY(up(L.jby, jby.data(), sizeof(NodeBlock) * jby.size()));
    HIP_TRY(up(L.jbz, jbz.data(), sizeof(NodeBlock) * jbz.size()));
  }
  // voxel-tiled diagonal: the groups and chunks holding each node, the first
  // node of each group's block (z: the planes its rows' z stencils reach)
  const DiagTiling& dg = t.dg;
  std::vector<Range1> dntx, dnty, dntz;
  std::vector<int> dorgx, dorgy, dorgz;
  if (dg.on) {
    const int DX = kDiagBX - 2, DY = kDiagBY - 2;
    dntx.resize(g.n[0]);
    dnty.resize(g.n[1]);
    dntz.resize(g.n[2]);
    dorgx.resize(dg.tiles_x);
    dorgy.resize(dg.tiles_y);
    dorgz.resize(dg.chunks);
    std::vector<int> dzend(dg.chunks);
    for (int i = 0; i < g.n[0]; ++i) dntx[i] = groups_touching(colx[i], DX, dg.tiles_x);
    for (int i = 0; i < g.n[1]; ++i) dnty[i] = groups_touching(coly[i], DY, dg.tiles_y);
    for (int i = 0; i < dg.tiles_x; ++i) dorgx[i] = cx[std::max(i * DX - 1, 0)].n0;
    for (int i = 0; i < dg.tiles_y; ++i) dorgy[i] = cy[std::max(i * DY - 1, 0)].n0;
    for (int i = 0; i < dg.chunks; ++i) {
      const int zb = i * dg.chunk_len, ze = std::min(zb + dg.chunk_len, g.m[2]);
      dorgz[i] = cz[std::max(zb - 1, 0)].n0;
      dzend[i] = cz[std::min(ze, g.m[2] - 1)].n0 + 2;
    }
    for (int k = 0; k < g.n[2]; ++k) {   // the chunks whose blocks hold node plane k (contiguous)
      int lo = dg.chunks, hi = -1;
      for (int i = 0; i < dg.chunks; ++i)
        if (dorgz[i] <= k && k < dzend[i]) {
          lo = std::min(lo, i);
          hi = std::max(hi, i);
        }
      dntz[k] = Range1{lo, hi};
    }
    HIP_TRY(up(L.dntx, dntx.data(), sizeof(Range1) * dntx.size()));
    HIP_TRY(up(L.dnty, dnty.data(), sizeof(Range1) * dnty.size()));
    HIP_TRY(up(L.dntz, dntz.data(), sizeof(Range1) * dntz.size()));
    HIP_TRY(up(L.dorgx, dorgx.data(), sizeof(int) * dorgx.size()));
    HIP_TRY(up(L.dorgy, dorgy.data(), sizeof(int) * dorgy.size()));
    HIP_TRY(up(L.dorgz, dorgz.data(), sizeof(int) * dorgz.size()));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));

  TileParams& p = c->tp;
  p.live = nullptr;
  p.mx = g.m[0];
  p.my = g.m[1];
  p.mz = g.m[2];
  p.nx = g.n[0];
  p.ny = g.n[1];
  p.nz = g.n[2];
  p.nbar = (int)g.nbar;
  p.mTx = g.mT[0];
  p.mTy = g.mT[1];
  p.mTz = g.mT[2];
  p.PX = g.mT[0] + 4;
  p.PY = g.mT[1] + 4;
  p.PXY = (long long)p.PX * p.PY;
  p.ih2x = (float)(1.0 / (g.h[0] * g.h[0]));
  p.ih2y = (float)(1.0 / (g.h[1] * g.h[1]));
  p.ih2z = (float)(1.0 / (g.h[2] * g.h[2]));
  p.hhx = (float)(0.5 / (g.h[0] * g.h[0]));
  p.hhy = (float)(0.5 / (g.h[1] * g.h[1]));
  p.hhz = (float)(0.5 / (g.h[2] * g.h[2]));
  p.ihTx = (float)(1.0 / g.hT[0]);
  p.ihTy = (float)(1.0 / g.hT[1]);
  p.ihTz = (float)(1.0 / g.hT[2]);
  const bool ssd = g.dist == MFR_DIST_SSD;   // tau, rho unused (and unchecked) for SSD
  p.ssd = ssd ? 1 : 0;
  p.reg = g.reg;
  p.kappa = (float)g.kappa();
  // tau^2 and rho^2 at least the smallest normal float: the NGF norms the kernels
  // take reciprocal square roots of are then never denormal
  p.tau2 = ssd ? 1.0f : std::max((float)(g.tau * g.tau), FLT_MIN);
  p.rho2 = ssd ? 1.0f : std::max((float)(g.rho * g.rho), FLT_MIN);
  p.taurho = ssd ? 1.0f : (float)(g.tau * g.rho);
  p.R = nullptr;
  p.Tp = at<float>(c->ws, L.Tp);
  p.Rbytes = (unsigned)(sizeof(float) * g.mbar);
  p.Tbytes = (unsigned)(sizeof(float) * (size_t)(g.mT[0] + 4) * (g.mT[1] + 4) * (g.mT[2] + 4));
  p.pxy24 = p.PXY < (1LL << 24) ? 1 : 0;
  p.cx = at<Conv1>(c->ws, L.cx);
  p.cy = at<Conv1>(c->ws, L.cy);
  p.cz = at<Conv1>(c->ws, L.cz);
  p.sx = at<Samp1>(c->ws, L.sx);
  p.sy = at<Samp1>(c->ws, L.sy);
  p.sz = at<Samp1>(c->ws, L.sz);
  p.tiles_x = t.tiles_x;
  p.tiles_y = t.tiles_y;
  p.chunks = t.chunks;
  p.chunk_len = t.chunk_len;
  p.nxt = t.nxt;
  p.nyt = t.nyt;
  p.nzt = t.nzt;
  p.part = at<float>(c->ws, L.part);
  p.smx = t.smx;
  p.smy = t.smy;
  p.smz = t.smz;
  p.red = at<double>(c->ws, L.red_tile);

  NodeParams& q = c->np;
  q.nx = g.n[0];
  q.ny = g.n[1];
  q.nz = g.n[2];
  q.nbar = (int)g.nbar;
  q.nc = 3;
  q.ihy2x = (float)(1.0 / (g.hy[0] * g.hy[0]));
  q.ihy2y = (float)(1.0 / (g.hy[1] * g.hy[1]));
  q.ihy2z = (float)(1.0 / (g.hy[2] * g.hy[2]));
  q.s_ngf = 0.0f;
  q.s_curv = (float)g.reg_scale();
  q.reg = g.reg;
  q.kappa = (float)g.kappa();
  q.div = at<float>(c->ws, L.div);
  q.tiles_x = t.tiles_x;
  q.tiles_y = t.tiles_y;
  q.nxt = t.nxt;
  q.nyt = t.nyt;
  q.nzt = t.nzt;
  q.part = p.part;
  q.smx = t.smx;
  q.smy = t.smy;
  q.smz = t.smz;
  q.ntx = at<Range1>(c->ws, L.ntx);
  q.nty = at<Range1>(c->ws, L.nty);
  q.ntz = at<Range1>(c->ws, L.ntz);
  q.orgx = at<int>(c->ws, L.orgx);
  q.orgy = at<int>(c->ws, L.orgy);
  q.orgz = at<int>(c->ws, L.orgz);
  q.red = at<double>(c->ws, L.red_node);
  q.lap = at<float>(c->ws, L.lap);
  q.live = nullptr;
  c->ctrl = at<int>(c->ws, L.ctrl);

  DiagParams& d = c->dp;
  d.t = p;
  d.rx = at<Range1>(c->ws, L.rx);
  d.ry = at<Range1>(c->ws, L.ry);
  d.rz = at<Range1>(c->ws, L.rz);
  d.s_ngf = (float)g.hess_scale();
  d.s_curv = q.s_curv;
  d.ihy2x = q.ihy2x;
  d.ihy2y = q.ihy2y;
  d.ihy2z = q.ihy2z;

  JacParams& jp = c->jp;
  jp.t = p;
  jp.bx = at<NodeBlock>(c->ws, L.jbx);
  jp.by = at<NodeBlock>(c->ws, L.jby);
  jp.bz = at<NodeBlock>(c->ws, L.jbz);
  jp.nbx = (int)jbx.size();
  jp.nby = (int)jby.size();
  jp.nbz = (int)jbz.size();
  jp.rx = d.rx;
  jp.ry = d.ry;
  jp.s_ngf = d.s_ngf;
  jp.s_curv = d.s_curv;
  jp.ihy2x = d.ihy2x;
  jp.ihy2y = d.ihy2y;
  jp.ihy2z = d.ihy2z;

  DiagTileParams& dt = c->dtp;
  dt = DiagTileParams{};
  dt.t = p;
  dt.t.tiles_x = dg.tiles_x;
  dt.t.tiles_y = dg.tiles_y;
  dt.t.chunks = dg.chunks;
  dt.t.chunk_len = dg.chunk_len;
  dt.t.nxt = dg.nxt;
  dt.t.nyt = dg.nyt;
  dt.t.nzt = dg.nzt;
  dt.t.part = at<float>(c->ws, L.dpart);
  dt.t.red = nullptr;
  dt.rx = d.rx;
  dt.ry = d.ry;
  dt.ntx = at<Range1>(c->ws, L.dntx);
  dt.nty = at<Range1>(c->ws, L.dnty);
  dt.ntz = at<Range1>(c->ws, L.dntz);
  dt.orgx = at<int>(c->ws, L.dorgx);
  dt.orgy = at<int>(c->ws, L.dorgy);
  dt.orgz = at<int>(c->ws, L.dorgz);
  dt.s_ngf = d.s_ngf;
  dt.s_curv = d.s_curv;
  dt.ihy2x = d.ihy2x;
  dt.ihy2y = d.ihy2y;
  dt.ihy2z = d.ihy2z;

  c->sc = at<double>(c->ws, L.sc);
  c->red_tile = p.red;
  c->red_node = q.red;
  for (int k = 0; k < 8; ++k) c->vec[k] = at<float>(c->ws, L.vec) + (size_t)k * 3 * g.nbar;
  c->vec_blocks = (int)std::min<size_t>((3 * g.nbar + kVecBlock - 1) / kVecBlock, 1024);
  return MFR_OK;
}

hipEvent_t prof_event(mfr_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipError_t enqueue_diag(mfr_ctx* c, const float* u, float* diag) {
  if (c->geo.dim == 2)
    return c->tiling.dg.on ? launch_diag_tile(c->dtp, u, diag, c->stream) : launch_plane_jacobi(c->dp, u, diag, c->stream);
  if (c->tiling.dg.on) return launch_diag_tile(c->dtp, u, diag, c->stream);
  if (c->jac_tiled) return launch_jacobi_tile(c->jp, u, diag, c->stream);
  return launch_jacobi_diag(c->dp, u, diag, c->stream);
}

// The Jacobi preconditioner of a CG solve: the exact diagonal with zero entries
// replaced by 1.
hipError_t enqueue_pcg_diag(mfr_ctx* c, const float* u, float* diag) {
  hipError_t e = enqueue_diag(c, u, diag);
  if (e != hipSuccess) return e;
  return launch_safe_diag((int)(c->geo.nc() * c->geo.nbar), diag, c->stream);
}

int node_blocks(const mfr_ctx* c) { return (int)((c->geo.nbar + kNodeBlock - 1) / kNodeBlock); }
int node_parts(const mfr_ctx* c) { return node_blocks(c); }   // one partial per block (all components)

mfr_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(MFR_EINVAL, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % 4 != 0) return fail(MFR_EINVAL, "%s is not 4-byte aligned", name);
  return MFR_OK;
}

mfr_status need_images(const mfr_ctx* c) {
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  if (!c->have_images) return fail(MFR_EINVAL, "mfr_set_images has not been called");
  return MFR_OK;
}

// The fused voxel-tile kernel of the context's dimension.
static hipError_t launch_tiles(const mfr_ctx* c, int mode, const TileParams& tp, const float* u, const float* p) {
  const Tiling& t = c->tiling;
  if (c->geo.dim == 2) return launch_plane_tile(mode, tp, u, p, t.grid(), c->stream);
  return launch_tile(t.shape, mode, tp, u, p, t.grid(), c->stream);
}

// Enqueue: D and S sums into sc[SC_D], sc[SC_S].
mfr_status enqueue_objective(mfr_ctx* c, const float* u) {
  const Tiling& t = c->tiling;
  HIP_TRY(timed(c, 0, [&] { return launch_tiles(c, MODE_OBJ, c->tp, u, nullptr); }));
  HIP_TRY(launch_sum(c->red_tile, t.grid(), c->sc + SC_D, c->stream));
  NodeParams q = c->np;
  HIP_TRY(timed(c, 4, [&] { return launch_node_pass(NP_S, q, u, nullptr, node_blocks(c), c->stream); }));
  HIP_TRY(launch_sum(c->red_node, node_blocks(c), c->sc + SC_S, c->stream));
  return MFR_OK;
}

mfr_status read_objective(mfr_ctx* c, double* J, double* D, double* S) {
  double h[SC_COUNT];
  HIP_TRY(hipMemcpyAsync(h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const double Dv = c->geo.hbar() * h[SC_D];
  const double Sv = c->geo.s_value(h[SC_S]);
  const double Jv = Dv + c->geo.alpha * Sv;
  if (J) *J = Jv;
  if (D) *D = Dv;
  if (S) *S = Sv;
  if (!std::isfinite(Jv)) return fail(MFR_ENONFINITE, "objective is not finite (D = %g, S = %g)", Dv, Sv);
  return MFR_OK;
}

mfr_status enqueue_gradient(mfr_ctx* c, const float* u, float* g) {
  const Tiling& t = c->tiling;
  HIP_TRY(timed(c, 1, [&] { return launch_tiles(c, MODE_GRAD, c->tp, u, nullptr); }));
  HIP_TRY(launch_sum(c->red_tile, t.grid(), c->sc + SC_D, c->stream));
  NodeParams q = c->np;
  q.s_ngf = (float)c->geo.grad_scale();
  HIP_TRY(timed(c, 4, [&] { return launch_node_pass(NP_GRAD, q, u, g, node_blocks(c), c->stream); }));
  HIP_TRY(launch_sum(c->red_node, node_parts(c), c->sc + SC_S, c->stream));
  return MFR_OK;
}

// q = A p; p . q partials left in red_node
mfr_status enqueue_hess_vec(mfr_ctx* c, const float* u, const float* p, float* q) {
  HIP_TRY(timed(c, 2, [&] { return launch_tiles(c, MODE_HV, c->tp, u, p); }));
  NodeParams np = c->np;
  np.s_ngf = (float)c->geo.hess_scale();
  HIP_TRY(timed(c, 4, [&] { return launch_node_pass(NP_HV, np, p, q, node_blocks(c), c->stream); }));
  return MFR_OK;
}

// CG iterations enqueued between two host checks of a device-steered solve.
constexpr int kSteerIters = 8;

// Plain or Jacobi-preconditioned CG steered on the device: alpha, beta, the
// convergence test and the iteration limit are evaluated by the CG kernels
// (the batched path's, with a table of one problem), which clear an active
// flag that turns every later kernel of the solve into a no-op.  The host
// enqueues kSteerIters iterations at a time and reads the flag once per
// batch of iterations instead of reading the scalars after every iteration;
// the solve stops at the iteration a check after every iteration would stop
// at, with the same iterate (on a breakdown, p.q <= 0, the update of that
// iteration is not applied).
mfr_status pcg_run_steered(mfr_ctx* c, const float* u, const float* b, float* s_out, const mfr_pcg_opts* o,
                           mfr_pcg_info* info, double* info_dev) {
  float* diag = nullptr;
  if (o->precond >= 1) {
    diag = c->vec[4];
    HIP_TRY(timed(c, 3, [&] { return enqueue_pcg_diag(c, u, diag); }));
  }
  VecJobs V{};
  V.n = 1;
  V.prefix[0] = 0;
  V.prefix[1] = c->vec_blocks;
  VecJob& v = V.jobs[0];
  v.r = c->vec[0];
  v.z = c->vec[1];
  v.p = c->vec[2];
  v.q = c->vec[3];
  v.s = s_out;
  v.b = b;
  v.diag = diag;
  v.sc = c->sc;
  v.state = c->ctrl + 1;
  v.red = c->red_node;
  v.red_pq = c->red_node;
  v.n_pq = node_parts(c);
  v.n3 = (int)(c->geo.nc() * c->geo.nbar);
  v.max_iter = o->max_iter;
  v.rtol = o->rtol;
  V.active_out = c->ctrl;
  HIP_TRY(launch_pcg_init_batch(V, c->stream));
  TileParams tp = c->tp;
  tp.live = c->ctrl;
  NodeParams np = c->np;
  np.s_ngf = (float)c->geo.hess_scale();
  np.live = c->ctrl;
  int done = 0, active = 1;
  if (info_dev) {
    // the whole launch sequence with no host reads (graph capture): iterations
    // after the device's convergence test has stopped the solve do nothing
    for (int i = 0; i < o->max_iter; ++i) {
      HIP_TRY(timed(c, 2, [&] { return launch_tiles(c, MODE_HV, tp, u, v.p); }));
      HIP_TRY(timed(c, 4, [&] { return launch_node_pass(NP_HV, np, v.p, v.q, node_blocks(c), c->stream); }));
      HIP_TRY(launch_pcg_alpha_batch(V, c->stream));
      HIP_TRY(launch_pcg_update_batch(V, c->stream));
      HIP_TRY(launch_pcg_beta_batch(V, c->stream));
      HIP_TRY(launch_pcg_direction_batch(V, c->stream));
    }
    HIP_TRY(launch_pcg_info_out(c->ctrl + 1, c->sc, info_dev, c->stream));
    return MFR_OK;
  }
  while (done < o->max_iter && active) {
    const int k = std::min(kSteerIters, o->max_iter - done);
    for (int i = 0; i < k; ++i) {
      HIP_TRY(timed(c, 2, [&] { return launch_tiles(c, MODE_HV, tp, u, v.p); }));
      HIP_TRY(timed(c, 4, [&] { return launch_node_pass(NP_HV, np, v.p, v.q, node_blocks(c), c->stream); }));
      HIP_TRY(launch_pcg_alpha_batch(V, c->stream));
      HIP_TRY(launch_pcg_update_batch(V, c->stream));
      HIP_TRY(launch_pcg_beta_batch(V, c->stream));
      HIP_TRY(launch_pcg_direction_batch(V, c->stream));
    }
    done += k;
    HIP_TRY(hipMemcpyAsync(&active, c->ctrl, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  double h[SC_COUNT];
  int st[ST_COUNT];
  HIP_TRY(hipMemcpyAsync(h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(st, c->ctrl + 1, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (!std::isfinite(h[SC_BB])) return fail(MFR_ENONFINITE, "right-hand side is not finite");
  mfr_pcg_info inf{st[ST_ITERS], h[SC_RELRES], st[ST_FLAG], 0};
  if (info) *info = inf;
  return MFR_OK;
}

// Flexible CG with the attached learned preconditioner, steered on the device
// like pcg_run_steered: beta = z_{k+1}.(r_{k+1} - r_k) / z_k.r_k, the
// convergence test in the kernel that forms |r|, and every kernel of the solve
// (the network's included) a no-op once the solve has stopped.  After
// fallback_iters iterations (if > 0 and the solve is still running) it continues
// as Jacobi-PCG from the current iterate with a fresh direction; the host knows
// that iteration number, so the switch is a fixed point of the launch sequence.
mfr_status pcg_run_flexible(mfr_ctx* c, const float* u, const float* b, float* s_out, const mfr_pcg_opts* o,
                            mfr_pcg_info* info) {
  if (!c->pc) return fail(MFR_EINVAL, "precond 2 needs a preconditioner attached with mfr_attach_pc");
  const int n3 = (int)(c->geo.nc() * c->geo.nbar);
  float* r = c->vec[0];
  float* z = c->vec[1];
  float* p = c->vec[2];
  float* q = c->vec[3];
  float* diag = c->vec[4];
  int* active = c->ctrl;
  int* state = c->ctrl + 1;
  HIP_TRY(timed(c, 3, [&] { return enqueue_pcg_diag(c, u, diag); }));
  VecJobs V{};
  V.n = 1;
  V.prefix[0] = 0;
  V.prefix[1] = c->vec_blocks;
  VecJob& v = V.jobs[0];
  v.r = r;
  v.z = z;
  v.p = p;
  v.q = q;
  v.s = s_out;
  v.b = b;
  v.diag = nullptr;   // start: z = r, replaced by the network below
  v.sc = c->sc;
  v.state = state;
  v.red = c->red_node;
  v.red_pq = c->red_node;
  v.n_pq = node_parts(c);
  v.n3 = n3;
  v.max_iter = o->max_iter;
  v.rtol = o->rtol;
  V.active_out = active;
  HIP_TRY(launch_pcg_init_batch(V, c->stream));
  VecJobs VJ = V;   // the Jacobi phase after a fallback
  VJ.jobs[0].diag = diag;
  double* fred = pc_red(c->pc);
  float* r_prev = pc_scratch_vec(c->pc);
  const int vb = c->vec_blocks;
  auto rz_dot = [&]() -> mfr_status {   // sc[SC_RZ] = z.r
    DotsArgs d{};
    DotsOut dout{};
    d.n = (size_t)n3;
    d.count = 1;
    d.a[0] = z;
    d.b[0] = r;
    d.live = active;
    dout.out[0] = c->sc + SC_RZ;
    HIP_TRY(launch_pc_dots(d, dout, fred, c->stream));
    return MFR_OK;
  };
  MFR_TRY(pc_begin_solve(c->pc, diag));
  MFR_TRY(pc_forward(c->pc, r, diag, z, false, nullptr, nullptr, active));
  HIP_TRY(hipMemcpyAsync(p, z, sizeof(float) * n3, hipMemcpyDeviceToDevice, c->stream));
  MFR_TRY(rz_dot());
  TileParams tp = c->tp;
  tp.live = active;
  NodeParams np = c->np;
  np.s_ngf = (float)c->geo.hess_scale();
  np.live = active;
  bool jacobi = false;
  int done = 0, act = 1;
  while (done < o->max_iter && act) {
    const int k = std::min(kSteerIters, o->max_iter - done);
    for (int i = 0; i < k; ++i) {
      const int it = done + i + 1;
      HIP_TRY(timed(c, 2, [&] { return launch_tiles(c, MODE_HV, tp, u, p); }));
      HIP_TRY(timed(c, 4, [&] { return launch_node_pass(NP_HV, np, p, q, node_blocks(c), c->stream); }));
      HIP_TRY(launch_pcg_alpha_batch(V, c->stream));
      if (jacobi) {
        HIP_TRY(launch_pcg_update_batch(VJ, c->stream));
        HIP_TRY(launch_pcg_beta_batch(VJ, c->stream));
        HIP_TRY(launch_pcg_direction_batch(VJ, c->stream));
        continue;
      }
      // s += alpha p, r_prev = r, r -= alpha q; |r|, the convergence test, the RMS scales
      HIP_TRY(launch_fpcg_update(n3, diag, p, q, s_out, r, r_prev, c->sc, c->red_node, vb, c->stream, active));
      HIP_TRY(launch_fpcg_scales(c->red_node, vb, n3, c->sc, pc_scalars(c->pc), c->stream, state, active));
      if (o->fallback_iters > 0 && it >= o->fallback_iters) {
        HIP_TRY(launch_pc_fallback(n3, r, diag, z, p, active, state, c->stream));
        MFR_TRY(rz_dot());
        jacobi = true;
        continue;
      }
      // z = M(r); the last layer leaves the partials of z.r and z.r_prev for beta
      MFR_TRY(pc_forward(c->pc, r, diag, z, true, r_prev, fred, active));
      HIP_TRY(launch_fpcg_beta_sum(fred, pc_conv_blocks(c->pc), c->sc, c->stream, active));
      HIP_TRY(launch_pcg_direction_batch(V, c->stream));
    }
    done += k;
    HIP_TRY(hipMemcpyAsync(&act, active, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  double h[SC_COUNT];
  int st[ST_COUNT];
  HIP_TRY(hipMemcpyAsync(h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(st, state, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (!std::isfinite(h[SC_BB])) return fail(MFR_ENONFINITE, "right-hand side is not finite");
  mfr_pcg_info inf{st[ST_ITERS], h[SC_RELRES], st[ST_FLAG], st[ST_FALLBACK]};
  if (info) *info = inf;
  return MFR_OK;
}

// Preconditioned CG (Sec. 2.3.1; CG from s = 0, relative recursive residual).
// precond 0 / 1: none / Jacobi (pcg_run_steered); precond 2: the attached
// learned preconditioner in flexible CG (pcg_run_flexible).
mfr_status pcg_run(mfr_ctx* c, const float* u, const float* b, float* s_out, const mfr_pcg_opts* o,
                   mfr_pcg_info* info) {
  if (o->precond == 2) return pcg_run_flexible(c, u, b, s_out, o, info);
  return pcg_run_steered(c, u, b, s_out, o, info, nullptr);
}

// One Gauss-Newton step (Sec. 2.3.1).  Vectors: vec[5] right-hand side -grad J,
// vec[6] trial point, vec[7] search direction.
mfr_status gn_step(mfr_ctx* c, float* u, const mfr_gn_opts* o, mfr_gn_info* out) {
  const int n3 = (int)(c->geo.nc() * c->geo.nbar);
  float* b = c->vec[5];
  float* trial = c->vec[6];
  float* dir = c->vec[7];
  mfr_gn_info inf{};
  MFR_TRY(enqueue_gradient(c, u, b));
  double Jv = 0.0;
  MFR_TRY(read_objective(c, &Jv, nullptr, nullptr));
  inf.J_before = Jv;
  inf.J_after = Jv;
  HIP_TRY(launch_axpy(n3, b, -2.0f, b, b, c->stream));   // b <- -grad J
  mfr_pcg_opts po{o->pcg_max, o->pcg_rtol, o->precond, o->fallback_iters, 0};
  mfr_pcg_info pinf{};
  MFR_TRY(pcg_run(c, u, b, dir, &po, &pinf));
  inf.pcg_iters = pinf.iters;
  inf.pcg_relres = pinf.relres;
  inf.pcg_flag = pinf.flag;
  // slope = grad J . s = -(b . s)
  HIP_TRY(launch_dot(n3, b, dir, c->red_node, c->vec_blocks, c->stream));
  HIP_TRY(launch_sum(c->red_node, c->vec_blocks, c->sc + SC_DOT, c->stream));
  double h[SC_COUNT];
  HIP_TRY(hipMemcpyAsync(h, c->sc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const double slope = -h[SC_DOT];
  inf.slope = slope;
  double eta = 1.0;
  for (int ls = 0; ls < o->armijo_max; ++ls) {
    HIP_TRY(launch_axpy(n3, u, (float)eta, dir, trial, c->stream));
    double Jn = 0.0;
    MFR_TRY(enqueue_objective(c, trial));
    mfr_status st = read_objective(c, &Jn, nullptr, nullptr);
    inf.ls_trials = ls + 1;
    if (st == MFR_OK && Jn <= Jv + o->armijo_c1 * eta * slope) {
      inf.accepted = 1;
      inf.eta = eta;
      inf.J_after = Jn;
      HIP_TRY(hipMemcpyAsync(u, trial, sizeof(float) * n3, hipMemcpyDeviceToDevice, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      break;
    }
    eta *= 0.5;
  }
  if (out) *out = inf;
  return MFR_OK;
}

}  // namespace mfr

extern "C" {

int mfr_abi_version(void) { return MFR_ABI_VERSION; }

const char* mfr_last_error(void) { return g_err.c_str(); }

mfr_status mfr_workspace_size(const mfr_grid* grid, size_t* bytes) {
  Geo g;
  MFR_TRY(make_geo(grid, &g));
  if (!bytes) return fail(MFR_EINVAL, "bytes is NULL");
  auto cx = conv_table(g.m[0], g.n[0]);
  auto cy = conv_table(g.m[1], g.n[1]);
  auto cz = conv_table(g.m[2], g.n[2]);
  Tiling t = make_tiling(g, cx, cy, cz);
  if (g.dim == 3 && !valid_shape(t.shape)) return fail(MFR_EINVAL, "unsupported tile shape %dx%d", t.shape.bx, t.shape.by);
  *bytes = make_layout(g, t).total;
  return MFR_OK;
}

mfr_status mfr_create(const mfr_grid* grid, void* hip_stream, void* workspace, size_t ws_bytes, mfr_ctx** out) {
  if (!out) return fail(MFR_EINVAL, "out is NULL");
  *out = nullptr;
  mfr_ctx* c = new (std::nothrow) mfr_ctx();
  if (!c) return fail(MFR_EINVAL, "host allocation failed");
  mfr_status s = ctx_init(c, grid, hip_stream, workspace, ws_bytes);
  if (s != MFR_OK) {
    delete c;
    return s;
  }
  *out = c;
  return MFR_OK;
}

void mfr_destroy(mfr_ctx* ctx) {
  // pending copies may still read host memory the context owns
  if (ctx) (void)hipStreamSynchronize(ctx->stream);
  if (ctx)
    for (mfr_pc* pc : ctx->bound_pcs) pc_release_context(pc);
  delete ctx;
}

mfr_status mfr_set_images(mfr_ctx* c, const float* R, const float* T) {
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  MFR_TRY(check_ptr(R, "R"));
  MFR_TRY(check_ptr(T, "T"));
  const Geo& g = c->geo;
  HIP_TRY(launch_pad_template(T, at<float>(c->ws, c->lay.Tp), g.mT[0], g.mT[1], g.mT[2], g.dim == 2 ? 0 : 2,
                              c->stream));
  c->R = R;
  c->tp.R = R;
  c->dp.t.R = R;
  c->jp.t.R = R;
  c->dtp.t.R = R;
  c->have_images = true;
  ++c->image_version;
  return MFR_OK;
}

mfr_status mfr_objective(mfr_ctx* c, const float* u, double* J, double* D, double* S) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(enqueue_objective(c, u));
  return read_objective(c, J, D, S);
}

mfr_status mfr_gradient(mfr_ctx* c, const float* u, double* J, float* g) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(g, "g"));
  if (g == u) return fail(MFR_EINVAL, "g must not alias u");
  MFR_TRY(enqueue_gradient(c, u, g));
  if (J) return read_objective(c, J, nullptr, nullptr);
  return MFR_OK;
}

// The scalars of the last objective or gradient into device memory.
static mfr_status objective_out(mfr_ctx* c, double* out, int count) {
  HIP_TRY(launch_objective_out(c->sc + SC_D, c->geo.hbar(), c->geo.s_mul(), c->geo.s_k(), c->geo.alpha, out, count,
                               c->stream));
  return MFR_OK;
}

mfr_status mfr_objective_async(mfr_ctx* c, const float* u, double* out) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  if (!out || reinterpret_cast<uintptr_t>(out) % 8 != 0) return fail(MFR_EINVAL, "out must be an 8-byte aligned device pointer");
  MFR_TRY(enqueue_objective(c, u));
  return objective_out(c, out, 3);
}

mfr_status mfr_gradient_async(mfr_ctx* c, const float* u, double* J, float* g) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(g, "g"));
  if (g == u) return fail(MFR_EINVAL, "g must not alias u");
  if (J && reinterpret_cast<uintptr_t>(J) % 8 != 0) return fail(MFR_EINVAL, "J must be an 8-byte aligned device pointer");
  MFR_TRY(enqueue_gradient(c, u, g));
  if (J) return objective_out(c, J, 1);
  return MFR_OK;
}

mfr_status mfr_hess_vec(mfr_ctx* c, const float* u, const float* p, float* q) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(p, "p"));
  MFR_TRY(check_ptr(q, "q"));
  if (q == u || q == p) return fail(MFR_EINVAL, "q must not alias u or p");
  return enqueue_hess_vec(c, u, p, q);
}

mfr_status mfr_jacobi_diag(mfr_ctx* c, const float* u, float* diag) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(diag, "diag"));
  HIP_TRY(timed(c, 3, [&] { return enqueue_diag(c, u, diag); }));   // the exact diagonal
  return MFR_OK;
}

mfr_status mfr_gn_step(mfr_ctx* c, float* u, const mfr_gn_opts* o, mfr_gn_info* info) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  if (!o) return fail(MFR_EINVAL, "opts is NULL");
  if (o->pcg_max < 0 || !(o->pcg_rtol >= 0) || o->precond < 0 || o->precond > 2 ||
      !(o->armijo_c1 >= 0 && o->armijo_c1 < 1) || o->armijo_max < 1 || o->fallback_iters < 0)
    return fail(MFR_EINVAL, "invalid Gauss-Newton options");
  if (o->precond == 2 && !c->pc) return fail(MFR_EINVAL, "precond 2 needs a preconditioner attached with mfr_attach_pc");
  for (int k = 5; k < 8; ++k)
    if (u == c->vec[k]) return fail(MFR_EINVAL, "u must not point into the context workspace");
  return gn_step(c, u, o, info);
}

mfr_status mfr_set_tile_config(const mfr_tile_config* cfg) {
  if (!cfg) return fail(MFR_EINVAL, "cfg is NULL");
  if (!valid_shape(TileShape{cfg->bx, cfg->by}) || cfg->chunk_len < 0 || cfg->target_groups < 0)
    return fail(MFR_EINVAL, "unsupported tile configuration %dx%d / %d / %d", cfg->bx, cfg->by, cfg->chunk_len,
                cfg->target_groups);
  set_tile_config(*cfg);
  return MFR_OK;
}

mfr_status mfr_get_tile_config(mfr_tile_config* cfg) {
  if (!cfg) return fail(MFR_EINVAL, "cfg is NULL");
  *cfg = current_tile_config();
  return MFR_OK;
}

mfr_status mfr_profile_enable(mfr_ctx* c, int32_t enable) {
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  c->prof_on = enable != 0;
  return MFR_OK;
}

mfr_status mfr_profile_read(mfr_ctx* c, mfr_profile_stats* st, int32_t reset) {
  if (!c) return fail(MFR_EINVAL, "context is NULL");
  if (!st) return fail(MFR_EINVAL, "stats is NULL");
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& p : c->prof_pending) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    c->prof_ms[p.first] += ms;
    c->prof_launches[p.first] += 1;
    c->prof_pool.push_back(p.second.first);
    c->prof_pool.push_back(p.second.second);
  }
  c->prof_pending.clear();
  for (int k = 0; k < 6; ++k) {
    st->launches[k] = c->prof_launches[k];
    st->ms[k] = c->prof_ms[k];
    if (reset) {
      c->prof_launches[k] = 0;
      c->prof_ms[k] = 0.0;
    }
  }
  return MFR_OK;
}

mfr_status mfr_pcg_solve(mfr_ctx* c, const float* u, const float* b, float* s, const mfr_pcg_opts* opts,
                         mfr_pcg_info* info) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(b, "b"));
  MFR_TRY(check_ptr(s, "s"));
  if (!opts) return fail(MFR_EINVAL, "opts is NULL");
  if (opts->max_iter < 0 || !(opts->rtol >= 0) || opts->precond < 0 || opts->precond > 2 || opts->fallback_iters < 0)
    return fail(MFR_EINVAL, "invalid PCG options");
  if (s == u || s == b) return fail(MFR_EINVAL, "s must not alias u or b");
  mfr_pcg_info inf{};
  MFR_TRY(pcg_run(c, u, b, s, opts, &inf));
  if (info) *info = inf;
  if (opts->require_converged && inf.flag == 1)
    return fail(MFR_ENOTCONV, "CG stopped after %d iterations at relative residual %g > rtol %g", inf.iters,
                inf.relres, opts->rtol);
  return MFR_OK;
}

mfr_status mfr_gn_step_async(mfr_ctx* c, float* u, const mfr_gn_opts* o, double* info) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  if (!o) return fail(MFR_EINVAL, "opts is NULL");
  if (o->pcg_max < 0 || !(o->pcg_rtol >= 0) || o->precond < 0 || o->precond > 1 ||
      !(o->armijo_c1 >= 0 && o->armijo_c1 < 1) || o->armijo_max < 1 || o->fallback_iters < 0)
    return fail(MFR_EINVAL, "invalid Gauss-Newton options (the capturable step takes precond 0 or 1)");
  for (int k = 5; k < 8; ++k)
    if (u == c->vec[k]) return fail(MFR_EINVAL, "u must not point into the context workspace");
  if (!info || reinterpret_cast<uintptr_t>(info) % 8 != 0)
    return fail(MFR_EINVAL, "info must be an 8-byte aligned device pointer");
  // the steps of gn_step, with every decision taken on the device
  const int n3 = (int)(c->geo.nc() * c->geo.nbar);
  float* b = c->vec[5];
  float* trial = c->vec[6];
  float* dir = c->vec[7];
  int* search = c->ctrl + 1 + ST_COUNT;
  const double dmul = c->geo.hbar(), smul = c->geo.s_mul(), sk = c->geo.s_k(), alpha = c->geo.alpha;
  MFR_TRY(enqueue_gradient(c, u, b));
  HIP_TRY(launch_ls_begin(c->sc + SC_D, dmul, smul, sk, alpha, search, info, c->stream));
  HIP_TRY(launch_axpy(n3, b, -2.0f, b, b, c->stream));   // b <- -grad J
  mfr_pcg_opts po{o->pcg_max, o->pcg_rtol, o->precond, 0, 0};
  MFR_TRY(pcg_run_steered(c, u, b, dir, &po, nullptr, info + 4));
  HIP_TRY(launch_dot(n3, b, dir, c->red_node, c->vec_blocks, c->stream));
  HIP_TRY(launch_sum(c->red_node, c->vec_blocks, c->sc + SC_DOT, c->stream));
  HIP_TRY(launch_ls_slope(c->sc + SC_DOT, info, c->stream));
  // Armijo trials eta = 1, 1/2, ...: each one's kernels do nothing once a step
  // length has been accepted
  TileParams tp = c->tp;
  tp.live = search;
  NodeParams q = c->np;
  q.live = search;
  double eta = 1.0;
  for (int ls = 0; ls < o->armijo_max; ++ls) {
    HIP_TRY(launch_ls_trial(n3, u, (float)eta, dir, trial, search, c->stream));
    HIP_TRY(timed(c, 0, [&] { return launch_tiles(c, MODE_OBJ, tp, trial, nullptr); }));
    HIP_TRY(launch_sum(c->red_tile, c->tiling.grid(), c->sc + SC_D, c->stream));
    HIP_TRY(timed(c, 4, [&] { return launch_node_pass(NP_S, q, trial, nullptr, node_blocks(c), c->stream); }));
    HIP_TRY(launch_sum(c->red_node, node_blocks(c), c->sc + SC_S, c->stream));
    HIP_TRY(launch_ls_check(c->sc + SC_D, dmul, smul, sk, alpha, o->armijo_c1, eta, ls, search, info, c->stream));
    eta *= 0.5;
  }
  HIP_TRY(launch_ls_commit(n3, trial, u, info, c->stream));
  return MFR_OK;
}

mfr_status mfr_pcg_solve_async(mfr_ctx* c, const float* u, const float* b, float* s, const mfr_pcg_opts* opts,
                               double* info) {
  MFR_TRY(need_images(c));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(b, "b"));
  MFR_TRY(check_ptr(s, "s"));
  if (!opts) return fail(MFR_EINVAL, "opts is NULL");
  if (opts->max_iter < 0 || !(opts->rtol >= 0) || opts->precond < 0 || opts->precond > 1)
    return fail(MFR_EINVAL, "invalid PCG options (the capturable solve takes precond 0 or 1)");
  if (opts->require_converged) return fail(MFR_EINVAL, "require_converged needs the synchronous solve");
  if (s == u || s == b) return fail(MFR_EINVAL, "s must not alias u or b");
  if (!info || reinterpret_cast<uintptr_t>(info) % 8 != 0)
    return fail(MFR_EINVAL, "info must be an 8-byte aligned device pointer");
  return pcg_run_steered(c, u, b, s, opts, nullptr, info);
}

// ---- multilevel ---------------------------------------------------------------
}  // extern "C"

namespace mfr {


mfr_status ml_levels(const mfr_grid* finest, int levels, std::vector<Level>* out, size_t* total) {
  if (levels < 1 || levels > 8) return fail(MFR_EINVAL, "levels must be in 1..8");
  std::vector<Level> L(levels);
  L[levels - 1].grid = *finest;
  MFR_TRY(make_geo(finest, &L[levels - 1].geo));
  for (int k = 0; k < 3; ++k) {   // the finest grid's template sizes made explicit (0 = same as the image)
    L[levels - 1].grid.mT[k] = L[levels - 1].geo.mT[k];
    L[levels - 1].grid.hT[k] = L[levels - 1].geo.hT[k];
  }
  for (int l = levels - 2; l >= 0; --l) {
    const Geo& f = L[l + 1].geo;
    mfr_grid g{};
    for (int k = 0; k < 3; ++k) {
      if (f.dim == 2 && k == 2) {   // a two-dimensional pyramid keeps its single cell and node along z
        g.m[2] = g.my[2] = g.mT[2] = 1;
        g.h[2] = g.hT[2] = 1.0;
        continue;
      }
      g.m[k] = (f.m[k] + 1) / 2;
      g.h[k] = 2.0 * f.h[k];
      g.my[k] = (f.n[k] - 1 + 1) / 2 + 1;
      g.mT[k] = (f.mT[k] + 1) / 2;
      g.hT[k] = 2.0 * f.hT[k];
    }
    g.tau = f.tau;
    g.rho = f.rho;
    g.alpha = f.alpha;
    g.distance = f.dist;
    g.regulariser = f.reg;
    g.lame_mu = f.lame_mu;
    g.lame_lambda = f.lame_lambda;
    L[l].grid = g;
    MFR_TRY(make_geo(&g, &L[l].geo));
  }
  size_t o = 0;
  size_t ctx_ws = 0;
  for (int l = 0; l < levels; ++l) {
    size_t b = 0;
    MFR_TRY(mfr_workspace_size(&L[l].grid, &b));
    ctx_ws = std::max(ctx_ws, b);
  }
  o = align_up(ctx_ws);
  for (int l = 0; l < levels; ++l) {
    const Geo& g = L[l].geo;
    L[l].off_R = o;
    o = align_up(o + sizeof(float) * g.mbar);
    L[l].off_T = o;
    o = align_up(o + sizeof(float) * (size_t)g.mT[0] * g.mT[1] * g.mT[2]);
    L[l].off_u = o;
    o = align_up(o + sizeof(float) * g.nc() * g.nbar);
  }
  const Geo& c = L[levels - 1].geo;  // prolongation tables of the finest level
  o = align_up(o + sizeof(Conv1) * (c.n[0] + c.n[1] + c.n[2]));
  *out = L;
  *total = o;
  return MFR_OK;
}

}  // namespace mfr

extern "C" {

mfr_status mfr_ml_workspace_size(const mfr_grid* finest, int32_t levels, size_t* bytes) {
  if (!bytes) return fail(MFR_EINVAL, "bytes is NULL");
  std::vector<Level> L;
  return ml_levels(finest, levels, &L, bytes);
}

mfr_status mfr_register_multilevel(const mfr_grid* finest, const mfr_ml_opts* o, void* hip_stream, void* workspace,
                                   size_t ws_bytes, const float* R, const float* T, float* u,
                                   mfr_ml_report* report) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!o) return fail(MFR_EINVAL, "opts is NULL");
  if (o->gn_iters < 0 || o->pcg_max < 0 || !(o->pcg_rtol >= 0) || !(o->armijo_c1 >= 0 && o->armijo_c1 < 1) ||
      o->armijo_max < 1 || o->precond < 0 || o->precond > 2 || o->fallback_iters < 0)
    return fail(MFR_EINVAL, "invalid multilevel options");
  if (o->precond == 2 && !o->pc) return fail(MFR_EINVAL, "precond 2 needs opts->pc");
  if (o->precond == 2) pc_unbind(o->pc);   // unbound whatever the outcome of the call
  MFR_TRY(check_ptr(R, "R"));
  MFR_TRY(check_ptr(T, "T"));
  MFR_TRY(check_ptr(u, "u"));
  if (o->u_init) MFR_TRY(check_ptr(o->u_init, "u_init"));
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(MFR_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  std::vector<Level> L;
  size_t need = 0;
  MFR_TRY(ml_levels(finest, o->levels, &L, &need));
  if (ws_bytes < need) return fail(MFR_ENOMEM, "workspace of %zu bytes is smaller than the required %zu", ws_bytes, need);
  const int nl = o->levels;
  if (o->precond == 2) MFR_TRY(pc_check_grid(o->pc, L[nl - 1].geo));   // before any level runs
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(workspace);
  mfr_ml_report rep{};

  // image pyramid (finest level copies the caller's images)
  const Geo& gf = L[nl - 1].geo;
  HIP_TRY(hipMemcpyAsync(ws + L[nl - 1].off_R, R, sizeof(float) * gf.mbar, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(ws + L[nl - 1].off_T, T, sizeof(float) * (size_t)gf.mT[0] * gf.mT[1] * gf.mT[2],
                         hipMemcpyDeviceToDevice, st));
  for (int l = nl - 2; l >= 0; --l) {
    const Geo& f = L[l + 1].geo;
    HIP_TRY(launch_restrict(at<float>(ws, L[l + 1].off_R), f.m[0], f.m[1], f.m[2], at<float>(ws, L[l].off_R), st));
    HIP_TRY(launch_restrict(at<float>(ws, L[l + 1].off_T), f.mT[0], f.mT[1], f.mT[2], at<float>(ws, L[l].off_T), st));
  }
  size_t ctx_ws = 0;
  for (int l = 0; l < nl; ++l) {
    size_t b = 0;
    MFR_TRY(mfr_workspace_size(&L[l].grid, &b));
    ctx_ws = std::max(ctx_ws, b);
  }
  const size_t off_ptab = align_up(L[nl - 1].off_u + sizeof(float) * gf.nc() * gf.nbar);

  double Jfinal = 0.0;
  for (int l = 0; l < nl; ++l) {
    const Geo& g = L[l].geo;
    float* ul = at<float>(ws, L[l].off_u);
    if (l == 0) {
      if (o->u_init)
        HIP_TRY(hipMemcpyAsync(ul, o->u_init, sizeof(float) * g.nc() * g.nbar, hipMemcpyDeviceToDevice, st));
      else
        HIP_TRY(launch_fill(g.nc() * g.nbar, 0.0f, ul, st));
    } else {
      const Geo& gc = L[l - 1].geo;
      auto px = prolong_table(g.n[0], g.hy[0], gc.n[0], gc.hy[0]);
      auto py = prolong_table(g.n[1], g.hy[1], gc.n[1], gc.hy[1]);
      auto pz = g.dim == 2 ? std::vector<Conv1>(1, Conv1{0, 0.0f}) : prolong_table(g.n[2], g.hy[2], gc.n[2], gc.hy[2]);
      Conv1* dt = at<Conv1>(ws, off_ptab);
      HIP_TRY(hipMemcpyAsync(dt, px.data(), sizeof(Conv1) * px.size(), hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(dt + g.n[0], py.data(), sizeof(Conv1) * py.size(), hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(dt + g.n[0] + g.n[1], pz.data(), sizeof(Conv1) * pz.size(), hipMemcpyHostToDevice, st));
      HIP_TRY(launch_prolong(at<float>(ws, L[l - 1].off_u), gc.n[0], gc.n[1], gc.n[2], ul, g.n[0], g.n[1], g.n[2],
                             dt, dt + g.n[0], dt + g.n[0] + g.n[1], g.nc(), st));
      HIP_TRY(hipStreamSynchronize(st));   // host tables must outlive the copies
    }
    mfr_ctx* c = nullptr;
    MFR_TRY(mfr_create(&L[l].grid, st, ws, ctx_ws, &c));
    struct Guard {
      mfr_ctx* c;
      ~Guard() { mfr_destroy(c); }
    } guard{c};
    MFR_TRY(mfr_set_images(c, at<float>(ws, L[l].off_R), at<float>(ws, L[l].off_T)));
    if (o->precond == 2) {   // unbound again when the level's context is destroyed
      MFR_TRY(mfr_pc_bind(o->pc, c));
      MFR_TRY(mfr_attach_pc(c, o->pc));
    }
    mfr_gn_opts go{o->pcg_max, o->pcg_rtol, o->precond, o->armijo_c1, o->armijo_max,
                   o->precond == 2 ? o->fallback_iters : 0};
    int gn_done = 0, pcg_tot = 0, status = 0;
    double Jv = 0.0;
    MFR_TRY(mfr_objective(c, ul, &Jv, nullptr, nullptr));
    rep.J_start[l] = Jv;
    for (int k = 0; k < o->gn_iters; ++k) {
      mfr_gn_info gi{};
      MFR_TRY(gn_step(c, ul, &go, &gi));
      pcg_tot += gi.pcg_iters;
      if (!gi.accepted) {
        status = MFR_ELINESEARCH;
        break;
      }
      Jv = gi.J_after;
      ++gn_done;
    }
    rep.gn_done[l] = gn_done;
    rep.pcg_total[l] = pcg_tot;
    rep.status[l] = status;
    rep.J_level[l] = Jv;
    Jfinal = Jv;
  }
  const Level& lf = L[nl - 1];
  HIP_TRY(hipMemcpyAsync(u, ws + lf.off_u, sizeof(float) * lf.geo.nc() * lf.geo.nbar, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  rep.J_final = Jfinal;
  rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (report) *report = rep;
  return MFR_OK;
}

mfr_status mfr_ml_level_grid(const mfr_grid* finest, int32_t levels, int32_t level, mfr_grid* out) {
  if (!out) return fail(MFR_EINVAL, "out is NULL");
  std::vector<Level> L;
  size_t need = 0;
  MFR_TRY(ml_levels(finest, levels, &L, &need));
  if (level < 0 || level >= levels) return fail(MFR_EINVAL, "level %d outside 0..%d", level, levels - 1);
  *out = L[level].grid;
  return MFR_OK;
}

mfr_status mfr_restrict_image(const int32_t m[3], const float* fine, float* coarse, void* hip_stream) {
  if (!m) return fail(MFR_EINVAL, "m is NULL");
  for (int k = 0; k < 3; ++k)
    if (m[k] < 1) return fail(MFR_EINVAL, "image size %d x %d x %d is invalid", m[0], m[1], m[2]);
  const size_t nf = (size_t)m[0] * m[1] * m[2];
  const size_t nc = (size_t)((m[0] + 1) / 2) * ((m[1] + 1) / 2) * ((m[2] + 1) / 2);
  if (nf * sizeof(float) >= ((size_t)1 << 40)) return fail(MFR_EINVAL, "image too large");
  MFR_TRY(check_ptr(fine, "fine"));
  MFR_TRY(check_ptr(coarse, "coarse"));
  const char* f0 = reinterpret_cast<const char*>(fine);
  const char* c0 = reinterpret_cast<const char*>(coarse);
  if (c0 < f0 + nf * sizeof(float) && f0 < c0 + nc * sizeof(float))
    return fail(MFR_EINVAL, "coarse must not overlap fine");
  HIP_TRY(launch_restrict(fine, m[0], m[1], m[2], coarse, reinterpret_cast<hipStream_t>(hip_stream)));
  return MFR_OK;
}

mfr_status mfr_prolong_workspace_size(const mfr_grid* fine, size_t* bytes) {
  if (!bytes) return fail(MFR_EINVAL, "bytes is NULL");
  Geo g;
  MFR_TRY(make_geo(fine, &g));
  *bytes = align_up(sizeof(Conv1) * (size_t)(g.n[0] + g.n[1] + g.n[2]));
  return MFR_OK;
}

mfr_status mfr_prolong(const mfr_grid* coarse, const mfr_grid* fine, const float* uc, float* uf, void* work,
                       size_t work_bytes, void* hip_stream) {
  Geo gc, gf;
  MFR_TRY(make_geo(coarse, &gc));
  MFR_TRY(make_geo(fine, &gf));
  MFR_TRY(check_ptr(uc, "uc"));
  MFR_TRY(check_ptr(uf, "uf"));
  if (!work || reinterpret_cast<uintptr_t>(work) % 256 != 0)
    return fail(MFR_EINVAL, "work must be non-NULL and 256-byte aligned");
  size_t need = 0;
  MFR_TRY(mfr_prolong_workspace_size(fine, &need));
  if (work_bytes < need) return fail(MFR_ENOMEM, "work buffer of %zu bytes is smaller than the required %zu", work_bytes, need);
  const char* a0 = reinterpret_cast<const char*>(uc);
  const char* b0 = reinterpret_cast<const char*>(uf);
  if (gc.dim != gf.dim) return fail(MFR_EINVAL, "coarse and fine grids must have the same dimension");
  const size_t vb = sizeof(float) * gf.nc();
  if (b0 < a0 + vb * gc.nbar && a0 < b0 + vb * gf.nbar) return fail(MFR_EINVAL, "uf must not overlap uc");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  auto px = prolong_table(gf.n[0], gf.hy[0], gc.n[0], gc.hy[0]);
  auto py = prolong_table(gf.n[1], gf.hy[1], gc.n[1], gc.hy[1]);
  auto pz = gf.dim == 2 ? std::vector<Conv1>(1, Conv1{0, 0.0f}) : prolong_table(gf.n[2], gf.hy[2], gc.n[2], gc.hy[2]);
  Conv1* dt = reinterpret_cast<Conv1*>(work);
  HIP_TRY(hipMemcpyAsync(dt, px.data(), sizeof(Conv1) * px.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dt + gf.n[0], py.data(), sizeof(Conv1) * py.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dt + gf.n[0] + gf.n[1], pz.data(), sizeof(Conv1) * pz.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_prolong(uc, gc.n[0], gc.n[1], gc.n[2], uf, gf.n[0], gf.n[1], gf.n[2], dt, dt + gf.n[0],
                         dt + gf.n[0] + gf.n[1], gf.nc(), st));
  HIP_TRY(hipStreamSynchronize(st));   // the host tables must outlive the copies
  return MFR_OK;
}

}  // extern "C"
