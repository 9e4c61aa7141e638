// Internal declarations of libmfr: kernel parameter blocks, lookup-table
// records and the host-side launch wrappers implemented in the .hip files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mfr {

constexpr int kVecBlock = 256;
constexpr int kNodeBlock = 256;
// Longest z chunk of the voxel-tile kernel: a group keeps the per-plane tables of
// its chunk (plus two planes either side) in LDS.
constexpr int kMaxChunk = 252;
// Threads (pixel columns) of a work-group of the two-dimensional tile kernel.
constexpr int kPlaneNT = 256;

// Reads of values that an earlier kernel wrote (CG scalars, control flags, scales):
// agent-scope atomic loads are served coherently, never from a stale scalar-cache
// or L1 line (plain uniform loads may be scalar loads through the scalar cache).
__device__ __forceinline__ double ld_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_coherent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid conversion along one axis (Sec. 4.3, eq. grid_conversion): voxel index
// a lies between nodes n0 and n0 + 1 with weights (1 - f, f).
struct Conv1 {
  int n0;
  float f;
};

// Template coordinate of a voxel centre along one axis: the continuous
// template index (a + 1/2) h / hT - 1/2 split into an integer and a fraction.
struct Samp1 {
  int base;
  float frac;
};

// Inclusive index range.
struct Range1 {
  int lo;
  int hi;
};

// The three computations the fused voxel-tile kernel performs.
enum TileMode : int {
  MODE_OBJ = 0,   // sum of 1 - r_i^2
  MODE_GRAD = 1,  // dr^T r, scaled by the template derivative, transposed conversion
  MODE_HV = 2     // dr^T dr (g . P p), scaled by the template derivative, transposed conversion
};

// Node-pass variants.
enum NodeMode : int {
  NP_S = 0,     // curvature energy only
  NP_GRAD = 1,  // gather + 2 alpha hbar^y L^T L u, and the curvature energy
  NP_HV = 2     // gather + 2 alpha hbar^y L^T L p, and p . q partials
};

// Parameters of the fused voxel-tile kernel (passed by value).
struct TileParams {
  int mx, my, mz;         // image cells
  int nx, ny, nz, nbar;   // deformation nodes
  int mTx, mTy, mTz;      // template cells
  int PX, PY;             // padded template row / plane pitch (mT + 4)
  long long PXY;          // padded template plane size
  float ih2x, ih2y, ih2z; // 1 / h^2
  float hhx, hhy, hhz;    // 1 / (2 h^2)
  float ihTx, ihTy, ihTz; // 1 / hT
  float tau2, rho2, taurho;
  const float* R;         // reference [mz][my][mx]
  const float* Tp;        // padded template [mTz+4][mTy+4][mTx+4]
  unsigned Rbytes, Tbytes; // their sizes in bytes (< 2^32; buffer descriptors)
  int pxy24;              // PXY < 2^24: plane offsets by 24-bit multiplies
  const Conv1* cx;        // per-voxel conversion tables (x, y, z)
  const Conv1* cy;
  const Conv1* cz;
  const Samp1* sx;        // per-voxel template coordinates (x, y, z)
  const Samp1* sy;
  const Samp1* sz;
  int tiles_x, tiles_y, chunks, chunk_len;
  int nxt, nyt, nzt;      // node extents of one tile's partial block
  // transposed-conversion partials: slot (chunk mod smz, tile_y mod smy, tile_x
  // mod smx) holds, per component, one float per node of the grid (index of the
  // node pass), written by the one group of that slot that overlaps the node
  int smx, smy, smz;
  float* part;
  double* red;            // one float64 partial per work-group
  const int* live;        // single-problem launches: skip all work while *live == 0 (nullable)
  int ssd;                // distance: 0 NGF, 1 sum of squared differences (dr/dT = identity)
  int reg;                // regulariser: 0 curvature, 1 diffusive, 2 elastic (for the diagonal kernels)
  float kappa;            // elastic: (lambda + mu) / mu
};

// Parameters of the node pass.
struct NodeParams {
  int nx, ny, nz, nbar;
  int nc;                     // components: 3, or 2 for a two-dimensional problem (viewed as nx x 1 x ny)
  float ihy2x, ihy2y, ihy2z;  // 1 / hy^2
  float s_ngf;                // scale of the gathered voxel contributions (+-2 hbar)
  float s_curv;               // 2 alpha hbar^y (curvature) or alpha hbar^y (diffusive)
  int reg;                    // 0 curvature (L L f), 1 diffusive (-L f), 2 elastic (-L f + kappa B^T B f)
  float kappa;                // elastic: (lambda + mu) / mu
  float* div;                 // elastic: divergence per cell ((nx-1)(ny-1)(nz-1) floats), first pass
  int tiles_x, tiles_y;
  int nxt, nyt, nzt;
  int smx, smy, smz;          // partial slots per axis (see TileParams)
  const float* part;
  const Range1* ntx;          // per node index: range of x tiles / y tiles / z chunks
  const Range1* nty;
  const Range1* ntz;
  const int* orgx;            // per tile: first node index of its partial block
  const int* orgy;
  const int* orgz;
  double* red;
  float* lap;                 // 3 nbar scratch: the curvature Laplacian of the input (first pass)
  const int* live;            // single-problem launches: skip all work while *live == 0 (nullable)
};

// Parameters of the Jacobi-diagonal kernel.
struct DiagParams {
  TileParams t;
  const Range1* rx;   // per node index: voxel rows whose dr row touches the node's support
  const Range1* ry;
  const Range1* rz;
  float s_ngf;        // 2 hbar
  float s_curv;       // regulariser scale (2 alpha hbar^y curvature, alpha hbar^y diffusive)
  float ihy2x, ihy2y, ihy2z;
};

// Parameters of the voxel-tiled Jacobi diagonal: the tile kernel's tables and
// images with a tiling of its own (t.tiles_x, tiles_y, chunks, chunk_len, nxt,
// nyt, nzt and part describe it: kDiagBX x kDiagBY groups), and the node pass
// that sums the partial diagonal blocks of the tiles overlapping each node.
constexpr int kDiagBX = 32, kDiagBY = 16;
struct DiagTileParams {
  TileParams t;
  const Range1* rx;   // per node index: voxel rows whose dr row touches the node's support
  const Range1* ry;
  const Range1* ntx;  // per node index: the x tiles, y tiles and z chunks whose blocks hold it
  const Range1* nty;
  const Range1* ntz;
  const int* orgx;    // per tile / chunk: first node index of its partial block
  const int* orgy;
  const int* orgz;
  float s_ngf;        // 2 hbar (hbar for SSD)
  float s_curv;       // regulariser scale
  float ihy2x, ihy2y, ihy2z;
  int plane;          // two-dimensional problem: x tiles and row chunks (as y tiles) of kPlaneNT columns
};

// A block of nodes along one axis for the Jacobi-diagonal kernel: node range
// [lo, hi] and a0, the voxel index of the block's first column (x, y) or, for
// z, one before its first voxel plane; for z, pad holds its last voxel plane.
struct NodeBlock {
  int lo, hi, a0, pad;
};

struct JacParams {
  TileParams t;
  const NodeBlock* bx;
  const NodeBlock* by;
  const NodeBlock* bz;
  int nbx, nby, nbz;
  const Range1* rx;   // per node index: voxel rows whose dr row touches the node's support
  const Range1* ry;
  float s_ngf;        // 2 hbar
  float s_curv;       // regulariser scale (2 alpha hbar^y curvature, alpha hbar^y diffusive)
  float ihy2x, ihy2y, ihy2z;
};

// Tile shape of the voxel kernel: the work-group covers BX x BY columns; it
// owns the rows of the inner (BX-2) x (BY-2), the rest is a one-column ring.
struct TileShape {
  int bx, by;
};

// One problem of a batched launch: its kernel parameters and vectors.
struct BatchJob {
  TileParams t;
  const float* u;
  const float* p;
};

// Work list of a persistent batched launch (passed by value, so the table
// sits in kernel-argument memory): problem j owns tiles [prefix[j],
// prefix[j+1]); counter is a device int the caller zeroes before the launch;
// active (may be null) masks problems out.
constexpr int kMaxBatch = 12;
struct BatchJobs {
  BatchJob jobs[kMaxBatch];
  int prefix[kMaxBatch + 1];
  int n, total;
  int* counter;
  const int* active;
};

// Node pass of one problem in a batched launch; problem j owns node blocks
// [prefix[j], prefix[j+1]).
struct NodeJob {
  NodeParams q;
  const float* f;
  float* out;
};
struct NodeJobs {
  NodeJob jobs[kMaxBatch];
  int prefix[kMaxBatch + 1];
  int n;
  const int* active;
};

// Fixed-order sum of n partials (stride apart) into *out, one group per problem.
struct SumJob {
  const double* parts;
  int n, stride;
  double* out;
};
struct SumJobs {
  SumJob jobs[kMaxBatch];
  int n;
  const int* active;
};

// y = x + eta s for one problem.
struct AxpyJob {
  const float* x;
  const float* s;
  float* y;
  float eta;
  int n;
};
struct AxpyJobs {
  AxpyJob jobs[kMaxBatch];
  int prefix[kMaxBatch + 1];
  int n;
  const int* active;
};

// Conjugate-gradient vectors and device-side control of one problem.
// ST_MAXIT and SC_RTOL are copied from the job table by the start kernel, so
// launches captured once stay valid for later solves with other limits.
enum PcgState : int { ST_ACTIVE = 0, ST_ITERS = 1, ST_FLAG = 2, ST_MAXIT = 3, ST_FALLBACK = 4, ST_COUNT = 5 };
struct VecJob {
  float *r, *z, *p, *q, *s;
  const float* b;
  const float* diag;
  double* sc;
  int* state;
  double* red;
  const double* red_pq;
  int n_pq, n3, max_iter;
  double rtol;
};
struct VecJobs {
  VecJob jobs[kMaxBatch];
  int prefix[kMaxBatch + 1];
  int n;
  int* active_out;
};

// ---- launch wrappers (return hipError_t of the launch) ----------------------
hipError_t launch_tile(const TileShape& s, int mode, const TileParams& p, const float* u,
                       const float* pv, int grid, hipStream_t st);
// groups <= 0: as many work-groups as fit on the device at once.
hipError_t launch_tile_batch(const TileShape& s, int mode, const BatchJobs& j, int groups, hipStream_t st);
hipError_t launch_node_pass(int mode, const NodeParams& q, const float* f, float* out, int blocks,
                            hipStream_t st);
hipError_t launch_sum(const double* parts, int n, double* out, hipStream_t st);
// bz: zero border along z (2; 0 for a two-dimensional template, mz = 1)
hipError_t launch_pad_template(const float* T, float* Tp, int mx, int my, int mz, int bz, hipStream_t st);
// Two-dimensional problems (plane_tile.hip): the fused tile kernel and the exact
// Jacobi diagonal; TileParams with mz = nz = 1, y rows marched in chunks.
hipError_t launch_plane_tile(int mode, const TileParams& p, const float* u, const float* pv, int grid,
                             hipStream_t st);
hipError_t launch_plane_jacobi(const DiagParams& d, const float* u, float* diag, hipStream_t st);
hipError_t launch_jacobi_diag(const DiagParams& d, const float* u, float* diag, hipStream_t st);
hipError_t launch_jacobi_tile(const JacParams& j, const float* u, float* diag, hipStream_t st);
hipError_t launch_diag_tile(const DiagTileParams& d, const float* u, float* diag, hipStream_t st);
constexpr int kJacAX = 32, kJacAY = 32;   // voxel columns covered by one Jacobi work-group

// L-BFGS initial-matrix solve (lbfgs_kernels.hip): orthonormal DCT-II matrices
// C[d] (n_d x n_d, row k = cosine k), their transposes Ct[d], and the per-axis
// eigenvalues of the Neumann second difference (lam: x, then y, then z).
struct H0Tables {
  int n[3];
  int nc;   // components (3; 2 for a two-dimensional problem, n[2] = 1)
  const float* C[3];
  const float* Ct[3];
  const float* lam;
};
// x = (c2 L^T L + c1 L + gamma I)^{-1} v per component (L diagonal in the cosine
// basis with eigenvalue lx + ly + lz); ta, tb: scratch node vectors (x may
// alias v, not ta or tb).
hipError_t launch_h0_solve(const H0Tables& t, const float* v, float* x, float* ta, float* tb, float c2, float c1,
                           float gamma, hipStream_t st);

// PCG vector kernels.  sc: device scalars (see PcgSlot).
enum PcgSlot : int {
  SC_BB = 0, SC_RZ = 1, SC_PQ = 2, SC_RR = 3, SC_RZNEW = 4, SC_ALPHA = 5, SC_BETA = 6,
  SC_D = 8, SC_S = 9, SC_J = 10, SC_DOT = 11, SC_RELRES = 12, SC_RTOL = 13, SC_ZR = 14, SC_ZRP = 15,
  SC_COUNT = 16
};
// zero entries of a Jacobi diagonal -> 1 (the preconditioner leaves them unscaled)
hipError_t launch_safe_diag(int n3, float* d, hipStream_t st);
hipError_t launch_pcg_init(int n3, const float* b, const float* diag, float* s, float* r, float* z,
                           float* p, double* red, int blocks, hipStream_t st);
hipError_t launch_pcg_alpha(const double* red_pq, int nred, double* sc, hipStream_t st);
hipError_t launch_pcg_update(int n3, const float* diag, const float* p, const float* q, float* s,
                             float* r, float* z, const double* sc, double* red, int blocks,
                             hipStream_t st);
hipError_t launch_pcg_beta(const double* red, int nred, double* sc, hipStream_t st);
hipError_t launch_pcg_direction(int n3, const float* z, float* p, const double* sc, int blocks,
                                hipStream_t st);
hipError_t launch_pcg_init_finish(const double* red, int nred, double* sc, hipStream_t st);

// float64 partial sums of x . y, one per block (then launch_sum).
hipError_t launch_dot(int n, const float* x, const float* y, double* red, int blocks, hipStream_t st);
// y = x + eta * s (GN trial points / updates).
hipError_t launch_axpy(int n, const float* x, float eta, const float* s, float* y, hipStream_t st);
// Image restriction (2 x 2 x 2 mean, ceil(m/2) cells).
hipError_t launch_fill(size_t n, float v, float* y, hipStream_t st);
hipError_t launch_restrict(const float* fine, int mx, int my, int mz, float* coarse, hipStream_t st);
// Node-field prolongation with per-axis (lower index, fraction) tables.
// nc components; cnz = fnz = 1 for two-dimensional fields (tz is then not read).
hipError_t launch_prolong(const float* coarse, int cnx, int cny, int cnz, float* fine, int fnx,
                          int fny, int fnz, const Conv1* tx, const Conv1* ty, const Conv1* tz, int nc,
                          hipStream_t st);

// batched path
hipError_t launch_node_pass_batch(int mode, const NodeJobs& j, hipStream_t st);
hipError_t launch_sum_batch(const SumJobs& j, hipStream_t st);
hipError_t launch_zero_ints(int* p, int n, hipStream_t st);
hipError_t launch_axpy_batch(const AxpyJobs& j, hipStream_t st);
hipError_t launch_dot_batch(const VecJobs& j, hipStream_t st);
hipError_t launch_pcg_init_batch(const VecJobs& j, hipStream_t st);
hipError_t launch_pcg_alpha_batch(const VecJobs& j, hipStream_t st);
hipError_t launch_pcg_update_batch(const VecJobs& j, hipStream_t st);
hipError_t launch_pcg_beta_batch(const VecJobs& j, hipStream_t st);
hipError_t launch_pcg_direction_batch(const VecJobs& j, hipStream_t st);

// ---- learned preconditioner (cnn_kernels.hip, pc_kernels.hip) ---------------------
constexpr int kCnnLayers = 4;
constexpr int kCnnWeights = 27 * 16 * 16;                 // per layer
constexpr int kCnnLayerParams = kCnnWeights + 16;         // weights then biases
constexpr int kCnnParams = kCnnLayers * kCnnLayerParams;

// One 3x3x3 convolution launch.  x: input activations [n][16] bf16; w: [27][16][16]
// bf16.  transpose = 1 computes the backward-data product (flipped taps, in/out
// channels swapped).  Epilogue: + bias (nullable), ReLU, zero where mask <= 0
// (nullable), then any of: bf16 output y16, fp32 output y32 (both [n][16]), and
// the preconditioner output z[d][n] = r[d][n] / diag[d][n] + scale * out[d] (d < 3).
struct ConvArgs {
  int nx, ny, nz;
  const uint16_t* x;
  const uint16_t* w;
  const float* bias;
  int transpose, relu;
  int w_out_major;   // forward only: w laid out [27][16 out][16 in]
  const uint16_t* mask;
  uint16_t* y16;
  float* y32;
  float* z;
  const float* r;
  const float* diag;
  const double* scale;
  const float* rprev;   // with zred: per-group partials of z.r and z.rprev (2 per group)
  double* zred;
  const int* live;   // nullable: skip while *live == 0 (device-steered solve)
  // first layer with its input computed while staging (x null): the network
  // input of pc_features from r and diag (3 x n each), |grad R| (n) and the
  // scalars at PC_RMS_Y, PC_RMS_R, PC_RMS_D, PC_RMS_G of fsc
  const float* fr;
  const float* fdiag;
  const float* fgR;
  const double* fsc;
};

struct AdamArgs {
  float lr, beta1, beta2, eps, bc1, bc2;   // bc = 1 - beta^t
};

constexpr int kCnnMaxConvGroups = 1 << 16;
int cnn_conv_blocks(int nx, int ny, int nz);   // groups of one launch (one per tile, <= kCnnMaxConvGroups)
hipError_t launch_cnn_conv(const ConvArgs& a, hipStream_t st);

// Scalars of the learned preconditioner (device doubles).
enum PcSlot : int {
  PC_RMS_Y = 0, PC_RMS_R = 1, PC_RMS_D = 2, PC_RMS_G = 3, PC_ZR = 4, PC_ZAZ = 5, PC_YR = 6, PC_YAY = 7,
  PC_LOSS = 8, PC_CA = 9, PC_CR = 10, PC_COUNT = 16
};

// Up to four float64 dot products a_k . b_k over n floats (b_k null: a_k . a_k;
// den_k non-null: a_k / den_k elementwise), summed in a fixed order into *out[k];
// rms_scale[k] > 0 stores sqrt(sum * rms_scale[k]) instead.
struct DotsArgs {
  size_t n;
  int count;
  const float* a[4];
  const float* b[4];
  const float* den[4];
  const int* live;   // nullable: skip while *live == 0 (device-steered solve)
};
struct DotsOut {
  double* out[4];
  double rms_scale[4];
};
int pc_dots_blocks(size_t n);   // partials per product (red needs 4 x this many doubles)
hipError_t launch_pc_dots(const DotsArgs& d, const DotsOut& o, double* red, hipStream_t st);
hipError_t launch_pc_features(int n, const float* r, const float* diag, const float* gR, const double* sc,
                              uint16_t* h0, hipStream_t st, const int* live = nullptr);
hipError_t launch_pc_jacobi(int n3, const float* r, const float* diag, float* y, hipStream_t st);
// Switch of a device-steered flexible solve to Jacobi-PCG: z = r / diag, p = z,
// state[ST_FALLBACK] = 1; nothing while *live == 0.
hipError_t launch_pc_fallback(int n3, const float* r, const float* diag, float* z, float* p, const int* live,
                              int* state, hipStream_t st);
hipError_t launch_pc_loss(double* sc, hipStream_t st);
hipError_t launch_pc_grad_out(int n, const float* Az, const float* r, const double* sc, uint16_t* g16,
                              hipStream_t st);

// |grad R| restricted to the nodes (separable transposed grid conversion).
struct GmArgs {
  int mx, my, mz, nx, ny, nz;
  const float* R;
  const Conv1 *cx, *cy, *cz;
  const Range1 *rx, *ry, *rz;
  const float *wsx, *wsy, *wsz;   // per node: sum of its conversion weights along the axis
  float ih2x, ih2y, ih2z;
};
// tmp1: mz*my*nx floats, tmp2: mz*ny*nx floats, gR: nz*ny*nx floats
hipError_t launch_pc_gradmag(const GmArgs& g, float* tmp1, float* tmp2, float* gR, hipStream_t st);
// Flexible-CG update: s += alpha p, rprev = r, r -= alpha q; partials of r.r and
// (r/diag).(r/diag) per block (2 per block, `blocks` blocks).
// live (nullable): every flexible-CG kernel does nothing while *live == 0.
hipError_t launch_fpcg_update(int n3, const float* diag, const float* p, const float* q, float* s, float* r,
                              float* rprev, const double* sc, double* red, int blocks, hipStream_t st,
                              const int* live = nullptr);
// sc[SC_RR] = r.r; pc_sc[PC_RMS_R], pc_sc[PC_RMS_Y] = RMS of r and r/diag over n3 entries.
// With state (device-steered solve, state = PcgState, active = the solve's live
// flag): the iteration count, sc[SC_RELRES] and the convergence / iteration-limit
// test, which clears state[ST_ACTIVE] and *active.
hipError_t launch_fpcg_scales(const double* red, int blocks, int n3, double* sc, double* pc_sc, hipStream_t st,
                              int* state = nullptr, int* active = nullptr);
// beta from the final convolution's partials (z.r, z.rprev): beta = (zr - zrp) / sc[SC_RZ]; sc[SC_RZ] = zr
hipError_t launch_fpcg_beta_sum(const double* zred, int blocks, double* sc, hipStream_t st,
                                const int* live = nullptr);
int cnn_wgrad_groups(int nx, int ny, int nz);
// part: cnn_wgrad_groups(...) x kCnnLayerParams floats; out: kCnnLayerParams floats
hipError_t launch_cnn_wgrad(int nx, int ny, int nz, const uint16_t* x, const uint16_t* g, float* part,
                            float* out, hipStream_t st);
// w16: 2 x kCnnLayers x kCnnWeights bf16, layouts [t][in][out] then [t][out][in]
hipError_t launch_cnn_cast(float* params, uint16_t* w16, hipStream_t st);
hipError_t launch_cnn_adam(float* p, const float* g, float* m, float* v, uint16_t* w16, const AdamArgs& h,
                           hipStream_t st);

}  // namespace mfr
