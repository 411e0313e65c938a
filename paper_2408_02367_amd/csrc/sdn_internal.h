// Internal declarations of the stodip_nufft library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stodip_nufft.h"

namespace sdn {

constexpr int kMaxW = 8;        // widest kernel supported
constexpr int kMaxCoef = 16;    // polynomial coefficients per kernel piece
constexpr int kMaxB = 64;       // coils per minibatch
constexpr int kMaxK = 8;        // subspace channels
constexpr int kMaxRadices = 12; // FFT passes per axis
constexpr int kItemCap = 2048;  // points per interpolation work item
constexpr int kSpreadCap = 8192; // list entries per spreading work item
// Per-point weight record of the spreading kernels (W even): [x W][y W] then
// [z W][first node][W - 1 zeros], two 16-byte-aligned halves of 2W floats.
constexpr int wrec_stride(int W) { return 4 * W; }

// Piecewise-polynomial Kaiser-Bessel kernel: for a point with fractional
// offset t in [0,1), the weight of its i-th node is
//   sum_d c[i][d] z^d,  z = 2t - 1.
struct KerCoef {
  float c[kMaxW][kMaxCoef];
};

// Radix decomposition of one FFT length.
struct RadixPlan {
  int L;
  int n;
  int r[kMaxRadices];
};

// Coil indices of a minibatch, passed by value to kernels.
struct CoilList {
  int idx[kMaxB];
};

// Per-axis deapodisation tables and geometry (x = 0, y = 1, z = 2).
struct Axis {
  int N;      // image length
  int nf;     // fine length
  int half;   // floor(N / 2)
  int tile;   // interpolation tile edge
  int ntile;  // interpolation tiles along the axis
  int sblk;   // spreading block edge
  int nsblk;  // spreading blocks along the axis
};

constexpr int kSpreadBlock = 8;   // spreading blocks are 8 x 8 x 8 fine cells
constexpr int kVisitOffsets = 16; // z offsets -7 .. 7 of a list entry, one key slot each

// Every status-returning path records a message through this.
sdn_status fail(sdn_status s, const std::string &msg);
sdn_status hip_check(hipError_t e, const char *what);

// ---------------------------------------------------------------- host math
double kb_beta(int W, double sigma);
double bessel_i0(double x);
double kb_phi(double u, int W, double beta);
double kb_phi_hat(double xi, int W, double beta);
int fine_size(int64_t n, double sigma, int W);
bool smooth7(int64_t n);
int kernel_ncoef(int W);
void kernel_coefficients(int W, double beta, int ncoef, KerCoef *out);
RadixPlan radix_plan(int L);
std::vector<float> deapod_inverse(int N, int nf, int W, double beta);
std::vector<float> twiddles(int L);

}  // namespace sdn

// The plan object behind the opaque handle.
struct sdn_plan_s {
  uint32_t magic;
  int device;
  sdn::Axis ax[3];          // x, y, z
  int64_t M;
  int32_t T;
  int W;
  double sigma, beta;
  int ncoef;
  sdn::KerCoef coef;
  sdn::RadixPlan rp[3];     // x, y, z
  int max_points_per_item;
  size_t budget;

  // device tables
  float *dinv[3] = {nullptr, nullptr, nullptr};   // 1/phi_hat per image index
  float2 *tw[3] = {nullptr, nullptr, nullptr};    // exp(-2 pi i m / nf)

  // points in plan (tile-sorted) order
  float4 *rec = nullptr;     // (tx, ty, tz, bits of packed l0)
  int2 *pidx = nullptr;      // (frame, original index)
  int32_t *frame_user = nullptr;  // frame per point, user order
  int4 *work = nullptr;      // interpolation items: (tile, start, count, 0)
  float *wts = nullptr;      // per point (plan order), 4W floats: x and y weights, then z
                             // weights, the packed first node's bits and W - 1 zeros
  float *wts_t = nullptr;    // the same transposed, [3W][M], then [M] packed first-node bits:
                             // consecutive points' values are contiguous (interpolation)
  int *vlist = nullptr;      // spreading lists: plan indices of the points whose support
                             // touches a spreading block, grouped by block
  int2 *vinfo = nullptr;     // per list entry, matrix-core engine only: (frame, original
                             // index) of its point, so that a value fetch needs no pidx hop
  int4 *sitems = nullptr;    // spreading items: (block, list start, count, partial slot or -1)
  int4 *splits = nullptr;    // crowded blocks: (block, first slot, slots, 0)
  int64_t nsbins = 0;        // spreading blocks
  int64_t nbins = 0, nwork = 0, max_bin = 0, nvisit = 0;
  int64_t nsitems = 0, nsplit = 0, nslots = 0;

  // workspace
  float2 *grid = nullptr;
  size_t grid_cap = 0;       // complex elements
  float2 *vecbuf = nullptr;  // image-space vectors of the iterative solver
  size_t vecbuf_cap = 0;
  double *red = nullptr;     // reduction partials and solver scalars
  size_t red_cap = 0;
  float2 *kbuf = nullptr;    // k-space scratch (residual / plain path)
  size_t kbuf_cap = 0;
  float2 *part = nullptr;    // partial tiles of split spreading items
  size_t part_cap = 0;
  double *lpart = nullptr;   // per-workgroup partial losses of a DC interpolation
  size_t lpart_cap = 0;
  unsigned *absmax = nullptr; // 4 words: largest input magnitudes of a spreading call
  int spread_engine = 0;      // SDN_SPREAD_*

  // per-stage event timing
  struct StageEvents {
    int stage;
    hipEvent_t start, stop;
  };
  int prof = 0;
  std::vector<StageEvents> prof_ev;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[SDN_NUM_STAGES] = {};
  int64_t prof_n[SDN_NUM_STAGES] = {};
};

constexpr uint32_t kPlanMagic = 0x5d4e5546u;

namespace sdn {

// ----------------------------------------------------------- kernel launchers
// (defined in the .hip files; all enqueue on `st`)
hipError_t launch_fill_zero(float2 *a, size_t n, hipStream_t st);
hipError_t launch_fill_zero_f64(double *a, size_t n, hipStream_t st);

// Image-space reductions and updates (recon.hip).  Every sum of many terms
// is two fixed-order passes (per-block partials, then one block), so
// results do not depend on scheduling.
constexpr int kDotBlocks = 1024;
// part[0 .. kDotBlocks) = partial sums of Re <a, b> over n complex elements
hipError_t launch_dot(const float2 *a, const float2 *b, size_t n, double *part, hipStream_t st);
// *out = scale * sum(part[0 .. n)) (*out += ... when accumulate); with
// scratch (kSumChunks doubles) a long sum runs in two fixed-order levels
constexpr int kSumChunks = 256;
hipError_t launch_sum(const double *part, int n, double scale, double *out, hipStream_t st,
                      double *scratch = nullptr, bool accumulate = false);
// out[j][g] = scale w[orig(j)] y[g][orig(j)], plan order, for g < groups
hipError_t launch_weighted_plan(const sdn_plan_s &p, const float2 *y, int groups, const float *w,
                                float scale, float2 *out, hipStream_t st);
// y += lam x, and part = partials of Re <x, y> (after the update)
hipError_t launch_axpy_dot(float2 *y, const float2 *x, float lam, size_t n, double *part,
                           hipStream_t st);
// r = b - g, p = r, part = partials of |r|^2
hipError_t launch_cg_start(float2 *r, float2 *p, const float2 *g, size_t n, double *part,
                           hipStream_t st);
// alpha = rs / pAp (0 when pAp <= 0): x += alpha p, r -= alpha Ap,
// part = partials of |r|^2 (after the update)
hipError_t launch_cg_xr(float2 *x, float2 *r, const float2 *p, const float2 *Ap, size_t n,
                        const double *rs, const double *pAp, double *part, hipStream_t st);
// beta = rs_new / rs (0 when rs <= 0): p = r + beta p
hipError_t launch_cg_p(float2 *p, const float2 *r, size_t n, const double *rs_new,
                       const double *rs, hipStream_t st);
// s = num / den (0 when den <= 0): x *= s, *s_out = s (when non-null)
hipError_t launch_scale_ratio(float2 *x, size_t n, const double *num, const double *den,
                              double *s_out, hipStream_t st);
// Smoothed isotropic TV of x [K][Nz][Ny][Nx]: grad (+)= lam dTV/dx when grad
// is non-null; part[0 .. tv_blocks) = partial sums of the per-voxel terms
int tv_blocks(const sdn_plan_s &p, int K);
hipError_t launch_tv(const sdn_plan_s &p, const float2 *x, int K, float eps, float lam,
                     float2 *grad, int accumulate, double *part, hipStream_t st);
// Density compensation: one Pipe-Menon update (or w = 1 when first) and
// the real parts of complex-stored weights.
hipError_t launch_dcf_step(float2 *w, const float2 *cw, int64_t M, bool first, hipStream_t st);
hipError_t launch_real_part(const float2 *w, float *out, int64_t M, hipStream_t st);

// Fine grids are channel-major: P = B K grids [p][nfz][nfy][nfx], p = b K + k.
// Forward x-pass fused with coil multiply, deapodisation and zero padding.
hipError_t launch_pre_fftx(const sdn_plan_s &p, const float2 *x, int K, const float2 *smaps,
                           const CoilList &coils, int B, float2 *grid, hipStream_t st);
// Adjoint x-pass fused with crop, deapodisation, conj coil multiply and the
// sum over coils.
hipError_t launch_post_ifftx(const sdn_plan_s &p, const float2 *grid, int K,
                             const float2 *smaps, const CoilList &coils, int B, float2 *xout,
                             int accumulate, hipStream_t st);
// Strided y or z pass over P channels; inverse = +i sign.
// axis 1 = y, 2 = z.  prune_in / prune_out: only the N image rows are read /
// written (the others are known zeros / not needed).
hipError_t launch_fft_axis(const sdn_plan_s &p, float2 *grid, int P, int axis, bool inverse,
                           bool prune_in, bool prune_out, hipStream_t st);

// Interpolation (type 2) + optional subspace mix and DC epilogue.
struct InterpArgs {
  const float2 *grid;
  int P;          // channels in the grid
  int groups;     // output rows (coils for the mix, channels otherwise)
  int kg;         // channels per group
  const float2 *V;  // [T][K] or null (no mix: kg = 1)
  float2 *y;        // [groups][M] user order (may be null in DC mode)
  // DC epilogue (dc != 0): r = rscale w (y - d) in plan order and
  // loss += w |y - d|^2, with d = 0 where d is null
  int dc;
  float rscale;
  const float2 *d;  // [groups][M] user order, or null
  const float *w;   // [M] user order, or null
  float2 *r_plan;   // [M][groups] plan order, a point's coils side by side
  double *loss;
  double *loss_part;  // interp_loss_parts(p, groups) + kSumChunks doubles of scratch
  unsigned *rmax;   // DC mode, or null: set to the largest |component| of r
                    // (as float bits), for the spreading that follows
};
hipError_t launch_interp(const sdn_plan_s &p, const InterpArgs &a, hipStream_t st);
// Per-workgroup loss partials of a DC interpolation over `groups` coils.
size_t interp_loss_parts(const sdn_plan_s &p, int groups);
size_t interp_lds_bytes(const sdn_plan_s &p);
size_t max_lds_bytes();

// Spreading (type 1) of k-space values onto groups * K channel-major fine
// grids, which it overwrites completely.  Mix mode (V given): group b is a
// coil, channel (b, k) receives conj(V[t][k]) src[b][j].  Otherwise channel
// (g, k) receives src[g K + k][j].
struct SpreadArgs {
  float2 *grid;
  float2 *part;       // >= nslots * groups * K * tile cells complex
  int groups;
  int K;
  const float2 *V;    // [T][K] or null
  const float2 *src;  // user order: [rows][M]; plan order (mix mode only):
                      // [M][groups], a point's coils side by side
  bool src_plan_order;
  bool src_max_ready; // the plan's scale word 0 already holds the largest |component|
                      // of src (written by the interpolation that produced it)
};
hipError_t launch_spread(const sdn_plan_s &p, const SpreadArgs &a, hipStream_t st);
// Ragged volumes: the interpolation / spreading of up to kMaxFusedPlans
// plans (same kernel width, coils and channels; for spreading the same
// engine) as one launch over all their work items.
constexpr int kMaxFusedPlans = 8;
hipError_t launch_interp_fused(const sdn_plan_s *const *plans, const InterpArgs *args, int n,
                               hipStream_t st);
hipError_t launch_spread_fused(const sdn_plan_s *const *plans, const SpreadArgs *args, int n,
                               hipStream_t st);

// Ragged-volume group calls with one interpolation and one spreading launch
// for all volumes (api.hip); SDN_E_UNSUPPORTED, with nothing enqueued, when
// the volumes cannot share those launches.
sdn_status group_dc_grad_fused(sdn_plan const *plans, int n, const void *const *x, int K,
                               const void *const *smaps, const int *C,
                               const int32_t *const *coil_idx, int B, const void *const *V,
                               const void *const *d, const float *const *w, double *losses,
                               void *const *grad, void *stream);
sdn_status group_forward_fused(sdn_plan const *plans, int n, const void *const *x, int K,
                               const void *const *smaps, const int *C,
                               const int32_t *const *coil_idx, int B, const void *const *V,
                               void *const *y, void *stream);
sdn_status group_adjoint_fused(sdn_plan const *plans, int n, const void *const *y, int K,
                               const void *const *smaps, const int *C,
                               const int32_t *const *coil_idx, int B, const void *const *V,
                               void *const *x_out, int accumulate, void *stream);
// Engine (SDN_SPREAD_GATHER, _MATRIX or _PLANES) of a subspace-mixing
// spreading call with K channels per group and `groups` groups (coils).
int spread_engine_for(const sdn_plan_s &p, int K, int groups);
// Automatic engine choice: the plane-split matrix spreading from this many
// (coil, channel) pairs per call.
constexpr int kPlanesFrom = 32;
size_t spread_part_elems(const sdn_plan_s &p, int groups, int K);

// Plain-path subspace mix kernels (user order).
hipError_t launch_mix_fwd(const sdn_plan_s &p, const float2 *u, const float2 *V, int K, int k,
                          float2 *y, int accumulate, hipStream_t st);
hipError_t launch_mix_adj(const sdn_plan_s &p, const float2 *r, const float2 *V, int K, int k,
                          float2 *out, hipStream_t st);

}  // namespace sdn
