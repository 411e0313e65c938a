// Plan construction: fold and quantise the trajectory, bin the points into
// fine-grid tiles and sort them tile by tile, then split crowded tiles into
// work items; build the spreading lists of the 8 x 8 x 8 blocks.
//
// The sorts are stable radix sorts keyed by bin (the points by tile and
// LDS bank class, the points of crowded tiles then by first cell, the list
// entries by block and z offset, each in a fixed order within its bin), so
// a plan, and with it every summation order of the grid kernels, depends on
// the trajectory only.
//
// The trajectory of an MRF scan is fixed for every data-consistency step of
// the reconstruction (Sec. 3: thousands of iterations over one scan), so
// this runs once and everything per-step reads the sorted records.
#include <algorithm>
#include <cmath>
#include <cstring>

#include <hipcub/hipcub.hpp>

#include "nodes.h"
#include "sdn_internal.h"

namespace sdn {
const char *last_error();
}

using namespace sdn;

namespace {

constexpr float kMaxAbsCoord = 1048576.0f;   // 2^20 radians

struct FoldGeom {
  int nf[3];
  int tile[3];
  int ntile[3];
  int W;
  int T;
};

// Residue classes of a point's first tile cell in the interpolation
// kernel's LDS copy of the tile (pitches bx + W - 1 and by + W - 1, 8-byte
// cells).  gfx950 serves an 8-byte LDS read to 32 lanes at a time from 64
// four-byte banks, so 32 consecutive cells cover the banks once.
constexpr int kBankClasses = 32;
constexpr int kDenseCellBits = 15;   // tile cells < 2^15 (an LDS tile holds at most 20480)

// One thread per point.  Fine coordinate s = k nf / (2 pi) in FP64; the W
// nodes of the point are l0 .. l0+W-1 with l0 = floor(s - W/2) + 1 (the
// half-open rule s - W/2 < l <= s + W/2) and fractional offset
// t = (s - W/2) - floor(s - W/2) in [0, 1).  l0 is wrapped into [0, nf),
// which is exact because the fine grid is periodic.
__global__ void k_fold(const float *__restrict__ traj, int M, FoldGeom g,
                       const int32_t *__restrict__ frame, int *__restrict__ key,
                       float4 *__restrict__ rec, int *__restrict__ count, int *__restrict__ bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int l0[3];
  float t[3];
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float k = traj[3 * (size_t)j + d];
    if (!(fabsf(k) <= kMaxAbsCoord)) ok = false;   // also catches NaN
    const double s = (double)k * ((double)g.nf[d] / (2.0 * M_PI));
    const double a = s - 0.5 * g.W;
    const double fl = floor(a);
    t[d] = (float)(a - fl);
    double l = fl + 1.0;
    l -= (double)g.nf[d] * floor(l / (double)g.nf[d]);
    int li = (int)l;
    if (li >= g.nf[d]) li -= g.nf[d];
    if (li < 0) li += g.nf[d];
    l0[d] = li;
  }
  if (frame) {
    const int f = frame[j];
    if (f < 0 || f >= g.T) atomicOr(bad, 2);
  }
  if (!ok) {
    atomicOr(bad, 1);
    l0[0] = l0[1] = l0[2] = 0;
    t[0] = t[1] = t[2] = 0.f;
  }
  const int tx = l0[0] / g.tile[0], ty = l0[1] / g.tile[1], tz = l0[2] / g.tile[2];
  const int kk = (tz * g.ntile[1] + ty) * g.ntile[0] + tx;
  const int px = g.tile[0] + g.W - 1, py = g.tile[1] + g.W - 1;
  const int cell = ((l0[2] - tz * g.tile[2]) * py + (l0[1] - ty * g.tile[1])) * px +
                   (l0[0] - tx * g.tile[0]);
  const int kc = kk * kBankClasses + (cell & (kBankClasses - 1));
  key[j] = kc;
  const unsigned packed = (unsigned)l0[0] | ((unsigned)l0[1] << 10) | ((unsigned)l0[2] << 20);
  rec[j] = make_float4(t[0], t[1], t[2], __uint_as_float(packed));
  atomicAdd(&count[kc], 1);
}

__global__ void k_iota(int *__restrict__ v, int M) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M) v[j] = j;
}

// Plan order.  The sort leaves the points of a tile grouped by bank class
// (original order within a class); the i-th point of class c then goes to
// round i of a round-robin over the tile's classes:
//   pos = sum_c' min(n_c', i) + #{c' < c : n_c' > i},
// so that consecutive points mostly differ in class.
__global__ void k_place(const unsigned *__restrict__ skey, const int *__restrict__ order,
                        const float4 *__restrict__ rec_tmp, const int32_t *__restrict__ frame,
                        int M, const int *__restrict__ tile_start,
                        const int *__restrict__ class_count, float4 *__restrict__ rec,
                        int2 *__restrict__ pidx) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= M) return;
  const unsigned kv = skey[s];
  const int t = (int)(kv / kBankClasses), c = (int)(kv % kBankClasses);
  const int *n = class_count + (size_t)t * kBankClasses;
  int before = 0;
  for (int q = 0; q < c; ++q) before += n[q];
  const int i = s - tile_start[t] - before;
  int pos = 0;
  for (int q = 0; q < kBankClasses; ++q) pos += min(n[q], i) + (q < c && n[q] > i ? 1 : 0);
  const int dst = tile_start[t] + pos;
  const int j = order[s];
  rec[dst] = rec_tmp[j];
  pidx[dst] = make_int2(frame ? frame[j] : 0, j);
}

// Crowded tiles (at least half as many points as the tile has cells) are
// reordered by first cell after the round-robin: their points pile onto few
// cells, so classes run out early and the rounds stop lining up with the
// 32-lane groups, while 32 consecutive points in cell order span at most 32
// consecutive cells unless they are spread thin (lanes that read one cell
// share the read).  The points of the crowded tiles form one compact array,
// tile after tile; dense tile d holds compact entries doff[d] .. doff[d+1]-1
// and plan positions dstart[d] onward.
__device__ __forceinline__ int dense_tile_of(const int *doff, int nd, int i) {
  int lo = 0, hi = nd;   // largest d with doff[d] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (doff[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_dense_keys(const float4 *__restrict__ rec, FoldGeom g,
                             const int *__restrict__ dtile, const int *__restrict__ dstart,
                             const int *__restrict__ doff, int nd, int md, unsigned *__restrict__ key,
                             int *__restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= md) return;
  const int d = dense_tile_of(doff, nd, i);
  const int j = dstart[d] + (i - doff[d]);
  const unsigned u = __float_as_uint(rec[j].w);
  const int lx = (int)(u & 1023u), ly = (int)((u >> 10) & 1023u), lz = (int)((u >> 20) & 1023u);
  const int b = dtile[d];
  const int tx = b % g.ntile[0], ty = (b / g.ntile[0]) % g.ntile[1], tz = b / (g.ntile[0] * g.ntile[1]);
  const int px = g.tile[0] + g.W - 1, py = g.tile[1] + g.W - 1;
  const int cell = ((lz - tz * g.tile[2]) * py + (ly - ty * g.tile[1])) * px + (lx - tx * g.tile[0]);
  key[i] = ((unsigned)d << kDenseCellBits) | (unsigned)cell;
  val[i] = j;
}

// gather the sorted points (a copy), then write them back to their tiles' ranges
__global__ void k_dense_gather(const float4 *__restrict__ rec, const int2 *__restrict__ pidx,
                               const int *__restrict__ src, int md, float4 *__restrict__ rec_out,
                               int2 *__restrict__ pidx_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= md) return;
  rec_out[i] = rec[src[i]];
  pidx_out[i] = pidx[src[i]];
}

__global__ void k_dense_put(const float4 *__restrict__ rec_in, const int2 *__restrict__ pidx_in,
                            const int *__restrict__ dstart, const int *__restrict__ doff, int nd,
                            int md, float4 *__restrict__ rec, int2 *__restrict__ pidx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= md) return;
  const int d = dense_tile_of(doff, nd, i);
  const int j = dstart[d] + (i - doff[d]);
  rec[j] = rec_in[i];
  pidx[j] = pidx_in[i];
}

// Tiles of one axis touched by the W nodes l0 .. l0+W-1 (mod nf), in order.
__device__ __forceinline__ int axis_tiles(int l0, int W, int nf, int b, int (&t)[8]) {
  int n = 0, prev = -1;
  for (int i = 0; i < W; ++i) {
    int pos = l0 + i;
    if (pos >= nf) pos -= nf;
    const int tt = pos / b;
    if (tt != prev) {
      t[n++] = tt;
      prev = tt;
    }
  }
  if (n > 1 && t[n - 1] == t[0]) --n;
  return n;
}

// Spreading-list entries of one point.  Along x and y a point is listed
// under every block its W nodes touch.  Along z the entry also fixes the
// offset d of the first node against the block (register slot c = d + az
// for node az): d = e or d = e - nf with e = (l0 - oz) mod nf, whichever
// puts a node inside the block; on grids shorter than a block plus the
// kernel both can (a support that wraps onto both ends of the block), and
// the point is listed twice, once per side, each entry covering its own
// nodes.  Entries for the second form carry the complemented index.
struct VisitZ {
  int n;
  int blk[4];
  int d[4];
  bool neg[4];
};

__device__ __forceinline__ void visit_z(int l0, int W, int nf, VisitZ &v) {
  int t[8];
  const int nt = axis_tiles(l0, W, nf, kSpreadBlock, t);
  v.n = 0;
  for (int a = 0; a < nt; ++a) {
    const int oz = t[a] * kSpreadBlock;
    const int bw = min(kSpreadBlock, nf - oz);
    int e = l0 - oz;
    e += e < 0 ? nf : 0;
    if (e < bw) {
      v.blk[v.n] = t[a];
      v.d[v.n] = e;
      v.neg[v.n++] = false;
    }
    if (e - nf > -W) {
      v.blk[v.n] = t[a];
      v.d[v.n] = e - nf;
      v.neg[v.n++] = true;
    }
  }
}

// Pass 1: entries per point and per block.
__global__ void k_visit_count(const float4 *__restrict__ rec, int M, FoldGeom g,
                              int *__restrict__ per_block, int *__restrict__ per_point) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const unsigned u = __float_as_uint(rec[j].w);
  int tx[8], ty[8];
  const int nx = axis_tiles((int)(u & 1023u), g.W, g.nf[0], kSpreadBlock, tx);
  const int ny = axis_tiles((int)((u >> 10) & 1023u), g.W, g.nf[1], kSpreadBlock, ty);
  VisitZ vz;
  visit_z((int)((u >> 20) & 1023u), g.W, g.nf[2], vz);
  for (int a = 0; a < vz.n; ++a)
    for (int c = 0; c < ny; ++c)
      for (int i = 0; i < nx; ++i)
        atomicAdd(&per_block[(vz.blk[a] * g.ntile[1] + ty[c]) * g.ntile[0] + tx[i]], 1);
  per_point[j] = vz.n * ny * nx;
}

// (frame, original index) of every list entry's point, in list order.
__global__ void k_visit_info(const int *__restrict__ vlist, int n, const int2 *__restrict__ pidx,
                             int2 *__restrict__ vinfo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int raw = vlist[i];
  vinfo[i] = pidx[raw < 0 ? ~raw : raw];
}

// Pass 2: (block, offset) key and entry of every visit, at the point's
// position of the exclusive scan of pass 1 (so in plan order).
__global__ void k_visit_pairs(const float4 *__restrict__ rec, int M, FoldGeom g,
                              const int *__restrict__ pos, unsigned *__restrict__ key,
                              int *__restrict__ val) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const unsigned u = __float_as_uint(rec[j].w);
  int tx[8], ty[8];
  const int nx = axis_tiles((int)(u & 1023u), g.W, g.nf[0], kSpreadBlock, tx);
  const int ny = axis_tiles((int)((u >> 10) & 1023u), g.W, g.nf[1], kSpreadBlock, ty);
  VisitZ vz;
  visit_z((int)((u >> 20) & 1023u), g.W, g.nf[2], vz);
  int o = pos[j];
  for (int a = 0; a < vz.n; ++a)
    for (int c = 0; c < ny; ++c)
      for (int i = 0; i < nx; ++i) {
        const unsigned blk = (unsigned)((vz.blk[a] * g.ntile[1] + ty[c]) * g.ntile[0] + tx[i]);
        key[o] = blk * kVisitOffsets + (unsigned)(vz.d[a] + kVisitOffsets / 2 - 1);
        val[o++] = vz.neg[a] ? ~j : j;
      }
}

int key_bits(uint64_t nkeys) {
  int b = 1;
  while (b < 32 && (1ull << b) < nkeys) ++b;
  return b;
}

// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits.
template <typename KT>
sdn_status sort_pairs(const KT *kin, KT *kout, const int *vin, int *vout, int n, int bits,
                      hipStream_t st) {
  size_t tmp_bytes = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, kin, kout, vin, vout, n, 0, bits,
                                         st) != hipSuccess)
    return fail(SDN_E_HIP, "plan sort: temporary size query failed");
  void *tmp = nullptr;
  if (hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16)) != hipSuccess)
    return fail(SDN_E_NOMEM, "plan sort: no device memory for the sort");
  sdn_status s = hip_check(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin,
                                                              vout, n, 0, bits, st),
                           "plan sort");
  if (s == SDN_OK) s = hip_check(hipStreamSynchronize(st), "plan sync");
  (void)hipFree(tmp);
  return s;
}

sdn_status exclusive_sum(const int *in, int *out, int n, hipStream_t st) {
  size_t tmp_bytes = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, in, out, n, st) != hipSuccess)
    return fail(SDN_E_HIP, "plan scan: temporary size query failed");
  void *tmp = nullptr;
  if (hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16)) != hipSuccess)
    return fail(SDN_E_NOMEM, "plan scan: no device memory for the scan");
  sdn_status s = hip_check(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out, n, st),
                           "plan scan");
  if (s == SDN_OK) s = hip_check(hipStreamSynchronize(st), "plan sync");
  (void)hipFree(tmp);
  return s;
}

// Kernel weights of every point (plan order), evaluated once per plan with
// the same polynomial the grid kernels use.
// Both layouts: per point (spreading reads one scattered point per lane) and
// transposed (interpolation reads consecutive points per lane).
template <int W, int NC>
__global__ void k_weights(const float4 *__restrict__ rec, int M, KerCoef kc,
                          float *__restrict__ wts, float *__restrict__ wts_t) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const float4 r = rec[j];
  float w[W];
  float *o = wts + (size_t)j * wrec_stride(W);
  const float tc[3] = {r.x, r.y, r.z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    axis_weights<W, NC>(tc[d], kc, w);
#pragma unroll
    for (int i = 0; i < W; ++i) {
      o[(d < 2 ? d * W : 2 * W) + i] = w[i];
      wts_t[(size_t)(d * W + i) * M + j] = w[i];
    }
  }
  o[3 * W] = r.w;
#pragma unroll
  for (int i = 3 * W + 1; i < wrec_stride(W); ++i) o[i] = 0.f;
  wts_t[(size_t)3 * W * M + j] = r.w;
}

void free_plan_memory(sdn_plan_s *p) {
  for (auto &r : p->prof_ev) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  p->prof_ev.clear();
  for (auto e : p->ev_pool) (void)hipEventDestroy(e);
  p->ev_pool.clear();
  for (int d = 0; d < 3; ++d) {
    if (p->dinv[d]) (void)hipFree(p->dinv[d]);
    if (p->tw[d]) (void)hipFree(p->tw[d]);
    p->dinv[d] = nullptr;
    p->tw[d] = nullptr;
  }
  if (p->absmax) (void)hipFree(p->absmax);
  p->absmax = nullptr;
  if (p->rec) (void)hipFree(p->rec);
  if (p->pidx) (void)hipFree(p->pidx);
  if (p->frame_user) (void)hipFree(p->frame_user);
  if (p->work) (void)hipFree(p->work);
  if (p->vlist) (void)hipFree(p->vlist);
  if (p->vinfo) (void)hipFree(p->vinfo);
  p->vinfo = nullptr;
  if (p->wts) (void)hipFree(p->wts);
  if (p->wts_t) (void)hipFree(p->wts_t);
  p->wts = nullptr;
  p->wts_t = nullptr;
  if (p->sitems) (void)hipFree(p->sitems);
  if (p->splits) (void)hipFree(p->splits);
  if (p->part) (void)hipFree(p->part);
  if (p->lpart) (void)hipFree(p->lpart);
  p->lpart = nullptr;
  p->lpart_cap = 0;
  p->vlist = nullptr;
  p->sitems = nullptr;
  p->splits = nullptr;
  p->part = nullptr;
  p->part_cap = 0;
  if (p->grid) (void)hipFree(p->grid);
  if (p->kbuf) (void)hipFree(p->kbuf);
  if (p->vecbuf) (void)hipFree(p->vecbuf);
  if (p->red) (void)hipFree(p->red);
  p->vecbuf = nullptr;
  p->red = nullptr;
  p->vecbuf_cap = p->red_cap = 0;
  p->rec = nullptr;
  p->pidx = nullptr;
  p->frame_user = nullptr;
  p->work = nullptr;
  p->grid = nullptr;
  p->kbuf = nullptr;
  p->grid_cap = p->kbuf_cap = 0;
}

template <typename T>
sdn_status dalloc(T **ptr, size_t n, const char *what) {
  *ptr = nullptr;
  if (n == 0) return SDN_OK;
  return hip_check(hipMalloc((void **)ptr, n * sizeof(T)), what);
}

}  // namespace

extern "C" {

void sdn_default_opts(sdn_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->W = 6;
  o->sigma = 2.0;
  o->tile = 0;
  o->max_points_per_item = 0;
  o->workspace_budget = 0;
  o->spread_engine = SDN_SPREAD_AUTO;
  o->point_order = SDN_ORDER_AUTO;
}

const char *sdn_last_error(void) { return sdn::last_error(); }

sdn_status sdn_plan_create(sdn_plan *out, const int64_t shape[3], const float *traj,
                           int64_t M, const int32_t *frame_of_point, int32_t T,
                           const sdn_opts *opts, void *stream) {
  if (!out) return fail(SDN_E_INVALID, "sdn_plan_create: out is NULL");
  *out = nullptr;
  if (!shape) return fail(SDN_E_INVALID, "sdn_plan_create: shape is NULL");
  sdn_opts o;
  sdn_default_opts(&o);
  if (opts) o = *opts;
  if (o.W != 4 && o.W != 6 && o.W != 8)
    return fail(SDN_E_UNSUPPORTED, "sdn_plan_create: W must be 4, 6 or 8");
  if (!(o.sigma >= 1.25 && o.sigma <= 4.0))
    return fail(SDN_E_INVALID, "sdn_plan_create: sigma must be in [1.25, 4]");
  if (M < 0 || M > (int64_t)INT32_MAX - 1024)
    return fail(SDN_E_INVALID, "sdn_plan_create: M out of range [0, 2^31)");
  if (M > 0 && !traj) return fail(SDN_E_INVALID, "sdn_plan_create: traj is NULL");
  if (frame_of_point && T < 1)
    return fail(SDN_E_INVALID, "sdn_plan_create: frame_of_point given with T < 1");
  if (T < 0) return fail(SDN_E_INVALID, "sdn_plan_create: T < 0");
  for (int d = 0; d < 3; ++d)
    if (shape[d] < 1 || shape[d] > 4096)
      return fail(SDN_E_INVALID, "sdn_plan_create: image sizes must be in [1, 4096]");
  const double beta = kb_beta(o.W, o.sigma);
  if (!(M_PI * o.W / (2.0 * o.sigma) < beta))
    return fail(SDN_E_UNSUPPORTED, "sdn_plan_create: kernel too wide for this sigma");

  hipStream_t st = (hipStream_t)stream;
  sdn_plan_s *p = new sdn_plan_s();
  p->magic = kPlanMagic;
  (void)hipGetDevice(&p->device);
  p->M = M;
  p->T = frame_of_point ? T : (T < 1 ? 1 : T);
  p->W = o.W;
  p->sigma = o.sigma;
  p->beta = beta;
  p->ncoef = kernel_ncoef(o.W);
  kernel_coefficients(o.W, beta, p->ncoef, &p->coef);
  p->budget = o.workspace_budget;
  if (o.spread_engine < SDN_SPREAD_AUTO || o.spread_engine > SDN_SPREAD_PLANES)
    return delete p, fail(SDN_E_INVALID, "sdn_plan_create: unknown spread_engine");
  p->spread_engine = o.spread_engine;
  if (o.point_order != SDN_ORDER_AUTO && o.point_order != SDN_ORDER_CELL)
    return delete p, fail(SDN_E_INVALID, "sdn_plan_create: unknown point_order");
  // library choice: kItemCap points per interpolation item, fewer (a power of
  // two, >= 512) for plans of under a million points so that they still
  // spread over enough workgroups
  int auto_cap = 512;
  while (auto_cap < kItemCap && (int64_t)auto_cap * 2 * 512 <= M) auto_cap *= 2;
  p->max_points_per_item = o.max_points_per_item > 0 ? o.max_points_per_item : auto_cap;
  if (p->max_points_per_item > kItemCap)
    return delete p, fail(SDN_E_INVALID, "sdn_plan_create: max_points_per_item above 2048");

  // tiles: 16 x 16 x 8 fine cells (x, y, z), 16 x 16 x 4 for W = 8, unless
  // the caller fixes an edge
  const int tile_default[3] = {16, 16, o.W > 6 ? 4 : 8};
  if (o.tile != 0 && (o.tile < 4 || o.tile > 32))
    return delete p, fail(SDN_E_INVALID, "sdn_plan_create: tile edge must be in [4, 32]");
  // shape is (Nz, Ny, Nx); axis 0 = x
  for (int d = 0; d < 3; ++d) {
    Axis &a = p->ax[d];
    a.N = (int)shape[2 - d];
    a.nf = fine_size(a.N, o.sigma, o.W);
    a.half = a.N / 2;
    a.tile = std::min(o.tile > 0 ? o.tile : tile_default[d], a.nf);
    a.ntile = (a.nf + a.tile - 1) / a.tile;
    a.sblk = std::min(kSpreadBlock, a.nf);
    a.nsblk = (a.nf + a.sblk - 1) / a.sblk;
    p->rp[d] = radix_plan(a.nf);
    if (a.nf > 1024 || p->rp[d].n <= 0) {
      delete p;
      return fail(SDN_E_UNSUPPORTED, "sdn_plan_create: fine grid above 1024 per axis");
    }
  }

  if (interp_lds_bytes(*p) > max_lds_bytes()) {
    delete p;
    return fail(SDN_E_INVALID, "sdn_plan_create: tile too large for workgroup memory");
  }

  sdn_status s = SDN_OK;
  for (int d = 0; d < 3 && s == SDN_OK; ++d) {
    auto di = deapod_inverse(p->ax[d].N, p->ax[d].nf, p->W, beta);
    auto tw = twiddles(p->ax[d].nf);
    s = dalloc(&p->dinv[d], di.size(), "plan tables");
    if (s == SDN_OK) s = dalloc(&p->tw[d], (size_t)p->ax[d].nf, "plan tables");
    if (s == SDN_OK)
      s = hip_check(hipMemcpy(p->dinv[d], di.data(), di.size() * 4, hipMemcpyHostToDevice),
                    "plan tables upload");
    if (s == SDN_OK)
      s = hip_check(hipMemcpy(p->tw[d], tw.data(), tw.size() * 4, hipMemcpyHostToDevice),
                    "plan tables upload");
  }
  if (s == SDN_OK) s = dalloc(&p->absmax, 4, "plan scale words");
  p->nbins = (int64_t)p->ax[0].ntile * p->ax[1].ntile * p->ax[2].ntile;
  p->nsbins = (int64_t)p->ax[0].nsblk * p->ax[1].nsblk * p->ax[2].nsblk;

  // scratch of the two sorts, freed before returning
  int *key = nullptr, *key2 = nullptr, *ord_in = nullptr, *ord = nullptr, *count = nullptr;
  int *ccount = nullptr, *tstart = nullptr;
  int *bad = nullptr, *npv = nullptr, *ppos = nullptr, *vval = nullptr;
  unsigned *vkey = nullptr, *vkey2 = nullptr;
  float4 *rec_tmp = nullptr;
  if (s == SDN_OK && M > 0) {
    const int m = (int)M;
    const int nb = (int)p->nbins;
    const int nsb = (int)p->nsbins;
    const dim3 grd((m + 255) / 256);
    s = dalloc(&key, m, "plan sort");
    if (s == SDN_OK) s = dalloc(&key2, m, "plan sort");
    if (s == SDN_OK) s = dalloc(&ord_in, m, "plan sort");
    if (s == SDN_OK) s = dalloc(&ord, m, "plan sort");
    if (s == SDN_OK) s = dalloc(&rec_tmp, m, "plan sort");
    if (s == SDN_OK) s = dalloc(&ccount, (size_t)nb * kBankClasses, "plan sort");
    if (s == SDN_OK) s = dalloc(&tstart, nb, "plan sort");
    if (s == SDN_OK) s = dalloc(&count, nsb, "plan sort");
    if (s == SDN_OK) s = dalloc(&bad, 1, "plan sort");
    if (s == SDN_OK) s = dalloc(&p->rec, m, "plan points");
    if (s == SDN_OK) s = dalloc(&p->pidx, m, "plan points");
    if (s == SDN_OK && frame_of_point) {
      s = dalloc(&p->frame_user, m, "plan points");
      if (s == SDN_OK)
        s = hip_check(hipMemcpyAsync(p->frame_user, frame_of_point, (size_t)m * 4,
                                     hipMemcpyDeviceToDevice, st),
                      "plan frame copy");
    }
    if (s == SDN_OK)
      s = hip_check(hipMemsetAsync(ccount, 0, (size_t)nb * kBankClasses * 4, st), "plan memset");
    if (s == SDN_OK) s = hip_check(hipMemsetAsync(bad, 0, 4, st), "plan memset");
    FoldGeom g;
    for (int d = 0; d < 3; ++d) {
      g.nf[d] = p->ax[d].nf;
      g.tile[d] = p->ax[d].tile;
      g.ntile[d] = p->ax[d].ntile;
    }
    g.W = p->W;
    g.T = p->T;
    if (s == SDN_OK) {
      hipLaunchKernelGGL(k_fold, grd, dim3(256), 0, st, traj, m, g, frame_of_point, key, rec_tmp,
                         ccount, bad);
      hipLaunchKernelGGL(k_iota, grd, dim3(256), 0, st, ord_in, m);
      s = hip_check(hipGetLastError(), "plan fold kernel");
    }
    std::vector<int> hclass((size_t)nb * kBankClasses), hcount(nb), hstart(nb);
    int hbad = 0;
    if (s == SDN_OK)
      s = hip_check(hipMemcpyAsync(hclass.data(), ccount, hclass.size() * 4, hipMemcpyDeviceToHost,
                                   st),
                    "plan histogram download");
    if (s == SDN_OK)
      s = hip_check(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st), "plan flag download");
    if (s == SDN_OK) s = hip_check(hipStreamSynchronize(st), "plan sync");
    if (s == SDN_OK && (hbad & 1))
      s = fail(SDN_E_RANGE, "sdn_plan_create: non-finite coordinate or |k| > 2^20");
    if (s == SDN_OK && (hbad & 2))
      s = fail(SDN_E_RANGE, "sdn_plan_create: frame_of_point outside [0, T)");
    // interpolation items: the points of a tile, crowded tiles split
    if (s == SDN_OK) {
      std::vector<int4> items;
      int64_t acc = 0;
      const int cap = p->max_points_per_item;
      for (int b = 0; b < nb; ++b) {
        int c = 0;
        for (int q = 0; q < kBankClasses; ++q) c += hclass[(size_t)b * kBankClasses + q];
        hcount[b] = c;
        hstart[b] = (int)acc;
        p->max_bin = std::max<int64_t>(p->max_bin, c);
        for (int st0 = 0; st0 < c; st0 += cap)
          items.push_back(make_int4(b, (int)acc + st0, std::min(cap, c - st0), 0));
        acc += c;
      }
      // items stay in tile order (x fastest): the interpolation deals them
      // out to the XCDs in runs of neighbouring tiles, whose staged tiles
      // overlap, so the overlap is read through a shared L2
      p->nwork = (int64_t)items.size();
      s = dalloc(&p->work, items.size(), "plan work list");
      if (s == SDN_OK && !items.empty())
        s = hip_check(hipMemcpyAsync(p->work, items.data(), items.size() * sizeof(int4),
                                     hipMemcpyHostToDevice, st),
                      "plan work upload");
      if (s == SDN_OK)
        s = hip_check(hipMemcpyAsync(tstart, hstart.data(), (size_t)nb * 4, hipMemcpyHostToDevice,
                                     st),
                      "plan offsets upload");
    }
    // plan order: points sorted by tile and bank class (original order
    // within a class), then interleaved over the classes of their tile
    if (s == SDN_OK)
      s = sort_pairs(reinterpret_cast<const unsigned *>(key), reinterpret_cast<unsigned *>(key2),
                     ord_in, ord, m, key_bits((uint64_t)nb * kBankClasses), st);
    if (s == SDN_OK) {
      hipLaunchKernelGGL(k_place, grd, dim3(256), 0, st, reinterpret_cast<const unsigned *>(key2),
                         ord, rec_tmp, frame_of_point, m, tstart, ccount, p->rec, p->pidx);
      s = hip_check(hipGetLastError(), "plan placement kernel");
    }
    // crowded tiles (every tile with SDN_ORDER_CELL): reorder by first cell
    // (stable, so ties keep the round-robin order); skipped when there are
    // too many to key in 32 bits
    if (s == SDN_OK) {
      const int ncell = (g.tile[0] + g.W - 1) * (g.tile[1] + g.W - 1) * (g.tile[2] + g.W - 1);
      std::vector<int> dtile, dstart, doff;
      int md = 0;
      for (int b = 0; b < nb; ++b)
        if ((o.point_order == SDN_ORDER_CELL || 2 * (int64_t)hcount[b] >= ncell) && hcount[b] > 1) {
          dtile.push_back(b);
          dstart.push_back(hstart[b]);
          doff.push_back(md);
          md += hcount[b];
        }
      const int nd = (int)dtile.size();
      if (nd > 0 && nd <= (1 << (32 - kDenseCellBits)) && ncell <= (1 << kDenseCellBits)) {
        doff.push_back(md);
        int *ddev = nullptr;
        int2 *ptmp = nullptr;
        s = dalloc(&ddev, (size_t)3 * nd + 1, "plan dense tiles");
        if (s == SDN_OK) s = dalloc(&ptmp, md, "plan dense tiles");
        int *d_tile = ddev, *d_start = ddev + nd, *d_off = ddev + 2 * nd;
        if (s == SDN_OK)
          s = hip_check(hipMemcpyAsync(d_tile, dtile.data(), (size_t)nd * 4, hipMemcpyHostToDevice, st),
                        "plan dense upload");
        if (s == SDN_OK)
          s = hip_check(hipMemcpyAsync(d_start, dstart.data(), (size_t)nd * 4, hipMemcpyHostToDevice, st),
                        "plan dense upload");
        if (s == SDN_OK)
          s = hip_check(hipMemcpyAsync(d_off, doff.data(), (size_t)(nd + 1) * 4, hipMemcpyHostToDevice,
                                       st),
                        "plan dense upload");
        const dim3 gd((md + 255) / 256);
        if (s == SDN_OK) {
          // key / key2 / ord_in / ord and rec_tmp are free after the placement
          hipLaunchKernelGGL(k_dense_keys, gd, dim3(256), 0, st, p->rec, g, d_tile, d_start, d_off,
                             nd, md, reinterpret_cast<unsigned *>(key), ord_in);
          s = hip_check(hipGetLastError(), "plan dense key kernel");
        }
        if (s == SDN_OK)
          s = sort_pairs(reinterpret_cast<const unsigned *>(key), reinterpret_cast<unsigned *>(key2),
                         ord_in, ord, md, key_bits((uint64_t)nd << kDenseCellBits), st);
        if (s == SDN_OK) {
          hipLaunchKernelGGL(k_dense_gather, gd, dim3(256), 0, st, p->rec, p->pidx, ord, md, rec_tmp,
                             ptmp);
          hipLaunchKernelGGL(k_dense_put, gd, dim3(256), 0, st, rec_tmp, ptmp, d_start, d_off, nd, md,
                             p->rec, p->pidx);
          s = hip_check(hipGetLastError(), "plan dense placement kernels");
        }
        if (s == SDN_OK) s = hip_check(hipStreamSynchronize(st), "plan sync");
        (void)hipFree(ddev);
        (void)hipFree(ptmp);
      }
    }
    // per-point kernel weights
    if (s == SDN_OK) s = dalloc(&p->wts, (size_t)m * wrec_stride(p->W), "plan weights");
    if (s == SDN_OK) s = dalloc(&p->wts_t, (size_t)m * (3 * p->W + 1), "plan weights");
    if (s == SDN_OK) {
      if (p->W == 4)
        hipLaunchKernelGGL((k_weights<4, 8>), grd, dim3(256), 0, st, p->rec, m, p->coef, p->wts,
                           p->wts_t);
      else if (p->W == 8)
        hipLaunchKernelGGL((k_weights<8, 12>), grd, dim3(256), 0, st, p->rec, m, p->coef, p->wts,
                           p->wts_t);
      else
        hipLaunchKernelGGL((k_weights<6, 10>), grd, dim3(256), 0, st, p->rec, m, p->coef, p->wts,
                           p->wts_t);
      s = hip_check(hipGetLastError(), "plan weights kernel");
    }
    // spreading lists: entries per block and per point, scan, (block,
    // offset)-keyed pairs in plan order, stable sort
    FoldGeom gs = g;
    for (int d = 0; d < 3; ++d) {
      gs.tile[d] = p->ax[d].sblk;
      gs.ntile[d] = p->ax[d].nsblk;
    }
    std::vector<int> scount(nsb);
    if (s == SDN_OK) s = dalloc(&npv, m, "plan spreading lists");
    if (s == SDN_OK) s = dalloc(&ppos, m, "plan spreading lists");
    if (s == SDN_OK) s = hip_check(hipMemsetAsync(count, 0, (size_t)nsb * 4, st), "plan memset");
    if (s == SDN_OK) {
      hipLaunchKernelGGL(k_visit_count, grd, dim3(256), 0, st, p->rec, m, gs, count, npv);
      s = hip_check(hipGetLastError(), "plan visit count kernel");
    }
    if (s == SDN_OK)
      s = hip_check(hipMemcpyAsync(scount.data(), count, (size_t)nsb * 4, hipMemcpyDeviceToHost, st),
                    "plan visit download");
    if (s == SDN_OK) s = hip_check(hipStreamSynchronize(st), "plan sync");
    // spreading items: one per block (blocks without points still write
    // their zeros); a crowded block is split into several items whose
    // partial blocks are summed afterwards
    if (s == SDN_OK) {
      std::vector<int4> sitems, splits;
      int64_t acc = 0, slot = 0;
      // entries per item: kSpreadCap, or fewer when the whole plan has few
      // entries, so that a small, centre-heavy trajectory still spreads over
      // enough workgroups (a multiple of the 32-entry batches, >= 512)
      int64_t total = 0;
      for (int b = 0; b < nsb; ++b) total += scount[b];
      const int cap = (int)std::min<int64_t>(kSpreadCap,
                                             std::max<int64_t>(512, total / 2048 / 32 * 32));
      for (int b = 0; b < nsb; ++b) {
        const int c = scount[b];
        const int nch = std::max(1, (c + cap - 1) / cap);
        if (nch == 1) {
          sitems.push_back(make_int4(b, (int)acc, c, -1));
        } else {
          splits.push_back(make_int4(b, (int)slot, nch, 0));
          for (int q = 0; q < nch; ++q)
            sitems.push_back(make_int4(b, (int)acc + q * cap, std::min(cap, c - q * cap),
                                       (int)slot++));
        }
        acc += c;
        if (acc > INT32_MAX - 1024) break;
      }
      if (acc > INT32_MAX - 1024) s = fail(SDN_E_UNSUPPORTED, "sdn_plan_create: too many points");
      p->nvisit = acc;
      p->nslots = slot;
      std::stable_sort(sitems.begin(), sitems.end(),
                       [](const int4 &a, const int4 &b) { return a.z > b.z; });
      p->nsitems = (int64_t)sitems.size();
      p->nsplit = (int64_t)splits.size();
      if (s == SDN_OK) s = dalloc(&p->sitems, sitems.size(), "plan spreading items");
      if (s == SDN_OK) s = dalloc(&p->splits, splits.size(), "plan spreading items");
      if (s == SDN_OK)
        s = hip_check(hipMemcpyAsync(p->sitems, sitems.data(), sitems.size() * sizeof(int4),
                                     hipMemcpyHostToDevice, st), "plan items upload");
      if (s == SDN_OK && !splits.empty())
        s = hip_check(hipMemcpyAsync(p->splits, splits.data(), splits.size() * sizeof(int4),
                                     hipMemcpyHostToDevice, st), "plan items upload");
    }
    const int nv = (int)p->nvisit;
    if (s == SDN_OK) s = dalloc(&p->vlist, (size_t)std::max(nv, 1), "plan spreading lists");
    if (s == SDN_OK && nv > 0) {
      s = exclusive_sum(npv, ppos, m, st);
      if (s == SDN_OK) s = dalloc(&vkey, nv, "plan spreading lists");
      if (s == SDN_OK) s = dalloc(&vkey2, nv, "plan spreading lists");
      if (s == SDN_OK) s = dalloc(&vval, nv, "plan spreading lists");
      if (s == SDN_OK) {
        hipLaunchKernelGGL(k_visit_pairs, grd, dim3(256), 0, st, p->rec, m, gs, ppos, vkey, vval);
        s = hip_check(hipGetLastError(), "plan visit pairs kernel");
      }
      if (s == SDN_OK)
        s = sort_pairs(vkey, vkey2, vval, p->vlist, nv,
                       key_bits((uint64_t)nsb * kVisitOffsets), st);
      // the matrix-core engine reads each entry's frame and original index
      // beside the list; the gather engine does without
      const bool matrix_ok = p->spread_engine != SDN_SPREAD_GATHER && p->ax[0].nf >= 16 &&
                             p->ax[1].nf >= 16 && p->ax[2].nf >= 16;
      if (s == SDN_OK && matrix_ok) {
        s = dalloc(&p->vinfo, nv, "plan spreading lists");
        if (s == SDN_OK) {
          hipLaunchKernelGGL(k_visit_info, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st,
                             p->vlist, nv, p->pidx, p->vinfo);
          s = hip_check(hipGetLastError(), "plan visit info kernel");
        }
      }
    }
    if (s == SDN_OK) s = hip_check(hipStreamSynchronize(st), "plan sync");
  }
  for (void *q : {(void *)key, (void *)key2, (void *)ord_in, (void *)ord, (void *)rec_tmp,
                  (void *)count, (void *)ccount, (void *)tstart, (void *)bad, (void *)npv, (void *)ppos, (void *)vkey,
                  (void *)vkey2, (void *)vval})
    if (q) (void)hipFree(q);
  if (s != SDN_OK) {
    free_plan_memory(p);
    p->magic = 0;
    delete p;
    return s;
  }
  *out = p;
  return SDN_OK;
}

sdn_status sdn_plan_destroy(sdn_plan p) {
  if (!p) return SDN_OK;
  if (p->magic != kPlanMagic) return fail(SDN_E_STATE, "sdn_plan_destroy: not a live plan");
  free_plan_memory(p);
  p->magic = 0;
  delete p;
  return SDN_OK;
}

sdn_status sdn_plan_get_info(sdn_plan p, sdn_plan_info *info) {
  if (!p || p->magic != kPlanMagic) return fail(SDN_E_STATE, "sdn_plan_get_info: not a live plan");
  if (!info) return fail(SDN_E_INVALID, "sdn_plan_get_info: info is NULL");
  std::memset(info, 0, sizeof(*info));
  for (int d = 0; d < 3; ++d) {
    info->shape[2 - d] = p->ax[d].N;
    info->fine[2 - d] = p->ax[d].nf;
    info->tile[2 - d] = p->ax[d].tile;
  }
  info->M = p->M;
  info->T = p->T;
  info->W = p->W;
  info->sigma = p->sigma;
  info->beta = p->beta;
  info->nbins = p->nbins;
  info->nwork = p->nwork;
  info->max_bin = p->max_bin;
  info->nvisit = p->nvisit;
  info->spread_engine = spread_engine_for(*p, 2, 2);
  info->ncoef = p->ncoef;
  return SDN_OK;
}

sdn_status sdn_spread_engine(sdn_plan p, int B, int K, int *engine) {
  if (!p || p->magic != kPlanMagic) return fail(SDN_E_STATE, "sdn_spread_engine: not a live plan");
  if (!engine || B < 1 || K < 1) return fail(SDN_E_INVALID, "sdn_spread_engine: bad argument");
  *engine = spread_engine_for(*p, K, B);
  return SDN_OK;
}

}  // extern "C"
