// Kernel interpolation (type 2) and spreading (type 1) between the fine
// grids and the nonuniform points, with the temporal-subspace mix fused in.
//
// Fine grids are channel-major, [p][z][y][x] with p = b K + k, so one
// channel of one tile is a compact working set.  Both kernels work tile by
// tile (tiles of bx x by x bz fine cells):
//
// * interpolation: a workgroup takes the points whose first node lies in
//   one tile (a crowded tile is split into several items) and, channel by
//   channel, stages the tile plus its W-1 halo in LDS with coalesced loads,
//   then every lane interpolates its points from LDS and accumulates the
//   subspace mix y_b = sum_k V[t][k] u_{b,k} (running sums behind the tile);
// * spreading: an 8 x 8 x 8 block gathers the contributions of the points
//   whose support touches it (the plan's list for the block), either on the
//   matrix cores (a workgroup of one wave per coil, the block's sum as a
//   product over the list entries) or by a vector-ALU walk into registers,
//   then writes the block once - no atomics, no separate clear of the grid
//   (every block is written exactly once) and a fixed summation order.
//   Crowded blocks are split into several items whose partial blocks a
//   small reduction sums.
#include <algorithm>

#include "fft_lds.h"
#include "nodes.h"
#include "sdn_internal.h"

namespace sdn {

namespace {

// q = e / d via a float reciprocal of d: exact whenever e + d < 2^22 (the
// rounding error stays below the 1/(2d) distance to the next integer);
// used for tile-local indices only (e below 2^16).
__device__ __forceinline__ int fdiv(int e, float inv) { return (int)(((float)e + 0.5f) * inv); }

__device__ __forceinline__ int wrap(int v, int n) {
  v = v >= n ? v - n : v;
  return v >= n ? v - n : v;
}

struct TileGeom {
  int nfx, nfy, nfz;
  int bx, by, bz;
  int ntx, nty;
  size_t G;            // cells of one channel's grid
};

TileGeom tile_geom(const sdn_plan_s &p) {
  TileGeom g;
  g.nfx = p.ax[0].nf; g.nfy = p.ax[1].nf; g.nfz = p.ax[2].nf;
  g.bx = p.ax[0].tile; g.by = p.ax[1].tile; g.bz = p.ax[2].tile;
  g.ntx = p.ax[0].ntile; g.nty = p.ax[1].ntile;
  g.G = (size_t)g.nfx * g.nfy * g.nfz;
  return g;
}

// Ragged volumes: one launch over the work items of several plans.  The
// workgroups of volume v are start[v] .. start[v+1]-1 of the grid's x
// dimension; each reads its volume's descriptor.
constexpr int kMaxFused = kMaxFusedPlans;
template <typename Dev>
struct Fused {
  int n;
  int start[kMaxFused + 1];
  Dev dev[kMaxFused];
};

// Work order over the 8 XCDs.  The hardware deals the workgroups of a
// launch out to the XCDs round-robin (workgroup L to XCD L % 8), and each
// XCD has its own L2.  The items are dealt out in chunks of `chunk`
// consecutive items: XCD j runs chunks j, j + 8, j + 16, ..., and within a
// chunk each item for all its groups (coils or coil groups) in turn, so the
// groups of an item, which read the same point records, and neighbouring
// items of a chunk, which read overlapping grid cells when the items are in
// spatial order, run close together on one XCD.  The grid holds
// xcd_grid(items, groups, chunk) workgroups; those past the last item exit.
constexpr int kXcds = 8;
inline unsigned xcd_grid(int64_t items, int groups, int chunk = 1) {
  const int64_t chunks = (items + chunk - 1) / chunk;
  return (unsigned)((chunks + kXcds - 1) / kXcds * kXcds * chunk * groups);
}
__device__ __forceinline__ bool xcd_item(int items, int groups, int &item, int &group,
                                         int chunk = 1) {
  const int j = (int)blockIdx.x % kXcds, r = (int)blockIdx.x / kXcds;
  const int per = chunk * groups;             // workgroups of one chunk
  const int q = r / per, rr = r - q * per;
  const int g = rr / groups;
  item = (q * kXcds + j) * chunk + g;
  group = rr - g * groups;
  return item < items;
}

// Volume, item and group of this workgroup of a fused launch (items counted
// over all volumes: start[] are item offsets); -1 past the last item.
template <typename Dev>
__device__ __forceinline__ int fused_volume(const Fused<Dev> &f, int groups, int &item,
                                            int &group, int chunk = 1) {
  if (!xcd_item(f.start[f.n], groups, item, group, chunk)) return -1;
  int v = 0;
  while (v + 1 < f.n && item >= f.start[v + 1]) ++v;
  item -= f.start[v];
  return v;
}

struct InterpDev {
  const float4 *rec;
  const int2 *pidx;
  const float *wts_t;  // transposed weights [3W][M], then packed first nodes [M]
  unsigned row_bytes;  // 4 M
  unsigned rec_bytes;  // 4 M (3W + 1), when below 4 GiB
  const int4 *work;
  int M;
  TileGeom g;
  float inv_px, inv_py;
  const float2 *grid;
  int K;               // channels per group
  const float2 *V;     // [T][K] (mix mode)
  float2 *y;
  const float2 *d;
  const float *w;
  float2 *r_plan;
  double *loss_part;   // DC mode: one partial loss per workgroup, [groups][items]
  float rscale;
  unsigned *rmax;
  int nitems;          // work items of this plan (the loss partials' row length)
  int groups;          // output rows per point: coils (mix) or channel groups
  int chunk;           // items per XCD chunk (the items are in tile order)
};

constexpr int kThreads = 256;
constexpr int kIThreads = 512;                // interpolation workgroup

// grid = (items, groups).  Mix mode: a group is one coil and its K channels,
// output y_b = sum_k V[t][k] u_k (+ DC epilogue), the running sums kept in
// registers by the thread that owns the point.  Otherwise a group is K independent channels
// with outputs y_{gK+k} = u_k.  The plan orders the points of a tile so
// that 32 consecutive points mostly start at tile cells of distinct residues
// mod 32 (or, in crowded tiles, at the same or neighbouring cells); gfx950
// serves an 8-byte LDS read to 32 lanes at a time from 64 banks, so each
// half-wave's reads then hit distinct banks, or share a read, at every one
// of the W^3 offsets.
// End of a mixing interpolation item: the points' mixed sums acc[i] (point
// tid + i kIThreads of item wi) to y in user order, or in DC mode the
// residuals in plan order and the workgroup's partial loss and largest
// residual component.
template <bool DC, int NP>
__device__ __forceinline__ void interp_epilogue(const InterpDev &a, const int4 &wi, int grp, int tid,
                                                float2 (&acc)[NP], int item) {
  constexpr int kPts = NP;
  double my_loss = 0.0;
  float my_max = 0.f;
#pragma unroll
  for (int i = 0; i < kPts; ++i) {
    const int q = tid + i * kIThreads;
    if (q >= wi.z) break;
    const int orig = a.pidx[wi.y + q].y;
    if constexpr (DC) {
      const float2 dv = a.d ? a.d[(size_t)grp * a.M + orig] : make_float2(0.f, 0.f);
      const float2 df = csub(acc[i], dv);
      const float wt = a.w ? a.w[orig] : 1.f;
      my_loss += (double)wt * ((double)df.x * df.x + (double)df.y * df.y);
      const float sw = a.rscale * wt;
      const float2 rv = make_float2(sw * df.x, sw * df.y);
      my_max = fmaxf(my_max, fmaxf(fabsf(rv.x), fabsf(rv.y)));
      a.r_plan[(size_t)(wi.y + q) * a.groups + grp] = rv;
    } else {
      a.y[(size_t)grp * a.M + orig] = acc[i];
    }
  }
  if constexpr (DC) {
    __shared__ double part[kIThreads / 64];
    __shared__ float pmax[kIThreads / 64];
    for (int off = 32; off > 0; off >>= 1) {
      my_loss += __shfl_down(my_loss, off, 64);
      my_max = fmaxf(my_max, __shfl_xor(my_max, off, 64));
    }
    if ((tid & 63) == 0) {
      part[tid >> 6] = my_loss;
      pmax[tid >> 6] = my_max;
    }
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      float mx = 0.f;
      for (int i = 0; i < kIThreads / 64; ++i) {
        s += part[i];
        mx = fmaxf(mx, pmax[i]);
      }
      if (a.rmax) atomicMax(a.rmax, __float_as_uint(mx));
      // the partials are summed afterwards in a fixed order, so the loss
      // does not depend on the order in which workgroups finish
      a.loss_part[(size_t)grp * a.nitems + item] = s;
    }
  }
}

template <int W, bool MIX, bool DC, bool BUF>
__device__ __forceinline__ void interp_body(const InterpDev &a, int item, int grp) {
  extern __shared__ float2 tile[];
  // raw buffer over the transposed records (word 3: the gfx9 raw-buffer format)
  const __amdgpu_buffer_rsrc_t wrsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(a.wts_t), 0, (int)a.rec_bytes, 0x00020000);
  const TileGeom &g = a.g;
  const int4 wi = a.work[item];
  const int tid = threadIdx.x;
  const int tz = wi.x / (g.ntx * g.nty);
  const int rem = wi.x - tz * (g.ntx * g.nty);
  const int ty = rem / g.ntx, tx = rem - ty * g.ntx;
  const int ox = tx * g.bx, oy = ty * g.by, oz = tz * g.bz;
  const int PX = g.bx + W - 1, PY = g.by + W - 1, PZ = g.bz + W - 1;
  const int ncell = PX * PY * PZ;
  // running subspace sums of this thread's points (mix mode): point
  // q = tid + i kIThreads keeps its sum in acc[i] across the channels
  constexpr int kPts = kItemCap / kIThreads;
  static_assert(kItemCap % kIThreads == 0, "an item is a whole number of thread passes");
  float2 acc[kPts];
#pragma unroll
  for (int i = 0; i < kPts; ++i) acc[i] = make_float2(0.f, 0.f);
  for (int k = 0; k < a.K; ++k) {
    const float2 *gp = a.grid + (size_t)(grp * a.K + k) * g.G;
    // four loads in flight per thread before their LDS stores
    for (int e0 = tid; e0 < ncell; e0 += 4 * kIThreads) {
      float2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kIThreads;
        if (e < ncell) {
          const int row = fdiv(e, a.inv_px);
          const int cx = e - row * PX;
          const int cz = fdiv(row, a.inv_py);
          const int cy = row - cz * PY;
          const int gx = wrap(ox + cx, g.nfx), gy = wrap(oy + cy, g.nfy), gz = wrap(oz + cz, g.nfz);
          v[u] = gp[((size_t)gz * g.nfy + gy) * g.nfx + gx];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * kIThreads < ncell) tile[e0 + u * kIThreads] = v[u];
    }
    __syncthreads();
#pragma unroll 1
    for (int i = 0; i < kPts; ++i) {
      const int q = tid + i * kIThreads;
      if (q >= wi.z) break;
      const int2 id = a.pidx[wi.y + q];
      // transposed records: a wave's consecutive points are contiguous.
      // Buffer loads share one lane offset and take the row offset from a
      // scalar register (records under 4 GiB); else plain global loads.
      const unsigned jb = (unsigned)(wi.y + q) * 4u;
      auto row = [&](int c) -> float {
        if constexpr (BUF)
          return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
              wrsrc, (int)jb, (int)((unsigned)c * a.row_bytes), 0));
        else
          return a.wts_t[(size_t)c * a.M + wi.y + q];
      };
      int lx, ly, lz;
      unpack_l0(row(3 * W), lx, ly, lz);
      lx -= ox; ly -= oy; lz -= oz;
      float wx[W], wy[W], wz[W];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        wx[c] = row(c);
        wy[c] = row(W + c);
        wz[c] = row(2 * W + c);
      }
      // half a kernel plane at a time: its cells are read into registers
      // first, so those reads are in flight together.  Each cell is its own
      // 8-byte read: left alone, the compiler pairs neighbouring cells into
      // ds_read2_b64, whose two halves then meet bank conflicts whenever the
      // row starts at an odd cell (about 1.2x slower interpolation here).
      // Volatile LDS loads are never merged.
      static_assert(W % 2 == 0, "planes are read in halves");
      typedef const volatile __attribute__((address_space(3))) unsigned long long lds_cell;
      float ur = 0.f, ui = 0.f;
      const float2 *base = tile + (lz * PY + ly) * PX + lx;
#pragma unroll
      for (int az = 0; az < W; ++az) {
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          float2 v[W / 2][W];
#pragma unroll
          for (int ay = 0; ay < W / 2; ++ay)
#pragma unroll
            for (int c = 0; c < W; ++c) {
              const unsigned long long u = *(lds_cell *)(&base[(az * PY + hh * (W / 2) + ay) * PX + c]);
              v[ay][c] = make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
            }
#pragma unroll
          for (int ay = 0; ay < W / 2; ++ay) {
            float tr = 0.f, ti = 0.f;
#pragma unroll
            for (int c = 0; c < W; ++c) {
              tr = fmaf(wx[c], v[ay][c].x, tr);
              ti = fmaf(wx[c], v[ay][c].y, ti);
            }
            pr = fmaf(wy[hh * (W / 2) + ay], tr, pr);
            pi = fmaf(wy[hh * (W / 2) + ay], ti, pi);
          }
        }
        ur = fmaf(wz[az], pr, ur);
        ui = fmaf(wz[az], pi, ui);
      }
      const float2 u = make_float2(ur, ui);
      if constexpr (MIX) {
        // register-resident sums: a select per slot instead of an indexed write
        const float2 m = cmul(a.V[(size_t)id.x * a.K + k], u);
#pragma unroll
        for (int c = 0; c < kPts; ++c)
          if (c == i) acc[c] = cadd(acc[c], m);
      } else {
        a.y[(size_t)(grp * a.K + k) * a.M + id.y] = u;
      }
    }
    __syncthreads();
  }
  if constexpr (MIX) interp_epilogue<DC>(a, wi, grp, tid, acc, item);
}

// grid: items x groups workgroups (one dimension), in XCD order
template <int W, bool MIX, bool DC, bool BUF>
__global__ void __launch_bounds__(kIThreads) k_interp(InterpDev a) {
  int item, grp;
  if (!xcd_item(a.nitems, a.groups, item, grp, a.chunk)) return;
  interp_body<W, MIX, DC, BUF>(a, item, grp);
}

template <int W, bool MIX, bool DC, bool BUF>
__global__ void __launch_bounds__(kIThreads) k_interp_fused(Fused<InterpDev> f) {
  int item, grp;
  const int v = fused_volume(f, f.dev[0].groups, item, grp, f.dev[0].chunk);
  if (v < 0) return;
  interp_body<W, MIX, DC, BUF>(f.dev[v], item, grp);
}

struct SpreadDev {
  const int4 *items;   // (block, list start, count, partial slot or -1)
  const int *vlist;
  const int2 *vinfo;   // per list entry: (frame, original index); matrix-core engine
  const float4 *rec;
  const int2 *pidx;
  const float *wts;    // per point: W weights for x, y, z
  int M;
  int nfx, nfy, nfz;
  int nbx, nby;        // spreading blocks along x and y
  size_t G;
  float2 *grid;
  float2 *part;        // [slot][group][K][512]
  int groups;
  const float2 *V;
  const float2 *src;   // mix: [groups][M]; else [groups * K][M]
  int src_plan;
  const unsigned *absmax;  // matrix engines: largest input magnitudes (value scale)
  int nitems;          // spreading items of this plan
  int cgroups;         // coil groups (workgroups per item) of the launch
};

constexpr int kSB = kSpreadBlock;           // 8
constexpr int kSBCells = kSB * kSB * kSB;   // 512

// Spreading by gathering ("pull"), one wave per item: the wave owns an
// 8 x 8 x 8 block, lane (y, x) holds the block's 8 z cells of all K
// channels in registers, and the entries of the block's list are walked one
// at a time with every lane reading the same point.  A lane adds the point's
// contribution when its (y, x) lies in the point's support.  The plan sorts
// a block's list by the z offset d of the point against the block, so the
// walk meets runs of equal d in a fixed order: each run has its own loop,
// in which every register index is a compile-time constant.  Entries are
// fetched 64 at a time, one per lane (so their memory latency overlaps),
// into an LDS batch that the walk then reads by broadcast.  No atomics
// anywhere; crowded blocks are split into items whose partial blocks
// k_spread_reduce sums.
//
// Batch record of one entry: W z weights, K complex values, then the W x
// and W y weights (read per lane).
template <int W, int K>
struct PullRec {
  static constexpr int zw = 0;                     // z weights
  static constexpr int val = W;                    // values (re, im) x K
  static constexpr int xw = W + 2 * K;             // x weights
  static constexpr int yw = xw + W;                // y weights
  static constexpr int n = yw + W;
  static constexpr int stride = (n + 3) & ~3;      // whole float4s
};

struct PullLane {
  int gx, gy;          // the lane's column
  bool inside;         // column inside the grid
  int nfx, nfy;
};

// Entries v0 .. v1-1 of the batch, all with z offset D: node az of an entry
// lands in register slot D + az (kept when inside the block's 8).
template <int W, int K, int D>
__device__ __forceinline__ void pull_run(const float *bf, int v0, int v1, int l0_lane,
                                         const PullLane &pl, float (&ar)[kSB][K],
                                         float (&ai)[kSB][K]) {
  using R = PullRec<W, K>;
  constexpr int RS = R::stride;
#pragma unroll 1
  for (int v = v0; v < v1; ++v) {
    const float *pr = bf + v * RS;
    const unsigned u = (unsigned)__builtin_amdgcn_readlane(l0_lane, v);
    int dx = pl.gx - (int)(u & 1023u), dy = pl.gy - (int)((u >> 10) & 1023u);
    dx += dx < 0 ? pl.nfx : 0;
    dy += dy < 0 ? pl.nfy : 0;
    const bool on = pl.inside && dx < W && dy < W;
    const float wx = pr[R::xw + min(dx, W - 1)];
    const float wy = pr[R::yw + min(dy, W - 1)];
    const float wxy = on ? wx * wy : 0.f;
#pragma unroll
    for (int az = 0; az < W; ++az) {
      if (D + az >= 0 && D + az < kSB) {
        const float w = wxy * pr[R::zw + az];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
          ar[D + az][kk] = fmaf(w, pr[R::val + 2 * kk], ar[D + az][kk]);
          ai[D + az][kk] = fmaf(w, pr[R::val + 2 * kk + 1], ai[D + az][kk]);
        }
      }
    }
  }
}

template <int W, bool MIX, int K>
__device__ __forceinline__ void spread_gather_body(const SpreadDev &a, int item, int grp) {
  static_assert(W <= 8 && kSB == 8 && kVisitOffsets == 16, "offset cases cover -7 .. 7");
  using R = PullRec<W, K>;
  constexpr int RS = R::stride;
  __shared__ float4 batch[64 * RS / 4];
  float *bf = reinterpret_cast<float *>(batch);
  const int4 it = a.items[item];
  const int lane = threadIdx.x;
  const int bzi = it.x / (a.nbx * a.nby);
  const int rem = it.x - bzi * (a.nbx * a.nby);
  const int byi = rem / a.nbx, bxi = rem - byi * a.nbx;
  const int ox = bxi * kSB, oy = byi * kSB, oz = bzi * kSB;
  PullLane pl;
  pl.gx = ox + (lane & (kSB - 1));
  pl.gy = oy + lane / kSB;
  pl.inside = pl.gx < a.nfx && pl.gy < a.nfy;
  pl.nfx = a.nfx;
  pl.nfy = a.nfy;

  float ar[kSB][K], ai[kSB][K];
#pragma unroll
  for (int c = 0; c < kSB; ++c)
#pragma unroll
    for (int kk = 0; kk < K; ++kk) ar[c][kk] = ai[c][kk] = 0.f;

  for (int b0 = 0; b0 < it.z; b0 += 64) {
    const int nb = min(64, it.z - b0);
    // fetch: lane L loads entry b0 + L of the list
    int l0_lane = 0, d_lane = 0;
    if (lane < nb) {
      const int raw = a.vlist[it.y + b0 + lane];
      const int j = raw < 0 ? ~raw : raw;
      const float4 r = a.rec[j];
      const int2 id = a.pidx[j];
      const float *w = a.wts + (size_t)j * wrec_stride(W);
      float *o = bf + lane * RS;
      l0_lane = __float_as_int(r.w);
      int e = (int)((__float_as_uint(r.w) >> 20) & 1023u) - oz;
      e += e < 0 ? a.nfz : 0;
      d_lane = raw < 0 ? e - a.nfz : e;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        o[R::xw + i] = w[i];
        o[R::yw + i] = w[W + i];
        o[R::zw + i] = w[2 * W + i];
      }
      const int col = a.src_plan ? j : id.y;
      if constexpr (MIX) {
        const float2 rv = a.src_plan ? a.src[(size_t)j * a.groups + grp]
                                     : a.src[(size_t)grp * a.M + col];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
          const float2 v = cmulc(rv, a.V[(size_t)id.x * K + kk]);
          o[R::val + 2 * kk] = v.x;
          o[R::val + 2 * kk + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
          const float2 v = a.src[(size_t)(grp * K + kk) * a.M + col];
          o[R::val + 2 * kk] = v.x;
          o[R::val + 2 * kk + 1] = v.y;
        }
      }
    }
    // a batch is a piece of a list sorted by offset, so the entries of one
    // offset form one run and the runs come in increasing offset order
    __syncthreads();
#define SDN_DRUN(D)                                                             \
  {                                                                             \
    const unsigned long long m = __ballot(lane < nb && d_lane == D);            \
    if (m) {                                                                    \
      const int v0 = (int)__builtin_ctzll(m);                                   \
      pull_run<W, K, D>(bf, v0, v0 + (int)__builtin_popcountll(m), l0_lane, pl, ar, ai); \
    }                                                                           \
  }
    SDN_DRUN(-7) SDN_DRUN(-6) SDN_DRUN(-5) SDN_DRUN(-4) SDN_DRUN(-3)
    SDN_DRUN(-2) SDN_DRUN(-1) SDN_DRUN(0) SDN_DRUN(1) SDN_DRUN(2)
    SDN_DRUN(3) SDN_DRUN(4) SDN_DRUN(5) SDN_DRUN(6) SDN_DRUN(7)
#undef SDN_DRUN
    __syncthreads();
  }
  const int gx = pl.gx, gy = pl.gy;
  if (it.w >= 0) {
    float2 *pp = a.part + ((size_t)it.w * a.groups + grp) * K * kSBCells;
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
#pragma unroll
      for (int c = 0; c < kSB; ++c)
        pp[(size_t)kk * kSBCells + c * 64 + lane] = make_float2(ar[c][kk], ai[c][kk]);
    return;
  }
  if (!pl.inside) return;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    float2 *gp = a.grid + (size_t)(grp * K + kk) * a.G;
#pragma unroll
    for (int c = 0; c < kSB; ++c)
      if (oz + c < a.nfz)
        gp[((size_t)(oz + c) * a.nfy + gy) * a.nfx + gx] = make_float2(ar[c][kk], ai[c][kk]);
  }
}

// grids of the spreading kernels: items x coil groups workgroups (one
// dimension, XCD order); a.cgroups coil groups of the launch
template <int W, bool MIX, int K>
__global__ void __launch_bounds__(64) k_spread(SpreadDev a) {
  int item, grp;
  if (!xcd_item(a.nitems, a.cgroups, item, grp)) return;
  spread_gather_body<W, MIX, K>(a, item, grp);
}

template <int W, bool MIX, int K>
__global__ void __launch_bounds__(64) k_spread_fused(Fused<SpreadDev> f) {
  int item, grp;
  const int v = fused_volume(f, f.dev[0].cgroups, item, grp);
  if (v < 0) return;
  spread_gather_body<W, MIX, K>(f.dev[v], item, grp);
}

// ---------------------------------------------------------------------------
// Spreading as a matrix product on the matrix cores.
//
// For one 8 x 8 x 8 block, the sum over its list entries p is
//   H[(y,x), (k, re/im, z)] = sum_p A[(y,x), p] B[p, (k, re/im, z)],
//   A = wy_p(y) wx_p(x),   B = wz_p(z) (v_{p,k}).re/im,
// a product of a 64 x P and a P x 16K matrix, done 32 entries at a time with
// v_mfma_f32_16x16x32_f16.  FP32 accuracy is kept by splitting each operand
// into fp16 hi + lo parts (x = hi + lo to ~2^-22) and summing the three
// products hi.hi + hi.lo + lo.hi in the FP32 accumulators; the values are
// scaled by a power of two s (from the largest input magnitude) so that they
// sit in fp16 range, and the block is scaled back by 1/s on write-out.
// Used when every fine axis is at least 16 cells, so that no kernel support
// can touch both ends of a block.
typedef _Float16 sdn_half8 __attribute__((ext_vector_type(8)));
typedef float sdn_float4v __attribute__((ext_vector_type(4)));

constexpr int kMmaBatch = 32;                 // list entries per matrix step
constexpr int kWinPad = 8;                    // zeros before a weight row
constexpr int kWinLen = 24;                   // zeros, W weights, zeros

// fp16 hi/lo split of two floats, packed as (entry p0, entry p1) pairs.
__device__ __forceinline__ void split2(float a0, float a1, unsigned &hi, unsigned &lo) {
  const auto h = __builtin_amdgcn_cvt_pkrtz(a0, a1);
  const float r0 = a0 - (float)h[0], r1 = a1 - (float)h[1];
  const auto l = __builtin_amdgcn_cvt_pkrtz(r0, r1);
  hi = __builtin_bit_cast(unsigned, h);
  lo = __builtin_bit_cast(unsigned, l);
}

// Offset of the block start against a point's first node along one axis,
// as the index shift into the point's zero-padded weight row.
__device__ __forceinline__ int win_shift(int o, int l0, int nf, int W) {
  int s = o - l0;
  s += s < -kWinPad ? nf : 0;
  s -= s > W ? nf : 0;
  return min(max(s, -kWinPad), W);
}

// Power-of-two scale that brings the largest value to below 2^14.
__device__ __forceinline__ float value_scale(const unsigned *absmax, bool mix) {
  const float m = __uint_as_float(absmax[0]) * (mix ? 2.f * __uint_as_float(absmax[1]) : 1.f);
  if (!(m > 0.f) || !(m < 3.0e38f)) return 1.f;
  int e;
  (void)frexpf(m, &e);
  return ldexpf(1.f, 14 - e);
}

// The workgroup takes one block for NG coils, one wave per coil: the point
// data of a batch (first node, weights) is fetched and staged once for all
// of them, the four (y,x) operand tiles are built cooperatively into LDS,
// and each wave builds only its own coil's value operand and products.
//
// Each entry goes through two fetch stages, so that no load waits on
// another load issued in the same batch: the list stage (two batches
// ahead) reads the entry and its (frame, original index); the point stage
// (one batch ahead) reads, through those, the point's weight record (wave
// 0, one half per lane: lanes 0..31 the x/y weights, lanes 32..63 the z
// weights and the first node), the residuals of all the workgroup's coils
// (wave 1, or 0 for a single coil) and the frame's K basis values (the
// last wave, each half-wave a half of them).  A load instruction costs the
// memory pipeline about one cycle per cache line it touches, so each
// scattered value is loaded once per workgroup, not once per coil.
struct MmaList {
  int j;      // plan index of the point
  int2 id;    // (frame, original index)
  bool ok;
};

template <int W, bool MIX, int K>
struct MmaFetch {
  static constexpr int NV = (K + 1) / 2;   // basis values per lane (half of K)
  float w[2 * W];     // x, y weights (lanes 0..31); z weights, first node (32..63)
  float2 r[2];        // mixing: residuals of coil slots h and h + 2 (h = lane / 32)
  float2 v[NV];
};

__device__ __forceinline__ void mma_list(const SpreadDev &a, const int4 &it, int e, bool all_lanes,
                                         int lane, MmaList &L) {
  L.ok = e < it.z;
  // kept as loaded (decoded where it is used): decoding it here would wait
  // for this load, and with it for the point loads issued just before
  L.j = L.ok ? a.vlist[it.y + e] : 0;
  L.id = (L.ok && (all_lanes || lane < kMmaBatch)) ? a.vinfo[it.y + e] : make_int2(0, 0);
}

template <int W, bool MIX, int K, int NG>
__device__ __forceinline__ void mma_fetch(const SpreadDev &a, const MmaList &L, int grp, bool coil_ok,
                                          bool v_wave, bool r_wave, int g0, int wv, int lane,
                                          MmaFetch<W, MIX, K> &f) {
  const bool ok = L.ok;
  // a complemented entry is a support that starts in an earlier block (z
  // offset below 0); on grids of at least 16 cells per axis no support
  // meets a block twice, so it is an ordinary entry here
  const int j = L.j < 0 ? ~L.j : L.j;
  if (wv == 0) {
    // one half of the point's record per lane, 16-byte loads: lanes 0..31
    // the x and y weights, lanes 32..63 the z weights and the first node
    static_assert((2 * W) % 4 == 0, "record halves are whole float4s");
    const float4 *wl = reinterpret_cast<const float4 *>(
        a.wts + (size_t)j * wrec_stride(W) + (lane < kMmaBatch ? 0 : 2 * W));
#pragma unroll
    for (int i = 0; i < W / 2; ++i) {
      const float4 v = ok ? wl[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      f.w[4 * i] = v.x;
      f.w[4 * i + 1] = v.y;
      f.w[4 * i + 2] = v.z;
      f.w[4 * i + 3] = v.w;
    }
  }
  static_assert(MIX, "the matrix-core spreading serves the subspace-mixing calls");
  (void)grp;
  (void)coil_ok;
  {
    if (r_wave) {
      // the residuals of all coils of the workgroup: in plan order a point's
      // coils are side by side, so both half-waves read the same lines
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int c = (lane >> 5) + 2 * i;
        const int g = g0 + c;
        const bool rok = ok && c < NG && g < a.groups;
        f.r[i] = !rok ? make_float2(0.f, 0.f)
                      : a.src_plan ? a.src[(size_t)j * a.groups + g]
                                   : a.src[(size_t)g * a.M + L.id.y];
      }
    }
    if (v_wave) {
      const int k0 = (lane >> 5) * f.NV;
#pragma unroll
      for (int i = 0; i < f.NV; ++i)
        f.v[i] = k0 + i < K ? a.V[(size_t)L.id.x * K + k0 + i] : make_float2(0.f, 0.f);
    }
  }
}

template <int W, bool MIX, int K, int NG>
__device__ __forceinline__ void spread_mma_body(const SpreadDev &a, int item, int cg) {
  const unsigned *absmax = a.absmax;
  // values per entry and coil: [re/im][k], K padded to even so that a lane
  // reads its component's K values with 8-byte loads
  constexpr int KP = (K + 1) & ~1;
  // double-buffered staging: batch n is read from buffer n & 1 while batch
  // n + 1 is written to the other, so one barrier per batch suffices
  __shared__ float wrow[2][3][kMmaBatch][kWinLen];
  __shared__ __align__(16) float vals[2][NG][kMmaBatch][2 * KP];
  __shared__ __align__(16) float2 vbas[2][kMmaBatch][KP];   // mixing: the frame's basis values
  __shared__ float2 rsd[2][NG][kMmaBatch];                    // mixing: each coil's residual
  __shared__ int shifts[2][kMmaBatch];
  __shared__ uint4 sA[2][2][4][64];   // [buffer][hi/lo][row tile][lane]: (y,x) operand fragments
  const int4 it = a.items[item];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int grp = cg * NG + wv;
  const bool coil_ok = grp < a.groups;
  const bool v_wave = MIX && wv == NG - 1;   // loads the basis values for all coils
  const bool r_wave = MIX && wv == (NG > 1 ? 1 : 0);   // loads the residuals of all coils
  const int g0 = cg * NG;
  const int bzi = it.x / (a.nbx * a.nby);
  const int rem = it.x - bzi * (a.nbx * a.nby);
  const int byi = rem / a.nbx, bxi = rem - byi * a.nbx;
  const int ox = bxi * kSB, oy = byi * kSB, oz = bzi * kSB;
  // an empty block only writes zeros: no need to wait for the scale
  const float s = it.z > 0 ? value_scale(absmax, MIX) : 1.f;

  // zero the weight rows once; each batch rewrites only the W weights
  for (int i = tid; i < 2 * 3 * kMmaBatch * kWinLen; i += 64 * NG) (&wrow[0][0][0][0])[i] = 0.f;

  sdn_float4v acc[4][K];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[t][k] = sdn_float4v{0.f, 0.f, 0.f, 0.f};

  const int p = lane & (kMmaBatch - 1);   // fetch: this lane's entry
  const int r16 = lane & 15;              // fragment row (A) / column (B)
  const int e0 = 8 * (lane >> 4);         // fragment entries e0 .. e0+7
  const int fx = r16 & 7, fy = r16 >> 3;  // A: x and y offset of the row
  const int fz = r16 & 7, fri = r16 >> 3; // B: z and re/im of the column

  MmaList L;
  MmaFetch<W, MIX, K> f;
  // stage the fetched batch into buffer bf: wave 0 the point data, the last
  // wave the basis values, wave 1 (or 0) the coils' residuals
  auto stage = [&](int bf) {
    if (wv == 0) {
      if (lane < kMmaBatch) {
#pragma unroll
        for (int i = 0; i < W; ++i) {
          wrow[bf][0][p][kWinPad + i] = f.w[i];
          wrow[bf][1][p][kWinPad + i] = f.w[W + i];
        }
      } else {
        const unsigned u = __float_as_uint(f.w[W]);
        const int sx = win_shift(ox, (int)(u & 1023u), a.nfx, W);
        const int sy = win_shift(oy, (int)((u >> 10) & 1023u), a.nfy, W);
        const int sz = win_shift(oz, (int)((u >> 20) & 1023u), a.nfz, W);
        shifts[bf][p] = (sx + kWinPad) | ((sy + kWinPad) << 8) | ((sz + kWinPad) << 16);
#pragma unroll
        for (int i = 0; i < W; ++i) wrow[bf][2][p][kWinPad + i] = f.w[i];
      }
    }
    if constexpr (MIX) {
      if (v_wave) {
        const int k0 = (lane >> 5) * f.NV;
#pragma unroll
        for (int i = 0; i < f.NV; ++i)
          if (k0 + i < K) vbas[bf][p][k0 + i] = f.v[i];
      }
      if (r_wave) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int c = (lane >> 5) + 2 * i;
          if (c < NG) rsd[bf][c][p] = f.r[i];
        }
      }
    }
  };
  // mixing, after the barrier that published the basis values: this coil's
  // values r conj(V_k), written and later read by this wave only
  auto mix_values = [&](int bf) {
    if constexpr (MIX) {
      if (lane < kMmaBatch) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float2 v = cmulc(rsd[bf][wv][p], vbas[bf][p][k]);
          vals[bf][wv][p][k] = v.x * s;
          vals[bf][wv][p][KP + k] = v.y * s;
        }
      }
    }
  };
  // the fetch pipeline: the point data one batch ahead of its staging, the
  // list two batches ahead
  auto advance = [&](int e) {
    if (e < it.z) {
      mma_fetch<W, MIX, K, NG>(a, L, grp, coil_ok, v_wave, r_wave, g0, wv, lane, f);
      if (e + kMmaBatch < it.z) mma_list(a, it, e + kMmaBatch + p, v_wave || r_wave, lane, L);
    }
  };

  if (it.z > 0) {
    mma_list(a, it, p, v_wave || r_wave, lane, L);
    mma_fetch<W, MIX, K, NG>(a, L, grp, coil_ok, v_wave, r_wave, g0, wv, lane, f);
    if (kMmaBatch < it.z) mma_list(a, it, kMmaBatch + p, v_wave || r_wave, lane, L);
  }
  __syncthreads();   // rows zeroed
  if (it.z > 0) {
    stage(0);
    advance(kMmaBatch);
  }
  __syncthreads();
  mix_values(0);
  int bf = 0;
  for (int b0 = 0; b0 < it.z; b0 += kMmaBatch, bf ^= 1) {
    // (y,x) operand tiles, shared by the coils: wave wv builds tiles wv, wv+NG, ...
#pragma unroll
    for (int t0 = 0; t0 < 4; t0 += NG) {
      const int t = t0 + wv;
      if (NG * ((4 + NG - 1) / NG) == 4 || t < 4) {
        float ax[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int q = e0 + e;
          const int sh = shifts[bf][q];
          ax[e] = wrow[bf][1][q][((sh >> 8) & 255) + 2 * t + fy] * wrow[bf][0][q][(sh & 255) + fx];
        }
        unsigned hi[4], lo[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) split2(ax[2 * e], ax[2 * e + 1], hi[e], lo[e]);
        sA[bf][0][t][lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        sA[bf][1][t][lane] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
      }
    }
    // this coil's value operand: B[e][(re/im, z)] = wz v
    float bvv[K][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int q = e0 + e;
      const float bz = wrow[bf][2][q][((shifts[bf][q] >> 16) & 255) + fz];
      const float2 *vr = reinterpret_cast<const float2 *>(&vals[bf][wv][q][fri * KP]);
#pragma unroll
      for (int k2 = 0; k2 < KP / 2; ++k2) {
        const float2 v = vr[k2];
        bvv[2 * k2][e] = bz * v.x;
        if (2 * k2 + 1 < K) bvv[2 * k2 + 1][e] = bz * v.y;
      }
    }
    // the next batch goes to the other buffer while this one is in use
    const bool more = b0 + kMmaBatch < it.z;
    if (more) {
      stage(bf ^ 1);
      advance(b0 + 2 * kMmaBatch);
    }
    __syncthreads();
    if (more) mix_values(bf ^ 1);
    sdn_half8 ah[4], al[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ah[t] = __builtin_bit_cast(sdn_half8, sA[bf][0][t][lane]);
      al[t] = __builtin_bit_cast(sdn_half8, sA[bf][1][t][lane]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      unsigned hi[4], lo[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) split2(bvv[k][2 * e], bvv[k][2 * e + 1], hi[e], lo[e]);
      const sdn_half8 bh = __builtin_bit_cast(sdn_half8, make_uint4(hi[0], hi[1], hi[2], hi[3]));
      const sdn_half8 bl = __builtin_bit_cast(sdn_half8, make_uint4(lo[0], lo[1], lo[2], lo[3]));
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[t][k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[t], bh, acc[t][k], 0, 0, 0);
        acc[t][k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[t], bl, acc[t][k], 0, 0, 0);
        acc[t][k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[t], bh, acc[t][k], 0, 0, 0);
      }
    }
  }
  if (!coil_ok) return;
  // lane holds rows (y,x) = 16t + 4(lane/16) + i, column (re/im, z) =
  // lane % 16.  Lane ^ 8 holds the other component of the same cells:
  // after one exchange, lane re/im = 0 holds (re, im) of cells x0 and
  // x0 + 1 of its row, lane re/im = 1 those of x0 + 2 and x0 + 3, so each
  // lane writes 16 bytes and a store writes whole 64-byte rows of 8 cells.
  const float inv = 1.f / s;
  const int ri = (lane >> 3) & 1, z = lane & 7, qq = lane >> 4;
  const int xc = 4 * (qq & 1) + 2 * ri;   // the first of this lane's two cells
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float v0 = acc[t][k][0] * inv, v1 = acc[t][k][1] * inv;
      const float v2 = acc[t][k][2] * inv, v3 = acc[t][k][3] * inv;
      const float p0 = __shfl_xor(ri ? v0 : v2, 8, 64);
      const float p1 = __shfl_xor(ri ? v1 : v3, 8, 64);
      const float4 out = ri ? make_float4(p0, v2, p1, v3) : make_float4(v0, p0, v1, p1);
      const int y = 2 * t + (qq >> 1);
      if (it.w >= 0) {
        *reinterpret_cast<float4 *>(a.part + (((size_t)it.w * a.groups + grp) * K + k) * kSBCells +
                                    z * 64 + y * 8 + xc) = out;
      } else if (oz + z < a.nfz && oy + y < a.nfy && ox + xc < a.nfx) {
        // fine sizes are even, so both cells of the pair lie inside
        *reinterpret_cast<float4 *>(a.grid + (size_t)(grp * K + k) * a.G +
                                    ((size_t)(oz + z) * a.nfy + oy + y) * a.nfx + ox + xc) = out;
      }
    }
}

template <int W, bool MIX, int K, int NG>
__global__ void __launch_bounds__(64 * NG) k_spread_mma(SpreadDev a) {
  int item, cg;
  if (!xcd_item(a.nitems, a.cgroups, item, cg)) return;
  spread_mma_body<W, MIX, K, NG>(a, item, cg);
}

template <int W, bool MIX, int K, int NG>
__global__ void __launch_bounds__(64 * NG) k_spread_mma_fused(Fused<SpreadDev> f) {
  int item, cg;
  const int v = fused_volume(f, f.dev[0].cgroups, item, cg);
  if (v < 0) return;
  spread_mma_body<W, MIX, K, NG>(f.dev[v], item, cg);
}

// ---------------------------------------------------------------------------
// Spreading as a matrix product, split by planes (many coils and channels).
//
// For one 8 x 8 x 8 block and the coils g of a workgroup, the sum over the
// block's list entries p is, plane by plane,
//   H_z[(y,x), (g,k,re/im)] = sum_p A_z[(y,x), p] B[p, (g,k,re/im)],
//   A_z = wz_p(z) wy_p(y) wx_p(x),   B = r_g(p) conj(V[t_p][k]),
// products of 16 x 32 and 32 x 16 tiles (v_mfma_f32_16x16x32_f16, 32 list
// entries per step).  FP32 accuracy is kept by splitting each operand into
// fp16 hi + lo parts (x = hi + lo to ~2^-22) and summing the three products
// hi.hi + hi.lo + lo.hi in the FP32 accumulators; the values are scaled by
// a power of two s (from the largest input magnitude) so that they sit in
// fp16 range, and the block is scaled back by 1/s on write-out.
//
// Work split: the value operand B does not depend on the plane, so each of
// its 16-column tiles is built once per batch (by one wave) into LDS; the
// sixteen waves of the workgroup split the 32 (plane, y-pair) row tiles,
// wave w taking two y pairs of plane w / 2, and build their A tiles
// themselves from weight rows staged at the block's own coordinates.  A
// block's list is sorted by the z offset of the points, so the supports of
// one batch cover few planes: a wave whose plane no entry of the batch
// touches skips the batch (its operand build and products).  The entries'
// data are loaded by two alternating sets of eight waves (one piece per
// lane: the weights of one axis with the packed first node, two basis
// values or two residuals), two batches ahead of their use, and their list
// entries two batches ahead of that.  Used when every fine axis is at
// least 16 cells, so that no kernel support can touch both ends of a
// block.
constexpr int kPwWaves = 16;                  // waves of a plane-split workgroup
constexpr int kPwCols = 96;                   // value columns per workgroup at most
// A staged weight row holds the 8 weights of one axis at the block's own
// coordinates (zero where the support does not reach); rows are 9 floats
// apart, so the four lane groups of a fragment, which read rows of entries
// 8 apart, start 8 banks apart instead of on the same banks.
constexpr int kPwRow = 9;

// Coils of one plane-split workgroup for kernel width W and K channels:
// 2 K value columns each, at most kPwCols, and at most 16 (a fetch set then
// always loads a batch: see the piece layout in the kernel).
__host__ __device__ constexpr int pw_coils(int W, int K) {
  static_cast<void>(W);   // the weight rows take three pieces whatever the width
  const int g = kPwCols / (2 * K);
  return g < 16 ? g : 16;
}

// A lane's list entry: plan index of the point, (frame, original index).
struct PwList {
  int j;
  int2 id;
};

template <int W, int K, int NCT>
__device__ __forceinline__ void spread_pw_body(const SpreadDev &a, int item, int cg) {
  const unsigned *absmax = a.absmax;
  constexpr int GMAX = pw_coils(W, K);        // coils of a full workgroup
  constexpr int NVP = (K + 1) / 2;            // basis pieces per entry
  constexpr int NRP = (GMAX + 1) / 2;         // residual pieces per entry
  // pieces of a fetch set: weight rows in lanes 0-95 (waves 0-1), basis
  // pieces from lane 128, residual pieces from the next whole wave, so
  // that no wave mixes piece kinds (a wave that ran two kinds' loads in
  // turn would wait for the first kind's loads before issuing the second)
  constexpr int kQv = 4 * kMmaBatch;
  constexpr int kQr = kQv + (kMmaBatch * NVP + 63) / 64 * 64;
  static_assert(kQr + kMmaBatch * NRP <= 512, "one fetch set loads a batch");
  static_assert(W <= kSB, "a weight row covers the block");
  // double-buffered staging: batch n is staged into buffer n & 1 one
  // barrier interval ahead; its value tiles are built into buffer n & 1 and
  // its A tiles into registers in the next interval, and its products run
  // in the interval after that
  __shared__ float wsh[2][3][kMmaBatch][kPwRow];  // block-relative weight rows x, y, z
  __shared__ unsigned pmask[2];                    // planes the entries of a batch touch
  __shared__ float2 vbas[2][kMmaBatch][2 * NVP];
  __shared__ float2 rsd[2][kMmaBatch][2 * NRP];
  __shared__ uint4 sB[2][NCT][2][64];         // [buffer][column tile][hi/lo][lane]

  const int4 it = a.items[item];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int g0 = cg * GMAX;
  const int G = min(GMAX, a.groups - g0);     // coils of this workgroup
  const int bzi = it.x / (a.nbx * a.nby);
  const int rem = it.x - bzi * (a.nbx * a.nby);
  const int byi = rem / a.nbx, bxi = rem - byi * a.nbx;
  const int ox = bxi * kSB, oy = byi * kSB, oz = bzi * kSB;
  // an empty block only writes zeros: no need to wait for the scale
  const float s = it.z > 0 ? value_scale(absmax, true) : 1.f;
  const int nb = (it.z + kMmaBatch - 1) / kMmaBatch;

  // this wave's row tiles: y pairs 2 h and 2 h + 1 of plane z
  const int z = wv >> 1, h = wv & 1;
  sdn_float4v acc[2][NCT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[t][c] = sdn_float4v{0.f, 0.f, 0.f, 0.f};

  const int r16 = lane & 15;              // fragment row (A) / column (B)
  const int e0 = 8 * (lane >> 4);         // fragment entries e0 .. e0+7
  const int fx = r16 & 7, fy = 4 * h + (r16 >> 3);   // A: x, and y of the first tile

  // fetch set (wv / 8) loads the batches of its parity; lane q of the set
  // takes one piece of entry pe: the W weights of one axis and the packed
  // first node (q < 96, axis q / 32), two basis values, or two residuals
  const int q = (wv & 7) * 64 + lane;
  const int set = wv >> 3;
  int kind, pe, pc;
  if (q < 3 * kMmaBatch) {
    kind = 0; pe = q & (kMmaBatch - 1); pc = q / kMmaBatch;
  } else if (q >= kQv && q < kQv + kMmaBatch * NVP) {
    kind = 1; pe = (q - kQv) / NVP; pc = q - kQv - pe * NVP;
  } else if (q >= kQr && q < kQr + kMmaBatch * NRP) {
    kind = 2; pe = (q - kQr) / NRP; pc = q - kQr - pe * NRP;
  } else {
    kind = 3; pe = 0; pc = 0;
  }
  // the axis of a weight lane: block origin and fine size
  const int o_ax = pc == 0 ? ox : pc == 1 ? oy : oz;
  const int nf_ax = pc == 0 ? a.nfx : pc == 1 ? a.nfy : a.nfz;
  PwList L{0, make_int2(0, 0)};
  float fr[W + 1];                        // this lane's piece of its batch
  // list entry of batch b for this lane's piece
  auto list = [&](int b) {
    const int e = b * kMmaBatch + pe;
    if (kind == 3 || e >= it.z) return;
    // kept as loaded: decoding it here would wait for the load at once
    L.j = a.vlist[it.y + e];
    if (kind != 0) L.id = a.vinfo[it.y + e];
  };
  // this lane's piece of batch b (zeros past the list's end)
  auto fetch = [&](int b) {
#pragma unroll
    for (int i = 0; i <= W; ++i) fr[i] = 0.f;
    if (kind == 3 || b * kMmaBatch + pe >= it.z) return;
    // a complemented entry is a support that starts in an earlier block (z
    // offset below 0); on grids of at least 16 cells per axis no support
    // meets a block twice, so it is an ordinary entry here
    const int j = L.j < 0 ? ~L.j : L.j;
    // the lane's piece index, opaque to the compiler: otherwise it keeps a
    // 64-bit address per piece kind live across the whole loop (and spills
    // them, and a spill reload waits for every load in flight)
    int pco = pc;
    asm volatile("" : "+v"(pco));
    if (kind == 0) {
      const size_t r = (size_t)j * wrec_stride(W);
      const float2 *r2 = reinterpret_cast<const float2 *>(a.wts + (r + pco * W));
#pragma unroll
      for (int i = 0; i < W / 2; ++i) {
        const float2 v = r2[i];
        fr[2 * i] = v.x;
        fr[2 * i + 1] = v.y;
      }
      fr[W] = a.wts[r + 3 * W];
    } else if (kind == 1) {
      const int k = 2 * pco;
      const float2 *vp = a.V + ((size_t)L.id.x * K + k);
      const float2 v0 = vp[0];
      const float2 v1 = k + 1 < K ? vp[1] : make_float2(0.f, 0.f);
      fr[0] = v0.x; fr[1] = v0.y; fr[2] = v1.x; fr[3] = v1.y;
    } else {
      const int c = 2 * pco;
      float2 r0 = make_float2(0.f, 0.f), r1 = make_float2(0.f, 0.f);
      if (a.src_plan) {
        const float2 *sp = a.src + ((size_t)j * a.groups + g0 + c);
        if (c < G) r0 = sp[0];
        if (c + 1 < G) r1 = sp[1];
      } else {
        const float2 *sp = a.src + ((size_t)(g0 + c) * a.M + L.id.y);
        if (c < G) r0 = sp[0];
        if (c + 1 < G) r1 = sp[a.M];
      }
      fr[0] = r0.x; fr[1] = r0.y; fr[2] = r1.x; fr[3] = r1.y;
    }
  };
  // store this lane's piece of batch b into buffer bf.  A weight lane
  // writes its axis row at block coordinates: cell f of the block is weight
  // f + sh of the support, sh the offset of the block start against the
  // first node.  The z lanes (lanes 0-31 of the set's second wave) also
  // combine the planes their supports touch into the batch's plane mask.
  auto stage = [&](int bf, int b) {
    unsigned planes = 0;
    if (kind == 0) {
      const unsigned bits = __float_as_uint(fr[W]);
      const int l0 = (int)((bits >> (10 * pc)) & 1023u);
      const int sh = win_shift(o_ax, l0, nf_ax, W);
      float *row = &wsh[bf][pc][pe][0];
#pragma unroll
      for (int f = 0; f < kSB; ++f) {
        float v = 0.f;
#pragma unroll
        for (int i = 0; i < W; ++i) v = (f + sh == i) ? fr[i] : v;
        row[f] = v;
      }
      const int lo = max(0, -sh), hi = min(kSB, W - sh);
      if (pc == 2 && b * kMmaBatch + pe < it.z && hi > lo)
        planes = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
    } else if (kind == 1) {
      vbas[bf][pe][2 * pc] = make_float2(fr[0], fr[1]);
      vbas[bf][pe][2 * pc + 1] = make_float2(fr[2], fr[3]);
    } else if (kind == 2) {
      rsd[bf][pe][2 * pc] = make_float2(fr[0], fr[1]);
      rsd[bf][pe][2 * pc + 1] = make_float2(fr[2], fr[3]);
    }
    if ((wv & 7) == 1) {
      unsigned pm = 0;
#pragma unroll
      for (int f = 0; f < kSB; ++f) pm |= __ballot((planes >> f) & 1u) != 0 ? 1u << f : 0u;
      if (lane == 0) pmask[bf] = pm;
    }
  };
  // the value tile c of batch bf: column n of the tile is (coil, channel,
  // re/im) = 16 c + n, its 8 entries e0 .. e0 + 7
  auto build_values = [&](int bf, int c) {
    const int col = 16 * c + r16;
    const int gl = col / (2 * K), kk = (col >> 1) - gl * K, ri = col & 1;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float x = 0.f;
      if (gl < G) {
        const float2 m = cmulc(rsd[bf][e0 + e][gl], vbas[bf][e0 + e][kk]);
        x = (ri ? m.y : m.x) * s;
      }
      v[e] = x;
    }
    unsigned hi[4], lo[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split2(v[2 * e], v[2 * e + 1], hi[e], lo[e]);
    sB[bf][c][0][lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
    sB[bf][c][1][lane] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
  };

  // prologue: set 0 stages batch 0 and holds batch 2 and the list of batch
  // 4; set 1 holds batch 1 and the list of batch 3
  if (set == 0) {
    list(0);
    fetch(0);
    list(2);
  } else {
    list(1);
    fetch(1);
    list(3);
  }
  if (set == 0 && nb > 0) {
    stage(0, 0);
    fetch(2);
    list(4);
  }
  __syncthreads();
  // Between two barriers a wave runs the products of batch n - 1 and builds
  // the operands of batch n.  The set that stages batch n + 1 does that
  // first (its loads were issued two batches earlier) and its products
  // after, while the other set starts with its products and then builds the
  // value tiles: the matrix cores and the vector ALU then work for
  // different waves at the same time instead of in turn.
  uint4 ah[2], al[2];
  bool act_prev = false;
  for (int n = 0; n <= nb; ++n) {
    const int bf = n & 1;
    // the set of batch n + 1 stages it into the other buffer and loads
    // batch n + 3 and the list of batch n + 5
    if (set == ((n + 1) & 1) && n + 1 < nb) {
      stage(bf ^ 1, n + 1);
      if (n + 3 < nb) {
        fetch(n + 3);
        if (n + 5 < nb) list(n + 5);
      }
    }
    if (act_prev) {
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const sdn_half8 b_hi = __builtin_bit_cast(sdn_half8, sB[bf ^ 1][c][0][lane]);
        const sdn_half8 b_lo = __builtin_bit_cast(sdn_half8, sB[bf ^ 1][c][1][lane]);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const sdn_half8 a_hi = __builtin_bit_cast(sdn_half8, ah[t]);
          const sdn_half8 a_lo = __builtin_bit_cast(sdn_half8, al[t]);
          acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_hi, b_hi, acc[t][c], 0, 0, 0);
          acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_hi, b_lo, acc[t][c], 0, 0, 0);
          acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_lo, b_hi, acc[t][c], 0, 0, 0);
        }
      }
    }
    if (n == nb) break;
    // the value tiles of batch n: waves 0 .. NCT - 1 of the set that does
    // not stage in this interval
    if (set == bf && (wv & 7) < NCT) build_values(bf, wv & 7);
    act_prev = (pmask[bf] >> z) & 1u;
    // this wave's A tiles, into registers: A[(y, x), entry] =
    // wz(z) wy(y) wx(x) from the staged rows of this batch
    if (act_prev) {
      float a0[8], a1[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int qe = e0 + e;
        const float zx = wsh[bf][2][qe][z] * wsh[bf][0][qe][fx];
        a0[e] = zx * wsh[bf][1][qe][fy];
        a1[e] = zx * wsh[bf][1][qe][fy + 2];
      }
      unsigned hi0[4], lo0[4], hi1[4], lo1[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        split2(a0[2 * e], a0[2 * e + 1], hi0[e], lo0[e]);
        split2(a1[2 * e], a1[2 * e + 1], hi1[e], lo1[e]);
      }
      ah[0] = make_uint4(hi0[0], hi0[1], hi0[2], hi0[3]);
      al[0] = make_uint4(lo0[0], lo0[1], lo0[2], lo0[3]);
      ah[1] = make_uint4(hi1[0], hi1[1], hi1[2], hi1[3]);
      al[1] = make_uint4(lo1[0], lo1[1], lo1[2], lo1[3]);
    }
    __syncthreads();
  }
  // lane holds rows 4 (lane / 16) + i of its row tiles t, i.e. cells
  // (y, x) = (4 h + 2 t + (lane / 16) / 2, 4 ((lane / 16) & 1) + i), of
  // column 16 c + lane % 16 = (coil, channel, re/im)
  // The partner lane (lane ^ 1) holds the other component of the same
  // cells: after one exchange, lane re/im = 0 holds (re, im) of cells x0
  // and x0 + 1, lane re/im = 1 those of x0 + 2 and x0 + 3, so each lane
  // writes 16 bytes and a store instruction writes whole 64-byte rows of
  // 8 cells (single 4-byte stores of interleaved components, half the
  // lanes per cell, took about 40% of the kernel's time).
  const float inv = 1.f / s;
  const int qq = lane >> 4;
  const int ri = lane & 1;
  const int xc = 4 * (qq & 1) + 2 * ri;   // the first of this lane's two cells
#pragma unroll
  for (int c = 0; c < NCT; ++c) {
    const int col = 16 * c + r16;
    const int gl = col / (2 * K), kk = (col >> 1) - gl * K;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const float v0 = acc[t][c][0] * inv, v1 = acc[t][c][1] * inv;
      const float v2 = acc[t][c][2] * inv, v3 = acc[t][c][3] * inv;
      const float p0 = __shfl_xor(ri ? v0 : v2, 1, 64);
      const float p1 = __shfl_xor(ri ? v1 : v3, 1, 64);
      const float4 out = ri ? make_float4(p0, v2, p1, v3) : make_float4(v0, p0, v1, p1);
      if (gl >= G) continue;
      const int g = g0 + gl;
      const int y = 4 * h + 2 * t + (qq >> 1);
      if (it.w >= 0) {
        *reinterpret_cast<float4 *>(
            a.part + (((size_t)it.w * a.groups + g) * K + kk) * kSBCells + z * 64 + y * 8 + xc) = out;
      } else if (oz + z < a.nfz && oy + y < a.nfy && ox + xc < a.nfx) {
        // fine sizes are even, so both cells of the pair lie inside
        *reinterpret_cast<float4 *>(a.grid + (size_t)(g * K + kk) * a.G +
                                    ((size_t)(oz + z) * a.nfy + oy + y) * a.nfx + ox + xc) = out;
      }
    }
  }
}

template <int W, int K, int NCT>
__global__ void __launch_bounds__(64 * kPwWaves) k_spread_pw(SpreadDev a) {
  int item, cg;
  if (!xcd_item(a.nitems, a.cgroups, item, cg)) return;
  spread_pw_body<W, K, NCT>(a, item, cg);
}

template <int W, int K, int NCT>
__global__ void __launch_bounds__(64 * kPwWaves) k_spread_pw_fused(Fused<SpreadDev> f) {
  int item, cg;
  const int v = fused_volume(f, f.dev[0].cgroups, item, cg);
  if (v < 0) return;
  spread_pw_body<W, K, NCT>(f.dev[v], item, cg);
}

// Largest |component| of n complex values, as float bits (non-negative
// floats order like their bit patterns) into *out, which starts at zero.
// Four 8-byte loads per thread are in flight per step.
__global__ void __launch_bounds__(256) k_absmax(const float2 *x, size_t n, unsigned *out) {
  float m = 0.f;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i0 = (size_t)blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
    float2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t i = i0 + u * stride;
      v[u] = i < n ? x[i] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) m = fmaxf(m, fmaxf(fabsf(v[u].x), fabsf(v[u].y)));
  }
  // one atomic per workgroup: the waves' maxima meet in LDS first
  __shared__ float wmax[4];
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(out, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
}

__global__ void k_zero_u32(unsigned *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// grid = (split blocks, groups): sum the partial blocks of a crowded block.
__global__ void __launch_bounds__(kThreads) k_spread_reduce(SpreadDev a, const int4 *splits, int K) {
  const int4 sp = splits[blockIdx.x];
  const int grp = blockIdx.y;
  const int bzi = sp.x / (a.nbx * a.nby);
  const int rem = sp.x - bzi * (a.nbx * a.nby);
  const int byi = rem / a.nbx, bxi = rem - byi * a.nbx;
  const int ox = bxi * kSB, oy = byi * kSB, oz = bzi * kSB;
  for (int e = threadIdx.x; e < K * kSBCells; e += kThreads) {
    const int kk = e / kSBCells, cell = e - kk * kSBCells;
    const int c = cell / 64, lane = cell - c * 64;
    const int gx = ox + (lane & (kSB - 1)), gy = oy + lane / kSB, gz = oz + c;
    if (gx >= a.nfx || gy >= a.nfy || gz >= a.nfz) continue;
    float sr = 0.f, si = 0.f;
#pragma unroll 8
    for (int q = 0; q < sp.z; ++q) {
      const float2 v = a.part[(((size_t)(sp.y + q) * a.groups + grp) * K + kk) * kSBCells + cell];
      sr += v.x;
      si += v.y;
    }
    a.grid[(size_t)(grp * K + kk) * a.G + ((size_t)gz * a.nfy + gy) * a.nfx + gx] =
        make_float2(sr, si);
  }
}

__global__ void k_fill_zero(float4 *a, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_fill_zero_f64(double *a, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = 0.0;
}

__global__ void k_mix_fwd(const float2 *u, const float2 *V, const int32_t *frame, int K, int k,
                          int M, float2 *y, int accumulate) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int t = frame ? frame[j] : 0;
  float2 v = cmul(V[(size_t)t * K + k], u[j]);
  if (accumulate) v = cadd(v, y[j]);
  y[j] = v;
}

__global__ void k_mix_adj(const float2 *r, const float2 *V, const int32_t *frame, int K, int k,
                          int M, float2 *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int t = frame ? frame[j] : 0;
  out[j] = cmulc(r[j], V[(size_t)t * K + k]);
}

}  // namespace

// LDS of an interpolation workgroup: the staged tile plus the running sums.
size_t interp_lds_bytes(const sdn_plan_s &p) {
  return (size_t)(p.ax[0].tile + p.W - 1) * (p.ax[1].tile + p.W - 1) * (p.ax[2].tile + p.W - 1) *
         sizeof(float2);
}

namespace {

template <typename F>
hipError_t allow_lds_fwd(F *kernel, size_t bytes);

template <int W, bool MIX, bool DC, bool BUF>
hipError_t interp_one(const InterpDev &d, const Fused<InterpDev> *fz, dim3 grd, size_t lds,
                      hipStream_t st) {
  if (fz) {
    hipError_t e = allow_lds_fwd(k_interp_fused<W, MIX, DC, BUF>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_interp_fused<W, MIX, DC, BUF>), grd, dim3(kIThreads), lds, st, *fz);
  } else {
    hipError_t e = allow_lds_fwd(k_interp<W, MIX, DC, BUF>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_interp<W, MIX, DC, BUF>), grd, dim3(kIThreads), lds, st, d);
  }
  return hipGetLastError();
}

template <int W, bool BUF>
hipError_t interp_launch_b(const InterpDev &d, const Fused<InterpDev> *fz, bool mix, bool dc,
                           dim3 grd, size_t lds, hipStream_t st) {
  if (mix && dc) return interp_one<W, true, true, BUF>(d, fz, grd, lds, st);
  if (mix) return interp_one<W, true, false, BUF>(d, fz, grd, lds, st);
  return interp_one<W, false, false, BUF>(d, fz, grd, lds, st);
}

// buf: every plan's transposed records are under 2 GiB (raw buffer loads)
template <int W>
hipError_t interp_launch(const InterpDev &d, const Fused<InterpDev> *fz, bool buf, bool mix,
                         bool dc, dim3 grd, size_t lds, hipStream_t st) {
  return buf ? interp_launch_b<W, true>(d, fz, mix, dc, grd, lds, st)
             : interp_launch_b<W, false>(d, fz, mix, dc, grd, lds, st);
}

}  // namespace

// Workgroup LDS limit of the current device (gfx950: 160 KB), queried once.
size_t max_lds_bytes() {
  static size_t cached = 0;
  if (cached == 0) {
    int dev = 0, v = 0;
    size_t lim = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      lim = (size_t)v;
    cached = std::min<size_t>(lim, 160 * 1024);
  }
  return cached;
}

namespace {
// Raise a kernel's dynamic-LDS cap when a launch needs more than 64 KB.
template <typename F>
hipError_t allow_lds(F *kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
template <typename F>
hipError_t allow_lds_fwd(F *kernel, size_t bytes) {
  return allow_lds(kernel, bytes);
}
}  // namespace

namespace {

// Descriptor of one plan's interpolation call.
InterpDev interp_dev(const sdn_plan_s &p, const InterpArgs &a) {
  InterpDev d;
  d.rec = p.rec;
  d.pidx = p.pidx;
  d.wts_t = p.wts_t;
  const uint64_t rec_bytes = (uint64_t)p.M * (3 * p.W + 1) * 4;
  const bool buf = rec_bytes < (1ull << 31);
  d.row_bytes = (unsigned)(p.M * 4);
  d.rec_bytes = buf ? (unsigned)rec_bytes : 0u;
  d.work = p.work;
  d.M = (int)p.M;
  d.g = tile_geom(p);
  d.inv_px = 1.0f / (float)(d.g.bx + p.W - 1);
  d.inv_py = 1.0f / (float)(d.g.by + p.W - 1);
  d.grid = a.grid;
  d.K = a.kg;
  d.V = a.V;
  d.y = a.y;
  d.d = a.d;
  d.w = a.w;
  d.r_plan = a.r_plan;
  d.loss_part = a.loss_part;
  d.rscale = a.rscale;
  d.rmax = a.dc ? a.rmax : nullptr;
  d.nitems = (int)p.nwork;
  d.groups = a.groups;
  d.chunk = std::max(1, p.ax[0].ntile);   // about one row of tiles along x
  return d;
}

bool interp_args_ok(const sdn_plan_s &p, const InterpArgs &a) {
  const bool mix = a.V != nullptr;
  if (a.dc && (!mix || a.r_plan == nullptr || a.loss == nullptr || a.loss_part == nullptr))
    return false;
  return interp_lds_bytes(p) <= max_lds_bytes();
}

// loss += the workgroups' partials, two fixed-order levels
hipError_t interp_loss_sum(const sdn_plan_s &p, const InterpArgs &a, hipStream_t st) {
  const size_t nparts = interp_loss_parts(p, a.groups);
  return launch_sum(a.loss_part, (int)nparts, 1.0, a.loss, st, a.loss_part + nparts, true);
}

}  // namespace

hipError_t launch_interp(const sdn_plan_s &p, const InterpArgs &a, hipStream_t st) {
  if (p.M == 0 || p.nwork == 0) return hipSuccess;
  if (!interp_args_ok(p, a)) return hipErrorInvalidValue;
  const InterpDev d = interp_dev(p, a);
  const bool mix = a.V != nullptr;
  const bool dc = a.dc != 0;
  const size_t lds = interp_lds_bytes(p);
  if (d.rmax) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, d.rmax, 1);
  dim3 grd(xcd_grid(p.nwork, a.groups, d.chunk));
  hipError_t e;
  switch (p.W) {
    case 4: e = interp_launch<4>(d, nullptr, d.rec_bytes != 0, mix, dc, grd, lds, st); break;
    case 8: e = interp_launch<8>(d, nullptr, d.rec_bytes != 0, mix, dc, grd, lds, st); break;
    default: e = interp_launch<6>(d, nullptr, d.rec_bytes != 0, mix, dc, grd, lds, st); break;
  }
  if (e != hipSuccess || !dc) return e;
  return interp_loss_sum(p, a, st);
}

hipError_t launch_interp_fused(const sdn_plan_s *const *plans, const InterpArgs *args, int n,
                               hipStream_t st) {
  if (n < 1 || n > kMaxFused) return hipErrorInvalidValue;
  Fused<InterpDev> f{};
  f.n = n;
  size_t lds = 0;
  bool buf = true;
  int total = 0;
  const bool mix = args[0].V != nullptr, dc = args[0].dc != 0;
  for (int v = 0; v < n; ++v) {
    const sdn_plan_s &p = *plans[v];
    const InterpArgs &a = args[v];
    if (p.M == 0 || p.nwork == 0 || p.W != plans[0]->W || a.groups != args[0].groups ||
        (a.V != nullptr) != mix || (a.dc != 0) != dc || a.kg != args[0].kg || !interp_args_ok(p, a))
      return hipErrorInvalidValue;
    f.dev[v] = interp_dev(p, a);
    buf = buf && f.dev[v].rec_bytes != 0;
    lds = std::max(lds, interp_lds_bytes(p));
    f.start[v] = total;
    total += (int)p.nwork;
    if (f.dev[v].rmax) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, f.dev[v].rmax, 1);
  }
  f.start[n] = total;
  dim3 grd(xcd_grid(total, args[0].groups, f.dev[0].chunk));
  hipError_t e;
  switch (plans[0]->W) {
    case 4: e = interp_launch<4>(f.dev[0], &f, buf, mix, dc, grd, lds, st); break;
    case 8: e = interp_launch<8>(f.dev[0], &f, buf, mix, dc, grd, lds, st); break;
    default: e = interp_launch<6>(f.dev[0], &f, buf, mix, dc, grd, lds, st); break;
  }
  if (e != hipSuccess || !dc) return e;
  for (int v = 0; v < n && e == hipSuccess; ++v) e = interp_loss_sum(*plans[v], args[v], st);
  return e;
}

size_t interp_loss_parts(const sdn_plan_s &p, int groups) { return (size_t)p.nwork * groups; }

size_t spread_part_elems(const sdn_plan_s &p, int groups, int K) {
  return (size_t)p.nslots * groups * K * kSBCells;
}

namespace {
// The launch grids: items x coil groups workgroups; the coil-group count
// goes into the descriptors.
unsigned spread_grid(SpreadDev &d, Fused<SpreadDev> *fz, int cgroups) {
  d.cgroups = cgroups;
  if (!fz) return xcd_grid(d.nitems, cgroups);
  for (int v = 0; v < fz->n; ++v) fz->dev[v].cgroups = cgroups;
  return xcd_grid(fz->start[fz->n], cgroups);
}

template <int W, bool MIX>
hipError_t spread_mma(SpreadDev d, Fused<SpreadDev> *fz, int K, hipStream_t st) {
  // up to four coils per workgroup, one wave each
  const int ng = std::min(d.groups, 4);
  const dim3 grd(spread_grid(d, fz, (d.groups + ng - 1) / ng));
  switch (K * 8 + ng) {
#define SDN_SPM(KV, NGV)                                                                    \
  case KV * 8 + NGV:                                                                        \
    if (fz)                                                                                 \
      hipLaunchKernelGGL((k_spread_mma_fused<W, MIX, KV, NGV>), grd, dim3(64 * NGV), 0, st, *fz); \
    else                                                                                    \
      hipLaunchKernelGGL((k_spread_mma<W, MIX, KV, NGV>), grd, dim3(64 * NGV), 0, st, d);   \
    break;
#define SDN_SPM4(KV) SDN_SPM(KV, 1) SDN_SPM(KV, 2) SDN_SPM(KV, 3) SDN_SPM(KV, 4)
    SDN_SPM4(2) SDN_SPM4(3) SDN_SPM4(4) SDN_SPM4(5) SDN_SPM4(6) SDN_SPM4(7) SDN_SPM4(8)
#undef SDN_SPM4
#undef SDN_SPM
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W>
hipError_t spread_pw(SpreadDev d, Fused<SpreadDev> *fz, int K, hipStream_t st) {
  // a workgroup takes up to pw_coils(K) coils: 2 K value columns each, in
  // 16-column tiles (5 tiles run as 6)
  const int gmax = pw_coils(W, K);
  const int G = std::min(d.groups, gmax);
  int nct = (2 * K * G + 15) / 16;
  if (nct == 5) nct = 6;
  const dim3 grd(spread_grid(d, fz, (d.groups + gmax - 1) / gmax));
  switch (K * 8 + nct) {
#define SDN_SPW(KV, NV)                                                                         \
  case KV * 8 + NV:                                                                             \
    if (fz)                                                                                     \
      hipLaunchKernelGGL((k_spread_pw_fused<W, KV, NV>), grd, dim3(64 * kPwWaves), 0, st, *fz); \
    else                                                                                        \
      hipLaunchKernelGGL((k_spread_pw<W, KV, NV>), grd, dim3(64 * kPwWaves), 0, st, d);         \
    break;
#define SDN_SPW5(KV) SDN_SPW(KV, 1) SDN_SPW(KV, 2) SDN_SPW(KV, 3) SDN_SPW(KV, 4) SDN_SPW(KV, 6)
    SDN_SPW5(2) SDN_SPW5(3) SDN_SPW5(4) SDN_SPW5(5) SDN_SPW5(6) SDN_SPW5(7) SDN_SPW5(8)
#undef SDN_SPW5
#undef SDN_SPW
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// The matrix-core spreadings serve the subspace-mixing calls; they need
// every fine axis >= 16 cells (no support touches both ends of a block) and
// at least two channels per coil.
int spread_engine_for(const sdn_plan_s &p, int K, int groups) {
  if (p.spread_engine == SDN_SPREAD_GATHER) return SDN_SPREAD_GATHER;
  const bool ok = K >= 2 && p.ax[0].nf >= 16 && p.ax[1].nf >= 16 && p.ax[2].nf >= 16 &&
                  p.absmax != nullptr && (p.vinfo != nullptr || p.nvisit == 0);
  if (!ok) return SDN_SPREAD_GATHER;
  if (p.spread_engine != SDN_SPREAD_AUTO) return p.spread_engine;
  // automatic choice: the matrix cores pay once several coils share the
  // point data of a block (a single coil keeps the gather); the plane split
  // builds the value operand once for all coils and channels, which pays
  // from about 32 of them
  if (groups < 2) return SDN_SPREAD_GATHER;
  return K * groups >= kPlanesFrom ? SDN_SPREAD_PLANES : SDN_SPREAD_MATRIX;
}

namespace {

template <int W, bool MIX>
hipError_t spread_k(SpreadDev d, Fused<SpreadDev> *fz, int K, hipStream_t st) {
  const dim3 grd(spread_grid(d, fz, d.groups));
  switch (K) {
#define SDN_SPK(KV)                                                                     \
  case KV:                                                                              \
    if (fz)                                                                             \
      hipLaunchKernelGGL((k_spread_fused<W, MIX, KV>), grd, dim3(64), 0, st, *fz);      \
    else                                                                                \
      hipLaunchKernelGGL((k_spread<W, MIX, KV>), grd, dim3(64), 0, st, d);              \
    break;
    SDN_SPK(1) SDN_SPK(2) SDN_SPK(3) SDN_SPK(4) SDN_SPK(5) SDN_SPK(6) SDN_SPK(7) SDN_SPK(8)
#undef SDN_SPK
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Descriptor of one plan's spreading call.
SpreadDev spread_dev(const sdn_plan_s &p, const SpreadArgs &a) {
  SpreadDev d;
  d.items = p.sitems;
  d.vlist = p.vlist;
  d.vinfo = p.vinfo;
  d.rec = p.rec;
  d.pidx = p.pidx;
  d.wts = p.wts;
  d.M = (int)p.M;
  d.nfx = p.ax[0].nf; d.nfy = p.ax[1].nf; d.nfz = p.ax[2].nf;
  d.nbx = p.ax[0].nsblk; d.nby = p.ax[1].nsblk;
  d.G = (size_t)d.nfx * d.nfy * d.nfz;
  d.grid = a.grid;
  d.part = a.part;
  d.groups = a.groups;
  d.V = a.V;
  d.src = a.src;
  d.src_plan = a.src_plan_order ? 1 : 0;
  d.absmax = p.absmax;
  d.nitems = (int)p.nsitems;
  d.cgroups = a.groups;
  return d;
}

bool spread_args_ok(const sdn_plan_s &p, const SpreadArgs &a) {
  if (p.M == 0 || p.sitems == nullptr) return false;
  if (a.src_plan_order && a.V == nullptr) return false;
  if (p.nslots > 0 && a.part == nullptr) return false;
  return a.K >= 1 && a.K <= kMaxK;
}

// The matrix engines' value scale: the largest component of the values
// (unless the interpolation that produced them recorded it) and of V.
hipError_t spread_scale(const sdn_plan_s &p, const SpreadArgs &a, hipStream_t st) {
  if (a.src_max_ready) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, p.absmax + 1, 1);
  } else {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, p.absmax, 2);
    const size_t nsrc = (size_t)a.groups * p.M;
    const unsigned nblk = (unsigned)std::min<size_t>(2048, (nsrc + 1023) / 1024);
    hipLaunchKernelGGL(k_absmax, dim3(nblk), dim3(256), 0, st, a.src, nsrc, p.absmax);
  }
  hipLaunchKernelGGL(k_absmax, dim3(1), dim3(256), 0, st, a.V, (size_t)p.T * a.K, p.absmax + 1);
  return hipGetLastError();
}

hipError_t spread_engine_launch(const SpreadDev &d, Fused<SpreadDev> *fz, int engine, int W,
                                bool mix, int K, hipStream_t st) {
  if (engine == SDN_SPREAD_PLANES) {
    switch (W) {
      case 4: return spread_pw<4>(d, fz, K, st);
      case 8: return spread_pw<8>(d, fz, K, st);
      default: return spread_pw<6>(d, fz, K, st);
    }
  }
  if (engine == SDN_SPREAD_MATRIX) {
    switch (W) {
      case 4: return spread_mma<4, true>(d, fz, K, st);
      case 8: return spread_mma<8, true>(d, fz, K, st);
      default: return spread_mma<6, true>(d, fz, K, st);
    }
  }
  switch (W) {
    case 4: return mix ? spread_k<4, true>(d, fz, K, st) : spread_k<4, false>(d, fz, K, st);
    case 8: return mix ? spread_k<8, true>(d, fz, K, st) : spread_k<8, false>(d, fz, K, st);
    default: return mix ? spread_k<6, true>(d, fz, K, st) : spread_k<6, false>(d, fz, K, st);
  }
}

// Sum of the partial blocks of the plan's crowded blocks.
hipError_t spread_reduce(const sdn_plan_s &p, const SpreadDev &d, int K, hipStream_t st) {
  if (p.nsplit == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spread_reduce, dim3((unsigned)p.nsplit, (unsigned)d.groups), dim3(kThreads),
                     0, st, d, (const int4 *)p.splits, K);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_spread(const sdn_plan_s &p, const SpreadArgs &a, hipStream_t st) {
  if (!spread_args_ok(p, a)) return hipErrorInvalidValue;
  const SpreadDev d = spread_dev(p, a);
  const bool mix = a.V != nullptr;
  const int engine = mix ? spread_engine_for(p, a.K, a.groups) : SDN_SPREAD_GATHER;
  hipError_t e = engine != SDN_SPREAD_GATHER ? spread_scale(p, a, st) : hipSuccess;
  if (e != hipSuccess) return e;
  e = spread_engine_launch(d, nullptr, engine, p.W, mix, a.K, st);
  if (e != hipSuccess) return e;
  return spread_reduce(p, d, a.K, st);
}

hipError_t launch_spread_fused(const sdn_plan_s *const *plans, const SpreadArgs *args, int n,
                               hipStream_t st) {
  if (n < 1 || n > kMaxFused) return hipErrorInvalidValue;
  const bool mix = args[0].V != nullptr;
  const int K = args[0].K, groups = args[0].groups, W = plans[0]->W;
  const int engine = mix ? spread_engine_for(*plans[0], K, groups) : SDN_SPREAD_GATHER;
  Fused<SpreadDev> f{};
  f.n = n;
  int total = 0;
  for (int v = 0; v < n; ++v) {
    const sdn_plan_s &p = *plans[v];
    const SpreadArgs &a = args[v];
    if (!spread_args_ok(p, a) || p.W != W || a.K != K || a.groups != groups ||
        (a.V != nullptr) != mix || (mix ? spread_engine_for(p, K, groups) : SDN_SPREAD_GATHER) != engine)
      return hipErrorInvalidValue;
    f.dev[v] = spread_dev(p, a);
    f.start[v] = total;
    total += (int)p.nsitems;
    if (engine != SDN_SPREAD_GATHER) {
      const hipError_t e = spread_scale(p, a, st);
      if (e != hipSuccess) return e;
    }
  }
  f.start[n] = total;
  hipError_t e = spread_engine_launch(f.dev[0], &f, engine, W, mix, K, st);
  for (int v = 0; v < n && e == hipSuccess; ++v) e = spread_reduce(*plans[v], f.dev[v], K, st);
  return e;
}

hipError_t launch_fill_zero(float2 *a, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // n complex = n/2 float4; workspace buffers hold a whole number of float4s
  const size_t n4 = (n + 1) / 2;
  const unsigned blocks = (unsigned)std::min<size_t>((n4 + 255) / 256, 1u << 16);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, st, (float4 *)a, n4);
  return hipGetLastError();
}

namespace {
// Pipe-Menon step on complex-stored real weights: w <- w / Re(C w); w = 1
// when first is set.  Imaginary parts stay zero.
__global__ void k_dcf_step(float2 *w, const float2 *cw, int64_t M, int first) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M;
       j += (int64_t)gridDim.x * blockDim.x) {
    if (first) {
      w[j] = make_float2(1.f, 0.f);
    } else {
      w[j] = make_float2(w[j].x / cw[j].x, 0.f);
    }
  }
}

__global__ void k_real_part(const float2 *w, float *out, int64_t M) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M;
       j += (int64_t)gridDim.x * blockDim.x)
    out[j] = w[j].x;
}
}  // namespace

hipError_t launch_dcf_step(float2 *w, const float2 *cw, int64_t M, bool first, hipStream_t st) {
  if (M == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((M + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(k_dcf_step, dim3(blocks), dim3(256), 0, st, w, cw, M, first ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_real_part(const float2 *w, float *out, int64_t M, hipStream_t st) {
  if (M == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((M + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(k_real_part, dim3(blocks), dim3(256), 0, st, w, out, M);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f64(double *a, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero_f64, dim3(1), dim3(64), 0, st, a, n);
  return hipGetLastError();
}

hipError_t launch_mix_fwd(const sdn_plan_s &p, const float2 *u, const float2 *V, int K, int k,
                          float2 *y, int accumulate, hipStream_t st) {
  if (p.M == 0) return hipSuccess;
  const int M = (int)p.M;
  hipLaunchKernelGGL(k_mix_fwd, dim3((M + 255) / 256), dim3(256), 0, st, u, V, p.frame_user, K,
                     k, M, y, accumulate);
  return hipGetLastError();
}

hipError_t launch_mix_adj(const sdn_plan_s &p, const float2 *r, const float2 *V, int K, int k,
                          float2 *out, hipStream_t st) {
  if (p.M == 0) return hipSuccess;
  const int M = (int)p.M;
  hipLaunchKernelGGL(k_mix_adj, dim3((M + 255) / 256), dim3(256), 0, st, r, V, p.frame_user, K,
                     k, M, out);
  return hipGetLastError();
}

}  // namespace sdn
