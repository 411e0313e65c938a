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
//   subspace mix y_b = sum_k V[t][k] u_{b,k} in registers;
// * spreading: a workgroup owns one output tile.  It walks the plan's list
//   of points whose kernel support touches the tile, accumulates their
//   contributions (with the conjugate mix) into the tile in LDS, and writes
//   the tile once with coalesced stores - no global atomics and no separate
//   clear of the grid, since every tile is written exactly once.
#include <algorithm>

#include "fft_lds.h"
#include "sdn_internal.h"

namespace sdn {

namespace {

// Node weights of one axis: piece i of the kernel polynomial at z = 2t - 1.
template <int W, int NC>
__device__ __forceinline__ void axis_weights(float t, const KerCoef &kc, float (&w)[W]) {
  const float z = 2.f * t - 1.f;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    float acc = kc.c[i][NC - 1];
#pragma unroll
    for (int d = NC - 2; d >= 0; --d) acc = fmaf(acc, z, kc.c[i][d]);
    w[i] = acc;
  }
}

__device__ __forceinline__ void unpack_l0(float bits, int &lx, int &ly, int &lz) {
  const unsigned u = __float_as_uint(bits);
  lx = (int)(u & 1023u);
  ly = (int)((u >> 10) & 1023u);
  lz = (int)((u >> 20) & 1023u);
}

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

struct InterpDev {
  const float4 *rec;
  const int2 *pidx;
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
  double *loss;
};

constexpr int kThreads = 256;
constexpr int kIThreads = 512;                // interpolation workgroup
constexpr int kPPT = kItemCap / kIThreads;    // points per thread per item

// grid = (items, groups).  Mix mode: a group is one coil and its K channels,
// output y_b = sum_k V[t][k] u_k (+ DC epilogue), the running sums kept in
// LDS behind the staged tile.  Otherwise a group is K independent channels
// with outputs y_{gK+k} = u_k.
template <int W, int NC, bool MIX, bool DC>
__global__ void __launch_bounds__(kIThreads) k_interp(InterpDev a, KerCoef kc) {
  extern __shared__ float2 tile[];
  const TileGeom &g = a.g;
  const int4 wi = a.work[blockIdx.x];
  const int grp = blockIdx.y;
  const int tid = threadIdx.x;
  const int tz = wi.x / (g.ntx * g.nty);
  const int rem = wi.x - tz * (g.ntx * g.nty);
  const int ty = rem / g.ntx, tx = rem - ty * g.ntx;
  const int ox = tx * g.bx, oy = ty * g.by, oz = tz * g.bz;
  const int PX = g.bx + W - 1, PY = g.by + W - 1, PZ = g.bz + W - 1;
  const int ncell = PX * PY * PZ;
  float2 *acc = tile + ncell;   // [kItemCap] running subspace sums (mix mode)

  if constexpr (MIX) {
    for (int q = tid; q < wi.z; q += kIThreads) acc[q] = make_float2(0.f, 0.f);
  }
  for (int k = 0; k < a.K; ++k) {
    const float2 *gp = a.grid + (size_t)(grp * a.K + k) * g.G;
    for (int e = tid; e < ncell; e += kIThreads) {
      const int row = fdiv(e, a.inv_px);
      const int cx = e - row * PX;
      const int cz = fdiv(row, a.inv_py);
      const int cy = row - cz * PY;
      const int gx = wrap(ox + cx, g.nfx), gy = wrap(oy + cy, g.nfy), gz = wrap(oz + cz, g.nfz);
      tile[e] = gp[((size_t)gz * g.nfy + gy) * g.nfx + gx];
    }
    __syncthreads();
#pragma unroll 1
    for (int q = tid; q < wi.z; q += kIThreads) {
      const float4 rc = a.rec[wi.y + q];
      const int2 id = a.pidx[wi.y + q];
      int lx, ly, lz;
      unpack_l0(rc.w, lx, ly, lz);
      lx -= ox; ly -= oy; lz -= oz;
      float wx[W], wy[W], wz[W];
      axis_weights<W, NC>(rc.x, kc, wx);
      axis_weights<W, NC>(rc.y, kc, wy);
      axis_weights<W, NC>(rc.z, kc, wz);
      float ur = 0.f, ui = 0.f;
#pragma unroll
      for (int az = 0; az < W; ++az) {
#pragma unroll
        for (int ay = 0; ay < W; ++ay) {
          const float2 *row = tile + ((lz + az) * PY + (ly + ay)) * PX + lx;
          float tr = 0.f, ti = 0.f;
#pragma unroll
          for (int i = 0; i < W; ++i) {
            const float2 v = row[i];
            tr = fmaf(wx[i], v.x, tr);
            ti = fmaf(wx[i], v.y, ti);
          }
          const float wzy = wz[az] * wy[ay];
          ur = fmaf(wzy, tr, ur);
          ui = fmaf(wzy, ti, ui);
        }
      }
      const float2 u = make_float2(ur, ui);
      if constexpr (MIX) {
        acc[q] = cadd(acc[q], cmul(a.V[(size_t)id.x * a.K + k], u));
      } else {
        a.y[(size_t)(grp * a.K + k) * a.M + id.y] = u;
      }
    }
    __syncthreads();
  }
  if constexpr (MIX) {
    double my_loss = 0.0;
    for (int q = tid; q < wi.z; q += kIThreads) {
      const int orig = a.pidx[wi.y + q].y;
      if constexpr (DC) {
        const float2 dv = a.d[(size_t)grp * a.M + orig];
        const float2 df = csub(acc[q], dv);
        const float wt = a.w ? a.w[orig] : 1.f;
        my_loss += (double)wt * ((double)df.x * df.x + (double)df.y * df.y);
        a.r_plan[(size_t)grp * a.M + wi.y + q] = make_float2(2.f * wt * df.x, 2.f * wt * df.y);
      } else {
        a.y[(size_t)grp * a.M + orig] = acc[q];
      }
    }
    if constexpr (DC) {
      __shared__ double part[kIThreads / 64];
      for (int off = 32; off > 0; off >>= 1) my_loss += __shfl_down(my_loss, off, 64);
      if ((tid & 63) == 0) part[tid >> 6] = my_loss;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < kIThreads / 64; ++i) s += part[i];
        atomicAdd(a.loss, s);
      }
    }
  }
}

struct SpreadDev {
  const float4 *rec;
  const int2 *pidx;
  const int4 *items;
  const int *vlist;
  int M;
  TileGeom g;
  float inv_bx, inv_bxy;
  float2 *grid;
  float2 *part;        // [slot][group][K][tile cells]
  int groups;
  int K;               // channels per group
  int KC;              // channels per LDS pass
  const float2 *V;
  const float2 *src;   // mix: [groups][M]; else [groups * K][M]
  int src_plan;
};

constexpr int kMaxKC = 8;

// grid = (items, groups).  An item is one tile's spreading list (or a slice
// of a crowded tile's list) for one group's channels.  An unsplit item owns
// its tile and writes it to the grid; a slice writes a partial tile to its
// slot, summed by k_spread_reduce.
template <int W, int NC, bool MIX>
__global__ void __launch_bounds__(kThreads) k_spread(SpreadDev a, KerCoef kc) {
  extern __shared__ float acc[];   // [cell][KC] complex as float pairs
  const TileGeom &g = a.g;
  const int4 it = a.items[blockIdx.x];
  const int T = it.x;
  const int grp = blockIdx.y;
  const int tid = threadIdx.x;
  const int tz = T / (g.ntx * g.nty);
  const int rem = T - tz * (g.ntx * g.nty);
  const int ty = rem / g.ntx, tx = rem - ty * g.ntx;
  const int ox = tx * g.bx, oy = ty * g.by, oz = tz * g.bz;
  const int ex = min(g.bx, g.nfx - ox), ey = min(g.by, g.nfy - oy), ez = min(g.bz, g.nfz - oz);
  const int ncell = g.bx * g.by * g.bz;
  const int v0 = it.y, nv = it.z;
  const int KC = a.KC;
  for (int k0 = 0; k0 < a.K; k0 += KC) {
    const int kcn = min(KC, a.K - k0);
    for (int e = tid; e < ncell * KC * 2; e += kThreads) acc[e] = 0.f;
    __syncthreads();
    for (int e = tid; e < nv; e += kThreads) {
      const int j = a.vlist[v0 + e];
      const float4 r = a.rec[j];
      const int2 id = a.pidx[j];
      const int col = a.src_plan ? j : id.y;
      float2 val[kMaxKC];
      if constexpr (MIX) {
        const float2 rv = a.src[(size_t)grp * a.M + col];
#pragma unroll
        for (int kk = 0; kk < kMaxKC; ++kk)
          if (kk < kcn) val[kk] = cmulc(rv, a.V[(size_t)id.x * a.K + k0 + kk]);
      } else {
#pragma unroll
        for (int kk = 0; kk < kMaxKC; ++kk)
          if (kk < kcn) val[kk] = a.src[(size_t)(grp * a.K + k0 + kk) * a.M + col];
      }
      int l0x, l0y, l0z;
      unpack_l0(r.w, l0x, l0y, l0z);
      float wx[W], wy[W], wz[W];
      axis_weights<W, NC>(r.x, kc, wx);
      axis_weights<W, NC>(r.y, kc, wy);
      axis_weights<W, NC>(r.z, kc, wz);
      int lx[W], ly[W], lz[W];
#pragma unroll
      for (int i = 0; i < W; ++i) {
        lx[i] = wrap(l0x + i, g.nfx) - ox;
        ly[i] = wrap(l0y + i, g.nfy) - oy;
        lz[i] = wrap(l0z + i, g.nfz) - oz;
      }
#pragma unroll
      for (int az = 0; az < W; ++az) {
        if (lz[az] < 0 || lz[az] >= ez) continue;
#pragma unroll
        for (int ay = 0; ay < W; ++ay) {
          if (ly[ay] < 0 || ly[ay] >= ey) continue;
          const float wzy = wz[az] * wy[ay];
          const int rowc = (lz[az] * g.by + ly[ay]) * g.bx;
#pragma unroll
          for (int i = 0; i < W; ++i) {
            if (lx[i] < 0 || lx[i] >= ex) continue;
            const float w = wzy * wx[i];
            float *cell = acc + (size_t)(rowc + lx[i]) * KC * 2;
#pragma unroll
            for (int kk = 0; kk < kMaxKC; ++kk) {
              if (kk < kcn) {
                atomicAdd(cell + 2 * kk, w * val[kk].x);
                atomicAdd(cell + 2 * kk + 1, w * val[kk].y);
              }
            }
          }
        }
      }
    }
    __syncthreads();
    for (int kk = 0; kk < kcn; ++kk) {
      const int ch = grp * a.K + k0 + kk;
      if (it.w < 0) {
        float2 *gp = a.grid + (size_t)ch * g.G;
        for (int c = tid; c < ncell; c += kThreads) {
          const int rowi = fdiv(c, a.inv_bx);
          const int cx = c - rowi * g.bx;
          const int cz = fdiv(c, a.inv_bxy);
          const int cy = rowi - cz * g.by;
          if (cx < ex && cy < ey && cz < ez) {
            const float *sv = acc + (size_t)c * KC * 2 + 2 * kk;
            gp[((size_t)(oz + cz) * g.nfy + (oy + cy)) * g.nfx + (ox + cx)] =
                make_float2(sv[0], sv[1]);
          }
        }
      } else {
        float2 *pp = a.part + ((size_t)it.w * a.groups * a.K + ch) * ncell;
        for (int c = tid; c < ncell; c += kThreads) {
          const float *sv = acc + (size_t)c * KC * 2 + 2 * kk;
          pp[c] = make_float2(sv[0], sv[1]);
        }
      }
    }
    __syncthreads();
  }
}

// grid = (split tiles, groups): sum the partial tiles of a crowded tile.
__global__ void __launch_bounds__(kThreads) k_spread_reduce(SpreadDev a, const int4 *splits) {
  const TileGeom &g = a.g;
  const int4 sp = splits[blockIdx.x];
  const int T = sp.x;
  const int grp = blockIdx.y;
  const int tz = T / (g.ntx * g.nty);
  const int rem = T - tz * (g.ntx * g.nty);
  const int ty = rem / g.ntx, tx = rem - ty * g.ntx;
  const int ox = tx * g.bx, oy = ty * g.by, oz = tz * g.bz;
  const int ex = min(g.bx, g.nfx - ox), ey = min(g.by, g.nfy - oy), ez = min(g.bz, g.nfz - oz);
  const int ncell = g.bx * g.by * g.bz;
  for (int k = 0; k < a.K; ++k) {
    const int ch = grp * a.K + k;
    float2 *gp = a.grid + (size_t)ch * g.G;
    for (int c = threadIdx.x; c < ncell; c += kThreads) {
      const int rowi = fdiv(c, a.inv_bx);
      const int cx = c - rowi * g.bx;
      const int cz = fdiv(c, a.inv_bxy);
      const int cy = rowi - cz * g.by;
      if (cx >= ex || cy >= ey || cz >= ez) continue;
      float sr = 0.f, si = 0.f;
      for (int q = 0; q < sp.z; ++q) {
        const float2 v = a.part[((size_t)(sp.y + q) * a.groups * a.K + ch) * ncell + c];
        sr += v.x;
        si += v.y;
      }
      gp[((size_t)(oz + cz) * g.nfy + (oy + cy)) * g.nfx + (ox + cx)] = make_float2(sr, si);
    }
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
  return ((size_t)(p.ax[0].tile + p.W - 1) * (p.ax[1].tile + p.W - 1) * (p.ax[2].tile + p.W - 1) +
          kItemCap) * sizeof(float2);
}

namespace {

template <int W, int NC>
hipError_t interp_launch(const InterpDev &d, const KerCoef &kc, bool mix, bool dc, dim3 grd,
                         size_t lds, hipStream_t st) {
  if (mix && dc)
    hipLaunchKernelGGL((k_interp<W, NC, true, true>), grd, dim3(kIThreads), lds, st, d, kc);
  else if (mix)
    hipLaunchKernelGGL((k_interp<W, NC, true, false>), grd, dim3(kIThreads), lds, st, d, kc);
  else
    hipLaunchKernelGGL((k_interp<W, NC, false, false>), grd, dim3(kIThreads), lds, st, d, kc);
  return hipGetLastError();
}

}  // namespace

size_t max_lds_bytes() { return 65536; }
size_t spread_cell_bytes(const sdn_plan_s &p) {
  return (size_t)p.ax[0].tile * p.ax[1].tile * p.ax[2].tile * sizeof(float2);
}

hipError_t launch_interp(const sdn_plan_s &p, const InterpArgs &a, hipStream_t st) {
  if (p.M == 0 || p.nwork == 0) return hipSuccess;
  InterpDev d;
  d.rec = p.rec;
  d.pidx = p.pidx;
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
  d.loss = a.loss;
  const bool mix = a.V != nullptr;
  const bool dc = a.d != nullptr;
  const size_t lds = interp_lds_bytes(p);
  if (lds > max_lds_bytes()) return hipErrorInvalidValue;
  dim3 grd((unsigned)p.nwork, (unsigned)a.groups);
  switch (p.W) {
    case 4: return interp_launch<4, 8>(d, p.coef, mix, dc, grd, lds, st);
    case 8: return interp_launch<8, 12>(d, p.coef, mix, dc, grd, lds, st);
    default: return interp_launch<6, 10>(d, p.coef, mix, dc, grd, lds, st);
  }
}

size_t spread_part_elems(const sdn_plan_s &p, int groups, int K) {
  return (size_t)p.nslots * groups * K * p.ax[0].tile * p.ax[1].tile * p.ax[2].tile;
}

hipError_t launch_spread(const sdn_plan_s &p, const SpreadArgs &a, hipStream_t st) {
  if (p.M == 0 || p.sitems == nullptr) return hipErrorInvalidValue;
  if (p.nslots > 0 && a.part == nullptr) return hipErrorInvalidValue;
  SpreadDev d;
  d.rec = p.rec;
  d.pidx = p.pidx;
  d.items = p.sitems;
  d.vlist = p.vlist;
  d.M = (int)p.M;
  d.g = tile_geom(p);
  d.inv_bx = 1.0f / (float)d.g.bx;
  d.inv_bxy = 1.0f / (float)(d.g.bx * d.g.by);
  d.grid = a.grid;
  d.part = a.part;
  d.groups = a.groups;
  d.K = a.K;
  d.V = a.V;
  d.src = a.src;
  d.src_plan = a.src_plan_order ? 1 : 0;
  const size_t cell_bytes = spread_cell_bytes(p);
  int kc_max = (int)std::min<size_t>(kMaxKC, max_lds_bytes() / cell_bytes);
  if (kc_max < 1) return hipErrorInvalidValue;
  const int passes = (a.K + kc_max - 1) / kc_max;
  d.KC = (a.K + passes - 1) / passes;
  const size_t lds = (size_t)d.KC * cell_bytes;
  dim3 grd((unsigned)p.nsitems, (unsigned)a.groups);
  const bool mix = a.V != nullptr;
  switch (p.W) {
    case 4:
      if (mix) hipLaunchKernelGGL((k_spread<4, 8, true>), grd, dim3(kThreads), lds, st, d, p.coef);
      else hipLaunchKernelGGL((k_spread<4, 8, false>), grd, dim3(kThreads), lds, st, d, p.coef);
      break;
    case 8:
      if (mix) hipLaunchKernelGGL((k_spread<8, 12, true>), grd, dim3(kThreads), lds, st, d, p.coef);
      else hipLaunchKernelGGL((k_spread<8, 12, false>), grd, dim3(kThreads), lds, st, d, p.coef);
      break;
    default:
      if (mix) hipLaunchKernelGGL((k_spread<6, 10, true>), grd, dim3(kThreads), lds, st, d, p.coef);
      else hipLaunchKernelGGL((k_spread<6, 10, false>), grd, dim3(kThreads), lds, st, d, p.coef);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.nsplit == 0) return e;
  hipLaunchKernelGGL(k_spread_reduce, dim3((unsigned)p.nsplit, (unsigned)a.groups), dim3(kThreads),
                     0, st, d, (const int4 *)p.splits);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float2 *a, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // n complex = n/2 float4; workspace buffers hold a whole number of float4s
  const size_t n4 = (n + 1) / 2;
  const unsigned blocks = (unsigned)std::min<size_t>((n4 + 255) / 256, 1u << 16);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, st, (float4 *)a, n4);
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
