// Kernel interpolation (type 2) and spreading (type 1) between the fine
// grids and the nonuniform points, with the temporal-subspace mix fused in.
//
// Points are read in plan order (sorted by fine-grid tile), so neighbouring
// threads touch neighbouring grid cells.  The fine grid is [z][y][x][p]
// with channel p = b K + k innermost: the K channels of one coil at one
// cell are contiguous.
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

struct GridGeom {
  int nfx, nfy, nfz;
  int tbx, tby, tbz;      // tile edges
  int ntx, nty;           // tiles along x and y
};

GridGeom grid_geom(const sdn_plan_s &p) {
  GridGeom g;
  g.nfx = p.ax[0].nf; g.nfy = p.ax[1].nf; g.nfz = p.ax[2].nf;
  g.tbx = p.ax[0].tile; g.tby = p.ax[1].tile; g.tbz = p.ax[2].tile;
  g.ntx = p.ax[0].ntile; g.nty = p.ax[1].ntile;
  return g;
}

struct InterpDev {
  const float4 *rec;
  const int2 *pidx;
  int M;
  GridGeom g;
  const float2 *grid;
  int P, groups, K;
  const float2 *V;
  float2 *y;
  const float2 *d;
  const float *w;
  float2 *r_plan;
  double *loss;
};

// One thread per (point, group).  A group is the K channels of one coil
// (mix mode: output y_b = sum_k V[t][k] u_{b,k}) or a single channel.
template <int W, int NC, int KG, bool MIX, bool DC>
__global__ void __launch_bounds__(256) k_interp(InterpDev a, KerCoef kc) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)(gt / a.groups);
  const int grp = (int)(gt % a.groups);
  double my_loss = 0.0;
  if (j < a.M) {
    const float4 r = a.rec[j];
    const int2 id = a.pidx[j];
    int lx, ly, lz;
    unpack_l0(r.w, lx, ly, lz);
    float wx[W], wy[W], wz[W];
    axis_weights<W, NC>(r.x, kc, wx);
    axis_weights<W, NC>(r.y, kc, wy);
    axis_weights<W, NC>(r.z, kc, wz);
    const GridGeom &g = a.g;
    float2 acc[KG];
#pragma unroll
    for (int q = 0; q < KG; ++q) acc[q] = make_float2(0.f, 0.f);
    int xs[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const int x = lx + i;
      xs[i] = x >= g.nfx ? x - g.nfx : x;
    }
    const float2 *gbase = a.grid + (size_t)grp * KG;
#pragma unroll
    for (int az = 0; az < W; ++az) {
      int zc = lz + az;
      zc = zc >= g.nfz ? zc - g.nfz : zc;
#pragma unroll
      for (int ay = 0; ay < W; ++ay) {
        int yc = ly + ay;
        yc = yc >= g.nfy ? yc - g.nfy : yc;
        const float wzy = wz[az] * wy[ay];
        const float2 *row = gbase + ((size_t)zc * g.nfy + yc) * g.nfx * a.P;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const float ww = wzy * wx[i];
          const float2 *cell = row + (size_t)xs[i] * a.P;
#pragma unroll
          for (int q = 0; q < KG; ++q) {
            const float2 v = cell[q];
            acc[q].x = fmaf(ww, v.x, acc[q].x);
            acc[q].y = fmaf(ww, v.y, acc[q].y);
          }
        }
      }
    }
    const int orig = id.y;
    if constexpr (MIX) {
      const float2 *vr = a.V + (size_t)id.x * a.K;
      float2 yv = make_float2(0.f, 0.f);
#pragma unroll
      for (int q = 0; q < KG; ++q) yv = cadd(yv, cmul(vr[q], acc[q]));
      if constexpr (DC) {
        const float2 dv = a.d[(size_t)grp * a.M + orig];
        const float2 df = csub(yv, dv);
        const float wt = a.w ? a.w[orig] : 1.f;
        my_loss = (double)wt * ((double)df.x * df.x + (double)df.y * df.y);
        a.r_plan[(size_t)grp * a.M + j] = make_float2(2.f * wt * df.x, 2.f * wt * df.y);
      } else {
        a.y[(size_t)grp * a.M + orig] = yv;
      }
    } else {
#pragma unroll
      for (int q = 0; q < KG; ++q) a.y[(size_t)(grp * KG + q) * a.M + orig] = acc[q];
    }
  }
  if constexpr (DC) {
    // block reduction of the loss, one double atomic per block
    __shared__ double part[4];
    for (int off = 32; off > 0; off >>= 1) my_loss += __shfl_down(my_loss, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = my_loss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += part[i];
      atomicAdd(a.loss, s);
    }
  }
}

struct SpreadDev {
  const float4 *rec;
  const int2 *pidx;
  const int4 *work;
  int M;
  GridGeom g;
  float2 *grid;
  int P, K, Pc;
  const float2 *V;
  const float2 *src;
  int src_plan;
};

// One workgroup per (work item, channel chunk): the points of one tile (or
// a slice of a crowded tile) are spread into an LDS copy of the tile plus
// its (W-1)-cell halo, which is then added to the fine grid.  Tiles overlap
// through their halos, so the write-back uses float atomics; cells that
// stayed zero are skipped.
template <int W, int NC, bool MIX>
__global__ void __launch_bounds__(256) k_spread(SpreadDev a, KerCoef kc) {
  extern __shared__ float2 tile[];
  const GridGeom &g = a.g;
  const int4 wi = a.work[blockIdx.x];
  const int tid = threadIdx.x;
  const int tz = wi.x / (g.ntx * g.nty);
  const int rem = wi.x % (g.ntx * g.nty);
  const int ty = rem / g.ntx, tx = rem % g.ntx;
  const int ox = tx * g.tbx, oy = ty * g.tby, oz = tz * g.tbz;
  const int PX = g.tbx + W - 1, PY = g.tby + W - 1, PZ = g.tbz + W - 1;
  const int ncell = PX * PY * PZ;
  const int p0 = blockIdx.y * a.Pc;
  const int pc = min(a.Pc, a.P - p0);
  const int Pc = a.Pc;
  for (int e = tid; e < ncell * Pc; e += 256) tile[e] = make_float2(0.f, 0.f);
  __syncthreads();
  const int slots = 256 / Pc;
  const int slot = tid / Pc, pp = tid % Pc;
  if (slot < slots && pp < pc) {
    const int p = p0 + pp;
    for (int q = slot; q < wi.z; q += slots) {
      const int j = wi.y + q;
      const float4 r = a.rec[j];
      const int2 id = a.pidx[j];
      const int col = a.src_plan ? j : id.y;
      float2 val;
      if constexpr (MIX) {
        const int b = p / a.K, k = p % a.K;
        val = cmulc(a.src[(size_t)b * a.M + col], a.V[(size_t)id.x * a.K + k]);
      } else {
        val = a.src[(size_t)p * a.M + col];
      }
      int lx, ly, lz;
      unpack_l0(r.w, lx, ly, lz);
      lx -= ox; ly -= oy; lz -= oz;
      float wx[W], wy[W], wz[W];
      axis_weights<W, NC>(r.x, kc, wx);
      axis_weights<W, NC>(r.y, kc, wy);
      axis_weights<W, NC>(r.z, kc, wz);
#pragma unroll
      for (int az = 0; az < W; ++az) {
#pragma unroll
        for (int ay = 0; ay < W; ++ay) {
          const float wzy = wz[az] * wy[ay];
          float2 *row = tile + ((size_t)((lz + az) * PY + (ly + ay)) * PX + lx) * Pc + pp;
#pragma unroll
          for (int i = 0; i < W; ++i) {
            const float ww = wzy * wx[i];
            atomicAdd(&row[i * Pc].x, ww * val.x);
            atomicAdd(&row[i * Pc].y, ww * val.y);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < ncell * pc; e += 256) {
    const int q = e % pc, cell = e / pc;
    const float2 v = tile[cell * Pc + q];
    if (v.x == 0.f && v.y == 0.f) continue;
    const int cx = cell % PX, cyz = cell / PX;
    const int cy = cyz % PY, cz = cyz / PY;
    int gx = ox + cx, gy = oy + cy, gz = oz + cz;
    gx = gx >= g.nfx ? gx - g.nfx : gx;
    gy = gy >= g.nfy ? gy - g.nfy : gy;
    gz = gz >= g.nfz ? gz - g.nfz : gz;
    float2 *dst = a.grid + (((size_t)gz * g.nfy + gy) * g.nfx + gx) * a.P + p0 + q;
    unsafeAtomicAdd(&dst->x, v.x);
    unsafeAtomicAdd(&dst->y, v.y);
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

template <int W, int NC>
hipError_t interp_dispatch_kg(const InterpDev &d, const KerCoef &kc, int kg, bool mix, bool dc,
                              dim3 grd, hipStream_t st) {
#define SDN_INTERP(KGV)                                                                     \
  case KGV:                                                                                 \
    if (mix && dc)                                                                          \
      hipLaunchKernelGGL((k_interp<W, NC, KGV, true, true>), grd, dim3(256), 0, st, d, kc); \
    else if (mix)                                                                           \
      hipLaunchKernelGGL((k_interp<W, NC, KGV, true, false>), grd, dim3(256), 0, st, d, kc);\
    else                                                                                    \
      hipLaunchKernelGGL((k_interp<W, NC, KGV, false, false>), grd, dim3(256), 0, st, d, kc);\
    break;
  switch (kg) {
    SDN_INTERP(1)
    SDN_INTERP(2)
    SDN_INTERP(3)
    SDN_INTERP(4)
    SDN_INTERP(5)
    SDN_INTERP(6)
    SDN_INTERP(7)
    SDN_INTERP(8)
    default: return hipErrorInvalidValue;
  }
#undef SDN_INTERP
  return hipGetLastError();
}

}  // namespace

hipError_t launch_interp(const sdn_plan_s &p, const InterpArgs &a, hipStream_t st) {
  if (p.M == 0) return hipSuccess;
  InterpDev d;
  d.rec = p.rec;
  d.pidx = p.pidx;
  d.M = (int)p.M;
  d.g = grid_geom(p);
  d.grid = a.grid;
  d.P = a.P;
  d.groups = a.groups;
  d.K = a.kg;
  d.V = a.V;
  d.y = a.y;
  d.d = a.d;
  d.w = a.w;
  d.r_plan = a.r_plan;
  d.loss = a.loss;
  const bool mix = a.V != nullptr;
  const bool dc = a.d != nullptr;
  const int64_t nthr = (int64_t)p.M * a.groups;
  dim3 grd((unsigned)((nthr + 255) / 256));
  switch (p.W) {
    case 4: return interp_dispatch_kg<4, 8>(d, p.coef, a.kg, mix, dc, grd, st);
    case 8: return interp_dispatch_kg<8, 12>(d, p.coef, a.kg, mix, dc, grd, st);
    default: return interp_dispatch_kg<6, 10>(d, p.coef, a.kg, mix, dc, grd, st);
  }
}

hipError_t launch_spread(const sdn_plan_s &p, const SpreadArgs &a, hipStream_t st) {
  if (p.M == 0 || p.nwork == 0) return hipSuccess;
  SpreadDev d;
  d.rec = p.rec;
  d.pidx = p.pidx;
  d.work = p.work;
  d.M = (int)p.M;
  d.g = grid_geom(p);
  d.grid = a.grid;
  d.P = a.P;
  d.K = a.K;
  d.V = a.V;
  d.src = a.src;
  d.src_plan = a.src_plan_order ? 1 : 0;
  const int ncell = (d.g.tbx + p.W - 1) * (d.g.tby + p.W - 1) * (d.g.tbz + p.W - 1);
  const int max_pc = std::max(1, (int)(65536 / (sizeof(float2) * (size_t)ncell)));
  d.Pc = std::min(a.P, std::min(max_pc, 256));
  const size_t lds = (size_t)ncell * d.Pc * sizeof(float2);
  dim3 grd((unsigned)p.nwork, (unsigned)((a.P + d.Pc - 1) / d.Pc));
  const bool mix = a.V != nullptr;
  switch (p.W) {
    case 4:
      if (mix) hipLaunchKernelGGL((k_spread<4, 8, true>), grd, dim3(256), lds, st, d, p.coef);
      else hipLaunchKernelGGL((k_spread<4, 8, false>), grd, dim3(256), lds, st, d, p.coef);
      break;
    case 8:
      if (mix) hipLaunchKernelGGL((k_spread<8, 12, true>), grd, dim3(256), lds, st, d, p.coef);
      else hipLaunchKernelGGL((k_spread<8, 12, false>), grd, dim3(256), lds, st, d, p.coef);
      break;
    default:
      if (mix) hipLaunchKernelGGL((k_spread<6, 10, true>), grd, dim3(256), lds, st, d, p.coef);
      else hipLaunchKernelGGL((k_spread<6, 10, false>), grd, dim3(256), lds, st, d, p.coef);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_fill_zero(float2 *a, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // n complex = n/2 float4 (+ one float2 tail handled by rounding up the
  // buffer: workspace buffers are allocated in whole float4s)
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
