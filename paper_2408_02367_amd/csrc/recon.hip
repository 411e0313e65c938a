// Image-space kernels around the operator: the total-variation penalty of
// Alg. 1 (StoDIP + TV) and the reductions and vector updates of the
// conjugate-gradient and scaled-adjoint initialisers of Sec. 2.2.
//
// All of these are HBM-bound streams over K image volumes.  Sums are taken
// in FP64 in two fixed-order passes (per-block partials, then one block),
// so a result does not depend on scheduling, and the scalars of an
// iteration (alpha, beta, the adjoint's scale) are formed on the device
// from those sums: a whole solve is enqueued without a host round trip.

#include <algorithm>

#include "sdn_internal.h"

namespace sdn {
namespace {

constexpr int kRedThreads = 256;

// Sum of one double per thread of a 256-thread block (1D, or 2D with
// blockDim.x a multiple of 64), in a fixed order; the result is valid in
// thread 0.
__device__ double block_sum(double v) {
  __shared__ double part[kRedThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  if ((tid & 63) == 0) part[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int i = 0; i < kRedThreads / 64; ++i) s += part[i];
  return s;
}

__global__ void __launch_bounds__(kRedThreads) k_dot(const float2 *__restrict__ a,
                                                     const float2 *__restrict__ b, size_t n,
                                                     double *__restrict__ part) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kRedThreads) {
    const float2 u = a[i], v = b[i];
    s += (double)u.x * v.x + (double)u.y * v.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads) k_sum(const double *__restrict__ part, int n,
                                                     double scale, double *__restrict__ out,
                                                     int accumulate) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kRedThreads) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *out = accumulate ? *out + scale * s : scale * s;
}

// First level of a long sum: block b adds the b-th contiguous chunk.
__global__ void __launch_bounds__(kRedThreads) k_sum_chunks(const double *__restrict__ part,
                                                            int n, double *__restrict__ out) {
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double s = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += kRedThreads) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void k_weighted_plan(const int2 *__restrict__ pidx, int M, const float2 *__restrict__ y,
                                const float *__restrict__ w, float scale, float2 *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int g = blockIdx.y;
  const int orig = pidx[j].y;
  const float s = w ? scale * w[orig] : scale;
  const float2 v = y[(size_t)g * M + orig];
  out[(size_t)j * gridDim.y + g] = make_float2(s * v.x, s * v.y);
}

__global__ void __launch_bounds__(kRedThreads) k_axpy_dot(float2 *__restrict__ y,
                                                          const float2 *__restrict__ x, float lam,
                                                          size_t n, double *__restrict__ part) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kRedThreads) {
    const float2 u = x[i];
    float2 v = y[i];
    v.x = fmaf(lam, u.x, v.x);
    v.y = fmaf(lam, u.y, v.y);
    y[i] = v;
    s += (double)u.x * v.x + (double)u.y * v.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// r holds b on entry; g is the normal operator applied to the start point
__global__ void __launch_bounds__(kRedThreads) k_cg_start(float2 *__restrict__ r,
                                                          float2 *__restrict__ p,
                                                          const float2 *__restrict__ g, size_t n,
                                                          double *__restrict__ part) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kRedThreads) {
    const float2 b = r[i], gi = g[i];
    const float2 v = make_float2(b.x - gi.x, b.y - gi.y);
    r[i] = v;
    p[i] = v;
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads) k_cg_xr(float2 *__restrict__ x,
                                                       float2 *__restrict__ r,
                                                       const float2 *__restrict__ p,
                                                       const float2 *__restrict__ Ap, size_t n,
                                                       const double *__restrict__ rs,
                                                       const double *__restrict__ pAp,
                                                       double *__restrict__ part) {
  const double den = *pAp;
  const float alpha = den > 0.0 ? (float)(*rs / den) : 0.f;
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kRedThreads) {
    const float2 pi = p[i], api = Ap[i];
    float2 xi = x[i], ri = r[i];
    xi.x = fmaf(alpha, pi.x, xi.x);
    xi.y = fmaf(alpha, pi.y, xi.y);
    ri.x = fmaf(-alpha, api.x, ri.x);
    ri.y = fmaf(-alpha, api.y, ri.y);
    x[i] = xi;
    r[i] = ri;
    s += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_cg_p(float2 *__restrict__ p, const float2 *__restrict__ r, size_t n,
                       const double *__restrict__ rs_new, const double *__restrict__ rs) {
  const double den = *rs;
  const float beta = den > 0.0 ? (float)(*rs_new / den) : 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float2 ri = r[i];
    float2 pi = p[i];
    pi.x = fmaf(beta, pi.x, ri.x);
    pi.y = fmaf(beta, pi.y, ri.y);
    p[i] = pi;
  }
}

__global__ void k_scale_ratio(float2 *__restrict__ x, size_t n, const double *__restrict__ num,
                              const double *__restrict__ den, double *__restrict__ s_out) {
  const double d = *den;
  const double sd = d > 0.0 ? *num / d : 0.0;
  const float s = (float)sd;
  if (s_out && blockIdx.x == 0 && threadIdx.x == 0) *s_out = sd;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float2 v = x[i];
    x[i] = make_float2(s * v.x, s * v.y);
  }
}

// ----------------------------------------------------------------------- TV
// One thread per voxel m of channel k.  With u_d[n] the forward difference
// along axis d (zero at the last index) and t[n] = sqrt(sum_d |u_d[n]|^2 +
// eps^2), the gradient is sum_d (u_d[m - e_d] / t[m - e_d] - u_d[m] / t[m]),
// the first term present when m_d > 0; it needs t at m and at its three
// lower neighbours, i.e. x at m, m +- e_d and m - e_d + e_d'.  The voxel's
// own term t[m] goes into the block's partial sum of the value.
struct TvDev {
  const float2 *x;
  float2 *grad;
  double *part;
  int nx, ny, nz;
  size_t nvox, total;
  float eps2, lam;
  int accumulate;
};

__device__ __forceinline__ float tv_term(const float2 *xc, int x, int y, int z, int nx, int ny,
                                         int nz, float eps2, float2 &ux, float2 &uy, float2 &uz) {
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const size_t i = ((size_t)z * ny + y) * nx + x;
  const float2 c = xc[i];
  ux = uy = uz = make_float2(0.f, 0.f);
  if (x + 1 < nx) {
    const float2 v = xc[i + 1];
    ux = make_float2(v.x - c.x, v.y - c.y);
  }
  if (y + 1 < ny) {
    const float2 v = xc[i + sy];
    uy = make_float2(v.x - c.x, v.y - c.y);
  }
  if (z + 1 < nz) {
    const float2 v = xc[i + sz];
    uz = make_float2(v.x - c.x, v.y - c.y);
  }
  const float s = ux.x * ux.x + ux.y * ux.y + uy.x * uy.x + uy.y * uy.y + uz.x * uz.x +
                  uz.y * uz.y + eps2;
  // 1 / t from the hardware reciprocal square root (s >= eps^2 > 0); the
  // caller forms t = s / t and the quotients u / t by multiplication
  return rsqrtf(s);
}

// Grid (ceil(Nx / 64), ceil(Ny / 4), Nz K), block 64 x 4: the voxel's
// (x, y, z, k) comes from the indices without per-voxel divisions.
__global__ void __launch_bounds__(kRedThreads) k_tv(TvDev a) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z / a.nz, z = blockIdx.z - k * a.nz;
  double own = 0.0;
  if (x < a.nx && y < a.ny) {
    const size_t gi = (size_t)k * a.nvox + ((size_t)z * a.ny + y) * a.nx + x;
    const float2 *xc = a.x + (size_t)k * a.nvox;
    float2 ux, uy, uz;
    const float it = tv_term(xc, x, y, z, a.nx, a.ny, a.nz, a.eps2, ux, uy, uz);
    const float s = ux.x * ux.x + ux.y * ux.y + uy.x * uy.x + uy.y * uy.y + uz.x * uz.x +
                    uz.y * uz.y + a.eps2;
    own = (double)(s * it);   // t = s / sqrt(s)
    if (a.grad) {
      float gx = -(ux.x + uy.x + uz.x) * it;
      float gy = -(ux.y + uy.y + uz.y) * it;
      float2 px, py, pz;
      if (x > 0) {
        const float itn = tv_term(xc, x - 1, y, z, a.nx, a.ny, a.nz, a.eps2, px, py, pz);
        gx = fmaf(px.x, itn, gx);
        gy = fmaf(px.y, itn, gy);
      }
      if (y > 0) {
        const float itn = tv_term(xc, x, y - 1, z, a.nx, a.ny, a.nz, a.eps2, px, py, pz);
        gx = fmaf(py.x, itn, gx);
        gy = fmaf(py.y, itn, gy);
      }
      if (z > 0) {
        const float itn = tv_term(xc, x, y, z - 1, a.nx, a.ny, a.nz, a.eps2, px, py, pz);
        gx = fmaf(pz.x, itn, gx);
        gy = fmaf(pz.y, itn, gy);
      }
      float2 g = make_float2(a.lam * gx, a.lam * gy);
      if (a.accumulate) {
        const float2 o = a.grad[gi];
        g.x += o.x;
        g.y += o.y;
      }
      a.grad[gi] = g;
    }
  }
  own = block_sum(own);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    a.part[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = own;
}

unsigned stream_blocks(size_t n) {
  return (unsigned)std::min<size_t>((n + kRedThreads - 1) / kRedThreads, kDotBlocks);
}

}  // namespace

hipError_t launch_dot(const float2 *a, const float2 *b, size_t n, double *part, hipStream_t st) {
  hipLaunchKernelGGL(k_dot, dim3(kDotBlocks), dim3(kRedThreads), 0, st, a, b, n, part);
  return hipGetLastError();
}

hipError_t launch_sum(const double *part, int n, double scale, double *out, hipStream_t st,
                      double *scratch, bool accumulate) {
  if (scratch && n > 16 * kRedThreads) {
    hipLaunchKernelGGL(k_sum_chunks, dim3(kSumChunks), dim3(kRedThreads), 0, st, part, n,
                       scratch);
    part = scratch;
    n = kSumChunks;
  }
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kRedThreads), 0, st, part, n, scale, out,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_weighted_plan(const sdn_plan_s &p, const float2 *y, int groups, const float *w,
                                float scale, float2 *out, hipStream_t st) {
  if (p.M == 0) return hipSuccess;
  dim3 grd((unsigned)((p.M + 255) / 256), (unsigned)groups);
  hipLaunchKernelGGL(k_weighted_plan, grd, dim3(256), 0, st, p.pidx, (int)p.M, y, w, scale, out);
  return hipGetLastError();
}

hipError_t launch_axpy_dot(float2 *y, const float2 *x, float lam, size_t n, double *part,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_dot, dim3(kDotBlocks), dim3(kRedThreads), 0, st, y, x, lam, n, part);
  return hipGetLastError();
}

hipError_t launch_cg_start(float2 *r, float2 *p, const float2 *g, size_t n, double *part,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_cg_start, dim3(kDotBlocks), dim3(kRedThreads), 0, st, r, p, g, n, part);
  return hipGetLastError();
}

hipError_t launch_cg_xr(float2 *x, float2 *r, const float2 *p, const float2 *Ap, size_t n,
                        const double *rs, const double *pAp, double *part, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_xr, dim3(kDotBlocks), dim3(kRedThreads), 0, st, x, r, p, Ap, n, rs, pAp,
                     part);
  return hipGetLastError();
}

hipError_t launch_cg_p(float2 *p, const float2 *r, size_t n, const double *rs_new,
                       const double *rs, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_p, dim3(stream_blocks(n)), dim3(kRedThreads), 0, st, p, r, n, rs_new, rs);
  return hipGetLastError();
}

hipError_t launch_scale_ratio(float2 *x, size_t n, const double *num, const double *den,
                              double *s_out, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_ratio, dim3(stream_blocks(n)), dim3(kRedThreads), 0, st, x, n, num,
                     den, s_out);
  return hipGetLastError();
}

dim3 tv_grid(const sdn_plan_s &p, int K) {
  return dim3((unsigned)((p.ax[0].N + 63) / 64), (unsigned)((p.ax[1].N + 3) / 4),
              (unsigned)(K * p.ax[2].N));
}

int tv_blocks(const sdn_plan_s &p, int K) {
  const dim3 g = tv_grid(p, K);
  return (int)(g.x * g.y * g.z);
}

hipError_t launch_tv(const sdn_plan_s &p, const float2 *x, int K, float eps, float lam,
                     float2 *grad, int accumulate, double *part, hipStream_t st) {
  TvDev a;
  a.x = x;
  a.grad = grad;
  a.part = part;
  a.nx = (int)p.ax[0].N;
  a.ny = (int)p.ax[1].N;
  a.nz = (int)p.ax[2].N;
  a.nvox = (size_t)a.nx * a.ny * a.nz;
  a.total = (size_t)K * a.nvox;
  a.eps2 = eps * eps;
  a.lam = lam;
  a.accumulate = accumulate;
  if ((int64_t)K * p.ax[2].N > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tv, tv_grid(p, K), dim3(64, 4), 0, st, a);
  return hipGetLastError();
}

}  // namespace sdn
