// The sigma-oversampled 3D FFT of the gridding NUFFT, as three LDS-staged
// line passes over a fine grid stored [z][y][x][p] (P channels innermost).
//
// Forward (image -> fine grid spectrum):
//   x pass: fused with the coil multiply, deapodisation and zero padding -
//           reads x_k and S_c directly, writes only the N_z*N_y lines that
//           hold image data;
//   y pass: reads the N_y nonzero rows of the N_z nonzero planes;
//   z pass: reads the N_z nonzero planes, writes the whole grid.
// Adjoint (fine grid -> image), the same passes reversed with the output
// pruned to the image modes; the last x pass is fused with the crop,
// deapodisation, conj(S_c) multiply and the sum over coils.
#include <algorithm>

#include "fft_lds.h"
#include "sdn_internal.h"

namespace sdn {

namespace {

// fine-grid position of array index q of an axis with N modes
__device__ __forceinline__ int fine_pos(int q, int half, int nf) {
  const int n = q - half;
  return n < 0 ? n + nf : n;
}

struct LineGeom {
  int Nx, Ny, Nz;
  int nfx, nfy, nfz;
  int hx, hy, hz;
};

LineGeom line_geom(const sdn_plan_s &p) {
  LineGeom g;
  g.Nx = p.ax[0].N; g.Ny = p.ax[1].N; g.Nz = p.ax[2].N;
  g.nfx = p.ax[0].nf; g.nfy = p.ax[1].nf; g.nfz = p.ax[2].nf;
  g.hx = p.ax[0].half; g.hy = p.ax[1].half; g.hz = p.ax[2].half;
  return g;
}

struct PreArgs {
  const float2 *x;      // [K][Nz][Ny][Nx]
  const float2 *smaps;  // [C][Nz][Ny][Nx] or null
  CoilList coils;
  int K, P;             // P = B K, channel p = b K + k
  int Pc, NL;           // channels and lines per workgroup
  float2 *grid;         // [nfz][nfy][nfx][P]
  const float *dx, *dy, *dz;
  const float2 *tw;
  RadixPlan rp;
  LineGeom g;
};

__global__ void __launch_bounds__(kFftThreads)
k_pre_fftx(PreArgs a) {
  extern __shared__ float2 smem[];
  const LineGeom &g = a.g;
  const int L = g.nfx;
  const int C = a.NL * a.Pc;
  float2 *lds = smem;
  float2 *tw = smem + L * C;
  const int tid = threadIdx.x;
  const int line0 = blockIdx.x * a.NL;
  const int p0 = blockIdx.y * a.Pc;
  const int nlines = g.Nz * g.Ny;
  for (int m = tid; m < L; m += kFftThreads) tw[m] = a.tw[m];
  // zero the padding rows
  const int nzero = (L - g.Nx) * C;
  for (int e = tid; e < nzero; e += kFftThreads) {
    const int c = e % C, r = e / C;
    const int l = (g.Nx - g.hx) + r;   // rows [N - half, nf - half) are padding
    lds[l * C + c] = make_float2(0.f, 0.f);
  }
  // coil * image / deapodisation, placed at fine positions
  const int nload = a.NL * a.Pc * g.Nx;
  for (int e = tid; e < nload; e += kFftThreads) {
    const int xq = e % g.Nx;
    const int rest = e / g.Nx;
    const int pp = rest % a.Pc, ls = rest / a.Pc;
    const int line = line0 + ls, p = p0 + pp;
    float2 v = make_float2(0.f, 0.f);
    if (line < nlines && p < a.P) {
      const int z = line / g.Ny, y = line % g.Ny;
      const int b = p / a.K, k = p % a.K;
      const size_t vox = ((size_t)z * g.Ny + y) * g.Nx + xq;
      const size_t nvox = (size_t)g.Nz * g.Ny * g.Nx;
      v = a.x[(size_t)k * nvox + vox];
      if (a.smaps) v = cmul(a.smaps[(size_t)a.coils.idx[b] * nvox + vox], v);
      const float s = a.dx[xq] * a.dy[y] * a.dz[z];
      v.x *= s;
      v.y *= s;
    }
    lds[fine_pos(xq, g.hx, L) * C + ls * a.Pc + pp] = v;
  }
  __syncthreads();
  fft_lds<false>(lds, L, C, a.rp, tw);
  // write the transformed lines
  const int nst = a.NL * L * a.Pc;
  for (int e = tid; e < nst; e += kFftThreads) {
    const int pp = e % a.Pc;
    const int rest = e / a.Pc;
    const int l = rest % L, ls = rest / L;
    const int line = line0 + ls, p = p0 + pp;
    if (line >= nlines || p >= a.P) continue;
    const int z = line / g.Ny, y = line % g.Ny;
    const size_t zf = fine_pos(z, g.hz, g.nfz), yf = fine_pos(y, g.hy, g.nfy);
    a.grid[((zf * g.nfy + yf) * L + l) * a.P + p] = lds[l * C + ls * a.Pc + pp];
  }
}

struct PostArgs {
  const float2 *grid;   // [nfz][nfy][nfx][P]
  const float2 *smaps;  // [C][Nz][Ny][Nx] or null
  CoilList coils;
  int K, B, P;
  int Bc, NL;           // coils per chunk, lines per workgroup
  float2 *xout;         // [K][Nz][Ny][Nx]
  int accumulate;
  const float *dx, *dy, *dz;
  const float2 *tw;
  RadixPlan rp;
  LineGeom g;
};

__global__ void __launch_bounds__(kFftThreads)
k_post_ifftx(PostArgs a) {
  extern __shared__ float2 smem[];
  const LineGeom &g = a.g;
  const int L = g.nfx;
  const int Pc = a.Bc * a.K;
  const int C = a.NL * Pc;
  float2 *lds = smem;
  float2 *tw = smem + L * C;
  const int tid = threadIdx.x;
  const int line0 = blockIdx.x * a.NL;
  const int nlines = g.Nz * g.Ny;
  const size_t nvox = (size_t)g.Nz * g.Ny * g.Nx;
  for (int m = tid; m < L; m += kFftThreads) tw[m] = a.tw[m];
  for (int b0 = 0; b0 < a.B; b0 += a.Bc) {
    const int p0 = b0 * a.K;
    const int nld = a.NL * L * Pc;
    for (int e = tid; e < nld; e += kFftThreads) {
      const int pp = e % Pc;
      const int rest = e / Pc;
      const int l = rest % L, ls = rest / L;
      const int line = line0 + ls, p = p0 + pp;
      float2 v = make_float2(0.f, 0.f);
      if (line < nlines && p < a.P) {
        const int z = line / g.Ny, y = line % g.Ny;
        const size_t zf = fine_pos(z, g.hz, g.nfz), yf = fine_pos(y, g.hy, g.nfy);
        v = a.grid[((zf * g.nfy + yf) * L + l) * a.P + p];
      }
      lds[l * C + ls * Pc + pp] = v;
    }
    __syncthreads();
    fft_lds<true>(lds, L, C, a.rp, tw);
    const int nout = a.NL * a.K * g.Nx;
    for (int e = tid; e < nout; e += kFftThreads) {
      const int xq = e % g.Nx;
      const int rest = e / g.Nx;
      const int k = rest % a.K, ls = rest / a.K;
      const int line = line0 + ls;
      if (line >= nlines) continue;
      const int z = line / g.Ny, y = line % g.Ny;
      const size_t vox = ((size_t)z * g.Ny + y) * g.Nx + xq;
      const int l = fine_pos(xq, g.hx, L);
      float2 acc = make_float2(0.f, 0.f);
      for (int bb = 0; bb < a.Bc && b0 + bb < a.B; ++bb) {
        const float2 h = lds[l * C + ls * Pc + bb * a.K + k];
        if (a.smaps) {
          const float2 s = a.smaps[(size_t)a.coils.idx[b0 + bb] * nvox + vox];
          acc = cadd(acc, cmulc(h, s));   // conj(S) * h
        } else {
          acc = cadd(acc, h);
        }
      }
      const float s = a.dx[xq] * a.dy[y] * a.dz[z];
      acc.x *= s;
      acc.y *= s;
      float2 *o = a.xout + (size_t)k * nvox + vox;
      if (a.accumulate || b0 > 0) acc = cadd(acc, *o);
      *o = acc;
    }
    __syncthreads();
  }
}

struct AxisArgs {
  float2 *data;
  int L;
  int64_t I;            // contiguous inner extent (columns)
  int C;                // columns per workgroup
  int64_t so;           // elements between outer slabs
  int o_lo, o_gap;      // outer o -> slab o < o_lo ? o : o + o_gap
  int in_lo, in_gap;    // rows [in_lo, in_lo + in_gap) are known zeros
  int Lout, out_lo, out_gap;   // rows written: q -> q < out_lo ? q : q + out_gap
  const float2 *tw;
  RadixPlan rp;
};

template <bool INV>
__global__ void __launch_bounds__(kFftThreads)
k_fft_axis(AxisArgs a) {
  extern __shared__ float2 smem[];
  const int L = a.L, C = a.C;
  float2 *lds = smem;
  float2 *tw = smem + L * C;
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * C;
  const int o = blockIdx.y;
  const int64_t slab = o < a.o_lo ? o : o + a.o_gap;
  float2 *base = a.data + slab * a.so + c0;
  for (int m = tid; m < L; m += kFftThreads) tw[m] = a.tw[m];
  for (int e = tid; e < L * C; e += kFftThreads) {
    const int c = e % C, l = e / C;
    float2 v = make_float2(0.f, 0.f);
    if (l < a.in_lo || l >= a.in_lo + a.in_gap) v = base[(int64_t)l * a.I + c];
    lds[l * C + c] = v;
  }
  __syncthreads();
  fft_lds<INV>(lds, L, C, a.rp, tw);
  for (int e = tid; e < a.Lout * C; e += kFftThreads) {
    const int c = e % C, q = e / C;
    const int l = q < a.out_lo ? q : q + a.out_gap;
    base[(int64_t)l * a.I + c] = lds[l * C + c];
  }
}

int cols_for(int L, int cap) {
  int c = 1;
  while (c * 2 <= cap && (c * 2 + 1) * L <= kFftLdsElems) c *= 2;
  return c;
}

size_t lds_bytes(int L, int C) { return ((size_t)L * C + L) * sizeof(float2); }

}  // namespace

hipError_t launch_pre_fftx(const sdn_plan_s &p, const float2 *x, int K, const float2 *smaps,
                           const CoilList &coils, int B, float2 *grid, hipStream_t st) {
  PreArgs a;
  a.x = x;
  a.smaps = smaps;
  a.coils = coils;
  a.K = K;
  a.P = B * K;
  a.g = line_geom(p);
  const int L = a.g.nfx;
  const int cap = kFftLdsElems / L - 1;      // columns that fit beside the twiddles
  a.Pc = std::min(a.P, cap);
  a.NL = std::max(1, std::min(cap / a.Pc, 16));
  a.grid = grid;
  a.dx = p.dinv[0]; a.dy = p.dinv[1]; a.dz = p.dinv[2];
  a.tw = p.tw[0];
  a.rp = p.rp[0];
  const int nlines = a.g.Nz * a.g.Ny;
  dim3 grd((nlines + a.NL - 1) / a.NL, (a.P + a.Pc - 1) / a.Pc);
  hipLaunchKernelGGL(k_pre_fftx, grd, dim3(kFftThreads), lds_bytes(L, a.NL * a.Pc), st, a);
  return hipGetLastError();
}

hipError_t launch_post_ifftx(const sdn_plan_s &p, const float2 *grid, int K,
                             const float2 *smaps, const CoilList &coils, int B, float2 *xout,
                             int accumulate, hipStream_t st) {
  PostArgs a;
  a.grid = grid;
  a.smaps = smaps;
  a.coils = coils;
  a.K = K;
  a.B = B;
  a.P = B * K;
  a.g = line_geom(p);
  const int L = a.g.nfx;
  const int cap = kFftLdsElems / L - 1;
  if (K > cap) return hipErrorInvalidValue;
  a.Bc = std::max(1, std::min(B, cap / K));
  a.NL = std::max(1, std::min(cap / (a.Bc * K), 16));
  a.xout = xout;
  a.accumulate = accumulate;
  a.dx = p.dinv[0]; a.dy = p.dinv[1]; a.dz = p.dinv[2];
  a.tw = p.tw[0];
  a.rp = p.rp[0];
  const int nlines = a.g.Nz * a.g.Ny;
  dim3 grd((nlines + a.NL - 1) / a.NL);
  hipLaunchKernelGGL(k_post_ifftx, grd, dim3(kFftThreads), lds_bytes(L, a.NL * a.Bc * K), st, a);
  return hipGetLastError();
}

hipError_t launch_fft_axis(const sdn_plan_s &p, float2 *grid, int P, int axis, bool inverse,
                           bool prune_in, bool prune_out, hipStream_t st) {
  const Axis &ax = p.ax[axis];
  AxisArgs a;
  a.data = grid;
  a.L = ax.nf;
  a.tw = p.tw[axis];
  a.rp = p.rp[axis];
  const int64_t nfx = p.ax[0].nf, nfy = p.ax[1].nf;
  int outer;
  if (axis == 1) {
    a.I = nfx * P;
    a.so = (int64_t)ax.nf * a.I;
    // only the image z planes carry data in either direction
    const Axis &az = p.ax[2];
    outer = az.N;
    a.o_lo = az.N - az.half;
    a.o_gap = az.nf - az.N;
  } else {
    a.I = nfy * nfx * P;
    a.so = 0;
    outer = 1;
    a.o_lo = 1;
    a.o_gap = 0;
  }
  // image rows sit at [0, N - half) and [nf - half, nf)
  if (prune_in) {
    a.in_lo = ax.N - ax.half;
    a.in_gap = ax.nf - ax.N;
  } else {
    a.in_lo = ax.nf;
    a.in_gap = 0;
  }
  if (prune_out) {
    a.Lout = ax.N;
    a.out_lo = ax.N - ax.half;
    a.out_gap = ax.nf - ax.N;
  } else {
    a.Lout = ax.nf;
    a.out_lo = ax.nf;
    a.out_gap = 0;
  }
  int C = cols_for(a.L, 64);
  while (C > 1 && a.I % C) C /= 2;
  a.C = C;
  dim3 grd((unsigned)(a.I / C), (unsigned)outer);
  if (inverse)
    hipLaunchKernelGGL(k_fft_axis<true>, grd, dim3(kFftThreads), lds_bytes(a.L, C), st, a);
  else
    hipLaunchKernelGGL(k_fft_axis<false>, grd, dim3(kFftThreads), lds_bytes(a.L, C), st, a);
  return hipGetLastError();
}

}  // namespace sdn
