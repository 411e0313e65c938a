// The sigma-oversampled 3D FFT of the gridding NUFFT, as three LDS-staged
// line passes over P channel-major fine grids stored [p][z][y][x].
//
// Forward (image -> fine grid spectrum):
//   x pass: fused with the coil multiply, deapodisation and zero padding -
//           reads x_k and S_c directly, writes only the N_z*N_y lines that
//           hold image data;
//   y pass: reads the N_y nonzero rows of the N_z nonzero planes;
//   z pass: reads the N_z nonzero planes, writes the whole grid.
// Adjoint (fine grid -> image), the same passes reversed with the output
// pruned to the image modes; the last x pass is fused with the crop,
// deapodisation, conj(S_c) multiply and the sum over coils (for coil counts
// dividing 16; otherwise the crop and the coil sum are two kernels).
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
  int NL;               // lines (columns) per workgroup
  int S;                // LDS row stride (>= NL, odd)
  float2 *grid;         // [P][nfz][nfy][nfx]
  const float *dx, *dy, *dz;
  const float2 *tw;
  RadixPlan rp;
  LineGeom g;
};

// One workgroup transforms NL x-lines; line n = (z Ny + y) P + p, so the
// lines of one workgroup share (z, y) and reuse the image and coil rows.
__global__ void __launch_bounds__(kFftThreads)
k_pre_fftx(PreArgs a) {
  extern __shared__ float2 smem[];
  const LineGeom &g = a.g;
  const int L = g.nfx, C = a.NL, S = a.S;
  float2 *lds = smem;
  float2 *tw = smem + L * S;
  const int tid = threadIdx.x;
  const int line0 = blockIdx.x * C;
  const int nlines = g.Nz * g.Ny * a.P;
  const size_t nvox = (size_t)g.Nz * g.Ny * g.Nx;
  for (int m = tid; m < L; m += kFftThreads) tw[m] = a.tw[m];
  // zero the padding rows [N - half, nf - half)
  const int nzero = (L - g.Nx) * C;
  for (int e = tid; e < nzero; e += kFftThreads) {
    const int c = e % C, r = e / C;
    lds[((g.Nx - g.hx) + r) * S + c] = make_float2(0.f, 0.f);
  }
  // coil * image / deapodisation, placed at fine positions
  for (int e = tid; e < C * g.Nx; e += kFftThreads) {
    const int xq = e % g.Nx, c = e / g.Nx;
    const int line = line0 + c;
    float2 v = make_float2(0.f, 0.f);
    if (line < nlines) {
      const int p = line % a.P, zy = line / a.P;
      const int z = zy / g.Ny, y = zy % g.Ny;
      const int b = p / a.K, k = p % a.K;
      const size_t vox = (size_t)zy * g.Nx + xq;
      v = a.x[(size_t)k * nvox + vox];
      if (a.smaps) v = cmul(a.smaps[(size_t)a.coils.idx[b] * nvox + vox], v);
      const float s = a.dx[xq] * a.dy[y] * a.dz[z];
      v.x *= s;
      v.y *= s;
    }
    lds[fine_pos(xq, g.hx, L) * S + c] = v;
  }
  __syncthreads();
  fft_lds<false>(lds, L, C, S, a.rp, tw);
  for (int e = tid; e < C * L; e += kFftThreads) {
    const int l = e % L, c = e / L;
    const int line = line0 + c;
    if (line >= nlines) continue;
    const int p = line % a.P, zy = line / a.P;
    const int z = zy / g.Ny, y = zy % g.Ny;
    const size_t zf = fine_pos(z, g.hz, g.nfz), yf = fine_pos(y, g.hy, g.nfy);
    a.grid[(((size_t)p * g.nfz + zf) * g.nfy + yf) * L + l] = lds[l * S + c];
  }
}

struct PostArgs {
  const float2 *grid;   // [P][nfz][nfy][nfx]
  const float2 *smaps;  // [C][Nz][Ny][Nx] or null
  CoilList coils;
  int K, B, P;
  int Bc, NL;           // coils per chunk, (z, y) lines per workgroup
  int S;                // LDS row stride
  float2 *xout;         // [K][Nz][Ny][Nx]
  int accumulate;
  const float *dx, *dy, *dz;
  const float2 *tw;
  RadixPlan rp;
  LineGeom g;
};

// One workgroup: NL (z, y) image lines, all channels of Bc coils at a time
// (column c = line slot * Bc K + b K + k), so the sum over coils stays in
// the workgroup.
__global__ void __launch_bounds__(kFftThreads)
k_post_ifftx(PostArgs a) {
  extern __shared__ float2 smem[];
  const LineGeom &g = a.g;
  const int L = g.nfx;
  const int Pc = a.Bc * a.K;
  const int C = a.NL * Pc, S = a.S;
  float2 *lds = smem;
  float2 *tw = smem + L * S;
  const int tid = threadIdx.x;
  const int line0 = blockIdx.x * a.NL;
  const int nlines = g.Nz * g.Ny;
  const size_t nvox = (size_t)g.Nz * g.Ny * g.Nx;
  for (int m = tid; m < L; m += kFftThreads) tw[m] = a.tw[m];
  for (int b0 = 0; b0 < a.B; b0 += a.Bc) {
    const int p0 = b0 * a.K;
    for (int e = tid; e < C * L; e += kFftThreads) {
      const int l = e % L, c = e / L;
      const int ls = c / Pc, pp = c % Pc;
      const int line = line0 + ls, p = p0 + pp;
      float2 v = make_float2(0.f, 0.f);
      if (line < nlines && p < a.P) {
        const int z = line / g.Ny, y = line % g.Ny;
        const size_t zf = fine_pos(z, g.hz, g.nfz), yf = fine_pos(y, g.hy, g.nfy);
        v = a.grid[(((size_t)p * g.nfz + zf) * g.nfy + yf) * L + l];
      }
      lds[l * S + c] = v;
    }
    __syncthreads();
    fft_lds<true>(lds, L, C, S, a.rp, tw);
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
        const float2 h = lds[l * S + ls * Pc + bb * a.K + k];
        if (a.smaps) {
          const float2 sv = a.smaps[(size_t)a.coils.idx[b0 + bb] * nvox + vox];
          acc = cadd(acc, cmulc(h, sv));   // conj(S) * h
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
  int O2;               // outer = (o1 channel, o2 plane): o = o1 * O2 + o2
  int64_t so1, so2;     // element strides of o1 and of a plane
  int o_lo, o_gap;      // plane o2 -> o2 < o_lo ? o2 : o2 + o_gap
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
  const int o1 = o / a.O2, o2 = o - o1 * a.O2;
  const int64_t plane = o2 < a.o_lo ? o2 : o2 + a.o_gap;
  float2 *base = a.data + o1 * a.so1 + plane * a.so2 + c0;
  for (int m = tid; m < L; m += kFftThreads) tw[m] = a.tw[m];
  for (int e = tid; e < L * C; e += kFftThreads) {
    const int c = e % C, l = e / C;
    float2 v = make_float2(0.f, 0.f);
    if (l < a.in_lo || l >= a.in_lo + a.in_gap) v = base[(int64_t)l * a.I + c];
    lds[l * C + c] = v;
  }
  __syncthreads();
  fft_lds<INV>(lds, L, C, C, a.rp, tw);
  for (int e = tid; e < a.Lout * C; e += kFftThreads) {
    const int c = e % C, q = e / C;
    const int l = q < a.out_lo ? q : q + a.out_gap;
    base[(int64_t)l * a.I + c] = lds[l * C + c];
  }
}

// columns (consecutive x) per workgroup of the y and z passes: 16 read and
// write whole 128-byte rows; 8 (64-byte segments) measured 1.4x slower
constexpr int kAxisCols = 16;
// threads per workgroup of the y and z passes: 512 for L >= 128 (the same
// LDS as 256, twice the waves to overlap its loads, transforms and stores;
// 11-17% faster at L = 400), 256 for the short lines of small grids

// Specialised strided pass: L and C columns known at compile time.
template <bool INV, int L, int C, int kAxThreads>
__global__ void __launch_bounds__(kAxThreads)
k_fft_axis_ct(AxisArgs a) {
  __shared__ float2 lds[L * C];
  __shared__ float2 tw[L];
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * C;
  const int o = blockIdx.y;
  const int o1 = o / a.O2, o2 = o - o1 * a.O2;
  const int64_t plane = o2 < a.o_lo ? o2 : o2 + a.o_gap;
  float2 *base = a.data + o1 * a.so1 + plane * a.so2 + c0;
  for (int m = tid; m < L; m += kAxThreads) tw[m] = a.tw[m];
  constexpr int NE = (L * C + kAxThreads - 1) / kAxThreads;
  constexpr bool whole = L * C % kAxThreads == 0;
  float2 v[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * kAxThreads;
    const int c = e % C, l = e / C;
    v[q] = (whole || e < L * C) && (l < a.in_lo || l >= a.in_lo + a.in_gap)
               ? base[(int64_t)l * a.I + c]
               : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int q = 0; q < NE; ++q)
    if (whole || tid + q * kAxThreads < L * C) lds[tid + q * kAxThreads] = v[q];
  __syncthreads();
  RadixSeq<L>::template run<INV, C, C, kAxThreads>(lds, tw);
  for (int e = tid; e < a.Lout * C; e += kAxThreads) {
    const int c = e % C, q = e / C;
    const int l = q < a.out_lo ? q : q + a.out_gap;
    base[(int64_t)l * a.I + c] = lds[l * C + c];
  }
}

// q / d via a float reciprocal of d: (q + 1/2) / d lies at least 1/(2d)
// away from an integer, and the two roundings move it by less than
// (q/d + 1) 2^-23, so the truncation is exact whenever q + d < 2^22.
__device__ __forceinline__ int qdiv(int q, float inv) { return (int)(((float)q + 0.5f) * inv); }

constexpr int kPreLines = 8;   // lines per workgroup of the compile-time forward x pass
// its threads per workgroup: 512 for lines of 384 points and more (0.33 ->
// 0.29 ms at L = 400), 256 below (512 measured slower at L = 320)
constexpr int kPreThreads(int L) { return L >= 384 ? 512 : 256; }

// Compile-time forward x pass: C lines per workgroup (line n = (z Ny + y) P + p).
template <int L, int C, int NT>
__global__ void __launch_bounds__(NT)
k_pre_fftx_ct(PreArgs a, float inv_nx, float inv_p) {
  constexpr int S = C + 1;
  __shared__ float2 lds[L * S];
  __shared__ float2 tw[L];
  const LineGeom &g = a.g;
  const int tid = threadIdx.x;
  const int line0 = blockIdx.x * C;
  const int nlines = g.Nz * g.Ny * a.P;
  const size_t nvox = (size_t)g.Nz * g.Ny * g.Nx;
  // per-line geometry, once per workgroup: image and coil rows, the y/z
  // deapodisation factor and the output line (none: line past the end)
  __shared__ const float2 *xrow[C], *srow[C];
  __shared__ float scyz[C];
  __shared__ float2 *orow[C];
  if (tid < C) {
    const int line = line0 + tid;
    xrow[tid] = srow[tid] = nullptr;
    orow[tid] = nullptr;
    scyz[tid] = 0.f;
    if (line < nlines) {
      const int zy = qdiv(line, inv_p);
      const int p = line - zy * a.P;
      const int z = zy / g.Ny, y = zy - z * g.Ny;
      const int b = p / a.K, k = p - b * a.K;
      xrow[tid] = a.x + (size_t)k * nvox + (size_t)zy * g.Nx;
      srow[tid] = a.smaps ? a.smaps + (size_t)a.coils.idx[b] * nvox + (size_t)zy * g.Nx : nullptr;
      scyz[tid] = a.dy[y] * a.dz[z];
      const size_t zf = fine_pos(z, g.hz, g.nfz), yf = fine_pos(y, g.hy, g.nfy);
      orow[tid] = a.grid + (((size_t)p * g.nfz + zf) * g.nfy + yf) * L;
    }
  }
  for (int m = tid; m < L; m += NT) tw[m] = a.tw[m];
  for (int e = tid; e < (L - g.Nx) * C; e += NT) {
    const int c = e % C, r = e / C;
    lds[((g.Nx - g.hx) + r) * S + c] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  // every thread issues all its loads before using any (Nx <= L, so
  // C Nx <= C L elements cover the workgroup)
  constexpr int NE = (L * C + NT - 1) / NT;
  float2 xv[NE], sv[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = tid + i * NT;
    xv[i] = sv[i] = make_float2(0.f, 0.f);
    if (e < C * g.Nx) {
      const int c = qdiv(e, inv_nx);
      const int xq = e - c * g.Nx;
      if (xrow[c]) {
        xv[i] = xrow[c][xq];
        sv[i] = srow[c] ? srow[c][xq] : make_float2(1.f, 0.f);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = tid + i * NT;
    if (e < C * g.Nx) {
      const int c = qdiv(e, inv_nx);
      const int xq = e - c * g.Nx;
      float2 v = cmul(sv[i], xv[i]);
      const float sc = a.dx[xq] * scyz[c];
      v.x *= sc;
      v.y *= sc;
      lds[fine_pos(xq, g.hx, L) * S + c] = v;
    }
  }
  __syncthreads();
  RadixSeq<L>::template run<false, C, S, NT>(lds, tw);
  for (int e = tid; e < C * L; e += NT) {
    const int l = e % L, c = e / L;
    if (orow[c]) orow[c][l] = lds[l * S + c];
  }
}

struct CropArgs {
  float2 *grid;     // [P][nfz][nfy][nfx]
  int P;
  const float2 *tw;
  LineGeom g;
};

// Compile-time inverse x pass over the P Nz Ny image lines (line n = (p Nz
// + z) Ny + y): the N_x image samples of each transformed line are written
// back to the first N_x cells of the same line, in image order.
template <int L>
__global__ void __launch_bounds__(kFftThreads)
k_ifftx_crop_ct(CropArgs a, float inv_nx) {
  constexpr int C = 16, S = 17;
  __shared__ float2 lds[L * S];
  __shared__ float2 tw[L];
  const LineGeom &g = a.g;
  const int tid = threadIdx.x;
  const int line0 = blockIdx.x * C;
  const int nlines = a.P * g.Nz * g.Ny;
  // the grid line of every column, once per workgroup (none: past the end)
  __shared__ float2 *row[C];
  if (tid < C) {
    const int line = line0 + tid;
    row[tid] = nullptr;
    if (line < nlines) {
      const int y = line % g.Ny, pz = line / g.Ny;
      const int z = pz % g.Nz, p = pz / g.Nz;
      const size_t zf = fine_pos(z, g.hz, g.nfz), yf = fine_pos(y, g.hy, g.nfy);
      row[tid] = a.grid + (((size_t)p * g.nfz + zf) * g.nfy + yf) * L;
    }
  }
  for (int m = tid; m < L; m += kFftThreads) tw[m] = a.tw[m];
  __syncthreads();
  {
    constexpr int NE = L * C / kFftThreads;
    float2 v[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + i * kFftThreads;
      const int l = e % L, c = e / L;
      v[i] = row[c] ? row[c][l] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + i * kFftThreads;
      lds[(e % L) * S + e / L] = v[i];
    }
  }
  __syncthreads();
  RadixSeq<L>::template run<true, C, S, kFftThreads>(lds, tw);
  for (int e = tid; e < C * g.Nx; e += kFftThreads) {
    const int c = qdiv(e, inv_nx);
    const int xq = e - c * g.Nx;
    if (row[c]) row[c][xq] = lds[fine_pos(xq, g.hx, L) * S + c];
  }
}

// threads per workgroup of the fused inverse x pass: 512 (0.57 -> 0.54 ms
// at c4, 0.44 -> 0.33 ms at the 400-point lines of the paper shape; the
// forward x pass stays at 256, which measured faster at c4)
constexpr int kPostThreads = 512;

// Inverse x pass fused with the coil combine, for B coils with B | C: the
// C columns of a workgroup are the B coils' lines of C / B image rows of
// one (channel k, plane z), column c = r B + b.  After the transform the
// workgroup forms xout[k] (+)= sum_b conj(S_b) h_b / deapodisation for its
// rows directly from LDS, so the cropped lines never go back to HBM.
// Grid: (ceil(Ny / R), Nz, K) with R = C / B rows per workgroup; C = 8
// when B | 8 (twice the workgroups per CU of C = 16), else 16.
template <int L, int C>
__global__ void __launch_bounds__(kPostThreads)
k_ifftx_post_ct(PostArgs a) {
  constexpr int S = C + 1;
  __shared__ float2 lds[L * S];
  __shared__ float2 tw[L];
  __shared__ const float2 *col[C];
  const LineGeom &g = a.g;
  const int tid = threadIdx.x;
  const int B = a.B, R = C / B;
  // channels fastest: the K workgroups of one image row run together and
  // read its coil maps while they are in the caches
  const int k = (int)blockIdx.x % a.K;
  const int y0 = (int)blockIdx.x / a.K * R, z = blockIdx.y;
  const size_t zf = fine_pos(z, g.hz, g.nfz);
  if (tid < C) {
    const int r = tid / B, b = tid - r * B;
    const int y = y0 + r;
    col[tid] = nullptr;
    if (y < g.Ny) {
      const size_t yf = fine_pos(y, g.hy, g.nfy);
      col[tid] = a.grid + (((size_t)(b * a.K + k) * g.nfz + zf) * g.nfy + yf) * L;
    }
  }
  for (int m = tid; m < L; m += kPostThreads) tw[m] = a.tw[m];
  __syncthreads();
  {
    constexpr int NE = (L * C + kPostThreads - 1) / kPostThreads;
    constexpr bool whole = L * C % kPostThreads == 0;
    float2 v[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + i * kPostThreads;
      const int l = e % L, c = e / L;
      v[i] = (whole || e < L * C) && col[c] ? col[c][l] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + i * kPostThreads;
      if (whole || e < L * C) lds[(e % L) * S + e / L] = v[i];
    }
  }
  __syncthreads();
  RadixSeq<L>::template run<true, C, S, kPostThreads>(lds, tw);
  const size_t nvox = (size_t)g.Nz * g.Ny * g.Nx;
  const float sz = a.dz[z];
  for (int e = tid; e < R * g.Nx; e += kPostThreads) {
    const int r = e / g.Nx, xq = e - r * g.Nx;
    const int y = y0 + r;
    if (y >= g.Ny) continue;
    const size_t vox = ((size_t)z * g.Ny + y) * g.Nx + xq;
    const float2 *h = lds + fine_pos(xq, g.hx, L) * S + r * B;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 4
    for (int b = 0; b < B; ++b) {
      if (a.smaps) acc = cadd(acc, cmulc(h[b], a.smaps[(size_t)a.coils.idx[b] * nvox + vox]));
      else acc = cadd(acc, h[b]);
    }
    const float sc = a.dx[xq] * a.dy[y] * sz;
    acc.x *= sc;
    acc.y *= sc;
    const size_t i = (size_t)k * nvox + vox;
    if (a.accumulate) acc = cadd(acc, a.xout[i]);
    a.xout[i] = acc;
  }
}

// xout[k] (+)= sum_b conj(S_b) h_{b,k} / deapodisation, h the cropped lines.
// Grid (ceil(Nx / 64), ceil(Ny / 4), Nz K): the row (k, z, y) comes from the
// block and thread indices, no per-voxel division.
__global__ void __launch_bounds__(256) k_combine(PostArgs a) {
  const LineGeom &g = a.g;
  const int xq = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (xq >= g.Nx || y >= g.Ny) return;
  const int k = blockIdx.z / g.Nz, z = blockIdx.z - k * g.Nz;
  const size_t nvox = (size_t)g.Nz * g.Ny * g.Nx;
  const size_t vox = ((size_t)z * g.Ny + y) * g.Nx + xq;
  const size_t zf = fine_pos(z, g.hz, g.nfz), yf = fine_pos(y, g.hy, g.nfy);
  const size_t G = (size_t)g.nfz * g.nfy * g.nfx;
  const float2 *h = a.grid + (zf * g.nfy + yf) * g.nfx + xq;
  float2 acc = make_float2(0.f, 0.f);
  for (int b = 0; b < a.B; ++b) {
    const float2 hv = h[(size_t)(b * a.K + k) * G];
    if (a.smaps) acc = cadd(acc, cmulc(hv, a.smaps[(size_t)a.coils.idx[b] * nvox + vox]));
    else acc = cadd(acc, hv);
  }
  const float sc = a.dx[xq] * a.dy[y] * a.dz[z];
  acc.x *= sc;
  acc.y *= sc;
  const size_t i = (size_t)k * nvox + vox;
  if (a.accumulate) acc = cadd(acc, a.xout[i]);
  a.xout[i] = acc;
}

bool fft_len_ct(int L) {
  switch (L) {
    case 64: case 96: case 128: case 160: case 192: case 224: case 256: case 288: case 320:
    case 384: case 400: case 448:
      return true;
    default: return false;
  }
}

int cols_for(int L, int cap) {
  int c = 1;
  while (c * 2 <= cap && (c * 2 + 1) * L <= kFftLdsElems) c *= 2;
  return c;
}

size_t lds_bytes(int L, int S) { return ((size_t)L * S + L) * sizeof(float2); }

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
  a.grid = grid;
  a.dx = p.dinv[0]; a.dy = p.dinv[1]; a.dz = p.dinv[2];
  a.tw = p.tw[0];
  a.rp = p.rp[0];
  const int64_t nl_all = (int64_t)a.g.Nz * a.g.Ny * a.P;
  if (fft_len_ct(L) && nl_all + a.P < (1 << 22)) {
    const int64_t nl = nl_all;
    const float inv_nx = 1.0f / a.g.Nx, inv_p = 1.0f / a.P;
    // 8 lines per workgroup: 22 KB of LDS at L = 320, so up to 7 workgroups
    // share a CU and overlap their loads, transforms and stores
    constexpr int C = kPreLines;
    dim3 grd((unsigned)((nl + C - 1) / C));
#define SDN_PRE_CT(LEN) \
  case LEN: hipLaunchKernelGGL((k_pre_fftx_ct<LEN, C, kPreThreads(LEN)>), grd, dim3(kPreThreads(LEN)), 0, st, a, inv_nx, inv_p); break;
    switch (L) {
      SDN_PRE_CT(64) SDN_PRE_CT(96) SDN_PRE_CT(128) SDN_PRE_CT(160) SDN_PRE_CT(192) SDN_PRE_CT(224) SDN_PRE_CT(256)
      SDN_PRE_CT(288) SDN_PRE_CT(320) SDN_PRE_CT(384) SDN_PRE_CT(400) SDN_PRE_CT(448)
    }
#undef SDN_PRE_CT
    return hipGetLastError();
  }
  a.NL = std::max(1, std::min(kFftLdsElems / L - 2, 32));   // columns beside twiddles
  a.S = a.NL | 1;
  a.grid = grid;
  a.dx = p.dinv[0]; a.dy = p.dinv[1]; a.dz = p.dinv[2];
  a.tw = p.tw[0];
  a.rp = p.rp[0];
  const int64_t nlines = (int64_t)a.g.Nz * a.g.Ny * a.P;
  dim3 grd((unsigned)((nlines + a.NL - 1) / a.NL));
  hipLaunchKernelGGL(k_pre_fftx, grd, dim3(kFftThreads), lds_bytes(L, a.S), st, a);
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
  a.xout = xout;
  a.accumulate = accumulate;
  a.dx = p.dinv[0]; a.dy = p.dinv[1]; a.dz = p.dinv[2];
  a.tw = p.tw[0];
  a.rp = p.rp[0];
  if (fft_len_ct(L) && B <= 16 && 16 % B == 0 && a.g.Nz <= 65535 && K <= 65535) {
    const bool c8 = 8 % B == 0;
    const int R = (c8 ? 8 : 16) / B;
    dim3 grd((unsigned)((a.g.Ny + R - 1) / R * K), (unsigned)a.g.Nz);
#define SDN_POST_CT(LEN)                                                                    \
  case LEN:                                                                                 \
    if (c8) hipLaunchKernelGGL((k_ifftx_post_ct<LEN, 8>), grd, dim3(kPostThreads), 0, st, a); \
    else hipLaunchKernelGGL((k_ifftx_post_ct<LEN, 16>), grd, dim3(kPostThreads), 0, st, a);   \
    break;
    switch (L) {
      SDN_POST_CT(64) SDN_POST_CT(96) SDN_POST_CT(128) SDN_POST_CT(160) SDN_POST_CT(192)
      SDN_POST_CT(224) SDN_POST_CT(256) SDN_POST_CT(288) SDN_POST_CT(320) SDN_POST_CT(384)
      SDN_POST_CT(400) SDN_POST_CT(448)
    }
#undef SDN_POST_CT
    return hipGetLastError();
  }
  if (fft_len_ct(L)) {
    CropArgs c;
    c.grid = const_cast<float2 *>(grid);
    c.P = a.P;
    c.tw = p.tw[0];
    c.g = a.g;
    const int64_t nl = (int64_t)a.P * a.g.Nz * a.g.Ny;
    const float inv_nx = 1.0f / a.g.Nx;
    dim3 grd((unsigned)((nl + 15) / 16));
#define SDN_CROP_CT(LEN) \
  case LEN: hipLaunchKernelGGL(k_ifftx_crop_ct<LEN>, grd, dim3(kFftThreads), 0, st, c, inv_nx); break;
    switch (L) {
      SDN_CROP_CT(64) SDN_CROP_CT(96) SDN_CROP_CT(128) SDN_CROP_CT(160) SDN_CROP_CT(192) SDN_CROP_CT(224) SDN_CROP_CT(256)
      SDN_CROP_CT(288) SDN_CROP_CT(320) SDN_CROP_CT(384) SDN_CROP_CT(400) SDN_CROP_CT(448)
    }
#undef SDN_CROP_CT
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((int64_t)K * a.g.Nz > 65535) return hipErrorInvalidValue;
    dim3 cg((unsigned)((a.g.Nx + 63) / 64), (unsigned)((a.g.Ny + 3) / 4),
             (unsigned)(K * a.g.Nz));
    hipLaunchKernelGGL(k_combine, cg, dim3(64, 4), 0, st, a);
    return hipGetLastError();
  }
  const int cap = kFftLdsElems / L - 2;
  if (K > cap) return hipErrorInvalidValue;
  a.Bc = std::max(1, std::min(B, cap / K));
  a.NL = std::max(1, std::min(cap / (a.Bc * K), 16));
  a.S = (a.NL * a.Bc * K) | 1;
  a.xout = xout;
  a.accumulate = accumulate;
  a.dx = p.dinv[0]; a.dy = p.dinv[1]; a.dz = p.dinv[2];
  a.tw = p.tw[0];
  a.rp = p.rp[0];
  const int nlines = a.g.Nz * a.g.Ny;
  dim3 grd((nlines + a.NL - 1) / a.NL);
  hipLaunchKernelGGL(k_post_ifftx, grd, dim3(kFftThreads), lds_bytes(L, a.S), st, a);
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
  const int64_t nfx = p.ax[0].nf, nfy = p.ax[1].nf, nfz = p.ax[2].nf;
  a.so1 = nfx * nfy * nfz;   // one channel's grid
  if (axis == 1) {
    // planes: only the image z planes carry data in either direction
    const Axis &az = p.ax[2];
    a.I = nfx;
    a.O2 = az.N;
    a.so2 = nfy * nfx;
    a.o_lo = az.N - az.half;
    a.o_gap = az.nf - az.N;
  } else {
    a.I = nfy * nfx;
    a.O2 = 1;
    a.so2 = 0;
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
  const int64_t outer = (int64_t)P * a.O2;
  if (outer > 65535) return hipErrorInvalidValue;
  if (a.I % kAxisCols == 0) {
    constexpr int C = kAxisCols;
    a.C = C;
    dim3 grd((unsigned)(a.I / C), (unsigned)outer);
#define SDN_AXIS_CT(LEN)                                                                        \
  case LEN:                                                                                     \
    {                                                                                           \
      constexpr int NT = LEN >= 128 ? 512 : 256;                                                \
      if (inverse) hipLaunchKernelGGL((k_fft_axis_ct<true, LEN, C, NT>), grd, dim3(NT), 0, st, a); \
      else hipLaunchKernelGGL((k_fft_axis_ct<false, LEN, C, NT>), grd, dim3(NT), 0, st, a);        \
    }                                                                                           \
    return hipGetLastError();
    switch (a.L) {
      SDN_AXIS_CT(64)
      SDN_AXIS_CT(96)
      SDN_AXIS_CT(128)
      SDN_AXIS_CT(160)
      SDN_AXIS_CT(192)
      SDN_AXIS_CT(224)
      SDN_AXIS_CT(256)
      SDN_AXIS_CT(288)
      SDN_AXIS_CT(320)
      SDN_AXIS_CT(384)
      SDN_AXIS_CT(400)
      SDN_AXIS_CT(448)
      default: break;
    }
#undef SDN_AXIS_CT
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
