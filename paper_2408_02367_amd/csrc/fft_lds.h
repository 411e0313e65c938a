// Batched mixed-radix Stockham FFT of C columns of length L held in LDS.
//
// Layout: element (l, c) at lds[l * S + c] (row stride S >= C); a
// workgroup transforms all C columns together.  Each radix-R pass reads every thread's butterflies into
// registers, synchronises, then writes them to their self-sorting (Stockham)
// positions, so the transform runs in place in one LDS buffer and leaves
// the output in natural order.
//
// Pass with radix R after passes of total length Ns: butterfly j of a
// column (0 <= j < L/R), k = j mod Ns, takes inputs j + r L/R, multiplies
// input r by w^(r k L/(Ns R)) with w = exp(-+2 pi i / L), applies a length-R
// DFT and stores output q at (j / Ns) Ns R + k + q Ns.
#pragma once

#include <hip/hip_runtime.h>

#include "sdn_internal.h"

namespace sdn {

constexpr int kFftThreads = 256;
constexpr int kFftLdsElems = 8192;   // L * C complex values per workgroup

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot_i(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R>
struct RootTable;
template <>
struct RootTable<3> {
  static constexpr float c[3] = {1.0f, -0.5f, -0.5f};
  static constexpr float s[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
};
template <>
struct RootTable<5> {
  static constexpr float c[5] = {1.0f, 0.30901699437494745f, -0.80901699437494734f,
                                 -0.80901699437494734f, 0.30901699437494745f};
  static constexpr float s[5] = {0.0f, 0.95105651629515353f, 0.58778525229247325f,
                                 -0.58778525229247325f, -0.95105651629515353f};
};
template <>
struct RootTable<6> {
  static constexpr float c[6] = {1.0f, 0.5f, -0.5f, -1.0f, -0.5f, 0.5f};
  static constexpr float s[6] = {0.0f, 0.86602540378443865f, 0.86602540378443865f, 0.0f,
                                 -0.86602540378443865f, -0.86602540378443865f};
};
template <>
struct RootTable<7> {
  static constexpr float c[7] = {1.0f, 0.62348980185873359f, -0.22252093395631434f,
                                 -0.90096886790241903f, -0.90096886790241903f,
                                 -0.22252093395631434f, 0.62348980185873359f};
  static constexpr float s[7] = {0.0f, 0.78183148246802981f, 0.97492791218182362f,
                                 0.43388373911755823f, -0.43388373911755823f,
                                 -0.97492791218182362f, -0.78183148246802981f};
};

// In-register DFT of length R: v_q <- sum_r v_r exp(-+2 pi i r q / R).
template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = rot_i<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else if constexpr (R == 8) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, INV>(e);
    dft<4, INV>(o);
    constexpr float h = 0.70710678118654752f;
    // o_q *= w^q, w = exp(-+2 pi i / 8)
    o[1] = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
               : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    o[2] = rot_i<INV>(o[2]);
    o[3] = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
               : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = cadd(e[q], o[q]);
      v[q + 4] = csub(e[q], o[q]);
    }
  } else {
    float2 out[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int m = (r * q) % R;
        const float c = RootTable<R>::c[m];
        const float s = INV ? -RootTable<R>::s[m] : RootTable<R>::s[m];
        // (a + ib)(c - is)
        re += v[r].x * c + v[r].y * s;
        im += v[r].y * c - v[r].x * s;
      }
      out[q] = make_float2(re, im);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = out[q];
  }
}

template <int R, bool INV>
__device__ __forceinline__ void fft_pass(float2 *lds, int L, int C, int S, int Ns,
                                         const float2 *tw) {
  constexpr int MAXB = (kFftLdsElems / R + kFftThreads - 1) / kFftThreads;
  const int nbf = L / R;
  const int total = nbf * C;
  const int tstride = L / (Ns * R);
  const int tid = threadIdx.x;
  float2 v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * kFftThreads;
    if (b < total) {
      const int c = b % C, j = b / C;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = lds[(j + r * nbf) * S + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * kFftThreads;
    if (b < total) {
      const int c = b % C, j = b / C;
      const int k = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw[r * k * tstride];
          v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
        }
      }
      dft<R, INV>(v[q]);
      const int d = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(d + r * Ns) * S + c] = v[q][r];
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------------
// Compile-time variant for the common fine-grid lengths: L, C, the row
// stride S and every pass's Ns are constants, so index arithmetic folds and
// each thread holds exactly the butterflies it needs.
template <int R, bool INV, int L, int C, int S, int Ns, int NT>
__device__ __forceinline__ void fft_pass_ct(float2 *lds, const float2 *tw) {
  constexpr int nbf = L / R;
  constexpr int total = nbf * C;
  constexpr int MAXB = (total + NT - 1) / NT;
  constexpr int tstride = L / (Ns * R);
  const int tid = threadIdx.x;
  float2 v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * NT;
    if (total % NT == 0 || b < total) {
      const int c = b % C, j = b / C;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = lds[(j + r * nbf) * S + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = tid + q * NT;
    if (total % NT == 0 || b < total) {
      const int c = b % C, j = b / C;
      const int k = j % Ns;
      if constexpr (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw[r * k * tstride];
          v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
        }
      }
      dft<R, INV>(v[q]);
      const int d = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(d + r * Ns) * S + c] = v[q][r];
    }
  }
  __syncthreads();
}

template <bool INV, int L, int C, int S, int NT, int Ns, int... Rs>
struct FftPasses {
  static __device__ __forceinline__ void run(float2 *, const float2 *) {}
};
template <bool INV, int L, int C, int S, int NT, int Ns, int R, int... Rs>
struct FftPasses<INV, L, C, S, NT, Ns, R, Rs...> {
  static __device__ __forceinline__ void run(float2 *lds, const float2 *tw) {
    fft_pass_ct<R, INV, L, C, S, Ns, NT>(lds, tw);
    FftPasses<INV, L, C, S, NT, Ns * R, Rs...>::run(lds, tw);
  }
};

// Radix sequences of the specialised lengths (the host radix_plan order).
template <int L>
struct RadixSeq;
#define SDN_RADIX_SEQ(LEN, ...)                                                      \
  template <>                                                                        \
  struct RadixSeq<LEN> {                                                             \
    template <bool INV, int C, int S, int NT>                                        \
    static __device__ __forceinline__ void run(float2 *lds, const float2 *tw) {      \
      FftPasses<INV, LEN, C, S, NT, 1, __VA_ARGS__>::run(lds, tw);                   \
    }                                                                                \
  };
SDN_RADIX_SEQ(64, 8, 8)
SDN_RADIX_SEQ(128, 4, 4, 8)
SDN_RADIX_SEQ(192, 8, 8, 3)
SDN_RADIX_SEQ(256, 4, 8, 8)
SDN_RADIX_SEQ(320, 8, 8, 5)
SDN_RADIX_SEQ(384, 6, 8, 8)
SDN_RADIX_SEQ(448, 8, 8, 7)
SDN_RADIX_SEQ(96, 4, 8, 3)
SDN_RADIX_SEQ(160, 4, 8, 5)
SDN_RADIX_SEQ(224, 4, 8, 7)
SDN_RADIX_SEQ(288, 4, 8, 3, 3)
SDN_RADIX_SEQ(400, 4, 4, 5, 5)
#undef SDN_RADIX_SEQ

// Transform all C columns; `tw` = exp(-2 pi i m / L) (inverse uses conj).
template <bool INV>
__device__ void fft_lds(float2 *lds, int L, int C, int S, const RadixPlan &rp, const float2 *tw) {
  int Ns = 1;
  for (int p = 0; p < rp.n; ++p) {
    switch (rp.r[p]) {
      case 2: fft_pass<2, INV>(lds, L, C, S, Ns, tw); break;
      case 3: fft_pass<3, INV>(lds, L, C, S, Ns, tw); break;
      case 4: fft_pass<4, INV>(lds, L, C, S, Ns, tw); break;
      case 5: fft_pass<5, INV>(lds, L, C, S, Ns, tw); break;
      case 6: fft_pass<6, INV>(lds, L, C, S, Ns, tw); break;
      case 7: fft_pass<7, INV>(lds, L, C, S, Ns, tw); break;
      default: fft_pass<8, INV>(lds, L, C, S, Ns, tw); break;
    }
    Ns *= rp.r[p];
  }
}

}  // namespace sdn
