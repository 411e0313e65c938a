// Per-point kernel nodes shared by the plan and the grid kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sdn_internal.h"

namespace sdn {

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

// First node (l0x, l0y, l0z) of a point, packed 10 bits per axis.
__device__ __forceinline__ void unpack_l0(float bits, int &lx, int &ly, int &lz) {
  const unsigned u = __float_as_uint(bits);
  lx = (int)(u & 1023u);
  ly = (int)((u >> 10) & 1023u);
  lz = (int)((u >> 20) & 1023u);
}

}  // namespace sdn
