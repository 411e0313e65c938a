// Autotuner: the plan options (interpolation tile, points per work item,
// spreading engine) that make one data-consistency step fastest for a
// given trajectory, image shape and minibatch, found by timing candidate
// plans on synthetic device data.  Runs once per trajectory, like the plan.
#include <algorithm>
#include <vector>

#include "sdn_internal.h"

using namespace sdn;

#define SDN_TRY(expr)                      \
  do {                                     \
    sdn_status _s = (expr);                \
    if (_s != SDN_OK) return _s;           \
  } while (0)
#define SDN_TRY_HIP(expr, what) SDN_TRY(hip_check((expr), what))

namespace {

// Deterministic synthetic values (a hash of the index), in [-1, 1).
__global__ void k_synth(float *a, size_t n, unsigned salt) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)i * 2654435761u ^ salt;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    a[i] = (float)(h & 0xffffff) * (2.f / 16777216.f) - 1.f;
  }
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

sdn_status synth(DevBuf &b, size_t floats, unsigned salt, hipStream_t st) {
  SDN_TRY_HIP(hipMalloc(&b.p, std::max<size_t>(floats, 1) * sizeof(float)), "autotune buffers");
  hipLaunchKernelGGL(k_synth, dim3(1024), dim3(256), 0, st, (float *)b.p, floats, salt);
  return hip_check(hipGetLastError(), "autotune fill");
}

}  // namespace

extern "C" {

sdn_status sdn_autotune(const int64_t shape[3], const float *traj, int64_t M,
                        const int32_t *frame_of_point, int32_t T, int B, int K,
                        const sdn_opts *base, sdn_opts *best, double *best_ms, void *stream) {
  if (!shape || !best || B < 1 || B > kMaxB || K < 1 || K > kMaxK)
    return fail(SDN_E_INVALID, "sdn_autotune: bad argument");
  if (M > 0 && !traj) return fail(SDN_E_INVALID, "sdn_autotune: traj is NULL");
  hipStream_t st = (hipStream_t)stream;
  sdn_opts o0;
  sdn_default_opts(&o0);
  if (base) o0 = *base;
  const int Tn = std::max(T, 1);
  const size_t nvox = (size_t)shape[0] * shape[1] * shape[2];
  DevBuf x, smaps, V, d, grad, loss;
  SDN_TRY(synth(x, 2 * (size_t)K * nvox, 1u, st));
  SDN_TRY(synth(smaps, 2 * (size_t)B * nvox, 2u, st));
  SDN_TRY(synth(V, 2 * (size_t)Tn * K, 3u, st));
  SDN_TRY(synth(d, 2 * (size_t)B * std::max<int64_t>(M, 1), 4u, st));
  SDN_TRY(synth(grad, 2 * (size_t)K * nvox, 5u, st));
  SDN_TRY_HIP(hipMalloc(&loss.p, sizeof(double)), "autotune buffers");
  std::vector<int32_t> coils(B);
  for (int b = 0; b < B; ++b) coils[b] = b;

  std::vector<sdn_opts> cand;
  for (int tile : {0, 8, 16})
    for (int cap : {0, 1024})
      for (int eng : {SDN_SPREAD_GATHER, SDN_SPREAD_MATRIX, SDN_SPREAD_PLANES})
        for (int order : {SDN_ORDER_AUTO, SDN_ORDER_CELL}) {
          if (eng != SDN_SPREAD_GATHER && order == SDN_ORDER_CELL) continue;
          // one channel per coil always gathers: the matrix engines would
          // only repeat the gather candidates
          if (eng != SDN_SPREAD_GATHER && K < 2) continue;
          sdn_opts o = o0;
          o.tile = tile;
          o.max_points_per_item = cap;
          o.spread_engine = eng;
          o.point_order = order;
          cand.push_back(o);
        }
  hipEvent_t e0, e1;
  SDN_TRY_HIP(hipEventCreate(&e0), "autotune events");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(SDN_E_HIP, "autotune events");
  }
  double best_t = -1.0;
  sdn_status err = SDN_OK;
  for (const sdn_opts &o : cand) {
    sdn_plan p = nullptr;
    if (sdn_plan_create(&p, shape, traj, M, frame_of_point, T, &o, stream) != SDN_OK) continue;
    auto step = [&]() {
      return sdn_mrf_dc_grad(p, x.p, K, smaps.p, B, coils.data(), B, V.p, d.p, nullptr,
                             (double *)loss.p, grad.p, stream);
    };
    sdn_status s = step();   // sizes the workspace
    float ms = 0.f;
    if (s == SDN_OK) s = hip_check(hipEventRecord(e0, st), "autotune timing");
    for (int r = 0; r < 3 && s == SDN_OK; ++r) s = step();
    if (s == SDN_OK) s = hip_check(hipEventRecord(e1, st), "autotune timing");
    if (s == SDN_OK) s = hip_check(hipEventSynchronize(e1), "autotune timing");
    if (s == SDN_OK) s = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune timing");
    (void)sdn_plan_destroy(p);
    if (s != SDN_OK) {
      // an option set the device cannot run (e.g. memory) is skipped
      if (s == SDN_E_HIP) err = s;
      continue;
    }
    const double t = ms / 3.0;
    if (best_t < 0.0 || t < best_t) {
      best_t = t;
      *best = o;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_t < 0.0)
    return err != SDN_OK ? err : fail(SDN_E_UNSUPPORTED, "sdn_autotune: no candidate ran");
  if (best_ms) *best_ms = best_t;
  return SDN_OK;
}

}  // extern "C"
