// Ragged volumes: several plans (image shapes, trajectories) evaluated as
// one call on the caller's stream.  The interpolation and the spreading of
// all volumes each run as one launch over the work items of every volume
// (the FFT passes, whose lengths differ between volumes, run volume by
// volume); volumes that cannot share those launches (different kernel
// widths or spreading engines, coil passes under a workspace budget, more
// than eight volumes) run each member plan's call in turn.  The group adds
// the loss reduction over volumes.
#include <vector>

#include "sdn_internal.h"

namespace sdn {
const char *last_error();
}

using namespace sdn;

namespace {

constexpr uint32_t kGroupMagic = 0x53444e47u;   // "SDNG"

__global__ void k_sum_f64(const double *in, int n, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += in[i];   // fixed order: volume order
  *out = s;
}

}  // namespace

struct sdn_group_s {
  uint32_t magic = kGroupMagic;
  std::vector<sdn_plan> plans;
  double *losses = nullptr;   // [n] per-volume losses
};

extern "C" {

sdn_status sdn_group_create(sdn_group *out, const sdn_plan *plans, int n) {
  if (!out) return fail(SDN_E_INVALID, "sdn_group_create: out is NULL");
  *out = nullptr;
  if (!plans || n < 1) return fail(SDN_E_INVALID, "sdn_group_create: need at least one plan");
  sdn_plan_info info;
  for (int v = 0; v < n; ++v)
    if (sdn_plan_get_info(plans[v], &info) != SDN_OK)
      return fail(SDN_E_STATE, "sdn_group_create: not a live plan");
  auto *g = new sdn_group_s;
  g->plans.assign(plans, plans + n);
  sdn_status s = hip_check(hipMalloc((void **)&g->losses, (size_t)n * sizeof(double)),
                           "sdn_group_create: loss slots");
  if (s != SDN_OK) {
    delete g;
    return s;
  }
  *out = g;
  return SDN_OK;
}

sdn_status sdn_group_destroy(sdn_group g) {
  if (!g) return SDN_OK;
  if (g->magic != kGroupMagic) return fail(SDN_E_STATE, "sdn_group_destroy: not a live group");
  if (g->losses) (void)hipFree(g->losses);
  g->magic = 0;
  delete g;
  return SDN_OK;
}

#define SDN_GROUP_CHECK(g, fn)                                                      \
  do {                                                                              \
    if (!(g) || (g)->magic != kGroupMagic) return fail(SDN_E_STATE, fn ": not a live group"); \
  } while (0)

sdn_status sdn_group_mrf_forward(sdn_group g, const void *const *x, int K,
                                 const void *const *smaps, const int *C,
                                 const int32_t *const *coil_idx, int B, const void *const *V,
                                 void *const *y, void *stream) {
  SDN_GROUP_CHECK(g, "sdn_group_mrf_forward");
  if (!x || !smaps || !C || !coil_idx || !V || !y)
    return fail(SDN_E_INVALID, "sdn_group_mrf_forward: null argument array");
  const sdn_status fs = group_forward_fused(g->plans.data(), (int)g->plans.size(), x, K, smaps, C,
                                            coil_idx, B, V, y, stream);
  if (fs != SDN_E_UNSUPPORTED) return fs;
  for (size_t v = 0; v < g->plans.size(); ++v) {
    const sdn_status s = sdn_mrf_forward(g->plans[v], x[v], K, smaps[v], C[v], coil_idx[v], B,
                                         V[v], y[v], stream);
    if (s != SDN_OK) return s;
  }
  return SDN_OK;
}

sdn_status sdn_group_mrf_adjoint(sdn_group g, const void *const *y, int K,
                                 const void *const *smaps, const int *C,
                                 const int32_t *const *coil_idx, int B, const void *const *V,
                                 void *const *x_out, int accumulate, void *stream) {
  SDN_GROUP_CHECK(g, "sdn_group_mrf_adjoint");
  if (!y || !smaps || !C || !coil_idx || !V || !x_out)
    return fail(SDN_E_INVALID, "sdn_group_mrf_adjoint: null argument array");
  const sdn_status fs = group_adjoint_fused(g->plans.data(), (int)g->plans.size(), y, K, smaps, C,
                                            coil_idx, B, V, x_out, accumulate, stream);
  if (fs != SDN_E_UNSUPPORTED) return fs;
  for (size_t v = 0; v < g->plans.size(); ++v) {
    const sdn_status s = sdn_mrf_adjoint(g->plans[v], y[v], K, smaps[v], C[v], coil_idx[v], B,
                                         V[v], x_out[v], accumulate, stream);
    if (s != SDN_OK) return s;
  }
  return SDN_OK;
}

sdn_status sdn_group_mrf_dc_grad(sdn_group g, const void *const *x, int K,
                                 const void *const *smaps, const int *C,
                                 const int32_t *const *coil_idx, int B, const void *const *V,
                                 const void *const *d, const float *const *w, double *loss,
                                 void *const *grad, void *stream) {
  SDN_GROUP_CHECK(g, "sdn_group_mrf_dc_grad");
  if (!x || !smaps || !C || !coil_idx || !V || !d || !grad || !loss)
    return fail(SDN_E_INVALID, "sdn_group_mrf_dc_grad: null argument");
  const int n = (int)g->plans.size();
  const sdn_status fs = group_dc_grad_fused(g->plans.data(), n, x, K, smaps, C, coil_idx, B, V, d,
                                            w, g->losses, grad, stream);
  if (fs != SDN_E_UNSUPPORTED && fs != SDN_OK) return fs;
  for (int v = 0; v < n && fs == SDN_E_UNSUPPORTED; ++v) {
    const sdn_status s = sdn_mrf_dc_grad(g->plans[v], x[v], K, smaps[v], C[v], coil_idx[v], B,
                                         V[v], d[v], w ? w[v] : nullptr, g->losses + v,
                                         grad[v], stream);
    if (s != SDN_OK) return s;
  }
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, (hipStream_t)stream, g->losses, n, loss);
  return hip_check(hipGetLastError(), "sdn_group_mrf_dc_grad: loss sum");
}

}  // extern "C"
