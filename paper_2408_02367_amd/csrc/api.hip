// Entry points of the C ABI: plain type-2 / type-1 NUFFTs, the batched MRF
// subspace operator A_c and its adjoint, the fused DC gradient, and the
// plain per-coil/per-channel form of the same operators.
//
// Batched calls put all B*K (coil, channel) pairs of the minibatch through
// each stage in one launch: fused x pass, y pass, z pass, interpolation
// with the subspace mix (forward) and spread with the conjugate mix, two
// inverse passes and the fused x pass that sums over coils (adjoint).  The
// forward's fine grids are never kept for the adjoint: A is linear, so its
// adjoint needs none of them, and the same workspace serves both.
#include <algorithm>
#include <mutex>
#include <string>

#include "sdn_internal.h"

using namespace sdn;

namespace {

sdn_status check_plan(sdn_plan p, const char *fn) {
  if (!p || p->magic != kPlanMagic)
    return fail(SDN_E_STATE, std::string(fn) + ": not a live plan");
  return SDN_OK;
}

size_t fine_cells(const sdn_plan_s &p) {
  return (size_t)p.ax[0].nf * p.ax[1].nf * p.ax[2].nf;
}

size_t image_voxels(const sdn_plan_s &p) {
  return (size_t)p.ax[0].N * p.ax[1].N * p.ax[2].N;
}

sdn_status ensure_grid(sdn_plan_s *p, size_t elems) {
  elems += elems & 1;   // whole float4s for the fill kernel
  if (p->grid_cap >= elems) return SDN_OK;
  if (p->grid) (void)hipFree(p->grid);
  p->grid = nullptr;
  p->grid_cap = 0;
  sdn_status s = hip_check(hipMalloc((void **)&p->grid, elems * sizeof(float2)),
                           "fine-grid workspace");
  if (s == SDN_OK) p->grid_cap = elems;
  return s;
}

sdn_status ensure_kbuf(sdn_plan_s *p, size_t elems) {
  if (p->kbuf_cap >= elems) return SDN_OK;
  if (p->kbuf) (void)hipFree(p->kbuf);
  p->kbuf = nullptr;
  p->kbuf_cap = 0;
  sdn_status s = hip_check(hipMalloc((void **)&p->kbuf, elems * sizeof(float2)),
                           "k-space workspace");
  if (s == SDN_OK) p->kbuf_cap = elems;
  return s;
}

sdn_status ensure_part(sdn_plan_s *p, int groups, int K) {
  const size_t elems = spread_part_elems(*p, groups, K);
  if (p->part_cap >= elems) return SDN_OK;
  if (p->part) (void)hipFree(p->part);
  p->part = nullptr;
  p->part_cap = 0;
  sdn_status s = hip_check(hipMalloc((void **)&p->part, elems * sizeof(float2)),
                           "spreading partials");
  if (s == SDN_OK) p->part_cap = elems;
  return s;
}

sdn_status ensure_lpart(sdn_plan_s *p, int groups) {
  const size_t n = interp_loss_parts(*p, groups) + kSumChunks;
  if (p->lpart_cap >= n) return SDN_OK;
  if (p->lpart) (void)hipFree(p->lpart);
  p->lpart = nullptr;
  p->lpart_cap = 0;
  sdn_status s = hip_check(hipMalloc((void **)&p->lpart, n * sizeof(double)), "loss partials");
  if (s == SDN_OK) p->lpart_cap = n;
  return s;
}

// Channels of P-channel grids that fit the workspace budget at once.
sdn_status channels_per_pass(const sdn_plan_s &p, int unit, int units, int *per,
                             const char *fn) {
  const size_t bytes_unit = (size_t)unit * fine_cells(p) * sizeof(float2);
  if (p.budget == 0) {
    *per = units;
    return SDN_OK;
  }
  const size_t n = p.budget / bytes_unit;
  if (n < 1)
    return fail(SDN_E_NOMEM, std::string(fn) + ": workspace budget below one coil's grids");
  *per = (int)std::min<size_t>(n, (size_t)units);
  return SDN_OK;
}

#define SDN_TRY(expr)                      \
  do {                                     \
    sdn_status _s = (expr);                \
    if (_s != SDN_OK) return _s;           \
  } while (0)
#define SDN_HIP(expr, what) SDN_TRY(hip_check((expr), what))

hipEvent_t pooled_event(sdn_plan_s *p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch one stage; while profiling, bracket it with events on `st`.
#define SDN_STAGE(p, stage, expr, what)                                         \
  do {                                                                          \
    hipEvent_t _e0 = (p)->prof ? pooled_event(p) : nullptr;                     \
    if (_e0) (void)hipEventRecord(_e0, st);                                     \
    SDN_HIP((expr), what);                                                      \
    if (_e0) {                                                                  \
      hipEvent_t _e1 = pooled_event(p);                                         \
      if (_e1) {                                                                \
        (void)hipEventRecord(_e1, st);                                          \
        (p)->prof_ev.push_back({(stage), _e0, _e1});                            \
      } else {                                                                  \
        (p)->ev_pool.push_back(_e0);                                            \
      }                                                                         \
    }                                                                           \
  } while (0)

sdn_status check_mrf_args(const sdn_plan_s &p, const char *fn, const void *x, int K,
                          const void *smaps, int C, const int32_t *coil_idx, int B,
                          const void *V, const void *y) {
  if (K < 1 || K > kMaxK) return fail(SDN_E_INVALID, std::string(fn) + ": K must be in [1, 8]");
  if (B < 1 || B > kMaxB) return fail(SDN_E_INVALID, std::string(fn) + ": B must be in [1, 64]");
  if (C < 1) return fail(SDN_E_INVALID, std::string(fn) + ": C must be >= 1");
  if (!x || !smaps || !coil_idx || !V)
    return fail(SDN_E_INVALID, std::string(fn) + ": null array argument");
  if (!y && p.M > 0) return fail(SDN_E_INVALID, std::string(fn) + ": null k-space argument");
  for (int b = 0; b < B; ++b)
    if (coil_idx[b] < 0 || coil_idx[b] >= C)
      return fail(SDN_E_RANGE, std::string(fn) + ": coil index outside [0, C)");
  if (p.ax[0].nf / K < 2)
    return fail(SDN_E_UNSUPPORTED, std::string(fn) + ": too many channels for this grid");
  return SDN_OK;
}

CoilList coil_list(const int32_t *idx, int b0, int n) {
  CoilList c{};
  for (int i = 0; i < n; ++i) c.idx[i] = idx[b0 + i];
  return c;
}

// forward stages for one chunk of coils: grid <- FFT3(pad(deapod(S x)))
sdn_status forward_grid(sdn_plan_s *p, const float2 *x, int K, const float2 *smaps,
                        const CoilList &coils, int B, float2 *grid, hipStream_t st) {
  const int P = B * K;
  SDN_STAGE(p, SDN_STAGE_PRE_FFTX, launch_pre_fftx(*p, x, K, smaps, coils, B, grid, st), "forward x pass");
  SDN_STAGE(p, SDN_STAGE_FFT_Y, launch_fft_axis(*p, grid, P, 1, false, true, false, st), "forward y pass");
  SDN_STAGE(p, SDN_STAGE_FFT_Z, launch_fft_axis(*p, grid, P, 2, false, true, false, st), "forward z pass");
  return SDN_OK;
}
sdn_status forward_grid(sdn_plan_s *p, const float2 *x, int K, const float2 *smaps,
                        const CoilList &coils, int B, hipStream_t st) {
  return forward_grid(p, x, K, smaps, coils, B, p->grid, st);
}

// adjoint stages after spreading: x_out (+)= sum_b conj(S_b) crop(IFFT3(grid)) / deapod
sdn_status adjoint_grid(sdn_plan_s *p, int K, const float2 *smaps, const CoilList &coils, int B,
                        float2 *xout, int accumulate, float2 *grid, hipStream_t st) {
  const int P = B * K;
  SDN_STAGE(p, SDN_STAGE_IFFT_Z, launch_fft_axis(*p, grid, P, 2, true, false, true, st), "adjoint z pass");
  SDN_STAGE(p, SDN_STAGE_IFFT_Y, launch_fft_axis(*p, grid, P, 1, true, false, true, st), "adjoint y pass");
  SDN_STAGE(p, SDN_STAGE_POST_IFFTX,
            launch_post_ifftx(*p, grid, K, smaps, coils, B, xout, accumulate, st),
            "adjoint x pass");
  return SDN_OK;
}
sdn_status adjoint_grid(sdn_plan_s *p, int K, const float2 *smaps, const CoilList &coils, int B,
                        float2 *xout, int accumulate, hipStream_t st) {
  return adjoint_grid(p, K, smaps, coils, B, xout, accumulate, p->grid, st);
}

__global__ void k_zero_c64(float2 *a, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = make_float2(0.f, 0.f);
}

sdn_status zero_user(float2 *a, size_t n, hipStream_t st) {
  if (n == 0) return SDN_OK;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 1u << 16);
  hipLaunchKernelGGL(k_zero_c64, dim3(blocks), dim3(256), 0, st, a, n);
  return hip_check(hipGetLastError(), "zero fill");
}

sdn_status ensure_vec(sdn_plan_s *p, size_t elems) {
  if (p->vecbuf_cap >= elems) return SDN_OK;
  if (p->vecbuf) (void)hipFree(p->vecbuf);
  p->vecbuf = nullptr;
  p->vecbuf_cap = 0;
  sdn_status s = hip_check(hipMalloc((void **)&p->vecbuf, elems * sizeof(float2)),
                           "solver vectors");
  if (s == SDN_OK) p->vecbuf_cap = elems;
  return s;
}

sdn_status ensure_red(sdn_plan_s *p, size_t n) {
  if (p->red_cap >= n) return SDN_OK;
  if (p->red) (void)hipFree(p->red);
  p->red = nullptr;
  p->red_cap = 0;
  sdn_status s = hip_check(hipMalloc((void **)&p->red, n * sizeof(double)), "reduction scratch");
  if (s == SDN_OK) p->red_cap = n;
  return s;
}

// A^H W A x over the listed coils, chunked by the workspace budget, into
// out (accumulated across chunks; onto out's contents when accumulate);
// loss += sum w |A x|^2.  With adjoint = false only the forward half runs
// (loss only; out untouched).
sdn_status normal_pass(sdn_plan_s *p, const float2 *x, int K, const float2 *smaps,
                       const int32_t *coil_idx, int B, const float2 *V, const float *w,
                       float2 *out, int accumulate, double *loss, bool adjoint, hipStream_t st) {
  if (p->M == 0) {
    if (adjoint && !accumulate) return zero_user(out, (size_t)K * image_voxels(*p), st);
    return SDN_OK;
  }
  int per;
  SDN_TRY(channels_per_pass(*p, K, B, &per, "normal operator"));
  SDN_TRY(ensure_kbuf(p, (size_t)per * p->M));
  SDN_TRY(ensure_lpart(p, per));
  for (int b0 = 0; b0 < B; b0 += per) {
    const int bc = std::min(per, B - b0);
    const CoilList coils = coil_list(coil_idx, b0, bc);
    SDN_TRY(ensure_grid(p, (size_t)bc * K * fine_cells(*p)));
    SDN_TRY(forward_grid(p, x, K, smaps, coils, bc, st));
    InterpArgs a{};
    a.grid = p->grid;
    a.P = bc * K;
    a.groups = bc;
    a.kg = K;
    a.V = V;
    a.dc = 1;
    a.rscale = 1.f;
    a.d = nullptr;
    a.w = w;
    a.r_plan = p->kbuf;
    a.loss = loss;
    a.loss_part = p->lpart;
    a.rmax = p->absmax;
    SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp(*p, a, st), "interpolation + weighting");
    if (!adjoint) continue;
    SDN_TRY(ensure_part(p, bc, K));
    SpreadArgs s{};
    s.grid = p->grid;
    s.part = p->part;
    s.groups = bc;
    s.K = K;
    s.V = V;
    s.src = p->kbuf;
    s.src_plan_order = true;
    s.src_max_ready = true;   // recorded by the interpolation above
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread(*p, s, st), "spreading");
    SDN_TRY(adjoint_grid(p, K, smaps, coils, bc, out, (accumulate || b0 > 0) ? 1 : 0, st));
  }
  return SDN_OK;
}

// A^H W y over the listed coils (y [B][M] in user order) into out.
sdn_status rhs_pass(sdn_plan_s *p, const float2 *y, int K, const float2 *smaps,
                    const int32_t *coil_idx, int B, const float2 *V, const float *w, float2 *out,
                    hipStream_t st) {
  if (p->M == 0) return zero_user(out, (size_t)K * image_voxels(*p), st);
  int per;
  SDN_TRY(channels_per_pass(*p, K, B, &per, "adjoint of the data"));
  SDN_TRY(ensure_kbuf(p, (size_t)per * p->M));
  for (int b0 = 0; b0 < B; b0 += per) {
    const int bc = std::min(per, B - b0);
    const CoilList coils = coil_list(coil_idx, b0, bc);
    SDN_TRY(ensure_grid(p, (size_t)bc * K * fine_cells(*p)));
    SDN_TRY(ensure_part(p, bc, K));
    SDN_HIP(launch_weighted_plan(*p, y + (size_t)b0 * p->M, bc, w, 1.f, p->kbuf, st),
            "weighted data");
    SpreadArgs s{};
    s.grid = p->grid;
    s.part = p->part;
    s.groups = bc;
    s.K = K;
    s.V = V;
    s.src = p->kbuf;
    s.src_plan_order = true;
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread(*p, s, st), "spreading");
    SDN_TRY(adjoint_grid(p, K, smaps, coils, bc, out, b0 > 0 ? 1 : 0, st));
  }
  return SDN_OK;
}

// Buffers of one DC-gradient call for `per` coils at a time: fine grids
// (per K channels), plan-order residuals (per coils), spreading partials and
// the interpolation's loss partials.
struct DcWork {
  float2 *grid;
  float2 *kbuf;
  float2 *part;
  double *lpart;
};

// Complex elements (grid, kbuf, part) and doubles (lpart) that DcWork
// needs for `per` coils of K channels.
void dc_work_sizes(const sdn_plan_s &p, int per, int K, size_t *grid, size_t *kbuf, size_t *part,
                   size_t *lpart) {
  *grid = (size_t)per * K * fine_cells(p);
  *grid += *grid & 1;   // whole float4s for the fill kernel
  *kbuf = (size_t)per * p.M;
  *part = spread_part_elems(p, per, K);
  *lpart = interp_loss_parts(p, per) + kSumChunks;
}

// loss = sum_b w |A_b x - d_b|^2 and grad = 2 A^H w (A x - d), coils in
// chunks of `per` (the arguments have been checked).
sdn_status dc_grad_pass(sdn_plan_s *p, const DcWork &ws, int per, const float2 *x, int K,
                        const float2 *smaps, const int32_t *coil_idx, int B, const float2 *V,
                        const float2 *d, const float *w, double *loss, float2 *grad,
                        hipStream_t st) {
  SDN_HIP(launch_fill_zero_f64(loss, 1, st), "loss clear");
  if (p->M == 0) return zero_user(grad, (size_t)K * image_voxels(*p), st);
  for (int b0 = 0; b0 < B; b0 += per) {
    const int bc = std::min(per, B - b0);
    const CoilList coils = coil_list(coil_idx, b0, bc);
    SDN_TRY(forward_grid(p, x, K, smaps, coils, bc, ws.grid, st));
    InterpArgs a{};
    a.grid = ws.grid;
    a.P = bc * K;
    a.groups = bc;
    a.kg = K;
    a.V = V;
    a.dc = 1;
    a.rscale = 2.f;
    a.d = d + (size_t)b0 * p->M;
    a.w = w;
    a.r_plan = ws.kbuf;
    a.loss = loss;
    a.loss_part = ws.lpart;
    a.rmax = p->absmax;
    SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp(*p, a, st), "interpolation + residual");
    SpreadArgs s{};
    s.grid = ws.grid;
    s.part = ws.part;
    s.groups = bc;
    s.K = K;
    s.V = V;
    s.src = ws.kbuf;
    s.src_plan_order = true;
    s.src_max_ready = true;   // recorded by the interpolation above
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread(*p, s, st), "spreading");
    SDN_TRY(adjoint_grid(p, K, smaps, coils, bc, grad, b0 > 0 ? 1 : 0, ws.grid, st));
  }
  return SDN_OK;
}

// ------------------------------------------- the DC gradient without allocation
// Buffers of sdn_mrf_dc_grad_noalloc: one array per GPU in the code object,
// held until the process ends.  In host code `scratch` is a host-side
// stand-in; its device address is looked up once per device.
static __device__ __align__(256) unsigned char scratch[SDN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct ScratchAddrs {
  std::mutex m;
  unsigned char *ptr[kMaxDevices] = {};
};

ScratchAddrs &scratch_addrs() {
  static ScratchAddrs s;
  return s;
}

// Device address of `scratch` on `device` (looked up with that device
// current, on the first call for it).
sdn_status scratch_on(int device, unsigned char **out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(SDN_E_UNSUPPORTED, "sdn_mrf_dc_grad_noalloc: device index out of range");
  ScratchAddrs &s = scratch_addrs();
  std::lock_guard<std::mutex> lock(s.m);
  if (s.ptr[device] == nullptr) {
    int cur = -1;
    SDN_HIP(hipGetDevice(&cur), "sdn_mrf_dc_grad_noalloc: current device");
    if (cur != device) SDN_HIP(hipSetDevice(device), "sdn_mrf_dc_grad_noalloc: set device");
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    SDN_HIP(e, "sdn_mrf_dc_grad_noalloc: static workspace address");
    if (ptr == nullptr) return fail(SDN_E_HIP, "sdn_mrf_dc_grad_noalloc: no static workspace");
    s.ptr[device] = (unsigned char *)ptr;
  }
  *out = s.ptr[device];
  return SDN_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Bytes of the DcWork of `per` coils carved from one block (256-byte
// aligned pieces).
size_t dc_work_bytes(const sdn_plan_s &p, int per, int K) {
  size_t g, kb, pt, lp;
  dc_work_sizes(p, per, K, &g, &kb, &pt, &lp);
  return align256(g * sizeof(float2)) + align256(kb * sizeof(float2)) +
         align256(pt * sizeof(float2)) + align256(lp * sizeof(double));
}

}  // namespace

extern "C" {

sdn_status sdn_forward(sdn_plan p, const void *img, void *ksp, int batch, void *stream) {
  SDN_TRY(check_plan(p, "sdn_forward"));
  if (batch < 0) return fail(SDN_E_INVALID, "sdn_forward: batch < 0");
  if (batch == 0 || p->M == 0) return SDN_OK;
  if (!img || !ksp) return fail(SDN_E_INVALID, "sdn_forward: null array argument");
  hipStream_t st = (hipStream_t)stream;
  int per;
  SDN_TRY(channels_per_pass(*p, 1, batch, &per, "sdn_forward"));
  const int cap = std::max(1, 8192 / p->ax[0].nf - 1);
  per = std::min(per, std::max(1, cap));
  const size_t nvox = image_voxels(*p);
  CoilList one{};
  for (int c0 = 0; c0 < batch; c0 += per) {
    const int pc = std::min(per, batch - c0);
    SDN_TRY(ensure_grid(p, (size_t)pc * fine_cells(*p)));
    SDN_TRY(forward_grid(p, (const float2 *)img + c0 * nvox, pc, nullptr, one, 1, st));
    InterpArgs a{};
    a.grid = p->grid;
    a.P = pc;
    a.groups = pc;
    a.kg = 1;
    a.y = (float2 *)ksp + (size_t)c0 * p->M;
    SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp(*p, a, st), "interpolation");
  }
  return SDN_OK;
}

sdn_status sdn_adjoint(sdn_plan p, const void *ksp, void *img, int batch, void *stream) {
  SDN_TRY(check_plan(p, "sdn_adjoint"));
  if (batch < 0) return fail(SDN_E_INVALID, "sdn_adjoint: batch < 0");
  if (batch == 0) return SDN_OK;
  if (!img || (!ksp && p->M > 0)) return fail(SDN_E_INVALID, "sdn_adjoint: null array argument");
  hipStream_t st = (hipStream_t)stream;
  const size_t nvox = image_voxels(*p);
  if (p->M == 0) return zero_user((float2 *)img, (size_t)batch * nvox, st);
  int per;
  SDN_TRY(channels_per_pass(*p, 1, batch, &per, "sdn_adjoint"));
  const int cap = std::max(1, 8192 / p->ax[0].nf - 1);
  per = std::min(per, cap);
  CoilList one{};
  for (int c0 = 0; c0 < batch; c0 += per) {
    const int pc = std::min(per, batch - c0);
    const size_t cells = (size_t)pc * fine_cells(*p);
    SDN_TRY(ensure_grid(p, cells));
    SDN_TRY(ensure_part(p, pc, 1));
    SpreadArgs s{};
    s.grid = p->grid;
    s.part = p->part;
    s.groups = pc;
    s.K = 1;
    s.V = nullptr;
    s.src = (const float2 *)ksp + (size_t)c0 * p->M;
    s.src_plan_order = false;
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread(*p, s, st), "spreading");
    SDN_TRY(adjoint_grid(p, pc, nullptr, one, 1, (float2 *)img + c0 * nvox, 0, st));
  }
  return SDN_OK;
}

sdn_status sdn_mrf_forward(sdn_plan p, const void *x, int K, const void *smaps, int C,
                           const int32_t *coil_idx, int B, const void *V, void *y,
                           void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_forward"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_forward", x, K, smaps, C, coil_idx, B, V, y));
  if (p->M == 0) return SDN_OK;
  hipStream_t st = (hipStream_t)stream;
  int per;
  SDN_TRY(channels_per_pass(*p, K, B, &per, "sdn_mrf_forward"));
  for (int b0 = 0; b0 < B; b0 += per) {
    const int bc = std::min(per, B - b0);
    const CoilList coils = coil_list(coil_idx, b0, bc);
    SDN_TRY(ensure_grid(p, (size_t)bc * K * fine_cells(*p)));
    SDN_TRY(forward_grid(p, (const float2 *)x, K, (const float2 *)smaps, coils, bc, st));
    InterpArgs a{};
    a.grid = p->grid;
    a.P = bc * K;
    a.groups = bc;
    a.kg = K;
    a.V = (const float2 *)V;
    a.y = (float2 *)y + (size_t)b0 * p->M;
    SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp(*p, a, st), "interpolation");
  }
  return SDN_OK;
}

sdn_status sdn_mrf_adjoint(sdn_plan p, const void *y, int K, const void *smaps, int C,
                           const int32_t *coil_idx, int B, const void *V, void *x_out,
                           int accumulate, void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_adjoint"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_adjoint", x_out, K, smaps, C, coil_idx, B, V, y));
  hipStream_t st = (hipStream_t)stream;
  if (p->M == 0) {
    if (!accumulate) return zero_user((float2 *)x_out, (size_t)K * image_voxels(*p), st);
    return SDN_OK;
  }
  int per;
  SDN_TRY(channels_per_pass(*p, K, B, &per, "sdn_mrf_adjoint"));
  for (int b0 = 0; b0 < B; b0 += per) {
    const int bc = std::min(per, B - b0);
    const CoilList coils = coil_list(coil_idx, b0, bc);
    const size_t cells = (size_t)bc * K * fine_cells(*p);
    SDN_TRY(ensure_grid(p, cells));
    SDN_TRY(ensure_part(p, bc, K));
    SpreadArgs s{};
    s.grid = p->grid;
    s.part = p->part;
    s.groups = bc;
    s.K = K;
    s.V = (const float2 *)V;
    s.src = (const float2 *)y + (size_t)b0 * p->M;
    s.src_plan_order = false;
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread(*p, s, st), "spreading");
    SDN_TRY(adjoint_grid(p, K, (const float2 *)smaps, coils, bc, (float2 *)x_out,
                         (accumulate || b0 > 0) ? 1 : 0, st));
  }
  return SDN_OK;
}

sdn_status sdn_mrf_dc_grad(sdn_plan p, const void *x, int K, const void *smaps, int C,
                           const int32_t *coil_idx, int B, const void *V, const void *d,
                           const float *w, double *loss, void *grad, void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_dc_grad"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_dc_grad", x, K, smaps, C, coil_idx, B, V, d));
  if (!loss || !grad) return fail(SDN_E_INVALID, "sdn_mrf_dc_grad: null output argument");
  hipStream_t st = (hipStream_t)stream;
  int per = 1;
  if (p->M > 0) {
    SDN_TRY(channels_per_pass(*p, K, B, &per, "sdn_mrf_dc_grad"));
    SDN_TRY(ensure_kbuf(p, (size_t)per * p->M));
    SDN_TRY(ensure_grid(p, (size_t)per * K * fine_cells(*p)));
    SDN_TRY(ensure_part(p, per, K));
    SDN_TRY(ensure_lpart(p, per));
  }
  const DcWork ws{p->grid, p->kbuf, p->part, p->lpart};
  return dc_grad_pass(p, ws, per, (const float2 *)x, K, (const float2 *)smaps, coil_idx, B,
                      (const float2 *)V, (const float2 *)d, w, loss, (float2 *)grad, st);
}

sdn_status sdn_mrf_forward_plain(sdn_plan p, const void *x, int K, const void *smaps, int C,
                                 const int32_t *coil_idx, int B, const void *V, void *y,
                                 void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_forward_plain"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_forward_plain", x, K, smaps, C, coil_idx, B, V, y));
  if (p->M == 0) return SDN_OK;
  hipStream_t st = (hipStream_t)stream;
  const size_t nvox = image_voxels(*p);
  SDN_TRY(ensure_grid(p, fine_cells(*p)));
  SDN_TRY(ensure_kbuf(p, (size_t)p->M));
  for (int b = 0; b < B; ++b) {
    const CoilList coil = coil_list(coil_idx, b, 1);
    for (int k = 0; k < K; ++k) {
      SDN_TRY(forward_grid(p, (const float2 *)x + k * nvox, 1, (const float2 *)smaps, coil, 1, st));
      InterpArgs a{};
      a.grid = p->grid;
      a.P = 1;
      a.groups = 1;
      a.kg = 1;
      a.y = p->kbuf;
      SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp(*p, a, st), "interpolation");
      SDN_STAGE(p, SDN_STAGE_MIX, launch_mix_fwd(*p, p->kbuf, (const float2 *)V, K, k, (float2 *)y + (size_t)b * p->M,
                             k > 0 ? 1 : 0, st), "subspace mix");
    }
  }
  return SDN_OK;
}

sdn_status sdn_mrf_adjoint_plain(sdn_plan p, const void *y, int K, const void *smaps, int C,
                                 const int32_t *coil_idx, int B, const void *V, void *x_out,
                                 int accumulate, void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_adjoint_plain"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_adjoint_plain", x_out, K, smaps, C, coil_idx, B, V, y));
  hipStream_t st = (hipStream_t)stream;
  const size_t nvox = image_voxels(*p);
  if (p->M == 0) {
    if (!accumulate) return zero_user((float2 *)x_out, (size_t)K * nvox, st);
    return SDN_OK;
  }
  SDN_TRY(ensure_grid(p, fine_cells(*p)));
  SDN_TRY(ensure_kbuf(p, (size_t)p->M));
  for (int b = 0; b < B; ++b) {
    const CoilList coil = coil_list(coil_idx, b, 1);
    for (int k = 0; k < K; ++k) {
      SDN_STAGE(p, SDN_STAGE_MIX, launch_mix_adj(*p, (const float2 *)y + (size_t)b * p->M, (const float2 *)V, K, k,
                             p->kbuf, st), "subspace mix");
      SDN_TRY(ensure_part(p, 1, 1));
      SpreadArgs s{};
      s.grid = p->grid;
      s.part = p->part;
      s.groups = 1;
      s.K = 1;
      s.V = nullptr;
      s.src = p->kbuf;
      s.src_plan_order = false;
      SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread(*p, s, st), "spreading");
      SDN_TRY(adjoint_grid(p, 1, (const float2 *)smaps, coil, 1, (float2 *)x_out + k * nvox,
                           (accumulate || b > 0) ? 1 : 0, st));
    }
  }
  return SDN_OK;
}

sdn_status sdn_dcf_estimate(sdn_plan p, int iterations, float *w_out, void *stream) {
  SDN_TRY(check_plan(p, "sdn_dcf_estimate"));
  if (iterations < 1 || iterations > 1000)
    return fail(SDN_E_INVALID, "sdn_dcf_estimate: iterations outside 1 .. 1000");
  if (p->M > 0 && !w_out) return fail(SDN_E_INVALID, "sdn_dcf_estimate: w_out is NULL");
  if (p->M == 0) return SDN_OK;
  hipStream_t st = (hipStream_t)stream;
  SDN_TRY(ensure_grid(p, fine_cells(*p)));
  SDN_TRY(ensure_part(p, 1, 1));
  SDN_TRY(ensure_kbuf(p, 2 * (size_t)p->M));
  float2 *w = p->kbuf, *cw = p->kbuf + p->M;
  SDN_HIP(launch_dcf_step(w, cw, p->M, true, st), "dcf init");
  for (int it = 0; it < iterations; ++it) {
    // C w: spread w onto the fine grid, interpolate it back (no FFT)
    SpreadArgs s{};
    s.grid = p->grid;
    s.part = p->part;
    s.groups = 1;
    s.K = 1;
    s.V = nullptr;
    s.src = w;
    s.src_plan_order = false;
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread(*p, s, st), "dcf spreading");
    InterpArgs a{};
    a.grid = p->grid;
    a.P = 1;
    a.groups = 1;
    a.kg = 1;
    a.y = cw;
    SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp(*p, a, st), "dcf interpolation");
    SDN_HIP(launch_dcf_step(w, cw, p->M, false, st), "dcf update");
  }
  SDN_HIP(launch_real_part(w, w_out, p->M, st), "dcf output");
  return SDN_OK;
}

sdn_status sdn_mrf_normal(sdn_plan p, const void *x, int K, const void *smaps, int C,
                          const int32_t *coil_idx, int B, const void *V, const float *w,
                          float lambda, void *out, void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_normal"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_normal", x, K, smaps, C, coil_idx, B, V, x));
  if (!out) return fail(SDN_E_INVALID, "sdn_mrf_normal: null output argument");
  if (!(lambda >= 0.f) || lambda > 3.0e38f)
    return fail(SDN_E_INVALID, "sdn_mrf_normal: lambda must be finite and >= 0");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)K * image_voxels(*p);
  SDN_TRY(ensure_red(p, kDotBlocks + 1));
  double *part = p->red, *loss = p->red + kDotBlocks;
  SDN_HIP(launch_fill_zero_f64(loss, 1, st), "scratch clear");
  SDN_TRY(normal_pass(p, (const float2 *)x, K, (const float2 *)smaps, coil_idx, B,
                      (const float2 *)V, w, (float2 *)out, 0, loss, true, st));
  if (lambda != 0.f)
    SDN_HIP(launch_axpy_dot((float2 *)out, (const float2 *)x, lambda, n, part, st),
            "Tikhonov term");
  return SDN_OK;
}

sdn_status sdn_mrf_cg(sdn_plan p, const void *y, int K, const void *smaps, int C,
                      const int32_t *coil_idx, int B, const void *V, const float *w, float lambda,
                      int iterations, void *x, double *history, void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_cg"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_cg", x, K, smaps, C, coil_idx, B, V, y));
  if (iterations < 0 || iterations > 100000)
    return fail(SDN_E_INVALID, "sdn_mrf_cg: iterations must be in [0, 100000]");
  if (!(lambda >= 0.f) || lambda > 3.0e38f)
    return fail(SDN_E_INVALID, "sdn_mrf_cg: lambda must be finite and >= 0");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)K * image_voxels(*p);
  SDN_TRY(ensure_vec(p, 3 * n));
  SDN_TRY(ensure_red(p, (size_t)kDotBlocks + iterations + 3));
  float2 *xx = (float2 *)x, *r = p->vecbuf, *q = p->vecbuf + n, *Ap = p->vecbuf + 2 * n;
  double *part = p->red, *hist = p->red + kDotBlocks;
  double *pAp = hist + iterations + 1, *loss = pAp + 1;
  const float2 *S = (const float2 *)smaps, *VV = (const float2 *)V;
  SDN_HIP(launch_fill_zero_f64(loss, 1, st), "scratch clear");
  // r = b - (A^H W A + lambda) x0, q = r
  SDN_TRY(rhs_pass(p, (const float2 *)y, K, S, coil_idx, B, VV, w, r, st));
  SDN_TRY(normal_pass(p, xx, K, S, coil_idx, B, VV, w, Ap, 0, loss, true, st));
  if (lambda != 0.f) SDN_HIP(launch_axpy_dot(Ap, xx, lambda, n, part, st), "Tikhonov term");
  SDN_HIP(launch_cg_start(r, q, Ap, n, part, st), "cg start");
  SDN_HIP(launch_sum(part, kDotBlocks, 1.0, hist, st), "cg residual");
  for (int it = 0; it < iterations; ++it) {
    SDN_TRY(normal_pass(p, q, K, S, coil_idx, B, VV, w, Ap, 0, loss, true, st));
    SDN_HIP(launch_axpy_dot(Ap, q, lambda, n, part, st), "cg curvature");
    SDN_HIP(launch_sum(part, kDotBlocks, 1.0, pAp, st), "cg curvature");
    SDN_HIP(launch_cg_xr(xx, r, q, Ap, n, hist + it, pAp, part, st), "cg update");
    SDN_HIP(launch_sum(part, kDotBlocks, 1.0, hist + it + 1, st), "cg residual");
    SDN_HIP(launch_cg_p(q, r, n, hist + it + 1, hist + it, st), "cg direction");
  }
  if (history)
    SDN_HIP(hipMemcpyAsync(history, hist, (size_t)(iterations + 1) * sizeof(double),
                           hipMemcpyDeviceToDevice, st),
            "cg history");
  return SDN_OK;
}

sdn_status sdn_mrf_scaled_adjoint(sdn_plan p, const void *y, int K, const void *smaps, int C,
                                  const int32_t *coil_idx, int B, const void *V, const float *w,
                                  void *x_out, double *scale, void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_scaled_adjoint"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_scaled_adjoint", x_out, K, smaps, C, coil_idx, B, V, y));
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)K * image_voxels(*p);
  SDN_TRY(ensure_red(p, kDotBlocks + 2));
  double *part = p->red, *num = p->red + kDotBlocks, *den = num + 1;
  float2 *z = (float2 *)x_out;
  const float2 *S = (const float2 *)smaps, *VV = (const float2 *)V;
  SDN_TRY(rhs_pass(p, (const float2 *)y, K, S, coil_idx, B, VV, w, z, st));
  SDN_HIP(launch_fill_zero_f64(den, 1, st), "scratch clear");
  SDN_TRY(normal_pass(p, z, K, S, coil_idx, B, VV, w, nullptr, 0, den, false, st));
  SDN_HIP(launch_dot(z, z, n, part, st), "adjoint norm");
  SDN_HIP(launch_sum(part, kDotBlocks, 1.0, num, st), "adjoint norm");
  SDN_HIP(launch_scale_ratio(z, n, num, den, scale, st), "adjoint scale");
  return SDN_OK;
}

sdn_status sdn_tv_grad(sdn_plan p, const void *x, int K, float eps, float lambda, double *value,
                       void *grad, int accumulate, void *stream) {
  SDN_TRY(check_plan(p, "sdn_tv_grad"));
  if (!x) return fail(SDN_E_INVALID, "sdn_tv_grad: null image argument");
  if (!value && !grad) return fail(SDN_E_INVALID, "sdn_tv_grad: no output requested");
  if (K < 1 || K > kMaxK) return fail(SDN_E_INVALID, "sdn_tv_grad: K must be in [1, 8]");
  if (!(eps > 0.f) || eps > 1.0e18f)
    return fail(SDN_E_INVALID, "sdn_tv_grad: eps must be finite and > 0");
  if (!(lambda >= 0.f) || lambda > 3.0e38f)
    return fail(SDN_E_INVALID, "sdn_tv_grad: lambda must be finite and >= 0");
  hipStream_t st = (hipStream_t)stream;
  const int nb = tv_blocks(*p, K);
  SDN_TRY(ensure_red(p, (size_t)nb + kSumChunks));
  SDN_HIP(launch_tv(*p, (const float2 *)x, K, eps, lambda, (float2 *)grad, accumulate ? 1 : 0,
                    p->red, st),
          "total variation");
  if (value)
    SDN_HIP(launch_sum(p->red, nb, (double)lambda, value, st, p->red + nb),
            "total variation sum");
  return SDN_OK;
}

sdn_status sdn_workspace_size(sdn_plan p, int B, int K, size_t *bytes) {
  SDN_TRY(check_plan(p, "sdn_workspace_size"));
  if (!bytes || B < 1 || K < 1) return fail(SDN_E_INVALID, "sdn_workspace_size: bad argument");
  int per;
  SDN_TRY(channels_per_pass(*p, K, B, &per, "sdn_workspace_size"));
  size_t g, kb, pt, lp;
  dc_work_sizes(*p, per, K, &g, &kb, &pt, &lp);
  *bytes = (g + kb + pt) * sizeof(float2) + lp * sizeof(double);
  return SDN_OK;
}

sdn_status sdn_profile_enable(sdn_plan p, int enable) {
  SDN_TRY(check_plan(p, "sdn_profile_enable"));
  p->prof = enable ? 1 : 0;
  return SDN_OK;
}

sdn_status sdn_profile_read(sdn_plan p, double *ms, int64_t *launches, int reset) {
  SDN_TRY(check_plan(p, "sdn_profile_read"));
  for (auto &r : p->prof_ev) {
    SDN_HIP(hipEventSynchronize(r.stop), "profile event wait");
    float t = 0.f;
    SDN_HIP(hipEventElapsedTime(&t, r.start, r.stop), "profile event time");
    p->prof_ms[r.stage] += t;
    p->prof_n[r.stage] += 1;
    p->ev_pool.push_back(r.start);
    p->ev_pool.push_back(r.stop);
  }
  p->prof_ev.clear();
  for (int i = 0; i < SDN_NUM_STAGES; ++i) {
    if (ms) ms[i] = p->prof_ms[i];
    if (launches) launches[i] = p->prof_n[i];
    if (reset) {
      p->prof_ms[i] = 0.0;
      p->prof_n[i] = 0;
    }
  }
  return SDN_OK;
}

sdn_status sdn_release_workspace(sdn_plan p) {
  SDN_TRY(check_plan(p, "sdn_release_workspace"));
  if (p->grid) (void)hipFree(p->grid);
  if (p->kbuf) (void)hipFree(p->kbuf);
  if (p->part) (void)hipFree(p->part);
  if (p->vecbuf) (void)hipFree(p->vecbuf);
  if (p->red) (void)hipFree(p->red);
  if (p->lpart) (void)hipFree(p->lpart);
  p->grid = nullptr;
  p->kbuf = nullptr;
  p->part = nullptr;
  p->vecbuf = nullptr;
  p->red = nullptr;
  p->lpart = nullptr;
  p->grid_cap = p->kbuf_cap = p->part_cap = p->vecbuf_cap = p->red_cap = p->lpart_cap = 0;
  return SDN_OK;
}

sdn_status sdn_mrf_dc_grad_noalloc(sdn_plan p, const void *x, int K, const void *smaps, int C,
                                   const int32_t *coil_idx, int B, const void *V, const void *d,
                                   const float *w, double *loss, void *grad, void *stream) {
  SDN_TRY(check_plan(p, "sdn_mrf_dc_grad_noalloc"));
  SDN_TRY(check_mrf_args(*p, "sdn_mrf_dc_grad_noalloc", x, K, smaps, C, coil_idx, B, V, d));
  if (!loss || !grad) return fail(SDN_E_INVALID, "sdn_mrf_dc_grad_noalloc: null output argument");
  unsigned char *base = nullptr;
  SDN_TRY(scratch_on(p->device, &base));
  // the most coils per pass whose buffers fit the static workspace
  int per = B;
  while (per > 1 && dc_work_bytes(*p, per, K) > SDN_NOALLOC_SCRATCH_BYTES) --per;
  if (p->M > 0 && dc_work_bytes(*p, per, K) > SDN_NOALLOC_SCRATCH_BYTES)
    return fail(SDN_E_NOMEM, "sdn_mrf_dc_grad_noalloc: one coil's grids, residuals and partial "
                             "sums (" + std::to_string(dc_work_bytes(*p, 1, K)) +
                             " bytes) exceed the static workspace (" +
                             std::to_string((size_t)SDN_NOALLOC_SCRATCH_BYTES) + " bytes)");
  size_t g, kb, pt, lp;
  dc_work_sizes(*p, per, K, &g, &kb, &pt, &lp);
  DcWork ws;
  unsigned char *q = base;
  ws.grid = (float2 *)q;
  q += align256(g * sizeof(float2));
  ws.kbuf = (float2 *)q;
  q += align256(kb * sizeof(float2));
  ws.part = (float2 *)q;
  q += align256(pt * sizeof(float2));
  ws.lpart = (double *)q;
  // no stage events either: recording them may create events
  const int prof = p->prof;
  p->prof = 0;
  const sdn_status s = dc_grad_pass(p, ws, per, (const float2 *)x, K, (const float2 *)smaps,
                                    coil_idx, B, (const float2 *)V, (const float2 *)d, w, loss,
                                    (float2 *)grad, (hipStream_t)stream);
  p->prof = prof;
  return s;
}

}  // extern "C"

namespace sdn {

// Ragged volumes as one launch per gridding stage: the per-volume passes
// (forward x/y/z, inverse z/y/x) run volume by volume, the interpolation
// and the spreading of all volumes each as one launch over their work
// items.  Returns SDN_E_UNSUPPORTED (nothing enqueued) when the volumes
// cannot share those launches: more than kMaxFusedPlans, different kernel
// widths or spreading engines, an empty plan, or a minibatch that a
// workspace budget would split into coil passes.  The fused stages are
// timed on the first plan's stage events.
namespace {

sdn_status group_prepare(sdn_plan const *plans, int n, const void *const *x, int K,
                         const void *const *smaps, const int *C, const int32_t *const *coil_idx,
                         int B, const void *const *V, const void *const *k_arr, const char *fn,
                         bool need_kbuf, bool need_part) {
  if (n < 1 || n > kMaxFusedPlans) return SDN_E_UNSUPPORTED;
  for (int v = 0; v < n; ++v) {
    SDN_TRY(check_plan(plans[v], fn));
    SDN_TRY(check_mrf_args(*plans[v], fn, x[v], K, smaps[v], C[v], coil_idx[v], B, V[v], k_arr[v]));
  }
  const int engine = spread_engine_for(*plans[0], K, B);
  for (int v = 0; v < n; ++v) {
    const sdn_plan_s &p = *plans[v];
    int per = 0;
    if (p.M == 0 || p.W != plans[0]->W || spread_engine_for(p, K, B) != engine ||
        channels_per_pass(p, K, B, &per, fn) != SDN_OK || per < B)
      return SDN_E_UNSUPPORTED;
  }
  for (int v = 0; v < n; ++v) {
    sdn_plan_s *p = plans[v];
    SDN_TRY(ensure_grid(p, (size_t)B * K * fine_cells(*p)));
    if (need_kbuf) SDN_TRY(ensure_kbuf(p, (size_t)B * p->M));
    if (need_kbuf) SDN_TRY(ensure_lpart(p, B));
    if (need_part) SDN_TRY(ensure_part(p, B, K));
  }
  return SDN_OK;
}

}  // namespace

sdn_status group_dc_grad_fused(sdn_plan const *plans, int n, const void *const *x, int K,
                               const void *const *smaps, const int *C,
                               const int32_t *const *coil_idx, int B, const void *const *V,
                               const void *const *d, const float *const *w, double *losses,
                               void *const *grad, void *stream) {
  SDN_TRY(group_prepare(plans, n, x, K, smaps, C, coil_idx, B, V, d, "sdn_group_mrf_dc_grad",
                        true, true));
  hipStream_t st = (hipStream_t)stream;
  sdn_plan_s *p0 = plans[0];
  InterpArgs ia[kMaxFusedPlans];
  SpreadArgs sa[kMaxFusedPlans];
  const sdn_plan_s *cp[kMaxFusedPlans];
  for (int v = 0; v < n; ++v) {
    sdn_plan_s *p = plans[v];
    cp[v] = p;
    SDN_HIP(launch_fill_zero_f64(losses + v, 1, st), "loss clear");
    SDN_TRY(forward_grid(p, (const float2 *)x[v], K, (const float2 *)smaps[v],
                         coil_list(coil_idx[v], 0, B), B, p->grid, st));
    InterpArgs &a = ia[v];
    a = InterpArgs{};
    a.grid = p->grid;
    a.P = B * K;
    a.groups = B;
    a.kg = K;
    a.V = (const float2 *)V[v];
    a.dc = 1;
    a.rscale = 2.f;
    a.d = (const float2 *)d[v];
    a.w = w ? w[v] : nullptr;
    a.r_plan = p->kbuf;
    a.loss = losses + v;
    a.loss_part = p->lpart;
    a.rmax = p->absmax;
    SpreadArgs &b = sa[v];
    b = SpreadArgs{};
    b.grid = p->grid;
    b.part = p->part;
    b.groups = B;
    b.K = K;
    b.V = (const float2 *)V[v];
    b.src = p->kbuf;
    b.src_plan_order = true;
    b.src_max_ready = true;
  }
  {
    sdn_plan_s *p = p0;
    SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp_fused(cp, ia, n, st), "fused interpolation + residual");
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread_fused(cp, sa, n, st), "fused spreading");
  }
  for (int v = 0; v < n; ++v)
    SDN_TRY(adjoint_grid(plans[v], K, (const float2 *)smaps[v], coil_list(coil_idx[v], 0, B), B,
                         (float2 *)grad[v], 0, plans[v]->grid, st));
  return SDN_OK;
}

sdn_status group_forward_fused(sdn_plan const *plans, int n, const void *const *x, int K,
                               const void *const *smaps, const int *C,
                               const int32_t *const *coil_idx, int B, const void *const *V,
                               void *const *y, void *stream) {
  SDN_TRY(group_prepare(plans, n, x, K, smaps, C, coil_idx, B, V, (const void *const *)y,
                        "sdn_group_mrf_forward", false, false));
  hipStream_t st = (hipStream_t)stream;
  InterpArgs ia[kMaxFusedPlans];
  const sdn_plan_s *cp[kMaxFusedPlans];
  for (int v = 0; v < n; ++v) {
    sdn_plan_s *p = plans[v];
    cp[v] = p;
    SDN_TRY(forward_grid(p, (const float2 *)x[v], K, (const float2 *)smaps[v],
                         coil_list(coil_idx[v], 0, B), B, p->grid, st));
    InterpArgs &a = ia[v];
    a = InterpArgs{};
    a.grid = p->grid;
    a.P = B * K;
    a.groups = B;
    a.kg = K;
    a.V = (const float2 *)V[v];
    a.y = (float2 *)y[v];
  }
  sdn_plan_s *p = plans[0];
  SDN_STAGE(p, SDN_STAGE_INTERP, launch_interp_fused(cp, ia, n, st), "fused interpolation");
  return SDN_OK;
}

sdn_status group_adjoint_fused(sdn_plan const *plans, int n, const void *const *y, int K,
                               const void *const *smaps, const int *C,
                               const int32_t *const *coil_idx, int B, const void *const *V,
                               void *const *x_out, int accumulate, void *stream) {
  SDN_TRY(group_prepare(plans, n, (const void *const *)x_out, K, smaps, C, coil_idx, B, V, y,
                        "sdn_group_mrf_adjoint", false, true));
  hipStream_t st = (hipStream_t)stream;
  SpreadArgs sa[kMaxFusedPlans];
  const sdn_plan_s *cp[kMaxFusedPlans];
  for (int v = 0; v < n; ++v) {
    sdn_plan_s *p = plans[v];
    cp[v] = p;
    SpreadArgs &b = sa[v];
    b = SpreadArgs{};
    b.grid = p->grid;
    b.part = p->part;
    b.groups = B;
    b.K = K;
    b.V = (const float2 *)V[v];
    b.src = (const float2 *)y[v];
    b.src_plan_order = false;
  }
  {
    sdn_plan_s *p = plans[0];
    SDN_STAGE(p, SDN_STAGE_SPREAD, launch_spread_fused(cp, sa, n, st), "fused spreading");
  }
  for (int v = 0; v < n; ++v)
    SDN_TRY(adjoint_grid(plans[v], K, (const float2 *)smaps[v], coil_list(coil_idx[v], 0, B), B,
                         (float2 *)x_out[v], accumulate, plans[v]->grid, st));
  return SDN_OK;
}

}  // namespace sdn
