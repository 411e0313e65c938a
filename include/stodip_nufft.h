/*
 * stodip_nufft.h - C ABI of the MI355X multicoil subspace NUFFT library.
 *
 * The library evaluates the forward operator of MRF reconstruction and its
 * adjoint (StoDIP, arXiv 2408.02367, Sec. 2 and Eq. 1-3):
 *
 *   A_c : x (K subspace images) -> coil c k-space
 *   y_b(j) = sum_k V[t_j, k] * NUFFT2(S_{c_b} * x_k)(k_j)
 *   xbar_k = sum_b conj(S_{c_b}) * NUFFT1(conj(V[t_j, k]) * r_b(j))
 *
 * where the NUFFT is a Kaiser-Bessel gridding NUFFT (width W, oversampling
 * sigma) and t_j is the timeframe of sample j.  The DC loss of Eq. 2-3 and
 * its gradient are sdn_mrf_dc_grad.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns sdn_status (0 = SDN_OK, negative = error); no C++
 *   exception crosses the ABI.  sdn_last_error() gives a message for the
 *   last non-OK status of the calling thread.
 * - "dev" pointers are HIP device pointers owned by the caller; the library
 *   never frees or retains them beyond the call.  Complex arrays are
 *   complex64 (interleaved float re, im) and contiguous.
 * - Images are [..][Nz][Ny][Nx] with x fastest; mode n_d sits at array
 *   index n_d + floor(N_d/2) (centred).  Trajectories are [M][3] float32
 *   radians per voxel with columns (kx, ky, kz) paired with (x, y, z).
 * - The type-2 transform uses exp(-i k.n), the type-1 exp(+i k.n); neither
 *   is normalised, so the adjoint is the exact adjoint.
 * - k-space arrays are in the caller's point order.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *   enqueued asynchronously; only sdn_plan_create synchronises.
 * - One call in flight per plan at a time (the plan owns its workspace).
 */
#ifndef STODIP_NUFFT_H
#define STODIP_NUFFT_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define SDN_API __attribute__((visibility("default")))
#else
#define SDN_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdn_plan_s *sdn_plan;

typedef enum {
  SDN_OK = 0,
  SDN_E_INVALID = -1,     /* bad argument: null pointer, bad size or shape */
  SDN_E_RANGE = -2,       /* non-finite coordinate, index out of range     */
  SDN_E_NOMEM = -3,       /* device allocation failed or budget too small  */
  SDN_E_UNSUPPORTED = -4, /* valid request the library does not implement  */
  SDN_E_HIP = -5,         /* a HIP runtime call or kernel launch failed    */
  SDN_E_STATE = -6        /* plan in the wrong state (e.g. destroyed)      */
} sdn_status;

/* Plan options.  Fill with sdn_default_opts() and override. */
typedef struct {
  int W;                   /* kernel width in fine-grid cells: 4, 6 or 8 (default 6) */
  double sigma;            /* oversampling ratio, 1.25 <= sigma <= 4 (default 2.0)   */
  int tile;                /* tile edge in fine cells, 4..32 on every axis;
                              0 = library choice (16 x 16 x 8)                      */
  int max_points_per_item; /* cap on points per interpolation work item, <= 2048;
                              0 = library choice (2048; a power of two down to
                              512 for plans of under a million points)            */
  size_t workspace_budget; /* bytes of fine-grid workspace; 0 = unlimited.  Calls
                              whose coil minibatch does not fit run coil-chunked.   */
  int spread_engine;       /* type-1 spreading kernel: SDN_SPREAD_AUTO (default:
                              the matrix cores when a call spreads >= 2 coils of
                              >= 2 channels - split by planes from 32 (coil,
                              channel) pairs, by coils below - else the gather),
                              SDN_SPREAD_GATHER (vector ALU gather into
                              registers), SDN_SPREAD_MATRIX (matrix cores, one
                              wave per coil, split fp16 products with FP32
                              accumulation) or SDN_SPREAD_PLANES (matrix cores,
                              waves split by block planes, the value operand
                              built once for all coils and channels).  The
                              matrix engines serve the subspace calls with >= 2
                              channels and every fine axis >= 16, else the
                              gather runs; the plain type-1 call always gathers.  */
  int point_order;         /* order of the points within an interpolation tile:
                              SDN_ORDER_AUTO (default: round-robin over the 32
                              LDS residue classes of their first cell, tiles with
                              at least half as many points as padded cells by
                              first cell) or SDN_ORDER_CELL (every tile by first
                              cell: more interpolation bank conflicts, but the
                              gather spreading of one-coil calls reads its points
                              more coherently; plans with more than 131072
                              populated tiles keep the default order).  Results
                              agree to rounding.                                   */
} sdn_opts;

/* Values of sdn_opts.spread_engine. */
enum { SDN_SPREAD_AUTO = 0, SDN_SPREAD_GATHER = 1, SDN_SPREAD_MATRIX = 2, SDN_SPREAD_PLANES = 3 };

/* Values of sdn_opts.point_order. */
enum { SDN_ORDER_AUTO = 0, SDN_ORDER_CELL = 1 };

/* Plan facts, for callers and tests. */
typedef struct {
  int64_t shape[3];        /* (Nz, Ny, Nx) image shape                               */
  int64_t fine[3];         /* (nfz, nfy, nfx) oversampled grid                       */
  int64_t M;               /* points                                                */
  int32_t T;               /* frames (rows of V)                                    */
  int W;
  double sigma, beta;      /* Kaiser-Bessel shape parameter                          */
  int64_t tile[3];         /* (bz, by, bx) tile edges in fine cells                  */
  int64_t nbins;           /* tiles of the fine grid                                */
  int64_t nwork;           /* interpolation work items (crowded tiles split)        */
  int64_t max_bin;         /* points in the most populated tile                      */
  int ncoef;               /* coefficients per piece of the kernel polynomial        */
  int64_t nvisit;          /* (point, tile) pairs of the spreading lists             */
  int spread_engine;       /* engine a call with >= 2 coils of >= 2 channels
                              uses: SDN_SPREAD_GATHER, _MATRIX or _PLANES; see
                              sdn_spread_engine for a given minibatch              */
} sdn_plan_info;

/* Library defaults: W = 6, sigma = 2, automatic tiles, no budget. */
SDN_API void sdn_default_opts(sdn_opts *opts);

/*
 * Build a plan for one trajectory and image shape (the "plan(traj, N, sigma,
 * W)" call; the trajectory is fixed across all DC steps of a scan, Sec. 3).
 *
 *   shape           host int64[3] = (Nz, Ny, Nx), each >= 1
 *   traj            dev float32 [M][3] radians per voxel; any finite value is
 *                   folded modulo 2 pi; |k| > 2^20 or NaN/Inf -> SDN_E_RANGE
 *   M               points, >= 0 (M = 0 is a valid, empty plan)
 *   frame_of_point  dev int32 [M] timeframe of each point in [0, T), or NULL
 *                   (all points in frame 0; T may then be 0 or 1)
 *   opts            NULL = defaults
 * The plan sorts the points into fine-grid tiles on the device and keeps
 * its own copy of everything it needs; the caller may free traj and
 * frame_of_point afterwards.  Synchronises `stream`.
 */
SDN_API sdn_status sdn_plan_create(sdn_plan *out, const int64_t shape[3], const float *traj,
                           int64_t M, const int32_t *frame_of_point, int32_t T,
                           const sdn_opts *opts, void *stream);

/* Free every device and host resource of the plan.  NULL is a no-op. */
SDN_API sdn_status sdn_plan_destroy(sdn_plan plan);

SDN_API sdn_status sdn_plan_get_info(sdn_plan plan, sdn_plan_info *info);

/* Spreading engine (SDN_SPREAD_GATHER, _MATRIX or _PLANES) that the subspace
 * calls of this plan use for a minibatch of B coils of K channels, into
 * *engine (host int).  SDN_E_INVALID for B or K below 1 or a NULL engine. */
SDN_API sdn_status sdn_spread_engine(sdn_plan plan, int B, int K, int *engine);

/*
 * Plain type-2 NUFFT of `batch` images (uniform -> nonuniform):
 *   ksp[b][j] = sum_n img[b][n] exp(-i k_j . n)
 *   img  dev complex64 [batch][Nz][Ny][Nx];  ksp dev complex64 [batch][M]
 */
SDN_API sdn_status sdn_forward(sdn_plan plan, const void *img, void *ksp, int batch, void *stream);

/*
 * Plain type-1 NUFFT (nonuniform -> uniform), the adjoint of sdn_forward:
 *   img[b][n] = sum_j ksp[b][j] exp(+i k_j . n)
 */
SDN_API sdn_status sdn_adjoint(sdn_plan plan, const void *ksp, void *img, int batch, void *stream);

/*
 * MRF subspace forward operator for a coil minibatch (Sec. 2; Eq. 3's A_c;
 * Algorithm 1's forward step), all B*K (coil, channel) pairs batched:
 *   y[b][j] = sum_k V[t_j][k] * NUFFT2(smaps[coil_idx[b]] * x[k])(k_j)
 *
 *   x        dev complex64 [K][Nz][Ny][Nx], 1 <= K <= 8
 *   smaps    dev complex64 [C][Nz][Ny][Nx] coil sensitivities
 *   coil_idx host int32 [B], each in [0, C), 1 <= B <= 64
 *   V        dev complex64 [T][K] temporal subspace basis (row t_j is used)
 *   y        dev complex64 [B][M] (overwritten)
 */
SDN_API sdn_status sdn_mrf_forward(sdn_plan plan, const void *x, int K, const void *smaps, int C,
                           const int32_t *coil_idx, int B, const void *V, void *y,
                           void *stream);

/*
 * Adjoint of sdn_mrf_forward (the backward of Algorithm 1's loss.backward()):
 *   x_out[k] (+)= sum_b conj(smaps[coil_idx[b]]) * NUFFT1(conj(V[t_j][k]) * y[b][j])
 *   y      dev complex64 [B][M];  x_out dev complex64 [K][Nz][Ny][Nx]
 *   accumulate = 0 overwrites x_out, 1 adds to it.
 */
SDN_API sdn_status sdn_mrf_adjoint(sdn_plan plan, const void *y, int K, const void *smaps, int C,
                           const int32_t *coil_idx, int B, const void *V, void *x_out,
                           int accumulate, void *stream);

/*
 * Data-consistency loss and gradient of Eq. 2-3 for a coil minibatch, fused:
 *   loss = sum_b sum_j w_j |(A x)_b(j) - d[b][j]|^2
 *   grad = 2 A^H (w (A x - d))          (PyTorch's complex gradient convention)
 *   d     dev complex64 [B][M] measured k-space of the minibatch coils
 *   w     dev float32 [M] density-compensation weights, or NULL (w = 1)
 *   loss  dev double [1] (overwritten)
 *   grad  dev complex64 [K][Nz][Ny][Nx] (overwritten)
 */
SDN_API sdn_status sdn_mrf_dc_grad(sdn_plan plan, const void *x, int K, const void *smaps, int C,
                           const int32_t *coil_idx, int B, const void *V, const void *d,
                           const float *w, double *loss, void *grad, void *stream);

/*
 * The DC loss and gradient of sdn_mrf_dc_grad (same arguments, same
 * results), for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no allocating routine.  Its fine grids, residuals and partial sums
 * live in a static device array of SDN_NOALLOC_SCRATCH_BYTES inside the
 * library (one per GPU, held until the process ends), and coils are
 * processed in passes of as many as fit in it (the plan's workspace budget
 * does not apply).  SDN_E_NOMEM when one coil's K grids, its residuals and
 * partial sums exceed it (e.g. K = 5 on a 64^3 fine grid fits; on 320^3 it
 * does not).  Every call on one GPU, for any plan and on any stream, uses
 * that one array and leaves it holding its last contents: calls that
 * overlap on one GPU race, so the caller serialises them.
 */
#define SDN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
SDN_API sdn_status sdn_mrf_dc_grad_noalloc(sdn_plan plan, const void *x, int K, const void *smaps,
                                           int C, const int32_t *coil_idx, int B, const void *V,
                                           const void *d, const float *w, double *loss,
                                           void *grad, void *stream);

/*
 * Ragged volumes: a group of plans of different image shapes, each with its
 * own trajectory (and V), evaluated as one call on one stream (Sec. 3.1
 * evaluates five scanned volumes; each is reconstructed on its own, and the
 * group only shares launches between them).  The interpolation and the
 * spreading each run as one launch over the work items of all volumes; the
 * FFT passes run volume by volume.  Volumes that cannot share those
 * launches (different kernel widths or spreading engines, coil passes under
 * a workspace budget, more than eight volumes) run the member plans' calls
 * in turn.  Either way the results equal those of the member plans called
 * one by one, bit for bit.
 *
 *   sdn_group_create  plans: host array of n >= 1 live plans (not owned: they
 *                     must outlive the group); the group holds n doubles of
 *                     device memory for per-volume losses.
 *   Per-volume arguments are host arrays of length n (x[v], smaps[v], C[v],
 *   coil_idx[v], V[v], y[v], d[v], w[v] (entries may be NULL), grad[v]),
 *   each entry laid out as for the single-plan call on plans[v]; K and B are
 *   common to all volumes.
 *   sdn_group_mrf_dc_grad: loss = dev double [1], the sum of the volumes'
 *   losses (overwritten).
 * Errors: as the single-plan calls; a failing volume stops the call.
 */
typedef struct sdn_group_s *sdn_group;
SDN_API sdn_status sdn_group_create(sdn_group *out, const sdn_plan *plans, int n);
SDN_API sdn_status sdn_group_destroy(sdn_group group);
SDN_API sdn_status sdn_group_mrf_forward(sdn_group group, const void *const *x, int K,
                                         const void *const *smaps, const int *C,
                                         const int32_t *const *coil_idx, int B,
                                         const void *const *V, void *const *y, void *stream);
SDN_API sdn_status sdn_group_mrf_adjoint(sdn_group group, const void *const *y, int K,
                                         const void *const *smaps, const int *C,
                                         const int32_t *const *coil_idx, int B,
                                         const void *const *V, void *const *x_out,
                                         int accumulate, void *stream);
SDN_API sdn_status sdn_group_mrf_dc_grad(sdn_group group, const void *const *x, int K,
                                         const void *const *smaps, const int *C,
                                         const int32_t *const *coil_idx, int B,
                                         const void *const *V, const void *const *d,
                                         const float *const *w, double *loss,
                                         void *const *grad, void *stream);

/*
 * The same operators evaluated the plain way, one (coil, channel) pair per
 * NUFFT with separate subspace-mix kernels: the per-coil/per-channel
 * baseline the batched calls are measured against.  Arguments as above.
 */
SDN_API sdn_status sdn_mrf_forward_plain(sdn_plan plan, const void *x, int K, const void *smaps,
                                 int C, const int32_t *coil_idx, int B, const void *V,
                                 void *y, void *stream);
SDN_API sdn_status sdn_mrf_adjoint_plain(sdn_plan plan, const void *y, int K, const void *smaps,
                                 int C, const int32_t *coil_idx, int B, const void *V,
                                 void *x_out, int accumulate, void *stream);

/*
 * Density compensation weights for Eq. 2 (the paper uses a DCF as the
 * loss's preconditioner, Sec. 2; it does not say how it is computed): the
 * Pipe-Menon fixed-point iteration with the plan's gridding kernel
 * (normalised to 1 at its centre on every axis), w_0 = 1,
 *   w_{n+1} = w_n / (C w_n),  (C w)_j = sum_l phi(s_j - l) sum_i phi(s_i - l) w_i,
 * evaluated as spreading onto the fine grid and interpolating back (no
 * FFT).  w_out: dev float32 [M], user point order (overwritten); 1 <=
 * iterations <= 1000.  Uses the plan's workspace (one fine grid and 2 M
 * complex values).  The weights are the `w` argument of sdn_mrf_dc_grad.
 */
SDN_API sdn_status sdn_dcf_estimate(sdn_plan plan, int iterations, float *w_out, void *stream);

/*
 * Initialisers of the TSMI x^(0) (Sec. 2.2, "Initialisation of x^(0)",
 * starts the network from an estimate of the inverse problem of Eq. 1:
 * the SVD-MRF adjoint with a
 * scaling factor, and low-rank least squares by conjugate gradients, with
 * or without Tikhonov regularisation).  The paper names the three only;
 * the operators here, over the B listed coils with the DCF weight
 * W = diag(w) of Eq. 2 (w NULL: 1):
 *
 *   normal operator  N x = sum_b A_b^H W A_b x + lambda x
 *   data term        b   = sum_b A_b^H W y_b
 *
 * Arguments as for sdn_mrf_dc_grad; y: dev complex64 [B][M] user order,
 * row b the samples of coil coil_idx[b] (all C coils for a full solve);
 * lambda >= 0 and finite.  Image vectors are dev complex64 [K][Nz][Ny][Nx].
 * Coils go through the stages in chunks that fit the workspace budget.
 *
 * sdn_mrf_normal:  out = N x (overwritten).
 * sdn_mrf_cg:      x holds the start point on entry and the result after
 *                  `iterations` (0 .. 100000) conjugate-gradient steps on
 *                  N x = b (Hestenes-Stiefel).  history: dev double
 *                  [iterations + 1] or NULL; entry i is |b - N x_i|^2.
 *                  Every scalar of the iteration is formed on the device
 *                  (FP64 sums in a fixed order), so the whole solve is
 *                  enqueued without a host round trip.  A zero curvature
 *                  or residual gives a zero step (the iteration stalls
 *                  instead of producing NaN).  Uses 3 image vectors of
 *                  plan workspace beside the grids.
 * sdn_mrf_scaled_adjoint: x_out = s z with z = b and the least-squares
 *                  scale s = |z|^2 / sum_b <A_b z, W A_b z> (0 if the
 *                  denominator is 0); scale: dev double [1] receiving s,
 *                  or NULL.
 * Errors: as sdn_mrf_dc_grad; SDN_E_INVALID for a negative or non-finite
 * lambda or an iteration count outside the range.
 */
SDN_API sdn_status sdn_mrf_normal(sdn_plan plan, const void *x, int K, const void *smaps, int C,
                                  const int32_t *coil_idx, int B, const void *V, const float *w,
                                  float lambda, void *out, void *stream);
SDN_API sdn_status sdn_mrf_cg(sdn_plan plan, const void *y, int K, const void *smaps, int C,
                              const int32_t *coil_idx, int B, const void *V, const float *w,
                              float lambda, int iterations, void *x, double *history,
                              void *stream);
SDN_API sdn_status sdn_mrf_scaled_adjoint(sdn_plan plan, const void *y, int K, const void *smaps,
                                          int C, const int32_t *coil_idx, int B, const void *V,
                                          const float *w, void *x_out, double *scale,
                                          void *stream);

/*
 * Total-variation penalty of Alg. 1 (the StoDIP + TV variant adds lambda
 * TV(x_hat) to the per-coil loss; Sec. 2.2 does not define the TV form).
 * The form computed: isotropic over the three spatial axes, per channel,
 * forward differences that are zero at the last index of an axis, and a
 * smoothing eps > 0:
 *   TV(x) = sum_k sum_n sqrt(|D_x x_k[n]|^2 + |D_y x_k[n]|^2 + |D_z x_k[n]|^2 + eps^2)
 * on the plan's image shape.
 *   x      dev complex64 [K][Nz][Ny][Nx]
 *   value  dev double [1] receiving lambda TV(x) (FP64 sum in a fixed
 *          order), or NULL
 *   grad   dev complex64 [K][Nz][Ny][Nx] receiving lambda dTV/dRe x +
 *          i lambda dTV/dIm x (added to its contents when accumulate is
 *          non-zero, so it can follow sdn_mrf_dc_grad), or NULL
 * One fused stencil pass; uses plan scratch of one double per 256 voxels.
 * Errors: SDN_E_INVALID for a null x, both outputs NULL, K outside [1, 8],
 * eps not finite and > 0, or lambda negative or not finite.
 */
SDN_API sdn_status sdn_tv_grad(sdn_plan plan, const void *x, int K, float eps, float lambda,
                               double *value, void *grad, int accumulate, void *stream);

/*
 * Autotuner: builds candidate plans for one trajectory (interpolation tile
 * edge 16x16x8 / 8 / 16, up to 2048 or 1024 points per work item, gather or
 * matrix-core spreading, the gather also with every tile in cell order, all
 * other options from `base`), times three
 * synthetic DC-gradient steps (coil minibatch B, K channels) of each on
 * `stream`, and returns the fastest option set in *best and its time per
 * step (ms) in *best_ms (may be NULL).  Arguments as sdn_plan_create; the
 * tuner allocates its own synthetic inputs and frees everything before
 * returning.  Candidates the device cannot run are skipped; SDN_E_UNSUPPORTED
 * if none ran.  Synchronises `stream`.
 */
SDN_API sdn_status sdn_autotune(const int64_t shape[3], const float *traj, int64_t M,
                                const int32_t *frame_of_point, int32_t T, int B, int K,
                                const sdn_opts *base, sdn_opts *best, double *best_ms,
                                void *stream);

/* Device workspace (bytes) a call with B coils and K channels would hold:
 * the fine grids of one pass (all B coils, or the coil chunk the budget
 * allows), the k-space residual of those coils and the partial blocks of
 * split spreading items. */
SDN_API sdn_status sdn_workspace_size(sdn_plan plan, int B, int K, size_t *bytes);

/* Release the plan's cached workspace (it is re-allocated on demand). */
SDN_API sdn_status sdn_release_workspace(sdn_plan plan);

/* Stages of the operator, for per-stage timing. */
typedef enum {
  SDN_STAGE_PRE_FFTX = 0,   /* coil multiply + deapodise + pad + x FFT     */
  SDN_STAGE_FFT_Y = 1,      /* forward y FFT pass                          */
  SDN_STAGE_FFT_Z = 2,      /* forward z FFT pass                          */
  SDN_STAGE_INTERP = 3,     /* interpolation + subspace mix (+ residual)   */
  SDN_STAGE_CLEAR = 4,      /* fine-grid clear before spreading            */
  SDN_STAGE_SPREAD = 5,     /* spreading with the conjugate subspace mix   */
  SDN_STAGE_IFFT_Z = 6,     /* adjoint z FFT pass                          */
  SDN_STAGE_IFFT_Y = 7,     /* adjoint y FFT pass                          */
  SDN_STAGE_POST_IFFTX = 8, /* x IFFT + crop + deapodise + conj coil sum   */
  SDN_STAGE_MIX = 9,        /* separate subspace-mix kernels (plain path)  */
  SDN_NUM_STAGES = 10
} sdn_stage;

/*
 * Per-stage timing with HIP events recorded on the caller's stream around
 * every kernel launch of the plan while enabled.  sdn_profile_read waits for
 * the recorded events and returns, per stage, the summed kernel time in ms
 * and the number of launches since the last reset.
 */
SDN_API sdn_status sdn_profile_enable(sdn_plan plan, int enable);
SDN_API sdn_status sdn_profile_read(sdn_plan plan, double *ms, int64_t *launches, int reset);

/*
 * Host-only view of the kernel tables a plan would use (no device work):
 * the shape parameter beta, the fine length of an axis of N modes, the
 * piecewise-polynomial kernel (coef[i * 16 + d] is the z^d coefficient of
 * node i, z = 2t - 1, normalised so the kernel peak is 1) and the
 * deapodisation factors 1 / phi_hat(n / nf) on the same normalisation for
 * array index n + floor(N/2).  coef: host float[8 * 16]; deapod_inv: host
 * float[N] or NULL.  For tests and diagnostics.
 */
SDN_API sdn_status sdn_kernel_tables(int W, double sigma, int64_t N, double *beta, int *nf,
                                     int *ncoef, float *coef, float *deapod_inv);

/* Message for the calling thread's last non-OK status ("" if none). */
SDN_API const char *sdn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STODIP_NUFFT_H */
