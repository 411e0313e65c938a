"""MI355X multicoil subspace NUFFT: the data-consistency hot path of StoDIP.

Python binding of ``libstodip_nufft.so`` (C ABI in ``include/stodip_nufft.h``).
This module only marshals arguments: every step of the operator runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.  If the
library is not built, every call raises; there is no fallback.

The operator (StoDIP, arXiv 2408.02367, Sec. 2 and Eq. 1-3):

    y_b(j) = sum_k V[t_j, k] * NUFFT2(S_{c_b} * x_k)(k_j)            A_c
    xbar_k = sum_b conj(S_{c_b}) * NUFFT1(conj(V[t_j, k]) * y_b(j))  A_c^H

``MRFForward`` wraps A_c as a ``torch.autograd.Function`` whose backward is
the hand-written adjoint (Algorithm 1's ``loss.backward()``), so a DIP loop
differentiates through the NUFFT without autograd tracing it.
"""

import ctypes
import os

import numpy as np
import torch  # imported before the library so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstodip_nufft.so")

SDN_OK = 0
_STATUS = {0: "SDN_OK", -1: "SDN_E_INVALID", -2: "SDN_E_RANGE", -3: "SDN_E_NOMEM",
           -4: "SDN_E_UNSUPPORTED", -5: "SDN_E_HIP", -6: "SDN_E_STATE"}

# every symbol the header declares
API = ["sdn_default_opts", "sdn_plan_create", "sdn_plan_destroy", "sdn_plan_get_info",
       "sdn_forward", "sdn_adjoint", "sdn_mrf_forward", "sdn_mrf_adjoint", "sdn_mrf_dc_grad",
       "sdn_mrf_forward_plain", "sdn_mrf_adjoint_plain", "sdn_workspace_size",
       "sdn_release_workspace", "sdn_profile_enable", "sdn_profile_read",
       "sdn_kernel_tables", "sdn_last_error", "sdn_group_create", "sdn_group_destroy",
       "sdn_group_mrf_forward", "sdn_group_mrf_adjoint", "sdn_group_mrf_dc_grad",
       "sdn_autotune", "sdn_dcf_estimate", "sdn_mrf_normal", "sdn_mrf_cg",
       "sdn_mrf_scaled_adjoint", "sdn_tv_grad", "sdn_mrf_dc_grad_noalloc",
       "sdn_spread_engine"]

# stage names, in the order of the sdn_stage enum
STAGES = ["pre_fftx", "fft_y", "fft_z", "interp", "clear", "spread", "ifft_z", "ifft_y",
          "post_ifftx", "mix"]


class SdnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int), ("sigma", ctypes.c_double), ("tile", ctypes.c_int),
                ("max_points_per_item", ctypes.c_int), ("workspace_budget", ctypes.c_size_t),
                ("spread_engine", ctypes.c_int), ("point_order", ctypes.c_int)]


SPREAD_ENGINES = {"auto": 0, "gather": 1, "matrix": 2, "planes": 3}
POINT_ORDERS = {"auto": 0, "cell": 1}
_ENGINE_NAMES = {1: "gather", 2: "matrix", 3: "planes"}


class PlanInfo(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int64 * 3), ("fine", ctypes.c_int64 * 3),
                ("M", ctypes.c_int64), ("T", ctypes.c_int32), ("W", ctypes.c_int),
                ("sigma", ctypes.c_double), ("beta", ctypes.c_double),
                ("tile", ctypes.c_int64 * 3), ("nbins", ctypes.c_int64),
                ("nwork", ctypes.c_int64), ("max_bin", ctypes.c_int64), ("ncoef", ctypes.c_int),
                ("nvisit", ctypes.c_int64), ("spread_engine", ctypes.c_int)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2408_02367_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.sdn_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.sdn_default_opts.restype = None
        L.sdn_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), vp, i64, vp,
                                      ctypes.c_int32, ctypes.POINTER(Opts), vp]
        L.sdn_plan_destroy.argtypes = [vp]
        L.sdn_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.sdn_spread_engine.argtypes = [vp, i32, i32, ctypes.POINTER(i32)]
        L.sdn_forward.argtypes = [vp, vp, vp, i32, vp]
        L.sdn_adjoint.argtypes = [vp, vp, vp, i32, vp]
        mrf = [vp, vp, i32, vp, i32, ctypes.POINTER(ctypes.c_int32), i32, vp, vp]
        L.sdn_mrf_forward.argtypes = mrf + [vp]
        L.sdn_mrf_forward_plain.argtypes = mrf + [vp]
        L.sdn_mrf_adjoint.argtypes = mrf + [i32, vp]
        L.sdn_mrf_adjoint_plain.argtypes = mrf + [i32, vp]
        L.sdn_mrf_dc_grad.argtypes = mrf + [vp, vp, vp, vp]
        L.sdn_mrf_dc_grad_noalloc.argtypes = mrf + [vp, vp, vp, vp]
        L.sdn_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.sdn_release_workspace.argtypes = [vp]
        L.sdn_profile_enable.argtypes = [vp, i32]
        L.sdn_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32]
        L.sdn_kernel_tables.argtypes = [i32, ctypes.c_double, i64, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float)]
        arr = ctypes.POINTER(vp)
        gm = [vp, arr, i32, arr, ctypes.POINTER(i32), arr, i32, arr]
        L.sdn_group_create.argtypes = [ctypes.POINTER(vp), arr, i32]
        L.sdn_group_destroy.argtypes = [vp]
        L.sdn_group_mrf_forward.argtypes = gm + [arr, vp]
        L.sdn_group_mrf_adjoint.argtypes = gm + [arr, i32, vp]
        L.sdn_group_mrf_dc_grad.argtypes = gm + [arr, arr, vp, arr, vp]
        L.sdn_autotune.argtypes = [ctypes.POINTER(i64), vp, i64, vp, ctypes.c_int32, i32, i32,
                                   ctypes.POINTER(Opts), ctypes.POINTER(Opts),
                                   ctypes.POINTER(ctypes.c_double), vp]
        L.sdn_dcf_estimate.argtypes = [vp, i32, vp, vp]
        f32 = ctypes.c_float
        L.sdn_mrf_normal.argtypes = [vp, vp, i32, vp, i32, ctypes.POINTER(ctypes.c_int32), i32, vp,
                                     vp, f32, vp, vp]
        L.sdn_mrf_cg.argtypes = [vp, vp, i32, vp, i32, ctypes.POINTER(ctypes.c_int32), i32, vp, vp,
                                 f32, i32, vp, vp, vp]
        L.sdn_mrf_scaled_adjoint.argtypes = [vp, vp, i32, vp, i32, ctypes.POINTER(ctypes.c_int32),
                                             i32, vp, vp, vp, vp, vp]
        L.sdn_tv_grad.argtypes = [vp, vp, i32, f32, f32, vp, vp, i32, vp]
        L.sdn_last_error.argtypes = []
        L.sdn_last_error.restype = ctypes.c_char_p
        for name in API:
            if name not in ("sdn_default_opts", "sdn_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status):
    if status != SDN_OK:
        raise SdnError(status, lib().sdn_last_error().decode())


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _coils(coil_idx):
    a = np.ascontiguousarray(np.asarray(
        coil_idx.cpu() if isinstance(coil_idx, torch.Tensor) else coil_idx, dtype=np.int32).ravel())
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def kernel_tables(W=6, sigma=2.0, N=32):
    """Host-side kernel tables of the library (no GPU needed)."""
    beta, nf, nc = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
    coef = (ctypes.c_float * (8 * 16))()
    dinv = (ctypes.c_float * int(N))()
    _check(lib().sdn_kernel_tables(int(W), float(sigma), int(N), ctypes.byref(beta),
                                   ctypes.byref(nf), ctypes.byref(nc), coef, dinv))
    return dict(beta=beta.value, nf=nf.value, ncoef=nc.value,
                coef=np.frombuffer(coef, dtype=np.float32).reshape(8, 16).copy(),
                deapod_inv=np.frombuffer(dinv, dtype=np.float32).copy())


class Plan:
    """A trajectory sorted onto the fine grid of one image shape.

    ``traj``: [M, 3] float32 (kx, ky, kz) radians/voxel on the GPU;
    ``shape``: (Nz, Ny, Nx); ``frame_of_point``: [M] int32 in [0, T) or None.
    """

    def __init__(self, traj, shape, sigma=2.0, W=6, frame_of_point=None, T=None, tile=0,
                 max_points_per_item=0, workspace_budget=0, spread_engine="auto",
                 point_order="auto"):
        L = lib()
        self._h = ctypes.c_void_p()
        traj = torch.as_tensor(traj)
        dev = traj.device if traj.is_cuda else torch.device("cuda", torch.cuda.current_device())
        traj = traj.to(dev, torch.float32).contiguous()
        if traj.ndim != 2 or traj.shape[1] != 3:
            raise ValueError("traj must be [M, 3]")
        self.device = dev
        self.shape = tuple(int(s) for s in shape)
        self.M = int(traj.shape[0])
        fptr = None
        if frame_of_point is not None:
            frame_of_point = torch.as_tensor(frame_of_point).to(dev, torch.int32).contiguous()
            if T is None:
                T = int(frame_of_point.max().item()) + 1 if self.M else 1
            fptr = ctypes.c_void_p(frame_of_point.data_ptr())
        self.T = int(T) if T is not None else 1
        o = Opts()
        L.sdn_default_opts(ctypes.byref(o))
        o.W, o.sigma, o.tile = int(W), float(sigma), int(tile)
        o.max_points_per_item, o.workspace_budget = int(max_points_per_item), int(workspace_budget)
        o.spread_engine = SPREAD_ENGINES[spread_engine]
        o.point_order = POINT_ORDERS[point_order]
        sh = (ctypes.c_int64 * 3)(*self.shape)
        with torch.cuda.device(dev):
            _check(L.sdn_plan_create(ctypes.byref(self._h), sh,
                                     ctypes.c_void_p(traj.data_ptr()) if self.M else None,
                                     self.M, fptr, self.T, ctypes.byref(o), _stream(traj)))

    @property
    def handle(self):
        if not self._h:
            raise SdnError(-6, "plan destroyed")
        return self._h

    def info(self):
        i = PlanInfo()
        _check(lib().sdn_plan_get_info(self.handle, ctypes.byref(i)))
        return dict(shape=tuple(i.shape), fine=tuple(i.fine), M=i.M, T=i.T, W=i.W,
                    sigma=i.sigma, beta=i.beta, tile=tuple(i.tile), nbins=i.nbins,
                    nwork=i.nwork, max_bin=i.max_bin, ncoef=i.ncoef, nvisit=i.nvisit,
                    spread_engine=_ENGINE_NAMES.get(i.spread_engine, "gather"))

    def spread_engine(self, B, K):
        """Spreading engine of the subspace calls for B coils of K channels."""
        e = ctypes.c_int()
        _check(lib().sdn_spread_engine(self.handle, int(B), int(K), ctypes.byref(e)))
        return _ENGINE_NAMES[e.value]

    def workspace_size(self, B, K):
        n = ctypes.c_size_t()
        _check(lib().sdn_workspace_size(self.handle, int(B), int(K), ctypes.byref(n)))
        return n.value

    def profile(self, enable=True):
        """Record HIP events around every kernel launch of this plan."""
        _check(lib().sdn_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self, reset=True):
        """{stage: (summed kernel ms, launches)} since the last reset."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        _check(lib().sdn_profile_read(self.handle, ms, n, 1 if reset else 0))
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES) if n[i]}

    def release_workspace(self):
        _check(lib().sdn_release_workspace(self.handle))

    def close(self):
        if self._h:
            _check(lib().sdn_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- plain type 2 / type 1 ------------------------------------------
    def forward(self, img, out=None):
        """ksp[b, j] = sum_n img[b, n] exp(-i k_j.n); img [batch, Nz, Ny, Nx]."""
        batch = img.shape[0] if img.ndim == 4 else 1
        if tuple(img.shape[-3:]) != self.shape:
            raise ValueError("image shape mismatch")
        if out is None:
            out = torch.empty(batch, self.M, dtype=torch.complex64, device=img.device)
        _check(lib().sdn_forward(self.handle, _dev(img, torch.complex64, "img"),
                                 _dev(out, torch.complex64, "ksp"), batch, _stream(img)))
        return out

    def adjoint(self, ksp, out=None):
        """img[b, n] = sum_j ksp[b, j] exp(+i k_j.n); ksp [batch, M]."""
        batch = ksp.shape[0] if ksp.ndim == 2 else 1
        if ksp.shape[-1] != self.M:
            raise ValueError("k-space length mismatch")
        if out is None:
            out = torch.empty((batch,) + self.shape, dtype=torch.complex64, device=ksp.device)
        _check(lib().sdn_adjoint(self.handle, _dev(ksp, torch.complex64, "ksp"),
                                 _dev(out, torch.complex64, "img"), batch, _stream(ksp)))
        return out


def _mrf_common(plan, x_like_K, smaps, coil_idx, V):
    if smaps.ndim != 4 or tuple(smaps.shape[1:]) != plan.shape:
        raise ValueError("smaps must be [C, Nz, Ny, Nx]")
    ci, cptr = _coils(coil_idx)
    if V.ndim != 2 or V.shape[1] != x_like_K or V.shape[0] < plan.T:
        raise ValueError("V must be [T, K]")
    return ci, cptr


def mrf_forward(plan, x, smaps, coil_idx, V, out=None, plain=False):
    """y[b, j] = sum_k V[t_j, k] NUFFT2(smaps[coil_idx[b]] x[k])(k_j)."""
    K = x.shape[0]
    ci, cptr = _mrf_common(plan, K, smaps, coil_idx, V)
    if out is None:
        out = torch.empty(len(ci), plan.M, dtype=torch.complex64, device=x.device)
    fn = lib().sdn_mrf_forward_plain if plain else lib().sdn_mrf_forward
    _check(fn(plan.handle, _dev(x, torch.complex64, "x"), K,
              _dev(smaps, torch.complex64, "smaps"), smaps.shape[0], cptr, len(ci),
              _dev(V, torch.complex64, "V"), _dev(out, torch.complex64, "y"), _stream(x)))
    return out


def mrf_adjoint(plan, y, smaps, coil_idx, V, out=None, accumulate=False, plain=False):
    """x[k] (+)= sum_b conj(smaps[coil_idx[b]]) NUFFT1(conj(V[t_j, k]) y[b, j])."""
    K = V.shape[1]
    ci, cptr = _mrf_common(plan, K, smaps, coil_idx, V)
    if y.shape != (len(ci), plan.M):
        raise ValueError("y must be [B, M]")
    if out is None:
        out = torch.empty((K,) + plan.shape, dtype=torch.complex64, device=y.device)
        accumulate = False
    fn = lib().sdn_mrf_adjoint_plain if plain else lib().sdn_mrf_adjoint
    _check(fn(plan.handle, _dev(y, torch.complex64, "y"), K,
              _dev(smaps, torch.complex64, "smaps"), smaps.shape[0], cptr, len(ci),
              _dev(V, torch.complex64, "V"), _dev(out, torch.complex64, "x_out"),
              1 if accumulate else 0, _stream(y)))
    return out


def mrf_dc_grad(plan, x, smaps, coil_idx, V, d, w=None, grad=None, loss=None):
    """(loss, grad): loss = sum w |A x - d|^2 (float64 [1]), grad = 2 A^H w (A x - d)."""
    K = x.shape[0]
    ci, cptr = _mrf_common(plan, K, smaps, coil_idx, V)
    if d.shape != (len(ci), plan.M):
        raise ValueError("d must be [B, M]")
    if grad is None:
        grad = torch.empty_like(x)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=x.device)
    wptr = _dev(w, torch.float32, "w") if w is not None else None
    _check(lib().sdn_mrf_dc_grad(plan.handle, _dev(x, torch.complex64, "x"), K,
                                 _dev(smaps, torch.complex64, "smaps"), smaps.shape[0], cptr,
                                 len(ci), _dev(V, torch.complex64, "V"),
                                 _dev(d, torch.complex64, "d"), wptr,
                                 _dev(loss, torch.float64, "loss"),
                                 _dev(grad, torch.complex64, "grad"), _stream(x)))
    return loss, grad


def dcf_estimate(plan, iterations=10, out=None):
    """Pipe-Menon density compensation weights [M] (float32, user order)."""
    if out is None:
        out = torch.empty(plan.M, dtype=torch.float32, device=plan.device)
    _check(lib().sdn_dcf_estimate(plan.handle, int(iterations),
                                  _dev(out, torch.float32, "w") if plan.M else None, _stream(out)))
    return out


def _all_coils(smaps, coil_idx):
    return list(range(smaps.shape[0])) if coil_idx is None else coil_idx


def mrf_normal(plan, x, smaps, V, coil_idx=None, w=None, lam=0.0, out=None):
    """sum_b A_b^H W A_b x + lam x over the listed coils (default: all)."""
    K = x.shape[0]
    ci, cptr = _mrf_common(plan, K, smaps, _all_coils(smaps, coil_idx), V)
    if out is None:
        out = torch.empty_like(x)
    wptr = _dev(w, torch.float32, "w") if w is not None else None
    _check(lib().sdn_mrf_normal(plan.handle, _dev(x, torch.complex64, "x"), K,
                                _dev(smaps, torch.complex64, "smaps"), smaps.shape[0], cptr,
                                len(ci), _dev(V, torch.complex64, "V"), wptr, float(lam),
                                _dev(out, torch.complex64, "out"), _stream(x)))
    return out


def mrf_cg(plan, y, smaps, V, x0=None, iterations=10, coil_idx=None, w=None, lam=0.0, K=None):
    """(x, history): conjugate gradients on (sum_b A_b^H W A_b + lam) x =
    sum_b A_b^H W y_b from x0 (default 0); history[i] = |b - N x_i|^2."""
    if x0 is None:
        if K is None:
            K = V.shape[1]
        x = torch.zeros((K,) + plan.shape, dtype=torch.complex64, device=y.device)
    else:
        x = x0.clone()
    K = x.shape[0]
    ci, cptr = _mrf_common(plan, K, smaps, _all_coils(smaps, coil_idx), V)
    if y.shape != (len(ci), plan.M):
        raise ValueError("y must be [B, M]")
    hist = torch.empty(int(iterations) + 1, dtype=torch.float64, device=x.device)
    wptr = _dev(w, torch.float32, "w") if w is not None else None
    _check(lib().sdn_mrf_cg(plan.handle, _dev(y, torch.complex64, "y"), K,
                            _dev(smaps, torch.complex64, "smaps"), smaps.shape[0], cptr, len(ci),
                            _dev(V, torch.complex64, "V"), wptr, float(lam), int(iterations),
                            _dev(x, torch.complex64, "x"), _dev(hist, torch.float64, "history"),
                            _stream(x)))
    return x, hist


def mrf_scaled_adjoint(plan, y, smaps, V, coil_idx=None, w=None, out=None):
    """(s z, s) with z = sum_b A_b^H W y_b and the least-squares scale s."""
    K = V.shape[1]
    ci, cptr = _mrf_common(plan, K, smaps, _all_coils(smaps, coil_idx), V)
    if y.shape != (len(ci), plan.M):
        raise ValueError("y must be [B, M]")
    if out is None:
        out = torch.empty((K,) + plan.shape, dtype=torch.complex64, device=y.device)
    s = torch.empty(1, dtype=torch.float64, device=y.device)
    wptr = _dev(w, torch.float32, "w") if w is not None else None
    _check(lib().sdn_mrf_scaled_adjoint(plan.handle, _dev(y, torch.complex64, "y"), K,
                                        _dev(smaps, torch.complex64, "smaps"), smaps.shape[0],
                                        cptr, len(ci), _dev(V, torch.complex64, "V"), wptr,
                                        _dev(out, torch.complex64, "x"),
                                        _dev(s, torch.float64, "scale"), _stream(y)))
    return out, s


def tv_grad(plan, x, eps, lam=1.0, grad=None, accumulate=False, value=None, want_grad=True):
    """(value, grad): lam TV(x) (float64 [1]) and lam dTV/dx (added to ``grad``
    when accumulate) for the smoothed isotropic TV on the plan's image shape."""
    if x.ndim != 4 or tuple(x.shape[1:]) != plan.shape:
        raise ValueError("x must be [K, Nz, Ny, Nx]")
    if value is None:
        value = torch.empty(1, dtype=torch.float64, device=x.device)
    if want_grad and grad is None:
        grad = torch.zeros_like(x) if accumulate else torch.empty_like(x)
    _check(lib().sdn_tv_grad(plan.handle, _dev(x, torch.complex64, "x"), x.shape[0], float(eps),
                             float(lam), _dev(value, torch.float64, "value"),
                             _dev(grad, torch.complex64, "grad") if want_grad else None,
                             1 if accumulate else 0, _stream(x)))
    return value, grad


TUNED_KEYS = ("tile", "max_points_per_item", "spread_engine", "point_order")


def tune_key(traj, shape, B, K, W=6, sigma=2.0, frame_of_point=None, device_name=""):
    """Cache key of an autotuning result: image shape, minibatch, kernel and
    a hash of the trajectory (and frames) as the library sees them."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(torch.as_tensor(traj).detach().cpu().numpy(),
                                  dtype=np.float32).tobytes())
    if frame_of_point is not None:
        h.update(np.ascontiguousarray(torch.as_tensor(frame_of_point).detach().cpu().numpy(),
                                      dtype=np.int32).tobytes())
    return (f"{device_name}|shape={tuple(int(s) for s in shape)}|B={int(B)}|K={int(K)}|W={int(W)}"
            f"|sigma={float(sigma)}|traj={h.hexdigest()[:32]}")


def autotune(traj, shape, B, K, frame_of_point=None, T=None, W=6, sigma=2.0, cache=None,
             workspace_budget=0):
    """Plan options that make a DC step fastest for this trajectory.

    Returns a dict of Plan keyword arguments (tile, max_points_per_item,
    spread_engine, point_order) plus ``ms`` (time per synthetic step).  With ``cache``
    (a JSON file path) a result for the same key is reused and new results
    are stored.
    """
    import json
    traj = torch.as_tensor(traj)
    dev = traj.device if traj.is_cuda else torch.device("cuda", torch.cuda.current_device())
    key = tune_key(traj, shape, B, K, W, sigma, frame_of_point,
                   torch.cuda.get_device_name(dev))
    table = {}
    if cache is not None and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return dict(table[key])
    traj = traj.to(dev, torch.float32).contiguous()
    M = int(traj.shape[0])
    fptr = None
    if frame_of_point is not None:
        frame_of_point = torch.as_tensor(frame_of_point).to(dev, torch.int32).contiguous()
        if T is None:
            T = int(frame_of_point.max().item()) + 1 if M else 1
        fptr = ctypes.c_void_p(frame_of_point.data_ptr())
    base, best = Opts(), Opts()
    lib().sdn_default_opts(ctypes.byref(base))
    base.W, base.sigma, base.workspace_budget = int(W), float(sigma), int(workspace_budget)
    ms = ctypes.c_double()
    sh = (ctypes.c_int64 * 3)(*[int(s) for s in shape])
    with torch.cuda.device(dev):
        _check(lib().sdn_autotune(sh, ctypes.c_void_p(traj.data_ptr()) if M else None, M, fptr,
                                  int(T) if T is not None else 1, int(B), int(K),
                                  ctypes.byref(base), ctypes.byref(best), ctypes.byref(ms),
                                  _stream(traj)))
    engines = {v: k for k, v in SPREAD_ENGINES.items()}
    orders = {v: k for k, v in POINT_ORDERS.items()}
    out = {"tile": best.tile, "max_points_per_item": best.max_points_per_item,
           "spread_engine": engines[best.spread_engine], "point_order": orders[best.point_order],
           "ms": ms.value}
    if cache is not None:
        table[key] = out
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


class PlanGroup:
    """Ragged volumes: several plans (own shapes, trajectories and V)
    evaluated by one call; per-volume arguments are lists in plan order."""

    def __init__(self, plans):
        self.plans = list(plans)
        self._h = ctypes.c_void_p()
        hs = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        _check(lib().sdn_group_create(ctypes.byref(self._h), hs, len(self.plans)))

    def close(self):
        if self._h:
            _check(lib().sdn_group_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _common(self, K, smaps, coil_idx, V):
        n = len(self.plans)
        if not (len(smaps) == len(coil_idx) == len(V) == n):
            raise ValueError("one smaps, coil_idx and V per volume")
        cis = [_mrf_common(p, K, s, c, v)[0] for p, s, c, v in zip(self.plans, smaps, coil_idx, V)]
        B = len(cis[0])
        if any(len(c) != B for c in cis):
            raise ValueError("every volume takes the same number of coils")
        keep = cis
        cptrs = (ctypes.c_void_p * n)(*[c.ctypes.data for c in cis])
        Cs = (ctypes.c_int * n)(*[s.shape[0] for s in smaps])
        sp = (ctypes.c_void_p * n)(*[_dev(s, torch.complex64, "smaps").value for s in smaps])
        vp = (ctypes.c_void_p * n)(*[_dev(v, torch.complex64, "V").value for v in V])
        return B, keep, cptrs, Cs, sp, vp

    def _ptrs(self, ts, name):
        if len(ts) != len(self.plans):
            raise ValueError(f"{name}: one tensor per volume ({len(self.plans)})")
        return (ctypes.c_void_p * len(ts))(*[_dev(t, torch.complex64, name).value for t in ts])

    def mrf_forward(self, x, smaps, coil_idx, V):
        if len(x) != len(self.plans):
            raise ValueError(f"x: one tensor per volume ({len(self.plans)})")
        K = x[0].shape[0]
        B, keep, cptrs, Cs, sp, vp = self._common(K, smaps, coil_idx, V)
        ys = [torch.empty(B, p.M, dtype=torch.complex64, device=x[0].device) for p in self.plans]
        _check(lib().sdn_group_mrf_forward(self._h, self._ptrs(x, "x"), K, sp, Cs, cptrs, B, vp,
                                           self._ptrs(ys, "y"), _stream(x[0])))
        return ys

    def mrf_adjoint(self, y, smaps, coil_idx, V):
        if len(y) != len(self.plans):
            raise ValueError(f"y: one tensor per volume ({len(self.plans)})")
        K = V[0].shape[1]
        B, keep, cptrs, Cs, sp, vp = self._common(K, smaps, coil_idx, V)
        xs = [torch.empty((K,) + p.shape, dtype=torch.complex64, device=y[0].device)
              for p in self.plans]
        _check(lib().sdn_group_mrf_adjoint(self._h, self._ptrs(y, "y"), K, sp, Cs, cptrs, B, vp,
                                           self._ptrs(xs, "x_out"), 0, _stream(y[0])))
        return xs

    def mrf_dc_grad(self, x, smaps, coil_idx, V, d):
        """(loss summed over volumes, per-volume gradients)."""
        if len(x) != len(self.plans):
            raise ValueError(f"x: one tensor per volume ({len(self.plans)})")
        K = x[0].shape[0]
        B, keep, cptrs, Cs, sp, vp = self._common(K, smaps, coil_idx, V)
        grads = [torch.empty_like(t) for t in x]
        loss = torch.empty(1, dtype=torch.float64, device=x[0].device)
        _check(lib().sdn_group_mrf_dc_grad(self._h, self._ptrs(x, "x"), K, sp, Cs, cptrs, B, vp,
                                           self._ptrs(d, "d"), None,
                                           _dev(loss, torch.float64, "loss"),
                                           self._ptrs(grads, "grad"), _stream(x[0])))
        return loss, grads


class MRFForward(torch.autograd.Function):
    """y = A_c x with backward A_c^H gy (the hand-written adjoint).

    PyTorch's complex gradient convention (dL/dRe + i dL/dIm) makes the
    gradient of a C-linear map the adjoint applied to the output gradient,
    so for L = ||A x - d||^2 autograd yields 2 A^H (A x - d).  Nothing of
    the forward (no fine grid) is saved: A is linear.
    """

    @staticmethod
    def forward(ctx, x, plan, smaps, coil_idx, V):
        ctx.plan, ctx.smaps, ctx.coil_idx, ctx.V = plan, smaps, coil_idx, V
        return mrf_forward(plan, x.contiguous(), smaps, coil_idx, V)

    @staticmethod
    def backward(ctx, gy):
        gx = mrf_adjoint(ctx.plan, gy.contiguous(), ctx.smaps, ctx.coil_idx, ctx.V)
        return gx, None, None, None, None


def mrf_operator(x, plan, smaps, coil_idx, V):
    return MRFForward.apply(x, plan, smaps, coil_idx, V)
