"""Python binding of the CCMF solver library (include/ccmf.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory and the stream; there is no fallback
path -- if the library is not built, importing or calling this raises.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

__all__ = ["Plan", "SolveResult", "effective_crack_energy", "GeffFunction", "stream_copy"]

_DT = {torch.float64: _lib.CCMF_F64, torch.float32: _lib.CCMF_F32}


@dataclass
class SolveResult:
    geff: np.ndarray            # [F, L] effective crack energy per field and load
    iterations: np.ndarray      # [F, L] number of xi-steps taken
    residual: np.ndarray        # [F, L] |e^k - xi^{k+1/2}|_{L2} at the stopping iterate
    dual_est: np.ndarray        # [F, L] <A xibar, v^k>
    converged: bool
    mean_flux: np.ndarray = None          # [F, L, 3] <A* v^k>: d geff / d xibar at the optimum
    history: Optional[np.ndarray] = None  # [F, L, I, 4] residual, rho, energy, |<v>| per iteration
    phi: Optional[torch.Tensor] = None    # [F, L, N1, N2, N3], float64
    flux: Optional[torch.Tensor] = None   # [F, L, 3, N1, N2, N3]


def _dptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A solver plan for F crack-resistance fields kappa of one grid size.

    kappa: CUDA tensor [N1, N2, N3] or [F, N1, N2, N3], float64 (FP64 mode) or
    float32 (FP32 fields, FP64 reductions).  The plan copies it.
    """

    def __init__(self, kappa: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
        lib = _lib.load()
        if not kappa.is_cuda:
            raise ValueError("kappa must be a CUDA (HIP) tensor")
        if kappa.dtype not in _DT:
            raise ValueError("kappa must be float32 or float64")
        if kappa.dim() == 3:
            kappa = kappa.unsqueeze(0)
        if kappa.dim() != 4:
            raise ValueError("kappa must have shape [N1,N2,N3] or [F,N1,N2,N3]")
        kappa = kappa.contiguous()
        self.dtype = kappa.dtype
        self.device = kappa.device
        self.n_fields = int(kappa.shape[0])
        self.dims = tuple(int(d) for d in kappa.shape[1:])
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        dims = (ctypes.c_int64 * 3)(*self.dims)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib.ccmf_setup(ctypes.byref(handle), dims, self.n_fields, _DT[self.dtype],
                                      _dptr(kappa), ctypes.c_void_p(self.stream.cuda_stream)))
        self._h = handle
        self._lib = lib
        self.n_loads = 0

    @property
    def N(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ccmf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, xi: Sequence[Sequence[float]], tol: float = 1e-4, *, delta: float = 0.25,
              rule: str = "bb", rho0: float = 0.0, max_iter: int = 20000, check_every: int = 32,
              want_phi: bool = False, want_flux: bool = False, time_kernels: bool = False,
              raise_not_converged: bool = False, bb_min_corr: float = 0.0, eta0: float = 0.0,
              k0: float = 0.0, eager: bool = False, autotune: bool = True,
              warm_start: bool = False, record_history: bool = False) -> SolveResult:
        xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(-1, 3))
        L = xi.shape[0]
        B = self.n_fields * L
        opt = _lib.Options(delta=delta, rho0=rho0, rule=_lib.RULES[rule], max_iter=max_iter,
                           check_every=check_every, time_kernels=int(bool(time_kernels)),
                           bb_min_corr=bb_min_corr, eta0=eta0, k0=k0, eager=int(bool(eager)),
                           no_autotune=int(not autotune), warm_start=int(bool(warm_start)),
                           record_history=int(bool(record_history)))
        geff = np.zeros(B)
        iters = np.zeros(B, dtype=np.int32)
        res = np.zeros(B)
        dual = np.zeros(B)
        phi = flux = None
        if want_phi:
            phi = torch.empty((self.n_fields, L) + self.dims, dtype=torch.float64, device=self.device)
        if want_flux:
            flux = torch.empty((self.n_fields, L, 3) + self.dims, dtype=self.dtype, device=self.device)
        dp = ctypes.POINTER(ctypes.c_double)
        with torch.cuda.device(self.device):
            code = self._lib.ccmf_solve(
                self._h, xi.ctypes.data_as(dp), L, float(tol), ctypes.byref(opt),
                geff.ctypes.data_as(dp), iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                res.ctypes.data_as(dp), dual.ctypes.data_as(dp),
                _dptr(phi) if phi is not None else None, _dptr(flux) if flux is not None else None)
        _lib.check(code, allow_not_converged=not raise_not_converged)
        self.n_loads = L
        shape = (self.n_fields, L)
        mflux = np.zeros((B, 3))
        _lib.check(self._lib.ccmf_mean_flux(self._h, mflux.ctypes.data_as(dp)))
        hist = None
        if record_history:
            n = int(iters.max())
            hist = np.zeros((B, n, 4))
            _lib.check(self._lib.ccmf_history(self._h, n, hist.ctypes.data_as(dp)))
            hist = hist.reshape(shape + (n, 4))
        return SolveResult(geff.reshape(shape), iters.reshape(shape), res.reshape(shape),
                           dual.reshape(shape), code == _lib.CCMF_OK, mflux.reshape(shape + (3,)), hist, phi, flux)

    def get_state(self):
        """(v, e, rho, k) of the plan's state: v, e [F, L, 6, N1, N2, N3] in the plan's dtype."""
        B = self.n_fields * self.n_loads
        if B == 0:   # no solve yet: the library reports the missing state
            _lib.check(self._lib.ccmf_get_state(self._h, None, None, None, None))
        v = torch.empty((self.n_fields, self.n_loads, 6) + self.dims, dtype=self.dtype, device=self.device)
        e = torch.empty_like(v)
        rho = np.zeros(B)
        k = np.zeros(B, dtype=np.int32)
        with torch.cuda.device(self.device):
            _lib.check(self._lib.ccmf_get_state(self._h, _dptr(v), _dptr(e),
                                                rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return v, e, rho.reshape(self.n_fields, -1), k.reshape(self.n_fields, -1)

    def set_state(self, v: torch.Tensor, e: torch.Tensor, rho, k):
        """Load (v, e, rho, k), v and e [F, L, 6, N1, N2, N3], for solve(..., warm_start=True)."""
        L = v.numel() // (self.n_fields * 6 * self.N)
        if v.shape != e.shape or v.numel() != self.n_fields * L * 6 * self.N or L < 1:
            raise ValueError("v and e must have shape [F, L, 6, N1, N2, N3]")
        v = v.to(self.dtype).contiguous()
        e = e.to(self.dtype).contiguous()
        B = self.n_fields * L
        rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64).reshape(-1), (B,)))
        k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32).reshape(-1), (B,)))
        with torch.cuda.device(self.device):
            _lib.check(self._lib.ccmf_set_state(self._h, L, _dptr(v), _dptr(e),
                                                rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        self.n_loads = L

    def grad_kappa(self, dL_dgeff) -> torch.Tensor:
        """Envelope gradient of the last solve: sum_l dL/dgeff[f,l] * |xi*_{f,l}[x]|/N."""
        dl = np.ascontiguousarray(np.asarray(dL_dgeff, dtype=np.float64).reshape(-1))
        if self.n_loads and dl.size != self.n_fields * self.n_loads:
            raise ValueError("dL_dgeff must have one entry per (field, load) of the last solve")
        out = torch.empty((self.n_fields,) + self.dims, dtype=self.dtype, device=self.device)
        with torch.cuda.device(self.device):
            _lib.check(self._lib.ccmf_grad_kappa(self._h, dl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 _dptr(out)))
        return out

    def certificate(self):
        """(cert, sigma) per (field, load) of the last solve: cert <= geff_true <= geff."""
        B = self.n_fields * self.n_loads
        cert = np.zeros(B)
        sig = np.zeros(B)
        dp = ctypes.POINTER(ctypes.c_double)
        with torch.cuda.device(self.device):
            _lib.check(self._lib.ccmf_certificate(self._h, cert.ctypes.data_as(dp), sig.ctypes.data_as(dp)))
        return cert.reshape(self.n_fields, -1), sig.reshape(self.n_fields, -1)

    def kernel_times(self):
        """(average ms, launches, algorithmic bytes per launch and problem) of the fused update kernel."""
        avg = ctypes.c_double()
        cnt = ctypes.c_int64()
        by = ctypes.c_double()
        _lib.check(self._lib.ccmf_kernel_times(self._h, ctypes.byref(avg), ctypes.byref(cnt), ctypes.byref(by)))
        return avg.value, cnt.value, by.value

    def laplace_pinv(self, r: torch.Tensor) -> torch.Tensor:
        """(div^- grad^+)^dagger applied to each field of r [..., N1, N2, N3]; float64 result."""
        r = r.to(self.dtype).contiguous()
        out = torch.empty(r.shape, dtype=torch.float64, device=r.device)
        count = r.numel() // self.N
        with torch.cuda.device(self.device):
            _lib.check(self._lib.ccmf_laplace_pinv(self._h, _dptr(r), _dptr(out), count))
        return out

    def hartley_axis(self, data: torch.Tensor, axis: int) -> torch.Tensor:
        """Unnormalised Hartley transform along one axis of each field (in place on a copy)."""
        out = data.to(self.dtype).contiguous().clone()
        count = out.numel() // self.N
        with torch.cuda.device(self.device):
            _lib.check(self._lib.ccmf_hartley_axis(self._h, _dptr(out), count, int(axis)))
        return out


def stream_copy(dst: torch.Tensor, src: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    lib = _lib.load()
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    nbytes = src.numel() * src.element_size()
    _lib.check(lib.ccmf_stream_copy(_dptr(dst), _dptr(src), nbytes, ctypes.c_void_p(s.cuda_stream)))


class GeffFunction(torch.autograd.Function):
    """geff(kappa; xi) differentiable in kappa (envelope theorem on the min-cut form) and
    in the loads xi [L, 3]: the value is geff of the unit direction xi/|xi|, whose gradient
    is (m - geff xi/|xi|)/|xi| with m the mean face flux (the gradient of the 1-homogeneous
    extension)."""

    @staticmethod
    def forward(ctx, kappa, xi, tol, solve_kwargs):
        plan = Plan(kappa.detach())
        xin = np.asarray(xi.detach().cpu().double().numpy() if torch.is_tensor(xi) else xi,
                         dtype=np.float64).reshape(-1, 3)
        res = plan.solve(xin, tol, **(solve_kwargs or {}))
        ctx.plan = plan
        ctx.kappa_shape = kappa.shape
        ctx.xi_tensor = torch.is_tensor(xi)
        ctx.xi_meta = (xi.shape, xi.dtype, xi.device) if torch.is_tensor(xi) else None
        ctx.xin = xin
        ctx.geff = res.geff
        ctx.mflux = res.mean_flux
        return torch.as_tensor(res.geff, dtype=torch.float64, device=kappa.device).reshape(
            (plan.n_fields, -1) if kappa.dim() == 4 else (-1,))

    @staticmethod
    def backward(ctx, grad_out):
        plan = ctx.plan
        go = grad_out.detach().double().cpu().numpy().reshape(plan.n_fields, -1)
        g = plan.grad_kappa(go) if ctx.needs_input_grad[0] else None
        plan.close()
        gxi = None
        if ctx.xi_tensor and ctx.needs_input_grad[1]:
            nr = np.linalg.norm(ctx.xin, axis=1)                       # [L]
            u = ctx.xin / nr[:, None]
            tang = (ctx.mflux - ctx.geff[..., None] * u[None]) / nr[None, :, None]   # [F, L, 3]
            shape, dtype, device = ctx.xi_meta
            gxi = torch.as_tensor((go[..., None] * tang).sum(0)).reshape(shape).to(device=device, dtype=dtype)
        return (g.reshape(ctx.kappa_shape) if g is not None else None), gxi, None, None


def effective_crack_energy(kappa: torch.Tensor, xi, tol: float = 1e-4, **solve_kwargs) -> torch.Tensor:
    """Differentiable geff(kappa; xi) (float64 result, one value per field and load)."""
    return GeffFunction.apply(kappa, xi, tol, solve_kwargs)
