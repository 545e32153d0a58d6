"""Python binding of libxrdvi (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels; PyTorch supplies
device memory and the current stream.

The functions carry the C names (xrdvi_profile, xrdvi_window_plan,
xrdvi_elbo_fwd, xrdvi_elbo_bwd, ...).  ``XrdviELBO`` wraps the forward and
the recomputing adjoint as a ``torch.autograd.Function``.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# XRDVI_LIB selects another build of the same library (e.g. to compare
# kernel variants); the default is the in-tree build.
LIB_PATH = os.environ.get("XRDVI_LIB", os.path.join(_PKG, "libxrdvi.so"))
HEADER = os.path.join(os.path.dirname(_PKG), "include", "xrdvi.h")

XRDVI_OK, XRDVI_PENDING = 0, 1
XRDVI_EINVAL, XRDVI_ENOMEM, XRDVI_EDEVICE = -1, -2, -3
XRDVI_EBUSY, XRDVI_ENOENT, XRDVI_ECANCELED = -4, -5, -6


class XrdviError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"xrdvi error {code}: {msg}")
        self.code = code


class Prior(C.Structure):
    _fields_ = [("lambda_h", C.c_double), ("mu_sd", C.c_double),
                ("w_shape", C.c_double), ("w_rate", C.c_double),
                ("alpha_mean", C.c_double), ("alpha_sd", C.c_double)]


class ProblemDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("bg", C.POINTER(C.c_double)),
                ("peak_off", C.POINTER(C.c_int32)),
                ("peak_pos", C.POINTER(C.c_double)),
                ("peak_int", C.POINTER(C.c_double)),
                ("cutoff", C.c_double), ("prior", Prior),
                ("asymmetric", C.c_int32), ("width_law", C.c_int32)]


_DP = C.POINTER(C.c_double)


class Request(C.Structure):
    _fields_ = [("problem", ProblemDesc), ("S", C.c_int32),
                ("steps", C.c_int32), ("seed", C.c_uint64), ("lr", C.c_double),
                ("init_loc", _DP), ("init_logscale", _DP), ("out_loc", _DP),
                ("out_logscale", _DP), ("out_elbo_trace", _DP)]


class Status(C.Structure):
    _fields_ = [("state", C.c_int32), ("steps_done", C.c_int32),
                ("t_arrive", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("final_elbo", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_slots", C.c_int32),
                ("max_queue", C.c_int32), ("steps_per_launch", C.c_int32),
                ("use_graph", C.c_int32), ("arena", C.c_void_p),
                ("arena_bytes", C.c_size_t), ("resident_bytes", C.c_size_t)]


class HmcConfig(C.Structure):
    _fields_ = [("chains", C.c_int32), ("n_warmup", C.c_int32),
                ("n_draws", C.c_int32), ("n_leapfrog", C.c_int32),
                ("step_size", C.c_double), ("target_accept", C.c_double),
                ("seed", C.c_uint64)]


_lib = None
_VP = C.c_void_p


def exported_symbols():
    """Names declared XRDVI_API in include/xrdvi.h."""
    txt = open(HEADER).read()
    return re.findall(r"XRDVI_API\s+[\w\s\*]+?\b(xrdvi_\w+)\s*\(", txt)


def load():
    """Loads libxrdvi.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_2501_09308_amd.build` (there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    i32, u64, dbl = C.c_int32, C.c_uint64, C.c_double
    sig = {
        "xrdvi_last_error": ([], C.c_char_p),
        "xrdvi_version": ([], C.c_int),
        "xrdvi_validate": ([C.POINTER(ProblemDesc)], C.c_int),
        "xrdvi_ctx_create": ([C.c_int, C.POINTER(_VP)], C.c_int),
        "xrdvi_ctx_destroy": ([_VP], C.c_int),
        "xrdvi_problem_create": ([_VP, C.POINTER(ProblemDesc), C.POINTER(_VP)], C.c_int),
        "xrdvi_problem_destroy": ([_VP], C.c_int),
        "xrdvi_problem_info": ([_VP, C.POINTER(i32), C.POINTER(i32),
                                C.POINTER(i32), C.POINTER(dbl)], C.c_int),
        "xrdvi_tape_create": ([_VP, _VP, i32, C.POINTER(_VP)], C.c_int),
        "xrdvi_tape_destroy": ([_VP], C.c_int),
        "xrdvi_profile": ([_VP, _VP, i32, _VP, _VP, _VP], C.c_int),
        "xrdvi_profile_static": ([_VP, _VP, i32, _VP, _VP, _VP], C.c_int),
        "xrdvi_window_plan": ([_VP, _VP, i32, _VP, _VP, _VP, _VP], C.c_int),
        "xrdvi_elbo_fwd": ([_VP, _VP, i32, _VP, _VP, _VP, u64, u64, i32, _VP,
                            _VP, _VP, _VP], C.c_int),
        "xrdvi_elbo_bwd": ([_VP, _VP, dbl, _VP, _VP, _VP, _VP], C.c_int),
        "xrdvi_tape_samples": ([_VP, _VP, _VP, _VP], C.c_int),
        "xrdvi_adam_step": ([_VP, i32, _VP, _VP, _VP, _VP, i32, dbl, dbl, dbl,
                             dbl, _VP], C.c_int),
        "xrdvi_server_create": ([C.POINTER(ServerConfig), C.POINTER(_VP)], C.c_int),
        "xrdvi_server_destroy": ([_VP], C.c_int),
        "xrdvi_submit": ([_VP, C.POINTER(Request), C.POINTER(C.c_uint64)], C.c_int),
        "xrdvi_poll": ([_VP, C.c_uint64, C.POINTER(Status)], C.c_int),
        "xrdvi_request_footprint": ([C.POINTER(Request), C.POINTER(C.c_size_t)],
                                    C.c_int),
        "xrdvi_cancel": ([_VP, C.c_uint64], C.c_int),
        "xrdvi_server_clock": ([_VP], C.c_double),
        "xrdvi_plain_run": ([_VP, C.POINTER(Request), C.POINTER(Status), _VP],
                            C.c_int),
        "xrdvi_readout": ([i32, _VP, _VP, _VP, _VP, dbl, _VP, _VP, _VP, _VP],
                          C.c_int),
        "xrdvi_problem_latents": ([_VP], C.c_int),
        "xrdvi_background": ([_VP, i32, i32, _VP, dbl, dbl, i32, _VP, _VP, _VP],
                             C.c_int),
        "xrdvi_logpost": ([_VP, _VP, i32, _VP, _VP, _VP, _VP, _VP], C.c_int),
        "xrdvi_hmc": ([_VP, _VP, C.POINTER(HmcConfig), _VP, _VP, _VP, _VP, _VP,
                       _VP], C.c_int),
        "xrdvi_timing_enable": ([_VP, i32], C.c_int),
        "xrdvi_timing_read": ([_VP, C.POINTER(dbl), C.POINTER(C.c_int64), i32],
                              C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        msg = load().xrdvi_last_error().decode(errors="replace")
        raise XrdviError(rc, msg)
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f64(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.contiguous()


def make_desc(x, y, bg, peak_off, peak_pos, peak_int, cutoff=0.0,
              lambda_h=0.0, mu_sd=0.03, w_shape=3.0, w_rate=100.0,
              asymmetric=False, alpha_mean=1.0, alpha_sd=0.2, width_law=0):
    """Builds a ProblemDesc over host arrays; returns (desc, keepalive).
    width_law: 0 (FWHM w) or 1 / "sec" (FWHM w sec(rho / 2))."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, bg)]
    off = np.ascontiguousarray(peak_off, dtype=np.int32)
    pos = np.ascontiguousarray(peak_pos, dtype=np.float64)
    inten = np.ascontiguousarray(peak_int, dtype=np.float64)
    if pos.size == 0:
        pos = np.zeros(1); inten = np.zeros(1)
    d = ProblemDesc()
    d.N = len(arrs[0]); d.K = len(off) - 1
    P = C.POINTER(C.c_double)
    d.x = arrs[0].ctypes.data_as(P); d.y = arrs[1].ctypes.data_as(P)
    d.bg = arrs[2].ctypes.data_as(P)
    d.peak_off = off.ctypes.data_as(C.POINTER(C.c_int32))
    d.peak_pos = pos.ctypes.data_as(P); d.peak_int = inten.ctypes.data_as(P)
    d.cutoff = float(cutoff)
    d.prior = Prior(lambda_h, mu_sd, w_shape, w_rate, alpha_mean, alpha_sd)
    d.asymmetric = 1 if asymmetric else 0
    d.width_law = 1 if width_law == "sec" else int(width_law or 0)
    return d, (arrs, off, pos, inten)


def xrdvi_validate(**kw):
    d, keep = make_desc(**kw)
    return _check(load().xrdvi_validate(C.byref(d)))


class Context:
    def __init__(self, device: int = 0):
        self.lib = load()
        h = _VP()
        _check(self.lib.xrdvi_ctx_create(int(device), C.byref(h)))
        self.handle = h
        self.device = int(device)

    def close(self):
        if self.handle:
            self.lib.xrdvi_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def xrdvi_timing_enable(ctx: Context, enable: bool = True):
    _check(ctx.lib.xrdvi_timing_enable(ctx.handle, 1 if enable else 0))


def xrdvi_timing_read(ctx: Context, reset: bool = True):
    """(total ms, launches) of the fused kernel since the last reset."""
    ms, n = C.c_double(), C.c_int64()
    _check(ctx.lib.xrdvi_timing_read(ctx.handle, C.byref(ms), C.byref(n),
                                     1 if reset else 0))
    return ms.value, n.value


def xrdvi_ctx_create(device: int = 0) -> Context:
    return Context(device)


class Problem:
    """A prepared problem on the device (xrdvi_problem_create)."""

    def __init__(self, ctx: Context, x, y, bg, peak_off, peak_pos, peak_int,
                 cutoff=0.0, lambda_h=0.0, mu_sd=0.03, w_shape=3.0,
                 w_rate=100.0, asymmetric=False, alpha_mean=1.0, alpha_sd=0.2,
                 width_law=0):
        self.ctx = ctx
        d, keep = make_desc(x, y, bg, peak_off, peak_pos, peak_int, cutoff,
                            lambda_h, mu_sd, w_shape, w_rate, asymmetric,
                            alpha_mean, alpha_sd, width_law)
        h = _VP()
        _check(ctx.lib.xrdvi_problem_create(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h
        N, K, T, lam = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        _check(ctx.lib.xrdvi_problem_info(h, C.byref(N), C.byref(K), C.byref(T),
                                          C.byref(lam)))
        self.N, self.K, self.T, self.lambda_h = N.value, K.value, T.value, lam.value
        self.cutoff = float(cutoff)
        self.D = 5 if asymmetric else 4     # latent types per phase
        self.width_law = d.width_law

    @classmethod
    def from_workload(cls, ctx, prob, y, **kw):
        return cls(ctx, prob.x, y, prob.bg, prob.peak_off, prob.peak_pos,
                   prob.peak_int, kw.pop("cutoff", prob.cutoff), **kw)

    def close(self):
        if self.handle:
            self.ctx.lib.xrdvi_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def xrdvi_problem_create(ctx, *a, **kw) -> Problem:
    return Problem(ctx, *a, **kw)


class Tape:
    def __init__(self, ctx: Context, prob: Problem, S: int):
        self.ctx, self.prob, self.S = ctx, prob, int(S)
        h = _VP()
        _check(ctx.lib.xrdvi_tape_create(ctx.handle, prob.handle, int(S), C.byref(h)))
        self.handle = h
        self.version = 0

    def close(self):
        if self.handle:
            self.ctx.lib.xrdvi_tape_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def xrdvi_tape_create(ctx, prob, S) -> Tape:
    return Tape(ctx, prob, S)


def xrdvi_profile(ctx: Context, prob: Problem, phi: torch.Tensor,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """f[S][N] (float32) at constrained phi[S][D][K] (float64, device)."""
    if phi.dim() == 2:
        phi = phi.unsqueeze(0)
    S = phi.shape[0]
    phi = _dev_f64(phi, (S, prob.D, prob.K), "phi")
    if out is None:
        out = torch.empty((S, prob.N), dtype=torch.float32, device=phi.device)
    _check(ctx.lib.xrdvi_profile(ctx.handle, prob.handle, S, _ptr(phi), _ptr(out),
                                 _stream(phi.device)))
    return out


def xrdvi_profile_static(ctx: Context, prob: Problem, phi: torch.Tensor,
                         out: torch.Tensor) -> torch.Tensor:
    """As xrdvi_profile, through the allocation-free entry point: the caller
    passes the output f[S][N] (float32, device)."""
    if phi.dim() == 2:
        phi = phi.unsqueeze(0)
    S = phi.shape[0]
    phi = _dev_f64(phi, (S, prob.D, prob.K), "phi")
    if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
            and tuple(out.shape) == (S, prob.N)):
        raise TypeError(f"out must be a contiguous float32 CUDA tensor of shape "
                        f"({S}, {prob.N})")
    _check(ctx.lib.xrdvi_profile_static(ctx.handle, prob.handle, S, _ptr(phi),
                                        _ptr(out), _stream(phi.device)))
    return out


def xrdvi_window_plan(ctx: Context, prob: Problem, phi: torch.Tensor):
    """(lo, hi) int32 [S][T] in the caller's peak order."""
    if phi.dim() == 2:
        phi = phi.unsqueeze(0)
    S = phi.shape[0]
    phi = _dev_f64(phi, (S, prob.D, prob.K), "phi")
    lo = torch.empty((S, max(prob.T, 1)), dtype=torch.int32, device=phi.device)
    hi = torch.empty_like(lo)
    _check(ctx.lib.xrdvi_window_plan(ctx.handle, prob.handle, S, _ptr(phi),
                                     _ptr(lo), _ptr(hi), _stream(phi.device)))
    return lo[:, :prob.T], hi[:, :prob.T]


def xrdvi_elbo_fwd(ctx: Context, prob: Problem, tape: Tape, loc, logscale,
                   eps=None, seed=0, step=0, need_grad=True, elbo_out=None,
                   loglik_out=None):
    """Returns (elbo [1], loglik [S]) float64 device tensors."""
    K, S, D = prob.K, tape.S, prob.D
    loc = _dev_f64(loc, (D, K), "loc")
    logscale = _dev_f64(logscale, (D, K), "logscale")
    if eps is not None:
        eps = _dev_f64(eps, (S, D, K), "eps")
    dev = loc.device
    if elbo_out is None:
        elbo_out = torch.empty(1, dtype=torch.float64, device=dev)
    if loglik_out is None:
        loglik_out = torch.empty(S, dtype=torch.float64, device=dev)
    _check(ctx.lib.xrdvi_elbo_fwd(ctx.handle, prob.handle, S, _ptr(loc),
                                  _ptr(logscale), _ptr(eps), C.c_uint64(seed),
                                  C.c_uint64(step), 1 if need_grad else 0,
                                  _ptr(elbo_out), _ptr(loglik_out), tape.handle,
                                  _stream(dev)))
    tape.version += 1
    return elbo_out, loglik_out


def xrdvi_tape_samples(ctx: Context, tape: Tape, out=None):
    """Constrained samples [S][D][K] of the last forward on `tape`."""
    if out is None:
        out = torch.empty((tape.S, tape.prob.D, tape.prob.K), dtype=torch.float64,
                          device=torch.device("cuda", ctx.device))
    _check(ctx.lib.xrdvi_tape_samples(ctx.handle, tape.handle, _ptr(out),
                                      _stream(out.device)))
    return out


def xrdvi_elbo_bwd(ctx: Context, tape: Tape, grad_scale=1.0,
                   grad_scale_dev: torch.Tensor | None = None,
                   grad_loc=None, grad_logscale=None, device=None):
    K, D = tape.prob.K, tape.prob.D
    dev = device if device is not None else torch.device("cuda", ctx.device)
    if grad_loc is None:
        grad_loc = torch.empty((D, K), dtype=torch.float64, device=dev)
    if grad_logscale is None:
        grad_logscale = torch.empty((D, K), dtype=torch.float64, device=dev)
    if grad_scale_dev is not None:
        grad_scale_dev = grad_scale_dev.to(torch.float64).contiguous()
    _check(ctx.lib.xrdvi_elbo_bwd(ctx.handle, tape.handle, float(grad_scale),
                                  _ptr(grad_scale_dev), _ptr(grad_loc),
                                  _ptr(grad_logscale), _stream(dev)))
    return grad_loc, grad_logscale


class XrdviELBO(torch.autograd.Function):
    """ELBO estimate as a differentiable function of (loc, logscale).

    Forward runs the fused profile + likelihood + recomputing adjoint; the
    backward only applies the chain rule to the saved per-tile sums (no
    S x K x N basis is stored).  One tape holds one pending backward: a
    second forward on the same tape invalidates the first graph."""

    @staticmethod
    def forward(fctx, loc, logscale, ctx_, prob, tape, eps, seed, step):
        need = bool(fctx.needs_input_grad[0] or fctx.needs_input_grad[1])
        elbo, _ = xrdvi_elbo_fwd(ctx_, prob, tape, loc.detach(),
                                 logscale.detach(), eps=eps, seed=seed,
                                 step=step, need_grad=need)
        fctx.ctx_, fctx.tape = ctx_, tape
        fctx.version = tape.version
        return elbo[0]

    @staticmethod
    def backward(fctx, g):
        if fctx.tape.version != fctx.version:
            raise RuntimeError("the tape was reused by a later forward before "
                               "this backward")
        gl, gs = xrdvi_elbo_bwd(fctx.ctx_, fctx.tape, 1.0,
                                grad_scale_dev=g.reshape(1),
                                device=g.device)
        return gl, gs, None, None, None, None, None, None


def elbo(ctx, prob, tape, loc, logscale, eps=None, seed=0, step=0):
    return XrdviELBO.apply(loc, logscale, ctx, prob, tape, eps, seed, step)


def xrdvi_adam_step(ctx: Context, theta, m1, m2, grad, t, lr=1e-2, beta1=0.9,
                    beta2=0.999, eps=1e-8):
    """In-place Adam ascent step on float64 CUDA tensors."""
    for name, a in (("theta", theta), ("m1", m1), ("m2", m2), ("grad", grad)):
        if not (a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    _check(ctx.lib.xrdvi_adam_step(ctx.handle, theta.numel(), _ptr(theta),
                                   _ptr(m1), _ptr(m2), _ptr(grad), int(t),
                                   float(lr), float(beta1), float(beta2),
                                   float(eps), _stream(theta.device)))


class _Submission:
    """Host buffers of one request, kept alive until it completes."""

    def __init__(self, x, y, bg, peak_off, peak_pos, peak_int, cutoff, S,
                 steps, seed, lr, init, prior):
        self.desc, self.keep = make_desc(x, y, bg, peak_off, peak_pos,
                                         peak_int, cutoff, **prior)
        K = len(peak_off) - 1
        D = 5 if prior.get("asymmetric") else 4
        self.loc = np.zeros((D, K))
        self.logscale = np.zeros((D, K))
        self.trace = np.zeros(int(steps))
        self.init = None
        if init is not None:
            self.init = [np.ascontiguousarray(a, dtype=np.float64) for a in init]
        r = Request()
        r.problem = self.desc
        r.S, r.steps, r.seed, r.lr = int(S), int(steps), int(seed), float(lr)
        if self.init is not None:
            r.init_loc = self.init[0].ctypes.data_as(_DP)
            r.init_logscale = self.init[1].ctypes.data_as(_DP)
        r.out_loc = self.loc.ctypes.data_as(_DP)
        r.out_logscale = self.logscale.ctypes.data_as(_DP)
        r.out_elbo_trace = self.trace.ctypes.data_as(_DP)
        self.req = r


def _request_args(prob, y, S, steps, seed, lr=0.0, init=None, cutoff=None,
                  **prior):
    return (prob.x, y, prob.bg, prob.peak_off, prob.peak_pos, prob.peak_int,
            prob.cutoff if cutoff is None else cutoff, S, steps, seed, lr,
            init, prior)


class Server:
    """xrdvi_server: continuous batching of whole analyses (see xrdvi.h)."""

    def __init__(self, device=0, max_slots=16, max_queue=1 << 16,
                 steps_per_launch=10, use_graph=True, arena=None,
                 arena_bytes=None, resident_bytes=0):
        self.lib = load()
        cfg = ServerConfig()
        cfg.device, cfg.max_slots, cfg.max_queue = device, max_slots, max_queue
        cfg.steps_per_launch, cfg.use_graph = steps_per_launch, 1 if use_graph else 0
        if arena is not None:
            cfg.arena = C.c_void_p(arena.data_ptr())
            cfg.arena_bytes = arena.numel() * arena.element_size()
        else:
            cfg.arena = None
            cfg.arena_bytes = int(arena_bytes or (8 << 30))
        cfg.resident_bytes = int(resident_bytes)
        self._arena = arena
        h = _VP()
        _check(self.lib.xrdvi_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        self._subs = {}

    def submit(self, prob, y, S, steps, seed, lr=0.0, init=None, **kw):
        sub = _Submission(*_request_args(prob, y, S, steps, seed, lr, init, **kw))
        t = C.c_uint64()
        _check(self.lib.xrdvi_submit(self.handle, C.byref(sub.req), C.byref(t)))
        self._subs[t.value] = sub
        return t.value

    def poll(self, ticket):
        """(state, status dict, outputs or None).  Outputs are returned once
        the request is done: dict(loc, logscale, trace)."""
        st = Status()
        rc = self.lib.xrdvi_poll(self.handle, C.c_uint64(ticket), C.byref(st))
        if rc == XRDVI_ENOENT:
            raise XrdviError(rc, "unknown ticket")
        info = dict(state=st.state, steps_done=st.steps_done,
                    t_arrive=st.t_arrive, t_admit=st.t_admit, t_done=st.t_done,
                    final_elbo=st.final_elbo)
        out = None
        if rc != XRDVI_PENDING:
            sub = self._subs.pop(ticket)
            if rc == XRDVI_OK:
                out = dict(loc=sub.loc, logscale=sub.logscale, trace=sub.trace)
        return rc, info, out

    def cancel(self, ticket):
        _check(self.lib.xrdvi_cancel(self.handle, C.c_uint64(ticket)))

    def clock(self):
        return self.lib.xrdvi_server_clock(self.handle)

    def close(self):
        if self.handle:
            self.lib.xrdvi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_footprint(prob, y, S, steps, seed=0, **kw) -> int:
    """Arena bytes the request would occupy while resident (host only)."""
    sub = _Submission(*_request_args(prob, y, S, steps, seed, 0.0, None, **kw))
    out = C.c_size_t()
    _check(load().xrdvi_request_footprint(C.byref(sub.req), C.byref(out)))
    return int(out.value)


def xrdvi_plain_run(ctx: Context, prob, y, S, steps, seed, lr=0.0, init=None,
                    **kw):
    """One analysis with per-step launches (the sequential reference)."""
    sub = _Submission(*_request_args(prob, y, S, steps, seed, lr, init, **kw))
    st = Status()
    _check(ctx.lib.xrdvi_plain_run(ctx.handle, C.byref(sub.req), C.byref(st),
                                   _stream()))
    return dict(loc=sub.loc, logscale=sub.logscale, trace=sub.trace,
                final_elbo=st.final_elbo)


def xrdvi_readout(peak_off, peak_int, loc, logscale, threshold=0.01):
    """Posterior readout (host): dict(mean_h, sd_h, area_ratio, selected)
    from the h rows of (loc, logscale)."""
    off = np.ascontiguousarray(peak_off, dtype=np.int32)
    inten = np.ascontiguousarray(peak_int, dtype=np.float64)
    if inten.size == 0:
        inten = np.zeros(1)
    K = len(off) - 1
    m = np.ascontiguousarray(np.asarray(loc)[0], dtype=np.float64)
    s = np.ascontiguousarray(np.asarray(logscale)[0], dtype=np.float64)
    if m.shape != (K,) or s.shape != (K,):
        raise ValueError(f"loc and logscale must have K={K} columns")
    out = {k: np.empty(K) for k in ("mean_h", "sd_h", "area_ratio")}
    sel = np.empty(K, dtype=np.int32)
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(load().xrdvi_readout(K, P(off), P(inten), P(m), P(s),
                                float(threshold), P(out["mean_h"]),
                                P(out["sd_h"]), P(out["area_ratio"]), P(sel)))
    out["selected"] = np.nonzero(sel)[0]
    return out


def xrdvi_logpost(ctx: Context, prob: Problem, tape: Tape, z, grad=True):
    """(logp [S], grad [S][D][K] or None) at positions z [S][D][K]."""
    S = tape.S
    z = _dev_f64(z, (S, prob.D, prob.K), "z")
    logp = torch.empty(S, dtype=torch.float64, device=z.device)
    g = torch.empty_like(z) if grad else None
    _check(ctx.lib.xrdvi_logpost(ctx.handle, prob.handle, S, _ptr(z), _ptr(logp),
                                 _ptr(g), tape.handle, _stream(z.device)))
    tape.version += 1
    return logp, g


def xrdvi_hmc(ctx: Context, prob: Problem, z, n_warmup, n_draws, n_leapfrog,
              step_size, seed, target_accept=0.8, keep_draws=True):
    """Hamiltonian Monte Carlo from positions z [chains][D][K] (a contiguous
    float64 CUDA tensor, updated in place to the final positions).
    Returns dict(draws [n_draws][chains][D][K] or None, logp
    [n_draws][chains], accept [chains], step [chains])."""
    nc = z.shape[0]
    if not (isinstance(z, torch.Tensor) and z.is_cuda and z.dtype == torch.float64
            and z.is_contiguous() and tuple(z.shape) == (nc, prob.D, prob.K)):
        raise ValueError(f"z must be a contiguous float64 CUDA tensor of shape "
                         f"({nc}, {prob.D}, {prob.K})")
    cfg = HmcConfig(nc, int(n_warmup), int(n_draws), int(n_leapfrog),
                    float(step_size), float(target_accept), int(seed))
    draws = (torch.empty((n_draws, nc, prob.D, prob.K), dtype=torch.float64,
                         device=z.device) if keep_draws and n_draws else None)
    logp = torch.empty((max(n_draws, 1), nc), dtype=torch.float64, device=z.device)
    acc = np.zeros(nc)
    step = np.zeros(nc)
    _check(ctx.lib.xrdvi_hmc(ctx.handle, prob.handle, C.byref(cfg), _ptr(z),
                             _ptr(draws), _ptr(logp),
                             acc.ctypes.data_as(C.c_void_p),
                             step.ctypes.data_as(C.c_void_p), _stream(z.device)))
    return dict(draws=draws, logp=logp[:n_draws], accept=acc, step=step)


def xrdvi_background(ctx: Context, y, lam=1e6, p=0.01, n_iter=10):
    """Asymmetric-least-squares background of spectra y [B][N] (or [N]),
    float64 CUDA tensor; returns a tensor of the same shape."""
    squeeze = y.dim() == 1
    y2 = y.unsqueeze(0) if squeeze else y
    B, N = y2.shape
    y2 = _dev_f64(y2, (B, N), "y")
    out = torch.empty_like(y2)
    scratch = torch.empty(4 * B * N, dtype=torch.float64, device=y2.device)
    _check(ctx.lib.xrdvi_background(ctx.handle, B, N, _ptr(y2), float(lam),
                                    float(p), int(n_iter), _ptr(out),
                                    _ptr(scratch), _stream(y2.device)))
    return out[0] if squeeze else out
