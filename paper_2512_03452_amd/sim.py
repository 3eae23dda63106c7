"""Python front end of libsipf.so: device memory and streams come from torch,
every step of the method runs in the library's HIP kernels."""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype(prm):
    return torch.float32 if prm.precision == _lib.SIPF_FP32 else torch.float64


def _dim(prm):
    return 2 if prm.dim == 2 else 3


def _shapes(H, d):
    """Shapes of the fields of the ABI in dimension d: rho, grad, alpha (re/im last)."""
    if d == 2:
        return {"rho": (H, H), "grad": (2, H, H), "alpha": (H, H // 2 + 1, 2)}
    return {"rho": (H, H, H), "grad": (3, H, H, H), "alpha": (H, H, H // 2 + 1, 2)}


class Sim:
    """One SIPF-PIC simulation (Algorithm 4) held by the library.

    X0: (P, d) positions (numpy array or torch tensor); alpha0: optional
    complex half spectrum of c(x, 0), (H, H, H/2+1) in 3-D or (H, H/2+1) in
    2-D.  Keyword arguments are ``sipf_params`` fields (scheme/precision may
    be given as strings; dim=2 selects the two-dimensional variant, eps=0 the
    elliptic c-equation).
    """

    def __init__(self, X0, alpha0=None, stream=None, **params):
        lib = _lib.load()
        self.params = _lib.default_params(**params)
        self.dtype = _dtype(self.params)
        self.device = torch.device("cuda", torch.cuda.current_device())
        X = torch.as_tensor(np.asarray(X0) if not torch.is_tensor(X0) else X0)
        X = X.to(device=self.device, dtype=self.dtype).contiguous()
        self.dim = _dim(self.params)
        if X.ndim != 2 or X.shape[1] != self.dim:
            raise ValueError(f"X0 must have shape (P, {self.dim})")
        self.P = int(X.shape[0])
        self.H = int(self.params.H)
        a_ptr = None
        if alpha0 is not None:
            a = torch.as_tensor(alpha0)
            cdt = torch.complex64 if self.dtype == torch.float32 else torch.complex128
            a = a.to(device=self.device, dtype=cdt).contiguous()
            want = _shapes(self.H, self.dim)["alpha"][:-1]
            if tuple(a.shape) != want:
                raise ValueError(f"alpha0 must have shape {want}")
            a_ptr = ctypes.c_void_p(a.data_ptr())
        self._stream = stream
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        check(lib.sipf_init(ctypes.byref(self.params), self.P, ctypes.c_void_p(X.data_ptr()), 1,
                            a_ptr, 1, _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    # -- stepping ------------------------------------------------------------
    def step(self):
        check(_lib.load().sipf_step(self._h))

    def run(self, nsteps):
        check(_lib.load().sipf_run(self._h, int(nsteps)))

    def prepare_run(self, nsteps):
        """Capture every graph that run(nsteps) issued next would replay (runs nothing)."""
        check(_lib.load().sipf_prepare_run(self._h, int(nsteps)))

    def sync(self):
        check(_lib.load().sipf_sync(self._h))

    @property
    def n(self):
        v = ctypes.c_int64()
        check(_lib.load().sipf_get_step(self._h, ctypes.byref(v)))
        return v.value

    # -- state ----------------------------------------------------------------
    def positions(self):
        out = torch.empty((self.P, self.dim), dtype=self.dtype, device=self.device)
        check(_lib.load().sipf_get_positions(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def field(self, which):
        H = self.H
        lib = _lib.load()
        shp = _shapes(H, self.dim)
        if which in ("rho", _lib.SIPF_FIELD_RHO):
            out = torch.empty(shp["rho"], dtype=self.dtype, device=self.device)
            check(lib.sipf_get_field(self._h, _lib.SIPF_FIELD_RHO, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        if which in ("grad", _lib.SIPF_FIELD_GRAD):
            out = torch.empty(shp["grad"], dtype=self.dtype, device=self.device)
            check(lib.sipf_get_field(self._h, _lib.SIPF_FIELD_GRAD, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        if which in ("alpha", _lib.SIPF_FIELD_ALPHA):
            out = torch.empty(shp["alpha"], dtype=self.dtype, device=self.device)
            check(lib.sipf_get_field(self._h, _lib.SIPF_FIELD_ALPHA, ctypes.c_void_p(out.data_ptr()), 1))
            return torch.view_as_complex(out)
        raise ValueError("which must be 'rho', 'alpha' or 'grad'")

    def diagnostics(self):
        """Diagnostics of the current state (sipf_diagnostics) as a dict:
        step, mass, rho_max, hf_share, c_integral, r_num, m2."""
        d = _lib.SipfDiag()
        check(_lib.load().sipf_diagnostics(self._h, ctypes.byref(d)))
        return d.as_dict()

    def profile(self, enable=True):
        """Start (clearing the accumulators) or stop per-phase event timing."""
        check(_lib.load().sipf_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{phase: (total ms, launches)} since profiling was enabled (synchronises)."""
        n = len(_lib.PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        check(_lib.load().sipf_profile_read(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_lib.PHASES)}

    def adjoint(self, nsteps, ckpt_every=10, phi_bar=None):
        """Pathwise gradient of a final-density loss (the context must be at step 0).

        Runs nsteps forward steps, then the reverse sweep.  With phi_bar None the
        loss is sum(phi^2) for phi the deposit of X^(N); otherwise it is
        sum(phi_bar * phi).  Returns (loss, dL/dchi, dL/dmu, dL/dX0) with dX0 a
        (P, 3) device tensor in original particle order.
        """
        loss, dchi, dmu = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        dX0 = torch.empty((self.P, 3), dtype=self.dtype, device=self.device)
        pb = None
        if phi_bar is not None:
            phi_bar = torch.as_tensor(phi_bar).to(device=self.device, dtype=self.dtype).contiguous()
            if tuple(phi_bar.shape) != (self.H, self.H, self.H):
                raise ValueError("phi_bar must have shape (H, H, H)")
            pb = ctypes.c_void_p(phi_bar.data_ptr())
        check(_lib.load().sipf_adjoint(self._h, int(nsteps), int(ckpt_every), pb, ctypes.byref(loss),
                                       ctypes.byref(dchi), ctypes.byref(dmu), ctypes.c_void_p(dX0.data_ptr())))
        return loss.value, dchi.value, dmu.value, dX0

    def save(self, path):
        check(_lib.load().sipf_save(self._h, str(path).encode()))

    @classmethod
    def load(cls, path, stream=None):
        """Context restored from a snapshot written by save()."""
        lib = _lib.load()
        self = cls.__new__(cls)
        h = ctypes.c_void_p()
        check(lib.sipf_load(str(path).encode(), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._stream = stream
        p = _lib.SipfParams()
        P = ctypes.c_int64()
        check(lib.sipf_get_params(h, ctypes.byref(p), ctypes.byref(P)))
        self.params = p
        self.P = P.value
        self.H = int(p.H)
        self.dim = _dim(p)
        self.dtype = _dtype(p)
        self.device = torch.device("cuda", torch.cuda.current_device())
        return self

    def use_graphs(self, enable=True):
        """Replay captured HIP graphs in run() (default) or enqueue every step."""
        check(_lib.load().sipf_use_graphs(self._h, 1 if enable else 0))

    def positivity_stats(self):
        """(particles switched to order 2, rounds) of the last positive deposit."""
        sw, r = ctypes.c_int64(), ctypes.c_int32()
        check(_lib.load().sipf_positivity_stats(self._h, ctypes.byref(sw), ctypes.byref(r)))
        return int(sw.value), int(r.value)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.load().sipf_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Independent SIPF-PIC instances advanced together (one persistent
    particle launch and one launch per FFT phase and grid size per step).

    instances: list of dicts with keys ``params`` (sipf_params fields),
    ``X0`` ((P_i, 3) positions).  All instances share precision and scheme.
    """

    def __init__(self, instances, stream=None):
        lib = _lib.load()
        n = len(instances)
        if n < 1:
            raise ValueError("a batch needs at least one instance")
        prm = (_lib.SipfParams * n)()
        Ps = (ctypes.c_int64 * n)()
        ptrs = (ctypes.c_void_p * n)()
        self.params, self.P, self.H = [], [], []
        self.dim = None
        keep = []
        for i, inst in enumerate(instances):
            p = _lib.default_params(**inst["params"])
            prm[i] = p
            self.params.append(p)
            dt = _dtype(p)
            X = inst["X0"]
            X = torch.as_tensor(np.asarray(X) if not torch.is_tensor(X) else X)
            X = X.to(device="cuda", dtype=dt).contiguous()
            if self.dim is None:
                self.dim = _dim(p)
            if X.ndim != 2 or X.shape[1] != _dim(p):
                raise ValueError(f"instance {i}: X0 must have shape (P, 3)")
            keep.append(X)
            Ps[i] = int(X.shape[0])
            ptrs[i] = X.data_ptr()
            self.P.append(int(X.shape[0]))
            self.H.append(int(p.H))
        self.dtype = _dtype(self.params[0])
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.n = n
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        check(lib.sipf_batch_init(n, prm, Ps, ptrs, 1, _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def run(self, nsteps):
        check(_lib.load().sipf_batch_run(self._h, int(nsteps)))

    def prepare_run(self, nsteps):
        """Capture every graph that run(nsteps) issued next would replay (runs nothing)."""
        check(_lib.load().sipf_batch_prepare_run(self._h, int(nsteps)))

    def use_graphs(self, enable=True):
        check(_lib.load().sipf_batch_use_graphs(self._h, 1 if enable else 0))

    def sync(self):
        check(_lib.load().sipf_batch_sync(self._h))

    def step_count(self, i):
        v = ctypes.c_int64()
        check(_lib.load().sipf_batch_get_step(self._h, int(i), ctypes.byref(v)))
        return v.value

    def positions(self, i):
        out = torch.empty((self.P[i], self.dim), dtype=self.dtype, device=self.device)
        check(_lib.load().sipf_batch_get_positions(self._h, int(i), ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def field(self, i, which):
        H = self.H[i]
        shp = _shapes(H, self.dim)
        codes = {"rho": (_lib.SIPF_FIELD_RHO, shp["rho"]), "grad": (_lib.SIPF_FIELD_GRAD, shp["grad"]),
                 "alpha": (_lib.SIPF_FIELD_ALPHA, shp["alpha"])}
        code, shape = codes[which]
        out = torch.empty(shape, dtype=self.dtype, device=self.device)
        check(_lib.load().sipf_batch_get_field(self._h, int(i), code, ctypes.c_void_p(out.data_ptr()), 1))
        return torch.view_as_complex(out) if which == "alpha" else out

    def diagnostics(self):
        """Diagnostics of every instance (sipf_batch_diagnostics): list of dicts."""
        d = (_lib.SipfDiag * self.n)()
        check(_lib.load().sipf_batch_diagnostics(self._h, d))
        return [x.as_dict() for x in d]

    def profile(self, enable=True):
        check(_lib.load().sipf_batch_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        n = len(_lib.PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        check(_lib.load().sipf_batch_profile_read(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_lib.PHASES)}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.load().sipf_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(X0, nsteps=8, stream=None, **params):
    """Run the library's tile / chunk / re-sort / particle-pass search (sipf_autotune) for
    positions X0 and parameters ``params``; returns (tuned params dict, ms/step)."""
    p = _lib.default_params(**params)
    X = torch.as_tensor(np.asarray(X0) if not torch.is_tensor(X0) else X0)
    X = X.to(device="cuda", dtype=_dtype(p)).contiguous()
    best = _lib.SipfParams()
    ms = ctypes.c_double()
    torch.cuda.synchronize()
    check(_lib.load().sipf_autotune(ctypes.byref(p), int(X.shape[0]), ctypes.c_void_p(X.data_ptr()), 1,
                                    int(nsteps), _stream_handle(stream), ctypes.byref(best), ctypes.byref(ms)))
    return ({"tile": best.tile, "chunk": best.chunk, "resort_every": best.resort_every,
             "particle_pass": best.particle_pass}, ms.value)


def dbg_philox(ctr, seed, precision="fp32"):
    """Raw Philox outputs and the six normals for counters ctr (n, 4) uint32."""
    ctr = torch.as_tensor(np.asarray(ctr, dtype=np.uint32).view(np.int32)).cuda().contiguous()
    n = ctr.shape[0]
    raw = torch.empty((n, 4), dtype=torch.int32, device=ctr.device)
    dt = torch.float32 if precision == "fp32" else torch.float64
    z = torch.empty((n, 6), dtype=dt, device=ctr.device)
    prec = _lib.SIPF_FP32 if precision == "fp32" else _lib.SIPF_FP64
    check(_lib.load().sipf_dbg_philox(int(seed), n, ctypes.c_void_p(ctr.data_ptr()), ctypes.c_void_p(raw.data_ptr()),
                                      ctypes.c_void_p(z.data_ptr()), prec, _stream_handle()))
    return raw.cpu().numpy().view(np.uint32), z


def dbg_cells(X, **params):
    p = _lib.default_params(**params)
    X = torch.as_tensor(X).to(device="cuda", dtype=_dtype(p)).contiguous()
    out = torch.empty((X.shape[0], 3), dtype=torch.int32, device=X.device)
    check(_lib.load().sipf_dbg_cells(ctypes.byref(p), X.shape[0], ctypes.c_void_p(X.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream_handle()))
    return out


def dbg_deposit(X, **params):
    p = _lib.default_params(**params)
    X = torch.as_tensor(X).to(device="cuda", dtype=_dtype(p)).contiguous()
    H = p.H
    out = torch.empty((H, H, H), dtype=_dtype(p), device=X.device)
    check(_lib.load().sipf_dbg_deposit(ctypes.byref(p), X.shape[0], ctypes.c_void_p(X.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream_handle()))
    return out


class Rollout(torch.autograd.Function):
    """phi^(N) = deposit of the positions after N SIPF-PIC steps from X0.

    Differentiable in X0, chi and mu along the fixed Philox noise path; the
    backward pass runs the library's adjoint (sipf_adjoint) with the incoming
    gradient as phi_bar, checkpointing positions every ``ckpt_every`` steps.
    ``params`` holds the other sipf_params fields.
    """

    @staticmethod
    def forward(ctx, X0, chi, mu, params, nsteps, ckpt_every=10):
        p = dict(params, chi=float(chi), mu=float(mu))
        sim = Sim(X0.detach(), **p)
        sim.run(int(nsteps))
        phi = sim.field("rho")
        sim.close()
        ctx.save_for_backward(X0)
        ctx.p = p
        ctx.nsteps = int(nsteps)
        ctx.ckpt = int(ckpt_every)
        ctx.chi_like = torch.as_tensor(chi)
        ctx.mu_like = torch.as_tensor(mu)
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        (X0,) = ctx.saved_tensors
        sim = Sim(X0.detach(), **ctx.p)
        _, dchi, dmu, dX0 = sim.adjoint(ctx.nsteps, ctx.ckpt, phi_bar=grad_phi)
        sim.close()
        gchi = torch.full_like(ctx.chi_like, dchi, dtype=torch.float64)
        gmu = torch.full_like(ctx.mu_like, dmu, dtype=torch.float64)
        return dX0.to(X0.dtype), gchi.to(ctx.chi_like.dtype), gmu.to(ctx.mu_like.dtype), None, None, None
