"""ctypes binding of libvegas_hip.so (include/vegas.h).

Argument marshalling only: every step of the iteration runs in the HIP
kernels of the library.  PyTorch supplies device memory (the workspace
tensor) and the stream.  There is no fallback: if the library is missing,
importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VEGAS_HIP_LIB") or os.path.join(_HERE, "libvegas_hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_2408_09229_amd/build.py`")

# torch first: its HIP runtime is then the one the library binds to, so
# that device memory and streams from torch are valid in the library
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

VEGAS_OK, VEGAS_EINVAL, VEGAS_ENOMEM, VEGAS_EDEVICE, VEGAS_ESTATE, VEGAS_ENONFINITE, VEGAS_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_FP32 = 0, 1
ACC_FP64, ACC_KAHAN, ACC_ORDERED = 0, 1, 2
BATCH_STREAMS, BATCH_PERSISTENT = 0, 1
STATIC_SCRATCH_BYTES = 64 << 20     # VEGAS_STATIC_SCRATCH_BYTES
_SCHEDULES = {"streams": BATCH_STREAMS, "persistent": BATCH_PERSISTENT}


class vegas_config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_intervals", C.c_int32), ("n_eval", C.c_int64),
                ("n_strat", C.c_int32), ("n_min", C.c_int32), ("alpha", C.c_double),
                ("beta", C.c_double), ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("precision", C.c_int32), ("accum", C.c_int32), ("adapt_map", C.c_int32),
                ("adapt_strat", C.c_int32), ("max_iter", C.c_int32)]


class vegas_integrand(C.Structure):
    _fields_ = [("family", C.c_int32), ("n_params", C.c_int32),
                ("params", C.POINTER(C.c_double)), ("lo", C.POINTER(C.c_double)),
                ("hi", C.POINTER(C.c_double))]


class vegas_estimate(C.Structure):
    _fields_ = [("integral", C.c_double), ("sigma2", C.c_double), ("chi2_dof", C.c_double),
                ("n_iter_combined", C.c_int32), ("n_iter_total", C.c_int32),
                ("n_eval_total", C.c_int64), ("n_nonfinite", C.c_int64)]


class vegas_info(C.Structure):
    _fields_ = [("n_strat", C.c_int64), ("n_cubes", C.c_int64), ("n_rest", C.c_int64),
                ("tile", C.c_int32), ("n_tiles", C.c_int32), ("n_workgroups", C.c_int32),
                ("lds_hist", C.c_int32), ("workspace_bytes", C.c_size_t)]


class vegas_flow_config(C.Structure):
    _fields_ = [("lr", C.c_float), ("train", C.c_int32), ("loss", C.c_int32), ("judge", C.c_int32),
                ("steps_per_iter", C.c_int32), ("control_period", C.c_int32), ("train_stride", C.c_int32),
                ("init_seed", C.c_uint64)]


class vegas_batch_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("per_lane", C.c_int32), ("item_samples", C.c_int64),
                ("n_items", C.c_int64), ("n_tiles", C.c_int64), ("n_workgroups", C.c_int32),
                ("tuned", C.c_int32), ("tune_ms", C.c_double), ("lds_bytes", C.c_size_t),
                ("workspace_bytes", C.c_size_t), ("n_eval_total", C.c_int64), ("n_cubes_total", C.c_int64),
                ("schedule", C.c_int32), ("n_streams", C.c_int32)]


_vp = C.c_void_p
_st = C.c_int
_DECL = {
    "vegas_workspace_size": (_st, [C.POINTER(vegas_config), C.POINTER(vegas_integrand), C.POINTER(C.c_size_t)]),
    "vegas_create": (_st, [C.POINTER(vegas_config), C.POINTER(vegas_integrand), _vp, C.c_size_t, _vp,
                           C.POINTER(_vp)]),
    "vegas_create_static": (_st, [C.POINTER(vegas_config), C.POINTER(vegas_integrand), _vp, C.POINTER(_vp)]),
    "vegas_create_user": (_st, [C.POINTER(vegas_config), C.POINTER(vegas_integrand), _vp, _vp, C.c_size_t, _vp,
                                C.POINTER(_vp)]),
    "vegas_user_compile": (_st, [C.c_char_p, C.c_int32, C.c_int32, C.POINTER(_vp)]),
    "vegas_user_check": (_st, [C.c_char_p, C.c_int32, C.c_int32]),
    "vegas_user_destroy": (None, [_vp]),
    "vegas_adapt": (_st, [_vp, C.c_int32]),
    "vegas_integrate": (_st, [_vp, C.c_int32]),
    "vegas_result": (_st, [_vp, C.POINTER(vegas_estimate)]),
    "vegas_destroy": (None, [_vp]),
    "vegas_get_info": (_st, [_vp, C.POINTER(vegas_info)]),
    "vegas_get_map": (_st, [_vp, _vp]),
    "vegas_set_map": (_st, [_vp, _vp]),
    "vegas_set_params": (_st, [_vp, _vp]),
    "vegas_set_adapt": (_st, [_vp, C.c_int32, C.c_int32]),
    "vegas_get_nh": (_st, [_vp, _vp]),
    "vegas_set_nh": (_st, [_vp, _vp]),
    "vegas_get_accumulators": (_st, [_vp, _vp, _vp, _vp]),
    "vegas_set_accumulators": (_st, [_vp, _vp, _vp, _vp]),
    "vegas_update": (_st, [_vp]),
    "vegas_get_iterations": (_st, [_vp, _vp, _vp, C.c_int32, C.POINTER(C.c_int32)]),
    "vegas_get_state": (_st, [_vp, _vp, C.POINTER(C.c_size_t)]),
    "vegas_set_state": (_st, [_vp, _vp, C.c_size_t]),
    "vegas_sample_probe": (_st, [_vp, C.c_uint32, C.c_uint64, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vegas_set_timing": (_st, [_vp, C.c_int32]),
    "vegas_get_timing": (_st, [_vp, _vp, C.POINTER(C.c_int32)]),
    "vegas_flow_n_params": (C.c_int32, []),
    "vegas_flow_workspace_size": (_st, [_vp, C.POINTER(C.c_size_t)]),
    "vegas_flow_attach": (_st, [_vp, C.POINTER(vegas_flow_config), _vp, _vp, C.c_size_t]),
    "vegas_flow_set_config": (_st, [_vp, C.POINTER(vegas_flow_config)]),
    "vegas_flow_enable": (_st, [_vp, C.c_int32]),
    "vegas_flow_get_kinds": (_st, [_vp, _vp, C.c_int32, C.POINTER(C.c_int32)]),
    "vegas_flow_set_timing": (_st, [_vp, C.c_int32]),
    "vegas_flow_get_timing": (_st, [_vp, _vp, C.POINTER(C.c_int32)]),
    "vegas_flow_get_grad_timing": (_st, [_vp, _vp, C.POINTER(C.c_int32)]),
    "vegas_flow_status": (_st, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "vegas_flow_get_params": (_st, [_vp, _vp]),
    "vegas_flow_set_params": (_st, [_vp, _vp]),
    "vegas_flow_get_samples": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "vegas_flow_grad": (_st, [_vp, _vp]),
    "vegas_flow_adam_step": (_st, [_vp, _vp]),
    "vegas_mfma_probe": (_st, [_vp, _vp, _vp]),
    "vegas_batch_workspace_size": (_st, [C.c_int32, _vp, _vp, C.c_int32, C.POINTER(C.c_size_t)]),
    "vegas_batch_create": (_st, [C.c_int32, _vp, _vp, _vp, C.c_size_t, _vp, C.c_int32, C.c_char_p,
                                 C.POINTER(_vp)]),
    "vegas_batch_destroy": (None, [_vp]),
    "vegas_batch_set_layout": (_st, [_vp, C.c_int32, C.c_int64]),
    "vegas_batch_set_streams": (_st, [_vp, C.c_int32]),
    "vegas_batch_adapt": (_st, [_vp, C.c_int32]),
    "vegas_batch_integrate": (_st, [_vp, C.c_int32]),
    "vegas_batch_results": (_st, [_vp, _vp]),
    "vegas_batch_get_iterations": (_st, [_vp, C.c_int32, _vp, _vp, C.c_int32, C.POINTER(C.c_int32)]),
    "vegas_batch_get_map": (_st, [_vp, C.c_int32, _vp]),
    "vegas_batch_get_nh": (_st, [_vp, C.c_int32, _vp]),
    "vegas_batch_get_info": (_st, [_vp, C.POINTER(vegas_batch_info)]),
    "vegas_batch_set_timing": (_st, [_vp, C.c_int32]),
    "vegas_batch_get_timing": (_st, [_vp, _vp, C.POINTER(C.c_int32)]),
    "vegas_status_string": (C.c_char_p, [_st]),
    "vegas_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _DECL.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn

EXPORTED = tuple(_DECL)


class VegasError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = _lib.vegas_last_error().decode()
        super().__init__(f"{what}: {_lib.vegas_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, what: str, allow=()):
    if status != VEGAS_OK and status not in allow:
        raise VegasError(status, what)
    return status


def _dptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def make_config(dim, n_intervals, n_eval, *, n_strat=0, n_min=2, alpha=0.5, beta=0.75, seed=0,
                instance=0, precision="f64", accum="fp64", adapt_map=True, adapt_strat=True,
                max_iter=0) -> vegas_config:
    return vegas_config(dim, n_intervals, n_eval, n_strat, n_min, alpha, beta, seed, instance,
                        PREC_FP64 if precision == "f64" else PREC_FP32,
                        {"fp64": ACC_FP64, "kahan": ACC_KAHAN, "ordered": ACC_ORDERED}[accum],
                        int(adapt_map), int(adapt_strat), max_iter)


class _Integrand:
    """Keeps the numpy arrays behind a vegas_integrand alive."""

    def __init__(self, family, params, lo=None, hi=None):
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.lo = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64)
        self.hi = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        self.s = vegas_integrand(family, self.params.size, self.params.ctypes.data_as(dp),
                                 None if self.lo is None else self.lo.ctypes.data_as(dp),
                                 None if self.hi is None else self.hi.ctypes.data_as(dp))


def workspace_size(cfg: vegas_config, family, params, lo=None, hi=None) -> int:
    it = _Integrand(family, params, lo, hi)
    n = C.c_size_t()
    check(vegas_workspace_size(C.byref(cfg), C.byref(it.s), C.byref(n)), "vegas_workspace_size")
    return n.value


class UserIntegrand:
    """An integrand compiled at run time (hipRTC) from device source that
    defines ``__device__ vegas_real vegas_user_f(const vegas_real* x, int dim,
    const double* params)`` (vegas_real: double for "f64", float for "f32")."""

    def __init__(self, source: str, dim: int, precision: str = "f64"):
        h = C.c_void_p()
        check(vegas_user_compile(source.encode(), dim, PREC_FP64 if precision == "f64" else PREC_FP32, C.byref(h)),
              "vegas_user_compile")
        self.h = h
        self.dim = dim

    @staticmethod
    def check(source: str, dim: int, precision: str = "f64"):
        """Compile for gfx950 without a device (raises VegasError with the
        compiler's log on failure)."""
        check(vegas_user_check(source.encode(), dim, PREC_FP64 if precision == "f64" else PREC_FP32),
              "vegas_user_check")

    def close(self):
        if getattr(self, "h", None):
            vegas_user_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


VEGAS_USER = 12


class Vegas:
    """One VEGAS+ problem on the current HIP device.

    ``Vegas(cfg, family, params)`` allocates the workspace as a torch uint8
    tensor and runs on torch's current stream (or ``stream``).  With
    ``static=True`` the context uses the library's own device array instead
    (vegas_create_static: no allocation; one such context per device at a
    time).
    """

    def __init__(self, cfg: vegas_config, family: int, params, lo=None, hi=None, *, stream=None,
                 device=None, static: bool = False, user: "UserIntegrand" = None):
        import torch
        self.cfg = cfg
        self.user = user          # kept alive with the context
        if user is not None:
            family = VEGAS_USER
        self._it = _Integrand(family, params, lo, hi)
        self.device = torch.device(device or "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        if static:
            self.ws = None
            check(vegas_create_static(C.byref(cfg), C.byref(self._it.s), C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h)), "vegas_create_static")
        else:
            n = C.c_size_t()
            check(vegas_workspace_size(C.byref(cfg), C.byref(self._it.s), C.byref(n)), "vegas_workspace_size")
            self.ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
            if user is not None:
                check(vegas_create_user(C.byref(cfg), C.byref(self._it.s), user.h, C.c_void_p(self.ws.data_ptr()),
                                        n.value, C.c_void_p(self.stream.cuda_stream), C.byref(h)), "vegas_create_user")
            else:
                check(vegas_create(C.byref(cfg), C.byref(self._it.s), C.c_void_p(self.ws.data_ptr()), n.value,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h)), "vegas_create")
        self.h = h
        self.info = vegas_info()
        check(vegas_get_info(self.h, C.byref(self.info)), "vegas_get_info")

    def close(self):
        if getattr(self, "h", None):
            vegas_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # -- the iteration ----------------------------------------------------
    def adapt(self, n: int):
        check(vegas_adapt(self.h, n), "vegas_adapt")

    def integrate(self, n: int):
        check(vegas_integrate(self.h, n), "vegas_integrate")

    def result(self, allow_nonfinite=False) -> vegas_estimate:
        r = vegas_estimate()
        check(vegas_result(self.h, C.byref(r)), "vegas_result",
              allow=(VEGAS_ENONFINITE,) if allow_nonfinite else ())
        return r

    def update(self):
        check(vegas_update(self.h), "vegas_update")

    # -- hooks --------------------------------------------------------------
    @property
    def dim(self):
        return self.cfg.dim

    @property
    def n_g(self):
        return self.cfg.n_intervals

    def get_map(self):
        g = np.zeros((self.dim, self.n_g + 1))
        check(vegas_get_map(self.h, _dptr(g)), "vegas_get_map")
        return g

    def set_map(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        check(vegas_set_map(self.h, _dptr(g)), "vegas_set_map")

    def set_adapt(self, adapt_map: bool = True, adapt_strat: bool = True):
        check(vegas_set_adapt(self.h, int(adapt_map), int(adapt_strat)), "vegas_set_adapt")

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float64)
        check(vegas_set_params(self.h, _dptr(p)), "vegas_set_params")

    def get_nh(self):
        nh = np.zeros(self.info.n_cubes, np.uint32)
        check(vegas_get_nh(self.h, _dptr(nh)), "vegas_get_nh")
        return nh

    def set_nh(self, nh):
        nh = np.ascontiguousarray(nh, dtype=np.uint32)
        check(vegas_set_nh(self.h, _dptr(nh)), "vegas_set_nh")

    def get_accumulators(self):
        H = np.zeros((self.dim, self.n_g))
        Cn = np.zeros((self.dim, self.n_g))
        v = np.zeros(self.info.n_cubes)
        check(vegas_get_accumulators(self.h, _dptr(H), _dptr(Cn), _dptr(v)), "vegas_get_accumulators")
        return H, Cn, v

    def set_accumulators(self, H, Cn, v):
        H = np.ascontiguousarray(H, dtype=np.float64)
        Cn = np.ascontiguousarray(Cn, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        check(vegas_set_accumulators(self.h, _dptr(H), _dptr(Cn), _dptr(v)), "vegas_set_accumulators")

    def get_iterations(self):
        n = C.c_int32()
        cap = self.cfg.max_iter or 4096
        I = np.zeros(cap)
        s2 = np.zeros(cap)
        check(vegas_get_iterations(self.h, _dptr(I), _dptr(s2), cap, C.byref(n)), "vegas_get_iterations")
        return I[:n.value].copy(), s2[:n.value].copy()

    def get_state(self) -> bytes:
        n = C.c_size_t()
        check(vegas_get_state(self.h, None, C.byref(n)), "vegas_get_state")
        buf = (C.c_char * n.value)()
        check(vegas_get_state(self.h, buf, C.byref(n)), "vegas_get_state")
        return bytes(buf)

    def set_state(self, b: bytes):
        buf = (C.c_char * len(b)).from_buffer_copy(b)
        check(vegas_set_state(self.h, buf, len(b)), "vegas_set_state")

    def set_timing(self, on: bool):
        check(vegas_set_timing(self.h, int(on)), "vegas_set_timing")

    def get_timing(self):
        """(ms per phase [fill, fixup+estimate, allocation, map], iterations)."""
        ms = np.zeros(4)
        n = C.c_int32()
        check(vegas_get_timing(self.h, _dptr(ms), C.byref(n)), "vegas_get_timing")
        return ms, n.value

    # -- learned warp -------------------------------------------------------
    @staticmethod
    def _flow_config(lr, train, loss, judge, steps_per_iter, control_period, train_stride, init_seed):
        j = {False: 0, True: 1, 0: 0, 1: 1, 2: 2, "guard": 1, "cost": 2}[judge]
        return vegas_flow_config(lr, int(train), {"variance": 0, "kl": 1}[loss], j, steps_per_iter,
                                 control_period, train_stride, init_seed)

    def attach_flow(self, params=None, lr: float = 1e-4, train: bool = False, loss: str = "variance",
                    judge=0, steps_per_iter: int = 1, control_period: int = 16, train_stride: int = 1,
                    init_seed: int = 0):
        """Attach a coupling-flow warp: initial FP32 parameters ``params``, or
        None for the library's own seeded starting weights (identity warp).
        ``judge``: 0 / False none, 1 / True / "guard", 2 / "cost"."""
        import torch
        n = C.c_size_t()
        check(vegas_flow_workspace_size(self.h, C.byref(n)), "vegas_flow_workspace_size")
        self.fws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        p = None
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.size != vegas_flow_n_params():
                raise ValueError("wrong number of flow parameters")
        self.fcfg = self._flow_config(lr, train, loss, judge, steps_per_iter, control_period, train_stride,
                                      init_seed)
        check(vegas_flow_attach(self.h, C.byref(self.fcfg), _dptr(p), C.c_void_p(self.fws.data_ptr()), n.value),
              "vegas_flow_attach")

    def set_flow_config(self, lr: float = 1e-4, train: bool = False, loss: str = "variance", judge=0,
                        steps_per_iter: int = 1, control_period: int = 16, train_stride: int = 1):
        self.fcfg = self._flow_config(lr, train, loss, judge, steps_per_iter, control_period, train_stride,
                                      self.fcfg.init_seed)
        check(vegas_flow_set_config(self.h, C.byref(self.fcfg)), "vegas_flow_set_config")

    def set_flow_timing(self, on: bool):
        check(vegas_flow_set_timing(self.h, int(on)), "vegas_flow_set_timing")

    def flow_timing(self):
        """Per warped iteration, ms of the sampling pass and of the training;
        per launch, ms of the gradient kernel."""
        ms = np.zeros(2)
        n = C.c_int32()
        check(vegas_flow_get_timing(self.h, _dptr(ms), C.byref(n)), "vegas_flow_get_timing")
        k = max(n.value, 1)
        g = np.zeros(1)
        ng = C.c_int32()
        check(vegas_flow_get_grad_timing(self.h, _dptr(g), C.byref(ng)), "vegas_flow_get_grad_timing")
        return {"sample_ms": ms[0] / k if n.value else None, "train_ms": ms[1] / k if n.value else None,
                "n": n.value, "grad_launch_ms": g[0] / ng.value if ng.value else None, "grad_launches": ng.value}

    def flow_kinds(self):
        """Per iteration: 0 plain, 1 through the warp, 2 plain control of the judge."""
        n = C.c_int32()
        cap = self.cfg.max_iter or 4096
        k = np.zeros(cap, np.int32)
        check(vegas_flow_get_kinds(self.h, _dptr(k), cap, C.byref(n)), "vegas_flow_get_kinds")
        return k[:n.value].copy()

    def enable_flow(self, on: bool = True):
        check(vegas_flow_enable(self.h, int(on)), "vegas_flow_enable")

    def flow_status(self):
        """(enabled, warped iterations kept, rejected) as judged."""
        on, a, r = C.c_int32(), C.c_int32(), C.c_int32()
        check(vegas_flow_status(self.h, C.byref(on), C.byref(a), C.byref(r)), "vegas_flow_status")
        return bool(on.value), a.value, r.value

    def flow_params(self):
        p = np.zeros(vegas_flow_n_params(), np.float32)
        check(vegas_flow_get_params(self.h, _dptr(p)), "vegas_flow_get_params")
        return p

    def set_flow_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        check(vegas_flow_set_params(self.h, _dptr(p)), "vegas_flow_set_params")

    def flow_grad(self):
        """Gradient of the warp's loss on the last warped iteration's samples."""
        g = np.zeros(vegas_flow_n_params(), np.float32)
        check(vegas_flow_grad(self.h, _dptr(g)), "vegas_flow_grad")
        return g

    def flow_adam_step(self, grad):
        """One Adam step of the warp on a given gradient (test hook)."""
        g = np.ascontiguousarray(grad, dtype=np.float32)
        check(vegas_flow_adam_step(self.h, _dptr(g)), "vegas_flow_adam_step")

    def flow_samples(self, with_z: bool = False):
        """(w [N][16], log J_F [N], omega [N]) of the last warped iteration,
        and the final Gaussian coordinates z_4 [N][16] with with_z."""
        n = self.cfg.n_eval
        w = np.zeros((n, 16), np.float32)
        lj = np.zeros(n, np.float32)
        om = np.zeros(n, np.float32)
        z = np.zeros((n, 16), np.float32) if with_z else None
        check(vegas_flow_get_samples(self.h, _dptr(w), _dptr(lj), _dptr(om), _dptr(z)), "vegas_flow_get_samples")
        return (w, lj, om, z) if with_z else (w, lj, om)

    def probe(self, t: int, k0: int, n: int):
        """Per-sample path for samples k0..k0+n-1 of iteration t (torch tensors)."""
        import torch
        D = self.dim
        dev = self.device
        out = dict(cube=torch.empty(n, dtype=torch.int32, device=dev),
                   bins=torch.empty(n * D, dtype=torch.int32, device=dev),
                   delta=torch.empty(n * D, dtype=torch.float64, device=dev),
                   x=torch.empty(n * D, dtype=torch.float64, device=dev),
                   jac=torch.empty(n, dtype=torch.float64, device=dev),
                   f=torch.empty(n, dtype=torch.float64, device=dev))
        p = {k: C.c_void_p(v.data_ptr()) for k, v in out.items()}
        check(vegas_sample_probe(self.h, t, k0, n, p["cube"], p["bins"], p["delta"], p["x"], p["jac"], p["f"]),
              "vegas_sample_probe")
        self.stream.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["cube"] = res["cube"].view(np.uint32)
        res["bins"] = res["bins"].view(np.uint32).reshape(n, D)
        res["delta"] = res["delta"].reshape(n, D)
        res["x"] = res["x"].reshape(n, D)
        return res


class _BatchSpec:
    """Host arrays of n configs and integrands (kept alive for the calls)."""

    def __init__(self, cfgs, integrands):
        n = len(cfgs)
        if n != len(integrands):
            raise ValueError("one integrand per config")
        self.its = [_Integrand(*spec) for spec in integrands]
        self.cfgs = (vegas_config * n)(*cfgs)
        self.fs = (vegas_integrand * n)(*[it.s for it in self.its])
        self.n = n


def batch_workspace_size(cfgs, integrands, schedule: str = "streams") -> int:
    sp = _BatchSpec(cfgs, integrands)
    n = C.c_size_t()
    check(vegas_batch_workspace_size(sp.n, sp.cfgs, sp.fs, _SCHEDULES[schedule], C.byref(n)),
          "vegas_batch_workspace_size")
    return n.value


class VegasBatch:
    """n independent VEGAS+ problems advanced together on the current device.

    ``cfgs`` is a list of vegas_config, ``integrands`` a list of
    (family, params[, lo, hi]) tuples.  ``schedule``: "streams" (one
    context per problem over a few streams) or "persistent" (switched off in
    the library).  ``tune_cache``: path of the autotuner's text cache, or
    None for the default schedule.
    """

    def __init__(self, cfgs, integrands, *, schedule="streams", tune_cache=None, stream=None, device=None):
        import torch
        self._spec = _BatchSpec(cfgs, integrands)
        self.n = self._spec.n
        self.cfgs = list(cfgs)
        self.schedule = _SCHEDULES[schedule]
        nb = C.c_size_t()
        check(vegas_batch_workspace_size(self.n, self._spec.cfgs, self._spec.fs, self.schedule, C.byref(nb)),
              "vegas_batch_workspace_size")
        self.device = torch.device(device or "cuda")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        check(vegas_batch_create(self.n, self._spec.cfgs, self._spec.fs, C.c_void_p(self.ws.data_ptr()), nb.value,
                                 C.c_void_p(self.stream.cuda_stream), self.schedule,
                                 None if tune_cache is None else os.fsencode(tune_cache), C.byref(h)),
              "vegas_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            vegas_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def info(self) -> vegas_batch_info:
        r = vegas_batch_info()
        check(vegas_batch_get_info(self.h, C.byref(r)), "vegas_batch_get_info")
        return r

    def set_layout(self, per_lane: int, item_samples: int):
        check(vegas_batch_set_layout(self.h, per_lane, item_samples), "vegas_batch_set_layout")

    def set_streams(self, n_streams: int):
        check(vegas_batch_set_streams(self.h, n_streams), "vegas_batch_set_streams")

    def adapt(self, n: int):
        check(vegas_batch_adapt(self.h, n), "vegas_batch_adapt")

    def integrate(self, n: int):
        check(vegas_batch_integrate(self.h, n), "vegas_batch_integrate")

    def results(self, allow_nonfinite=False):
        """Structured numpy array of the n combined estimates."""
        out = (vegas_estimate * self.n)()
        check(vegas_batch_results(self.h, out), "vegas_batch_results",
              allow=(VEGAS_ENONFINITE,) if allow_nonfinite else ())
        return np.ctypeslib.as_array(out).copy()

    def get_iterations(self, i: int):
        cap = 4096
        I = np.zeros(cap)
        s2 = np.zeros(cap)
        n = C.c_int32()
        check(vegas_batch_get_iterations(self.h, i, _dptr(I), _dptr(s2), cap, C.byref(n)),
              "vegas_batch_get_iterations")
        m = min(n.value, cap)
        return I[:m].copy(), s2[:m].copy()

    def get_map(self, i: int):
        c = self.cfgs[i]
        g = np.zeros((c.dim, c.n_intervals + 1))
        check(vegas_batch_get_map(self.h, i, _dptr(g)), "vegas_batch_get_map")
        return g

    def get_nh(self, i: int, n_cubes: int):
        nh = np.zeros(n_cubes, np.uint32)
        check(vegas_batch_get_nh(self.h, i, _dptr(nh)), "vegas_batch_get_nh")
        return nh

    def set_timing(self, on: bool):
        check(vegas_batch_set_timing(self.h, int(on)), "vegas_batch_set_timing")

    def get_timing(self):
        ms = np.zeros(4)
        n = C.c_int32()
        check(vegas_batch_get_timing(self.h, _dptr(ms), C.byref(n)), "vegas_batch_get_timing")
        return ms, n.value


def mfma_probe(A, B):
    """D = bf16(A) bf16(B) by one 32x32x16 BF16 MFMA on the current device."""
    import torch
    a = torch.tensor(np.ascontiguousarray(A, np.float32), device="cuda")
    b = torch.tensor(np.ascontiguousarray(B, np.float32), device="cuda")
    d = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    check(vegas_mfma_probe(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_void_p(d.data_ptr())),
          "vegas_mfma_probe")
    return d.cpu().numpy()
