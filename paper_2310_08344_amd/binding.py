"""ctypes binding of the C ABI in ``include/lx.h`` (argument marshalling only).

Every step of the path runs in the HIP library ``_lx.so``; this module only
turns torch tensors into device pointers and host results into Python
values.  Loading fails loudly when the library has not been built: there is
no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lx.so")

LX_OK, LX_EINVAL, LX_ENOMEM, LX_ENOTCONV, LX_ENONFINITE, LX_EDEVICE = range(6)
LX_OP_DIFFADV2D, LX_OP_BURGERS2D, LX_OP_DIFFADV2D_UP3 = 1, 2, 3
LX_FP64, LX_FP32_SWEEP = 0, 1
LX_ROS_EULER = 2
LX_EXPRB32 = 32
LX_EXPRB42 = 42
LX_K_MAX = 4
LX_MAX_ITERS = 1000

STATUS_NAMES = {0: "ok", 1: "einval", 2: "enomem", 3: "notconv", 4: "nonfinite", 5: "edevice"}


class LxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Operator(C.Structure):
    _fields_ = [("kind", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("D", C.c_double),
                ("vx", C.c_double), ("vy", C.c_double), ("nu", C.c_double),
                ("prec", C.c_int)]


class LejaOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_iters", C.c_int),
                ("fp32_switch", C.c_double), ("substeps", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("n_apply", C.c_int), ("n_fp32", C.c_int),
                ("iters", C.c_int * LX_K_MAX), ("err", C.c_double * LX_K_MAX),
                ("pnorm", C.c_double * LX_K_MAX), ("rho_hat", C.c_double),
                ("plan_ms", C.c_double), ("loop_ms", C.c_double), ("sweep_ms", C.c_double),
                ("first_sweep_ms", C.c_double), ("bytes", C.c_double), ("n_launch", C.c_int),
                ("depth", C.c_int), ("step_err", C.c_double), ("substeps", C.c_int), ("marching", C.c_int),
                ("batch_graph", C.c_int)]

    def as_dict(self) -> dict:
        return {"status": self.status, "n_apply": self.n_apply, "n_fp32": self.n_fp32,
                "iters": list(self.iters), "err": list(self.err), "pnorm": list(self.pnorm),
                "rho_hat": self.rho_hat, "plan_ms": self.plan_ms, "loop_ms": self.loop_ms,
                "sweep_ms": self.sweep_ms, "first_sweep_ms": self.first_sweep_ms,
                "bytes": self.bytes, "n_launch": self.n_launch, "depth": self.depth,
                "step_err": self.step_err, "substeps": self.substeps, "marching": self.marching,
                "batch_graph": self.batch_graph}


class Instance(C.Structure):
    _fields_ = [("op", Operator), ("d_u", C.c_void_p), ("d_v", C.c_void_p), ("d_out", C.c_void_p),
                ("d_x0", C.c_void_p), ("l", C.c_int), ("h", C.c_double), ("c", C.c_double),
                ("gamma", C.c_double), ("budget", C.c_int)]


class InstanceResult(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("err", C.c_double), ("pnorm", C.c_double),
                ("rho_hat", C.c_double), ("c", C.c_double), ("gamma", C.c_double), ("fallback", C.c_int)]

    def as_dict(self) -> dict:
        return {"status": self.status, "iters": self.iters, "err": self.err, "pnorm": self.pnorm,
                "rho_hat": self.rho_hat, "c": self.c, "gamma": self.gamma, "fallback": bool(self.fallback)}


_P = C.c_void_p
_D = C.c_double
_I = C.c_int


def _signatures(lib: C.CDLL) -> None:
    lib.lx_create.argtypes = [C.POINTER(_P), C.c_size_t, _I, _P]
    lib.lx_create.restype = _I
    lib.lx_destroy.argtypes = [_P]
    lib.lx_destroy.restype = None
    lib.lx_set_stream.argtypes = [_P, _P]
    lib.lx_set_stream.restype = _I
    lib.lx_set_timing.argtypes = [_P, _I]
    lib.lx_set_timing.restype = _I
    lib.lx_last_error.argtypes = [_P]
    lib.lx_last_error.restype = C.c_char_p
    lib.lx_status_string.argtypes = [_I]
    lib.lx_status_string.restype = C.c_char_p
    lib.lx_get_stats.argtypes = [_P, C.POINTER(Stats)]
    lib.lx_get_stats.restype = _I
    lib.lx_spectrum.argtypes = [_P, C.POINTER(Operator), _P, _P, _I, _D,
                                C.POINTER(_D), C.POINTER(_D), C.POINTER(_D)]
    lib.lx_spectrum.restype = _I
    lib.lx_phi_leja.argtypes = [_P, C.POINTER(Operator), _P, _P, _I, C.POINTER(_I),
                                C.POINTER(_D), C.POINTER(_D), C.POINTER(_P), _D, _D, _D,
                                C.POINTER(LejaOpts), C.POINTER(_I), C.POINTER(_D)]
    lib.lx_phi_leja.restype = _I
    lib.lx_phi_leja_static.argtypes = [_P, C.POINTER(Operator), _P, _P, _I, C.POINTER(_I),
                                       C.POINTER(_D), C.POINTER(_D), C.POINTER(_P), _D, _D, _D,
                                       C.POINTER(LejaOpts), C.POINTER(_I), C.POINTER(_D)]
    lib.lx_phi_leja_static.restype = _I
    lib.lx_exprb_step.argtypes = [_P, C.POINTER(Operator), _I, _P, _P, _P, C.POINTER(_D), _D, _D, _D,
                                  C.POINTER(LejaOpts), C.POINTER(_I)]
    lib.lx_exprb_step.restype = _I
    lib.lx_linear_step.argtypes = [_P, C.POINTER(Operator), _P, _P, _P, _D, _D, _D, C.POINTER(LejaOpts),
                                   C.POINTER(_I)]
    lib.lx_linear_step.restype = _I
    lib.lx_phi_leja_batched.argtypes = [_P, _I, C.POINTER(Instance), _I, _D, C.POINTER(LejaOpts),
                                        C.POINTER(InstanceResult)]
    lib.lx_phi_leja_batched.restype = _I
    lib.lx_tune_batched.argtypes = [_P, _I, C.POINTER(Instance), _I, _D, C.POINTER(LejaOpts), _I, C.c_char_p,
                                    C.c_size_t]
    lib.lx_tune_batched.restype = _I
    lib.lx_set_batch_shape.argtypes = [_P, _I, C.POINTER(Instance), _I, _I, _I]
    lib.lx_set_batch_shape.restype = _I
    lib.lx_set_batch_graphs.argtypes = [_P, _I]
    lib.lx_set_batch_graphs.restype = _I
    lib.lx_predictor_create.argtypes = [_P, C.c_ulonglong, C.POINTER(_P)]
    lib.lx_predictor_create.restype = _I
    lib.lx_predictor_destroy.argtypes = [_P]
    lib.lx_predictor_destroy.restype = None
    lib.lx_predictor_state_size.argtypes = []
    lib.lx_predictor_state_size.restype = _I
    lib.lx_predictor_set_scaling.argtypes = [_P, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                             C.POINTER(C.c_float), C.POINTER(C.c_float)]
    lib.lx_predictor_set_scaling.restype = _I
    lib.lx_predictor_get_state.argtypes = [_P, C.POINTER(C.c_float)]
    lib.lx_predictor_get_state.restype = _I
    lib.lx_predictor_set_state.argtypes = [_P, C.POINTER(C.c_float)]
    lib.lx_predictor_set_state.restype = _I
    lib.lx_predictor_save.argtypes = [_P, C.c_char_p]
    lib.lx_predictor_save.restype = _I
    lib.lx_predictor_load.argtypes = [_P, C.c_char_p]
    lib.lx_predictor_load.restype = _I
    lib.lx_predictor_gradient.argtypes = [_P, _P, _P, _I, C.POINTER(C.c_float), C.POINTER(_D)]
    lib.lx_predictor_gradient.restype = _I
    lib.lx_predictor_train.argtypes = [_P, _P, _P, _I, _I, _I, C.c_float, C.c_ulonglong, C.POINTER(_I),
                                       C.POINTER(_D)]
    lib.lx_predictor_train.restype = _I
    lib.lx_predictor_infer.argtypes = [_P, _P, _I, _P]
    lib.lx_predictor_infer.restype = _I
    lib.lx_instance_features.argtypes = [_P, _I, C.POINTER(Instance), _P]
    lib.lx_instance_features.restype = _I
    lib.lx_phi_leja_learned.argtypes = [_P, _P, _I, C.POINTER(Instance), _D, _D, _I, _D, C.POINTER(LejaOpts),
                                        C.POINTER(InstanceResult), C.POINTER(_I)]
    lib.lx_phi_leja_learned.restype = _I
    lib.lx_tune.argtypes = [_P, C.POINTER(Operator), _I, _I, C.c_char_p, C.c_size_t]
    lib.lx_tune.restype = _I
    lib.lx_set_tile.argtypes = [_P, _I, _I, _I, _I, _I]
    lib.lx_set_tile.restype = _I
    lib.lx_set_depth.argtypes = [_P, _I, _I, _I]
    lib.lx_set_depth.restype = _I
    lib.lx_set_window_kernel.argtypes = [_P, _I, _I, _I]
    lib.lx_set_window_kernel.restype = _I
    lib.lx_bandwidth_probe.argtypes = [_P, _I, C.c_size_t, _I, C.POINTER(_D)]
    lib.lx_bandwidth_probe.restype = _I
    lib.lx_leja_points.argtypes = [_I, C.POINTER(_D)]
    lib.lx_leja_points.restype = _I
    lib.lx_phi_scalar.argtypes = [_I, _D]
    lib.lx_phi_scalar.restype = _D
    lib.lx_newton_coeffs.argtypes = [_I, _D, _D, _D, _D, _D, _I, C.POINTER(_D)]
    lib.lx_newton_coeffs.restype = _I


EXPORTED = ["lx_create", "lx_destroy", "lx_set_stream", "lx_set_timing", "lx_last_error",
            "lx_status_string", "lx_get_stats", "lx_spectrum", "lx_phi_leja", "lx_phi_leja_static", "lx_exprb_step", "lx_linear_step",
            "lx_phi_leja_batched", "lx_tune_batched", "lx_set_batch_shape", "lx_set_batch_graphs", "lx_tune", "lx_set_tile", "lx_set_depth", "lx_set_window_kernel", "lx_bandwidth_probe",
            "lx_predictor_create", "lx_predictor_destroy", "lx_predictor_state_size", "lx_predictor_set_scaling",
            "lx_predictor_get_state", "lx_predictor_set_state", "lx_predictor_save", "lx_predictor_load",
            "lx_predictor_gradient", "lx_predictor_train", "lx_predictor_infer", "lx_instance_features",
            "lx_phi_leja_learned",
            "lx_leja_points", "lx_phi_scalar", "lx_newton_coeffs"]


def make_operator(problem=None, *, kind=None, n=None, nx=None, ny=None, dx=None, dy=None, D=0.0,
                  vx=0.0, vy=0.0, nu=0.0, prec=LX_FP64) -> Operator:
    """lx_operator from a workload Problem or from keywords."""
    if problem is not None:
        kind = {"diffadv": LX_OP_DIFFADV2D, "diffadv3": LX_OP_DIFFADV2D_UP3,
                "burgers": LX_OP_BURGERS2D}[problem.kind]
        nx = ny = problem.n
        dx, dy = problem.dx, problem.dy
        D, vx, vy, nu = problem.D, problem.vx, problem.vy, problem.nu
    else:
        nx = nx if nx is not None else n
        ny = ny if ny is not None else n
        dx = dx if dx is not None else 1.0 / nx
        dy = dy if dy is not None else 1.0 / ny
    return Operator(int(kind), int(nx), int(ny), float(dx), float(dy), float(D), float(vx), float(vy),
                    float(nu), int(prec))


def _ptr(t) -> int:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("vectors must be contiguous float64 tensors on the GPU")
    return t.data_ptr()


@dataclass
class PhiResult:
    status: int
    iters: list
    err: list
    stats: dict


class Batch:
    """A prepared lx_instance array (Context.prepare) and the instance dicts
    whose tensors it points to."""

    def __init__(self, array, keep):
        self.array = array
        self.keep = keep

    def __len__(self):
        return len(self.keep)


class Context:
    """An lx_ctx: workspaces for grids of at most n_max points."""

    def __init__(self, lib: "Library", n_max: int, k_max: int = LX_K_MAX, stream=None):
        import torch
        self.lib = lib
        self._h = _P()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        st = lib.c.lx_create(C.byref(self._h), C.c_size_t(int(n_max)), int(k_max), _P(int(stream)))
        if st != LX_OK:
            raise LxError(st, "lx_create failed")
        self.n_max, self.k_max = int(n_max), int(k_max)
        import weakref
        self._predictors = weakref.WeakSet()

    def close(self) -> None:
        if self._h:
            # lx_destroy frees the context's predictors: their handles go first
            for p in list(self._predictors):
                p._h = _P()
            self.lib.c.lx_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int, allow=(LX_OK,)) -> int:
        if st not in allow:
            raise LxError(st, self.lib.c.lx_last_error(self._h).decode())
        return st

    def last_error(self) -> str:
        return self.lib.c.lx_last_error(self._h).decode()

    def set_timing(self, on: bool) -> None:
        self._check(self.lib.c.lx_set_timing(self._h, 1 if on else 0))

    def set_stream(self, stream) -> None:
        self._check(self.lib.c.lx_set_stream(self._h, _P(int(stream))))

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.c.lx_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def tune(self, op: Operator, K: int = 1, sweeps: int = 10) -> list:
        """Times the candidate launch shapes (lx_tune); returns
        [(depth, tx, ty, rows, vec, workgroups, microseconds per iteration), ...]
        with rows = ry (depth 1) or tile rows th (depth 2)."""
        buf = C.create_string_buffer(8192)
        self._check(self.lib.c.lx_tune(self._h, C.byref(op), int(K), int(sweeps), buf, C.c_size_t(8192)))
        rows = []
        for line in buf.value.decode().splitlines():
            d, tx, ty, ry, vec, nb, us = line.split()
            rows.append((int(d), int(tx), int(ty), int(ry), int(vec), int(nb), float(us)))
        return rows

    def set_tile(self, tx=0, ty=0, ry=0, vec=0, nb=0) -> None:
        self._check(self.lib.c.lx_set_tile(self._h, int(tx), int(ty), int(ry), int(vec), int(nb)))

    def set_depth(self, depth=0, th=0, nb=0) -> None:
        """Leja iterations per launch (lx_set_depth): 0 automatic, 1, 2, 3, 4, 6 or 8."""
        self._check(self.lib.c.lx_set_depth(self._h, int(depth), int(th), int(nb)))

    def set_window_kernel(self, kind=0, bands=0, nb=0) -> None:
        """Kernel of windows and power iteration (lx_set_window_kernel): 0
        automatic, 1 LDS tiles, 2 register marching."""
        self._check(self.lib.c.lx_set_window_kernel(self._h, int(kind), int(bands), int(nb)))

    def bandwidth_probe(self, kind: int, n: int, reps: int = 20) -> float:
        """GB/s of the copy (kind 0) or z = ax + by (kind 1) probe."""
        g = _D()
        self._check(self.lib.c.lx_bandwidth_probe(self._h, int(kind), C.c_size_t(int(n)), int(reps), C.byref(g)))
        return g.value

    def spectrum(self, op: Operator, u=None, x0=None, iters: int = 20, safety: float = 1.05,
                 raise_on_error: bool = True):
        """Returns (rho_hat, c, gamma) (lx_spectrum)."""
        rho, c, g = _D(), _D(), _D()
        st = self.lib.c.lx_spectrum(self._h, C.byref(op), _ptr(u), _ptr(x0), int(iters), float(safety),
                                    C.byref(rho), C.byref(c), C.byref(g))
        if raise_on_error:
            self._check(st)
        return rho.value, c.value, g.value

    def phi_leja(self, op: Operator, v, outs, ls, h, c, gamma, u=None, alphas=None, sigmas=None,
                 rtol=1e-8, atol=0.0, max_iters=500, fp32_switch=1e4, raise_on_error=True,
                 substeps=0, static=False) -> PhiResult:
        """outs[k] = sigma_k phi_{l_k}(alpha_k h A) v (lx_phi_leja); substeps 0 = automatic.
        static=True calls lx_phi_leja_static (the static device scratch; no allocation)."""
        K = len(outs)
        larr = (_I * K)(*[int(x) for x in ls])
        aarr = (_D * K)(*[float(x) for x in alphas]) if alphas is not None else None
        sarr = (_D * K)(*[float(x) for x in sigmas]) if sigmas is not None else None
        oarr = (_P * K)(*[_ptr(t) for t in outs])
        opts = LejaOpts(float(rtol), float(atol), int(max_iters), float(fp32_switch), int(substeps))
        it = (_I * K)()
        er = (_D * K)()
        fn = self.lib.c.lx_phi_leja_static if static else self.lib.c.lx_phi_leja
        st = fn(self._h, C.byref(op), _ptr(u), _ptr(v), K, larr, aarr, sarr, oarr, float(h), float(c), float(gamma),
                C.byref(opts), it, er)
        if raise_on_error:
            self._check(st, allow=(LX_OK, LX_ENOTCONV))
        return PhiResult(st, list(it), list(er), self.stats())

    def prepare(self, instances) -> "Batch":
        """The lx_instance array of a batch, built once and reusable: the
        dicts' tensors are kept alive with it."""
        return Batch(self._instances(instances), list(instances))

    @staticmethod
    def _instances(instances):
        if isinstance(instances, Batch):
            return instances.array
        n = len(instances)
        arr = (Instance * n)()
        for i, q in enumerate(instances):
            arr[i].op = q["op"]
            arr[i].d_u = _ptr(q.get("u"))
            arr[i].d_v = _ptr(q["v"])
            arr[i].d_out = _ptr(q["out"]) if q.get("out") is not None else None
            arr[i].d_x0 = _ptr(q.get("x0"))
            arr[i].l = int(q.get("l", 0))
            arr[i].h = float(q["h"])
            arr[i].c = float(q.get("c", 0.0))
            arr[i].gamma = float(q.get("gamma", 0.0))
            arr[i].budget = int(q.get("budget", 0))
        return arr

    def phi_leja_batched(self, instances, power_iters=0, safety=1.05, rtol=1e-8, atol=0.0, max_iters=500,
                         raise_on_error=True):
        """Batched phi actions (lx_phi_leja_batched).  instances: list of
        dicts with keys op, v, out and optionally u, x0, l (0), h, c, gamma,
        budget (0).  Returns (status, [result dict per instance])."""
        n = len(instances)
        arr = self._instances(instances)
        res = (InstanceResult * n)()
        opts = LejaOpts(float(rtol), float(atol), int(max_iters), 1e4)
        st = self.lib.c.lx_phi_leja_batched(self._h, n, arr, int(power_iters), float(safety), C.byref(opts), res)
        if raise_on_error:
            self._check(st, allow=(LX_OK, LX_ENOTCONV))
        return st, [r.as_dict() for r in res]

    def tune_batched(self, instances, power_iters=0, safety=1.05, rtol=1e-8, atol=0.0, max_iters=500,
                     repeats=3) -> list:
        """lx_tune_batched: runs the batch under every candidate shape and keeps
        the fastest for its class.  Returns [(depth, th, points_per_workgroup,
        median_ms), ...]."""
        n = len(instances)
        arr = self._instances(instances)
        opts = LejaOpts(float(rtol), float(atol), int(max_iters), 1e4)
        buf = C.create_string_buffer(4096)
        self._check(self.lib.c.lx_tune_batched(self._h, n, arr, int(power_iters), float(safety), C.byref(opts),
                                               int(repeats), buf, C.c_size_t(4096)))
        rows = []
        for line in buf.value.decode().splitlines():
            d, th, ppw, ms = line.split()
            rows.append((int(d), int(th), int(ppw), float(ms)))
        return rows

    def set_batch_shape(self, instances, depth=0, th=0, ppw=0) -> None:
        """lx_set_batch_shape for the class of this batch (all 0: forget it)."""
        self._check(self.lib.c.lx_set_batch_shape(self._h, len(instances), self._instances(instances), int(depth),
                                                  int(th), int(ppw)))

    def set_batch_graphs(self, on: bool) -> None:
        """lx_set_batch_graphs: capture and replay of batch pipelines."""
        self._check(self.lib.c.lx_set_batch_graphs(self._h, 1 if on else 0))

    def phi_leja_learned(self, instances, predictor, margin_log_rho, margin_log_sweeps, power_iters=20, safety=1.05,
                         rtol=1e-8, atol=0.0, max_iters=500, raise_on_error=True):
        """lx_phi_leja_learned: the predictor's bound and budget, plain-method
        fallback.  Returns (status, [result dict per instance], fallbacks)."""
        n = len(instances)
        arr = self._instances(instances)
        res = (InstanceResult * n)()
        opts = LejaOpts(float(rtol), float(atol), int(max_iters), 1e4)
        nf = _I()
        st = self.lib.c.lx_phi_leja_learned(self._h, predictor._h, n, arr, float(margin_log_rho),
                                            float(margin_log_sweeps), int(power_iters), float(safety),
                                            C.byref(opts), res, C.byref(nf))
        if raise_on_error:
            self._check(st, allow=(LX_OK, LX_ENOTCONV))
        return st, [r.as_dict() for r in res], nf.value

    def features(self, instances, out):
        """lx_instance_features: out is a float32 CUDA tensor [n, 8]."""
        import torch
        n = len(instances)
        if out.dtype != torch.float32 or not out.is_cuda or tuple(out.shape) != (n, 8) or not out.is_contiguous():
            raise ValueError("features need a contiguous float32 CUDA tensor of shape [n, 8]")
        self._check(self.lib.c.lx_instance_features(self._h, n, self._instances(instances), out.data_ptr()))
        return out

    def predictor(self, seed: int = 0) -> "Predictor":
        return Predictor(self, seed)

    def exprb_step(self, op: Operator, u, u_out, h, c, gamma, rtol=1e-8, atol=0.0, max_iters=500,
                   fp32_switch=1e4, scheme=LX_EXPRB42, raise_on_error=True, substeps=0, u_low=None) -> PhiResult:
        """lx_exprb_step.  iters: the step's phi actions in the order taken
        (Ros-Euler [phi_1]; EXPRB32 [phi_1, phi_3]; EXPRB42 [(3/4) phi_1,
        phi_1, phi_3]); err: [the embedded estimate] (EXPRB32; 0 otherwise);
        u_low receives EXPRB32's embedded second-order solution."""
        opts = LejaOpts(float(rtol), float(atol), int(max_iters), float(fp32_switch), int(substeps))
        it = (_I * 3)()
        e = _D(0.0)
        st = self.lib.c.lx_exprb_step(self._h, C.byref(op), int(scheme), _ptr(u), _ptr(u_out),
                                      _ptr(u_low) if u_low is not None else None, C.byref(e), float(h),
                                      float(c), float(gamma), C.byref(opts), it)
        if raise_on_error:
            self._check(st, allow=(LX_OK, LX_ENOTCONV))
        s = self.stats()
        n = {LX_ROS_EULER: 1, LX_EXPRB32: 2}.get(int(scheme), 3)
        return PhiResult(st, list(it)[:n], [e.value], s)


    def linear_step(self, op: Operator, u, u_out, h, c, gamma, source=None, rtol=1e-12, atol=0.0,
                    max_iters=500, fp32_switch=1e4, raise_on_error=True, substeps=0) -> PhiResult:
        """lx_linear_step: exp(hA)u, or u + h phi_1(hA)(Au + S) with a source."""
        opts = LejaOpts(float(rtol), float(atol), int(max_iters), float(fp32_switch), int(substeps))
        it = _I(0)
        st = self.lib.c.lx_linear_step(self._h, C.byref(op), _ptr(u), _ptr(source) if source is not None else None,
                                       _ptr(u_out), float(h), float(c), float(gamma), C.byref(opts), C.byref(it))
        if raise_on_error:
            self._check(st, allow=(LX_OK, LX_ENOTCONV))
        s = self.stats()
        return PhiResult(st, [it.value], s["err"][:1], s)


def _fptr(t, cols):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() \
            or t.dim() != 2 or t.shape[1] != cols:
        raise ValueError(f"expected a contiguous float32 CUDA tensor of shape [n, {cols}]")
    return t.data_ptr()


class Predictor:
    """lx_predictor: the spectral/budget MLP on a context's device."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        self.c = ctx.lib.c
        self._h = _P()
        ctx._check(self.c.lx_predictor_create(ctx._h, C.c_ulonglong(int(seed)), C.byref(self._h)))
        self.state_size = int(self.c.lx_predictor_state_size())
        ctx._predictors.add(self)

    def close(self):
        if self._h:
            self.c.lx_predictor_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scaling(self, mean_x, std_x, mean_y, std_y):
        f = lambda a, n: (C.c_float * n)(*[float(x) for x in a])
        self.ctx._check(self.c.lx_predictor_set_scaling(self._h, f(mean_x, 8), f(std_x, 8), f(mean_y, 2),
                                                        f(std_y, 2)))

    def get_state(self):
        import numpy as np
        buf = (C.c_float * self.state_size)()
        self.ctx._check(self.c.lx_predictor_get_state(self._h, buf))
        return np.frombuffer(buf, dtype=np.float32).copy()

    def set_state(self, state):
        import numpy as np
        a = np.ascontiguousarray(state, dtype=np.float32)
        if a.size != self.state_size:
            raise ValueError("state size mismatch")
        self.ctx._check(self.c.lx_predictor_set_state(self._h, a.ctypes.data_as(C.POINTER(C.c_float))))

    def save(self, path):
        self.ctx._check(self.c.lx_predictor_save(self._h, str(path).encode()))

    def load(self, path):
        self.ctx._check(self.c.lx_predictor_load(self._h, str(path).encode()))

    def gradient(self, X, Y):
        import numpy as np
        n = X.shape[0]
        g = (C.c_float * LX_MLP_PARAMS)()
        loss = _D()
        self.ctx._check(self.c.lx_predictor_gradient(self._h, _fptr(X, 8), _fptr(Y, 2), n, g, C.byref(loss)))
        return loss.value, np.frombuffer(g, dtype=np.float32).copy()

    def train(self, X, Y, steps, batch, lr, seed=0, order=None):
        n = X.shape[0]
        o = None
        if order is not None:
            o = (_I * len(order))(*[int(x) for x in order])
        loss = _D()
        self.ctx._check(self.c.lx_predictor_train(self._h, _fptr(X, 8), _fptr(Y, 2), n, int(steps), int(batch),
                                                  float(lr), C.c_ulonglong(int(seed)), o, C.byref(loss)))
        return loss.value

    def infer(self, X, out):
        self.ctx._check(self.c.lx_predictor_infer(self._h, _fptr(X, 8), X.shape[0], _fptr(out, 2)))
        return out


LX_MLP_PARAMS = 4866


class Library:
    """The loaded ``_lx.so``."""

    _instance = None

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} is missing "
                               "(run python -m paper_2310_08344_amd.build)")
        self.path = path
        # PyTorch ships its own HIP runtime under the same soname as the one
        # the library links; loading torch first makes both use that single
        # runtime (a second one would not know torch's streams)
        import torch  # noqa: F401
        self.c = C.CDLL(path)
        _signatures(self.c)

    @classmethod
    def load(cls) -> "Library":
        if cls._instance is None:
            cls._instance = cls()
        return cls._instance

    def context(self, n_max: int, k_max: int = LX_K_MAX, stream=None) -> Context:
        return Context(self, n_max, k_max, stream)

    # host-only planner
    def leja_points(self, M: int):
        import numpy as np
        out = (_D * M)()
        st = self.c.lx_leja_points(int(M), out)
        if st != LX_OK:
            raise LxError(st, "lx_leja_points")
        return np.array(out[:], dtype=np.float64)

    def newton_coeffs(self, l, h, c, gamma, M, alpha=1.0, sigma=1.0):
        import numpy as np
        out = (_D * M)()
        st = self.c.lx_newton_coeffs(int(l), float(alpha), float(sigma), float(h), float(c), float(gamma),
                                     int(M), out)
        if st != LX_OK:
            raise LxError(st, "lx_newton_coeffs")
        return np.array(out[:], dtype=np.float64)

    def phi_scalar(self, l: int, z: float) -> float:
        return float(self.c.lx_phi_scalar(int(l), float(z)))
