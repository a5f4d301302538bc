"""Python binding of libhsd (argument marshalling only; every step of the
computation runs in the HIP kernels behind the C ABI of include/hsd.h)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


class HsdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hsd error {L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int) -> int:
    if status < 0:
        msg = L.load().hsd_last_error().decode(errors="replace")
        raise HsdError(status, msg)
    return status


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _host_f64(a, shape_last=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape_last is not None:
        a = a.reshape(-1, shape_last)
    return a


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32)).reshape(-1, 3)


_FORMS = {"fp64": L.FORM_FP64, "mixed": L.FORM_MIXED}
_METHODS = {"direct": L.METHOD_DIRECT, "nufft3": L.METHOD_NUFFT3}
_TRI_RULES = {"dunavant7": L.TRI_DUNAVANT7, "gl8x8": L.TRI_GL8X8}


@dataclass
class Params:
    """Per-call parameters (hsd_params)."""
    s: float = 1.0
    form: str = "fp64"
    method: str = "direct"
    taylor_tau: float = 1e-2
    tri_rule: str = "dunavant7"
    nufft_tol: float = 1e-9
    nufft_width: int = 0
    nufft_sigma: float = 2.0
    k_splits: int = 0
    # kappa of the weight (1+(|xi|/kappa)^2)^-s; 2 pi gives the paper's
    # exp(-2 pi i eta.x) convention for nodes xi = 2 pi eta (section 2.1)
    freq_unit: float = 1.0

    def to_c(self) -> L.Params:
        p = L.Params()
        L.load().hsd_params_default(C.byref(p))
        p.s = float(self.s)
        p.form = _FORMS[self.form]
        p.method = _METHODS[self.method]
        p.taylor_tau = float(self.taylor_tau)
        p.tri_rule = _TRI_RULES[self.tri_rule]
        p.nufft_tol = float(self.nufft_tol)
        p.nufft_width = int(self.nufft_width)
        p.nufft_sigma = float(self.nufft_sigma)
        p.k_splits = int(self.k_splits)
        p.freq_unit = float(self.freq_unit)
        return p


@dataclass
class Result:
    d2: float
    rel_err_stated: float
    pairs: float
    device_ms: float
    transform_ms: float

    @staticmethod
    def from_c(r: L.Result) -> "Result":
        return Result(r.d2, r.rel_err_stated, r.pairs, r.device_ms, r.transform_ms)


class Context:
    """A device context (hsd_init).  Binds torch's current stream if torch
    is available and a GPU is present."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, bind_torch_stream: bool = True):
        self._lib = L.load()
        h = C.c_void_p()
        _check(self._lib.hsd_init(int(device), int(budget_bytes), C.byref(h)))
        self.handle = h
        self.device = device
        if bind_torch_stream:
            try:
                import torch
                if torch.cuda.is_available():
                    self.set_stream(torch.cuda.current_stream(device).cuda_stream)
            except ImportError:
                pass

    def set_stream(self, stream_ptr) -> None:
        _check(self._lib.hsd_ctx_set_stream(self.handle, C.c_void_p(int(stream_ptr) if stream_ptr else 0)))

    def bytes_in_use(self) -> int:
        return int(self._lib.hsd_ctx_bytes_in_use(self.handle))

    def set_stage_timing(self, enable: bool = True) -> None:
        """Record the NUFFT path's stage times (hsd_ctx_set_stage_timing)."""
        _check(self._lib.hsd_ctx_set_stage_timing(self.handle, 1 if enable else 0))

    def nufft_stage_stats(self) -> dict:
        """{stage: (ms, algorithmic bytes)} of the last timed NUFFT transform."""
        ms = (C.c_double * 5)()
        by = (C.c_double * 5)()
        _check(self._lib.hsd_nufft_stage_stats(self.handle, ms, by))
        names = ("points_sort", "spread", "predeconv", "fft", "readout")
        return {n: (ms[i], by[i]) for i, n in enumerate(names)}

    def close(self) -> None:
        if self.handle:
            self._lib.hsd_finalize(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Mesh:
    """A device-resident triangle mesh (hsd_create_mesh).  verts [nv,3]
    float64 and tris [nt,3] int32, numpy arrays or torch tensors (device
    tensors are read in place)."""

    def __init__(self, ctx: Context, verts, tris):
        self.ctx = ctx
        lib = ctx._lib
        h = C.c_void_p()
        if _is_torch(verts) and verts.is_cuda:
            import torch
            v = verts.detach().to(torch.float64).contiguous()
            t = tris.to(device=v.device, dtype=torch.int32).contiguous()
            _check(lib.hsd_create_mesh(ctx.handle, C.c_void_p(v.data_ptr()), v.shape[0],
                                       C.c_void_p(t.data_ptr()), t.shape[0], L.MEM_DEVICE, C.byref(h)))
        else:
            if _is_torch(verts):
                verts = verts.detach().cpu().numpy()
            if _is_torch(tris):
                tris = tris.cpu().numpy()
            v = _host_f64(verts, 3)
            t = _host_i32(tris)
            _check(lib.hsd_create_mesh(ctx.handle, v.ctypes.data_as(C.c_void_p), len(v),
                                       t.ctypes.data_as(C.c_void_p), len(t), L.MEM_HOST, C.byref(h)))
        self.handle = h

    @property
    def num_triangles(self) -> int:
        return int(self.ctx._lib.hsd_mesh_num_triangles(self.handle))

    @property
    def num_vertices(self) -> int:
        return int(self.ctx._lib.hsd_mesh_num_vertices(self.handle))

    def close(self):
        if self.handle:
            self.ctx._lib.hsd_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PointMeasure(Mesh):
    """A weighted point measure sum_q c_q delta(x - y_q) (hsd_create_point_measure),
    e.g. a quadrature of a smooth parametrised surface; usable wherever a Mesh
    is (except as the differentiated measure of distance_grad).  points [n,3]
    and weights [n] float64, numpy arrays or torch tensors (device tensors are
    read in place)."""

    def __init__(self, ctx: Context, points, weights):
        self.ctx = ctx
        lib = ctx._lib
        h = C.c_void_p()
        if _is_torch(points) and points.is_cuda:
            import torch
            x = points.detach().to(torch.float64).contiguous()
            w = weights.detach().to(device=x.device, dtype=torch.float64).contiguous()
            _check(lib.hsd_create_point_measure(ctx.handle, C.c_void_p(x.data_ptr()), C.c_void_p(w.data_ptr()),
                                                x.shape[0], L.MEM_DEVICE, C.byref(h)))
        else:
            if _is_torch(points):
                points = points.detach().cpu().numpy()
            if _is_torch(weights):
                weights = weights.detach().cpu().numpy()
            x = _host_f64(points, 3)
            w = _host_f64(weights).ravel()
            if len(w) != len(x):
                raise HsdError(L.HSD_EINVAL, f"{len(x)} points but {len(w)} weights")
            _check(lib.hsd_create_point_measure(ctx.handle, x.ctypes.data_as(C.c_void_p),
                                                w.ctypes.data_as(C.c_void_p), len(x), L.MEM_HOST, C.byref(h)))
        self.handle = h


class SurfaceMeasure(Mesh):
    """A built-in smooth parametrised surface as a quadrature point measure
    (hsd_create_surface_measure): ``SurfaceMeasure.ellipsoid`` and
    ``SurfaceMeasure.torus``."""

    def __init__(self, ctx: Context, desc: L.SurfaceDesc):
        self.ctx = ctx
        h = C.c_void_p()
        _check(ctx._lib.hsd_create_surface_measure(ctx.handle, C.byref(desc), C.byref(h)))
        self.handle = h

    @classmethod
    def ellipsoid(cls, ctx, a=1.0, b=1.0, c=1.0, n_u=64, n_v=128, center=(0.0, 0.0, 0.0)):
        d = L.SurfaceDesc()
        d.kind, d.n_u, d.n_v = L.SURFACE_ELLIPSOID, int(n_u), int(n_v)
        d.a, d.b, d.c = float(a), float(b), float(c)
        d.center[:] = [float(x) for x in center]
        return cls(ctx, d)

    @classmethod
    def torus(cls, ctx, R=2.0, r=0.5, n_u=128, n_v=64, center=(0.0, 0.0, 0.0)):
        d = L.SurfaceDesc()
        d.kind, d.n_u, d.n_v = L.SURFACE_TORUS, int(n_u), int(n_v)
        d.a, d.b = float(R), float(r)
        d.center[:] = [float(x) for x in center]
        return cls(ctx, d)


class Rule:
    """A device-resident frequency quadrature (hsd_freq_rule)."""

    def __init__(self, ctx: Context, desc: L.RuleDesc, keep=()):
        self.ctx = ctx
        h = C.c_void_p()
        _check(ctx._lib.hsd_freq_rule(ctx.handle, C.byref(desc), C.byref(h)))
        self.handle = h
        self.kind = desc.kind
        self.desc = {f: getattr(desc, f) for f, _ in L.RuleDesc._fields_ if f not in ("nodes", "weights")}

    @classmethod
    def spherical_product(cls, ctx, r_max, n_panels, n_per_panel, n_cos, n_phi) -> "Rule":
        d = L.RuleDesc()
        d.kind = L.RULE_SPHERICAL_PRODUCT
        d.r_max, d.n_panels, d.n_per_panel, d.n_cos, d.n_phi = float(r_max), n_panels, n_per_panel, n_cos, n_phi
        return cls(ctx, d)

    @classmethod
    def explicit(cls, ctx, nodes, weights) -> "Rule":
        x = _host_f64(nodes, 3)
        w = _host_f64(weights).ravel()
        d = L.RuleDesc()
        d.kind = L.RULE_EXPLICIT
        d.nodes = x.ctypes.data_as(L.dp)
        d.weights = w.ctypes.data_as(L.dp)
        d.n_nodes = len(x)
        return cls(ctx, d)

    @classmethod
    def cube_trapezoid(cls, ctx, xi_max, M) -> "Rule":
        d = L.RuleDesc()
        d.kind = L.RULE_CUBE_TRAPEZOID
        d.xi_max, d.M = float(xi_max), int(M)
        return cls(ctx, d)

    def __len__(self) -> int:
        return int(self.ctx._lib.hsd_rule_num_nodes(self.handle))

    def nodes(self):
        n = len(self)
        x = np.empty((n, 3))
        w = np.empty(n)
        _check(self.ctx._lib.hsd_rule_nodes(self.handle, x.ctypes.data_as(L.dp), w.ctypes.data_as(L.dp)))
        return x, w

    def close(self):
        if self.handle:
            self.ctx._lib.hsd_rule_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def distance(ctx: Context, mu: Mesh, nu: Mesh | None, rule: Rule, params: Params | None = None) -> Result:
    """Squared H^-s distance (hsd_distance); nu None is the unit sphere."""
    p = (params or Params()).to_c()
    r = L.Result()
    _check(ctx._lib.hsd_distance(ctx.handle, mu.handle, nu.handle if nu is not None else None,
                                 rule.handle, C.byref(p), C.byref(r)))
    return Result.from_c(r)


def distance_noalloc(ctx: Context, mu: Mesh, nu: Mesh | None, rule: Rule,
                     params: Params | None = None) -> Result:
    """Squared distance without any device allocation (hsd_distance_noalloc):
    the library's fixed per-GPU scratch array holds every per-call buffer;
    direct method only."""
    p = (params or Params()).to_c()
    r = L.Result()
    _check(ctx._lib.hsd_distance_noalloc(ctx.handle, mu.handle, nu.handle if nu is not None else None,
                                         rule.handle, C.byref(p), C.byref(r)))
    return Result.from_c(r)


def distance_grad(ctx: Context, mu: Mesh, nu: Mesh | None, rule: Rule, params: Params | None = None,
                  out=None):
    """(Result, grad[nv,3]) (hsd_distance_grad).  ``out`` may be a device
    torch tensor [nv,3] float64 (written on the bound stream)."""
    p = (params or Params()).to_c()
    r = L.Result()
    if out is not None and _is_torch(out) and out.is_cuda:
        _check(ctx._lib.hsd_distance_grad(ctx.handle, mu.handle, nu.handle if nu is not None else None,
                                          rule.handle, C.byref(p), C.c_void_p(out.data_ptr()),
                                          L.MEM_DEVICE, C.byref(r)))
        return Result.from_c(r), out
    g = np.zeros((mu.num_vertices, 3))
    _check(ctx._lib.hsd_distance_grad(ctx.handle, mu.handle, nu.handle if nu is not None else None,
                                      rule.handle, C.byref(p), g.ctypes.data_as(C.c_void_p),
                                      L.MEM_HOST, C.byref(r)))
    return Result.from_c(r), g


def transform(ctx: Context, mesh: Mesh, nodes, params: Params | None = None) -> np.ndarray:
    """mu_h^ at arbitrary nodes [n,3] (hsd_transform) -> complex128[n]."""
    p = (params or Params()).to_c()
    x = _host_f64(nodes, 3)
    out = np.empty(2 * len(x))
    _check(ctx._lib.hsd_transform(ctx.handle, mesh.handle, x.ctypes.data_as(C.c_void_p), len(x),
                                  L.MEM_HOST, C.byref(p), out.ctypes.data_as(C.c_void_p), L.MEM_HOST))
    return out[0::2] + 1j * out[1::2]


def transform_rule(ctx: Context, mesh: Mesh, rule: Rule, params: Params | None = None) -> np.ndarray:
    """mu_h^ at every node of a rule (hsd_transform_rule) -> complex128[n]."""
    p = (params or Params()).to_c()
    out = np.empty(2 * len(rule))
    _check(ctx._lib.hsd_transform_rule(ctx.handle, mesh.handle, rule.handle, C.byref(p),
                                       out.ctypes.data_as(C.c_void_p), L.MEM_HOST))
    return out[0::2] + 1j * out[1::2]


@dataclass
class Ticket:
    status: int
    result: Result
    arrival_s: float
    admitted_s: float
    finished_s: float
    footprint: int
    error: str = ""

    @property
    def latency_s(self) -> float:
        return self.finished_s - self.arrival_s


class Server:
    """Continuous-batching request loop (hsd_server_*).  Requests are copied
    at submit; results are fetched with poll() / wait()."""

    def __init__(self, ctx: Context | None, slots: int = 4, queue_capacity: int = 4096,
                 budget_bytes: int = 64 << 30, chunk_pairs: int = 20_000_000_000, _fake_rate: float | None = None):
        self.ctx = ctx
        # the simulated executor lives in the test-hooks build of the library
        self._lib = L.load() if _fake_rate is None else L.load_test_hooks()
        cfg = L.ServerCfg()
        cfg.slots, cfg.queue_capacity = int(slots), int(queue_capacity)
        cfg.hbm_budget_bytes, cfg.chunk_pairs = int(budget_bytes), int(chunk_pairs)
        h = C.c_void_p()
        if _fake_rate is None:
            _check(self._lib.hsd_server_create(ctx.handle, C.byref(cfg), C.byref(h)))
        else:
            f = self._lib.hsd__server_create_fake
            f.restype = C.c_int32
            f.argtypes = [C.POINTER(L.ServerCfg), C.c_double, C.POINTER(C.c_void_p)]
            _check(f(C.byref(cfg), float(_fake_rate), C.byref(h)))
        self.handle = h
        self._keep = {}

    @classmethod
    def fake(cls, slots=2, queue_capacity=64, budget_bytes=1 << 30, chunk_pairs=1_000_000,
             pairs_per_s=1e8) -> "Server":
        """A server whose executor simulates the work on the CPU (tests)."""
        return cls(None, slots, queue_capacity, budget_bytes, chunk_pairs, _fake_rate=pairs_per_s)

    def submit(self, verts, tris, rule: Rule | None = None, params: Params | None = None,
               verts2=None, tris2=None, tag: int = 0) -> int:
        v = _host_f64(verts, 3)
        t = _host_i32(tris)
        req = L.Request()
        req.verts, req.nv = v.ctypes.data_as(L.dp), len(v)
        req.tris, req.nt = t.ctypes.data_as(L.ip), len(t)
        if verts2 is not None:
            v2 = _host_f64(verts2, 3)
            t2 = _host_i32(tris2)
            req.verts2, req.nv2 = v2.ctypes.data_as(L.dp), len(v2)
            req.tris2, req.nt2 = t2.ctypes.data_as(L.ip), len(t2)
        req.rule = rule.handle if rule is not None else None
        req.params = (params or Params()).to_c()
        req.tag = int(tag)
        tk = C.c_uint64()
        _check(self._lib.hsd_submit(self.handle, C.byref(req), C.byref(tk)))
        return int(tk.value)

    def _ticket(self, st, r, tm) -> Ticket:
        err = self._lib.hsd_last_error().decode(errors="replace") if st < 0 else ""
        return Ticket(int(st), Result.from_c(r), tm.arrival_s, tm.admitted_s, tm.finished_s, tm.footprint, err)

    def poll(self, ticket: int) -> Ticket:
        r, tm = L.Result(), L.RequestTimes()
        st = self._lib.hsd_poll(self.handle, C.c_uint64(ticket), C.byref(r), C.byref(tm))
        if st == L.HSD_ENOTFOUND:
            _check(st)
        return self._ticket(st, r, tm)

    def wait(self, ticket: int, timeout_s: float = -1.0) -> Ticket:
        r, tm = L.Result(), L.RequestTimes()
        st = self._lib.hsd_wait(self.handle, C.c_uint64(ticket), float(timeout_s), C.byref(r), C.byref(tm))
        if st == L.HSD_ENOTFOUND:
            _check(st)
        return self._ticket(st, r, tm)

    def cancel(self, ticket: int) -> None:
        _check(self._lib.hsd_cancel(self.handle, C.c_uint64(ticket)))

    def release(self, ticket: int) -> None:
        _check(self._lib.hsd_release(self.handle, C.c_uint64(ticket)))

    def close(self) -> None:
        if self.handle:
            self._lib.hsd_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
