"""ctypes binding of libcesim.so (include/cesim.h).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch supplies device memory (field buffers are torch tensors on
the GPU) and the current HIP stream.  The library must have been built
(``paper_2109_11044_amd/build_lib.py`` or ``__graft_entry__.build()``);
loading fails loudly otherwise -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcesim.so")

OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "NEGATIVE_EIGENVALUE",
                3: "NOT_POSITIVE_DEFINITE", 4: "OBS_OUTSIDE_GRID",
                5: "OUT_OF_MEMORY", 6: "HIP", 7: "BAD_STATE"}
PREC = {"fp64": 0, "mixed": 1}

EXPORTS = ["ce_setup", "ce_simulate", "ce_simulate_noalloc", "offgrid_nnkrige", "condition",
           "ce_get_info", "ce_copy_spectrum", "offgrid_copy_weights",
           "condition_copy_coefficients", "cesim_covariance_host",
           "cesim_philox_host", "cesim_status_string", "ce_destroy",
           "cesim_set_default_timing", "ce_set_timing", "ce_get_stage_times",
           "cesim_stage_name", "cesim_release_cached_memory", "ce_set_param",
           "cesim_batch_create", "cesim_batch_run", "cesim_batch_get_info",
           "cesim_batch_destroy", "cesim_run_events", "ce_autotune",
           "cesim_tune_save", "cesim_tune_load", "cesim_tune_entries", "cesim_tune_clear",
           "ce_grad_linear", "ce_grad_vjp", "ce_prediction_se", "nn_surrogate"]
PARAM_GEMM_TILE = 1
PARAM_DRAW_CHUNK_PAIRS = 2
PARAM_GEMM_SPLIT = 3
PARAM_EVENT_ID = 4
PARAM_DRAW_COLS = 6
PARAM_DRAW_ROWS = 7
PARAM_JOINT_BOXES = 8
PARAM_SE_CHUNK_NODES = 9
BATCH_AUTOTUNE = 1
NUM_STAGES = 16
VOID_EXPORTS = ("cesim_status_string", "ce_destroy", "cesim_set_default_timing",
                "cesim_stage_name", "cesim_release_cached_memory", "cesim_batch_destroy",
                "cesim_tune_clear")


class CesimError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name} ({_status_string(status)})")


class Cov(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("sigma2", ctypes.c_double),
                ("range", ctypes.c_double), ("aniso_ratio", ctypes.c_double),
                ("aniso_angle", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("m1", ctypes.c_int), ("m2", ctypes.c_int),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("t1", ctypes.c_int), ("t2", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("t1", ctypes.c_int), ("t2", ctypes.c_int),
                ("lam_min", ctypes.c_double), ("lam_max", ctypes.c_double),
                ("lam_sum", ctypes.c_double), ("max_imag", ctypes.c_double),
                ("nobs", ctypes.c_int), ("k", ctypes.c_int),
                ("gamma_min", ctypes.c_double), ("gamma_max", ctypes.c_double),
                ("ms_setup", ctypes.c_double), ("ms_offgrid", ctypes.c_double),
                ("precision", ctypes.c_int), ("torus_tries", ctypes.c_int)]


class Event(ctypes.Structure):
    _fields_ = [("cov", Cov), ("grid", Grid), ("nobs", ctypes.c_int),
                ("obs_xy", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("nugget", ctypes.c_double), ("k", ctypes.c_int),
                ("nreal", ctypes.c_int), ("first_real", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("event_id", ctypes.c_uint32),
                ("fields", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libcesim.so once; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    dp = ctypes.POINTER(ctypes.c_double)
    L.ce_setup.argtypes = [ctypes.POINTER(Cov), ctypes.POINTER(Grid), i, vp,
                           ctypes.POINTER(vp)]
    L.ce_simulate.argtypes = [vp, i, u64, i, vp]
    L.ce_simulate_noalloc.argtypes = [vp, i, u64, i, vp]
    L.offgrid_nnkrige.argtypes = [vp, i, dp, i]
    L.condition.argtypes = [vp, dp, d, vp]
    L.ce_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.ce_copy_spectrum.argtypes = [vp, vp]
    L.offgrid_copy_weights.argtypes = [vp, vp, vp, vp]
    L.condition_copy_coefficients.argtypes = [vp, vp]
    L.cesim_covariance_host.argtypes = [ctypes.POINTER(Cov), i, dp, dp, dp]
    L.cesim_philox_host.argtypes = [u64, i, ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint32,
                                    ctypes.POINTER(ctypes.c_uint32)]
    L.cesim_status_string.argtypes = [i]
    L.cesim_status_string.restype = ctypes.c_char_p
    L.ce_destroy.argtypes = [vp]
    L.ce_destroy.restype = None
    L.cesim_set_default_timing.argtypes = [i]
    L.cesim_set_default_timing.restype = None
    L.ce_set_timing.argtypes = [vp, i]
    L.ce_set_param.argtypes = [vp, i, i]
    L.ce_get_stage_times.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong), i, i]
    L.cesim_stage_name.argtypes = [i]
    L.cesim_stage_name.restype = ctypes.c_char_p
    L.cesim_release_cached_memory.argtypes = []
    L.cesim_release_cached_memory.restype = None
    ip = ctypes.POINTER(ctypes.c_int)
    L.cesim_batch_create.argtypes = [ctypes.POINTER(Event), i, i, vp, i, ip, ctypes.POINTER(vp)]
    L.cesim_batch_run.argtypes = [vp, i]
    L.cesim_batch_get_info.argtypes = [vp, i, ctypes.POINTER(Info)]
    L.cesim_batch_destroy.argtypes = [vp]
    L.cesim_batch_destroy.restype = None
    L.cesim_run_events.argtypes = [ctypes.POINTER(Event), i, i, vp, ip]
    L.ce_autotune.argtypes = [vp, i, vp]
    L.cesim_tune_save.argtypes = [ctypes.c_char_p]
    L.cesim_tune_load.argtypes = [ctypes.c_char_p]
    L.cesim_tune_entries.argtypes = []
    L.cesim_tune_clear.argtypes = []
    L.cesim_tune_clear.restype = None
    L.ce_grad_linear.argtypes = [vp, dp, d, i, u64, i, vp, dp, dp]
    L.ce_grad_vjp.argtypes = [vp, dp, d, i, u64, i, vp, dp, dp]
    L.ce_prediction_se.argtypes = [vp, d, vp, vp]
    L.nn_surrogate.argtypes = [vp, i, dp, dp, d, i, i, dp, dp, ctypes.POINTER(ctypes.c_int)]
    for name in EXPORTS:
        if name not in VOID_EXPORTS:
            getattr(L, name).restype = i
    _lib = L
    return L


def _status_string(s):
    try:
        return lib().cesim_status_string(s).decode()
    except Exception:
        return "?"


def _check(status, where):
    if status != OK:
        raise CesimError(status, where)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_cov(nu=0.5, sigma2=1.0, range=0.1, aniso_ratio=1.0, aniso_angle=0.0):
    return Cov(float(nu), float(sigma2), float(range), float(aniso_ratio),
               float(aniso_angle))


def unit_square_grid(m, torus=0):
    dx = 1.0 / (m - 1)
    return Grid(m, m, 0.0, 0.0, dx, dx, torus, torus)


def covariance_host(cov, hx, hy):
    """The library's covariance source evaluated on the host (FP64)."""
    hx = np.ascontiguousarray(hx, dtype=np.float64).ravel()
    hy = np.ascontiguousarray(hy, dtype=np.float64).ravel()
    out = np.empty_like(hx)
    _check(lib().cesim_covariance_host(ctypes.byref(cov), hx.size, _dptr(hx),
                                       _dptr(hy), _dptr(out)), "covariance_host")
    return out


def philox_host(seed, ctr0, c1, c2, c3):
    ctr0 = np.ascontiguousarray(ctr0, dtype=np.uint32).ravel()
    out = np.empty((ctr0.size, 4), dtype=np.uint32)
    P = ctypes.POINTER(ctypes.c_uint32)
    _check(lib().cesim_philox_host(int(seed), ctr0.size, ctr0.ctypes.data_as(P),
                                   int(c1), int(c2), int(c3),
                                   out.ctypes.data_as(P)), "philox_host")
    return out


def stage_names():
    return [lib().cesim_stage_name(i).decode() for i in range(NUM_STAGES)]


def set_default_timing(enable):
    lib().cesim_set_default_timing(1 if enable else 0)


def release_cached_memory():
    lib().cesim_release_cached_memory()


def tune_save(path):
    _check(lib().cesim_tune_save(os.fsencode(path)), "cesim_tune_save")


def tune_load(path):
    _check(lib().cesim_tune_load(os.fsencode(path)), "cesim_tune_load")


def tune_entries():
    return lib().cesim_tune_entries()


def tune_clear():
    lib().cesim_tune_clear()


class Context:
    """One event: covariance, grid and precision; owns the C context."""

    def __init__(self, cov, grid, precision="fp64", stream=None):
        import torch
        self._torch = torch
        self.cov, self.grid = cov, grid
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().ce_setup(ctypes.byref(cov), ctypes.byref(grid),
                              PREC[precision], ctypes.c_void_p(stream.cuda_stream),
                              ctypes.byref(h)), "ce_setup")
        self._h = h
        self.nobs = 0
        self.k = 0

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().ce_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _fields_check(self, fields, nreal):
        t = self._torch
        g = self.grid
        if not (isinstance(fields, t.Tensor) and fields.is_cuda and
                fields.dtype == self.dtype and fields.is_contiguous() and
                fields.numel() >= nreal * g.m1 * g.m2):
            raise ValueError("fields must be a contiguous CUDA tensor of "
                             f"{self.dtype} with nreal*m2*m1 elements")

    def simulate(self, nreal, seed, first_real=0, out=None):
        t = self._torch
        g = self.grid
        if out is None:
            out = t.empty((nreal, g.m2, g.m1), dtype=self.dtype, device="cuda")
        self._fields_check(out, nreal)
        _check(lib().ce_simulate(self._h, int(nreal), int(seed), int(first_real),
                                 ctypes.c_void_p(out.data_ptr())), "ce_simulate")
        self.nreal = nreal
        return out

    def offgrid(self, obs_xy, k):
        xy = np.ascontiguousarray(obs_xy, dtype=np.float64).reshape(-1, 2)
        _check(lib().offgrid_nnkrige(self._h, xy.shape[0], _dptr(xy), int(k)),
               "offgrid_nnkrige")
        self.nobs, self.k = xy.shape[0], int(k)

    def condition(self, z, nugget, fields):
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        if z.size != self.nobs:
            raise ValueError("z must hold one value per observation")
        self._fields_check(fields, getattr(self, "nreal", 1))
        _check(lib().condition(self._h, _dptr(z), float(nugget),
                               ctypes.c_void_p(fields.data_ptr())), "condition")
        return fields

    def info(self):
        inf = Info()
        _check(lib().ce_get_info(self._h, ctypes.byref(inf)), "ce_get_info")
        return {f: getattr(inf, f) for f, _ in Info._fields_}

    def autotune(self, nreal, fields):
        """Tune the launch shapes for this context's problem (overwrites
        ``fields``); the choice goes into the process-wide table."""
        self._fields_check(fields, nreal)
        _check(lib().ce_autotune(self._h, int(nreal), ctypes.c_void_p(fields.data_ptr())),
               "ce_autotune")

    def set_param(self, param, value):
        _check(lib().ce_set_param(self._h, int(param), int(value)), "ce_set_param")

    def set_timing(self, enable):
        _check(lib().ce_set_timing(self._h, 1 if enable else 0), "ce_set_timing")

    def stage_times(self, reset=True):
        """{stage: (ms, launches)} accumulated since the last reset."""
        ms = np.zeros(NUM_STAGES)
        calls = np.zeros(NUM_STAGES, dtype=np.int64)
        _check(lib().ce_get_stage_times(self._h, _dptr(ms),
                                        calls.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                        NUM_STAGES, 1 if reset else 0), "ce_get_stage_times")
        return {n: (float(ms[i]), int(calls[i])) for i, n in enumerate(stage_names())}

    def spectrum(self):
        t = self._torch
        inf = self.info()
        out = t.empty((inf["t2"], inf["t1"]), dtype=t.float64, device="cuda")
        _check(lib().ce_copy_spectrum(self._h, ctypes.c_void_p(out.data_ptr())),
               "ce_copy_spectrum")
        return out

    def weights(self):
        t = self._torch
        cor = t.empty((self.nobs, 2), dtype=t.int32, device="cuda")
        w = t.empty((self.nobs, self.k), dtype=t.float64, device="cuda")
        gm = t.empty((self.nobs,), dtype=t.float64, device="cuda")
        _check(lib().offgrid_copy_weights(self._h, ctypes.c_void_p(cor.data_ptr()),
                                          ctypes.c_void_p(w.data_ptr()),
                                          ctypes.c_void_p(gm.data_ptr())),
               "offgrid_copy_weights")
        return cor, w, gm

    def grad_linear(self, z, nugget, nreal, seed, weights, first_real=0):
        """L = mean over the realizations of sum_g weights[g] v_r[g] and its
        gradient: {"L", "d_range", "d_sigma2", "d_nugget", "d_z"} (FP64).
        weights: CUDA float64 tensor of m2 x m1 grid weights."""
        t = self._torch
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        if z.size != self.nobs:
            raise ValueError("z must hold one value per observation")
        if (not weights.is_cuda or weights.dtype != t.float64 or not weights.is_contiguous()
                or weights.numel() != self.grid.m1 * self.grid.m2):
            raise ValueError("weights must be a contiguous CUDA float64 tensor of m2 x m1")
        out = np.zeros(4)
        dz = np.zeros(self.nobs)
        _check(lib().ce_grad_linear(self._h, _dptr(z), float(nugget), int(nreal), int(seed),
                                    int(first_real), ctypes.c_void_p(weights.data_ptr()),
                                    _dptr(out), _dptr(dz)), "ce_grad_linear")
        return {"L": float(out[0]), "d_range": float(out[1]), "d_sigma2": float(out[2]),
                "d_nugget": float(out[3]), "d_z": dz}

    def grad_vjp(self, z, nugget, nreal, seed, vbar, first_real=0):
        """Vector-Jacobian product of the conditional fields (FP64 path):
        vbar is the CUDA float64 tensor (nreal, m2, m1) of derivatives of a
        statistic with respect to the fields of realizations first_real ...;
        returns {"vbar_dot_v", "d_range", "d_sigma2", "d_nugget", "d_z"}."""
        t = self._torch
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        if z.size != self.nobs:
            raise ValueError("z must hold one value per observation")
        if (not vbar.is_cuda or vbar.dtype != t.float64 or not vbar.is_contiguous()
                or vbar.numel() != int(nreal) * self.grid.m1 * self.grid.m2):
            raise ValueError("vbar must be a contiguous CUDA float64 tensor of nreal x m2 x m1")
        out = np.zeros(4)
        dz = np.zeros(self.nobs)
        _check(lib().ce_grad_vjp(self._h, _dptr(z), float(nugget), int(nreal), int(seed),
                                 int(first_real), ctypes.c_void_p(vbar.data_ptr()), _dptr(out),
                                 _dptr(dz)), "ce_grad_vjp")
        return {"vbar_dot_v": float(out[0]), "d_range": float(out[1]), "d_sigma2": float(out[2]),
                "d_nugget": float(out[3]), "d_z": dz}

    def nn_surrogate(self, obs_xy, z, nugget, k):
        """Nearest-neighbour Kriging: install the surrogate sites of the
        observations as the stations; returns (site_xy, z_site) as numpy
        arrays (sites in ascending node index)."""
        xy = np.ascontiguousarray(obs_xy, dtype=np.float64).reshape(-1, 2)
        z = np.ascontiguousarray(z, dtype=np.float64).ravel()
        if z.size != xy.shape[0]:
            raise ValueError("z must hold one value per observation")
        cap = xy.shape[0] * int(k)
        sxy = np.empty((cap, 2))
        zs = np.empty(cap)
        ns = ctypes.c_int(0)
        st = lib().nn_surrogate(self._h, xy.shape[0], _dptr(xy), _dptr(z), float(nugget), int(k),
                                cap, _dptr(sxy), _dptr(zs), ctypes.byref(ns))
        if st != OK:                    # the context holds the observations, or none
            inf = self.info()
            self.nobs, self.k = inf["nobs"], inf["k"]
            _check(st, "nn_surrogate")
        self.nobs, self.k = ns.value, 4
        return sxy[:ns.value].copy(), zs[:ns.value].copy()

    def prediction_se(self, nugget):
        """(SE_E, SE_L): exact and local-Kriging prediction standard errors on
        the grid, CUDA float64 tensors of m2 x m1."""
        t = self._torch
        g = self.grid
        se_e = t.empty((g.m2, g.m1), dtype=t.float64, device="cuda")
        se_l = t.empty((g.m2, g.m1), dtype=t.float64, device="cuda")
        _check(lib().ce_prediction_se(self._h, float(nugget), ctypes.c_void_p(se_e.data_ptr()),
                                      ctypes.c_void_p(se_l.data_ptr())), "ce_prediction_se")
        return se_e, se_l

    def coefficients(self):
        t = self._torch
        out = t.empty((self.nreal, self.nobs), dtype=t.float64, device="cuda")
        _check(lib().condition_copy_coefficients(self._h, ctypes.c_void_p(out.data_ptr())),
               "condition_copy_coefficients")
        return out


class BatchError(CesimError):
    """A batch could not be planned; .event_status lists each event's status."""

    def __init__(self, status, where, event_status):
        super().__init__(status, where)
        self.event_status = list(event_status)


class Batch:
    """Independent events planned once and run with one graph launch each.

    ``events`` is a list of dicts with keys cov, grid, obs_xy, z, nugget, k,
    nreal, seed and optionally first_real (0) and event_id (its position).
    Field tensors are allocated here ([nreal, m2, m1]; float64 for "fp64",
    float32 for "mixed") and overwritten by every run."""

    def __init__(self, events, precision="fp64", stream=None, autotune=False):
        import torch
        self._torch = torch
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        ne = len(events)
        self.fields, keep = [], []
        table = (Event * ne)()
        for e, ev in enumerate(events):
            g = ev["grid"]
            xy = np.ascontiguousarray(ev["obs_xy"], dtype=np.float64).reshape(-1, 2)
            z = np.ascontiguousarray(ev["z"], dtype=np.float64).ravel()
            if z.size != xy.shape[0]:
                raise ValueError(f"event {e}: z must hold one value per observation")
            f = torch.empty((int(ev["nreal"]), g.m2, g.m1), dtype=self.dtype, device="cuda")
            self.fields.append(f)
            keep += [xy, z]
            table[e] = Event(ev["cov"], g, xy.shape[0], xy.ctypes.data, z.ctypes.data,
                             float(ev["nugget"]), int(ev["k"]), int(ev["nreal"]),
                             int(ev.get("first_real", 0)), int(ev["seed"]),
                             int(ev.get("event_id", e)), f.data_ptr())
        st = (ctypes.c_int * ne)()
        h = ctypes.c_void_p()
        rc = lib().cesim_batch_create(table, ne, PREC[precision],
                                      ctypes.c_void_p(stream.cuda_stream),
                                      BATCH_AUTOTUNE if autotune else 0, st, ctypes.byref(h))
        self.event_status = [STATUS_NAMES.get(v, str(v)) for v in st]
        if rc != OK:
            raise BatchError(rc, "cesim_batch_create", self.event_status)
        self._h = h

    def run(self, real_offset=0):
        _check(lib().cesim_batch_run(self._h, int(real_offset)), "cesim_batch_run")
        return self.fields

    def info(self, e):
        inf = Info()
        _check(lib().cesim_batch_get_info(self._h, int(e), ctypes.byref(inf)),
               "cesim_batch_get_info")
        return {f: getattr(inf, f) for f, _ in Info._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().cesim_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _ensemble_linear_stat_function():
    import torch

    class EnsembleLinearStat(torch.autograd.Function):
        """L(range, sigma2, nugget, z) = mean over realizations of the
        weighted grid sum of the conditional fields; backward is the
        library's hand-written adjoint (ce_grad_linear)."""

        @staticmethod
        def forward(ctx, range_, sigma2, nugget, z, spec):
            cov = make_cov(spec["nu"], float(sigma2), float(range_), spec.get("aniso_ratio", 1.0),
                           spec.get("aniso_angle", 0.0))
            with Context(cov, spec["grid"], spec.get("precision", "fp64")) as c:
                c.set_param(PARAM_EVENT_ID, spec.get("event_id", 0))
                c.offgrid(spec["obs_xy"], spec["k"])
                g = c.grad_linear(z.detach().cpu().numpy(), float(nugget), spec["nreal"],
                                  spec["seed"], spec["weights"], spec.get("first_real", 0))
            f64 = dict(dtype=torch.float64)
            ctx.save_for_backward(torch.tensor(g["d_range"], **f64),
                                  torch.tensor(g["d_sigma2"], **f64),
                                  torch.tensor(g["d_nugget"], **f64),
                                  torch.as_tensor(g["d_z"], **f64))
            return torch.tensor(g["L"], **f64)

        @staticmethod
        def backward(ctx, grad_out):
            dr, ds, dn, dz = ctx.saved_tensors
            return grad_out * dr, grad_out * ds, grad_out * dn, grad_out * dz, None

    return EnsembleLinearStat


def _conditional_fields_function():
    import torch

    def context(range_, sigma2, spec):
        cov = make_cov(spec["nu"], float(sigma2), float(range_), spec.get("aniso_ratio", 1.0),
                       spec.get("aniso_angle", 0.0))
        c = Context(cov, spec["grid"], "fp64")
        c.set_param(PARAM_EVENT_ID, spec.get("event_id", 0))
        c.offgrid(spec["obs_xy"], spec["k"])
        return c

    class ConditionalFields(torch.autograd.Function):
        """The conditional realizations (FP64 path) as a function of the
        range, sigma2, the nugget and the observed values; backward is the
        library's vector-Jacobian product (ce_grad_vjp), so any statistic of
        the ensemble computed from them with torch is differentiable."""

        @staticmethod
        def forward(ctx, range_, sigma2, nugget, z, spec):
            R, g = spec["nreal"], spec["grid"]
            zh = z.detach().cpu().numpy()
            with context(range_, sigma2, spec) as c:
                f = torch.empty((R, g.m2, g.m1), dtype=torch.float64, device="cuda")
                c.simulate(R, spec["seed"], spec.get("first_real", 0), out=f)
                c.condition(zh, float(nugget), f)
            ctx.spec = spec
            ctx.save_for_backward(range_.detach(), sigma2.detach(), nugget.detach(), z.detach())
            return f

        @staticmethod
        def backward(ctx, grad_out):
            range_, sigma2, nugget, z = ctx.saved_tensors
            spec = ctx.spec
            vbar = grad_out.detach().to(torch.float64).contiguous()
            with context(range_, sigma2, spec) as c:
                g = c.grad_vjp(z.cpu().numpy(), float(nugget), spec["nreal"], spec["seed"], vbar,
                               spec.get("first_real", 0))
            f64 = dict(dtype=torch.float64)
            return (torch.tensor(g["d_range"], **f64), torch.tensor(g["d_sigma2"], **f64),
                    torch.tensor(g["d_nugget"], **f64), torch.as_tensor(g["d_z"], **f64), None)

    return ConditionalFields


def conditional_fields(range_, sigma2, nugget, z, spec):
    """Differentiable (torch.autograd) conditional realizations on the FP64
    path: (nreal, m2, m1) float64 CUDA tensor; see ConditionalFields.
    range_, sigma2, nugget: 0-d float64 tensors; z: 1-d float64 tensor;
    spec: nu, grid, obs_xy, k, nreal, seed and optionally aniso_ratio,
    aniso_angle, event_id, first_real."""
    global _CF
    if _CF is None:
        _CF = _conditional_fields_function()
    return _CF.apply(range_, sigma2, nugget, z, spec)


_CF = None


def ensemble_linear_stat(range_, sigma2, nugget, z, spec):
    """Differentiable (torch.autograd) linear ensemble statistic; see
    EnsembleLinearStat.  range_, sigma2, nugget: 0-d float64 tensors; z: 1-d
    float64 tensor; spec: nu, grid, obs_xy, k, nreal, seed, weights (CUDA
    float64 m2 x m1) and optionally aniso_ratio, aniso_angle, precision,
    event_id, first_real."""
    global _ELS
    if _ELS is None:
        _ELS = _ensemble_linear_stat_function()
    return _ELS.apply(range_, sigma2, nugget, z, spec)


_ELS = None
