"""ctypes binding of libpint.so (the C ABI in include/pint.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch tensors (float64, contiguous, on the GPU);
complex coefficients are stored as (re, im) pairs, so a batch of B states is a
float64 tensor of shape (B, 3, ncoef, 2) (or any tensor with that many
elements).  The library must have been built (``python -m
paper_2306_09497_amd.build``); importing this module without it raises.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpint.so")

T_LG, T_LC, T_NL, T_VISC, T_ALL = 1, 2, 4, 8, 15
PARAREAL, MGRIT = 0, 1

FP64, LEG_FP32, LEG_BF16X3 = 0, 1, 2    # pint_config.precision

STATUS = {0: "PINT_OK", -1: "PINT_E_INVAL", -2: "PINT_E_NOMEM", -3: "PINT_E_HIP",
          -4: "PINT_E_DIVERGED", -5: "PINT_E_NOTCONV"}

EXPORTS = ["pint_plan_create", "pint_plan_destroy", "pint_plan_info", "pint_plan_workspace_bytes",
           "pint_plan_reserve", "pint_grid_coords",
           "pint_synthesis", "pint_analysis", "pint_tendency", "pint_implicit", "pint_step", "pint_step_noalloc",
           "pint_sl_steps", "pint_parareal_sl", "pint_solve", "pint_rel_diff", "pint_ke_spectrum", "pint_spectral_errors",
           "pint_grid_l2_errors", "pint_stability_map", "pint_server_create", "pint_server_destroy",
           "pint_server_submit", "pint_server_tick", "pint_server_status", "pint_server_clock",
           "pint_profile_enable", "pint_profile_read", "pint_last_error"]

REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3

PROF_KINDS = ["prep", "legendre_synth", "ring_tendency", "legendre_anal", "assemble_rk",
              "cn_solve", "layout", "pint_ops", "scalar_ring", "sl_points"]


class Config(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("nlon", ctypes.c_int), ("nlat", ctypes.c_int),
                ("a", ctypes.c_double), ("omega", ctypes.c_double), ("g", ctypes.c_double),
                ("phibar", ctypes.c_double), ("max_batch", ctypes.c_int),
                ("precision", ctypes.c_int)]


class Stepper(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("visc_order", ctypes.c_int),
                ("visc_nu", ctypes.c_double), ("terms", ctypes.c_uint)]


class SlStepper(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("traj_iters", ctypes.c_int),
                ("visc_order", ctypes.c_int), ("visc_nu", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("nlon", ctypes.c_int), ("nlat", ctypes.c_int),
                ("ncoef", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("state_doubles", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("allocations", ctypes.c_longlong), ("gemm_shape", (ctypes.c_int * 2) * 2),
                ("gemm_us", (ctypes.c_double * 2) * 2), ("ring_threads", ctypes.c_int * 2),
                ("ring_us", ctypes.c_double * 2)]


class PintParams(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("n_intervals", ctypes.c_int),
                ("fine", Stepper), ("fine_steps", ctypes.c_int),
                ("coarse", Stepper), ("coarse_steps", ctypes.c_int),
                ("nrelax", ctypes.c_int), ("max_iter", ctypes.c_int), ("tol", ctypes.c_double),
                ("resume", ctypes.c_int), ("levels", ctypes.c_int), ("cfactor1", ctypes.c_int),
                ("coarse2", Stepper), ("coarse2_steps", ctypes.c_int), ("cycles1", ctypes.c_int),
                ("coarse_plan", ctypes.c_void_p), ("coarse_sl", ctypes.POINTER(SlStepper))]


class ProfEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("batch", ctypes.c_int),
                ("launches", ctypes.c_longlong), ("total_ms", ctypes.c_double)]


class StabilityCfg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("coarse", ctypes.c_int), ("xl_re", ctypes.c_double),
                ("xl_im", ctypes.c_double), ("re0", ctypes.c_double), ("re1", ctypes.c_double),
                ("nre", ctypes.c_int), ("im0", ctypes.c_double), ("im1", ctypes.c_double),
                ("nim", ctypes.c_int), ("n", ctypes.c_int), ("k", ctypes.c_int),
                ("cfactor", ctypes.c_int), ("n_c", ctypes.c_int), ("nrelax", ctypes.c_int),
                ("n_ks", ctypes.c_int)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_plans", ctypes.c_int), ("plans", ctypes.POINTER(ctypes.c_void_p)),
                ("arena_bytes", ctypes.c_size_t), ("steps_per_tick", ctypes.c_int),
                ("stage_states", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_int), ("params", PintParams), ("u0", ctypes.c_void_p),
                ("u_slices", ctypes.c_void_p)]


class RequestStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("incr", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("fine_slice_steps", ctypes.c_longlong), ("coarse_steps", ctypes.c_longlong)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("incr", ctypes.c_double * 128),
                ("incr_field", (ctypes.c_double * 4) * 128),
                ("seconds", ctypes.c_double * 128), ("fine_seconds", ctypes.c_double * 128),
                ("coarse_seconds", ctypes.c_double * 128), ("fine_slice_steps", ctypes.c_longlong),
                ("coarse_steps", ctypes.c_longlong), ("graph_iters", ctypes.c_int)]


class PintError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path=LIB_PATH):
    """Load libpint.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built: run python -m paper_2306_09497_amd.build")
    # torch ships its own HIP runtime; load it first so that libpint binds to
    # the same libamdhip64 instance (one runtime per process).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    lib.pint_plan_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
    lib.pint_plan_destroy.argtypes = [vp]
    lib.pint_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
    lib.pint_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(PintParams),
                                              ctypes.POINTER(SlStepper),
                                              ctypes.POINTER(ctypes.c_size_t)]
    lib.pint_plan_reserve.argtypes = [vp, ctypes.POINTER(PintParams), ctypes.POINTER(SlStepper),
                                      vp]
    lib.pint_grid_coords.argtypes = [vp, dp, dp, vp]
    lib.pint_synthesis.argtypes = [vp, vp, vp, ip, vp]
    lib.pint_analysis.argtypes = [vp, vp, vp, ip, vp]
    lib.pint_tendency.argtypes = [vp, vp, vp, ip, vp]
    lib.pint_implicit.argtypes = [vp, ctypes.POINTER(Stepper), vp, vp, ip, vp]
    lib.pint_step.argtypes = [vp, ctypes.POINTER(Stepper), vp, vp, ip, ip, vp]
    lib.pint_step_noalloc.argtypes = [vp, ctypes.POINTER(Stepper), vp, vp, ip, ip, vp]
    lib.pint_solve.argtypes = [vp, ctypes.POINTER(PintParams), vp, vp, ctypes.POINTER(Report), vp]
    lib.pint_rel_diff.argtypes = [vp, vp, vp, dp, ip, vp]
    lib.pint_ke_spectrum.argtypes = [vp, vp, vp, ip, vp]
    lib.pint_spectral_errors.argtypes = [vp, vp, vp, vp, ip, vp]
    lib.pint_grid_l2_errors.argtypes = [vp, vp, vp, dp, ip, vp]
    lib.pint_stability_map.argtypes = [ctypes.POINTER(StabilityCfg), vp, vp]
    lib.pint_server_create.argtypes = [ctypes.POINTER(ServerConfig), vp, ctypes.POINTER(vp)]
    lib.pint_server_destroy.argtypes = [vp]
    lib.pint_server_submit.argtypes = [vp, ctypes.POINTER(Request),
                                       ctypes.POINTER(ctypes.c_longlong)]
    lib.pint_server_tick.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.pint_server_status.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(RequestStatus)]
    lib.pint_server_clock.argtypes = [vp, dp]
    lib.pint_profile_enable.argtypes = [vp, ctypes.c_uint, ip]
    lib.pint_profile_read.argtypes = [vp, ctypes.POINTER(ProfEntry), ip,
                                      ctypes.POINTER(ctypes.c_int), vp]
    lib.pint_last_error.argtypes = []
    lib.pint_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-1]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        msg = _lib.pint_last_error().decode(errors="replace")
        raise PintError(status, msg)


def _ptr(t, numel=None):
    """Device pointer of a contiguous float64 GPU tensor holding at least
    numel elements (the library reads and writes that many)."""
    if t is None:
        return None
    import torch
    if numel is not None and t.numel() < numel:
        raise ValueError(f"device array holds {t.numel()} doubles, the call needs {numel}")
    if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("device arrays must be contiguous float64 CUDA/HIP tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def stepper(dt, visc_order=2, visc_nu=0.0, terms=T_ALL):
    return Stepper(float(dt), int(visc_order), float(visc_nu), int(terms))


def sl_stepper(dt, traj_iters=2, visc_order=2, visc_nu=0.0):
    return SlStepper(float(dt), int(traj_iters), int(visc_order), float(visc_nu))


class Plan:
    """A truncation / grid / planet and the device tables and workspace.

    precision: FP64 (default); LEG_FP32 for Legendre GEMMs, Fourier rows and
    the grid-space tendencies in FP32 (state, implicit solve and time
    integration stay FP64); LEG_BF16X3 as LEG_FP32 with the GEMM products as
    three BF16 matrix-core products of split operands."""

    def __init__(self, M, nlon, nlat, a=6.37122e6, omega=7.292e-5, g=9.80616,
                 phibar=2.94e4, max_batch=64, stream=None, precision=FP64):
        lib = load()
        self.cfg = Config(M, nlon, nlat, a, omega, g, phibar, max_batch, precision)
        self.precision = precision
        h = ctypes.c_void_p()
        _check(lib.pint_plan_create(ctypes.byref(self.cfg), _stream(stream), ctypes.byref(h)))
        self._h = h
        info = Info()
        _check(lib.pint_plan_info(h, ctypes.byref(info)))
        self.M, self.nlon, self.nlat, self.ncoef = M, nlon, nlat, info.ncoef
        self.max_batch = info.max_batch
        self.workspace_bytes = info.workspace_bytes

    def info(self):
        info = Info()
        _check(load().pint_plan_info(self._h, ctypes.byref(info)))
        return info

    def workspace_query(self, params=None, sl=None):
        """Device bytes the plan holds once reserved for pint_solve(params)
        and pint_sl_steps(sl) (either may be None)."""
        n = ctypes.c_size_t()
        _check(load().pint_plan_workspace_bytes(
            self._h, None if params is None else ctypes.byref(params),
            None if sl is None else ctypes.byref(sl), ctypes.byref(n)))
        return n.value

    def reserve(self, params=None, sl=None, stream=None):
        _check(load().pint_plan_reserve(self._h, None if params is None else ctypes.byref(params),
                                        None if sl is None else ctypes.byref(sl),
                                        _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().pint_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers ------------------------------------------------------
    def state_numel(self, B=1):
        return B * 3 * self.ncoef * 2

    def grid_coords(self, stream=None):
        import numpy as np
        mu = np.zeros(self.nlat)
        w = np.zeros(self.nlat)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().pint_grid_coords(self._h, mu.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                       _stream(stream)))
        return mu, w

    # ---- entry points -------------------------------------------------
    def synthesis(self, spec, grid, B, stream=None):
        _check(load().pint_synthesis(self._h, _ptr(spec, B * self.ncoef * 2),
                                     _ptr(grid, B * self.nlat * self.nlon), int(B),
                                     _stream(stream)))

    def analysis(self, grid, spec, B, stream=None):
        _check(load().pint_analysis(self._h, _ptr(grid, B * self.nlat * self.nlon),
                                    _ptr(spec, B * self.ncoef * 2), int(B), _stream(stream)))

    def tendency(self, u, out, B, stream=None):
        n = self.state_numel(B)
        _check(load().pint_tendency(self._h, _ptr(u, n), _ptr(out, n), int(B), _stream(stream)))

    def implicit(self, st, u, x, B, stream=None):
        n = self.state_numel(B)
        _check(load().pint_implicit(self._h, ctypes.byref(st), _ptr(u, n), _ptr(x, n), int(B),
                                    _stream(stream)))

    def step(self, st, u_in, u_out, B, nsteps, stream=None):
        n = self.state_numel(B)
        _check(load().pint_step(self._h, ctypes.byref(st), _ptr(u_in, n), _ptr(u_out, n), int(B),
                                int(nsteps), _stream(stream)))

    def step_noalloc(self, st, u_in, u_out, B, nsteps, stream=None):
        """pint_step without device allocation (the library's static scratch)."""
        n = self.state_numel(B)
        _check(load().pint_step_noalloc(self._h, ctypes.byref(st), _ptr(u_in, n), _ptr(u_out, n),
                                        int(B), int(nsteps), _stream(stream)))

    def sl_steps(self, st, u, out, B, nsteps, u_prev=None, out_prev=None, stream=None):
        """nsteps SL-SI-SETTLS steps; u_prev None = one-step first step."""
        n = self.state_numel(B)
        _check(load().pint_sl_steps(self._h, ctypes.byref(st), _ptr(u_prev, n), _ptr(u, n),
                                    _ptr(out, n), _ptr(out_prev, n), int(B), int(nsteps),
                                    _stream(stream)))

    def parareal_sl(self, fine, fine_steps, coarse, coarse_steps, n_slices, n_iter, u0, u_slices,
                    n_inst=1, coarse_plan=None, restart=False, stream=None):
        """Parareal with an SL-SI-SETTLS coarse propagator (fine: IMEX stepper);
        u0 [n_inst] states, u_slices [n_slices + 1][n_inst] states.  The sweep
        carries the two-step scheme across slices (restart=True: one-step
        variant at every slice start)."""
        cp = None if coarse_plan is None else coarse_plan._h
        _check(load().pint_parareal_sl(self._h, ctypes.byref(fine), int(fine_steps), cp,
                                       ctypes.byref(coarse), int(coarse_steps), int(n_slices),
                                       int(n_inst), int(n_iter), int(bool(restart)),
                                       _ptr(u0, self.state_numel(n_inst)),
                                       _ptr(u_slices, self.state_numel((n_slices + 1) * n_inst)),
                                       _stream(stream)))

    def solve(self, params, u0, u_slices, stream=None):
        rep = Report()
        _check(load().pint_solve(self._h, ctypes.byref(params), _ptr(u0, self.state_numel()),
                                 _ptr(u_slices, self.state_numel(params.n_intervals + 1)),
                                 ctypes.byref(rep), _stream(stream)))
        return rep

    def solve_status(self, params, u0, u_slices, stream=None):
        """Like solve() but returns (status, report, message) instead of raising."""
        rep = Report()
        st = load().pint_solve(self._h, ctypes.byref(params), _ptr(u0, self.state_numel()),
                               _ptr(u_slices, self.state_numel(params.n_intervals + 1)),
                               ctypes.byref(rep), _stream(stream))
        msg = load().pint_last_error().decode(errors="replace") if st else ""
        return st, rep, msg

    def profile(self, kinds=None, min_batch=0):
        """Time kernel launches of the given kinds (names from PROF_KINDS; None =
        all, [] = off) processing at least min_batch states."""
        if kinds is None:
            mask = (1 << len(PROF_KINDS)) - 1
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << PROF_KINDS.index(k)
        _check(load().pint_profile_enable(self._h, mask, int(min_batch)))

    def profile_read(self, stream=None):
        """{(kind name, batch): (launches, total_ms)} since the last read."""
        buf = (ProfEntry * 64)()
        n = ctypes.c_int(0)
        _check(load().pint_profile_read(self._h, buf, 64, ctypes.byref(n), _stream(stream)))
        return {(PROF_KINDS[e.kind], e.batch): (e.launches, e.total_ms) for e in buf[:n.value]}

    def rel_diff(self, a, c, B, stream=None):
        import numpy as np
        out = np.zeros((B, 4))
        dp = ctypes.POINTER(ctypes.c_double)
        n = self.state_numel(B)
        _check(load().pint_rel_diff(self._h, _ptr(a, n), _ptr(c, n), out.ctypes.data_as(dp),
                                    int(B), _stream(stream)))
        return out

    # ---- diagnostics (Sec. 5, Sec. 5.1) ---------------------------------
    def ke_spectrum(self, u, e, B, stream=None):
        """e (device [B][M+1]) <- kinetic-energy spectrum of the B states u."""
        _check(load().pint_ke_spectrum(self._h, _ptr(u, self.state_numel(B)),
                                       _ptr(e, B * (self.M + 1)), int(B), _stream(stream)))

    def spectral_errors(self, u, ref, e, B, stream=None):
        """e (device [B][3][M+1]) <- E_{psi,R} of (Phi', xi, delta), R = 0..M."""
        n = self.state_numel(B)
        _check(load().pint_spectral_errors(self._h, _ptr(u, n), _ptr(ref, n),
                                           _ptr(e, B * 3 * (self.M + 1)), int(B),
                                           _stream(stream)))

    def grid_l2_errors(self, u, ref, B, stream=None):
        """Host [B][3] physical-space relative L2 errors of (Phi', xi, delta)."""
        import numpy as np
        out = np.zeros((B, 3))
        dp = ctypes.POINTER(ctypes.c_double)
        n = self.state_numel(B)
        _check(load().pint_grid_l2_errors(self._h, _ptr(u, n), _ptr(ref, n),
                                          out.ctypes.data_as(dp), int(B), _stream(stream)))
        return out


def params(method, n_intervals, fine, fine_steps, coarse, coarse_steps, nrelax=0, max_iter=1,
           tol=0.0, resume=False, levels=2, cfactor1=0, coarse2=None, coarse2_steps=1,
           cycles1=1, coarse_plan=None, coarse_sl=None):
    """Parameters of Plan.solve; coarse_plan (a Plan at a truncation <= this
    plan's) runs the coarse levels with spatial coarsening; coarse_sl (an
    sl_stepper) makes the coarse level of two-level MGRIT SL-SI-SETTLS, one
    step per C-interval (then `coarse` is not used: pass None)."""
    c2 = coarse2 if coarse2 is not None else Stepper(0.0, 2, 0.0, 0)
    c1 = coarse if coarse is not None else Stepper(0.0, 2, 0.0, 0)
    cp = coarse_plan._h.value if coarse_plan is not None else None
    csl = ctypes.pointer(coarse_sl) if coarse_sl is not None else None
    return PintParams(int(method), int(n_intervals), fine, int(fine_steps), c1,
                      int(coarse_steps), int(nrelax), int(max_iter), float(tol), int(resume),
                      int(levels), int(cfactor1), c2, int(coarse2_steps), int(cycles1), cp, csl)


class Server:
    """Continuous-batching server over borrowed plans (see pint_server_create).

    submit() queues a solve and returns its id; tick() runs one scheduling
    step and returns the number of requests still queued or running."""

    def __init__(self, plans, arena_bytes, steps_per_tick=8, stage_states=64, stream=None):
        lib = load()
        self._plans = list(plans)           # keep the plans alive
        arr = (ctypes.c_void_p * len(self._plans))(*[p._h.value for p in self._plans])
        self._arr = arr
        cfg = ServerConfig(len(self._plans), ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)),
                           int(arena_bytes), int(steps_per_tick), int(stage_states))
        h = ctypes.c_void_p()
        _check(lib.pint_server_create(ctypes.byref(cfg), _stream(stream), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            load().pint_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, plan_index, params, u0, u_slices):
        ok = 0 <= plan_index < len(self._plans)      # else the library refuses the index
        pl = self._plans[plan_index] if ok else None
        req = Request(int(plan_index), params, _ptr(u0, pl.state_numel() if ok else None),
                      _ptr(u_slices, pl.state_numel(params.n_intervals + 1) if ok else None))
        rid = ctypes.c_longlong()
        _check(load().pint_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._keep[rid.value] = (u0, u_slices)      # device buffers outlive the request
        return rid.value

    def tick(self):
        n = ctypes.c_int()
        _check(load().pint_server_tick(self._h, ctypes.byref(n)))
        return n.value

    def status(self, rid):
        st = RequestStatus()
        _check(load().pint_server_status(self._h, int(rid), ctypes.byref(st)))
        return st

    def clock(self):
        t = ctypes.c_double()
        _check(load().pint_server_clock(self._h, ctypes.byref(t)))
        return t.value

    def run(self, max_ticks=1 << 30):
        """Tick until nothing is queued or running; returns the tick count."""
        for i in range(max_ticks):
            if self.tick() == 0:
                return i + 1
        raise RuntimeError("server did not drain")


def stability_map(out, kind, coarse, xl, re_range, im_range, n=100, k=5, cfactor=2, n_c=1,
                  nrelax=0, n_ks=20, stream=None):
    """out (device [nim][nre] float64) <- max |A| on the xi_N grid (see
    pint_stability_map); kind "scheme" or "mgrit", coarse "imex" or "settls";
    re_range / im_range = (first, last)."""
    nim, nre = out.shape
    cfg = StabilityCfg({"scheme": 0, "mgrit": 1}[kind], {"imex": 0, "settls": 1}[coarse],
                       complex(xl).real, complex(xl).imag, re_range[0], re_range[1], nre,
                       im_range[0], im_range[1], nim, n, k, cfactor, n_c, nrelax, n_ks)
    _check(load().pint_stability_map(ctypes.byref(cfg), _ptr(out), _stream(stream)))
