"""ctypes binding of libgdw (the C ABI in include/gdw.h).

Argument marshalling only: every step of the time loop runs in the HIP kernels of
libgdw.so.  Torch is used for device memory and for the current HIP stream.  If
the library has not been built this module raises at import time -- there is no
CPU fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GDW_LIB") or os.path.join(_HERE, "libgdw.so")

GDW_OK, GDW_EINVAL, GDW_ENOMEM, GDW_EHIP, GDW_ENOCONV, GDW_ENONFINITE, GDW_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
GDW_FLUX_CENTRAL, GDW_FLUX_UPWIND, GDW_FLUX_ALTERNATING = 0, 1, 2
GDW_FP64, GDW_MIXED_FP32, GDW_MIXED_PC32 = 0, 1, 2
GDW_SOLVE_AUTO, GDW_SOLVE_FDM, GDW_SOLVE_PCG = 0, 1, 2
GDW_BC_PERIODIC, GDW_BC_DIRICHLET, GDW_BC_NEUMANN = 0, 1, 2
_BC = {"periodic": GDW_BC_PERIODIC, "dirichlet": GDW_BC_DIRICHLET, "neumann": GDW_BC_NEUMANN}

_STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOCONV",
                 -5: "ENONFINITE", -6: "EUNSUPPORTED"}


class gdw_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("N", ctypes.c_int),
                ("p", ctypes.c_int), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("c2", ctypes.c_double),
                ("flux", ctypes.c_int), ("xi", ctypes.c_double), ("precision", ctypes.c_int),
                ("solver", ctypes.c_int), ("coeff_variable", ctypes.c_int), ("mapped", ctypes.c_int),
                ("pcg_rtol", ctypes.c_double), ("pcg_maxit", ctypes.c_int),
                ("bc", ctypes.c_int * 4), ("dim", ctypes.c_int), ("nz", ctypes.c_int),
                ("z0", ctypes.c_double), ("Lz", ctypes.c_double), ("bcz", ctypes.c_int * 2)]


class gdw_stats(ctypes.Structure):
    _fields_ = [("steps_taken", ctypes.c_longlong), ("dof_updates", ctypes.c_longlong),
                ("n1", ctypes.c_int), ("precision", ctypes.c_int), ("solver", ctypes.c_int),
                ("fail_elem", ctypes.c_int), ("mean_it_S", ctypes.c_double),
                ("mean_it_M", ctypes.c_double), ("max_it_S", ctypes.c_int), ("max_it_M", ctypes.c_int),
                ("solves", ctypes.c_longlong), ("mean_refine", ctypes.c_double)]


class GdwError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__("%s: %s (%s)" % (where, _STATUS_NAMES.get(status, status), msg))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgdw.so is not built (run `python -m paper_2105_01722_amd.build`); "
                          "there is no CPU fallback")
    # The library receives torch's device pointers and streams, so it must run on the HIP
    # runtime torch has loaded.  torch ships its own libamdhip64.so.7 and HSA runtime;
    # importing torch first makes the dynamic loader bind the library's libamdhip64.so.7
    # dependency to that copy.  Loaded the other way round, the process would hold two HSA
    # runtimes, and the second one to start reports that no GPU is present.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, None
    sig = {
        "gdw_version": (ctypes.c_char_p, []),
        "gdw_last_error": (ctypes.c_char_p, []),
        "gdw_create": (I, [ctypes.POINTER(gdw_desc), ctypes.POINTER(P)]),
        "gdw_set_coeff": (I, [P, P, P, P, P]),
        "gdw_set_state": (I, [P, P, P, P]),
        "gdw_set_forcing": (I, [P, I, P, ctypes.POINTER(D), ctypes.POINTER(D), P]),
        "gdw_run": (I, [P, D, I, P]),
        "gdw_get_state": (I, [P, P, P, P]),
        "gdw_energy": (I, [P, ctypes.POINTER(D), P]),
        "gdw_get_stats": (I, [P, ctypes.POINTER(gdw_stats), P]),
        "gdw_destroy": (V, [P]),
        "gdw_mlp_create": (I, [I, I, I, ctypes.c_ulonglong, I, ctypes.POINTER(P)]),
        "gdw_mlp_num_params": (I, [P, ctypes.POINTER(ctypes.c_longlong)]),
        "gdw_mlp_get_params": (I, [P, P]),
        "gdw_mlp_set_params": (I, [P, P]),
        "gdw_mlp_forward": (I, [P, P, I, P, P]),
        "gdw_mlp_grad": (I, [P, P, P, I, P, ctypes.POINTER(D), P]),
        "gdw_mlp_grad_noalloc": (I, [P, P, P, I, P, P, P]),
        "gdw_mlp_train": (I, [P, P, P, I, I, I, ctypes.c_float, P, P]),
        "gdw_mlp_destroy": (V, [P]),
        "gdw_precond_data": (I, [P, P, P, P]),
        "gdw_set_precond_mlp": (I, [P, P, P]),
        "gdw_set_precond_log": (I, [P, P, P]),
        "gdw_ic0_solve": (I, [P, I, P, P, D, I, P, P]),
        "gdw_batch_create": (I, [I, ctypes.POINTER(gdw_desc), ctypes.POINTER(P)]),
        "gdw_batch_ctx": (I, [P, I, ctypes.POINTER(P)]),
        "gdw_batch_tune": (I, [P, ctypes.POINTER(D), P]),
        "gdw_batch_run": (I, [P, ctypes.POINTER(D), I, P]),
        "gdw_batch_step_times": (I, [P, ctypes.POINTER(ctypes.c_float), I]),
        "gdw_batch_plan": (ctypes.c_char_p, [P]),
        "gdw_batch_destroy": (V, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(status, where):
    if status != GDW_OK:
        raise GdwError(status, where, lib.gdw_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous float64 tensor with %d entries" % (name, n))
    return ctypes.c_void_p(t.data_ptr())


# --- thin wrappers with the C names ---------------------------------------------------
def gdw_version():
    return lib.gdw_version().decode()


def gdw_create(desc):
    ctx = ctypes.c_void_p()
    _check(lib.gdw_create(ctypes.byref(desc), ctypes.byref(ctx)), "gdw_create")
    return ctx


def gdw_set_coeff(ctx, c2_ptr, X_ptr, Y_ptr, stream=None):
    _check(lib.gdw_set_coeff(ctx, c2_ptr, X_ptr, Y_ptr, _stream(stream)), "gdw_set_coeff")


def gdw_set_state(ctx, U_ptr, V_ptr, stream=None):
    _check(lib.gdw_set_state(ctx, U_ptr, V_ptr, _stream(stream)), "gdw_set_state")


def gdw_run(ctx, dt, steps, stream=None):
    _check(lib.gdw_run(ctx, float(dt), int(steps), _stream(stream)), "gdw_run")


def gdw_get_state(ctx, U_ptr, V_ptr, stream=None):
    _check(lib.gdw_get_state(ctx, U_ptr, V_ptr, _stream(stream)), "gdw_get_state")


def gdw_energy(ctx, stream=None):
    e = ctypes.c_double()
    _check(lib.gdw_energy(ctx, ctypes.byref(e), _stream(stream)), "gdw_energy")
    return e.value


def gdw_get_stats(ctx, stream=None, check=True):
    s = gdw_stats()
    st = lib.gdw_get_stats(ctx, ctypes.byref(s), _stream(stream))
    out = {f: getattr(s, f) for f, _ in gdw_stats._fields_}
    out["status"] = st
    if check:
        _check(st, "gdw_get_stats")
    return out


def gdw_destroy(ctx):
    lib.gdw_destroy(ctx)


# --- convenience wrapper -----------------------------------------------------------------
def make_desc(nx, ny, N, p, c2=1.0, flux="central", xi=1.0, precision="fp64", solver="auto",
              Lx=1.0, Ly=1.0, x0=0.0, y0=0.0, coeff_variable=False, mapped=False,
              pcg_rtol=1e-12, pcg_maxit=200, bc=("periodic",) * 4, nz=0, z0=0.0, Lz=1.0,
              bcz=("periodic",) * 2):
    """A gdw_desc from keyword arguments (names as in include/gdw.h); bc: the kinds of
    the E, W, N, S sides ("periodic", "dirichlet", "neumann" or the gdw_bc values).
    nz > 0 makes a 3D problem of nx x ny x nz box elements (bcz: the T, B sides)."""
    d = gdw_desc()
    d.nx, d.ny, d.N, d.p = nx, ny, N, p
    d.x0, d.y0, d.Lx, d.Ly = x0, y0, Lx, Ly
    d.c2 = c2
    d.flux = {"central": GDW_FLUX_CENTRAL, "upwind": GDW_FLUX_UPWIND,
              "alternating": GDW_FLUX_ALTERNATING}[flux]
    d.xi = xi
    d.precision = {"fp64": GDW_FP64, "fp32": GDW_MIXED_FP32, "mixed": GDW_MIXED_FP32,
                   "pc32": GDW_MIXED_PC32}[precision]
    d.solver = {"auto": GDW_SOLVE_AUTO, "fdm": GDW_SOLVE_FDM, "pcg": GDW_SOLVE_PCG}[solver]
    d.coeff_variable = int(bool(coeff_variable))
    d.mapped = int(bool(mapped))
    d.pcg_rtol = pcg_rtol
    d.pcg_maxit = pcg_maxit
    if len(bc) != 4:
        raise ValueError("bc: four side kinds (E, W, N, S)")
    for k, b in enumerate(bc):
        d.bc[k] = _BC[b] if isinstance(b, str) else int(b)
    if nz:
        d.dim, d.nz, d.z0, d.Lz = 3, nz, z0, Lz
        if len(bcz) != 2:
            raise ValueError("bcz: two side kinds (T, B)")
        for k, b in enumerate(bcz):
            d.bcz[k] = _BC[b] if isinstance(b, str) else int(b)
    return d


class Solver:
    """One problem: nx x ny elements (periodic unless walls are given), N cells, odd degree
    p (see include/gdw.h)."""

    def __init__(self, nx, ny, N, p, **kw):
        self._attach(make_desc(nx, ny, N, p, **kw), None)

    def _attach(self, d, ctx):
        self.desc = d
        if d.dim == 3:
            self.shape = (d.nz, d.ny, d.nx, d.N + 1, d.N + 1, d.N + 1)
        else:
            self.shape = (d.ny, d.nx, d.N + 1, d.N + 1)
        self.n = 1
        for k in self.shape:
            self.n *= k
        self._owned = ctx is None
        self.ctx = gdw_create(d) if ctx is None else ctx

    @classmethod
    def view(cls, desc, ctx):
        """A Solver on a context owned elsewhere (a batch member); close() does not free it."""
        s = cls.__new__(cls)
        s._attach(desc, ctx)
        return s

    def set_state(self, U, V, stream=None):
        import torch
        U = torch.as_tensor(U, dtype=torch.float64, device="cuda").contiguous()
        V = torch.as_tensor(V, dtype=torch.float64, device="cuda").contiguous()
        gdw_set_state(self.ctx, _dptr(U, self.n, "U"), _dptr(V, self.n, "V"), stream)
        self._keep = (U, V)  # alive until the queued copy has run

    def set_coeff(self, c2=None, X=None, Y=None, stream=None):
        """Nodal c^2 and node coordinates (None = constant c^2 / Cartesian nodes)."""
        import torch
        keep, ptrs = [], []
        for name, a in (("c2", c2), ("X", X), ("Y", Y)):
            if a is None:
                ptrs.append(None)
                continue
            t = torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
            keep.append(t)
            ptrs.append(_dptr(t, self.n, name))
        gdw_set_coeff(self.ctx, *ptrs, stream=stream)
        torch.cuda.current_stream().synchronize() if stream is None else None
        self._keep_coeff = keep

    def set_forcing(self, terms, stream=None):
        """Source term f = sum_k sin(omega_k t + phase_k) g_k (include/gdw.h,
        gdw_set_forcing): terms is a list of (g_nodal, omega, phase), at most 4; [] removes
        it.  t counts from the last set_state."""
        import torch
        k = len(terms)
        if k == 0:
            _check(lib.gdw_set_forcing(self.ctx, 0, None, None, None, _stream(stream)),
                   "gdw_set_forcing")
            return
        g = torch.stack([torch.as_tensor(t[0], dtype=torch.float64).reshape(self.shape)
                         for t in terms]).to("cuda").contiguous()
        om = (ctypes.c_double * k)(*[float(t[1]) for t in terms])
        ph = (ctypes.c_double * k)(*[float(t[2]) for t in terms])
        _check(lib.gdw_set_forcing(self.ctx, k, ctypes.c_void_p(g.data_ptr()), om, ph,
                                   _stream(stream)), "gdw_set_forcing")

    def precond_data(self, stream=None):
        """(samples [n_el, 64], targets [n_el, (N+1)^2 - 1]) as float32 CUDA tensors."""
        import torch
        nel = self.desc.nx * self.desc.ny
        nn = (self.desc.N + 1) ** 2
        smp = torch.empty((nel, 64), dtype=torch.float32, device="cuda")
        tgt = torch.empty((nel, nn - 1), dtype=torch.float32, device="cuda")
        _check(lib.gdw_precond_data(self.ctx, ctypes.c_void_p(smp.data_ptr()),
                                    ctypes.c_void_p(tgt.data_ptr()), _stream(stream)),
               "gdw_precond_data")
        return smp, tgt

    def ic0_solve(self, op, b, rtol=1e-12, maxit=200, stream=None):
        """IC(0)-PCG solve of every element system (op 0: S_hat, op 1: M_J) for the
        right-hand sides b [n_el, (N+1)^2] (float64 CUDA tensor); returns (x, its)."""
        import torch
        d = self.desc
        nel, nn = d.nx * d.ny, (d.N + 1) ** 2
        bp = _dptr(b, nel * nn, "b")
        x = torch.empty((nel, nn), dtype=torch.float64, device="cuda")
        its = torch.empty(nel, dtype=torch.int32, device="cuda")
        _check(lib.gdw_ic0_solve(self.ctx, int(op), bp, ctypes.c_void_p(x.data_ptr()),
                                 float(rtol), int(maxit), ctypes.c_void_p(its.data_ptr()),
                                 _stream(stream)), "gdw_ic0_solve")
        return x, its

    def set_precond_log(self, o=None, stream=None):
        import torch
        if o is None:
            _check(lib.gdw_set_precond_log(self.ctx, None, _stream(stream)), "gdw_set_precond_log")
            return
        d = self.desc
        n = d.nx * d.ny * ((d.N + 1) ** 2 - 1)
        o = torch.as_tensor(o, dtype=torch.float32, device="cuda").contiguous()
        if o.numel() != n:
            raise ValueError("log_scale must hold nx * ny * ((N+1)^2 - 1) = %d entries, got %d"
                             % (n, o.numel()))
        _check(lib.gdw_set_precond_log(self.ctx, ctypes.c_void_p(o.data_ptr()), _stream(stream)),
               "gdw_set_precond_log")
        torch.cuda.current_stream().synchronize()

    def set_precond_mlp(self, net, stream=None):
        _check(lib.gdw_set_precond_mlp(self.ctx, net.h, _stream(stream)), "gdw_set_precond_mlp")

    def run(self, dt, steps, stream=None):
        gdw_run(self.ctx, dt, steps, stream)

    def get_state(self, stream=None):
        import torch
        U = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        V = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        gdw_get_state(self.ctx, _dptr(U, self.n, "U"), _dptr(V, self.n, "V"), stream)
        return U, V

    def energy(self, stream=None):
        return gdw_energy(self.ctx, stream)

    def stats(self, stream=None, check=True):
        return gdw_get_stats(self.ctx, stream, check)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            if self._owned:
                gdw_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The preconditioner-correction network (include/gdw.h, gdw_mlp_*)."""

    def __init__(self, n_in=64, hidden=128, n_out=168, seed=0, max_batch=4096):
        self.h = ctypes.c_void_p()
        _check(lib.gdw_mlp_create(n_in, hidden, n_out, seed, max_batch, ctypes.byref(self.h)),
               "gdw_mlp_create")
        n = ctypes.c_longlong()
        _check(lib.gdw_mlp_num_params(self.h, ctypes.byref(n)), "gdw_mlp_num_params")
        self.n_in, self.hidden, self.n_out, self.np = n_in, hidden, n_out, n.value

    def get_params(self):
        import numpy as np
        a = np.empty(self.np, dtype=np.float32)
        _check(lib.gdw_mlp_get_params(self.h, a.ctypes.data_as(ctypes.c_void_p)), "gdw_mlp_get_params")
        return a

    def set_params(self, theta):
        import numpy as np
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.np
        _check(lib.gdw_mlp_set_params(self.h, a.ctypes.data_as(ctypes.c_void_p)), "gdw_mlp_set_params")

    def forward(self, x, stream=None):
        import torch
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        out = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        _check(lib.gdw_mlp_forward(self.h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream)), "gdw_mlp_forward")
        return out

    def grad(self, x, y, stream=None):
        import torch
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        y = torch.as_tensor(y, dtype=torch.float32, device="cuda").contiguous()
        g = torch.empty(self.np, dtype=torch.float32, device="cuda")
        loss = ctypes.c_double()
        _check(lib.gdw_mlp_grad(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                x.shape[0], ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss),
                                _stream(stream)), "gdw_mlp_grad")
        return g, loss.value

    def grad_noalloc(self, x, y, grad, loss, stream=None):
        """gdw_mlp_grad_noalloc: gradient into `grad` (float32 CUDA tensor of num_params
        entries) and the loss into `loss` (float64 CUDA tensor of one entry), asynchronous,
        with no device allocation inside the library."""
        import torch
        for t, name, dt, k in ((x, "x", torch.float32, None), (y, "y", torch.float32, None),
                               (grad, "grad", torch.float32, self.np),
                               (loss, "loss", torch.float64, 1)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt \
                    or not t.is_contiguous() or (k is not None and t.numel() != k):
                raise ValueError("%s must be a contiguous %s CUDA tensor%s" % (
                    name, dt, "" if k is None else " of %d entries" % k))
        if x.dim() != 2 or x.shape[1] != self.n_in or y.shape != (x.shape[0], self.n_out):
            raise ValueError("x must be [n, %d] and y [n, %d]" % (self.n_in, self.n_out))
        _check(lib.gdw_mlp_grad_noalloc(self.h, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(y.data_ptr()), x.shape[0],
                                        ctypes.c_void_p(grad.data_ptr()),
                                        ctypes.c_void_p(loss.data_ptr()), _stream(stream)),
               "gdw_mlp_grad_noalloc")

    def train(self, x, y, epochs, batch=256, lr=1e-3, stream=None):
        import numpy as np
        import torch
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        y = torch.as_tensor(y, dtype=torch.float32, device="cuda").contiguous()
        losses = np.zeros(max(epochs, 1), dtype=np.float64)
        _check(lib.gdw_mlp_train(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 x.shape[0], epochs, batch, ctypes.c_float(lr),
                                 losses.ctypes.data_as(ctypes.c_void_p), _stream(stream)), "gdw_mlp_train")
        return losses[:epochs]

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            lib.gdw_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems advanced together (include/gdw.h, gdw_batch_*).

    problems: list of keyword dicts for make_desc (each with nx, ny, N, p, ...).
    `self.problems[i]` is a Solver view of problem i (set_coeff / set_state / get_state /
    energy / stats work on it as on a single problem)."""

    def __init__(self, problems):
        n = len(problems)
        descs = (gdw_desc * n)(*[make_desc(**p) for p in problems])
        self.h = ctypes.c_void_p()
        _check(lib.gdw_batch_create(n, descs, ctypes.byref(self.h)), "gdw_batch_create")
        self.problems = []
        for i in range(n):
            c = ctypes.c_void_p()
            _check(lib.gdw_batch_ctx(self.h, i, ctypes.byref(c)), "gdw_batch_ctx")
            self.problems.append(Solver.view(descs[i], c))
        self._steps = 0

    @staticmethod
    def _dt(dt, n):
        arr = (ctypes.c_double * n)(*[float(x) for x in dt])
        return arr

    def tune(self, dt, stream=None):
        _check(lib.gdw_batch_tune(self.h, self._dt(dt, len(self.problems)), _stream(stream)),
               "gdw_batch_tune")

    def run(self, dt, steps, stream=None):
        _check(lib.gdw_batch_run(self.h, self._dt(dt, len(self.problems)), int(steps),
                                 _stream(stream)), "gdw_batch_run")
        self._steps = int(steps)

    def step_times(self):
        ms = (ctypes.c_float * max(1, self._steps))()
        _check(lib.gdw_batch_step_times(self.h, ms, self._steps), "gdw_batch_step_times")
        return [ms[i] for i in range(self._steps)]

    def plan(self):
        return lib.gdw_batch_plan(self.h).decode()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            for p in self.problems:
                p.ctx = None
            lib.gdw_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def header_symbols(header_path=None):
    """Names of the functions declared in include/gdw.h (for the export test)."""
    import re
    header_path = header_path or os.path.join(os.path.dirname(_HERE), "include", "gdw.h")
    src = open(header_path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gdw_[a-z_0-9]+)\s*\(", src)))

