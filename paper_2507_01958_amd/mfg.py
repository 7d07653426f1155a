"""Thin ctypes binding of libmfg (include/mfg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Vectors are torch float64 CUDA tensors (contiguous); their data pointers are
passed straight through. Functions keep the C names and raise MFGError on a
non-zero status (the status code is kept on the exception).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_long, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfg.so")

MFG_OK = 0
STATUS = {0: "MFG_OK", 1: "MFG_ERR_INVALID_ARG", 2: "MFG_ERR_UNSUPPORTED",
          3: "MFG_ERR_NOT_CONVERGED", 4: "MFG_ERR_BREAKDOWN", 5: "MFG_ERR_NONFINITE",
          6: "MFG_ERR_HIP", 7: "MFG_ERR_OOM"}
# one type on every axis, or (bc_x, bc_y) for d = 2
BC = {"periodic": 0, "neumann": 1, ("periodic", "periodic"): 0, ("neumann", "neumann"): 1,
      ("periodic", "neumann"): 2, ("neumann", "periodic"): 3}
PRECISION = {"fp64": 0, "mixed_fp32": 1, "mixed_fp16": 2, "mixed_bf16": 3}
COUPLING = {"linear": 0, "quadratic": 1, "potential": 2}


class MFGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("d", c_int), ("n", c_int * 2), ("nt", c_int), ("T", c_double),
                ("lo", c_double * 2), ("hi", c_double * 2), ("bc", c_int), ("nu", c_double),
                ("qprime", c_double), ("gamma", c_double), ("l", c_int), ("precision", c_int),
                ("coupling", c_int), ("beta", c_double)]


class State(ctypes.Structure):
    _fields_ = [("xi", c_void_p), ("y", c_void_p), ("ybar", c_void_p), ("sigma", c_double),
                ("tau", c_double), ("theta", c_double), ("iter", c_long)]


class Stats(ctypes.Structure):
    _fields_ = [("pcg_iters", POINTER(c_int)), ("pcg_relres", POINTER(c_double)),
                ("dm", POINTER(c_double)), ("mass_drift", POINTER(c_double))]


# name -> (restype, argtypes); the exported API of include/mfg.h
SIGNATURES = {
    "mfg_plan": (c_int, [POINTER(Problem), c_void_p, c_void_p, c_void_p, POINTER(c_void_p)]),
    "mfg_destroy": (c_int, [c_void_p]),
    "mfg_set_stream": (c_int, [c_void_p, c_void_p]),
    "mfg_set_data": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mfg_set_target": (c_int, [c_void_p, c_void_p]),
    "mfg_set_warm_start": (c_int, [c_void_p, c_int]),
    "mfg_value_function": (c_int, [c_void_p, POINTER(State), c_double, c_int, c_void_p]),
    "mfg_hjb_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mfg_prox": (c_int, [c_void_p, c_void_p, c_double, c_void_p]),
    "mfg_apply_AAt": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mfg_apply_C": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mfg_apply_CT": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mfg_precond": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mfg_pcg": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, POINTER(c_int),
                        POINTER(c_double)]),
    "mfg_cp_init": (c_int, [c_void_p, POINTER(State)]),
    "mfg_cp_solve": (c_int, [c_void_p, POINTER(State), c_int, c_double, c_int, POINTER(Stats)]),
    "mfg_cp_solve_tol": (c_int, [c_void_p, POINTER(State), c_int, c_double, c_int,
                                 POINTER(c_int), POINTER(Stats)]),
    "mfg_cp_adjoint": (c_int, [c_void_p, POINTER(State), c_int, c_int, c_int, c_void_p, c_double,
                               c_int, c_void_p, c_void_p]),
    "mfg_autotune": (c_int, [c_void_p, c_int]),
    "mfg_batch_autotune": (c_int, [c_void_p, c_int]),
    "mfg_plan_batch": (c_int, [POINTER(Problem), POINTER(c_void_p), POINTER(c_void_p), c_int,
                               c_void_p, POINTER(c_void_p)]),
    "mfg_batch_plan": (c_int, [c_void_p, c_int, POINTER(c_void_p)]),
    "mfg_batch_destroy": (c_int, [c_void_p]),
    "mfg_batch_cp_solve": (c_int, [c_void_p, POINTER(State), c_int, c_double, c_int, c_int,
                                   POINTER(c_int)]),
    "mfg_pcg_noalloc": (c_int, [POINTER(Problem), c_void_p, c_void_p, c_double, c_int, c_void_p,
                                POINTER(c_int), POINTER(c_double)]),
    "mfg_profile": (c_int, [c_void_p, c_int]),
    "mfg_profile_report": (c_int, [c_void_p, ctypes.c_char_p, c_int]),
    "mfg_last_error": (c_char_p, []),
    "mfg_version": (c_char_p, []),
}

_lib = None


def load():
    """Load libmfg.so (built in-tree by paper_2507_01958_amd.build), or the
    library file MFG_LIBRARY names (the host-AddressSanitizer build). Raises if
    it is missing: there is no fallback path."""
    global _lib
    if _lib is None:
        path = os.environ.get("MFG_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run `python -m paper_2507_01958_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, allow=()):
    if rc != MFG_OK and rc not in allow:
        raise MFGError(rc, load().mfg_last_error().decode())
    return rc


def _ptr(t):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def make_problem(d, nx, ny, nt, bc, nu, gamma, l=1, precision="fp64", T=1.0, lo=None, hi=None,
                 qprime=2.0, coupling="linear", beta=0.0) -> Problem:
    pb = Problem()
    pb.d = d
    pb.n[0] = nx
    pb.n[1] = ny if d == 2 else 1
    pb.nt = nt
    pb.T = T
    lo = lo or (0.0, 0.0)
    hi = hi or (1.0, 1.0)
    pb.lo[0], pb.lo[1] = lo[0], (lo[1] if len(lo) > 1 else 0.0)
    pb.hi[0], pb.hi[1] = hi[0], (hi[1] if len(hi) > 1 else 1.0)
    pb.bc = BC[bc] if isinstance(bc, str) else BC[tuple(bc)] if isinstance(bc, (tuple, list)) \
        else int(bc)
    pb.nu = nu
    pb.qprime = qprime
    pb.gamma = gamma
    pb.l = l
    pb.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    pb.coupling = COUPLING[coupling] if isinstance(coupling, str) else int(coupling)
    pb.beta = beta
    return pb


class Plan:
    """Owns an mfg_plan_t; use close() (or a with-block) to release it."""

    def __init__(self, problem: Problem, V, m0, stream=None, _handle=None):
        self._shape(problem)
        if _handle is not None:  # borrowed from a batch: not released here
            self.handle = _handle
            self._owned = False
            return
        h = c_void_p()
        _check(load().mfg_plan(ctypes.byref(problem), _ptr(V), _ptr(m0), _stream(stream),
                               ctypes.byref(h)))
        self.handle = h
        self._owned = True

    def _shape(self, problem):
        self.problem = problem
        self.d = problem.d
        self.nx, self.ny = problem.n[0], (problem.n[1] if problem.d == 2 else 1)
        self.nt = problem.nt
        self.M = self.nx * self.ny
        self.n = self.nt * self.M
        self.nprimal = (1 + 2 * self.d) * self.n

    def close(self):
        if self._owned and self.handle is not None and self.handle.value:
            _check(load().mfg_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mfg_plan(problem: Problem, V, m0, stream=None) -> Plan:
    return Plan(problem, V, m0, stream)


def mfg_destroy(plan: Plan):
    plan.close()


def mfg_set_stream(plan: Plan, stream):
    _check(load().mfg_set_stream(plan.handle, _stream(stream)))


def mfg_set_data(plan: Plan, V=None, m0=None):
    _check(load().mfg_set_data(plan.handle, _ptr(V), _ptr(m0)))


def mfg_set_target(plan: Plan, mbar):
    _check(load().mfg_set_target(plan.handle, _ptr(mbar)))


def mfg_set_warm_start(plan: Plan, enable: bool):
    _check(load().mfg_set_warm_start(plan.handle, 1 if enable else 0))


def mfg_prox(plan: Plan, v, tau: float, y):
    _check(load().mfg_prox(plan.handle, _ptr(v), float(tau), _ptr(y)))


def mfg_apply_AAt(plan: Plan, u, q):
    _check(load().mfg_apply_AAt(plan.handle, _ptr(u), _ptr(q)))


def mfg_apply_C(plan: Plan, y, b):
    _check(load().mfg_apply_C(plan.handle, _ptr(y), _ptr(b)))


def mfg_apply_CT(plan: Plan, u, y):
    _check(load().mfg_apply_CT(plan.handle, _ptr(u), _ptr(y)))


def mfg_precond(plan: Plan, r, z):
    _check(load().mfg_precond(plan.handle, _ptr(r), _ptr(z)))


def mfg_pcg(plan: Plan, b, u, rtol: float, maxit: int, true_residual: bool = True,
            raise_not_converged: bool = True):
    """Returns (iterations, true relative residual or None, status)."""
    its = c_int(0)
    rel = c_double(0.0)
    rc = load().mfg_pcg(plan.handle, _ptr(b), _ptr(u), float(rtol), int(maxit), ctypes.byref(its),
                        ctypes.byref(rel) if true_residual else None)
    _check(rc, allow=() if raise_not_converged else (3,))
    return its.value, (rel.value if true_residual else None), rc


def mfg_pcg_noalloc(problem: Problem, b, u, rtol: float, maxit: int, stream=None,
                    raise_not_converged: bool = True):
    """PCG without a plan or any device allocation. Returns (iterations, true
    relative residual, status)."""
    its = c_int(0)
    rel = c_double(0.0)
    rc = load().mfg_pcg_noalloc(ctypes.byref(problem), _ptr(b), _ptr(u), float(rtol), int(maxit),
                                _stream(stream), ctypes.byref(its), ctypes.byref(rel))
    _check(rc, allow=() if raise_not_converged else (3,))
    return its.value, rel.value, rc


class CPState:
    """Device tensors of the Chambolle-Pock state plus its scalars."""

    def __init__(self, plan: Plan, device=None):
        import torch
        dev = device or torch.device("cuda")
        self.xi = torch.zeros(plan.nprimal, dtype=torch.float64, device=dev)
        self.y = torch.zeros(plan.nprimal, dtype=torch.float64, device=dev)
        self.ybar = torch.zeros(plan.nprimal, dtype=torch.float64, device=dev)
        self.c = State()
        self._sync_ptrs()

    def _sync_ptrs(self):
        self.c.xi = self.xi.data_ptr()
        self.c.y = self.y.data_ptr()
        self.c.ybar = self.ybar.data_ptr()

    @property
    def sigma(self):
        return self.c.sigma

    @property
    def tau(self):
        return self.c.tau

    @property
    def iter(self):
        return self.c.iter

    def snapshot(self):
        return dict(xi=self.xi.clone(), y=self.y.clone(), ybar=self.ybar.clone(),
                    sigma=self.c.sigma, tau=self.c.tau, theta=self.c.theta, iter=self.c.iter)

    def restore(self, snap):
        self.xi.copy_(snap["xi"])
        self.y.copy_(snap["y"])
        self.ybar.copy_(snap["ybar"])
        self.c.sigma, self.c.tau, self.c.theta, self.c.iter = (snap["sigma"], snap["tau"],
                                                              snap["theta"], snap["iter"])


def mfg_cp_init(plan: Plan, st: CPState):
    st._sync_ptrs()
    _check(load().mfg_cp_init(plan.handle, ctypes.byref(st.c)))


def mfg_cp_solve(plan: Plan, st: CPState, n_iter: int, pcg_rtol: float, pcg_maxit: int,
                 stats: bool = True, raise_not_converged: bool = True, mass: bool = False):
    """Runs n_iter CP iterations; returns dict of per-iteration statistics
    (with mass=True also the mass drift, at one extra read of m per iteration)."""
    st._sync_ptrs()
    out = {}
    sp = None
    if stats and n_iter > 0:
        its = (c_int * n_iter)()
        rel = (c_double * n_iter)()
        dm = (c_double * n_iter)()
        md = (c_double * n_iter)()
        s = Stats()
        s.pcg_iters = ctypes.cast(its, POINTER(c_int))
        s.pcg_relres = ctypes.cast(rel, POINTER(c_double))
        s.dm = ctypes.cast(dm, POINTER(c_double))
        if mass:
            s.mass_drift = ctypes.cast(md, POINTER(c_double))
        sp = ctypes.byref(s)
    rc = load().mfg_cp_solve(plan.handle, ctypes.byref(st.c), int(n_iter), float(pcg_rtol),
                             int(pcg_maxit), sp)
    _check(rc, allow=() if raise_not_converged else (3,))
    if sp is not None:
        out = dict(pcg_iters=list(its), pcg_relres=list(rel), dm=list(dm))
        if mass:
            out["mass_drift"] = list(md)
    out["status"] = rc
    return out


def mfg_cp_solve_tol(plan: Plan, st: CPState, max_iter: int, cp_tol: float, pcg_maxit: int,
                     raise_not_converged: bool = True, mass: bool = False):
    """CP iterations with the Section 5 stopping and inner-tolerance rules;
    returns dict with n_done and the per-iteration statistics."""
    st._sync_ptrs()
    n = max(int(max_iter), 1)
    its = (c_int * n)()
    rel = (c_double * n)()
    dm = (c_double * n)()
    s = Stats()
    s.pcg_iters = ctypes.cast(its, POINTER(c_int))
    s.pcg_relres = ctypes.cast(rel, POINTER(c_double))
    s.dm = ctypes.cast(dm, POINTER(c_double))
    md = (c_double * n)()
    if mass:
        s.mass_drift = ctypes.cast(md, POINTER(c_double))
    done = c_int(0)
    rc = load().mfg_cp_solve_tol(plan.handle, ctypes.byref(st.c), int(max_iter), float(cp_tol),
                                 int(pcg_maxit), ctypes.byref(done), ctypes.byref(s))
    _check(rc, allow=() if raise_not_converged else (3,))
    k = done.value
    out = dict(n_done=k, pcg_iters=list(its)[:k], pcg_relres=list(rel)[:k], dm=list(dm)[:k],
               status=rc)
    if mass:
        out["mass_drift"] = list(md)[:k]
    return out


def mfg_cp_adjoint(plan: Plan, ckpts, every: int, n_iter: int, gy, pcg_rtol: float,
                   pcg_maxit: int, g_m0, g_V, raise_not_converged: bool = True):
    """ckpts: list of snapshot dicts (CPState.snapshot()) taken after 0, every,
    2*every, ... iterations. Writes g_m0 and g_V (float64 CUDA tensors, M values)."""
    arr = (State * len(ckpts))()
    for k, c in enumerate(ckpts):
        arr[k].xi = c["xi"].data_ptr()
        arr[k].y = c["y"].data_ptr()
        arr[k].ybar = c["ybar"].data_ptr()
        arr[k].sigma, arr[k].tau, arr[k].theta, arr[k].iter = (c["sigma"], c["tau"], c["theta"],
                                                               c["iter"])
    rc = load().mfg_cp_adjoint(plan.handle, arr, len(ckpts), int(every), int(n_iter), _ptr(gy),
                               float(pcg_rtol), int(pcg_maxit), _ptr(g_m0), _ptr(g_V))
    _check(rc, allow=() if raise_not_converged else (3,))
    return rc


def mfg_value_function(plan: Plan, st: "CPState", pcg_rtol: float, pcg_maxit: int, u,
                       raise_not_converged: bool = True):
    """Writes u ((N_t + 1) M values) from the state's multiplier; returns the status."""
    st._sync_ptrs()
    rc = load().mfg_value_function(plan.handle, ctypes.byref(st.c), float(pcg_rtol),
                                   int(pcg_maxit), _ptr(u))
    _check(rc, allow=() if raise_not_converged else (3,))
    return rc


def mfg_hjb_residual(plan: Plan, y, u, R):
    _check(load().mfg_hjb_residual(plan.handle, _ptr(y), _ptr(u), _ptr(R)))


class Batch:
    """Owns an mfg_batch_t; `plans[i]` are the instances' (borrowed) plans."""

    def __init__(self, problems, Vs, m0s, stream=None):
        n = len(problems)
        arr = (Problem * n)(*problems)
        vp = (c_void_p * n)(*[_ptr(v).value for v in Vs])
        mp = (c_void_p * n)(*[_ptr(m).value for m in m0s])
        h = c_void_p()
        _check(load().mfg_plan_batch(arr, vp, mp, n, _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.count = n
        self.plans = []
        for i in range(n):
            ph = c_void_p()
            _check(load().mfg_batch_plan(h, i, ctypes.byref(ph)))
            self.plans.append(Plan(problems[i], None, None, _handle=ph))

    def close(self):
        if self.handle is not None and self.handle.value:
            for p in self.plans:
                p.handle = None
            _check(load().mfg_batch_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mfg_plan_batch(problems, Vs, m0s, stream=None) -> Batch:
    return Batch(problems, Vs, m0s, stream)


def mfg_autotune(plan: Plan, effort: int = 1):
    _check(load().mfg_autotune(plan.handle, int(effort)))


def mfg_batch_autotune(batch: Batch, effort: int = 1):
    _check(load().mfg_batch_autotune(batch.handle, int(effort)))


def mfg_batch_destroy(batch: Batch):
    batch.close()


def mfg_batch_cp_solve(batch: Batch, states, n_iter: int, pcg_rtol: float, pcg_maxit: int,
                       use_graph: bool = True, raise_not_converged: bool = True):
    """Runs n_iter CP iterations on every instance (states: list of CPState);
    returns the PCG iteration counts as a list of per-iteration lists."""
    n = batch.count
    arr = (State * n)()
    for i, st in enumerate(states):
        st._sync_ptrs()
        arr[i] = st.c
    its = (c_int * max(1, n_iter * n))()
    rc = load().mfg_batch_cp_solve(batch.handle, arr, int(n_iter), float(pcg_rtol),
                                   int(pcg_maxit), 1 if use_graph else 0,
                                   ctypes.cast(its, POINTER(c_int)))
    for i, st in enumerate(states):
        st.c.sigma, st.c.tau, st.c.theta, st.c.iter = (arr[i].sigma, arr[i].tau, arr[i].theta,
                                                      arr[i].iter)
    _check(rc, allow=() if raise_not_converged else (3,))
    return [list(its[k * n:(k + 1) * n]) for k in range(n_iter)]


def mfg_profile(plan: Plan, enable: bool):
    _check(load().mfg_profile(plan.handle, 1 if enable else 0))


def mfg_profile_report(plan: Plan) -> dict:
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().mfg_profile_report(plan.handle, buf, len(buf)))
    return json.loads(buf.value.decode())


def mfg_last_error() -> str:
    return load().mfg_last_error().decode()


def mfg_version() -> str:
    return load().mfg_version().decode()
