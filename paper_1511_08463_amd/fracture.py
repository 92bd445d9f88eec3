"""Python binding of the C ABI in ``include/fracture.h`` (ctypes).

Argument marshalling only: every step of the solver runs in the HIP library
``libfracture.so``.  PyTorch supplies the device workspace and the stream.
The functions keep the C names; ``Fracture`` bundles them for convenience.
Importing this module does not load the library; the first call does, and
raises ``RuntimeError`` when it is missing (there is no fallback path).
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfracture.so")

FRACTURE_OK = 0
FRACTURE_EINVAL = -1
FRACTURE_ENOMEM = -2
FRACTURE_ENOTCONV = -3
FRACTURE_ENONFINITE = -4
FRACTURE_EDEVICE = -5
FRACTURE_ESCRATCH = -6

FRACTURE_AT1 = 1
FRACTURE_AT2 = 2
FRACTURE_LOAD_TENSION_2D = 0
FRACTURE_LOAD_THERMAL_3D = 1
FRACTURE_LOAD_SURFING_2D = 2
FRACTURE_LOAD_THERMAL_SHOCK_2D = 3
FRACTURE_RELAX_PROJECT = 0
FRACTURE_RELAX_RATIO = 1
FRACTURE_RELAX_BISECT = 2
FRACTURE_STOP_DALPHA = 0
FRACTURE_STOP_PHI = 1
FRACTURE_FP64 = 0
FRACTURE_MIXED = 1

FRACTURE_STAGE_NONE = 0
FRACTURE_STAGE_PCG = 1
FRACTURE_STAGE_VI = 2
FRACTURE_STAGE_VI_SEARCH = 3
FRACTURE_STAGE_NEWTON = 4
FRACTURE_STAGE_SWEEPS = 5
FRACTURE_STAGE_OTHER = 6

FRACTURE_OP_ELASTICITY = 0
FRACTURE_OP_LEVEL = 1
FRACTURE_OP_DAMAGE_HESS = 2
FRACTURE_OP_COUPLING = 3
FRACTURE_OP_COUPLING_T = 4
FRACTURE_OP_PRECOND = 5
FRACTURE_OP_RESIDUAL = 6

FRACTURE_KERNEL_APPLY = 0
FRACTURE_KERNEL_SMOOTH = 1
FRACTURE_KERNEL_VI_EVAL = 2
FRACTURE_KERNEL_HELM = 3
FRACTURE_KERNEL_COPY = 4


class fracture_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("model", ctypes.c_int), ("plane_stress", ctypes.c_int),
        ("E", ctypes.c_double), ("nu", ctypes.c_double), ("Gc", ctypes.c_double),
        ("ell", ctypes.c_double), ("k_ell", ctypes.c_double),
        ("load_kind", ctypes.c_int), ("thermal_depth", ctypes.c_double),
        ("surf_ki", ctypes.c_double), ("surf_v", ctypes.c_double), ("surf_lc", ctypes.c_double),
        ("precision", ctypes.c_int), ("omega", ctypes.c_double), ("relax_mode", ctypes.c_int),
        ("newton", ctypes.c_int), ("am_stop", ctypes.c_int), ("am_tol", ctypes.c_double),
        ("switch_tol", ctypes.c_double), ("switch_rel", ctypes.c_double),
        ("final_tol", ctypes.c_double), ("pcg_rtol", ctypes.c_double), ("vi_tol", ctypes.c_double),
        ("vi_cg_rtol", ctypes.c_double), ("minres_rtol", ctypes.c_double),
        ("max_am", ctypes.c_int), ("max_pcg", ctypes.c_int), ("max_vi", ctypes.c_int),
        ("max_vi_cg", ctypes.c_int), ("max_newton", ctypes.c_int), ("max_minres", ctypes.c_int),
        ("cheb_degree", ctypes.c_int), ("coarse_max_dofs", ctypes.c_int),
        ("newton_vcycles", ctypes.c_int), ("newton_forcing", ctypes.c_double),
        ("use_graphs", ctypes.c_int), ("vcycle_tail", ctypes.c_int),
        ("newton_precond", ctypes.c_int), ("newton_forcing_mode", ctypes.c_int),
        ("pcg_reduction", ctypes.c_double), ("newton_stall", ctypes.c_double),
        ("omega_auto", ctypes.c_int),
        ("thermal_dT", ctypes.c_double),
        ("deflate", ctypes.c_int), ("deflate_theta", ctypes.c_double),
        ("deflate_min_nodes", ctypes.c_int), ("deflate_max_fragments", ctypes.c_int),
        ("vi_reduction", ctypes.c_double), ("elem3d_min_nodes", ctypes.c_int),
    ]


class fracture_stats(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int), ("pcg_iters", ctypes.c_int), ("vi_iters", ctypes.c_int),
        ("vi_cg_iters", ctypes.c_int), ("newton_iters", ctypes.c_int),
        ("newton_failures", ctypes.c_int), ("minres_iters", ctypes.c_int),
        ("converged", ctypes.c_int), ("dalpha_inf", ctypes.c_double), ("phi_l2", ctypes.c_double),
        ("ms_total", ctypes.c_double), ("ms_pcg", ctypes.c_double), ("ms_vi", ctypes.c_double),
        ("ms_newton", ctypes.c_double), ("stopped_in", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "fracture_default_params", "fracture_workspace_bytes", "fracture_sizes", "fracture_create",
    "fracture_set_load", "fracture_solve_step", "fracture_solve_steps", "fracture_energy",
    "fracture_get_state", "fracture_set_state", "fracture_apply", "fracture_update_coefficients",
    "fracture_gradient", "fracture_levels", "fracture_level_shape", "fracture_strerror",
    "fracture_time_kernel", "fracture_kernel_timing", "fracture_kernel_timing_read",
    "fracture_set_monitor", "fracture_fragments", "fracture_deflation_matrix",
    "fracture_destroy", "fracture_energy_noalloc",
]

MONITOR_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double)

_lib = None


def load_library(path=LIB_PATH):
    """Load ``libfracture.so`` and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname; load it first so
    # that this library binds to it and device pointers from torch tensors
    # belong to the runtime the library calls.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    dp = P(ctypes.c_double)
    sig = {
        "fracture_default_params": (None, [P(fracture_params), ctypes.c_int, ctypes.c_int]),
        "fracture_workspace_bytes": (ctypes.c_size_t, [P(fracture_params)]),
        "fracture_sizes": (ctypes.c_int, [P(fracture_params), P(ctypes.c_int64), P(ctypes.c_int64)]),
        "fracture_create": (ctypes.c_int, [P(fracture_params), vp, vp, ctypes.c_size_t, vp, P(vp)]),
        "fracture_set_load": (ctypes.c_int, [vp, ctypes.c_double]),
        "fracture_solve_step": (ctypes.c_int, [vp, P(fracture_stats)]),
        "fracture_solve_steps": (ctypes.c_int, [P(vp), ctypes.c_int, P(fracture_stats), P(ctypes.c_int)]),
        "fracture_energy": (ctypes.c_int, [vp, dp, dp]),
        "fracture_energy_noalloc": (ctypes.c_int, [P(fracture_params), ctypes.c_double, vp, vp, vp, vp]),
        "fracture_get_state": (ctypes.c_int, [vp, vp, vp, vp]),
        "fracture_set_state": (ctypes.c_int, [vp, vp, vp, vp]),
        "fracture_apply": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp]),
        "fracture_update_coefficients": (ctypes.c_int, [vp]),
        "fracture_gradient": (ctypes.c_int, [vp, vp, vp]),
        "fracture_levels": (ctypes.c_int, [vp, P(ctypes.c_int)]),
        "fracture_level_shape": (ctypes.c_int, [vp, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int)]),
        "fracture_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "fracture_time_kernel": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, dp, dp]),
        "fracture_kernel_timing": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int]),
        "fracture_kernel_timing_read": (ctypes.c_int, [vp, P(ctypes.c_int), dp, dp]),
        "fracture_set_monitor": (ctypes.c_int, [vp, MONITOR_FN, vp]),
        "fracture_fragments": (ctypes.c_int, [vp, P(ctypes.c_int), vp]),
        "fracture_deflation_matrix": (ctypes.c_int, [vp, P(ctypes.c_int), dp]),
        "fracture_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FractureError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = load_library().fracture_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")


def _check(code, where):
    if code != FRACTURE_OK:
        raise FractureError(code, where)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def fracture_default_params(nx, ny):
    p = fracture_params()
    load_library().fracture_default_params(ctypes.byref(p), nx, ny)
    return p


def make_params(**kw):
    """fracture_params from the documented defaults overridden by keywords
    (model may be given as "AT1"/"AT2")."""
    p = fracture_default_params(kw.get("nx", 64), kw.get("ny", 64))
    for k, v in kw.items():
        if k == "model" and isinstance(v, str):
            v = FRACTURE_AT1 if v == "AT1" else FRACTURE_AT2
        if k == "precision" and isinstance(v, str):
            v = FRACTURE_MIXED if v == "mixed" else FRACTURE_FP64
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def fracture_workspace_bytes(p):
    return load_library().fracture_workspace_bytes(ctypes.byref(p))


def fracture_sizes(p):
    n, d = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().fracture_sizes(ctypes.byref(p), ctypes.byref(n), ctypes.byref(d)), "fracture_sizes")
    return n.value, d.value


# ---------------------------------------------------------------------------
# the C entry points, by name
# ---------------------------------------------------------------------------

def fracture_create(p, notch_mask, workspace_ptr, ws_bytes, stream_ptr):
    lib = load_library()
    h = ctypes.c_void_p()
    if notch_mask is not None:
        notch_mask = np.ascontiguousarray(notch_mask, dtype=np.uint8)
        nm = notch_mask.ctypes.data_as(ctypes.c_void_p)
    else:
        nm = None
    _check(lib.fracture_create(ctypes.byref(p), nm, ctypes.c_void_p(workspace_ptr), ws_bytes,
                               ctypes.c_void_p(stream_ptr), ctypes.byref(h)), "fracture_create")
    return h


def fracture_set_load(h, load):
    _check(load_library().fracture_set_load(h, float(load)), "fracture_set_load")


def fracture_solve_step(h):
    st = fracture_stats()
    code = load_library().fracture_solve_step(h, ctypes.byref(st))
    return code, st.as_dict()


def fracture_solve_steps(hs):
    n = len(hs)
    arr = (ctypes.c_void_p * n)(*[h.value for h in hs])
    stats = (fracture_stats * n)()
    codes = (ctypes.c_int * n)()
    load_library().fracture_solve_steps(arr, n, stats, codes)
    return list(codes), [s.as_dict() for s in stats]


def fracture_energy_noalloc(p, load, d_u, d_alpha, stream, d_out):
    """Energies of the state (d_u, d_alpha) into d_out[0:2] (device pointers,
    as ints), queued on ``stream`` without any allocation."""
    _check(load_library().fracture_energy_noalloc(ctypes.byref(p), float(load), d_u, d_alpha,
                                                  stream, d_out), "fracture_energy_noalloc")


def fracture_energy(h):
    el, su = ctypes.c_double(), ctypes.c_double()
    _check(load_library().fracture_energy(h, ctypes.byref(el), ctypes.byref(su)), "fracture_energy")
    return el.value, su.value


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.dtype == np.float64 and a.flags.c_contiguous
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


def fracture_get_state(h, u, alpha, alpha_prev):
    _check(load_library().fracture_get_state(h, _ptr(u), _ptr(alpha), _ptr(alpha_prev)), "fracture_get_state")


def fracture_set_state(h, u, alpha, alpha_prev):
    _check(load_library().fracture_set_state(h, _ptr(u), _ptr(alpha), _ptr(alpha_prev)), "fracture_set_state")


def fracture_apply(h, op, level, x, y):
    _check(load_library().fracture_apply(h, op, level, _ptr(x), _ptr(y)), "fracture_apply")


def fracture_update_coefficients(h):
    _check(load_library().fracture_update_coefficients(h), "fracture_update_coefficients")


def fracture_gradient(h, Eu, Ea):
    _check(load_library().fracture_gradient(h, _ptr(Eu), _ptr(Ea)), "fracture_gradient")


def fracture_fragments(h, fid):
    """Fragments of the current alpha: their number; fid (device int32
    tensor of N) receives each node's fragment index or -1."""
    n = ctypes.c_int()
    _check(load_library().fracture_fragments(h, ctypes.byref(n), _ptr(fid)), "fracture_fragments")
    return n.value


def fracture_deflation_matrix(h):
    """E = W^T K W of the current fragments as an m x m float64 array."""
    m = ctypes.c_int()
    buf = (ctypes.c_double * (24 * 24))()
    _check(load_library().fracture_deflation_matrix(h, ctypes.byref(m), buf),
           "fracture_deflation_matrix")
    return np.frombuffer(buf, dtype=np.float64)[: m.value * m.value].reshape(m.value, m.value).copy()


def fracture_levels(h):
    n = ctypes.c_int()
    _check(load_library().fracture_levels(h, ctypes.byref(n)), "fracture_levels")
    return n.value


def fracture_level_shape(h, level):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().fracture_level_shape(h, level, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "fracture_level_shape")
    return a.value, b.value, c.value


def fracture_time_kernel(h, kernel, reps):
    ms, b = ctypes.c_double(), ctypes.c_double()
    _check(load_library().fracture_time_kernel(h, kernel, reps, ctypes.byref(ms), ctypes.byref(b)),
           "fracture_time_kernel")
    return ms.value, b.value


def fracture_kernel_timing(h, kernel, capacity):
    _check(load_library().fracture_kernel_timing(h, kernel, capacity), "fracture_kernel_timing")


def fracture_kernel_timing_read(h):
    """(count, total_ms, total_bytes) of the timed launches since the last read."""
    n, ms, b = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().fracture_kernel_timing_read(h, ctypes.byref(n), ctypes.byref(ms),
                                                      ctypes.byref(b)),
           "fracture_kernel_timing_read")
    return n.value, ms.value, b.value


def fracture_set_monitor(h, fn):
    """fn(sweep, dalpha_inf, phi_l2) or None; returns the ctypes callback,
    which the caller must keep alive while it is installed."""
    cb = MONITOR_FN(lambda user, sweep, da, phi: fn(sweep, da, phi)) if fn else MONITOR_FN()
    _check(load_library().fracture_set_monitor(h, cb, None), "fracture_set_monitor")
    return cb


def fracture_destroy(h):
    load_library().fracture_destroy(h)


# ---------------------------------------------------------------------------
# convenience wrapper: torch owns the workspace and the stream
# ---------------------------------------------------------------------------

class Fracture:
    """One solver instance on a CUDA (HIP) device."""

    def __init__(self, params, notch_mask=None, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.params = params
        self.device = torch.device(device)
        self.N, self.ndof = fracture_sizes(params)
        self.ws_bytes = fracture_workspace_bytes(params)
        if self.ws_bytes == 0:
            raise FractureError(FRACTURE_EINVAL, "fracture_workspace_bytes")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.h = fracture_create(params, notch_mask, aligned, self.ws_bytes, self.stream.cuda_stream)

    def close(self):
        if self.h is not None:
            fracture_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_monitor(self, fn):
        self._monitor_cb = fracture_set_monitor(self.h, fn)

    def set_load(self, t):
        fracture_set_load(self.h, t)

    def solve_step(self, raise_on_error=True):
        code, st = fracture_solve_step(self.h)
        if raise_on_error and code != FRACTURE_OK:
            raise FractureError(code, "fracture_solve_step")
        st["code"] = code
        return st

    def energy(self):
        return fracture_energy(self.h)

    def state(self):
        u = np.empty(self.ndof)
        a = np.empty(self.N)
        ap = np.empty(self.N)
        fracture_get_state(self.h, u, a, ap)
        return u, a, ap

    def set_state(self, u=None, alpha=None, alpha_prev=None):
        conv = lambda v: None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        fracture_set_state(self.h, conv(u), conv(alpha), conv(alpha_prev))

    def apply(self, op, x, level=0, out_len=None):
        torch = self.torch
        xt = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=self.device)
        if out_len is None:
            out_len = xt.numel()
        yt = torch.empty(out_len, dtype=torch.float64, device=self.device)
        fracture_apply(self.h, op, level, xt, yt)
        return yt.cpu().numpy()

    def gradient(self):
        torch = self.torch
        Eu = torch.empty(self.ndof, dtype=torch.float64, device=self.device)
        Ea = torch.empty(self.N, dtype=torch.float64, device=self.device)
        fracture_gradient(self.h, Eu, Ea)
        return Eu.cpu().numpy(), Ea.cpu().numpy()

    def fragments(self):
        """(nfrag, fid) of the current alpha (params.deflate = 1)."""
        torch = self.torch
        fid = torch.empty(self.N, dtype=torch.int32, device=self.device)
        n = fracture_fragments(self.h, fid)
        return n, fid.cpu().numpy()

    def deflation_matrix(self):
        return fracture_deflation_matrix(self.h)

    def levels(self):
        return [fracture_level_shape(self.h, l) for l in range(fracture_levels(self.h))]
