"""MI355X node-patch Poisson-Boltzmann solver: Python binding of libafmpb.

Argument marshalling only: every step of the method runs in the HIP library
(``libafmpb.so``, C ABI declared in ``include/afmpb.h``).  The functions below
carry the C names; ``Solver`` is a small convenience wrapper over them.  If the
library has not been built, any call raises ``RuntimeError`` -- there is no
fallback implementation.

Device memory and streams may come from PyTorch: ``afmpb_create`` takes a
``hipStream_t`` (``torch.cuda.current_stream().cuda_stream``) and an optional
device memory supplier (``TorchAllocator`` binds PyTorch's caching allocator),
and ``afmpb_matvec_dev`` takes raw device pointers (``tensor.data_ptr()``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafmpb.so")

AFMPB_OK = 0
AFMPB_E_INVALID = -1
AFMPB_E_MESH = -2
AFMPB_E_OOM = -3
AFMPB_E_NOT_CONVERGED = -4
AFMPB_E_NUMERIC = -5
AFMPB_E_DEVICE = -6
AFMPB_E_STATE = -7
AFMPB_E_PENDING = -8
AFMPB_E_CANCELLED = -9
AFMPB_FP64 = 0
AFMPB_FP32_REFINED = 1
AFMPB_FP32_BF16M2L_REFINED = 2

STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_MESH", -3: "E_OOM",
                -4: "E_NOT_CONVERGED", -5: "E_NUMERIC", -6: "E_DEVICE", -7: "E_STATE",
                -8: "E_PENDING", -9: "E_CANCELLED"}

ABI_FUNCTIONS = (
    "afmpb_default_params", "afmpb_create", "afmpb_destroy", "afmpb_last_error",
    "afmpb_set_molecule", "afmpb_matvec", "afmpb_matvec_dev", "afmpb_solve",
    "afmpb_rhs", "afmpb_energy", "afmpb_energy_dev_noalloc", "afmpb_set_precision",
    "afmpb_tree_info", "afmpb_debug_tree",
    "afmpb_profile_enable", "afmpb_profile_read", "afmpb_profile_only", "afmpb_setup_times",
    "afmpb_server_create", "afmpb_server_set_tuning", "afmpb_server_submit",
    "afmpb_server_poll", "afmpb_server_cancel", "afmpb_server_stats", "afmpb_server_destroy",
)


class afmpb_params(ctypes.Structure):
    _fields_ = [("eps_p", ctypes.c_double), ("eps_s", ctypes.c_double),
                ("kappa", ctypes.c_double), ("order_p", ctypes.c_int),
                ("leaf_cap", ctypes.c_int), ("precision", ctypes.c_int),
                ("rel_tol", ctypes.c_double), ("abs_tol", ctypes.c_double),
                ("restart", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("near_eta", ctypes.c_double), ("m2l_layout", ctypes.c_int),
                ("rhs_fmm", ctypes.c_int), ("overlap", ctypes.c_int),
                ("wx_expand", ctypes.c_int)]


class afmpb_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int),
                ("inner_products", ctypes.c_longlong),
                ("rel_residual_estimate", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("converged", ctypes.c_int),
                ("refinement_steps", ctypes.c_int), ("ms_setup", ctypes.c_double),
                ("ms_rhs", ctypes.c_double), ("ms_gmres", ctypes.c_double),
                ("ms_energy", ctypes.c_double), ("ms_total", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class afmpb_tree_sizes(ctypes.Structure):
    _fields_ = [(k, ctypes.c_longlong) for k in
                ("n_nodes", "n_boxes", "n_levels", "n_u", "n_v", "n_w", "n_x", "n_near",
                 "n_p2p_pairs", "n_m2l_pairs")] + [("order_p", ctypes.c_int),
                                                   ("leaf_cap", ctypes.c_int),
                                                   ("n_m2l_slots", ctypes.c_longlong),
                                                   ("m2l_layout", ctypes.c_int),
                                                   ("rhs_mode", ctypes.c_int),
                                                   ("rhs_boxes", ctypes.c_longlong),
                                                   ("n_wx_far", ctypes.c_longlong),
                                                   ("n_wx_pairs", ctypes.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_TREE_FIELDS = ("keys", "perm", "level", "parent", "child_begin", "n_child", "pt_begin",
                "pt_end", "prefix", "u_ptr", "u_idx", "v_ptr", "v_idx", "v_class", "w_ptr",
                "w_idx", "x_ptr", "x_idx", "near_ptr", "near_col", "near_delta")


class afmpb_tree_view(ctypes.Structure):
    _fields_ = [(k, _P) for k in _TREE_FIELDS]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class afmpb_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class TorchAllocator:
    """Hands the library's device buffers to PyTorch's caching allocator
    (``torch.cuda.caching_allocator_alloc`` / ``caching_allocator_delete``),
    so that PyTorch owns the solver's device memory.  Keeps count of the live
    buffers and bytes.  The object must outlive every context that uses it."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self.calls = 0
        self.peak_bytes = 0
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = afmpb_allocator(self._alloc, self._free, None)

    @property
    def live_bytes(self) -> int:
        return sum(self.live.values())

    def _do_alloc(self, nbytes, stream, user):
        try:
            p = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                         int(stream or 0))
        except Exception:
            return None
        self.live[int(p)] = int(nbytes)
        self.calls += 1
        self.peak_bytes = max(self.peak_bytes, self.live_bytes)
        return p

    def _do_free(self, ptr, user):
        if ptr:
            self.live.pop(int(ptr), None)
            self._torch.cuda.caching_allocator_delete(int(ptr))


class afmpb_molecule(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_longlong), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("n_tri", ctypes.c_longlong), ("tri", ctypes.POINTER(ctypes.c_int)),
                ("n_atoms", ctypes.c_longlong), ("atom_xyz", ctypes.POINTER(ctypes.c_double)),
                ("charge", ctypes.POINTER(ctypes.c_double))]


class afmpb_tuning_entry(ctypes.Structure):
    _fields_ = [("max_nodes", ctypes.c_longlong), ("leaf_cap", ctypes.c_int),
                ("order_p", ctypes.c_int)]


class afmpb_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n_nodes", ctypes.c_longlong),
                ("energy", ctypes.c_double), ("info", afmpb_solve_info),
                ("device_bytes", ctypes.c_longlong), ("ms_admit", ctypes.c_double),
                ("ms_ready", ctypes.c_double), ("ms_done", ctypes.c_double),
                ("message", ctypes.c_char * 128)]


class afmpb_server_counts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_longlong) for k in
                ("queued", "active", "completed", "failed", "device_bytes",
                 "device_bytes_peak")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def _torch_runtime_first():
    """PyTorch ships its own copy of the HIP runtime under the same library
    name.  Loaded first, it is the one this library binds to, so both share
    one runtime (streams, events and device pointers interchangeable).  Loaded
    after the system runtime that this library would otherwise pull in, it
    starts a second runtime in the process, which finds no device.  So import
    (and, with a GPU present, initialise) PyTorch before loading the library
    when it is installed."""
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


def lib():
    """The loaded library; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is None:
        _torch_runtime_first()
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libafmpb.so not found at {LIB_PATH}; build it with "
                "`python -m paper_1710_06316_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        ll = ctypes.c_longlong
        L.afmpb_default_params.argtypes = [ctypes.POINTER(afmpb_params)]
        L.afmpb_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(afmpb_allocator),
                                   ctypes.POINTER(vp)]
        L.afmpb_destroy.argtypes = [vp]
        L.afmpb_last_error.argtypes = [vp]
        L.afmpb_last_error.restype = ctypes.c_char_p
        L.afmpb_set_molecule.argtypes = [vp, ll, dp, ll, ip, ll, dp, dp, dp,
                                         ctypes.POINTER(afmpb_params)]
        L.afmpb_matvec.argtypes = [vp, dp, dp]
        L.afmpb_matvec_dev.argtypes = [vp, vp, vp]
        L.afmpb_solve.argtypes = [vp, dp, dp, dp, dp, ctypes.POINTER(afmpb_solve_info)]
        L.afmpb_rhs.argtypes = [vp, dp]
        L.afmpb_energy.argtypes = [vp, dp, dp]
        L.afmpb_energy_dev_noalloc.argtypes = [vp, vp, vp]
        L.afmpb_set_precision.argtypes = [vp, ctypes.c_int]
        L.afmpb_tree_info.argtypes = [vp, ctypes.POINTER(afmpb_tree_sizes)]
        L.afmpb_debug_tree.argtypes = [vp, ctypes.POINTER(afmpb_tree_view)]
        L.afmpb_profile_enable.argtypes = [vp, ctypes.c_int]
        L.afmpb_profile_only.argtypes = [vp, ctypes.c_char_p]
        L.afmpb_profile_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                         dp, ctypes.POINTER(ll)]
        L.afmpb_setup_times.argtypes = [vp, dp]
        L.afmpb_server_create.argtypes = [ctypes.POINTER(afmpb_params), ll, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.afmpb_server_set_tuning.argtypes = [vp, ctypes.c_int,
                                              ctypes.POINTER(afmpb_tuning_entry)]
        L.afmpb_server_submit.argtypes = [vp, ctypes.POINTER(afmpb_molecule),
                                          ctypes.POINTER(ctypes.c_ulonglong)]
        L.afmpb_server_poll.argtypes = [vp, ctypes.c_ulonglong, ctypes.c_int,
                                        ctypes.POINTER(afmpb_result), dp, dp]
        L.afmpb_server_cancel.argtypes = [vp, ctypes.c_ulonglong]
        L.afmpb_server_stats.argtypes = [vp, ctypes.POINTER(afmpb_server_counts)]
        L.afmpb_server_destroy.argtypes = [vp]
        for name in ABI_FUNCTIONS:
            if name != "afmpb_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class AfmpbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- the C entry points, one marshalling wrapper each -------------------------

def afmpb_default_params() -> afmpb_params:
    p = afmpb_params()
    lib().afmpb_default_params(ctypes.byref(p))
    return p


def afmpb_create(device: int = 0, stream: int | None = None, allocator=None):
    """allocator: None (the library's own hipMalloc) or a TorchAllocator (or
    any object with a ``struct`` of type afmpb_allocator kept alive by the
    caller)."""
    h = ctypes.c_void_p()
    al = ctypes.byref(allocator.struct) if allocator is not None else None
    st = lib().afmpb_create(int(device), ctypes.c_void_p(stream or 0), al, ctypes.byref(h))
    if st != AFMPB_OK:
        raise AfmpbError(st, "afmpb_create failed")
    return h


def afmpb_destroy(ctx) -> int:
    return lib().afmpb_destroy(ctx)


def afmpb_last_error(ctx) -> str:
    return lib().afmpb_last_error(ctx).decode()


def _check(ctx, st, allow=(AFMPB_OK,)):
    if st not in allow:
        raise AfmpbError(st, afmpb_last_error(ctx))
    return st


def afmpb_set_molecule(ctx, xyz, tri, atom_xyz, charge, radius, params: afmpb_params):
    xyz = _f64(xyz).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    ax = _f64(atom_xyz).reshape(-1, 3)
    q = _f64(charge).reshape(-1)
    rad = None if radius is None else _f64(radius).reshape(-1)
    st = lib().afmpb_set_molecule(ctx, len(xyz), _dp(xyz), len(tri), _ip(tri), len(q), _dp(ax),
                                  _dp(q), _dp(rad), ctypes.byref(params))
    return _check(ctx, st)


def afmpb_matvec(ctx, x):
    x = _f64(x)
    y = np.empty_like(x)
    _check(ctx, lib().afmpb_matvec(ctx, _dp(x), _dp(y)))
    return y


def afmpb_matvec_dev(ctx, x_ptr: int, y_ptr: int):
    return _check(ctx, lib().afmpb_matvec_dev(ctx, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)))


def afmpb_solve(ctx, n_nodes: int, x0=None, allow_not_converged=False):
    f = np.empty(n_nodes)
    h = np.empty(n_nodes)
    e = ctypes.c_double()
    info = afmpb_solve_info()
    x0 = None if x0 is None else _f64(x0)
    st = lib().afmpb_solve(ctx, _dp(x0), _dp(f), _dp(h), ctypes.byref(e), ctypes.byref(info))
    allow = (AFMPB_OK, AFMPB_E_NOT_CONVERGED) if allow_not_converged else (AFMPB_OK,)
    _check(ctx, st, allow)
    return f, h, e.value, info, st


def afmpb_rhs(ctx, n_nodes: int):
    b = np.empty(2 * n_nodes)
    _check(ctx, lib().afmpb_rhs(ctx, _dp(b)))
    return b


def afmpb_energy(ctx, x):
    x = _f64(x)
    e = ctypes.c_double()
    _check(ctx, lib().afmpb_energy(ctx, _dp(x), ctypes.byref(e)))
    return e.value


def afmpb_energy_dev_noalloc(ctx, x_ptr: int, energy_ptr: int):
    return _check(ctx, lib().afmpb_energy_dev_noalloc(ctx, ctypes.c_void_p(x_ptr),
                                                      ctypes.c_void_p(energy_ptr)))


def afmpb_set_precision(ctx, precision: int):
    return _check(ctx, lib().afmpb_set_precision(ctx, int(precision)))


def afmpb_tree_info(ctx) -> afmpb_tree_sizes:
    s = afmpb_tree_sizes()
    _check(ctx, lib().afmpb_tree_info(ctx, ctypes.byref(s)))
    return s


def afmpb_debug_tree(ctx) -> dict:
    s = afmpb_tree_info(ctx)
    n, nb = s.n_nodes, s.n_boxes
    arr = {
        "keys": np.zeros(n, np.uint64), "perm": np.zeros(n, np.int32),
        "level": np.zeros(nb, np.int32), "parent": np.zeros(nb, np.int32),
        "child_begin": np.zeros(nb, np.int32), "n_child": np.zeros(nb, np.int32),
        "pt_begin": np.zeros(nb, np.int32), "pt_end": np.zeros(nb, np.int32),
        "prefix": np.zeros(nb, np.uint64),
        "u_ptr": np.zeros(nb + 1, np.int32), "u_idx": np.zeros(max(s.n_u, 1), np.int32),
        "v_ptr": np.zeros(nb + 1, np.int32), "v_idx": np.zeros(max(s.n_v, 1), np.int32),
        "v_class": np.zeros(max(s.n_v, 1), np.int32),
        "w_ptr": np.zeros(nb + 1, np.int32), "w_idx": np.zeros(max(s.n_w, 1), np.int32),
        "x_ptr": np.zeros(nb + 1, np.int32), "x_idx": np.zeros(max(s.n_x, 1), np.int32),
        "near_ptr": np.zeros(n + 1, np.int64), "near_col": np.zeros(max(s.n_near, 1), np.int32),
        "near_delta": np.zeros((max(s.n_near, 1), 4)),
    }
    view = afmpb_tree_view(**{k: arr[k].ctypes.data for k in _TREE_FIELDS})
    _check(ctx, lib().afmpb_debug_tree(ctx, ctypes.byref(view)))
    for k, cnt in (("u_idx", s.n_u), ("v_idx", s.n_v), ("v_class", s.n_v), ("w_idx", s.n_w),
                   ("x_idx", s.n_x), ("near_col", s.n_near), ("near_delta", s.n_near)):
        arr[k] = arr[k][:cnt]
    arr["sizes"] = s.as_dict()
    return arr


SETUP_PHASES = ("geometry", "keys_sort", "tree", "lists", "near", "operators", "buffers_checks",
                "rhs_tree", "near_coeffs_wait")


def afmpb_setup_times(ctx) -> dict:
    ms = np.zeros(len(SETUP_PHASES))
    _check(ctx, lib().afmpb_setup_times(ctx, _dp(ms)))
    return dict(zip(SETUP_PHASES, ms.tolist()))


def afmpb_profile_enable(ctx, enable: bool):
    return _check(ctx, lib().afmpb_profile_enable(ctx, 1 if enable else 0))


def afmpb_profile_only(ctx, scope=None):
    return _check(ctx, lib().afmpb_profile_only(ctx, scope.encode() if scope else None))


def afmpb_profile_read(ctx) -> dict:
    out = {}
    i = 0
    name = ctypes.c_char_p()
    ms = ctypes.c_double()
    cnt = ctypes.c_longlong()
    while lib().afmpb_profile_read(ctx, i, ctypes.byref(name), ctypes.byref(ms),
                                   ctypes.byref(cnt)) == AFMPB_OK:
        out[name.value.decode()] = (ms.value, cnt.value)
        i += 1
    return out


# --- convenience wrapper --------------------------------------------------------

class Solver:
    """One context holding one molecule."""

    def __init__(self, device: int = 0, stream: int | None = None, allocator=None):
        self.allocator = allocator            # kept alive with the context
        self.ctx = afmpb_create(device, stream, allocator)
        self.n = 0

    def close(self):
        if self.ctx is not None:
            afmpb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def params(**kw) -> afmpb_params:
        p = afmpb_default_params()
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    def set_molecule(self, xyz, tri, atom_xyz, charge, radius=None, **params):
        afmpb_set_molecule(self.ctx, xyz, tri, atom_xyz, charge, radius, self.params(**params))
        self.n = int(np.asarray(xyz).reshape(-1, 3).shape[0])

    def load(self, mol, **params):
        kw = dict(eps_p=mol.eps_p, eps_s=mol.eps_s, kappa=mol.kappa)
        kw.update(params)
        self.set_molecule(mol.xyz, mol.tri, mol.atom_xyz, mol.charge, mol.radius, **kw)

    def matvec(self, x):
        return afmpb_matvec(self.ctx, x)

    def matvec_dev(self, x_ptr, y_ptr):
        return afmpb_matvec_dev(self.ctx, x_ptr, y_ptr)

    def solve(self, x0=None, allow_not_converged=False):
        return afmpb_solve(self.ctx, self.n, x0, allow_not_converged)

    def rhs(self):
        return afmpb_rhs(self.ctx, self.n)

    def energy(self, x):
        return afmpb_energy(self.ctx, x)

    def energy_dev_noalloc(self, x_ptr, energy_ptr):
        return afmpb_energy_dev_noalloc(self.ctx, x_ptr, energy_ptr)

    def set_precision(self, precision: int):
        afmpb_set_precision(self.ctx, precision)

    def tree_info(self):
        return afmpb_tree_info(self.ctx).as_dict()

    def debug_tree(self):
        return afmpb_debug_tree(self.ctx)

    def setup_times(self):
        return afmpb_setup_times(self.ctx)

    def profile(self, enable: bool):
        afmpb_profile_enable(self.ctx, enable)

    def profile_read(self):
        return afmpb_profile_read(self.ctx)

    def profile_only(self, scope=None):
        afmpb_profile_only(self.ctx, scope)


# --- solve server ---------------------------------------------------------------

def afmpb_server_create(params: afmpb_params, hbm_budget_bytes: int, max_active: int,
                        setup_threads: int = 1, device: int = 0, stream: int | None = None):
    h = ctypes.c_void_p()
    st = lib().afmpb_server_create(ctypes.byref(params), int(hbm_budget_bytes), int(max_active),
                                   int(setup_threads), int(device), ctypes.c_void_p(stream or 0),
                                   ctypes.byref(h))
    if st != AFMPB_OK:
        raise AfmpbError(st, "afmpb_server_create failed")
    return h


def afmpb_server_set_tuning(srv, table):
    """table: sequence of (max_nodes, leaf_cap, order_p), ascending max_nodes."""
    arr = (afmpb_tuning_entry * max(len(table), 1))()
    for i, (mx, leaf, p) in enumerate(table):
        arr[i] = afmpb_tuning_entry(int(mx), int(leaf), int(p))
    st = lib().afmpb_server_set_tuning(srv, len(table), arr)
    if st != AFMPB_OK:
        raise AfmpbError(st, "bad tuning table")


def afmpb_server_submit(srv, xyz, tri, atom_xyz, charge) -> int:
    xyz = _f64(xyz).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    ax = _f64(atom_xyz).reshape(-1, 3)
    q = _f64(charge).reshape(-1)
    m = afmpb_molecule(len(xyz), _dp(xyz), len(tri), _ip(tri), len(q), _dp(ax), _dp(q))
    t = ctypes.c_ulonglong()
    st = lib().afmpb_server_submit(srv, ctypes.byref(m), ctypes.byref(t))
    if st != AFMPB_OK:
        raise AfmpbError(st, "afmpb_server_submit failed")
    return t.value


def afmpb_server_poll(srv, ticket: int, n_nodes: int, wait: bool = False):
    """(status, result, f, h); status AFMPB_E_PENDING while the request runs."""
    res = afmpb_result()
    f = np.empty(n_nodes)
    h = np.empty(n_nodes)
    st = lib().afmpb_server_poll(srv, ctypes.c_ulonglong(ticket), 1 if wait else 0,
                                 ctypes.byref(res), _dp(f), _dp(h))
    if st not in (AFMPB_OK, AFMPB_E_PENDING):
        raise AfmpbError(st, "afmpb_server_poll failed")
    return st, res, f, h


def afmpb_server_cancel(srv, ticket: int):
    st = lib().afmpb_server_cancel(srv, ctypes.c_ulonglong(ticket))
    if st != AFMPB_OK:
        raise AfmpbError(st, "afmpb_server_cancel failed")


def afmpb_server_stats(srv) -> dict:
    c = afmpb_server_counts()
    st = lib().afmpb_server_stats(srv, ctypes.byref(c))
    if st != AFMPB_OK:
        raise AfmpbError(st, "afmpb_server_stats failed")
    return c.as_dict()


def afmpb_server_destroy(srv):
    return lib().afmpb_server_destroy(srv)


class Server:
    """Continuous-batching solve server (one device)."""

    def __init__(self, hbm_budget_bytes: int = 32 << 30, max_active: int = 64,
                 setup_threads: int = 1, device: int = 0, tuning=None, stream=None, **params):
        p = afmpb_default_params()
        for k, v in params.items():
            setattr(p, k, v)
        self.srv = afmpb_server_create(p, hbm_budget_bytes, max_active, setup_threads, device,
                                       stream)
        self.n_of = {}
        if tuning:
            afmpb_server_set_tuning(self.srv, tuning)

    def submit(self, mol) -> int:
        t = afmpb_server_submit(self.srv, mol.xyz, mol.tri, mol.atom_xyz, mol.charge)
        self.n_of[t] = int(np.asarray(mol.xyz).reshape(-1, 3).shape[0])
        return t

    def poll(self, ticket: int, wait: bool = False):
        st, res, f, h = afmpb_server_poll(self.srv, ticket, self.n_of[ticket], wait)
        if st == AFMPB_OK:
            del self.n_of[ticket]
        return st, res, f, h

    def wait(self, ticket: int):
        return self.poll(ticket, wait=True)[1:]

    def cancel(self, ticket: int):
        afmpb_server_cancel(self.srv, ticket)

    def stats(self) -> dict:
        return afmpb_server_stats(self.srv)

    def close(self):
        if self.srv is not None:
            afmpb_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
