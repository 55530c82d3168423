"""ctypes binding of libopf (include/opf.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions keep the C names; :class:`Model` adds ownership of the handle and
accepts torch tensors (device arrays) for the evaluation calls.  Importing
this module loads ``libopf.so`` from the package directory and raises if it
is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libopf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "opf.h")

# libopf must share one HIP runtime instance with torch (stream handles and
# device pointers are per runtime).  torch ships its own libamdhip64 with
# the same soname, so load torch first: the dynamic loader then resolves
# libopf's dependency to the runtime torch already mapped.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2405_14032_amd/build_lib.py "
                      "(or __graft_entry__.build())")
lib = C.CDLL(LIB_PATH)

OPF_OK, OPF_EINVAL, OPF_ERANGE, OPF_ENOMEM, OPF_EHIP, OPF_ENODEV = 0, -1, -2, -3, -4, -5
OPF_IPM_CONVERGED, OPF_IPM_MAX_ITER, OPF_IPM_STALLED = 0, 1, 2
IPM_STATUS = {OPF_IPM_CONVERGED: "converged", OPF_IPM_MAX_ITER: "max_iter", OPF_IPM_STALLED: "stalled"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class opf_instance_desc(C.Structure):
    _fields_ = [
        ("nbus", C.c_int32), ("nbranch", C.c_int32), ("ngen", C.c_int32),
        ("nperiod", C.c_int32), ("ref_bus", C.c_int32),
        ("vmin", _dp), ("vmax", _dp),
        ("f_bus", _ip), ("t_bus", _ip),
        ("r", _dp), ("x", _dp), ("b_charge", _dp),
        ("rate", _dp), ("angmin", _dp), ("angmax", _dp),
        ("tap", _dp), ("shift", _dp),
        ("gen_bus", _ip),
        ("c2", _dp), ("c1", _dp), ("c0", _dp),
        ("pmin", _dp), ("pmax", _dp), ("qmin", _dp), ("qmax", _dp), ("ramp", _dp),
        ("pd", _dp), ("qd", _dp),
    ]


class opf_dims(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("nnz_jac", C.c_int64),
                ("nnz_hess", C.c_int64), ("nnz_kkt", C.c_int64), ("ninst", C.c_int32)]


class opf_sweep_args(C.Structure):
    _fields_ = [("x", C.c_void_p), ("lambda_", C.c_void_p), ("sigma", C.c_double),
                ("v", C.c_void_p), ("diag_x", C.c_void_p), ("dcon", C.c_void_p),
                ("f", C.c_void_p), ("grad", C.c_void_p), ("c", C.c_void_p),
                ("jvals", C.c_void_p), ("hvals", C.c_void_p), ("jtv", C.c_void_p),
                ("kvals", C.c_void_p)]


class opf_chol_info(C.Structure):
    _fields_ = [("factor_entries", C.c_int64), ("arena_entries", C.c_int64), ("flops", C.c_double),
                ("flops_interior", C.c_double), ("nodes", C.c_int32), ("levels", C.c_int32),
                ("chunk", C.c_int32), ("large_nodes", C.c_int32)]


class opf_ipm_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("relax", C.c_double), ("sigma", C.c_double),
                ("tau", C.c_double), ("delta_c", C.c_double), ("dw_first", C.c_double), ("dw_grow", C.c_double),
                ("dw_max", C.c_double), ("pivot_tol", C.c_double), ("verbose", C.c_int32),
                ("line_search", C.c_int32), ("mu_init", C.c_double), ("kappa_eps", C.c_double),
                ("kappa_mu", C.c_double), ("theta_mu", C.c_double), ("tau_min", C.c_double),
                ("gamma_theta", C.c_double), ("gamma_phi", C.c_double), ("eta_phi", C.c_double),
                ("s_theta", C.c_double), ("s_phi", C.c_double), ("delta", C.c_double), ("gamma_alpha", C.c_double),
                ("kappa_sigma", C.c_double), ("stall_iter", C.c_int32), ("dw_grow_first", C.c_double),
                ("dw_shrink", C.c_double), ("dw_min", C.c_double)]


class opf_ipm_result(C.Structure):
    _fields_ = [("converged", C.c_int32), ("iterations", C.c_int32), ("factorizations", C.c_int32),
                ("objective", C.c_double), ("err", C.c_double), ("seconds", C.c_double), ("t_eval", C.c_double),
                ("t_factor", C.c_double), ("t_solve", C.c_double), ("status", C.c_int32), ("trials", C.c_int32),
                ("theta", C.c_double)]


class opf_ipm_state(C.Structure):
    _fields_ = [("x", C.c_void_p), ("s", C.c_void_p), ("y", C.c_void_p),
                ("zl", C.c_void_p), ("zu", C.c_void_p), ("vl", C.c_void_p), ("vu", C.c_void_p),
                ("xl", C.c_void_p), ("xu", C.c_void_p), ("sl", C.c_void_p), ("su", C.c_void_p),
                ("mu", C.c_double), ("delta_w", C.c_double), ("delta_c", C.c_double)]


_vp = C.c_void_p
_SIGS = {
    "opf_validate": (C.c_int, [C.POINTER(opf_instance_desc), C.c_int32]),
    "opf_model_create": (C.c_int, [C.POINTER(opf_instance_desc), C.c_int32, C.c_int, C.POINTER(_vp)]),
    "opf_model_destroy": (None, [_vp]),
    "opf_model_dims": (C.c_int, [_vp, C.POINTER(opf_dims)]),
    "opf_instance_offsets": (C.c_int, [_vp, _lp, _lp, _lp, _lp, _lp]),
    "opf_set_stream": (C.c_int, [_vp, _vp]),
    "opf_bounds": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "opf_jac_structure": (C.c_int, [_vp, _vp, _vp]),
    "opf_hess_structure": (C.c_int, [_vp, _vp, _vp]),
    "opf_kkt_structure": (C.c_int, [_vp, _vp, _vp]),
    "opf_eval_obj": (C.c_int, [_vp, _vp, _vp]),
    "opf_eval_grad": (C.c_int, [_vp, _vp, _vp]),
    "opf_eval_cons": (C.c_int, [_vp, _vp, _vp]),
    "opf_eval_jac": (C.c_int, [_vp, _vp, _vp]),
    "opf_eval_hess": (C.c_int, [_vp, _vp, _vp, C.c_double, _vp]),
    "opf_jtprod": (C.c_int, [_vp, _vp, _vp, _vp]),
    "opf_set_load": (C.c_int, [_vp, _vp, _vp]),
    "opf_load_adjoint": (C.c_int, [_vp, _vp, _vp, _vp]),
    "opf_assemble_condensed": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "opf_eval_jhk": (C.c_int, [_vp, _vp, _vp, C.c_double, _vp, _vp, _vp, _vp, _vp]),
    "opf_sweep": (C.c_int, [_vp, C.POINTER(opf_sweep_args)]),
    "opf_sweep_graph": (C.c_int, [_vp, C.POINTER(opf_sweep_args)]),
    "opf_sweep_noalloc": (C.c_int, [_vp, C.POINTER(opf_sweep_args)]),
    "opf_sweep_check": (C.c_int, [_vp, C.POINTER(C.c_int32)]),
    "opf_jprod": (C.c_int, [_vp, _vp, _vp, _vp]),
    "opf_condensed_rhs": (C.c_int, [_vp, C.POINTER(opf_ipm_state), _vp, _vp, _vp, _vp, _vp]),
    "opf_recover_step": (C.c_int, [_vp, C.POINTER(opf_ipm_state), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "opf_autotune": (C.c_int, [_vp, C.c_char_p]),
    "opf_chol_analyze": (C.c_int, [_vp, C.POINTER(_vp)]),
    "opf_chol_destroy": (None, [_vp]),
    "opf_chol_get_info": (C.c_int, [_vp, C.POINTER(opf_chol_info)]),
    "opf_chol_tree_size": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "opf_chol_tree": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "opf_chol_factor": (C.c_int, [_vp, _vp, C.c_double, C.c_double, _vp]),
    "opf_chol_solve": (C.c_int, [_vp, _vp, _vp]),
    "opf_chol_set_graph": (C.c_int, [_vp, C.c_int]),
    "opf_chol_set_stop_on_pivot": (C.c_int, [_vp, C.c_int]),
    "opf_chol_stop_on_pivot": (C.c_int, [_vp]),
    "opf_ipm_default_options": (None, [C.POINTER(opf_ipm_options)]),
    "opf_ipm_solve": (C.c_int, [_vp, _vp, C.POINTER(opf_ipm_options), _vp, _vp, C.POINTER(opf_ipm_result)]),
    "opf_set_timing": (C.c_int, [_vp, C.c_int]),
    "opf_kernel_stats": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_char_p), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]),
    "opf_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


def header_symbols(path: str = HEADER) -> list[str]:
    """Function names declared in include/opf.h."""
    text = open(path).read()
    return sorted(set(re.findall(r"\b(opf_[a-z_]+)\s*\(", text)))


class OpfError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.opf_last_error().decode(errors="replace")
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def check(code: int, where: str) -> None:
    if code != OPF_OK:
        raise OpfError(code, where)


# ---------------------------------------------------------------- descriptors
_DOUBLE_FIELDS = ["vmin", "vmax", "r", "x", "b_charge", "rate", "angmin", "angmax", "tap", "shift",
                  "c2", "c1", "c0", "pmin", "pmax", "qmin", "qmax", "ramp", "pd", "qd"]
_INT_FIELDS = ["f_bus", "t_bus", "gen_bus"]


def make_desc(net, keep: list) -> opf_instance_desc:
    """Fill a descriptor from an object with the Network attributes (host
    numpy arrays); ``keep`` receives the contiguous copies that must outlive
    the call."""
    d = opf_instance_desc()
    d.nbus, d.nbranch, d.ngen, d.nperiod = int(net.N), int(net.B), int(net.G), int(net.T)
    d.ref_bus = int(net.ref_bus)
    for name in _DOUBLE_FIELDS:
        val = getattr(net, name, None)
        if val is None:
            setattr(d, name, None)
            continue
        arr = np.ascontiguousarray(np.asarray(val, dtype=np.float64).reshape(-1))
        keep.append(arr)
        setattr(d, name, arr.ctypes.data_as(_dp))
    for name in _INT_FIELDS:
        arr = np.ascontiguousarray(np.asarray(getattr(net, name), dtype=np.int32).reshape(-1))
        keep.append(arr)
        setattr(d, name, arr.ctypes.data_as(_ip))
    return d


def make_descs(nets) -> tuple:
    keep: list = []
    arr = (opf_instance_desc * len(nets))()
    for k, net in enumerate(nets):
        arr[k] = make_desc(net, keep)
    return arr, keep


def validate(nets) -> int:
    descs, keep = make_descs(nets)
    return opf_validate(descs, len(nets))


def _ptr(t) -> int | None:
    """Device address of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _dev_arg(t, device: int, count: int, dtype: str, what: str, optional: bool = False) -> int | None:
    """Device address of a torch tensor after checking that the library can
    use it: a contiguous tensor of the given dtype ("f64", "i32" or "i64") on
    the model's HIP device with at least ``count`` elements.  None passes NULL
    where the call allows it.  Raises before anything reaches the C ABI, so
    a wrong argument never becomes an out-of-bounds device access."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{what}: a tensor is required")
    import torch
    want = {"f64": torch.float64, "i32": torch.int32, "i64": torch.int64}[dtype]
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != want:
        raise TypeError(f"{what}: dtype {t.dtype}, expected {want}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if t.numel() < count:
        raise ValueError(f"{what}: {t.numel()} elements, need {count}")
    if device < 0:
        raise ValueError(f"{what}: the model is host-only (created with device < 0)")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{what}: tensor on {t.device}, the model is on cuda:{device}")
    return t.data_ptr()


class Model:
    """Owns an opf_model handle.  device >= 0 puts it on that HIP device;
    device < 0 makes a host-only model (dims, offsets, host KKT pattern)."""

    def __init__(self, nets, device: int = 0):
        if not isinstance(nets, (list, tuple)):
            nets = [nets]
        self.nets = list(nets)
        descs, keep = make_descs(self.nets)
        h = _vp()
        check(opf_model_create(descs, len(self.nets), int(device), C.byref(h)), "opf_model_create")
        self.h = h
        self.device = device
        d = opf_dims()
        check(opf_model_dims(self.h, C.byref(d)), "opf_model_dims")
        self.n, self.m = d.n, d.m
        self.nnz_jac, self.nnz_hess, self.nnz_kkt = d.nnz_jac, d.nnz_hess, d.nnz_kkt
        self.ninst = d.ninst
        k = self.ninst + 1
        offs = [np.zeros(k, dtype=np.int64) for _ in range(5)]
        check(opf_instance_offsets(self.h, *[o.ctypes.data_as(_lp) for o in offs]), "opf_instance_offsets")
        self.x_off, self.c_off, self.j_off, self.h_off, self.k_off = offs
        self.nload = int(sum(int(net.T) * int(net.N) for net in self.nets))
        self._stream = None

    def _a(self, t, count, what, dtype="f64", optional=False):
        return _dev_arg(t, self.device, count, dtype, what, optional)

    def close(self):
        if getattr(self, "h", None):
            opf_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # stream -----------------------------------------------------------------
    def set_stream(self, stream_handle: int | None):
        check(opf_set_stream(self.h, stream_handle), "opf_set_stream")
        self._stream = stream_handle

    def use_current_torch_stream(self):
        import torch
        self.set_stream(torch.cuda.current_stream().cuda_stream)

    # structure --------------------------------------------------------------
    def bounds(self, lv, uv, lc, uc):
        n, m = self.n, self.m
        check(opf_bounds(self.h, self._a(lv, n, "lvar"), self._a(uv, n, "uvar"), self._a(lc, m, "lcon"),
                         self._a(uc, m, "ucon")), "opf_bounds")

    def jac_structure(self, rows, cols):
        k = self.nnz_jac
        check(opf_jac_structure(self.h, self._a(rows, k, "rows", "i32"), self._a(cols, k, "cols", "i32")),
              "opf_jac_structure")

    def hess_structure(self, rows, cols):
        k = self.nnz_hess
        check(opf_hess_structure(self.h, self._a(rows, k, "rows", "i32"), self._a(cols, k, "cols", "i32")),
              "opf_hess_structure")

    def kkt_structure(self, rowptr, colind):
        check(opf_kkt_structure(self.h, self._a(rowptr, self.n + 1, "rowptr", "i64"),
                                self._a(colind, self.nnz_kkt, "colind", "i32")), "opf_kkt_structure")

    def kkt_structure_host(self):
        """Host-only models: the K pattern as numpy arrays."""
        rp = np.zeros(self.n + 1, dtype=np.int64)
        ci = np.zeros(self.nnz_kkt, dtype=np.int32)
        check(opf_kkt_structure(self.h, rp.ctypes.data, ci.ctypes.data), "opf_kkt_structure")
        return rp, ci

    # evaluation -------------------------------------------------------------
    def eval_obj(self, x, f):
        check(opf_eval_obj(self.h, self._a(x, self.n, "x"), self._a(f, self.ninst, "f")), "opf_eval_obj")

    def eval_grad(self, x, g):
        check(opf_eval_grad(self.h, self._a(x, self.n, "x"), self._a(g, self.n, "grad")), "opf_eval_grad")

    def eval_cons(self, x, c):
        check(opf_eval_cons(self.h, self._a(x, self.n, "x"), self._a(c, self.m, "c")), "opf_eval_cons")

    def eval_jac(self, x, jv):
        check(opf_eval_jac(self.h, self._a(x, self.n, "x"), self._a(jv, self.nnz_jac, "jvals")), "opf_eval_jac")

    def eval_hess(self, x, lam, sigma, hv):
        check(opf_eval_hess(self.h, self._a(x, self.n, "x"), self._a(lam, self.m, "lambda"), float(sigma),
                            self._a(hv, self.nnz_hess, "hvals")), "opf_eval_hess")

    def jtprod(self, x, v, out):
        check(opf_jtprod(self.h, self._a(x, self.n, "x"), self._a(v, self.m, "v"), self._a(out, self.n, "jtv")),
              "opf_jtprod")

    def set_load(self, pd, qd):
        check(opf_set_load(self.h, self._a(pd, self.nload, "pd"), self._a(qd, self.nload, "qd")), "opf_set_load")

    def load_adjoint(self, lam, gpd, gqd):
        check(opf_load_adjoint(self.h, self._a(lam, self.m, "lambda"), self._a(gpd, self.nload, "gpd"),
                               self._a(gqd, self.nload, "gqd")), "opf_load_adjoint")

    def assemble_condensed(self, hv, jv, diag_x, dcon, kv):
        check(opf_assemble_condensed(self.h, self._a(hv, self.nnz_hess, "hvals"), self._a(jv, self.nnz_jac, "jvals"),
                                     self._a(diag_x, self.n, "diag_x", optional=True), self._a(dcon, self.m, "dcon"),
                                     self._a(kv, self.nnz_kkt, "kvals")), "opf_assemble_condensed")

    def eval_jhk(self, x, lam, sigma, diag_x, dcon, jv, hv, kv):
        check(opf_eval_jhk(self.h, self._a(x, self.n, "x"), self._a(lam, self.m, "lambda"), float(sigma),
                           self._a(diag_x, self.n, "diag_x", optional=True), self._a(dcon, self.m, "dcon"),
                           self._a(jv, self.nnz_jac, "jvals"), self._a(hv, self.nnz_hess, "hvals"),
                           self._a(kv, self.nnz_kkt, "kvals")), "opf_eval_jhk")

    def jprod(self, x, v, out):
        check(opf_jprod(self.h, self._a(x, self.n, "x"), self._a(v, self.n, "v"), self._a(out, self.m, "jv")),
              "opf_jprod")

    def ipm_state(self, x, s, y, zl, zu, vl, vu, xl, xu, sl, su, mu, delta_w, delta_c) -> opf_ipm_state:
        """The C state struct over device tensors (the tensors must outlive
        the calls that use it)."""
        n, m = self.n, self.m
        st = opf_ipm_state()
        st.x, st.s, st.y = self._a(x, n, "x"), self._a(s, m, "s"), self._a(y, m, "y")
        st.zl, st.zu = self._a(zl, n, "zl"), self._a(zu, n, "zu")
        st.vl, st.vu = self._a(vl, m, "vl"), self._a(vu, m, "vu")
        st.xl, st.xu = self._a(xl, n, "xl"), self._a(xu, n, "xu")
        st.sl, st.su = self._a(sl, m, "sl"), self._a(su, m, "su")
        st.mu, st.delta_w, st.delta_c = float(mu), float(delta_w), float(delta_c)
        return st

    def condensed_rhs(self, st, grad, c, diag_x, dcon, rhs):
        n, m = self.n, self.m
        check(opf_condensed_rhs(self.h, C.byref(st), self._a(grad, n, "grad"), self._a(c, m, "c"),
                                self._a(diag_x, n, "diag_x"), self._a(dcon, m, "dcon"), self._a(rhs, n, "rhs")),
              "opf_condensed_rhs")

    def recover_step(self, st, c, dx, ds, dy, dzl, dzu, dvl, dvu):
        n, m = self.n, self.m
        check(opf_recover_step(self.h, C.byref(st), self._a(c, m, "c"), self._a(dx, n, "dx"), self._a(ds, m, "ds"),
                               self._a(dy, m, "dy"), self._a(dzl, n, "dzl"), self._a(dzu, n, "dzu"),
                               self._a(dvl, m, "dvl"), self._a(dvu, m, "dvu")), "opf_recover_step")

    def sweep_args(self, x=None, lam=None, sigma=1.0, v=None, diag_x=None, dcon=None, f=None, grad=None, c=None,
                   jvals=None, hvals=None, jtv=None, kvals=None) -> opf_sweep_args:
        """The sweep's argument struct; every tensor given is checked, an
        argument left None passes NULL (the C side decides which may be)."""
        n, m = self.n, self.m
        a = opf_sweep_args()
        o = dict(optional=True)
        a.x, a.lambda_, a.sigma = self._a(x, n, "x", **o), self._a(lam, m, "lambda", **o), float(sigma)
        a.v, a.diag_x, a.dcon = self._a(v, m, "v", **o), self._a(diag_x, n, "diag_x", **o), self._a(dcon, m, "dcon", **o)
        a.f, a.grad, a.c = self._a(f, self.ninst, "f", **o), self._a(grad, n, "grad", **o), self._a(c, m, "c", **o)
        a.jvals, a.hvals = self._a(jvals, self.nnz_jac, "jvals", **o), self._a(hvals, self.nnz_hess, "hvals", **o)
        a.jtv, a.kvals = self._a(jtv, n, "jtv", **o), self._a(kvals, self.nnz_kkt, "kvals", **o)
        return a

    def sweep(self, args: opf_sweep_args):
        check(opf_sweep(self.h, C.byref(args)), "opf_sweep")

    def sweep_graph(self, args: opf_sweep_args):
        check(opf_sweep_graph(self.h, C.byref(args)), "opf_sweep_graph")

    def sweep_noalloc(self, args: opf_sweep_args):
        check(opf_sweep_noalloc(self.h, C.byref(args)), "opf_sweep_noalloc")

    def sweep_check(self) -> int:
        """Status bits of the one-launch sweeps since the last call (0: all
        completed as designed); waits for the model's stream."""
        st = C.c_int32(0)
        check(opf_sweep_check(self.h, C.byref(st)), "opf_sweep_check")
        return st.value

    def set_timing(self, enable: bool):
        check(opf_set_timing(self.h, 1 if enable else 0), "opf_set_timing")

    def kernel_stats(self) -> dict:
        """{kernel family: (timed launches, summed ms)} for families with launches."""
        out = {}
        i = 0
        while True:
            name, cnt, ms = C.c_char_p(), C.c_int64(), C.c_double()
            rc = opf_kernel_stats(self.h, i, C.byref(name), C.byref(cnt), C.byref(ms))
            if rc == OPF_ERANGE:
                break
            check(rc, "opf_kernel_stats")
            if cnt.value:
                out[name.value.decode()] = (cnt.value, ms.value)
            i += 1
        return out

    def autotune(self, cache_path: str | None = None):
        check(opf_autotune(self.h, cache_path.encode() if cache_path else None), "opf_autotune")


class Chol:
    """Owns an opf_chol handle: the static-pivot sparse Cholesky of the
    model's condensed matrix (analysis at construction; factor / solve on
    device arrays)."""

    def __init__(self, model: Model):
        h = _vp()
        check(opf_chol_analyze(model.h, C.byref(h)), "opf_chol_analyze")
        self.h = h
        self.model = model

    def close(self):
        if getattr(self, "h", None):
            opf_chol_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = opf_chol_info()
        check(opf_chol_get_info(self.h, C.byref(i)), "opf_chol_get_info")
        return {k: getattr(i, k) for k, _ in opf_chol_info._fields_}

    def tree(self, inst: int = 0) -> dict:
        """The analysis of one instance as numpy arrays (host)."""
        nn, nr = C.c_int32(), C.c_int64()
        check(opf_chol_tree_size(self.h, inst, C.byref(nn), C.byref(nr)), "opf_chol_tree_size")
        net = self.model.nets[inst]
        n_p = 2 * net.N + 2 * net.G + 4 * net.B
        perm = np.zeros(n_p, dtype=np.int32)
        first = np.zeros(nn.value, dtype=np.int32)
        npiv = np.zeros(nn.value, dtype=np.int32)
        parent = np.zeros(nn.value, dtype=np.int32)
        rowptr = np.zeros(nn.value + 1, dtype=np.int64)
        rows = np.zeros(max(1, nr.value), dtype=np.int32)
        check(opf_chol_tree(self.h, inst, perm.ctypes.data, first.ctypes.data, npiv.ctypes.data,
                            parent.ctypes.data, rowptr.ctypes.data, rows.ctypes.data), "opf_chol_tree")
        return dict(perm=perm, first=first, npiv=npiv, parent=parent, rowptr=rowptr, rows=rows[:nr.value])

    def factor(self, kvals, pivot_tol: float, pivot_repl: float, npert):
        M = self.model
        check(opf_chol_factor(self.h, M._a(kvals, M.nnz_kkt, "kvals"), float(pivot_tol), float(pivot_repl),
                              M._a(npert, 1, "npert", "i32", optional=True)), "opf_chol_factor")

    def solve(self, b, x):
        M = self.model
        check(opf_chol_solve(self.h, M._a(b, M.n, "b"), M._a(x, M.n, "x")), "opf_chol_solve")

    def set_stop_on_pivot(self, enable: bool):
        check(opf_chol_set_stop_on_pivot(self.h, 1 if enable else 0), "opf_chol_set_stop_on_pivot")

    def set_graph(self, enable: bool):
        check(opf_chol_set_graph(self.h, int(enable)), "opf_chol_set_graph")


def ipm_options(**kw) -> opf_ipm_options:
    """Default interior-point options with the given fields replaced."""
    o = opf_ipm_options()
    opf_ipm_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def ipm_solve(model: Model, chol: Chol, x_out, y_out=None, **opts) -> dict:
    """Runs the lifted-KKT interior-point loop (opf_ipm_solve); x_out (and
    y_out) are device arrays receiving the final point (multipliers)."""
    if chol.model is not model:
        raise ValueError("chol was analysed from another model")
    o = ipm_options(**opts)
    r = opf_ipm_result()
    check(opf_ipm_solve(model.h, chol.h, C.byref(o), model._a(x_out, model.n, "x_out"),
                        model._a(y_out, model.m, "y_out", optional=True), C.byref(r)), "opf_ipm_solve")
    out = {k: getattr(r, k) for k, _ in opf_ipm_result._fields_}
    out["status_name"] = IPM_STATUS.get(out["status"], str(out["status"]))
    return out
