"""ctypes binding of liblsh.so (declared in include/lsh.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Device memory comes from torch (``torch.empty(..., device='cuda')``)
and work is queued on torch's current stream.  Importing this module fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsh.so")

DIRICHLET, DIRICHLET_MODIFIED, DLVP, BOXSPLINE = 0, 1, 2, 3
FP64, FP32_MIXED = 0, 1
KINDS = {"dirichlet": DIRICHLET, "dirichlet_modified": DIRICHLET_MODIFIED, "dlvp": DLVP, "box": BOXSPLINE}
PRECISIONS = {"fp64": FP64, "fp32": FP32_MIXED}

STATUS = {0: "LSH_OK", -1: "LSH_EINVAL", -2: "LSH_ESINGULAR", -3: "LSH_ENOINTERP", -4: "LSH_ENOTELLIPTIC",
          -5: "LSH_ENOTCONVERGED", -6: "LSH_ENONFINITE", -7: "LSH_EDEVICE", -8: "LSH_EWORKSPACE",
          -9: "LSH_EUNSUPPORTED", -10: "LSH_ESTATE"}

EXPORTS = ["lsh_create_pattern", "lsh_destroy", "lsh_pattern_info", "lsh_pattern_snf", "lsh_pattern_points",
           "lsh_set_kernel", "lsh_set_stiffness", "lsh_persistent_bytes", "lsh_bind", "lsh_gamma_probe",
           "lsh_solve_bytes", "lsh_solve", "lsh_solve_noalloc", "lsh_batch_bytes", "lsh_solve_batch", "lsh_profile_enable",
           "lsh_profile_select", "lsh_profile_read", "lsh_last_error", "lsh_autotune", "lsh_tune_reset", "lsh_tune_set", "lsh_set_scheme", "lsh_unet_create", "lsh_unet_destroy", "lsh_unet_param_count",
           "lsh_unet_param_bytes", "lsh_unet_bind", "lsh_unet_get_params", "lsh_unet_act_bytes",
           "lsh_unet_train_step", "lsh_unet_zero_grad", "lsh_unet_get_grads", "lsh_unet_predict", "lsh_unet_head",
           "lsh_unet_layers", "lsh_unet_pack_target"]

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")

# torch first: its HIP runtime (SONAME libamdhip64.so.7) then satisfies the
# library's dependency, so the process holds a single HIP runtime.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_DP = ctypes.POINTER(ctypes.c_double)


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class Task(ctypes.Structure):
    _fields_ = [("p", _P), ("nload", ctypes.c_int), ("eps0_voigt", _DP), ("sigma_out", _DP),
                ("stats", ctypes.POINTER(Stats)), ("dev_E_init", _P), ("dev_E_out", _P)]


_sig = {
    "lsh_create_pattern": ([ctypes.c_int, _I64P, ctypes.POINTER(_P)], ctypes.c_int),
    "lsh_destroy": ([_P], None),
    "lsh_pattern_info": ([_P, _I64P, _I64P], ctypes.c_int),
    "lsh_pattern_snf": ([_P, _I64P, _I64P], ctypes.c_int),
    "lsh_pattern_points": ([_P, _I64P], ctypes.c_int),
    "lsh_set_kernel": ([_P, ctypes.c_int, _DP, ctypes.c_int], ctypes.c_int),
    "lsh_set_stiffness": ([_P, ctypes.c_int, _DP, _DP, ctypes.POINTER(ctypes.c_uint8)], ctypes.c_int),
    "lsh_persistent_bytes": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lsh_bind": ([_P, ctypes.c_int, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "lsh_gamma_probe": ([_P, ctypes.c_int, _I64P, ctypes.c_int, _DP, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "lsh_solve_bytes": ([_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lsh_solve": ([_P, ctypes.c_int, _DP, ctypes.c_double, ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t, _P,
                   _P, _P, _DP, ctypes.POINTER(Stats), _DP], ctypes.c_int),
    "lsh_solve_noalloc": ([_P, ctypes.c_int, _DP, ctypes.c_double, ctypes.c_int, ctypes.c_int, _P, _P, _P, _DP,
                           ctypes.POINTER(Stats), _DP], ctypes.c_int),
    "lsh_batch_bytes": ([ctypes.POINTER(Task), ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                        ctypes.c_int),
    "lsh_solve_batch": ([ctypes.POINTER(Task), ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, _P,
                         ctypes.c_size_t, _P], ctypes.c_int),
    "lsh_profile_enable": ([ctypes.c_int], ctypes.c_int),
    "lsh_profile_select": ([ctypes.c_uint], ctypes.c_int),
    "lsh_profile_read": ([_DP, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int], ctypes.c_int),
    "lsh_last_error": ([], ctypes.c_char_p),
    "lsh_autotune": ([_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t, _P, _P], ctypes.c_int),
    "lsh_tune_reset": ([_P], ctypes.c_int),
    "lsh_set_scheme": ([_P, ctypes.c_int], ctypes.c_int),
    "lsh_tune_set": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "lsh_unet_create": ([ctypes.c_int, ctypes.POINTER(_P)], ctypes.c_int),
    "lsh_unet_destroy": ([_P], None),
    "lsh_unet_param_count": ([_P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "lsh_unet_param_bytes": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lsh_unet_bind": ([_P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_float), _P], ctypes.c_int),
    "lsh_unet_get_params": ([_P, ctypes.POINTER(ctypes.c_float), _P], ctypes.c_int),
    "lsh_unet_act_bytes": ([_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lsh_unet_train_step": ([_P, _P, _P, ctypes.c_int, ctypes.c_float, _P, ctypes.c_size_t, _P, _DP], ctypes.c_int),
    "lsh_unet_zero_grad": ([_P, _P], ctypes.c_int),
    "lsh_unet_get_grads": ([_P, ctypes.POINTER(ctypes.c_float), _P], ctypes.c_int),
    "lsh_unet_predict": ([_P, _P, ctypes.c_int, _DP, ctypes.c_int, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "lsh_unet_head": ([_P, ctypes.c_int, _P, _P], ctypes.c_int),
    "lsh_unet_layers": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "lsh_unet_pack_target": ([_P, ctypes.c_int, _P, _P], ctypes.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class LshError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(rc, allow=()):
    if rc != 0 and rc not in allow:
        raise LshError(rc, _lib.lsh_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(_DP)


def exported_symbols():
    """Names of the C-ABI entry points this binding resolves."""
    return [n for n in EXPORTS if hasattr(_lib, n)]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_SOLVE_STREAM = None


def _solve_stream():
    """A non-default stream for solves (the library captures its iterations in a
    HIP graph there); ordered after torch's current stream."""
    global _SOLVE_STREAM
    torch = _torch()
    if _SOLVE_STREAM is None:
        _SOLVE_STREAM = torch.cuda.Stream()
    _SOLVE_STREAM.wait_stream(torch.cuda.current_stream())
    return _SOLVE_STREAM, ctypes.c_void_p(_SOLVE_STREAM.cuda_stream)


def _done_on(stream):
    torch = _torch()
    torch.cuda.current_stream().wait_stream(stream)


def _device_bytes(n):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device="cuda")


class TuneResult(ctypes.Structure):
    _fields_ = [("choice", ctypes.c_int * 4), ("ncand", ctypes.c_int * 4), ("ms", (ctypes.c_float * 8) * 4)]


class Pattern:
    """A pattern P(M) with its generating function, stiffness and device data.

    M is 3x3, or 2x2 for a pattern of the plane (plane strain; strains,
    stresses and stiffness matrices then use the 2-D Voigt order 11, 22, 12,
    and fields carry 3 components).  Kernels: 'dirichlet',
    'dirichlet_modified', 'dlvp' ({"alpha": [d values]}) and 'box'
    ({"Xi": d x s directions, "R": alias radius, "tail": add the aliases
    beyond R along slow axes}).  Schemes (set_scheme): 'ls', 've', 'cg', 'ls_inc'.
    """

    def __init__(self, M):
        M = np.asarray(M, dtype=np.int64)
        d = int(M.shape[0]) if M.ndim == 2 else 3
        M = np.ascontiguousarray(M.reshape(d, d))
        h = _P()
        _check(_lib.lsh_create_pattern(d, M.ctypes.data_as(_I64P), ctypes.byref(h)))
        self.d = d
        self.nc = 3 if d == 2 else 6   # strain / stress components (Voigt)
        self._h = h
        m = ctypes.c_int64()
        e = np.zeros(3, dtype=np.int64)
        _check(_lib.lsh_pattern_info(h, ctypes.byref(m), e.ctypes.data_as(_I64P)))
        self.m = int(m.value)
        self.e = tuple(int(v) for v in e)
        self._persist = None
        self._prec = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.lsh_destroy(h)
            self._h = None

    def snf(self):
        U = np.zeros(9, dtype=np.int64)
        V = np.zeros(9, dtype=np.int64)
        _check(_lib.lsh_pattern_snf(self._h, U.ctypes.data_as(_I64P), V.ctypes.data_as(_I64P)))
        return U.reshape(3, 3), V.reshape(3, 3)

    def point_numerators(self):
        y = np.zeros((self.m, self.d), dtype=np.int64)
        _check(_lib.lsh_pattern_points(self._h, y.ctypes.data_as(_I64P)))
        return y

    def points(self):
        return self.point_numerators().astype(np.float64) / self.m

    def set_kernel(self, kind, params=None):
        k = KINDS[kind] if isinstance(kind, str) else int(kind)
        if k == BOXSPLINE and isinstance(params, dict):
            Xi = np.asarray(params["Xi"], dtype=np.float64)
            flat = [float(Xi.shape[1])] + list(Xi.reshape(-1)) + [float(params.get("R", 16))]
            if params.get("tail"):
                flat.append(1.0)
        elif k == DLVP and isinstance(params, dict):
            flat = list(np.asarray(params["alpha"], dtype=np.float64))
        else:
            flat = [] if params is None else list(np.asarray(params, dtype=np.float64).reshape(-1))
        arr = np.ascontiguousarray(flat, dtype=np.float64)
        _check(_lib.lsh_set_kernel(self._h, k, _dptr(arr) if len(arr) else None, len(arr)))
        self._prec = None

    def set_stiffness(self, C_phases_voigt, C0_voigt, phase):
        nc = self.nc
        C = np.ascontiguousarray(np.asarray(C_phases_voigt, dtype=np.float64).reshape(-1, nc, nc))
        C0 = np.ascontiguousarray(np.asarray(C0_voigt, dtype=np.float64).reshape(nc, nc))
        ph = np.ascontiguousarray(np.asarray(phase, dtype=np.uint8).reshape(-1))
        if ph.size != self.m:
            raise ValueError("phase map must have m entries")
        _check(_lib.lsh_set_stiffness(self._h, C.shape[0], _dptr(C), _dptr(C0),
                                      ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        self._prec = None

    def set_scheme(self, scheme):
        """'ls' (Lippmann-Schwinger, default), 've' (variational), 'cg' (conjugate
        gradients, Dirichlet kernel, odd m) or 'ls_inc' (the Lippmann-Schwinger
        iterates computed from their increments); rebind afterwards."""
        _check(_lib.lsh_set_scheme(self._h, {"ls": 0, "ve": 1, "cg": 2, "ls_inc": 3}[scheme]))
        self._prec = None

    def bind(self, precision="fp64"):
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        n = ctypes.c_size_t()
        _check(_lib.lsh_persistent_bytes(self._h, p, ctypes.byref(n)))
        buf = _device_bytes(n.value)
        _check(_lib.lsh_bind(self._h, p, ctypes.c_void_p(buf.data_ptr()), n.value, _stream()))
        self._persist = buf
        self._prec = p
        return n.value

    def gamma_probe(self, bins):
        bins = np.ascontiguousarray(np.asarray(bins, dtype=np.int64).reshape(-1, 3))
        n = len(bins)
        out = np.zeros((n, 21), dtype=np.float64)
        scratch = _device_bytes(256 + 24 * n + 256 + 168 * n + 512)
        _check(_lib.lsh_gamma_probe(self._h, self._prec, bins.ctypes.data_as(_I64P), n, _dptr(out),
                                    ctypes.c_void_p(scratch.data_ptr()), scratch.numel(), _stream()))
        return out

    def workspace_bytes(self, nload, precision=None):
        p = self._prec if precision is None else (PRECISIONS[precision] if isinstance(precision, str) else precision)
        n = ctypes.c_size_t()
        _check(_lib.lsh_solve_bytes(self._h, int(nload), p, ctypes.byref(n)))
        return n.value

    def autotune(self, nload=6, workspace=None):
        """Time each pass's kernel variants on this pattern (lsh_autotune); later
        solves at the bound precision use the fastest.  Returns the choices."""
        if self._prec is None:
            raise RuntimeError("call bind() first")
        need = self.workspace_bytes(nload)
        ws = workspace if workspace is not None and workspace.numel() >= need else _device_bytes(need)
        res = TuneResult()
        S, sh = _solve_stream()
        rc = _lib.lsh_autotune(self._h, int(nload), self._prec, ctypes.c_void_p(ws.data_ptr()), ws.numel(), sh,
                               ctypes.byref(res))
        _done_on(S)
        _check(rc)
        names = ["stress", "axis2", "green", "schedule"]
        return {n: {"choice": res.choice[i], "ms": [round(res.ms[i][c], 5) for c in range(res.ncand[i])]}
                for i, n in enumerate(names)}

    def tune_reset(self):
        _check(_lib.lsh_tune_reset(self._h))

    def tune_set(self, choice, precision=None):
        """Force the variants: (stress, axis2, green[, schedule]); schedule 0 is
        the four-pass iteration, i > 0 the two-pass variant i - 1."""
        p = self._prec if precision is None else (PRECISIONS[precision] if isinstance(precision, str) else precision)
        ch = [int(c) for c in choice] + [0] * (4 - len(choice))
        arr = (ctypes.c_int * 4)(*ch)
        _check(_lib.lsh_tune_set(self._h, int(p), arr))

    def solve(self, eps0_voigt, tol=1e-10, max_iter=1000, E_init=None, return_E=False, history=False,
              workspace=None, allow_notconverged=False):
        """Basic Scheme for all load cases (rows of eps0_voigt)."""
        torch = _torch()
        nc = self.nc
        eps = np.ascontiguousarray(np.asarray(eps0_voigt, dtype=np.float64).reshape(-1, nc))
        nload = eps.shape[0]
        if self._prec is None:
            raise RuntimeError("call bind() first")
        need = self.workspace_bytes(nload)
        ws = workspace if workspace is not None and workspace.numel() >= need else _device_bytes(need)
        Eout = torch.empty((nload, nc, self.m), dtype=torch.float64, device="cuda") if return_E else None
        if E_init is not None:
            if E_init.dtype != torch.float64 or not E_init.is_cuda or E_init.numel() != nload * nc * self.m:
                raise ValueError(f"E_init must be a cuda float64 tensor with nload*{nc}*m entries")
            E_init = E_init.contiguous()
        sig = np.zeros((nload, nc), dtype=np.float64)
        stats = (Stats * nload)()
        hist = np.full((nload, max_iter), np.nan) if history else None
        S, sh = _solve_stream()
        rc = _lib.lsh_solve(self._h, nload, _dptr(eps), float(tol), int(max_iter), self._prec,
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), sh,
                            ctypes.c_void_p(E_init.data_ptr()) if E_init is not None else None,
                            ctypes.c_void_p(Eout.data_ptr()) if Eout is not None else None,
                            _dptr(sig), stats, _dptr(hist) if hist is not None else None)
        _done_on(S)
        _check(rc, allow=(-5,) if allow_notconverged else ())
        out = dict(sigma=sig, status=rc,
                   iterations=np.array([s.iterations for s in stats]),
                   converged=np.array([bool(s.converged) for s in stats]),
                   residual=np.array([s.residual for s in stats]),
                   seconds=stats[0].seconds)
        if return_E:
            out["E"] = Eout
        if history:
            out["history"] = hist
        return out


def solve_batch(patterns, eps0_list, tol=1e-6, max_iter=1000, precision="fp32", workspace=None,
                allow_notconverged=False, E_init=None, return_E=False):
    """Solve many bound patterns at once (lsh_solve_batch).

    patterns: list of Pattern (bound at `precision`); eps0_list: per pattern an
    (nload, nc) array of Voigt strains (nc = 6, or 3 for a 2-D pattern).
    E_init: optional list (one entry per pattern, None for a zero start) of cuda
    float64 tensors (nload, nc, m).  return_E: also return each task's final
    field (nload, nc, m) as "E".
    Returns per pattern a dict with sigma (nload, nc), iterations, converged,
    residual, and the call's status.
    """
    torch = _torch()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = len(patterns)
    tasks = (Task * n)()
    keep = []
    outs = []
    for i, (P, e) in enumerate(zip(patterns, eps0_list)):
        e = np.ascontiguousarray(np.asarray(e, dtype=np.float64).reshape(-1, P.nc))
        sig = np.zeros_like(e)
        st = (Stats * e.shape[0])()
        keep += [e, sig, st]
        tasks[i].p = P._h
        tasks[i].nload = e.shape[0]
        tasks[i].eps0_voigt = _dptr(e)
        tasks[i].sigma_out = _dptr(sig)
        tasks[i].stats = st
        E0 = None if E_init is None else E_init[i]
        if E0 is not None:
            if E0.dtype != torch.float64 or not E0.is_cuda or E0.numel() != e.shape[0] * P.nc * P.m:
                raise ValueError(f"E_init[{i}] must be a cuda float64 tensor with nload*{P.nc}*m entries")
            E0 = E0.contiguous()
            keep.append(E0)
            tasks[i].dev_E_init = E0.data_ptr()
        Eo = torch.empty((e.shape[0], P.nc, P.m), dtype=torch.float64, device="cuda") if return_E else None
        if Eo is not None:
            tasks[i].dev_E_out = Eo.data_ptr()
        outs.append((sig, st, Eo))
    nb = ctypes.c_size_t()
    _check(_lib.lsh_batch_bytes(tasks, n, prec, ctypes.byref(nb)))
    ws = workspace if workspace is not None and workspace.numel() >= nb.value else _device_bytes(nb.value)
    S, sh = _solve_stream()
    rc = _lib.lsh_solve_batch(tasks, n, float(tol), int(max_iter), prec, ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), sh)
    _done_on(S)
    _check(rc, allow=(-5,) if allow_notconverged else ())
    res = []
    for sig, st, Eo in outs:
        r = dict(sigma=sig, iterations=np.array([s.iterations for s in st]),
                 converged=np.array([bool(s.converged) for s in st]),
                 residual=np.array([s.residual for s in st]), status=rc)
        if Eo is not None:
            r["E"] = Eo
        res.append(r)
    return res


def batch_workspace_bytes(patterns, nloads, precision="fp32"):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = len(patterns)
    tasks = (Task * n)()
    dummy = np.zeros((max(nloads), 6))
    for i, (P, k) in enumerate(zip(patterns, nloads)):
        tasks[i].p = P._h
        tasks[i].nload = int(k)
        tasks[i].eps0_voigt = _dptr(dummy)
        tasks[i].sigma_out = _dptr(dummy)
    nb = ctypes.c_size_t()
    _check(_lib.lsh_batch_bytes(tasks, n, prec, ctypes.byref(nb)))
    return nb.value


def profile_enable(on=True):
    _check(_lib.lsh_profile_enable(1 if on else 0))


def profile_select(slots):
    """Time only the given slots (0 stress, 1 axis-2 forward, 2 Green pass,
    3 residual, 4 axis-2 inverse, 5 final stress) while profiling is on."""
    mask = 0
    for i in slots:
        mask |= 1 << int(i)
    _check(_lib.lsh_profile_select(mask))


def profile_read():
    ms = np.zeros(8)
    cnt = np.zeros(8, dtype=np.int64)
    _check(_lib.lsh_profile_read(_dptr(ms), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), 8))
    return ms, cnt


class UNet:
    """Learned warm start (include/lsh_unet.h): a 3-level 3-D U-Net in bf16/MFMA.

    Initial parameters are an input (``lsh_inputs.unet_init_params``).
    """

    def __init__(self, params):
        h = _P()
        _check(_lib.lsh_unet_create(32, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(_lib.lsh_unet_param_count(h, ctypes.byref(n)))
        self.nparam = int(n.value)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if p.size != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        nb = ctypes.c_size_t()
        _check(_lib.lsh_unet_param_bytes(h, ctypes.byref(nb)))
        self._pbuf = _device_bytes(nb.value)
        _check(_lib.lsh_unet_bind(h, ctypes.c_void_p(self._pbuf.data_ptr()), nb.value,
                                  p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream()))
        self._act = {}

    @staticmethod
    def layers():
        h = _P()
        _check(_lib.lsh_unet_create(32, ctypes.byref(h)))
        nl = ctypes.c_int()
        a, b, c = (ctypes.c_int * 16)(), (ctypes.c_int * 16)(), (ctypes.c_int * 16)()
        _check(_lib.lsh_unet_layers(h, ctypes.byref(nl), a, b, c))
        _lib.lsh_unet_destroy(h)
        return [(a[i], b[i], c[i]) for i in range(nl.value)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.lsh_unet_destroy(h)
            self._h = None

    def _workspace(self, n, training):
        key = (n, bool(training))
        if key not in self._act:
            nb = ctypes.c_size_t()
            _check(_lib.lsh_unet_act_bytes(self._h, n, 1 if training else 0, ctypes.byref(nb)))
            self._act[key] = _device_bytes(nb.value)
        return self._act[key]

    def train_step(self, phase, target, n, lr):
        """phase: cuda uint8 (n^3,); target: cuda float32 (n^3, 36).  Returns the loss."""
        ws = self._workspace(n, True)
        loss = ctypes.c_double()
        _check(_lib.lsh_unet_train_step(self._h, ctypes.c_void_p(phase.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                        n, float(lr), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(),
                                        ctypes.byref(loss)))
        return loss.value

    def zero_grad(self):
        _check(_lib.lsh_unet_zero_grad(self._h, _stream()))

    def grads(self):
        g = np.zeros(self.nparam, dtype=np.float32)
        _check(_lib.lsh_unet_get_grads(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream()))
        return g

    def params(self):
        p = np.zeros(self.nparam, dtype=np.float32)
        _check(_lib.lsh_unet_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream()))
        return p

    def head(self, n):
        torch = _torch()
        out = torch.empty((n ** 3, 64), dtype=torch.float32, device="cuda")
        _check(_lib.lsh_unet_head(self._h, n, ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def predict(self, phase, n, eps0_voigt):
        """Start fluctuations [nload][6][n^3] (Voigt, engineering shear) for lsh_solve."""
        torch = _torch()
        eps = np.ascontiguousarray(np.asarray(eps0_voigt, dtype=np.float64).reshape(-1, 6))
        out = torch.empty((eps.shape[0], 6, n ** 3), dtype=torch.float64, device="cuda")
        ws = self._workspace(n, False)
        _check(_lib.lsh_unet_predict(self._h, ctypes.c_void_p(phase.data_ptr()), n, _dptr(eps), eps.shape[0],
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream()))
        return out

    @staticmethod
    def pack_target(E6, n):
        """Six unit-load fields [6][6][n^3] (lsh_solve's E out) -> float32 [n^3][36] (Mandel)."""
        torch = _torch()
        T = torch.empty((n ** 3, 36), dtype=torch.float32, device="cuda")
        _check(_lib.lsh_unet_pack_target(ctypes.c_void_p(E6.data_ptr()), n, ctypes.c_void_p(T.data_ptr()), _stream()))
        return T
