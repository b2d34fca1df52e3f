"""Python binding of the C ABI in include/chem.h (argument marshalling only).

Every step of the integration runs in the HIP library ``libchem.so``; PyTorch
only provides device memory (tensors are passed by ``data_ptr()``) and the
current HIP stream.  Importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchem.so")

CHEM_OK = 0
ERRORS = {-1: "EINVAL", -2: "EHIP", -3: "ENOMEM", -4: "EUNSUPPORTED"}
CELL_STATUS = {0: "OK", 1: "TOO_MANY_STEPS", 2: "STEP_UNDERFLOW", 3: "SINGULAR", 4: "NONFINITE", 5: "TAPE_FULL"}


class ChemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32), ("W", C.c_void_p),
                ("nasa7", C.c_void_p), ("rtype", C.c_void_p), ("reac", C.c_void_p), ("prod", C.c_void_p),
                ("lnA", C.c_void_p), ("b", C.c_void_p), ("theta", C.c_void_p), ("eff", C.c_void_p),
                ("troe", C.c_void_p), ("low", C.c_void_p), ("n_elements", C.c_int32), ("elem", C.c_void_p)]


class RefMap(C.Structure):
    """chem_refmap (reference-cell mapping of low-reactivity cells); see include/chem.h."""
    _fields_ = [("weight", C.c_void_p), ("z0", C.c_double), ("z_max", C.c_double), ("dT", C.c_double),
                ("ref_of", C.c_void_p)]

    def __init__(self, weight, z0=0.0, z_max=0.0, dT=0.0, ref_of=None):
        """weight: float64 CUDA tensor [K]; ref_of: None or an int32 CUDA tensor [ncells] (output)."""
        _dev(weight, torch.float64, "weight")
        _dev(ref_of, torch.int32, "ref_of")
        super().__init__(weight.data_ptr(), z0, z_max, dT, ref_of.data_ptr() if ref_of is not None else None)
        self._keep = (weight, ref_of)


class Options(C.Structure):
    """chem_options; see include/chem.h for the meaning and defaults."""
    _fields_ = [("method", C.c_int32), ("max_steps", C.c_int32), ("fac_safe", C.c_double),
                ("fac_min", C.c_double), ("fac_max", C.c_double), ("h_min", C.c_double),
                ("persistent", C.c_int32), ("waves_per_block", C.c_int32), ("grid_mult", C.c_int32),
                ("cost_order", C.c_int32), ("use_graph", C.c_int32), ("phase_cycles", C.c_void_p),
                ("jac_mode", C.c_int32), ("lu_pivot", C.c_int32), ("refmap", C.POINTER(RefMap)),
                ("jac_slots", C.c_int32), ("fail_lu_lo", C.c_int64), ("fail_lu_hi", C.c_int64)]

    def __init__(self, method=0, max_steps=100000, fac_safe=0.9, fac_min=0.2, fac_max=6.0, h_min=1e-20,
                 persistent=-1, waves_per_block=0, grid_mult=0, cost_order=0, use_graph=0, phase_cycles=None,
                 jac_mode=0, lu_pivot=0, refmap=None, jac_slots=0, fail_lu=(0, 0)):
        """phase_cycles: None or an int64 CUDA tensor [ncells, 8] (per-phase shader cycles);
        jac_mode 1 / lu_pivot 1 select the finite-difference Jacobian / unpivoted LU (ablation);
        refmap: None or a RefMap; fail_lu = (lo, hi): testing, cells lo..hi-1 see every
        factorisation as singular."""
        ptr = phase_cycles.data_ptr() if phase_cycles is not None else None
        rp = C.pointer(refmap) if refmap is not None else None
        super().__init__(method, max_steps, fac_safe, fac_min, fac_max, h_min, persistent, waves_per_block,
                         grid_mult, cost_order, use_graph, ptr, jac_mode, lu_pivot, rp, jac_slots,
                         int(fail_lu[0]), int(fail_lu[1]))
        self._keep = (phase_cycles, refmap)


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2105_12070_amd.build.build() "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        L.chem_last_error.restype = C.c_char_p
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.chem_load_mechanism.argtypes = [C.POINTER(_Desc), C.POINTER(vp)]
        L.chem_free_mechanism.argtypes = [vp]
        L.chem_free_mechanism.restype = None
        L.chem_mech_sizes.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.chem_set_arrhenius.argtypes = [vp, vp, vp, vp, vp]
        L.chem_integrate.argtypes = [vp, i64, i64, vp, vp, d, d, d, d, C.POINTER(Options), vp, vp, vp, vp]
        L.chem_integrate_adjoint.argtypes = [vp, i64, i64, vp, vp, d, d, d, d, C.POINTER(Options), vp, vp, vp,
                                             vp, i32, i32, vp, vp, vp]
        L.chem_rhs.argtypes = [vp, i64, i64, vp, d, vp, vp]
        L.chem_jacobian.argtypes = [vp, i64, i64, vp, d, vp, vp, vp]
        L.chem_lu_solve.argtypes = [i64, i32, vp, vp, vp, vp]
        L.chem_lu_factor.argtypes = [i64, i32, vp, vp, vp, vp, vp]
        L.chem_failed_count.argtypes = [vp, C.POINTER(i64), vp]
        L.chem_integrate_noalloc.argtypes = [vp, i64, i64, vp, vp, d, d, d, d, C.POINTER(Options), vp, vp, vp,
                                             vp]
        L.chem_autotune.argtypes = [vp, i64, i64, vp, vp, d, d, d, d, vp, vp, vp]
        L.chem_set_variant.argtypes = [vp, vp]
        L.chem_set_adjoint_record_budget.argtypes = [C.c_uint64]
        _lib = L
    return _lib


def _check(rc):
    if rc != CHEM_OK:
        raise ChemError(rc, lib().chem_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, name):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return t


class Mechanism:
    """A mechanism uploaded to the current device (owns a chem_mech handle)."""

    def __init__(self, mech: dict):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        self._arrays = dict(W=f64(mech["W"]), nasa7=f64(mech["nasa7"]), rtype=i32(mech["rtype"]),
                            reac=i32(mech["reac"]), prod=i32(mech["prod"]), lnA=f64(mech["lnA"]),
                            b=f64(mech["b"]), theta=f64(mech["theta"]), eff=f64(mech["eff"]),
                            troe=f64(mech["troe"]), low=f64(mech["low"]))
        a = self._arrays
        if mech.get("elem") is not None:
            a["elem"] = i32(mech["elem"])
        desc = _Desc(int(mech["n_species"]), int(mech["n_reactions"]),
                     *(a[k].ctypes.data for k in ("W", "nasa7", "rtype", "reac", "prod", "lnA", "b", "theta",
                                                  "eff", "troe", "low")),
                     int(a["elem"].shape[1]) if "elem" in a else 0,
                     a["elem"].ctypes.data if "elem" in a else None)
        h = C.c_void_p()
        _check(lib().chem_load_mechanism(C.byref(desc), C.byref(h)))
        self._h = h
        self.K = int(mech["n_species"])
        self.R = int(mech["n_reactions"])
        self.N = self.K + 1

    @property
    def handle(self):
        return self._h

    def set_arrhenius(self, lnA, b, theta):
        for t, n in ((lnA, "lnA"), (b, "b"), (theta, "theta")):
            _dev(t, torch.float64, n)
        _check(lib().chem_set_arrhenius(self._h, _ptr(lnA), _ptr(b), _ptr(theta), _stream()))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.chem_free_mechanism(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def integrate(mech: Mechanism, state, h, p, dt, rtol=1e-6, atol=1e-10, options: Options | None = None,
              steps=None, rejects=None, status=None, ncells=None):
    """chem_integrate on an [N, ld] float64 CUDA tensor, in place."""
    _dev(state, torch.float64, "state")
    _dev(h, torch.float64, "h")
    for t, n in ((steps, "steps"), (rejects, "rejects"), (status, "status")):
        _dev(t, torch.int32, n)
    N, ld = state.shape
    if N != mech.N:
        raise ValueError(f"state has {N} rows, mechanism needs {mech.N}")
    nc = ld if ncells is None else int(ncells)
    opt = C.byref(options) if options is not None else None
    _check(lib().chem_integrate(mech.handle, nc, ld, _ptr(state), _ptr(h), float(p), float(dt), float(rtol),
                                float(atol), opt, _ptr(steps), _ptr(rejects), _ptr(status), _stream()))


def integrate_noalloc(mech: Mechanism, state, h, p, dt, rtol=1e-6, atol=1e-10, options: Options | None = None,
                      steps=None, rejects=None, status=None, ncells=None):
    """chem_integrate_noalloc (no device allocation; scratch in the library's
    per-GPU array) on an [N, ld] float64 CUDA tensor, in place."""
    _dev(state, torch.float64, "state")
    _dev(h, torch.float64, "h")
    for t, n in ((steps, "steps"), (rejects, "rejects"), (status, "status")):
        _dev(t, torch.int32, n)
    N, ld = state.shape
    if N != mech.N:
        raise ValueError(f"state has {N} rows, mechanism needs {mech.N}")
    nc = ld if ncells is None else int(ncells)
    opt = C.byref(options) if options is not None else None
    _check(lib().chem_integrate_noalloc(mech.handle, nc, ld, _ptr(state), _ptr(h), float(p), float(dt),
                                        float(rtol), float(atol), opt, _ptr(steps), _ptr(rejects), _ptr(status),
                                        _stream()))


def integrate_adjoint(mech: Mechanism, state0, h, p, dt, rtol, atol, lambda_final, options: Options | None = None,
                      checkpoint_every=8, max_tape=0, want_lambda0=True):
    """chem_integrate_adjoint; returns (state_final, lambda0, grad[3, R], steps, status)."""
    _dev(state0, torch.float64, "state0")
    _dev(h, torch.float64, "h")
    _dev(lambda_final, torch.float64, "lambda_final")
    N, ld = state0.shape
    out = torch.empty_like(state0)
    lam0 = torch.empty_like(state0) if want_lambda0 else None
    grad = torch.empty((3, mech.R), dtype=torch.float64, device=state0.device)
    steps = torch.empty(ld, dtype=torch.int32, device=state0.device)
    status = torch.empty(ld, dtype=torch.int32, device=state0.device)
    opt = C.byref(options) if options is not None else None
    _check(lib().chem_integrate_adjoint(mech.handle, ld, ld, _ptr(state0), _ptr(h), float(p), float(dt),
                                        float(rtol), float(atol), opt, _ptr(lambda_final), _ptr(out), _ptr(lam0),
                                        _ptr(grad), int(checkpoint_every), int(max_tape), _ptr(steps),
                                        _ptr(status), _stream()))
    return out, lam0, grad, steps, status


class IntegrateFn(torch.autograd.Function):
    """state_final = integrate(state0; lnA, b, theta) with a discrete-adjoint backward.

    The forward pass is chem_integrate from a cold step size; the backward pass
    calls chem_integrate_adjoint, which recomputes the forward pass with its
    tape (identical arithmetic, so the same accepted steps) and sweeps it
    backwards.  Gradients flow to state0 and to the three Arrhenius arrays
    (device tensors of length R in descriptor order, loaded into the
    mechanism on every call).
    """

    @staticmethod
    def forward(ctx, state0, lnA, b, theta, mech, p, dt, rtol, atol, options, checkpoint_every, max_tape):
        mech.set_arrhenius(lnA.detach().contiguous(), b.detach().contiguous(), theta.detach().contiguous())
        st = state0.detach().clone().contiguous()
        h = torch.zeros(st.shape[1], dtype=torch.float64, device=st.device)
        status = torch.empty(st.shape[1], dtype=torch.int32, device=st.device)
        integrate(mech, st, h, p, dt, rtol, atol, options=options, status=status)
        _raise_failed(status, "forward integration")
        ctx.save_for_backward(state0.detach(), lnA.detach(), b.detach(), theta.detach())
        ctx.cfg = (mech, p, dt, rtol, atol, options, checkpoint_every, max_tape)
        return st

    @staticmethod
    def backward(ctx, gout):
        state0, lnA, b, theta = ctx.saved_tensors
        mech, p, dt, rtol, atol, options, ck, mt = ctx.cfg
        mech.set_arrhenius(lnA.contiguous(), b.contiguous(), theta.contiguous())
        h = torch.zeros(state0.shape[1], dtype=torch.float64, device=state0.device)
        _, lam0, grad, _, status = integrate_adjoint(mech, state0.contiguous(), h, p, dt, rtol, atol,
                                                     gout.contiguous(), options=options, checkpoint_every=ck,
                                                     max_tape=mt)
        # a cell without a complete reverse sweep (TAPE_FULL, or a failed
        # forward) would contribute lambda0 = lambda_final and no parameter
        # gradient: refuse to return such gradients
        _raise_failed(status, "adjoint")
        return lam0, grad[0], grad[1], grad[2], None, None, None, None, None, None, None, None


def _raise_failed(status, what):
    bad = status != 0
    if bool(bad.any()):
        codes = torch.unique(status[bad]).tolist()
        raise ChemError(-1, f"{what}: {int(bad.sum())} cells ended with status "
                        f"{', '.join(CELL_STATUS.get(c, str(c)) for c in codes)}")


def integrate_diff(mech: Mechanism, state0, lnA, b, theta, p, dt, rtol=1e-6, atol=1e-10,
                   options: Options | None = None, checkpoint_every=8, max_tape=0):
    """Differentiable integration over one CFD step (see IntegrateFn).  max_tape
    bounds the accepted steps per cell that the backward pass records (0 =
    4096); forward and backward raise ChemError if any cell fails."""
    return IntegrateFn.apply(state0, lnA, b, theta, mech, p, dt, rtol, atol, options, checkpoint_every, max_tape)


def rhs(mech: Mechanism, state, p):
    _dev(state, torch.float64, "state")
    N, ld = state.shape
    f = torch.empty_like(state)
    _check(lib().chem_rhs(mech.handle, ld, ld, _ptr(state), float(p), _ptr(f), _stream()))
    return f


def jacobian(mech: Mechanism, state, p):
    _dev(state, torch.float64, "state")
    N, ld = state.shape
    J = torch.empty((ld, N, N), dtype=torch.float64, device=state.device)
    f = torch.empty_like(state)
    _check(lib().chem_jacobian(mech.handle, ld, ld, _ptr(state), float(p), _ptr(J), _ptr(f), _stream()))
    return J, f


def lu_solve(A, b):
    """Batched A x = b (A [nmat, n, n], b [nmat, n]); returns (x, info)."""
    _dev(A, torch.float64, "A")
    _dev(b, torch.float64, "b")
    nmat, n, _ = A.shape
    x = b.clone()
    info = torch.empty(nmat, dtype=torch.int32, device=A.device)
    _check(lib().chem_lu_solve(nmat, n, _ptr(A), _ptr(x), _ptr(info), _stream()))
    return x, info


def lu_factor(A):
    """Batched getrf (A [nmat, n, n]); returns (LU, ipiv (0-based), info)."""
    _dev(A, torch.float64, "A")
    nmat, n, _ = A.shape
    LU = torch.empty_like(A)
    ipiv = torch.empty((nmat, n), dtype=torch.int32, device=A.device)
    info = torch.empty(nmat, dtype=torch.int32, device=A.device)
    _check(lib().chem_lu_factor(nmat, n, _ptr(A), _ptr(LU), _ptr(ipiv), _ptr(info), _stream()))
    return LU, ipiv, info


def failed_count(mech: Mechanism) -> int:
    """chem_failed_count: cells with a nonzero status in the mechanism's last integration."""
    out = C.c_int64()
    _check(lib().chem_failed_count(mech.handle, C.byref(out), _stream()))
    return out.value


VARIANT_KEYS = ("persistent", "waves_per_block", "grid_mult", "jac_slots")


def _tune_key(mech: Mechanism, method: str) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    return f"{arch}/N={mech.N}/R={mech.R}/{method}"


def default_tune_cache() -> str:
    return os.environ.get("CHEM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2105_12070_amd", "autotune.json"))


def set_variant(mech: Mechanism, variant: dict) -> None:
    """chem_set_variant: install a stored launch variant as the mechanism's default."""
    v = (C.c_int32 * 4)(*(int(variant[k]) for k in VARIANT_KEYS))
    _check(lib().chem_set_variant(mech.handle, C.cast(v, C.c_void_p)))


def autotune(mech: Mechanism, state, h, p, dt, rtol=1e-6, atol=1e-10, cache: str | None = None,
             method: str = "ros4"):
    """Launch variant of the mechanism: from the JSON cache (keyed by GPU
    architecture, N, R and method) when it holds one, else timed by
    chem_autotune on (a scratch copy of) the input and stored there.  Returns
    (variant dict, ms or None when it came from the cache).  cache=None uses
    default_tune_cache(); cache="" disables it."""
    import json
    _dev(state, torch.float64, "state")
    _dev(h, torch.float64, "h")
    path = default_tune_cache() if cache is None else cache
    key = _tune_key(mech, method)
    table = {}
    if path and os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
        if key in table:
            set_variant(mech, table[key])
            return dict(table[key]), None
    N, ld = state.shape
    v = (C.c_int32 * 4)()
    ms = C.c_double()
    _check(lib().chem_autotune(mech.handle, ld, ld, _ptr(state), _ptr(h), float(p), float(dt), float(rtol),
                               float(atol), C.cast(v, C.c_void_p), C.cast(C.pointer(ms), C.c_void_p), _stream()))
    variant = dict(zip(VARIANT_KEYS, list(v)))
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        table[key] = variant
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return variant, ms.value


def set_adjoint_record_budget(nbytes: int) -> None:
    """chem_set_adjoint_record_budget: bytes of per-step records the adjoint
    may keep for its backward walk (0 = replay every step)."""
    _check(lib().chem_set_adjoint_record_budget(int(nbytes)))


EXPORTED = ["chem_load_mechanism", "chem_free_mechanism", "chem_max_n", "chem_mech_sizes", "chem_set_arrhenius",
            "chem_integrate", "chem_integrate_adjoint", "chem_set_adjoint_record_budget", "chem_rhs",
            "chem_jacobian", "chem_lu_solve", "chem_lu_factor", "chem_failed_count", "chem_autotune",
            "chem_last_error", "chem_integrate_noalloc", "chem_set_variant"]
