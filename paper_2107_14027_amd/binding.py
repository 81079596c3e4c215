"""ctypes binding of libfr.so (include/fr.h): same entry-point names, argument
marshalling only.  Device arrays are torch tensors on a ROCm device; every step
of the computation runs in the HIP library.  There is no fallback: if the
library is not built, or a call fails, an exception is raised."""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FR_LIBRARY", os.path.join(HERE, "libfr.so"))

FR_OK, FR_EINVAL, FR_ENOMEM, FR_EHIP, FR_ENONFINITE, FR_ENOCONV, FR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
(FR_OPT_PRECISION, FR_OPT_VARIANT, FR_OPT_BLOCK, FR_OPT_PROFILE, FR_OPT_GUESS_BASE,
 FR_OPT_GRAPH, FR_OPT_FUSE_STAGE, FR_OPT_PSEUDO, FR_OPT_FORM) = 1, 2, 3, 4, 5, 6, 7, 8, 9
KERNELS = ("trace", "fused", "u_project", "u_flux", "u_div", "u_common", "u_correct",
           "u_negsrc", "stage")
FR_F64, FR_F32 = 0, 1
FR_K_TRACE, FR_K_FUSED = 0, 1
FR_FUSED, FR_UNFUSED, FR_MFMA = 0, 1, 2
FR_FORM_AUTO, FR_FORM_POINT, FR_FORM_LINES, FR_FORM_HALO = 0, 1, 2, 3
FR_INFO_RESIDUAL_FORM, FR_INFO_STAGE_PATH = 100, 101
FR_STAGE_SEPARATE, FR_STAGE_POINT, FR_STAGE_HALO = 0, 1, 2
NV = 13

EXPORTED = ("fr_plan_create", "fr_plan_set_int", "fr_plan_get_int", "fr_plan_destroy",
            "fr_state_len", "fr_residual", "fr_rk_step", "fr_dual_step", "fr_guess_extrap",
            "fr_strerror", "fr_last_error", "fr_plan_operators", "fr_plan_kernel_stats",
            "fr_mlp_state_floats", "fr_mlp_init", "fr_mlp_sample", "fr_mlp_fit_norm",
            "fr_mlp_forward", "fr_mlp_grad", "fr_mlp_train_step", "fr_mlp_guess",
            "fr_pmg_create", "fr_pmg_dual_step", "fr_pmg_destroy", "fr_diagnostics",
            "fr_acm_create", "fr_acm_residual", "fr_acm_gradient", "fr_acm_dual_step",
            "fr_acm_destroy", "fr_lhex_create", "fr_lhex_residual", "fr_lhex_destroy",
            "fr_launch_shape", "fr_mlp_guess_checked", "fr_residual_noalloc")


class FrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_strerror(code), code, msg))
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libfr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfr.so is not built (run: python -m paper_2107_14027_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        I, D = ctypes.c_int, ctypes.c_double
        L.fr_plan_create.argtypes = [I, I, I, I, _dp, D, _dp]
        L.fr_plan_create.restype = _vp
        L.fr_plan_set_int.argtypes = [_vp, I, I]
        L.fr_plan_get_int.argtypes = [_vp, I, ctypes.POINTER(I)]
        L.fr_plan_destroy.argtypes = [_vp]
        L.fr_plan_destroy.restype = None
        L.fr_state_len.argtypes = [_vp]
        L.fr_state_len.restype = ctypes.c_size_t
        L.fr_residual.argtypes = [_vp, _vp, _vp, _vp]
        L.fr_residual_noalloc.argtypes = [_vp, _vp, _vp, _vp]
        L.fr_rk_step.argtypes = [_vp, _vp, D, I, _vp]
        L.fr_dual_step.argtypes = [_vp, _vp, _vp, _vp, D, D, D, I, I, ctypes.POINTER(I), _dp, _vp]
        L.fr_guess_extrap.argtypes = [_vp, _vp, _vp, _vp, I, _vp, _vp]
        L.fr_strerror.argtypes = [I]
        L.fr_strerror.restype = ctypes.c_char_p
        L.fr_last_error.argtypes = []
        L.fr_last_error.restype = ctypes.c_char_p
        L.fr_plan_operators.argtypes = [I, _dp]
        L.fr_launch_shape.argtypes = [I, I, I, ctypes.POINTER(I)]
        L.fr_plan_kernel_stats.argtypes = [_vp, I, _dp, ctypes.POINTER(ctypes.c_int64), I]
        I64, F = ctypes.c_int64, ctypes.c_float
        L.fr_mlp_state_floats.argtypes = []
        L.fr_mlp_state_floats.restype = ctypes.c_size_t
        L.fr_mlp_init.argtypes = [_vp, ctypes.c_uint64, _vp]
        L.fr_mlp_sample.argtypes = [_vp, _vp, _vp, _vp, _vp, I64, I64, I64, _vp, _vp, _vp]
        L.fr_mlp_fit_norm.argtypes = [_vp, _vp, _vp, _vp, I64, _vp]
        L.fr_mlp_forward.argtypes = [_vp, _vp, _vp, I64, _vp, _vp]
        L.fr_mlp_grad.argtypes = [_vp, _vp, _vp, _vp, I64, _vp, _vp, _vp]
        L.fr_mlp_train_step.argtypes = [_vp, _vp, _vp, _vp, I64, F, I, _vp, _vp]
        L.fr_mlp_guess.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.fr_mlp_guess_checked.argtypes = [_vp, _vp, _vp, _vp, _vp, D, D, _vp, ctypes.POINTER(I),
                                           _dp, _vp]
        L.fr_pmg_create.argtypes = [_vp, I, ctypes.POINTER(I), ctypes.POINTER(I), D]
        L.fr_pmg_create.restype = _vp
        L.fr_pmg_dual_step.argtypes = [_vp, _vp, _vp, _vp, D, D, D, I, ctypes.POINTER(I), _dp, _vp]
        L.fr_diagnostics.argtypes = [_vp, _vp, _dp, _vp]
        L.fr_pmg_destroy.argtypes = [_vp]
        L.fr_pmg_destroy.restype = None
        L.fr_acm_create.argtypes = [_vp, D, D]
        L.fr_acm_create.restype = _vp
        L.fr_acm_residual.argtypes = [_vp, _vp, _vp, _vp]
        L.fr_acm_gradient.argtypes = [_vp, _vp, _vp, _vp]
        L.fr_acm_dual_step.argtypes = [_vp, _vp, _vp, _vp, D, D, D, I, I, ctypes.POINTER(I), _dp, _vp]
        L.fr_lhex_create.argtypes = [_vp]
        L.fr_lhex_create.restype = _vp
        L.fr_lhex_residual.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.fr_lhex_destroy.argtypes = [_vp]
        L.fr_lhex_destroy.restype = None
        L.fr_acm_destroy.argtypes = [_vp]
        L.fr_acm_destroy.restype = None
        for n in ("fr_plan_set_int", "fr_plan_get_int", "fr_residual", "fr_rk_step", "fr_pmg_dual_step", "fr_diagnostics",
                  "fr_dual_step", "fr_guess_extrap", "fr_plan_operators", "fr_plan_kernel_stats",
                  "fr_mlp_init", "fr_mlp_sample", "fr_mlp_fit_norm", "fr_mlp_forward",
                  "fr_mlp_grad", "fr_mlp_train_step", "fr_mlp_guess", "fr_acm_residual",
                  "fr_acm_gradient", "fr_acm_dual_step", "fr_lhex_residual"):
            getattr(L, n).restype = I
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().fr_strerror(code).decode()
    except Exception:  # pragma: no cover
        return "error"


def _check(rc):
    if rc != FR_OK:
        raise FrError(rc, lib().fr_last_error().decode())
    return rc


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _dev(t, dtype=None, n=None, name="array"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a torch tensor on the GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return _vp(t.data_ptr())


# --------------------------------------------------------------------------- entry points
def fr_plan_create(p, nx, ny, nz, jac, acm_zeta, hd_relax):
    j = None if jac is None else np.ascontiguousarray(jac, dtype=np.float64).reshape(9)
    h = np.ascontiguousarray(hd_relax, dtype=np.float64).reshape(2)
    ptr = lib().fr_plan_create(p, nx, ny, nz, None if j is None else j.ctypes.data_as(_dp),
                               float(acm_zeta), h.ctypes.data_as(_dp))
    if not ptr:
        raise FrError(FR_EINVAL, lib().fr_last_error().decode())
    return ptr


def fr_plan_set_int(plan, key, value):
    return _check(lib().fr_plan_set_int(plan, key, value))


def fr_plan_get_int(plan, key):
    v = ctypes.c_int()
    _check(lib().fr_plan_get_int(plan, key, ctypes.byref(v)))
    return v.value


def fr_plan_destroy(plan):
    lib().fr_plan_destroy(plan)


def fr_state_len(plan):
    return lib().fr_state_len(plan)


def fr_residual(plan, U, R, stream=None):
    import torch
    n = fr_state_len(plan)
    dt = torch.float64 if fr_plan_get_int(plan, FR_OPT_PRECISION) == FR_F64 else torch.float32
    return _check(lib().fr_residual(plan, _dev(U, dt, n, "U"), _dev(R, dt, n, "R"),
                                    _stream(stream)))


def fr_residual_noalloc(plan, U, R, stream=None):
    import torch
    n = fr_state_len(plan)
    dt = torch.float64 if fr_plan_get_int(plan, FR_OPT_PRECISION) == FR_F64 else torch.float32
    return _check(lib().fr_residual_noalloc(plan, _dev(U, dt, n, "U"), _dev(R, dt, n, "R"),
                                            _stream(stream)))


def fr_rk_step(plan, U, dt, nsteps, stream=None):
    import torch
    n = fr_state_len(plan)
    return _check(lib().fr_rk_step(plan, _dev(U, torch.float64, n, "U"), float(dt), int(nsteps),
                                   _stream(stream)))


def fr_dual_step(plan, U, Un, Unm1, dt, dtau, tol, max_iters, check_every=1, stream=None,
                 raise_on_error=True):
    """Returns (status, iters, resid)."""
    import torch
    n = fr_state_len(plan)
    it = ctypes.c_int()
    res = ctypes.c_double()
    rc = lib().fr_dual_step(plan, _dev(U, torch.float64, n, "U"), _dev(Un, torch.float64, n, "Un"),
                            None if Unm1 is None else _dev(Unm1, torch.float64, n, "Unm1"),
                            float(dt), float(dtau), float(tol), int(max_iters), int(check_every),
                            ctypes.byref(it), ctypes.byref(res), _stream(stream))
    if raise_on_error and rc not in (FR_OK, FR_ENOCONV):
        _check(rc)
    return rc, it.value, res.value


def fr_pmg_create(plan, cycle=None, factor=1.75):
    """cycle: list of (order, pseudo-steps), or None for the paper's cycle shape."""
    if cycle is None:
        ptr = lib().fr_pmg_create(plan, 0, None, None, float(factor))
    else:
        o = (ctypes.c_int * len(cycle))(*[int(c[0]) for c in cycle])
        k = (ctypes.c_int * len(cycle))(*[int(c[1]) for c in cycle])
        ptr = lib().fr_pmg_create(plan, len(cycle), o, k, float(factor))
    if not ptr:
        raise FrError(FR_EINVAL, lib().fr_last_error().decode())
    return ptr


def fr_pmg_dual_step(mg, U, Un, Unm1, dt, dtau, tol, max_cycles, n, stream=None,
                     raise_on_error=True):
    """Returns (status, cycles, resid); n is the fine plan's state length."""
    import torch
    cyc = ctypes.c_int()
    res = ctypes.c_double()
    rc = lib().fr_pmg_dual_step(mg, _dev(U, torch.float64, n, "U"), _dev(Un, torch.float64, n, "Un"),
                                None if Unm1 is None else _dev(Unm1, torch.float64, n, "Unm1"),
                                float(dt), float(dtau), float(tol), int(max_cycles),
                                ctypes.byref(cyc), ctypes.byref(res), _stream(stream))
    if raise_on_error and rc not in (FR_OK, FR_ENOCONV):
        _check(rc)
    return rc, cyc.value, res.value


def fr_diagnostics(plan, U, stream=None):
    """(kinetic energy, enstrophy) of a double state U."""
    import torch
    out = np.zeros(2)
    _check(lib().fr_diagnostics(plan, _dev(U, torch.float64, fr_state_len(plan), "U"),
                                out.ctypes.data_as(_dp), _stream(stream)))
    return float(out[0]), float(out[1])


def fr_pmg_destroy(mg):
    lib().fr_pmg_destroy(mg)


def fr_acm_create(plan, beta=0.5, tau=0.1):
    ptr = lib().fr_acm_create(plan, float(beta), float(tau))
    if not ptr:
        raise FrError(FR_EINVAL, lib().fr_last_error().decode())
    return ptr


def fr_acm_residual(acm, U, R, n, stream=None):
    """R = -div F of the standard-ACM state U (both [ne][4][m^3] double, n values)."""
    import torch
    return _check(lib().fr_acm_residual(acm, _dev(U, torch.float64, n, "U"),
                                        _dev(R, torch.float64, n, "R"), _stream(stream)))


def fr_acm_gradient(acm, U, Q, n, stream=None):
    """Q[e][3 i + j][m^3] = du_i/dx_j of the standard-ACM state U (n values)."""
    import torch
    return _check(lib().fr_acm_gradient(acm, _dev(U, torch.float64, n, "U"),
                                        _dev(Q, torch.float64, n // 4 * 9, "Q"), _stream(stream)))


def fr_acm_dual_step(acm, U, Un, Unm1, dt, dtau, tol, max_iters, n, check_every=1, stream=None,
                     raise_on_error=True):
    """Returns (status, iters, resid) of one BDF physical step of the standard-ACM state U."""
    import torch
    it = ctypes.c_int()
    res = ctypes.c_double()
    rc = lib().fr_acm_dual_step(acm, _dev(U, torch.float64, n, "U"), _dev(Un, torch.float64, n, "Un"),
                                None if Unm1 is None else _dev(Unm1, torch.float64, n, "Unm1"),
                                float(dt), float(dtau), float(tol), int(max_iters), int(check_every),
                                ctypes.byref(it), ctypes.byref(res), _stream(stream))
    if raise_on_error and rc not in (FR_OK, FR_ENOCONV):
        _check(rc)
    return rc, it.value, res.value


def fr_acm_destroy(acm):
    lib().fr_acm_destroy(acm)


FR_GUESS_KEEP_P = 0x10   # or-ed into the order of fr_guess_extrap: pressure from Un


def fr_guess_extrap(plan, Un, Unm1, Unm2, order, G, stream=None):
    import torch
    n = fr_state_len(plan)
    f = lambda t, nm: None if t is None else _dev(t, torch.float64, n, nm)
    return _check(lib().fr_guess_extrap(plan, f(Un, "Un"), f(Unm1, "Unm1"), f(Unm2, "Unm2"),
                                        int(order), f(G, "G"), _stream(stream)))


def fr_plan_kernel_stats(plan, kernel, reset=False):
    """(total_ms, launches) recorded for a kernel id while FR_OPT_PROFILE was on."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().fr_plan_kernel_stats(plan, int(kernel), ctypes.byref(ms), ctypes.byref(n),
                                      int(bool(reset))))
    return ms.value, n.value


# --------------------------------------------------------------------------- learned guess
MLP_NPAR = 5252
MLP_SHAPES = (("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (4, 64)), ("b3", (4,)))


def fr_mlp_state_floats():
    return lib().fr_mlp_state_floats()


def mlp_new_state(seed=0, stream=None):
    """A device float32 tensor holding an initialised network state."""
    import torch
    st = torch.zeros(fr_mlp_state_floats(), dtype=torch.float32, device="cuda")
    _check(lib().fr_mlp_init(_vp(st.data_ptr()), int(seed), _stream(stream)))
    return st


def mlp_params(state):
    """Split the parameter part of a state tensor into named views."""
    out, o = {}, 0
    for k, shp in MLP_SHAPES:
        n = int(np.prod(shp))
        out[k] = state[o:o + n].view(*shp)
        o += n
    return out


def fr_mlp_sample(plan, Un, Unm1, Unm2, Unp1, offset, stride, n, X, Y, stream=None):
    import torch
    ns = fr_state_len(plan)
    d = lambda t, nm: None if t is None else _dev(t, torch.float64, ns, nm)
    return _check(lib().fr_mlp_sample(plan, d(Un, "Un"), d(Unm1, "Unm1"), d(Unm2, "Unm2"),
                                      d(Unp1, "Unp1"), int(offset), int(stride), int(n),
                                      _dev(X, torch.float32, 12 * n, "X"),
                                      _dev(Y, torch.float32, 4 * n, "Y"), _stream(stream)))


def fr_mlp_fit_norm(plan, state, X, Y, stream=None):
    import torch
    n = X.numel() // 12
    return _check(lib().fr_mlp_fit_norm(plan, _dev(state, torch.float32, None, "state"),
                                        _dev(X, torch.float32, 12 * n, "X"),
                                        _dev(Y, torch.float32, 4 * n, "Y"), n, _stream(stream)))


def fr_mlp_forward(plan, state, X, Yout, stream=None):
    import torch
    n = X.numel() // 12
    return _check(lib().fr_mlp_forward(plan, _dev(state, torch.float32, None, "state"),
                                       _dev(X, torch.float32, 12 * n, "X"), n,
                                       _dev(Yout, torch.float32, 4 * n, "Yout"), _stream(stream)))


def fr_mlp_grad(plan, state, X, Y, grad, loss=None, stream=None):
    import torch
    n = X.numel() // 12
    return _check(lib().fr_mlp_grad(plan, _dev(state, torch.float32, None, "state"),
                                    _dev(X, torch.float32, 12 * n, "X"),
                                    _dev(Y, torch.float32, 4 * n, "Y"), n,
                                    _dev(grad, torch.float32, MLP_NPAR, "grad"),
                                    None if loss is None else _dev(loss, torch.float32, None, "loss"),
                                    _stream(stream)))


def fr_mlp_train_step(plan, state, X, Y, lr, step, loss=None, stream=None):
    import torch
    n = X.numel() // 12
    return _check(lib().fr_mlp_train_step(plan, _dev(state, torch.float32, None, "state"),
                                          _dev(X, torch.float32, 12 * n, "X"),
                                          _dev(Y, torch.float32, 4 * n, "Y"), n, float(lr),
                                          int(step),
                                          None if loss is None else _dev(loss, torch.float32, None, "loss"),
                                          _stream(stream)))


def fr_mlp_guess(plan, state, Un, Unm1, Unm2, G, stream=None):
    import torch
    ns = fr_state_len(plan)
    return _check(lib().fr_mlp_guess(plan, _dev(state, torch.float32, None, "state"),
                                     _dev(Un, torch.float64, ns, "Un"),
                                     _dev(Unm1, torch.float64, ns, "Unm1"),
                                     _dev(Unm2, torch.float64, ns, "Unm2"),
                                     _dev(G, torch.float64, ns, "G"), _stream(stream)))


def fr_mlp_guess_checked(plan, state, Un, Unm1, Unm2, dt, G, accept_ratio=1.0, stream=None):
    """Learned guess with extrapolation as fallback; returns (used_network,
    network's initial norm, extrapolation's initial norm)."""
    import torch
    ns = fr_state_len(plan)
    used = ctypes.c_int(0)
    norms = np.zeros(2)
    _check(lib().fr_mlp_guess_checked(plan, _dev(state, torch.float32, None, "state"),
                                      _dev(Un, torch.float64, ns, "Un"),
                                      _dev(Unm1, torch.float64, ns, "Unm1"),
                                      _dev(Unm2, torch.float64, ns, "Unm2"), dt, accept_ratio,
                                      _dev(G, torch.float64, ns, "G"), ctypes.byref(used),
                                      norms.ctypes.data_as(_dp), _stream(stream)))
    return bool(used.value), float(norms[0]), float(norms[1])


def fr_launch_shape(p, precision, kernel):
    """Host-only: (elements per batch, threads per workgroup, LDS bytes) of the
    fused path's trace (FR_K_TRACE) or fused (FR_K_FUSED) kernel."""
    out = (ctypes.c_int * 3)()
    _check(lib().fr_launch_shape(p, precision, kernel, out))
    return tuple(out)


def fr_plan_operators(p):
    """Host-only: dict of the plan's double-precision 1D operators."""
    m = p + 1
    out = np.zeros(m * (6 + 2 * m))
    _check(lib().fr_plan_operators(p, out.ctypes.data_as(_dp)))
    o, r = 0, {}
    for name, size, shape in (("x", m, (m,)), ("w", m, (m,)), ("D", m * m, (m, m)),
                              ("lm", m, (m,)), ("lp", m, (m,)), ("gl", m, (m,)), ("gr", m, (m,)),
                              ("Dt", m * m, (m, m))):
        r[name] = out[o:o + size].reshape(shape)
        o += size
    return r


class LinearHex:
    """Owning wrapper around an fr_lhex handle: the ACM-HD residual on linear
    hexahedra given by their corners (the plan must stay open)."""

    def __init__(self, plan):
        self.plan = plan
        self.handle = lib().fr_lhex_create(plan.handle)
        if not self.handle:
            raise FrError(FR_EINVAL, lib().fr_last_error().decode())

    def residual(self, corners, U, R, stream=None):
        import torch
        n = self.plan.state_len
        ne = n // NV // (self.plan.p + 1) ** 3
        return _check(lib().fr_lhex_residual(self.handle, _dev(corners, torch.float64, ne * 24, "corners"),
                                             _dev(U, torch.float64, n, "U"), _dev(R, torch.float64, n, "R"),
                                             _stream(stream)))

    def close(self):
        if self.handle:
            lib().fr_lhex_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Acm:
    """Owning wrapper around an fr_acm handle (standard ACM with LDG; the plan
    must stay open).  state_len: values of a [ne][4][m^3] state."""

    def __init__(self, plan, beta=0.5, tau=0.1):
        self.plan = plan
        self.state_len = plan.state_len // NV * 4
        self.handle = fr_acm_create(plan.handle, beta, tau)

    def residual(self, U, R, stream=None):
        return fr_acm_residual(self.handle, U, R, self.state_len, stream)

    def gradient(self, U, Q, stream=None):
        return fr_acm_gradient(self.handle, U, Q, self.state_len, stream)

    def dual_step(self, U, Un, Unm1, dt, dtau, tol, max_iters, check_every=1, stream=None,
                  raise_on_error=True):
        return fr_acm_dual_step(self.handle, U, Un, Unm1, dt, dtau, tol, max_iters, self.state_len,
                                check_every, stream, raise_on_error)

    def close(self):
        if self.handle:
            fr_acm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pmg:
    """Owning wrapper around an fr_pmg handle (the plan must stay open)."""

    def __init__(self, plan, cycle=None, factor=1.75):
        self.plan = plan
        self.handle = fr_pmg_create(plan.handle, cycle, factor)

    def dual_step(self, U, Un, Unm1, dt, dtau, tol, max_cycles, stream=None, raise_on_error=True):
        return fr_pmg_dual_step(self.handle, U, Un, Unm1, dt, dtau, tol, max_cycles,
                                self.plan.state_len, stream, raise_on_error)

    def close(self):
        if self.handle:
            fr_pmg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owning wrapper around an fr_plan handle."""

    def __init__(self, p, n, zeta, nu, T, jac=None, precision=FR_F64, variant=FR_FUSED, block=0):
        self.p, self.n = p, tuple(n)
        self.handle = fr_plan_create(p, n[0], n[1], n[2], jac, zeta, (nu, T))
        fr_plan_set_int(self.handle, FR_OPT_PRECISION, precision)
        fr_plan_set_int(self.handle, FR_OPT_VARIANT, variant)
        if block:
            fr_plan_set_int(self.handle, FR_OPT_BLOCK, block)

    @property
    def state_len(self):
        return fr_state_len(self.handle)

    def set(self, key, value):
        fr_plan_set_int(self.handle, key, value)

    def close(self):
        if self.handle:
            fr_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
