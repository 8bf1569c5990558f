"""Taylor-Couette projection step on MI355X: Python binding of libtc.

This module only marshals arguments for the C ABI declared in
``include/tc.h`` (device pointers of torch tensors, the HIP stream, sizes);
every step of the computation runs in the library's HIP kernels.  Importing
it does not need a GPU; creating a :class:`Solver` needs the built library
(``python -m paper_1311_2481_amd.build``) and a GPU, and raises otherwise.

Spectral arrays are complex128 torch tensors on the GPU with shape
(fields, n_r, m_z, m_theta) (see ``include/tc.h`` for the layout).
"""
import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime that libtc.so then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK, TC_EINVAL, TC_ENOMEM, TC_ESINGULAR, TC_EHIP, TC_ENONFINITE = range(6)
STATUS_NAMES = {0: "TC_OK", 1: "TC_EINVAL", 2: "TC_ENOMEM", 3: "TC_ESINGULAR", 4: "TC_EHIP", 5: "TC_ENONFINITE"}
SOLVE_KINDS = {"P": 0, "Up": 1, "Um": 2, "Uz": 3, "Phi": 4}
PRECISIONS = {"fp64": 0, "fp32_bulk": 1}
FORMS = {"rot": 0, "conv": 1}
KERNELS = {"pc": 0, "curl": 1, "zinv": 2, "theta": 3, "zfwd": 4}


class TcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int32), ("m_theta", ctypes.c_int32), ("m_z", ctypes.c_int32),
                ("p_theta", ctypes.c_int32), ("p_z", ctypes.c_int32), ("k_theta", ctypes.c_double),
                ("k_z", ctypes.c_double), ("alpha", ctypes.c_double), ("n_s", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("form", ctypes.c_int32)]


_lib = None
EXPORTS = ["tc_init", "tc_destroy", "tc_last_error", "tc_radial_nodes", "tc_set_state", "tc_get_state",
           "tc_get_history", "tc_step", "tc_nonlinear", "tc_helmholtz_solve", "tc_helmholtz_solve_transposed",
           "tc_step_adjoint", "tc_perturbation_energy_gradient", "tc_adjoint_seed", "tc_adjoint_initial_history",
           "tc_control_velocity", "tc_control_gradient", "tc_control_ascent_update", "tc_get_diag", "tc_get_diag_noalloc", "tc_check_finite", "tc_set_timing", "tc_kernel_time", "tc_factor_backward_error",
           "tc_memory_bytes"]


def load_library(path=LIB_PATH):
    """Load libtc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1311_2481_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.tc_init.argtypes = [ctypes.POINTER(_Grid), dbl, dbl, dbl, dbl, vp, ctypes.POINTER(vp)]
    lib.tc_destroy.argtypes = [vp]
    lib.tc_last_error.argtypes = [vp]
    lib.tc_last_error.restype = ctypes.c_char_p
    lib.tc_radial_nodes.argtypes = [vp, ctypes.POINTER(dbl)]
    lib.tc_set_state.argtypes = [vp, vp, vp, vp]
    lib.tc_get_state.argtypes = [vp, vp, vp]
    lib.tc_get_history.argtypes = [vp, vp, vp]
    lib.tc_step.argtypes = [vp, i32]
    lib.tc_nonlinear.argtypes = [vp, vp, vp]
    lib.tc_helmholtz_solve.argtypes = [vp, i32, vp, vp]
    lib.tc_helmholtz_solve_transposed.argtypes = [vp, i32, vp, vp]
    lib.tc_step_adjoint.argtypes = [vp, vp, vp, vp]
    lib.tc_perturbation_energy_gradient.argtypes = [vp, vp, vp]
    lib.tc_adjoint_seed.argtypes = [vp, vp, dbl, vp]
    lib.tc_adjoint_initial_history.argtypes = [vp, vp, vp, vp]
    lib.tc_control_velocity.argtypes = [vp, vp, vp]
    lib.tc_control_gradient.argtypes = [vp, vp, vp]
    lib.tc_control_ascent_update.argtypes = [vp, vp, vp, vp, dbl, dbl, vp, ctypes.POINTER(dbl)]
    lib.tc_get_diag.argtypes = [vp, ctypes.POINTER(dbl)]
    lib.tc_get_diag_noalloc.argtypes = [vp, ctypes.POINTER(dbl)]
    lib.tc_check_finite.argtypes = [vp]
    lib.tc_set_timing.argtypes = [vp, i32]
    lib.tc_kernel_time.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i32)]
    lib.tc_memory_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.tc_factor_backward_error.argtypes = [vp, ctypes.POINTER(dbl)]
    for name in EXPORTS:
        if name != "tc_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class Solver:
    """One Taylor-Couette configuration on one GPU (wraps a tc_ctx)."""

    def __init__(self, n_r, m_theta, m_z, eta, Re_i, Re_o, dt, k_theta=1.0, k_z=1.0, alpha=0.0,
                 precision="fp64", p_theta=0, p_z=0, device="cuda", form="rot", stream=None):
        """stream: the torch.cuda.Stream the context enqueues its work on
        (default: the current stream at construction)."""
        self.lib = load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (torch.cuda is not available)")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.n_r, self.m_theta, self.m_z = int(n_r), int(m_theta), int(m_z)
        self.eta, self.Re_i, self.Re_o, self.dt = float(eta), float(Re_i), float(Re_o), float(dt)
        self.k_theta, self.k_z, self.alpha = float(k_theta), float(k_z), float(alpha)
        self.precision = precision
        self.form = form
        self.p_theta, self.p_z = int(p_theta), int(p_z)
        g = _Grid(self.n_r, self.m_theta, self.m_z, int(p_theta), int(p_z), self.k_theta, self.k_z, self.alpha, 9,
                  PRECISIONS[precision], FORMS[form])
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
            ctx = ctypes.c_void_p()
            st = self.lib.tc_init(ctypes.byref(g), self.eta, self.Re_i, self.Re_o, self.dt,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if st != TC_OK:
            raise TcError(st, self.lib.tc_last_error(None).decode())
        self.ctx = ctx
        self.shape = (self.n_r, self.m_z, self.m_theta)

    # -------------------------------------------------------------- helpers
    def _check(self, st):
        if st != TC_OK:
            raise TcError(st, self.lib.tc_last_error(self.ctx).decode())

    def _arr(self, t, nfields, name):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.complex128 or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex128 tensor on {self.device}")
        if tuple(t.shape) != (nfields,) + self.shape and not (nfields == 1 and tuple(t.shape) == self.shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {(nfields,) + self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self, nfields=3):
        shape = (nfields,) + self.shape if nfields != 1 else self.shape
        return torch.empty(shape, dtype=torch.complex128, device=self.device)

    def zeros(self, nfields=3):
        shape = (nfields,) + self.shape if nfields != 1 else self.shape
        return torch.zeros(shape, dtype=torch.complex128, device=self.device)

    # -------------------------------------------------------------- API
    def radial_nodes(self):
        r = np.empty(self.n_r)
        self._check(self.lib.tc_radial_nodes(self.ctx, r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return r

    def set_state(self, u, u_prev=None, N_prev=None):
        self._check(self.lib.tc_set_state(self.ctx, self._arr(u, 3, "u"), self._arr(u_prev, 3, "u_prev"),
                                          self._arr(N_prev, 3, "N_prev")))

    def get_state(self, with_pressure=True, out=None):
        u = self.empty(3) if out is None else out
        p = self.empty(1) if with_pressure else None
        self._check(self.lib.tc_get_state(self.ctx, self._arr(u, 3, "u"), self._arr(p, 1, "p")))
        return (u, p) if with_pressure else u

    def get_history(self):
        up, Np = self.empty(3), self.empty(3)
        self._check(self.lib.tc_get_history(self.ctx, self._arr(up, 3, "u_prev"), self._arr(Np, 3, "N_prev")))
        return up, Np

    def step(self, nsteps=1):
        self._check(self.lib.tc_step(self.ctx, int(nsteps)))

    def nonlinear(self, u, out=None):
        N = self.empty(3) if out is None else out
        self._check(self.lib.tc_nonlinear(self.ctx, self._arr(u, 3, "u"), self._arr(N, 3, "N")))
        return N

    def solve(self, kind, rhs, out=None, transposed=False):
        x = self.empty(1) if out is None else out
        fn = self.lib.tc_helmholtz_solve_transposed if transposed else self.lib.tc_helmholtz_solve
        self._check(fn(self.ctx, SOLVE_KINDS[kind], self._arr(rhs, 1, "rhs"), self._arr(x, 1, "x")))
        return x

    def step_adjoint(self, fwd, adj_in, adj_out=None):
        out = self.empty(9) if adj_out is None else adj_out
        self._check(self.lib.tc_step_adjoint(self.ctx, self._arr(fwd, 6, "fwd"), self._arr(adj_in, 9, "adj_in"),
                                             self._arr(out, 9, "adj_out")))
        return out

    def energy_gradient(self, u, out=None):
        g = self.empty(3) if out is None else out
        self._check(self.lib.tc_perturbation_energy_gradient(self.ctx, self._arr(u, 3, "u"), self._arr(g, 3, "g")))
        return g

    def adjoint_seed(self, uT, scale=1.0, out=None):
        g = self.empty(3) if out is None else out
        self._check(self.lib.tc_adjoint_seed(self.ctx, self._arr(uT, 3, "uT"), float(scale), self._arr(g, 3, "g")))
        return g

    def adjoint_initial_history(self, u0, adj_in, out=None):
        g = self.empty(3) if out is None else out
        self._check(self.lib.tc_adjoint_initial_history(self.ctx, self._arr(u0, 3, "u0"),
                                                        self._arr(adj_in, 9, "adj_in"), self._arr(g, 3, "g")))
        return g

    # -------------------------------------------------------------- optimal-perturbation control
    @property
    def control_shape(self):
        return (3, 4, self.m_z, self.m_theta)

    def _ctl(self, t, name):
        if t is None:
            return None
        if (not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or t.device != self.device
                or not t.is_contiguous() or tuple(t.shape) != self.control_shape):
            raise ValueError(f"{name} must be a contiguous complex128 tensor of shape {self.control_shape} "
                             f"on {self.device}")
        return ctypes.c_void_p(t.data_ptr())

    def control_zeros(self):
        return torch.zeros(self.control_shape, dtype=torch.complex128, device=self.device)

    def control_velocity(self, a, out=None):
        u = self.empty(3) if out is None else out
        self._check(self.lib.tc_control_velocity(self.ctx, self._ctl(a, "a"), self._arr(u, 3, "u")))
        return u

    def control_gradient(self, g, out=None):
        ga = self.control_zeros() if out is None else out
        self._check(self.lib.tc_control_gradient(self.ctx, self._arr(g, 3, "g"), self._ctl(ga, "ga")))
        return ga

    def control_ascent_update(self, a, gJ, gE, tau, E0, out=None):
        res = self.control_zeros() if out is None else out
        st = np.zeros(5)
        self._check(self.lib.tc_control_ascent_update(self.ctx, self._ctl(a, "a"), self._ctl(gJ, "gJ"),
                                                      self._ctl(gE, "gE"), float(tau), float(E0),
                                                      self._ctl(res, "a_out"),
                                                      st.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return res, dict(beta=st[0], energy_before=st[1], scale=st[2], step_norm=st[3], control_norm=st[4])

    def factor_backward_error(self):
        err = ctypes.c_double()
        self._check(self.lib.tc_factor_backward_error(self.ctx, ctypes.byref(err)))
        return err.value

    def diag(self):
        out = np.zeros(8)
        self._check(self.lib.tc_get_diag(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return dict(energy=out[0], perturbation_energy=out[1], max_div=out[2], slip=out[3], cfl=out[4],
                    steps=int(out[5]), nu_inner=out[6], nu_outer=out[7])

    def check_finite(self):
        st = self.lib.tc_check_finite(self.ctx)
        if st == TC_ENONFINITE:
            return False
        self._check(st)
        return True

    def set_timing(self, enable=True):
        self._check(self.lib.tc_set_timing(self.ctx, 1 if enable else 0))

    def kernel_time(self, which):
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        self._check(self.lib.tc_kernel_time(self.ctx, KERNELS[which], ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def memory_bytes(self):
        b = ctypes.c_uint64()
        self._check(self.lib.tc_memory_bytes(self.ctx, ctypes.byref(b)))
        return b.value

    def twin(self, stream):
        """A second context with the same grid, parameters and factors
        (recomputed by its own tc_init), enqueuing on ``stream``."""
        return Solver(self.n_r, self.m_theta, self.m_z, self.eta, self.Re_i, self.Re_o, self.dt,
                      k_theta=self.k_theta, k_z=self.k_z, alpha=self.alpha, precision=self.precision,
                      p_theta=self.p_theta, p_z=self.p_z, device=self.device, form=self.form, stream=stream)

    def close(self):
        tw = getattr(self, "_twin", None)
        if tw is not None:
            tw.close()
            self._twin = None
        if getattr(self, "ctx", None):
            self.lib.tc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
