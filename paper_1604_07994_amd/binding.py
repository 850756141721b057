"""Thin ctypes binding of libiss.so (include/iss.h).

Argument marshalling only: every computation runs in the HIP library.  Torch
tensors provide device memory and the current HIP stream.  If the library
is missing this module raises; there is no fallback path.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libiss.so")

FORMS = {"gradient": 0, "strain": 1, "interface": 2}
BLOCKS = {"velocity": 0, "full": 1}
OUTER = {"richardson": 0, "fgmres": 1}
COARSE_MU = {"centroid": 0, "average": 1}
PREC_F64, PREC_F32 = 0, 1
PREC_BF16 = 2            # vectors stored in BF16, arithmetic in FP32
PREC_F16 = 3             # vectors stored in FP16, arithmetic in FP32
PRECS = {"fp64": PREC_F64, "fp32": PREC_F32, "bf16": PREC_BF16, "fp16": PREC_F16}

_lib = None


class IssError(RuntimeError):
    pass


class Inclusion(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("phase", ctypes.c_int), ("a", ctypes.c_double * 6)]


class Options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("omega", ctypes.c_double),
                ("stab_beta", ctypes.c_double), ("outer", ctypes.c_int), ("restart", ctypes.c_int),
                ("coarse_mu", ctypes.c_int), ("coarse_form", ctypes.c_int), ("nu_inc", ctypes.c_int),
                ("mid_form", ctypes.c_int), ("merge_max_n", ctypes.c_int), ("spec_wide_min", ctypes.c_int),
                ("cycles", ctypes.c_int), ("f16_rms", ctypes.c_double), ("coarse_rhs_mod", ctypes.c_int),
                ("bc", ctypes.c_int), ("split_align", ctypes.c_int), ("coarse_solver", ctypes.c_int),
                ("minres_iters", ctypes.c_int), ("minres_cg", ctypes.c_int)]

BCS = {"noslip": 0, "freeslip": 1}
COARSE_SOLVERS = {"direct": 0, "minres": 1}


# iss_launch_kind: smoother kernel shapes counted by iss_launch_counts
LAUNCH_KINDS = ["vel_rhs", "gs_vel_bulk", "gs_vel_special", "gs_vel_merged", "p_rhs_grouped",
                "p_rhs_merged", "gs_p_bulk", "gs_p_special", "gs_p_special_wide", "gs_p_merged",
                "apply_bulk", "apply_tiled"]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("history_len", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)),
                ("net_accepted", ctypes.c_int), ("net_rejected", ctypes.c_int)]


EXPORTS = ["iss_default_options", "iss_problem_create", "iss_problem_destroy", "iss_num_vertices",
           "iss_vertex_class", "iss_rhs_buoyancy", "iss_rhs_nodal_force", "iss_num_elements", "iss_p1p0_apply",
           "iss_p1p0_flux", "iss_apply", "iss_residual", "iss_smooth",
           "iss_restrict", "iss_prolong_add", "iss_coarse_solve", "iss_vcycle", "iss_solve",
           "iss_dot", "iss_last_error", "iss_net_create", "iss_net_destroy", "iss_net_info",
           "iss_net_band", "iss_net_set_weights", "iss_net_features", "iss_net_forward",
           "iss_net_targets", "iss_net_backward", "iss_adam_step", "iss_problem_set_net",
           "iss_net_correction", "iss_net_output_grad", "iss_smooth_timed", "iss_launch_counts",
           "iss_smooth_noalloc", "iss_asymptotic_rate", "iss_net_save_input", "iss_net_load_input",
           "iss_axpby", "iss_problem_create_elems", "iss_workspace_bytes", "iss_bind_workspace"]


def lib():
    """Load libiss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise IssError("libiss.so not built: run python -m paper_1604_07994_amd.build")
    # torch ships its own HIP runtime (same soname libamdhip64.so.7); load it
    # first so that libiss binds to that one runtime and torch's device
    # memory and stream handles are valid inside the library.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, cint, cdbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.iss_last_error.restype = ctypes.c_char_p
    L.iss_default_options.argtypes = [ctypes.POINTER(Options)]
    L.iss_problem_create.argtypes = [cint, cint, cint, cint, ctypes.POINTER(Inclusion), cint,
                                     ctypes.POINTER(cdbl), cint, ctypes.POINTER(Options),
                                     ctypes.POINTER(vp)]
    L.iss_problem_destroy.argtypes = [vp]
    L.iss_problem_destroy.restype = None
    L.iss_num_vertices.argtypes = [vp, cint, ctypes.POINTER(i64)]
    L.iss_vertex_class.argtypes = [vp, cint, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.iss_rhs_buoyancy.argtypes = [vp, cint, ctypes.POINTER(cint), cint, cdbl, vp, vp]
    L.iss_rhs_nodal_force.argtypes = [vp, cint, vp, vp, vp]
    L.iss_num_elements.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.iss_p1p0_apply.argtypes = [vp, cint, cdbl, vp, vp, vp]
    L.iss_p1p0_flux.argtypes = [vp, cdbl, vp, vp, vp]
    L.iss_apply.argtypes = [vp, cint, cint, cint, cint, vp, vp, vp]
    L.iss_residual.argtypes = [vp, cint, cint, cint, vp, vp, vp, ctypes.POINTER(cdbl), vp]
    L.iss_smooth.argtypes = [vp, cint, cint, cint, cint, vp, vp, vp]
    L.iss_smooth_noalloc.argtypes = [vp, cint, cint, cint, cint, vp, vp, vp]
    L.iss_smooth_timed.argtypes = [vp, cint, cint, cint, cint, vp, vp, vp, ctypes.POINTER(cdbl)]
    L.iss_restrict.argtypes = [vp, cint, cint, vp, vp, vp]
    L.iss_prolong_add.argtypes = [vp, cint, cint, vp, vp, vp]
    L.iss_coarse_solve.argtypes = [vp, cint, vp, vp, vp]
    L.iss_vcycle.argtypes = [vp, cint, cint, vp, vp, vp]
    L.iss_solve.argtypes = [vp, cint, cint, cdbl, cint, vp, vp, ctypes.POINTER(SolveInfo), vp]
    L.iss_dot.argtypes = [vp, vp, vp, i64, ctypes.POINTER(cdbl), vp]
    L.iss_net_create.argtypes = [vp, ctypes.POINTER(vp)]
    L.iss_net_destroy.argtypes = [vp]
    L.iss_net_destroy.restype = None
    L.iss_net_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.iss_net_band.argtypes = [vp, vp]
    L.iss_net_set_weights.argtypes = [vp, vp, vp]
    L.iss_net_features.argtypes = [vp, vp, ctypes.POINTER(cdbl), vp]
    L.iss_net_forward.argtypes = [vp, vp, vp]
    L.iss_net_targets.argtypes = [vp, vp, vp, vp]
    L.iss_net_backward.argtypes = [vp, vp, vp, ctypes.POINTER(cdbl), vp]
    L.iss_adam_step.argtypes = [i64, vp, vp, vp, vp, ctypes.c_float, cint, vp]
    L.iss_problem_set_net.argtypes = [vp, vp]
    L.iss_net_correction.argtypes = [vp, vp, vp]
    L.iss_net_output_grad.argtypes = [vp, vp, cdbl, vp]
    L.iss_launch_counts.argtypes = [vp, ctypes.POINTER(i64), cint, cint]
    L.iss_asymptotic_rate.argtypes = [vp, cint, cint, vp, ctypes.POINTER(cdbl), vp]
    L.iss_net_save_input.argtypes = [vp, vp, vp]
    L.iss_net_load_input.argtypes = [vp, vp, vp]
    L.iss_axpby.argtypes = [cdbl, vp, cdbl, vp, i64, vp]
    L.iss_problem_create_elems.argtypes = [cint, cint, cint, cint, vp, ctypes.POINTER(cdbl), cint,
                                           ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.iss_workspace_bytes.argtypes = [vp, cint, ctypes.POINTER(ctypes.c_size_t)]
    L.iss_bind_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise IssError("libiss error %d: %s" % (rc, lib().iss_last_error().decode()))


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prec(t):
    import torch
    if t.dtype == torch.float64:
        return PREC_F64
    if t.dtype == torch.float32:
        return PREC_F32
    if t.dtype == torch.bfloat16:
        return PREC_BF16
    if t.dtype == torch.float16:
        return PREC_F16
    raise ValueError("vectors must be float64, float32, bfloat16 or float16")


def inclusions_to_c(inclusions):
    arr = (Inclusion * max(1, len(inclusions)))()
    for i, inc in enumerate(inclusions):
        if inc["kind"] == "sphere":
            c = list(inc["center"]) + [0.0] * (3 - len(inc["center"]))
            arr[i].kind, arr[i].phase = 0, int(inc["phase"])
            arr[i].a[:] = [c[0], c[1], c[2], inc["radius"], 0.0, 0.0]
        elif inc["kind"] == "halfspace":
            arr[i].kind, arr[i].phase = 1, int(inc["phase"])
            arr[i].a[:] = [float(inc["axis"]), inc["threshold"], 0.0, 0.0, 0.0, 0.0]
        elif inc["kind"] == "box":
            lo = list(inc["lo"]) + [0.0] * (3 - len(inc["lo"]))
            hi = list(inc["hi"]) + [0.0] * (3 - len(inc["hi"]))
            arr[i].kind, arr[i].phase = 2, int(inc["phase"])
            arr[i].a[:] = [lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]]
        else:
            raise ValueError(inc["kind"])
    return arr


class Problem:
    """A refined Kuhn-lattice Stokes problem owned by libiss."""

    def __init__(self, dim, macro, levels, coarse, inclusions, mu, nu1=3, nu2=3, omega=0.3,
                 stab_beta=1.0 / 12.0, outer="richardson", restart=40, coarse_mu="average",
                 coarse_form=None, nu_inc=0, mid_form=None, merge_max_n=64, spec_wide_min=65536, cycles=1,
                 f16_rms=1.0 / 1024.0, coarse_rhs_mod=False, elem_phase=None, bc="noslip", split_align=0,
                 coarse_solver="direct", minres_iters=30, minres_cg=5):
        L = lib()
        self.dim, self.macro, self.levels, self.coarse = dim, macro, levels, coarse
        opt = Options(nu1, nu2, omega, stab_beta, OUTER[outer], restart, COARSE_MU[coarse_mu],
                      -1 if coarse_form is None else FORMS[coarse_form], nu_inc,
                      -1 if mid_form is None else FORMS[mid_form], merge_max_n, spec_wide_min, cycles, f16_rms,
                      int(bool(coarse_rhs_mod)), BCS[bc], split_align, COARSE_SOLVERS[coarse_solver],
                      minres_iters, minres_cg)
        self.bc = bc
        mu_arr = (ctypes.c_double * len(mu))(*mu)
        h = ctypes.c_void_p()
        self._h = None
        if elem_phase is not None:
            ph = np.ascontiguousarray(elem_phase, dtype=np.uint8)
            _check(L.iss_problem_create_elems(dim, macro, levels, coarse, ph.ctypes.data_as(ctypes.c_void_p),
                                              mu_arr, len(mu), ctypes.byref(opt), ctypes.byref(h)))
        else:
            incs = inclusions_to_c(inclusions)
            _check(L.iss_problem_create(dim, macro, levels, coarse, incs, len(inclusions), mu_arr,
                                        len(mu), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, w, **kw):
        if "bc" in w:
            kw.setdefault("bc", w["bc"])
        return cls(w["dim"], w["macro"], w["levels"], w["coarse"], w["inclusions"], w["mu"], **kw)

    @classmethod
    def from_elems(cls, dim, macro, levels, coarse, elem_phase, mu, **kw):
        """Problem with one phase per finest-level element (library element
        order, see iss_problem_create_elems)."""
        kw.setdefault("coarse_mu", "average")
        return cls(dim, macro, levels, coarse, [], mu, elem_phase=elem_phase, **kw)

    def workspace_bytes(self, prec="fp64"):
        out = ctypes.c_size_t()
        _check(lib().iss_workspace_bytes(self._h, PRECS[prec],
                                         ctypes.byref(out)))
        return out.value

    def bind_workspace(self, buf):
        """Take every work buffer from the caller's device tensor buf (kept
        referenced here until close)."""
        _check(lib().iss_bind_workspace(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))
        self._workspace = buf

    def close(self):
        if getattr(self, "_h", None):
            lib().iss_problem_destroy(self._h)
            self._h = None
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- sizes ------------------------------------------------------------
    def num_vertices(self, level=None):
        level = self.levels if level is None else level
        n = ctypes.c_int64()
        _check(lib().iss_num_vertices(self._h, level, ctypes.byref(n)))
        return n.value

    def vector_size(self, level=None):
        return (self.dim + 1) * self.num_vertices(level)

    def vertex_class(self, level=None):
        level = self.levels if level is None else level
        cls = np.zeros(self.num_vertices(level), dtype=np.uint8)
        ni, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().iss_vertex_class(self._h, level, cls.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(ni), ctypes.byref(nb)))
        return cls, ni.value, nb.value

    def _vec(self, t, level, dtype=None):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
            raise ValueError("expected a contiguous CUDA (HIP) tensor")
        if t.numel() != self.vector_size(level):
            raise ValueError("vector has %d entries, level needs %d" % (t.numel(), self.vector_size(level)))
        if dtype is not None and t.dtype != dtype:
            raise ValueError("expected dtype %s" % dtype)
        return ctypes.c_void_p(t.data_ptr())

    # -- operators --------------------------------------------------------
    def rhs_buoyancy(self, b, phases, rho=1.0, level=None):
        import torch
        level = self.levels if level is None else level
        ph = (ctypes.c_int * max(1, len(phases)))(*phases)
        _check(lib().iss_rhs_buoyancy(self._h, level, ph, len(phases), rho,
                                      self._vec(b, level, torch.float64), _stream()))
        return b

    def rhs_nodal_force(self, f, b, level=None):
        """b = (M f_1 | .. | M f_d | 0) from nodal force values f (FP64
        device tensor of d N entries)."""
        import torch
        level = self.levels if level is None else level
        if not (isinstance(f, torch.Tensor) and f.is_cuda and f.is_contiguous() and f.dtype == torch.float64
                and f.numel() == self.dim * self.num_vertices(level)):
            raise ValueError("f must be a contiguous FP64 CUDA tensor of dim * N entries")
        _check(lib().iss_rhs_nodal_force(self._h, level, ctypes.c_void_p(f.data_ptr()),
                                         self._vec(b, level, torch.float64), _stream()))
        return b

    # -- stabilised P1-P0 (finest level) ------------------------------------
    def num_elements(self):
        ne = ctypes.c_int64()
        _check(lib().iss_num_elements(self._h, ctypes.byref(ne)))
        return ne.value

    def _p0vec(self, t, size):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dtype == torch.float64):
            raise ValueError("expected a contiguous FP64 CUDA tensor")
        if t.numel() != size:
            raise ValueError("vector has %d entries, needs %d" % (t.numel(), size))
        return ctypes.c_void_p(t.data_ptr())

    def p1p0_size(self):
        return self.dim * self.num_vertices() + self.num_elements()

    def p1p0_apply(self, form, x, y, gamma=1.0):
        n = self.p1p0_size()
        _check(lib().iss_p1p0_apply(self._h, FORMS[form], gamma, self._p0vec(x, n), self._p0vec(y, n), _stream()))
        return y

    def p1p0_flux(self, x, flux, gamma=1.0):
        _check(lib().iss_p1p0_flux(self._h, gamma, self._p0vec(x, self.p1p0_size()),
                                   self._p0vec(flux, (self.dim + 1) * self.num_elements()), _stream()))
        return flux

    def apply(self, form, x, y, level=None, block="full"):
        level = self.levels if level is None else level
        if x.dtype != y.dtype:
            raise ValueError("x and y must share a dtype")
        _check(lib().iss_apply(self._h, FORMS[form], BLOCKS[block], level, _prec(x),
                               self._vec(x, level), self._vec(y, level), _stream()))
        return y

    def residual(self, form, x, b, r, level=None, norms=False):
        level = self.levels if level is None else level
        out = (ctypes.c_double * (self.dim + 2))() if norms else None
        _check(lib().iss_residual(self._h, FORMS[form], level, _prec(x), self._vec(x, level),
                                  self._vec(b, level), self._vec(r, level), out, _stream()))
        return list(out) if norms else r

    def smooth(self, form, x, b, nsteps=1, level=None):
        level = self.levels if level is None else level
        _check(lib().iss_smooth(self._h, FORMS[form], level, _prec(x), nsteps,
                                self._vec(x, level), self._vec(b, level), _stream()))
        return x

    def smooth_noalloc(self, form, x, b, nsteps=1, level=None):
        """iss_smooth_noalloc: the same steps as smooth() with the library's
        static per-GPU scratch (no allocation; levels up to its size)."""
        level = self.levels if level is None else level
        _check(lib().iss_smooth_noalloc(self._h, FORMS[form], level, _prec(x), nsteps,
                                        self._vec(x, level), self._vec(b, level), _stream()))
        return x

    def smooth_timed(self, form, x, b, nsteps=1, level=None):
        """iss_smooth with HIP-event timing: returns (average bulk velocity
        colour-phase launch, average step) in milliseconds."""
        level = self.levels if level is None else level
        ms = (ctypes.c_double * 2)()
        _check(lib().iss_smooth_timed(self._h, FORMS[form], level, _prec(x), nsteps,
                                      self._vec(x, level), self._vec(b, level), _stream(), ms))
        return ms[0], ms[1]

    def restrict(self, rf, rc, level=None):
        level = self.levels if level is None else level
        _check(lib().iss_restrict(self._h, level, _prec(rf), self._vec(rf, level),
                                  self._vec(rc, level - 1), _stream()))
        return rc

    def prolong_add(self, ec, xf, level=None):
        level = self.levels if level is None else level
        _check(lib().iss_prolong_add(self._h, level, _prec(xf), self._vec(ec, level - 1),
                                     self._vec(xf, level), _stream()))
        return xf

    def coarse_solve(self, form, b, x):
        import torch
        _check(lib().iss_coarse_solve(self._h, FORMS[form], self._vec(b, self.coarse, torch.float64),
                                      self._vec(x, self.coarse, torch.float64), _stream()))
        return x

    def vcycle(self, form, x, b):
        _check(lib().iss_vcycle(self._h, FORMS[form], _prec(x), self._vec(x, self.levels),
                                self._vec(b, self.levels), _stream()))
        return x

    def solve(self, form, x, b, prec="fp64", rtol=1e-8, maxit=200, raise_on_fail=True):
        import torch
        hist = (ctypes.c_double * (maxit + 1))()
        info = SolveInfo(0, 0.0, 0.0, 0, ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), 0, 0)
        rc = lib().iss_solve(self._h, FORMS[form], PRECS[prec], rtol,
                             maxit, self._vec(x, self.levels, torch.float64),
                             self._vec(b, self.levels, torch.float64), ctypes.byref(info), _stream())
        if rc != 0 and raise_on_fail:
            _check(rc)
        return {"status": rc, "iterations": info.iterations, "relres": info.relres,
                "seconds": info.seconds, "history": [hist[i] for i in range(info.history_len)],
                "net_accepted": info.net_accepted, "net_rejected": info.net_rejected}

    def asymptotic_rate(self, form, x, iters=200):
        """Residual reduction per stationary V-cycle of the homogeneous
        problem, rescaled every cycle (iss_asymptotic_rate); x is the start
        (overwritten).  Returns the list of per-cycle rates."""
        import torch
        rates = (ctypes.c_double * iters)()
        _check(lib().iss_asymptotic_rate(self._h, FORMS[form], iters, self._vec(x, self.levels, torch.float64),
                                         rates, _stream()))
        return list(rates)

    def launch_counts(self, reset=False):
        """Smoother kernel launches per kernel shape since creation (or the
        last reset), as a dict keyed by LAUNCH_KINDS."""
        c = (ctypes.c_int64 * len(LAUNCH_KINDS))()
        _check(lib().iss_launch_counts(self._h, c, len(LAUNCH_KINDS), int(reset)))
        return dict(zip(LAUNCH_KINDS, list(c)))

    def axpby(self, a, x, b, y):
        """y = a x + b y (FP64 device vectors of equal length)."""
        import torch
        for t in (x, y):
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64):
                raise ValueError("axpby needs contiguous float64 CUDA tensors")
        if x.numel() != y.numel():
            raise ValueError("size mismatch")
        _check(lib().iss_axpby(float(a), _ptr(x), float(b), _ptr(y), y.numel(), _stream()))
        return y

    def dot(self, a, b):
        import torch
        for t in (a, b):
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64):
                raise ValueError("dot needs contiguous float64 CUDA tensors")
        if a.numel() != b.numel():
            raise ValueError("size mismatch")
        out = ctypes.c_double()
        _check(lib().iss_dot(self._h, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                             a.numel(), ctypes.byref(out), _stream()))
        return out.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class BandNet:
    """The learned band correction of a (3D) Problem; weights are FP32 torch
    tensors on the device, flat [W1 | W2 | W3]."""

    def __init__(self, problem):
        h = ctypes.c_void_p()
        _check(lib().iss_net_create(problem._h, ctypes.byref(h)))
        self._h = h
        self.problem = problem
        m, npar = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().iss_net_info(h, ctypes.byref(m), ctypes.byref(npar)))
        self.band_size, self.num_params = m.value, npar.value

    def close(self):
        if getattr(self, "_h", None):
            lib().iss_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def band(self):
        out = np.zeros(self.band_size, dtype=np.int32)
        _check(lib().iss_net_band(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_weights(self, w):
        _check(lib().iss_net_set_weights(self._h, _ptr(w), _stream()))

    def features(self, r):
        sc = (ctypes.c_double * 2)()
        _check(lib().iss_net_features(self._h, _ptr(r), sc, _stream()))
        return sc[0], sc[1]

    def forward(self, y=None):
        _check(lib().iss_net_forward(self._h, _ptr(y) if y is not None else None, _stream()))
        return y

    def targets(self, e, t):
        _check(lib().iss_net_targets(self._h, _ptr(e), _ptr(t), _stream()))
        return t

    def backward(self, t, grad):
        """MSE against targets t, or (t None) the output gradient set by
        output_grad(); returns the MSE value or None."""
        loss = ctypes.c_double()
        _check(lib().iss_net_backward(self._h, _ptr(t) if t is not None else None, _ptr(grad),
                                      ctypes.byref(loss) if t is not None else None, _stream()))
        return loss.value if t is not None else None

    def save_input(self, dst):
        """Band rows of the current input (M x 8 BF16 bit patterns) into the
        int16 device tensor dst."""
        if dst.numel() != self.band_size * 8 or dst.element_size() != 2:
            raise ValueError("need a 2-byte tensor of band_size * 8 entries")
        _check(lib().iss_net_save_input(self._h, _ptr(dst), _stream()))
        return dst

    def load_input(self, src):
        if src.numel() != self.band_size * 8 or src.element_size() != 2:
            raise ValueError("need a 2-byte tensor of band_size * 8 entries")
        _check(lib().iss_net_load_input(self._h, _ptr(src), _stream()))

    def correction(self, c):
        _check(lib().iss_net_correction(self._h, _ptr(c), _stream()))
        return c

    def output_grad(self, g, factor=1.0):
        """dL/dc = factor * g."""
        _check(lib().iss_net_output_grad(self._h, _ptr(g), factor, _stream()))

    def attach(self, on=True):
        _check(lib().iss_problem_set_net(self.problem._h, self._h if on else None))


def adam_step(w, m, v, g, lr, step):
    _check(lib().iss_adam_step(w.numel(), _ptr(w), _ptr(m), _ptr(v), _ptr(g), lr, step, _stream()))
