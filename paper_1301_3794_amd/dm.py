"""ctypes binding of the C ABI in ``include/dm.h``.

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device buffers are torch tensors (PyTorch supplies device memory and
streams); the library is loaded from this package directory and its absence
is an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdm.so")

DM_OK = 0
DM_NOT_CONVERGED = 1
DM_EINVAL, DM_ENOMEM, DM_EHIP, DM_ESINGULAR, DM_EBREAKDOWN, DM_ENAN, DM_ENODEVICE = range(-1, -8, -1)

GEOM_BOX, GEOM_ELLIPSOID, GEOM_ELLIPTIC_BOR, GEOM_USER, GEOM_LEVELSET = 0, 1, 2, 3, 4
BC_PEC, BC_PMC = 0, 1
APPLY_M, APPLY_K, APPLY_A, APPLY_DA, APPLY_DT, APPLY_S = range(6)
SOLVE_PCG64, SOLVE_FGMRES_MG64, SOLVE_FGMRES_MG32, SOLVE_FGMRES_MG32_LEARNED = range(4)
NET_WEIGHTS = 12528
NET_LOSS_ERROR, NET_LOSS_RESIDUAL = 0, 1

EXPORTS = (
    "dm_default_options", "dm_build_operator", "dm_destroy", "dm_set_shift",
    "dm_compute_fractions", "dm_field_layout", "dm_get_fractions", "dm_apply",
    "dm_residual", "dm_smooth", "dm_restrict", "dm_prolong_add", "dm_vcycle", "dm_vcycle_block",
    "dm_project", "dm_project_block", "dm_solve", "dm_solve_block", "dm_default_eig_options", "dm_eigs", "dm_strerror",
    "dm_last_error_message", "dm_time_kernel", "dm_time_block_kernel", "dm_net_create", "dm_net_destroy",
    "dm_net_get_weights", "dm_net_set_weights", "dm_net_attach", "dm_net_apply",
    "dm_net_loss_grad", "dm_net_make_pair", "dm_net_train", "dm_batch_create", "dm_batch_destroy",
    "dm_batch_member", "dm_batch_info", "dm_batch_vcycle", "dm_batch_time_vcycle", "dm_batch_eigs",
)
(KERNEL_APPLY, KERNEL_RESIDUAL, KERNEL_SMOOTH, KERNEL_SWEEP, KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_VCYCLE,
 KERNEL_NET) = range(8)


class DMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Geometry(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("center", ctypes.c_double * 3),
        ("semi_axes", ctypes.c_double * 3),
        ("axis_xy", ctypes.c_double * 2),
        ("z_start", ctypes.c_double),
        ("n_cells", ctypes.c_int),
        ("r_equator", ctypes.c_double),
        ("r_iris", ctypes.c_double),
        ("cell_length", ctypes.c_double),
        ("tube_length", ctypes.c_double),
        ("user_fractions_host", ctypes.POINTER(ctypes.c_double)),
        ("bc_lo", ctypes.c_int * 3),
        ("a_min", ctypes.c_double),
        ("levelset_host", ctypes.POINTER(ctypes.c_double)),
        ("levelset_refine", ctypes.c_int),
    ]


class Options(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("fgmres_restart", ctypes.c_int), ("verbose", ctypes.c_int),
                ("cut_wave_split", ctypes.c_int), ("learned_patience", ctypes.c_int),
                ("grad_div_volume", ctypes.c_int), ("tilde_transfers", ctypes.c_int),
                ("krylov_basis_f32", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("learned_accepted", ctypes.c_int), ("learned_rejected", ctypes.c_int)]


class EigOptions(ctypes.Structure):
    _fields_ = [("solve_mode", ctypes.c_int), ("inner_rtol", ctypes.c_double),
                ("proj_rtol", ctypes.c_double), ("block", ctypes.c_int),
                ("max_basis", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("verbose", ctypes.c_int), ("start_dev", ctypes.c_void_p)]


class BatchStats(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("threads_per_block", ctypes.c_int),
                ("tuned_ms", ctypes.c_double * 3), ("launches_per_vcycle", ctypes.c_int),
                ("cells", ctypes.c_int64), ("active_faces", ctypes.c_int64)]


class EigInfo(ctypes.Structure):
    _fields_ = [("n_converged", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("restarts", ctypes.c_int), ("inner_iterations", ctypes.c_int),
                ("projection_iterations", ctypes.c_int), ("max_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]


_lib = None


def lib():
    """The loaded ``libdm.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1301_3794_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    L.dm_default_options.argtypes = [ctypes.POINTER(Options)]
    L.dm_default_options.restype = None
    L.dm_build_operator.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(ctypes.c_int), d, d,
                                    ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.dm_destroy.argtypes = [vp]
    L.dm_destroy.restype = None
    L.dm_set_shift.argtypes = [vp, d]
    L.dm_compute_fractions.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(ctypes.c_int), d, dp]
    L.dm_field_layout.argtypes = [vp, i, ctypes.POINTER(i64)]
    L.dm_get_fractions.argtypes = [vp, i, dp]
    L.dm_apply.argtypes = [vp, i, i, i, vp, vp, vp]
    L.dm_residual.argtypes = [vp, i, i, vp, vp, vp, vp]
    L.dm_smooth.argtypes = [vp, i, i, i, i, vp, vp, vp]
    L.dm_restrict.argtypes = [vp, i, i, vp, vp, vp]
    L.dm_prolong_add.argtypes = [vp, i, i, vp, vp, vp]
    L.dm_vcycle.argtypes = [vp, i, vp, vp, vp]
    L.dm_vcycle_block.argtypes = [vp, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.dm_project.argtypes = [vp, vp, vp, d, vp]
    L.dm_solve.argtypes = [vp, i, vp, vp, d, i, ctypes.POINTER(SolveInfo), vp]
    L.dm_project_block.argtypes = [vp, i, ctypes.POINTER(vp), ctypes.POINTER(vp), d, vp]
    L.dm_solve_block.argtypes = [vp, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp), d, i,
                                 ctypes.POINTER(SolveInfo), vp]
    L.dm_default_eig_options.argtypes = [ctypes.POINTER(EigOptions)]
    L.dm_default_eig_options.restype = None
    L.dm_eigs.argtypes = [vp, i, d, d, ctypes.c_uint64, ctypes.POINTER(EigOptions), dp, vp, dp,
                          ctypes.POINTER(EigInfo), vp]
    L.dm_time_kernel.argtypes = [vp, i, i, i, i, dp]
    L.dm_sample_e.argtypes = [vp, vp, d, i, dp, dp, vp]
    L.dm_time_block_kernel.argtypes = [vp, i, i, i, i, i, ctypes.POINTER(d)]
    L.dm_strerror.argtypes = [i]
    L.dm_strerror.restype = ctypes.c_char_p
    L.dm_last_error_message.argtypes = []
    L.dm_last_error_message.restype = ctypes.c_char_p
    fp = ctypes.POINTER(ctypes.c_float)
    L.dm_net_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
    L.dm_net_destroy.argtypes = [vp]
    L.dm_net_destroy.restype = None
    L.dm_net_get_weights.argtypes = [vp, fp]
    L.dm_net_set_weights.argtypes = [vp, fp]
    L.dm_net_attach.argtypes = [vp, vp]
    L.dm_net_apply.argtypes = [vp, vp, d, vp, vp]
    L.dm_net_loss_grad.argtypes = [vp, i, vp, vp, d, dp, fp, vp]
    L.dm_net_make_pair.argtypes = [vp, ctypes.c_uint64, vp, vp, vp]
    L.dm_net_train.argtypes = [vp, i, i, ctypes.c_float, ctypes.c_uint64, fp, vp]
    L.dm_net_train_pairs.argtypes = [vp, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_float, fp, vp]
    L.dm_batch_create.argtypes = [i, ctypes.POINTER(Geometry), ctypes.POINTER(ctypes.c_int), dp, d,
                                  ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.dm_batch_destroy.argtypes = [vp]
    L.dm_batch_destroy.restype = None
    L.dm_batch_member.argtypes = [vp, i, ctypes.POINTER(vp)]
    L.dm_batch_info.argtypes = [vp, ctypes.POINTER(BatchStats)]
    L.dm_batch_vcycle.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.dm_batch_time_vcycle.argtypes = [vp, i, dp]
    L.dm_batch_eigs.argtypes = [vp, i, d, d, ctypes.c_uint64, ctypes.POINTER(EigOptions), dp, dp,
                                ctypes.POINTER(EigInfo), dp]
    _lib = L
    return L


def _check(rc, allow_warning=False):
    if rc == DM_OK or (allow_warning and rc > 0):
        return rc
    L = lib()
    raise DMError(rc, f"{L.dm_strerror(rc).decode()}: {L.dm_last_error_message().decode()}")


# ---------------------------------------------------------------------------
# geometry helpers
# ---------------------------------------------------------------------------

def box(bc_lo=(BC_PEC,) * 3, a_min=0.0) -> Geometry:
    g = Geometry()
    g.kind = GEOM_BOX
    g.bc_lo[:] = list(bc_lo)
    g.a_min = a_min
    return g


def ellipsoid(center, semi_axes, a_min=0.0) -> Geometry:
    g = Geometry()
    g.kind = GEOM_ELLIPSOID
    g.center[:] = list(center)
    g.semi_axes[:] = list(semi_axes)
    g.a_min = a_min
    return g


def sphere(center=(0.5, 0.5, 0.5), radius=0.45, a_min=0.0) -> Geometry:
    return ellipsoid(center, (radius,) * 3, a_min)


def elliptic_bor(axis_xy, z_start, n_cells, r_equator, r_iris, cell_length, tube_length,
                 bc_lo=(BC_PEC,) * 3, a_min=0.0) -> Geometry:
    g = Geometry()
    g.kind = GEOM_ELLIPTIC_BOR
    g.axis_xy[:] = list(axis_xy)
    g.z_start = z_start
    g.n_cells = n_cells
    g.r_equator, g.r_iris = r_equator, r_iris
    g.cell_length, g.tube_length = cell_length, tube_length
    g.bc_lo[:] = list(bc_lo)
    g.a_min = a_min
    return g


def user_fractions(frac7: np.ndarray, bc_lo=(BC_PEC,) * 3) -> Geometry:
    """Geometry from caller fractions: a (7, P) float64 array (ax..v) in the
    padded layout of level 0.  The array must outlive the build call."""
    g = Geometry()
    g.kind = GEOM_USER
    arr = np.ascontiguousarray(frac7, dtype=np.float64)
    g._keep = arr
    g.user_fractions_host = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    g.bc_lo[:] = list(bc_lo)
    return g


def levelset(phi_nodes: np.ndarray, refine: int, bc_lo=(BC_PEC,) * 3, a_min=0.0) -> Geometry:
    """General cavity {phi < 0} (DM_GEOM_LEVELSET): phi on the nodes of the
    grid refined `refine` times per cell, an array of shape
    (refine Nz + 1, refine Ny + 1, refine Nx + 1) (x fastest).  The array must
    outlive the build call."""
    g = Geometry()
    g.kind = GEOM_LEVELSET
    arr = np.ascontiguousarray(phi_nodes, dtype=np.float64)
    g._keep = arr
    g.levelset_host = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    g.levelset_refine = int(refine)
    g.bc_lo[:] = list(bc_lo)
    g.a_min = a_min
    return g


def padded_size(dims):
    return (dims[0] + 2) * (dims[1] + 2) * (dims[2] + 2)


def compute_fractions(geom: Geometry, dims, h) -> np.ndarray:
    """Host-side fractions (no GPU): (7, P) array ax ay az lx ly lz v."""
    P = padded_size(dims)
    out = np.zeros(7 * P)
    d = (ctypes.c_int * 3)(*dims)
    _check(lib().dm_compute_fractions(ctypes.byref(geom), d, float(h),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(7, P)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------

class Operator:
    """A built operator hierarchy (``dm_build_operator``)."""

    def __init__(self, geom: Geometry, dims, h, sigma, levels=0, nu_pre=2, nu_post=2,
                 fgmres_restart=30, verbose=0, cut_wave_split=None, learned_patience=None,
                 grad_div_volume=None, tilde_transfers=None, krylov_basis_f32=None):
        L = lib()
        opt = Options()
        L.dm_default_options(ctypes.byref(opt))
        opt.levels, opt.nu_pre, opt.nu_post = levels, nu_pre, nu_post
        opt.fgmres_restart, opt.verbose = fgmres_restart, verbose
        if cut_wave_split is not None:
            opt.cut_wave_split = int(cut_wave_split)
        if learned_patience is not None:
            opt.learned_patience = int(learned_patience)
        if grad_div_volume is not None:
            opt.grad_div_volume = int(grad_div_volume)
        if tilde_transfers is not None:
            opt.tilde_transfers = int(tilde_transfers)
        if krylov_basis_f32 is not None:
            opt.krylov_basis_f32 = int(krylov_basis_f32)
        self._op = ctypes.c_void_p()
        self._net = None
        self.dims = tuple(int(x) for x in dims)
        self.h = float(h)
        self._geom = geom
        d = (ctypes.c_int * 3)(*self.dims)
        _check(L.dm_build_operator(ctypes.byref(geom), d, self.h, float(sigma), ctypes.byref(opt),
                                   ctypes.byref(self._op)))
        self.sigma = float(sigma)

    def close(self):
        if self._op:
            lib().dm_destroy(self._op)
            self._op = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- layout
    def layout(self, level=0):
        out = (ctypes.c_int64 * 7)()
        _check(lib().dm_field_layout(self._op, level, out))
        return dict(dims=(out[0], out[1], out[2]), P=out[3], active_faces=out[4],
                    active_cells=out[5], levels=out[6])

    @property
    def levels(self):
        return self.layout(0)["levels"]

    def fractions(self, level=0) -> np.ndarray:
        P = self.layout(level)["P"]
        out = np.zeros(7 * P)
        _check(lib().dm_get_fractions(self._op, level,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(7, P)

    def set_shift(self, sigma):
        _check(lib().dm_set_shift(self._op, float(sigma)))
        self.sigma = float(sigma)

    # -- device tensors
    def face_tensor(self, level=0, dtype=None, device="cuda"):
        import torch
        return torch.zeros(3 * self.layout(level)["P"], dtype=dtype or torch.float64, device=device)

    def cell_tensor(self, level=0, device="cuda"):
        import torch
        return torch.zeros(self.layout(level)["P"], dtype=torch.float64, device=device)

    @staticmethod
    def _prec(t):
        import torch
        return 64 if t.dtype == torch.float64 else 32

    def apply(self, which, x, y, level=0, stream=None):
        _check(lib().dm_apply(self._op, which, self._prec(x), level, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def residual(self, f, x, r, level=0, stream=None):
        _check(lib().dm_residual(self._op, self._prec(x), level, _ptr(f), _ptr(x), _ptr(r), _stream(stream)))
        return r

    def smooth(self, f, x, sweeps=1, reverse=False, level=0, stream=None):
        _check(lib().dm_smooth(self._op, self._prec(x), level, sweeps, int(bool(reverse)), _ptr(f), _ptr(x),
                               _stream(stream)))
        return x

    def restrict(self, r, fc, level=0, stream=None):
        _check(lib().dm_restrict(self._op, self._prec(r), level, _ptr(r), _ptr(fc), _stream(stream)))
        return fc

    def prolong_add(self, xc, x, level=0, stream=None):
        _check(lib().dm_prolong_add(self._op, self._prec(x), level, _ptr(xc), _ptr(x), _stream(stream)))
        return x

    def vcycle(self, f, x, stream=None):
        _check(lib().dm_vcycle(self._op, self._prec(f), _ptr(f), _ptr(x), _stream(stream)))
        return x

    def vcycle_block(self, fs, xs, stream=None):
        """x_r = B f_r for every pair (1..4 vectors of one precision)."""
        n = len(fs)
        fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        _check(lib().dm_vcycle_block(self._op, self._prec(fs[0]), n, fp, xp, _stream(stream)))
        return xs

    def project(self, b, out, rtol=1e-13, stream=None):
        _check(lib().dm_project(self._op, _ptr(b), _ptr(out), float(rtol), _stream(stream)))
        return out

    def solve(self, f, x, mode=SOLVE_FGMRES_MG64, rtol=1e-10, maxit=500, stream=None):
        info = SolveInfo()
        rc = _check(lib().dm_solve(self._op, mode, _ptr(f), _ptr(x), float(rtol), int(maxit),
                                   ctypes.byref(info), _stream(stream)), allow_warning=True)
        return dict(status=rc, iterations=info.iterations, restarts=info.restarts,
                    rel_residual=info.rel_residual, seconds=info.seconds,
                    learned_accepted=info.learned_accepted, learned_rejected=info.learned_rejected)

    def project_block(self, bs, outs, rtol=1e-13, stream=None):
        """P_DM b_r for 1..4 vectors in lockstep."""
        n = len(bs)
        bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        op_ = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        _check(lib().dm_project_block(self._op, n, bp, op_, float(rtol), _stream(stream)))
        return outs

    def solve_block(self, fs, xs, mode=SOLVE_FGMRES_MG32, rtol=1e-10, maxit=500, stream=None):
        """M x_r = f_r for 1..4 systems in lockstep; one dict per system."""
        n = len(fs)
        fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        info = (SolveInfo * n)()
        rc = _check(lib().dm_solve_block(self._op, mode, n, fp, xp, float(rtol), int(maxit), info,
                                         _stream(stream)), allow_warning=True)
        return [dict(status=rc, iterations=q.iterations, restarts=q.restarts, rel_residual=q.rel_residual,
                     seconds=q.seconds) for q in info]

    def sample_e(self, b, lam, points, stream=None) -> np.ndarray:
        """Electric field C^T b / k of the eigenpair (b, lam) interpolated at
        points (n x 3 array of coordinates); NaN where the stencil leaves the grid."""
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        out = np.zeros_like(pts)
        _check(lib().dm_sample_e(self._op, _ptr(b), float(lam), pts.shape[0],
                                 pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)))
        return out

    def time_block_kernel(self, kernel, nrhs, prec=32, level=0, reps=50):
        """Milliseconds per launch of the block form of a kernel on nrhs vectors."""
        ms = ctypes.c_double()
        _check(lib().dm_time_block_kernel(self._op, kernel, prec, level, int(nrhs), reps, ctypes.byref(ms)))
        return ms.value

    def time_kernel(self, kernel, prec=32, level=0, reps=50):
        """Milliseconds per launch of a library kernel (HIP events)."""
        ms = ctypes.c_double()
        _check(lib().dm_time_kernel(self._op, kernel, prec, level, reps, ctypes.byref(ms)))
        return ms.value

    def eigs(self, k, sigma=None, tol=1e-10, seed=1301, vecs=None, solve_mode=SOLVE_FGMRES_MG64,
             inner_rtol=1e-11, proj_rtol=1e-13, block=4, max_basis=40, max_restarts=20,
             verbose=0, stream=None, start=None):
        """``start``: None, or a tensor of block face vectors (FP64, device)
        used as the start block."""
        L = lib()
        o = EigOptions()
        L.dm_default_eig_options(ctypes.byref(o))
        o.solve_mode, o.inner_rtol, o.proj_rtol = solve_mode, inner_rtol, proj_rtol
        o.block, o.max_basis, o.max_restarts, o.verbose = block, max_basis, max_restarts, verbose
        if start is not None:
            if start.dtype.is_floating_point is False or start.element_size() != 8 or \
                    start.numel() != block * 3 * self.layout(0)["P"]:
                raise ValueError("start block: block x 3P float64 values")
            o.start_dev = start.data_ptr()
        lam = np.zeros(k)
        res = np.zeros(k)
        info = EigInfo()
        sig = self.sigma if sigma is None else float(sigma)
        rc = _check(L.dm_eigs(self._op, int(k), sig, float(tol), ctypes.c_uint64(seed), ctypes.byref(o),
                              lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              _ptr(vecs) if vecs is not None else None,
                              res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              ctypes.byref(info), _stream(stream)), allow_warning=True)
        self.sigma = sig
        return dict(status=rc, lam=lam, residuals=res, n_converged=info.n_converged,
                    outer_iterations=info.outer_iterations, restarts=info.restarts,
                    inner_iterations=info.inner_iterations,
                    projection_iterations=info.projection_iterations,
                    max_residual=info.max_residual, seconds=info.seconds)


# ---------------------------------------------------------------------------
# learned correction
# ---------------------------------------------------------------------------

class Net:
    """The learned correction's network (``dm_net_*``)."""

    def __init__(self, seed=0):
        self._net = ctypes.c_void_p()
        _check(lib().dm_net_create(ctypes.c_uint64(seed), ctypes.byref(self._net)))

    def close(self):
        if self._net:
            lib().dm_net_destroy(self._net)
            self._net = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self) -> np.ndarray:
        w = np.zeros(NET_WEIGHTS, dtype=np.float32)
        _check(lib().dm_net_get_weights(self._net, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != NET_WEIGHTS:
            raise ValueError(f"expected {NET_WEIGHTS} weights")
        _check(lib().dm_net_set_weights(self._net, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def attach(self, op: "Operator"):
        _check(lib().dm_net_attach(op._op, self._net))
        op._net = self

    @staticmethod
    def detach(op: "Operator"):
        _check(lib().dm_net_attach(op._op, None))
        op._net = None


def net_apply(op: "Operator", r, out, scale=0.0, stream=None):
    _check(lib().dm_net_apply(op._op, _ptr(r), float(scale), _ptr(out), _stream(stream)))
    return out


def net_loss_grad(op: "Operator", r, e, scale=0.0, kind=NET_LOSS_ERROR, stream=None):
    loss = ctypes.c_double()
    g = np.zeros(NET_WEIGHTS, dtype=np.float32)
    _check(lib().dm_net_loss_grad(op._op, int(kind), _ptr(r), _ptr(e) if e is not None else None,
                                  float(scale), ctypes.byref(loss),
                                  g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
    return loss.value, g


def net_make_pair(op: "Operator", seed, r, e, stream=None):
    _check(lib().dm_net_make_pair(op._op, ctypes.c_uint64(seed), _ptr(r), _ptr(e), _stream(stream)))
    return r, e


def net_train(op: "Operator", steps, lr=1e-3, seed=0, kind=NET_LOSS_RESIDUAL, stream=None) -> np.ndarray:
    loss = np.zeros(max(1, steps), dtype=np.float32)
    _check(lib().dm_net_train(op._op, int(kind), int(steps), ctypes.c_float(lr), ctypes.c_uint64(seed),
                              loss.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
    return loss[:steps]


def net_train_pairs(op: "Operator", rs, es=None, lr=1e-3, kind=NET_LOSS_RESIDUAL, stream=None) -> np.ndarray:
    """One Adam step per given pair (r, e): device face vectors (float64)."""
    n = len(rs)
    loss = np.zeros(max(1, n), dtype=np.float32)
    rp = (ctypes.c_void_p * max(1, n))(*[r.data_ptr() for r in rs])
    ep = (ctypes.c_void_p * max(1, n))(*[e.data_ptr() for e in es]) if es is not None else None
    _check(lib().dm_net_train_pairs(op._op, int(kind), n, rp, ep, ctypes.c_float(lr),
                                    loss.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(stream)))
    return loss[:n]


# ---------------------------------------------------------------------------
# batched cavities
# ---------------------------------------------------------------------------

class _Member(Operator):
    """A batch member: an operator owned by its batch (never destroyed here)."""

    def __init__(self, handle, dims, h, sigma):   # noqa: D401 - no build
        self._op = handle
        self._net = None
        self.dims = tuple(int(x) for x in dims)
        self.h = float(h)
        self.sigma = float(sigma)

    def close(self):
        self._op = ctypes.c_void_p()


class Batch:
    """``dm_batch_*``: cavities whose FP32 V-cycles run as one fused V-cycle."""

    def __init__(self, geoms, dims, hs, sigma, levels=0, nu_pre=2, nu_post=2, fgmres_restart=30):
        L = lib()
        n = len(geoms)
        garr = (Geometry * n)(*geoms)
        darr = (ctypes.c_int * (3 * n))(*[int(v) for d3 in dims for v in d3])
        harr = (ctypes.c_double * n)(*[float(x) for x in hs])
        opt = Options()
        L.dm_default_options(ctypes.byref(opt))
        opt.levels, opt.nu_pre, opt.nu_post, opt.fgmres_restart = levels, nu_pre, nu_post, fgmres_restart
        self._b = ctypes.c_void_p()
        self._geoms = garr
        _check(L.dm_batch_create(n, garr, darr, harr, float(sigma), ctypes.byref(opt), ctypes.byref(self._b)))
        self.members = []
        for q in range(n):
            hdl = ctypes.c_void_p()
            _check(L.dm_batch_member(self._b, q, ctypes.byref(hdl)))
            self.members.append(_Member(hdl, dims[q], hs[q], sigma))
        self.sigma = float(sigma)

    def close(self):
        if self._b:
            for m in self.members:
                m.close()
            lib().dm_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        st = BatchStats()
        _check(lib().dm_batch_info(self._b, ctypes.byref(st)))
        return dict(count=st.count, threads_per_block=st.threads_per_block, tuned_ms=list(st.tuned_ms),
                    launches_per_vcycle=st.launches_per_vcycle, cells=st.cells, active_faces=st.active_faces)

    def vcycle(self, fs, xs, stream=None):
        n = len(self.members)
        fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        _check(lib().dm_batch_vcycle(self._b, fp, xp, _stream(stream)))
        return xs

    def time_vcycle(self, reps=10):
        ms = ctypes.c_double()
        _check(lib().dm_batch_time_vcycle(self._b, int(reps), ctypes.byref(ms)))
        return ms.value

    def eigs(self, k, sigma=None, tol=1e-10, seed=1301, inner_rtol=1e-11, proj_rtol=1e-13, block=4,
             max_basis=40, max_restarts=20):
        L = lib()
        n = len(self.members)
        o = EigOptions()
        L.dm_default_eig_options(ctypes.byref(o))
        o.solve_mode, o.inner_rtol, o.proj_rtol = SOLVE_FGMRES_MG32, inner_rtol, proj_rtol
        o.block, o.max_basis, o.max_restarts = block, max_basis, max_restarts
        lam = np.zeros(n * k)
        res = np.zeros(n * k)
        infos = (EigInfo * n)()
        secs = ctypes.c_double()
        sig = self.sigma if sigma is None else float(sigma)
        rc = _check(L.dm_batch_eigs(self._b, int(k), sig, float(tol), ctypes.c_uint64(seed), ctypes.byref(o),
                                    lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), infos,
                                    ctypes.byref(secs)), allow_warning=True)
        self.sigma = sig
        for m in self.members:
            m.sigma = sig
        return dict(status=rc, lam=lam.reshape(n, k), residuals=res.reshape(n, k), seconds=secs.value,
                    n_converged=[infos[q].n_converged for q in range(n)],
                    inner_iterations=[infos[q].inner_iterations for q in range(n)],
                    outer_iterations=[infos[q].outer_iterations for q in range(n)])
