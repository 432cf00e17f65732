"""Studies of the paper's accuracy and solver-sensitivity results, run through
the library (argument marshalling and bookkeeping only: every eigensolve,
solve and field sample runs in the library's kernels).

* ``frequency_convergence`` -- Sec. 6.2 and Fig. freqErr3d: the relative
  error of the lowest mode of the sphere's positive octant (symmetry planes
  x = 0, y = 0, z = 0 taken as perfect conductors, sphere centred on the
  origin), against the resolution, with every cut face kept and with faces
  below a_min neglected (Sec. 3).  For these symmetries the lowest mode is
  the sphere's TM mode of degree 3 whose angular part is x y z / r^3; its
  wavenumber is x_3 / R with x_3 the first root of d/dx [x j_3(x)] = 0.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import dm


def tm_root(l: int, lo: float, hi: float) -> float:
    """Root of d/dx [x j_l(x)] = j_l(x) + x j_l'(x) in (lo, hi): the TM modes
    of a perfectly conducting sphere have k R equal to such roots."""
    from scipy import optimize, special

    def f(x):
        return special.spherical_jn(l, x) + x * special.spherical_jn(l, x, derivative=True)
    return optimize.brentq(f, lo, hi, xtol=1e-15, rtol=1e-15)


def fit_order(h, err) -> float:
    """Least-squares slope of log(err) against log(h)."""
    return float(np.polyfit(np.log(np.asarray(h, float)), np.log(np.asarray(err, float)), 1)[0])


def octant_operator(n: int, radius=0.45, box=0.5, a_min=0.0, sigma=40.0, **kw) -> dm.Operator:
    """The sphere's positive octant on n^3 cells of size box / n: the sphere
    centred on the grid's corner node, conducting planes x = 0, y = 0, z = 0
    (the domain's low walls), faces with area fraction below a_min
    neglected."""
    geom = dm.ellipsoid((0.0, 0.0, 0.0), (radius, radius, radius), a_min=a_min)
    return dm.Operator(geom, (n, n, n), box / n, sigma, **kw)


def frequency_convergence(ns=(16, 24, 32, 48, 64), a_mins=(0.0, 0.1), radius=0.45, box=0.5, sigma=40.0,
                          tol=1e-10, solve_mode=None):
    """Relative error |omega - omega_0| / omega_0 = |sqrt(lambda) - k_0| / k_0
    of the octant's lowest eigenvalue for every resolution and a_min, with
    k_0 = x_3 / R; also the resolution in vacuum wavelengths per cell,
    lambda_vac / h = 2 pi / (k_0 h) (the paper's abscissa), and the orders
    fitted over the three finest grids."""
    mode = dm.SOLVE_FGMRES_MG32 if solve_mode is None else solve_mode
    k0 = tm_root(3, 4.5, 5.5) / radius
    rows = []
    for a_min in a_mins:
        for n in ns:
            h = box / n
            t0 = time.perf_counter()
            with octant_operator(n, radius, box, a_min, sigma) as op:
                out = op.eigs(1, sigma=sigma, tol=tol, seed=1, solve_mode=mode, block=2, max_basis=24,
                              max_restarts=40)
                faces = op.layout(0)["active_faces"]
            lam = float(out["lam"][0])
            rows.append(dict(a_min=a_min, n=n, h=h, active_faces=faces, lam=lam, status=out["status"],
                             rel_freq_err=abs(math.sqrt(lam) - k0) / k0,
                             wavelengths_per_cell=2.0 * math.pi / (k0 * h), residual=out["max_residual"],
                             seconds=time.perf_counter() - t0))
    orders = {}
    for a_min in a_mins:
        sel = [r for r in rows if r["a_min"] == a_min][-3:]
        orders[str(a_min)] = fit_order([r["h"] for r in sel], [r["rel_freq_err"] for r in sel])
    return dict(k0=k0, lambda0=k0 * k0, rows=rows, orders_finest3=orders)


# ---------------------------------------------------------------------------
# Solver sensitivity (Sec. 6.1, Table volPert1; Sec. 5.3, eq. fullMat2)
# ---------------------------------------------------------------------------

def perturb_volumes(frac7: np.ndarray, kind: str, amount: float, seed: int) -> np.ndarray:
    """The volume-error models of Sec. 6.1 on the cut cells (0 < v < 1) of a
    padded fraction array (7 blocks, v last), f uniform in [-1, 1] per cell
    from a NumPy generator keyed by seed:
      kind 'log'  (eq. volPert1): v~ = 10^(f eps) v,   eps = amount;
      kind 'add'  (eq. volPert2): v~ = |v + f dv|,      dv = amount (in cell
                  volumes; the magnitude keeps a volume positive where the
                  error exceeds the volume itself).
    Everything else is left as it is."""
    out = np.array(frac7, dtype=np.float64, copy=True)
    v = out[6]
    cut = np.flatnonzero((v > 0.0) & (v < 1.0))
    f = np.random.default_rng(seed).uniform(-1.0, 1.0, cut.size)
    if kind == "log":
        v[cut] = 10.0 ** (f * amount) * v[cut]
    elif kind == "add":
        w = np.abs(v[cut] + f * amount)
        v[cut] = np.where(w > 0.0, w, v[cut])
    else:
        raise ValueError(kind)
    return out


def average_inner_iterations(op: dm.Operator, seeds=(1, 2, 3), rtol=1e-6, maxit=2000, mode=None):
    """Mean FGMRES iterations of M x = A w for w ~ N(0,1) on the active faces
    (one right-hand side per seed), and whether every solve converged."""
    import torch
    mode = dm.SOLVE_FGMRES_MG64 if mode is None else mode
    mask = torch.tensor(op.fractions(0)[:3].reshape(-1) > 0)
    its, ok = [], True
    for sd in seeds:
        w = (torch.randn(mask.numel(), dtype=torch.float64, generator=torch.Generator().manual_seed(sd)) * mask).cuda()
        f = op.apply(dm.APPLY_A, w, op.face_tensor())
        out = op.solve(f, op.face_tensor(), mode=mode, rtol=rtol, maxit=maxit)
        its.append(out["iterations"])
        ok &= out["status"] == 0
    return float(np.mean(its)), bool(ok)


def solver_sensitivity(n=32, radius=0.49, sigma=5.0, eps=(0.1, 0.3, 0.5, 1.0, 2.0, 3.0), dv=(1e-5, 1e-4, 1e-3),
                       trials=3, restart=40, rtol=1e-6, maxit=2000):
    """Average inner iterations of the sphere (radius 0.49 of the unit box,
    as in Sec. 6.1) at n^3 for the method and its variants: volume errors of
    eq. volPert1 (eps) and eq. volPert2 (dv, in cell volumes), `trials`
    perturbations each; V^-1 left out of the operator; the tilde form's
    V-cycle (eq. fullMat2).  FGMRES(restart), FP64 V-cycle, tolerance rtol
    as in the paper (1e-6)."""
    h = 1.0 / n
    geom = dm.sphere((0.5, 0.5, 0.5), radius)
    frac = dm.compute_fractions(geom, (n, n, n), h).reshape(7, -1)
    rows = []

    def run(label, value, fr7=None, **kw):
        g = geom if fr7 is None else dm.user_fractions(fr7)
        with dm.Operator(g, (n, n, n), h, sigma, fgmres_restart=restart, **kw) as op:
            its, ok = average_inner_iterations(op, rtol=rtol, maxit=maxit)
        return its, ok

    its, ok = run("method", None)
    rows.append(dict(variant="method", value=None, avg_iterations=its, converged=ok))
    for kind, values in (("log", eps), ("add", dv)):
        for val in values:
            res = [run(kind, val, perturb_volumes(frac, kind, val, 100 + t)) for t in range(trials)]
            rows.append(dict(variant="volume error " + ("eq. volPert1, eps" if kind == "log" else
                                                        "eq. volPert2, dv/v_vac"),
                             value=val, avg_iterations=float(np.mean([r[0] for r in res])),
                             converged=all(r[1] for r in res)))
    its, ok = run("novol", None, grad_div_volume=0)
    rows.append(dict(variant="V^-1 left out", value=None, avg_iterations=its, converged=ok))
    its, ok = run("tilde", None, tilde_transfers=1)
    rows.append(dict(variant="tilde form (eq. fullMat2) V-cycle", value=None, avg_iterations=its, converged=ok))
    return dict(grid=[n, n, n], radius=radius, sigma=sigma, restart=restart, rtol=rtol, maxit=maxit, rows=rows)


# ---------------------------------------------------------------------------
# General geometry: tetrahedral cut-cell volumes (Sec. 6.1)
# ---------------------------------------------------------------------------

def sphere_levelset(n: int, s: int, radius=0.45, center=(0.5, 0.5, 0.5)) -> np.ndarray:
    """|x - c| - R on the nodes of the n^3 grid of the unit box refined s
    times per cell, array [K, J, I]."""
    h = 1.0 / n
    t = np.arange(s * n + 1) * (h / s)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2) - radius


def levelset_convergence(n=32, refinements=(1, 2, 4, 8), radius=0.45, sigma=5.0, k=3, tol=1e-10):
    """The sphere as a general geometry (level set sampled on the grid refined
    s times, tetrahedral fractions) against its analytic fractions: the
    relative error of the total cut-cell volume against 4 pi R^3 / 3, and the
    lowest k eigenvalues' largest relative difference from those computed
    with the analytic fractions, per refinement."""
    h = 1.0 / n
    exact = 4.0 / 3.0 * math.pi * radius ** 3
    with dm.Operator(dm.sphere((0.5, 0.5, 0.5), radius), (n, n, n), h, sigma) as op:
        ref = op.eigs(k, tol=tol, seed=1, solve_mode=dm.SOLVE_FGMRES_MG32, block=k, max_restarts=40)["lam"]
        v_analytic = float(op.fractions(0)[6].sum()) * h ** 3
    rows = []
    for s in refinements:
        phi = sphere_levelset(n, s, radius)
        geom = dm.levelset(phi, s)
        vol = float(dm.compute_fractions(geom, (n, n, n), h)[6].sum()) * h ** 3
        with dm.Operator(geom, (n, n, n), h, sigma) as op:
            out = op.eigs(k, tol=tol, seed=1, solve_mode=dm.SOLVE_FGMRES_MG32, block=k, max_restarts=40)
        rows.append(dict(refine=s, volume_rel_err=abs(vol - exact) / exact, status=out["status"],
                         lam=out["lam"].tolist(),
                         max_rel_diff_vs_analytic=float(np.max(abs(out["lam"] - ref) / ref))))
    return dict(grid=[n, n, n], analytic_volume_rel_err=abs(v_analytic - exact) / exact,
                lam_analytic=ref.tolist(), rows=rows)


# ---------------------------------------------------------------------------
# Surface fields (Sec. 6.2, eq. errorNorm, Fig. fieldErr3d)
# ---------------------------------------------------------------------------

def tm3_xyz_field(points, k0):
    """Electric field (unnormalised) of the sphere's TM mode of degree 3 with
    angular part x y z / r^3, centred on the origin, wavenumber k0: with
    psi = j_3(k0 r) Y, Y = x y z / r^3, the TM field is curl (r x grad psi),
    and curl (r x grad psi) = -grad(d/dr (r psi)) - k0^2 psi r_vec for a
    Helmholtz solution psi, so E = grad(g Y) + k0^2 f Y r_vec with
    f = j_3(k0 r) and g = (r f)' = j_3 + k0 r j_3'; it is radial on the wall
    where g(R) = 0 (the TM condition [x j_3(x)]' = 0)."""
    from scipy import special
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    r = np.sqrt(x * x + y * y + z * z)
    kr = k0 * r
    j = special.spherical_jn(3, kr)
    jp = special.spherical_jn(3, kr, derivative=True)
    # spherical Bessel equation: x^2 j'' + 2 x j' + (x^2 - 12) j = 0
    jpp = -2.0 / kr * jp - (1.0 - 12.0 / (kr * kr)) * j
    g = j + kr * jp
    gp = k0 * (2.0 * jp + kr * jpp)
    Y = x * y * z / r ** 3
    grad_y = np.stack([y * z, x * z, x * y], axis=1) / r[:, None] ** 3 - 3.0 * (Y / r ** 2)[:, None] * p
    return (gp * Y / r)[:, None] * p + g[:, None] * grad_y + (k0 * k0 * j * Y)[:, None] * p


def octant_directions(count=400):
    """Unit vectors spread over the positive octant (a Fibonacci lattice on
    the sphere, kept where every component is positive)."""
    m = 8 * count
    i = np.arange(m) + 0.5
    phi = np.arccos(1.0 - 2.0 * i / m)
    theta = np.pi * (1.0 + 5 ** 0.5) * i
    d = np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)], axis=1)
    return d[(d > 0).all(axis=1)]


def surface_field_convergence(ns=(16, 24, 32, 48, 64), a_mins=(0.0, 0.1), radius=0.45, box=0.5, sigma=40.0,
                              tol=1e-10, shell_cells=3.0):
    """eq. errorNorm on the sphere octant's lowest mode: the relative l2 error
    of the computed electric field (dm_sample_e: C^T b / k, trilinear) against
    the analytic one on a shell shell_cells cells inside the wall, after both
    are scaled to unit l2 norm over one fixed set of points filling the
    cavity (and the computed one's sign matched).  Test points lie at least
    one cell of the coarsest grid from the symmetry planes, where trilinear
    interpolation needs no mirrored values (a reading: the paper samples the
    whole shell)."""
    import torch
    k0 = tm_root(3, 4.5, 5.5) / radius
    h_max = box / min(ns)
    dirs = octant_directions()
    g = np.arange(h_max, radius, radius / 14.0)
    vol = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    vol = vol[(np.linalg.norm(vol, axis=1) <= radius - shell_cells * h_max) & (vol >= h_max).all(axis=1)]
    e_vol = tm3_xyz_field(vol, k0)
    e_vol /= np.linalg.norm(e_vol)
    rows = []
    for a_min in a_mins:
        for n in ns:
            h = box / n
            shell = (radius - shell_cells * h) * dirs
            shell = shell[(shell >= h_max).all(axis=1)]
            e_sh = tm3_xyz_field(shell, k0)
            with octant_operator(n, radius, box, a_min, sigma) as op:
                P = op.layout(0)["P"]
                vecs = torch.zeros(3 * P, dtype=torch.float64, device="cuda")
                out = op.eigs(1, sigma=sigma, tol=tol, seed=1, vecs=vecs, solve_mode=dm.SOLVE_FGMRES_MG32,
                              block=2, max_basis=24, max_restarts=40)
                lam = float(out["lam"][0])
                c_vol = op.sample_e(vecs, lam, vol)
                c_sh = op.sample_e(vecs, lam, shell)
            scale = 1.0 / np.linalg.norm(c_vol)
            sign = 1.0 if np.sum(c_vol * e_vol) >= 0 else -1.0
            ref_scale = 1.0 / np.linalg.norm(tm3_xyz_field(vol, k0))
            diff = sign * scale * c_sh - ref_scale * e_sh
            err = float(np.sqrt(np.sum(diff * diff) / np.sum((ref_scale * e_sh) ** 2)))
            rows.append(dict(a_min=a_min, n=n, h=h, status=out["status"], lam=lam, shell_points=int(len(shell)),
                             rel_field_err=err, wavelengths_per_cell=2.0 * math.pi / (k0 * h)))
    orders = {}
    for a_min in a_mins:
        sel = [r for r in rows if r["a_min"] == a_min][-3:]
        orders[str(a_min)] = fit_order([r["h"] for r in sel], [r["rel_field_err"] for r in sel])
    return dict(k0=k0, volume_points=int(len(vol)), rows=rows, orders_finest3=orders)
