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
