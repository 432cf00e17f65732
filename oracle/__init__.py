"""CPU oracle for the Dey--Mittra cut-cell cavity eigensolver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
product path (the C-ABI library and its Python binding) never imports,
links or executes this package, and this package never imports the product.

The oracle is deliberately plain and slow: NumPy/SciPy in float64, sparse
matrices assembled entry by entry from the definitions in the paper, dense
``eigh`` for tiny grids and a plain shift-and-invert Lanczos with CG inner
solves for larger ones.  Each function cites the section / equation of
Bauer, Werner & Cary, "A fast multigrid-based electromagnetic eigensolver
for curved metal boundaries on the Yee mesh" (arXiv:1301.3794) it follows.

Modules
-------
geometry   cut face-area, edge-length and cell-volume fractions (Sec. 2,
           eq. farInt; Sec. 5.1, eq. divBInt) for box, sphere, ellipsoid
           and elliptic-cell bodies of revolution.
operators  staggered Yee index sets and the sparse matrices C^T, D, A, L,
           V, K = C L C^T, G = A D^T V^-1 D A, M = K + G - sigma A and
           S = D A D^T (eqs. discWaveBDM, divBDM, discLaplDM, proj).
eigs       dense generalized eigensolve of (K, A) and shift-and-invert
           Lanczos on P_DM M^-1 A (eqs. shiftInv, fullMat) with CG.
multigrid  the V-cycle definition the GPU path must reproduce (geometric
           coarsening by exact fraction summation, component x colour
           Gauss--Seidel, staggered transfers, dense coarsest solve).
symmetry   PMC symmetry planes (Sec. 6.3 quarter cavities) through the
           full mirrored cavity.
learned    the learned correction's 3-layer conv network, loss, gradients
           and Adam step (not in the paper), with optional bfloat16
           rounding at the points the device stores bfloat16.

Parity status of every function is recorded in its docstring; the only
"parity unpinned" items are listed in ``UNPINNED`` below.
"""

UNPINNED = (
    # The V-cycle transfer operators and smoother ordering are this project's
    # reading (the paper used algebraic multigrid).  Pinned indirectly: the
    # V-cycle operator is symmetric, reduces to the exact inverse with one
    # level, and contracts the error; its exact values have no closed form.
    "multigrid.vcycle: transfer/smoother choice is a reading, pinned by "
    "symmetry, one-level exactness and contraction only",
)
