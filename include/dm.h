/*
 * dm.h -- C ABI of the MI355X Dey--Mittra cut-cell cavity eigensolver.
 *
 * Problem (Bauer, Werner & Cary, arXiv:1301.3794): find the lowest
 * electromagnetic eigenpairs k^2, b of a perfectly conducting cavity on the
 * Yee mesh with Dey--Mittra cut cells, i.e. the smallest lambda > 0 of the
 * symmetric pencil  K b = lambda A b,  K = C L C^T  (Sec. 2, eq. discWaveBDM
 * multiplied by A).  The work is the shift-and-invert Krylov iteration of
 * eq. fullMat:  T = P_DM M^-1 A  with
 *      M    = C L C^T + A D^T V^-1 D A - sigma A          (eq. discLaplDM)
 *      P_DM = I - D^T (D A D^T)^-1 D A                     (eq. proj)
 * M is inverted by a multigrid-preconditioned Krylov solve (Sec. 6); every
 * step of that runs in this library's HIP kernels on the GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: Nx x Ny x Nz cubic cells of size h (Sec. 6, cubic cells), cell
 * (i,j,k) = [ih,(i+1)h] x [jh,(j+1)h] x [kh,(k+1)h].  Face b_x[i,j,k] is the
 * x = ih face of cell (i,j,k); edge e_x[i,j,k] runs from node (i,j,k) in +x.
 *
 * Field layout ("padded SoA"): every per-face, per-edge or per-cell array of
 * a grid level is one contiguous block of P = (Nx+2)(Ny+2)(Nz+2) elements;
 * element (i,j,k), -1 <= i <= Nx (same for j, k), sits at
 *      (i+1) + (Nx+2) * ((j+1) + (Ny+2) * (k+1)).
 * A face vector is three such blocks back to back (b_x, b_y, b_z): 3P
 * elements.  Entries of inactive faces (area fraction 0) and of the padding
 * are zero on input and are returned zero.  A cell vector is one block.
 * dm_field_layout() returns the sizes.  Fraction arrays (dm_get_fractions,
 * user fractions) are seven blocks in the order ax, ay, az, lx, ly, lz, v.
 *
 * Memory: pointers named *_dev are device pointers of the op's GPU (e.g.
 * torch tensor data), owned by the caller, contiguous, aligned to 8 bytes;
 * the library keeps no pointer after a call returns.  *_host are host
 * pointers.  The library owns the dm_op and all internal device buffers.
 *
 * Streams: `stream` is a hipStream_t passed as void*; NULL means the op's
 * own stream.  Calls enqueue their work on that stream and return after it
 * has completed (every entry point synchronises before returning), so
 * caller buffers may be reused at once.  One dm_op must not be used from two
 * host threads at the same time.
 *
 * Errors: 0 on success, a negative DM_E* code on error (the op is left
 * usable unless DM_EHIP), a positive code for a warning with a usable
 * partial result.  dm_strerror() names every code; dm_last_error_message()
 * gives the detail of the last error of the calling thread.
 */
#ifndef DM_H
#define DM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DM_OK               0
#define DM_NOT_CONVERGED    1    /* warning: iteration limit hit; partial result */
#define DM_EINVAL          (-1)  /* bad argument (size, pointer, option) */
#define DM_ENOMEM          (-2)  /* device or host allocation failed */
#define DM_EHIP            (-3)  /* HIP runtime error (detail in message) */
#define DM_ESINGULAR       (-4)  /* coarsest operator singular: sigma hits a
                                    coarse eigenvalue; choose another shift */
#define DM_EBREAKDOWN      (-5)  /* Krylov breakdown (e.g. zero start vector) */
#define DM_ENAN            (-6)  /* NaN/Inf met in an iterate or residual */
#define DM_ENODEVICE       (-7)  /* no HIP device available */

/* ---- geometry ---------------------------------------------------------- */
#define DM_GEOM_BOX          0   /* the domain box itself is the cavity */
#define DM_GEOM_ELLIPSOID    1   /* open axis-aligned ellipsoid (sphere: equal axes) */
#define DM_GEOM_ELLIPTIC_BOR 2   /* body of revolution about the line x=axis_xy[0],
                                    y=axis_xy[1]: beam tube, n_cells elliptic cells,
                                    beam tube (see fields below) */
#define DM_GEOM_USER         3   /* caller-supplied fractions */
#define DM_GEOM_LEVELSET     4   /* general cavity {phi < 0} from a sampled level set,
                                    volumes from conforming tetrahedra (Sec. 6.1);
                                    see levelset_host */

#define DM_BC_PEC 0              /* perfect electric conductor wall */
#define DM_BC_PMC 1              /* perfect magnetic conductor symmetry plane */

typedef struct {
    int kind;                    /* DM_GEOM_* */
    double center[3];            /* ellipsoid centre */
    double semi_axes[3];         /* ellipsoid semi-axes (sphere: all = R) */
    /* DM_GEOM_ELLIPTIC_BOR: radius profile r(z) of n_cells cells of length
       cell_length, each an elliptic arc from r_iris (cell ends) to r_equator
       (cell middle); tubes of radius r_iris and length tube_length on both
       sides; the structure starts at z = z_start and the end plates are
       perfect conductors. */
    double axis_xy[2];
    double z_start;
    int n_cells;
    double r_equator, r_iris, cell_length, tube_length;
    /* DM_GEOM_USER: 7 host blocks (ax, ay, az, lx, ly, lz, v) in the padded
       layout of level 0, copied at build time. */
    const double *user_fractions_host;
    /* boundary type of the low side x=0, y=0, z=0 of the domain (the high
       sides are always perfect electric conductors).  A PMC plane is a
       symmetry plane of the cavity (Sec. 6.3, quarter cavity). */
    int bc_lo[3];
    /* face neglect (Sec. 3): faces with area fraction below a_min are
       removed together with the edges around them; 0 keeps every cut face
       (the paper's choice for all its timing runs). */
    double a_min;
    /* DM_GEOM_LEVELSET: phi (< 0 in the cavity, >= 0 in the conductor) on the
       nodes of the grid refined s = levelset_refine >= 1 times per cell:
       (s Nx + 1)(s Ny + 1)(s Nz + 1) host doubles, x fastest, node (I, J, K)
       at (I, J, K) h / s; read at build time.  The cavity is where the
       piecewise-linear interpolant of phi on the Kuhn tetrahedra of the
       refined lattice (6 per refined cube, sharing its main diagonal) is
       negative, a polyhedron whose facets conform to those tetrahedra; cell
       volumes are sums of tetrahedral subvolumes, face areas and edge
       lengths those of the same polyhedron, so all three measure one body
       and converge with the refinement for smooth surfaces. */
    const double *levelset_host;
    int levelset_refine;
} dm_geometry;

/* ---- options ----------------------------------------------------------- */
typedef struct {
    int levels;          /* multigrid levels, 0 = halve while every dimension is
                            even, the largest exceeds 8 and the smallest is >= 4 */
    int nu_pre;          /* red-black sweeps before coarse correction (2) */
    int nu_post;         /* red-black sweeps after (2) */
    int fgmres_restart;  /* FGMRES restart length (30) */
    int verbose;         /* 0 silent, 1 per-solve lines on stderr */
    int cut_wave_split;  /* block smoother (2..4 vectors): a component whose list
                            of non-vacuum rows (both colours) is shorter than this
                            gives each vector its own wavefront; a longer list
                            takes one thread per row looping over the vectors
                            (65536; 0 always takes the loop).  Both give the same
                            values. */
    int learned_patience; /* DM_SOLVE_FGMRES_MG32_LEARNED: a solve stops trying the
                            network's correction after this many rejections (the
                            correction no longer lowers the residual there); 0
                            never stops.  (1) */
    /* Solver-sensitivity variants (Sec. 6.1 and Sec. 5.3), not for production
       runs; they change the operator or the preconditioner, not what the
       eigensolve converges to: */
    int grad_div_volume;  /* 1: the grad-div term is A D^T V^-1 D A (the method,
                            eq. discLaplDM); 0: V^-1 is left out, A D^T D A, on
                            every level (Sec. 6.1: inversions no longer
                            converge in reasonable time).  (1) */
    int tilde_transfers;  /* 0: the V-cycle of M; 1: the same V-cycle built for
                            the symmetric form of eq. fullMat2, M~ = A^-1/2 M
                            A^-1/2 (transfers P~ = A_f^-1/2 P A_c^1/2 and
                            R~ = P~^T / 8 in the variables of M; the smoother
                            is unchanged by the scaling).  Single-vector
                            V-cycles only: the block entry points and dm_eigs
                            refuse it.  (0) */
    int krylov_basis_f32; /* block FGMRES in the plain FP32-multigrid mode
                            (DM_SOLVE_FGMRES_MG32, dm_solve_block and dm_eigs
                            with block >= 2; even vector lengths): 1 keeps the
                            Krylov basis in FP32.  Each new column is still
                            formed and orthogonalised in FP64, then rounded
                            for storage, and every sum widens the stored
                            values, so only the storage is FP32: the
                            Gram--Schmidt passes read half the bytes.  The
                            Arnoldi relation then holds to FP32 rounding, so
                            one cycle lowers the true residual by about 1e-7
                            at most and a tighter tolerance takes restarts
                            (which FGMRES checks with the FP64 residual):
                            a gain for long, restarted solves, a loss where
                            one cycle would reach the tolerance.  Other modes
                            and single-vector solves ignore it.  (0) */
} dm_options;

/* Fills `opt` with the defaults listed above. */
void dm_default_options(dm_options *opt);

typedef struct dm_op dm_op;   /* opaque, owned by the library */

/* Builds the operator hierarchy on the current HIP device.
 *   geom   geometry description (host); copied.
 *   dims   Nx, Ny, Nz >= 2, each divisible by 2^(levels-1).
 *   h      cell size (> 0).
 *   sigma  shift of M (k^2 units, Sec. 4.1 eq. shiftInv); must not be an
 *          eigenvalue of the coarsest operator.
 *   opt    NULL for defaults.
 *   out    receives the new op.
 * Computes the cut fractions of every level on the host (coarse fractions
 * are exact sums of fine ones), uploads them in FP64 and FP32, and factors
 * the coarsest vector and scalar operators densely in FP64.
 * Errors: DM_EINVAL, DM_ENOMEM, DM_EHIP, DM_ENODEVICE, DM_ESINGULAR. */
int dm_build_operator(const dm_geometry *geom, const int dims[3], double h,
                      double sigma, const dm_options *opt, dm_op **out);

/* Releases the op and all its device memory.  NULL is ignored. */
void dm_destroy(dm_op *op);

/* Changes sigma (re-factors the coarsest level).  Errors: DM_ESINGULAR. */
int dm_set_shift(dm_op *op, double sigma);

/* Cut fractions on the host, without a GPU (setup step of build).
 *   out_host  7 * P doubles (level-0 padded layout, order ax..v).
 * Same values dm_build_operator uploads.  Errors: DM_EINVAL. */
int dm_compute_fractions(const dm_geometry *geom, const int dims[3], double h,
                         double *out_host);

/* Sizes of level `level`: out[0..2] = Nx, Ny, Nz of that level, out[3] = P
 * (elements per block), out[4] = number of active faces, out[5] = number of
 * active cells, out[6] = number of levels.  Errors: DM_EINVAL. */
int dm_field_layout(const dm_op *op, int level, int64_t out[7]);

/* Copies the fractions of `level` (7 * P doubles, order ax..v; v holds the
 * volume fraction, not its inverse). */
int dm_get_fractions(const dm_op *op, int level, double *out_host);

/* ---- operator applications (parity hooks and building blocks) ---------- */
#define DM_APPLY_M   0   /* y = M x = C L C^T x + A D^T V^-1 D A x - sigma A x  (eq. discLaplDM) */
#define DM_APPLY_K   1   /* y = K x = C L C^T x                               (eq. discWaveBDM times A) */
#define DM_APPLY_A   2   /* y = A x */
#define DM_APPLY_DA  3   /* cells: y = D A x   (eq. divBInt without V^-1) */
#define DM_APPLY_DT  4   /* faces: y = D^T x for a cell vector x (minus the gradient, eq. gradPhi) */
#define DM_APPLY_S   5   /* cells: y = D A D^T x  (scalar Laplacian of eq. proj) */

/* prec: 64 (double) or 32 (float) for M/K/A; DA/DT/S are FP64 only.
 * x_dev, y_dev: face or cell vectors of `level` in the padded layout. */
int dm_apply(dm_op *op, int which, int prec, int level, const void *x_dev,
             void *y_dev, void *stream);

/* r = f - M x on `level` (prec 64 or 32).  M acts on the active faces only:
 * rows of inactive faces (zero area fraction, ghosts) are written as zero,
 * whatever f holds there. */
int dm_residual(dm_op *op, int prec, int level, const void *f_dev,
                const void *x_dev, void *r_dev, void *stream);

/* n_sweeps red-black Gauss--Seidel sweeps of M x = f on `level`, in place on
 * x.  Sec. 6 smooths on every level on the way down and up of its
 * multigrid cycle (its smoother was a polynomial one in algebraic
 * multigrid); this smoother is a reading of that step for the geometric
 * V-cycle: one sweep updates the six classes (component, colour
 * (i+j+k) mod 2) in the order (x,0)(x,1)(y,0)(y,1)(z,0)(z,1); reverse != 0
 * uses the reverse order (post-smoothing).  prec 64 or 32. */
int dm_smooth(dm_op *op, int prec, int level, int n_sweeps, int reverse,
              const void *f_dev, void *x_dev, void *stream);

/* Staggered transfers between `level` and `level`+1 (prec 64 or 32), the
 * grid transfers of the geometric V-cycle that stands in for Sec. 6's
 * algebraic multigrid (the paper is silent on them; a reading).
 * Prolongation P: constant across the face normal; along it, a fine face
 * on a coarse face takes its value and one between two coarse faces takes
 * their mean weighted by the coarse area fractions, (a0 x0 + a1 x1) /
 * (a0 + a1); inactive faces of either level dropped.  Restriction
 * R = P^T / 8.
 *   dm_restrict:    f_coarse = R r_fine
 *   dm_prolong_add: x_fine  += P x_coarse */
int dm_restrict(dm_op *op, int prec, int level, const void *r_fine_dev,
                void *f_coarse_dev, void *stream);
int dm_prolong_add(dm_op *op, int prec, int level, const void *x_coarse_dev,
                   void *x_fine_dev, void *stream);

/* One multigrid V-cycle x = B f for M on level 0, zero initial guess (the
 * preconditioner of Sec. 6's inversions of M, eq. discLaplDM, as a
 * geometric V-cycle: a reading of the paper's algebraic one): nu_pre
 * sweeps, residual, restriction, recursion, prolongation, nu_post reverse
 * sweeps; exact dense FP64 solve on the coarsest level.  prec 64
 * (all FP64) or 32 (FP32 smoothing/transfers, FP64 coarsest solve).
 * Runs the same captured HIP graph the solvers use (f and x are copied to
 * and from the op's own buffers); the graph is recorded on first use and
 * re-recorded after dm_set_shift. */
int dm_vcycle(dm_op *op, int prec, const void *f_dev, void *x_dev, void *stream);

/* The same V-cycle on nrhs (1..4) vectors at once (Sec. 6: the block
 * eigensolver's inversions of one outer step share M).  Each launch serves
 * every vector, so each coefficient is read once per block; the values are
 * those of nrhs calls of dm_vcycle.  f_dev, x_dev: host arrays of nrhs
 * device pointers (face vectors of level 0, FP64 for prec 64, FP32 for 32).
 * A graph per (prec, nrhs) is recorded on first use. */
int dm_vcycle_block(dm_op *op, int prec, int nrhs, const void *const *f_dev, void *const *x_dev,
                    void *stream);

/* Divergence projection b_out = P_DM b (eq. proj); the scalar system
 * D A D^T psi = D A b is solved by CG preconditioned with a cell-centred
 * multigrid V-cycle until ||D A D^T psi - D A b||_2 <= rtol ||b||_A / h, a
 * bound on the scale of the field (not of its divergence), so nearly
 * divergence-free input costs few iterations.  FP64.  b and b_out may alias. */
int dm_project(dm_op *op, const double *b_dev, double *out_dev, double rtol,
               void *stream);
/* dm_project on nrhs (1..4) vectors at once (the projections of one block
 * step of the eigensolver): each vector runs its own CG on S, in lockstep,
 * with one block S apply and one block scalar V-cycle per step; the values
 * are those of nrhs calls of dm_project.  b_dev, out_dev: host arrays of
 * nrhs device pointers (FP64 face vectors); out may equal b. */
int dm_project_block(dm_op *op, int nrhs, const double *const *b_dev, double *const *out_dev, double rtol,
                     void *stream);

/* ---- linear solve of M x = f (Sec. 6: the inner inversion) -------------- */
#define DM_SOLVE_PCG64        0  /* CG + FP64 V-cycle (M must be SPD: sigma below
                                    the lowest eigenvalue of (K+G, A)) */
#define DM_SOLVE_FGMRES_MG64  1  /* flexible GMRES, FP64 V-cycle preconditioner */
#define DM_SOLVE_FGMRES_MG32  2  /* flexible GMRES (FP64), FP32 V-cycle */
#define DM_SOLVE_FGMRES_MG32_LEARNED 3  /* as MG32, then the attached network's
                                    correction (dm_net_attach), kept only where it
                                    lowers the FP64 residual of the V-cycle's answer;
                                    DM_EINVAL without an attached network */

typedef struct {
    int iterations;          /* preconditioner applications */
    int restarts;
    double rel_residual;     /* ||f - M x||_2 / ||f||_2, recomputed in FP64 */
    double seconds;
    int learned_accepted;    /* LEARNED mode: corrections kept / rejected */
    int learned_rejected;
} dm_solve_info;

/* x = M^-1 f to ||f - M x|| <= rtol ||f||, starting from x = 0.  FP64 in
 * and out.  The system is that of the active faces, so f should vanish on
 * inactive faces (M x does).  In the FGMRES modes the entries of f outside
 * the 128-byte lines that hold an active face (or a PMC ghost image of one)
 * are ignored, and x is zero there.  Returns
 * DM_NOT_CONVERGED if maxit preconditioner applications did not reach rtol
 * (x holds the best iterate). */
int dm_solve(dm_op *op, int mode, const double *f_dev, double *x_dev,
             double rtol, int maxit, dm_solve_info *info, void *stream);

/* ---- eigensolve (Sec. 4.1, Sec. 5.2 eq. fullMat) ------------------------ */
typedef struct {
    int solve_mode;      /* DM_SOLVE_* used for M^-1 (default FGMRES_MG64) */
    double inner_rtol;   /* relative tolerance of each M solve (1e-11) */
    double proj_rtol;    /* tolerance of each projection, see dm_project (1e-13) */
    int block;           /* block size of the Krylov--Schur iteration (4) */
    int max_basis;       /* basis size before a thick restart (40) */
    int max_restarts;    /* (20) */
    int verbose;
    /* NULL, or `block` face vectors (block * 3P doubles, device) taken as the
       start block instead of the seeded random one (a warm start from earlier
       eigenvectors); they are projected and A-orthonormalised like the
       random block.  A block that vanishes there (all zero, or gradients
       only) gives DM_EBREAKDOWN. */
    const double *start_dev;
} dm_eig_options;

void dm_default_eig_options(dm_eig_options *opt);

typedef struct {
    int n_converged;
    int outer_iterations;    /* block applications of T */
    int restarts;
    int inner_iterations;    /* total preconditioner applications in M solves */
    int projection_iterations;
    double max_residual;     /* max over returned pairs of rho (below) */
    double seconds;
} dm_eig_info;

/* The k smallest eigenvalues lambda > 0 of K b = lambda A b, by block
 * Krylov--Schur in the A-inner product (eq. bInner) on T = P_DM M^-1 A with
 * shift sigma, stopping when every pair has
 *     rho = ||K b - lambda A b||_{A^-1} / (lambda ||b||_A) <= tol.
 *   sigma        shift (M is re-factored if it differs from the op's); it
 *                may lie above some of the wanted eigenvalues (Sec. 4.1 puts
 *                it near the wanted ones): thick restarts keep the Ritz pairs
 *                whose estimate lambda = sigma + 1/theta is smallest and
 *                positive, below the shift as well as above it.
 *   seed         start block: N(0,1) on active faces from a counter-based
 *                generator keyed by seed.
 *   lambda_host  k doubles, ascending.
 *   vecs_dev     NULL or k face vectors (k * 3P doubles), A-orthonormal.
 *   residuals_host  NULL or k doubles (rho of each pair).
 * Returns DM_NOT_CONVERGED with info->n_converged if max_restarts is hit. */
/* nrhs (1..4) solves M x_r = f_r at once (the inversions of one block step
 * of the eigensolver, Sec. 4.3): each system runs its own FGMRES exactly as
 * dm_solve does, in lockstep, with the preconditioner applications of a step
 * done as one block V-cycle (dm_vcycle_block) and the products M z as one
 * block apply.  mode: an FGMRES mode (PCG64 is refused).  f_dev, x_dev: host
 * arrays of nrhs device pointers (FP64 face vectors); info: nrhs entries or
 * NULL (seconds and learned counts are those of the whole call).  Returns
 * DM_NOT_CONVERGED if any system did not reach rtol.  dm_eigs uses this path
 * for its blocks unless the op is a batch member or the mode is PCG64. */
int dm_solve_block(dm_op *op, int mode, int nrhs, const double *const *f_dev, double *const *x_dev,
                   double rtol, int maxit, dm_solve_info *info, void *stream);

int dm_eigs(dm_op *op, int k, double sigma, double tol, uint64_t seed,
            const dm_eig_options *opt, double *lambda_host, double *vecs_dev,
            double *residuals_host, dm_eig_info *info, void *stream);

/* ---- solve without allocation -------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as dm_solve(op, DM_SOLVE_PCG64, ...) -- same iterates, iterations
 * and result -- that calls no hipMalloc/hipFree.  Its four work vectors
 * (4 * 3P doubles) live in a static device array of
 * DM_NOALLOC_SCRATCH_BYTES per GPU, held from the first operator build on
 * that GPU until the process ends, so the op's level-0 grid must satisfy
 * 4 * 3P * 8 <= DM_NOALLOC_SCRATCH_BYTES (3P <= 1,048,576, e.g. 64^3 cells);
 * a larger op gets DM_EINVAL.  Every call on one GPU shares that array and
 * overwrites it: calls that overlap on one GPU (from several threads or
 * streams) race and must be serialised by the caller.  Errors as dm_solve. */
#define DM_NOALLOC_SCRATCH_BYTES (32u << 20)
int dm_solve_pcg_noalloc(dm_op *op, const double *f_dev, double *x_dev, double rtol, int maxit,
                         dm_solve_info *info, void *stream);

/* ---- batched cavities (one fused V-cycle for many operators) -------------
 * A batch owns `count` operators (cavities of their own grids and cell
 * sizes, no PMC planes).  Their FP32 V-cycles are merged level by level into
 * shared launches -- one launch per smoothing class, residual, transfer and
 * coarsest solve for all members -- recorded in one HIP graph; the block size
 * of those launches (64, 128 or 256 threads) is picked at creation by timing
 * each (autotuner).  Each member's values are exactly those of its own
 * V-cycle. */
typedef struct dm_batch dm_batch;   /* opaque, owned by the library */

typedef struct {
    int count;
    int threads_per_block;      /* chosen by the autotuner */
    double tuned_ms[3];         /* fused V-cycle at 64, 128, 256 threads per block */
    int launches_per_vcycle;
    int64_t cells;              /* finest cells over all members */
    int64_t active_faces;
} dm_batch_stats;

/* geoms[count], dims[3*count], h[count]; every member gets sigma and opt.
 * Errors as dm_build_operator; DM_EINVAL for PMC planes or mixed smoothing
 * counts. */
int dm_batch_create(int count, const dm_geometry *geoms, const int *dims, const double *h, double sigma,
                    const dm_options *opt, dm_batch **out);
void dm_batch_destroy(dm_batch *b);
/* the i-th member (owned by the batch; use it like any operator) */
int dm_batch_member(dm_batch *b, int i, dm_op **op);
int dm_batch_info(const dm_batch *b, dm_batch_stats *stats);
/* One fused FP32 V-cycle: x_i = B_i f_i for every member i (host arrays of
 * device pointers to FP32 face vectors of the members' finest grids). */
int dm_batch_vcycle(dm_batch *b, const float *const *f_dev, float *const *x_dev, void *stream);
/* Average milliseconds of one fused V-cycle (graph replay, HIP events). */
int dm_batch_time_vcycle(dm_batch *b, int reps, double *ms);
/* dm_eigs on every member (k pairs each, FP32-multigrid solve mode forced;
 * opt->start_dev must be NULL),
 * each on its own host thread and stream; every preconditioner application
 * of all running members is one fused V-cycle.  lambda_host: count*k,
 * residuals_host: count*k or NULL, info_host: count or NULL, seconds: wall
 * time or NULL.  Returns the worst member status (an error names the
 * member). */
int dm_batch_eigs(dm_batch *b, int k, double sigma, double tol, uint64_t seed, const dm_eig_options *opt,
                  double *lambda_host, double *residuals_host, dm_eig_info *info_host, double *seconds);

/* ---- learned correction (not in the paper) ------------------------------
 * A 3-D convolutional network on the cell grid corrects the FP32 V-cycle's
 * answer.  Input per cell (10 channels): the residual r of the V-cycle's
 * answer at the cell's low x, y, z faces divided by s = ||r||_2 / sqrt(number
 * of active faces), and the fractions a_x a_y a_z l_x l_y l_z v of the cell.
 * Layers: conv 3^3 10->16, ReLU, conv 3^3 16->16, ReLU, conv 3^3 16->3, no
 * bias (12,528 weights); bfloat16 weights and activations on MFMA with FP32
 * accumulation; zero outside the grid.  Output channel c at a cell, times
 * s h^2, is the correction of face component c there (0 on inactive faces).
 * Master weights are FP32, flat, layer by layer, [27 taps][in][out] with tap
 * = (dz+1)*9 + (dy+1)*3 + (dx+1).  Training runs Adam (Kingma & Ba) on the
 * FP32 master weights over pairs (r, e) with M e = r, minimising per pair
 *   DM_NET_LOSS_ERROR:    sum_active (y - e/(s h^2))^2 / sum_active (e/(s h^2))^2
 *   DM_NET_LOSS_RESIDUAL: ||r - M d||^2 / ||r||^2, d = the correction,
 * the second being what the learned solve mode judges (M symmetric: PEC
 * operators without symmetry planes).
 * A network is used by at most one operator at a time (dm_net_attach);
 * destroying either side detaches it. */
#define DM_NET_WEIGHTS 12528
typedef struct dm_net dm_net;   /* opaque, owned by the library */

/* He-uniform weights from a counter-based generator keyed by seed (last
 * layer scaled by 0.1).  Errors: DM_ENOMEM, DM_EHIP, DM_ENODEVICE. */
int dm_net_create(uint64_t seed, dm_net **out);
void dm_net_destroy(dm_net *net);
/* DM_NET_WEIGHTS floats, host memory, flat layout above. */
int dm_net_get_weights(const dm_net *net, float *weights_host);
int dm_net_set_weights(dm_net *net, const float *weights_host);
/* Bind net to op (NULL detaches); builds the fraction channels of op's
 * finest grid.  Both must live on the same device. */
int dm_net_attach(dm_op *op, dm_net *net);
/* out = network correction for residual r (face vectors, 3P doubles, device).
 * scale > 0 is used as s, else s is computed from r. */
int dm_net_apply(dm_op *op, const double *r_dev, double scale, double *out_dev, void *stream);
#define DM_NET_LOSS_ERROR    0
#define DM_NET_LOSS_RESIDUAL 1
/* Loss of one pair (r, e) (scale as above; e may be NULL for the residual
 * loss) and its gradient with respect to the master weights (DM_NET_WEIGHTS
 * floats to grad_host, may be NULL). */
int dm_net_loss_grad(dm_op *op, int kind, const double *r_dev, const double *e_dev, double scale,
                     double *loss_host, float *grad_host, void *stream);
/* A training pair on op's grid: x* = V(w) for w ~ N(0,1) on active faces
 * (counter-based, keyed by seed), f = M x*, z = V(f) (FP32 V-cycles), and
 * r = f - M z, e = x* - z, so that M e = r.  r_dev, e_dev: 3P doubles. */
int dm_net_make_pair(dm_op *op, uint64_t seed, double *r_dev, double *e_dev, void *stream);
/* `steps` Adam steps with learning rate lr, one fresh pair (seed + step)
 * per step; loss_host (may be NULL) receives the loss of every step. */
int dm_net_train(dm_op *op, int kind, int steps, float lr, uint64_t seed, float *loss_host,
                 void *stream);
/* `npairs` Adam steps on caller-given pairs, one pair per step in order:
 * r_dev[i] (and e_dev[i] for the error loss; e_dev may be NULL for the
 * residual loss) are host arrays of device face vectors (3P doubles) on
 * op's finest grid, s computed from r.  Continues the network's Adam state
 * (step count and moments, reset by dm_net_set_weights), as dm_net_train
 * does.  loss_host (may be NULL): the loss of every step. */
int dm_net_train_pairs(dm_op *op, int kind, int npairs, const double *const *r_dev, const double *const *e_dev,
                       float lr, float *loss_host, void *stream);

/* ---- fields of an eigenpair --------------------------------------------- */
/* Electric field of an eigenpair (b, lambda = k^2) of the op's finest grid at
 * npts points (Sec. 6.2, surface fields): e = C^T b / k on every edge with
 * l > 0 and 0 on the others (the Yee scheme's Ampere law in the frequency
 * domain, whose Faraday law a b = C L e / k closes K b = lambda A b),
 * interpolated trilinearly from each component's own edge lattice: e_x at
 * ((i + 1/2) h, j h, k h), e_y at (i h, (j + 1/2) h, k h), e_z likewise.
 *   b_dev    one face vector (3P doubles, device), e.g. from dm_eigs.
 *   pts_host npts x 3 coordinates (host); e_host npts x 3 values (host).
 * A point whose interpolation stencil leaves the grid gets NaN.  Errors:
 * DM_EINVAL (lambda <= 0, npts < 0, NULL pointers). */
int dm_sample_e(dm_op *op, const double *b_dev, double lambda, int npts, const double *pts_host,
                double *e_host, void *stream);

/* ---- measurement -------------------------------------------------------- */
#define DM_KERNEL_APPLY     0  /* y = M x on `level` */
#define DM_KERNEL_RESIDUAL  1  /* r = f - M x on `level` */
#define DM_KERNEL_SMOOTH    2  /* one class update: component x, colour 0 */
#define DM_KERNEL_SWEEP     3  /* the six class updates of one red-black sweep */
#define DM_KERNEL_RESTRICT  4  /* `level` -> `level`+1 */
#define DM_KERNEL_PROLONG   5  /* `level`+1 -> `level` */
#define DM_KERNEL_VCYCLE    6  /* one whole V-cycle, replayed from the solver's
                                  captured graph (level must be 0) */
#define DM_KERNEL_NET       7  /* the attached learned network's forward pass: its
                                  three convolutions on the finest grid (bfloat16
                                  MFMA; level 0, prec 32, a network attached
                                  with dm_net_attach, else DM_EINVAL) */

/* Average duration of one launch of `kernel` (prec 64 or 32) on seeded
 * N(0,1) data in library-owned buffers: 2 untimed launches, then `reps`
 * launches bracketed by HIP events on the op's stream.  Writes the
 * milliseconds per launch.  Used for roofline figures; touches no caller
 * memory.  Errors: DM_EINVAL, DM_ENOMEM, DM_EHIP. */
int dm_time_kernel(dm_op *op, int kernel, int prec, int level, int reps,
                   double *ms_per_launch);
/* The same for the block form of `kernel` on nrhs (1..4) vectors (the
 * kernels of dm_vcycle_block; DM_KERNEL_VCYCLE replays its graph). */
int dm_time_block_kernel(dm_op *op, int kernel, int prec, int level, int nrhs, int reps,
                         double *ms_per_launch);

/* ---- diagnostics -------------------------------------------------------- */
const char *dm_strerror(int code);
const char *dm_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* DM_H */
