// Internal declarations of the Dey--Mittra eigensolver library.
//
// Field layout: padded SoA blocks of P = (Nx+2)(Ny+2)(Nz+2) elements, element
// (i,j,k) at (i+1) + sy (j+1) + sz (k+1), x fastest; a face vector is the
// three blocks b_x, b_y, b_z back to back.  Coefficient blocks per level:
// ax ay az (face area fractions), lx ly lz (edge length fractions), vinv
// (1 / cell volume fraction, 0 for cells outside the cavity).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "dm.h"

namespace dm {

struct Grid {
    int nx, ny, nz;
    int sy;        // j stride = nx + 2
    int64_t sz;    // k stride = (nx+2)(ny+2)
    int64_t P;     // elements per block
    double h;
    int pmc;       // bit a set: the low side of axis a is a PMC symmetry plane
};

inline Grid make_grid(int nx, int ny, int nz, double h, int pmc = 0) {
    Grid g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.sy = nx + 2;
    g.sz = (int64_t)(nx + 2) * (ny + 2);
    g.P = g.sz * (nz + 2);
    g.h = h;
    g.pmc = pmc;
    return g;
}

__host__ __device__ inline int64_t pidx(const Grid &g, int i, int j, int k) {
    return (int64_t)(i + 1) + (int64_t)(j + 1) * g.sy + (int64_t)(k + 1) * g.sz;
}

// ---------------------------------------------------------------------------
// PMC symmetry planes (quarter-cavity runs, Sec. 6.3).  A low-side plane of
// axis a is a node plane; the field continues across it as a mirror image:
// the face component normal to a is even (ghost at -1 = value at +1), the
// tangential components and cell scalars are odd (ghost at -1 = -value at 0).
// The padding layer holds these ghosts, so the stencil rows below evaluate
// the full-cavity operator on the symmetric field.  Every kernel that writes
// a vector also writes the ghost images of what it owns.
// ---------------------------------------------------------------------------

// Ghost images of face component `comp` owned by cell (i,j,k): up to 7
// (offset, sign) pairs (both planes and their corner).  Returns the count.
__host__ __device__ inline int face_images(const Grid &g, int comp, int i, int j, int k,
                                           int64_t off[7], signed char sgn[7]) {
    int64_t o1[3];
    signed char s1[3];
    int na = 0;
    const int idx[3] = {i, j, k};
    const int64_t stride[3] = {1, g.sy, g.sz};
    for (int a = 0; a < 3; ++a) {
        if (!((g.pmc >> a) & 1)) continue;
        if (comp == a && idx[a] == 1) { o1[na] = -2 * stride[a]; s1[na] = 1; ++na; }
        else if (comp != a && idx[a] == 0) { o1[na] = -stride[a]; s1[na] = -1; ++na; }
    }
    int cnt = 0;
    for (int m = 1; m < (1 << na); ++m) {
        int64_t o = 0;
        int s = 1;
        for (int b = 0; b < na; ++b)
            if ((m >> b) & 1) { o += o1[b]; s *= s1[b]; }
        off[cnt] = o;
        sgn[cnt] = (signed char)s;
        ++cnt;
    }
    return cnt;
}

// Ghost images of a cell scalar (odd across every PMC plane) at (i,j,k).
__host__ __device__ inline int cell_images(const Grid &g, int i, int j, int k, int64_t off[7],
                                           signed char sgn[7]) {
    int64_t o1[3];
    int na = 0;
    const int idx[3] = {i, j, k};
    const int64_t stride[3] = {1, g.sy, g.sz};
    for (int a = 0; a < 3; ++a)
        if (((g.pmc >> a) & 1) && idx[a] == 0) o1[na++] = -stride[a];
    int cnt = 0;
    for (int m = 1; m < (1 << na); ++m) {
        int64_t o = 0;
        int s = 1;
        for (int b = 0; b < na; ++b)
            if ((m >> b) & 1) { o += o1[b]; s = -s; }
        off[cnt] = o;
        sgn[cnt] = (signed char)s;
        ++cnt;
    }
    return cnt;
}

template <class T>
__host__ __device__ inline void put_face(const Grid &g, T *arr, int comp, int i, int j, int k,
                                         int64_t p, T v) {
    arr[p] = v;
    if (g.pmc) {
        int64_t off[7];
        signed char sg[7];
        const int n = face_images(g, comp, i, j, k, off, sg);
        for (int q = 0; q < n; ++q) arr[p + off[q]] = sg[q] > 0 ? v : -v;
    }
}

template <class T>
__host__ __device__ inline void put_cell(const Grid &g, T *arr, int i, int j, int k, int64_t p, T v) {
    arr[p] = v;
    if (g.pmc) {
        int64_t off[7];
        signed char sg[7];
        const int n = cell_images(g, i, j, k, off, sg);
        for (int q = 0; q < n; ++q) arr[p + off[q]] = sg[q] > 0 ? v : -v;
    }
}

// extra diagonal of the curl-curl row from the odd mirror of a tangential
// component on a PMC plane (the edge in the plane sees the value twice)
template <class T>
__host__ __device__ inline T pmc_diag_extra(const Grid &g, const T *lx, const T *ly, const T *lz,
                                            int comp, int i, int j, int k, int64_t p) {
    if (!g.pmc) return T(0);
    T e = T(0);
    if ((g.pmc & 1) && i == 0) e += comp == 1 ? lz[p] : (comp == 2 ? ly[p] : T(0));
    if ((g.pmc & 2) && j == 0) e += comp == 0 ? lz[p] : (comp == 2 ? lx[p] : T(0));
    if ((g.pmc & 4) && k == 0) e += comp == 0 ? ly[p] : (comp == 1 ? lx[p] : T(0));
    return e;
}

enum { CAX = 0, CAY, CAZ, CLX, CLY, CLZ, CVINV, NCOEF };

template <class T>
struct Coefs {
    const T *ax, *ay, *az, *lx, *ly, *lz, *vinv;
    // per-cell row classes (device coefficient blocks only, see kFaceActive):
    // P bytes stored right after the 7 coefficient blocks
    const uint8_t *flags;
};

template <class T>
__host__ __device__ inline Coefs<T> coefs_of(const T *base, int64_t P) {
    Coefs<T> c;
    c.ax = base; c.ay = base + P; c.az = base + 2 * P;
    c.lx = base + 3 * P; c.ly = base + 4 * P; c.lz = base + 5 * P;
    c.vinv = base + 6 * P;
    c.flags = reinterpret_cast<const uint8_t *>(base + 7 * P);
    return c;
}

// Row classes of the faces of a cell, one byte per cell: bit c (kFaceActive
// << c) is set when face component c is active (a > 0); bit 3 + c
// (kFaceVacuum << c) when every coefficient in the 3^3 block of cells around
// is that of vacuum (a = l = v = 1) and the cell touches no PMC plane.  On a
// vacuum row the curl-curl and grad-div cross terms cancel and M is the
// 7-point Laplacian of the face's own component:
//     (M x)_f = (6 x_f - sum of the 6 same-component neighbours) / h^2 - sigma x_f.
constexpr uint8_t kFaceActive = 1, kFaceVacuum = 8;

// ---------------------------------------------------------------------------
// Stencil rows of M (Sec. 2 eq. farInt for C L C^T, Sec. 5.1 eq. divBInt for
// the grad-div part), without the 1/h^2 factor and without -sigma a x.
// Shared by the GPU kernels and by the host assembly of the coarsest matrix.
// ---------------------------------------------------------------------------

// The vectors may be stored in a narrower type TX than the arithmetic type T
// (FP32 preconditioned vectors in an FP64 product): every loaded value is
// converted to T before any arithmetic, so the result equals that of the
// widened vector.

// flux divergence of cell q (times vinv, no 1/h)
template <class T, class TX = T>
__host__ __device__ inline T cell_div(const Coefs<T> &c, const TX *X, const TX *Y, const TX *Z,
                                      int64_t q, int64_t dy, int64_t dz) {
    return c.vinv[q] * (c.ax[q + 1] * T(X[q + 1]) - c.ax[q] * T(X[q]) + c.ay[q + dy] * T(Y[q + dy]) -
                        c.ay[q] * T(Y[q]) + c.az[q + dz] * T(Z[q + dz]) - c.az[q] * T(Z[q]));
}

template <class T, bool GD, class TX = T>
__host__ __device__ inline T row_x(const Coefs<T> &c, const TX *X, const TX *Y, const TX *Z,
                                   int64_t p, int64_t dy, int64_t dz) {
    const T wy0 = c.ly[p] * (T(X[p]) - T(X[p - dz]) - T(Z[p]) + T(Z[p - 1]));
    const T wyz = c.ly[p + dz] * (T(X[p + dz]) - T(X[p]) - T(Z[p + dz]) + T(Z[p + dz - 1]));
    const T wz0 = c.lz[p] * (T(Y[p]) - T(Y[p - 1]) - T(X[p]) + T(X[p - dy]));
    const T wzy = c.lz[p + dy] * (T(Y[p + dy]) - T(Y[p + dy - 1]) - T(X[p + dy]) + T(X[p]));
    T s = wy0 - wyz + wzy - wz0;
    if (GD) s += c.ax[p] * (cell_div<T, TX>(c, X, Y, Z, p - 1, dy, dz) - cell_div<T, TX>(c, X, Y, Z, p, dy, dz));
    return s;
}

template <class T, bool GD, class TX = T>
__host__ __device__ inline T row_y(const Coefs<T> &c, const TX *X, const TX *Y, const TX *Z,
                                   int64_t p, int64_t dy, int64_t dz) {
    const T wx0 = c.lx[p] * (T(Z[p]) - T(Z[p - dy]) - T(Y[p]) + T(Y[p - dz]));
    const T wxz = c.lx[p + dz] * (T(Z[p + dz]) - T(Z[p + dz - dy]) - T(Y[p + dz]) + T(Y[p]));
    const T wz0 = c.lz[p] * (T(Y[p]) - T(Y[p - 1]) - T(X[p]) + T(X[p - dy]));
    const T wzx = c.lz[p + 1] * (T(Y[p + 1]) - T(Y[p]) - T(X[p + 1]) + T(X[p + 1 - dy]));
    T s = -wx0 + wxz + wz0 - wzx;
    if (GD) s += c.ay[p] * (cell_div<T, TX>(c, X, Y, Z, p - dy, dy, dz) - cell_div<T, TX>(c, X, Y, Z, p, dy, dz));
    return s;
}

template <class T, bool GD, class TX = T>
__host__ __device__ inline T row_z(const Coefs<T> &c, const TX *X, const TX *Y, const TX *Z,
                                   int64_t p, int64_t dy, int64_t dz) {
    const T wx0 = c.lx[p] * (T(Z[p]) - T(Z[p - dy]) - T(Y[p]) + T(Y[p - dz]));
    const T wxy = c.lx[p + dy] * (T(Z[p + dy]) - T(Z[p]) - T(Y[p + dy]) + T(Y[p + dy - dz]));
    const T wy0 = c.ly[p] * (T(X[p]) - T(X[p - dz]) - T(Z[p]) + T(Z[p - 1]));
    const T wyx = c.ly[p + 1] * (T(X[p + 1]) - T(X[p + 1 - dz]) - T(Z[p + 1]) + T(Z[p]));
    T s = wx0 - wxy - wy0 + wyx;
    if (GD) s += c.az[p] * (cell_div<T, TX>(c, X, Y, Z, p - dz, dy, dz) - cell_div<T, TX>(c, X, Y, Z, p, dy, dz));
    return s;
}

// diagonal of M (with 1/h^2 and shift): d/dx_f of the row of face f
template <class T>
__host__ __device__ inline T diag_of(const Coefs<T> &c, int comp, int64_t p, int64_t dy,
                                     int64_t dz, T inv_h2, T sigma) {
    if (comp == 0)
        return inv_h2 * (c.ly[p] + c.ly[p + dz] + c.lz[p] + c.lz[p + dy] +
                         c.ax[p] * c.ax[p] * (c.vinv[p - 1] + c.vinv[p])) - sigma * c.ax[p];
    if (comp == 1)
        return inv_h2 * (c.lx[p] + c.lx[p + dz] + c.lz[p] + c.lz[p + 1] +
                         c.ay[p] * c.ay[p] * (c.vinv[p - dy] + c.vinv[p])) - sigma * c.ay[p];
    return inv_h2 * (c.lx[p] + c.lx[p + dy] + c.ly[p] + c.ly[p + 1] +
                     c.az[p] * c.az[p] * (c.vinv[p - dz] + c.vinv[p])) - sigma * c.az[p];
}

// ---------------------------------------------------------------------------
// Tabulated cut rows of the smoother.  The row of M at a face of component
// c reads 15 stored entries (PMC ghost images counted as entries of their
// own): 7 of its own component (t < kCutOwn) and 4 of each other one, at
// fixed offsets (cut_term).  For every listed cut row the operator stores
// kCutW values, term-major over the component's list: the 15 weights w_t of
// the row of K + G (with 1/h^2), the face's area fraction a, and the
// diagonal d0 of K + G at the face including the PMC self-coupling; a class
// update is
//     x_f += (f_f - sum_t w_t x_t + sigma a x_f) / (d0 - sigma a),
// the same update as from the fractions (the shift stays out of the table).
// ---------------------------------------------------------------------------
constexpr int kCutTerms = 15, kCutW = kCutTerms + 2, kCutOwn = 7;
struct CutTerm {
    int comp, di, dj, dk;
};
__host__ __device__ constexpr CutTerm cut_term(int comp, int t) {
    // own component: the face, its neighbours -z +z -y +y -x +x (reordered
    // per component so that t = 0 is the face itself), then the other two
    // components' four entries each
    return comp == 0 ? (t == 0 ? CutTerm{0, 0, 0, 0} : t == 1 ? CutTerm{0, 0, 0, -1} : t == 2 ? CutTerm{0, 0, 0, 1}
                        : t == 3 ? CutTerm{0, 0, -1, 0} : t == 4 ? CutTerm{0, 0, 1, 0} : t == 5 ? CutTerm{0, -1, 0, 0}
                        : t == 6 ? CutTerm{0, 1, 0, 0} : t == 7 ? CutTerm{1, 0, 0, 0} : t == 8 ? CutTerm{1, -1, 0, 0}
                        : t == 9 ? CutTerm{1, 0, 1, 0} : t == 10 ? CutTerm{1, -1, 1, 0} : t == 11 ? CutTerm{2, 0, 0, 0}
                        : t == 12 ? CutTerm{2, -1, 0, 0} : t == 13 ? CutTerm{2, 0, 0, 1} : CutTerm{2, -1, 0, 1})
         : comp == 1 ? (t == 0 ? CutTerm{1, 0, 0, 0} : t == 1 ? CutTerm{1, 0, 0, -1} : t == 2 ? CutTerm{1, 0, 0, 1}
                        : t == 3 ? CutTerm{1, -1, 0, 0} : t == 4 ? CutTerm{1, 1, 0, 0} : t == 5 ? CutTerm{1, 0, -1, 0}
                        : t == 6 ? CutTerm{1, 0, 1, 0} : t == 7 ? CutTerm{0, 0, 0, 0} : t == 8 ? CutTerm{0, 0, -1, 0}
                        : t == 9 ? CutTerm{0, 1, 0, 0} : t == 10 ? CutTerm{0, 1, -1, 0} : t == 11 ? CutTerm{2, 0, 0, 0}
                        : t == 12 ? CutTerm{2, 0, -1, 0} : t == 13 ? CutTerm{2, 0, 0, 1} : CutTerm{2, 0, -1, 1})
                     : (t == 0 ? CutTerm{2, 0, 0, 0} : t == 1 ? CutTerm{2, 0, -1, 0} : t == 2 ? CutTerm{2, 0, 1, 0}
                        : t == 3 ? CutTerm{2, -1, 0, 0} : t == 4 ? CutTerm{2, 1, 0, 0} : t == 5 ? CutTerm{2, 0, 0, -1}
                        : t == 6 ? CutTerm{2, 0, 0, 1} : t == 7 ? CutTerm{0, 0, 0, 0} : t == 8 ? CutTerm{0, 0, 0, -1}
                        : t == 9 ? CutTerm{0, 1, 0, 0} : t == 10 ? CutTerm{0, 1, 0, -1} : t == 11 ? CutTerm{1, 0, 0, 0}
                        : t == 12 ? CutTerm{1, 0, 0, -1} : t == 13 ? CutTerm{1, 0, 1, 0} : CutTerm{1, 0, 1, -1});
}

// ---------------------------------------------------------------------------
// Batched launches: one launch performs the same V-cycle step for several
// operators (cavities), each its own grid, coefficients and buffers.  A job
// is one operator's share; its work items occupy blocks [block0, block0 +
// its block count) of the launch.  Used only without PMC planes.
// ---------------------------------------------------------------------------
struct BJob {
    Grid g, gc;           // the job's level (and the next coarser one)
    const void *c;        // coefficient base of g (7 blocks + row classes)
    const void *cc;       // coefficient base of gc
    const void *in;       // f (smooth, residual), r (restrict), xc (prolong), f (coarse)
    const void *aux;      // x (residual)
    void *out;            // x (smooth, prolong, zero, coarse), r (residual), fc (restrict)
    const double *inv;    // coarsest dense inverse (coarse)
    const int64_t *idx;   // its active-face index (coarse)
    int64_t items;        // work items of the job
    int ncoarse;          // coarsest active faces (coarse)
    double sigma;
    int64_t block0;
};

enum BatchStep { BS_ZERO = 0, BS_SMOOTH, BS_RESID, BS_RESTRICT, BS_PROLONG, BS_COARSE };

// one batched launch of `step` over `njobs` jobs (device array) covering
// `nblocks` blocks of `tpb` threads (tpb <= 256; the coarse step uses 256)
void launch_batched(int step, int comp, int colour, const BJob *jobs, int njobs, int64_t nblocks, int tpb,
                    hipStream_t s);

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All take a stream; none synchronise.
// ---------------------------------------------------------------------------
enum ApplyKind { AK_M = 0, AK_K = 1, AK_RESID = 2 };

// Block solves: up to kMaxRhs vectors of one level, passed by value as an
// array of device pointers (any subset of a block, no stride assumed).
constexpr int kMaxRhs = 4;
template <class T>
struct VPtr {
    T *p[kMaxRhs];
};
template <class T>
__host__ __device__ inline VPtr<T> vptr1(T *x) {
    VPtr<T> v{};
    v.p[0] = x;
    return v;
}
template <class T>
__host__ __device__ inline VPtr<const T> as_const(const VPtr<T> &x) {
    VPtr<const T> v{};
    for (int q = 0; q < kMaxRhs; ++q) v.p[q] = x.p[q];
    return v;
}

// The non-vacuum (cut) rows of one smoother class as padded indices; with a
// list the class update runs as two parts (see k_smooth_split).
struct ClassList {
    // smoother: the cut rows of one component, both colours, in index order;
    // apply and residual: the cells with a cut row
    const int32_t *idx = nullptr;
    int64_t n = 0;
    // for the smoother's vacuum part: the grid rows (k * ny + j) holding a
    // vacuum row of any component; the colour sweep visits only these
    const int32_t *rows = nullptr;
    int64_t nrows = 0;
    // block smoother: below this many listed rows each vector gets its own
    // wavefront, else one thread per row loops over the vectors
    int64_t wave_split_max = 65536;
    // the tabulated rows of the listed cut rows (kCutW x n, term-major), per
    // precision (see cut_term)
    const double *w64 = nullptr;
    const float *w32 = nullptr;
    // smoother only: how the update of the rows of colour `colour` is paired
    // with the other colour's (the other components do not change between the
    // two colour updates of a component, so the cross-component part of a
    // row is the same in both):
    //   kPairNone   one class update on its own (every term inline);
    //   kPairFirst  the first of the two: this colour's rows take every term,
    //               the other colour's rows store the sum of their
    //               cross-component terms in s (n per vector);
    //   kPairSecond the second: this colour's rows take their own-component
    //               terms and the sum stored in s by the first
    int pair = 0;
    void *s = nullptr;
};
constexpr int kPairNone = 0, kPairFirst = 1, kPairSecond = 2;
template <class T>
inline const T *cut_weights(const ClassList &cl);
template <>
inline const double *cut_weights<double>(const ClassList &cl) { return cl.w64; }
template <>
inline const float *cut_weights<float>(const ClassList &cl) { return cl.w32; }

// Units of kSpanUnit consecutive doubles (one 128-byte line) of a level-0
// face vector that can hold a nonzero entry: an active face, or a PMC ghost
// image of one.  The Krylov reductions and multi-axpys visit only the listed
// units (ascending indices); every vector they read is zero elsewhere and
// what they write is left untouched there.  An empty span means the whole
// vector.
constexpr int kSpanUnit = 16;
struct Span {
    const int32_t *u = nullptr;
    int64_t n = 0;
};

// the block forms of the V-cycle's kernels: nr (1..kMaxRhs) vectors per
// launch, each coefficient loaded once for all of them
// with a cut-cell list (cells with an active non-vacuum row) the launch runs
// as two parts, the listed cells and the vacuum-only rest (M and residual)
template <class T>
void launch_apply_b(const Grid &g, const T *coef, T sigma, int kind, int nr, const VPtr<const T> &f,
                    const VPtr<const T> &x, const VPtr<T> &y, hipStream_t s, ClassList cut = {});
template <class T>
void launch_smooth_b(const Grid &g, const T *coef, T sigma, int comp, int colour, int nr, const VPtr<const T> &f,
                     const VPtr<T> &x, hipStream_t s, ClassList cut = {});
// xz (optional, one coarse iterate per vector): set to zero in the same pass;
// rows (optional): the coarse grid rows (k * ny + j) to visit, those holding
// an active face (fc and xz stay zero on the others)
template <class T>
void launch_restrict_b(const Grid &gf, const Grid &gc, const T *coef_c, int nr, const VPtr<const T> &r,
                       const VPtr<T> &fc, hipStream_t s, const VPtr<T> &xz = {}, const int32_t *rows = nullptr,
                       int64_t nrows = 0);
template <class T>
void launch_prolong_add_b(const Grid &gf, const Grid &gc, const T *coef_f, const T *coef_c, int nr,
                          const VPtr<const T> &xc, const VPtr<T> &x, hipStream_t s, const int32_t *rows = nullptr,
                          int64_t nrows = 0);
template <class T>
void launch_coarse_solve_b(int n, const double *inv, const int64_t *idx, int nr, const VPtr<const T> &f,
                           const VPtr<T> &x, hipStream_t s);

template <class T>
void launch_apply(const Grid &g, const T *coef, T sigma, int kind, const T *f, const T *x, T *y,
                  hipStream_t s, ClassList cut = {});
template <class T>
void launch_smooth(const Grid &g, const T *coef, T sigma, int comp, int colour, const T *f, T *x,
                   hipStream_t s, ClassList cut = {});
template <class T>
void launch_restrict(const Grid &gf, const Grid &gc, const T *coef_c, const T *r, T *fc,
                     hipStream_t s);
template <class T>
void launch_prolong_add(const Grid &gf, const Grid &gc, const T *coef_f, const T *coef_c, const T *xc, T *x,
                        hipStream_t s);
// out = (TO) in; with a span, over its listed units only (out is left
// untouched elsewhere)
template <class TI, class TO>
void launch_cast(const TI *in, TO *out, int64_t n, hipStream_t s, Span sp = {});
template <class T>
void launch_coarse_solve(int n, const double *inv, const int64_t *idx, const T *f, T *x,
                         hipStream_t s);
void launch_apply_A(const Grid &g, const double *coef, const double *x, double *y, hipStream_t s);
template <class T>
void launch_apply_A_t(const Grid &g, const T *coef, const T *x, T *y, hipStream_t s);

// block forms of the scalar-Laplacian kernels (projection), nr = 1..kMaxRhs
void launch_div_DA_b(const Grid &g, const double *coef, int nr, const VPtr<const double> &b,
                     const VPtr<double> &out, hipStream_t s);
void launch_grad_sub_b(const Grid &g, const double *coef, int nr, const VPtr<const double> &psi,
                       const VPtr<const double> &b_in, const VPtr<double> &b_out, double scale, hipStream_t s);
// (FP64, or FP32 with the FP32 coefficient blocks: the preconditioner of the
// projection's conjugate gradients)
// (rows, optional: the grid rows, k * ny + j, to visit -- those holding an
// active cell; y, fc, xz and x stay as they are on the other rows)
template <class T>
void launch_s_apply_b(const Grid &g, const T *coef, double w, int resid, int nr, const VPtr<const T> &f,
                      const VPtr<const T> &x, const VPtr<T> &y, hipStream_t s, const int32_t *rows = nullptr,
                      int64_t nrows = 0);
// (rows: optional list of the grid rows, k * ny + j, holding an active cell;
// the colour sweep then visits only those)
template <class T>
void launch_s_smooth_b(const Grid &g, const T *coef, double w, int colour, int nr, const VPtr<const T> &f,
                       const VPtr<T> &x, hipStream_t s, const int32_t *rows = nullptr, int64_t nrows = 0);
// (xz: optional coarse iterates, set to zero in the same pass)
template <class T>
void launch_s_restrict_b(const Grid &gf, const Grid &gc, const T *coef_c, int nr, const VPtr<const T> &r,
                         const VPtr<T> &fc, hipStream_t s, const VPtr<T> &xz = {}, const int32_t *rows = nullptr,
                         int64_t nrows = 0);
template <class T>
void launch_s_prolong_add_b(const Grid &gf, const Grid &gc, const T *coef_f, int nr, const VPtr<const T> &xc,
                            const VPtr<T> &x, hipStream_t s, const int32_t *rows = nullptr, int64_t nrows = 0);

// PMC ghost layers of a face / cell vector from the adjacent values (no-op
// without PMC planes)
template <class T>
void launch_mirror_faces(const Grid &g, T *x, hipStream_t s);
template <class T>
void launch_mirror_cells(const Grid &g, T *x, hipStream_t s);

// scalar (cell-centred) Laplacian S = D A D^T with per-level weight `w`
void launch_div_DA(const Grid &g, const double *coef, const double *b, double *gout,
                   hipStream_t s);
void launch_grad_sub(const Grid &g, const double *coef, const double *psi, double *b_in,
                     double *b_out, double scale, hipStream_t s);
void launch_s_apply(const Grid &g, const double *coef, double w, int resid, const double *f,
                    const double *x, double *y, hipStream_t s);
void launch_s_smooth(const Grid &g, const double *coef, double w, int colour, const double *f,
                     double *x, hipStream_t s);
void launch_s_restrict(const Grid &gf, const Grid &gc, const double *coef_c, const double *r,
                       double *fc, hipStream_t s);
void launch_s_prolong_add(const Grid &gf, const Grid &gc, const double *coef_f,
                          const double *xc, double *x, hipStream_t s);

// BLAS-1 style FP64 helpers on flat arrays
void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s);
// y = M x (FP64 arithmetic and output) for FP32-stored x: each value of x is
// widened before use, so y equals the product with the widened x; takes the
// cut-cell list of the level (the split form), and with its rows leaves y
// untouched on the other rows
void launch_apply_m_f32in(const Grid &g, const double *coef, double sigma, int nr, const VPtr<const float> &x,
                          const VPtr<double> &y, hipStream_t s, ClassList cut);
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
void launch_scale(int64_t n, double a, double *x, hipStream_t s);
template <class T>
void launch_zero(int64_t n, T *x, hipStream_t s);
void launch_copy(int64_t n, const double *x, double *y, hipStream_t s);
// out[i] = sum_n V_i[n] w[n] (wt[n]) for i < nv; V_i = V + i*ld; results left in
// device buffer `dout` (nv doubles); `part` scratch of nv * kReduceBlocks doubles
constexpr int kReduceBlocks = 1024;
void launch_mdot(int nv, const double *V, int64_t ld, const double *w, const double *wt,
                 int64_t n, double *part, double *dout, hipStream_t s, Span sp = {});
// the same with an FP32 basis (each value widened; FP64 sums)
void launch_mdot(int nv, const float *V, int64_t ld, const double *w, const double *wt, int64_t n, double *part,
                 double *dout, hipStream_t s, Span sp = {});
constexpr int kMultiMax = 8;   // vectors per launch of the two kernels below
// dout[i*nw + q] = V_i . (W_q * wt) for i < nv, q < nw (nw <= 8, nv*nw <= 256;
// W_q = W + q*ldw); the basis is read once
void launch_mdot_multi(int nv, const double *V, int64_t ld, const double *W, int64_t ldw, int nw,
                       const double *wt, int64_t n, double *part, double *dout, hipStream_t s, Span sp = {});
// Y_q = sum_i C[i*nw + q] V_i (overwrite) or Y_q -= ... for q < nw (nw <= 8;
// C on device; Y_q = Y + q*ldy); the basis is read once
void launch_maxpy_multi(int nv, const double *V, int64_t ld, const double *C, int nw, double *Y, int64_t ldy,
                        int64_t n, int overwrite, hipStream_t s, Span sp = {});
// y -= sum_i c[i] V_i  (c on device)  or  y = sum_i c[i] V_i when overwrite;
// with cscale (device, nv values) the coefficients are c[i] * cscale[i]
void launch_maxpy(int nv, const double *V, int64_t ld, const double *c, double *y, int64_t n,
                  int overwrite, hipStream_t s, const double *cscale = nullptr, Span sp = {});
// the same with an FP32 basis (each value widened; FP64 arithmetic)
void launch_maxpy(int nv, const float *V, int64_t ld, const double *c, double *y, int64_t n, int overwrite,
                  hipStream_t s, const double *cscale = nullptr, Span sp = {});
// y -= sum_i c[i] V_i for FP32 columns V_i (c on device; FP64 arithmetic)
void launch_maxpy_f32(int nv, const float *V, int64_t ld, const double *c, double *y, int64_t n, hipStream_t s,
                      Span sp = {});
// fused Gram--Schmidt step: w -= sum c_i V_i (c_i times cscale_i if given),
// then dout[0..nv-1] = V_i . w and dout[nv] = |w|^2 (device results); one
// pass over the basis for nv <= 32, two above
void launch_maxpy_mdot_norm(int nv, const double *V, int64_t ld, const double *c, double *w,
                            int64_t n, double *part, double *dout, hipStream_t s, const double *cscale = nullptr,
                            Span sp = {});
// the same with an FP32 basis (each value widened; FP64 arithmetic)
void launch_maxpy_mdot_norm(int nv, const float *V, int64_t ld, const double *c, double *w, int64_t n,
                            double *part, double *dout, hipStream_t s, const double *cscale = nullptr,
                            Span sp = {});
// out = scale * (w - sum c_i V_i)
void launch_maxpy_scale(int nv, const double *V, int64_t ld, const double *c, const double *w,
                        double scale, double *out, int64_t n, hipStream_t s);
// Per-vector scalars of a block launch, passed by value
struct Coef4 {
    double v[kMaxRhs] = {};
};
// Block forms for the conjugate-gradient solves of the projection; each acts
// on the vector slots q < nr whose first pointer is set, results to
// dout[q * dstride] (device), `part` scratch of kMaxRhs * kReduceBlocks doubles:
//   dot_pairs: dout[q] = X_q . (Y_q * wt)     (wt optional, read once)
//   cg_update: psi_q += a_q p_q, r_q -= a_q q_q, dout[q] = r_q . (r_q * wt)
//   xpby_b:    Y_q = X_q + b_q Y_q
//   sub_masked_b: X_q -= scale * val[q * stride] where mask != 0
// The first three visit only the listed units of sp (the whole vectors
// without a list): every vector they read is zero outside those units, and
// what they write is left untouched there.
void launch_dot_pairs(int nr, const VPtr<const double> &X, const VPtr<const double> &Y, const double *wt,
                      int64_t n, double *part, double *dout, int64_t dstride, hipStream_t s, Span sp = {});
void launch_cg_update(int nr, const VPtr<const double> &Pv, const VPtr<const double> &Qv, const VPtr<double> &Psi,
                      const VPtr<double> &R, const Coef4 &a, const double *wt, int64_t n, double *part, double *dout,
                      int64_t dstride, hipStream_t s, Span sp = {});
void launch_xpby_b(int nr, const VPtr<const double> &X, const Coef4 &b, const VPtr<double> &Y, int64_t n,
                   hipStream_t s, Span sp = {});
void launch_sub_masked_b(int nr, int64_t n, const double *mask, const double *val, int64_t stride, double scale,
                         const VPtr<double> &X, hipStream_t s);
// masked shift: x[n] -= scale * val[0] where mask[n] != 0 (val on device)
void launch_sub_masked(int64_t n, const double *mask, const double *val, double scale, double *x,
                       hipStream_t s);
void launch_randn(int64_t n, uint64_t seed, int64_t offset, const double *mask, double *x,
                  hipStream_t s);
void launch_mask_mul(int64_t n, const double *mask, double *x, hipStream_t s);
// x = in on the mask's nonzero entries, 0 elsewhere
void launch_copy_masked(int64_t n, const double *in, const double *mask, double *x, hipStream_t s);
// e = C^T b / k at npts points (device arrays pts: 3 per point, out: 3 per point)
void launch_sample_e(const Grid &g, const double *coef, const double *b, double k, int npts, const double *pts,
                     double *out, hipStream_t s);
// tilde-form transfers: x *= a^(power/2) per face (coef: the level's
// coefficient blocks, whose first 3P entries are ax ay az); x += a^(-1/2) r
template <class T>
void launch_scale_a(int64_t n, const T *coef, int power, T *x, hipStream_t s);
template <class T>
void launch_add_scaled_a(int64_t n, const T *coef, const T *r, T *x, hipStream_t s);

}  // namespace dm
