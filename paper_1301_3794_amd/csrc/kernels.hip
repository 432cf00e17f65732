// HIP kernels of the Dey--Mittra eigensolver (gfx950, wave64).
//
// Stencil kernels map one thread to one cell (i,j,k); the cell owns its three
// low faces b_x[i,j,k], b_y[i,j,k], b_z[i,j,k].  Blocks are remapped so that
// each of the 8 XCDs (which receive workgroups round-robin) works on one
// contiguous slab of the grid and keeps its stencil neighbours in its own L2.
// The stencil path is memory bound: no MFMA here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <type_traits>

#include "dm_internal.h"

namespace dm {

namespace {

constexpr int kThreads = 256;
constexpr int kXcd = 8;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// grid of `n` work items in blocks of kThreads, padded to a multiple of 8 blocks
inline dim3 xcd_grid(int64_t n) {
    int64_t nb = ceil_div(n, kThreads);
    int64_t per = ceil_div(nb, kXcd);
    return dim3((unsigned)(per * kXcd));
}

// logical block of this workgroup: XCD x gets blocks [x*per, (x+1)*per)
__device__ inline int64_t xcd_item() {
    const int64_t per = gridDim.x / kXcd;
    const int64_t b = blockIdx.x;
    const int64_t logical = (b % kXcd) * per + b / kXcd;
    return logical * kThreads + threadIdx.x;
}

// Block kernels over nr vectors: a workgroup of 64 * nr threads takes 64
// consecutive items, wave q the vector q (coalesced loads per wave; the waves
// of a workgroup share the coefficient lines of their cells in the CU's
// cache).  Grid: ceil(items / 64) workgroups, padded to a multiple of 8.
inline dim3 xcd_grid_waves(int64_t items) {
    int64_t nb = ceil_div(items, 64);
    int64_t per = ceil_div(nb, kXcd);
    return dim3((unsigned)(per * kXcd));
}

__device__ inline int64_t wave_item(int &q) {
    const int64_t per = gridDim.x / kXcd;
    const int64_t b = blockIdx.x;
    const int64_t logical = (b % kXcd) * per + b / kXcd;
    q = threadIdx.x >> 6;
    return logical * 64 + (threadIdx.x & 63);
}

__device__ inline bool cell_of(const Grid &g, int64_t t, int &i, int &j, int &k) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    if (t >= n) return false;
    i = (int)(t % g.nx);
    const int64_t r = t / g.nx;
    j = (int)(r % g.ny);
    k = (int)(r / g.ny);
    return true;
}

// Item t of a launch over listed grid rows (k * ny + j, ascending) -> the
// cell item of the whole grid (past its end for t past the listed rows);
// without a list the item itself
__device__ inline int64_t listed_item(const Grid &g, const int32_t *rows, int64_t nrows, int64_t t) {
    if (!rows) return t;
    if (t >= nrows * g.nx) return (int64_t)g.nx * g.ny * g.nz;
    return (int64_t)rows[t / g.nx] * g.nx + t % g.nx;
}

template <class T>
__device__ inline T inv_h2_of(const Grid &g) {
    return (T)(1.0 / (g.h * g.h));
}

// ---------------------------------------------------------------------------
// y = M x, y = K x, or r = f - M x
// ---------------------------------------------------------------------------
// 7-point vacuum row of component array C at p (no 1/h^2)
template <class T, class TX = T>
__device__ inline T vac_row(const TX *C, int64_t p, int64_t dy, int64_t dz) {
    return T(6) * T(C[p]) - (T(C[p - 1]) + T(C[p + 1])) - (T(C[p - dy]) + T(C[p + dy])) -
           (T(C[p - dz]) + T(C[p + dz]));
}

// NR right-hand sides at once (block solves): the coefficients of a row are
// loaded once and serve every vector; all rows are formed before any store.
template <class T, int KIND, class TX = T>
__device__ __forceinline__ void apply_body(const Grid &g, const Coefs<T> &c, T sigma, const T *__restrict__ f,
                                           const TX *__restrict__ x, T *__restrict__ y, int64_t item) {
    int i, j, k;
    if (!cell_of(g, item, i, j, k)) return;
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    const int64_t p = pidx(g, i, j, k);
    const TX *X = x, *Y = x + P, *Z = x + 2 * P;
    const T ih2 = inv_h2_of<T>(g);
    const uint8_t fl = c.flags[p];
    T yx = T(0), yy = T(0), yz = T(0);
    if (KIND == AK_K) {
        if (fl & (kFaceActive << 0)) yx = ih2 * row_x<T, false, TX>(c, X, Y, Z, p, dy, dz);
        if (fl & (kFaceActive << 1)) yy = ih2 * row_y<T, false, TX>(c, X, Y, Z, p, dy, dz);
        if (fl & (kFaceActive << 2)) yz = ih2 * row_z<T, false, TX>(c, X, Y, Z, p, dy, dz);
    } else {
        if (fl & (kFaceActive << 0)) {
            yx = (fl & (kFaceVacuum << 0))
                     ? ih2 * vac_row<T, TX>(X, p, dy, dz) - sigma * T(X[p])
                     : ih2 * row_x<T, true, TX>(c, X, Y, Z, p, dy, dz) - sigma * c.ax[p] * T(X[p]);
            if (KIND == AK_RESID) yx = f[p] - yx;
        }
        if (fl & (kFaceActive << 1)) {
            yy = (fl & (kFaceVacuum << 1))
                     ? ih2 * vac_row<T, TX>(Y, p, dy, dz) - sigma * T(Y[p])
                     : ih2 * row_y<T, true, TX>(c, X, Y, Z, p, dy, dz) - sigma * c.ay[p] * T(Y[p]);
            if (KIND == AK_RESID) yy = f[P + p] - yy;
        }
        if (fl & (kFaceActive << 2)) {
            yz = (fl & (kFaceVacuum << 2))
                     ? ih2 * vac_row<T, TX>(Z, p, dy, dz) - sigma * T(Z[p])
                     : ih2 * row_z<T, true, TX>(c, X, Y, Z, p, dy, dz) - sigma * c.az[p] * T(Z[p]);
            if (KIND == AK_RESID) yz = f[2 * P + p] - yz;
        }
    }
    put_face<T>(g, y, 0, i, j, k, p, yx);
    put_face<T>(g, y + P, 1, i, j, k, p, yy);
    put_face<T>(g, y + 2 * P, 2, i, j, k, p, yz);
}

// apply_body of M or the residual for the cells whose active rows are all
// vacuum rows (the other cells are listed and run the full body): the same
// values, written the same way, zeros on the inactive components included.
// (K alone has no vacuum shortcut: its rows keep the cross terms.)
template <class T, int KIND, class TX = T>
__device__ __forceinline__ void apply_vac_body(const Grid &g, T sigma, uint8_t fl, const T *__restrict__ f,
                                               const TX *__restrict__ x, T *__restrict__ y, int i, int j, int k,
                                               int64_t p) {
    static_assert(KIND == AK_M || KIND == AK_RESID, "vacuum rows of M only");
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    const T ih2 = inv_h2_of<T>(g);
    T v[3];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const TX *C = x + comp * P;
        v[comp] = T(0);
        if (fl & (kFaceActive << comp)) {
            v[comp] = ih2 * vac_row<T, TX>(C, p, dy, dz) - sigma * T(C[p]);
            if (KIND == AK_RESID) v[comp] = f[comp * P + p] - v[comp];
        }
    }
    put_face<T>(g, y, 0, i, j, k, p, v[0]);
    put_face<T>(g, y + P, 1, i, j, k, p, v[1]);
    put_face<T>(g, y + 2 * P, 2, i, j, k, p, v[2]);
}

// cells with an active non-vacuum row (those in the cut-cell list)
__device__ inline bool has_cut_row(uint8_t fl) {
    return ((fl & 7) & ~(fl >> 3)) != 0;
}

template <class T, int KIND>
__global__ void __launch_bounds__(kThreads)
k_apply(Grid g, Coefs<T> c, T sigma, const T *__restrict__ f, const T *__restrict__ x,
        T *__restrict__ y) {
    apply_body<T, KIND>(g, c, sigma, f, x, y, xcd_item());
}

// Block forms of apply, restriction and prolongation: wave q of a workgroup
// applies the one-vector body to vector q of the workgroup's 64 cells (see
// wave_item), so every lane keeps the register budget of the one-vector
// body.  (Looping over the vectors inside a thread kept every vector's loads
// and addresses live at once: 170-240 VGPRs, two waves per SIMD; giving the
// vectors to neighbouring lanes split every load of a wave over NR arrays.)

template <class T, int KIND, int NR>
__global__ void __launch_bounds__(kThreads)
k_apply_b(Grid g, Coefs<T> c, T sigma, VPtr<const T> f, VPtr<const T> x, VPtr<T> y) {
    int q;
    const int64_t t = wave_item(q);
    apply_body<T, KIND>(g, c, sigma, f.p[q], x.p[q], y.p[q], t);
}

// The block apply in two parts, as the smoother's class updates: the first
// ncb workgroups (a multiple of 8) take the cut-cell list (full body), the
// rest all cells, skipping listed ones (vacuum rows only); wave q of a
// workgroup takes vector q of 64 entries in either part.
// M x or f - M x at listed cell e (padded index p) from the cell's tabulated
// rows W (3 x kCutW x ncut; see cut_term); inactive faces (a = 0) get 0
template <class T, int KIND, class TX>
__device__ __forceinline__ void apply_cut_tab(const Grid &g, T sigma, const T *__restrict__ W, int64_t ncut,
                                              int64_t e, int64_t p, const T *__restrict__ f,
                                              const TX *__restrict__ x, T *__restrict__ y) {
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    T v[3];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const T *Wc = W + (int64_t)comp * kCutW * ncut;
        const T a = Wc[kCutTerms * ncut + e];
        v[comp] = T(0);
        if (a != T(0)) {
            T row = -sigma * a * T(x[comp * P + p]);
#pragma unroll
            for (int t = 0; t < kCutTerms; ++t) {
                const CutTerm ct = cut_term(comp, t);
                row += Wc[t * ncut + e] * T(x[ct.comp * P + p + ct.di + ct.dj * dy + ct.dk * dz]);
            }
            v[comp] = KIND == AK_RESID ? f[comp * P + p] - row : row;
        }
    }
    const int64_t kk = p / dz, rr = p - kk * dz, jj = rr / dy;
    const int i = (int)(rr - jj * dy) - 1, j = (int)jj - 1, k = (int)kk - 1;
    put_face<T>(g, y, 0, i, j, k, p, v[0]);
    put_face<T>(g, y + P, 1, i, j, k, p, v[1]);
    put_face<T>(g, y + 2 * P, 2, i, j, k, p, v[2]);
}

template <class T, int KIND, int NR, class TX = T>
__global__ void __launch_bounds__(kThreads)
k_apply_split(Grid g, Coefs<T> c, T sigma, const int32_t *__restrict__ cut, int64_t ncut, int64_t ncb,
              const T *__restrict__ W, const int32_t *__restrict__ rows, int64_t nrows, VPtr<const T> f,
              VPtr<const TX> x, VPtr<T> y) {
    const int64_t b = blockIdx.x;
    const int q = threadIdx.x >> 6;
    if (b < ncb) {
        const int64_t e = ((b % kXcd) * (ncb / kXcd) + b / kXcd) * 64 + (threadIdx.x & 63);
        if (e >= ncut) return;
        apply_cut_tab<T, KIND, TX>(g, sigma, W, ncut, e, cut[e], f.p[q], x.p[q], y.p[q]);
    } else {
        const int64_t bv = b - ncb, nvb = (int64_t)gridDim.x - ncb;
        const int64_t t = ((bv % kXcd) * (nvb / kXcd) + bv / kXcd) * 64 + (threadIdx.x & 63);
        int i, j, k;
        if (!cell_of(g, listed_item(g, rows, nrows, t), i, j, k)) return;
        const int64_t p = pidx(g, i, j, k);
        const uint8_t fl = c.flags[p];
        if (has_cut_row(fl)) return;
        apply_vac_body<T, KIND, TX>(g, sigma, fl, f.p[q], x.p[q], y.p[q], i, j, k, p);
    }
}

// y = A x
template <class T>
__global__ void __launch_bounds__(kThreads)
k_apply_A(Grid g, Coefs<T> c, const T *__restrict__ x, T *__restrict__ y) {
    int i, j, k;
    if (!cell_of(g, xcd_item(), i, j, k)) return;
    const int64_t P = g.P, p = pidx(g, i, j, k);
    put_face<T>(g, y, 0, i, j, k, p, c.ax[p] * x[p]);
    put_face<T>(g, y + P, 1, i, j, k, p, c.ay[p] * x[P + p]);
    put_face<T>(g, y + 2 * P, 2, i, j, k, p, c.az[p] * x[2 * P + p]);
}

// ---------------------------------------------------------------------------
// Red-black Gauss--Seidel: one (component, colour) class, colour = (i+j+k)&1.
// Threads cover half the cells of each row: i = 2*ih + ((j+k+colour)&1).
// A thread also refreshes the PMC ghost images of the value it updates; no
// row of the same class reads those images except its own.
// ---------------------------------------------------------------------------
template <class T, int COMP, int NR>
__device__ __forceinline__ void smooth_body_n(const Grid &g, const Coefs<T> &c, T sigma, int colour,
                                              const VPtr<const T> &f, const VPtr<T> &x, int64_t t) {
    const int nxh = (g.nx + 1) >> 1;
    if (t >= (int64_t)nxh * g.ny * g.nz) return;
    const int ih = (int)(t % nxh);
    const int64_t r = t / nxh;
    const int j = (int)(r % g.ny), k = (int)(r / g.ny);
    const int i = 2 * ih + ((j + k + colour) & 1);
    if (i >= g.nx) return;
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    const int64_t p = pidx(g, i, j, k);
    const T ih2 = inv_h2_of<T>(g);
    const uint8_t fl = c.flags[p];
    if (!(fl & (kFaceActive << COMP))) return;
    T nv[NR];
    if (fl & (kFaceVacuum << COMP)) {
        const T d = T(6) * ih2 - sigma;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const T *xc = x.p[q] + COMP * P;
            const T xp = xc[p];
            const T row = ih2 * vac_row<T>(xc, p, dy, dz) - sigma * xp;
            nv[q] = xp + (f.p[q][COMP * P + p] - row) / d;
        }
    } else {
        const T *a = COMP == 0 ? c.ax : (COMP == 1 ? c.ay : c.az);
        const T d = diag_of<T>(c, COMP, p, dy, dz, ih2, sigma) +
                    ih2 * pmc_diag_extra<T>(g, c.lx, c.ly, c.lz, COMP, i, j, k, p);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const T *X = x.p[q], *Y = X + P, *Z = X + 2 * P;
            const T *xc = COMP == 0 ? X : (COMP == 1 ? Y : Z);
            T row;
            if (COMP == 0) row = row_x<T, true>(c, X, Y, Z, p, dy, dz);
            else if (COMP == 1) row = row_y<T, true>(c, X, Y, Z, p, dy, dz);
            else row = row_z<T, true>(c, X, Y, Z, p, dy, dz);
            row = ih2 * row - sigma * a[p] * xc[p];
            nv[q] = xc[p] + (f.p[q][COMP * P + p] - row) / d;
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) put_face<T>(g, x.p[q] + COMP * P, COMP, i, j, k, p, nv[q]);
}

// The two parts of a class update when the class's cut rows are listed:
// smooth_vac_n updates the vacuum rows of the colour sweep and skips every
// other row; smooth_cut_n updates entry e of the list of the class's
// non-vacuum rows.  Rows of one class do not read each other, so the parts
// may run in any order; separating them keeps the waves of the colour sweep
// on the short vacuum path (a cut row in a wave made the whole wave take
// the long path as well).
template <class T, int COMP, int NR>
__device__ __forceinline__ void smooth_vac_n(const Grid &g, const Coefs<T> &c, T sigma, int colour,
                                             const VPtr<const T> &f, const VPtr<T> &x, int64_t t,
                                             const int32_t *__restrict__ rows, int64_t nrows) {
    const int nxh = (g.nx + 1) >> 1;
    if (t >= (rows ? nrows : (int64_t)g.ny * g.nz) * nxh) return;
    const int ih = (int)(t % nxh);
    const int64_t r = rows ? (int64_t)rows[t / nxh] : t / nxh;
    const int j = (int)(r % g.ny), k = (int)(r / g.ny);
    const int i = 2 * ih + ((j + k + colour) & 1);
    if (i >= g.nx) return;
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    const int64_t p = pidx(g, i, j, k);
    if (!(c.flags[p] & (kFaceVacuum << COMP))) return;
    const T ih2 = inv_h2_of<T>(g);
    const T d = T(6) * ih2 - sigma;
    T nv[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const T *xc = x.p[q] + COMP * P;
        const T xp = xc[p];
        const T row = ih2 * vac_row<T>(xc, p, dy, dz) - sigma * xp;
        nv[q] = xp + (f.p[q][COMP * P + p] - row) / d;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) put_face<T>(g, x.p[q] + COMP * P, COMP, i, j, k, p, nv[q]);
}

// entry e of the component's cut list (both colours, index order) from its
// tabulated row W (kCutW x ncut, term-major; see cut_term), for the update of
// colour `colour` paired as `pair` says (see ClassList): the row is
// -sigma a x_f + (own-component terms) + (cross-component terms), the latter
// summed first, inline or taken from S (ncut per vector, vector q0 + q);
// the weights are loaded once for the NR vectors
template <class T, int COMP, int NR>
__device__ __forceinline__ void smooth_cut_n(const Grid &g, T sigma, const int32_t *__restrict__ cut, int64_t ncut,
                                             const T *__restrict__ W, int colour, int pair, T *__restrict__ S,
                                             int q0, const VPtr<const T> &f, const VPtr<T> &x, int64_t e) {
    if (e >= ncut) return;
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    const int64_t p = cut[e];
    const int64_t kk = p / dz, rr = p - kk * dz, jj = rr / dy;
    const int i = (int)(rr - jj * dy) - 1, j = (int)jj - 1, k = (int)kk - 1;
    const bool mine = ((i + j + k) & 1) == colour;
    // the other colour's rows: nothing, or (first of a pair) their cross sums
    if (!mine && pair != kPairFirst) return;
    T cross[NR];
    if (pair == kPairSecond) {
#pragma unroll
        for (int q = 0; q < NR; ++q) cross[q] = S[(int64_t)(q0 + q) * ncut + e];
    } else {
        T w[kCutTerms - kCutOwn];
#pragma unroll
        for (int t = kCutOwn; t < kCutTerms; ++t) w[t - kCutOwn] = W[t * ncut + e];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const T *X = x.p[q];
            T c = T(0);
#pragma unroll
            for (int t = kCutOwn; t < kCutTerms; ++t) {
                const CutTerm ct = cut_term(COMP, t);
                c += w[t - kCutOwn] * X[ct.comp * P + p + ct.di + ct.dj * dy + ct.dk * dz];
            }
            cross[q] = c;
        }
        if (!mine) {
#pragma unroll
            for (int q = 0; q < NR; ++q) S[(int64_t)(q0 + q) * ncut + e] = cross[q];
            return;
        }
    }
    T w[kCutOwn];
#pragma unroll
    for (int t = 0; t < kCutOwn; ++t) w[t] = W[t * ncut + e];
    const T a = W[kCutTerms * ncut + e];
    const T d = W[(kCutTerms + 1) * ncut + e] - sigma * a;
    T nv[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const T *X = x.p[q];
        const T xs = X[COMP * P + p];
        T row = -sigma * a * xs;
#pragma unroll
        for (int t = 0; t < kCutOwn; ++t) {
            const CutTerm ct = cut_term(COMP, t);
            row += w[t] * X[ct.comp * P + p + ct.di + ct.dj * dy + ct.dk * dz];
        }
        row += cross[q];
        nv[q] = xs + (f.p[q][COMP * P + p] - row) / d;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) put_face<T>(g, x.p[q] + COMP * P, COMP, i, j, k, p, nv[q]);
}

template <class T, int COMP>
__device__ __forceinline__ void smooth_body(const Grid &g, const Coefs<T> &c, T sigma, int colour,
                                            const T *__restrict__ f, T *__restrict__ x, int64_t t) {
    smooth_body_n<T, COMP, 1>(g, c, sigma, colour, vptr1(f), vptr1(x), t);
}

template <class T, int COMP>
__global__ void __launch_bounds__(kThreads)
k_smooth(Grid g, Coefs<T> c, T sigma, int colour, const T *__restrict__ f, T *__restrict__ x) {
    smooth_body<T, COMP>(g, c, sigma, colour, f, x, xcd_item());
}

template <class T, int COMP, int NR>
__global__ void __launch_bounds__(kThreads)
k_smooth_b(Grid g, Coefs<T> c, T sigma, int colour, VPtr<const T> f, VPtr<T> x) {
    smooth_body_n<T, COMP, NR>(g, c, sigma, colour, f, x, xcd_item());
}

// A class update from its two parts: the first ncb workgroups (a multiple of
// 8) take the cut-row list, the rest the vacuum rows of the colour sweep;
// each part maps its workgroups to the XCDs as xcd_item does.  With several
// vectors and a short list (wave_split) a cut workgroup takes 64 rows, wave
// q the vector q: the cut rows are latency-bound, and one thread per row and
// vector keeps more of them in flight (the waves share the rows' coefficient
// lines in cache); a long list fills the GPU with one thread per row looping
// over the vectors, which reuses the coefficients in registers.
template <class T, int COMP, int NR>
__global__ void __launch_bounds__(kThreads)
k_smooth_split(Grid g, Coefs<T> c, T sigma, int colour, const int32_t *__restrict__ cut, int64_t ncut, int64_t ncb,
               int wave_split, const T *__restrict__ W, int pair, T *__restrict__ S,
               const int32_t *__restrict__ rows, int64_t nrows, VPtr<const T> f, VPtr<T> x) {
    const int64_t b = blockIdx.x;
    if (b < ncb) {
        const int64_t L = (b % kXcd) * (ncb / kXcd) + b / kXcd;
        if (!wave_split) {
            smooth_cut_n<T, COMP, NR>(g, sigma, cut, ncut, W, colour, pair, S, 0, f, x, L * kThreads + threadIdx.x);
        } else {
            const int q = threadIdx.x >> 6;
            if (q >= NR) return;
            smooth_cut_n<T, COMP, 1>(g, sigma, cut, ncut, W, colour, pair, S, q, vptr1(f.p[q]), vptr1(x.p[q]),
                                     L * 64 + (threadIdx.x & 63));
        }
    } else {
        const int64_t bv = b - ncb, nvb = (int64_t)gridDim.x - ncb;
        const int64_t L = (bv % kXcd) * (nvb / kXcd) + bv / kXcd;
        smooth_vac_n<T, COMP, NR>(g, c, sigma, colour, f, x, L * kThreads + threadIdx.x, rows, nrows);
    }
}

// ---------------------------------------------------------------------------
// Staggered transfers.  P: linear along the normal, constant across; R = P^T/8.
// ---------------------------------------------------------------------------
template <class T>
// xz (optional): the coarse iterate, set to zero on the cell's faces (and
// their PMC ghost images) in the same pass, as the coarse V-cycle starts
// from zero
__device__ __forceinline__ void restrict_body(const Grid &gf, const Grid &gc, const Coefs<T> &cc,
                                              const T *__restrict__ r, T *__restrict__ fc, int64_t item,
                                              T *__restrict__ xz = nullptr) {
    int I, J, K;
    if (!cell_of(gc, item, I, J, K)) return;
    const int64_t Pf = gf.P, Pc = gc.P, fy = gf.sy, fz = gf.sz;
    const int64_t pc = pidx(gc, I, J, K);
    const T *RX = r, *RY = r + Pf, *RZ = r + 2 * Pf;
    const int64_t q = pidx(gf, 2 * I, 2 * J, 2 * K);
    // transpose of the area-weighted normal interpolation: the fine face
    // between coarse faces c and c' gives c the share a_c / (a_c + a_c')
    const T ax = cc.ax[pc], ay = cc.ay[pc], az = cc.az[pc];
    const T xm = ax > T(0) ? ax / (ax + cc.ax[pc - 1]) : T(0);
    const T xp = ax > T(0) ? ax / (ax + cc.ax[pc + 1]) : T(0);
    const T ym = ay > T(0) ? ay / (ay + cc.ay[pc - gc.sy]) : T(0);
    const T yp = ay > T(0) ? ay / (ay + cc.ay[pc + gc.sy]) : T(0);
    const T zm = az > T(0) ? az / (az + cc.az[pc - gc.sz]) : T(0);
    const T zp = az > T(0) ? az / (az + cc.az[pc + gc.sz]) : T(0);
    T sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            // x: tangential offsets in y (a) and z (b)
            const int64_t qx = q + a * fy + b * fz;
            sx += RX[qx] + xm * RX[qx - 1] + xp * RX[qx + 1];
            const int64_t qy = q + a + b * fz;
            sy += RY[qy] + ym * RY[qy - fy] + yp * RY[qy + fy];
            const int64_t qz = q + a + b * fy;
            sz += RZ[qz] + zm * RZ[qz - fz] + zp * RZ[qz + fz];
        }
    const T e = T(0.125);
    put_face<T>(gc, fc, 0, I, J, K, pc, ax != T(0) ? e * sx : T(0));
    put_face<T>(gc, fc + Pc, 1, I, J, K, pc, ay != T(0) ? e * sy : T(0));
    put_face<T>(gc, fc + 2 * Pc, 2, I, J, K, pc, az != T(0) ? e * sz : T(0));
    if (xz) {
        put_face<T>(gc, xz, 0, I, J, K, pc, T(0));
        put_face<T>(gc, xz + Pc, 1, I, J, K, pc, T(0));
        put_face<T>(gc, xz + 2 * Pc, 2, I, J, K, pc, T(0));
    }
}

template <class T>
__global__ void __launch_bounds__(kThreads)
k_restrict(Grid gf, Grid gc, Coefs<T> cc, const T *__restrict__ r, T *__restrict__ fc) {
    restrict_body<T>(gf, gc, cc, r, fc, xcd_item());
}

template <class T, int NR>
__global__ void __launch_bounds__(kThreads)
k_restrict_b(Grid gf, Grid gc, Coefs<T> cc, const int32_t *__restrict__ rows, int64_t nrows, VPtr<const T> r,
             VPtr<T> fc, VPtr<T> xz) {
    int q;
    const int64_t t = wave_item(q);
    restrict_body<T>(gf, gc, cc, r.p[q], fc.p[q], listed_item(gc, rows, nrows, t), xz.p[q]);
}

// fine value between coarse faces c0, c1: (a0 x0 + a1 x1) / (a0 + a1)
template <class T>
__device__ __forceinline__ T wmean(T a0, T x0, T a1, T x1) {
    const T t = a0 + a1;
    return t > T(0) ? (a0 * x0 + a1 * x1) / t : T(0);
}

template <class T>
__device__ __forceinline__ void prolong_body(const Grid &gf, const Grid &gc, const Coefs<T> &cf, const Coefs<T> &cc,
                                             const T *__restrict__ xc, T *__restrict__ x, int64_t item) {
    int i, j, k;
    if (!cell_of(gf, item, i, j, k)) return;
    const int64_t Pf = gf.P, Pc = gc.P, cy = gc.sy, cz = gc.sz;
    const int64_t p = pidx(gf, i, j, k);
    const int64_t q = pidx(gc, i >> 1, j >> 1, k >> 1);
    const T *CX = xc, *CY = xc + Pc, *CZ = xc + 2 * Pc;
    if (cf.ax[p] != T(0))
        put_face<T>(gf, x, 0, i, j, k, p,
                    x[p] + ((i & 1) ? wmean(cc.ax[q], CX[q], cc.ax[q + 1], CX[q + 1]) : CX[q]));
    if (cf.ay[p] != T(0))
        put_face<T>(gf, x + Pf, 1, i, j, k, p,
                    x[Pf + p] + ((j & 1) ? wmean(cc.ay[q], CY[q], cc.ay[q + cy], CY[q + cy]) : CY[q]));
    if (cf.az[p] != T(0))
        put_face<T>(gf, x + 2 * Pf, 2, i, j, k, p,
                    x[2 * Pf + p] + ((k & 1) ? wmean(cc.az[q], CZ[q], cc.az[q + cz], CZ[q + cz]) : CZ[q]));
}

template <class T>
__global__ void __launch_bounds__(kThreads)
k_prolong_add(Grid gf, Grid gc, Coefs<T> cf, Coefs<T> cc, const T *__restrict__ xc,
              T *__restrict__ x) {
    prolong_body<T>(gf, gc, cf, cc, xc, x, xcd_item());
}

template <class T, int NR>
__global__ void __launch_bounds__(kThreads)
k_prolong_add_b(Grid gf, Grid gc, Coefs<T> cf, Coefs<T> cc, const int32_t *__restrict__ rows, int64_t nrows,
                VPtr<const T> xc, VPtr<T> x) {
    int q;
    const int64_t t = wave_item(q);
    prolong_body<T>(gf, gc, cf, cc, xc.p[q], x.p[q], listed_item(gf, rows, nrows, t));
}

// x = 0 (a kernel, not a memset: it may be recorded into a HIP graph)
template <class T>
__global__ void __launch_bounds__(kThreads) k_zero(int64_t n, T *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads)
        x[e] = T(0);
}

template <class TI, class TO>
__global__ void k_cast(const TI *__restrict__ in, TO *__restrict__ out, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads)
        out[e] = (TO)in[e];
}

// the cast over the listed units of a face vector (see Span)
template <class TI, class TO>
__global__ void k_cast_units(const TI *__restrict__ in, TO *__restrict__ out, int64_t n,
                             const int32_t *__restrict__ units, int64_t nunits) {
    const int64_t cnt = nunits * kSpanUnit;
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt;
         it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = (int64_t)units[it / kSpanUnit] * kSpanUnit + it % kSpanUnit;
        if (e < n) out[e] = (TO)in[e];
    }
}

// Coarsest level: x[idx[r]] = sum_c inv[r, c] f[idx[c]] (FP64 arithmetic);
// one row of the inverse serves every right-hand side
template <class T, int NR>
__device__ __forceinline__ void coarse_body_n(int n, const double *__restrict__ inv, const int64_t *__restrict__ idx,
                                              const VPtr<const T> &f, const VPtr<T> &x, int row) {
    double s[NR];
#pragma unroll
    for (int v = 0; v < NR; ++v) s[v] = 0.0;
    for (int col = threadIdx.x; col < n; col += kThreads) {
        const double w = inv[(int64_t)row * n + col];
        const int64_t e = idx[col];
#pragma unroll
        for (int v = 0; v < NR; ++v) s[v] += w * (double)f.p[v][e];
    }
    __shared__ double sh[NR][kThreads / 64];
#pragma unroll
    for (int v = 0; v < NR; ++v) {
        for (int off = 32; off > 0; off >>= 1) s[v] += __shfl_down(s[v], off, 64);
        if ((threadIdx.x & 63) == 0) sh[v][threadIdx.x >> 6] = s[v];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int v = 0; v < NR; ++v) {
            double t = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) t += sh[v][w];
            x.p[v][idx[row]] = (T)t;
        }
    }
}

template <class T>
__device__ __forceinline__ void coarse_body(int n, const double *__restrict__ inv, const int64_t *__restrict__ idx,
                                            const T *__restrict__ f, T *__restrict__ x, int row) {
    coarse_body_n<T, 1>(n, inv, idx, vptr1(f), vptr1(x), row);
}

template <class T>
__global__ void __launch_bounds__(kThreads)
k_coarse_solve(int n, const double *__restrict__ inv, const int64_t *__restrict__ idx,
               const T *__restrict__ f, T *__restrict__ x) {
    coarse_body<T>(n, inv, idx, f, x, blockIdx.x);
}

template <class T, int NR>
__global__ void __launch_bounds__(kThreads)
k_coarse_solve_b(int n, const double *__restrict__ inv, const int64_t *__restrict__ idx, VPtr<const T> f,
                 VPtr<T> x) {
    coarse_body_n<T, NR>(n, inv, idx, f, x, blockIdx.x);
}

// PMC ghost layer of one plane (axis a) from the values next to it; planes
// are filled in the order x, y, z so corner ghosts get both mirrors.
template <class T>
__global__ void k_mirror_faces(Grid g, int a, T *__restrict__ x) {
    const int n[3] = {g.nx, g.ny, g.nz};
    const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
    const int nb = n[b] + 2, nd = n[d] + 2;
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (int64_t)nb * nd) return;
    int idx[3];
    idx[b] = (int)(t % nb) - 1;
    idx[d] = (int)(t / nb) - 1;
    idx[a] = -1;
    const int64_t stride[3] = {1, g.sy, g.sz};
    const int64_t pg = pidx(g, idx[0], idx[1], idx[2]);
    for (int comp = 0; comp < 3; ++comp) {
        T *arr = x + comp * g.P;
        arr[pg] = comp == a ? arr[pg + 2 * stride[a]] : -arr[pg + stride[a]];
    }
}

template <class T>
__global__ void k_mirror_cells(Grid g, int a, T *__restrict__ x) {
    const int n[3] = {g.nx, g.ny, g.nz};
    const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
    const int nb = n[b] + 2, nd = n[d] + 2;
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (int64_t)nb * nd) return;
    int idx[3];
    idx[b] = (int)(t % nb) - 1;
    idx[d] = (int)(t / nb) - 1;
    idx[a] = -1;
    const int64_t stride[3] = {1, g.sy, g.sz};
    const int64_t pg = pidx(g, idx[0], idx[1], idx[2]);
    x[pg] = -x[pg + stride[a]];
}

// ---------------------------------------------------------------------------
// Scalar problem: g = D A b, b -= D^T psi, S = D A D^T (weight w per level)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void div_DA_body(const Grid &g, const Coefs<double> &c, const double *__restrict__ b,
                                            double *__restrict__ out, int64_t item) {
    int i, j, k;
    if (!cell_of(g, item, i, j, k)) return;
    const int64_t P = g.P, dy = g.sy, dz = g.sz, p = pidx(g, i, j, k);
    const double *X = b, *Y = b + P, *Z = b + 2 * P;
    const double s = c.ax[p + 1] * X[p + 1] - c.ax[p] * X[p] + c.ay[p + dy] * Y[p + dy] -
                     c.ay[p] * Y[p] + c.az[p + dz] * Z[p + dz] - c.az[p] * Z[p];
    put_cell<double>(g, out, i, j, k, p, c.vinv[p] != 0.0 ? s / g.h : 0.0);
}

__device__ __forceinline__ void grad_sub_body(const Grid &g, const Coefs<double> &c, const double *__restrict__ psi,
                                              const double *bin, double *bout, double scale, int64_t item) {
    int i, j, k;
    if (!cell_of(g, item, i, j, k)) return;
    const int64_t P = g.P, dy = g.sy, dz = g.sz, p = pidx(g, i, j, k);
    const double s = scale / g.h;
    const double pp = psi[p];
    const double vx = c.ax[p] != 0.0 ? bin[p] - s * (psi[p - 1] - pp) : 0.0;
    const double vy = c.ay[p] != 0.0 ? bin[P + p] - s * (psi[p - dy] - pp) : 0.0;
    const double vz = c.az[p] != 0.0 ? bin[2 * P + p] - s * (psi[p - dz] - pp) : 0.0;
    put_face<double>(g, bout, 0, i, j, k, p, vx);
    put_face<double>(g, bout + P, 1, i, j, k, p, vy);
    put_face<double>(g, bout + 2 * P, 2, i, j, k, p, vz);
}

template <class T>
__device__ inline T s_row(const Coefs<T> &c, const T *x, int64_t p, int64_t dy, int64_t dz) {
    const T xp = x[p];
    return c.ax[p] * (xp - x[p - 1]) + c.ax[p + 1] * (xp - x[p + 1]) +
           c.ay[p] * (xp - x[p - dy]) + c.ay[p + dy] * (xp - x[p + dy]) +
           c.az[p] * (xp - x[p - dz]) + c.az[p + dz] * (xp - x[p + dz]);
}

template <class T>
__device__ __forceinline__ void s_apply_body(const Grid &g, const Coefs<T> &c, T w, int resid,
                                             const T *__restrict__ f, const T *__restrict__ x, T *__restrict__ y,
                                             int64_t item) {
    int i, j, k;
    if (!cell_of(g, item, i, j, k)) return;
    const int64_t p = pidx(g, i, j, k);
    T v = w * s_row<T>(c, x, p, g.sy, g.sz);
    if (resid) v = f[p] - v;
    put_cell<T>(g, y, i, j, k, p, c.vinv[p] != T(0) ? v : T(0));
}

// rows: optional list of the grid rows (k * ny + j) holding an active cell;
// the colour sweep then visits only those
template <class T>
__device__ __forceinline__ void s_smooth_body(const Grid &g, const Coefs<T> &c, T w, int colour,
                                              const T *__restrict__ f, T *__restrict__ x, int64_t t,
                                              const int32_t *__restrict__ rows = nullptr, int64_t nrows = 0) {
    const int nxh = (g.nx + 1) >> 1;
    if (t >= (rows ? nrows : (int64_t)g.ny * g.nz) * nxh) return;
    const int ih = (int)(t % nxh);
    const int64_t r = rows ? (int64_t)rows[t / nxh] : t / nxh;
    const int j = (int)(r % g.ny), k = (int)(r / g.ny);
    const int i = 2 * ih + ((j + k + colour) & 1);
    if (i >= g.nx) return;
    const int64_t dy = g.sy, dz = g.sz, p = pidx(g, i, j, k);
    if (c.vinv[p] == T(0)) return;
    T d = c.ax[p] + c.ax[p + 1] + c.ay[p] + c.ay[p + dy] + c.az[p] + c.az[p + dz];
    // odd mirror across a PMC plane: the face in the plane counts twice
    if ((g.pmc & 1) && i == 0) d += c.ax[p];
    if ((g.pmc & 2) && j == 0) d += c.ay[p];
    if ((g.pmc & 4) && k == 0) d += c.az[p];
    d *= w;
    if (d == T(0)) return;
    put_cell<T>(g, x, i, j, k, p, x[p] + (f[p] - w * s_row<T>(c, x, p, dy, dz)) / d);
}

template <class T>
__device__ __forceinline__ void s_restrict_body(const Grid &gf, const Grid &gc, const Coefs<T> &cc,
                                                const T *__restrict__ r, T *__restrict__ fc, int64_t item,
                                                T *__restrict__ xz = nullptr) {
    int I, J, K;
    if (!cell_of(gc, item, I, J, K)) return;
    const int64_t pc = pidx(gc, I, J, K), q = pidx(gf, 2 * I, 2 * J, 2 * K);
    const int64_t fy = gf.sy, fz = gf.sz;
    T s = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) s += r[q + a * fy + b * fz] + r[q + 1 + a * fy + b * fz];
    put_cell<T>(gc, fc, I, J, K, pc, cc.vinv[pc] != T(0) ? T(0.125) * s : T(0));
    if (xz) put_cell<T>(gc, xz, I, J, K, pc, T(0));   // the coarse iterate starts at zero
}

template <class T>
__device__ __forceinline__ void s_prolong_body(const Grid &gf, const Grid &gc, const Coefs<T> &cf,
                                               const T *__restrict__ xc, T *__restrict__ x, int64_t item) {
    int i, j, k;
    if (!cell_of(gf, item, i, j, k)) return;
    const int64_t p = pidx(gf, i, j, k);
    if (cf.vinv[p] != T(0)) put_cell<T>(gf, x, i, j, k, p, x[p] + xc[pidx(gc, i >> 1, j >> 1, k >> 1)]);
}

__global__ void __launch_bounds__(kThreads)
k_div_DA(Grid g, Coefs<double> c, const double *__restrict__ b, double *__restrict__ out) {
    div_DA_body(g, c, b, out, xcd_item());
}

__global__ void __launch_bounds__(kThreads)
k_grad_sub(Grid g, Coefs<double> c, const double *__restrict__ psi, const double *bin, double *bout, double scale) {
    grad_sub_body(g, c, psi, bin, bout, scale, xcd_item());
}

__global__ void __launch_bounds__(kThreads)
k_s_apply(Grid g, Coefs<double> c, double w, int resid, const double *__restrict__ f,
          const double *__restrict__ x, double *__restrict__ y) {
    s_apply_body<double>(g, c, w, resid, f, x, y, xcd_item());
}

__global__ void __launch_bounds__(kThreads)
k_s_smooth(Grid g, Coefs<double> c, double w, int colour, const double *__restrict__ f,
           double *__restrict__ x) {
    s_smooth_body<double>(g, c, w, colour, f, x, xcd_item());
}

__global__ void __launch_bounds__(kThreads)
k_s_restrict(Grid gf, Grid gc, Coefs<double> cc, const double *__restrict__ r,
             double *__restrict__ fc) {
    s_restrict_body<double>(gf, gc, cc, r, fc, xcd_item());
}

__global__ void __launch_bounds__(kThreads)
k_s_prolong_add(Grid gf, Grid gc, Coefs<double> cf, const double *__restrict__ xc,
                double *__restrict__ x) {
    s_prolong_body<double>(gf, gc, cf, xc, x, xcd_item());
}

// block forms of the scalar kernels: NR lanes per cell, one vector each
template <int NR>
__global__ void __launch_bounds__(kThreads)
k_div_DA_b(Grid g, Coefs<double> c, VPtr<const double> b, VPtr<double> out) {
    int q;
    const int64_t t = wave_item(q);
    div_DA_body(g, c, b.p[q], out.p[q], t);
}

template <int NR>
__global__ void __launch_bounds__(kThreads)
k_grad_sub_b(Grid g, Coefs<double> c, VPtr<const double> psi, VPtr<const double> bin, VPtr<double> bout,
             double scale) {
    int q;
    const int64_t t = wave_item(q);
    grad_sub_body(g, c, psi.p[q], bin.p[q], bout.p[q], scale, t);
}

template <class T, int NR>
__global__ void __launch_bounds__(kThreads)
k_s_apply_b(Grid g, Coefs<T> c, T w, int resid, const int32_t *__restrict__ rows, int64_t nrows, VPtr<const T> f,
            VPtr<const T> x, VPtr<T> y) {
    int q;
    const int64_t t = wave_item(q);
    s_apply_body<T>(g, c, w, resid, f.p[q], x.p[q], y.p[q], listed_item(g, rows, nrows, t));
}

template <class T, int NR>
__global__ void __launch_bounds__(kThreads)
k_s_smooth_b(Grid g, Coefs<T> c, T w, int colour, const int32_t *__restrict__ rows, int64_t nrows, VPtr<const T> f,
             VPtr<T> x) {
    int q;
    const int64_t t = wave_item(q);
    s_smooth_body<T>(g, c, w, colour, f.p[q], x.p[q], t, rows, nrows);
}

template <class T, int NR>
__global__ void __launch_bounds__(kThreads)
k_s_restrict_b(Grid gf, Grid gc, Coefs<T> cc, const int32_t *__restrict__ rows, int64_t nrows, VPtr<const T> r,
               VPtr<T> fc, VPtr<T> xz) {
    int q;
    const int64_t t = wave_item(q);
    s_restrict_body<T>(gf, gc, cc, r.p[q], fc.p[q], listed_item(gc, rows, nrows, t), xz.p[q]);
}

template <class T, int NR>
__global__ void __launch_bounds__(kThreads)
k_s_prolong_add_b(Grid gf, Grid gc, Coefs<T> cf, const int32_t *__restrict__ rows, int64_t nrows,
                  VPtr<const T> xc, VPtr<T> x) {
    int q;
    const int64_t t = wave_item(q);
    s_prolong_body<T>(gf, gc, cf, xc.p[q], x.p[q], listed_item(gf, rows, nrows, t));
}

// ---------------------------------------------------------------------------
// FP64 vector helpers
// ---------------------------------------------------------------------------
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads)
        y[e] = a * x[e] + b * y[e];
}

__global__ void k_axpy(int64_t n, double a, const double *__restrict__ x, double *__restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads)
        y[e] += a * x[e];
}

__global__ void k_scale(int64_t n, double a, double *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads)
        x[e] *= a;
}

constexpr int kChunk = 8;  // vectors reduced per pass of k_mdot

// Reductions and multi-axpys stream long FP64 vectors: they read pairs of
// doubles (16-byte loads) when every pointer is 16-byte aligned and the
// length / stride are even (VEC = 2), else single doubles (VEC = 1).
template <int VEC>
struct Vec;
template <>
struct Vec<1> {
    using T = double;
    __device__ static T ld(const double *p, int64_t e) { return p[e]; }
    __device__ static void st(double *p, int64_t e, T v) { p[e] = v; }
    __device__ static double dot(T a, T b) { return a * b; }
    __device__ static T fma(double c, T a, T b) { return b + c * a; }
    __device__ static T mul(T a, T b) { return a * b; }
    __device__ static T scale(double c, T a) { return c * a; }
    __device__ static T zero() { return 0.0; }
};
template <>
struct Vec<2> {
    using T = double2;
    __device__ static T ld(const double *p, int64_t e) { return reinterpret_cast<const double2 *>(p)[e]; }
    __device__ static void st(double *p, int64_t e, T v) { reinterpret_cast<double2 *>(p)[e] = v; }
    __device__ static double dot(T a, T b) { return a.x * b.x + a.y * b.y; }
    __device__ static T fma(double c, T a, T b) { return make_double2(b.x + c * a.x, b.y + c * a.y); }
    __device__ static T mul(T a, T b) { return make_double2(a.x * b.x, a.y * b.y); }
    __device__ static T scale(double c, T a) { return make_double2(c * a.x, c * a.y); }
    __device__ static T zero() { return make_double2(0.0, 0.0); }
};

// Four doubles (two 16-byte loads): the width at which an FP32 basis column
// is read with 16-byte loads as well (VEC = 4 needs lengths and strides that
// are multiples of 4 and 16-byte aligned pointers)
struct D4 {
    double2 a, b;
};
template <>
struct Vec<4> {
    using T = D4;
    __device__ static T ld(const double *p, int64_t e) {
        const double2 *q = reinterpret_cast<const double2 *>(p) + 2 * e;
        return {q[0], q[1]};
    }
    __device__ static void st(double *p, int64_t e, T v) {
        double2 *q = reinterpret_cast<double2 *>(p) + 2 * e;
        q[0] = v.a;
        q[1] = v.b;
    }
    __device__ static double dot(T a, T b) { return Vec<2>::dot(a.a, b.a) + Vec<2>::dot(a.b, b.b); }
    __device__ static T fma(double c, T a, T b) { return {Vec<2>::fma(c, a.a, b.a), Vec<2>::fma(c, a.b, b.b)}; }
    __device__ static T mul(T a, T b) { return {Vec<2>::mul(a.a, b.a), Vec<2>::mul(a.b, b.b)}; }
    __device__ static T scale(double c, T a) { return {Vec<2>::scale(c, a.a), Vec<2>::scale(c, a.b)}; }
    __device__ static T zero() { return {Vec<2>::zero(), Vec<2>::zero()}; }
};

// VEC consecutive entries of a Krylov basis column in FP64: FP64 columns
// as they are, FP32 columns widened (the basis kept in FP32; every sum and
// update is still FP64)
template <int VEC, class TV>
struct BasisLd;
template <int VEC>
struct BasisLd<VEC, double> {
    __device__ static typename Vec<VEC>::T ld(const double *p, int64_t e) { return Vec<VEC>::ld(p, e); }
};
template <>
struct BasisLd<1, float> {
    __device__ static double ld(const float *p, int64_t e) { return (double)p[e]; }
};
template <>
struct BasisLd<2, float> {
    __device__ static double2 ld(const float *p, int64_t e) {
        const float2 v = reinterpret_cast<const float2 *>(p)[e];
        return make_double2((double)v.x, (double)v.y);
    }
};
template <>
struct BasisLd<4, float> {
    __device__ static D4 ld(const float *p, int64_t e) {
        const float4 v = reinterpret_cast<const float4 *>(p)[e];
        return {make_double2((double)v.x, (double)v.y), make_double2((double)v.z, (double)v.w)};
    }
};

// Index i of a grid-stride loop -> element (in VEC units) of the listed
// units; the whole vector without a list.  Elements past nvec (a partial
// last unit) are skipped by the caller.
template <int VEC>
__device__ __forceinline__ int64_t span_count(const Span &sp, int64_t nvec) {
    return sp.u ? sp.n * (kSpanUnit / VEC) : nvec;
}
template <int VEC>
__device__ __forceinline__ int64_t span_elem(const Span &sp, int64_t i) {
    constexpr int per = kSpanUnit / VEC;
    return sp.u ? (int64_t)sp.u[i / per] * per + (i % per) : i;
}

// part[i][block] = partial sums of V_i . (w * wt) over the block's elements
template <int VEC, class TV = double>
__global__ void __launch_bounds__(kThreads)
k_mdot(int nv, const TV *__restrict__ V, int64_t ld, const double *__restrict__ w,
       const double *__restrict__ wt, int64_t n, double *__restrict__ part, Span sp) {
    using O = Vec<VEC>;
    const int64_t nvec = n / VEC, ldv = ld / VEC, cnt = span_count<VEC>(sp, nvec);
    for (int c0 = 0; c0 < nv; c0 += kChunk) {
        const int cn = min(kChunk, nv - c0);
        double acc[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) acc[q] = 0.0;
        for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt;
             it += (int64_t)gridDim.x * kThreads) {
            const int64_t e = span_elem<VEC>(sp, it);
            if (e >= nvec) continue;
            typename O::T wv = O::ld(w, e);
            if (wt) wv = O::mul(wv, O::ld(wt, e));
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
                if (q < cn) acc[q] += O::dot(BasisLd<VEC, TV>::ld(V + (int64_t)(c0 + q) * ldv * VEC, e), wv);
        }
        if (VEC == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const double wv = w[n - 1] * (wt ? wt[n - 1] : 1.0);
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
                if (q < cn) acc[q] += V[(int64_t)(c0 + q) * ld + n - 1] * wv;
        }
        __shared__ double sh[kThreads / 64][kChunk];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            double v = acc[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) sh[wave][q] = v;
        }
        __syncthreads();
        if (threadIdx.x < cn) {
            double t = 0.0;
            for (int u = 0; u < kThreads / 64; ++u) t += sh[u][threadIdx.x];
            part[(int64_t)(c0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// part rows 0..nv-1: V_i . w; row nv: |w|^2  (chunks of kChunk vectors)
template <int VEC, class TV = double>
__global__ void __launch_bounds__(kThreads)
k_mdot_norm(int nv, const TV *__restrict__ V, int64_t ld, const double *__restrict__ w,
            int64_t n, double *__restrict__ part, Span sp) {
    using O = Vec<VEC>;
    const int64_t nvec = n / VEC, ldv = ld / VEC, cnt = span_count<VEC>(sp, nvec);
    __shared__ double sh[kThreads / 64][kChunk + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = 0; c0 < nv; c0 += kChunk) {
        const int cn = min(kChunk, nv - c0);
        const bool last = c0 + kChunk >= nv;
        double acc[kChunk + 1];
#pragma unroll
        for (int q = 0; q <= kChunk; ++q) acc[q] = 0.0;
        for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt;
             it += (int64_t)gridDim.x * kThreads) {
            const int64_t e = span_elem<VEC>(sp, it);
            if (e >= nvec) continue;
            const typename O::T wv = O::ld(w, e);
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
                if (q < cn) acc[q] += O::dot(BasisLd<VEC, TV>::ld(V + (int64_t)(c0 + q) * ldv * VEC, e), wv);
            if (last) acc[kChunk] += O::dot(wv, wv);
        }
        if (VEC == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const double wv = w[n - 1];
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
                if (q < cn) acc[q] += V[(int64_t)(c0 + q) * ld + n - 1] * wv;
            if (last) acc[kChunk] += wv * wv;
        }
#pragma unroll
        for (int q = 0; q <= kChunk; ++q) {
            double v = acc[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) sh[wave][q] = v;
        }
        __syncthreads();
        if (threadIdx.x < cn || (last && threadIdx.x == cn)) {
            const int q = threadIdx.x < cn ? threadIdx.x : kChunk;
            double t = 0.0;
            for (int u = 0; u < kThreads / 64; ++u) t += sh[u][q];
            part[(int64_t)(c0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads)
k_mdot_final(int nblk, const double *__restrict__ part, double *__restrict__ out) {
    const int v = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) s += part[(int64_t)v * nblk + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double sh[kThreads / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int u = 0; u < kThreads / 64; ++u) t += sh[u];
        out[v] = t;
    }
}

// Dot products of up to kMaxRhs pairs in one pass:
//   part[q][block] = partial sum of X_q . (Y_q * wt) for the pairs with X_q set
// (wt, when given, is read once for all pairs), over the listed units of sp
template <int VEC>
__global__ void __launch_bounds__(kThreads)
k_dot_pairs(VPtr<const double> X, VPtr<const double> Y, const double *__restrict__ wt, int64_t n,
            double *__restrict__ part, Span sp) {
    using O = Vec<VEC>;
    const int64_t nvec = n / VEC, cnt = span_count<VEC>(sp, nvec);
    double acc[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) acc[q] = 0.0;
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt; it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = span_elem<VEC>(sp, it);
        if (e >= nvec) continue;
        const typename O::T w = wt ? O::ld(wt, e) : typename O::T{};
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q)
            if (X.p[q]) {
                const typename O::T x = O::ld(X.p[q], e);
                acc[q] += O::dot(wt ? O::mul(x, w) : x, O::ld(Y.p[q], e));
            }
    }
    if (VEC == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const double w = wt ? wt[n - 1] : 1.0;
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q)
            if (X.p[q]) acc[q] += X.p[q][n - 1] * w * Y.p[q][n - 1];
    }
    __shared__ double sh[kThreads / 64][kMaxRhs];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sh[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kMaxRhs) {
        double t = 0.0;
        for (int u = 0; u < kThreads / 64; ++u) t += sh[u][threadIdx.x];
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// out[v * stride] = sum of part row v (rows of nblk partial sums)
__global__ void __launch_bounds__(kThreads)
k_mdot_final_strided(int nblk, const double *__restrict__ part, double *__restrict__ out, int64_t stride) {
    const int v = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) s += part[(int64_t)v * nblk + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    __shared__ double sh[kThreads / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int u = 0; u < kThreads / 64; ++u) t += sh[u];
        out[(int64_t)v * stride] = t;
    }
}

// One conjugate-gradient update of the vectors with Pv_q set:
//   psi_q += a_q p_q,  r_q -= a_q q_q,  part[q][block] = partial of r_q . (r_q * wt)
// over the listed units of sp
__global__ void __launch_bounds__(kThreads)
k_cg_update(VPtr<const double> Pv, VPtr<const double> Qv, VPtr<double> Psi, VPtr<double> R, Coef4 a,
            const double *__restrict__ wt, int64_t n, double *__restrict__ part, Span sp) {
    double acc[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) acc[q] = 0.0;
    const int64_t cnt = span_count<1>(sp, n);
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt; it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = span_elem<1>(sp, it);
        if (e >= n) continue;
        const double w = wt[e];
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q)
            if (Pv.p[q]) {
                Psi.p[q][e] += a.v[q] * Pv.p[q][e];
                const double r = R.p[q][e] - a.v[q] * Qv.p[q][e];
                R.p[q][e] = r;
                acc[q] += r * r * w;
            }
    }
    __shared__ double sh[kThreads / 64][kMaxRhs];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sh[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kMaxRhs) {
        double t = 0.0;
        for (int u = 0; u < kThreads / 64; ++u) t += sh[u][threadIdx.x];
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// Y_q = X_q + b_q Y_q for the vectors with Y_q set, over the listed units of sp
__global__ void __launch_bounds__(kThreads)
k_xpby_b(VPtr<const double> X, Coef4 b, VPtr<double> Y, int64_t n, Span sp) {
    const int64_t cnt = span_count<1>(sp, n);
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt; it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = span_elem<1>(sp, it);
        if (e >= n) continue;
#pragma unroll
        for (int q = 0; q < kMaxRhs; ++q)
            if (Y.p[q]) Y.p[q][e] = X.p[q][e] + b.v[q] * Y.p[q][e];
    }
}

// X_q -= scale * val[q * stride] where mask != 0, for the vectors with X_q set
__global__ void __launch_bounds__(kThreads)
k_sub_masked_b(int64_t n, const double *__restrict__ mask, const double *__restrict__ val, int64_t stride,
               double scale, VPtr<double> X) {
    double m[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) m[q] = X.p[q] ? val[q * stride] * scale : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads)
        if (mask[e] != 0.0)
#pragma unroll
            for (int q = 0; q < kMaxRhs; ++q)
                if (X.p[q]) X.p[q][e] -= m[q];
}

// Block forms for the eigensolver's basis work (NW <= 8 vectors at once):
// part[(i*NW + q)][block] = partial sums of V_i . (W_q * wt) for i < nv; the
// basis is read once, W once per chunk of CH basis vectors (CH * NW ~ 16
// accumulators per thread)

template <int VEC, int NW, int CH>
__global__ void __launch_bounds__(kThreads)
k_mdot_multi(int nv, const double *__restrict__ V, int64_t ld, const double *__restrict__ W, int64_t ldw,
             const double *__restrict__ wt, int64_t n, double *__restrict__ part, Span sp) {
    using O = Vec<VEC>;
    const int64_t nvec = n / VEC, ldv = ld / VEC, ldwv = ldw / VEC, cnt = span_count<VEC>(sp, nvec);
    __shared__ double sh[kThreads / 64][CH * NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = 0; c0 < nv; c0 += CH) {
        const int cn = min(CH, nv - c0);
        double acc[CH][NW];
#pragma unroll
        for (int a = 0; a < CH; ++a)
#pragma unroll
            for (int q = 0; q < NW; ++q) acc[a][q] = 0.0;
        for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt;
             it += (int64_t)gridDim.x * kThreads) {
            const int64_t e = span_elem<VEC>(sp, it);
            if (e >= nvec) continue;
            typename O::T wv[NW];
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                wv[q] = O::ld(W + (int64_t)q * ldwv * VEC, e);
                if (wt) wv[q] = O::mul(wv[q], O::ld(wt, e));
            }
#pragma unroll
            for (int a = 0; a < CH; ++a)
                if (a < cn) {
                    const typename O::T v = O::ld(V + (int64_t)(c0 + a) * ldv * VEC, e);
#pragma unroll
                    for (int q = 0; q < NW; ++q) acc[a][q] += O::dot(v, wv[q]);
                }
        }
        if (VEC == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const double tv = wt ? wt[n - 1] : 1.0;
            for (int a = 0; a < cn; ++a)
                for (int q = 0; q < NW; ++q)
                    acc[a][q] += V[(int64_t)(c0 + a) * ld + n - 1] * W[(int64_t)q * ldw + n - 1] * tv;
        }
#pragma unroll
        for (int a = 0; a < CH; ++a)
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                double v = acc[a][q];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
                if (lane == 0) sh[wave][a * NW + q] = v;
            }
        __syncthreads();
        for (int t = threadIdx.x; t < cn * NW; t += kThreads) {
            double v = 0.0;
            for (int u = 0; u < kThreads / 64; ++u) v += sh[u][t];
            part[(int64_t)(c0 * NW + t) * gridDim.x + blockIdx.x] = v;
        }
        __syncthreads();
    }
}

// Y_q = sum_i C[i][q] V_i (overwrite) or Y_q -= sum_i C[i][q] V_i for q < NW;
// C row-major (nv x NW, device); one read of the basis
template <int VEC, int NW>
__global__ void __launch_bounds__(kThreads)
k_maxpy_multi(int nv, const double *__restrict__ V, int64_t ld, const double *__restrict__ C,
              double *__restrict__ Y, int64_t ldy, int64_t n, int overwrite, Span sp) {
    using O = Vec<VEC>;
    __shared__ double cs[256 * NW];
    for (int t = threadIdx.x; t < nv * NW; t += kThreads) cs[t] = C[t];
    __syncthreads();
    const int64_t nvec = n / VEC, ldv = ld / VEC, ldyv = ldy / VEC, cnt = span_count<VEC>(sp, nvec);
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt;
         it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = span_elem<VEC>(sp, it);
        if (e >= nvec) continue;
        typename O::T acc[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) acc[q] = O::zero();
        for (int i = 0; i < nv; ++i) {
            const typename O::T v = O::ld(V + (int64_t)i * ldv * VEC, e);
#pragma unroll
            for (int q = 0; q < NW; ++q) acc[q] = O::fma(cs[i * NW + q], v, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            double *y = Y + (int64_t)q * ldyv * VEC;
            O::st(y, e, overwrite ? acc[q] : O::fma(-1.0, acc[q], O::ld(y, e)));
        }
    }
    if (VEC == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        for (int q = 0; q < NW; ++q) {
            double sacc = 0.0;
            for (int i = 0; i < nv; ++i) sacc += cs[i * NW + q] * V[(int64_t)i * ld + n - 1];
            double *y = Y + (int64_t)q * ldy;
            y[n - 1] = overwrite ? sacc : y[n - 1] - sacc;
        }
    }
}

// y = sum_i c_i V_i (overwrite) or y -= sum_i c_i V_i; w: optional input
// (out = scale * (w - sum c_i V_i) when w != nullptr)
template <int VEC, class TV = double>
__global__ void __launch_bounds__(kThreads)
k_maxpy(int nv, const TV *__restrict__ V, int64_t ld, const double *__restrict__ c,
        const double *__restrict__ cscale, const double *w, double scale, double *y, int64_t n, int overwrite,
        Span sp) {
    using O = Vec<VEC>;
    __shared__ double cs[256];
    for (int q = threadIdx.x; q < nv; q += kThreads) cs[q] = cscale ? c[q] * cscale[q] : c[q];
    __syncthreads();
    const int64_t nvec = n / VEC, ldv = ld / VEC, cnt = span_count<VEC>(sp, nvec);
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt;
         it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = span_elem<VEC>(sp, it);
        if (e >= nvec) continue;
        typename O::T s = O::zero();
        for (int q = 0; q < nv; ++q) s = O::fma(cs[q], BasisLd<VEC, TV>::ld(V + (int64_t)q * ldv * VEC, e), s);
        typename O::T r;
        if (w) r = O::scale(scale, O::fma(-1.0, s, O::ld(w, e)));
        else if (overwrite) r = s;
        else r = O::fma(-1.0, s, O::ld(y, e));
        O::st(y, e, r);
    }
    if (VEC == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < nv; ++q) s += cs[q] * V[(int64_t)q * ld + n - 1];
        y[n - 1] = w ? scale * (w[n - 1] - s) : (overwrite ? s : y[n - 1] - s);
    }
}

// y -= sum_i c_i V_i for FP32 columns V_i, in FP64 (each value widened
// before use: the same result as with the widened columns), over the
// listed units of the span
__global__ void __launch_bounds__(kThreads)
k_maxpy_f32(int nv, const float *__restrict__ V, int64_t ld, const double *__restrict__ c, double *y, int64_t n,
            Span sp) {
    __shared__ double cs[256];
    for (int q = threadIdx.x; q < nv; q += kThreads) cs[q] = c[q];
    __syncthreads();
    const int64_t nvec = n / 2, cnt = span_count<2>(sp, nvec);
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt; it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = span_elem<2>(sp, it);
        if (e >= nvec) continue;
        double2 acc = make_double2(0.0, 0.0);
        for (int q = 0; q < nv; ++q) {
            const float2 v = reinterpret_cast<const float2 *>(V + (int64_t)q * ld)[e];
            acc = Vec<2>::fma(cs[q], make_double2((double)v.x, (double)v.y), acc);
        }
        double2 *yy = reinterpret_cast<double2 *>(y);
        yy[e] = Vec<2>::fma(-1.0, acc, yy[e]);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double acc = 0.0;
        for (int q = 0; q < nv; ++q) acc += cs[q] * (double)V[(int64_t)q * ld + n - 1];
        y[n - 1] -= acc;
    }
}

// Fused Gram--Schmidt step for nv <= MAXV basis vectors:
//   w' = w - sum_i c_i V_i      (written back to w)
//   part rows 0..nv-1: V_i . w', row nv: |w'|^2
// One read of the basis (held in registers) serves the update and the dots.
constexpr int kFuseMax = 32;

// REREAD: the basis values are loaded a second time for the dot products
// instead of being held in registers (more vectors than registers allow; the
// second load is served by the L2 or the Infinity Cache).  Measured: for 32
// vectors holding them took 212 VGPRs (2 waves per SIMD) and rereading 149
// (3 waves), 3% faster on the 9-cell quarter; for 16 vectors holding them
// (144 VGPRs) stays faster than rereading (85).
template <int VEC, int MAXV, bool REREAD, class TV = double>
__global__ void __launch_bounds__(kThreads)
k_maxpy_mdot_norm(int nv, const TV *__restrict__ V, int64_t ld, const double *__restrict__ c,
                  const double *__restrict__ cscale, double *__restrict__ w, int64_t n, double *__restrict__ part,
                  Span sp) {
    using O = Vec<VEC>;
    __shared__ double cs[MAXV];
    for (int q = threadIdx.x; q < nv; q += kThreads) cs[q] = cscale ? c[q] * cscale[q] : c[q];
    __syncthreads();
    double acc[MAXV + 1];
#pragma unroll
    for (int q = 0; q <= MAXV; ++q) acc[q] = 0.0;
    const int64_t nvec = n / VEC, ldv = ld / VEC, cnt = span_count<VEC>(sp, nvec);
    for (int64_t it = (int64_t)blockIdx.x * kThreads + threadIdx.x; it < cnt;
         it += (int64_t)gridDim.x * kThreads) {
        const int64_t e = span_elem<VEC>(sp, it);
        if (e >= nvec) continue;
        typename O::T s = O::ld(w, e);
        if (REREAD) {
#pragma unroll
            for (int q = 0; q < MAXV; ++q)
                if (q < nv) s = O::fma(-cs[q], BasisLd<VEC, TV>::ld(V + (int64_t)q * ldv * VEC, e), s);
            O::st(w, e, s);
            // keep the compiler from holding the first loads in registers
            // for the second use (that costs 200+ VGPRs, 2 waves per SIMD)
            asm volatile("" ::: "memory");
#pragma unroll
            for (int q = 0; q < MAXV; ++q)
                if (q < nv) acc[q] += O::dot(BasisLd<VEC, TV>::ld(V + (int64_t)q * ldv * VEC, e), s);
        } else {
            typename O::T vv[REREAD ? 1 : MAXV];
#pragma unroll
            for (int q = 0; q < MAXV; ++q)
                if (q < nv) {
                    vv[q] = BasisLd<VEC, TV>::ld(V + (int64_t)q * ldv * VEC, e);
                    s = O::fma(-cs[q], vv[q], s);
                }
            O::st(w, e, s);
#pragma unroll
            for (int q = 0; q < MAXV; ++q)
                if (q < nv) acc[q] += O::dot(vv[q], s);
        }
        acc[MAXV] += O::dot(s, s);
    }
    if (VEC == 2 && (n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double t = w[n - 1];
#pragma unroll
        for (int q = 0; q < MAXV; ++q)
            if (q < nv) t -= cs[q] * V[(int64_t)q * ld + n - 1];
        w[n - 1] = t;
#pragma unroll
        for (int q = 0; q < MAXV; ++q)
            if (q < nv) acc[q] += V[(int64_t)q * ld + n - 1] * t;
        acc[MAXV] += t * t;
    }
    __shared__ double sh[kThreads / 64][MAXV + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q <= MAXV; ++q) {
        if (q < nv || q == MAXV) {
            double v = acc[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) sh[wave][q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x <= nv) {  // row nv carries |w'|^2
        const int q = threadIdx.x < nv ? threadIdx.x : MAXV;
        double t = 0.0;
        for (int u = 0; u < kThreads / 64; ++u) t += sh[u][q];
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

__global__ void k_sub_masked(int64_t n, const double *__restrict__ mask,
                             const double *__restrict__ val, double scale, double *__restrict__ x) {
    const double m = val[0] * scale;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads)
        if (mask[e] != 0.0) x[e] -= m;
}

__global__ void k_mask_mul(int64_t n, const double *__restrict__ mask, double *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads)
        if (mask[e] == 0.0) x[e] = 0.0;
}

// SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based hash:
// the value for counter c is the generator's output after c+1 steps from seed.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void k_randn(int64_t n, uint64_t seed, int64_t offset, const double *__restrict__ mask,
                        double *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads) {
        if (mask[e] == 0.0) {
            x[e] = 0.0;
            continue;
        }
        const uint64_t c = 2 * (uint64_t)(e + offset);
        const double u1 = ((double)(splitmix64_at(seed, c) >> 11) + 1.0) * 0x1.0p-53;
        const double u2 = (double)(splitmix64_at(seed, c + 1) >> 11) * 0x1.0p-53;
        x[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

// The transfers of the tilde form (eq. fullMat2): entry e of a face vector
// scaled by a^(1/2) (power > 0) or a^(-1/2) (power < 0) of its own face,
// a = coef[e] (the first three coefficient blocks are ax ay az in the face
// vector's layout); inactive entries become 0
template <class T>
__global__ void k_scale_a(int64_t n, const T *__restrict__ a, int power, T *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
        const T ae = a[e];
        x[e] = ae > T(0) ? (power > 0 ? x[e] * sqrt(ae) : x[e] / sqrt(ae)) : T(0);
    }
}

// x += a^(-1/2) r on the active entries
template <class T>
__global__ void k_add_scaled_a(int64_t n, const T *__restrict__ a, const T *__restrict__ r, T *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
        const T ae = a[e];
        if (ae > T(0)) x[e] += r[e] / sqrt(ae);
    }
}

// Electric field of an eigenvector at sample points: e = C^T b / k on the
// edges with l > 0 (zero on the others, e.g. the conducting walls), the
// circulation of b around each edge divided by h (the Yee scheme's Ampere
// law in the frequency domain), interpolated trilinearly from each
// component's own edge lattice (e_x at ((i + 1/2) h, j h, k h), ...).  One
// thread per point; a point whose stencil leaves the grid gets NaN.
__device__ inline double edge_e(const Grid &g, const Coefs<double> &c, const double *__restrict__ b, int comp, int i,
                                int j, int k, double inv_kh) {
    const int64_t P = g.P, dy = g.sy, dz = g.sz, p = pidx(g, i, j, k);
    const double *X = b, *Y = b + P, *Z = b + 2 * P;
    if (comp == 0) {
        if (!(c.lx[p] > 0.0)) return 0.0;
        return (Z[p] - Z[p - dy] - Y[p] + Y[p - dz]) * inv_kh;
    }
    if (comp == 1) {
        if (!(c.ly[p] > 0.0)) return 0.0;
        return (X[p] - X[p - dz] - Z[p] + Z[p - 1]) * inv_kh;
    }
    if (!(c.lz[p] > 0.0)) return 0.0;
    return (Y[p] - Y[p - 1] - X[p] + X[p - dy]) * inv_kh;
}

__global__ void k_sample_e(Grid g, Coefs<double> c, const double *__restrict__ b, double inv_kh, int npts,
                           const double *__restrict__ pts, double *__restrict__ out) {
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q >= npts) return;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int comp = 0; comp < 3; ++comp) {
        int i0[3];
        double t[3];
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            const double u = pts[3 * q + a] / g.h - (a == comp ? 0.5 : 0.0);
            const double f = floor(u);
            i0[a] = (int)f;
            t[a] = u - f;
            // edge lattice along comp: 0 .. n-1; across: 0 .. n
            const int hi = a == comp ? n[a] - 1 : n[a];
            if (!(f >= 0.0) || i0[a] + 1 > hi) ok = false;
        }
        double v = 0.0;
        if (ok) {
            for (int corner = 0; corner < 8; ++corner) {
                const int dx = corner & 1, dy = (corner >> 1) & 1, dz = corner >> 2;
                const double w = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
                if (w != 0.0) v += w * edge_e(g, c, b, comp, i0[0] + dx, i0[1] + dy, i0[2] + dz, inv_kh);
            }
        } else {
            v = __builtin_nan("");
        }
        out[3 * q + comp] = v;
    }
}

// x = in where mask != 0, else 0
__global__ void k_copy_masked(int64_t n, const double *__restrict__ in, const double *__restrict__ mask,
                              double *__restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads)
        x[e] = mask[e] != 0.0 ? in[e] : 0.0;
}

// ---------------------------------------------------------------------------
// Batched V-cycle steps (see BJob): the same bodies as the single-operator
// kernels, the job found from the block index.
// ---------------------------------------------------------------------------
__device__ inline int find_job(const BJob *__restrict__ jobs, int nj, int64_t b) {
    int lo = 0, hi = nj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int STEP, int COMP>
__global__ void __launch_bounds__(kThreads)
kb_step(const BJob *__restrict__ jobs, int nj, int colour) {
    const BJob &J = jobs[find_job(jobs, nj, blockIdx.x)];
    const int64_t lb = (int64_t)blockIdx.x - J.block0;
    const int64_t item = lb * blockDim.x + threadIdx.x;
    using T = float;
    if (STEP == BS_ZERO) {
        if (item < J.items) ((T *)J.out)[item] = T(0);
    } else if (STEP == BS_SMOOTH) {
        smooth_body<T, COMP>(J.g, coefs_of((const T *)J.c, J.g.P), (T)J.sigma, colour, (const T *)J.in, (T *)J.out,
                             item);
    } else if (STEP == BS_RESID) {
        apply_body<T, AK_RESID>(J.g, coefs_of((const T *)J.c, J.g.P), (T)J.sigma, (const T *)J.in,
                                (const T *)J.aux, (T *)J.out, item);
    } else if (STEP == BS_RESTRICT) {
        restrict_body<T>(J.g, J.gc, coefs_of((const T *)J.cc, J.gc.P), (const T *)J.in, (T *)J.out, item);
    } else if (STEP == BS_PROLONG) {
        prolong_body<T>(J.g, J.gc, coefs_of((const T *)J.c, J.g.P), coefs_of((const T *)J.cc, J.gc.P),
                        (const T *)J.in, (T *)J.out, item);
    } else {
        coarse_body<T>(J.ncoarse, J.inv, J.idx, (const T *)J.in, (T *)J.out, (int)lb);
    }
}

}  // namespace

void launch_batched(int step, int comp, int colour, const BJob *jobs, int njobs, int64_t nblocks, int tpb,
                    hipStream_t s) {
    const dim3 grid((unsigned)nblocks), block((unsigned)(step == BS_COARSE ? kThreads : tpb));
    switch (step) {
        case BS_ZERO: hipLaunchKernelGGL((kb_step<BS_ZERO, 0>), grid, block, 0, s, jobs, njobs, colour); break;
        case BS_SMOOTH:
            if (comp == 0) hipLaunchKernelGGL((kb_step<BS_SMOOTH, 0>), grid, block, 0, s, jobs, njobs, colour);
            else if (comp == 1) hipLaunchKernelGGL((kb_step<BS_SMOOTH, 1>), grid, block, 0, s, jobs, njobs, colour);
            else hipLaunchKernelGGL((kb_step<BS_SMOOTH, 2>), grid, block, 0, s, jobs, njobs, colour);
            break;
        case BS_RESID: hipLaunchKernelGGL((kb_step<BS_RESID, 0>), grid, block, 0, s, jobs, njobs, colour); break;
        case BS_RESTRICT: hipLaunchKernelGGL((kb_step<BS_RESTRICT, 0>), grid, block, 0, s, jobs, njobs, colour); break;
        case BS_PROLONG: hipLaunchKernelGGL((kb_step<BS_PROLONG, 0>), grid, block, 0, s, jobs, njobs, colour); break;
        default: hipLaunchKernelGGL((kb_step<BS_COARSE, 0>), grid, block, 0, s, jobs, njobs, colour); break;
    }
}

namespace {

inline dim3 flat_grid(int64_t n) {
    int64_t nb = ceil_div(n, kThreads);
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    return dim3((unsigned)nb);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class T>
void launch_apply(const Grid &g, const T *coef, T sigma, int kind, const T *f, const T *x, T *y,
                  hipStream_t s, ClassList cut) {
    if (cut.idx && (kind == AK_M || kind == AK_RESID)) {
        launch_apply_b<T>(g, coef, sigma, kind, 1, vptr1(f), vptr1(x), vptr1(y), s, cut);
        return;
    }
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    Coefs<T> c = coefs_of(coef, g.P);
    if (kind == AK_M)
        hipLaunchKernelGGL((k_apply<T, AK_M>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma, f, x, y);
    else if (kind == AK_K)
        hipLaunchKernelGGL((k_apply<T, AK_K>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma, f, x, y);
    else
        hipLaunchKernelGGL((k_apply<T, AK_RESID>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma, f, x, y);
}

template <class T>
void launch_apply_A_t(const Grid &g, const T *coef, const T *x, T *y, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((k_apply_A<T>), xcd_grid(n), dim3(kThreads), 0, s, g, coefs_of(coef, g.P), x, y);
}

void launch_apply_A(const Grid &g, const double *coef, const double *x, double *y, hipStream_t s) {
    launch_apply_A_t<double>(g, coef, x, y, s);
}

template <class T>
void launch_smooth(const Grid &g, const T *coef, T sigma, int comp, int colour, const T *f, T *x,
                   hipStream_t s, ClassList cut) {
    if (cut.idx) {
        VPtr<const T> F{};
        VPtr<T> X{};
        F.p[0] = f;
        X.p[0] = x;
        launch_smooth_b<T>(g, coef, sigma, comp, colour, 1, F, X, s, cut);
        return;
    }
    const int64_t n = (int64_t)((g.nx + 1) >> 1) * g.ny * g.nz;
    Coefs<T> c = coefs_of(coef, g.P);
    if (comp == 0)
        hipLaunchKernelGGL((k_smooth<T, 0>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma, colour, f, x);
    else if (comp == 1)
        hipLaunchKernelGGL((k_smooth<T, 1>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma, colour, f, x);
    else
        hipLaunchKernelGGL((k_smooth<T, 2>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma, colour, f, x);
}

template <class T>
void launch_restrict(const Grid &gf, const Grid &gc, const T *coef_c, const T *r, T *fc,
                     hipStream_t s) {
    const int64_t n = (int64_t)gc.nx * gc.ny * gc.nz;
    hipLaunchKernelGGL((k_restrict<T>), xcd_grid(n), dim3(kThreads), 0, s, gf, gc,
                       coefs_of(coef_c, gc.P), r, fc);
}

template <class T>
void launch_prolong_add(const Grid &gf, const Grid &gc, const T *coef_f, const T *coef_c, const T *xc,
                        T *x, hipStream_t s) {
    const int64_t n = (int64_t)gf.nx * gf.ny * gf.nz;
    hipLaunchKernelGGL((k_prolong_add<T>), xcd_grid(n), dim3(kThreads), 0, s, gf, gc,
                       coefs_of(coef_f, gf.P), coefs_of(coef_c, gc.P), xc, x);
}

// cut rows of a component (both colours) below which the block smoother
// gives each vector its own wave: ClassList::wave_split_max, an operator
// option (default 65536, measured on the 128^3 sphere: ~60k rows per colour
// on the finest level favour the in-thread loop, ~15k rows on the next the
// waves)

// ---- block forms: dispatch nr (1..kMaxRhs) to the template
#define DM_NR_SWITCH(nr, CALL)                      \
    switch (nr) {                                   \
        case 1: { constexpr int NR = 1; CALL; } break; \
        case 2: { constexpr int NR = 2; CALL; } break; \
        case 3: { constexpr int NR = 3; CALL; } break; \
        case 4: { constexpr int NR = 4; CALL; } break; \
        default: throw std::runtime_error("block of more than 4 vectors"); \
    }

template <class T>
void launch_apply_b(const Grid &g, const T *coef, T sigma, int kind, int nr, const VPtr<const T> &f,
                    const VPtr<const T> &x, const VPtr<T> &y, hipStream_t s, ClassList cut) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const Coefs<T> c = coefs_of(coef, g.P);
    if (cut.idx && (kind == AK_M || kind == AK_RESID)) {
        if (cut.n > 0 && !cut_weights<T>(cut)) throw std::runtime_error("apply: cut-cell list without its row table");
        // the vacuum part visits the listed grid rows (every row without a list)
        const int64_t ncb = ceil_div(ceil_div(cut.n, 64), kXcd) * kXcd;
        const int64_t nvac = cut.rows ? cut.nrows * g.nx : n;
        const int64_t nvb = ceil_div(ceil_div(nvac, 64), kXcd) * kXcd;
        const dim3 grid((unsigned)(ncb + nvb));
        if (kind == AK_M)
            DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_apply_split<T, AK_M, NR>), grid, dim3(64 * NR), 0, s, g, c, sigma,
                                                cut.idx, cut.n, ncb, cut_weights<T>(cut), cut.rows, cut.nrows, f, x, y))
        else
            DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_apply_split<T, AK_RESID, NR>), grid, dim3(64 * NR), 0, s, g, c,
                                                sigma, cut.idx, cut.n, ncb, cut_weights<T>(cut), cut.rows, cut.nrows, f, x, y))
        return;
    }
    if (kind == AK_M)
        DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_apply_b<T, AK_M, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, g, c,
                                            sigma, f, x, y))
    else if (kind == AK_RESID)
        DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_apply_b<T, AK_RESID, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, g,
                                            c, sigma, f, x, y))
    else
        throw std::runtime_error("block apply: M or residual only");
}

void launch_apply_m_f32in(const Grid &g, const double *coef, double sigma, int nr, const VPtr<const float> &x,
                         const VPtr<double> &y, hipStream_t s, ClassList cut) {
    // the split form; without cut cells (no list) every cell takes the vacuum part
    if (!cut.idx && cut.n != 0) throw std::runtime_error("apply with FP32 input: cut-cell list missing");
    if (cut.n > 0 && !cut.w64) throw std::runtime_error("apply: cut-cell list without its row table");
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const Coefs<double> c = coefs_of(coef, g.P);
    const int64_t ncb = cut.idx ? ceil_div(ceil_div(cut.n, 64), kXcd) * kXcd : 0;
    const int64_t nvac = cut.rows ? cut.nrows * g.nx : n;
    const int64_t nvb = ceil_div(ceil_div(nvac, 64), kXcd) * kXcd;
    const dim3 grid((unsigned)(ncb + nvb));
    const VPtr<const double> f{};
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_apply_split<double, AK_M, NR, float>), grid, dim3(64 * NR), 0, s, g, c,
                                        sigma, cut.idx, cut.n, ncb, cut_weights<double>(cut), cut.rows, cut.nrows, f, x, y))
}

template <class T>
void launch_smooth_b(const Grid &g, const T *coef, T sigma, int comp, int colour, int nr, const VPtr<const T> &f,
                     const VPtr<T> &x, hipStream_t s, ClassList cut) {
    const int64_t n = (int64_t)((g.nx + 1) >> 1) * g.ny * g.nz;
    const Coefs<T> c = coefs_of(coef, g.P);
    if (cut.idx) {
        if (cut.n > 0 && !cut_weights<T>(cut)) throw std::runtime_error("smoother: cut list without its row table");
        if (cut.pair != kPairNone && !cut.s) throw std::runtime_error("smoother: paired update without its sums");
        T *S = static_cast<T *>(cut.s);
        const int wave_split = nr > 1 && cut.n < cut.wave_split_max;
        const int64_t ncb = ceil_div(ceil_div(cut.n, wave_split ? 64 : kThreads), kXcd) * kXcd;
        // the vacuum part sweeps the listed rows (every row without a list)
        const int64_t nvac = cut.rows ? cut.nrows * ((g.nx + 1) >> 1) : n;
        const int64_t nvb = ceil_div(ceil_div(nvac, kThreads), kXcd) * kXcd;
        const dim3 grid((unsigned)(ncb + nvb));
        if (comp == 0)
            DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_smooth_split<T, 0, NR>), grid, dim3(kThreads), 0, s, g, c, sigma,
                                                colour, cut.idx, cut.n, ncb, wave_split, cut_weights<T>(cut), cut.pair,
                                                S, cut.rows, cut.nrows, f, x))
        else if (comp == 1)
            DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_smooth_split<T, 1, NR>), grid, dim3(kThreads), 0, s, g, c, sigma,
                                                colour, cut.idx, cut.n, ncb, wave_split, cut_weights<T>(cut), cut.pair,
                                                S, cut.rows, cut.nrows, f, x))
        else
            DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_smooth_split<T, 2, NR>), grid, dim3(kThreads), 0, s, g, c, sigma,
                                                colour, cut.idx, cut.n, ncb, wave_split, cut_weights<T>(cut), cut.pair,
                                                S, cut.rows, cut.nrows, f, x))
        return;
    }
    if (comp == 0)
        DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_smooth_b<T, 0, NR>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma,
                                            colour, f, x))
    else if (comp == 1)
        DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_smooth_b<T, 1, NR>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma,
                                            colour, f, x))
    else
        DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_smooth_b<T, 2, NR>), xcd_grid(n), dim3(kThreads), 0, s, g, c, sigma,
                                            colour, f, x))
}

template <class T>
void launch_restrict_b(const Grid &gf, const Grid &gc, const T *coef_c, int nr, const VPtr<const T> &r,
                       const VPtr<T> &fc, hipStream_t s, const VPtr<T> &xz, const int32_t *rows, int64_t nrows) {
    const int64_t n = rows ? nrows * gc.nx : (int64_t)gc.nx * gc.ny * gc.nz;
    const Coefs<T> cc = coefs_of(coef_c, gc.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_restrict_b<T, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, gf, gc, cc,
                                        rows, nrows, r, fc, xz))
}

template <class T>
void launch_prolong_add_b(const Grid &gf, const Grid &gc, const T *coef_f, const T *coef_c, int nr,
                          const VPtr<const T> &xc, const VPtr<T> &x, hipStream_t s, const int32_t *rows,
                          int64_t nrows) {
    const int64_t n = rows ? nrows * gf.nx : (int64_t)gf.nx * gf.ny * gf.nz;
    const Coefs<T> cf = coefs_of(coef_f, gf.P), cc = coefs_of(coef_c, gc.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_prolong_add_b<T, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, gf, gc, cf,
                                        cc, rows, nrows, xc, x))
}

template <class T>
void launch_coarse_solve_b(int n, const double *inv, const int64_t *idx, int nr, const VPtr<const T> &f,
                           const VPtr<T> &x, hipStream_t s) {
    if (n <= 0) return;
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_coarse_solve_b<T, NR>), dim3(n), dim3(kThreads), 0, s, n, inv, idx, f, x))
}

void launch_div_DA_b(const Grid &g, const double *coef, int nr, const VPtr<const double> &b,
                     const VPtr<double> &out, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const Coefs<double> c = coefs_of(coef, g.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_div_DA_b<NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, g, c, b, out))
}

void launch_grad_sub_b(const Grid &g, const double *coef, int nr, const VPtr<const double> &psi,
                       const VPtr<const double> &b_in, const VPtr<double> &b_out, double scale, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const Coefs<double> c = coefs_of(coef, g.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_grad_sub_b<NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, g, c, psi, b_in,
                                        b_out, scale))
}

template <class T>
void launch_s_apply_b(const Grid &g, const T *coef, double w, int resid, int nr, const VPtr<const T> &f,
                      const VPtr<const T> &x, const VPtr<T> &y, hipStream_t s, const int32_t *rows, int64_t nrows) {
    const int64_t n = rows ? nrows * g.nx : (int64_t)g.nx * g.ny * g.nz;
    const Coefs<T> c = coefs_of(coef, g.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_s_apply_b<T, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, g, c, (T)w,
                                        resid, rows, nrows, f, x, y))
}

template <class T>
void launch_s_smooth_b(const Grid &g, const T *coef, double w, int colour, int nr, const VPtr<const T> &f,
                       const VPtr<T> &x, hipStream_t s, const int32_t *rows, int64_t nrows) {
    const int64_t n = (int64_t)((g.nx + 1) >> 1) * (rows ? nrows : (int64_t)g.ny * g.nz);
    const Coefs<T> c = coefs_of(coef, g.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_s_smooth_b<T, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, g, c, (T)w,
                                        colour, rows, nrows, f, x))
}

template <class T>
void launch_s_restrict_b(const Grid &gf, const Grid &gc, const T *coef_c, int nr, const VPtr<const T> &r,
                         const VPtr<T> &fc, hipStream_t s, const VPtr<T> &xz, const int32_t *rows, int64_t nrows) {
    const int64_t n = rows ? nrows * gc.nx : (int64_t)gc.nx * gc.ny * gc.nz;
    const Coefs<T> cc = coefs_of(coef_c, gc.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_s_restrict_b<T, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, gf, gc, cc,
                                        rows, nrows, r, fc, xz))
}

template <class T>
void launch_s_prolong_add_b(const Grid &gf, const Grid &gc, const T *coef_f, int nr, const VPtr<const T> &xc,
                            const VPtr<T> &x, hipStream_t s, const int32_t *rows, int64_t nrows) {
    const int64_t n = rows ? nrows * gf.nx : (int64_t)gf.nx * gf.ny * gf.nz;
    const Coefs<T> cf = coefs_of(coef_f, gf.P);
    DM_NR_SWITCH(nr, hipLaunchKernelGGL((k_s_prolong_add_b<T, NR>), xcd_grid_waves(n), dim3(64 * NR), 0, s, gf, gc,
                                        cf, rows, nrows, xc, x))
}

#define DM_SCALAR_BLOCK(T)                                                                                        \
    template void launch_s_apply_b<T>(const Grid &, const T *, double, int, int, const VPtr<const T> &,           \
                                      const VPtr<const T> &, const VPtr<T> &, hipStream_t, const int32_t *,       \
                                      int64_t);                                                                   \
    template void launch_s_smooth_b<T>(const Grid &, const T *, double, int, int, const VPtr<const T> &,          \
                                       const VPtr<T> &, hipStream_t, const int32_t *, int64_t);                   \
    template void launch_s_restrict_b<T>(const Grid &, const Grid &, const T *, int, const VPtr<const T> &,       \
                                         const VPtr<T> &, hipStream_t, const VPtr<T> &, const int32_t *,          \
                                         int64_t);                                                                \
    template void launch_s_prolong_add_b<T>(const Grid &, const Grid &, const T *, int, const VPtr<const T> &,    \
                                            const VPtr<T> &, hipStream_t, const int32_t *, int64_t);
DM_SCALAR_BLOCK(double)
DM_SCALAR_BLOCK(float)
#undef DM_SCALAR_BLOCK

#undef DM_NR_SWITCH

template <class TI, class TO>
void launch_cast(const TI *in, TO *out, int64_t n, hipStream_t s, Span sp) {
    if (sp.u)
        hipLaunchKernelGGL((k_cast_units<TI, TO>), flat_grid(sp.n * kSpanUnit), dim3(kThreads), 0, s, in, out, n,
                           sp.u, sp.n);
    else
        hipLaunchKernelGGL((k_cast<TI, TO>), flat_grid(n), dim3(kThreads), 0, s, in, out, n);
}

template <class T>
void launch_coarse_solve(int n, const double *inv, const int64_t *idx, const T *f, T *x,
                         hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_coarse_solve<T>), dim3(n), dim3(kThreads), 0, s, n, inv, idx, f, x);
}

void launch_div_DA(const Grid &g, const double *coef, const double *b, double *gout,
                   hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_div_DA, xcd_grid(n), dim3(kThreads), 0, s, g, coefs_of(coef, g.P), b, gout);
}

void launch_grad_sub(const Grid &g, const double *coef, const double *psi, double *b_in,
                     double *b_out, double scale, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_grad_sub, xcd_grid(n), dim3(kThreads), 0, s, g, coefs_of(coef, g.P), psi,
                       (const double *)b_in, b_out, scale);
}

void launch_s_apply(const Grid &g, const double *coef, double w, int resid, const double *f,
                    const double *x, double *y, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_s_apply, xcd_grid(n), dim3(kThreads), 0, s, g, coefs_of(coef, g.P), w,
                       resid, f, x, y);
}

void launch_s_smooth(const Grid &g, const double *coef, double w, int colour, const double *f,
                     double *x, hipStream_t s) {
    const int64_t n = (int64_t)((g.nx + 1) >> 1) * g.ny * g.nz;
    hipLaunchKernelGGL(k_s_smooth, xcd_grid(n), dim3(kThreads), 0, s, g, coefs_of(coef, g.P), w,
                       colour, f, x);
}

void launch_s_restrict(const Grid &gf, const Grid &gc, const double *coef_c, const double *r,
                       double *fc, hipStream_t s) {
    const int64_t n = (int64_t)gc.nx * gc.ny * gc.nz;
    hipLaunchKernelGGL(k_s_restrict, xcd_grid(n), dim3(kThreads), 0, s, gf, gc,
                       coefs_of(coef_c, gc.P), r, fc);
}

void launch_s_prolong_add(const Grid &gf, const Grid &gc, const double *coef_f,
                          const double *xc, double *x, hipStream_t s) {
    const int64_t n = (int64_t)gf.nx * gf.ny * gf.nz;
    hipLaunchKernelGGL(k_s_prolong_add, xcd_grid(n), dim3(kThreads), 0, s, gf, gc,
                       coefs_of(coef_f, gf.P), xc, x);
}

template <class T>
void launch_mirror_faces(const Grid &g, T *x, hipStream_t s) {
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        if (!((g.pmc >> a) & 1)) continue;
        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
        const int64_t cnt = (int64_t)(n[b] + 2) * (n[d] + 2);
        hipLaunchKernelGGL((k_mirror_faces<T>), dim3((unsigned)ceil_div(cnt, kThreads)), dim3(kThreads), 0, s, g, a, x);
    }
}

template <class T>
void launch_mirror_cells(const Grid &g, T *x, hipStream_t s) {
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        if (!((g.pmc >> a) & 1)) continue;
        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
        const int64_t cnt = (int64_t)(n[b] + 2) * (n[d] + 2);
        hipLaunchKernelGGL(k_mirror_cells<T>, dim3((unsigned)ceil_div(cnt, kThreads)), dim3(kThreads), 0, s, g, a, x);
    }
}
template void launch_mirror_cells<double>(const Grid &, double *, hipStream_t);
template void launch_mirror_cells<float>(const Grid &, float *, hipStream_t);

template void launch_mirror_faces<double>(const Grid &, double *, hipStream_t);
template void launch_mirror_faces<float>(const Grid &, float *, hipStream_t);

void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, flat_grid(n), dim3(kThreads), 0, s, n, a, x, y);
}
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, flat_grid(n), dim3(kThreads), 0, s, n, a, x, b, y);
}
template <class T>
void launch_zero(int64_t n, T *x, hipStream_t s) {
    hipLaunchKernelGGL(k_zero<T>, flat_grid(n), dim3(kThreads), 0, s, n, x);
}
template void launch_zero<double>(int64_t, double *, hipStream_t);
template void launch_zero<float>(int64_t, float *, hipStream_t);

void launch_scale(int64_t n, double a, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_scale, flat_grid(n), dim3(kThreads), 0, s, n, a, x);
}
void launch_copy(int64_t n, const double *x, double *y, hipStream_t s) {
    (void)hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, s);
}

namespace {
inline bool vec2_ok(int64_t n, int64_t ld, std::initializer_list<const void *> ptrs) {
    if ((n & 1) && ld != 0) return false;
    if (ld & 1) return false;
    for (const void *p : ptrs)
        if (p && ((uintptr_t)p & 15)) return false;
    return true;
}
// the same for a Krylov basis of element type TV with the FP64 vectors in
// `ptrs`: FP32 columns are read as pairs of floats (8-byte aligned)
template <class TV>
inline bool vec2_basis_ok(int64_t n, int64_t ld, const TV *V, std::initializer_list<const void *> ptrs) {
    if (sizeof(TV) == 8) return vec2_ok(n, ld, {V}) && vec2_ok(n, ld, ptrs);
    return ((uintptr_t)V & 7) == 0 && vec2_ok(n, ld, ptrs);
}
// an FP32 basis read four floats at a time: lengths and strides multiples
// of 4, every pointer 16-byte aligned
template <class TV>
inline bool vec4_basis_ok(int64_t n, int64_t ld, const TV *V, std::initializer_list<const void *> ptrs) {
    if (sizeof(TV) == 8 || (n & 3) || (ld & 3) || ((uintptr_t)V & 15)) return false;
    for (const void *p : ptrs)
        if (p && ((uintptr_t)p & 15)) return false;
    return true;
}
// f(width) with the widest load width (a std::integral_constant) that the
// basis type and the pointers allow: 4 (FP32 basis only), 2 or 1
template <class TV, class F>
inline void with_basis_width(int64_t n, int64_t ld, const TV *V, std::initializer_list<const void *> ptrs, F &&f) {
    if constexpr (sizeof(TV) == 4)
        if (vec4_basis_ok(n, ld, V, ptrs)) return f(std::integral_constant<int, 4>{});
    if (vec2_basis_ok(n, ld, V, ptrs)) return f(std::integral_constant<int, 2>{});
    f(std::integral_constant<int, 1>{});
}

template <class TV>
void launch_mdot_t(int nv, const TV *V, int64_t ld, const double *w, const double *wt, int64_t n, double *part,
                   double *dout, hipStream_t s, Span sp) {
    if (nv <= 0) return;
    if (nv > 256) throw std::runtime_error("launch_mdot: more than 256 vectors");
    with_basis_width(n, ld, V, {w, wt}, [&](auto width) {
        constexpr int W = decltype(width)::value;
        hipLaunchKernelGGL((k_mdot<W, TV>), dim3(kReduceBlocks), dim3(kThreads), 0, s, nv, V, ld, w, wt, n, part, sp);
    });
    hipLaunchKernelGGL(k_mdot_final, dim3(nv), dim3(kThreads), 0, s, (int)kReduceBlocks,
                       (const double *)part, dout);
}
}  // namespace

void launch_mdot(int nv, const double *V, int64_t ld, const double *w, const double *wt,
                 int64_t n, double *part, double *dout, hipStream_t s, Span sp) {
    launch_mdot_t<double>(nv, V, ld, w, wt, n, part, dout, s, sp);
}
void launch_mdot(int nv, const float *V, int64_t ld, const double *w, const double *wt, int64_t n, double *part,
                 double *dout, hipStream_t s, Span sp) {
    launch_mdot_t<float>(nv, V, ld, w, wt, n, part, dout, s, sp);
}

#define DM_NW_SWITCH(nw, CALL)                                   \
    switch (nw) {                                                \
        case 1: { constexpr int NW = 1, CH = 16; CALL; } break;  \
        case 2: { constexpr int NW = 2, CH = 8; CALL; } break;   \
        case 3: { constexpr int NW = 3, CH = 5; CALL; } break;   \
        case 4: { constexpr int NW = 4, CH = 4; CALL; } break;   \
        case 5: { constexpr int NW = 5, CH = 2; CALL; } break;   \
        case 6: { constexpr int NW = 6, CH = 2; CALL; } break;   \
        case 7: { constexpr int NW = 7, CH = 2; CALL; } break;   \
        default: { constexpr int NW = 8, CH = 2; CALL; } break;  \
    }

void launch_mdot_multi(int nv, const double *V, int64_t ld, const double *W, int64_t ldw, int nw,
                       const double *wt, int64_t n, double *part, double *dout, hipStream_t s, Span sp) {
    if (nv <= 0 || nw <= 0) return;
    if (nw > kMultiMax || nv * nw > 256) throw std::runtime_error("launch_mdot_multi: too many products");
    const bool v2 = vec2_ok(n, ld, {V, W, wt}) && (ldw % 2 == 0);
    const dim3 g(kReduceBlocks), b(kThreads);
    if (v2) DM_NW_SWITCH(nw, hipLaunchKernelGGL((k_mdot_multi<2, NW, CH>), g, b, 0, s, nv, V, ld, W, ldw, wt, n, part,
                                                sp))
    else DM_NW_SWITCH(nw, hipLaunchKernelGGL((k_mdot_multi<1, NW, CH>), g, b, 0, s, nv, V, ld, W, ldw, wt, n, part, sp))
    hipLaunchKernelGGL(k_mdot_final, dim3(nv * nw), dim3(kThreads), 0, s, (int)kReduceBlocks,
                       (const double *)part, dout);
}

void launch_maxpy_multi(int nv, const double *V, int64_t ld, const double *C, int nw, double *Y, int64_t ldy,
                        int64_t n, int overwrite, hipStream_t s, Span sp) {
    if (nw <= 0 || (nv <= 0 && !overwrite)) return;
    if (nw > kMultiMax || nv > 256) throw std::runtime_error("launch_maxpy_multi: too many vectors");
    const int64_t cnt = sp.u ? sp.n * kSpanUnit : n;
    if (vec2_ok(n, ld, {V, Y}) && ldy % 2 == 0)
        DM_NW_SWITCH(nw, hipLaunchKernelGGL((k_maxpy_multi<2, NW>), flat_grid(cnt / 2), dim3(kThreads), 0, s, nv, V,
                                            ld, C, Y, ldy, n, overwrite, sp))
    else
        DM_NW_SWITCH(nw, hipLaunchKernelGGL((k_maxpy_multi<1, NW>), flat_grid(cnt), dim3(kThreads), 0, s, nv, V, ld,
                                            C, Y, ldy, n, overwrite, sp))
}

#undef DM_NW_SWITCH

namespace {
template <class TV>
void launch_maxpy_t(int nv, const TV *V, int64_t ld, const double *c, double *y, int64_t n, int overwrite,
                    hipStream_t s, const double *cscale, Span sp) {
    if (nv <= 0 && !overwrite) return;
    if (nv > 256) throw std::runtime_error("launch_maxpy: more than 256 vectors");
    const int64_t cnt = sp.u ? sp.n * kSpanUnit : n;
    with_basis_width(n, ld, V, {y}, [&](auto width) {
        constexpr int W = decltype(width)::value;
        hipLaunchKernelGGL((k_maxpy<W, TV>), flat_grid(cnt / W), dim3(kThreads), 0, s, nv, V, ld, c, cscale,
                           (const double *)nullptr, 1.0, y, n, overwrite, sp);
    });
}
}  // namespace

void launch_maxpy(int nv, const double *V, int64_t ld, const double *c, double *y, int64_t n,
                  int overwrite, hipStream_t s, const double *cscale, Span sp) {
    launch_maxpy_t<double>(nv, V, ld, c, y, n, overwrite, s, cscale, sp);
}
void launch_maxpy(int nv, const float *V, int64_t ld, const double *c, double *y, int64_t n, int overwrite,
                  hipStream_t s, const double *cscale, Span sp) {
    launch_maxpy_t<float>(nv, V, ld, c, y, n, overwrite, s, cscale, sp);
}

void launch_maxpy_f32(int nv, const float *V, int64_t ld, const double *c, double *y, int64_t n, hipStream_t s,
                      Span sp) {
    if (nv <= 0) return;
    if (nv > 256) throw std::runtime_error("launch_maxpy_f32: more than 256 vectors");
    if ((ld & 1) || ((uintptr_t)V & 7) || ((uintptr_t)y & 15))
        throw std::runtime_error("launch_maxpy_f32: columns must be 8-byte and y 16-byte aligned, ld even");
    const int64_t cnt = sp.u ? sp.n * kSpanUnit : n;
    hipLaunchKernelGGL(k_maxpy_f32, flat_grid(cnt / 2), dim3(kThreads), 0, s, nv, V, ld, c, y, n, sp);
}

// Workgroups of a grid-stride reduction kernel: as many as are resident at
// once (its occupancy times the CUs), at most kReduceBlocks.  Every
// workgroup carries the same share of the work, so a grid beyond what is
// resident leaves a partial second round (1024 workgroups of a kernel with
// three resident per CU ran as 768 + 256).  Computed once per kernel.
template <auto KERN>
int reduce_blocks() {
    static const int nb = [] {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, KERN, kThreads, 0) != hipSuccess || cus <= 0 ||
            per <= 0)
            return kReduceBlocks;
        return std::min(kReduceBlocks, cus * per);
    }();
    return nb;
}

namespace {
template <class TV>
void launch_maxpy_mdot_norm_t(int nv, const TV *V, int64_t ld, const double *c, double *w, int64_t n,
                              double *part, double *dout, hipStream_t s, const double *cscale, Span sp) {
    if (nv < 1 || nv + 1 > 256) throw std::runtime_error("launch_maxpy_mdot_norm: nv out of range");
    const dim3 b(kThreads);
    int nb = kReduceBlocks;
    // one fused kernel for nv <= 32 (the basis held in registers)
    auto fused = [&](auto kern, int blocks) {
        nb = blocks;
        hipLaunchKernelGGL(kern, dim3(nb), b, 0, s, nv, V, ld, c, cscale, w, n, part, sp);
    };
    with_basis_width(n, ld, V, {w}, [&](auto width) {
        constexpr int W = decltype(width)::value;
        if (nv <= 8) {
            fused(k_maxpy_mdot_norm<W, 8, false, TV>, reduce_blocks<k_maxpy_mdot_norm<W, 8, false, TV>>());
        } else if (nv <= 16) {
            fused(k_maxpy_mdot_norm<W, 16, false, TV>, reduce_blocks<k_maxpy_mdot_norm<W, 16, false, TV>>());
        } else if (nv <= 32) {
            fused(k_maxpy_mdot_norm<W, 32, true, TV>, reduce_blocks<k_maxpy_mdot_norm<W, 32, true, TV>>());
        } else {
            // too many vectors to hold in registers: update w, then a second
            // pass for the dots (the basis is read twice)
            launch_maxpy_t<TV>(nv, V, ld, c, w, n, 0, s, cscale, sp);
            hipLaunchKernelGGL((k_mdot_norm<W, TV>), dim3(kReduceBlocks), b, 0, s, nv, V, ld, (const double *)w, n,
                               part, sp);
        }
    });
    hipLaunchKernelGGL(k_mdot_final, dim3(nv + 1), dim3(kThreads), 0, s, nb, (const double *)part, dout);
}
}  // namespace

void launch_maxpy_mdot_norm(int nv, const double *V, int64_t ld, const double *c, double *w,
                            int64_t n, double *part, double *dout, hipStream_t s, const double *cscale,
                            Span sp) {
    launch_maxpy_mdot_norm_t<double>(nv, V, ld, c, w, n, part, dout, s, cscale, sp);
}
void launch_maxpy_mdot_norm(int nv, const float *V, int64_t ld, const double *c, double *w, int64_t n,
                            double *part, double *dout, hipStream_t s, const double *cscale, Span sp) {
    launch_maxpy_mdot_norm_t<float>(nv, V, ld, c, w, n, part, dout, s, cscale, sp);
}

void launch_maxpy_scale(int nv, const double *V, int64_t ld, const double *c, const double *w,
                        double scale, double *out, int64_t n, hipStream_t s) {
    if (nv < 0 || nv > 256) throw std::runtime_error("launch_maxpy_scale: nv out of range");
    if (vec2_ok(n, ld, {V, w, out}))
        hipLaunchKernelGGL(k_maxpy<2>, flat_grid(n / 2), dim3(kThreads), 0, s, nv, V, ld, c,
                           (const double *)nullptr, w, scale, out, n, 0, Span{});
    else
        hipLaunchKernelGGL(k_maxpy<1>, flat_grid(n), dim3(kThreads), 0, s, nv, V, ld, c,
                           (const double *)nullptr, w, scale, out, n, 0, Span{});
}

void launch_dot_pairs(int nr, const VPtr<const double> &X, const VPtr<const double> &Y, const double *wt,
                      int64_t n, double *part, double *dout, int64_t dstride, hipStream_t s, Span sp) {
    if (nr < 1 || nr > kMaxRhs) throw std::runtime_error("launch_dot_pairs: 1 to 4 pairs");
    VPtr<const double> x{}, y{};
    for (int q = 0; q < nr; ++q) {
        x.p[q] = X.p[q];
        y.p[q] = X.p[q] ? Y.p[q] : nullptr;
    }
    bool v2 = vec2_ok(n, 0, {wt});
    for (int q = 0; q < nr; ++q) v2 = v2 && vec2_ok(n, 0, {x.p[q], y.p[q]});
    if (v2) hipLaunchKernelGGL(k_dot_pairs<2>, dim3(kReduceBlocks), dim3(kThreads), 0, s, x, y, wt, n, part, sp);
    else hipLaunchKernelGGL(k_dot_pairs<1>, dim3(kReduceBlocks), dim3(kThreads), 0, s, x, y, wt, n, part, sp);
    hipLaunchKernelGGL(k_mdot_final_strided, dim3(nr), dim3(kThreads), 0, s, (int)kReduceBlocks,
                       (const double *)part, dout, dstride);
}

void launch_cg_update(int nr, const VPtr<const double> &Pv, const VPtr<const double> &Qv, const VPtr<double> &Psi,
                      const VPtr<double> &R, const Coef4 &a, const double *wt, int64_t n, double *part, double *dout,
                      int64_t dstride, hipStream_t s, Span sp) {
    if (nr < 1 || nr > kMaxRhs) throw std::runtime_error("launch_cg_update: 1 to 4 vectors");
    VPtr<const double> pv{};
    for (int q = 0; q < nr; ++q) pv.p[q] = Pv.p[q];
    hipLaunchKernelGGL(k_cg_update, dim3(kReduceBlocks), dim3(kThreads), 0, s, pv, Qv, Psi, R, a, wt, n, part, sp);
    hipLaunchKernelGGL(k_mdot_final_strided, dim3(nr), dim3(kThreads), 0, s, (int)kReduceBlocks,
                       (const double *)part, dout, dstride);
}

void launch_xpby_b(int nr, const VPtr<const double> &X, const Coef4 &b, const VPtr<double> &Y, int64_t n,
                   hipStream_t s, Span sp) {
    VPtr<double> y{};
    for (int q = 0; q < nr && q < kMaxRhs; ++q) y.p[q] = Y.p[q];
    hipLaunchKernelGGL(k_xpby_b, flat_grid(sp.u ? sp.n * kSpanUnit : n), dim3(kThreads), 0, s, X, b, y, n, sp);
}

void launch_sub_masked_b(int nr, int64_t n, const double *mask, const double *val, int64_t stride, double scale,
                         const VPtr<double> &X, hipStream_t s) {
    VPtr<double> x{};
    for (int q = 0; q < nr && q < kMaxRhs; ++q) x.p[q] = X.p[q];
    hipLaunchKernelGGL(k_sub_masked_b, flat_grid(n), dim3(kThreads), 0, s, n, mask, val, stride, scale, x);
}

void launch_sub_masked(int64_t n, const double *mask, const double *val, double scale, double *x,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_sub_masked, flat_grid(n), dim3(kThreads), 0, s, n, mask, val, scale, x);
}

void launch_mask_mul(int64_t n, const double *mask, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_mul, flat_grid(n), dim3(kThreads), 0, s, n, mask, x);
}

void launch_randn(int64_t n, uint64_t seed, int64_t offset, const double *mask, double *x,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_randn, flat_grid(n), dim3(kThreads), 0, s, n, seed, offset, mask, x);
}

void launch_sample_e(const Grid &g, const double *coef, const double *b, double k, int npts, const double *pts,
                     double *out, hipStream_t s) {
    if (npts <= 0) return;
    hipLaunchKernelGGL(k_sample_e, dim3((unsigned)ceil_div(npts, kThreads)), dim3(kThreads), 0, s, g,
                       coefs_of(coef, g.P), b, 1.0 / (k * g.h), npts, pts, out);
}

void launch_copy_masked(int64_t n, const double *in, const double *mask, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_masked, flat_grid(n), dim3(kThreads), 0, s, n, in, mask, x);
}

template <class T>
void launch_scale_a(int64_t n, const T *coef, int power, T *x, hipStream_t s) {
    hipLaunchKernelGGL((k_scale_a<T>), flat_grid(n), dim3(kThreads), 0, s, n, coef, power, x);
}
template <class T>
void launch_add_scaled_a(int64_t n, const T *coef, const T *r, T *x, hipStream_t s) {
    hipLaunchKernelGGL((k_add_scaled_a<T>), flat_grid(n), dim3(kThreads), 0, s, n, coef, r, x);
}
template void launch_scale_a<double>(int64_t, const double *, int, double *, hipStream_t);
template void launch_scale_a<float>(int64_t, const float *, int, float *, hipStream_t);
template void launch_add_scaled_a<double>(int64_t, const double *, const double *, double *, hipStream_t);
template void launch_add_scaled_a<float>(int64_t, const float *, const float *, float *, hipStream_t);

// explicit instantiations
#define DM_BLOCK_INST(T)                                                                                   \
    template void launch_apply_b<T>(const Grid &, const T *, T, int, int, const VPtr<const T> &,                 \
                                    const VPtr<const T> &, const VPtr<T> &, hipStream_t, ClassList);              \
    template void launch_smooth_b<T>(const Grid &, const T *, T, int, int, int, const VPtr<const T> &,           \
                                     const VPtr<T> &, hipStream_t, ClassList);                                    \
    template void launch_restrict_b<T>(const Grid &, const Grid &, const T *, int, const VPtr<const T> &,        \
                                       const VPtr<T> &, hipStream_t, const VPtr<T> &, const int32_t *, int64_t);                                             \
    template void launch_prolong_add_b<T>(const Grid &, const Grid &, const T *, const T *, int,                 \
                                          const VPtr<const T> &, const VPtr<T> &, hipStream_t, const int32_t *,   \
                                          int64_t);                   \
    template void launch_coarse_solve_b<T>(int, const double *, const int64_t *, int, const VPtr<const T> &,     \
                                           const VPtr<T> &, hipStream_t);
DM_BLOCK_INST(double)
DM_BLOCK_INST(float)
#undef DM_BLOCK_INST
template void launch_apply<double>(const Grid &, const double *, double, int, const double *,
                                   const double *, double *, hipStream_t, ClassList);
template void launch_apply<float>(const Grid &, const float *, float, int, const float *,
                                  const float *, float *, hipStream_t, ClassList);
template void launch_apply_A_t<float>(const Grid &, const float *, const float *, float *, hipStream_t);
template void launch_apply_A_t<double>(const Grid &, const double *, const double *, double *, hipStream_t);
template void launch_smooth<double>(const Grid &, const double *, double, int, int, const double *,
                                    double *, hipStream_t, ClassList);
template void launch_smooth<float>(const Grid &, const float *, float, int, int, const float *,
                                   float *, hipStream_t, ClassList);
template void launch_restrict<double>(const Grid &, const Grid &, const double *, const double *,
                                      double *, hipStream_t);
template void launch_restrict<float>(const Grid &, const Grid &, const float *, const float *,
                                     float *, hipStream_t);
template void launch_prolong_add<double>(const Grid &, const Grid &, const double *, const double *, const double *,
                                         double *, hipStream_t);
template void launch_prolong_add<float>(const Grid &, const Grid &, const float *, const float *, const float *,
                                        float *, hipStream_t);
template void launch_cast<double, float>(const double *, float *, int64_t, hipStream_t, Span);
template void launch_cast<float, double>(const float *, double *, int64_t, hipStream_t, Span);
template void launch_cast<float, float>(const float *, float *, int64_t, hipStream_t, Span);
template void launch_coarse_solve<double>(int, const double *, const int64_t *, const double *,
                                          double *, hipStream_t);
template void launch_coarse_solve<float>(int, const double *, const int64_t *, const float *,
                                         float *, hipStream_t);

}  // namespace dm
