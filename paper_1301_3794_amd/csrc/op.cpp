// Operator hierarchy: fractions of every level, device coefficient blocks,
// and the dense FP64 inverses of the coarsest vector and scalar operators.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "geometry.h"
#include "op.h"

namespace dm {

namespace {

// In-place inverse of a dense row-major n x n matrix by Gauss--Jordan with
// partial pivoting.  Returns the smallest |pivot| / largest |pivot|.
double invert_dense(std::vector<double> &a, int n) {
    std::vector<double> inv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    double pmin = INFINITY, pmax = 0.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = std::fabs(a[(size_t)c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            const double v = std::fabs(a[(size_t)r * n + c]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        pmin = std::min(pmin, best);
        pmax = std::max(pmax, best);
        if (best == 0.0) return 0.0;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)c * n + k], a[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        }
        const double d = 1.0 / a[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            a[(size_t)c * n + k] *= d;
            inv[(size_t)c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double m = a[(size_t)r * n + c];
            if (m == 0.0) continue;
            double *ar = &a[(size_t)r * n], *ac = &a[(size_t)c * n];
            double *ir = &inv[(size_t)r * n], *ic = &inv[(size_t)c * n];
            for (int k = 0; k < n; ++k) {
                ar[k] -= m * ac[k];
                ir[k] -= m * ic[k];
            }
        }
    }
    a.swap(inv);
    return pmax > 0.0 ? pmin / pmax : 0.0;
}

std::vector<double> to_coefs(const Grid &g, const std::vector<double> &fr) {
    std::vector<double> c(fr.begin(), fr.end());
    const int64_t P = g.P;
    for (int64_t p = 0; p < P; ++p) {
        const double v = fr[6 * P + p];
        c[6 * P + p] = v > 0.0 ? 1.0 / v : 0.0;
    }
    return c;
}

}  // namespace

void build_hierarchy(dm_op *op, const double *user_frac) {
    const int nl = op->opt.levels;
    Grid g0 = make_grid(op->dims[0], op->dims[1], op->dims[2], op->h);
    std::vector<double> fr;
    if (op->geom.kind == DM_GEOM_USER) {
        fr.assign(user_frac, user_frac + 7 * g0.P);
    } else {
        std::unique_ptr<Body> body = make_body(op->geom);
        if (!body) throw DmError{DM_EINVAL, "unknown or unsupported geometry kind"};
        compute_fractions(*body, g0, op->geom.bc_lo, fr);
    }
    neglect_faces(g0, op->geom.a_min, fr);
    op->frac.clear();
    op->frac.push_back(fr);
    std::vector<Grid> grids = {g0};
    for (int l = 1; l < nl; ++l) {
        const Grid &gf = grids.back();
        Grid gc = make_grid(gf.nx / 2, gf.ny / 2, gf.nz / 2, gf.h * 2.0);
        std::vector<double> fc;
        coarsen_fractions(gf, op->frac.back(), gc, fc);
        op->frac.push_back(fc);
        grids.push_back(gc);
    }
    op->lv.resize(nl);
    for (int l = 0; l < nl; ++l) {
        Level &L = op->lv[l];
        L.g = grids[l];
        const int64_t P = L.g.P;
        std::vector<double> c = to_coefs(L.g, op->frac[l]);
        std::vector<float> c32(c.begin(), c.end());
        L.coef64 = op->dalloc<double>(7 * P);
        L.coef32 = op->dalloc<float>(7 * P);
        DM_HIP(hipMemcpyAsync(L.coef64, c.data(), 7 * P * sizeof(double), hipMemcpyHostToDevice, op->stream));
        DM_HIP(hipMemcpyAsync(L.coef32, c32.data(), 7 * P * sizeof(float), hipMemcpyHostToDevice, op->stream));
        DM_HIP(hipStreamSynchronize(op->stream));
        L.sweight = 1.0 / (std::ldexp(1.0, l) * op->h * op->h);
        int64_t naf = 0, nac = 0;
        for (int64_t p = 0; p < 3 * P; ++p) naf += op->frac[l][p] > 0.0;
        for (int64_t p = 0; p < P; ++p) nac += op->frac[l][6 * P + p] > 0.0;
        L.n_act_faces = naf;
        L.n_act_cells = nac;
        if (l > 0) {
            L.x64 = op->dalloc<double>(3 * P);
            L.f64 = op->dalloc<double>(3 * P);
            L.x32 = op->dalloc<float>(3 * P);
            L.f32 = op->dalloc<float>(3 * P);
            L.sx = op->dalloc<double>(P);
            L.sf = op->dalloc<double>(P);
        }
        L.r64 = op->dalloc<double>(3 * P);
        L.r32 = op->dalloc<float>(3 * P);
        L.sr = op->dalloc<double>(P);
    }
    // level-0 masks
    const Grid &g = op->lv[0].g;
    std::vector<double> fm(3 * g.P), cm(g.P);
    for (int64_t p = 0; p < 3 * g.P; ++p) fm[p] = op->frac[0][p] > 0.0 ? 1.0 : 0.0;
    for (int64_t p = 0; p < g.P; ++p) cm[p] = op->frac[0][6 * g.P + p] > 0.0 ? 1.0 : 0.0;
    op->fmask = op->dalloc<double>(3 * g.P);
    op->cmask = op->dalloc<double>(g.P);
    DM_HIP(hipMemcpyAsync(op->fmask, fm.data(), fm.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipMemcpyAsync(op->cmask, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
    op->part = op->dalloc<double>((size_t)kReduceBlocks * kMaxDots);
    op->dres = op->dalloc<double>(kMaxDots);
    DM_HIP(hipHostMalloc((void **)&op->hres, kMaxDots * sizeof(double), hipHostMallocDefault));
    DM_HIP(hipStreamSynchronize(op->stream));
    // the scalar problem is singular (constants) unless a PMC plane pins psi
    op->s_floating = !(op->geom.bc_lo[0] == DM_BC_PMC || op->geom.bc_lo[1] == DM_BC_PMC ||
                       op->geom.bc_lo[2] == DM_BC_PMC);
}

// Dense coarsest operators.  Vector: M on the active faces of the coarsest
// level, assembled column by column from the stencil rows.  Scalar: the
// level's cell Laplacian, plus (mean diagonal / n) 1 1^T when the constant
// is in its null space (the inverse then maps mean-free right-hand sides to
// the mean-free solution).
void factor_coarse(dm_op *op) {
    Level &L = op->lv.back();
    const Grid &g = L.g;
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    std::vector<double> c = to_coefs(g, op->frac.back());
    Coefs<double> cf = coefs_of(c.data(), P);
    const double ih2 = 1.0 / (g.h * g.h);
    // ---- vector
    std::vector<int64_t> idx;
    std::unordered_map<int64_t, int> row_of;
    for (int comp = 0; comp < 3; ++comp)
        for (int k = 0; k < g.nz; ++k)
            for (int j = 0; j < g.ny; ++j)
                for (int i = 0; i < g.nx; ++i) {
                    const int64_t p = pidx(g, i, j, k);
                    if (c[comp * P + p] > 0.0) {
                        row_of[comp * P + p] = (int)idx.size();
                        idx.push_back(comp * P + p);
                    }
                }
    const int n = (int)idx.size();
    std::vector<double> Md((size_t)n * n, 0.0), e(3 * P, 0.0);
    for (int col = 0; col < n; ++col) {
        const int64_t pc = idx[col] % P;
        e[idx[col]] = 1.0;
        const int ic = (int)(pc % dy) - 1, jc = (int)((pc / dy) % (g.ny + 2)) - 1,
                  kc = (int)(pc / dz) - 1;
        for (int k = std::max(0, kc - 2); k <= std::min(g.nz - 1, kc + 2); ++k)
            for (int j = std::max(0, jc - 2); j <= std::min(g.ny - 1, jc + 2); ++j)
                for (int i = std::max(0, ic - 2); i <= std::min(g.nx - 1, ic + 2); ++i) {
                    const int64_t p = pidx(g, i, j, k);
                    const double *X = e.data(), *Y = e.data() + P, *Z = e.data() + 2 * P;
                    for (int comp = 0; comp < 3; ++comp) {
                        auto it = row_of.find(comp * P + p);
                        if (it == row_of.end()) continue;
                        double v;
                        if (comp == 0) v = ih2 * row_x<double, true>(cf, X, Y, Z, p, dy, dz) - op->sigma * cf.ax[p] * X[p];
                        else if (comp == 1) v = ih2 * row_y<double, true>(cf, X, Y, Z, p, dy, dz) - op->sigma * cf.ay[p] * Y[p];
                        else v = ih2 * row_z<double, true>(cf, X, Y, Z, p, dy, dz) - op->sigma * cf.az[p] * Z[p];
                        Md[(size_t)it->second * n + col] = v;
                    }
                }
        e[idx[col]] = 0.0;
    }
    const double ratio = invert_dense(Md, n);
    if (!(ratio > 1e-13))
        throw DmError{DM_ESINGULAR, "coarsest operator is singular at this shift (pivot ratio " +
                                        std::to_string(ratio) + ")"};
    op->nc = n;
    if (!op->cinv) {  // the active set does not change with the shift
        op->cinv = op->dalloc<double>((size_t)n * n);
        op->cidx = op->dalloc<int64_t>(n);
    }
    DM_HIP(hipMemcpyAsync(op->cinv, Md.data(), (size_t)n * n * sizeof(double), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipMemcpyAsync(op->cidx, idx.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, op->stream));
    // ---- scalar
    std::vector<int64_t> sidx;
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                const int64_t p = pidx(g, i, j, k);
                if (cf.vinv[p] > 0.0) sidx.push_back(p);
            }
    const int ns = (int)sidx.size();
    std::unordered_map<int64_t, int> srow;
    for (int r = 0; r < ns; ++r) srow[sidx[r]] = r;
    std::vector<double> Sd((size_t)ns * ns, 0.0);
    const double w = L.sweight;
    double dsum = 0.0;
    for (int r = 0; r < ns; ++r) {
        const int64_t p = sidx[r];
        const int64_t nb[6] = {p - 1, p + 1, p - dy, p + dy, p - dz, p + dz};
        const double wt[6] = {cf.ax[p], cf.ax[p + 1], cf.ay[p], cf.ay[p + dy], cf.az[p], cf.az[p + dz]};
        double d = 0.0;
        for (int q = 0; q < 6; ++q) {
            d += wt[q];
            auto it = srow.find(nb[q]);
            if (it != srow.end()) Sd[(size_t)r * ns + it->second] -= w * wt[q];
        }
        Sd[(size_t)r * ns + r] += w * d;
        dsum += w * d;
    }
    if (op->s_floating && ns > 0) {
        const double add = dsum / ns / ns;
        for (auto &v : Sd) v += add;
    }
    const double sratio = invert_dense(Sd, ns);
    if (!(sratio > 1e-14))
        throw DmError{DM_ESINGULAR, "coarsest scalar Laplacian is singular (disconnected cavity?)"};
    op->ns = ns;
    if (!op->sinv) {
        op->sinv = op->dalloc<double>((size_t)ns * ns);
        op->sidx = op->dalloc<int64_t>(ns);
    }
    DM_HIP(hipMemcpyAsync(op->sinv, Sd.data(), (size_t)ns * ns * sizeof(double), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipMemcpyAsync(op->sidx, sidx.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipStreamSynchronize(op->stream));
}

}  // namespace dm
