// Operator hierarchy: fractions of every level, device coefficient blocks,
// and the dense FP64 inverses of the coarsest vector and scalar operators.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "geometry.h"
#include "op.h"

namespace dm {

namespace {

// largest coarsest level factored densely (its inverse is n^2 doubles)
constexpr int kMaxCoarse = 4000;

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
        // eliminate column c from every other row (rows split over threads)
        auto elim = [&](int r0, int r1) {
            const double *ac = &a[(size_t)c * n], *ic = &inv[(size_t)c * n];
            for (int r = r0; r < r1; ++r) {
                if (r == c) continue;
                const double m = a[(size_t)r * n + c];
                if (m == 0.0) continue;
                double *ar = &a[(size_t)r * n], *ir = &inv[(size_t)r * n];
                for (int k = 0; k < n; ++k) {
                    ar[k] -= m * ac[k];
                    ir[k] -= m * ic[k];
                }
            }
        };
        const int nt = n >= 512 ? std::min(16, (int)std::max(1u, std::thread::hardware_concurrency())) : 1;
        if (nt == 1) {
            elim(0, n);
        } else {
            std::vector<std::thread> th;
            for (int t = 0; t < nt; ++t) th.emplace_back(elim, (int)((int64_t)n * t / nt), (int)((int64_t)n * (t + 1) / nt));
            for (auto &t : th) t.join();
        }
    }
    a.swap(inv);
    return pmax > 0.0 ? pmin / pmax : 0.0;
}

// host version of the PMC ghost fill of a face vector (planes x, y, z in order)
void mirror_faces_host(const Grid &g, double *x) {
    if (!g.pmc) return;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int64_t stride[3] = {1, g.sy, g.sz};
    for (int a = 0; a < 3; ++a) {
        if (!((g.pmc >> a) & 1)) continue;
        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
        for (int u = -1; u <= n[b]; ++u)
            for (int v = -1; v <= n[d]; ++v) {
                int idx[3];
                idx[a] = -1;
                idx[b] = u;
                idx[d] = v;
                const int64_t pg = pidx(g, idx[0], idx[1], idx[2]);
                for (int c = 0; c < 3; ++c) {
                    double *arr = x + c * g.P;
                    arr[pg] = c == a ? arr[pg + 2 * stride[a]] : -arr[pg + stride[a]];
                }
            }
    }
}

// use_v = false: the grad-div term without V^-1 (1 on every cell with v > 0)
std::vector<double> to_coefs(const Grid &g, const std::vector<double> &fr, bool use_v) {
    std::vector<double> c(fr.begin(), fr.end());
    const int64_t P = g.P;
    for (int64_t p = 0; p < P; ++p) {
        const double v = fr[6 * P + p];
        c[6 * P + p] = v > 0.0 ? (use_v ? 1.0 / v : 1.0) : 0.0;
    }
    return c;
}

}  // namespace

// row classes of every cell (kFaceActive / kFaceVacuum bits) from the
// coefficient blocks ax ay az lx ly lz vinv of one level
std::vector<uint8_t> row_flags(const Grid &g, const std::vector<double> &c) {
    const int64_t P = g.P;
    std::vector<uint8_t> fl(P, 0);
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                const int64_t p = pidx(g, i, j, k);
                const int idx[3] = {i, j, k};
                bool vac = true;
                for (int a = 0; a < 3; ++a)
                    if (((g.pmc >> a) & 1) && idx[a] == 0) vac = false;
                for (int dz = -1; dz <= 1 && vac; ++dz)
                    for (int dy = -1; dy <= 1 && vac; ++dy)
                        for (int dx = -1; dx <= 1 && vac; ++dx) {
                            const int64_t q = p + dx + (int64_t)dy * g.sy + (int64_t)dz * g.sz;
                            for (int b = 0; b < 7; ++b)
                                if (c[b * P + q] != 1.0) { vac = false; break; }
                        }
                uint8_t f = 0;
                for (int a = 0; a < 3; ++a)
                    if (c[a * P + p] != 0.0) f |= (uint8_t)((kFaceActive << a) | (vac ? (kFaceVacuum << a) : 0));
                fl[p] = f;
            }
    return fl;
}

// One tabulated row (see cut_term): the weights of the row of K + G at the
// face of component comp in cell p for its 15 stored entries, read off by
// evaluating the row on unit vectors in a 3^3 window of cells around the
// face (local strides 3 and 9), then a and the diagonal d0; written to
// dst[t * stride], t = 0 .. kCutW - 1.  An inactive face gets zeros.
static void tab_row(const Grid &g, const std::vector<double> &c, const Coefs<double> &cg, int comp, int64_t p,
                    double *dst, int64_t stride) {
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    const double ih2 = 1.0 / (g.h * g.h);
    if (!(c[comp * P + p] > 0.0)) {
        for (int t = 0; t < kCutW; ++t) dst[t * stride] = 0.0;
        return;
    }
    double cw[7 * 27], xw[3 * 27];
    Coefs<double> cl;
    cl.ax = cw; cl.ay = cw + 27; cl.az = cw + 54; cl.lx = cw + 81; cl.ly = cw + 108; cl.lz = cw + 135;
    cl.vinv = cw + 162;
    cl.flags = nullptr;
    for (int a = 0; a < 7; ++a)
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di)
                    cw[a * 27 + 13 + di + 3 * dj + 9 * dk] = c[a * P + p + di + dj * dy + dk * dz];
    std::fill(xw, xw + 3 * 27, 0.0);
    for (int t = 0; t < kCutTerms; ++t) {
        const CutTerm ct = cut_term(comp, t);
        double &slot = xw[ct.comp * 27 + 13 + ct.di + 3 * ct.dj + 9 * ct.dk];
        slot = 1.0;
        double v;
        if (comp == 0) v = row_x<double, true>(cl, xw, xw + 27, xw + 54, 13, 3, 9);
        else if (comp == 1) v = row_y<double, true>(cl, xw, xw + 27, xw + 54, 13, 3, 9);
        else v = row_z<double, true>(cl, xw, xw + 27, xw + 54, 13, 3, 9);
        dst[t * stride] = ih2 * v;
        slot = 0.0;
    }
    const int64_t kk = p / dz, rr = p - kk * dz, jj = rr / dy;
    const int i = (int)(rr - jj * dy) - 1, j = (int)jj - 1, k = (int)kk - 1;
    dst[kCutTerms * stride] = c[comp * P + p];
    dst[(kCutTerms + 1) * stride] = diag_of<double>(cg, comp, p, dy, dz, ih2, 0.0) +
                                    ih2 * pmc_diag_extra<double>(g, cg.lx, cg.ly, cg.lz, comp, i, j, k, p);
}

// A row that the 3^3 rule of row_flags leaves out can still be a vacuum row:
// the rule looks at every coefficient of the cells around, the row at the
// few that enter it.  Every active row without the vacuum bit and away from
// the PMC planes (where ghost images couple a face to itself) is tabulated;
// one whose weights are exactly those of the 7-point vacuum stencil (own
// component 6/h^2 and -1/h^2, no cross terms, a = 1, diagonal 6/h^2) gets
// the bit, so that it takes the short path (the same matrix row, summed in
// another order).  Threaded over planes.
static void refine_vacuum_flags(const Grid &g, const std::vector<double> &c, std::vector<uint8_t> &fl) {
    const Coefs<double> cg = coefs_of(c.data(), g.P);
    const double ih2 = 1.0 / (g.h * g.h);
    auto work = [&](int k0, int k1) {
        double w[kCutW];
        for (int k = k0; k < k1; ++k)
            for (int j = 0; j < g.ny; ++j)
                for (int i = 0; i < g.nx; ++i) {
                    const int idx[3] = {i, j, k};
                    bool pmc = false;
                    for (int a = 0; a < 3; ++a)
                        if (((g.pmc >> a) & 1) && idx[a] == 0) pmc = true;
                    if (pmc) continue;
                    const int64_t p = pidx(g, i, j, k);
                    for (int comp = 0; comp < 3; ++comp) {
                        if (!(fl[p] & (kFaceActive << comp)) || (fl[p] & (kFaceVacuum << comp))) continue;
                        tab_row(g, c, cg, comp, p, w, 1);
                        bool vac = w[0] == 6.0 * ih2 && w[kCutTerms] == 1.0 && w[kCutTerms + 1] == 6.0 * ih2;
                        for (int t = 1; t < 7 && vac; ++t) vac = w[t] == -ih2;
                        for (int t = 7; t < kCutTerms && vac; ++t) vac = w[t] == 0.0;
                        if (vac) fl[p] |= (uint8_t)(kFaceVacuum << comp);
                    }
                }
    };
    const int nt = std::max(1, std::min(16, g.nz));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back(work, (int)((int64_t)g.nz * t / nt), (int)((int64_t)g.nz * (t + 1) / nt));
    for (auto &t : th) t.join();
}

// The tables of a level: its components' cut lists (component c's rows,
// term-major, starting at kCutW * cut_off[c]) and its list of cells with a
// cut row (the three components' rows of each cell: entry (comp, t) of cell
// e at (comp * kCutW + t) * ncells + e).  Threaded.
static void cut_tables(const Grid &g, const std::vector<double> &c, const std::vector<int32_t> &cut,
                       const int64_t cut_off[4], const std::vector<int32_t> &cells, std::vector<double> &rows_tab,
                       std::vector<double> &cells_tab) {
    const Coefs<double> cg = coefs_of(c.data(), g.P);
    rows_tab.assign((size_t)kCutW * cut.size(), 0.0);
    cells_tab.assign((size_t)3 * kCutW * cells.size(), 0.0);
    const int64_t nc = (int64_t)cells.size();
    constexpr int kParts = 4;   // threads per component list
    auto work = [&](int part) {
        if (part < 3 * kParts) {
            const int comp = part / kParts, piece = part % kParts;
            const int64_t n = cut_off[comp + 1] - cut_off[comp];
            double *T = rows_tab.data() + (size_t)kCutW * cut_off[comp];
            for (int64_t e = n * piece / kParts; e < n * (piece + 1) / kParts; ++e)
                tab_row(g, c, cg, comp, cut[cut_off[comp] + e], T + e, n);
        } else {
            const int comp = part - 3 * kParts;
            for (int64_t e = 0; e < nc; ++e)
                tab_row(g, c, cg, comp, cells[e], cells_tab.data() + (size_t)comp * kCutW * nc + e, nc);
        }
    };
    std::vector<std::thread> th;
    for (int q = 0; q < 3 * kParts + 3; ++q) th.emplace_back(work, q);
    for (auto &t : th) t.join();
}

void build_hierarchy(dm_op *op, const double *user_frac) {
    const int nl = op->opt.levels;
    int pmc = 0;
    for (int a = 0; a < 3; ++a)
        if (op->geom.bc_lo[a] == DM_BC_PMC) pmc |= 1 << a;
    Grid g0 = make_grid(op->dims[0], op->dims[1], op->dims[2], op->h, pmc);
    std::vector<double> fr;
    if (op->geom.kind == DM_GEOM_USER) {
        fr.assign(user_frac, user_frac + 7 * g0.P);
    } else if (op->geom.kind == DM_GEOM_LEVELSET) {
        compute_levelset_fractions(g0, op->geom.levelset_host, op->geom.levelset_refine, op->geom.bc_lo, fr);
    } else {
        std::unique_ptr<Body> body = make_body(op->geom);
        if (!body) throw DmError{DM_EINVAL, "unknown or unsupported geometry kind"};
        compute_fractions(*body, g0, op->geom.bc_lo, fr);
    }
    enforce_fraction_consistency(g0, fr);
    neglect_faces(g0, op->geom.a_min, fr);
    mirror_fraction_ghosts(g0, fr);
    op->frac.clear();
    op->frac.push_back(fr);
    std::vector<Grid> grids = {g0};
    for (int l = 1; l < nl; ++l) {
        const Grid &gf = grids.back();
        Grid gc = make_grid(gf.nx / 2, gf.ny / 2, gf.nz / 2, gf.h * 2.0, pmc);
        std::vector<double> fc;
        coarsen_fractions(gf, op->frac.back(), gc, fc);
        mirror_fraction_ghosts(gc, fc);
        op->frac.push_back(fc);
        grids.push_back(gc);
    }
    op->lv.resize(nl);
    for (int l = 0; l < nl; ++l) {
        Level &L = op->lv[l];
        L.g = grids[l];
        L.cut_wave_split = op->opt.cut_wave_split;
        const int64_t P = L.g.P;
        std::vector<double> c = to_coefs(L.g, op->frac[l], op->opt.grad_div_volume != 0);
        std::vector<float> c32(c.begin(), c.end());
        std::vector<uint8_t> fl = row_flags(L.g, c);
        refine_vacuum_flags(L.g, c, fl);
        // coefficient blocks followed by the P row-class bytes
        L.coef64 = op->dalloc<double>(7 * P + (P + 7) / 8);
        L.coef32 = op->dalloc<float>(7 * P + (P + 3) / 4);
        DM_HIP(hipMemcpyAsync(L.coef64, c.data(), 7 * P * sizeof(double), hipMemcpyHostToDevice, op->stream));
        DM_HIP(hipMemcpyAsync(L.coef32, c32.data(), 7 * P * sizeof(float), hipMemcpyHostToDevice, op->stream));
        DM_HIP(hipMemcpyAsync(L.coef64 + 7 * P, fl.data(), P, hipMemcpyHostToDevice, op->stream));
        DM_HIP(hipMemcpyAsync(L.coef32 + 7 * P, fl.data(), P, hipMemcpyHostToDevice, op->stream));
        // the cut (non-vacuum) rows of every component, both colours, in
        // index order
        std::vector<int32_t> cut;
        for (int comp = 0; comp < 3; ++comp) {
            L.cut_off[comp] = (int64_t)cut.size();
            for (int k = 0; k < L.g.nz; ++k)
                for (int j = 0; j < L.g.ny; ++j)
                    for (int i = 0; i < L.g.nx; ++i) {
                        const int64_t p = pidx(L.g, i, j, k);
                        if ((fl[p] & (kFaceActive << comp)) && !(fl[p] & (kFaceVacuum << comp)))
                            cut.push_back((int32_t)p);
                    }
        }
        L.cut_off[3] = (int64_t)cut.size();
        std::vector<int32_t> cutc;
        for (int k = 0; k < L.g.nz; ++k)
            for (int j = 0; j < L.g.ny; ++j)
                for (int i = 0; i < L.g.nx; ++i) {
                    const int64_t p = pidx(L.g, i, j, k);
                    if ((fl[p] & 7) & ~(fl[p] >> 3)) cutc.push_back((int32_t)p);
                }
        L.ncutc = (int64_t)cutc.size();
        std::vector<int32_t> vrows;
        for (int k = 0; k < L.g.nz; ++k)
            for (int j = 0; j < L.g.ny; ++j) {
                bool any = false;
                for (int i = 0; i < L.g.nx && !any; ++i) any = (fl[pidx(L.g, i, j, k)] >> 3) & 7;
                if (any) vrows.push_back((int32_t)(k * L.g.ny + j));
            }
        std::vector<int32_t> arows;
        for (int k = 0; k < L.g.nz; ++k)
            for (int j = 0; j < L.g.ny; ++j) {
                bool any = false;
                for (int i = 0; i < L.g.nx && !any; ++i) any = c[6 * P + pidx(L.g, i, j, k)] != 0.0;
                if (any) arows.push_back((int32_t)(k * L.g.ny + j));
            }
        std::vector<int32_t> frows;
        for (int k = 0; k < L.g.nz; ++k)
            for (int j = 0; j < L.g.ny; ++j) {
                bool any = false;
                for (int i = 0; i < L.g.nx && !any; ++i) any = fl[pidx(L.g, i, j, k)] & 7;
                if (any) frows.push_back((int32_t)(k * L.g.ny + j));
            }
        // tabulated rows of the cut lists and of the cells with a cut row
        {
            std::vector<double> tab, ctab;
            cut_tables(L.g, c, cut, L.cut_off, cutc, tab, ctab);
            auto upload = [&](const std::vector<double> &t, double *&d64, float *&d32) {
                if (t.empty()) return;
                std::vector<float> t32(t.begin(), t.end());
                d64 = op->dalloc<double>(t.size());
                d32 = op->dalloc<float>(t.size());
                DM_HIP(hipMemcpyAsync(d64, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
                DM_HIP(hipMemcpyAsync(d32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice, op->stream));
                DM_HIP(hipStreamSynchronize(op->stream));
            };
            upload(tab, L.cutw64, L.cutw32);
            upload(ctab, L.cellw64, L.cellw32);
        }
        L.nfrows = (int64_t)frows.size();
        if (!frows.empty()) {
            L.frows = op->dalloc<int32_t>(frows.size());
            DM_HIP(hipMemcpyAsync(L.frows, frows.data(), frows.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  op->stream));
        }
        L.narows = (int64_t)arows.size();
        if (!arows.empty()) {
            L.arows = op->dalloc<int32_t>(arows.size());
            DM_HIP(hipMemcpyAsync(L.arows, arows.data(), arows.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  op->stream));
        }
        L.nvrows = (int64_t)vrows.size();
        if (!vrows.empty()) {
            L.vrows = op->dalloc<int32_t>(vrows.size());
            DM_HIP(hipMemcpyAsync(L.vrows, vrows.data(), vrows.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  op->stream));
        }
        if (!cutc.empty()) {
            L.cutc = op->dalloc<int32_t>(cutc.size());
            DM_HIP(hipMemcpyAsync(L.cutc, cutc.data(), cutc.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  op->stream));
        }
        if (P > INT32_MAX) throw DmError{DM_EINVAL, "grid too large for 32-bit row lists"};
        if (!cut.empty()) {
            L.cut = op->dalloc<int32_t>(cut.size());
            DM_HIP(hipMemcpyAsync(L.cut, cut.data(), cut.size() * sizeof(int32_t), hipMemcpyHostToDevice, op->stream));
        }
        if (l == 0) {
            // units of 16 doubles of a face vector holding an active face or
            // a PMC ghost image (rows of a mirrored plane at index -1)
            const int64_t n = 3 * P, nu = (n + kSpanUnit - 1) / kSpanUnit;
            std::vector<uint8_t> live(nu, 0);
            const int nn[3] = {L.g.nx, L.g.ny, L.g.nz};
            for (int k = -1; k <= L.g.nz; ++k)
                for (int j = -1; j <= L.g.ny; ++j)
                    for (int i = -1; i <= L.g.nx; ++i) {
                        const int idx[3] = {i, j, k};
                        const int64_t p = pidx(L.g, i, j, k);
                        bool owned = true, ghost = false;
                        for (int a = 0; a < 3; ++a) {
                            if (idx[a] < 0 || idx[a] >= nn[a]) owned = false;
                            if (idx[a] == -1 && ((L.g.pmc >> a) & 1)) ghost = true;
                        }
                        for (int a = 0; a < 3; ++a)
                            if (ghost || (owned && (fl[p] & (kFaceActive << a)))) live[(a * P + p) / kSpanUnit] = 1;
                    }
            std::vector<int32_t> units;
            for (int64_t u = 0; u < nu; ++u)
                if (live[u]) units.push_back((int32_t)u);
            op->nvunit = (int64_t)units.size();
            if (!units.empty()) {
                op->vunit = op->dalloc<int32_t>(units.size());
                DM_HIP(hipMemcpyAsync(op->vunit, units.data(), units.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                      op->stream));
            }
        }
        DM_HIP(hipStreamSynchronize(op->stream));
        L.sweight = 1.0 / (std::ldexp(1.0, l) * op->h * op->h);
        int64_t naf = 0, nac = 0;  // owned entries only (not PMC ghosts)
        for (int k = 0; k < L.g.nz; ++k)
            for (int j = 0; j < L.g.ny; ++j)
                for (int i = 0; i < L.g.nx; ++i) {
                    const int64_t p = pidx(L.g, i, j, k);
                    for (int c = 0; c < 3; ++c) naf += op->frac[l][c * P + p] > 0.0;
                    nac += op->frac[l][6 * P + p] > 0.0;
                }
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
    {
        int64_t m = 1;
        for (const Level &L : op->lv) m = std::max(m, L.max_cut_rows());
        op->cut_s = op->dalloc<double>((size_t)m * kMaxRhs);
    }
    // level-0 masks and weights over the owned (non-ghost) entries:
    //   fmask  1 on active faces;  cmask 1 on active cells;
    //   wface  W: 1/2 per PMC plane the face lies in (the face is shared with
    //          its mirror image), else 1 -- the half-cavity pencil
    //          (W K, W A) is the symmetric restriction of the full cavity's;
    //   wa = W a and wainv = W / a (inner product and residual norm weights)
    const Grid &g = op->lv[0].g;
    const int64_t P0 = g.P;
    std::vector<double> fm(3 * P0, 0.0), cm(P0, 0.0), wf(3 * P0, 0.0), wa(3 * P0, 0.0), wi(3 * P0, 0.0);
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                const int64_t p = pidx(g, i, j, k);
                const int idx[3] = {i, j, k};
                cm[p] = op->frac[0][6 * P0 + p] > 0.0 ? 1.0 : 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double a = op->frac[0][c * P0 + p];
                    if (!(a > 0.0)) continue;
                    double w = 1.0;
                    if (((pmc >> c) & 1) && idx[c] == 0) w = 0.5;
                    fm[c * P0 + p] = 1.0;
                    wf[c * P0 + p] = w;
                    wa[c * P0 + p] = w * a;
                    wi[c * P0 + p] = w / a;
                }
            }
    op->fmask = op->dalloc<double>(3 * P0);
    op->cmask = op->dalloc<double>(P0);
    op->wface = op->dalloc<double>(3 * P0);
    op->wa = op->dalloc<double>(3 * P0);
    op->wainv = op->dalloc<double>(3 * P0);
    DM_HIP(hipMemcpyAsync(op->fmask, fm.data(), fm.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipMemcpyAsync(op->cmask, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipMemcpyAsync(op->wface, wf.data(), wf.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipMemcpyAsync(op->wa, wa.data(), wa.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
    DM_HIP(hipMemcpyAsync(op->wainv, wi.data(), wi.size() * sizeof(double), hipMemcpyHostToDevice, op->stream));
    // units of kSpanUnit doubles of a level-0 cell vector holding an active
    // cell or a PMC ghost image (index -1 on a PMC axis)
    {
        std::vector<uint8_t> live((P0 + kSpanUnit - 1) / kSpanUnit, 0);
        const int nn[3] = {g.nx, g.ny, g.nz};
        for (int k = -1; k <= g.nz; ++k)
            for (int j = -1; j <= g.ny; ++j)
                for (int i = -1; i <= g.nx; ++i) {
                    const int idx[3] = {i, j, k};
                    const int64_t p = pidx(g, i, j, k);
                    bool owned = true, ghost = false;
                    for (int a = 0; a < 3; ++a) {
                        if (idx[a] < 0 || idx[a] >= nn[a]) owned = false;
                        if (idx[a] == -1 && ((pmc >> a) & 1)) ghost = true;
                    }
                    if (ghost || (owned && cm[p] != 0.0)) live[p / kSpanUnit] = 1;
                }
        std::vector<int32_t> units;
        for (int64_t u = 0; u < (int64_t)live.size(); ++u)
            if (live[u]) units.push_back((int32_t)u);
        op->ncunit = (int64_t)units.size();
        if (!units.empty()) {
            op->cunit = op->dalloc<int32_t>(units.size());
            DM_HIP(hipMemcpyAsync(op->cunit, units.data(), units.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  op->stream));
        }
    }
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
    std::vector<double> c = to_coefs(g, op->frac.back(), op->opt.grad_div_volume != 0);
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
    if (n > kMaxCoarse)
        throw DmError{DM_EINVAL, "coarsest level has " + std::to_string(n) + " active faces (limit " +
                                     std::to_string(kMaxCoarse) + "): use more multigrid levels"};
    std::vector<double> Md((size_t)n * n, 0.0), e(3 * P, 0.0);
    for (int col = 0; col < n; ++col) {
        const int64_t pc = idx[col] % P;
        e[idx[col]] = 1.0;
        mirror_faces_host(g, e.data());
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
        mirror_faces_host(g, e.data());
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
        // odd mirror across a PMC plane: the neighbour is -psi, the face counts twice
        {
            const int i = (int)(p % dy) - 1, j = (int)((p / dy) % (g.ny + 2)) - 1, kk = (int)(p / dz) - 1;
            if ((g.pmc & 1) && i == 0) d += wt[0];
            if ((g.pmc & 2) && j == 0) d += wt[2];
            if ((g.pmc & 4) && kk == 0) d += wt[4];
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
