// extern "C" entry points of dm.h: argument checks, error mapping, stream
// handling.  Every entry point synchronises its stream before returning.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <thread>

#include "geometry.h"
#include "learned.h"
#include "op.h"

namespace dm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const DmError &e) {
        set_error(e.msg);
        return e.code;
    } catch (const HipError &e) {
        set_error(std::string(hipGetErrorString(e.e)) + " in " + e.where);
        return DM_EHIP;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return DM_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return DM_EINVAL;
    }
}

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

hipStream_t stream_of(dm_op *op, void *stream) {
    return stream ? (hipStream_t)stream : op->stream;
}

// run `f` on the op's device, then synchronise and surface launch errors
template <class F>
int on_device(dm_op *op, void *stream, F &&f) {
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(op->device));
        hipStream_t s = stream_of(op, stream);
        const int rc = f(s);
        DM_HIP(hipGetLastError());
        DM_HIP(hipStreamSynchronize(s));
        return rc;
    });
}

bool valid_geometry(const dm_geometry *g, std::string &why) {
    if (!g) {
        why = "geometry is NULL";
        return false;
    }
    if (g->kind < DM_GEOM_BOX || g->kind > DM_GEOM_LEVELSET) {
        why = "unknown geometry kind";
        return false;
    }
    if (g->kind == DM_GEOM_ELLIPSOID)
        for (int a = 0; a < 3; ++a)
            if (!(g->semi_axes[a] > 0.0)) {
                why = "ellipsoid semi-axes must be positive";
                return false;
            }
    if (g->kind == DM_GEOM_USER && !g->user_fractions_host) {
        why = "user geometry without fractions";
        return false;
    }
    if (g->kind == DM_GEOM_LEVELSET && (!g->levelset_host || g->levelset_refine < 1 || g->levelset_refine > 64)) {
        why = "level-set geometry needs levelset_host and levelset_refine in 1..64";
        return false;
    }
    for (int a = 0; a < 3; ++a)
        if (g->bc_lo[a] != DM_BC_PEC && g->bc_lo[a] != DM_BC_PMC) {
            why = "bc_lo must be DM_BC_PEC or DM_BC_PMC";
            return false;
        }
    if (!(g->a_min >= 0.0 && g->a_min < 1.0)) {
        why = "a_min must be in [0, 1)";
        return false;
    }
    return true;
}

// PMC planes: refresh the ghost layer of a caller face / cell vector that a
// kernel reads across the plane (writes the caller's padding only)
void fill_ghosts(const Level &L, int prec, const void *v, bool cells, hipStream_t s) {
    if (!L.g.pmc) return;
    if (cells) launch_mirror_cells(L.g, (double *)v, s);
    else if (prec == 64) launch_mirror_faces<double>(L.g, (double *)v, s);
    else launch_mirror_faces<float>(L.g, (float *)v, s);
}

int auto_levels(const int d[3]) {
    int l = 1, n[3] = {d[0], d[1], d[2]};
    while (n[0] % 2 == 0 && n[1] % 2 == 0 && n[2] % 2 == 0 &&
           std::max(n[0], std::max(n[1], n[2])) > 8 && std::min(n[0], std::min(n[1], n[2])) >= 4) {
        for (int a = 0; a < 3; ++a) n[a] /= 2;
        ++l;
    }
    return l;
}

}  // namespace
}  // namespace dm

using namespace dm;


static void free_op(dm_op *op) {
    if (!op) return;
    if (op->net) op->net->op = nullptr;
    invalidate_graphs(op);
    hipSetDevice(op->device);
    if (op->stream) hipStreamSynchronize(op->stream);
    for (void *p : op->allocs) hipFree(p);
    if (op->hres) hipHostFree(op->hres);
    if (op->bk_hres) hipHostFree(op->bk_hres);
    if (op->hres2) hipHostFree(op->hres2);
    if (op->ln_hflag) hipHostFree(op->ln_hflag);
    if (op->bk_hsc2) hipHostFree(op->bk_hsc2);   // bk_hres2 lies inside bk_hres
    if (op->stream) hipStreamDestroy(op->stream);
    delete op;
}

extern "C" {

void dm_default_options(dm_options *opt) {
    if (!opt) return;
    opt->levels = 0;
    opt->nu_pre = 2;
    opt->nu_post = 2;
    opt->fgmres_restart = 30;
    opt->verbose = 0;
    opt->cut_wave_split = 65536;
    opt->learned_patience = 1;
    opt->grad_div_volume = 1;
    opt->tilde_transfers = 0;
    opt->krylov_basis_f32 = 0;
}

void dm_default_eig_options(dm_eig_options *opt) {
    if (!opt) return;
    opt->solve_mode = DM_SOLVE_FGMRES_MG64;
    opt->inner_rtol = 1e-11;
    opt->proj_rtol = 1e-13;
    opt->block = 4;
    opt->max_basis = 40;
    opt->max_restarts = 20;
    opt->verbose = 0;
    opt->start_dev = nullptr;
}

const char *dm_strerror(int code) {
    switch (code) {
        case DM_OK: return "success";
        case DM_NOT_CONVERGED: return "iteration limit reached before the tolerance (partial result)";
        case DM_EINVAL: return "invalid argument";
        case DM_ENOMEM: return "out of memory";
        case DM_EHIP: return "HIP runtime error";
        case DM_ESINGULAR: return "coarsest operator singular at this shift";
        case DM_EBREAKDOWN: return "Krylov breakdown";
        case DM_ENAN: return "NaN or Inf encountered";
        case DM_ENODEVICE: return "no HIP device available";
        default: return "unknown status code";
    }
}

const char *dm_last_error_message(void) { return dm::g_last_error.c_str(); }

int dm_compute_fractions(const dm_geometry *geom, const int dims[3], double h, double *out_host) {
    return guarded([&]() -> int {
        std::string why;
        if (!valid_geometry(geom, why)) return fail(DM_EINVAL, why);
        if (!dims || dims[0] < 2 || dims[1] < 2 || dims[2] < 2) return fail(DM_EINVAL, "dims must be >= 2");
        if (!(h > 0.0)) return fail(DM_EINVAL, "h must be positive");
        if (!out_host) return fail(DM_EINVAL, "out_host is NULL");
        if (geom->kind == DM_GEOM_USER) return fail(DM_EINVAL, "user geometry has no computed fractions");
        int pmc = 0;
        for (int a = 0; a < 3; ++a)
            if (geom->bc_lo[a] == DM_BC_PMC) pmc |= 1 << a;
        Grid g = make_grid(dims[0], dims[1], dims[2], h, pmc);
        std::vector<double> fr;
        if (geom->kind == DM_GEOM_LEVELSET) {
            compute_levelset_fractions(g, geom->levelset_host, geom->levelset_refine, geom->bc_lo, fr);
        } else {
            std::unique_ptr<Body> body = make_body(*geom);
            if (!body) return fail(DM_EINVAL, "geometry kind not available");
            compute_fractions(*body, g, geom->bc_lo, fr);
        }
        enforce_fraction_consistency(g, fr);
        neglect_faces(g, geom->a_min, fr);
        mirror_fraction_ghosts(g, fr);
        std::memcpy(out_host, fr.data(), fr.size() * sizeof(double));
        return DM_OK;
    });
}

int dm_build_operator(const dm_geometry *geom, const int dims[3], double h, double sigma,
                      const dm_options *opt, dm_op **out) {
    if (!out) return fail(DM_EINVAL, "out is NULL");
    *out = nullptr;
    dm_op *op = nullptr;
    const int rc = guarded([&]() -> int {
        std::string why;
        if (!valid_geometry(geom, why)) return fail(DM_EINVAL, why);
        if (!dims || dims[0] < 2 || dims[1] < 2 || dims[2] < 2) return fail(DM_EINVAL, "dims must be >= 2");
        if (!(h > 0.0) || !std::isfinite(h)) return fail(DM_EINVAL, "h must be positive");
        if (!std::isfinite(sigma)) return fail(DM_EINVAL, "sigma must be finite");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(DM_ENODEVICE, "no HIP device");
        op = new dm_op();
        op->geom = *geom;
        for (int a = 0; a < 3; ++a) op->dims[a] = dims[a];
        op->h = h;
        op->sigma = sigma;
        if (opt) op->opt = *opt;
        else dm_default_options(&op->opt);
        if (op->opt.levels <= 0) op->opt.levels = auto_levels(dims);
        if (op->opt.nu_pre < 0 || op->opt.nu_post < 0 || op->opt.fgmres_restart < 1 ||
            op->opt.fgmres_restart > kMaxDots - 2 || op->opt.cut_wave_split < 0 ||
            op->opt.learned_patience < 0 || (op->opt.grad_div_volume != 0 && op->opt.grad_div_volume != 1) ||
            (op->opt.tilde_transfers != 0 && op->opt.tilde_transfers != 1) ||
            (op->opt.krylov_basis_f32 != 0 && op->opt.krylov_basis_f32 != 1))
            return fail(DM_EINVAL, "bad smoothing, restart, wave-split or variant option");
        const int div = 1 << (op->opt.levels - 1);
        for (int a = 0; a < 3; ++a)
            if (dims[a] % div != 0 || dims[a] / div < 1)
                return fail(DM_EINVAL, "dims not divisible by 2^(levels-1)");
        DM_HIP(hipGetDevice(&op->device));
        noalloc_init(op->device);   // the no-allocation entry point's scratch on this device
        DM_HIP(hipStreamCreate(&op->stream));
        build_hierarchy(op, geom->user_fractions_host);
        if (op->lv[0].n_act_faces == 0) return fail(DM_EINVAL, "the geometry leaves no active face on this grid");
        factor_coarse(op);
        DM_HIP(hipStreamSynchronize(op->stream));
        return DM_OK;
    });
    if (rc != DM_OK) {
        free_op(op);
        return rc;
    }
    *out = op;
    return DM_OK;
}

void dm_destroy(dm_op *op) { free_op(op); }

int dm_set_shift(dm_op *op, double sigma) {
    if (!op) return fail(DM_EINVAL, "op is NULL");
    if (!std::isfinite(sigma)) return fail(DM_EINVAL, "sigma must be finite");
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(op->device));
        const double old = op->sigma;
        op->sigma = sigma;
        invalidate_graphs(op);
        try {
            factor_coarse(op);
        } catch (...) {
            op->sigma = old;
            factor_coarse(op);
            throw;
        }
        return DM_OK;
    });
}

int dm_field_layout(const dm_op *op, int level, int64_t out[7]) {
    if (!op || !out) return fail(DM_EINVAL, "NULL argument");
    if (level < 0 || level >= op->nlev()) return fail(DM_EINVAL, "level out of range");
    const Level &L = op->lv[level];
    out[0] = L.g.nx;
    out[1] = L.g.ny;
    out[2] = L.g.nz;
    out[3] = L.g.P;
    out[4] = L.n_act_faces;
    out[5] = L.n_act_cells;
    out[6] = op->nlev();
    return DM_OK;
}

int dm_get_fractions(const dm_op *op, int level, double *out_host) {
    if (!op || !out_host) return fail(DM_EINVAL, "NULL argument");
    if (level < 0 || level >= op->nlev()) return fail(DM_EINVAL, "level out of range");
    std::memcpy(out_host, op->frac[level].data(), op->frac[level].size() * sizeof(double));
    return DM_OK;
}

int dm_apply(dm_op *op, int which, int prec, int level, const void *x, void *y, void *stream) {
    if (!op || !x || !y) return fail(DM_EINVAL, "NULL argument");
    if (level < 0 || level >= op->nlev()) return fail(DM_EINVAL, "level out of range");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    if (which < DM_APPLY_M || which > DM_APPLY_S) return fail(DM_EINVAL, "unknown operator");
    if (which >= DM_APPLY_DA && prec != 64) return fail(DM_EINVAL, "scalar operators are FP64 only");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        const Level &L = op->lv[level];
        fill_ghosts(L, prec, x, which == DM_APPLY_DT || which == DM_APPLY_S, s);
        switch (which) {
            case DM_APPLY_M:
            case DM_APPLY_K: {
                const int kind = which == DM_APPLY_M ? AK_M : AK_K;
                if (prec == 64)
                    launch_apply<double>(L.g, L.coef64, op->sigma, kind, nullptr, (const double *)x, (double *)y, s,
                                         L.cut_cells());
                else
                    launch_apply<float>(L.g, L.coef32, (float)op->sigma, kind, nullptr, (const float *)x, (float *)y, s,
                                        L.cut_cells());
                break;
            }
            case DM_APPLY_A:
                if (prec == 64) launch_apply_A_t<double>(L.g, L.coef64, (const double *)x, (double *)y, s);
                else launch_apply_A_t<float>(L.g, L.coef32, (const float *)x, (float *)y, s);
                break;
            case DM_APPLY_DA:
                launch_div_DA(L.g, L.coef64, (const double *)x, (double *)y, s);
                break;
            case DM_APPLY_DT:
                // y = D^T x on active faces: grad_sub with zero input and scale -1
                DM_HIP(hipMemsetAsync(y, 0, 3 * L.g.P * sizeof(double), s));
                launch_grad_sub(L.g, L.coef64, (const double *)x, (double *)y, (double *)y, -1.0, s);
                break;
            case DM_APPLY_S:
                launch_s_apply(L.g, L.coef64, 1.0 / (L.g.h * L.g.h), 0, nullptr, (const double *)x, (double *)y, s);
                break;
        }
        return DM_OK;
    });
}

int dm_residual(dm_op *op, int prec, int level, const void *f, const void *x, void *r, void *stream) {
    if (!op || !f || !x || !r) return fail(DM_EINVAL, "NULL argument");
    if (level < 0 || level >= op->nlev()) return fail(DM_EINVAL, "level out of range");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        const Level &L = op->lv[level];
        fill_ghosts(L, prec, x, false, s);
        if (prec == 64)
            launch_apply<double>(L.g, L.coef64, op->sigma, AK_RESID, (const double *)f, (const double *)x, (double *)r, s,
                                 L.cut_cells());
        else
            launch_apply<float>(L.g, L.coef32, (float)op->sigma, AK_RESID, (const float *)f, (const float *)x, (float *)r, s,
                                L.cut_cells());
        return DM_OK;
    });
}

int dm_smooth(dm_op *op, int prec, int level, int n_sweeps, int reverse, const void *f, void *x,
              void *stream) {
    if (!op || !f || !x) return fail(DM_EINVAL, "NULL argument");
    if (level < 0 || level >= op->nlev()) return fail(DM_EINVAL, "level out of range");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    if (n_sweeps < 0) return fail(DM_EINVAL, "n_sweeps must be >= 0");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        const Level &L = op->lv[level];
        fill_ghosts(L, prec, x, false, s);
        for (int it = 0; it < n_sweeps; ++it)
            for (int q = 0; q < 6; ++q) {
                const int cls = reverse ? 5 - q : q;
                const int comp = cls / 2, col = cls % 2;
                // the first colour of each component leaves the second's cross sums
                const ClassList cl = L.cut_list(comp, col, (q % 2) == 0 ? kPairFirst : kPairSecond, op->cut_s);
                if (prec == 64)
                    launch_smooth<double>(L.g, L.coef64, op->sigma, comp, col, (const double *)f, (double *)x, s, cl);
                else
                    launch_smooth<float>(L.g, L.coef32, (float)op->sigma, comp, col, (const float *)f, (float *)x, s, cl);
            }
        return DM_OK;
    });
}

int dm_restrict(dm_op *op, int prec, int level, const void *r, void *fc, void *stream) {
    if (!op || !r || !fc) return fail(DM_EINVAL, "NULL argument");
    if (level < 0 || level + 1 >= op->nlev()) return fail(DM_EINVAL, "level out of range");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        const Level &F = op->lv[level], &C = op->lv[level + 1];
        fill_ghosts(F, prec, r, false, s);
        if (prec == 64) launch_restrict<double>(F.g, C.g, C.coef64, (const double *)r, (double *)fc, s);
        else launch_restrict<float>(F.g, C.g, C.coef32, (const float *)r, (float *)fc, s);
        return DM_OK;
    });
}

int dm_prolong_add(dm_op *op, int prec, int level, const void *xc, void *x, void *stream) {
    if (!op || !xc || !x) return fail(DM_EINVAL, "NULL argument");
    if (level < 0 || level + 1 >= op->nlev()) return fail(DM_EINVAL, "level out of range");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        const Level &F = op->lv[level], &C = op->lv[level + 1];
        fill_ghosts(F, prec, x, false, s);
        if (prec == 64) launch_prolong_add<double>(F.g, C.g, F.coef64, C.coef64, (const double *)xc, (double *)x, s);
        else launch_prolong_add<float>(F.g, C.g, F.coef32, C.coef32, (const float *)xc, (float *)x, s);
        return DM_OK;
    });
}

int dm_vcycle(dm_op *op, int prec, const void *f, void *x, void *stream) {
    if (!op || !f || !x) return fail(DM_EINVAL, "NULL argument");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        fill_ghosts(op->lv[0], prec, f, false, s);
        // through the solver's captured V-cycle graph, between its fixed buffers
        ensure_krylov_small(op);
        const int64_t n = op->n0();
        const size_t bytes = n * (prec == 64 ? sizeof(double) : sizeof(float));
        void *fin = prec == 64 ? (void *)op->gv_f64 : (void *)op->fg_f32;
        void *xout = prec == 64 ? (void *)op->gv_x64 : (void *)op->fg_x32;
        DM_HIP(hipMemcpyAsync(fin, f, bytes, hipMemcpyDeviceToDevice, s));
        vcycle_graphed(op, prec, s);
        DM_HIP(hipMemcpyAsync(x, xout, bytes, hipMemcpyDeviceToDevice, s));
        return DM_OK;
    });
}

int dm_vcycle_block(dm_op *op, int prec, int nrhs, const void *const *f, void *const *x, void *stream) {
    if (op && op->opt.tilde_transfers) return fail(DM_EINVAL, "tilde transfers: single-vector V-cycles only");
    if (!op || !f || !x) return fail(DM_EINVAL, "NULL argument");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(DM_EINVAL, "nrhs must be 1..4");
    for (int q = 0; q < nrhs; ++q)
        if (!f[q] || !x[q]) return fail(DM_EINVAL, "NULL vector in the block");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        ensure_block(op, prec);
        const int64_t n = op->n0();
        const size_t es = prec == 64 ? sizeof(double) : sizeof(float);
        char *fin = prec == 64 ? (char *)op->lv[0].bf64 : (char *)op->lv[0].bf32;
        char *xout = prec == 64 ? (char *)op->lv[0].bx64 : (char *)op->lv[0].bx32;
        for (int q = 0; q < nrhs; ++q) {
            fill_ghosts(op->lv[0], prec, f[q], false, s);
            DM_HIP(hipMemcpyAsync(fin + q * n * es, f[q], n * es, hipMemcpyDeviceToDevice, s));
        }
        vcycle_block_graphed(op, prec, nrhs, s);
        for (int q = 0; q < nrhs; ++q)
            DM_HIP(hipMemcpyAsync(x[q], xout + q * n * es, n * es, hipMemcpyDeviceToDevice, s));
        return DM_OK;
    });
}

int dm_project(dm_op *op, const double *b, double *out, double rtol, void *stream) {
    if (!op || !b || !out) return fail(DM_EINVAL, "NULL argument");
    if (!(rtol > 0.0)) return fail(DM_EINVAL, "rtol must be positive");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        fill_ghosts(op->lv[0], 64, b, false, s);
        return project(op, b, out, rtol, 2000, s, nullptr);
    });
}

int dm_project_block(dm_op *op, int nrhs, const double *const *b, double *const *out, double rtol, void *stream) {
    if (!op || !b || !out) return fail(DM_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(DM_EINVAL, "nrhs must be 1..4");
    if (!(rtol > 0.0)) return fail(DM_EINVAL, "rtol must be positive");
    for (int q = 0; q < nrhs; ++q)
        if (!b[q] || !out[q]) return fail(DM_EINVAL, "NULL vector in the block");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        for (int q = 0; q < nrhs; ++q) fill_ghosts(op->lv[0], 64, b[q], false, s);
        return project_block(op, nrhs, b, out, rtol, 2000, s, nullptr);
    });
}

int dm_solve(dm_op *op, int mode, const double *f, double *x, double rtol, int maxit,
             dm_solve_info *info, void *stream) {
    if (!op || !f || !x) return fail(DM_EINVAL, "NULL argument");
    if (mode < DM_SOLVE_PCG64 || mode > DM_SOLVE_FGMRES_MG32_LEARNED) return fail(DM_EINVAL, "unknown solve mode");
    if (mode == DM_SOLVE_FGMRES_MG32_LEARNED && !op->net)
        return fail(DM_EINVAL, "learned solve mode without an attached network");
    if (!(rtol > 0.0) || maxit < 1) return fail(DM_EINVAL, "rtol must be positive and maxit >= 1");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        fill_ghosts(op->lv[0], 64, f, false, s);
        return solve(op, mode, f, x, rtol, maxit, info, s);
    });
}

int dm_solve_pcg_noalloc(dm_op *op, const double *f, double *x, double rtol, int maxit, dm_solve_info *info,
                         void *stream) {
    if (!op || !f || !x) return fail(DM_EINVAL, "NULL argument");
    if (!(rtol > 0.0) || maxit < 1) return fail(DM_EINVAL, "rtol must be positive and maxit >= 1");
    const int64_t n = op->n0();
    if ((uint64_t)4 * (uint64_t)n * sizeof(double) > (uint64_t)DM_NOALLOC_SCRATCH_BYTES)
        return fail(DM_EINVAL, "grid too large for the no-allocation scratch (4 * 3P doubles > " +
                                   std::to_string(DM_NOALLOC_SCRATCH_BYTES) + " bytes)");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        double *work = noalloc_scratch(op->device);
        if (!work) throw DmError{DM_EHIP, "no-allocation scratch not set up on this device"};
        fill_ghosts(op->lv[0], 64, f, false, s);
        return solve_pcg_with(op, f, x, rtol, maxit, info, s, work);
    });
}

int dm_sample_e(dm_op *op, const double *b, double lambda, int npts, const double *pts, double *e, void *stream) {
    if (!op || !b || (npts > 0 && (!pts || !e))) return fail(DM_EINVAL, "NULL argument");
    if (!(lambda > 0.0) || npts < 0) return fail(DM_EINVAL, "lambda must be positive and npts >= 0");
    if (npts == 0) return DM_OK;
    return on_device(op, stream, [&](hipStream_t s) -> int {
        const Level &L = op->lv[0];
        // points and values: a temporary device buffer of this call
        struct Buf {
            double *p = nullptr;
            ~Buf() { if (p) (void)hipFree(p); }
        } buf;
        DM_HIP(hipMalloc((void **)&buf.p, (size_t)6 * npts * sizeof(double)));
        double *dp = buf.p;
        DM_HIP(hipMemcpyAsync(dp, pts, (size_t)3 * npts * sizeof(double), hipMemcpyHostToDevice, s));
        fill_ghosts(L, 64, b, false, s);
        launch_sample_e(L.g, L.coef64, b, std::sqrt(lambda), npts, dp, dp + (size_t)3 * npts, s);
        DM_HIP(hipMemcpyAsync(e, dp + (size_t)3 * npts, (size_t)3 * npts * sizeof(double), hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        return DM_OK;
    });
}

int dm_solve_block(dm_op *op, int mode, int nrhs, const double *const *f, double *const *x, double rtol,
                   int maxit, dm_solve_info *info, void *stream) {
    if (op && op->opt.tilde_transfers) return fail(DM_EINVAL, "tilde transfers: single-vector solves only");
    if (!op || !f || !x) return fail(DM_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(DM_EINVAL, "nrhs must be 1..4");
    if (mode < DM_SOLVE_FGMRES_MG64 || mode > DM_SOLVE_FGMRES_MG32_LEARNED)
        return fail(DM_EINVAL, "block solves take the FGMRES modes");
    if (mode == DM_SOLVE_FGMRES_MG32_LEARNED && !op->net)
        return fail(DM_EINVAL, "learned solve mode without an attached network");
    if (!(rtol > 0.0) || maxit < 1) return fail(DM_EINVAL, "rtol must be positive and maxit >= 1");
    for (int q = 0; q < nrhs; ++q)
        if (!f[q] || !x[q]) return fail(DM_EINVAL, "NULL vector in the block");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        for (int q = 0; q < nrhs; ++q) fill_ghosts(op->lv[0], 64, f[q], false, s);
        return solve_block(op, mode, nrhs, f, x, rtol, maxit, info, s);
    });
}

int dm_eigs(dm_op *op, int k, double sigma, double tol, uint64_t seed, const dm_eig_options *opt,
            double *lambda_host, double *vecs_dev, double *residuals_host, dm_eig_info *info,
            void *stream) {
    if (op && op->opt.tilde_transfers) return fail(DM_EINVAL, "tilde transfers: linear solves only (no eigensolve)");
    if (!op || !lambda_host) return fail(DM_EINVAL, "NULL argument");
    if (k < 1) return fail(DM_EINVAL, "k must be >= 1");
    if (!(tol > 0.0)) return fail(DM_EINVAL, "tol must be positive");
    dm_eig_options o;
    if (opt) o = *opt;
    else dm_default_eig_options(&o);
    if (o.block < 1 || o.max_restarts < 0 || !(o.inner_rtol > 0) || !(o.proj_rtol > 0) ||
        o.solve_mode < DM_SOLVE_PCG64 || o.solve_mode > DM_SOLVE_FGMRES_MG32_LEARNED ||
        (o.solve_mode == DM_SOLVE_FGMRES_MG32_LEARNED && !op->net))
        return fail(DM_EINVAL, "bad eig options");
    if (sigma != op->sigma) {
        const int rc = dm_set_shift(op, sigma);
        if (rc != DM_OK) return rc;
    }
    return on_device(op, stream, [&](hipStream_t s) -> int {
        return eigs(op, k, tol, seed, o, lambda_host, vecs_dev, residuals_host, info, s);
    });
}

/* ---- batched cavities ---------------------------------------------------- */

static void free_batch(dm_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    batch_release(b);
    for (dm_op *op : b->ops) {
        op->batch = nullptr;
        dm_destroy(op);
    }
    for (hipEvent_t e : b->ev_in) (void)hipEventDestroy(e);
    if (b->ev_done) (void)hipEventDestroy(b->ev_done);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int dm_batch_create(int count, const dm_geometry *geoms, const int *dims, const double *h, double sigma,
                    const dm_options *opt, dm_batch **out) {
    if (opt && (opt->tilde_transfers || !opt->grad_div_volume))
        return fail(DM_EINVAL, "batched cavities: the solver-sensitivity variants are not supported");
    if (!out) return fail(DM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !geoms || !dims || !h) return fail(DM_EINVAL, "bad batch arguments");
    dm_batch *b = new dm_batch();
    for (int i = 0; i < count; ++i) {
        dm_op *op = nullptr;
        const int rc = dm_build_operator(&geoms[i], dims + 3 * i, h[i], sigma, opt, &op);
        if (rc != DM_OK) {
            free_batch(b);
            return rc;
        }
        op->batch_index = i;
        b->ops.push_back(op);
    }
    const int rc = guarded([&]() -> int {
        DM_HIP(hipGetDevice(&b->device));
        DM_HIP(hipStreamCreate(&b->stream));
        b->ev_in.resize(count, nullptr);
        for (int i = 0; i < count; ++i) DM_HIP(hipEventCreateWithFlags(&b->ev_in[i], hipEventDisableTiming));
        DM_HIP(hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
        b->pending.assign(count, 0);
        batch_setup(b);
        return DM_OK;
    });
    if (rc != DM_OK) {
        free_batch(b);
        return rc;
    }
    *out = b;
    return DM_OK;
}

void dm_batch_destroy(dm_batch *b) { free_batch(b); }

int dm_batch_member(dm_batch *b, int i, dm_op **op) {
    if (!b || !op || i < 0 || i >= (int)b->ops.size()) return fail(DM_EINVAL, "bad batch member");
    *op = b->ops[i];
    return DM_OK;
}

int dm_batch_info(const dm_batch *b, dm_batch_stats *st) {
    if (!b || !st) return fail(DM_EINVAL, "NULL argument");
    st->count = (int)b->ops.size();
    st->threads_per_block = b->tpb;
    for (int q = 0; q < 3; ++q) st->tuned_ms[q] = b->tuned_ms[q];
    st->launches_per_vcycle = b->nsteps;
    int64_t c = 0, a = 0;
    for (const dm_op *op : b->ops) {
        const dm::Grid &g = op->lv[0].g;
        c += (int64_t)g.nx * g.ny * g.nz;
        a += op->lv[0].n_act_faces;
    }
    st->cells = c;
    st->active_faces = a;
    return DM_OK;
}

int dm_batch_vcycle(dm_batch *b, const float *const *f_dev, float *const *x_dev, void *stream) {
    if (!b || !f_dev || !x_dev) return fail(DM_EINVAL, "NULL argument");
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(b->device));
        hipStream_t s = stream ? (hipStream_t)stream : b->stream;
        for (size_t i = 0; i < b->ops.size(); ++i) {
            if (!f_dev[i] || !x_dev[i]) return fail(DM_EINVAL, "NULL member vector");
            DM_HIP(hipMemcpyAsync(b->ops[i]->fg_f32, f_dev[i], b->ops[i]->n0() * sizeof(float),
                                  hipMemcpyDeviceToDevice, s));
        }
        DM_HIP(hipGraphLaunch(b->graph, s));
        for (size_t i = 0; i < b->ops.size(); ++i)
            DM_HIP(hipMemcpyAsync(x_dev[i], b->ops[i]->fg_x32, b->ops[i]->n0() * sizeof(float),
                                  hipMemcpyDeviceToDevice, s));
        DM_HIP(hipStreamSynchronize(s));
        return DM_OK;
    });
}

int dm_batch_time_vcycle(dm_batch *b, int reps, double *ms) {
    if (!b || !ms || reps < 1) return fail(DM_EINVAL, "bad arguments");
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(b->device));
        hipEvent_t e0, e1;
        DM_HIP(hipEventCreate(&e0));
        DM_HIP(hipEventCreate(&e1));
        DM_HIP(hipGraphLaunch(b->graph, b->stream));
        DM_HIP(hipEventRecord(e0, b->stream));
        for (int r = 0; r < reps; ++r) DM_HIP(hipGraphLaunch(b->graph, b->stream));
        DM_HIP(hipEventRecord(e1, b->stream));
        DM_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        DM_HIP(hipEventElapsedTime(&t, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms = t / reps;
        return DM_OK;
    });
}

int dm_batch_eigs(dm_batch *b, int k, double sigma, double tol, uint64_t seed, const dm_eig_options *opt,
                  double *lambda_host, double *residuals_host, dm_eig_info *info_host, double *seconds) {
    if (!b || !lambda_host) return fail(DM_EINVAL, "NULL argument");
    if (k < 1 || !(tol > 0.0)) return fail(DM_EINVAL, "bad k or tol");
    dm_eig_options o;
    if (opt) o = *opt;
    else dm_default_eig_options(&o);
    if (o.start_dev) return fail(DM_EINVAL, "batched eigensolves draw their own start blocks");
    o.solve_mode = DM_SOLVE_FGMRES_MG32;
    const int n = (int)b->ops.size();
    // a change of shift re-factors every member and re-records the fused V-cycle
    bool reshift = false;
    for (dm_op *op : b->ops)
        if (op->sigma != sigma) {
            const int rc = dm_set_shift(op, sigma);
            if (rc != DM_OK) return rc;
            reshift = true;
        }
    if (reshift) {
        const int rc = guarded([&]() -> int {
            DM_HIP(hipSetDevice(b->device));
            batch_setup(b);
            return DM_OK;
        });
        if (rc != DM_OK) return rc;
    }
    std::vector<int> codes(n, DM_OK);
    std::vector<std::string> msgs(n);
    std::vector<dm_eig_info> infos(n);
    b->active = n;
    b->submitted = 0;
    std::fill(b->pending.begin(), b->pending.end(), 0);
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> th;
    for (int i = 0; i < n; ++i)
        th.emplace_back([&, i]() {
            dm_op *op = b->ops[i];
            op->batch = b;
            codes[i] = guarded([&]() -> int {
                DM_HIP(hipSetDevice(op->device));
                const int rc = eigs(op, k, tol, seed, o, lambda_host + (size_t)i * k, nullptr,
                                    residuals_host ? residuals_host + (size_t)i * k : nullptr, &infos[i],
                                    op->stream);
                DM_HIP(hipStreamSynchronize(op->stream));
                return rc;
            });
            if (codes[i] < 0) msgs[i] = dm_last_error_message();
            op->batch = nullptr;
            batch_leave(b);
        });
    for (auto &t : th) t.join();
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info_host)
        for (int i = 0; i < n; ++i) info_host[i] = infos[i];
    int worst = DM_OK;
    for (int i = 0; i < n; ++i) {
        if (codes[i] < 0) return fail(codes[i], "member " + std::to_string(i) + ": " + msgs[i]);
        worst = std::max(worst, codes[i]);
    }
    return worst;
}

/* ---- learned correction ------------------------------------------------- */

int dm_net_create(uint64_t seed, dm_net **out) {
    if (!out) return fail(DM_EINVAL, "NULL argument");
    *out = nullptr;
    return guarded([&]() -> int {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(DM_ENODEVICE, "no HIP device");
        dm_net *net = new dm_net();
        try {
            net_init(net, seed);
        } catch (...) {
            net_free(net);
            delete net;
            throw;
        }
        *out = net;
        return DM_OK;
    });
}

void dm_net_destroy(dm_net *net) {
    if (!net) return;
    if (net->op) net->op->net = nullptr;
    net_free(net);
    delete net;
}

int dm_net_get_weights(const dm_net *net, float *weights_host) {
    if (!net || !weights_host) return fail(DM_EINVAL, "NULL argument");
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(net->device));
        DM_HIP(hipMemcpy(weights_host, net->w32, kNetWeights * sizeof(float), hipMemcpyDeviceToHost));
        return DM_OK;
    });
}

int dm_net_set_weights(dm_net *net, const float *weights_host) {
    if (!net || !weights_host) return fail(DM_EINVAL, "NULL argument");
    for (int q = 0; q < kNetWeights; ++q)
        if (!std::isfinite(weights_host[q])) return fail(DM_ENAN, "non-finite network weight");
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(net->device));
        net_upload_weights(net, weights_host);
        net->step = 0;
        DM_HIP(hipMemset(net->adam_m, 0, kNetWeights * sizeof(float)));
        DM_HIP(hipMemset(net->adam_v, 0, kNetWeights * sizeof(float)));
        return DM_OK;
    });
}

int dm_net_attach(dm_op *op, dm_net *net) {
    if (!op) return fail(DM_EINVAL, "NULL operator");
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(op->device));
        DM_HIP(hipStreamSynchronize(op->stream));
        net_attach(op, net);
        DM_HIP(hipDeviceSynchronize());
        return DM_OK;
    });
}

int dm_net_apply(dm_op *op, const double *r_dev, double scale, double *out_dev, void *stream) {
    if (!op || !r_dev || !out_dev) return fail(DM_EINVAL, "NULL argument");
    if (!op->net) return fail(DM_EINVAL, "no network attached");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        net_apply(op, r_dev, scale, out_dev, s);
        return DM_OK;
    });
}

int dm_net_loss_grad(dm_op *op, int kind, const double *r_dev, const double *e_dev, double scale,
                     double *loss_host, float *grad_host, void *stream) {
    if (!op || !r_dev || !loss_host) return fail(DM_EINVAL, "NULL argument");
    if (kind != DM_NET_LOSS_ERROR && kind != DM_NET_LOSS_RESIDUAL) return fail(DM_EINVAL, "unknown loss");
    if (kind == DM_NET_LOSS_ERROR && !e_dev) return fail(DM_EINVAL, "error loss needs e");
    if (!op->net) return fail(DM_EINVAL, "no network attached");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        *loss_host = net_loss_grad(op, kind, r_dev, e_dev, scale, s);
        if (grad_host)
            DM_HIP(hipMemcpyAsync(grad_host, op->net->grad, kNetWeights * sizeof(float),
                                  hipMemcpyDeviceToHost, s));
        return DM_OK;
    });
}

int dm_net_make_pair(dm_op *op, uint64_t seed, double *r_dev, double *e_dev, void *stream) {
    if (!op || !r_dev || !e_dev) return fail(DM_EINVAL, "NULL argument");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        net_make_pair(op, seed, r_dev, e_dev, s);
        return DM_OK;
    });
}

int dm_net_train(dm_op *op, int kind, int steps, float lr, uint64_t seed, float *loss_host, void *stream) {
    if (!op) return fail(DM_EINVAL, "NULL operator");
    if (kind != DM_NET_LOSS_ERROR && kind != DM_NET_LOSS_RESIDUAL) return fail(DM_EINVAL, "unknown loss");
    if (!op->net) return fail(DM_EINVAL, "no network attached");
    if (steps < 0 || !(lr > 0.f)) return fail(DM_EINVAL, "steps must be >= 0 and lr > 0");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        net_train(op, kind, steps, lr, seed, loss_host, s);
        return DM_OK;
    });
}

int dm_net_train_pairs(dm_op *op, int kind, int npairs, const double *const *r_dev, const double *const *e_dev,
                       float lr, float *loss_host, void *stream) {
    if (!op || (npairs > 0 && !r_dev)) return fail(DM_EINVAL, "NULL argument");
    if (kind != DM_NET_LOSS_ERROR && kind != DM_NET_LOSS_RESIDUAL) return fail(DM_EINVAL, "unknown loss");
    if (kind == DM_NET_LOSS_ERROR && !e_dev) return fail(DM_EINVAL, "error loss needs e");
    if (!op->net) return fail(DM_EINVAL, "no network attached");
    if (npairs < 0 || !(lr > 0.f)) return fail(DM_EINVAL, "npairs must be >= 0 and lr > 0");
    for (int i = 0; i < npairs; ++i)
        if (!r_dev[i] || (kind == DM_NET_LOSS_ERROR && !e_dev[i])) return fail(DM_EINVAL, "NULL pair vector");
    return on_device(op, stream, [&](hipStream_t s) -> int {
        net_train_pairs(op, kind, npairs, r_dev, e_dev, lr, loss_host, s);
        return DM_OK;
    });
}

// nrhs == 0: the one-vector kernels; 1..kMaxRhs: their block forms
static int time_kernel_impl(dm_op *op, int kernel, int prec, int level, int nrhs, int reps,
                            double *ms_per_launch) {
    if (!op || !ms_per_launch) return fail(DM_EINVAL, "NULL argument");
    if (prec != 64 && prec != 32) return fail(DM_EINVAL, "prec must be 64 or 32");
    if (kernel < DM_KERNEL_APPLY || kernel > DM_KERNEL_NET) return fail(DM_EINVAL, "unknown kernel");
    if (kernel == DM_KERNEL_NET && (!op->net || level != 0 || prec != 32 || nrhs > 1))
        return fail(DM_EINVAL, "network timing: attach a network; level 0, prec 32, one vector");
    if (reps < 1) return fail(DM_EINVAL, "reps must be >= 1");
    if (nrhs < 0 || nrhs > kMaxRhs) return fail(DM_EINVAL, "nrhs must be 1..4");
    const bool pair = kernel == DM_KERNEL_RESTRICT || kernel == DM_KERNEL_PROLONG;
    if (level < 0 || level >= op->nlev() || (pair && level + 1 >= op->nlev()) ||
        (kernel == DM_KERNEL_VCYCLE && level != 0))
        return fail(DM_EINVAL, "level out of range for this kernel");
    return guarded([&]() -> int {
        DM_HIP(hipSetDevice(op->device));
        hipStream_t s = op->stream;
        const Level &L = op->lv[level];
        const int nv = std::max(nrhs, 1);
        const int64_t n = 3 * L.g.P;
        const int64_t nc = pair ? 3 * op->lv[level + 1].g.P : 0;
        const size_t es = prec == 64 ? sizeof(double) : sizeof(float);
        std::vector<void *> tmp;
        auto alloc = [&](int64_t cnt) {
            void *p = nullptr;
            DM_HIP(hipMalloc(&p, std::max<int64_t>(cnt, 1) * es));
            tmp.push_back(p);
            return p;
        };
        int rc = DM_OK;
        try {
            char *x = (char *)alloc(nv * n), *f = (char *)alloc(nv * n), *y = (char *)alloc(nv * n);
            char *c = (char *)alloc(std::max(nv * nc, (int64_t)1));
            double *g64 = nullptr;
            DM_HIP(hipMalloc((void **)&g64, n * sizeof(double)));
            tmp.push_back(g64);
            // seeded data on the active faces of `level` (mask = its area fractions)
            std::vector<double> m(n);
            for (int64_t p = 0; p < n; ++p) m[p] = op->frac[level][p] > 0.0 ? 1.0 : 0.0;
            double *mask = nullptr;
            DM_HIP(hipMalloc((void **)&mask, n * sizeof(double)));
            tmp.push_back(mask);
            DM_HIP(hipMemcpyAsync(mask, m.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
            for (int v = 0; v < nv; ++v)
                for (int q = 0; q < 2; ++q) {
                    launch_randn(n, 97 + 2 * v + q, 0, mask, g64, s);
                    char *dst = (q == 0 ? x : f) + v * n * es;
                    if (prec == 64) launch_copy(n, g64, (double *)dst, s);
                    else launch_cast<double, float>(g64, (float *)dst, n, s);
                }
            DM_HIP(hipMemsetAsync(y, 0, nv * n * es, s));
            DM_HIP(hipMemsetAsync(c, 0, std::max(nv * nc, (int64_t)1) * es, s));
            const Level &C = op->lv[std::min(level + 1, op->nlev() - 1)];
            auto one = [&]() {
                switch (kernel) {
                    case DM_KERNEL_APPLY:
                    case DM_KERNEL_RESIDUAL: {
                        const int kind = kernel == DM_KERNEL_APPLY ? AK_M : AK_RESID;
                        if (prec == 64) launch_apply<double>(L.g, L.coef64, op->sigma, kind, (double *)f, (double *)x, (double *)y, s, L.cut_cells());
                        else launch_apply<float>(L.g, L.coef32, (float)op->sigma, kind, (float *)f, (float *)x, (float *)y, s, L.cut_cells());
                        break;
                    }
                    case DM_KERNEL_SMOOTH:
                    case DM_KERNEL_SWEEP:
                        for (int q = 0; q < (kernel == DM_KERNEL_SMOOTH ? 1 : 6); ++q) {
                            // a sweep pairs the two colours of a component as the V-cycle does
                            const ClassList cl = kernel == DM_KERNEL_SMOOTH
                                                     ? L.cut_list(0, 0)
                                                     : L.cut_list(q / 2, q % 2, q % 2 ? kPairSecond : kPairFirst, op->cut_s);
                            if (prec == 64) launch_smooth<double>(L.g, L.coef64, op->sigma, q / 2, q % 2, (double *)f, (double *)x, s, cl);
                            else launch_smooth<float>(L.g, L.coef32, (float)op->sigma, q / 2, q % 2, (float *)f, (float *)x, s, cl);
                        }
                        break;
                    case DM_KERNEL_RESTRICT:
                        if (prec == 64) launch_restrict<double>(L.g, C.g, C.coef64, (double *)x, (double *)c, s);
                        else launch_restrict<float>(L.g, C.g, C.coef32, (float *)x, (float *)c, s);
                        break;
                    case DM_KERNEL_PROLONG:
                        if (prec == 64) launch_prolong_add<double>(L.g, C.g, L.coef64, C.coef64, (double *)c, (double *)y, s);
                        else launch_prolong_add<float>(L.g, C.g, L.coef32, C.coef32, (float *)c, (float *)y, s);
                        break;
                    case DM_KERNEL_NET:      // the network's own activation buffers
                        net_forward(op, s);
                        break;
                    case DM_KERNEL_VCYCLE:   // the solver's graph, between its own buffers
                        vcycle_graphed(op, prec, s);
                        break;
                }
            };
            auto block = [&](auto tag) {
                using T = decltype(tag);
                VPtr<T> X{}, F{}, Y{}, Cc{};
                for (int v = 0; v < nrhs; ++v) {
                    X.p[v] = (T *)x + v * n;
                    F.p[v] = (T *)f + v * n;
                    Y.p[v] = (T *)y + v * n;
                    Cc.p[v] = (T *)c + v * nc;
                }
                const T *coef = prec == 64 ? (const T *)L.coef64 : (const T *)L.coef32;
                const T *ccoef = prec == 64 ? (const T *)C.coef64 : (const T *)C.coef32;
                switch (kernel) {
                    case DM_KERNEL_APPLY:
                    case DM_KERNEL_RESIDUAL:
                        launch_apply_b<T>(L.g, coef, (T)op->sigma, kernel == DM_KERNEL_APPLY ? AK_M : AK_RESID, nrhs,
                                          as_const(F), as_const(X), Y, s, L.cut_cells());
                        break;
                    case DM_KERNEL_SMOOTH:
                    case DM_KERNEL_SWEEP:
                        for (int q = 0; q < (kernel == DM_KERNEL_SMOOTH ? 1 : 6); ++q)
                            launch_smooth_b<T>(L.g, coef, (T)op->sigma, q / 2, q % 2, nrhs, as_const(F), X, s,
                                               kernel == DM_KERNEL_SMOOTH
                                                   ? L.cut_list(q / 2, q % 2)
                                                   : L.cut_list(q / 2, q % 2, q % 2 ? kPairSecond : kPairFirst, op->cut_s));
                        break;
                    case DM_KERNEL_RESTRICT:
                        launch_restrict_b<T>(L.g, C.g, ccoef, nrhs, as_const(X), Cc, s);
                        break;
                    case DM_KERNEL_PROLONG:
                        launch_prolong_add_b<T>(L.g, C.g, coef, ccoef, nrhs, as_const(Cc), Y, s);
                        break;
                    case DM_KERNEL_VCYCLE:
                        vcycle_block_graphed(op, prec, nrhs, s);
                        break;
                }
            };
            auto launch = [&]() {
                if (nrhs == 0) one();
                else if (prec == 64) block(double{});
                else block(float{});
            };
            launch();
            launch();
            hipEvent_t e0, e1;
            DM_HIP(hipEventCreate(&e0));
            DM_HIP(hipEventCreate(&e1));
            DM_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) launch();
            DM_HIP(hipEventRecord(e1, s));
            DM_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            DM_HIP(hipEventElapsedTime(&ms, e0, e1));
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            DM_HIP(hipGetLastError());
            *ms_per_launch = (double)ms / reps;
        } catch (...) {
            hipStreamSynchronize(s);
            for (void *p : tmp) hipFree(p);
            throw;
        }
        DM_HIP(hipStreamSynchronize(s));
        for (void *p : tmp) hipFree(p);
        return rc;
    });
}

int dm_time_kernel(dm_op *op, int kernel, int prec, int level, int reps, double *ms_per_launch) {
    return time_kernel_impl(op, kernel, prec, level, 0, reps, ms_per_launch);
}

int dm_time_block_kernel(dm_op *op, int kernel, int prec, int level, int nrhs, int reps, double *ms_per_launch) {
    if (nrhs < 1) return fail(DM_EINVAL, "nrhs must be 1..4");
    return time_kernel_impl(op, kernel, prec, level, nrhs, reps, ms_per_launch);
}

}  // extern "C"
