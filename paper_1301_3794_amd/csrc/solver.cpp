// Host-driven solvers over the HIP kernels:
//  * V-cycles for M (FP64 or FP32) and for the scalar Laplacian S = D A D^T;
//  * the divergence projection P_DM (eq. proj) by multigrid-preconditioned CG;
//  * FGMRES (FP64, right-preconditioned by a V-cycle of either precision) and
//    PCG for M x = f (Sec. 6: the inner inversions);
//  * block Krylov--Schur on T = P_DM M^-1 A in the A-inner product
//    (eqs. fullMat, bInner) with Rayleigh quotients and residuals on (K, A).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <random>

#include "op.h"

namespace dm {

namespace {

template <class T>
struct Prec;
template <>
struct Prec<double> {
    static const double *coef(const Level &L) { return L.coef64; }
    static double *x(Level &L) { return L.x64; }
    static double *f(Level &L) { return L.f64; }
    static double *r(Level &L) { return L.r64; }
};
template <>
struct Prec<float> {
    static const float *coef(const Level &L) { return L.coef32; }
    static float *x(Level &L) { return L.x32; }
    static float *f(Level &L) { return L.f32; }
    static float *r(Level &L) { return L.r32; }
};

template <class T>
struct BPrec;
template <>
struct BPrec<double> {
    static double *x(Level &L) { return L.bx64; }
    static double *f(Level &L) { return L.bf64; }
    static double *r(Level &L) { return L.br64; }
};
template <>
struct BPrec<float> {
    static float *x(Level &L) { return L.bx32; }
    static float *f(Level &L) { return L.bf32; }
    static float *r(Level &L) { return L.br32; }
};

// the scalar block V-cycle's buffers and coefficients per precision
template <class T>
struct SPrec;
template <>
struct SPrec<double> {
    static const double *coef(const Level &L) { return L.coef64; }
    static double *x(Level &L) { return L.bsx; }
    static double *f(Level &L) { return L.bsf; }
    static double *r(Level &L) { return L.bsr; }
};
template <>
struct SPrec<float> {
    static const float *coef(const Level &L) { return L.coef32; }
    static float *x(Level &L) { return L.bsx32; }
    static float *f(Level &L) { return L.bsf32; }
    static float *r(Level &L) { return L.bsr32; }
};

// nr consecutive slots of `stride` elements from base
template <class T>
VPtr<T> slots(T *base, int64_t stride, int nr) {
    VPtr<T> v{};
    for (int q = 0; q < nr; ++q) v.p[q] = base + q * stride;
    return v;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Symmetric eigendecomposition of a small dense matrix by cyclic Jacobi
// rotations.  a: n x n row-major (destroyed); w: eigenvalues; v: columns.
void jacobi_eig(std::vector<double> a, int n, std::vector<double> &w, std::vector<double> &v) {
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

void to_device_coef(dm_op *op, const double *h, int nv, hipStream_t s) {
    DM_HIP(hipMemcpyAsync(op->dcoef, h, nv * sizeof(double), hipMemcpyHostToDevice, s));
}

// x -= mean of x over active cells (device-side, no host sync)
void demean_cells(dm_op *op, double *x, hipStream_t s) {
    const Level &L = op->lv[0];
    launch_mdot(1, x, 0, op->cmask, nullptr, L.g.P, op->part, op->dres, s);
    launch_sub_masked(L.g.P, op->cmask, op->dres, 1.0 / (double)std::max<int64_t>(1, L.n_act_cells), x, s);
}


// FGMRES(m), right-preconditioned.  The basis is kept unnormalised: column
// u_i of V stands for v_i = sc[i] u_i, and the preconditioner output Z_i for
// z_i = sc[i] Z_i (the V-cycles and the learned correction are equivariant
// under scaling, and FGMRES accepts any z_i).  The scales are folded into the
// host-side coefficients, so a step makes two passes over the basis:
// (1) d = U^T w; (2) w -= U c fused with d2 = U^T w and |w|^2.  The product
// w = M Z_j is formed in the next column's slot and stays there as u_{j+1}.
// A third pass (w -= U c2, classical Gram--Schmidt's second correction) runs
// only when the remaining projection |h2| exceeds kReorth of the new
// column's norm; otherwise the Arnoldi relation M z_j = V h + hn v_{j+1}
// holds with the first-pass coefficients and the basis keeps orthogonality
// to 1e-10.  Convergence is always confirmed by the true residual.
constexpr double kReorth = 1e-10;
// The same threshold for a basis stored in FP32 (krylov_basis_f32): its
// columns are orthogonal only to FP32 rounding, so the second pass's
// projection sits near 1e-7 of the first one's whatever is done, and a
// third pass (which cannot lower it) is taken only well above that level.
constexpr double kReorthF32 = 1e-5;

int fgmres(dm_op *op, int mode, const double *f, double *x, double rtol, int maxit,
           dm_solve_info *info, hipStream_t s) {
    ensure_krylov(op);
    const Level &L = op->lv[0];
    const int64_t n = op->n0();
    const int m = op->fg_m;
    double *V = op->fg_V, *Z = op->fg_Z;
    const Span sp = op->vspan();
    DM_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
    const double bnorm = std::sqrt(dot1(op, f, f, nullptr, n, s, sp));
    int total = 0, restarts = 0;
    int learned_rejections = 0;   // learned mode: rejected corrections in this solve
    double rel = 0.0;
    if (bnorm == 0.0) {
        if (info) *info = dm_solve_info{0, 0, 0.0, 0.0, 0, 0};
        return DM_OK;
    }
    if (!std::isfinite(bnorm)) throw DmError{DM_ENAN, "right-hand side is not finite"};
    // c, c3, cx: coefficients of passes (2), (3) and of the update of x, each
    // in its own host array (a queued copy never reads an overwritten array)
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1), h2(m + 1), c(m + 1),
        c3(m + 1), cx(m + 1), sc(m + 1), sc2h(m + 1);
    bool conv = false;
    while (true) {
        if (total == 0) launch_copy(n, f, V, s);
        else launch_apply<double>(L.g, L.coef64, op->sigma, AK_RESID, f, x, V, s, L.cut_cells());
        const double beta = std::sqrt(dot1(op, V, V, nullptr, n, s, sp));
        if (!std::isfinite(beta)) throw DmError{DM_ENAN, "FGMRES residual is not finite"};
        rel = beta / bnorm;
        if (beta <= rtol * bnorm) {
            conv = true;
            break;
        }
        if (total >= maxit) break;
        sc[0] = 1.0 / beta;
        sc2h[0] = sc[0] * sc[0];
        DM_HIP(hipMemcpyAsync(op->sc2d, sc2h.data(), sizeof(double), hipMemcpyHostToDevice, s));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        std::fill(H.begin(), H.end(), 0.0);
        int j = 0;
        for (; j < m;) {
            double *uj = V + (int64_t)j * n, *zj = Z + (int64_t)j * n, *w = V + (int64_t)(j + 1) * n;
            precondition(op, mode, uj, zj, s, &learned_rejections);
            launch_apply<double>(L.g, L.coef64, op->sigma, AK_M, nullptr, zj, w, s, L.cut_cells());
            // (1) d = U^T w, then (2) w -= U c with c_i = sc_i^2 d_i formed on
            // the device, fused with d2 = U^T w and |w|^2: one host sync
            launch_mdot(j + 1, V, n, w, nullptr, n, op->part, op->dres, s, sp);
            launch_maxpy_mdot_norm(j + 1, V, n, op->dres, w, n, op->part, op->dres2, s, op->sc2d, sp);
            DM_HIP(hipMemcpyAsync(op->hres, op->dres, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
            DM_HIP(hipMemcpyAsync(op->hres2, op->dres2, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
            DM_HIP(hipStreamSynchronize(s));
            for (int i = 0; i <= j; ++i) h[i] = sc[i] * sc[j] * op->hres[i];   // true coefficients
            const double wn2 = op->hres2[j + 1] * sc[j] * sc[j];
            double c2 = 0.0;
            for (int i = 0; i <= j; ++i) {
                h2[i] = sc[i] * sc[j] * op->hres2[i];
                c2 += h2[i] * h2[i];
            }
            double hn;
            if (c2 > kReorth * kReorth * wn2) {
                // (3) second classical Gram--Schmidt correction
                for (int i = 0; i <= j; ++i) {
                    c3[i] = sc[i] * sc[i] * op->hres2[i];
                    h[i] += h2[i];
                }
                to_device_coef(op, c3.data(), j + 1, s);
                launch_maxpy(j + 1, V, n, op->dcoef, w, n, 0, s, nullptr, sp);
                hn = std::sqrt(std::max(wn2 - c2, 0.0));
            } else {
                hn = std::sqrt(wn2);
            }
            if (!std::isfinite(hn)) throw DmError{DM_ENAN, "FGMRES iterate is not finite"};
            sc[j + 1] = hn > 0.0 ? sc[j] / hn : 0.0;
            sc2h[j + 1] = sc[j + 1] * sc[j + 1];
            DM_HIP(hipMemcpyAsync(op->sc2d + j + 1, &sc2h[j + 1], sizeof(double), hipMemcpyHostToDevice, s));
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double r = std::hypot(a, b);
            cs[j] = r > 0 ? a / r : 1.0;
            sn[j] = r > 0 ? b / r : 0.0;
            H[(size_t)j * m + j] = r;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            ++j;
            if (std::fabs(g[j]) <= rtol * bnorm || total >= maxit || hn == 0.0) break;
        }
        for (int i = j - 1; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k < j; ++k) t -= H[(size_t)i * m + k] * y[k];
            y[i] = t / H[(size_t)i * m + i];
        }
        for (int i = 0; i < j; ++i) cx[i] = -y[i] * sc[i];   // x += sum y_i z_i, z_i = sc_i Z_i
        to_device_coef(op, cx.data(), j, s);
        launch_maxpy(j, Z, n, op->dcoef, x, n, 0, s, nullptr, sp);
        ++restarts;
    }
    if (info) {
        info->iterations = total;
        info->restarts = restarts > 0 ? restarts - 1 : 0;
        info->rel_residual = rel;
    }
    return conv ? DM_OK : DM_NOT_CONVERGED;
}

// CG preconditioned by the FP64 V-cycle (direct launches, the op's level
// buffers), with the work vectors r, z, p, q (n = 3P doubles each) given
int pcg_work(dm_op *op, const double *f, double *x, double rtol, int maxit, dm_solve_info *info,
             hipStream_t s, double *r, double *z, double *p, double *q) {
    const Level &L = op->lv[0];
    const int64_t n = op->n0();
    launch_zero<double>(n, x, s);
    const double bnorm = std::sqrt(dot1(op, f, f, op->wface, n, s));
    if (bnorm == 0.0) {
        if (info) *info = dm_solve_info{0, 0, 0.0, 0.0, 0, 0};
        return DM_OK;
    }
    launch_copy(n, f, r, s);
    vcycle<double>(op, 0, r, z, s);
    launch_copy(n, z, p, s);
    double rz = dot1(op, r, z, op->wface, n, s);
    int it = 0;
    double rel = 1.0;
    bool conv = false;
    while (it < maxit) {
        launch_apply<double>(L.g, L.coef64, op->sigma, AK_M, nullptr, p, q, s, L.cut_cells());
        const double pq = dot1(op, p, q, op->wface, n, s);
        if (!(pq > 0.0)) throw DmError{pq == pq ? DM_EBREAKDOWN : DM_ENAN,
                                       "PCG: operator not positive definite at this shift"};
        const double alpha = rz / pq;
        launch_axpy(n, alpha, p, x, s);
        launch_axpy(n, -alpha, q, r, s);
        ++it;
        rel = std::sqrt(dot1(op, r, r, op->wface, n, s)) / bnorm;
        if (!std::isfinite(rel)) throw DmError{DM_ENAN, "PCG residual is not finite"};
        if (rel <= rtol) {
            conv = true;
            break;
        }
        vcycle<double>(op, 0, r, z, s);
        const double rz2 = dot1(op, r, z, op->wface, n, s);
        launch_axpby(n, 1.0, z, rz2 / rz, p, s);
        rz = rz2;
    }
    // true residual
    launch_apply<double>(L.g, L.coef64, op->sigma, AK_RESID, f, x, r, s, L.cut_cells());
    rel = std::sqrt(dot1(op, r, r, op->wface, n, s)) / bnorm;
    if (info) {
        info->iterations = it;
        info->restarts = 0;
        info->rel_residual = rel;
    }
    return conv ? DM_OK : DM_NOT_CONVERGED;
}

int pcg(dm_op *op, const double *f, double *x, double rtol, int maxit, dm_solve_info *info,
        hipStream_t s) {
    ensure_krylov(op);
    const int64_t n = op->n0();
    return pcg_work(op, f, x, rtol, maxit, info, s, op->fg_V, op->fg_V + n, op->fg_V + 2 * n, op->fg_w);
}

}  // namespace

int solve_pcg_with(dm_op *op, const double *f, double *x, double rtol, int maxit, dm_solve_info *info,
                   hipStream_t s, double *work) {
    const double t0 = now_s();
    const int64_t n = op->n0();
    const int rc = pcg_work(op, f, x, rtol, maxit, info, s, work, work + n, work + 2 * n, work + 3 * n);
    DM_HIP(hipStreamSynchronize(s));
    if (info) {
        info->seconds = now_s() - t0;
        info->learned_accepted = info->learned_rejected = 0;
    }
    return rc;
}

void ensure_proj(dm_op *op) {
    if (!op->pj_g) {
        const int64_t P = op->lv[0].g.P;
        op->pj_g = op->dalloc<double>(P);
        op->pj_psi = op->dalloc<double>(P);
        op->pj_r = op->dalloc<double>(P);
        op->pj_z = op->dalloc<double>(P);
        op->pj_p = op->dalloc<double>(P);
        op->pj_q = op->dalloc<double>(P);
    }
}

void ensure_krylov_small(dm_op *op) {
    const int64_t n = op->n0();
    if (!op->fg_w) {
        op->fg_w = op->dalloc<double>(n);
        op->fg_f32 = op->dalloc<float>(n);
        op->fg_x32 = op->dalloc<float>(n);
        op->gv_f64 = op->dalloc<double>(n);
        op->gv_x64 = op->dalloc<double>(n);
        op->dcoef = op->dalloc<double>(kMaxDots);
        op->dres2 = op->dalloc<double>(kMaxDots);
        op->sc2d = op->dalloc<double>(kMaxDots);
        DM_HIP(hipHostMalloc((void **)&op->hres2, kMaxDots * sizeof(double), hipHostMallocDefault));
    }
}

void ensure_krylov(dm_op *op) {
    ensure_krylov_small(op);
    const int64_t n = op->n0();
    if (!op->fg_V) {
        const int m = op->opt.fgmres_restart;
        op->fg_m = m;
        // at least 3 vectors: PCG borrows r, z, p from this block
        op->fg_V = op->dalloc<double>((size_t)std::max(m + 1, 3) * n);
        op->fg_Z = op->dalloc<double>((size_t)m * n);
    }
}


double dot1(dm_op *op, const double *x, const double *y, const double *wt, int64_t n,
            hipStream_t s, Span sp) {
    dots(op, 1, x, 0, y, wt, n, s, sp);
    return op->hres[0];
}

void precondition(dm_op *op, int mode, const double *v, double *z, hipStream_t s, int *rejections) {
    const int64_t n = op->n0();
    if (mode == DM_SOLVE_FGMRES_MG32 || mode == DM_SOLVE_FGMRES_MG32_LEARNED) {
        // as in precondition_block: casts over the listed units only
        launch_cast<double, float>(v, op->fg_f32, n, s, op->vspan());
        if (op->batch && mode == DM_SOLVE_FGMRES_MG32) batch_vcycle_lockstep(op, s);
        else vcycle_graphed(op, 32, s);
        launch_cast<float, double>(op->fg_x32, z, n, s, op->vspan());
        if (mode == DM_SOLVE_FGMRES_MG32_LEARNED) {
            int none = 0;
            net_correct_patient(op, v, z, rejections ? rejections : &none, s);
        }
    } else {
        launch_copy(n, v, op->gv_f64, s);
        vcycle_graphed(op, 64, s);
        launch_copy(n, op->gv_x64, z, s);
    }
}


// ---------------------------------------------------------------------------
void dots(dm_op *op, int nv, const double *V, int64_t ld, const double *w, const double *wt,
          int64_t n, hipStream_t s, Span sp) {
    launch_mdot(nv, V, ld, w, wt, n, op->part, op->dres, s, sp);
    DM_HIP(hipMemcpyAsync(op->hres, op->dres, nv * sizeof(double), hipMemcpyDeviceToHost, s));
    DM_HIP(hipStreamSynchronize(s));
}

template <class T>
void vcycle(dm_op *op, int l, const T *f, T *x, hipStream_t s) {
    Level &L = op->lv[l];
    const Grid &g = L.g;
    const T sig = (T)op->sigma;
    launch_zero<T>(3 * g.P, x, s);
    if (l == op->nlev() - 1) {
        launch_coarse_solve<T>(op->nc, op->cinv, op->cidx, f, x, s);
        launch_mirror_faces<T>(g, x, s);
        return;
    }
    const T *c = Prec<T>::coef(L);
    // the two colour updates of a component are paired: the first leaves the
    // second colour's cross-component sums in op->cut_s
    for (int it = 0; it < op->opt.nu_pre; ++it)
        for (int comp = 0; comp < 3; ++comp)
            for (int col = 0; col < 2; ++col)
                launch_smooth<T>(g, c, sig, comp, col, f, x, s,
                                 L.cut_list(comp, col, col == 0 ? kPairFirst : kPairSecond, op->cut_s));
    T *r = Prec<T>::r(L);
    launch_apply<T>(g, c, sig, AK_RESID, f, x, r, s, L.cut_cells());
    Level &C = op->lv[l + 1];
    T *fc = Prec<T>::f(C), *xc = Prec<T>::x(C);
    const T *cc = Prec<T>::coef(C);
    // tilde form (eq. fullMat2): transfers A_c^1/2 R A_f^-1/2 and A_f^-1/2 P A_c^1/2
    const bool tilde = op->opt.tilde_transfers != 0;
    if (tilde) launch_scale_a<T>(3 * g.P, c, -1, r, s);
    launch_restrict<T>(g, C.g, cc, r, fc, s);
    if (tilde) launch_scale_a<T>(3 * C.g.P, cc, +1, fc, s);
    vcycle<T>(op, l + 1, fc, xc, s);
    if (tilde) {
        launch_scale_a<T>(3 * C.g.P, cc, +1, xc, s);
        launch_zero<T>(3 * g.P, r, s);
        launch_prolong_add<T>(g, C.g, c, cc, xc, r, s);
        launch_add_scaled_a<T>(3 * g.P, c, r, x, s);
    } else {
        launch_prolong_add<T>(g, C.g, c, cc, xc, x, s);
    }
    for (int it = 0; it < op->opt.nu_post; ++it)
        for (int comp = 2; comp >= 0; --comp)
            for (int col = 1; col >= 0; --col)
                launch_smooth<T>(g, c, sig, comp, col, f, x, s,
                                 L.cut_list(comp, col, col == 1 ? kPairFirst : kPairSecond, op->cut_s));
}

template void vcycle<double>(dm_op *, int, const double *, double *, hipStream_t);
template void vcycle<float>(dm_op *, int, const float *, float *, hipStream_t);

// The V-cycle above on nr vectors at once (the level's block slots, f and x
// of level 0 included): the same operations per vector, each launch serving
// all of them.
template <class T>
void vcycle_b(dm_op *op, int l, int nr, hipStream_t s) {
    Level &L = op->lv[l];
    const Grid &g = L.g;
    const int64_t n3 = 3 * g.P;
    const T sig = (T)op->sigma;
    const VPtr<T> F = slots(BPrec<T>::f(L), n3, nr), X = slots(BPrec<T>::x(L), n3, nr);
    // the iterate starts at zero: here on the finest level, on the coarser
    // ones in the restriction that forms their right-hand side
    if (l == 0) launch_zero<T>(nr * n3, BPrec<T>::x(L), s);
    if (l == op->nlev() - 1) {
        launch_coarse_solve_b<T>(op->nc, op->cinv, op->cidx, nr, as_const(F), X, s);
        for (int q = 0; q < nr; ++q) launch_mirror_faces<T>(g, X.p[q], s);
        return;
    }
    const T *c = Prec<T>::coef(L);
    for (int it = 0; it < op->opt.nu_pre; ++it)
        for (int comp = 0; comp < 3; ++comp)
            for (int col = 0; col < 2; ++col)
                launch_smooth_b<T>(g, c, sig, comp, col, nr, as_const(F), X, s,
                                   L.cut_list(comp, col, col == 0 ? kPairFirst : kPairSecond, op->cut_s));
    const VPtr<T> R = slots(BPrec<T>::r(L), n3, nr);
    // the residual, restriction and prolongation visit only the grid rows
    // holding an active face: the residual slots, the coarse right-hand
    // sides and iterates stay zero on the others (written only here)
    launch_apply_b<T>(g, c, sig, AK_RESID, nr, as_const(F), as_const(X), R, s, L.cut_cells_rows());
    Level &C = op->lv[l + 1];
    const int64_t c3 = 3 * C.g.P;
    launch_restrict_b<T>(g, C.g, Prec<T>::coef(C), nr, as_const(R), slots(BPrec<T>::f(C), c3, nr), s,
                         slots(BPrec<T>::x(C), c3, nr), C.frows, C.nfrows);
    vcycle_b<T>(op, l + 1, nr, s);
    launch_prolong_add_b<T>(g, C.g, c, Prec<T>::coef(C), nr, as_const(slots(BPrec<T>::x(C), c3, nr)), X, s,
                            L.frows, L.nfrows);
    for (int it = 0; it < op->opt.nu_post; ++it)
        for (int comp = 2; comp >= 0; --comp)
            for (int col = 1; col >= 0; --col)
                launch_smooth_b<T>(g, c, sig, comp, col, nr, as_const(F), X, s,
                                   L.cut_list(comp, col, col == 1 ? kPairFirst : kPairSecond, op->cut_s));
}

void svcycle(dm_op *op, int l, const double *f, double *x, hipStream_t s) {
    Level &L = op->lv[l];
    const Grid &g = L.g;
    launch_zero<double>(g.P, x, s);
    if (l == op->nlev() - 1) {
        launch_coarse_solve<double>(op->ns, op->sinv, op->sidx, f, x, s);
        launch_mirror_cells(g, x, s);
        return;
    }
    for (int it = 0; it < op->opt.nu_pre; ++it)
        for (int col = 0; col < 2; ++col) launch_s_smooth(g, L.coef64, L.sweight, col, f, x, s);
    launch_s_apply(g, L.coef64, L.sweight, 1, f, x, L.sr, s);
    Level &C = op->lv[l + 1];
    launch_s_restrict(g, C.g, C.coef64, L.sr, C.sf, s);
    svcycle(op, l + 1, C.sf, C.sx, s);
    launch_s_prolong_add(g, C.g, L.coef64, C.sx, x, s);
    for (int it = 0; it < op->opt.nu_post; ++it)
        for (int col = 1; col >= 0; --col) launch_s_smooth(g, L.coef64, L.sweight, col, f, x, s);
}

// svcycle() on nr vectors at once (the level's scalar block slots), in FP64
// or in FP32 (FP32 coefficient blocks and slots)
template <class T>
void svcycle_b(dm_op *op, int l, int nr, hipStream_t s) {
    using S = SPrec<T>;
    Level &L = op->lv[l];
    const Grid &g = L.g;
    const int64_t P = g.P;
    const T *c = S::coef(L);
    const VPtr<T> F = slots(S::f(L), P, nr), X = slots(S::x(L), P, nr);
    if (l == 0) launch_zero<T>(nr * P, S::x(L), s);   // coarser levels: zeroed by the restriction
    if (l == op->nlev() - 1) {
        launch_coarse_solve_b<T>(op->ns, op->sinv, op->sidx, nr, as_const(F), X, s);
        for (int q = 0; q < nr; ++q) launch_mirror_cells<T>(g, X.p[q], s);
        return;
    }
    for (int it = 0; it < op->opt.nu_pre; ++it)
        for (int col = 0; col < 2; ++col)
            launch_s_smooth_b<T>(g, c, L.sweight, col, nr, as_const(F), X, s, L.arows, L.narows);
    const VPtr<T> R = slots(S::r(L), P, nr);
    // residual and transfers on the grid rows holding an active cell (the
    // slots stay zero on the others)
    launch_s_apply_b<T>(g, c, L.sweight, 1, nr, as_const(F), as_const(X), R, s, L.arows, L.narows);
    Level &C = op->lv[l + 1];
    launch_s_restrict_b<T>(g, C.g, S::coef(C), nr, as_const(R), slots(S::f(C), C.g.P, nr), s,
                           slots(S::x(C), C.g.P, nr), C.arows, C.narows);
    svcycle_b<T>(op, l + 1, nr, s);
    launch_s_prolong_add_b<T>(g, C.g, c, nr, as_const(slots(S::x(C), C.g.P, nr)), X, s, L.arows, L.narows);
    for (int it = 0; it < op->opt.nu_post; ++it)
        for (int col = 1; col >= 0; --col)
            launch_s_smooth_b<T>(g, c, L.sweight, col, nr, as_const(F), X, s, L.arows, L.narows);
}

// ---------------------------------------------------------------------------
// V-cycles replayed from captured HIP graphs.  A V-cycle is a fixed sequence
// of ~27 launches per level, short on the coarse levels, so per-launch
// overhead dominates its time; the graph is recorded once per operator (on
// the op's own stream) between fixed buffers and launched on the caller's
// stream.  The captured sequence holds kernels only (no memsets).  Graphs
// bake in the shift and the coarsest inverse, so a change of shift drops them.
// ---------------------------------------------------------------------------
namespace {

template <class F>
hipGraphExec_t capture(dm_op *op, F &&record) {
    hipGraph_t gph = nullptr;
    hipGraphExec_t exec = nullptr;
    DM_HIP(hipStreamBeginCapture(op->stream, hipStreamCaptureModeThreadLocal));
    try {
        record(op->stream);
    } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(op->stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        throw;
    }
    DM_HIP(hipStreamEndCapture(op->stream, &gph));
    const hipError_t e = hipGraphInstantiate(&exec, gph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gph);
    DM_HIP(e);
    return exec;
}

}  // namespace

void invalidate_graphs(dm_op *op) {
    for (hipGraphExec_t *e : {&op->g_vc32, &op->g_vc64, &op->g_svc}) {
        if (*e) (void)hipGraphExecDestroy(*e);
        *e = nullptr;
    }
    for (int q = 0; q <= kMaxRhs; ++q)
        for (hipGraphExec_t *e : {&op->g_vb32[q], &op->g_vb64[q], &op->g_svb[q], &op->g_svb32[q]}) {
            if (*e) (void)hipGraphExecDestroy(*e);
            *e = nullptr;
        }
}

void ensure_block_results(dm_op *op) {
    if (!op->bk_dres) {
        const size_t nd = (size_t)kMaxRhs * kMaxDots;
        op->bk_dres = op->dalloc<double>(2 * nd);
        op->bk_dres2 = op->bk_dres + nd;
        op->bk_dcoef = op->dalloc<double>(nd);
        DM_HIP(hipHostMalloc((void **)&op->bk_hres, 2 * nd * sizeof(double), hipHostMallocDefault));
        op->bk_hres2 = op->bk_hres + nd;
        op->bk_sc2 = op->dalloc<double>(nd);
        DM_HIP(hipHostMalloc((void **)&op->bk_hsc2, nd * sizeof(double), hipHostMallocDefault));
    }
}

void ensure_block(dm_op *op, int prec) {
    op->bk_m = op->opt.fgmres_restart;   // the bases are allocated by the block FGMRES, in its precision
    ensure_block_results(op);
    for (Level &L : op->lv) {
        const size_t cnt = (size_t)kMaxRhs * 3 * L.g.P;
        if (prec == 32 && !L.bx32) {
            L.bx32 = op->dalloc<float>(cnt);
            L.bf32 = op->dalloc<float>(cnt);
            L.br32 = op->dalloc<float>(cnt);
        }
        if (prec == 64 && !L.bx64) {
            L.bx64 = op->dalloc<double>(cnt);
            L.bf64 = op->dalloc<double>(cnt);
            L.br64 = op->dalloc<double>(cnt);
        }
    }
}

void vcycle_block_graphed(dm_op *op, int prec, int nr, hipStream_t s) {
    if (nr < 1 || nr > kMaxRhs) throw DmError{DM_EINVAL, "block of 1 to 4 vectors"};
    ensure_block(op, prec);
    hipGraphExec_t &g = prec == 32 ? op->g_vb32[nr] : op->g_vb64[nr];
    if (!g)
        g = capture(op, [&](hipStream_t cs) {
            if (prec == 32) vcycle_b<float>(op, 0, nr, cs);
            else vcycle_b<double>(op, 0, nr, cs);
        });
    DM_HIP(hipGraphLaunch(g, s));
}

void vcycle_graphed(dm_op *op, int prec, hipStream_t s) {
    ensure_krylov_small(op);
    if (prec == 32) {
        if (!op->g_vc32)
            op->g_vc32 = capture(op, [&](hipStream_t cs) { vcycle<float>(op, 0, op->fg_f32, op->fg_x32, cs); });
        DM_HIP(hipGraphLaunch(op->g_vc32, s));
    } else {
        if (!op->g_vc64)
            op->g_vc64 = capture(op, [&](hipStream_t cs) { vcycle<double>(op, 0, op->gv_f64, op->gv_x64, cs); });
        DM_HIP(hipGraphLaunch(op->g_vc64, s));
    }
}

void svcycle_graphed(dm_op *op, hipStream_t s) {
    if (!op->g_svc)
        op->g_svc = capture(op, [&](hipStream_t cs) { svcycle(op, 0, op->pj_r, op->pj_z, cs); });
    DM_HIP(hipGraphLaunch(op->g_svc, s));
}

int project(dm_op *op, const double *b, double *out, double rtol, int maxit, hipStream_t s,
            int *iters) {
    ensure_proj(op);
    const Level &L = op->lv[0];
    const Grid &g = L.g;
    const int64_t P = g.P;
    double *gv = op->pj_g, *psi = op->pj_psi, *r = op->pj_r, *z = op->pj_z, *p = op->pj_p,
           *q = op->pj_q;
    launch_div_DA(g, L.coef64, b, gv, s);
    if (op->s_floating) demean_cells(op, gv, s);
    const double gnorm = std::sqrt(dot1(op, gv, gv, op->cmask, P, s));
    // Stop on the scale of the field, not of its divergence: the gradient
    // left in the output is then at most ~rtol of |b|_A, however nearly
    // divergence-free b already was (the usual case inside the eigensolve).
    const double stop = rtol * std::sqrt(dot1(op, b, b, op->wa, op->n0(), s)) / g.h;
    DM_HIP(hipMemsetAsync(psi, 0, P * sizeof(double), s));
    int it = 0;
    if (!std::isfinite(gnorm)) throw DmError{DM_ENAN, "projection input is not finite"};
    if (gnorm > stop) {
        launch_copy(P, gv, r, s);
        svcycle_graphed(op, s);            // r -> z
        if (op->s_floating) demean_cells(op, z, s);
        launch_copy(P, z, p, s);
        double rz = dot1(op, r, z, op->cmask, P, s);
        while (it < maxit) {
            launch_s_apply(g, L.coef64, L.sweight, 0, nullptr, p, q, s);
            const double pq = dot1(op, p, q, op->cmask, P, s);
            if (!(pq > 0.0)) break;
            const double alpha = rz / pq;
            launch_axpy(P, alpha, p, psi, s);
            launch_axpy(P, -alpha, q, r, s);
            ++it;
            const double rn = std::sqrt(dot1(op, r, r, op->cmask, P, s));
            if (rn <= stop) break;
            svcycle_graphed(op, s);        // r -> z
            if (op->s_floating) demean_cells(op, z, s);
            const double rz2 = dot1(op, r, z, op->cmask, P, s);
            launch_axpby(P, 1.0, z, rz2 / rz, p, s);
            rz = rz2;
        }
    }
    launch_grad_sub(g, L.coef64, psi, const_cast<double *>(b), out, 1.0, s);
    if (iters) *iters = it;
    op->last_proj_iters = it;
    return DM_OK;
}

// project() on nr vectors in lockstep: the CG iterations of every vector
// that has not met its stopping test share one block S apply and one block
// scalar V-cycle per step, and one host sync per inner product.  r and z of
// vector q live in the level-0 slots of the block scalar V-cycle.
int project_block(dm_op *op, int nr, const double *const *b, double *const *out, double rtol, int maxit,
                  hipStream_t s, int *iters, int prec) {
    if (nr < 1 || nr > kMaxRhs) throw DmError{DM_EINVAL, "block of 1 to 4 vectors"};
    if (prec != 64 && prec != 32) throw DmError{DM_EINVAL, "scalar V-cycle precision must be 64 or 32"};
    ensure_block_results(op);
    Level &L = op->lv[0];
    const Grid &g = L.g;
    const int64_t P = g.P, n = op->n0();
    if (!op->pjb_g) {
        op->pjb_g = op->dalloc<double>((size_t)kMaxRhs * P);
        op->pjb_psi = op->dalloc<double>((size_t)kMaxRhs * P);
        op->pjb_p = op->dalloc<double>((size_t)kMaxRhs * P);
        op->pjb_q = op->dalloc<double>((size_t)kMaxRhs * P);
    }
    for (Level &Lv : op->lv)
        if (!Lv.bsx) {
            Lv.bsx = op->dalloc<double>((size_t)kMaxRhs * Lv.g.P);
            Lv.bsf = op->dalloc<double>((size_t)kMaxRhs * Lv.g.P);
            Lv.bsr = op->dalloc<double>((size_t)kMaxRhs * Lv.g.P);
        }
    if (prec == 32)
        for (Level &Lv : op->lv)
            if (!Lv.bsx32) {
                Lv.bsx32 = op->dalloc<float>((size_t)kMaxRhs * Lv.g.P);
                Lv.bsf32 = op->dalloc<float>((size_t)kMaxRhs * Lv.g.P);
                Lv.bsr32 = op->dalloc<float>((size_t)kMaxRhs * Lv.g.P);
            }
    const VPtr<double> G = slots(op->pjb_g, P, nr), PSI = slots(op->pjb_psi, P, nr), PP = slots(op->pjb_p, P, nr),
                       Q = slots(op->pjb_q, P, nr), R = slots(L.bsf, P, nr), Z = slots(L.bsx, P, nr);
    VPtr<const double> B{};
    for (int q = 0; q < nr; ++q) B.p[q] = b[q];
    auto dres = [&](int q) { return op->bk_dres + (int64_t)q * kMaxDots; };
    auto hres = [&](int q) { return op->bk_hres + (int64_t)q * kMaxDots; };
    auto fetch = [&]() {
        DM_HIP(hipMemcpyAsync(op->bk_hres, op->bk_dres, (size_t)nr * kMaxDots * sizeof(double),
                              hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
    };
    // the CG's reductions and updates visit the units of the cell vectors
    // that hold an active cell or a PMC ghost image: g = D A b, the V-cycle's
    // z, S p and every combination of them are zero elsewhere (as is psi,
    // cleared below), and so stay zero there
    const Span csp = op->cspan();
    // z = B r for every slot: the FP64 V-cycle on the slots themselves, or
    // the FP32 one between two casts (the slots are consecutive)
    auto graph = [&]() {
        hipGraphExec_t &gx = prec == 64 ? op->g_svb[nr] : op->g_svb32[nr];
        if (!gx)
            gx = capture(op, [&](hipStream_t cs) {
                if (prec == 64) {
                    svcycle_b<double>(op, 0, nr, cs);
                } else {
                    launch_cast<double, float>(L.bsf, L.bsf32, (int64_t)nr * P, cs);
                    svcycle_b<float>(op, 0, nr, cs);
                    launch_cast<float, double>(L.bsx32, L.bsx, (int64_t)nr * P, cs);
                }
            });
        DM_HIP(hipGraphLaunch(gx, s));
    };
    // the vectors of the slots whose flag is set (the rest left out of a launch)
    auto pick = [&](const VPtr<double> &X, const bool *on) {
        VPtr<double> v{};
        for (int q = 0; q < nr; ++q) v.p[q] = on[q] ? X.p[q] : nullptr;
        return v;
    };
    // x_q -= its mean over the active cells (a floating scalar problem)
    const double inv_cells = 1.0 / (double)std::max<int64_t>(1, L.n_act_cells);
    auto demean = [&](const VPtr<double> &X) {
        if (!op->s_floating) return;
        VPtr<const double> M{};
        for (int q = 0; q < nr; ++q) M.p[q] = op->cmask;
        launch_dot_pairs(nr, as_const(X), M, nullptr, P, op->part, op->bk_dres + 2, kMaxDots, s, csp);
        launch_sub_masked_b(nr, P, op->cmask, op->bk_dres + 2, kMaxDots, inv_cells, X, s);
    };
    launch_div_DA_b(g, L.coef64, nr, B, G, s);
    demean(G);
    launch_dot_pairs(nr, as_const(G), as_const(G), op->cmask, P, op->part, op->bk_dres, kMaxDots, s, csp);
    launch_dot_pairs(nr, B, B, op->wa, n, op->part, op->bk_dres + 1, kMaxDots, s);
    fetch();
    double stop[kMaxRhs], rz[kMaxRhs];
    bool act[kMaxRhs] = {};
    int its[kMaxRhs];
    bool any = false;
    for (int q = 0; q < nr; ++q) {
        const double gnorm = std::sqrt(hres(q)[0]);
        if (!std::isfinite(gnorm)) throw DmError{DM_ENAN, "projection input is not finite"};
        // stop on the scale of the field, as project() does
        stop[q] = rtol * std::sqrt(hres(q)[1]) / g.h;
        act[q] = gnorm > stop[q];
        its[q] = 0;
        any = any || act[q];
    }
    DM_HIP(hipMemsetAsync(op->pjb_psi, 0, (size_t)nr * P * sizeof(double), s));
    if (any) {
        launch_copy((int64_t)nr * P, G.p[0], R.p[0], s);   // the slots are consecutive
        graph();                                   // r -> z, every slot
        demean(Z);
        launch_copy((int64_t)nr * P, Z.p[0], PP.p[0], s);
        launch_dot_pairs(nr, as_const(R), as_const(Z), op->cmask, P, op->part, op->bk_dres, kMaxDots, s, csp);
        fetch();
        for (int q = 0; q < nr; ++q) rz[q] = hres(q)[0];
        int it = 0;
        while (it < maxit) {
            // q = S p on the rows holding an active cell (q is zero elsewhere)
            launch_s_apply_b(g, L.coef64, L.sweight, 0, nr, VPtr<const double>{}, as_const(PP), Q, s, L.arows,
                             L.narows);
            launch_dot_pairs(nr, as_const(pick(PP, act)), as_const(Q), op->cmask, P, op->part, op->bk_dres,
                             kMaxDots, s, csp);
            fetch();
            Coef4 alpha;
            for (int q = 0; q < nr; ++q) {
                if (!act[q]) continue;
                const double pq = hres(q)[0];
                if (!(pq > 0.0)) {
                    act[q] = false;
                    continue;
                }
                alpha.v[q] = rz[q] / pq;
                ++its[q];
            }
            bool upd = false;
            for (int q = 0; q < nr; ++q) upd = upd || act[q];
            if (!upd) break;
            // psi += alpha p, r -= alpha q and |r|^2, every active system
            launch_cg_update(nr, as_const(pick(PP, act)), as_const(Q), PSI, R, alpha, op->cmask, P, op->part,
                             op->bk_dres, kMaxDots, s, csp);
            ++it;
            fetch();
            any = false;
            for (int q = 0; q < nr; ++q) {
                if (act[q] && std::sqrt(hres(q)[0]) <= stop[q]) act[q] = false;
                any = any || act[q];
            }
            if (!any) break;
            graph();                               // r -> z
            demean(pick(Z, act));
            launch_dot_pairs(nr, as_const(pick(R, act)), as_const(Z), op->cmask, P, op->part, op->bk_dres,
                             kMaxDots, s, csp);
            fetch();
            Coef4 beta;
            for (int q = 0; q < nr; ++q) {
                if (!act[q]) continue;
                const double rz2 = hres(q)[0];
                beta.v[q] = rz2 / rz[q];
                rz[q] = rz2;
            }
            launch_xpby_b(nr, as_const(Z), beta, pick(PP, act), P, s, csp);   // p = z + beta p
        }
    }
    VPtr<double> O{};
    for (int q = 0; q < nr; ++q) O.p[q] = out[q];
    launch_grad_sub_b(g, L.coef64, nr, as_const(PSI), B, O, 1.0, s);
    if (iters)
        for (int q = 0; q < nr; ++q) iters[q] = its[q];
    return DM_OK;
}

int solve(dm_op *op, int mode, const double *f, double *x, double rtol, int maxit,
          dm_solve_info *info, hipStream_t s) {
    const double t0 = now_s();
    int rc;
    op->ln_accepted = op->ln_rejected = 0;
    if (mode == DM_SOLVE_PCG64) rc = pcg(op, f, x, rtol, maxit, info, s);
    else rc = fgmres(op, mode, f, x, rtol, maxit, info, s);
    DM_HIP(hipStreamSynchronize(s));
    if (info) {
        info->seconds = now_s() - t0;
        info->learned_accepted = op->ln_accepted;
        info->learned_rejected = op->ln_rejected;
    }
    return rc;
}

// ---------------------------------------------------------------------------
// Block solves: nr systems M x_r = f_r in lockstep.  Every system runs the
// FGMRES(m) of fgmres() above step for step; one lockstep step applies the
// preconditioner of all open systems as one block V-cycle and their matrix
// products as one block apply (each coefficient read once for all of them),
// and gathers the dot products of every system before one host sync.
// ---------------------------------------------------------------------------
namespace {

void precondition_block(dm_op *op, int mode, int nr, const double *const *v, double *const *z, hipStream_t s,
                        int *const *rejections = nullptr) {
    const int64_t n = op->n0();
    if (mode == DM_SOLVE_FGMRES_MG32 || mode == DM_SOLVE_FGMRES_MG32_LEARNED) {
        ensure_block(op, 32);
        // the V-cycle reads f on active rows only, and z is zero outside the
        // listed units (written only here)
        const Span sp = op->vspan();
        for (int q = 0; q < nr; ++q) launch_cast<double, float>(v[q], op->lv[0].bf32 + q * n, n, s, sp);
        vcycle_block_graphed(op, 32, nr, s);
        for (int q = 0; q < nr; ++q) launch_cast<float, double>(op->lv[0].bx32 + q * n, z[q], n, s, sp);
        if (mode == DM_SOLVE_FGMRES_MG32_LEARNED)
            for (int q = 0; q < nr; ++q) {
                int none = 0;
                net_correct_patient(op, v[q], z[q], rejections ? rejections[q] : &none, s);
            }
    } else {
        ensure_block(op, 64);
        for (int q = 0; q < nr; ++q) launch_copy(n, v[q], op->lv[0].bf64 + q * n, s);
        vcycle_block_graphed(op, 64, nr, s);
        for (int q = 0; q < nr; ++q) launch_copy(n, op->lv[0].bx64 + q * n, z[q], s);
    }
}

// The plain FP32-multigrid preconditioner with FP32 answers: the V-cycle's
// output is FP32 already, so the Z columns keep it as it is (half the bytes
// of the widened copy).  The products M z and the update of x read them
// widened to FP64, so every value equals that of the FP64 columns.  The
// inputs are FP64 basis columns, or FP32 ones (krylov_basis_f32).
template <class TV>
void precondition_block_f32(dm_op *op, int nr, const TV *const *v, float *const *z, hipStream_t s) {
    const int64_t n = op->n0();
    ensure_block(op, 32);
    const Span sp = op->vspan();
    for (int q = 0; q < nr; ++q) launch_cast<TV, float>(v[q], op->lv[0].bf32 + q * n, n, s, sp);
    vcycle_block_graphed(op, 32, nr, s);
    for (int q = 0; q < nr; ++q) launch_cast<float, float>(op->lv[0].bx32 + q * n, z[q], n, s, sp);
}

struct BlockRhs {
    const double *f = nullptr;
    double *x = nullptr;
    double bnorm = 0.0, rel = 0.0;
    int total = 0, restarts = 0, j = 0;
    int learned_rejections = 0;   // learned mode: rejected corrections in this solve
    bool open = false, done = false, conv = false;
    std::vector<double> H, cs, sn, g, y, h, h2, c3, cx, sc, sc2;   // as in fgmres()
};

int fgmres_block(dm_op *op, int mode, int nb, const double *const *f, double *const *x, double rtol, int maxit,
                 dm_solve_info *info, hipStream_t s) {
    ensure_block(op, mode == DM_SOLVE_FGMRES_MG64 ? 64 : 32);
    const Level &L = op->lv[0];
    const int64_t n = op->n0();
    const int m = op->bk_m;
    const int64_t ld = (int64_t)nb * n;   // stride between the columns of one system
    const Span sp = op->vspan();
    auto Vc = [&](int r, int j) { return op->bk_V + (int64_t)j * ld + (int64_t)r * n; };
    // FP32 Z columns in the plain FP32-multigrid mode (even lengths: pairs of
    // floats per load), FP64 ones otherwise
    const bool z32 = mode == DM_SOLVE_FGMRES_MG32 && n % 2 == 0;
    // FP32 basis (krylov_basis_f32): each new column is formed and
    // orthogonalised in the system's FP64 column W_r, then rounded into the
    // FP32 basis; every dot product and update widens the stored values
    const bool b32 = z32 && op->opt.krylov_basis_f32 != 0;
    if (b32) {
        if (!op->bk_V32) op->bk_V32 = op->dalloc<float>((size_t)(m + 1) * kMaxRhs * n);
        if (!op->bk_W) op->bk_W = op->dalloc<double>((size_t)kMaxRhs * n);
    } else if (!op->bk_V) {
        op->bk_V = op->dalloc<double>((size_t)(m + 1) * kMaxRhs * n);
    }
    auto Vc32 = [&](int r, int j) { return op->bk_V32 + (int64_t)j * ld + (int64_t)r * n; };
    // the FP64 column in which column j of system r is formed
    auto Fc = [&](int r, int j) { return b32 ? op->bk_W + (int64_t)r * n : Vc(r, j); };
    if (z32 && !op->bk_Z32) op->bk_Z32 = op->dalloc<float>((size_t)m * kMaxRhs * n);
    if (!z32 && !op->bk_Z) op->bk_Z = op->dalloc<double>((size_t)m * kMaxRhs * n);
    auto Zc = [&](int r, int j) { return op->bk_Z + (int64_t)j * ld + (int64_t)r * n; };
    auto Zc32 = [&](int r, int j) { return op->bk_Z32 + (int64_t)j * ld + (int64_t)r * n; };
    auto dres = [&](int r) { return op->bk_dres + (int64_t)r * kMaxDots; };
    auto dcoef = [&](int r) { return op->bk_dcoef + (int64_t)r * kMaxDots; };
    auto hres = [&](int r) { return op->bk_hres + (int64_t)r * kMaxDots; };
    auto dres2 = [&](int r) { return op->bk_dres2 + (int64_t)r * kMaxDots; };
    auto hres2 = [&](int r) { return op->bk_hres2 + (int64_t)r * kMaxDots; };
    auto dsc2 = [&](int r) { return op->bk_sc2 + (int64_t)r * kMaxDots; };
    // the scales sc^2 of every system go to the device in one copy of their
    // pinned host image; it is written only after a host sync that follows
    // the previous copy, so no copy in flight reads it
    auto hsc2 = [&](int r) { return op->bk_hsc2 + (int64_t)r * kMaxDots; };
    bool put_sc2 = false;
    auto send_sc2 = [&]() {
        if (put_sc2)
            DM_HIP(hipMemcpyAsync(op->bk_sc2, op->bk_hsc2, (size_t)nb * kMaxDots * sizeof(double),
                                  hipMemcpyHostToDevice, s));
        put_sc2 = false;
    };
    // every system's device results to the host, one sync
    auto fetch = [&]() {
        DM_HIP(hipMemcpyAsync(op->bk_hres, op->bk_dres, (size_t)nb * kMaxDots * sizeof(double),
                              hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
    };
    std::vector<BlockRhs> st(nb);
    for (int r = 0; r < nb; ++r) {
        BlockRhs &R = st[r];
        R.f = f[r];
        R.x = x[r];
        R.H.assign((size_t)(m + 1) * m, 0.0);
        R.cs.assign(m, 0.0);
        R.sn.assign(m, 0.0);
        R.g.assign(m + 1, 0.0);
        R.y.assign(m, 0.0);
        R.h.assign(m + 1, 0.0);
        R.h2.assign(m + 1, 0.0);
        R.sc2.assign(m + 1, 0.0);
        R.c3.assign(m + 1, 0.0);
        R.cx.assign(m + 1, 0.0);
        R.sc.assign(m + 1, 0.0);
        DM_HIP(hipMemsetAsync(R.x, 0, n * sizeof(double), s));
        launch_mdot(1, R.f, 0, R.f, nullptr, n, op->part, dres(r), s, sp);
    }
    fetch();
    for (int r = 0; r < nb; ++r) {
        BlockRhs &R = st[r];
        R.bnorm = std::sqrt(hres(r)[0]);
        if (!std::isfinite(R.bnorm)) throw DmError{DM_ENAN, "right-hand side is not finite"};
        if (R.bnorm == 0.0) R.done = R.conv = true;
    }
    std::vector<int> act;
    const double *vin[kMaxRhs];
    double *zout[kMaxRhs];
    while (true) {
        // (re)start the systems without an open cycle: r0 = f - M x, beta
        act.clear();
        for (int r = 0; r < nb; ++r)
            if (!st[r].done && !st[r].open) act.push_back(r);
        if (!act.empty()) {
            VPtr<const double> bf{}, bx{};
            VPtr<double> by{};
            int nres = 0;
            for (int r : act) {
                if (st[r].total == 0) {
                    launch_copy(n, st[r].f, Fc(r, 0), s);
                } else {
                    bf.p[nres] = st[r].f;
                    bx.p[nres] = st[r].x;
                    by.p[nres] = Fc(r, 0);
                    ++nres;
                }
            }
            if (nres) launch_apply_b<double>(L.g, L.coef64, op->sigma, AK_RESID, nres, bf, bx, by, s, L.cut_cells());
            for (int r : act) {
                launch_mdot(1, Fc(r, 0), 0, Fc(r, 0), nullptr, n, op->part, dres(r), s, sp);
                if (b32) launch_cast<double, float>(Fc(r, 0), Vc32(r, 0), n, s, sp);
            }
            fetch();
            for (int r : act) {
                BlockRhs &R = st[r];
                const double beta = std::sqrt(hres(r)[0]);
                if (!std::isfinite(beta)) throw DmError{DM_ENAN, "FGMRES residual is not finite"};
                R.rel = beta / R.bnorm;
                if (beta <= rtol * R.bnorm) {
                    R.done = R.conv = true;
                    continue;
                }
                if (R.total >= maxit) {
                    R.done = true;
                    continue;
                }
                R.sc[0] = 1.0 / beta;   // unnormalised basis, as in fgmres()
                R.sc2[0] = R.sc[0] * R.sc[0];
                hsc2(r)[0] = R.sc2[0];
                put_sc2 = true;
                std::fill(R.g.begin(), R.g.end(), 0.0);
                R.g[0] = beta;
                std::fill(R.H.begin(), R.H.end(), 0.0);
                R.j = 0;
                R.open = true;
            }
        }
        act.clear();
        for (int r = 0; r < nb; ++r)
            if (st[r].open) act.push_back(r);
        if (act.empty()) break;
        const int na = (int)act.size();
        // z_j = B v_j and w = M z_j for every open system
        VPtr<const double> zc{};
        VPtr<const float> zc32{};
        VPtr<double> wv{};
        float *zout32[kMaxRhs];
        const float *vin32[kMaxRhs];
        int *rej[kMaxRhs];
        for (int q = 0; q < na; ++q) {
            const int r = act[q];
            if (b32) vin32[q] = Vc32(r, st[r].j);
            else vin[q] = Vc(r, st[r].j);
            rej[q] = &st[r].learned_rejections;
            if (z32) {
                zout32[q] = Zc32(r, st[r].j);
                zc32.p[q] = zout32[q];
            } else {
                zout[q] = Zc(r, st[r].j);
                zc.p[q] = zout[q];
            }
            wv.p[q] = Fc(r, st[r].j + 1);          // w = M Z_j in the next column's slot
        }
        // w = M z on the rows holding an active face: the slots of columns
        // 1..m are zero on the others (written only here and, within the
        // listed units, by the Gram--Schmidt updates of zero entries)
        if (z32) {
            if (b32) precondition_block_f32<float>(op, na, vin32, zout32, s);
            else precondition_block_f32<double>(op, na, vin, zout32, s);
            launch_apply_m_f32in(L.g, L.coef64, op->sigma, na, zc32, wv, s, L.cut_cells_rows());
        } else {
            precondition_block(op, mode, na, vin, zout, s, rej);
            launch_apply_b<double>(L.g, L.coef64, op->sigma, AK_M, na, VPtr<const double>{}, zc, wv, s,
                                   L.cut_cells_rows());
        }
        // Gram--Schmidt as in fgmres(): (1) d = U^T w, (2) w -= U (sc^2 d)
        // fused with d2 = U^T w and |w|^2, every open system, one sync
        send_sc2();
        for (int r : act) {
            const int j = st[r].j;
            if (b32) {
                launch_mdot(j + 1, Vc32(r, 0), ld, Fc(r, j + 1), nullptr, n, op->part, dres(r), s, sp);
                launch_maxpy_mdot_norm(j + 1, Vc32(r, 0), ld, dres(r), Fc(r, j + 1), n, op->part, dres2(r), s,
                                       dsc2(r), sp);
            } else {
                launch_mdot(j + 1, Vc(r, 0), ld, Vc(r, j + 1), nullptr, n, op->part, dres(r), s, sp);
                launch_maxpy_mdot_norm(j + 1, Vc(r, 0), ld, dres(r), Vc(r, j + 1), n, op->part, dres2(r), s,
                                       dsc2(r), sp);
            }
        }
        // dres2 follows dres: one copy brings both
        DM_HIP(hipMemcpyAsync(op->bk_hres, op->bk_dres, (size_t)(kMaxRhs + nb) * kMaxDots * sizeof(double),
                              hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        // (3) the second correction where needed; Hessenberg column, Givens
        for (int r : act) {
            BlockRhs &R = st[r];
            int j = R.j;
            double *w = Fc(r, j + 1);
            for (int i = 0; i <= j; ++i) R.h[i] = R.sc[i] * R.sc[j] * hres(r)[i];   // true coefficients
            const double wn2 = hres2(r)[j + 1] * R.sc[j] * R.sc[j];
            double c2 = 0.0;
            for (int i = 0; i <= j; ++i) {
                R.h2[i] = R.sc[i] * R.sc[j] * hres2(r)[i];
                c2 += R.h2[i] * R.h2[i];
            }
            double hn;
            const double reorth = b32 ? kReorthF32 : kReorth;
            if (c2 > reorth * reorth * wn2) {
                for (int i = 0; i <= j; ++i) {
                    R.c3[i] = R.sc[i] * R.sc[i] * hres2(r)[i];
                    R.h[i] += R.h2[i];
                }
                DM_HIP(hipMemcpyAsync(dcoef(r), R.c3.data(), (j + 1) * sizeof(double), hipMemcpyHostToDevice, s));
                if (b32) launch_maxpy(j + 1, Vc32(r, 0), ld, dcoef(r), w, n, 0, s, nullptr, sp);
                else launch_maxpy(j + 1, Vc(r, 0), ld, dcoef(r), w, n, 0, s, nullptr, sp);
                hn = std::sqrt(std::max(wn2 - c2, 0.0));
            } else {
                hn = std::sqrt(wn2);
            }
            if (!std::isfinite(hn)) throw DmError{DM_ENAN, "FGMRES iterate is not finite"};
            R.sc[j + 1] = hn > 0.0 ? R.sc[j] / hn : 0.0;
            R.sc2[j + 1] = R.sc[j + 1] * R.sc[j + 1];
            hsc2(r)[j + 1] = R.sc2[j + 1];
            put_sc2 = true;
            double *H = R.H.data();
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = R.h[i];
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = R.cs[i] * a + R.sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -R.sn[i] * a + R.cs[i] * b;
            }
            const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a, b);
            R.cs[j] = rr > 0 ? a / rr : 1.0;
            R.sn[j] = rr > 0 ? b / rr : 0.0;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            R.g[j + 1] = -R.sn[j] * R.g[j];
            R.g[j] = R.cs[j] * R.g[j];
            ++R.total;
            R.j = ++j;
            const bool close = std::fabs(R.g[j]) <= rtol * R.bnorm || R.total >= maxit || hn == 0.0 || j == m;
            if (!close) {
                if (b32) launch_cast<double, float>(Fc(r, j), Vc32(r, j), n, s, sp);   // store the new column
                continue;
            }
            // end of the cycle: x += Z y, y from the triangular system
            for (int i = j - 1; i >= 0; --i) {
                double t = R.g[i];
                for (int c = i + 1; c < j; ++c) t -= H[(size_t)i * m + c] * R.y[c];
                R.y[i] = t / H[(size_t)i * m + i];
            }
            for (int i = 0; i < j; ++i) R.cx[i] = -R.y[i] * R.sc[i];
            DM_HIP(hipMemcpyAsync(dcoef(r), R.cx.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
            if (z32) launch_maxpy_f32(j, Zc32(r, 0), ld, dcoef(r), R.x, n, s, sp);
            else launch_maxpy(j, Zc(r, 0), ld, dcoef(r), R.x, n, 0, s, nullptr, sp);
            ++R.restarts;
            R.open = false;
        }
    }
    int rc = DM_OK;
    for (int r = 0; r < nb; ++r) {
        if (!st[r].conv) rc = DM_NOT_CONVERGED;
        if (info) {
            info[r].iterations = st[r].total;
            info[r].restarts = st[r].restarts > 0 ? st[r].restarts - 1 : 0;
            info[r].rel_residual = st[r].rel;
        }
    }
    return rc;
}

}  // namespace

int solve_block(dm_op *op, int mode, int nrhs, const double *const *f, double *const *x, double rtol, int maxit,
                dm_solve_info *info, hipStream_t s) {
    if (nrhs < 1 || nrhs > kMaxRhs) throw DmError{DM_EINVAL, "block of 1 to 4 systems"};
    if (mode == DM_SOLVE_PCG64) throw DmError{DM_EINVAL, "block solves use FGMRES modes"};
    const double t0 = now_s();
    op->ln_accepted = op->ln_rejected = 0;
    const int rc = fgmres_block(op, mode, nrhs, f, x, rtol, maxit, info, s);
    DM_HIP(hipStreamSynchronize(s));
    if (info)
        for (int r = 0; r < nrhs; ++r) {
            info[r].seconds = now_s() - t0;
            info[r].learned_accepted = op->ln_accepted;
            info[r].learned_rejected = op->ln_rejected;
        }
    return rc;
}

// ---------------------------------------------------------------------------
// Block Krylov--Schur (symmetric) on T = P_DM M^-1 A, A-inner product.
// ---------------------------------------------------------------------------
int eigs(dm_op *op, int k, double tol, uint64_t seed, const dm_eig_options &opt, double *lam,
         double *vecs, double *res_out, dm_eig_info *info, hipStream_t s) {
    const double t0 = now_s();
    const Level &L = op->lv[0];
    const int64_t n = op->n0();
    const int b = std::max(1, opt.block);
    int m = std::max(opt.max_basis, k + 2 * b);
    m = (m + b - 1) / b * b;                 // basis columns that get expanded
    const int keep_max = std::min(m - b, ((k + b + b - 1) / b) * b);
    const int cap = m + b + keep_max;
    if (cap > kMaxDots) throw DmError{DM_EINVAL, "eigs: basis too large"};
    if (op->eg_cap < cap) {
        op->eg_V = op->dalloc<double>((size_t)cap * n);
        op->eg_W = op->dalloc<double>((size_t)b * n);
        op->eg_T = op->dalloc<double>((size_t)3 * n);
        op->eg_cap = cap;
    }
    // the block's M solves in lockstep (one block V-cycle per step) unless
    // the op's preconditioner is a batch's fused V-cycle or the mode is PCG
    const bool blocked = b > 1 && !op->batch && opt.solve_mode != DM_SOLVE_PCG64;
    // the projection's scalar V-cycle follows the inner solves' V-cycle: FP32
    // with the FP32-multigrid forms, FP64 with the FP64 one
    const int sprec = opt.solve_mode == DM_SOLVE_FGMRES_MG64 ? 64 : 32;
    if (blocked && !op->eg_F) op->eg_F = op->dalloc<double>((size_t)kMaxRhs * n);
    if (blocked) ensure_krylov_small(op);
    else ensure_krylov(op);
    if (b > kMultiMax) throw DmError{DM_EINVAL, "eigs: block size above 8"};
    if (!op->eg_C) op->eg_C = op->dalloc<double>((size_t)256 * kMultiMax);
    if (op->eg_kv_cap < b) {
        op->eg_KV = op->dalloc<double>((size_t)b * n);
        op->eg_kv_cap = b;
    }
    if (op->eg_r_cap < k) {
        op->eg_R = op->dalloc<double>((size_t)3 * k * n);
        op->eg_r_cap = k;
    }
    double *V = op->eg_V, *W = op->eg_W, *t1 = op->eg_T, *t2 = op->eg_T + n, *t3 = op->eg_T + 2 * n;
    double *SCR = V + (size_t)(m + b) * n;   // room for keep_max Ritz vectors
    double *RB = op->eg_R, *RK = op->eg_R + (size_t)k * n, *RA = op->eg_R + (size_t)2 * k * n;
    // block basis work: every product of nv basis vectors with up to
    // kMultiMax vectors reads the basis once (launch_mdot_multi /
    // launch_maxpy_multi); results through op->dres / hres, coefficients
    // through eg_C (a host array of its own per upload)
    std::vector<double> cbuf((size_t)256 * kMultiMax), mres((size_t)cap * kMultiMax);
    // every basis, Ritz and work vector of the eigensolver is zero outside
    // the listed units of the face vectors (solves, projections, A and K
    // products and random starts all write zeros there)
    const Span vsp = op->vspan();
    // mres[i*nw + q] = V_i . (W_q * wt), i < nv (chunks of basis columns whose
    // products fit the kMaxDots result buffer)
    auto multi_dots = [&](int nv, const double *W0, int nw, const double *wt) {
        const int rows = kMaxDots / nw;
        for (int i0 = 0; i0 < nv; i0 += rows) {
            const int cnt = std::min(rows, nv - i0);
            launch_mdot_multi(cnt, V + (size_t)i0 * n, n, W0, n, nw, wt, n, op->part, op->dres, s, vsp);
            DM_HIP(hipMemcpyAsync(op->hres, op->dres, (size_t)cnt * nw * sizeof(double), hipMemcpyDeviceToHost, s));
            DM_HIP(hipStreamSynchronize(s));
            std::copy(op->hres, op->hres + (size_t)cnt * nw, mres.begin() + (size_t)i0 * nw);
        }
    };
    // Y_q = sum_r coefficient(r, q) V_r for q < nq, in chunks of kMultiMax;
    // with the span (internal buffers, zero outside it) only its units are
    // written, without it (a caller's buffer) every element
    auto combine = [&](int nv, int nq, double *Y0, auto coefficient, Span csp) {
        for (int q0 = 0; q0 < nq; q0 += kMultiMax) {
            const int nw = std::min(kMultiMax, nq - q0);
            std::vector<double> c((size_t)nv * nw);
            for (int r = 0; r < nv; ++r)
                for (int q = 0; q < nw; ++q) c[(size_t)r * nw + q] = coefficient(r, q0 + q);
            DM_HIP(hipMemcpyAsync(op->eg_C, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, s));
            launch_maxpy_multi(nv, V, n, op->eg_C, nw, Y0 + (size_t)q0 * n, n, n, 1, s, csp);
            DM_HIP(hipStreamSynchronize(s));   // c goes out of scope
        }
    };
    // inner products over the owned active faces: (u, v) = u^T W A v
    // (eq. bInner; W = 1/2 on faces in a PMC plane), K-forms with W, and
    // the residual norm with W / A
    const double *a = op->wa, *wk = op->wface, *ainv = op->wainv;
    int inner_its = 0, proj_its = 0, outer = 0, restarts = 0;
    dm_solve_info sinfo;
    auto A_normalize = [&](double *v) -> double {
        const double nrm = std::sqrt(dot1(op, v, v, a, n, s, vsp));
        if (nrm > 0) launch_scale(n, 1.0 / nrm, v, s);
        return nrm;
    };
    // orthogonalise v against `cnt` A-orthonormal columns starting at B, twice;
    // accumulates the coefficients into coef (size cnt)
    std::vector<double> hc(cap);
    auto orth = [&](const double *B, int cnt, double *v, double *coef) {
        if (cnt <= 0) return;
        for (int pass = 0; pass < 2; ++pass) {
            dots(op, cnt, B, n, v, a, n, s, vsp);
            std::copy(op->hres, op->hres + cnt, hc.begin());
            if (coef)
                for (int i = 0; i < cnt; ++i) coef[i] += hc[i];
            to_device_coef(op, hc.data(), cnt, s);
            launch_maxpy(cnt, B, n, op->dcoef, v, n, 0, s, nullptr, vsp);
        }
    };
    int pj;
    // G = V^T K V of the basis, kept on the host: one K apply and one
    // multi-dot per new basis vector; thick restarts transform it in place.
    std::vector<double> GK((size_t)cap * cap, 0.0);
    auto Gat = [&](int r, int c) -> double & { return GK[(size_t)r * cap + c]; };
    auto add_gk = [&](int q) {
        launch_apply<double>(L.g, L.coef64, 0.0, AK_K, nullptr, V + (size_t)q * n, t2, s);
        dots(op, q + 1, V, n, t2, wk, n, s, vsp);
        for (int i = 0; i <= q; ++i) Gat(i, q) = Gat(q, i) = op->hres[i];
    };
    // start block: random vectors, projected together where the block path
    // runs (the projections are independent), then A-orthonormalised
    // A-norms of the start vectors before the projection: a vector that the
    // projection and orthogonalisation reduce to rounding noise (zero, or
    // gradients only) is a breakdown
    std::vector<double> nrm0(b);
    for (int c = 0; c < b; ++c) {
        double *v = V + (size_t)c * n;
        if (opt.start_dev) {   // caller's start block (warm start), active faces only
            launch_copy_masked(n, opt.start_dev + (size_t)c * n, op->fmask, v, s);
        } else {
            launch_randn(n, seed, (int64_t)c * n, op->fmask, v, s);
        }
        launch_mirror_faces<double>(L.g, v, s);
        nrm0[c] = std::sqrt(dot1(op, v, v, a, n, s, vsp));
    }
    if (blocked) {
        for (int c0 = 0; c0 < b; c0 += kMaxRhs) {
            const int nr = std::min(kMaxRhs, b - c0);
            const double *bp[kMaxRhs];
            double *op_[kMaxRhs];
            int pits[kMaxRhs];
            for (int q = 0; q < nr; ++q) bp[q] = op_[q] = V + (size_t)(c0 + q) * n;
            project_block(op, nr, bp, op_, opt.proj_rtol, 1000, s, pits, sprec);
            for (int q = 0; q < nr; ++q) proj_its += pits[q];
        }
    }
    for (int c = 0; c < b; ++c) {
        double *v = V + (size_t)c * n;
        if (!blocked) {
            project(op, v, v, opt.proj_rtol, 1000, s, &pj);
            proj_its += pj;
        }
        orth(V, c, v, nullptr);
        if (!(A_normalize(v) > 1e-10 * nrm0[c]) || !(nrm0[c] > 0.0))
            throw DmError{DM_EBREAKDOWN, "eigs: start vector " + std::to_string(c) +
                                             " is zero, or gradients only, or dependent on the others"};
        add_gk(c);
    }
    const int HR = m + b;  // rows of H
    std::vector<double> H((size_t)HR * m, 0.0);
    auto Hat = [&](int r, int c) -> double & { return H[(size_t)r * m + c]; };
    int cur = b;           // basis vectors present
    std::vector<double> theta, Y, mu, Z, lam_h(k), res_h(k, INFINITY);
    std::vector<int> wanted(k);
    std::vector<double> coef(cap);
    int status = DM_NOT_CONVERGED;
    int nconv = 0;
    while (true) {
        // ---- expand by one block: W = T V_last, orthogonalise, append
        {
            const int j0 = cur - b;
            if (blocked) {
                // the block's solves in lockstep, kMaxRhs at a time
                for (int c0 = 0; c0 < b; c0 += kMaxRhs) {
                    const int nr = std::min(kMaxRhs, b - c0);
                    const double *fp[kMaxRhs];
                    double *xp[kMaxRhs];
                    dm_solve_info bi[kMaxRhs];
                    for (int q = 0; q < nr; ++q) {
                        launch_apply_A(L.g, L.coef64, V + (size_t)(j0 + c0 + q) * n, op->eg_F + (size_t)q * n, s);
                        fp[q] = op->eg_F + (size_t)q * n;
                        xp[q] = W + (size_t)(c0 + q) * n;
                    }
                    const int rc = solve_block(op, opt.solve_mode, nr, fp, xp, opt.inner_rtol, 2000, bi, s);
                    if (rc < 0) return rc;
                    for (int q = 0; q < nr; ++q) inner_its += bi[q].iterations;
                }
                for (int c0 = 0; c0 < b; c0 += kMaxRhs) {
                    const int nr = std::min(kMaxRhs, b - c0);
                    const double *bp[kMaxRhs];
                    double *op_[kMaxRhs];
                    int pits[kMaxRhs];
                    for (int q = 0; q < nr; ++q) bp[q] = op_[q] = W + (size_t)(c0 + q) * n;
                    project_block(op, nr, bp, op_, opt.proj_rtol, 1000, s, pits, sprec);
                    for (int q = 0; q < nr; ++q) proj_its += pits[q];
                }
            } else {
                for (int c = 0; c < b; ++c) {
                    double *w = W + (size_t)c * n;
                    launch_apply_A(L.g, L.coef64, V + (size_t)(j0 + c) * n, t1, s);
                    const int rc = solve(op, opt.solve_mode, t1, w, opt.inner_rtol, 2000, &sinfo, s);
                    if (rc < 0) return rc;
                    inner_its += sinfo.iterations;
                    project(op, w, w, opt.proj_rtol, 1000, s, &pj);
                    proj_its += pj;
                }
            }
            ++outer;
            double *Vn = V + (size_t)cur * n;
            DM_HIP(hipMemcpyAsync(Vn, W, (size_t)b * n * sizeof(double), hipMemcpyDeviceToDevice, s));
            // block classical Gram--Schmidt twice against the cur old columns
            // (one read of the basis per pass for the whole block) ...
            std::vector<double> cb((size_t)cur * b, 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                multi_dots(cur, Vn, b, a);
                for (int t = 0; t < cur * b; ++t) {
                    cbuf[t] = mres[t];
                    cb[t] += mres[t];
                }
                DM_HIP(hipMemcpyAsync(op->eg_C, cbuf.data(), (size_t)cur * b * sizeof(double), hipMemcpyHostToDevice,
                                      s));
                launch_maxpy_multi(cur, V, n, op->eg_C, b, Vn, n, n, 0, s, vsp);
                DM_HIP(hipStreamSynchronize(s));   // cbuf is reused
            }
            // ... then within the block, column by column
            for (int c = 0; c < b; ++c) {
                double *v = Vn + (size_t)c * n;
                std::fill(coef.begin(), coef.end(), 0.0);
                orth(Vn, c, v, coef.data());
                for (int i = 0; i < cur; ++i) Hat(i, j0 + c) += cb[(size_t)i * b + c];
                for (int i = 0; i < c; ++i) Hat(cur + i, j0 + c) += coef[i];
                const double nrm = A_normalize(v);
                if (!std::isfinite(nrm)) throw DmError{DM_ENAN, "eigs: basis vector not finite"};
                Hat(cur + c, j0 + c) = nrm;
                if (nrm <= 1e-300) throw DmError{DM_EBREAKDOWN, "eigs: Krylov breakdown"};
            }
            // V^T K V: the block's K images against the whole basis, one pass
            for (int c = 0; c < b; ++c)
                launch_apply<double>(L.g, L.coef64, 0.0, AK_K, nullptr, Vn + (size_t)c * n, op->eg_KV + (size_t)c * n,
                                     s);
            multi_dots(cur + b, op->eg_KV, b, wk);
            for (int c = 0; c < b; ++c)
                for (int i = 0; i < cur + b; ++i) Gat(i, cur + c) = Gat(cur + c, i) = mres[(size_t)i * b + c];
            cur += b;
        }
        const bool full = cur >= m + b;
        if (cur - b < k) continue;
        // ---- Krylov--Schur Ritz vectors of T (restarts): the expanded columns
        const int mm = cur - b;
        std::vector<double> Hs((size_t)mm * mm);
        for (int i = 0; i < mm; ++i)
            for (int j = 0; j < mm; ++j) Hs[(size_t)i * mm + j] = 0.5 * (Hat(i, j) + Hat(j, i));
        jacobi_eig(Hs, mm, theta, Y);
        // restart order: the wanted pairs are the smallest lambda > 0, and
        // theta = 1 / (lambda - sigma), so rank each Ritz value by its
        // lambda = sigma + 1/theta, ascending over lambda > 0 (theta > 0 for
        // lambda above the shift, theta < 0 below it), then the rest by
        // |theta| descending.  With sigma below every wanted eigenvalue this
        // is theta descending.
        std::vector<int> order(mm);
        for (int i = 0; i < mm; ++i) order[i] = i;
        const double sig_r = op->sigma;
        auto lam_of = [&](int x) { return theta[x] != 0.0 ? sig_r + 1.0 / theta[x] : -1.0; };
        std::sort(order.begin(), order.end(), [&](int x, int y) {
            const double lx = lam_of(x), ly = lam_of(y);
            const bool px = lx > 0.0, py = ly > 0.0;
            if (px != py) return px;
            if (px) return lx < ly;
            return std::fabs(theta[x]) > std::fabs(theta[y]);
        });
        // ---- Rayleigh--Ritz on (K, A) over the whole basis (answers): the
        // basis is A-orthonormal, so the projected pencil is (V^T K V, I)
        const int nb = cur;
        {
            std::vector<double> Gs((size_t)nb * nb);
            double gmax = 0.0;
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j) {
                    Gs[(size_t)i * nb + j] = 0.5 * (Gat(i, j) + Gat(j, i));
                    gmax = std::max(gmax, std::fabs(Gs[(size_t)i * nb + j]));
                }
            jacobi_eig(Gs, nb, mu, Z);
            std::vector<int> ord(nb);
            for (int i = 0; i < nb; ++i) ord[i] = i;
            std::sort(ord.begin(), ord.end(), [&](int x, int y) { return mu[x] < mu[y]; });
            int w = 0;
            for (int i = 0; i < nb && w < k; ++i)
                if (mu[ord[i]] > 1e-10 * gmax) wanted[w++] = ord[i];
            // fewer than k nonzero Rayleigh quotients: keep the lowest ones
            for (int i = 0; w < k && i < nb; ++i)
                if (!(mu[ord[i]] > 1e-10 * gmax)) wanted[w++] = ord[i];
        }
        // ---- explicit residuals of the k wanted Ritz pairs on (K, A): the
        // k Ritz vectors b_i = V y_i from one read of the basis (per chunk of
        // kMultiMax), their K and A images, and two host syncs for all
        nconv = 0;
        double maxres = 0.0;
        std::vector<double> yk(std::max(mm, nb));
        combine(nb, k, RB, [&](int r, int i) { return Z[(size_t)r * nb + wanted[i]]; }, vsp);
        for (int i = 0; i < k; ++i) {
            launch_apply<double>(L.g, L.coef64, 0.0, AK_K, nullptr, RB + (size_t)i * n, RK + (size_t)i * n, s);
            launch_apply_A(L.g, L.coef64, RB + (size_t)i * n, RA + (size_t)i * n, s);
            launch_mdot(1, RB + (size_t)i * n, 0, RK + (size_t)i * n, wk, n, op->part, op->dres + 2 * i, s, vsp);
            launch_mdot(1, RB + (size_t)i * n, 0, RB + (size_t)i * n, a, n, op->part, op->dres + 2 * i + 1, s, vsp);
        }
        DM_HIP(hipMemcpyAsync(op->hres, op->dres, (size_t)2 * k * sizeof(double), hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        std::vector<double> bKb(k), bAb(k);
        for (int i = 0; i < k; ++i) {
            bKb[i] = op->hres[2 * i];
            bAb[i] = op->hres[2 * i + 1];
            lam_h[i] = bKb[i] / bAb[i];
            // K b - lr A b
            launch_axpy(n, -lam_h[i], RA + (size_t)i * n, RK + (size_t)i * n, s);
            launch_mdot(1, RK + (size_t)i * n, 0, RK + (size_t)i * n, ainv, n, op->part, op->dres + i, s, vsp);
        }
        DM_HIP(hipMemcpyAsync(op->hres, op->dres, (size_t)k * sizeof(double), hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < k; ++i) {
            const double rho = std::sqrt(op->hres[i]) / (std::fabs(lam_h[i]) * std::sqrt(bAb[i]));
            res_h[i] = rho;
            maxres = std::max(maxres, rho);
            if (rho <= tol) ++nconv;
        }
        if (opt.verbose)
            fprintf(stderr, "[dm_eigs] outer %d restart %d dim %d: max rho %.3e, %d/%d converged\n",
                    outer, restarts, mm, maxres, nconv, k);
        if (nconv == k) status = DM_OK;
        if (nconv == k || (full && restarts >= opt.max_restarts)) {
            // outputs: Ritz vectors of the k wanted pairs, sorted by lambda
            std::vector<int> idx(k);
            for (int i = 0; i < k; ++i) idx[i] = i;
            std::sort(idx.begin(), idx.end(), [&](int x, int y) { return lam_h[x] < lam_h[y]; });
            for (int q = 0; q < k; ++q) {
                const int i = idx[q];
                lam[q] = lam_h[i];
                if (res_out) res_out[q] = res_h[i];
            }
            if (vecs) combine(nb, k, vecs, [&](int r, int q) { return Z[(size_t)r * nb + wanted[idx[q]]]; }, Span{});
            if (info) {
                info->n_converged = nconv;
                info->outer_iterations = outer;
                info->restarts = restarts;
                info->inner_iterations = inner_its;
                info->projection_iterations = proj_its;
                double mr = 0;
                for (int i = 0; i < k; ++i) mr = std::max(mr, res_h[i]);
                info->max_residual = mr;
            }
            break;
        }
        if (!full) continue;
        // ---- thick restart: keep the keep_max leading Ritz vectors
        const int keep = keep_max;
        combine(mm, keep, SCR, [&](int r, int i) { return Y[(size_t)r * mm + order[i]]; }, vsp);
        std::vector<double> Bc((size_t)b * keep, 0.0);  // coupling of the last block
        for (int r = 0; r < b; ++r)
            for (int i = 0; i < keep; ++i) {
                double sacc = 0.0;
                for (int c = 0; c < mm; ++c) sacc += Hat(mm + r, c) * Y[(size_t)c * mm + order[i]];
                Bc[(size_t)r * keep + i] = sacc;
            }
        DM_HIP(hipMemcpyAsync(V, SCR, (size_t)keep * n * sizeof(double), hipMemcpyDeviceToDevice, s));
        DM_HIP(hipMemcpyAsync(V + (size_t)keep * n, V + (size_t)mm * n, (size_t)b * n * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
        std::fill(H.begin(), H.end(), 0.0);
        for (int i = 0; i < keep; ++i) Hat(i, i) = theta[order[i]];
        for (int r = 0; r < b; ++r)
            for (int i = 0; i < keep; ++i) Hat(keep + r, i) = Bc[(size_t)r * keep + i];
        // V^T K V of the new basis: Q^T G Q with Q = diag(Y_keep, I_b)
        {
            const int nn = keep + b, no = mm + b;
            std::vector<double> Q((size_t)no * nn, 0.0);
            for (int r = 0; r < mm; ++r)
                for (int i = 0; i < keep; ++i) Q[(size_t)r * nn + i] = Y[(size_t)r * mm + order[i]];
            for (int r = 0; r < b; ++r) Q[(size_t)(mm + r) * nn + keep + r] = 1.0;
            std::vector<double> GQ((size_t)no * nn, 0.0), Gn((size_t)nn * nn, 0.0);
            for (int r = 0; r < no; ++r)
                for (int c = 0; c < no; ++c) {
                    const double g = Gat(r, c);
                    if (g == 0.0) continue;
                    for (int j = 0; j < nn; ++j) GQ[(size_t)r * nn + j] += g * Q[(size_t)c * nn + j];
                }
            for (int r = 0; r < no; ++r)
                for (int i = 0; i < nn; ++i) {
                    const double q = Q[(size_t)r * nn + i];
                    if (q == 0.0) continue;
                    for (int j = 0; j < nn; ++j) Gn[(size_t)i * nn + j] += q * GQ[(size_t)r * nn + j];
                }
            std::fill(GK.begin(), GK.end(), 0.0);
            for (int i = 0; i < nn; ++i)
                for (int j = 0; j < nn; ++j) Gat(i, j) = Gn[(size_t)i * nn + j];
        }
        cur = keep + b;
        ++restarts;
    }
    DM_HIP(hipStreamSynchronize(s));
    if (info) info->seconds = now_s() - t0;
    return status;
}

}  // namespace dm
