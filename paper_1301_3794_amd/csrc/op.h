// The operator object behind the C ABI: level hierarchy, device buffers,
// coarsest-level dense inverses and Krylov workspaces.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "dm_internal.h"

namespace dm {

struct Level {
    Grid g;
    double *coef64 = nullptr;  // 7P: ax ay az lx ly lz vinv
    float *coef32 = nullptr;   // same, FP32
    double sweight = 0.0;      // weight of the scalar Laplacian on this level
    double *x64 = nullptr, *f64 = nullptr, *r64 = nullptr;  // 3P each
    float *x32 = nullptr, *f32 = nullptr, *r32 = nullptr;   // 3P each
    double *sx = nullptr, *sf = nullptr, *sr = nullptr;     // P each (scalar MG)
    // block V-cycle buffers: kMaxRhs vectors of 3P each (allocated on first use)
    double *bx64 = nullptr, *bf64 = nullptr, *br64 = nullptr;
    float *bx32 = nullptr, *bf32 = nullptr, *br32 = nullptr;
    double *bsx = nullptr, *bsf = nullptr, *bsr = nullptr;  // kMaxRhs * P (scalar MG)
    float *bsx32 = nullptr, *bsf32 = nullptr, *bsr32 = nullptr;  // the same, FP32 scalar MG
    int64_t n_act_faces = 0, n_act_cells = 0;
    // non-vacuum rows of each component c (both colours, index order) as
    // padded indices: cut[cut_off[c] .. cut_off[c+1])
    int32_t *cut = nullptr;
    int64_t cut_off[4] = {};
    // cells with an active non-vacuum row (any component), padded indices
    int32_t *cutc = nullptr;
    int64_t ncutc = 0;
    // tabulated rows of the cells in cutc (3 components x kCutW per cell)
    double *cellw64 = nullptr;
    float *cellw32 = nullptr;
    ClassList cut_cells() const {
        ClassList cl{cutc, ncutc};
        cl.w64 = cellw64;
        cl.w32 = cellw32;
        return cl;
    }
    // grid rows (k * ny + j) with a vacuum row of any component
    int32_t *vrows = nullptr;
    int64_t nvrows = 0;
    // grid rows (k * ny + j) with an active cell (the scalar problem's unknowns)
    int32_t *arows = nullptr;
    int64_t narows = 0;
    // grid rows (k * ny + j) with an active face
    int32_t *frows = nullptr;
    int64_t nfrows = 0;
    // the cut-cell list with the rows holding an active face: for outputs
    // that stay zero on the other rows (the block V-cycle's residual)
    ClassList cut_cells_rows() const {
        ClassList cl = cut_cells();
        cl.rows = frows;
        cl.nrows = nfrows;
        return cl;
    }
    // the block smoother's threshold for one wave per vector (dm_options)
    int64_t cut_wave_split = 65536;
    // tabulated rows of the cut lists (kCutW values per row, term-major per
    // component: component c's table starts at kCutW * cut_off[c])
    double *cutw64 = nullptr;
    float *cutw32 = nullptr;
    // the smoother's list for class (comp, colour): the component's cut rows,
    // paired as `pair` says (kPairNone, kPairFirst, kPairSecond) with the
    // cross sums in s (at least the list's length times the vectors)
    ClassList cut_list(int comp, int colour, int pair = kPairNone, void *s = nullptr) const {
        ClassList cl{cut ? cut + cut_off[comp] : nullptr, cut_off[comp + 1] - cut_off[comp], vrows, nvrows,
                     cut_wave_split};
        if (cutw64) cl.w64 = cutw64 + kCutW * cut_off[comp];
        if (cutw32) cl.w32 = cutw32 + kCutW * cut_off[comp];
        cl.pair = pair;
        cl.s = s;
        return cl;
    }
    int64_t max_cut_rows() const {
        int64_t m = 0;
        for (int c = 0; c < 3; ++c) m = std::max(m, cut_off[c + 1] - cut_off[c]);
        return m;
    }
};

// thread-local error reporting
void set_error(const std::string &msg);

struct HipError {
    hipError_t e;
    std::string where;
};

#define DM_HIP(call)                                                        \
    do {                                                                    \
        hipError_t e__ = (call);                                            \
        if (e__ != hipSuccess) throw ::dm::HipError{e__, #call};            \
    } while (0)

struct DmError {
    int code;
    std::string msg;
};

}  // namespace dm

struct dm_net;
struct dm_batch;

struct dm_op {
    dm_geometry geom{};
    int dims[3] = {0, 0, 0};
    double h = 0.0, sigma = 0.0;
    dm_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<dm::Level> lv;
    std::vector<std::vector<double>> frac;  // host fractions per level (7P, v not vinv)
    // coarsest vector level: dense FP64 inverse over active faces
    // the smoother's cross-component sums between the two colour updates of
    // a component (kPairFirst / kPairSecond): the longest cut list of any
    // level and component times kMaxRhs, in doubles
    void *cut_s = nullptr;
    int nc = 0;
    double *cinv = nullptr;
    int64_t *cidx = nullptr;
    // coarsest scalar level
    int ns = 0;
    double *sinv = nullptr;
    int64_t *sidx = nullptr;
    bool s_floating = true;
    // level-0 masks
    double *fmask = nullptr;  // 3P, 1 on active faces
    double *cmask = nullptr;  // P, 1 on active cells
    double *wface = nullptr;  // 3P, W (1/2 on faces in a PMC plane, 1 else, 0 off)
    double *wa = nullptr;     // 3P, W a
    double *wainv = nullptr;  // 3P, W / a
    // reductions
    double *part = nullptr;   // kReduceBlocks * kMaxDots
    double *dres = nullptr;   // kMaxDots device results
    double *hres = nullptr;   // kMaxDots pinned host results
    // Krylov workspaces (allocated on first use)
    int fg_m = 0;
    double *fg_V = nullptr, *fg_Z = nullptr, *fg_w = nullptr, *dcoef = nullptr;
    // second-pass results of FGMRES's Gram--Schmidt (device / pinned host) and
    // the squared column scales of its unnormalised basis (device)
    double *dres2 = nullptr, *hres2 = nullptr, *sc2d = nullptr;
    float *fg_f32 = nullptr, *fg_x32 = nullptr;
    double *gv_f64 = nullptr, *gv_x64 = nullptr;       // fixed in/out of the FP64 V-cycle graph
    hipGraphExec_t g_vc32 = nullptr, g_vc64 = nullptr, g_svc = nullptr;
    double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr;
    double *pj_g = nullptr, *pj_psi = nullptr, *pj_r = nullptr, *pj_z = nullptr,
           *pj_p = nullptr, *pj_q = nullptr;
    int eg_cap = 0;
    double *eg_V = nullptr, *eg_W = nullptr, *eg_T = nullptr, *eg_F = nullptr;
    // block basis work: coefficients (256 x 8, device), K of the new block,
    // Ritz vectors with their K and A images
    double *eg_C = nullptr, *eg_KV = nullptr, *eg_R = nullptr;
    int eg_kv_cap = 0, eg_r_cap = 0;
    // block solves (allocated on first use): FGMRES bases of kMaxRhs systems,
    // column j of system r at bk_V + (j * nrhs + r) * n0; per-system device
    // results / coefficients (kMaxDots each) and pinned host results
    int bk_m = 0;
    double *bk_V = nullptr, *bk_Z = nullptr;
    float *bk_Z32 = nullptr;   // FP32 preconditioned columns (plain FP32-multigrid mode)
    // FP32 basis (option krylov_basis_f32; same layout as bk_V) and the FP64
    // column of each system in which a new basis column is formed
    float *bk_V32 = nullptr;
    double *bk_W = nullptr;
    double *bk_dres = nullptr, *bk_dcoef = nullptr, *bk_hres = nullptr;
    // dres2 / hres2 follow dres / hres in the same allocations (one copy
    // brings both); hsc2 is the pinned host image of sc2
    double *bk_dres2 = nullptr, *bk_hres2 = nullptr, *bk_sc2 = nullptr, *bk_hsc2 = nullptr;
    hipGraphExec_t g_vb32[dm::kMaxRhs + 1] = {}, g_vb64[dm::kMaxRhs + 1] = {};
    // block projection: per-vector CG state (kMaxRhs * P each) and graphs
    double *pjb_g = nullptr, *pjb_psi = nullptr, *pjb_p = nullptr, *pjb_q = nullptr;
    hipGraphExec_t g_svb[dm::kMaxRhs + 1] = {};
    hipGraphExec_t g_svb32[dm::kMaxRhs + 1] = {};  // FP32 scalar block V-cycle with its casts
    std::vector<void *> allocs;  // everything to free
    int last_proj_iters = 0;
    // learned correction: the attached network (not owned) and its scratch
    dm_net *net = nullptr;
    double *ln_t1 = nullptr, *ln_t2 = nullptr, *ln_t3 = nullptr, *ln_t4 = nullptr;  // 3P each
    int ln_accepted = 0, ln_rejected = 0;
    // the residual judge on the device: two sums of squares, the decision
    // and its pinned host copy
    double *ln_d = nullptr;
    int *ln_flag = nullptr, *ln_hflag = nullptr;
    // batched runs: the batch whose fused V-cycle serves this op's FP32
    // preconditioner while dm_batch_eigs runs (not owned), and the op's index
    dm_batch *batch = nullptr;
    int batch_index = -1;
    // units of a level-0 face vector the Krylov solvers' reductions visit
    int32_t *vunit = nullptr;
    int64_t nvunit = 0;
    dm::Span vspan() const { return dm::Span{vunit, nvunit}; }
    // the same for a level-0 cell vector: units holding an active cell or a
    // PMC ghost image (the projection's conjugate-gradient vectors)
    int32_t *cunit = nullptr;
    int64_t ncunit = 0;
    dm::Span cspan() const { return dm::Span{cunit, ncunit}; }

    template <class T>
    T *dalloc(size_t count) {
        void *p = nullptr;
        DM_HIP(hipMalloc(&p, count * sizeof(T) + 256));
        allocs.push_back(p);
        DM_HIP(hipMemsetAsync(p, 0, count * sizeof(T) + 256, stream));
        return (T *)p;
    }
    int nlev() const { return (int)lv.size(); }
    int64_t n0() const { return 3 * lv[0].g.P; }
};

namespace dm {

constexpr int kMaxDots = 256;

// op.cpp
void build_hierarchy(dm_op *op, const double *user_frac);
void factor_coarse(dm_op *op);
double host_dot_sync(dm_op *op, hipStream_t s);

// solver.cpp
template <class T>
void vcycle(dm_op *op, int level, const T *f, T *x, hipStream_t s);
// dm_solve in the PCG64 mode with caller-provided work memory (4 * 3P
// doubles): r, z, p, q; allocates nothing
int solve_pcg_with(dm_op *op, const double *f, double *x, double rtol, int maxit, dm_solve_info *info,
                   hipStream_t s, double *work);
// the no-allocation entry point's scratch array (noalloc.hip): looked up once
// per device, with that device current; the device address, or NULL if the
// lookup failed (then the failure is thrown as DM_EHIP by noalloc_init)
void noalloc_init(int device);
double *noalloc_scratch(int device);
void svcycle(dm_op *op, int level, const double *f, double *x, hipStream_t s);
// device dots; results copied to op->hres (synchronises the stream)
void dots(dm_op *op, int nv, const double *V, int64_t ld, const double *w, const double *wt,
          int64_t n, hipStream_t s, Span sp = {});
int project(dm_op *op, const double *b, double *out, double rtol, int maxit, hipStream_t s,
            int *iters);
// project() on nr (1..kMaxRhs) vectors in lockstep; iters: nr entries or NULL;
// prec: precision of the scalar V-cycle preconditioning the conjugate
// gradients (64 or 32; the gradients themselves run in FP64 either way)
int project_block(dm_op *op, int nr, const double *const *b, double *const *out, double rtol, int maxit,
                  hipStream_t s, int *iters, int prec = 64);
int solve(dm_op *op, int mode, const double *f, double *x, double rtol, int maxit,
          dm_solve_info *info, hipStream_t s);
// nrhs (1..kMaxRhs) systems M x_r = f_r in lockstep, FGMRES modes only;
// info: nrhs entries or NULL; returns the worst status
int solve_block(dm_op *op, int mode, int nrhs, const double *const *f, double *const *x, double rtol, int maxit,
                dm_solve_info *info, hipStream_t s);
// block V-cycle graph: prec 32 runs lv[0].bf32 -> lv[0].bx32 (nrhs slots of
// 3P), prec 64 lv[0].bf64 -> lv[0].bx64
void ensure_block(dm_op *op, int prec);
void vcycle_block_graphed(dm_op *op, int prec, int nrhs, hipStream_t s);
// rejections: the solve's count of rejected learned corrections (learned mode)
void precondition(dm_op *op, int mode, const double *v, double *z, hipStream_t s, int *rejections = nullptr);
void ensure_krylov(dm_op *op);
// the single-vector solver's small buffers (casts, graph in/out, coefficients)
// without its FGMRES basis
void ensure_krylov_small(dm_op *op);
void ensure_proj(dm_op *op);
void invalidate_graphs(dm_op *op);
// V-cycle graphs: prec 32 runs fg_f32 -> fg_x32, prec 64 gv_f64 -> gv_x64;
// the scalar one pj_r -> pj_z
void vcycle_graphed(dm_op *op, int prec, hipStream_t s);
void svcycle_graphed(dm_op *op, hipStream_t s);
double dot1(dm_op *op, const double *x, const double *y, const double *wt, int64_t n, hipStream_t s,
            Span sp = {});
int eigs(dm_op *op, int k, double tol, uint64_t seed, const dm_eig_options &opt, double *lam,
         double *vecs, double *res, dm_eig_info *info, hipStream_t s);

}  // namespace dm

// The learned correction's network (learned.cpp): FP32 master weights, Adam
// state, bfloat16 device weights and the activation buffers of the grid of
// the operator it is attached to.
struct dm_net {
    int device = 0;
    float *w32 = nullptr, *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
    uint16_t *wf = nullptr, *wb = nullptr;   // [3][27][16][16] forward / data-gradient
    float *part = nullptr;                   // weight-gradient partials
    double *lpart = nullptr, *hl = nullptr;  // loss partials (device, pinned host)
    int64_t cap = 0;                         // cells the activation buffers hold
    uint16_t *x0 = nullptr, *a1 = nullptr, *a2 = nullptr, *dy = nullptr, *d2 = nullptr, *d1 = nullptr;
    float *y = nullptr;
    int64_t step = 0;
    dm_op *op = nullptr;                     // attached operator
    std::vector<void *> fixed_allocs, act_allocs;
};

namespace dm {
// learned.cpp
void net_init(dm_net *net, uint64_t seed);
void net_free(dm_net *net);
void net_upload_weights(dm_net *net, const float *host);
void net_attach(dm_op *op, dm_net *net);
void net_apply(dm_op *op, const double *r, double scale, double *out, hipStream_t s);
// the attached network's three convolutions on its current activations
void net_forward(dm_op *op, hipStream_t s);
double net_loss_grad(dm_op *op, int kind, const double *r, const double *e, double scale, hipStream_t s);
void net_make_pair(dm_op *op, uint64_t seed, double *r, double *e, hipStream_t s);
void net_train(dm_op *op, int kind, int steps, float lr, uint64_t seed, float *loss, hipStream_t s);
void net_train_pairs(dm_op *op, int kind, int npairs, const double *const *r, const double *const *e, float lr,
                     float *loss, hipStream_t s);
bool net_correct(dm_op *op, const double *v, double *z, hipStream_t s);
// the learned correction of one system of a solve, while its rejections stay
// below the op's patience (dm_options.learned_patience; 0: always)
inline void net_correct_patient(dm_op *op, const double *v, double *z, int *rejections, hipStream_t s) {
    const int pat = op->opt.learned_patience;
    if (pat > 0 && *rejections >= pat) return;
    if (!net_correct(op, v, z, s)) ++*rejections;
}
}  // namespace dm

// A batch of operators (cavities) whose FP32 V-cycles run as one fused
// sequence of batched launches recorded in one HIP graph (batch.cpp).
struct dm_batch {
    std::vector<dm_op *> ops;
    int device = 0;
    hipStream_t stream = nullptr;
    hipGraphExec_t graph = nullptr;   // fused V-cycle: every op's fg_f32 -> fg_x32
    int tpb = 256;                    // threads per block chosen by the autotuner
    double tuned_ms[3] = {0, 0, 0};   // graph time for 64, 128, 256 threads per block
    int nsteps = 0;                   // batched launches per fused V-cycle
    std::vector<void *> tables;       // device job tables of the current graph
    // lockstep: threads of dm_batch_eigs meet at every preconditioner call
    std::mutex mu;
    std::condition_variable cv;
    int active = 0, submitted = 0;
    uint64_t round = 0;
    std::vector<char> pending;
    std::vector<hipEvent_t> ev_in;
    hipEvent_t ev_done = nullptr;
};

namespace dm {
// batch.cpp
void batch_setup(dm_batch *b);                   // schedule, autotune, capture
void batch_release(dm_batch *b);
void batch_vcycle_lockstep(dm_op *op, hipStream_t s);   // op->fg_f32 -> op->fg_x32
void batch_leave(dm_batch *b);
}  // namespace dm
