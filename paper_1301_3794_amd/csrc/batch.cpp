// Batched cavities: one fused FP32 V-cycle for every operator of a batch.
//
// The V-cycles of the members are merged level by level into batched
// launches (kernels.hip, launch_batched): at depth d every member that still
// has a coarser level smooths, forms its residual and restricts; a member
// whose coarsest level is d solves it there; on the way up the members
// prolong and post-smooth.  Each member's sequence of operations is exactly
// its own V-cycle's, so the results are those of the single-operator
// V-cycle; only the launches are shared.  The fused sequence is recorded in
// one HIP graph, for the block size (64, 128 or 256 threads) that the
// autotuner timed fastest.
//
// dm_batch_eigs runs every member's eigensolve on its own host thread and
// stream; at each FP32 preconditioner call the threads meet, and the last to
// arrive launches the graph once for all of them (ordered after every
// member's input by events, and every member waits for its completion).
#include <algorithm>
#include <chrono>
#include <cstring>

#include "op.h"

namespace dm {

namespace {

struct HostStep {
    int kind, comp, colour;
    std::vector<BJob> jobs;
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct LevelBufs {
    const float *c;
    float *f, *x, *r;
};

LevelBufs bufs(dm_op *op, int l) {
    Level &L = op->lv[l];
    if (l == 0) return {L.coef32, op->fg_f32, op->fg_x32, L.r32};
    return {L.coef32, L.f32, L.x32, L.r32};
}

int64_t cells(const Grid &g) { return (int64_t)g.nx * g.ny * g.nz; }

// the fused V-cycle as a list of batched steps
std::vector<HostStep> schedule(dm_batch *b) {
    std::vector<HostStep> st;
    int dmax = 0;
    for (dm_op *op : b->ops) dmax = std::max(dmax, op->nlev());
    const int nu_pre = b->ops[0]->opt.nu_pre, nu_post = b->ops[0]->opt.nu_post;
    auto add = [&](int kind, int comp, int colour, std::vector<BJob> jobs) {
        if (!jobs.empty()) st.push_back({kind, comp, colour, std::move(jobs)});
    };
    auto job = [&](dm_op *op, int l) {
        BJob J{};
        J.g = op->lv[l].g;
        if (l + 1 < op->nlev()) {
            J.gc = op->lv[l + 1].g;
            J.cc = op->lv[l + 1].coef32;
        }
        J.c = op->lv[l].coef32;
        J.sigma = op->sigma;
        return J;
    };
    for (int d = 0; d < dmax; ++d) {
        std::vector<BJob> zero, coarse, resid, restr;
        for (dm_op *op : b->ops) {
            const int nl = op->nlev();
            if (d >= nl) continue;
            const LevelBufs B = bufs(op, d);
            BJob z = job(op, d);
            z.out = B.x;
            z.items = 3 * z.g.P;
            zero.push_back(z);
            if (d == nl - 1) {
                BJob c = job(op, d);
                c.in = B.f;
                c.out = B.x;
                c.inv = op->cinv;
                c.idx = op->cidx;
                c.ncoarse = op->nc;
                c.items = op->nc;
                coarse.push_back(c);
            }
        }
        add(BS_ZERO, 0, 0, zero);
        add(BS_COARSE, 0, 0, coarse);
        std::vector<BJob> sm;
        for (dm_op *op : b->ops)
            if (d < op->nlev() - 1) {
                const LevelBufs B = bufs(op, d);
                BJob J = job(op, d);
                J.in = B.f;
                J.out = B.x;
                J.items = (int64_t)((J.g.nx + 1) >> 1) * J.g.ny * J.g.nz;
                sm.push_back(J);
                BJob R = job(op, d);
                R.in = B.f;
                R.aux = B.x;
                R.out = B.r;
                R.items = cells(R.g);
                resid.push_back(R);
                BJob T = job(op, d);
                T.in = B.r;
                T.out = bufs(op, d + 1).f;
                T.items = cells(T.gc);
                restr.push_back(T);
            }
        for (int it = 0; it < nu_pre; ++it)
            for (int comp = 0; comp < 3; ++comp)
                for (int col = 0; col < 2; ++col) add(BS_SMOOTH, comp, col, sm);
        add(BS_RESID, 0, 0, resid);
        add(BS_RESTRICT, 0, 0, restr);
    }
    for (int d = dmax - 2; d >= 0; --d) {
        std::vector<BJob> pro, sm;
        for (dm_op *op : b->ops)
            if (d < op->nlev() - 1) {
                const LevelBufs B = bufs(op, d);
                BJob P = job(op, d);
                P.in = bufs(op, d + 1).x;
                P.out = B.x;
                P.items = cells(P.g);
                pro.push_back(P);
                BJob J = job(op, d);
                J.in = B.f;
                J.out = B.x;
                J.items = (int64_t)((J.g.nx + 1) >> 1) * J.g.ny * J.g.nz;
                sm.push_back(J);
            }
        add(BS_PROLONG, 0, 0, pro);
        for (int it = 0; it < nu_post; ++it)
            for (int comp = 2; comp >= 0; --comp)
                for (int col = 1; col >= 0; --col) add(BS_SMOOTH, comp, col, sm);
    }
    return st;
}

void free_tables(dm_batch *b) {
    for (void *p : b->tables) (void)hipFree(p);
    b->tables.clear();
}

// job tables for block size tpb, then the fused V-cycle recorded into a graph
hipGraphExec_t capture(dm_batch *b, const std::vector<HostStep> &steps, int tpb) {
    std::vector<std::pair<const BJob *, std::pair<int, int64_t>>> launches;
    for (const HostStep &h : steps) {
        std::vector<BJob> jobs = h.jobs;
        int64_t blocks = 0;
        for (BJob &J : jobs) {
            J.block0 = blocks;
            blocks += h.kind == BS_COARSE ? J.items : std::max<int64_t>(1, cdiv(J.items, tpb));
        }
        void *dev = nullptr;
        DM_HIP(hipMalloc(&dev, jobs.size() * sizeof(BJob)));
        b->tables.push_back(dev);
        DM_HIP(hipMemcpy(dev, jobs.data(), jobs.size() * sizeof(BJob), hipMemcpyHostToDevice));
        launches.push_back({(const BJob *)dev, {(int)jobs.size(), blocks}});
    }
    hipGraph_t gph = nullptr;
    hipGraphExec_t exec = nullptr;
    DM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (size_t q = 0; q < steps.size(); ++q)
        launch_batched(steps[q].kind, steps[q].comp, steps[q].colour, launches[q].first, launches[q].second.first,
                       launches[q].second.second, tpb, b->stream);
    const hipError_t e1 = hipStreamEndCapture(b->stream, &gph);
    if (e1 != hipSuccess) {
        if (gph) (void)hipGraphDestroy(gph);
        DM_HIP(e1);
    }
    const hipError_t e2 = hipGraphInstantiate(&exec, gph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gph);
    DM_HIP(e2);
    return exec;
}

double time_graph(dm_batch *b, hipGraphExec_t g, int reps) {
    hipEvent_t e0, e1;
    DM_HIP(hipEventCreate(&e0));
    DM_HIP(hipEventCreate(&e1));
    DM_HIP(hipGraphLaunch(g, b->stream));
    DM_HIP(hipEventRecord(e0, b->stream));
    for (int r = 0; r < reps; ++r) DM_HIP(hipGraphLaunch(g, b->stream));
    DM_HIP(hipEventRecord(e1, b->stream));
    DM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DM_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}

// launch the fused V-cycle for the members that submitted (caller holds mu)
void run_round(dm_batch *b) {
    for (size_t i = 0; i < b->ops.size(); ++i)
        if (b->pending[i]) DM_HIP(hipStreamWaitEvent(b->stream, b->ev_in[i], 0));
    DM_HIP(hipGraphLaunch(b->graph, b->stream));
    DM_HIP(hipEventRecord(b->ev_done, b->stream));
    std::fill(b->pending.begin(), b->pending.end(), 0);
    b->submitted = 0;
    ++b->round;
    b->cv.notify_all();
}

}  // namespace

void batch_setup(dm_batch *b) {
    for (dm_op *op : b->ops) {
        if (op->lv[0].g.pmc) throw DmError{DM_EINVAL, "batched cavities without PMC planes only"};
        if (op->opt.nu_pre != b->ops[0]->opt.nu_pre || op->opt.nu_post != b->ops[0]->opt.nu_post)
            throw DmError{DM_EINVAL, "batch members need the same smoothing counts"};
        ensure_krylov_small(op);   // fg_f32 / fg_x32: the fused V-cycle's level-0 buffers
    }
    DM_HIP(hipDeviceSynchronize());
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    free_tables(b);
    const std::vector<HostStep> steps = schedule(b);
    b->nsteps = (int)steps.size();
    // autotuner: time the fused V-cycle at 64, 128 and 256 threads per block
    const int cand[3] = {64, 128, 256};
    double best = 1e300;
    int best_tpb = 256;
    for (int q = 0; q < 3; ++q) {
        hipGraphExec_t g = capture(b, steps, cand[q]);
        b->tuned_ms[q] = time_graph(b, g, 5);
        (void)hipGraphExecDestroy(g);
        if (b->tuned_ms[q] < best) {
            best = b->tuned_ms[q];
            best_tpb = cand[q];
        }
        DM_HIP(hipStreamSynchronize(b->stream));
        free_tables(b);
    }
    b->tpb = best_tpb;
    b->graph = capture(b, steps, best_tpb);
    DM_HIP(hipStreamSynchronize(b->stream));
}

void batch_release(dm_batch *b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    free_tables(b);
}

void batch_vcycle_lockstep(dm_op *op, hipStream_t s) {
    dm_batch *b = op->batch;
    const int me = op->batch_index;
    DM_HIP(hipEventRecord(b->ev_in[me], s));
    {
        std::unique_lock<std::mutex> lk(b->mu);
        const uint64_t my_round = b->round;
        b->pending[me] = 1;
        ++b->submitted;
        if (b->submitted == b->active) run_round(b);
        else b->cv.wait(lk, [&] { return b->round != my_round; });
    }
    DM_HIP(hipStreamWaitEvent(s, b->ev_done, 0));
}

void batch_leave(dm_batch *b) {
    std::unique_lock<std::mutex> lk(b->mu);
    --b->active;
    if (b->submitted > 0 && b->submitted == b->active) run_round(b);
}

}  // namespace dm
