// Learned correction, host side: weights, attachment to an operator, the
// correction inside the FP32-multigrid preconditioner, training pairs from
// the solver, loss/gradient and Adam training.  Kernels in learned.hip.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "learned.h"
#include "op.h"

namespace dm {

namespace {

constexpr int kLossBlocks = 512;

uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

template <class T>
T *net_alloc(size_t count, std::vector<void *> &list) {
    void *p = nullptr;
    DM_HIP(hipMalloc(&p, count * sizeof(T) + 256));
    DM_HIP(hipMemset(p, 0, count * sizeof(T) + 256));
    list.push_back(p);
    return (T *)p;
}

// activation buffers for op's finest grid; cleared whenever the grid
// changes, so that the padding layer of every buffer is zero
void ensure_activations(dm_net *net, const Grid &g) {
    const int64_t P = g.P;
    if (P > net->cap) {
        for (void *p : net->act_allocs) hipFree(p);
        net->act_allocs.clear();
        net->x0 = net_alloc<uint16_t>(P * kNetCh, net->act_allocs);
        net->a1 = net_alloc<uint16_t>(P * kNetCh, net->act_allocs);
        net->a2 = net_alloc<uint16_t>(P * kNetCh, net->act_allocs);
        net->dy = net_alloc<uint16_t>(P * kNetCh, net->act_allocs);
        net->d2 = net_alloc<uint16_t>(P * kNetCh, net->act_allocs);
        net->d1 = net_alloc<uint16_t>(P * kNetCh, net->act_allocs);
        net->y = net_alloc<float>(P * 4, net->act_allocs);
        net->cap = P;
    } else {
        const size_t bf = (size_t)net->cap * kNetCh * sizeof(uint16_t);
        for (uint16_t *b : {net->x0, net->a1, net->a2, net->dy, net->d2, net->d1})
            DM_HIP(hipMemset(b, 0, bf));
        DM_HIP(hipMemset(net->y, 0, (size_t)net->cap * 4 * sizeof(float)));
    }
}

void ensure_scratch(dm_op *op) {
    if (!op->ln_t1) {
        const int64_t n = op->n0();
        op->ln_t1 = op->dalloc<double>(n);
        op->ln_t2 = op->dalloc<double>(n);
        op->ln_t3 = op->dalloc<double>(n);
        op->ln_t4 = op->dalloc<double>(n);
        op->ln_d = op->dalloc<double>(2);
        op->ln_flag = op->dalloc<int>(1);
        DM_HIP(hipHostMalloc((void **)&op->ln_hflag, sizeof(int), hipHostMallocDefault));
    }
}

dm_net *attached(dm_op *op) {
    if (!op->net) throw DmError{DM_EINVAL, "no network attached to the operator (dm_net_attach)"};
    return op->net;
}

// the three forward layers on x0 (channels 0..2 already packed): y [P][4]
void forward(dm_net *net, const Grid &g, hipStream_t s) {
    launch_net_conv(NET_RELU, g, net->x0, net->wf, nullptr, net->a1, nullptr, s);
    launch_net_conv(NET_RELU, g, net->a1, net->wf + 27 * 256, nullptr, net->a2, nullptr, s);
    launch_net_conv(NET_LINEAR, g, net->a2, net->wf + 2 * 27 * 256, nullptr, nullptr, net->y, s);
}

// s = ||r|| / sqrt(active faces), over owned entries only
double rms_of(dm_op *op, const double *r, hipStream_t s) {
    const double n2 = dot1(op, r, r, op->wface, op->n0(), s);
    const double na = (double)std::max<int64_t>(1, op->lv[0].n_act_faces);
    return std::sqrt(n2 / na);
}

}  // namespace

void net_init(dm_net *net, uint64_t seed) {
    DM_HIP(hipGetDevice(&net->device));
    std::vector<void *> &fa = net->fixed_allocs;
    net->w32 = net_alloc<float>(kNetWeights, fa);
    net->adam_m = net_alloc<float>(kNetWeights, fa);
    net->adam_v = net_alloc<float>(kNetWeights, fa);
    net->grad = net_alloc<float>(kNetWeights, fa);
    net->wf = net_alloc<uint16_t>(3 * 27 * 256, fa);
    net->wb = net_alloc<uint16_t>(3 * 27 * 256, fa);
    net->part = net_alloc<float>((size_t)kNetWaves * 27 * 256, fa);
    net->lpart = net_alloc<double>(2 * kLossBlocks, fa);
    DM_HIP(hipHostMalloc((void **)&net->hl, 2 * kLossBlocks * sizeof(double), hipHostMallocDefault));
    net->cap = 0;
    std::vector<float> w(kNetWeights);
    uint64_t ctr = 0;
    for (int l = 0; l < 3; ++l) {
        const int64_t o = net_offset(l), n = 27LL * kNetIn[l] * kNetOut[l];
        const double bound = std::sqrt(6.0 / (27.0 * kNetIn[l])) * (l == 2 ? 0.1 : 1.0);
        for (int64_t q = 0; q < n; ++q) {
            const double u = (double)(splitmix64(seed ^ splitmix64(ctr++)) >> 11) * 0x1.0p-53;
            w[o + q] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    net_upload_weights(net, w.data());
}

void net_free(dm_net *net) {
    hipSetDevice(net->device);
    hipDeviceSynchronize();
    for (void *p : net->act_allocs) hipFree(p);
    for (void *p : net->fixed_allocs) hipFree(p);
    net->act_allocs.clear();
    net->fixed_allocs.clear();
    if (net->hl) hipHostFree(net->hl);
}

void net_upload_weights(dm_net *net, const float *host) {
    DM_HIP(hipMemcpy(net->w32, host, kNetWeights * sizeof(float), hipMemcpyHostToDevice));
    launch_net_pack_weights(net->w32, net->wf, net->wb, nullptr);
    DM_HIP(hipGetLastError());
    DM_HIP(hipDeviceSynchronize());
}

void net_attach(dm_op *op, dm_net *net) {
    if (op->net && op->net != net) op->net->op = nullptr;
    op->net = nullptr;
    if (!net) return;
    if (net->device != op->device) throw DmError{DM_EINVAL, "network and operator on different devices"};
    if (net->op && net->op != op) net->op->net = nullptr;
    // a fresh binding: activation buffers for this grid, fraction channels 3..9
    const Grid &g = op->lv[0].g;
    ensure_activations(net, g);
    const int64_t P = g.P;
    const std::vector<double> &fr = op->frac[0];   // ax ay az lx ly lz v (7P)
    std::vector<uint16_t> host((size_t)P * kNetCh, 0);
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                const int64_t p = pidx(g, i, j, k);
                for (int c = 0; c < 7; ++c) host[(size_t)p * kNetCh + 3 + c] = f2bf((float)fr[c * P + p]);
            }
    DM_HIP(hipMemcpy(net->x0, host.data(), host.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    ensure_scratch(op);
    op->net = net;
    net->op = op;
}

void net_forward(dm_op *op, hipStream_t s) {
    dm_net *net = attached(op);
    forward(net, op->lv[0].g, s);
}

void net_apply(dm_op *op, const double *r, double scale, double *out, hipStream_t s) {
    dm_net *net = attached(op);
    const Level &L = op->lv[0];
    const double sc = scale > 0.0 ? scale : rms_of(op, r, s);
    if (!(sc > 0.0) || !std::isfinite(sc)) {
        DM_HIP(hipMemsetAsync(out, 0, op->n0() * sizeof(double), s));
        return;
    }
    launch_net_pack_r<double>(L.g, r, 1.0 / sc, net->x0, s);
    forward(net, L.g, s);
    launch_net_unpack<double>(L.g, L.coef64, net->y, sc * L.g.h * L.g.h, out, s);
}

// z += correction of the V-cycle's answer z for right-hand side v, kept only
// if it lowers ||v - M z||; returns whether it was kept
bool net_correct(dm_op *op, const double *v, double *z, hipStream_t s) {
    dm_net *net = attached(op);
    const Level &L = op->lv[0];
    const int64_t n = op->n0();
    double *r2 = op->ln_t1, *dz = op->ln_t2, *r3 = op->ln_t3;
    const double inv_cnt = 1.0 / (double)std::max<int64_t>(1, L.n_act_faces);
    // r' = v - M z and |r'|^2; the input scale s = |r'| / sqrt(active faces)
    // is read on the device, so nothing waits for the host before the judge
    launch_apply<double>(L.g, L.coef64, op->sigma, AK_RESID, v, z, r2, s, L.cut_cells());
    launch_mdot(1, r2, 0, r2, op->wface, n, op->part, op->ln_d, s, op->vspan());
    launch_net_pack_r_dev(L.g, r2, op->ln_d, inv_cnt, net->x0, s);
    forward(net, L.g, s);
    launch_net_unpack_dev(L.g, L.coef64, net->y, L.g.h * L.g.h, op->ln_d, inv_cnt, dz, s);
    launch_apply<double>(L.g, L.coef64, op->sigma, AK_RESID, r2, dz, r3, s, L.cut_cells());
    launch_mdot(1, r3, 0, r3, op->wface, n, op->part, op->ln_d + 1, s, op->vspan());
    launch_net_accept(n, op->ln_d, dz, z, op->ln_flag, s);
    DM_HIP(hipMemcpyAsync(op->ln_hflag, op->ln_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DM_HIP(hipStreamSynchronize(s));
    if (*op->ln_hflag) {
        ++op->ln_accepted;
        return true;
    }
    ++op->ln_rejected;
    return false;
}

double net_loss_grad(dm_op *op, int kind, const double *r, const double *e, double scale, hipStream_t s) {
    dm_net *net = attached(op);
    const Level &L = op->lv[0];
    const Grid &g = L.g;
    const int64_t n = op->n0();
    const double sc = scale > 0.0 ? scale : rms_of(op, r, s);
    if (!(sc > 0.0) || !std::isfinite(sc)) throw DmError{DM_EINVAL, "training pair with a zero residual"};
    launch_net_pack_r<double>(g, r, 1.0 / sc, net->x0, s);
    forward(net, g, s);
    const double c = sc * g.h * g.h;   // output scale
    double loss = 0.0;
    if (kind == DM_NET_LOSS_ERROR) {
        if (!e) throw DmError{DM_EINVAL, "error loss needs the error e"};
        // pass 0: sum t^2; pass 1: dy and sum (y - t)^2, t = e / c
        launch_net_loss(g, L.coef64, net->y, e, 1.0 / c, 0.0, net->dy, net->lpart, kLossBlocks, 0, s);
        DM_HIP(hipMemcpyAsync(net->hl, net->lpart, 2 * kLossBlocks * sizeof(double), hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        double st = 0.0;
        for (int q = 0; q < kLossBlocks; ++q) st += net->hl[2 * q + 1];
        if (!(st > 0.0)) throw DmError{DM_EINVAL, "training pair with a zero target"};
        launch_net_loss(g, L.coef64, net->y, e, 1.0 / c, 1.0 / st, net->dy, net->lpart, kLossBlocks, 1, s);
        DM_HIP(hipMemcpyAsync(net->hl, net->lpart, 2 * kLossBlocks * sizeof(double), hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        double se = 0.0;
        for (int q = 0; q < kLossBlocks; ++q) se += net->hl[2 * q];
        loss = se / st;
    } else {
        // d = correction, r3 = r - M d, L = |r3|^2 / |r|^2, dL/dd = -2 M r3 / |r|^2
        double *d = op->ln_t3, *r3 = op->ln_t4;
        launch_net_unpack<double>(g, L.coef64, net->y, c, d, s);
        launch_apply<double>(g, L.coef64, op->sigma, AK_RESID, r, d, r3, s, L.cut_cells());
        const double rr = dot1(op, r, r, op->wface, n, s);
        const double r33 = dot1(op, r3, r3, op->wface, n, s);
        launch_apply<double>(g, L.coef64, op->sigma, AK_M, nullptr, r3, d, s, L.cut_cells());
        launch_net_dy_from_face(g, L.coef64, d, -2.0 * c / rr, net->dy, s);
        loss = r33 / rr;
    }
    // layer 3: weights from a2 and dy; data gradient into d2 (masked by a2 > 0)
    launch_net_wgrad(g, net->a2, net->dy, net->part, s);
    launch_net_wgrad_reduce(net->part, kNetIn[2], kNetOut[2], net->grad + net_offset(2), s);
    launch_net_conv(NET_MASKED, g, net->dy, net->wb + 2 * 27 * 256, net->a2, net->d2, nullptr, s);
    // layer 2
    launch_net_wgrad(g, net->a1, net->d2, net->part, s);
    launch_net_wgrad_reduce(net->part, kNetIn[1], kNetOut[1], net->grad + net_offset(1), s);
    launch_net_conv(NET_MASKED, g, net->d2, net->wb + 27 * 256, net->a1, net->d1, nullptr, s);
    // layer 1
    launch_net_wgrad(g, net->x0, net->d1, net->part, s);
    launch_net_wgrad_reduce(net->part, kNetIn[0], kNetOut[0], net->grad, s);
    DM_HIP(hipGetLastError());
    return loss;
}

void net_make_pair(dm_op *op, uint64_t seed, double *r, double *e, hipStream_t s) {
    ensure_scratch(op);
    const Level &L = op->lv[0];
    const int64_t n = op->n0();
    double *w = op->ln_t3, *f = op->ln_t4;
    ensure_krylov_small(op);   // the FP32 V-cycle's cast buffers
    launch_randn(n, seed, 0, op->fmask, w, s);
    precondition(op, DM_SOLVE_FGMRES_MG32, w, e, s);          // e holds x* for now
    launch_apply<double>(L.g, L.coef64, op->sigma, AK_M, nullptr, e, f, s, L.cut_cells());
    precondition(op, DM_SOLVE_FGMRES_MG32, f, w, s);          // w = z
    launch_apply<double>(L.g, L.coef64, op->sigma, AK_RESID, f, w, r, s, L.cut_cells());
    launch_axpy(n, -1.0, w, e, s);                            // e = x* - z
    DM_HIP(hipGetLastError());
}

namespace {

// one Adam step (Kingma & Ba) of the FP32 master weights from net->grad
void adam_step(dm_net *net, float lr, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    ++net->step;
    const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
    launch_net_adam(net->grad, net->w32, net->adam_m, net->adam_v, kNetWeights, lr, b1, b2, eps, c1, c2, s);
    launch_net_pack_weights(net->w32, net->wf, net->wb, s);
}

}  // namespace

void net_train(dm_op *op, int kind, int steps, float lr, uint64_t seed, float *loss, hipStream_t s) {
    dm_net *net = attached(op);
    ensure_scratch(op);
    for (int it = 0; it < steps; ++it) {
        net_make_pair(op, seed + (uint64_t)it, op->ln_t1, op->ln_t2, s);
        const double L = net_loss_grad(op, kind, op->ln_t1, op->ln_t2, 0.0, s);
        if (loss) loss[it] = (float)L;
        adam_step(net, lr, s);
    }
    DM_HIP(hipGetLastError());
    DM_HIP(hipStreamSynchronize(s));
}

void net_train_pairs(dm_op *op, int kind, int npairs, const double *const *r, const double *const *e, float lr,
                     float *loss, hipStream_t s) {
    dm_net *net = attached(op);
    ensure_scratch(op);
    for (int it = 0; it < npairs; ++it) {
        const double L = net_loss_grad(op, kind, r[it], e ? e[it] : nullptr, 0.0, s);
        if (loss) loss[it] = (float)L;
        adam_step(net, lr, s);
    }
    DM_HIP(hipGetLastError());
    DM_HIP(hipStreamSynchronize(s));
}

}  // namespace dm
