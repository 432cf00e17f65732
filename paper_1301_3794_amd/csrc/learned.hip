// Learned correction kernels: 3-D convolutions on MFMA (bfloat16 in, FP32
// accumulate), weight gradients, loss, packing and Adam.
//
// MFMA tile (v_mfma_f32_16x16x16_bf16, one wavefront): A is 16 x 16 (rows x
// k), B is 16 x 16 (k x cols), D = A B + C is 16 x 16 FP32.  Lane l holds
// A[l % 16][4 (l / 16) + 0..3], B[4 (l / 16) + 0..3][l % 16] and
// D[4 (l / 16) + 0..3][l % 16].
//
// Convolution as 27 accumulated tile products: rows = 16 consecutive cells
// along x, k = the 16 input channels at one tap, cols = the 16 output
// channels.  A wavefront owns one 16-cell segment of an x-row; the weights
// of the layer (27 x 16 x 16 bfloat16, 13.5 KB) sit in LDS.  The padding
// layer of every activation buffer is zero, so taps that leave the grid read
// zeros; cells past the ragged row end are neither read nor written.

#include "learned.h"

namespace dm {
namespace {

constexpr int kT = 256;  // threads per block (4 wavefronts)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline int64_t tap_offset(const Grid &g, int t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    return (int64_t)dx + (int64_t)dy * g.sy + (int64_t)dz * g.sz;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A workgroup computes one tile of 16 x kTileY x kTileZ cells: the input
// cells of the tile and its one-cell halo (18 x (kTileY + 2) x (kTileZ + 2),
// 16 channels each) are staged in LDS once, so each activation is fetched
// from memory about twice instead of once per tap; wave w then takes the
// x-segments of y-row w, one z-plane after another.  Cells outside the padded
// grid are staged as zeros (the padding layer itself holds zeros).  Each
// wave keeps the layer's weights for its lanes in registers (27 x 8 bytes),
// and staged cells sit 48 bytes apart, so that the 8-byte reads of half a
// wavefront (16 cells x 2 channel groups) fall on 64 distinct banks.
constexpr int kTileY = 4, kTileZ = 8;
constexpr int kTileCells = 18 * (kTileY + 2) * (kTileZ + 2);
constexpr int kCellStride = 3;   // in 16-byte units (32 bytes of data, 16 of padding)

template <int MODE>
__global__ void __launch_bounds__(kT)
k_net_conv(Grid g, const uint16_t *__restrict__ in, const uint16_t *__restrict__ w,
           const uint16_t *__restrict__ mask, uint16_t *__restrict__ out_bf, float *__restrict__ out_f) {
    static_assert(kT / 64 == kTileY, "one wave per y-row of the tile");
    __shared__ uint4 xs[kTileCells * kCellStride];
    const int nsx = (g.nx + 15) >> 4, nty = (g.ny + kTileY - 1) / kTileY;
    const int64_t b = blockIdx.x;
    const int sx = (int)(b % nsx);
    const int64_t rest = b / nsx;
    const int j0 = (int)(rest % nty) * kTileY, k0 = (int)(rest / nty) * kTileZ;
    const int i0 = sx * 16;
    for (int e = threadIdx.x; e < kTileCells * 2; e += kT) {
        const int c = e >> 1, half = e & 1;
        const int xi = c % 18, yi = (c / 18) % (kTileY + 2), zi = c / (18 * (kTileY + 2));
        // cell (i, j, k) of the grid, padding at -1 and n
        const int i = i0 - 1 + xi, j = j0 - 1 + yi, k = k0 - 1 + zi;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (i <= g.nx && j <= g.ny && k <= g.nz)
            v = reinterpret_cast<const uint4 *>(in + pidx(g, i, j, k) * kNetCh)[half];
        xs[c * kCellStride + half] = v;
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, kg = lane >> 4;
    // this lane's A operands: output channel col, input channels 4 kg .. 4 kg + 3, every tap
    uint2 wr[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) wr[t] = *reinterpret_cast<const uint2 *>(w + t * 256 + col * 16 + 4 * kg);
    __syncthreads();
    const int j = j0 + wv;
    if (j >= g.ny) return;
    const int ia = i0 + col;
    const bool va = ia < g.nx;
    const uint2 *xs2 = reinterpret_cast<const uint2 *>(xs);
    // two z-planes at a time: their product chains are independent, so one
    // hides the other's latency
    for (int zz = 0; zz < kTileZ; zz += 2) {
        if (k0 + zz >= g.nz) break;
        // all 2 x 27 taps from LDS before the first product
        uint2 raw[2][27];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int t = 0; t < 27; ++t) {
                const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
                const int c = (col + 1 + dx) + 18 * ((wv + 1 + dy) + (kTileY + 2) * (zz + h + 1 + dz));
                raw[h][t] = xs2[c * (2 * kCellStride) + kg];
            }
        // D = W X: rows the output channels (A = the tap's weights, row = output
        // channel, k = input channel), columns the 16 cells (B = the inputs,
        // k = input channel, column = cell); lane (col, kg) ends with output
        // channels 4 kg .. 4 kg + 3 of cell i0 + col, stored as one 8-byte
        // write (a wavefront writes the segment's 512 contiguous bytes)
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const bf16x4 aw = *reinterpret_cast<const bf16x4 *>(&wr[t]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint2 xv = va ? raw[h][t] : make_uint2(0u, 0u);
                const bf16x4 bx = *reinterpret_cast<const bf16x4 *>(&xv);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aw, bx, acc[h], 0, 0, 0);
            }
        }
        if (!va) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = k0 + zz + h;
            if (k >= g.nz) break;
            const int64_t p = pidx(g, ia, j, k);
            if (MODE == NET_LINEAR) {
                if (kg == 0)
                    *reinterpret_cast<float4 *>(out_f + p * 4) = make_float4(acc[h][0], acc[h][1], acc[h][2], acc[h][3]);
                continue;
            }
            uint16_t o[4];
            if (MODE == NET_RELU) {
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = f2bf(acc[h][r] > 0.f ? acc[h][r] : 0.f);
            } else {
                const uint2 mraw = *reinterpret_cast<const uint2 *>(mask + p * kNetCh + 4 * kg);
                const uint16_t *m = reinterpret_cast<const uint16_t *>(&mraw);
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = f2bf(bf2f(m[r]) > 0.f ? acc[h][r] : 0.f);
            }
            *reinterpret_cast<uint2 *>(out_bf + p * kNetCh + 4 * kg) =
                make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16));
        }
    }
}

// Weight gradient: per tap, D[c][o] += sum over 16 cells of x[cell + off][c] d[cell][o]
// (A = x^T: rows c, k = cells; B = d: k = cells, cols o).  Each wavefront
// sweeps segments with a stride of kNetWaves and writes its 27 tiles.
__global__ void __launch_bounds__(kT)
k_net_wgrad(Grid g, const uint16_t *__restrict__ x, const uint16_t *__restrict__ d, float *__restrict__ part) {
    const int wave = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, col = lane & 15, kg = lane >> 4;
    const int nsx = (g.nx + 15) >> 4;
    const int64_t nseg = (int64_t)nsx * g.ny * g.nz;
    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t seg = wave; seg < nseg; seg += kNetWaves) {
        const int sx = (int)(seg % nsx);
        const int64_t rest = seg / nsx;
        const int j = (int)(rest % g.ny), k = (int)(rest / g.ny);
        // this lane's 4 cells: i0 + 4 kg + 0..3
        int64_t pc[4];
        bool vc[4];
        bf16x4 b;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = sx * 16 + 4 * kg + r;
            vc[r] = i < g.nx;
            pc[r] = pidx(g, vc[r] ? i : 0, j, k);
            b[r] = vc[r] ? (short)d[pc[r] * kNetCh + col] : (short)0;
        }
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int64_t off = tap_offset(g, t);
            bf16x4 a;
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = vc[r] ? (short)x[(pc[r] + off) * kNetCh + col] : (short)0;
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
    float *dst = part + (int64_t)wave * 27 * 256;
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[t * 256 + (4 * kg + r) * 16 + col] = acc[t][r];
}

__global__ void __launch_bounds__(kT)
k_net_wgrad_reduce(const float *__restrict__ part, int cin, int cout, float *__restrict__ grad) {
    // one block per (tap, c); threads over waves, 16 outputs each
    const int t = blockIdx.x / 16, c = blockIdx.x % 16;
    __shared__ float red[kT][17];
    float s[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) s[o] = 0.f;
    for (int wv = threadIdx.x; wv < kNetWaves; wv += kT) {
        const float *src = part + (int64_t)wv * 27 * 256 + t * 256 + c * 16;
#pragma unroll
        for (int o = 0; o < 16; ++o) s[o] += src[o];
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) red[threadIdx.x][o] = s[o];
    __syncthreads();
    if (threadIdx.x < 16 && c < cin && (int)threadIdx.x < cout) {
        float tot = 0.f;
        for (int q = 0; q < kT; ++q) tot += red[q][threadIdx.x];
        grad[(t * cin + c) * cout + threadIdx.x] = tot;
    }
}

template <class T>
__global__ void __launch_bounds__(kT)
k_net_pack_r(Grid g, const T *__restrict__ r, double inv_s, const double *__restrict__ ss, double inv_cnt,
             uint16_t *__restrict__ x0) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= n) return;
    if (ss) {
        // the scale from a sum of squares on the device: s = sqrt(ss * inv_cnt)
        const double sc = sqrt(ss[0] * inv_cnt);
        inv_s = sc > 0.0 ? 1.0 / sc : 0.0;
    }
    const int i = (int)(t % g.nx);
    const int64_t q = t / g.nx;
    const int j = (int)(q % g.ny), k = (int)(q / g.ny);
    const int64_t p = pidx(g, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c) x0[p * kNetCh + c] = f2bf((float)((double)r[c * g.P + p] * inv_s));
}

template <class T>
__global__ void __launch_bounds__(kT)
k_net_unpack(Grid g, const T *__restrict__ coef, const float *__restrict__ y, double scale,
             const double *__restrict__ ss, double inv_cnt, T *__restrict__ out) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= n) return;
    if (ss) scale *= sqrt(ss[0] * inv_cnt);
    const int i = (int)(t % g.nx);
    const int64_t q = t / g.nx;
    const int j = (int)(q % g.ny), k = (int)(q / g.ny);
    const int64_t p = pidx(g, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c)
        put_face<T>(g, out + c * g.P, c, i, j, k, p,
                    coef[c * g.P + p] != T(0) ? (T)((double)y[p * 4 + c] * scale) : T(0));
}

__global__ void __launch_bounds__(kT)
k_net_loss(Grid g, const double *__restrict__ coef, const float *__restrict__ y, const double *__restrict__ e,
           double t_scale, double inv_norm, uint16_t *__restrict__ dy, double *__restrict__ part, int pass) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    double s_err = 0.0, s_t = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < n; t += (int64_t)gridDim.x * kT) {
        const int i = (int)(t % g.nx);
        const int64_t q = t / g.nx;
        const int j = (int)(q % g.ny), k = (int)(q / g.ny);
        const int64_t p = pidx(g, i, j, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (coef[c * g.P + p] == 0.0) {
                if (pass == 1) dy[p * kNetCh + c] = 0;
                continue;
            }
            const double tv = e[c * g.P + p] * t_scale;
            if (pass == 0) {
                s_t += tv * tv;
            } else {
                const double diff = (double)y[p * 4 + c] - tv;
                s_err += diff * diff;
                dy[p * kNetCh + c] = f2bf((float)(2.0 * diff * inv_norm));
            }
        }
    }
    __shared__ double red[2][kT];
    red[0][threadIdx.x] = s_err;
    red[1][threadIdx.x] = s_t;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

// dy channel c = bf16(g_c * factor) on active faces, 0 elsewhere
__global__ void __launch_bounds__(kT)
k_net_dy_from_face(Grid g, const double *__restrict__ coef, const double *__restrict__ gv, double factor,
                   uint16_t *__restrict__ dy) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= n) return;
    const int i = (int)(t % g.nx);
    const int64_t q = t / g.nx;
    const int j = (int)(q % g.ny), k = (int)(q / g.ny);
    const int64_t p = pidx(g, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c)
        dy[p * kNetCh + c] = coef[c * g.P + p] != 0.0 ? f2bf((float)(gv[c * g.P + p] * factor)) : (uint16_t)0;
}

// wf[l][t][o][c] = bf16(W_l[t][c][o]);  wb[l][t][c][o] = bf16(W_l[26 - t][c][o])
// (the data gradient is the forward conv of d with the flipped taps and the
// roles of in and out channels exchanged); zero-padded to 16 x 16.
__global__ void __launch_bounds__(kT)
k_net_pack_weights(const float *__restrict__ w32, uint16_t *__restrict__ wf, uint16_t *__restrict__ wb) {
    const int l = blockIdx.x / 27, t = blockIdx.x % 27;
    const int a = threadIdx.x / 16, b = threadIdx.x % 16;   // row, column of the 16 x 16 tile
    const int cin = kNetIn[l], cout = kNetOut[l];
    int64_t base = 0;
    for (int q = 0; q < l; ++q) base += 27 * kNetIn[q] * kNetOut[q];
    // forward: row = out channel a, column = in channel b
    const float vf = (b < cin && a < cout) ? w32[base + (t * cin + b) * cout + a] : 0.f;
    wf[((int64_t)l * 27 + t) * 256 + a * 16 + b] = f2bf(vf);
    // data gradient: row = in channel a of the layer (its output), column = out channel b
    const float vb = (a < cin && b < cout) ? w32[base + ((26 - t) * cin + a) * cout + b] : 0.f;
    wb[((int64_t)l * 27 + t) * 256 + a * 16 + b] = f2bf(vb);
}

// Adam (Kingma & Ba, Algorithm 1); c1 = 1 - b1^step, c2 = 1 - b2^step
__global__ void __launch_bounds__(kT)
k_net_adam(const float *__restrict__ g, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
           int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int q = blockIdx.x * kT + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

}  // namespace

void launch_net_conv(int mode, const Grid &g, const uint16_t *in, const uint16_t *w, const uint16_t *mask,
                     uint16_t *out_bf, float *out_f, hipStream_t s) {
    // one workgroup per tile of 16 x kTileY x kTileZ cells
    const dim3 grid((unsigned)(ceil_div(g.nx, 16) * ceil_div(g.ny, kTileY) * ceil_div(g.nz, kTileZ)));
    if (mode == NET_RELU)
        hipLaunchKernelGGL(k_net_conv<NET_RELU>, grid, dim3(kT), 0, s, g, in, w, mask, out_bf, out_f);
    else if (mode == NET_MASKED)
        hipLaunchKernelGGL(k_net_conv<NET_MASKED>, grid, dim3(kT), 0, s, g, in, w, mask, out_bf, out_f);
    else
        hipLaunchKernelGGL(k_net_conv<NET_LINEAR>, grid, dim3(kT), 0, s, g, in, w, mask, out_bf, out_f);
}

void launch_net_wgrad(const Grid &g, const uint16_t *x, const uint16_t *d, float *part, hipStream_t s) {
    hipLaunchKernelGGL(k_net_wgrad, dim3(kNetWaves / (kT / 64)), dim3(kT), 0, s, g, x, d, part);
}

void launch_net_wgrad_reduce(const float *part, int cin, int cout, float *grad, hipStream_t s) {
    hipLaunchKernelGGL(k_net_wgrad_reduce, dim3(27 * 16), dim3(kT), 0, s, part, cin, cout, grad);
}

template <class T>
void launch_net_pack_r(const Grid &g, const T *r, double inv_s, uint16_t *x0, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_net_pack_r<T>, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, g, r, inv_s,
                       (const double *)nullptr, 0.0, x0);
}

void launch_net_pack_r_dev(const Grid &g, const double *r, const double *ss, double inv_cnt, uint16_t *x0,
                           hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_net_pack_r<double>, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, g, r, 0.0, ss,
                       inv_cnt, x0);
}

template <class T>
void launch_net_unpack(const Grid &g, const T *coef, const float *y, double scale, T *out, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_net_unpack<T>, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, g, coef, y, scale,
                       (const double *)nullptr, 0.0, out);
}

void launch_net_unpack_dev(const Grid &g, const double *coef, const float *y, double h2, const double *ss,
                           double inv_cnt, double *out, hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_net_unpack<double>, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, g, coef, y, h2, ss,
                       inv_cnt, out);
}

// The residual judge on the device: d[0] = |v - M z|^2, d[1] = |v - M (z +
// dz)|^2; z += dz when the correction lowers the residual (or the residual
// is already zero, where dz is zero as well); flag = whether it was kept.
// One workgroup per kThreads entries; every workgroup reads the same two
// numbers, workgroup 0 writes the flag.
__global__ void __launch_bounds__(kT)
k_net_accept(int64_t n, const double *__restrict__ d, const double *__restrict__ dz, double *__restrict__ z,
             int *__restrict__ flag) {
    const bool keep = d[1] < d[0] || d[0] == 0.0;
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t == 0) *flag = keep ? 1 : 0;
    if (keep && t < n) z[t] += dz[t];
}

void launch_net_accept(int64_t n, const double *d, const double *dz, double *z, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_net_accept, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, n, d, dz, z, flag);
}

void launch_net_loss(const Grid &g, const double *coef, const float *y, const double *e, double t_scale,
                     double inv_norm, uint16_t *dy, double *part, int nblocks, int pass, hipStream_t s) {
    hipLaunchKernelGGL(k_net_loss, dim3(nblocks), dim3(kT), 0, s, g, coef, y, e, t_scale, inv_norm, dy, part, pass);
}

void launch_net_dy_from_face(const Grid &g, const double *coef, const double *gv, double factor, uint16_t *dy,
                             hipStream_t s) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_net_dy_from_face, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, g, coef, gv, factor, dy);
}

void launch_net_pack_weights(const float *w32, uint16_t *wf, uint16_t *wb, hipStream_t s) {
    hipLaunchKernelGGL(k_net_pack_weights, dim3(3 * 27), dim3(kT), 0, s, w32, wf, wb);
}

void launch_net_adam(const float *g, float *w, float *m, float *v, int n, float lr, float b1, float b2,
                     float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_net_adam, dim3((unsigned)ceil_div(n, kT)), dim3(kT), 0, s, g, w, m, v, n, lr, b1, b2,
                       eps, c1, c2);
}

template void launch_net_pack_r<double>(const Grid &, const double *, double, uint16_t *, hipStream_t);
template void launch_net_pack_r<float>(const Grid &, const float *, double, uint16_t *, hipStream_t);
template void launch_net_unpack<double>(const Grid &, const double *, const float *, double, double *,
                                        hipStream_t);
template void launch_net_unpack<float>(const Grid &, const float *, const float *, double, float *, hipStream_t);

}  // namespace dm
