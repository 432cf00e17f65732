// Internal declarations of the learned correction: a 3-layer 3-D conv
// network on the cell grid (10 -> 16 -> 16 -> 3 channels, 3^3 kernels, no
// bias, ReLU between layers), bfloat16 storage, FP32 accumulation on MFMA.
//
// Activation layout: channels-last bfloat16, 16 channels per padded cell
// ([P][16], 32 B per cell), the padding layer held at zero, which is the
// zero extension outside the grid.  Weights for one layer on the device:
// [27 taps][16 out][16 in] bfloat16, zero-padded to 16 x 16.  Master
// weights: FP32, flat, layer by layer [27][in][out] (12,528 values).
#pragma once

#include <cstdint>

#include "dm_internal.h"

namespace dm {

constexpr int kNetIn[3] = {10, 16, 16};
constexpr int kNetOut[3] = {16, 16, 3};
constexpr int kNetWeights = 27 * (10 * 16 + 16 * 16 + 16 * 3);  // 12528
constexpr int kNetCh = 16;                                      // padded channels
constexpr int kNetWaves = 1024;                                 // weight-gradient partials

inline int64_t net_offset(int layer) {
    int64_t o = 0;
    for (int l = 0; l < layer; ++l) o += 27 * kNetIn[l] * kNetOut[l];
    return o;
}

// bfloat16 from float, round to nearest even (finite inputs)
__host__ __device__ inline uint16_t f2bf(float f) {
    uint32_t u;
#ifdef __HIP_DEVICE_COMPILE__
    u = __float_as_uint(f);
#else
    __builtin_memcpy(&u, &f, 4);
#endif
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

enum { NET_RELU = 0, NET_LINEAR = 1, NET_MASKED = 2 };

// conv layer: in [P][16] bf16, w [27][16][16] bf16 (out, in).
//   NET_RELU:   out_bf [P][16] = bf16(max(conv, 0))
//   NET_LINEAR: out_f  [P][4]  = conv (channels 0..3)
//   NET_MASKED: out_bf [P][16] = bf16(conv * (mask[P][16] > 0))
void launch_net_conv(int mode, const Grid &g, const uint16_t *in, const uint16_t *w,
                     const uint16_t *mask, uint16_t *out_bf, float *out_f, hipStream_t s);
// per-wave partial weight gradients: part[wave][27][16 in][16 out] of
// sum_p x[p + off][c] * d[p][o] over interior cells
void launch_net_wgrad(const Grid &g, const uint16_t *x, const uint16_t *d, float *part, hipStream_t s);
// grad[t][c][o] (c < cin, o < cout, flat layer layout) = sum over waves of part
void launch_net_wgrad_reduce(const float *part, int cin, int cout, float *grad, hipStream_t s);
// channels 0..2 of x0 = bf16(r_comp * inv_s) on interior cells
template <class T>
void launch_net_pack_r(const Grid &g, const T *r, double inv_s, uint16_t *x0, hipStream_t s);
// y [P][4] -> face vector out_comp = (a_comp > 0) ? y[c] * scale : 0 (with PMC ghost images)
template <class T>
void launch_net_unpack(const Grid &g, const T *coef, const float *y, double scale, T *out, hipStream_t s);
// the same with the residual scale s = sqrt(ss[0] * inv_cnt) read on the
// device (ss: a sum of squares): the input is r / s, the output y * s * h2
void launch_net_pack_r_dev(const Grid &g, const double *r, const double *ss, double inv_cnt, uint16_t *x0,
                           hipStream_t s);
void launch_net_unpack_dev(const Grid &g, const double *coef, const float *y, double h2, const double *ss,
                           double inv_cnt, double *out, hipStream_t s);
// z += dz where d[1] < d[0] (or d[0] == 0); *flag = 1 if kept, else 0
void launch_net_accept(int64_t n, const double *d, const double *dz, double *z, int *flag, hipStream_t s);
// loss of one pair: target t = e * t_scale on active faces (a > 0);
// dy [P][16] channels 0..2 = bf16(2 (y - t) / norm); partial sums of
// (y - t)^2 and t^2 per block into part[2 * nblocks] (FP64)
void launch_net_loss(const Grid &g, const double *coef, const float *y, const double *e,
                     double t_scale, double inv_norm, uint16_t *dy, double *part, int nblocks,
                     int pass, hipStream_t s);
// dy [P][16] channels 0..2 = bf16(g_c * factor) on active faces (a_c > 0), else 0
void launch_net_dy_from_face(const Grid &g, const double *coef, const double *gv, double factor, uint16_t *dy,
                             hipStream_t s);
// FP32 master -> bf16 forward weights of all layers; and the transposed,
// tap-flipped weights of layers 2 and 3 for the data gradient
void launch_net_pack_weights(const float *w32, uint16_t *wf, uint16_t *wb, hipStream_t s);
void launch_net_adam(const float *g, float *w, float *m, float *v, int n, float lr, float b1,
                     float b2, float eps, float c1, float c2, hipStream_t s);

}  // namespace dm
