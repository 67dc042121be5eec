// HIP kernels of the learned birth proposal (gfx950).
//
// Network 2 -> 128 -> 128 -> 128 -> 36 with ReLU, mapping a measurement to a
// 4-component diagonal Gaussian mixture over [x, vx, y, vy] (definition in
// include/pphd_mlp.h).  Layers 2-4 and their backward products run on the
// matrix cores (v_mfma_f32_16x16x32_bf16, gfx950's BF16 form with 32-deep
// contractions: BF16 operands, FP32 accumulation; the 16-deep form only for
// the last 16 of the output layer's 48 padded rows); layer 1, the mixture
// head and the loss run in FP32 on the vector units.
//
// One workgroup (4 wavefronts) takes a tile of 64 pairs and keeps every
// activation of the tile in LDS, so a training step reads each weight matrix
// from L2 a few times per tile and writes one gradient partial per tile; a
// second kernel sums the partials in a fixed order and takes the Adam step.
//
// MFMA operand layouts (lane l, r = l % 16, q = l / 16):
//   16x16x32: A[r][8q + i],  B[8q + i][r] (i = 0..7),  C[4q + e][r] (e = 0..3);
//   16x16x16: A[r][4q + e],  B[4q + e][r],  C[4q + e][r].
// Matrix products are arranged so that every operand read from a row-major
// array is 8 (or 4) consecutive BF16 values (one 16- or 8-byte load), except
// the weight gradients, whose contraction runs over the pairs and gathers 8
// rows.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_internal.h"
#include "philox_dev.h"

namespace pphd {
namespace mlp {

constexpr int H = 128;    // hidden width
constexpr int NO = 36;    // outputs: 4 components x (logit, 4 means, 4 log-stds)
constexpr int NOP = 48;   // outputs padded to whole 16-row blocks
constexpr int TS = 64;    // pairs per workgroup tile
constexpr int HP = 136;   // LDS row pitch of an activation tile (BF16 values)
constexpr int NTHR = 256;
// offsets in the flat parameter vector
constexpr int P_W1 = 0, P_B1 = P_W1 + 2 * H, P_W2 = P_B1 + H, P_B2 = P_W2 + H * H, P_W3 = P_B2 + H,
              P_B3 = P_W3 + H * H, P_W4 = P_B3 + H, P_B4 = P_W4 + NO * H, P_ALL = P_B4 + NO;
static_assert(P_ALL == 38052, "parameter count");
constexpr float LOGSTD_MIN = -12.0f, LOGSTD_MAX = 6.0f;
constexpr double LOG_2PI = 1.8378770664093454836;
constexpr int TAB = MIX_TAB;  // doubles per mixture-table entry

enum : uint32_t { RNG_PAIRS = 6, RNG_MLP_INIT = 7 };

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Features and normalised state: f = ((s + r (cos, sin) th) - c) / h,
// xi = ((x - c_x)/h_x, vx/sv, (y - c_y)/h_y, vy/sv).
struct Norm {
    double sx, sy, cx, cy, hx, hy, sv;
    double log_scale_sum;  // log h_x + log sv + log h_y + log sv
    // simulation of training pairs
    double reg0, reg1, reg2, reg3, sigma_r, sigma_th;
    uint32_t key0, key1;
};

// Network weights as the kernels read them.  theta: FP32 master vector (layer
// 1 and every bias are read from it); Wt*: BF16 row = output unit
// ([out][in]); Wi*: BF16 row = input unit ([in][out]).  Wt4 has NOP rows and
// Wi4 rows of NOP values, the padding zero.
struct Net {
    const float* theta;
    const uint16_t *Wt2, *Wi2, *Wt3, *Wi3, *Wt4, *Wi4;
};

__device__ __forceinline__ uint32_t bf16_bits(float x)  // round to nearest even
{
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint64_t pack4(float a, float b, float c, float d)
{
    const uint32_t lo = bf16_bits(a) | (bf16_bits(b) << 16);
    const uint32_t hi = bf16_bits(c) | (bf16_bits(d) << 16);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ float bf16_value(uint32_t bits) { return __builtin_bit_cast(float, bits << 16); }
__device__ __forceinline__ bf4 ld8(const uint16_t* p) { return __builtin_bit_cast(bf4, *(const uint64_t*)p); }
__device__ __forceinline__ bf8 ld16(const uint16_t* p) { return __builtin_bit_cast(bf8, *(const u4v*)p); }
__device__ __forceinline__ bf8 gather8(const uint16_t* p, int stride)
{
    u4v v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (uint32_t)p[2 * i * stride] | ((uint32_t)p[(2 * i + 1) * stride] << 16);
    return __builtin_bit_cast(bf8, v);
}
__device__ __forceinline__ f4 mma(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f4 mma32(bf8 a, bf8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
// 1 where a stored ReLU output is positive (its BF16 magnitude bits nonzero)
__device__ __forceinline__ float relu_mask(uint64_t v, int e) { return ((v >> (16 * e)) & 0x7FFFu) ? 1.0f : 0.0f; }

// ---- layers ----------------------------------------------------------------

// Layer 1 (2 -> 128, FP32) for the tile: h1[s][j] = relu(W1[j] . f[s] + b1[j]).
__device__ __forceinline__ void layer1(const float* __restrict__ theta, const float (*f)[2], uint16_t* h1)
{
    for (int idx = threadIdx.x; idx < TS * H; idx += NTHR) {
        const int s = idx / H, j = idx % H;
        const float v = fmaf(theta[P_W1 + 2 * j], f[s][0], fmaf(theta[P_W1 + 2 * j + 1], f[s][1], theta[P_B1 + j]));
        h1[s * HP + j] = (uint16_t)bf16_bits(fmaxf(v, 0.0f));
    }
}

// Hidden layer (128 -> 128): Out[s][j] = relu(sum_k W[j][k] In[s][k] + b[j]),
// computed as Out^T = W In^T so that both operands and the result rows are
// contiguous.  Wavefront w takes output rows [32 w, 32 w + 32).
__device__ __forceinline__ void hidden_fwd(const uint16_t* __restrict__ Wt, const float* __restrict__ b,
                                           const uint16_t* In, uint16_t* Out, int w, int lane)
{
    const int r = lane & 15, q = lane >> 4;
    f4 acc[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) acc[t][sb] = f4{ 0, 0, 0, 0 };
#pragma unroll 2
    for (int kb = 0; kb < H / 32; ++kb) {
        const bf8 a0 = ld16(Wt + ((2 * w) * 16 + r) * H + kb * 32 + 8 * q);
        const bf8 a1 = ld16(Wt + ((2 * w + 1) * 16 + r) * H + kb * 32 + 8 * q);
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            const bf8 bb = ld16(In + (sb * 16 + r) * HP + kb * 32 + 8 * q);
            acc[0][sb] = mma32(a0, bb, acc[0][sb]);
            acc[1][sb] = mma32(a1, bb, acc[1][sb]);
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int j0 = (2 * w + t) * 16 + 4 * q;
        const float b0 = b[j0], b1 = b[j0 + 1], b2 = b[j0 + 2], b3 = b[j0 + 3];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            const int s = sb * 16 + r;
            *(uint64_t*)(Out + s * HP + j0) =
                pack4(fmaxf(acc[t][sb][0] + b0, 0.0f), fmaxf(acc[t][sb][1] + b1, 0.0f),
                      fmaxf(acc[t][sb][2] + b2, 0.0f), fmaxf(acc[t][sb][3] + b3, 0.0f));
        }
    }
}

// Output layer (128 -> 36, padded to 48): o[s][j] in FP32.  Wavefronts 0-2
// take one 16-row block each.
__device__ __forceinline__ void output_fwd(const uint16_t* __restrict__ Wt4, const float* __restrict__ b4,
                                           const uint16_t* In, float* o, int w, int lane)
{
    if (w >= NOP / 16) return;
    const int r = lane & 15, q = lane >> 4;
    f4 acc[4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) acc[sb] = f4{ 0, 0, 0, 0 };
#pragma unroll 2
    for (int kb = 0; kb < H / 32; ++kb) {
        const bf8 a = ld16(Wt4 + (w * 16 + r) * H + kb * 32 + 8 * q);
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) acc[sb] = mma32(a, ld16(In + (sb * 16 + r) * HP + kb * 32 + 8 * q), acc[sb]);
    }
    const int j0 = w * 16 + 4 * q;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
        const int s = sb * 16 + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) o[s * NOP + j0 + e] = acc[sb][e] + (j0 + e < NO ? b4[j0 + e] : 0.0f);
    }
}

// Backward through a layer's weights: G_out[s][k] = mask(Hk[s][k]) *
// sum_j G_in[s][j] W[j][k], with Wi = W^T stored row-major ([k][j], row
// length NJ) and the contraction over j in 32-deep steps (a 16-deep one for
// the rest when NJ is an odd multiple of 16).
template <int NJ>
__device__ __forceinline__ void back_data(const uint16_t* __restrict__ Wi, const uint16_t* Gin, const uint16_t* Hk,
                                          uint16_t* Gout, int w, int lane)
{
    const int r = lane & 15, q = lane >> 4;
    f4 acc[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) acc[t][sb] = f4{ 0, 0, 0, 0 };
    static_assert(NJ % 16 == 0, "whole 16-deep blocks");
#pragma unroll 2
    for (int jb = 0; jb < NJ / 32; ++jb) {
        const bf8 a0 = ld16(Wi + ((2 * w) * 16 + r) * NJ + jb * 32 + 8 * q);
        const bf8 a1 = ld16(Wi + ((2 * w + 1) * 16 + r) * NJ + jb * 32 + 8 * q);
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            const bf8 bb = ld16(Gin + (sb * 16 + r) * HP + jb * 32 + 8 * q);
            acc[0][sb] = mma32(a0, bb, acc[0][sb]);
            acc[1][sb] = mma32(a1, bb, acc[1][sb]);
        }
    }
    if constexpr (NJ % 32 == 16) {
        constexpr int j0 = NJ - 16;
        const bf4 a0 = ld8(Wi + ((2 * w) * 16 + r) * NJ + j0 + 4 * q);
        const bf4 a1 = ld8(Wi + ((2 * w + 1) * 16 + r) * NJ + j0 + 4 * q);
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            const bf4 bb = ld8(Gin + (sb * 16 + r) * HP + j0 + 4 * q);
            acc[0][sb] = mma(a0, bb, acc[0][sb]);
            acc[1][sb] = mma(a1, bb, acc[1][sb]);
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int k0 = (2 * w + t) * 16 + 4 * q;
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            const int s = sb * 16 + r;
            const uint64_t hv = *(const uint64_t*)(Hk + s * HP + k0);
            *(uint64_t*)(Gout + s * HP + k0) =
                pack4(acc[t][sb][0] * relu_mask(hv, 0), acc[t][sb][1] * relu_mask(hv, 1),
                      acc[t][sb][2] * relu_mask(hv, 2), acc[t][sb][3] * relu_mask(hv, 3));
        }
    }
}

// Weight gradient of one tile: dW[j][k] = sum_s G[s][j] Hk[s][k] for output
// rows [16 jb0, 16 (jb0 + NJB)) and input columns [16 kb0, 16 (kb0 + NKB)),
// written to the tile's partial (row length H) for rows j < jmax.
template <int NJB, int NKB>
__device__ __forceinline__ void weight_grad(const uint16_t* G, int jb0, const uint16_t* Hk, int kb0, float* part,
                                            int jmax, int lane)
{
    const int r = lane & 15, q = lane >> 4;
    f4 acc[NJB][NKB];
#pragma unroll
    for (int t = 0; t < NJB; ++t)
#pragma unroll
        for (int u = 0; u < NKB; ++u) acc[t][u] = f4{ 0, 0, 0, 0 };
    static_assert(TS % 32 == 0, "whole 32-deep blocks of pairs");
#pragma unroll
    for (int ss = 0; ss < TS / 32; ++ss) {
        const int s0 = ss * 32 + 8 * q;
        bf8 a[NJB], b[NKB];
#pragma unroll
        for (int t = 0; t < NJB; ++t) a[t] = gather8(G + s0 * HP + (jb0 + t) * 16 + r, HP);
#pragma unroll
        for (int u = 0; u < NKB; ++u) b[u] = gather8(Hk + s0 * HP + (kb0 + u) * 16 + r, HP);
#pragma unroll
        for (int t = 0; t < NJB; ++t)
#pragma unroll
            for (int u = 0; u < NKB; ++u) acc[t][u] = mma32(a[t], b[u], acc[t][u]);
    }
#pragma unroll
    for (int t = 0; t < NJB; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = (jb0 + t) * 16 + 4 * q + e;
            if (j < jmax) {
#pragma unroll
                for (int u = 0; u < NKB; ++u) part[j * H + (kb0 + u) * 16 + r] = acc[t][u][e];
            }
        }
}

// bias gradient: db[j] = sum over the tile of G[s][j] (threads j < n)
__device__ __forceinline__ void bias_grad(const uint16_t* G, int n, float* part)
{
    const int j = threadIdx.x;
    if (j < n) {
        float acc = 0.0f;
        for (int s = 0; s < TS; ++s) acc += bf16_value(G[s * HP + j]);
        part[j] = acc;
    }
}

// ---- mixture head ---------------------------------------------------------

// Loss of one pair and d loss / d o (FP32).  o: the pair's 36 outputs, replaced
// by the derivative; f: features; xi: normalised state.  Returns the loss.
__device__ __forceinline__ float loss_head(float* o, const float* f, const float* xi)
{
    float logit[4], lmax = -INFINITY;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        logit[c] = o[9 * c];
        lmax = fmaxf(lmax, logit[c]);
    }
    float z = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) z += expf(logit[c] - lmax);
    const float lse_pi = lmax + logf(z);
    float a[4], e[4][4], isg[4][4], inside[4][4];
    float amax = -INFINITY;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float mean[4] = { f[0] + o[9 * c + 1], o[9 * c + 2], f[1] + o[9 * c + 3], o[9 * c + 4] };
        float ln = 0.0f;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const float sr = o[9 * c + 5 + d];
            const float s = fminf(fmaxf(sr, LOGSTD_MIN), LOGSTD_MAX);
            inside[c][d] = (sr > LOGSTD_MIN && sr < LOGSTD_MAX) ? 1.0f : 0.0f;
            isg[c][d] = expf(-s);
            e[c][d] = (xi[d] - mean[d]) * isg[c][d];
            ln += -0.5f * e[c][d] * e[c][d] - s;
        }
        a[c] = (logit[c] - lse_pi) + ln - 2.0f * (float)LOG_2PI;
        amax = fmaxf(amax, a[c]);
    }
    float za = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) za += expf(a[c] - amax);
    const float lse = amax + logf(za);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float resp = expf(a[c] - lse);
        const float pi = expf(logit[c] - lse_pi);
        o[9 * c] = pi - resp;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            o[9 * c + 1 + d] = -resp * e[c][d] * isg[c][d];
            o[9 * c + 5 + d] = -resp * (e[c][d] * e[c][d] - 1.0f) * inside[c][d];
        }
    }
    return -lse;
}

// Mixture-table entries of one measurement (double): o its 36 outputs, f its
// features (double).  tab: 4 entries of TAB doubles.
__device__ __forceinline__ void mixture_entries(const Norm& n, const float* o, const double* f, double* tab)
{
    double lmax = -INFINITY;
#pragma unroll
    for (int c = 0; c < 4; ++c) lmax = fmax(lmax, (double)o[9 * c]);
    double z = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) z += exp((double)o[9 * c] - lmax);
    const double lse = lmax + log(z);
    const double off[4] = { n.cx, 0.0, n.cy, 0.0 }, sc[4] = { n.hx, n.sv, n.hy, n.sv };
    double cum = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double* t = tab + c * TAB;
        const double logpi = (double)o[9 * c] - lse;
        cum += exp(logpi);
        const double mean[4] = { f[0] + (double)o[9 * c + 1], (double)o[9 * c + 2], f[1] + (double)o[9 * c + 3],
                                 (double)o[9 * c + 4] };
        double ssum = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double s = fmin(fmax((double)o[9 * c + 5 + d], (double)LOGSTD_MIN), (double)LOGSTD_MAX);
            ssum += s;
            const double sig = sc[d] * exp(s);
            t[4 + d] = off[d] + sc[d] * mean[d];
            t[8 + d] = sig;
            t[12 + d] = 1.0 / sig;
        }
        t[0] = logpi;
        t[1] = cum;
        t[2] = logpi - ssum - n.log_scale_sum - 2.0 * LOG_2PI;
        t[3] = 0.0;
    }
}

__device__ __forceinline__ void features_of(const Norm& n, double r, double th, double* f)
{
    double sn, cs;
    sincos(th, &sn, &cs);
    f[0] = (n.sx + r * cs - n.cx) / n.hx;
    f[1] = (n.sy + r * sn - n.cy) / n.hy;
}

// ---- kernels ---------------------------------------------------------------

// (activation rows are read 16 bytes at a time: 16-byte aligned, a row
// pitch of 272 bytes)
struct TrainLds {
    alignas(16) uint16_t h[3][TS * HP];  // h1, h2, h3 of the tile, [pair][unit]
    alignas(16) uint16_t g[2][TS * HP];  // back-propagated terms, [pair][unit]
    float o[TS * NOP];       // outputs, then d loss / d o
    float f[TS][2];
    float xi[TS][4];
    float loss[TS];
};

// One training tile: forward, loss, backward.  Pairs [base + 64 b, +64) of
// (z, x) (indices taken modulo D), the first n_valid - 64 b of them real.
// part: per-tile gradient sums (P_ALL floats per tile); ploss: per-tile loss sums.
__global__ __launch_bounds__(NTHR) void k_mlp_train(Net net, Norm nrm, const float* __restrict__ z,
                                                    const float* __restrict__ x, int64_t base, int64_t D,
                                                    int n_valid, float* __restrict__ part,
                                                    double* __restrict__ ploss)
{
    __shared__ TrainLds L;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int tile = blockIdx.x;
    const int valid = min(TS, n_valid - tile * TS);
    float* P = part + (size_t)tile * P_ALL;
    if (threadIdx.x < TS) {
        const int s = threadIdx.x;
        float f0 = 0.0f, f1 = 0.0f, xs[4] = { 0, 0, 0, 0 };
        if (s < valid) {
            const int64_t i = (base + (int64_t)tile * TS + s) % D;
            const float r = z[2 * i], th = z[2 * i + 1];
            float sn, cs;
            sincosf(th, &sn, &cs);
            f0 = ((float)nrm.sx + r * cs - (float)nrm.cx) / (float)nrm.hx;
            f1 = ((float)nrm.sy + r * sn - (float)nrm.cy) / (float)nrm.hy;
            xs[0] = (x[4 * i] - (float)nrm.cx) / (float)nrm.hx;
            xs[1] = x[4 * i + 1] / (float)nrm.sv;
            xs[2] = (x[4 * i + 2] - (float)nrm.cy) / (float)nrm.hy;
            xs[3] = x[4 * i + 3] / (float)nrm.sv;
        }
        L.f[s][0] = f0;
        L.f[s][1] = f1;
#pragma unroll
        for (int d = 0; d < 4; ++d) L.xi[s][d] = xs[d];
    }
    __syncthreads();
    layer1(net.theta, L.f, L.h[0]);
    __syncthreads();
    hidden_fwd(net.Wt2, net.theta + P_B2, L.h[0], L.h[1], w, lane);
    __syncthreads();
    hidden_fwd(net.Wt3, net.theta + P_B3, L.h[1], L.h[2], w, lane);
    __syncthreads();
    output_fwd(net.Wt4, net.theta + P_B4, L.h[2], L.o, w, lane);
    __syncthreads();
    if (threadIdx.x < TS) {
        const int s = threadIdx.x;
        float* os = L.o + s * NOP;
        float l = 0.0f;
        if (s < valid) {
            l = loss_head(os, L.f[s], L.xi[s]);
        } else {
            for (int j = 0; j < NO; ++j) os[j] = 0.0f;
        }
        for (int j = NO; j < NOP; ++j) os[j] = 0.0f;
        L.loss[s] = l;
        for (int j = 0; j < NOP; j += 4)
            *(uint64_t*)(L.g[0] + s * HP + j) = pack4(os[j], os[j + 1], os[j + 2], os[j + 3]);
    }
    __syncthreads();
    // output layer: dW4, db4 and the term of h3
    weight_grad<3, 2>(L.g[0], 0, L.h[2], 2 * w, P + P_W4, NO, lane);
    if (threadIdx.x < NO) {
        float acc = 0.0f;
        for (int s = 0; s < TS; ++s) acc += L.o[s * NOP + threadIdx.x];
        P[P_B4 + threadIdx.x] = acc;
    }
    back_data<NOP>(net.Wi4, L.g[0], L.h[2], L.g[1], w, lane);
    __syncthreads();
    weight_grad<2, 8>(L.g[1], 2 * w, L.h[1], 0, P + P_W3, H, lane);
    bias_grad(L.g[1], H, P + P_B3);
    back_data<H>(net.Wi3, L.g[1], L.h[1], L.g[0], w, lane);
    __syncthreads();
    weight_grad<2, 8>(L.g[0], 2 * w, L.h[0], 0, P + P_W2, H, lane);
    bias_grad(L.g[0], H, P + P_B2);
    back_data<H>(net.Wi2, L.g[0], L.h[0], L.g[1], w, lane);
    __syncthreads();
    if (threadIdx.x < H) {
        const int j = threadIdx.x;
        float a0 = 0.0f, a1 = 0.0f, ab = 0.0f;
        for (int s = 0; s < TS; ++s) {
            const float gv = bf16_value(L.g[1][s * HP + j]);
            a0 = fmaf(gv, L.f[s][0], a0);
            a1 = fmaf(gv, L.f[s][1], a1);
            ab += gv;
        }
        P[P_W1 + 2 * j] = a0;
        P[P_W1 + 2 * j + 1] = a1;
        P[P_B1 + j] = ab;
    }
    if (threadIdx.x == H) {
        double acc = 0.0;
        for (int s = 0; s < TS; ++s) acc += (double)L.loss[s];
        ploss[tile] = acc;
    }
}

struct InferLds {
    alignas(16) uint16_t h[2][TS * HP];
    float o[TS * NOP];
    float f[TS][2];
};

// Forward pass of a tile of measurements (double[M][2]); writes the outputs
// (out, float[M][36], nullable) and/or the mixture table (tab, nullable).
__global__ __launch_bounds__(NTHR) void k_mlp_infer(Net net, Norm nrm, const double* __restrict__ zin, int M,
                                                    float* __restrict__ out, double* __restrict__ tab)
{
    __shared__ InferLds L;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int base = blockIdx.x * TS;
    if (threadIdx.x < TS) {
        const int s = threadIdx.x;
        double f[2] = { 0.0, 0.0 };
        if (base + s < M) features_of(nrm, zin[2 * (base + s)], zin[2 * (base + s) + 1], f);
        L.f[s][0] = (float)f[0];
        L.f[s][1] = (float)f[1];
    }
    __syncthreads();
    layer1(net.theta, L.f, L.h[0]);
    __syncthreads();
    hidden_fwd(net.Wt2, net.theta + P_B2, L.h[0], L.h[1], w, lane);
    __syncthreads();
    hidden_fwd(net.Wt3, net.theta + P_B3, L.h[1], L.h[0], w, lane);
    __syncthreads();
    output_fwd(net.Wt4, net.theta + P_B4, L.h[0], L.o, w, lane);
    __syncthreads();
    for (int idx = threadIdx.x; idx < TS * NO; idx += NTHR) {
        const int s = idx / NO, j = idx % NO;
        if (out && base + s < M) out[(size_t)(base + s) * NO + j] = L.o[s * NOP + j];
    }
    if (tab && threadIdx.x < TS && base + (int)threadIdx.x < M) {
        const int p = base + threadIdx.x;
        double f[2];
        features_of(nrm, zin[2 * p], zin[2 * p + 1], f);
        mixture_entries(nrm, L.o + threadIdx.x * NOP, f, tab + (size_t)p * 4 * TAB);
    }
}

// Mixture table from given outputs (float[M][36]).  One thread per measurement.
__global__ __launch_bounds__(NTHR) void k_mix_head(Norm nrm, const double* __restrict__ zin,
                                                   const float* __restrict__ raw, int M, double* __restrict__ tab)
{
    const int p = blockIdx.x * NTHR + threadIdx.x;
    if (p >= M) return;
    float o[NO];
    for (int j = 0; j < NO; ++j) o[j] = raw[(size_t)p * NO + j];
    double f[2];
    features_of(nrm, zin[2 * p], zin[2 * p + 1], f);
    mixture_entries(nrm, o, f, tab + (size_t)p * 4 * TAB);
}

// Sum of the tile partials (fixed order) and, by mode:
//   0: grad = mean gradient;  1: Adam step, then the BF16 copies;  2: BF16 copies only.
// loss_out[0] (nullable) = mean loss.
struct Adam {
    float lr, beta1, beta2, eps, bc1, bc2;  // bc = 1 / (1 - beta^t)
};
// Sum of the tiles' gradient partials, Adam step and the BF16 copies.  A
// workgroup takes RP consecutive parameters; its threads (chunk c, parameter
// u) add the tiles of chunk c (RC chunks of consecutive tiles) in tile
// order, and the RC chunk sums are added in chunk order, so the order is
// fixed; many workgroups keep enough reads in flight.  grid (ceil(P_ALL/RP)).
constexpr int RP = 32, RC = NTHR / RP;
__global__ __launch_bounds__(NTHR) void k_mlp_reduce(int mode, const float* __restrict__ part,
                                                     const double* __restrict__ ploss, int ntiles, double inv_n,
                                                     float* theta, float* am, float* av, float* grad, Adam ad,
                                                     uint16_t* Wt2, uint16_t* Wi2, uint16_t* Wt3, uint16_t* Wi3,
                                                     uint16_t* Wt4, uint16_t* Wi4, float* loss_out)
{
    __shared__ double s_acc[RC][RP];
    const int u = threadIdx.x % RP, c = threadIdx.x / RP;
    const int p = blockIdx.x * RP + u;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss_out) {
        double acc = 0.0;
        for (int t = 0; t < ntiles; ++t) acc += ploss[t];
        *loss_out = (float)(acc * inv_n);
    }
    const int per = (ntiles + RC - 1) / RC, t0 = c * per, t1 = t0 + per < ntiles ? t0 + per : ntiles;
    if (mode != 2) {
        double acc = 0.0;
        if (p < P_ALL) {
            for (int ta = t0; ta < t1; ta += 8) {
                float v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = ta + k < t1 ? part[(size_t)(ta + k) * P_ALL + p] : 0.0f;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (ta + k < t1) acc += (double)v[k];
            }
        }
        s_acc[c][u] = acc;
    }
    __syncthreads();
    if (c != 0 || p >= P_ALL) return;
    float th = theta[p];
    if (mode != 2) {
        double acc = 0.0;
        for (int k = 0; k < RC; ++k) acc += s_acc[k][u];
        const float g = (float)(acc * inv_n);
        if (mode == 0) {
            grad[p] = g;
            return;
        }
        const float m = ad.beta1 * am[p] + (1.0f - ad.beta1) * g;
        const float v = ad.beta2 * av[p] + (1.0f - ad.beta2) * g * g;
        am[p] = m;
        av[p] = v;
        th -= ad.lr * (m * ad.bc1) / (sqrtf(v * ad.bc2) + ad.eps);
        theta[p] = th;
    }
    const uint16_t b = (uint16_t)bf16_bits(th);
    if (p >= P_W2 && p < P_B2) {
        const int i = p - P_W2, j = i / H, k = i % H;
        Wt2[j * H + k] = b;
        Wi2[k * H + j] = b;
    } else if (p >= P_W3 && p < P_B3) {
        const int i = p - P_W3, j = i / H, k = i % H;
        Wt3[j * H + k] = b;
        Wi3[k * H + j] = b;
    } else if (p >= P_W4 && p < P_B4) {
        const int i = p - P_W4, j = i / H, k = i % H;
        Wt4[j * H + k] = b;
        Wi4[k * NOP + j] = b;
    }
}

// Uniform He initialisation (see pphd_mlp_init_params).
__global__ __launch_bounds__(NTHR) void k_mlp_init(float* theta, float* am, float* av, uint32_t key0, uint32_t key1,
                                                   uint32_t init_id)
{
    const int p = blockIdx.x * NTHR + threadIdx.x;
    if (p >= P_ALL) return;
    const Block4 r = rng_block(key0, key1, (uint32_t)p, 0, RNG_MLP_INIT, 0, init_id);
    const float u = (float)(2.0 * uniform53(r.a, r.b) - 1.0);
    float v = 0.0f;
    if (p < P_B1) v = u * sqrtf(6.0f / 2.0f);
    else if ((p >= P_W2 && p < P_B2) || (p >= P_W3 && p < P_B3)) v = u * sqrtf(6.0f / (float)H);
    else if (p >= P_W4 && p < P_B4) v = 0.1f * u * sqrtf(6.0f / (float)H);
    else if (p >= P_B4) {
        const int j = (p - P_B4) % 9;
        v = (j == 5 || j == 7) ? logf(0.05f) : 0.0f;
    }
    theta[p] = v;
    am[p] = 0.0f;
    av[p] = 0.0f;
}

// Simulated training pairs: x from the birth density, z from the sensor model.
__global__ __launch_bounds__(NTHR) void k_mlp_simulate(Norm n, double sigma_v, uint32_t run, float* z, float* x,
                                                       int64_t D)
{
    const int64_t i = (int64_t)blockIdx.x * NTHR + threadIdx.x;
    if (i >= D) return;
    const Block4 a = rng_block(n.key0, n.key1, (uint32_t)i, 0, RNG_PAIRS, 0, run);
    const Block4 v = rng_block(n.key0, n.key1, (uint32_t)i, 0, RNG_PAIRS, 1, run);
    const Block4 e = rng_block(n.key0, n.key1, (uint32_t)i, 0, RNG_PAIRS, 2, run);
    const double px = n.reg0 + uniform53(a.a, a.b) * (n.reg1 - n.reg0);
    const double py = n.reg2 + uniform53(a.c, a.d) * (n.reg3 - n.reg2);
    double n1, n2, e1, e2;
    normal_pair(uniform53(v.a, v.b), uniform53(v.c, v.d), n1, n2);
    normal_pair(uniform53(e.a, e.b), uniform53(e.c, e.d), e1, e2);
    const double dx = px - n.sx, dy = py - n.sy;
    const double two_pi = 2.0 * 3.14159265358979323846;
    double th = atan2(dy, dx) + n.sigma_th * e2;
    th -= two_pi * floor((th + 3.14159265358979323846) / two_pi);
    x[4 * i] = (float)px;
    x[4 * i + 1] = (float)(sigma_v * n1);
    x[4 * i + 2] = (float)py;
    x[4 * i + 3] = (float)(sigma_v * n2);
    z[2 * i] = (float)(sqrt(dx * dx + dy * dy) + n.sigma_r * e1);
    z[2 * i + 1] = (float)th;
}

}  // namespace mlp
}  // namespace pphd
