// HIP kernels of libpphd for gfx950 (CDNA4, 64-lane wavefronts).
//
// Particle layout: structure of arrays in device memory.  Component d of slot s
// of group j lives at X[d][j*cap + s]; the weight at W[j*cap + s].  Group j
// occupies slots [0, n_j).  Every kernel is templated on the storage type T
// (double or float); per-particle geometry and all cross-thread totals are kept
// in double, the per-pair exponential runs in T.
//
// Likelihood in scaled units (section 4 sensor model): with
//   c_r = sqrt(log2(e)/2)/sigma_r,  c_t = sqrt(log2(e)/2)/sigma_theta,
//   q(z, x) = ((r_z - rho(x)) c_r)^2 + (wrap(theta_z - phi(x)) c_t)^2,
// the Gaussian factor of g(z|x) is 2^-q, and g = 2^-q / (2 pi sigma_r sigma_theta).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox_dev.h"

namespace pphd {

struct DevModel {
    double T, sigma_a, sx, sy;
    double pS, pD, nu, kappa;
    double birth_mass, reg0, reg1, reg2, reg3, sigma_v, init_mass, Rj, xfrac;
    double cr, ct, period, inv_period, wscale;  // scaled likelihood, see above
    int K, J, cap, M0;
    uint32_t key0, key1, run, pad;
};

template <typename T>
struct SoA {
    T* x[4];
    T* w;
};

__device__ __forceinline__ int births_in(const DevModel& m, int j)
{
    return m.J / m.K + (j < m.J % m.K ? 1 : 0);
}

// ---------------------------------------------------------------------------
// wavefront reductions (64 lanes)
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V wave_sum(V v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename V>
__device__ __forceinline__ V wave_max(V v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        V u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double fast_exp2(double x) { return exp2(x); }

// ---------------------------------------------------------------------------
// draws from the normalised birth density: position uniform over the region,
// velocity N(0, sigma_v^2 I)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void draw_birth(const DevModel& m, uint32_t slot, uint32_t step, uint32_t purpose,
                                           double s[4])
{
    Block4 a = rng_block(m.key0, m.key1, slot, step, purpose, 0, m.run);
    Block4 b = rng_block(m.key0, m.key1, slot, step, purpose, 1, m.run);
    double ux = uniform53(a.a, a.b), uy = uniform53(a.c, a.d);
    double n1, n2;
    normal_pair(uniform53(b.a, b.b), uniform53(b.c, b.d), n1, n2);
    s[0] = m.reg0 + ux * (m.reg1 - m.reg0);
    s[1] = m.sigma_v * n1;
    s[2] = m.reg2 + uy * (m.reg3 - m.reg2);
    s[3] = m.sigma_v * n2;
}

// ---------------------------------------------------------------------------
// t = 0: round(R_j) particles per group from the birth density.
// grid (ceil(M0/256), K)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_init(DevModel m, SoA<T> st, int* __restrict__ nsurv)
{
    const int j = blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) nsurv[j] = m.M0;
    if (s >= m.M0) return;
    const size_t g = (size_t)j * m.cap + s;
    double v[4];
    draw_birth(m, (uint32_t)g, 0u, RNG_INIT, v);
#pragma unroll
    for (int d = 0; d < 4; ++d) st.x[d][g] = (T)v[d];
    st.w[g] = (T)(m.init_mass / (double)m.M0);
}

// ---------------------------------------------------------------------------
// Step 1 (Eqs 5, 6): survivors through the CV model, births appended.
// grid (ceil(cap/256), K)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_predict(DevModel m, SoA<T> st, const int* __restrict__ nsurv,
                                                 int* __restrict__ ncur, uint32_t step)
{
    const int j = blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int ns = nsurv[j];
    const int Jj = births_in(m, j);
    // the host guarantees ns + J_j <= cap; the clamp keeps every store inside the group
    const int total = ns + Jj < m.cap ? ns + Jj : m.cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) ncur[j] = total;
    if (s >= total) return;
    const size_t g = (size_t)j * m.cap + s;
    if (s < ns) {
        Block4 r = rng_block(m.key0, m.key1, (uint32_t)g, step, RNG_PREDICT, 0, m.run);
        double n1, n2;
        normal_pair(uniform53(r.a, r.b), uniform53(r.c, r.d), n1, n2);
        const double ax = m.sigma_a * n1, ay = m.sigma_a * n2;
        const double half_t2 = m.T * m.T / 2;
        double x = st.x[0][g], vx = st.x[1][g], y = st.x[2][g], vy = st.x[3][g];
        st.x[0][g] = (T)(x + m.T * vx + half_t2 * ax);
        st.x[1][g] = (T)(vx + m.T * ax);
        st.x[2][g] = (T)(y + m.T * vy + half_t2 * ay);
        st.x[3][g] = (T)(vy + m.T * ay);
        st.w[g] = (T)(m.pS * (double)st.w[g]);
    } else {
        double v[4];
        draw_birth(m, (uint32_t)g, step, RNG_BIRTH, v);
#pragma unroll
        for (int d = 0; d < 4; ++d) st.x[d][g] = (T)v[d];
        st.w[g] = (T)(m.birth_mass / (double)Jj);
    }
}

// per-particle geometry in scaled units
__device__ __forceinline__ void geometry(const DevModel& m, double x, double y, double& rho, double& phi)
{
    const double dx = x - m.sx, dy = y - m.sy;
    rho = sqrt(dx * dx + dy * dy) * m.cr;
    phi = atan2(dy, dx) * m.ct;
}

// scaled squared residual q(z, x) + c
__device__ __forceinline__ double sq_resid(const DevModel& m, double zr, double zt, double rho, double phi,
                                           double c)
{
    const double dr = zr - rho;
    double dt = zt - phi;
    dt = fma(-rint(dt * m.inv_period), m.period, dt);
    return fma(dr, dr, fma(dt, dt, c));
}

// ---------------------------------------------------------------------------
// Step 2, first pass (Eq 11): C_j(z) for every group and measurement.
// Each wavefront owns WT = 64*PT consecutive slots of one group (lane l takes
// slots base + 64 i + l) and, per measurement, returns the scaled partial sum
//   s = sum_i 2^(-q_i + log2(wscale w_i) - h),  h = ceil(max_i of the exponent),
// so that C = 2^h s exactly represents p_D sum g w with no underflow of the
// dominant term (log-sum-exp scaling with an integer shift).
// Partials: ps/ph[(j*wtiles + wave_tile)*Mmax + p]; pw[j*wtiles + wave_tile]
// holds the wave's sum of w.  grid (ceil(wtiles/4), K), 256 threads.
// ---------------------------------------------------------------------------
template <typename T, int PT>
__global__ __launch_bounds__(256) void k_cz(DevModel m, SoA<T> st, const int* __restrict__ ncur,
                                            const double* __restrict__ Z, int M, int Mmax, int wtiles,
                                            double* __restrict__ ps, int* __restrict__ ph,
                                            double* __restrict__ pw)
{
    constexpr int WT = 64 * PT;
    const int j = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wtile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int n = ncur[j];
    const int base = wtile * WT;
    if (wtile >= wtiles || base >= n) return;
    const size_t gb = (size_t)j * m.cap;
    double rho[PT], phi[PT], nlw[PT];
    double wsum = 0.0;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        rho[i] = 0.0;
        phi[i] = 0.0;
        nlw[i] = __builtin_inf();
        if (s < n) {
            const double w = (double)st.w[gb + s];
            geometry(m, (double)st.x[0][gb + s], (double)st.x[2][gb + s], rho[i], phi[i]);
            if (w > 0.0) nlw[i] = -log2(m.wscale * w);
            wsum += w;
        }
    }
    wsum = wave_sum(wsum);
    if (lane == 0) pw[(size_t)j * wtiles + wtile] = wsum;
    const size_t pbase = ((size_t)j * wtiles + wtile) * Mmax;
    for (int p = 0; p < M; ++p) {
        const double zr = Z[2 * p] * m.cr, zt = Z[2 * p + 1] * m.ct;
        // exponents stay in double until the shift is removed: far from every
        // particle they reach -1e3 and more, where a float has lost 1e-4
        double a[PT];
        double amax = -__builtin_inf();
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            a[i] = -sq_resid(m, zr, zt, rho[i], phi[i], nlw[i]);
            amax = a[i] > amax ? a[i] : amax;
        }
        const float wmax = wave_max((float)amax);
        const double h = (wmax == -__builtin_inff()) ? 0.0 : (double)ceilf(wmax);
        T s = 0;
#pragma unroll
        for (int i = 0; i < PT; ++i) s += fast_exp2((T)(a[i] - h));
        const double sd = wave_sum((double)s);
        if (lane == 0) {
            ps[pbase + p] = sd;
            ph[pbase + p] = (int)h;
        }
    }
}

// ---------------------------------------------------------------------------
// Combine the first-pass partials of group j (one workgroup per group):
//   H = max h over waves with s > 0, S = sum s 2^(h - H)    (double, fixed order)
//   C = 2^H S,  F = 1/(kappa 2^-H + S) = 2^H/(kappa + C),  dW = S F = C/(kappa + C)
// The candidate labels for Step 3 are the top min(LT_c + 1, #dW>0) measurements
// by dW (ties to the lower index), where LT_c = round(nu sum w + sum dW) is the
// closed form of the updated mass (the sums of Eq 8 swapped); the exact count
// LT differs from LT_c by at most one, so the candidates always cover it.
// grid (K), 256 threads, dynamic LDS Mmax doubles.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_cz_combine(DevModel m, const int* __restrict__ ncur, int M, int Mmax,
                                                    int wtiles, int WT, const double* __restrict__ ps,
                                                    const int* __restrict__ ph, const double* __restrict__ pw,
                                                    int* __restrict__ zH, T* __restrict__ zF,
                                                    double* __restrict__ zC, double* __restrict__ zdW,
                                                    int* __restrict__ zflag, int* __restrict__ cand,
                                                    int* __restrict__ ncand)
{
    extern __shared__ double sm_dw[];
    __shared__ double red[256];
    __shared__ int redi[256];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int n = ncur[j];
    const int nw = (n + WT - 1) / WT;
    const size_t zb = (size_t)j * Mmax;
    double dsum = 0.0;
    for (int p = tid; p < M; p += 256) {
        int H = -2147483647 - 1;
        for (int w = 0; w < nw; ++w) {
            const size_t o = ((size_t)j * wtiles + w) * Mmax + p;
            if (ps[o] > 0.0 && ph[o] > H) H = ph[o];
        }
        double S = 0.0;
        for (int w = 0; w < nw; ++w) {
            const size_t o = ((size_t)j * wtiles + w) * Mmax + p;
            if (ps[o] > 0.0) S += ldexp(ps[o], ph[o] - H);
        }
        double C = 0.0, F = 0.0, dW = 0.0;
        if (S > 0.0) {
            const double D = ldexp(m.kappa, -H) + S;
            F = 1.0 / D;
            dW = S / D;
            C = ldexp(S, H);
        } else {
            H = 0;
        }
        zH[zb + p] = H;
        zF[zb + p] = (T)F;
        zC[zb + p] = C;
        zdW[zb + p] = dW;
        zflag[zb + p] = 0;
        sm_dw[p] = dW;
        dsum += dW;
    }
    // pre-update mass and sum of dW
    double wsum = 0.0;
    if (tid == 0)
        for (int w = 0; w < nw; ++w) wsum += pw[(size_t)j * wtiles + w];
    red[tid] = dsum;
    int pos = 0;
    for (int p = tid; p < M; p += 256) pos += sm_dw[p] > 0.0 ? 1 : 0;
    redi[tid] = pos;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            red[tid] += red[tid + o];
            redi[tid] += redi[tid + o];
        }
        __syncthreads();
    }
    __shared__ int s_nc;
    if (tid == 0) {
        const double mass_c = m.nu * wsum + red[0];
        double lt = floor(mass_c + 0.5);
        int LTc = lt < 0.0 ? 0 : (lt > (double)M ? M : (int)lt);
        int nc = LTc + 1;
        if (nc > redi[0]) nc = redi[0];
        s_nc = nc;
        ncand[j] = nc;
    }
    __syncthreads();
    const int nc = s_nc;
    for (int p = tid; p < M; p += 256) {
        const double v = sm_dw[p];
        if (!(v > 0.0)) continue;
        int rank = 0;
        for (int q = 0; q < M; ++q) {
            const double u = sm_dw[q];
            rank += (u > v || (u == v && q < p)) ? 1 : 0;
        }
        if (rank < nc) {
            cand[zb + rank] = p;
            zflag[zb + p] = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Step 2, second pass (Eqs 12-15) and the sums of Step 3 (Eqs 16-18):
//   w_i <- nu w_i + wscale w_i sum_p 2^(-q_ip - H_p) F_p
// For the candidate labels (visited first) the wave also accumulates
//   u_i = wscale w_i 2^(-q_ip - H_p),  sum u_i x_i (4 components) and sum u_i,
// whose ratio is the local estimate of Eq 18 (F cancels).
// Partials: pmass/pmax[j*wtiles + wave_tile] (sum and max of the stored new
// weights), pzeta[((j*wtiles + wave_tile)*Mmax + c)*5 + k].
// grid (ceil(wtiles/4), K), 256 threads.
// ---------------------------------------------------------------------------
template <typename T, int PT>
__global__ __launch_bounds__(256) void k_weight(DevModel m, SoA<T> st, const int* __restrict__ ncur,
                                                const double* __restrict__ Z, int M, int Mmax, int wtiles,
                                                const int* __restrict__ zH, const T* __restrict__ zF,
                                                const int* __restrict__ zflag, const int* __restrict__ cand,
                                                const int* __restrict__ ncand, double* __restrict__ pmass,
                                                double* __restrict__ pmax, double* __restrict__ pzeta)
{
    constexpr int WT = 64 * PT;
    const int j = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wtile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int n = ncur[j];
    const int base = wtile * WT;
    if (wtile >= wtiles || base >= n) return;
    const size_t gb = (size_t)j * m.cap;
    const size_t zb = (size_t)j * Mmax;
    double rho[PT], phi[PT];
    T wt[PT], acc[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        rho[i] = 0.0;
        phi[i] = 0.0;
        wt[i] = 0;
        acc[i] = 0;
        if (s < n) {
            geometry(m, (double)st.x[0][gb + s], (double)st.x[2][gb + s], rho[i], phi[i]);
            wt[i] = (T)(m.wscale * (double)st.w[gb + s]);
        }
    }
    const int nc = ncand[j];
    const size_t pz = ((size_t)j * wtiles + wtile) * Mmax;
    for (int c = 0; c < nc; ++c) {
        const int p = cand[zb + c];
        const double zr = Z[2 * p] * m.cr, zt = Z[2 * p + 1] * m.ct;
        const double H = (double)zH[zb + p];
        const T F = zF[zb + p];
        T u0 = 0, u1 = 0, u2 = 0, u3 = 0, u4 = 0;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const T e = fast_exp2(-(T)sq_resid(m, zr, zt, rho[i], phi[i], H));
            acc[i] += e * F;
            const int s = base + i * 64 + lane;
            if (s < n) {
                const T u = e * wt[i];
                u0 += u * st.x[0][gb + s];
                u1 += u * st.x[1][gb + s];
                u2 += u * st.x[2][gb + s];
                u3 += u * st.x[3][gb + s];
                u4 += u;
            }
        }
        const double r0 = wave_sum((double)u0), r1 = wave_sum((double)u1), r2 = wave_sum((double)u2),
                     r3 = wave_sum((double)u3), r4 = wave_sum((double)u4);
        if (lane == 0) {
            double* o = pzeta + (pz + c) * 5;
            o[0] = r0;
            o[1] = r1;
            o[2] = r2;
            o[3] = r3;
            o[4] = r4;
        }
    }
    for (int p = 0; p < M; ++p) {
        if (zflag[zb + p]) continue;
        const double zr = Z[2 * p] * m.cr, zt = Z[2 * p + 1] * m.ct;
        const double H = (double)zH[zb + p];
        const T F = zF[zb + p];
#pragma unroll
        for (int i = 0; i < PT; ++i) acc[i] += fast_exp2(-(T)sq_resid(m, zr, zt, rho[i], phi[i], H)) * F;
    }
    double msum = 0.0, mmax = 0.0;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        if (s < n) {
            const double w = (double)st.w[gb + s];
            const T wn = (T)(m.nu * w + (double)wt[i] * (double)acc[i]);
            st.w[gb + s] = wn;
            msum += (double)wn;
            mmax = (double)wn > mmax ? (double)wn : mmax;
        }
    }
    msum = wave_sum(msum);
    mmax = wave_max(mmax);
    if (lane == 0) {
        pmass[(size_t)j * wtiles + wtile] = msum;
        pmax[(size_t)j * wtiles + wtile] = mmax;
    }
}

__device__ __forceinline__ int ceil_log2(int n)
{
    int b = 0;
    while ((1ll << b) < (long long)n) ++b;
    return b;
}

// quantisation shift of resampling: the largest S with n * max_w * 2^S < 2^52
__device__ __forceinline__ int quant_shift(double wmax, int n)
{
    if (!(wmax > 0.0) || n <= 0) return 0;
    int e;
    frexp(wmax, &e);
    return 52 - ceil_log2(n) - e;
}

// ---------------------------------------------------------------------------
// Step 3 per group (one workgroup per group): mass N_j, LT_j = round(N_j)
// capped at M, the first LT_j candidates become the label set I_j, and their
// local estimates zeta = sum u x / sum u.  Also the quantisation shift of the
// group's resampling.  grid (K), 256 threads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(const int* __restrict__ ncur, int M, int Mmax, int wtiles,
                                                  int WT, const double* __restrict__ pmass,
                                                  const double* __restrict__ pmax, const double* __restrict__ pzeta,
                                                  const int* __restrict__ cand, const int* __restrict__ ncand,
                                                  double* __restrict__ fmass, int* __restrict__ fLT,
                                                  int* __restrict__ rsS, int* __restrict__ sel,
                                                  double* __restrict__ zeta)
{
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int n = ncur[j];
    const int nw = (n + WT - 1) / WT;
    const size_t zb = (size_t)j * Mmax;
    __shared__ int s_nsel;
    for (int p = tid; p < M; p += 256) {
        sel[zb + p] = 0;
#pragma unroll
        for (int d = 0; d < 4; ++d) zeta[(zb + p) * 4 + d] = 0.0;
    }
    if (tid == 0) {
        double mass = 0.0, wmax = 0.0;
        for (int w = 0; w < nw; ++w) {
            mass += pmass[(size_t)j * wtiles + w];
            wmax = pmax[(size_t)j * wtiles + w] > wmax ? pmax[(size_t)j * wtiles + w] : wmax;
        }
        double lt = floor(mass + 0.5);
        int LT = lt < 0.0 ? 0 : (lt > (double)M ? M : (int)lt);
        fmass[j] = mass;
        fLT[j] = LT;
        rsS[j] = quant_shift(wmax, n);
        s_nsel = LT < ncand[j] ? LT : ncand[j];
    }
    __syncthreads();
    const int nsel = s_nsel;
    for (int c = tid; c < nsel; c += 256) {
        const int p = cand[zb + c];
        double a[5] = { 0, 0, 0, 0, 0 };
        for (int w = 0; w < nw; ++w) {
            const double* o = pzeta + (((size_t)j * wtiles + w) * Mmax + c) * 5;
#pragma unroll
            for (int k = 0; k < 5; ++k) a[k] += o[k];
        }
        sel[zb + p] = 1;
        if (a[4] > 0.0) {
#pragma unroll
            for (int d = 0; d < 4; ++d) zeta[(zb + p) * 4 + d] = a[d] / a[4];
        }
    }
}

// ---------------------------------------------------------------------------
// Step 4, fusion at the central unit (one workgroup): a label is kept when
// 2*votes > K; its estimate is the mean of the reporting groups' estimates in
// group order; records are written in label order.  grid (1), 256 threads.
// ---------------------------------------------------------------------------
struct EstimateRec {
    double state[4];
    int32_t label;
    int32_t votes;
};

__global__ __launch_bounds__(256) void k_fuse(int K, int M, int Mmax, const int* __restrict__ sel,
                                              const double* __restrict__ zeta, EstimateRec* __restrict__ out,
                                              int cap, int* __restrict__ nout)
{
    __shared__ int scan[256];
    const int tid = threadIdx.x;
    int offset = 0;
    for (int p0 = 0; p0 < M; p0 += 256) {
        const int p = p0 + tid;
        int votes = 0;
        if (p < M)
            for (int j = 0; j < K; ++j) votes += sel[(size_t)j * Mmax + p];
        const int keep = (p < M && 2 * votes > K) ? 1 : 0;
        scan[tid] = keep;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            int v = tid >= o ? scan[tid - o] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const int idx = offset + scan[tid] - keep;
        if (keep && idx < cap) {
            double acc[4] = { 0, 0, 0, 0 };
            for (int j = 0; j < K; ++j) {
                if (!sel[(size_t)j * Mmax + p]) continue;
#pragma unroll
                for (int d = 0; d < 4; ++d) acc[d] += zeta[((size_t)j * Mmax + p) * 4 + d];
            }
            EstimateRec r;
#pragma unroll
            for (int d = 0; d < 4; ++d) r.state[d] = acc[d] / (double)votes;
            r.label = p;
            r.votes = votes;
            out[idx] = r;
        }
        offset += scan[255];
        __syncthreads();
    }
    if (tid == 0) *nout = offset;
}

// ---------------------------------------------------------------------------
// Quantisation shift when the weights come from the host (no update pass ran).
// grid (K), 256 threads.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_wmax(DevModel m, const T* __restrict__ w, const int* __restrict__ ncur,
                                              int* __restrict__ rsS)
{
    __shared__ double red[256];
    const int j = blockIdx.x;
    const int n = ncur[j];
    double mx = 0.0;
    for (int s = threadIdx.x; s < n; s += 256) {
        const double v = (double)w[(size_t)j * m.cap + s];
        mx = v > mx ? v : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = red[threadIdx.x + o] > red[threadIdx.x] ? red[threadIdx.x + o] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) rsS[j] = quant_shift(red[0], n);
}

// ---------------------------------------------------------------------------
// Step 5, resampling, pass A: integer-valued weights q = floor(w 2^S) and their
// exact per-tile totals (tiles of 256*PR parents).  grid (rtiles, K).
// ---------------------------------------------------------------------------
template <typename T, int PR>
__global__ __launch_bounds__(256) void k_rs_tiles(DevModel m, const T* __restrict__ w, const int* __restrict__ ncur,
                                                  const int* __restrict__ rsS, int rtiles, double* __restrict__ tsum)
{
    constexpr int TR = 256 * PR;
    __shared__ double red[4];
    const int j = blockIdx.y, t = blockIdx.x;
    const int n = ncur[j];
    const int base = t * TR;
    if (base >= n) return;
    const int S = rsS[j];
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < PR; ++i) {
        const int s = base + i * 256 + threadIdx.x;
        if (s < n) q += floor(ldexp((double)w[(size_t)j * m.cap + s], S));
    }
    q = wave_sum(q);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) tsum[(size_t)j * rtiles + t] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Number of systematic points below the cumulative boundary c:
//   N(c) = #{ m in [0, L) : (m 2^32 + r) Q < c L 2^32 }.
// A double estimate is corrected with exact 128-bit comparisons.
__device__ __forceinline__ long long points_below(uint64_t c, uint64_t Q, long long L, uint32_t r)
{
    const unsigned __int128 rhs = ((unsigned __int128)c * (unsigned __int128)(uint64_t)L) << 32;
    double est = ceil((double)c * (double)L / (double)Q - (double)r * 0x1p-32);
    long long m0 = est < 0.0 ? 0 : (est > (double)L ? L : (long long)est);
    auto below = [&](long long mm) {
        const unsigned __int128 lhs = (unsigned __int128)((((uint64_t)mm) << 32) + (uint64_t)r) * (unsigned __int128)Q;
        return lhs < rhs;
    };
    while (m0 > 0 && !below(m0 - 1)) --m0;
    while (m0 < L && below(m0)) ++m0;
    return m0;
}

// L' = floor(N R_j + 0.5) with two separate roundings (no fused multiply-add)
__device__ __forceinline__ double children_count(double mq, double Rj)
{
#pragma clang fp contract(off)
    double t = mq * Rj;
    t = t + 0.5;
    return floor(t);
}

// ---------------------------------------------------------------------------
// Step 5, pass B: exact prefix of q, child counts and parent-order expansion
// into the other particle set.  Thread t of a tile owns parents
// [base + t*PR, base + t*PR + PR); the workgroup writes the children of its
// parents, which occupy one contiguous slot range, with coalesced stores
// (each child finds its parent by binary search over the tile's child offsets
// held in LDS).  grid (rtiles, K), 256 threads.
// ---------------------------------------------------------------------------
template <typename T, int PR>
__global__ __launch_bounds__(256) void k_rs_expand(DevModel m, SoA<T> in, SoA<T> out,
                                                   const int* __restrict__ ncur, int* __restrict__ nsurv,
                                                   const int* __restrict__ rsS, const double* __restrict__ tsum,
                                                   int rtiles, uint32_t step, double* __restrict__ massq,
                                                   int* __restrict__ clampctr, int* __restrict__ counts,
                                                   int record)
{
    constexpr int TR = 256 * PR;
    __shared__ int s_off[TR + 1];
    __shared__ T s_x[4][TR];
    __shared__ double red[256];
    const int j = blockIdx.y, t = blockIdx.x;
    const int tid = threadIdx.x;
    const int n = ncur[j];
    const int ntl = (n + TR - 1) / TR;
    if (t > 0 && t >= ntl) return;
    const size_t gb = (size_t)j * m.cap;
    const int base = t * TR;
    // group total Q and this tile's exclusive prefix P (exact integer sums)
    double qa = 0.0, qp = 0.0;
    for (int u = tid; u < ntl; u += 256) {
        const double v = tsum[(size_t)j * rtiles + u];
        qa += v;
        if (u < t) qp += v;
    }
    red[tid] = qa;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    const double Qd = red[0];
    __syncthreads();
    red[tid] = qp;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    const double Pd = red[0];
    __syncthreads();
    const int S = rsS[j];
    const int Jj = births_in(m, j);
    long long L = 0;
    double mq = 0.0;
    if (Qd > 0.0) {
        mq = ldexp(Qd, -S);
        double Lf = children_count(mq, m.Rj);
        const double lim = (double)(m.cap - Jj);
        bool clamped = false;
        if (Lf > lim) {
            Lf = lim;
            clamped = true;
        }
        if (Lf < 0.0) Lf = 0.0;
        L = (long long)Lf;
        if (t == 0 && tid == 0 && clamped) atomicAdd(clampctr, 1);
    }
    if (t == 0 && tid == 0) {
        nsurv[j] = (int)L;
        massq[j] = mq;
    }
    if (L == 0 || base >= n) {
        if (record) {
            for (int s = base + tid; s < n && s < base + TR; s += 256) counts[gb + s] = 0;
        }
        return;
    }
    const double wc = mq / (double)L;
    const uint32_t r = rng_block(m.key0, m.key1, (uint32_t)j, step, RNG_RESAMPLE, 0, m.run).a;
    const uint64_t Q = (uint64_t)Qd;
    // parents of this thread, their integer weights and inclusive prefix
    double q[PR];
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < PR; ++i) {
        const int s = base + tid * PR + i;
        q[i] = (s < n) ? floor(ldexp((double)in.w[gb + s], S)) : 0.0;
        tot += q[i];
    }
    // workgroup exclusive scan of thread totals (exact)
    red[tid] = tot;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const double v = tid >= o ? red[tid - o] : 0.0;
        __syncthreads();
        red[tid] += v;
        __syncthreads();
    }
    const double excl = red[tid] - tot;
    double cprev = Pd + excl;
    long long nprev = points_below((uint64_t)cprev, Q, L, r);
#pragma unroll
    for (int i = 0; i < PR; ++i) {
        const int li = tid * PR + i;
        s_off[li] = (int)nprev;
        const double c = cprev + q[i];
        const long long nc = (q[i] > 0.0) ? points_below((uint64_t)c, Q, L, r) : nprev;
        if (record && base + li < n) counts[gb + base + li] = (int)(nc - nprev);
        cprev = c;
        nprev = nc;
    }
    if (tid == 255) s_off[TR] = (int)nprev;
    // stage parent states in LDS (coalesced)
#pragma unroll
    for (int i = 0; i < PR; ++i) {
        const int li = i * 256 + tid;
        const int s = base + li;
        if (s < n) {
#pragma unroll
            for (int d = 0; d < 4; ++d) s_x[d][li] = in.x[d][gb + s];
        }
    }
    __syncthreads();
    const int c0 = s_off[0], c1 = s_off[TR];
    for (int c = c0 + tid; c < c1; c += 256) {
        // last parent li with s_off[li] <= c
        int lo = 0, hi = TR - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= c) lo = mid; else hi = mid - 1;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) out.x[d][gb + c] = s_x[d][lo];
        out.w[gb + c] = (T)wc;
    }
}

// ---------------------------------------------------------------------------
// Step 6, ring exchange j -> j+1.  One count L = floor(rho_x min_j n_j) for all
// groups; group j's chosen slots are S_j(m) = (o_j + m floor(n_j/L)) mod n_j
// with o_j from the EXCHANGE stream, and the couple in S_j(m) replaces the one
// in S_{j+1}(m).  A gather into a staging buffer followed by a scatter (two
// launches) makes every read see the state before the exchange, so the
// exchange is a permutation of the particles.  grid (ceil(Lmax/256), K).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int exchange_count(const DevModel& m, const int* __restrict__ nsurv)
{
    int mn = nsurv[0];
    for (int j = 1; j < m.K; ++j) mn = nsurv[j] < mn ? nsurv[j] : mn;
    return (int)floor(m.xfrac * (double)mn);
}

__device__ __forceinline__ uint64_t exchange_slot(const DevModel& m, int j, int nj, int L, int mm, uint32_t step)
{
    const Block4 a = rng_block(m.key0, m.key1, (uint32_t)j, step, RNG_EXCHANGE, 0, m.run);
    const uint64_t o = ((uint64_t)a.a * (uint64_t)nj) >> 32;
    return (o + (uint64_t)mm * (uint64_t)(nj / L)) % (uint64_t)nj;
}

template <typename T>
__global__ __launch_bounds__(256) void k_xchg_gather(DevModel m, SoA<T> st, const int* __restrict__ nsurv,
                                                     T* __restrict__ stage, int Lmax, uint32_t step)
{
    const int j = blockIdx.y;
    const int mm = blockIdx.x * 256 + threadIdx.x;
    const int L = exchange_count(m, nsurv);
    if (mm >= L || mm >= Lmax) return;
    const size_t src = (size_t)j * m.cap + (size_t)exchange_slot(m, j, nsurv[j], L, mm, step);
    T* o = stage + ((size_t)j * Lmax + mm) * 5;
#pragma unroll
    for (int d = 0; d < 4; ++d) o[d] = st.x[d][src];
    o[4] = st.w[src];
}

template <typename T>
__global__ __launch_bounds__(256) void k_xchg_scatter(DevModel m, SoA<T> st, const int* __restrict__ nsurv,
                                                      const T* __restrict__ stage, int Lmax, uint32_t step)
{
    const int j = blockIdx.y;
    const int mm = blockIdx.x * 256 + threadIdx.x;
    const int L = exchange_count(m, nsurv);
    if (mm >= L || mm >= Lmax) return;
    const int jn = (j + 1) % m.K;
    const size_t dst = (size_t)jn * m.cap + (size_t)exchange_slot(m, jn, nsurv[jn], L, mm, step);
    const T* o = stage + ((size_t)j * Lmax + mm) * 5;
#pragma unroll
    for (int d = 0; d < 4; ++d) st.x[d][dst] = o[d];
    st.w[dst] = o[4];
}

}  // namespace pphd
