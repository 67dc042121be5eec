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

#include "mlp_internal.h"
#include "philox_dev.h"

namespace pphd {

struct DevModel {
    double T, sigma_a, sx, sy;
    double pS, pD, nu, kappa;
    double birth_mass, reg0, reg1, reg2, reg3, sigma_v, init_mass, Rj, xfrac;
    double cr, ct, period, inv_period, wscale;  // scaled likelihood, see above
    double sigma_r, sigma_th, inv_area, alpha;  // measurement-driven birth proposal
    int K, J, cap, M0, proposal, density;  // density: birth density option (1 = Gaussian)
    uint32_t key0, key1, run, one_run;  // one_run: every group belongs to run 0
    double bmean[4], bstd[4];              // Gaussian birth density
    int dim, tile_major;                   // dim 4: CV [x, vx, y, vy]; 5: coordinated turn, + omega
                                           // tile_major: per-slot grids are (tiles, groups)
    double sigma_w, birth_sigma_w;         // turn-rate noise and birth spread (dim 5)
};

__device__ __forceinline__ int slot_group(const DevModel& m) { return m.tile_major ? blockIdx.y : blockIdx.x; }
__device__ __forceinline__ int slot_tile(const DevModel& m) { return m.tile_major ? blockIdx.x : blockIdx.y; }

// ---------------------------------------------------------------------------
// Bearing order: before the systematic resampling (Step 5) every group's
// parents, and once drawn its births, are taken in bearing-bucket order
// (buckets ascending, slot order inside a bucket), so that nearby particles
// sit together and a likelihood-pass tile spans a narrow bearing range.  The
// bucket is the "diamond angle" d in [0, 4) of the offset from the sensor
// (monotonic in the bearing counter-clockwise from +x, one correctly rounded
// division), times BEARING_BUCKETS/4, rounded down; a birth's bucket is that
// of its position as drawn (in double, before the storage rounding).  A
// stable counting sort: per-tile bucket histograms, bucket-major offsets per
// group, a scatter into the other particle set.
// ---------------------------------------------------------------------------
constexpr int BEARING_BUCKETS = 64;
// Each group's quantised parent total Q is accumulated in QSLOTS partial
// sums (exact integers in any order), so that the atomic additions of the
// resampling's scatter spread over that many addresses.  Slot-major, slot s
// of group g at qtot[s K + g]: a wavefront reading consecutive groups' totals
// (every expansion workgroup does, for the exchange count) reads QSLOTS
// contiguous rows instead of one cache line per group.
constexpr int QSLOTS = 8;
__device__ __forceinline__ double& qslot(double* qtot, int g, int s, int K) { return qtot[(size_t)s * K + g]; }
__device__ __forceinline__ double group_q(const double* __restrict__ qtot, int g, int K)
{
    double q[QSLOTS];
#pragma unroll
    for (int s = 0; s < QSLOTS; ++s) q[s] = qtot[(size_t)s * K + g];
    return ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
}

__device__ __forceinline__ int bearing_bucket(const DevModel& m, double x, double y)
{
    const double dx = x - m.sx, dy = y - m.sy;
    // the quadrant's offset plus one quotient, selected rather than branched
    // (one division per slot): 0 + dy/(dx+dy), 1 + (-dx)/(dy-dx),
    // 2 + (-dy)/(-dx-dy), 3 + dx/(dx-dy); negating a quotient's numerator
    // negates the correctly rounded quotient exactly
    const bool up = dy >= 0.0, right = dx >= 0.0;
    const double num = up ? (right ? dy : -dx) : (right ? dx : -dy);
    const double den = up ? (right ? dx + dy : dy - dx) : (right ? dx - dy : -dx - dy);
    const double off = up ? (right ? 0.0 : 1.0) : (right ? 3.0 : 2.0);
    const double d = (dx == 0.0 && dy == 0.0) ? 0.0 : off + num / den;
    const int b = (int)floor(d * (BEARING_BUCKETS / 4.0));
    return b < 0 ? 0 : (b > BEARING_BUCKETS - 1 ? BEARING_BUCKETS - 1 : b);
}

template <typename T>
struct SoA {
    T* x[5];  // x[4] (the turn rate) only with dim 5
    T* w;
};

// Per-slot kernels run on grids (groups, tiles of the capacity), so that
// every group's first tiles (which hold its particles) are dispatched before
// the capacity's empty tail.  Groups of clearly different sizes use (tiles,
// groups) instead (DevModel::tile_major): consecutive workgroups then take
// consecutive tiles of one group, spread over the chip's dies, where the
// group-major order would give whole groups to one die each.

// Per-group constants.  A filter is a batch of independent runs; each run has
// K_r groups (partitions), and global group g owns the particle slots
// [g*cap, g*cap + cap).  The random-number counters of a group use its
// run-local slot index jl*cap + s and its run's Philox run word, so a run
// draws the same numbers alone or inside a batch.
struct Grp {
    int jl, K, g0, run;  // partition within the run, partitions of the run, run's first group, run index
    int Jj, M0;          // births per step, initial particles
    uint32_t rng_run;    // Philox run word of the run
    int gz;              // 1 when one C(z) spans the run's groups (they split one PHD): Step 3's LT and
                         // Step 5's L' then take the run's total mass instead of the group's own
    double kappa, Rj;    // clutter density of the run; particles per target of the group (R/K)
};

// Measurement window of a run in a batched update: offset (in measurements)
// into the step's concatenated set and count.
struct ZWin {
    int off, M;
};

// the step index: a value, or (captured graphs) a device counter
__device__ __forceinline__ uint32_t step_of(uint32_t step, const uint32_t* dstep) { return dstep ? *dstep : step; }

// this group's measurements: from its run's window (batched update) or the
// whole set (single run, win == nullptr)
struct ZView {
    const double* Z;
    int M;
};
__device__ __forceinline__ ZView zview(const Grp& g, const ZWin* win, const double* Z, int M)
{
    if (!win) return ZView{ Z, M };
    const ZWin w = win[g.run];
    return ZView{ Z + 2 * (size_t)w.off, w.M };
}

// ---------------------------------------------------------------------------
// wavefront reductions (64 lanes, all lanes active).  Within each row of 16
// lanes the data-parallel-primitive (DPP) lane swizzles combine neighbours in
// four steps (quad swaps, half-row and row mirrors); the four row results are
// then read into scalars and combined, so every lane gets the same value and
// the tree order is fixed (results are reproducible).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
__device__ __forceinline__ float lane_value(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_value(double v, int l)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}
__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
// element i of an array at a wave-uniform base, addressed by a 32-bit byte
// offset (a base pointer in scalar registers plus one vector register per
// load instead of a 64-bit vector address); i * sizeof(U) must stay below
// 2^32, which holds within one group's slots (at most 65535 * 256)
template <typename U>
__device__ __forceinline__ U ld_slot(const U* __restrict__ base, uint32_t i)
{
    return *reinterpret_cast<const U*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(U));
}
// index of this thread's wavefront in the workgroup, as a wave-uniform value
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
// quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E, row_half_mirror = 0x141, row_mirror = 0x140
template <typename V>
__device__ __forceinline__ V wave_sum(V v)
{
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}
template <typename V>
__device__ __forceinline__ V vmax(V a, V b) { return a > b ? a : b; }
template <typename V>
__device__ __forceinline__ V wave_max(V v)
{
    v = vmax(v, dpp<0xB1>(v));
    v = vmax(v, dpp<0x4E>(v));
    v = vmax(v, dpp<0x141>(v));
    v = vmax(v, dpp<0x140>(v));
    return vmax(vmax(lane_value(v, 0), lane_value(v, 16)), vmax(lane_value(v, 32), lane_value(v, 48)));
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double fast_exp2(double x) { return exp2(x); }

// inclusive prefix sum over the 64 lanes: row_shr 1, 2, 4, 8 within each row of
// 16 lanes (a missing source lane reads 0), then the row totals are added to
// the rows above them
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double v) { return dpp<CTRL>(v); }
__device__ __forceinline__ double wave_incl_scan(double v)
{
    const int lane = threadIdx.x & 63;
    v += dpp<0x111>(v);
    v += dpp<0x112>(v);
    v += dpp<0x114>(v);
    v += dpp<0x118>(v);
    const double r0 = lane_value(v, 15), r1 = lane_value(v, 31), r2 = lane_value(v, 47);
    const int row = lane >> 4;
    if (row >= 1) v += r0;
    if (row >= 2) v += r1;
    if (row >= 3) v += r2;
    return v;
}

// ---------------------------------------------------------------------------
// draws from the normalised birth density: position uniform over the region,
// velocity N(0, sigma_v^2 I); or (density 1) the Gaussian N(mean, diag std^2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void draw_birth(const DevModel& m, uint32_t slot, uint32_t step, uint32_t purpose,
                                           uint32_t run, double s[5])
{
    Block4 a = rng_block(m.key0, m.key1, slot, step, purpose, 0, run);
    Block4 b = rng_block(m.key0, m.key1, slot, step, purpose, 1, run);
    s[4] = 0.0;
    if (m.dim == 5) {
        // turn rate N(0, birth_sigma_w^2) from a third block
        const Block4 c = rng_block(m.key0, m.key1, slot, step, purpose, 2, run);
        double w1, w2;
        normal_pair(uniform53(c.a, c.b), uniform53(c.c, c.d), w1, w2);
        s[4] = m.birth_sigma_w * w1;
    }
    double ux = uniform53(a.a, a.b), uy = uniform53(a.c, a.d);
    double n1, n2;
    normal_pair(uniform53(b.a, b.b), uniform53(b.c, b.d), n1, n2);
    if (m.density == 1) {
        // Gaussian birth intensity: position normals from the first block
        double p1, p2;
        normal_pair(ux, uy, p1, p2);
        s[0] = m.bmean[0] + m.bstd[0] * p1;
        s[1] = m.bmean[1] + m.bstd[1] * n1;
        s[2] = m.bmean[2] + m.bstd[2] * p2;
        s[3] = m.bmean[3] + m.bstd[3] * n2;
        return;
    }
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
__global__ __launch_bounds__(256) void k_init(DevModel m, const Grp* __restrict__ gd, SoA<T> st,
                                              int* __restrict__ nsurv)
{
    const int j = slot_group(m);
    const Grp gr = gd[j];
    const int s = slot_tile(m) * 256 + threadIdx.x;
    if (slot_tile(m) == 0 && threadIdx.x == 0) nsurv[j] = gr.M0;
    if (s >= gr.M0) return;
    const size_t g = (size_t)j * m.cap + s;
    double v[5];
    draw_birth(m, (uint32_t)(gr.jl * m.cap + s), 0u, RNG_INIT, gr.rng_run, v);
    for (int d = 0; d < m.dim; ++d) st.x[d][g] = (T)v[d];
    st.w[g] = (T)(m.init_mass / (double)gr.M0);
}

// ---------------------------------------------------------------------------
// Per-particle geometry used by the two likelihood passes, in scaled units:
// rho' = |p - s| c_r, phi' = atan2 c_t, and lw = log2(wscale w) (-inf for
// w = 0).  Written by predict (and by k_geom when the state comes from the
// host), so the passes never evaluate sqrt/atan2/log.
// ---------------------------------------------------------------------------
struct Geo {
    double* rho;
    double* phi;   // bearing c_t in [-pi, pi) c_t
    double* phib;  // the same bearing in a frame turned by pi, also in [-pi, pi) c_t
    double* lw;
};

// log2 of a positive weight: in double for FP64 storage; for FP32 storage
// the exponent exactly and the mantissa's log2 in float (within about 2e-7,
// a relative change of the same size in the particle's likelihood terms,
// far below the weights' own storage rounding)
__device__ __forceinline__ double weight_log2(double v, double) { return log2(v); }
__device__ __forceinline__ double weight_log2(double v, float)
{
    int e;
    const double f = frexp(v, &e);  // v = f 2^e, f in [1/2, 1)
    return (double)e + (double)log2f((float)f);
}

template <typename T>
__device__ __forceinline__ void store_geometry(const DevModel& m, Geo geo, size_t g, double x, double y, double w)
{
    const double dx = x - m.sx, dy = y - m.sy;
    geo.rho[g] = sqrt(dx * dx + dy * dy) * m.cr;
    const double ph = atan2(dy, dx);
    geo.phi[g] = ph * m.ct;
    geo.phib[g] = (ph < 0.0 ? ph + 3.14159265358979323846 : ph - 3.14159265358979323846) * m.ct;
    geo.lw[g] = (w > 0.0) ? weight_log2(m.wscale * w, T(0)) : -__builtin_inf();
}

// ---------------------------------------------------------------------------
// Step 1 (Eqs 5, 6): survivors through the CV model, births appended.
// grid (ceil(cap/256), K)
// ---------------------------------------------------------------------------
// one slot of k_predict
template <typename T>
__device__ __forceinline__ void predict_slot(const DevModel& m, const Grp& gr, const SoA<T>& st, const Geo& geo,
                                             int ns, int Jj, int j, int s, uint32_t step, int* __restrict__ bkt)
{
    const size_t g = (size_t)j * m.cap + s;
    const uint32_t c0 = (uint32_t)(gr.jl * m.cap + s);
    double v[5], w;
    if (s < ns) {
        // the state first: its reads are in flight while the noise is drawn
        // (x[0] stands in for an absent turn rate)
        const double x = st.x[0][g], vx = st.x[1][g], y = st.x[2][g], vy = st.x[3][g];
        const double om = st.x[m.dim == 5 ? 4 : 0][g];
        const double wold = (double)st.w[g];
        Block4 r = rng_block(m.key0, m.key1, c0, step, RNG_PREDICT, 0, gr.rng_run);
        double n1, n2;
        normal_pair(uniform53(r.a, r.b), uniform53(r.c, r.d), n1, n2);
        const double ax = m.sigma_a * n1, ay = m.sigma_a * n2;
        const double half_t2 = m.T * m.T / 2;
        if (m.dim == 5) {
            // coordinated turn at the particle's rate: the velocity turns by
            // omega T, the position follows the arc (limits T and 0 at omega = 0)
            double sn, cs;
            sincos(om * m.T, &sn, &cs);
            const double fa = om != 0.0 ? sn / om : m.T;
            const double fb = om != 0.0 ? (1.0 - cs) / om : 0.0;
            v[0] = x + fa * vx - fb * vy + half_t2 * ax;
            v[1] = cs * vx - sn * vy + m.T * ax;
            v[2] = y + fb * vx + fa * vy + half_t2 * ay;
            v[3] = sn * vx + cs * vy + m.T * ay;
            const Block4 r2 = rng_block(m.key0, m.key1, c0, step, RNG_PREDICT, 1, gr.rng_run);
            double w1, w2;
            normal_pair(uniform53(r2.a, r2.b), uniform53(r2.c, r2.d), w1, w2);
            v[4] = om + m.T * m.sigma_w * w1;
        } else {
            v[0] = x + m.T * vx + half_t2 * ax;
            v[1] = vx + m.T * ax;
            v[2] = y + m.T * vy + half_t2 * ay;
            v[3] = vy + m.T * ay;
            v[4] = 0.0;
        }
        w = m.pS * wold;
    } else {
        if (m.proposal != 0) return;  // drawn by k_birth_draw once Z_k is known
        draw_birth(m, c0, step, RNG_BIRTH, gr.rng_run, v);
        w = m.birth_mass / (double)Jj;
    }
    T t[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        t[d] = (T)v[d];
        st.x[d][g] = t[d];
    }
    if (m.dim == 5) st.x[4][g] = (T)v[4];
    const T tw = (T)w;
    st.w[g] = tw;
    // births get their geometry once put in bearing order, by the bucket of
    // the position as drawn
    if (s < ns) store_geometry<T>(m, geo, g, (double)t[0], (double)t[2], (double)tw);
    else bkt[g] = bearing_bucket(m, v[0], v[2]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_predict(DevModel m, const Grp* __restrict__ gd, SoA<T> st, Geo geo,
                                                 const int* __restrict__ nsurv, int* __restrict__ ncur,
                                                 uint32_t step_arg, const uint32_t* __restrict__ dstep,
                                                 int* __restrict__ bkt)
{
    const int j = slot_group(m);
    const Grp gr = gd[j];
    const uint32_t step = step_of(step_arg, dstep);
    const int ns = nsurv[j];
    const int Jj = gr.Jj;
    // the host guarantees ns + J_j <= cap; the clamp keeps every store inside the group
    const int total = ns + Jj < m.cap ? ns + Jj : m.cap;
    if (slot_tile(m) == 0 && threadIdx.x == 0) ncur[j] = total;
    // one tile per workgroup (a loop over tiles would keep the math
    // library's constants live across it, tripling the registers)
    const int s = slot_tile(m) * 256 + threadIdx.x;
    if (s < total) predict_slot(m, gr, st, geo, ns, Jj, j, s, step, bkt);
}

// Step 1 for 2048 slots of one group, as k_predict does it for 256 (the
// prediction rides in the births' launch when the births are drawn there):
// part w takes group w mod K, slots [2048 floor(w / K), +2048), two per
// thread, so every group's first slots come first (groups of clearly
// different sizes: the group's slot blocks one after another, spreading it
// over the chip's dies).  Two slots per thread halve the workgroups to
// dispatch, most of which are empty (the parts follow the capacity)
template <typename T>
__device__ __forceinline__ void predict_part(const DevModel& m, const Grp* __restrict__ gd, const SoA<T>& st,
                                             const Geo& geo, const int* __restrict__ nsurv, int* __restrict__ ncur,
                                             uint32_t step, int* __restrict__ bkt, int w, int K)
{
    int j, t4;
    if (m.tile_major) {
        const int per = (m.cap + 2047) / 2048;
        j = w / per;
        t4 = w - j * per;
    } else {
        j = w % K;
        t4 = w / K;
    }
    const Grp gr = gd[j];
    const int ns = nsurv[j];
    const int total = ns + gr.Jj < m.cap ? ns + gr.Jj : m.cap;
    if (t4 == 0 && threadIdx.x == 0) ncur[j] = total;
    const int s = t4 * 2048 + threadIdx.x;
    if (s < ns) predict_slot(m, gr, st, geo, ns, gr.Jj, j, s, step, bkt);
    if (s + 1024 < ns) predict_slot(m, gr, st, geo, ns, gr.Jj, j, s + 1024, step, bkt);
}

// dim 5: the turn rate of a birth drawn from a measurement-driven or learned
// proposal comes from the birth density's N(0, birth_sigma_w^2) (block sub 4),
// so its density cancels in the Eq 6 weight
__device__ __forceinline__ double birth_turn_rate(const DevModel& m, uint32_t c0, uint32_t step, uint32_t run)
{
    const Block4 c = rng_block(m.key0, m.key1, c0, step, RNG_BIRTH, 4, run);
    double w1, w2;
    normal_pair(uniform53(c.a, c.b), uniform53(c.c, c.d), w1, w2);
    return m.birth_sigma_w * w1;
}

// geometry of a state written from the host.  grid (ceil(cap/256), K)
template <typename T>
__global__ __launch_bounds__(256) void k_geom(DevModel m, SoA<T> st, Geo geo, const int* __restrict__ ncur)
{
    const int j = slot_group(m);
    const int s = slot_tile(m) * 256 + threadIdx.x;
    if (s >= ncur[j]) return;
    const size_t g = (size_t)j * m.cap + s;
    store_geometry<T>(m, geo, g, (double)st.x[0][g], (double)st.x[2][g], (double)st.w[g]);
}

// ---------------------------------------------------------------------------
// Births from a measurement-driven proposal of Eq 6 in three launches: the
// draw (positions and velocities, the weight left for later), the bearing
// order (k_birth_sort / the range sort, which also records each birth's
// drawing index), and the weight (one lane per ordered birth: the birth's
// position is drawn again from its drawing slot's Philox numbers, in double,
// and its proposal density summed over the terms that the wavefront's
// bounding box does not put below the exponential's underflow).
//
// birth_proposal 1 (the measurement-driven mixture):
//   q(x) = alpha gamma(x)/m_b + (1 - alpha) (1/M) sum_p q_p(x),
// q_p drawing range N(r_p, sigma_r^2) and bearing N(theta_p, sigma_theta^2)
// around the sensor.  Position density of q_p at distance rho, bearing phi:
// [N(rho - r_p) N(wrap(phi - theta_p)) + N(rho + r_p) N(wrap(phi + pi - theta_p))]
// / rho (a negative drawn range lands on the opposite side; 1/rho is the
// polar Jacobian).  Weight gamma/(J_j q) = m_b U(x) / (J_j q_pos(x)) since
// both components draw velocity from N(0, sigma_v^2 I).
// birth_proposal 2 (the learned mixtures):
//   q(x) = alpha gamma(x)/m_b + (1 - alpha) (1/M) sum_p sum_c pi_pc N(x; mu_pc, diag sigma_pc^2),
// draws per slot: position uniforms (sub 0), velocity normals (sub 1), the
// choice of measurement and component (sub 2) and the two position normals
// of a Gaussian component (sub 3); weight gamma(x) / (J_j q(x)), gamma(x) =
// m_b U(x, y) N(vx; 0, sv^2) N(vy; 0, sv^2).
// ---------------------------------------------------------------------------
// d - 2 pi k, the integer k nearest d / (2 pi): the residual in [-pi, pi]
// up to rounding (a product by 1/(2 pi) in place of a division; at the
// seam either sign gives the same square)
__device__ __forceinline__ double wrap_pi(double d)
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    return d - two_pi * rint(d * (1.0 / two_pi));
}

// exp(-a) for a >= 0: hardware exp2 in float for the FP32 path (terms below
// 2^-126 vanish, far under the mixture's alpha U floor), exp in double otherwise
__device__ __forceinline__ double neg_exp(double a, float) { return (double)__builtin_amdgcn_exp2f((float)(-a * 1.4426950408889634)); }
__device__ __forceinline__ double neg_exp(double a, double) { return exp(-a); }
// exponent beyond which neg_exp returns 0 (or a denormal): e^-104 < 2^-149 in
// float, e^-745 below the smallest double; a term whose partial exponent
// already exceeds it is skipped without changing the sum by more than a denormal
__device__ __forceinline__ double neg_exp_cut(float) { return 104.0; }
__device__ __forceinline__ double neg_exp_cut(double) { return 745.0; }

__device__ __forceinline__ double normal_pdf(double d, double sigma)
{
    const double e = d / sigma;
    return exp(-0.5 * e * e) / (2.5066282746310002 * sigma);
}

// the measurements or mixture rows of group gr's run
struct BirthSrc {
    const double* Z;    // proposal 1: the run's measurements
    const double* tab;  // proposal 2: the run's mixture table
    int M;
};
__device__ __forceinline__ BirthSrc birth_src(const Grp& gr, const ZWin* win, const double* Zall,
                                              const double* taball, int Mall)
{
    BirthSrc b{ Zall, taball, Mall };
    if (win) {
        const ZWin w = win[gr.run];
        b.Z = Zall ? Zall + 2 * (size_t)w.off : nullptr;
        b.tab = taball ? taball + (size_t)w.off * 4 * MIX_TAB : nullptr;
        b.M = w.M;
    }
    return b;
}

// one birth of proposal PROP drawn at Philox slot c0: state [x, vx, y, vy]
template <int PROP>
__device__ __forceinline__ void draw_proposal_birth(const DevModel& m, uint32_t c0, uint32_t step, uint32_t run,
                                                    const BirthSrc& src, double* x)
{
    const Block4 a = rng_block(m.key0, m.key1, c0, step, RNG_BIRTH, 0, run);
    const Block4 v = rng_block(m.key0, m.key1, c0, step, RNG_BIRTH, 1, run);
    const Block4 c = rng_block(m.key0, m.key1, c0, step, RNG_BIRTH, 2, run);
    double n1, n2;
    normal_pair(uniform53(v.a, v.b), uniform53(v.c, v.d), n1, n2);
    const double uc = uniform53(c.a, c.b);
    const int M = src.M;
    if (M == 0 || uc <= m.alpha) {
        x[0] = m.reg0 + uniform53(a.a, a.b) * (m.reg1 - m.reg0);
        x[1] = m.sigma_v * n1;
        x[2] = m.reg2 + uniform53(a.c, a.d) * (m.reg3 - m.reg2);
        x[3] = m.sigma_v * n2;
        return;
    }
    int p = (int)floor((uc - m.alpha) / (1.0 - m.alpha) * (double)M);
    p = p > M - 1 ? M - 1 : p;
    if (PROP == 1) {
        double e1, e2;
        normal_pair(uniform53(a.a, a.b), uniform53(a.c, a.d), e1, e2);
        const double R = src.Z[2 * p] + m.sigma_r * e1;
        const double th = src.Z[2 * p + 1] + m.sigma_th * e2;
        x[0] = m.sx + R * cos(th);
        x[1] = m.sigma_v * n1;
        x[2] = m.sy + R * sin(th);
        x[3] = m.sigma_v * n2;
    } else {
        const double uk = uniform53(c.c, c.d);
        int comp = 3;
        for (int k = 0; k < 4; ++k) {
            if (uk <= src.tab[(size_t)(p * 4 + k) * MIX_TAB + 1]) {
                comp = k;
                break;
            }
        }
        const double* t = src.tab + (size_t)(p * 4 + comp) * MIX_TAB;
        const Block4 e = rng_block(m.key0, m.key1, c0, step, RNG_BIRTH, 3, run);
        double e1, e2;
        normal_pair(uniform53(e.a, e.b), uniform53(e.c, e.d), e1, e2);
        x[0] = t[4] + t[8] * e1;
        x[1] = t[5] + t[9] * n1;
        x[2] = t[6] + t[10] * e2;
        x[3] = t[7] + t[11] * n2;
    }
}

// the draw: births b < (placed births of group j) at slots nsurv_j + b, with
// their turn rates (dim 5); weights follow in k_birth_weight.
// grid (groups, ceil(J_max/256)) (or transposed, DevModel::tile_major).
template <typename T, int PROP>
__global__ __launch_bounds__(256) void k_birth_draw(DevModel m, const Grp* __restrict__ gd, SoA<T> st,
                                                    const int* __restrict__ nsurv, const int* __restrict__ ncur,
                                                    const double* __restrict__ Zall, const double* __restrict__ taball,
                                                    int Mall, const ZWin* __restrict__ win, uint32_t step_arg,
                                                    const uint32_t* __restrict__ dstep, int* __restrict__ bkt)
{
    const int j = slot_group(m);
    const Grp gr = gd[j];
    const int ns = nsurv[j], nb = ncur[j] - ns;
    const int b = slot_tile(m) * 256 + threadIdx.x;
    if (b >= nb) return;
    const uint32_t step = step_of(step_arg, dstep);
    const BirthSrc src = birth_src(gr, win, Zall, taball, Mall);
    const uint32_t c0 = (uint32_t)(gr.jl * m.cap + ns + b);
    double x[4];
    draw_proposal_birth<PROP>(m, c0, step, gr.rng_run, src, x);
    const size_t g = (size_t)j * m.cap + ns + b;
#pragma unroll
    for (int d = 0; d < 4; ++d) st.x[d][g] = (T)x[d];
    if (m.dim == 5) st.x[4][g] = (T)birth_turn_rate(m, c0, step, gr.rng_run);
    st.w[g] = (T)0;
    bkt[g] = bearing_bucket(m, x[0], x[2]);
}

// distance of t from the arc [lo, lo + span] (span in [0, 2 pi])
__device__ __forceinline__ double arc_dist(double t, double lo, double span)
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    double u = wrap_pi(t - lo);
    if (u < 0.0) u += two_pi;  // [0, 2 pi)
    return u <= span ? 0.0 : fmin(u - span, two_pi - u);
}
// distance of v from [lo, hi]
__device__ __forceinline__ double box_gap(double v, double lo, double hi) { return fmax(0.0, fmax(lo - v, v - hi)); }

// The Eq 6 weight of a birth at x drawn from the measurement-driven
// (PROP 1) or learned-mixture (PROP 2) proposal: lane = one birth of the
// wavefront (active: a birth is there), whose 64 births bound the density's
// terms: proposal 1 by their range interval and bearing arc, proposal 2 by
// their x and y intervals.  Terms whose bound reaches the cut are exactly
// those the per-term test of the full sum skips, or below it by a denormal
// at most.  All 64 lanes call it.
template <typename T, int PROP>
__device__ __forceinline__ double birth_weight_at(const DevModel& m, const BirthSrc& src, int Jj, const double* x,
                                                  bool active)
{
    const int lane = threadIdx.x & 63;
    const int M = src.M;
    const bool inside = x[0] >= m.reg0 && x[0] <= m.reg1 && x[2] >= m.reg2 && x[2] <= m.reg3;
    double bd = inside ? m.inv_area : 0.0;  // gamma / m_b at x (proposal 1: the position part)
    if (PROP == 2 && inside) bd *= normal_pdf(x[1], m.sigma_v) * normal_pdf(x[3], m.sigma_v);
    const bool use = active && bd > 0.0;    // births whose weight needs the density
    const double cut = neg_exp_cut(T(0));
    double mix = 0.0;
    if (M > 0 && __ballot(use) != 0) {
        const double inf = __builtin_inf();
        if (PROP == 1) {
            const double dx = x[0] - m.sx, dy = x[2] - m.sy;
            const double rho = sqrt(dx * dx + dy * dy), phi = atan2(dy, dx);
            const double isr = 1.0 / m.sigma_r, ist = 1.0 / m.sigma_th;
            // the births' range interval and smallest bearing arc (in the
            // frame whose seam the births avoid)
            const double pi = 3.14159265358979323846;
            const double phb = phi > 0.0 ? phi - pi : phi + pi;
            const double rlo = -wave_max(use ? -rho : -inf), rhi = wave_max(use ? rho : -inf);
            const double alo = -wave_max(use ? -phi : -inf), ahi = wave_max(use ? phi : -inf);
            const double blo = -wave_max(use ? -phb : -inf), bhi = wave_max(use ? phb : -inf);
            const bool fa = ahi - alo <= bhi - blo;
            const double lo = fa ? alo : blo + pi, span = fa ? ahi - alo : bhi - blo;
            for (int c0 = 0; c0 < M; c0 += 64) {
                const int p = c0 + lane;
                bool need = false;
                double zr = 0.0, zt = 0.0;
                if (p < M) {
                    zr = src.Z[2 * p];
                    zt = src.Z[2 * p + 1];
                    const double er = box_gap(zr, rlo, rhi) * isr, et = arc_dist(zt, lo, span) * ist;
                    need = 0.5 * (er * er + et * et) < cut;
                    if (zr < 40.0 * m.sigma_r) {
                        const double fr = box_gap(-zr, rlo, rhi) * isr, ft = arc_dist(zt - pi, lo, span) * ist;
                        need = need || 0.5 * (fr * fr + ft * ft) < cut;
                    }
                }
                for (uint64_t live = __ballot(need); live; live &= live - 1) {
                    const int l = __builtin_ctzll(live);
                    const double r_p = lane_value(zr, l), t_p = lane_value(zt, l);
                    const double er = (rho - r_p) * isr;
                    double t = 0.0;
                    // the range residual alone decides most far measurements
                    if (0.5 * er * er < cut) {
                        const double et = wrap_pi(phi - t_p) * ist;
                        t = neg_exp(0.5 * (er * er + et * et), T(0));
                    }
                    // the negative-range branch: exactly zero in double once r_p > 40 sigma_r
                    if (r_p < 40.0 * m.sigma_r) {
                        const double fr = (rho + r_p) * isr, ft = wrap_pi(phi + pi - t_p) * ist;
                        t += neg_exp(0.5 * (fr * fr + ft * ft), T(0));
                    }
                    mix += t;
                }
            }
            mix *= 1.0 / (2.0 * pi * m.sigma_r * m.sigma_th * rho);
        } else {
            const double xlo = -wave_max(use ? -x[0] : -inf), xhi = wave_max(use ? x[0] : -inf);
            const double ylo = -wave_max(use ? -x[2] : -inf), yhi = wave_max(use ? x[2] : -inf);
            for (int e0 = 0; e0 < 4 * M; e0 += 64) {
                const int e = e0 + lane;
                bool need = false;
                // the bound reads the five values it needs
                if (e < 4 * M) {
                    const double* t = src.tab + (size_t)e * MIX_TAB;
                    const double d0 = box_gap(t[4], xlo, xhi) * t[12], d2 = box_gap(t[6], ylo, yhi) * t[14];
                    need = 0.5 * (d0 * d0 + d2 * d2) - t[2] < cut;
                }
                // a kept term's entry is the same for the whole wavefront
                // (scalar reads); position part first: a far component is
                // skipped before its exponential
                for (uint64_t live = __ballot(need); live; live &= live - 1) {
                    const int l = __builtin_ctzll(live);
                    const double* t = src.tab + (size_t)(e0 + l) * MIX_TAB;
                    const double d0 = (x[0] - t[4]) * t[12];
                    const double d2 = (x[2] - t[6]) * t[14];
                    const double ap = 0.5 * (d0 * d0 + d2 * d2) - t[2];
                    if (ap < cut) {
                        const double d1 = (x[1] - t[5]) * t[13];
                        const double d3 = (x[3] - t[7]) * t[15];
                        mix += neg_exp(ap + 0.5 * (d1 * d1 + d3 * d3), T(0));
                    }
                }
            }
        }
    }
    double w = 0.0;
    if (active && bd > 0.0) {
        const double q = M > 0 ? m.alpha * bd + (1.0 - m.alpha) * mix / (double)M : bd;
        w = m.birth_mass * bd / ((double)Jj * q);
    }
    return w;
}

// the weights of ordered births: lane = ordered birth s of group j (drawn at
// index borig[slot], drawn again here), then the geometry.
// grid (groups, ceil(J_max/256)) (or transposed).
template <typename T, int PROP>
__global__ __launch_bounds__(256) void k_birth_weight(DevModel m, const Grp* __restrict__ gd, SoA<T> st, Geo geo,
                                                      const int* __restrict__ nsurv, const int* __restrict__ ncur,
                                                      const int* __restrict__ borig, const double* __restrict__ Zall,
                                                      const double* __restrict__ taball, int Mall,
                                                      const ZWin* __restrict__ win, uint32_t step_arg,
                                                      const uint32_t* __restrict__ dstep)
{
    const int j = slot_group(m);
    const Grp gr = gd[j];
    const int ns = nsurv[j], nb = ncur[j] - ns;
    if (slot_tile(m) * 256 >= nb) return;  // whole workgroup idle
    const int b = slot_tile(m) * 256 + threadIdx.x;
    const bool active = b < nb;
    if (__ballot(active) == 0) return;     // whole wavefront idle
    const uint32_t step = step_of(step_arg, dstep);
    const BirthSrc src = birth_src(gr, win, Zall, taball, Mall);
    const size_t g = (size_t)j * m.cap + ns + (active ? b : 0);
    const int o = active ? borig[g] : 0;
    double x[4];
    draw_proposal_birth<PROP>(m, (uint32_t)(gr.jl * m.cap + ns + o), step, gr.rng_run, src, x);
    const double w = birth_weight_at<T, PROP>(m, src, gr.Jj, x, active);
    if (!active) return;
    const T tw = (T)w;
    st.w[g] = tw;
    // the stored position is the drawn one at storage precision
    store_geometry<T>(m, geo, g, (double)(T)x[0], (double)(T)x[2], (double)tw);
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

// Bearing frames.  With kappa > 0 the passes skip the modulo-2 pi wrap: a
// measurement with |theta| <= pi/2 is compared with the particle bearings as
// they are (frame A), any other with both turned by pi (frame B, where its
// bearing is within pi/2 of zero).  In either frame a pair whose residual
// would need wrapping is more than pi/2 apart in bearing, i.e. > 78 sigma_theta
// for the workloads here, so its term underflows to exactly 0 with or without
// the wrap.  kappa = 0 (EXACT) keeps the wrap, since there every C matters.
struct ZFrame {
    double zr, zt;
    bool b;
};
__device__ __forceinline__ ZFrame z_frame(const DevModel& m, double r, double th)
{
    ZFrame f;
    f.zr = r * m.cr;
    f.b = fabs(th) > 0.5 * 3.14159265358979323846;
    f.zt = (f.b ? (th < 0.0 ? th + 3.14159265358979323846 : th - 3.14159265358979323846) : th) * m.ct;
    return f;
}
// scaled squared residual in a frame, + c
__device__ __forceinline__ double sq_resid_nowrap(double zr, double zt, double rho, double phi, double c)
{
    const double dr = zr - rho, dt = zt - phi;
    return fma(dr, dr, fma(dt, dt, c));
}

// Work split of the two likelihood passes: group j's slots are cut into wave
// tiles of WT = 64*PT particles (lane l takes slots base + 64 i + l) and its
// M measurements into zsplit = clamp(ceil(M/mz), 1, ZSPLIT_MAX) chunks of
// MZ = ceil(M/zsplit); one wavefront takes one (tile, chunk) pair, chunks of a
// tile sitting in the same workgroup.  The chunking follows from M alone, so
// a run splits its measurements the same way alone or in a batch.
constexpr int ZSPLIT_MAX = 16;
struct Split {
    int wtiles, mz;
};
__device__ __forceinline__ int zsplit_for(int M, int mz)
{
    const int z = (M + mz - 1) / mz;
    return z < 1 ? 1 : (z > ZSPLIT_MAX ? ZSPLIT_MAX : z);
}

// ---------------------------------------------------------------------------
// Step 2, first pass (Eq 11): C_j(z) for every group and measurement.
// Per wave and measurement the wave returns the scaled partial sum
//   s = sum_i 2^(-q_i + lw_i - h),   C = 2^h s  (h an integer shift),
// written to ps[(j*wtiles + tile)*Mmax + p] with its shift at the same index
// of ph (one shift per (tile, measurement)); pw[j*wtiles + tile] holds the
// tile's sum of weights.  The bearing-frame pass (k_cz_frames) has one shift
// per tile and writes it only at column 0 of the tile's row of ph.
// EXACT = false (kappa > 0): h = ceil(max_i lw_i) of the wave, a bound that
//   needs no per-pair work; a term lost to float underflow is below
//   2^-126 w_i, far under the 1e-5 kappa tolerance of C.
// EXACT = true (kappa = 0, where every C matters): h = ceil(max_i exponent)
//   per measurement (log-sum-exp scaling), so the largest term is >= 1/2.
// Exponents stay in double until the shift is removed: far from every
// particle they reach -1e3, where a float has lost 1e-4.
// grid (ceil(wtiles*zsplit/4), K), 256 threads.
// ---------------------------------------------------------------------------
enum : int { PASS_FRAMES = 0, PASS_WRAP = 1, PASS_EXACT = 2 };

template <typename T, int PT, int MODE>
__global__ __launch_bounds__(256) void k_cz(DevModel m, const Grp* __restrict__ gd, Geo geo, const T* __restrict__ W,
                                            const int* __restrict__ ncur, const double* __restrict__ Zall, int Mall,
                                            const ZWin* __restrict__ win, int Mmax, Split sp,
                                            double* __restrict__ ps, int* __restrict__ ph, double* __restrict__ pw)
{
    constexpr int WT = 64 * PT;
    constexpr bool EXACT = MODE == PASS_EXACT, FRAMES = MODE == PASS_FRAMES;
    const int j = blockIdx.y;
    const ZView zv = zview(gd[j], win, Zall, Mall);
    const double* Z = zv.Z;
    const int M = zv.M;
    const int zsplit = zsplit_for(M, sp.mz), MZ = (M + zsplit - 1) / zsplit;
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + wave_in_block();
    const int tile = gw / zsplit, zc = gw - tile * zsplit;
    const int n = ncur[j];
    const int base = tile * WT;
    if (tile >= sp.wtiles || base >= n) return;
    const size_t gb = (size_t)j * m.cap;
    double rho[PT], phi[PT], phib[PT], nlw[PT];
    double lwmax = -__builtin_inf();
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        // unconditional loads (lanes past the group's end read its slot base
        // and drop the value), so all of them are in flight at once
        const bool ok = s < n;
        const size_t g = gb + (ok ? s : base);
        const double r = geo.rho[g], a = geo.phi[g], b = FRAMES ? geo.phib[g] : 0.0, lw = geo.lw[g];
        rho[i] = ok ? r : 0.0;
        phi[i] = ok ? a : 0.0;
        phib[i] = ok ? b : 0.0;
        nlw[i] = ok ? -lw : __builtin_inf();
        lwmax = ok && lw > lwmax ? lw : lwmax;
    }
    if (zc == 0) {
        double ws = 0.0;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int s = base + i * 64 + lane;
            const double wv = (double)W[gb + (s < n ? s : base)];
            ws += s < n ? wv : 0.0;
        }
        ws = wave_sum(ws);
        if (lane == 0) pw[(size_t)j * sp.wtiles + tile] = ws;
    }
    double hw = 0.0;
    if (!EXACT) {
        const double wmx = wave_max(lwmax);
        hw = (wmx == -__builtin_inf()) ? 0.0 : ceil(wmx);
#pragma unroll
        for (int i = 0; i < PT; ++i) nlw[i] += hw;  // exponent - h folded into the particle term
    }
    const size_t pbase = ((size_t)j * sp.wtiles + tile) * Mmax;
    const int p0 = zc * MZ, p1 = (p0 + MZ < M) ? p0 + MZ : M;
    // measurements of the chunk, 64 at a time: lane l holds measurement pb + l,
    // each iteration broadcasts one with v_readlane (no memory latency in the loop)
    for (int pb = p0; pb < p1; pb += 64) {
        const int pe = (pb + 64 < p1) ? pb + 64 : p1;
        double lzr = 0.0, lzt = 0.0;
        int lfb = 0;
        if (pb + lane < pe) {
            const int q = pb + lane;
            if (FRAMES) {
                const ZFrame zf = z_frame(m, Z[2 * q], Z[2 * q + 1]);
                lzr = zf.zr;
                lzt = zf.zt;
                lfb = zf.b ? 1 : 0;
            } else {
                lzr = Z[2 * q] * m.cr;
                lzt = Z[2 * q + 1] * m.ct;
            }
        }
        for (int p = pb; p < pe; ++p) {
            const double zr = lane_value(lzr, p - pb), zt = lane_value(lzt, p - pb);
            T s = 0;
            double h = hw;
            if (EXACT) {
                double a[PT];
                double amax = -__builtin_inf();
#pragma unroll
                for (int i = 0; i < PT; ++i) {
                    a[i] = -sq_resid(m, zr, zt, rho[i], phi[i], nlw[i]);
                    amax = a[i] > amax ? a[i] : amax;
                }
                const float wmx = wave_max((float)amax);
                h = (wmx == -__builtin_inff()) ? 0.0 : (double)ceilf(wmx);
#pragma unroll
                for (int i = 0; i < PT; ++i) s += fast_exp2((T)(a[i] - h));
            } else if (FRAMES) {
                if (lane_value(lfb, p - pb)) {
#pragma unroll
                    for (int i = 0; i < PT; ++i) s += fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], phib[i], nlw[i]));
                } else {
#pragma unroll
                    for (int i = 0; i < PT; ++i) s += fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], phi[i], nlw[i]));
                }
            } else {
#pragma unroll
                for (int i = 0; i < PT; ++i) s += fast_exp2(-(T)sq_resid(m, zr, zt, rho[i], phi[i], nlw[i]));
            }
            const T sw = wave_sum(s);
            if (lane == 0) {
                ps[pbase + p] = (double)sw;
                ph[pbase + p] = (int)h;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Bearing-frame passes (kappa > 0, PASS_FRAMES), measurement side prepared
// once per update by k_zprep: each run's measurements are scaled (r c_r and
// the frame's bearing times c_t) and stably reordered so that frame A
// (|theta| <= pi/2) comes first.  The passes walk that order with scalar
// (wave-uniform) loads, one select-free loop per frame, and map each entry
// back to its original index for every per-measurement output.
// ---------------------------------------------------------------------------
struct ZPrep {
    double* zs;   // [rows][2]: scaled range, scaled frame bearing, in frame order per run
    int* orig;    // [rows]: original index of the entry within its run
    int* pos;     // [rows]: frame-order position of original measurement p (the inverse)
    int* rec;     // [runs][4]: window offset, measurement count, entries of frame A, 0
};
struct ZPrepC {
    const double* zs;
    const int* orig;
    const int* pos;
    const int* rec;
};
// per-group measurement results of the first pass again in frame order, for
// the second pass (H, F and the candidate flag of k_cz_combine)
template <typename T>
struct ZSorted {
    int* H;
    T* F;
    int* flag;
};

// one workgroup per run.  grid (runs), 256 threads.
template <int NT>
__device__ __forceinline__ void zprep_run(const DevModel& m, const double* __restrict__ Zall, int Mall,
                                          const ZWin* __restrict__ win, const ZPrep& zp, int run)
{
    constexpr int NW = NT / 64;
    __shared__ int s_cnt[NW];
    __shared__ int s_base;
    int off = 0, M = Mall;
    if (win) {
        off = win[run].off;
        M = win[run].M;
    }
    const double* Z = Zall + 2 * (size_t)off;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // pass 1: number of frame-A measurements
    int cA = 0;
    for (int p = threadIdx.x; p < M; p += NT) cA += fabs(Z[2 * p + 1]) > 0.5 * 3.14159265358979323846 ? 0 : 1;
    cA = (int)wave_sum((double)cA);
    if (lane == 0) s_cnt[wv] = cA;
    __syncthreads();
    int nA = 0;
    for (int w2 = 0; w2 < NW; ++w2) nA += s_cnt[w2];
    if (threadIdx.x == 0) {
        // the record the likelihood passes read in one scalar load
        *reinterpret_cast<int4*>(zp.rec + 4 * run) = make_int4(off, M, nA, 0);
        s_base = 0;
    }
    // pass 2: stable positions, NT measurements at a time
    for (int p0 = 0; p0 < M; p0 += NT) {
        __syncthreads();
        const int p = p0 + threadIdx.x;
        const bool valid = p < M;
        ZFrame zf{ 0.0, 0.0, false };
        if (valid) zf = z_frame(m, Z[2 * p], Z[2 * p + 1]);
        const int isA = valid && !zf.b ? 1 : 0;
        const int incl = (int)wave_incl_scan((double)isA);
        if (lane == 63) s_cnt[wv] = incl;
        __syncthreads();
        int before = s_base;
        for (int w2 = 0; w2 < wv; ++w2) before += s_cnt[w2];
        const int exA = before + incl - isA;  // frame-A entries before p in the run
        if (valid) {
            const int pos = isA ? exA : nA + (p - exA);
            zp.zs[2 * ((size_t)off + pos)] = zf.zr;
            zp.zs[2 * ((size_t)off + pos) + 1] = zf.zt;
            zp.orig[(size_t)off + pos] = p;
            zp.pos[(size_t)off + p] = pos;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w2 = 0; w2 < NW; ++w2) s_base += s_cnt[w2];
    }
}
__global__ __launch_bounds__(256) void k_zprep(DevModel m, const double* __restrict__ Zall, int Mall,
                                               const ZWin* __restrict__ win, ZPrep zp)
{
    zprep_run<256>(m, Zall, Mall, win, zp, blockIdx.x);
}

// 64-lane sum left in lane 63 (other lanes hold partial sums): quad and row
// swizzles, then the row broadcasts 15 and 31 fold rows 0-2 into row 3.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ float wave_sum_last(float v)
{
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    v += dpp_rows<0x142, 0xA>(v);
    v += dpp_rows<0x143, 0xC>(v);
    return v;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
// In lane 63 the same value as wave_sum: every lane of a row holds the same
// row sum R_r after the swizzles, and (R3 + R2) + (R1 + R0) equals
// (R0 + R1) + (R2 + R3) exactly (each addition commutes).
__device__ __forceinline__ double wave_sum_last(double v)
{
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    v += dpp_rows<0x142, 0xA>(v);
    v += dpp_rows<0x143, 0xC>(v);
    return v;
}

// Tile culling.  A term 2^-e with e above exp2_cut<T>() is exactly zero in T
// (2^-150 rounds to zero in float, 2^-1075 in double; the cuts leave a wide
// margin for the rounding of the bound itself).  Every exponent of a tile is
// at least the squared distance of the scaled measurement from the tile's
// box [rho_lo, rho_hi] x [ang_lo, ang_hi] (plus the pass's shift), so a
// measurement whose bound exceeds the cut contributes exactly zero to every
// sum of the tile and is skipped; each lane tests one measurement and a
// ballot leaves the ones to evaluate.  Results are bit-identical to the full
// evaluation: the skipped terms are +0 and every sum starts at +0.
template <typename T>
__device__ __forceinline__ constexpr double exp2_cut();
template <>
__device__ __forceinline__ constexpr double exp2_cut<float>() { return 200.0; }
template <>
__device__ __forceinline__ constexpr double exp2_cut<double>() { return 1100.0; }

// Bounds of a wave tile's scaled range and two frame bearings, in float.
// Float rounding moves the bound by far less than the cut's margin over the
// underflow point (50 in float, 25 in double, against errors below 1e-2 at
// these scales), so a measurement whose bound passes the cut still has
// exactly zero terms.
struct TileBox {
    float rlo, rhi, alo, ahi, blo, bhi;
};
// the 64-lane maximum in every lane: quad and row swizzles, the row
// broadcasts (rows left out take -inf), then lane 63's value
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows_max(float v)
{
    const int ninf = __builtin_bit_cast(int, -__builtin_inff());
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(ninf, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ float wave_max_f(float v)
{
    v = fmaxf(v, dpp<0xB1>(v));
    v = fmaxf(v, dpp<0x4E>(v));
    v = fmaxf(v, dpp<0x141>(v));
    v = fmaxf(v, dpp<0x140>(v));
    v = fmaxf(v, dpp_rows_max<0x142, 0xA>(v));
    v = fmaxf(v, dpp_rows_max<0x143, 0xC>(v));
    return lane_value(v, 63);
}
__device__ __forceinline__ float wave_min_f(float v) { return -wave_max_f(-v); }
template <int PT>
__device__ __forceinline__ TileBox tile_box(const double* rho, const double* phi, const double* phib, int base, int n,
                                            int lane)
{
    const float inf = __builtin_inff();
    float rlo = inf, rhi = -inf, alo = inf, ahi = -inf, blo = inf, bhi = -inf;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        if (base + i * 64 + lane < n) {
            const float r = (float)rho[i], a = (float)phi[i], c = (float)phib[i];
            rlo = fminf(rlo, r);
            rhi = fmaxf(rhi, r);
            alo = fminf(alo, a);
            ahi = fmaxf(ahi, a);
            blo = fminf(blo, c);
            bhi = fmaxf(bhi, c);
        }
    }
    return TileBox{ wave_min_f(rlo), wave_max_f(rhi), wave_min_f(alo), wave_max_f(ahi), wave_min_f(blo), wave_max_f(bhi) };
}
// the measurement's terms in the tile can reach 2^-cut: squared distance
// from the box in the measurement's frame, plus the pass's shift
__device__ __forceinline__ bool box_needed(const TileBox& b, bool frame_b, float zr, float zt, float shift, float cut)
{
    const float lo = frame_b ? b.blo : b.alo, hi = frame_b ? b.bhi : b.ahi;
    const float dr = fmaxf(0.0f, fmaxf(b.rlo - zr, zr - b.rhi));
    const float dt = fmaxf(0.0f, fmaxf(lo - zt, zt - hi));
    return fmaf(dr, dr, fmaf(dt, dt, shift)) <= cut;
}

// ---------------------------------------------------------------------------
// Work items of the frame passes.  Group j's wave tiles (WT slots each) are
// its work items, numbered in slot order.  With groups of one size the grid
// is (groups, X), X fixed by the group count, and the 4X wavefronts of group
// j take its items w, w + 4X, ... (the workgroups of low X, which hold most of
// the work, are dispatched first).  With groups of different sizes (a batch
// of unlike runs) the items of all groups form one list (pre[j]: group j's
// first item, pre[K]: all items, grp[e]: the group of item e) that a 1-D grid
// strides over, so every wavefront gets about the same number of items.
// Either way the grid does not follow the particle counts (it can be
// captured in a graph) and a wavefront never holds an empty tile.  When
// a group has few births (under 16 tiles' worth: their bearing order then
// still leaves each birth tile spread over many buckets, keeping most
// measurements), each tile holding births is BIRTH_CHUNKS items, each with
// a contiguous part of the measurements: item e is tile e for e < tA_j (the
// tiles before the first birth) and else tile tA_j + (e - tA_j) / chunks,
// chunk (e - tA_j) mod chunks.
// ---------------------------------------------------------------------------
constexpr int BIRTH_CHUNKS = 4;
struct TileItem {
    int tile, chunk, chunks;
};
// (clamped to [0, tiles]: a state written from the host may leave any
// survivor count, and the item count must stay within BIRTH_CHUNKS per tile)
__device__ __forceinline__ int tiles_before_births(int n, int ns, int WT)
{
    const int nt = (n + WT - 1) / WT, ta = ns > 0 ? ns / WT : 0;
    return ta < nt ? ta : nt;
}
__device__ __forceinline__ int birth_chunks(int n, int ns, int WT)
{
    return n - (ns > 0 ? ns : 0) < 16 * WT ? BIRTH_CHUNKS : 1;
}
__device__ __forceinline__ int tile_items(int n, int ns, int WT)
{
    const int nt = (n + WT - 1) / WT, ta = tiles_before_births(n, ns, WT);
    return ta + (nt - ta) * birth_chunks(n, ns, WT);
}
// a group's span in the flat list: its items rounded up to a multiple of 4,
// so that the four chunks of a birth tile (items 4q .. 4q + 3 of the group)
// fall to the four wavefronts of one workgroup; the padding items are empty
__device__ __forceinline__ int list_items(int n, int ns, int WT) { return (tile_items(n, ns, WT) + 3) & ~3; }
// item e of a group, counted from its last item: the birth tiles (the
// heaviest items) go to the first wavefronts
__device__ __forceinline__ TileItem tile_item(int e, int n, int ns, int WT)
{
    const int ta = tiles_before_births(n, ns, WT), z = birth_chunks(n, ns, WT);
    e = tile_items(n, ns, WT) - 1 - e;
    if (e < ta) return TileItem{ e, 0, 1 };
    return TileItem{ ta + (e - ta) / z, (e - ta) % z, z };
}
// Heavy tiles of the second pass.  A survivors' tile whose first-pass
// wavefront kept at least HEAVY_KEPT measurements is taken by the second
// pass as BIRTH_CHUNKS items too (measurement chunks in one workgroup, their
// sums meeting in LDS), so that a few tiles spanning many measurements do
// not set the pass's length.  The first pass records each survivors' tile's
// kept count; k_cz_combine then writes each group's item table for the
// second pass (tile | chunk << 20 | chunked << 23): the chunked tiles first
// (births', then heavy survivors' tiles, whole 4-item spans), the others
// after.  Which tiles are heavy follows from the first pass's results alone,
// so a run splits the same way alone or in a batch.
constexpr int HEAVY_KEPT = 16;
__device__ __forceinline__ TileItem item_decode(int v)
{
    const int chunked = (v >> 23) & 1;
    return TileItem{ v & 0xFFFFF, chunked ? (v >> 20) & 3 : 0, chunked ? BIRTH_CHUNKS : 1 };
}
// group j's item table (one 1024-thread workgroup; contains barriers)
__device__ void build_items(int j, int n, int ns, int WT, const int* __restrict__ tkept, int wtiles,
                            int* __restrict__ items, int imax, int* __restrict__ nitems)
{
    constexpr int HMAX = 4096;  // survivors' tiles a table can split (beyond: none split)
    __shared__ int s_nh;
    __shared__ unsigned char s_heavy[HMAX];
    const int nt = (n + WT - 1) / WT, ta = tiles_before_births(n, ns, WT), z = birth_chunks(n, ns, WT);
    const int nbc = z > 1 ? nt - ta : 0;  // chunked birth tiles
    int* it = items + (size_t)j * imax;
    const int lane = threadIdx.x & 63;
    const int tah = ta <= HMAX ? ta : 0;
    for (int t = threadIdx.x; t < tah; t += 1024) s_heavy[t] = tkept[(size_t)j * wtiles + t] >= HEAVY_KEPT ? 1 : 0;
    __syncthreads();
    auto heavy = [&](int t) { return t < tah && s_heavy[t] != 0; };
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    // wavefront 0 places the heavy survivors' tiles (4 items each, after the
    // births' chunked tiles), 64 at a time
    if (threadIdx.x < 64) {
        int nh = 0;
        for (int t0 = 0; t0 < ta; t0 += 64) {
            const int t = t0 + lane;
            const bool hv = t < ta && heavy(t);
            const unsigned long long bh = __ballot(hv);
            if (hv) {
                const int pos = 4 * (nbc + nh + __popcll(bh & below));
#pragma unroll
                for (int c = 0; c < 4; ++c) it[pos + c] = t | (c << 20) | (1 << 23);
            }
            nh += __popcll(bh);
        }
        if (lane == 0) s_nh = nh;
    }
    __syncthreads();
    // the births' tiles: chunked first, or light at the end
    for (int e = threadIdx.x; e < 4 * nbc; e += 1024) it[e] = (ta + e / 4) | ((e % 4) << 20) | (1 << 23);
    const int lbase = 4 * (nbc + s_nh);
    if (threadIdx.x < 64) {
        int nl = 0;
        for (int t0 = 0; t0 < ta; t0 += 64) {
            const int t = t0 + lane;
            const bool light = t < ta && !heavy(t);
            const unsigned long long bl = __ballot(light);
            if (light) it[lbase + nl + __popcll(bl & below)] = t;
            nl += __popcll(bl);
        }
        const int nbl = z > 1 ? 0 : nt - ta;
        for (int b = lane; b < nbl; b += 64) it[lbase + nl + b] = ta + b;
        if (lane == 0) nitems[j] = lbase + nl + nbl;
    }
}

// the flat list: item counts and their prefix (one workgroup of 1024 threads,
// thread i taking a contiguous run of ceil(K/1024) groups; cnt: the groups'
// item tables' counts, else the counts the sizes give) ...
__global__ __launch_bounds__(1024) void k_items_scan(const int* __restrict__ ncur, const int* __restrict__ nsurv,
                                                     int K, int WT, int* __restrict__ pre,
                                                     const int* __restrict__ cnt)
{
    __shared__ int s_w[16];
    const int G = (K + 1023) / 1024;
    const int j0 = threadIdx.x * G < K ? threadIdx.x * G : K, j1 = j0 + G < K ? j0 + G : K;
    auto items_of = [&](int j) { return cnt ? (cnt[j] + 3) & ~3 : list_items(ncur[j], nsurv[j], WT); };
    int c = 0;
    for (int j = j0; j < j1; ++j) c += items_of(j);
    const int incl = (int)wave_incl_scan((double)c);  // exact: counts stay below 2^53
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) s_w[wv] = incl;
    __syncthreads();
    int pos = incl - c;
    for (int w = 0; w < wv; ++w) pos += s_w[w];
    for (int j = j0; j < j1; ++j) {
        pre[j] = pos;
        pos += items_of(j);
    }
    if (threadIdx.x == 1023) pre[K] = pos;
}
// ... and every group's entries of grp (grid (K), 256 threads)
__global__ __launch_bounds__(256) void k_items_fill(const int* __restrict__ pre, int* __restrict__ grp)
{
    const int j = blockIdx.x;
    for (int e = pre[j] + threadIdx.x; e < pre[j + 1]; e += 256) grp[e] = j;
}

// the run of a work item's group: read per item from the flat lists, else the
// workgroup's group's run read once at the start, or 0 without a read when
// the filter is one run (the measurement record's read then starts at once
// instead of after the group's); the empty asm keeps the per-item read
// behind its branch, so it is not made for every item
__device__ __forceinline__ int item_run(const Grp* __restrict__ gd, bool flat, int j, int run0)
{
    if (!flat) return run0;
    int jj = j;
    __asm__ volatile("" : "+s"(jj));
    return gd[jj].run;
}
// the particle count and survivor count of a work item's group, the same way
__device__ __forceinline__ int2 item_sizes(const int* __restrict__ ncur, const int* __restrict__ nsurv, bool flat,
                                           int j, int2 s0)
{
    if (!flat) return s0;
    int jj = j;
    __asm__ volatile("" : "+s"(jj));
    return make_int2(ncur[jj], nsurv[jj]);
}

// first pass in frames: as k_cz (PASS_FRAMES), the measurement side read
// from the prepared order, tiles culled; tile `tile` of group j, every
// measurement of the run in one wavefront
template <typename T, int PT>
__device__ __forceinline__ void cz_frames_tile(const DevModel& m, const Grp* __restrict__ gd, const Geo& geo,
                                               const T* __restrict__ W, int n, int Mall,
                                               const ZWin* __restrict__ win, const ZPrepC& zp, int Mmax,
                                               const Split& sp, double* __restrict__ ps, int* __restrict__ ph,
                                               double* __restrict__ pw, const int* __restrict__ zrec, int j,
                                               int zrun, int tile, int zc, int zsplit, int* __restrict__ tkept)
{
    constexpr int WT = 64 * PT;
    const int lane = threadIdx.x & 63;
    const int base = tile * WT;
    if (base >= n) return;
    const size_t gb = (size_t)j * m.cap;
    double rho[PT], phi[PT], phib[PT], nlw[PT];
    double lwmax = -__builtin_inf();
    // the particles first: they need only the group's size, so they are in
    // flight while the run's measurement window is looked up
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        // unconditional loads (lanes past the group's end read its slot base
        // and drop the value), so all of them are in flight at once
        const bool ok = s < n;
        const size_t g = gb + (ok ? s : base);
        const double r = geo.rho[g], a = geo.phi[g], b = geo.phib[g], lw = geo.lw[g];
        rho[i] = ok ? r : 0.0;
        phi[i] = ok ? a : 0.0;
        phib[i] = ok ? b : 0.0;
        nlw[i] = ok ? -lw : __builtin_inf();
        lwmax = ok && lw > lwmax ? lw : lwmax;
    }
    // the run's frame split and window, read together
    // the run's window and frame split (one record)
    const int4 zr4 = *reinterpret_cast<const int4*>(zrec + 4 * zrun);
    const int off = zr4.x, M = zr4.y, nA = zr4.z;
    const int MZ = (M + zsplit - 1) / zsplit;
    const int p0 = zc * MZ < M ? zc * MZ : M, p1 = p0 + MZ < M ? p0 + MZ : M;
    const double* zs = zp.zs + 2 * (size_t)off;
    // the first 64 measurements of each frame in [p0, p1)
    const int a1 = p1 < nA ? p1 : nA, b0 = p0 > nA ? p0 : nA;
    const int qa = p0 + lane < a1 ? p0 + lane : 0, qb = b0 + lane < p1 ? b0 + lane : 0;
    const double zra0 = M > 0 ? zs[2 * qa] : 0.0, zta0 = M > 0 ? zs[2 * qa + 1] : 0.0;
    const double zrb0 = M > 0 ? zs[2 * qb] : 0.0, ztb0 = M > 0 ? zs[2 * qb + 1] : 0.0;
    if (zc == 0) {
        double ws = 0.0;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int s = base + i * 64 + lane;
            const double wv = (double)W[gb + (s < n ? s : base)];
            ws += s < n ? wv : 0.0;
        }
        ws = wave_sum(ws);
        if (lane == 0) pw[(size_t)j * sp.wtiles + tile] = ws;
    }
    const double wmx = wave_max(lwmax);
    const double hw = (wmx == -__builtin_inf()) ? 0.0 : ceil(wmx);
#pragma unroll
    for (int i = 0; i < PT; ++i) nlw[i] += hw;
    const size_t pbase = ((size_t)j * sp.wtiles + tile) * Mmax;
    // every partial of the tile has the exponent hw: stored once, in the
    // first column of the tile's row
    if (zc == 0 && lane == 0) ph[pbase] = (int)hw;
    const TileBox bx = tile_box<PT>(rho, phi, phib, base, n, lane);
    auto one = [&](int p, double zr, double zt, const double* ang) {
        T s = 0;
#pragma unroll
        for (int i = 0; i < PT; ++i) s += fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], ang[i], nlw[i]));
        const T sw = wave_sum_last(s);
        if (lane == 63) ps[pbase + p] = (double)sw;  // frame order; k_cz_combine maps back
    };
    // two measurements at once: independent chains for the latency-bound
    // tiles that keep many of them
    auto two = [&](int p, double zr, double zt, int q, double yr, double yt, const double* ang) {
        T s = 0, t = 0;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            s += fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], ang[i], nlw[i]));
            t += fast_exp2(-(T)sq_resid_nowrap(yr, yt, rho[i], ang[i], nlw[i]));
        }
        const T sw = wave_sum_last(s), tw = wave_sum_last(t);
        if (lane == 63) {
            ps[pbase + p] = (double)sw;
            ps[pbase + q] = (double)tw;
        }
    };
    // every nlw is >= 0 (hw is the ceiling of the tile's largest log weight).
    // Lane l tests measurement c0 + l; the ones left are read from their lane.
    int kept = 0;  // measurements this wavefront keeps (the whole tile's when zsplit = 1)
    auto frame = [&](int pa, int pb, const double* ang, bool fb, double zr0, double zt0) {
        for (int c0 = pa; c0 < pb; c0 += 64) {
            const int p = c0 + lane;
            bool need = false;
            double zr = 0.0, zt = 0.0;
            if (p < pb) {
                zr = c0 == pa ? zr0 : zs[2 * p];
                zt = c0 == pa ? zt0 : zs[2 * p + 1];
                need = box_needed(bx, fb, (float)zr, (float)zt, 0.0f, (float)exp2_cut<T>());
                if (!need) ps[pbase + p] = 0.0;
            }
            uint64_t live = __ballot(need);
            kept += __popcll(live);
            while (live) {
                const int l = __builtin_ctzll(live);
                live &= live - 1;
                if (live) {
                    const int l2 = __builtin_ctzll(live);
                    live &= live - 1;
                    two(c0 + l, lane_value(zr, l), lane_value(zt, l), c0 + l2, lane_value(zr, l2),
                        lane_value(zt, l2), ang);
                } else {
                    one(c0 + l, lane_value(zr, l), lane_value(zt, l), ang);
                }
            }
        }
    };
    frame(p0, a1, phi, false, zra0, zta0);
    frame(b0, p1, phib, true, zrb0, ztb0);
    if (tkept && zsplit == 1 && lane == 0) tkept[(size_t)j * sp.wtiles + tile] = kept;
}

template <typename T, int PT>
__global__ __launch_bounds__(256) void k_cz_frames(DevModel m, const Grp* __restrict__ gd, Geo geo,
                                                   const T* __restrict__ W, const int* __restrict__ ncur,
                                                   int Mall, const ZWin* __restrict__ win, ZPrepC zp, int Mmax,
                                                   Split sp, double* __restrict__ ps, int* __restrict__ ph,
                                                   double* __restrict__ pw, const int* __restrict__ nsurv, int K,
                                                   const int* __restrict__ tpre, const int* __restrict__ tgrp,
                                                   const int* __restrict__ zrec, int* __restrict__ tkept)
{
    // per group (tpre null, grid (K, X)) or over the flat list (grid (X))
    const bool flat = tpre != nullptr;
    const int w0 = (flat ? blockIdx.x : blockIdx.y) * 4 + wave_in_block();
    const int stride = (flat ? gridDim.x : gridDim.y) * 4;
    // the group's sizes and run, read once (kept apart from the per-item reads
    // of the flat lists, so they are not read again per item)
    int2 s0 = flat ? make_int2(0, 0) : make_int2(ncur[blockIdx.x], nsurv[blockIdx.x]);
    int run0 = flat || m.one_run ? 0 : gd[blockIdx.x].run;
    __asm__ volatile("" : "+s"(run0), "+s"(s0.x), "+s"(s0.y));
    const int end = flat ? tpre[K] : tile_items(s0.x, s0.y, 64 * PT);
    for (int e = w0; e < end; e += stride) {
        const int j = flat ? tgrp[e] : (int)blockIdx.x;
        const int le = flat ? e - tpre[j] : e;
        const int2 sz = item_sizes(ncur, nsurv, flat, j, s0);
        if (le >= tile_items(sz.x, sz.y, 64 * PT)) continue;  // a list's padding
        const TileItem it = tile_item(le, sz.x, sz.y, 64 * PT);
        cz_frames_tile<T, PT>(m, gd, geo, W, sz.x, Mall, win, zp, Mmax, sp, ps, ph, pw, zrec, j,
                              item_run(gd, flat && !m.one_run, j, run0), it.tile, it.chunk, it.chunks, tkept);
    }
}

// The second pass finalizes its tiles (wave tiles of 256k slots): the new
// weights, the parents' bearing buckets, and per 256-slot tile the bucket
// histogram and the weight sum and maximum, each formed exactly as k_wfinal
// forms them (the same sums in the same order).  A birth tile split into
// chunks is finalized by its chunk-0 wavefront once the workgroup's four
// chunk sums are in LDS, so k_wfinal is not needed.
template <typename T>
struct WFin {
    int on;        // finalize the tiles here
    T* W;          // weights, replaced in place
    int* bkt;      // bearing bucket of every slot
    int* bhist;    // per 256-slot tile bucket counts
    double* pmass; // per 256-slot tile weight sum
    double* pmax;  // per 256-slot tile weight maximum
    int tiles256;  // 256-slot tiles per group
};
template <typename T, int PT>
__device__ __forceinline__ void finalize_tile(const DevModel& m, const WFin<T>& fin, const T* wv, const T* xa,
                                              const T* xb, const T* acc, int j, int tile, int base, int n, int lane)
{
    static_assert(PT % 4 == 0, "wave tiles of 256k slots");
    __shared__ int hfin[4][BEARING_BUCKETS];
    int* h = hfin[wave_in_block()];
    const size_t gb = (size_t)j * m.cap;
    T* Wj = fin.W + gb;
#pragma unroll
    for (int k = 0; k < PT / 4; ++k) {
        const int t256 = tile * (PT / 4) + k;
        if (t256 * 256 >= n) break;
        h[lane] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        double wn[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int i = 4 * k + w;
            const int s = base + i * 64 + lane;
            wn[w] = 0.0;
            if (s < n) {
                const double wo = (double)wv[i];
                const T t = (T)(m.nu * wo + m.wscale * wo * (double)acc[i]);
                Wj[s] = t;
                wn[w] = (double)t;
                const int b = bearing_bucket(m, (double)xa[i], (double)xb[i]);
                fin.bkt[gb + s] = b;
                atomicAdd(&h[b], 1);
            }
        }
        // the 256-slot tile's sum and maximum in k_wfinal's order: the four
        // slots of a lane first, then one wavefront reduction each
        const double ts = wave_sum_last((wn[0] + wn[1]) + (wn[2] + wn[3]));
        const double tm = wave_max(vmax(vmax(wn[0], wn[1]), vmax(wn[2], wn[3])));
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int hv = h[lane];
        const size_t o = (size_t)j * fin.tiles256 + t256;
        if (lane == 63) {
            fin.pmass[o] = ts;
            fin.pmax[o] = tm;
        }
        fin.bhist[o * BEARING_BUCKETS + lane] = hv;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// second pass in frames: as k_weight<T, PT, true>, the measurement side read
// from the prepared order, tiles culled; tile `tile` of group j, every
// measurement of the run in one wavefront
template <typename T, int PT>
__device__ __forceinline__ void weight_frames_tile(const DevModel& m, const Grp* __restrict__ gd, const SoA<T>& st,
                                                   const Geo& geo, int n, int Mall,
                                                   const ZWin* __restrict__ win, const ZPrepC& zp, int Mmax,
                                                   const Split& sp, const int* __restrict__ zHs,
                                                   const T* __restrict__ zFs, const int* __restrict__ zfls,
                                                   double* __restrict__ pzeta, T* __restrict__ accp,
                                                   const int* __restrict__ zrec, int j, int zrun, int tile, int zc,
                                                   int zsplit, const WFin<T>& fin, int& quads)
{
    constexpr int WT = 64 * PT;
    const int lane = threadIdx.x & 63;
    const int base = tile * WT;
    if (base >= n) return;
    const size_t gb = (size_t)j * m.cap;
    // the group's arrays (wave-uniform bases, slot offsets below 2^32 bytes)
    const double *grho = geo.rho + gb, *gphi = geo.phi + gb, *gphib = geo.phib + gb;
    const T *gw = st.w + gb, *gx0 = st.x[0] + gb, *gx1 = st.x[1] + gb, *gx2 = st.x[2] + gb, *gx3 = st.x[3] + gb;
    double rho[PT], phi[PT], phib[PT];
    T acc[PT];
    // the geometry, the weight and the position (the finalization and the
    // candidates' sums use them; the velocities are read by candidates),
    // issued before the run's measurement window is looked up: they need only
    // the group's size, so they are in flight during those reads
    T wv[PT], xa[PT], xb[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        // unconditional loads, values of lanes past the group's end dropped
        const bool ok = s < n;
        const uint32_t g = ok ? s : base;
        const double r = ld_slot(grho, g), a = ld_slot(gphi, g), b = ld_slot(gphib, g);
        wv[i] = ld_slot(gw, g);
        xa[i] = ld_slot(gx0, g);
        xb[i] = ld_slot(gx2, g);
        rho[i] = ok ? r : 0.0;
        phi[i] = ok ? a : 0.0;
        phib[i] = ok ? b : 0.0;
        acc[i] = 0;
    }
    // the run's frame split and window, read together
    // the run's window and frame split (one record)
    const int4 zr4 = *reinterpret_cast<const int4*>(zrec + 4 * zrun);
    const int off = zr4.x, M = zr4.y, nA = zr4.z;
    const int MZ = (M + zsplit - 1) / zsplit;
    const int p0 = zc * MZ < M ? zc * MZ : M, p1 = p0 + MZ < M ? p0 + MZ : M;
    const size_t zb = (size_t)j * Mmax;
    const double* zs = zp.zs + 2 * (size_t)off;
    // lane l holds the operands of measurement c0 + l of [p0, p1) (frame
    // order: frame A below nA, frame B from nA); the first 64 are loaded
    // right after the particles
    struct ZOp {
        double zr, zt;
        int H;
        T F;
        int fl;
    };
    auto zop = [&](int q) { return ZOp{ zs[2 * q], zs[2 * q + 1], zHs[zb + q], zFs[zb + q], zfls[zb + q] }; };
    const ZOp z0 = p0 < p1 ? zop(p0 + lane < p1 ? p0 + lane : p0) : ZOp{ 0.0, 0.0, 0, (T)0, 0 };
    const size_t pz = ((size_t)j * sp.wtiles + tile) * Mmax;
    // the velocities, read once by tiles that keep a candidate label: issued
    // when a chunk first holds one, so the reads overlap that chunk's other
    // measurements instead of stalling every candidate
    T v1[PT], v3[PT];
    bool have_v = false;
    auto load_velocities = [&]() {
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int s = base + i * 64 + lane;
            uint32_t g = s < n ? s : base;
            // formed here, not hoisted out of the measurement loop (live
            // 64-bit addresses would cost registers for the whole pass)
            __asm__ volatile("" : "+v"(g));
            v1[i] = ld_slot(gx1, g);
            v3[i] = ld_slot(gx3, g);
        }
        have_v = true;
    };
    // a candidate label's local-estimate sums (0 in empty slots)
    auto cand = [&](double zr, double zt, double H, T F, int fl, const double* ang) {
        T u0 = 0, u1 = 0, u2 = 0, u3 = 0, u4 = 0;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int s = base + i * 64 + lane;
            const bool ok = s < n;
            const T x1 = v1[i], x3 = v3[i];
            const T e = fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], ang[i], H));
            acc[i] += e * F;
            const T u = ok ? e * (T)(m.wscale * (double)wv[i]) : (T)0;
            u0 += u * xa[i];
            u1 += u * x1;
            u2 += u * xb[i];
            u3 += u * x3;
            u4 += u;
        }
        const double r0 = wave_sum_last((double)u0), r1 = wave_sum_last((double)u1),
                     r2 = wave_sum_last((double)u2), r3 = wave_sum_last((double)u3),
                     r4 = wave_sum_last((double)u4);
        if (lane == 63) {
            double* o = pzeta + (pz + (fl - 1)) * 5;
            o[0] = r0;
            o[1] = r1;
            o[2] = r2;
            o[3] = r3;
            o[4] = r4;
        }
    };
    auto one = [&](double zr, double zt, double H, T F, const double* ang) {
#pragma unroll
        for (int i = 0; i < PT; ++i) acc[i] += fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], ang[i], H)) * F;
    };
    const TileBox bx = tile_box<PT>(rho, phi, phib, base, n, lane);
    // two non-candidate measurements at once (independent exponentials; each
    // particle's sum still takes the measurements in order)
    auto two = [&](double zr, double zt, double H, T F, double yr, double yt, double G, T E, const double* ang) {
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const T e = fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], ang[i], H));
            const T f = fast_exp2(-(T)sq_resid_nowrap(yr, yt, rho[i], ang[i], G));
            acc[i] += e * F;
            acc[i] += f * E;
        }
    };
    // the kept measurements of one frame in a chunk, in measurement order:
    // candidates (fl != 0) one at a time, two consecutive others at once
    auto run = [&](uint64_t live, uint64_t cset, const ZOp& o, const double* ang) {
        while (live) {
            const int l = __builtin_ctzll(live);
            live &= live - 1;
            if ((cset >> l) & 1ull) {
                cand(lane_value(o.zr, l), lane_value(o.zt, l), (double)lane_value(o.H, l), lane_value(o.F, l),
                     lane_value(o.fl, l), ang);
            } else if (live && !((cset >> __builtin_ctzll(live)) & 1ull)) {
                const int l2 = __builtin_ctzll(live);
                live &= live - 1;
                two(lane_value(o.zr, l), lane_value(o.zt, l), (double)lane_value(o.H, l), lane_value(o.F, l),
                    lane_value(o.zr, l2), lane_value(o.zt, l2), (double)lane_value(o.H, l2), lane_value(o.F, l2),
                    ang);
            } else {
                one(lane_value(o.zr, l), lane_value(o.zt, l), (double)lane_value(o.H, l), lane_value(o.F, l), ang);
            }
        }
    };
    // the exponent is the squared distance plus the measurement's shift H;
    // lane l tests measurement c0 + l in its own frame
    for (int c0 = p0; c0 < p1; c0 += 64) {
        const int p = c0 + lane;
        bool need = false;
        ZOp o{ 0.0, 0.0, 0, (T)0, 0 };
        if (p < p1) {
            o = c0 == p0 ? z0 : zop(p);
            need = box_needed(bx, p >= nA, (float)o.zr, (float)o.zt, (float)o.H, (float)exp2_cut<T>());
            if (!need && o.fl != 0) {
                double* q = pzeta + (pz + (o.fl - 1)) * 5;
                q[0] = 0.0;
                q[1] = 0.0;
                q[2] = 0.0;
                q[3] = 0.0;
                q[4] = 0.0;
            }
        }
        const uint64_t cset = __ballot(need && o.fl != 0);
        const uint64_t live = __ballot(need);
        if (cset && !have_v) load_velocities();
        const int na = nA - c0 < 0 ? 0 : (nA - c0 > 64 ? 64 : nA - c0);
        const uint64_t amask = na >= 64 ? ~0ull : ((1ull << na) - 1ull);
        run(live & amask, cset, o, phi);
        run(live & ~amask, cset, o, phib);
    }
    if constexpr (PT % 4 == 0) {
        if (fin.on) {
            if (zsplit == 1) {
                finalize_tile<T, PT>(m, fin, wv, xa, xb, acc, j, tile, base, n, lane);
                return;
            }
            // a birth tile in BIRTH_CHUNKS items: its chunks are the four
            // wavefronts of this workgroup (items 4q .. 4q + 3 of the group),
            // all here together; the chunk-0 wavefront adds the partials in
            // chunk order (as k_wfinal adds them) and finalizes the tile.
            // Consecutive chunked tiles of the workgroup alternate buffers:
            // a buffer is written again only after the next tile's barrier,
            // which its reader reaches once done, so the other wavefronts go
            // on at once
            __shared__ T s_acc[2][BIRTH_CHUNKS][PT][64];
            const int buf = quads & 1;
            ++quads;
#pragma unroll
            for (int i = 0; i < PT; ++i) s_acc[buf][zc][i][lane] = acc[i];
            __syncthreads();
            if (zc == 0) {
                T tot[PT];
#pragma unroll
                for (int i = 0; i < PT; ++i) {
                    T a = 0;
                    for (int c = 0; c < BIRTH_CHUNKS; ++c) a += s_acc[buf][c][i][lane];
                    tot[i] = a;
                }
                finalize_tile<T, PT>(m, fin, wv, xa, xb, tot, j, tile, base, n, lane);
            }
            return;
        }
    }
    const size_t KC = (size_t)m.K * m.cap;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        if (s < n) accp[(size_t)zc * KC + gb + s] = acc[i];
    }
}

template <typename T, int PT>
__global__ __launch_bounds__(256) void k_weight_frames(DevModel m, const Grp* __restrict__ gd, SoA<T> st, Geo geo,
                                                       const int* __restrict__ ncur, int Mall,
                                                       const ZWin* __restrict__ win, ZPrepC zp, int Mmax, Split sp,
                                                       const int* __restrict__ zHs, const T* __restrict__ zFs,
                                                       const int* __restrict__ zfls, double* __restrict__ pzeta,
                                                       T* __restrict__ accp, const int* __restrict__ nsurv, int K,
                                                       const int* __restrict__ tpre, const int* __restrict__ tgrp,
                                                       WFin<T> fin, const int* __restrict__ zrec,
                                                       const int* __restrict__ items, int imax,
                                                       const int* __restrict__ nitems)
{
    // per group (tpre null, grid (K, X)) or over the flat list (grid (X));
    // items: the groups' item tables (heavy tiles split), else the items the
    // sizes give
    const bool flat = tpre != nullptr;
    const int w0 = (flat ? blockIdx.x : blockIdx.y) * 4 + wave_in_block();
    const int stride = (flat ? gridDim.x : gridDim.y) * 4;
    // the group's sizes and run, read once (kept apart from the per-item reads
    // of the flat lists, so they are not read again per item)
    int2 s0 = flat ? make_int2(0, 0) : make_int2(ncur[blockIdx.x], nsurv[blockIdx.x]);
    int run0 = flat || m.one_run ? 0 : gd[blockIdx.x].run;
    int n0 = flat || !items ? 0 : nitems[blockIdx.x];
    __asm__ volatile("" : "+s"(run0), "+s"(s0.x), "+s"(s0.y), "+s"(n0));
    const int end = flat ? tpre[K] : (items ? n0 : tile_items(s0.x, s0.y, 64 * PT));
    int quads = 0;  // chunked tiles finalized so far (the same count in all four wavefronts)
    for (int e = w0; e < end; e += stride) {
        const int j = flat ? tgrp[e] : (int)blockIdx.x;
        const int le = flat ? e - tpre[j] : e;
        const int2 sz = item_sizes(ncur, nsurv, flat, j, s0);
        int cnt = items ? n0 : 0;
        if (items && flat) {
            int jj = j;
            __asm__ volatile("" : "+s"(jj));
            cnt = nitems[jj];
        }
        if (le >= (items ? cnt : tile_items(sz.x, sz.y, 64 * PT))) continue;  // a list's padding
        const TileItem it = items ? item_decode(items[(size_t)j * imax + le]) : tile_item(le, sz.x, sz.y, 64 * PT);
        weight_frames_tile<T, PT>(m, gd, st, geo, sz.x, Mall, win, zp, Mmax, sp, zHs, zFs, zfls, pzeta, accp, zrec,
                                  j, item_run(gd, flat && !m.one_run, j, run0), it.tile, it.chunk, it.chunks, fin, quads);
    }
}

// ---------------------------------------------------------------------------
// Combine the first-pass partials of group j (one 1024-thread workgroup per
// group).  Lanes take 64 consecutive measurements (one tile's row of partials
// per load), wavefront w the tiles w, w + 16, ...; each lane keeps a running
// exponent and sum, rescaled by a power of two when a larger exponent comes
// (exact outside the subnormal range), and the 16 wavefronts' pairs are then
// added in wavefront order:
//   H = max h over tiles with s > 0, S = sum s 2^(h - H)
//   C = 2^H S,  F = 1/(kappa 2^-H + S) = 2^H/(kappa + C),  dW = S F = C/(kappa + C)
// Then the candidate labels for Step 3: the top min(LT_c + 1, #dW>0)
// measurements by dW (ties to the lower index), where LT_c = round(nu sum w +
// sum dW) is the closed form of the updated mass (the sums of Eq 8 swapped);
// the exact count LT differs from LT_c by at most one, so the candidates
// always cover it.  zflag[p] = 1 + rank, or 0.
// With zS (one C over all groups of the run) the workgroup only stores each
// measurement's (S, H) of its group, and C = 2^H S; k_cz_global does the rest.
// grid (K), 1024 threads, dynamic LDS Mmax doubles.
// ---------------------------------------------------------------------------
// this thread's share of the group's tile weight sums (threads take tiles
// tid, tid + 1024, ...), read ahead of the candidates that use it
__device__ __forceinline__ double tile_weight_share(const double* __restrict__ pw, int j, int wtiles, int nw)
{
    double wsum = 0.0;
    for (int t = threadIdx.x; t < nw; t += 1024) wsum += pw[(size_t)j * wtiles + t];
    return wsum;
}

// The candidate count is LT + 1 (LT from the group's mass, or, with
// run_mass >= 0, from the run's total mass when one C(z) spans the groups):
// one more than Step 3 keeps, so that a rounding difference from the final
// mass cannot leave out a label.
template <typename T>
__device__ __forceinline__ void combine_candidates(const DevModel& m, const Grp& gr, int j, int M, double wsum,
                                                   const double* __restrict__ sm_dw, int zoff,
                                                   const int* __restrict__ zpos, ZSorted<T> zsort, size_t zb,
                                                   int* __restrict__ zflag, int* __restrict__ cand,
                                                   int* __restrict__ ncand, double run_mass)
{
    __shared__ double s_red[16];
    __shared__ int s_redi[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_in_block();
    double dsum = 0.0;
    int pos = 0;
    for (int q = tid; q < M; q += 1024) {
        dsum += sm_dw[q];
        pos += sm_dw[q] > 0.0 ? 1 : 0;
    }
    dsum = wave_sum(dsum);
    wsum = wave_sum(wsum);
    pos = (int)wave_sum((double)pos);
    if (lane == 0) {
        s_red[wv] = m.nu * wsum + dsum;
        s_redi[wv] = pos;
    }
    __syncthreads();
    double mass_c = 0.0;
    int npos = 0;
    for (int w2 = 0; w2 < 16; ++w2) {
        mass_c += s_red[w2];
        npos += s_redi[w2];
    }
    const double lt = floor((run_mass >= 0.0 ? run_mass : mass_c) + 0.5);
    const int LTc = lt < 0.0 ? 0 : (lt > (double)M ? M : (int)lt);
    const int nc = LTc + 1 < npos ? LTc + 1 : npos;
    if (tid == 0) ncand[j] = nc;
    for (int q = tid; q < M; q += 1024) {
        const double v = sm_dw[q];
        if (!(v > 0.0)) continue;
        int rank = 0;
        for (int r = 0; r < M; ++r) {
            const double u = sm_dw[r];
            rank += (u > v || (u == v && r < q)) ? 1 : 0;
        }
        if (rank < nc) {
            cand[zb + rank] = q;
            zflag[zb + q] = rank + 1;
            if (zpos) zsort.flag[zb + zpos[zoff + q]] = rank + 1;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_cz_combine(DevModel m, const Grp* __restrict__ gd,
                                                     const int* __restrict__ ncur, int Mall,
                                                     const ZWin* __restrict__ win, const int* __restrict__ zpos,
                                                     ZSorted<T> zsort, int Mmax,
                                                     int wtiles, int WT, const double* __restrict__ ps,
                                                     const int* __restrict__ ph, const double* __restrict__ pw,
                                                     int* __restrict__ zH, T* __restrict__ zF,
                                                     double* __restrict__ zC, double* __restrict__ zdW,
                                                     int* __restrict__ zflag, int* __restrict__ cand,
                                                     int* __restrict__ ncand, double* __restrict__ zS,
                                                     const int* __restrict__ nsurv, const int* __restrict__ tkept,
                                                     int* __restrict__ items, int imax, int WT2,
                                                     int* __restrict__ nitems)
{
    extern __shared__ double sm_dw[];
    const int j = blockIdx.x;
    const Grp gr = gd[j];
    const int M = zview(gr, win, nullptr, Mall).M;
    // the second pass's item table of this group (heavy tiles split)
    if (items) build_items(j, ncur[j], nsurv[j], WT2, tkept, wtiles, items, imax, nitems);
    // frame-order passes (zpos != nullptr) keep their partials, and want H, F
    // and the flag, in frame order
    const int zoff = win ? win[gr.run].off : 0;
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_in_block();
    const int n = ncur[j];
    const int nw = (n + WT - 1) / WT;
    const size_t zb = (size_t)j * Mmax;
    const double wsum = zS ? 0.0 : tile_weight_share(pw, j, wtiles, nw);
    __shared__ int s_h[16][64];
    __shared__ double s_s[16][64];
    constexpr int RC = 8;  // tiles per wavefront whose loads are in flight together
    for (int p0 = 0; p0 < M; p0 += 64) {
        const int p = p0 + lane;
        const bool live = p < M;
        const int pp = live ? (zpos ? zpos[zoff + p] : p) : 0;
        int Hl = -2147483647 - 1;
        double Sl = 0.0;
        for (int t0 = wv; t0 < nw; t0 += 16 * RC) {
            double v[RC];
            int h[RC];
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                const int t = t0 + 16 * r;
                const size_t o = ((size_t)j * wtiles + (t < nw ? t : 0)) * Mmax + pp;
                const double x = ps[o];
                // the frame passes store a tile's one exponent in its row's
                // first column
                h[r] = ph[zpos ? o - pp : o];
                v[r] = live && t < nw ? x : 0.0;
            }
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                if (!(v[r] > 0.0)) continue;
                if (h[r] > Hl) {
                    Sl = Sl > 0.0 ? ldexp(Sl, Hl - h[r]) : 0.0;
                    Hl = h[r];
                }
                Sl += ldexp(v[r], h[r] - Hl);
            }
        }
        s_h[wv][lane] = Hl;
        s_s[wv][lane] = Sl;
        __syncthreads();
        if (wv == 0 && live) {
            int H = s_h[0][lane];
            for (int w2 = 1; w2 < 16; ++w2) H = s_h[w2][lane] > H ? s_h[w2][lane] : H;
            double S = 0.0;
            for (int w2 = 0; w2 < 16; ++w2) {
                const double sw = s_s[w2][lane];
                if (sw > 0.0) S += ldexp(sw, s_h[w2][lane] - H);
            }
            double C = 0.0, F = 0.0, dW = 0.0;
            if (S > 0.0) {
                const double D = ldexp(gr.kappa, -H) + S;
                F = 1.0 / D;
                dW = S / D;
                C = ldexp(S, H);
            } else {
                H = 0;
            }
            if (zS) {
                // one C over all groups: this group's (S, H) for k_cz_global
                zS[zb + p] = S;
                zH[zb + p] = H;
                zC[zb + p] = C;
            } else {
                zH[zb + p] = H;
                zF[zb + p] = (T)F;
                zC[zb + p] = C;
                zdW[zb + p] = dW;
                zflag[zb + p] = 0;
                sm_dw[p] = dW;
                if (zpos) {
                    zsort.H[zb + pp] = H;
                    zsort.F[zb + pp] = (T)F;
                    zsort.flag[zb + pp] = 0;
                }
            }
        }
        // wavefront 0 has read this chunk's pairs before any wavefront writes
        // the next chunk's
        __syncthreads();
    }
    if (zS) return;
    __syncthreads();
    combine_candidates<T>(m, gr, j, M, wsum, sm_dw, zoff, zpos, zsort, zb, zflag, cand, ncand, -1.0);
}

// ---------------------------------------------------------------------------
// One C(z) over all groups of a run (the global-C reading of Eq 11): for
// every measurement of group j's run, the groups' pairs (S_q, H_q) from
// k_cz_combine give
//   H = max H_q over the groups with S_q > 0,  S = sum_q S_q 2^(H_q - H)
// (lanes over the groups, one wavefront tree sum), and group j takes
//   F = 1/(kappa 2^-H + S) = 2^H/(kappa + C),  dW_j = S_j 2^(H_j - H) F = C_j/(kappa + C)
// with C = 2^H S, so the second pass divides every term by kappa + C.  The
// group's candidate labels then follow as in k_cz_combine, with LT from the
// run's total mass nu sum_q sum_i w_i + sum_p S/(kappa 2^-H + S) (thread q
// adds group q's tile weight sums in tile order; wavefront w the labels w,
// w + 16, ...; both reduced in wavefront order).  Every group of a run forms
// the same H, S and total in the same order.
// grid (K), 1024 threads, dynamic LDS Mmax doubles.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_cz_global(DevModel m, const Grp* __restrict__ gd,
                                                    const int* __restrict__ ncur, int Mall,
                                                    const ZWin* __restrict__ win, const int* __restrict__ zpos,
                                                    ZSorted<T> zsort, int Mmax, int wtiles, int WT,
                                                    const double* __restrict__ pw, const double* __restrict__ zS,
                                                    const int* __restrict__ zHg, int* __restrict__ zH,
                                                    T* __restrict__ zF, double* __restrict__ zdW,
                                                    int* __restrict__ zflag, int* __restrict__ cand,
                                                    int* __restrict__ ncand)
{
    extern __shared__ double sm_dw[];
    const int j = blockIdx.x;
    const Grp gr = gd[j];
    const int M = zview(gr, win, nullptr, Mall).M;
    const int zoff = win ? win[gr.run].off : 0;
    const int lane = threadIdx.x & 63, wv = wave_in_block();
    const size_t zb = (size_t)j * Mmax;
    const double wsum = tile_weight_share(pw, j, wtiles, (ncur[j] + WT - 1) / WT);
    double wrun = 0.0, drun = 0.0;
    for (int q = threadIdx.x; q < gr.K; q += 1024) {
        const int g = gr.g0 + q;
        const int nwq = (ncur[g] + WT - 1) / WT;
        for (int t = 0; t < nwq; ++t) wrun += pw[(size_t)g * wtiles + t];
    }
    for (int p = wv; p < M; p += 16) {
        int hl = -2147483647 - 1;
        for (int q0 = 0; q0 < gr.K; q0 += 64) {
            const int q = q0 + lane;
            if (q < gr.K) {
                const size_t o = (size_t)(gr.g0 + q) * Mmax + p;
                if (zS[o] > 0.0) hl = zHg[o] > hl ? zHg[o] : hl;
            }
        }
        const int H = wave_max(hl);
        double sl = 0.0;
        for (int q0 = 0; q0 < gr.K; q0 += 64) {
            const int q = q0 + lane;
            if (q < gr.K) {
                const size_t o = (size_t)(gr.g0 + q) * Mmax + p;
                if (zS[o] > 0.0) sl += ldexp(zS[o], zHg[o] - H);
            }
        }
        const double S = wave_sum(sl);
        if (lane == 0) {
            const double Sj = zS[zb + p];
            double F = 0.0, dW = 0.0;
            int Hs = 0;
            if (S > 0.0) {
                const double D = ldexp(gr.kappa, -H) + S;
                F = 1.0 / D;
                dW = Sj > 0.0 ? ldexp(Sj, zHg[zb + p] - H) / D : 0.0;
                Hs = H;
                drun += S / D;
            }
            zH[zb + p] = Hs;
            zF[zb + p] = (T)F;
            zdW[zb + p] = dW;
            zflag[zb + p] = 0;
            sm_dw[p] = dW;
            if (zpos) {
                const int pp = zpos[zoff + p];
                zsort.H[zb + pp] = Hs;
                zsort.F[zb + pp] = (T)F;
                zsort.flag[zb + pp] = 0;
            }
        }
    }
    __shared__ double s_run[16][2];
    wrun = wave_sum(wrun);
    if (lane == 0) {
        s_run[wv][0] = wrun;
        s_run[wv][1] = drun;
    }
    __syncthreads();
    double wr = 0.0, dr = 0.0;
    for (int w2 = 0; w2 < 16; ++w2) {
        wr += s_run[w2][0];
        dr += s_run[w2][1];
    }
    combine_candidates<T>(m, gr, j, M, wsum, sm_dw, zoff, zpos, zsort, zb, zflag, cand, ncand, m.nu * wr + dr);
}

// ---------------------------------------------------------------------------
// Step 2, second pass (Eqs 12-15) and the sums of Step 3 (Eqs 16-18), per
// (tile, chunk) wave:  acc_i = sum over the chunk of 2^(-q_ip - H_p) F_p,
// stored to accp[zc][slot]; k_wfinal then forms
//   w_i <- nu w_i + wscale w_i sum_chunks acc_i.
// For a candidate label p the wave also sums u_i = wscale w_i 2^(-q_ip - H_p),
// u_i x_i (4 components) and writes them to pzeta[((j*wtiles + tile)*Mmax +
// rank)*5 + k]; their ratio is the local estimate of Eq 18 (F cancels).
// grid (ceil(wtiles*zsplit/4), K), 256 threads.
// ---------------------------------------------------------------------------
template <typename T, int PT, bool FRAMES>
__global__ __launch_bounds__(256) void k_weight(DevModel m, const Grp* __restrict__ gd, SoA<T> st, Geo geo,
                                                const int* __restrict__ ncur, const double* __restrict__ Zall,
                                                int Mall, const ZWin* __restrict__ win, int Mmax, Split sp,
                                                const int* __restrict__ zH, const T* __restrict__ zF,
                                                const int* __restrict__ zflag, double* __restrict__ pzeta,
                                                T* __restrict__ accp)
{
    constexpr int WT = 64 * PT;
    const int j = blockIdx.y;
    const ZView zv = zview(gd[j], win, Zall, Mall);
    const double* Z = zv.Z;
    const int M = zv.M;
    const int zsplit = zsplit_for(M, sp.mz), MZ = (M + zsplit - 1) / zsplit;
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + wave_in_block();
    const int tile = gw / zsplit, zc = gw - tile * zsplit;
    const int n = ncur[j];
    const int base = tile * WT;
    if (tile >= sp.wtiles || base >= n) return;
    const size_t gb = (size_t)j * m.cap;
    const size_t zb = (size_t)j * Mmax;
    double rho[PT], phi[PT], phib[PT];
    T acc[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        const bool ok = s < n;
        const size_t g = gb + (ok ? s : base);
        const double r = geo.rho[g], a = geo.phi[g], b = FRAMES ? geo.phib[g] : 0.0;
        rho[i] = ok ? r : 0.0;
        phi[i] = ok ? a : 0.0;
        phib[i] = ok ? b : 0.0;
        acc[i] = 0;
    }
    // exponential of one pair in the measurement's frame (or with the wrap)
    auto term = [&](double zr, double zt, bool fb, double H, int i) -> T {
        if (FRAMES) return fast_exp2(-(T)sq_resid_nowrap(zr, zt, rho[i], fb ? phib[i] : phi[i], H));
        return fast_exp2(-(T)sq_resid(m, zr, zt, rho[i], phi[i], H));
    };
    const size_t pz = ((size_t)j * sp.wtiles + tile) * Mmax;
    const int p0 = zc * MZ, p1 = (p0 + MZ < M) ? p0 + MZ : M;
    for (int pb = p0; pb < p1; pb += 64) {
        const int pe = (pb + 64 < p1) ? pb + 64 : p1;
        double lzr = 0.0, lzt = 0.0;
        int lH = 0, lfl = 0, lfb = 0;
        T lF = 0;
        if (pb + lane < pe) {
            const int q = pb + lane;
            if (FRAMES) {
                const ZFrame zf = z_frame(m, Z[2 * q], Z[2 * q + 1]);
                lzr = zf.zr;
                lzt = zf.zt;
                lfb = zf.b ? 1 : 0;
            } else {
                lzr = Z[2 * q] * m.cr;
                lzt = Z[2 * q + 1] * m.ct;
            }
            lH = zH[zb + q];
            lF = zF[zb + q];
            lfl = zflag[zb + q];
        }
        for (int p = pb; p < pe; ++p) {
            const int l = p - pb;
            const double zr = lane_value(lzr, l), zt = lane_value(lzt, l);
            const double H = (double)lane_value(lH, l);
            const T F = lane_value(lF, l);
            const int fl = lane_value(lfl, l);
            const bool fb = FRAMES && lane_value(lfb, l) != 0;
            if (fl == 0) {
                if (fb) {
#pragma unroll
                    for (int i = 0; i < PT; ++i) acc[i] += term(zr, zt, true, H, i) * F;
                } else {
#pragma unroll
                    for (int i = 0; i < PT; ++i) acc[i] += term(zr, zt, false, H, i) * F;
                }
            } else {
                T u0 = 0, u1 = 0, u2 = 0, u3 = 0, u4 = 0;
#pragma unroll
                for (int i = 0; i < PT; ++i) {
                    const T e = term(zr, zt, fb, H, i);
                    acc[i] += e * F;
                    const int s = base + i * 64 + lane;
                    if (s < n) {
                        const T u = e * (T)(m.wscale * (double)st.w[gb + s]);
                        u0 += u * st.x[0][gb + s];
                        u1 += u * st.x[1][gb + s];
                        u2 += u * st.x[2][gb + s];
                        u3 += u * st.x[3][gb + s];
                        u4 += u;
                    }
                }
                const double r0 = wave_sum_last((double)u0), r1 = wave_sum_last((double)u1),
                             r2 = wave_sum_last((double)u2), r3 = wave_sum_last((double)u3),
                             r4 = wave_sum_last((double)u4);
                if (lane == 63) {
                    double* o = pzeta + (pz + (fl - 1)) * 5;
                    o[0] = r0;
                    o[1] = r1;
                    o[2] = r2;
                    o[3] = r3;
                    o[4] = r4;
                }
            }
        }
    }
    const size_t KC = (size_t)m.K * m.cap;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int s = base + i * 64 + lane;
        if (s < n) accp[(size_t)zc * KC + gb + s] = acc[i];
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


// Bucket-major exclusive offsets of group j's ntl tiles, off[t][b] = all
// slots of lower buckets + slots of bucket b in lower tiles, by a workgroup
// of NW wavefronts: lane b of wave g sums bucket b over the g-th of NW
// contiguous tile segments; the segment totals meet in LDS.
template <int NW>
__device__ __forceinline__ void bucket_offsets(int j, int ntl, int rtiles, const int* __restrict__ hist,
                                               int* __restrict__ off)
{
    __shared__ int seg[NW][BEARING_BUCKETS];
    __shared__ int base[BEARING_BUCKETS];
    const int b = threadIdx.x & 63, g = wave_in_block();
    const int per = (ntl + NW - 1) / NW;
    const int t0 = g * per < ntl ? g * per : ntl, t1 = t0 + per < ntl ? t0 + per : ntl;
    const int* hj = hist + (size_t)j * rtiles * BEARING_BUCKETS;
    // tiles in runs of 8, the reads of a run issued together (clamped to the
    // wave's last tile, values past it dropped)
    int tot = 0;
    for (int t = t0; t < t1; t += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = hj[(size_t)(t + u < t1 ? t + u : t1 - 1) * BEARING_BUCKETS + b];
#pragma unroll
        for (int u = 0; u < 8; ++u) tot += t + u < t1 ? v[u] : 0;
    }
    seg[g][b] = tot;
    __syncthreads();
    if (g == 0) {
        int all = 0;
        for (int q = 0; q < NW; ++q) all += seg[q][b];
        const int incl = (int)wave_incl_scan((double)all);  // exact: counts stay below 2^53
        base[b] = incl - all;
    }
    __syncthreads();
    int run = base[b];
    for (int q = 0; q < g; ++q) run += seg[q][b];
    int* oj = off + (size_t)j * rtiles * BEARING_BUCKETS;
    for (int t = t0; t < t1; t += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = hj[(size_t)(t + u < t1 ? t + u : t1 - 1) * BEARING_BUCKETS + b];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (t + u < t1) {
                oj[(size_t)(t + u) * BEARING_BUCKETS + b] = run;
                run += v[u];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// New weights from the chunk sums (chunk order fixed) and Step 3 per group.
// k_wfinal: every workgroup turns 256 slots into
//   w <- nu w + wscale w sum_chunks acc
// and writes the tile's sum and maximum of the stored weights.
// grid (tiles256, K).  k_finalize (grid K) then forms the mass N_j,
// LT_j = round(N_j) capped at M, the label set I_j (the first LT_j
// candidates), their local estimates zeta = sum u x / sum u, and the
// quantisation shift of the group's resampling.  k_wfinal: 256 threads;
// k_finalize: NW wavefronts (4; 16 measured slower at the benchmark shape).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_wfinal(DevModel m, const Grp* __restrict__ gd, T* __restrict__ W,
                                                const int* __restrict__ ncur, const T* __restrict__ accp, int Mall,
                                                const ZWin* __restrict__ win, int mz, int tiles256,
                                                double* __restrict__ pmass, double* __restrict__ pmax,
                                                const T* __restrict__ X0, const T* __restrict__ X2,
                                                int* __restrict__ bkt, int* __restrict__ bhist, int wt_births,
                                                const int* __restrict__ nsurv)
{
    __shared__ double s_wn[4][64];
    __shared__ int h[BEARING_BUCKETS];
    const int j = slot_group(m);
    // the slot counts first: the capacity's empty tiles leave after one read
    const int n = ncur[j], ns = nsurv[j];
    const int tile = slot_tile(m);
    const int nt = (n + 255) / 256;
    const int active = nt > 0 ? nt : 1;
    if (tile >= active) return;
    // chunks of the second pass: the run's zsplit, or (frame passes, wt_births
    // = their tile) one, and BIRTH_CHUNKS in the tiles holding births
    const int s = tile * 256 + threadIdx.x;
    const int zsplit = wt_births > 0 ? (s / wt_births >= tiles_before_births(n, ns, wt_births)
                                            ? birth_chunks(n, ns, wt_births)
                                            : 1)
                                     : zsplit_for(zview(gd[j], win, nullptr, Mall).M, mz);
    const int lane = threadIdx.x & 63, wv = wave_in_block();
    const size_t KC = (size_t)m.K * m.cap;
    const size_t g = (size_t)j * m.cap + s;
    if (threadIdx.x < BEARING_BUCKETS) h[threadIdx.x] = 0;
    __syncthreads();
    double wn = 0.0;
    if (s < n) {
        T acc = 0;
#pragma unroll 4
        for (int zc = 0; zc < zsplit; ++zc) acc += accp[(size_t)zc * KC + g];
        const double w = (double)W[g];
        const T t = (T)(m.nu * w + m.wscale * w * (double)acc);
        W[g] = t;
        wn = (double)t;
        // the parent's bearing bucket for the resampling's order (the
        // positions stay as they are until then)
        const int b = bearing_bucket(m, (double)X0[g], (double)X2[g]);
        bkt[g] = b;
        atomicAdd(&h[b], 1);
    }
    // the tile's sum and maximum: lane l adds slots l, l + 64, l + 128 and
    // l + 192 pairwise, then one wavefront reduction (the order the fused
    // second pass uses)
    s_wn[wv][lane] = wn;
    __syncthreads();
    if (wv == 0) {
        const double a = s_wn[0][lane], b = s_wn[1][lane], c = s_wn[2][lane], d = s_wn[3][lane];
        const double sm = wave_sum_last((a + b) + (c + d)), mx = wave_max(vmax(vmax(a, b), vmax(c, d)));
        if (lane == 63) {
            pmass[(size_t)j * tiles256 + tile] = sm;
            pmax[(size_t)j * tiles256 + tile] = mx;
        }
    }
    if (threadIdx.x < BEARING_BUCKETS) bhist[((size_t)j * tiles256 + tile) * BEARING_BUCKETS + threadIdx.x] =
        h[threadIdx.x];
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_finalize(const Grp* __restrict__ gd, const int* __restrict__ ncur,
                                                  int tiles256, const double* __restrict__ pmass,
                                                  const double* __restrict__ pmax, int Mall,
                                                  const ZWin* __restrict__ win, int Mmax, int wtiles2, int WT2,
                                                  const double* __restrict__ pzeta, const int* __restrict__ cand,
                                                  const int* __restrict__ ncand, double* __restrict__ fmass,
                                                  int* __restrict__ fLT, int* __restrict__ rsS,
                                                  int* __restrict__ sel, double* __restrict__ zeta,
                                                  int rtiles, const int* __restrict__ bhist, int* __restrict__ boff,
                                                  double* __restrict__ tsum, double* __restrict__ qtot)
{
    const int j = blockIdx.x;
    const int M = zview(gd[j], win, nullptr, Mall).M;
    const int n = ncur[j];
    const int nt = (n + 255) / 256;
    const int lane = threadIdx.x & 63, wv = wave_in_block();
    const size_t zb = (size_t)j * Mmax;
    for (int p = threadIdx.x; p < M; p += 64 * NW) {
        sel[zb + p] = 0;
#pragma unroll
        for (int d = 0; d < 4; ++d) zeta[(zb + p) * 4 + d] = 0.0;
    }
    // Every read that does not wait for the group's mass goes out first: the
    // tile masses and maxima (wavefront 0), the first round of candidate
    // labels' partial sums (labels c, c + NW, c + 2 NW, c + 3 NW of wavefront
    // c, those below the candidate count; the count LT decides later which
    // are kept), and, inside bucket_offsets, the tiles' bucket histograms.
    const int nc = ncand[j];
    const int nw = (n + WT2 - 1) / WT2;
    double ms = 0.0, mm = 0.0;
    if (wv == 0) {
#pragma unroll 4
        for (int t = lane; t < nt; t += 64) {
            ms += pmass[(size_t)j * tiles256 + t];
            mm = vmax(mm, pmax[(size_t)j * tiles256 + t]);
        }
    }
    // one C(z) over the run's groups: LT from the run's total mass (thread q
    // adds group q's tile masses in tile order, then a reduction in
    // wavefront order; every group of the run forms the same total)
    const Grp gr = gd[j];
    double mrun = 0.0;
    if (gr.gz) {
        for (int q = threadIdx.x; q < gr.K; q += 64 * NW) {
            const int g = gr.g0 + q;
            const int ntq = (ncur[g] + 255) / 256;
            for (int t = 0; t < ntq; ++t) mrun += pmass[(size_t)g * tiles256 + t];
        }
        mrun = wave_sum(mrun);
    }
    // candidate round of labels cb, cb + NW, cb + 2 NW, cb + 3 NW (below lim;
    // the others clamped to cb, values dropped)
    auto load_round = [&](int cb, int lim, double (&a)[4][5], int (&pc)[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            pc[r] = cand[zb + (cb + NW * r < lim ? cb + NW * r : cb)];
#pragma unroll
            for (int k = 0; k < 5; ++k) a[r][k] = 0.0;
        }
        for (int t = lane; t < nw; t += 64) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = cb + NW * r < lim ? cb + NW * r : cb;
                const double* o = pzeta + (((size_t)j * wtiles2 + t) * Mmax + c) * 5;
#pragma unroll
                for (int k = 0; k < 5; ++k) a[r][k] += o[k];
            }
        }
    };
    auto finish_round = [&](int cb, int lim, const double (&a)[4][5], const int (&pc)[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (cb + NW * r >= lim) break;
            double e[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) e[k] = wave_sum(a[r][k]);
            if (lane == 0) {
                const int p = pc[r];
                sel[zb + p] = 1;
                if (e[4] > 0.0) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) zeta[(zb + p) * 4 + d] = e[d] / e[4];
                }
            }
        }
    };
    double a0[4][5];
    int pc0[4];
    if (wv < nc) load_round(wv, nc, a0, pc0);
    // the resampling's parent order (bucket offsets of the group's tiles from
    // the weight pass's histograms) and its tile sums and group total cleared
    // for k_bk_scatter
    for (int t = threadIdx.x; t < nt; t += 64 * NW) tsum[(size_t)j * rtiles + t] = 0.0;
    if (threadIdx.x < QSLOTS) qslot(qtot, j, threadIdx.x, gridDim.x) = 0.0;
    bucket_offsets<NW>(j, nt, rtiles, bhist, boff);
    __shared__ double s_ms, s_mm, s_mrun[NW];
    if (lane == 0) s_mrun[wv] = mrun;
    if (wv == 0) {
        ms = wave_sum(ms);
        mm = wave_max(mm);
        if (lane == 0) {
            s_ms = ms;
            s_mm = mm;
        }
    }
    __syncthreads();
    ms = s_ms;
    mm = s_mm;
    double mr = 0.0;
    if (gr.gz)
        for (int w2 = 0; w2 < NW; ++w2) mr += s_mrun[w2];
    const double lt = floor((gr.gz ? mr : ms) + 0.5);
    const int LT = lt < 0.0 ? 0 : (lt > (double)M ? M : (int)lt);
    const int nsel = LT < nc ? LT : nc;
    if (threadIdx.x == 0) {
        fmass[j] = ms;
        fLT[j] = LT;
        rsS[j] = quant_shift(mm, n);
    }
    // (the labels' zeroing above happened before the barriers in between)
    if (wv < nsel) finish_round(wv, nsel, a0, pc0);
    for (int cb = wv + 4 * NW; cb < nsel; cb += 4 * NW) {
        double a[4][5];
        int pc[4];
        load_round(cb, nsel, a, pc);
        finish_round(cb, nsel, a, pc);
    }
}

// ---------------------------------------------------------------------------
// Step 4, fusion at the central unit (one workgroup of NW wavefronts per run).
// Labels go 64 at a time, one per lane; wavefront w takes the run's groups
// w, w + NW, w + 2 NW, ... and counts and sums the estimates of the groups
// that report the label (every read of the chunk issued before any sum); the
// NW wavefronts' partial sums are then added in wavefront order in LDS, so
// the order of the additions is fixed for a given NW.  A label is kept when
// 2 votes > K, and the kept records are written in label order to the run's
// output (cap records at out + run cap, count at nout[run]).  It runs as
// k_fuse or in the first workgroups of the resampling's scatter launch
// (which needs the same update's results and nothing the fusion writes), in
// both with 4 wavefronts, so both give the same sums.
// ---------------------------------------------------------------------------
struct EstimateRec {
    double state[4];
    int32_t label;
    int32_t votes;
};

struct FuseArgs {
    const Grp* rgd;  // each run's first group
    int Mall;        // measurements (single run) or 0 with win
    const ZWin* win;
    int Mmax;
    const int* sel;
    const double* zeta;
    EstimateRec* out;
    int cap;
    int* nout;
    int nruns;  // 0: no fusion in the launch
};

template <int NW>
__device__ __forceinline__ void fuse_run(const FuseArgs& fa, int run, double (*s_part)[5][64])
{
    constexpr int GPT = 4;  // groups per thread whose reads go out together
    const Grp gr = fa.rgd[run];  // the run's first group
    const int K = gr.K;
    const int M = zview(gr, fa.win, nullptr, fa.Mall).M;
    const int Mmax = fa.Mmax;
    const int* sel = fa.sel + (size_t)gr.g0 * Mmax;
    const double* zeta = fa.zeta + (size_t)gr.g0 * Mmax * 4;
    EstimateRec* out = fa.out + (size_t)run * fa.cap;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int offset = 0;
    for (int p0 = 0; p0 < M; p0 += 64) {
        const int p = p0 + lane;
        const bool live = p < M;
        const int pc = live ? p : 0;
        double v = 0.0, a[4] = { 0.0, 0.0, 0.0, 0.0 };
        for (int j0 = wv; j0 < K; j0 += NW * GPT) {
            int sv[GPT];
            double4 zv[GPT];
#pragma unroll
            for (int u = 0; u < GPT; ++u) {
                const int j = j0 + NW * u < K ? j0 + NW * u : wv;
                sv[u] = sel[(size_t)j * Mmax + pc];
                zv[u] = *reinterpret_cast<const double4*>(zeta + ((size_t)j * Mmax + pc) * 4);
            }
#pragma unroll
            for (int u = 0; u < GPT; ++u) {
                if (j0 + NW * u < K && live && sv[u]) {
                    v += 1.0;
                    a[0] += zv[u].x;
                    a[1] += zv[u].y;
                    a[2] += zv[u].z;
                    a[3] += zv[u].w;
                }
            }
        }
        s_part[wv][0][lane] = v;
#pragma unroll
        for (int d = 0; d < 4; ++d) s_part[wv][1 + d][lane] = a[d];
        __syncthreads();
        if (wv == 0) {
            double vs = 0.0, r[4] = { 0.0, 0.0, 0.0, 0.0 };
            for (int w2 = 0; w2 < NW; ++w2) {
                vs += s_part[w2][0][lane];
#pragma unroll
                for (int d = 0; d < 4; ++d) r[d] += s_part[w2][1 + d][lane];
            }
            const int votes = (int)vs;
            const bool keep = live && 2 * votes > K;
            const unsigned long long kb = __ballot(keep);
            const int idx = offset + __popcll(kb & (lane ? (~0ull >> (64 - lane)) : 0ull));
            if (keep && idx < fa.cap) {
                EstimateRec e;
#pragma unroll
                for (int d = 0; d < 4; ++d) e.state[d] = r[d] / (double)votes;
                e.label = p;
                e.votes = votes;
                out[idx] = e;
            }
            offset += __popcll(kb);
        }
        // (wavefront 0's offset is the only one used; the LDS partials are
        // read before the next chunk writes them)
        __syncthreads();
    }
    if (tid == 0) fa.nout[run] = offset;
}

constexpr int FUSE_WAVES = 4;
// grid (runs), 256 threads
__global__ __launch_bounds__(256) void k_fuse(FuseArgs fa)
{
    __shared__ double s_part[FUSE_WAVES][5][64];
    fuse_run<FUSE_WAVES>(fa, blockIdx.x, s_part);
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

// The sort runs over the slots [first_j, end_j) of every group j: all of a
// group's particles (first == nullptr: from slot 0) before the resampling, or
// its births once drawn (first = the survivor count).
__device__ __forceinline__ int range_first(const int* first, int j) { return first ? first[j] : 0; }

// grid (tiles, K), 256 threads: bucket of every slot, per-tile histograms
// keys_stored: the slots' buckets are already in bkt (births)
template <typename T>
__global__ __launch_bounds__(256) void k_bk_hist(DevModel m, SoA<T> st, const int* __restrict__ first,
                                                 const int* __restrict__ end, int rtiles, int* __restrict__ bkt,
                                                 int* __restrict__ hist, int keys_stored)
{
    __shared__ int h[BEARING_BUCKETS];
    const int j = slot_group(m), t = slot_tile(m);
    const int a = range_first(first, j), n = end[j] - a;
    if (t * 256 >= n) return;
    if (threadIdx.x < BEARING_BUCKETS) h[threadIdx.x] = 0;
    __syncthreads();
    const int s = t * 256 + threadIdx.x;
    const size_t g = (size_t)j * m.cap + a + s;
    if (s < n) {
        const int b = keys_stored ? bkt[g] : bearing_bucket(m, (double)st.x[0][g], (double)st.x[2][g]);
        if (!keys_stored) bkt[g] = b;
        atomicAdd(&h[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < BEARING_BUCKETS)
        hist[((size_t)j * rtiles + t) * BEARING_BUCKETS + threadIdx.x] = h[threadIdx.x];
}

// grid (K), 1024 threads; tsum (optional): the group's resampling tile sums,
// cleared for k_bk_scatter to accumulate
__global__ __launch_bounds__(1024) void k_bk_scan(const int* __restrict__ first, const int* __restrict__ end,
                                                  int rtiles, const int* __restrict__ hist, int* __restrict__ off,
                                                  double* __restrict__ tsum, double* __restrict__ qtot)
{
    const int j = blockIdx.x;
    const int ntl = (end[j] - range_first(first, j) + 255) / 256;
    if (tsum) {
        for (int t = threadIdx.x; t < ntl; t += 1024) tsum[(size_t)j * rtiles + t] = 0.0;
        if (threadIdx.x < QSLOTS) qslot(qtot, j, threadIdx.x, gridDim.x) = 0.0;
    }
    bucket_offsets<16>(j, ntl, rtiles, hist, off);
}

// grid (tiles, K), 256 threads: slot s of the range goes to off[t][b] + (slots
// of bucket b before it in its tile), in the other particle set.  With
// frows > 0 the first frows tile rows of the grid (dispatched first) are the
// fusion of Step 4 instead: workgroup (group j, row r) fuses run j frows + r
// (those below fa.nruns), the scatter's tiles following at row frows.
// With tsum (the parents before Step 5), each parent's integer weight
// q = floor(w 2^S) is also added to the sum of the resampling tile it lands
// in: exact integer sums in FP64 (below 2^53), so the order of the atomic
// additions does not matter.
template <typename T, int NH>
__global__ __launch_bounds__(256) void k_bk_scatter(DevModel m, SoA<T> in, SoA<T> out, const int* __restrict__ first,
                                                    const int* __restrict__ end, int rtiles,
                                                    const int* __restrict__ bkt, const int* __restrict__ off,
                                                    const int* __restrict__ rsS, double* __restrict__ tsum,
                                                    int* __restrict__ orig, double* __restrict__ qtot, FuseArgs fa,
                                                    int frows)
{
    // one LDS buffer: the fusion's partial sums, or the scatter's per-half,
    // per-wave bucket counts
    __shared__ double s_lds[FUSE_WAVES * 5 * 64];
    static_assert(NH * 4 * BEARING_BUCKETS * sizeof(int) <= sizeof(s_lds), "bucket counts fit");
    const int j = slot_group(m), trow = slot_tile(m);
    if (trow < frows) {
        const int run = j * frows + trow;
        if (run < fa.nruns) fuse_run<FUSE_WAVES>(fa, run, reinterpret_cast<double(*)[5][64]>(s_lds));
        return;
    }
    // a workgroup takes NH 256-slot tiles of the range (half h: tile
    // NH t2 + h, one slot per thread; NH = 2 where the capacity spans enough
    // workgroups, else 1), each ranked exactly as a workgroup of its own would
    // rank it; the reads of all go out first
    int(*wh)[4][BEARING_BUCKETS] = reinterpret_cast<int(*)[4][BEARING_BUCKETS]>(s_lds);
    const int t2 = trow - frows;
    const int a = range_first(first, j), n = end[j] - a;
    if (t2 * 256 * NH >= n) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < NH * 4 * BEARING_BUCKETS; i += 256) (&wh[0][0][0])[i] = 0;
    __syncthreads();
    const size_t gb = (size_t)j * m.cap + a;
    // the parents' buckets and states (every component: x[0] stands in for
    // an absent turn rate; lanes past the range read slot 0), then each
    // bucket's offset in its tile once the bucket is in
    int s[NH], b[NH], ob[NH];
    bool live[NH];
    T v[NH][5], pw[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        s[h] = (NH * t2 + h) * 256 + threadIdx.x;
        live[h] = s[h] < n;
        b[h] = live[h] ? bkt[gb + s[h]] : BEARING_BUCKETS;
        const size_t gs = gb + (live[h] ? s[h] : 0);
#pragma unroll
        for (int d = 0; d < 5; ++d) v[h][d] = in.x[d < m.dim ? d : 0][gs];
        pw[h] = in.w[gs];
    }
    const int S = tsum ? rsS[j] : 0;
#pragma unroll
    for (int h = 0; h < NH; ++h)
        ob[h] = live[h] ? off[((size_t)j * rtiles + NH * t2 + h) * BEARING_BUCKETS + b[h]] : 0;
    // lanes of this wave with the same bucket: intersect the ballots of the
    // seven bits of b (bit 6 tells the out-of-range lanes apart)
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int rank[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        unsigned long long peers = ~0ull;
        for (int bit = 0; bit < 7; ++bit) {
            const unsigned long long q = __ballot((b[h] >> bit) & 1);
            peers &= ((b[h] >> bit) & 1) ? q : ~q;
        }
        rank[h] = __popcll(peers & below);
        if (live[h] && rank[h] == 0) wh[h][wv][b[h]] = __popcll(peers);
    }
    __syncthreads();
    int dst[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        dst[h] = -1;
        if (live[h]) {
            int r = rank[h];
            for (int w = 0; w < wv; ++w) r += wh[h][w][b[h]];
            dst[h] = ob[h] + r;
#pragma unroll
            for (int d = 0; d < 5; ++d)
                if (d < m.dim) out.x[d][gb + dst[h]] = v[h][d];
            out.w[gb + dst[h]] = pw[h];
            if (orig) orig[gb + dst[h]] = s[h];
        }
    }
    if (!tsum) return;
    // per destination tile: one wave sum and one atomic addition per distinct
    // tile (integer-valued sums below 2^53: exact in any order); the group's
    // total Q the same way, one addition per workgroup into one of the
    // group's QSLOTS partial sums
    __shared__ double s_qw[4];
    double qw = 0.0;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const double q = live[h] ? floor(ldexp((double)pw[h], S)) : 0.0;
        int tile = live[h] ? (dst[h] >> 8) : -1;
        for (;;) {
            const uint64_t act = __ballot(tile >= 0);
            if (!act) break;
            const int lead = __builtin_ctzll(act);
            const int tl = __builtin_amdgcn_readlane(tile, lead);
            const bool mine = tile == tl;
            const double sq = wave_sum(mine ? q : 0.0);
            if (lane == lead) atomicAdd(&tsum[(size_t)j * rtiles + tl], sq);
            qw += sq;
            if (mine) tile = -1;
        }
    }
    if (lane == 0) s_qw[wv] = qw;
    __syncthreads();
    const double qg = (s_qw[0] + s_qw[1]) + (s_qw[2] + s_qw[3]);
    if (threadIdx.x == 0 && qg > 0.0) atomicAdd(&qslot(qtot, j, t2 & (QSLOTS - 1), m.K), qg);
}

// The ranking of k_birth_sort: births c * 1024 + thread (c < BS, first nb
// of them live) with their states v, weights w and buckets b in registers
// are written at slot gb + rank (stable within a bucket), with borig and the
// geometry as asked.  All 1024 threads of the workgroup call it.
template <typename T, int BS>
__device__ __forceinline__ void sort_births_block(const DevModel& m, const SoA<T>& st, const Geo& geo, size_t gb,
                                                  int nb, T (&v)[BS][5], const T (&w)[BS], const int (&b)[BS],
                                                  int* __restrict__ borig, int with_geo, int (&dst)[BS],
                                                  bool write_w = true)
{
    __shared__ int s_off[BEARING_BUCKETS];
    __shared__ int s_w[16][BEARING_BUCKETS];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < BEARING_BUCKETS) s_off[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        dst[c] = -1;
        if (b[c] < BEARING_BUCKETS) atomicAdd(&s_off[b[c]], 1);
    }
    __syncthreads();
    if (wv == 0) {
        const int cnt = s_off[lane];
        const int incl = (int)wave_incl_scan((double)cnt);
        s_off[lane] = incl - cnt;
    }
    __syncthreads();
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        if (c * 1024 >= nb) break;
        s_w[wv][lane] = 0;
        __syncthreads();
        unsigned long long peers = ~0ull;
        for (int bit = 0; bit < 7; ++bit) {
            const unsigned long long q = __ballot((b[c] >> bit) & 1);
            peers &= ((b[c] >> bit) & 1) ? q : ~q;
        }
        const int rank = __popcll(peers & below);
        if (b[c] < BEARING_BUCKETS && rank == 0) s_w[wv][b[c]] = __popcll(peers);
        __syncthreads();
        if (b[c] < BEARING_BUCKETS) {
            int r = s_off[b[c]] + rank;
            for (int w2 = 0; w2 < wv; ++w2) r += s_w[w2][b[c]];
            dst[c] = r;
        }
        __syncthreads();
        if (wv == 0) {
            int tot = 0;
            for (int w2 = 0; w2 < 16; ++w2) tot += s_w[w2][lane];
            s_off[lane] += tot;
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        if (dst[c] < 0) continue;
        const size_t g = gb + dst[c];
#pragma unroll
        for (int d = 0; d < 5; ++d)
            if (d < m.dim) st.x[d][g] = v[c][d];
        if (write_w) st.w[g] = w[c];
        if (borig) borig[g] = c * 1024 + tid;
        if (with_geo) store_geometry<T>(m, geo, g, (double)v[c][0], (double)v[c][2], (double)w[c]);
    }
}

// A group's births in bearing-bucket order in one workgroup, for groups of at
// most 1024 * BS births: every thread holds up to BS births in registers
// (slots nsurv + i, i = c * 1024 + thread), the bucket histogram and its
// offsets sit in LDS, the stable rank of each birth comes chunk by chunk
// (ballot peers within a wave, earlier waves' counts of the chunk, earlier
// chunks' counts), and after a barrier every birth is written back in place
// at its rank with its geometry.  grid (K), 1024 threads.
// borig (optional): each ordered slot's drawing index; with_geo: write the
// geometry (births whose weights are already final)
template <typename T, int BS>
__global__ __launch_bounds__(1024) void k_birth_sort(DevModel m, SoA<T> st, Geo geo, const int* __restrict__ nsurv,
                                                     const int* __restrict__ ncur, int* __restrict__ borig,
                                                     int with_geo, const int* __restrict__ bkt)
{
    const int j = blockIdx.x;
    const int a = nsurv[j], nb = ncur[j] - a;
    if (nb <= 0) return;
    const int tid = threadIdx.x;
    const size_t gb = (size_t)j * m.cap + a;
    T v[BS][5], w[BS];
    int b[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        const int i = c * 1024 + tid;
        b[c] = BEARING_BUCKETS;
        if (i < nb) {
#pragma unroll
            for (int d = 0; d < 5; ++d) v[c][d] = d < m.dim ? st.x[d][gb + i] : (T)0;
            w[c] = st.w[gb + i];
            b[c] = bkt[gb + i];  // the bucket of the birth as drawn
        }
    }
    int dst[BS];
    sort_births_block<T, BS>(m, st, geo, gb, nb, v, w, b, borig, with_geo, dst);
}

// The births of the measurement-driven proposals drawn and put in bearing
// order in one workgroup per group (groups of at most 1024 * BS births):
// birth i is drawn exactly as k_birth_draw draws it (its counter, its bucket
// from the drawn position), held in registers, and written once at its rank
// with borig = i.  WEIGHT (FP32, the measurement-driven proposal, groups of
// at most BIRTH_FUSED_MAX births): the drawn positions also go to LDS (by
// drawing index, with the drawing index of every rank), and each wavefront
// then gives 64 consecutive ordered births their Eq 6 weights and geometry,
// as k_birth_weight would (the same births per wavefront, the same
// positions); else the weights are 0 until k_birth_weight.  grid (K),
// 1024 threads.
constexpr int BIRTH_FUSED_MAX = 1152;
template <typename T, int BS, int PROP, bool WEIGHT>
__global__ __launch_bounds__(1024) void k_birth_draw_sort(DevModel m, const Grp* __restrict__ gd, SoA<T> st,
                                                          Geo geo, const int* __restrict__ nsurv,
                                                          int* __restrict__ ncur,
                                                          const double* __restrict__ Zall,
                                                          const double* __restrict__ taball, int Mall,
                                                          const ZWin* __restrict__ win, uint32_t step_arg,
                                                          const uint32_t* __restrict__ dstep, int* __restrict__ borig,
                                                          int K0, ZPrep zp, int zruns, int* __restrict__ bkt)
{
    // workgroups past the K0 groups prepare the measurements of run
    // blockIdx.x - K0 for the likelihood passes (no birth reads them); the
    // ones past those, if any, predict the survivors (Step 1), 2048 slots
    // each: the births fill the slots after the survivors, so the two parts
    // touch different slots and run side by side
    if ((int)blockIdx.x >= K0) {
        const int w = (int)blockIdx.x - K0;
        if (w < zruns) {
            zprep_run<1024>(m, Zall, Mall, win, zp, w);
            return;
        }
        predict_part<T>(m, gd, st, geo, nsurv, ncur, step_of(step_arg, dstep), bkt, w - zruns, K0);
        return;
    }
    static_assert(!WEIGHT || 1024 * BS >= BIRTH_FUSED_MAX, "the fused form holds every birth");
    // a group's births are one workgroup's chain of draws, ranking and
    // weights, the launch's longest path: their wavefronts issue ahead of the
    // prediction's on a shared compute unit
    __builtin_amdgcn_s_setprio(3);
    const int j = blockIdx.x;
    const Grp gr = gd[j];
    // the births' slots [ns, min(ns + J_j, cap)), as the prediction sets them
    const int ns = nsurv[j], nb = (ns + gr.Jj < m.cap ? ns + gr.Jj : m.cap) - ns;
    if (nb <= 0) return;
    const int tid = threadIdx.x;
    const size_t gb = (size_t)j * m.cap + ns;
    const uint32_t step = step_of(step_arg, dstep);
    const BirthSrc src = birth_src(gr, win, Zall, taball, Mall);
    T v[BS][5], w[BS];
    int b[BS];
    __shared__ double s_xd[WEIGHT ? BIRTH_FUSED_MAX : 1][4];  // positions by drawing index
    __shared__ int s_inv[WEIGHT ? BIRTH_FUSED_MAX : 1];       // drawing index of each rank
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        const int i = c * 1024 + tid;
        b[c] = BEARING_BUCKETS;
        w[c] = (T)0;
        if (c * 1024 < nb && i < nb) {
            const uint32_t c0 = (uint32_t)(gr.jl * m.cap + ns + i);
            double x[4];
            draw_proposal_birth<PROP>(m, c0, step, gr.rng_run, src, x);
#pragma unroll
            for (int d = 0; d < 4; ++d) v[c][d] = (T)x[d];
            v[c][4] = m.dim == 5 ? (T)birth_turn_rate(m, c0, step, gr.rng_run) : (T)0;
            b[c] = bearing_bucket(m, x[0], x[2]);
            if constexpr (WEIGHT) {
                if (i < BIRTH_FUSED_MAX) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) s_xd[i][d] = x[d];
                }
            }
        }
    }
    int dst[BS];
    sort_births_block<T, BS>(m, st, geo, gb, nb, v, w, b, borig, 0, dst, !WEIGHT);
    if constexpr (WEIGHT) {
        if (nb > BIRTH_FUSED_MAX) return;  // (the host launches this form only below it)
#pragma unroll
        for (int c = 0; c < BS; ++c)
            if (dst[c] >= 0) s_inv[dst[c]] = c * 1024 + tid;
        __syncthreads();
        const int lane = tid & 63, wv = tid >> 6;
        for (int t0 = wv * 64; t0 < nb; t0 += 1024) {
            const int i = t0 + lane;
            const bool active = i < nb;
            double x[4];
            const int o = active ? s_inv[i] : 0;
#pragma unroll
            for (int d = 0; d < 4; ++d) x[d] = active ? s_xd[o][d] : 0.0;
            const double wt = birth_weight_at<T, PROP>(m, src, gr.Jj, x, active);
            if (active) {
                const size_t g = gb + i;
                const T tw = (T)wt;
                st.w[g] = tw;
                // the stored position is the drawn one at storage precision
                store_geometry<T>(m, geo, g, (double)(T)x[0], (double)(T)x[2], (double)tw);
            }
        }
    }
}

// births back from the other set in their sorted order, with their geometry
// (a function of the stored state).  grid (ceil(Jmax/256), K)
template <typename T>
__global__ __launch_bounds__(256) void k_bk_back(DevModel m, SoA<T> from, SoA<T> to, Geo geo,
                                                 const int* __restrict__ first, const int* __restrict__ end,
                                                 int with_geo)
{
    const int j = slot_group(m);
    const int s = first[j] + slot_tile(m) * 256 + threadIdx.x;
    if (s >= end[j]) return;
    const size_t g = (size_t)j * m.cap + s;
    // every component read before any is written (x[0] stands in for an
    // absent turn rate)
    T v[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) v[d] = from.x[d < m.dim ? d : 0][g];
    const T w = from.w[g];
#pragma unroll
    for (int d = 0; d < 5; ++d)
        if (d < m.dim) to.x[d][g] = v[d];
    const T x = v[0], y = v[2];
    to.w[g] = w;
    if (with_geo) store_geometry<T>(m, geo, g, (double)x, (double)y, (double)w);
}

// ---------------------------------------------------------------------------
// Step 5, resampling: integer-valued weights q = floor(w 2^S) and their exact
// per-tile totals (tiles of 256 ordered parents) come from k_bk_scatter.
// ---------------------------------------------------------------------------
// Number of systematic points below the cumulative boundary c:
//   N(c) = #{ m in [0, L) : (m 2^32 + r) Q < c L 2^32 }.
// A double estimate is corrected with exact 128-bit comparisons.
// (LQ = L / Q in double, formed once per workgroup: the estimate is within
// one of the count and the exact comparisons settle it)
__device__ __forceinline__ long long points_below(uint64_t c, uint64_t Q, long long L, uint32_t r, double LQ)
{
    const unsigned __int128 rhs = ((unsigned __int128)c * (unsigned __int128)(uint64_t)L) << 32;
    double est = ceil((double)c * LQ - (double)r * 0x1p-32);
    long long m0 = est < 0.0 ? 0 : (est > (double)L ? L : (long long)est);
    auto below = [&](long long mm) {
        const unsigned __int128 lhs = (unsigned __int128)((((uint64_t)mm) << 32) + (uint64_t)r) * (unsigned __int128)Q;
        return lhs < rhs;
    };
    while (m0 > 0 && !below(m0 - 1)) --m0;
    while (m0 < L && below(m0)) ++m0;
    return m0;
}

// L' = floor(N R_j + 0.5) with separate roundings (no fused multiply-add)
__device__ __forceinline__ double children_count(double N, double Rj)
{
#pragma clang fp contract(off)
    double t = N * Rj;
    t = t + 0.5;
    return floor(t);
}

// a group's child count L' from its exact quantised total Q (0: no children)
// and the mass N that Step 5 counts with (the group's 2^-S Q, or the run's
// total when one C(z) spans the groups), clamped to [0, cap - J_j]; *clamped
// tells whether the capacity cut it
__device__ __forceinline__ long long group_children(double Qd, double N, const Grp& g, int cap, bool* clamped)
{
    *clamped = false;
    if (!(Qd > 0.0)) return 0;
    double Lf = children_count(N, g.Rj);
    const double lim = (double)(cap - g.Jj);
    if (Lf > lim) {
        Lf = lim;
        *clamped = true;
    }
    if (Lf < 0.0) Lf = 0.0;
    return (long long)Lf;
}

// The run's total quantised mass, the sum over its groups, in group order, of
// 2^-S_q Q_q: the mass Step 5 counts with when one C(z) spans the groups.
// Every thread of the 256-thread workgroup gets it (contains barriers).
__device__ double run_quantised_mass(const Grp& gr, const double* __restrict__ qtot, const int* __restrict__ rsS,
                                     int K)
{
    __shared__ double s_m[256];
    __shared__ double s_tot;
    double tot = 0.0;  // thread 0's running sum
    for (int q0 = 0; q0 < gr.K; q0 += 256) {
        const int q = q0 + (int)threadIdx.x;
        if (q < gr.K) {
            const double Qq = group_q(qtot, gr.g0 + q, K);
            s_m[threadIdx.x] = Qq > 0.0 ? ldexp(Qq, -rsS[gr.g0 + q]) : 0.0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int e = gr.K - q0 < 256 ? gr.K - q0 : 256;
            for (int i = 0; i < e; ++i) tot += s_m[i];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) s_tot = tot;
    __syncthreads();
    return s_tot;
}

// ---------------------------------------------------------------------------
// Step 5, pass B: exact prefix of q, child counts and parent-order expansion
// into the other particle set.  A workgroup owns 256 NH consecutive parents
// (NH of the 256-slot tiles whose sums k_bk_scatter formed; NH = 2 where the
// capacity spans enough workgroups, else 1), thread t parents base + t,
// base + 256 + t, ...; parent i's children occupy slots [N(c_{i-1}),
// N(c_i)).  The workgroup's children form one contiguous slot range written
// with coalesced stores (each child finds its parent by binary search over
// the workgroup's child offsets in LDS).
// grid (ceil(rtiles/NH), K) (or transposed), 256 threads.
// ---------------------------------------------------------------------------
template <typename T, int NH>
__global__ __launch_bounds__(256) void k_rs_expand(DevModel m, const Grp* __restrict__ gd, SoA<T> in, SoA<T> out,
                                                   const int* __restrict__ ncur, int* __restrict__ nsurv,
                                                   const int* __restrict__ rsS, const double* __restrict__ tsum,
                                                   int rtiles, uint32_t step_arg, const uint32_t* __restrict__ dstep,
                                                   double* __restrict__ massq, int* __restrict__ clampctr,
                                                   int* __restrict__ counts, int record,
                                                   const double* __restrict__ qtot, int xchg, uint32_t xstep_arg,
                                                   const uint32_t* __restrict__ xdstep)
{
    constexpr int RS_TILE = 256 * NH;
    __shared__ long long s_end[RS_TILE];
    __shared__ long long s_first;
    __shared__ T s_x[5][RS_TILE];
    __shared__ double s_q[2 + NH][4];
    const int j = slot_group(m), t = slot_tile(m);
    const int tid = threadIdx.x, lane = tid & 63, wv = wave_in_block();
    const Grp gr = gd[j];
    const int n = ncur[j];
    const int ntl = (n + RS_TILE - 1) / RS_TILE;
    if (t > 0 && t >= ntl) return;
    const size_t gb = (size_t)j * m.cap;
    const int base = t * RS_TILE;
    const int S = rsS[j];
    // the parents' states and weights first (independent of the sums below;
    // every component read: x[0] stands in for an absent turn rate)
    bool have[NH];
    T pv[NH][5], pwt[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const int sidx = base + h * 256 + tid;
        have[h] = sidx < n;
        const size_t gs = gb + (have[h] ? sidx : 0);
#pragma unroll
        for (int d = 0; d < 5; ++d) pv[h][d] = in.x[d < m.dim ? d : 0][gs];
        pwt[h] = in.w[gs];
    }
    // Step 6 in the same pass (xchg): the run's exchange count
    // Lx = floor(rho_x min_i L'_i) from every group's total (each L'_i formed
    // exactly as group i's own workgroups form it), and the strata offsets of
    // this group and the next; child c = S_j(m) of this group is written to
    // slot S_{j+1}(m) of the next group instead of its own slot, which in
    // turn receives child S_{j-1}(m) of the previous group.  Every slot is
    // written once and no child is read, so this is the exchange of the
    // resampled set.  The run's counts are read here, with the parents, and
    // meet at the workgroup's one barrier below.
    __shared__ double s_xmin[4];
    __shared__ long long s_nnext;
    const bool xrun = xchg && gr.K >= 2;
    const int jn = gr.jl + 1 < gr.K ? gr.jl + 1 : 0;
    const double ntot = gr.gz ? run_quantised_mass(gr, qtot, rsS, m.K) : 0.0;
    uint32_t xa = 0, xan = 0;
    if (xrun) {
        // (counts below 2^31: exact in double)
        double mn = 1e300;
        for (int i = tid; i < gr.K; i += 256) {
            const int g = gr.g0 + i;
            bool c2;
            const double Qg = group_q(qtot, g, m.K);
            const double Ng = gr.gz ? ntot : (Qg > 0.0 ? ldexp(Qg, -rsS[g]) : 0.0);
            const long long Li = group_children(Qg, Ng, gd[g], m.cap, &c2);
            mn = (double)Li < mn ? (double)Li : mn;
            if (i == jn) s_nnext = Li;
        }
        mn = -wave_max(-mn);
        if (lane == 0) s_xmin[wv] = mn;
        const uint32_t xs = step_of(xstep_arg, xdstep);
        xa = rng_block(m.key0, m.key1, (uint32_t)gr.jl, xs, RNG_EXCHANGE, 0, gr.rng_run).a;
        xan = rng_block(m.key0, m.key1, (uint32_t)jn, xs, RNG_EXCHANGE, 0, gr.rng_run).a;
    }
    // group total Q and this workgroup's exclusive prefix P over the 256-slot
    // tile sums (exact integer sums), in runs of four per thread
    const int ntl256 = (n + 255) / 256, t256 = t * (RS_TILE / 256);
    double qa = 0.0, qp = 0.0;
    for (int u0 = tid; u0 < ntl256; u0 += 1024) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = tsum[(size_t)j * rtiles + (u0 + 256 * k < ntl256 ? u0 + 256 * k : u0)];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int u = u0 + 256 * k;
            if (u < ntl256) {
                qa += v[k];
                if (u < t256) qp += v[k];
            }
        }
    }
    // each parent's integer weight and its in-wave inclusive prefix, per half
    double q[NH], qin[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        q[h] = have[h] ? floor(ldexp((double)pwt[h], S)) : 0.0;
        qin[h] = wave_incl_scan(q[h]);
    }
    qa = wave_sum(qa);
    qp = wave_sum(qp);
    if (lane == 0) {
        s_q[0][wv] = qa;
        s_q[1][wv] = qp;
#pragma unroll
        for (int h = 0; h < NH; ++h) s_q[2 + h][wv] = lane_value(qin[h], 63);
    }
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        if (have[h]) {
#pragma unroll
            for (int d = 0; d < 5; ++d)
                if (d < m.dim) s_x[d][h * 256 + tid] = pv[h][d];
        }
    }
    __syncthreads();
    const double Qd = (s_q[0][0] + s_q[0][1]) + (s_q[0][2] + s_q[0][3]);
    const double Pd = (s_q[1][0] + s_q[1][1]) + (s_q[1][2] + s_q[1][3]);
    // before this thread's wave in each half, and the halves before it
    double wpre[NH], hpre[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        wpre[h] = 0.0;
        for (int w2 = 0; w2 < wv; ++w2) wpre[h] += s_q[2 + h][w2];
        hpre[h] = h == 0 ? 0.0 : hpre[h - 1] + ((s_q[1 + h][0] + s_q[1 + h][1]) + (s_q[1 + h][2] + s_q[1 + h][3]));
    }
    bool clamped = false;
    const double mq = Qd > 0.0 ? ldexp(Qd, -S) : 0.0;
    const long long L = group_children(Qd, gr.gz ? ntot : mq, gr, m.cap, &clamped);
    if (t == 0 && tid == 0) {
        if (clamped) atomicAdd(clampctr, 1);
        nsurv[j] = (int)L;
        massq[j] = mq;
    }
    long long xL = 0, xb = 0, xn = 0, xbn = 0;
    size_t xgb = 0;
    if (xrun) {
        double mn = s_xmin[0];
        for (int w2 = 1; w2 < 4; ++w2) mn = s_xmin[w2] < mn ? s_xmin[w2] : mn;
        xL = (long long)floor(m.xfrac * mn);
        if (xL > 0) {
            xn = s_nnext;
            xb = (long long)(((uint64_t)xa * (uint64_t)L) >> 32);
            xbn = (long long)(((uint64_t)xan * (uint64_t)xn) >> 32);
            xgb = (size_t)(gr.g0 + jn) * m.cap;
        }
    }
    if (L == 0 || base >= n) {
        if (record) {
#pragma unroll
            for (int h = 0; h < NH; ++h)
                if (have[h]) counts[gb + base + h * 256 + tid] = 0;
        }
        return;
    }
    const double wc = mq / (double)L;
    const uint32_t r = rng_block(m.key0, m.key1, (uint32_t)gr.jl, step_of(step_arg, dstep), RNG_RESAMPLE, 0,
                                 gr.rng_run).a;
    const uint64_t Q = (uint64_t)Qd;
    const double LQ = (double)L / Qd;
    // c_i = q_0 + ... + q_i of the group (exact: integers below 2^53)
    long long nend[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        nend[h] = points_below((uint64_t)(Pd + hpre[h] + wpre[h] + qin[h]), Q, L, r, LQ);
        s_end[h * 256 + tid] = nend[h];
    }
    if (tid == 0) s_first = points_below((uint64_t)Pd, Q, L, r, LQ);
    __syncthreads();
    if (record) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int i = h * 256 + tid;
            const long long b0 = i == 0 ? s_first : s_end[i - 1];
            if (have[h]) counts[gb + base + i] = (int)(nend[h] - b0);
        }
    }
    const long long cb = s_first, ce = s_end[RS_TILE - 1];
    const double rL = 1.0 / (double)L, rxL = xL > 0 ? 1.0 / (double)xL : 0.0;
    for (long long c = cb + tid; c < ce; c += 256) {
        // last parent li with start(li) <= c, start(0) = s_first, start(li) = s_end[li-1]
        int lo = 0, hi = RS_TILE - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_end[mid - 1] <= c) lo = mid; else hi = mid - 1;
        }
        size_t dst = gb + c;
        if (xL > 0) {
            // the stratum m with S_j(m) = floor((m L' + b_j) / Lx) = c, if any:
            // the least m with m L' + b_j >= c Lx (strata lie at least
            // L'/Lx > 1 slots apart, so there is at most one).  The quotients
            // are estimated in double (products by the workgroup's
            // reciprocals 1/L' and 1/Lx: within one of the quotient) and
            // settled by exact integer products (all below 2^53), which
            // avoids 64-bit division per child.
            const long long lo = c * xL;
            long long mm = (long long)ceil((double)(lo - xb) * rL);
            mm = mm < 0 ? 0 : mm;
            if (mm * L + xb < lo) ++mm;
            else if (mm > 0 && (mm - 1) * L + xb >= lo) --mm;
            if (mm < xL && mm * L + xb < lo + xL) {
                // S_{j+1}(m) = floor((m L'_{j+1} + b_{j+1}) / Lx)
                const long long num = mm * xn + xbn;
                long long q = (long long)floor((double)num * rxL);
                if (q * xL > num) --q;
                else if ((q + 1) * xL <= num) ++q;
                dst = xgb + (size_t)q;
            }
        }
        for (int d = 0; d < m.dim; ++d) out.x[d][dst] = s_x[d][lo];
        out.w[dst] = (T)wc;
    }
}

// ---------------------------------------------------------------------------
// Step 6, ring exchange j -> j+1 within each run.  One count L = floor(rho_x
// min_j n_j) over the run's groups; group j's chosen slots are a systematic
// sample, one per stratum: S_j(m) = floor((m n_j + b_j)/L), b_j = floor(u_j
// n_j) with u_j from the EXCHANGE stream, so S_j(m) sits at the quantile m/L
// of the group's slot order (kept in bearing order by the resampling); the
// couple in S_j(m) replaces the one in S_{j+1}(m).  A gather into a staging
// buffer followed by a scatter (two launches) makes every read see the state
// before the exchange, so the exchange is a permutation of the particles.
// grid (ceil(Lmax/256), groups).
// ---------------------------------------------------------------------------
// exchange count L = floor(rho_x min_j n_j) over the run's groups; called by
// all threads of a workgroup
__device__ __forceinline__ int exchange_count(const DevModel& m, const Grp& gr, const int* __restrict__ nsurv)
{
    __shared__ int s_min[4];
    int mn = 2147483647;
    for (int j = threadIdx.x; j < gr.K; j += 256) mn = nsurv[gr.g0 + j] < mn ? nsurv[gr.g0 + j] : mn;
    mn = -wave_max(-mn);
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = mn;
    __syncthreads();
    mn = s_min[0];
    for (int w = 1; w < 4; ++w) mn = s_min[w] < mn ? s_min[w] : mn;
    return (int)floor(m.xfrac * (double)mn);
}

__device__ __forceinline__ uint64_t exchange_slot(const DevModel& m, const Grp& gr, int jl, int nj, int L, int mm,
                                                  uint32_t step)
{
    const Block4 a = rng_block(m.key0, m.key1, (uint32_t)jl, step, RNG_EXCHANGE, 0, gr.rng_run);
    const uint64_t b = ((uint64_t)a.a * (uint64_t)nj) >> 32;
    return ((uint64_t)mm * (uint64_t)nj + b) / (uint64_t)L;
}

template <typename T>
__global__ __launch_bounds__(256) void k_xchg_gather(DevModel m, const Grp* __restrict__ gd, SoA<T> st,
                                                     const int* __restrict__ nsurv, T* __restrict__ stage, int Lmax,
                                                     uint32_t step_arg, const uint32_t* __restrict__ dstep)
{
    const int j = slot_group(m);
    const Grp gr = gd[j];
    if (gr.K < 2) return;
    const int mm = slot_tile(m) * 256 + threadIdx.x;
    const int L = exchange_count(m, gr, nsurv);
    if (mm >= L || mm >= Lmax) return;
    const uint32_t step = step_of(step_arg, dstep);
    const size_t src = (size_t)j * m.cap + (size_t)exchange_slot(m, gr, gr.jl, nsurv[j], L, mm, step);
    T* o = stage + ((size_t)j * Lmax + mm) * 6;
    T v[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) v[d] = st.x[d < m.dim ? d : 0][src];
    const T wv = st.w[src];
#pragma unroll
    for (int d = 0; d < 5; ++d)
        if (d < m.dim) o[d] = v[d];
    o[5] = wv;
}

template <typename T>
__global__ __launch_bounds__(256) void k_xchg_scatter(DevModel m, const Grp* __restrict__ gd, SoA<T> st,
                                                      const int* __restrict__ nsurv, const T* __restrict__ stage,
                                                      int Lmax, uint32_t step_arg, const uint32_t* __restrict__ dstep)
{
    const int j = slot_group(m);
    const Grp gr = gd[j];
    if (gr.K < 2) return;
    const int mm = slot_tile(m) * 256 + threadIdx.x;
    const int L = exchange_count(m, gr, nsurv);
    if (mm >= L || mm >= Lmax) return;
    const uint32_t step = step_of(step_arg, dstep);
    const int jln = (gr.jl + 1) % gr.K;
    const int jn = gr.g0 + jln;
    const size_t dst = (size_t)jn * m.cap + (size_t)exchange_slot(m, gr, jln, nsurv[jn], L, mm, step);
    const T* o = stage + ((size_t)j * Lmax + mm) * 6;
    T v[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) v[d] = o[d];
#pragma unroll
    for (int d = 0; d < 5; ++d)
        if (d < m.dim) st.x[d][dst] = v[d];
    st.w[dst] = v[5];
}

// Step 6 in one launch for runs of at most 1024 groups: stratum m moves one
// couple per group, S_j(m) -> S_{j+1}(m), so a workgroup that holds whole
// strata of one run (1024 / K_r strata, thread = (group, stratum)) reads its
// couples, waits, and writes each to the next group's slot of the same
// stratum.  Workgroups touch different strata, so every read still sees the
// state before the exchange.  The run's count L and each group's offset b_j
// are formed once per workgroup.  grid (runs, ceil(Lmax / (1024 / K_r))).
template <typename T>
__global__ __launch_bounds__(1024) void k_xchg_ring(DevModel m, const Grp* __restrict__ rgd, SoA<T> st,
                                                   const int* __restrict__ nsurv, int Lmax, uint32_t step_arg,
                                                   const uint32_t* __restrict__ dstep)
{
    __shared__ T s_c[6][1024];
    __shared__ uint64_t s_b[1024];
    __shared__ int s_n[1024];
    __shared__ int s_min[16];
    const Grp g0 = rgd[blockIdx.x];  // the run's first group
    const int Kr = g0.K;
    if (Kr < 2 || Kr > 1024) return;
    const int spb = 1024 / Kr;
    if ((int)blockIdx.y * spb >= Lmax) return;  // whole workgroup idle
    const uint32_t step = step_of(step_arg, dstep);
    const int tid = threadIdx.x;
    int mn = 2147483647;
    if (tid < Kr) {
        const int n = nsurv[g0.g0 + tid];
        const Block4 a = rng_block(m.key0, m.key1, (uint32_t)tid, step, RNG_EXCHANGE, 0, g0.rng_run);
        s_n[tid] = n;
        s_b[tid] = ((uint64_t)a.a * (uint64_t)n) >> 32;
        mn = n;
    }
    mn = -wave_max(-mn);
    if ((tid & 63) == 0) s_min[tid >> 6] = mn;
    __syncthreads();
    mn = s_min[0];
    for (int w = 1; w < 16; ++w) mn = s_min[w] < mn ? s_min[w] : mn;
    const int L = (int)floor(m.xfrac * (double)mn);
    // stratum fastest: neighbouring lanes take neighbouring strata of one
    // group, whose slots lie about n/L apart
    const int jl = tid / spb, ml = tid - jl * spb;
    const int mm = (int)blockIdx.y * spb + ml;
    const bool live = jl < Kr && mm < L;
    if (live) {
        const size_t src = (size_t)(g0.g0 + jl) * m.cap + ((uint64_t)mm * (uint64_t)s_n[jl] + s_b[jl]) / (uint64_t)L;
        // every component read at once (x[0] stands in for an absent turn rate)
        T v[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) v[d] = st.x[d < m.dim ? d : 0][src];
        const T wv = st.w[src];
#pragma unroll
        for (int d = 0; d < 5; ++d) s_c[d][tid] = v[d];
        s_c[5][tid] = wv;
    }
    __syncthreads();
    if (live) {
        const int jn = jl + 1 < Kr ? jl + 1 : 0;
        const size_t dst = (size_t)(g0.g0 + jn) * m.cap + ((uint64_t)mm * (uint64_t)s_n[jn] + s_b[jn]) / (uint64_t)L;
        for (int d = 0; d < m.dim; ++d) st.x[d][dst] = s_c[d][tid];
        st.w[dst] = s_c[5][tid];
    }
}

// ---------------------------------------------------------------------------
// Batched updates: the runs' measurement windows as given, clamped into the
// step's set (count to [0, max_meas], the window inside [0, zrows)), so no
// window can lead a kernel outside the set.  grid (ceil(runs/256)).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_windows(const int32_t* __restrict__ uw, int nruns, int zrows,
                                                       int max_meas, ZWin* __restrict__ win)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= nruns) return;
    int off = uw[2 * r], M = uw[2 * r + 1];
    M = M < 0 ? 0 : (M > max_meas ? max_meas : M);
    M = M > zrows ? zrows : M;
    off = off < 0 ? 0 : off;
    off = off > zrows - M ? zrows - M : off;
    win[r] = ZWin{ off, M };
}

// advances the step counter of a captured step (one thread)
__global__ void k_step_next(uint32_t* dstep)
{
    if (threadIdx.x == 0) dstep[0] = dstep[0] + 1u;
}

}  // namespace pphd
