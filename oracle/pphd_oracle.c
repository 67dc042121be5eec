/*
 * Oracle for the distributed particle PHD filter -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64, single thread, no blocking or fusion: every function follows one
 * step of the paper in the paper's order and notation so that it can be read
 * against the text.  Built with -O2 -ffp-contract=off (no fused multiply-add),
 * so every expression rounds exactly as written.  See pphd_oracle.h for the
 * state layout.  Only the test suite, the smoke check and the CPU baseline of
 * the benchmark may load this file; the GPU library never does.
 *
 * Readings of points the paper leaves open are marked "Reading:".
 */
#include <omp.h>
#include "pphd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Random numbers.                                                           */
/* ------------------------------------------------------------------------ */

/* Philox-4x32-10 block function (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11).  Each of the ten rounds multiplies
 * counter words 0 and 2 by the two round multipliers (full 64-bit products);
 * the new word 0 is hi(M1*c2) ^ c1 ^ k0, word 1 is lo(M1*c2), word 2 is
 * hi(M0*c0) ^ c3 ^ k1 and word 3 is lo(M0*c0).  The key is advanced by the two
 * Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void orc_block(uint64_t seed, uint32_t c0, uint32_t step, uint32_t purpose,
                      uint32_t sub, uint32_t run, uint32_t out[4])
{
    uint32_t ctr[4] = { c0, step, purpose * 16u + sub, run };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform on (0, 1]: the 53-bit integer formed from all of a and the top 21
 * bits of b, plus one, times 2^-53 (exact in FP64). */
/* Threads of the per-group loops (OpenMP; results do not depend on it). */
void orc_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}
int orc_threads(void)
{
    return omp_get_max_threads();
}

double orc_u53(uint32_t a, uint32_t b)
{
    uint64_t k = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return ldexp((double)(k + 1u), -53);
}

/* Box-Muller transform: two independent standard normals from two uniforms. */
void orc_normal_pair(double u1, double u2, double* n1, double* n2)
{
    double rad = sqrt(-2.0 * log(u1));
    *n1 = rad * cos(2.0 * ORC_PI * u2);
    *n2 = rad * sin(2.0 * ORC_PI * u2);
}

/* ------------------------------------------------------------------------ */
/* Model pieces (section 4 simulation model; parameter values are inputs).  */
/* ------------------------------------------------------------------------ */

/* Step 1 of section 3.1 splits the J births equally over the K groups.
 * Reading: the first J mod K groups take one extra birth. */
int orc_births_in_partition(const orc_model* m, int j)
{
    int K = m->partitions, J = m->births_per_step;
    return J / K + (j < J % K ? 1 : 0);
}

/* Clutter intensity kappa(z) = lambda * c(z) with c uniform over the
 * range-bearing region (section 4, Poisson clutter). */
double orc_kappa(const orc_model* m)
{
    double area = (m->r_max - m->r_min) * (m->th_max - m->th_min);
    return m->clutter_rate / area;
}

/* The global-C reading of Eq 11 (global_cz = 1).  Eq 11 sums over one
 * group's particles; read instead as one C_k(z) over every group, the K
 * particle sets become K parts of a single PHD, each carrying 1/K of its
 * mass: the initial mass and the birth mass are split over the groups
 * (omega_0 = 1/(M K)).  The target number is then the run's total mass:
 * Step 3 takes LT = round(sum over groups of their masses) in every group,
 * and Step 5 allocates children non-proportionally, as in the DRNA scheme
 * the method builds on: every group draws round(N_total R_j) children (its
 * share of the particles for the whole PHD), each of weight N_j / L'_j, so
 * that a group's weight, not its particle count, carries its share of the
 * mass.  With global_cz = 0 every quantity below is the paper's per-group
 * one. */
static double orc_birth_mass(const orc_model* m)
{
    return m->global_cz ? m->birth_mass / (double)m->partitions : m->birth_mass;
}
static double orc_init_mass(const orc_model* m)
{
    return m->global_cz ? m->init_mass / (double)m->partitions : m->init_mass;
}
/* the mass that Step 3's LT and Step 5's child count take for group j:
 * its own, or (global_cz) the run's total, added in group order */
static double orc_count_mass(const orc_model* m, const double* mass, int j)
{
    if (!m->global_cz) return mass[j];
    double tot = 0.0;
    for (int q = 0; q < m->partitions; ++q) tot += mass[q];
    return tot;
}

static double orc_wrap(double d)
{
    /* Reading: the bearing residual is taken modulo 2*pi into [-pi, pi). */
    return d - 2.0 * ORC_PI * floor((d + ORC_PI) / (2.0 * ORC_PI));
}

/* Single-target likelihood g(z | x) of the range-bearing sensor of section 4:
 * z = [R, theta] + v with R the distance to the sensor, theta the bearing
 * (atan2), and v independent zero-mean Gaussian noise (sigma_r, sigma_theta).
 * Reading: untruncated product of the two Gaussian densities. */
double orc_likelihood(const orc_model* m, double zr, double zth, double x, double y)
{
    double dx = x - m->sensor_x, dy = y - m->sensor_y;
    double range = sqrt(dx * dx + dy * dy);
    double bearing = atan2(dy, dx);
    double er = (zr - range) / m->sigma_r;
    double et = orc_wrap(zth - bearing) / m->sigma_theta;
    double norm = 1.0 / (2.0 * ORC_PI * m->sigma_r * m->sigma_theta);
    return norm * exp(-0.5 * (er * er + et * et));
}

/* Draw one particle from the normalised birth density gamma/m_b:
 * position uniform over the surveillance region, velocity N(0, sigma_v^2 I)
 * (birth_density 0; reading: a uniform birth density stands in for the
 * paper's Gaussian one on the large workloads), or the Gaussian N(x_bar, Q)
 * of section 4 with diagonal Q (birth_density 1). */
static void orc_draw_birth(const orc_model* m, uint64_t seed, uint32_t c0, uint32_t step,
                           uint32_t purpose, uint32_t run, double s[5])
{
    uint32_t a[4], b[4];
    orc_block(seed, c0, step, purpose, 0, run, a);
    orc_block(seed, c0, step, purpose, 1, run, b);
    s[4] = 0.0;
    if (m->dim == 5) {
        /* turn rate N(0, birth_sigma_w^2) from a third block */
        uint32_t c[4];
        double w1, w2;
        orc_block(seed, c0, step, purpose, 2, run, c);
        orc_normal_pair(orc_u53(c[0], c[1]), orc_u53(c[2], c[3]), &w1, &w2);
        s[4] = m->birth_sigma_w * w1;
    }
    double ux = orc_u53(a[0], a[1]), uy = orc_u53(a[2], a[3]);
    double n1, n2;
    orc_normal_pair(orc_u53(b[0], b[1]), orc_u53(b[2], b[3]), &n1, &n2);
    if (m->birth_density == 1) {
        /* the paper's Gaussian birth intensity (section 4): position normals
         * from the first block, velocity normals from the second */
        double p1, p2;
        orc_normal_pair(ux, uy, &p1, &p2);
        s[0] = m->birth_mean[0] + m->birth_std[0] * p1;
        s[1] = m->birth_mean[1] + m->birth_std[1] * n1;
        s[2] = m->birth_mean[2] + m->birth_std[2] * p2;
        s[3] = m->birth_mean[3] + m->birth_std[3] * n2;
        return;
    }
    s[0] = m->region[0] + ux * (m->region[1] - m->region[0]);
    s[1] = m->birth_sigma_v * n1;
    s[2] = m->region[2] + uy * (m->region[3] - m->region[2]);
    s[3] = m->birth_sigma_v * n2;
}

#define XS(X, d, g) (X)[(size_t)(d) * (size_t)KC + (size_t)(g)]

/* ------------------------------------------------------------------------ */
/* t = 0 (section 3.1): M particles per group with equal weights.            */
/* ------------------------------------------------------------------------ */
int orc_init(const orc_model* m, int cap, uint64_t seed, uint32_t run,
             double* X, double* W, int32_t* n)
{
    int K = m->partitions;
    size_t KC = (size_t)K * (size_t)cap;
    double Rj = m->particles_per_target / (double)K;
    int M0 = (int)floor(Rj + 0.5);
    if (M0 < 1) M0 = 1;
    if (M0 > cap) return -3;
    for (int j = 0; j < K; ++j) {
        for (int s = 0; s < M0; ++s) {
            uint32_t g = (uint32_t)(j * cap + s);
            double st[5];
            orc_draw_birth(m, seed, g, 0, ORC_INIT, run, st);
            for (int d = 0; d < m->dim; ++d) XS(X, d, g) = st[d];
            /* Reading: omega_0 = 1/M generalises to init_mass / M. */
            W[g] = orc_init_mass(m) / (double)M0;
        }
        n[j] = M0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 1, prediction (Eqs 5 and 6; algorithm 1, first two loops).           */
/* ------------------------------------------------------------------------ */
int orc_predict(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                double* X, double* W, int32_t* n)
{
    int K = m->partitions;
    size_t KC = (size_t)K * (size_t)cap;
    double T = m->T;
    /* Constant-velocity transition and noise gain of section 4. */
    double F[4][4] = { { 1, T, 0, 0 }, { 0, 1, 0, 0 }, { 0, 0, 1, T }, { 0, 0, 0, 1 } };
    /* Reading: the gain column per axis is [T^2/2, T] (the paper prints 1,
     * which equals T at T = 1). */
    double G[4][2] = { { T * T / 2, 0 }, { T, 0 }, { 0, T * T / 2 }, { 0, T } };
    for (int j = 0; j < K; ++j)
        if (n[j] + orc_births_in_partition(m, j) > cap) return -3;
    /* groups are independent: one thread per group (results do not depend
     * on the thread count) */
    int err = 0;
#pragma omp parallel for schedule(dynamic) reduction(min : err)
    for (int j = 0; j < K; ++j) {
        int Jj = orc_births_in_partition(m, j);
        int ns = n[j];
        /* Survivors, Eq 5 with proposal q = f and no spawning:
         * x~ = F x + Gamma (sigma_a * nu), weight phi/q * w = p_S * w. */
        for (int s = 0; s < ns; ++s) {
            uint32_t g = (uint32_t)(j * cap + s);
            uint32_t r[4];
            orc_block(seed, g, step, ORC_PREDICT, 0, run, r);
            double v[2];
            orc_normal_pair(orc_u53(r[0], r[1]), orc_u53(r[2], r[3]), &v[0], &v[1]);
            v[0] *= m->sigma_a;
            v[1] *= m->sigma_a;
            double x[4], y[4];
            for (int d = 0; d < 4; ++d) x[d] = XS(X, d, g);
            if (m->dim == 5) {
                /* Coordinated turn at the particle's rate w (not in the paper;
                 * the textbook model): the velocity turns by wT and the
                 * position follows the arc, x' = x + (sin wT / w) vx -
                 * ((1 - cos wT) / w) vy, y' = y + ((1 - cos wT) / w) vx +
                 * (sin wT / w) vy, with the limits T and 0 at w = 0; then
                 * the same acceleration noise as the CV model, and
                 * w' = w + T sigma_w n. */
                double w = XS(X, 4, g);
                double sn = sin(w * T), cs = cos(w * T);
                double fa = w != 0.0 ? sn / w : T;
                double fb = w != 0.0 ? (1.0 - cs) / w : 0.0;
                double Fc[4][4] = { { 1, fa, 0, -fb }, { 0, cs, 0, -sn }, { 0, fb, 1, fa }, { 0, sn, 0, cs } };
                for (int a = 0; a < 4; ++a) {
                    double acc = 0.0;
                    for (int b = 0; b < 4; ++b) acc += Fc[a][b] * x[b];
                    for (int b = 0; b < 2; ++b) acc += G[a][b] * v[b];
                    y[a] = acc;
                }
                uint32_t r2[4];
                double nw1, nw2;
                orc_block(seed, g, step, ORC_PREDICT, 1, run, r2);
                orc_normal_pair(orc_u53(r2[0], r2[1]), orc_u53(r2[2], r2[3]), &nw1, &nw2);
                XS(X, 4, g) = w + T * m->sigma_w * nw1;
            } else {
                for (int a = 0; a < 4; ++a) {
                    double acc = 0.0;
                    for (int b = 0; b < 4; ++b) acc += F[a][b] * x[b];
                    for (int b = 0; b < 2; ++b) acc += G[a][b] * v[b];
                    y[a] = acc;
                }
            }
            for (int d = 0; d < 4; ++d) XS(X, d, g) = y[d];
            W[g] = m->p_S * W[g];
        }
        /* Births, Eq 6 with proposal p_k = gamma / m_b: weight m_b / J_j.
         * Reading: each group carries the full birth mass (J_j births).
         * With the measurement-driven proposal the J_j slots are reserved
         * here and drawn by orc_birth_from_measurements once Z_k is known. */
        for (int b = 0; b < Jj && m->birth_proposal == 0; ++b) {
            uint32_t g = (uint32_t)(j * cap + ns + b);
            double st[5];
            orc_draw_birth(m, seed, g, step, ORC_BIRTH, run, st);
            for (int d = 0; d < m->dim; ++d) XS(X, d, g) = st[d];
            W[g] = orc_birth_mass(m) / (double)Jj;
        }
        if (m->birth_proposal == 0 && orc_sort_by_bucket(m, KC, X, W, (size_t)j * cap + ns, Jj) != 0) err = -2;
        n[j] = ns + Jj;
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* Births from a measurement-driven proposal p_k(. | Z_k) (Eq 6).            */
/* Reading: the proposal is the defensive mixture                            */
/*   q(x) = alpha gamma(x)/m_b + (1 - alpha) (1/M) sum_p q_p(x),              */
/* where q_p draws R ~ N(r_p, sigma_r^2), Theta ~ N(theta_p, sigma_theta^2)   */
/* (the inverse of the sensor model) and puts the particle at                */
/* s + R (cos Theta, sin Theta), with velocity N(0, sigma_v^2 I) as in the    */
/* birth density.  The weight of Eq 6 is gamma(x) / (J_j q(x)); the velocity */
/* factors cancel, leaving m_b U(x) / (J_j q_pos(x)) with U the uniform       */
/* density of the surveillance region.                                        */
/* ------------------------------------------------------------------------ */

/* dim 5: the turn rate of a birth drawn from a measurement-driven or learned
 * proposal comes from the birth density's own N(0, birth_sigma_w^2) (block
 * sub 4), so its density cancels in the Eq 6 weight. */
static void orc_birth_turn_rate(const orc_model* m, uint64_t seed, uint32_t g, uint32_t step, uint32_t run,
                                double* X, size_t KC)
{
    if (m->dim != 5) return;
    uint32_t c[4];
    double w1, w2;
    orc_block(seed, g, step, ORC_BIRTH, 4, run, c);
    orc_normal_pair(orc_u53(c[0], c[1]), orc_u53(c[2], c[3]), &w1, &w2);
    XS(X, 4, g) = m->birth_sigma_w * w1;
}

static double orc_gauss(double d, double sigma)
{
    double e = d / sigma;
    return exp(-0.5 * e * e) / (sqrt(2.0 * ORC_PI) * sigma);
}

/* Position density of the proposal at (x, y).  A point at distance rho and
 * bearing phi is reached by R = rho, Theta = phi (mod 2 pi) and by R = -rho,
 * Theta = phi + pi (mod 2 pi); the Jacobian of the polar map is 1/rho.  The
 * wrapped normal of Theta is represented by its nearest branch (the others
 * are below exp(-(pi/sigma_theta)^2/2)). */
double orc_birth_proposal_density(const orc_model* m, const double* Z, int M, double x, double y)
{
    double area = (m->region[1] - m->region[0]) * (m->region[3] - m->region[2]);
    int inside = x >= m->region[0] && x <= m->region[1] && y >= m->region[2] && y <= m->region[3];
    double u = inside ? 1.0 / area : 0.0;
    if (M == 0) return u;
    double dx = x - m->sensor_x, dy = y - m->sensor_y;
    double rho = sqrt(dx * dx + dy * dy);
    double phi = atan2(dy, dx);
    double mix = 0.0;
    for (int p = 0; p < M; ++p) {
        double a = orc_gauss(rho - Z[2 * p], m->sigma_r) * orc_gauss(orc_wrap(phi - Z[2 * p + 1]), m->sigma_theta);
        double b = orc_gauss(rho + Z[2 * p], m->sigma_r) * orc_gauss(orc_wrap(phi + ORC_PI - Z[2 * p + 1]), m->sigma_theta);
        mix += (a + b) / rho;
    }
    return m->birth_alpha * u + (1.0 - m->birth_alpha) * mix / (double)M;
}

int orc_birth_from_measurements(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                                const double* Z, int M, double* X, double* W, const int32_t* n)
{
    int K = m->partitions;
    size_t KC = (size_t)K * (size_t)cap;
    double area = (m->region[1] - m->region[0]) * (m->region[3] - m->region[2]);
    for (int j = 0; j < K; ++j)
        if (n[j] < orc_births_in_partition(m, j)) return -1;
    int err = 0;
#pragma omp parallel for schedule(dynamic) reduction(min : err)
    for (int j = 0; j < K; ++j) {
        int Jj = orc_births_in_partition(m, j);
        int ns = n[j] - Jj;
        for (int b = 0; b < Jj; ++b) {
            uint32_t g = (uint32_t)(j * cap + ns + b);
            uint32_t a[4], v[4], c[4];
            orc_block(seed, g, step, ORC_BIRTH, 0, run, a);
            orc_block(seed, g, step, ORC_BIRTH, 1, run, v);
            orc_block(seed, g, step, ORC_BIRTH, 2, run, c);
            double u1 = orc_u53(a[0], a[1]), u2 = orc_u53(a[2], a[3]);
            double uc = orc_u53(c[0], c[1]);
            double x, y;
            if (M == 0 || uc <= m->birth_alpha) {
                x = m->region[0] + u1 * (m->region[1] - m->region[0]);
                y = m->region[2] + u2 * (m->region[3] - m->region[2]);
            } else {
                int p = (int)floor((uc - m->birth_alpha) / (1.0 - m->birth_alpha) * (double)M);
                if (p > M - 1) p = M - 1;
                double e1, e2;
                orc_normal_pair(u1, u2, &e1, &e2);
                double R = Z[2 * p] + m->sigma_r * e1;
                double Th = Z[2 * p + 1] + m->sigma_theta * e2;
                x = m->sensor_x + R * cos(Th);
                y = m->sensor_y + R * sin(Th);
            }
            double n1, n2;
            orc_normal_pair(orc_u53(v[0], v[1]), orc_u53(v[2], v[3]), &n1, &n2);
            XS(X, 0, g) = x;
            XS(X, 1, g) = m->birth_sigma_v * n1;
            XS(X, 2, g) = y;
            XS(X, 3, g) = m->birth_sigma_v * n2;
            orc_birth_turn_rate(m, seed, g, step, run, X, KC);
            int inside = x >= m->region[0] && x <= m->region[1] && y >= m->region[2] && y <= m->region[3];
            double q = orc_birth_proposal_density(m, Z, M, x, y);
            W[g] = inside ? orc_birth_mass(m) * (1.0 / area) / ((double)Jj * q) : 0.0;
        }
        if (orc_sort_by_bucket(m, KC, X, W, (size_t)j * cap + ns, Jj) != 0) err = -2;
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* Step 2, update with the measurement-labelled decomposition (Eqs 10-15),   */
/* plus the sums of Step 3 (Eqs 16-18).                                      */
/*   C[j*M+p]          C_k(z_p) of group j, Eq 11 (Eq 7 restricted to j)      */
/*   dW[j*M+p]         Delta W^{j,p}, Eq 16                                   */
/*   dW0[j]            Delta W^{j,0}, Eq 17                                   */
/*   zeta_num[(j*M+p)*4+d]  sum_i Delta w^{i,p,j} x~_i[d] (numerator of Eq 18) */
/*   mass[j]           sum_i w~_k^{i,j} after the update                      */
/* W is overwritten with the updated weights (Eq 15).                        */
/* Reading: C is computed per group, over the group's own particles.         */
/* With global_cz = 1 (the global-C reading) C still holds each group's own  */
/* C_j(z_p), but the denominator of Eq 12 is kappa + sum_j C_j(z_p) over all */
/* groups, added in group order.                                             */
/* ------------------------------------------------------------------------ */
static double* orc_psi(const orc_model* m, size_t KC, const double* Z, int M, const double* X, size_t base, int nj)
{
    /* psi_{k,z}(x) = p_D g(z|x) for every particle/measurement pair. */
    double* psi = (double*)malloc(sizeof(double) * (size_t)(nj > 0 ? nj : 1) * (size_t)(M > 0 ? M : 1));
    if (!psi) return NULL;
    for (int i = 0; i < nj; ++i)
        for (int p = 0; p < M; ++p)
            psi[(size_t)i * M + p] = m->p_D * orc_likelihood(m, Z[2 * p], Z[2 * p + 1],
                                                             XS(X, 0, base + i), XS(X, 2, base + i));
    return psi;
}

int orc_update(const orc_model* m, int cap, const double* Z, int M,
               const double* X, double* W, const int32_t* n,
               double* C, double* dW, double* dW0, double* zeta_num, double* mass)
{
    int K = m->partitions;
    size_t KC = (size_t)K * (size_t)cap;
    double kappa = orc_kappa(m);
    double nu = 1.0 - m->p_D; /* nu(x) = 1 - P_D(x), from Eq 4 */
    /* the global C of every measurement (global_cz = 1): each group's Eq 11
     * first, then their sum */
    double* Cg = NULL;
    int err = 0;
    if (m->global_cz) {
        Cg = (double*)calloc((size_t)(M > 0 ? M : 1), sizeof(double));
        if (!Cg) return -2;
#pragma omp parallel for schedule(dynamic) reduction(min : err)
        for (int j = 0; j < K; ++j) {
            size_t base = (size_t)j * (size_t)cap;
            double* psi = orc_psi(m, KC, Z, M, X, base, n[j]);
            if (!psi) { err = -2; continue; }
            for (int p = 0; p < M; ++p) {
                double c = 0.0;
                for (int i = 0; i < n[j]; ++i) c += psi[(size_t)i * M + p] * W[base + i];
                C[(size_t)j * M + p] = c;
            }
            free(psi);
        }
        if (err) { free(Cg); return err; }
        for (int p = 0; p < M; ++p)
            for (int j = 0; j < K; ++j) Cg[p] += C[(size_t)j * M + p];
    }
    /* groups are independent once C is known: one thread per group */
#pragma omp parallel for schedule(dynamic) reduction(min : err)
    for (int j = 0; j < K; ++j) {
        int nj = n[j];
        size_t base = (size_t)j * (size_t)cap;
        double* psi = orc_psi(m, KC, Z, M, X, base, nj);
        if (!psi) { err = -2; continue; }
        /* Eq 11 */
        for (int p = 0; p < M; ++p) {
            double c = 0.0;
            for (int i = 0; i < nj; ++i) c += psi[(size_t)i * M + p] * W[base + i];
            C[(size_t)j * M + p] = c;
        }
        for (int p = 0; p < M; ++p) {
            dW[(size_t)j * M + p] = 0.0;
            for (int d = 0; d < 4; ++d) zeta_num[((size_t)j * M + p) * 4 + d] = 0.0;
        }
        double w0sum = 0.0, msum = 0.0;
        for (int i = 0; i < nj; ++i) {
            double wpred = W[base + i];
            double wnew = 0.0;
            for (int p = 0; p < M; ++p) {
                /* Eq 12 and Eq 13 */
                double den = kappa + (Cg ? Cg[p] : C[(size_t)j * M + p]);
                double G = psi[(size_t)i * M + p] / den;
                double dw = G * wpred;
                wnew += dw;
                dW[(size_t)j * M + p] += dw;                       /* Eq 16 */
                for (int d = 0; d < 4; ++d)                          /* Eq 18 numerator */
                    zeta_num[((size_t)j * M + p) * 4 + d] += dw * XS(X, d, base + i);
            }
            double dw0 = nu * wpred;                                 /* Eq 14 */
            wnew += dw0;                                             /* Eq 15 */
            w0sum += dw0;                                            /* Eq 17 */
            W[base + i] = wnew;
            msum += wnew;
        }
        dW0[j] = w0sum;
        mass[j] = msum;
        free(psi);
    }
    free(Cg);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Step 3, local estimation.                                                 */
/*   LT_j = round(sum of the group's updated weights).                       */
/*   I_j  = the LT_j measurements with the largest Delta W^{j,p}.            */
/*   zeta_{j,l} = sum_i Delta w^{i,l,j} x~_i / Delta W^{j,l}   (Eq 18).       */
/* Readings: round(x) = floor(x + 0.5); LT is capped at M_k; ties in Delta W */
/* go to the lower measurement index; a measurement with Delta W = 0 carries */
/* no particle support and is never selected.                                */
/* ------------------------------------------------------------------------ */
int orc_extract(const orc_model* m, int M, const double* dW, const double* zeta_num,
                const double* mass, int32_t* LT, int32_t* sel, double* zeta)
{
    int K = m->partitions;
    for (int j = 0; j < K; ++j) {
        double lt = floor(orc_count_mass(m, mass, j) + 0.5);
        int L = lt < 0 ? 0 : (lt > (double)M ? M : (int)lt);
        LT[j] = L;
        for (int p = 0; p < M; ++p) {
            sel[(size_t)j * M + p] = 0;
            for (int d = 0; d < 4; ++d) zeta[((size_t)j * M + p) * 4 + d] = 0.0;
        }
        for (int t = 0; t < L; ++t) {
            int best = -1;
            for (int p = 0; p < M; ++p) {
                if (sel[(size_t)j * M + p]) continue;
                if (!(dW[(size_t)j * M + p] > 0.0)) continue;
                if (best < 0 || dW[(size_t)j * M + p] > dW[(size_t)j * M + best]) best = p;
            }
            if (best < 0) break;
            sel[(size_t)j * M + best] = 1;
            for (int d = 0; d < 4; ++d)
                zeta[((size_t)j * M + best) * 4 + d] =
                    zeta_num[((size_t)j * M + best) * 4 + d] / dW[(size_t)j * M + best];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 4, global estimation at the central unit.  Local estimates that     */
/* carry the same measurement label are averaged; a label is kept only when */
/* more than half of the K groups report it.                                 */
/* Readings: strict majority (2*votes > K); unweighted mean over the         */
/* reporting groups in group order; output sorted by label.                  */
/* ------------------------------------------------------------------------ */
int orc_fuse(const orc_model* m, int M, const int32_t* sel, const double* zeta,
             double* est_state, int32_t* est_label, int32_t* est_votes, int32_t* n_est)
{
    int K = m->partitions;
    int cnt = 0;
    for (int p = 0; p < M; ++p) {
        int votes = 0;
        double acc[4] = { 0, 0, 0, 0 };
        for (int j = 0; j < K; ++j) {
            if (!sel[(size_t)j * M + p]) continue;
            votes += 1;
            for (int d = 0; d < 4; ++d) acc[d] += zeta[((size_t)j * M + p) * 4 + d];
        }
        if (2 * votes > K) {
            for (int d = 0; d < 4; ++d) est_state[(size_t)cnt * 4 + d] = acc[d] / (double)votes;
            est_label[cnt] = p;
            est_votes[cnt] = votes;
            cnt += 1;
        }
    }
    *n_est = cnt;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 5, local resampling (algorithm 1: the M+J_k particles of a group     */
/* become N_k(j) R_k particles).                                             */
/* Readings:                                                                 */
/*  - R_j = particles per target in each group = R / K.                      */
/*  - The scheme is systematic resampling with one uniform per group.        */
/*  - Weights are first quantised to integers q_i = floor(w_i 2^S), with S   */
/*    the largest shift that keeps the group total below 2^52, so that the   */
/*    cumulative sums are exact in any order.  The group mass is then        */
/*    N = Q 2^-S with Q = sum q_i, the new size is L' = floor(N R_j + 0.5)   */
/*    clamped to [0, cap - J_j], and every child carries weight N / L'.      */
/*  - Children are written in parent order.                                  */
/* counts[j*cap+i] receives the number of children of parent slot i.         */
/* ------------------------------------------------------------------------ */
/* Bearing bucket of a position, 0 .. ORC_BUCKETS-1: the "diamond angle"
 * d in [0, 4) of the offset from the sensor (a monotonic stand-in for the
 * bearing measured counter-clockwise from the +x axis, computed with one
 * correctly rounded division), times ORC_BUCKETS/4, rounded down. */
#define ORC_BUCKETS 64
int orc_bearing_bucket(const orc_model* m, double x, double y)
{
    double dx = x - m->sensor_x, dy = y - m->sensor_y;
    double d;
    if (dx == 0.0 && dy == 0.0) d = 0.0;
    else if (dy >= 0.0) d = dx >= 0.0 ? dy / (dx + dy) : 1.0 - dx / (dy - dx);
    else d = dx < 0.0 ? 2.0 - dy / (-dx - dy) : 3.0 + dx / (dx - dy);
    int b = (int)floor(d * (ORC_BUCKETS / 4.0));
    return b < 0 ? 0 : (b > ORC_BUCKETS - 1 ? ORC_BUCKETS - 1 : b);
}

/* Reading (order of the births): a group's births are drawn slot by slot, each
 * from the random numbers of the slot it is drawn in, and then put in stable
 * bearing-bucket order over those same slots (buckets ascending, drawing
 * order inside a bucket), as the parents of the resampling are, so that
 * neighbouring slots hold births of similar bearing.  Counting sort over the
 * slots [base, base + count) of a particle array with KC slots per component. */
int orc_sort_by_bucket(const orc_model* m, size_t KC, double* X, double* W, size_t base, int count)
{
    if (count <= 1) return 0;
    int* key = (int*)malloc(sizeof(int) * (size_t)count);
    double* tx = (double*)malloc(sizeof(double) * (size_t)count * 5);
    double* tw = (double*)malloc(sizeof(double) * (size_t)count);
    if (!key || !tx || !tw) { free(key); free(tx); free(tw); return -2; }
    int start[ORC_BUCKETS + 1];
    for (int b = 0; b <= ORC_BUCKETS; ++b) start[b] = 0;
    for (int i = 0; i < count; ++i) {
        key[i] = orc_bearing_bucket(m, XS(X, 0, base + i), XS(X, 2, base + i));
        start[key[i] + 1] += 1;
    }
    for (int b = 0; b < ORC_BUCKETS; ++b) start[b + 1] += start[b];
    for (int i = 0; i < count; ++i) {
        int to = start[key[i]]++;
        for (int d = 0; d < m->dim; ++d) tx[(size_t)d * count + to] = XS(X, d, base + i);
        tw[to] = W[base + i];
    }
    for (int i = 0; i < count; ++i) {
        for (int d = 0; d < m->dim; ++d) XS(X, d, base + i) = tx[(size_t)d * count + i];
        W[base + i] = tw[i];
    }
    free(key);
    free(tx);
    free(tw);
    return 0;
}

/* Quantised mass Q 2^-S of n weights (w_max < 2^e, S = 52 - ceil(log2 n) - e,
 * q_i = floor(w_i 2^S), Q their sum); 0 for no positive weight.  The sum is
 * of integers, so it does not depend on the order of the weights. */
static double orc_quantised_mass(const double* w, int n)
{
    double wmax = 0.0;
    for (int i = 0; i < n; ++i)
        if (w[i] > wmax) wmax = w[i];
    if (n <= 0 || wmax <= 0.0) return 0.0;
    int e, b = 0;
    frexp(wmax, &e);
    while (((int64_t)1 << b) < (int64_t)n) ++b;
    int S = 52 - b - e;
    uint64_t Q = 0;
    for (int i = 0; i < n; ++i) Q += (uint64_t)floor(ldexp(w[i], S));
    return Q > 0 ? ldexp((double)Q, -S) : 0.0;
}

int orc_resample(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                 const double* X, const double* W, const int32_t* n,
                 double* Xout, double* Wout, int32_t* nout, int32_t* counts, double* mass_q)
{
    int K = m->partitions;
    size_t KC = (size_t)K * (size_t)cap;
    double Rj = m->particles_per_target / (double)K;
    int err = 0;
    /* each group's quantised mass first (Step 5's count may take the run's
     * total); the quantisation is order-free */
    double* mqa = (double*)calloc((size_t)K, sizeof(double));
    if (!mqa) return -2;
    for (int j = 0; j < K; ++j) mqa[j] = orc_quantised_mass(W + (size_t)j * cap, n[j]);
    /* groups resample independently: one thread per group */
#pragma omp parallel for schedule(dynamic) reduction(min : err)
    for (int j = 0; j < K; ++j) {
        uint64_t* q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(cap > 0 ? cap : 1));
        int* order = (int*)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
        if (!q || !order) { free(q); free(order); err = -2; continue; }
        size_t base = (size_t)j * (size_t)cap;
        int nj = n[j];
        int cap_children = cap - orc_births_in_partition(m, j);
        for (int i = 0; i < cap; ++i) counts[base + i] = 0;
        /* Reading (order of the parents): the parents are taken in bearing-
         * bucket order, buckets ascending and slot order within a bucket (a
         * stable counting sort), so that children near each other in bearing
         * sit next to each other; counts[] follows that order. */
        int hist[ORC_BUCKETS + 1];
        for (int b = 0; b <= ORC_BUCKETS; ++b) hist[b] = 0;
        for (int i = 0; i < nj; ++i) hist[1 + orc_bearing_bucket(m, XS(X, 0, base + i), XS(X, 2, base + i))] += 1;
        for (int b = 0; b < ORC_BUCKETS; ++b) hist[b + 1] += hist[b];
        for (int i = 0; i < nj; ++i) order[hist[orc_bearing_bucket(m, XS(X, 0, base + i), XS(X, 2, base + i))]++] = i;
        /* quantisation */
        double wmax = 0.0;
        for (int i = 0; i < nj; ++i)
            if (W[base + i] > wmax) wmax = W[base + i];
        uint64_t Q = 0;
        int S = 0;
        if (nj > 0 && wmax > 0.0) {
            int e;
            frexp(wmax, &e); /* wmax < 2^e */
            int b = 0;
            while (((int64_t)1 << b) < (int64_t)nj) ++b; /* 2^b >= n */
            S = 52 - b - e;
            for (int i = 0; i < nj; ++i) {
                q[i] = (uint64_t)floor(ldexp(W[base + order[i]], S));
                Q += q[i];
            }
        }
        int64_t L = 0;
        double mq = 0.0;
        if (Q > 0) {
            mq = ldexp((double)Q, -S);
            double t = orc_count_mass(m, mqa, j) * Rj;
            t = t + 0.5;
            double Lf = floor(t);
            if (Lf > (double)cap_children) Lf = (double)cap_children;
            if (Lf < 0.0) Lf = 0.0;
            L = (int64_t)Lf;
        }
        mass_q[j] = mq;
        nout[j] = (int32_t)L;
        if (L == 0) { free(q); free(order); continue; }
        uint32_t r4[4];
        orc_block(seed, (uint32_t)j, step, ORC_RESAMPLE, 0, run, r4);
        uint64_t r = r4[0];
        /* Systematic points u_m = (m + r/2^32) Q / L', m = 0..L'-1.  Child m is
         * the parent i with c_{i-1} <= u_m < c_i.  The comparison
         * u_m < c_i is done exactly as (m 2^32 + r) Q < c_i L' 2^32. */
        int i = 0;
        unsigned __int128 c = q[0];
        for (int64_t mm = 0; mm < L; ++mm) {
            unsigned __int128 lhs = ((unsigned __int128)(((uint64_t)mm << 32) + r)) * Q;
            for (;;) {
                unsigned __int128 rhs = (c * (unsigned __int128)L) << 32;
                if (lhs < rhs) break;
                ++i;
                c += q[i];
            }
            size_t dst = base + (size_t)mm;
            for (int d = 0; d < m->dim; ++d) XS(Xout, d, dst) = XS(X, d, base + order[i]);
            Wout[dst] = mq / (double)L;
            counts[base + i] += 1;
        }
        free(q);
        free(order);
    }
    free(mqa);
    if (err) return err;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 6, local exchange over the ring k -> k+1 (mod K).                    */
/* The paper moves particle i of group k onto particle i of group k+1 for    */
/* i = 1..L, for every k at once, with the L particles chosen at random.     */
/* Readings: one L for all groups, L = floor(rho_x min_j n_j) (so L < n_j/2); */
/* group j's L slots are a systematic sample, one slot per stratum: with a    */
/* uniform u_j = a/2^32 from the EXCHANGE stream and b_j = floor(u_j n_j),    */
/*   S_j(m) = floor((m n_j + b_j) / L),  m = 0..L-1,                          */
/* so every slot is chosen with probability about L/n_j and S_j(m) is the    */
/* floor of a point of [m n_j/L, (m+1) n_j/L): the quantile m/L of the        */
/* group's slot order (distinct slots, as n_j/L >= 2).  The                    */
/* particle-weight couple in S_j(m) replaces the one in S_{j+1}(m).  All     */
/* copies read the state before the exchange, so the exchange permutes the   */
/* particles: group sizes and the global multiset of couples are unchanged.  */
/* ------------------------------------------------------------------------ */
static uint64_t orc_exchange_slot(uint64_t seed, uint32_t step, uint32_t run, int j, int nj, int L, int mm)
{
    uint32_t a[4];
    orc_block(seed, (uint32_t)j, step, ORC_EXCHANGE, 0, run, a);
    uint64_t b = ((uint64_t)a[0] * (uint64_t)nj) >> 32;
    return ((uint64_t)mm * (uint64_t)nj + b) / (uint64_t)L;
}

int orc_exchange(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                 double* X, double* W, const int32_t* n)
{
    int K = m->partitions;
    if (K < 2) return 0;
    int nmin = n[0];
    for (int j = 1; j < K; ++j) if (n[j] < nmin) nmin = n[j];
    int L = (int)floor(m->exchange_fraction * (double)nmin);
    if (L <= 0) return 0;
    size_t KC = (size_t)K * (size_t)cap;
    double* Xs = (double*)malloc(sizeof(double) * (size_t)m->dim * KC);
    double* Ws = (double*)malloc(sizeof(double) * KC);
    if (!Xs || !Ws) { free(Xs); free(Ws); return -2; }
    memcpy(Xs, X, sizeof(double) * (size_t)m->dim * KC);
    memcpy(Ws, W, sizeof(double) * KC);
    for (int j = 0; j < K; ++j) {
        int jn = (j + 1) % K;
        for (int mm = 0; mm < L; ++mm) {
            size_t src = (size_t)j * cap + (size_t)orc_exchange_slot(seed, step, run, j, n[j], L, mm);
            size_t dst = (size_t)jn * cap + (size_t)orc_exchange_slot(seed, step, run, jn, n[jn], L, mm);
            for (int d = 0; d < m->dim; ++d) XS(X, d, dst) = XS(Xs, d, src);
            W[dst] = Ws[src];
        }
    }
    free(Xs);
    free(Ws);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The textbook particle PHD filter of section 2.2 on one particle set,      */
/* written separately from the grouped functions above: Eq 5 (survivors),    */
/* Eq 6 (births), Eq 7 (C_k), Eq 8 (weights), then the mass N_k and the      */
/* resampling of the same section, with no reordering of the particles.  It  */
/* uses the same random streams as the grouped filter with one group, so at  */
/* K = 1 the two agree up to the order of the births and of the parents     */
/* (the grouped filter's bearing order).                                     */
/* Wupd receives the updated (pre-resampling) weights.                       */
/* ------------------------------------------------------------------------ */
int orc_textbook_step(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                      const double* Z, int M, double* X, double* W, int32_t* n,
                      double* Wupd, double* Xout, double* Wout, int32_t* nout)
{
    if (m->partitions != 1 || m->dim != 4) return -1;
    size_t KC = (size_t)cap;
    int L0 = n[0];
    int Jk = m->births_per_step;
    if (L0 + Jk > cap) return -3;
    double T = m->T, sa = m->sigma_a;
    /* 1) prediction, Eq 5: x~ ~ f(.|x), w~ = p_S w */
    for (int i = 0; i < L0; ++i) {
        uint32_t r[4];
        orc_block(seed, (uint32_t)i, step, ORC_PREDICT, 0, run, r);
        double e1, e2;
        orc_normal_pair(orc_u53(r[0], r[1]), orc_u53(r[2], r[3]), &e1, &e2);
        double px = XS(X, 0, i), pvx = XS(X, 1, i), py = XS(X, 2, i), pvy = XS(X, 3, i);
        XS(X, 0, i) = px + T * pvx + (T * T / 2) * (sa * e1);
        XS(X, 1, i) = pvx + T * (sa * e1);
        XS(X, 2, i) = py + T * pvy + (T * T / 2) * (sa * e2);
        XS(X, 3, i) = pvy + T * (sa * e2);
        W[i] = m->p_S * W[i];
    }
    /* Eq 6: births from gamma/m_b, weight gamma/p_k / J_k = m_b / J_k */
    for (int i = L0; i < L0 + Jk; ++i) {
        uint32_t a[4], b[4];
        orc_block(seed, (uint32_t)i, step, ORC_BIRTH, 0, run, a);
        orc_block(seed, (uint32_t)i, step, ORC_BIRTH, 1, run, b);
        double ux = orc_u53(a[0], a[1]), uy = orc_u53(a[2], a[3]);
        double v1, v2;
        orc_normal_pair(orc_u53(b[0], b[1]), orc_u53(b[2], b[3]), &v1, &v2);
        XS(X, 0, i) = m->region[0] + ux * (m->region[1] - m->region[0]);
        XS(X, 1, i) = m->birth_sigma_v * v1;
        XS(X, 2, i) = m->region[2] + uy * (m->region[3] - m->region[2]);
        XS(X, 3, i) = m->birth_sigma_v * v2;
        W[i] = m->birth_mass / (double)Jk;
    }
    int N = L0 + Jk;
    n[0] = N;
    /* 2) update, Eq 7 and Eq 8 */
    double kappa = orc_kappa(m);
    double* Ck = (double*)calloc((size_t)(M > 0 ? M : 1), sizeof(double));
    if (!Ck) return -2;
    for (int p = 0; p < M; ++p)
        for (int i = 0; i < N; ++i)
            Ck[p] += m->p_D * orc_likelihood(m, Z[2 * p], Z[2 * p + 1], XS(X, 0, i), XS(X, 2, i)) * W[i];
    for (int i = 0; i < N; ++i) {
        double bracket = 1.0 - m->p_D;
        for (int p = 0; p < M; ++p)
            bracket += m->p_D * orc_likelihood(m, Z[2 * p], Z[2 * p + 1], XS(X, 0, i), XS(X, 2, i))
                       / (kappa + Ck[p]);
        Wupd[i] = bracket * W[i];
    }
    free(Ck);
    /* 3) resampling: mass N_k, then L_k = round(N_k R) systematic draws over
     * the particles in slot order (births in drawing order after the
     * survivors; no reordering anywhere in this filter).  Same quantisation
     * and point rule as the grouped filter, so the two draw the same number
     * of children from the same weights, each parent's count being the floor
     * or the ceiling of L_k w_i / sum w in either order. */
    double wmax = 0.0;
    for (int i = 0; i < N; ++i) if (Wupd[i] > wmax) wmax = Wupd[i];
    uint64_t* q = (uint64_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(uint64_t));
    int* list = (int*)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
    if (!q || !list) { free(q); free(list); return -2; }
    for (int i = 0; i < N; ++i) list[i] = i;
    uint64_t Q = 0;
    int S = 0;
    if (N > 0 && wmax > 0.0) {
        int e, b = 0;
        frexp(wmax, &e);
        while (((int64_t)1 << b) < (int64_t)N) ++b;
        S = 52 - b - e;
        for (int i = 0; i < N; ++i) { q[i] = (uint64_t)floor(ldexp(Wupd[list[i]], S)); Q += q[i]; }
    }
    int64_t L = 0;
    double Nk = 0.0;
    if (Q > 0) {
        Nk = ldexp((double)Q, -S);
        double t = Nk * m->particles_per_target;
        t = t + 0.5;
        double Lf = floor(t);
        if (Lf > (double)(cap - Jk)) Lf = (double)(cap - Jk);
        L = (int64_t)Lf;
    }
    *nout = (int32_t)L;
    if (L > 0) {
        uint32_t r4[4];
        orc_block(seed, 0u, step, ORC_RESAMPLE, 0, run, r4);
        /* cumulative boundaries, walked with one pointer */
        int i = 0;
        unsigned __int128 c = q[0];
        for (int64_t k = 0; k < L; ++k) {
            unsigned __int128 point = ((unsigned __int128)(((uint64_t)k << 32) + (uint64_t)r4[0])) * Q;
            while (!(point < ((c * (unsigned __int128)L) << 32))) { ++i; c += q[i]; }
            for (int d = 0; d < 4; ++d) XS(Xout, d, k) = XS(X, d, list[i]);
            Wout[k] = Nk / (double)L;
        }
    }
    free(q);
    free(list);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Births from a learned proposal p_k(. | Z_k) (Eq 6, birth_proposal 2).     */
/* Reading: as for birth_proposal 1 the proposal is a defensive mixture,     */
/*   q(x) = alpha gamma(x)/m_b + (1 - alpha) (1/M) sum_p q_p(x),              */
/* but q_p is a 4-component Gaussian mixture over the full state, with the   */
/* parameters a network maps measurement z_p to (the table).  The velocity   */
/* factors no longer cancel, so the weight of Eq 6 is                        */
/*   gamma(x) / (J_j q(x)),  gamma(x) = m_b U(x, y) N(vx; 0, sv^2) N(vy; 0, sv^2). */
/* Draws per birth slot: uniforms (sub 0) for a position from U, normals    */
/* (sub 1) for the two velocities, uniforms (sub 2) choosing the mixture     */
/* term (measurement, then component), normals (sub 3) for the two position */
/* coordinates of a Gaussian component.                                      */
/* ------------------------------------------------------------------------ */

static double orc_prior_density(const orc_model* m, const double x[4])
{
    double area = (m->region[1] - m->region[0]) * (m->region[3] - m->region[2]);
    int inside = x[0] >= m->region[0] && x[0] <= m->region[1] && x[2] >= m->region[2] && x[2] <= m->region[3];
    if (!inside) return 0.0;
    return (1.0 / area) * orc_gauss(x[1], m->birth_sigma_v) * orc_gauss(x[3], m->birth_sigma_v);
}

double orc_mixture_proposal_density(const orc_model* m, const double* table, int M, const double x[4])
{
    double b = orc_prior_density(m, x);
    if (M == 0) return b;
    double mix = 0.0;
    for (int p = 0; p < M; ++p) {
        for (int c = 0; c < 4; ++c) {
            const double* t = table + (size_t)(p * 4 + c) * 9;
            double term = exp(t[0]);
            for (int d = 0; d < 4; ++d) term *= orc_gauss(x[d] - t[1 + d], t[5 + d]);
            mix += term;
        }
    }
    return m->birth_alpha * b + (1.0 - m->birth_alpha) * mix / (double)M;
}

int orc_birth_from_mixture(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                           const double* table, int M, double* X, double* W, const int32_t* n)
{
    int K = m->partitions;
    size_t KC = (size_t)K * (size_t)cap;
    for (int j = 0; j < K; ++j)
        if (n[j] < orc_births_in_partition(m, j)) return -1;
    int err = 0;
#pragma omp parallel for schedule(dynamic) reduction(min : err)
    for (int j = 0; j < K; ++j) {
        int Jj = orc_births_in_partition(m, j);
        int ns = n[j] - Jj;
        for (int b = 0; b < Jj; ++b) {
            uint32_t g = (uint32_t)(j * cap + ns + b);
            uint32_t a[4], v[4], c[4], e[4];
            orc_block(seed, g, step, ORC_BIRTH, 0, run, a);
            orc_block(seed, g, step, ORC_BIRTH, 1, run, v);
            orc_block(seed, g, step, ORC_BIRTH, 2, run, c);
            orc_block(seed, g, step, ORC_BIRTH, 3, run, e);
            double nv1, nv2, e1, e2;
            orc_normal_pair(orc_u53(v[0], v[1]), orc_u53(v[2], v[3]), &nv1, &nv2);
            double uc = orc_u53(c[0], c[1]), uk = orc_u53(c[2], c[3]);
            double x[4];
            if (M == 0 || uc <= m->birth_alpha) {
                x[0] = m->region[0] + orc_u53(a[0], a[1]) * (m->region[1] - m->region[0]);
                x[1] = m->birth_sigma_v * nv1;
                x[2] = m->region[2] + orc_u53(a[2], a[3]) * (m->region[3] - m->region[2]);
                x[3] = m->birth_sigma_v * nv2;
            } else {
                int p = (int)floor((uc - m->birth_alpha) / (1.0 - m->birth_alpha) * (double)M);
                if (p > M - 1) p = M - 1;
                /* component: the first whose cumulative weight reaches uk */
                int comp = 3;
                double cum = 0.0;
                for (int k = 0; k < 4; ++k) {
                    cum += exp(table[(size_t)(p * 4 + k) * 9]);
                    if (uk <= cum) { comp = k; break; }
                }
                const double* t = table + (size_t)(p * 4 + comp) * 9;
                orc_normal_pair(orc_u53(e[0], e[1]), orc_u53(e[2], e[3]), &e1, &e2);
                x[0] = t[1] + t[5] * e1;
                x[1] = t[2] + t[6] * nv1;
                x[2] = t[3] + t[7] * e2;
                x[3] = t[4] + t[8] * nv2;
            }
            for (int d = 0; d < 4; ++d) XS(X, d, g) = x[d];
            orc_birth_turn_rate(m, seed, g, step, run, X, KC);
            double gam = orc_birth_mass(m) * orc_prior_density(m, x);
            W[g] = gam > 0.0 ? gam / ((double)Jj * orc_mixture_proposal_density(m, table, M, x)) : 0.0;
        }
        if (orc_sort_by_bucket(m, KC, X, W, (size_t)j * cap + ns, Jj) != 0) err = -2;
    }
    return err;
}

/* Training pairs for the learned proposal: state from the birth density,
 * measurement from the range-bearing model of section 4 (bearing wrapped to
 * [-pi, pi)). */
int orc_simulate_pairs(const orc_model* m, uint64_t seed, uint32_t run, int first, int n, double* z, double* x)
{
    for (int i = 0; i < n; ++i) {
        uint32_t idx = (uint32_t)(first + i);
        uint32_t a[4], v[4], e[4];
        orc_block(seed, idx, 0, ORC_PAIRS, 0, run, a);
        orc_block(seed, idx, 0, ORC_PAIRS, 1, run, v);
        orc_block(seed, idx, 0, ORC_PAIRS, 2, run, e);
        double px = m->region[0] + orc_u53(a[0], a[1]) * (m->region[1] - m->region[0]);
        double py = m->region[2] + orc_u53(a[2], a[3]) * (m->region[3] - m->region[2]);
        double n1, n2, e1, e2;
        orc_normal_pair(orc_u53(v[0], v[1]), orc_u53(v[2], v[3]), &n1, &n2);
        orc_normal_pair(orc_u53(e[0], e[1]), orc_u53(e[2], e[3]), &e1, &e2);
        double dx = px - m->sensor_x, dy = py - m->sensor_y;
        x[4 * i + 0] = px;
        x[4 * i + 1] = m->birth_sigma_v * n1;
        x[4 * i + 2] = py;
        x[4 * i + 3] = m->birth_sigma_v * n2;
        z[2 * i + 0] = sqrt(dx * dx + dy * dy) + m->sigma_r * e1;
        z[2 * i + 1] = orc_wrap(atan2(dy, dx) + m->sigma_theta * e2);
    }
    return 0;
}
