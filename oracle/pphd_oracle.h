/*
 * Oracle for the distributed particle PHD filter -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of one filter step
 * of the distributed computation particle PHD filter (DCPFPHD), written from
 * the paper "Distributed Computation Particle PHD filter" (Wang, Zhao, Su, Ma;
 * arXiv 1503.03769).  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library; the two meet only through seeded inputs.
 *
 * State layout used by every function (all arrays owned by the caller):
 *   X : double[dim][K*cap]  component d of slot s in partition j is X[d*K*cap + j*cap + s]
 *                           (dim = 4 or 5, the model's)
 *   W : double[K*cap]       weight of the same slot
 *   n : int32[K]            number of occupied slots of partition j (slots 0..n[j]-1)
 *
 * Random numbers: one Philox-4x32-10 block per (slot, step, purpose, run),
 * key = (seed low word, seed high word), counter = (c0, step, purpose*16+sub, run).
 */
#ifndef PPHD_ORACLE_H
#define PPHD_ORACLE_H
#include <stddef.h>
#include <stdint.h>

typedef struct {
    int32_t dim;              /* 4: constant-velocity state [x, vx, y, vy];
                                 5: coordinated-turn state [x, vx, y, vy, omega] */
    int32_t partitions;       /* K, number of processing elements / groups */
    int32_t births_per_step;  /* J, split over the K groups */
    int32_t global_cz;        /* 0: C_k(z) per group, Eq 11 as printed (each group carries the
                                    full PHD mass);
                                 1: C_k(z) summed over all groups before Eq 12, the groups
                                    splitting the PHD mass (each carries 1/K of it) */
    double T, sigma_a;                              /* CV model */
    double sensor_x, sensor_y, sigma_r, sigma_theta; /* range-bearing sensor */
    double p_S, p_D;
    double clutter_rate;                            /* lambda */
    double r_min, r_max, th_min, th_max;            /* clutter region */
    double birth_mass;                              /* m_b */
    double region[4];                               /* xmin, xmax, ymin, ymax */
    double birth_sigma_v;
    double init_mass;
    double particles_per_target;                    /* R over all groups */
    double exchange_fraction;                       /* rho_x */
    int32_t birth_proposal;   /* 0: births from gamma/m_b; 1: measurement-driven mixture;
                                 2: learned per-measurement Gaussian mixtures */
    int32_t reserved2;
    double birth_alpha;       /* weight of gamma/m_b in the mixture (proposal 1) */
    int32_t birth_density;    /* 0: U(region) x N(0, sigma_v^2 I);  1: N(birth_mean, diag(birth_std^2)) */
    int32_t reserved3;
    double birth_mean[4];
    double birth_std[4];
    double sigma_w;           /* dim 5: turn-rate noise (rad/s per unit time) */
    double birth_sigma_w;     /* dim 5: turn-rate spread of the birth density */
} orc_model;

enum { ORC_INIT = 1, ORC_PREDICT = 2, ORC_BIRTH = 3, ORC_RESAMPLE = 4, ORC_EXCHANGE = 5, ORC_PAIRS = 6 };

void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* The per-group loops of predict, births, update and resample run one group
 * per thread (OpenMP); the results are the same for any thread count. */
void   orc_set_threads(int n);
int    orc_threads(void);
double orc_u53(uint32_t a, uint32_t b);
void   orc_normal_pair(double u1, double u2, double* n1, double* n2);
int    orc_births_in_partition(const orc_model* m, int j);
double orc_kappa(const orc_model* m);
double orc_likelihood(const orc_model* m, double zr, double zth, double x, double y);

int orc_init(const orc_model* m, int cap, uint64_t seed, uint32_t run,
             double* X, double* W, int32_t* n);
int orc_predict(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                double* X, double* W, int32_t* n);
double orc_birth_proposal_density(const orc_model* m, const double* Z, int M, double x, double y);
int orc_birth_from_measurements(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                                const double* Z, int M, double* X, double* W, const int32_t* n);
/* Learned proposal (birth_proposal 2).  table holds, for each measurement p
 * and mixture component c, 9 doubles at table[(p*4 + c)*9]: log pi_c (the
 * normalised log weight), the mean (4, state units) and the standard
 * deviations (4, state units) of a diagonal Gaussian over [x, vx, y, vy]. */
double orc_mixture_proposal_density(const orc_model* m, const double* table, int M, const double x[4]);
int orc_birth_from_mixture(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                           const double* table, int M, double* X, double* W, const int32_t* n);
/* Training pairs (z, x): x drawn from gamma/m_b, z = (range, bearing) drawn
 * from the sensor model given x.  Pair i (i = first .. first+n-1) goes to
 * z[2*(i-first)], x[4*(i-first)]. */
int orc_simulate_pairs(const orc_model* m, uint64_t seed, uint32_t run, int first, int n, double* z, double* x);
int orc_update(const orc_model* m, int cap, const double* Z, int M,
               const double* X, double* W, const int32_t* n,
               double* C, double* dW, double* dW0, double* zeta_num, double* mass);
int orc_extract(const orc_model* m, int M, const double* dW, const double* zeta_num,
                const double* mass, int32_t* LT, int32_t* sel, double* zeta);
int orc_fuse(const orc_model* m, int M, const int32_t* sel, const double* zeta,
             double* est_state, int32_t* est_label, int32_t* est_votes, int32_t* n_est);
int orc_bearing_bucket(const orc_model* m, double x, double y);
/* Stable bearing-bucket order of the slots [base, base + count) of a particle
 * array with KC slots per component (births, after they are drawn). */
int orc_sort_by_bucket(const orc_model* m, size_t KC, double* X, double* W, size_t base, int count);
int orc_resample(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                 const double* X, const double* W, const int32_t* n,
                 double* Xout, double* Wout, int32_t* nout, int32_t* counts, double* mass_q);
int orc_exchange(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                 double* X, double* W, const int32_t* n);
int orc_textbook_step(const orc_model* m, int cap, uint32_t step, uint64_t seed, uint32_t run,
                      const double* Z, int M, double* X, double* W, int32_t* n,
                      double* Wupd, double* Xout, double* Wout, int32_t* nout);

#endif
