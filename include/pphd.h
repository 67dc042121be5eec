/*
 * pphd.h -- C ABI of libpphd, the gfx950 (MI355X) implementation of the per-step
 * recursion of the distributed computation particle PHD filter (DCPFPHD) of
 * Wang, Zhao, Su and Ma, "Distributed Computation Particle PHD filter"
 * (arXiv 1503.03769).
 *
 * The K processing elements ("groups") of the paper's section 3 become K
 * partitions of one particle array in device memory.  Every partition runs a
 * full local particle PHD filter on its own particles and sees every
 * measurement; partitions hand particles to their ring neighbour and a central
 * step fuses their estimates.  Every stage runs in HIP kernels on one stream.
 *
 * Conventions for every entry point:
 *  - The return value is a pphd_status; PPHD_OK (0) on success, a negative
 *    code otherwise.  pphd_last_error() then returns a message (thread-local,
 *    valid until the next failing call on the same thread).
 *  - No C++ type, exception or allocation crosses this boundary.
 *  - Device pointers are HIP device pointers on the device that was current
 *    when the filter was created; host pointers are ordinary host memory.
 *  - All device work is queued on the hipStream_t given to pphd_create, in
 *    call order.  Calls that return host data synchronise that stream; the
 *    others return as soon as the work is queued.
 *  - A filter handle may be used from one thread at a time.
 *  - The call order of one filter step follows algorithm 1 and Steps 1-6 of
 *    section 3.1: predict -> update -> [extract] -> resample -> [exchange].
 *    A call out of that order returns PPHD_ESTATE and changes nothing.
 */
#ifndef PPHD_H
#define PPHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PPHD_OK = 0,
    PPHD_EINVAL = -1,     /* a bad argument (null pointer, size out of range)         */
    PPHD_ENOMEM = -2,     /* the workspace is too small or a host allocation failed   */
    PPHD_ECAPACITY = -3,  /* the capacity cannot hold the initial or born particles   */
    PPHD_EDEVICE = -4,    /* a HIP call failed (message holds the HIP error string)  */
    PPHD_ESTATE = -5      /* call out of order for the filter's current phase         */
} pphd_status;

typedef enum { PPHD_FP64 = 0, PPHD_FP32 = 1 } pphd_precision;

/* Phases a filter moves through within one step (see pphd_write_state). */
typedef enum {
    PPHD_PHASE_READY = 1,      /* after init or exchange: next call is predict        */
    PPHD_PHASE_PREDICTED = 2,  /* after predict: next call is update                  */
    PPHD_PHASE_UPDATED = 3,    /* after update (or extract): next is extract/resample */
    PPHD_PHASE_RESAMPLED = 4   /* after resample: next is exchange or predict         */
} pphd_phase;

/*
 * Model of one filter run (section 4 simulation model; parameters are the
 * caller's).  State is 4-D constant velocity [x, vx, y, vy]; the sensor
 * measures [range, bearing] = [|p - s|, atan2(p_y - s_y, p_x - s_x)] with
 * independent Gaussian noise.  State arrays of the ABI hold dim components
 * (double[dim][K*cap]); estimates report [x, vx, y, vy].
 */
typedef struct {
    int32_t dim;              /* 4: constant velocity [x, vx, y, vy] (section 4);        */
                              /* 5: coordinated turn [x, vx, y, vy, omega] (not in the    */
                              /*    paper): x' = x + (sin wT/w) vx - ((1-cos wT)/w) vy,   */
                              /*    y' = y + ((1-cos wT)/w) vx + (sin wT/w) vy, the       */
                              /*    velocity turned by wT, plus the CV acceleration noise */
    int32_t partitions;       /* K >= 1 groups (processing elements)                    */
    int32_t births_per_step;  /* J >= 0 births per step over all groups; group j gets   */
                              /* J/K, plus one when j < J mod K (Step 1, section 3.1)   */
    int32_t precision;        /* pphd_precision: storage and likelihood precision       */
    double T, sigma_a;                                  /* sampling period, accel. noise */
    double sensor_x, sensor_y, sigma_r, sigma_theta;    /* range-bearing sensor          */
    double p_S, p_D;                                    /* survival, detection prob.     */
    double clutter_rate;                                /* lambda (Poisson mean)         */
    double r_min, r_max, th_min, th_max;                /* clutter region; kappa = lambda/area */
    double birth_mass;                                  /* m_b, mass of the birth PHD    */
    double region[4];                                   /* xmin, xmax, ymin, ymax        */
    double birth_sigma_v;                               /* birth velocity std. dev.      */
    double init_mass;                                   /* PHD mass of each group at t=0 */
    double particles_per_target;                        /* R over all groups; R_j = R/K  */
    double exchange_fraction;                           /* rho_x in [0, 0.5)             */
    int32_t birth_proposal;   /* 0: births drawn from gamma/m_b in pphd_predict;          */
                              /* 1: births drawn in pphd_update from the measurement-     */
                              /*    driven mixture of Eq 6's p_k(.|Z_k) (see below);      */
                              /* 2: births drawn in pphd_update from the learned          */
                              /*    per-measurement mixtures (pphd_mlp.h)                 */
    int32_t global_cz;        /* 0: C_k(z) of Eq 11 per group, each group carrying the     */
                              /*    full PHD mass (the paper's Step 2);                    */
                              /* 1: one C_k(z) summed over all groups of the run before    */
                              /*    Eq 12, the groups splitting the PHD mass: initial and  */
                              /*    birth masses are divided by K, and Step 3's LT and     */
                              /*    Step 5's child count take K times a group's mass.      */
                              /*    Batches need every run to have the same partitions.   */
    double birth_alpha;       /* proposals 1, 2: weight of gamma/m_b in the mixture, [0,1] */
    int32_t birth_density;    /* 0: gamma/m_b = U(region) x N(0, birth_sigma_v^2 I);       */
                              /* 1: gamma/m_b = N(birth_mean, diag(birth_std^2)), the      */
                              /*    Gaussian birth intensity of section 4 (proposal 0 only) */
    int32_t reserved2;        /* must be 0                                                */
    double birth_mean[4];     /* density 1: mean of [x, vx, y, vy]                        */
    double birth_std[4];      /* density 1: standard deviations (> 0)                     */
    double sigma_w;           /* dim 5: turn-rate noise, omega' = omega + T sigma_w n     */
    double birth_sigma_w;     /* dim 5: births draw omega ~ N(0, birth_sigma_w^2)         */
} pphd_model;

/* One fused (global) estimate: the mean of the local estimates that carry the
 * same measurement label (Step 4, section 3.1). */
typedef struct {
    double state[4];   /* x, vx, y, vy                                   */
    int32_t label;     /* index of the measurement in this step's set   */
    int32_t votes;     /* number of groups that reported the label      */
} pphd_estimate;

typedef struct pphd_filter pphd_filter;

/* Bytes of device workspace a filter with this model needs.
 * cap_per_partition: particle slots per group, 1 .. 65535 * 256 (must hold
 * round(R/K) initial particles and L' + J_j after every resampling; L' is
 * clamped to fit).
 * max_meas: the largest measurement count a later pphd_update may pass, in
 * [1, 6144] (the C(z) combination keeps one double per measurement in LDS).
 * Returns PPHD_EINVAL for an invalid model or sizes. */
pphd_status pphd_workspace_size(const pphd_model* model, int64_t cap_per_partition,
                                int32_t max_meas, size_t* bytes);

/* Creates a filter.  workspace: caller-owned device memory of at least
 * pphd_workspace_size() bytes, 256-byte aligned; it holds every device array
 * of the filter (two particle sets, per-stage partial results, outputs) and
 * must stay allocated until pphd_destroy.  The library never frees it.
 * seed, run_id: key and counter word of the Philox-4x32-10 streams.
 * stream: a hipStream_t (NULL = default stream).  The handle is
 * library-owned; release it with pphd_destroy. */
pphd_status pphd_create(const pphd_model* model, int64_t cap_per_partition, int32_t max_meas,
                        void* workspace, size_t workspace_bytes, uint64_t seed, uint32_t run_id,
                        void* stream, pphd_filter** out);

/* t = 0 of section 3.1: every group draws round(R/K) particles from the
 * normalised birth density, each with weight init_mass / round(R/K).
 * Allowed in any phase; moves the filter to PPHD_PHASE_READY. */
pphd_status pphd_init(pphd_filter* f);

/* Step 1 (Eqs 5 and 6): survivors move through the CV model with Philox noise
 * and take weight p_S * w; group j appends J_j births.  With birth_proposal 0
 * they are drawn here from the birth density with weight m_b / J_j; with
 * birth_proposal 1 their slots are reserved and pphd_update draws them from
 *   q(x|Z_k) = alpha gamma(x)/m_b + (1 - alpha) (1/M) sum_p q_p(x),
 * q_p placing the particle at range N(r_p, sigma_r^2), bearing
 * N(theta_p, sigma_theta^2) with velocity N(0, sigma_v^2 I), and weight
 * gamma(x) / (J_j q(x)) (Eq 6); birth_proposal 2 reserves them the same way for
 * the learned mixtures of pphd_mlp.h.  Once drawn (each from the Philox
 * numbers of the slot it is drawn in), a group's births are put in stable
 * bearing-bucket order over their slots, as the resampling orders parents.
 * step: the time index k >= 1.
 * Phase READY or RESAMPLED -> PREDICTED. */
pphd_status pphd_predict(pphd_filter* f, uint32_t step);

/* Step 2 (Eqs 7, 8 and 10-15): C_j(z_p) = sum over group j of p_D g(z_p|x) w
 * for every measurement, then w <- [1 - p_D + sum_p p_D g(z_p|x)/(kappa +
 * C_j(z_p))] w, plus the sums that Step 3 needs.
 * z: m pairs (range, bearing), double[m][2], on the host (z_on_device = 0;
 * copied before the call returns) or on the device (z_on_device = 1; read in
 * stream order, so it must stay valid until the stream reaches this work).
 * 0 <= m <= max_meas.  Phase PREDICTED -> UPDATED. */
pphd_status pphd_update(pphd_filter* f, const double* z, int32_t m, int32_t z_on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pphd_update
 * with the first likelihood pass's partial sums in a static device array of
 * the library (64 MiB per device, held until the process ends) instead of the
 * workspace.  Same arguments, phases and results as pphd_update, bit for bit;
 * it calls no allocating routine.  The partials need
 * K * ceil(cap / (64 p)) * (12 max_meas + 8) bytes, p = 4 in FP32 and 2 in
 * FP64 (each of the three parts rounded up to 256 bytes); a filter above
 * 64 MiB gets PPHD_EINVAL.  All filters on one device share the array: calls
 * that overlap on one device (other streams or threads) race.  Not with
 * kernel timing on (PPHD_EINVAL); not for batches. */
pphd_status pphd_update_noalloc(pphd_filter* f, const double* z, int32_t m, int32_t z_on_device);

/* Steps 3 and 4: each group keeps its round(sum w) best-supported measurement
 * labels with local estimates (Eqs 16-18); labels reported by more than half
 * of the groups are averaged into global estimates, ordered by label.
 * out: host array of cap records; *n_out receives the number written.
 * mass_per_partition: nullable host double[K], receives each group's
 * updated PHD mass.  Synchronises the stream.  Phase UPDATED (unchanged). */
pphd_status pphd_extract(pphd_filter* f, pphd_estimate* out, int32_t cap, int32_t* n_out,
                         double* mass_per_partition);

/* As pphd_extract, but the records and their count are written to device
 * memory in stream order (d_out: cap records, d_n_out: one int32); no
 * synchronisation.  Records beyond cap are dropped; *d_n_out holds the full
 * count.  The first such call after an update also sorts the parents for the
 * coming pphd_resample in the same launch (into the other particle set, which
 * no other call reads); the estimates are complete when the stream reaches
 * the call, as with any launch. */
pphd_status pphd_extract_device(pphd_filter* f, pphd_estimate* d_out, int32_t cap,
                                int32_t* d_n_out);

/* Step 5: every group quantises its weights, draws L' = round(N_j R_j)
 * children by systematic resampling (one Philox uniform per group) over its
 * parents taken in bearing-bucket order (the "diamond angle" of the offset
 * from the sensor in 64 buckets, ascending; slot order inside a bucket;
 * children in that parent order), clamps L' to cap - J_j and gives each
 * child weight N_j / L'.  step: the time index of the preceding predict.
 * Phase UPDATED -> RESAMPLED. */
pphd_status pphd_resample(pphd_filter* f, uint32_t step);

/* Step 6: ring exchange j -> j+1 (mod K) within each run of L = floor(rho_x
 * min_j L'_j) particle-weight couples per group, all read before any is
 * written.  Group j sends a systematic sample of its slots, one per stratum:
 * S_j(m) = floor((m L'_j + floor(u_j L'_j)) / L), u_j a Philox uniform per
 * group and step; the couple in S_j(m) replaces the one in S_{j+1}(m).  No-op
 * for K = 1.  Phase RESAMPLED -> READY. */
pphd_status pphd_exchange(pphd_filter* f, uint32_t step);

/* Releases the handle and its host resources (not the workspace).
 * Synchronises the stream.  NULL is accepted. */
pphd_status pphd_destroy(pphd_filter* f);

/* Message of the last failing call on this thread ("" if none). */
const char* pphd_last_error(void);

/* ---- state access (stage tests, checkpoint and restore) ---------------- */

/* Copies the current particle set to host memory, converted to double.
 * x: double[4][K*cap] (component d of slot s of group j at d*K*cap + j*cap + s),
 * w: double[K*cap], count: int32[K] (occupied slots per group).  Any of the
 * three may be NULL.  Slots beyond count are unspecified.  Synchronises. */
pphd_status pphd_read_state(pphd_filter* f, double* x, double* w, int32_t* count);

/* Overwrites the current particle set from host memory (same layout as
 * pphd_read_state; values are rounded to the storage precision) and puts the
 * filter into the given phase: READY or RESAMPLED (next: predict / exchange)
 * or PREDICTED (next: update) or UPDATED (next: resample only).
 * count[j] must be <= cap.  Synchronises. */
pphd_status pphd_write_state(pphd_filter* f, const double* x, const double* w,
                             const int32_t* count, int32_t phase);

/* Results of the last update, copied to host memory (any pointer may be NULL):
 * C: double[K][m], C_j(z_p) of Eq 11 (0 where it underflows double);
 * dW: double[K][m], Delta W^{j,p} of Eq 16; mass: double[K], each group's
 * updated PHD mass; LT: int32[K], round(mass) capped at m.  Synchronises. */
pphd_status pphd_read_update(pphd_filter* f, double* C, double* dW, double* mass, int32_t* LT);

/* Local estimates of the last update (Step 3): sel: int32[K][m], 1 where
 * measurement p is in group j's label set I_j; zeta: double[K][m][4], the
 * local estimate of that label (0 elsewhere).  Synchronises. */
pphd_status pphd_read_local(pphd_filter* f, int32_t* sel, double* zeta);

/* Tile shape of the two likelihood passes of pphd_update: particles per
 * thread of the C(z) pass and of the weight pass (4, 8 or 16 with FP32
 * storage; 2, 4 or 8 with FP64) and the target number of measurements per
 * wavefront (1..4096; the measurement loop is cut into at most 16 chunks).
 * Results depend on it only through floating-point summation order.
 * Defaults: 8, 8, 16 (FP32); 4, 4, 16 (FP64).  Takes effect at the next
 * update; must not be called between pphd_update and pphd_resample. */
pphd_status pphd_set_tuning(pphd_filter* f, int32_t pt_cz, int32_t pt_weight, int32_t meas_per_wave);

/* Launch shape of the other tunable kernels (the autotuner's second set of
 * knobs; results do not change, only the schedule):
 * pass_workgroups: workgroups of one bearing-frame pass launch (their
 *   wavefronts stride over the work items); 0 = 1024, else [64, 65535].
 * rs_tiles: 256-slot tiles per workgroup of the resampling's scatter and
 *   expansion, 1 or 2; 0 = two where K * cap >= 2^20, else one.
 * Allowed in any phase. */
pphd_status pphd_set_launch_shape(pphd_filter* f, int32_t pass_workgroups, int32_t rs_tiles);

/* Enables (1) or disables (0) recording of per-parent child counts in
 * resample, which costs one int32 store per parent. */
pphd_status pphd_set_record_counts(pphd_filter* f, int32_t enable);

/* Results of the last resample: counts: int32[K*cap], children of parent
 * slot j*cap+i (only if recording was enabled); mass_q: double[K], the
 * quantised group mass N_j; clamped: total number of group resamplings so
 * far whose L' was clamped to the capacity.  Synchronises. */
pphd_status pphd_read_resample(pphd_filter* f, int32_t* counts, double* mass_q, int64_t* clamped);

/* ---- timing ------------------------------------------------------------- */

/* Kernel classes timed by the library; a class may span several kernels:
 *   PREDICT k_predict; CZ k_cz_frames or k_cz; CZ_COMBINE k_cz_combine;
 *   WEIGHT k_weight_frames (which also finalizes the weights) or k_weight;
 *   WFINAL k_wfinal (passes other than the bearing-frame ones); FINALIZE
 *   k_finalize; FUSE k_fuse; RS_ORDER the parents' bucket order
 *   (k_bk_scatter, with k_bk_hist and k_bk_scan when the update did not
 *   prepare it); RS_EXPAND k_rs_expand; XCHG_SCATTER k_xchg_ring or
 *   k_xchg_scatter; XCHG_GATHER k_xchg_gather; BIRTH k_birth_draw and
 *   k_birth_weight (proposal 1); BIRTH_MIX the same for proposal 2;
 *   BIRTH_ORDER k_birth_draw_sort (whose launch also prepares the
 *   measurements of the bearing-frame passes when it runs), k_birth_sort, or
 *   the births' bucket order; MLP_INFER the mixture table; ZPREP k_zprep
 *   (when no k_birth_draw_sort launch prepared the measurements) and the
 *   work lists;
 *   INIT, WMAX, GEOM their kernels.  RS_TILES times nothing (kept for the
 *   numbering). */
enum {
    PPHD_K_PREDICT = 0, PPHD_K_CZ = 1, PPHD_K_CZ_COMBINE = 2, PPHD_K_WEIGHT = 3,
    PPHD_K_FINALIZE = 4, PPHD_K_FUSE = 5, PPHD_K_RS_TILES = 6, PPHD_K_RS_EXPAND = 7,
    PPHD_K_XCHG_GATHER = 8, PPHD_K_XCHG_SCATTER = 9, PPHD_K_INIT = 10, PPHD_K_WMAX = 11,
    PPHD_K_GEOM = 12, PPHD_K_WFINAL = 13, PPHD_K_BIRTH = 14, PPHD_K_MLP_INFER = 15,
    PPHD_K_BIRTH_MIX = 16, PPHD_K_ZPREP = 17, PPHD_K_RS_ORDER = 18,
    PPHD_K_BIRTH_ORDER = 19, PPHD_K_COUNT = 20
};

/* Enables (1) or disables (0) per-launch HIP-event timing on the filter's
 * stream, and clears the accumulated times. */
pphd_status pphd_set_timing(pphd_filter* f, int32_t enable);

/* Total milliseconds and launch counts per kernel class since timing was
 * enabled: ms: double[PPHD_K_COUNT], launches: int64[PPHD_K_COUNT].
 * Synchronises. */
pphd_status pphd_read_timing(pphd_filter* f, double* ms, int64_t* launches);

/* Kernel name of a class (for profiler cross-reference), or NULL. */
const char* pphd_kernel_name(int32_t kernel_class);

/* ---- batches of independent runs ---------------------------------------- */

/* A batch runs many independent filters (runs) of the same model in one set
 * of launches per stage: every kernel covers the groups of all runs.  The
 * per-run fields of the model (partitions, births_per_step, clutter_rate,
 * particles_per_target) are replaced by a run table; everything else is
 * shared.  Run r uses Philox run word run_id and, for group j of the run,
 * the slot counters j*cap + s, so it draws exactly the numbers it would draw
 * as a single filter created with the same seed and run_id: its particles,
 * weights and estimates equal that filter's (the same arithmetic in the same
 * order).  pphd_init, pphd_predict, pphd_resample, pphd_exchange,
 * pphd_read_state, pphd_write_state, pphd_set_tuning, pphd_set_timing and
 * pphd_destroy accept a batch handle; state arrays hold the groups of all runs
 * in run order (group g = run_g0 + j).  With birth_proposal 2 the attached
 * network (pphd_attach_mlp) runs once over the step's concatenated set. */
typedef struct {
    int32_t partitions;           /* K_r >= 1 groups of the run                      */
    int32_t births_per_step;      /* J_r >= 0, split over its groups as for a filter */
    double clutter_rate;          /* lambda_r; kappa_r = lambda_r / clutter area      */
    double particles_per_target;  /* R_r                                             */
    uint32_t run_id;              /* Philox run word of the run                      */
    int32_t reserved;             /* must be 0                                       */
} pphd_run_desc;

/* Workspace bytes of a batch: nruns runs, cap slots per group,
 * max_meas_per_run measurements per run and step. */
pphd_status pphd_batch_workspace_size(const pphd_model* model, const pphd_run_desc* runs, int32_t nruns,
                                      int64_t cap_per_partition, int32_t max_meas_per_run, size_t* bytes);

/* Creates a batch (see pphd_create for workspace, seed and stream). */
pphd_status pphd_batch_create(const pphd_model* model, const pphd_run_desc* runs, int32_t nruns,
                              int64_t cap_per_partition, int32_t max_meas_per_run, void* workspace,
                              size_t workspace_bytes, uint64_t seed, void* stream, pphd_filter** out);

/* Step 2 for every run.  z: the step's measurement sets of all runs,
 * concatenated, double[z_count][2] (z_count <= nruns * max_meas_per_run);
 * windows: int32[nruns][2], (offset, count) of run r's set in z (count <=
 * max_meas_per_run).  Both on the host (copied before the call returns;
 * windows outside the set return PPHD_EINVAL) or both on the device
 * (on_device = 1; read in stream order, windows clamped into the set).
 * Phase PREDICTED -> UPDATED. */
pphd_status pphd_batch_update(pphd_filter* f, const double* z, int32_t z_count, const int32_t* windows,
                              int32_t on_device);

/* Steps 3 and 4 per run: run r's fused estimates go to out + r*cap (at most
 * cap records, in label order), their count to n_out[r].  Host version:
 * synchronises; mass (nullable) receives every group's updated mass.
 * Device version: d_n_out[r] holds the full count, records beyond cap (and
 * beyond max_meas_per_run) are dropped. */
pphd_status pphd_batch_extract(pphd_filter* f, pphd_estimate* out, int32_t cap, int32_t* n_out, double* mass);
pphd_status pphd_batch_extract_device(pphd_filter* f, pphd_estimate* d_out, int32_t cap, int32_t* d_n_out);

/* Captures one whole step of the batch (predict, update over the device
 * buffers d_z / d_windows, fused estimates to d_out / d_n_out as in
 * pphd_batch_extract_device, resample, exchange) into HIP graphs, one per
 * particle-set parity.  Nothing runs at capture.  The step index is a device
 * counter set to first_step here and advanced at the end of every replay.
 * The caller refills d_z and d_windows (z_count rows at most) between
 * replays.  Phase READY or RESAMPLED; timing must be off. */
pphd_status pphd_batch_capture(pphd_filter* f, const double* d_z, int32_t z_count, const int32_t* d_windows,
                               pphd_estimate* d_out, int32_t cap, int32_t* d_n_out, uint32_t first_step);

/* Replays the captured step once on the batch's stream (one graph launch).
 * Phase READY or RESAMPLED -> READY. */
pphd_status pphd_batch_launch(pphd_filter* f);

#ifdef __cplusplus
}
#endif
#endif /* PPHD_H */
